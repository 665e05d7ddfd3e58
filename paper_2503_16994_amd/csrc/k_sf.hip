// Schroedinger-functional boundary source (paper Sec. 3.3: boundary-to-bulk
// propagators for Dirichlet boundary conditions, the input of f_P and f_A).
//
// The boundary quark field at y0 = 0 couples to the bulk through the time
// link U_t(y0 = 0, y) and the projector P+ = (1 + g_t)/2, so the 12 source
// columns (spin s, colour c) of the boundary-to-bulk propagator are the
// columns of P+ U_t(0, y)^+ on the slice y0 = 1:
//   eta_{3s+c}(y)[al][a] = P+[al][s] conj(U_t(0, y)[c][a])   (y0 = 1).
// In the chiral basis g_t pairs spin al with al ^ 2 (entries -1), so
// P+[al][s] = 1/2 for al = s, -1/2 for al = s ^ 2, 0 otherwise.  One thread
// per spatial site; the link is read from the FP64 copy in the internal
// layout (two-row links rebuilt), the output is canonical.
#include "lqcd_kernels.h"

namespace lqcd {

__global__ void k_sf_source(KGeom g, const double2* __restrict__ U64, int two_row, double2* eta) {
  const long V3 = (long)g.L[0] * g.L[1] * g.L[2], V = V3 * g.L[3];
  const long lx = (long)blockIdx.x * blockDim.x + threadIdx.x;  // spatial site (x fastest)
  if (lx >= V3) return;
  const int x = (int)(lx % g.L[0]);
  const int y = (int)((lx / g.L[0]) % g.L[1]);
  const int z = (int)(lx / ((long)g.L[0] * g.L[1]));
  const int p = (x + y + z) & 1;  // parity of (x, y, z, 0)
  const long s = lx >> 1;         // index within the parity (lex / 2, lex = lx at y0 = 0)
  const int ne = two_row ? 6 : 9;
  const double2* up = U64 + (size_t)p * 4 * ne * g.V2p + tix(s, 4 * ne) + 3 * ne * kTile;  // mu = t
  cpx<double> u[9];
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const double2 v = up[e * kTile];
    u[e] = {v.x, v.y};
  }
  if (two_row) {
    su3_third_row(u);
  } else {
#pragma unroll
    for (int e = 6; e < 9; ++e) {
      const double2 v = up[e * kTile];
      u[e] = {v.x, v.y};
    }
  }
  const long site = V3 + lx;  // (x, y, z, 1)
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double2* col = eta + ((size_t)(3 * sp + c) * V + site) * 12;
#pragma unroll
      for (int al = 0; al < 4; ++al) {
        const double w = (al == sp) ? 0.5 : ((al == (sp ^ 2)) ? -0.5 : 0.0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const cpx<double> v = u[3 * c + a];  // U[c][a]
          col[3 * al + a] = make_double2(w * v.re, -w * v.im);
        }
      }
    }
}

hipError_t launch_sf_source(const KGeom& g, const double2* U64, int two_row, double2* eta, hipStream_t st) {
  const long V3 = (long)g.L[0] * g.L[1] * g.L[2];
  if (g.L[3] < 2 || V3 <= 0) return hipErrorInvalidValue;
  k_sf_source<<<(unsigned)((V3 + 127) / 128), 128, 0, st>>>(g, U64, two_row, eta);
  return hipGetLastError();
}

}  // namespace lqcd
