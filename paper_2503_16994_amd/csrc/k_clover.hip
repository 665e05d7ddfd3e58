// Clover term (the Csw! step of paper Sec. 3.3), computed in FP64.
//
// Per site: the clover-leaf field strength of the six planes, made
// anti-Hermitian and traceless; then, in the chiral basis, the diagonal term
// splits into two Hermitian 6x6 blocks (row index 3*spin + colour within a
// chirality):
//   A_+- = (4 + m0 + d_bnd (cF-1)) 1 + (csw/2) [[ i E3, i E1 + E2 ],
//                                              [ i E1 - E2, -i E3 ]],
//   E_k = +-F_{t k} - B_k,  B_1 = F_{yz}, B_2 = F_{zx}, B_3 = F_{xy}.
// This is the sigma_{mu nu} (x) F_{mu nu} sum written out for the chiral
// basis (sigma_{kl} = -eps_{klm} diag(s_m, s_m), sigma_{tk} = diag(s_k, -s_k)).
// The inverse of each block on the odd sites is formed by an unpivoted
// LDL^H factorisation, with Gauss-Jordan elimination under partial pivoting
// as the fallback for an indefinite block with a tiny LDL^H pivot
// (clover_inv.h); a block that is singular to working precision is reported
// as a numerical error.
#include "clover_inv.h"
#include "lqcd_kernels.h"

namespace lqcd {

using cd = cpx<double>;

struct M3 {
  cd m[9];
};

__device__ inline M3 m3_mul(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cd v = cmul(a.m[3 * i], b.m[j]);
      v = cadd(v, cmul(a.m[3 * i + 1], b.m[3 + j]));
      v = cadd(v, cmul(a.m[3 * i + 2], b.m[6 + j]));
      r.m[3 * i + j] = v;
    }
  return r;
}

// a * b^+
__device__ inline M3 m3_mul_nd(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cd v = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const cd bb = b.m[3 * j + k];
        v = cadd(v, cmul(a.m[3 * i + k], cd{bb.re, -bb.im}));
      }
      r.m[3 * i + j] = v;
    }
  return r;
}

// a^+ * b
__device__ inline M3 m3_mul_dn(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cd v = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) v = cadd(v, cmulc(a.m[3 * k + i], b.m[3 * k + j]));
      r.m[3 * i + j] = v;
    }
  return r;
}

__device__ inline M3 load_link(const KGeom& g, const double2* U, bool two_row, int x, int y, int z,
                               int t, int mu) {
  x = (x + g.L[0]) % g.L[0];
  y = (y + g.L[1]) % g.L[1];
  z = (z + g.L[2]) % g.L[2];
  t = (t + g.L[3]) % g.L[3];
  const long lex = x + (long)g.L[0] * (y + (long)g.L[1] * (z + (long)g.L[2] * t));
  const int p = (x + y + z + t) & 1;
  const size_t s = (size_t)(lex >> 1);
  const int ne = two_row ? 6 : 9;  // stored complex per link
  const double2* u = U + (size_t)p * 4 * ne * g.V2p + tix(s, 4 * ne) + mu * ne * kTile;
  M3 r;
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    double2 v = u[e * kTile];
    r.m[e] = {v.x, v.y};
  }
  if (two_row) {
    su3_third_row(r.m);
  } else {
#pragma unroll
    for (int e = 6; e < 9; ++e) {
      double2 v = u[e * kTile];
      r.m[e] = {v.x, v.y};
    }
  }
  return r;
}

// traceless anti-Hermitian part of (Q - Q^+)/8 for the (mu, nu) plane at x
__device__ inline M3 field_strength(const KGeom& g, const double2* U, bool two_row, const int (&x)[4],
                                    int mu, int nu) {
  int dm[4] = {0, 0, 0, 0}, dn[4] = {0, 0, 0, 0};
  dm[mu] = 1;
  dn[nu] = 1;
#define LNK(ox, oy, oz, ot, d) load_link(g, U, two_row, x[0] + (ox), x[1] + (oy), x[2] + (oz), x[3] + (ot), d)
  const M3 Um_x = LNK(0, 0, 0, 0, mu);
  const M3 Un_x = LNK(0, 0, 0, 0, nu);
  const M3 Un_xpm = LNK(dm[0], dm[1], dm[2], dm[3], nu);
  const M3 Um_xpn = LNK(dn[0], dn[1], dn[2], dn[3], mu);
  const M3 Um_xmm = LNK(-dm[0], -dm[1], -dm[2], -dm[3], mu);
  const M3 Un_xmm = LNK(-dm[0], -dm[1], -dm[2], -dm[3], nu);
  const M3 Um_xmmpn = LNK(dn[0] - dm[0], dn[1] - dm[1], dn[2] - dm[2], dn[3] - dm[3], mu);
  const M3 Um_xmmmn = LNK(-dm[0] - dn[0], -dm[1] - dn[1], -dm[2] - dn[2], -dm[3] - dn[3], mu);
  const M3 Un_xmmmn = LNK(-dm[0] - dn[0], -dm[1] - dn[1], -dm[2] - dn[2], -dm[3] - dn[3], nu);
  const M3 Um_xmn = LNK(-dn[0], -dn[1], -dn[2], -dn[3], mu);
  const M3 Un_xmn = LNK(-dn[0], -dn[1], -dn[2], -dn[3], nu);
  const M3 Un_xpmmn = LNK(dm[0] - dn[0], dm[1] - dn[1], dm[2] - dn[2], dm[3] - dn[3], nu);
#undef LNK
  // four counter-clockwise leaves starting and ending at x
  M3 l1 = m3_mul_nd(m3_mul_nd(m3_mul(Um_x, Un_xpm), Um_xpn), Un_x);
  M3 l2 = m3_mul(m3_mul_nd(m3_mul_nd(Un_x, Um_xmmpn), Un_xmm), Um_xmm);
  // Um(x-m)^+ Un(x-m-n)^+ = (Un(x-m-n) Um(x-m))^+, then * Um(x-m-n) * Un(x-n)
  M3 l3 = m3_mul(m3_mul_dn(m3_mul(Un_xmmmn, Um_xmm), Um_xmmmn), Un_xmn);
  M3 l4 = m3_mul_nd(m3_mul(m3_mul_dn(Un_xmn, Um_xmn), Un_xpmmn), Um_x);
  M3 F;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cd q = cadd(cadd(l1.m[3 * i + j], l2.m[3 * i + j]), cadd(l3.m[3 * i + j], l4.m[3 * i + j]));
      cd qt = cadd(cadd(l1.m[3 * j + i], l2.m[3 * j + i]), cadd(l3.m[3 * j + i], l4.m[3 * j + i]));
      F.m[3 * i + j] = {(q.re - qt.re) * 0.125, (q.im + qt.im) * 0.125};
    }
  const double tr_im = (F.m[0].im + F.m[4].im + F.m[8].im) / 3.0;
  F.m[0].im -= tr_im;
  F.m[4].im -= tr_im;
  F.m[8].im -= tr_im;
  F.m[0].re = F.m[4].re = F.m[8].re = 0.0;
  return F;
}

__device__ inline cd times_i(cd a) { return {-a.im, a.re}; }

// Hermitian 6x6 block from E1, E2, E3 (anti-Hermitian 3x3), full storage
__device__ inline void make_block(const M3& E1, const M3& E2, const M3& E3, double c, double d,
                                  cd (&B)[6][6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const cd e1 = E1.m[3 * a + b], e2 = E2.m[3 * a + b], e3 = E3.m[3 * a + b];
      const cd ie3 = times_i(e3), ie1 = times_i(e1);
      B[a][b] = cscale(c, ie3);
      B[3 + a][3 + b] = cscale(-c, ie3);
      B[a][3 + b] = cscale(c, cadd(ie1, e2));
      B[3 + a][b] = cscale(c, csub(ie1, e2));
    }
#pragma unroll
  for (int i = 0; i < 6; ++i) B[i][i].re += d;
}

// block B into components c0 .. c0+17 of site s of a tiled 36-component field
template <typename S>
__device__ inline void store_packed(S* field, size_t s, int c0, const cd (&B)[6][6]) {
  S* base = field + tix(s, 36) + c0 * kTile;
  st(base + 0 * kTile, cd{B[0][0].re, B[1][1].re});
  st(base + 1 * kTile, cd{B[2][2].re, B[3][3].re});
  st(base + 2 * kTile, cd{B[4][4].re, B[5][5].re});
#pragma unroll
  for (int i = 1; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < i; ++j) st(base + tri_index(i, j) * kTile, B[i][j]);
}

__global__ __launch_bounds__(128) void k_clover(const CloverLaunch c) {
  const KGeom& g = c.g;
  const int p = blockIdx.y;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V2) return;
  const Coord co = site_coord(g, s, p);
  const int x[4] = {co.x, co.y, co.z, co.t};
  const size_t par = (size_t)p * 36 * g.V2p;  // parity p of the clover field

  // planes: 0 xy, 1 xz, 2 xt, 3 yz, 4 yt, 5 zt
  const M3 Fxy = field_strength(g, c.U64, c.two_row != 0, x, 0, 1);
  const M3 Fxz = field_strength(g, c.U64, c.two_row != 0, x, 0, 2);
  const M3 Fxt = field_strength(g, c.U64, c.two_row != 0, x, 0, 3);
  const M3 Fyz = field_strength(g, c.U64, c.two_row != 0, x, 1, 2);
  const M3 Fyt = field_strength(g, c.U64, c.two_row != 0, x, 1, 3);
  const M3 Fzt = field_strength(g, c.U64, c.two_row != 0, x, 2, 3);

  const int T = g.L[3];
  bool bnd = false;
  if (g.bc == BC_SF) bnd = (co.t == 1) || (co.t == T - 1);
  if (g.bc == BC_OPEN) bnd = (co.t == 0) || (co.t == T - 1);
  const double d = 4.0 + c.m0 + (bnd ? (c.cF - 1.0) : 0.0);
  const double cc = 0.5 * c.csw;

#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const double sg = (b == 0) ? 1.0 : -1.0;
    // E_k = sg F_{tk} - B_k with F_{tk} = -F_{kt}
    M3 E1, E2, E3;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      E1.m[e] = csub(cscale(-sg, Fxt.m[e]), Fyz.m[e]);
      E2.m[e] = cadd(cscale(-sg, Fyt.m[e]), Fxz.m[e]);
      E3.m[e] = csub(cscale(-sg, Fzt.m[e]), Fxy.m[e]);
    }
    cd B[6][6];
    make_block(E1, E2, E3, cc, d, B);
    store_packed(c.C64 + par, s, 18 * b, B);
    if (c.C32) store_packed(c.C32 + par, s, 18 * b, B);
    if (c.C16) store_packed(c.C16 + par, s, 18 * b, B);
    if (p == 1 && c.mu == 0.0) {
      cd R[6][6];
      if (blk6::herm_inverse(B, R) == blk6::INV_SINGULAR) atomicOr(c.err_flag, 1);
      store_packed(c.Ci64, s, 18 * b, R);
      if (c.Ci32) store_packed(c.Ci32, s, 18 * b, R);
      if (c.Ci16) store_packed(c.Ci16, s, 18 * b, R);
    } else if (p == 1) {
      // twisted mass: the block of chirality b is B + i sg mu (g5 = sg on
      // it).  B is Hermitian, so (B + i m)^{-1} = (B^2 + mu^2)^{-1} (B - i m)
      // for m = +-mu (and the adjoint is the same with -m): the odd sites
      // store the Hermitian positive definite Q^{-1} = (B^2 + mu^2)^{-1}
      // (LDL^H), the hop kernels apply B and the i m term themselves
      cd Q[6][6], Qi[6][6];
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          cd v = {i == j ? c.mu * c.mu : 0.0, 0.0};
#pragma unroll
          for (int k = 0; k < 6; ++k) v = cadd(v, cmul(B[i][k], B[k][j]));
          Q[i][j] = v;
        }
      if (blk6::herm_inverse(Q, Qi) == blk6::INV_SINGULAR) atomicOr(c.err_flag, 1);
      store_packed(c.Ci64, s, 18 * b, Qi);
      if (c.Ci32) store_packed(c.Ci32, s, 18 * b, Qi);
      if (c.Ci16) store_packed(c.Ci16, s, 18 * b, Qi);
    }
  }
}

hipError_t launch_clover(const CloverLaunch& c, hipStream_t st) {
  dim3 grid((c.g.V2 + 127) / 128, 2);
  k_clover<<<grid, 128, 0, st>>>(c);
  return hipGetLastError();
}

}  // namespace lqcd
