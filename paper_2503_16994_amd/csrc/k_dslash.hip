// Hopping-term (Wilson "Dslash") kernels with the clover block fused in.
//
// One thread owns one output site of parity p_out and NR right-hand sides.
// For each of the 8 hops it loads the link once (9 site-coalesced complex
// loads), and for each of its NR rhs the neighbour spinor (12 loads), spin
// projects it to a half spinor, multiplies by U or U^+ and accumulates the
// reconstructed full spinor.  The clover block (two Hermitian 6x6 blocks,
// 36 complex loads) is likewise read once per thread for all NR rhs.  The
// only cross-lane work is the optional |out|^2 block reduction (wave64
// butterfly + LDS across the block's waves), which is deterministic.
//
// This is a 3x3 complex mat-vec stencil: there is no dense contraction to
// give to the matrix cores, so the kernel is bound by HBM bandwidth and is
// written for coalescing (unit-stride SoA loads over sites) and occupancy.
#include "lqcd_kernels.h"

namespace lqcd {

constexpr int kHopBlock = 256;

template <int BS>
__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) s += sh[i];
  }
  return s;
}

template <int MU, int DIR, int NR, typename A, typename SG, typename SI>
__device__ inline void hop_dir(cpx<A> (&acc)[NR][4][3], const HopLaunch& a, const SI* yb, int p,
                               int s, const Coord& c, int rhs0) {
  const KGeom& g = a.g;
  const int coord = coord_of(c, MU);
  const bool edge = (DIR > 0) ? (coord == g.L[MU] - 1) : (coord == 0);
  A pr = 1, pi = 0;
  if (edge) {
    pr = (A)(DIR > 0 ? g.fwd_re[MU] : g.bwd_re[MU]);
    pi = (A)(DIR > 0 ? g.fwd_im[MU] : g.bwd_im[MU]);
  }
  // Schroedinger functional: the backward hop from t = 1 lands on the
  // Dirichlet slice t = 0, whose field is ignored.
  if (MU == 3 && DIR < 0 && g.bc == BC_SF && c.t == 1) { pr = 0; pi = 0; }
  if (pr == (A)0 && pi == (A)0) return;

  const int sn = nb_index(g, s, c, MU, DIR);
  const size_t V2 = (size_t)g.V2;
  const SG* Ub = static_cast<const SG*>(a.U);
  const SG* up = (DIR > 0) ? Ub + (size_t)((p * 4 + MU) * 9) * V2 + s
                           : Ub + (size_t)(((1 - p) * 4 + MU) * 9) * V2 + sn;
  cpx<A> U[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) U[e] = ld(up + e * V2);

#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const SI* yp = yb + (size_t)(rhs0 + r) * a.y_rs + sn;
    cpx<A> psi[4][3];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      auto v = ld(yp + k * V2);
      psi[k / 3][k % 3] = {(A)v.re, (A)v.im};
    }
    cpx<A> h[2][3], w[2][3];
    spin_project<MU, DIR>(psi, h);
    if (DIR > 0) su3_mul(U, h, w);
    else su3_dag_mul(U, h, w);
    if (edge) {
      const cpx<A> ph = {pr, pi};
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int a2 = 0; a2 < 3; ++a2) w[q][a2] = cmul(ph, w[q][a2]);
    }
    spin_accumulate<MU, DIR>(acc[r], w);
  }
}

template <typename A, typename SG>
__device__ inline void load_block(const SG* C, int blk, size_t V2, int s, cpx<A> (&m)[18]) {
#pragma unroll
  for (int e = 0; e < 18; ++e) {
    auto v = ld(C + (size_t)(blk * 18 + e) * V2 + s);
    m[e] = {(A)v.re, (A)v.im};
  }
}

template <typename SG, typename SI, typename SO, int PRE, int POST, bool HOP, int NR>
__global__ __launch_bounds__(kHopBlock) void k_hop(const HopLaunch a) {
  using A = typename StoreTraits<SG>::acc;
  __shared__ double red[kHopBlock / 64];
  const KGeom& g = a.g;
  const int rhs0 = blockIdx.y * NR;
  if (a.done) {
    bool all = true;
#pragma unroll
    for (int r = 0; r < NR; ++r)
      all = all && (a.done[(rhs0 + r) * (int)(sizeof(CGState) / sizeof(int))] != 0);
    if (all) return;
  }
  // parity of this block's output sites and its site index
  int p = a.p_out, bx = blockIdx.x;
  if (a.both) {
    const int nbh = gridDim.x >> 1;
    p = (bx >= nbh) ? 1 : 0;
    bx -= p * nbh;
  }
  const int s = bx * kHopBlock + threadIdx.x;
  const bool active = s < g.V2;
  const size_t V2 = (size_t)g.V2;
  const SI* yb = static_cast<const SI*>(a.y);
  const SI* zb = static_cast<const SI*>(a.z);
  SO* ob = static_cast<SO*>(a.out);
  const SG* cpre = static_cast<const SG*>(a.Cpre);
  if (a.both) {
    yb += (1 - p) * a.par_stride;
    if (zb) zb += p * a.par_stride;
    ob += p * a.par_stride;
    if (cpre) cpre += p * a.cpre_par;
  }

  cpx<A> acc[NR][4][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int b = 0; b < 3; ++b) acc[r][q][b] = {(A)0, (A)0};

  Coord c;
  c.t = 0;
  if (active) {
    c = site_coord(g, s, p);
    if (HOP) {
      hop_dir<0, +1, NR, A, SG, SI>(acc, a, yb, p, s, c, rhs0);
      hop_dir<0, -1, NR, A, SG, SI>(acc, a, yb, p, s, c, rhs0);
      hop_dir<1, +1, NR, A, SG, SI>(acc, a, yb, p, s, c, rhs0);
      hop_dir<1, -1, NR, A, SG, SI>(acc, a, yb, p, s, c, rhs0);
      hop_dir<2, +1, NR, A, SG, SI>(acc, a, yb, p, s, c, rhs0);
      hop_dir<2, -1, NR, A, SG, SI>(acc, a, yb, p, s, c, rhs0);
      hop_dir<3, +1, NR, A, SG, SI>(acc, a, yb, p, s, c, rhs0);
      hop_dir<3, -1, NR, A, SG, SI>(acc, a, yb, p, s, c, rhs0);
    }
  }
  const bool masked = (g.bc == BC_SF) && (c.t == 0);
  const A scale = (A)a.scale;

  cpx<A> Cm[2][18];
  if (active && PRE == PRE_CLOV) {
    load_block(cpre, 0, V2, s, Cm[0]);
    load_block(cpre, 1, V2, s, Cm[1]);
  }
  cpx<A> Ci[2][18];
  if (active && POST == POST_CLOV) {
    load_block(static_cast<const SG*>(a.Cpost), 0, V2, s, Ci[0]);
    load_block(static_cast<const SG*>(a.Cpost), 1, V2, s, Ci[1]);
  }

#pragma unroll
  for (int r = 0; r < NR; ++r) {
    double nrm = 0.0;
    if (active) {
      cpx<A> v[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = cscale(scale, acc[r][k / 3][k % 3]);
      if (PRE != PRE_NONE) {
        const SI* zp = zb + (size_t)(rhs0 + r) * a.z_rs + s;
        cpx<A> zv[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          auto t = ld(zp + k * V2);
          zv[k] = {(A)t.re, (A)t.im};
        }
        if (PRE == PRE_IDENT) {
#pragma unroll
          for (int k = 0; k < 12; ++k) v[k] = cadd(v[k], zv[k]);
        } else {
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            cpx<A> in6[6], o6[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) in6[i] = zv[6 * b + i];
            herm6_mul(Cm[b], in6, o6);
#pragma unroll
            for (int i = 0; i < 6; ++i) v[6 * b + i] = cadd(v[6 * b + i], o6[i]);
          }
        }
      }
      if (POST == POST_CLOV) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          cpx<A> in6[6], o6[6];
#pragma unroll
          for (int i = 0; i < 6; ++i) in6[i] = v[6 * b + i];
          herm6_mul(Ci[b], in6, o6);
#pragma unroll
          for (int i = 0; i < 6; ++i) v[6 * b + i] = o6[i];
        }
      }
      if (a.g5) {
#pragma unroll
        for (int k = 6; k < 12; ++k) v[k] = {-v[k].re, -v[k].im};
      }
      if (masked) {
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = {(A)0, (A)0};
      }
      SO* op = ob + (size_t)(rhs0 + r) * a.out_rs + s;
#pragma unroll
      for (int k = 0; k < 12; ++k) st(op + k * V2, v[k]);
      if (a.partials) {
#pragma unroll
        for (int k = 0; k < 12; ++k)
          nrm += (double)v[k].re * (double)v[k].re + (double)v[k].im * (double)v[k].im;
      }
    }
    if (a.partials) {
      double bs = block_sum<kHopBlock>(nrm, red);
      if (threadIdx.x == 0) a.partials[(size_t)(rhs0 + r) * gridDim.x + blockIdx.x] = bs;
    }
  }
}

int hop_nblocks(const HopLaunch& h) {
  const int nb = (h.g.V2 + kHopBlock - 1) / kHopBlock;
  return h.both ? 2 * nb : nb;
}

template <typename SG, typename SI, typename SO, int PRE, int POST, bool HOP>
static hipError_t launch_nr(const HopLaunch& h, hipStream_t st) {
  const int nb = hop_nblocks(h);
  const int nr = h.nr_tile;
  if (h.nrhs % nr != 0) return hipErrorInvalidValue;
  dim3 grid(nb, h.nrhs / nr);
  switch (nr) {
    case 1: k_hop<SG, SI, SO, PRE, POST, HOP, 1><<<grid, kHopBlock, 0, st>>>(h); break;
    case 2: k_hop<SG, SI, SO, PRE, POST, HOP, 2><<<grid, kHopBlock, 0, st>>>(h); break;
    case 3: k_hop<SG, SI, SO, PRE, POST, HOP, 3><<<grid, kHopBlock, 0, st>>>(h); break;
    case 4: k_hop<SG, SI, SO, PRE, POST, HOP, 4><<<grid, kHopBlock, 0, st>>>(h); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename SG, typename SI, typename SO, int PRE, int POST, bool HOP>
static hipError_t launch_nr1(const HopLaunch& h, hipStream_t st) {
  if (h.nr_tile != 1) return hipErrorInvalidValue;
  dim3 grid(hop_nblocks(h), h.nrhs);
  k_hop<SG, SI, SO, PRE, POST, HOP, 1><<<grid, kHopBlock, 0, st>>>(h);
  return hipGetLastError();
}

// Dispatch on the operator shape; the two hot shapes (e->o with the clover
// inverse after, o->e with the clover before) get every rhs tile.
template <typename SG, typename SI, typename SO>
static hipError_t dispatch_mode(const HopLaunch& h, hipStream_t st) {
  if (h.hop && h.pre == PRE_NONE && h.post == POST_CLOV)
    return launch_nr<SG, SI, SO, PRE_NONE, POST_CLOV, true>(h, st);
  if (h.hop && h.pre == PRE_CLOV && h.post == POST_NONE)
    return launch_nr<SG, SI, SO, PRE_CLOV, POST_NONE, true>(h, st);
  if (h.hop && h.pre == PRE_IDENT && h.post == POST_NONE)
    return launch_nr1<SG, SI, SO, PRE_IDENT, POST_NONE, true>(h, st);
  if (h.hop && h.pre == PRE_IDENT && h.post == POST_CLOV)
    return launch_nr1<SG, SI, SO, PRE_IDENT, POST_CLOV, true>(h, st);
  if (!h.hop && h.pre == PRE_IDENT && h.post == POST_CLOV)
    return launch_nr1<SG, SI, SO, PRE_IDENT, POST_CLOV, false>(h, st);
  if (!h.hop && h.pre == PRE_CLOV && h.post == POST_NONE)
    return launch_nr1<SG, SI, SO, PRE_CLOV, POST_NONE, false>(h, st);
  if (h.hop && h.pre == PRE_NONE && h.post == POST_NONE)
    return launch_nr1<SG, SI, SO, PRE_NONE, POST_NONE, true>(h, st);
  return hipErrorInvalidValue;
}

hipError_t launch_hop(const HopLaunch& h, hipStream_t st) {
  if (h.g.V2 <= 0 || h.nrhs <= 0) return hipErrorInvalidValue;
  if (h.prec == P_F64 && h.in_prec == P_F64 && h.out_prec == P_F64)
    return dispatch_mode<double2, double2, double2>(h, st);
  if (h.prec == P_F32 && h.in_prec == P_F32 && h.out_prec == P_F32)
    return dispatch_mode<float2, float2, float2>(h, st);
  if (h.prec == P_BF16 && h.in_prec == P_BF16 && h.out_prec == P_BF16)
    return dispatch_mode<bf16x2, bf16x2, bf16x2>(h, st);
  if (h.prec == P_BF16 && h.in_prec == P_BF16 && h.out_prec == P_F32)
    return dispatch_mode<bf16x2, bf16x2, float2>(h, st);
  return hipErrorInvalidValue;
}

}  // namespace lqcd
