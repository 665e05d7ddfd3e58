// Hopping-term (Wilson "Dslash") kernels with the clover block fused in.
//
// Work decomposition.  A thread owns one output site of parity p_out and NR
// right-hand sides; RL consecutive lanes share one site and own RL different
// rhs groups (so a 128-thread workgroup covers 128/RL sites and RL*NR rhs;
// 128 rather than 256 threads gives the one-rhs launches on a 16^3x32 lattice
// two workgroups per CU instead of one).  Per
// hop a thread loads the link (9 site-coalesced complex loads, or 6 when the
// field keeps two rows per link and the third is rebuilt in registers; the RL
// lanes of a site issue identical addresses, which the memory pipeline serves once)
// and, for each of its NR rhs, the neighbour spinor (12 loads), spin-projects
// it to a half spinor, multiplies by U or U^+ and accumulates.  The clover
// blocks (two Hermitian 6x6 blocks) are loaded one chirality at a time and
// applied to all NR rhs.  Links and clover blocks are read once per launch, so
// they are loaded non-temporally, leaving L2 to the spinors that neighbouring
// sites re-read.  The only cross-lane work is the optional per-rhs |out|^2
// block reduction (wave64 butterfly over the lanes of one rhs, then LDS
// across the block's waves), which is deterministic.
//
// This is a 3x3 complex mat-vec stencil: there is no dense contraction to
// give to the matrix cores; the kernel is bound by HBM bandwidth and is
// written for coalescing (unit-stride SoA loads over sites), L2 reuse (the
// block orders below) and occupancy (RL instead of NR keeps registers low).
#include <type_traits>

#include "lqcd_kernels.h"

namespace lqcd {

constexpr int kHopBlock = 128;  // threads per workgroup

// Raw operands of one hop (the link and the NR neighbour spinors, in their
// storage types), so that a hop's loads can be issued before the arithmetic
// of the hop before it.
template <int NR, typename SG, typename SI>
struct HopOperands {
  SG u[9];
  SI y[NR][12];
};

template <typename S>
__device__ inline S raw_ld(const S* p) {
  return *p;
}
__device__ inline double2 raw_ld_nt(const double2* p) {
  nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
  return make_double2(v.x, v.y);
}
__device__ inline float2 raw_ld_nt(const float2* p) {
  nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
  return make_float2(v.x, v.y);
}
__device__ inline bf16x2 raw_ld_nt(const bf16x2* p) {
  return bf16x2{__builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p))};
}
template <typename A, typename S>
__device__ inline cpx<A> widen(const S& v) {
  const auto c = StoreTraits<S>::load(&v);
  return {(A)c.re, (A)c.im};
}

// Phase of the hop x -> x + DIR mu at a site: the boundary phase on the edge,
// zero where the hop is cut (the Schroedinger-functional backward hop from
// t = 1 lands on the Dirichlet slice t = 0, whose field is ignored).
template <int MU, int DIR, typename A>
__device__ inline bool hop_phase(const KGeom& g, const Coord& c, bool& edge, A& pr, A& pi) {
  const int coord = coord_of(c, MU);
  edge = (DIR > 0) ? (coord == g.L[MU] - 1) : (coord == 0);
  pr = 1;
  pi = 0;
  if (edge) {
    pr = (A)(DIR > 0 ? g.fwd_re[MU] : g.bwd_re[MU]);
    pi = (A)(DIR > 0 ? g.fwd_im[MU] : g.bwd_im[MU]);
  }
  if (MU == 3 && DIR < 0 && g.bc == BC_SF && c.t == 1) {
    pr = 0;
    pi = 0;
  }
  return !(pr == (A)0 && pi == (A)0);
}

template <int MU, int DIR, int NR, typename SG, typename SI>
__device__ inline void hop_fetch(HopOperands<NR, SG, SI>& f, const HopLaunch& a, const SI* yb, int p, int s,
                                 const Coord& c, int rhs0) {
  const KGeom& g = a.g;
  const int sn = nb_index(g, s, c, MU, DIR);
  const int ne = a.two_row ? 6 : 9;                // stored complex per link
  const size_t par = (size_t)4 * ne * g.V2p;      // one parity of the link field
  const SG* Ub = static_cast<const SG*>(a.U);
  const SG* up = (DIR > 0) ? Ub + p * par + tix(s, 4 * ne) + MU * ne * kTile
                           : Ub + (1 - p) * par + tix(sn, 4 * ne) + MU * ne * kTile;
#pragma unroll
  for (int e = 0; e < 6; ++e) f.u[e] = a.cached_gauge ? raw_ld(up + e * kTile) : raw_ld_nt(up + e * kTile);
  if (!a.two_row) {
#pragma unroll
    for (int e = 6; e < 9; ++e) f.u[e] = a.cached_gauge ? raw_ld(up + e * kTile) : raw_ld_nt(up + e * kTile);
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const SI* yp = yb + (size_t)(rhs0 + r) * a.y_rs + tix(sn, 12);
#pragma unroll
    for (int k = 0; k < 12; ++k) f.y[r][k] = raw_ld(yp + k * kTile);
  }
}

template <int MU, int DIR, int NR, typename A, typename SG, typename SI>
__device__ inline void hop_apply(cpx<A> (&acc)[NR][4][3], const HopOperands<NR, SG, SI>& f, const HopLaunch& a,
                                 const Coord& c) {
  bool edge;
  A pr, pi;
  if (!hop_phase<MU, DIR, A>(a.g, c, edge, pr, pi)) return;
  cpx<A> U[9];
#pragma unroll
  for (int e = 0; e < 6; ++e) U[e] = widen<A>(f.u[e]);
  if (a.two_row) {
    su3_third_row(U);
  } else {
#pragma unroll
    for (int e = 6; e < 9; ++e) U[e] = widen<A>(f.u[e]);
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    cpx<A> psi[4][3];
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k / 3][k % 3] = widen<A>(f.y[r][k]);
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

// Hop k of the eight: direction k / 2, forward for even k.
template <int K, int NR, typename SG, typename SI>
__device__ inline void fetch_k(HopOperands<NR, SG, SI>& f, const HopLaunch& a, const SI* yb, int p, int s,
                               const Coord& c, int rhs0) {
  hop_fetch<K / 2, (K & 1) ? -1 : 1, NR, SG, SI>(f, a, yb, p, s, c, rhs0);
}

// Hops K .. K1-1 in order, one hop ahead: the loads of hop k+1 are issued
// before the arithmetic of hop k (f[k & 1] holds hop k).  The accumulation
// order is that of the plain sequence.
template <int K, int K1, int NR, typename A, typename SG, typename SI>
__device__ inline void hops_ahead(cpx<A> (&acc)[NR][4][3], HopOperands<NR, SG, SI> (&f)[2], const HopLaunch& a,
                                  const SI* yb, int p, int s, const Coord& c, int rhs0) {
  if constexpr (K + 1 < K1) fetch_k<K + 1>(f[(K + 1) & 1], a, yb, p, s, c, rhs0);
  hop_apply<K / 2, (K & 1) ? -1 : 1, NR, A, SG, SI>(acc, f[K & 1], a, c);
  if constexpr (K + 1 < K1) hops_ahead<K + 1, K1>(acc, f, a, yb, p, s, c, rhs0);
}

// Hops K0 .. K1-1 accumulated into acc.  With AHEAD the loads run one hop
// ahead of the arithmetic (two hops' operands live in registers); without,
// each hop loads and computes in turn and a cut hop loads nothing.
template <bool AHEAD, int K0, int K1, int NR, typename A, typename SG, typename SI>
__device__ inline void hop_range(cpx<A> (&acc)[NR][4][3], const HopLaunch& a, const SI* yb, int p, int s,
                                 const Coord& c, int rhs0) {
  if constexpr (AHEAD) {
    HopOperands<NR, SG, SI> f[2];
    fetch_k<K0>(f[K0 & 1], a, yb, p, s, c, rhs0);
    hops_ahead<K0, K1>(acc, f, a, yb, p, s, c, rhs0);
  } else {
    HopOperands<NR, SG, SI> f;
    bool edge;
    A pr, pi;
    if (hop_phase<K0 / 2, (K0 & 1) ? -1 : 1, A>(a.g, c, edge, pr, pi)) {
      fetch_k<K0>(f, a, yb, p, s, c, rhs0);
      hop_apply<K0 / 2, (K0 & 1) ? -1 : 1, NR, A, SG, SI>(acc, f, a, c);
    }
    if constexpr (K0 + 1 < K1) hop_range<false, K0 + 1, K1, NR, A, SG, SI>(acc, a, yb, p, s, c, rhs0);
  }
}

// Loads one hop ahead where one hop's raw operands take at most 48 registers
// per lane (BF16 with up to 3 rhs per thread, FP32 with one): the
// reduced-precision multi-rhs launches are latency-bound, and FP64 would
// give up too much occupancy.
template <int NR, typename SG, typename SI>
constexpr bool kHopAhead = 9 * sizeof(SG) + 12 * NR * sizeof(SI) <= 192;

// out6 += i m in6 (m = +-mu: the twisted-mass term of one chirality block)
template <typename A>
__device__ inline void add_tm(A m, const cpx<A> (&in6)[6], cpx<A> (&o6)[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) o6[i] = {o6[i].re - m * in6[i].im, o6[i].im + m * in6[i].re};
}

template <typename A, typename SG>
__device__ inline void load_block(const SG* C, int blk, int s, bool cached, cpx<A> (&m)[18]) {
  const SG* c = C + tix(s, 36) + blk * 18 * kTile;
#pragma unroll
  for (int e = 0; e < 18; ++e) {
    auto v = cached ? ld(c + e * kTile) : ld_nt(c + e * kTile);
    m[e] = {(A)v.re, (A)v.im};
  }
}

// Mapping of the 1-D grid (nbs site blocks x ntiles rhs tiles) to work.
// Workgroup b runs on XCD b mod 8 (round-robin dispatch), each XCD with its
// own L2.
//   order 0: site block b mod nbs, rhs tile b / nbs (plain order);
//   order 1: XCD-contiguous: every XCD walks one contiguous range of
//            (site block, tile) pairs with the tiles of a site block adjacent;
//   order 2: XCD z-slabs: XCD x owns z-planes [x Lz/8, (x+1) Lz/8) for all t;
//            it walks, innermost first, the rhs tiles, the site blocks of a
//            (z, t) plane, the planes of its slab, then t.  The t-neighbours
//            of a site are then a slab plane (a few blocks) away.  Requires
//            Lz % 8 == 0 and a whole number of site blocks per (z, t) plane
//            (else order 1).
//   order 3: as 1, with the rhs tile outermost (the whole lattice per tile);
//   order 4: as 2, with the rhs tile outermost;
//   orders 5, 6: as 2 with slabs of 1 or 2 planes: XCD x sweeps t over the
//            planes z = d (x + 8 k) .. d (x + 8 k) + d - 1 for pass k = 0, 1,
//            ... (d = 1 or 2); a t-step then holds d/(Lz/8) of the data of
//            order 2, so the t-neighbours stay in L2 with many rhs per site,
//            at the price of z-neighbours in another XCD's L2 (6 requires
//            Lz % 16 == 0).
// Tile-inner orders read each link once for all tiles but need a reuse window
// holding all rhs; tile-outer orders read the links once per tile and keep
// the reuse window of a single tile.  A launch over both parities maps each parity like a one-parity launch (nb
// and nbs per parity); the parities alternate every round of eight
// workgroups (see hop_thread).
__device__ inline void block_order(const HopLaunch& a, int b, int nb, int nbs, int ntiles, int& sb, int& tile) {
  if (a.order == 0) {
    sb = b % nbs;
    tile = b / nbs;
    return;
  }
  const int x = b & 7, j = b >> 3;
  if (a.order == 3) {
    const int l = xcd_remap(b, nb);
    tile = l / nbs;
    sb = l % nbs;
    return;
  }
  if (a.order == 2 || a.order >= 4) {
    const int bpp = a.bpp, Lz = a.g.L[2];
    const int depth = (a.order == 5) ? 1 : (a.order == 6 ? 2 : (Lz >> 3));  // planes per slab
    int q;
    if (a.order != 4) {
      tile = j % ntiles;
      q = j / ntiles;
    } else {
      const int per_tile = nbs >> 3;  // site blocks per XCD and tile
      tile = j / per_tile;
      q = j % per_tile;
    }
    const int pb = q % bpp;
    q /= bpp;
    const int zl = q % depth;
    q /= depth;
    const int t = q % a.g.L[3];
    const int pass = q / a.g.L[3];  // 0 unless depth < Lz / 8
    sb = pb + bpp * (depth * (x + 8 * pass) + zl + Lz * t);
    return;
  }
  const int l = xcd_remap(b, nb);
  tile = l % ntiles;
  sb = l / ntiles;
}

// per-rhs block sum: lanes l and l' hold the same rhs iff l = l' mod RL
template <int RL>
__device__ inline double block_sum_rl(double v, double* sh) {
#pragma unroll
  for (int off = 32; off >= RL; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l < RL) sh[w * RL + l] = v;
  __syncthreads();
  double s = 0.0;
  if ((int)threadIdx.x < RL) {
#pragma unroll
    for (int i = 0; i < kHopBlock / 64; ++i) s += sh[i * RL + threadIdx.x];
  }
  return s;
}

// Everything a hop launch computes for one thread before the output stage:
// block decode, the 8 hops, the clover blocks.  Leaves the NR output
// spinors in v (scaled hop sum plus pre(z), then post), and the site, its
// coordinates and the rhs indices in the outputs.
struct ThreadSite {
  int sb, rhs_tile0, rhs0, s, p;
  int c0;  // first output component this thread owns (0, or 6 w when split)
  bool active, masked;
};

// Direction split (SPLIT; one rhs per thread only).  The two waves of a
// workgroup share its 64 sites: wave w computes the hops in directions 2w and
// 2w+1, the waves swap halves of their partial sums through LDS (xch, 2 x 6 x 64
// complex), and wave w then owns the six output components of chirality w
// (spins 2w, 2w+1) and their clover block.  Twice the waves per site at half
// the dependent loads each: for lattices too small to fill the GPU.  The hop
// sum is (x, y terms) + (z, t terms) instead of one chain over the eight, so
// results differ from the unsplit kernel in the last bits.
template <typename SG, typename SI, int PRE, int POST, bool HOP, int NR, int RL, bool SPLIT, bool TM, typename A>
__device__ inline bool hop_thread(const HopLaunch& a, ThreadSite& ts, cpx<A> (&v)[NR][12], cpx<A>* xch) {
  static_assert(!SPLIT || (NR == 1 && RL == 1 && HOP), "direction split: one rhs per thread");
  static_assert(!TM || (NR == 1 && RL == 1), "twisted mass: one rhs per thread");
  constexpr int SPB = SPLIT ? 64 : kHopBlock / RL;  // sites per block
  // wave index (uniform over the wave; only the split uses it)
  const int wv = SPLIT ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : 0;
  ts.c0 = 6 * wv;
  const KGeom& g = a.g;
  int tile, p = a.p_out, b = blockIdx.x, nb = gridDim.x, nbs = a.nbs;
  if (a.both) {
    // Both parities: with a whole number of XCD rounds per parity, the
    // parities alternate every XCD round (workgroups 8j .. 8j+7 run parity
    // j mod 2, one per XCD), so that each XCD handles parity-0 and parity-1
    // blocks of the same sites together and the links that a parity-1 site
    // reads backward (stored with its parity-0 neighbour) were just read
    // forward by the parity-0 block, and are L2 hits; otherwise parity 0
    // takes the first half of the grid and parity 1 the second.
    nb >>= 1;
    nbs >>= 1;
    if ((nb & 7) == 0) {
      const int j = b >> 3;
      p = j & 1;
      b = ((j >> 1) << 3) | (b & 7);
    } else {
      p = (b >= nb) ? 1 : 0;
      b -= p * nb;
    }
  }
  int bx;  // site block within the parity
  block_order(a, b, nb, nbs, a.nrhs / (NR * RL), bx, tile);
  ts.sb = p * nbs + bx;  // partial-sum slot
  const int lane_r = (RL > 1) ? (int)(threadIdx.x % RL) : 0;
  ts.rhs_tile0 = tile * NR * RL;
  ts.rhs0 = ts.rhs_tile0 + lane_r * NR;  // this lane's first rhs
  if (a.done) {
    bool all = true;
    for (int r = 0; r < NR * RL; ++r)
      all = all && (a.done[(ts.rhs_tile0 + r) * (int)(sizeof(CGState) / sizeof(int))] != 0);
    if (all) return false;
  }
  ts.p = p;
  const int s = bx * SPB + (SPLIT ? (int)(threadIdx.x & 63) : (int)(threadIdx.x / RL));
  ts.s = s;
  ts.active = s < g.V2;
  const SI* yb = static_cast<const SI*>(a.y);
  const SI* zb = static_cast<const SI*>(a.z);
  const SG* cpre = static_cast<const SG*>(a.Cpre);
  if (a.both) {
    yb += (1 - p) * a.par_stride;
    if (zb) zb += p * a.par_stride;
    if (cpre) cpre += p * a.cpre_par;
  }
  const int rhs0 = ts.rhs0;

  cpx<A> acc[NR][4][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int b = 0; b < 3; ++b) acc[r][q][b] = {(A)0, (A)0};

  Coord c;
  c.t = 0;
  if (ts.active) {
    c = site_coord(g, s, p);
    if (HOP) {
      constexpr bool AH = kHopAhead<NR, SG, SI>;
      if (!SPLIT) {
        hop_range<AH, 0, 8, NR, A, SG, SI>(acc, a, yb, p, s, c, rhs0);
      } else if (wv == 0) {
        hop_range<AH, 0, 4, NR, A, SG, SI>(acc, a, yb, p, s, c, rhs0);
      } else {
        hop_range<AH, 4, 8, NR, A, SG, SI>(acc, a, yb, p, s, c, rhs0);
      }
    }
  }
  ts.masked = (g.bc == BC_SF) && (c.t == 0);
  const A scale = (A)a.scale;

  if constexpr (SPLIT) {
    // region 0 of xch receives wave 1's spins 0, 1 (for wave 0), region 1
    // wave 0's spins 2, 3 (for wave 1); every thread of the workgroup gets here
    const int l = threadIdx.x & 63;
    if (wv == 0) {
#pragma unroll
      for (int k = 0; k < 6; ++k) xch[(6 + k) * 64 + l] = acc[0][2 + k / 3][k % 3];
    } else {
#pragma unroll
      for (int k = 0; k < 6; ++k) xch[k * 64 + l] = acc[0][k / 3][k % 3];
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int k = 0; k < 6; ++k) v[0][k] = cscale(scale, cadd(acc[0][k / 3][k % 3], xch[k * 64 + l]));
    } else {
#pragma unroll
      for (int k = 0; k < 6; ++k)
        v[0][k] = cscale(scale, cadd(xch[(6 + k) * 64 + l], acc[0][2 + k / 3][k % 3]));
    }
    if (ts.active && PRE != PRE_NONE) {
      cpx<A> Cm[18];
      if (PRE == PRE_CLOV) load_block(cpre, wv, s, a.cached_gauge != 0, Cm);
      const SI* zp = zb + (size_t)rhs0 * a.z_rs + tix(s, 12) + 6 * wv * kTile;
      cpx<A> in6[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        auto t = ld(zp + i * kTile);
        in6[i] = {(A)t.re, (A)t.im};
      }
      if (PRE == PRE_IDENT) {
#pragma unroll
        for (int i = 0; i < 6; ++i) v[0][i] = cadd(v[0][i], in6[i]);
      } else {
        cpx<A> o6[6];
        herm6_mul(Cm, in6, o6);
        if constexpr (TM) add_tm((A)(wv == 0 ? a.tm_mu : -a.tm_mu), in6, o6);
#pragma unroll
        for (int i = 0; i < 6; ++i) v[0][i] = cadd(v[0][i], o6[i]);
      }
    }
    if (ts.active && POST == POST_CLOV) {
      cpx<A> in6[6], o6[6], Ci[18];
#pragma unroll
      for (int i = 0; i < 6; ++i) in6[i] = v[0][i];
      if constexpr (TM) {  // (A + i m)^{-1} = Q^{-1} (A - i m), m = tm_mu g5
        load_block(static_cast<const SG*>(a.Ctm), wv, s, a.cached_gauge != 0, Ci);
        herm6_mul(Ci, in6, o6);
        add_tm((A)(wv == 0 ? -a.tm_mu : a.tm_mu), in6, o6);
#pragma unroll
        for (int i = 0; i < 6; ++i) in6[i] = o6[i];
      }
      load_block(static_cast<const SG*>(a.Cpost), wv, s, a.cached_gauge != 0, Ci);
      herm6_mul(Ci, in6, o6);
#pragma unroll
      for (int i = 0; i < 6; ++i) v[0][i] = o6[i];
    }
    if (a.g5 && wv == 1) {
#pragma unroll
      for (int k = 0; k < 6; ++k) v[0][k] = {-v[0][k].re, -v[0][k].im};
    }
    if (ts.masked) {
#pragma unroll
      for (int k = 0; k < 6; ++k) v[0][k] = {(A)0, (A)0};
    }
    return true;
  }

#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int k = 0; k < 12; ++k) v[r][k] = cscale(scale, acc[r][k / 3][k % 3]);
  if (ts.active && PRE != PRE_NONE) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cpx<A> Cm[18];
      if (PRE == PRE_CLOV) load_block(cpre, b, s, a.cached_gauge != 0, Cm);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const SI* zp = zb + (size_t)(rhs0 + r) * a.z_rs + tix(s, 12);
        cpx<A> in6[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          auto t = ld(zp + (6 * b + i) * kTile);
          in6[i] = {(A)t.re, (A)t.im};
        }
        if (PRE == PRE_IDENT) {
#pragma unroll
          for (int i = 0; i < 6; ++i) v[r][6 * b + i] = cadd(v[r][6 * b + i], in6[i]);
        } else {
          cpx<A> o6[6];
          herm6_mul(Cm, in6, o6);
          if constexpr (TM) add_tm((A)(b == 0 ? a.tm_mu : -a.tm_mu), in6, o6);
#pragma unroll
          for (int i = 0; i < 6; ++i) v[r][6 * b + i] = cadd(v[r][6 * b + i], o6[i]);
        }
      }
    }
  }
  if (TM && ts.active && POST == POST_CLOV) {
    // twisted mass: (A + i m)^{-1} = Q^{-1} (A - i m) per chirality
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      {
        cpx<A> Cm[18];
        load_block(static_cast<const SG*>(a.Ctm), b, s, a.cached_gauge != 0, Cm);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          cpx<A> in6[6], o6[6];
#pragma unroll
          for (int i = 0; i < 6; ++i) in6[i] = v[r][6 * b + i];
          herm6_mul(Cm, in6, o6);
          add_tm((A)(b == 0 ? -a.tm_mu : a.tm_mu), in6, o6);
#pragma unroll
          for (int i = 0; i < 6; ++i) v[r][6 * b + i] = o6[i];
        }
      }
      cpx<A> Ci[18];
      load_block(static_cast<const SG*>(a.Cpost), b, s, a.cached_gauge != 0, Ci);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        cpx<A> in6[6], o6[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) in6[i] = v[r][6 * b + i];
        herm6_mul(Ci, in6, o6);
#pragma unroll
        for (int i = 0; i < 6; ++i) v[r][6 * b + i] = o6[i];
      }
    }
  } else if (ts.active && POST == POST_CLOV) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cpx<A> Ci[18];
      load_block(static_cast<const SG*>(a.Cpost), b, s, a.cached_gauge != 0, Ci);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        cpx<A> in6[6], o6[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) in6[i] = v[r][6 * b + i];
        herm6_mul(Ci, in6, o6);
#pragma unroll
        for (int i = 0; i < 6; ++i) v[r][6 * b + i] = o6[i];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (a.g5) {
#pragma unroll
      for (int k = 6; k < 12; ++k) v[r][k] = {-v[r][k].re, -v[r][k].im};
    }
    if (ts.masked) {
#pragma unroll
      for (int k = 0; k < 12; ++k) v[r][k] = {(A)0, (A)0};
    }
  }
  return true;
}

// alpha = rr / pAp for the rhs this workgroup owns (see HopLaunch::alpha_cg):
// a fixed-order sum (thread-strided partial sums, wavefront butterfly, the
// waves in order)
__device__ inline void fused_alpha(const HopLaunch& a, double* sh) {
  for (int r = blockIdx.x; r < a.nrhs; r += gridDim.x) {
    CGState& c = a.alpha_cg[r];
    if (c.done) {  // uniform over the workgroup
      if (a.alpha_slot >= 0 && threadIdx.x == 0) c.alpha_w[a.alpha_slot] = 0.0;
      continue;
    }
    const double* p = a.alpha_parts + (size_t)r * a.alpha_nparts;
    double acc = 0.0;
    for (int i = threadIdx.x; i < a.alpha_nparts; i += kHopBlock) acc += p[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double v = 0.0;
      for (int w = 0; w < kHopBlock / 64; ++w) v += sh[w];  // waves in order
      c.pAp = v;
      c.alpha = (v > 0.0) ? c.rr / v : 0.0;
      c.rr_prev = c.rr;
      if (a.alpha_slot >= 0) c.alpha_w[a.alpha_slot] = c.alpha;
    }
  }
  __syncthreads();
}

template <typename SG, typename SI, typename SO, int PRE, int POST, bool HOP, int NR, int RL, bool SPLIT, bool TM>
__global__ __launch_bounds__(kHopBlock) void k_hop(const HopLaunch a) {
  using A = typename StoreTraits<SG>::acc;
  constexpr int NC = SPLIT ? 6 : 12;  // output components per thread
  __shared__ double red[(kHopBlock / 64) * RL > 4 ? (kHopBlock / 64) * RL : 4];
  __shared__ cpx<A> xch[SPLIT ? 2 * 6 * 64 : 1];
  if (a.alpha_cg) fused_alpha(a, red);
  ThreadSite ts;
  cpx<A> v[NR][12];
  if (!hop_thread<SG, SI, PRE, POST, HOP, NR, RL, SPLIT, TM>(a, ts, v, xch)) return;
  SO* ob = static_cast<SO*>(a.out);
  if (a.both) ob += ts.p * a.par_stride;
  // padding sites of the last tile (inactive, v = 0) are written too, so
  // every output vector holds zeros there
  const bool store = ts.s < a.g.V2p;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    double nrm = 0.0;
    if (store) {
      SO* op = ob + (size_t)(ts.rhs0 + r) * a.out_rs + tix(ts.s, 12) + ts.c0 * kTile;
      if (a.nt_out) {
#pragma unroll
        for (int k = 0; k < NC; ++k) st_nt(op + k * kTile, v[r][k]);
      } else {
#pragma unroll
        for (int k = 0; k < NC; ++k) st(op + k * kTile, v[r][k]);
      }
      if (a.partials) {
#pragma unroll
        for (int k = 0; k < NC; ++k)
          nrm += (double)v[r][k].re * (double)v[r][k].re + (double)v[r][k].im * (double)v[r][k].im;
      }
    }
    if (a.partials) {
      const double bs = block_sum_rl<RL>(nrm, red);
      if ((int)threadIdx.x < RL)
        a.partials[(size_t)(ts.rhs_tile0 + (int)threadIdx.x * NR + r) * a.nbs + ts.sb] = bs;
    }
  }
}

// The last hop of a CG iteration fused with the vector update: with
// Ap = g5 (A_ee q + 1/2 H t) computed in registers, every rhs that is not done
// gets x += alpha p, r -= alpha Ap (x, r of type SV, p of the operator's
// input type SI: the very vector the operator was applied to) and the
// per-block |r|^2 partial.  Ap is never stored.  With x null the x update is
// left to a later flush of the deferred updates.
template <typename SG, typename SI, typename SV, int NR, int RL, bool SPLIT, bool TM>
__global__ __launch_bounds__(kHopBlock) void k_hop_xr(const HopLaunch a) {
  using A = typename StoreTraits<SG>::acc;
  using AV = typename StoreTraits<SV>::acc;
  constexpr int NC = SPLIT ? 6 : 12;  // output components per thread
  __shared__ double red[(kHopBlock / 64) * RL];
  __shared__ cpx<A> xch[SPLIT ? 2 * 6 * 64 : 1];
  ThreadSite ts;
  cpx<A> v[NR][12];
  if (!hop_thread<SG, SI, PRE_CLOV, POST_NONE, true, NR, RL, SPLIT, TM>(a, ts, v, xch)) return;
  SV* xb = static_cast<SV*>(a.xr_x);
  SV* rb = static_cast<SV*>(a.xr_r);
  const SI* pb = static_cast<const SI*>(a.xr_p);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int q = ts.rhs0 + r;
    const CGState& cs = a.cg[q];
    double nrm = 0.0;
    if (ts.active && !cs.done) {
      const double alpha_d = cs.alpha;
      const AV alpha = (AV)alpha_d;
      const size_t o = (size_t)q * a.xr_rs + tix(ts.s, 12) + ts.c0 * kTile,
                   ox = (size_t)q * a.xr_xrs + tix(ts.s, 12) + ts.c0 * kTile;
      if (xb) {  // uniform over the launch
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          auto pv = ld(pb + o + k * kTile);
          auto xv = ld(xb + ox + k * kTile);
          xv.re += (AV)alpha_d * pv.re;
          xv.im += (AV)alpha_d * pv.im;
          st(xb + ox + k * kTile, xv);
        }
      }
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        auto rv = ld(rb + o + k * kTile);
        rv.re -= alpha * (AV)v[r][k].re;
        rv.im -= alpha * (AV)v[r][k].im;
        st(rb + o + k * kTile, rv);
        nrm += (double)rv.re * (double)rv.re + (double)rv.im * (double)rv.im;
      }
    }
    const double bs = block_sum_rl<RL>(nrm, red);
    if ((int)threadIdx.x < RL)
      a.partials[(size_t)(ts.rhs_tile0 + (int)threadIdx.x * NR + r) * a.nbs + ts.sb] = bs;
  }
}

static int sites_per_block(int rl, bool split = false) {
  return split ? 64 : kHopBlock / (rl < 1 ? 1 : rl);
}
// the direction split applies to launches with one rhs per thread only
static bool split_on(const HopLaunch& h) { return h.dir_split && h.nr_tile == 1 && h.rhs_lanes == 1; }
// twisted-mass kernels exist for one rhs per thread (the launch helpers of
// the library set nr_tile = rhs_lanes = 1 whenever mu != 0)
static bool tm_on(const HopLaunch& h) { return h.tm_post != 0 || h.tm_mu != 0.0; }

// Unused dynamic LDS that caps the workgroups resident per CU (160 KiB of LDS
// per CU, plus each workgroup's small static reduction array): level 1 -> 4,
// 2 -> 3, 3 -> 2 workgroups.  A smaller live set per XCD keeps more neighbour
// spinors in L2 when every site carries many rhs.
static unsigned lds_cap_bytes(int level) {
  switch (level) {
    case 1: return 39u << 10;
    case 2: return 53u << 10;
    case 3: return 63u << 10;
    default: return 0u;
  }
}

// most partial sums per rhs any hop launch writes on V2 sites per parity:
// 4 rhs lanes (fewest sites per workgroup), or both parities split
int hop_max_parts(long V2) {
  const long one = (V2 + sites_per_block(4) - 1) / sites_per_block(4);
  const long both = 2 * ((V2 + sites_per_block(1, true) - 1) / sites_per_block(1, true));
  return (int)(one > both ? one : both);
}

int hop_nblocks(const HopLaunch& h) {
  const int spb = sites_per_block(h.rhs_lanes, split_on(h));
  const int nb = (h.g.V2 + spb - 1) / spb;
  return h.both ? 2 * nb : nb;
}

// per-rhs partial sums a launch of the tiled shapes writes (its site blocks)
int hop_nparts(const HopLaunch& h0) {
  HopLaunch h = h0;
  if (h.prec == P_F64) h.rhs_lanes = 1;
  return hop_nblocks(h);
}

// fill in nbs/bpp and validate the block order for this launch
static bool prepare(HopLaunch& h) {
  if (h.rhs_lanes != 1 && h.rhs_lanes != 2 && h.rhs_lanes != 4) return false;
  if (h.nr_tile < 1 || h.nr_tile > 3) return false;
  if (h.nrhs % (h.nr_tile * h.rhs_lanes) != 0) return false;
  h.nbs = hop_nblocks(h);
  h.lds_cap = lds_cap_bytes(h.occ_cap);
  const int spb = sites_per_block(h.rhs_lanes, split_on(h));
  const long P = (long)h.g.Lxh * h.g.L[1];
  h.bpp = (int)(P / spb);
  const bool slab_ok = (h.g.L[2] % 8) == 0 && (P % spb) == 0;
  if ((h.order == 2 || h.order == 5) && !slab_ok) h.order = 1;
  if (h.order == 6 && !(slab_ok && (h.g.L[2] % 16) == 0)) h.order = 1;
  if (h.order == 4 && !slab_ok) h.order = 3;
  if (h.order < 0 || h.order > 6) h.order = 1;
  return true;
}

template <typename SG, typename SI, typename SO, int PRE, int POST, bool HOP, int RL>
static hipError_t launch_rl(const HopLaunch& h, hipStream_t st) {
  const unsigned grid = (unsigned)h.nbs * (unsigned)(h.nrhs / (h.nr_tile * RL));
  switch (h.nr_tile) {
    case 1:
      if constexpr (RL == 1) {
        if (tm_on(h)) {
          if (split_on(h))
            k_hop<SG, SI, SO, PRE, POST, HOP, 1, 1, true, true><<<grid, kHopBlock, h.lds_cap, st>>>(h);
          else
            k_hop<SG, SI, SO, PRE, POST, HOP, 1, 1, false, true><<<grid, kHopBlock, h.lds_cap, st>>>(h);
          break;
        }
        if (split_on(h)) {
          k_hop<SG, SI, SO, PRE, POST, HOP, 1, 1, true, false><<<grid, kHopBlock, h.lds_cap, st>>>(h);
          break;
        }
      }
      if (tm_on(h)) return hipErrorInvalidValue;
      k_hop<SG, SI, SO, PRE, POST, HOP, 1, RL, false, false><<<grid, kHopBlock, h.lds_cap, st>>>(h);
      break;
    case 2:
      if (tm_on(h)) return hipErrorInvalidValue;
      k_hop<SG, SI, SO, PRE, POST, HOP, 2, RL, false, false><<<grid, kHopBlock, h.lds_cap, st>>>(h);
      break;
    case 3:
      if (tm_on(h)) return hipErrorInvalidValue;
      k_hop<SG, SI, SO, PRE, POST, HOP, 3, RL, false, false><<<grid, kHopBlock, h.lds_cap, st>>>(h);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// the two hot shapes: every (nr_tile, rhs_lanes); FP64 only with rhs_lanes 1
template <typename SG, typename SI, typename SO, int PRE, int POST, bool HOP>
static hipError_t launch_tiled(const HopLaunch& h0, hipStream_t st) {
  HopLaunch h = h0;
  if (std::is_same<SG, double2>::value) h.rhs_lanes = 1;
  if (!prepare(h)) return hipErrorInvalidValue;
  if constexpr (std::is_same<SG, double2>::value) {
    return launch_rl<SG, SI, SO, PRE, POST, HOP, 1>(h, st);
  } else {
    switch (h.rhs_lanes) {
      case 1: return launch_rl<SG, SI, SO, PRE, POST, HOP, 1>(h, st);
      case 2: return launch_rl<SG, SI, SO, PRE, POST, HOP, 2>(h, st);
      case 4: return launch_rl<SG, SI, SO, PRE, POST, HOP, 4>(h, st);
      default: return hipErrorInvalidValue;
    }
  }
}

template <typename SG, typename SI, typename SV, int RL>
static hipError_t launch_xr_rl(const HopLaunch& h, hipStream_t st) {
  const unsigned grid = (unsigned)h.nbs * (unsigned)(h.nrhs / (h.nr_tile * RL));
  switch (h.nr_tile) {
    case 1:
      if constexpr (RL == 1) {
        if (tm_on(h)) {
          if (split_on(h))
            k_hop_xr<SG, SI, SV, 1, 1, true, true><<<grid, kHopBlock, h.lds_cap, st>>>(h);
          else
            k_hop_xr<SG, SI, SV, 1, 1, false, true><<<grid, kHopBlock, h.lds_cap, st>>>(h);
          break;
        }
        if (split_on(h)) {
          k_hop_xr<SG, SI, SV, 1, 1, true, false><<<grid, kHopBlock, h.lds_cap, st>>>(h);
          break;
        }
      }
      if (tm_on(h)) return hipErrorInvalidValue;
      k_hop_xr<SG, SI, SV, 1, RL, false, false><<<grid, kHopBlock, h.lds_cap, st>>>(h);
      break;
    case 2:
      if (tm_on(h)) return hipErrorInvalidValue;
      k_hop_xr<SG, SI, SV, 2, RL, false, false><<<grid, kHopBlock, h.lds_cap, st>>>(h);
      break;
    case 3:
      if (tm_on(h)) return hipErrorInvalidValue;
      k_hop_xr<SG, SI, SV, 3, RL, false, false><<<grid, kHopBlock, h.lds_cap, st>>>(h);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename SG, typename SI, typename SV>
static hipError_t launch_xr(const HopLaunch& h0, hipStream_t st) {
  HopLaunch h = h0;
  if (std::is_same<SG, double2>::value) h.rhs_lanes = 1;
  if (!prepare(h) || h.both || !h.partials || !h.cg) return hipErrorInvalidValue;
  if constexpr (std::is_same<SG, double2>::value) {
    return launch_xr_rl<SG, SI, SV, 1>(h, st);
  } else {
    switch (h.rhs_lanes) {
      case 1: return launch_xr_rl<SG, SI, SV, 1>(h, st);
      case 2: return launch_xr_rl<SG, SI, SV, 2>(h, st);
      case 4: return launch_xr_rl<SG, SI, SV, 4>(h, st);
      default: return hipErrorInvalidValue;
    }
  }
}

hipError_t launch_hop_xr(const HopLaunch& h, hipStream_t st) {
  if (h.g.V2 <= 0 || h.nrhs <= 0 || !h.hop || h.pre != PRE_CLOV || h.post != POST_NONE)
    return hipErrorInvalidValue;
  if (h.prec == P_F64 && h.in_prec == P_F64 && h.xr_prec == P_F64)
    return launch_xr<double2, double2, double2>(h, st);
  if (h.prec == P_F32 && h.in_prec == P_F32 && h.xr_prec == P_F32)
    return launch_xr<float2, float2, float2>(h, st);
  if (h.prec == P_BF16 && h.in_prec == P_BF16 && h.xr_prec == P_F32)
    return launch_xr<bf16x2, bf16x2, float2>(h, st);
  return hipErrorInvalidValue;
}

// set-up shapes (source preparation, reconstruction, block application):
// one rhs per thread
template <typename SG, typename SI, typename SO, int PRE, int POST, bool HOP>
static hipError_t launch_single(const HopLaunch& h0, hipStream_t st) {
  HopLaunch h = h0;
  h.nr_tile = 1;
  h.rhs_lanes = 1;
  h.dir_split = 0;
  if (!prepare(h)) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)h.nbs * (unsigned)h.nrhs;
  if (tm_on(h))
    k_hop<SG, SI, SO, PRE, POST, HOP, 1, 1, false, true><<<grid, kHopBlock, 0, st>>>(h);
  else
    k_hop<SG, SI, SO, PRE, POST, HOP, 1, 1, false, false><<<grid, kHopBlock, 0, st>>>(h);
  return hipGetLastError();
}

template <typename SG, typename SI, typename SO>
static hipError_t dispatch_mode(const HopLaunch& h, hipStream_t st) {
  if (h.hop && h.pre == PRE_NONE && h.post == POST_CLOV)
    return launch_tiled<SG, SI, SO, PRE_NONE, POST_CLOV, true>(h, st);
  if (h.hop && h.pre == PRE_CLOV && h.post == POST_NONE)
    return launch_tiled<SG, SI, SO, PRE_CLOV, POST_NONE, true>(h, st);
  if (h.hop && h.pre == PRE_IDENT && h.post == POST_NONE)
    return launch_single<SG, SI, SO, PRE_IDENT, POST_NONE, true>(h, st);
  if (h.hop && h.pre == PRE_IDENT && h.post == POST_CLOV)
    return launch_single<SG, SI, SO, PRE_IDENT, POST_CLOV, true>(h, st);
  if (!h.hop && h.pre == PRE_IDENT && h.post == POST_CLOV)
    return launch_single<SG, SI, SO, PRE_IDENT, POST_CLOV, false>(h, st);
  if (!h.hop && h.pre == PRE_CLOV && h.post == POST_NONE)
    return launch_single<SG, SI, SO, PRE_CLOV, POST_NONE, false>(h, st);
  if (h.hop && h.pre == PRE_NONE && h.post == POST_NONE)
    return launch_single<SG, SI, SO, PRE_NONE, POST_NONE, true>(h, st);
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
