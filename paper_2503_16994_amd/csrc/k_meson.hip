// Meson two-point functions from a 12-column point-source propagator.
//
// The paper's propagator functions produce the quark propagator from which
// correlation functions are contracted (Sec. 3.3); this is that contraction.
// With S(x)[al a][be c] = psi_(3 be + c)(x)[al][a] (column j = 3 s + c of the
// propagator: source spin s, colour c), the colour-traced spin tensor per
// time slice
//   G_t[al][be][al'][be'] = sum_{x in slice t} sum_{a, c} S(x)[al a][be c] conj(S(x)[al' a][be' c])
// carries every meson correlator: by g5-hermiticity the backward propagator
// is g5 S^+ g5, so
//   C_t(Gamma, Gamma') = sum_x tr[Gamma S(x) Gamma' g5 S(x)^+ g5]
//                      = sum Gamma[de][al] Gamma'[be][ga] g5[ga] g5[de] G_t[al][be][de][ga].
// Gamma is named by a 4-bit mask m: Gamma_m = g_t^{m3} g_x^{m0} g_y^{m1} g_z^{m2}
// (ordered product, t first, so m = 15 is g5 = g_t g_x g_y g_z).
//
// Kernel 1 (k_meson_partial): workgroup (b, t) stages 16 sites at a time of
// its 256-site chunk of slice t in LDS (12 x 12 complex each, read coalesced
// from the canonical columns); thread (site lane, al, al') accumulates the
// 16 (be, be') entries; the 16 site lanes of a pair are summed by a wave
// butterfly and the waves in order, giving one partial G per chunk.
// Kernel 2 (k_meson_reduce): workgroup t sums the chunk partials of every
// entry in chunk order and contracts with the requested Gamma pairs (a fixed-
// order block sum).  FP64 throughout; deterministic, no atomics.  The work
// is a stream of 2304 B per site (HBM bound at FP64: ~9 flop/B).
#include "lqcd_kernels.h"

namespace lqcd {

constexpr int kMesonBlock = 256;
constexpr int kMesonPass = 16;    // sites staged per pass
constexpr int kMesonChunk = 256;  // sites per workgroup

using cd = cpx<double>;

__global__ __launch_bounds__(kMesonBlock) void k_meson_partial(const double2* __restrict__ psi, long V, long V3,
                                                               int nchunk, double2* partials) {
  __shared__ double2 S[kMesonPass][12][12];  // [site][row al a][col be c]
  const int t = blockIdx.y, b = blockIdx.x, tid = threadIdx.x;
  const long s0 = (long)t * V3 + (long)b * kMesonChunk;
  const long s_end = min((long)(t + 1) * V3, s0 + kMesonChunk);
  const int sl = tid >> 4, pr = tid & 15, al = pr >> 2, al2 = pr & 3;
  cd acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = {0.0, 0.0};
  for (long base = s0; base < s_end; base += kMesonPass) {
    // e = (column j, site, component k): consecutive e are consecutive in
    // memory within a column (16 sites x 12 components)
    for (int e = tid; e < kMesonPass * 144; e += kMesonBlock) {
      const int j = e / (kMesonPass * 12), r = e % (kMesonPass * 12);
      const int site = r / 12, k = r % 12;
      const long x = base + site;
      double2 v = make_double2(0.0, 0.0);
      if (x < s_end) v = psi[((size_t)j * V + x) * 12 + k];
      S[site][k][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cd r1[12], r2[12];
#pragma unroll
      for (int q = 0; q < 12; ++q) {
        const double2 u = S[sl][3 * al + a][q], w = S[sl][3 * al2 + a][q];
        r1[q] = {u.x, u.y};
        r2[q] = {w.x, w.y};
      }
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int be = 0; be < 4; ++be)
#pragma unroll
          for (int be2 = 0; be2 < 4; ++be2)
            acc[be][be2] = cmacc(acc[be][be2], r2[3 * be2 + c], r1[3 * be + c]);  // += r1 conj(r2), four FMAs
    }
    __syncthreads();
  }
  // sum the 16 site lanes of every (al, al') pair: lanes pr + 16 k of a wave,
  // then the four waves in order
  __shared__ double2 red[kMesonBlock / 64][16][16];
  const int w = tid >> 6, l = tid & 63;
#pragma unroll
  for (int be = 0; be < 4; ++be)
#pragma unroll
    for (int be2 = 0; be2 < 4; ++be2) {
      cd v = acc[be][be2];
#pragma unroll
      for (int off = 16; off < 64; off <<= 1) {
        v.re += __shfl_xor(v.re, off, 64);
        v.im += __shfl_xor(v.im, off, 64);
      }
      if (l < 16) red[w][pr][4 * be + be2] = make_double2(v.re, v.im);
    }
  __syncthreads();
  // output entry i = ((al be) al' be'): pair (al, al'), component (be, be')
  const int i = tid;
  const int oal = i >> 6, obe = (i >> 4) & 3, oal2 = (i >> 2) & 3, obe2 = i & 3;
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int ww = 0; ww < kMesonBlock / 64; ++ww) {
    const double2 v = red[ww][4 * oal + oal2][4 * obe + obe2];
    s.x += v.x;
    s.y += v.y;
  }
  partials[((size_t)t * nchunk + b) * 256 + i] = s;
}

// chiral-basis gamma matrices g_x, g_y, g_z, g_t (mu = 0..3): each has one
// non-zero per row; row r of g_mu holds `val` in column `col`
__device__ inline void gamma_row(int mu, int r, int& col, cd& val) {
  switch (mu) {
    case 0:  // g_x = [[0, -i s1], [i s1, 0]]
      col = 3 - r;
      val = (r < 2) ? cd{0.0, -1.0} : cd{0.0, 1.0};
      break;
    case 1:  // g_y = [[0, -i s2], [i s2, 0]]
      col = 3 - r;
      val = (r == 0 || r == 3) ? cd{-1.0, 0.0} : cd{1.0, 0.0};
      break;
    case 2:  // g_z = [[0, -i s3], [i s3, 0]]
      col = r ^ 2;
      val = (r == 0 || r == 3) ? cd{0.0, -1.0} : cd{0.0, 1.0};
      break;
    default:  // g_t = [[0, -1], [-1, 0]]
      col = r ^ 2;
      val = cd{-1.0, 0.0};
      break;
  }
}

// entry (r, c) of Gamma_m = g_t^{m3} g_x^{m0} g_y^{m1} g_z^{m2}: the single
// non-zero of row r is followed through the ordered product
__device__ inline cd gamma_entry(int m, int r, int c) {
  int k = r;
  cd p = {1.0, 0.0};
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int mu = (f == 0) ? 3 : f - 1;
    if ((m >> mu) & 1) {
      int col;
      cd v;
      gamma_row(mu, k, col, v);
      p = cmul(p, v);
      k = col;
    }
  }
  return (k == c) ? p : cd{0.0, 0.0};
}

struct MesonPairs {
  int n;
  int m[kMaxMesonPairs][2];
  double scale;                   // applied to every correlator
  double2* out[kMaxMesonPairs];   // correlator of pair p: out[p][t]
};

__global__ __launch_bounds__(256) void k_meson_reduce(const double2* __restrict__ partials, int nchunk, double2* G,
                                                      MesonPairs pairs) {
  __shared__ double red[2][4];
  const int t = blockIdx.x, i = threadIdx.x;
  double2 g = make_double2(0.0, 0.0);
  for (int b = 0; b < nchunk; ++b) {
    const double2 v = partials[((size_t)t * nchunk + b) * 256 + i];
    g.x += v.x;
    g.y += v.y;
  }
  if (G) G[(size_t)t * 256 + i] = g;
  // entry i = G[al][be][de][ga]
  const int al = i >> 6, be = (i >> 4) & 3, de = (i >> 2) & 3, ga = i & 3;
  const double g5ga = ga < 2 ? 1.0 : -1.0, g5de = de < 2 ? 1.0 : -1.0;
  for (int p = 0; p < pairs.n; ++p) {
    const cd coef = cmul(gamma_entry(pairs.m[p][0], de, al), gamma_entry(pairs.m[p][1], be, ga));
    cd term = cmul(coef, cd{g.x, g.y});
    term = {term.re * g5ga * g5de, term.im * g5ga * g5de};
    double re = term.re, im = term.im;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      re += __shfl_xor(re, off, 64);
      im += __shfl_xor(im, off, 64);
    }
    const int w = i >> 6, l = i & 63;
    if (l == 0) {
      red[0][w] = re;
      red[1][w] = im;
    }
    __syncthreads();
    if (i == 0) {
      double sr = 0.0, si = 0.0;
      for (int ww = 0; ww < 4; ++ww) {
        sr += red[0][ww];
        si += red[1][ww];
      }
      pairs.out[p][t] = make_double2(pairs.scale * sr, pairs.scale * si);
    }
    __syncthreads();
  }
}

int meson_nchunk(long V3) { return (int)((V3 + kMesonChunk - 1) / kMesonChunk); }

hipError_t launch_meson(const KGeom& g, const double2* psi, int npairs, const int* masks, double2* const* outs,
                        double scale, double2* G, double2* scratch, hipStream_t st) {
  if (npairs < 0 || npairs > kMaxMesonPairs) return hipErrorInvalidValue;
  const long V3 = (long)g.L[0] * g.L[1] * g.L[2], V = V3 * g.L[3];
  const int nchunk = meson_nchunk(V3);
  MesonPairs pairs;
  pairs.n = npairs;
  pairs.scale = scale;
  for (int p = 0; p < kMaxMesonPairs; ++p) {
    pairs.m[p][0] = p < npairs ? masks[2 * p] : 0;
    pairs.m[p][1] = p < npairs ? masks[2 * p + 1] : 0;
    pairs.out[p] = p < npairs ? outs[p] : nullptr;
  }
  k_meson_partial<<<dim3(nchunk, g.L[3]), kMesonBlock, 0, st>>>(psi, V, V3, nchunk, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_meson_reduce<<<g.L[3], 256, 0, st>>>(scratch, nchunk, G, pairs);
  return hipGetLastError();
}

}  // namespace lqcd
