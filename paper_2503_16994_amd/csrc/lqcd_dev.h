// Device-side building blocks of the gfx950 Wilson-clover library: storage
// types, even-odd site geometry, spin projection of the hopping term and the
// 6x6 clover block algebra.
//
// Internal layout, tiled structure-of-arrays: the sites of one parity are
// grouped in tiles of kTile = 64 (one wavefront), and a field with nc complex
// components per site stores tile after tile, each tile as nc rows of 64
// sites.  Component k of site s is at  tix(s, nc) + 64 k,  so the 64 lanes of
// a wavefront that own the 64 sites of a tile make unit-stride loads, and the
// components of a site are 512 B (FP32) to 1 KiB (FP64) apart instead of a
// whole parity plane (a power of two of MiB on the benchmark lattices, which
// maps every component of a site onto the same L2 set).
//   site index     s = lex >> 1 within parity p = (x+y+z+t) & 1, where
//                  lex = x + Lx (y + Ly (z + Lz t)), V2 = V/2 sites and
//                  V2p = V2 rounded up to a multiple of kTile (padding sites
//                  hold zeros in vectors and are never read by the stencil);
//   spinor         psi[rhs][p] = 12-component field, k = 3*spin + colour;
//   links          U[p] = 36-component field, component 9*mu + 3*a + b;
//   clover block   C[p] = 36-component field, component 18*blk + e,
//                  blk = chirality (spins 0,1 / 2,3), e = 0..2 the six real
//                  diagonal entries as pairs, e = 3..17 the 15 complex
//                  strictly-lower entries (i>j) in row order (Hermitian);
//   odd inverse    Ci = 36-component field (odd sites) with the same packing.
// Every stored element is one complex number: double2 (FP64), float2 (FP32)
// or two bfloat16 packed in a uint32 (BF16, re in the low half).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lqcd {

constexpr int kTile = 64;

// offset of component 0 of site s in a tiled field with nc components per site
__host__ __device__ inline size_t tix(size_t s, int nc) {
  return (s >> 6) * (size_t)(nc * kTile) + (s & (kTile - 1));
}
__host__ __device__ inline long padded_sites(long v2) { return (v2 + kTile - 1) / kTile * kTile; }

// ---------------------------------------------------------------------------
// Storage element types and conversion to the accumulation type
// ---------------------------------------------------------------------------
struct bf16x2 {
  uint32_t v;
};

template <typename A>
struct cpx {
  A re, im;
};

template <typename S>
struct StoreTraits;

template <>
struct StoreTraits<double2> {
  using acc = double;
  __device__ static inline cpx<double> load(const double2* p) {
    double2 v = *p;
    return {v.x, v.y};
  }
  __device__ static inline void store(double2* p, cpx<double> c) { *p = make_double2(c.re, c.im); }
  __device__ static inline void store(double2* p, cpx<float> c) {
    *p = make_double2((double)c.re, (double)c.im);
  }
};

template <>
struct StoreTraits<float2> {
  using acc = float;
  __device__ static inline cpx<float> load(const float2* p) {
    float2 v = *p;
    return {v.x, v.y};
  }
  __device__ static inline void store(float2* p, cpx<float> c) { *p = make_float2(c.re, c.im); }
  __device__ static inline void store(float2* p, cpx<double> c) {
    *p = make_float2((float)c.re, (float)c.im);
  }
};

// float -> bfloat16 with round-to-nearest-even on the bits; NaN stays NaN
// (quiet bit set).  Used where the source is an FP64 value: its FP32
// rounding comes first, and bit arithmetic keeps the compiler from folding
// the two roundings into one FP64 -> BF16 conversion.
__device__ __host__ inline uint32_t f32_to_bf16_rne(float f) {
  union {
    float f;
    uint32_t u;
  } x;
  x.f = f;
  uint32_t u = x.u;
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (u >> 16) | 0x40u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// two floats -> packed bfloat16 pair (re low, im high) by the hardware
// conversion (v_cvt_pk_bf16_f32), round to nearest even; a NaN stays a NaN
__device__ inline uint32_t pack_bf16x2(float re, float im) {
  const __bf16 lo = (__bf16)re, hi = (__bf16)im;
  return (uint32_t)__builtin_bit_cast(unsigned short, lo) |
         ((uint32_t)__builtin_bit_cast(unsigned short, hi) << 16);
}

__device__ __host__ inline float bf16_to_f32(uint32_t h) {
  union {
    float f;
    uint32_t u;
  } x;
  x.u = h << 16;
  return x.f;
}

template <>
struct StoreTraits<bf16x2> {
  using acc = float;
  __device__ static inline cpx<float> load(const bf16x2* p) {
    uint32_t v = p->v;
    return {__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u)};
  }
  __device__ static inline void store(bf16x2* p, cpx<float> c) { p->v = pack_bf16x2(c.re, c.im); }
  // FP64 -> FP32 -> BF16, each step round-to-nearest-even
  __device__ static inline void store(bf16x2* p, cpx<double> c) {
    p->v = f32_to_bf16_rne((float)c.re) | (f32_to_bf16_rne((float)c.im) << 16);
  }
};

template <typename S>
__device__ inline auto ld(const S* p) {
  return StoreTraits<S>::load(p);
}

// Non-temporal load (read-once data: links, clover blocks).  The streaming
// hint keeps such lines from displacing the spinor lines that neighbouring
// sites re-read from L2.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
__device__ inline cpx<double> ld_nt(const double2* p) {
  nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
  return {v.x, v.y};
}
__device__ inline cpx<float> ld_nt(const float2* p) {
  nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
  return {v.x, v.y};
}
__device__ inline cpx<float> ld_nt(const bf16x2* p) {
  uint32_t v = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p));
  return {__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u)};
}

// Non-temporal (streaming) vector stores: for outputs written once per
// launch, so that they do not displace re-read data from L2.
template <typename A>
__device__ inline void st_nt(double2* p, cpx<A> c) {
  nt_d2 v = {(double)c.re, (double)c.im};
  __builtin_nontemporal_store(v, reinterpret_cast<nt_d2*>(p));
}
template <typename A>
__device__ inline void st_nt(float2* p, cpx<A> c) {
  nt_f2 v = {(float)c.re, (float)c.im};
  __builtin_nontemporal_store(v, reinterpret_cast<nt_f2*>(p));
}
template <typename A>
__device__ inline void st_nt(bf16x2* p, cpx<A> c) {
  bf16x2 t;
  StoreTraits<bf16x2>::store(&t, c);  // the rounding of an ordinary store
  __builtin_nontemporal_store(t.v, reinterpret_cast<uint32_t*>(p));
}

// Block index remap for the 8 XCDs of the MI355X.  Workgroups are handed to
// the XCDs round-robin (workgroup b runs on XCD b mod 8, each XCD with its own
// L2); this maps the b-th workgroup to logical block
//   start(b mod 8) + b/8,  start(x) = x*floor(nb/8) + min(x, nb mod 8),
// a bijection on [0, nb) under which every XCD walks one contiguous range of
// sites, so the y, z and t neighbours of its sites are mostly its own.
__device__ inline int xcd_remap(int b, int nb) {
  const int x = b & 7, j = b >> 3, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + j;
}
template <typename S, typename A>
__device__ inline void st(S* p, cpx<A> c) {
  StoreTraits<S>::store(p, c);
}

// ---------------------------------------------------------------------------
// Complex helpers
// ---------------------------------------------------------------------------
template <typename A>
__device__ inline cpx<A> cadd(cpx<A> a, cpx<A> b) { return {a.re + b.re, a.im + b.im}; }
template <typename A>
__device__ inline cpx<A> csub(cpx<A> a, cpx<A> b) { return {a.re - b.re, a.im - b.im}; }
template <typename A>
__device__ inline cpx<A> cmul(cpx<A> a, cpx<A> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename A>
__device__ inline cpx<A> cmulc(cpx<A> a, cpx<A> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// a + i b, a - i b
template <typename A>
__device__ inline cpx<A> cadd_i(cpx<A> a, cpx<A> b) { return {a.re - b.im, a.im + b.re}; }
template <typename A>
__device__ inline cpx<A> csub_i(cpx<A> a, cpx<A> b) { return {a.re + b.im, a.im - b.re}; }
template <typename A>
__device__ inline cpx<A> cscale(A s, cpx<A> a) { return {s * a.re, s * a.im}; }
// acc + a b and acc + conj(a) b with each of the four real products fused
// into the running sum (four FMAs per complex multiply-accumulate; the
// expression acc + (a b) would cost a multiply, an FMA and an add per part)
template <typename A>
__device__ inline cpx<A> cmac(cpx<A> acc, cpx<A> a, cpx<A> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}
template <typename A>
__device__ inline cpx<A> cmacc(cpx<A> acc, cpx<A> a, cpx<A> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
  return acc;
}

// Third row of an SU(3) matrix (row major, m[3 a + b]) from its first two.
// For a unitary matrix of determinant one the inverse is both the adjoint
// and the adjugate, so each entry of row 2 is the complex conjugate of its
// cofactor: row 2 = conj(row 0 x row 1).
template <typename A>
__device__ inline void su3_third_row(cpx<A> (&m)[9]) {
  const cpx<A> c0 = cmac(cmul(m[1], m[5]), cpx<A>{-m[2].re, -m[2].im}, m[4]);
  const cpx<A> c1 = cmac(cmul(m[2], m[3]), cpx<A>{-m[0].re, -m[0].im}, m[5]);
  const cpx<A> c2 = cmac(cmul(m[0], m[4]), cpx<A>{-m[1].re, -m[1].im}, m[3]);
  m[6] = {c0.re, -c0.im};
  m[7] = {c1.re, -c1.im};
  m[8] = {c2.re, -c2.im};
}

// ---------------------------------------------------------------------------
// Fast unsigned division by a runtime constant (Granlund-Montgomery style):
// q = (umulhi(n, m) + n) >> l  with l = ceil(log2 d), m = 2^32 (2^l - d)/d + 1,
// exact for n < 2^31.
// ---------------------------------------------------------------------------
struct FastDiv {
  uint32_t d, m, l;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  f.l = l;
  f.m = (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
  return f;
}

__device__ inline uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return (__umulhi(n, f.m) + n) >> f.l;
}

// ---------------------------------------------------------------------------
// Geometry passed to every kernel by value
// ---------------------------------------------------------------------------
enum { BC_PERIODIC = 0, BC_SF = 1, BC_OPEN = 2 };

struct KGeom {
  int L[4];       // Lx, Ly, Lz, T
  int Lxh;        // Lx / 2
  int V2;         // sites per parity
  int V2p;        // V2 rounded up to a multiple of kTile (tiled field rows)
  int sy, sz, st; // eo-index strides of y, z, t: Lxh, Lxh*Ly, Lxh*Ly*Lz
  int bc;
  FastDiv div_xh, div_y, div_z;
  // Boundary phase factors: fwd[mu] multiplies the forward hop leaving
  // x_mu = L_mu-1, bwd[mu] the backward hop leaving x_mu = 0.  Zero = cut.
  double fwd_re[4], fwd_im[4], bwd_re[4], bwd_im[4];
};

struct Coord {
  int x, y, z, t, xh;
};

__device__ inline Coord site_coord(const KGeom& g, int s, int p) {
  Coord c;
  uint32_t q1 = fdiv((uint32_t)s, g.div_xh);
  c.xh = s - (int)q1 * g.Lxh;
  uint32_t q2 = fdiv(q1, g.div_y);
  c.y = (int)q1 - (int)q2 * g.L[1];
  uint32_t q3 = fdiv(q2, g.div_z);
  c.z = (int)q2 - (int)q3 * g.L[2];
  c.t = (int)q3;
  c.x = 2 * c.xh + ((c.y + c.z + c.t + p) & 1);
  return c;
}

// eo index of the neighbour x + dir*mu (opposite parity)
__device__ inline int nb_index(const KGeom& g, int s, const Coord& c, int mu, int dir) {
  if (mu == 0) {
    int x = c.x + dir;
    x = (x == g.L[0]) ? 0 : ((x < 0) ? g.L[0] - 1 : x);
    return s - c.xh + (x >> 1);
  }
  int coord = (mu == 1) ? c.y : (mu == 2 ? c.z : c.t);
  int stride = (mu == 1) ? g.sy : (mu == 2 ? g.sz : g.st);
  int Lm = g.L[mu];
  if (dir > 0) return (coord == Lm - 1) ? s - (Lm - 1) * stride : s + stride;
  return (coord == 0) ? s + (Lm - 1) * stride : s - stride;
}

__device__ inline int coord_of(const Coord& c, int mu) {
  return mu == 0 ? c.x : (mu == 1 ? c.y : (mu == 2 ? c.z : c.t));
}

// ---------------------------------------------------------------------------
// Spin structure of the hopping term, chiral basis.
// Forward hop:  (1 - g_mu) U psi(x+mu): project psi to h = (h0, h1), multiply by
// U, then the lower two spins are a fixed combination of U h.
// Backward hop: (1 + g_mu) U^+ psi(x-mu), same pattern with the opposite sign.
// ---------------------------------------------------------------------------
template <int MU, int DIR, typename A>
__device__ inline void spin_project(const cpx<A> (&p)[4][3], cpx<A> (&h)[2][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (DIR > 0) {
      if (MU == 0) { h[0][a] = cadd_i(p[0][a], p[3][a]); h[1][a] = cadd_i(p[1][a], p[2][a]); }
      if (MU == 1) { h[0][a] = cadd(p[0][a], p[3][a]);   h[1][a] = csub(p[1][a], p[2][a]); }
      if (MU == 2) { h[0][a] = cadd_i(p[0][a], p[2][a]); h[1][a] = csub_i(p[1][a], p[3][a]); }
      if (MU == 3) { h[0][a] = cadd(p[0][a], p[2][a]);   h[1][a] = cadd(p[1][a], p[3][a]); }
    } else {
      if (MU == 0) { h[0][a] = csub_i(p[0][a], p[3][a]); h[1][a] = csub_i(p[1][a], p[2][a]); }
      if (MU == 1) { h[0][a] = csub(p[0][a], p[3][a]);   h[1][a] = cadd(p[1][a], p[2][a]); }
      if (MU == 2) { h[0][a] = csub_i(p[0][a], p[2][a]); h[1][a] = cadd_i(p[1][a], p[3][a]); }
      if (MU == 3) { h[0][a] = csub(p[0][a], p[2][a]);   h[1][a] = csub(p[1][a], p[3][a]); }
    }
  }
}

// acc += reconstruct(w), w = U h (forward) or U^+ h (backward)
template <int MU, int DIR, typename A>
__device__ inline void spin_accumulate(cpx<A> (&acc)[4][3], const cpx<A> (&w)[2][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc[0][a] = cadd(acc[0][a], w[0][a]);
    acc[1][a] = cadd(acc[1][a], w[1][a]);
    if (DIR > 0) {
      if (MU == 0) { acc[2][a] = csub_i(acc[2][a], w[1][a]); acc[3][a] = csub_i(acc[3][a], w[0][a]); }
      if (MU == 1) { acc[2][a] = csub(acc[2][a], w[1][a]);   acc[3][a] = cadd(acc[3][a], w[0][a]); }
      if (MU == 2) { acc[2][a] = csub_i(acc[2][a], w[0][a]); acc[3][a] = cadd_i(acc[3][a], w[1][a]); }
      if (MU == 3) { acc[2][a] = cadd(acc[2][a], w[0][a]);   acc[3][a] = cadd(acc[3][a], w[1][a]); }
    } else {
      if (MU == 0) { acc[2][a] = cadd_i(acc[2][a], w[1][a]); acc[3][a] = cadd_i(acc[3][a], w[0][a]); }
      if (MU == 1) { acc[2][a] = cadd(acc[2][a], w[1][a]);   acc[3][a] = csub(acc[3][a], w[0][a]); }
      if (MU == 2) { acc[2][a] = cadd_i(acc[2][a], w[0][a]); acc[3][a] = csub_i(acc[3][a], w[1][a]); }
      if (MU == 3) { acc[2][a] = csub(acc[2][a], w[0][a]);   acc[3][a] = csub(acc[3][a], w[1][a]); }
    }
  }
}

// w = U h  (U row-major 3x3)
template <typename A>
__device__ inline void su3_mul(const cpx<A> (&U)[9], const cpx<A> (&h)[2][3], cpx<A> (&w)[2][3]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<A> v = cmul(U[3 * a + 0], h[s][0]);
      v = cmac(v, U[3 * a + 1], h[s][1]);
      v = cmac(v, U[3 * a + 2], h[s][2]);
      w[s][a] = v;
    }
}

// w = U^+ h
template <typename A>
__device__ inline void su3_dag_mul(const cpx<A> (&U)[9], const cpx<A> (&h)[2][3],
                                   cpx<A> (&w)[2][3]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<A> v = cmulc(U[0 * 3 + a], h[s][0]);
      v = cmacc(v, U[1 * 3 + a], h[s][1]);
      v = cmacc(v, U[2 * 3 + a], h[s][2]);
      w[s][a] = v;
    }
}

// ---------------------------------------------------------------------------
// Hermitian 6x6 block times a 6-vector (packed storage described above)
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int tri_index(int i, int j) { return 3 + i * (i - 1) / 2 + j; }

template <typename A>
__device__ inline void herm6_mul(const cpx<A> (&m)[18], const cpx<A> (&v)[6], cpx<A> (&o)[6]) {
  A d[6] = {m[0].re, m[0].im, m[1].re, m[1].im, m[2].re, m[2].im};
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    cpx<A> acc = cscale(d[i], v[i]);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if (j < i) acc = cmac(acc, m[tri_index(i, j)], v[j]);
      if (j > i) acc = cmacc(acc, m[tri_index(j, i)], v[j]);
    }
    o[i] = acc;
  }
}

}  // namespace lqcd
