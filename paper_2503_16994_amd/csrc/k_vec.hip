// Layout conversion, BLAS-1 and CG scalar kernels.
//
// Reductions: every kernel that produces a sum writes one FP64 partial per
// block (wave64 butterfly, then LDS across the block's waves); a single
// block then adds the partials in a fixed order.  No atomics, so every
// result is bitwise reproducible run to run, and independent of what else
// runs on the device.
#include "lqcd_kernels.h"

namespace lqcd {

constexpr int kVecBlock = 256;
constexpr int kVecMaxBlocks = 2048;

__device__ inline double block_sum256(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = sh[0] + sh[1] + sh[2] + sh[3];
  return s;
}

// ---------------------------------------------------------------------------
// Gauge import
// ---------------------------------------------------------------------------
__global__ void k_import_gauge(KGeom g, const double2* __restrict__ Uc, double2* U64, float2* U32,
                               bf16x2* U16, bool two_row, int* bad) {
  const long V = 2L * g.V2;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;  // (site, mu)
  if (i >= 4 * V) return;
  const long lex = i >> 2;
  const int mu = (int)(i & 3);
  const int x = (int)(lex % g.L[0]);
  long r = lex / g.L[0];
  const int y = (int)(r % g.L[1]);
  r /= g.L[1];
  const int z = (int)(r % g.L[2]);
  const int t = (int)(r / g.L[2]);
  const int p = (x + y + z + t) & 1;
  const long s = lex >> 1;
  const bool zero = (g.bc == BC_OPEN) && (mu == 3) && (t == g.L[3] - 1);
  const int ne = two_row ? 6 : 9;  // stored complex per link
  const size_t base = (size_t)p * 4 * ne * g.V2p + tix(s, 4 * ne) + mu * ne * kTile;
  cpx<double> m[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    const double2 v = zero ? make_double2(0.0, 0.0) : Uc[i * 9 + e];
    m[e] = {v.x, v.y};
  }
  for (int e = 0; e < ne; ++e) {
    const size_t o = base + e * kTile;
    U64[o] = make_double2(m[e].re, m[e].im);
    if (U32) st(U32 + o, m[e]);
    if (U16) st(U16 + o, m[e]);
  }
  if (two_row) {
    cpx<double> w[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) w[e] = m[e];
    su3_third_row(w);
    bool off = false;
#pragma unroll
    for (int e = 6; e < 9; ++e) off = off || !(hypot(w[e].re - m[e].re, w[e].im - m[e].im) <= 1e-10);
    if (off) *bad = 1;  // every writer stores the same value
  }
}

hipError_t launch_import_gauge(const KGeom& g, const double2* Uc, double2* U64, float2* U32,
                               bf16x2* U16, bool two_row, int* bad, hipStream_t st) {
  if (two_row && !bad) return hipErrorInvalidValue;
  const long n = 4L * 2 * g.V2;
  k_import_gauge<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(g, Uc, U64, U32, U16, two_row, bad);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Spinor pack / unpack: canonical [rhs][lex][12] <-> internal [rhs][p] tiled
// 12-component fields.  Pack also zeroes the padding sites of both parities.
// ---------------------------------------------------------------------------
template <typename S>
__global__ void k_pack(KGeom g, const double2* __restrict__ canon, S* out, bool g5) {
  const long V = 2L * g.V2;
  const long lex = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  const size_t vec = (size_t)r * 24 * g.V2p;
  if (lex >= V) {
    const long pad = g.V2p - g.V2, j = lex - V;
    if (j >= 2 * pad) return;
    const long ps = j / pad, sp = g.V2 + j % pad;
    S* dst = out + vec + (size_t)ps * 12 * g.V2p + tix(sp, 12);
#pragma unroll
    for (int k = 0; k < 12; ++k) st(dst + k * kTile, cpx<double>{0.0, 0.0});
    return;
  }
  const int x = (int)(lex % g.L[0]);
  long q = lex / g.L[0];
  const int y = (int)(q % g.L[1]);
  q /= g.L[1];
  const int z = (int)(q % g.L[2]);
  const int t = (int)(q / g.L[2]);
  const int p = (x + y + z + t) & 1;
  const long s = lex >> 1;
  const double2* src = canon + ((size_t)r * V + lex) * 12;
  S* dst = out + vec + (size_t)p * 12 * g.V2p + tix(s, 12);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    double2 v = src[k];
    if (g5 && k >= 6) v = make_double2(-v.x, -v.y);
    st(dst + k * kTile, cpx<double>{v.x, v.y});
  }
}

template <typename S>
__global__ void k_unpack(KGeom g, const S* __restrict__ in, double2* canon) {
  const long V = 2L * g.V2;
  const long lex = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (lex >= V) return;
  const int x = (int)(lex % g.L[0]);
  long q = lex / g.L[0];
  const int y = (int)(q % g.L[1]);
  q /= g.L[1];
  const int z = (int)(q % g.L[2]);
  const int t = (int)(q / g.L[2]);
  const int p = (x + y + z + t) & 1;
  const long s = lex >> 1;
  const S* src = in + (size_t)r * 24 * g.V2p + (size_t)p * 12 * g.V2p + tix(s, 12);
  double2* dst = canon + ((size_t)r * V + lex) * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    auto v = ld(src + k * kTile);
    dst[k] = make_double2((double)v.re, (double)v.im);
  }
}

hipError_t launch_pack(const KGeom& g, const double2* canon, void* internal, int prec, int nrhs,
                       bool g5, hipStream_t st) {
  const long n = 2L * g.V2p;  // every site of both parities, padding included
  dim3 grid((unsigned)((n + 255) / 256), nrhs);
  if (prec == P_F64) k_pack<double2><<<grid, 256, 0, st>>>(g, canon, (double2*)internal, g5);
  else if (prec == P_F32) k_pack<float2><<<grid, 256, 0, st>>>(g, canon, (float2*)internal, g5);
  else k_pack<bf16x2><<<grid, 256, 0, st>>>(g, canon, (bf16x2*)internal, g5);
  return hipGetLastError();
}

hipError_t launch_unpack(const KGeom& g, const void* internal, int prec, double2* canon, int nrhs,
                         hipStream_t st) {
  const long V = 2L * g.V2;
  dim3 grid((unsigned)((V + 255) / 256), nrhs);
  if (prec == P_F64) k_unpack<double2><<<grid, 256, 0, st>>>(g, (const double2*)internal, canon);
  else if (prec == P_F32) k_unpack<float2><<<grid, 256, 0, st>>>(g, (const float2*)internal, canon);
  else k_unpack<bf16x2><<<grid, 256, 0, st>>>(g, (const bf16x2*)internal, canon);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// BLAS-1 on flat arrays (n complex per rhs; rhs stride rs elements)
// ---------------------------------------------------------------------------
int blas_nblocks(long n) {
  long nb = (n + kVecBlock - 1) / kVecBlock;
  return (int)(nb < kVecMaxBlocks ? nb : kVecMaxBlocks);
}

template <typename S>
__global__ void k_norm2(const S* __restrict__ x, long n, long rs, double* partials) {
  __shared__ double sh[4];
  const int r = blockIdx.y;
  const S* xr = x + (size_t)r * rs;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * kVecBlock + threadIdx.x; i < n; i += (long)gridDim.x * kVecBlock) {
    auto v = ld(xr + i);
    acc += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
  }
  double b = block_sum256(acc, sh);
  if (threadIdx.x == 0) partials[(size_t)r * gridDim.x + blockIdx.x] = b;
}

hipError_t launch_norm2(const void* x, int prec, long n, long rs, int nrhs, double* partials,
                        hipStream_t st) {
  dim3 grid(blas_nblocks(n), nrhs);
  if (prec == P_F64) k_norm2<double2><<<grid, kVecBlock, 0, st>>>((const double2*)x, n, rs, partials);
  else if (prec == P_F32) k_norm2<float2><<<grid, kVecBlock, 0, st>>>((const float2*)x, n, rs, partials);
  else k_norm2<bf16x2><<<grid, kVecBlock, 0, st>>>((const bf16x2*)x, n, rs, partials);
  return hipGetLastError();
}

// fixed-order sum of nparts partials by one block per rhs
__device__ inline double sum_partials(const double* p, int nparts, double* sh) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kVecBlock) acc += p[i];
  double s = block_sum256(acc, sh);
  __shared__ double out;
  if (threadIdx.x == 0) out = s;
  __syncthreads();
  return out;
}

__global__ void k_reduce(const double* partials, int nparts, double* dst) {
  __shared__ double sh[4];
  const int r = blockIdx.x;
  double s = sum_partials(partials + (size_t)r * nparts, nparts, sh);
  if (threadIdx.x == 0) dst[r] = s;
}

hipError_t launch_reduce(const double* partials, int nparts, int nrhs, double* dst, hipStream_t st) {
  k_reduce<<<nrhs, kVecBlock, 0, st>>>(partials, nparts, dst);
  return hipGetLastError();
}

// ---- generic elementwise ---------------------------------------------------
template <typename SX, typename SY>
__global__ void k_axpby(double a, const SX* __restrict__ x, double b, SY* y, long n, long rsx,
                        long rsy) {
  const int q = blockIdx.y;
  for (long i = (long)blockIdx.x * kVecBlock + threadIdx.x; i < n; i += (long)gridDim.x * kVecBlock) {
    auto xv = ld(x + (size_t)q * rsx + i);
    auto yv = ld(y + (size_t)q * rsy + i);
    cpx<double> o = {a * (double)xv.re + b * (double)yv.re, a * (double)xv.im + b * (double)yv.im};
    st(y + (size_t)q * rsy + i, o);
  }
}

template <typename SX, typename SY>
__global__ void k_convert(const SX* __restrict__ x, SY* y, long n, long rsx, long rsy) {
  const int q = blockIdx.y;
  for (long i = (long)blockIdx.x * kVecBlock + threadIdx.x; i < n; i += (long)gridDim.x * kVecBlock) {
    auto xv = ld(x + (size_t)q * rsx + i);
    st(y + (size_t)q * rsy + i, cpx<double>{(double)xv.re, (double)xv.im});
  }
}

#define LQCD_CONVERT_CASE(XP, YP, SXT, SYT)                                                 \
  if (xprec == XP && yprec == YP) {                                                        \
    k_convert<SXT, SYT><<<grid, kVecBlock, 0, st>>>((const SXT*)x, (SYT*)y, n, rsx, rsy); \
    return hipGetLastError();                                                              \
  }

hipError_t launch_convert(const void* x, int xprec, void* y, int yprec, long n, long rsx, long rsy,
                          int nrhs, hipStream_t st) {
  dim3 grid(blas_nblocks(n), nrhs);
  LQCD_CONVERT_CASE(P_F64, P_F64, double2, double2)
  LQCD_CONVERT_CASE(P_F64, P_F32, double2, float2)
  LQCD_CONVERT_CASE(P_F64, P_BF16, double2, bf16x2)
  LQCD_CONVERT_CASE(P_F32, P_F64, float2, double2)
  LQCD_CONVERT_CASE(P_F32, P_F32, float2, float2)
  LQCD_CONVERT_CASE(P_F32, P_BF16, float2, bf16x2)
  LQCD_CONVERT_CASE(P_BF16, P_F32, bf16x2, float2)
  LQCD_CONVERT_CASE(P_BF16, P_F64, bf16x2, double2)
  return hipErrorInvalidValue;
}
#undef LQCD_CONVERT_CASE

hipError_t launch_axpby(double a, const void* x, int xprec, double b, void* y, int yprec, long n,
                        long rsx, long rsy, int nrhs, hipStream_t st) {
  dim3 grid(blas_nblocks(n), nrhs);
  if (xprec == P_F64 && yprec == P_F64)
    k_axpby<double2, double2><<<grid, kVecBlock, 0, st>>>(a, (const double2*)x, b, (double2*)y, n, rsx, rsy);
  else if (xprec == P_F32 && yprec == P_F64)
    k_axpby<float2, double2><<<grid, kVecBlock, 0, st>>>(a, (const float2*)x, b, (double2*)y, n, rsx, rsy);
  else if (xprec == P_F32 && yprec == P_F32)
    k_axpby<float2, float2><<<grid, kVecBlock, 0, st>>>(a, (const float2*)x, b, (float2*)y, n, rsx, rsy);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// out = x - y with partial |out|^2
__global__ void k_sub_norm(const double2* __restrict__ x, const double2* __restrict__ y, double2* out,
                           long n, long rs, double* partials) {
  __shared__ double sh[4];
  const int q = blockIdx.y;
  const size_t o = (size_t)q * rs;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * kVecBlock + threadIdx.x; i < n; i += (long)gridDim.x * kVecBlock) {
    double2 a = x[o + i], b = y[o + i];
    double2 d = make_double2(a.x - b.x, a.y - b.y);
    out[o + i] = d;
    acc += d.x * d.x + d.y * d.y;
  }
  double b = block_sum256(acc, sh);
  if (threadIdx.x == 0) partials[(size_t)q * gridDim.x + blockIdx.x] = b;
}

hipError_t launch_sub_norm(const double2* x, const double2* y, double2* out, long n, long rs, int nrhs,
                           double* partials, hipStream_t st) {
  dim3 grid(blas_nblocks(n), nrhs);
  k_sub_norm<<<grid, kVecBlock, 0, st>>>(x, y, out, n, rs, partials);
  return hipGetLastError();
}

// zero fill with a kernel (graph-capturable, unlike a memset node)
__global__ void k_fill_zero(uint4* p, size_t n16) {
  for (size_t i = (size_t)blockIdx.x * kVecBlock + threadIdx.x; i < n16; i += (size_t)gridDim.x * kVecBlock)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}
__global__ void k_fill_zero_bytes(unsigned char* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kVecBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kVecBlock)
    p[i] = 0;
}

hipError_t launch_fill_zero(void* x, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  if (((uintptr_t)x % 16) == 0 && bytes % 16 == 0) {
    size_t n16 = bytes / 16;
    size_t nb = (n16 + kVecBlock - 1) / kVecBlock;
    if (nb > kVecMaxBlocks) nb = kVecMaxBlocks;
    k_fill_zero<<<(unsigned)nb, kVecBlock, 0, st>>>((uint4*)x, n16);
  } else {
    size_t nb = (bytes + kVecBlock - 1) / kVecBlock;
    if (nb > kVecMaxBlocks) nb = kVecMaxBlocks;
    k_fill_zero_bytes<<<(unsigned)nb, kVecBlock, 0, st>>>((unsigned char*)x, bytes);
  }
  return hipGetLastError();
}

// g5 on a half vector (one parity, tiled 12-component field): negate
// components k >= 6, i.e. the upper half of every tile
template <typename S>
__global__ void k_g5(S* x, long V2p, long rs) {
  const int q = blockIdx.y;
  const long n = 6 * V2p;
  constexpr long half = 6 * kTile;
  for (long i = (long)blockIdx.x * kVecBlock + threadIdx.x; i < n; i += (long)gridDim.x * kVecBlock) {
    S* p = x + (size_t)q * rs + (i / half) * 2 * half + half + i % half;
    auto v = ld(p);
    v.re = -v.re;
    v.im = -v.im;
    st(p, v);
  }
}

hipError_t launch_g5(void* x, int prec, long V2p, long rs, int nrhs, hipStream_t st) {
  dim3 grid(blas_nblocks(6 * V2p), nrhs);
  if (prec == P_F64) k_g5<double2><<<grid, kVecBlock, 0, st>>>((double2*)x, V2p, rs);
  else if (prec == P_F32) k_g5<float2><<<grid, kVecBlock, 0, st>>>((float2*)x, V2p, rs);
  else k_g5<bf16x2><<<grid, kVecBlock, 0, st>>>((bf16x2*)x, V2p, rs);
  return hipGetLastError();
}

}  // namespace lqcd
