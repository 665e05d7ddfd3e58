// CG scalar and vector kernels with the iteration control kept on the device.
//
// Every right-hand side carries a CGState.  The recursion (alpha, beta, the
// fused x/r update) runs in the inner precision; a reliable update
// (residual recomputed in FP64 from the FP64 solution) is requested by the
// beta kernel when |r|^2 has dropped below delta^2 times its maximum since the
// last update, or when it reaches the inner target.  The update kernels run
// at fixed points of the iteration sequence and skip every rhs that has no
// pending request, so a captured graph contains them unconditionally.  The
// update's finish kernel also performs the convergence test on the true
// residual and marks the rhs done.  The host only polls the done flags.
//
// Stall detection.  A low-precision recursion on a system whose condition
// number times the unit roundoff of the inner precision approaches one
// (e.g. near-zero modes) makes little or no progress on the true residual
// however long it runs.  Every reliable update compares the true residual
// with the best one so far; consecutive updates that do not halve it add to
// a count, and when the count reaches stall_max the rhs is marked CG_STALLED
// and the host continues it in FP64 from the current solution.  An update
// requested because the recursive |r| fell tenfold (or reached the inner
// target) and yet bought less than a halving of the true residual is the
// signature of a recursion that no longer tracks the true residual: it adds
// kDropWeight, so two in a row stall the rhs.  An update requested by the
// iteration count alone adds one: slow but real progress of an
// ill-conditioned system is not a stall, and eight such updates without a
// halving are needed.  Healthy solves gain about a factor ten per update.
#include <algorithm>

#include "lqcd_kernels.h"

namespace lqcd {

constexpr int kB = 256;
constexpr double kGain2 = 0.25;  // required gain on |eta - Dw x|^2 (halving the residual)
constexpr int kDropWeight = 4;   // stall count of a drop-requested update without gain

__device__ inline double bsum(double v, double* sh) {
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

// fixed-order sum of n partials, result broadcast to the block
__device__ inline double psum(const double* p, int n, double* sh) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) acc += p[i];
  double s = bsum(acc, sh);
  __shared__ double out;
  if (threadIdx.x == 0) out = s;
  __syncthreads();
  return out;
}

__device__ inline bool finite(double v) { return v == v && fabs(v) <= 1.7976931348623157e308; }

__global__ void k_cg_setup(CGState* s, const double* b2, const double* eta2, CGSetup cfg) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= cfg.nrhs) return;
  CGState& c = s[r];
  const double b = b2[r];
  c.rr = b;
  c.rr_prev = b;
  c.rr_max = b;
  c.pAp = 0.0;
  c.alpha = 0.0;
  c.beta = 0.0;
  c.bnorm2 = b;
  c.eta2 = eta2[r];
  c.tol2 = cfg.tol * cfg.tol * eta2[r];
  c.target2 = cfg.inner_rel * cfg.inner_rel * b;
  c.delta2 = cfg.delta2;
  c.rho2 = 1.0;
  c.iters = 0;
  c.maxiter = cfg.maxiter;
  c.rupd = 0;
  c.restarts = 0;
  c.inner_hit = 0;
  c.ru_every = cfg.ru_every;
  c.last_ru = 0;
  c.skip_ru = 1;
  c.target0 = c.target2;
  c.no_gain = 0;
  c.best_rho2 = 1.0;
  c.stall_max = cfg.stall_max;
  c.fp64_from = 0;
  c.ru_drop = 0;
  for (int j = 0; j < kXWindow; ++j) c.alpha_w[j] = 0.0;
  const bool zero = !(b > 0.0) || !(eta2[r] > 0.0);
  c.done = zero ? 1 : 0;
  c.status = zero ? CG_CONVERGED : CG_RUNNING;
  if (zero) c.rho2 = 0.0;
}

__global__ void k_cg_alpha(CGState* s, const double* partials, int nparts) {
  __shared__ double sh[4];
  const int r = blockIdx.x;
  if (s[r].done) return;
  const double v = psum(partials + (size_t)r * nparts, nparts, sh);
  if (threadIdx.x == 0) {
    CGState& c = s[r];
    c.pAp = v;
    c.alpha = (v > 0.0) ? c.rr / v : 0.0;
    c.rr_prev = c.rr;
  }
}

// beta and the iteration control from the new |r|^2 = v; the denominator is
// rr_prev, the |r|^2 the alpha step of this iteration divided by (alpha sets
// it), so the fused beta/p kernel below can replace rr while its other
// workgroups still divide by the old value
__device__ inline void beta_step(CGState& c, double v) {
  c.iters += 1;
  if (!finite(v) || !finite(c.alpha)) {
    c.done = 1;
    c.status = CG_NONFINITE;
    c.skip_ru = 1;
    return;
  }
  const bool hit = v <= c.target2;
  const bool due = c.ru_every > 0 && c.iters - c.last_ru >= c.ru_every;
  const bool drop = v < c.delta2 * c.rr_max;
  if (hit || due || drop) {
    if (c.skip_ru) c.ru_drop = 0;  // a new request
    c.skip_ru = 0;
    if (hit) c.inner_hit = 1;
    if (hit || drop) c.ru_drop = 1;
  }
  c.beta = (c.rr_prev > 0.0) ? v / c.rr_prev : 0.0;
  c.rr = v;
  if (v > c.rr_max) c.rr_max = v;
  if (c.iters >= c.maxiter && c.skip_ru) {
    c.done = 1;
    c.status = CG_MAXITER;
  }
}

__global__ void k_cg_beta(CGState* s, const double* partials, int nparts) {
  __shared__ double sh[4];
  const int r = blockIdx.x;
  if (s[r].done) return;
  const double v = psum(partials + (size_t)r * nparts, nparts, sh);
  if (threadIdx.x == 0) beta_step(s[r], v);
}

// x += alpha p ; r -= alpha Ap ; |r|^2 partials   (x may be wider than r)
template <typename SX, typename S>
__global__ void k_cg_xr(SX* x, S* r, const S* __restrict__ p, const S* __restrict__ Ap, long n,
                        long rsx, long rs, const CGState* cs, double* partials) {
  __shared__ double sh[4];
  const int q = blockIdx.y;
  if (cs[q].done) return;
  using A = typename StoreTraits<S>::acc;
  const double alpha_d = cs[q].alpha;
  const A alpha = (A)alpha_d;
  const size_t o = (size_t)q * rs, ox = (size_t)q * rsx;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) {
    auto pv = ld(p + o + i);
    auto av = ld(Ap + o + i);
    auto xv = ld(x + ox + i);
    auto rv = ld(r + o + i);
    using AX = decltype(xv.re);
    xv.re += (AX)alpha_d * (AX)pv.re;
    xv.im += (AX)alpha_d * (AX)pv.im;
    rv.re -= alpha * av.re;
    rv.im -= alpha * av.im;
    st(x + ox + i, xv);
    st(r + o + i, rv);
    acc += (double)rv.re * (double)rv.re + (double)rv.im * (double)rv.im;
  }
  double b = bsum(acc, sh);
  if (threadIdx.x == 0) partials[(size_t)q * gridDim.x + blockIdx.x] = b;
}

// Four consecutive complex elements per access (16 bytes of BF16, 32 of
// FP32): the streaming kernels of BF16-operand iterations move whole 16-byte
// words per lane.  p must be 16-byte aligned (element offsets multiples of 4).
__device__ inline void ld4(const bf16x2* p, cpx<float> (&v)[4]) {
  const uint4 w = *reinterpret_cast<const uint4*>(p);
  const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = {__uint_as_float(u[k] << 16), __uint_as_float(u[k] & 0xffff0000u)};
}
__device__ inline void st4(bf16x2* p, const cpx<float> (&v)[4]) {
  *reinterpret_cast<uint4*>(p) = make_uint4(pack_bf16x2(v[0].re, v[0].im), pack_bf16x2(v[1].re, v[1].im),
                                            pack_bf16x2(v[2].re, v[2].im), pack_bf16x2(v[3].re, v[3].im));
}
__device__ inline void ld4(const float2* p, cpx<float> (&v)[4]) {
  const float4 a = *reinterpret_cast<const float4*>(p), b = *reinterpret_cast<const float4*>(p + 2);
  v[0] = {a.x, a.y};
  v[1] = {a.z, a.w};
  v[2] = {b.x, b.y};
  v[3] = {b.z, b.w};
}
__device__ inline void st4(float2* p, const cpx<float> (&v)[4]) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0].re, v[0].im, v[1].re, v[1].im);
  *reinterpret_cast<float4*>(p + 2) = make_float4(v[2].re, v[2].im, v[3].re, v[3].im);
}

// pn = r + beta p over the n elements of one rhs (offset o), and plo = pn if
// given; p and pn may be the same vector
template <typename S, typename SP, typename SL, typename A>
__device__ inline void p_update(const SP* p, SP* pn, const S* r, SL* plo, A beta, size_t o, long n) {
  for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) {
    const auto p0 = ld(p + o + i);
    const auto rv = ld(r + o + i);
    const cpx<A> pv = {rv.re + beta * (A)p0.re, rv.im + beta * (A)p0.im};
    st(pn + o + i, pv);
    if (plo) st(plo + o + i, pv);
  }
}
// the BF16-only direction of BF16-operand iterations, four elements a lane
__device__ inline void p_update(const bf16x2* p, bf16x2* pn, const float2* r, bf16x2* plo, float beta, size_t o,
                                long n) {
  if (plo != nullptr || (n & 3) != 0 || (o & 3) != 0) {
    p_update<float2, bf16x2, bf16x2, float>(p, pn, r, plo, beta, o, n);
    return;
  }
  for (long i = (long)blockIdx.x * kB + threadIdx.x; i < (n >> 2); i += (long)gridDim.x * kB) {
    cpx<float> pv[4], rv[4];
    ld4(p + o + 4 * i, pv);
    ld4(r + o + 4 * i, rv);
#pragma unroll
    for (int k = 0; k < 4; ++k) pv[k] = {rv[k].re + beta * pv[k].re, rv[k].im + beta * pv[k].im};
    st4(pn + o + 4 * i, pv);
  }
}

// p = r + beta p ; optional low-precision copy of p
template <typename S, typename SP, typename SL>
__global__ void k_cg_p(const SP* p, SP* pn, const S* __restrict__ r, long n, long rs, const CGState* cs, SL* plo) {
  const int q = blockIdx.y;
  if (cs[q].done) return;
  using A = typename StoreTraits<S>::acc;
  const A beta = (A)cs[q].beta;
  p_update(p, pn, r, plo, beta, (size_t)q * rs, n);
}

// beta step fused with p = r + beta p (iterations without a reliable update):
// every workgroup sums the |r|^2 partials in the same fixed order, so all
// agree on beta bit for bit; workgroup 0 alone updates the control state.
// A rhs that workgroup 0 marks done meanwhile may see p updated by only some
// workgroups, which is harmless: done is final here (only the reliable
// update's finish kernel sets the resumable CG_STALLED).
template <typename S, typename SP, typename SL>
__global__ void k_cg_beta_p(const SP* p, SP* pn, const S* __restrict__ r, long n, long rs, CGState* cs, SL* plo,
                            const double* partials, int nparts) {
  __shared__ double sh[4];
  const int q = blockIdx.y;
  CGState& c = cs[q];
  if (c.done) return;
  const double v = psum(partials + (size_t)q * nparts, nparts, sh);
  const double rr0 = c.rr_prev;
  if (blockIdx.x == 0 && threadIdx.x == 0) beta_step(c, v);
  if (!finite(v)) return;
  using A = typename StoreTraits<S>::acc;
  const A beta = (A)((rr0 > 0.0) ? v / rr0 : 0.0);
  p_update(p, pn, r, plo, beta, (size_t)q * rs, n);
}

__device__ inline bool ru_skip(const CGState& c) { return c.skip_ru != 0 || c.done != 0; }

// x += sum_j alpha_w[j] p_j (the deferred updates of one window), summed in
// slot order in FP32; a slot whose alpha is 0 (an iteration the rhs skipped)
// is not read.  With X given, a rhs with a pending reliable update also gets
// the update's first step here: X += x (FP64), x = 0, so that x is not
// written and read back in between.
__global__ void k_cg_xflush(float2* x, long rsx, const PWindow pw, long n, long rs, const CGState* cs,
                            double2* X, long rsX) {
  const int q = blockIdx.y;
  float a[kXWindow];
  bool any = false;
#pragma unroll
  for (int j = 0; j < kXWindow; ++j) {
    a[j] = (float)cs[q].alpha_w[j];
    any = any || a[j] != 0.f;
  }
  const bool fold = X != nullptr && !ru_skip(cs[q]);
  if (!any && !fold) return;
  const size_t o = (size_t)q * rs, ox = (size_t)q * rsx, oX = (size_t)q * rsX;
  if (((n | (long)o | (long)ox) & 3) == 0) {  // four elements a lane
    for (long i = (long)blockIdx.x * kB + threadIdx.x; i < (n >> 2); i += (long)gridDim.x * kB) {
      cpx<float> xv[4];
      ld4(x + ox + 4 * i, xv);
#pragma unroll
      for (int j = 0; j < kXWindow; ++j) {
        if (a[j] == 0.f) continue;  // uniform over the workgroup
        cpx<float> pv[4];
        ld4(pw.p[j] + o + 4 * i, pv);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          xv[k].re += a[j] * pv[k].re;
          xv[k].im += a[j] * pv[k].im;
        }
      }
      if (fold) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          double2* xp = X + oX + 4 * i + k;
          const double2 b = *xp;
          *xp = make_double2(b.x + (double)xv[k].re, b.y + (double)xv[k].im);
          xv[k] = {0.f, 0.f};
        }
      }
      st4(x + ox + 4 * i, xv);
    }
    return;
  }
  for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) {
    float2 xv = x[ox + i];
#pragma unroll
    for (int j = 0; j < kXWindow; ++j) {
      if (a[j] == 0.f) continue;  // uniform over the workgroup
      const auto pv = ld(pw.p[j] + o + i);
      xv.x += a[j] * pv.re;
      xv.y += a[j] * pv.im;
    }
    if (fold) {
      const double2 b = X[oX + i];
      X[oX + i] = make_double2(b.x + (double)xv.x, b.y + (double)xv.y);
      xv = make_float2(0.f, 0.f);
    }
    x[ox + i] = xv;
  }
}

// reliable update, step 1: fold the low-precision correction into x (FP64)
__global__ void k_ru_fold(double2* X, long rsX, float2* xl, long rsl, long n, const CGState* cs) {
  const int q = blockIdx.y;
  if (ru_skip(cs[q])) return;
  for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) {
    float2 a = xl[(size_t)q * rsl + i];
    double2 b = X[(size_t)q * rsX + i];
    X[(size_t)q * rsX + i] = make_double2(b.x + (double)a.x, b.y + (double)a.y);
    xl[(size_t)q * rsl + i] = make_float2(0.f, 0.f);
  }
}

// step 2: s = g5 (b - y) with |s|^2 partials (y = Dhat x or Dw x); b, y, s
// are tiled 12-component fields (one or two parities per rhs), spins 2,3 (the
// upper half of every tile) negated
__global__ void k_ru_sub(const double2* __restrict__ b, const double2* __restrict__ y, double2* s, long n,
                         long rs, const CGState* cs, double* partials) {
  __shared__ double sh[4];
  const int q = blockIdx.y;
  if (ru_skip(cs[q])) return;
  const size_t o = (size_t)q * rs;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) {
    double2 u = b[o + i], v = y[o + i];
    double2 d = make_double2(u.x - v.x, u.y - v.y);
    acc += d.x * d.x + d.y * d.y;
    const long k = (i % (12 * kTile)) / kTile;  // component index within its tile
    if (k >= 6) d = make_double2(-d.x, -d.y);
    s[o + i] = d;
  }
  double t = bsum(acc, sh);
  if (threadIdx.x == 0) partials[(size_t)q * gridDim.x + blockIdx.x] = t;
}

// step 3 (mixed only): r_lo = (float) r_true
template <typename S>
__global__ void k_ru_copy(const S* __restrict__ R, long rsR, float2* rl, long rsl, long n, const CGState* cs) {
  const int q = blockIdx.y;
  if (ru_skip(cs[q])) return;
  for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) {
    const S v = R[(size_t)q * rsR + i];
    rl[(size_t)q * rsl + i] = make_float2((float)v.x, (float)v.y);
  }
}

// step 4: convergence test on the true residual and restart of the recursion
__global__ void k_ru_finish(CGState* s, const double* part_res, int n_res, const double* part_r,
                            int n_r) {
  __shared__ double sh[4];
  const int r = blockIdx.x;
  if (ru_skip(s[r])) return;
  const double res2 = psum(part_res + (size_t)r * n_res, n_res, sh);
  const double rr = psum(part_r + (size_t)r * n_r, n_r, sh);
  if (threadIdx.x != 0) return;
  CGState& c = s[r];
  c.rupd += 1;
  c.last_ru = c.iters;
  c.rho2 = res2 / c.eta2;
  c.skip_ru = 1;
  if (!finite(res2) || !finite(rr)) {
    c.done = 1;
    c.status = CG_NONFINITE;
    return;
  }
  if (res2 <= c.tol2) {
    c.done = 1;
    c.status = CG_CONVERGED;
    return;
  }
  if (c.stall_max > 0) {
    if (c.rho2 < kGain2 * c.best_rho2) {
      c.best_rho2 = c.rho2;
      c.no_gain = 0;
    } else {
      c.no_gain += c.ru_drop ? kDropWeight : 1;
    }
    if (c.no_gain >= c.stall_max) {
      c.done = 1;
      c.status = CG_STALLED;
      return;
    }
  }
  if (c.inner_hit) {  // inner target reached without the true one: tighten it
    c.target2 *= 0.01;
    c.restarts += 1;
    c.inner_hit = 0;
  }
  // the recursion continues from the true residual (p is kept)
  c.rr = rr;
  c.rr_max = rr;
  if (c.iters >= c.maxiter) {
    c.done = 1;
    c.status = CG_MAXITER;
  }
}

__global__ void k_cg_escalate(CGState* s, int n) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  CGState& c = s[r];
  if (c.status != CG_STALLED) {
    c.skip_ru = 1;
    return;
  }
  c.done = 0;
  c.status = CG_RUNNING;
  c.skip_ru = 0;  // the first FP64 step recomputes r from x
  c.stall_max = 0;
  c.no_gain = 0;
  c.ru_drop = 0;
  c.delta2 = 0.0;
  c.ru_every = 0;
  c.inner_hit = 0;
  c.target2 = c.target0;
  c.alpha = 0.0;
  c.beta = 0.0;  // p = r after the update
  c.fp64_from = c.iters;
}

// a reliable update is pending for every rhs that is not done (the first
// residual of a solve from an initial guess)
__global__ void k_cg_force_ru(CGState* s, int n) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  if (!s[r].done) s[r].skip_ru = 0;
}

// ---------------------------------------------------------------------------
hipError_t launch_cg_force_ru(CGState* s, int nrhs, hipStream_t st) {
  k_cg_force_ru<<<(nrhs + 63) / 64, 64, 0, st>>>(s, nrhs);
  return hipGetLastError();
}
hipError_t launch_cg_escalate(CGState* s, int nrhs, hipStream_t st) {
  k_cg_escalate<<<(nrhs + 63) / 64, 64, 0, st>>>(s, nrhs);
  return hipGetLastError();
}
hipError_t launch_cg_setup(CGState* s, const double* b2, const double* eta2, const CGSetup& cfg,
                           hipStream_t st) {
  k_cg_setup<<<(cfg.nrhs + 63) / 64, 64, 0, st>>>(s, b2, eta2, cfg);
  return hipGetLastError();
}
hipError_t launch_cg_alpha(CGState* s, const double* partials, int nparts, int nrhs, hipStream_t st) {
  k_cg_alpha<<<nrhs, kB, 0, st>>>(s, partials, nparts);
  return hipGetLastError();
}
hipError_t launch_cg_beta(CGState* s, const double* partials, int nparts, int nrhs, hipStream_t st) {
  k_cg_beta<<<nrhs, kB, 0, st>>>(s, partials, nparts);
  return hipGetLastError();
}

hipError_t launch_cg_xr(void* x, int xprec, long rsx, void* r, const void* p, const void* Ap, int prec,
                        long n, long rs, int nrhs, const CGState* s, double* partials, hipStream_t st) {
  dim3 grid(blas_nblocks(n), nrhs);
  if (prec == P_F64 && xprec == P_F64)
    k_cg_xr<double2, double2><<<grid, kB, 0, st>>>((double2*)x, (double2*)r, (const double2*)p,
                                                   (const double2*)Ap, n, rsx, rs, s, partials);
  else if (prec == P_F32 && xprec == P_F32)
    k_cg_xr<float2, float2><<<grid, kB, 0, st>>>((float2*)x, (float2*)r, (const float2*)p,
                                                 (const float2*)Ap, n, rsx, rs, s, partials);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_cg_p(void* p, const void* r, int prec, long n, long rs, int nrhs, const CGState* s,
                       void* plo, int lo_prec, hipStream_t st, void* pnext) {
  dim3 grid(blas_nblocks(n), nrhs);
  if (prec == P_F64 && p)
    k_cg_p<double2, double2, double2><<<grid, kB, 0, st>>>((const double2*)p, (double2*)p, (const double2*)r, n,
                                                           rs, s, (double2*)nullptr);
  else if (prec == P_F32 && p && (plo == nullptr || lo_prec == P_F32))
    k_cg_p<float2, float2, float2><<<grid, kB, 0, st>>>((const float2*)p, (float2*)p, (const float2*)r, n, rs, s,
                                                        (float2*)plo);
  else if (prec == P_F32 && p && plo && lo_prec == P_BF16)
    k_cg_p<float2, float2, bf16x2><<<grid, kB, 0, st>>>((const float2*)p, (float2*)p, (const float2*)r, n, rs, s,
                                                        (bf16x2*)plo);
  else if (prec == P_F32 && !p && plo && lo_prec == P_BF16)  // the direction lives in BF16 only
    k_cg_p<float2, bf16x2, bf16x2><<<grid, kB, 0, st>>>((const bf16x2*)plo, (bf16x2*)(pnext ? pnext : plo),
                                                        (const float2*)r, n, rs, s, (bf16x2*)nullptr);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_cg_beta_p(void* p, const void* r, int prec, long n, long rs, int nrhs, CGState* s,
                            void* plo, int lo_prec, const double* partials, int nparts, hipStream_t st,
                            void* pnext) {
  // every workgroup re-sums its rhs's partials before streaming p: with many
  // rhs, fewer workgroups per rhs (at least 256, each streaming more) keep
  // that repeated sum small while the whole grid stays as large
  const int nb = blas_nblocks(n);
  const int nbx = std::min(nb, std::max(256, nb / nrhs));
  dim3 grid(nbx, nrhs);
  if (prec == P_F64 && p)
    k_cg_beta_p<double2, double2, double2><<<grid, kB, 0, st>>>((const double2*)p, (double2*)p,
                                                                (const double2*)r, n, rs, s, (double2*)nullptr,
                                                                partials, nparts);
  else if (prec == P_F32 && p && (plo == nullptr || lo_prec == P_F32))
    k_cg_beta_p<float2, float2, float2><<<grid, kB, 0, st>>>((const float2*)p, (float2*)p, (const float2*)r, n,
                                                             rs, s, (float2*)plo, partials, nparts);
  else if (prec == P_F32 && p && plo && lo_prec == P_BF16)
    k_cg_beta_p<float2, float2, bf16x2><<<grid, kB, 0, st>>>((const float2*)p, (float2*)p, (const float2*)r, n,
                                                             rs, s, (bf16x2*)plo, partials, nparts);
  else if (prec == P_F32 && !p && plo && lo_prec == P_BF16)  // the direction lives in BF16 only
    k_cg_beta_p<float2, bf16x2, bf16x2><<<grid, kB, 0, st>>>((const bf16x2*)plo,
                                                             (bf16x2*)(pnext ? pnext : plo), (const float2*)r,
                                                             n, rs, s, (bf16x2*)nullptr, partials, nparts);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_cg_xflush(float2* x, long rsx, const PWindow& pw, long n, long rs, int nrhs, const CGState* s,
                            hipStream_t st, double2* X, long rsX) {
  dim3 grid(blas_nblocks(n), nrhs);
  k_cg_xflush<<<grid, kB, 0, st>>>(x, rsx, pw, n, rs, s, X, rsX);
  return hipGetLastError();
}

hipError_t launch_ru_fold(double2* X, long rsX, float2* xl, long rsl, long n, int nrhs, const CGState* s,
                          hipStream_t st) {
  dim3 grid(blas_nblocks(n), nrhs);
  k_ru_fold<<<grid, kB, 0, st>>>(X, rsX, xl, rsl, n, s);
  return hipGetLastError();
}
hipError_t launch_ru_sub(const double2* b, const double2* y, double2* s_out, long n, long rs,
                         int nrhs, const CGState* s, double* partials, hipStream_t st) {
  dim3 grid(blas_nblocks(n), nrhs);
  k_ru_sub<<<grid, kB, 0, st>>>(b, y, s_out, n, rs, s, partials);
  return hipGetLastError();
}
hipError_t launch_ru_copy(const double2* R, long rsR, float2* rl, long rsl, long n, int nrhs,
                          const CGState* s, hipStream_t st) {
  dim3 grid(blas_nblocks(n), nrhs);
  k_ru_copy<double2><<<grid, kB, 0, st>>>(R, rsR, rl, rsl, n, s);
  return hipGetLastError();
}
hipError_t launch_ru_copy(const float2* R, long rsR, float2* rl, long rsl, long n, int nrhs,
                          const CGState* s, hipStream_t st) {
  dim3 grid(blas_nblocks(n), nrhs);
  k_ru_copy<float2><<<grid, kB, 0, st>>>(R, rsR, rl, rsl, n, s);
  return hipGetLastError();
}
hipError_t launch_ru_finish(CGState* s, const double* part_res, int n_res, const double* part_r, int n_r,
                            int nrhs, hipStream_t st) {
  k_ru_finish<<<nrhs, kB, 0, st>>>(s, part_res, n_res, part_r, n_r);
  return hipGetLastError();
}

}  // namespace lqcd
