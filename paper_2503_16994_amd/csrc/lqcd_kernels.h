// Host-side launch interface of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lqcd_dev.h"

namespace lqcd {

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16 = 2 };

inline size_t elem_bytes(int prec) { return prec == P_F64 ? 16 : (prec == P_F32 ? 8 : 4); }

// Self-term of a hop launch
enum PreMode { PRE_NONE = 0, PRE_IDENT = 1, PRE_CLOV = 2 };
// Matrix applied to the whole result
enum PostMode { POST_NONE = 0, POST_CLOV = 1 };

// One launch of the hopping kernel:
//   out = post( pre(z) + scale * H y ),  H = sum_mu [(1-g)U y(x+mu) + (1+g)U^+ y(x-mu)]
// on the sites of parity p_out, then optionally g5, the SF output mask and
// per-block |out|^2 partial sums.  All vector pointers point at the first
// rhs of the relevant parity; *_rs are element strides between rhs.
struct HopLaunch {
  KGeom g;
  int prec;       // storage precision of links/clover (P_*)
  int in_prec;    // storage precision of y, z
  int out_prec;   // storage precision of out
  int p_out;
  const void* U;     // links (both parities), precision prec
  int two_row;       // links stored as their first two rows (6 of 9 complex)
  const void* y;     // opposite-parity input
  const void* z;     // same-parity input (PRE_IDENT / PRE_CLOV)
  const void* Cpre;  // clover blocks of parity p_out (tiled 36-component field)
  const void* Cpost; // clover inverse blocks of parity p_out
  void* out;
  long y_rs, z_rs, out_rs;
  int nrhs;
  int pre, post;
  bool g5;
  bool hop;          // false: no hopping term (pure block application)
  double scale;
  double* partials;  // [nrhs][nblocks] or nullptr
  const int* done;   // early-exit flag (device) or nullptr
  int nr_tile;       // rhs per thread (1, 2, 3, 4)
  // both = true: one launch covers both parities (first half of the grid
  // parity 0, second half parity 1); y, z, out then point at the parity-0
  // part of full vectors, parity 1 lies par_stride elements further and the
  // Cpre blocks of parity 1 cpre_par elements further.
  bool both;
  long par_stride;
  long cpre_par;
  // tuning: block order (0..6, see block_order in k_dslash.hip) and the
  // number of lanes that share a site and split its rhs (1, 2, 4)
  int order;
  int rhs_lanes;
  int nt_out;        // 1: non-temporal stores of the output spinor
  int cached_gauge;  // 1: ordinary (cached) loads of links and clover blocks
                     // instead of non-temporal ones (rhs tiles re-read them)
  int occ_cap;       // 0..3: cap on resident workgroups per CU (unused LDS)
  int dir_split;     // 1: two waves per site block split the hop directions
                     // (launches with nr_tile = rhs_lanes = 1 only)
  // twisted mass tm_mu (+-mu: -mu in launches of the adjoint operator,
  // since D(mu)^+ = g5 D(-mu) g5): PRE_CLOV adds i tm_mu g5 z; with tm_post
  // POST_CLOV applies (A + i tm_mu g5)^{-1} = Q^{-1} (A - i tm_mu g5) per
  // chirality, with Q^{-1} = (A^2 + mu^2)^{-1} in Cpost and A in Ctm
  double tm_mu;
  int tm_post;
  const void* Ctm;  // clover blocks A of the output parity (tm_post only)
  unsigned lds_cap;  // dynamic LDS bytes of the launch (set by the launcher)
  // filled in by the launcher
  int nbs;  // site blocks (both parities in `both` mode)
  int bpp;  // site blocks per (z, t) plane
  // fused CG update (launch_hop_xr): x += alpha p, r -= alpha out for every
  // rhs not done, |r|^2 partials into `partials`; out itself is not stored
  void* xr_x;
  void* xr_r;
  const void* xr_p;
  int xr_prec;   // precision of x and r (p has the operator's input precision)
  long xr_rs;    // rhs stride of r and p
  long xr_xrs;   // rhs stride of x
  const struct CGState* cg;
  // CG alpha fused into a hop launch that does not need it (k_hop only):
  // alpha = rr / pAp with pAp the fixed-order sum of alpha_nparts partials per
  // rhs; rhs r is handled by workgroup r mod grid, before its stencil work.
  struct CGState* alpha_cg;   // nullptr: no alpha step
  const double* alpha_parts;  // [nrhs][alpha_nparts]
  int alpha_nparts;
  int alpha_slot;             // >= 0: also record alpha in alpha_w[alpha_slot] (0 for a done rhs)
};

int hop_nblocks(const HopLaunch& h);
int hop_max_parts(long V2);  // bound on partials per rhs of any hop launch
int hop_nparts(const HopLaunch& h);  // partials per rhs of a tiled hop launch
hipError_t launch_hop(const HopLaunch& h, hipStream_t st);
hipError_t launch_hop_xr(const HopLaunch& h, hipStream_t st);

// Gauge import: canonical complex128 U -> internal links (any non-null
// precision pointer is written); OPEN zeroes U_t(T-1).  two_row: store the
// first two rows only, and set *bad (zeroed by the caller) when a link's
// third row differs from the rebuilt one by more than 1e-10.
hipError_t launch_import_gauge(const KGeom& g, const double2* Ucanon, double2* U64, float2* U32,
                               bf16x2* U16, bool two_row, int* bad, hipStream_t st);

// Meson two-point functions (k_meson.hip): colour-traced spin tensor G per
// time slice of a 12-column canonical propagator (G may be null) and the
// correlators of up to kMaxMesonPairs (Gamma, Gamma') mask pairs, times
// `scale`, into outs[p][t]; scratch holds T x meson_nchunk(V3) x 256
// complex partials.
constexpr int kMaxMesonPairs = 32;
int meson_nchunk(long V3);
hipError_t launch_meson(const KGeom& g, const double2* psi, int npairs, const int* masks, double2* const* outs,
                        double scale, double2* G, double2* scratch, hipStream_t st);
// SF boundary source (k_sf.hip): writes the slice y0 = 1 of the 12-column
// canonical field eta (the rest must be zero) from the FP64 links
hipError_t launch_sf_source(const KGeom& g, const double2* U64, int two_row, double2* eta, hipStream_t st);

// Spinor layout conversion.  Internal "full" vector: [rhs][parity][k][s].
// pack: canonical [rhs][site][12] -> internal (g5 optional), precision prec.
hipError_t launch_pack(const KGeom& g, const double2* canon, void* internal, int prec, int nrhs,
                       bool g5, hipStream_t st);
hipError_t launch_unpack(const KGeom& g, const void* internal, int prec, double2* canon,
                         int nrhs, hipStream_t st);

// Clover: builds A on both parities (FP64 + optional lower precisions) and the
// inverse on the odd sites.  err_flag gets bit 1 for a singular block.
struct CloverLaunch {
  KGeom g;
  const double2* U64;
  int two_row;  // links stored as their first two rows (6 complex)
  double m0, csw, cF;
  double mu;    // twisted mass: odd sites hold (A^2 + mu^2)^{-1} instead of A^{-1}
  double2* C64;     // two parities, each a tiled 36-component field
  double2* Ci64;    // tiled 36-component field: inverse on the odd sites
  float2* C32;
  float2* Ci32;
  bf16x2* C16;
  bf16x2* Ci16;
  int* err_flag;
};
hipError_t launch_clover(const CloverLaunch& c, hipStream_t st);

// ---- vector algebra on flat arrays of n complex elements per rhs -----------
// CG_STALLED: the low-precision recursion no longer tracks the true residual
// (see k_ru_finish); the rhs continues in FP64 after launch_cg_escalate.
enum CGStatus { CG_RUNNING = 0, CG_CONVERGED = 1, CG_MAXITER = 2, CG_NONFINITE = 3, CG_STALLED = 4 };

// CG control of one right-hand side (device memory)
// Iterations whose x updates a BF16-operand recursion defers: their alpha
// (CGState::alpha_w) and search directions are kept, and one flush kernel
// adds them to x at every reliable-update slot (every kXWindow-th iteration).
constexpr int kXWindow = 5;

struct CGState {
  double rr;       // |r|^2 of the recursion
  double rr_prev;  // |r|^2 this iteration's alpha divided by (set by alpha, read by beta)
  double rr_max;   // max |r|^2 since the last reliable update
  double pAp;      // |Dhat p|^2
  double alpha, beta;
  double bnorm2;   // |b|^2, b the normal-equation right-hand side
  double eta2;     // |eta|^2
  double tol2;     // converged when |eta - Dw x|^2 <= tol2
  double target2;  // inner target on |r|^2 (reliable update when reached)
  double delta2;   // reliable update when |r|^2 < delta2 * rr_max (0: never)
  double rho2;     // last true residual |eta - Dw x|^2 / |eta|^2
  int done;        // 1: no further updates
  int skip_ru;     // 0: a reliable update is pending
  int status;      // CGStatus
  int iters;
  int maxiter;
  int rupd;        // reliable updates performed
  int restarts;    // inner target tightenings
  int inner_hit;
  int ru_every;    // reliable update at least every ru_every iterations (0: off)
  int last_ru;     // iteration of the last reliable update
  double target0;    // initial inner target
  double best_rho2;  // smallest true residual^2 (relative) at a reliable update
  int no_gain;       // weighted count of consecutive reliable updates that did not halve best_rho2
  int stall_max;     // CG_STALLED when no_gain reaches this (0: never)
  int fp64_from;     // iteration at which the rhs continued in FP64 (0: never)
  int ru_drop;       // the pending reliable update was requested by a drop of |r|^2
                     // (tenfold, or the inner target), not by the iteration count
  double alpha_w[kXWindow];  // alpha of the deferred x updates, by slot (0: none)
};

struct CGSetup {
  int nrhs;
  int maxiter;
  double tol;        // true relative residual target
  double inner_rel;  // initial inner target relative to |b|
  double delta2;
  int ru_every;
  int stall_max;
};

int blas_nblocks(long n);
hipError_t launch_norm2(const void* x, int prec, long n, long rs, int nrhs, double* partials,
                        hipStream_t st);
// sum partials (fixed order) into dst[r] (FP64)
hipError_t launch_reduce(const double* partials, int nparts, int nrhs, double* dst,
                         hipStream_t st);
hipError_t launch_cg_setup(CGState* s, const double* b2, const double* eta2, const CGSetup& cfg,
                           hipStream_t st);
hipError_t launch_cg_alpha(CGState* s, const double* partials, int nparts, int nrhs,
                           hipStream_t st);
hipError_t launch_cg_beta(CGState* s, const double* partials, int nparts, int nrhs,
                          hipStream_t st);
hipError_t launch_cg_xr(void* x, int xprec, long rsx, void* r, const void* p, const void* Ap,
                        int prec, long n, long rs, int nrhs, const CGState* s, double* partials,
                        hipStream_t st);
// p = r + beta p, also written to p_lo (precision lo_prec) if given; with p
// null the direction is kept in BF16 alone (r FP32): p_next = r + beta p_lo,
// written to p_next (p_lo itself when p_next is null)
hipError_t launch_cg_p(void* p, const void* r, int prec, long n, long rs, int nrhs,
                       const CGState* s, void* p_lo, int lo_prec, hipStream_t st, void* p_next = nullptr);
// beta step and p update in one launch (nparts |r|^2 partials per rhs)
hipError_t launch_cg_beta_p(void* p, const void* r, int prec, long n, long rs, int nrhs, CGState* s,
                            void* p_lo, int lo_prec, const double* partials, int nparts, hipStream_t st,
                            void* p_next = nullptr);
// deferred x updates: x += sum_j alpha_w[j] p_j over the kXWindow BF16
// directions p_j (slots with alpha_w[j] = 0 are not read); x FP32.  With X
// (FP64) given, every rhs with a pending reliable update then also has x
// folded into X and zeroed (the update's fold step).
struct PWindow {
  const bf16x2* p[kXWindow];
};
hipError_t launch_cg_xflush(float2* x, long rsx, const PWindow& pw, long n, long rs, int nrhs, const CGState* s,
                            hipStream_t st, double2* X = nullptr, long rsX = 0);
// reliable-update kernels (each skips rhs without a pending update)
hipError_t launch_ru_fold(double2* X, long rsX, float2* xl, long rsl, long n, int nrhs,
                          const CGState* s, hipStream_t st);
hipError_t launch_ru_sub(const double2* b, const double2* y, double2* s_out, long n, long rs,
                         int nrhs, const CGState* s, double* partials, hipStream_t st);
// rl = R (rounded to FP32) for every rhs with a pending reliable update
hipError_t launch_ru_copy(const double2* R, long rsR, float2* rl, long rsl, long n, int nrhs,
                          const CGState* s, hipStream_t st);
hipError_t launch_ru_copy(const float2* R, long rsR, float2* rl, long rsl, long n, int nrhs,
                          const CGState* s, hipStream_t st);
hipError_t launch_ru_finish(CGState* s, const double* part_res, int n_res, const double* part_r,
                            int n_r, int nrhs, hipStream_t st);
// every CG_STALLED rhs becomes a running FP64 rhs with a pending reliable
// update (which recomputes r from x); every other rhs keeps its state and has
// no pending update
hipError_t launch_cg_escalate(CGState* s, int nrhs, hipStream_t st);
// every rhs that is not done gets a pending reliable update
hipError_t launch_cg_force_ru(CGState* s, int nrhs, hipStream_t st);

// y = a*x + b*y  (element types by precision), per-rhs scalars not needed
hipError_t launch_axpby(double a, const void* x, int xprec, double b, void* y, int yprec,
                        long n, long rs_x, long rs_y, int nrhs, hipStream_t st);
// y = x converted between precisions
hipError_t launch_convert(const void* x, int xprec, void* y, int yprec, long n, long rs_x,
                          long rs_y, int nrhs, hipStream_t st);
// out = x - y (FP64) with partial |out|^2
hipError_t launch_sub_norm(const double2* x, const double2* y, double2* out, long n, long rs,
                           int nrhs, double* partials, hipStream_t st);
hipError_t launch_fill_zero(void* x, size_t bytes, hipStream_t st);
// x (even half vector) *= g5 in place
hipError_t launch_g5(void* x, int prec, long V2p, long rs, int nrhs, hipStream_t st);

}  // namespace lqcd
