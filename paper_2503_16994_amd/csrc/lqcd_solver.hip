// lqcd_solve: conjugate gradient on the normal equations (paper Sec. 3.3,
// CG!/propagator!), on the full lattice or even-odd preconditioned, with an
// optional reduced-precision inner iteration and FP64 reliable updates.
//
// Even-odd form.  With A the site-diagonal clover term and H the hopping
// sum, Dw = [[A_ee, D_eo], [D_oe, A_oo]], D = -H/2, and the Schur complement
//   Dhat = A_ee - D_eo A_oo^{-1} D_oe
// acts on even sites.  The solve is
//   eta_hat = eta_e - D_eo A_oo^{-1} eta_o,   CG on Dhat^+ Dhat x = Dhat^+ eta_hat,
//   psi_e = x,  psi_o = A_oo^{-1} (eta_o - D_oe psi_e),
// and Dhat^+ = g5 Dhat g5.  One CG iteration is four hop launches (the g5 and
// |Dhat p|^2 fused into the second), one alpha, the fused x/r update with
// |r|^2, one beta and the p update.  All CG scalars stay on the device; the
// host reads them once per chunk of iterations.
//
// Stopping and reliable updates.  The target is the true relative residual
// |eta - Dw psi|/|eta| <= tol.  The recursion runs in the inner precision.
// A reliable update recomputes the residual in FP64 from the FP64 solution
// (Sleijpen and van der Vorst's reliable updates, as used for mixed-precision
// lattice solvers by Clark et al.): s = eta_hat - Dhat x, whose norm equals
// the full-lattice residual because the odd rows are solved exactly, then
// r = Dhat^+ s with the search direction p kept.  It is requested by the beta
// kernel when |r| has dropped by delta = 0.1 since the last update (mixed
// precision only) or reaches the inner target (tol/10)|b|; the update kernels
// sit after every fifth iteration and skip rhs without a request.  The
// update's last kernel declares an rhs converged when |s|/|eta| <= tol, and
// otherwise tightens the inner target tenfold if it had been reached.  All
// control stays on the device: the host polls the done flags once per chunk
// of iterations, and a chunk can be captured in a hipGraph and replayed.  At
// the end psi is reconstructed and |eta - Dw psi| is recomputed with the FP64
// full-lattice operator.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "lqcd_internal.h"

using namespace lqcd;

namespace {

struct Ctl {
  hipStream_t st;
  const lqcd_geom_t* g;
  const lqcd_gauge* u;
  lqcd_ws* w;
  int nrhs;
  double mu;         // twisted mass
  bool dag = false;  // launches of the adjoint operator g5 D(-mu) g5
};

// the same context for the adjoint operator (D(mu)^+ = g5 D(-mu) g5)
Ctl dg(const Ctl& c) {
  Ctl d = c;
  d.dag = true;
  return d;
}

const void* links_of(const lqcd_gauge* u, int prec) {
  return prec == P_F64 ? (const void*)u->U64 : (prec == P_F32 ? (const void*)u->U32 : (const void*)u->U16);
}
const void* clov_of(const lqcd_ws* w, int prec) {
  return prec == P_F64 ? (const void*)w->m.C64 : (prec == P_F32 ? (const void*)w->m.C32 : (const void*)w->m.C16);
}
const void* cloi_of(const lqcd_ws* w, int prec) {
  return prec == P_F64 ? (const void*)w->m.Ci64 : (prec == P_F32 ? (const void*)w->m.Ci32 : (const void*)w->m.Ci16);
}

// a vector operand: base pointer of rhs 0 at the relevant parity, its
// storage precision and its rhs stride (elements)
struct Vec {
  void* p;
  int prec;
  long rs;
};

Vec odd_part(const Vec& v, long V2) {
  return Vec{(char*)v.p + (size_t)12 * V2 * elem_bytes(v.prec), v.prec, v.rs};
}

HopLaunch mk(const Ctl& c, int lprec) {
  HopLaunch h;
  memset(&h, 0, sizeof(h));
  h.g = c.g->kg;
  h.prec = lprec;
  h.U = links_of(c.u, lprec);
  h.two_row = c.u->two_row;
  h.nrhs = c.nrhs;
  h.hop = true;
  h.tm_mu = c.dag ? -c.mu : c.mu;
  h.tm_post = c.mu != 0.0 ? 1 : 0;
  apply_tuning(h, c.w->tune[lprec]);
  if (c.mu != 0.0) single_tile(h);  // twisted-mass kernels: one rhs per thread
  return h;
}

// out_o = A_oo^{-1} D_oe y_e = A_oo^{-1} (-1/2 H y_e); with alpha_cg the
// launch also computes the CG alpha of every rhs from alpha_parts (and
// records it in window slot alpha_slot if that is >= 0)
hipError_t hop_eo(const Ctl& c, int lprec, Vec y, Vec out_o, const int* done, int nr_tile,
                  CGState* alpha_cg = nullptr, const double* alpha_parts = nullptr, int alpha_nparts = 0,
                  int alpha_slot = -1) {
  HopLaunch h = mk(c, lprec);
  h.alpha_cg = alpha_cg;
  h.alpha_parts = alpha_parts;
  h.alpha_nparts = alpha_nparts;
  h.alpha_slot = alpha_slot;
  h.p_out = 1;
  h.in_prec = y.prec;
  h.out_prec = out_o.prec;
  h.y = y.p;
  h.y_rs = y.rs;
  h.out = out_o.p;
  h.out_rs = out_o.rs;
  h.Cpost = cloi_of(c.w, lprec);
  h.Ctm = (const char*)clov_of(c.w, lprec) + (size_t)36 * c.g->V2p * elem_bytes(lprec);  // A, odd sites
  h.pre = PRE_NONE;
  h.post = POST_CLOV;
  h.scale = -0.5;
  h.done = done;
  if (nr_tile == 1) single_tile(h);
  return launch_hop(h, c.st);
}

// out_e = [g5] (A_ee z_e + 1/2 H t_o), optional |out|^2 partials
hipError_t hop_oe(const Ctl& c, int lprec, Vec z, Vec t_o, Vec out, bool g5, double* partials,
                  const int* done, int nr_tile) {
  HopLaunch h = mk(c, lprec);
  h.p_out = 0;
  h.in_prec = z.prec;
  h.out_prec = out.prec;
  h.y = t_o.p;
  h.y_rs = t_o.rs;
  h.z = z.p;
  h.z_rs = z.rs;
  h.out = out.p;
  h.out_rs = out.rs;
  h.Cpre = clov_of(c.w, lprec);
  h.pre = PRE_CLOV;
  h.post = POST_NONE;
  h.scale = 0.5;
  h.g5 = g5;
  h.partials = partials;
  h.done = done;
  if (nr_tile == 1) single_tile(h);
  return launch_hop(h, c.st);
}

// fused last hop + CG update: Ap = g5 (A_ee q_e + 1/2 H t_o) in registers,
// x += alpha p, r -= alpha Ap, |r|^2 partials (x and r in the recursion's
// precision, p in the operator's input precision)
hipError_t hop_oe_xr(const Ctl& c, int lprec, Vec q, Vec t_o, Vec x, Vec r, Vec p, double* partials,
                     const CGState* cg, const int* done) {
  HopLaunch h = mk(c, lprec);
  h.p_out = 0;
  h.in_prec = q.prec;
  h.out_prec = r.prec;
  h.y = t_o.p;
  h.y_rs = t_o.rs;
  h.z = q.p;
  h.z_rs = q.rs;
  h.Cpre = clov_of(c.w, lprec);
  h.pre = PRE_CLOV;
  h.post = POST_NONE;
  h.scale = 0.5;
  h.g5 = true;
  h.partials = partials;
  h.done = done;
  h.xr_x = x.p;
  h.xr_r = r.p;
  h.xr_p = p.p;
  h.xr_prec = r.prec;
  h.xr_rs = r.rs;
  h.xr_xrs = x.rs;
  h.cg = cg;
  return launch_hop_xr(h, c.st);
}

// partial sums per rhs that the tuned iteration hops of precision lprec write
int iter_parts(const Ctl& c, int lprec) { return hop_nparts(mk(c, lprec)); }

// the launch shape of dw_full (both parities, the FP64 tuning)
HopLaunch dw_full_launch(const Ctl& c) {
  HopLaunch h = mk(c, P_F64);
  h.both = true;
  return h;
}
// partial sums per rhs that a dw_full launch writes (its own site blocks:
// the tuned rhs tile and direction split decide the block size)
int full_parts(const Ctl& c) { return hop_nparts(dw_full_launch(c)); }

// out (full, both parities) = [g5] Dw y, optional partials
hipError_t dw_full(const Ctl& c, const double2* y, double2* out, bool g5, double* partials,
                   const int* done) {
  HopLaunch h = dw_full_launch(c);
  const long V2 = c.g->V2p;  // field rows per parity
  h.in_prec = h.out_prec = P_F64;
  h.par_stride = 12 * V2;
  h.cpre_par = 36 * V2;
  h.y = y;
  h.z = y;
  h.out = out;
  h.y_rs = h.z_rs = h.out_rs = 24 * V2;
  h.Cpre = c.w->m.C64;
  h.pre = PRE_CLOV;
  h.post = POST_NONE;
  h.scale = -0.5;
  h.g5 = g5;
  h.partials = partials;
  h.done = done;
  return launch_hop(h, c.st);
}

// out_e = z_e + 1/2 H y_o   (eta_hat from eta_e and A_oo^{-1} eta_o)
hipError_t hop_oe_ident(const Ctl& c, Vec z, Vec y_o, Vec out) {
  HopLaunch h = mk(c, P_F64);
  h.p_out = 0;
  h.in_prec = h.out_prec = P_F64;
  h.y = y_o.p;
  h.y_rs = y_o.rs;
  h.z = z.p;
  h.z_rs = z.rs;
  h.out = out.p;
  h.out_rs = out.rs;
  h.pre = PRE_IDENT;
  h.post = POST_NONE;
  h.scale = 0.5;
  return launch_hop(h, c.st);
}

// out_o = A_oo^{-1} (z_o + s H y_e)  (hop = false: A_oo^{-1} z_o)
hipError_t clover_inv_apply(const Ctl& c, Vec z_o, Vec y_e, Vec out_o, bool hop, double s) {
  HopLaunch h = mk(c, P_F64);
  h.p_out = 1;
  h.in_prec = h.out_prec = P_F64;
  h.y = y_e.p;
  h.y_rs = y_e.rs;
  h.z = z_o.p;
  h.z_rs = z_o.rs;
  h.out = out_o.p;
  h.out_rs = out_o.rs;
  h.Cpost = c.w->m.Ci64;
  h.Ctm = c.w->m.C64 + (size_t)36 * c.g->V2p;  // A on the odd sites
  h.pre = PRE_IDENT;
  h.post = POST_CLOV;
  h.hop = hop;
  h.scale = s;
  return launch_hop(h, c.st);
}

}  // namespace

extern "C" int lqcd_solve(const lqcd_gauge_t* u, const lqcd_solve_params* prm, const void* eta, void* psi,
                          lqcd_ws_t* w, void* stream, lqcd_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!u || !prm || !eta || !psi || !w || !info) return fail(LQCD_EINVAL, "lqcd_solve: null pointer");
  int rc = check_dirac(&prm->d);
  if (rc) return rc;
  const int N = prm->nrhs;
  if (N < 1 || N > w->nrhs) return fail(LQCD_EINVAL, "lqcd_solve: nrhs=%d (workspace holds %d)", N, w->nrhs);
  if (prm->solver != LQCD_SOLVER_CG_FULL && prm->solver != LQCD_SOLVER_CG_EO)
    return fail(LQCD_EINVAL, "lqcd_solve: unknown solver %d", prm->solver);
  const int ip = prm->inner_prec;
  if (ip < LQCD_F64 || ip > LQCD_BF16) return fail(LQCD_EINVAL, "lqcd_solve: bad inner precision %d", ip);
  if (prm->solver == LQCD_SOLVER_CG_FULL && ip != LQCD_F64)
    return fail(LQCD_EINVAL, "lqcd_solve: the full-lattice solver runs in FP64 only");
  if (!((1 << ip) & u->pmask) || !((1 << ip) & w->pmask))
    return fail(LQCD_EINVAL, "lqcd_solve: inner precision %d not held by gauge field and workspace", ip);
  if (!(prm->tol > 0.0) || !(prm->tol < 1.0)) return fail(LQCD_EINVAL, "lqcd_solve: tol must be in (0,1)");
  if (prm->maxiter < 1) return fail(LQCD_EINVAL, "lqcd_solve: maxiter must be >= 1");
  if (eta == psi) return fail(LQCD_EINVAL, "lqcd_solve: eta and psi must differ");

  hipStream_t st = (hipStream_t)stream;
  rc = ensure_clover(u, &prm->d, w, st);
  if (rc) return rc;

  const lqcd_geom_t* g = w->g;
  const long V2 = g->V2p;  // field rows per parity (sites incl. padding)
  const WsLayout& m = w->m;
  Ctl c{st, g, u, w, N, prm->d.mu};
  const long FRS = 24 * V2, HRS = 12 * V2;
  const bool eo = (prm->solver == LQCD_SOLVER_CG_EO);
  const bool mixed = eo && ip != LQCD_F64;
  const double tol = prm->tol;

  // ---- validate the source (and x0): finite, and zero on the SF Dirichlet slice
  double* parts = m.partials;
  double* parts2 = m.partials2;
  // [0,N) |b|^2  [N,2N) |eta|^2  [2N,3N) |eta(t=0)|^2  [3N,4N) final residual^2
  // [4N,5N) |x0|^2  [5N,6N) |x0(t=0)|^2
  double* scal = m.scal;
  std::vector<double> h_eta2(N);
  const void* x0 = prm->x0;
  {
    const long nsite = g->V * 12;
    const bool sf = g->desc.bc == LQCD_BC_SF;
    const long nslice = g->V / g->desc.L[3] * 12;  // t = 0 is the first slice
    auto norms = [&](const void* v, double* dst_all, double* dst_t0) -> hipError_t {
      hipError_t e = launch_norm2(v, P_F64, nsite, nsite, N, parts, st);
      if (e == hipSuccess) e = launch_reduce(parts, blas_nblocks(nsite), N, dst_all, st);
      if (e == hipSuccess && sf) e = launch_norm2(v, P_F64, nslice, nsite, N, parts, st);
      if (e == hipSuccess && sf) e = launch_reduce(parts, blas_nblocks(nslice), N, dst_t0, st);
      return e;
    };
    LQCD_HIP(norms(eta, scal + N, scal + 2 * N));
    if (x0) LQCD_HIP(norms(x0, scal + 4 * N, scal + 5 * N));
    std::vector<double> tmp(6 * N, 0.0);
    LQCD_HIP(hipMemcpyAsync(tmp.data(), scal, sizeof(double) * 6 * N, hipMemcpyDeviceToHost, st));
    LQCD_HIP(hipStreamSynchronize(st));
    for (int r = 0; r < N; ++r) {
      h_eta2[r] = tmp[N + r];
      if (!isfinite(tmp[N + r])) return fail(LQCD_ENUMERIC, "lqcd_solve: source %d has NaN/Inf entries", r);
      if (sf && tmp[2 * N + r] != 0.0)
        return fail(LQCD_EINVAL, "lqcd_solve: source %d is non-zero on the SF boundary slice t=0", r);
      if (x0 && !isfinite(tmp[4 * N + r]))
        return fail(LQCD_ENUMERIC, "lqcd_solve: initial guess %d has NaN/Inf entries", r);
      if (x0 && sf && tmp[5 * N + r] != 0.0)
        return fail(LQCD_EINVAL, "lqcd_solve: initial guess %d is non-zero on the SF boundary slice t=0", r);
    }
  }

  // ---- operands -------------------------------------------------------------
  const Vec E{m.E, P_F64, FRS}, X{m.X, P_F64, FRS}, TMP{m.TMP, P_F64, FRS}, R{m.R, P_F64, FRS},
      P{m.P, P_F64, FRS}, Q{m.Q, P_F64, FRS}, AP{m.AP, P_F64, FRS}, EH{m.EH, P_F64, FRS};
  const size_t full_bytes = (size_t)N * FRS * 16;
  CGState* cg = m.cg;
  const int* done = &cg[0].done;
  const int* skip_ru = &cg[0].skip_ru;
  // partials per rhs of an FP64 single-tile hop launch (setup, and the
  // reliable updates of FP64 phases), and of an FP64 launch in the
  // workspace's tuning (the reliable updates of low-precision phases)
  HopLaunch h1 = mk(c, P_F64);
  single_tile(h1);
  const int nb_hop = hop_nparts(h1);
  const int nb_hop_tuned = hop_nparts(mk(c, P_F64));
  // With FP32 operators at hand, a low-precision phase's reliable update
  // computes the recursion's new r = Dhat^+ s with them (s itself, and with
  // it the convergence test, stays FP64): r only has to be as accurate as the
  // FP32 recursion that continues from it.
  const bool ru32 = mixed && eo && u->U32 != nullptr && w->m.C32 != nullptr && w->m.Ci32 != nullptr;
  const int nb_ru32 = ru32 ? iter_parts(c, P_F32) : 0;

  LQCD_HIP(launch_pack(g->kg, (const double2*)eta, m.E, P_F64, N, false, st));
  if (x0)
    LQCD_HIP(launch_pack(g->kg, (const double2*)x0, m.X, P_F64, N, false, st));
  else
    LQCD_HIP(launch_fill_zero(m.X, full_bytes, st));

  // b = Dhat^+ eta_hat (eo) or Dw^+ eta (full) into R, with |b|^2
  int nb_op;  // partial count of the norm-producing operator launch
  if (eo) {
    LQCD_HIP(launch_fill_zero(m.EH, full_bytes, st));
    LQCD_HIP(launch_fill_zero(m.TMP, full_bytes, st));
    LQCD_HIP(clover_inv_apply(c, odd_part(E, V2), E, odd_part(TMP, V2), false, 0.0));  // A_oo^-1 eta_o
    LQCD_HIP(hop_oe_ident(c, E, odd_part(TMP, V2), EH));                               // eta_hat
    LQCD_HIP(hipMemcpyAsync(m.AP, m.EH, full_bytes, hipMemcpyDeviceToDevice, st));
    LQCD_HIP(launch_g5(m.AP, P_F64, V2, FRS, N, st));
    LQCD_HIP(hop_eo(dg(c), P_F64, AP, odd_part(TMP, V2), nullptr, 1));
    LQCD_HIP(hop_oe(dg(c), P_F64, AP, odd_part(TMP, V2), R, true, parts, nullptr, 1));
    nb_op = nb_hop;
  } else {
    LQCD_HIP(launch_pack(g->kg, (const double2*)eta, m.Q, P_F64, N, true, st));  // g5 eta
    LQCD_HIP(dw_full(dg(c), m.Q, m.R, true, parts, nullptr));
    nb_op = full_parts(c);
  }
  LQCD_HIP(launch_reduce(parts, nb_op, N, scal, st));

  // inner operands of a phase: the low-precision recursion (mixed solves) or
  // FP64 (plain solves, and the continuation of stalled mixed rhs)
  bool lo = false, lo16 = false;  // phase in low precision; BF16 operator operands
  Vec xi, ri, pi, qi, api, ti, pin, qin, tin;
  const long n_vec = eo ? 12 * V2 : 24 * V2;  // complex elements per rhs of one inner vector
  int lprec = P_F64, nb_blas = blas_nblocks(n_vec);
  auto select = [&](bool low) {
    lo = low;
    lo16 = low && ip == LQCD_BF16;
    lprec = low ? ip : P_F64;
    if (!low) {
      xi = X; ri = R; pi = P; qi = Q; api = AP; ti = odd_part(TMP, V2);
      pin = pi; qin = qi; tin = ti;
    } else {
      xi = Vec{m.xl, P_F32, HRS}; ri = Vec{m.rl, P_F32, HRS}; pi = Vec{m.pl, P_F32, HRS};
      qi = Vec{m.ql, P_F32, HRS}; api = Vec{m.apl, P_F32, HRS}; ti = Vec{m.tl, P_F32, HRS};
      if (lo16) {
        pin = Vec{m.pb, P_BF16, HRS}; qin = Vec{m.qb, P_BF16, HRS}; tin = Vec{m.tb, P_BF16, HRS};
      } else {
        pin = pi; qin = qi; tin = ti;
      }
    }
  };
  select(mixed);
  if (!mixed) {
    LQCD_HIP(hipMemcpyAsync(m.P, m.R, full_bytes, hipMemcpyDeviceToDevice, st));
  } else {
    LQCD_HIP(launch_fill_zero(m.xl, (size_t)N * HRS * 8, st));
    LQCD_HIP(launch_convert(m.R, P_F64, m.rl, P_F32, n_vec, FRS, HRS, N, st));
    if (lo16) LQCD_HIP(launch_convert(m.rl, P_F32, m.pb, P_BF16, n_vec, HRS, HRS, N, st));
    else LQCD_HIP(launch_convert(m.rl, P_F32, m.pl, P_F32, n_vec, HRS, HRS, N, st));
  }
  const int nr_tile = 0;  // 0: the workspace's tuned tile

  CGSetup cfg;
  cfg.nrhs = N;
  cfg.maxiter = prm->maxiter;
  cfg.tol = tol;
  cfg.inner_rel = 0.1 * tol;
  cfg.delta2 = mixed ? 0.01 : 0.0;
  cfg.ru_every = mixed ? (prm->reliable_every > 0 ? prm->reliable_every : 100) : 0;
  cfg.stall_max = mixed ? 8 : 0;
  LQCD_HIP(launch_cg_setup(cg, scal, scal + N, cfg, st));

  // ---- reliable update group (skips rhs without a pending request) ---------
  // The FP64 hops skip whole rhs tiles whose rhs have no pending request.  In
  // an FP64 phase the update writes the recursion's own residual R, so every
  // rhs is its own tile; in a low-precision phase the hops write only FP64
  // scratch (TMP, Q, AP) that the other rhs do not use (the fold, the
  // residual and the copy into the recursion skip them), so the hops run in
  // the workspace's FP64 tuning: with the rhs of a propagator requesting
  // their updates together, one multi-rhs launch instead of one per rhs.
  auto reliable_update = [&]() -> hipError_t {
    hipError_t e;
    if (eo) {
      const int ru_tile = lo ? 0 : 1;
      const int nb_ru = lo ? nb_hop_tuned : nb_hop;
      // (with deferred x updates the flush before the update has folded x)
      if (lo && !lo16 && (e = launch_ru_fold(m.X, FRS, m.xl, HRS, 12 * V2, N, cg, st))) return e;
      if ((e = hop_eo(c, P_F64, X, odd_part(TMP, V2), skip_ru, ru_tile))) return e;
      if ((e = hop_oe(c, P_F64, X, odd_part(TMP, V2), Q, false, nullptr, skip_ru, ru_tile))) return e;
      if ((e = launch_ru_sub(m.EH, m.Q, m.AP, 12 * V2, FRS, N, cg, parts2, st))) return e;
      if (lo && ru32) {
        // s rounded into FP32 scratch, Dhat^+ in the workspace's FP32 tuning,
        // the result copied into the recursion's r (pending rhs only).  The
        // scratch vectors are free at this point of an iteration: the FP32
        // t and Ap, and the FP32 q (FP32 recursion) or the two window slots
        // kept in the FP32 p (BF16 recursion), which the flush has consumed.
        const Vec s32{m.apl, P_F32, HRS}, t32{m.tl, P_F32, HRS}, r32{lo16 ? m.pl : m.ql, P_F32, HRS};
        if ((e = launch_ru_copy(m.AP, FRS, m.apl, HRS, 12 * V2, N, cg, st))) return e;
        if ((e = hop_eo(dg(c), P_F32, s32, t32, skip_ru, 0))) return e;
        if ((e = hop_oe(dg(c), P_F32, s32, t32, r32, true, parts, skip_ru, 0))) return e;
        if ((e = launch_ru_copy((const float2*)r32.p, HRS, m.rl, HRS, 12 * V2, N, cg, st))) return e;
        return launch_ru_finish(cg, parts2, blas_nblocks(12 * V2), parts, nb_ru32, N, st);
      }
      if ((e = hop_eo(dg(c), P_F64, AP, odd_part(TMP, V2), skip_ru, ru_tile))) return e;
      if ((e = hop_oe(dg(c), P_F64, AP, odd_part(TMP, V2), lo ? Q : R, true, parts, skip_ru, ru_tile))) return e;
      if (lo && (e = launch_ru_copy(m.Q, FRS, m.rl, HRS, 12 * V2, N, cg, st))) return e;
      return launch_ru_finish(cg, parts2, blas_nblocks(12 * V2), parts, nb_ru, N, st);
    }
    if ((e = dw_full(c, m.X, m.TMP, false, nullptr, skip_ru))) return e;
    if ((e = launch_ru_sub(m.E, m.TMP, m.AP, 24 * V2, FRS, N, cg, parts2, st))) return e;
    if ((e = dw_full(dg(c), m.AP, m.R, true, parts, skip_ru))) return e;
    return launch_ru_finish(cg, parts2, blas_nblocks(24 * V2), parts, full_parts(c), N, st);
  };

  // ---- initial guess: the first residual comes from a reliable update ------
  // (r = Dhat^+ (eta_hat - Dhat x0) in FP64, or Dw^+ (eta - Dw x0); an rhs
  // whose x0 already meets tol is done), then p = r
  if (x0) {
    LQCD_HIP(launch_cg_force_ru(cg, N, st));
    LQCD_HIP(reliable_update());
    LQCD_HIP(launch_cg_p(lo16 ? nullptr : pi.p, ri.p, pi.prec, n_vec, pi.rs, N, cg, lo16 ? pin.p : nullptr,
                         lo16 ? P_BF16 : P_F32, st));
  }

  // ---- one CG iteration (graph-capturable: kernels only) --------------------
  // eo: hop, hop (+g5, |Dhat p|^2), hop (+alpha), hop fused with the x/r
  // update (+|r|^2), then beta fused with the p update, or, every kRuStride-th
  // iteration, beta, the reliable-update group and the p update.
  // With BF16 operands the x updates of kXWindow iterations are deferred: the
  // search direction of iteration i lives in window buffer i mod kXWindow,
  // the p update writes the next buffer, the alpha step records alpha in the
  // same slot, and the flush before each reliable update adds all of them to
  // x (chunks and phases start at multiples of kRuStride, so the slot of an
  // iteration is fixed in a captured graph and every window is whole).
  constexpr int kRuStride = 5;
  static_assert(kRuStride == kXWindow, "x window = reliable-update stride");
  Vec pwin[kXWindow];
  PWindow pw{};
  if (mixed && ip == LQCD_BF16 && eo) {
    // the FP32 p and q vectors are not used by BF16-operand iterations; each
    // holds two BF16 vectors of the same rhs stride
    bf16x2* spare[4] = {(bf16x2*)m.pl, (bf16x2*)m.pl + (size_t)N * HRS, (bf16x2*)m.ql,
                        (bf16x2*)m.ql + (size_t)N * HRS};
    pwin[0] = Vec{m.pb, P_BF16, HRS};
    for (int j = 1; j < kXWindow; ++j) pwin[j] = Vec{spare[j - 1], P_BF16, HRS};
    for (int j = 0; j < kXWindow; ++j) pw.p[j] = (const bf16x2*)pwin[j].p;
    // rhs that finish early leave their later slots unwritten; zeros keep the
    // hops of partly finished rhs tiles finite
    LQCD_HIP(launch_fill_zero(m.pl, (size_t)N * HRS * 8, st));
    LQCD_HIP(launch_fill_zero(m.ql, (size_t)N * HRS * 8, st));
  }
  auto iteration = [&](int i) -> hipError_t {
    hipError_t e;
    int nb_r;  // |r|^2 partials per rhs
    const int slot = i % kXWindow;
    const bool win = lo16 && eo;  // deferred x updates
    if (win) pin = pwin[slot];
    if (eo) {
      const int nb_it = iter_parts(c, lprec);
      if ((e = hop_eo(c, lprec, pin, tin, done, nr_tile))) return e;
      if ((e = hop_oe(c, lprec, pin, tin, qin, true, parts, done, nr_tile))) return e;
      if ((e = hop_eo(dg(c), lprec, qin, tin, done, nr_tile, cg, parts, nb_it, win ? slot : -1)))
        return e;  // + alpha
      if ((e = hop_oe_xr(dg(c), lprec, qin, tin, win ? Vec{nullptr, P_F32, HRS} : xi, ri, pin, parts, cg, done)))
        return e;
      nb_r = nb_it;
    } else {
      if ((e = dw_full(c, (const double2*)pin.p, (double2*)qin.p, true, parts, done))) return e;
      if ((e = launch_cg_alpha(cg, parts, nb_op, N, st))) return e;
      if ((e = dw_full(dg(c), (const double2*)qin.p, (double2*)api.p, true, nullptr, done))) return e;
      if ((e = launch_cg_xr(xi.p, xi.prec, xi.rs, ri.p, pi.p, api.p, ri.prec, n_vec, ri.rs, N, cg, parts,
                            st)))
        return e;
      nb_r = nb_blas;
    }
    // with BF16 operands the search direction is kept in BF16 alone: the
    // recursion then updates x with the very vector the operator saw
    void* p = lo16 ? nullptr : pi.p;
    void* plo = lo16 ? pin.p : nullptr;
    void* pnext = win ? pwin[(slot + 1) % kXWindow].p : nullptr;
    const int plo_prec = lo16 ? P_BF16 : P_F32;
    if ((i + 1) % kRuStride != 0)
      return launch_cg_beta_p(p, ri.p, pi.prec, n_vec, pi.rs, N, cg, plo, plo_prec, parts, nb_r, st, pnext);
    if ((e = launch_cg_beta(cg, parts, nb_r, N, st))) return e;
    if (win && (e = launch_cg_xflush(m.xl, HRS, pw, n_vec, HRS, N, cg, st, m.X, FRS))) return e;
    if ((e = reliable_update())) return e;
    return launch_cg_p(p, ri.p, pi.prec, n_vec, pi.rs, N, cg, plo, plo_prec, st, pnext);
  };
  constexpr int K = 10 * kRuStride;      // iterations per chunk (host poll / graph)
  constexpr int K_TAIL = 2 * kRuStride;  // chunk length near convergence
  const bool use_graph = prm->use_graph && st != nullptr;
  // a chunk of len iterations, replayed from a graph cached in the workspace
  // (keyed by everything the captured launches depend on); chunk lengths
  // are multiples of kRuStride, so the reliable-update slots keep their
  // place in the iteration count whatever the mix of lengths
  auto run_chunk = [&](const int len) -> int {
    if (use_graph) {
      const int key_prec = lo ? ip : LQCD_F64;
      hipGraphExec_t exec = nullptr;
      for (auto& e : w->graphs)
        if (e.gauge_uid == u->uid && e.solver == prm->solver && e.inner_prec == key_prec && e.nrhs == N &&
            e.chunk == len && e.mu == c.mu && same_tuning(e.tune_inner, w->tune[key_prec]) &&
            same_tuning(e.tune_f64, w->tune[P_F64]) && same_tuning(e.tune_f32, w->tune[P_F32]))
          exec = e.exec;
      if (!exec) {
        LQCD_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int i = 0; i < len && e == hipSuccess; ++i) e = iteration(i);
        hipGraph_t gr = nullptr;
        hipError_t e2 = hipStreamEndCapture(st, &gr);
        if (e != hipSuccess) {
          if (gr) (void)hipGraphDestroy(gr);
          return hip_status(e, "graph capture");
        }
        if (e2 != hipSuccess) return hip_status(e2, "hipStreamEndCapture");
        hipError_t e3 = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
        if (e3 != hipSuccess) {
          (void)hipGraphDestroy(gr);
          return hip_status(e3, "hipGraphInstantiate");
        }
        w->graphs.push_back(GraphEntry{u->uid, prm->solver, key_prec, N, len, c.mu, w->tune[key_prec],
                                       w->tune[P_F64], w->tune[P_F32], gr, exec});
      }
      LQCD_HIP(hipGraphLaunch(exec, st));
      return LQCD_OK;
    }
    for (int i = 0; i < len; ++i) LQCD_HIP(iteration(i));
    return LQCD_OK;
  };

  std::vector<CGState> hs(N);
  const bool trace = getenv("LQCD_TRACE") != nullptr;  // per-chunk progress on stderr
  const long max_launched = (long)prm->maxiter + 3L * K;
  long launched = 0;  // iterations launched (done rhs skip theirs)
  // runs chunks until every rhs is done; returns whether one is CG_STALLED.
  // Chunks are K iterations long, or K_TAIL when every rhs still running is
  // predicted to reach its inner target within half a chunk: the prediction
  // extrapolates each rhs's |r|^2 decay rate since the previous poll, so the
  // last chunk does not launch up to K - 1 iterations past convergence.  The
  // first poll of a phase predicts nothing: |r|^2 falls fastest in the first
  // iterations, and a rate measured from iteration 0 would switch to short
  // chunks (and extra polls) too early.  The chunk lengths change only when
  // the host polls, never the arithmetic.
  auto run_phase = [&](bool& stalled) -> int {
    stalled = false;
    std::vector<double> rr_last(N, -1.0);  // < 0: no previous point
    std::vector<int> it_last(N, 0);
    int k_next = K;
    for (;;) {
      int rc2 = run_chunk(k_next);
      launched += k_next;
      if (rc2) return rc2;
      LQCD_HIP(hipMemcpyAsync(hs.data(), cg, sizeof(CGState) * N, hipMemcpyDeviceToHost, st));
      LQCD_HIP(hipStreamSynchronize(st));
      bool all_done = true;
      stalled = false;
      for (int r = 0; r < N; ++r) {
        all_done = all_done && hs[r].done;
        stalled = stalled || hs[r].status == CG_STALLED;
        if (trace)
          fprintf(stderr, "[lqcd] rhs %d iters %d done %d status %d rr/b2 %.3e rho %.3e rupd %d%s\n", r,
                  hs[r].iters, hs[r].done, hs[r].status, hs[r].rr / hs[r].bnorm2, sqrt(hs[r].rho2),
                  hs[r].rupd, lo ? "" : " fp64");
      }
      if (all_done || launched >= max_launched) return LQCD_OK;
      bool known = true;
      double need = 0.0;  // predicted iterations to the slowest inner target
      for (int r = 0; r < N; ++r) {
        if (hs[r].done) continue;
        const double rr = hs[r].rr;
        const int di = hs[r].iters - it_last[r];
        if (rr_last[r] > 0.0 && di > 0 && rr > 0.0 && rr < rr_last[r]) {
          const double rate = log(rr / rr_last[r]) / di;  // < 0
          if (rr > hs[r].target2) need = std::max(need, log(hs[r].target2 / rr) / rate);
        } else {
          known = false;
        }
        rr_last[r] = rr;
        it_last[r] = hs[r].iters;
      }
      k_next = (known && need + kRuStride <= K / 2) ? K_TAIL : K;
      if (trace) fprintf(stderr, "[lqcd] next chunk %d (predicted %.1f iterations, known %d)\n", k_next, need, known);
    }
  };
  bool stalled = false;
  rc = run_phase(stalled);
  if (rc) return rc;
  if (stalled) {
    // FP64 continuation of the stalled rhs from their current solution: the
    // first FP64 reliable update recomputes r, and p = r (beta = 0)
    LQCD_HIP(launch_axpby(1.0, m.xl, P_F32, 1.0, m.X, P_F64, n_vec, HRS, FRS, N, st));
    LQCD_HIP(launch_fill_zero(m.xl, (size_t)N * HRS * 8, st));
    LQCD_HIP(launch_fill_zero(m.P, full_bytes, st));
    LQCD_HIP(launch_cg_escalate(cg, N, st));
    select(false);
    LQCD_HIP(reliable_update());
    LQCD_HIP(launch_cg_p(m.P, m.R, P_F64, n_vec, FRS, N, cg, nullptr, P_F32, st));
    rc = run_phase(stalled);
    if (rc) return rc;
  }

  // ---- reconstruct the odd sites, unpack, FP64 full-lattice residual -------
  if (mixed) LQCD_HIP(launch_axpby(1.0, m.xl, P_F32, 1.0, m.X, P_F64, n_vec, HRS, FRS, N, st));
  if (eo) LQCD_HIP(clover_inv_apply(c, odd_part(E, V2), X, odd_part(X, V2), true, 0.5));
  LQCD_HIP(launch_unpack(g->kg, m.X, P_F64, (double2*)psi, N, st));
  LQCD_HIP(dw_full(c, m.X, m.TMP, false, nullptr, nullptr));
  LQCD_HIP(launch_sub_norm(m.E, m.TMP, m.AP, 24 * V2, FRS, N, parts, st));
  LQCD_HIP(launch_reduce(parts, blas_nblocks(24 * V2), N, scal + 3 * N, st));
  std::vector<double> fres(N);
  LQCD_HIP(hipMemcpyAsync(fres.data(), scal + 3 * N, sizeof(double) * N, hipMemcpyDeviceToHost, st));
  LQCD_HIP(hipMemcpyAsync(hs.data(), cg, sizeof(CGState) * N, hipMemcpyDeviceToHost, st));
  LQCD_HIP(hipStreamSynchronize(st));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int overall = LQCD_OK;
  for (int r = 0; r < N; ++r) {
    info[r].iters = hs[r].iters;
    info[r].reliable_updates = hs[r].rupd;
    info[r].restarts = hs[r].restarts;
    info[r].fp64_from = hs[r].fp64_from;
    info[r].reserved = 0;
    info[r].true_residual = (h_eta2[r] > 0.0) ? sqrt(fres[r] / h_eta2[r]) : 0.0;
    info[r].seconds = secs;
    int stt = LQCD_OK;
    if (hs[r].status == CG_NONFINITE) stt = LQCD_ENUMERIC;
    else if (hs[r].status != CG_CONVERGED || !(info[r].true_residual <= tol)) stt = LQCD_ENOCONV;
    info[r].status = stt;
    if (stt == LQCD_ENUMERIC) overall = LQCD_ENUMERIC;
    else if (stt != LQCD_OK && overall == LQCD_OK) overall = LQCD_ENOCONV;
  }
  if (overall != LQCD_OK) set_error("lqcd_solve: not every rhs reached tol=%g", tol);
  return overall;
}
