// C ABI: handles, validation, gauge import, workspace planning, clover
// caching and operator application.  Declarations and contracts are in
// include/lqcd.h.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <new>

#include "lqcd_internal.h"

using namespace lqcd;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local char g_last_error[512] = "";

namespace lqcd {
void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
}
int fail(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return status;
}
}  // namespace lqcd

extern "C" const char* lqcd_last_error(void) { return g_last_error; }

extern "C" const char* lqcd_strerror(int s) {
  switch (s) {
    case LQCD_OK: return "ok";
    case LQCD_PENDING: return "pending";
    case LQCD_EINVAL: return "invalid argument";
    case LQCD_ENOMEM: return "memory too small";
    case LQCD_EDEVICE: return "device error";
    case LQCD_ENOCONV: return "solver did not converge";
    case LQCD_ENUMERIC: return "numerical error";
    case LQCD_ENOTFOUND: return "not found";
    case LQCD_EBUSY: return "busy";
    case LQCD_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
extern "C" int lqcd_geom(const lqcd_geom_desc* d, lqcd_geom_t** out) {
  if (!d || !out) return fail(LQCD_EINVAL, "lqcd_geom: null pointer");
  *out = nullptr;
  int64_t V = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (d->L[mu] < 2 || (d->L[mu] & 1))
      return fail(LQCD_EINVAL, "lqcd_geom: extent L[%d]=%d must be even and >= 2", mu, d->L[mu]);
    V *= d->L[mu];
  }
  if (V >= (int64_t(1) << 31)) return fail(LQCD_EINVAL, "lqcd_geom: volume %lld too large", (long long)V);
  if (d->bc != LQCD_BC_PERIODIC && d->bc != LQCD_BC_SF && d->bc != LQCD_BC_OPEN)
    return fail(LQCD_EINVAL, "lqcd_geom: unknown boundary condition %d", d->bc);
  if (d->bc != LQCD_BC_PERIODIC && d->L[3] < 4)
    return fail(LQCD_EINVAL, "lqcd_geom: SF/open boundaries need T >= 4");
  for (int mu = 0; mu < 4; ++mu) {
    double a = hypot(d->theta_re[mu], d->theta_im[mu]);
    if (!(fabs(a - 1.0) <= 1e-12))
      return fail(LQCD_EINVAL, "lqcd_geom: |theta[%d]| = %.17g, must be 1", mu, a);
  }
  lqcd_geom_t* g = new (std::nothrow) lqcd_geom_t;
  if (!g) return fail(LQCD_ENOMEM, "lqcd_geom: host allocation failed");
  g->desc = *d;
  g->V = V;
  g->V2 = (int)(V / 2);
  g->V2p = (int)padded_sites(g->V2);
  KGeom& k = g->kg;
  memset(&k, 0, sizeof(k));
  for (int mu = 0; mu < 4; ++mu) k.L[mu] = d->L[mu];
  k.Lxh = d->L[0] / 2;
  k.V2 = g->V2;
  k.V2p = g->V2p;
  k.sy = k.Lxh;
  k.sz = k.Lxh * d->L[1];
  k.st = k.Lxh * d->L[1] * d->L[2];
  k.bc = d->bc;
  k.div_xh = make_fastdiv(k.Lxh);
  k.div_y = make_fastdiv(d->L[1]);
  k.div_z = make_fastdiv(d->L[2]);
  for (int mu = 0; mu < 4; ++mu) {
    double re = d->theta_re[mu], im = d->theta_im[mu];
    if (mu == 3 && d->bc != LQCD_BC_PERIODIC) re = im = 0.0;  // time hops cut at the boundary
    k.fwd_re[mu] = re;
    k.fwd_im[mu] = im;
    k.bwd_re[mu] = re;
    k.bwd_im[mu] = -im;
  }
  *out = g;
  return LQCD_OK;
}

extern "C" void lqcd_geom_free(lqcd_geom_t* g) { delete g; }
extern "C" int64_t lqcd_geom_volume(const lqcd_geom_t* g) { return g ? g->V : 0; }

// ---------------------------------------------------------------------------
// gauge field
// ---------------------------------------------------------------------------
static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// complex elements of one precision copy of the links: 4 directions x (9, or
// 6 with two rows per link) per site, both parities
static size_t link_elems(const lqcd_geom_t* g, int pmask) {
  return (size_t)2 * 4 * ((pmask & LQCD_PM_TWO_ROW) ? 6 : 9) * g->V2p;
}

extern "C" size_t lqcd_gauge_bytes(const lqcd_geom_t* g, int pmask) {
  if (!g) return 0;
  const size_t n = link_elems(g, pmask);
  size_t b = align_up(n * 16);
  if (pmask & LQCD_PM_F32) b += align_up(n * 8);
  if (pmask & LQCD_PM_BF16) b += align_up(n * 4);
  if (pmask & LQCD_PM_TWO_ROW) b += 256;  // flag of the SU(3) check
  return b;
}

static std::atomic<uint64_t> g_uid{1};

extern "C" int lqcd_gauge_create(const lqcd_geom_t* g, const void* U_dev, int pmask, void* mem,
                                 size_t mem_bytes, void* stream, lqcd_gauge_t** out) {
  if (!g || !U_dev || !mem || !out) return fail(LQCD_EINVAL, "lqcd_gauge_create: null pointer");
  *out = nullptr;
  if (pmask & ~15) return fail(LQCD_EINVAL, "lqcd_gauge_create: bad precision mask %d", pmask);
  const size_t need = lqcd_gauge_bytes(g, pmask);
  if (mem_bytes < need)
    return fail(LQCD_ENOMEM, "lqcd_gauge_create: %zu bytes given, %zu needed", mem_bytes, need);
  if (((uintptr_t)mem & 255) || ((uintptr_t)U_dev & 15))
    return fail(LQCD_EINVAL, "lqcd_gauge_create: misaligned device pointer");
  lqcd_gauge* u = new (std::nothrow) lqcd_gauge;
  if (!u) return fail(LQCD_ENOMEM, "lqcd_gauge_create: host allocation failed");
  const bool two_row = (pmask & LQCD_PM_TWO_ROW) != 0;
  const size_t n = link_elems(g, pmask);
  char* p = (char*)mem;
  u->g = g;
  u->pmask = pmask | LQCD_PM_F64;
  u->uid = g_uid.fetch_add(1);
  u->two_row = two_row ? 1 : 0;
  u->U64 = (double2*)p;
  p += align_up(n * 16);
  u->U32 = nullptr;
  u->U16 = nullptr;
  if (pmask & LQCD_PM_F32) {
    u->U32 = (float2*)p;
    p += align_up(n * 8);
  }
  if (pmask & LQCD_PM_BF16) {
    u->U16 = (bf16x2*)p;
    p += align_up(n * 4);
  }
  int* bad = two_row ? (int*)p : nullptr;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (bad) e = launch_fill_zero(bad, 256, st);
  if (e == hipSuccess)
    e = launch_import_gauge(g->kg, (const double2*)U_dev, u->U64, u->U32, u->U16, two_row, bad, st);
  int h_bad = 0;
  if (e == hipSuccess && bad) e = hipMemcpyAsync(&h_bad, bad, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && bad) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete u;
    return hip_status(e, "gauge import");
  }
  if (h_bad) {
    delete u;
    return fail(LQCD_EINVAL,
                "lqcd_gauge_create: LQCD_PM_TWO_ROW needs SU(3) links, but a third row differs from "
                "conj(row0 x row1) by more than 1e-10");
  }
  *out = u;
  return LQCD_OK;
}

extern "C" void lqcd_gauge_free(lqcd_gauge_t* u) { delete u; }

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
namespace lqcd {

WsLayout plan_ws(const lqcd_geom_t* g, int pmask, int nrhs, char* base) {
  WsLayout m;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* r = base ? base + off : nullptr;
    off += align_up(bytes);
    return r;
  };
  const size_t V2 = (size_t)g->V2p;  // field rows: sites per parity incl. padding
  m.C64 = (double2*)take(72 * V2 * 16);
  m.Ci64 = (double2*)take(36 * V2 * 16);
  if (pmask & LQCD_PM_F32) {
    m.C32 = (float2*)take(72 * V2 * 8);
    m.Ci32 = (float2*)take(36 * V2 * 8);
  }
  if (pmask & LQCD_PM_BF16) {
    m.C16 = (bf16x2*)take(72 * V2 * 4);
    m.Ci16 = (bf16x2*)take(36 * V2 * 4);
  }
  m.err_flag = (int*)take(256);
  const size_t full64 = (size_t)nrhs * 24 * V2 * 16;
  m.E = (double2*)take(full64);
  m.X = (double2*)take(full64);
  m.TMP = (double2*)take(full64);
  m.R = (double2*)take(full64);
  m.P = (double2*)take(full64);
  m.Q = (double2*)take(full64);
  m.AP = (double2*)take(full64);
  m.EH = (double2*)take(full64);
  if (pmask & (LQCD_PM_F32 | LQCD_PM_BF16)) {
    const size_t half32 = (size_t)nrhs * 12 * V2 * 8;
    m.xl = (float2*)take(half32);
    m.rl = (float2*)take(half32);
    m.pl = (float2*)take(half32);
    m.ql = (float2*)take(half32);
    m.apl = (float2*)take(half32);
    m.tl = (float2*)take(half32);
  }
  if (pmask & LQCD_PM_BF16) {
    const size_t half16 = (size_t)nrhs * 12 * V2 * 4;
    m.pb = (bf16x2*)take(half16);
    m.qb = (bf16x2*)take(half16);
    m.tb = (bf16x2*)take(half16);
  }
  const int hop_parts = hop_max_parts(g->V2);
  m.max_parts = hop_parts > 2048 ? hop_parts : 2048;
  m.partials = (double*)take((size_t)nrhs * m.max_parts * sizeof(double));
  m.partials2 = (double*)take((size_t)nrhs * m.max_parts * sizeof(double));
  m.cg = (CGState*)take((size_t)nrhs * sizeof(CGState));
  m.scal = (double*)take((size_t)8 * nrhs * sizeof(double));
  m.bytes = off;
  return m;
}

}  // namespace lqcd

extern "C" size_t lqcd_ws_bytes(const lqcd_geom_t* g, int pmask, int nrhs) {
  if (!g || nrhs < 1) return 0;
  return plan_ws(g, pmask, nrhs, nullptr).bytes;
}

extern "C" int lqcd_ws_create(const lqcd_geom_t* g, int pmask, int nrhs, void* mem, size_t mem_bytes,
                              lqcd_ws_t** out) {
  if (!g || !mem || !out) return fail(LQCD_EINVAL, "lqcd_ws_create: null pointer");
  *out = nullptr;
  if (nrhs < 1 || nrhs > 64) return fail(LQCD_EINVAL, "lqcd_ws_create: nrhs=%d out of range", nrhs);
  if (pmask & ~7) return fail(LQCD_EINVAL, "lqcd_ws_create: bad precision mask %d", pmask);
  if ((uintptr_t)mem & 255) return fail(LQCD_EINVAL, "lqcd_ws_create: memory not 256-byte aligned");
  WsLayout m = plan_ws(g, pmask, nrhs, (char*)mem);
  if (mem_bytes < m.bytes)
    return fail(LQCD_ENOMEM, "lqcd_ws_create: %zu bytes given, %zu needed", mem_bytes, m.bytes);
  lqcd_ws* w = new (std::nothrow) lqcd_ws;
  if (!w) return fail(LQCD_ENOMEM, "lqcd_ws_create: host allocation failed");
  w->g = g;
  w->pmask = pmask | LQCD_PM_F64;
  w->nrhs = nrhs;
  w->m = m;
  *out = w;
  return LQCD_OK;
}

extern "C" void lqcd_ws_free(lqcd_ws_t* w) {
  if (!w) return;
  for (auto& e : w->graphs) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
  }
  delete w;
}

extern "C" size_t lqcd_vec_bytes(const lqcd_geom_t* g, int prec, int nrhs, int nparity) {
  if (!g || nrhs < 1 || nparity < 1 || nparity > 2 || prec < 0 || prec > 2) return 0;
  return (size_t)nrhs * nparity * 12 * g->V2p * elem_bytes(prec);
}

// ---------------------------------------------------------------------------
// clover (Csw!)
// ---------------------------------------------------------------------------
namespace lqcd {

int check_dirac(const lqcd_dirac* d) {
  if (!d) return fail(LQCD_EINVAL, "null Dirac parameters");
  if (!(d->kappa > 0.0) || !isfinite(d->kappa)) return fail(LQCD_EINVAL, "kappa must be > 0");
  if (!isfinite(d->csw) || !isfinite(d->cF)) return fail(LQCD_EINVAL, "csw and cF must be finite");
  if (!isfinite(d->mu)) return fail(LQCD_EINVAL, "mu must be finite");
  return LQCD_OK;
}

int ensure_clover(const lqcd_gauge_t* u, const lqcd_dirac* d, lqcd_ws_t* w, hipStream_t st) {
  int rc = check_dirac(d);
  if (rc) return rc;
  if (u->g != w->g && memcmp(&u->g->desc, &w->g->desc, sizeof(lqcd_geom_desc)) != 0)
    return fail(LQCD_EINVAL, "gauge field and workspace have different geometries");
  const int want = w->pmask & u->pmask;
  if (w->clover_valid && w->clover_uid == u->uid && w->kappa == d->kappa && w->csw == d->csw &&
      w->cF == d->cF && w->mu == d->mu && (w->clover_pmask & want) == want)
    return LQCD_OK;
  CloverLaunch c;
  c.g = w->g->kg;
  c.U64 = u->U64;
  c.two_row = u->two_row;
  c.m0 = 1.0 / (2.0 * d->kappa) - 4.0;
  c.csw = d->csw;
  c.cF = d->cF;
  c.mu = d->mu;
  c.C64 = w->m.C64;
  c.Ci64 = w->m.Ci64;
  c.C32 = (want & LQCD_PM_F32) ? w->m.C32 : nullptr;
  c.Ci32 = (want & LQCD_PM_F32) ? w->m.Ci32 : nullptr;
  c.C16 = (want & LQCD_PM_BF16) ? w->m.C16 : nullptr;
  c.Ci16 = (want & LQCD_PM_BF16) ? w->m.Ci16 : nullptr;
  c.err_flag = w->m.err_flag;
  LQCD_HIP(launch_fill_zero(w->m.err_flag, 256, st));
  LQCD_HIP(launch_clover(c, st));
  int err = 0;
  LQCD_HIP(hipMemcpyAsync(&err, w->m.err_flag, sizeof(int), hipMemcpyDeviceToHost, st));
  LQCD_HIP(hipStreamSynchronize(st));
  w->clover_valid = false;
  if (err) return fail(LQCD_ENUMERIC, "clover block numerically singular (kappa=%g csw=%g)", d->kappa, d->csw);
  w->clover_valid = true;
  w->clover_uid = u->uid;
  w->kappa = d->kappa;
  w->csw = d->csw;
  w->cF = d->cF;
  w->mu = d->mu;
  w->clover_pmask = want | LQCD_PM_F64;
  return LQCD_OK;
}

}  // namespace lqcd

extern "C" int lqcd_clover(const lqcd_gauge_t* u, const lqcd_dirac* d, lqcd_ws_t* w, void* stream) {
  if (!u || !d || !w) return fail(LQCD_EINVAL, "lqcd_clover: null pointer");
  return ensure_clover(u, d, w, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// operator application
// ---------------------------------------------------------------------------
namespace lqcd {

struct OpCtx {
  const lqcd_gauge* u;
  lqcd_ws* w;
  int prec;
  int nrhs;
  hipStream_t st;
  double mu;  // twisted mass
};

static const void* links_of(const lqcd_gauge* u, int prec) {
  return prec == P_F64 ? (const void*)u->U64 : (prec == P_F32 ? (const void*)u->U32 : (const void*)u->U16);
}
static const void* clov_of(const lqcd_ws* w, int prec) {
  return prec == P_F64 ? (const void*)w->m.C64 : (prec == P_F32 ? (const void*)w->m.C32 : (const void*)w->m.C16);
}
static const void* cloi_of(const lqcd_ws* w, int prec) {
  return prec == P_F64 ? (const void*)w->m.Ci64 : (prec == P_F32 ? (const void*)w->m.Ci32 : (const void*)w->m.Ci16);
}

// dag: the launch belongs to the adjoint operator g5 D(-mu) g5 (twisted
// mass -mu, adjoint odd-site inverse); no difference for mu = 0
static HopLaunch base_launch(const OpCtx& c, bool dag) {
  HopLaunch h;
  memset(&h, 0, sizeof(h));
  h.g = c.w->g->kg;
  h.prec = h.in_prec = h.out_prec = c.prec;
  h.U = links_of(c.u, c.prec);
  h.two_row = c.u->two_row;
  h.nrhs = c.nrhs;
  h.hop = true;
  h.tm_mu = dag ? -c.mu : c.mu;
  h.tm_post = c.mu != 0.0 ? 1 : 0;
  apply_tuning(h, c.w->tune[c.prec]);
  if (c.mu != 0.0) single_tile(h);  // twisted-mass kernels: one rhs per thread
  return h;
}

// full-layout element strides
static long full_rs(const lqcd_geom_t* g) { return 24L * g->V2p; }
static long par_off(const lqcd_geom_t* g) { return 12L * g->V2p; }

static char* elem_ptr(void* base, int prec, long elems) {
  return (char*)base + (size_t)elems * elem_bytes(prec);
}

// out (full) = Dw y on both parities, optional g5 on the output and partials
static hipError_t apply_dw_full(const OpCtx& c, const void* y, void* out, bool g5, double* partials,
                                bool dag = false) {
  const lqcd_geom_t* g = c.w->g;
  HopLaunch h = base_launch(c, dag);
  h.both = true;
  h.par_stride = par_off(g);
  h.cpre_par = 36L * g->V2p;
  h.y = y;
  h.z = y;
  h.out = out;
  h.y_rs = h.z_rs = h.out_rs = full_rs(g);
  h.Cpre = clov_of(c.w, c.prec);
  h.pre = PRE_CLOV;
  h.post = POST_NONE;
  h.scale = -0.5;
  h.g5 = g5;
  h.partials = partials;
  return launch_hop(h, c.st);
}

// t_o = A_oo^{-1} D_oe y_e (tmp odd part of `t` full vector)
static hipError_t apply_hop_eo(const OpCtx& c, const void* y_full, void* t_full, bool dag = false) {
  const lqcd_geom_t* g = c.w->g;
  HopLaunch h = base_launch(c, dag);
  h.p_out = 1;
  h.y = y_full;
  h.out = elem_ptr(t_full, c.prec, par_off(g));
  h.y_rs = h.out_rs = full_rs(g);
  h.Cpost = cloi_of(c.w, c.prec);
  h.Ctm = elem_ptr((void*)clov_of(c.w, c.prec), c.prec, 36L * g->V2p);  // A on the odd sites
  h.pre = PRE_NONE;
  h.post = POST_CLOV;
  h.scale = -0.5;
  return launch_hop(h, c.st);
}

// out_e = A_ee z_e + 1/2 H t_o  (= Dhat z when t = A_oo^{-1} D_oe z)
static hipError_t apply_hop_oe(const OpCtx& c, const void* z_full, const void* t_full, void* out_full,
                               bool g5, double* partials, bool dag = false) {
  const lqcd_geom_t* g = c.w->g;
  HopLaunch h = base_launch(c, dag);
  h.p_out = 0;
  h.y = elem_ptr((void*)t_full, c.prec, par_off(g));
  h.z = z_full;
  h.out = out_full;
  h.y_rs = h.z_rs = h.out_rs = full_rs(g);
  h.Cpre = clov_of(c.w, c.prec);
  h.pre = PRE_CLOV;
  h.post = POST_NONE;
  h.scale = 0.5;
  h.g5 = g5;
  h.partials = partials;
  return launch_hop(h, c.st);
}

}  // namespace lqcd

extern "C" int lqcd_dw_apply(const lqcd_gauge_t* u, const lqcd_dirac* d, int op, int prec, int layout,
                             int nrhs, const void* in, void* out, lqcd_ws_t* w, void* stream) {
  if (!u || !d || !in || !out || !w) return fail(LQCD_EINVAL, "lqcd_dw_apply: null pointer");
  if (op < LQCD_OP_DW || op > LQCD_OP_HOP_OE) return fail(LQCD_EINVAL, "lqcd_dw_apply: bad op %d", op);
  if (prec < 0 || prec > 2) return fail(LQCD_EINVAL, "lqcd_dw_apply: bad precision %d", prec);
  if (layout != LQCD_LAYOUT_CANON && layout != LQCD_LAYOUT_INTERNAL)
    return fail(LQCD_EINVAL, "lqcd_dw_apply: bad layout %d", layout);
  if (nrhs < 1 || nrhs > w->nrhs) return fail(LQCD_EINVAL, "lqcd_dw_apply: nrhs=%d (workspace %d)", nrhs, w->nrhs);
  const int pbit = 1 << prec;
  if (!(u->pmask & pbit) || !(w->pmask & pbit))
    return fail(LQCD_EINVAL, "lqcd_dw_apply: precision %d not held by gauge field and workspace", prec);
  if (in == out) return fail(LQCD_EINVAL, "lqcd_dw_apply: in and out must differ");
  hipStream_t st = (hipStream_t)stream;
  int rc = ensure_clover(u, d, w, st);
  if (rc) return rc;

  const lqcd_geom_t* g = w->g;
  OpCtx c{u, w, prec, nrhs, st, d->mu};
  // internal-layout operands: caller's memory or workspace FP64 slots reused
  // as storage of any precision (they are the widest)
  const void* vin = in;
  void* vout = out;
  const bool canon = (layout == LQCD_LAYOUT_CANON);
  const bool g5in = (op == LQCD_OP_DW_DAG || op == LQCD_OP_SCHUR_DAG);
  if (canon) {
    vin = w->m.X;
    vout = w->m.TMP;
    LQCD_HIP(launch_pack(g->kg, (const double2*)in, (void*)vin, prec, nrhs, g5in, st));
  }
  const size_t full_bytes = (size_t)nrhs * 24 * g->V2p * elem_bytes(prec);
  void* tmp = w->m.R;  // scratch full vector
  void* tmp2 = w->m.P;
  switch (op) {
    case LQCD_OP_DW:
    case LQCD_OP_G5DW:
      LQCD_HIP(apply_dw_full(c, vin, vout, op == LQCD_OP_G5DW, nullptr));
      break;
    case LQCD_OP_DW_DAG:
      if (!canon) {  // g5 on the input of an internal vector: copy with g5
        LQCD_HIP(hipMemcpyAsync(tmp2, vin, full_bytes, hipMemcpyDeviceToDevice, st));
        LQCD_HIP(launch_g5(tmp2, prec, g->V2p, 12L * g->V2p, 2 * nrhs, st));
        vin = tmp2;
      }
      LQCD_HIP(apply_dw_full(c, vin, vout, true, nullptr, true));
      break;
    case LQCD_OP_DWDAGDW:  // g5 D(-mu) g5 D(mu)
      LQCD_HIP(apply_dw_full(c, vin, tmp, true, nullptr));
      LQCD_HIP(apply_dw_full(c, tmp, vout, true, nullptr, true));
      break;
    case LQCD_OP_SCHUR:
    case LQCD_OP_SCHUR_DAG:
      if (op == LQCD_OP_SCHUR_DAG && !canon) {
        LQCD_HIP(hipMemcpyAsync(tmp2, vin, full_bytes, hipMemcpyDeviceToDevice, st));
        LQCD_HIP(launch_g5(tmp2, prec, g->V2p, 12L * g->V2p, 2 * nrhs, st));
        vin = tmp2;
      }
      if (canon) LQCD_HIP(launch_fill_zero(vout, full_bytes, st));
      {
        const bool dag = (op == LQCD_OP_SCHUR_DAG);  // g5 Dhat(-mu) g5
        LQCD_HIP(apply_hop_eo(c, vin, tmp, dag));
        LQCD_HIP(apply_hop_oe(c, vin, tmp, vout, dag, nullptr, dag));
      }
      break;
    case LQCD_OP_SCHUR_NORMAL:  // g5 Dhat(-mu) g5 Dhat(mu)
      if (canon) LQCD_HIP(launch_fill_zero(vout, full_bytes, st));
      LQCD_HIP(apply_hop_eo(c, vin, tmp));
      LQCD_HIP(apply_hop_oe(c, vin, tmp, tmp2, true, nullptr));
      LQCD_HIP(apply_hop_eo(c, tmp2, tmp, true));
      LQCD_HIP(apply_hop_oe(c, tmp2, tmp, vout, true, nullptr, true));
      break;
    case LQCD_OP_HOP_EO:
      if (canon) LQCD_HIP(launch_fill_zero(vout, full_bytes, st));
      LQCD_HIP(apply_hop_eo(c, vin, vout));
      break;
    case LQCD_OP_HOP_OE: {
      if (canon) LQCD_HIP(launch_fill_zero(vout, full_bytes, st));
      LQCD_HIP(apply_hop_oe(c, vin, vin, vout, false, nullptr));
      break;
    }
  }
  if (canon) LQCD_HIP(launch_unpack(g->kg, vout, prec, (double2*)out, nrhs, st));
  return LQCD_OK;
}

// ---------------------------------------------------------------------------
// meson two-point functions
// ---------------------------------------------------------------------------
namespace lqcd {
int meson_check(const char* who, const lqcd_geom_t* g, const void* psi, int npairs, const int32_t* pairs,
                const void* C, const void* G) {
  if (!g || !psi) return fail(LQCD_EINVAL, "%s: null pointer", who);
  if (npairs < 0 || npairs > kMaxMesonPairs)
    return fail(LQCD_EINVAL, "%s: npairs=%d (0..%d)", who, npairs, kMaxMesonPairs);
  if (npairs > 0 && (!pairs || !C)) return fail(LQCD_EINVAL, "%s: pairs and C needed for npairs > 0", who);
  if (npairs == 0 && !G) return fail(LQCD_EINVAL, "%s: nothing to compute (no pairs, no G)", who);
  for (int p = 0; p < 2 * npairs; ++p)
    if (pairs[p] < 0 || pairs[p] > 15) return fail(LQCD_EINVAL, "%s: gamma mask %d (0..15)", who, pairs[p]);
  if (((uintptr_t)psi & 15) || ((uintptr_t)C & 15) || ((uintptr_t)G & 15))
    return fail(LQCD_EINVAL, "%s: misaligned device pointer", who);
  return LQCD_OK;
}

size_t meson_scratch_bytes(const lqcd_geom_t* g) {
  const long V3 = (long)g->desc.L[0] * g->desc.L[1] * g->desc.L[2];
  return (size_t)g->desc.L[3] * meson_nchunk(V3) * 256 * sizeof(double2);
}
}  // namespace lqcd

extern "C" int lqcd_meson(const lqcd_geom_t* g, const void* psi, int npairs, const int32_t* pairs, void* C,
                          void* G, lqcd_ws_t* w, void* stream) {
  if (!w) return fail(LQCD_EINVAL, "lqcd_meson: null pointer");
  const int rc = meson_check("lqcd_meson", g, psi, npairs, pairs, C, G);
  if (rc) return rc;
  if (w->g != g && memcmp(&w->g->desc, &g->desc, sizeof(lqcd_geom_desc)) != 0)
    return fail(LQCD_EINVAL, "lqcd_meson: workspace of another geometry");
  const size_t need = meson_scratch_bytes(g);
  const size_t have = (size_t)8 * w->nrhs * 24 * g->V2p * sizeof(double2);  // the FP64 vectors E..EH
  if (need > have) return fail(LQCD_EINVAL, "lqcd_meson: workspace scratch %zu < %zu bytes", have, need);
  double2* outs[kMaxMesonPairs];
  for (int p = 0; p < npairs; ++p) outs[p] = (double2*)C + (size_t)p * g->desc.L[3];
  LQCD_HIP(launch_meson(g->kg, (const double2*)psi, npairs, pairs, outs, 1.0, (double2*)G, w->m.E,
                        (hipStream_t)stream));
  return LQCD_OK;
}

// ---------------------------------------------------------------------------
// Schroedinger functional: boundary source and f_P, f_A
// ---------------------------------------------------------------------------
extern "C" int lqcd_sf_source(const lqcd_gauge_t* u, void* eta, void* stream) {
  if (!u || !eta) return fail(LQCD_EINVAL, "lqcd_sf_source: null pointer");
  const lqcd_geom_t* g = u->g;
  if (g->desc.bc != LQCD_BC_SF) return fail(LQCD_EINVAL, "lqcd_sf_source: the gauge field is not SF");
  if ((uintptr_t)eta & 15) return fail(LQCD_EINVAL, "lqcd_sf_source: misaligned device pointer");
  hipStream_t st = (hipStream_t)stream;
  LQCD_HIP(launch_fill_zero(eta, (size_t)12 * g->V * 12 * sizeof(double2), st));
  LQCD_HIP(launch_sf_source(g->kg, u->U64, u->two_row, (double2*)eta, st));
  return LQCD_OK;
}

extern "C" int lqcd_sf_correlators(const lqcd_gauge_t* u, const lqcd_solve_params* prm, void* eta, void* psi,
                                   void* fP, void* fA, lqcd_ws_t* w, void* stream, lqcd_solve_info* info) {
  if (!u || !prm || !eta || !psi || !fP || !fA || !w || !info)
    return fail(LQCD_EINVAL, "lqcd_sf_correlators: null pointer");
  if (w->nrhs < 12) return fail(LQCD_EINVAL, "lqcd_sf_correlators: workspace for %d < 12 rhs", w->nrhs);
  if (((uintptr_t)fP & 15) || ((uintptr_t)fA & 15))
    return fail(LQCD_EINVAL, "lqcd_sf_correlators: misaligned device pointer");
  int rc = lqcd_sf_source(u, eta, stream);
  if (rc) return rc;
  lqcd_solve_params p12 = *prm;
  p12.nrhs = 12;
  rc = lqcd_solve(u, &p12, eta, psi, w, stream, info);
  if (rc) return rc;
  // f_P = 1/2 C(g5, g5), f_A = -1/2 C(g5 g_t, g5) = 1/2 C(Gamma_7, g5)
  const int32_t pairs[4] = {15, 15, 7, 15};
  double2* outs[2] = {(double2*)fP, (double2*)fA};
  LQCD_HIP(launch_meson(u->g->kg, (const double2*)psi, 2, pairs, outs, 0.5, nullptr, w->m.E, (hipStream_t)stream));
  return LQCD_OK;
}

// ---------------------------------------------------------------------------
// tuning
// ---------------------------------------------------------------------------
extern "C" int lqcd_ws_set_tuning(lqcd_ws_t* w, int prec, const lqcd_tuning* t) {
  if (!w || !t) return fail(LQCD_EINVAL, "lqcd_ws_set_tuning: null pointer");
  if (prec < 0 || prec > 2) return fail(LQCD_EINVAL, "lqcd_ws_set_tuning: bad precision %d", prec);
  if (t->nr_tile < 1 || t->nr_tile > 3 || t->block_order < 0 || t->block_order > 6 ||
      (t->rhs_lanes != 1 && t->rhs_lanes != 2 && t->rhs_lanes != 4) || (t->flags & ~(LQCD_TUNE_NT_STORE | LQCD_TUNE_CACHED_GAUGE | (3 << LQCD_TUNE_OCC_SHIFT) |
                     LQCD_TUNE_DIR_SPLIT)))
    return fail(LQCD_EINVAL, "lqcd_ws_set_tuning: value out of range");
  w->tune[prec] = *t;
  return LQCD_OK;
}

extern "C" int lqcd_ws_get_tuning(const lqcd_ws_t* w, int prec, lqcd_tuning* t) {
  if (!w || !t) return fail(LQCD_EINVAL, "lqcd_ws_get_tuning: null pointer");
  if (prec < 0 || prec > 2) return fail(LQCD_EINVAL, "lqcd_ws_get_tuning: bad precision %d", prec);
  *t = w->tune[prec];
  return LQCD_OK;
}

extern "C" int lqcd_autotune(const lqcd_gauge_t* u, const lqcd_dirac* d, int prec, int nrhs, lqcd_ws_t* w,
                             void* stream, lqcd_tuning* best, double* best_us) {
  if (!u || !d || !w) return fail(LQCD_EINVAL, "lqcd_autotune: null pointer");
  if (prec < 0 || prec > 2) return fail(LQCD_EINVAL, "lqcd_autotune: bad precision %d", prec);
  if (nrhs < 1 || nrhs > w->nrhs) return fail(LQCD_EINVAL, "lqcd_autotune: nrhs=%d (workspace %d)", nrhs, w->nrhs);
  const int pbit = 1 << prec;
  if (!(u->pmask & pbit) || !(w->pmask & pbit))
    return fail(LQCD_EINVAL, "lqcd_autotune: precision %d not held by gauge field and workspace", prec);
  hipStream_t st = (hipStream_t)stream;
  int rc = ensure_clover(u, d, w, st);
  if (rc) return rc;
  // operands: two full-layout vectors of the FP64 slots (wide enough for any precision)
  const size_t full_bytes = (size_t)nrhs * 24 * w->g->V2p * elem_bytes(prec);
  LQCD_HIP(launch_fill_zero(w->m.X, full_bytes, st));
  hipEvent_t e0, e1;
  LQCD_HIP(hipEventCreate(&e0));
  LQCD_HIP(hipEventCreate(&e1));
  const lqcd_tuning saved = w->tune[prec];
  const int keep = saved.flags & LQCD_TUNE_DIR_SPLIT;  // the caller's choice
  double best_t = 1e300;
  lqcd_tuning best_cfg = saved;
  OpCtx c{u, w, prec, nrhs, st, d->mu};
  hipError_t err = hipSuccess;
  // LQCD_TUNE_LOG=1: every candidate's time on stderr (diagnostics)
  const char* log_env = getenv("LQCD_TUNE_LOG");
  const bool log_trials = log_env && log_env[0] == '1';
  // times the workspace's current tuning; keeps it if it is the fastest so far
  auto trial = [&]() {
    auto once = [&]() -> hipError_t {
      hipError_t e = apply_hop_eo(c, w->m.X, w->m.R);
      if (e == hipSuccess) e = apply_hop_oe(c, w->m.X, w->m.R, w->m.TMP, false, nullptr);
      return e;
    };
    for (int i = 0; i < 2 && err == hipSuccess; ++i) err = once();
    // the fastest of several timed applications: robust to a stray slow one
    const int reps = 6;
    double us = 1e300;
    for (int i = 0; i < reps && err == hipSuccess; ++i) {
      err = hipEventRecord(e0, st);
      if (err == hipSuccess) err = once();
      if (err == hipSuccess) err = hipEventRecord(e1, st);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err == hipSuccess && 1e3 * ms < us) us = 1e3 * ms;
    }
    if (err == hipSuccess && log_trials) {
      const lqcd_tuning& t = w->tune[prec];
      fprintf(stderr, "lqcd_autotune V=%lld prec=%d nrhs=%d nr_tile=%d rhs_lanes=%d order=%d flags=%d us=%.2f\n",
              (long long)w->g->V, prec, nrhs, t.nr_tile, t.rhs_lanes, t.block_order, t.flags, us);
    }
    if (err == hipSuccess && us < best_t) {
      best_t = us;
      best_cfg = w->tune[prec];
    }
  };
  // pass 1: rhs lanes, rhs tile, block order, store and load kinds
  for (int rl = 1; rl <= 4 && err == hipSuccess; rl *= 2) {
    if (nrhs % rl || (prec == P_F64 && rl > 1)) continue;
    for (int nr = 1; nr <= 3 && err == hipSuccess; ++nr) {
      if (nrhs % (nr * rl)) continue;
      if (keep && (nr != 1 || rl != 1)) continue;  // the split's shape only
      for (int cfg = 0; cfg < 28 && err == hipSuccess; ++cfg) {
        const int order = cfg >> 2;
        const int flags = ((cfg & 1) ? LQCD_TUNE_NT_STORE : 0) | ((cfg & 2) ? LQCD_TUNE_CACHED_GAUGE : 0) | keep;
        w->tune[prec] = lqcd_tuning{nr, order, rl, flags};
        trial();
      }
    }
  }
  // pass 2: occupancy caps on the best configuration
  const lqcd_tuning base = best_cfg;
  for (int level = 1; level <= 3 && err == hipSuccess; ++level) {
    w->tune[prec] = base;
    w->tune[prec].flags = (base.flags & ~(3 << LQCD_TUNE_OCC_SHIFT)) | (level << LQCD_TUNE_OCC_SHIFT);
    trial();
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) {
    w->tune[prec] = saved;
    return hip_status(err, "lqcd_autotune");
  }
  w->tune[prec] = best_cfg;
  tune_cache_put(u, prec, nrhs, d->mu != 0.0, best_cfg, best_t);
  if (best) *best = best_cfg;
  if (best_us) *best_us = best_t;
  return LQCD_OK;
}
