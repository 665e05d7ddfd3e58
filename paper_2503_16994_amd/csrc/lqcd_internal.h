// Internal host-side state behind the opaque handles of lqcd.h.
#pragma once

#include <stdarg.h>
#include <stdio.h>

#include <string>
#include <vector>

#include "../../include/lqcd.h"
#include "lqcd_kernels.h"

struct lqcd_geom {
  lqcd_geom_desc desc;
  lqcd::KGeom kg;
  int64_t V;
  int V2;
  int V2p;  // V2 rounded up to the 64-site layout tile
};

struct lqcd_gauge {
  const lqcd_geom_t* g;
  int pmask;
  uint64_t uid;  // distinguishes gauge fields for the clover cache
  int two_row;   // links stored as their first two rows
  double2* U64;
  float2* U32;
  lqcd::bf16x2* U16;
};

// Device memory map of a workspace (all pointers into the caller's memory).
struct WsLayout {
  size_t bytes = 0;
  // clover: A on both parities (tiled 36-component fields), inverse on the odd sites
  double2 *C64 = nullptr, *Ci64 = nullptr;
  float2 *C32 = nullptr, *Ci32 = nullptr;
  lqcd::bf16x2 *C16 = nullptr, *Ci16 = nullptr;
  int* err_flag = nullptr;
  // FP64 full-lattice vectors [nrhs][2 parities] of tiled 12-component fields
  double2 *E = nullptr, *X = nullptr, *TMP = nullptr, *R = nullptr, *P = nullptr, *Q = nullptr,
          *AP = nullptr, *EH = nullptr;
  // inner-precision half vectors [nrhs] of tiled 12-component fields (FP32) and BF16 copies
  float2 *xl = nullptr, *rl = nullptr, *pl = nullptr, *ql = nullptr, *apl = nullptr, *tl = nullptr;
  lqcd::bf16x2 *pb = nullptr, *qb = nullptr, *tb = nullptr;
  // reductions
  double* partials = nullptr;  // [nrhs][max_parts]
  double* partials2 = nullptr; // [nrhs][max_parts]
  int max_parts = 0;
  lqcd::CGState* cg = nullptr; // [nrhs]
  double* scal = nullptr;      // [8][nrhs]
};

// A captured chunk of solver iterations, valid for the workspace's lifetime
// (its kernels read and write only the gauge field and workspace memory).
// A captured chunk of CG iterations.  Its launches depend on the gauge
// field, the solver, the precision of the recursion, the rhs count, the chunk
// length and the hop-kernel tunings of that precision and of FP64 (reliable
// updates); the workspace's buffers are fixed for its lifetime.
struct GraphEntry {
  uint64_t gauge_uid;
  int solver, inner_prec, nrhs, chunk;
  double mu;  // twisted mass (a kernel argument of the captured launches)
  lqcd_tuning tune_inner, tune_f64, tune_f32;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

inline bool same_tuning(const lqcd_tuning& a, const lqcd_tuning& b) {
  return a.nr_tile == b.nr_tile && a.block_order == b.block_order && a.rhs_lanes == b.rhs_lanes &&
         a.flags == b.flags;
}

struct lqcd_ws {
  const lqcd_geom_t* g;
  int pmask;
  int nrhs;
  WsLayout m;
  // clover cache key
  bool clover_valid = false;
  uint64_t clover_uid = 0;
  double kappa = 0, csw = 0, cF = 0, mu = 0;
  int clover_pmask = 0;
  std::vector<GraphEntry> graphs;
  lqcd_tuning tune[3] = {{1, 1, 1, 0}, {1, 1, 1, 0}, {1, 1, 1, 0}};  // nr, order, lanes, flags
};

namespace lqcd {

void set_error(const char* fmt, ...);
int fail(int status, const char* fmt, ...);
WsLayout plan_ws(const lqcd_geom_t* g, int pmask, int nrhs, char* base);
int ensure_clover(const lqcd_gauge_t* u, const lqcd_dirac* d, lqcd_ws_t* w, hipStream_t st);
int check_dirac(const lqcd_dirac* d);
// argument checks shared by the meson entry points (status, last error set)
int meson_check(const char* who, const lqcd_geom_t* g, const void* psi, int npairs, const int32_t* pairs,
                const void* C, const void* G);
// FP64 complex partials of the meson contraction: T x chunks x 256 entries
size_t meson_scratch_bytes(const lqcd_geom_t* g);
// adds an autotuning result to the process-wide tuning cache (lqcd_tune.hip)
void tune_cache_put(const lqcd_gauge_t* u, int prec, int nrhs, int twisted, const lqcd_tuning& t, double us);

inline int hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return LQCD_OK;
  return fail(LQCD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define LQCD_HIP(call)                                        \
  do {                                                        \
    hipError_t _e = (call);                                   \
    if (_e != hipSuccess) return ::lqcd::hip_status(_e, #call); \
  } while (0)

// Description of one hop launch over a full-layout vector: parity p_out of
// `out` from parity 1-p_out of `y` (and p_out of `z`).
struct HopSpec {
  int prec;  // links/clover precision
  int in_prec, out_prec;
  int pre, post;
  bool hop = true;
  bool g5 = false;
  double scale = 0.0;
};

// rhs tiling of a launch over nrhs fields: rhs_lanes lanes per site, each
// with nr_tile rhs; both are reduced until their product divides nrhs
inline void apply_tuning(HopLaunch& h, const lqcd_tuning& t) {
  int rl = (t.rhs_lanes == 2 || t.rhs_lanes == 4) ? t.rhs_lanes : 1;
  int nr = t.nr_tile < 1 ? 1 : (t.nr_tile > 3 ? 3 : t.nr_tile);
  while (h.nrhs % rl) rl >>= 1;
  while (h.nrhs % (nr * rl)) --nr;
  h.nr_tile = nr;
  h.rhs_lanes = rl;
  h.order = t.block_order;
  h.nt_out = (t.flags & LQCD_TUNE_NT_STORE) ? 1 : 0;
  h.cached_gauge = (t.flags & LQCD_TUNE_CACHED_GAUGE) ? 1 : 0;
  h.occ_cap = (t.flags >> LQCD_TUNE_OCC_SHIFT) & 3;
  h.dir_split = (t.flags & LQCD_TUNE_DIR_SPLIT) ? 1 : 0;  // used where nr_tile = rhs_lanes = 1
}
inline void single_tile(HopLaunch& h) {
  h.nr_tile = 1;
  h.rhs_lanes = 1;
}

}  // namespace lqcd
