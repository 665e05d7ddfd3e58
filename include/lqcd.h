/*
 * lqcd.h -- C ABI of the MI355X (gfx950) Wilson-clover library.
 *
 * The library applies the O(a)-improved Wilson-Dirac operator Dw (paper
 * Sec. 3.3: Dw!, g5Dw!, DwdagDw!, with the clover term precomputed by Csw!)
 * and solves Dw psi = eta for fermion propagators by conjugate gradient on
 * the normal equations (paper Sec. 3.3: CG!, propagator!).  Lattice
 * geometry and boundary conditions follow paper Sec. 2.1 (time is the last
 * extent; periodic, Schroedinger-functional and open boundaries); the Dirac
 * parameters follow the DiracParam structure of Sec. 3.3 (bare mass via
 * kappa, csw, theta boundary phase factors with |theta| = 1, twisted mass
 * mu, boundary coefficient cF).
 *
 * Operator (chiral Euclidean gamma basis, g5 = diag(1,1,-1,-1)):
 *   (Dw psi)(x) = A(x) psi(x) - 1/2 sum_mu [ ph+ (1-g_mu) U_mu(x) psi(x+mu)
 *                                        + ph- (1+g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *   A(x) = (4 + m0 + d_bnd(x)(cF-1)) + csw (i/4) sum_{mu!=nu} s_{mu nu} F_{mu nu}(x),
 *   m0 = 1/(2 kappa) - 4, F the traceless clover-leaf field strength.
 * With a twisted mass mu the operator is D(mu) = Dw + i mu g5 on every site
 * (its adjoint is g5 D(-mu) g5); every call below that takes lqcd_dirac
 * applies or inverts D(mu) (Dw for mu = 0).
 * Boundary handling: PERIODIC multiplies hops crossing the edge of direction
 * mu by theta_mu (conj(theta_mu) backwards); SF makes slice t = 0 a
 * Dirichlet slice (output 0 there, input there ignored, d_bnd = 1 on
 * t = 1, T-1); OPEN cuts the time hops across the boundary and treats the
 * links U_t(t = T-1) as zero (d_bnd = 1 on t = 0, T-1).
 *
 * Canonical data layout at this boundary (device memory, complex128 =
 * interleaved pairs of doubles, C order, x fastest):
 *   gauge  U  [t][z][y][x][mu][a][b]     mu = 0..3 = x,y,z,t
 *   spinor psi[rhs][t][z][y][x][alpha][a] alpha = spin (chiral basis), a = colour
 * The internal layout (site-coalesced, even-odd split, per precision) is
 * opaque; LQCD_LAYOUT_INTERNAL exists so that benchmarks can time the
 * kernels without layout conversion.
 *
 * Ownership: the caller owns every buffer.  The library allocates no device
 * memory in any entry point: gauge storage and workspaces live in caller
 * memory whose size the *_bytes() queries return, and the library keeps
 * pointers into it until the corresponding *_free()/destroy().  Host-side
 * handles are allocated with malloc and released by *_free().
 *
 * Streams: `stream` arguments are hipStream_t values passed as void*; NULL
 * is the default stream.  Device work is enqueued on that stream; calls
 * return once their device work is enqueued, except lqcd_solve, which
 * synchronises the stream (it reads convergence flags) before returning.
 *
 * Errors: every entry point returns an LQCD_* status.  Arguments are
 * validated before any device work; on a validation error nothing is
 * modified.  lqcd_last_error() returns a thread-local message describing the
 * last failure on the calling thread.  No C++ exception crosses this ABI.
 */
#ifndef LQCD_H
#define LQCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
enum {
  LQCD_OK = 0,
  LQCD_PENDING = 1,      /* lqcd_poll: request not finished yet */
  LQCD_EINVAL = -1,      /* invalid argument (see lqcd_last_error) */
  LQCD_ENOMEM = -2,      /* caller-provided memory too small */
  LQCD_EDEVICE = -3,     /* HIP runtime error */
  LQCD_ENOCONV = -4,     /* solver did not reach tol within maxiter */
  LQCD_ENUMERIC = -5,    /* NaN/Inf in an input or a singular clover block */
  LQCD_ENOTFOUND = -6,   /* unknown ticket or gauge id */
  LQCD_EBUSY = -7,       /* request queue full */
  LQCD_EUNSUPPORTED = -8 /* valid request this build does not implement */
};

const char *lqcd_strerror(int status);
/* Message of the last failing call on this thread ("" if none). */
const char *lqcd_last_error(void);

/* ---- geometry (paper Sec. 2.1, SpaceParm) ------------------------------ */
enum { LQCD_BC_PERIODIC = 0, LQCD_BC_SF = 1, LQCD_BC_OPEN = 2 };

typedef struct lqcd_geom_desc {
  int32_t L[4];         /* extents x, y, z, t; each even and >= 2 */
  int32_t bc;           /* LQCD_BC_* */
  double theta_re[4];   /* boundary phase factors, |theta_mu| = 1 (Sec. 3.3); */
  double theta_im[4];   /*   theta_t is used only with LQCD_BC_PERIODIC       */
} lqcd_geom_desc;

typedef struct lqcd_geom lqcd_geom_t;

/* Validates desc (EINVAL: extent odd or < 2, bc unknown, |theta| != 1
 * beyond 1e-12, SF/OPEN with T < 4) and creates a host-side handle. */
int lqcd_geom(const lqcd_geom_desc *desc, lqcd_geom_t **out);
void lqcd_geom_free(lqcd_geom_t *g);
/* Lattice volume V (number of sites). */
int64_t lqcd_geom_volume(const lqcd_geom_t *g);

/* ---- precisions --------------------------------------------------------- */
enum { LQCD_F64 = 0, LQCD_F32 = 1, LQCD_BF16 = 2 };
/* Bit masks naming the precisions a gauge field or workspace must hold.
 * LQCD_PM_TWO_ROW (gauge fields only) stores every link, in every precision,
 * as its first two rows: the paper's SU(3) type (Sec. 2.2) keeps two rows
 * and recovers the third from unitarity and unit determinant, row 2 =
 * complex conjugate of (row 0 x row 1).  This moves 12 instead of 18 reals
 * per link and is exact (to rounding) for SU(3) links only. */
enum { LQCD_PM_F64 = 1, LQCD_PM_F32 = 2, LQCD_PM_BF16 = 4, LQCD_PM_TWO_ROW = 8 };

/* ---- gauge field (paper Sec. 2.2: device-resident vector_field) -------- */
typedef struct lqcd_gauge lqcd_gauge_t;

/* Device bytes that lqcd_gauge_create needs for the precisions in pmask
 * (FP64 is always stored). */
size_t lqcd_gauge_bytes(const lqcd_geom_t *g, int pmask);

/* Imports the canonical FP64 field U_dev (device memory, read only during
 * the call's device work) into `mem` (device, >= lqcd_gauge_bytes) in the
 * internal layout, in FP64 and in the other precisions of pmask (FP32 and
 * BF16 by round-to-nearest-even).  U is used as given, except that with
 * LQCD_BC_OPEN the stored U_t(t = T-1) is set to zero.  With LQCD_PM_TWO_ROW
 * the call also checks, on the device, that every link's third row equals
 * the one rebuilt from its first two within 1e-10 (absolute, per complex
 * element); it then waits for the stream and returns LQCD_EINVAL, with no
 * handle, for a field that is not SU(3).  The handle refers to g and mem:
 * both must outlive it. */
int lqcd_gauge_create(const lqcd_geom_t *g, const void *U_dev, int pmask, void *mem,
                      size_t mem_bytes, void *stream, lqcd_gauge_t **out);
void lqcd_gauge_free(lqcd_gauge_t *u);

/* ---- workspace (paper Sec. 2.2, DiracWorkspace) ------------------------ */
typedef struct lqcd_ws lqcd_ws_t;

/* Device bytes of a workspace for solves/applications with up to nrhs
 * right-hand sides in the precisions of pmask. */
size_t lqcd_ws_bytes(const lqcd_geom_t *g, int pmask, int nrhs);
int lqcd_ws_create(const lqcd_geom_t *g, int pmask, int nrhs, void *mem, size_t mem_bytes,
                   lqcd_ws_t **out);
void lqcd_ws_free(lqcd_ws_t *w);

/* ---- Dirac parameters (paper Sec. 3.3, DiracParam) --------------------- */
typedef struct lqcd_dirac {
  double kappa;  /* hopping parameter > 0; m0 = 1/(2 kappa) - 4 */
  double csw;    /* Sheikholeslami-Wohlert coefficient */
  double cF;     /* boundary coefficient (c~_t) for SF/OPEN; 1 = tree level */
  double mu;     /* twisted mass: D(mu) = Dw + i mu g5 (0: plain Dw) */
} lqcd_dirac;

/* Csw! analogue (paper Sec. 3.3): computes the clover term of (u, d) into
 * the workspace, in FP64 and in the other precisions the workspace holds:
 * A(x) on every site and A(x)^{-1} on the odd sites (FP64 6x6 LDL^H per
 * chirality block); with mu != 0 the odd sites hold (A + i mu g5)^{-1} per
 * chirality, (A^2 + mu^2)^{-1}(A -+ i mu), as general 6x6 blocks.  ENUMERIC
 * if a block is numerically singular.  Later
 * calls with the same (u, d) reuse it; lqcd_dw_apply and lqcd_solve call
 * this themselves when needed. */
int lqcd_clover(const lqcd_gauge_t *u, const lqcd_dirac *d, lqcd_ws_t *w, void *stream);

/* ---- operator application (paper Sec. 3.3: Dw!, g5Dw!, DwdagDw!) ------- */
enum {
  LQCD_OP_DW = 0,          /* full-lattice Dw */
  LQCD_OP_DW_DAG = 1,      /* D^+ = g5 D(-mu) g5 */
  LQCD_OP_G5DW = 2,        /* g5 Dw */
  LQCD_OP_DWDAGDW = 3,     /* D^+ D */
  LQCD_OP_SCHUR = 4,       /* Dhat = A_ee - D_eo A_oo^{-1} D_oe on even sites */
  LQCD_OP_SCHUR_DAG = 5,   /* Dhat^+ = g5 Dhat(-mu) g5 */
  LQCD_OP_SCHUR_NORMAL = 6,/* Dhat^+ Dhat */
  LQCD_OP_HOP_EO = 7,      /* A_oo^{-1} D_oe: even input -> odd output */
  LQCD_OP_HOP_OE = 8       /* A_ee x_e - D_eo y_o: see lqcd_dw_apply */
};
enum { LQCD_LAYOUT_CANON = 0, LQCD_LAYOUT_INTERNAL = 1 };

/* Applies `op` to nrhs spinor fields.  With LQCD_LAYOUT_CANON `in` and `out`
 * are canonical complex128 full-lattice fields (nrhs stacked); the Schur
 * operators read the even sites of `in` and write the even sites of `out`
 * (odd sites set to 0); HOP_EO reads the even sites and writes the odd sites
 * (even sites set to 0); HOP_OE reads x_e from the even and y_o from the odd
 * sites of `in` and writes even sites.  With LQCD_LAYOUT_INTERNAL `in` and
 * `out` are internal-layout vectors of precision `prec` (size from
 * lqcd_vec_bytes).  `in` and `out` must not overlap.  The clover term is
 * (re)built in `w` when (u, d) differs from the cached one. */
/* With LQCD_LAYOUT_INTERNAL each operator is exactly its kernel launches
 * (HOP_EO and HOP_OE are one launch each, SCHUR two): the parity an operator
 * does not produce is left unchanged in `out`. */
int lqcd_dw_apply(const lqcd_gauge_t *u, const lqcd_dirac *d, int op, int prec, int layout,
                  int nrhs, const void *in, void *out, lqcd_ws_t *w, void *stream);

/* Bytes of one internal-layout vector: nrhs fields on `nparity` (1 or 2)
 * parities in precision prec. */
size_t lqcd_vec_bytes(const lqcd_geom_t *g, int prec, int nrhs, int nparity);

/* ---- meson two-point functions (paper Sec. 3.3: correlation functions
 * contracted from the propagator) --------------------------------------- */
/* From a 12-column point-source propagator psi (device, canonical
 * complex128, 12 fields of V x 12, column j = 3 s + c for source spin s and
 * colour c, e.g. the solution of the 12 point sources of lqcd_solve), with
 * S(x)[al a][be c] = psi_(3 be + c)(x)[al][a]:
 *   G (device complex128 [T][4][4][4][4], may be NULL):
 *     G[t][al][be][al'][be'] = sum_{x in slice t} sum_{a,c} S(x)[al a][be c] conj(S(x)[al' a][be' c]);
 *   C (device complex128 [npairs][T]): for each pair (m, m') of `pairs`
 *     (host, npairs x 2 masks 0..15),
 *     C[p][t] = sum_{x in slice t} tr[Gamma_m S(x) Gamma_m' g5 S(x)^+ g5],
 *     the meson correlator with the backward propagator g5 S^+ g5 (no
 *     fermion-loop sign), Gamma_m = g_t^{m3} g_x^{m0} g_y^{m1} g_z^{m2} in
 *     the chiral basis (m = 0: identity, 15: g5, 8: g_t, 1/2/4: g_x/y/z).
 * npairs 0..32 (C and pairs unused for 0); at least one of C and G.  The
 * workspace w (same geometry, any precisions, any nrhs) provides scratch;
 * its vectors are overwritten.  FP64, deterministic (fixed-order sums).
 * EINVAL for bad arguments, without device work. */
int lqcd_meson(const lqcd_geom_t *g, const void *psi, int npairs, const int32_t *pairs, void *C, void *G,
               lqcd_ws_t *w, void *stream);

/* ---- entry points that allocate nothing -------------------------------- */
/* For callers that cannot allocate device memory or pass a workspace (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation).  Their scratch memory is one fixed device array of the
 * library per GPU, LQCD_NOALLOC_SCRATCH_BYTES long, that each GPU the library
 * runs on holds until the process ends.  Every call on a GPU shares that
 * GPU's array: calls that overlap in time on one GPU (two streams, two
 * threads) race and give wrong results; serialise them.  The array keeps the
 * last call's contents, which no call reads before writing. */
#define LQCD_NOALLOC_SCRATCH_BYTES (32u << 20)
size_t lqcd_noalloc_scratch_bytes(void);

/* lqcd_meson without a workspace: same arguments, results and errors, and
 * the same kernels, with the T x ceil(Lx Ly Lz / 256) x 256 complex128
 * partials in the fixed array instead of the workspace (32^3x64 needs all
 * 32 MiB).  EINVAL, without device work, for a lattice whose partials exceed
 * LQCD_NOALLOC_SCRATCH_BYTES.  Calls no allocating routine; the first call
 * on a device looks up the array's address there (EDEVICE if that fails). */
int lqcd_meson_noalloc(const lqcd_geom_t *g, const void *psi, int npairs, const int32_t *pairs, void *C,
                       void *G, void *stream);

/* ---- kernel tuning (autotuner) ------------------------------------------ */
typedef struct lqcd_tuning {
  int32_t nr_tile;     /* right-hand sides per thread in the hop kernels: 1..3
                          (a fourth needs more registers than a lane has) */
  int32_t block_order; /* workgroup -> sites: 0 plain; 1 every XCD walks a
                          contiguous range; 2 every XCD owns a z-slab and walks
                          it plane by plane in t (needs Lz % 8 == 0 and a
                          whole number of workgroups per (z, t) plane, else 1
                          is used); 3 and 4 as 1 and 2 with the rhs tiles one
                          after the other; 5 and 6 as 2 with slabs of 1 or 2
                          planes swept in several passes (6 needs
                          Lz % 16 == 0) */
  int32_t rhs_lanes;   /* lanes sharing one site, each with its own nr_tile
                          rhs: 1, 2 or 4 (FP64 uses 1) */
  int32_t flags;       /* LQCD_TUNE_NT_STORE: the hop kernels write their
                          output spinors with non-temporal stores;
                          LQCD_TUNE_CACHED_GAUGE: links and clover blocks
                          are read with ordinary (cached) loads instead of
                          non-temporal ones; bits 2-3 (level << 
                          LQCD_TUNE_OCC_SHIFT): at most 4, 3 or 2 resident
                          workgroups per CU for level 1, 2, 3 (0: no cap);
                          LQCD_TUNE_DIR_SPLIT: launches with one rhs per
                          thread (nr_tile 1, rhs_lanes 1) give each site two
                          waves, one for the x and y hops and one for the z
                          and t hops, each then producing one chirality of the
                          output: twice the parallelism for lattices too small
                          to fill the GPU */
} lqcd_tuning;
enum { LQCD_TUNE_NT_STORE = 1, LQCD_TUNE_CACHED_GAUGE = 2, LQCD_TUNE_OCC_SHIFT = 2,
       LQCD_TUNE_DIR_SPLIT = 16 };

/* Hop-kernel configuration used by a workspace for precision `prec`
 * (default: nr_tile 1, block_order 1, rhs_lanes 1).  A launch over n rhs uses
 * the largest rhs_lanes and nr_tile not above these whose product divides n.
 * EINVAL for values out of range.  None of these changes the arithmetic of
 * any rhs, except LQCD_TUNE_DIR_SPLIT: with it the eight hop terms of a site
 * are summed as (x, y terms) + (z, t terms) rather than in one chain, which
 * changes results in the last bits (results are bitwise reproducible for a
 * given split setting). */
int lqcd_ws_set_tuning(lqcd_ws_t *w, int prec, const lqcd_tuning *t);
int lqcd_ws_get_tuning(const lqcd_ws_t *w, int prec, lqcd_tuning *t);

/* Autotuner: times every candidate configuration (nr_tile x rhs_lanes
 * dividing nrhs, block_order, flags) of one Schur-operator application (both hop kernels)
 * in precision `prec` on nrhs fields of the workspace, with HIP events on
 * `stream`, at the workspace's real lattice shape; stores the fastest in the
 * workspace and in the process-wide tuning cache (below), and returns it with
 * its time in microseconds.  The
 * LQCD_TUNE_DIR_SPLIT bit is the caller's choice and is kept as set in the
 * workspace; with it set only nr_tile = rhs_lanes = 1 (the shape it applies
 * to) is searched, so autotuning never changes a result.  Overwrites the
 * workspace's vectors (not its clover term).  Requires nrhs <= the
 * workspace's nrhs and `prec` held by gauge field and workspace. */
int lqcd_autotune(const lqcd_gauge_t *u, const lqcd_dirac *d, int prec, int nrhs, lqcd_ws_t *w,
                  void *stream, lqcd_tuning *best, double *best_us);

/* ---- tuning cache --------------------------------------------------------
 * A process-wide table of autotuned configurations keyed by the device
 * architecture (e.g. gfx950), the lattice extents and boundary type, the
 * link storage (two rows or full), the precision, the rhs count, whether a
 * twisted mass is set (twisted != 0) and the direction-split choice.
 * lqcd_autotune adds its result; callers that must not tune while they run
 * (a serving loop) look entries up, and the table can be written to and read
 * from a text file so that later processes need not tune again.  No entry
 * changes a result (except through the split bit, which is part of the key).
 * Thread-safe. */
/* OK with *t set, or ENOTFOUND. */
int lqcd_tune_cache_find(const lqcd_gauge_t *u, int prec, int nrhs, int twisted, int dir_split,
                         lqcd_tuning *t);
/* Adds (or replaces) an entry; the split part of the key is t's
 * LQCD_TUNE_DIR_SPLIT bit.  EINVAL for values out of range. */
int lqcd_tune_cache_put(const lqcd_gauge_t *u, int prec, int nrhs, int twisted, const lqcd_tuning *t);
int lqcd_tune_cache_size(void);
void lqcd_tune_cache_clear(void);
/* One line per entry; load adds a file's entries (replacing equal keys) and
 * adds nothing if a line is malformed (EINVAL) or the file is missing
 * (ENOTFOUND). */
int lqcd_tune_cache_save(const char *path);
int lqcd_tune_cache_load(const char *path);

/* ---- solver (paper Sec. 3.3: CG!, propagator!) ------------------------- */
enum {
  LQCD_SOLVER_CG_FULL = 0, /* CG on Dw^+ Dw over the full lattice */
  LQCD_SOLVER_CG_EO = 1    /* CG on Dhat^+ Dhat (even-odd preconditioned) */
};

typedef struct lqcd_solve_params {
  lqcd_dirac d;
  int32_t solver;          /* LQCD_SOLVER_* */
  int32_t inner_prec;      /* LQCD_F64, LQCD_F32 or LQCD_BF16 (CG_EO only) */
  int32_t reliable_every;  /* mixed precision: an FP64 reliable update at least
                              every reliable_every iterations (0 selects 100),
                              besides one whenever |r| has dropped tenfold
                              since the last update */
  int32_t maxiter;         /* bound on CG iterations per right-hand side */
  double tol;              /* target true relative residual |eta-Dw psi|/|eta| */
  int32_t nrhs;            /* number of right-hand sides solved together */
  int32_t use_graph;       /* capture iteration chunks in a hipGraph */
  const void *x0;          /* initial guess (paper Sec. 3.3: CG! updates the
                              solution field it is given): NULL starts from
                              psi = 0; otherwise nrhs canonical complex128
                              fields on the device (may be the psi argument
                              itself: it is read before psi is written).  The
                              first residual is an FP64 recomputation
                              eta - Dw x0; a column whose x0 already meets tol
                              takes no iteration.  In lqcd_submit x0 is a host
                              buffer like eta. */
} lqcd_solve_params;

typedef struct lqcd_solve_info {
  int32_t status;           /* LQCD_OK or LQCD_ENOCONV for this rhs */
  int32_t iters;            /* CG iterations (applications of the normal op) */
  int32_t reliable_updates; /* FP64 residual recomputations */
  int32_t restarts;         /* tightenings of the inner target */
  int32_t fp64_from;        /* mixed precision: iteration after which this rhs
                               continued in FP64 because the low-precision
                               recursion stopped reducing the true residual
                               (0: never) */
  int32_t reserved;
  double true_residual;     /* |eta - Dw psi|/|eta| recomputed in FP64 with the
                               full-lattice operator after the solve */
  double seconds;           /* wall time of the whole call */
} lqcd_solve_info;

/* Mixed precision (inner_prec FP32 or BF16): when eight consecutive reliable
 * updates have not halved the best true residual of a rhs (the inner
 * precision cannot resolve the system: its condition number times the unit
 * roundoff is near one), that rhs continues as FP64 CG from its current
 * solution (info.fp64_from).  The result still meets tol. */
/* Solves Dw psi_j = eta_j for j < nrhs.  eta and psi are canonical
 * complex128 fields on the device (nrhs stacked).  With SF boundaries eta
 * must vanish on slice t = 0 (EINVAL otherwise).  Returns LQCD_OK if every
 * rhs reached tol, LQCD_ENOCONV otherwise (psi then holds the last
 * iterates and info[] the residuals reached).  info must hold nrhs
 * entries. */
int lqcd_solve(const lqcd_gauge_t *u, const lqcd_solve_params *p, const void *eta,
               void *psi, lqcd_ws_t *w, void *stream, lqcd_solve_info *info);

/* ---- Schroedinger functional: boundary-to-bulk propagator, f_P and f_A
 * (paper Sec. 3.3: boundary-to-bulk propagators for Dirichlet boundary
 * conditions and the correlators f_P, f_A) ------------------------------ */
/* Boundary source: eta (device, canonical complex128, 12 fields of V x 12)
 * is overwritten with the 12 columns (s, c) of P+ U_t(y0 = 0, y)^+ on the
 * slice y0 = 1 (zero elsewhere), P+ = (1 + g_t)/2:
 *   eta_{3s+c}(y)[al][a] = P+[al][s] conj(U_t(0, y)[c][a]).
 * EINVAL unless u has SF boundary conditions. */
int lqcd_sf_source(const lqcd_gauge_t *u, void *eta, void *stream);

/* f_P(x0) = 1/2 sum_x tr[H(x)^+ H(x)] and f_A(x0) = -1/2 sum_x tr[H(x)^+ g_t H(x)]
 * of the boundary-to-bulk propagator H = Dw^{-1} eta (eta from
 * lqcd_sf_source), for x0 = 0..T-1.  Runs lqcd_sf_source into `eta`, the
 * 12-rhs solve of `p` (p->nrhs is taken as 12; solver, precision and
 * tolerance as given) into `psi` (= H on return, canonical, 12 x V x 12),
 * then the meson contraction: fP and fA are device complex128 [T] (real
 * parts; imaginary parts zero to rounding).  w: workspace with nrhs >= 12.
 * info: 12 entries.  Returns the solve's status (fP, fA are written only on
 * LQCD_OK). */
int lqcd_sf_correlators(const lqcd_gauge_t *u, const lqcd_solve_params *p, void *eta, void *psi, void *fP,
                        void *fA, lqcd_ws_t *w, void *stream, lqcd_solve_info *info);


/* ---- serving: continuous batching of propagator solves ------------------ */
/* A server keeps gauge fields resident in a caller-provided device arena and
 * runs solve requests as they arrive.  `max_streams` worker threads, each with
 * its own HIP stream, take requests from a queue; a request is admitted when
 * a worker is free and its device footprint (workspace + source/solution
 * staging, lqcd_request_bytes) fits in the free part of the arena.  Requests
 * behind a head that does not fit may be admitted first (at most 8 times in a
 * row, so the head is not starved).  Kernels of different requests overlap on
 * the device.  Every request's result is the same as the same solve alone:
 * requests share only read-only gauge fields.  The paper runs independent
 * jobs side by side across GPUs (Sec. 1) and keeps fields and workspaces
 * resident on the device (Sec. 2.2); here the independent jobs are requests
 * sharing one GPU. */
typedef struct lqcd_server lqcd_server_t;

enum { LQCD_ECANCELED = -9 }; /* request cancelled by lqcd_server_destroy */

/* arena: device memory (>= 256-byte aligned) owned by the caller, used for
 * gauge fields and request workspaces; max_streams in [1, 16]; queue_cap >= 1
 * bounds the queued (not yet admitted) requests.  With arena == NULL the
 * server runs in simulation mode: no device work at all, each admitted
 * request holds its footprint for sim_seconds and completes with status OK
 * (for testing the scheduler without a GPU); sim_seconds is ignored
 * otherwise. */
int lqcd_server_create(void *arena, size_t arena_bytes, int max_streams, int queue_cap,
                       double sim_seconds, lqcd_server_t **out);
/* Registers a gauge field: U is canonical complex128 in host memory, copied
 * into the arena in FP64 and the precisions of pmask (on a stream of the
 * server's own, not a worker's).  Returns its id.  Gauge fields are
 * registered before requests are served: EBUSY while a request is queued or
 * running, so that the arena left to admitted and queued requests never
 * shrinks. */
int lqcd_server_add_gauge(lqcd_server_t *s, const lqcd_geom_desc *desc, const void *U_host,
                          int pmask, int *gauge_id);
/* Autotunes the hop kernels of gauge field gauge_id for requests of
 * precision inner_prec with nrhs right-hand sides (for a low-precision
 * inner_prec and nrhs > 1 also the FP64 kernels of their reliable updates),
 * on an otherwise idle GPU (a workspace borrowed from the arena, the server's
 * own stream; no request is admitted meanwhile), and stores the results in
 * the tuning cache.  Requests never tune: each takes the cached tunings of
 * its lattice, precisions and rhs count (mu != 0 and the split bit as keys;
 * the server never sets the split), else the default, and tunings never
 * change a result.  Does nothing if the entries exist.  EBUSY while a
 * request is queued or running; ENOMEM if the arena has no room for the
 * workspace. */
int lqcd_server_warmup(lqcd_server_t *s, int gauge_id, int inner_prec, int nrhs);
/* Device bytes one request with these parameters holds while it runs. */
size_t lqcd_request_bytes(lqcd_server_t *s, int gauge_id, const lqcd_solve_params *p);
/* Enqueues Dw psi = eta for gauge_id (thread-safe, non-blocking).  eta and
 * psi are canonical complex128 host buffers of p->nrhs fields that must stay
 * valid until lqcd_poll returns a final status.  EBUSY if the queue is full,
 * ENOMEM if the request can never fit in the arena, ENOTFOUND for an unknown
 * gauge id. */
int lqcd_submit(lqcd_server_t *s, int gauge_id, const lqcd_solve_params *p, const void *eta,
                void *psi, uint64_t *ticket);
/* PENDING while the request is queued or running; otherwise its final
 * status (as lqcd_solve, or ECANCELED), with info[nrhs] filled and, if times
 * is not NULL, times[0..2] = submit, admission and completion times in
 * seconds since the server was created.  A final status releases the ticket
 * (later polls return ENOTFOUND).  Thread-safe. */
int lqcd_poll(lqcd_server_t *s, uint64_t ticket, lqcd_solve_info *info, double *times);
/* Peak bytes of the arena in use since creation. */
size_t lqcd_server_peak_bytes(lqcd_server_t *s);
/* Stops the server: no further submissions; with cancel_pending, queued
 * requests end with ECANCELED, otherwise they are run first; running
 * requests always finish.  Returns once the workers have exited; tickets can
 * still be polled afterwards. */
int lqcd_server_stop(lqcd_server_t *s, int cancel_pending);
/* lqcd_server_stop (if not yet stopped), then frees the handle, its gauge
 * fields and any unpolled tickets. */
int lqcd_server_destroy(lqcd_server_t *s, int cancel_pending);

#ifdef __cplusplus
}
#endif
#endif /* LQCD_H */
