/*
 * lqcd_oracle.c -- plain, slow, FP64 CPU reference for the O(a)-improved
 * (Sheikholeslami-Wohlert) Wilson-Dirac operator Dw and for the conjugate
 * gradient solve of Dw psi = eta through its normal equations.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library, and the GPU library never
 * calls it.
 *
 * What the paper fixes (Sec. 3.3, "Fermionic observables"): the operator is
 * the Wilson operator with the Sheikholeslami-Wohlert clover term, with
 * parameters (m0, csw, theta, mu, cF); theta holds full boundary phase
 * factors |theta_i| = 1 applied at the boundaries; cF (c~_t) is the boundary
 * improvement coefficient for Dirichlet (SF) and open boundaries; the clover
 * term is precomputed from the gauge field and added on every application;
 * Dw, g5Dw and DwdagDw are provided and CG solves for propagators.
 * Sec. 2.1 fixes the time direction as the last lattice extent and the
 * boundary types (periodic, SF, open).  The paper prints no formula, so the
 * operator below is the textbook SW operator in openQCD's conventions (the
 * code Sec. 1 says the package was checked against):
 *
 *   (Dw psi)(x) = A(x) psi(x)
 *       - 1/2 sum_mu [ ph+ (1 - g_mu) U_mu(x) psi(x+mu)
 *                    + ph- (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *   A(x) = (4 + m0 + d_bnd(x)(cF - 1)) 1 + csw (i/4) sum_{mu!=nu} s_{mu nu} F_{mu nu}(x)
 *   s_{mu nu} = (i/2)[g_mu, g_nu],   F = (1/8)(Q - Q^+) made traceless,
 *   Q = sum of the four plaquette leaves in the (mu,nu) plane around x.
 *
 * Twisted mass: D(mu) = Dw + i mu g5 on every site, i.e. the site matrix
 * A(x) + i mu g5 (the caller adds i mu g5 to A, see oracle.py); the adjoint
 * uses g5 A^+ g5 for the site term (g5_adjoint_sites), so D(mu)^+ =
 * g5 D(-mu) g5.
 *
 * Chiral Euclidean gamma basis: g_t = [[0,-1],[-1,0]],
 * g_k = [[0,-i s_k],[i s_k,0]], g5 = g_t g_x g_y g_z = diag(1,1,-1,-1).
 *
 * Boundaries (phases act on fermion hops only, never inside the leaves):
 *   PERIODIC: a hop that crosses x_mu = L_mu-1 -> 0 is multiplied by theta_mu
 *             (forward) or conj(theta_mu) (backward).
 *   OPEN:     the links U_t(t = T-1) are zero everywhere (hops and leaves);
 *             time hops across the boundary are cut; d_bnd = 1 on t = 0, T-1.
 *   SF:       slice t = 0 is the Dirichlet boundary: the output there is 0
 *             and the input there is ignored; d_bnd = 1 on t = 1, T-1.
 * Spatial theta applies for every boundary type.
 *
 * Canonical layouts (complex128, C order):
 *   U  [t][z][y][x][mu][a][b]   mu = 0,1,2,3 = x,y,z,t
 *   psi[t][z][y][x][alpha][a]   alpha = spin (chiral basis), a = colour
 *   A  [t][z][y][x][12][12]     row/column index 3*alpha + a
 *   F  [t][z][y][x][6][3][3]    planes (x,y),(x,z),(x,t),(y,z),(y,t),(z,t)
 *
 * Vector sums (norms, dot products) run sequentially in site order.  Only
 * the site loops of the operator are split over OpenMP threads; each output
 * site is computed by one thread, so results do not depend on the thread
 * count.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cd;

enum { BC_PERIODIC = 0, BC_SF = 1, BC_OPEN = 2 };

typedef struct {
  int L[4];
  long V;
  int bc;
  cd theta[4];
} lat_t;

static lat_t make_lat(const int *L, int bc, const double *theta_re,
                      const double *theta_im) {
  lat_t g;
  g.V = 1;
  for (int mu = 0; mu < 4; ++mu) {
    g.L[mu] = L[mu];
    g.V *= L[mu];
    g.theta[mu] = theta_re ? theta_re[mu] + I * theta_im[mu] : 1.0;
  }
  g.bc = bc;
  return g;
}

static long site_index(const lat_t *g, const int x[4]) {
  return x[0] + (long)g->L[0] * (x[1] + (long)g->L[1] * (x[2] + (long)g->L[2] * x[3]));
}

static void site_coords(const lat_t *g, long i, int x[4]) {
  for (int mu = 0; mu < 4; ++mu) {
    x[mu] = (int)(i % g->L[mu]);
    i /= g->L[mu];
  }
}

/* y = x + step * mu_hat, periodic wrap of the stored lattice */
static void shift(const lat_t *g, const int x[4], int mu, int step, int y[4]) {
  for (int nu = 0; nu < 4; ++nu) y[nu] = x[nu];
  y[mu] = ((x[mu] + step) % g->L[mu] + g->L[mu]) % g->L[mu];
}

/* ---------------------------------------------------------------------- */
/* Small dense linear algebra                                              */
/* ---------------------------------------------------------------------- */

static void m3_mul(cd r[3][3], cd a[3][3], cd b[3][3]) {
  cd t[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      t[i][j] = 0;
      for (int k = 0; k < 3; ++k) t[i][j] += a[i][k] * b[k][j];
    }
  memcpy(r, t, sizeof(t));
}

static void m3_dag(cd r[3][3], cd a[3][3]) {
  cd t[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) t[i][j] = conj(a[j][i]);
  memcpy(r, t, sizeof(t));
}

/* U_mu(x) with the OPEN-boundary rule: U_t(t = T-1) is zero */
static void link(const lat_t *g, const cd *U, const int x[4], int mu, cd M[3][3]) {
  if (g->bc == BC_OPEN && mu == 3 && x[3] == g->L[3] - 1) {
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) M[a][b] = 0;
    return;
  }
  const cd *p = U + (site_index(g, x) * 4 + mu) * 9;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) M[a][b] = p[3 * a + b];
}

/* Gamma matrices in the chiral basis; mu = 0..3 (x,y,z,t), mu = 4 gives g5 */
static void gamma_mat(int mu, cd g[4][4]) {
  memset(g, 0, 16 * sizeof(cd));
  if (mu == 3) { /* g_t = [[0,-1],[-1,0]] */
    g[0][2] = -1; g[1][3] = -1; g[2][0] = -1; g[3][1] = -1;
    return;
  }
  if (mu == 4) { /* g5 = g_t g_x g_y g_z */
    cd a[4][4], b[4][4], t[4][4];
    gamma_mat(3, a);
    for (int nu = 0; nu < 3; ++nu) {
      gamma_mat(nu, b);
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          t[i][j] = 0;
          for (int k = 0; k < 4; ++k) t[i][j] += a[i][k] * b[k][j];
        }
      memcpy(a, t, sizeof(t));
    }
    memcpy(g, a, sizeof(a));
    return;
  }
  /* Pauli matrix sigma_{mu+1} */
  cd s[2][2];
  if (mu == 0) { s[0][0] = 0; s[0][1] = 1; s[1][0] = 1; s[1][1] = 0; }
  else if (mu == 1) { s[0][0] = 0; s[0][1] = -I; s[1][0] = I; s[1][1] = 0; }
  else { s[0][0] = 1; s[0][1] = 0; s[1][0] = 0; s[1][1] = -1; }
  /* g_k = [[0, -i s_k], [i s_k, 0]] */
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      g[i][2 + j] = -I * s[i][j];
      g[2 + i][j] = I * s[i][j];
    }
}

static void sigma_mat(int mu, int nu, cd s[4][4]) {
  cd a[4][4], b[4][4];
  gamma_mat(mu, a);
  gamma_mat(nu, b);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cd c = 0;
      for (int k = 0; k < 4; ++k) c += a[i][k] * b[k][j] - b[i][k] * a[k][j];
      s[i][j] = 0.5 * I * c;
    }
}

/* ---------------------------------------------------------------------- */
/* Clover field strength and the diagonal term A(x)                        */
/* ---------------------------------------------------------------------- */

static const int PLANE_MU[6] = {0, 0, 0, 1, 1, 2};
static const int PLANE_NU[6] = {1, 2, 3, 2, 3, 3};

/* F_{mu nu}(x) = traceless part of (Q - Q^+)/8, Q = sum of the four leaves
 * of the (mu,nu) plane that touch x, each read counter-clockwise from x. */
static void field_strength_site(const lat_t *g, const cd *U, const int x[4],
                                int mu, int nu, cd F[3][3]) {
  int xpm[4], xpn[4], xmm[4], xmn[4], xmmpn[4], xmmmn[4], xpmmn[4];
  shift(g, x, mu, +1, xpm);
  shift(g, x, nu, +1, xpn);
  shift(g, x, mu, -1, xmm);
  shift(g, x, nu, -1, xmn);
  shift(g, xmm, nu, +1, xmmpn);
  shift(g, xmm, nu, -1, xmmmn);
  shift(g, xpm, nu, -1, xpmmn);
  cd a[3][3], b[3][3], c[3][3], d[3][3], t[3][3], Q[3][3];
  memset(Q, 0, sizeof(Q));

  /* leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ */
  link(g, U, x, mu, a); link(g, U, xpm, nu, b);
  link(g, U, xpn, mu, c); m3_dag(c, c);
  link(g, U, x, nu, d); m3_dag(d, d);
  m3_mul(t, a, b); m3_mul(t, t, c); m3_mul(t, t, d);
  for (int i = 0; i < 9; ++i) (&Q[0][0])[i] += (&t[0][0])[i];

  /* leaf 2: U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu) */
  link(g, U, x, nu, a);
  link(g, U, xmmpn, mu, b); m3_dag(b, b);
  link(g, U, xmm, nu, c); m3_dag(c, c);
  link(g, U, xmm, mu, d);
  m3_mul(t, a, b); m3_mul(t, t, c); m3_mul(t, t, d);
  for (int i = 0; i < 9; ++i) (&Q[0][0])[i] += (&t[0][0])[i];

  /* leaf 3: U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu) */
  link(g, U, xmm, mu, a); m3_dag(a, a);
  link(g, U, xmmmn, nu, b); m3_dag(b, b);
  link(g, U, xmmmn, mu, c);
  link(g, U, xmn, nu, d);
  m3_mul(t, a, b); m3_mul(t, t, c); m3_mul(t, t, d);
  for (int i = 0; i < 9; ++i) (&Q[0][0])[i] += (&t[0][0])[i];

  /* leaf 4: U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+ */
  link(g, U, xmn, nu, a); m3_dag(a, a);
  link(g, U, xmn, mu, b);
  link(g, U, xpmmn, nu, c);
  link(g, U, x, mu, d); m3_dag(d, d);
  m3_mul(t, a, b); m3_mul(t, t, c); m3_mul(t, t, d);
  for (int i = 0; i < 9; ++i) (&Q[0][0])[i] += (&t[0][0])[i];

  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) F[i][j] = (Q[i][j] - conj(Q[j][i])) / 8.0;
  cd tr = (F[0][0] + F[1][1] + F[2][2]) / 3.0;
  for (int i = 0; i < 3; ++i) F[i][i] -= tr;
}

void or_field_strength(const int *L, int bc, const cd *U, cd *F) {
  lat_t g = make_lat(L, bc, NULL, NULL);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < g.V; ++i) {
    int x[4];
    site_coords(&g, i, x);
    for (int p = 0; p < 6; ++p)
      field_strength_site(&g, U, x, PLANE_MU[p], PLANE_NU[p],
                          (cd(*)[3])(F + (i * 6 + p) * 9));
  }
}

static int bnd_slice(const lat_t *g, int t) {
  int T = g->L[3];
  if (g->bc == BC_SF) return t == 1 || t == T - 1;
  if (g->bc == BC_OPEN) return t == 0 || t == T - 1;
  return 0;
}

/* A(x) as a full 12x12 matrix (index 3*alpha + a) on every site */
void or_clover_matrix(const int *L, int bc, const cd *U, double m0, double csw,
                      double cF, cd *A) {
  lat_t g = make_lat(L, bc, NULL, NULL);
  cd sig[4][4][4][4];
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = 0; nu < 4; ++nu) sigma_mat(mu, nu, sig[mu][nu]);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < g.V; ++i) {
    int x[4];
    site_coords(&g, i, x);
    cd F[4][4][3][3];
    memset(F, 0, sizeof(F));
    for (int p = 0; p < 6; ++p) {
      int mu = PLANE_MU[p], nu = PLANE_NU[p];
      field_strength_site(&g, U, x, mu, nu, F[mu][nu]);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) F[nu][mu][a][b] = -F[mu][nu][a][b];
    }
    cd *Ai = A + i * 144;
    double diag = 4.0 + m0 + (bnd_slice(&g, x[3]) ? (cF - 1.0) : 0.0);
    for (int r = 0; r < 12; ++r)
      for (int c = 0; c < 12; ++c) {
        int al = r / 3, a = r % 3, be = c / 3, b = c % 3;
        cd v = (r == c) ? diag : 0.0;
        for (int mu = 0; mu < 4; ++mu)
          for (int nu = 0; nu < 4; ++nu) {
            if (mu == nu) continue;
            v += csw * 0.25 * I * sig[mu][nu][al][be] * F[mu][nu][a][b];
          }
        Ai[r * 12 + c] = v;
      }
  }
}

/* ---------------------------------------------------------------------- */
/* Hopping term and the full operator                                      */
/* ---------------------------------------------------------------------- */

/* phase multiplying the hop from x in direction mu (dir = +1 forward,
 * -1 backward); zero for a cut hop */
static cd hop_phase(const lat_t *g, const int x[4], int mu, int dir) {
  int at_edge = (dir > 0) ? (x[mu] == g->L[mu] - 1) : (x[mu] == 0);
  if (!at_edge) return 1.0;
  if (mu == 3 && g->bc != BC_PERIODIC) return 0.0;
  return dir > 0 ? g->theta[mu] : conj(g->theta[mu]);
}

static int inactive(const lat_t *g, const int x[4]) {
  return g->bc == BC_SF && x[3] == 0;
}

/* out(x) = -1/2 sum_mu [ ... ] (the off-diagonal part of Dw) for one site */
static void hop_site(const lat_t *g, const cd *U, const cd *psi, const int x[4],
                     cd out[12]) {
  cd gm[4][4][4];
  for (int mu = 0; mu < 4; ++mu) gamma_mat(mu, gm[mu]);
  for (int k = 0; k < 12; ++k) out[k] = 0;
  if (inactive(g, x)) return;
  for (int mu = 0; mu < 4; ++mu)
    for (int dir = +1; dir >= -1; dir -= 2) {
      int y[4];
      shift(g, x, mu, dir, y);
      cd ph = hop_phase(g, x, mu, dir);
      if (inactive(g, y)) ph = 0.0;
      if (ph == 0.0) continue;
      cd M[3][3];
      if (dir > 0) link(g, U, x, mu, M);
      else { link(g, U, y, mu, M); m3_dag(M, M); }
      const cd *py = psi + site_index(g, y) * 12;
      cd chi[4][3];
      for (int al = 0; al < 4; ++al)
        for (int a = 0; a < 3; ++a) {
          chi[al][a] = 0;
          for (int b = 0; b < 3; ++b) chi[al][a] += M[a][b] * py[3 * al + b];
        }
      /* (1 -/+ g_mu) chi */
      double sgn = (dir > 0) ? -1.0 : 1.0;
      for (int al = 0; al < 4; ++al)
        for (int a = 0; a < 3; ++a) {
          cd v = chi[al][a];
          for (int be = 0; be < 4; ++be) v += sgn * gm[mu][al][be] * chi[be][a];
          out[3 * al + a] += -0.5 * ph * v;
        }
    }
}

void or_hop(const int *L, int bc, const double *th_re, const double *th_im,
            const cd *U, const cd *psi, cd *out) {
  lat_t g = make_lat(L, bc, th_re, th_im);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < g.V; ++i) {
    int x[4];
    site_coords(&g, i, x);
    hop_site(&g, U, psi, x, out + i * 12);
  }
}

static void dw_apply(const lat_t *g, const cd *U, const cd *A, const cd *psi, cd *out) {
#pragma omp parallel for schedule(static)
  for (long i = 0; i < g->V; ++i) {
    int x[4];
    site_coords(g, i, x);
    cd h[12];
    hop_site(g, U, psi, x, h);
    cd *o = out + i * 12;
    if (inactive(g, x)) {
      for (int r = 0; r < 12; ++r) o[r] = 0;
      continue;
    }
    const cd *Ai = A + i * 144;
    const cd *pi = psi + i * 12;
    for (int r = 0; r < 12; ++r) {
      cd v = h[r];
      for (int c = 0; c < 12; ++c) v += Ai[r * 12 + c] * pi[c];
      o[r] = v;
    }
  }
}

/* g5 on every site: negate spins 2 and 3 */
static void g5_apply(const lat_t *g, const cd *in, cd *out) {
  cd g5[4][4];
  gamma_mat(4, g5);
  for (long i = 0; i < g->V; ++i)
    for (int al = 0; al < 4; ++al)
      for (int a = 0; a < 3; ++a) {
        cd v = 0;
        for (int be = 0; be < 4; ++be) v += g5[al][be] * in[i * 12 + 3 * be + a];
        out[i * 12 + 3 * al + a] = v;
      }
}

void or_dw(const int *L, int bc, const double *th_re, const double *th_im,
           const cd *U, const cd *A, const cd *psi, cd *out) {
  lat_t g = make_lat(L, bc, th_re, th_im);
  dw_apply(&g, U, A, psi, out);
}

/* Site matrices g5 A(x)^+ g5.  The hopping term H of Dw = A + H satisfies
 * H^+ = g5 H g5, so Dw^+ = g5 (g5 A^+ g5 + H) g5: the adjoint is Dw with
 * g5 A^+ g5 in place of A, between two g5.  For the clover term A is
 * Hermitian and commutes with g5, so g5 A^+ g5 = A; a twisted mass
 * i mu g5 in A turns into -i mu g5. */
static cd *g5_adjoint_sites(const lat_t *g, const cd *A) {
  cd *Ad = malloc((size_t)g->V * 144 * sizeof(cd));
#pragma omp parallel for schedule(static)
  for (long x = 0; x < g->V; ++x)
    for (int r = 0; r < 12; ++r)
      for (int c = 0; c < 12; ++c) {
        const double sg = ((r < 6) == (c < 6)) ? 1.0 : -1.0;  /* g5_r g5_c */
        Ad[x * 144 + r * 12 + c] = sg * conj(A[x * 144 + c * 12 + r]);
      }
  return Ad;
}

/* Dw^+ psi; Ad from g5_adjoint_sites */
static void dwdag_apply(const lat_t *g, const cd *U, const cd *Ad, const cd *psi,
                        cd *out, cd *tmp) {
  g5_apply(g, psi, tmp);
  dw_apply(g, U, Ad, tmp, out);
  g5_apply(g, out, tmp);
  memcpy(out, tmp, (size_t)g->V * 12 * sizeof(cd));
}

void or_dw_dag(const int *L, int bc, const double *th_re, const double *th_im,
               const cd *U, const cd *A, const cd *psi, cd *out) {
  lat_t g = make_lat(L, bc, th_re, th_im);
  cd *tmp = malloc((size_t)g.V * 12 * sizeof(cd));
  cd *Ad = g5_adjoint_sites(&g, A);
  dwdag_apply(&g, U, Ad, psi, out, tmp);
  free(Ad);
  free(tmp);
}

void or_gamma(int mu, cd *g) { gamma_mat(mu, (cd(*)[4])g); }

/* ---------------------------------------------------------------------- */
/* Conjugate gradient on Dw^+ Dw psi = Dw^+ eta                             */
/* ---------------------------------------------------------------------- */

static double norm2(long n, const cd *v) {
  double s = 0.0;
  for (long i = 0; i < n; ++i) s += creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
  return s;
}

/* True relative residual |eta - Dw psi| / |eta| */
static double true_residual(const lat_t *g, const cd *U, const cd *A, const cd *eta,
                            const cd *psi, cd *tmp) {
  long n = g->V * 12;
  dw_apply(g, U, A, psi, tmp);
  for (long i = 0; i < n; ++i) tmp[i] = eta[i] - tmp[i];
  return sqrt(norm2(n, tmp) / norm2(n, eta));
}

/*
 * Solve Dw psi = eta by CG on the normal equations, starting from psi = 0.
 * The inner loop stops when |r| <= target |b| (r the normal-equation
 * residual, b = Dw^+ eta), starting with target = tol/10.  The true residual
 * rho = |eta - Dw psi|/|eta| is then recomputed from scratch; if rho > tol the
 * recursion restarts from the true residual with the target ten times
 * smaller.  Returns 0 on success, 1 when maxiter was reached (psi then holds
 * the last iterate).  iters_out counts applications of Dw^+ Dw in the loop.
 */
int or_cg(const int *L, int bc, const double *th_re, const double *th_im,
          const cd *U, const cd *A, const cd *eta, cd *psi, double tol,
          int maxiter, double *rho_out, int *iters_out) {
  lat_t g = make_lat(L, bc, th_re, th_im);
  long n = g.V * 12;
  cd *r = malloc(n * sizeof(cd)), *p = malloc(n * sizeof(cd));
  cd *q = malloc(n * sizeof(cd)), *s = malloc(n * sizeof(cd));
  cd *tmp = malloc(n * sizeof(cd));
  cd *Ad = g5_adjoint_sites(&g, A);
  for (long i = 0; i < n; ++i) psi[i] = 0;

  dwdag_apply(&g, U, Ad, eta, r, tmp);       /* r = b = Dw^+ eta */
  double bnorm = sqrt(norm2(n, r));
  double target = tol / 10.0;
  int it = 0, status = 1;
  double rho = 1.0;
  if (bnorm == 0.0) {
    status = 0; rho = 0.0;
    goto done;
  }
  memcpy(p, r, n * sizeof(cd));
  double rr = norm2(n, r);
  while (it < maxiter) {
    dw_apply(&g, U, A, p, q);               /* q = Dw p */
    double pAp = norm2(n, q);               /* <p, Dw^+ Dw p> = |Dw p|^2 */
    double alpha = rr / pAp;
    dwdag_apply(&g, U, Ad, q, s, tmp);       /* s = Dw^+ Dw p */
    for (long i = 0; i < n; ++i) {
      psi[i] += alpha * p[i];
      r[i] -= alpha * s[i];
    }
    ++it;
    double rr_new = norm2(n, r);
    if (sqrt(rr_new) <= target * bnorm) {
      rho = true_residual(&g, U, A, eta, psi, tmp);
      if (rho <= tol) { status = 0; break; }
      /* restart from the true residual */
      dw_apply(&g, U, A, psi, q);
      for (long i = 0; i < n; ++i) q[i] = eta[i] - q[i];
      dwdag_apply(&g, U, Ad, q, r, tmp);
      target /= 10.0;
      memcpy(p, r, n * sizeof(cd));
      rr = norm2(n, r);
      continue;
    }
    double beta = rr_new / rr;
    for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
    rr = rr_new;
  }
  if (status != 0) rho = true_residual(&g, U, A, eta, psi, tmp);
done:
  if (rho_out) *rho_out = rho;
  if (iters_out) *iters_out = it;
  free(r); free(p); free(q); free(s); free(tmp); free(Ad);
  return status;
}

/* Run exactly niter CG iterations (no stopping test); used to time the
 * reference on a bounded sample.  Returns the normal-equation residual
 * |r|/|b| reached. */
double or_cg_fixed(const int *L, int bc, const double *th_re, const double *th_im,
                   const cd *U, const cd *A, const cd *eta, cd *psi, int niter) {
  lat_t g = make_lat(L, bc, th_re, th_im);
  long n = g.V * 12;
  cd *r = malloc(n * sizeof(cd)), *p = malloc(n * sizeof(cd));
  cd *q = malloc(n * sizeof(cd)), *s = malloc(n * sizeof(cd));
  cd *tmp = malloc(n * sizeof(cd));
  cd *Ad = g5_adjoint_sites(&g, A);
  for (long i = 0; i < n; ++i) psi[i] = 0;
  dwdag_apply(&g, U, Ad, eta, r, tmp);
  double bb = norm2(n, r);
  memcpy(p, r, n * sizeof(cd));
  double rr = bb;
  for (int it = 0; it < niter && rr > 0.0; ++it) {
    dw_apply(&g, U, A, p, q);
    double alpha = rr / norm2(n, q);
    dwdag_apply(&g, U, Ad, q, s, tmp);
    for (long i = 0; i < n; ++i) {
      psi[i] += alpha * p[i];
      r[i] -= alpha * s[i];
    }
    double rr_new = norm2(n, r);
    double beta = rr_new / rr;
    for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
    rr = rr_new;
  }
  free(r); free(p); free(q); free(s); free(tmp); free(Ad);
  return bb > 0.0 ? sqrt(rr / bb) : 0.0;
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
