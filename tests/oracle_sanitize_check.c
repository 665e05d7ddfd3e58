/* Host-sanitizer run of the C oracle (built by tests/test_sanitizers_cpu.py
 * under AddressSanitizer + UndefinedBehaviorSanitizer): every exported
 * routine on small lattices of each boundary type, including a lattice with
 * unequal extents, so that an out-of-bounds index, a leak or undefined
 * arithmetic in the oracle's site and neighbour bookkeeping is reported.
 * The links are random U(1) phases times the identity (unitary, so CG on the
 * normal equations converges quickly); the check prints the true residual of
 * each solve and exits non-zero if one misses 1e-10. */
#include <stdio.h>

#include "../oracle/lqcd_oracle.c"

static unsigned long long st = 12345;
static double urand(void) {
  st = st * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(st >> 11) / 9007199254740992.0;
}

static int run(const int L[4], int bc) {
  const long V = (long)L[0] * L[1] * L[2] * L[3];
  const double th_re[4] = {1, 1, 0, bc == BC_PERIODIC ? -1 : 1}, th_im[4] = {0, 0, 1, 0};
  cd *U = calloc((size_t)V * 36, sizeof(cd)), *A = calloc((size_t)V * 144, sizeof(cd));
  cd *F = calloc((size_t)V * 54, sizeof(cd));
  cd *eta = calloc((size_t)V * 12, sizeof(cd)), *psi = calloc((size_t)V * 12, sizeof(cd));
  cd *out = calloc((size_t)V * 12, sizeof(cd));
  for (long i = 0; i < V * 4; ++i) {
    const double ph = 0.3 * (urand() - 0.5);
    for (int a = 0; a < 3; ++a) U[i * 9 + 4 * a] = cos(ph) + I * sin(ph);
  }
  if (bc == BC_OPEN) /* the cut links of the open boundary are zero */
    for (long i = V - V / L[3]; i < V; ++i)
      for (int e = 0; e < 9; ++e) U[(i * 4 + 3) * 9 + e] = 0;
  for (long i = 0; i < V * 12; ++i) eta[i] = urand() - 0.5 + I * (urand() - 0.5);
  if (bc == BC_SF)
    for (long i = 0; i < V / L[3] * 12; ++i) eta[i] = 0;
  or_field_strength(L, bc, U, F);
  or_clover_matrix(L, bc, U, 1.0 / (2 * 0.12) - 4.0, 1.5, 1.1, A);
  or_hop(L, bc, th_re, th_im, U, eta, out);
  or_dw(L, bc, th_re, th_im, U, A, eta, out);
  or_dw_dag(L, bc, th_re, th_im, U, A, eta, out);
  double rho = 1.0;
  int iters = 0;
  const int status = or_cg(L, bc, th_re, th_im, U, A, eta, psi, 1e-10, 2000, &rho, &iters);
  const double rn = or_cg_fixed(L, bc, th_re, th_im, U, A, eta, psi, 5);
  cd g[16];
  for (int mu = 0; mu < 4; ++mu) or_gamma(mu, g);
  printf("L=%dx%dx%dx%d bc=%d cg status=%d iters=%d rho=%.3e fixed5=%.3e threads=%d\n", L[0], L[1], L[2], L[3], bc,
         status, iters, rho, rn, or_num_threads());
  free(U); free(A); free(F); free(eta); free(psi); free(out);
  return status == 0 && rho <= 1e-10 && rn > 0.0;
}

int main(void) {
  const int L1[4] = {4, 4, 4, 6}, L2[4] = {6, 4, 2, 4};
  int ok = 1;
  for (int bc = 0; bc < 3; ++bc) {
    ok = run(L1, bc) && ok;
    ok = run(L2, bc) && ok;
  }
  printf("%s\n", ok ? "all ok" : "FAILED");
  return ok ? 0 : 1;
}
