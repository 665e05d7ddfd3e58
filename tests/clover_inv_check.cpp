// Host-side check of the 6x6 clover-block inverse (csrc/clover_inv.h): the
// LDL^H route on well-conditioned Hermitian blocks, the pivoted fallback on
// nonsingular indefinite blocks whose leading pivots vanish, and the report
// of singular blocks.  Built by tests/test_clover_inverse_cpu.py (plain and
// with the host sanitizers); prints one line per case and exits non-zero on
// the first failure.
#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include "clover_inv.h"

struct Z {
  double re, im;
};
using Blk = Z[6][6];
using namespace lqcd::blk6;

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double urand() {  // splitmix64 -> [-1, 1)
  uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static void random_hermitian(Blk& A, double diag, double off) {
  for (int i = 0; i < 6; ++i) {
    A[i][i] = Z{diag + off * urand(), 0.0};
    for (int j = 0; j < i; ++j) {
      A[i][j] = Z{off * urand(), off * urand()};
      A[j][i] = Z{A[i][j].re, -A[i][j].im};
    }
  }
}

// max |A R - 1| and max |R - R^+|
static void residuals(const Blk& A, const Blk& R, double& e_inv, double& e_herm) {
  e_inv = e_herm = 0.0;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      double re = (i == j) ? -1.0 : 0.0, im = 0.0;
      for (int k = 0; k < 6; ++k) {
        re += A[i][k].re * R[k][j].re - A[i][k].im * R[k][j].im;
        im += A[i][k].re * R[k][j].im + A[i][k].im * R[k][j].re;
      }
      e_inv = fmax(e_inv, hypot(re, im));
      e_herm = fmax(e_herm, hypot(R[i][j].re - R[j][i].re, R[i][j].im + R[j][i].im));
    }
}

static int failures = 0;
static void expect(bool ok, const char* what, int n, double a, double b) {
  printf("%s %s: cases=%d max|AR-1|=%.3e max|R-R^+|=%.3e\n", ok ? "ok" : "FAIL", what, n, a, b);
  if (!ok) ++failures;
}

int main() {
  Blk A, R;
  double ei, eh, wi = 0, wh = 0;
  bool ok = true;
  // 1: clover-like blocks d 1 + (small Hermitian): LDL^H, accurate
  for (int n = 0; n < 2000; ++n) {
    random_hermitian(A, 4.0 + 1.0 / (2 * 0.135) - 4.0 + 3.7, 0.6);
    ok = ok && herm_inverse(A, R) == INV_LDL;
    residuals(A, R, ei, eh);
    wi = fmax(wi, ei);
    wh = fmax(wh, eh);
  }
  expect(ok && wi < 1e-13 && wh == 0.0, "well-conditioned blocks take LDL^H", 2000, wi, wh);
  // 2: indefinite, nonsingular, zero leading pivot: LDL^H fails, the
  // pivoted route inverts it and the result is exactly Hermitian
  ok = true;
  wi = wh = 0;
  for (int n = 0; n < 2000; ++n) {
    random_hermitian(A, 0.0, 1.0);
    A[0][0] = Z{0.0, 0.0};
    if (n % 2) {  // also a vanishing second pivot: A[1][1] = |A10|^2 / 0 path avoided by a zero 2x2 leading block
      A[1][1] = Z{0.0, 0.0};
    }
    Blk Rl;
    const bool ldl_ok = inverse_ldl(A, Rl);
    const int r = herm_inverse(A, R);
    residuals(A, R, ei, eh);
    // cond of these random blocks is modest; skip the rare near-singular draw
    if (ei > 1e-8) continue;
    ok = ok && !ldl_ok && r == INV_PIVOTED;
    wi = fmax(wi, ei);
    wh = fmax(wh, eh);
  }
  expect(ok && wi < 1e-11 && wh == 0.0, "indefinite blocks with a zero pivot take the pivoted route", 2000, wi, wh);
  // 3: a permuted identity-like block [[0,1],[1,0]] + diag: exact inverse
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) A[i][j] = Z{0.0, 0.0};
  A[0][1] = A[1][0] = Z{1.0, 0.0};
  for (int i = 2; i < 6; ++i) A[i][i] = Z{(double)i, 0.0};
  residuals(A, R, ei, eh);  // (R is overwritten below)
  const int r3 = herm_inverse(A, R);
  residuals(A, R, ei, eh);
  expect(r3 == INV_PIVOTED && ei < 1e-15, "swap block", 1, ei, eh);
  // 4: singular blocks: rank 5 (a null vector), zero, and a duplicated row
  int sing = 0, nsing = 0;
  for (int n = 0; n < 500; ++n) {
    Z v[5][6];
    for (int k = 0; k < 5; ++k)
      for (int i = 0; i < 6; ++i) v[k][i] = Z{urand(), urand()};
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        double re = 0, im = 0;
        for (int k = 0; k < 5; ++k) {  // sum_k s_k v_k v_k^+, indefinite signs
          const double s = (k % 2) ? -1.0 : 1.0;
          re += s * (v[k][i].re * v[k][j].re + v[k][i].im * v[k][j].im);
          im += s * (v[k][i].im * v[k][j].re - v[k][i].re * v[k][j].im);
        }
        A[i][j] = Z{re, im};
      }
    for (int i = 0; i < 6; ++i) A[i][i].im = 0.0;
    ++nsing;
    if (herm_inverse(A, R) == INV_SINGULAR) ++sing;
  }
  expect(sing == nsing, "rank-5 blocks are reported singular", nsing, 0.0, 0.0);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) A[i][j] = Z{0.0, 0.0};
  expect(herm_inverse(A, R) == INV_SINGULAR, "zero block is reported singular", 1, 0.0, 0.0);
  return failures ? 1 : 0;
}
