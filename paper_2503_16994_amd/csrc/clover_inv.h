// Inverse of one 6x6 chirality block of the clover term (host and device).
//
// The blocks are Hermitian.  The primary route is an unpivoted LDL^H
// factorisation, exact in structure and cheap; it fails only on a pivot that
// is tiny against the block's scale, which a nonsingular but indefinite block
// can produce (rough gauge fields, large csw).  Such a block is inverted
// again by Gauss-Jordan elimination with partial (row) pivoting, valid for any
// nonsingular matrix, and the result is made exactly Hermitian by averaging
// it with its adjoint.  A block whose pivoted elimination also meets a pivot
// below kSingularRel of its infinity norm is reported as singular.
//
// Templates over a complex type with members re, im, so that the kernels use
// them on their own complex type and a host program can test them alone.
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define LQCD_HD __host__ __device__
#else
#define LQCD_HD
#endif

namespace lqcd {
namespace blk6 {

constexpr double kLdlPivotRel = 1e-12;   // LDL^H pivot floor, relative to max |A_ii|
constexpr double kSingularRel = 1e-13;   // pivoted elimination floor, relative to |A|_inf

enum { INV_LDL = 0, INV_PIVOTED = 1, INV_SINGULAR = -1 };

template <typename C>
LQCD_HD inline C zmul(C a, C b) {
  return C{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename C>
LQCD_HD inline C zmulc(C a, C b) {
  return C{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

// Inverse by LDL^H without pivoting; false if a pivot is below kLdlPivotRel of
// the largest diagonal entry (R is then not valid).
template <typename C>
LQCD_HD inline bool inverse_ldl(const C (&A)[6][6], C (&R)[6][6]) {
  C L[6][6];
  double D[6];
  double scale = 0.0;
#pragma unroll
  for (int i = 0; i < 6; ++i) scale = fmax(scale, fabs(A[i][i].re));
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double dj = A[j][j].re;
#pragma unroll
    for (int k = 0; k < j; ++k) dj -= (L[j][k].re * L[j][k].re + L[j][k].im * L[j][k].im) * D[k];
    if (!(fabs(dj) > kLdlPivotRel * scale)) ok = false;
    D[j] = dj;
    const double inv = 1.0 / dj;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      C v = A[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) {
        const C t = zmulc(L[j][k], L[i][k]);  // L_ik conj(L_jk)
        v = C{v.re - D[k] * t.re, v.im - D[k] * t.im};
      }
      L[i][j] = C{inv * v.re, inv * v.im};
    }
  }
  // X = L^{-1} (unit lower triangular)
  C X[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) X[i][j] = C{i == j ? 1.0 : 0.0, 0.0};
#pragma unroll
  for (int i = 1; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < i; ++j) {
      C v = C{0.0, 0.0};
#pragma unroll
      for (int k = j; k < i; ++k) {
        const C t = zmul(L[i][k], X[k][j]);
        v = C{v.re + t.re, v.im + t.im};
      }
      X[i][j] = C{-v.re, -v.im};
    }
  // A^{-1} = X^+ D^{-1} X
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      C v = C{0.0, 0.0};
#pragma unroll
      for (int k = i; k < 6; ++k) {
        const C t = zmulc(X[k][i], X[k][j]);
        const double s = 1.0 / D[k];
        v = C{v.re + s * t.re, v.im + s * t.im};
      }
      R[i][j] = v;
      R[j][i] = C{v.re, -v.im};
    }
  return ok;
}

// Inverse of a general complex 6x6 matrix by Gauss-Jordan elimination with
// partial pivoting (the largest |entry| of the column below the diagonal);
// false if a pivot is below kSingularRel |A|_inf.
template <typename C>
LQCD_HD inline bool inverse_pivoted(const C (&A)[6][6], C (&R)[6][6]) {
  C M[6][6];
  double norm = 0.0;
  for (int i = 0; i < 6; ++i) {
    double row = 0.0;
    for (int j = 0; j < 6; ++j) {
      M[i][j] = A[i][j];
      R[i][j] = C{i == j ? 1.0 : 0.0, 0.0};
      row += sqrt(A[i][j].re * A[i][j].re + A[i][j].im * A[i][j].im);
    }
    norm = fmax(norm, row);
  }
  if (!(norm > 0.0)) return false;
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    double best = -1.0;
    for (int r = c; r < 6; ++r) {
      const double a = M[r][c].re * M[r][c].re + M[r][c].im * M[r][c].im;
      if (a > best) {
        best = a;
        piv = r;
      }
    }
    if (!(sqrt(best) > kSingularRel * norm)) return false;
    if (piv != c) {
      for (int j = 0; j < 6; ++j) {
        const C tm = M[c][j];
        M[c][j] = M[piv][j];
        M[piv][j] = tm;
        const C tr = R[c][j];
        R[c][j] = R[piv][j];
        R[piv][j] = tr;
      }
    }
    // row c /= pivot
    const double d = M[c][c].re * M[c][c].re + M[c][c].im * M[c][c].im;
    const C ip = C{M[c][c].re / d, -M[c][c].im / d};
    for (int j = 0; j < 6; ++j) {
      M[c][j] = zmul(ip, M[c][j]);
      R[c][j] = zmul(ip, R[c][j]);
    }
    // eliminate column c from every other row
    for (int r = 0; r < 6; ++r) {
      if (r == c) continue;
      const C f = M[r][c];
      for (int j = 0; j < 6; ++j) {
        const C tm = zmul(f, M[c][j]), tr = zmul(f, R[c][j]);
        M[r][j] = C{M[r][j].re - tm.re, M[r][j].im - tm.im};
        R[r][j] = C{R[r][j].re - tr.re, R[r][j].im - tr.im};
      }
    }
  }
  return true;
}

template <typename C>
LQCD_HD inline double norm_inf(const C (&A)[6][6]) {
  double n = 0.0;
  for (int i = 0; i < 6; ++i) {
    double row = 0.0;
    for (int j = 0; j < 6; ++j) row += sqrt(A[i][j].re * A[i][j].re + A[i][j].im * A[i][j].im);
    n = fmax(n, row);
  }
  return n;
}

// Inverse of a Hermitian block: LDL^H, else pivoted elimination made
// Hermitian.  Either result is accepted only if |A|_inf |R|_inf, an estimate
// of the condition number, stays within 1 / kSingularRel: unpivoted LDL^H can
// pass its pivot test on a singular indefinite block through element growth,
// and then returns an inverse of enormous norm.  Returns INV_LDL, INV_PIVOTED
// or INV_SINGULAR (R not valid).
template <typename C>
LQCD_HD inline int herm_inverse(const C (&A)[6][6], C (&R)[6][6]) {
  const double na = norm_inf(A);
  if (inverse_ldl(A, R) && na * norm_inf(R) * kSingularRel <= 1.0) return INV_LDL;
  if (!inverse_pivoted(A, R) || !(na * norm_inf(R) * kSingularRel <= 1.0)) return INV_SINGULAR;
  for (int i = 0; i < 6; ++i) {
    R[i][i].im = 0.0;
    for (int j = 0; j < i; ++j) {
      const C h = C{0.5 * (R[i][j].re + R[j][i].re), 0.5 * (R[i][j].im - R[j][i].im)};
      R[i][j] = h;
      R[j][i] = C{h.re, -h.im};
    }
  }
  return INV_PIVOTED;
}

}  // namespace blk6
}  // namespace lqcd
