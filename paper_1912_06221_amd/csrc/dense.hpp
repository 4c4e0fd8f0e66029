// Small dense FP64 linear algebra for the host-side operator setup.
#pragma once

#include <cmath>
#include <cstddef>
#include <stdexcept>
#include <vector>

namespace ardg {

struct Mat {
  int r = 0, c = 0;
  std::vector<double> a;
  Mat() = default;
  Mat(int rows, int cols, double v = 0.0) : r(rows), c(cols), a((size_t)rows * cols, v) {}
  double& operator()(int i, int j) { return a[(size_t)i * c + j]; }
  double operator()(int i, int j) const { return a[(size_t)i * c + j]; }
  static Mat eye(int n) {
    Mat m(n, n);
    for (int i = 0; i < n; ++i) m(i, i) = 1.0;
    return m;
  }
};

inline Mat matmul(const Mat& A, const Mat& B) {
  if (A.c != B.r) throw std::runtime_error("matmul shape");
  Mat C(A.r, B.c);
  for (int i = 0; i < A.r; ++i)
    for (int k = 0; k < A.c; ++k) {
      const double aik = A(i, k);
      if (aik == 0.0) continue;
      for (int j = 0; j < B.c; ++j) C(i, j) += aik * B(k, j);
    }
  return C;
}

inline Mat transpose(const Mat& A) {
  Mat T(A.c, A.r);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < A.c; ++j) T(j, i) = A(i, j);
  return T;
}

inline Mat sub(const Mat& A, int r0, int c0, int nr, int nc) {
  Mat S(nr, nc);
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nc; ++j) S(i, j) = A(r0 + i, c0 + j);
  return S;
}

inline Mat add(const Mat& A, const Mat& B, double beta = 1.0) {
  Mat C = A;
  for (size_t i = 0; i < C.a.size(); ++i) C.a[i] += beta * B.a[i];
  return C;
}

inline Mat hcat(const Mat& A, const Mat& B) {
  Mat C(A.r, A.c + B.c);
  for (int i = 0; i < A.r; ++i) {
    for (int j = 0; j < A.c; ++j) C(i, j) = A(i, j);
    for (int j = 0; j < B.c; ++j) C(i, A.c + j) = B(i, j);
  }
  return C;
}

inline Mat vcat(const Mat& A, const Mat& B) {
  Mat C(A.r + B.r, A.c);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < A.c; ++j) C(i, j) = A(i, j);
  for (int i = 0; i < B.r; ++i)
    for (int j = 0; j < B.c; ++j) C(A.r + i, j) = B(i, j);
  return C;
}

inline Mat blockdiag(const Mat& A, const Mat& B) {
  Mat C(A.r + B.r, A.c + B.c);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < A.c; ++j) C(i, j) = A(i, j);
  for (int i = 0; i < B.r; ++i)
    for (int j = 0; j < B.c; ++j) C(A.r + i, A.c + j) = B(i, j);
  return C;
}

// Inverse by LU with partial pivoting (Doolittle), solving for each unit column.
inline Mat inverse(const Mat& A) {
  const int n = A.r;
  if (A.c != n) throw std::runtime_error("inverse: not square");
  Mat LU = A;
  std::vector<int> piv(n);
  for (int i = 0; i < n; ++i) piv[i] = i;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(LU(k, k));
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(LU(i, k)) > best) { best = std::fabs(LU(i, k)); p = i; }
    if (best == 0.0) throw std::runtime_error("inverse: singular");
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(LU(k, j), LU(p, j));
      std::swap(piv[k], piv[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      LU(i, k) /= LU(k, k);
      const double l = LU(i, k);
      for (int j = k + 1; j < n; ++j) LU(i, j) -= l * LU(k, j);
    }
  }
  Mat X(n, n);
  std::vector<double> y(n);
  for (int col = 0; col < n; ++col) {
    for (int i = 0; i < n; ++i) {
      double s = (piv[i] == col) ? 1.0 : 0.0;
      for (int j = 0; j < i; ++j) s -= LU(i, j) * y[j];
      y[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = y[i];
      for (int j = i + 1; j < n; ++j) s -= LU(i, j) * X(j, col);
      X(i, col) = s / LU(i, i);
    }
  }
  return X;
}

// Moore-Penrose pseudo-inverse of a tall full-column-rank matrix via
// Householder QR: A = Q R, A^+ = R^{-1} Q^T.  Returns false if the smallest
// |R_ii| falls below rank_tol * max |R_ii|.
inline bool pinv_tall(const Mat& A, Mat& out, double rank_tol, double* cond_est) {
  const int m = A.r, n = A.c;
  if (m < n) return false;
  Mat R = A;
  Mat Qt = Mat::eye(m);  // accumulates H_n ... H_1
  std::vector<double> v(m);
  for (int k = 0; k < n; ++k) {
    double nrm = 0.0;
    for (int i = k; i < m; ++i) nrm += R(i, k) * R(i, k);
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) return false;
    const double alpha = (R(k, k) > 0) ? -nrm : nrm;
    for (int i = 0; i < m; ++i) v[i] = 0.0;
    v[k] = R(k, k) - alpha;
    for (int i = k + 1; i < m; ++i) v[i] = R(i, k);
    double vv = 0.0;
    for (int i = k; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int i = k; i < m; ++i) s += v[i] * R(i, j);
      s = 2.0 * s / vv;
      for (int i = k; i < m; ++i) R(i, j) -= s * v[i];
    }
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int i = k; i < m; ++i) s += v[i] * Qt(i, j);
      s = 2.0 * s / vv;
      for (int i = k; i < m; ++i) Qt(i, j) -= s * v[i];
    }
  }
  double dmax = 0.0, dmin = 1e300;
  for (int i = 0; i < n; ++i) {
    dmax = std::fmax(dmax, std::fabs(R(i, i)));
    dmin = std::fmin(dmin, std::fabs(R(i, i)));
  }
  if (cond_est) *cond_est = dmax / dmin;
  if (dmin < rank_tol * dmax) return false;
  // X = R^{-1} (Q^T)[0:n, :]
  out = Mat(n, m);
  for (int col = 0; col < m; ++col) {
    for (int i = n - 1; i >= 0; --i) {
      double s = Qt(i, col);
      for (int j = i + 1; j < n; ++j) s -= R(i, j) * out(j, col);
      out(i, col) = s / R(i, i);
    }
  }
  return true;
}

}  // namespace ardg
