// Small dense complex linear algebra on the host, FP64.  Written from the
// textbook algorithms (Householder reflections, implicitly shifted QR with
// Wilkinson shifts, triangular back substitution, LU with partial pivoting);
// used for the Hessenberg least-squares problems, harmonic Ritz values and
// vectors and the GCRO-DR recycle-space refresh.
#pragma once

#include <complex>
#include <string>
#include <vector>

namespace dc {

using cd = std::complex<double>;

// Column-major complex matrix.
struct Mat {
  int r = 0, c = 0;
  std::vector<cd> a;
  Mat() = default;
  Mat(int rows, int cols) : r(rows), c(cols), a(size_t(rows) * cols, cd(0.0)) {}
  cd& operator()(int i, int j) { return a[size_t(i) + size_t(j) * r]; }
  const cd& operator()(int i, int j) const { return a[size_t(i) + size_t(j) * r]; }
  static Mat eye(int n) {
    Mat m(n, n);
    for (int i = 0; i < n; ++i) m(i, i) = 1.0;
    return m;
  }
};

Mat matmul(const Mat& A, const Mat& B);
Mat adjoint(const Mat& A);
Mat block(const Mat& A, int r0, int c0, int rows, int cols);

// Least squares min ||b - A x|| (rows >= cols) via Householder QR.
// Returns x (cols); *resnorm = ||b - A x|| computed from the transformed rhs.
std::vector<cd> lstsq(const Mat& A, const std::vector<cd>& b, double* resnorm);

// Thin QR of A (rows >= cols): A = Q R, Q rows x cols with orthonormal
// columns, R cols x cols upper triangular.
void qr_thin(const Mat& A, Mat& Q, Mat& R);

// Solve A X = B with LU (partial pivoting).  Returns false if A is singular.
bool lu_solve(const Mat& A, Mat& B);

// Inverse of an upper triangular matrix.
Mat tri_inverse(const Mat& R);

// Eigen-decomposition of a general complex matrix: w eigenvalues, Z (if
// wanted) unit-norm eigenvectors.  Returns false if QR does not converge.
bool eig(const Mat& A, std::vector<cd>& w, Mat* Z);

// Harmonic Ritz values (and vectors if Z != nullptr) from a (d+1) x d
// Hessenberg matrix: eig(H_d + |h_{d+1,d}|^2 H_d^{-H} e_d e_d^T).
bool harmonic_ritz(const Mat& Hbar, std::vector<cd>& theta, Mat* Z);

// Leja order (ties: larger Im, larger Re, lower index).
std::vector<cd> leja_order(const std::vector<cd>& theta);

// Indices of the k entries of smallest modulus (stable).
std::vector<int> smallest_k(const std::vector<cd>& w, int k);

}  // namespace dc
