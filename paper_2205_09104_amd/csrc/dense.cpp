// Host FP64 dense linear algebra; see dense.hpp.
#include "dense.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace dc {

// The inner loops below spell complex products out in real arithmetic on the
// interleaved (re, im) storage: the library operator* of std::complex carries
// a NaN/infinity recovery path that keeps these loops from vectorising.

// y[0..n) += b x[0..n) (complex, contiguous)
static inline void caxpy(int n, cd b, const cd* x, cd* y) {
  const double br = b.real(), bi = b.imag();
  const double* xd = reinterpret_cast<const double*>(x);
  double* yd = reinterpret_cast<double*>(y);
  for (int i = 0; i < n; ++i) {
    const double xr = xd[2 * i], xi = xd[2 * i + 1];
    yd[2 * i] += br * xr - bi * xi;
    yd[2 * i + 1] += br * xi + bi * xr;
  }
}

// sum_i conj(x_i) y_i (complex, contiguous)
static inline cd cdotc(int n, const cd* x, const cd* y) {
  const double* xd = reinterpret_cast<const double*>(x);
  const double* yd = reinterpret_cast<const double*>(y);
  double sr = 0.0, si = 0.0;
  for (int i = 0; i < n; ++i) {
    const double xr = xd[2 * i], xi = xd[2 * i + 1], yr = yd[2 * i], yi = yd[2 * i + 1];
    sr += xr * yr + xi * yi;
    si += xr * yi - xi * yr;
  }
  return cd(sr, si);
}

static inline cd cmul(cd a, cd b) {
  return cd(a.real() * b.real() - a.imag() * b.imag(), a.real() * b.imag() + a.imag() * b.real());
}

Mat matmul(const Mat& A, const Mat& B) {
  Mat C(A.r, B.c);
  for (int j = 0; j < B.c; ++j)
    for (int k = 0; k < A.c; ++k) {
      const cd b = B(k, j);
      if (b == cd(0.0)) continue;
      caxpy(A.r, b, &A.a[size_t(k) * A.r], &C.a[size_t(j) * C.r]);
    }
  return C;
}

Mat adjoint(const Mat& A) {
  Mat H(A.c, A.r);
  for (int j = 0; j < A.c; ++j)
    for (int i = 0; i < A.r; ++i) H(j, i) = std::conj(A(i, j));
  return H;
}

Mat block(const Mat& A, int r0, int c0, int rows, int cols) {
  Mat B(rows, cols);
  for (int j = 0; j < cols; ++j)
    for (int i = 0; i < rows; ++i) B(i, j) = A(r0 + i, c0 + j);
  return B;
}

// Householder vector for x = A(k.., k): returns beta and fills v (v[0] = 1
// convention not used; v is unnormalised with tau = 2 / v^H v).
static double householder(std::vector<cd>& v, double& alpha_abs) {
  double nx = 0.0;
  for (auto& z : v) nx += std::norm(z);
  nx = std::sqrt(nx);
  alpha_abs = nx;
  if (nx == 0.0) return 0.0;
  const cd x0 = v[0];
  const cd phase = (std::abs(x0) == 0.0) ? cd(1.0) : x0 / std::abs(x0);
  v[0] = x0 + phase * nx;          // v = x + e^{i arg x0} ||x|| e_1
  double vv = 0.0;
  for (auto& z : v) vv += std::norm(z);
  return vv == 0.0 ? 0.0 : 2.0 / vv;
}

// Apply (I - tau v v^H) from the left to rows k.. of columns c0..c1-1.
static void reflect_left(Mat& A, int k, const std::vector<cd>& v, double tau, int c0, int c1) {
  if (tau == 0.0) return;
  const int m = int(v.size());
  for (int j = c0; j < c1; ++j) {
    cd* col = &A(k, j);
    const cd s = tau * cdotc(m, v.data(), col);
    caxpy(m, -s, v.data(), col);
  }
}

// Apply (I - tau v v^H) from the right to columns k.. of rows r0..r1-1:
// s = A v over the rows, then A -= tau s v^H, column by column.
static void reflect_right(Mat& A, int k, const std::vector<cd>& v, double tau, int r0, int r1) {
  if (tau == 0.0 || r1 <= r0) return;
  const int rows = r1 - r0;
  std::vector<cd> sv(size_t(rows), cd(0.0));
  for (size_t j = 0; j < v.size(); ++j) caxpy(rows, v[j], &A(r0, k + int(j)), sv.data());
  for (size_t j = 0; j < v.size(); ++j)
    caxpy(rows, -tau * std::conj(v[j]), sv.data(), &A(r0, k + int(j)));
}

std::vector<cd> lstsq(const Mat& A0, const std::vector<cd>& b0, double* resnorm) {
  Mat A = A0;
  std::vector<cd> b = b0;
  const int m = A.r, n = A.c;
  for (int k = 0; k < n && k < m; ++k) {
    std::vector<cd> v(m - k);
    for (int i = k; i < m; ++i) v[i - k] = A(i, k);
    double an;
    const double tau = householder(v, an);
    reflect_left(A, k, v, tau, k, n);
    if (tau != 0.0) {
      cd s = 0.0;
      for (int i = k; i < m; ++i) s += std::conj(v[i - k]) * b[i];
      s *= tau;
      for (int i = k; i < m; ++i) b[i] -= v[i - k] * s;
    }
  }
  std::vector<cd> x(n, cd(0.0));
  for (int i = n - 1; i >= 0; --i) {
    cd s = b[i];
    for (int j = i + 1; j < n; ++j) s -= A(i, j) * x[j];
    x[i] = (std::abs(A(i, i)) == 0.0) ? cd(0.0) : s / A(i, i);
  }
  if (resnorm) {
    double r = 0.0;
    for (int i = n; i < m; ++i) r += std::norm(b[i]);
    *resnorm = std::sqrt(r);
  }
  return x;
}

void qr_thin(const Mat& A0, Mat& Q, Mat& R) {
  Mat A = A0;
  const int m = A.r, n = A.c;
  std::vector<std::vector<cd>> vs(n);
  std::vector<double> taus(n);
  for (int k = 0; k < n; ++k) {
    std::vector<cd> v(m - k);
    for (int i = k; i < m; ++i) v[i - k] = A(i, k);
    double an;
    taus[k] = householder(v, an);
    reflect_left(A, k, v, taus[k], k, n);
    vs[k] = v;
  }
  R = Mat(n, n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= j; ++i) R(i, j) = A(i, j);
  // Q = H_0 H_1 ... H_{n-1} applied to the first n columns of I
  Q = Mat(m, n);
  for (int i = 0; i < n; ++i) Q(i, i) = 1.0;
  for (int k = n - 1; k >= 0; --k) reflect_left(Q, k, vs[k], taus[k], 0, n);
}

bool lu_solve(const Mat& A0, Mat& B) {
  Mat A = A0;
  const int n = A.r;
  std::vector<int> piv(n);
  double amax = 0.0;
  for (auto& z : A.a) amax = std::max(amax, std::abs(z));
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::abs(A(k, k));
    for (int i = k + 1; i < n; ++i)
      if (std::abs(A(i, k)) > best) { best = std::abs(A(i, k)); p = i; }
    if (best == 0.0 || best <= 1e-300 * (amax > 0 ? amax : 1.0)) return false;
    piv[k] = p;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A(k, j), A(p, j));
      for (int j = 0; j < B.c; ++j) std::swap(B(k, j), B(p, j));
    }
    // multipliers l_i = A(i,k) / A(k,k) in column k, then every later column
    // of A and every column of B updated by a contiguous axpy
    const cd inv = 1.0 / A(k, k);
    const int below = n - k - 1;
    for (int i = k + 1; i < n; ++i) A(i, k) = cmul(A(i, k), inv);
    for (int j = k + 1; j < n; ++j) caxpy(below, -A(k, j), &A(k + 1, k), &A(k + 1, j));
    for (int j = 0; j < B.c; ++j) caxpy(below, -B(k, j), &A(k + 1, k), &B(k + 1, j));
  }
  // back substitution, column-oriented: x_i = b_i / A(i,i), then the rows
  // above lose x_i A(0..i-1, i)
  for (int j = 0; j < B.c; ++j)
    for (int i = n - 1; i >= 0; --i) {
      const cd x = B(i, j) / A(i, i);
      B(i, j) = x;
      if (i > 0) caxpy(i, -x, &A(0, i), &B(0, j));
    }
  return true;
}

Mat tri_inverse(const Mat& R) {
  const int n = R.r;
  Mat X = Mat::eye(n);
  for (int j = 0; j < n; ++j)
    for (int i = j; i >= 0; --i) {   // column j of R^{-1} is zero below row j
      const cd x = X(i, j) / R(i, i);
      X(i, j) = x;
      if (i > 0) caxpy(i, -x, &R(0, i), &X(0, j));
    }
  return X;
}

// Reduce A to upper Hessenberg H = Q^H A Q.
static void hessenberg(Mat& H, Mat& Q) {
  const int n = H.r;
  Q = Mat::eye(n);
  for (int k = 0; k + 2 < n; ++k) {
    std::vector<cd> v(n - k - 1);
    for (int i = k + 1; i < n; ++i) v[i - k - 1] = H(i, k);
    double an;
    const double tau = householder(v, an);
    reflect_left(H, k + 1, v, tau, 0, n);
    reflect_right(H, k + 1, v, tau, 0, n);
    reflect_right(Q, k + 1, v, tau, 0, n);
    for (int i = k + 2; i < n; ++i) H(i, k) = 0.0;
  }
}

// Columns x, y (length n) <- (c x + conj(s) y, -s x + c y): the right
// multiplication of the pair by G^H.
static inline void rot_cols(int n, double c, cd s, cd* x, cd* y) {
  const double sr = s.real(), si = s.imag();
  double* xd = reinterpret_cast<double*>(x);
  double* yd = reinterpret_cast<double*>(y);
  for (int i = 0; i < n; ++i) {
    const double xr = xd[2 * i], xi = xd[2 * i + 1], yr = yd[2 * i], yi = yd[2 * i + 1];
    xd[2 * i] = c * xr + sr * yr + si * yi;        // c x + conj(s) y
    xd[2 * i + 1] = c * xi + sr * yi - si * yr;
    yd[2 * i] = c * yr - (sr * xr - si * xi);      // -s x + c y
    yd[2 * i + 1] = c * yi - (sr * xi + si * xr);
  }
}

// Complex Givens rotation G = [[c, s], [-conj(s), c]] with G [a; b] = [r; 0].
static void givens(cd a, cd b, double& c, cd& s) {
  const double aa = std::abs(a), bb = std::abs(b);
  if (bb == 0.0) { c = 1.0; s = 0.0; return; }
  if (aa == 0.0) { c = 0.0; s = std::conj(b) / bb; return; }
  const double r = std::hypot(aa, bb);
  c = aa / r;
  s = (a / aa) * std::conj(b) / r;
}

bool eig(const Mat& A, std::vector<cd>& w, Mat* Z) {
  const int n = A.r;
  w.assign(n, cd(0.0));
  if (n == 0) return true;
  Mat H = A, Q;
  hessenberg(H, Q);
  double hnorm = 0.0;
  for (auto& z : H.a) hnorm = std::max(hnorm, std::abs(z));
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int iter_since = 0, total = 0;
  const int max_total = 60 * std::max(n, 1) + 100;
  while (hi >= 0) {
    // find the start of the active unreduced block
    int l = hi;
    while (l > 0) {
      const double s = std::abs(H(l - 1, l - 1)) + std::abs(H(l, l));
      if (std::abs(H(l, l - 1)) <= eps * (s == 0.0 ? hnorm : s)) {
        H(l, l - 1) = 0.0;
        break;
      }
      --l;
    }
    if (l == hi) {          // 1x1 block converged
      w[hi] = H(hi, hi);
      --hi;
      iter_since = 0;
      continue;
    }
    if (++total > max_total) return false;
    ++iter_since;
    // Wilkinson shift from the trailing 2x2 of the active block
    cd sigma;
    const cd a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
    if (iter_since % 11 == 10) {
      sigma = d + cd(0.75 * std::abs(H(hi, hi - 1)), 0.0);   // exceptional shift
    } else {
      const cd half = 0.5 * (a - d);
      const cd disc = std::sqrt(half * half + b * c);
      const cd e1 = 0.5 * (a + d) + disc, e2 = 0.5 * (a + d) - disc;
      sigma = (std::abs(e1 - d) < std::abs(e2 - d)) ? e1 : e2;
    }
    // implicit single-shift QR sweep on rows/cols l..hi (bulge chase)
    cd x = H(l, l) - sigma, y = H(l + 1, l);
    for (int k = l; k < hi; ++k) {
      double cs;
      cd sn;
      givens(x, y, cs, sn);
      // rows k, k+1 (left multiplication by G): the two entries of a column
      // are adjacent in memory
      {
        const double sr = sn.real(), si = sn.imag();
        const int j0 = (k > l ? k - 1 : l);
        double* p = reinterpret_cast<double*>(&H(k, j0));
        const size_t stride = 2 * size_t(H.r);
        for (int j = j0; j < n; ++j, p += stride) {
          const double ar = p[0], ai = p[1], br = p[2], bi = p[3];
          p[0] = cs * ar + sr * br - si * bi;        // cs t1 + sn t2
          p[1] = cs * ai + sr * bi + si * br;
          p[2] = cs * br - (sr * ar + si * ai);      // -conj(sn) t1 + cs t2
          p[3] = cs * bi - (sr * ai - si * ar);
        }
      }
      if (k > l) H(k + 1, k - 1) = 0.0;      // the bulge just chased away
      // columns k, k+1 (right multiplication by G^H)
      const int rmax = std::min(k + 2, hi);
      rot_cols(rmax + 1, cs, sn, &H(0, k), &H(0, k + 1));
      rot_cols(n, cs, sn, &Q(0, k), &Q(0, k + 1));
      if (k + 1 < hi) {
        x = H(k + 1, k);
        y = H(k + 2, k);
      }
    }
  }
  if (Z) {
    // H is now upper triangular (Schur form T); eigenvectors of T by back
    // substitution (column-oriented: once y_j is known, the rows above
    // collect H(0..j-1, j) y_j), then Z = Q y, normalised.
    Mat Y(n, n);
    const double small = eps * (hnorm > 0 ? hnorm : 1.0);
    for (int k = 0; k < n; ++k) {
      cd* y = &Y(0, k);     // holds the partial sums above the row solved last
      y[k] = 1.0;
      if (k > 0) caxpy(k, cd(1.0), &H(0, k), y);
      for (int i = k - 1; i >= 0; --i) {
        cd den = H(i, i) - H(k, k);
        if (std::abs(den) < small) den = small;
        const cd yi = -y[i] / den;
        y[i] = yi;
        if (i > 0) caxpy(i, yi, &H(0, i), y);
      }
    }
    *Z = matmul(Q, Y);
    for (int k = 0; k < n; ++k) {
      double nn = 0.0;
      for (int i = 0; i < n; ++i) nn += std::norm((*Z)(i, k));
      nn = std::sqrt(nn);
      if (nn > 0)
        for (int i = 0; i < n; ++i) (*Z)(i, k) /= nn;
    }
  }
  return true;
}

bool harmonic_ritz(const Mat& Hbar, std::vector<cd>& theta, Mat* Z) {
  const int d = Hbar.c;
  Mat Hd = block(Hbar, 0, 0, d, d);
  const double h2 = std::norm(Hbar(d, d - 1));
  Mat M = Hd;
  if (h2 != 0.0) {
    Mat f(d, 1);
    f(d - 1, 0) = 1.0;
    if (!lu_solve(adjoint(Hd), f)) return false;
    for (int i = 0; i < d; ++i) M(i, d - 1) += h2 * f(i, 0);
  }
  return eig(M, theta, Z);
}

std::vector<cd> leja_order(const std::vector<cd>& theta) {
  const int d = int(theta.size());
  std::vector<double> score(d);
  std::vector<char> taken(d, 0);
  std::vector<cd> out;
  out.reserve(d);
  for (int i = 0; i < d; ++i) score[i] = std::log(std::abs(theta[i]));
  for (int step = 0; step < d; ++step) {
    double best = -INFINITY;
    for (int i = 0; i < d; ++i)
      if (!taken[i] && score[i] > best) best = score[i];
    int pick = -1;
    const bool finite = std::isfinite(best);
    const double tol = finite ? 1e-10 * std::max(1.0, std::abs(best)) : 0.0;
    for (int i = 0; i < d; ++i) {
      if (taken[i]) continue;
      const bool cand = finite ? (score[i] >= best - tol) : (score[i] == best);
      if (!cand) continue;
      if (pick < 0) { pick = i; continue; }
      const cd a = theta[i], b = theta[pick];
      if (a.imag() > b.imag() || (a.imag() == b.imag() && a.real() > b.real())) pick = i;
    }
    taken[pick] = 1;
    out.push_back(theta[pick]);
    for (int i = 0; i < d; ++i) {
      const double dist = std::log(std::abs(theta[i] - theta[pick]));
      score[i] = (step == 0 ? 0.0 : score[i]) + dist;
    }
  }
  return out;
}

std::vector<int> smallest_k(const std::vector<cd>& w, int k) {
  std::vector<int> idx(w.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    double x = std::abs(w[a]), y = std::abs(w[b]);
    if (!std::isfinite(x)) x = INFINITY;
    if (!std::isfinite(y)) y = INFINITY;
    return x < y;
  });
  if (int(idx.size()) > k) idx.resize(k);
  return idx;
}

}  // namespace dc
