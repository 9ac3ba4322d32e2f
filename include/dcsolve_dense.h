/*
 * dcsolve_dense.h - the host-side small dense linear algebra of the solver,
 * exported so that it can be checked on a machine without a GPU.  None of
 * these calls touches a device.
 *
 * Matrices are complex128, column-major (entry (i, j) at 2*(i + j*ld)), with
 * ld = number of rows.  Return values follow dcsolve.h (0 = success, < 0
 * error, message in dc_last_error()).
 */
#ifndef DCSOLVE_DENSE_H
#define DCSOLVE_DENSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Eigenvalues w[2n] (re, im) and, if Z != NULL, unit-norm eigenvectors Z
 * (n x n) of a general complex matrix A (n x n): Hessenberg reduction by
 * Householder reflections, shifted QR iteration to Schur form, back
 * substitution for the eigenvectors.  DC_ERR_INVALID if the iteration does
 * not converge in 60 n sweeps. */
int dc_dense_eig(int32_t n, const double* A, double* w, double* Z);

/* Least squares min ||b - A x|| for A rows x cols (rows >= cols) by
 * Householder QR; x[2*cols]; *resnorm = ||b - A x||. */
int dc_dense_lstsq(int32_t rows, int32_t cols, const double* A, const double* b,
                   double* x, double* resnorm);

/* Solve A X = B for A (n x n) and B (n x nrhs, overwritten with X) by LU
 * with partial pivoting (the recycle refresh's generalised problem is
 * reduced to a standard one this way).  DC_ERR_INVALID if A is singular to
 * working precision. */
int dc_dense_solve(int32_t n, const double* A, int32_t nrhs, double* B);

/* Harmonic Ritz values of d Arnoldi steps (Sec. 3.3): eigenvalues of
 * H_d + |h_{d+1,d}|^2 f e_d^T with f = H_d^{-H} e_d; hbar is (d+1) x d. */
int dc_harmonic_ritz(int32_t d, const double* hbar, double* theta);

/* Leja order (Alg. 2) of d values; ties within a relative 1e-10 of the best
 * log-product go to the larger imaginary part, then the larger real part,
 * then the lower index. */
int dc_leja_order(int32_t d, const double* theta_in, double* theta_out);

#ifdef __cplusplus
}
#endif
#endif /* DCSOLVE_DENSE_H */
