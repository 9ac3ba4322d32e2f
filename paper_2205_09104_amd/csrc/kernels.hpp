// Launchers of the HIP kernels (implemented in kernels.hip).  All launchers
// enqueue on `st` and return immediately; `done` (may be null) is a device flag
// that makes every kernel of a pending Arnoldi cycle exit at entry once set.
#pragma once

#include "common.hpp"

namespace dc {

// ---------------------------------------------------------------- fixed scratch
// Size of the file-scope device array behind the no-allocation reduced apply
// (the odd-row temporary: V/2 x n complex values of the vector precision).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
// Device address of that array on the current device.  setup = true looks
// it up (hipGetSymbolAddress) on the first call for the device and keeps it;
// setup = false returns null if that has not happened yet.
void* noalloc_scratch(bool setup);

// Deterministic two-stage reduction scratch: each block of a reduction kernel
// stores its partial sums value-major, a one-wave-per-value finalize kernel
// sums them in a fixed order (results do not depend on block scheduling).
struct Reducer {
  double* partials = nullptr;   // capacity: kRedCap doubles
};
constexpr int kRedCap = 65536;

// ---------------------------------------------------------------- operator
// Re-lay out FP64 input blocks (self [V][n][n] + hops [V][4][n][n], device,
// row-major) into the tiled per-lane layout of each requested precision.
void launch_layout_blocks(const z64* self_in, const z64* hops_in, int V, int n,
                          void* out64, void* out32, void* out16, float* scales16,
                          hipStream_t st);

// Neighbour table int32 [8][V]: rows 0..3 = x + mu, rows 4..7 = x - mu.
void launch_neighbours(int* nbr, int L0, int L1, int L2, int L3, hipStream_t st);

// Apply, stage 1: each stored block is read once; the self block writes
// A_x psi_x + i*tm*Gamma5 psi_x into slot 4 of gbuf[x], the hop block B[x,mu]
// writes B psi_{x+mu} into slot 5+mu of gbuf[x] and the backward contribution
// Gamma5 B^H Gamma5 psi_x into slot mu of gbuf[x+mu].  gbuf: [V][9][n] in the
// vector precision.
// ev0/ev1 (optional): events that the dispatch records at its start and end.
void launch_apply_blocks(Prec p, int n, int V, const void* blocks, const float* scales,
                         const void* in, void* gbuf, const int* nbr, double tm,
                         const int* done, hipStream_t st, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);

// Apply, stage 2 (sum of the 9 slots in a fixed order) with an epilogue.
//   store : out = s
//   poly  : prod = prod - ca*s;  y = y + cb*prod         (polynomial chain step)
//   resid : out = b - s; result[0] = ||out||^2           (true residual)
void launch_gather_store(Prec p, int n, int V, const void* gbuf, void* out,
                         const int* done, hipStream_t st);
void launch_gather_poly(Prec p, int n, int V, const void* gbuf, void* prod, void* y,
                        z64 ca, z64 cb, const int* done, hipStream_t st);
//   poly_first : s = A v;  prod = v - ca*s;  y = c0*v + cb*prod  (first chain step)
void launch_gather_poly_first(Prec p, int n, int V, const void* gbuf, const void* v, void* prod,
                              void* y, z64 c0, z64 ca, z64 cb, const int* done, hipStream_t st);
void launch_gather_resid(Prec p, int n, int V, const void* gbuf, const void* b, void* out,
                         Reducer red, double* result, hipStream_t st);

// ---------------------------------------------------------------- block Jacobi
// Inverse of each site's self block A_x + i*tm*Gamma5 (Gauss-Jordan with
// partial pivoting), read from the tiled FP64 operator storage (slot 0) and
// written tiled in each requested precision; *singular is set to 1 if a zero
// pivot occurs.
void launch_invert_blocks(const void* tiled64, int V, int n, double tm, void* out64, void* out32,
                          void* out16, float* scales16, int* singular, hipStream_t st);
// out = B^{-1} in (plain vector)
void launch_bj_vec(Prec p, int n, int V, const void* inv, const float* scales, const void* in,
                   void* out, hipStream_t st);
// out = B^{-1} (sum of the gbuf slots), and the polynomial-chain variants
void launch_bj_gather_store(Prec p, int n, int V, const void* inv, const float* scales,
                            const void* gbuf, void* out, const int* done, hipStream_t st);
void launch_bj_gather_poly_first(Prec p, int n, int V, const void* inv, const float* scales,
                                 const void* gbuf, const void* v, void* prod, void* y, z64 c0,
                                 z64 ca, z64 cb, const int* done, hipStream_t st);
void launch_bj_gather_poly(Prec p, int n, int V, const void* inv, const float* scales,
                           const void* gbuf, void* prod, void* y, z64 ca, z64 cb, const int* done,
                           hipStream_t st);

// out_r = B_{site(r)}^{-1} in_r for rows r < rows of a compressed vector, where
// rowsite[r] is the lattice site of row r (null: row r is site r).
void launch_bj_rows(Prec p, int n, int rows, const int* rowsite, const void* inv,
                    const float* scales, const void* in, void* out, hipStream_t st);

// ---------------------------------------------------------------- odd-even reduction
// The reduced operator S = A_e - D_eo A_o^{-1} D_oe over compressed vectors
// (site x of a parity at row x / 2, every extent even), two site-centric kernels.
// launch_reduced_oe: t_o = A_o^{-1} D_oe x_e, with inv / invsc the self-block
// inverses of every site (tiled, indexed by site) and osite: int32 [V/2] odd
// row -> site.
void launch_reduced_oe(Prec p, int n, int V, const void* blocks, const float* scales,
                       const void* inv, const float* invsc, const void* x_e, void* t_o,
                       const int* nbr, const int* osite, const int* done, hipStream_t st,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// launch_reduced_eo: s = A_e x_e - D_eo t_o (x_e null: -D_eo t_o) with the
// epilogue epi: 0 out = s; 1 p = e - ca s, out = p, y = c0 e + cb p; 2 p = out -
// ca s, out = p, y += cb p; 3 out = e - s.  esite: int32 [V/2] even row -> site.
// einv (null: none) selects the left block-Jacobi form with B = D_ee:
// s = x_e - A_e^{-1} D_eo t_o (= B^{-1} of the above), with einv / einvsc the
// self-block inverses of every site (tiled, indexed by site); epi 0..2 only.
void launch_reduced_eo(Prec p, int epi, int n, int V, const void* blocks, const float* scales,
                       const void* einv, const float* einvsc, const void* x_e, const void* t_o,
                       const int* nbr, const int* esite, double tm, void* out, const void* e,
                       void* y, z64 c0, z64 ca, z64 cb, const int* done, hipStream_t st,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Single-read form of the same operator (FP32 / FP16 blocks, n a multiple of
// 8 up to 64): launch_reduced_scatter forms t_o as launch_reduced_oe does and,
// from the same read of each hop block, the eight D_eo products of t_o that each
// even row needs, into hp: [V/2][8][n] vectors of the vector precision (slots
// 0-3 forward hops mu, 4-7 backward hops mu); launch_reduced_gather sums them
// and finishes the rows as launch_reduced_eo does (same arguments, hp in place
// of t_o).  Results equal the two-kernel form's bit for bit.
void launch_reduced_scatter(Prec p, int n, int V, const void* blocks, const float* scales,
                            const void* inv, const float* invsc, const void* x_e, void* hp,
                            const int* nbr, const int* osite, const int* done, hipStream_t st,
                            hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
void launch_reduced_gather(Prec p, int epi, int n, int V, const void* blocks,
                           const float* scales, const void* einv, const float* einvsc,
                           const void* x_e, const void* hp, const int* esite, double tm,
                           void* out, const void* e, void* y, z64 c0, z64 ca, z64 cb,
                           const int* done, hipStream_t st, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr);
// Which form the solver's reduced applies take (process-wide): mode 0
// (default) the single-read pair where it applies (reduced_single_read), 1
// always the two-kernel form.
void set_reduced_mode(int mode);
int reduced_mode();
bool reduced_single_read(Prec p, int n);
// split a full-lattice vector into its compressed even and odd halves, or merge
// them back (dir 0: split, 1: merge); esite/osite: int32 [V/2] row -> site
void launch_oddeven_split(Prec p, int n, int half_sites, const int* esite, const int* osite,
                          void* full, void* ve, void* vo, int dir, hipStream_t st);

// ---------------------------------------------------------------- multi-RHS apply
// yout[r] = D xin[r] for r < R (device arrays of R vector pointers, vectors in
// the precision's vector type), MFMA based; g5io bit 0 multiplies inputs and
// bit 1 outputs by Gamma5 (adjoint through Gamma5 D(-mu) Gamma5 with tm = -mu).
void launch_apply_multi(Prec p, int n, int V, const void* blocks, const float* scales,
                        const void* const* xin, void* const* yout, int R, const int* nbr, double tm,
                        int g5io, hipStream_t st);
size_t multi_lds_bytes(int n, bool dbl, int rb);
// right-hand-side tile chosen for a multi-apply shape (0: not tuned yet), and
// the tuning mode (0: autotune, 16/32/64: force that tile; 0 clears the table)
int multi_tile_for(Prec p, int n, int rmax, unsigned sites);
void set_multi_tile_mode(int mode);
// The same over a work list of several operators with one block size n (a
// mixed batch of lattices): operator i contributes V sites and R right-hand
// sides (its own pointer arrays xin/yout, twisted mass tm); one launch.
constexpr int kMaxMultiOps = 8;
struct MultiOpDesc {
  const void* blocks = nullptr;
  const float* scales = nullptr;
  const int* nbr = nullptr;
  const void* const* xin = nullptr;
  void* const* yout = nullptr;
  int V = 0, R = 0, site0 = 0;   // site0: set by the launcher
  double tm = 0.0;
};
struct MultiOps {
  MultiOpDesc op[kMaxMultiOps];
  int n_ops, n, g5io;
};
void launch_apply_multi_ops(Prec p, int n, const MultiOpDesc* desc, int n_ops, int g5io,
                            hipStream_t st);
// batched polynomial-chain step over R vectors (device pointer arrays):
//   first:  prod = v - ca t;  y = c0 v + cb prod;   else: prod -= ca t;  y += cb prod
void launch_chain_multi(Prec p, const void* const* t, const void* const* v, void* const* prod,
                        void* const* y, int R, size_t N, z64 c0, z64 ca, z64 cb, int first,
                        hipStream_t st);

// ---------------------------------------------------------------- BLAS-1/2
// result[q] = basis_q^H w (complex, q < q0 + q1; basis_q = b0 + q*N for q < q0,
// b1 + (q-q0)*N after), and if want_norm result[q0+q1] = ||w||^2 (real part).
void launch_multidot(Prec p, const void* b0, int q0, const void* b1, int q1, size_t N,
                     const void* w, int want_norm, Reducer red, double* result,
                     const int* done, hipStream_t st);
// w -= sum_q coef[q] basis_q (coef device complex [q0+q1]); if want_norm,
// result[0] = ||w||^2 after the update.
void launch_multiaxpy(Prec p, void* w, const void* b0, int q0, const void* b1, int q1,
                      size_t N, const double* coef, int want_norm, Reducer red,
                      double* result, const int* done, hipStream_t st);
// w = (w - sum_q coef_q basis_q) * (*scale) for Arnoldi step j: runs only if
// that step's bookkeeping ran (*jdone == j + 1); no norm.
void launch_multiaxpy_scaled(Prec p, void* w, const void* b0, int q0, const void* b1, int q1,
                             size_t N, const double* coef, const double* scale, const int* jdone,
                             int j, hipStream_t st);
// out_r (= or +=) sum_q coef[r*Q + q] basis_q for r < R, Q = q0 + q1; coef
// device complex; outputs are R vectors with stride N, not overlapping the
// basis.  Products and sums in FP64 (16 or more outputs: on MFMA tiles).
void launch_combine(Prec p, const void* b0, int q0, const void* b1, int q1, size_t N,
                    const double* coef, int R, void* out, int accumulate, hipStream_t st);
// ---------------------------------------------------------------- block products
// Number of row chunks the Gram product of qa and rb vectors of length N is
// split into (at most 256; at most part_cap / (qa rb) when part_cap > 0).
int block_gram_parts(size_t N, int qa, int rb, size_t part_cap = 0);
// out = A^H B (qa x rb, column-major, FP64 complex; the chunks summed in FP64)
// for qa vectors A and rb vectors B of N entries each (stride N) in the
// precision's vector type, MFMA based.  The products are formed in FP64 for
// FP64 vectors, and for FP32 vectors when fp64_products is set, else in FP32.
// part: device scratch of block_gram_parts(N, qa, rb, part_cap) * qa * rb
// complex values of the product type.
void launch_block_gram(Prec p, const void* A, int qa, const void* B, int rb, size_t N, void* part,
                       z64* out, hipStream_t st, bool fp64_products = false,
                       size_t part_cap = 0);
// C = beta C + alpha A S: A k vectors, C r vectors (N entries each, stride N),
// S k x r column-major (leading dimension k) in the vector type; C must not
// overlap A.  MFMA based, products in the vector type.
void launch_block_update(Prec p, const void* A, int k, const void* S, void* C, int r, size_t N,
                         z64 alpha, z64 beta, hipStream_t st);
// out = in * (*scale_dev) (scale real, device) or in * s (if scale_dev null).
void launch_scale(Prec p, const void* in, void* out, size_t N, const double* scale_dev,
                  double s, const int* done, hipStream_t st);
// out = c * in (complex c); in == out allowed
void launch_cscale(Prec p, const void* in, void* out, size_t N, z64 c, const int* done,
                   hipStream_t st);
// v *= *inv_h if *jdone == j + 1 (normalise the new Arnoldi vector of step j)
void launch_scale_step(Prec p, void* v, size_t N, const double* inv_h, const int* jdone, int j,
                       hipStream_t st);
// x = 0
void launch_zero(Prec p, void* x, size_t N, hipStream_t st);
// bytes (a multiple of 4, both pointers 4-byte aligned) from src to dst, one of
// them host-mapped pinned memory given by its device address
void launch_copy_words(const void* src, void* dst, size_t bytes, hipStream_t st);
// up to kCopySegMax independent copies of 4-byte words in one launch
constexpr int kCopySegMax = 8;
struct CopySegments {
  const uint32_t* src[kCopySegMax];
  uint32_t* dst[kCopySegMax];
  size_t words[kCopySegMax];
  int count = 0;
};
void launch_copy_segments(const CopySegments& s, hipStream_t st);
// y = a*x + y (complex a)
void launch_axpy(Prec p, z64 a, const void* x, void* y, size_t N, hipStream_t st);
// result[0] = ||x||^2
void launch_norm2(Prec p, const void* x, size_t N, Reducer red, double* result, hipStream_t st);
// result[i] = ||x_i||^2 for the q vectors x_i = x + i*N (q <= kRedCap)
void launch_colnorm2(Prec p, const void* x, int q, size_t N, Reducer red, double* result,
                     hipStream_t st);
// out = Gamma5 in (per-site sign); in == out allowed
void launch_gamma5(Prec p, const void* in, void* out, int V, int n, hipStream_t st);
// precision conversions (with optional Gamma5): out = g5? * in
void launch_convert_64to32(const z64* in, z32* out, size_t N, int n, int g5, hipStream_t st);
void launch_convert_32to64(const z32* in, z64* out, size_t N, int n, int g5, hipStream_t st);
// standard complex Gaussians from Philox4x32-10 (counter = (index, stream, 0))
void launch_gaussian(z64* out, size_t N, uint64_t seed, uint32_t stream_id, hipStream_t st);

// ---------------------------------------------------------------- Arnoldi
// One-wave bookkeeping kernel after the two Gram-Schmidt passes of step j:
// H(:, j) = c1 + c2 (the V part), Bk(:, j) = (C part), h_{j+1,j} = sqrt(nrm2),
// Givens update of the residual estimate, done flag on convergence
// (estimate <= target) or breakdown (h_{j+1,j} <= brk * ||A v_j||).
struct ArnoldiDev {
  int ldh = 0;      // leading dimension of H (>= steps + 1)
  int ldb = 1;      // leading dimension of Bk (>= kC, >= 1)
  double* H;        // complex ldh x steps column-major
  double* Bk;       // complex ldb x steps column-major
  double* giv;      // complex g[ldh+1], c[ldh] (real parts used), s[ldh]
  double* inv_h;    // 1 / h_{j+1,j}
  double* est;      // |g[j+1]|
  int* done;        // cycle flag
  int* jdone;       // steps completed
  int* brk_flag;    // 1 if the cycle ended by breakdown
  int* hdone = nullptr;  // optional host-mapped copy of the done flag (set to 1 with it)
  double* hest = nullptr;  // optional host-mapped per-step estimates: hest[j] after step j
  const double* target_dev = nullptr;  // optional: the stopping target read from device memory
                                       // (replaces the value argument; graph replays)
};
// c2 null: the single-sync process (one pass of coefficients c1, whose entry
// kC + j + 1 is ||A v_j||^2; h_{j+1,j}^2 = ||A v_j||^2 - sum |c1|^2; nrm2 unused).
void launch_arnoldi_finish(ArnoldiDev a, int steps, int kC, int j, const double* c1,
                           const double* c2, const double* nrm2, double target, double brk,
                           hipStream_t st);
// beta_dev: take beta from device memory instead
void launch_arnoldi_init(ArnoldiDev a, double beta, hipStream_t st,
                         const double* beta_dev = nullptr);

// Batched Gram-Schmidt: the launches of one classical Gram-Schmidt step (as
// launch_multidot / launch_multiaxpy / launch_arnoldi_finish /
// launch_scale_step) for up to kOrthCols independent columns at once, each
// column with its own basis, vector length, reduction partials and stop flag.
// Every column takes exactly the grid, partial layout and sums of its own
// launch, so results are the per-column launches' bit for bit.  The columns of
// one call need equal basis sizes q0 + q1; the tables travel as kernel
// arguments (graph capture records them).
constexpr int kOrthCols = 16;
struct OrthCol {
  const void* b0 = nullptr;      // basis part 0: q0 vectors of N (or null)
  const void* b1 = nullptr;      // basis part 1: q1 vectors of N
  void* w = nullptr;             // the column's vector (updated in place)
  double* partials = nullptr;    // the column's own reduction partials (kRedCap doubles)
  double* result = nullptr;      // dots: 2 (q0 + q1 [+ 1 norm]) doubles; update: the norm
  const double* coef = nullptr;  // update coefficients (complex, q0 + q1)
  const int* done = nullptr;     // the column's stop flag (null: never stops)
  size_t N = 0;
  int q0 = 0, q1 = 0;
  unsigned gx = 0;               // set by the launchers
};
struct OrthCols {
  OrthCol c[kOrthCols];
  int count = 0;
};
// result = [b0 b1]^H w (and ||w||^2 after them if want_norm), per column
void launch_multidot_cols(Prec p, const OrthCols& t, int want_norm, hipStream_t st);
// w -= [b0 b1] coef per column; with want_norm result = ||w||^2 after it
void launch_multiaxpy_cols(Prec p, const OrthCols& t, int want_norm, hipStream_t st);
struct FinishCol {
  ArnoldiDev a;
  const double* c1 = nullptr;
  const double* c2 = nullptr;
  const double* nrm2 = nullptr;
  double target = 0.0;
  int kC = 0;
};
struct FinishCols {
  FinishCol c[kOrthCols];
  int count = 0;
};
void launch_arnoldi_finish_cols(const FinishCols& t, int steps, int j, double brk,
                                hipStream_t st);
struct ScaleCols {
  void* v[kOrthCols] = {};
  size_t N[kOrthCols] = {};
  const double* inv_h[kOrthCols] = {};
  const int* jdone[kOrthCols] = {};
  int count = 0;
};
void launch_scale_step_cols(Prec p, const ScaleCols& t, int j, hipStream_t st);
// the tables travel as kernel arguments, which must stay within 4 KB
static_assert(sizeof(OrthCols) + 16 <= 4096, "column table too large for kernel arguments");
static_assert(sizeof(FinishCols) + 32 <= 4096, "finish table too large for kernel arguments");
static_assert(sizeof(ScaleCols) + 16 <= 4096, "scale table too large for kernel arguments");
// launch_chain_multi for up to kChainGroups operators' column sets in one
// launch (each with its own pointer tables, length and coefficients).
constexpr int kChainGroups = 8;
struct ChainGroups {
  const void* t[kChainGroups] = {};
  const void* v[kChainGroups] = {};
  const void* prod[kChainGroups] = {};
  const void* y[kChainGroups] = {};
  size_t N[kChainGroups] = {};
  int R[kChainGroups] = {};
  z64 c0[kChainGroups] = {}, ca[kChainGroups] = {}, cb[kChainGroups] = {};
  int count = 0;
};
void launch_chain_groups(Prec p, const ChainGroups& g, int first, hipStream_t st);
static_assert(sizeof(ChainGroups) + 16 <= 4096, "chain table too large for kernel arguments");
// Whether lockstep batches use the column / operator tables above (1,
// default) or launch per column and per operator (0); process-wide, equal
// results.
void set_batch_launches(int batched);
int batch_launches();
// out[0] = sqrt(*nrm2), out[1] = its reciprocal (0 for a zero norm); device pointers
void launch_norm_root(const double* nrm2, double* out, hipStream_t st);

// ---------------------------------------------------------------- gradient
void launch_grad_hops(const z64* lam, const z64* x, z64* grad, const int* nbr, int V, int n,
                      int tied, hipStream_t st);

}  // namespace dc
