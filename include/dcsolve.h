/*
 * dcsolve.h - C ABI of the MI355X coarsest-level solver.
 *
 * The library solves D_c x = b for the coarsest-level operator of an
 * aggregation-based multigrid for lattice QCD (Espinoza-Valverde, Frommer,
 * Ramirez-Hidalgo, Rottmann, "Coarsest-level improvements in multigrid for
 * lattice QCD on large-scale computers"):
 *   - D_c is a nearest-neighbour block stencil on a periodic 4D lattice
 *     (Sec. 2.2, coarsest-level structure) with n = 2*n_tv variables per site:
 *       (D psi)_x = A_x psi_x + i*mu*Gamma5 psi_x
 *                 + sum_mu B[x,mu] psi_{x+mu} + sum_mu Gamma5 B[x-mu,mu]^H Gamma5 psi_{x-mu},
 *     Gamma5 = diag(+1 (n_tv times), -1 (n_tv times)), mu the twisted mass
 *     (Sec. 2.1, twisted-mass operator).
 *   - the solver is restarted GMRES (Sec. 3.1) with optional block-Jacobi left
 *     preconditioning (Sec. 3.2), GMRES-polynomial right preconditioning from
 *     Leja-ordered harmonic Ritz values (Sec. 3.3, Alg. 2, Alg. 3), and GCRO-DR
 *     deflated restarts with recycling across right-hand sides (Sec. 3.4),
 *     rebuilt lazily after the matrix changes (Sec. 3.6).
 *
 * Conventions for every entry point:
 *   - Complex numbers are interleaved (re, im).  "complex128" = 2 doubles,
 *     "complex64" = 2 floats.
 *   - Lattice sites are numbered x = x0 + L0*(x1 + L1*(x2 + L2*x3)); direction
 *     mu = 0..3 moves x_mu by +1, periodically.
 *   - Vectors are [V][n] complex, site-major.  Blocks are [n][n] row-major
 *     (entry (i, j) at i*n + j; row i is the output variable).
 *   - Device pointers point to memory on the current HIP device; `stream` is a
 *     hipStream_t (NULL = the null stream).  All device work of a call is
 *     enqueued on that stream; calls that return host values synchronise it.
 *   - Return value: DC_OK (0), a positive status (result written, see below)
 *     or a negative error; nothing is thrown across the ABI.  After a negative
 *     return, dc_last_error() gives a message (thread-local).
 *   - Ownership: the library copies what it keeps.  A handle from
 *     build_coarse_op owns its device memory (allocated with hipMalloc at
 *     build time and on first use of a solver variant) and frees it in
 *     destroy_coarse_op; a handle from build_coarse_op_ws takes all of it from
 *     two caller-owned ranges (dc_workspace_bytes gives their sizes).
 *   - A handle is used by one host thread and one stream at a time.
 */
#ifndef DCSOLVE_H
#define DCSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dc_op_s* dc_op_t;

/* status codes: > 0 the best iterate is written and the stats are valid,
 * < 0 no result */
enum {
  DC_OK = 0,
  DC_NOT_CONVERGED = 1,   /* cap reached: best iterate written, stats valid   */
  DC_BREAKDOWN = 2,       /* stopped on h_{j+1,j} = 0 at the first step of a
                             cycle (Alg. 1: the Krylov space cannot grow) with
                             the tolerance not met; best iterate written      */
  DC_ERR_INVALID = -1,    /* bad argument (null pointer, size, option)        */
  DC_ERR_HIP = -2,        /* a HIP runtime call failed                        */
  DC_ERR_WORKSPACE = -3,  /* a caller-provided workspace is too small         */
  DC_ERR_STATE = -4,      /* handle state does not allow the call             */
  DC_ERR_NOMEM = -5       /* device allocation failed                         */
};

/* block storage precisions kept by a handle (bit mask); FP64 is always kept */
enum { DC_STORE_F64 = 1, DC_STORE_F32 = 2, DC_STORE_F16S = 4 };

/* arithmetic of a Krylov solve / apply:
 *  F64  : FP64 blocks and vectors
 *  F32  : FP32 blocks and vectors, dot products accumulated in FP64
 *  F16S : FP16 blocks with one FP32 scale per block, FP32 vectors */
enum { DC_PREC_F64 = 0, DC_PREC_F32 = 1, DC_PREC_F16S = 2 };

/* where caller-supplied block arrays live */
enum { DC_WHERE_HOST = 0, DC_WHERE_DEVICE = 1 };

typedef struct {
  int32_t dims[4];  /* L0..L3 >= 1                                              */
  int32_t n_tv;     /* 1..32: n = 2*n_tv variables per site                     */
  int32_t store;    /* DC_STORE_* mask; F64 is added if missing                 */
  int32_t where;    /* DC_WHERE_HOST or DC_WHERE_DEVICE                         */
  double mu;        /* twisted mass (0 = clover-Wilson)                         */
} dc_op_desc;

typedef struct {
  int32_t m;            /* basis vectors per cycle: GMRES(m), GCRO-DR(m, k)     */
  int32_t k;            /* recycled vectors (0 = plain restarted GMRES)         */
  int32_t d;            /* polynomial: number of harmonic Ritz values (<=1 off) */
  int32_t u;            /* recycle-space refreshes before it is frozen          */
  int32_t max_cycles;   /* cap on restart cycles of one (inner) solve           */
  int32_t block_jacobi; /* 1: left block-Jacobi preconditioner (Sec. 3.2)       */
  int32_t prec;         /* DC_PREC_* of the Krylov solve                        */
  int32_t outer;        /* 1: FP64 flexible GMRES outer loop around the solve   */
  int32_t m_outer;      /* outer basis size                                     */
  int32_t max_outer;    /* cap on outer iterations                              */
  double inner_tol;     /* relative residual asked of each inner solve          */
  uint64_t seed;        /* seed of the polynomial's random start vector         */
  const void* v0;       /* optional start vector of the polynomial construction,
                           device complex128 [V][n] ([V/2][n] with schur);
                           NULL = seeded Gaussian                               */
  int32_t schur;        /* 1: solve the odd-even reduced system (Sec. 2.2):
                           S = D_ee - D_eo D_oo^{-1} D_oe on the even sites in
                           factored form, then x_o = D_oo^{-1}(b_o - D_oe x_e);
                           needs every extent even, excludes the batched
                           solves.  With block_jacobi the left preconditioner
                           is B = D_ee (Sec. 3.2: the even sites' self
                           blocks) and the polynomial is built from B^{-1} S
                           (Sec. 3.3).  b, x stay full-lattice; the
                           polynomial, recycle space and Arnoldi vectors of a
                           reduced variant are even-site compressed [V/2][n]
                           (site x at row x / 2).                               */
  int32_t ortho;        /* Arnoldi orthogonalisation of the single-RHS solves:
                           0 classical Gram-Schmidt applied twice; 1 the
                           single-sync process of Sec. 3.5 (one pass whose
                           reduction also yields ||A v_j||^2, h_{j+1,j}^2 =
                           ||A v_j||^2 - sum |h|^2, normalisation fused into
                           the update; less stable on long cycles, breakdown
                           when that difference is not positive).  The
                           batched solves take 0 only.                          */
  const void* x_ref;    /* optional reference solutions, device complex128
                           [n_rhs][V][n]: each solve then reports
                           ||x - x_ref|| / ||x_ref|| (FP64) in err_vs_ref;
                           NULL = none                                          */
  int32_t graphs;       /* 1: Arnoldi cycles that the host enqueues in one piece
                           (lattices small enough that launch overhead, not
                           HBM, bounds a step) are recorded once as HIP graphs
                           and replayed, one graph launch per cycle; same
                           kernels and results as 0 (eager launches).  Not used
                           while dc_profile_apply is recording.                */
} dc_solve_opts;

typedef struct {
  int32_t status;       /* DC_OK / DC_NOT_CONVERGED                              */
  int32_t cycles;       /* restart cycles (inner cycles when an outer loop runs)  */
  int32_t iters;        /* Arnoldi steps                                          */
  int32_t matvecs;      /* applications of D_c (any precision)                    */
  int32_t outer_iters;  /* flexible-GMRES outer iterations (0 without one)        */
  int32_t rebuilt;      /* bit 0: polynomial rebuilt, bit 1: recycle space built  */
  double rel_res_true;  /* ||b - D_c x|| / ||b|| computed in FP64 at the end      */
  double rel_res_est;   /* last least-squares residual estimate (relative)        */
  double t_setup_ms;    /* polynomial / recycle construction time in this call    */
  double t_solve_ms;    /* wall time of the call                                  */
  double err_vs_ref;    /* ||x - x_ref|| / ||x_ref|| if opts->x_ref, else -1      */
  int32_t breakdowns;   /* Arnoldi cycles that ended on h_{j+1,j} = 0 (Alg. 1's
                           happy breakdown: the least-squares solution is exact
                           in the space built so far)                             */
  int32_t refresh_failed; /* recycle refreshes whose dense generalised eigen-
                           problem failed; the space is then kept as it is and
                           frozen (no further refreshes)                          */
  int32_t stagnated;    /* 1 if the solve stopped because its FP64 residual had
                           not fallen below 0.9 of its best over three outer
                           refinement steps (solve_coarse_block)                  */
} dc_solve_stats;

/* Fill `o` with defaults: m=30, k=0, d=0, u=10, max_cycles=100000,
 * block_jacobi=0, prec=F64, outer=0, m_outer=10, max_outer=50,
 * inner_tol=1e-4, seed=0, v0=NULL, schur=0, ortho=0, x_ref=NULL, graphs=0. */
int dc_default_opts(dc_solve_opts* o);

/* Device memory a handle needs when the caller provides it (build_coarse_op_ws):
 *   *persistent_bytes: what the handle keeps for its lifetime -- the blocks
 *     in every stored precision (desc->store), FP16 scales, neighbour and
 *     parity tables, the self-block inverses that block Jacobi (Sec. 3.2) and
 *     the odd-even reduction (Sec. 2.2) use, and the recycle spaces U, C and
 *     q(A~) U of GCRO-DR (Sec. 3.4) for the variants `opts` selects (both
 *     signs of mu when mu != 0, so that adjoint solves fit too);
 *   *scratch_bytes: everything else -- apply partials, Krylov bases,
 *     polynomial chains, outer-loop vectors and residual temporaries of the
 *     single-right-hand-side calls (applies, dc_poly_*, dc_arnoldi with at
 *     most opts->m steps, solve_coarse / solve_coarse_adjoint) with these
 *     options, and dc_apply_multi with up to max_rhs right-hand sides.
 * Both are upper bounds for those calls; other options may need more (the
 * call then returns DC_ERR_WORKSPACE).  Pure host computation: no device is
 * touched.  DC_ERR_INVALID for bad descriptors or options. */
int dc_workspace_bytes(const dc_op_desc* desc, const dc_solve_opts* opts, int32_t max_rhs,
                       size_t* persistent_bytes, size_t* scratch_bytes);

/* build_coarse_op on caller-owned device memory: the handle carves every
 * device buffer it uses from the two ranges (first fit, 256-byte aligned) and
 * calls no hipMalloc of its own, so memory can come from a framework's
 * allocator (e.g. two torch uint8 CUDA tensors).  persistent_ws must stay
 * valid, and untouched by the caller, until destroy_coarse_op; scratch_ws
 * likewise (the handle keeps its Krylov workspaces there between calls).
 * Sizes come from dc_workspace_bytes.  Returns DC_ERR_WORKSPACE, before any
 * device work, if either range cannot hold what the build itself needs, and
 * from any later call whose buffers do not fit.  The batched and block
 * solvers (solve_coarse_batch, solve_coarse_multi, solve_coarse_block) are
 * not available on such a handle (DC_ERR_STATE).  Other arguments and errors
 * as build_coarse_op. */
int build_coarse_op_ws(const dc_op_desc* desc, const void* self_blocks, const void* hop_blocks,
                       void* persistent_ws, size_t persistent_bytes, void* scratch_ws,
                       size_t scratch_bytes, void* stream, dc_op_t* out);

/* Peak bytes a handle built by build_coarse_op_ws has used of each range so
 * far.  DC_ERR_STATE for a handle that allocates its own memory. */
int dc_workspace_used(dc_op_t op, size_t* persistent_peak, size_t* scratch_peak);

/* Arnoldi-cycle graphs of a handle (opts.graphs = 1): how many were captured
 * and how many graph launches replayed them.  Either pointer may be NULL. */
int dc_graph_stats(dc_op_t op, int64_t* captured, int64_t* launched);

/* Process-wide count of device allocations (hipMalloc) the library has made,
 * and the bytes they hold now (handles built on caller workspaces add
 * nothing).  Either pointer may be NULL. */
int dc_device_allocations(int64_t* count, int64_t* bytes_held);

/* Build a handle for D_c (Sec. 2.2; twisted mass Sec. 2.1).
 *   self_blocks: complex128 [V][n][n], the self couplings A_x (without the
 *                twisted-mass term, which the library adds from desc->mu);
 *   hop_blocks : complex128 [V][4][n][n], B[x,mu] coupling x to x+mu; the
 *                coupling of x+mu back to x is Gamma5 B[x,mu]^H Gamma5.
 * Both on host or device as desc->where says; they are copied (re-laid out,
 * and converted to the stored precisions), so the caller may free them once
 * the stream has synchronised.  Errors: DC_ERR_INVALID for null pointers,
 * dims < 1, n_tv outside 1..32; DC_ERR_NOMEM; DC_ERR_HIP. */
int build_coarse_op(const dc_op_desc* desc, const void* self_blocks,
                    const void* hop_blocks, void* stream, dc_op_t* out);

/* Replace the blocks (same layout and sizes as build_coarse_op) and mark the
 * block-Jacobi inverse, the polynomial and the recycle space stale, so that
 * the next solve rebuilds them in that order (Sec. 3.6). */
int update_coarse_op(dc_op_t op, const void* self_blocks, const void* hop_blocks,
                     void* stream);

/* Free everything the handle owns (synchronises its last stream). */
void destroy_coarse_op(dc_op_t op);

/* out = D_c in (adjoint = 0) or D_c^H in (adjoint = 1) with the blocks of
 * precision `prec`; in/out device [V][n], complex128 for DC_PREC_F64 and
 * complex64 otherwise; in and out must not overlap.  The adjoint uses
 * D^H = Gamma5 D(-mu) Gamma5.  DC_ERR_INVALID if the precision is not stored. */
int dc_apply(dc_op_t op, int32_t prec, int32_t adjoint, const void* in, void* out,
             void* stream);

/* The odd-even reduced operator (Sec. 2.2, factored form):
 * out = (D_ee - D_eo D_oo^{-1} D_oe) in (adjoint = 1: its adjoint, through
 * Gamma5 with -mu) on compressed even-site vectors, device [V/2][n] (site x at
 * row x / 2; complex128 for DC_PREC_F64, complex64 otherwise), in and out must
 * not overlap.  D_oo^{-1} are the odd sites' self-block inverses in the same
 * precision (built on first use).  DC_ERR_INVALID if an extent is odd or the
 * precision is not stored. */
int dc_apply_reduced(dc_op_t op, int32_t prec, int32_t adjoint, const void* in, void* out,
                     void* stream);

/* dc_apply_reduced for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * result, always through the two-kernel form of dc_set_reduced_kernels (equal
 * bit for bit to the other), with the odd-row temporary t_o = D_oo^{-1} D_oe in kept
 * in a fixed device array of the library (64 MiB per GPU, held until the
 * process ends) instead of the handle's memory.  It calls no allocating
 * routine at all, so:
 *   - V/2 * n * (16 for DC_PREC_F64, else 8) bytes must fit 64 MiB
 *     (DC_ERR_INVALID otherwise; e.g. 16^3 x 32 sites with n = 48 fit in FP64);
 *   - the odd self-block inverses for this adjoint flag must already exist:
 *     call dc_apply_reduced (or a reduced solve) once first after building or
 *     updating the handle (DC_ERR_STATE otherwise).
 * Every call on one GPU shares the array: calls that overlap in time on the
 * same GPU (different streams or threads) race and give wrong results; calls
 * in one stream are ordered and safe.  Arguments as dc_apply_reduced. */
int dc_apply_reduced_noalloc(dc_op_t op, int32_t prec, int32_t adjoint, const void* in,
                             void* out, void* stream);

/* The reduced operator with the left block-Jacobi preconditioner of Sec. 3.2,
 * which for the reduced system takes B = D_ee, the even sites' self blocks
 * (A_x + i mu Gamma5; not the block diagonal of S, a choice the paper makes
 * knowingly): out = D_ee^{-1} (D_ee - D_eo D_oo^{-1} D_oe) in
 *                 = in - D_ee^{-1} D_eo D_oo^{-1} D_oe in,
 * vectors as in dc_apply_reduced.  The self-block inverses of every site are
 * built on first use (DC_ERR_STATE if one is singular).  DC_ERR_INVALID as for
 * dc_apply_reduced. */
int dc_apply_reduced_bj(dc_op_t op, int32_t prec, const void* in, void* out, void* stream);

/* Multi-right-hand-side apply (MFMA): out_r = D_c in_r (adjoint = 0) or
 * D_c^H in_r (adjoint = 1) for r < n_rhs; in, out device [n_rhs][V][n],
 * complex128 for DC_PREC_F64 (FP64 MFMA) and complex64 otherwise (FP32 MFMA;
 * FP16 blocks are widened to FP32 on chip).  Each block times an n x n_rhs
 * panel is a dense complex contraction (the same operator as dc_apply, one
 * launch for all right-hand sides).  in and out must not overlap. */
int dc_apply_multi(dc_op_t op, int32_t prec, int32_t adjoint, int32_t n_rhs, const void* in,
                   void* out, void* stream);

/* out = B^{-1} in with B the block diagonal of the self couplings A_x + i mu
 * Gamma5 (Sec. 3.2); complex128 device vectors. Builds the inverses if stale. */
int dc_apply_block_jacobi(dc_op_t op, const void* in, void* out, void* stream);

/* Build (or rebuild) the preconditioning polynomial of `opts` (Alg. 3, first
 * three steps): opts->d Arnoldi steps of the (block-Jacobi preconditioned)
 * operator in precision opts->prec from opts->v0 (or a seeded Gaussian),
 * harmonic Ritz values, Leja order (Alg. 2).  theta_out (host, may be NULL)
 * receives 2*d doubles (re, im) in Leja order; *d_used the number kept (fewer
 * than d after an early breakdown). */
int dc_poly_setup(dc_op_t op, const dc_solve_opts* opts, void* stream,
                  double* theta_out, int32_t* d_used);

/* Install the polynomial q of Sec. 3.3 from caller-given roots theta (host,
 * 2*d doubles re, im; d == opts->d) for (opts->prec, opts->block_jacobi,
 * opts->schur) instead of building it: the chain uses them in the given order
 * (Leja order, Alg. 2, for stability), e.g. roots computed once for several
 * handles of the same operator.  It applies to D_c's own variant (adjoint
 * solves with mu != 0 keep building theirs).  A recycle space of that variant
 * built with another polynomial is dropped.  DC_ERR_INVALID for d != opts->d
 * or a zero or non-finite root. */
int dc_poly_set(dc_op_t op, const dc_solve_opts* opts, const double* theta, int32_t d);

/* out = q(A~) in with the polynomial built for (opts->prec, opts->block_jacobi)
 * (Sec. 3.3, Newton-like form, d-1 applications); vectors as in dc_apply. */
int dc_poly_apply(dc_op_t op, const dc_solve_opts* opts, const void* in, void* out,
                  void* stream);

/* Run `steps` Arnoldi steps (Alg. 1, classical Gram-Schmidt applied twice) of
 * the operator selected by opts (precision, block Jacobi, polynomial if
 * opts->d > 1) from the device vector v (complex128 [V][n], normalised
 * inside).  hbar_out (host) receives the (steps+1) x steps Hessenberg matrix,
 * column-major complex128; *steps_done the steps completed before a breakdown. */
int dc_arnoldi(dc_op_t op, const dc_solve_opts* opts, const void* v, int32_t steps,
               void* stream, double* hbar_out, int32_t* steps_done);

/* Solve D_c x_r = b_r for r < n_rhs to true relative residual tol[r]
 * (||b - D_c x|| / ||b|| in FP64).  b, x: device complex128 [n_rhs][V][n];
 * tol: host [n_rhs]; use_x0 = 1 takes x as the initial guess, else x0 = 0;
 * stats: host [n_rhs] or NULL.  The right-hand sides are solved one after
 * another and share the polynomial and the recycle space (Sec. 3.4: recycling
 * across right-hand sides).  Returns DC_OK if every solve converged, else
 * DC_NOT_CONVERGED with the best iterates written. */
int solve_coarse(dc_op_t op, const dc_solve_opts* opts, int32_t n_rhs, const void* b,
                 void* x, const double* tol, int32_t use_x0, void* stream,
                 dc_solve_stats* stats);

/* Same for D_c^H x = b, through Gamma5: D(mu)^H = Gamma5 D(-mu) Gamma5, so
 * x = Gamma5 solve(D(-mu), Gamma5 b).  For mu = 0 this reuses the polynomial
 * and recycle space of solve_coarse; for mu != 0 the D(-mu) variant keeps its
 * own, built on first use. */
int solve_coarse_adjoint(dc_op_t op, const dc_solve_opts* opts, int32_t n_rhs,
                         const void* b, void* x, const double* tol, int32_t use_x0,
                         void* stream, dc_solve_stats* stats);

/* Batched solve: the n_rhs systems D_c x_r = b_r (adjoint = 1: D_c^H x_r = b_r)
 * advance in lockstep, each with its own Krylov space, and share one MFMA
 * multi-right-hand-side apply per step (dc_apply_multi); per-right-hand-side
 * tolerances tol[r]; converged right-hand sides leave the active set at cycle
 * ends.  Restarted GMRES(m) with the polynomial of opts->d and block Jacobi of
 * opts->block_jacobi (Sec. 3.1-3.3); if opts->k > 0 and a recycle space was
 * built by solve_coarse for the same variant, every cycle is deflated against
 * it (Sec. 3.4), without refreshing it.  With opts->prec F32/F16S the batch is
 * the inner solve of an FP64 iterative-refinement loop (x += ||r|| solve(r/||r||)
 * to opts->inner_tol, at most opts->max_outer times).  b, x, tol, stats as in
 * solve_coarse.  Returns DC_OK if all converged, else DC_NOT_CONVERGED. */
int solve_coarse_batch(dc_op_t op, const dc_solve_opts* opts, int32_t adjoint, int32_t n_rhs,
                       const void* b, void* x, const double* tol, int32_t use_x0, void* stream,
                       dc_solve_stats* stats);

/* Block GMRES over n_rhs right-hand sides with one shared Krylov space (the
 * batching configuration's block GMRES; solve_coarse_batch keeps a space per
 * right-hand side).  Each restart cycle builds block Arnoldi vectors from the
 * block of current residuals of the columns not yet converged (block
 * classical Gram-Schmidt twice, Cholesky QR twice of each new block), with
 * the polynomial of opts->d as right preconditioner on every block and the
 * MFMA multi-right-hand-side apply (dc_apply_multi) as block matvec; every
 * column takes its minimal-residual correction in the whole block space and
 * leaves the block when its true residual meets tol[r].  A cycle ends after
 * opts->m block steps, when all columns' least-squares residuals meet their
 * targets, or when a new block is rank deficient.  Numerically dependent
 * residual columns: the space grows from a well-conditioned subset of them
 * (pivoted Cholesky of their scaled Gram matrix) and every column takes its
 * minimiser over it.  With opts->k > 0 the solve recycles (Sec. 3.4, in
 * block form): if the variant (prec, d, full lattice) holds no recycle space
 * of dimension k, the first cycle with at least k basis vectors builds one
 * from the k harmonic Ritz vectors of its block Arnoldi relation with the
 * smallest |theta|; the following cycles are deflated against it (new
 * residual blocks start with x += q(A) U C^H r, r -= C C^H r, the block
 * Arnoldi runs on (I - C C^H) A, each column's correction has the recycled
 * part -q(A) U B_k y) and refresh it from the relation
 * A q(A) [U D, V] = [C, V'] G until it has been updated opts->u times.  The
 * space is the one solve_coarse uses for the same variant (either solver
 * continues what the other built).  A cycle that ends on a rank-deficient
 * block leaves the space unchanged; a failed dense eigenproblem freezes it and
 * counts in stats.refresh_failed.  Full lattice, no block Jacobi (schur,
 * block_jacobi must be 0).
 * opts->prec F64: the block solve in FP64; F32 / F16S: an FP64
 * iterative-refinement loop (r = b - D x in FP64, block solve of D e = r to
 * opts->inner_tol per column in the reduced precision, x += e; at most
 * opts->max_outer times).  b, x: device complex128 [n_rhs][V][n]; use_x0 = 1
 * starts from the x passed in (the solve is then D e = b - D x to
 * tol ||b|| / ||b - D x|| and x += e, so a solve can be continued), else from
 * zero; tol host [n_rhs]; stats host [n_rhs] or
 * NULL (iters: block steps the column took part in; matvecs: single-vector
 * applications divided by n_rhs).  Device memory: about (2 m + 7) n_rhs
 * vectors of the precision.  Returns DC_OK if all converged, else
 * DC_NOT_CONVERGED; DC_ERR_INVALID for bad options or tolerances. */
int solve_coarse_block(dc_op_t op, const dc_solve_opts* opts, int32_t n_rhs, const void* b,
                       void* x, const double* tol, int32_t use_x0, void* stream,
                       dc_solve_stats* stats);

/* Mixed batch of lattices: the batched solve of solve_coarse_batch over
 * n_ops operators at once (every operator with the same n = 2 n_tv and the
 * precision opts->prec stored; no operator twice).  Operator o solves n_rhs[o]
 * systems: b[o], x[o] device complex128 [n_rhs[o]][V_o][n], tol[o] host
 * [n_rhs[o]], stats[o] host [n_rhs[o]] (NULL entries allowed).  Each step
 * runs one multi-right-hand-side apply launch over a work list of the sites of
 * every operator (up to 8 operators per launch); polynomial, block Jacobi and
 * frozen recycle space are each operator's own.  Returns DC_OK if every
 * system converged, else DC_NOT_CONVERGED; DC_ERR_INVALID for mismatched n,
 * repeated or null handles, or bad tolerances. */
int solve_coarse_multi(const dc_op_t* ops, int32_t n_ops, const dc_solve_opts* opts,
                       int32_t adjoint, const int32_t* n_rhs, const void* const* b,
                       void* const* x, const double* const* tol, int32_t use_x0, void* stream,
                       dc_solve_stats* const* stats);

/* Gradient of a real loss with respect to the hop blocks, given lambda =
 * D^{-H} dL/dx and x (device complex128 [V][n]).
 *   tied = 0: grad device complex128 [V][8][n][n]; direction mu < 4 is the
 *             coupling x -> x+mu: -lambda_x x_{x+mu}^H; direction 4+mu the
 *             coupling x -> x-mu: -lambda_x x_{x-mu}^H.
 *   tied = 1: grad device complex128 [V][4][n][n] w.r.t. B[x,mu] whose
 *             backward coupling is Gamma5 B^H Gamma5:
 *             -lambda_x x_{x+mu}^H - Gamma5 x_x lambda_{x+mu}^H Gamma5.
 * (grad = dL/dRe + i dL/dIm of each entry.) */
int dc_grad_hops(dc_op_t op, const void* lambda, const void* x, void* grad,
                 int32_t tied, void* stream);

/* Neighbour table used by the kernels, copied to host int32 [8][V]:
 * rows 0..3 = x + mu, rows 4..7 = x - mu. */
int dc_neighbours(dc_op_t op, int32_t* out);

/* FP16 block codes and scales in the input layout (for checking the
 * quantisation): codes host uint16 [V][5][n][n][2] (re, im bit patterns;
 * block 0 = A_x, 1 + mu = B[x,mu]), scales host float [V][5].
 * DC_ERR_INVALID if FP16 storage was not requested. */
int dc_export_f16(dc_op_t op, uint16_t* codes, float* scales);

/* Copy the current recycle space of the solver variant (opts->prec,
 * opts->block_jacobi, opts->d, adjoint) to device complex128 [k][V][n]
 * arrays U and C with k = opts->k (either may be NULL); *k_out = its
 * dimension (<= opts->k; 0 if the variant holds no space built for this k
 * and the current operator). */
int dc_export_recycle(dc_op_t op, const dc_solve_opts* opts, int32_t adjoint,
                      void* U, void* C, int32_t* k_out, void* stream);

/* Timing of the kernels that stream the stored blocks (diagnostics, not part
 * of the method): the full lattice's block kernel and the two kernels of the
 * odd-even reduced operator (Sec. 2.2).  every >= 1 clears the totals and has
 * one in `every` later dispatches of each of these kernels record a start and
 * an end HIP event on their launch stream (events passed to
 * hipExtLaunchKernel); every = 0 stops recording; every < 0 is
 * DC_ERR_INVALID.  Launches that a finished Arnoldi cycle turned into no-ops
 * are counted separately. */
int dc_profile_apply(dc_op_t op, int32_t every);

/* Totals since the last dc_profile_apply for the blocks used in precision
 * prec (DC_PREC_F64 / DC_PREC_F32 / DC_PREC_F16S) and kernel 0 (the full
 * lattice's block kernel), 1 (the reduced operator's t_o = A_o^{-1} D_oe x_e
 * kernel) or 2 (its A_e x_e - D_eo t_o kernel with the chain epilogue): *launches = launches that did work, *total_ms = their summed
 * event-to-event duration; *launches_all, *total_ms_all = the same over every
 * recorded launch, no-op launches of finished cycles included (what a kernel
 * tracer sees).  Any output pointer may be NULL.  Waits for the recorded events
 * to complete. */
int dc_profile_apply_read(dc_op_t op, int32_t prec, int32_t kernel, int64_t* launches,
                          double* total_ms, int64_t* launches_all, double* total_ms_all);

/* Vector passes of the launches that dc_profile_apply_read counts as having
 * done work (same prec and kernel): per launch, the distinct vectors it reads
 * plus the vectors it writes, each spanning the kernel's rows (V for kernel 0,
 * V/2 for kernels 1 and 2).  Kernel 0: 1 (its input); kernel 1: 2 (x_e,
 * t_o); kernel 2: 2-5 by epilogue.  Together with the blocks a launch streams
 * this gives the algorithmic bytes of the timed launches.  passes may be NULL. */
int dc_profile_apply_passes(dc_op_t op, int32_t prec, int32_t kernel, int64_t* passes);

/* Right-hand-side tile (right-hand sides per workgroup: 16, 32 or 64) of the
 * multi-right-hand-side apply.  The first launch of a shape class (block size
 * n, precision, n_rhs bucket <=16 / <=32 / <=64 / more, floor(log2(sites)))
 * times the candidate tiles on its operands with HIP events and keeps the
 * fastest for the process.  dc_multi_tile returns the tile chosen for a shape
 * (0 if not tuned yet); dc_set_multi_tile_mode(0) returns to autotuning and
 * forgets the table, 16 / 32 / 64 forces that tile (FP64 uses 32 for 64);
 * other values are DC_ERR_INVALID.  Results do not depend on the tile (same arithmetic per
 * output entry). */
int dc_multi_tile(int32_t prec, int32_t n, int32_t n_rhs, int32_t sites);
int dc_set_multi_tile_mode(int32_t mode);

/* Kernel form of the reduced operator S = D_ee - D_eo D_oo^{-1} D_oe (Sec. 2.2,
 * factored form) in dc_apply_reduced, dc_apply_reduced_bj and the reduced
 * solves; process-wide.  mode 0 (default): for FP32 and FP16 blocks with n a
 * multiple of 8 (n <= 64), one kernel over the odd rows reads every hop block
 * once, forms D_oo^{-1} D_oe in and from the same read the D_eo products, and a
 * second kernel sums those per even row (ten blocks read per even/odd site
 * pair); FP64 and other n use the two-kernel form.  mode 1: always the
 * two-kernel form (each kernel reads the hop blocks of its rows: eighteen
 * blocks per pair).  The two forms add the same terms in the same order, so
 * results are equal bit for bit.  Other values: DC_ERR_INVALID.  Set it while
 * no call of the library runs on another thread. */
int dc_set_reduced_kernels(int32_t mode);

/* Launches of the lockstep batched solves (solve_coarse_batch,
 * solve_coarse_multi): batched = 1 (default) takes every pass of one Arnoldi
 * step's classical Gram-Schmidt (applied twice) for up to 16 columns with the
 * same deflation-space size in one launch, and each polynomial chain step
 * (Sec. 3.3) of up to 8 operators in one launch; batched = 0 launches them per
 * column and per operator.  Each column's sums are the same either way, so
 * results are equal bit for bit; the batched form removes most launches of a
 * step on lattices small enough that launches, not HBM, bound it.
 * Process-wide; set it while no call of the library runs on another thread.
 * Other values: DC_ERR_INVALID. */
int dc_set_batch_launches(int32_t batched);

/* Message of the last error on this thread ("" if none). */
const char* dc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DCSOLVE_H */
