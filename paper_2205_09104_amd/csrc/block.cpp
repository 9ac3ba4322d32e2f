// Block GMRES over many right-hand sides of one operator with one shared
// Krylov space (the batching configuration's block GMRES; the lockstep batched
// solver keeps one space per right-hand side).  The block matvec is the MFMA
// multi-right-hand-side apply, the polynomial preconditioner of Sec. 3.3 runs
// on whole blocks, block Gram-Schmidt (classical, twice) and the Cholesky QR
// of each new block are tall-skinny complex products on MFMA tiles (the block
// Gram and block update kernels), and the block
// Hessenberg matrix is reduced by Householder transformations on the host as
// it grows, which gives every column's least-squares residual after every
// block step.  Reduced-precision blocks (FP32, FP16 + scale) run inside an
// FP64 iterative-refinement loop.  With k > 0 the solver deflates against the
// variant's recycle space and builds and refreshes it from its own block
// cycles (the GCRO-DR update with the block Arnoldi relation).
#include "solver.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <vector>

namespace dc {
namespace {

// Cholesky factor of a Hermitian r x r matrix after diagonal scaling:
// G = D Gs D with D = diag(sqrt(G_ii)), Gs = L L^H; returns R = L^H D (upper,
// G = R^H R) or false when a pivot of Gs falls to rel_pivot (a rank-deficient
// block: its columns span fewer than r directions).
bool scaled_cholesky(const Mat& G, double rel_pivot, Mat& R) {
  const int r = G.r;
  std::vector<double> d(r);
  for (int i = 0; i < r; ++i) {
    const double g = G(i, i).real();
    if (!(g > 0.0)) return false;
    d[i] = std::sqrt(g);
  }
  Mat L(r, r);
  for (int j = 0; j < r; ++j) {
    cd s = G(j, j) / (d[j] * d[j]);
    for (int k = 0; k < j; ++k) s -= L(j, k) * std::conj(L(j, k));
    if (!(s.real() > rel_pivot)) return false;
    const double ljj = std::sqrt(s.real());
    L(j, j) = ljj;
    for (int i = j + 1; i < r; ++i) {
      cd t = G(i, j) / (d[i] * d[j]);
      for (int k = 0; k < j; ++k) t -= L(i, k) * std::conj(L(j, k));
      L(i, j) = t / ljj;
    }
  }
  R = Mat(r, r);
  for (int i = 0; i < r; ++i)
    for (int j = i; j < r; ++j) R(i, j) = std::conj(L(j, i)) * d[j];
  return true;
}

// Householder reduction of a (2r x r) block to upper-triangular form:
// returns Q^H (2r x 2r) with Q^H A = [R; 0]; A is overwritten with [R; 0].
Mat householder_qh(Mat& A) {
  const int m = A.r, n = A.c;
  Mat QH = Mat::eye(m);
  std::vector<cd> v(m);
  for (int k = 0; k < n; ++k) {
    double nx = 0.0;
    for (int i = k; i < m; ++i) nx += std::norm(A(i, k));
    nx = std::sqrt(nx);
    if (nx == 0.0) continue;
    const cd x0 = A(k, k);
    const cd ph = (std::abs(x0) > 0.0) ? x0 / std::abs(x0) : cd(1.0);
    const cd alpha = -ph * nx;
    for (int i = k; i < m; ++i) v[i] = A(i, k);
    v[k] -= alpha;
    double nv = 0.0;
    for (int i = k; i < m; ++i) nv += std::norm(v[i]);
    nv = std::sqrt(nv);
    if (nv == 0.0) continue;
    for (int i = k; i < m; ++i) v[i] /= nv;
    // A <- (I - 2 v v^H) A on rows k.., QH likewise
    for (int j = k; j < n; ++j) {
      cd s(0.0);
      for (int i = k; i < m; ++i) s += std::conj(v[i]) * A(i, j);
      for (int i = k; i < m; ++i) A(i, j) -= 2.0 * v[i] * s;
    }
    for (int j = 0; j < m; ++j) {
      cd s(0.0);
      for (int i = k; i < m; ++i) s += std::conj(v[i]) * QH(i, j);
      for (int i = k; i < m; ++i) QH(i, j) -= 2.0 * v[i] * s;
    }
    for (int i = k + 1; i < m; ++i) A(i, k) = 0.0;
  }
  return QH;
}

template <typename VR>
struct BlockGmres {
  using Z = cx<VR>;
  Op& op;
  Variant& var;
  const SolveOpts& o;
  Prec p;
  hipStream_t st;
  size_t N;
  int m, Rmax;
  Z *V = nullptr, *Zb = nullptr, *W = nullptr, *T1 = nullptr, *TA = nullptr, *PROD = nullptr,
    *U = nullptr;
  Z *Hd = nullptr, *Gd = nullptr, *Rd = nullptr, *Yd = nullptr;
  Z* Pt = nullptr;      // per-chunk partial Gram products
  z64* Sum = nullptr;   // their FP64 sum
  void** tabs = nullptr;
  long applies = 0;   // operator applications to single vectors
  int refreshes = 0, refresh_failed = 0;   // recycle builds / refreshes, failed ones
  // frozen recycle space of the single-RHS solver's variant (GCRO-DR, Sec. 3.4):
  // the cycles run on (I - C C^H) A; kc = 0 without one
  int kc = 0;
  const Z *Cr = nullptr, *Ur = nullptr, *MUr = nullptr;
  Z* Bd = nullptr;   // device C^H W, kc x r

  // apply_only: just the multi-apply (and its pointer tables), no Krylov workspace
  BlockGmres(Op& op_, Variant& v, const SolveOpts& o_, Prec p_, int R, hipStream_t st_,
             bool apply_only = false)
      : op(op_), var(v), o(o_), p(p_), st(st_), N(op_.N()), m(std::max(o_.m, 1)), Rmax(R) {
    const size_t vb = N * sizeof(Z) * size_t(R);
    const bool poly = has_poly();
    Op::BlockWS& b = (sizeof(VR) == 8) ? op.bk64 : op.bk32;
    b.tab.ensure(size_t(8) * R * sizeof(void*));
    tabs = b.tab.as<void*>();
    b.small.ensure(std::max<size_t>(size_t(R), 32) * sizeof(double));
    Gd = b.small.as<Z>();
    if (apply_only) return;
    b.V.ensure(vb * size_t(m + 1));
    if (poly) b.Z.ensure(vb * size_t(m));
    b.W.ensure(vb);
    b.T1.ensure(vb);
    b.TA.ensure(vb);
    b.PROD.ensure(vb);
    b.U.ensure(vb);
    const size_t ns = size_t(m + 1) * R * R + 2 * size_t(R) * R + size_t(m) * R * R;
    const int kmax = std::max(o.k, 0);
    const size_t qrmax = std::max(size_t(m + 1) * R * R, size_t(kmax) * R);
    b.small.ensure(ns * sizeof(Z));
    // the Gram kernel's chunk partials (the most chunks a product takes is
    // that of a single output tile) or the multidot path's FP64 results, then
    // the FP64 sum
    const size_t pbytes = std::max(size_t(block_gram_parts(N, 1, 1)) * qrmax * sizeof(Z),
                                   qrmax * 2 * sizeof(double));
    b.part.ensure(pbytes + qrmax * sizeof(z64));
    V = b.V.as<Z>();
    Zb = poly ? b.Z.as<Z>() : nullptr;
    W = b.W.as<Z>();
    T1 = b.T1.as<Z>();
    TA = b.TA.as<Z>();
    PROD = b.PROD.as<Z>();
    U = b.U.as<Z>();
    Hd = b.small.as<Z>();
    Gd = Hd + size_t(m + 1) * R * R;
    Rd = Gd + size_t(R) * R;
    Yd = Rd + size_t(R) * R;
    Pt = b.part.as<Z>();
    Sum = reinterpret_cast<z64*>(b.part.as<unsigned char>() + pbytes);
    if (o.k > 0) {
      b.Bc.ensure(2 * size_t(o.k) * R * sizeof(Z));
      Bd = b.Bc.as<Z>();
    }
    if (o.k > 0 && v.kcur > 0 && v.recycle_version == op.version && v.k_built == o.k) {
      kc = v.kcur;
      Cr = v.C.as<Z>();
      Ur = v.U.as<Z>();
      MUr = (v.mu_ok && poly) ? v.MU.as<Z>() : nullptr;
    }
  }

  // X[cols] += q(A) U c for the columns' coefficients c (kc x r, device,
  // leading dimension kc): through MU = q(A) U when it is kept, else by
  // applying the polynomial to U c
  void add_recycled(const Z* cdev, int r, const std::vector<Z*>& xcols) {
    if (has_poly() && !MUr) {
      update(Ur, kc, cdev, U, r, 1.0, 0.0);
      Q(U, W, r);
      for (int a = 0; a < r; ++a) launch_axpy(p, mk(1.0, 0.0), W + size_t(a) * N, xcols[a], N, st);
      return;
    }
    update(has_poly() ? MUr : Ur, kc, cdev, U, r, 1.0, 0.0);
    for (int a = 0; a < r; ++a) launch_axpy(p, mk(1.0, 0.0), U + size_t(a) * N, xcols[a], N, st);
  }

  // ||x_a||^2 for r contiguous vectors, read to the host
  std::vector<double> colnorms(const Z* x, int r) {
    std::vector<double> out(r);
    double* d = reinterpret_cast<double*>(Gd);   // >= max(R, 32) doubles
    for (int c0 = 0; c0 < r; c0 += 32) {
      const int k = std::min(32, r - c0);
      launch_colnorm2(p, x + size_t(c0) * N, k, N, op.red(), d, st);
      op.hs.read(out.data() + c0, d, sizeof(double) * size_t(k), st);
      op.hs.wait(st);
    }
    return out;
  }

  bool has_poly() const { return var.d > 1 && int(var.theta.size()) > 1; }

  // out[a] = D in[a] for a < r (one multi-right-hand-side launch)
  void apply(const std::vector<const Z*>& in, const std::vector<Z*>& out) {
    const int r = int(in.size());
    std::vector<void*> t(2 * size_t(r));
    for (int a = 0; a < r; ++a) {
      t[a] = const_cast<Z*>(in[a]);
      t[r + a] = out[a];
    }
    op.hs.write(tabs, t.data(), t.size() * sizeof(void*), st);
    MultiOpDesc e{};
    e.blocks = op.blocks(p);
    e.scales = op.scales(p);
    e.nbr = op.nbr.as<int>();
    e.xin = const_cast<const void* const*>(tabs);
    e.yout = tabs + r;
    e.V = op.V;
    e.R = r;
    e.tm = op.mu;
    launch_apply_multi_ops(p, op.n, &e, 1, 0, st);
    applies += r;
  }
  std::vector<const Z*> cols(const Z* base, int r) const {
    std::vector<const Z*> v(r);
    for (int a = 0; a < r; ++a) v[a] = base + size_t(a) * N;
    return v;
  }
  std::vector<Z*> cols(Z* base, int r) const {
    std::vector<Z*> v(r);
    for (int a = 0; a < r; ++a) v[a] = base + size_t(a) * N;
    return v;
  }
  void apply_block(const Z* in, Z* out, int r) { apply(cols(in, r), cols(out, r)); }

  // out = q(A) in on a block of r vectors (Newton-like chain, d - 1 applies);
  // the chain updates are elementwise, so the block is one vector of r N entries
  void Q(const Z* in, Z* out, int r) {
    auto inv = [](cd t) { const cd q = 1.0 / t; return mk(q.real(), q.imag()); };
    const auto& th = var.theta;
    const int d = int(th.size());
    const size_t L = size_t(r) * N;
    const void* tt = TA;
    const void* vv = in;
    void* pp = PROD;
    void* yy = out;
    void** ct = tabs + 2 * size_t(Rmax);   // four one-entry tables after the apply tables
    void* h4[4] = {const_cast<void*>(tt), const_cast<void*>(vv), pp, yy};
    op.hs.write(ct, h4, sizeof(h4), st);
    apply_block(in, TA, r);
    launch_chain_multi(p, const_cast<const void* const*>(ct), const_cast<const void* const*>(ct + 1),
                       ct + 2, ct + 3, 1, L, inv(th[0]), inv(th[0]), inv(th[1]), 1, st);
    for (int i = 2; i < d; ++i) {
      apply_block(PROD, TA, r);
      launch_chain_multi(p, const_cast<const void* const*>(ct), nullptr, ct + 2, ct + 3, 1, L,
                         mk(0.0, 0.0), inv(th[i - 1]), inv(th[i]), 0, st);
    }
  }

  // C = be C + al A S (A: kk vectors, S: kk x nn on the device, C: nn vectors)
  void update(const Z* A, int kk, const Z* S, Z* C, int nn, cd al, cd be) {
    launch_block_update(p, A, kk, S, C, nn, N, mk(al.real(), al.imag()), mk(be.real(), be.imag()),
                        st);
  }

  // A^H B for qa contiguous vectors A and rb contiguous vectors B, read to the
  // host.  The block Gram kernel splits the inner dimension N into row chunks
  // (one output tile has too little work to spread over the chip) and sums
  // the chunks' partial products in FP64.  Narrow blocks (rb <= 16) take one
  // multidot launch per column of B instead (grid-wide partials, FP64
  // accumulation throughout).
  Mat tn(const Z* A, int qa, const Z* B, int rb) {
    if (rb <= 16) {
      double* dd = reinterpret_cast<double*>(Pt);
      for (int b = 0; b < rb; ++b)
        launch_multidot(p, A, qa, nullptr, 0, N, B + size_t(b) * N, 0, op.red(),
                        dd + 2 * size_t(qa) * b, nullptr, st);
      std::vector<double> hb(2 * size_t(qa) * rb);
      op.hs.read(hb.data(), dd, hb.size() * sizeof(double), st);
      op.hs.wait(st);
      Mat M(qa, rb);
      for (int b = 0; b < rb; ++b)
        for (int i = 0; i < qa; ++i)
          M(i, b) = cd(hb[2 * (size_t(b) * qa + i)], hb[2 * (size_t(b) * qa + i) + 1]);
      return M;
    }
    const size_t qr = size_t(qa) * rb;
    launch_block_gram(p, A, qa, B, rb, N, Pt, Sum, st);
    std::vector<z64> hbuf(qr);
    op.hs.read(hbuf.data(), Sum, qr * sizeof(z64), st);
    op.hs.wait(st);
    Mat M(qa, rb);
    for (int b = 0; b < rb; ++b)
      for (int i = 0; i < qa; ++i) {
        const z64 z = hbuf[size_t(b) * qa + i];
        M(i, b) = cd(z.re, z.im);
      }
    return M;
  }

  Mat read_mat(const Z* d, int rows, int colsn) {
    std::vector<Z> hbuf(size_t(rows) * colsn);
    op.hs.read(hbuf.data(), d, hbuf.size() * sizeof(Z), st);
    op.hs.wait(st);
    Mat M(rows, colsn);
    for (int j = 0; j < colsn; ++j)
      for (int i = 0; i < rows; ++i) {
        const Z z = hbuf[size_t(j) * rows + i];
        M(i, j) = cd(double(z.re), double(z.im));
      }
    return M;
  }
  void write_mat(Z* d, const Mat& M) {
    std::vector<Z> hbuf(size_t(M.r) * M.c);
    for (int j = 0; j < M.c; ++j)
      for (int i = 0; i < M.r; ++i) {
        const cd z = M(i, j);
        hbuf[size_t(j) * M.r + i] = mk(VR(z.real()), VR(z.imag()));
      }
    op.hs.write(d, hbuf.data(), hbuf.size() * sizeof(Z), st);
  }

  // Cholesky QR, twice: dst = src R^{-1} with src = dst R; false on rank deficiency
  bool cholqr2(Z* src, Z* dst, int r, Mat& Rtot) {
    const double piv = (sizeof(VR) == 8) ? 1e-24 : 1e-10;
    Rtot = Mat::eye(r);
    Z* a = src;
    Z* b = T1;
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1) {
        a = T1;
        b = dst;
      }
      const Mat G = tn(a, r, a, r);
      Mat R;
      if (!scaled_cholesky(G, piv, R)) return false;
      write_mat(Rd, tri_inverse(R));
      update(a, r, Rd, b, r, 1.0, 0.0);
      Rtot = matmul(R, Rtot);
    }
    return true;
  }

  // Residual columns R (nr of them, in V) that are numerically dependent: the
  // block that generates the Krylov space is the orthonormalised subset of
  // columns picked by a pivoted Cholesky factorisation of their scaled Gram
  // matrix (each pick keeps at least sel_piv of its squared norm outside the
  // span of the earlier picks).  On return V holds that basis V_0 (the count is
  // returned), S0 = V_0^H R (nb x nr) and drop[a] = ||R_a - V_0 S0_a||; R is
  // kept in U.  0 if not even the first pick orthonormalises.
  // Greedy pivoted Cholesky of the scaled Gram matrix G of nr columns: each
  // pick has the largest squared part outside the span of the earlier picks
  // (the lowest index among equal ones), kept while that part exceeds sel_piv.
  std::vector<int> pivot_picks(int nr, const Mat& G) const {
    std::vector<double> d(nr);
    for (int i = 0; i < nr; ++i) d[i] = std::sqrt(std::max(G(i, i).real(), 0.0));
    // pivoted Cholesky of Gs = D^{-1} G D^{-1}: Schur-complement diagonal
    const double sel_piv = (sizeof(VR) == 8) ? 1e-12 : 1e-6;
    std::vector<double> rest(nr);
    for (int i = 0; i < nr; ++i) rest[i] = d[i] > 0.0 ? 1.0 : 0.0;
    Mat L(nr, nr);
    std::vector<int> pick;
    for (int k = 0; k < nr; ++k) {
      int best = -1;
      for (int i = 0; i < nr; ++i)
        if (std::find(pick.begin(), pick.end(), i) == pick.end() &&
            (best < 0 || rest[i] > rest[best]))
          best = i;
      if (best < 0 || !(rest[best] > sel_piv)) break;
      const double lkk = std::sqrt(rest[best]);
      for (int i = 0; i < nr; ++i) {
        if (std::find(pick.begin(), pick.end(), i) != pick.end() || i == best) continue;
        if (!(d[i] > 0.0)) continue;
        cd t = G(i, best) / (d[i] * d[best]);
        for (int q = 0; q < k; ++q) t -= L(i, q) * std::conj(L(best, q));
        L(i, k) = t / lkk;
        rest[i] -= std::norm(L(i, k));
      }
      L(best, k) = lkk;
      pick.push_back(best);
    }
    return pick;
  }

  int select_block(int nr, const Mat& G, const std::vector<int>& pick, Mat& S0,
                   std::vector<double>& drop) {
    const int nb = int(pick.size());
    if (nb == 0) return 0;
    DC_HIP(hipMemcpyAsync(U, V, size_t(nr) * N * sizeof(Z), hipMemcpyDeviceToDevice, st));
    for (int t = 0; t < nb; ++t)
      DC_HIP(hipMemcpyAsync(T1 + size_t(t) * N, U + size_t(pick[size_t(t)]) * N, N * sizeof(Z),
                            hipMemcpyDeviceToDevice, st));
    Mat Rsel;
    DC_HIP(hipMemcpyAsync(V, T1, size_t(nb) * N * sizeof(Z), hipMemcpyDeviceToDevice, st));
    if (!cholqr2(V, V, nb, Rsel)) return 0;
    S0 = tn(V, nb, U, nr);
    // drop[a] = ||R_a - V_0 S0_a||, formed explicitly (T1 = R - V_0 S0), not
    // by subtracting squared norms
    DC_HIP(hipMemcpyAsync(T1, U, size_t(nr) * N * sizeof(Z), hipMemcpyDeviceToDevice, st));
    write_mat(Rd, S0);
    update(V, nb, Rd, T1, nr, -1.0, 1.0);
    const std::vector<double> e2 = colnorms(T1, nr);
    drop.assign(nr, 0.0);
    for (int a = 0; a < nr; ++a) drop[a] = std::sqrt(std::max(e2[a], 0.0));
    return nb;
  }

  struct Cycle {
    int steps = 0;
    bool full = true;   // every block of the cycle had full rank
    Mat Y;          // (steps r) x r coefficients
    Mat Bk;         // kc x (m r): C^H A V of the deflated process
    Mat Hb;         // the block Hessenberg matrix before its reduction
    std::vector<double> est;
  };

  // One cycle from the orthonormal block V_0 (nr columns) for nc residual
  // columns R_0 = V_0 S0 + E (S0 nr x nc; E orthogonal to V_0, column norms
  // drop, zero when V_0 spans R_0); every column takes its least-squares
  // minimiser over the block space.  The cycle ends when every column's
  // residual is at or below its target, after m steps, or when a new block is
  // rank deficient.
  // Dependent columns (nr < nc, the residual columns kept in U): every block
  // V_{j+1} also takes the coefficients V_{j+1}^H R of the residual columns
  // into the least-squares right-hand side (their parts outside V_0 are not
  // orthogonal to the later blocks), and the cycle runs up to
  // m nc / nr block steps so that its space keeps the dimension m nc that
  // nc independent columns would give (bounded by the basis storage).
  Cycle cycle(int nr, int nc, const Mat& S0, const std::vector<double>& target,
              const std::vector<double>& drop) {
    Cycle c;
    const bool dep = nr < nc;
    const int msteps = dep ? std::max(m, std::min(m * nc / nr, (m + 1) * nc / nr - 1)) : m;
    c.Bk = Mat(std::max(kc, 1), msteps * nr);
    c.Hb = Mat((msteps + 1) * nr, msteps * nr);
    Mat Rf((msteps + 1) * nr, msteps * nr);
    Mat G((msteps + 1) * nr, nc);
    for (int j = 0; j < nc; ++j)
      for (int i = 0; i < nr; ++i) G(i, j) = S0(i, j);
    // squared parts of the residual columns outside the blocks so far
    std::vector<double> outside(nc);
    for (int a = 0; a < nc; ++a) outside[a] = drop[size_t(a)] * drop[size_t(a)];
    std::vector<Mat> qhs;
    c.est.assign(nc, 0.0);
    for (int a = 0; a < nc; ++a) {
      double s = outside[a];
      for (int i = 0; i < nr; ++i) s += std::norm(S0(i, a));
      c.est[a] = std::sqrt(s);
    }
    for (int j = 0; j < msteps; ++j) {
      Z* Vj = V + size_t(j) * nr * N;
      const Z* src = Vj;
      if (has_poly()) {
        Q(Vj, Zb + size_t(j) * nr * N, nr);
        src = Zb + size_t(j) * nr * N;
      }
      apply_block(src, W, nr);
      const int q = (j + 1) * nr;
      Mat hcol(q, nr);
      for (int pass = 0; pass < 2; ++pass) {
        if (kc) {   // deflation: W -= C (C^H W), coefficients B_k
          const Mat bp = tn(Cr, kc, W, nr);
          write_mat(Bd, bp);
          update(Cr, kc, Bd, W, nr, -1.0, 1.0);
          for (int b = 0; b < nr; ++b)
            for (int i = 0; i < kc; ++i) c.Bk(i, j * nr + b) += bp(i, b);
        }
        const Mat hp = tn(V, q, W, nr);
        write_mat(Hd, hp);
        update(V, q, Hd, W, nr, -1.0, 1.0);
        for (int b = 0; b < nr; ++b)
          for (int i = 0; i < q; ++i) hcol(i, b) += hp(i, b);
      }
      Mat Hsub;
      const bool full = cholqr2(W, V + size_t(j + 1) * nr * N, nr, Hsub);
      if (dep && full) {   // coefficients of the residual columns on the new block
        const Mat e = tn(V + size_t(j + 1) * nr * N, nr, U, nc);
        for (int a = 0; a < nc; ++a)
          for (int t = 0; t < nr; ++t) {
            G((j + 1) * nr + t, a) = e(t, a);
            outside[a] -= std::norm(e(t, a));
          }
      }
      // the new block column of Hbar, reduced by the earlier reflections
      Mat col((j + 2) * nr, nr);
      for (int b = 0; b < nr; ++b) {
        for (int i = 0; i < q; ++i) col(i, b) = hcol(i, b);
        for (int i = 0; i < nr; ++i) col(q + i, b) = full ? Hsub(i, b) : cd(0.0);
        for (int i = 0; i < q + nr; ++i) c.Hb(i, j * nr + b) = col(i, b);
      }
      c.full = full;
      for (int i = 0; i < j; ++i) {
        Mat sub(2 * nr, nr);
        for (int b = 0; b < nr; ++b)
          for (int t = 0; t < 2 * nr; ++t) sub(t, b) = col(i * nr + t, b);
        const Mat rs = matmul(qhs[size_t(i)], sub);
        for (int b = 0; b < nr; ++b)
          for (int t = 0; t < 2 * nr; ++t) col(i * nr + t, b) = rs(t, b);
      }
      Mat blk(2 * nr, nr);
      for (int b = 0; b < nr; ++b)
        for (int t = 0; t < 2 * nr; ++t) blk(t, b) = col(j * nr + t, b);
      const Mat qh = householder_qh(blk);
      for (int b = 0; b < nr; ++b) {
        for (int i = 0; i < j * nr; ++i) Rf(i, j * nr + b) = col(i, b);
        for (int t = 0; t < nr; ++t) Rf(j * nr + t, j * nr + b) = blk(t, b);
      }
      qhs.push_back(qh);
      {
        Mat gs(2 * nr, nc);
        for (int b = 0; b < nc; ++b)
          for (int t = 0; t < 2 * nr; ++t) gs(t, b) = G(j * nr + t, b);
        const Mat gr = matmul(qh, gs);
        for (int b = 0; b < nc; ++b)
          for (int t = 0; t < 2 * nr; ++t) G(j * nr + t, b) = gr(t, b);
      }
      c.steps = j + 1;
      bool done = true;
      for (int a = 0; a < nc; ++a) {
        double s = std::max(outside[a], 0.0);
        for (int t = 0; t < nr; ++t) s += std::norm(G((j + 1) * nr + t, a));
        c.est[a] = std::sqrt(s);
        if (c.est[a] > target[size_t(a)]) done = false;
      }
      if (done || !full) break;
    }
    // back substitution: Rf(0:s, 0:s) Y = G(0:s, :)
    const int s = c.steps * nr;
    c.Y = Mat(s, nc);
    for (int b = 0; b < nc; ++b)
      for (int i = s - 1; i >= 0; --i) {
        cd t = G(i, b);
        for (int k = i + 1; k < s; ++k) t -= Rf(i, k) * c.Y(k, b);
        c.Y(i, b) = (std::abs(Rf(i, i)) > 0.0) ? t / Rf(i, i) : cd(0.0);
      }
    return c;
  }

  // Build (no recycle space yet) or refresh (fewer than u updates so far) the
  // recycle space of the variant from a cycle's block relation
  // A M [U D, V_s] = [C, V_{s+nb}] G, D = diag(1 / ||u_i||),
  // G = [[D, B_k], [0, Hbar]] (G = Hbar without a space; the GCRO-DR update of
  // Sec. 3.4 with the block Arnoldi relation): the k harmonic Ritz vectors of
  // G^H G z = theta G^H (What^H Vhat) z with the smallest |theta|, P_k;
  // [Q, R] = qr(G P_k), C = What Q, U = Vhat P_k R^{-1}, and M U by the same
  // combination of the M V_j.  A cycle that ended on a rank-deficient block
  // leaves the space as it is.  Returns true if the space changed.
  bool recycle(const Cycle& c, int nb) {
    if (o.k <= 0 || !c.full || c.steps == 0) return false;
    const int s = c.steps * nb;
    const bool build = kc == 0;
    if (build ? s < o.k : var.updates >= o.u) return false;
    const int k0 = build ? 0 : kc, kk = build ? o.k : kc;
    const int nrow = k0 + s + nb, ncol = k0 + s;
    std::vector<double> un(size_t(k0), 1.0);
    if (!build) {
      const std::vector<double> u2 = colnorms(Ur, kc);
      for (int i = 0; i < kc; ++i) un[size_t(i)] = std::sqrt(std::max(u2[size_t(i)], 0.0));
    }
    Mat G(nrow, ncol), WV(nrow, ncol);
    for (int i = 0; i < k0; ++i) {
      G(i, i) = 1.0 / un[size_t(i)];
      for (int q = 0; q < s; ++q) G(i, k0 + q) = c.Bk(i, q);
    }
    for (int i = 0; i < s + nb; ++i)
      for (int q = 0; q < s; ++q) G(k0 + i, k0 + q) = c.Hb(i, q);
    for (int i = 0; i < s; ++i) WV(k0 + i, k0 + i) = 1.0;   // V_{s+nb}^H V_s
    if (!build) {   // C^H U D and V_{s+nb}^H U D
      const Mat CU = tn(Cr, kc, Ur, kc);
      const Mat VU = tn(V, s + nb, Ur, kc);
      for (int q = 0; q < kc; ++q) {
        for (int i = 0; i < kc; ++i) WV(i, q) = CU(i, q) / un[size_t(q)];
        for (int i = 0; i < s + nb; ++i) WV(kc + i, q) = VU(i, q) / un[size_t(q)];
      }
    }
    const Mat GH = adjoint(G);
    Mat Bm = matmul(GH, WV), Am = matmul(GH, G);
    std::vector<cd> th;
    Mat Zv;
    if (!lu_solve(Bm, Am) || !eig(Am, th, &Zv)) {   // Am <- Bm^{-1} Am
      var.updates = o.u;                            // frozen, as in the single solver
      ++refresh_failed;
      return false;
    }
    const auto idx = smallest_k(th, kk);
    Mat P(ncol, kk);
    for (int t = 0; t < kk; ++t)
      for (int i = 0; i < ncol; ++i) P(i, t) = Zv(i, idx[size_t(t)]);
    Mat Qm, Rq;
    qr_thin(matmul(G, P), Qm, Rq);
    const Mat PR = matmul(P, tri_inverse(Rq));
    // coefficients, output-major: C from [C, V_{s+nb}], U from [U, V_s] (D
    // folded in), M U from [M U, M V_s]
    std::vector<z64> cq(size_t(kk) * nrow), cu(size_t(kk) * ncol);
    for (int r = 0; r < kk; ++r) {
      for (int q = 0; q < nrow; ++q) cq[size_t(r) * nrow + q] = mk(Qm(q, r).real(), Qm(q, r).imag());
      for (int q = 0; q < ncol; ++q) {
        const cd v = q < k0 ? PR(q, r) / un[size_t(q)] : PR(q, r);
        cu[size_t(r) * ncol + q] = mk(v.real(), v.imag());
      }
    }
    Op::BlockWS& b = (sizeof(VR) == 8) ? op.bk64 : op.bk32;
    b.rcoef.ensure((cq.size() + cu.size()) * sizeof(z64));
    const bool mu = has_poly();
    const bool mu_old = mu && k0 && !MUr;   // M U of the old space to be formed
    b.rtmp.ensure(size_t(mu ? (mu_old ? 4 : 3) : 2) * kk * N * sizeof(Z));
    z64* dq = b.rcoef.as<z64>();
    z64* du = dq + cq.size();
    op.hs.write(dq, cq.data(), cq.size() * sizeof(z64), st);
    op.hs.write(du, cu.data(), cu.size() * sizeof(z64), st);
    Z* Cn = b.rtmp.as<Z>();
    Z* Un = Cn + size_t(kk) * N;
    Z* MUn = Un + size_t(kk) * N;
    const double* cqd = reinterpret_cast<const double*>(dq);
    const double* cud = reinterpret_cast<const double*>(du);
    launch_combine(p, k0 ? Cr : nullptr, k0, V, s + nb, N, cqd, kk, Cn, 0, st);
    launch_combine(p, k0 ? Ur : nullptr, k0, V, s, N, cud, kk, Un, 0, st);
    if (mu) {
      // M U: from the kept M U, else by applying M to the old U (once)
      const Z* mur = MUr;
      if (mu_old) {   // M applied to the old U, Rmax columns at a time
        Z* MUo = MUn + size_t(kk) * N;
        for (int c0 = 0; c0 < kc; c0 += Rmax) {
          const int r = std::min(Rmax, kc - c0);
          Q(Ur + size_t(c0) * N, W, r);
          DC_HIP(hipMemcpyAsync(MUo + size_t(c0) * N, W, size_t(r) * N * sizeof(Z),
                                hipMemcpyDeviceToDevice, st));
        }
        mur = MUo;
      }
      launch_combine(p, k0 ? mur : nullptr, k0, Zb, s, N, cud, kk, MUn, 0, st);
    }
    const size_t vb = N * sizeof(Z) * size_t(kk);
    var.U.ensure(vb);
    var.C.ensure(vb);
    if (mu) var.MU.ensure(vb);
    DC_HIP(hipMemcpyAsync(var.C.p, Cn, vb, hipMemcpyDeviceToDevice, st));
    DC_HIP(hipMemcpyAsync(var.U.p, Un, vb, hipMemcpyDeviceToDevice, st));
    if (mu) DC_HIP(hipMemcpyAsync(var.MU.p, MUn, vb, hipMemcpyDeviceToDevice, st));
    var.mu_ok = mu;
    var.kcur = kk;
    var.k_built = o.k;
    var.recycle_version = op.version;
    var.updates = build ? 1 : var.updates + 1;
    kc = kk;
    Cr = var.C.as<Z>();
    Ur = var.U.as<Z>();
    MUr = mu ? var.MU.as<Z>() : nullptr;
    const std::vector<double> u2 = colnorms(Ur, kc);
    var.unorm.assign(size_t(kc), 1.0);
    for (int i = 0; i < kc; ++i) var.unorm[size_t(i)] = std::sqrt(std::max(u2[size_t(i)], 0.0));
    ++refreshes;
    return true;
  }

  // Solve D X = B for R columns (this precision) to relative tolerances tol,
  // X starting at zero; per-column statistics accumulate into stats.
  void solve(const Z* B, Z* X, int R, const std::vector<double>& tol, int max_cycles,
             std::vector<SolveStats>& stats, std::vector<double>& rel) {
    launch_zero(p, X, size_t(R) * N, st);
    std::vector<double> bn = colnorms(B, R);
    for (double& x : bn) x = std::sqrt(std::max(x, 0.0));
    rel.assign(R, 0.0);
    std::vector<int> act;
    for (int c = 0; c < R; ++c)
      if (bn[c] > 0.0) act.push_back(c);
    bool first = true;
    for (int cyc = 0;; ++cyc) {
      const int r = int(act.size());
      if (r == 0) break;
      // residual block of the active columns in V_0
      if (first) {
        for (int a = 0; a < r; ++a)
          DC_HIP(hipMemcpyAsync(V + size_t(a) * N, B + size_t(act[a]) * N, N * sizeof(Z),
                                hipMemcpyDeviceToDevice, st));
      } else {
        std::vector<const Z*> in(r);
        for (int a = 0; a < r; ++a) in[a] = X + size_t(act[a]) * N;
        apply(in, cols(V, r));
        for (int a = 0; a < r; ++a) {
          Z* v = V + size_t(a) * N;
          launch_scale(p, v, v, N, nullptr, -1.0, nullptr, st);
          launch_axpy(p, mk(1.0, 0.0), B + size_t(act[a]) * N, v, N, st);
        }
      }
      first = false;
      const std::vector<double> rn = colnorms(V, r);
      std::vector<int> keep;
      for (int a = 0; a < r; ++a) {
        const int c = act[a];
        rel[c] = std::sqrt(std::max(rn[a], 0.0)) / bn[c];
        if (rel[c] > tol[c] && cyc < max_cycles) keep.push_back(a);
      }
      if (keep.empty()) break;
      // compact the residual block to the columns still active
      for (size_t t = 0; t < keep.size(); ++t)
        if (int(t) != keep[t])
          DC_HIP(hipMemcpyAsync(V + t * N, V + size_t(keep[t]) * N, N * sizeof(Z),
                                hipMemcpyDeviceToDevice, st));
      std::vector<int> act2(keep.size());
      for (size_t t = 0; t < keep.size(); ++t) act2[t] = act[size_t(keep[t])];
      act = act2;
      const int nr = int(act.size());
      if (kc) {   // new residuals with a recycle space: x += q(A) U C^H r; r -= C C^H r
        write_mat(Bd, tn(Cr, kc, V, nr));
        update(Cr, kc, Bd, V, nr, -1.0, 1.0);
        std::vector<Z*> xc(nr);
        for (int a = 0; a < nr; ++a) xc[a] = X + size_t(act[a]) * N;
        add_recycled(Bd, nr, xc);
      }
      // the block that generates the space: every residual column, or a
      // well-conditioned subset of them when they are numerically dependent
      Mat S0;
      std::vector<double> drop(nr, 0.0);
      int nb = nr;
      const Mat G0 = tn(V, nr, V, nr);
      const std::vector<int> picks = pivot_picks(nr, G0);
      if (int(picks.size()) < nr || !cholqr2(V, V, nr, S0)) {
        nb = select_block(nr, G0, picks.size() < size_t(nr) ? picks : pivot_picks(nr, G0), S0,
                          drop);
        if (nb == 0) break;
      }
      std::vector<double> target(nr);
      for (int a = 0; a < nr; ++a) target[a] = tol[act[a]] * bn[act[a]];
      const Cycle c = cycle(nb, nr, S0, target, drop);
      for (int a = 0; a < nr; ++a) {
        stats[act[a]].iters += c.steps;
        stats[act[a]].cycles += 1;
      }
      const int s = c.steps * nb;
      if (s == 0) break;
      write_mat(Yd, c.Y);
      update(has_poly() ? Zb : V, s, Yd, U, nr, 1.0, 0.0);
      std::vector<Z*> xc(nr);
      for (int a = 0; a < nr; ++a) {
        xc[a] = X + size_t(act[a]) * N;
        launch_axpy(p, mk(1.0, 0.0), U + size_t(a) * N, xc[a], N, st);
      }
      if (kc) {
        // the recycled part of the least-squares solution: the rows of C are met
        // exactly by -B_k y (the block form of the GCRO-DR problem)
        Mat By(kc, nr);
        for (int b = 0; b < nr; ++b)
          for (int i = 0; i < kc; ++i) {
            cd t(0.0);
            for (int q2 = 0; q2 < s; ++q2) t += c.Bk(i, q2) * c.Y(q2, b);
            By(i, b) = -t;
          }
        write_mat(Bd, By);
        add_recycled(Bd, nr, xc);
      }
      recycle(c, nb);
    }
  }
};

}  // namespace

int op_solve_block(Op& op, const SolveOpts& o, int R, const void* b, void* x, const double* tol,
                   int use_x0, hipStream_t st, SolveStats* stats) {
  if (op.caller_ws())
    throw BadState("block GMRES sizes its device buffers per call (the workspace query does "
                   "not cover them): not available on a handle built on caller workspaces");
  if (R < 1) throw InvalidArg("n_rhs must be >= 1");
  if (!b || !x || !tol) throw InvalidArg("null pointer");
  if (o.schur) throw InvalidArg("the block solver works on the full lattice (schur = 0)");
  if (o.block_jacobi) throw InvalidArg("the block solver has no block-Jacobi preconditioning");
  if (o.m < 1 || o.max_cycles < 0) throw InvalidArg("bad solver options");
  if (o.prec != P64 && (o.max_outer < 1 || !(o.inner_tol > 0.0)))
    throw InvalidArg("bad outer-loop options");
  check_prec(op, o.prec);
  for (int r = 0; r < R; ++r)
    if (!(tol[r] > 0.0)) throw InvalidArg("tolerances must be positive");
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<SolveStats> stt(R);
  Variant& var = op.variant(o.prec, +1, 0, o.d, 0);
  const auto ts = std::chrono::steady_clock::now();
  ensure_poly(op, var, o, st, &stt[0]);
  const double t_setup = ms_since(ts);
  const size_t N = op.N(), NR = N * size_t(R);
  const z64* B64 = static_cast<const z64*>(b);
  z64* X64 = static_cast<z64*>(x);
  std::vector<double> tl(tol, tol + R), rel(R, 0.0);
  long applies = 0;
  // FP64 applies and norms; in the FP64 path it is not used once the full
  // solver below has (re)sized the shared FP64 workspace
  BlockGmres<double> K64(op, var, o, P64, R, st, true);
  const std::vector<double> bn0 = K64.colnorms(B64, R);
  // With a start vector the solve is D e = b - D x0, to tol ||b|| / ||b - D x0||,
  // and x = x0 + e; its right-hand side is kept in bk64.E0, e in bk64.E.
  const z64* rhs = B64;
  z64* sol = X64;
  if (use_x0) {
    op.bk64.X0.ensure(NR * sizeof(z64));
    op.bk64.E0.ensure(NR * sizeof(z64));
    op.bk64.E.ensure(NR * sizeof(z64));
    z64* X0 = op.bk64.X0.as<z64>();
    z64* Rb = op.bk64.E0.as<z64>();
    DC_HIP(hipMemcpyAsync(X0, X64, NR * sizeof(z64), hipMemcpyDeviceToDevice, st));
    K64.apply(K64.cols(static_cast<const z64*>(X0), R), K64.cols(Rb, R));
    launch_scale(P64, Rb, Rb, NR, nullptr, -1.0, nullptr, st);
    launch_axpy(P64, mk(1.0, 0.0), B64, Rb, NR, st);
    const std::vector<double> rn2 = K64.colnorms(Rb, R);
    for (int c = 0; c < R; ++c) {
      const double rn = std::sqrt(std::max(rn2[c], 0.0)), bnc = std::sqrt(std::max(bn0[c], 0.0));
      tl[c] = rn > 0.0 ? tol[c] * bnc / rn : 1.0;
    }
    rhs = Rb;
    sol = op.bk64.E.as<z64>();
  }
  if (o.prec == P64) {
    BlockGmres<double> K(op, var, o, P64, R, st);
    K.solve(rhs, sol, R, tl, o.max_cycles, stt, rel);
    applies += K.applies;
    for (SolveStats& x : stt) x.refresh_failed += K.refresh_failed;
  } else {
    // FP64 iterative refinement: r = rhs - D sol in FP64, the block solve of
    // D e = r in the reduced precision to inner_tol, sol += e
    BlockGmres<float> K(op, var, o, o.prec, R, st);
    op.bk64.R.ensure(NR * sizeof(z64));
    op.bk32.R.ensure(N * sizeof(z32) * size_t(R));
    op.bk32.X.ensure(N * sizeof(z32) * size_t(R));
    z64* Rr = op.bk64.R.as<z64>();
    z32* Rin = op.bk32.R.as<z32>();
    z32* E = op.bk32.X.as<z32>();
    launch_zero(P64, sol, NR, st);
    std::vector<double> bn = K64.colnorms(rhs, R);
    for (double& v : bn) v = std::sqrt(std::max(v, 0.0));
    std::vector<int> act;
    for (int c = 0; c < R; ++c)
      if (bn[c] > 0.0) act.push_back(c);
    // a column whose FP64 residual has not fallen below 0.9 of its best for
    // three refinement steps in a row stops refining (stagnation)
    std::vector<double> best(R, std::numeric_limits<double>::infinity());
    std::vector<int> stall(R, 0);
    for (int outer = 0; !act.empty(); ++outer) {
      const int r = int(act.size());
      std::vector<const z64*> in(r);
      std::vector<z64*> out(r);
      for (int a = 0; a < r; ++a) {
        in[a] = sol + size_t(act[a]) * N;
        out[a] = Rr + size_t(a) * N;
      }
      K64.apply(in, out);
      for (int a = 0; a < r; ++a) {
        launch_scale(P64, out[a], out[a], N, nullptr, -1.0, nullptr, st);
        launch_axpy(P64, mk(1.0, 0.0), rhs + size_t(act[a]) * N, out[a], N, st);
      }
      const std::vector<double> rn = K64.colnorms(Rr, r);
      std::vector<int> keep;
      for (int a = 0; a < r; ++a) {
        const int c = act[a];
        rel[c] = std::sqrt(std::max(rn[a], 0.0)) / bn[c];
        if (rel[c] < 0.9 * best[c]) {
          best[c] = rel[c];
          stall[c] = 0;
        } else if (++stall[c] >= 3) {
          stt[c].stagnated = 1;
        }
        if (rel[c] > tl[c] && outer < o.max_outer && !stt[c].stagnated) keep.push_back(a);
      }
      if (keep.empty()) break;
      const int nr = int(keep.size());
      for (int t = 0; t < nr; ++t)
        launch_convert_64to32(Rr + size_t(keep[t]) * N, Rin + size_t(t) * N, N, op.n, 0, st);
      std::vector<double> itol(nr, o.inner_tol), irel;
      std::vector<SolveStats> ist(nr);
      K.solve(Rin, E, nr, itol, o.max_cycles, ist, irel);
      std::vector<int> act2(nr);
      for (int t = 0; t < nr; ++t) {
        const int c = act[size_t(keep[t])];
        act2[t] = c;
        stt[c].iters += ist[t].iters;
        stt[c].cycles += ist[t].cycles;
        stt[c].outer_iters += 1;
        // sol += e (through the FP64 residual buffer as staging)
        launch_convert_32to64(E + size_t(t) * N, Rr + size_t(t) * N, N, op.n, 0, st);
        launch_axpy(P64, mk(1.0, 0.0), Rr + size_t(t) * N, sol + size_t(c) * N, N, st);
      }
      act = act2;
    }
    applies += K.applies;
    for (SolveStats& x : stt) x.refresh_failed += K.refresh_failed;
  }
  applies += K64.applies;
  if (use_x0) {
    // x = x0 + e, and the residuals relative to b
    DC_HIP(hipMemcpyAsync(X64, op.bk64.X0.p, NR * sizeof(z64), hipMemcpyDeviceToDevice, st));
    launch_axpy(P64, mk(1.0, 0.0), sol, X64, NR, st);
    for (int c = 0; c < R; ++c) rel[c] = tl[c] > 0.0 ? rel[c] * tol[c] / tl[c] : rel[c];
  }
  int all_ok = 1;
  const double t_solve = ms_since(t0);
  for (int r = 0; r < R; ++r) {
    SolveStats& s = stt[r];
    s.rel_res_true = rel[r];
    s.status = rel[r] <= tol[r] * (1.0 + 1e-12) ? 0 : 1;
    if (s.status) all_ok = 0;
    s.matvecs = int(applies / R);
    s.t_setup_ms = t_setup;
    s.t_solve_ms = t_solve;
    if (stats) stats[r] = s;
  }
  return all_ok ? 0 : 1;
}

}  // namespace dc
