// extern "C" entry points (include/dcsolve.h, include/dcsolve_dense.h): argument
// checks, exception-to-status mapping, thread-local error messages.
#include <cstring>
#include <exception>
#include <memory>
#include <string>
#include <vector>

#include "../../include/dcsolve.h"
#include "../../include/dcsolve_dense.h"
#include "solver.hpp"

struct dc_op_s {
  dc::Op op;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

template <typename F>
int guarded(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const dc::InvalidArg& e) {
    return fail(DC_ERR_INVALID, e.what());
  } catch (const dc::NoMem& e) {
    return fail(DC_ERR_NOMEM, e.what());
  } catch (const dc::BadState& e) {
    return fail(DC_ERR_STATE, e.what());
  } catch (const dc::WorkspaceShort& e) {
    return fail(DC_ERR_WORKSPACE, e.what());
  } catch (const dc::HipError& e) {
    return fail(DC_ERR_HIP, e.what());
  } catch (const std::bad_alloc&) {
    return fail(DC_ERR_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(DC_ERR_INVALID, e.what());
  }
}

dc::SolveOpts convert(const dc_solve_opts* o) {
  dc::SolveOpts s;
  if (!o) return s;
  s.m = o->m;
  s.k = o->k;
  s.d = o->d;
  s.u = o->u;
  s.max_cycles = o->max_cycles;
  s.block_jacobi = o->block_jacobi;
  if (o->prec < 0 || o->prec > 2) throw dc::InvalidArg("unknown precision");
  s.prec = dc::Prec(o->prec);
  s.outer = o->outer;
  s.m_outer = o->m_outer;
  s.max_outer = o->max_outer;
  s.inner_tol = o->inner_tol;
  s.seed = o->seed;
  s.v0 = o->v0;
  s.x_ref = o->x_ref;
  if (o->graphs != 0 && o->graphs != 1) throw dc::InvalidArg("graphs must be 0 or 1");
  s.graphs = o->graphs;
  if (o->schur != 0 && o->schur != 1) throw dc::InvalidArg("schur must be 0 or 1");
  s.schur = o->schur;
  if (o->ortho != 0 && o->ortho != 1) throw dc::InvalidArg("ortho must be 0 or 1");
  s.ortho = o->ortho;
  return s;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

void copy_stats(const dc::SolveStats& a, dc_solve_stats* b) {
  b->status = a.status;
  b->cycles = a.cycles;
  b->iters = a.iters;
  b->matvecs = a.matvecs;
  b->outer_iters = a.outer_iters;
  b->rebuilt = a.rebuilt;
  b->rel_res_true = a.rel_res_true;
  b->rel_res_est = a.rel_res_est;
  b->t_setup_ms = a.t_setup_ms;
  b->t_solve_ms = a.t_solve_ms;
  b->err_vs_ref = a.err_vs_ref;
  b->breakdowns = a.breakdowns;
  b->refresh_failed = a.refresh_failed;
  b->stagnated = a.stagnated;
}

}  // namespace

extern "C" {

const char* dc_last_error(void) { return g_err.c_str(); }

int dc_default_opts(dc_solve_opts* o) {
  if (!o) return fail(DC_ERR_INVALID, "null options pointer");
  std::memset(o, 0, sizeof(*o));
  o->m = 30;
  o->k = 0;
  o->d = 0;
  o->u = 10;
  o->max_cycles = 100000;
  o->block_jacobi = 0;
  o->prec = DC_PREC_F64;
  o->outer = 0;
  o->m_outer = 10;
  o->max_outer = 50;
  o->inner_tol = 1e-4;
  o->seed = 0;
  o->v0 = nullptr;
  o->schur = 0;
  o->ortho = 0;
  o->x_ref = nullptr;
  o->graphs = 0;
  return DC_OK;
}

int dc_workspace_bytes(const dc_op_desc* desc, const dc_solve_opts* opts, int32_t max_rhs,
                       size_t* persistent_bytes, size_t* scratch_bytes) {
  return guarded([&] {
    if (!desc || !persistent_bytes || !scratch_bytes) throw dc::InvalidArg("null pointer");
    if (desc->where != DC_WHERE_HOST && desc->where != DC_WHERE_DEVICE)
      throw dc::InvalidArg("desc.where must be DC_WHERE_HOST or DC_WHERE_DEVICE");
    if (desc->store & ~7) throw dc::InvalidArg("unknown bits in desc.store");
    const dc::SolveOpts o = convert(opts);
    dc::workspace_bytes(desc->dims, desc->n_tv, desc->store, desc->mu,
                        desc->where == DC_WHERE_HOST, o, max_rhs, persistent_bytes,
                        scratch_bytes);
    return DC_OK;
  });
}

int build_coarse_op_ws(const dc_op_desc* desc, const void* self_blocks, const void* hop_blocks,
                       void* persistent_ws, size_t persistent_bytes, void* scratch_ws,
                       size_t scratch_bytes, void* stream, dc_op_t* out) {
  return guarded([&] {
    if (!desc || !out) throw dc::InvalidArg("null descriptor or output handle");
    *out = nullptr;
    if (!persistent_ws || !scratch_ws) throw dc::InvalidArg("null workspace pointer");
    if (desc->where != DC_WHERE_HOST && desc->where != DC_WHERE_DEVICE)
      throw dc::InvalidArg("desc.where must be DC_WHERE_HOST or DC_WHERE_DEVICE");
    if (desc->store & ~7) throw dc::InvalidArg("unknown bits in desc.store");
    // what the build itself takes, checked before any device work
    dc::SolveOpts o0;
    size_t p_all = 0, s_all = 0, p_build = 0, s_build = 0;
    dc::workspace_bytes(desc->dims, desc->n_tv, desc->store, desc->mu,
                        desc->where == DC_WHERE_HOST, o0, 0, &p_all, &s_all, &p_build, &s_build);
    // each arena loses up to one granule to aligning the caller's pointer
    const size_t g = dc::Arena::kArenaAlign;
    if (persistent_bytes < p_build + g || scratch_bytes < s_build + g)
      throw dc::WorkspaceShort("workspace too small to build the operator: persistent " +
                               std::to_string(persistent_bytes) + " < " +
                               std::to_string(p_build + g) + " or scratch " +
                               std::to_string(scratch_bytes) + " < " +
                               std::to_string(s_build + g) + " bytes");
    auto h = new dc_op_s;
    try {
      h->op.persist = std::make_unique<dc::Arena>(persistent_ws, persistent_bytes);
      h->op.scratch = std::make_unique<dc::Arena>(scratch_ws, scratch_bytes);
      h->op.bind_arenas();
      dc::op_build(h->op, desc->dims, desc->n_tv, desc->store, desc->mu, self_blocks, hop_blocks,
                   desc->where == DC_WHERE_DEVICE, as_stream(stream));
      dc::noalloc_scratch(true);   // set-up of dc_apply_reduced_noalloc on this device
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
    return DC_OK;
  });
}

int dc_graph_stats(dc_op_t op, int64_t* captured, int64_t* launched) {
  return guarded([&] {
    if (!op) throw dc::InvalidArg("null handle");
    if (captured) *captured = op->op.graphs.captured;
    if (launched) *launched = op->op.graphs.launched;
    return DC_OK;
  });
}

int dc_device_allocations(int64_t* count, int64_t* bytes_held) {
  if (count) *count = dc::device_allocations();
  if (bytes_held) *bytes_held = dc::device_bytes_held();
  return DC_OK;
}

int dc_workspace_used(dc_op_t op, size_t* persistent_peak, size_t* scratch_peak) {
  return guarded([&] {
    if (!op) throw dc::InvalidArg("null handle");
    if (!op->op.caller_ws()) throw dc::BadState("the handle was not built on caller workspaces");
    if (persistent_peak) *persistent_peak = op->op.persist->peak;
    if (scratch_peak) *scratch_peak = op->op.scratch->peak;
    return DC_OK;
  });
}

int build_coarse_op(const dc_op_desc* desc, const void* self_blocks, const void* hop_blocks,
                    void* stream, dc_op_t* out) {
  return guarded([&] {
    if (!desc || !out) throw dc::InvalidArg("null descriptor or output handle");
    *out = nullptr;
    if (desc->where != DC_WHERE_HOST && desc->where != DC_WHERE_DEVICE)
      throw dc::InvalidArg("desc.where must be DC_WHERE_HOST or DC_WHERE_DEVICE");
    if (desc->store & ~7) throw dc::InvalidArg("unknown bits in desc.store");
    auto h = new dc_op_s;
    try {
      dc::op_build(h->op, desc->dims, desc->n_tv, desc->store, desc->mu, self_blocks, hop_blocks,
                   desc->where == DC_WHERE_DEVICE, as_stream(stream));
      dc::noalloc_scratch(true);   // set-up of dc_apply_reduced_noalloc on this device
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
    return DC_OK;
  });
}

int update_coarse_op(dc_op_t op, const void* self_blocks, const void* hop_blocks, void* stream) {
  return guarded([&] {
    if (!op) throw dc::InvalidArg("null handle");
    // the same placement as at build time is required; detect device pointers
    hipPointerAttribute_t attr;
    bool on_dev = false;
    if (hipPointerGetAttributes(&attr, self_blocks) == hipSuccess)
      on_dev = (attr.type == hipMemoryTypeDevice);
    (void)hipGetLastError();
    dc::op_update(op->op, self_blocks, hop_blocks, on_dev, as_stream(stream));
    return DC_OK;
  });
}

void destroy_coarse_op(dc_op_t op) {
  if (!op) return;
  (void)hipDeviceSynchronize();
  delete op;
}

int dc_apply(dc_op_t op, int32_t prec, int32_t adjoint, const void* in, void* out, void* stream) {
  return guarded([&] {
    if (!op) throw dc::InvalidArg("null handle");
    if (prec < 0 || prec > 2) throw dc::InvalidArg("unknown precision");
    dc::op_apply(op->op, dc::Prec(prec), adjoint, in, out, as_stream(stream));
    return DC_OK;
  });
}

int dc_apply_reduced(dc_op_t op, int32_t prec, int32_t adjoint, const void* in, void* out,
                     void* stream) {
  return guarded([&] {
    if (!op) throw dc::InvalidArg("null handle");
    if (prec < 0 || prec > 2) throw dc::InvalidArg("unknown precision");
    dc::op_apply_reduced(op->op, dc::Prec(prec), adjoint, 0, in, out, as_stream(stream));
    return DC_OK;
  });
}

int dc_apply_reduced_noalloc(dc_op_t op, int32_t prec, int32_t adjoint, const void* in,
                             void* out, void* stream) {
  return guarded([&] {
    if (!op) throw dc::InvalidArg("null handle");
    if (prec < 0 || prec > 2) throw dc::InvalidArg("unknown precision");
    dc::op_apply_reduced_noalloc(op->op, dc::Prec(prec), adjoint, in, out, as_stream(stream));
    return DC_OK;
  });
}

int dc_apply_reduced_bj(dc_op_t op, int32_t prec, const void* in, void* out, void* stream) {
  return guarded([&] {
    if (!op) throw dc::InvalidArg("null handle");
    if (prec < 0 || prec > 2) throw dc::InvalidArg("unknown precision");
    dc::op_apply_reduced(op->op, dc::Prec(prec), 0, 1, in, out, as_stream(stream));
    return DC_OK;
  });
}

int dc_apply_multi(dc_op_t op, int32_t prec, int32_t adjoint, int32_t n_rhs, const void* in,
                   void* out, void* stream) {
  return guarded([&] {
    if (!op) throw dc::InvalidArg("null handle");
    if (prec < 0 || prec > 2) throw dc::InvalidArg("unknown precision");
    dc::op_apply_multi(op->op, dc::Prec(prec), adjoint, n_rhs, in, out, as_stream(stream));
    return DC_OK;
  });
}

int dc_apply_block_jacobi(dc_op_t op, const void* in, void* out, void* stream) {
  return guarded([&] {
    if (!op) throw dc::InvalidArg("null handle");
    dc::op_apply_bj(op->op, in, out, as_stream(stream));
    return DC_OK;
  });
}

int dc_poly_setup(dc_op_t op, const dc_solve_opts* opts, void* stream, double* theta_out,
                  int32_t* d_used) {
  return guarded([&] {
    if (!op || !opts) throw dc::InvalidArg("null handle or options");
    std::vector<dc::cd> th;
    const int d = dc::op_poly_setup(op->op, convert(opts), as_stream(stream), th);
    if (theta_out)
      for (int i = 0; i < d; ++i) {
        theta_out[2 * i] = th[i].real();
        theta_out[2 * i + 1] = th[i].imag();
      }
    if (d_used) *d_used = d;
    return DC_OK;
  });
}

int dc_poly_set(dc_op_t op, const dc_solve_opts* opts, const double* theta, int32_t d) {
  return guarded([&] {
    if (!op || !opts || !theta) throw dc::InvalidArg("null handle, options or roots");
    if (d < 1) throw dc::InvalidArg("d must be >= 1");
    std::vector<dc::cd> th(static_cast<size_t>(d));
    for (int i = 0; i < d; ++i) th[size_t(i)] = dc::cd(theta[2 * i], theta[2 * i + 1]);
    dc::op_poly_set(op->op, convert(opts), th);
    return DC_OK;
  });
}

int dc_poly_apply(dc_op_t op, const dc_solve_opts* opts, const void* in, void* out, void* stream) {
  return guarded([&] {
    if (!op || !opts) throw dc::InvalidArg("null handle or options");
    dc::op_poly_apply(op->op, convert(opts), in, out, as_stream(stream));
    return DC_OK;
  });
}

int dc_arnoldi(dc_op_t op, const dc_solve_opts* opts, const void* v, int32_t steps, void* stream,
               double* hbar_out, int32_t* steps_done) {
  return guarded([&] {
    if (!op || !opts || !hbar_out) throw dc::InvalidArg("null argument");
    std::vector<dc::cd> h;
    const int jd = dc::op_arnoldi(op->op, convert(opts), v, steps, as_stream(stream), h);
    for (size_t i = 0; i < h.size(); ++i) {
      hbar_out[2 * i] = h[i].real();
      hbar_out[2 * i + 1] = h[i].imag();
    }
    if (steps_done) *steps_done = jd;
    return DC_OK;
  });
}

static int solve_common(dc_op_t op, const dc_solve_opts* opts, int adjoint, int32_t n_rhs,
                        const void* b, void* x, const double* tol, int32_t use_x0, void* stream,
                        dc_solve_stats* stats) {
  return guarded([&] {
    if (!op || !opts) throw dc::InvalidArg("null handle or options");
    std::vector<dc::SolveStats> st(n_rhs > 0 ? n_rhs : 0);
    const int rc = dc::op_solve(op->op, convert(opts), adjoint, n_rhs, b, x, tol, use_x0,
                                as_stream(stream), st.data());
    if (stats)
      for (int r = 0; r < n_rhs; ++r) copy_stats(st[r], stats + r);
    return rc == 0 ? DC_OK : DC_NOT_CONVERGED;
  });
}

int solve_coarse(dc_op_t op, const dc_solve_opts* opts, int32_t n_rhs, const void* b, void* x,
                 const double* tol, int32_t use_x0, void* stream, dc_solve_stats* stats) {
  return solve_common(op, opts, 0, n_rhs, b, x, tol, use_x0, stream, stats);
}

int solve_coarse_adjoint(dc_op_t op, const dc_solve_opts* opts, int32_t n_rhs, const void* b,
                         void* x, const double* tol, int32_t use_x0, void* stream,
                         dc_solve_stats* stats) {
  return solve_common(op, opts, 1, n_rhs, b, x, tol, use_x0, stream, stats);
}

int solve_coarse_batch(dc_op_t op, const dc_solve_opts* opts, int32_t adjoint, int32_t n_rhs,
                       const void* b, void* x, const double* tol, int32_t use_x0, void* stream,
                       dc_solve_stats* stats) {
  return guarded([&] {
    if (!op || !opts) throw dc::InvalidArg("null handle or options");
    std::vector<dc::SolveStats> st(n_rhs > 0 ? n_rhs : 0);
    const int rc = dc::op_solve_batch(op->op, convert(opts), adjoint, n_rhs, b, x, tol, use_x0,
                                      as_stream(stream), st.data());
    if (stats)
      for (int r = 0; r < n_rhs; ++r) copy_stats(st[r], stats + r);
    return rc == 0 ? DC_OK : DC_NOT_CONVERGED;
  });
}

int solve_coarse_block(dc_op_t op, const dc_solve_opts* opts, int32_t n_rhs, const void* b,
                       void* x, const double* tol, int32_t use_x0, void* stream,
                       dc_solve_stats* stats) {
  return guarded([&] {
    if (!op || !opts) throw dc::InvalidArg("null handle or options");
    std::vector<dc::SolveStats> st(n_rhs > 0 ? n_rhs : 0);
    const int rc = dc::op_solve_block(op->op, convert(opts), n_rhs, b, x, tol, use_x0,
                                      as_stream(stream), st.data());
    if (stats)
      for (int r = 0; r < n_rhs; ++r) copy_stats(st[r], stats + r);
    return rc == 0 ? DC_OK : DC_NOT_CONVERGED;
  });
}

int solve_coarse_multi(const dc_op_t* ops, int32_t n_ops, const dc_solve_opts* opts,
                       int32_t adjoint, const int32_t* n_rhs, const void* const* b,
                       void* const* x, const double* const* tol, int32_t use_x0, void* stream,
                       dc_solve_stats* const* stats) {
  return guarded([&] {
    if (!ops || !opts || !n_rhs || !b || !x || !tol || n_ops < 1)
      throw dc::InvalidArg("null argument or n_ops < 1");
    std::vector<dc::Op*> o(n_ops);
    std::vector<int> R(n_ops);
    std::vector<const void*> bb(n_ops);
    std::vector<void*> xx(n_ops);
    std::vector<const double*> tt(n_ops);
    std::vector<std::vector<dc::SolveStats>> st(n_ops);
    std::vector<dc::SolveStats*> sp(n_ops);
    for (int i = 0; i < n_ops; ++i) {
      if (!ops[i]) throw dc::InvalidArg("null operator handle");
      o[i] = &ops[i]->op;
      R[i] = n_rhs[i];
      if (R[i] < 0) throw dc::InvalidArg("negative n_rhs");
      bb[i] = b[i];
      xx[i] = x[i];
      tt[i] = tol[i];
      st[i].resize(R[i]);
      sp[i] = st[i].data();
    }
    const int rc = dc::op_solve_multi(o, convert(opts), adjoint, R, bb, xx, tt, use_x0,
                                      as_stream(stream), sp);
    if (stats)
      for (int i = 0; i < n_ops; ++i)
        if (stats[i])
          for (int r = 0; r < R[i]; ++r) copy_stats(st[i][r], stats[i] + r);
    return rc == 0 ? DC_OK : DC_NOT_CONVERGED;
  });
}

int dc_grad_hops(dc_op_t op, const void* lambda, const void* x, void* grad, int32_t tied,
                 void* stream) {
  return guarded([&] {
    if (!op || !lambda || !x || !grad) throw dc::InvalidArg("null argument");
    dc::launch_grad_hops(static_cast<const dc::z64*>(lambda), static_cast<const dc::z64*>(x),
                         static_cast<dc::z64*>(grad), op->op.nbr.as<int>(), op->op.V, op->op.n,
                         tied ? 1 : 0, as_stream(stream));
    return DC_OK;
  });
}

int dc_neighbours(dc_op_t op, int32_t* out) {
  return guarded([&] {
    if (!op || !out) throw dc::InvalidArg("null argument");
    DC_HIP(hipMemcpy(out, op->op.nbr.p, size_t(8) * op->op.V * sizeof(int), hipMemcpyDeviceToHost));
    return DC_OK;
  });
}

int dc_export_f16(dc_op_t op, uint16_t* codes, float* scales) {
  return guarded([&] {
    if (!op || !codes || !scales) throw dc::InvalidArg("null argument");
    const dc::Op& o = op->op;
    if (!(o.store & DC_STORE_F16S)) throw dc::InvalidArg("FP16 storage was not requested");
    const int n = o.n, T = dc::tile_T(n);
    const int tt16 = dc::tile_elems(n, 4);
    const size_t nb = size_t(o.V) * 5;
    std::vector<uint32_t> tiled(nb * tt16 * 64);
    DC_HIP(hipMemcpy(tiled.data(), o.blk16.p, tiled.size() * 4, hipMemcpyDeviceToHost));
    DC_HIP(hipMemcpy(scales, o.sc16.p, nb * sizeof(float), hipMemcpyDeviceToHost));
    for (size_t blk = 0; blk < nb; ++blk)
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < T * T; ++e) {
          const int i = (lane >> 3) * T + e / T, j = (lane & 7) * T + e % T;
          if (i >= n || j >= n) continue;
          const uint32_t w = tiled[blk * tt16 * 64 + (size_t(e >> 2) * 64 + lane) * 4 + (e & 3)];
          uint16_t* dst = codes + ((blk * n + i) * n + j) * 2;
          dst[0] = uint16_t(w & 0xffffu);
          dst[1] = uint16_t(w >> 16);
        }
    return DC_OK;
  });
}

int dc_export_recycle(dc_op_t op, const dc_solve_opts* opts, int32_t adjoint, void* U, void* C,
                      int32_t* k_out, void* stream) {
  return guarded([&] {
    if (!op || !opts) throw dc::InvalidArg("null handle or options");
    const int k = dc::op_export_recycle(op->op, convert(opts), adjoint, U, C, as_stream(stream));
    if (k_out) *k_out = k;
    return DC_OK;
  });
}

int dc_multi_tile(int32_t prec, int32_t n, int32_t n_rhs, int32_t sites) {
  if (prec < 0 || prec > 2 || n < 1 || n_rhs < 1 || sites < 1) return 0;
  return dc::multi_tile_for(dc::Prec(prec), n, n_rhs, unsigned(sites));
}

int dc_set_multi_tile_mode(int32_t mode) {
  return guarded([&] {
    dc::set_multi_tile_mode(mode);
    return DC_OK;
  });
}

int dc_set_batch_launches(int32_t batched) {
  return guarded([&] {
    dc::set_batch_launches(batched);
    return DC_OK;
  });
}

int dc_set_reduced_kernels(int32_t mode) {
  return guarded([&] {
    dc::set_reduced_mode(mode);
    return DC_OK;
  });
}

int dc_profile_apply(dc_op_t op, int32_t every) {
  return guarded([&] {
    if (!op) throw dc::InvalidArg("null handle");
    dc::op_profile(op->op, every);
    return DC_OK;
  });
}

int dc_profile_apply_read(dc_op_t op, int32_t prec, int32_t kernel, int64_t* launches,
                          double* total_ms, int64_t* launches_all, double* total_ms_all) {
  return guarded([&] {
    if (!op) throw dc::InvalidArg("null handle");
    if (prec < 0 || prec > 2) throw dc::InvalidArg("unknown precision");
    long n = 0, na = 0;
    double ms = 0.0, msa = 0.0;
    dc::op_profile_read(op->op, dc::Prec(prec), kernel, &n, &ms, nullptr, &na, &msa);
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    if (launches_all) *launches_all = na;
    if (total_ms_all) *total_ms_all = msa;
    return DC_OK;
  });
}

int dc_profile_apply_passes(dc_op_t op, int32_t prec, int32_t kernel, int64_t* passes) {
  return guarded([&] {
    if (!op) throw dc::InvalidArg("null handle");
    if (prec < 0 || prec > 2) throw dc::InvalidArg("unknown precision");
    long v = 0;
    dc::op_profile_read(op->op, dc::Prec(prec), kernel, nullptr, nullptr, &v, nullptr, nullptr);
    if (passes) *passes = v;
    return DC_OK;
  });
}

// ------------------------------------------------------------------ dense (host only)

static dc::Mat read_mat(int r, int c, const double* a) {
  dc::Mat m(r, c);
  for (size_t i = 0; i < size_t(r) * c; ++i) m.a[i] = dc::cd(a[2 * i], a[2 * i + 1]);
  return m;
}

int dc_dense_eig(int32_t n, const double* A, double* w, double* Z) {
  return guarded([&] {
    if (n < 0 || !A || !w) throw dc::InvalidArg("bad arguments");
    std::vector<dc::cd> ev;
    dc::Mat Zm;
    if (!dc::eig(read_mat(n, n, A), ev, Z ? &Zm : nullptr))
      throw dc::InvalidArg("QR iteration did not converge");
    for (int i = 0; i < n; ++i) {
      w[2 * i] = ev[i].real();
      w[2 * i + 1] = ev[i].imag();
    }
    if (Z)
      for (size_t i = 0; i < size_t(n) * n; ++i) {
        Z[2 * i] = Zm.a[i].real();
        Z[2 * i + 1] = Zm.a[i].imag();
      }
    return DC_OK;
  });
}

int dc_dense_lstsq(int32_t rows, int32_t cols, const double* A, const double* b, double* x,
                   double* resnorm) {
  return guarded([&] {
    if (rows < cols || cols < 0 || !A || !b || !x) throw dc::InvalidArg("bad arguments");
    std::vector<dc::cd> bb(rows);
    for (int i = 0; i < rows; ++i) bb[i] = dc::cd(b[2 * i], b[2 * i + 1]);
    double rn = 0.0;
    const auto xs = dc::lstsq(read_mat(rows, cols, A), bb, &rn);
    for (int i = 0; i < cols; ++i) {
      x[2 * i] = xs[i].real();
      x[2 * i + 1] = xs[i].imag();
    }
    if (resnorm) *resnorm = rn;
    return DC_OK;
  });
}

int dc_dense_solve(int32_t n, const double* A, int32_t nrhs, double* B) {
  return guarded([&] {
    if (n < 1 || nrhs < 0 || !A || !B) throw dc::InvalidArg("bad arguments");
    dc::Mat X = read_mat(n, nrhs, B);
    if (!dc::lu_solve(read_mat(n, n, A), X)) throw dc::InvalidArg("singular matrix");
    for (int j = 0; j < nrhs; ++j)
      for (int i = 0; i < n; ++i) {
        B[2 * (i + size_t(j) * n)] = X(i, j).real();
        B[2 * (i + size_t(j) * n) + 1] = X(i, j).imag();
      }
    return DC_OK;
  });
}

int dc_harmonic_ritz(int32_t d, const double* hbar, double* theta) {
  return guarded([&] {
    if (d < 1 || !hbar || !theta) throw dc::InvalidArg("bad arguments");
    std::vector<dc::cd> th;
    if (!dc::harmonic_ritz(read_mat(d + 1, d, hbar), th, nullptr))
      throw dc::InvalidArg("harmonic Ritz computation failed");
    for (int i = 0; i < d; ++i) {
      theta[2 * i] = th[i].real();
      theta[2 * i + 1] = th[i].imag();
    }
    return DC_OK;
  });
}

int dc_leja_order(int32_t d, const double* theta_in, double* theta_out) {
  return guarded([&] {
    if (d < 0 || !theta_in || !theta_out) throw dc::InvalidArg("bad arguments");
    std::vector<dc::cd> th(d);
    for (int i = 0; i < d; ++i) th[i] = dc::cd(theta_in[2 * i], theta_in[2 * i + 1]);
    const auto o = dc::leja_order(th);
    for (int i = 0; i < d; ++i) {
      theta_out[2 * i] = o[i].real();
      theta_out[2 * i + 1] = o[i].imag();
    }
    return DC_OK;
  });
}

}  // extern "C"
