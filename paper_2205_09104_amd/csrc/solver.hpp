// Coarse operator handle and the Krylov solvers driving the HIP kernels.
#pragma once

#include <chrono>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include "dense.hpp"
#include "kernels.hpp"

namespace dc {

// Device memory that the caller owns, carved into a handle's buffers: first
// fit over a free list, blocks of kArenaAlign-byte granules, neighbouring
// free blocks merged on release.  take() throws WorkspaceShort when no free
// block is large enough.
struct Arena {
  static constexpr size_t kArenaAlign = 256;
  char* base = nullptr;
  size_t cap = 0, used = 0, peak = 0;
  std::map<size_t, size_t> free_;   // offset -> length (granule multiples)
  Arena(void* p, size_t bytes);
  void* take(size_t bytes, const char* what);
  void give(void* p, size_t bytes);
  static size_t round(size_t b) { return (b + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }
};

// Number of device allocations (hipMalloc) the library has made in this
// process, and the bytes they hold now.
long long device_allocations();
long long device_bytes_held();

// Owning device allocation: hipMalloc, or a block of an Arena when `ar` is set
// (a handle built on caller-owned workspaces).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Arena* ar = nullptr;
  const char* what = "buffer";   // named in workspace errors
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), ar(o.ar), what(o.what) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; ar = o.ar; what = o.what;
      o.p = nullptr; o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t b);
  void ensure(size_t b) { if (b > bytes) alloc(b); }
  void release();
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

struct SolveOpts {
  int m = 30, k = 0, d = 0, u = 10, max_cycles = 100000;
  int block_jacobi = 0;
  Prec prec = P64;
  int outer = 0, m_outer = 10, max_outer = 50;
  double inner_tol = 1e-4;
  int schur = 0;   // solve the odd-even reduced system (Sec. 2.2)
  int ortho = 0;   // 0: CGS applied twice; 1: single-sync process (Sec. 3.5)
  int graphs = 0;  // 1: replay whole Arnoldi cycles as captured HIP graphs (latency-bound lattices)
  uint64_t seed = 0;
  const void* v0 = nullptr;     // device complex128 [V][n]
  const void* x_ref = nullptr;  // optional reference solutions, device complex128 [n_rhs][V][n]
};

struct SolveStats {
  int status = 0, cycles = 0, iters = 0, matvecs = 0, outer_iters = 0, rebuilt = 0;
  double rel_res_true = 0, rel_res_est = 0, t_setup_ms = 0, t_solve_ms = 0;
  double err_vs_ref = -1.0;     // ||x - x_ref|| / ||x_ref|| in FP64 (-1: no reference)
  int breakdowns = 0;           // cycles that ended on h_{j+1,j} = 0 (happy breakdown)
  int refresh_failed = 0;       // recycle refreshes whose dense problem failed (space frozen)
  int stagnated = 0;            // stopped because the FP64 residual no longer fell
};

struct Op;

// State of one solver variant: (precision, sign of mu, block Jacobi, d).
struct Variant {
  Prec prec;
  int sign;        // +1: D(mu); -1: D(-mu) (adjoint through Gamma5)
  int bj;
  int d;
  int schur = 0;   // works on the odd-even reduced operator (compressed even vectors)
  // polynomial
  std::vector<cd> theta;
  long poly_version = -1;
  long poly_serial = 0;        // bumped by every polynomial build
  // recycle space (vectors of the variant's precision)
  DevBuf U, C;
  int kcur = 0;
  int k_built = 0;   // recycle dimension requested when the space was built
  int updates = 0;
  long recycle_version = -1;
  std::vector<double> unorm;   // ||u_i||
  // q(A~) U, kept in step with U by the same linear combinations (the single-
  // RHS solver's recycle updates), so that x += q(A~) U c needs no polynomial
  // application; mu_ok: MU matches the current U and polynomial
  DevBuf MU;
  bool mu_ok = false;
  DevBuf ws, sm;               // Krylov workspace: vectors and small device arrays
};

// Optional timing of the apply's block kernel (stage 1) with HIP events that
// its dispatch records on the launch stream.  Launches inside an Arnoldi cycle carry the cycle step they
// belong to; steps past the one where the cycle stopped ran as no-ops (device
// done flag) and are dropped once the cycle's step count is known.
struct ApplyProfile {
  // passes: algorithmic vector passes of the launch (reads of distinct input
  // vectors plus output writes, each over the kernel's rows)
  struct Rec { hipEvent_t a, b; int prec; int tag; bool noop; int passes; };
  bool on = false;
  int every = 1;                  // time one launch in `every` of each kernel
  int tag = -1;                   // step of the pending cycle (-1: outside a cycle)
  std::vector<hipEvent_t> idle, owned;
  std::vector<Rec> recs;
  // slot = kernel * 3 + precision; kernel 0: full-lattice block kernel,
  // 1: the reduced operator's A_o^{-1} D_oe kernel, 2: its A_e - D_eo kernel
  static constexpr int kSlotsP = 9;
  long seen[kSlotsP] = {};        // launches since enabling
  double ms[kSlotsP] = {}, ms_all[kSlotsP] = {};
  long count[kSlotsP] = {}, count_all[kSlotsP] = {};   // *_all: no-op launches included
  long passes[kSlotsP] = {};      // vector passes of the counted work launches
  bool sample(int slot) { return on && (seen[slot]++ % every) == 0; }
  long missed = 0;                // launches not recorded (event cap reached)
  static constexpr size_t kMaxEvents = 16384;
  void reset();
  bool take(hipEvent_t* a, hipEvent_t* b);
  void end_cycle(int steps_done);
  void flush();
  ~ApplyProfile();
};

// Pinned host staging for the solver's small transfers.  A copy between the
// device and pageable host memory makes the runtime drain the stream before
// it issues the copy, so every such read or upload leaves the GPU idle for a
// host round trip; copies from and to pinned memory queue behind the kernels.
// Reads are queued (read) and land in their destinations at the next wait();
// uploads go through a ring of pinned slots, each reused only after the event
// recorded behind its previous copy has completed.
// Small transfers between the host logic and the device, in host-mapped
// pinned memory moved by copy kernels on the stream.  Uploads are queued in
// order with the kernels around them.  Reads are gathered: the copies run, in
// as few launches as possible, when wait() is called, so work queued between
// read() and wait() must not change what is read.  Areas that kernels have
// touched are released only with the stage.
struct HostStage {
  struct Pending { void* dst; const void* src; size_t off, bytes; };
  char* rd = nullptr;            // read area (host address)
  char* rd_dev = nullptr;        // its device address
  size_t rd_cap = 0, rd_used = 0;
  std::vector<Pending> pending;
  std::vector<void*> retired;    // outgrown read areas
  static constexpr int kSlots = 8;
  static constexpr size_t kSlotBytes = size_t(1) << 18;
  char* up = nullptr;            // kSlots upload slots (host address)
  char* up_dev = nullptr;
  hipEvent_t ev[kSlots] = {};
  bool ev_live[kSlots] = {};
  int next = 0;
  void read(void* dst, const void* src, size_t bytes, hipStream_t st);
  void wait(hipStream_t st);     // completes the stream's work, then scatters the reads
  void write(void* dst, const void* src, size_t bytes, hipStream_t st);
  ~HostStage();
};

// Waits for the stream by polling it (lower wake-up latency than a blocking
// wait; the solver's host thread has nothing else to do meanwhile).
void stream_wait(hipStream_t st);

// Arnoldi cycles captured as HIP graphs and replayed: a cycle that the host
// enqueues in one piece (small lattices, where launch overhead dominates) is
// recorded once on a private capture stream and launched as one graph on the
// caller's stream afterwards.  Entries are keyed by everything a captured
// kernel argument depends on (workspace and recycle-space addresses, the
// polynomial's version, the step count, the deflation count, the
// orthogonalisation mode, the host-mapped signal areas); the stopping target
// is read from device memory.  `broken`: capture failed once, stay eager.
struct GraphCache {
  struct Entry {
    std::vector<uintptr_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  static constexpr size_t kMaxEntries = 64;   // recordings kept (oldest dropped first)
  hipStream_t cap = nullptr;
  std::vector<Entry> entries;
  bool broken = false;
  long captured = 0, launched = 0;
  hipGraphExec_t find(const std::vector<uintptr_t>& key) const;
  void add(const std::vector<uintptr_t>& key, hipGraph_t graph, hipGraphExec_t exec);
  ~GraphCache();
};

// Host-mapped stop flag of the pending Arnoldi cycle, its per-step residual
// estimates, and two events that pace the host's enqueueing a bounded
// distance ahead of the device.
struct CycleSignal {
  int* host = nullptr;    // pinned, mapped
  int* dev = nullptr;     // its device address
  double* est_host = nullptr;  // pinned, mapped: estimate after each step
  double* est_dev = nullptr;
  int est_cap = 0;
  std::vector<void*> retired;  // outgrown estimate areas
  hipEvent_t ev[2] = {nullptr, nullptr};
  void ensure();
  void ensure_est(int steps);
  ~CycleSignal();
};

struct Op {
  // caller-owned device workspaces (build_coarse_op_ws): blocks, inverses,
  // tables and recycle spaces come from `persist`, every other buffer from
  // `scratch`; null: the handle allocates with hipMalloc.  Declared first so
  // that they outlive every buffer carved from them.
  std::unique_ptr<Arena> persist, scratch;
  bool caller_ws() const { return persist != nullptr; }
  void bind_arenas();             // point every buffer at its arena
  Arena* scratch_arena() const { return scratch.get(); }
  int dims[4] = {0, 0, 0, 0};
  int V = 0, n = 0, store = 0;
  double mu = 0.0;
  long version = 0;     // bumped by update_coarse_op
  hipStream_t stream = nullptr;
  DevBuf nbr, blk64, blk32, blk16, sc16;
  struct BJ {                        // block-Jacobi inverses (tiled), per sign of mu
    DevBuf b64, b32, b16, sc16;
    long version = -1;
  } bj[2];
  const BJ& ensure_bj(int sign, hipStream_t st);
  DevBuf gbuf64, gbuf32;
  // odd-even reduction: compressed row -> site maps and the odd-row temporary
  // t_o = A_o^{-1} D_oe x_e, per vector precision
  bool oddeven = false;              // every extent even
  DevBuf esite, osite;
  DevBuf ts64, ts32;
  DevBuf rbe, rbo, rxe, rto;         // FP64 half vectors of the reduced solve's wrapper
  DevBuf wvbuf;                      // recycle refresh: What^H U and its Gram partials
  // block GMRES workspaces (FP64 and reduced-precision vectors)
  struct BlockWS {
    DevBuf V, Z, W, T1, TA, PROD, U, small, tab, R, X, Bc, part, X0, E0, E;
    DevBuf rcoef, rtmp;   // recycle build / refresh: coefficients, new U, C, q(A) U
  } bk64, bk32;
  void* tmp_s(Prec p);
  DevBuf redpart;           // reducer scratch
  DevBuf scal;              // a few device doubles
  DevBuf t64a, t64b, t32a, t32b, zouter;  // per-solve vector scratch, kept across calls
  DevBuf ptrs;              // device pointer arrays of the multi-RHS apply
  DevBuf bpart;             // lockstep batches: per-column reduction partials
  std::vector<DevBuf> bws, bsm;            // per right-hand-side workspaces of batched solves
  DevBuf bx64, bb64, b32, x32, r64;        // batched-solve vectors
  ApplyProfile prof;
  CycleSignal sig;
  HostStage hs;
  GraphCache graphs;

  Reducer red() const { return Reducer{redpart.as<double>()}; }
  std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<Variant>> variants;
  size_t N() const { return size_t(V) * n; }
  Variant& variant(Prec p, int sign, int bj, int d, int schur = 0);
  const void* blocks(Prec p) const;
  const float* scales(Prec p) const { return p == P16S ? sc16.as<float>() : nullptr; }
  void* gbuf(Prec p) const { return p == P64 ? gbuf64.p : gbuf32.p; }
};

void op_build(Op& op, const int dims[4], int n_tv, int store, double mu, const void* self_blocks,
              const void* hop_blocks, bool on_device, hipStream_t st);

// Device bytes a handle needs when the caller provides its memory: the
// persistent part (blocks in every stored precision, FP16 scales, neighbour
// and parity tables, block-Jacobi / odd-site inverses for the signs of mu the
// options can use, recycle spaces) and the scratch part (apply partials,
// Krylov bases, vector temporaries), for the single-right-hand-side solves,
// applies, polynomial and Arnoldi calls with options o and multi-RHS applies
// of up to max_rhs vectors.  Each buffer is rounded up to the arena granule.
void workspace_bytes(const int dims[4], int n_tv, int store, double mu, bool host_input,
                     const SolveOpts& o, int max_rhs, size_t* persistent, size_t* scratch,
                     size_t* build_persistent = nullptr, size_t* build_scratch = nullptr);
void op_update(Op& op, const void* self_blocks, const void* hop_blocks, bool on_device,
               hipStream_t st);

// Precision-level entry points used by the C ABI.
void op_apply(Op& op, Prec p, int adjoint, const void* in, void* out, hipStream_t st);
void op_apply_bj(Op& op, const void* in, void* out, hipStream_t st);
// block_jacobi: out = D_ee^{-1} S in (left block Jacobi of the reduced system)
void op_apply_reduced(Op& op, Prec p, int adjoint, int block_jacobi, const void* in, void* out,
                      hipStream_t st);
// The reduced apply with its odd-row temporary in the fixed device scratch
// (noalloc_scratch): no allocation of any kind; the inverses must exist.
void op_apply_reduced_noalloc(Op& op, Prec p, int adjoint, const void* in, void* out,
                              hipStream_t st);
void op_apply_multi(Op& op, Prec p, int adjoint, int R, const void* in, void* out, hipStream_t st);
int op_poly_setup(Op& op, const SolveOpts& o, hipStream_t st, std::vector<cd>& theta);
// Install caller-given polynomial roots (used in the given order) for the
// variant of o; o.d must equal theta.size().
void op_poly_set(Op& op, const SolveOpts& o, const std::vector<cd>& theta);
void op_poly_apply(Op& op, const SolveOpts& o, const void* in, void* out, hipStream_t st);
int op_arnoldi(Op& op, const SolveOpts& o, const void* v, int steps, hipStream_t st,
               std::vector<cd>& hbar);
int op_solve(Op& op, const SolveOpts& o, int adjoint, int n_rhs, const void* b, void* x,
             const double* tol, int use_x0, hipStream_t st, SolveStats* stats);
int op_export_recycle(Op& op, const SolveOpts& o, int adjoint, void* U, void* C, hipStream_t st);
void op_profile(Op& op, int every);
void op_profile_read(Op& op, Prec p, int kernel, long* launches, double* total_ms, long* passes,
                     long* launches_all, double* total_ms_all);
int op_solve_multi(const std::vector<Op*>& ops, const SolveOpts& o, int adjoint,
                   const std::vector<int>& R, const std::vector<const void*>& b,
                   const std::vector<void*>& x, const std::vector<const double*>& tol, int use_x0,
                   hipStream_t st, const std::vector<SolveStats*>& stats);
int op_solve_batch(Op& op, const SolveOpts& o, int adjoint, int R, const void* b, void* x,
                   const double* tol, int use_x0, hipStream_t st, SolveStats* stats);
// block GMRES with one shared Krylov space over R right-hand sides
int op_solve_block(Op& op, const SolveOpts& o, int R, const void* b, void* x, const double* tol,
                   int use_x0, hipStream_t st, SolveStats* stats);
// shared helpers of the solvers
void check_prec(const Op& op, Prec p);
void ensure_poly(Op& op, Variant& var, const SolveOpts& o, hipStream_t st, SolveStats* stt);
double ms_since(std::chrono::steady_clock::time_point t0);

}  // namespace dc
