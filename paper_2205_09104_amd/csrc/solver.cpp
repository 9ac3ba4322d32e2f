// Coarse-operator handle and Krylov solvers: restarted GMRES (Sec. 3.1),
// GMRES-polynomial right preconditioning (Sec. 3.3), GCRO-DR deflated restarts
// with recycling (Sec. 3.4, algorithm of Parks et al. 2006), lazy rebuild after
// a matrix change (Sec. 3.6), and an FP64 flexible-GMRES outer loop around a
// reduced-precision inner solve.  Every vector operation runs in the HIP
// kernels of kernels.hip; the host keeps only the small dense problems
// (Hessenberg least squares, harmonic Ritz values and vectors, QR of k x k
// systems), done redundantly as the paper does per process.
#include "solver.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <atomic>
#include <cstring>

namespace dc {

static std::atomic<long long> g_allocs{0}, g_held{0};

long long device_allocations() { return g_allocs.load(); }
long long device_bytes_held() { return g_held.load(); }

Arena::Arena(void* p, size_t bytes) : base(static_cast<char*>(p)) {
  // use the granule-aligned part of the caller's range
  const uintptr_t a = reinterpret_cast<uintptr_t>(base);
  const uintptr_t a2 = (a + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
  const size_t skip = size_t(a2 - a);
  cap = bytes > skip ? (bytes - skip) / kArenaAlign * kArenaAlign : 0;
  base += skip;
  if (cap) free_[0] = cap;
}

void* Arena::take(size_t bytes, const char* what) {
  const size_t need = round(bytes);
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < need) continue;
    const size_t off = it->first, len = it->second;
    free_.erase(it);
    if (len > need) free_[off + need] = len - need;
    used += need;
    peak = std::max(peak, used);
    return base + off;
  }
  throw WorkspaceShort(std::string("caller workspace too small for ") + what + " (" +
                       std::to_string(need) + " bytes; " + std::to_string(cap - used) +
                       " of " + std::to_string(cap) + " free, fragmented)");
}

void Arena::give(void* p, size_t bytes) {
  size_t off = size_t(static_cast<char*>(p) - base);
  size_t len = round(bytes);
  used -= len;
  auto next = free_.lower_bound(off);
  if (next != free_.end() && off + len == next->first) {   // merge with the block after
    len += next->second;
    next = free_.erase(next);
  }
  if (next != free_.begin()) {                              // and the block before
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += len;
      return;
    }
  }
  free_[off] = len;
}

void DevBuf::alloc(size_t b) {
  release();
  if (b == 0) return;
  if (ar) {
    p = ar->take(b, what);
    bytes = b;
    return;
  }
  const hipError_t e = hipMalloc(&p, b);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    throw NoMem("hipMalloc of " + std::to_string(b) + " bytes failed: " + hipGetErrorString(e));
  }
  g_allocs += 1;
  g_held += (long long)b;
  bytes = b;
}

void DevBuf::release() {
  if (p) {
    if (ar) {
      ar->give(p, bytes);
    } else {
      (void)hipFree(p);
      g_held -= (long long)bytes;
    }
  }
  p = nullptr;
  bytes = 0;
}

void Op::bind_arenas() {
  Arena* P = persist.get();
  Arena* S = scratch.get();
  auto bind = [](DevBuf& b, Arena* a, const char* what) { b.ar = a; b.what = what; };
  bind(nbr, P, "neighbour table");
  bind(blk64, P, "FP64 blocks");
  bind(blk32, P, "FP32 blocks");
  bind(blk16, P, "FP16 blocks");
  bind(sc16, P, "FP16 scales");
  for (auto& b : bj) {
    bind(b.b64, P, "block inverses");
    bind(b.b32, P, "block inverses");
    bind(b.b16, P, "block inverses");
    bind(b.sc16, P, "block inverse scales");
  }
  bind(esite, P, "parity table");
  bind(osite, P, "parity table");
  for (DevBuf* b : {&gbuf64, &gbuf32, &ts64, &ts32, &rbe, &rbo, &rxe, &rto, &wvbuf, &redpart, &scal,
                    &t64a, &t64b, &t32a, &t32b, &zouter, &ptrs, &bpart, &bx64, &bb64, &b32, &x32,
                    &r64})
    bind(*b, S, "vector scratch");
  for (BlockWS* w : {&bk64, &bk32})
    for (DevBuf* b : {&w->V, &w->Z, &w->W, &w->T1, &w->TA, &w->PROD, &w->U, &w->small, &w->tab,
                      &w->R, &w->X, &w->Bc, &w->part, &w->X0, &w->E0, &w->E})
      bind(*b, S, "block-solver scratch");
}

static size_t block_units(int n, Prec p) {
  const int epl = (p == P64) ? 1 : (p == P32 ? 2 : 4);
  return size_t(tile_elems(n, epl) / epl) * 64;  // 16-byte units per block
}

void* Op::tmp_s(Prec p) {
  const size_t len = size_t(V / 2) * n;
  if (p == P64) {
    ts64.ensure(len * sizeof(z64));
    return ts64.p;
  }
  ts32.ensure(len * sizeof(z32));
  return ts32.p;
}

const void* Op::blocks(Prec p) const {
  if (p == P64) return blk64.p;
  if (p == P32) return blk32.p;
  return blk16.p;
}

Variant& Op::variant(Prec p, int sign, int bj, int d, int schur) {
  auto key = std::make_tuple(int(p), sign, bj, d, schur);
  auto it = variants.find(key);
  if (it != variants.end()) return *it->second;
  auto v = std::make_unique<Variant>();
  if (caller_ws()) {
    for (DevBuf* b : {&v->U, &v->C, &v->MU}) { b->ar = persist.get(); b->what = "recycle space"; }
    for (DevBuf* b : {&v->ws, &v->sm}) { b->ar = scratch.get(); b->what = "Krylov workspace"; }
  }
  v->prec = p;
  v->sign = sign;
  v->bj = bj;
  v->d = d;
  v->schur = schur;
  Variant& ref = *v;
  variants.emplace(key, std::move(v));
  return ref;
}

static void copy_blocks_in(Op& op, const void* self_blocks, const void* hop_blocks, bool on_device,
                           hipStream_t st) {
  const size_t nn = size_t(op.n) * op.n;
  const z64* dself = static_cast<const z64*>(self_blocks);
  const z64* dhops = static_cast<const z64*>(hop_blocks);
  DevBuf stage;
  stage.ar = op.scratch_arena();
  stage.what = "host block staging";
  if (!on_device) {
    stage.alloc(size_t(op.V) * 5 * nn * sizeof(z64));
    z64* s = stage.as<z64>();
    DC_HIP(hipMemcpyAsync(s, self_blocks, size_t(op.V) * nn * sizeof(z64), hipMemcpyHostToDevice, st));
    DC_HIP(hipMemcpyAsync(s + size_t(op.V) * nn, hop_blocks, size_t(op.V) * 4 * nn * sizeof(z64),
                          hipMemcpyHostToDevice, st));
    dself = s;
    dhops = s + size_t(op.V) * nn;
  }
  launch_layout_blocks(dself, dhops, op.V, op.n, op.blk64.p, op.blk32.p, op.blk16.p,
                       op.sc16.as<float>(), st);
  DC_HIP(hipStreamSynchronize(st));
}

void op_build(Op& op, const int dims[4], int n_tv, int store, double mu, const void* self_blocks,
              const void* hop_blocks, bool on_device, hipStream_t st) {
  for (int i = 0; i < 4; ++i) {
    if (dims[i] < 1) throw InvalidArg("lattice extents must be >= 1");
    op.dims[i] = dims[i];
  }
  if (n_tv < 1 || n_tv > 32) throw InvalidArg("n_tv must be in 1..32");
  if (!self_blocks || !hop_blocks) throw InvalidArg("null block pointer");
  if (!std::isfinite(mu)) throw InvalidArg("mu must be finite");
  const long long V = 1LL * dims[0] * dims[1] * dims[2] * dims[3];
  if (V > (1LL << 30)) throw InvalidArg("lattice too large");
  op.V = int(V);
  op.n = 2 * n_tv;
  op.store = store | 1;
  op.mu = mu;
  op.stream = st;
  op.nbr.alloc(size_t(8) * op.V * sizeof(int));
  launch_neighbours(op.nbr.as<int>(), dims[0], dims[1], dims[2], dims[3], st);
  const size_t nb = size_t(op.V) * 5;
  op.blk64.alloc(nb * block_units(op.n, P64) * 16);
  if (op.store & 2) op.blk32.alloc(nb * block_units(op.n, P32) * 16);
  if (op.store & 4) {
    op.blk16.alloc(nb * block_units(op.n, P16S) * 16);
    op.sc16.alloc(nb * sizeof(float));
  }
  op.gbuf64.alloc(size_t(op.V) * 9 * op.n * sizeof(z64));
  if (op.store & 6) op.gbuf32.alloc(size_t(op.V) * 9 * op.n * sizeof(z32));
  op.redpart.alloc(size_t(kRedCap) * sizeof(double));
  op.scal.alloc(256);
  // checkerboard tables for the odd-even reduction (every extent even): site
  // parity and the sites of each parity in increasing order (row r of a
  // compressed vector is site esite[r] / osite[r]; for even L0 that is 2r or 2r+1)
  op.oddeven = (dims[0] % 2 == 0) && (dims[1] % 2 == 0) && (dims[2] % 2 == 0) &&
               (dims[3] % 2 == 0);
  if (op.oddeven) {
    std::vector<int> es, os;
    es.reserve(op.V / 2);
    os.reserve(op.V / 2);
    for (int x = 0; x < op.V; ++x) {
      const int x0 = x % dims[0], x1 = (x / dims[0]) % dims[1];
      const int x2 = (x / (dims[0] * dims[1])) % dims[2], x3 = x / (dims[0] * dims[1] * dims[2]);
      (((x0 + x1 + x2 + x3) & 1) ? os : es).push_back(x);
    }
    op.esite.alloc(es.size() * sizeof(int));
    op.osite.alloc(os.size() * sizeof(int));
    DC_HIP(hipMemcpyAsync(op.esite.p, es.data(), es.size() * sizeof(int), hipMemcpyHostToDevice, st));
    DC_HIP(hipMemcpyAsync(op.osite.p, os.data(), os.size() * sizeof(int), hipMemcpyHostToDevice, st));
    DC_HIP(hipStreamSynchronize(st));  // host tables must outlive the copies
  }
  copy_blocks_in(op, self_blocks, hop_blocks, on_device, st);
}

void op_update(Op& op, const void* self_blocks, const void* hop_blocks, bool on_device,
               hipStream_t st) {
  if (!self_blocks || !hop_blocks) throw InvalidArg("null block pointer");
  copy_blocks_in(op, self_blocks, hop_blocks, on_device, st);
  op.version += 1;  // block Jacobi, polynomial and recycle space become stale
}

// ------------------------------------------------------------------ apply profile
static int prec_slot(Prec p) { return p == P64 ? 0 : (p == P32 ? 1 : 2); }

void ApplyProfile::reset() {
  flush();
  for (int i = 0; i < kSlotsP; ++i) {
    ms[i] = ms_all[i] = 0.0;
    count[i] = count_all[i] = 0;
    passes[i] = 0;
    seen[i] = 0;
  }
  missed = 0;
  tag = -1;
}

bool ApplyProfile::take(hipEvent_t* a, hipEvent_t* b) {
  while (idle.size() < 2 && owned.size() + 2 <= kMaxEvents) {
    hipEvent_t e;
    DC_HIP(hipEventCreate(&e));
    owned.push_back(e);
    idle.push_back(e);
  }
  if (idle.size() < 2) return false;
  *a = idle.back(); idle.pop_back();
  *b = idle.back(); idle.pop_back();
  return true;
}

void ApplyProfile::end_cycle(int steps_done) {
  for (Rec& r : recs)
    if (r.tag >= 0) {
      if (r.tag >= steps_done) r.noop = true;
      r.tag = -1;
    }
  tag = -1;
}

void ApplyProfile::flush() {
  for (Rec& r : recs) {
    DC_HIP(hipEventSynchronize(r.b));
    float t = 0.f;
    DC_HIP(hipEventElapsedTime(&t, r.a, r.b));
    ms_all[r.prec] += t;
    ++count_all[r.prec];
    if (!r.noop) {
      ms[r.prec] += t;
      ++count[r.prec];
      passes[r.prec] += r.passes;
    }
    idle.push_back(r.a);
    idle.push_back(r.b);
  }
  recs.clear();
}

ApplyProfile::~ApplyProfile() {
  for (hipEvent_t e : owned) (void)hipEventDestroy(e);
}

void GraphCache::add(const std::vector<uintptr_t>& key, hipGraph_t graph, hipGraphExec_t exec) {
  if (entries.size() >= kMaxEntries) {   // drop the oldest recording
    Entry& e = entries.front();
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
    entries.erase(entries.begin());
  }
  entries.push_back({key, graph, exec});
}

hipGraphExec_t GraphCache::find(const std::vector<uintptr_t>& key) const {
  for (const Entry& e : entries)
    if (e.key == key) return e.exec;
  return nullptr;
}

GraphCache::~GraphCache() {
  for (Entry& e : entries) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
  }
  if (cap) (void)hipStreamDestroy(cap);
}

void stream_wait(hipStream_t st) {
  for (;;) {
    const hipError_t e = hipStreamQuery(st);
    if (e == hipSuccess) return;
    if (e != hipErrorNotReady) DC_HIP(e);
  }
}

static char* mapped_alloc(size_t bytes, char** dev) {
  void* h = nullptr;
  DC_HIP(hipHostMalloc(&h, bytes, hipHostMallocMapped | hipHostMallocCoherent));
  void* d = nullptr;
  DC_HIP(hipHostGetDevicePointer(&d, h, 0));
  *dev = static_cast<char*>(d);
  return static_cast<char*>(h);
}

void HostStage::read(void* dst, const void* src, size_t bytes, hipStream_t st) {
  const size_t off = (rd_used + 15) & ~size_t(15);
  if (off + bytes > rd_cap) {
    wait(st);                    // no read may be pending while the area is replaced
    size_t cap = std::max<size_t>(size_t(1) << 20, 2 * rd_cap);
    while (cap < bytes) cap *= 2;
    if (rd) retired.push_back(rd);
    rd = mapped_alloc(cap, &rd_dev);
    rd_cap = cap;
    read(dst, src, bytes, st);
    return;
  }
  if (bytes % 4 != 0 || reinterpret_cast<uintptr_t>(src) % 4 != 0)
    throw InvalidArg("staged reads move aligned 4-byte words");
  pending.push_back({dst, src, off, bytes});
  rd_used = off + bytes;
}

void HostStage::wait(hipStream_t st) {
  CopySegments seg;
  for (const Pending& q : pending) {
    if (q.bytes == 0) continue;
    if (seg.count == kCopySegMax) {
      launch_copy_segments(seg, st);
      seg.count = 0;
    }
    seg.src[seg.count] = static_cast<const uint32_t*>(q.src);
    seg.dst[seg.count] = reinterpret_cast<uint32_t*>(rd_dev + q.off);
    seg.words[seg.count] = q.bytes / 4;
    ++seg.count;
  }
  launch_copy_segments(seg, st);
  stream_wait(st);
  for (const Pending& q : pending) std::memcpy(q.dst, rd + q.off, q.bytes);
  pending.clear();
  rd_used = 0;
}

void HostStage::write(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes > kSlotBytes) {      // large uploads (rare): through the read path's wait
    DC_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    wait(st);
    return;
  }
  if (!up) {
    up = mapped_alloc(kSlots * kSlotBytes, &up_dev);
    for (auto& e : ev) DC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  const int s = next;
  next = (next + 1) % kSlots;
  if (ev_live[s]) DC_HIP(hipEventSynchronize(ev[s]));   // its previous copy has run
  std::memcpy(up + size_t(s) * kSlotBytes, src, bytes);
  launch_copy_words(up_dev + size_t(s) * kSlotBytes, dst, bytes, st);
  DC_HIP(hipEventRecord(ev[s], st));
  ev_live[s] = true;
}

HostStage::~HostStage() {
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (rd) (void)hipHostFree(rd);
  for (void* r : retired) (void)hipHostFree(r);
  if (up) (void)hipHostFree(up);
}

void CycleSignal::ensure() {
  if (host) return;
  void* h = nullptr;
  DC_HIP(hipHostMalloc(&h, 64, hipHostMallocMapped | hipHostMallocCoherent));
  host = static_cast<int*>(h);
  *host = 0;
  void* d = nullptr;
  DC_HIP(hipHostGetDevicePointer(&d, h, 0));
  dev = static_cast<int*>(d);
  for (auto& e : ev) DC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

void CycleSignal::ensure_est(int steps) {
  if (est_host && est_cap >= steps) return;
  if (est_host) retired.push_back(est_host);   // kernels wrote it: released with the signal
  est_host = nullptr;
  est_dev = nullptr;
  est_cap = 0;
  const int cap = std::max(steps, 256);
  void* h = nullptr;
  DC_HIP(hipHostMalloc(&h, size_t(cap) * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
  est_host = static_cast<double*>(h);
  void* d = nullptr;
  DC_HIP(hipHostGetDevicePointer(&d, h, 0));
  est_dev = static_cast<double*>(d);
  est_cap = cap;
}

CycleSignal::~CycleSignal() {
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (host) (void)hipHostFree(host);
  if (est_host) (void)hipHostFree(est_host);
  for (void* r : retired) (void)hipHostFree(r);
}

// Stage 1 of the apply, timed when profiling is on (one in `every` launches
// of each kernel).  Records are flushed outside cycles once many have
// accumulated, so the event pool stays small.
static void stage1(Op& op, Prec p, int n, int V, const void* blocks, const float* scales,
                   const void* in, void* gbuf, const int* nbr, double tm, const int* done,
                   hipStream_t st) {
  ApplyProfile& pr = op.prof;
  hipEvent_t a = nullptr, b = nullptr;
  const int slot = prec_slot(p);
  if (pr.sample(slot)) {
    if (pr.tag < 0 && pr.recs.size() >= 2048) pr.flush();
    if (!pr.take(&a, &b)) ++pr.missed;
  }
  launch_apply_blocks(p, n, V, blocks, scales, in, gbuf, nbr, tm, done, st, a, b);
  if (a) pr.recs.push_back({a, b, slot, done ? pr.tag : -1, false, 1});
}

// The reduced operator's kernels (Sec. 2.2, factored form), timed like stage1:
// t_o = A_o^{-1} D_oe x_e, then A_e x_e - D_eo t_o with an epilogue.
static void reduced_oe(Op& op, Prec p, const void* inv, const float* invsc, const void* x_e,
                       void* t_o, const int* done, hipStream_t st) {
  ApplyProfile& pr = op.prof;
  hipEvent_t a = nullptr, b = nullptr;
  const int slot = 3 + prec_slot(p);
  if (pr.sample(slot)) {
    if (pr.tag < 0 && pr.recs.size() >= 2048) pr.flush();
    if (!pr.take(&a, &b)) ++pr.missed;
  }
  launch_reduced_oe(p, op.n, op.V, op.blocks(p), op.scales(p), inv, invsc, x_e, t_o,
                    op.nbr.as<int>(), op.osite.as<int>(), done, st, a, b);
  if (a) pr.recs.push_back({a, b, slot, done ? pr.tag : -1, false, 2});
}

static void reduced_eo(Op& op, Prec p, int epi, const void* einv, const float* einvsc,
                       const void* x_e, const void* t_o, double tm, void* out, const void* e,
                       void* y, z64 c0, z64 ca, z64 cb, const int* done, hipStream_t st) {
  ApplyProfile& pr = op.prof;
  hipEvent_t a = nullptr, b = nullptr;
  const int slot = 6 + prec_slot(p);
  if (pr.sample(slot)) {
    if (pr.tag < 0 && pr.recs.size() >= 2048) pr.flush();
    if (!pr.take(&a, &b)) ++pr.missed;
  }
  launch_reduced_eo(p, epi, op.n, op.V, op.blocks(p), op.scales(p), einv, einvsc, x_e, t_o,
                    op.nbr.as<int>(), op.esite.as<int>(), tm, out, e, y, c0, ca, cb, done, st, a, b);
  if (a) {
    // distinct vectors read (x_e, t_o and the epilogue's inputs) plus writes
    int passes = 1 + (x_e ? 1 : 0);
    if ((epi == 1 || epi == 3) && e != x_e) ++passes;
    if (epi == 2) passes += (out != x_e ? 1 : 0) + 1;
    passes += (epi == 1 || epi == 2) ? 2 : 1;
    pr.recs.push_back({a, b, slot, done ? pr.tag : -1, false, passes});
  }
}

// The single-read pair (launch_reduced_scatter / launch_reduced_gather), timed
// in the same slots as the two-kernel form's first and second kernel.  hp is
// the full-lattice apply's partial buffer (V x 9 x n vectors, at least the
// V/2 x 8 x n the pair needs); the two uses never overlap on the stream.
static void reduced_scatter(Op& op, Prec p, const void* inv, const float* invsc,
                            const void* x_e, void* hp, const int* done, hipStream_t st) {
  ApplyProfile& pr = op.prof;
  hipEvent_t a = nullptr, b = nullptr;
  const int slot = 3 + prec_slot(p);
  if (pr.sample(slot)) {
    if (pr.tag < 0 && pr.recs.size() >= 2048) pr.flush();
    if (!pr.take(&a, &b)) ++pr.missed;
  }
  launch_reduced_scatter(p, op.n, op.V, op.blocks(p), op.scales(p), inv, invsc, x_e, hp,
                         op.nbr.as<int>(), op.osite.as<int>(), done, st, a, b);
  // x_e read once, eight partial vectors written
  if (a) pr.recs.push_back({a, b, slot, done ? pr.tag : -1, false, 9});
}

static void reduced_gather(Op& op, Prec p, int epi, const void* einv, const float* einvsc,
                           const void* x_e, const void* hp, double tm, void* out, const void* e,
                           void* y, z64 c0, z64 ca, z64 cb, const int* done, hipStream_t st) {
  ApplyProfile& pr = op.prof;
  hipEvent_t a = nullptr, b = nullptr;
  const int slot = 6 + prec_slot(p);
  if (pr.sample(slot)) {
    if (pr.tag < 0 && pr.recs.size() >= 2048) pr.flush();
    if (!pr.take(&a, &b)) ++pr.missed;
  }
  launch_reduced_gather(p, epi, op.n, op.V, op.blocks(p), op.scales(p), einv, einvsc, x_e, hp,
                        op.esite.as<int>(), tm, out, e, y, c0, ca, cb, done, st, a, b);
  if (a) {
    // the eight partial vectors, x_e, the epilogue's inputs, and the writes
    int passes = 8 + (x_e ? 1 : 0);
    if ((epi == 1 || epi == 3) && e != x_e) ++passes;
    if (epi == 2) passes += (out != x_e ? 1 : 0) + 1;
    passes += (epi == 1 || epi == 2) ? 2 : 1;
    pr.recs.push_back({a, b, slot, done ? pr.tag : -1, false, passes});
  }
}

void op_profile(Op& op, int every) {
  if (every < 0) throw InvalidArg("sampling period must be >= 0");
  op.prof.reset();
  op.prof.on = every != 0;
  op.prof.every = every > 0 ? every : 1;
}

void op_profile_read(Op& op, Prec p, int kernel, long* launches, double* total_ms, long* passes,
                     long* launches_all, double* total_ms_all) {
  if (kernel < 0 || kernel > 2) throw InvalidArg("kernel must be 0, 1 or 2");
  op.prof.flush();
  const int i = 3 * kernel + prec_slot(p);
  if (launches) *launches = op.prof.count[i];
  if (total_ms) *total_ms = op.prof.ms[i];
  if (passes) *passes = op.prof.passes[i];
  if (launches_all) *launches_all = op.prof.count_all[i];
  if (total_ms_all) *total_ms_all = op.prof.ms_all[i];
}

void check_prec(const Op& op, Prec p) {
  if (p == P32 && !(op.store & 2)) throw InvalidArg("FP32 blocks were not stored (desc.store)");
  if (p == P16S && !(op.store & 4)) throw InvalidArg("FP16 blocks were not stored (desc.store)");
  if (p != P64 && p != P32 && p != P16S) throw InvalidArg("unknown precision");
}

static size_t vec_bytes(Prec p) { return p == P64 ? sizeof(z64) : sizeof(z32); }

void op_apply(Op& op, Prec p, int adjoint, const void* in, void* out, hipStream_t st) {
  check_prec(op, p);
  if (!in || !out) throw InvalidArg("null vector pointer");
  if (in == out) throw InvalidArg("in and out must not overlap");
  if (!adjoint) {
    stage1(op, p, op.n, op.V, op.blocks(p), op.scales(p), in, op.gbuf(p), op.nbr.as<int>(),
                        op.mu, nullptr, st);
    launch_gather_store(p, op.n, op.V, op.gbuf(p), out, nullptr, st);
  } else {
    // D(mu)^H = Gamma5 D(-mu) Gamma5
    launch_gamma5(p, in, out, op.V, op.n, st);
    stage1(op, p, op.n, op.V, op.blocks(p), op.scales(p), out, op.gbuf(p),
                        op.nbr.as<int>(), -op.mu, nullptr, st);
    launch_gather_store(p, op.n, op.V, op.gbuf(p), out, nullptr, st);
    launch_gamma5(p, out, out, op.V, op.n, st);
  }
}

const Op::BJ& Op::ensure_bj(int sign, hipStream_t st) {
  BJ& b = bj[sign > 0 ? 0 : 1];
  if (b.version == version) return b;
  const size_t nb = size_t(V);
  b.b64.ensure(nb * block_units(n, P64) * 16);
  if (store & 2) b.b32.ensure(nb * block_units(n, P32) * 16);
  if (store & 4) {
    b.b16.ensure(nb * block_units(n, P16S) * 16);
    b.sc16.ensure(nb * sizeof(float));
  }
  int* flag = reinterpret_cast<int*>(scal.as<double>() + 16);
  DC_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  launch_invert_blocks(blk64.p, V, n, sign * mu, b.b64.p, (store & 2) ? b.b32.p : nullptr,
                       (store & 4) ? b.b16.p : nullptr, (store & 4) ? b.sc16.as<float>() : nullptr,
                       flag, st);
  int h = 0;
  hs.read(&h, flag, sizeof(int), st);
  hs.wait(st);
  if (h) throw BadState("a self block is singular: block-Jacobi preconditioning is not defined");
  b.version = version;
  return b;
}

static const void* bj_blocks(const Op::BJ& b, Prec p) {
  return p == P64 ? b.b64.p : (p == P32 ? b.b32.p : b.b16.p);
}

void op_apply_reduced(Op& op, Prec p, int adjoint, int block_jacobi, const void* in, void* out,
                      hipStream_t st) {
  check_prec(op, p);
  if (!op.oddeven) throw InvalidArg("the odd-even reduction needs every lattice extent even");
  if (!in || !out) throw InvalidArg("null vector pointer");
  const int half = op.V / 2;
  const size_t N = size_t(half) * op.n;
  {
    const char* a = static_cast<const char*>(in);
    const char* b = static_cast<const char*>(out);
    const size_t span = N * vec_bytes(p);
    if (a < b + span && b < a + span) throw InvalidArg("in and out overlap");
  }
  // S(mu)^H = Gamma5 S(-mu) Gamma5, as for the full operator
  const int sign = adjoint ? -1 : +1;
  const double tm = sign * op.mu;
  const Op::BJ& bj = op.ensure_bj(sign, st);
  const void* inv = bj_blocks(bj, p);
  const float* invsc = (p == P16S) ? bj.sc16.as<float>() : nullptr;
  // left block Jacobi B = D_ee (Sec. 3.2): the even sites' inverses, same arrays
  const void* bj_e = block_jacobi ? inv : nullptr;
  const float* bj_esc = block_jacobi ? invsc : nullptr;
  void* ts = op.tmp_s(p);
  const void* src = in;
  if (adjoint) {
    launch_gamma5(p, in, out, half, op.n, st);
    src = out;
  }
  const z64 z = mk(0.0, 0.0);
  if (reduced_single_read(p, op.n)) {
    void* hp = op.gbuf(p);
    reduced_scatter(op, p, inv, invsc, src, hp, nullptr, st);
    reduced_gather(op, p, 0, bj_e, bj_esc, src, hp, tm, out, nullptr, nullptr, z, z, z, nullptr,
                   st);
  } else {
    reduced_oe(op, p, inv, invsc, src, ts, nullptr, st);
    // the D_eo kernel reads src only on its own row before writing that row of out
    reduced_eo(op, p, 0, bj_e, bj_esc, src, ts, tm, out, nullptr, nullptr, z, z, z, nullptr, st);
  }
  if (adjoint) launch_gamma5(p, out, out, half, op.n, st);
}

void op_apply_reduced_noalloc(Op& op, Prec p, int adjoint, const void* in, void* out,
                              hipStream_t st) {
  check_prec(op, p);
  if (!op.oddeven) throw InvalidArg("the odd-even reduction needs every lattice extent even");
  if (!in || !out) throw InvalidArg("null vector pointer");
  const int half = op.V / 2;
  const size_t N = size_t(half) * op.n;
  const size_t span = N * vec_bytes(p);
  {
    const char* a = static_cast<const char*>(in);
    const char* b = static_cast<const char*>(out);
    if (a < b + span && b < a + span) throw InvalidArg("in and out overlap");
  }
  // the odd-row temporary must fit the fixed scratch
  if (span > kNoAllocScratchBytes)
    throw InvalidArg("the odd-row temporary (" + std::to_string(span) +
                     " bytes) exceeds the fixed scratch of " +
                     std::to_string(kNoAllocScratchBytes) + " bytes");
  const int sign = adjoint ? -1 : +1;
  const Op::BJ& bj = op.bj[sign > 0 ? 0 : 1];
  if (bj.version != op.version)
    throw BadState("the odd self-block inverses of this operator are not built yet: call "
                   "dc_apply_reduced (or a reduced solve) with the same adjoint flag first");
  void* t = noalloc_scratch(true);   // looked up once per device (at build, normally)
  const void* inv = bj_blocks(bj, p);
  const float* invsc = (p == P16S) ? bj.sc16.as<float>() : nullptr;
  const double tm = sign * op.mu;
  const void* src = in;
  if (adjoint) {
    launch_gamma5(p, in, out, half, op.n, st);
    src = out;
  }
  const z64 z = mk(0.0, 0.0);
  launch_reduced_oe(p, op.n, op.V, op.blocks(p), op.scales(p), inv, invsc, src, t,
                    op.nbr.as<int>(), op.osite.as<int>(), nullptr, st);
  launch_reduced_eo(p, 0, op.n, op.V, op.blocks(p), op.scales(p), nullptr, nullptr, src, t,
                    op.nbr.as<int>(), op.esite.as<int>(), tm, out, nullptr, nullptr, z, z, z,
                    nullptr, st);
  if (adjoint) launch_gamma5(p, out, out, half, op.n, st);
}

void op_apply_bj(Op& op, const void* in, void* out, hipStream_t st) {
  if (!in || !out || in == out) throw InvalidArg("bad vector pointers");
  const Op::BJ& b = op.ensure_bj(+1, st);
  launch_bj_vec(P64, op.n, op.V, b.b64.p, nullptr, in, out, st);
}

void op_apply_multi(Op& op, Prec p, int adjoint, int R, const void* in, void* out, hipStream_t st) {
  check_prec(op, p);
  if (R < 0) throw InvalidArg("n_rhs must be >= 0");
  if (R == 0) return;
  if (!in || !out) throw InvalidArg("bad vector pointers");
  const size_t vb = op.N() * vec_bytes(p);
  {
    const char* a = static_cast<const char*>(in);
    const char* b = static_cast<const char*>(out);
    const size_t span = size_t(R) * vb;
    if (a < b + span && b < a + span) throw InvalidArg("in and out overlap");
  }
  std::vector<const void*> h(2 * size_t(R));
  for (int r = 0; r < R; ++r) {
    h[r] = static_cast<const char*>(in) + size_t(r) * vb;
    h[R + r] = static_cast<char*>(out) + size_t(r) * vb;
  }
  op.ptrs.ensure(h.size() * sizeof(void*));
  op.hs.write(op.ptrs.p, h.data(), h.size() * sizeof(void*), st);
  void** table = op.ptrs.as<void*>();
  const void* const* xin = const_cast<const void* const*>(table);
  void* const* yout = table + R;
  launch_apply_multi(p, op.n, op.V, op.blocks(p), op.scales(p), xin, yout, R, op.nbr.as<int>(),
                     adjoint ? -op.mu : op.mu, adjoint ? 3 : 0, st);
}

// ============================================================================ Krylov

namespace {


// min || beta e_{k+1} - G y || for the GCRO-DR matrix G = [[D_k, B_k], [0, Hbar]]
// (D_k = diag(1 / unorm)): the first k rows are met exactly by
// y_1 = -D_k^{-1} B_k y_2, so only the (j+1) x j Hessenberg part is a least-
// squares problem.  O(j^2 + k j) instead of a dense QR of the whole G.
static std::vector<cd> gcrodr_lstsq(const Mat& Hbar, const Mat& Bk,
                                    const std::vector<double>& unorm, double beta, double* res) {
  const int k = Bk.r, j = Hbar.c;
  std::vector<cd> y(size_t(k) + j, cd(0.0));
  if (j == 0) {
    if (res) *res = beta;
    return y;
  }
  std::vector<cd> e1(j + 1, cd(0.0));
  e1[0] = beta;
  const auto y2 = lstsq(Hbar, e1, res);
  for (int i = 0; i < k; ++i) {
    cd acc(0.0);
    for (int q = 0; q < j; ++q) acc += Bk(i, q) * y2[q];
    y[i] = -acc * unorm[i];
  }
  for (int q = 0; q < j; ++q) y[size_t(k) + q] = y2[q];
  return y;
}

// Device workspace of one Krylov solver instance: the basis (m + 2 vectors,
// with a polynomial also the z_j), recycle refresh temporaries, 8 work
// vectors, and the small arrays (coefficients, Hessenberg, B_k, Givens).
// Device bytes of the recycle refresh's Gram products for kk recycled vectors
// and up to mr Arnoldi vectors: C^H U, V^H U (FP64 complex) and the chunk
// partials of either (at most kRefreshGramParts chunks of kk x mr).
constexpr size_t kRefreshGramParts = 32;
static size_t refresh_gram_bytes(int kk, int mr) {
  return (size_t(kk) * kk + size_t(kk) * mr * (1 + kRefreshGramParts)) * sizeof(z64);
}

struct KrylovSizes {
  int kmax, ldh, nbasis, ktmp, nz, kz;
  size_t ws_bytes, sm_bytes;
};
static KrylovSizes krylov_sizes(size_t N, size_t zbytes, int k, int d, int steps_max,
                                bool recycle_tmp) {
  KrylovSizes s;
  s.kmax = std::max(k, 0);
  s.ldh = std::max(steps_max, std::max(d, 1)) + 2;
  s.nbasis = s.ldh + 1;
  s.ktmp = recycle_tmp ? s.kmax : 0;
  s.nz = (recycle_tmp && d > 1) ? s.nbasis : 0;
  s.kz = s.nz ? s.ktmp : 0;
  const size_t nvec = size_t(s.nbasis) + 2 * size_t(s.ktmp) + size_t(s.nz) + size_t(s.kz) + 8;
  s.ws_bytes = nvec * N * zbytes;
  const int kmax = s.kmax, ldh = s.ldh;
  const size_t q = size_t(kmax + ldh + 4);
  const size_t nd = 2 * q * 2 + 8 + 2 * size_t(std::max(kmax + ldh + 2, 1)) * std::max(kmax, 2) +
                    2 * size_t(ldh) * ldh + 2 * size_t(std::max(kmax, 1)) * ldh +
                    2 * 3 * size_t(ldh + 1) + 64;
  s.sm_bytes = nd * sizeof(double) + 64 * sizeof(int);
  return s;
}

template <typename VR>
struct Krylov {
  using Z = cx<VR>;
  Op& op;
  Variant& var;
  const SolveOpts& o;
  Prec p;
  double tm;  // twisted mass used in the apply (sign * mu)
  hipStream_t st;
  size_t N;
  int ldh = 0, kmax = 0, nbasis = 0;
  // device workspace (owned by the variant so it persists across calls)
  DevBuf& ws;
  DevBuf& sm;
  // Zb: z_j = q(A~) v_j of the cycle's steps (flexible-GMRES storage, with a
  // polynomial and a recycle-capable workspace); MUtmp: q(A~) U during refresh
  Z *Zb = nullptr, *MUtmp = nullptr;
  // orthogonalisation of the next cycle (see use_ortho); ss_off: a single-sync
  // cycle broke down (||A v||^2 - sum |h|^2 not positive, which loss of
  // orthogonality can cause as well as an invariant subspace) and the rest of
  // the solve uses Gram-Schmidt twice, whose breakdown test is reliable
  int ortho_now = 0;
  bool ss_off = false;
  // inner solves of the FP64 flexible outer loop stop on the recursively
  // updated residual of the deflated GCRO-DR cycles (rhat, which without a
  // left preconditioner is the residual of this precision's operator) instead
  // of re-applying the operator: the outer loop's FP64 residual decides
  bool inner_est = false;
  double bn_hint = -1.0;   // ||b|| when the caller knows it (inner solves: unit vectors)
  std::vector<double> Hh_, Bh_;   // host copies of the cycle's Hessenberg and B_k columns
  Z *Vb = nullptr, *Ctmp = nullptr, *Utmp = nullptr, *prod = nullptr, *ybuf = nullptr,
    *tmp = nullptr, *tmp2 = nullptr, *rhat = nullptr, *rtrue = nullptr, *ta = nullptr, *tb = nullptr;
  double *res1 = nullptr, *res2 = nullptr, *nrm = nullptr, *coef = nullptr, *scal = nullptr;
  ArnoldiDev ad{};
  long matvecs = 0;
  int refresh_failed = 0;         // refreshes whose dense problem failed
  int breakdowns = 0;             // cycles ended by a happy breakdown
  bool stuck = false;             // the last cycle broke down at its first step
  double brk;
  const void* bjinv = nullptr;   // block-Jacobi inverses of this precision, if used
  const float* bjsc = nullptr;
  int rows = 0;                   // rows of the vectors (sites, or half of them when reduced)
  void* gb = nullptr;             // gbuf of the full lattice's stage 1
  const void* oinv = nullptr;     // odd-even reduction: A_o^{-1} blocks, odd-row temporary
  const float* oinvsc = nullptr;
  Z* ts = nullptr;

  // recycle_tmp = false: no U/C refresh buffers (members of a batched solve)
  Krylov(Op& op_, Variant& v, const SolveOpts& o_, DevBuf& ws_, DevBuf& sm_, int steps_max,
         hipStream_t st_, bool recycle_tmp = true)
      : op(op_), var(v), o(o_), p(v.prec), tm(v.sign * op_.mu), st(st_),
        N(v.schur ? op_.N() / 2 : op_.N()), ws(ws_), sm(sm_) {
    brk = (p == P64) ? 1e-14 : 1e-6;
    ortho_now = o.ortho;   // entry points that run cycles directly (Arnoldi)
    rows = v.schur ? op.V / 2 : op.V;
    if (v.schur) {
      if (!op.oddeven) throw InvalidArg("the odd-even reduction needs every lattice extent even");
      const Op::BJ& b = op.ensure_bj(v.sign, st);   // D_oo^{-1}: inverses of the odd self blocks
      oinv = bj_blocks(b, p);
      oinvsc = (p == P16S) ? b.sc16.as<float>() : nullptr;
      ts = static_cast<Z*>(op.tmp_s(p));
    }
    gb = op.gbuf(p);   // full-lattice partials, or the single-read pair's hp
    if (v.bj) {
      const Op::BJ& b = op.ensure_bj(v.sign, st);
      bjinv = bj_blocks(b, p);
      bjsc = (p == P16S) ? b.sc16.as<float>() : nullptr;
    }
    const KrylovSizes ks = krylov_sizes(N, sizeof(Z), o.k, o.d, steps_max, recycle_tmp);
    kmax = ks.kmax;
    ldh = ks.ldh;
    nbasis = ks.nbasis;
    const int ktmp = ks.ktmp, nz = ks.nz, kz = ks.kz;
    ws.ensure(ks.ws_bytes);
    Z* base = ws.as<Z>();
    Vb = base;
    Ctmp = Vb + size_t(nbasis) * N;
    Utmp = Ctmp + size_t(ktmp) * N;
    Z* after = Utmp + size_t(ktmp) * N;
    if (nz) {
      Zb = after;
      MUtmp = Zb + size_t(nz) * N;
      after = MUtmp + size_t(kz) * N;
    }
    prod = after;
    ybuf = prod + N;
    tmp = ybuf + N;
    tmp2 = tmp + N;
    rhat = tmp2 + N;
    rtrue = rhat + N;
    ta = rtrue + N;
    tb = ta + N;
    // small area (doubles)
    const size_t q = size_t(kmax + ldh + 4);
    sm.ensure(ks.sm_bytes);
    double* d = sm.as<double>();
    res1 = d;
    res2 = res1 + 2 * q;
    nrm = res2 + 2 * q;
    scal = nrm + 4;  // inv_h, est
    coef = scal + 4;
    double* after_coef = coef + 2 * size_t(std::max(kmax + ldh + 2, 1)) * std::max(kmax, 2);
    ad.ldh = ldh;
    ad.ldb = std::max(kmax, 1);
    ad.H = after_coef;
    ad.Bk = ad.H + 2 * size_t(ldh) * ldh;
    ad.giv = ad.Bk + 2 * size_t(ad.ldb) * ldh;
    double* end = ad.giv + 2 * 3 * size_t(ldh + 1);
    ad.inv_h = scal;
    ad.est = scal + 1;
    int* ip = reinterpret_cast<int*>(end + 8);
    ad.done = ip;
    ad.jdone = ip + 1;
    ad.brk_flag = ip + 2;
  }

  Z* V(int j) const { return Vb + size_t(j) * N; }
  Z* Uv() const { return var.U.as<Z>(); }
  Z* Cv() const { return var.C.as<Z>(); }
  Z* MUv() const { return var.MU.as<Z>(); }
  Z* Zj(int j) const { return Zb + size_t(j) * N; }
  bool zstore() const { return Zb != nullptr && has_poly(); }

  // Stage 1 of one full-lattice apply into gb.
  void stage(const Z* in, const int* done) {
    stage1(op, p, op.n, op.V, op.blocks(p), op.scales(p), in, gb, op.nbr.as<int>(), tm, done, st);
  }

  // One apply of the reduced operator S = A_e - D_eo A_o^{-1} D_oe on compressed
  // even vectors (Sec. 2.2, factored form) with the D_eo kernel's epilogue
  // (0 store, 1 first chain step, 2 later chain step, 3 residual).  Its
  // epilogue reads and writes only the row it computes, so out may alias in.
  // With block Jacobi (B = D_ee, Sec. 3.2) epilogues 0-2 act on B^{-1} S in:
  // the inverses of the even self blocks replace them in the D_eo kernel.
  // The residual epilogue (3) always takes S itself.
  void reduced(const Z* in, int epi, Z* out, const Z* e, Z* y, z64 c0, z64 ca, z64 cb,
               const int* done) {
    const bool lbj = bjinv && epi != 3;
    if (reduced_single_read(p, op.n)) {
      reduced_scatter(op, p, oinv, oinvsc, in, gb, done, st);
      reduced_gather(op, p, epi, lbj ? bjinv : nullptr, lbj ? bjsc : nullptr, in, gb, tm, out, e,
                     y, c0, ca, cb, done, st);
      return;
    }
    reduced_oe(op, p, oinv, oinvsc, in, ts, done, st);
    reduced_eo(op, p, epi, lbj ? bjinv : nullptr, lbj ? bjsc : nullptr, in, ts, tm, out, e, y,
               c0, ca, cb, done, st);
  }

  // A~ in = (B^{-1}) D in (one matvec)
  void A(const Z* in, Z* out, const int* done) {
    if (var.schur) {
      const z64 z = mk(0.0, 0.0);
      reduced(in, 0, out, nullptr, nullptr, z, z, z, done);
      ++matvecs;
      return;
    }
    stage(in, done);
    if (bjinv) launch_bj_gather_store(p, op.n, rows, bjinv, bjsc, gb, out, done, st);
    else launch_gather_store(p, op.n, rows, gb, out, done, st);
    ++matvecs;
  }

  // rhat = B^{-1} r (or a copy without block Jacobi); on the reduced system
  // B = D_ee, the even rows' self blocks
  void left_precondition(const Z* r, Z* out) {
    if (bjinv && var.schur)
      launch_bj_rows(p, op.n, rows, op.esite.as<int>(), bjinv, bjsc, r, out, st);
    else if (bjinv) launch_bj_vec(p, op.n, rows, bjinv, bjsc, r, out, st);
    else launch_copy_words(r, out, N * sizeof(Z), st);
  }

  bool has_poly() const { return var.d > 1 && int(var.theta.size()) > 1; }

  // out = q(A~) in  (Newton-like form, d-1 matvecs); out must differ from in
  void Q(const Z* in, Z* out, const int* done) {
    const auto& th = var.theta;
    const int d = int(th.size());
    auto inv = [](cd t) { const cd r = 1.0 / t; return mk(r.real(), r.imag()); };
    if (d <= 1) {
      const z64 c = (d == 1) ? inv(th[0]) : mk(1.0, 0.0);
      launch_cscale(p, in, out, N, c, done, st);
      return;
    }
    // i = 1: prod = v - A v / theta_0;  y = v / theta_0 + prod / theta_1
    if (var.schur) {
      reduced(in, 1, prod, in, out, inv(th[0]), inv(th[0]), inv(th[1]), done);
      ++matvecs;
      for (int i = 2; i < d; ++i) {
        reduced(prod, 2, prod, nullptr, out, mk(0.0, 0.0), inv(th[i - 1]), inv(th[i]), done);
        ++matvecs;
      }
      return;
    }
    stage(in, done);
    if (bjinv)
      launch_bj_gather_poly_first(p, op.n, rows, bjinv, bjsc, gb, in, prod, out, inv(th[0]),
                                  inv(th[0]), inv(th[1]), done, st);
    else
      launch_gather_poly_first(p, op.n, rows, gb, in, prod, out, inv(th[0]), inv(th[0]),
                               inv(th[1]), done, st);
    ++matvecs;
    for (int i = 2; i < d; ++i) {
      stage(prod, done);
      if (bjinv)
        launch_bj_gather_poly(p, op.n, rows, bjinv, bjsc, gb, prod, out, inv(th[i - 1]),
                              inv(th[i]), done, st);
      else
        launch_gather_poly(p, op.n, rows, gb, prod, out, inv(th[i - 1]), inv(th[i]), done, st);
      ++matvecs;
    }
  }

  // out = A~ q(A~) in
  void Ahat(const Z* in, Z* out, const int* done) {
    if (!has_poly()) {
      A(in, out, done);
      return;
    }
    Q(in, ybuf, done);
    A(ybuf, out, done);
  }

  // r = b - D x (true residual in the variant's precision); returns ||r||
  double true_resid(const Z* x, const Z* b, Z* r) {
    if (var.schur) {
      const z64 z = mk(0.0, 0.0);
      reduced(x, 3, r, b, nullptr, z, z, z, nullptr);
      launch_norm2(p, r, N, op.red(), nrm, st);
    } else {
      stage(x, nullptr);
      launch_gather_resid(p, op.n, rows, gb, b, r, op.red(), nrm, st);
    }
    ++matvecs;
    double h;
    op.hs.read(&h, nrm, sizeof(double), st);
    op.hs.wait(st);
    return std::sqrt(std::max(h, 0.0));
  }

  double norm(const Z* x) {
    launch_norm2(p, x, N, op.red(), nrm, st);
    double h;
    op.hs.read(&h, nrm, sizeof(double), st);
    op.hs.wait(st);
    return std::sqrt(std::max(h, 0.0));
  }

  // Gram-Schmidt of V(j+1) against [C, V(0..j)] (classical, applied twice),
  // then the bookkeeping kernel and normalisation.
  void orth_step(int j, int kC, int steps, double target) {
    Z* w = V(j + 1);
    const Z* Cb = kC ? Cv() : nullptr;
    if (ortho_now == 1) {
      // single-sync process (Sec. 3.5): one reduction yields the coefficients
      // and ||A v_j||^2, h_{j+1,j} follows from their difference, and the
      // update and normalisation are one pass
      launch_multidot(p, Cb, kC, V(0), j + 1, N, w, 1, op.red(), res1, ad.done, st);
      launch_arnoldi_finish(ad, steps, kC, j, res1, nullptr, nullptr, target, brk, st);
      launch_multiaxpy_scaled(p, w, Cb, kC, V(0), j + 1, N, res1, ad.inv_h, ad.jdone, j, st);
      return;
    }
    launch_multidot(p, Cb, kC, V(0), j + 1, N, w, 1, op.red(), res1, ad.done, st);
    launch_multiaxpy(p, w, Cb, kC, V(0), j + 1, N, res1, 0, op.red(), nrm, ad.done, st);
    launch_multidot(p, Cb, kC, V(0), j + 1, N, w, 0, op.red(), res2, ad.done, st);
    launch_multiaxpy(p, w, Cb, kC, V(0), j + 1, N, res2, 1, op.red(), nrm, ad.done, st);
    launch_arnoldi_finish(ad, steps, kC, j, res1, res2, nrm, target, brk, st);
    launch_scale_step(p, w, N, ad.inv_h, ad.jdone, j, st);
  }

  struct CycleOut {
    int jd = 0;
    bool breakdown = false;
    double est = 0;
    double beta = 0;  // norm of the start vector
    Mat H;   // (jd+1) x jd
    Mat Bk;  // kC x jd
  };

  // One Arnoldi cycle of up to `steps` steps of A^ from rv (norm beta), with
  // deflation against the first kC columns of C.  The device stops the cycle
  // when the least-squares residual estimate reaches `target` (not before
  // min_steps steps) or on breakdown.  beta < 0: the norm is on the device
  // (nrm[2], its reciprocal nrm[3]) and is read back with the cycle's results.
  CycleOut cycle(const Z* rv, double beta, int steps, int kC, double target, int min_steps) {
    const bool dev_beta = beta < 0.0;
    if (dev_beta) {
      launch_scale(p, rv, V(0), N, nrm + 3, 0.0, nullptr, st);
      launch_arnoldi_init(ad, 0.0, st, nrm + 2);
    } else {
      launch_scale(p, rv, V(0), N, nullptr, 1.0 / beta, nullptr, st);
      launch_arnoldi_init(ad, beta, st);
    }
    // The host enqueues the cycle in chunks of about a millisecond of device
    // work and stays at most two chunks ahead; once the device has set the stop
    // flag no further chunks are enqueued (the steps already queued past the
    // stopping one exit at entry).  With one step per chunk, when the estimate
    // of the finished step extrapolated geometrically reaches the target, the
    // host waits for the running step before enqueueing the next, which then
    // is not enqueued at all if that step converged.
    const double per_step = double(N) * (has_poly() ? double(var.theta.size()) : 1.0);
    const int chunk = std::max(1, std::min(steps, int(std::ceil(1.0e6 / per_step))));
    op.sig.ensure();
    op.sig.ensure_est(steps);
    *op.sig.host = 0;
    ad.hdone = op.sig.dev;
    ad.hest = op.sig.est_dev;
    double last_est = beta;
    int nchunk = 0, enqueued = 0;
    // the whole cycle in one piece: replay it as a captured graph when asked
    if (o.graphs && chunk >= steps && min_steps == 0 && target >= 0.0 && !op.prof.on &&
        !op.graphs.broken && graph_cycle(kC, steps, target)) {
      enqueued = steps;
    } else {
      enqueue_steps(kC, steps, target, min_steps, chunk, beta, enqueued, nchunk, last_est);
    }
    ad.hdone = nullptr;
    ad.hest = nullptr;
    ad.target_dev = nullptr;
    op.prof.tag = -1;
    return finish_cycle(kC, enqueued, beta, dev_beta);
  }

  // Enqueue the steps of a cycle in chunks of about a millisecond of device
  // work, paced by events (see cycle()).
  void enqueue_steps(int kC, int steps, double target, int min_steps, int chunk, double beta,
                     int& enqueued, int& nchunk, double& last_est) {
    last_est = beta;
    for (int j = 0; j < steps; ++j) {
      op.prof.tag = j;
      if (zstore()) {            // keep z_j = q(A~) v_j for the update of x
        Q(V(j), Zj(j), ad.done);
        A(Zj(j), V(j + 1), ad.done);
      } else {
        Ahat(V(j), V(j + 1), ad.done);
      }
      orth_step(j, kC, steps, (j + 1 < min_steps) ? -1.0 : target);
      enqueued = j + 1;
      if ((j + 1) % chunk == 0 && j + 1 < steps) {
        DC_HIP(hipEventRecord(op.sig.ev[nchunk & 1], st));
        if (nchunk >= 1) {
          DC_HIP(hipEventSynchronize(op.sig.ev[(nchunk - 1) & 1]));
          if (__atomic_load_n(op.sig.host, __ATOMIC_ACQUIRE)) break;
          if (chunk == 1 && target >= 0.0 && j + 1 >= min_steps) {
            // step j - 1 has finished: its estimate is final
            const double e = static_cast<volatile const double*>(op.sig.est_host)[j - 1];
            const double ratio = last_est > 0.0 ? std::min(1.0, e / last_est) : 1.0;
            last_est = e;
            if (e * ratio <= target) {
              DC_HIP(hipEventSynchronize(op.sig.ev[nchunk & 1]));
              if (__atomic_load_n(op.sig.host, __ATOMIC_ACQUIRE)) break;
            }
          }
        }
        ++nchunk;
      }
    }
  }

  // The steps of one cycle (no pacing) as a HIP graph: looked up by the
  // arguments its kernels capture, else recorded on the capture stream.  The
  // stopping target goes to device memory first (the finishing kernel reads
  // it there).  Returns false, and stays eager from then on, if capture fails.
  bool graph_cycle(int kC, int steps, double target) {
    double* tdev = nrm + 1;   // free slot of the small area (nrm[0] and nrm[2..3] are used)
    op.hs.write(tdev, &target, sizeof(double), st);
    ad.target_dev = tdev;
    const std::vector<uintptr_t> key = {
        uintptr_t(&var), uintptr_t(var.poly_serial), uintptr_t(op.version), uintptr_t(ws.p),
        uintptr_t(sm.p), uintptr_t(var.C.p), uintptr_t(kC), uintptr_t(steps),
        uintptr_t(ortho_now), uintptr_t(zstore()), uintptr_t(p), uintptr_t(ad.hdone),
        uintptr_t(ad.hest), uintptr_t(var.theta.size()), uintptr_t(bjinv), uintptr_t(ts),
        uintptr_t(gb), uintptr_t(oinv), uintptr_t(op.blocks(p))};
    hipGraphExec_t exec = op.graphs.find(key);
    if (!exec) {
      GraphCache& gc = op.graphs;
      if (!gc.cap && hipStreamCreateWithFlags(&gc.cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        gc.cap = nullptr;
        gc.broken = true;
        ad.target_dev = nullptr;
        return false;
      }
      if (hipStreamBeginCapture(gc.cap, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipGetLastError();
        gc.broken = true;
        ad.target_dev = nullptr;
        return false;
      }
      const hipStream_t saved = st;
      const long mv_saved = matvecs;   // recording runs nothing
      st = gc.cap;
      bool ok = true;
      try {
        int enq = 0, nch = 0;
        double le = 0.0;
        enqueue_steps(kC, steps, target, 0, steps, 1.0, enq, nch, le);
      } catch (const std::exception&) {
        ok = false;
      }
      st = saved;
      matvecs = mv_saved;
      hipGraph_t graph = nullptr;
      if (hipStreamEndCapture(gc.cap, &graph) != hipSuccess || !ok || !graph) {
        (void)hipGetLastError();
        if (graph) (void)hipGraphDestroy(graph);
        gc.broken = true;
        ad.target_dev = nullptr;
        return false;
      }
      if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(graph);
        gc.broken = true;
        ad.target_dev = nullptr;
        return false;
      }
      gc.add(key, graph, exec);
      ++gc.captured;
    }
    DC_HIP(hipGraphLaunch(exec, st));
    ++op.graphs.launched;
    // the applications the replayed steps make, as the eager enqueue counts them
    matvecs += long(steps) * (has_poly() ? long(var.theta.size()) : 1L);
    return true;
  }

  CycleOut finish_cycle(int kC, int enqueued, double beta, bool dev_beta) {
    CycleOut c;
    int flags[3];
    op.hs.read(flags, ad.done, 3 * sizeof(int), st);
    double est;
    op.hs.read(&est, ad.est, sizeof(double), st);
    if (dev_beta) op.hs.read(&beta, nrm + 2, sizeof(double), st);
    // columns 0 .. enqueued-1 hold every step that can have run
    std::vector<double>& Hh = Hh_;
    std::vector<double>& Bh = Bh_;
    const size_t hcols = size_t(std::max(enqueued, 1));
    if (Hh.size() < 2 * size_t(ldh) * hcols) Hh.resize(2 * size_t(ldh) * hcols);
    op.hs.read(Hh.data(), ad.H, 2 * size_t(ldh) * hcols * sizeof(double), st);
    if (kC) {
      if (Bh.size() < 2 * size_t(ad.ldb) * hcols) Bh.resize(2 * size_t(ad.ldb) * hcols);
      op.hs.read(Bh.data(), ad.Bk, 2 * size_t(ad.ldb) * hcols * sizeof(double), st);
    }
    op.hs.wait(st);
    c.jd = flags[1];
    c.breakdown = flags[2] != 0;
    if (c.breakdown) ++breakdowns;
    if (c.breakdown && ortho_now == 1) ss_off = true;
    op.prof.end_cycle(c.jd);
    // steps past the stopping one were enqueued but exited at entry
    matvecs -= long(enqueued - c.jd) * (has_poly() ? long(var.theta.size()) : 1L);
    c.est = est;
    c.beta = beta;
    c.H = Mat(c.jd + 1, c.jd);
    for (int jj = 0; jj < c.jd; ++jj)
      for (int i = 0; i <= jj + 1; ++i)
        c.H(i, jj) = cd(Hh[2 * (size_t(jj) * ldh + i)], Hh[2 * (size_t(jj) * ldh + i) + 1]);
    c.Bk = Mat(kC, c.jd);
    for (int jj = 0; jj < c.jd; ++jj)
      for (int i = 0; i < kC; ++i)
        c.Bk(i, jj) = cd(Bh[2 * (size_t(jj) * ad.ldb + i)], Bh[2 * (size_t(jj) * ad.ldb + i) + 1]);
    return c;
  }

  void upload_coef(const std::vector<cd>& c) {
    std::vector<double> h(2 * c.size());
    for (size_t i = 0; i < c.size(); ++i) {
      h[2 * i] = c[i].real();
      h[2 * i + 1] = c[i].imag();
    }
    op.hs.write(coef, h.data(), h.size() * sizeof(double), st);
  }

  // x += q(A~) (sum_q c_q basis_q)
  void add_preconditioned(Z* x, const Z* b0, int q0, const Z* b1, int q1,
                          const std::vector<cd>& c) {
    upload_coef(c);
    if (!has_poly()) {
      launch_combine(p, b0, q0, b1, q1, N, coef, 1, x, 1, st);
      return;
    }
    launch_combine(p, b0, q0, b1, q1, N, coef, 1, tmp, 0, st);
    Q(tmp, tmp2, nullptr);
    launch_axpy(p, mk(1.0, 0.0), tmp2, x, N, st);
  }

  void ensure_recycle_storage() {
    const size_t vb = N * sizeof(Z) * size_t(std::max(kmax, 1));
    var.U.ensure(vb);
    var.C.ensure(vb);
    if (zstore()) var.MU.ensure(vb);
  }

  // x += q(A~) ([U] c_U + V_jd c_V) after a cycle: from the stored z_j (and
  // MU = q(A~) U) when available, else by applying q to the combination
  void update_x(Z* x, int kk, int jd, const std::vector<cd>& c) {
    if (zstore() && (kk == 0 || var.mu_ok)) {
      upload_coef(c);
      launch_combine(p, kk ? MUv() : nullptr, kk, Zj(0), jd, N, coef, 1, x, 1, st);
      return;
    }
    add_preconditioned(x, kk ? Uv() : nullptr, kk, V(0), jd, c);
  }

  void refresh_unorm() {
    var.unorm.assign(var.kcur, 1.0);
    if (var.kcur == 0) return;
    launch_colnorm2(p, Uv(), var.kcur, N, op.red(), res1, st);  // res1 holds >= kmax doubles
    op.hs.read(var.unorm.data(), res1, sizeof(double) * size_t(var.kcur), st);
    op.hs.wait(st);
    for (double& u : var.unorm) u = std::sqrt(std::max(u, 0.0));
  }

  // New recycle space from an (unpreconditioned-residual) GMRES cycle:
  // harmonic Ritz vectors of H_m for the k smallest |theta|.
  void construct_recycle(const CycleOut& c) {
    const int jd = c.jd;
    const int kk = std::min(kmax, jd);
    if (kk <= 0) return;
    std::vector<cd> th;
    Mat Zv;
    if (!harmonic_ritz(c.H, th, &Zv)) return;
    const auto idx = smallest_k(th, kk);
    Mat P(jd, kk);
    for (int t = 0; t < kk; ++t)
      for (int i = 0; i < jd; ++i) P(i, t) = Zv(i, idx[t]);
    Mat Qm, R;
    qr_thin(matmul(c.H, P), Qm, R);
    const Mat PR = matmul(P, tri_inverse(R));
    ensure_recycle_storage();
    // C = V_{jd+1} Q ; U = V_jd P R^{-1}
    std::vector<cd> cq(size_t(kk) * (jd + 1)), cu(size_t(kk) * jd);
    for (int r = 0; r < kk; ++r) {
      for (int q = 0; q <= jd; ++q) cq[size_t(r) * (jd + 1) + q] = Qm(q, r);
      for (int q = 0; q < jd; ++q) cu[size_t(r) * jd + q] = PR(q, r);
    }
    upload_coef(cq);
    launch_combine(p, nullptr, 0, V(0), jd + 1, N, coef, kk, Cv(), 0, st);
    upload_coef(cu);
    launch_combine(p, nullptr, 0, V(0), jd, N, coef, kk, Uv(), 0, st);
    // q(A~) U by the same combination of the z_j
    if (zstore()) launch_combine(p, nullptr, 0, Zj(0), jd, N, coef, kk, MUv(), 0, st);
    var.mu_ok = zstore();
    var.kcur = kk;
    var.k_built = kmax;
    var.updates = 1;
    var.recycle_version = op.version;
    refresh_unorm();
  }

  // The single-sync process for the next cycle only where its Hessenberg does
  // not define the recycle space: the construction cycle and the cycles that
  // still refresh U, C (fewer than u updates) use Gram-Schmidt twice, since
  // the single-sync basis loses orthogonality over long cycles and a recycle
  // space built from it would stay inaccurate once frozen.
  void use_ortho(bool defines_recycle) {
    ortho_now = (o.ortho == 1 && !ss_off && !defines_recycle) ? 1 : 0;
  }

  // New right-hand side with a recycle space: x += q(A~) U C^H rhat;
  // rhat -= C C^H rhat.
  void deflate_start(Z* x) {
    launch_multidot(p, Cv(), var.kcur, nullptr, 0, N, rhat, 0, op.red(), res1, nullptr, st);
    launch_multiaxpy(p, rhat, Cv(), var.kcur, nullptr, 0, N, res1, 1, op.red(), nrm, nullptr, st);
    if (!has_poly()) {
      launch_combine(p, Uv(), var.kcur, nullptr, 0, N, res1, 1, x, 1, st);
    } else if (zstore() && var.mu_ok) {
      launch_combine(p, MUv(), var.kcur, nullptr, 0, N, res1, 1, x, 1, st);
    } else {
      launch_combine(p, Uv(), var.kcur, nullptr, 0, N, res1, 1, tmp, 0, st);
      Q(tmp, tmp2, nullptr);
      launch_axpy(p, mk(1.0, 0.0), tmp2, x, N, st);
    }
  }

  // Solve D x = b to relative true residual tol; b, x device vectors of this
  // precision.  Returns true if converged.
  bool solve(const Z* b, Z* x, double tol, bool use_x0, int max_cycles, SolveStats& stt,
             double& relres) {
    const long mv0 = matvecs;
    if (!use_x0) launch_zero(p, x, N, st);
    const double bn = bn_hint > 0.0 ? bn_hint : norm(b);
    if (bn == 0.0) {
      launch_zero(p, x, N, st);
      relres = 0.0;
      return true;
    }
    // matrix changed, or a different recycle dimension requested: rebuild lazily
    if (var.recycle_version != op.version || var.k_built != kmax) {
      var.kcur = 0;
      var.updates = 0;
    }
    const int k = kmax;
    const int m = o.m;
    double rn = bn;                  // x = 0: the residual is b itself
    if (use_x0) rn = true_resid(x, b, rtrue);
    else launch_copy_words(b, rtrue, N * sizeof(Z), st);
    relres = rn / bn;
    if (relres <= tol) {
      stt.matvecs += int(matvecs - mv0);
      return true;
    }
    // left-preconditioned residual rhat = B^{-1} r; the least-squares estimates
    // track ||rhat||, so the in-cycle target is scaled by ||rhat|| / ||r||
    left_precondition(rtrue, rhat);
    double beta = bjinv ? norm(rhat) : rn;
    const double ratio = beta / rn;
    const double target_abs = tol * bn * ratio;
    int cycles = 0;
    bool converged = false;
    if (k > 0 && var.kcur > 0) {
      deflate_start(x);
      if (inner_est) {
        launch_norm_root(nrm, nrm + 2, st);   // ||rhat|| stays on the device
        beta = -1.0;
      } else {
        beta = norm(rhat);
      }
    } else if (k > 0) {
      // construction cycle: GMRES(m) of at least k steps
      const int steps = std::min(m, ldh - 2);
      use_ortho(true);
      CycleOut c = cycle(rhat, beta, steps, 0, target_abs, k);
      ++cycles;
      stt.iters += c.jd;
      std::vector<cd> e1(c.jd + 1, cd(0.0));
      e1[0] = beta;
      double lsres;
      const auto y = lstsq(c.H, e1, &lsres);
      update_x(x, 0, c.jd, y);
      // rhat = V_{jd+1} (beta e1 - H y)
      std::vector<cd> rr(c.jd + 1);
      const auto Hy = matmul(c.H, [&] { Mat t(c.jd, 1); for (int i = 0; i < c.jd; ++i) t(i, 0) = y[i]; return t; }());
      for (int i = 0; i <= c.jd; ++i) rr[i] = e1[i] - Hy(i, 0);
      upload_coef(rr);
      launch_combine(p, nullptr, 0, V(0), c.jd + 1, N, coef, 1, rhat, 0, st);
      stt.rel_res_est = lsres / bn;
      stt.rebuilt |= 2;
      construct_recycle(c);
      beta = norm(rhat);
    }
    double best = rn;
    int stall = 0;
    while (true) {
      // inner solves stop on the recursively updated (left-preconditioned)
      // residual, compared with the target on its own scale (ratio)
      const bool by_est = inner_est && k > 0 && var.kcur > 0;
      if (by_est && beta < 0.0) {
        // the deflated start's norm is on the device: straight to a cycle
        if (cycles >= max_cycles) break;
      } else {
        rn = by_est ? beta / ratio : true_resid(x, b, rtrue);
        relres = rn / bn;
        if (relres <= tol) {
          converged = true;
          break;
        }
        if (cycles >= max_cycles) break;
        if (rn < 0.99 * best) {
          best = rn;
          stall = 0;
        } else if (++stall >= 10 && o.ortho == 1 && k > 0 && var.kcur > 0) {
          // single-sync solves: the recursively updated residual no longer tracks
          // the true one (loss of orthogonality); restart from the true
          // residual, deflated, with Gram-Schmidt twice
          stall = 0;
          ss_off = true;
          if (by_est) rn = true_resid(x, b, rtrue);
          left_precondition(rtrue, rhat);
          deflate_start(x);
          beta = norm(rhat);
        }
      }
      if (k == 0 || var.kcur == 0) {
        // plain GMRES(m) cycle from the (left-preconditioned) true residual
        const int steps = std::min(m, ldh - 2);
        double b0 = rn;
        if (bjinv) {
          left_precondition(rtrue, rhat);
          b0 = norm(rhat);
        }
        use_ortho(false);
        CycleOut c = cycle(bjinv ? rhat : rtrue, b0, steps, 0, target_abs, 0);
        ++cycles;
        stt.iters += c.jd;
        std::vector<cd> e1(c.jd + 1, cd(0.0));
        e1[0] = b0;
        double lsres;
        const auto y = lstsq(c.H, e1, &lsres);
        stt.rel_res_est = lsres / bn;
        update_x(x, 0, c.jd, y);
        if (c.jd == 0) {        // immediate breakdown: nothing more to gain
          stuck = true;
          break;
        }
        continue;
      }
      // GCRO-DR cycle
      const int kk = var.kcur;
      const int steps = std::min(m - kk, ldh - 2);
      if (steps < 1) throw InvalidArg("GCRO-DR needs m > k");
      use_ortho(var.updates < o.u);
      CycleOut c = cycle(rhat, beta, steps, kk, target_abs, 0);
      ++cycles;
      stt.iters += c.jd;
      const int jd = c.jd;
      // G = [[D_k, B_k], [0, Hbar]], formed only when the residual update or
      // a refresh needs it
      Mat G;
      bool have_G = false;
      auto get_G = [&]() -> const Mat& {
        if (!have_G) {
          G = Mat(kk + jd + 1, kk + jd);
          for (int i = 0; i < kk; ++i) G(i, i) = 1.0 / var.unorm[i];
          for (int jj = 0; jj < jd; ++jj) {
            for (int i = 0; i < kk; ++i) G(i, kk + jj) = c.Bk(i, jj);
            for (int i = 0; i <= jj + 1; ++i) G(kk + i, kk + jj) = c.H(i, jj);
          }
          have_G = true;
        }
        return G;
      };
      double lsres;
      const auto y = gcrodr_lstsq(c.H, c.Bk, var.unorm, c.beta, &lsres);
      stt.rel_res_est = lsres / bn;
      // x += q(A~) Vhat y, Vhat = [U D_k, V_jd]
      std::vector<cd> cy(kk + jd);
      for (int i = 0; i < kk; ++i) cy[i] = y[i] / var.unorm[i];
      for (int i = 0; i < jd; ++i) cy[kk + i] = y[kk + i];
      update_x(x, kk, jd, cy);
      // inner solves: the least-squares residual is the norm the update of
      // rhat would give, so a converged cycle skips that update
      const bool est_conv = by_est && lsres <= target_abs;
      if (!est_conv) {
        // rhat -= What (G y), What = [C, V_{jd+1}]
        Mat ym(kk + jd, 1);
        for (int i = 0; i < kk + jd; ++i) ym(i, 0) = y[i];
        const Mat Gy = matmul(get_G(), ym);
        std::vector<cd> gy(kk + jd + 1);
        for (int i = 0; i < kk + jd + 1; ++i) gy[i] = Gy(i, 0);
        upload_coef(gy);
        launch_multiaxpy(p, rhat, Cv(), kk, V(0), jd + 1, N, coef, 1, op.red(), nrm, nullptr, st);
        double h;
        op.hs.read(&h, nrm, sizeof(double), st);
        op.hs.wait(st);
        beta = std::sqrt(std::max(h, 0.0));
      }
      if (var.updates < o.u && jd > 0) refresh_recycle(c, get_G());
      if (est_conv) {
        converged = true;
        relres = lsres / (bn * ratio);
        break;
      }
      if (jd == 0) {
        stuck = true;
        break;
      }
    }
    stt.cycles += cycles;
    stt.matvecs += int(matvecs - mv0);
    return converged;
  }

  // Refresh U, C from the generalised harmonic Ritz problem
  // G^H G z = theta G^H (What^H Vhat) z.
  void refresh_recycle(const CycleOut& c, const Mat& G) {
    const int kk = var.kcur, jd = c.jd;
    const int nr = kk + jd + 1, nc = kk + jd;
    // What^H Vhat = [[C^H U D_k, 0], [V^H U D_k, I]]
    Mat WV(nr, nc);
    // C^H U and V_{jd+1}^H U as two MFMA Gram products formed in FP64; the
    // buffer is sized for the longest cycle (jd + 1 <= m + 1), so later
    // refreshes reuse it: both results, then the chunk partials
    const size_t mr = size_t(std::max(nr - kk, o.m + 1));
    op.wvbuf.ensure(refresh_gram_bytes(kk, int(mr)));
    z64* sc = op.wvbuf.as<z64>();
    z64* sv = sc + size_t(kk) * kk;
    z64* part = sv + size_t(kk) * mr;
    const size_t cap = kRefreshGramParts * size_t(kk) * mr;
    launch_block_gram(p, Cv(), kk, Uv(), kk, N, part, sc, st, true, cap);
    launch_block_gram(p, V(0), jd + 1, Uv(), kk, N, part, sv, st, true, cap);
    std::vector<z64> hc(size_t(kk) * kk), hv(size_t(kk) * (jd + 1));
    op.hs.read(hc.data(), sc, hc.size() * sizeof(z64), st);
    op.hs.read(hv.data(), sv, hv.size() * sizeof(z64), st);
    op.hs.wait(st);
    for (int i = 0; i < kk; ++i)
      for (int r = 0; r < nr; ++r) {
        const z64 z = r < kk ? hc[size_t(i) * kk + r] : hv[size_t(i) * (jd + 1) + (r - kk)];
        WV(r, i) = cd(z.re, z.im) / var.unorm[i];
      }
    for (int jj = 0; jj < jd; ++jj) WV(kk + jj, kk + jj) = 1.0;
    const Mat GH = adjoint(G);
    Mat Bm = matmul(GH, WV);
    Mat Am = matmul(GH, G);
    // a failed dense problem leaves U, C as they are and freezes them (no
    // further refresh attempts in this or later solves)
    if (!lu_solve(Bm, Am)) {  // Am <- Bm^{-1} Am
      var.updates = o.u;
      ++refresh_failed;
      return;
    }
    std::vector<cd> th;
    Mat Zv;
    if (!eig(Am, th, &Zv)) {
      var.updates = o.u;
      ++refresh_failed;
      return;
    }
    const auto idx = smallest_k(th, kk);
    Mat P(nc, kk);
    for (int t = 0; t < kk; ++t)
      for (int i = 0; i < nc; ++i) P(i, t) = Zv(i, idx[t]);
    Mat Qm, R;
    qr_thin(matmul(G, P), Qm, R);
    const Mat PR = matmul(P, tri_inverse(R));
    // C_new = What Q (inputs C, V_{jd+1}); U_new = Vhat P R^{-1} (inputs U D_k, V_jd)
    std::vector<cd> cq(size_t(kk) * nr), cu(size_t(kk) * nc);
    for (int r = 0; r < kk; ++r) {
      for (int q = 0; q < nr; ++q) cq[size_t(r) * nr + q] = Qm(q, r);
      for (int q = 0; q < nc; ++q)
        cu[size_t(r) * nc + q] = (q < kk) ? PR(q, r) / var.unorm[q] : PR(q, r);
    }
    upload_coef(cq);
    launch_combine(p, Cv(), kk, V(0), jd + 1, N, coef, kk, Ctmp, 0, st);
    upload_coef(cu);
    launch_combine(p, Uv(), kk, V(0), jd, N, coef, kk, Utmp, 0, st);
    const bool mu = zstore() && var.mu_ok;
    if (mu) launch_combine(p, MUv(), kk, Zj(0), jd, N, coef, kk, MUtmp, 0, st);
    DC_HIP(hipMemcpyAsync(Cv(), Ctmp, size_t(kk) * N * sizeof(Z), hipMemcpyDeviceToDevice, st));
    DC_HIP(hipMemcpyAsync(Uv(), Utmp, size_t(kk) * N * sizeof(Z), hipMemcpyDeviceToDevice, st));
    if (mu) DC_HIP(hipMemcpyAsync(MUv(), MUtmp, size_t(kk) * N * sizeof(Z), hipMemcpyDeviceToDevice, st));
    var.mu_ok = mu;
    var.updates += 1;
    refresh_unorm();
  }
};

template <typename VR>
void build_poly(Op& op, Variant& var, const SolveOpts& o, hipStream_t st) {
  using Z = cx<VR>;
  SolveOpts po = o;
  po.ortho = 0;   // harmonic Ritz values from the Gram-Schmidt-twice Hessenberg
  // sized as the solve's workspace (po.k kept), so the solve reuses it; the
  // construction cycle below runs without deflation
  Krylov<VR> K(op, var, po, var.ws, var.sm, std::max(o.d, o.m), st);
  var.theta.clear();  // build with A~ itself (no polynomial yet)
  const size_t N = K.N;
  // start vector: caller's v0 (complex128) or a seeded Gaussian
  DevBuf v64;
  v64.ar = op.scratch_arena();
  v64.what = "polynomial start vector";
  const z64* src = static_cast<const z64*>(o.v0);
  if (!src) {
    v64.alloc(N * sizeof(z64));
    launch_gaussian(v64.as<z64>(), N, o.seed, 4u, st);
    src = v64.as<z64>();
  }
  if (var.prec == P64) {
    DC_HIP(hipMemcpyAsync(K.tmp, src, N * sizeof(z64), hipMemcpyDeviceToDevice, st));
  } else {
    launch_convert_64to32(src, reinterpret_cast<z32*>(K.tmp), N, op.n, 0, st);
  }
  const double beta = K.norm(K.tmp);
  if (beta == 0.0) throw InvalidArg("polynomial start vector is zero");
  auto c = K.cycle(K.tmp, beta, o.d, 0, -1.0, 0);
  std::vector<cd> th;
  if (c.breakdown) {
    Mat Hs = block(c.H, 0, 0, c.jd, c.jd);
    if (!eig(Hs, th, nullptr)) throw InvalidArg("eigenvalue iteration failed");
  } else {
    if (!harmonic_ritz(c.H, th, nullptr)) throw InvalidArg("harmonic Ritz computation failed");
  }
  for (const auto& t : th)
    if (!(std::abs(t) > 0.0) || !std::isfinite(t.real()) || !std::isfinite(t.imag()))
      throw InvalidArg("degenerate harmonic Ritz value");
  var.theta = leja_order(th);
  var.poly_version = op.version;
  ++var.poly_serial;
  (void)sizeof(Z);
}

}  // namespace

void ensure_poly(Op& op, Variant& var, const SolveOpts& o, hipStream_t st, SolveStats* stt) {
  if (o.d <= 1) {
    var.theta.clear();
    return;
  }
  if (var.poly_version == op.version && int(var.theta.size()) > 0) return;
  if (var.prec == P64) build_poly<double>(op, var, o, st);
  else build_poly<float>(op, var, o, st);
  if (stt) stt->rebuilt |= 1;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

void op_poly_set(Op& op, const SolveOpts& o, const std::vector<cd>& theta) {
  check_prec(op, o.prec);
  if (theta.empty() || int(theta.size()) != o.d) throw InvalidArg("d must equal the number of roots");
  for (const cd& t : theta)
    if (!(std::abs(t) > 0.0) || !std::isfinite(t.real()) || !std::isfinite(t.imag()))
      throw InvalidArg("polynomial roots must be finite and nonzero");
  Variant& var = op.variant(o.prec, +1, o.block_jacobi ? 1 : 0, o.d, o.schur);
  var.theta = theta;
  var.poly_version = op.version;
  ++var.poly_serial;
  // a recycle space built with another polynomial no longer satisfies C = A q(A) U
  var.kcur = 0;
  var.mu_ok = false;
}

int op_poly_setup(Op& op, const SolveOpts& o, hipStream_t st, std::vector<cd>& theta) {
  check_prec(op, o.prec);
  if (o.d < 1) throw InvalidArg("d must be >= 1");
  Variant& var = op.variant(o.prec, +1, o.block_jacobi ? 1 : 0, o.d, o.schur);
  var.poly_version = -1;
  if (var.prec == P64) build_poly<double>(op, var, o, st);
  else build_poly<float>(op, var, o, st);
  theta = var.theta;
  return int(theta.size());
}

void op_poly_apply(Op& op, const SolveOpts& o, const void* in, void* out, hipStream_t st) {
  check_prec(op, o.prec);
  if (!in || !out || in == out) throw InvalidArg("bad vector pointers");
  Variant& var = op.variant(o.prec, +1, o.block_jacobi ? 1 : 0, o.d, o.schur);
  if (var.poly_version != op.version) throw BadState("polynomial not built for this operator");
  if (var.prec == P64) {
    Krylov<double> K(op, var, o, var.ws, var.sm, std::max(o.m, o.d), st);
    K.Q(static_cast<const z64*>(in), static_cast<z64*>(out), nullptr);
  } else {
    Krylov<float> K(op, var, o, var.ws, var.sm, std::max(o.m, o.d), st);
    K.Q(static_cast<const z32*>(in), static_cast<z32*>(out), nullptr);
  }
}

int op_arnoldi(Op& op, const SolveOpts& o, const void* v, int steps, hipStream_t st,
               std::vector<cd>& hbar) {
  check_prec(op, o.prec);
  if (!v || steps < 1) throw InvalidArg("bad Arnoldi arguments");
  Variant& var = op.variant(o.prec, +1, o.block_jacobi ? 1 : 0, o.d, o.schur);
  ensure_poly(op, var, o, st, nullptr);
  auto run = [&](auto tag) -> int {
    using VR = decltype(tag);
    Krylov<VR> K(op, var, o, var.ws, var.sm, std::max(steps, o.d), st);
    const z64* src = static_cast<const z64*>(v);
    if (var.prec == P64) DC_HIP(hipMemcpyAsync(K.tmp, src, K.N * sizeof(z64), hipMemcpyDeviceToDevice, st));
    else launch_convert_64to32(src, reinterpret_cast<z32*>(K.tmp), K.N, op.n, 0, st);
    const double beta = K.norm(K.tmp);
    auto c = K.cycle(K.tmp, beta, steps, 0, -1.0, 0);
    hbar.assign(size_t(steps + 1) * steps, cd(0.0));
    for (int j = 0; j < c.jd; ++j)
      for (int i = 0; i <= j + 1; ++i) hbar[size_t(j) * (steps + 1) + i] = c.H(i, j);
    return c.jd;
  };
  if (var.prec == P64) return run(double(0));
  return run(float(0));
}

// ||b - D x|| / ||b|| (or with D^H) in FP64, using the handle's scratch.
static double fp64_relres(Op& op, const z64* x, const z64* b, int adjoint, hipStream_t st) {
  const size_t N = op.N();
  op.t64a.ensure(N * sizeof(z64));
  op.t64b.ensure(N * sizeof(z64));
  double* d = op.scal.as<double>();
  launch_norm2(P64, b, N, op.red(), d, st);
  if (!adjoint) {
    stage1(op, P64, op.n, op.V, op.blocks(P64), nullptr, x, op.gbuf(P64),
                        op.nbr.as<int>(), op.mu, nullptr, st);
    launch_gather_resid(P64, op.n, op.V, op.gbuf(P64), b, op.t64a.p, op.red(), d + 1, st);
  } else {
    op_apply(op, P64, 1, x, op.t64a.p, st);
    launch_scale(P64, op.t64a.p, op.t64b.p, N, nullptr, -1.0, nullptr, st);
    launch_axpy(P64, mk(1.0, 0.0), b, op.t64b.p, N, st);
    launch_norm2(P64, op.t64b.p, N, op.red(), d + 1, st);
  }
  double h[2];
  op.hs.read(h, d, 2 * sizeof(double), st);
  op.hs.wait(st);
  const double bn = std::sqrt(std::max(h[0], 0.0)), rn = std::sqrt(std::max(h[1], 0.0));
  return bn > 0 ? rn / bn : 0.0;
}

// ||x - x_ref|| / ||x_ref|| in FP64 (full-lattice vectors), using the handle's scratch.
static double fp64_relerr(Op& op, const z64* x, const z64* xref, hipStream_t st) {
  const size_t N = op.N();
  op.t64a.ensure(N * sizeof(z64));
  double* d = op.scal.as<double>();
  launch_copy_words(x, op.t64a.p, N * sizeof(z64), st);
  launch_axpy(P64, mk(-1.0, 0.0), xref, op.t64a.p, N, st);
  launch_norm2(P64, op.t64a.p, N, op.red(), d, st);
  launch_norm2(P64, xref, N, op.red(), d + 1, st);
  double h[2];
  op.hs.read(h, d, 2 * sizeof(double), st);
  op.hs.wait(st);
  return h[1] > 0.0 ? std::sqrt(std::max(h[0], 0.0) / h[1]) : std::sqrt(std::max(h[0], 0.0));
}

int op_solve(Op& op, const SolveOpts& o, int adjoint, int n_rhs, const void* b, void* x,
             const double* tol, int use_x0, hipStream_t st, SolveStats* stats) {
  check_prec(op, o.prec);
  if (!b || !x || !tol || n_rhs < 0) throw InvalidArg("null pointer or negative n_rhs");
  if (o.m < 1 || o.k < 0 || o.max_cycles < 0 || o.u < 0) throw InvalidArg("bad solver options");
  if (o.k > 0 && o.k >= o.m) throw InvalidArg("GCRO-DR needs m > k");
  if (o.outer && o.prec == P64) throw InvalidArg("the outer loop wraps a reduced-precision solve");
  if (o.outer && (o.m_outer < 1 || o.max_outer < 1 || !(o.inner_tol > 0.0)))
    throw InvalidArg("bad outer-loop options");
  for (int r = 0; r < n_rhs; ++r)
    if (!(tol[r] > 0.0)) throw InvalidArg("tolerances must be positive");
  if (o.schur && !op.oddeven) throw InvalidArg("the odd-even reduction needs every lattice extent even");
  const int sign = (adjoint && op.mu != 0.0) ? -1 : +1;
  const size_t Nfull = op.N();
  // system size: the full lattice, or the even sites of the reduced system
  const size_t N = o.schur ? Nfull / 2 : Nfull;
  const int half = op.V / 2;
  int all_ok = 1, worst = 1;
  for (int r = 0; r < n_rhs; ++r) {
    const auto t0 = std::chrono::steady_clock::now();
    SolveStats s;
    const z64* br = static_cast<const z64*>(b) + size_t(r) * Nfull;
    z64* xr = static_cast<z64*>(x) + size_t(r) * Nfull;
    Variant& var = op.variant(o.prec, sign, o.block_jacobi ? 1 : 0, o.d, o.schur);
    const auto ts = std::chrono::steady_clock::now();
    ensure_poly(op, var, o, st, &s);
    s.t_setup_ms = ms_since(ts);
    // adjoint through Gamma5: x = Gamma5 solve(D(-mu), Gamma5 b)
    const z64* bb = br;
    z64* xx = xr;
    if (adjoint) {
      op.t64a.ensure(Nfull * sizeof(z64));
      op.t64b.ensure(Nfull * sizeof(z64));
      launch_gamma5(P64, br, op.t64a.p, op.V, op.n, st);
      if (use_x0) launch_gamma5(P64, xr, op.t64b.p, op.V, op.n, st);
      bb = op.t64a.as<z64>();
      xx = op.t64b.as<z64>();
    }
    // odd-even reduction (Sec. 2.2): solve S x_e = b_e - D_eo A_o^{-1} b_o on
    // compressed even vectors to tol ||b|| / ||b^_e|| (the odd rows of the full
    // residual vanish), then x_o = A_o^{-1} b_o - A_o^{-1} D_oe x_e
    const z64* bfull = bb;
    z64* xfull = xx;
    double tol_r = tol[r];
    DevBuf& be = op.rbe;
    DevBuf& bo = op.rbo;
    DevBuf& xe = op.rxe;
    DevBuf& to = op.rto;
    const int* esite = op.esite.as<int>();
    const int* osite = op.osite.as<int>();
    const double tm = sign * op.mu;
    const void* oinv = nullptr;
    const z64 z0 = mk(0.0, 0.0);
    if (o.schur) {
      oinv = op.ensure_bj(sign, st).b64.p;
      be.ensure(N * sizeof(z64));
      bo.ensure(N * sizeof(z64));
      xe.ensure(N * sizeof(z64));
      to.ensure(N * sizeof(z64));
      launch_oddeven_split(P64, op.n, half, esite, osite, const_cast<z64*>(bfull), be.p, bo.p, 0, st);
      if (use_x0) launch_oddeven_split(P64, op.n, half, esite, osite, xfull, xe.p, nullptr, 0, st);
      launch_bj_rows(P64, op.n, half, osite, oinv, nullptr, bo.p, to.p, st);   // A_o^{-1} b_o
      // -D_eo A_o^{-1} b_o (set-up and recovery launches are not profiled)
      launch_reduced_eo(P64, 0, op.n, op.V, op.blocks(P64), nullptr, nullptr, nullptr, nullptr, to.p,
                        op.nbr.as<int>(), esite, tm, op.tmp_s(P64), nullptr, nullptr, z0, z0, z0,
                        nullptr, st);
      launch_axpy(P64, mk(1.0, 0.0), op.tmp_s(P64), be.p, N, st);   // be := b^_e
      double nb[2];
      launch_norm2(P64, bfull, Nfull, op.red(), op.scal.as<double>(), st);
      launch_norm2(P64, be.p, N, op.red(), op.scal.as<double>() + 1, st);
      op.hs.read(nb, op.scal.p, 2 * sizeof(double), st);
      op.hs.wait(st);
      if (nb[1] > 0.0) tol_r = tol[r] * std::sqrt(nb[0] / nb[1]);
      bb = be.as<z64>();
      xx = xe.as<z64>();
    }
    double rel = 0.0;
    bool stuck = false;   // stopped on a breakdown at the first step of a cycle
    auto collect = [&](const auto& K) {
      s.breakdowns += K.breakdowns;
      s.refresh_failed += K.refresh_failed;
    };
    if (o.prec == P64) {
      Krylov<double> K(op, var, o, var.ws, var.sm, o.m, st);
      K.solve(bb, xx, tol_r, use_x0 != 0, o.max_cycles, s, rel);
      collect(K);
      stuck = K.stuck;
    } else if (!o.outer) {
      Krylov<float> K(op, var, o, var.ws, var.sm, o.m, st);
      op.t32a.ensure(N * sizeof(z32));
      op.t32b.ensure(N * sizeof(z32));
      z32* b32 = op.t32a.as<z32>();
      z32* x32 = op.t32b.as<z32>();
      launch_convert_64to32(bb, b32, N, op.n, 0, st);
      if (use_x0) launch_convert_64to32(xx, x32, N, op.n, 0, st);
      K.solve(b32, x32, tol_r, use_x0 != 0, o.max_cycles, s, rel);
      collect(K);
      stuck = K.stuck;
      launch_convert_32to64(x32, xx, N, op.n, 0, st);
    } else {
      // FP64 flexible GMRES outer loop; its preconditioner is the
      // reduced-precision solve of the variant (polynomial + recycling)
      SolveOpts oo = o;
      oo.k = 0;
      oo.d = 0;
      oo.m = o.m_outer;
      oo.ortho = 0;   // the FP64 outer loop keeps Gram-Schmidt twice
      Variant& vo = op.variant(P64, sign, 0, -1, o.schur);  // holds the outer workspace
      Krylov<double> KO(op, vo, oo, vo.ws, vo.sm, o.m_outer, st);
      op.zouter.ensure(size_t(o.m_outer) * N * sizeof(z64));
      z64* Zb = op.zouter.as<z64>();
      Krylov<float> KI(op, var, o, var.ws, var.sm, o.m, st);
      KI.inner_est = true;
      KI.bn_hint = 1.0;   // the right-hand sides are the outer basis vectors
      op.t32a.ensure(N * sizeof(z32));
      op.t32b.ensure(N * sizeof(z32));
      z32* b32 = op.t32a.as<z32>();
      z32* x32 = op.t32b.as<z32>();
      if (!use_x0) launch_zero(P64, xx, N, st);
      const double bn = KO.norm(bb);
      int outer_done = 0;
      // residual of the current x: b itself for a zero start; after a cycle
      // whose FP64 least-squares residual is below half the target the cycle's
      // estimate (the Arnoldi relation of FP64 applies holds to rounding)
      double rknown = use_x0 ? -1.0 : bn;
      while (bn > 0.0) {
        const bool known = rknown >= 0.0;
        const double rn = known ? rknown : KO.true_resid(xx, bb, KO.rtrue);
        rknown = -1.0;
        rel = rn / bn;
        if (rel <= tol_r || outer_done >= o.max_outer) break;
        launch_scale(P64, known ? bb : KO.rtrue, KO.V(0), N, nullptr, 1.0 / rn, nullptr, st);
        launch_arnoldi_init(KO.ad, rn, st);
        int jd = 0;
        for (int j = 0; j < o.m_outer && outer_done < o.max_outer; ++j) {
          launch_convert_64to32(KO.V(j), b32, N, op.n, 0, st);
          double irel;
          KI.solve(b32, x32, o.inner_tol, false, o.max_cycles, s, irel);
          launch_convert_32to64(x32, Zb + size_t(j) * N, N, op.n, 0, st);
          KO.A(Zb + size_t(j) * N, KO.V(j + 1), nullptr);
          KO.orth_step(j, 0, o.m_outer, tol_r * bn);
          ++outer_done;
          int flags[3];
          op.hs.read(flags, KO.ad.done, 3 * sizeof(int), st);
          op.hs.wait(st);
          jd = flags[1];
          if (flags[0]) break;
        }
        std::vector<double> Hh(2 * size_t(KO.ldh) * KO.ldh);
        op.hs.read(Hh.data(), KO.ad.H, Hh.size() * sizeof(double), st);
        op.hs.wait(st);
        Mat H(jd + 1, jd);
        for (int jj = 0; jj < jd; ++jj)
          for (int i = 0; i <= jj + 1; ++i)
            H(i, jj) = cd(Hh[2 * (size_t(jj) * KO.ldh + i)], Hh[2 * (size_t(jj) * KO.ldh + i) + 1]);
        std::vector<cd> e1(jd + 1, cd(0.0));
        e1[0] = rn;
        double lsres;
        const auto y = lstsq(H, e1, &lsres);
        s.rel_res_est = lsres / bn;
        KO.upload_coef(y);
        launch_combine(P64, nullptr, 0, Zb, jd, N, KO.coef, 1, xx, 1, st);
        if (jd == 0) {
          stuck = true;
          break;
        }
        if (lsres <= 0.5 * tol_r * bn) {
          rel = lsres / bn;
          break;
        }
      }
      s.outer_iters = outer_done;
      s.matvecs += int(KO.matvecs);
      collect(KI);
      s.breakdowns += KO.breakdowns;
    }
    if (o.schur) {
      launch_reduced_oe(P64, op.n, op.V, op.blocks(P64), nullptr, oinv, nullptr, xe.p, bo.p,
                        op.nbr.as<int>(), osite, nullptr, st);       // A_o^{-1} D_oe x_e
      launch_axpy(P64, mk(-1.0, 0.0), bo.p, to.p, N, st);           // x_o = A_o^{-1} b_o - that
      launch_oddeven_split(P64, op.n, half, esite, osite, xfull, xe.p, to.p, 1, st);
      xx = xfull;
    }
    if (adjoint) launch_gamma5(P64, xx, xr, op.V, op.n, st);
    (void)rel;
    s.rel_res_true = fp64_relres(op, xr, br, adjoint, st);
    if (o.x_ref)
      s.err_vs_ref = fp64_relerr(op, xr, static_cast<const z64*>(o.x_ref) + size_t(r) * Nfull, st);
    const bool conv = s.rel_res_true <= tol[r];
    // positive statuses: the best iterate is written
    s.status = conv ? 0 : (stuck ? 2 : 1);
    if (!conv) {
      all_ok = 0;
      worst = std::max(worst, s.status);
    }
    s.t_solve_ms = ms_since(t0);
    if (stats) stats[r] = s;
  }
  return all_ok ? 0 : worst;
}

// ============================================================================ batched
// Right-hand sides solved in lockstep (independent Krylov spaces, one MFMA
// multi-apply per step for all active right-hand sides of all operators):
// restarted GMRES(m) with each operator's polynomial and block-Jacobi
// preconditioners and, when its variant already holds a recycle space,
// deflation against it (frozen: the shared space is not refreshed by the
// batch).  A batch holds one group per operator (a mixed batch of lattices
// with one block size); converged right-hand sides drop out of the active set
// at cycle ends.

namespace {

template <typename VR>
struct Batch {
  using Z = cx<VR>;
  struct Group {
    Op* op;
    Variant* var;
    size_t N;
    int R;                                          // columns of this operator
    SolveOpts ko;                                   // options of its Krylov objects
    std::vector<std::unique_ptr<Krylov<VR>>> K;     // per column
    std::vector<int> act;                           // active columns
    size_t toff = 0;                                // offset of its tables (pointers)
    std::vector<const Z*> b;
    std::vector<Z*> x;
  };
  const SolveOpts& o;
  Prec p;
  hipStream_t st;
  std::vector<Group> g;
  DevBuf& tab;                    // device pointer tables of the active sets
  std::vector<void*> htab;        // host copy
  int ldh;
  long matvecs = 0;
  // per group, table layout (pointers): [slot][Ra_g]
  enum { T_PROD, T_Y, T_TA, T_TB, T_TMP, T_TMP2, T_X, T_B, T_RT, T_NFIX };

  Batch(const std::vector<Op*>& ops, const std::vector<Variant*>& vars, const SolveOpts& o_,
        const std::vector<int>& R, hipStream_t st_, DevBuf& tab_)
      : o(o_), p(vars[0]->prec), st(st_), tab(tab_) {
    g.resize(ops.size());
    for (size_t i = 0; i < ops.size(); ++i) {
      Group& gr = g[i];
      gr.op = ops[i];
      gr.var = vars[i];
      gr.N = ops[i]->N();
      gr.R = R[i];
      gr.ko = o;
      gr.ko.k = vars[i]->kcur;  // dot-product arrays sized for the (frozen) deflation space
      Op& op = *ops[i];
      op.bws.resize(std::max<size_t>(op.bws.size(), size_t(R[i])));
      op.bsm.resize(std::max<size_t>(op.bsm.size(), size_t(R[i])));
      for (int r = 0; r < R[i]; ++r)
        gr.K.emplace_back(std::make_unique<Krylov<VR>>(op, *vars[i], gr.ko, op.bws[r], op.bsm[r],
                                                       o.m, st, false));
    }
    ldh = std::max(o.m, std::max(o.d, 1)) + 2;  // as every Krylov object of the batch
    for (const Group& gr : g)
      if (!gr.K.empty() && gr.K[0]->ldh != ldh) throw BadState("batched Krylov size mismatch");
    size_t cols = 0;
    for (int r : R) cols += size_t(r);
    ops[0]->bpart.ensure(std::max<size_t>(cols, 1) * kRedCap * sizeof(double));
  }

  // device pointer array of slot s of group gi (T_NFIX + j: basis vector j)
  Z* const* slot(int gi, int s) const {
    return reinterpret_cast<Z* const*>(static_cast<void**>(tab.p) + g[gi].toff + size_t(s) * g[gi].act.size());
  }
  std::vector<Z*> host_slot(int gi, int s) const {
    const size_t Ra = g[gi].act.size(), off = g[gi].toff + size_t(s) * Ra;
    std::vector<Z*> out(Ra);
    for (size_t a = 0; a < Ra; ++a) out[a] = static_cast<Z*>(htab[off + a]);
    return out;
  }
  bool any_active() const {
    for (const Group& gr : g)
      if (!gr.act.empty()) return true;
    return false;
  }

  void upload_tables() {
    const int ns = T_NFIX + ldh + 1;
    size_t total = 0;
    for (Group& gr : g) {
      gr.toff = total;
      total += size_t(ns) * gr.act.size();
    }
    std::vector<void*> h(std::max<size_t>(total, 1));
    for (Group& gr : g) {
      const size_t Ra = gr.act.size();
      for (size_t a = 0; a < Ra; ++a) {
        Krylov<VR>& k = *gr.K[gr.act[a]];
        void** t = h.data() + gr.toff;
        t[T_PROD * Ra + a] = k.prod;
        t[T_Y * Ra + a] = k.ybuf;
        t[T_TA * Ra + a] = k.ta;
        t[T_TB * Ra + a] = k.tb;
        t[T_TMP * Ra + a] = k.tmp;
        t[T_TMP2 * Ra + a] = k.tmp2;
        t[T_X * Ra + a] = gr.x[gr.act[a]];
        t[T_B * Ra + a] = const_cast<Z*>(gr.b[gr.act[a]]);
        t[T_RT * Ra + a] = k.rtrue;
        for (int j = 0; j <= ldh; ++j) t[(T_NFIX + j) * Ra + a] = k.V(j);
      }
    }
    tab.ensure(h.size() * sizeof(void*));
    g[0].op->hs.write(tab.p, h.data(), h.size() * sizeof(void*), st);
    htab = std::move(h);
  }

  // one multi-apply over every group with active columns: slot `out` = D slot `in`
  void multi_apply(Prec pa, int in, int out) {
    std::vector<MultiOpDesc> d;
    int n = 0;
    for (size_t gi = 0; gi < g.size(); ++gi) {
      const Group& gr = g[gi];
      if (gr.act.empty()) continue;
      MultiOpDesc e{};
      e.blocks = gr.op->blocks(pa);
      e.scales = gr.op->scales(pa);
      e.nbr = static_cast<const int*>(gr.op->nbr.p);
      e.xin = reinterpret_cast<const void* const*>(slot(int(gi), in));
      e.yout = reinterpret_cast<void* const*>(slot(int(gi), out));
      e.V = gr.op->V;
      e.R = int(gr.act.size());
      e.tm = gr.var->sign * gr.op->mu;
      d.push_back(e);
      n = gr.op->n;
    }
    for (size_t i = 0; i < d.size(); i += kMaxMultiOps)
      launch_apply_multi_ops(pa, n, d.data() + i, int(std::min<size_t>(kMaxMultiOps, d.size() - i)),
                             0, st);
  }

  // slot out = A~ slot in for the active set (A~ = B^{-1} D with block Jacobi)
  void A(int in, int out) {
    bool bj = false;
    for (const Group& gr : g) bj = bj || (!gr.act.empty() && gr.K[0]->bjinv);
    multi_apply(p, in, bj ? T_TB : out);
    if (bj)
      for (size_t gi = 0; gi < g.size(); ++gi) {
        Group& gr = g[gi];
        const std::vector<Z*> ho = host_slot(int(gi), out);
        for (size_t a = 0; a < gr.act.size(); ++a) {
          Krylov<VR>& k = *gr.K[gr.act[a]];
          launch_bj_vec(p, gr.op->n, gr.op->V, k.bjinv, k.bjsc, k.tb, ho[a], st);
        }
      }
    matvecs += 1;
  }

  static bool has_poly(const Variant& v) { return v.d > 1 && int(v.theta.size()) > 1; }

  // slot out = q(A~) slot in (Newton-like chain per operator), out distinct from in.
  // Every operator of a batch shares d (same options), each has its own theta.
  void Q(int in, int out) {
    auto inv = [](cd t) { const cd r = 1.0 / t; return mk(r.real(), r.imag()); };
    const int d = int(g[0].var->theta.size());
    if (d <= 1) {
      for (size_t gi = 0; gi < g.size(); ++gi) {
        Group& gr = g[gi];
        const std::vector<Z*> ho = host_slot(int(gi), out), hi = host_slot(int(gi), in);
        const auto& th = gr.var->theta;
        const z64 c = (int(th.size()) == 1) ? inv(th[0]) : mk(1.0, 0.0);
        for (size_t a = 0; a < gr.act.size(); ++a) launch_cscale(p, hi[a], ho[a], gr.N, c, nullptr, st);
      }
      return;
    }
    A(in, T_TA);
    chain_step(in, out, 1);
    for (int i = 2; i < d; ++i) {
      A(T_PROD, T_TA);
      chain_step(in, out, i);
    }
  }

  // Chain step i (1: the first) of every group with active columns: slot
  // T_PROD and slot out from slot T_TA (and slot in for the first), with the
  // group's own roots; one launch for up to kChainGroups groups, or one per
  // group when the batch runs its launches per column.
  void chain_step(int in, int out, int i) {
    auto inv = [](cd t) { const cd r = 1.0 / t; return mk(r.real(), r.imag()); };
    const bool first = i == 1;
    ChainGroups cg;
    auto flush = [&]() {
      launch_chain_groups(p, cg, first ? 1 : 0, st);
      cg = ChainGroups{};
    };
    for (size_t gi = 0; gi < g.size(); ++gi) {
      const Group& gr = g[gi];
      if (gr.act.empty()) continue;
      const auto& th = gr.var->theta;
      const z64 c0 = first ? inv(th[0]) : mk(0.0, 0.0);
      const z64 ca = inv(th[i - 1]), cb = inv(th[i]);
      const void* const* tv = reinterpret_cast<const void* const*>(slot(int(gi), T_TA));
      const void* const* vv = first ? reinterpret_cast<const void* const*>(slot(int(gi), in)) : nullptr;
      void* const* pv = reinterpret_cast<void* const*>(slot(int(gi), T_PROD));
      void* const* yv = reinterpret_cast<void* const*>(slot(int(gi), out));
      if (!batch_launches()) {
        launch_chain_multi(p, tv, vv, pv, yv, int(gr.act.size()), gr.N, c0, ca, cb, first ? 1 : 0,
                           st);
        continue;
      }
      const int c = cg.count++;
      cg.t[c] = tv;
      cg.v[c] = vv;
      cg.prod[c] = pv;
      cg.y[c] = yv;
      cg.N[c] = gr.N;
      cg.R[c] = int(gr.act.size());
      cg.c0[c] = c0;
      cg.ca[c] = ca;
      cg.cb[c] = cb;
      if (cg.count == kChainGroups) flush();
    }
    if (cg.count) flush();
  }

  void Ahat(int in, int out) {
    if (has_poly(*g[0].var)) {
      Q(in, T_Y);
      A(T_Y, out);
    } else {
      A(in, out);
    }
  }

  // true residuals r = b - D x (in the batch precision) for every active column
  std::vector<std::vector<double>> true_resid() {
    multi_apply(p, T_X, T_TA);
    matvecs += 1;
    std::vector<std::vector<double>> rn(g.size());
    for (Group& gr : g) {
      for (int c : gr.act) {
        Krylov<VR>& k = *gr.K[c];
        launch_scale(p, k.ta, k.rtrue, gr.N, nullptr, -1.0, nullptr, st);
        launch_axpy(p, mk(1.0, 0.0), gr.b[c], k.rtrue, gr.N, st);
        launch_norm2(p, k.rtrue, gr.N, gr.op->red(), k.nrm, st);
      }
    }
    for (size_t gi = 0; gi < g.size(); ++gi) {
      Group& gr = g[gi];
      rn[gi].resize(gr.act.size());
      for (size_t a = 0; a < gr.act.size(); ++a)
        g[0].op->hs.read(&rn[gi][a], gr.K[gr.act[a]]->nrm, sizeof(double), st);
    }
    g[0].op->hs.wait(st);
    for (auto& v : rn)
      for (double& x : v) x = std::sqrt(std::max(x, 0.0));
    return rn;
  }

  // The Arnoldi steps of one lockstep cycle: per step one multi-apply chain
  // over every active column of every operator, then each column's
  // orthogonalisation (the device stops a column's steps once its estimate
  // meets the target).
  void enqueue_steps(int steps, const std::vector<std::vector<double>>& target) {
    for (int j = 0; j < steps; ++j) {
      Ahat(T_NFIX + j, T_NFIX + j + 1);
      if (batch_launches()) {
        orth_batched(j, steps, target);
        continue;
      }
      for (size_t gi = 0; gi < g.size(); ++gi) {
        Group& gr = g[gi];
        for (size_t a = 0; a < gr.act.size(); ++a)
          gr.K[gr.act[a]]->orth_step(j, gr.var->kcur, steps, target[gi][a]);
      }
    }
  }

  // Step j's Gram-Schmidt (classical, twice) of every active column, one
  // launch per pass for up to kOrthCols columns of equal deflation-space size:
  // the launches of Krylov::orth_step with ortho = 0, for many columns at once
  // (same sums, so the same results), each column with its own slice of the
  // batch's reduction partials.
  void orth_batched(int j, int steps, const std::vector<std::vector<double>>& target) {
    struct Col {
      Krylov<VR>* k;
      int kC;
      double target;
    };
    std::vector<Col> cols;
    for (size_t gi = 0; gi < g.size(); ++gi) {
      Group& gr = g[gi];
      for (size_t a = 0; a < gr.act.size(); ++a)
        cols.push_back({gr.K[gr.act[a]].get(), gr.var->kcur, target[gi][a]});
    }
    std::stable_sort(cols.begin(), cols.end(),
                     [](const Col& x, const Col& y) { return x.kC < y.kC; });
    double* part = g[0].op->bpart.template as<double>();
    for (size_t s0 = 0; s0 < cols.size();) {
      size_t e = s0;
      while (e < cols.size() && e - s0 < size_t(kOrthCols) && cols[e].kC == cols[s0].kC) ++e;
      OrthCols d1, a1, d2, a2;
      FinishCols f;
      ScaleCols sc;
      double brk = 0.0;
      for (size_t i = s0; i < e; ++i) {
        Krylov<VR>& k = *cols[i].k;
        const int c = int(i - s0);
        OrthCol base;
        base.b0 = cols[i].kC ? k.Cv() : nullptr;
        base.q0 = cols[i].kC;
        base.b1 = k.V(0);
        base.q1 = j + 1;
        base.w = k.V(j + 1);
        base.N = k.N;
        base.done = k.ad.done;
        base.partials = part + i * size_t(kRedCap);
        d1.c[c] = base;
        d1.c[c].result = k.res1;
        a1.c[c] = base;
        a1.c[c].coef = k.res1;
        a1.c[c].result = k.nrm;
        d2.c[c] = base;
        d2.c[c].result = k.res2;
        a2.c[c] = base;
        a2.c[c].coef = k.res2;
        a2.c[c].result = k.nrm;
        f.c[c].a = k.ad;
        f.c[c].c1 = k.res1;
        f.c[c].c2 = k.res2;
        f.c[c].nrm2 = k.nrm;
        f.c[c].target = cols[i].target;
        f.c[c].kC = cols[i].kC;
        sc.v[c] = k.V(j + 1);
        sc.N[c] = k.N;
        sc.inv_h[c] = k.ad.inv_h;
        sc.jdone[c] = k.ad.jdone;
        brk = k.brk;
      }
      const int n = int(e - s0);
      d1.count = a1.count = d2.count = a2.count = f.count = sc.count = n;
      launch_multidot_cols(p, d1, 1, st);
      launch_multiaxpy_cols(p, a1, 0, st);
      launch_multidot_cols(p, d2, 0, st);
      launch_multiaxpy_cols(p, a2, 1, st);
      launch_arnoldi_finish_cols(f, steps, j, brk, st);
      launch_scale_step_cols(p, sc, j, st);
      s0 = e;
    }
  }

  // Whether every multi-apply of the active set already has its tile chosen
  // (tuning times launches and cannot run inside a graph recording).
  bool tiles_tuned() const {
    int rmax = 0, cnt = 0, n = 0;
    unsigned sites = 0;
    for (const Group& gr : g) {
      if (gr.act.empty()) continue;
      rmax = std::max(rmax, int(gr.act.size()));
      sites += unsigned(gr.op->V);
      n = gr.op->n;
      if (++cnt == kMaxMultiOps) {
        if (!multi_tile_for(p, n, rmax, sites)) return false;
        rmax = 0;
        sites = 0;
        cnt = 0;
      }
    }
    return cnt == 0 || multi_tile_for(p, n, rmax, sites) != 0;
  }

  // The cycle's steps recorded once per active set and shape as a HIP graph
  // and replayed as one launch per cycle (the batching configuration's one
  // launch for a mixed batch): every kernel argument depends only on the key
  // below; each column's stopping target is read from device memory.
  bool graph_steps(int steps, const std::vector<std::vector<double>>& target) {
    Op& op0 = *g[0].op;
    GraphCache& gc = op0.graphs;
    if (gc.broken || op0.prof.on || !tiles_tuned()) return false;
    std::vector<uintptr_t> key = {0xBA7C4u, uintptr_t(tab.p), uintptr_t(steps), uintptr_t(p),
                                  uintptr_t(ldh), uintptr_t(g.size()), uintptr_t(op0.bpart.p),
                                  uintptr_t(batch_launches())};
    for (size_t gi = 0; gi < g.size(); ++gi) {
      Group& gr = g[gi];
      key.insert(key.end(), {uintptr_t(gr.op), uintptr_t(gr.var), uintptr_t(gr.var->poly_serial),
                             uintptr_t(gr.op->version), uintptr_t(gr.var->kcur),
                             uintptr_t(gr.var->C.p), uintptr_t(gr.act.size())});
      for (size_t a = 0; a < gr.act.size(); ++a) {
        Krylov<VR>& k = *gr.K[gr.act[a]];
        key.insert(key.end(), {uintptr_t(gr.act[a]), uintptr_t(k.ws.p), uintptr_t(k.sm.p),
                               uintptr_t(k.bjinv)});
        double* tdev = k.nrm + 1;   // free slot of the column's small area
        op0.hs.write(tdev, &target[gi][a], sizeof(double), st);
        k.ad.target_dev = tdev;
      }
    }
    auto clear_targets = [&]() {
      for (Group& gr : g)
        for (int c : gr.act) gr.K[c]->ad.target_dev = nullptr;
    };
    hipGraphExec_t exec = gc.find(key);
    const long per_step = has_poly(*g[0].var) ? long(g[0].var->theta.size()) : 1L;
    if (!exec) {
      if (!gc.cap && hipStreamCreateWithFlags(&gc.cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        gc.cap = nullptr;
        gc.broken = true;
        clear_targets();
        return false;
      }
      if (hipStreamBeginCapture(gc.cap, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipGetLastError();
        gc.broken = true;
        clear_targets();
        return false;
      }
      // every launch of the steps goes to the capture stream while recording
      const hipStream_t saved = st;
      const long mv_saved = matvecs;   // recording runs nothing
      st = gc.cap;
      for (Group& gr : g)
        for (int c : gr.act) gr.K[c]->st = gc.cap;
      bool ok = true;
      try {
        enqueue_steps(steps, target);
      } catch (const std::exception&) {
        ok = false;
      }
      st = saved;
      for (Group& gr : g)
        for (int c : gr.act) gr.K[c]->st = saved;
      matvecs = mv_saved;
      hipGraph_t graph = nullptr;
      if (hipStreamEndCapture(gc.cap, &graph) != hipSuccess || !ok || !graph) {
        (void)hipGetLastError();
        if (graph) (void)hipGraphDestroy(graph);
        gc.broken = true;
        clear_targets();
        return false;
      }
      if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(graph);
        gc.broken = true;
        clear_targets();
        return false;
      }
      gc.add(key, graph, exec);
      ++gc.captured;
    }
    DC_HIP(hipGraphLaunch(exec, st));
    ++gc.launched;
    matvecs += long(steps) * per_step;   // the applications the replayed steps make
    clear_targets();
    return true;
  }

  // Solve D_g x_{g,r} = b_{g,r} to tolerances tol[g][r]; stt, relres likewise indexed.
  void solve(bool use_x0, int max_cycles, const std::vector<std::vector<double>>& tol,
             std::vector<std::vector<SolveStats>>& stt, std::vector<std::vector<double>>& relres) {
    const int steps_req = o.m;
    std::vector<std::vector<int>> conv(g.size()), cycles(g.size());
    std::vector<std::vector<double>> bn(g.size());
    for (size_t gi = 0; gi < g.size(); ++gi) {
      Group& gr = g[gi];
      conv[gi].assign(gr.R, 0);
      cycles[gi].assign(gr.R, 0);
      bn[gi].assign(gr.R, 0.0);
      for (int r = 0; r < gr.R; ++r) {
        if (!use_x0) launch_zero(p, gr.x[r], gr.N, st);
        bn[gi][r] = gr.K[r]->norm(gr.b[r]);
        if (bn[gi][r] == 0.0) {
          launch_zero(p, gr.x[r], gr.N, st);
          conv[gi][r] = 1;
          relres[gi][r] = 0.0;
        }
      }
      if (gr.R > 0 && std::min(steps_req - gr.var->kcur, ldh - 2) < 1)
        throw InvalidArg("batched solve needs m > k");
    }
    const bool poly = has_poly(*g[0].var);
    for (int cyc = 0;; ++cyc) {
      for (size_t gi = 0; gi < g.size(); ++gi) {
        Group& gr = g[gi];
        gr.act.clear();
        for (int r = 0; r < gr.R; ++r)
          if (!conv[gi][r] && cycles[gi][r] <= max_cycles) gr.act.push_back(r);
      }
      if (!any_active()) break;
      upload_tables();
      const long mv0 = matvecs;
      const auto rn = true_resid();
      bool any = false, changed = false;
      for (size_t gi = 0; gi < g.size(); ++gi) {
        Group& gr = g[gi];
        std::vector<int> keep;
        for (size_t a = 0; a < gr.act.size(); ++a) {
          const int r = gr.act[a];
          relres[gi][r] = rn[gi][a] / bn[gi][r];
          stt[gi][r].matvecs += int(matvecs - mv0);
          if (relres[gi][r] <= tol[gi][r]) conv[gi][r] = 1;
          else if (cycles[gi][r] < max_cycles) keep.push_back(r);
        }
        if (keep.size() != gr.act.size()) changed = true;
        gr.act = keep;
        any = any || !keep.empty();
      }
      if (!any) break;
      if (changed) upload_tables();
      // start vectors: rhat = B^{-1} r, deflated against C (x += q U C^H rhat)
      std::vector<std::vector<double>> beta(g.size()), target(g.size());
      bool defl = false;
      for (size_t gi = 0; gi < g.size(); ++gi) {
        Group& gr = g[gi];
        const int kC = gr.var->kcur;
        beta[gi].resize(gr.act.size());
        target[gi].resize(gr.act.size());
        for (size_t a = 0; a < gr.act.size(); ++a) {
          const int r = gr.act[a];
          Krylov<VR>& k = *gr.K[r];
          k.left_precondition(k.rtrue, k.rhat);
          const double rr = relres[gi][r] * bn[gi][r];
          const double b0 = k.bjinv ? k.norm(k.rhat) : rr;
          target[gi][a] = tol[gi][r] * bn[gi][r] * (b0 / std::max(rr, 1e-300));
          if (kC > 0) {
            launch_multidot(p, k.Cv(), kC, nullptr, 0, gr.N, k.rhat, 0, gr.op->red(), k.res1,
                            nullptr, st);
            launch_multiaxpy(p, k.rhat, k.Cv(), kC, nullptr, 0, gr.N, k.res1, 0, gr.op->red(),
                             k.nrm, nullptr, st);
            launch_combine(p, k.Uv(), kC, nullptr, 0, gr.N, k.res1, 1, k.tmp, 0, st);
            defl = true;
          }
          beta[gi][a] = (kC > 0) ? k.norm(k.rhat) : b0;
        }
      }
      if (defl) {  // x += q(A~) U c for the active columns of deflated groups
        if (poly) Q(T_TMP, T_TMP2);
        for (Group& gr : g) {
          if (gr.var->kcur == 0) continue;
          for (int r : gr.act) {
            Krylov<VR>& k = *gr.K[r];
            launch_axpy(p, mk(1.0, 0.0), poly ? k.tmp2 : k.tmp, gr.x[r], gr.N, st);
          }
        }
      }
      for (size_t gi = 0; gi < g.size(); ++gi) {
        Group& gr = g[gi];
        for (size_t a = 0; a < gr.act.size(); ++a) {
          Krylov<VR>& k = *gr.K[gr.act[a]];
          launch_scale(p, k.rhat, k.V(0), gr.N, nullptr, 1.0 / beta[gi][a], nullptr, st);
          launch_arnoldi_init(k.ad, beta[gi][a], st);
        }
      }
      const long mv1 = matvecs;
      int steps = ldh - 2;
      for (const Group& gr : g)
        if (!gr.act.empty()) steps = std::min(steps, steps_req - gr.var->kcur);
      if (!(o.graphs && graph_steps(steps, target))) enqueue_steps(steps, target);
      // per right-hand side: least squares and the update of x
      for (size_t gi = 0; gi < g.size(); ++gi) {
        Group& gr = g[gi];
        const int kC = gr.var->kcur;
        for (size_t a = 0; a < gr.act.size(); ++a) {
          const int r = gr.act[a];
          Krylov<VR>& k = *gr.K[r];
          int flags[3];
          HostStage& hst = g[0].op->hs;
          hst.read(flags, k.ad.done, 3 * sizeof(int), st);
          std::vector<double> Hh(2 * size_t(k.ldh) * k.ldh), Bh(2 * size_t(k.ad.ldb) * k.ldh);
          hst.read(Hh.data(), k.ad.H, Hh.size() * sizeof(double), st);
          if (kC) hst.read(Bh.data(), k.ad.Bk, Bh.size() * sizeof(double), st);
          hst.wait(st);
          const int jd = flags[1];
          stt[gi][r].iters += jd;
          stt[gi][r].matvecs += int(matvecs - mv1);
          cycles[gi][r] += 1;
          stt[gi][r].cycles += 1;
          // G = [[D_k, B_k], [0, Hbar]] with D_k = diag(1 / unorm)
          Mat Hb(jd + 1, jd), Bk(kC, jd);
          for (int jj = 0; jj < jd; ++jj) {
            for (int i = 0; i < kC; ++i)
              Bk(i, jj) = cd(Bh[2 * (size_t(jj) * k.ad.ldb + i)], Bh[2 * (size_t(jj) * k.ad.ldb + i) + 1]);
            for (int i = 0; i <= jj + 1; ++i)
              Hb(i, jj) = cd(Hh[2 * (size_t(jj) * k.ldh + i)], Hh[2 * (size_t(jj) * k.ldh + i) + 1]);
          }
          double lsres = 0.0;
          const auto y = gcrodr_lstsq(Hb, Bk, gr.var->unorm, beta[gi][a], &lsres);
          stt[gi][r].rel_res_est = lsres / bn[gi][r];
          std::vector<cd> cy(kC + jd);
          for (int i = 0; i < kC; ++i) cy[i] = y[i] / gr.var->unorm[i];
          for (int i = 0; i < jd; ++i) cy[kC + i] = y[kC + i];
          k.upload_coef(cy);
          launch_combine(p, kC ? k.Uv() : nullptr, kC, k.V(0), jd, gr.N, k.coef, 1,
                         poly ? k.tmp : gr.x[r], poly ? 0 : 1, st);
        }
      }
      if (poly) {
        Q(T_TMP, T_TMP2);
        for (Group& gr : g)
          for (int r : gr.act) launch_axpy(p, mk(1.0, 0.0), gr.K[r]->tmp2, gr.x[r], gr.N, st);
      }
    }
  }
};

}  // namespace

// Batched solve over one or more operators (same block size, precision
// stored, options); b[g], x[g]: device complex128 [R[g]][V_g][n]; tol[g][r].
static int solve_groups(const std::vector<Op*>& ops, const SolveOpts& o, int adjoint,
                        const std::vector<int>& R, const std::vector<const void*>& b,
                        const std::vector<void*>& x, const std::vector<const double*>& tol,
                        int use_x0, hipStream_t st, const std::vector<SolveStats*>& stats) {
  const size_t G = ops.size();
  if (G == 0) return 0;
  if (o.m < 1 || o.max_cycles < 0) throw InvalidArg("bad solver options");
  if (o.schur) throw InvalidArg("the batched solve works on the full lattice (schur = 0)");
  if (o.ortho) throw InvalidArg("the batched solve orthogonalises with Gram-Schmidt twice (ortho = 0)");
  for (size_t gi = 0; gi < G; ++gi) {
    if (!ops[gi]) throw InvalidArg("null operator handle");
    check_prec(*ops[gi], o.prec);
    if (ops[gi]->n != ops[0]->n) throw InvalidArg("every operator of a batch needs the same n");
    if (R[gi] < 0 || (R[gi] > 0 && (!b[gi] || !x[gi] || !tol[gi])))
      throw InvalidArg("null pointer or negative n_rhs");
    for (int r = 0; r < R[gi]; ++r)
      if (!(tol[gi][r] > 0.0)) throw InvalidArg("tolerances must be positive");
    for (size_t gj = 0; gj < gi; ++gj)
      if (ops[gj] == ops[gi]) throw InvalidArg("an operator appears twice in a batch");
  }
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<std::vector<SolveStats>> stt(G);
  std::vector<Variant*> vars(G);
  std::vector<int> kc_saved(G);
  std::vector<double> t_setup(G, 0.0);
  for (size_t gi = 0; gi < G; ++gi) {
    Op& op = *ops[gi];
    stt[gi].resize(std::max(R[gi], 1));
    const int sign = (adjoint && op.mu != 0.0) ? -1 : +1;
    Variant& var = op.variant(o.prec, sign, o.block_jacobi ? 1 : 0, o.d);
    const auto ts = std::chrono::steady_clock::now();
    ensure_poly(op, var, o, st, &stt[gi][0]);
    if (var.recycle_version != op.version || var.k_built != o.k) var.kcur = 0;
    t_setup[gi] = ms_since(ts);
    kc_saved[gi] = var.kcur;
    if (o.k <= 0) var.kcur = 0;
    vars[gi] = &var;
  }
  // caller vectors (complex128); adjoint through Gamma5 on copies
  std::vector<z64*> B64(G), X64(G);
  for (size_t gi = 0; gi < G; ++gi) {
    Op& op = *ops[gi];
    const size_t N = op.N();
    op.bx64.ensure(size_t(std::max(R[gi], 1)) * N * sizeof(z64));
    op.bb64.ensure(size_t(std::max(R[gi], 1)) * N * sizeof(z64));
    B64[gi] = op.bb64.as<z64>();
    X64[gi] = op.bx64.as<z64>();
    for (int r = 0; r < R[gi]; ++r) {
      const z64* br = static_cast<const z64*>(b[gi]) + size_t(r) * N;
      const z64* xr = static_cast<const z64*>(x[gi]) + size_t(r) * N;
      if (adjoint) {
        launch_gamma5(P64, br, B64[gi] + size_t(r) * N, op.V, op.n, st);
        if (use_x0) launch_gamma5(P64, xr, X64[gi] + size_t(r) * N, op.V, op.n, st);
      } else {
        DC_HIP(hipMemcpyAsync(B64[gi] + size_t(r) * N, br, N * sizeof(z64), hipMemcpyDeviceToDevice, st));
        if (use_x0) DC_HIP(hipMemcpyAsync(X64[gi] + size_t(r) * N, xr, N * sizeof(z64), hipMemcpyDeviceToDevice, st));
      }
    }
  }
  std::vector<std::vector<double>> tl(G), rel(G);
  for (size_t gi = 0; gi < G; ++gi) {
    tl[gi].assign(tol[gi], tol[gi] + R[gi]);
    rel[gi].assign(R[gi], 0.0);
  }
  DevBuf& tab = ops[0]->ptrs;
  if (o.prec == P64) {
    Batch<double> Bt(ops, vars, o, R, st, tab);
    for (size_t gi = 0; gi < G; ++gi) {
      const size_t N = ops[gi]->N();
      for (int r = 0; r < R[gi]; ++r) {
        Bt.g[gi].b.push_back(B64[gi] + size_t(r) * N);
        Bt.g[gi].x.push_back(X64[gi] + size_t(r) * N);
      }
    }
    Bt.solve(use_x0 != 0, o.max_cycles, tl, stt, rel);
  } else {
    // FP64 iterative refinement around the batched reduced-precision solve:
    // x += ||r|| solve32(D, r / ||r||) until the FP64 residual meets tol
    std::vector<z32*> B32(G), X32(G);
    std::vector<z64*> R64(G);
    std::vector<std::vector<int>> done(G);
    std::vector<std::vector<double>> bn(G);
    for (size_t gi = 0; gi < G; ++gi) {
      Op& op = *ops[gi];
      const size_t N = op.N(), Rg = size_t(std::max(R[gi], 1));
      if (!use_x0) for (int r = 0; r < R[gi]; ++r) launch_zero(P64, X64[gi] + size_t(r) * N, N, st);
      op.b32.ensure(Rg * N * sizeof(z32));
      op.x32.ensure(Rg * N * sizeof(z32));
      op.r64.ensure(Rg * N * sizeof(z64));
      B32[gi] = op.b32.as<z32>();
      X32[gi] = op.x32.as<z32>();
      R64[gi] = op.r64.as<z64>();
      done[gi].assign(R[gi], 0);
      bn[gi].assign(R[gi], 0.0);
      for (int r = 0; r < R[gi]; ++r) {
        launch_norm2(P64, B64[gi] + size_t(r) * N, N, op.red(), op.scal.as<double>(), st);
        op.hs.read(&bn[gi][r], op.scal.p, sizeof(double), st);
        op.hs.wait(st);
        bn[gi][r] = std::sqrt(bn[gi][r]);
        if (bn[gi][r] == 0.0) done[gi][r] = 1;
      }
    }
    for (int outer = 0; outer <= o.max_outer; ++outer) {
      // FP64 residuals of every active column: one multi-apply over all operators
      std::vector<std::vector<int>> act(G);
      std::vector<void*> h;
      std::vector<size_t> off(G);
      bool any = false;
      for (size_t gi = 0; gi < G; ++gi) {
        for (int r = 0; r < R[gi]; ++r)
          if (!done[gi][r]) act[gi].push_back(r);
        any = any || !act[gi].empty();
      }
      if (!any) break;
      for (size_t gi = 0; gi < G; ++gi) {
        const size_t N = ops[gi]->N();
        off[gi] = h.size();
        for (int r : act[gi]) h.push_back(X64[gi] + size_t(r) * N);
        for (int r : act[gi]) h.push_back(R64[gi] + size_t(r) * N);
      }
      tab.ensure(h.size() * sizeof(void*));
      ops[0]->hs.write(tab.p, h.data(), h.size() * sizeof(void*), st);
      std::vector<MultiOpDesc> d;
      for (size_t gi = 0; gi < G; ++gi) {
        if (act[gi].empty()) continue;
        MultiOpDesc e{};
        e.blocks = ops[gi]->blocks(P64);
        e.nbr = ops[gi]->nbr.as<int>();
        e.xin = const_cast<const void* const*>(tab.as<void*>() + off[gi]);
        e.yout = tab.as<void*>() + off[gi] + act[gi].size();
        e.V = ops[gi]->V;
        e.R = int(act[gi].size());
        e.tm = vars[gi]->sign * ops[gi]->mu;
        d.push_back(e);
      }
      for (size_t i = 0; i < d.size(); i += kMaxMultiOps)
        launch_apply_multi_ops(P64, ops[0]->n, d.data() + i,
                               int(std::min<size_t>(kMaxMultiOps, d.size() - i)), 0, st);
      std::vector<std::vector<int>> inner_r(G);
      std::vector<std::vector<double>> scale(G);
      bool any_inner = false;
      for (size_t gi = 0; gi < G; ++gi) {
        Op& op = *ops[gi];
        const size_t N = op.N();
        for (int r : act[gi]) {
          z64* rr = R64[gi] + size_t(r) * N;
          launch_scale(P64, rr, rr, N, nullptr, -1.0, nullptr, st);
          launch_axpy(P64, mk(1.0, 0.0), B64[gi] + size_t(r) * N, rr, N, st);
          launch_norm2(P64, rr, N, op.red(), op.scal.as<double>(), st);
          double h2;
          op.hs.read(&h2, op.scal.p, sizeof(double), st);
          op.hs.wait(st);
          const double rn = std::sqrt(std::max(h2, 0.0));
          rel[gi][r] = rn / bn[gi][r];
          if (rel[gi][r] <= tl[gi][r] || outer == o.max_outer) {
            done[gi][r] = 1;
            continue;
          }
          stt[gi][r].outer_iters += 1;
          inner_r[gi].push_back(r);
          scale[gi].push_back(rn);
          launch_convert_64to32(rr, B32[gi] + size_t(r) * N, N, op.n, 0, st);
          launch_cscale(P32, B32[gi] + size_t(r) * N, B32[gi] + size_t(r) * N, N, mk(1.0 / rn, 0.0),
                        nullptr, st);
          any_inner = true;
        }
      }
      if (!any_inner) break;
      // inner batched solve on the still-active right-hand sides of every operator
      std::vector<int> Ri(G);
      std::vector<std::vector<double>> itol(G), irel(G);
      std::vector<std::vector<SolveStats>> ist(G);
      for (size_t gi = 0; gi < G; ++gi) {
        Ri[gi] = int(inner_r[gi].size());
        itol[gi].assign(Ri[gi], o.inner_tol);
        irel[gi].assign(Ri[gi], 0.0);
        ist[gi].resize(Ri[gi]);
      }
      Batch<float> Bi(ops, vars, o, Ri, st, tab);
      for (size_t gi = 0; gi < G; ++gi) {
        const size_t N = ops[gi]->N();
        for (int r : inner_r[gi]) {
          Bi.g[gi].b.push_back(B32[gi] + size_t(r) * N);
          Bi.g[gi].x.push_back(X32[gi] + size_t(r) * N);
        }
      }
      Bi.solve(false, o.max_cycles, itol, ist, irel);
      for (size_t gi = 0; gi < G; ++gi) {
        const size_t N = ops[gi]->N();
        for (size_t i = 0; i < inner_r[gi].size(); ++i) {
          const int r = inner_r[gi][i];
          stt[gi][r].iters += ist[gi][i].iters;
          stt[gi][r].cycles += ist[gi][i].cycles;
          stt[gi][r].matvecs += ist[gi][i].matvecs + 1;
          launch_convert_32to64(X32[gi] + size_t(r) * N, R64[gi] + size_t(r) * N, N, ops[gi]->n, 0, st);
          launch_axpy(P64, mk(scale[gi][i], 0.0), R64[gi] + size_t(r) * N, X64[gi] + size_t(r) * N, N, st);
        }
      }
    }
  }
  int all_ok = 1;
  for (size_t gi = 0; gi < G; ++gi) {
    Op& op = *ops[gi];
    vars[gi]->kcur = kc_saved[gi];
    const size_t N = op.N();
    for (int r = 0; r < R[gi]; ++r) {
      const z64* br = static_cast<const z64*>(b[gi]) + size_t(r) * N;
      z64* xr = static_cast<z64*>(x[gi]) + size_t(r) * N;
      if (adjoint) launch_gamma5(P64, X64[gi] + size_t(r) * N, xr, op.V, op.n, st);
      else DC_HIP(hipMemcpyAsync(xr, X64[gi] + size_t(r) * N, N * sizeof(z64), hipMemcpyDeviceToDevice, st));
      stt[gi][r].rel_res_true = fp64_relres(op, xr, br, adjoint, st);
      stt[gi][r].status = stt[gi][r].rel_res_true <= tol[gi][r] ? 0 : 1;
      if (stt[gi][r].status) all_ok = 0;
      stt[gi][r].t_setup_ms = (r == 0) ? t_setup[gi] : 0.0;
      stt[gi][r].t_solve_ms = ms_since(t0);
      if (gi < stats.size() && stats[gi]) stats[gi][r] = stt[gi][r];
    }
  }
  return all_ok ? 0 : 1;
}

int op_solve_batch(Op& op, const SolveOpts& o, int adjoint, int R, const void* b, void* x,
                   const double* tol, int use_x0, hipStream_t st, SolveStats* stats) {
  if (op.caller_ws())
    throw BadState("the batched solve allocates per-right-hand-side memory: not available on a "
                   "handle built on caller workspaces");
  if (R < 0) throw InvalidArg("negative n_rhs");
  if (R == 0) return 0;
  return solve_groups({&op}, o, adjoint, {R}, {b}, {x}, {tol}, use_x0, st, {stats});
}

int op_solve_multi(const std::vector<Op*>& ops, const SolveOpts& o, int adjoint,
                   const std::vector<int>& R, const std::vector<const void*>& b,
                   const std::vector<void*>& x, const std::vector<const double*>& tol, int use_x0,
                   hipStream_t st, const std::vector<SolveStats*>& stats) {
  for (const Op* q : ops)
    if (q && q->caller_ws())
      throw BadState("the batched solve allocates per-right-hand-side memory: not available on "
                     "a handle built on caller workspaces");
  if (ops.empty()) throw InvalidArg("no operators");
  if (ops.size() > size_t(kMaxMultiOps) * 64) throw InvalidArg("too many operators");
  return solve_groups(ops, o, adjoint, R, b, x, tol, use_x0, st, stats);
}

void workspace_bytes(const int dims[4], int n_tv, int store, double mu, bool host_input,
                     const SolveOpts& o, int max_rhs, size_t* persistent, size_t* scratch,
                     size_t* build_persistent, size_t* build_scratch) {
  for (int i = 0; i < 4; ++i)
    if (dims[i] < 1) throw InvalidArg("lattice extents must be >= 1");
  if (n_tv < 1 || n_tv > 32) throw InvalidArg("n_tv must be in 1..32");
  if (o.m < 1 || o.k < 0 || (o.k > 0 && o.k >= o.m) || o.m_outer < 1 || max_rhs < 0)
    throw InvalidArg("bad solver options");
  store |= 1;
  const long long Vll = 1LL * dims[0] * dims[1] * dims[2] * dims[3];
  if (Vll > (1LL << 30)) throw InvalidArg("lattice too large");
  const size_t V = size_t(Vll), n = size_t(2 * n_tv), half = V / 2;
  const bool oddeven = dims[0] % 2 == 0 && dims[1] % 2 == 0 && dims[2] % 2 == 0 &&
                       dims[3] % 2 == 0;
  if (o.schur && !oddeven) throw InvalidArg("the odd-even reduction needs every lattice extent even");
  const auto R = [](size_t b) { return Arena::round(b); };
  const size_t z64b = sizeof(z64), z32b = sizeof(z32);
  const size_t vsys = o.prec == P64 ? z64b : z32b;
  const size_t Nfull = V * n, Nsys = o.schur ? half * n : Nfull;
  const int nsign = mu != 0.0 ? 2 : 1;    // the adjoint's D(-mu) variant keeps its own state
  // persistent: tables, blocks, inverses, recycle spaces
  size_t P = R(8 * V * sizeof(int)) + R(5 * V * block_units(int(n), P64) * 16);
  if (store & 2) P += R(5 * V * block_units(int(n), P32) * 16);
  if (store & 4) P += R(5 * V * block_units(int(n), P16S) * 16) + R(5 * V * sizeof(float));
  if (oddeven) P += 2 * R(half * sizeof(int));
  if (build_persistent) *build_persistent = P;
  if (o.block_jacobi || o.schur) {
    size_t inv = R(V * block_units(int(n), P64) * 16);
    if (store & 2) inv += R(V * block_units(int(n), P32) * 16);
    if (store & 4) inv += R(V * block_units(int(n), P16S) * 16) + R(V * sizeof(float));
    P += size_t(nsign) * inv;
  }
  if (o.k > 0) {
    const size_t kv = R(size_t(o.k) * Nsys * vsys);
    P += size_t(nsign) * (2 + (o.d > 1 ? 1 : 0)) * kv;
  }
  // scratch at build: apply partials, reduction partials, host staging
  size_t gb = R(V * 9 * n * z64b) + ((store & 6) ? R(V * 9 * n * z32b) : 0);
  const size_t fixed = gb + R(size_t(kRedCap) * sizeof(double)) + R(256);
  const size_t build = fixed + (host_input ? R(V * 5 * n * n * z64b) : 0);
  if (build_scratch) *build_scratch = build;
  // scratch of the calls
  size_t run = fixed;
  run += 2 * R(Nfull * z64b);                                      // FP64 residual / adjoint
  if (oddeven) run += R(half * n * z64b) + ((store & 6) ? R(half * n * z32b) : 0);  // t_o
  if (o.schur) run += 4 * R(half * n * z64b);                      // reduced rhs / recovery
  if (o.prec != P64) run += 2 * R(Nsys * z32b);
  const KrylovSizes ki = krylov_sizes(Nsys, vsys, o.k, o.d, std::max(o.m, o.d), true);
  run += size_t(nsign) * (R(ki.ws_bytes) + R(ki.sm_bytes));
  if (o.outer) {
    const KrylovSizes ko = krylov_sizes(Nsys, z64b, 0, 0, o.m_outer, true);
    run += size_t(nsign) * (R(ko.ws_bytes) + R(ko.sm_bytes)) + R(size_t(o.m_outer) * Nsys * z64b);
  }
  if (o.k > 0) run += R(refresh_gram_bytes(o.k, o.m + 1));
  if (o.d > 1 && !o.v0) run += R(Nsys * z64b);                     // polynomial start vector
  if (max_rhs > 0) run += R(2 * size_t(max_rhs) * sizeof(void*)); // multi-apply pointer table
  const size_t slack = 64 * Arena::kArenaAlign;
  *persistent = P + slack;
  *scratch = std::max(build, run) + slack;
}

int op_export_recycle(Op& op, const SolveOpts& o, int adjoint, void* U, void* C, hipStream_t st) {
  const int sign = (adjoint && op.mu != 0.0) ? -1 : +1;
  Variant& var = op.variant(o.prec, sign, o.block_jacobi ? 1 : 0, o.d, o.schur);
  const size_t N = o.schur ? op.N() / 2 : op.N();
  // only a space built for this k fits the caller's [k][V][n] arrays
  if (var.kcur == 0 || var.k_built != o.k || var.recycle_version != op.version) return 0;
  if (var.prec == P64) {
    if (U) DC_HIP(hipMemcpyAsync(U, var.U.p, size_t(var.kcur) * N * sizeof(z64), hipMemcpyDeviceToDevice, st));
    if (C) DC_HIP(hipMemcpyAsync(C, var.C.p, size_t(var.kcur) * N * sizeof(z64), hipMemcpyDeviceToDevice, st));
  } else {
    for (int i = 0; i < var.kcur; ++i) {
      if (U) launch_convert_32to64(var.U.as<z32>() + size_t(i) * N, static_cast<z64*>(U) + size_t(i) * N, N, op.n, 0, st);
      if (C) launch_convert_32to64(var.C.as<z32>() + size_t(i) * N, static_cast<z64*>(C) + size_t(i) * N, N, op.n, 0, st);
    }
  }
  DC_HIP(hipStreamSynchronize(st));
  return var.kcur;
}

}  // namespace dc
