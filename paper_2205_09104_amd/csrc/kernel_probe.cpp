// dc_kernel_probe: a torch-free driver of the library's kernels for hardware
// counter collection (rocprofv3 --pmc) and kernel traces.  It builds a coarse
// operator from host blocks filled by a fixed pseudo-random sequence (values
// only need the operator's shape and a well-conditioned self block here),
// then launches one kind of apply a number of times through the C ABI.
//
//   dc_kernel_probe multi   L0 L1 L2 L3 n_tv prec n_rhs reps [mu]
//   dc_kernel_probe reduced L0 L1 L2 L3 n_tv prec reps [mu]     (block Jacobi form)
//   dc_kernel_probe chain   L0 L1 L2 L3 n_tv prec reps [mu]     (q(B^-1 S) chains, d = 24)
//   dc_kernel_probe reduced2 | chain2 ...                      (the same, two-kernel form)
//   dc_kernel_probe copy    MiB                                 (5 device copies)
//
// The chain mode runs the solver's polynomial-chain launches on the odd-even
// reduced system with block Jacobi: each q application is d - 1 applies of
// B^-1 S with the chain epilogues.  reduced / chain use the library's default
// kernel form of the reduced operator, reduced2 / chain2 the two-kernel form.
//
// The copy mode calibrates byte counters: each copy reads and writes exactly
// MiB mebibytes of HBM-resident data.
// prec: f64 | f32 | f16s.  Prints one line per phase; exits non-zero on any
// library or HIP error.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dcsolve.h"

namespace {

using cd = std::complex<double>;

void hip_ok(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    std::exit(3);
  }
}

void dc_ok(int rc, const char* what) {
  if (rc < 0) {
    std::fprintf(stderr, "%s failed (%d): %s\n", what, rc, dc_last_error());
    std::exit(4);
  }
}

// splitmix64, mapped to [-1, 1)
struct Seq {
  uint64_t s;
  double next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return double(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
};

int prec_of(const std::string& p) {
  if (p == "f64") return DC_PREC_F64;
  if (p == "f32") return DC_PREC_F32;
  if (p == "f16s") return DC_PREC_F16S;
  std::fprintf(stderr, "unknown precision %s\n", p.c_str());
  std::exit(2);
}

}  // namespace

int main(int argc, char** argv) {
  if (argc == 3 && std::string(argv[1]) == "copy") {
    const size_t bytes = size_t(std::atol(argv[2])) << 20;
    if (bytes == 0) return 2;
    void *a = nullptr, *b = nullptr;
    hip_ok(hipMalloc(&a, bytes), "hipMalloc");
    hip_ok(hipMalloc(&b, bytes), "hipMalloc");
    hip_ok(hipMemset(a, 1, bytes), "hipMemset");
    hip_ok(hipDeviceSynchronize(), "memset");
    for (int r = 0; r < 5; ++r) hip_ok(hipMemcpy(b, a, bytes, hipMemcpyDeviceToDevice), "copy");
    hip_ok(hipDeviceSynchronize(), "copies");
    std::printf("[probe] copy %s MiB x 5\n", argv[2]);
    hip_ok(hipFree(a), "hipFree");
    hip_ok(hipFree(b), "hipFree");
    return 0;
  }
  if (argc < 9) {
    std::fprintf(stderr,
                 "usage: %s multi L0 L1 L2 L3 n_tv prec n_rhs reps [mu]\n"
                 "       %s reduced|chain|reduced2|chain2 L0 L1 L2 L3 n_tv prec reps [mu]\n"
                 "       %s copy MiB\n",
                 argv[0], argv[0], argv[0]);
    return 2;
  }
  const std::string mode = argv[1];
  const bool two = mode == "reduced2" || mode == "chain2";
  const bool multi = mode == "multi", chain = mode == "chain" || mode == "chain2";
  if (!multi && !chain && mode != "reduced" && mode != "reduced2") {
    std::fprintf(stderr, "unknown mode %s\n", mode.c_str());
    return 2;
  }
  if (multi && argc < 10) {
    std::fprintf(stderr, "multi needs n_rhs and reps\n");
    return 2;
  }
  dc_op_desc desc{};
  for (int i = 0; i < 4; ++i) desc.dims[i] = std::atoi(argv[2 + i]);
  desc.n_tv = std::atoi(argv[6]);
  const int prec = prec_of(argv[7]);
  const int n_rhs = multi ? std::atoi(argv[8]) : 1;
  const int reps = std::atoi(argv[multi ? 9 : 8]);
  const int mu_arg = multi ? 10 : 9;
  desc.mu = argc > mu_arg ? std::atof(argv[mu_arg]) : 0.0;
  desc.store = DC_STORE_F64 | DC_STORE_F32 | DC_STORE_F16S;
  desc.where = DC_WHERE_HOST;
  const size_t V = size_t(desc.dims[0]) * desc.dims[1] * desc.dims[2] * desc.dims[3];
  const size_t n = size_t(2 * desc.n_tv);
  if (V == 0 || n == 0 || n_rhs < 1 || reps < 1) {
    std::fprintf(stderr, "bad sizes\n");
    return 2;
  }
  // self blocks 4 I + 0.5 R / sqrt(n) (R uniform complex): well away from
  // singular; hops uniform complex / sqrt(n)
  std::vector<cd> self(V * n * n), hops(V * 4 * n * n);
  Seq g{12345};
  const double sc = 1.0 / std::sqrt(double(n));
  for (size_t x = 0; x < V; ++x)
    for (size_t i = 0; i < n; ++i)
      for (size_t j = 0; j < n; ++j)
        self[(x * n + i) * n + j] = cd(0.5 * sc * g.next(), 0.5 * sc * g.next()) + (i == j ? 4.0 : 0.0);
  for (cd& h : hops) h = cd(sc * g.next(), sc * g.next());
  dc_op_t op = nullptr;
  auto t0 = std::chrono::steady_clock::now();
  dc_ok(build_coarse_op(&desc, self.data(), hops.data(), nullptr, &op), "build_coarse_op");
  hip_ok(hipDeviceSynchronize(), "build");
  std::printf("[probe] operator %zu sites, n %zu built in %.1f s\n", V, n,
              std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  self.clear();
  self.shrink_to_fit();
  hops.clear();
  hops.shrink_to_fit();
  // vectors: complex128 for FP64, complex64 otherwise
  const size_t rows = multi ? V : V / 2;
  const size_t count = rows * n * size_t(n_rhs);
  const size_t zb = prec == DC_PREC_F64 ? 16 : 8;
  std::vector<double> h64;
  std::vector<float> h32;
  if (zb == 16) {
    h64.resize(2 * count);
    for (double& v : h64) v = g.next();
  } else {
    h32.resize(2 * count);
    for (float& v : h32) v = float(g.next());
  }
  void *x = nullptr, *y = nullptr;
  hip_ok(hipMalloc(&x, count * zb), "hipMalloc");
  hip_ok(hipMalloc(&y, count * zb), "hipMalloc");
  hip_ok(hipMemcpy(x, zb == 16 ? static_cast<const void*>(h64.data()) : h32.data(), count * zb,
                   hipMemcpyHostToDevice), "hipMemcpy");
  if (two) dc_ok(dc_set_reduced_kernels(1), "dc_set_reduced_kernels");
  dc_solve_opts po;
  dc_ok(dc_default_opts(&po), "dc_default_opts");
  po.d = 24;
  po.prec = prec;
  po.schur = 1;
  po.block_jacobi = 1;
  po.seed = 1;
  if (chain) {
    int32_t dused = 0;
    dc_ok(dc_poly_setup(op, &po, nullptr, nullptr, &dused), "dc_poly_setup");
    std::printf("[probe] polynomial of degree %d built\n", int(dused));
  }
  auto launch = [&]() {
    if (multi)
      dc_ok(dc_apply_multi(op, prec, 0, n_rhs, x, y, nullptr), "dc_apply_multi");
    else if (chain)
      dc_ok(dc_poly_apply(op, &po, x, y, nullptr), "dc_poly_apply");
    else
      dc_ok(dc_apply_reduced_bj(op, prec, x, y, nullptr), "dc_apply_reduced_bj");
  };
  launch();   // first call: tile choice / inverses
  hip_ok(hipDeviceSynchronize(), "warm-up");
  t0 = std::chrono::steady_clock::now();
  for (int r = 0; r < reps; ++r) launch();
  hip_ok(hipDeviceSynchronize(), "timed");
  const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  std::printf("[probe] %s %s n_rhs %d: %d applies, %.3f ms each\n", mode.c_str(), argv[7], n_rhs,
              reps, 1e3 * s / reps);
  hip_ok(hipFree(x), "hipFree");
  hip_ok(hipFree(y), "hipFree");
  destroy_coarse_op(op);
  return 0;
}
