// Shared types and helpers of the HIP library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

namespace dc {

// Interleaved complex value; 16-byte aligned for double (one dwordx4 load).
template <typename R>
struct alignas(2 * sizeof(R)) cx {
  R re, im;
};
using z64 = cx<double>;
using z32 = cx<float>;

template <typename R>
__host__ __device__ inline cx<R> mk(R re, R im) {
  cx<R> z;
  z.re = re;
  z.im = im;
  return z;
}

// Precision of a Krylov solve or an apply (matches DC_PREC_* in dcsolve.h).
enum Prec : int { P64 = 0, P32 = 1, P16S = 2 };

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct InvalidArg : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct NoMem : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct BadState : std::runtime_error {
  using std::runtime_error::runtime_error;
};
// A caller-provided workspace is too small for what the call needs.
struct WorkspaceShort : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define DC_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw ::dc::HipError(std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

// Number of sub-tile elements a lane holds for block size n: the n x n block
// is cut into an 8 x 8 grid of T x T sub-tiles, T = ceil(n / 8), one per lane
// of a 64-wide wavefront; the count is padded to a multiple of the elements
// one 16-byte load carries (1 complex double, 2 complex floats, 4 complex
// halves).
inline int tile_T(int n) { return (n + 7) / 8; }
inline int tile_elems(int n, int epl) {
  const int t = tile_T(n) * tile_T(n);
  return (t + epl - 1) / epl * epl;
}

}  // namespace dc
