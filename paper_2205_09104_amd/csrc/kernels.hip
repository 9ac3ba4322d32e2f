// HIP kernels for gfx950 (CDNA4): coarse-operator apply, Gram-Schmidt
// reductions, tall-skinny combinations, conversions and the gradient kernel.
#include "kernels.hpp"

#include <hip/hip_ext.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include <hip/hip_fp16.h>

// Scratch of the no-allocation reduced apply (dc_apply_reduced_noalloc): the
// odd-row temporary t_o lives in this file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes `scratch` itself
// to a kernel (in host code it names a host-side stand-in): it passes the
// device address that hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) unsigned char scratch[dc::kNoAllocScratchBytes];

namespace dc {

namespace {
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

void* noalloc_scratch(bool setup) {
  int dev = 0;
  DC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw InvalidArg("device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    if (!setup) return nullptr;
    void* p = nullptr;
    DC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw HipError("hipGetSymbolAddress returned a null address for the scratch array");
    g_scratch_dev[dev] = p;
  }
  return g_scratch_dev[dev];
}

namespace {

constexpr int kWave = 64;

template <typename T>
__device__ inline T shfl_xor(T v, int m) {
  return __shfl_xor(v, m, kWave);
}

__device__ inline double gam(int i, int n) { return i < (n >> 1) ? 1.0 : -1.0; }

template <typename R>
__device__ inline cx<R> ld(const cx<R>* p) {
  return *p;
}

// Block-wide sum of W doubles per thread (blockDim.x a multiple of 64, <= 1024),
// written as this block's partial: partials[w * nblk + block].  A second
// kernel (k_finalize) sums the partials of each value in a fixed order, so
// every reduction is deterministic.
template <int W>
__device__ void block_partials_at(double (&v)[W], double* partials, int bid, int nblk) {
  __shared__ double sh[16][W];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int t = 0; t < W; ++t) {
    double s = v[t];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += shfl_xor(s, o);
    if (lane == 0) sh[wave][t] = s;
  }
  __syncthreads();
  if (threadIdx.x < W) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[w][threadIdx.x];
    partials[size_t(threadIdx.x) * nblk + bid] = s;
  }
}

template <int W>
__device__ void block_partials(double (&v)[W], double* partials) {
  block_partials_at<W>(v, partials, blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
}

// result[v] = sum_b partials[v * nparts + b]; one 64-lane wave per value.
__device__ inline void finalize_value(const double* __restrict__ partials, int nparts,
                                      double* __restrict__ result, int v) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += 64) s += partials[size_t(v) * nparts + b];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += shfl_xor(s, o);
  if (threadIdx.x == 0) result[v] = s;
}

__global__ __launch_bounds__(64) void k_finalize(const double* __restrict__ partials, int nparts,
                                                 double* __restrict__ result,
                                                 const int* __restrict__ done) {
  if (done && *done) return;
  finalize_value(partials, nparts, result, blockIdx.x);
}

// ------------------------------------------------------------------ layout
// Tiled layout: block = 8 x 8 lane grid of T x T sub-tiles; lane l = lr*8+lc
// owns rows lr*T .. lr*T+T-1 and columns lc*T .. lc*T+T-1; its element
// e = a*T + b is (lr*T + a, lc*T + b).  Element e of lane l lives in 16-byte
// unit (e / EPL)*64 + l, slot e % EPL.

__device__ uint16_t f64_to_f16_rne(double x) {
  const uint64_t b = __double_as_longlong(x);
  const uint16_t sign = uint16_t((b >> 48) & 0x8000u);
  const int exp = int((b >> 52) & 0x7ff);
  const uint64_t mant = b & ((uint64_t(1) << 52) - 1);
  if (exp == 0x7ff) return sign | 0x7c00u | (mant ? 0x200u : 0u);
  if (exp == 0) return sign;  // FP64 subnormals are far below the FP16 range
  const int e = exp - 1023;
  if (e > 15) return sign | 0x7c00u;
  const uint64_t m = mant | (uint64_t(1) << 52);
  const int shift = (e >= -14) ? 42 : 42 + (-14 - e);
  if (shift >= 64) return sign;
  uint64_t keep = m >> shift;
  const uint64_t rem = m & ((uint64_t(1) << shift) - 1);
  const uint64_t half = uint64_t(1) << (shift - 1);
  if (rem > half || (rem == half && (keep & 1))) keep += 1;
  if (e >= -14) {
    uint32_t hexp = uint32_t(e + 15);
    if (keep >= (uint64_t(1) << 11)) {
      keep >>= 1;
      hexp += 1;
    }
    if (hexp >= 31) return sign | 0x7c00u;
    return uint16_t(sign | (hexp << 10) | uint32_t(keep & 0x3ffu));
  }
  return uint16_t(sign | uint32_t(keep));  // subnormal (or the smallest normal)
}

__global__ void k_layout(const z64* __restrict__ self_in, const z64* __restrict__ hops_in,
                         int V, int n, z64* __restrict__ o64, z32* __restrict__ o32,
                         uint32_t* __restrict__ o16, float* __restrict__ sc16) {
  const int blk = blockIdx.x;  // site*5 + slot
  const int site = blk / 5, slot = blk % 5;
  const size_t nn = size_t(n) * n;
  const z64* src = (slot == 0) ? self_in + size_t(site) * nn
                               : hops_in + (size_t(site) * 4 + (slot - 1)) * nn;
  const int T = (n + 7) / 8;
  const int TT = T * T;
  // block max of |Re|, |Im| for the FP16 scale
  __shared__ double smax[256];
  double mx = 0.0;
  for (size_t t = threadIdx.x; t < nn; t += blockDim.x) {
    const z64 z = src[t];
    mx = fmax(mx, fmax(fabs(z.re), fabs(z.im)));
  }
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    __syncthreads();
  }
  const float scale = float(smax[0]);
  const double dscale = double(scale);
  if (o16 && threadIdx.x == 0) sc16[blk] = scale;
  const int tt64 = ((TT + 0) / 1) * 1, tt32 = (TT + 1) / 2 * 2, tt16 = (TT + 3) / 4 * 4;
  const int total = 64 * tt16;  // covers every padded position of every layout
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int lane = t & 63, e = t >> 6;
    const int lr = lane >> 3, lc = lane & 7;
    const int a = e / T, bcol = e - a * T;
    const int i = lr * T + a, j = lc * T + bcol;
    z64 z = mk(0.0, 0.0);
    if (e < TT && i < n && j < n) z = src[size_t(i) * n + j];
    if (o64 && e < tt64) o64[size_t(blk) * tt64 * 64 + size_t(e) * 64 + lane] = z;
    if (o32 && e < tt32)
      o32[size_t(blk) * tt32 * 64 + (size_t(e >> 1) * 64 + lane) * 2 + (e & 1)] =
          mk(float(z.re), float(z.im));
    if (o16) {
      uint16_t cr = 0, ci = 0;
      if (dscale > 0.0) {
        cr = f64_to_f16_rne(z.re / dscale);
        ci = f64_to_f16_rne(z.im / dscale);
      }
      o16[size_t(blk) * tt16 * 64 + (size_t(e >> 2) * 64 + lane) * 4 + (e & 3)] =
          uint32_t(cr) | (uint32_t(ci) << 16);
    }
  }
}

__global__ void k_neighbours(int* nbr, int L0, int L1, int L2, int L3) {
  const int V = L0 * L1 * L2 * L3;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= V) return;
  int c[4];
  c[0] = x % L0;
  c[1] = (x / L0) % L1;
  c[2] = (x / (L0 * L1)) % L2;
  c[3] = x / (L0 * L1 * L2);
  const int L[4] = {L0, L1, L2, L3};
  for (int mu = 0; mu < 4; ++mu) {
    for (int dir = 0; dir < 2; ++dir) {
      int d[4] = {c[0], c[1], c[2], c[3]};
      d[mu] = dir == 0 ? (d[mu] + 1) % L[mu] : (d[mu] + L[mu] - 1) % L[mu];
      nbr[(dir * 4 + mu) * V + x] = d[0] + L0 * (d[1] + L1 * (d[2] + L2 * d[3]));
    }
  }
}

// ------------------------------------------------------------------ apply
// Element loaders of one lane's sub-tile for each storage precision.
template <int T, int P>
struct Tile;

template <int T>
struct Tile<T, P64> {
  using A = double;
  static constexpr int TT = T * T;
  static constexpr int UNITS = TT;  // one complex double per 16-byte unit
  __device__ static void load(const void* base, int lane, cx<double> (&m)[TT]) {
    const double2* p = static_cast<const double2*>(base);
#pragma unroll
    for (int e = 0; e < TT; ++e) {
      const double2 v = p[e * 64 + lane];
      m[e] = mk(v.x, v.y);
    }
  }
};

template <int T>
struct Tile<T, P32> {
  using A = float;
  static constexpr int TT = T * T;
  static constexpr int UNITS = (TT + 1) / 2;
  __device__ static void load(const void* base, int lane, cx<float> (&m)[TT]) {
    const float4* p = static_cast<const float4*>(base);
#pragma unroll
    for (int u = 0; u < UNITS; ++u) {
      const float4 v = p[u * 64 + lane];
      m[2 * u] = mk(v.x, v.y);
      if (2 * u + 1 < TT) m[2 * u + 1] = mk(v.z, v.w);
    }
  }
};

__device__ inline float h2f(uint32_t bits16) {
  return __half2float(__ushort_as_half(static_cast<unsigned short>(bits16 & 0xffffu)));
}

template <int T>
struct Tile<T, P16S> {
  using A = float;
  static constexpr int TT = T * T;
  static constexpr int UNITS = (TT + 3) / 4;
  __device__ static void load(const void* base, int lane, cx<float> (&m)[TT]) {
    const uint4* p = static_cast<const uint4*>(base);
#pragma unroll
    for (int u = 0; u < UNITS; ++u) {
      const uint4 v = p[u * 64 + lane];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (4 * u + q < TT) m[4 * u + q] = mk(h2f(w[q]), h2f(w[q] >> 16));
    }
  }
};

template <int P>
struct VecOf {
  using R = float;
};
template <>
struct VecOf<P64> {
  using R = double;
};

// Cross-lane sums inside a wavefront.  Lanes are l = lr*8 + lc.  Row sums
// (over lc, lanes l^1, l^2, l^4) use DPP quad permutes and the half-row mirror;
// column sums (over lr, lanes l^8, l^16, l^32) use a DPP row rotation by 8 and
// the gfx950 permlane16/32 swaps, whose two outputs add to v[l] + v[l^16]
// (resp. v[l^32]) in every lane.
__device__ inline int dpp_xor1(int v) { return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false); }
__device__ inline int dpp_xor2(int v) { return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false); }
__device__ inline int dpp_hmirror(int v) { return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false); }
__device__ inline int dpp_ror8(int v) { return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false); }

template <int CTL>
__device__ inline float dppf(float v) {
  int i = __float_as_int(v);
  if (CTL == 1) i = dpp_xor1(i);
  if (CTL == 2) i = dpp_xor2(i);
  if (CTL == 4) i = dpp_hmirror(i);
  if (CTL == 8) i = dpp_ror8(i);
  return __int_as_float(i);
}
template <int CTL>
__device__ inline double dppd(double v) {
  const long long b = __double_as_longlong(v);
  const float lo = dppf<CTL>(__int_as_float(int(b & 0xffffffff)));
  const float hi = dppf<CTL>(__int_as_float(int(b >> 32)));
  return __longlong_as_double((long long)(unsigned(__float_as_int(lo))) |
                              ((long long)(__float_as_int(hi)) << 32));
}
__device__ inline float dpp_any(float v, int ctl) {
  return ctl == 1 ? dppf<1>(v) : ctl == 2 ? dppf<2>(v) : ctl == 4 ? dppf<4>(v) : dppf<8>(v);
}

__device__ inline float sum_row8(float v) {  // over lc
  v += dppf<1>(v);
  v += dppf<2>(v);
  v += dppf<4>(v);
  return v;
}
__device__ inline double sum_row8(double v) {
  v += dppd<1>(v);
  v += dppd<2>(v);
  v += dppd<4>(v);
  return v;
}
__device__ inline float swap_sum16(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline float swap_sum32(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline double swap_pair16(double v, double& other) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = unsigned(b & 0xffffffff), hi = unsigned(b >> 32);
  const auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  other = __longlong_as_double((long long)rl[1] | ((long long)rh[1] << 32));
  return __longlong_as_double((long long)rl[0] | ((long long)rh[0] << 32));
}
__device__ inline double swap_pair32(double v, double& other) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = unsigned(b & 0xffffffff), hi = unsigned(b >> 32);
  const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  other = __longlong_as_double((long long)rl[1] | ((long long)rh[1] << 32));
  return __longlong_as_double((long long)rl[0] | ((long long)rh[0] << 32));
}
__device__ inline float sum_col8(float v) {  // over lr
  v += dppf<8>(v);
  v = swap_sum16(v);
  return swap_sum32(v);
}
__device__ inline double sum_col8(double v) {
  v += dppd<8>(v);
  double o;
  double a = swap_pair16(v, o);
  v = a + o;
  a = swap_pair32(v, o);
  return a + o;
}

// gbuf slots per site: 0..3 receive the backward hops Gamma5 B[x-mu,mu]^H
// Gamma5 psi_{x-mu}; 4 the self block (with i*tm*Gamma5 psi_x); 5..8 the
// forward hops B[x,mu] psi_{x+mu}.
constexpr int kSlots = 9;

// Block element access: FP64 / FP32 tiles are decoded into complex values,
// FP16 tiles stay packed (re in the low, im in the high half of a 32-bit
// word) and are widened inside the mixed-precision FMAs.
template <int T, int P>
struct TileRegs {
  cx<typename Tile<T, P>::A> m[T * T];
  __device__ void load(const void* base, int lane) { Tile<T, P>::load(base, lane, m); }
  __device__ void load_stream(const void* base, int lane) { load(base, lane); }
  __device__ float re(int e) const { return m[e].re; }
};

template <int T>
struct TileRegs<T, P16S> {
  static constexpr int TT = T * T;
  static constexpr int UNITS = (TT + 3) / 4;
  uint32_t w[UNITS * 4];
  __device__ void load(const void* base, int lane) {
    const uint4* p = static_cast<const uint4*>(base);
#pragma unroll
    for (int u = 0; u < UNITS; ++u) {
      const uint4 v = p[u * 64 + lane];
      w[4 * u] = v.x;
      w[4 * u + 1] = v.y;
      w[4 * u + 2] = v.z;
      w[4 * u + 3] = v.w;
    }
  }
  // the same with non-temporal loads, for tiles that one launch reads once
  __device__ void load_stream(const void* base, int lane) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4* p = static_cast<const u32x4*>(base);
#pragma unroll
    for (int u = 0; u < UNITS; ++u) {
      const u32x4 v = __builtin_nontemporal_load(p + u * 64 + lane);
      w[4 * u] = v.x;
      w[4 * u + 1] = v.y;
      w[4 * u + 2] = v.z;
      w[4 * u + 3] = v.w;
    }
  }
};

__device__ inline float lo_h(uint32_t w) {
  return float(__builtin_bit_cast(_Float16, static_cast<unsigned short>(w & 0xffffu)));
}
__device__ inline float hi_h(uint32_t w) {
  return float(__builtin_bit_cast(_Float16, static_cast<unsigned short>(w >> 16)));
}

// Accumulate one lane's sub-tile: f_a += z_ac pc_c and (hop blocks)
// g_c += conj(z_ac) pr_a.  npc_im = -Im(pc), npr_re = -Re(pr) avoid sign flips
// per element.
// f += M pc (row products, DOF) and g += M^T pr (column products, DOG) over one
// lane's T x T sub-tile.
template <int T, int P, bool DOF, bool DOG, typename A>
__device__ inline void tile_products(const TileRegs<T, P>& R, const cx<A> (&pc)[T],
                                     const A (&npc_im)[T], const cx<A> (&pr)[T],
                                     const A (&npr_re)[T], cx<A> (&f)[T], cx<A> (&g)[T]) {
#pragma unroll
  for (int a = 0; a < T; ++a)
#pragma unroll
    for (int c = 0; c < T; ++c) {
      A zr, zi;
      if constexpr (P == P16S) {
        zr = lo_h(R.w[a * T + c]);
        zi = hi_h(R.w[a * T + c]);
      } else {
        zr = R.m[a * T + c].re;
        zi = R.m[a * T + c].im;
      }
      if constexpr (DOF) {
        f[a].re = fma(zr, pc[c].re, f[a].re);
        f[a].re = fma(zi, npc_im[c], f[a].re);
        f[a].im = fma(zr, pc[c].im, f[a].im);
        f[a].im = fma(zi, pc[c].re, f[a].im);
      }
      if constexpr (DOG) {
        g[c].re = fma(zr, pr[a].re, g[c].re);
        g[c].re = fma(zi, pr[a].im, g[c].re);
        g[c].im = fma(zr, pr[a].im, g[c].im);
        g[c].im = fma(zi, npr_re[a], g[c].im);
      }
    }
}

// One stored block of one site, processed by one wave.  Full lattice (the
// default): the self block writes slot 4 of gbuf[x]; a hop block B[x,mu]
// writes B psi_{x+mu} into slot 5+mu of gbuf[x] and Gamma5 B^H Gamma5 psi_x
// into slot mu of gbuf[x+mu].  The odd-even reduction selects one direction
// (DIRS: 1 forward only, 2 backward only), addresses vectors and gbuf by the
// compressed index x / 2 of one parity (COMP) and may negate the products (NEG).
template <int T, int P, bool FULL, bool HOP, int DIRS = 3, bool COMP = false, bool NEG = false>
__device__ __forceinline__ void apply_one_block(
    const uint4* __restrict__ bp, const float* __restrict__ scales,
    const cx<typename VecOf<P>::R>* __restrict__ psi, cx<typename VecOf<P>::R>* __restrict__ gbuf,
    int item, int site, int slot, int src, int n, double tm) {
  using A = typename Tile<T, P>::A;
  using VR = typename VecOf<P>::R;
  constexpr bool DOF = !HOP || (DIRS & 1);
  constexpr bool DOG = HOP && (DIRS & 2);
  const int lane = threadIdx.x;
  const int lr = lane >> 3, lc = lane & 7;
  const int vsite = COMP ? (site >> 1) : site, vsrc = COMP ? (src >> 1) : src;
  TileRegs<T, P> R;
  R.load(bp, lane);
  cx<A> pc[T], pr[T];
  A npc_im[T], npr_re[T];
#pragma unroll
  for (int q = 0; q < T; ++q) {
    const int col = lc * T + q;
    pc[q] = mk(A(0), A(0));
    if (DOF && (FULL || col < n)) {
      const cx<VR> z = psi[size_t(HOP ? vsrc : vsite) * n + col];
      pc[q] = mk(A(z.re), A(z.im));
    }
    npc_im[q] = -pc[q].im;
    pr[q] = mk(A(0), A(0));
    if (DOG) {
      const int row = lr * T + q;
      if (FULL || row < n) {
        const cx<VR> z = psi[size_t(vsite) * n + row];
        pr[q] = (row < (n >> 1)) ? mk(A(z.re), A(z.im)) : mk(A(-z.re), A(-z.im));
      }
    }
    npr_re[q] = -pr[q].re;
  }
  cx<A> f[T], g[T];
#pragma unroll
  for (int q = 0; q < T; ++q) {
    f[q] = mk(A(0), A(0));
    g[q] = mk(A(0), A(0));
  }
  tile_products<T, P, DOF, DOG>(R, pc, npc_im, pr, npr_re, f, g);
  A s = A(1);
  if (P == P16S) s = A(scales[item]);
  if (NEG) s = -s;
  if constexpr (DOF) {
#pragma unroll
    for (int q = 0; q < T; ++q) {
      f[q].re = sum_row8(f[q].re) * s;
      f[q].im = sum_row8(f[q].im) * s;
    }
    if (lc == 0) {
      cx<VR>* dst = gbuf + (size_t(vsite) * kSlots + (HOP ? 4 + slot : 4)) * n;
#pragma unroll
      for (int q = 0; q < T; ++q) {
        const int row = lr * T + q;
        if (FULL || row < n) {
          cx<A> v = f[q];
          if (!HOP && tm != 0.0) {  // i * tm * Gamma5 psi_x in the accumulation precision
            const A t = A(row < (n >> 1) ? tm : -tm);
            const cx<VR> z = psi[size_t(vsite) * n + row];
            v.re -= t * A(z.im);
            v.im += t * A(z.re);
          }
          dst[row] = mk(VR(v.re), VR(v.im));
        }
      }
    }
  }
  if constexpr (DOG) {
#pragma unroll
    for (int q = 0; q < T; ++q) {
      g[q].re = sum_col8(g[q].re) * s;
      g[q].im = sum_col8(g[q].im) * s;
    }
    if (lr == 0) {
      cx<VR>* dst = gbuf + (size_t(vsrc) * kSlots + (slot - 1)) * n;  // x + mu receives it
#pragma unroll
      for (int q = 0; q < T; ++q) {
        const int col = lc * T + q;
        if (FULL || col < n) {
          const A gg = (col < (n >> 1)) ? A(1) : A(-1);
          dst[col] = mk(VR(gg * g[q].re), VR(gg * g[q].im));
        }
      }
    }
  }
}

// One 64-lane workgroup per (site, stored block).  The wave reads its block
// once with 16-byte loads (1 KB contiguous per load instruction) and forms
// from registers both the forward product B psi_{x+mu} (row sums) and the
// backward product Gamma5 B^H Gamma5 psi_x (column sums).  No barrier: waves
// of different sites overlap their loads with each other's arithmetic.
template <int T, int P, bool FULL>
__global__ __launch_bounds__(64) void k_apply_blocks(
    const void* __restrict__ blocks, const float* __restrict__ scales,
    const cx<typename VecOf<P>::R>* __restrict__ psi, cx<typename VecOf<P>::R>* __restrict__ gbuf,
    const int* __restrict__ nbr, int V, int n, int chunk, double tm, const int* __restrict__ done) {
  if (done && *done) return;
  // XCD-aware order: workgroup b runs on XCD b % 8; each XCD gets a
  // contiguous range of (site, block) items, so a site's blocks are streamed
  // together and neighbour vectors are shared through that XCD's L2.
  const int b = blockIdx.x;
  const int item = (b & 7) * chunk + (b >> 3);
  if (item >= 5 * V) return;
  const int site = item / 5, slot = item - 5 * site;  // slot 0 = A, 1 + mu = B[x, mu]
  const size_t blk_units = size_t(Tile<T, P>::UNITS) * 64;
  const uint4* bp = static_cast<const uint4*>(blocks) + size_t(item) * blk_units;
  if (slot == 0) {
    apply_one_block<T, P, FULL, false>(bp, scales, psi, gbuf, item, site, 0, site, n, tm);
  } else {
    const int src = nbr[(slot - 1) * V + site];
    apply_one_block<T, P, FULL, true>(bp, scales, psi, gbuf, item, site, slot, src, n, tm);
  }
}

// ------------------------------------------------------------------ odd-even reduction
// S = A_e - D_eo A_o^{-1} D_oe (Sec. 2.2) in factored form over compressed
// vectors (the site x of either parity sits at row x / 2).  A hop block
// B[x,mu] couples an even and an odd site, and each factor needs it in one
// direction only, so both kernels are site-centric: one workgroup per row, one
// wave per block of that row (every block is read once per launch), each
// wave's n-vector product into LDS, then a fixed-order sum (deterministic).

// One wave's product of a stored block (registers R, scale s) with the
// n-vector v, into dst (LDS): DIR 1 forward B v (row sums), DIR 2 backward
// Gamma5 B^H Gamma5 v (column sums), DIR 0 self block B v + i tm Gamma5 v.
template <int T, int P, bool FULL, int DIR>
__device__ __forceinline__ void wave_product(const TileRegs<T, P>& R, typename Tile<T, P>::A s,
                                             const cx<typename VecOf<P>::R>* __restrict__ v,
                                             cx<typename VecOf<P>::R>* dst, int n, double tm,
                                             int lane) {
  using A = typename Tile<T, P>::A;
  using VR = typename VecOf<P>::R;
  constexpr bool DOF = DIR != 2, DOG = DIR == 2;
  const int lr = lane >> 3, lc = lane & 7;
  cx<A> pc[T], pr[T], f[T], g[T];
  A npc_im[T], npr_re[T];
#pragma unroll
  for (int q = 0; q < T; ++q) {
    pc[q] = mk(A(0), A(0));
    pr[q] = mk(A(0), A(0));
    if (DOF) {
      const int col = lc * T + q;
      if (FULL || col < n) {
        const cx<VR> z = v[col];
        pc[q] = mk(A(z.re), A(z.im));
      }
    }
    if (DOG) {
      const int row = lr * T + q;
      if (FULL || row < n) {
        const cx<VR> z = v[row];
        pr[q] = (row < (n >> 1)) ? mk(A(z.re), A(z.im)) : mk(A(-z.re), A(-z.im));
      }
    }
    npc_im[q] = -pc[q].im;
    npr_re[q] = -pr[q].re;
    f[q] = mk(A(0), A(0));
    g[q] = mk(A(0), A(0));
  }
  tile_products<T, P, DOF, DOG>(R, pc, npc_im, pr, npr_re, f, g);
  if constexpr (DOF) {
#pragma unroll
    for (int q = 0; q < T; ++q) {
      f[q].re = sum_row8(f[q].re) * s;
      f[q].im = sum_row8(f[q].im) * s;
    }
    if (lc == 0) {
#pragma unroll
      for (int q = 0; q < T; ++q) {
        const int row = lr * T + q;
        if (FULL || row < n) {
          cx<A> w = f[q];
          if (DIR == 0 && tm != 0.0) {  // i * tm * Gamma5 v in the accumulation precision
            const A t = A(row < (n >> 1) ? tm : -tm);
            const cx<VR> z = v[row];
            w.re -= t * A(z.im);
            w.im += t * A(z.re);
          }
          dst[row] = mk(VR(w.re), VR(w.im));
        }
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < T; ++q) {
      g[q].re = sum_col8(g[q].re) * s;
      g[q].im = sum_col8(g[q].im) * s;
    }
    if (lr == 0) {
#pragma unroll
      for (int q = 0; q < T; ++q) {
        const int col = lc * T + q;
        if (FULL || col < n) {
          const A gg = (col < (n >> 1)) ? A(1) : A(-1);
          dst[col] = mk(VR(gg * g[q].re), VR(gg * g[q].im));
        }
      }
    }
  }
}

constexpr int kRedWaves = 9;   // waves per workgroup of the reduced kernels

template <int T, int P>
__device__ __forceinline__ const uint4* block_ptr(const void* blocks, size_t item) {
  return static_cast<const uint4*>(blocks) + item * (size_t(Tile<T, P>::UNITS) * 64);
}

// t_o = A_o^{-1} D_oe x_e.  Workgroup per odd row r (site x = osite[r]):
// waves 0-3 the forward hops B[x,mu] x_e(x+mu), waves 4-7 the backward hops
// Gamma5 B[x-mu,mu]^H Gamma5 x_e(x-mu), then wave 8 applies the inverse of
// x's self block to the sum of the eight products.
// Rows are ordered XCD-aware as in k_apply_blocks (contiguous rows per XCD).
template <int T, int P, bool FULL>
__global__ __launch_bounds__(64 * kRedWaves) void k_reduced_oe(
    const void* __restrict__ blocks, const float* __restrict__ scales,
    const void* __restrict__ inv, const float* __restrict__ invsc,
    const cx<typename VecOf<P>::R>* __restrict__ x_e, cx<typename VecOf<P>::R>* __restrict__ t_o,
    const int* __restrict__ nbr, const int* __restrict__ osite, int V, int n, int chunk,
    const int* __restrict__ done) {
  using A = typename Tile<T, P>::A;
  using VR = typename VecOf<P>::R;
  __shared__ cx<VR> part[8][64];
  if (done && *done) return;
  const int b = blockIdx.x;
  const int r = (b & 7) * chunk + (b >> 3);
  if (r >= (V >> 1)) return;
  const int x = osite[r];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  TileRegs<T, P> R;
  if (w < 4) {
    const int item = 5 * x + 1 + w;
    R.load(block_ptr<T, P>(blocks, size_t(item)), lane);
    const A s = (P == P16S) ? A(scales[item]) : A(1);
    const int src = nbr[w * V + x];
    wave_product<T, P, FULL, 1>(R, s, x_e + size_t(src >> 1) * n, part[w], n, 0.0, lane);
  } else if (w < 8) {
    const int mu = w - 4;
    const int y = nbr[(4 + mu) * V + x];
    const int item = 5 * y + 1 + mu;
    R.load(block_ptr<T, P>(blocks, size_t(item)), lane);
    const A s = (P == P16S) ? A(scales[item]) : A(1);
    wave_product<T, P, FULL, 2>(R, s, x_e + size_t(y >> 1) * n, part[w], n, 0.0, lane);
  }
  __syncthreads();
  if (w != 8) return;
  // loaded after the barrier: holding the tile across it would raise the
  // kernel's register count past what three 9-wave workgroups per CU allow
  // (staging it in LDS before the barrier measured no faster)
  R.load(block_ptr<T, P>(inv, size_t(x)), lane);
  const int lr = lane >> 3, lc = lane & 7;
  cx<A> pc[T], pr[T], f[T], g[T];
  A npc_im[T], npr_re[T];
#pragma unroll
  for (int q = 0; q < T; ++q) {
    const int col = lc * T + q;
    cx<VR> t = mk(VR(0), VR(0));
    if (FULL || col < n) {
      t = part[0][col];
#pragma unroll
      for (int k = 1; k < 8; ++k) {
        t.re += part[k][col].re;
        t.im += part[k][col].im;
      }
    }
    pc[q] = mk(A(t.re), A(t.im));
    npc_im[q] = -pc[q].im;
    pr[q] = mk(A(0), A(0));
    npr_re[q] = A(0);
    f[q] = mk(A(0), A(0));
    g[q] = mk(A(0), A(0));
  }
  tile_products<T, P, true, false>(R, pc, npc_im, pr, npr_re, f, g);
  const A s = (P == P16S) ? A(invsc[x]) : A(1);
#pragma unroll
  for (int q = 0; q < T; ++q) {
    f[q].re = sum_row8(f[q].re) * s;
    f[q].im = sum_row8(f[q].im) * s;
  }
  if (lc != 0) return;
#pragma unroll
  for (int q = 0; q < T; ++q) {
    const int row = lr * T + q;
    if (FULL || row < n) t_o[size_t(r) * n + row] = mk(VR(f[q].re), VR(f[q].im));
  }
}

// Epilogue of the reduced operator on one entry i of its output (t = the
// operator applied to the input at i; e = v, the apply's chain input, where
// it is read):
//   EPI 0: out = t
//   EPI 1: p = e - ca t; out = p; y = c0 e + cb p       (first chain step)
//   EPI 2: p = out - ca t; out = p; y += cb p            (later chain steps)
//   EPI 3: out = e - t                                    (residual, e = b)
template <int EPI, typename VR>
__device__ __forceinline__ void reduced_epilogue(size_t i, cx<VR> t, cx<VR>* out,
                                                 const cx<VR>* e, cx<VR>* y, z64 c0, z64 ca,
                                                 z64 cb) {
  if (EPI == 0) {
    out[i] = t;
  } else if (EPI == 3) {
    const cx<VR> bb = e[i];
    out[i] = mk(VR(bb.re - t.re), VR(bb.im - t.im));
  } else {
    const VR ar = VR(ca.re), ai = VR(ca.im), br = VR(cb.re), bi = VR(cb.im);
    const cx<VR> base = (EPI == 1) ? e[i] : out[i];
    cx<VR> p = base;
    p.re -= ar * t.re - ai * t.im;
    p.im -= ar * t.im + ai * t.re;
    out[i] = p;
    cx<VR> yv;
    if (EPI == 1) {
      const VR zr = VR(c0.re), zi = VR(c0.im);
      yv.re = zr * base.re - zi * base.im + (br * p.re - bi * p.im);
      yv.im = zr * base.im + zi * base.re + (br * p.im + bi * p.re);
    } else {
      yv = y[i];
      yv.re += br * p.re - bi * p.im;
      yv.im += br * p.im + bi * p.re;
    }
    y[i] = yv;
  }
}

// s = A_e x_e - D_eo t_o (A_e x_e omitted when x_e is null), workgroup per
// even row r (site x = esite[r]): wave 0 the self block, waves 1-4 the forward
// hops B[x,mu] t_o(x+mu), waves 5-8 the backward hops Gamma5 B[x-mu,mu]^H
// Gamma5 t_o(x-mu), both negated; summed in that order.
// BJ (left block Jacobi with B = D_ee, Sec. 3.2): s = x_e - A_e^{-1} D_eo t_o
// = B^{-1} (A_e x_e - D_eo t_o); wave 0 loads the inverse of x's self block
// (einv, same tiled layout, indexed by site) before the barrier, in place of
// the self block, and applies it to the sum of the eight hop products.
// Epilogue on row r: reduced_epilogue<EPI> (EPI 3 only without BJ).
template <int T, int P, bool FULL, int EPI, bool BJ>
__global__ __launch_bounds__(64 * kRedWaves) void k_reduced_eo(
    const void* __restrict__ blocks, const float* __restrict__ scales,
    const void* __restrict__ einv, const float* __restrict__ einvsc,
    const cx<typename VecOf<P>::R>* x_e, const cx<typename VecOf<P>::R>* __restrict__ t_o,
    const int* __restrict__ nbr, const int* __restrict__ esite, int V, int n, int chunk, double tm,
    cx<typename VecOf<P>::R>* out, const cx<typename VecOf<P>::R>* e, cx<typename VecOf<P>::R>* y,
    z64 c0, z64 ca, z64 cb, const int* __restrict__ done) {
  using A = typename Tile<T, P>::A;
  using VR = typename VecOf<P>::R;
  __shared__ cx<VR> part[kRedWaves][64];
  // BJ with FP32 / FP16 tiles: wave 0 stages the inverse in LDS before the
  // barrier (18 / 9 KB at n = 48); holding it in registers across the barrier
  // would cost a third of the resident workgroups.  FP64 tiles (37 KB) are
  // loaded after the barrier instead.
  constexpr bool STAGE = BJ && P != P64;
  constexpr int SU = STAGE ? Tile<T, P>::UNITS * 64 : 1;
  __shared__ uint4 inv_lds[SU];
  if (done && *done) return;
  const int b = blockIdx.x;
  const int r = (b & 7) * chunk + (b >> 3);
  if (r >= (V >> 1)) return;
  const int x = esite[r];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  TileRegs<T, P> R;
  if (w == 0) {
    if (STAGE) {
      const uint4* src = block_ptr<T, P>(einv, size_t(x));
#pragma unroll
      for (int u = 0; u < Tile<T, P>::UNITS; ++u) inv_lds[u * 64 + lane] = src[u * 64 + lane];
    } else if (BJ) {
      // FP64: loaded after the barrier
    } else if (x_e) {
      const int item = 5 * x;
      R.load(block_ptr<T, P>(blocks, size_t(item)), lane);
      const A s = (P == P16S) ? A(scales[item]) : A(1);
      wave_product<T, P, FULL, 0>(R, s, x_e + size_t(r) * n, part[0], n, tm, lane);
    } else {
      for (int i = lane; i < n; i += 64) part[0][i] = mk(VR(0), VR(0));
    }
  } else if (w < 5) {
    const int mu = w - 1;
    const int item = 5 * x + 1 + mu;
    R.load(block_ptr<T, P>(blocks, size_t(item)), lane);
    const A s = (P == P16S) ? A(scales[item]) : A(1);
    const int src = nbr[mu * V + x];
    wave_product<T, P, FULL, 1>(R, -s, t_o + size_t(src >> 1) * n, part[w], n, 0.0, lane);
  } else {
    const int mu = w - 5;
    const int yy = nbr[(4 + mu) * V + x];
    const int item = 5 * yy + 1 + mu;
    R.load(block_ptr<T, P>(blocks, size_t(item)), lane);
    const A s = (P == P16S) ? A(scales[item]) : A(1);
    wave_product<T, P, FULL, 2>(R, -s, t_o + size_t(yy >> 1) * n, part[w], n, 0.0, lane);
  }
  __syncthreads();
  if (w != 0) return;
  if constexpr (BJ) {
    if (STAGE) R.load(inv_lds, lane);
    else R.load(block_ptr<T, P>(einv, size_t(x)), lane);
    const int lr = lane >> 3, lc = lane & 7;
    cx<A> pc[T], pr[T], f[T], g[T];
    A npc_im[T], npr_re[T];
#pragma unroll
    for (int q = 0; q < T; ++q) {
      const int col = lc * T + q;
      cx<VR> t = mk(VR(0), VR(0));
      if (FULL || col < n) {
        t = part[1][col];
#pragma unroll
        for (int k = 2; k < kRedWaves; ++k) {
          t.re += part[k][col].re;
          t.im += part[k][col].im;
        }
      }
      pc[q] = mk(A(t.re), A(t.im));
      npc_im[q] = -pc[q].im;
      pr[q] = mk(A(0), A(0));
      npr_re[q] = A(0);
      f[q] = mk(A(0), A(0));
      g[q] = mk(A(0), A(0));
    }
    tile_products<T, P, true, false>(R, pc, npc_im, pr, npr_re, f, g);
    const A s = (P == P16S) ? A(einvsc[x]) : A(1);
    // the row sums leave row lr*T + q's value in all eight lanes of row group
    // lr; lane lc takes row lr*T + lc
    cx<A> mine = mk(A(0), A(0));
#pragma unroll
    for (int q = 0; q < T; ++q) {
      const A fr = sum_row8(f[q].re) * s, fi = sum_row8(f[q].im) * s;
      if (q == lc) mine = mk(fr, fi);
    }
    const int row = lr * T + lc;
    if (lc >= T || !(FULL || row < n)) return;
    const size_t i = size_t(r) * n + row;
    cx<VR> t = mk(VR(mine.re), VR(mine.im));
    if (x_e) {
      const cx<VR> xv = x_e[i];
      t.re += xv.re;
      t.im += xv.im;
    }
    reduced_epilogue<EPI>(i, t, out, e, y, c0, ca, cb);
  } else {
    for (int c = lane; c < n; c += 64) {
      cx<VR> t = part[0][c];
#pragma unroll
      for (int k = 1; k < kRedWaves; ++k) {
        t.re += part[k][c].re;
        t.im += part[k][c].im;
      }
      reduced_epilogue<EPI>(size_t(r) * n + c, t, out, e, y, c0, ca, cb);
    }
  }
}

// Single-read form of the same operator.  Each hop block couples exactly one
// odd and one even site, so the odd row's workgroup can apply it in both
// directions while it holds it: k_reduced_scatter forms t_o(x) as k_reduced_oe
// does (same products, same order), keeps the eight hop tiles in registers
// across the barriers, and then applies each of them the other way to t_o(x),
// which gives one of the eight D_eo products of the even neighbour it couples
// to.  Those go to hp[row][slot][n] of that even row: slots 0-3 its forward hops
// B[e,mu] t_o(e+mu), 4-7 its backward hops Gamma5 B[e-mu,mu]^H Gamma5 t_o(e-mu);
// every (row, slot) has exactly one writer.  k_reduced_gather then sums the
// eight slots in that order and finishes the row with A_e (or A_e^{-1} for
// block Jacobi) and the epilogue.  Per site pair ten blocks are read instead
// of eighteen; the sums and signs are those of the two-kernel form, so the
// results agree with it bit for bit.
//
// Eight waves per workgroup, one per hop tile; the tiles and the inverse are
// loaded non-temporally (one launch reads each once).  The odd site's inverse tile is
// staged in LDS and its product with the summed hop products is split over the
// eight waves: wave w takes rows w T .. w T + T - 1, which lane group lr = w
// holds in the one-wave tile layout; its lane (a, lc) forms the partial sum
// that lane (w, lc) forms for row a there, and the same row reduction over lc
// finishes it.  FP16 tiles up to n = 48 fit three workgroups per CU (7 waves
// per SIMD, 70 registers, no spill); at 8 waves per SIMD the registers spill
// and the kernel runs slower.
template <int T, int P>
constexpr int scatter_min_waves() { return (P == P16S && T <= 6) ? 7 : 1; }

template <int T, int P>
__global__ __launch_bounds__(512, (scatter_min_waves<T, P>())) void k_reduced_scatter(
    const void* __restrict__ blocks, const float* __restrict__ scales,
    const void* __restrict__ inv, const float* __restrict__ invsc,
    const cx<typename VecOf<P>::R>* __restrict__ x_e, cx<typename VecOf<P>::R>* __restrict__ hp,
    const int* __restrict__ nbr, const int* __restrict__ osite, int V, int n, int chunk,
    const int* __restrict__ done) {
  using A = typename Tile<T, P>::A;
  using VR = typename VecOf<P>::R;
  constexpr int UNITS = Tile<T, P>::UNITS;
  __shared__ cx<VR> part[8][64];
  __shared__ cx<VR> tsum[64];
  __shared__ cx<VR> tx[64];
  __shared__ uint4 inv_lds[UNITS * 64];
  if (done && *done) return;
  const int b = blockIdx.x;
  const int r = (b & 7) * chunk + (b >> 3);
  if (r >= (V >> 1)) return;   // uniform per workgroup: no barrier is skipped by part of it
  const int x = osite[r];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  {
    const uint4* ip = block_ptr<T, P>(inv, size_t(x));
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    for (int u = w; u < UNITS; u += 8) {   // read once per launch: non-temporal
      const u32x4 q = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(ip) + u * 64 + lane);
      inv_lds[u * 64 + lane] = make_uint4(q.x, q.y, q.z, q.w);
    }
  }
  TileRegs<T, P> R;
  A s = A(1);
  size_t dst = 0;   // element offset of this wave's D_eo product in hp
  if (w < 4) {
    const int item = 5 * x + 1 + w;
    R.load_stream(block_ptr<T, P>(blocks, size_t(item)), lane);
    if (P == P16S) s = A(scales[item]);
    const int src = nbr[w * V + x];
    wave_product<T, P, true, 1>(R, s, x_e + size_t(src >> 1) * n, part[w], n, 0.0, lane);
    dst = (size_t(src >> 1) * 8 + 4 + w) * n;        // backward hop mu = w of even x + mu
  } else {
    const int mu = w - 4;
    const int y = nbr[(4 + mu) * V + x];
    const int item = 5 * y + 1 + mu;
    R.load_stream(block_ptr<T, P>(blocks, size_t(item)), lane);
    if (P == P16S) s = A(scales[item]);
    wave_product<T, P, true, 2>(R, s, x_e + size_t(y >> 1) * n, part[w], n, 0.0, lane);
    dst = (size_t(y >> 1) * 8 + mu) * n;             // forward hop mu of even x - mu
  }
  __syncthreads();
  if (w == 0) {   // the eight products summed in a fixed order
    cx<VR> t = mk(VR(0), VR(0));
    if (lane < n) {
      t = part[0][lane];
#pragma unroll
      for (int k = 1; k < 8; ++k) {
        t.re += part[k][lane].re;
        t.im += part[k][lane].im;
      }
    }
    tsum[lane] = t;
  }
  __syncthreads();
  {
    // rows w T + a of A_o^{-1} tsum: lane (a, lc) forms sum_c z[wT+a][lc T+c]
    // tsum[lc T + c] over its T columns (the tile element a T + c of layout
    // lane w*8 + lc), the row reduction adds the eight lanes of a row
    const int a = lane >> 3, lc = lane & 7;
    const int src_lane = w * 8 + lc;
    cx<A> f = mk(A(0), A(0));
    if (a < T) {
#pragma unroll
      for (int c = 0; c < T; ++c) {
        const int e = a * T + c;
        const cx<VR> t = tsum[lc * T + c];
        const A pr_ = A(t.re), pi_ = A(t.im);
        A zr, zi;
        if constexpr (P == P16S) {
          const uint4 q = inv_lds[(e >> 2) * 64 + src_lane];
          const uint32_t word = (e & 3) == 0 ? q.x : (e & 3) == 1 ? q.y : (e & 3) == 2 ? q.z : q.w;
          zr = lo_h(word);
          zi = hi_h(word);
        } else {
          const float4 q = reinterpret_cast<const float4*>(inv_lds)[(e >> 1) * 64 + src_lane];
          zr = (e & 1) ? q.z : q.x;
          zi = (e & 1) ? q.w : q.y;
        }
        f.re = fma(zr, pr_, f.re);
        f.re = fma(zi, -pi_, f.re);
        f.im = fma(zr, pi_, f.im);
        f.im = fma(zi, pr_, f.im);
      }
    }
    const A si = (P == P16S) ? A(invsc[x]) : A(1);
    f.re = sum_row8(f.re) * si;
    f.im = sum_row8(f.im) * si;
    if (lc == 0 && a < T) tx[w * T + a] = mk(VR(f.re), VR(f.im));
  }
  __syncthreads();
  if (w < 4)
    wave_product<T, P, true, 2>(R, s, tx, hp + dst, n, 0.0, lane);
  else
    wave_product<T, P, true, 1>(R, s, tx, hp + dst, n, 0.0, lane);
}

// Second kernel of the single-read form: one wave per even row r (site
// x = esite[r]); its block is loaded non-temporally (read once per launch).  The eight slots of hp[r], negated and summed in slot order,
// are the hop terms k_reduced_eo sums from its own products; the row is then
// finished as there: BJ x_e + A_e^{-1} (sum), else A_e x_e (+ i tm Gamma5 x_e)
// with the terms added one by one, and the epilogue.
template <int T, int P, int EPI, bool BJ>
__global__ __launch_bounds__(64) void k_reduced_gather(
    const void* __restrict__ blocks, const float* __restrict__ scales,
    const void* __restrict__ einv, const float* __restrict__ einvsc,
    const cx<typename VecOf<P>::R>* x_e, const cx<typename VecOf<P>::R>* __restrict__ hp,
    const int* __restrict__ esite, int V, int n, int chunk, double tm,
    cx<typename VecOf<P>::R>* out, const cx<typename VecOf<P>::R>* e, cx<typename VecOf<P>::R>* y,
    z64 c0, z64 ca, z64 cb, const int* __restrict__ done) {
  using A = typename Tile<T, P>::A;
  using VR = typename VecOf<P>::R;
  __shared__ cx<VR> self_part[64];
  __shared__ cx<VR> tsum[64];
  if (done && *done) return;
  const int b = blockIdx.x;
  const int r = (b & 7) * chunk + (b >> 3);
  if (r >= (V >> 1)) return;
  const int x = esite[r];
  const int lane = threadIdx.x;
  TileRegs<T, P> R;
  if (BJ) R.load_stream(block_ptr<T, P>(einv, size_t(x)), lane);
  cx<VR> h[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    h[k] = mk(VR(0), VR(0));
    if (lane < n) h[k] = hp[(size_t(r) * 8 + k) * n + lane];
  }
  if constexpr (BJ) {
    cx<VR> t = mk(-h[0].re, -h[0].im);
#pragma unroll
    for (int k = 1; k < 8; ++k) {
      t.re += -h[k].re;
      t.im += -h[k].im;
    }
    tsum[lane] = t;
    __syncthreads();
    const int lr = lane >> 3, lc = lane & 7;
    cx<A> pc[T], pr[T], f[T], g[T];
    A npc_im[T], npr_re[T];
#pragma unroll
    for (int q = 0; q < T; ++q) {
      const cx<VR> u = tsum[lc * T + q];
      pc[q] = mk(A(u.re), A(u.im));
      npc_im[q] = -pc[q].im;
      pr[q] = mk(A(0), A(0));
      npr_re[q] = A(0);
      f[q] = mk(A(0), A(0));
      g[q] = mk(A(0), A(0));
    }
    tile_products<T, P, true, false>(R, pc, npc_im, pr, npr_re, f, g);
    const A s = (P == P16S) ? A(einvsc[x]) : A(1);
    cx<A> mine = mk(A(0), A(0));
#pragma unroll
    for (int q = 0; q < T; ++q) {
      const A fr = sum_row8(f[q].re) * s, fi = sum_row8(f[q].im) * s;
      if (q == lc) mine = mk(fr, fi);
    }
    const int row = lr * T + lc;
    if (lc >= T) return;
    const size_t i = size_t(r) * n + row;
    cx<VR> o = mk(VR(mine.re), VR(mine.im));
    if (x_e) {
      const cx<VR> xv = x_e[i];
      o.re += xv.re;
      o.im += xv.im;
    }
    reduced_epilogue<EPI>(i, o, out, e, y, c0, ca, cb);
  } else {
    if (x_e) {
      const int item = 5 * x;
      R.load_stream(block_ptr<T, P>(blocks, size_t(item)), lane);
      const A s = (P == P16S) ? A(scales[item]) : A(1);
      wave_product<T, P, true, 0>(R, s, x_e + size_t(r) * n, self_part, n, tm, lane);
    } else {
      self_part[lane] = mk(VR(0), VR(0));
    }
    __syncthreads();
    if (lane >= n) return;
    cx<VR> o = self_part[lane];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      o.re += -h[k].re;
      o.im += -h[k].im;
    }
    reduced_epilogue<EPI>(size_t(r) * n + lane, o, out, e, y, c0, ca, cb);
  }
}

// Sum of the 9 slots in a fixed order: self, forward hops, backward hops.
template <typename VR>
__device__ inline cx<VR> gather5(const cx<VR>* __restrict__ gbuf, size_t i, int n) {
  const size_t site = i / n, c = i - site * n;
  const size_t base = site * kSlots * n + c;
  cx<VR> s = gbuf[base + 4 * size_t(n)];
#pragma unroll
  for (int w = 5; w < 9; ++w) {
    const cx<VR> t = gbuf[base + size_t(w) * n];
    s.re += t.re;
    s.im += t.im;
  }
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const cx<VR> t = gbuf[base + size_t(w) * n];
    s.re += t.re;
    s.im += t.im;
  }
  return s;
}

// ------------------------------------------------------------------ block Jacobi
// In-place Gauss-Jordan inversion (partial pivoting) of each site's self
// block A_x + i*tm*Gamma5, one workgroup per site, matrix in LDS; the inverse
// is written in the tiled layout of every requested precision.
__device__ void write_tiled(const z64* M, int n, int blk, z64* o64, z32* o32, uint32_t* o16,
                            float* sc16, double* red) {
  const int T = (n + 7) / 8, TT = T * T;
  const int tt32 = (TT + 1) / 2 * 2, tt16 = (TT + 3) / 4 * 4;
  double mx = 0.0;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x)
    mx = fmax(mx, fmax(fabs(M[t].re), fabs(M[t].im)));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const float scale = float(red[0]);
  const double dscale = double(scale);
  if (o16 && threadIdx.x == 0) sc16[blk] = scale;
  for (int t = threadIdx.x; t < 64 * tt16; t += blockDim.x) {
    const int lane = t & 63, e = t >> 6;
    const int i = (lane >> 3) * T + e / T, j = (lane & 7) * T + e % T;
    z64 z = mk(0.0, 0.0);
    if (e < TT && i < n && j < n) z = M[i * n + j];
    if (o64 && e < TT) o64[size_t(blk) * TT * 64 + size_t(e) * 64 + lane] = z;
    if (o32 && e < tt32)
      o32[size_t(blk) * tt32 * 64 + (size_t(e >> 1) * 64 + lane) * 2 + (e & 1)] =
          mk(float(z.re), float(z.im));
    if (o16) {
      uint16_t cr = 0, ci = 0;
      if (dscale > 0.0) {
        cr = f64_to_f16_rne(z.re / dscale);
        ci = f64_to_f16_rne(z.im / dscale);
      }
      o16[size_t(blk) * tt16 * 64 + (size_t(e >> 2) * 64 + lane) * 4 + (e & 3)] =
          uint32_t(cr) | (uint32_t(ci) << 16);
    }
  }
}

__global__ __launch_bounds__(256) void k_invert_blocks(const z64* __restrict__ tiled64, int n,
                                                       double tm, z64* o64, z32* o32,
                                                       uint32_t* o16, float* sc16,
                                                       int* __restrict__ singular) {
  extern __shared__ z64 M[];               // n*n entries
  __shared__ int perm[64];
  __shared__ double red[256];
  __shared__ int piv_row;
  __shared__ z64 pivot_row[64];
  __shared__ z64 pivot_col[64];
  const int site = blockIdx.x;
  const int nn = n * n;
  const int T = (n + 7) / 8, TT = T * T;
  const z64* src = tiled64 + size_t(site) * 5 * TT * 64;  // slot 0 of the site: A_x
  for (int t = threadIdx.x; t < nn; t += blockDim.x) {
    const int i = t / n, j = t % n;
    const int lane = (i / T) * 8 + j / T, e = (i % T) * T + (j % T);
    z64 z = src[size_t(e) * 64 + lane];
    if (i == j) z.im += (i < (n >> 1)) ? tm : -tm;
    M[t] = z;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // pivot: largest |M[i][k]| for i >= k (first wave; ties to the lower row)
    if (threadIdx.x < 64) {
      double best = -1.0;
      int bi = k;
      for (int i = k + int(threadIdx.x); i < n; i += 64) {
        const double a = fabs(M[i * n + k].re) + fabs(M[i * n + k].im);
        if (a > best) { best = a; bi = i; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (threadIdx.x == 0) {
        piv_row = bi;
        perm[k] = bi;
        if (!(best > 0.0)) *singular = 1;
      }
    }
    __syncthreads();
    const int p = piv_row;
    if (p != k)
      for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const z64 a = M[k * n + j];
        M[k * n + j] = M[p * n + j];
        M[p * n + j] = a;
      }
    __syncthreads();
    const z64 akk = M[k * n + k];
    const double den = akk.re * akk.re + akk.im * akk.im;
    const z64 d = den > 0.0 ? mk(akk.re / den, -akk.im / den) : mk(0.0, 0.0);  // 1 / a_kk
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const z64 a = (j == k) ? mk(1.0, 0.0) : M[k * n + j];
      pivot_row[j] = mk(a.re * d.re - a.im * d.im, a.re * d.im + a.im * d.re);
      pivot_col[j] = M[j * n + k];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nn; t += blockDim.x) {
      const int i = t / n, j = t % n;
      if (i == k) {
        M[t] = pivot_row[j];
      } else {
        const z64 f = pivot_col[i];
        const z64 r = (j == k) ? mk(0.0, 0.0) : M[t];
        const z64 pr = pivot_row[j];
        // M[i][j] = (j == k ? 0 : M[i][j]) - f * pivot_row[j]
        M[t] = mk(r.re - (f.re * pr.re - f.im * pr.im), r.im - (f.re * pr.im + f.im * pr.re));
      }
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int k = n - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k)
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const z64 a = M[i * n + k];
        M[i * n + k] = M[i * n + p];
        M[i * n + p] = a;
      }
    __syncthreads();
  }
  write_tiled(M, n, site, o64, o32, o16, sc16, red);
}

// out_x = M_x t_x with M_x the stored inverse and t either the sum of the 9
// gbuf slots (t = D psi) or a plain vector; one wave per site; epilogue as in
// the gather kernels (0 store, 1 poly_first, 2 poly).
template <int T, int P, bool FULL, bool FROMBUF, int EPI>
__global__ __launch_bounds__(64) void k_block_jacobi(
    const void* __restrict__ blocks, const float* __restrict__ scales,
    const cx<typename VecOf<P>::R>* __restrict__ tin, cx<typename VecOf<P>::R>* out,
    const cx<typename VecOf<P>::R>* vin, cx<typename VecOf<P>::R>* y, int V, int n, int chunk,
    z64 c0, z64 ca, z64 cb, const int* __restrict__ done, const int* __restrict__ rowsite) {
  using A = typename Tile<T, P>::A;
  using VR = typename VecOf<P>::R;
  if (done && *done) return;
  const int b = blockIdx.x;
  const int site = (b & 7) * chunk + (b >> 3);   // row of the vectors
  if (site >= V) return;
  const int blk = rowsite ? rowsite[site] : site;  // block of that row's lattice site
  const int lane = threadIdx.x, lr = lane >> 3, lc = lane & 7;
  const size_t blk_units = size_t(Tile<T, P>::UNITS) * 64;
  TileRegs<T, P> R;
  R.load(static_cast<const uint4*>(blocks) + size_t(blk) * blk_units, lane);
  cx<A> pc[T], pr[T], f[T], g[T];
  A npc_im[T], npr_re[T];
#pragma unroll
  for (int q = 0; q < T; ++q) {
    const int col = lc * T + q;
    cx<A> t = mk(A(0), A(0));
    if (FULL || col < n) {
      if (FROMBUF) {
        const cx<VR> z = gather5(tin, size_t(site) * n + col, n);
        t = mk(A(z.re), A(z.im));
      } else {
        const cx<VR> z = tin[size_t(site) * n + col];
        t = mk(A(z.re), A(z.im));
      }
    }
    pc[q] = t;
    npc_im[q] = -t.im;
    pr[q] = mk(A(0), A(0));
    npr_re[q] = A(0);
    f[q] = mk(A(0), A(0));
    g[q] = mk(A(0), A(0));
  }
  tile_products<T, P, true, false>(R, pc, npc_im, pr, npr_re, f, g);
  A s = A(1);
  if (P == P16S) s = A(scales[blk]);
#pragma unroll
  for (int q = 0; q < T; ++q) {
    f[q].re = sum_row8(f[q].re) * s;
    f[q].im = sum_row8(f[q].im) * s;
  }
  if (lc != 0) return;
#pragma unroll
  for (int q = 0; q < T; ++q) {
    const int row = lr * T + q;
    if (!(FULL || row < n)) continue;
    const size_t i = size_t(site) * n + row;
    const VR sr = VR(f[q].re), si = VR(f[q].im);
    if (EPI == 0) {
      out[i] = mk(sr, si);
    } else {
      const cx<VR> base = (EPI == 1) ? vin[i] : out[i];
      cx<VR> p = base;
      p.re -= VR(ca.re) * sr - VR(ca.im) * si;
      p.im -= VR(ca.re) * si + VR(ca.im) * sr;
      out[i] = p;
      cx<VR> yy = (EPI == 1) ? mk(VR(VR(c0.re) * base.re - VR(c0.im) * base.im),
                                  VR(VR(c0.re) * base.im + VR(c0.im) * base.re))
                             : y[i];
      yy.re += VR(cb.re) * p.re - VR(cb.im) * p.im;
      yy.im += VR(cb.re) * p.im + VR(cb.im) * p.re;
      y[i] = yy;
    }
  }
}

// ------------------------------------------------------------------ batched chain step
// For r < R (device pointer arrays): first step (first != 0):
//   prod_r = v_r - ca t_r;  y_r = c0 v_r + cb prod_r,
// later steps: prod_r -= ca t_r;  y_r += cb prod_r  (t_r = A~ of the chain input).
template <typename VR>
__device__ __forceinline__ void chain_multi_body(const cx<VR>* const* __restrict__ t,
                                                 const cx<VR>* const* __restrict__ v,
                                                 cx<VR>* const* __restrict__ prod,
                                                 cx<VR>* const* __restrict__ y, size_t N, z64 c0,
                                                 z64 ca, z64 cb, int first, int r) {
  const cx<VR>* tr = t[r];
  cx<VR>* pr = prod[r];
  cx<VR>* yr = y[r];
  const VR ar = VR(ca.re), ai = VR(ca.im), br = VR(cb.re), bi = VR(cb.im);
  const VR zr = VR(c0.re), zi = VR(c0.im);
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
    const cx<VR> s = tr[i];
    const cx<VR> base = first ? v[r][i] : pr[i];
    cx<VR> p = base;
    p.re -= ar * s.re - ai * s.im;
    p.im -= ar * s.im + ai * s.re;
    pr[i] = p;
    cx<VR> yy = first ? mk(VR(zr * base.re - zi * base.im), VR(zr * base.im + zi * base.re)) : yr[i];
    yy.re += br * p.re - bi * p.im;
    yy.im += br * p.im + bi * p.re;
    yr[i] = yy;
  }
}

template <typename VR>
__global__ void k_chain_multi(const cx<VR>* const* __restrict__ t, const cx<VR>* const* __restrict__ v,
                              cx<VR>* const* __restrict__ prod, cx<VR>* const* __restrict__ y,
                              size_t N, z64 c0, z64 ca, z64 cb, int first) {
  chain_multi_body<VR>(t, v, prod, y, N, c0, ca, cb, first, blockIdx.y);
}

// The chain step of several operators' column sets in one launch: blockIdx.z
// is the operator, blockIdx.y its column (elementwise, so any grid gives the
// per-operator launches' results).
template <typename VR>
__global__ void k_chain_groups(ChainGroups g, int first) {
  const int gi = int(blockIdx.z), r = int(blockIdx.y);
  if (gi >= g.count || r >= g.R[gi]) return;
  chain_multi_body<VR>(static_cast<const cx<VR>* const*>(g.t[gi]),
                       static_cast<const cx<VR>* const*>(g.v[gi]),
                       static_cast<cx<VR>* const*>(g.prod[gi]), static_cast<cx<VR>* const*>(g.y[gi]),
                       g.N[gi], g.c0[gi], g.ca[gi], g.cb[gi], first, r);
}

// ------------------------------------------------------------------ multi-RHS apply
// Y_r = D X_r for R right-hand sides at once.  One workgroup (4 waves) per
// site accumulates the 9 couplings of the site into an n x R output panel
// held in MFMA accumulators: each coupling stages its block (as the vector
// precision) and the source panel in LDS, and the complex product runs as
// three real GEMMs (Re M Re P, Im M Im P, (Re M + Im M)(Re P + Im P)) on
// 16x16x4 MFMA tiles.
// Backward hops Gamma5 B^H Gamma5 read the staged forward block transposed.
// Every stored block is read once per site that uses it (9 block reads per
// site; the MFMA work, 72 V n^2 R flops, dominates for R >= 16).
template <typename VT>
struct Mfma;
template <>
struct Mfma<float> {
  using acc_t = __attribute__((ext_vector_type(4))) float;
  __device__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lk, int q) { return lk * 4 + q; }
};
template <>
struct Mfma<double> {
  using acc_t = __attribute__((ext_vector_type(4))) double;
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lk, int q) { return lk + 4 * q; }
};


// The grid runs over a work list of the sites of up to kMaxMultiOps operators
// (a mixed batch of lattices with one block size n): workgroup x belongs to the
// operator whose site range [site0, site0 + V) contains it; grid.y tiles the
// right-hand sides of the operator with the most, tiles past an operator's own
// count exit at entry.
template <int NP, int P, typename VT, int RB>
__global__ __launch_bounds__(256) void k_apply_multi(MultiOps ops) {
  static_assert(RB % 16 == 0 && RB <= 64, "right-hand-side tile of 16, 32 or 64");
  using acc_t = typename Mfma<VT>::acc_t;
  // select this workgroup's operator (uniform; fields copied by select so the
  // kernel-argument array is never indexed dynamically)
  int o = 0;
#pragma unroll
  for (int i = 1; i < kMaxMultiOps; ++i)
    if (i < ops.n_ops && int(blockIdx.x) >= ops.op[i].site0) o = i;
  const void* blocks = ops.op[0].blocks;
  const float* scales = ops.op[0].scales;
  const int* nbr = ops.op[0].nbr;
  const void* const* xin_v = ops.op[0].xin;
  void* const* yout_v = ops.op[0].yout;
  int V = ops.op[0].V, R = ops.op[0].R, site0 = ops.op[0].site0;
  double tm = ops.op[0].tm;
#pragma unroll
  for (int i = 1; i < kMaxMultiOps; ++i)
    if (i == o) {
      blocks = ops.op[i].blocks;
      scales = ops.op[i].scales;
      nbr = ops.op[i].nbr;
      xin_v = ops.op[i].xin;
      yout_v = ops.op[i].yout;
      V = ops.op[i].V;
      R = ops.op[i].R;
      site0 = ops.op[i].site0;
      tm = ops.op[i].tm;
    }
  const int n = ops.n, g5io = ops.g5io;
  const auto* const* xin = reinterpret_cast<const cx<VT>* const*>(xin_v);
  auto* const* yout = reinterpret_cast<cx<VT>* const*>(yout_v);
  if (int(blockIdx.y) * RB >= R) return;
  constexpr int LD = NP + 1;                  // padded row stride of every LDS plane
  extern __shared__ unsigned char smem[];
  VT* Mr = reinterpret_cast<VT*>(smem);       // [NP][LD] coupling matrix, real part
  VT* Mi = Mr + NP * LD;                      // imaginary part
  VT* Pr = Mi + NP * LD;                      // [RB][LD] panel: row r = x_r at the source
  VT* Pi = Pr + RB * LD;
  const int site = int(blockIdx.x) - site0;
  const int r0 = blockIdx.y * RB;
  const int Rc = min(RB, R - r0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lk = lane >> 4;
  const int T = (n + 7) / 8, TT = T * T;
  constexpr int epl = (P == P64) ? 1 : (P == P32 ? 2 : 4);   // block entries per 16-byte unit
  const int upl = (TT + epl - 1) / epl;                      // units per lane of a block
  const int nunits = 64 * upl;
  const int half = n >> 1;
  // output tiles (16 x 16): RT row tiles x RB/16 column tiles; a partial
  // right-hand-side tile computes on zero padding and stores only its Rc
  // columns.  FP32 products: every wave gets the same share of MFMA work --
  // the k range is split KS ways (KS = 4 / gcd(NT, 4)) and wave w takes k
  // part w % KS of the TPW tiles (w / KS) TPW .. + TPW - 1 (3 row tiles x 1
  // column tile, n = 48 with 16 right-hand sides, give each wave all 3 tiles
  // over a quarter of k), the KS partial panels summed in LDS at the end.
  // FP64 products keep one k range per tile (tile t = wave + 4 i): their
  // wider accumulators would cost the occupancy the balance gains.
  constexpr bool SPLIT = sizeof(VT) == 4;
  constexpr int RT = NP / 16;
  constexpr int NT = RT * (RB / 16);
  constexpr int KS = !SPLIT ? 1 : ((NT % 4 == 0) ? 1 : ((NT % 2 == 0) ? 2 : 4));
  constexpr int TPW = SPLIT ? NT * KS / 4 : (NT + 3) / 4;   // tiles per wave
  constexpr int KSTEPS = NP / 4 / KS;   // 4-deep k steps per wave
  static_assert((NP / 4) % KS == 0, "k range splits evenly");
  const int kpart = wave % KS, tile0 = (wave / KS) * TPW;
  auto tile_of = [&](int it) { return SPLIT ? tile0 + it : wave + 4 * it; };
  // Staging with 16-byte loads.  Blocks: thread t takes units u = t + 256 s of
  // the tiled block (lane u % 64, unit u / 64 of that lane), each holding epl
  // entries whose (row, column) are fixed per thread and computed once.
  // Panel: thread t takes 16-byte chunks c = t + 256 s (right-hand side c / CPR,
  // chunk c % CPR of its n entries at the source site).
  constexpr int TMAX = NP / 8;
  constexpr int MU = (64 * ((TMAX * TMAX + epl - 1) / epl) + 255) / 256;
  constexpr int VPC = 16 / int(sizeof(cx<VT>));             // vector entries per chunk
  constexpr int CPRMAX = NP / VPC;
  constexpr int PU = (RB * CPRMAX + 255) / 256;
  const int cpr = n / VPC;                                   // chunks per right-hand side
  int uoff[MU];                  // unit offset in the block (in 16-byte units), -1 if none
  int ij[MU][epl];               // packed (row, column) of each entry, -1 if padding
#pragma unroll
  for (int s2 = 0; s2 < MU; ++s2) {
    const int u = threadIdx.x + 256 * s2;
    uoff[s2] = -1;
#pragma unroll
    for (int q = 0; q < epl; ++q) ij[s2][q] = -1;
    if (u < nunits) {
      const int l = u % 64, k = u / 64;
      uoff[s2] = k * 64 + l;
#pragma unroll
      for (int q = 0; q < epl; ++q) {
        const int e = k * epl + q;
        if (e < TT) {
          const int i = (l / 8) * T + e / T, j = (l % 8) * T + e % T;
          if (i < n && j < n) ij[s2][q] = (i << 8) | j;
        }
      }
    }
  }
  const cx<VT>* prow[PU];        // this thread's panel chunk sources (right-hand-side base)
  int pr_[PU], pk_[PU];          // right-hand side and first component of each chunk
#pragma unroll
  for (int s2 = 0; s2 < PU; ++s2) {
    const int c = threadIdx.x + 256 * s2;
    const int r = c / cpr, k = (c % cpr) * VPC;
    pr_[s2] = -1;
    pk_[s2] = k;
    prow[s2] = nullptr;
    if (c < RB * cpr && r < Rc) {
      pr_[s2] = r;
      prow[s2] = xin[r0 + r];
    }
  }
  // zero both planes once: padding rows / columns are never written again
  for (int t = threadIdx.x; t < 2 * (NP + RB) * LD; t += blockDim.x) Mr[t] = VT(0);
  __syncthreads();   // the zero fill must land before any staged value
  // three real products per complex one: Re C = Mr Pr - Mi Pi,
  // Im C = (Mr + Mi)(Pr + Pi) - Mr Pr - Mi Pi
  acc_t crr[TPW], cii[TPW], css[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    crr[t] = acc_t{0, 0, 0, 0};
    cii[t] = acc_t{0, 0, 0, 0};
    css[t] = acc_t{0, 0, 0, 0};
  }
  uint4 mreg[MU], preg[PU];      // the next coupling's raw 16-byte units
  int cblk = 0, csrc = 0;
  float csc = 1.0f;
  auto fetch = [&](int c, int& blk, int& src, float& sc) {
    // coupling c: 0 self, 1..4 forward hop mu = c-1, 5..8 backward hop mu = c-5
    if (c == 0) {
      src = site;
      blk = site * 5;
    } else if (c < 5) {
      src = nbr[(c - 1) * V + site];
      blk = site * 5 + c;
    } else {
      src = nbr[(4 + c - 5) * V + site];       // x - mu
      blk = src * 5 + (c - 4);                 // B[x-mu, mu]
    }
    sc = (P == P16S) ? scales[blk] : 1.0f;
    const uint4* bu = reinterpret_cast<const uint4*>(blocks) + size_t(blk) * size_t(upl) * 64;
#pragma unroll
    for (int s2 = 0; s2 < MU; ++s2)
      mreg[s2] = uoff[s2] >= 0 ? bu[uoff[s2]] : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int s2 = 0; s2 < PU; ++s2)
      preg[s2] = pr_[s2] >= 0
                     ? *reinterpret_cast<const uint4*>(prow[s2] + size_t(src) * n + pk_[s2])
                     : make_uint4(0, 0, 0, 0);
  };
  fetch(0, cblk, csrc, csc);
  for (int c = 0; c < 9; ++c) {
    const bool trans = c >= 5;
    const float sc = csc;
    // raw units -> LDS planes (the previous coupling's products are done)
#pragma unroll
    for (int s2 = 0; s2 < MU; ++s2) {
      const uint32_t w[4] = {mreg[s2].x, mreg[s2].y, mreg[s2].z, mreg[s2].w};
#pragma unroll
      for (int q = 0; q < epl; ++q) {
        const int pij = ij[s2][q];
        if (pij < 0) continue;
        const int bi = pij >> 8, bj = pij & 255;
        VT re, im;
        if (P == P64) {
          re = VT(__builtin_bit_cast(double, (uint64_t(w[1]) << 32) | w[0]));
          im = VT(__builtin_bit_cast(double, (uint64_t(w[3]) << 32) | w[2]));
        } else if (P == P32) {
          re = VT(__builtin_bit_cast(float, w[2 * q]));
          im = VT(__builtin_bit_cast(float, w[2 * q + 1]));
        } else {
          re = VT(lo_h(w[q]) * sc);
          im = VT(hi_h(w[q]) * sc);
        }
        int i = bi, j = bj;
        if (trans) {
          // backward hop Gamma5 B^H Gamma5: M[i][j] = g_i g_j conj(B[j][i])
          i = bj;
          j = bi;
          const VT sg = ((i < half) == (j < half)) ? VT(1) : VT(-1);
          re = sg * re;
          im = -sg * im;
        }
        if (c == 0 && i == j) im += VT(i < half ? tm : -tm);  // i * tm * Gamma5
        Mr[i * LD + j] = re;
        Mi[i * LD + j] = im;
      }
    }
#pragma unroll
    for (int s2 = 0; s2 < PU; ++s2) {
      if (pr_[s2] < 0) continue;
      const uint32_t w[4] = {preg[s2].x, preg[s2].y, preg[s2].z, preg[s2].w};
      const int r = pr_[s2];
#pragma unroll
      for (int q = 0; q < VPC; ++q) {
        const int k = pk_[s2] + q;
        VT re, im;
        if (sizeof(VT) == 8) {
          re = VT(__builtin_bit_cast(double, (uint64_t(w[1]) << 32) | w[0]));
          im = VT(__builtin_bit_cast(double, (uint64_t(w[3]) << 32) | w[2]));
        } else {
          re = VT(__builtin_bit_cast(float, w[2 * q]));
          im = VT(__builtin_bit_cast(float, w[2 * q + 1]));
        }
        if ((g5io & 1) && k >= half) {
          re = -re;
          im = -im;
        }
        Pr[r * LD + k] = re;
        Pi[r * LD + k] = im;
      }
    }
    __syncthreads();
    // the next coupling's loads are in flight while this one multiplies
    if (c + 1 < 9) fetch(c + 1, cblk, csrc, csc);
    // C += M P with the three products Mr Pr, Mi Pi, (Mr + Mi)(Pr + Pi)
    // (16x16x4 tiles), k outermost so the wave's tiles interleave their MFMA
    // chains
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
      const int k = 4 * (kpart * KSTEPS + ks);
#pragma unroll
      for (int it = 0; it < TPW; ++it) {
        const int t = tile_of(it);
        if (SPLIT || t < NT) {   // split tiles always exist
          const int rt = t % RT, ct = t / RT;
          const int ao = (rt * 16 + l16) * LD + lk + k, bo = (ct * 16 + l16) * LD + lk + k;
          const VT a_r = Mr[ao], a_i = Mi[ao], b_r = Pr[bo], b_i = Pi[bo];
          crr[it] = Mfma<VT>::mma(a_r, b_r, crr[it]);
          cii[it] = Mfma<VT>::mma(a_i, b_i, cii[it]);
          css[it] = Mfma<VT>::mma(a_r + a_i, b_r + b_i, css[it]);
        }
      }
    }
    __syncthreads();
  }
  // accumulators -> LDS panel planes (row r = right-hand side) -> coalesced
  // stores; the k parts add their partial panels one after another
#pragma unroll
  for (int part = 0; part < KS; ++part) {
    if (kpart == part) {
#pragma unroll
      for (int it = 0; it < TPW; ++it) {
        const int t = tile_of(it);
        if (!SPLIT && t >= NT) continue;
        const int rt = t % RT, ct = t / RT;
        const int col = ct * 16 + l16;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // accumulator value q of a lane: row 4*(lane/16)+q for the FP32
          // 16x16x4 MFMA, row lane/16 + 4*q for the FP64 one
          const int row = rt * 16 + Mfma<VT>::row(lk, q);
          const VT re = crr[it][q] - cii[it][q], im = css[it][q] - crr[it][q] - cii[it][q];
          if (part == 0) {
            Pr[col * LD + row] = re;
            Pi[col * LD + row] = im;
          } else {
            Pr[col * LD + row] += re;
            Pi[col * LD + row] += im;
          }
        }
      }
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < Rc * n; t += blockDim.x) {
    const int r = t / n, i = t % n;
    cx<VT> z = mk(Pr[r * LD + i], Pi[r * LD + i]);
    if ((g5io & 2) && i >= half) z = mk(VT(-z.re), VT(-z.im));
    yout[r0 + r][size_t(site) * n + i] = z;
  }
}

template <typename VR>
__global__ void k_gather_store(const cx<VR>* __restrict__ gbuf, cx<VR>* __restrict__ out,
                               size_t N, int n, const int* __restrict__ done) {
  if (done && *done) return;
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  out[i] = gather5(gbuf, i, n);
}

template <typename VR>
__global__ void k_gather_poly(const cx<VR>* __restrict__ gbuf, cx<VR>* __restrict__ prod,
                              cx<VR>* __restrict__ y, size_t N, int n, z64 ca, z64 cb,
                              const int* __restrict__ done) {
  if (done && *done) return;
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const cx<VR> s = gather5(gbuf, i, n);
  cx<VR> p = prod[i];
  const VR ar = VR(ca.re), ai = VR(ca.im), br = VR(cb.re), bi = VR(cb.im);
  p.re -= ar * s.re - ai * s.im;
  p.im -= ar * s.im + ai * s.re;
  prod[i] = p;
  cx<VR> yy = y[i];
  yy.re += br * p.re - bi * p.im;
  yy.im += br * p.im + bi * p.re;
  y[i] = yy;
}

template <typename VR>
__global__ void k_gather_poly_first(const cx<VR>* __restrict__ gbuf, const cx<VR>* __restrict__ v,
                                    cx<VR>* __restrict__ prod, cx<VR>* __restrict__ y, size_t N,
                                    int n, z64 c0, z64 ca, z64 cb, const int* __restrict__ done) {
  if (done && *done) return;
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const cx<VR> s = gather5(gbuf, i, n);
  const cx<VR> vv = v[i];
  cx<VR> p = vv;
  const VR ar = VR(ca.re), ai = VR(ca.im), br = VR(cb.re), bi = VR(cb.im);
  const VR zr = VR(c0.re), zi = VR(c0.im);
  p.re -= ar * s.re - ai * s.im;
  p.im -= ar * s.im + ai * s.re;
  prod[i] = p;
  cx<VR> yy;
  yy.re = zr * vv.re - zi * vv.im + (br * p.re - bi * p.im);
  yy.im = zr * vv.im + zi * vv.re + (br * p.im + bi * p.re);
  y[i] = yy;
}

template <typename VR>
__global__ void k_gather_resid(const cx<VR>* __restrict__ gbuf, const cx<VR>* __restrict__ b,
                               cx<VR>* __restrict__ out, size_t N, int n, Reducer red,
                               double* result) {
  double acc[1] = {0.0};
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N;
       i += size_t(gridDim.x) * blockDim.x) {
    const cx<VR> s = gather5(gbuf, i, n);
    const cx<VR> bb = b[i];
    const cx<VR> r = mk(VR(bb.re - s.re), VR(bb.im - s.im));
    out[i] = r;
    acc[0] += double(r.re) * double(r.re) + double(r.im) * double(r.im);
  }
  block_partials<1>(acc, red.partials);
}

// ------------------------------------------------------------------ BLAS
// Dot products and updates against a basis of Q vectors.  Each thread takes
// E elements per pass and issues the loads of all G basis vectors of a chunk
// before any arithmetic, so 2*G*E independent loads are in flight per lane
// (a load-use-load chain would leave one).  Accumulation is in FP64.
constexpr int kDotE = 2;     // elements per thread per pass
constexpr int kAxpyG = 16;   // basis vectors per chunk of the update kernel

template <typename VR>
__device__ inline const cx<VR>* basis_ptr(const cx<VR>* b0, int q0, const cx<VR>* b1, size_t N,
                                          int q) {
  return q < q0 ? b0 + size_t(q) * N : b1 + size_t(q - q0) * N;
}

// Wave sums of V per-lane values (V a power of two, at most 64) by halving
// exchanges: at each step a lane keeps one half of its values, sends the other
// half to its partner and adds what it receives, so after log2(V) steps lane l
// holds one value, index l / (64 / V), summed over V lanes; the remaining
// steps are a plain butterfly.  V - 1 + 6 - log2(V) exchanges instead of 6 V,
// in a fixed order.
template <int V, int S = 0>
__device__ inline void halving_steps(double (&acc)[V], int lane) {
  if constexpr ((V >> S) > 1) {
    constexpr int half = V >> (S + 1);
    constexpr int o = 32 >> S;
    const bool upper = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const double send = upper ? acc[i] : acc[i + half];
      const double keep = upper ? acc[i + half] : acc[i];
      acc[i] = keep + shfl_xor(send, o);
    }
    halving_steps<V, S + 1>(acc, lane);
  }
}

template <int V>
__device__ inline double wave_sum_many(double (&acc)[V], int lane) {
  halving_steps<V>(acc, lane);
  double v = acc[0];
#pragma unroll
  for (int o = 32 / V; o > 0; o >>= 1) v += shfl_xor(v, o);
  return v;
}

// result value v = by * 2G + t of the group; t = 2*(q - g0) + re/im.  Block
// bx of gx along the vector, by along the values (blockIdx of a plain launch).
template <typename VR, int G>
__device__ __forceinline__ void multidot_body(const cx<VR>* __restrict__ b0, int q0,
                                              const cx<VR>* __restrict__ b1, int q1, size_t N,
                                              const cx<VR>* __restrict__ w,
                                              double* __restrict__ partials, int bx, int gx,
                                              int by) {
  const int Qb = q0 + q1;
  const int g0 = by * G;
  const cx<VR>* ptr[G];
#pragma unroll
  for (int t = 0; t < G; ++t) {
    const int q = g0 + t;
    ptr[t] = q < Qb ? basis_ptr(b0, q0, b1, N, q) : w;  // past the basis: w itself (the norm)
  }
  double acc[2 * G];
#pragma unroll
  for (int t = 0; t < 2 * G; ++t) acc[t] = 0.0;
  const size_t chunk = size_t(blockDim.x) * kDotE;
  const size_t stride = size_t(gx) * chunk;
  for (size_t base = size_t(bx) * chunk + threadIdx.x; base < N; base += stride) {
    size_t idx[kDotE];
    double wr[kDotE], wi[kDotE];
#pragma unroll
    for (int e = 0; e < kDotE; ++e) {
      const size_t i = base + size_t(e) * blockDim.x;
      idx[e] = i < N ? i : N - 1;
    }
    cx<VR> v[G][kDotE], wv[kDotE];
#pragma unroll
    for (int e = 0; e < kDotE; ++e) wv[e] = w[idx[e]];
#pragma unroll
    for (int t = 0; t < G; ++t)
#pragma unroll
      for (int e = 0; e < kDotE; ++e) v[t][e] = ptr[t][idx[e]];
    __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the arithmetic
#pragma unroll
    for (int e = 0; e < kDotE; ++e) {
      const bool ok = base + size_t(e) * blockDim.x < N;
      wr[e] = ok ? double(wv[e].re) : 0.0;
      wi[e] = ok ? double(wv[e].im) : 0.0;
    }
#pragma unroll
    for (int t = 0; t < G; ++t)
#pragma unroll
      for (int e = 0; e < kDotE; ++e) {
        const double vr = v[t][e].re, vi = v[t][e].im;
        acc[2 * t] = fma(vr, wr[e], fma(vi, wi[e], acc[2 * t]));        // Re conj(v) w
        acc[2 * t + 1] = fma(vr, wi[e], fma(-vi, wr[e], acc[2 * t + 1]));  // Im conj(v) w
      }
  }
  __shared__ double sh[4][2 * G];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double s = wave_sum_many<2 * G>(acc, lane);
  constexpr int kSpan = 64 / (2 * G);   // lanes holding the same value
  if (lane % kSpan == 0) sh[wave][lane / kSpan] = s;
  __syncthreads();
  if (threadIdx.x < 2 * G) {
    double s = 0.0;
    for (int wv2 = 0; wv2 < int(blockDim.x >> 6); ++wv2) s += sh[wv2][threadIdx.x];
    partials[(size_t(by) * 2 * G + threadIdx.x) * gx + bx] = s;
  }
}

template <typename VR, int G>
__global__ __launch_bounds__(256) void k_multidot(const cx<VR>* __restrict__ b0, int q0,
                                                  const cx<VR>* __restrict__ b1, int q1,
                                                  size_t N, const cx<VR>* __restrict__ w,
                                                  int want_norm, Reducer red,
                                                  const int* __restrict__ done) {
  if (done && *done) return;
  (void)want_norm;
  multidot_body<VR, G>(b0, q0, b1, q1, N, w, red.partials, blockIdx.x, gridDim.x, blockIdx.y);
}

// The update kernels split the basis between the kSplitWaves waves of a
// workgroup: each wave takes every kSplitWaves-th chunk of kAxpyG vectors (the
// loads of a chunk issued before their arithmetic) for the same 64 kDotE
// elements, so a wave waits on a quarter of the chunks; the partial sums are
// then combined through LDS in a fixed order.  Elements of a pass:
// base + e 64 + lane.
constexpr int kSplitWaves = 4;   // waves per workgroup (256 threads)

template <typename VR>
__device__ inline void split_sums(const cx<VR>* __restrict__ b0, int q0,
                                  const cx<VR>* __restrict__ b1, size_t N, int Q,
                                  const double* __restrict__ coef, size_t base, int lane,
                                  int wave, size_t (&idx)[kDotE], double (&sr)[kDotE],
                                  double (&si)[kDotE]) {
#pragma unroll
  for (int e = 0; e < kDotE; ++e) {
    const size_t i = base + size_t(e) * 64 + lane;
    idx[e] = i < N ? i : N - 1;
    sr[e] = si[e] = 0.0;
  }
  for (int qc = wave * kAxpyG; qc < Q; qc += kSplitWaves * kAxpyG) {
    cx<VR> v[kAxpyG][kDotE];
#pragma unroll
    for (int t = 0; t < kAxpyG; ++t) {
      const int q = min(qc + t, Q - 1);
      const cx<VR>* p = basis_ptr(b0, q0, b1, N, q);
#pragma unroll
      for (int e = 0; e < kDotE; ++e) v[t][e] = p[idx[e]];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < kAxpyG; ++t) {
      const int q = qc + t;
      const double cr = q < Q ? coef[2 * q] : 0.0, ci = q < Q ? coef[2 * q + 1] : 0.0;
#pragma unroll
      for (int e = 0; e < kDotE; ++e) {
        const double vr = v[t][e].re, vi = v[t][e].im;
        sr[e] = fma(cr, vr, fma(-ci, vi, sr[e]));
        si[e] = fma(cr, vi, fma(ci, vr, si[e]));
      }
    }
  }
}

// out = (w - sum_q coef_q basis_q) (times *scale when scale is given; then the
// launch belongs to Arnoldi step j and runs only if that step's bookkeeping
// ran, *jdone == j + 1, instead of checking the stop flag).  out may be w.
// Block bx of gx (blockIdx.x / gridDim.x of a plain launch); sc scales the result.
template <typename VR>
__device__ __forceinline__ void multiaxpy_split_body(const cx<VR>* w, cx<VR>* out,
                                                     const cx<VR>* __restrict__ b0, int q0,
                                                     const cx<VR>* __restrict__ b1, int q1,
                                                     size_t N, const double* __restrict__ coef,
                                                     int want_norm, double* partials, double sc,
                                                     int bx, int gx) {
  const int Q = q0 + q1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ double part[kSplitWaves][kDotE][2][64];
  double nacc[1] = {0.0};
  const size_t span = size_t(64) * kDotE;
  for (size_t base = size_t(bx) * span; base < N; base += size_t(gx) * span) {
    size_t idx[kDotE];
    double sr[kDotE], si[kDotE];
    split_sums<VR>(b0, q0, b1, N, Q, coef, base, lane, wave, idx, sr, si);
#pragma unroll
    for (int e = 0; e < kDotE; ++e) {
      part[wave][e][0][lane] = sr[e];
      part[wave][e][1][lane] = si[e];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int e = 0; e < kDotE; ++e) {
        if (base + size_t(e) * 64 + lane < N) {
          const cx<VR> wv = w[idx[e]];
          double r = wv.re, im = wv.im;
#pragma unroll
          for (int v2 = 0; v2 < kSplitWaves; ++v2) {
            r -= part[v2][e][0][lane];
            im -= part[v2][e][1][lane];
          }
          const cx<VR> o = mk(VR(r * sc), VR(im * sc));
          out[idx[e]] = o;
          nacc[0] += double(o.re) * double(o.re) + double(o.im) * double(o.im);
        }
      }
    }
    __syncthreads();
  }
  if (want_norm) block_partials_at<1>(nacc, partials, bx, gx);
}

template <typename VR>
__global__ __launch_bounds__(256) void k_multiaxpy(const cx<VR>* w, cx<VR>* out,
                                                   const cx<VR>* __restrict__ b0, int q0,
                                                   const cx<VR>* __restrict__ b1, int q1,
                                                   size_t N, const double* __restrict__ coef,
                                                   int want_norm, Reducer red,
                                                   const int* __restrict__ done,
                                                   const double* __restrict__ scale,
                                                   const int* __restrict__ jdone, int j) {
  if (scale) {
    if (*jdone != j + 1) return;
  } else if (done && *done) {
    return;
  }
  multiaxpy_split_body<VR>(w, out, b0, q0, b1, q1, N, coef, want_norm, red.partials,
                           scale ? *scale : 1.0, blockIdx.x, gridDim.x);
}

// Bases of at most one chunk (kAxpyG vectors): nothing to split between the
// waves, so each thread takes its own kDotE elements through the whole basis.
template <typename VR>
__device__ __forceinline__ void multiaxpy_flat_body(const cx<VR>* w, cx<VR>* out,
                                                    const cx<VR>* __restrict__ b0, int q0,
                                                    const cx<VR>* __restrict__ b1, int q1,
                                                    size_t N, const double* __restrict__ coef,
                                                    int want_norm, double* partials, double sc,
                                                    int bx, int gx) {
  const int Q = q0 + q1;
  double nacc[1] = {0.0};
  const size_t chunk = size_t(blockDim.x) * kDotE;
  const size_t stride = size_t(gx) * chunk;
  for (size_t base = size_t(bx) * chunk + threadIdx.x; base < N; base += stride) {
    size_t idx[kDotE];
    double sr[kDotE], si[kDotE];
#pragma unroll
    for (int e = 0; e < kDotE; ++e) {
      const size_t i = base + size_t(e) * blockDim.x;
      idx[e] = i < N ? i : N - 1;
      const cx<VR> wv = w[idx[e]];
      sr[e] = wv.re;
      si[e] = wv.im;
    }
    for (int qc = 0; qc < Q; qc += kAxpyG) {
      cx<VR> v[kAxpyG][kDotE];
#pragma unroll
      for (int t = 0; t < kAxpyG; ++t) {
        const int q = min(qc + t, Q - 1);
        const cx<VR>* p = basis_ptr(b0, q0, b1, N, q);
#pragma unroll
        for (int e = 0; e < kDotE; ++e) v[t][e] = p[idx[e]];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < kAxpyG; ++t) {
        const int q = qc + t;
        const double cr = q < Q ? coef[2 * q] : 0.0, ci = q < Q ? coef[2 * q + 1] : 0.0;
#pragma unroll
        for (int e = 0; e < kDotE; ++e) {
          const double vr = v[t][e].re, vi = v[t][e].im;
          sr[e] = fma(-cr, vr, fma(ci, vi, sr[e]));
          si[e] = fma(-cr, vi, fma(-ci, vr, si[e]));
        }
      }
    }
#pragma unroll
    for (int e = 0; e < kDotE; ++e) {
      if (base + size_t(e) * blockDim.x < N) {
        const cx<VR> o = mk(VR(sr[e] * sc), VR(si[e] * sc));
        out[idx[e]] = o;
        nacc[0] += double(o.re) * double(o.re) + double(o.im) * double(o.im);
      }
    }
  }
  if (want_norm) block_partials_at<1>(nacc, partials, bx, gx);
}

template <typename VR>
__global__ __launch_bounds__(256) void k_multiaxpy_flat(const cx<VR>* w, cx<VR>* out,
                                                   const cx<VR>* __restrict__ b0, int q0,
                                                   const cx<VR>* __restrict__ b1, int q1,
                                                   size_t N, const double* __restrict__ coef,
                                                   int want_norm, Reducer red,
                                                   const int* __restrict__ done,
                                                   const double* __restrict__ scale,
                                                   const int* __restrict__ jdone, int j) {
  if (scale) {
    if (*jdone != j + 1) return;
  } else if (done && *done) {
    return;
  }
  multiaxpy_flat_body<VR>(w, out, b0, q0, b1, q1, N, coef, want_norm, red.partials,
                          scale ? *scale : 1.0, blockIdx.x, gridDim.x);
}

constexpr int kCombR = 16;  // outputs per pass of the combine kernel
constexpr int kCombMfmaMin = 16;   // from this many outputs on: the MFMA block update

template <typename VR>
__global__ __launch_bounds__(256) void k_combine(const cx<VR>* __restrict__ b0, int q0,
                                                 const cx<VR>* __restrict__ b1, int q1,
                                                 size_t N, const double* __restrict__ coef,
                                                 int R, cx<VR>* __restrict__ out, int accumulate) {
  const int Q = q0 + q1;
  const int r0 = blockIdx.y * kCombR;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
    double ar[kCombR], ai[kCombR];
#pragma unroll
    for (int t = 0; t < kCombR; ++t) ar[t] = ai[t] = 0.0;
    for (int q = 0; q < Q; ++q) {
      const cx<VR> v = (q < q0) ? b0[size_t(q) * N + i] : b1[size_t(q - q0) * N + i];
      const double vr = v.re, vi = v.im;
#pragma unroll
      for (int t = 0; t < kCombR; ++t) {
        const int r = r0 + t;
        if (r < R) {
          const double cr = coef[2 * (size_t(r) * Q + q)], ci = coef[2 * (size_t(r) * Q + q) + 1];
          ar[t] += cr * vr - ci * vi;
          ai[t] += cr * vi + ci * vr;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < kCombR; ++t) {
      const int r = r0 + t;
      if (r < R) {
        cx<VR>* o = out + size_t(r) * N + i;
        if (accumulate) {
          const cx<VR> old = *o;
          *o = mk(VR(double(old.re) + ar[t]), VR(double(old.im) + ai[t]));
        } else {
          *o = mk(VR(ar[t]), VR(ai[t]));
        }
      }
    }
  }
}

// One output (R = 1): out (+)= sum_q coef_q basis_q with the basis split
// between the waves as in the update kernel (the general kernel above walks
// the basis one load at a time).
template <typename VR>
__global__ __launch_bounds__(256) void k_combine1(const cx<VR>* __restrict__ b0, int q0,
                                                  const cx<VR>* __restrict__ b1, int q1,
                                                  size_t N, const double* __restrict__ coef,
                                                  cx<VR>* __restrict__ out, int accumulate) {
  const int Q = q0 + q1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ double part[kSplitWaves][kDotE][2][64];
  const size_t span = size_t(64) * kDotE;
  for (size_t base = size_t(blockIdx.x) * span; base < N; base += size_t(gridDim.x) * span) {
    size_t idx[kDotE];
    double sr[kDotE], si[kDotE];
    split_sums<VR>(b0, q0, b1, N, Q, coef, base, lane, wave, idx, sr, si);
#pragma unroll
    for (int e = 0; e < kDotE; ++e) {
      part[wave][e][0][lane] = sr[e];
      part[wave][e][1][lane] = si[e];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int e = 0; e < kDotE; ++e) {
        if (base + size_t(e) * 64 + lane < N) {
          double r = 0.0, im = 0.0;
          if (accumulate) {
            const cx<VR> old = out[idx[e]];
            r = old.re;
            im = old.im;
          }
#pragma unroll
          for (int v2 = 0; v2 < kSplitWaves; ++v2) {
            r += part[v2][e][0][lane];
            im += part[v2][e][1][lane];
          }
          out[idx[e]] = mk(VR(r), VR(im));
        }
      }
    }
    __syncthreads();
  }
}

template <typename VR>
__global__ void k_scale(const cx<VR>* __restrict__ in, cx<VR>* __restrict__ out, size_t N,
                        const double* __restrict__ sdev, double s, const int* __restrict__ done) {
  if (done && *done) return;
  const double sc = sdev ? *sdev : s;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
    const cx<VR> z = in[i];
    out[i] = mk(VR(z.re * sc), VR(z.im * sc));
  }
}

template <typename VR>
__global__ void k_cscale(const cx<VR>* in, cx<VR>* out, size_t N, z64 c,
                         const int* __restrict__ done) {
  if (done && *done) return;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
    const cx<VR> z = in[i];
    out[i] = mk(VR(c.re * double(z.re) - c.im * double(z.im)),
                VR(c.re * double(z.im) + c.im * double(z.re)));
  }
}

template <typename VR>
__global__ void k_scale_step(cx<VR>* v, size_t N, const double* __restrict__ inv_h,
                             const int* __restrict__ jdone, int j) {
  if (*jdone != j + 1) return;
  const double sc = *inv_h;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
    const cx<VR> z = v[i];
    v[i] = mk(VR(double(z.re) * sc), VR(double(z.im) * sc));
  }
}

template <typename VR>
__global__ void k_zero(cx<VR>* x, size_t N) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride)
    x[i] = mk(VR(0), VR(0));
}

template <typename VR>
__global__ void k_axpy(z64 a, const cx<VR>* __restrict__ x, cx<VR>* __restrict__ y, size_t N) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
    const cx<VR> xv = x[i];
    cx<VR> yv = y[i];
    yv.re = VR(double(yv.re) + a.re * double(xv.re) - a.im * double(xv.im));
    yv.im = VR(double(yv.im) + a.re * double(xv.im) + a.im * double(xv.re));
    y[i] = yv;
  }
}

template <typename VR>
__global__ __launch_bounds__(256) void k_norm2(const cx<VR>* __restrict__ x, size_t N,
                                               Reducer red) {
  // column blockIdx.y of [q][N]; partial of block (bx, by) at by * gx + bx
  const cx<VR>* col = x + size_t(blockIdx.y) * N;
  double acc[1] = {0.0};
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
    const cx<VR> z = col[i];
    acc[0] += double(z.re) * double(z.re) + double(z.im) * double(z.im);
  }
  block_partials<1>(acc, red.partials);
}

template <typename VR>
__global__ void k_gamma5(const cx<VR>* in, cx<VR>* out, size_t N, int n) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
    const int c = int(i % n);
    const cx<VR> z = in[i];
    out[i] = (c < (n >> 1)) ? z : mk(VR(-z.re), VR(-z.im));
  }
}

__global__ void k_cvt64to32(const z64* __restrict__ in, z32* __restrict__ out, size_t N, int n,
                            int g5) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
    const z64 z = in[i];
    const double s = (g5 && int(i % n) >= (n >> 1)) ? -1.0 : 1.0;
    out[i] = mk(float(s * z.re), float(s * z.im));
  }
}

__global__ void k_cvt32to64(const z32* __restrict__ in, z64* __restrict__ out, size_t N, int n,
                            int g5) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
    const z32 z = in[i];
    const double s = (g5 && int(i % n) >= (n >> 1)) ? -1.0 : 1.0;
    out[i] = mk(s * double(z.re), s * double(z.im));
  }
}

// Philox4x32-10 (Salmon et al., SC'11) and Box-Muller, as in the input generator.
__device__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    if (r < 9) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
  }
}

__global__ void k_gaussian(z64* out, size_t N, uint64_t seed, uint32_t stream_id) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
    uint32_t c[4] = {uint32_t(i), uint32_t(uint64_t(i) >> 32), stream_id, 0u};
    philox(c, uint32_t(seed), uint32_t(seed >> 32));
    const double two53 = 9007199254740992.0;
    const double u1 = (double(uint64_t(c[0] >> 5) * 67108864ull + (c[1] >> 6)) + 0.5) / two53;
    const double u2 = (double(uint64_t(c[2] >> 5) * 67108864ull + (c[3] >> 6)) + 0.5) / two53;
    const double r = sqrt(-2.0 * log(u1)) * 0.70710678118654752440;
    double sn, cs;
    sincos(6.283185307179586477 * u2, &sn, &cs);
    out[i] = mk(r * cs, r * sn);
  }
}

// ------------------------------------------------------------------ block products
// The tall-skinny complex products of block GMRES (one Krylov space shared by
// many right-hand sides) and of the recycle-space construction and refresh:
// Gram matrices A^H B of two blocks of vectors and block updates
// C = beta C + alpha A S with a small coefficient matrix S.  Both stage
// 64-wide panels in LDS as real and imaginary planes with a padded stride and
// multiply on 16x16x4 MFMA tiles with three real products per complex one;
// wave w owns output row tile w and all four column tiles of a 64 x 64 output
// tile.  VS is the storage type of the vectors, VC the type the products are
// formed and accumulated in (FP32 vectors may be combined in FP64).
constexpr int kBpT = 64;          // output tile edge
constexpr int kBpK = 32;          // inner-dimension rows staged per LDS round
constexpr int kBpLD = kBpK + 1;   // padded plane stride
constexpr int kGramMaxParts = 256;

// part[c] = A_c^H B_c for row chunk c = blockIdx.x (rows [c L, min(c L + L, N))),
// output tile (blockIdx.y % tq, blockIdx.y / tq) of the qa x rb result, tq =
// ceil(qa / 64); part layout [chunk][j qa + i].  A: qa vectors, B: rb vectors,
// each N long with stride N.
template <typename VS, typename VC>
__global__ __launch_bounds__(256) void k_block_gram(const cx<VS>* __restrict__ A, int qa,
                                                     const cx<VS>* __restrict__ B, int rb,
                                                     size_t N, size_t L,
                                                     cx<VC>* __restrict__ part) {
  using acc_t = typename Mfma<VC>::acc_t;
  __shared__ VC Ar[kBpT * kBpLD], Ai[kBpT * kBpLD], Br[kBpT * kBpLD], Bi[kBpT * kBpLD];
  const int tq = (qa + kBpT - 1) / kBpT;
  const int i0 = int(blockIdx.y % unsigned(tq)) * kBpT, j0 = int(blockIdx.y / unsigned(tq)) * kBpT;
  const int ni = min(kBpT, qa - i0), nj = min(kBpT, rb - j0);
  const size_t r0 = size_t(blockIdx.x) * L, r1 = min(N, r0 + L);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lk = lane >> 4;
  const int nct = (nj + 15) / 16;    // column tiles with at least one column
  acc_t prr[4], pii[4], pss[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    prr[t] = acc_t{0, 0, 0, 0};
    pii[t] = acc_t{0, 0, 0, 0};
    pss[t] = acc_t{0, 0, 0, 0};
  }
  // panels: column c of the tile, rows k0 .. k0 + 31 (consecutive threads
  // read consecutive rows of one vector); thread t holds elements
  // u = t + 256 e, e < 8, of each panel in registers: those of the next round
  // are loaded while the current one multiplies
  constexpr int EPT = kBpT * kBpK / 256;
  cx<VS> ra[EPT], rb_[EPT];
  auto fetch = [&](size_t k0) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int u = int(threadIdx.x) + 256 * e;
      const int c = u / kBpK, r = u % kBpK;
      const size_t row = k0 + size_t(r);
      ra[e] = mk(VS(0), VS(0));
      rb_[e] = mk(VS(0), VS(0));
      if (row < r1) {
        if (c < ni) ra[e] = A[size_t(i0 + c) * N + row];
        if (c < nj) rb_[e] = B[size_t(j0 + c) * N + row];
      }
    }
  };
  if (r0 < r1) fetch(r0);
  for (size_t k0 = r0; k0 < r1; k0 += kBpK) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {   // A is conjugated here
      const int u = int(threadIdx.x) + 256 * e;
      const int c = u / kBpK, r = u % kBpK;
      Ar[c * kBpLD + r] = VC(ra[e].re);
      Ai[c * kBpLD + r] = -VC(ra[e].im);
      Br[c * kBpLD + r] = VC(rb_[e].re);
      Bi[c * kBpLD + r] = VC(rb_[e].im);
    }
    __syncthreads();
    if (k0 + kBpK < r1) fetch(k0 + kBpK);
    if (wave * 16 < ni) {
#pragma unroll 2
      for (int kk = 0; kk < kBpK; kk += 4) {
        const int ao = (wave * 16 + l16) * kBpLD + kk + lk;
        const VC a_r = Ar[ao], a_i = Ai[ao];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          if (ct < nct) {
            const int bo = (ct * 16 + l16) * kBpLD + kk + lk;
            const VC b_r = Br[bo], b_i = Bi[bo];
            prr[ct] = Mfma<VC>::mma(a_r, b_r, prr[ct]);
            pii[ct] = Mfma<VC>::mma(a_i, b_i, pii[ct]);
            pss[ct] = Mfma<VC>::mma(a_r + a_i, b_r + b_i, pss[ct]);
          }
        }
      }
    }
    __syncthreads();
  }
  const size_t qr = size_t(qa) * size_t(rb);
  cx<VC>* out = part + size_t(blockIdx.x) * qr;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int j = ct * 16 + l16;
    if (ct >= nct || j >= nj) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = wave * 16 + Mfma<VC>::row(lk, q);
      if (i < ni)
        out[size_t(j0 + j) * qa + (i0 + i)] =
            mk(VC(prr[ct][q] - pii[ct][q]), VC(pss[ct][q] - prr[ct][q] - pii[ct][q]));
    }
  }
}

// out[e] = sum over the P chunks of part[c][e] (FP64, chunk order fixed)
template <typename VC>
__global__ void k_block_gram_sum(const cx<VC>* __restrict__ part, int P, size_t qr,
                                 z64* __restrict__ out) {
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= qr) return;
  double re = 0.0, im = 0.0;
  for (int c = 0; c < P; ++c) {
    const cx<VC> z = part[size_t(c) * qr + e];
    re += double(z.re);
    im += double(z.im);
  }
  out[e] = mk(re, im);
}

// C[:, j] = beta C[:, j] + alpha sum_i A_i S[i + j ldS] for j < r, over the
// k = q0 + q1 vectors A_i = b0 + i N (i < q0), b1 + (i - q0) N (after); C has r
// vectors (each N long, stride N); S is column-major in the product type.
// Workgroup t: column tile t % nct (nct = ceil(r / 64)), rows 64 (t / nct)
// .. + 63, so the workgroups that share a row panel of the A_i run together.
// C must not overlap the A_i.
template <typename VS, typename VC>
__global__ __launch_bounds__(256) void k_block_update(const cx<VS>* __restrict__ b0, int q0,
                                                       const cx<VS>* __restrict__ b1, int q1,
                                                       const cx<VC>* __restrict__ S, int ldS,
                                                       cx<VS>* C, int r, size_t N, z64 alpha,
                                                       z64 beta) {
  using acc_t = typename Mfma<VC>::acc_t;
  // four planes while multiplying ([row][kk] of A, [col][kk] of S); the
  // 64 x 64 output planes ([col][row], stride 65) reuse them afterwards
  constexpr int PL = kBpT * kBpLD;
  __shared__ VC sm[4 * PL];
  static_assert(2 * kBpT * (kBpT + 1) <= 4 * PL, "output planes fit");
  VC* Ar = sm;
  VC* Ai = sm + PL;
  VC* Sr = sm + 2 * PL;
  VC* Si = sm + 3 * PL;
  const int k = q0 + q1;
  const int nctile = (r + kBpT - 1) / kBpT;
  const size_t row0 = size_t(blockIdx.x / unsigned(nctile)) * kBpT;
  const int j0 = int(blockIdx.x % unsigned(nctile)) * kBpT;
  const int nj = min(kBpT, r - j0);
  const int nrow = int(min(size_t(kBpT), N - row0));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, lk = lane >> 4;
  const int nct = (nj + 15) / 16;
  acc_t prr[4], pii[4], pss[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    prr[t] = acc_t{0, 0, 0, 0};
    pii[t] = acc_t{0, 0, 0, 0};
    pss[t] = acc_t{0, 0, 0, 0};
  }
  // A panel: vector k0 + kk, rows row0 .. row0 + 63 (consecutive threads,
  // consecutive rows); S panel: column j, rows k0 .. k0 + 31.  Thread t holds
  // elements u = t + 256 e of each in registers; the next round's are loaded
  // while the current one multiplies.
  constexpr int EPT = kBpT * kBpK / 256;
  cx<VS> ra[EPT];
  cx<VC> rs[EPT];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int u = int(threadIdx.x) + 256 * e;
      const int kk = u / kBpT, rr = u % kBpT;
      const int i = k0 + kk;
      ra[e] = mk(VS(0), VS(0));
      if (i < k && rr < nrow)
        ra[e] = (i < q0 ? b0 + size_t(i) * N : b1 + size_t(i - q0) * N)[row0 + rr];
      const int j = u / kBpK, kq = u % kBpK;
      rs[e] = mk(VC(0), VC(0));
      if (j < nj && k0 + kq < k) rs[e] = S[size_t(j0 + j) * ldS + k0 + kq];
    }
  };
  if (k > 0) fetch(0);
  for (int k0 = 0; k0 < k; k0 += kBpK) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int u = int(threadIdx.x) + 256 * e;
      const int kk = u / kBpT, rr = u % kBpT;
      Ar[rr * kBpLD + kk] = VC(ra[e].re);
      Ai[rr * kBpLD + kk] = VC(ra[e].im);
      const int j = u / kBpK, kq = u % kBpK;
      Sr[j * kBpLD + kq] = rs[e].re;
      Si[j * kBpLD + kq] = rs[e].im;
    }
    __syncthreads();
    if (k0 + kBpK < k) fetch(k0 + kBpK);
#pragma unroll 2
    for (int kk = 0; kk < kBpK; kk += 4) {
      const int ao = (wave * 16 + l16) * kBpLD + kk + lk;
      const VC a_r = Ar[ao], a_i = Ai[ao];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        if (ct < nct) {
          const int bo = (ct * 16 + l16) * kBpLD + kk + lk;
          const VC b_r = Sr[bo], b_i = Si[bo];
          prr[ct] = Mfma<VC>::mma(a_r, b_r, prr[ct]);
          pii[ct] = Mfma<VC>::mma(a_i, b_i, pii[ct]);
          pss[ct] = Mfma<VC>::mma(a_r + a_i, b_r + b_i, pss[ct]);
        }
      }
    }
    __syncthreads();
  }
  // accumulators -> output planes [col][row] -> coalesced column stores
  constexpr int OL = kBpT + 1;
  VC* Or = sm;
  VC* Oi = sm + kBpT * OL;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    if (ct >= nct) continue;
    const int col = ct * 16 + l16;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = wave * 16 + Mfma<VC>::row(lk, q);
      Or[col * OL + row] = prr[ct][q] - pii[ct][q];
      Oi[col * OL + row] = pss[ct][q] - prr[ct][q] - pii[ct][q];
    }
  }
  __syncthreads();
  const bool keep = beta.re != 0.0 || beta.im != 0.0;
  for (int u = threadIdx.x; u < kBpT * kBpT; u += 256) {
    const int col = u / kBpT, rr = u % kBpT;
    if (col >= nj || rr >= nrow) continue;
    const double pr = double(Or[col * OL + rr]), pi = double(Oi[col * OL + rr]);
    double yr = alpha.re * pr - alpha.im * pi, yi = alpha.re * pi + alpha.im * pr;
    cx<VS>* c = C + size_t(j0 + col) * N + row0 + rr;
    if (keep) {
      const cx<VS> z = *c;
      yr += beta.re * double(z.re) - beta.im * double(z.im);
      yi += beta.re * double(z.im) + beta.im * double(z.re);
    }
    *c = mk(VS(yr), VS(yi));
  }
}

// ------------------------------------------------------------------ odd-even split
template <typename VR>
__global__ void k_oddeven_split(int n, int H, const int* __restrict__ esite,
                                const int* __restrict__ osite, cx<VR>* full, cx<VR>* ve,
                                cx<VR>* vo, int dir) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= size_t(H) * n) return;
  const int r = int(i / n), c = int(i % n);
  const size_t fe = size_t(esite[r]) * n + c, fo = size_t(osite[r]) * n + c;
  if (dir == 0) {
    if (ve) ve[i] = full[fe];
    if (vo) vo[i] = full[fo];
  } else {
    full[fe] = ve ? ve[i] : mk(VR(0), VR(0));
    full[fo] = vo ? vo[i] : mk(VR(0), VR(0));
  }
}

// ------------------------------------------------------------------ Arnoldi
__global__ void k_arnoldi_init(ArnoldiDev a, double beta, const double* __restrict__ beta_dev) {
  if (threadIdx.x == 0) {
    if (beta_dev) beta = *beta_dev;
    *a.done = 0;
    *a.jdone = 0;
    *a.brk_flag = 0;
    *a.est = beta;
    double* g = a.giv;
    for (int i = 0; i < 2 * (a.ldh + 1); ++i) g[i] = 0.0;
    g[0] = beta;
  }
}

// Givens storage in a.giv: g[0..ldh] (complex), then c[0..ldh) (real, stored
// in the even slots of complex entries), then s[0..ldh) (complex).
constexpr int kFinishLds = 512;  // Hessenberg column length staged in LDS

// One workgroup of 64 lanes: the lanes combine the two Gram-Schmidt passes'
// coefficients in parallel and stage the new column and the stored rotations in
// LDS; lane 0 then runs the (inherently serial) Givens update from LDS.
// Single-sync process (c2 null, Sec. 3.5): the coefficients come from one pass
// and h_{j+1,j}^2 = ||A v_j||^2 - sum |coefficients|^2 (nrm2 unused); a value
// at or below (brk ||A v_j||)^2 is a breakdown.
__device__ __forceinline__ void arnoldi_finish_body(const ArnoldiDev& a, int steps, int kC, int j,
                                                    const double* c1, const double* c2,
                                                    const double* nrm2, double target,
                                                    double brk) {
  if (*a.done) return;
  __shared__ double hcol[2 * (kFinishLds + 2)], csl[kFinishLds], snl[2 * kFinishLds];
  const bool staged = j + 2 <= kFinishLds;
  double* Hc = a.H + 2 * size_t(j) * a.ldh;
  double* g = a.giv;
  double* cs = a.giv + 2 * (a.ldh + 1);
  double* sn = cs + 2 * a.ldh;
  const bool ss = (c2 == nullptr);
  double sq = 0.0;   // single-sync: this lane's share of sum |coefficients|^2
  for (int i = threadIdx.x; i < kC; i += 64) {
    const double br = c1[2 * i] + (ss ? 0.0 : c2[2 * i]);
    const double bi = c1[2 * i + 1] + (ss ? 0.0 : c2[2 * i + 1]);
    a.Bk[2 * (size_t(j) * a.ldb + i)] = br;
    a.Bk[2 * (size_t(j) * a.ldb + i) + 1] = bi;
    sq += br * br + bi * bi;
  }
  for (int i = threadIdx.x; i <= j; i += 64) {
    const double hr = c1[2 * (kC + i)] + (ss ? 0.0 : c2[2 * (kC + i)]);
    const double hi = c1[2 * (kC + i) + 1] + (ss ? 0.0 : c2[2 * (kC + i) + 1]);
    sq += hr * hr + hi * hi;
    Hc[2 * i] = hr;
    Hc[2 * i + 1] = hi;
    if (staged) {
      hcol[2 * i] = hr;
      hcol[2 * i + 1] = hi;
    }
  }
  if (staged)
    for (int i = threadIdx.x; i < j; i += 64) {
      csl[i] = cs[2 * i];
      snl[2 * i] = sn[2 * i];
      snl[2 * i + 1] = sn[2 * i + 1];
    }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sq += shfl_xor(sq, o);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double* hsrc = staged ? hcol : Hc;
  const double wn2 = c1[2 * (kC + j + 1)];   // ||A v_j||^2 before orthogonalisation
  const double wn0 = sqrt(fmax(wn2, 0.0));
  double h;
  bool breakdown;
  if (ss) {
    const double t = wn2 - sq;
    breakdown = !(t > brk * brk * wn2);
    h = breakdown ? 0.0 : sqrt(t);
  } else {
    h = sqrt(fmax(*nrm2, 0.0));
    breakdown = !(h > brk * wn0);
  }
  const double hh = breakdown ? 0.0 : h;
  Hc[2 * (j + 1)] = hh;
  Hc[2 * (j + 1) + 1] = 0.0;
  *a.inv_h = breakdown ? 0.0 : 1.0 / h;
  // carry the running entry through the previous rotations:
  // [h_i; h_{i+1}] <- [[c_i, s_i], [-conj(s_i), c_i]] [h_i; h_{i+1}]
  double xr = hsrc[0], xi = hsrc[1];
  for (int i = 0; i < j; ++i) {
    const double c = staged ? csl[i] : cs[2 * i];
    const double sr = staged ? snl[2 * i] : sn[2 * i];
    const double si = staged ? snl[2 * i + 1] : sn[2 * i + 1];
    const double yr = hsrc[2 * (i + 1)], yi = hsrc[2 * (i + 1) + 1];
    const double nyr = -(sr * xr + si * xi) + c * yr;
    const double nyi = -(sr * xi - si * xr) + c * yi;
    xr = nyr;
    xi = nyi;
  }
  const double ax = sqrt(xr * xr + xi * xi);
  double c, sr, si;
  if (hh == 0.0) {
    c = 1.0;
    sr = si = 0.0;
  } else if (ax == 0.0) {
    c = 0.0;
    sr = 1.0;
    si = 0.0;
  } else {
    const double r = sqrt(ax * ax + hh * hh);
    c = ax / r;
    sr = (xr / ax) * hh / r;  // s = (x/|x|) h / r
    si = (xi / ax) * hh / r;
  }
  cs[2 * j] = c;
  cs[2 * j + 1] = 0.0;
  sn[2 * j] = sr;
  sn[2 * j + 1] = si;
  const double gr = g[2 * j], gi = g[2 * j + 1];
  g[2 * j] = c * gr;
  g[2 * j + 1] = c * gi;
  g[2 * (j + 1)] = -(sr * gr + si * gi);  // -conj(s) g_j
  g[2 * (j + 1) + 1] = -(sr * gi - si * gr);
  const double est = sqrt(g[2 * (j + 1)] * g[2 * (j + 1)] + g[2 * (j + 1) + 1] * g[2 * (j + 1) + 1]);
  *a.est = est;
  if (a.hest) a.hest[j] = est;
  *a.jdone = j + 1;
  if (breakdown) *a.brk_flag = 1;
  if (a.target_dev) target = *a.target_dev;
  if (breakdown || est <= target || j + 1 >= steps) {
    *a.done = 1;
    if (a.hdone) *a.hdone = 1;
  }
}

__global__ __launch_bounds__(64) void k_arnoldi_finish(ArnoldiDev a, int steps, int kC, int j,
                                                       const double* c1, const double* c2,
                                                       const double* nrm2, double target,
                                                       double brk) {
  arnoldi_finish_body(a, steps, kC, j, c1, c2, nrm2, target, brk);
}

// ------------------------------------------------------------------ batched Gram-Schmidt
// The launches of one classical Gram-Schmidt step for up to kOrthCols
// independent columns (a lockstep batch) at once: blockIdx.z is the column,
// and each column runs exactly the blocks, partial layout and sums of its own
// single launch (its grid extent gx; the launch covers the largest), so its
// results are those of the per-column launches bit for bit.
template <typename VR, int G>
__global__ __launch_bounds__(256) void k_multidot_cols(OrthCols t) {
  if (int(blockIdx.z) >= t.count) return;
  const OrthCol& a = t.c[blockIdx.z];
  if (a.done && *a.done) return;
  if (blockIdx.x >= a.gx) return;
  multidot_body<VR, G>(static_cast<const cx<VR>*>(a.b0), a.q0, static_cast<const cx<VR>*>(a.b1),
                       a.q1, a.N, static_cast<const cx<VR>*>(a.w), a.partials, int(blockIdx.x),
                       int(a.gx), int(blockIdx.y));
}

__global__ __launch_bounds__(64) void k_finalize_cols(OrthCols t) {
  if (int(blockIdx.z) >= t.count) return;
  const OrthCol& a = t.c[blockIdx.z];
  if (a.done && *a.done) return;
  finalize_value(a.partials, int(a.gx), a.result, int(blockIdx.x));
}

template <typename VR, bool SPLIT>
__global__ __launch_bounds__(256) void k_multiaxpy_cols(OrthCols t, int want_norm) {
  if (int(blockIdx.z) >= t.count) return;
  const OrthCol& a = t.c[blockIdx.z];
  if (a.done && *a.done) return;
  if (blockIdx.x >= a.gx) return;
  cx<VR>* w = static_cast<cx<VR>*>(a.w);
  const cx<VR>* b0 = static_cast<const cx<VR>*>(a.b0);
  const cx<VR>* b1 = static_cast<const cx<VR>*>(a.b1);
  if constexpr (SPLIT)
    multiaxpy_split_body<VR>(w, w, b0, a.q0, b1, a.q1, a.N, a.coef, want_norm, a.partials, 1.0,
                             int(blockIdx.x), int(a.gx));
  else
    multiaxpy_flat_body<VR>(w, w, b0, a.q0, b1, a.q1, a.N, a.coef, want_norm, a.partials, 1.0,
                            int(blockIdx.x), int(a.gx));
}

__global__ __launch_bounds__(64) void k_arnoldi_finish_cols(FinishCols t, int steps, int j,
                                                            double brk) {
  if (int(blockIdx.x) >= t.count) return;
  const FinishCol& f = t.c[blockIdx.x];
  arnoldi_finish_body(f.a, steps, f.kC, j, f.c1, f.c2, f.nrm2, f.target, brk);
}

template <typename VR>
__global__ void k_scale_step_cols(ScaleCols t, int j) {
  if (int(blockIdx.z) >= t.count) return;
  const int c = int(blockIdx.z);
  if (*t.jdone[c] != j + 1) return;
  const double sc = *t.inv_h[c];
  cx<VR>* v = static_cast<cx<VR>*>(t.v[c]);
  const size_t N = t.N[c];
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
    const cx<VR> z = v[i];
    v[i] = mk(VR(double(z.re) * sc), VR(double(z.im) * sc));
  }
}

// ------------------------------------------------------------------ gradient
__global__ void k_grad_hops(const z64* __restrict__ lam, const z64* __restrict__ x,
                            z64* __restrict__ grad, const int* __restrict__ nbr, int V, int n,
                            int tied) {
  const int site = blockIdx.x;
  const int dir = blockIdx.y;  // 0..7 untied, 0..3 tied
  const int y = nbr[dir * V + site];
  const size_t nn = size_t(n) * n;
  z64* out = grad + (size_t(site) * (tied ? 4 : 8) + dir) * nn;
  for (size_t t = threadIdx.x; t < nn; t += blockDim.x) {
    const int i = int(t / n), j = int(t % n);
    const z64 l = lam[size_t(site) * n + i];
    const z64 xv = x[size_t(y) * n + j];
    // -lambda_x,i * conj(x_y,j)
    double gr = -(l.re * xv.re + l.im * xv.im);
    double gi = -(l.im * xv.re - l.re * xv.im);
    if (tied) {
      // - g5_i x_x,i conj(lambda_y,j) g5_j
      const z64 xx = x[size_t(site) * n + i];
      const z64 ly = lam[size_t(y) * n + j];
      const double s = gam(i, n) * gam(j, n);
      gr -= s * (xx.re * ly.re + xx.im * ly.im);
      gi -= s * (xx.im * ly.re - xx.re * ly.im);
    }
    out[t] = mk(gr, gi);
  }
}

inline unsigned grid_for(size_t N, int threads, unsigned cap = 4096) {
  size_t b = (N + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return unsigned(b);
}

}  // namespace

// ====================================================================== launchers

void launch_layout_blocks(const z64* self_in, const z64* hops_in, int V, int n, void* out64,
                          void* out32, void* out16, float* scales16, hipStream_t st) {
  hipLaunchKernelGGL(k_layout, dim3(unsigned(V) * 5u), dim3(256), 0, st, self_in, hops_in, V, n,
                     static_cast<z64*>(out64), static_cast<z32*>(out32),
                     static_cast<uint32_t*>(out16), scales16);
  DC_HIP(hipGetLastError());
}

void launch_neighbours(int* nbr, int L0, int L1, int L2, int L3, hipStream_t st) {
  const int V = L0 * L1 * L2 * L3;
  hipLaunchKernelGGL(k_neighbours, dim3((V + 255) / 256), dim3(256), 0, st, nbr, L0, L1, L2, L3);
  DC_HIP(hipGetLastError());
}

template <int P>
static void apply_T(int n, int V, const void* blocks, const float* scales, const void* in,
                    void* gbuf, const int* nbr, double tm, const int* done, hipStream_t st,
                    hipEvent_t ev0, hipEvent_t ev1) {
  using VR = typename VecOf<P>::R;
  const int chunk = (5 * V + 7) / 8;
  const dim3 grid(unsigned(chunk) * 8u), block(64);
  const auto* pin = static_cast<const cx<VR>*>(in);
  auto* pg = static_cast<cx<VR>*>(gbuf);
  const bool full = (n % 8) == 0;
  switch (tile_T(n)) {
  // with events: the dispatch itself records its start and end (no marker packets)
#define DC_CASE(TV)                                                                           \
  case TV:                                                                                    \
    if (full)                                                                                 \
      hipExtLaunchKernelGGL((k_apply_blocks<TV, P, true>), grid, block, 0, st, ev0, ev1, 0,   \
                            blocks, scales, pin, pg, nbr, V, n, chunk, tm, done);            \
    else                                                                                      \
      hipExtLaunchKernelGGL((k_apply_blocks<TV, P, false>), grid, block, 0, st, ev0, ev1, 0,  \
                            blocks, scales, pin, pg, nbr, V, n, chunk, tm, done);            \
    break;
    DC_CASE(1) DC_CASE(2) DC_CASE(3) DC_CASE(4) DC_CASE(5) DC_CASE(6) DC_CASE(7) DC_CASE(8)
#undef DC_CASE
    default:
      throw InvalidArg("block size n > 64 is not supported");
  }
  DC_HIP(hipGetLastError());
}

void launch_apply_blocks(Prec p, int n, int V, const void* blocks, const float* scales,
                         const void* in, void* gbuf, const int* nbr, double tm, const int* done,
                         hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (p == P64) apply_T<P64>(n, V, blocks, scales, in, gbuf, nbr, tm, done, st, ev0, ev1);
  else if (p == P32) apply_T<P32>(n, V, blocks, scales, in, gbuf, nbr, tm, done, st, ev0, ev1);
  else apply_T<P16S>(n, V, blocks, scales, in, gbuf, nbr, tm, done, st, ev0, ev1);
}

void launch_invert_blocks(const void* tiled64, int V, int n, double tm, void* out64, void* out32,
                          void* out16, float* scales16, int* singular, hipStream_t st) {
  const size_t lds = size_t(n) * n * sizeof(z64);
  DC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_invert_blocks),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  hipLaunchKernelGGL(k_invert_blocks, dim3(unsigned(V)), dim3(256), lds, st,
                     static_cast<const z64*>(tiled64), n, tm,
                     static_cast<z64*>(out64), static_cast<z32*>(out32),
                     static_cast<uint32_t*>(out16), scales16, singular);
  DC_HIP(hipGetLastError());
}

template <int P, bool FROMBUF, int EPI>
static void bj_T(int n, int V, const void* blocks, const float* scales, const void* tin, void* out,
                 const void* vin, void* y, z64 c0, z64 ca, z64 cb, const int* done,
                 hipStream_t st, const int* rowsite = nullptr) {
  using VR = typename VecOf<P>::R;
  const int chunk = (V + 7) / 8;
  const dim3 grid(unsigned(chunk) * 8u), block(64);
  const auto* ti = static_cast<const cx<VR>*>(tin);
  auto* o = static_cast<cx<VR>*>(out);
  const auto* vi = static_cast<const cx<VR>*>(vin);
  auto* yy = static_cast<cx<VR>*>(y);
  const bool full = (n % 8) == 0;
  switch (tile_T(n)) {
#define DC_CASE(TV)                                                                              \
  case TV:                                                                                       \
    if (full)                                                                                    \
      hipLaunchKernelGGL((k_block_jacobi<TV, P, true, FROMBUF, EPI>), grid, block, 0, st, blocks, \
                         scales, ti, o, vi, yy, V, n, chunk, c0, ca, cb, done, rowsite);         \
    else                                                                                         \
      hipLaunchKernelGGL((k_block_jacobi<TV, P, false, FROMBUF, EPI>), grid, block, 0, st,       \
                         blocks, scales, ti, o, vi, yy, V, n, chunk, c0, ca, cb, done, rowsite); \
    break;
    DC_CASE(1) DC_CASE(2) DC_CASE(3) DC_CASE(4) DC_CASE(5) DC_CASE(6) DC_CASE(7) DC_CASE(8)
#undef DC_CASE
    default:
      throw InvalidArg("block size n > 64 is not supported");
  }
  DC_HIP(hipGetLastError());
}

template <bool FROMBUF, int EPI>
static void bj_P(Prec p, int n, int V, const void* blocks, const float* scales, const void* tin,
                 void* out, const void* vin, void* y, z64 c0, z64 ca, z64 cb, const int* done,
                 hipStream_t st, const int* rowsite = nullptr) {
  if (p == P64) bj_T<P64, FROMBUF, EPI>(n, V, blocks, scales, tin, out, vin, y, c0, ca, cb, done, st, rowsite);
  else if (p == P32) bj_T<P32, FROMBUF, EPI>(n, V, blocks, scales, tin, out, vin, y, c0, ca, cb, done, st, rowsite);
  else bj_T<P16S, FROMBUF, EPI>(n, V, blocks, scales, tin, out, vin, y, c0, ca, cb, done, st, rowsite);
}

void launch_bj_vec(Prec p, int n, int V, const void* inv, const float* scales, const void* in,
                   void* out, hipStream_t st) {
  const z64 z = mk(0.0, 0.0);
  bj_P<false, 0>(p, n, V, inv, scales, in, out, nullptr, nullptr, z, z, z, nullptr, st);
}

void launch_bj_gather_store(Prec p, int n, int V, const void* inv, const float* scales,
                            const void* gbuf, void* out, const int* done, hipStream_t st) {
  const z64 z = mk(0.0, 0.0);
  bj_P<true, 0>(p, n, V, inv, scales, gbuf, out, nullptr, nullptr, z, z, z, done, st);
}

void launch_bj_rows(Prec p, int n, int rows, const int* rowsite, const void* inv,
                    const float* scales, const void* in, void* out, hipStream_t st) {
  const z64 z = mk(0.0, 0.0);
  bj_P<false, 0>(p, n, rows, inv, scales, in, out, nullptr, nullptr, z, z, z, nullptr, st, rowsite);
}

template <int P>
static void reduced_oe_T(int n, int V, const void* blocks, const float* scales, const void* inv,
                         const float* invsc, const void* x_e, void* t_o, const int* nbr,
                         const int* osite, const int* done, hipStream_t st, hipEvent_t ev0,
                         hipEvent_t ev1) {
  using VR = typename VecOf<P>::R;
  const int rows = V / 2;
  const int chunk = (rows + 7) / 8;
  const dim3 grid(unsigned(chunk) * 8u), block(64 * kRedWaves);
  const auto* xe = static_cast<const cx<VR>*>(x_e);
  auto* to = static_cast<cx<VR>*>(t_o);
  const bool full = (n % 8) == 0;
  switch (tile_T(n)) {
#define DC_CASE(TV)                                                                           \
  case TV:                                                                                    \
    if (full)                                                                                 \
      hipExtLaunchKernelGGL((k_reduced_oe<TV, P, true>), grid, block, 0, st, ev0, ev1, 0,     \
                            blocks, scales, inv, invsc, xe, to, nbr, osite, V, n, chunk, done); \
    else                                                                                      \
      hipExtLaunchKernelGGL((k_reduced_oe<TV, P, false>), grid, block, 0, st, ev0, ev1, 0,    \
                            blocks, scales, inv, invsc, xe, to, nbr, osite, V, n, chunk, done); \
    break;
    DC_CASE(1) DC_CASE(2) DC_CASE(3) DC_CASE(4) DC_CASE(5) DC_CASE(6) DC_CASE(7) DC_CASE(8)
#undef DC_CASE
    default:
      throw InvalidArg("block size n > 64 is not supported");
  }
  DC_HIP(hipGetLastError());
}

void launch_reduced_oe(Prec p, int n, int V, const void* blocks, const float* scales,
                       const void* inv, const float* invsc, const void* x_e, void* t_o,
                       const int* nbr, const int* osite, const int* done, hipStream_t st,
                       hipEvent_t ev0, hipEvent_t ev1) {
  if (V < 2 || V % 2) throw InvalidArg("the reduced operator needs an even number of sites");
  if (p == P64) reduced_oe_T<P64>(n, V, blocks, scales, inv, invsc, x_e, t_o, nbr, osite, done, st, ev0, ev1);
  else if (p == P32) reduced_oe_T<P32>(n, V, blocks, scales, inv, invsc, x_e, t_o, nbr, osite, done, st, ev0, ev1);
  else reduced_oe_T<P16S>(n, V, blocks, scales, inv, invsc, x_e, t_o, nbr, osite, done, st, ev0, ev1);
}

template <int P, int EPI, bool BJ>
static void reduced_eo_T(int n, int V, const void* blocks, const float* scales, const void* einv,
                         const float* einvsc, const void* x_e, const void* t_o, const int* nbr,
                         const int* esite, double tm, void* out, const void* e, void* y, z64 c0,
                         z64 ca, z64 cb, const int* done, hipStream_t st, hipEvent_t ev0,
                         hipEvent_t ev1) {
  using VR = typename VecOf<P>::R;
  const int rows = V / 2;
  const int chunk = (rows + 7) / 8;
  const dim3 grid(unsigned(chunk) * 8u), block(64 * kRedWaves);
  const auto* xe = static_cast<const cx<VR>*>(x_e);
  const auto* to = static_cast<const cx<VR>*>(t_o);
  auto* o = static_cast<cx<VR>*>(out);
  const auto* ee = static_cast<const cx<VR>*>(e);
  auto* yy = static_cast<cx<VR>*>(y);
  const bool full = (n % 8) == 0;
  switch (tile_T(n)) {
#define DC_CASE(TV)                                                                              \
  case TV:                                                                                       \
    if (full)                                                                                    \
      hipExtLaunchKernelGGL((k_reduced_eo<TV, P, true, EPI, BJ>), grid, block, 0, st, ev0, ev1,  \
                            0, blocks, scales, einv, einvsc, xe, to, nbr, esite, V, n, chunk, tm, \
                            o, ee, yy, c0, ca, cb, done);                                        \
    else                                                                                         \
      hipExtLaunchKernelGGL((k_reduced_eo<TV, P, false, EPI, BJ>), grid, block, 0, st, ev0, ev1, \
                            0, blocks, scales, einv, einvsc, xe, to, nbr, esite, V, n, chunk, tm, \
                            o, ee, yy, c0, ca, cb, done);                                        \
    break;
    DC_CASE(1) DC_CASE(2) DC_CASE(3) DC_CASE(4) DC_CASE(5) DC_CASE(6) DC_CASE(7) DC_CASE(8)
#undef DC_CASE
    default:
      throw InvalidArg("block size n > 64 is not supported");
  }
  DC_HIP(hipGetLastError());
}

template <int P>
static void reduced_eo_P(int epi, int n, int V, const void* blocks, const float* scales,
                         const void* einv, const float* einvsc, const void* x_e, const void* t_o,
                         const int* nbr, const int* esite, double tm, void* out, const void* e,
                         void* y, z64 c0, z64 ca, z64 cb, const int* done, hipStream_t st,
                         hipEvent_t ev0, hipEvent_t ev1) {
#define DC_ARGS n, V, blocks, scales, einv, einvsc, x_e, t_o, nbr, esite, tm, out, e, y, c0, ca, cb, done, st, ev0, ev1
  if (einv) {
    switch (epi) {
      case 0: reduced_eo_T<P, 0, true>(DC_ARGS); break;
      case 1: reduced_eo_T<P, 1, true>(DC_ARGS); break;
      default: reduced_eo_T<P, 2, true>(DC_ARGS); break;
    }
    return;
  }
  switch (epi) {
    case 0: reduced_eo_T<P, 0, false>(DC_ARGS); break;
    case 1: reduced_eo_T<P, 1, false>(DC_ARGS); break;
    case 2: reduced_eo_T<P, 2, false>(DC_ARGS); break;
    default: reduced_eo_T<P, 3, false>(DC_ARGS); break;
  }
#undef DC_ARGS
}

void launch_reduced_eo(Prec p, int epi, int n, int V, const void* blocks, const float* scales,
                       const void* einv, const float* einvsc, const void* x_e, const void* t_o,
                       const int* nbr, const int* esite, double tm, void* out, const void* e,
                       void* y, z64 c0, z64 ca, z64 cb, const int* done, hipStream_t st,
                       hipEvent_t ev0, hipEvent_t ev1) {
  if (epi < 0 || epi > 3) throw InvalidArg("reduced epilogue must be 0..3");
  if (einv && epi == 3) throw InvalidArg("the residual epilogue takes the unpreconditioned operator");
  if (einv && p == P16S && !einvsc) throw InvalidArg("FP16 inverses need their scales");
  if (V < 2 || V % 2) throw InvalidArg("the reduced operator needs an even number of sites");
  if (!t_o || !out) throw InvalidArg("null vector pointer");
  if ((epi == 1 || epi == 3) && !e) throw InvalidArg("null epilogue input");
  if ((epi == 1 || epi == 2) && !y) throw InvalidArg("null chain output");
#define DC_ARGS epi, n, V, blocks, scales, einv, einvsc, x_e, t_o, nbr, esite, tm, out, e, y, c0, ca, cb, done, st, ev0, ev1
  if (p == P64) reduced_eo_P<P64>(DC_ARGS);
  else if (p == P32) reduced_eo_P<P32>(DC_ARGS);
  else reduced_eo_P<P16S>(DC_ARGS);
#undef DC_ARGS
}

namespace {
int g_reduced_mode = 0;
}

void set_reduced_mode(int mode) {
  if (mode < 0 || mode > 1) throw InvalidArg("reduced kernel mode must be 0 or 1");
  g_reduced_mode = mode;
}

int reduced_mode() { return g_reduced_mode; }

bool reduced_single_read(Prec p, int n) {
  return g_reduced_mode != 1 && p != P64 && n % 8 == 0 && n >= 8 && n <= 64;
}

template <int P>
static void reduced_scatter_T(int n, int V, const void* blocks, const float* scales,
                              const void* inv, const float* invsc, const void* x_e, void* hp,
                              const int* nbr, const int* osite, const int* done, hipStream_t st,
                              hipEvent_t ev0, hipEvent_t ev1) {
  using VR = typename VecOf<P>::R;
  const int rows = V / 2;
  const int chunk = (rows + 7) / 8;
  const dim3 grid(unsigned(chunk) * 8u), block(512);
  const auto* xe = static_cast<const cx<VR>*>(x_e);
  auto* h = static_cast<cx<VR>*>(hp);
  switch (n / 8) {
#define DC_CASE(TV)                                                                          \
  case TV:                                                                                   \
    hipExtLaunchKernelGGL((k_reduced_scatter<TV, P>), grid, block, 0, st, ev0, ev1, 0, blocks, \
                          scales, inv, invsc, xe, h, nbr, osite, V, n, chunk, done);         \
    break;
    DC_CASE(1) DC_CASE(2) DC_CASE(3) DC_CASE(4) DC_CASE(5) DC_CASE(6) DC_CASE(7) DC_CASE(8)
#undef DC_CASE
    default:
      throw InvalidArg("the single-read reduced kernels need n = 8, 16, ..., 64");
  }
  DC_HIP(hipGetLastError());
}

void launch_reduced_scatter(Prec p, int n, int V, const void* blocks, const float* scales,
                            const void* inv, const float* invsc, const void* x_e, void* hp,
                            const int* nbr, const int* osite, const int* done, hipStream_t st,
                            hipEvent_t ev0, hipEvent_t ev1) {
  if (V < 2 || V % 2) throw InvalidArg("the reduced operator needs an even number of sites");
  if (p == P64 || n % 8 || n < 8 || n > 64)
    throw InvalidArg("the single-read reduced kernels take FP32 / FP16 blocks with n = 8, ..., 64");
  if (p == P16S && (!scales || !invsc)) throw InvalidArg("FP16 blocks need their scales");
  if (!x_e || !hp || !inv) throw InvalidArg("null pointer");
  if (p == P32) reduced_scatter_T<P32>(n, V, blocks, scales, inv, invsc, x_e, hp, nbr, osite, done, st, ev0, ev1);
  else reduced_scatter_T<P16S>(n, V, blocks, scales, inv, invsc, x_e, hp, nbr, osite, done, st, ev0, ev1);
}

template <int P, int EPI, bool BJ>
static void reduced_gather_T(int n, int V, const void* blocks, const float* scales,
                             const void* einv, const float* einvsc, const void* x_e,
                             const void* hp, const int* esite, double tm, void* out,
                             const void* e, void* y, z64 c0, z64 ca, z64 cb, const int* done,
                             hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  using VR = typename VecOf<P>::R;
  const int rows = V / 2;
  const int chunk = (rows + 7) / 8;
  const dim3 grid(unsigned(chunk) * 8u), block(64);
  const auto* xe = static_cast<const cx<VR>*>(x_e);
  const auto* h = static_cast<const cx<VR>*>(hp);
  auto* o = static_cast<cx<VR>*>(out);
  const auto* ee = static_cast<const cx<VR>*>(e);
  auto* yy = static_cast<cx<VR>*>(y);
  switch (n / 8) {
#define DC_CASE(TV)                                                                            \
  case TV:                                                                                     \
    hipExtLaunchKernelGGL((k_reduced_gather<TV, P, EPI, BJ>), grid, block, 0, st, ev0, ev1, 0, \
                          blocks, scales, einv, einvsc, xe, h, esite, V, n, chunk, tm, o, ee, yy, \
                          c0, ca, cb, done);                                                   \
    break;
    DC_CASE(1) DC_CASE(2) DC_CASE(3) DC_CASE(4) DC_CASE(5) DC_CASE(6) DC_CASE(7) DC_CASE(8)
#undef DC_CASE
    default:
      throw InvalidArg("the single-read reduced kernels need n = 8, 16, ..., 64");
  }
  DC_HIP(hipGetLastError());
}

template <int P>
static void reduced_gather_P(int epi, int n, int V, const void* blocks, const float* scales,
                             const void* einv, const float* einvsc, const void* x_e,
                             const void* hp, const int* esite, double tm, void* out,
                             const void* e, void* y, z64 c0, z64 ca, z64 cb, const int* done,
                             hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
#define DC_ARGS n, V, blocks, scales, einv, einvsc, x_e, hp, esite, tm, out, e, y, c0, ca, cb, done, st, ev0, ev1
  if (einv) {
    switch (epi) {
      case 0: reduced_gather_T<P, 0, true>(DC_ARGS); break;
      case 1: reduced_gather_T<P, 1, true>(DC_ARGS); break;
      default: reduced_gather_T<P, 2, true>(DC_ARGS); break;
    }
    return;
  }
  switch (epi) {
    case 0: reduced_gather_T<P, 0, false>(DC_ARGS); break;
    case 1: reduced_gather_T<P, 1, false>(DC_ARGS); break;
    case 2: reduced_gather_T<P, 2, false>(DC_ARGS); break;
    default: reduced_gather_T<P, 3, false>(DC_ARGS); break;
  }
#undef DC_ARGS
}

void launch_reduced_gather(Prec p, int epi, int n, int V, const void* blocks,
                           const float* scales, const void* einv, const float* einvsc,
                           const void* x_e, const void* hp, const int* esite, double tm,
                           void* out, const void* e, void* y, z64 c0, z64 ca, z64 cb,
                           const int* done, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (epi < 0 || epi > 3) throw InvalidArg("reduced epilogue must be 0..3");
  if (einv && epi == 3) throw InvalidArg("the residual epilogue takes the unpreconditioned operator");
  if (p == P64 || n % 8 || n < 8 || n > 64)
    throw InvalidArg("the single-read reduced kernels take FP32 / FP16 blocks with n = 8, ..., 64");
  if (p == P16S && ((einv && !einvsc) || (!einv && !scales)))
    throw InvalidArg("FP16 blocks need their scales");
  if (V < 2 || V % 2) throw InvalidArg("the reduced operator needs an even number of sites");
  if (!hp || !out) throw InvalidArg("null vector pointer");
  if (einv && !x_e) throw InvalidArg("block Jacobi needs x_e");
  if ((epi == 1 || epi == 3) && !e) throw InvalidArg("null epilogue input");
  if ((epi == 1 || epi == 2) && !y) throw InvalidArg("null chain output");
#define DC_ARGS epi, n, V, blocks, scales, einv, einvsc, x_e, hp, esite, tm, out, e, y, c0, ca, cb, done, st, ev0, ev1
  if (p == P32) reduced_gather_P<P32>(DC_ARGS);
  else reduced_gather_P<P16S>(DC_ARGS);
#undef DC_ARGS
}

void launch_oddeven_split(Prec p, int n, int half_sites, const int* esite, const int* osite,
                          void* full, void* ve, void* vo, int dir, hipStream_t st) {
  const size_t N = size_t(half_sites) * n;
  if (N == 0) return;
  const dim3 grid(unsigned((N + 255) / 256)), block(256);
  if (p == P64)
    hipLaunchKernelGGL(k_oddeven_split<double>, grid, block, 0, st, n, half_sites, esite, osite,
                       static_cast<z64*>(full), static_cast<z64*>(ve), static_cast<z64*>(vo), dir);
  else
    hipLaunchKernelGGL(k_oddeven_split<float>, grid, block, 0, st, n, half_sites, esite, osite,
                       static_cast<z32*>(full), static_cast<z32*>(ve), static_cast<z32*>(vo), dir);
  DC_HIP(hipGetLastError());
}

void launch_bj_gather_poly_first(Prec p, int n, int V, const void* inv, const float* scales,
                                 const void* gbuf, const void* v, void* prod, void* y, z64 c0,
                                 z64 ca, z64 cb, const int* done, hipStream_t st) {
  bj_P<true, 1>(p, n, V, inv, scales, gbuf, prod, v, y, c0, ca, cb, done, st);
}

void launch_bj_gather_poly(Prec p, int n, int V, const void* inv, const float* scales,
                           const void* gbuf, void* prod, void* y, z64 ca, z64 cb, const int* done,
                           hipStream_t st) {
  const z64 z = mk(0.0, 0.0);
  bj_P<true, 2>(p, n, V, inv, scales, gbuf, prod, nullptr, y, z, ca, cb, done, st);
}

static int multi_np(int n) { return (n + 15) / 16 * 16; }

void launch_chain_multi(Prec p, const void* const* t, const void* const* v, void* const* prod,
                        void* const* y, int R, size_t N, z64 c0, z64 ca, z64 cb, int first,
                        hipStream_t st) {
  if (R <= 0) return;
  const dim3 grid(grid_for(N, 256, 512), unsigned(R)), block(256);
  if (p == P64)
    hipLaunchKernelGGL(k_chain_multi<double>, grid, block, 0, st,
                       reinterpret_cast<const z64* const*>(t), reinterpret_cast<const z64* const*>(v),
                       reinterpret_cast<z64* const*>(prod), reinterpret_cast<z64* const*>(y), N, c0,
                       ca, cb, first);
  else
    hipLaunchKernelGGL(k_chain_multi<float>, grid, block, 0, st,
                       reinterpret_cast<const z32* const*>(t), reinterpret_cast<const z32* const*>(v),
                       reinterpret_cast<z32* const*>(prod), reinterpret_cast<z32* const*>(y), N, c0,
                       ca, cb, first);
  DC_HIP(hipGetLastError());
}

void launch_chain_groups(Prec p, const ChainGroups& g, int first, hipStream_t st) {
  if (g.count < 0 || g.count > kChainGroups) throw InvalidArg("chain table holds 0..8 operators");
  if (g.count == 0) return;
  size_t nmax = 1;
  int rmax = 0;
  for (int i = 0; i < g.count; ++i) {
    if (g.R[i] < 0) throw InvalidArg("negative column count");
    if (first && g.R[i] > 0 && !g.v[i]) throw InvalidArg("the first chain step needs v");
    nmax = std::max(nmax, g.N[i]);
    rmax = std::max(rmax, g.R[i]);
  }
  if (rmax == 0) return;
  const dim3 grid(grid_for(nmax, 256, 512), unsigned(rmax), unsigned(g.count)), block(256);
  if (p == P64) hipLaunchKernelGGL(k_chain_groups<double>, grid, block, 0, st, g, first);
  else hipLaunchKernelGGL(k_chain_groups<float>, grid, block, 0, st, g, first);
  DC_HIP(hipGetLastError());
}

size_t multi_lds_bytes(int n, bool dbl, int rb) {
  const int np = multi_np(n);
  return size_t(2) * (size_t(np) + rb) * (np + 1) * (dbl ? sizeof(double) : sizeof(float));
}

template <int NP, int P, typename VT, int RB>
static void multi_launch(const MultiOps& ops, unsigned sites, int rmax, hipStream_t st) {
  const size_t lds = multi_lds_bytes(ops.n, sizeof(VT) == 8, RB);
  DC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_apply_multi<NP, P, VT, RB>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  const unsigned rtiles = unsigned((rmax + RB - 1) / RB);
  hipLaunchKernelGGL((k_apply_multi<NP, P, VT, RB>), dim3(sites, rtiles), dim3(256), lds, st, ops);
  DC_HIP(hipGetLastError());
}

template <int NP, typename VT, int P>
static void multi_rb_launch(int rb, const MultiOps& ops, unsigned sites, int rmax, hipStream_t st) {
  if (rb == 16) multi_launch<NP, P, VT, 16>(ops, sites, rmax, st);
  else if (rb == 32 || sizeof(VT) == 8) multi_launch<NP, P, VT, 32>(ops, sites, rmax, st);
  else multi_launch<NP, P, VT, (sizeof(VT) == 8 ? 32 : 64)>(ops, sites, rmax, st);
}

template <int NP>
static void multi_np_launch(Prec p, int rb, const MultiOps& ops, unsigned sites, int rmax,
                            hipStream_t st) {
  if (p == P64) multi_rb_launch<NP, double, P64>(rb, ops, sites, rmax, st);
  else if (p == P32) multi_rb_launch<NP, float, P32>(rb, ops, sites, rmax, st);
  else multi_rb_launch<NP, float, P16S>(rb, ops, sites, rmax, st);
}

static void multi_dispatch(Prec p, int rb, const MultiOps& ops, unsigned sites, int rmax,
                           hipStream_t st) {
  switch (multi_np(ops.n)) {
    case 16: multi_np_launch<16>(p, rb, ops, sites, rmax, st); break;
    case 32: multi_np_launch<32>(p, rb, ops, sites, rmax, st); break;
    case 48: multi_np_launch<48>(p, rb, ops, sites, rmax, st); break;
    case 64: multi_np_launch<64>(p, rb, ops, sites, rmax, st); break;
    default: throw InvalidArg("block size n > 64 is not supported");
  }
}

// Autotuned right-hand-side tile (16, 32 or 64 per workgroup): the first launch
// of a shape class (block size, precision, right-hand-side and site-count
// buckets) times each candidate on the actual operands with HIP events and
// keeps the fastest; later launches of the class use it.
namespace {
struct TuneKey {
  int np, prec, rbucket, vbucket;
  bool operator<(const TuneKey& o) const {
    return std::tie(np, prec, rbucket, vbucket) < std::tie(o.np, o.prec, o.rbucket, o.vbucket);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
int g_tune_mode = 0;  // 0: autotune; 16/32/64: forced tile

TuneKey tune_key(Prec p, int n, int rmax, unsigned sites) {
  int rbk = 0;
  while ((16 << rbk) < rmax && rbk < 3) ++rbk;   // <=16, <=32, <=64, >64
  int vb = 0;
  while ((1u << (vb + 1)) <= sites && vb < 30) ++vb;  // floor(log2(sites))
  return TuneKey{multi_np(n), int(p), rbk, vb};
}
}  // namespace

int multi_tile_for(Prec p, int n, int rmax, unsigned sites) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tune_mode) return g_tune_mode;
  const auto it = g_tune.find(tune_key(p, n, rmax, sites));
  return it == g_tune.end() ? 0 : it->second;
}

void set_multi_tile_mode(int mode) {
  if (mode != 0 && mode != 16 && mode != 32 && mode != 64)
    throw InvalidArg("tile mode must be 0 (autotune), 16, 32 or 64");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_mode = mode;
  if (mode == 0) g_tune.clear();
}

void launch_apply_multi_ops(Prec p, int n, const MultiOpDesc* desc, int n_ops, int g5io,
                            hipStream_t st) {
  if (n_ops < 1 || n_ops > kMaxMultiOps) throw InvalidArg("1..8 operators per multi-apply");
  if (multi_np(n) > 64) throw InvalidArg("block size n > 64 is not supported");
  MultiOps ops{};
  ops.n_ops = n_ops;
  ops.n = n;
  ops.g5io = g5io;
  unsigned sites = 0;
  int rmax = 0;
  for (int i = 0; i < n_ops; ++i) {
    ops.op[i] = desc[i];
    ops.op[i].site0 = int(sites);
    sites += unsigned(desc[i].V);
    rmax = std::max(rmax, desc[i].R);
  }
  if (rmax <= 0 || sites == 0) return;
  int rb = multi_tile_for(p, n, rmax, sites);
  if (rb == 0) {
    // time every candidate (each fully overwrites the outputs)
    hipEvent_t e0, e1;
    DC_HIP(hipEventCreate(&e0));
    DC_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    for (int cand : {16, 32, 64}) {
      if (cand > 16 && (cand / 2) >= rmax) break;   // wider tiles than the batch
      if (cand == 64 && p == P64) break;            // FP64 accumulators of 64 would spill
      multi_dispatch(p, cand, ops, sites, rmax, st);   // warm
      DC_HIP(hipEventRecord(e0, st));
      for (int rep = 0; rep < 3; ++rep) multi_dispatch(p, cand, ops, sites, rmax, st);
      DC_HIP(hipEventRecord(e1, st));
      DC_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      DC_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        rb = cand;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(p, n, rmax, sites)] = rb;
    // the outputs come from the chosen tile, as in every later call (the FP32
    // tiles split their sums differently and agree only to rounding)
  }
  multi_dispatch(p, rb, ops, sites, rmax, st);
}

void launch_apply_multi(Prec p, int n, int V, const void* blocks, const float* scales,
                        const void* const* xin, void* const* yout, int R, const int* nbr, double tm,
                        int g5io, hipStream_t st) {
  MultiOpDesc d{};
  d.blocks = blocks;
  d.scales = scales;
  d.nbr = nbr;
  d.xin = xin;
  d.yout = yout;
  d.V = V;
  d.R = R;
  d.tm = tm;
  launch_apply_multi_ops(p, n, &d, 1, g5io, st);
}

void launch_gather_store(Prec p, int n, int V, const void* gbuf, void* out, const int* done,
                         hipStream_t st) {
  const size_t N = size_t(V) * n;
  const dim3 grid(unsigned((N + 255) / 256)), block(256);
  if (p == P64)
    hipLaunchKernelGGL(k_gather_store<double>, grid, block, 0, st,
                       static_cast<const z64*>(gbuf), static_cast<z64*>(out), N, n, done);
  else
    hipLaunchKernelGGL(k_gather_store<float>, grid, block, 0, st,
                       static_cast<const z32*>(gbuf), static_cast<z32*>(out), N, n, done);
  DC_HIP(hipGetLastError());
}

void launch_gather_poly(Prec p, int n, int V, const void* gbuf, void* prod, void* y, z64 ca,
                        z64 cb, const int* done, hipStream_t st) {
  const size_t N = size_t(V) * n;
  const dim3 grid(unsigned((N + 255) / 256)), block(256);
  if (p == P64)
    hipLaunchKernelGGL(k_gather_poly<double>, grid, block, 0, st, static_cast<const z64*>(gbuf),
                       static_cast<z64*>(prod), static_cast<z64*>(y), N, n, ca, cb, done);
  else
    hipLaunchKernelGGL(k_gather_poly<float>, grid, block, 0, st, static_cast<const z32*>(gbuf),
                       static_cast<z32*>(prod), static_cast<z32*>(y), N, n, ca, cb, done);
  DC_HIP(hipGetLastError());
}

void launch_gather_poly_first(Prec p, int n, int V, const void* gbuf, const void* v, void* prod,
                              void* y, z64 c0, z64 ca, z64 cb, const int* done, hipStream_t st) {
  const size_t N = size_t(V) * n;
  const dim3 grid(unsigned((N + 255) / 256)), block(256);
  if (p == P64)
    hipLaunchKernelGGL(k_gather_poly_first<double>, grid, block, 0, st,
                       static_cast<const z64*>(gbuf), static_cast<const z64*>(v),
                       static_cast<z64*>(prod), static_cast<z64*>(y), N, n, c0, ca, cb, done);
  else
    hipLaunchKernelGGL(k_gather_poly_first<float>, grid, block, 0, st,
                       static_cast<const z32*>(gbuf), static_cast<const z32*>(v),
                       static_cast<z32*>(prod), static_cast<z32*>(y), N, n, c0, ca, cb, done);
  DC_HIP(hipGetLastError());
}

// blocks of a single-value reduction over N elements: >= 4 elements per
// thread, at most 512 partials
static unsigned red_blocks(size_t N) {
  size_t b = (N + 1023) / 1024;
  if (b < 1) b = 1;
  if (b > 512) b = 512;
  return unsigned(b);
}

static void finalize(const double* partials, int nvals, int nparts, double* result,
                     const int* done, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(unsigned(nvals)), dim3(64), 0, st, partials, nparts, result,
                     done);
  DC_HIP(hipGetLastError());
}

void launch_gather_resid(Prec p, int n, int V, const void* gbuf, const void* b, void* out,
                         Reducer red, double* result, hipStream_t st) {
  const size_t N = size_t(V) * n;
  const unsigned nb = red_blocks(N);
  const dim3 grid(nb), block(256);
  if (p == P64)
    hipLaunchKernelGGL(k_gather_resid<double>, grid, block, 0, st, static_cast<const z64*>(gbuf),
                       static_cast<const z64*>(b), static_cast<z64*>(out), N, n, red, result);
  else
    hipLaunchKernelGGL(k_gather_resid<float>, grid, block, 0, st, static_cast<const z32*>(gbuf),
                       static_cast<const z32*>(b), static_cast<z32*>(out), N, n, red, result);
  DC_HIP(hipGetLastError());
  finalize(red.partials, 1, int(nb), result, nullptr, st);
}

// blocks per dot group: about one pass per thread, bounded by the partials
// capacity over all groups and values
static unsigned dot_blocks(size_t N, int values) {
  size_t b = (N + 256 * kDotE - 1) / (256 * kDotE);
  const size_t cap = size_t(kRedCap) / size_t(values > 0 ? values : 1);
  if (b > cap) b = cap;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return unsigned(b);
}

template <typename VR, int G>
static void multidot_g(const void* b0, int q0, const void* b1, int q1, size_t N, const void* w,
                       int want_norm, Reducer red, const int* done, int Q, hipStream_t st,
                       unsigned* gx_out) {
  const int gy = (Q + G - 1) / G;
  const unsigned gx = dot_blocks(N, gy * 2 * G);
  hipLaunchKernelGGL((k_multidot<VR, G>), dim3(gx, unsigned(gy)), dim3(256), 0, st,
                     static_cast<const cx<VR>*>(b0), q0, static_cast<const cx<VR>*>(b1), q1, N,
                     static_cast<const cx<VR>*>(w), want_norm, red, done);
  *gx_out = gx;
}

template <typename VR>
static unsigned multidot_t(const void* b0, int q0, const void* b1, int q1, size_t N,
                           const void* w, int want_norm, Reducer red, const int* done, int Q,
                           hipStream_t st) {
  unsigned gx = 0;
  if (Q <= 2) multidot_g<VR, 2>(b0, q0, b1, q1, N, w, want_norm, red, done, Q, st, &gx);
  else if (Q <= 4) multidot_g<VR, 4>(b0, q0, b1, q1, N, w, want_norm, red, done, Q, st, &gx);
  else if (Q <= 8) multidot_g<VR, 8>(b0, q0, b1, q1, N, w, want_norm, red, done, Q, st, &gx);
  else multidot_g<VR, 16>(b0, q0, b1, q1, N, w, want_norm, red, done, Q, st, &gx);
  return gx;
}

void launch_multidot(Prec p, const void* b0, int q0, const void* b1, int q1, size_t N,
                     const void* w, int want_norm, Reducer red, double* result, const int* done,
                     hipStream_t st) {
  const int Q = q0 + q1 + (want_norm ? 1 : 0);
  if (Q == 0) return;
  const unsigned gx = p == P64 ? multidot_t<double>(b0, q0, b1, q1, N, w, want_norm, red, done, Q, st)
                               : multidot_t<float>(b0, q0, b1, q1, N, w, want_norm, red, done, Q, st);
  DC_HIP(hipGetLastError());
  // value v of the launch is result v (value = group * 2G + 2*(q - g0) + re/im = 2q + re/im)
  finalize(red.partials, 2 * Q, int(gx), result, done, st);
}

// The update over Q basis vectors: the wave-split kernel when the basis has
// more than one chunk, else the flat one.  Returns the number of norm partials.
static unsigned multiaxpy_any(Prec p, void* w, const void* b0, int q0, const void* b1, int q1,
                              size_t N, const double* coef, int want_norm, Reducer red,
                              const int* done, const double* scale, const int* jdone, int j,
                              hipStream_t st) {
  const bool split = q0 + q1 > kAxpyG;
  const size_t per = split ? size_t(64) * kDotE : size_t(256) * kDotE;
  size_t nb = (N + per - 1) / per;
  const size_t cap = split ? 4096 : 2048;
  if (nb > cap) nb = cap;
  if (nb < 1) nb = 1;
  const dim3 grid{static_cast<unsigned>(nb)}, block{256};
  if (p == P64) {
    auto k = split ? k_multiaxpy<double> : k_multiaxpy_flat<double>;
    hipLaunchKernelGGL(k, grid, block, 0, st, static_cast<const z64*>(w), static_cast<z64*>(w),
                       static_cast<const z64*>(b0), q0, static_cast<const z64*>(b1), q1, N, coef,
                       want_norm, red, done, scale, jdone, j);
  } else {
    auto k = split ? k_multiaxpy<float> : k_multiaxpy_flat<float>;
    hipLaunchKernelGGL(k, grid, block, 0, st, static_cast<const z32*>(w), static_cast<z32*>(w),
                       static_cast<const z32*>(b0), q0, static_cast<const z32*>(b1), q1, N, coef,
                       want_norm, red, done, scale, jdone, j);
  }
  DC_HIP(hipGetLastError());
  return unsigned(nb);
}

void launch_multiaxpy(Prec p, void* w, const void* b0, int q0, const void* b1, int q1, size_t N,
                      const double* coef, int want_norm, Reducer red, double* result,
                      const int* done, hipStream_t st) {
  if (q0 + q1 == 0 && !want_norm) return;
  const unsigned nb = multiaxpy_any(p, w, b0, q0, b1, q1, N, coef, want_norm, red, done, nullptr,
                                    nullptr, 0, st);
  if (want_norm) finalize(red.partials, 1, int(nb), result, done, st);
}

namespace {
int g_batch_launches = 1;
}

void set_batch_launches(int batched) {
  if (batched != 0 && batched != 1) throw InvalidArg("batched launch mode must be 0 or 1");
  g_batch_launches = batched;
}

int batch_launches() { return g_batch_launches; }

static void check_cols(int count) {
  if (count < 0 || count > kOrthCols) throw InvalidArg("column table holds 0..16 columns");
}

static int common_q(const OrthCols& t) {
  const int Q = t.c[0].q0 + t.c[0].q1;
  for (int c = 1; c < t.count; ++c)
    if (t.c[c].q0 + t.c[c].q1 != Q) throw InvalidArg("batched columns need equal basis sizes");
  return Q;
}

template <typename VR, int G>
static void multidot_cols_g(OrthCols t, int Q, hipStream_t st) {
  const int gy = (Q + G - 1) / G;
  unsigned gmax = 1;
  for (int c = 0; c < t.count; ++c) {
    t.c[c].gx = dot_blocks(t.c[c].N, gy * 2 * G);   // as its own launch would take
    gmax = std::max(gmax, t.c[c].gx);
  }
  hipLaunchKernelGGL((k_multidot_cols<VR, G>), dim3(gmax, unsigned(gy), unsigned(t.count)),
                     dim3(256), 0, st, t);
  DC_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_finalize_cols, dim3(unsigned(2 * Q), 1u, unsigned(t.count)), dim3(64), 0,
                     st, t);
  DC_HIP(hipGetLastError());
}

template <typename VR>
static void multidot_cols_t(const OrthCols& t, int Q, hipStream_t st) {
  if (Q <= 2) multidot_cols_g<VR, 2>(t, Q, st);
  else if (Q <= 4) multidot_cols_g<VR, 4>(t, Q, st);
  else if (Q <= 8) multidot_cols_g<VR, 8>(t, Q, st);
  else multidot_cols_g<VR, 16>(t, Q, st);
}

void launch_multidot_cols(Prec p, const OrthCols& t, int want_norm, hipStream_t st) {
  check_cols(t.count);
  if (t.count == 0) return;
  const int Q = common_q(t) + (want_norm ? 1 : 0);
  if (Q == 0) return;
  if (p == P64) multidot_cols_t<double>(t, Q, st);
  else multidot_cols_t<float>(t, Q, st);
}

void launch_multiaxpy_cols(Prec p, const OrthCols& t0, int want_norm, hipStream_t st) {
  check_cols(t0.count);
  if (t0.count == 0) return;
  const int Q = common_q(t0);
  if (Q == 0 && !want_norm) return;
  OrthCols t = t0;
  // the grid of each column's own launch (multiaxpy_any)
  const bool split = Q > kAxpyG;
  const size_t per = split ? size_t(64) * kDotE : size_t(256) * kDotE;
  const size_t cap = split ? 4096 : 2048;
  unsigned gmax = 1;
  for (int c = 0; c < t.count; ++c) {
    size_t nb = (t.c[c].N + per - 1) / per;
    if (nb > cap) nb = cap;
    if (nb < 1) nb = 1;
    t.c[c].gx = unsigned(nb);
    gmax = std::max(gmax, t.c[c].gx);
  }
  const dim3 grid(gmax, 1u, unsigned(t.count));
  if (p == P64) {
    if (split) hipLaunchKernelGGL((k_multiaxpy_cols<double, true>), grid, dim3(256), 0, st, t, want_norm);
    else hipLaunchKernelGGL((k_multiaxpy_cols<double, false>), grid, dim3(256), 0, st, t, want_norm);
  } else {
    if (split) hipLaunchKernelGGL((k_multiaxpy_cols<float, true>), grid, dim3(256), 0, st, t, want_norm);
    else hipLaunchKernelGGL((k_multiaxpy_cols<float, false>), grid, dim3(256), 0, st, t, want_norm);
  }
  DC_HIP(hipGetLastError());
  if (want_norm) {
    hipLaunchKernelGGL(k_finalize_cols, dim3(1u, 1u, unsigned(t.count)), dim3(64), 0, st, t);
    DC_HIP(hipGetLastError());
  }
}

void launch_arnoldi_finish_cols(const FinishCols& t, int steps, int j, double brk,
                                hipStream_t st) {
  check_cols(t.count);
  if (t.count == 0) return;
  hipLaunchKernelGGL(k_arnoldi_finish_cols, dim3(unsigned(t.count)), dim3(64), 0, st, t, steps, j,
                     brk);
  DC_HIP(hipGetLastError());
}

void launch_scale_step_cols(Prec p, const ScaleCols& t, int j, hipStream_t st) {
  check_cols(t.count);
  if (t.count == 0) return;
  size_t nmax = 1;
  for (int c = 0; c < t.count; ++c) nmax = std::max(nmax, t.N[c]);
  const dim3 grid(grid_for(nmax, 256), 1u, unsigned(t.count)), block(256);
  if (p == P64) hipLaunchKernelGGL(k_scale_step_cols<double>, grid, block, 0, st, t, j);
  else hipLaunchKernelGGL(k_scale_step_cols<float>, grid, block, 0, st, t, j);
  DC_HIP(hipGetLastError());
}

void launch_multiaxpy_scaled(Prec p, void* w, const void* b0, int q0, const void* b1, int q1,
                             size_t N, const double* coef, const double* scale, const int* jdone,
                             int j, hipStream_t st) {
  const Reducer none{};
  multiaxpy_any(p, w, b0, q0, b1, q1, N, coef, 0, none, nullptr, scale, jdone, j, st);
}

int block_gram_parts(size_t N, int qa, int rb, size_t part_cap) {
  // enough chunks that chunks x output tiles fill the chip twice over, each
  // chunk at least 8 LDS rounds long, within the partials' capacity
  const size_t tiles = size_t((qa + kBpT - 1) / kBpT) * size_t((rb + kBpT - 1) / kBpT);
  size_t P = (2048 + tiles - 1) / std::max<size_t>(tiles, 1);
  P = std::min<size_t>(P, kGramMaxParts);
  P = std::min<size_t>(P, std::max<size_t>(N / (8 * kBpK), 1));
  if (part_cap) P = std::min<size_t>(P, part_cap / std::max<size_t>(size_t(qa) * size_t(rb), 1));
  return int(std::max<size_t>(P, 1));
}

template <typename VS, typename VC>
static void block_gram_t(const void* A, int qa, const void* B, int rb, size_t N, size_t part_cap,
                         void* part, z64* out, hipStream_t st) {
  const int P0 = block_gram_parts(N, qa, rb, part_cap);
  size_t L = (N + size_t(P0) - 1) / size_t(P0);
  L = (L + kBpK - 1) / kBpK * kBpK;
  const int P = int((N + L - 1) / L);
  const unsigned tiles = unsigned((qa + kBpT - 1) / kBpT) * unsigned((rb + kBpT - 1) / kBpT);
  const size_t qr = size_t(qa) * size_t(rb);
  hipLaunchKernelGGL((k_block_gram<VS, VC>), dim3(unsigned(P), tiles), dim3(256), 0, st,
                     static_cast<const cx<VS>*>(A), qa, static_cast<const cx<VS>*>(B), rb, N, L,
                     static_cast<cx<VC>*>(part));
  DC_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_block_gram_sum<VC>, dim3(unsigned((qr + 255) / 256)), dim3(256), 0, st,
                     static_cast<const cx<VC>*>(part), P, qr, out);
  DC_HIP(hipGetLastError());
}

void launch_block_gram(Prec p, const void* A, int qa, const void* B, int rb, size_t N, void* part,
                       z64* out, hipStream_t st, bool fp64_products, size_t part_cap) {
  if (qa <= 0 || rb <= 0) return;
  if (p == P64)
    block_gram_t<double, double>(A, qa, B, rb, N, part_cap, part, out, st);
  else if (fp64_products)
    block_gram_t<float, double>(A, qa, B, rb, N, part_cap, part, out, st);
  else
    block_gram_t<float, float>(A, qa, B, rb, N, part_cap, part, out, st);
}

template <typename VS, typename VC>
static void block_update_t(const void* b0, int q0, const void* b1, int q1, const void* S, int ldS,
                           void* C, int r, size_t N, z64 alpha, z64 beta, hipStream_t st) {
  const size_t tiles = ((N + kBpT - 1) / kBpT) * size_t((r + kBpT - 1) / kBpT);
  if (tiles > 0xffffffffull) throw InvalidArg("block update too large");
  hipLaunchKernelGGL((k_block_update<VS, VC>), dim3(unsigned(tiles)), dim3(256), 0, st,
                     static_cast<const cx<VS>*>(b0), q0, static_cast<const cx<VS>*>(b1), q1,
                     static_cast<const cx<VC>*>(S), ldS, static_cast<cx<VS>*>(C), r, N, alpha,
                     beta);
  DC_HIP(hipGetLastError());
}

void launch_block_update(Prec p, const void* A, int k, const void* S, void* C, int r, size_t N,
                         z64 alpha, z64 beta, hipStream_t st) {
  if (r <= 0 || N == 0) return;
  if (p == P64)
    block_update_t<double, double>(A, k, nullptr, 0, S, k, C, r, N, alpha, beta, st);
  else
    block_update_t<float, float>(A, k, nullptr, 0, S, k, C, r, N, alpha, beta, st);
}

void launch_combine(Prec p, const void* b0, int q0, const void* b1, int q1, size_t N,
                    const double* coef, int R, void* out, int accumulate, hipStream_t st) {
  if (R <= 0) return;
  if (R == 1) {
    size_t nb = (N + 64 * kDotE - 1) / (64 * kDotE);
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    const dim3 grid{static_cast<unsigned>(nb)}, block{256};
    if (q0 + q1 == 0) {
      if (!accumulate) launch_zero(p, out, N, st);
      return;
    }
    if (p == P64)
      hipLaunchKernelGGL(k_combine1<double>, grid, block, 0, st, static_cast<const z64*>(b0), q0,
                         static_cast<const z64*>(b1), q1, N, coef, static_cast<z64*>(out),
                         accumulate);
    else
      hipLaunchKernelGGL(k_combine1<float>, grid, block, 0, st, static_cast<const z32*>(b0), q0,
                         static_cast<const z32*>(b1), q1, N, coef, static_cast<z32*>(out),
                         accumulate);
    DC_HIP(hipGetLastError());
    return;
  }
  if (R >= kCombMfmaMin && q0 + q1 > 0) {
    // many outputs: the MFMA block update with FP64 products and sums (the
    // coefficients are FP64), out = sum + (accumulate ? out : 0)
    const z64 one = mk(1.0, 0.0), beta = mk(accumulate ? 1.0 : 0.0, 0.0);
    if (p == P64)
      block_update_t<double, double>(b0, q0, b1, q1, coef, q0 + q1, out, R, N, one, beta, st);
    else
      block_update_t<float, double>(b0, q0, b1, q1, coef, q0 + q1, out, R, N, one, beta, st);
    return;
  }
  const int gy = (R + kCombR - 1) / kCombR;
  const dim3 grid(grid_for(N, 256, 2048), unsigned(gy)), block(256);
  if (p == P64)
    hipLaunchKernelGGL(k_combine<double>, grid, block, 0, st, static_cast<const z64*>(b0), q0,
                       static_cast<const z64*>(b1), q1, N, coef, R, static_cast<z64*>(out),
                       accumulate);
  else
    hipLaunchKernelGGL(k_combine<float>, grid, block, 0, st, static_cast<const z32*>(b0), q0,
                       static_cast<const z32*>(b1), q1, N, coef, R, static_cast<z32*>(out),
                       accumulate);
  DC_HIP(hipGetLastError());
}

void launch_scale(Prec p, const void* in, void* out, size_t N, const double* scale_dev, double s,
                  const int* done, hipStream_t st) {
  const dim3 grid(grid_for(N, 256)), block(256);
  if (p == P64)
    hipLaunchKernelGGL(k_scale<double>, grid, block, 0, st, static_cast<const z64*>(in),
                       static_cast<z64*>(out), N, scale_dev, s, done);
  else
    hipLaunchKernelGGL(k_scale<float>, grid, block, 0, st, static_cast<const z32*>(in),
                       static_cast<z32*>(out), N, scale_dev, s, done);
  DC_HIP(hipGetLastError());
}

void launch_cscale(Prec p, const void* in, void* out, size_t N, z64 c, const int* done,
                   hipStream_t st) {
  const dim3 grid(grid_for(N, 256)), block(256);
  if (p == P64)
    hipLaunchKernelGGL(k_cscale<double>, grid, block, 0, st, static_cast<const z64*>(in),
                       static_cast<z64*>(out), N, c, done);
  else
    hipLaunchKernelGGL(k_cscale<float>, grid, block, 0, st, static_cast<const z32*>(in),
                       static_cast<z32*>(out), N, c, done);
  DC_HIP(hipGetLastError());
}

void launch_scale_step(Prec p, void* v, size_t N, const double* inv_h, const int* jdone, int j,
                       hipStream_t st) {
  const dim3 grid(grid_for(N, 256)), block(256);
  if (p == P64)
    hipLaunchKernelGGL(k_scale_step<double>, grid, block, 0, st, static_cast<z64*>(v), N, inv_h,
                       jdone, j);
  else
    hipLaunchKernelGGL(k_scale_step<float>, grid, block, 0, st, static_cast<z32*>(v), N, inv_h,
                       jdone, j);
  DC_HIP(hipGetLastError());
}

// 4-byte words from src to dst; one side is host-mapped pinned memory (the
// staged transfers between the solver's host logic and the device, which as
// kernels queue without the host-side cost of a copy call).
__global__ void k_copy_words(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                             size_t n) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

void launch_copy_words(const void* src, void* dst, size_t bytes, hipStream_t st) {
  if (bytes == 0) return;
  if (bytes % 4 != 0 || reinterpret_cast<uintptr_t>(src) % 4 != 0 ||
      reinterpret_cast<uintptr_t>(dst) % 4 != 0)
    throw std::invalid_argument("staged copies move aligned 4-byte words");
  const size_t n = bytes / 4;
  const dim3 grid(grid_for(n, 256, 2048)), block(256);
  hipLaunchKernelGGL(k_copy_words, grid, block, 0, st, static_cast<const uint32_t*>(src),
                     static_cast<uint32_t*>(dst), n);
  DC_HIP(hipGetLastError());
}

// Several segments of 4-byte words in one launch (blockIdx.y = segment).
__global__ void k_copy_segments(CopySegments s) {
  const int g = blockIdx.y;
  const uint32_t* __restrict__ src = s.src[g];
  uint32_t* __restrict__ dst = s.dst[g];
  const size_t n = s.words[g];
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

void launch_copy_segments(const CopySegments& s, hipStream_t st) {
  if (s.count <= 0) return;
  if (s.count > kCopySegMax) throw std::invalid_argument("too many copy segments");
  size_t most = 0;
  for (int g = 0; g < s.count; ++g) most = std::max(most, s.words[g]);
  const dim3 grid(grid_for(most, 256, 256), unsigned(s.count)), block(256);
  hipLaunchKernelGGL(k_copy_segments, grid, block, 0, st, s);
  DC_HIP(hipGetLastError());
}

void launch_zero(Prec p, void* x, size_t N, hipStream_t st) {
  const dim3 grid(grid_for(N, 256)), block(256);
  if (p == P64)
    hipLaunchKernelGGL(k_zero<double>, grid, block, 0, st, static_cast<z64*>(x), N);
  else
    hipLaunchKernelGGL(k_zero<float>, grid, block, 0, st, static_cast<z32*>(x), N);
  DC_HIP(hipGetLastError());
}

void launch_axpy(Prec p, z64 a, const void* x, void* y, size_t N, hipStream_t st) {
  const dim3 grid(grid_for(N, 256)), block(256);
  if (p == P64)
    hipLaunchKernelGGL(k_axpy<double>, grid, block, 0, st, a, static_cast<const z64*>(x),
                       static_cast<z64*>(y), N);
  else
    hipLaunchKernelGGL(k_axpy<float>, grid, block, 0, st, a, static_cast<const z32*>(x),
                       static_cast<z32*>(y), N);
  DC_HIP(hipGetLastError());
}

void launch_colnorm2(Prec p, const void* x, int q, size_t N, Reducer red, double* result,
                     hipStream_t st) {
  if (q <= 0) return;
  unsigned nb = red_blocks(N);
  const unsigned cap = unsigned(size_t(kRedCap) / size_t(q));
  if (nb > cap) nb = cap;
  const dim3 grid(nb, unsigned(q)), block(256);
  if (p == P64)
    hipLaunchKernelGGL(k_norm2<double>, grid, block, 0, st, static_cast<const z64*>(x), N, red);
  else
    hipLaunchKernelGGL(k_norm2<float>, grid, block, 0, st, static_cast<const z32*>(x), N, red);
  DC_HIP(hipGetLastError());
  finalize(red.partials, q, int(nb), result, nullptr, st);
}

void launch_norm2(Prec p, const void* x, size_t N, Reducer red, double* result, hipStream_t st) {
  launch_colnorm2(p, x, 1, N, red, result, st);
}

void launch_gamma5(Prec p, const void* in, void* out, int V, int n, hipStream_t st) {
  const size_t N = size_t(V) * n;
  const dim3 grid(grid_for(N, 256)), block(256);
  if (p == P64)
    hipLaunchKernelGGL(k_gamma5<double>, grid, block, 0, st, static_cast<const z64*>(in),
                       static_cast<z64*>(out), N, n);
  else
    hipLaunchKernelGGL(k_gamma5<float>, grid, block, 0, st, static_cast<const z32*>(in),
                       static_cast<z32*>(out), N, n);
  DC_HIP(hipGetLastError());
}

void launch_convert_64to32(const z64* in, z32* out, size_t N, int n, int g5, hipStream_t st) {
  hipLaunchKernelGGL(k_cvt64to32, dim3(grid_for(N, 256)), dim3(256), 0, st, in, out, N, n, g5);
  DC_HIP(hipGetLastError());
}

void launch_convert_32to64(const z32* in, z64* out, size_t N, int n, int g5, hipStream_t st) {
  hipLaunchKernelGGL(k_cvt32to64, dim3(grid_for(N, 256)), dim3(256), 0, st, in, out, N, n, g5);
  DC_HIP(hipGetLastError());
}

void launch_gaussian(z64* out, size_t N, uint64_t seed, uint32_t stream_id, hipStream_t st) {
  hipLaunchKernelGGL(k_gaussian, dim3(grid_for(N, 256)), dim3(256), 0, st, out, N, seed,
                     stream_id);
  DC_HIP(hipGetLastError());
}

void launch_arnoldi_finish(ArnoldiDev a, int steps, int kC, int j, const double* c1,
                           const double* c2, const double* nrm2, double target, double brk,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_arnoldi_finish, dim3(1), dim3(64), 0, st, a, steps, kC, j, c1, c2, nrm2,
                     target, brk);
  DC_HIP(hipGetLastError());
}

void launch_arnoldi_init(ArnoldiDev a, double beta, hipStream_t st, const double* beta_dev) {
  hipLaunchKernelGGL(k_arnoldi_init, dim3(1), dim3(64), 0, st, a, beta, beta_dev);
  DC_HIP(hipGetLastError());
}

// out[0] = sqrt(max(*nrm2, 0)), out[1] = 1 / out[0] (0 for a zero norm)
__global__ void k_norm_root(const double* __restrict__ nrm2, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    const double b = sqrt(fmax(*nrm2, 0.0));
    out[0] = b;
    out[1] = b > 0.0 ? 1.0 / b : 0.0;
  }
}

void launch_norm_root(const double* nrm2, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_norm_root, dim3(1), dim3(64), 0, st, nrm2, out);
  DC_HIP(hipGetLastError());
}

void launch_grad_hops(const z64* lam, const z64* x, z64* grad, const int* nbr, int V, int n,
                      int tied, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_hops, dim3(unsigned(V), tied ? 4u : 8u), dim3(256), 0, st, lam, x,
                     grad, nbr, V, n, tied);
  DC_HIP(hipGetLastError());
}

}  // namespace dc
