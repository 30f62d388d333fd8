// Device-wide exclusive scan with a fused consumer (reduce-then-scan).
//
// scan_apply(load, apply, N, ws): for every i < N, apply(i, prefix_i, x_i)
// with x_i = load(i) and prefix_i = sum_{j<i} x_j.  Phase 1 reduces tiles of
// 4096 elements to partial sums, phase 2 scans the partials (recursively),
// phase 3 rescans each tile in registers and calls the consumer, so a
// compaction or an offset table is written in the same pass that computes
// its positions.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace wedge {

constexpr int kScanWG = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanWG * kScanItems;

template <class T>
__device__ __forceinline__ T wave_incl_scan(T x, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

template <class T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <class T, class Load>
__global__ __launch_bounds__(kScanWG) void k_scan_reduce(Load load, uint64_t N, T* partials) {
  __shared__ T s_w[kScanWG / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  T sum = 0;
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    uint64_t g = base + (uint64_t)it * kScanWG + tid;
    if (g < N) sum += load(g);
  }
  sum = wave_sum(sum);
  if (lane == 0) s_w[wave] = sum;
  __syncthreads();
  if (tid == 0) {
    T tot = 0;
#pragma unroll
    for (int w = 0; w < kScanWG / 64; ++w) tot += s_w[w];
    partials[blockIdx.x] = tot;
  }
}

// Element (it, tid) of a tile is global index base + it * 256 + tid (striped,
// coalesced).  Each of the 16 rows is scanned across the wave with shuffles;
// the four wave totals of every row go through LDS.
template <class T, class Load, class Apply>
__global__ __launch_bounds__(kScanWG) void k_scan_apply(Load load, Apply apply, uint64_t N,
                                                        const T* block_prefix) {
  __shared__ T s_tot[kScanItems][kScanWG / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  T v[kScanItems], ex[kScanItems];
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    const uint64_t g = base + (uint64_t)it * kScanWG + tid;
    v[it] = g < N ? load(g) : T(0);
  }
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    const T incl = wave_incl_scan(v[it], lane);
    ex[it] = incl - v[it];
    if (lane == 63) s_tot[it][wave] = incl;
  }
  __syncthreads();
  T run = block_prefix ? block_prefix[blockIdx.x] : T(0);
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    T row = 0, before = 0;
#pragma unroll
    for (int w = 0; w < kScanWG / 64; ++w) {
      const T x = s_tot[it][w];
      if (w < wave) before += x;
      row += x;
    }
    const uint64_t g = base + (uint64_t)it * kScanWG + tid;
    if (g < N) apply(g, run + before + ex[it], v[it]);
    run += row;
  }
}

template <class T>
struct LoadArray {
  const T* p;
  __device__ T operator()(uint64_t i) const { return p[i]; }
};
template <class T>
struct StoreExclusive {
  T* p;
  __device__ void operator()(uint64_t i, T prefix, T) const { p[i] = prefix; }
};

// Elements of scratch (type T) that scan_apply needs for N inputs.
inline size_t scan_ws_elems(uint64_t N) {
  size_t tot = 0;
  uint64_t n = N;
  while (n > (uint64_t)kScanTile) {
    uint64_t nb = ceil_div(n, kScanTile);
    tot += nb + 1;
    n = nb + 1;
  }
  return tot + 1;
}

template <class T, class Load, class Apply>
int scan_apply(Load load, Apply apply, uint64_t N, T* ws, hipStream_t st) {
  if (N == 0) return WEDGE_OK;
  uint64_t nb = ceil_div(N, kScanTile);
  if (nb == 1) {
    k_scan_apply<T, Load, Apply><<<1, kScanWG, 0, st>>>(load, apply, N, (const T*)nullptr);
    WEDGE_LAUNCH_CHECK("k_scan_apply");
    return WEDGE_OK;
  }
  T* part = ws;  // nb + 1 partial sums; the extra one reduces to 0 -> total
  k_scan_reduce<T, Load><<<(unsigned)(nb + 1), kScanWG, 0, st>>>(load, N, part);
  WEDGE_LAUNCH_CHECK("k_scan_reduce");
  int rc = scan_apply<T>(LoadArray<T>{part}, StoreExclusive<T>{part}, nb + 1, ws + nb + 1, st);
  if (rc != WEDGE_OK) return rc;
  k_scan_apply<T, Load, Apply><<<(unsigned)nb, kScanWG, 0, st>>>(load, apply, N, part);
  WEDGE_LAUNCH_CHECK("k_scan_apply");
  return WEDGE_OK;
}

// Fill kernel (used instead of hipMemsetAsync so that the calls can be
// captured into a HIP graph).
template <class T>
__global__ void k_fill(T* p, uint64_t n, T value) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = value;
}

template <class T>
int fill(T* p, uint64_t n, T value, hipStream_t st) {
  if (n == 0) return WEDGE_OK;
  uint64_t blocks = ceil_div(n, 256);
  if (blocks > 65536) blocks = 65536;
  k_fill<T><<<(unsigned)blocks, 256, 0, st>>>(p, n, value);
  WEDGE_LAUNCH_CHECK("k_fill");
  return WEDGE_OK;
}

}  // namespace wedge
