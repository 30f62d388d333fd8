// Kernels and driver of the LSD radix sort declared in radix.hpp.
#include "radix.hpp"

namespace wedge {

__global__ __launch_bounds__(kRadixWG) void k_radix_hist(const uint64_t* __restrict__ keys,
                                                         uint64_t N, int shift,
                                                         uint32_t* __restrict__ hist,
                                                         uint32_t ntiles) {
  __shared__ uint32_t s_h[kRadixWG / 64][256];
  const int tid = threadIdx.x, wave = tid >> 6;
  for (int i = tid; i < (kRadixWG / 64) * 256; i += kRadixWG) (&s_h[0][0])[i] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kRadixTile;
#pragma unroll
  for (int it = 0; it < kRadixItems; ++it) {
    uint64_t g = base + (uint64_t)it * kRadixWG + tid;
    if (g < N) atomicAdd(&s_h[wave][(keys[g] >> shift) & 255], 1u);
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < kRadixWG / 64; ++w) c += s_h[w][tid];
  hist[(uint64_t)blockIdx.x * 256 + tid] = c;
}

// Column scan of the tile-major histogram table hist[tile][digit]:
// offs[tile][d] = base[d] + sum_{t < tile} hist[t][d], base[d] = number of
// keys with a smaller digit.  Chunks of kChunk tiles: per-chunk column sums,
// one workgroup scans chunks and digits, then each chunk writes its rows.
constexpr uint32_t kChunk = 256;

__global__ __launch_bounds__(256) void k_colsum(const uint32_t* __restrict__ hist,
                                                uint32_t ntiles,
                                                uint64_t* __restrict__ chunk_sum) {
  const uint32_t d = threadIdx.x;
  const uint64_t t0 = (uint64_t)blockIdx.x * kChunk;
  const uint64_t t1 = min(t0 + kChunk, (uint64_t)ntiles);
  uint64_t s = 0;
  for (uint64_t t = t0; t < t1; ++t) s += hist[t * 256 + d];
  chunk_sum[(uint64_t)blockIdx.x * 256 + d] = s;
}

__global__ __launch_bounds__(256) void k_colscan_top(uint64_t* __restrict__ chunk_sum,
                                                     uint32_t nchunks) {
  __shared__ uint64_t s_w[4];
  const uint32_t d = threadIdx.x, lane = d & 63, wave = d >> 6;
  uint64_t total = 0;
  for (uint32_t c = 0; c < nchunks; ++c) total += chunk_sum[(uint64_t)c * 256 + d];
  const uint64_t incl = wave_incl_scan(total, (int)lane);
  if (lane == 63) s_w[wave] = incl;
  __syncthreads();
  uint64_t run = incl - total;
  for (uint32_t w = 0; w < wave; ++w) run += s_w[w];
  for (uint32_t c = 0; c < nchunks; ++c) {  // in place: exclusive prefix per chunk
    const uint64_t x = chunk_sum[(uint64_t)c * 256 + d];
    chunk_sum[(uint64_t)c * 256 + d] = run;
    run += x;
  }
}

__global__ __launch_bounds__(256) void k_colscan_apply(const uint32_t* __restrict__ hist,
                                                       uint32_t ntiles,
                                                       const uint64_t* __restrict__ chunk_pre,
                                                       uint64_t* __restrict__ offs) {
  const uint32_t d = threadIdx.x;
  const uint64_t t0 = (uint64_t)blockIdx.x * kChunk;
  const uint64_t t1 = min(t0 + kChunk, (uint64_t)ntiles);
  uint64_t run = chunk_pre[(uint64_t)blockIdx.x * 256 + d];
  for (uint64_t t = t0; t < t1; ++t) {
    offs[t * 256 + d] = run;
    run += hist[t * 256 + d];
  }
}


__global__ __launch_bounds__(kRadixWG) void k_radix_scatter(const uint64_t* __restrict__ in,
                                                            uint64_t* __restrict__ out, uint64_t N,
                                                            int shift,
                                                            const uint64_t* __restrict__ offs,
                                                            uint32_t ntiles) {
  __shared__ uint64_t s_keys[kRadixTile];
  __shared__ uint32_t s_cnt[kRadixWG / 64][256];  // per-wave digit counts -> wave offsets
  __shared__ uint32_t s_tile_off[256];
  __shared__ uint64_t s_glob[256];
  __shared__ uint32_t s_wsum[kRadixWG / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t tile = blockIdx.x;
  const uint64_t base = tile * kRadixTile;
  for (int i = tid; i < (kRadixWG / 64) * 256; i += kRadixWG) (&s_cnt[0][0])[i] = 0;
  s_glob[tid] = offs[tile * 256 + tid];
  __syncthreads();

  // Wave w owns tile positions [w*64*I, (w+1)*64*I); item i of lane l sits at
  // w*64*I + i*64 + l, so processing items in order ranks keys stably.
  uint64_t key[kRadixItems];
  uint32_t rank[kRadixItems];
  const uint64_t lt_mask = (1ULL << lane) - 1;
#pragma unroll
  for (int it = 0; it < kRadixItems; ++it) {
    const uint64_t g = base + (uint64_t)wave * 64 * kRadixItems + (uint64_t)it * 64 + lane;
    const bool valid = g < N;
    key[it] = valid ? in[g] : 0;
    const uint32_t d = (uint32_t)(key[it] >> shift) & 255;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    uint32_t before = 0;
    if (valid) before = s_cnt[wave][d];
    const uint32_t r = (uint32_t)__popcll(peers & lt_mask);
    rank[it] = before + r;
    // the lowest lane of each peer group advances the wave's counter
    if (valid && (peers & lt_mask) == 0) s_cnt[wave][d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // per digit: exclusive offsets of the waves, then the tile-local digit start
  {
    const int d = tid;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kRadixWG / 64; ++w) {
      uint32_t c = s_cnt[w][d];
      s_cnt[w][d] = run;
      run += c;
    }
    // exclusive scan of `run` over the 256 digits
    uint32_t incl = wave_incl_scan(run, lane);
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    uint32_t off = incl - run;
    for (int w = 0; w < wave; ++w) off += s_wsum[w];
    s_tile_off[d] = off;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kRadixItems; ++it) {
    const uint64_t g = base + (uint64_t)wave * 64 * kRadixItems + (uint64_t)it * 64 + lane;
    if (g < N) {
      const uint32_t d = (uint32_t)(key[it] >> shift) & 255;
      s_keys[s_tile_off[d] + s_cnt[wave][d] + rank[it]] = key[it];
    }
  }
  __syncthreads();
  const uint64_t valid_n = (N - base) < (uint64_t)kRadixTile ? (N - base) : (uint64_t)kRadixTile;
  for (int j = tid; j < (int)valid_n; j += kRadixWG) {
    const uint64_t k = s_keys[j];
    const uint32_t d = (uint32_t)(k >> shift) & 255;
    const uint64_t at = s_glob[d] + (uint64_t)(j - (int)s_tile_off[d]);
    if (at < N) out[at] = k;
  }
}

// Sorts keys[0..N) by the digits at `shifts` (least significant first),
// ping-ponging with alt.  *result receives whichever buffer holds the
// output.
int radix_sort(uint64_t* keys, uint64_t* alt, uint64_t N, const int* shifts, int npass,
                      RadixScratch sc, hipStream_t st, uint64_t** result) {
  uint64_t* a = keys;
  uint64_t* b = alt;
  if (N > 0) {
    const uint64_t nt = radix_tiles(N);
    for (int p = 0; p < npass; ++p) {
      k_radix_hist<<<(unsigned)nt, kRadixWG, 0, st>>>(a, N, shifts[p], sc.hist, (uint32_t)nt);
      WEDGE_LAUNCH_CHECK("k_radix_hist");
      const uint32_t nchunks = (uint32_t)ceil_div(nt, kChunk);
      k_colsum<<<nchunks, 256, 0, st>>>(sc.hist, (uint32_t)nt, sc.scan_ws);
      WEDGE_LAUNCH_CHECK("k_colsum");
      k_colscan_top<<<1, 256, 0, st>>>(sc.scan_ws, nchunks);
      WEDGE_LAUNCH_CHECK("k_colscan_top");
      k_colscan_apply<<<nchunks, 256, 0, st>>>(sc.hist, (uint32_t)nt, sc.scan_ws, sc.offs);
      WEDGE_LAUNCH_CHECK("k_colscan_apply");
      k_radix_scatter<<<(unsigned)nt, kRadixWG, 0, st>>>(a, b, N, shifts[p], sc.offs,
                                                         (uint32_t)nt);
      WEDGE_LAUNCH_CHECK("k_radix_scatter");
      uint64_t* t = a;
      a = b;
      b = t;
    }
  }
  *result = a;
  return WEDGE_OK;
}

}  // namespace wedge
