// Device-wide exclusive prefix sum of uint32 counts (reduce-then-scan).
// Used for the ordered compaction of kept pairs and for the placement of
// (splat, tile) entries; each block owns 4096 consecutive items.
#include "internal.h"

namespace nvgs {

constexpr int kScanThreads = 256;
constexpr int kScanItems = kScanBlock / kScanThreads;  // 16 per thread

// exclusive scan of one value per thread across a 256-thread block
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_wave, uint32_t* block_total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) {
    uint32_t t = s_wave[w];
    base += (w < wave) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  if (block_total) *block_total = tot;
  return base + x - v;
}

__device__ __forceinline__ int64_t scan_n(int64_t n, const uint32_t* n_dev) {
  return n_dev ? (int64_t)min((uint64_t)*n_dev, (uint64_t)n) : n;
}

// wrap: if given, bit 2 (value 4) is set when a sum reaches 2^32 (the
// 32-bit offsets would wrap)
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n_cap,
                                                              const uint32_t* __restrict__ n_dev,
                                                              uint32_t* __restrict__ partials,
                                                              uint32_t* __restrict__ wrap) {
  __shared__ uint32_t s_wave[kScanThreads / 64];
  __shared__ unsigned long long s_wide[kScanThreads / 64];
  const int64_t n = scan_n(n_cap, n_dev);
  const int64_t blk0 = (int64_t)blockIdx.x * kScanBlock;
  unsigned long long s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {  // coalesced: consecutive threads read consecutive items
    const int64_t i = blk0 + k * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  uint32_t tot;
  block_exclusive_scan((uint32_t)s, s_wave, &tot);
  if (wrap) {
    unsigned long long w = s;
    for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o);
    if ((threadIdx.x & 63) == 0) s_wide[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long b = 0;
      for (int q = 0; q < kScanThreads / 64; ++q) b += s_wide[q];
      if (b >> 32) atomicOr(wrap, 4u);
    }
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// single work-group: exclusive scan of the block partials, total to *total
__global__ __launch_bounds__(kScanThreads) void k_scan_partials(uint32_t* __restrict__ partials, int64_t nb,
                                                                uint32_t* __restrict__ total,
                                                                uint32_t* __restrict__ wrap) {
  __shared__ uint32_t s_wave[kScanThreads / 64];
  uint32_t carry = 0;
  unsigned long long wide = 0;
  for (int64_t off = 0; off < nb; off += kScanBlock) {
    const int64_t base = off + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      v[k] = base + k < nb ? partials[base + k] : 0u;
      s += v[k];
    }
    uint32_t tot;
    uint32_t pre = block_exclusive_scan(s, s_wave, &tot) + carry;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (base + k < nb) partials[base + k] = pre;
      pre += v[k];
    }
    carry += tot;
    wide += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
  if (threadIdx.x == 0 && wrap && (wide >> 32)) atomicOr(wrap, 4u);
}

// The block's items are read and written coalesced (consecutive threads,
// consecutive items) and transposed through LDS so that each thread scans 16
// consecutive items; one padding word per 16 keeps both access patterns free
// of bank conflicts.
__device__ __forceinline__ int scan_pad(int i) { return i + (i >> 4); }

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t* in, uint32_t* out,  // may alias
                                                            int64_t n_cap, const uint32_t* __restrict__ n_dev,
                                                            const uint32_t* __restrict__ partials) {
  __shared__ uint32_t s_wave[kScanThreads / 64];
  __shared__ uint32_t s_x[kScanBlock + kScanBlock / 16];
  const int64_t n = scan_n(n_cap, n_dev);
  const int64_t blk0 = (int64_t)blockIdx.x * kScanBlock;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int i = k * kScanThreads + threadIdx.x;
    s_x[scan_pad(i)] = blk0 + i < n ? in[blk0 + i] : 0u;
  }
  __syncthreads();
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = s_x[scan_pad(threadIdx.x * kScanItems + k)];
    s += v[k];
  }
  // (the scan's barriers also order the reads above before the writes below)
  uint32_t pre = block_exclusive_scan(s, s_wave, nullptr) + partials[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    s_x[scan_pad(threadIdx.x * kScanItems + k)] = pre;
    pre += v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int i = k * kScanThreads + threadIdx.x;
    if (blk0 + i < n) out[blk0 + i] = s_x[scan_pad(i)];
  }
}

size_t scan_partials_needed(int64_t n) { return (size_t)((n + kScanBlock - 1) / kScanBlock) + 1; }

// n: capacity (grid size); if n_dev is given the live count is min(*n_dev, n)
hipError_t launch_scan_u32_dev(const uint32_t* in, uint32_t* out, int64_t n, const uint32_t* n_dev, uint32_t* total,
                               uint32_t* partials, hipStream_t st, uint32_t* wrap) {
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb == 0) {  // empty input: the partials kernel alone writes total = 0
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, st, partials, (int64_t)0, total, wrap);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, n_dev, partials, wrap);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, st, partials, nb, total, wrap);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, out, n, n_dev, partials);
  return hipGetLastError();
}

hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* partials,
                           hipStream_t st) {
  return launch_scan_u32_dev(in, out, n, nullptr, total, partials, st, nullptr);
}

}  // namespace nvgs
