// Stable LSD radix sort of (uint32 key, uint32 value) pairs, 8-bit digits,
// for the (tile, depth, id) ordering of splats (Sec. 3.3, original 3DGS
// binning).  Stability is what makes the id the final tie-break: values
// enter in id order and equal keys never swap.
//
// Per pass: a histogram kernel (per-block digit counts, digit-major), a row
// scan (one work-group per digit: exclusive scan of that digit's block counts
// and the digit's total), and a scatter kernel, which turns the 256 digit
// totals into digit bases with an in-block scan.  The
// scatter ranks keys inside a block with 64-lane ballots (eight ballots give
// the set of lanes sharing a digit), so the rank is exact and in input order
// without atomics deciding the order; the block's keys are then reordered by
// digit in LDS so that consecutive threads write consecutive addresses of
// each digit's output run.
#include <algorithm>
#include <utility>

#include "internal.h"

namespace nvgs {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
static_assert(kSortThreads == 256, "the scatter gives one thread to each of the 256 digits");
// keys per block: kSortBlock (2,048) below kSortBigKeys keys, twice that from
// there on (measured for 6.4M-661M keys: 2,048 is the fastest at 6.4M,
// 4,096 from 25M on, 35 % faster at 400M-1G; 8,192 never)
constexpr int kSortBlockBig = 2 * kSortBlock;
constexpr int64_t kSortBigKeys = (int64_t)24 << 20;
// work-groups per pass (they loop over the live blocks); these grids were
// the fastest of 1024-4096 groups for 6-100M keys
constexpr int64_t kSortGrid = 2048;  // scatter: 8 per CU
constexpr int64_t kHistGrid = 4096;  // histogram: 16 per CU

__device__ __forceinline__ int64_t live_n(const uint32_t* n_dev, int64_t cap) {
  return n_dev ? (int64_t)min((uint64_t)*n_dev, (uint64_t)cap) : cap;
}

// blocks of `block` keys holding live keys (the launches are sized by the
// capacity; work-groups loop over the live blocks only)
__device__ __forceinline__ int64_t live_blocks(const uint32_t* n_dev, int64_t cap, int block) {
  return (live_n(n_dev, cap) + block - 1) / block;
}

template <int BLOCK>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ n_dev, int64_t cap, int shift,
                                                             uint32_t dmask, uint32_t* __restrict__ hist, int64_t nblocks) {
  constexpr int kPerWave = BLOCK / kSortWaves;  // 512 or 1024 keys per wave
  constexpr int kRounds = kPerWave / 64;
  __shared__ uint32_t s_h[kSortWaves][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t n = live_n(n_dev, cap);
  const int64_t nbl = live_blocks(n_dev, cap, BLOCK);
  // the wave's keys of a block (beyond the live keys: none); the next block's
  // are loaded while this one is counted
  auto load = [&](int64_t blk, uint32_t* kv) {
    const int64_t base = blk * BLOCK + wave * kPerWave;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int64_t idx = base + r * 64 + lane;
      kv[r] = idx < n ? keys[idx] : 0xffffffffu;
    }
  };
  uint32_t kv[kRounds];
  load(blockIdx.x, kv);
  for (int64_t blk = blockIdx.x; blk < nbl; blk += gridDim.x) {
    uint32_t kn[kRounds];
    load(blk + gridDim.x, kn);
    for (int d = threadIdx.x; d < kSortWaves * 256; d += kSortThreads) (&s_h[0][0])[d] = 0;
    __syncthreads();
    const int64_t base = blk * BLOCK + wave * kPerWave;
#pragma unroll
    for (int r = 0; r < kRounds; ++r)
      if (base + r * 64 + lane < n) atomicAdd(&s_h[wave][(kv[r] >> shift) & dmask], 1u);
    __syncthreads();
    for (int d = threadIdx.x; d < 256; d += kSortThreads) {
      uint32_t s = 0;
      for (int w = 0; w < kSortWaves; ++w) s += s_h[w][d];
      hist[(int64_t)d * nblocks + blk] = s;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) kv[r] = kn[r];
  }
}

// one work-group per digit: exclusive scan of hist[d][0..nblocks) in place,
// the row total to tot[d].  The row is read and written coalesced and
// transposed through LDS (one padding word per 16) so that each thread scans
// 16 consecutive entries.
constexpr int kRowItems = 16;
constexpr int kRowTile = kSortThreads * kRowItems;
__device__ __forceinline__ int row_pad(int i) { return i + (i >> 4); }

__global__ __launch_bounds__(kSortThreads) void k_radix_rowscan(uint32_t* __restrict__ hist, int64_t nblocks,
                                                                const uint32_t* __restrict__ n_dev, int64_t cap,
                                                                int block, uint32_t* __restrict__ tot) {
  __shared__ uint32_t s_w[kSortWaves];
  __shared__ uint32_t s_x[kRowTile + kRowTile / 16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t* row = hist + (int64_t)blockIdx.x * nblocks;
  const int64_t nbl = live_blocks(n_dev, cap, block);  // the row's live entries
  uint32_t carry = 0;
  // a tile's entries, coalesced; the next tile's are loaded while this one is scanned
  auto load = [&](int64_t off, uint32_t* v) {
#pragma unroll
    for (int k = 0; k < kRowItems; ++k) {
      const int64_t i = off + k * kSortThreads + threadIdx.x;
      v[k] = i < nbl ? row[i] : 0u;
    }
  };
  uint32_t cur[kRowItems];
  load(0, cur);
  for (int64_t off = 0; off < nbl; off += kRowTile) {
    uint32_t nxt[kRowItems];
    load(off + kRowTile, nxt);  // the entries past this tile, which its stores below do not touch
#pragma unroll
    for (int k = 0; k < kRowItems; ++k) s_x[row_pad(k * kSortThreads + threadIdx.x)] = cur[k];
    __syncthreads();
    uint32_t v[kRowItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kRowItems; ++k) {
      v[k] = s_x[row_pad(threadIdx.x * kRowItems + k)];
      s += v[k];
    }
    uint32_t x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();  // also orders every thread's reads of s_x before the writes below
    uint32_t pre = carry, all = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) {
      pre += (w < wave) ? s_w[w] : 0u;
      all += s_w[w];
    }
    pre += x - s;
#pragma unroll
    for (int k = 0; k < kRowItems; ++k) {
      s_x[row_pad(threadIdx.x * kRowItems + k)] = pre;
      pre += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRowItems; ++k) {
      const int i = k * kSortThreads + threadIdx.x;
      if (off + i < nbl) row[off + i] = s_x[row_pad(i)];
    }
    carry += all;
    __syncthreads();  // s_w and s_x are reused by the next tile
#pragma unroll
    for (int k = 0; k < kRowItems; ++k) cur[k] = nxt[k];
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

template <int BLOCK, bool GATHER>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, const uint32_t* __restrict__ n_dev, int64_t cap, int shift, uint32_t dmask,
    int nbits, const uint32_t* __restrict__ offs, int64_t nblocks, const uint32_t* __restrict__ digit_tot,
    int iota_vals, SortGather gather) {
  __shared__ uint32_t s_cnt[kSortWaves][256];  // per-wave digit counts, then per-wave digit bases in the block
  __shared__ uint32_t s_start[256];            // first block-local position of each digit
  __shared__ uint32_t s_glob[256];             // global position of each digit's first key of this block
  __shared__ uint32_t s_wsum[kSortWaves];
  __shared__ uint32_t s_gsum[kSortWaves];
  constexpr int kPerWave = BLOCK / kSortWaves;
  constexpr int kRounds = kPerWave / 64;
  __shared__ uint32_t s_k[BLOCK];
  __shared__ uint32_t s_v[BLOCK];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t n = live_n(n_dev, cap);
  const int64_t nbl = live_blocks(n_dev, cap, BLOCK);
  // the wave's keys and values of a block; the next block's are loaded while
  // this one is ranked and written
  auto load = [&](int64_t blk, uint32_t* k, uint32_t* v) {
    const int64_t base = blk * BLOCK + wave * kPerWave;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int64_t idx = base + r * 64 + lane;
      const bool ok = idx < n;
      k[r] = ok ? keys_in[idx] : 0u;
      v[r] = ok ? (iota_vals ? (uint32_t)idx : vals_in[idx]) : 0u;
    }
  };
  uint32_t key[kRounds], val[kRounds];
  load(blockIdx.x, key, val);
  for (int64_t blk = blockIdx.x; blk < nbl; blk += gridDim.x) {
    uint32_t nkey[kRounds], nval[kRounds];
    load(blk + gridDim.x, nkey, nval);
    for (int d = threadIdx.x; d < kSortWaves * 256; d += kSortThreads) (&s_cnt[0][0])[d] = 0;
    __syncthreads();
    const int64_t block0 = blk * BLOCK;
    const int64_t base = block0 + wave * kPerWave;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t local[kRounds];
    // phase 1: rank every key among the equal digits of this wave, in order
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int64_t idx = base + r * 64 + lane;
      const bool ok = idx < n;
      const uint32_t d = (key[r] >> shift) & dmask;
      uint64_t peers = __ballot(ok);
      for (int b = 0; b < nbits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
      }
      const uint32_t before = s_cnt[wave][d];
      local[r] = before + (uint32_t)__popcll(peers & lt);
      // the highest peer publishes the new running count (one writer per digit)
      if (ok && (peers >> lane) == 1ull) s_cnt[wave][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // phase 2: one thread per digit: block total, per-wave bases, global base;
    // then an exclusive scan of the digit totals gives each digit's block start
    const int d = threadIdx.x;  // kSortThreads == 256 digits
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) {
      const uint32_t c = s_cnt[w][d];
      s_cnt[w][d] = tot;
      tot += c;
    }
    // digit d's global base: the exclusive scan of the digit totals plus this
    // block's row-exclusive count
    const uint32_t gt = digit_tot[d];
    uint32_t x = tot, xg = gt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o), yg = __shfl_up(xg, o);
      if (lane >= o) {
        x += y;
        xg += yg;
      }
    }
    if (lane == 63) {
      s_wsum[wave] = x;
      s_gsum[wave] = xg;
    }
    __syncthreads();
    uint32_t wbase = 0, gbase = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) {
      wbase += (w < wave) ? s_wsum[w] : 0u;
      gbase += (w < wave) ? s_gsum[w] : 0u;
    }
    s_start[d] = wbase + x - tot;
    s_glob[d] = gbase + xg - gt + offs[(int64_t)d * nblocks + blk];
    __syncthreads();
    // phase 3: keys and values into LDS in (digit, input) order
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int64_t idx = base + r * 64 + lane;
      if (idx < n) {
        const uint32_t dg = (key[r] >> shift) & dmask;
        const uint32_t p = s_start[dg] + s_cnt[wave][dg] + local[r];
        s_k[p] = key[r];
        s_v[p] = val[r];
      }
    }
    __syncthreads();
    // phase 4: consecutive threads write consecutive positions of each digit run
    const int cnt = (int)min<int64_t>(BLOCK, n - block0);
    if constexpr (GATHER) {
      // every rectangle read of the thread is issued before the first write
      constexpr int PER = BLOCK / kSortThreads;
      uint32_t pos[PER], v[PER];
      uint2 r[PER];
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int p = (int)threadIdx.x + i * kSortThreads;
        if (p < cnt) {
          const uint32_t dg = (s_k[p] >> shift) & dmask;
          pos[i] = s_glob[dg] + (uint32_t)p - s_start[dg];
          v[i] = s_v[p];
          r[i] = gather.rect[v[i]];
        }
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        if ((int)threadIdx.x + i * kSortThreads < cnt) {
          vals_out[pos[i]] = v[i];
          gather.rect_out[pos[i]] = r[i];
          gather.count_out[pos[i]] = (r[i].y & 0xffffu) * (r[i].y >> 16);
        }
      }
    } else {
      for (int p = threadIdx.x; p < cnt; p += kSortThreads) {
        const uint32_t k = s_k[p];
        const uint32_t dg = (k >> shift) & dmask;
        const uint32_t pos = s_glob[dg] + (uint32_t)p - s_start[dg];
        keys_out[pos] = k;
        vals_out[pos] = s_v[p];
      }
    }
    __syncthreads();  // LDS is reused by the next block
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      key[r] = nkey[r];
      val[r] = nval[r];
    }
  }
}

// The rectangles and counts of a sort with SortGather below kSortBigKeys
// keys: a pass of its own after the sort, one sorted value per thread (the
// scatter's last pass holds too few reads in flight at these sizes; from
// kSortBigKeys keys on it does the gather itself, which saves reading the
// sorted values and writing the sorted keys again)
__global__ void k_sort_gather(const uint32_t* __restrict__ vals, const uint32_t* __restrict__ n_dev, int64_t cap,
                              SortGather g) {
  const int64_t n = live_n(n_dev, cap);
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const uint2 r = g.rect[vals[j]];
    g.count_out[j] = (r.y & 0xffffu) * (r.y >> 16);
    g.rect_out[j] = r;
  }
}

// digit-major block counts, then the 256 digit totals (sized for the
// smaller block, an upper bound for both)
size_t radix_hist_words(int64_t cap) {
  int64_t nb = (cap + kSortBlock - 1) / kSortBlock;
  return (size_t)(256 * ((nb > 0 ? nb : 1) + 1));
}

// Sorts keys[0..n) (n = *n_dev, at most cap) by bits [begin_bit, end_bit).
// Buffers ping-pong between (keys, vals) and (keys_tmp, vals_tmp); the result
// ends in the tmp pair when the number of passes is odd (*result_in_tmp).
// With `gather` the sorted values' rectangles and counts are written too: by
// the last pass, in place of the sorted keys (the output key buffer is then
// left as it was), from kSortBigKeys keys on, else by a pass after the sort.
hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp,
                             const uint32_t* n_dev, int64_t cap, int begin_bit, int end_bit, int iota_vals,
                             uint32_t* hist, uint32_t* partials, bool* result_in_tmp, hipStream_t st,
                             const SortGather* gather) {
  const bool big = cap >= kSortBigKeys;
  const int block = big ? kSortBlockBig : kSortBlock;
  const int64_t nb = (cap + block - 1) / block;
  bool in_tmp = false;
  if (nb == 0 || end_bit <= begin_bit) {
    *result_in_tmp = false;
    return hipSuccess;
  }
  // at most kSortGrid work-groups, each looping over the live blocks
  const unsigned grid = (unsigned)std::min<int64_t>(nb, kSortGrid);
  const unsigned hgrid = (unsigned)std::min<int64_t>(nb, kHistGrid);
  uint32_t* kin = keys;
  uint32_t* vin = vals;
  uint32_t* kout = keys_tmp;
  uint32_t* vout = vals_tmp;
  bool first = true;
  for (int shift = begin_bit; shift < end_bit; shift += 8) {
    const int nbits = min(8, end_bit - shift);
    const uint32_t dmask = (1u << nbits) - 1u;
    uint32_t* tot = hist + 256 * nb;
    if (big)
      hipLaunchKernelGGL(k_radix_hist<kSortBlockBig>, dim3(hgrid), dim3(kSortThreads), 0, st, kin, n_dev, cap, shift,
                         dmask, hist, nb);
    else
      hipLaunchKernelGGL(k_radix_hist<kSortBlock>, dim3(hgrid), dim3(kSortThreads), 0, st, kin, n_dev, cap, shift,
                         dmask, hist, nb);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(kSortThreads), 0, st, hist, nb, n_dev, cap, block, tot);
    const bool g = big && gather && shift + 8 >= end_bit;  // the last pass of a large sort
    const SortGather ga = g ? *gather : SortGather{nullptr, nullptr, nullptr};
    const int iv = (first && iota_vals) ? 1 : 0;
#define NVGS_SCATTER(B, G)                                                                                         \
  hipLaunchKernelGGL((k_radix_scatter<B, G>), dim3(grid), dim3(kSortThreads), 0, st, kin, vin, kout, vout, n_dev, cap, \
                     shift, dmask, nbits, hist, nb, tot, iv, ga)
    if (big) {
      if (g) NVGS_SCATTER(kSortBlockBig, true); else NVGS_SCATTER(kSortBlockBig, false);
    } else {
      if (g) NVGS_SCATTER(kSortBlock, true); else NVGS_SCATTER(kSortBlock, false);
    }
#undef NVGS_SCATTER
    first = false;
    std::swap(kin, kout);
    std::swap(vin, vout);
    in_tmp = !in_tmp;
  }
  *result_in_tmp = in_tmp;
  if (gather && !big) {
    const unsigned ggrid = (unsigned)std::min<int64_t>((cap + 255) / 256, 65536);
    hipLaunchKernelGGL(k_sort_gather, dim3(ggrid), dim3(256), 0, st, in_tmp ? vals_tmp : vals, n_dev, cap, *gather);
  }
  return hipGetLastError();
}

}  // namespace nvgs
