// Wave- and block-level primitives shared by the Huffman kernels: prefix
// sums over a 64-lane wave and over a block, and a single-block stable radix
// sort.  All are called by every thread of the block (they synchronise).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace szg {

// Workgroup barrier that orders LDS accesses only: global loads and stores in
// flight stay in flight across it (a plain __syncthreads waits for them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------ block scans

__device__ inline uint32_t wave_incl_scan_u32(uint32_t v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}
// Inclusive scan over the 64 lanes with DPP lane moves (no LDS traffic):
// shifts by 1, 2, 4 and 8 within each row of 16 lanes, then the last lane of
// row 0 (and of row 2) added to row 1 (and row 3), then the last lane of
// row 1 added to rows 2 and 3.  Lanes without a source add 0.
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false); // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false); // row_bcast:31
  return v;
}

__device__ inline uint64_t wave_incl_scan_u64(uint64_t v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint64_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}
__device__ inline uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Exclusive scan across the block (blockDim.x a multiple of 64, <= 1024).
// sh must hold 16 entries.  *total receives the block sum (all threads).
__device__ inline uint32_t block_excl_scan_u32(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t inc = wave_incl_scan_u32(v, lane);
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int k = 0; k < nw; k++) {
    uint32_t s = sh[k];
    if (k < w) before += s;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

__device__ inline uint64_t block_excl_scan_u64(uint64_t v, uint64_t* sh, uint64_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint64_t inc = wave_incl_scan_u64(v, lane);
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  uint64_t before = 0, all = 0;
  for (int k = 0; k < nw; k++) {
    uint64_t s = sh[k];
    if (k < w) before += s;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

// -------------------------------------------------- single-block radix sort
// Stable LSD sort of 64-bit keys on bits [lo_bit, hi_bit), 8 bits per pass,
// by one block.  Each wave takes a contiguous segment of the keys and walks
// it in tiles of 64 (coalesced loads); within a tile the lanes holding the
// same digit are found with ballots over the digit's bits, so a key's rank
// among equal digits of its tile is a population count.  A pass counts each
// wave's keys per digit, scans the counts in (digit, wave) order (stable
// destinations), then scatters.  cnt: LDS table of at least 256 * waves
// counters.  Returns the buffer holding the result.
__device__ inline uint64_t* block_radix_sort(uint64_t* a, uint64_t* b, uint32_t K, int lo_bit,
                                             int hi_bit, uint32_t* cnt, uint32_t* sh16) {
  const uint32_t T = blockDim.x, t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = T >> 6;
  const uint32_t seg = ((K + nw - 1) / nw + 63) & ~63u;
  const uint32_t beg = wv * seg < K ? wv * seg : K;
  const uint32_t end = beg + seg < K ? beg + seg : K;
  const uint64_t below = (1ull << lane) - 1;
  // lanes whose digit equals this lane's (invalid lanes match each other only)
  auto peers = [&](uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
    m = valid ? m : ~m;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const uint64_t bk = __ballot((d >> k) & 1u);
      m &= ((d >> k) & 1u) ? bk : ~bk;
    }
    return m;
  };
  for (int bit = lo_bit; bit < hi_bit; bit += 8) {
    const uint32_t width = hi_bit - bit < 8 ? (uint32_t)(hi_bit - bit) : 8u;
    const uint64_t mask = (1ull << width) - 1;
    for (uint32_t i = t; i < 256 * nw; i += T) cnt[i] = 0;
    __syncthreads();
    // counts per (digit, wave): one leader per digit adds its tile's count
    for (uint32_t base = beg; base < end; base += 64) {
      const uint32_t i = base + lane;
      const bool valid = i < end;
      const uint32_t d = valid ? (uint32_t)((a[i] >> bit) & mask) : 0u;
      const uint64_t pm = peers(d, valid);
      if (valid && (pm & below) == 0) cnt[d * nw + wv] += (uint32_t)__popcll(pm);
    }
    __syncthreads();
    // exclusive scan of the table in (digit, wave) order: 4 entries a thread
    {
      const uint32_t per = (256 * nw + T - 1) / T;
      uint32_t loc[8];
      uint32_t sum = 0;
      for (uint32_t k = 0; k < per; k++) {
        const uint32_t i = t * per + k;
        loc[k] = i < 256 * nw ? cnt[i] : 0u;
        sum += loc[k];
      }
      uint32_t tot;
      uint32_t run = block_excl_scan_u32(sum, sh16, &tot);
      for (uint32_t k = 0; k < per; k++) {
        const uint32_t i = t * per + k;
        if (i < 256 * nw) cnt[i] = run;
        run += loc[k];
      }
    }
    __syncthreads();
    // scatter: the digit's next slot for this wave, plus the rank in the tile
    for (uint32_t base = beg; base < end; base += 64) {
      const uint32_t i = base + lane;
      const bool valid = i < end;
      const uint64_t key = valid ? a[i] : 0ull;
      const uint32_t d = (uint32_t)((key >> bit) & mask);
      const uint64_t pm = peers(d, valid);
      const uint32_t slot = d * nw + wv;
      const uint32_t pos = valid ? cnt[slot] + (uint32_t)__popcll(pm & below) : 0u;
      if (valid) b[pos] = key;
      // (a wave's LDS accesses take effect in order: every lane has read the
      // slot before its leader advances it)
      if (valid && (pm & below) == 0) cnt[slot] += (uint32_t)__popcll(pm);
    }
    __syncthreads();
    uint64_t* tmp = a;
    a = b;
    b = tmp;
  }
  return a;
}

}  // namespace szg
