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
// Stable LSD sort of 64-bit keys on bits [lo_bit, hi_bit), 4 bits per pass,
// by one block.  cnt: LDS table of 16 * blockDim.x counters (digit-major, so
// the exclusive scan of the table gives stable destinations).  Returns the
// buffer holding the result.

__device__ inline uint64_t* block_radix_sort(uint64_t* a, uint64_t* b, uint32_t K, int lo_bit,
                                      int hi_bit, uint32_t* cnt, uint32_t* sh16) {
  const uint32_t T = blockDim.x, t = threadIdx.x;
  const uint32_t seg = (K + T - 1) / T;
  const uint32_t beg = t * seg < K ? t * seg : K;
  const uint32_t end = beg + seg < K ? beg + seg : K;
  for (int bit = lo_bit; bit < hi_bit; bit += 4) {
    for (int d = 0; d < 16; d++) cnt[d * T + t] = 0;
    for (uint32_t i = beg; i < end; i++) cnt[((a[i] >> bit) & 15) * T + t]++;
    __syncthreads();
    // exclusive scan of the 16*T table: each thread owns 16 consecutive slots
    uint32_t loc[16];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) {
      loc[k] = cnt[t * 16 + k];
      sum += loc[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan_u32(sum, sh16, &tot);
#pragma unroll
    for (int k = 0; k < 16; k++) {
      cnt[t * 16 + k] = run;
      run += loc[k];
    }
    __syncthreads();
    for (uint32_t i = beg; i < end; i++) {
      uint64_t key = a[i];
      uint32_t slot = ((key >> bit) & 15) * T + t;
      b[cnt[slot]++] = key;
    }
    __syncthreads();
    uint64_t* tmp = a;
    a = b;
    b = tmp;
  }
  return a;
}

}  // namespace szg
