// Huffman stage on gfx950: code histogram, code lengths, canonical codebook,
// chunked bit packing, stream tables, and chunked decoding.
//
// Paper: SZ3 (arXiv 2111.02925), Section 3.2 "Encoder": the Huffman encoder
// builds a tree greedily from the symbol frequencies, derives the codebook
// from it and encodes the quantization codes; decode reverses it and
// save/load keeps the tree with the stream.  Algorithm 1 (Section 3.3): every
// code exists before encoding starts, and the quantizer's unpredictable values
// and the encoder's table are saved with the bitstream.
//
// Chunking (symbols cut into fixed-size chunks, each padded to a 32-bit word)
// is not in the paper; it makes every chunk independently decodable.
#include "common.h"

namespace szg {

// ------------------------------------------------------------ block scans

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint64_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Exclusive scan across the block (blockDim.x a multiple of 64, <= 1024).
// sh must hold 16 entries.  *total receives the block sum (all threads).
__device__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t* sh, uint32_t* total) {
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

__device__ uint64_t block_excl_scan_u64(uint64_t v, uint64_t* sh, uint64_t* total) {
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

// -------------------------------------------------------------- histogram
// Privatised per block: the bins nearest the radius (where the mass of an
// error-bounded prediction residual sits) are counted in LDS, the rest with
// global atomics.  A wave counts lanes that hit the radius bin together.

constexpr uint32_t kHistWindow = 8192;

__global__ __launch_bounds__(256) void k_histogram(const uint16_t* __restrict__ codes, uint64_t n,
                                                   uint32_t nsym, uint32_t R, uint32_t* hist) {
  __shared__ uint32_t sh[kHistWindow];
  const uint32_t lo = R > kHistWindow / 2 ? R - kHistWindow / 2 : 0;
  const uint32_t win = nsym - lo < kHistWindow ? nsym - lo : kHistWindow;
  for (uint32_t i = threadIdx.x; i < win; i += blockDim.x) sh[i] = 0;
  __syncthreads();
  const uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += gs) {
    uint32_t c = codes[i];
    uint64_t same = __ballot(c == R);
    if (c == R) {
      if ((threadIdx.x & 63) == (uint32_t)(__ffsll((long long)same) - 1))
        atomicAdd(&sh[R - lo], (uint32_t)__popcll(same));
    } else if (c - lo < win) {
      atomicAdd(&sh[c - lo], 1u);
    } else {
      atomicAdd(&hist[c], 1u);
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < win; i += blockDim.x)
    if (sh[i]) atomicAdd(&hist[lo + i], sh[i]);
}

hipError_t launch_histogram(const uint16_t* codes, uint64_t n, uint32_t nsym, uint32_t radius,
                            uint32_t* hist, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 256 * 32 - 1) / (256 * 32);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_histogram, dim3((unsigned)blocks), dim3(256), 0, st, codes, n, nsym,
                     radius, hist);
  return hipGetLastError();
}

// -------------------------------------------------- single-block radix sort
// Stable LSD sort of 64-bit keys on bits [lo_bit, hi_bit), 4 bits per pass,
// by one block.  cnt: LDS table of 16 * blockDim.x counters (digit-major, so
// the exclusive scan of the table gives stable destinations).  Returns the
// buffer holding the result.

__device__ uint64_t* block_radix_sort(uint64_t* a, uint64_t* b, uint32_t K, int lo_bit,
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

// --------------------------------------------------------------- codebook
// Huffman code lengths by the two-queue greedy merge (leaves sorted by
// (count, symbol); internal nodes in creation order, whose weights never
// decrease; each merge takes the lighter front twice, the leaf on equal
// weights), computed in parallel phases that reproduce the sequential merge
// exactly: with t the weight of the next node the sequential merge creates,
// every item present now with weight <= t (all queued internal nodes and the
// leaves up to t) is consumed, in merged order and in pairs, before any node
// created from them; an odd item out waits for the next phase.  The number of
// phases is about the longest code length.  Then canonical codes (RFC 1951
// section 3.2.2: within a length, codes are consecutive in symbol order).

constexpr int kCbThreads = 512;

__device__ __forceinline__ uint32_t lower_bound_w(const uint32_t* w, uint32_t lo, uint32_t hi,
                                                  uint64_t v) {
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if ((uint64_t)w[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}
__device__ __forceinline__ uint32_t upper_bound_w(const uint32_t* w, uint32_t lo, uint32_t hi,
                                                  uint64_t v) {
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if ((uint64_t)w[mid] <= v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Compact the symbols with nonzero `val` in ascending symbol order; returns K.
__device__ uint32_t compact_used(const uint32_t* hist, const uint8_t* lens, uint32_t nsym,
                                 uint64_t* keys, uint32_t* symtab, uint32_t* sh16) {
  const uint32_t T = blockDim.x, t = threadIdx.x;
  const uint32_t seg = (nsym + T - 1) / T;
  const uint32_t beg = t * seg < nsym ? t * seg : nsym;
  const uint32_t end = beg + seg < nsym ? beg + seg : nsym;
  uint32_t c = 0;
  for (uint32_t s = beg; s < end; s++) c += hist ? (hist[s] != 0) : (lens[s] != 0);
  uint32_t K;
  uint32_t pos = block_excl_scan_u32(c, sh16, &K);
  for (uint32_t s = beg; s < end; s++) {
    if (hist) {
      if (hist[s]) keys[pos++] = ((uint64_t)hist[s] << 32) | s;
    } else if (lens[s]) {
      keys[pos] = ((uint64_t)lens[s] << 16) | s;
      if (symtab) symtab[pos] = s | ((uint32_t)lens[s] << 16);
      pos++;
    }
  }
  __syncthreads();
  return K;
}

__global__ __launch_bounds__(kCbThreads) void k_codebook(const uint32_t* __restrict__ hist,
                                                          uint32_t nsym, CodebookScratch s,
                                                          uint64_t* enc_code, uint8_t* enc_len,
                                                          uint32_t* symtab, Meta* m) {
  __shared__ uint32_t cnt[16 * kCbThreads];
  __shared__ uint32_t sh16[16];
  __shared__ uint32_t sh_li, sh_qi, sh_qn, sh_cl, sh_ci, sh_done, sh_nphase;
  __shared__ uint32_t sh_maxw, sh_maxlen;
  __shared__ uint32_t bl_count[kMaxCodeLen + 2];
  __shared__ uint64_t first_code[kMaxCodeLen + 2];
  __shared__ uint32_t len_offset[kMaxCodeLen + 2];
  const uint32_t T = blockDim.x, t = threadIdx.x;

  for (uint32_t i = t; i < nsym; i += T) enc_len[i] = 0;
  if (t == 0) {
    m->n_unpred = hist[0];
    sh_maxw = 0;
    sh_maxlen = 0;
  }
  if (t <= kMaxCodeLen + 1) bl_count[t] = 0;
  __syncthreads();

  // 1. used symbols in symbol order, key = count << 32 | symbol
  const uint32_t K = compact_used(hist, nullptr, nsym, s.keys_a, nullptr, sh16);
  if (K == 0) {
    if (t == 0) {
      m->nsym_used = 0;
      m->max_len = 0;
    }
    return;
  }
  if (K == 1) {
    if (t == 0) {
      uint32_t sym = (uint32_t)(s.keys_a[0] & 0xFFFF);
      enc_len[sym] = 1;
      enc_code[sym] = 0;
      symtab[0] = sym | (1u << 16);
      m->nsym_used = 1;
      m->max_len = 1;
    }
    return;
  }
  for (uint32_t i = t; i < K; i += T) atomicMax(&sh_maxw, (uint32_t)(s.keys_a[i] >> 32));
  __syncthreads();
  int wbits = 32 - __clz(sh_maxw);
  int hi_bit = 32 + ((wbits + 3) & ~3);

  // 2. stable sort by count -> leaves ordered by (count, symbol)
  uint64_t* sorted = block_radix_sort(s.keys_a, s.keys_b, K, 32, hi_bit, cnt, sh16);
  for (uint32_t i = t; i < K; i += T) {
    uint64_t key = sorted[i];
    s.w[i] = (uint32_t)(key >> 32);
    s.leaf_sym[i] = (uint16_t)(key & 0xFFFF);
  }
  if (t == 0) {
    sh_li = 0;
    sh_qi = K;
    sh_qn = K;
    sh_nphase = 0;
    sh_done = 0;
  }
  __syncthreads();

  // 3. phases of the two-queue merge
  uint32_t* w = s.w;
  for (;;) {
    if (t == 0) {
      uint32_t li = sh_li, qi = sh_qi, qn = sh_qn;
      if ((K - li) + (qn - qi) <= 1) {
        sh_done = 1;
      } else {
        uint32_t a = li, b = qi;
        uint64_t tw = 0;
        for (int k = 0; k < 2; k++) {
          if (a < K && (b >= qn || w[a] <= w[b]))
            tw += w[a++];
          else
            tw += w[b++];
        }
        sh_cl = upper_bound_w(w, li, K, tw) - li;
        sh_ci = qn - qi;
      }
    }
    __syncthreads();
    if (sh_done) break;
    const uint32_t li = sh_li, qi = sh_qi, qn = sh_qn, cl = sh_cl, ci = sh_ci;
    if (cl + ci < 2 || sh_nphase >= K) {  // cannot happen with sorted leaves; never spin
      if (t == 0) atomicOr(&m->status, kStatusCodeTooLong);
      return;
    }
    for (uint32_t a = t; a < cl; a += T) {
      uint32_t wa = w[li + a];
      uint32_t pos = a + (lower_bound_w(w, qi, qn, wa) - qi);
      s.merged[pos] = li + a;
    }
    for (uint32_t b = t; b < ci; b += T) {
      uint32_t wb = w[qi + b];
      uint32_t pos = b + (upper_bound_w(w, li, li + cl, wb) - li);
      s.merged[pos] = qi + b;
    }
    __syncthreads();
    const uint32_t c = cl + ci, np = c >> 1;
    for (uint32_t p = t; p < np; p += T) {
      uint32_t u = s.merged[2 * p], v = s.merged[2 * p + 1];
      w[qn + p] = w[u] + w[v];
      s.parent[u] = qn + p;
      s.parent[v] = qn + p;
    }
    __syncthreads();
    if (t == 0) {
      if (c & 1) {
        uint32_t last = s.merged[c - 1];
        sh_li = li + cl - (last < K ? 1 : 0);
        sh_qi = qi + ci - (last >= K ? 1 : 0);
      } else {
        sh_li = li + cl;
        sh_qi = qi + ci;
      }
      sh_qn = qn + np;
      s.phase_end[sh_nphase++] = qn + np;
    }
    __syncthreads();
  }

  // 4. depths: nodes of a phase have their parents in later phases
  const uint32_t root = 2 * K - 2;
  const uint32_t nph = sh_nphase;
  if (t == 0) s.depth[root] = 0;
  __syncthreads();
  for (int p = (int)nph - 1; p >= 0; p--) {
    uint32_t b0 = p == 0 ? K : s.phase_end[p - 1];
    uint32_t b1 = s.phase_end[p];
    for (uint32_t i = b0 + t; i < b1; i += T)
      if (i != root) s.depth[i] = s.depth[s.parent[i]] + 1;
    __syncthreads();
  }
  for (uint32_t i = t; i < K; i += T) {
    uint32_t d = s.depth[s.parent[i]] + 1;
    if (d > kMaxCodeLen) {
      atomicOr(&m->status, kStatusCodeTooLong);
      d = kMaxCodeLen;
    }
    enc_len[s.leaf_sym[i]] = (uint8_t)d;
    atomicMax(&sh_maxlen, d);
  }
  __syncthreads();

  // 5. canonical codes: (length, symbol) order
  compact_used(nullptr, enc_len, nsym, s.keys_a, symtab, sh16);
  uint64_t* bylen = block_radix_sort(s.keys_a, s.keys_b, K, 16, 24, cnt, sh16);
  for (uint32_t i = t; i < K; i += T) atomicAdd(&bl_count[(bylen[i] >> 16) & 0xFF], 1u);
  __syncthreads();
  if (t == 0) {
    uint64_t code = 0;
    uint32_t off = 0;
    for (int l = 1; l <= kMaxCodeLen; l++) {
      code = (code + (l > 1 ? bl_count[l - 1] : 0)) << 1;
      first_code[l] = code;
      len_offset[l] = off;
      off += bl_count[l];
    }
    m->nsym_used = K;
    m->max_len = sh_maxlen;
  }
  __syncthreads();
  for (uint32_t j = t; j < K; j += T) {
    uint64_t key = bylen[j];
    uint32_t l = (uint32_t)(key >> 16) & 0xFF, sym = (uint32_t)(key & 0xFFFF);
    enc_code[sym] = first_code[l] + (j - len_offset[l]);
  }
}

hipError_t launch_codebook(const uint32_t* hist, uint32_t nsym, CodebookScratch s,
                           uint64_t* enc_code, uint8_t* enc_len, uint32_t* symtab, Meta* m,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_codebook, dim3(1), dim3(kCbThreads), 0, st, hist, nsym, s, enc_code,
                     enc_len, symtab, m);
  return hipGetLastError();
}

// ------------------------------------------------------------------ encode
// One wave per chunk of `chunk` symbols (a multiple of 64); lane L owns the
// contiguous run [L*m, (L+1)*m), m = chunk / 64.

__global__ __launch_bounds__(256) void k_encode_count(const uint16_t* __restrict__ codes, uint64_t n,
                                                      uint32_t chunk,
                                                      const uint8_t* __restrict__ enc_len,
                                                      uint32_t* chunk_words,
                                                      uint32_t* chunk_unpred, uint64_t nchunks) {
  const uint64_t c = blockIdx.x * 4ull + (threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63;
  if (c >= nchunks) return;
  const uint64_t beg = c * chunk, end = beg + chunk < n ? beg + chunk : n;
  uint32_t bits = 0, zeros = 0;
  for (uint64_t i = beg + lane; i < end; i += 64) {
    uint32_t sym = codes[i];
    bits += enc_len[sym];
    zeros += sym == 0;
  }
  bits = wave_sum_u32(bits);
  zeros = wave_sum_u32(zeros);
  if (lane == 0) {
    chunk_words[c] = (bits + 31) / 32;
    chunk_unpred[c] = zeros;
  }
}

hipError_t launch_encode_count(const uint16_t* codes, uint64_t n, uint32_t chunk,
                               const uint8_t* enc_len, uint32_t* chunk_words,
                               uint32_t* chunk_unpred, hipStream_t st) {
  uint64_t nchunks = (n + chunk - 1) / chunk;
  if (nchunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_encode_count, dim3((unsigned)((nchunks + 3) / 4)), dim3(256), 0, st,
                     codes, n, chunk, enc_len, chunk_words, chunk_unpred, nchunks);
  return hipGetLastError();
}

// Three-kernel exclusive scan of u32 -> u64 (1024 elements per block).
constexpr uint32_t kScanPerBlock = 1024;

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* __restrict__ in, uint64_t n,
                                                     uint64_t* block_sums) {
  __shared__ uint64_t sh[16];
  uint64_t base = blockIdx.x * (uint64_t)kScanPerBlock;
  uint64_t v = 0;
  for (uint32_t k = 0; k < 4; k++) {
    uint64_t i = base + threadIdx.x * 4 + k;
    if (i < n) v += in[i];
  }
  uint64_t tot;
  block_excl_scan_u64(v, sh, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_blocks(uint64_t* block_sums, uint64_t nb,
                                                      uint64_t* total) {
  __shared__ uint64_t sh[16];
  const uint64_t T = blockDim.x;
  const uint64_t seg = (nb + T - 1) / T;
  const uint64_t beg = threadIdx.x * seg < nb ? threadIdx.x * seg : nb;
  const uint64_t end = beg + seg < nb ? beg + seg : nb;
  uint64_t v = 0;
  for (uint64_t i = beg; i < end; i++) v += block_sums[i];
  uint64_t tot;
  uint64_t run = block_excl_scan_u64(v, sh, &tot);
  for (uint64_t i = beg; i < end; i++) {
    uint64_t x = block_sums[i];
    block_sums[i] = run;
    run += x;
  }
  if (threadIdx.x == 0 && total) *total = tot;
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* __restrict__ in, uint64_t n,
                                                    const uint64_t* block_sums, uint64_t* out) {
  __shared__ uint64_t sh[16];
  uint64_t base = blockIdx.x * (uint64_t)kScanPerBlock;
  uint32_t loc[4];
  uint64_t v = 0;
  for (uint32_t k = 0; k < 4; k++) {
    uint64_t i = base + threadIdx.x * 4 + k;
    loc[k] = i < n ? in[i] : 0;
    v += loc[k];
  }
  uint64_t tot;
  uint64_t run = block_excl_scan_u64(v, sh, &tot) + block_sums[blockIdx.x];
  for (uint32_t k = 0; k < 4; k++) {
    uint64_t i = base + threadIdx.x * 4 + k;
    if (i < n) out[i] = run;
    run += loc[k];
  }
}

hipError_t launch_exclusive_scan_u32(const uint32_t* in, uint64_t* out, uint64_t n,
                                     uint64_t* block_sums, uint64_t* total, hipStream_t st) {
  uint64_t nb = (n + kScanPerBlock - 1) / kScanPerBlock;
  if (nb == 0) nb = 1;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(256), 0, st, in, n, block_sums);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, block_sums, nb, total);
  if (n) hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, st, in, n,
                            block_sums, out);
  return hipGetLastError();
}

__device__ __forceinline__ void guarded_store_u32(uint8_t* out, uint64_t cap, uint64_t off,
                                                  uint32_t v) {
  if (off + 4 <= cap) *reinterpret_cast<uint32_t*>(out + off) = v;
}
__device__ __forceinline__ void guarded_or_u32(uint8_t* out, uint64_t cap, uint64_t off,
                                               uint32_t v) {
  if (off + 4 <= cap && v) atomicOr(reinterpret_cast<uint32_t*>(out + off), v);
}

// Zero the bitstream section (partial words shared by two lanes are ORed).
__global__ __launch_bounds__(256) void k_zero_bits(uint8_t* out, uint64_t cap, uint64_t nchunks,
                                                   uint32_t tsize, const Meta* m) {
  Layout l = stream_layout(m->nsym_used, nchunks, m->n_unpred, tsize, m->total_words);
  const uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t wi = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; wi < m->total_words; wi += gs)
    guarded_store_u32(out, cap, l.off_bits + 4 * wi, 0u);
}

template <typename T>
__global__ __launch_bounds__(256) void k_encode_pack(const uint16_t* __restrict__ codes,
                                                     const T* __restrict__ x, uint64_t n,
                                                     uint32_t chunk,
                                                     const uint64_t* __restrict__ enc_code,
                                                     const uint8_t* __restrict__ enc_len,
                                                     const uint64_t* __restrict__ word_off,
                                                     const uint64_t* __restrict__ unpred_off,
                                                     uint8_t* out, uint64_t cap, uint64_t nchunks,
                                                     const Meta* __restrict__ m) {
  const uint64_t c = blockIdx.x * 4ull + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= nchunks) return;
  const Layout l = stream_layout(m->nsym_used, nchunks, m->n_unpred, sizeof(T), m->total_words);
  const uint32_t per = chunk / 64;
  const uint64_t cbeg = c * chunk;
  uint64_t beg = cbeg + (uint64_t)lane * per;
  uint64_t end = beg + per;
  if (beg > n) beg = n;
  if (end > n) end = n;
  uint64_t bits = 0;
  uint32_t zeros = 0;
  for (uint64_t i = beg; i < end; i++) {
    uint32_t sym = codes[i];
    bits += enc_len[sym];
    zeros += sym == 0;
  }
  const uint64_t bit0 = wave_incl_scan_u64(bits, lane) - bits;
  uint32_t zrank = wave_incl_scan_u32(zeros, lane) - zeros;
  // unpredictable values, flat order
  const uint64_t ubase = unpred_off[c];
  for (uint64_t i = beg; i < end && zeros; i++) {
    if (codes[i] == 0) {
      uint64_t off = l.off_unpred + (ubase + zrank) * sizeof(T);
      if (off + sizeof(T) <= cap) *reinterpret_cast<T*>(out + off) = x[i];
      zrank++;
    }
  }
  if (bits == 0) return;
  // bits: MSB-first into 32-bit words; whole words owned by this lane are
  // stored, the (at most two) words shared with neighbouring lanes are ORed
  const uint64_t wbase = l.off_bits + 4 * word_off[c];
  uint64_t wi = bit0 >> 5;
  const uint64_t first_wi = wi;
  const bool first_partial = (bit0 & 31) != 0;
  uint64_t acc = 0;  // pending bits, left-aligned at bit 63
  uint32_t nacc = (uint32_t)(bit0 & 31);
  auto flush = [&]() {
    uint32_t word = (uint32_t)(acc >> 32);
    if (wi == first_wi && first_partial)
      guarded_or_u32(out, cap, wbase + 4 * wi, word);
    else
      guarded_store_u32(out, cap, wbase + 4 * wi, word);
    wi++;
    acc <<= 32;
    nacc -= 32;
  };
  for (uint64_t i = beg; i < end; i++) {
    uint32_t sym = codes[i];
    uint32_t len = enc_len[sym];
    uint64_t cw = enc_code[sym];
    if (len > 32) {  // high part first
      uint32_t hl = len - 32;
      acc |= (cw >> 32) << (64 - hl - nacc);
      nacc += hl;
      if (nacc >= 32) flush();
      cw &= 0xFFFFFFFFull;
      len = 32;
    }
    acc |= cw << (64 - len - nacc);
    nacc += len;
    if (nacc >= 32) flush();
  }
  if (nacc) guarded_or_u32(out, cap, wbase + 4 * wi, (uint32_t)(acc >> 32));
}

hipError_t launch_encode_pack(const uint16_t* codes, const void* x, int dtype, uint64_t n,
                              uint32_t chunk, const uint64_t* enc_code, const uint8_t* enc_len,
                              const uint64_t* word_off, const uint64_t* unpred_off,
                              uint8_t* out, uint64_t capacity, Meta* m, hipStream_t st) {
  uint64_t nchunks = (n + chunk - 1) / chunk;
  if (nchunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_bits, dim3(1024), dim3(256), 0, st, out, capacity, nchunks,
                     dtype == SZ_F32 ? 4u : 8u, m);
  dim3 grid((unsigned)((nchunks + 3) / 4)), block(256);
  if (dtype == SZ_F32)
    hipLaunchKernelGGL(k_encode_pack<float>, grid, block, 0, st, codes, (const float*)x, n,
                       chunk, enc_code, enc_len, word_off, unpred_off, out, capacity, nchunks, m);
  else
    hipLaunchKernelGGL(k_encode_pack<double>, grid, block, 0, st, codes, (const double*)x, n,
                       chunk, enc_code, enc_len, word_off, unpred_off, out, capacity, nchunks, m);
  return hipGetLastError();
}

// Header, symbol table, chunk table and section padding.
struct HeaderBytes {
  uint8_t b[kHeaderBytes];
};

__global__ __launch_bounds__(256) void k_write_tables(uint8_t* out, uint64_t cap,
                                                      const uint32_t* __restrict__ symtab,
                                                      const uint32_t* __restrict__ chunk_words,
                                                      const uint32_t* __restrict__ chunk_unpred,
                                                      uint64_t nchunks, HeaderBytes hdr,
                                                      uint32_t tsize, Meta* m) {
  const uint64_t K = m->nsym_used;
  const Layout l = stream_layout(K, nchunks, m->n_unpred, tsize, m->total_words);
  const uint64_t gid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  if (gid == 0) {
    double eb = m->eb;
    uint64_t vals[5];
    __builtin_memcpy(&vals[0], &eb, 8);
    vals[1] = m->n_unpred;
    vals[2] = K;  // written as u32 followed by a zero u32
    vals[3] = m->total_words;
    vals[4] = l.size;
    uint8_t h[kHeaderBytes];
    for (int i = 0; i < (int)kHeaderBytes; i++) h[i] = hdr.b[i];
    const int at[5] = {56, 72, 80, 88, 96};
    for (int k = 0; k < 5; k++)
      for (int i = 0; i < 8; i++) h[at[k] + i] = (uint8_t)(vals[k] >> (8 * i));
    for (int i = 0; i < (int)kHeaderBytes; i += 4) {
      uint32_t v = h[i] | (h[i + 1] << 8) | (h[i + 2] << 16) | ((uint32_t)h[i + 3] << 24);
      guarded_store_u32(out, cap, i, v);
    }
    if (K & 1) guarded_store_u32(out, cap, l.off_sym + 4 * K, 0u);
    uint64_t ub = m->n_unpred * tsize;
    if (ub & 7) guarded_store_u32(out, cap, l.off_unpred + ub, 0u);
    m->stream_bytes = l.size;
  }
  for (uint64_t i = gid; i < K; i += gs) guarded_store_u32(out, cap, l.off_sym + 4 * i, symtab[i]);
  for (uint64_t c = gid; c < nchunks; c += gs) {
    guarded_store_u32(out, cap, l.off_chunk + 8 * c, chunk_words[c]);
    guarded_store_u32(out, cap, l.off_chunk + 8 * c + 4, chunk_unpred[c]);
  }
}

hipError_t launch_write_tables(uint8_t* out, uint64_t capacity, const uint32_t* symtab,
                               const uint32_t* chunk_words, const uint32_t* chunk_unpred,
                               uint64_t nchunks, const uint8_t* header_template, int dtype,
                               Meta* m, hipStream_t st) {
  HeaderBytes h;
  for (int i = 0; i < (int)kHeaderBytes; i++) h.b[i] = header_template[i];
  hipLaunchKernelGGL(k_write_tables, dim3(256), dim3(256), 0, st, out, capacity, symtab,
                     chunk_words, chunk_unpred, nchunks, h, dtype == SZ_F32 ? 4u : 8u, m);
  return hipGetLastError();
}

// ------------------------------------------------------------------ decode

// Build the canonical decoding tables from the stored (symbol, length) list:
// validate it (ascending symbols, lengths 1..64, a complete prefix code),
// sort by (length, symbol), and fill a lookup table indexed by the next
// kLutBits bits for codes no longer than that.
__global__ __launch_bounds__(kCbThreads) void k_decode_tables(const uint8_t* __restrict__ stream,
                                                              uint64_t off_sym, uint32_t K,
                                                              uint32_t nsym, DecodeTables d,
                                                              Meta* m) {
  __shared__ uint32_t cnt[16 * kCbThreads];
  __shared__ uint32_t sh16[16];
  __shared__ uint32_t bl[kMaxCodeLen + 2];
  __shared__ uint32_t bad;
  const uint32_t T = blockDim.x, t = threadIdx.x;
  if (t <= kMaxCodeLen + 1) bl[t] = 0;
  if (t == 0) bad = 0;
  for (uint32_t i = t; i < (1u << kLutBits); i += T) d.lut[i] = 0;
  __syncthreads();
  const uint32_t* tab = reinterpret_cast<const uint32_t*>(stream + off_sym);
  for (uint32_t i = t; i < K; i += T) {
    uint32_t e = tab[i];
    uint32_t sym = e & 0xFFFF, len = e >> 16;
    bool ok = sym < nsym && len >= 1 && len <= kMaxCodeLen;
    if (i > 0 && (tab[i - 1] & 0xFFFF) >= sym) ok = false;
    if (!ok) {
      bad = 1;
    } else {
      atomicAdd(&bl[len], 1u);
      d.keys_a[i] = ((uint64_t)len << 16) | sym;
    }
  }
  __syncthreads();
  if (t == 0 && !bad) {
    // complete prefix code: pairing nodes from the deepest level up must leave
    // exactly the root (a lone symbol must have length 1)
    if (K == 1) {
      if (bl[1] != 1) bad = 1;
    } else if (K > 1) {
      uint64_t carry = 0;
      for (int l = kMaxCodeLen; l >= 1; l--) {
        uint64_t nodes = bl[l] + carry;
        if (nodes & 1) {
          bad = 1;
          break;
        }
        carry = nodes >> 1;
      }
      if (!bad && carry != 1) bad = 1;
    }
    uint64_t code = 0;
    uint32_t off = 0;
    for (int l = 1; l <= kMaxCodeLen; l++) {
      code = (code + (l > 1 ? bl[l - 1] : 0)) << 1;
      d.first[l] = code;
      d.count[l] = bl[l];
      d.offset[l] = off;
      off += bl[l];
    }
    if (bad) atomicOr(&m->status, kStatusCorrupt);
  }
  __syncthreads();
  if (bad || K == 0) return;
  uint64_t* bylen = block_radix_sort(d.keys_a, d.keys_b, K, 16, 24, cnt, sh16);
  for (uint32_t j = t; j < K; j += T) {
    uint64_t key = bylen[j];
    uint32_t l = (uint32_t)(key >> 16) & 0xFF, sym = (uint32_t)(key & 0xFFFF);
    d.sorted_sym[j] = (uint16_t)sym;
    if (l <= kLutBits) {
      uint64_t code = d.first[l] + (j - d.offset[l]);
      uint32_t lo = (uint32_t)(code << (kLutBits - l)), span = 1u << (kLutBits - l);
      for (uint32_t k = 0; k < span; k++) d.lut[lo + k] = sym | (l << 16);
    }
  }
}

hipError_t launch_decode_tables(const uint8_t* stream, uint64_t off_sym, uint32_t nsym_used,
                                uint32_t nsym, DecodeTables t, Meta* m, hipStream_t st) {
  hipLaunchKernelGGL(k_decode_tables, dim3(1), dim3(kCbThreads), 0, st, stream, off_sym,
                     nsym_used, nsym, t, m);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_read_chunk_table(const uint8_t* __restrict__ stream,
                                                          uint64_t off_chunk, uint64_t nchunks,
                                                          uint32_t* chunk_words,
                                                          uint32_t* chunk_unpred) {
  const uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  const uint32_t* tab = reinterpret_cast<const uint32_t*>(stream + off_chunk);
  for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < nchunks; c += gs) {
    chunk_words[c] = tab[2 * c];
    chunk_unpred[c] = tab[2 * c + 1];
  }
}

hipError_t launch_chunk_table_scan(const uint8_t* stream, uint64_t off_chunk, uint64_t nchunks,
                                   uint32_t* chunk_words, uint32_t* chunk_unpred,
                                   uint64_t* word_off, uint64_t* unpred_off,
                                   uint64_t* block_sums, uint64_t* totals, hipStream_t st) {
  if (nchunks == 0) return hipSuccess;
  uint64_t blocks = (nchunks + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_read_chunk_table, dim3((unsigned)blocks), dim3(256), 0, st, stream,
                     off_chunk, nchunks, chunk_words, chunk_unpred);
  hipError_t e = launch_exclusive_scan_u32(chunk_words, word_off, nchunks, block_sums, totals, st);
  if (e != hipSuccess) return e;
  return launch_exclusive_scan_u32(chunk_unpred, unpred_off, nchunks, block_sums, totals + 1, st);
}

__global__ void k_check_totals(const uint64_t* totals, uint64_t total_words, uint64_t n_unpred,
                               Meta* m) {
  if (totals[0] != total_words || totals[1] != n_unpred) atomicOr(&m->status, kStatusCorrupt);
}

hipError_t launch_check_totals(const uint64_t* totals, uint64_t total_words, uint64_t n_unpred,
                               Meta* m, hipStream_t st) {
  hipLaunchKernelGGL(k_check_totals, dim3(1), dim3(1), 0, st, totals, total_words, n_unpred, m);
  return hipGetLastError();
}

// 64 stream bits starting at bit `pos` of a chunk of `nw` words (zeros past
// the end of the chunk).
__device__ __forceinline__ uint64_t peek64(const uint32_t* __restrict__ w, uint64_t nw,
                                           uint64_t pos) {
  uint64_t wi = pos >> 5;
  uint32_t o = (uint32_t)(pos & 31);
  uint64_t w0 = wi < nw ? w[wi] : 0, w1 = wi + 1 < nw ? w[wi + 1] : 0,
           w2 = wi + 2 < nw ? w[wi + 2] : 0;
  uint64_t v = (w0 << 32) | w1;
  if (o) v = (v << o) | (w2 >> (32 - o));
  return v;
}

template <typename T>
__global__ __launch_bounds__(64) void k_decode_chunks(
    const uint8_t* __restrict__ stream, uint64_t off_unpred, uint64_t off_bits,
    uint64_t total_words, uint64_t n_unpred, uint64_t n, uint32_t chunk, uint64_t nchunks,
    const uint32_t* __restrict__ chunk_words, const uint32_t* __restrict__ chunk_unpred,
    const uint64_t* __restrict__ word_off, const uint64_t* __restrict__ unpred_off,
    DecodeTables d, uint16_t* codes, T* out, Meta* m) {
  const uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (c >= nchunks || m->status) return;
  const uint64_t W = chunk_words[c], wbase = word_off[c];
  if (wbase + W > total_words) {
    atomicOr(&m->status, kStatusCorrupt);
    return;
  }
  const uint32_t* words = reinterpret_cast<const uint32_t*>(stream + off_bits) + wbase;
  const T* unpred = reinterpret_cast<const T*>(stream + off_unpred);
  const uint64_t nbits = W * 32, ubase = unpred_off[c], uexp = chunk_unpred[c];
  const uint64_t beg = c * chunk, end = beg + chunk < n ? beg + chunk : n;
  uint64_t pos = 0, ucnt = 0;
  for (uint64_t f = beg; f < end; f++) {
    uint64_t v = peek64(words, W, pos);
    uint32_t e = d.lut[v >> (64 - kLutBits)];
    uint32_t len = e >> 16, sym = e & 0xFFFF;
    if (len == 0) {
      for (uint32_t l = kLutBits + 1; l <= kMaxCodeLen; l++) {
        uint64_t cc = v >> (64 - l);
        if (d.count[l] && cc >= d.first[l] && cc - d.first[l] < d.count[l]) {
          sym = d.sorted_sym[d.offset[l] + (uint32_t)(cc - d.first[l])];
          len = l;
          break;
        }
      }
      if (len == 0) {
        atomicOr(&m->status, kStatusCorrupt);
        return;
      }
    }
    pos += len;
    if (pos > nbits) {
      atomicOr(&m->status, kStatusCorrupt);
      return;
    }
    codes[f] = (uint16_t)sym;
    if (sym == 0) {
      if (ucnt >= uexp || ubase + ucnt >= n_unpred) {
        atomicOr(&m->status, kStatusCorrupt);
        return;
      }
      out[f] = unpred[ubase + ucnt];
      ucnt++;
    }
  }
  if (ucnt != uexp || (pos + 31) / 32 != W) atomicOr(&m->status, kStatusCorrupt);
}

hipError_t launch_decode_chunks(const uint8_t* stream, uint64_t stream_size, uint64_t off_unpred,
                                uint64_t off_bits, uint64_t total_words, uint64_t n_unpred,
                                uint64_t n, uint32_t chunk, int dtype, const uint32_t* chunk_words,
                                const uint32_t* chunk_unpred, const uint64_t* word_off,
                                const uint64_t* unpred_off, DecodeTables t, uint16_t* codes,
                                void* out, Meta* m, hipStream_t st) {
  (void)stream_size;
  uint64_t nchunks = (n + chunk - 1) / chunk;
  if (nchunks == 0) return hipSuccess;
  dim3 grid((unsigned)((nchunks + 63) / 64)), block(64);
  if (dtype == SZ_F32)
    hipLaunchKernelGGL(k_decode_chunks<float>, grid, block, 0, st, stream, off_unpred, off_bits,
                       total_words, n_unpred, n, chunk, nchunks, chunk_words, chunk_unpred,
                       word_off, unpred_off, t, codes, (float*)out, m);
  else
    hipLaunchKernelGGL(k_decode_chunks<double>, grid, block, 0, st, stream, off_unpred, off_bits,
                       total_words, n_unpred, n, chunk, nchunks, chunk_words, chunk_unpred,
                       word_off, unpred_off, t, codes, (double*)out, m);
  return hipGetLastError();
}

}  // namespace szg
