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
#include "block_ops.h"
#include "common.h"

namespace szg {

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
      if (sym) {
        m->sym_lo = sym;
        m->sym_hi = sym;
      }
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
    if (sym) {
      atomicMin(&m->sym_lo, sym);
      atomicMax(&m->sym_hi, sym);
    }
  }
}

hipError_t launch_codebook(const uint32_t* hist, uint32_t nsym, CodebookScratch s,
                           uint64_t* enc_code, uint8_t* enc_len, uint32_t* symtab, Meta* m,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_codebook, dim3(1), dim3(kCbThreads), 0, st, hist, nsym, s, enc_code,
                     enc_len, symtab, m);
  return hipGetLastError();
}

}  // namespace szg
