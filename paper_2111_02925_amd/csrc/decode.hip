// Huffman decoding (the inverse of the encoder of Section 3.2 "Encoder" in
// SZ3, arXiv 2111.02925): rebuild canonical decoding tables from the stored
// code lengths (the encoder's saved state), locate each chunk by prefix sums
// over the chunk table, and decode every chunk independently, scattering the
// verbatim unpredictable values (the quantizer's saved state) into the output.
//
// Every read of the stream is bounded by the section sizes the host has
// validated; inconsistencies set a status bit instead of faulting.
#include "block_ops.h"
#include "common.h"

namespace szg {

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

// Both exclusive scans of two u32 sequences a[i * stride], b[i * stride] with
// the same three launches as one scan (1024 entries per block): block sums of
// both, a one-block scan of both block-sum rows (thread 0 writes the totals
// and, given a Meta, flags totals other than the expected ones), then the
// offsets (and copies of the inputs, when asked).
struct PairScan {
  const uint32_t* a;
  const uint32_t* b;
  uint32_t stride;
  uint64_t n;
  uint32_t* a_copy;
  uint32_t* b_copy;
  uint64_t* a_off;
  uint64_t* b_off;
  uint64_t* sums;     // 2 * nb: block sums of a, then of b
  uint64_t* a_total;
  uint64_t* b_total;
  uint64_t want_a, want_b;
  Meta* m;            // non-null: check the totals
};

__global__ __launch_bounds__(256) void k_scan2_reduce(PairScan p) {
  __shared__ uint64_t sh[16];
  const uint64_t base = blockIdx.x * (uint64_t)kScanPerBlock;
  uint64_t va = 0, vb = 0;
  for (uint32_t k = 0; k < 4; k++) {
    const uint64_t i = base + threadIdx.x * 4 + k;
    if (i < p.n) {
      va += p.a[i * p.stride];
      vb += p.b[i * p.stride];
    }
  }
  uint64_t ta, tb;
  block_excl_scan_u64(va, sh, &ta);
  block_excl_scan_u64(vb, sh, &tb);
  if (threadIdx.x == 0) {
    p.sums[blockIdx.x] = ta;
    p.sums[gridDim.x + blockIdx.x] = tb;
  }
}

__global__ __launch_bounds__(1024) void k_scan2_blocks(PairScan p, uint64_t nb) {
  __shared__ uint64_t sh[16];
  const uint64_t T = blockDim.x;
  const uint64_t seg = (nb + T - 1) / T;
  const uint64_t beg = threadIdx.x * seg < nb ? threadIdx.x * seg : nb;
  const uint64_t end = beg + seg < nb ? beg + seg : nb;
  uint64_t tot[2];
  for (int h = 0; h < 2; h++) {
    uint64_t* bs = p.sums + h * nb;
    uint64_t v = 0;
    for (uint64_t i = beg; i < end; i++) v += bs[i];
    uint64_t run = block_excl_scan_u64(v, sh, &tot[h]);
    for (uint64_t i = beg; i < end; i++) {
      const uint64_t x = bs[i];
      bs[i] = run;
      run += x;
    }
  }
  if (threadIdx.x == 0) {
    if (p.a_total) *p.a_total = tot[0];
    if (p.b_total) *p.b_total = tot[1];
    if (p.m && (tot[0] != p.want_a || tot[1] != p.want_b)) atomicOr(&p.m->status, kStatusCorrupt);
  }
}

__global__ __launch_bounds__(256) void k_scan2_apply(PairScan p) {
  __shared__ uint64_t sh[16];
  const uint64_t base = blockIdx.x * (uint64_t)kScanPerBlock;
  uint32_t la[4], lb[4];
  uint64_t va = 0, vb = 0;
  for (uint32_t k = 0; k < 4; k++) {
    const uint64_t i = base + threadIdx.x * 4 + k;
    la[k] = i < p.n ? p.a[i * p.stride] : 0;
    lb[k] = i < p.n ? p.b[i * p.stride] : 0;
    va += la[k];
    vb += lb[k];
  }
  uint64_t ta, tb;
  uint64_t ra = block_excl_scan_u64(va, sh, &ta) + p.sums[blockIdx.x];
  uint64_t rb = block_excl_scan_u64(vb, sh, &tb) + p.sums[gridDim.x + blockIdx.x];
  for (uint32_t k = 0; k < 4; k++) {
    const uint64_t i = base + threadIdx.x * 4 + k;
    if (i < p.n) {
      if (p.a_copy) p.a_copy[i] = la[k];
      if (p.b_copy) p.b_copy[i] = lb[k];
      p.a_off[i] = ra;
      p.b_off[i] = rb;
    }
    ra += la[k];
    rb += lb[k];
  }
}

// The chunk table's scans inside the table kernel: blocks 1, 2, ... take
// slices of kSliceEntries entries (kSlicePer a thread, in order), each
// writing the slice's own exclusive offsets and its totals; the block that
// finishes the last slice (counted in Meta) turns the slice totals into
// carries, the exclusive offsets of the slices in sums[] (words, then
// unpredictable values), which the chunk decoder adds, and checks the totals.
constexpr uint32_t kSlicePer = 4;
constexpr uint32_t kSliceEntries = kCbThreads * kSlicePer;
constexpr uint32_t kSliceBlocks = 256;  // most slice blocks of one launch
__device__ void scan_slices(const PairScan& p, uint32_t nsb, uint64_t* sh) {
  __shared__ uint32_t last;
  const uint32_t t = threadIdx.x;
  const uint64_t nslices = (p.n + kSliceEntries - 1) / kSliceEntries;
  for (uint64_t sl = blockIdx.x - 1; sl < nslices; sl += nsb) {
    const uint64_t i0 = sl * kSliceEntries + (uint64_t)t * kSlicePer;
    uint32_t la[kSlicePer], lb[kSlicePer];
    uint64_t va = 0, vb = 0;
#pragma unroll
    for (uint32_t k = 0; k < kSlicePer; k++) {
      const uint64_t i = i0 + k;
      la[k] = i < p.n ? p.a[i * p.stride] : 0u;
      lb[k] = i < p.n ? p.b[i * p.stride] : 0u;
      va += la[k];
      vb += lb[k];
    }
    uint64_t ta, tb;
    uint64_t ra = block_excl_scan_u64(va, sh, &ta);
    uint64_t rb = block_excl_scan_u64(vb, sh, &tb);
#pragma unroll
    for (uint32_t k = 0; k < kSlicePer; k++) {
      const uint64_t i = i0 + k;
      if (i < p.n) {
        p.a_copy[i] = la[k];
        p.b_copy[i] = lb[k];
        p.a_off[i] = ra;
        p.b_off[i] = rb;
      }
      ra += la[k];
      rb += lb[k];
    }
    if (t == 0) {
      p.sums[sl] = ta;
      p.sums[nslices + sl] = tb;
      __threadfence();
      last = atomicAdd(&p.m->slices_done, 1u) == nslices - 1 ? 1u : 0u;
    }
    __syncthreads();
    if (last) break;  // every slice is done (this block has no further one)
  }
  if (blockIdx.x - 1 >= nslices || !last) return;
  __threadfence();
  // the carries, in place (read past this CU's cache: other blocks wrote them)
  const uint64_t per = (nslices + blockDim.x - 1) / blockDim.x;
  const uint64_t b0 = t * per < nslices ? t * per : nslices;
  const uint64_t b1 = b0 + per < nslices ? b0 + per : nslices;
  uint64_t tot[2];
  for (int h = 0; h < 2; h++) {
    uint64_t* bs = p.sums + h * nslices;
    uint64_t v = 0;
    for (uint64_t i = b0; i < b1; i++) v += __hip_atomic_load(bs + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t run = block_excl_scan_u64(v, sh, &tot[h]);
    for (uint64_t i = b0; i < b1; i++) {
      const uint64_t x = __hip_atomic_load(bs + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      bs[i] = run;
      run += x;
    }
  }
  if (t == 0) {
    p.a_total[0] = tot[0];
    p.b_total[0] = tot[1];
    if (tot[0] != p.want_a || tot[1] != p.want_b) atomicOr(&p.m->status, kStatusCorrupt);
  }
}

// Blocks past the slice blocks read the whole stream once, so that the chunk
// decoder, launched next, finds it in the Infinity Cache instead of waiting on
// HBM for every lane's first words; the values are folded into a word that is
// stored only under a condition that never holds (so that the loads stay).
constexpr uint32_t kPrefetchBlocks = 256;
__device__ void prefetch_stream(const uint8_t* stream, uint64_t bytes, uint32_t pb, uint32_t npb,
                                Meta* m) {
  // (from the first 16-byte boundary: the stream is only 8-byte aligned)
  const uint64_t skip = (16 - ((uintptr_t)stream & 15)) & 15;
  const uint4* v = reinterpret_cast<const uint4*>(stream + skip);
  const uint64_t nv = bytes > skip ? (bytes - skip) / 16 : 0, step = (uint64_t)npb * blockDim.x;
  uint32_t acc = 0;
  for (uint64_t i = pb * (uint64_t)blockDim.x + threadIdx.x; i < nv; i += 4 * step) {
    uint4 a[4];
#pragma unroll
    for (int k = 0; k < 4; k++) a[k] = i + k * step < nv ? v[i + k * step] : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 4; k++) acc ^= a[k].x ^ a[k].y ^ a[k].z ^ a[k].w;
  }
  if (bytes == 0 && acc == 0x9E3779B9u) m->pad = acc;
}

// The header fields the table kernel needs, read on the device (the same
// fields and checks as the host's parse, at the same offsets): coded
// symbols, bins, chunk count, the chunk table's place and the totals.  False
// when the header does not pass them or the chunk buffers hold fewer than
// cap chunks; the host then launches the kernel itself once it has parsed
// the header.
__device__ bool front_from_header(const uint8_t* h, uint64_t stream_size, uint64_t cap,
                                  uint32_t& K, uint32_t& nsym, uint64_t& off_chunk,
                                  uint64_t& nch, uint64_t& words, uint64_t& unpred) {
  const uint32_t* w = reinterpret_cast<const uint32_t*>(h);
  const uint64_t* d = reinterpret_cast<const uint64_t*>(h);
  if (stream_size < kHeaderBytes || w[0] != 0x31475A53u /* "SZG1" */ || (w[1] & 0xFFFFu) != 1u)
    return false;
  const uint32_t ndim = h[7];
  if (ndim < 1 || ndim > (uint32_t)kMaxDims) return false;
  uint64_t n = 1;
  for (uint32_t k = 0; k < ndim; k++) {
    const uint64_t e = d[1 + k];
    if (e == 0 || e > kMaxPoints || n > kMaxPoints / e) return false;
    n *= e;
  }
  const uint32_t radius = w[16], chunk = w[17];
  K = w[20];
  unpred = d[9];
  words = d[11];
  if (radius < 1 || radius > kMaxRadius || chunk == 0 || K == 0 || K > 2 * radius) return false;
  nsym = 2 * radius;
  nch = (n + chunk - 1) / chunk;
  off_chunk = kHeaderBytes + pad8(4ull * K);
  return nch <= cap && off_chunk + 8 * nch <= stream_size;
}

static hipError_t launch_scan2(const PairScan& p, hipStream_t st) {
  uint64_t nb = (p.n + kScanPerBlock - 1) / kScanPerBlock;
  if (nb == 0) nb = 1;
  hipLaunchKernelGGL(k_scan2_reduce, dim3((unsigned)nb), dim3(256), 0, st, p);
  hipLaunchKernelGGL(k_scan2_blocks, dim3(1), dim3(1024), 0, st, p, nb);
  if (p.n) hipLaunchKernelGGL(k_scan2_apply, dim3((unsigned)nb), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_scan_pair(const uint32_t* a, const uint32_t* b, uint64_t n, uint64_t* a_off,
                            uint64_t* b_off, uint64_t* block_sums, uint64_t* a_total,
                            uint64_t* b_total, hipStream_t st) {
  PairScan p{a, b, 1u, n, nullptr, nullptr, a_off, b_off, block_sums, a_total, b_total, 0, 0,
             nullptr};
  return launch_scan2(p, st);
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

// Build the canonical decoding tables from the stored (symbol, length) list:
// validate it (ascending symbols, lengths 1..64, a complete prefix code),
// order it by (length, symbol), and fill a lookup table indexed by the next
// kLutBits bits for codes no longer than that.
//
// Up to kDtLdsCap coded symbols the list is handled in LDS: a symbol's place
// in (length, symbol) order is its length's offset plus the number of
// smaller symbols of the same length (counted a wave at a time with
// ballots), and each lookup entry finds the short code covering it by a
// binary search over the left-justified code starts, which ascend and tile
// the table from 0.  Longer lists take a radix sort in global scratch.
constexpr uint32_t kDtLdsCap = 2048;

__device__ bool check_lengths(const uint32_t* bl, uint32_t K) {
  // complete prefix code: pairing nodes from the deepest level up must leave
  // exactly the root (a lone symbol must have length 1)
  if (K == 1) return bl[1] == 1;
  uint64_t carry = 0;
  for (int l = kMaxCodeLen; l >= 1; l--) {
    const uint64_t nodes = bl[l] + carry;
    if (nodes & 1) return false;
    carry = nodes >> 1;
  }
  return carry == 1;
}

// The chunk decoder's view of the codes longer than the lookup table, from
// the per-length counts, first codes and offsets (a thread per length).
__device__ __forceinline__ void long_codes(uint32_t K, const uint32_t* bl, const uint64_t* first,
                                           const uint32_t* off, LongCodes* lc) {
  __shared__ uint32_t maxl, l0;
  const uint32_t t = threadIdx.x;
  if (t == 0) {
    maxl = 0;
    l0 = 33;
  }
  __syncthreads();
  if (t >= 1 && t <= (uint32_t)kMaxCodeLen && bl[t]) atomicMax(&maxl, t);
  __syncthreads();
  const uint32_t ml = maxl;
  const uint32_t lf = (uint32_t)kLutBits < ml ? off[kLutBits + 1] : K;
  // A window of a long code reaches the end of length l when win >= end32(l),
  // end32(l) = (first[l] + count[l]) << (32 - l) in [0, 2^32], nondecreasing
  // in l.  Ends that are 0 (no code of length <= l) are always reached and
  // are folded into l0; the rest compare as win > end32 - 1 in 32 bits, and
  // the ends past length 32 are never reached (limit 2^32 - 1), so the
  // count gives 33 exactly for codes longer than 32 bits.
  if (t > (uint32_t)kLutBits && t <= 32 && (t >= ml || first[t] + bl[t] != 0)) atomicMin(&l0, t);
  if (t >= 1 && t <= (uint32_t)kMaxCodeLen) {
    lc->base[t] = (uint64_t)off[t] - first[t];
    lc->end_lj[t] = t < (uint32_t)kMaxCodeLen ? (first[t] + bl[t]) << (64 - t) : ~0ull;
  }
  if (t <= 33)
    lc->base32[t] = t > (uint32_t)kLutBits && t <= 32 ? off[t] - (uint32_t)first[t] - lf : 0u;
  if (t == 0) {
    lc->end_lj[0] = 0;
    lc->base[0] = 0;
    lc->max_len = ml;
    lc->long_first = lf;
    lc->long_in_lds = K - lf <= kLongSymCap;
    lc->pad = 0;
  }
  __syncthreads();
  const uint32_t L0 = l0 < 33 ? l0 : 33;
  if (t == 0) lc->l0 = L0;
  if (t < (uint32_t)kWinLens) {
    const uint32_t l = L0 + t;
    uint64_t e = 1ull << 32;
    if (l <= 32 && l < ml) e = (first[l] + bl[l]) << (32 - l);
    lc->lim[t] = (uint32_t)(e - 1);
  }
}

// Multi-symbol table: for every kLutBits-bit window, the whole codes it holds
// from its start, up to three, with their symbols and the bits they end at
// (each found by a lookup of the window shifted past the codes before it; a
// code that fits the remaining bits is decided by them alone).  An entry
// stops before a second or third code of symbol 0, so that only its first
// symbol can be an unpredictable value.  Count 0: the first code is longer
// than the window.  Called by every thread.
constexpr uint32_t kMultiSyms = 3;
__device__ __forceinline__ uint64_t multi_entry(uint32_t c, const uint32_t (&sym)[kMultiSyms],
                                                const uint32_t (&end)[kMultiSyms]) {
  return (uint64_t)sym[0] | ((uint64_t)sym[1] << 16) | ((uint64_t)sym[2] << 32) |
         ((uint64_t)c << 48) | ((uint64_t)end[0] << 50) | ((uint64_t)end[1] << 54) |
         ((uint64_t)end[2] << 58);
}
__device__ void multi_symbol_table(DecodeTables d) {
  __syncthreads();  // the single-code table is complete
  for (uint32_t x = threadIdx.x; x < (1u << kLutBits); x += blockDim.x) {
    uint32_t sym[kMultiSyms] = {0, 0, 0}, end[kMultiSyms] = {0, 0, 0}, c = 0, pos = 0;
    for (uint32_t j = 0; j < kMultiSyms; j++) {
      const uint32_t e = d.lut[(x << pos) & ((1u << kLutBits) - 1)];
      const uint32_t l = e >> 16;
      if (l == 0 || pos + l > (uint32_t)kLutBits || (j > 0 && (e & 0xFFFFu) == 0)) break;
      sym[j] = e & 0xFFFFu;
      pos += l;
      end[j] = pos;
      c++;
    }
    d.lut2[x] = multi_entry(c, sym, end);
  }
}

// Second level for the windows that begin long codes.  With canonical codes
// the short codes fill the table windows [0, p0), p0 = first[kLutBits] +
// count[kLutBits], and every later window begins codes longer than the table.
// Block i serves window p0 + i: its entry y is the code that starts with that
// window followed by the kL2Bits bits of y, found among the lengths up to
// kLutBits + kL2Bits by its left-justified range.  The multi-symbol entries of
// the long windows point to their blocks.  Called by every thread once the
// single-code table has been read.
__device__ void second_level(DecodeTables d, const uint32_t* bl, const uint64_t* firsts,
                             const uint32_t* offs) {
  __syncthreads();
  const uint32_t p0 = (uint32_t)(firsts[kLutBits] + bl[kLutBits]);
  for (uint32_t e = threadIdx.x; e < kL2Prefixes * kL2Entries; e += blockDim.x) {
    const uint32_t p = p0 + e / kL2Entries;
    uint32_t ent = 0;
    if (p < (1u << kLutBits)) {
      const uint64_t v = ((uint64_t)p << (32 - kLutBits)) |
                         ((uint64_t)(e % kL2Entries) << (32 - kLutBits - kL2Bits));
      for (uint32_t l = kLutBits + 1; l <= kLutBits + kL2Bits; l++) {
        const uint64_t lo = firsts[l] << (32 - l), hi = (firsts[l] + bl[l]) << (32 - l);
        if (bl[l] && v >= lo && v < hi) {
          ent = (uint32_t)d.sorted_sym[offs[l] + (uint32_t)((v >> (32 - l)) - firsts[l])] | (l << 16);
          break;
        }
      }
    }
    d.l2[e] = ent;
  }
  for (uint32_t p = p0 + threadIdx.x; p < (1u << kLutBits); p += blockDim.x)
    d.lut2[p] = p - p0 < kL2Prefixes ? p - p0 : 0xFFFFu;
}

__global__ __launch_bounds__(kCbThreads) void k_decode_tables(const uint8_t* __restrict__ stream,
                                                              uint64_t off_sym, uint32_t K,
                                                              uint32_t nsym, DecodeTables d,
                                                              Meta* m, PairScan scan,
                                                              uint64_t hdr_size, uint64_t cap,
                                                              uint32_t nsb, uint64_t pf_bytes) {
  __shared__ union {
    uint32_t cnt[16 * kCbThreads];  // radix-sort table of the global path
    struct {
      uint32_t e[kDtLdsCap];        // stored entries, symbol order
      uint32_t lj[kDtLdsCap];       // left-justified start of each short code, sorted order
      uint32_t val[kDtLdsCap];      // lookup value of each short code, sorted order
    } s;
  } u;
  __shared__ uint32_t sh16[16];
  __shared__ uint32_t bl[kMaxCodeLen + 2], run[kMaxCodeLen + 2], offs[kMaxCodeLen + 2];
  __shared__ uint64_t firsts[kMaxCodeLen + 2];
  __shared__ uint32_t bad;
  __shared__ uint64_t sh64[16];
  if (blockIdx.x > nsb) {  // the stream's prefetch
    prefetch_stream(stream, pf_bytes, blockIdx.x - 1 - nsb, gridDim.x - 1 - nsb, m);
    return;
  }
  if (hdr_size) {  // the parameters from the header in device memory
    __shared__ uint32_t sk, sn, sok;
    __shared__ uint64_t soff, snch, swords, sunp;
    if (threadIdx.x == 0) {
      uint32_t k_ = 0, n_ = 0;
      uint64_t off_ = 0, nch_ = 0, w_ = 0, u_ = 0;
      sok = front_from_header(stream, hdr_size, cap, k_, n_, off_, nch_, w_, u_) ? 1u : 0u;
      sk = k_;
      sn = n_;
      soff = off_;
      snch = nch_;
      swords = w_;
      sunp = u_;
    }
    __syncthreads();
    if (!sok) return;
    K = sk;
    nsym = sn;
    off_sym = kHeaderBytes;
    const uint32_t* tab = reinterpret_cast<const uint32_t*>(stream + soff);
    scan.a = tab;
    scan.b = tab + 1;
    scan.n = snch;
    scan.want_a = swords;
    scan.want_b = sunp;
  }
  if (blockIdx.x > 0) {  // slices of the chunk table's scans
    scan_slices(scan, nsb, sh64);
    return;
  }
  const uint32_t T = blockDim.x, t = threadIdx.x;
  if (t <= kMaxCodeLen + 1) {
    bl[t] = 0;
    run[t] = 0;
  }
  if (t == 0) bad = 0;
  const uint32_t* tab = reinterpret_cast<const uint32_t*>(stream + off_sym);
  const bool in_lds = K <= kDtLdsCap;
  if (in_lds)
    for (uint32_t i = t; i < K; i += T) u.s.e[i] = tab[i];
  __syncthreads();
  for (uint32_t i = t; i < K; i += T) {
    const uint32_t e = in_lds ? u.s.e[i] : tab[i];
    const uint32_t sym = e & 0xFFFF, len = e >> 16;
    bool ok = sym < nsym && len >= 1 && len <= kMaxCodeLen;
    if (i > 0 && ((in_lds ? u.s.e[i - 1] : tab[i - 1]) & 0xFFFF) >= sym) ok = false;
    if (!ok) {
      bad = 1;
    } else {
      atomicAdd(&bl[len], 1u);
      if (!in_lds) d.keys_a[i] = ((uint64_t)len << 16) | sym;
    }
  }
  __syncthreads();
  if (t == 0) {
    if (!bad && K > 0 && !check_lengths(bl, K)) bad = 1;
    uint64_t code = 0;
    uint32_t off = 0;
    for (int l = 1; l <= kMaxCodeLen; l++) {
      code = (code + (l > 1 ? bl[l - 1] : 0)) << 1;
      d.first[l] = code;
      d.count[l] = bl[l];
      d.offset[l] = off;
      firsts[l] = code;
      offs[l] = off;
      off += bl[l];
    }
    if (bad) atomicOr(&m->status, kStatusCorrupt);
  }
  for (uint32_t i = t; i < (1u << kLutBits); i += T) d.lut[i] = 0;
  __syncthreads();
  if (bad || K == 0) return;
  long_codes(K, bl, firsts, offs, d.lc);
  if (!in_lds) {
    __syncthreads();  // the lookup table is cleared before it is filled
    uint64_t* bylen = block_radix_sort(d.keys_a, d.keys_b, K, 16, 24, u.cnt, sh16);
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
    multi_symbol_table(d);
    second_level(d, bl, firsts, offs);
    return;
  }
  // (length, symbol) order, a wave of symbols at a time
  if (t < 64) {
    const uint32_t lane = t;
    for (uint32_t base = 0; base < K; base += 64) {
      const uint32_t i = base + lane;
      const bool valid = i < K;
      const uint32_t e = valid ? u.s.e[i] : 0u;
      const uint32_t l = e >> 16, sym = e & 0xFFFF;
      uint64_t same = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 7; bit++) {
        const bool on = (l >> bit) & 1u;
        const uint64_t bb = __ballot(on);
        same &= on ? bb : ~bb;
      }
      const uint32_t below = (uint32_t)__popcll(same & ((1ull << lane) - 1));
      const uint32_t before = valid ? run[l] : 0u;
      __builtin_amdgcn_wave_barrier();
      if (valid) {
        const uint32_t r = before + below, pos = offs[l] + r;
        d.sorted_sym[pos] = (uint16_t)sym;
        if (l <= (uint32_t)kLutBits) {
          u.s.lj[pos] = (uint32_t)((firsts[l] + r) << (kLutBits - l));
          u.s.val[pos] = sym | (l << 16);
        }
        if ((same >> lane) == 1ull) run[l] = before + (uint32_t)__popcll(same);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  // lookup table: entry x holds the short code whose range covers it
  const uint32_t nshort = offs[kLutBits + 1];
  if (nshort > 0) {
    const uint32_t last = nshort - 1;
    const uint32_t end = u.s.lj[last] + (1u << (kLutBits - (u.s.val[last] >> 16)));
    for (uint32_t x = t; x < end; x += T) {
      uint32_t lo = 0, hi = last;  // largest j with lj[j] <= x
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (u.s.lj[mid] <= x)
          lo = mid;
        else
          hi = mid - 1;
      }
      d.lut[x] = u.s.val[lo];
    }
  }
  multi_symbol_table(d);
  second_level(d, bl, firsts, offs);
}

static unsigned slice_blocks(uint64_t nchunks) {
  const uint64_t ns = (nchunks + kSliceEntries - 1) / kSliceEntries;
  return (unsigned)(ns < kSliceBlocks ? ns : kSliceBlocks);
}
static unsigned prefetch_blocks(uint64_t bytes) {
  const uint64_t nb = (bytes + (64u << 10) - 1) / (64u << 10);  // at least 64 KiB a block
  return (unsigned)(nb < kPrefetchBlocks ? nb : kPrefetchBlocks);
}

hipError_t launch_decode_front(const uint8_t* stream, uint64_t stream_bytes, uint64_t off_sym,
                               uint32_t nsym_used,
                               uint32_t nsym, DecodeTables t, uint64_t off_chunk, uint64_t nchunks,
                               uint32_t* chunk_words, uint32_t* chunk_unpred, uint64_t* word_off,
                               uint64_t* unpred_off, uint64_t* block_sums, uint64_t* totals,
                               uint64_t total_words, uint64_t n_unpred, Meta* m, hipStream_t st) {
  // the chunk table's (words, unpredictable) pairs are read in place, copied
  // out for the decoder, scanned, and their totals checked
  const uint32_t* tab = reinterpret_cast<const uint32_t*>(stream + off_chunk);
  PairScan p{tab, tab + 1, 2u, nchunks, chunk_words, chunk_unpred, word_off, unpred_off,
             block_sums, totals, totals + 1, total_words, n_unpred, m};
  const unsigned nsb = slice_blocks(nchunks), npb = prefetch_blocks(stream_bytes);
  hipLaunchKernelGGL(k_decode_tables, dim3(1 + nsb + npb), dim3(kCbThreads), 0, st, stream,
                     off_sym, nsym_used, nsym, t, m, p, 0ull, 0ull, nsb, stream_bytes);
  return hipGetLastError();
}

hipError_t launch_decode_front_early(const uint8_t* stream, uint64_t stream_size, uint64_t cap,
                                     DecodeTables t, uint32_t* chunk_words, uint32_t* chunk_unpred,
                                     uint64_t* word_off, uint64_t* unpred_off,
                                     uint64_t* block_sums, uint64_t* totals, Meta* m,
                                     hipStream_t st) {
  if (cap == 0 || stream_size < kHeaderBytes) return hipErrorInvalidValue;
  PairScan p{nullptr, nullptr, 2u, 0, chunk_words, chunk_unpred, word_off, unpred_off,
             block_sums, totals, totals + 1, 0, 0, m};
  const unsigned nsb = slice_blocks(cap), npb = prefetch_blocks(stream_size);
  hipLaunchKernelGGL(k_decode_tables, dim3(1 + nsb + npb), dim3(kCbThreads), 0, st, stream,
                     kHeaderBytes, 0u, 0u, t, m, p, stream_size, cap, nsb, stream_size);
  return hipGetLastError();
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


// Decoding loop.  Each lane decodes one sub-chunk: a run of C/S symbols of a
// chunk whose starting bit offset the stream's sub-chunk table gives (S lanes
// share a chunk; S = 1 is the whole chunk).  The window `buf` holds the next
// `nb` stream bits left-aligned and the word `nxt` (index rd) follows them:
// used + nb == 32 * rd, with `used` counted from the chunk's first bit.
// Before every symbol at least 32 bits are present, which covers every code
// of up to 32 bits; a refill appends `nxt`, loaded one refill earlier, so its
// latency hides behind the symbols decoded in between.  Word reads are
// clamped to the bit-stream section instead of being masked: bits past the
// chunk's own words never decide a code of a well-formed chunk, and a run
// that ends anywhere but where the next one starts (or, for the last run,
// inside the chunk's last word) is detected once, from the bits consumed.
constexpr uint32_t kGroup = 32;               // codes staged in LDS per lane

struct RunResult {
  uint64_t used;   // bit offset, from the chunk's first bit, where the run ended
  uint32_t zeros;  // unpredictable symbols (code 0) in the run
};

// A lane's next stream words are staged in an LDS ring of kRing words,
// fetched kPre at a time at group boundaries (every lane passes them at the
// same symbol counts): the loads issued at one boundary are written to the
// ring at the next, a group of symbols later, so refills read the ring and
// never wait on memory while the lane stays within kPre words (256 bits) per
// group.  A lane that runs ahead reads the stream directly (taking the load
// inside the branch, so that the common path never waits on it).  The codes
// of a group are stored at the next boundary, before the next fetch: the wait
// for a fetch then only covers stores issued before it, a group earlier.
constexpr uint32_t kRing = 16;  // staged words per lane
constexpr uint32_t kPre = 8;    // words fetched per lane per group

// Decodes symbols [beg, end) starting at bit `start` of the chunk's words,
// writes their codes, and lists the offsets (from beg) of the code-0 symbols
// as u32 words at `zlist`, in increasing order.  ring: this lane's column of
// the ring (slot i at ring[i * nt]).
template <bool LONG_LDS>
__device__ __forceinline__ RunResult decode_run(
    const uint32_t* __restrict__ words, uint32_t wlast, uint32_t nt, const uint64_t* lut2,
    const LongCodes& lc, const uint32_t l0, const uint32_t (&lim)[kWinLens], const uint16_t* long_sym,
    const uint16_t* __restrict__ sorted_sym, const uint32_t* l2, uint16_t* stage, uint32_t* ring,
    uint64_t beg, uint64_t end, uint32_t start, uint32_t chunk, uint16_t* codes, uint32_t* zlist) {
  auto ld = [&](uint32_t i) { return words[i < wlast ? i : wlast]; };
  uint32_t zeros = 0;
  uint64_t used = start;
  const uint32_t wi0 = start >> 5, o0 = start & 31;
  uint32_t w0 = ld(wi0), w1 = ld(wi0 + 1);
  asm volatile("" : "+v"(w0), "+v"(w1));
  uint64_t buf = (((uint64_t)w0 << 32) | w1) << o0;
  uint32_t nb = 64 - o0, rd = wi0 + 2;
  uint32_t avail = rd;  // words [rd, avail) are in the ring
  uint32_t q[kPre];     // words [qp, qp + kPre), in flight since the last boundary
  uint32_t qp = rd;
  bool qwant = true;
#pragma unroll
  for (uint32_t k = 0; k < kPre; k++) q[k] = ld(qp + k);
  const bool vec = (chunk & 31) == 0;  // every run then starts on a 32-symbol boundary
  auto flush = [&](uint64_t g, uint32_t cnt) {
    if (vec && cnt == kGroup) {  // g is a multiple of 32 symbols: 64-byte aligned
      uint4* dst = reinterpret_cast<uint4*>(codes + g);
#pragma unroll
      for (int j = 0; j < (int)(kGroup / 8); j++) {
        uint32_t v[4];
#pragma unroll
        for (int h = 0; h < 4; h++)
          v[h] = (uint32_t)stage[(8 * j + 2 * h) * nt] |
                 ((uint32_t)stage[(8 * j + 2 * h + 1) * nt] << 16);
        dst[j] = make_uint4(v[0], v[1], v[2], v[3]);
      }
    } else {
      for (uint32_t j = 0; j < cnt; j++) codes[g + j] = stage[j * nt];
    }
  };
  uint64_t prev_g = beg;
  uint32_t prev_cnt = 0;
  for (uint64_t g = beg; g < end; g += kGroup) {
    // the words fetched at the last boundary into the ring
#pragma unroll
    for (uint32_t k = 0; k < kPre; k++) asm volatile("" ::"v"(q[k]));
    if (qwant) {
#pragma unroll
      for (uint32_t k = 0; k < kPre; k++) ring[((qp + k) & (kRing - 1)) * nt] = q[k];
      avail = qp + kPre;
    }
    if (prev_cnt) flush(prev_g, prev_cnt);
    // the next words, if the ring has room for them
    qp = avail > rd ? avail : rd;
    qwant = qp + kPre <= rd + kRing;
#pragma unroll
    for (uint32_t k = 0; k < kPre; k++) q[k] = ld(qp + k);

    const uint32_t cnt = (uint32_t)(end - g < kGroup ? end - g : kGroup);
    uint32_t zmask = 0;  // positions of unpredictable values in this group
    for (uint32_t k = 0; k < cnt;) {
      // the word after the window, read from the ring beside the lookup: the
      // refill below takes it without a second wait
      const uint32_t wr = ring[(rd & (kRing - 1)) * nt];
      // up to three whole codes of the next kLutBits bits at once; the
      // symbols past the group's end are written to the spare stage slots
      // and not counted
      const uint64_t e2 = lut2[(uint32_t)(buf >> (64 - kLutBits))];
      const uint32_t c = (uint32_t)(e2 >> 48) & 3u;
      if (c) {
        const uint32_t rem = cnt - k, mm = c < rem ? c : rem;
        const uint32_t s0 = (uint32_t)e2 & 0xFFFFu, s1 = (uint32_t)(e2 >> 16) & 0xFFFFu,
                       s2 = (uint32_t)(e2 >> 32) & 0xFFFFu;
        const uint32_t bits = mm == 1 ? (uint32_t)(e2 >> 50) & 15u
                                      : (mm == 2 ? (uint32_t)(e2 >> 54) & 15u : (uint32_t)(e2 >> 58) & 15u);
        stage[k * nt] = (uint16_t)s0;
        stage[(k + 1) * nt] = (uint16_t)s1;
        stage[(k + 2) * nt] = (uint16_t)s2;
        zmask |= (s0 == 0 ? 1u : 0u) << k;  // a later code of an entry is never 0
        used += bits;
        buf <<= bits;
        nb -= bits;
        k += mm;
      } else {  // a code longer than the table: its window's second level
        uint32_t sym, len;
        const uint32_t blk = (uint32_t)e2 & 0xFFFFu;
        const uint32_t ent =
            blk < kL2Prefixes
                ? l2[blk * kL2Entries + ((uint32_t)(buf >> (64 - kLutBits - kL2Bits)) & (kL2Entries - 1))]
                : 0u;
        if (ent >> 16) {  // a code of at most kLutBits + kL2Bits bits
          sym = ent & 0xFFFFu;
          len = ent >> 16;
          used += len;
          buf <<= len;
          nb -= len;
        } else {  // longer, or past the second level's windows: the window limits
          const uint32_t win = (uint32_t)(buf >> 32);
          uint32_t l = l0;
#pragma unroll
          for (int qq = 0; qq < kWinLens; qq++) l += win > lim[qq] ? 1u : 0u;
          if (l <= 32) {
            const uint32_t idx = lc.base32[l] + (win >> (32 - l));
            sym = LONG_LDS ? long_sym[idx] : sorted_sym[idx + lc.long_first];
            len = l;
            used += len;
            buf <<= len;
            nb -= len;
          } else {  // longer than 32 bits: exact read of the next 64 bits
            const uint32_t wi = (uint32_t)(used >> 5), o = (uint32_t)(used & 31);
            uint32_t a = ld(wi), b = ld(wi + 1), cc = ld(wi + 2);
            asm volatile("" : "+v"(a), "+v"(b), "+v"(cc));
            uint64_t w64 = ((uint64_t)a << 32) | b;
            if (o) w64 = (w64 << o) | (cc >> (32 - o));
            l = 33;
            for (uint32_t qq = 33; qq < lc.max_len; qq++) l += w64 >= lc.end_lj[qq] ? 1u : 0u;
            const uint32_t idx = (uint32_t)(lc.base[l] + (w64 >> (64 - l)));
            // a 32-bit read, so that this rare load is never merged with the
            // table reads above into one generic-address load
            uint32_t pair = reinterpret_cast<const uint32_t*>(sorted_sym)[idx >> 1];
            asm volatile("" : "+v"(pair));
            sym = (pair >> (16 * (idx & 1))) & 0xFFFFu;
            len = l;
            used += len;
            const uint32_t o2 = (uint32_t)(used & 31), w2 = (uint32_t)(used >> 5);
            uint32_t dd = ld(w2), f = ld(w2 + 1);
            asm volatile("" : "+v"(dd), "+v"(f));
            // the window restarts left-aligned at bit `used`: drop the o2 bits of
            // word w2 already consumed
            buf = (((uint64_t)dd << 32) | f) << o2;
            nb = 64 - o2;
            rd = w2 + 2;
          }
        }
        stage[k * nt] = (uint16_t)sym;
        zmask |= (sym == 0 ? 1u : 0u) << k;
        k++;
      }
      if (nb < 32) {  // append the next word: from the ring, or read directly
        uint32_t wv;
        if (rd < avail) {
          wv = wr;
        } else {
          wv = ld(rd);
          asm volatile("" : "+v"(wv));
        }
        buf |= (uint64_t)wv << (32 - nb);
        nb += 32;
        rd++;
      }
    }
    while (zmask) {
      const uint32_t k = __builtin_ctz(zmask);
      zmask &= zmask - 1;
      zlist[zeros++] = (uint32_t)(g + k - beg);
    }
    prev_g = g;
    prev_cnt = cnt;
  }
  if (prev_cnt) flush(prev_g, prev_cnt);
#pragma unroll
  for (uint32_t k = 0; k < kPre; k++) asm volatile("" ::"v"(q[k]));
  return RunResult{used, zeros};
}

// One lane per sub-chunk; the S lanes of a chunk are adjacent in a wave.
// The unpredictable values of a chunk are stored in flat order, so a lane's
// first one is the chunk's base plus the code-0 count of the lanes before
// it, known only after decoding: each lane lists its code-0 offsets in its
// own slice of the output (the slots of its run, which the values overwrite
// later), the counts are scanned across the S lanes, and the values are then
// scattered from the last listed offset down, so that a value never lands on
// a list entry still to be read (the j-th code-0 position is at least j
// slots past the run's start, above the slot of entry j and all earlier ones).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_decode_chunks(
    const uint8_t* __restrict__ stream, uint64_t off_sub, uint64_t off_unpred, uint64_t off_bits,
    uint64_t total_words, uint64_t n_unpred, uint64_t n, uint32_t chunk, uint32_t sub,
    uint64_t nchunks, uint32_t nsym_used, const uint32_t* __restrict__ chunk_words,
    const uint32_t* __restrict__ chunk_unpred, const uint64_t* __restrict__ word_off,
    const uint64_t* __restrict__ unpred_off, const uint64_t* __restrict__ carry, uint64_t nslices,
    DecodeTables d, uint16_t* codes, T* out, Meta* m) {
  __shared__ __align__(16) uint64_t lut2[1u << kLutBits];
  __shared__ LongCodes lc;
  __shared__ uint16_t long_sym[kLongSymCap];
  __shared__ uint16_t stage_all[NT * (kGroup + 2)];  // two spare slots per lane
  __shared__ uint32_t ring_all[NT * kRing];
  __shared__ uint32_t l2[kL2Prefixes * kL2Entries];
  uint16_t* stage = stage_all + threadIdx.x;
  uint32_t* ring = ring_all + threadIdx.x;
  {
    // lookup table and long-code tables: independent loads, all in flight at once
    constexpr uint32_t kLutVecs = (1u << kLutBits) / 2 / NT;
    const uint4* src = reinterpret_cast<const uint4*>(d.lut2);
    uint4 v[kLutVecs];
#pragma unroll
    for (uint32_t j = 0; j < kLutVecs; j++) v[j] = src[threadIdx.x + j * NT];
    constexpr uint32_t kLcWords = sizeof(LongCodes) / 4;
    static_assert(sizeof(LongCodes) % 4 == 0, "LongCodes is copied as words");
    uint32_t lw[(kLcWords + NT - 1) / NT];
#pragma unroll
    for (uint32_t j = 0; j < (kLcWords + NT - 1) / NT; j++) {
      const uint32_t i = threadIdx.x + j * NT;
      lw[j] = i < kLcWords ? reinterpret_cast<const uint32_t*>(d.lc)[i] : 0u;
    }
    constexpr uint32_t kL2Words = kL2Prefixes * kL2Entries;
    uint32_t l2w[(kL2Words + NT - 1) / NT];
#pragma unroll
    for (uint32_t j = 0; j < (kL2Words + NT - 1) / NT; j++) {
      const uint32_t i = threadIdx.x + j * NT;
      l2w[j] = i < kL2Words ? d.l2[i] : 0u;
    }
#pragma unroll
    for (uint32_t j = 0; j < kLutVecs; j++) reinterpret_cast<uint4*>(lut2)[threadIdx.x + j * NT] = v[j];
#pragma unroll
    for (uint32_t j = 0; j < (kLcWords + NT - 1) / NT; j++) {
      const uint32_t i = threadIdx.x + j * NT;
      if (i < kLcWords) reinterpret_cast<uint32_t*>(&lc)[i] = lw[j];
    }
#pragma unroll
    for (uint32_t j = 0; j < (kL2Words + NT - 1) / NT; j++) {
      const uint32_t i = threadIdx.x + j * NT;
      if (i < kL2Words) l2[i] = l2w[j];
    }
  }
  __syncthreads();
  if (lc.long_in_lds)
    for (uint32_t i = lc.long_first + threadIdx.x; i < nsym_used; i += blockDim.x)
      long_sym[i - lc.long_first] = d.sorted_sym[i];
  __syncthreads();
  // the window limits are the same for every lane: keep them in scalar registers
  uint32_t lim[kWinLens];
#pragma unroll
  for (int q = 0; q < kWinLens; q++) lim[q] = __builtin_amdgcn_readfirstlane(lc.lim[q]);
  const uint32_t l0 = __builtin_amdgcn_readfirstlane(lc.l0);
  const uint32_t lg = __builtin_ctz(sub);
  const uint64_t tg = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t c = tg >> lg;
  const uint32_t k = (uint32_t)(tg & (sub - 1));
  // S divides the block size, so the lanes of a chunk leave together
  if (c >= nchunks || m->status) return;
  // the offsets within the chunk's slice of the table plus the slice's carries
  const uint64_t sl = c / kSliceEntries;
  const uint64_t W = chunk_words[c], wbase = word_off[c] + carry[sl];
  const uint64_t uexp = chunk_unpred[c], ubase = unpred_off[c] + carry[nslices + sl];
  // a non-empty chunk holds at least one bit; its words and unpredictable
  // values must lie inside their sections (the same verdict for all S lanes)
  if (W == 0 || wbase + W > total_words || ubase + uexp > n_unpred) {
    atomicOr(&m->status, kStatusCorrupt);
    return;
  }
  const uint32_t* sub_bits = reinterpret_cast<const uint32_t*>(stream + off_sub) + c * (sub - 1);
  const uint32_t start = k ? sub_bits[k - 1] : 0u;
  const uint32_t next = k + 1 < sub ? sub_bits[k] : 0u;
  const uint32_t* words = reinterpret_cast<const uint32_t*>(stream + off_bits) + wbase;
  const uint64_t avail = total_words - wbase;  // >= W >= 1
  const uint32_t wlast = (uint32_t)((avail < W + 2 ? avail : W + 2) - 1);
  const uint64_t span = chunk >> lg;
  const uint64_t cend = c * chunk + chunk < n ? c * chunk + chunk : n;
  const uint64_t beg0 = c * chunk + k * span;
  const uint64_t beg = beg0 < cend ? beg0 : cend, end = beg + span < cend ? beg + span : cend;
  uint32_t* zlist = reinterpret_cast<uint32_t*>(out + beg);
  const RunResult res =
      lc.long_in_lds
          ? decode_run<true>(words, wlast, NT, lut2, lc, l0, lim, long_sym, d.sorted_sym, l2, stage,
                             ring, beg, end, start, chunk, codes, zlist)
          : decode_run<false>(words, wlast, NT, lut2, lc, l0, lim, long_sym, d.sorted_sym, l2, stage,
                              ring, beg, end, start, chunk, codes, zlist);
  bool bad = k + 1 < sub ? res.used != next : (res.used + 31) / 32 != W;
  // exclusive scan of the code-0 counts over the chunk's S lanes
  uint32_t incl = res.zeros;
  for (uint32_t dlt = 1; dlt < sub; dlt <<= 1) {
    const uint32_t v = __shfl_up(incl, dlt, sub);
    if (k >= dlt) incl += v;
  }
  const uint32_t total = __shfl(incl, sub - 1, sub);
  if (total != uexp) bad = true;
  if (bad) {
    atomicOr(&m->status, kStatusCorrupt);
    return;
  }
  const T* unpred = reinterpret_cast<const T*>(stream + off_unpred) + ubase + (incl - res.zeros);
  for (uint32_t j = res.zeros; j-- > 0;) {
    out[beg + zlist[j]] = unpred[j];
    // the list is read as u32 and the values stored as T: keep each store
    // behind the list reads before it
    asm volatile("" ::: "memory");
  }
}

hipError_t launch_decode_chunks(const uint8_t* stream, uint64_t stream_size, uint64_t off_sub,
                                uint64_t off_unpred, uint64_t off_bits, uint64_t total_words,
                                uint64_t n_unpred, uint64_t n, uint32_t chunk, uint32_t sub,
                                uint32_t nsym_used, int dtype, const uint32_t* chunk_words,
                                const uint32_t* chunk_unpred, const uint64_t* word_off,
                                const uint64_t* unpred_off, const uint64_t* carry, DecodeTables t,
                                uint16_t* codes, void* out, Meta* m, hipStream_t st) {
  (void)stream_size;
  const uint64_t nchunks = (n + chunk - 1) / chunk;
  const uint64_t nslices = (nchunks + kSliceEntries - 1) / kSliceEntries;
  if (nchunks == 0) return hipSuccess;
  if (!valid_sub(chunk, sub)) return hipErrorInvalidValue;
  const uint64_t lanes = nchunks * sub;
  // 64-lane blocks when there are few runs, so every CU gets work
  const bool small = lanes < 256ull * 256;  // fewer than one 256-lane block per CU
  const unsigned nt = small ? 64 : 256;
  dim3 grid((unsigned)((lanes + nt - 1) / nt)), block(nt);
#define SZG_DECODE_LAUNCH(TT, NTT)                                                               \
  hipLaunchKernelGGL((k_decode_chunks<TT, NTT>), grid, block, 0, st, stream, off_sub, off_unpred, \
                     off_bits, total_words, n_unpred, n, chunk, sub, nchunks, nsym_used,          \
                     chunk_words, chunk_unpred, word_off, unpred_off, carry, nslices, t, codes, \
                     (TT*)out, m)
  if (dtype == SZ_F32) {
    if (small)
      SZG_DECODE_LAUNCH(float, 64);
    else
      SZG_DECODE_LAUNCH(float, 256);
  } else {
    if (small)
      SZG_DECODE_LAUNCH(double, 64);
    else
      SZG_DECODE_LAUNCH(double, 256);
  }
#undef SZG_DECODE_LAUNCH
  return hipGetLastError();
}

}  // namespace szg
