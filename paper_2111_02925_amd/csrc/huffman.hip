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
// The codes of an error-bounded prediction residual pile up next to the
// radius R.  Each lane counts the kHistLane codes nearest R in counters of
// its own in LDS (no two lanes share an address, so the adds never collide);
// the other codes within kHistShared of R go to counters shared by the
// workgroup, code 0 (unpredictable) to a counter of its own, and codes
// further out to two overflow counters.  Each workgroup writes its counts to
// a row of partial histograms, which a second kernel sums into the
// histogram.  A workgroup whose overflow counters are not zero re-reads its
// codes and counts those far codes in a second window of kFarSlots counters
// (kFarHalf symbols on each side of the first window, in the LDS of the
// per-lane counters), stored in the far part of its row and flagged; codes
// beyond it go to the histogram with global atomics.

constexpr uint32_t kHistThreads = 256;
constexpr uint32_t kHistLane = 32;          // per-lane bins around R
constexpr uint32_t kHistShared = 4096;      // workgroup bins around R
constexpr uint32_t kHistSlots = kHistShared + 3;  // below | window | above | code 0
constexpr uint32_t kFarHalf = 4096;         // far-window symbols on each side
constexpr uint32_t kFarSlots = 2 * kFarHalf;
static_assert(kFarSlots <= kHistLane * kHistThreads, "the far window reuses the per-lane counters");
constexpr uint32_t kHistRow = kHistSlots + kFarSlots + 1;  // window | far window | far flag
constexpr uint32_t kHistVecs = 8;           // 8-code vectors per lane per tile
constexpr uint32_t kHistTile = kHistThreads * kHistVecs;  // vectors per tile
constexpr uint32_t kHistMaxBlocks = 768;

struct HistWindow {
  uint32_t plo;  // first per-lane bin
  uint32_t slo;  // first workgroup bin (slot 1)
};

__host__ __device__ inline HistWindow hist_window(uint32_t R) {
  HistWindow w;
  w.plo = R > kHistLane / 2 ? R - kHistLane / 2 : 0;
  w.slo = R > kHistShared / 2 ? R - kHistShared / 2 : 0;
  return w;
}

// slot of a code in the workgroup counters
__device__ __forceinline__ uint32_t hist_slot(uint32_t c, uint32_t slo) {
  int v = (int)c - (int)slo + 1;
  v = v < 0 ? 0 : (v > (int)kHistShared + 1 ? (int)kHistShared + 1 : v);
  return c == 0 ? kHistShared + 2 : (uint32_t)v;
}

// The far window: kFarHalf symbols below the first window, then kFarHalf
// above it.  Returns the slot of a far code, or kFarSlots beyond it.
__host__ __device__ __forceinline__ uint32_t far_slot(uint32_t c, uint32_t slo) {
  if (c < slo) return slo - c <= kFarHalf ? kFarHalf - (slo - c) : kFarSlots;
  const uint32_t d = c - (slo + kHistShared);
  return d < kFarHalf ? kFarHalf + d : kFarSlots;
}
// The symbol of a partial-row column, or 0xFFFFFFFF for none.
__host__ __device__ __forceinline__ uint32_t column_symbol(uint32_t col, uint32_t R) {
  const HistWindow hw = hist_window(R);
  if (col == kHistShared + 2) return 0;
  if (col >= 1 && col <= kHistShared) {
    // (symbol 0 is counted in its own column, never in the window)
    const uint32_t s = hw.slo + col - 1;
    return s >= 1 && s < 2 * R ? s : 0xFFFFFFFFu;
  }
  if (col < kHistSlots || col >= kHistSlots + kFarSlots) return 0xFFFFFFFFu;
  const uint32_t f = col - kHistSlots;
  uint32_t s;
  if (f < kFarHalf) {
    if (hw.slo < kFarHalf - f) return 0xFFFFFFFFu;
    s = hw.slo - (kFarHalf - f);
  } else {
    s = hw.slo + kHistShared + (f - kFarHalf);
  }
  return s >= 1 && s < 2 * R ? s : 0xFFFFFFFFu;
}

// The workgroup's counts go to its row of partial histograms, part + bid *
// kHistRow; (bid, nblk): this workgroup among the nblk that share the codes.
__device__ __forceinline__ void histogram_body(const uint16_t* __restrict__ codes, uint64_t n,
                                               uint32_t R, uint32_t* __restrict__ part,
                                               uint32_t* hist, Meta* m, uint32_t bid,
                                               uint32_t nblk) {
  __shared__ uint32_t lane_cnt[kHistLane * kHistThreads];
  __shared__ uint32_t shared_cnt[kHistSlots];
  const uint32_t t = threadIdx.x;
  const HistWindow hw = hist_window(R);
  for (uint32_t i = t; i < kHistLane * kHistThreads; i += kHistThreads) lane_cnt[i] = 0;
  for (uint32_t i = t; i < kHistSlots; i += kHistThreads) shared_cnt[i] = 0;
  __syncthreads();
  auto count = [&](uint32_t c) {
    const uint32_t d = c - hw.plo;
    uint32_t* p = d < kHistLane ? &lane_cnt[d * kHistThreads + t] : &shared_cnt[hist_slot(c, hw.slo)];
    atomicAdd(p, 1u);
  };
  const uint64_t nvec = n / 8;
  const uint4* v4 = reinterpret_cast<const uint4*>(codes);
  const uint64_t ntiles = (nvec + kHistTile - 1) / kHistTile;
  for (uint64_t tile = bid; tile < ntiles; tile += nblk) {
    const uint64_t base = tile * kHistTile + t;
    uint4 v[kHistVecs];
#pragma unroll
    for (uint32_t j = 0; j < kHistVecs; j++) {
      const uint64_t i = base + (uint64_t)j * kHistThreads;
      v[j] = i < nvec ? v4[i] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (uint32_t j = 0; j < kHistVecs; j++) {
      if (base + (uint64_t)j * kHistThreads < nvec) {
        const uint32_t w[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
#pragma unroll
        for (int h = 0; h < 4; h++) {
          count(w[h] & 0xFFFFu);
          count(w[h] >> 16);
        }
      }
    }
  }
  if (bid == 0 && t < (n & 7)) count(codes[nvec * 8 + t]);
  __syncthreads();
  // per-lane bins into the workgroup's window (rotated reads: distinct banks)
  {
    const uint32_t b = t & (kHistLane - 1), g = t / kHistLane;
    const uint32_t lanes = kHistThreads / (kHistThreads / kHistLane);
    uint32_t sum = 0;
    for (uint32_t j = 0; j < lanes; j++)
      sum += lane_cnt[b * kHistThreads + g * lanes + ((j + b) & (lanes - 1))];
    if (sum) atomicAdd(&shared_cnt[hist_slot(hw.plo + b, hw.slo)], sum);
  }
  __syncthreads();
  uint32_t* row = part + (uint64_t)bid * kHistRow;
  for (uint32_t i = t; i < kHistSlots; i += kHistThreads) row[i] = shared_cnt[i];
  const bool far_codes = (shared_cnt[0] | shared_cnt[kHistShared + 1]) != 0;
  if (t == 0) row[kHistRow - 1] = far_codes ? 1u : 0u;
  if (!far_codes) return;
  // far codes: re-read this workgroup's codes into the far window (the
  // per-lane counters, summed above, are free again)
  if (t == 0) atomicOr(&m->hist_far, 1u);
  __syncthreads();
  for (uint32_t i = t; i < kFarSlots; i += kHistThreads) lane_cnt[i] = 0;
  __syncthreads();
  auto far = [&](uint32_t c) {
    const uint32_t sl = hist_slot(c, hw.slo);
    if (sl == 0 || sl == kHistShared + 1) {
      const uint32_t f = far_slot(c, hw.slo);
      if (f < kFarSlots)
        atomicAdd(&lane_cnt[f], 1u);
      else
        atomicAdd(&hist[c], 1u);
    }
  };
  for (uint64_t tile = bid; tile < ntiles; tile += nblk)
    for (uint32_t j = 0; j < kHistVecs; j++) {
      const uint64_t i = tile * kHistTile + t + (uint64_t)j * kHistThreads;
      if (i < nvec) {
        const uint4 q = v4[i];
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
        for (int h = 0; h < 4; h++) {
          far(w[h] & 0xFFFFu);
          far(w[h] >> 16);
        }
      }
    }
  if (bid == 0 && t < (n & 7)) far(codes[nvec * 8 + t]);
  __syncthreads();
  for (uint32_t i = t; i < kFarSlots; i += kHistThreads) row[kHistSlots + i] = lane_cnt[i];
}

__global__ __launch_bounds__(kHistThreads) void k_histogram(const uint16_t* __restrict__ codes,
                                                            uint64_t n, uint32_t R,
                                                            uint32_t* __restrict__ part,
                                                            uint32_t* hist, Meta* m) {
  histogram_body(codes, n, R, part, hist, m, blockIdx.x, gridDim.x);
}

// every field of a batch: each job is a field's codes, into the field's rows
__global__ __launch_bounds__(kHistThreads) void k_b_histogram(BLaunch L) {
  BJob j;
  uint32_t local;
  if (!batch_job(L, j, local)) return;
  const BField& f = L.f[j.field];
  histogram_body(f.codes, f.n, f.R, f.hist_part, f.hist, f.m, local, j.nblk);
}

hipError_t launch_b_histogram(BLaunch L, uint32_t nwg, hipStream_t st) {
  if (nwg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_histogram, dim3(nwg), dim3(kHistThreads), 0, st, L);
  return hipGetLastError();
}

// Sums the partial rows: a workgroup takes 64 columns of 32 rows (a wave per
// 8 rows, lanes on consecutive columns) and adds its column sums to the
// histogram; far columns count only the rows flagged for them.
constexpr uint32_t kHistReduceRows = 32;

__global__ __launch_bounds__(256) void k_hist_reduce(const uint32_t* __restrict__ part,
                                                     uint32_t rows, uint32_t R, uint32_t* hist) {
  __shared__ uint32_t colsum[4][64];
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t col = blockIdx.x * 64 + lane;
  const bool far_col = col >= kHistSlots;
  const uint32_t r0 = blockIdx.y * kHistReduceRows + wv * (kHistReduceRows / 4);
  uint32_t sum = 0;
#pragma unroll
  for (uint32_t j = 0; j < kHistReduceRows / 4; j++) {
    const uint32_t r = r0 + j;
    if (r < rows && (!far_col || part[(uint64_t)r * kHistRow + kHistRow - 1]) && col < kHistRow - 1)
      sum += part[(uint64_t)r * kHistRow + col];
  }
  colsum[wv][lane] = sum;
  __syncthreads();
  if (wv == 0) {
    const uint32_t tot = colsum[0][lane] + colsum[1][lane] + colsum[2][lane] + colsum[3][lane];
    const uint32_t sym = col < kHistRow - 1 ? column_symbol(col, R) : 0xFFFFFFFFu;
    if (tot && sym != 0xFFFFFFFFu) atomicAdd(&hist[sym], tot);
  }
}

// The batch's rows: a workgroup per (field, 64 columns) sums all of the
// field's rows and stores the window's sums (no other writer touches those
// symbols) or adds the far window's nonzero sums.
__global__ __launch_bounds__(256) void k_b_hist_reduce(BLaunch L) {
  __shared__ uint32_t colsum[4][64];
  BJob j;
  uint32_t local;
  if (!batch_job(L, j, local)) return;
  const BField& f = L.f[j.field];
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t col = local * 64 + lane;
  const bool far_col = col >= kHistSlots;
  const uint32_t rows = j.flags;  // the field's histogram workgroups
  uint32_t sum = 0;
  if (col < kHistRow - 1) {
    const uint32_t* p = f.hist_part + col;
    const uint32_t* flag = f.hist_part + kHistRow - 1;
#pragma unroll 8
    for (uint32_t r = wv; r < rows; r += 4) {
      const uint32_t v = p[(uint64_t)r * kHistRow];
      const bool use = !far_col || flag[(uint64_t)r * kHistRow] != 0;
      sum += use ? v : 0u;
    }
  }
  colsum[wv][lane] = sum;
  __syncthreads();
  if (wv == 0) {
    const uint32_t tot = colsum[0][lane] + colsum[1][lane] + colsum[2][lane] + colsum[3][lane];
    const uint32_t sym = col < kHistRow - 1 ? column_symbol(col, f.R) : 0xFFFFFFFFu;
    if (sym != 0xFFFFFFFFu) {
      if (!far_col)
        f.hist[sym] = tot;
      else if (tot)
        atomicAdd(&f.hist[sym], tot);
    }
  }
}

hipError_t launch_b_hist_reduce(BLaunch L, uint32_t nwg, hipStream_t st) {
  if (nwg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_hist_reduce, dim3(nwg), dim3(256), 0, st, L);
  return hipGetLastError();
}

uint32_t hist_reduce_blocks() { return (kHistRow - 1 + 63) / 64; }
size_t hist_row_words() { return kHistRow; }

hipError_t launch_histogram(const uint16_t* codes, uint64_t n, uint32_t radius, uint32_t* part,
                            uint32_t* hist, Meta* m, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t tiles = (n / 8 + kHistTile - 1) / kHistTile;
  uint32_t blocks = (uint32_t)(tiles < kHistMaxBlocks ? tiles : kHistMaxBlocks);
  if (blocks == 0) blocks = 1;
  // a lane counts at most ceil(tiles / blocks) * 64 + 8 codes per bin, which
  // stays far below 2^32 for any field of up to 2^32 - 1 points
  hipLaunchKernelGGL(k_histogram, dim3(blocks), dim3(kHistThreads), 0, st, codes, n, radius,
                     part, hist, m);
  dim3 rgrid(hist_reduce_blocks(), (blocks + kHistReduceRows - 1) / kHistReduceRows);
  hipLaunchKernelGGL(k_hist_reduce, rgrid, dim3(256), 0, st, part, blocks, radius, hist);
  return hipGetLastError();
}

size_t histogram_scratch_bytes() { return sizeof(uint32_t) * (size_t)kHistMaxBlocks * kHistRow; }

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

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t x = __shfl_xor(v, o, 64);
    v = x > v ? x : v;
  }
  return v;
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t x = __shfl_xor(v, o, 64);
    v = x < v ? x : v;
  }
  return v;
}

// Compact the symbols with nonzero count (hist) or length (lens) in ascending
// symbol order; returns K.  Each wave takes a contiguous segment of the
// symbols, its lanes consecutive symbols (coalesced loads, kCompactLoads
// steps of 64 in flight: each pass over a segment is bound by the round trips
// to memory); a symbol's place is its wave's base (an exclusive scan of the
// waves' counts) plus the nonzero symbols before it in its wave, counted by
// ballots.
constexpr uint32_t kCompactLoads = 16, kCompactStep = 64 * kCompactLoads;
__device__ uint32_t compact_used(const uint32_t* hist, const uint8_t* lens, uint32_t nsym,
                                 uint64_t* keys, uint32_t* symtab, uint32_t* sh16) {
  const uint32_t T = blockDim.x, t = threadIdx.x, lane = t & 63, nw = T >> 6;
  const uint32_t seg = ((nsym + nw - 1) / nw + kCompactStep - 1) & ~(kCompactStep - 1);
  const uint32_t beg = (t >> 6) * seg < nsym ? (t >> 6) * seg : nsym;
  const uint32_t end = beg + seg < nsym ? beg + seg : nsym;
  const uint64_t below = (1ull << lane) - 1;
  auto load_step = [&](uint32_t b, uint32_t (&v)[kCompactLoads]) {
#pragma unroll
    for (int k = 0; k < (int)kCompactLoads; k++) {
      const uint32_t s = b + 64 * k + lane;
      v[k] = s < end ? (hist ? hist[s] : (uint32_t)lens[s]) : 0u;
    }
  };
  uint32_t c = 0;
  for (uint32_t b = beg; b < end; b += kCompactStep) {
    uint32_t v[kCompactLoads];
    load_step(b, v);
#pragma unroll
    for (int k = 0; k < (int)kCompactLoads; k++) c += (uint32_t)__popcll(__ballot(v[k] != 0));
  }
  uint32_t K;
  const uint32_t ex = block_excl_scan_u32(lane == 0 ? c : 0u, sh16, &K);
  uint32_t pos = __shfl(ex, 0, 64);  // the waves before this one
  for (uint32_t b = beg; b < end; b += kCompactStep) {
    uint32_t v[kCompactLoads];
    load_step(b, v);
#pragma unroll
    for (int k = 0; k < (int)kCompactLoads; k++) {
      const uint64_t bal = __ballot(v[k] != 0);
      if (v[k]) {
        const uint32_t p = pos + (uint32_t)__popcll(bal & below);
        const uint32_t s = b + 64 * k + lane;
        if (hist) {
          keys[p] = ((uint64_t)v[k] << 32) | s;
        } else {
          keys[p] = ((uint64_t)v[k] << 16) | s;
          if (symtab) symtab[p] = s | (v[k] << 16);
        }
      }
      pos += (uint32_t)__popcll(bal);
    }
  }
  __syncthreads();
  return K;
}

// Any K: the tree arrays live in global scratch.
// The node weights of the merge stay in LDS (w_lds, kCbWCap entries, sharing
// the radix sort's table) when the tree fits, so that the merge phases'
// binary searches read LDS.
constexpr uint32_t kCbWCap = 36864;

__device__ void codebook_global(const uint32_t* __restrict__ hist, uint32_t nsym,
                                CodebookScratch s, uint64_t* enc_code, uint8_t* enc_len,
                                uint32_t* symtab, Meta* m, uint32_t* cnt, uint32_t* sh16,
                                uint32_t* w_lds) {
  __shared__ uint32_t sh_li, sh_qi, sh_qn, sh_cl, sh_ci, sh_done, sh_nphase;
  __shared__ uint32_t sh_maxw, sh_maxlen;
  __shared__ uint32_t bl_count[kMaxCodeLen + 2];
  __shared__ uint64_t first_code[kMaxCodeLen + 2];
  __shared__ uint32_t len_offset[kMaxCodeLen + 2];
  const uint32_t T = blockDim.x, t = threadIdx.x;

  if (t == 0) {
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
  {  // the largest count: a wave reduction, then one LDS atomic per wave
    uint32_t mw = 0;
    for (uint32_t i = t; i < K; i += T) {
      const uint32_t c = (uint32_t)(s.keys_a[i] >> 32);
      mw = c > mw ? c : mw;
    }
    mw = wave_max_u32(mw);
    if ((t & 63) == 0) atomicMax(&sh_maxw, mw);
  }
  __syncthreads();
  int wbits = 32 - __clz(sh_maxw);
  int hi_bit = 32 + ((wbits + 3) & ~3);

  // 2. stable sort by count -> leaves ordered by (count, symbol)
  uint64_t* sorted = block_radix_sort(s.keys_a, s.keys_b, K, 32, hi_bit, cnt, sh16);
  __syncthreads();  // (the sort's table and w_lds share LDS)
  uint32_t* w = 2 * K <= kCbWCap ? w_lds : s.w;
  for (uint32_t i = t; i < K; i += T) {
    uint64_t key = sorted[i];
    w[i] = (uint32_t)(key >> 32);
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
  {
    uint32_t ml = 0;
    for (uint32_t i = t; i < K; i += T) {
      uint32_t d = s.depth[s.parent[i]] + 1;
      if (d > kMaxCodeLen) {
        atomicOr(&m->status, kStatusCodeTooLong);
        d = kMaxCodeLen;
      }
      enc_len[s.leaf_sym[i]] = (uint8_t)d;
      ml = d > ml ? d : ml;
    }
    ml = wave_max_u32(ml);
    if ((t & 63) == 0) atomicMax(&sh_maxlen, ml);
  }
  __syncthreads();

  // 5. canonical codes: (length, symbol) order
  compact_used(nullptr, enc_len, nsym, s.keys_a, symtab, sh16);
  uint64_t* bylen = block_radix_sort(s.keys_a, s.keys_b, K, 16, 24, cnt, sh16);
  // lengths per code length from the boundaries of the sorted runs
  for (uint32_t i = t; i < K; i += T) {
    const uint32_t l = (uint32_t)(bylen[i] >> 16) & 0xFF;
    if (i + 1 == K || ((uint32_t)(bylen[i + 1] >> 16) & 0xFF) != l) atomicAdd(&bl_count[l], i + 1);
    if (i > 0 && ((uint32_t)(bylen[i - 1] >> 16) & 0xFF) != l) atomicSub(&bl_count[l], i);
  }
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
  __shared__ uint32_t sh_lo, sh_hi;
  if (t == 0) {
    sh_lo = 0xFFFFFFFFu;
    sh_hi = 0;
  }
  __syncthreads();
  uint32_t lo = 0xFFFFFFFFu, hi = 0;
  for (uint32_t j = t; j < K; j += T) {
    uint64_t key = bylen[j];
    uint32_t l = (uint32_t)(key >> 16) & 0xFF, sym = (uint32_t)(key & 0xFFFF);
    enc_code[sym] = first_code[l] + (j - len_offset[l]);
    if (sym) {
      lo = sym < lo ? sym : lo;
      hi = sym > hi ? sym : hi;
    }
  }
  lo = wave_min_u32(lo);
  hi = wave_max_u32(hi);
  if ((t & 63) == 0) {
    atomicMin(&sh_lo, lo);
    atomicMax(&sh_hi, hi);
  }
  __syncthreads();
  if (t == 0 && sh_lo != 0xFFFFFFFFu) {
    atomicMin(&m->sym_lo, sh_lo);
    atomicMax(&m->sym_hi, sh_hi);
  }
}

// K <= kCbLdsCap: the whole tree in LDS, built by one wave, so that no step
// waits at a workgroup barrier (a wave's LDS accesses take effect in program
// order; an empty asm with a memory clobber keeps the compiler from moving
// them across the steps).  Leaves are sorted by (count, symbol) with a
// bitonic network; the bounds of each merge phase come from a 64-way search;
// canonical codes take, for each symbol, the number of smaller symbols of the
// same length, counted a wave of symbols at a time with ballots.
constexpr uint32_t kCbLdsCap = 2048;
constexpr uint32_t kCbScanBatch = 8;  // uint4 loads in flight per thread while scanning bins

struct CbLds {
  union {
    uint64_t key[kCbLdsCap];       // count << 32 | symbol-order index (until ranked)
    struct {
      uint16_t depth[2 * kCbLdsCap];
      uint16_t merged[kCbLdsCap];
      uint16_t phase_end[kCbLdsCap];
    };
  };
  uint32_t w[2 * kCbLdsCap];       // node weights: leaves by rank, then internal nodes
  uint16_t sym_of[kCbLdsCap];      // symbol of each symbol-order index
  uint16_t idx_of[kCbLdsCap];      // symbol-order index of each leaf rank
  uint16_t parent[2 * kCbLdsCap];
  uint8_t len_si[kCbLdsCap];       // code length by symbol-order index
  uint32_t bl_count[kMaxCodeLen + 2];
  uint32_t run[kMaxCodeLen + 2];
  uint64_t first_code[kMaxCodeLen + 2];
};

__device__ __forceinline__ void wave_step() { asm volatile("" ::: "memory"); }

// number of leading entries of the ascending w[lo, hi) that are <= v (hi - lo
// <= 4096), by two rounds of 64 probes
__device__ __forceinline__ uint32_t wave_count_le(const uint32_t* w, uint32_t lo, uint32_t hi,
                                                  uint64_t v, uint32_t lane) {
  const uint32_t len = hi - lo;
  if (len == 0) return 0;
  const uint32_t step = (len + 63) / 64;
  uint32_t i = lo + (lane + 1) * step - 1;
  const uint32_t c1 = (uint32_t)__popcll(__ballot(i < hi && (uint64_t)w[i] <= v));
  const uint32_t b = lo + c1 * step;
  i = b + lane;
  const uint32_t c2 = (uint32_t)__popcll(__ballot(lane < step && i < hi && (uint64_t)w[i] <= v));
  return c1 * step + c2;
}

// Leaves by rank: a bitonic network over P = 2^k >= K keys by the whole
// workgroup (keys are distinct; padding sorts last), each thread loading all
// its pairs of a step before exchanging them; then the weights and
// symbol-order indices by rank.  Called by every thread.
__device__ __forceinline__ void rank_leaves(uint32_t K, CbLds& L) {
  constexpr uint32_t kPairs = kCbLdsCap / 2 / kCbThreads;  // pairs per thread at most
  const uint32_t t = threadIdx.x;
  uint32_t P = 1;
  while (P < K) P <<= 1;
  for (uint32_t i = K + t; i < P; i += kCbThreads) L.key[i] = ~0ull;
  lds_barrier();
  for (uint32_t k = 2; k <= P; k <<= 1)
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      uint64_t x[kPairs], y[kPairs];
#pragma unroll
      for (uint32_t q = 0; q < kPairs; q++) {
        const uint32_t i = t + q * kCbThreads;
        const uint32_t a = 2 * i - (i & (j - 1));
        if (i < P / 2) {
          x[q] = L.key[a];
          y[q] = L.key[a + j];
        }
      }
#pragma unroll
      for (uint32_t q = 0; q < kPairs; q++) {
        const uint32_t i = t + q * kCbThreads;
        const uint32_t a = 2 * i - (i & (j - 1));
        if (i < P / 2 && (x[q] > y[q]) == ((a & k) == 0)) {
          L.key[a] = y[q];
          L.key[a + j] = x[q];
        }
      }
      lds_barrier();
    }
  for (uint32_t r = t; r < K; r += kCbThreads) {
    const uint64_t key = L.key[r];
    L.w[r] = (uint32_t)(key >> 32);
    L.idx_of[r] = (uint16_t)(key & 0xFFFFu);
  }
  lds_barrier();  // the key array is dead from here on
}

// Called by wave 0 alone, after rank_leaves.
__device__ __forceinline__ void codebook_wave(uint32_t K, uint64_t* enc_code, uint8_t* enc_len,
                                              uint32_t* symtab, Meta* m, CbLds& L) {
  const uint32_t lane = threadIdx.x;
  if (K == 1) {
    if (lane == 0) {
      const uint32_t sym = L.sym_of[0];
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
  for (uint32_t i = lane; i <= (uint32_t)kMaxCodeLen + 1; i += 64) {
    L.bl_count[i] = 0;
    L.run[i] = 0;
  }
  wave_step();

  // two-queue merge in phases (see the header of this section)
  uint32_t li = 0, qi = K, qn = K, nph = 0;
  uint32_t* w = L.w;
  constexpr uint64_t kInf = ~0ull;
  for (;;) {
    if ((K - li) + (qn - qi) <= 1) break;
    const uint64_t l0 = li < K ? w[li] : kInf, l1 = li + 1 < K ? w[li + 1] : kInf;
    const uint64_t q0 = qi < qn ? w[qi] : kInf, q1 = qi + 1 < qn ? w[qi + 1] : kInf;
    // the lighter front twice, the leaf on equal weights
    uint64_t tw;
    if (l0 <= q0)
      tw = l0 + (l1 <= q0 ? l1 : q0);
    else
      tw = q0 + (l0 <= q1 ? l0 : q1);
    const uint32_t cl = wave_count_le(w, li, K, tw, lane), ci = qn - qi;
    if (cl + ci < 2 || nph >= kCbLdsCap) {  // cannot happen with sorted leaves; never spin
      if (lane == 0) atomicOr(&m->status, kStatusCodeTooLong);
      return;
    }
    for (uint32_t x = lane; x < cl; x += 64)
      L.merged[x + lower_bound_w(w, qi, qn, w[li + x]) - qi] = (uint16_t)(li + x);
    for (uint32_t x = lane; x < ci; x += 64)
      L.merged[x + upper_bound_w(w, li, li + cl, w[qi + x]) - li] = (uint16_t)(qi + x);
    wave_step();
    const uint32_t c = cl + ci, np = c >> 1;
    for (uint32_t p = lane; p < np; p += 64) {
      const uint32_t u = L.merged[2 * p], v = L.merged[2 * p + 1];
      w[qn + p] = w[u] + w[v];
      L.parent[u] = (uint16_t)(qn + p);
      L.parent[v] = (uint16_t)(qn + p);
    }
    if (c & 1) {
      const uint32_t last = L.merged[c - 1];
      li += cl - (last < K ? 1 : 0);
      qi += ci - (last >= K ? 1 : 0);
    } else {
      li += cl;
      qi += ci;
    }
    qn += np;
    if (lane == 0) L.phase_end[nph] = (uint16_t)qn;
    nph++;
    wave_step();
  }

  // depths, root first: a phase's nodes have their parents in later phases
  const uint32_t root = 2 * K - 2;
  if (lane == 0) L.depth[root] = 0;
  wave_step();
  for (int p = (int)nph - 1; p >= 0; p--) {
    const uint32_t b0 = p == 0 ? K : L.phase_end[p - 1], b1 = L.phase_end[p];
    for (uint32_t i = b0 + lane; i < b1; i += 64)
      if (i != root) L.depth[i] = L.depth[L.parent[i]] + 1;
    wave_step();
  }
  uint32_t maxl = 0, bad = 0;
  for (uint32_t r = lane; r < K; r += 64) {
    uint32_t d = L.depth[L.parent[r]] + 1u;
    if (d > (uint32_t)kMaxCodeLen) {
      bad = 1;
      d = kMaxCodeLen;
    }
    L.len_si[L.idx_of[r]] = (uint8_t)d;
    atomicAdd(&L.bl_count[d], 1u);
    maxl = d > maxl ? d : maxl;
  }
  maxl = wave_max_u32(maxl);
  bad = wave_max_u32(bad);
  wave_step();
  if (lane == 0) {
    uint64_t code = 0;
    for (int l = 1; l <= kMaxCodeLen; l++) {
      code = (code + (l > 1 ? L.bl_count[l - 1] : 0)) << 1;
      L.first_code[l] = code;
    }
    if (bad) atomicOr(&m->status, kStatusCodeTooLong);
    m->nsym_used = K;
    m->max_len = maxl;
    const uint32_t lo = L.sym_of[0] ? L.sym_of[0] : L.sym_of[1], hi = L.sym_of[K - 1];
    m->sym_lo = lo;
    m->sym_hi = hi;
  }
  wave_step();
  // canonical codes: within a length, consecutive in symbol order
  for (uint32_t base = 0; base < K; base += 64) {
    const uint32_t i = base + lane;
    const bool valid = i < K;
    const uint32_t l = valid ? L.len_si[i] : 0u;
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 7; bit++) {
      const bool on = (l >> bit) & 1u;
      const uint64_t bb = __ballot(on);
      same &= on ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(same & ((1ull << lane) - 1));
    const uint32_t before = valid ? L.run[l] : 0u;
    wave_step();
    if (valid) {
      const uint32_t sym = L.sym_of[i];
      enc_code[sym] = L.first_code[l] + before + below;
      enc_len[sym] = (uint8_t)l;
      symtab[i] = sym | (l << 16);
      if ((same >> lane) == 1ull) L.run[l] = before + (uint32_t)__popcll(same);
    }
    wave_step();
  }
}

// The used symbols are found by scanning the histogram: only the window the
// histogram kernel counts in (and symbol 0) when no code fell outside it.
__device__ __forceinline__ void codebook_body(const uint32_t* __restrict__ hist, uint32_t nsym,
                                              const CodebookScratch& s, uint64_t* enc_code,
                                              uint8_t* enc_len, uint32_t* symtab, Meta* m) {
  __shared__ union {
    uint32_t cnt[16 * kCbThreads];  // radix-sort table of the global path
    uint32_t w[kCbWCap];            // its node weights, when they fit
    CbLds lds;
  } u;
  __shared__ uint32_t sh16[16];
  const uint32_t t = threadIdx.x;
  {
    uint4* z = reinterpret_cast<uint4*>(enc_len);  // kMaxSym bytes, 16-byte aligned
    for (uint32_t i = t; i < (nsym + 15) / 16; i += kCbThreads) z[i] = make_uint4(0, 0, 0, 0);
  }
  if (t == 0) m->n_unpred = hist[0];
  // bins [b0, b1) in aligned quads, plus bin 0 when the range leaves it out
  uint32_t b0 = 0, b1 = nsym;
  if (!m->hist_far) {
    const HistWindow hw = hist_window(nsym / 2);
    b0 = hw.slo;
    b1 = hw.slo + kHistShared < nsym ? hw.slo + kHistShared : nsym;
  }
  const uint32_t extra0 = b0 > 0 && hist[0] != 0;  // bin 0 outside the range, used
  const uint32_t q0 = b0 / 4, nq = (b1 + 3) / 4 - q0;   // quads to scan
  const uint32_t per = (nq + kCbThreads - 1) / kCbThreads;
  const uint32_t qa = q0 + (t * per < nq ? t * per : nq);
  const uint32_t qb = q0 + ((t + 1) * per < nq ? (t + 1) * per : nq);
  const uint4* h4 = reinterpret_cast<const uint4*>(hist);
  auto used = [&](uint32_t sym, uint32_t c) { return c != 0 && sym >= b0 && sym < b1; };
  uint32_t c = 0;
  for (uint32_t q = qa; q < qb; q += kCbScanBatch) {
    uint4 v[kCbScanBatch];
#pragma unroll
    for (uint32_t j = 0; j < kCbScanBatch; j++) v[j] = q + j < qb ? h4[q + j] : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (uint32_t j = 0; j < kCbScanBatch; j++) {
      const uint32_t s0 = 4 * (q + j);
      c += used(s0, v[j].x) + used(s0 + 1, v[j].y) + used(s0 + 2, v[j].z) + used(s0 + 3, v[j].w);
    }
  }
  uint32_t K;
  uint32_t pos = block_excl_scan_u32(c, sh16, &K) + extra0;
  K += extra0;
  if (K == 0) {
    if (t == 0) {
      m->nsym_used = 0;
      m->max_len = 0;
    }
    return;
  }
  if (K > kCbLdsCap) {
    codebook_global(hist, nsym, s, enc_code, enc_len, symtab, m, u.cnt, sh16, u.w);
    return;
  }
  // leaves in symbol order, at the scanned offsets
  CbLds& L = u.lds;
  if (t == 0 && extra0) {
    L.key[0] = (uint64_t)hist[0] << 32;
    L.sym_of[0] = 0;
  }
  for (uint32_t q = qa; c && q < qb; q += kCbScanBatch) {
    uint4 v[kCbScanBatch];
#pragma unroll
    for (uint32_t j = 0; j < kCbScanBatch; j++) v[j] = q + j < qb ? h4[q + j] : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (uint32_t j = 0; j < kCbScanBatch; j++) {
      const uint32_t e[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
#pragma unroll
      for (int h = 0; h < 4; h++) {
        const uint32_t sym = 4 * (q + j) + h;
        if (used(sym, e[h])) {
          L.key[pos] = ((uint64_t)e[h] << 32) | pos;
          L.sym_of[pos] = (uint16_t)sym;
          pos++;
        }
      }
    }
  }
  lds_barrier();
  if (K > 1) rank_leaves(K, L);
  if (t < 64) codebook_wave(K, enc_code, enc_len, symtab, m, L);
}

__global__ __launch_bounds__(kCbThreads) void k_codebook(const uint32_t* __restrict__ hist,
                                                          uint32_t nsym, CodebookScratch s,
                                                          uint64_t* enc_code, uint8_t* enc_len,
                                                          uint32_t* symtab, Meta* m) {
  codebook_body(hist, nsym, s, enc_code, enc_len, symtab, m);
}

// one workgroup per field of a batch
__global__ __launch_bounds__(kCbThreads) void k_b_codebook(BLaunch L) {
  BJob j;
  uint32_t local;
  if (!batch_job(L, j, local)) return;
  const BField& f = L.f[j.field];
  codebook_body(f.hist, 2 * f.R, f.cb, f.enc_code, f.enc_len, f.symtab, f.m);
}

hipError_t launch_b_codebook(BLaunch L, uint32_t nwg, hipStream_t st) {
  if (nwg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_codebook, dim3(nwg), dim3(kCbThreads), 0, st, L);
  return hipGetLastError();
}

hipError_t launch_codebook(const uint32_t* hist, uint32_t nsym, CodebookScratch s,
                           uint64_t* enc_code, uint8_t* enc_len, uint32_t* symtab, Meta* m,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_codebook, dim3(1), dim3(kCbThreads), 0, st, hist, nsym, s, enc_code,
                     enc_len, symtab, m);
  return hipGetLastError();
}

}  // namespace szg
