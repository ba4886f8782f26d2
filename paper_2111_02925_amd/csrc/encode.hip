// Huffman encoding of the quantization codes and stream assembly, gfx950.
//
// Paper: SZ3 (arXiv 2111.02925), Section 3.2 "Encoder" (compress the codes
// with the codebook built from their frequencies) and Algorithm 1 (the
// quantizer's unpredictable values and the encoder's table are saved with
// the bitstream).
//
// Three steps: (1) every chunk's size (code bits, unpredictable count) by one
// wave per chunk, (2) exclusive scans of the sizes, (3) packing.  In (1) and
// (3) lane L of the wave owns a contiguous run of m = max(32, chunk/64)
// symbols, so every lane but the last non-empty one writes at least 32 bits:
// a 32-bit output word then holds bits of at most two lanes, the full words a
// lane produces are stored directly, and the one word it shares with its
// predecessor is completed by that lane through a register shuffle.  Runs of
// up to 64 symbols stay in registers between the two passes over them.
//
// Codewords are looked up in an LDS copy of the codebook window that holds
// every coded symbol (the unpredictable symbol 0 lives in registers); when
// the coded symbols span more than the window, or a code is longer than 32
// bits, a variant that falls back to the global codebook runs instead.
#include "block_ops.h"
#include "common.h"

namespace szg {

constexpr uint32_t kEncWindow = 7168;  // LDS codebook entries
constexpr int kEncWaves = 4;
constexpr int kSeg = 64;  // symbols of a lane's run held in registers at once

__device__ __forceinline__ void guarded_store_u32(uint8_t* out, uint64_t cap, uint64_t off,
                                                  uint32_t v) {
  if (off + 4 <= cap) *reinterpret_cast<uint32_t*>(out + off) = v;
}

struct EncTables {
  uint32_t code[kEncWindow];
  uint8_t len[kEncWindow];
};

struct EncWindow {
  uint32_t lo;       // first symbol of the window
  uint32_t span;     // window entries to load: the coded symbols' range when lds_only
  bool lds_only;     // every coded symbol other than 0 is in the window, codes <= 32 bits
  uint64_t code0;    // codeword of symbol 0
  uint32_t len0;
  uint32_t max_len;
};

__device__ __forceinline__ EncWindow enc_window(const Meta* m, uint32_t R,
                                                const uint64_t* __restrict__ enc_code,
                                                const uint8_t* __restrict__ enc_len) {
  EncWindow w;
  const uint32_t slo = m->sym_lo, shi = m->sym_hi;
  const bool none = slo == 0xFFFFFFFFu;
  w.lds_only = (none || shi - slo < kEncWindow) && m->max_len <= 32;
  w.lo = w.lds_only ? (none ? 0u : slo) : (R > kEncWindow / 2 ? R - kEncWindow / 2 : 0u);
  w.span = w.lds_only ? (none ? 0u : shi - slo + 1) : kEncWindow;
  w.code0 = enc_code[0];
  w.len0 = enc_len[0];
  w.max_len = m->max_len;
  return w;
}

__device__ __forceinline__ void load_tables(EncTables& t, const EncWindow& w, uint32_t nsym,
                                            const uint64_t* __restrict__ enc_code,
                                            const uint8_t* __restrict__ enc_len, bool codes) {
  for (uint32_t i = threadIdx.x; i < w.span; i += blockDim.x) {
    const uint32_t s = w.lo + i;
    const uint32_t len = s < nsym ? enc_len[s] : 0u;
    t.len[i] = (uint8_t)(len <= 32 ? len : 0u);
    if (codes) t.code[i] = s < nsym ? (uint32_t)enc_code[s] : 0u;
  }
}

// Codeword of a symbol.  LDS_ONLY: straight from LDS (no global access, so
// nothing the compiler must wait for on the common path).
template <bool LDS_ONLY>
__device__ __forceinline__ void lookup(uint32_t sym, const EncTables& t, const EncWindow& w,
                                       const uint64_t* __restrict__ enc_code,
                                       const uint8_t* __restrict__ enc_len, uint64_t& cw,
                                       uint32_t& len) {
  if (sym == 0) {
    cw = w.code0;
    len = w.len0;
    return;
  }
  const uint32_t off = sym - w.lo;
  if (LDS_ONLY) {
    cw = t.code[off];
    len = t.len[off];
  } else {
    const uint32_t l = off < kEncWindow ? t.len[off] : 0u;
    if (l) {
      cw = t.code[off];
      len = l;
    } else {
      cw = enc_code[sym];
      len = enc_len[sym];
    }
  }
}

// The lane's symbols [i0, i0 + kSeg) clipped to `end`, two per word.
__device__ __forceinline__ void load_seg(const uint16_t* __restrict__ codes, uint64_t i0,
                                         uint64_t end, uint32_t (&w)[kSeg / 2]) {
  if (i0 + kSeg <= end) {
    const uint4* p = reinterpret_cast<const uint4*>(codes + i0);
#pragma unroll
    for (int k = 0; k < kSeg / 8; k++) {
      const uint4 a = p[k];
      w[4 * k] = a.x;
      w[4 * k + 1] = a.y;
      w[4 * k + 2] = a.z;
      w[4 * k + 3] = a.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kSeg / 2; k++) {
      const uint32_t a = i0 + 2 * k < end ? codes[i0 + 2 * k] : 0u;
      const uint32_t b = i0 + 2 * k + 1 < end ? codes[i0 + 2 * k + 1] : 0u;
      w[k] = a | (b << 16);
    }
  }
}

__device__ __forceinline__ uint32_t sym_at(const uint32_t (&w)[kSeg / 2], int k) {
  return (w[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
}

struct LaneRun {
  uint64_t beg, end;  // the lane's symbols [beg, end)
  uint32_t m;         // run length
};

__device__ __forceinline__ LaneRun lane_run(uint64_t c, uint32_t chunk, uint64_t n, int lane) {
  const uint32_t m = chunk / 64 > 32 ? chunk / 64 : 32;
  const uint64_t cbeg = c * chunk, cend = cbeg + chunk < n ? cbeg + chunk : n;
  LaneRun r;
  r.m = m;
  r.beg = cbeg + (uint64_t)m * lane;
  if (r.beg > cend) r.beg = cend;
  r.end = r.beg + m < cend ? r.beg + m : cend;
  return r;
}

// ------------------------------------------------------ lane-parallel path
// When every code is at most 32 bits and the coded symbols fit kFastWindow
// LDS entries, a wave takes a chunk kStep symbols at a time, 8 consecutive
// symbols per lane: the lanes' bit counts are scanned across the wave, and
// a lane's codewords (joined in a 64-bit register when they total at most 64
// bits, three buffer words at most; one by one otherwise) are ORed into a
// per-wave LDS bit buffer at their offset, so no step depends on a branch per
// symbol.  The buffer is stored when the chunk ends (consecutive lanes,
// consecutive words), or earlier when another step might not fit, then its
// partial last word moves to the front.  Stores inside the step loop would
// make every prefetch of the next step's codes wait for them to complete.

constexpr uint32_t kStep = 512;                // symbols per wave step, 8 per lane
constexpr uint32_t kBufWords = 768;            // bit buffer words per wave (a step needs at most 512)
constexpr uint32_t kBufAlloc = kBufWords + 3;  // plus the words a last step may touch
constexpr uint32_t kFastWindow = 3064;         // LDS codebook entries of the lane-parallel path
// with codes of at most 27 bits an entry takes 32 bits (code | len << 27), so
// the same LDS holds twice the window
constexpr uint32_t kFastWindow32 = 2 * (kFastWindow + 1) - 1;
constexpr uint32_t kLen32 = 27;

struct FastLds {
  union {
    // code | len << 32 by symbol - lo; the last entry is symbol 0's, with bit
    // 40 set so that summing entries >> 40 counts unpredictable values
    uint64_t ent[kFastWindow + 1];
    // code | len << 27 by symbol - lo; the last entry is symbol 0's
    uint32_t ent32[kFastWindow32 + 1];
  };
  uint32_t buf[kEncWaves][kBufAlloc];
};
union EncLds {
  EncTables t;
  FastLds f;
};

// 0: the per-lane-run path; 1: the lane-parallel path with 64-bit entries;
// 2: with 32-bit entries (codes of at most kLen32 bits)
__device__ __forceinline__ int fast_path(const EncWindow& w) {
  if (!w.lds_only) return 0;
  if (w.max_len <= kLen32 && w.span <= kFastWindow32) return 2;
  return w.span <= kFastWindow ? 1 : 0;
}

template <bool E32>
__device__ __forceinline__ void load_fast(FastLds& f, const EncWindow& w,
                                          const uint64_t* __restrict__ enc_code,
                                          const uint8_t* __restrict__ enc_len) {
  if (E32) {
    for (uint32_t i = threadIdx.x; i < w.span; i += blockDim.x)
      f.ent32[i] = ((uint32_t)enc_len[w.lo + i] << kLen32) | (uint32_t)enc_code[w.lo + i];
    if (threadIdx.x == 0) f.ent32[kFastWindow32] = (w.len0 << kLen32) | (uint32_t)w.code0;
  } else {
    for (uint32_t i = threadIdx.x; i < w.span; i += blockDim.x)
      f.ent[i] = ((uint64_t)enc_len[w.lo + i] << 32) | (uint32_t)enc_code[w.lo + i];
    if (threadIdx.x == 0)
      f.ent[kFastWindow] = (1ull << 40) | ((uint64_t)w.len0 << 32) | (uint32_t)w.code0;
  }
  for (uint32_t i = threadIdx.x; i < kEncWaves * kBufAlloc; i += blockDim.x)
    (&f.buf[0][0])[i] = 0;
}

// The 8 symbols [i0, i0 + 8) of a lane, packed two per word: one load,
// always taken (a load taken on a branch would be waited for where the
// branches join), from the last whole vector when i0 is past it.  The code
// buffer holds whole vectors; symbols past the field are ignored by the
// callers, which count only the first nv.
__device__ __forceinline__ uint4 load8(const uint16_t* __restrict__ codes, uint64_t i0,
                                       uint64_t last8) {
  return *reinterpret_cast<const uint4*>(codes + (i0 < last8 ? i0 : last8));
}

// Table entries of the 8 symbols; symbols at or past nv get an empty entry.
struct Sym8 {
  uint32_t code[8], len[8], zeros;
};
template <bool E32>
__device__ __forceinline__ Sym8 lookup8(const FastLds& f, uint32_t lo, uint4 v, uint32_t nv) {
  Sym8 r;
  r.zeros = 0;
  const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int j = 0; j < 8; j++) {
    const uint32_t s = (wd[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
    if (E32) {
      // (clamped: symbols past the field's end may be anything; symbols
      // below lo wrap to large offsets)
      const uint32_t k = min(s - lo, kFastWindow32);
      uint32_t e = f.ent32[s ? k : kFastWindow32];
      const bool in = (uint32_t)j < nv;
      e = in ? e : 0u;
      r.code[j] = e & ((1u << kLen32) - 1u);
      r.len[j] = e >> kLen32;
      r.zeros += (in && s == 0) ? 1u : 0u;
    } else {
      const uint32_t k = s - lo < kFastWindow ? s - lo : kFastWindow;
      uint64_t e = f.ent[s ? k : kFastWindow];
      e = (uint32_t)j < nv ? e : 0ull;
      r.code[j] = (uint32_t)e;
      r.len[j] = (uint32_t)(e >> 32) & 0xFFu;
      r.zeros += (uint32_t)(e >> 40);
    }
  }
  return r;
}

__device__ __forceinline__ void wave_step() { asm volatile("" ::: "memory"); }

// ------------------------------------------------ single read of the codes
// On the lane-parallel path the codes are read once: the first pass packs
// each chunk exactly as pack_fast does, but into a slot of its own (chunk c's
// words at word c * chunk of `slots`: a chunk of clen symbols of at most 32
// bits each fills at most clen words, so the slots of a field of n symbols
// fit n words), writing its chunk-table and sub-chunk entries (chunk-local
// values) and its sizes for the scans; the second pass copies every slot to
// its place in the bitstream and scatters the unpredictable values of the
// chunks that have some (ranked by ballots over the chunk's codes).

template <bool E32>
__device__ __forceinline__ void pack_fast_slots(
    const uint16_t* __restrict__ codes, uint64_t n, uint32_t chunk, uint32_t sub,
    uint64_t nchunks, FastLds& f, uint32_t lo, uint32_t* chunk_words, uint32_t* chunk_zeros,
    uint32_t* slots, const Layout& l, uint8_t* out, uint64_t cap, uint32_t bid, uint32_t nblk) {
  const uint32_t lane = threadIdx.x & 63;
  uint32_t* buf = f.buf[threadIdx.x >> 6];
  const uint32_t span = chunk / sub;
  const uint64_t wstride = (uint64_t)nblk * kEncWaves;
  const uint64_t last8 = (n - 1) & ~7ull;
  for (uint64_t c = bid * (uint64_t)kEncWaves + (threadIdx.x >> 6); c < nchunks;
       c += wstride) {
    const uint64_t cbeg = c * chunk, cend = cbeg + chunk < n ? cbeg + chunk : n;
    const uint32_t clen = (uint32_t)(cend - cbeg);
    uint32_t* slot = slots + cbeg;
    uint32_t have = 0, done = 0, written = 0, zeros = 0;
    uint32_t next_sub = span, k_sub = 1;
    uint4 nxt = load8(codes, cbeg + 8 * lane, last8);
    for (uint64_t g = cbeg; g < cend; g += kStep) {
      const uint4 cur = nxt;
      const uint64_t i0 = g + 8 * lane;
      nxt = load8(codes, i0 + kStep, last8);
      const uint32_t off = (uint32_t)(i0 - cbeg);
      const uint32_t nv = off < clen ? (clen - off < 8 ? clen - off : 8u) : 0u;
      const Sym8 r = lookup8<E32>(f, lo, cur, nv);
      uint32_t pre[8], t = 0;
      uint64_t acc = 0;
#pragma unroll
      for (int j = 0; j < 8; j++) {
        pre[j] = t;
        t += r.len[j];
        acc = (acc << r.len[j]) | r.code[j];
      }
      const uint32_t mine = t | (r.zeros << 16);
      const uint32_t incl = wave_incl_scan_dpp(mine);
      const uint32_t tot = __builtin_amdgcn_readlane(incl, 63), excl = incl - mine;
      const uint32_t e = excl & 0xFFFFu;
      const uint32_t step0 = (uint32_t)(g - cbeg);
      while (k_sub < sub && next_sub < clen && next_sub < step0 + kStep) {
        if (off == next_sub)
          guarded_store_u32(out, cap, l.off_sub + 4 * (c * (sub - 1) + k_sub - 1), done + e);
        next_sub += span;
        k_sub++;
      }
      const uint32_t o = have + e;
      if (t <= 64) {
        acc = t ? acc << (64 - t) : 0ull;
        const uint32_t sh = o & 31, wd = o >> 5;
        atomicOr(&buf[wd], (uint32_t)(acc >> (32 + sh)));
        atomicOr(&buf[wd + 1], (uint32_t)(acc >> sh));
        atomicOr(&buf[wd + 2], (uint32_t)(acc << (32 - sh)));
      } else {
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const uint32_t pos = o + pre[j], sh = pos & 31;
          const uint64_t v = r.len[j] ? (uint64_t)r.code[j] << (64 - r.len[j] - sh) : 0ull;
          atomicOr(&buf[pos >> 5], (uint32_t)(v >> 32));
          atomicOr(&buf[(pos >> 5) + 1], (uint32_t)v);
        }
      }
      have += tot & 0xFFFFu;
      done += tot & 0xFFFFu;
      zeros += tot >> 16;
      if (have > (kBufWords - kStep - 1) * 32) {
        wave_step();
        const uint32_t full = have >> 5;
        for (uint32_t k = lane; k < full; k += 64) slot[written + k] = buf[k];
        const uint32_t last = buf[full];
        wave_step();
        for (uint32_t k = lane; k <= full + 2; k += 64) buf[k] = k == 0 ? last : 0u;
        wave_step();
        written += full;
        have &= 31;
      }
    }
    wave_step();
    const uint32_t nw = (have + 31) >> 5;
    for (uint32_t k = lane; k < nw; k += 64) slot[written + k] = buf[k];
    wave_step();
    for (uint32_t k = lane; k < nw + 2; k += 64) buf[k] = 0u;
    wave_step();
    for (uint32_t k = lane + 1; k < sub; k += 64)
      if ((uint64_t)k * span >= clen)
        guarded_store_u32(out, cap, l.off_sub + 4 * (c * (sub - 1) + k - 1), done);
    if (lane == 0) {
      const uint32_t words = (done + 31) / 32;
      chunk_words[c] = words;
      chunk_zeros[c] = zeros;
      guarded_store_u32(out, cap, l.off_chunk + 8 * c, words);
      guarded_store_u32(out, cap, l.off_chunk + 8 * c + 4, zeros);
    }
  }
}

template <typename T>
__device__ __forceinline__ void copy_slots(
    const uint16_t* __restrict__ codes, const T* __restrict__ x, uint64_t n, uint32_t chunk,
    uint64_t nchunks, const uint32_t* __restrict__ chunk_words,
    const uint32_t* __restrict__ chunk_zeros, const uint64_t* __restrict__ word_off,
    const uint64_t* __restrict__ zero_off, const uint32_t* __restrict__ slots, const Layout& l,
    uint8_t* out, uint64_t cap, uint32_t bid, uint32_t nblk) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wstride = (uint64_t)nblk * kEncWaves;
  const uint64_t last8 = (n - 1) & ~7ull;
  for (uint64_t c = bid * (uint64_t)kEncWaves + (threadIdx.x >> 6); c < nchunks;
       c += wstride) {
    const uint64_t cbeg = c * chunk, cend = cbeg + chunk < n ? cbeg + chunk : n;
    const uint32_t nw = chunk_words[c];
    const uint32_t* src = slots + cbeg;
    const uint64_t dst = l.off_bits + 4 * word_off[c];
    uint32_t k = lane;
    for (; k + 192 < nw; k += 256) {  // four loads in flight
      const uint32_t a = src[k], b = src[k + 64], d = src[k + 128], e = src[k + 192];
      guarded_store_u32(out, cap, dst + 4 * (uint64_t)k, a);
      guarded_store_u32(out, cap, dst + 4 * (uint64_t)(k + 64), b);
      guarded_store_u32(out, cap, dst + 4 * (uint64_t)(k + 128), d);
      guarded_store_u32(out, cap, dst + 4 * (uint64_t)(k + 192), e);
    }
    for (; k < nw; k += 64) guarded_store_u32(out, cap, dst + 4 * (uint64_t)k, src[k]);
    if (chunk_zeros[c]) {  // unpredictable values, verbatim, flat order
      // 8 codes a lane per step; a lane's code-0 symbols are ranked by a
      // wave scan of the lanes' counts
      uint64_t rk = zero_off[c];
      const uint32_t clen = (uint32_t)(cend - cbeg);
      for (uint64_t g = cbeg; g < cend; g += kStep) {
        const uint64_t i0 = g + 8 * lane;
        const uint4 q = load8(codes, i0, last8);
        const uint32_t off = (uint32_t)(i0 - cbeg);
        const uint32_t nv = off < clen ? (clen - off < 8 ? clen - off : 8u) : 0u;
        const uint32_t wd[4] = {q.x, q.y, q.z, q.w};
        uint32_t zm = 0;
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const uint32_t sym = (wd[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
          zm |= (sym == 0 && (uint32_t)j < nv) ? 1u << j : 0u;
        }
        const uint32_t cnt = (uint32_t)__popc(zm);
        const uint32_t incl = wave_incl_scan_dpp(cnt);
        const uint32_t tot = __builtin_amdgcn_readlane(incl, 63);
        uint64_t r = rk + (incl - cnt);
        for (int j = 0; j < 8; j++)
          if ((zm >> j) & 1u) {
            const uint64_t o = l.off_unpred + r * sizeof(T);
            if (o + sizeof(T) <= cap) *reinterpret_cast<T*>(out + o) = x[i0 + j];
            r++;
          }
        rk += tot;
      }
    }
  }
}

// ------------------------------------------------------------- chunk sizes

template <bool LDS_ONLY>
__device__ __forceinline__ void size_chunks(const uint16_t* __restrict__ codes, uint64_t n,
                                            uint32_t chunk, uint64_t nchunks, const EncTables& t,
                                            const EncWindow& w,
                                            const uint64_t* __restrict__ enc_code,
                                            const uint8_t* __restrict__ enc_len,
                                            uint32_t* chunk_words, uint32_t* chunk_zeros,
                                            uint32_t bid, uint32_t nblk) {
  const int lane = threadIdx.x & 63;
  const uint64_t wstride = (uint64_t)nblk * kEncWaves;
  for (uint64_t c = bid * (uint64_t)kEncWaves + (threadIdx.x >> 6); c < nchunks;
       c += wstride) {
    const LaneRun r = lane_run(c, chunk, n, lane);
    uint32_t bits = 0, zeros = 0;
    for (uint64_t s0 = r.beg; s0 < r.end; s0 += kSeg) {
      uint32_t v[kSeg / 2];
      load_seg(codes, s0, r.end, v);
#pragma unroll
      for (int k = 0; k < kSeg; k++) {
        if (s0 + k < r.end) {
          const uint32_t sym = sym_at(v, k);
          uint64_t cw;
          uint32_t len;
          lookup<LDS_ONLY>(sym, t, w, enc_code, enc_len, cw, len);
          bits += len;
          zeros += sym == 0;
        }
      }
    }
    bits = wave_sum_u32(bits);
    zeros = wave_sum_u32(zeros);
    if (lane == 0) {
      chunk_words[c] = (bits + 31) / 32;
      chunk_zeros[c] = zeros;
    }
  }
}

template <typename T, bool LDS_ONLY, bool SLOTS>
__device__ __forceinline__ void pack_chunks(
    const uint16_t* __restrict__ codes, const T* __restrict__ x, uint64_t n, uint32_t chunk,
    uint32_t sub, uint64_t nchunks, const EncTables& t, const EncWindow& w,
    const uint64_t* __restrict__ enc_code, const uint8_t* __restrict__ enc_len,
    uint32_t* chunk_words, uint32_t* chunk_zeros, const uint64_t* __restrict__ word_off,
    const uint64_t* __restrict__ zero_off, uint32_t* slots, const Layout& l, uint8_t* out,
    uint64_t cap, uint32_t bid, uint32_t nblk);

// The first pass: the chunks' sizes, and on the lane-parallel path their
// bits packed into the slots (with their chunk-table and sub-chunk entries).
__device__ __forceinline__ void encode_size_body(
    EncLds& u, const uint16_t* __restrict__ codes, uint64_t n, uint32_t chunk, uint32_t sub,
    uint64_t nchunks, uint32_t R, uint32_t nsym, const uint64_t* __restrict__ enc_code,
    const uint8_t* __restrict__ enc_len, uint32_t* chunk_words, uint32_t* chunk_zeros,
    uint32_t* slots, uint8_t* out, uint64_t cap, const Meta* __restrict__ m, uint32_t bid,
    uint32_t nblk) {
  EncTables& t = u.t;
  const EncWindow w = enc_window(m, R, enc_code, enc_len);
  if (const int fp = fast_path(w)) {
    // (the chunk-table and sub-chunk sections do not depend on the totals)
    const Layout l = stream_layout(m->nsym_used, nchunks, sub, 0, 4, 0);
    if (fp == 2) {
      load_fast<true>(u.f, w, enc_code, enc_len);
      __syncthreads();
      pack_fast_slots<true>(codes, n, chunk, sub, nchunks, u.f, w.lo, chunk_words, chunk_zeros,
                            slots, l, out, cap, bid, nblk);
    } else {
      load_fast<false>(u.f, w, enc_code, enc_len);
      __syncthreads();
      pack_fast_slots<false>(codes, n, chunk, sub, nchunks, u.f, w.lo, chunk_words, chunk_zeros,
                             slots, l, out, cap, bid, nblk);
    }
    return;
  }
  if (w.max_len <= 32) {  // the per-lane-run path, into the slots
    load_tables(t, w, nsym, enc_code, enc_len, true);
    __syncthreads();
    const Layout l = stream_layout(m->nsym_used, nchunks, sub, 0, 4, 0);
    if (w.lds_only)
      pack_chunks<float, true, true>(codes, nullptr, n, chunk, sub, nchunks, t, w, enc_code,
                                     enc_len, chunk_words, chunk_zeros, nullptr, nullptr, slots, l,
                                     out, cap, bid, nblk);
    else
      pack_chunks<float, false, true>(codes, nullptr, n, chunk, sub, nchunks, t, w, enc_code,
                                      enc_len, chunk_words, chunk_zeros, nullptr, nullptr, slots, l,
                                      out, cap, bid, nblk);
    return;
  }
  // codes over 32 bits: the sizes here, the packing in the second pass
  load_tables(t, w, nsym, enc_code, enc_len, !w.lds_only);
  __syncthreads();
  if (w.lds_only)
    size_chunks<true>(codes, n, chunk, nchunks, t, w, enc_code, enc_len, chunk_words, chunk_zeros,
                      bid, nblk);
  else
    size_chunks<false>(codes, n, chunk, nchunks, t, w, enc_code, enc_len, chunk_words, chunk_zeros,
                       bid, nblk);
}

__global__ __launch_bounds__(kEncWaves * 64) void k_encode_size(
    const uint16_t* __restrict__ codes, uint64_t n, uint32_t chunk, uint32_t sub, uint64_t nchunks,
    uint32_t R, uint32_t nsym, const uint64_t* __restrict__ enc_code,
    const uint8_t* __restrict__ enc_len, uint32_t* chunk_words, uint32_t* chunk_zeros,
    uint32_t* slots, uint8_t* out, uint64_t cap, const Meta* __restrict__ m) {
  __shared__ EncLds u;
  encode_size_body(u, codes, n, chunk, sub, nchunks, R, nsym, enc_code, enc_len, chunk_words,
                   chunk_zeros, slots, out, cap, m, blockIdx.x, gridDim.x);
}

// the chunk sizes of every field of a batch
__global__ __launch_bounds__(kEncWaves * 64) void k_b_encode_size(BLaunch L) {
  __shared__ EncLds u;
  BJob j;
  uint32_t local;
  if (!batch_job(L, j, local)) return;
  const BField& f = L.f[j.field];
  encode_size_body(u, f.codes, f.n, f.chunk, f.sub, f.nchunks, f.R, 2 * f.R, f.enc_code,
                   f.enc_len, f.chunk_words, f.chunk_zeros, static_cast<uint32_t*>(f.rec), f.out,
                   f.cap, f.m, local, j.nblk);
}

// ------------------------------------------------------------------ packing

// SLOTS (codes of at most 32 bits): the chunk is packed into its slot (as on
// the lane-parallel path), its sizes and table entries written, and its
// unpredictable values left to the copy pass; otherwise packed into place
// from the scans' offsets.
template <typename T, bool LDS_ONLY, bool SLOTS>
__device__ __forceinline__ void pack_chunks(
    const uint16_t* __restrict__ codes, const T* __restrict__ x, uint64_t n, uint32_t chunk,
    uint32_t sub, uint64_t nchunks, const EncTables& t, const EncWindow& w,
    const uint64_t* __restrict__ enc_code, const uint8_t* __restrict__ enc_len,
    uint32_t* chunk_words, uint32_t* chunk_zeros, const uint64_t* __restrict__ word_off,
    const uint64_t* __restrict__ zero_off, uint32_t* slots, const Layout& l, uint8_t* out,
    uint64_t cap, uint32_t bid, uint32_t nblk) {
  const int lane = threadIdx.x & 63;
  const uint64_t wstride = (uint64_t)nblk * kEncWaves;
  for (uint64_t c = bid * (uint64_t)kEncWaves + (threadIdx.x >> 6); c < nchunks;
       c += wstride) {
    const LaneRun r = lane_run(c, chunk, n, lane);
    const bool cached = r.m <= kSeg;
    uint32_t v[kSeg / 2];
    // pass A: the lane's bits and unpredictable count
    uint32_t bits = 0, zeros = 0;
    for (uint64_t s0 = r.beg; s0 < r.end; s0 += kSeg) {
      load_seg(codes, s0, r.end, v);
#pragma unroll
      for (int k = 0; k < kSeg; k++) {
        if (s0 + k < r.end) {
          const uint32_t sym = sym_at(v, k);
          uint64_t cw;
          uint32_t len;
          lookup<LDS_ONLY>(sym, t, w, enc_code, enc_len, cw, len);
          bits += len;
          zeros += sym == 0;
        }
      }
    }
    const uint32_t bits_incl = wave_incl_scan_u32(bits, lane);
    const uint32_t zeros_incl = wave_incl_scan_u32(zeros, lane);
    const uint64_t bit0 = bits_incl - bits;
    uint64_t zrank = SLOTS ? 0 : zero_off[c] + (zeros_incl - zeros);
    const uint64_t wbase = SLOTS ? 0 : l.off_bits + 4 * word_off[c];
    uint32_t* slot = SLOTS ? slots + c * chunk : nullptr;
    if (SLOTS) {
      const uint32_t words = (__shfl(bits_incl, 63, 64) + 31) / 32;
      const uint32_t zc = __shfl(zeros_incl, 63, 64);
      if (lane == 0) {
        chunk_words[c] = words;
        chunk_zeros[c] = zc;
        guarded_store_u32(out, cap, l.off_chunk + 8 * c, words);
        guarded_store_u32(out, cap, l.off_chunk + 8 * c + 4, zc);
      }
    } else if (lane == 0) {
      guarded_store_u32(out, cap, l.off_chunk + 8 * c, chunk_words[c]);
      guarded_store_u32(out, cap, l.off_chunk + 8 * c + 4, chunk_zeros[c]);
    }
    // sub-chunk k starts with lane k * (chunk / sub) / m: its bit offset in the
    // chunk is that lane's exclusive prefix (the chunk's end for lanes past it)
    if (sub > 1) {
      const uint32_t lanes_per_sub = chunk / sub / r.m;
      if (lane > 0 && lane % lanes_per_sub == 0) {
        const uint32_t k = lane / lanes_per_sub;
        if (k < sub)
          guarded_store_u32(out, cap, l.off_sub + 4 * (c * (sub - 1) + k - 1), (uint32_t)bit0);
      }
    }
    // pass B: pack.  acc holds na pending bits left-aligned; the first word
    // of a run that starts inside a word goes to the previous lane.
    uint64_t wi = bit0 >> 5;
    uint32_t na = (uint32_t)(bit0 & 31);
    bool first_pending = na != 0;
    uint32_t first_contrib = 0;
    uint64_t acc = 0;
    auto emit = [&]() {
      const uint32_t word = (uint32_t)(acc >> 32);
      if (first_pending) {
        first_contrib = word;
        first_pending = false;
      } else if (SLOTS) {
        slot[wi] = word;
      } else {
        guarded_store_u32(out, cap, wbase + 4 * wi, word);
      }
      wi++;
      acc <<= 32;
      na -= 32;
    };
    for (uint64_t s0 = r.beg; s0 < r.end; s0 += kSeg) {
      if (!cached) load_seg(codes, s0, r.end, v);
#pragma unroll
      for (int k = 0; k < kSeg; k++) {
        if (s0 + k < r.end) {
          const uint32_t sym = sym_at(v, k);
          uint64_t cw;
          uint32_t len;
          lookup<LDS_ONLY>(sym, t, w, enc_code, enc_len, cw, len);
          if (len > 32) {
            const uint32_t hl = len - 32;
            acc |= (cw >> 32) << (64 - hl - na);
            na += hl;
            if (na >= 32) emit();
            cw &= 0xFFFFFFFFull;
            len = 32;
          }
          acc |= cw << (64 - len - na);
          na += len;
          if (na >= 32) emit();
          if (!SLOTS && sym == 0) {  // unpredictable value, verbatim, flat order
            const uint64_t off = l.off_unpred + zrank * sizeof(T);
            if (off + sizeof(T) <= cap) *reinterpret_cast<T*>(out + off) = x[s0 + k];
            zrank++;
          }
        }
      }
    }
    // the run's last, partial word: this lane's bits, completed with the
    // successor's first-word bits
    uint32_t last = 0;
    bool has_last = false;
    if (na) {
      last = (uint32_t)(acc >> 32);
      if (first_pending) {  // the whole run sits inside its first word
        first_contrib = last;
        first_pending = false;
      } else {
        has_last = true;
      }
    }
    uint32_t next = __shfl_down(first_contrib, 1, 64);
    if (lane == 63) next = 0;
    if (has_last) {
      if (SLOTS)
        slot[wi] = last | next;
      else
        guarded_store_u32(out, cap, wbase + 4 * wi, last | next);
    }
  }
}

// The second pass for codes over 32 bits: packed from scratch into place.
// (Otherwise k_encode_copy moves the slots instead.)
template <typename T>
__device__ __forceinline__ void encode_pack_body(
    EncLds& u, const uint16_t* __restrict__ codes, const T* __restrict__ x, uint64_t n,
    uint32_t chunk, uint32_t sub, uint64_t nchunks, uint32_t R, uint32_t nsym,
    const uint64_t* __restrict__ enc_code, const uint8_t* __restrict__ enc_len,
    const uint32_t* __restrict__ chunk_words, const uint32_t* __restrict__ chunk_zeros,
    const uint64_t* __restrict__ word_off, const uint64_t* __restrict__ zero_off,
    const uint32_t* __restrict__ slots, uint8_t* out, uint64_t cap, const Meta* __restrict__ m,
    uint32_t bid, uint32_t nblk) {
  EncTables& t = u.t;
  const EncWindow w = enc_window(m, R, enc_code, enc_len);
  const Layout l =
      stream_layout(m->nsym_used, nchunks, sub, m->n_unpred, sizeof(T), m->total_words);
  if (fast_path(w) || w.max_len <= 32) return;
  load_tables(t, w, nsym, enc_code, enc_len, true);
  __syncthreads();
  uint32_t* cw = const_cast<uint32_t*>(chunk_words);  // (read only without SLOTS)
  uint32_t* cz = const_cast<uint32_t*>(chunk_zeros);
  if (w.lds_only)
    pack_chunks<T, true, false>(codes, x, n, chunk, sub, nchunks, t, w, enc_code, enc_len, cw, cz,
                                word_off, zero_off, nullptr, l, out, cap, bid, nblk);
  else
    pack_chunks<T, false, false>(codes, x, n, chunk, sub, nchunks, t, w, enc_code, enc_len, cw, cz,
                                 word_off, zero_off, nullptr, l, out, cap, bid, nblk);
}

template <typename T>
__global__ __launch_bounds__(kEncWaves * 64) void k_encode_pack(
    const uint16_t* __restrict__ codes, const T* __restrict__ x, uint64_t n, uint32_t chunk,
    uint32_t sub, uint64_t nchunks, uint32_t R, uint32_t nsym, const uint64_t* __restrict__ enc_code,
    const uint8_t* __restrict__ enc_len, const uint32_t* __restrict__ chunk_words,
    const uint32_t* __restrict__ chunk_zeros, const uint64_t* __restrict__ word_off,
    const uint64_t* __restrict__ zero_off, const uint32_t* __restrict__ slots, uint8_t* out,
    uint64_t cap, const Meta* __restrict__ m) {
  __shared__ EncLds u;
  encode_pack_body<T>(u, codes, x, n, chunk, sub, nchunks, R, nsym, enc_code, enc_len, chunk_words,
                      chunk_zeros, word_off, zero_off, slots, out, cap, m, blockIdx.x, gridDim.x);
}

// the packing of every field of a batch, with the field-local chunk offsets
template <typename T>
__global__ __launch_bounds__(kEncWaves * 64) void k_b_encode_pack(BLaunch L) {
  __shared__ EncLds u;
  BJob j;
  uint32_t local;
  if (!batch_job(L, j, local)) return;
  const BField& f = L.f[j.field];
  encode_pack_body<T>(u, f.codes, static_cast<const T*>(f.x), f.n, f.chunk, f.sub, f.nchunks, f.R,
                      2 * f.R, f.enc_code, f.enc_len, f.chunk_words, f.chunk_zeros, f.lword_off,
                      f.lzero_off, static_cast<const uint32_t*>(f.rec), f.out, f.cap, f.m, local,
                      j.nblk);
}

// The second pass of the lane-parallel path: no LDS, a wave per chunk.
template <typename T>
__device__ __forceinline__ void encode_copy_body(
    const uint16_t* __restrict__ codes, const T* __restrict__ x, uint64_t n, uint32_t chunk,
    uint32_t sub, uint64_t nchunks, uint32_t R, const uint64_t* __restrict__ enc_code,
    const uint8_t* __restrict__ enc_len, const uint32_t* __restrict__ chunk_words,
    const uint32_t* __restrict__ chunk_zeros, const uint64_t* __restrict__ word_off,
    const uint64_t* __restrict__ zero_off, const uint32_t* __restrict__ slots, uint8_t* out,
    uint64_t cap, const Meta* __restrict__ m, uint32_t bid, uint32_t nblk) {
  const EncWindow w = enc_window(m, R, enc_code, enc_len);
  if (!fast_path(w) && w.max_len > 32) return;
  const Layout l =
      stream_layout(m->nsym_used, nchunks, sub, m->n_unpred, sizeof(T), m->total_words);
  copy_slots<T>(codes, x, n, chunk, nchunks, chunk_words, chunk_zeros, word_off, zero_off, slots, l,
                out, cap, bid, nblk);
}

template <typename T>
__global__ __launch_bounds__(kEncWaves * 64) void k_encode_copy(
    const uint16_t* __restrict__ codes, const T* __restrict__ x, uint64_t n, uint32_t chunk,
    uint32_t sub, uint64_t nchunks, uint32_t R, const uint64_t* __restrict__ enc_code,
    const uint8_t* __restrict__ enc_len, const uint32_t* __restrict__ chunk_words,
    const uint32_t* __restrict__ chunk_zeros, const uint64_t* __restrict__ word_off,
    const uint64_t* __restrict__ zero_off, const uint32_t* __restrict__ slots, uint8_t* out,
    uint64_t cap, const Meta* __restrict__ m) {
  encode_copy_body<T>(codes, x, n, chunk, sub, nchunks, R, enc_code, enc_len, chunk_words,
                      chunk_zeros, word_off, zero_off, slots, out, cap, m, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ __launch_bounds__(kEncWaves * 64) void k_b_encode_copy(BLaunch L) {
  BJob j;
  uint32_t local;
  if (!batch_job(L, j, local)) return;
  const BField& f = L.f[j.field];
  encode_copy_body<T>(f.codes, static_cast<const T*>(f.x), f.n, f.chunk, f.sub, f.nchunks, f.R,
                      f.enc_code, f.enc_len, f.chunk_words, f.chunk_zeros, f.lword_off, f.lzero_off,
                      static_cast<const uint32_t*>(f.rec), f.out, f.cap, f.m, local, j.nblk);
}

// workgroups of the second packing pass (codes over 32 bits only)
uint32_t encode_pack_blocks(uint64_t nchunks) {
  const uint64_t b = (nchunks + kEncWaves - 1) / kEncWaves;
  return (uint32_t)(b < 64 ? (b ? b : 1) : 64);
}

// workgroups of the copy pass: a wave per chunk
uint32_t encode_copy_blocks(uint64_t nchunks) {
  const uint64_t b = (nchunks + kEncWaves - 1) / kEncWaves;
  return (uint32_t)(b < 16384 ? (b ? b : 1) : 16384);
}

hipError_t launch_b_encode_copy(int dtype, BLaunch L, uint32_t nwg, hipStream_t st) {
  if (nwg == 0) return hipSuccess;
  if (dtype == SZ_F32)
    hipLaunchKernelGGL(k_b_encode_copy<float>, dim3(nwg), dim3(kEncWaves * 64), 0, st, L);
  else
    hipLaunchKernelGGL(k_b_encode_copy<double>, dim3(nwg), dim3(kEncWaves * 64), 0, st, L);
  return hipGetLastError();
}

hipError_t launch_encode(const uint16_t* codes, const void* x, int dtype, uint64_t n,
                         uint32_t chunk, uint32_t sub, uint32_t radius, const uint64_t* enc_code,
                         const uint8_t* enc_len, EncodeScratch es, uint32_t* slots, uint8_t* out,
                         uint64_t cap, Meta* m, hipStream_t st) {
  const uint64_t nchunks = (n + chunk - 1) / chunk;
  if (nchunks == 0) return hipSuccess;
  const uint32_t nsym = 2 * radius;
  uint64_t blocks = (nchunks + kEncWaves - 1) / kEncWaves;
  if (blocks > 2048) blocks = 2048;
  dim3 grid((unsigned)blocks);
  const dim3 block(kEncWaves * 64);
  hipLaunchKernelGGL(k_encode_size, grid, block, 0, st, codes, n, chunk, sub, nchunks, radius,
                     nsym, enc_code, enc_len, es.chunk_words, es.chunk_zeros, slots, out, cap, m);
  hipError_t e = launch_scan_pair(es.chunk_words, es.chunk_zeros, nchunks, es.word_off,
                                  es.zero_off, es.block_sums, &m->total_words, es.totals, st);
  if (e != hipSuccess) return e;
  // the second pass: the packing of codes over 32 bits (rare: a small grid),
  // or the slots' copy (each kernel returns at once when the other applies)
  const dim3 cgrid(encode_copy_blocks(nchunks));
  grid = dim3(encode_pack_blocks(nchunks));
  if (dtype == SZ_F32) {
    hipLaunchKernelGGL(k_encode_pack<float>, grid, block, 0, st, codes, (const float*)x, n, chunk,
                       sub, nchunks, radius, nsym, enc_code, enc_len, es.chunk_words,
                       es.chunk_zeros, es.word_off, es.zero_off, slots, out, cap, m);
    hipLaunchKernelGGL(k_encode_copy<float>, cgrid, block, 0, st, codes, (const float*)x, n, chunk,
                       sub, nchunks, radius, enc_code, enc_len, es.chunk_words, es.chunk_zeros,
                       es.word_off, es.zero_off, slots, out, cap, m);
  } else {
    hipLaunchKernelGGL(k_encode_pack<double>, grid, block, 0, st, codes, (const double*)x, n,
                       chunk, sub, nchunks, radius, nsym, enc_code, enc_len, es.chunk_words,
                       es.chunk_zeros, es.word_off, es.zero_off, slots, out, cap, m);
    hipLaunchKernelGGL(k_encode_copy<double>, cgrid, block, 0, st, codes, (const double*)x, n,
                       chunk, sub, nchunks, radius, enc_code, enc_len, es.chunk_words,
                       es.chunk_zeros, es.word_off, es.zero_off, slots, out, cap, m);
  }
  return hipGetLastError();
}

// Header (template from the host, patched with the device-side values),
// symbol table, and the zero padding that ends the symbol-table and
// unpredictable sections on 8-byte boundaries.
struct HeaderBytes {
  uint32_t w[kHeaderBytes / 4];
};

__device__ __forceinline__ void write_tables_body(uint8_t* out, uint64_t cap,
                                                  const uint32_t* __restrict__ symtab,
                                                  uint64_t nchunks, uint32_t sub,
                                                  const uint32_t* hdr, uint32_t tsize, Meta* m,
                                                  uint32_t bid, uint32_t nblk) {
  const uint64_t K = m->nsym_used;
  const Layout l = stream_layout(K, nchunks, sub, m->n_unpred, tsize, m->total_words);
  const uint64_t gid = bid * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t gs = (uint64_t)nblk * blockDim.x;
  if (gid < kHeaderBytes / 4) {
    // header word gid; the device-side fields are 8-byte values at 56, 72,
    // 80 (K, then the sub-chunk count from the template), 88 and 96
    const uint32_t byte = (uint32_t)gid * 4;
    uint64_t v64 = 0;
    bool patched = true;
    const uint32_t at = byte & ~7u;
    if (at == 56) {
      const double eb = m->eb;
      __builtin_memcpy(&v64, &eb, 8);
    } else if (at == 72) {
      v64 = m->n_unpred;
    } else if (at == 80) {
      v64 = K | ((uint64_t)hdr[84 / 4] << 32);
    } else if (at == 88) {
      v64 = m->total_words;
    } else if (at == 96) {
      v64 = l.size;
    } else {
      patched = false;
    }
    const uint32_t word = patched ? (uint32_t)(v64 >> ((byte & 4) ? 32 : 0)) : hdr[gid];
    guarded_store_u32(out, cap, byte, word);
  }
  if (gid == 0) {
    if (K & 1) guarded_store_u32(out, cap, l.off_sym + 4 * K, 0u);
    if ((nchunks * (sub - 1)) & 1) guarded_store_u32(out, cap, l.off_sub + 4 * nchunks * (sub - 1), 0u);
    const uint64_t ub = m->n_unpred * tsize;
    if (ub & 7) guarded_store_u32(out, cap, l.off_unpred + ub, 0u);
    m->stream_bytes = l.size;
  }
  for (uint64_t i = gid; i < K; i += gs) guarded_store_u32(out, cap, l.off_sym + 4 * i, symtab[i]);
}

__global__ __launch_bounds__(256) void k_write_tables(uint8_t* out, uint64_t cap,
                                                      const uint32_t* __restrict__ symtab,
                                                      uint64_t nchunks, uint32_t sub,
                                                      HeaderBytes hdr, uint32_t tsize, Meta* m) {
  write_tables_body(out, cap, symtab, nchunks, sub, hdr.w, tsize, m, blockIdx.x, gridDim.x);
}

// the header and symbol table of every field of a batch
__global__ __launch_bounds__(256) void k_b_write_tables(BLaunch L) {
  BJob j;
  uint32_t local;
  if (!batch_job(L, j, local)) return;
  const BField& f = L.f[j.field];
  write_tables_body(f.out, f.cap, f.symtab, f.nchunks, f.sub, f.hdr, f.dtype == SZ_F32 ? 4u : 8u,
                    f.m, local, j.nblk);
}

hipError_t launch_b_write_tables(BLaunch L, uint32_t nwg, hipStream_t st) {
  if (nwg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_write_tables, dim3(nwg), dim3(256), 0, st, L);
  return hipGetLastError();
}

hipError_t launch_b_encode_size(BLaunch L, uint32_t nwg, hipStream_t st) {
  if (nwg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_encode_size, dim3(nwg), dim3(kEncWaves * 64), 0, st, L);
  return hipGetLastError();
}

hipError_t launch_b_encode_pack(int dtype, BLaunch L, uint32_t nwg, hipStream_t st) {
  if (nwg == 0) return hipSuccess;
  if (dtype == SZ_F32)
    hipLaunchKernelGGL(k_b_encode_pack<float>, dim3(nwg), dim3(kEncWaves * 64), 0, st, L);
  else
    hipLaunchKernelGGL(k_b_encode_pack<double>, dim3(nwg), dim3(kEncWaves * 64), 0, st, L);
  return hipGetLastError();
}

// Field-local chunk offsets: the batch-wide exclusive scans minus the value
// at the field's first chunk; the field's totals (bitstream words) from its
// last chunk.  One job per field.
__global__ __launch_bounds__(256) void k_b_rebase(BLaunch L) {
  BJob j;
  uint32_t local;
  if (!batch_job(L, j, local)) return;
  const BField& f = L.f[j.field];
  const uint64_t wb = f.word_off[0], zb = f.zero_off[0];
  for (uint64_t c = local * (uint64_t)blockDim.x + threadIdx.x; c < f.nchunks;
       c += (uint64_t)j.nblk * blockDim.x) {
    f.lword_off[c] = f.word_off[c] - wb;
    f.lzero_off[c] = f.zero_off[c] - zb;
  }
  if (local == 0 && threadIdx.x == 0 && f.nchunks)
    f.m->total_words = f.word_off[f.nchunks - 1] + f.chunk_words[f.nchunks - 1] - wb;
}

hipError_t launch_b_rebase(BLaunch L, uint32_t nwg, hipStream_t st) {
  if (nwg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_rebase, dim3(nwg), dim3(256), 0, st, L);
  return hipGetLastError();
}

// (stream bytes, status) of every field, gathered for one copy to the host
__global__ void k_b_results(const BField* __restrict__ f, uint32_t nf, uint64_t* res) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  res[2 * i] = f[i].m->stream_bytes;
  res[2 * i + 1] = f[i].m->status;
}

hipError_t launch_b_results(const BField* f, uint32_t nf, uint64_t* res, hipStream_t st) {
  if (nf == 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_results, dim3((nf + 255) / 256), dim3(256), 0, st, f, nf, res);
  return hipGetLastError();
}

hipError_t launch_write_tables(uint8_t* out, uint64_t capacity, const uint32_t* symtab,
                               uint64_t nchunks, uint32_t sub, const uint8_t* header_template,
                               int dtype, Meta* m, hipStream_t st) {
  HeaderBytes h;
  for (int i = 0; i < (int)(kHeaderBytes / 4); i++)
    h.w[i] = header_template[4 * i] | (header_template[4 * i + 1] << 8) |
             (header_template[4 * i + 2] << 16) | ((uint32_t)header_template[4 * i + 3] << 24);
  hipLaunchKernelGGL(k_write_tables, dim3(16), dim3(256), 0, st, out, capacity, symtab, nchunks,
                     sub, h, dtype == SZ_F32 ? 4u : 8u, m);
  return hipGetLastError();
}

}  // namespace szg
