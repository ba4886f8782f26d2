// C ABI (include/szg.h): context, scratch, stream header, and the drivers that
// enqueue the compression and decompression kernels.
//
// Stream layout (little-endian; sections start on 8-byte boundaries):
//   header, 128 bytes
//     0 "SZG1"  4 u16 version=1  6 u8 dtype  7 u8 ndim  8 u64 dims[4] (unused=1)
//     40 u8 predictor  41 u8 dim_order[4]  45 u8 eb_mode  46 u16 0
//     48 f64 eb as passed  56 f64 eb in the field type  64 u32 radius
//     68 u32 chunk  72 u64 unpredictable count  80 u32 K (coded symbols)
//     84 u32 sub-chunks per chunk
//     88 u64 bitstream words  96 u64 stream bytes  104..127 0
//   symbol table   K x u32 (symbol | length << 16), ascending symbol
//                  (the encoder's saved state, Algorithm 1 "encoder.save")
//   chunk table    ceil(n/chunk) x (u32 words, u32 unpredictable count)
//   sub-chunks     ceil(n/chunk) x (sub - 1) x u32: bit offset of sub-chunks
//                  1..sub-1 from the chunk's first bit
//   unpredictable  count x T in flat order (Algorithm 1 "quantizer.save")
//   bitstream      words x u32, each chunk MSB-first and word-padded
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

using namespace szg;

// The size-dependent scratch of sz_compress_noalloc, for callers that cannot
// allocate device memory.  Host code never uses this name as a device address:
// each device's copy is reached through the address hipGetSymbolAddress gives
// for it, taken once per device when the first context on it is created.
constexpr size_t kNoAllocScratchBytes = SZ_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

struct Pending {
  const char* name;
  hipEvent_t a, b;
};

struct Stat {
  double ms = 0;
  uint64_t n = 0;
};

}  // namespace

struct sz_ctx {
  int device = 0;
  std::string err;
  // size-dependent scratch
  Buf rec, codes, chunk_words, chunk_unpred, word_off, unpred_off, block_sums;
  Buf ylog, signs;  // point-wise relative mode: the log field and the sign words
  Buf coarse;       // the stride-2 lattice for the strip kernel of the stride-1 level
  // fixed scratch
  Meta* meta = nullptr;
  uint32_t* hist = nullptr;
  uint32_t* hist_part = nullptr;  // partial-histogram rows
  uint64_t* enc_code = nullptr;
  uint8_t* enc_len = nullptr;
  uint32_t* symtab = nullptr;
  uint64_t* totals = nullptr;
  // adaptive interpolation: the orders' sampled sums ([order][level][linear,
  // cubic], or the candidate buckets), then the chosen order's level sums
  // and the order chosen on the device
  uint64_t* lvl_cost = nullptr;
  CodebookScratch cb{};
  DecodeTables dt{};
  uint64_t* mm_part = nullptr;  // the range pass's per-workgroup keys (2 x kMinmaxBlocks)
  Meta* h_meta = nullptr;       // pinned
  uint64_t* h_lvl = nullptr;    // pinned: the adaptive level sums, then the device's order choice
  uint8_t* h_header = nullptr;  // pinned
  uint64_t last_n = 0;
  const uint16_t* last_codes = nullptr;  // the codes of the last compression
  // plans of the levels and passes, reserved at creation so that planning a
  // call allocates nothing
  std::vector<LevelGeom> levels;
  std::vector<PassGeom> passes;
  // sz_compress_noalloc: this device's static scratch (its device address),
  // or the reason it is unavailable; that entry point records no events
  void* noalloc_scratch = nullptr;
  std::string noalloc_err;
  bool no_timing = false;
  BatchPlan* batch = nullptr;  // sz_compress_batch's plan for the last batch shapes
  // one launch per level (fields of up to three dimensions) instead of one
  // per (level, dimension) pass; SZG_FUSED_LEVELS=0 selects the pass kernels
  bool fused_levels = true;
  // timing
  bool timing = false;
  std::string timing_family;  // the one family timed; empty: every family
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  std::map<std::string, Stat> stats;
  hipEvent_t done = nullptr;  // marks the end of a call's work for the host to wait on
  hipEvent_t header = nullptr;  // marks a stream's header copied to the host
  // the rows that price the dimension orders (est_row_sampled) for one shape
  Buf est_rows;
  uint64_t est_nrows = 0;
  std::array<uint64_t, kMaxDims> est_dims{};
  int est_ndim = 0;
};

namespace {

int fail(sz_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int dev_fail(sz_ctx* c, hipError_t e, const char* where) {
  return fail(c, SZ_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define CHECK_HIP(expr, where)                 \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return dev_fail(ctx, e_, where); \
  } while (0)

hipError_t ensure(Buf& b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (b.cap >= bytes) return hipSuccess;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
  size_t want = bytes + bytes / 8;
  hipError_t e = hipMalloc(&b.p, want);
  if (e == hipSuccess) b.cap = want;
  return e;
}

hipEvent_t get_event(sz_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// The host's waits for the device (the header of a stream, a call's sizes and
// status): a marker on the stream, polled for up to kSpinMicros (the wait is
// usually a few tens of microseconds, and a blocking wait adds its wake-up
// time to every call), then waited for by blocking.
constexpr int kSpinMicros = 500;
constexpr int kSpinLongMicros = 2000;  // (a wait behind the whole adaptive estimate)
hipError_t mark(hipEvent_t& ev, hipStream_t st) {
  if (!ev) {
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  return hipEventRecord(ev, st);
}
hipError_t wait_mark(hipEvent_t ev, int spin_us = kSpinMicros) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t e = hipEventQuery(ev);
    if (e != hipErrorNotReady) return e;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(spin_us))
      return hipEventSynchronize(ev);
  }
}
hipError_t wait_stream(sz_ctx* c, hipStream_t st, int spin_us = kSpinMicros) {
  hipError_t e = mark(c->done, st);
  return e == hipSuccess ? wait_mark(c->done, spin_us) : e;
}

template <class F>
hipError_t timed(sz_ctx* c, const char* name, hipStream_t st, F&& f) {
  if (!c->timing || c->no_timing || (!c->timing_family.empty() && c->timing_family != name))
    return f();
  hipEvent_t a = get_event(c), b = get_event(c);
  (void)hipEventRecord(a, st);
  hipError_t e = f();
  (void)hipEventRecord(b, st);
  c->pending.push_back({name, a, b});
  return e;
}

void settle_timing(sz_ctx* c) {
  for (auto& p : c->pending) {
    (void)hipEventSynchronize(p.b);
    float ms = 0;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      Stat& s = c->stats[p.name];
      s.ms += ms;
      s.n += 1;
    }
    c->event_pool.push_back(p.a);
    c->event_pool.push_back(p.b);
  }
  c->pending.clear();
}

// ---------------------------------------------------------------- shapes

struct Shape {
  int dtype = 0, ndim = 0;
  uint64_t dims[kMaxDims] = {1, 1, 1, 1};
  uint8_t order[kMaxDims] = {0, 1, 2, 3};
  uint64_t n = 0;
  uint32_t radius = kMaxRadius, chunk = 4096, sub = 0;
  size_t tsize() const { return dtype == SZ_F64 ? 8 : 4; }
  uint64_t nchunks() const { return (n + chunk - 1) / chunk; }
};

bool valid_order(int ndim, const uint8_t* order) {
  bool seen[kMaxDims] = {false, false, false, false};
  for (int j = 0; j < ndim; j++) {
    if (order[j] >= ndim || seen[order[j]]) return false;
    seen[order[j]] = true;
  }
  return true;
}

// Validates shape and options shared by compress and the bound.
int make_shape(sz_ctx* c, int dtype, int ndim, const uint64_t* dims, const sz_options* opts,
               Shape* s) {
  if (dtype != SZ_F32 && dtype != SZ_F64) return fail(c, SZ_ERR_DTYPE, "dtype must be SZ_F32 or SZ_F64");
  if (ndim < 1 || ndim > kMaxDims || !dims) return fail(c, SZ_ERR_ARG, "ndim must be 1..4 with dims");
  s->dtype = dtype;
  s->ndim = ndim;
  bool empty = false;
  for (int d = 0; d < ndim; d++) {
    s->dims[d] = dims[d];
    if (dims[d] == 0) empty = true;
  }
  uint64_t n = 1;
  if (empty) {
    n = 0;
  } else {
    for (int d = 0; d < ndim; d++) {
      if (dims[d] > kMaxPoints || n > kMaxPoints / dims[d])
        return fail(c, SZ_ERR_ARG, "field has more than 2^32-1 points");
      n *= dims[d];
    }
  }
  s->n = n;
  if (opts) {
    s->radius = opts->radius;
    s->chunk = opts->chunk;
    s->sub = opts->subchunks;
    for (int j = 0; j < kMaxDims; j++) s->order[j] = j < ndim ? opts->dim_order[j] : (uint8_t)j;
  }
  if (s->radius < 1 || s->radius > kMaxRadius) return fail(c, SZ_ERR_ARG, "radius must be 1..32768");
  if (s->chunk < 64 || s->chunk > 65536 || (s->chunk & 63))
    return fail(c, SZ_ERR_ARG, "chunk must be a multiple of 64 in [64, 65536]");
  if (s->sub == 0) s->sub = default_sub(s->chunk);
  if (!valid_sub(s->chunk, s->sub))
    return fail(c, SZ_ERR_ARG, "subchunks must be 1, or 2, 4 or 8 splitting chunk into whole encoder runs");
  if (!valid_order(ndim, s->order)) return fail(c, SZ_ERR_ARG, "dim_order must be a permutation");
  return SZ_OK;
}

// The (level, dimension) passes of the multilevel traversal in execution
// order: levels L..1 with stride s = 2^(l-1), and inside a level the
// dimensions in `order`.  The origin is handled separately.
void build_passes(const Shape& s, std::vector<PassGeom>& out) {
  out.clear();
  const int L = level_count(s.ndim, s.dims);
  uint64_t stride[kMaxDims];
  uint64_t st = 1;
  for (int d = s.ndim - 1; d >= 0; d--) {
    stride[d] = st;
    st *= s.dims[d];
  }
  int pos[kMaxDims];
  for (int j = 0; j < s.ndim; j++) pos[s.order[j]] = j;
  for (int l = L; l >= 1; l--) {
    uint64_t sp = 1ull << (l - 1);
    for (int j = 0; j < s.ndim; j++) {
      PassGeom g{};
      g.ndim = s.ndim;
      g.d = s.order[j];
      g.s = (uint32_t)sp;
      g.nd = (uint32_t)s.dims[g.d];
      g.total = 1;
      for (int e = 0; e < s.ndim; e++) {
        uint64_t start = 0, step = 2 * sp;
        if (e == g.d)
          start = sp;
        else if (pos[e] < j)
          step = sp;
        g.start[e] = start;
        g.step[e] = step;
        g.cnt[e] = start < s.dims[e] ? (uint32_t)((s.dims[e] - start + step - 1) / step) : 0;
        g.stride[e] = stride[e];
        g.total *= g.cnt[e];
      }
      if (g.total) out.push_back(g);
    }
  }
}

void put_le(uint8_t* p, uint64_t v, int bytes) {
  for (int i = 0; i < bytes; i++) p[i] = (uint8_t)(v >> (8 * i));
}
uint64_t get_le(const uint8_t* p, int bytes) {
  uint64_t v = 0;
  for (int i = bytes - 1; i >= 0; i--) v = (v << 8) | p[i];
  return v;
}

void header_template(const Shape& s, int predictor, int eb_mode, double eb_user, uint8_t* h) {
  memset(h, 0, kHeaderBytes);
  memcpy(h, "SZG1", 4);
  put_le(h + 4, 1, 2);
  h[6] = (uint8_t)s.dtype;
  h[7] = (uint8_t)s.ndim;
  for (int d = 0; d < kMaxDims; d++) put_le(h + 8 + 8 * d, d < s.ndim ? s.dims[d] : 1, 8);
  h[40] = (uint8_t)predictor;
  for (int d = 0; d < kMaxDims; d++) h[41 + d] = s.order[d];
  h[45] = (uint8_t)eb_mode;
  uint64_t u;
  memcpy(&u, &eb_user, 8);
  put_le(h + 48, u, 8);
  put_le(h + 64, s.radius, 4);
  put_le(h + 68, s.chunk, 4);
  put_le(h + 84, s.sub, 4);
}

int parse_header(const uint8_t* h, sz_info* info) {
  if (memcmp(h, "SZG1", 4) != 0 || get_le(h + 4, 2) != 1) return SZ_ERR_CORRUPT;
  sz_info in{};
  in.dtype = h[6];
  in.ndim = h[7];
  in.predictor = h[40];
  in.eb_mode = h[45];
  if (in.dtype > 1 || in.ndim < 1 || in.ndim > kMaxDims || in.predictor > 3 || in.eb_mode > 2)
    return SZ_ERR_CORRUPT;
  // adaptive interpolation: bit l - 1 of the level mask set = level l cubic
  in.level_mask = (uint32_t)get_le(h + 124, 4);
  // point-wise relative mode: the coded field holds the logarithms (f64);
  // bytes 104.. give the field's own dtype and the sign section
  const bool pw = in.eb_mode == SZ_EB_PWREL;
  in.coded_dtype = in.dtype;
  in.signs = 0;
  in.off_signs = 0;
  if (pw) {
    if (in.coded_dtype != SZ_F64 || h[104] > 1 || h[105] > 1) return SZ_ERR_CORRUPT;
    for (int k = 106; k < 112; k++)
      if (h[k]) return SZ_ERR_CORRUPT;
    for (int k = 120; k < 124; k++)
      if (h[k]) return SZ_ERR_CORRUPT;
    in.dtype = h[104];
    in.signs = h[105];
    in.off_signs = get_le(h + 112, 8);
  }
  uint64_t n = 1;
  bool empty = false;
  for (int d = 0; d < kMaxDims; d++) {
    in.dims[d] = get_le(h + 8 + 8 * d, 8);
    in.dim_order[d] = h[41 + d];
    if (d >= in.ndim && (in.dims[d] != 1 || in.dim_order[d] != d)) return SZ_ERR_CORRUPT;
    if (d < in.ndim && in.dims[d] == 0) empty = true;
  }
  if (!valid_order(in.ndim, in.dim_order)) return SZ_ERR_CORRUPT;
  if (in.predictor == SZ_LORENZO)  // (flat order: no dimension order)
    for (int j = 0; j < in.ndim; j++)
      if (in.dim_order[j] != j) return SZ_ERR_CORRUPT;
  if (empty) {
    n = 0;
  } else {
    for (int d = 0; d < in.ndim; d++) {
      if (in.dims[d] > kMaxPoints || n > kMaxPoints / in.dims[d]) return SZ_ERR_CORRUPT;
      n *= in.dims[d];
    }
  }
  in.n = n;
  {
    const int L = level_count(in.ndim, in.dims);
    if (in.predictor == SZ_INTERP_ADAPTIVE ? (L < 32 && (in.level_mask >> L) != 0)
                                           : in.level_mask != 0)
      return SZ_ERR_CORRUPT;
  }
  uint64_t u = get_le(h + 48, 8);
  memcpy(&in.eb_user, &u, 8);
  u = get_le(h + 56, 8);
  memcpy(&in.eb, &u, 8);
  in.radius = (uint32_t)get_le(h + 64, 4);
  in.chunk = (uint32_t)get_le(h + 68, 4);
  in.n_unpred = get_le(h + 72, 8);
  in.nsym = (uint32_t)get_le(h + 80, 4);
  in.sub = (uint32_t)get_le(h + 84, 4);
  in.total_words = get_le(h + 88, 8);
  in.stream_bytes = get_le(h + 96, 8);
  if (!(in.eb >= 0.0) || !__builtin_isfinite(in.eb)) return SZ_ERR_CORRUPT;
  if (in.coded_dtype == SZ_F32 && (double)(float)in.eb != in.eb) return SZ_ERR_CORRUPT;
  if (in.radius < 1 || in.radius > kMaxRadius || in.chunk == 0) return SZ_ERR_CORRUPT;
  if (!valid_sub(in.chunk, in.sub)) return SZ_ERR_CORRUPT;
  if (in.nsym > 2 * in.radius || in.n_unpred > n || (in.nsym == 0) != (n == 0)) return SZ_ERR_CORRUPT;
  if (in.total_words > 64 * (n + 1)) return SZ_ERR_CORRUPT;
  uint64_t nchunks = (n + in.chunk - 1) / in.chunk;
  Layout l = stream_layout(in.nsym, nchunks, in.sub, in.n_unpred, in.coded_dtype == SZ_F64 ? 8 : 4,
                           in.total_words);
  if (pw && in.signs) {
    if (in.off_signs != pad8(l.size) || in.stream_bytes != in.off_signs + 8 * ((n + 63) / 64))
      return SZ_ERR_CORRUPT;
  } else if (in.off_signs != 0 || l.size != in.stream_bytes) {
    return SZ_ERR_CORRUPT;
  }
  *info = in;
  return SZ_OK;
}

int ensure_fixed(sz_ctx* ctx) {
  if (ctx->meta) return SZ_OK;
  CHECK_HIP(hipMalloc(&ctx->meta, sizeof(Meta)), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->hist, sizeof(uint32_t) * kMaxSym), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->hist_part, histogram_scratch_bytes()), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->enc_code, sizeof(uint64_t) * kMaxSym), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->enc_len, kMaxSym), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->symtab, sizeof(uint32_t) * kMaxSym), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->totals, sizeof(uint64_t) * 4), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->lvl_cost, sizeof(uint64_t) * (kCandBuckets + 2 * kMaxLevels + 1)),
            "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->mm_part, sizeof(uint64_t) * 2 * kMinmaxBlocks), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->cb.keys_a, sizeof(uint64_t) * kMaxSym), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->cb.keys_b, sizeof(uint64_t) * kMaxSym), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->cb.w, sizeof(uint32_t) * 2 * kMaxSym), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->cb.parent, sizeof(uint32_t) * 2 * kMaxSym), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->cb.depth, sizeof(uint32_t) * 2 * kMaxSym), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->cb.merged, sizeof(uint32_t) * kMaxSym), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->cb.phase_end, sizeof(uint32_t) * kMaxSym), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->cb.leaf_sym, sizeof(uint16_t) * kMaxSym), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->dt.lut, sizeof(uint32_t) << kLutBits), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->dt.lut2, sizeof(uint64_t) << kLutBits), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->dt.l2, sizeof(uint32_t) * kL2Prefixes * kL2Entries), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->dt.lc, sizeof(LongCodes)), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->dt.first, sizeof(uint64_t) * (kMaxCodeLen + 2)), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->dt.count, sizeof(uint32_t) * (kMaxCodeLen + 2)), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->dt.offset, sizeof(uint32_t) * (kMaxCodeLen + 2)), "hipMalloc");
  CHECK_HIP(hipMalloc(&ctx->dt.sorted_sym, sizeof(uint16_t) * kMaxSym), "hipMalloc");
  ctx->dt.keys_a = ctx->cb.keys_a;
  ctx->dt.keys_b = ctx->cb.keys_b;
  CHECK_HIP(hipHostMalloc((void**)&ctx->h_meta, sizeof(Meta), hipHostMallocDefault), "hipHostMalloc");
  CHECK_HIP(hipHostMalloc((void**)&ctx->h_lvl, sizeof(uint64_t) * (2 * kMaxLevels + 1),
                          hipHostMallocDefault), "hipHostMalloc");
  // the host's markers, made here so that no call creates them
  CHECK_HIP(hipEventCreateWithFlags(&ctx->done, hipEventDisableTiming), "hipEventCreate");
  CHECK_HIP(hipEventCreateWithFlags(&ctx->header, hipEventDisableTiming), "hipEventCreate");
  CHECK_HIP(hipHostMalloc((void**)&ctx->h_header, kHeaderBytes, hipHostMallocDefault), "hipHostMalloc");
  return SZ_OK;
}

int ensure_sized(sz_ctx* ctx, const Shape& s, bool need_rec) {
  uint64_t nch = s.nchunks();
  if (need_rec) CHECK_HIP(ensure(ctx->rec, s.n * s.tsize()), "hipMalloc(rec)");
  // whole 8-code vectors: the encoder reads the last one unmasked
  CHECK_HIP(ensure(ctx->codes, ((s.n + 7) & ~7ull) * 2), "hipMalloc(codes)");
  CHECK_HIP(ensure(ctx->chunk_words, nch * 4), "hipMalloc");
  CHECK_HIP(ensure(ctx->chunk_unpred, nch * 4), "hipMalloc");
  CHECK_HIP(ensure(ctx->word_off, nch * 8), "hipMalloc");
  CHECK_HIP(ensure(ctx->unpred_off, nch * 8), "hipMalloc");
  CHECK_HIP(ensure(ctx->block_sums, (2 * ((nch + 1023) / 1024) + 1) * 8), "hipMalloc");

  return SZ_OK;
}

// The size-dependent scratch of one compression.
struct Work {
  void* rec = nullptr;
  uint16_t* codes = nullptr;
  uint32_t* chunk_words = nullptr;
  uint32_t* chunk_unpred = nullptr;
  uint64_t* word_off = nullptr;
  uint64_t* unpred_off = nullptr;
  uint64_t* block_sums = nullptr;
  void* coarse = nullptr;  // the stride-2 lattice, when taken from the static scratch
};

uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

// Lays the pieces of Work out from `base` (each 256-byte aligned) and returns
// their bytes: reconstruction, codes (whole 8-code vectors), the four chunk
// tables, the scan's block sums, and room for the stride-2 lattice of a
// three-dimensional field (the product of ceil(n_d / 2), whatever the order).
uint64_t carve_work(const Shape& s, uint8_t* base, Work* w) {
  const uint64_t nch = s.nchunks();
  uint64_t lattice = 0;
  if (s.ndim == 3)
    lattice = ((s.dims[0] + 1) / 2) * ((s.dims[1] + 1) / 2) * ((s.dims[2] + 1) / 2) * s.tsize();
  const uint64_t bytes[8] = {s.n * s.tsize(), ((s.n + 7) & ~7ull) * 2, nch * 4, nch * 4, nch * 8,
                             nch * 8, (2 * ((nch + 1023) / 1024) + 1) * 8, lattice};
  void** slot[8] = {&w->rec, (void**)&w->codes, (void**)&w->chunk_words, (void**)&w->chunk_unpred,
                    (void**)&w->word_off, (void**)&w->unpred_off, (void**)&w->block_sums,
                    &w->coarse};
  uint64_t off = 0;
  for (int i = 0; i < 8; i++) {
    *slot[i] = base ? base + off : nullptr;
    off += align256(bytes[i] ? bytes[i] : 8);
  }
  return off;
}

// Work from the context's buffers (grown on demand), or for the
// no-allocation entry point from this device's static scratch.
int acquire_work(sz_ctx* ctx, const Shape& s, bool noalloc, Work* w) {
  if (noalloc) {
    if (!ctx->noalloc_scratch)
      return fail(ctx, SZ_ERR_DEVICE, "static scratch unavailable: " + ctx->noalloc_err);
    const uint64_t need = carve_work(s, nullptr, w);
    if (need > kNoAllocScratchBytes)
      return fail(ctx, SZ_ERR_NOMEM,
                  "sz_compress_noalloc: the field needs " + std::to_string(need) +
                      " bytes of scratch, more than the " + std::to_string(kNoAllocScratchBytes) +
                      " its static buffer holds");
    carve_work(s, static_cast<uint8_t*>(ctx->noalloc_scratch), w);
    return SZ_OK;
  }
  int rc = ensure_sized(ctx, s, true);
  if (rc) return rc;
  w->rec = ctx->rec.p;
  w->codes = static_cast<uint16_t*>(ctx->codes.p);
  w->chunk_words = static_cast<uint32_t*>(ctx->chunk_words.p);
  w->chunk_unpred = static_cast<uint32_t*>(ctx->chunk_unpred.p);
  w->word_off = static_cast<uint64_t*>(ctx->word_off.p);
  w->unpred_off = static_cast<uint64_t*>(ctx->unpred_off.p);
  w->block_sums = static_cast<uint64_t*>(ctx->block_sums.p);
  w->coarse = nullptr;
  return SZ_OK;
}

// Each device's static scratch, looked up once per device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_tried[kMaxDevices] = {};

// Called with `device` current.
void bind_static_scratch(sz_ctx* ctx, int device) {
  if (device >= kMaxDevices) {
    ctx->noalloc_err = "device index above " + std::to_string(kMaxDevices - 1);
    return;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_tried[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
    g_scratch_tried[device] = true;
  }
  ctx->noalloc_scratch = g_scratch_ptr[device];
  if (!ctx->noalloc_scratch)
    ctx->noalloc_err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(g_scratch_err[device]);
}

}  // namespace

// ---- scratch accounting for the server (server.hip)

namespace szg {

// The number of levels: L = max over dimensions of ceil(log2 n_d).
int level_count(int ndim, const uint64_t* dims) {
  int L = 0;
  for (int d = 0; d < ndim; d++) {
    int l = 0;
    while (l < 63 && (1ull << l) < dims[d]) l++;
    L = l > L ? l : L;
  }
  return L;
}

// The stride-2 level stores its lattice compactly for the strip kernel when
// both run: the stride-1 level takes the strip kernel and the stride-2 level
// the fixed-pitch kernel (not the coarsest-levels workgroup).  Returns the
// lattice's bytes, 0 if not.
uint64_t compact_bytes(const std::vector<LevelGeom>& levels, int dtype, const void* x,
                       const void* v, uint64_t s_small, size_t tsize) {
  const LevelGeom* g1 = nullptr;
  const LevelGeom* g2 = nullptr;
  for (const LevelGeom& g : levels) {
    if (g.s == 1) g1 = &g;
    if (g.s == 2) g2 = &g;
  }
  if (!g1 || !g2 || s_small <= 2 || !g2->pitch64 || !fine_usable(*g1, dtype, x, v)) return 0;
  return (uint64_t)g2->ext[0] * g2->ext[1] * g2->ext[2] * tsize;
}

// bit l - 1 set: level l takes the cubic predictor
uint32_t cubic_mask(const int* lvl_pred) {
  uint32_t m = 0;
  for (int l = 1; l <= kMaxLevels; l++)
    if (lvl_pred[l] == SZ_INTERP_CUBIC) m |= 1u << (l - 1);
  return m;
}

size_t pwrel_scratch_need(uint64_t n, bool compress) {
  auto grown = [](uint64_t b) { return b + b / 8; };
  return (size_t)(grown(n * 8) + (compress ? grown(((n + 63) / 64) * 8) : 0));
}

size_t scratch_need(uint64_t n, size_t tsize, uint32_t chunk, bool compress) {
  auto grown = [](uint64_t b) { return b + b / 8; };  // what ensure() allocates
  const uint64_t nch = chunk ? (n + chunk - 1) / chunk : 0;
  uint64_t total = grown(((n + 7) & ~7ull) * 2) + 2 * grown(nch * 4) + 2 * grown(nch * 8) +
                   grown((2 * ((nch + 1023) / 1024) + 1) * 8);
  if (compress) total += grown(n * tsize);
  // the stride-2 lattice of a field the strip kernel takes: below n / 3 points
  // (extents >= 2, 2 and 4)
  total += grown((n / 3 + 1) * tsize);
  return (size_t)total;
}

size_t ctx_scratch_bytes(const sz_ctx* ctx) {
  size_t t = 0;
  for (const Buf* b : {&ctx->rec, &ctx->codes, &ctx->chunk_words, &ctx->chunk_unpred,
                       &ctx->word_off, &ctx->unpred_off, &ctx->block_sums, &ctx->ylog,
                       &ctx->signs, &ctx->coarse, &ctx->est_rows})
    t += b->cap;
  return t;
}

void ctx_trim(sz_ctx* ctx) {
  (void)hipSetDevice(ctx->device);
  for (Buf* b : {&ctx->rec, &ctx->codes, &ctx->chunk_words, &ctx->chunk_unpred, &ctx->word_off,
                 &ctx->unpred_off, &ctx->block_sums, &ctx->ylog, &ctx->signs, &ctx->coarse,
                 &ctx->est_rows}) {
    if (b->p) (void)hipFree(b->p);
    b->p = nullptr;
    b->cap = 0;
  }
  ctx->est_ndim = 0;
}

size_t ctx_fixed_bytes() {
  return sizeof(Meta) + sizeof(uint32_t) * kMaxSym * 2 + histogram_scratch_bytes() +
         (sizeof(uint64_t) + 1) * kMaxSym + sizeof(uint64_t) * 4 + sizeof(uint64_t) * 2 * kMaxLevels * kMaxOrders +
         sizeof(uint64_t) * kMaxSym * 2 + sizeof(uint32_t) * kMaxSym * 9 + sizeof(uint16_t) * kMaxSym +
         (sizeof(uint32_t) << kLutBits) + (sizeof(uint64_t) << kLutBits) + sizeof(LongCodes) + 16 * (kMaxCodeLen + 2) +
         sizeof(uint16_t) * kMaxSym;
}

}  // namespace szg

extern "C" {

sz_ctx* sz_ctx_create(int device) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return nullptr;
  if (hipSetDevice(device) != hipSuccess) return nullptr;
  sz_ctx* ctx = new sz_ctx();
  ctx->device = device;
  if (const char* e = getenv("SZG_FUSED_LEVELS")) ctx->fused_levels = strcmp(e, "0") != 0;
  if (ensure_fixed(ctx) != SZ_OK) {
    sz_ctx_destroy(ctx);
    return nullptr;
  }
  ctx->levels.reserve(kMaxLevels);
  ctx->passes.reserve(kMaxLevels * kMaxDims);
  bind_static_scratch(ctx, device);
  return ctx;
}

void sz_ctx_destroy(sz_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  batch_plan_free(ctx->batch);
  for (Buf* b : {&ctx->rec, &ctx->codes, &ctx->chunk_words, &ctx->chunk_unpred, &ctx->word_off,
                 &ctx->unpred_off, &ctx->block_sums, &ctx->ylog, &ctx->signs, &ctx->coarse,
                 &ctx->est_rows})
    if (b->p) (void)hipFree(b->p);
  void* fixed[] = {ctx->meta, ctx->hist, ctx->hist_part, ctx->enc_code, ctx->enc_len, ctx->symtab, ctx->totals,
                   ctx->lvl_cost, ctx->mm_part,
                   ctx->cb.keys_a, ctx->cb.keys_b, ctx->cb.w, ctx->cb.parent, ctx->cb.depth,
                   ctx->cb.merged, ctx->cb.phase_end, ctx->cb.leaf_sym, ctx->dt.lut, ctx->dt.lut2, ctx->dt.l2, ctx->dt.lc,
                   ctx->dt.first, ctx->dt.count, ctx->dt.offset, ctx->dt.sorted_sym};
  for (void* p : fixed)
    if (p) (void)hipFree(p);
  if (ctx->h_meta) (void)hipHostFree(ctx->h_meta);
  if (ctx->h_lvl) (void)hipHostFree(ctx->h_lvl);
  if (ctx->h_header) (void)hipHostFree(ctx->h_header);
  for (auto& p : ctx->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  if (ctx->done) (void)hipEventDestroy(ctx->done);
  if (ctx->header) (void)hipEventDestroy(ctx->header);
  delete ctx;
}

const char* sz_last_error(const sz_ctx* ctx) {
  if (!ctx) return "no context";
  return ctx->err.c_str();
}

void sz_default_options(sz_options* o) {
  if (!o) return;
  o->radius = kMaxRadius;
  o->chunk = 4096;
  o->subchunks = 0;
  for (int j = 0; j < kMaxDims; j++) o->dim_order[j] = (uint8_t)j;
}

size_t sz_compress_bound(int dtype, int ndim, const uint64_t* dims, const sz_options* opts) {
  Shape s;
  if (make_shape(nullptr, dtype, ndim, dims, opts, &s) != SZ_OK) return 0;
  uint64_t nch = s.nchunks();
  uint64_t ksym = std::min<uint64_t>(2ull * s.radius, s.n);
  // Huffman is optimal, so its length is within one bit per symbol of the
  // entropy, itself at most log2(2R) <= 16 bits; each chunk pads < 32 bits.
  uint64_t words = (17 * s.n + 31) / 32 + nch;
  Layout l = stream_layout(ksym, nch, s.sub, s.n, s.tsize(), words);
  return (size_t)l.size;
}

size_t sz_compress_bound_pwrel(int dtype, int ndim, const uint64_t* dims, const sz_options* opts) {
  Shape s;
  if (make_shape(nullptr, dtype, ndim, dims, opts, &s) != SZ_OK) return 0;
  const size_t core = sz_compress_bound(SZ_F64, ndim, dims, opts);
  if (core == 0) return 0;
  return core + 8 + 8 * (size_t)((s.n + 63) / 64);
}

int sz_inspect(const void* h_stream, size_t len, sz_info* info) {
  if (!h_stream || !info || len < kHeaderBytes) return SZ_ERR_ARG;
  return parse_header(static_cast<const uint8_t*>(h_stream), info);
}

// The arguments of a compression with an absolute or range-relative bound:
// shape and options (into *s), bound, predictor, buffers and alignment.
static int check_compress(sz_ctx* ctx, const void* d_in, int dtype, int ndim,
                          const uint64_t* dims, int eb_mode, double eb, int predictor,
                          const sz_options* opts, const void* d_out, Shape* s) {
  int rc = make_shape(ctx, dtype, ndim, dims, opts, s);
  if (rc) return rc;
  if (eb_mode != SZ_EB_ABS && eb_mode != SZ_EB_REL) return fail(ctx, SZ_ERR_ARG, "bad eb_mode");
  if (predictor != SZ_INTERP_LINEAR && predictor != SZ_INTERP_CUBIC &&
      predictor != SZ_INTERP_ADAPTIVE && predictor != SZ_LORENZO)
    return fail(ctx, SZ_ERR_ARG, "bad predictor");
  if (!(eb >= 0.0) || !__builtin_isfinite(eb)) return fail(ctx, SZ_ERR_ARG, "eb must be finite and >= 0");
  if (eb_mode == SZ_EB_ABS && dtype == SZ_F32 && !__builtin_isfinite((float)eb))
    return fail(ctx, SZ_ERR_ARG, "eb not representable in float");
  if ((s->n && !d_in) || !d_out) return fail(ctx, SZ_ERR_ARG, "null buffer");
  if (((uintptr_t)d_in % 16) || ((uintptr_t)d_out % 8))
    return fail(ctx, SZ_ERR_ARG, "d_in must be 16-byte and d_out 8-byte aligned");
  if (predictor == SZ_LORENZO)
    for (int j = 0; j < s->ndim; j++)
      if (s->order[j] != j) return fail(ctx, SZ_ERR_ARG, "the Lorenzo predictor takes no dim_order");
  return SZ_OK;
}

static int compress_core(sz_ctx* ctx, const void* d_in, int dtype, int ndim, const uint64_t* dims,
                         int eb_mode, double eb, int predictor, const sz_options* opts,
                         void* d_out, size_t out_capacity, size_t* out_size, void* stream,
                         bool noalloc = false) {
  if (!ctx) return SZ_ERR_ARG;
  Shape s;
  int rc = make_shape(ctx, dtype, ndim, dims, opts, &s);
  if (rc) return rc;
  if (!out_size) return fail(ctx, SZ_ERR_ARG, "out_size is NULL");
  *out_size = 0;
  if ((rc = check_compress(ctx, d_in, dtype, ndim, dims, eb_mode, eb, predictor, opts, d_out, &s)))
    return rc;
  CHECK_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  Work w;
  if ((rc = acquire_work(ctx, s, noalloc, &w))) return rc;
  uint8_t* out = static_cast<uint8_t*>(d_out);
  uint16_t* codes = w.codes;
  const uint32_t nsym = 2 * s.radius;
  const uint64_t nch = s.nchunks();
  uint8_t hdr[kHeaderBytes];
  header_template(s, predictor, eb_mode, eb, hdr);

  // (the histogram cleared in the same launch)
  CHECK_HIP(launch_meta_init(ctx->meta, st, ctx->hist, nsym), "meta_init");
  if (eb_mode == SZ_EB_REL)
    CHECK_HIP(timed(ctx, "minmax", st, [&] {
                return launch_minmax(d_in, dtype, s.n, ctx->meta, ctx->mm_part, st);
              }),
              "minmax");
  CHECK_HIP(launch_resolve_eb(dtype, eb_mode, eb, ctx->meta, st, ctx->mm_part,
                              eb_mode == SZ_EB_REL && s.n ? (uint32_t)minmax_blocks(s.n) : 0u),
            "resolve_eb");
  // each level's predictor: the fixed one, or (adaptive) the cheaper one by
  // the levels' cost sums (cubic on ties), recorded as a mask in the header
  int lvl_pred[kMaxLevels + 1];
  for (int l = 0; l <= kMaxLevels; l++)
    lvl_pred[l] = predictor == SZ_INTERP_ADAPTIVE ? SZ_INTERP_CUBIC : predictor;
  if (predictor == SZ_INTERP_ADAPTIVE && s.n) {
    // the dimension order first (the default order only): every order priced
    // on the sampled rows as the sum over levels of the cheaper cost sum,
    // the cheapest first in lexicographic order
    bool identity = true;
    for (int j = 0; j < s.ndim; j++) identity = identity && s.order[j] == j;
    uint64_t* const lvl = ctx->lvl_cost + kCandBuckets;  // the chosen order's level sums
    uint8_t* const chosen = reinterpret_cast<uint8_t*>(lvl + 2 * kMaxLevels);
    bool device_order = false;  // (the order chosen on the device, read back below)
    std::array<std::array<uint8_t, kMaxDims>, kMaxOrders> perms;
    if (identity && s.ndim > 1) {
      size_t nperm = 0;
      std::array<uint8_t, kMaxDims> pm{0, 1, 2, 3};
      do perms[nperm++] = pm;
      while (std::next_permutation(pm.begin(), pm.begin() + s.ndim));
      uint8_t pos[kMaxOrders][kMaxDims] = {};
      for (size_t i = 0; i < nperm; i++)
        for (int j = 0; j < s.ndim; j++) pos[i][perms[i][j]] = (uint8_t)j;
      const size_t per = 2 * kMaxLevels;
      // (fields of up to three dimensions) the candidate buckets of one pass
      const bool cand = s.ndim <= 3;
      const size_t ncost = cand ? kCandBuckets : per * nperm;
      CHECK_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(ctx->lvl_cost), 0, 2 * ncost, st),
                "fill");
      if (noalloc) {  // (the sampled rows are found by the kernel)
        CHECK_HIP(timed(ctx, "estimate", st, [&] {
                    if (cand) {
                      const EstGeom eg = make_estimate_geom(s.ndim, s.dims, perms[0].data());
                      return launch_estimate_cand(d_in, dtype, eg, nullptr, s.n / s.dims[s.ndim - 1],
                                                  ctx->meta, s.radius, ctx->lvl_cost, st);
                    }
                    hipError_t e = hipSuccess;  // (four dimensions: one launch an order)
                    for (size_t i = 0; i < nperm && e == hipSuccess; i++) {
                      EstGeom eg = make_estimate_geom(s.ndim, s.dims, perms[i].data());
                      eg.sampled = 1;
                      e = launch_estimate(d_in, dtype, eg, ctx->meta, s.radius,
                                          ctx->lvl_cost + per * i, st);
                    }
                    return e;
                  }), "estimate");
      } else {
        // the sampled rows of this shape (kept while the shape repeats)
        bool same = ctx->est_ndim == s.ndim && ctx->est_rows.p;
        for (int d = 0; d < s.ndim; d++) same = same && ctx->est_dims[d] == s.dims[d];
        if (!same) {
          const uint64_t nrows_all = s.n / s.dims[s.ndim - 1];
          std::vector<uint32_t> rows;
          rows.reserve(nrows_all / 8 + 64);
          for (uint64_t r = 0; r < nrows_all; r++)
            if (est_row_sampled(r)) rows.push_back((uint32_t)r);
          if (cand) {  // grouped by class (ascending within a class)
            std::vector<uint64_t> keyed(rows.size());
            for (size_t i = 0; i < rows.size(); i++)
              keyed[i] = (uint64_t)cand_row_class(s.ndim, s.dims, rows[i]) << 32 | rows[i];
            std::sort(keyed.begin(), keyed.end());
            for (size_t i = 0; i < rows.size(); i++) rows[i] = (uint32_t)keyed[i];
          }
          CHECK_HIP(ensure(ctx->est_rows, std::max<size_t>(4, rows.size() * 4)), "hipMalloc(est_rows)");
          if (!rows.empty())
            CHECK_HIP(hipMemcpy(ctx->est_rows.p, rows.data(), rows.size() * 4, hipMemcpyHostToDevice),
                      "memcpy");
          ctx->est_nrows = rows.size();
          ctx->est_ndim = s.ndim;
          for (int d = 0; d < kMaxDims; d++) ctx->est_dims[d] = d < s.ndim ? s.dims[d] : 0;
        }
        const EstGeom eg = make_estimate_geom(s.ndim, s.dims, perms[0].data());
        CHECK_HIP(timed(ctx, "estimate", st, [&] {
                    if (cand)
                      return launch_estimate_cand(d_in, dtype, eg,
                                                  static_cast<const uint32_t*>(ctx->est_rows.p),
                                                  ctx->est_nrows, ctx->meta, s.radius,
                                                  ctx->lvl_cost, st);
                    return launch_estimate_orders(d_in, dtype, eg, pos, (uint32_t)nperm,
                                                  static_cast<const uint32_t*>(ctx->est_rows.p),
                                                  ctx->est_nrows, ctx->meta, s.radius, per,
                                                  ctx->lvl_cost, st);
                  }), "estimate");
      }
      const int L = level_count(s.ndim, s.dims);
      if (cand) {  // chosen on the device: the full estimate follows with no round trip
        // (the chosen order's sums over the sampled rows seed the level sums)
        CHECK_HIP(launch_choose_order(ctx->lvl_cost, s.ndim, pos, (uint32_t)nperm, L, chosen, lvl,
                                      st), "choose_order");
        device_order = true;
      } else {
        std::array<uint64_t, 2 * kMaxLevels * kMaxOrders> cost;
        CHECK_HIP(hipMemcpyAsync(cost.data(), ctx->lvl_cost, sizeof(uint64_t) * ncost,
                                 hipMemcpyDeviceToHost, st), "memcpy");
        CHECK_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
        uint64_t best = ~0ull;
        size_t bi = 0;
        for (size_t i = 0; i < nperm; i++) {
          uint64_t total = 0;
          for (int l = 1; l <= L; l++) {
            const uint64_t lin = cost[per * i + 2 * (l - 1)], cub = cost[per * i + 2 * (l - 1) + 1];
            total += cub < lin ? cub : lin;
          }
          if (total < best) {
            best = total;
            bi = i;
          }
        }
        for (int j = 0; j < s.ndim; j++) s.order[j] = perms[bi][j];
      }
    }
    if (!device_order)
      CHECK_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(lvl), 0, 4 * kMaxLevels, st), "fill");
    // (places: the device's choice, whose sampled rows are summed already)
    EstGeom eg = make_estimate_geom(s.ndim, s.dims, s.order);
    if (device_order) eg.sampled = 2;
    CHECK_HIP(timed(ctx, "estimate", st, [&] {
                return launch_estimate(d_in, dtype, eg, ctx->meta, s.radius, lvl, st,
                                       device_order ? chosen + 1 : nullptr);
              }), "estimate");
    const uint64_t* cost = ctx->h_lvl;  // the level sums, then the device's choice
    CHECK_HIP(hipMemcpyAsync(ctx->h_lvl, lvl, sizeof(uint64_t) * (2 * kMaxLevels + 1),
                             hipMemcpyDeviceToHost, st), "memcpy");
    CHECK_HIP(wait_stream(ctx, st, kSpinLongMicros), "wait");
    if (device_order) {
      const uint8_t bi = static_cast<uint8_t>(cost[2 * kMaxLevels] & 0xFF);
      for (int j = 0; j < s.ndim; j++) s.order[j] = perms[bi][j];
    }
    for (int j = 0; j < s.ndim; j++) hdr[41 + j] = s.order[j];
    uint32_t mask = 0;
    for (int l = 1; l <= kMaxLevels; l++) {
      lvl_pred[l] = cost[2 * (l - 1) + 1] <= cost[2 * (l - 1)] ? SZ_INTERP_CUBIC : SZ_INTERP_LINEAR;
      if (lvl_pred[l] == SZ_INTERP_CUBIC && l <= level_count(s.ndim, s.dims)) mask |= 1u << (l - 1);
    }
    put_le(hdr + 124, mask, 4);
  }
  auto pred_of = [&](uint32_t stride) { return lvl_pred[1 + __builtin_ctz(stride)]; };
  if (s.n && predictor == SZ_LORENZO) {
    CHECK_HIP(timed(ctx, "interp", st, [&] {
                return launch_lorenzo_compress(d_in, dtype, w.rec, codes, s.ndim, s.dims,
                                               ctx->meta, s.radius, st);
              }), "lorenzo");
  } else if (s.n) {
    // the origin and every level, timed as one region; with the fused
    // kernels, the origin and the coarsest levels (strides >= s_small) in one
    // workgroup first
    const SmallGeom sg = plan_small_levels(s.ndim, s.dims, s.order, level_count(s.ndim, s.dims),
                                           cubic_mask(lvl_pred), (int)s.tsize());
    const uint64_t s_small = ctx->fused_levels ? 1ull << (sg.l_stop - 1) : ~0ull;
    std::vector<LevelGeom>& levels = ctx->levels;
    const bool fused =
        ctx->fused_levels && plan_levels(s.ndim, s.dims, s.order, (int)s.tsize(), nullptr, levels);
    const uint64_t cb = fused ? compact_bytes(levels, dtype, d_in, w.rec, s_small, s.tsize()) : 0;
    // (the static scratch always holds room for the lattice of a 3-D field)
    if (cb && !noalloc) {
      CHECK_HIP(ensure(ctx->coarse, cb), "hipMalloc(coarse)");
      w.coarse = ctx->coarse.p;
    }
    void* cmp = cb ? w.coarse : nullptr;
    CHECK_HIP(timed(ctx, "interp", st, [&] {
                hipError_t e =
                    ctx->fused_levels
                        ? launch_small_levels_compress(d_in, dtype, w.rec, codes, sg,
                                                       ctx->meta, s.radius, st)
                        : launch_origin_compress(d_in, dtype, w.rec, codes, ctx->meta,
                                                 s.radius, st);
                if (fused) {
                  // the finest level's reconstruction is not read by anything later
                  for (const LevelGeom& g : levels)
                    if (e == hipSuccess && g.s < s_small)
                      e = launch_level_compress(d_in, dtype, pred_of(g.s), w.rec, codes, g,
                                                ctx->meta, s.radius, g.s > 1, cmp, st);
                } else {
                  build_passes(s, ctx->passes);
                  for (const PassGeom& g : ctx->passes)
                    if (e == hipSuccess && g.s < s_small)
                      e = launch_pass_compress(d_in, dtype, pred_of(g.s), w.rec, codes, g,
                                               ctx->meta, s.radius, st);
                }
                return e;
              }), "interp");
  }
  CHECK_HIP(timed(ctx, "histogram", st,
                  [&] { return launch_histogram(codes, s.n, s.radius, ctx->hist_part, ctx->hist, ctx->meta, st);
                  }),
            "histogram");
  CHECK_HIP(timed(ctx, "codebook", st, [&] {
              return launch_codebook(ctx->hist, nsym, ctx->cb, ctx->enc_code, ctx->enc_len,
                                     ctx->symtab, ctx->meta, st);
            }), "codebook");
  EncodeScratch es{w.chunk_words, w.chunk_unpred, w.word_off, w.unpred_off, w.block_sums,
                   ctx->totals};
  CHECK_HIP(timed(ctx, "encode", st, [&] {
              // (the reconstruction is dead once the levels are done: the
              // encoder packs its chunks there)
              return launch_encode(codes, d_in, dtype, s.n, s.chunk, s.sub, s.radius, ctx->enc_code,
                                   ctx->enc_len, es, static_cast<uint32_t*>(w.rec), out,
                                   out_capacity, ctx->meta, st);
            }), "encode");
  CHECK_HIP(timed(ctx, "other", st, [&] {
              return launch_write_tables(out, out_capacity, ctx->symtab, nch, s.sub, hdr, dtype, ctx->meta, st);
            }), "write_tables");
  CHECK_HIP(hipMemcpyAsync(ctx->h_meta, ctx->meta, sizeof(Meta), hipMemcpyDeviceToHost, st), "memcpy");
  CHECK_HIP(wait_stream(ctx, st), "wait");
  ctx->last_n = s.n;
  ctx->last_codes = codes;
  const Meta& m = *ctx->h_meta;
  if (m.status & kStatusEbNotFinite) return fail(ctx, SZ_ERR_ARG, "resolved error bound is not finite");
  if (m.status & kStatusCodeTooLong) return fail(ctx, SZ_ERR_UNSUPPORTED, "Huffman code longer than 64 bits");
  *out_size = (size_t)m.stream_bytes;
  if (m.stream_bytes > out_capacity)
    return fail(ctx, SZ_ERR_CAPACITY, "output capacity too small");
  return SZ_OK;
}

// The point-wise relative mode: the logarithmic transform into the log
// field (and the sign words), the log field through compress_core with the
// absolute bound delta, then the sign section and the mode's header fields.
static int compress_pwrel(sz_ctx* ctx, const void* d_in, int dtype, int ndim,
                          const uint64_t* dims, double eps, int predictor,
                          const sz_options* opts, void* d_out, size_t out_capacity,
                          size_t* out_size, void* stream) {
  Shape s;
  int rc = make_shape(ctx, dtype, ndim, dims, opts, &s);
  if (rc) return rc;
  if (!out_size) return fail(ctx, SZ_ERR_ARG, "out_size is NULL");
  *out_size = 0;
  const double delta = pwrel_delta(eps, dtype);
  if (!(delta > 0.0))
    return fail(ctx, SZ_ERR_ARG, "point-wise relative bound must be in (0, 1) and above the type's precision");
  if (predictor != SZ_INTERP_LINEAR && predictor != SZ_INTERP_CUBIC &&
      predictor != SZ_INTERP_ADAPTIVE && predictor != SZ_LORENZO)
    return fail(ctx, SZ_ERR_ARG, "bad predictor");
  if ((s.n && !d_in) || !d_out) return fail(ctx, SZ_ERR_ARG, "null buffer");
  if (((uintptr_t)d_in % 16) || ((uintptr_t)d_out % 8))
    return fail(ctx, SZ_ERR_ARG, "d_in must be 16-byte and d_out 8-byte aligned");
  CHECK_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const uint64_t nsw = (s.n + 63) / 64;
  CHECK_HIP(ensure(ctx->ylog, s.n * 8), "hipMalloc(ylog)");
  CHECK_HIP(ensure(ctx->signs, nsw * 8), "hipMalloc(signs)");
  double* y = static_cast<double*>(ctx->ylog.p);
  uint64_t* signs = static_cast<uint64_t*>(ctx->signs.p);
  uint32_t* any = reinterpret_cast<uint32_t*>(ctx->totals + 3);
  CHECK_HIP(launch_fill_u32(any, 0, 2, st), "fill");
  CHECK_HIP(launch_pwrel_forward(d_in, dtype, y, signs, s.n, any, st), "pwrel_forward");
  size_t ylen = 0;
  rc = compress_core(ctx, y, SZ_F64, ndim, dims, SZ_EB_ABS, delta, predictor, opts, d_out,
                     out_capacity, &ylen, stream);
  if (rc && rc != SZ_ERR_CAPACITY) return rc;
  uint32_t any_h = 0;
  CHECK_HIP(hipMemcpy(&any_h, any, sizeof(any_h), hipMemcpyDeviceToHost), "hipMemcpy");
  const uint64_t off_signs = any_h ? pad8(ylen) : 0;
  const uint64_t total = any_h ? off_signs + 8 * nsw : ylen;
  *out_size = (size_t)total;
  if (total > out_capacity) return fail(ctx, SZ_ERR_CAPACITY, "output capacity too small");
  CHECK_HIP(launch_pwrel_finish(static_cast<uint8_t*>(d_out), ylen, off_signs, signs, nsw, total,
                                eps, dtype, st),
            "pwrel_finish");
  CHECK_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
  return SZ_OK;
}

int sz_compress(sz_ctx* ctx, const void* d_in, int dtype, int ndim, const uint64_t* dims,
                int eb_mode, double eb, int predictor, const sz_options* opts, void* d_out,
                size_t out_capacity, size_t* out_size, void* stream) {
  if (!ctx) return SZ_ERR_ARG;
  if (eb_mode == SZ_EB_PWREL)
    return compress_pwrel(ctx, d_in, dtype, ndim, dims, eb, predictor, opts, d_out, out_capacity,
                          out_size, stream);
  return compress_core(ctx, d_in, dtype, ndim, dims, eb_mode, eb, predictor, opts, d_out,
                       out_capacity, out_size, stream);
}

int sz_compress_noalloc(sz_ctx* ctx, const void* d_in, int dtype, int ndim, const uint64_t* dims,
                        int eb_mode, double eb, int predictor, const sz_options* opts, void* d_out,
                        size_t out_capacity, size_t* out_size, void* stream) {
  if (!ctx) return SZ_ERR_ARG;
  if (eb_mode == SZ_EB_PWREL)
    return fail(ctx, SZ_ERR_UNSUPPORTED, "sz_compress_noalloc takes absolute and relative bounds only");
  ctx->no_timing = true;
  const int rc = compress_core(ctx, d_in, dtype, ndim, dims, eb_mode, eb, predictor, opts, d_out,
                               out_capacity, out_size, stream, true);
  ctx->no_timing = false;
  return rc;
}

int sz_decompress(sz_ctx* ctx, const void* d_stream, size_t stream_size, void* d_out,
                  size_t out_capacity, void* stream) {
  if (!ctx) return SZ_ERR_ARG;
  if (!d_stream) return fail(ctx, SZ_ERR_ARG, "null stream");
  if (((uintptr_t)d_stream % 8) || ((uintptr_t)d_out % 16))
    return fail(ctx, SZ_ERR_ARG, "d_stream must be 8-byte and d_out 16-byte aligned");
  if (stream_size < kHeaderBytes) return fail(ctx, SZ_ERR_CORRUPT, "stream shorter than its header");
  CHECK_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  // The per-call values are reset and the header is copied out; then the
  // decoding tables and the chunk table's scans start from the header in
  // device memory while the host waits for its copy (when the chunk buffers
  // hold the chunks; else, or when the buffers move below, the host launches
  // them once it has parsed the header).
  CHECK_HIP(launch_meta_init(ctx->meta, st), "meta_init");
  CHECK_HIP(hipMemcpyAsync(ctx->h_header, d_stream, kHeaderBytes, hipMemcpyDeviceToHost, st), "memcpy");
  CHECK_HIP(mark(ctx->header, st), "hipEventRecord");
  uint64_t cap = std::min({ctx->chunk_words.cap / 4, ctx->chunk_unpred.cap / 4, ctx->word_off.cap / 8,
                           ctx->unpred_off.cap / 8});
  cap = std::min<uint64_t>(cap, ctx->block_sums.cap >= 24 ? (ctx->block_sums.cap / 8 - 1) / 2 * 1024 : 0);
  const void* early_bufs[5] = {ctx->chunk_words.p, ctx->chunk_unpred.p, ctx->word_off.p,
                               ctx->unpred_off.p, ctx->block_sums.p};
  if (cap)
    CHECK_HIP(timed(ctx, "decode_tables", st, [&] {
                return launch_decode_front_early(
                    static_cast<const uint8_t*>(d_stream), stream_size, cap, ctx->dt,
                    static_cast<uint32_t*>(ctx->chunk_words.p), static_cast<uint32_t*>(ctx->chunk_unpred.p),
                    static_cast<uint64_t*>(ctx->word_off.p), static_cast<uint64_t*>(ctx->unpred_off.p),
                    static_cast<uint64_t*>(ctx->block_sums.p), ctx->totals, ctx->meta, st);
              }), "decode_tables");
  CHECK_HIP(wait_mark(ctx->header), "wait");
  sz_info in;
  if (parse_header(ctx->h_header, &in) != SZ_OK) return fail(ctx, SZ_ERR_CORRUPT, "invalid header");
  if (in.stream_bytes > stream_size) return fail(ctx, SZ_ERR_CORRUPT, "stream truncated");
  Shape s;
  const bool pw = in.eb_mode == SZ_EB_PWREL;
  s.dtype = in.coded_dtype;  // the pipeline decodes the coded field
  s.ndim = in.ndim;
  for (int d = 0; d < kMaxDims; d++) {
    s.dims[d] = in.dims[d];
    s.order[d] = in.dim_order[d];
  }
  s.n = in.n;
  s.radius = in.radius;
  s.chunk = in.chunk;
  s.sub = in.sub;
  if (s.n && !d_out) return fail(ctx, SZ_ERR_ARG, "null output buffer");
  if (out_capacity < s.n * (in.dtype == SZ_F64 ? 8 : 4))
    return fail(ctx, SZ_ERR_CAPACITY, "output capacity too small");
  int rc = ensure_sized(ctx, s, false);
  if (rc) return rc;
  // point-wise relative mode: the pipeline rebuilds the log field, then the
  // inverse transform writes the field
  void* field_out = d_out;
  if (pw) {
    CHECK_HIP(ensure(ctx->ylog, s.n * 8), "hipMalloc(ylog)");
    d_out = ctx->ylog.p;
  }
  const uint8_t* str = static_cast<const uint8_t*>(d_stream);
  const uint64_t nch = s.nchunks();
  Layout l = stream_layout(in.nsym, nch, s.sub, in.n_unpred, s.tsize(), in.total_words);
  uint16_t* codes = static_cast<uint16_t*>(ctx->codes.p);
  uint32_t* cwords = static_cast<uint32_t*>(ctx->chunk_words.p);
  uint32_t* cunp = static_cast<uint32_t*>(ctx->chunk_unpred.p);
  uint64_t* woff = static_cast<uint64_t*>(ctx->word_off.p);
  uint64_t* uoff = static_cast<uint64_t*>(ctx->unpred_off.p);
  uint64_t* bsum = static_cast<uint64_t*>(ctx->block_sums.p);

  if (s.n) {
    const void* bufs[5] = {cwords, cunp, woff, uoff, bsum};
    const bool early = cap && nch <= cap && std::equal(bufs, bufs + 5, early_bufs);
    if (!early) {
      // (the early launch may have run with the header's values: start over)
      CHECK_HIP(launch_meta_init(ctx->meta, st), "meta_init");
      CHECK_HIP(timed(ctx, "decode_tables", st, [&] {
                  return launch_decode_front(str, in.stream_bytes, l.off_sym, in.nsym, 2 * s.radius, ctx->dt,
                                             l.off_chunk, nch, cwords, cunp, woff, uoff, bsum,
                                             ctx->totals, in.total_words, in.n_unpred, ctx->meta, st);
                }), "decode_tables");
    }
    CHECK_HIP(timed(ctx, "decode", st, [&] {
                return launch_decode_chunks(str, stream_size, l.off_sub, l.off_unpred, l.off_bits,
                                            in.total_words, in.n_unpred, s.n, s.chunk, s.sub, in.nsym,
                                            s.dtype, cwords, cunp,
                                            woff, uoff, bsum, ctx->dt, codes, d_out, ctx->meta, st);
              }), "decode");
    int lvl_pred[kMaxLevels + 1];
    for (int l = 0; l <= kMaxLevels; l++)
      lvl_pred[l] = in.predictor != SZ_INTERP_ADAPTIVE   ? in.predictor
                    : l >= 1 && ((in.level_mask >> (l - 1)) & 1u) ? SZ_INTERP_CUBIC
                                                                    : SZ_INTERP_LINEAR;
    auto pred_of = [&](uint32_t stride) { return lvl_pred[1 + __builtin_ctz(stride)]; };
    const SmallGeom sg = plan_small_levels(s.ndim, s.dims, s.order, level_count(s.ndim, s.dims),
                                           cubic_mask(lvl_pred), (int)s.tsize());
    const uint64_t s_small = ctx->fused_levels ? 1ull << (sg.l_stop - 1) : ~0ull;
    std::vector<LevelGeom>& levels = ctx->levels;
    const bool fused = in.predictor != SZ_LORENZO && ctx->fused_levels &&
                       plan_levels(s.ndim, s.dims, s.order, (int)s.tsize(), nullptr, levels);
    const uint64_t cb = fused ? compact_bytes(levels, s.dtype, d_out, d_out, s_small, s.tsize()) : 0;
    if (cb) CHECK_HIP(ensure(ctx->coarse, cb), "hipMalloc(coarse)");
    void* cmp = cb ? ctx->coarse.p : nullptr;
    CHECK_HIP(timed(ctx, "recon", st, [&] {
                if (in.predictor == SZ_LORENZO)
                  return launch_lorenzo_recon(codes, s.dtype, d_out, s.ndim, s.dims, in.eb,
                                              s.radius, st);
                hipError_t e =
                    ctx->fused_levels
                        ? launch_small_levels_recon(codes, s.dtype, d_out, sg, in.eb, s.radius, st)
                        : launch_origin_recon(codes, s.dtype, d_out, in.eb, s.radius, st);
                if (fused) {
                  for (const LevelGeom& g : levels)
                    if (e == hipSuccess && g.s < s_small)
                      e = launch_level_recon(codes, s.dtype, pred_of(g.s), d_out, g, in.eb,
                                             s.radius, cmp, st);
                } else {
                  build_passes(s, ctx->passes);
                  for (const PassGeom& g : ctx->passes)
                    if (e == hipSuccess && g.s < s_small)
                      e = launch_pass_recon(codes, s.dtype, pred_of(g.s), d_out, g, in.eb,
                                            s.radius, st);
                }
                return e;
              }), "recon");
    if (pw)
      CHECK_HIP(launch_pwrel_inverse(static_cast<const double*>(d_out),
                                     in.signs ? reinterpret_cast<const uint64_t*>(str + in.off_signs)
                                              : nullptr,
                                     s.n, in.dtype, field_out, st),
                "pwrel_inverse");
  }
  CHECK_HIP(hipMemcpyAsync(ctx->h_meta, ctx->meta, sizeof(Meta), hipMemcpyDeviceToHost, st), "memcpy");
  CHECK_HIP(wait_stream(ctx, st), "wait");
  if (ctx->h_meta->status & kStatusCorrupt) return fail(ctx, SZ_ERR_CORRUPT, "stream failed validation");
  return SZ_OK;
}

int sz_compress_batch(sz_ctx* ctx, sz_field* fields, int nfields, const sz_options* opts,
                      void* stream) {
  if (!ctx || (nfields > 0 && !fields) || nfields < 0) return SZ_ERR_ARG;
  CHECK_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  // the fields the shared launches cover go to the batched path; the rest
  // (other predictors and bounds, four dimensions, empty or invalid fields)
  // take sz_compress one by one
  std::vector<BatchItem> items;
  std::vector<int> where, single;
  const bool batched = !(getenv("SZG_BATCH") && strcmp(getenv("SZG_BATCH"), "0") == 0);
  for (int i = 0; i < nfields; i++) {
    sz_field& f = fields[i];
    f.out_size = 0;
    Shape s;
    if (!batched || f.eb_mode == SZ_EB_PWREL ||
        check_compress(ctx, f.d_in, f.dtype, f.ndim, f.dims, f.eb_mode, f.eb, f.predictor, opts,
                       f.d_out, &s) != SZ_OK) {
      single.push_back(i);
      continue;
    }
    BatchItem it{};
    it.x = f.d_in;
    it.out = f.d_out;
    it.cap = f.out_capacity;
    it.dtype = s.dtype;
    it.ndim = s.ndim;
    for (int d = 0; d < kMaxDims; d++) {
      it.dims[d] = s.dims[d];
      it.order[d] = s.order[d];
    }
    it.eb_mode = f.eb_mode;
    it.eb = f.eb;
    it.pred = f.predictor;
    it.R = s.radius;
    it.chunk = s.chunk;
    it.sub = s.sub;
    header_template(s, f.predictor, f.eb_mode, f.eb, it.hdr);
    items.push_back(it);
    where.push_back(i);
  }
  // the cached plan covers exactly these fields, or each field is checked
  if (!batch_plan_covers(ctx->batch, items)) {
    size_t k = 0;
    for (size_t j = 0; j < items.size(); j++) {
      if (batch_item_supported(items[j])) {
        items[k] = items[j];
        where[k] = where[j];
        k++;
      } else {
        single.push_back(where[j]);
      }
    }
    items.resize(k);
    where.resize(k);
    std::sort(single.begin(), single.end());
  }
  std::string err;
  const int rc = batch_compress(ctx->device, &ctx->batch, items, st, err);
  for (size_t k = 0; k < items.size(); k++) {
    sz_field& f = fields[where[k]];
    f.status = rc ? rc : items[k].status;
    f.out_size = rc ? 0 : items[k].out_size;
  }
  if (rc) fail(ctx, rc, err);
  for (int i : single) {
    sz_field& f = fields[i];
    size_t sz = 0;
    f.status = sz_compress(ctx, f.d_in, f.dtype, f.ndim, f.dims, f.eb_mode, f.eb, f.predictor, opts,
                           f.d_out, f.out_capacity, &sz, stream);
    f.out_size = sz;
  }
  for (int i = 0; i < nfields; i++)
    if (fields[i].status != SZ_OK) return fields[i].status;
  return SZ_OK;
}

int sz_set_timing(sz_ctx* ctx, int enable) {
  if (!ctx) return SZ_ERR_ARG;
  ctx->timing = enable != 0;
  return SZ_OK;
}

int sz_set_timing_family(sz_ctx* ctx, const char* name) {
  if (!ctx) return SZ_ERR_ARG;
  ctx->timing_family = name ? name : "";
  return SZ_OK;
}

int sz_timing_get(sz_ctx* ctx, const char* name, double* total_ms, uint64_t* launches) {
  if (!ctx || !name) return SZ_ERR_ARG;
  settle_timing(ctx);
  auto it = ctx->stats.find(name);
  if (total_ms) *total_ms = it == ctx->stats.end() ? 0.0 : it->second.ms;
  if (launches) *launches = it == ctx->stats.end() ? 0 : it->second.n;
  return SZ_OK;
}

int sz_timing_reset(sz_ctx* ctx) {
  if (!ctx) return SZ_ERR_ARG;
  settle_timing(ctx);
  ctx->stats.clear();
  return SZ_OK;
}

int sz_debug_codes(sz_ctx* ctx, void* d_codes, size_t capacity, void* stream) {
  if (!ctx || !d_codes) return SZ_ERR_ARG;
  if (capacity < ctx->last_n * 2) return fail(ctx, SZ_ERR_CAPACITY, "capacity too small");
  if (ctx->last_n == 0) return SZ_OK;
  hipStream_t st = (hipStream_t)stream;
  CHECK_HIP(hipMemcpyAsync(d_codes, ctx->last_codes, ctx->last_n * 2, hipMemcpyDeviceToDevice, st),
            "memcpy");
  CHECK_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
  return SZ_OK;
}

}  // extern "C"
