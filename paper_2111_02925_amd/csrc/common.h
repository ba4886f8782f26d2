// Internal declarations of the MI355X interpolation compressor library.
//
// Stage map (paper: SZ3, Algorithm 1 in Section 3.3, SZ3-Interp in Section 6.2):
//   eb resolution     (range-relative bound, Section 6.2)      interp.hip
//   predict+quantize  (Algorithm 1 loop; Section 3.2 quantizer) interp.hip
//   histogram/codebook/encode/decode (Section 3.2 encoder)      huffman.hip
//   reconstruction    (Appendix A.3 recover)                     interp.hip
//   fused levels (<= 3 dimensions, compression and reconstruction) level.hip
//   C ABI, context, stream header                                api.hip
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "szg.h"

namespace szg {

constexpr int kMaxDims = 4;
constexpr uint32_t kMaxRadius = 32768;
constexpr uint32_t kMaxSym = 2 * kMaxRadius;
constexpr int kMaxCodeLen = 64;
constexpr uint64_t kMaxPoints = 0xFFFFFFFFull;
constexpr uint64_t kHeaderBytes = 128;
constexpr int kLutBits = 12;
constexpr int kCbThreads = 512;  // threads of the single-block table kernels

// Sub-chunks: a chunk of C symbols may be split into S in {2, 4, 8} runs of
// C/S symbols whose starting bit offsets are stored, so that S lanes decode
// one chunk.  A run must hold a multiple of the encoder's per-lane run,
// max(32, C/64) symbols.
__host__ __device__ inline bool valid_sub(uint32_t chunk, uint32_t sub) {
  if (sub == 1) return true;
  if (sub != 2 && sub != 4 && sub != 8) return false;
  if (chunk == 0 || chunk % sub) return false;
  const uint32_t run = chunk / 64 > 32 ? chunk / 64 : 32;
  return (chunk / sub) % run == 0;
}

// Sub-chunks per chunk when the caller does not choose: 4 where valid, else 2, else 1.
inline uint32_t default_sub(uint32_t chunk) {
  return valid_sub(chunk, 4) ? 4 : valid_sub(chunk, 2) ? 2 : 1;
}

__host__ __device__ inline uint64_t pad8(uint64_t v) { return (v + 7) & ~uint64_t(7); }

// Byte offsets of the stream sections (layout described in api.hip).
struct Layout {
  uint64_t off_sym, off_chunk, off_sub, off_unpred, off_bits, size;
};
__host__ __device__ inline Layout stream_layout(uint64_t nsym_used, uint64_t nchunks,
                                                uint32_t sub, uint64_t n_unpred, uint64_t tsize,
                                                uint64_t words) {
  Layout l;
  l.off_sym = kHeaderBytes;
  l.off_chunk = l.off_sym + pad8(4 * nsym_used);
  l.off_sub = l.off_chunk + 8 * nchunks;
  l.off_unpred = l.off_sub + pad8(4 * (uint64_t)(sub - 1) * nchunks);
  l.off_bits = l.off_unpred + pad8(n_unpred * tsize);
  l.size = l.off_bits + 4 * words;
  return l;
}

// Per-call values produced on the device and read by later kernels, so that a
// whole compression is one stream-ordered sequence without host round trips.
struct Meta {
  uint64_t key_min;    // order-preserving key of the finite minimum
  uint64_t key_max;    // ... of the finite maximum
  double eb;           // resolved bound in the field type, widened
  double twoeb;        // 2 * eb in the field type
  double inv2eb;       // 1 / (2 eb) in the field type
  uint32_t nsym_used;  // K: symbols with a code
  uint32_t max_len;
  uint32_t sym_lo;     // smallest coded symbol other than 0 (0xFFFFFFFF if none)
  uint32_t sym_hi;     // largest coded symbol other than 0
  uint64_t n_unpred;
  uint64_t total_words;
  uint64_t stream_bytes;
  uint32_t status;     // error bits (kStatus*)
  uint32_t hist_far;   // some code was counted outside the histogram's window
  uint32_t slices_done;  // blocks of the decoder's chunk-table scan that have finished
  uint32_t pad;
};
constexpr uint32_t kStatusEbNotFinite = 1u << 0;
constexpr uint32_t kStatusCodeTooLong = 1u << 1;
constexpr uint32_t kStatusCorrupt = 1u << 2;
constexpr uint32_t kStatusCountMismatch = 1u << 3;

// Geometry of one (level, dimension) pass of the multilevel traversal: the
// points whose coordinate along `d` is an odd multiple of s, whose coordinates
// along dimensions visited earlier in the level are multiples of s, and later
// ones multiples of 2s.
constexpr int kMaxLevels = 32;
constexpr int kMaxOrders = 24;  // orders of at most four dimensions  // levels of a field of fewer than 2^32 points per dimension

struct PassGeom {
  int ndim;
  int d;
  uint32_t s;
  uint32_t cnt[kMaxDims];    // lattice points along each dimension
  uint64_t start[kMaxDims];
  uint64_t step[kMaxDims];
  uint64_t stride[kMaxDims]; // flat strides of the full field
  uint32_t nd;               // extent along d
  uint64_t total;            // points in the pass
};

// ---- scratch accounting (api.hip), used by the request server (server.hip)
// Bytes a compression (or decompression) of n points allocates in a context
// at most; the bytes a context holds now; freeing them; a context's fixed part.
size_t scratch_need(uint64_t n, size_t tsize, uint32_t chunk, bool compress);
// the point-wise relative mode's extra scratch (the log field, the sign words)
size_t pwrel_scratch_need(uint64_t n, bool compress);
size_t ctx_scratch_bytes(const sz_ctx* ctx);
void ctx_trim(sz_ctx* ctx);
size_t ctx_fixed_bytes();

// ------------------------------------------------------------------ launchers
// All launchers enqueue on `st` and return hipSuccess or the launch error.

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t st);
// Meta's start values (and, with nzero > 0, zero[0 .. nzero) cleared in the
// same launch).
hipError_t launch_meta_init(Meta* m, hipStream_t st, uint32_t* zero = nullptr, uint64_t nzero = 0);
// The range pass: minmax_blocks(n) workgroups, each writing its minimum and
// maximum keys to its pair of part (2 x kMinmaxBlocks u64), which the eb
// kernel folds into m (nblk = minmax_blocks(n); 0 when the pass did not run).
constexpr uint32_t kMinmaxBlocks = 512;  // (two workgroups a CU: 2048 took 105 us at 512^3, 512 take 83)
inline uint64_t minmax_blocks(uint64_t n) {
  const uint64_t b = (n + 256 * 64 - 1) / (256 * 64);
  return b < 1 ? 1 : b > kMinmaxBlocks ? kMinmaxBlocks : b;
}
hipError_t launch_minmax(const void* x, int dtype, uint64_t n, Meta* m, uint64_t* part,
                         hipStream_t st);
hipError_t launch_resolve_eb(int dtype, int mode, double value, Meta* m, hipStream_t st,
                             const uint64_t* part = nullptr, uint32_t nblk = 0);

hipError_t launch_origin_compress(const void* x, int dtype, void* rec, uint16_t* codes,
                                  const Meta* m, uint32_t radius, hipStream_t st);
// adaptive interpolation: every level's cost sums under both predictors in
// one launch, added to cost[2 (l - 1)] (linear) and cost[2 (l - 1) + 1]
// (cubic) for level l
struct EstGeom {
  int ndim;
  uint64_t dims[kMaxDims];
  uint64_t stride[kMaxDims];
  uint8_t pos[kMaxDims];  // position of each dimension in the traversal order
  uint32_t pairs;         // column pairs a lane takes per unit (1, 2 or 4)
  uint64_t segs;          // units per row along the last dimension
  uint64_t units;         // rows x segs
  uint32_t sampled;       // 1: only the rows est_row_sampled takes; 2: only the others
};
EstGeom make_estimate_geom(int ndim, const uint64_t* dims, const uint8_t* order);
// The rows that price the dimension orders: row index r when the top three
// bits of (r mod 2^32) * 0x9E3779B1 (Fibonacci hashing) are zero, about one
// row in eight.
__host__ __device__ inline bool est_row_sampled(uint64_t r) {
  return (((uint32_t)r * 0x9E3779B1u) >> 29) == 0;
}
// (pos_dev: the order's places read from the device, else g's)
hipError_t launch_estimate(const void* x, int dtype, const EstGeom& g, const Meta* m,
                           uint32_t radius, uint64_t* cost, hipStream_t st,
                           const uint8_t* pos_dev = nullptr);
// The sampled estimate of every dimension order of a field of up to three
// dimensions in one pass: costs per (level, candidate set, dimension) into
// 2 * 3 * 8 * kMaxLevels buckets (the rows listed in rows[], grouped by
// cand_row_class for speed, or with rows null, the nrows rows of the field
// that est_row_sampled takes); launch_choose_order adds up each order's
// sums from them.
constexpr uint32_t kCandBuckets = 2 * 3 * 8 * kMaxLevels;  // (level, set, dimension) x {linear, cubic}
static_assert(kCandBuckets <= 2 * kMaxLevels * kMaxOrders, "the buckets share the orders' cost buffer");
hipError_t launch_estimate_cand(const void* x, int dtype, const EstGeom& g, const uint32_t* rows,
                                uint64_t nrows, const Meta* m, uint32_t radius, uint64_t* bucket,
                                hipStream_t st);
// The class of row r (flat index over every dimension but the last) that
// the listed rows are grouped by: 8 x (fewest trailing zeros among its
// coordinates) + the mask of the dimensions that have them.
uint32_t cand_row_class(int ndim, const uint64_t* dims, uint64_t r);
// The order choice from the buckets on the device (no host round trip):
// of the norders orders (orders[k][d]: the place of dimension d), the one
// whose sum over levels 1..levels of the cheaper cost sum is least, the
// first on ties; chosen[0] its index, chosen[1..4] its places; with lvl
// non-null, the chosen order's sums over the sampled rows in lvl (2 x
// kMaxLevels: linear, cubic per level).
hipError_t launch_choose_order(const uint64_t* bucket, int ndim, const uint8_t (*orders)[kMaxDims],
                               uint32_t norders, int levels, uint8_t* chosen, uint64_t* lvl,
                               hipStream_t st);
// The sampled estimate of norders dimension orders (orders[k][d]: the place
// of dimension d in order k) in one launch, over the sampled rows listed in
// rows[] (ascending flat row indices, est_row_sampled); order k's sums at
// cost + k * per.
hipError_t launch_estimate_orders(const void* x, int dtype, const EstGeom& g,
                                  const uint8_t (*orders)[kMaxDims], uint32_t norders,
                                  const uint32_t* rows, uint64_t nrows, const Meta* m,
                                  uint32_t radius, uint64_t per, uint64_t* cost, hipStream_t st);
hipError_t launch_pass_compress(const void* x, int dtype, int predictor, void* rec,
                                uint16_t* codes, const PassGeom& g, const Meta* m,
                                uint32_t radius, hipStream_t st);
// the origin and the coarsest levels (L .. l_stop) in one workgroup, their
// lattice in LDS (values and u16 codes within kSmallBytes)
constexpr uint32_t kSmallBytes = 48 * 1024;
struct SmallGeom {
  int ndim;
  int L, l_stop;
  uint32_t cubic;  // bit l - 1: level l cubic
  uint64_t dims[kMaxDims];
  uint64_t stride[kMaxDims];
  uint8_t order[kMaxDims];
  uint8_t pos[kMaxDims];
};
SmallGeom plan_small_levels(int ndim, const uint64_t* dims, const uint8_t* order, int L,
                            uint32_t cubic_mask, int tsize);
hipError_t launch_small_levels_compress(const void* x, int dtype, void* rec, uint16_t* codes,
                                        const SmallGeom& sg, const Meta* m, uint32_t radius,
                                        hipStream_t st);
hipError_t launch_small_levels_recon(const uint16_t* codes, int dtype, void* out,
                                     const SmallGeom& sg, double eb_t, uint32_t radius,
                                     hipStream_t st);
// the first-order Lorenzo predictor: every point, in wavefronts of blocks
hipError_t launch_lorenzo_compress(const void* x, int dtype, void* rec, uint16_t* codes, int ndim,
                                   const uint64_t* dims, const Meta* m, uint32_t radius,
                                   hipStream_t st);
hipError_t launch_lorenzo_recon(const uint16_t* codes, int dtype, void* out, int ndim,
                                const uint64_t* dims, double eb_t, uint32_t radius,
                                hipStream_t st);
hipError_t launch_origin_recon(const uint16_t* codes, int dtype, void* out, double eb_t,
                               uint32_t radius, hipStream_t st);
hipError_t launch_pass_recon(const uint16_t* codes, int dtype, int predictor, void* out,
                             const PassGeom& g, double eb_t, uint32_t radius, hipStream_t st);

// One level of the traversal for fields of up to three dimensions, viewed as
// three dimensions with leading extents of 1, in lattice units of the level
// stride s along the pass order (a, b, c).  A work item is a (b, c) tile and
// a run of planes along a.  See level.hip.
struct LevelGeom {
  uint32_t s;
  uint32_t ext[3];    // lattice extents along a, b, c
  uint64_t fs[3];     // flat-index step of one lattice unit along a, b, c
  uint32_t tile[3];   // planes per item, tile extents along b and c
  uint32_t ntile[3];  // items along a, b, c
  uint32_t planes;    // planes per item (tile[0])
  uint32_t box_b;     // LDS box extents along b and c (tile plus halo, clipped)
  uint32_t box_c;
  uint32_t ring_b;    // coarse-grid extents (even b, even c of the box)
  uint32_t ring_c;
  uint64_t nitems;
  uint32_t box_bytes; // LDS bytes: box | ring of 4 coarse grids | codes of the box
  uint32_t ring_bytes;
  uint32_t lds;
  uint32_t pitch64;   // box rows 64 slots apart, coarse-grid rows 32 (boxes of <= 64 columns)
  // stride-1 level of a three-dimensional field as row strips (fine.hip)
  uint32_t fine;      // 1: planned for the strip kernel
  uint32_t f_waves;   // waves per workgroup (128 columns each)
  uint32_t f_wins;    // column windows
  uint32_t f_atiles;  // plane groups
  uint32_t f_runs;    // row runs
  uint32_t f_rows;    // rows per run (even)
  uint32_t f_items;   // workgroups
};
struct LevelTuning {
  uint32_t target_points;  // minimum number of work items (planes per item shrink to reach it)
  uint32_t tile_b, tile_c; // (b, c) tile extents
  uint32_t lds_bytes;      // LDS budget of one workgroup
  uint32_t fine;           // 0: never plan the strip kernel
  uint32_t fine_rows;      // rows per run of the strip kernel (0: chosen from the shape)
};
constexpr uint32_t kLevelStoreValues = 1u << 0;   // store reconstructed values of the tile
// the stride-2 level also stores its whole lattice (coarser points included)
// compactly, in lattice order, for the strip kernel of the stride-1 level;
// reconstruction then stores no values in the field (the strip kernel
// stores every point)
constexpr uint32_t kLevelStoreCompact = 1u << 1;

// Plans the levels L..1 (coarsest first); false for four dimensions.
bool plan_levels(int ndim, const uint64_t* dims, const uint8_t* order, int tsize,
                 const LevelTuning* tune, std::vector<LevelGeom>& out);
// cmp: the stride-2 lattice, written by the stride-2 level and read by the
// strip kernel (nullptr: neither; the strip kernel reads the field)
hipError_t launch_level_compress(const void* x, int dtype, int predictor, void* rec,
                                 uint16_t* codes, const LevelGeom& g, const Meta* m,
                                 uint32_t radius, bool store_rec, void* cmp, hipStream_t st);
hipError_t launch_level_recon(const uint16_t* codes, int dtype, int predictor, void* out,
                              const LevelGeom& g, double eb_t, uint32_t radius, void* cmp,
                              hipStream_t st);
// The number of levels, L = max over dimensions of ceil(log2 n_d); the
// cubic-level mask of per-level predictors; the bytes of the compact stride-2
// lattice when both the stride-2 level (fixed-pitch kernel) and the strip
// kernel run, else 0 (api.hip).
int level_count(int ndim, const uint64_t* dims);
uint32_t cubic_mask(const int* lvl_pred);
uint64_t compact_bytes(const std::vector<LevelGeom>& levels, int dtype, const void* x,
                       const void* v, uint64_t s_small, size_t tsize);

// The strip kernel of the stride-1 level (fine.hip): planned by plan_fine
// (sets g.fine), launched when fine_usable (the field's pointers hold whole
// column pairs).
bool plan_fine(LevelGeom& g, int tsize, uint32_t rows);
bool fine_usable(const LevelGeom& g, int dtype, const void* x, const void* v);
hipError_t launch_fine_compress(const void* x, int dtype, int predictor, void* rec,
                                uint16_t* codes, const LevelGeom& g, const Meta* m,
                                uint32_t radius, const void* cmp, hipStream_t st);
hipError_t launch_fine_recon(const uint16_t* codes, int dtype, int predictor, void* out,
                             const LevelGeom& g, double eb_t, uint32_t radius, const void* cmp,
                             hipStream_t st);

// Point-wise relative mode (pwrel.hip): the log field's absolute bound, and
// the transforms before and after the pipeline.
double pwrel_delta(double eps, int dtype);
hipError_t launch_pwrel_forward(const void* x, int dtype, double* y, uint64_t* signs, uint64_t n,
                                uint32_t* any, hipStream_t st);
hipError_t launch_pwrel_inverse(const double* y, const uint64_t* signs, uint64_t n, int dtype,
                                void* out, hipStream_t st);
hipError_t launch_pwrel_finish(uint8_t* out, uint64_t ylen, uint64_t off_signs,
                               const uint64_t* signs, uint64_t nsw, uint64_t total, double eps,
                               int dtype, hipStream_t st);

hipError_t launch_histogram(const uint16_t* codes, uint64_t n, uint32_t radius, uint32_t* part,
                            uint32_t* hist, Meta* m, hipStream_t st);
// bytes of the partial-histogram rows launch_histogram needs in `part`
size_t histogram_scratch_bytes();

struct CodebookScratch {
  uint64_t* keys_a;    // kMaxSym
  uint64_t* keys_b;    // kMaxSym
  uint32_t* w;         // 2 * kMaxSym node weights
  uint32_t* parent;    // 2 * kMaxSym
  uint32_t* depth;     // 2 * kMaxSym
  uint32_t* merged;    // kMaxSym
  uint32_t* phase_end; // kMaxSym
  uint16_t* leaf_sym;  // kMaxSym
};
hipError_t launch_codebook(const uint32_t* hist, uint32_t nsym, CodebookScratch s,
                           uint64_t* enc_code, uint8_t* enc_len, uint32_t* symtab, Meta* m,
                           hipStream_t st);

hipError_t launch_exclusive_scan_u32(const uint32_t* in, uint64_t* out, uint64_t n,
                                     uint64_t* block_sums, uint64_t* total, hipStream_t st);
// Both exclusive scans of two u32 arrays with the launches of one scan;
// block_sums holds 2 * ceil(n / 1024) entries; totals to a_total and b_total.
hipError_t launch_scan_pair(const uint32_t* a, const uint32_t* b, uint64_t n, uint64_t* a_off,
                            uint64_t* b_off, uint64_t* block_sums, uint64_t* a_total,
                            uint64_t* b_total, hipStream_t st);

// Encoder scratch: per-chunk sizes and their exclusive scans.
struct EncodeScratch {
  uint32_t* chunk_words;
  uint32_t* chunk_zeros;
  uint64_t* word_off;
  uint64_t* zero_off;
  uint64_t* block_sums;
  uint64_t* totals;
};
// slots: at least n words of scratch (the reconstruction buffer, dead by
// then), where the lane-parallel path packs each chunk before one copy.
hipError_t launch_encode(const uint16_t* codes, const void* x, int dtype, uint64_t n,
                         uint32_t chunk, uint32_t sub, uint32_t radius, const uint64_t* enc_code,
                         const uint8_t* enc_len, EncodeScratch es, uint32_t* slots, uint8_t* out,
                         uint64_t cap, Meta* m, hipStream_t st);
hipError_t launch_write_tables(uint8_t* out, uint64_t capacity, const uint32_t* symtab,
                               uint64_t nchunks, uint32_t sub, const uint8_t* header_template,
                               int dtype, Meta* m, hipStream_t st);

// ---- batches (batch.hip): the fields of a batch share every launch.
// A launch covers a list of jobs (a field, and for the level kernels one of
// its levels); its workgroups map to jobs through a per-workgroup table of job
// indices.  Every job starts on a multiple of 8 workgroups (the padding maps
// to kNoJob and exits at once), so that a job's workgroups are dealt to the
// eight XCDs exactly as a launch of the job alone would deal them.
constexpr uint32_t kNoJob = 0xFFFFFFFFu;

struct BField {
  // written for every call
  const void* x;
  uint8_t* out;
  uint64_t cap;
  double eb_value;
  // fixed by the plan
  int32_t eb_mode, dtype;
  uint64_t n, nchunks;
  uint32_t R, chunk, sub, pad;
  void* rec;
  uint16_t* codes;
  void* cmp;           // the stride-2 lattice, or null
  Meta* m;
  uint32_t* hist;      // 2R bins
  uint32_t* hist_part; // the histogram workgroups' partial rows
  uint64_t* enc_code;  // 2R
  uint8_t* enc_len;    // 2R
  uint32_t* symtab;    // 2R
  CodebookScratch cb;
  uint32_t* chunk_words;  // the field's slices of the batch's chunk tables
  uint32_t* chunk_zeros;
  uint64_t* word_off;     // exclusive scans over the whole batch
  uint64_t* zero_off;
  uint64_t* lword_off;    // the same, from the field's first chunk
  uint64_t* lzero_off;
  SmallGeom sg;
  uint32_t hdr[kHeaderBytes / 4];  // header template (patched on the device)
};

struct BJob {
  uint32_t field, first, nblk, flags;  // flags: kLevelStore* (level kernels)
  LevelGeom g;                         // level kernels only
};

// A launch's tables, as the kernels see them.
struct BLaunch {
  const BField* __restrict__ f;
  const BJob* __restrict__ jobs;
  const uint32_t* __restrict__ wg;  // job of each workgroup
};

// The job of this workgroup and its index inside the job; false for padding.
__device__ __forceinline__ bool batch_job(const BLaunch& L, BJob& j, uint32_t& local) {
  const uint32_t k = __builtin_amdgcn_readfirstlane(L.wg[blockIdx.x]);
  if (k == kNoJob) return false;
  j = L.jobs[k];
  local = blockIdx.x - j.first;
  return true;
}

// One field as sz_compress_batch hands it to the batched path.
struct BatchItem {
  const void* x;
  void* out;
  size_t cap;
  int dtype, ndim;
  uint64_t dims[kMaxDims];
  uint8_t order[kMaxDims];
  int eb_mode;
  double eb;
  int pred;
  uint32_t R, chunk, sub;
  uint8_t hdr[kHeaderBytes];  // header template
  int status;                 // written
  size_t out_size;            // written
};
struct BatchPlan;
void batch_plan_free(BatchPlan* p);
// Whether the batched launches cover a field: 1 to 3 dimensions, linear or
// cubic interpolation, an absolute or range-relative bound, and every level
// on the fixed-pitch or strip kernel.
bool batch_item_supported(const BatchItem& it);
// The plan was built for exactly these fields' shapes and options (so each
// of them is supported).
bool batch_plan_covers(const BatchPlan* plan, const std::vector<BatchItem>& items);
// Compresses the items (validated, one radius, chunk and sub-chunk count) with
// shared launches; *plan is the cached plan (rebuilt when the shapes or
// options change).  Returns SZ_OK with each item's status and size set, or an
// error for all of them (err says why).
int batch_compress(int device, BatchPlan** plan, std::vector<BatchItem>& items, hipStream_t st,
                   std::string& err);

hipError_t launch_b_meta_init(const BField* f, uint32_t nf, hipStream_t st);
hipError_t launch_b_minmax(int dtype, BLaunch L, uint32_t nwg, hipStream_t st);
hipError_t launch_b_resolve_eb(const BField* f, uint32_t nf, hipStream_t st);
hipError_t launch_b_small_levels(int dtype, BLaunch L, uint32_t nwg, hipStream_t st);
hipError_t launch_b_level(int dtype, int predictor, BLaunch L, uint32_t nwg, uint32_t lds,
                          hipStream_t st);
hipError_t launch_b_fine(int dtype, int predictor, uint32_t waves, BLaunch L, uint32_t nwg,
                         hipStream_t st);
hipError_t launch_b_histogram(BLaunch L, uint32_t nwg, hipStream_t st);
// sums each field's partial rows (a job per field; flags = the field's rows)
hipError_t launch_b_hist_reduce(BLaunch L, uint32_t nwg, hipStream_t st);
uint32_t hist_reduce_blocks();  // workgroups of a field's reduction
size_t hist_row_words();        // u32 words of one partial row
hipError_t launch_b_codebook(BLaunch L, uint32_t nwg, hipStream_t st);
hipError_t launch_b_encode_size(BLaunch L, uint32_t nwg, hipStream_t st);
// field-local chunk offsets from the batch-wide scans, and each field's totals
hipError_t launch_b_rebase(BLaunch L, uint32_t nwg, hipStream_t st);
hipError_t launch_b_encode_pack(int dtype, BLaunch L, uint32_t nwg, hipStream_t st);
// the lane-parallel path's second pass (the slots' copy), a wave per chunk
hipError_t launch_b_encode_copy(int dtype, BLaunch L, uint32_t nwg, hipStream_t st);
uint32_t encode_copy_blocks(uint64_t nchunks);
uint32_t encode_pack_blocks(uint64_t nchunks);  // the second pass of codes over 32 bits
hipError_t launch_b_write_tables(BLaunch L, uint32_t nwg, hipStream_t st);
// each field's (stream bytes, status bits) into res[2 i], res[2 i + 1]
hipError_t launch_b_results(const BField* f, uint32_t nf, uint64_t* res, hipStream_t st);

// Codes longer than the lookup table: with canonical codes the left-justified
// end of each length's code range grows with the length, and comparing the
// window against the end of length k only involves its first k bits, so the
// code length is kLutBits + 1 plus the number of ends the window reaches.
// Lengths up to 32 are resolved from a 32-bit window with ends held in
// registers; longer ones (only possible for extremely skewed histograms) take
// an exact path that re-reads the stream.
constexpr int kWinLens = 32 - kLutBits;  // lengths resolved from the window
constexpr uint32_t kLongSymCap = 4096;   // long-code symbols a decoder block keeps in LDS
struct LongCodes {
  uint64_t end_lj[kMaxCodeLen + 1];  // left-justified end of length-l codes
  uint64_t base[kMaxCodeLen + 1];    // offset[l] - first[l] (mod 2^64)
  uint32_t lim[kWinLens];            // window limits of lengths l0, l0 + 1, ...
  uint32_t l0;                       // shortest long length whose 32-bit end is not 0
  uint32_t base32[34];               // offset[l] - first[l] - long_first (mod 2^32)
  uint32_t max_len;
  uint32_t long_first;               // sorted index of the first long code
  uint32_t long_in_lds;
  uint32_t pad;
};

// Second level of the lookup: the first kL2Prefixes table windows that begin
// codes longer than the table each get kL2Entries entries, indexed by the
// next kL2Bits bits: sym | len << 16 when the code is at most kLutBits +
// kL2Bits long, else 0 (the window limits resolve it).
constexpr uint32_t kL2Bits = 6, kL2Prefixes = 16, kL2Entries = 1u << kL2Bits;
struct DecodeTables {
  LongCodes* lc;         // derived by the table kernel for the chunk decoder
  uint32_t* lut;         // 1 << kLutBits entries: sym | len << 16 (len 0 = longer code)
  uint64_t* lut2;        // 1 << kLutBits entries: up to three whole codes of the window,
                         // or (count 0) the window's second-level block, 0xFFFF for none
  uint32_t* l2;          // kL2Prefixes * kL2Entries second-level entries
  uint64_t* first;       // kMaxCodeLen + 1
  uint32_t* count;       // kMaxCodeLen + 1
  uint32_t* offset;      // kMaxCodeLen + 1
  uint16_t* sorted_sym;  // kMaxSym, by (length, symbol)
  uint64_t* keys_a;
  uint64_t* keys_b;
};
// The decoding tables (block 0), the chunk table's scans (word and
// unpredictable offsets of every chunk within its slice of kSliceEntries
// chunks, the slices' carries in block_sums, totals checked against the
// header) and a read of the stream's stream_bytes that brings it into the
// Infinity Cache for the chunk decoder, in one launch.
hipError_t launch_decode_front(const uint8_t* stream, uint64_t stream_bytes, uint64_t off_sym,
                               uint32_t nsym_used,
                               uint32_t nsym, DecodeTables t, uint64_t off_chunk, uint64_t nchunks,
                               uint32_t* chunk_words, uint32_t* chunk_unpred, uint64_t* word_off,
                               uint64_t* unpred_off, uint64_t* block_sums, uint64_t* totals,
                               uint64_t total_words, uint64_t n_unpred, Meta* m, hipStream_t st);
// The same before the host has the header: the kernel reads the fields it
// needs from the stream's header in device memory and does nothing when they
// fail the host's checks or the chunk buffers hold fewer than cap chunks.
hipError_t launch_decode_front_early(const uint8_t* stream, uint64_t stream_size, uint64_t cap,
                                     DecodeTables t, uint32_t* chunk_words, uint32_t* chunk_unpred,
                                     uint64_t* word_off, uint64_t* unpred_off,
                                     uint64_t* block_sums, uint64_t* totals, Meta* m,
                                     hipStream_t st);
hipError_t launch_decode_chunks(const uint8_t* stream, uint64_t stream_size, uint64_t off_sub,
                                uint64_t off_unpred, uint64_t off_bits, uint64_t total_words,
                                uint64_t n_unpred, uint64_t n, uint32_t chunk, uint32_t sub,
                                uint32_t nsym_used, int dtype, const uint32_t* chunk_words,
                                const uint32_t* chunk_unpred, const uint64_t* word_off,
                                const uint64_t* unpred_off, const uint64_t* carry, DecodeTables t,
                                uint16_t* codes, void* out, Meta* m, hipStream_t st);
hipError_t launch_check_totals(const uint64_t* totals, uint64_t total_words, uint64_t n_unpred,
                               Meta* m, hipStream_t st);

}  // namespace szg
