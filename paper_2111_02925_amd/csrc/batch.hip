// Batched compression: the fields of a batch share every launch.
//
// Paper: SZ3 (arXiv 2111.02925), Algorithm 1 (Section 3.3) run for many
// fields at once; each field's stream is the one sz_compress writes for it
// alone (the kernels are the same bodies, only the launches are shared).
//
// A plan, built once for a batch's shapes and options and reused while they
// repeat, holds:
//   - every field's scratch (reconstruction, codes, the stride-2 lattice,
//     Meta, histogram, codebook and encoder tables) in one device arena;
//   - the chunk tables of all fields concatenated, so that one scan serves
//     every field (k_b_rebase makes the offsets field-local);
//   - a list of steps: one launch per stage, and per level stride one launch
//     for each (kernel, dtype, predictor) group of the fields that have that
//     level (the per-level work lists), each launch's jobs and the job of
//     each workgroup;
//   - the steps captured once in a HIP graph, replayed by every call.
// A call writes the fields' pointers and bounds into the plan's field table
// (one copy to the device), replays the graph, and copies every field's
// (stream bytes, status) back in one transfer: one host synchronisation for
// the whole batch.
//
// Tiles never change the bytes (the work items of a level write disjoint
// points with the same arithmetic), so the plan's first call may time every
// level under a few tilings and keep the fastest per level stride.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"

namespace szg {

namespace {

enum class Op : uint8_t {
  MetaInit, Minmax, Resolve, Small, Level, Fine, FillHist, Hist, HistReduce, Codebook, EncSize,
  Scan, Rebase, Pack, Copy, Tables, Results
};

struct Step {
  Op op;
  int dtype = 0, pred = 0;
  uint32_t waves = 0, lds = 0;
  uint32_t job0 = 0, wg0 = 0, nwg = 0;
  uint32_t stride = 0;  // level steps
};

uint64_t up256(uint64_t v) { return (v + 255) & ~uint64_t(255); }
uint32_t cdiv32(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }
// histogram workgroups (and partial rows) of a field of n points
uint32_t hist_blocks(uint64_t n) {
  return std::min<uint32_t>(256, std::max<uint32_t>(1, cdiv32(n, 65536)));
}

// The tilings the first call of a plan tries for each level stride.
const LevelTuning kTunings[] = {
    {2048, 32, 58, 64 * 1024, 1, 0},   // the single-field default
    {4096, 16, 58, 64 * 1024, 1, 16},  // more, shorter items
    {1024, 32, 58, 64 * 1024, 1, 32},  // fewer, longer items
    {8192, 8, 58, 64 * 1024, 1, 8},
};
constexpr int kNumTunings = sizeof(kTunings) / sizeof(kTunings[0]);

}  // namespace

struct BatchPlan {
  int device = 0;
  std::vector<uint64_t> key;  // shapes and options the plan was built for
  uint32_t nf = 0;
  std::vector<BField> fields;  // host copy (the plan's pointers; per-call values rewritten)
  std::vector<uint64_t> s_small;
  std::vector<std::vector<LevelGeom>> levels[kNumTunings];  // per tuning, per field
  std::vector<int> choice;  // tuning of each level stride (index = log2 stride)
  // device
  void* arena = nullptr;
  BField* d_fields = nullptr;
  BField* h_fields = nullptr;  // pinned staging of the field table
  uint64_t* d_res = nullptr;
  uint64_t* h_res = nullptr;   // pinned
  uint32_t* hist_all = nullptr;
  uint64_t hist_words = 0;
  uint32_t* cw_all = nullptr;
  uint32_t* cz_all = nullptr;
  uint64_t* wo_all = nullptr;
  uint64_t* zo_all = nullptr;
  uint64_t* block_sums = nullptr;
  uint64_t* totals = nullptr;
  uint64_t nchunks = 0;
  // steps and their tables
  std::vector<Step> steps;
  std::vector<BJob> jobs;
  std::vector<uint32_t> wg;
  BJob* d_jobs = nullptr;
  uint32_t* d_wg = nullptr;
  size_t jobs_cap = 0, wg_cap = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
  bool use_graph = true;
  int forced = -1;  // a tiling every stride takes (no tuning), or -1

  ~BatchPlan() {
    (void)hipSetDevice(device);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void* p : {(void*)arena, (void*)d_fields, (void*)d_res, (void*)d_jobs, (void*)d_wg})
      if (p) (void)hipFree(p);
    if (h_fields) (void)hipHostFree(h_fields);
    if (h_res) (void)hipHostFree(h_res);
  }
};

void batch_plan_free(BatchPlan* p) { delete p; }

namespace {

std::vector<uint64_t> plan_key(const std::vector<BatchItem>& items) {
  std::vector<uint64_t> k;
  k.reserve(items.size() * 10);
  for (const BatchItem& it : items) {
    k.push_back((uint64_t)it.dtype | (uint64_t)it.ndim << 8 | (uint64_t)it.eb_mode << 16 |
                (uint64_t)it.pred << 24 | (uint64_t)it.order[0] << 32 |
                (uint64_t)it.order[1] << 40 | (uint64_t)it.order[2] << 48 |
                (uint64_t)it.order[3] << 56);
    for (int d = 0; d < 4; d++) k.push_back(it.dims[d]);
    k.push_back((uint64_t)it.R | (uint64_t)it.chunk << 32);
    k.push_back(it.sub);
  }
  return k;
}

// The levels below the coarsest-levels workgroup's and their kernels: every
// one must be the fixed-pitch kernel's or (stride 1) the strip kernel's.
bool levels_batchable(const std::vector<LevelGeom>& levels, uint64_t s_small, int dtype,
                      const void* rec) {
  for (const LevelGeom& g : levels) {
    if (g.s >= s_small) continue;
    // a 16-byte aligned field and an arena pointer hold whole column pairs
    if (g.s == 1 && fine_usable(g, dtype, rec, rec)) continue;
    if (!g.pitch64) return false;
  }
  return true;
}

}  // namespace

bool batch_item_supported(const BatchItem& it) {
  if (it.ndim < 1 || it.ndim > 3) return false;
  if (it.pred != SZ_INTERP_LINEAR && it.pred != SZ_INTERP_CUBIC) return false;
  if (it.eb_mode != SZ_EB_ABS && it.eb_mode != SZ_EB_REL) return false;
  uint64_t n = 1;
  for (int d = 0; d < it.ndim; d++) n *= it.dims[d];
  if (n == 0) return false;
  const int tsize = it.dtype == SZ_F64 ? 8 : 4;
  const int L = level_count(it.ndim, it.dims);
  int lvl_pred[kMaxLevels + 1];
  for (int l = 0; l <= kMaxLevels; l++) lvl_pred[l] = it.pred;
  const SmallGeom sg = plan_small_levels(it.ndim, it.dims, it.order, L, cubic_mask(lvl_pred), tsize);
  const uint64_t s_small = 1ull << (sg.l_stop - 1);
  alignas(16) static const double probe[2] = {0, 0};
  for (int t = 0; t < kNumTunings; t++) {
    std::vector<LevelGeom> levels;
    if (!plan_levels(it.ndim, it.dims, it.order, tsize, &kTunings[t], levels)) return false;
    if (!levels_batchable(levels, s_small, it.dtype, probe)) return false;
  }
  return true;
}

bool batch_plan_covers(const BatchPlan* plan, const std::vector<BatchItem>& items) {
  return plan && !items.empty() && plan->key == plan_key(items);
}

namespace {

hipError_t dev_alloc(void** p, size_t bytes) { return hipMalloc(p, bytes ? bytes : 8); }

// Builds the plan's scratch and field table (everything but the steps).
int build_plan(BatchPlan& P, const std::vector<BatchItem>& items, std::string& err) {
  P.nf = (uint32_t)items.size();
  P.fields.assign(P.nf, BField{});
  P.s_small.assign(P.nf, 0);
  for (int t = 0; t < kNumTunings; t++) P.levels[t].assign(P.nf, {});
  std::vector<uint64_t> cmp_bytes(P.nf, 0);
  // sizes, in arena order: per field rec, codes, cmp, meta, enc tables,
  // codebook scratch; then the batch's histograms and chunk tables
  uint64_t total = 0, nch_all = 0;
  std::vector<uint64_t> off(P.nf * 16, 0), c0s(P.nf, 0), rows0(P.nf, 0);
  uint64_t rows_all = 0;
  for (uint32_t i = 0; i < P.nf; i++) {
    const BatchItem& it = items[i];
    BField& f = P.fields[i];
    const int tsize = it.dtype == SZ_F64 ? 8 : 4;
    uint64_t n = 1;
    for (int d = 0; d < it.ndim; d++) n *= it.dims[d];
    f.dtype = it.dtype;
    f.eb_mode = it.eb_mode;
    f.n = n;
    f.R = it.R;
    f.chunk = it.chunk;
    f.sub = it.sub;
    f.nchunks = (n + it.chunk - 1) / it.chunk;
    const int L = level_count(it.ndim, it.dims);
    int lvl_pred[kMaxLevels + 1];
    for (int l = 0; l <= kMaxLevels; l++) lvl_pred[l] = it.pred;
    f.sg = plan_small_levels(it.ndim, it.dims, it.order, L, cubic_mask(lvl_pred), tsize);
    P.s_small[i] = 1ull << (f.sg.l_stop - 1);
    for (int t = 0; t < kNumTunings; t++)
      if (!plan_levels(it.ndim, it.dims, it.order, tsize, &kTunings[t], P.levels[t][i])) {
        err = "field " + std::to_string(i) + ": no level plan";
        return SZ_ERR_UNSUPPORTED;
      }
    alignas(16) static const double probe[2] = {0, 0};
    cmp_bytes[i] = compact_bytes(P.levels[0][i], it.dtype, probe, probe, P.s_small[i], tsize);
    const uint64_t nsym = 2ull * it.R;
    const uint64_t sizes[] = {n * tsize, ((n + 7) & ~7ull) * 2, cmp_bytes[i], sizeof(Meta),
                              8 * nsym, (nsym + 15) & ~15ull, 4 * nsym,
                              // codebook scratch, as the context's
                              8ull * kMaxSym, 8ull * kMaxSym, 8ull * kMaxSym, 8ull * kMaxSym,
                              8ull * kMaxSym, 4ull * kMaxSym, 4ull * kMaxSym, 2ull * kMaxSym};
    for (int k = 0; k < 15; k++) {
      off[i * 16 + k] = total;
      total += up256(sizes[k] ? sizes[k] : 8);
    }
    c0s[i] = nch_all;
    nch_all += f.nchunks;
    rows0[i] = rows_all;
    rows_all += hist_blocks(n);
  }
  P.nchunks = nch_all;
  const uint64_t nsym = 2ull * items[0].R;  // one radius per batch
  P.hist_words = nsym * P.nf;
  const uint64_t off_hist = total;
  total += up256(4 * P.hist_words);
  const uint64_t off_rows = total;
  total += up256(4 * rows_all * hist_row_words());
  const uint64_t off_cw = total;
  total += up256(4 * (nch_all + 1));
  const uint64_t off_cz = total;
  total += up256(4 * (nch_all + 1));
  const uint64_t off_wo = total;
  total += up256(8 * (nch_all + 1));
  const uint64_t off_zo = total;
  total += up256(8 * (nch_all + 1));
  const uint64_t off_lwo = total;
  total += up256(8 * (nch_all + 1));
  const uint64_t off_lzo = total;
  total += up256(8 * (nch_all + 1));
  const uint64_t off_bs = total;
  total += up256(8 * (2 * ((nch_all + 1023) / 1024) + 2));
  const uint64_t off_tot = total;
  total += 256;
  if (dev_alloc(&P.arena, total) != hipSuccess) {
    err = "hipMalloc of " + std::to_string(total) + " bytes for the batch";
    return SZ_ERR_NOMEM;
  }
  uint8_t* A = static_cast<uint8_t*>(P.arena);
  P.hist_all = reinterpret_cast<uint32_t*>(A + off_hist);
  P.cw_all = reinterpret_cast<uint32_t*>(A + off_cw);
  P.cz_all = reinterpret_cast<uint32_t*>(A + off_cz);
  P.wo_all = reinterpret_cast<uint64_t*>(A + off_wo);
  P.zo_all = reinterpret_cast<uint64_t*>(A + off_zo);
  uint64_t* lwo = reinterpret_cast<uint64_t*>(A + off_lwo);
  uint64_t* lzo = reinterpret_cast<uint64_t*>(A + off_lzo);
  P.block_sums = reinterpret_cast<uint64_t*>(A + off_bs);
  P.totals = reinterpret_cast<uint64_t*>(A + off_tot);
  for (uint32_t i = 0; i < P.nf; i++) {
    BField& f = P.fields[i];
    const uint64_t c0 = c0s[i];
    const uint64_t* o = &off[i * 16];
    f.rec = A + o[0];
    f.codes = reinterpret_cast<uint16_t*>(A + o[1]);
    f.cmp = cmp_bytes[i] ? A + o[2] : nullptr;
    f.m = reinterpret_cast<Meta*>(A + o[3]);
    f.enc_code = reinterpret_cast<uint64_t*>(A + o[4]);
    f.enc_len = A + o[5];
    f.symtab = reinterpret_cast<uint32_t*>(A + o[6]);
    f.cb.keys_a = reinterpret_cast<uint64_t*>(A + o[7]);
    f.cb.keys_b = reinterpret_cast<uint64_t*>(A + o[8]);
    f.cb.w = reinterpret_cast<uint32_t*>(A + o[9]);
    f.cb.parent = reinterpret_cast<uint32_t*>(A + o[10]);
    f.cb.depth = reinterpret_cast<uint32_t*>(A + o[11]);
    f.cb.merged = reinterpret_cast<uint32_t*>(A + o[12]);
    f.cb.phase_end = reinterpret_cast<uint32_t*>(A + o[13]);
    f.cb.leaf_sym = reinterpret_cast<uint16_t*>(A + o[14]);
    f.hist = P.hist_all + (uint64_t)i * nsym;
    f.hist_part = reinterpret_cast<uint32_t*>(A + off_rows) + rows0[i] * hist_row_words();
    f.chunk_words = P.cw_all + c0;
    f.chunk_zeros = P.cz_all + c0;
    f.word_off = P.wo_all + c0;
    f.zero_off = P.zo_all + c0;
    f.lword_off = lwo + c0;
    f.lzero_off = lzo + c0;
  }
  if (dev_alloc((void**)&P.d_fields, sizeof(BField) * P.nf) != hipSuccess ||
      dev_alloc((void**)&P.d_res, sizeof(uint64_t) * 2 * P.nf) != hipSuccess ||
      hipHostMalloc((void**)&P.h_fields, sizeof(BField) * P.nf, hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&P.h_res, sizeof(uint64_t) * 2 * P.nf, hipHostMallocDefault) !=
          hipSuccess) {
    err = "allocation of the batch tables";
    return SZ_ERR_NOMEM;
  }
  return SZ_OK;
}

// Appends a step whose jobs are (field, workgroups); pad8: each job starts on
// a multiple of 8 workgroups (the level kernels' XCD-aware item order).
void add_step(BatchPlan& P, Step st, const std::vector<BJob>& js, bool pad8) {
  st.job0 = (uint32_t)P.jobs.size();
  st.wg0 = (uint32_t)P.wg.size();
  uint32_t nwg = 0;
  for (BJob j : js) {
    if (j.nblk == 0) continue;
    if (pad8)
      while (nwg & 7u) {
        P.wg.push_back(kNoJob);
        nwg++;
      }
    j.first = nwg;
    const uint32_t k = (uint32_t)P.jobs.size() - st.job0;
    P.jobs.push_back(j);
    for (uint32_t b = 0; b < j.nblk; b++) P.wg.push_back(k);
    nwg += j.nblk;
  }
  st.nwg = nwg;
  if (nwg) P.steps.push_back(st);
}

BJob field_job(uint32_t f, uint32_t nblk) {
  BJob j{};
  j.field = f;
  j.nblk = nblk;
  return j;
}

// The steps of the batch with tiling `choice[log2 stride]` per level stride
// (tune >= 0: every stride takes tiling `tune`).
void build_steps(BatchPlan& P, const std::vector<BatchItem>& items, const std::vector<int>& choice,
                 int tune) {
  P.steps.clear();
  P.jobs.clear();
  P.wg.clear();
  const uint32_t nf = P.nf;
  Step s{};
  s.op = Op::MetaInit;
  P.steps.push_back(s);
  for (int dt : {SZ_F32, SZ_F64}) {
    std::vector<BJob> js;
    // (a workgroup per 64K points, at most 512 a field: longer grid-stride
    // runs read faster, as in the single-field range pass)
    for (uint32_t i = 0; i < nf; i++)
      if (P.fields[i].dtype == dt && P.fields[i].eb_mode == SZ_EB_REL)
        js.push_back(field_job(i, std::min<uint32_t>(512, std::max<uint32_t>(1, cdiv32(P.fields[i].n, 256 * 256)))));
    Step m{};
    m.op = Op::Minmax;
    m.dtype = dt;
    add_step(P, m, js, false);
  }
  s.op = Op::Resolve;
  P.steps.push_back(s);
  for (int dt : {SZ_F32, SZ_F64}) {
    std::vector<BJob> js;
    for (uint32_t i = 0; i < nf; i++)
      if (P.fields[i].dtype == dt) js.push_back(field_job(i, 1));
    Step m{};
    m.op = Op::Small;
    m.dtype = dt;
    add_step(P, m, js, false);
  }
  // the levels below each field's coarsest-levels workgroup, by stride
  uint32_t smax = 0;
  for (uint32_t i = 0; i < nf; i++)
    for (const LevelGeom& g : P.levels[0][i])
      if (g.s < P.s_small[i]) smax = std::max(smax, g.s);
  for (uint32_t sp = smax; sp >= 1; sp /= 2) {
    const int lg = __builtin_ctz(sp);
    const int t = tune >= 0 ? tune : (lg < (int)choice.size() ? choice[lg] : 0);
    // groups: (fine?, dtype, predictor, waves)
    std::map<std::tuple<int, int, int, uint32_t>, std::vector<BJob>> groups;
    std::map<std::tuple<int, int, int, uint32_t>, uint32_t> lds;
    for (uint32_t i = 0; i < nf; i++) {
      if (sp >= P.s_small[i]) continue;
      const BatchItem& it = items[i];
      const void* rec = P.fields[i].rec;
      // the stride-2 level stores the compact lattice when the strip kernel
      // runs the stride-1 level (under this tiling) and reads it
      bool fine1 = false;
      for (const LevelGeom& g : P.levels[t][i])
        if (g.s == 1) fine1 = fine_usable(g, it.dtype, rec, rec);
      for (const LevelGeom& g : P.levels[t][i]) {
        if (g.s != sp) continue;
        BJob j{};
        j.field = i;
        j.g = g;
        if (sp == 1 && fine1) {
          j.nblk = g.f_items;
          j.flags = 0;
          groups[{1, it.dtype, it.pred, g.f_waves}].push_back(j);
        } else {
          const bool compact = P.fields[i].cmp && fine1 && g.s == 2 && g.pitch64;
          j.nblk = (uint32_t)g.nitems;
          j.flags = compact ? kLevelStoreCompact : (g.s > 1 ? kLevelStoreValues : 0u);
          auto key = std::make_tuple(0, it.dtype, it.pred, 0u);
          groups[key].push_back(j);
          lds[key] = std::max(lds[key], g.lds);
        }
      }
    }
    for (auto& kv : groups) {
      Step m{};
      m.op = std::get<0>(kv.first) ? Op::Fine : Op::Level;
      m.dtype = std::get<1>(kv.first);
      m.pred = std::get<2>(kv.first);
      m.waves = std::get<3>(kv.first);
      m.lds = m.op == Op::Level ? lds[kv.first] : 0;
      m.stride = sp;
      add_step(P, m, kv.second, true);
    }
    if (sp == 1) break;
  }
  s.op = Op::FillHist;
  P.steps.push_back(s);
  {
    std::vector<BJob> js;
    for (uint32_t i = 0; i < nf; i++)
      js.push_back(field_job(i, hist_blocks(P.fields[i].n)));
    Step m{};
    m.op = Op::Hist;
    add_step(P, m, js, false);
  }
  {
    std::vector<BJob> js;
    for (uint32_t i = 0; i < nf; i++) {
      BJob j = field_job(i, hist_reduce_blocks());
      j.flags = hist_blocks(P.fields[i].n);  // the rows to sum
      js.push_back(j);
    }
    Step m{};
    m.op = Op::HistReduce;
    add_step(P, m, js, false);
  }
  {
    std::vector<BJob> js;
    for (uint32_t i = 0; i < nf; i++) js.push_back(field_job(i, 1));
    Step m{};
    m.op = Op::Codebook;
    add_step(P, m, js, false);
  }
  auto enc_blocks = [&](uint32_t i) {
    return std::min<uint32_t>(2048, std::max<uint32_t>(1, cdiv32(P.fields[i].nchunks, 4)));
  };
  {
    std::vector<BJob> js;
    for (uint32_t i = 0; i < nf; i++) js.push_back(field_job(i, enc_blocks(i)));
    Step m{};
    m.op = Op::EncSize;
    add_step(P, m, js, false);
  }
  s.op = Op::Scan;
  P.steps.push_back(s);
  {
    std::vector<BJob> js;
    for (uint32_t i = 0; i < nf; i++)
      js.push_back(field_job(i, std::min<uint32_t>(64, std::max<uint32_t>(1, cdiv32(P.fields[i].nchunks, 256)))));
    Step m{};
    m.op = Op::Rebase;
    add_step(P, m, js, false);
  }
  for (int dt : {SZ_F32, SZ_F64}) {
    std::vector<BJob> js, jc;
    for (uint32_t i = 0; i < nf; i++)
      if (P.fields[i].dtype == dt) {
        js.push_back(field_job(i, encode_pack_blocks(P.fields[i].nchunks)));
        jc.push_back(field_job(i, encode_copy_blocks(P.fields[i].nchunks)));
      }
    Step m{};
    m.op = Op::Pack;
    m.dtype = dt;
    add_step(P, m, js, false);
    m.op = Op::Copy;
    add_step(P, m, jc, false);
  }
  {
    std::vector<BJob> js;
    for (uint32_t i = 0; i < nf; i++) js.push_back(field_job(i, 4));
    Step m{};
    m.op = Op::Tables;
    add_step(P, m, js, false);
  }
  s.op = Op::Results;
  P.steps.push_back(s);
}

// Copies the steps' tables to the device (growing them when needed).
hipError_t upload_steps(BatchPlan& P, hipStream_t st) {
  if (P.jobs.size() > P.jobs_cap) {
    if (P.d_jobs) (void)hipFree(P.d_jobs);
    P.d_jobs = nullptr;
    P.jobs_cap = P.jobs.size() + P.jobs.size() / 4 + 8;
    hipError_t e = hipMalloc((void**)&P.d_jobs, sizeof(BJob) * P.jobs_cap);
    if (e != hipSuccess) return e;
  }
  if (P.wg.size() > P.wg_cap) {
    if (P.d_wg) (void)hipFree(P.d_wg);
    P.d_wg = nullptr;
    P.wg_cap = P.wg.size() + P.wg.size() / 4 + 64;
    hipError_t e = hipMalloc((void**)&P.d_wg, sizeof(uint32_t) * P.wg_cap);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipMemcpyAsync(P.d_jobs, P.jobs.data(), sizeof(BJob) * P.jobs.size(),
                                hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(P.d_wg, P.wg.data(), sizeof(uint32_t) * P.wg.size(), hipMemcpyHostToDevice,
                     st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);  // (the host tables may change after this)
}

hipError_t run_step(BatchPlan& P, const Step& s, hipStream_t st) {
  const BLaunch L{P.d_fields, P.d_jobs + s.job0, P.d_wg + s.wg0};
  switch (s.op) {
    case Op::MetaInit: return launch_b_meta_init(P.d_fields, P.nf, st);
    case Op::Minmax: return launch_b_minmax(s.dtype, L, s.nwg, st);
    case Op::Resolve: return launch_b_resolve_eb(P.d_fields, P.nf, st);
    case Op::Small: return launch_b_small_levels(s.dtype, L, s.nwg, st);
    case Op::Level: return launch_b_level(s.dtype, s.pred, L, s.nwg, s.lds, st);
    case Op::Fine: return launch_b_fine(s.dtype, s.pred, s.waves, L, s.nwg, st);
    case Op::FillHist: return launch_fill_u32(P.hist_all, 0, P.hist_words, st);
    case Op::Hist: return launch_b_histogram(L, s.nwg, st);
    case Op::HistReduce: return launch_b_hist_reduce(L, s.nwg, st);
    case Op::Codebook: return launch_b_codebook(L, s.nwg, st);
    case Op::EncSize: return launch_b_encode_size(L, s.nwg, st);
    case Op::Scan:
      return launch_scan_pair(P.cw_all, P.cz_all, P.nchunks, P.wo_all, P.zo_all, P.block_sums,
                              P.totals, P.totals + 1, st);
    case Op::Rebase: return launch_b_rebase(L, s.nwg, st);
    case Op::Pack: return launch_b_encode_pack(s.dtype, L, s.nwg, st);
    case Op::Copy: return launch_b_encode_copy(s.dtype, L, s.nwg, st);
    case Op::Tables: return launch_b_write_tables(L, s.nwg, st);
    case Op::Results: return launch_b_results(P.d_fields, P.nf, P.d_res, st);
  }
  return hipErrorInvalidValue;
}

hipError_t run_steps(BatchPlan& P, hipStream_t st) {
  for (const Step& s : P.steps) {
    hipError_t e = run_step(P, s, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Times each level stride's launches under every tiling (events around the
// stride's steps) and keeps the fastest tiling per stride.  The inputs are the
// call's own fields; every run writes the same bytes.
hipError_t autotune(BatchPlan& P, const std::vector<BatchItem>& items, hipStream_t st) {
  uint32_t smax = 0;
  for (uint32_t i = 0; i < P.nf; i++)
    for (const LevelGeom& g : P.levels[0][i])
      if (g.s < P.s_small[i]) smax = std::max(smax, g.s);
  const int nlev = smax ? __builtin_ctz(smax) + 1 : 0;
  std::vector<std::vector<float>> ms(kNumTunings, std::vector<float>(nlev, 0.f));
  hipEvent_t ev[2 * 33];
  for (int k = 0; k < 2 * (nlev + 1); k++) (void)hipEventCreate(&ev[k]);
  hipError_t e = hipSuccess;
  for (int t = 0; t < kNumTunings && e == hipSuccess; t++) {
    build_steps(P, items, {}, t);
    e = upload_steps(P, st);
    const size_t ns = P.steps.size();
    auto stride_of = [&](size_t k) -> int {
      const Step& s = P.steps[k];
      return s.op == Op::Level || s.op == Op::Fine ? (int)s.stride : 0;
    };
    for (int rep = 0; rep < 2 && e == hipSuccess; rep++) {  // the second run is timed
      for (size_t k = 0; k < ns; k++) {
        // events before a stride's first launch and after its last
        const int sp = stride_of(k);
        const int lg = sp ? __builtin_ctz((uint32_t)sp) : 0;
        if (sp && (k == 0 || stride_of(k - 1) != sp)) (void)hipEventRecord(ev[2 * lg], st);
        e = run_step(P, P.steps[k], st);
        if (e != hipSuccess) break;
        if (sp && (k + 1 == ns || stride_of(k + 1) != sp)) (void)hipEventRecord(ev[2 * lg + 1], st);
      }
      if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    for (int lg = 0; lg < nlev && e == hipSuccess; lg++) {
      float v = 0;
      if (hipEventElapsedTime(&v, ev[2 * lg], ev[2 * lg + 1]) == hipSuccess) ms[t][lg] = v;
    }
  }
  for (int k = 0; k < 2 * (nlev + 1); k++) (void)hipEventDestroy(ev[k]);
  if (e != hipSuccess) return e;
  P.choice.assign(nlev, 0);
  for (int lg = 0; lg < nlev; lg++)
    for (int t = 1; t < kNumTunings; t++)
      if (ms[t][lg] < ms[P.choice[lg]][lg]) P.choice[lg] = t;
  return hipSuccess;
}

}  // namespace

int batch_compress(int device, BatchPlan** plan_slot, std::vector<BatchItem>& items,
                   hipStream_t st, std::string& err) {
  if (items.empty()) return SZ_OK;
  const std::vector<uint64_t> key = plan_key(items);
  // SZG_BATCH_TILING=t: every level stride takes tiling t (no tuning);
  // SZG_BATCH_GRAPH=0: launches without the graph; SZG_BATCH_TUNE=0: the
  // default tiling without tuning
  int forced = -1;
  if (const char* t = getenv("SZG_BATCH_TILING")) {
    forced = atoi(t);
    if (forced < 0 || forced >= kNumTunings) forced = -1;
  }
  bool use_graph = true;
  if (const char* g = getenv("SZG_BATCH_GRAPH")) use_graph = strcmp(g, "0") != 0;
  BatchPlan* P = *plan_slot;
  bool fresh = false;
  if (!P || P->key != key || P->forced != forced || P->use_graph != use_graph) {
    delete P;
    *plan_slot = nullptr;
    P = new BatchPlan();
    P->device = device;
    P->key = key;
    P->forced = forced;
    P->use_graph = use_graph;
    int rc = build_plan(*P, items, err);
    if (rc) {
      delete P;
      return rc;
    }
    *plan_slot = P;
    fresh = true;
  }
  // this call's pointers, bounds and headers into the field table
  for (uint32_t i = 0; i < P->nf; i++) {
    BField& f = P->fields[i];
    f.x = items[i].x;
    f.out = static_cast<uint8_t*>(items[i].out);
    f.cap = items[i].cap;
    f.eb_value = items[i].eb;
    for (int w = 0; w < (int)(kHeaderBytes / 4); w++)
      f.hdr[w] = items[i].hdr[4 * w] | (items[i].hdr[4 * w + 1] << 8) |
                 (items[i].hdr[4 * w + 2] << 16) | ((uint32_t)items[i].hdr[4 * w + 3] << 24);
  }
  memcpy(P->h_fields, P->fields.data(), sizeof(BField) * P->nf);
  hipError_t e = hipMemcpyAsync(P->d_fields, P->h_fields, sizeof(BField) * P->nf,
                                hipMemcpyHostToDevice, st);
  const bool tune = fresh && forced < 0 &&
                    !(getenv("SZG_BATCH_TUNE") && strcmp(getenv("SZG_BATCH_TUNE"), "0") == 0);
  if (e == hipSuccess && fresh) {
    P->choice.clear();
    if (tune) e = autotune(*P, items, st);
    if (e == hipSuccess) {
      build_steps(*P, items, P->choice, forced);
      e = upload_steps(*P, st);
    }
    if (e == hipSuccess && P->use_graph) {
      // capture on a stream of the plan's own (the caller's may be the null
      // stream, which cannot be captured)
      e = hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        hipError_t er = run_steps(*P, P->cap_stream);
        e = hipStreamEndCapture(P->cap_stream, &P->graph);
        if (er != hipSuccess) e = er;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
    }
  }
  if (e == hipSuccess) e = P->exec ? hipGraphLaunch(P->exec, st) : run_steps(*P, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(P->h_res, P->d_res, sizeof(uint64_t) * 2 * P->nf, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    err = std::string("batch: ") + hipGetErrorString(e);
    delete P;
    *plan_slot = nullptr;
    return SZ_ERR_DEVICE;
  }
  for (uint32_t i = 0; i < P->nf; i++) {
    BatchItem& it = items[i];
    const uint64_t bytes = P->h_res[2 * i];
    const uint32_t status = (uint32_t)P->h_res[2 * i + 1];
    it.out_size = (size_t)bytes;
    if (status & kStatusEbNotFinite)
      it.status = SZ_ERR_ARG;
    else if (status & kStatusCodeTooLong)
      it.status = SZ_ERR_UNSUPPORTED;
    else if (bytes > it.cap)
      it.status = SZ_ERR_CAPACITY;
    else
      it.status = SZ_OK;
  }
  return SZ_OK;
}

}  // namespace szg
