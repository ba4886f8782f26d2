/*
 * szo.c -- the CPU oracle (see szo.h for what it is and what it follows).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain single-threaded C, no SIMD intrinsics,
 * compiled with -O2 -ffp-contract=off -fno-fast-math.  Nothing here is
 * shared with the GPU library.
 */
#include "szo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define SZO_MAXD 4
#define SZO_NONE UINT64_MAX
#define SZO_MAX_POINTS 0xFFFFFFFFull /* the format's point limit */

/* ------------------------------------------------------------------ */
/* Grid and the multilevel traversal                                   */
/* ------------------------------------------------------------------ */

struct szo_grid {
  int ndim;
  uint64_t dims[SZO_MAXD];
  uint64_t strides[SZO_MAXD]; /* row-major: the last dimension is contiguous */
  uint8_t order[SZO_MAXD];    /* the order in which dimensions are visited */
  int pos[SZO_MAXD];          /* pos[d] = index of d in order */
  uint64_t n;
  int levels; /* L = max over d of ceil(log2 dims[d]) */
};

/* One pass = one (level, dimension) pair.  The multilevel interpolation of
 * SZ3-Interp (Section 6.2) goes from the coarsest level to the finest and,
 * inside a level, dimension by dimension.  Reading of the level structure
 * (the defining reference is not part of the paper): level l has stride
 * s = 2^(l-1), l = L..1.  The pass of dimension d = order[j] at stride s
 * visits the points whose coordinate along d is an odd multiple of s, whose
 * coordinates along the dimensions visited earlier in this level are
 * multiples of s, and whose coordinates along the dimensions visited later
 * are multiples of 2s.  With the origin handled first, every point is
 * visited exactly once, and every stencil point (+-s, +-3s along d) lies on
 * a coarser level or in an earlier pass of the same level. */
struct szo_pass {
  int level;
  int j;
  int d;
  uint64_t s;
  uint64_t start[SZO_MAXD];
  uint64_t step[SZO_MAXD];
};

static int grid_init(struct szo_grid* g, int ndim, const uint64_t* dims,
                     const uint8_t* order) {
  if (ndim < 1 || ndim > SZO_MAXD || !dims) return SZO_ERR_ARG;
  memset(g, 0, sizeof(*g));
  g->ndim = ndim;
  uint64_t n = 1;
  int any_zero = 0;
  for (int d = 0; d < ndim; d++) {
    g->dims[d] = dims[d];
    if (dims[d] == 0) any_zero = 1;
  }
  if (any_zero) {
    n = 0;
  } else {
    for (int d = 0; d < ndim; d++) {
      if (dims[d] > SZO_MAX_POINTS || n > SZO_MAX_POINTS / dims[d])
        return SZO_ERR_ARG;
      n *= dims[d];
    }
  }
  g->n = n;
  uint64_t st = 1;
  for (int d = ndim - 1; d >= 0; d--) {
    g->strides[d] = st;
    st *= (dims[d] ? dims[d] : 1);
  }
  int seen[SZO_MAXD] = {0, 0, 0, 0};
  for (int j = 0; j < ndim; j++) {
    int d = order ? order[j] : j;
    if (d < 0 || d >= ndim || seen[d]) return SZO_ERR_ARG;
    seen[d] = 1;
    g->order[j] = (uint8_t)d;
    g->pos[d] = j;
  }
  for (int j = ndim; j < SZO_MAXD; j++) g->order[j] = (uint8_t)j;
  int L = 0;
  for (int d = 0; d < ndim; d++) {
    int l = 0;
    while (l < 63 && (1ull << l) < dims[d]) l++;
    if (l > L) L = l;
  }
  g->levels = (n == 0) ? 0 : L;
  return SZO_OK;
}

static void pass_setup(const struct szo_grid* g, struct szo_pass* p) {
  p->s = 1ull << (p->level - 1);
  p->d = g->order[p->j];
  for (int e = 0; e < g->ndim; e++) {
    if (e == p->d) {
      p->start[e] = p->s;
      p->step[e] = 2 * p->s;
    } else if (g->pos[e] < p->j) {
      p->start[e] = 0;
      p->step[e] = p->s;
    } else {
      p->start[e] = 0;
      p->step[e] = 2 * p->s;
    }
  }
}

static int pass_first(const struct szo_grid* g, struct szo_pass* p) {
  if (g->levels == 0) return 0;
  p->level = g->levels;
  p->j = 0;
  pass_setup(g, p);
  return 1;
}

static int pass_next(const struct szo_grid* g, struct szo_pass* p) {
  p->j++;
  if (p->j == g->ndim) {
    p->j = 0;
    p->level--;
    if (p->level == 0) return 0;
  }
  pass_setup(g, p);
  return 1;
}

static uint64_t flat_of(const struct szo_grid* g, const uint64_t* q) {
  uint64_t f = 0;
  for (int e = 0; e < g->ndim; e++) f += q[e] * g->strides[e];
  return f;
}

static uint64_t pass_point_first(const struct szo_grid* g,
                                 const struct szo_pass* p, uint64_t* q) {
  for (int e = 0; e < g->ndim; e++) {
    q[e] = p->start[e];
    if (q[e] >= g->dims[e]) return SZO_NONE;
  }
  return flat_of(g, q);
}

/* row-major odometer over the pass's sub-lattice */
static uint64_t pass_point_next(const struct szo_grid* g,
                                const struct szo_pass* p, uint64_t* q) {
  for (int e = g->ndim - 1; e >= 0; e--) {
    q[e] += p->step[e];
    if (q[e] < g->dims[e]) return flat_of(g, q);
    q[e] = p->start[e];
  }
  return SZO_NONE;
}

/* ------------------------------------------------------------------ */
/* Typed arithmetic                                                    */
/* ------------------------------------------------------------------ */

/* The rows (along the last dimension) that price adaptive interpolation's
 * dimension orders: row index r is taken when the top three bits of
 * (r mod 2^32) * 0x9E3779B1 (Fibonacci hashing) are zero, about one row in
 * eight, spread evenly over the rows. */
static int row_sampled(uint64_t r) { return (((uint32_t)r * 0x9E3779B1u) >> 29) == 0; }

#define T float
#define FN(name) name##_f32
#define FABS fabsf
#define RINT rintf
#include "szo_typed.inc"
#undef T
#undef FN
#undef FABS
#undef RINT

#define T double
#define FN(name) name##_f64
#define FABS fabs
#define RINT rint
#include "szo_typed.inc"
#undef T
#undef FN
#undef FABS
#undef RINT

static size_t type_size(int dtype) { return dtype == SZO_F64 ? 8 : 4; }

int szo_resolve_eb(const void* x, uint64_t n, int dtype, int eb_mode,
                   double value, double* eb_t) {
  if (dtype != SZO_F32 && dtype != SZO_F64) return SZO_ERR_ARG;
  if (eb_mode != SZO_ABS && eb_mode != SZO_REL) return SZO_ERR_ARG;
  if (dtype == SZO_F32) return resolve_eb_f32((const float*)x, n, eb_mode, value, eb_t);
  return resolve_eb_f64((const double*)x, n, eb_mode, value, eb_t);
}

static int check_common(int dtype, int predictor, uint32_t radius) {
  if (dtype != SZO_F32 && dtype != SZO_F64) return SZO_ERR_ARG;
  if (predictor != SZO_LINEAR && predictor != SZO_CUBIC && predictor != SZO_ADAPTIVE &&
      predictor != SZO_LORENZO)
    return SZO_ERR_ARG;
  if (radius < 1 || radius > SZO_MAX_RADIUS) return SZO_ERR_ARG;
  return SZO_OK;
}

/* The predictor of every level: the fixed one, or (SZO_ADAPTIVE) the one
 * choose_levels picks from the original values. */
static void level_predictors(const void* x, int dtype, const struct szo_grid* g, int predictor,
                             double eb_t, uint32_t radius, uint8_t* level_pred) {
  memset(level_pred, predictor == SZO_ADAPTIVE ? SZO_CUBIC : predictor, 64);
  if (predictor != SZO_ADAPTIVE) return;
  if (dtype == SZO_F32)
    choose_levels_f32((const float*)x, g, (float)eb_t, radius, level_pred);
  else
    choose_levels_f64((const double*)x, g, eb_t, radius, level_pred);
}

/* The Lorenzo predictor runs in flat order: the dimension order must be
 * the identity. */
static int identity_order(const struct szo_grid* g) {
  for (int j = 0; j < g->ndim; j++)
    if (g->order[j] != j) return 0;
  return 1;
}

static void lorenzo_quantize(const void* x, int dtype, const struct szo_grid* g, double eb_t,
                             uint32_t radius, uint16_t* codes, void* recon) {
  if (dtype == SZO_F32)
    lorenzo_quantize_f32((const float*)x, g, (float)eb_t, radius, codes, (float*)recon);
  else
    lorenzo_quantize_f64((const double*)x, g, eb_t, radius, codes, (double*)recon);
}

static int lorenzo_reconstruct(const uint16_t* codes, const void* unpred, uint64_t n_unpred,
                               int dtype, const struct szo_grid* g, double eb_t,
                               uint32_t radius, void* out) {
  if (dtype == SZO_F32)
    return lorenzo_reconstruct_f32(codes, (const float*)unpred, n_unpred, g, (float)eb_t, radius,
                                   (float*)out);
  return lorenzo_reconstruct_f64(codes, (const double*)unpred, n_unpred, g, eb_t, radius,
                                 (double*)out);
}

/* bit l - 1 set: level l is cubic */
static uint32_t level_mask(const uint8_t* level_pred, int levels) {
  uint32_t mask = 0;
  for (int l = 1; l <= levels; l++)
    if (level_pred[l] == SZO_CUBIC) mask |= 1u << (l - 1);
  return mask;
}

int szo_predict_quantize(const void* x, int dtype, int ndim,
                         const uint64_t* dims, const uint8_t* order,
                         int predictor, double eb_t, uint32_t radius,
                         uint16_t* codes, void* recon) {
  struct szo_grid g;
  int rc = check_common(dtype, predictor, radius);
  if (rc) return rc;
  if ((rc = grid_init(&g, ndim, dims, order))) return rc;
  if (!(eb_t >= 0.0) || !isfinite(eb_t)) return SZO_ERR_ARG;
  if (predictor == SZO_LORENZO) {
    if (!identity_order(&g)) return SZO_ERR_ARG;
    lorenzo_quantize(x, dtype, &g, eb_t, radius, codes, recon);
    return SZO_OK;
  }
  uint8_t lp[64];
  level_predictors(x, dtype, &g, predictor, eb_t, radius, lp);
  if (dtype == SZO_F32)
    return predict_quantize_f32((const float*)x, &g, lp, (float)eb_t, radius, codes,
                                (float*)recon);
  return predict_quantize_f64((const double*)x, &g, lp, eb_t, radius, codes, (double*)recon);
}

static int reconstruct_levels(const uint16_t* codes, const void* unpred, uint64_t n_unpred,
                              int dtype, const struct szo_grid* g, const uint8_t* lp,
                              double eb_t, uint32_t radius, void* out) {
  if (dtype == SZO_F32)
    return reconstruct_f32(codes, (const float*)unpred, n_unpred, g, lp, (float)eb_t, radius,
                           (float*)out);
  return reconstruct_f64(codes, (const double*)unpred, n_unpred, g, lp, eb_t, radius,
                         (double*)out);
}

int szo_reconstruct(const uint16_t* codes, const void* unpred,
                    uint64_t n_unpred, int dtype, int ndim,
                    const uint64_t* dims, const uint8_t* order, int predictor,
                    double eb_t, uint32_t radius, void* out) {
  struct szo_grid g;
  int rc = check_common(dtype, predictor, radius);
  if (rc) return rc;
  if (predictor == SZO_ADAPTIVE) return SZO_ERR_ARG; /* (needs the stream's level mask) */
  if ((rc = grid_init(&g, ndim, dims, order))) return rc;
  if (predictor == SZO_LORENZO) {
    if (!identity_order(&g)) return SZO_ERR_ARG;
    return lorenzo_reconstruct(codes, unpred, n_unpred, dtype, &g, eb_t, radius, out);
  }
  uint8_t lp[64];
  memset(lp, predictor, 64);
  return reconstruct_levels(codes, unpred, n_unpred, dtype, &g, lp, eb_t, radius, out);
}

int szo_quantize_one(int dtype, const void* x, const void* pred, double eb_t,
                     uint32_t radius, uint16_t* code, void* recon) {
  if (radius < 1 || radius > SZO_MAX_RADIUS) return SZO_ERR_ARG;
  if (dtype == SZO_F32) {
    float eb = (float)eb_t, twoeb = 2.0f * eb, inv = 1.0f / twoeb;
    *code = quantize_f32(*(const float*)x, *(const float*)pred, eb, twoeb, inv,
                         radius, (float*)recon);
    return SZO_OK;
  }
  if (dtype == SZO_F64) {
    double eb = eb_t, twoeb = 2.0 * eb, inv = 1.0 / twoeb;
    *code = quantize_f64(*(const double*)x, *(const double*)pred, eb, twoeb,
                         inv, radius, (double*)recon);
    return SZO_OK;
  }
  return SZO_ERR_ARG;
}

/* Which stencil points the predictor reads: the same case analysis as
 * predict_*() in szo_typed.inc, without data. */
static int stencil_offsets(uint64_t i, uint64_t s, uint64_t nd, int predictor,
                           int64_t* off) {
  int k = 0;
  int has_a = i >= 3 * s, has_c = i + s < nd, has_e = i + 3 * s < nd;
  off[k++] = -1;
  if (!has_c) {
    if (has_a) off[k++] = -3;
    return k;
  }
  off[k++] = 1;
  if (predictor == SZO_LINEAR) return k;
  if (has_a && has_e) {
    off[k++] = -3;
    off[k++] = 3;
  } else if (has_e) {
    off[k++] = 3;
  } else if (has_a) {
    off[k++] = -3;
  }
  return k;
}

int szo_check_traversal(int ndim, const uint64_t* dims, const uint8_t* order,
                        int predictor, uint32_t* visits,
                        uint64_t* early_reads) {
  struct szo_grid g;
  int rc = grid_init(&g, ndim, dims, order);
  if (rc) return rc;
  *early_reads = 0;
  if (g.n == 0) return SZO_OK;
  /* pass index at which each point became final; UINT32_MAX = not yet */
  uint32_t* fin = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)g.n);
  if (!fin) return SZO_ERR_NOMEM;
  for (uint64_t f = 0; f < g.n; f++) {
    fin[f] = UINT32_MAX;
    visits[f] = 0;
  }
  visits[0]++;
  fin[0] = 0;
  uint32_t pass_id = 1;
  struct szo_pass p;
  for (int more = pass_first(&g, &p); more; more = pass_next(&g, &p), pass_id++) {
    uint64_t q[SZO_MAXD];
    for (uint64_t f = pass_point_first(&g, &p, q); f != SZO_NONE;
         f = pass_point_next(&g, &p, q)) {
      int64_t off[4];
      int k = stencil_offsets(q[p.d], p.s, g.dims[p.d], predictor, off);
      for (int t = 0; t < k; t++) {
        int64_t c = (int64_t)q[p.d] + off[t] * (int64_t)p.s;
        if (c < 0 || (uint64_t)c >= g.dims[p.d]) {
          (*early_reads)++; /* out of range would be a bug too */
          continue;
        }
        uint64_t nf = f + (uint64_t)(off[t] * (int64_t)p.s * (int64_t)g.strides[p.d]);
        if (fin[nf] >= pass_id) (*early_reads)++;
      }
      visits[f]++;
      if (fin[f] == UINT32_MAX) fin[f] = pass_id;
    }
  }
  free(fin);
  return SZO_OK;
}

/* ------------------------------------------------------------------ */
/* Huffman stage (Section 3.2 "Encoder")                               */
/* ------------------------------------------------------------------ */

int szo_histogram(const uint16_t* codes, uint64_t n, uint32_t nsym,
                  uint64_t* hist) {
  memset(hist, 0, sizeof(uint64_t) * nsym);
  for (uint64_t i = 0; i < n; i++) {
    if (codes[i] >= nsym) return SZO_ERR_ARG;
    hist[codes[i]]++;
  }
  return SZO_OK;
}

struct leaf {
  uint64_t w;
  uint32_t sym;
};

static int leaf_cmp(const void* a, const void* b) {
  const struct leaf* x = (const struct leaf*)a;
  const struct leaf* y = (const struct leaf*)b;
  if (x->w != y->w) return x->w < y->w ? -1 : 1;
  return x->sym < y->sym ? -1 : (x->sym > y->sym ? 1 : 0);
}

/* Greedy Huffman construction from the frequencies (Section 3.2
 * "Encoder"), as the two-queue merge: leaves sorted by (frequency, symbol),
 * internal nodes in a FIFO (their weights come out non-decreasing).  Each
 * merge takes the lighter front twice, the leaf when the two fronts weigh
 * the same.  A symbol's code length is its leaf's depth; a lone symbol gets
 * length 1.  (Tie-breaking is a reading: the paper does not fix it.) */
int szo_huffman_lengths(const uint64_t* hist, uint32_t nsym, uint8_t* lens) {
  memset(lens, 0, nsym);
  uint32_t K = 0;
  for (uint32_t s = 0; s < nsym; s++)
    if (hist[s]) K++;
  if (K == 0) return 0;
  struct leaf* lv = (struct leaf*)malloc(sizeof(struct leaf) * K);
  if (!lv) return SZO_ERR_NOMEM;
  K = 0;
  for (uint32_t s = 0; s < nsym; s++)
    if (hist[s]) {
      lv[K].w = hist[s];
      lv[K].sym = s;
      K++;
    }
  if (K == 1) {
    lens[lv[0].sym] = 1;
    free(lv);
    return 1;
  }
  qsort(lv, K, sizeof(struct leaf), leaf_cmp);
  uint32_t nodes = 2 * K - 1;
  uint64_t* w = (uint64_t*)malloc(sizeof(uint64_t) * nodes);
  uint32_t* parent = (uint32_t*)malloc(sizeof(uint32_t) * nodes);
  uint32_t* depth = (uint32_t*)malloc(sizeof(uint32_t) * nodes);
  if (!w || !parent || !depth) {
    free(lv);
    free(w);
    free(parent);
    free(depth);
    return SZO_ERR_NOMEM;
  }
  for (uint32_t i = 0; i < K; i++) w[i] = lv[i].w;
  uint32_t li = 0, qi = K, qn = K;
  while (qn < nodes) {
    uint32_t pick[2];
    for (int t = 0; t < 2; t++) {
      if (li < K && (qi >= qn || w[li] <= w[qi]))
        pick[t] = li++;
      else
        pick[t] = qi++;
    }
    w[qn] = w[pick[0]] + w[pick[1]];
    parent[pick[0]] = qn;
    parent[pick[1]] = qn;
    qn++;
  }
  depth[nodes - 1] = 0;
  for (uint32_t i = nodes - 1; i-- > 0;) depth[i] = depth[parent[i]] + 1;
  int maxlen = 0;
  int rc = 0;
  for (uint32_t i = 0; i < K; i++) {
    if (depth[i] > SZO_MAX_CODE_LEN) rc = SZO_ERR_ARG;
    lens[lv[i].sym] = (uint8_t)depth[i];
    if ((int)depth[i] > maxlen) maxlen = (int)depth[i];
  }
  free(lv);
  free(w);
  free(parent);
  free(depth);
  return rc ? rc : maxlen;
}

/* Canonical codes, RFC 1951 section 3.2.2: codes of one length are
 * consecutive in symbol order, and the first code of each length follows the
 * last code of the previous length, shifted. */
int szo_canonical_codes(const uint8_t* lens, uint32_t nsym,
                        uint64_t* codewords) {
  uint64_t bl_count[SZO_MAX_CODE_LEN + 1];
  uint64_t next_code[SZO_MAX_CODE_LEN + 1];
  memset(bl_count, 0, sizeof(bl_count));
  for (uint32_t s = 0; s < nsym; s++) {
    if (lens[s] > SZO_MAX_CODE_LEN) return SZO_ERR_ARG;
    if (lens[s]) bl_count[lens[s]]++;
  }
  uint64_t code = 0;
  next_code[0] = 0;
  for (int bits = 1; bits <= SZO_MAX_CODE_LEN; bits++) {
    code = (code + bl_count[bits - 1]) << 1;
    next_code[bits] = code;
  }
  for (uint32_t s = 0; s < nsym; s++) {
    codewords[s] = 0;
    if (lens[s]) codewords[s] = next_code[lens[s]]++;
  }
  return SZO_OK;
}

/* Chunked bit packing (reading: the paper's encoder emits one bitstream; the
 * stream is cut into chunks of `chunk` symbols in flat order so that chunks
 * can be decoded independently).  Inside a chunk each codeword is appended
 * most significant bit first; stream bit b of the chunk is bit 31 - (b % 32)
 * of the chunk's word b / 32; the chunk ends on a word boundary. */
/* Sub-chunks (reading: a chunk may be split into `sub` equal runs of
 * symbols whose starting bit offsets are stored, so that several decoders
 * can share a chunk; the bits themselves are unchanged). */
int szo_check_sub(uint32_t chunk, uint32_t sub) {
  if (sub == 1) return SZO_OK;
  if (sub != 2 && sub != 4 && sub != 8) return SZO_ERR_ARG;
  if (chunk == 0 || chunk % sub != 0) return SZO_ERR_ARG;
  uint32_t run = chunk / 64 > 32 ? chunk / 64 : 32;
  return (chunk / sub) % run == 0 ? SZO_OK : SZO_ERR_ARG;
}

int szo_pack(const uint16_t* codes, uint64_t n, const uint8_t* lens,
             const uint64_t* codewords, uint32_t chunk, uint32_t sub,
             uint32_t* words, uint32_t* chunk_words, uint32_t* sub_bits,
             uint64_t* total_words) {
  if (chunk == 0 || szo_check_sub(chunk, sub)) return SZO_ERR_ARG;
  uint64_t nchunks = (n + chunk - 1) / chunk;
  uint64_t base = 0;
  uint32_t span = chunk / sub;
  for (uint64_t c = 0; c < nchunks; c++) {
    uint64_t lo = c * chunk, hi = lo + chunk < n ? lo + chunk : n;
    uint64_t bit = 0;
    for (uint64_t i = lo; i < hi; i++) {
      uint64_t k = (i - lo) / span;
      if (sub_bits && k > 0 && (i - lo) % span == 0) {
        if (bit > UINT32_MAX) return SZO_ERR_ARG;
        sub_bits[c * (sub - 1) + k - 1] = (uint32_t)bit;
      }
      int len = lens[codes[i]];
      if (len == 0) return SZO_ERR_ARG;
      for (int b = len - 1; b >= 0; b--) {
        if (words && ((codewords[codes[i]] >> b) & 1u))
          words[base + (bit >> 5)] |= 0x80000000u >> (bit & 31);
        bit++;
      }
    }
    /* sub-chunks that start past the chunk's last symbol start at its end */
    if (sub_bits)
      for (uint32_t k = 1; k < sub; k++)
        if (lo + (uint64_t)k * span >= hi) sub_bits[c * (sub - 1) + k - 1] = (uint32_t)bit;
    uint64_t cw = (bit + 31) / 32;
    if (cw > UINT32_MAX) return SZO_ERR_ARG;
    chunk_words[c] = (uint32_t)cw;
    base += cw;
  }
  *total_words = base;
  return SZO_OK;
}

/* Canonical decoding, one bit at a time: a code of length len is valid when
 * it lies in [first[len], first[len] + count[len]). */
struct decoder {
  uint64_t count[SZO_MAX_CODE_LEN + 1];
  uint64_t first[SZO_MAX_CODE_LEN + 1];
  uint64_t offset[SZO_MAX_CODE_LEN + 1];
  uint16_t* sorted; /* symbols sorted by (length, symbol) */
};

static int decoder_init(struct decoder* dc, const uint8_t* lens,
                        uint32_t nsym) {
  memset(dc, 0, sizeof(*dc));
  uint64_t K = 0;
  for (uint32_t s = 0; s < nsym; s++) {
    if (lens[s] > SZO_MAX_CODE_LEN) return SZO_ERR_CORRUPT;
    if (lens[s]) {
      dc->count[lens[s]]++;
      K++;
    }
  }
  dc->sorted = (uint16_t*)malloc(sizeof(uint16_t) * (K ? K : 1));
  if (!dc->sorted) return SZO_ERR_NOMEM;
  uint64_t code = 0, off = 0;
  for (int len = 1; len <= SZO_MAX_CODE_LEN; len++) {
    code = (code + dc->count[len - 1]) << 1;
    dc->first[len] = code;
    dc->offset[len] = off;
    off += dc->count[len];
  }
  uint64_t fill[SZO_MAX_CODE_LEN + 1];
  memcpy(fill, dc->offset, sizeof(fill));
  for (uint32_t s = 0; s < nsym; s++)
    if (lens[s]) dc->sorted[fill[lens[s]]++] = (uint16_t)s;
  return SZO_OK;
}

int szo_unpack(const uint32_t* words, uint64_t total_words,
               const uint32_t* chunk_words, uint64_t n, uint32_t chunk,
               uint32_t sub, const uint32_t* sub_bits, const uint8_t* lens,
               uint32_t nsym, uint16_t* codes) {
  if (chunk == 0 || szo_check_sub(chunk, sub) || (sub > 1 && !sub_bits)) return SZO_ERR_ARG;
  uint32_t span = chunk / sub;
  struct decoder dc;
  int rc = decoder_init(&dc, lens, nsym);
  if (rc) return rc;
  uint64_t nchunks = (n + chunk - 1) / chunk;
  uint64_t base = 0;
  for (uint64_t c = 0; c < nchunks && !rc; c++) {
    uint64_t lo = c * chunk, hi = lo + chunk < n ? lo + chunk : n;
    uint64_t nbits = (uint64_t)chunk_words[c] * 32;
    if (base + chunk_words[c] > total_words) {
      rc = SZO_ERR_CORRUPT;
      break;
    }
    uint64_t bit = 0;
    for (uint64_t i = lo; i < hi && !rc; i++) {
      uint64_t k = (i - lo) / span;
      if (k > 0 && (i - lo) % span == 0 && sub_bits[c * (sub - 1) + k - 1] != bit) {
        rc = SZO_ERR_CORRUPT;
        break;
      }
      uint64_t code = 0;
      int len = 0;
      for (;;) {
        if (bit >= nbits || len == SZO_MAX_CODE_LEN) {
          rc = SZO_ERR_CORRUPT;
          break;
        }
        uint32_t wv = words[base + (bit >> 5)];
        code = (code << 1) | ((wv >> (31 - (bit & 31))) & 1u);
        bit++;
        len++;
        if (dc.count[len] && code >= dc.first[len] &&
            code - dc.first[len] < dc.count[len]) {
          codes[i] = dc.sorted[dc.offset[len] + (code - dc.first[len])];
          break;
        }
      }
    }
    if (!rc && (bit + 31) / 32 != chunk_words[c]) rc = SZO_ERR_CORRUPT;
    for (uint32_t k = 1; k < sub && !rc; k++)
      if (lo + (uint64_t)k * span >= hi && sub_bits[c * (sub - 1) + k - 1] != bit)
        rc = SZO_ERR_CORRUPT;
    base += chunk_words[c];
  }
  if (!rc && base != total_words) rc = SZO_ERR_CORRUPT;
  free(dc.sorted);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Stream format (little-endian; sections start on 8-byte boundaries)  */
/* ------------------------------------------------------------------ */
/*
 * header, 128 bytes:
 *   0  "SZG1"            4 u16 version (1)     6 u8 dtype   7 u8 ndim
 *   8  u64 dims[4] (unused = 1)
 *   40 u8 predictor      41 u8 order[4]        45 u8 eb_mode  46 u16 0
 *   48 f64 eb as given   56 f64 eb in the field type, widened
 *   64 u32 radius        68 u32 chunk          72 u64 unpredictable count
 *   80 u32 used symbols K                      84 u32 sub-chunks per chunk
 *   88 u64 bitstream words                     96 u64 stream bytes
 *   104..127 zero
 * symbol table: K x u32 (symbol | length << 16), ascending symbol
 * chunk table:  ceil(n/chunk) x (u32 words, u32 unpredictable count)
 * sub-chunk table: ceil(n/chunk) x (sub - 1) x u32 bit offsets of sub-chunks
 *               1..sub-1 from the chunk's first bit
 * unpredictable values: count x T, flat order (the quantizer's saved state,
 *                       Algorithm 1 "quantizer.save")
 * bitstream:    words x u32 (Algorithm 1 "encoder.encode")
 */

static void put_u16(uint8_t* p, uint16_t v) {
  p[0] = (uint8_t)v;
  p[1] = (uint8_t)(v >> 8);
}
static void put_u32(uint8_t* p, uint32_t v) {
  for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i));
}
static void put_u64(uint8_t* p, uint64_t v) {
  for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i));
}
static void put_f64(uint8_t* p, double v) {
  uint64_t u;
  memcpy(&u, &v, 8);
  put_u64(p, u);
}
static uint16_t get_u16(const uint8_t* p) {
  return (uint16_t)(p[0] | (p[1] << 8));
}
static uint32_t get_u32(const uint8_t* p) {
  uint32_t v = 0;
  for (int i = 3; i >= 0; i--) v = (v << 8) | p[i];
  return v;
}
static uint64_t get_u64(const uint8_t* p) {
  uint64_t v = 0;
  for (int i = 7; i >= 0; i--) v = (v << 8) | p[i];
  return v;
}
static double get_f64(const uint8_t* p) {
  uint64_t u = get_u64(p);
  double v;
  memcpy(&v, &u, 8);
  return v;
}
static uint64_t pad8(uint64_t v) { return (v + 7) & ~7ull; }

struct layout {
  uint64_t off_sym, off_chunk, off_sub, off_unpred, off_bits, size;
};

static void layout_of(uint64_t K, uint64_t nchunks, uint32_t sub, uint64_t n_unpred,
                      size_t ts, uint64_t words, struct layout* lo) {
  lo->off_sym = SZO_HEADER_BYTES;
  lo->off_chunk = lo->off_sym + pad8(4 * K);
  lo->off_sub = lo->off_chunk + 8 * nchunks;
  lo->off_unpred = lo->off_sub + pad8(4 * (uint64_t)(sub - 1) * nchunks);
  lo->off_bits = lo->off_unpred + pad8(n_unpred * ts);
  lo->size = lo->off_bits + 4 * words;
}

/* ------------------------------------------ point-wise relative mode ----
 * The logarithmic preprocessor (paper Section 3.1 / 3.2 "Preprocessor"):
 * x -> y = log2|x| as a double field, compressed with the absolute bound
 * szo_pwrel_delta(eps); the signs are kept as a bit per value when any is
 * set.  Zeros and subnormal values of T map to a level far below every
 * normal value's logarithm and come back as signed zeros; infinities map to
 * +inf, NaN to NaN (both unpredictable in the log field, stored verbatim).
 * The series below are evaluated in the order written (no contraction). */
#define SZO_SQRT_HALF 0.70710678118654752440
#define SZO_INV_LN2 1.4426950408889634074
#define SZO_LN2 0.69314718055994530942
#define SZO_LOG_ZERO (-1100.0)      /* log-domain level of zeros and subnormals */
#define SZO_LOG_ZERO_BELOW (-1050.0) /* reconstructed levels below this are zeros */

double szo_log2(double a) {
  int e;
  double m = frexp(a, &e); /* a = m 2^e, m in [1/2, 1) */
  if (m < SZO_SQRT_HALF) {
    m = m * 2.0;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  /* atanh(s) / s = 1 + s^2/3 + s^4/5 + ... + s^28/29 */
  double t = 1.0 / 29.0;
  t = t * s2 + 1.0 / 27.0;
  t = t * s2 + 1.0 / 25.0;
  t = t * s2 + 1.0 / 23.0;
  t = t * s2 + 1.0 / 21.0;
  t = t * s2 + 1.0 / 19.0;
  t = t * s2 + 1.0 / 17.0;
  t = t * s2 + 1.0 / 15.0;
  t = t * s2 + 1.0 / 13.0;
  t = t * s2 + 1.0 / 11.0;
  t = t * s2 + 1.0 / 9.0;
  t = t * s2 + 1.0 / 7.0;
  t = t * s2 + 1.0 / 5.0;
  t = t * s2 + 1.0 / 3.0;
  t = t * s2 + 1.0;
  const double ln_m = 2.0 * s * t;
  return (double)e + ln_m * SZO_INV_LN2;
}

double szo_exp2(double y) {
  const double k = rint(y);
  const double t = (y - k) * SZO_LN2; /* |t| <= ln(2)/2 */
  /* exp(t) = 1 + t + t^2/2! + ... + t^18/18! */
  double p = 1.0 / 6402373705728000.0;
  p = p * t + 1.0 / 355687428096000.0;
  p = p * t + 1.0 / 20922789888000.0;
  p = p * t + 1.0 / 1307674368000.0;
  p = p * t + 1.0 / 87178291200.0;
  p = p * t + 1.0 / 6227020800.0;
  p = p * t + 1.0 / 479001600.0;
  p = p * t + 1.0 / 39916800.0;
  p = p * t + 1.0 / 3628800.0;
  p = p * t + 1.0 / 362880.0;
  p = p * t + 1.0 / 40320.0;
  p = p * t + 1.0 / 5040.0;
  p = p * t + 1.0 / 720.0;
  p = p * t + 1.0 / 120.0;
  p = p * t + 1.0 / 24.0;
  p = p * t + 1.0 / 6.0;
  p = p * t + 0.5;
  p = p * t + 1.0;
  p = p * t + 1.0;
  return ldexp(p, (int)k);
}

/* The log field's absolute bound.  Relative margins: 4u for the exponential
 * series and the final rounding to T (u the unit roundoff of T), and the
 * factor (1 - 2^-20) for the series of the logarithm of the ratio.  Absolute
 * margins: y = log2|x| is rounded to within half an ulp of |y| (plus far
 * less for the series), and |y| < 2048 for every normal double (< 256 for
 * every normal float), so the computed y is within 2^-42 (2^-45) of the true
 * logarithm; the ratio (1 + eps)/(1 + 4u) takes two roundings in double,
 * which move its logarithm by less than 2^-50.  Both are subtracted.  A
 * bound too small to leave delta > 0 is rejected (for doubles, eps below
 * about 1.6e-13). */
double szo_pwrel_delta(double eps, int dtype) {
  if (!(eps > 0.0) || !(eps < 1.0)) return -1.0;
  const double u = dtype == SZO_F64 ? 0x1p-53 : 0x1p-24;
  const double e_abs = (dtype == SZO_F64 ? 0x1p-42 : 0x1p-45) + 0x1p-50;
  const double r = (1.0 + eps) / (1.0 + 4.0 * u);
  if (!(r > 1.0)) return -1.0;
  const double d = szo_log2(r) * (1.0 - 0x1p-20) - e_abs;
  return d > 0.0 ? d : -1.0;
}

/* the log-domain value of one field value (widened to double) */
static double log_of(double v, int dtype) {
  if (isnan(v)) return NAN;
  const double a = fabs(v);
  if (isinf(a)) return INFINITY;
  const double tmin = dtype == SZO_F64 ? 0x1p-1022 : 0x1p-126;
  if (a < tmin) return SZO_LOG_ZERO;
  return szo_log2(a);
}

/* one reconstructed value of T from its log-domain value and sign */
static void exp_of(double y, int neg, int dtype, void* out, uint64_t i) {
  if (dtype == SZO_F64) {
    uint64_t bits;
    if (isnan(y)) {
      bits = 0x7FF8000000000000ull;
    } else {
      double v;
      if (y == INFINITY)
        v = INFINITY;
      else if (y < SZO_LOG_ZERO_BELOW)
        v = 0.0;
      else if (y > 1100.0)
        v = 0x1.fffffffffffffp+1023;
      else {
        v = szo_exp2(y);
        if (v > 0x1.fffffffffffffp+1023) v = 0x1.fffffffffffffp+1023;
      }
      memcpy(&bits, &v, 8);
    }
    if (neg) bits |= 0x8000000000000000ull;
    memcpy((uint8_t*)out + 8 * i, &bits, 8);
  } else {
    uint32_t bits;
    if (isnan(y)) {
      bits = 0x7FC00000u;
    } else {
      double v;
      if (y == INFINITY)
        v = INFINITY;
      else if (y < SZO_LOG_ZERO_BELOW)
        v = 0.0;
      else if (y > 1100.0)
        v = 0x1.fffffep+127;
      else {
        v = szo_exp2(y);
        if (v > 0x1.fffffep+127) v = 0x1.fffffep+127;
      }
      const float f = (float)v;
      memcpy(&bits, &f, 4);
    }
    if (neg) bits |= 0x80000000u;
    memcpy((uint8_t*)out + 4 * i, &bits, 4);
  }
}

static int sign_of(const void* x, int dtype, uint64_t i) {
  if (dtype == SZO_F64) {
    uint64_t b;
    memcpy(&b, (const uint8_t*)x + 8 * i, 8);
    return (int)(b >> 63);
  }
  uint32_t b;
  memcpy(&b, (const uint8_t*)x + 4 * i, 4);
  return (int)(b >> 31);
}

static int compress_pwrel(const void* x, int dtype, int ndim, const uint64_t* dims, double eps,
                          int predictor, uint32_t radius, uint32_t chunk, uint32_t sub,
                          const uint8_t* order, uint8_t** stream, uint64_t* stream_size,
                          uint16_t* codes_out, void* recon_out) {
  if (dtype != SZO_F32 && dtype != SZO_F64) return SZO_ERR_ARG;
  const double delta = szo_pwrel_delta(eps, dtype);
  if (!(delta > 0.0)) return SZO_ERR_ARG;
  struct szo_grid g;
  int rc = grid_init(&g, ndim, dims, order);
  if (rc) return rc;
  const uint64_t n = g.n, nsw = (n + 63) / 64;
  double* y = (double*)malloc(sizeof(double) * (n ? n : 1));
  double* yrec = (double*)malloc(sizeof(double) * (n ? n : 1));
  uint64_t* signs = (uint64_t*)calloc(nsw ? nsw : 1, sizeof(uint64_t));
  uint8_t* ys = NULL;
  uint64_t ysize = 0;
  if (!y || !yrec || !signs) {
    rc = SZO_ERR_NOMEM;
    goto done;
  }
  int any = 0;
  for (uint64_t i = 0; i < n; i++) {
    const double v = dtype == SZO_F64 ? ((const double*)x)[i] : (double)((const float*)x)[i];
    y[i] = log_of(v, dtype);
    if (sign_of(x, dtype, i)) {
      signs[i / 64] |= 1ull << (i % 64);
      any = 1;
    }
  }
  /* the log field through the interpolation pipeline, absolute bound delta */
  rc = szo_compress(y, SZO_F64, ndim, dims, SZO_ABS, delta, predictor, radius, chunk, sub, order,
                    &ys, &ysize, codes_out, yrec);
  if (rc) goto done;
  {
    const uint64_t off_signs = any ? pad8(ysize) : 0;
    const uint64_t total = any ? off_signs + 8 * nsw : ysize;
    uint8_t* out = (uint8_t*)calloc(total ? total : 1, 1);
    if (!out) {
      rc = SZO_ERR_NOMEM;
      goto done;
    }
    memcpy(out, ys, ysize);
    out[45] = SZO_PWREL;
    put_f64(out + 48, eps);
    put_u64(out + 96, total);
    out[104] = (uint8_t)dtype; /* the field's type; the coded (log) field is f64 */
    out[105] = (uint8_t)any;
    put_u64(out + 112, off_signs);
    for (uint64_t w = 0; w < (any ? nsw : 0); w++) put_u64(out + off_signs + 8 * w, signs[w]);
    if (recon_out)
      for (uint64_t i = 0; i < n; i++)
        exp_of(yrec[i], (int)((signs[i / 64] >> (i % 64)) & 1), dtype, recon_out, i);
    *stream = out;
    *stream_size = total;
  }
done:
  free(y);
  free(yrec);
  free(signs);
  free(ys);
  return rc;
}

static int decompress_pwrel(const uint8_t* s, uint64_t size, void* outp, uint64_t out_bytes,
                            uint16_t* codes_out) {
  const int out_dtype = s[104], any = s[105];
  if (s[6] != SZO_F64 || out_dtype > 1 || any > 1) return SZO_ERR_CORRUPT;
  for (int k = 106; k < 112; k++)
    if (s[k]) return SZO_ERR_CORRUPT;
  for (int k = 120; k < 124; k++)
    if (s[k]) return SZO_ERR_CORRUPT;
  const uint64_t total = get_u64(s + 96), off_signs = get_u64(s + 112);
  if (total > size) return SZO_ERR_CORRUPT;
  const int ndim = s[7];
  if (ndim < 1 || ndim > 4) return SZO_ERR_CORRUPT;
  uint64_t n = 1;
  for (int d = 0; d < ndim; d++) {
    const uint64_t e = get_u64(s + 8 + 8 * d);
    if (e && n > UINT64_MAX / e) return SZO_ERR_CORRUPT;
    n *= e;
  }
  const uint64_t nsw = (n + 63) / 64;
  /* the log stream: its own header (absolute mode, its own size) */
  uint64_t ysize;
  if (any) {
    if (off_signs < SZO_HEADER_BYTES || off_signs % 8 || off_signs + 8 * nsw != total)
      return SZO_ERR_CORRUPT;
    ysize = off_signs; /* (the log stream, padded to 8 bytes) */
  } else {
    if (off_signs != 0) return SZO_ERR_CORRUPT;
    ysize = total;
  }
  const size_t ts = out_dtype == SZO_F64 ? 8 : 4;
  if (out_bytes < n * ts) return SZO_ERR_CAPACITY;
  uint8_t* ys = (uint8_t*)malloc(ysize);
  double* y = (double*)malloc(sizeof(double) * (n ? n : 1));
  int rc = SZO_OK;
  if (!ys || !y) {
    rc = SZO_ERR_NOMEM;
    goto done;
  }
  memcpy(ys, s, ysize);
  ys[45] = SZO_ABS;
  memset(ys + 104, 0, 20); /* (bytes 124.. keep the level mask) */
  {
    /* the log stream's size: the layout's, which must land on ysize
       (exactly, or padded to 8 when the sign section follows) */
    const uint64_t ylen = get_u64(ys + 96);
    (void)ylen;
    const uint64_t K = get_u32(ys + 80), n_unpred = get_u64(ys + 72);
    const uint32_t chunk = get_u32(ys + 68), sub = get_u32(ys + 84);
    const uint64_t words = get_u64(ys + 88);
    if (chunk == 0 || szo_check_sub(chunk, sub) || K > 65536 || n_unpred > n) {
      rc = SZO_ERR_CORRUPT;
      goto done;
    }
    struct layout lo;
    layout_of(K, (n + chunk - 1) / chunk, sub, n_unpred, 8, words, &lo);
    if (any ? pad8(lo.size) != ysize : lo.size != ysize) {
      rc = SZO_ERR_CORRUPT;
      goto done;
    }
    put_u64(ys + 96, lo.size);
    rc = szo_decompress(ys, lo.size, y, sizeof(double) * n, codes_out);
    if (rc) goto done;
  }
  for (uint64_t i = 0; i < n; i++) {
    const int neg = any ? (int)((get_u64(s + off_signs + 8 * (i / 64)) >> (i % 64)) & 1) : 0;
    exp_of(y[i], neg, out_dtype, outp, i);
  }
done:
  free(ys);
  free(y);
  return rc;
}

int szo_compress(const void* x, int dtype, int ndim, const uint64_t* dims,
                 int eb_mode, double eb, int predictor, uint32_t radius,
                 uint32_t chunk, uint32_t sub, const uint8_t* order,
                 uint8_t** stream, uint64_t* stream_size, uint16_t* codes_out,
                 void* recon_out) {
  if (eb_mode == SZO_PWREL)
    return compress_pwrel(x, dtype, ndim, dims, eb, predictor, radius, chunk, sub, order, stream,
                          stream_size, codes_out, recon_out);
  struct szo_grid g;
  int rc = check_common(dtype, predictor, radius);
  if (rc) return rc;
  if (chunk == 0 || szo_check_sub(chunk, sub)) return SZO_ERR_ARG;
  if (eb_mode != SZO_ABS && eb_mode != SZO_REL) return SZO_ERR_ARG;
  if ((rc = grid_init(&g, ndim, dims, order))) return rc;
  if (predictor == SZO_LORENZO && !identity_order(&g)) return SZO_ERR_ARG;
  size_t ts = type_size(dtype);
  uint64_t n = g.n;
  double eb_t;
  if ((rc = szo_resolve_eb(x, n, dtype, eb_mode, eb, &eb_t))) return rc;
  /* adaptive interpolation with the default (identity) order: the
     dimension order is chosen first */
  if (predictor == SZO_ADAPTIVE && identity_order(&g) && ndim > 1 && n > 0) {
    uint8_t ord[SZO_MAXD];
    if (dtype == SZO_F32)
      choose_order_f32((const float*)x, ndim, g.dims, (float)eb_t, radius, ord);
    else
      choose_order_f64((const double*)x, ndim, g.dims, eb_t, radius, ord);
    if ((rc = grid_init(&g, ndim, dims, ord))) return rc;
  }

  uint32_t nsym = 2 * radius;
  uint16_t* codes = (uint16_t*)malloc(sizeof(uint16_t) * (n ? n : 1));
  void* recon = malloc(ts * (n ? n : 1));
  uint64_t* hist = (uint64_t*)malloc(sizeof(uint64_t) * nsym);
  uint8_t* lens = (uint8_t*)malloc(nsym);
  uint64_t* cw = (uint64_t*)malloc(sizeof(uint64_t) * nsym);
  uint64_t nchunks = (n + chunk - 1) / chunk;
  uint32_t* chunk_words = (uint32_t*)malloc(sizeof(uint32_t) * (nchunks ? nchunks : 1));
  uint32_t* sub_bits = (uint32_t*)malloc(sizeof(uint32_t) * (nchunks * (sub - 1) + 1));
  uint32_t* words = NULL;
  uint8_t* out = NULL;
  if (!codes || !recon || !hist || !lens || !cw || !chunk_words || !sub_bits) {
    rc = SZO_ERR_NOMEM;
    goto done;
  }
  /* Algorithm 1: predict + quantize every point (adaptive: each level's
     predictor chosen first; Lorenzo: in flat order) */
  uint8_t lp[64];
  if (predictor == SZO_LORENZO) {
    lorenzo_quantize(x, dtype, &g, eb_t, radius, codes, recon);
  } else {
    level_predictors(x, dtype, &g, predictor, eb_t, radius, lp);
    if (dtype == SZO_F32)
      rc = predict_quantize_f32((const float*)x, &g, lp, (float)eb_t, radius, codes,
                                (float*)recon);
    else
      rc = predict_quantize_f64((const double*)x, &g, lp, eb_t, radius, codes, (double*)recon);
    if (rc) goto done;
  }
  /* Huffman: frequencies -> lengths -> canonical codebook */
  if ((rc = szo_histogram(codes, n, nsym, hist))) goto done;
  rc = szo_huffman_lengths(hist, nsym, lens);
  if (rc < 0) goto done;
  if ((rc = szo_canonical_codes(lens, nsym, cw))) goto done;
  uint64_t K = 0;
  for (uint32_t s = 0; s < nsym; s++)
    if (lens[s]) K++;
  uint64_t total_words;
  if ((rc = szo_pack(codes, n, lens, cw, chunk, sub, NULL, chunk_words, NULL, &total_words)))
    goto done;
  words = (uint32_t*)calloc(total_words ? total_words : 1, sizeof(uint32_t));
  if (!words) {
    rc = SZO_ERR_NOMEM;
    goto done;
  }
  if ((rc = szo_pack(codes, n, lens, cw, chunk, sub, words, chunk_words, sub_bits, &total_words)))
    goto done;
  uint64_t n_unpred = hist[0];
  struct layout lo;
  layout_of(K, nchunks, sub, n_unpred, ts, total_words, &lo);
  out = (uint8_t*)calloc(lo.size, 1);
  if (!out) {
    rc = SZO_ERR_NOMEM;
    goto done;
  }
  memcpy(out, "SZG1", 4);
  put_u16(out + 4, 1);
  out[6] = (uint8_t)dtype;
  out[7] = (uint8_t)ndim;
  for (int d = 0; d < 4; d++) put_u64(out + 8 + 8 * d, d < ndim ? g.dims[d] : 1);
  out[40] = (uint8_t)predictor;
  for (int d = 0; d < 4; d++) out[41 + d] = g.order[d];
  out[45] = (uint8_t)eb_mode;
  put_f64(out + 48, eb);
  put_f64(out + 56, eb_t);
  put_u32(out + 64, radius);
  put_u32(out + 68, chunk);
  put_u64(out + 72, n_unpred);
  put_u32(out + 80, (uint32_t)K);
  put_u32(out + 84, sub);
  put_u64(out + 88, total_words);
  put_u64(out + 96, lo.size);
  if (predictor == SZO_ADAPTIVE) put_u32(out + 124, level_mask(lp, g.levels));
  /* encoder.save: the code lengths, ascending symbol */
  uint64_t k = 0;
  for (uint32_t s = 0; s < nsym; s++)
    if (lens[s]) put_u32(out + lo.off_sym + 4 * k++, s | ((uint32_t)lens[s] << 16));
  /* chunk table */
  for (uint64_t c = 0; c < nchunks; c++) {
    uint64_t a = c * chunk, b = a + chunk < n ? a + chunk : n;
    uint32_t cu = 0;
    for (uint64_t i = a; i < b; i++)
      if (codes[i] == 0) cu++;
    put_u32(out + lo.off_chunk + 8 * c, chunk_words[c]);
    put_u32(out + lo.off_chunk + 8 * c + 4, cu);
  }
  for (uint64_t j = 0; j < nchunks * (sub - 1); j++) put_u32(out + lo.off_sub + 4 * j, sub_bits[j]);
  /* quantizer.save: unpredictable values verbatim, flat order */
  uint64_t u = 0;
  for (uint64_t i = 0; i < n; i++)
    if (codes[i] == 0) memcpy(out + lo.off_unpred + ts * u++, (const uint8_t*)x + ts * i, ts);
  for (uint64_t w = 0; w < total_words; w++) put_u32(out + lo.off_bits + 4 * w, words[w]);
  if (codes_out) memcpy(codes_out, codes, sizeof(uint16_t) * n);
  if (recon_out) memcpy(recon_out, recon, ts * n);
  *stream = out;
  *stream_size = lo.size;
  out = NULL;
  rc = SZO_OK;
done:
  free(codes);
  free(recon);
  free(hist);
  free(lens);
  free(cw);
  free(chunk_words);
  free(sub_bits);
  free(words);
  free(out);
  return rc;
}

int szo_decompress(const uint8_t* s, uint64_t size, void* outp,
                   uint64_t out_bytes, uint16_t* codes_out) {
  if (!s || size < SZO_HEADER_BYTES) return SZO_ERR_CORRUPT;
  if (memcmp(s, "SZG1", 4) != 0 || get_u16(s + 4) != 1) return SZO_ERR_CORRUPT;
  if (s[45] == SZO_PWREL) return decompress_pwrel(s, size, outp, out_bytes, codes_out);
  int dtype = s[6], ndim = s[7], predictor = s[40], eb_mode = s[45];
  if (dtype > 1 || ndim < 1 || ndim > 4 || predictor > 3 || eb_mode > 1)
    return SZO_ERR_CORRUPT;
  uint64_t dims[4];
  uint8_t order[4];
  for (int d = 0; d < 4; d++) {
    dims[d] = get_u64(s + 8 + 8 * d);
    order[d] = s[41 + d];
    if (d >= ndim && (dims[d] != 1 || order[d] != d)) return SZO_ERR_CORRUPT;
  }
  struct szo_grid g;
  if (grid_init(&g, ndim, dims, order)) return SZO_ERR_CORRUPT;
  if (predictor == SZO_LORENZO && !identity_order(&g)) return SZO_ERR_CORRUPT;
  double eb_t = get_f64(s + 56);
  uint32_t radius = get_u32(s + 64), chunk = get_u32(s + 68);
  uint64_t n_unpred = get_u64(s + 72);
  uint64_t K = get_u32(s + 80);
  uint32_t sub = get_u32(s + 84);
  uint64_t total_words = get_u64(s + 88), stream_bytes = get_u64(s + 96);
  if (!(eb_t >= 0.0) || !isfinite(eb_t)) return SZO_ERR_CORRUPT;
  if (dtype == SZO_F32 && (double)(float)eb_t != eb_t) return SZO_ERR_CORRUPT;
  if (radius < 1 || radius > SZO_MAX_RADIUS || chunk == 0) return SZO_ERR_CORRUPT;
  if (szo_check_sub(chunk, sub)) return SZO_ERR_CORRUPT;
  uint64_t n = g.n;
  uint32_t nsym = 2 * radius;
  if (K > nsym || n_unpred > n || (K == 0) != (n == 0)) return SZO_ERR_CORRUPT;
  if (total_words > 64 * (n + 1)) return SZO_ERR_CORRUPT;
  size_t ts = type_size(dtype);
  uint64_t nchunks = (n + chunk - 1) / chunk;
  struct layout lo;
  layout_of(K, nchunks, sub, n_unpred, ts, total_words, &lo);
  if (lo.size != stream_bytes || stream_bytes > size) return SZO_ERR_CORRUPT;
  if (out_bytes < n * ts) return SZO_ERR_CAPACITY;

  int rc = SZO_OK;
  uint8_t* lens = (uint8_t*)calloc(nsym, 1);
  uint32_t* chunk_words = (uint32_t*)malloc(sizeof(uint32_t) * (nchunks ? nchunks : 1));
  uint32_t* sub_bits = (uint32_t*)malloc(sizeof(uint32_t) * (nchunks * (sub - 1) + 1));
  uint32_t* words = (uint32_t*)malloc(sizeof(uint32_t) * (total_words ? total_words : 1));
  uint16_t* codes = (uint16_t*)malloc(sizeof(uint16_t) * (n ? n : 1));
  void* unpred = malloc(ts * (n_unpred ? n_unpred : 1));
  if (!lens || !chunk_words || !sub_bits || !words || !codes || !unpred) {
    rc = SZO_ERR_NOMEM;
    goto done;
  }
  /* encoder.load: lengths, validated as a complete prefix code */
  {
    int64_t prev = -1;
    unsigned __int128 kraft = 0;
    for (uint64_t k = 0; k < K; k++) {
      uint32_t e = get_u32(s + lo.off_sym + 4 * k);
      uint32_t sym = e & 0xFFFF, len = e >> 16;
      if ((int64_t)sym <= prev || sym >= nsym || len < 1 || len > SZO_MAX_CODE_LEN) {
        rc = SZO_ERR_CORRUPT;
        goto done;
      }
      prev = sym;
      lens[sym] = (uint8_t)len;
      kraft += (unsigned __int128)1 << (SZO_MAX_CODE_LEN - len);
    }
    unsigned __int128 full = (unsigned __int128)1 << SZO_MAX_CODE_LEN;
    if (K == 1 ? lens[prev] != 1 : (K > 1 && kraft != full)) {
      rc = SZO_ERR_CORRUPT;
      goto done;
    }
  }
  uint64_t sum_w = 0, sum_u = 0;
  for (uint64_t c = 0; c < nchunks; c++) {
    chunk_words[c] = get_u32(s + lo.off_chunk + 8 * c);
    sum_w += chunk_words[c];
    sum_u += get_u32(s + lo.off_chunk + 8 * c + 4);
  }
  if (sum_w != total_words || sum_u != n_unpred) {
    rc = SZO_ERR_CORRUPT;
    goto done;
  }
  for (uint64_t w = 0; w < total_words; w++) words[w] = get_u32(s + lo.off_bits + 4 * w);
  for (uint64_t j = 0; j < nchunks * (sub - 1); j++) sub_bits[j] = get_u32(s + lo.off_sub + 4 * j);
  memcpy(unpred, s + lo.off_unpred, ts * n_unpred);
  if ((rc = szo_unpack(words, total_words, chunk_words, n, chunk, sub, sub_bits, lens, nsym,
                       codes)))
    goto done;
  /* per-chunk unpredictable counts must match the decoded codes */
  for (uint64_t c = 0; c < nchunks; c++) {
    uint64_t a = c * chunk, b = a + chunk < n ? a + chunk : n;
    uint32_t cu = 0;
    for (uint64_t i = a; i < b; i++)
      if (codes[i] == 0) cu++;
    if (cu != get_u32(s + lo.off_chunk + 8 * c + 4)) {
      rc = SZO_ERR_CORRUPT;
      goto done;
    }
  }
  {
    /* each level's predictor: the fixed one, or the stream's level mask
       (adaptive; bits past the last level must be clear) */
    uint8_t lp[64];
    memset(lp, predictor == SZO_ADAPTIVE ? SZO_LINEAR : predictor, 64);
    const uint32_t mask = get_u32(s + 124);
    if (predictor == SZO_ADAPTIVE) {
      if (g.levels < 32 && (mask >> g.levels) != 0) {
        rc = SZO_ERR_CORRUPT;
        goto done;
      }
      for (int l = 1; l <= g.levels; l++) lp[l] = (mask >> (l - 1)) & 1 ? SZO_CUBIC : SZO_LINEAR;
    } else if (mask != 0) {
      rc = SZO_ERR_CORRUPT;
      goto done;
    }
    if (predictor == SZO_LORENZO) {
      rc = lorenzo_reconstruct(codes, unpred, n_unpred, dtype, &g, eb_t, radius, outp);
      goto codes_out;
    }
    rc = reconstruct_levels(codes, unpred, n_unpred, dtype, &g, lp, eb_t, radius, outp);
  }
codes_out:
  if (!rc && codes_out) memcpy(codes_out, codes, sizeof(uint16_t) * n);
done:
  free(lens);
  free(chunk_words);
  free(sub_bits);
  free(words);
  free(codes);
  free(unpred);
  return rc;
}

void szo_free(void* p) { free(p); }
