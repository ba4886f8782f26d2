/*
 * szg.h -- C ABI of the MI355X interpolation compressor.
 *
 * The library implements the data-parallel hot path of the SZ3-Interp
 * pipeline of "SZ3: A Modular Framework for Composing Prediction-Based
 * Error-Bounded Lossy Compressors" (Section 6.2): a multilevel linear/cubic
 * interpolation predictor, the linear-scaling quantizer with a radius
 * (Section 3.2 "Quantizer"), Huffman coding of the quantization codes
 * (Section 3.2 "Encoder"), and the matching reconstruction, in the stage
 * order of Algorithm 1 (Section 3.3).  Every stage runs in HIP kernels on the
 * device; the lossless back-end of the paper (zstd) is not part of the
 * library and, if wanted, is applied by the caller on the host.
 *
 * Conventions
 *  - All functions return an sz_status (0 = success, negative = error); no
 *    exception crosses the ABI.  sz_last_error() describes the last failure
 *    on a context.
 *  - "d_" pointers are device pointers (HBM of the context's device); "h_"
 *    pointers are host pointers.  The caller owns every buffer it passes; the
 *    library never frees them.  The context owns its scratch memory, grown on
 *    demand and released by sz_ctx_destroy.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is ordered on that stream.  Calls that return a size to the host
 *    synchronise the stream before returning.
 *  - Arrays are row-major: dims[ndim-1] is the contiguous dimension.
 *  - Alignment: field buffers (d_in of sz_compress, d_out of sz_decompress)
 *    must be 16-byte aligned and stream buffers 8-byte aligned (SZ_ERR_ARG
 *    otherwise); allocations from hipMalloc always are.
 *  - A context is not thread-safe: calls on one context must not overlap.
 *  - Limits: 1 <= ndim <= 4; a dimension may be 0 (empty field); the number
 *    of points n = prod(dims) is at most 2^32 - 1.
 */
#ifndef SZG_H
#define SZG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { SZ_F32 = 0, SZ_F64 = 1 } sz_dtype;

/* SZ_EB_ABS: eb = (T)value.  SZ_EB_REL: eb = (T)(value * (max - min)) over
 * the finite values of the field, computed in double (Section 6.2, caption
 * of the throughput figure: the relative bound is the bound normalised by
 * the value range); 0 when no value is finite.  value must be finite and
 * >= 0, and the resolved eb must be finite. */
/* SZ_EB_PWREL: point-wise relative, |x - x'| <= value * |x| for every
 * normal x, with 0 < value < 1 and value above the type's precision
 * (SZ_ERR_ARG otherwise).  A logarithmic preprocessor (Section 3.1 and
 * Section 3.2 "Preprocessor") maps y = log2|x| to a double field that the
 * same pipeline compresses with an absolute bound; the sign bits are stored
 * (a bit per value) when any is set.  Zeros and subnormal values come back
 * as signed zeros, infinities and NaN as themselves (NaN payloads are not
 * kept).  Size the output with sz_compress_bound_pwrel. */
typedef enum { SZ_EB_ABS = 0, SZ_EB_REL = 1, SZ_EB_PWREL = 2 } sz_eb_mode;

/* Interpolation along each dimension (Section 6.2, SZ3-Interp): linear
 * (midpoint of the two neighbours at +-s) or cubic (4-point Lagrange
 * midpoint rule, quadratic or linear near the boundary).  SZ_INTERP_ADAPTIVE
 * picks one of the two per level before compressing (SZ3-Interp selects
 * among its interpolation predictors): every point of the level is
 * predicted both ways from the original values, its cost is the quantizer's
 * bin index |k| capped at the radius, and the level takes cubic unless its
 * linear cost sum is smaller.  The choice is stored in the stream (a bit per
 * level) and costs one extra read of the field and one host round trip.
 * SZ_LORENZO is the first-order Lorenzo predictor (Section 3.2 "Predictor",
 * the predictor half of SZ3-LR): each point in flat order from the
 * reconstructed values of its 2^N - 1 lower neighbours (sum over the nonempty
 * sets S of dimensions of (-1)^(|S|+1) x'(q - e_S), outside the grid 0),
 * through the same quantizer, encoder and stream format; it takes no
 * dim_order.  Its points depend on each other through the quantizer, so it
 * runs as wavefronts of blocks (one launch per block diagonal). */
typedef enum {
  SZ_INTERP_LINEAR = 0,
  SZ_INTERP_CUBIC = 1,
  SZ_INTERP_ADAPTIVE = 2,
  SZ_LORENZO = 3
} sz_predictor;

typedef enum {
  SZ_OK = 0,
  SZ_ERR_ARG = -1,        /* invalid argument (shape, bound, options, pointers) */
  SZ_ERR_DTYPE = -2,      /* unknown dtype */
  SZ_ERR_CAPACITY = -3,   /* output buffer too small; required size returned */
  SZ_ERR_CORRUPT = -4,    /* stream fails validation */
  SZ_ERR_DEVICE = -5,     /* a HIP runtime call failed */
  SZ_ERR_NOMEM = -6,      /* device or host allocation failed */
  SZ_ERR_UNSUPPORTED = -7 /* valid request the library does not implement */
} sz_status;

/* Options that are recorded in the stream (they change the bytes). */
typedef struct {
  uint32_t radius;       /* quantizer radius R, 1..32768; codes are 0..2R-1, 0 =
                            unpredictable.  Default 32768. */
  uint32_t chunk;        /* symbols per independently decodable Huffman chunk,
                            a multiple of 64 in [64, 65536].  Default 4096. */
  uint8_t dim_order[4];  /* order in which each level visits the dimensions;
                            a permutation of 0..ndim-1.  Default identity. */
  uint32_t subchunks;    /* S: each chunk is split into S equal runs whose
                            starting bit offsets are stored, so S decoder lanes
                            share a chunk.  1, or 2, 4 or 8 where chunk/S is a
                            multiple of max(32, chunk/64).  0 (default) picks 4,
                            else 2, else 1. */
} sz_options;

/* Fields of a stream header, decoded on the host by sz_inspect. */
typedef struct {
  int dtype;
  int ndim;
  uint64_t dims[4];
  uint64_t n;
  int predictor;
  uint8_t dim_order[4];
  int eb_mode;
  double eb_user;      /* the bound value as passed to sz_compress */
  double eb;           /* the resolved bound in the field type, widened */
  uint32_t radius;
  uint32_t chunk;
  uint32_t sub;        /* sub-chunks per chunk */
  uint64_t n_unpred;   /* unpredictable values stored verbatim */
  uint32_t nsym;       /* symbols with a Huffman code */
  uint64_t total_words;/* 32-bit words of Huffman bitstream */
  uint64_t stream_bytes;
  int coded_dtype;     /* dtype of the coded field: dtype, or SZ_F64 (the
                          logarithms) in the point-wise relative mode */
  int signs;           /* point-wise relative mode: 1 if a sign section follows */
  uint64_t off_signs;  /* byte offset of that section (0 if none) */
  uint32_t level_mask; /* adaptive predictor: bit l - 1 set when level l
                          (stride 2^(l-1)) is cubic; 0 otherwise */
} sz_info;

typedef struct sz_ctx sz_ctx;

/* Create a context bound to HIP device `device` (the device is made current
 * for each call).  Returns NULL on failure. */
sz_ctx* sz_ctx_create(int device);
void sz_ctx_destroy(sz_ctx* ctx);
/* Human-readable description of the last error on ctx (never NULL). */
const char* sz_last_error(const sz_ctx* ctx);

void sz_default_options(sz_options* opts);

/* Upper bound on the compressed size in bytes for any field of this shape
 * and type (0 on invalid arguments).  Host only. */
size_t sz_compress_bound(int dtype, int ndim, const uint64_t* dims,
                         const sz_options* opts);

/* The same bound for eb_mode SZ_EB_PWREL (a double field of logarithms and
 * a sign section).  Host only. */
size_t sz_compress_bound_pwrel(int dtype, int ndim, const uint64_t* dims,
                               const sz_options* opts);

/* Compress the field d_in (device, n values of dtype) into d_out (device,
 * out_capacity bytes).  Stages, all on the device: error-bound resolution;
 * interpolation prediction + quantization level by level and dimension by
 * dimension (Algorithm 1, predict/quantize loop); code histogram; Huffman
 * code lengths and canonical codebook; chunked bit packing; compaction of the
 * unpredictable values; stream assembly.  On success *out_size (host) is the
 * stream length.  If the stream does not fit, returns SZ_ERR_CAPACITY with
 * *out_size = the required size and leaves d_out partially written.
 * opts may be NULL (defaults).  With eb_mode SZ_EB_PWREL the field first
 * goes through the logarithmic preprocessor (see sz_eb_mode) and the stream
 * ends with the sign section.  Synchronises `stream`. */
int sz_compress(sz_ctx* ctx, const void* d_in, int dtype, int ndim,
                const uint64_t* dims, int eb_mode, double eb, int predictor,
                const sz_options* opts, void* d_out, size_t out_capacity,
                size_t* out_size, void* stream);

/* sz_compress for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, stream bytes and status codes as sz_compress, except:
 * - the size-dependent scratch (reconstruction n*sizeof(dtype), codes 2n,
 *   four chunk tables of 24 bytes per chunk in all, and for three-dimensional
 *   fields room for the stride-2 lattice, ceil(n0/2)*ceil(n1/2)*ceil(n2/2)
 *   values; each piece rounded up to 256 bytes) lives in one static device
 *   array of SZ_NOALLOC_SCRATCH_BYTES per GPU, held from library load until
 *   the process ends.  A field that needs more returns SZ_ERR_NOMEM before
 *   any work is enqueued (fields of up to about 10M f32 or 6M f64 values fit);
 * - the context's fixed tables come from sz_ctx_create, so the call itself
 *   makes no hipMalloc, hipFree or other allocating call;
 * - SZ_EB_PWREL returns SZ_ERR_UNSUPPORTED, and timing (sz_set_timing) is
 *   not recorded.
 * Every call on a GPU shares that GPU's array, and the context's tables, and
 * the array keeps the last call's contents: calls that overlap on one GPU
 * (on any context or stream) race and must be serialised by the caller.
 * sz_debug_codes after this call reads the codes from the array.
 * Synchronises `stream`. */
#define SZ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int sz_compress_noalloc(sz_ctx* ctx, const void* d_in, int dtype, int ndim,
                        const uint64_t* dims, int eb_mode, double eb,
                        int predictor, const sz_options* opts, void* d_out,
                        size_t out_capacity, size_t* out_size, void* stream);

/* Decompress a stream (device, stream_size bytes) into d_out (device,
 * out_capacity bytes, n values of the stream's dtype): parse and validate
 * the header, decode the Huffman chunks, scatter the unpredictable values,
 * and rebuild the field with the same traversal and arithmetic as the
 * compressor, so the result equals the compressor's reconstruction bit for
 * bit (point-wise relative streams: then through the inverse transform,
 * into the original dtype).  Returns SZ_ERR_CORRUPT for an inconsistent stream (d_out may then be
 * partially written), SZ_ERR_CAPACITY if d_out is too small.  Synchronises
 * `stream`. */
int sz_decompress(sz_ctx* ctx, const void* d_stream, size_t stream_size,
                  void* d_out, size_t out_capacity, void* stream);

/* Decode the header of a stream held in host memory (at least the first 128
 * bytes).  Host only; validates the header fields. */
int sz_inspect(const void* h_stream, size_t len, sz_info* info);

/* Host lossless stage on a finished stream (paper Section 3: the lossless
 * module ends every pipeline; SZ3-Interp and SZ3-LR use zstd, Section 6.2,
 * for which zlib's deflate stands in here).  Both calls work on host memory
 * and treat the stream as opaque bytes; the GPU path does not depend on them.
 *
 * sz_lossless_bound: the largest packed size of n bytes.
 * sz_lossless_pack: h_in[0, n) to a zlib stream (RFC 1950) at `level` 0..9
 *   (zlib's levels; 1 is fastest) in h_out[0, capacity); *out_size = its
 *   length.  SZ_ERR_CAPACITY (with *out_size = the bound) when it does not
 *   fit; SZ_ERR_ARG for a bad level or null pointers; SZ_ERR_UNSUPPORTED for
 *   n >= 2^32.  The output equals zlib's compress2 of the same bytes.
 * sz_lossless_unpack: the inverse into h_out[0, capacity); *out_size = the
 *   restored length.  SZ_ERR_CAPACITY when the restored bytes do not fit,
 *   SZ_ERR_CORRUPT for invalid or truncated input or bytes after its end.
 * The caller owns every buffer; nothing is kept between calls. */
size_t sz_lossless_bound(size_t n);
int sz_lossless_pack(const void* h_in, size_t n, void* h_out, size_t capacity,
                     size_t* out_size, int level);
int sz_lossless_unpack(const void* h_in, size_t n, void* h_out, size_t capacity,
                       size_t* out_size);

/* One field of a batch (sz_compress_batch).  Inputs are read, outputs
 * (out_size, status) written by the call. */
typedef struct {
  const void* d_in;
  int dtype;
  int ndim;
  uint64_t dims[4];
  int eb_mode;
  double eb;
  int predictor;
  void* d_out;
  size_t out_capacity;
  size_t out_size;  /* written: stream bytes (or required bytes on CAPACITY) */
  int status;       /* written: sz_status of this field */
} sz_field;

/* Compress many fields of uneven shape and bound in one stream-ordered batch.
 * Each field's stream is byte-identical to what sz_compress produces for it
 * alone.  Returns SZ_OK when every field succeeded, else the first failing
 * field's status.  Synchronises `stream`. */
int sz_compress_batch(sz_ctx* ctx, sz_field* fields, int nfields,
                      const sz_options* opts, void* stream);

/* ---- request server -------------------------------------------------------
 * Many compression and decompression calls (Section 3.1's interfaces) run
 * side by side by a pool of `workers` threads, each with its own context and
 * HIP stream.  Requests are admitted in arrival order while the device
 * memory the library needs for them fits `budget_bytes`: every worker's
 * fixed tables, the scratch idle workers keep for reuse, and the scratch of
 * running requests (idle workers release theirs when the next request would
 * not fit otherwise).  The caller's input and output buffers are not counted
 * and must stay valid until the request is done.  A request's output is
 * byte-identical to the same sz_compress / sz_decompress call alone. */
typedef enum { SZ_REQ_COMPRESS = 0, SZ_REQ_DECOMPRESS = 1 } sz_request_kind;
typedef struct {
  int kind;               /* sz_request_kind */
  const void* d_in;       /* compress: the field; decompress: the stream (device) */
  size_t in_size;         /* decompress: stream bytes */
  int dtype;              /* compress: as sz_compress */
  int ndim;
  uint64_t dims[4];
  int eb_mode;
  double eb;
  int predictor;
  int has_options;        /* compress: 0 = default options */
  sz_options options;
  void* d_out;            /* the stream (compress) or the field (decompress) */
  size_t out_capacity;
  void* wait_event;       /* a hipEvent_t recorded where d_in was produced (and
                             where d_out was last used), or NULL: the request's
                             work waits for it on the device before it reads
                             or writes either buffer. The event must stay
                             valid until the request is done. */
} sz_request;
typedef struct sz_server sz_server;

/* NULL if the device is missing, workers is outside 1..64, or the workers'
 * fixed tables alone exceed the budget. */
sz_server* sz_server_create(int device, size_t budget_bytes, int workers);
/* Queues a request; *ticket identifies it.  SZ_ERR_ARG for a malformed
 * request, SZ_ERR_CORRUPT for an unreadable stream header, SZ_ERR_NOMEM when
 * the request could never fit the budget.  Errors of the call itself are
 * reported by poll / wait. */
int sz_server_submit(sz_server* s, const sz_request* req, uint64_t* ticket);
/* Non-blocking: *done = 1 once finished, with the call's status and output
 * bytes (stream bytes, or field bytes for decompression); a finished ticket
 * is then forgotten.  SZ_ERR_ARG for an unknown ticket. */
int sz_server_poll(sz_server* s, uint64_t ticket, int* done, int* status, size_t* out_size);
/* Blocks until the request is done, then as poll. */
int sz_server_wait(sz_server* s, uint64_t ticket, int* status, size_t* out_size);
/* Device bytes counted against the budget now. */
size_t sz_server_used_bytes(sz_server* s);
/* Finishes every submitted request, then frees the workers. */
void sz_server_destroy(sz_server* s);

/* ---- measurement and debugging ------------------------------------------
 * sz_set_timing(ctx, 1) records a pair of HIP events on the launch stream
 * around the kernels of each family a call runs; sz_timing_get() returns,
 * for the family `name`, the summed duration (ms) and the number of timed
 * regions since the last sz_timing_reset().  Names: compression "minmax",
 * "interp" (the origin and every level), "histogram", "codebook", "encode",
 * "other" (stream tables); decompression "decode_tables", "chunk_scan",
 * "decode" (the chunk decoder alone), "recon" (the origin and every level).
 * sz_set_timing_family(ctx, name) restricts the events to that family (NULL
 * or "": every family), which keeps the cost of timing off the others. */
int sz_set_timing(sz_ctx* ctx, int enable);
int sz_set_timing_family(sz_ctx* ctx, const char* name);
int sz_timing_get(sz_ctx* ctx, const char* name, double* total_ms,
                  uint64_t* launches);
int sz_timing_reset(sz_ctx* ctx);

/* Copy the quantization codes (n u16, flat order) of the last sz_compress
 * on ctx into d_codes (device). */
int sz_debug_codes(sz_ctx* ctx, void* d_codes, size_t capacity, void* stream);

#ifdef __cplusplus
}
#endif
#endif
