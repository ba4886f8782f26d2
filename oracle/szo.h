/*
 * szo.h -- the CPU oracle for the interpolation compressor hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, single-threaded
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke entry point and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * What it follows (paper: "SZ3: A Modular Framework for Composing
 * Prediction-Based Error-Bounded Lossy Compressors"):
 *   - Algorithm 1 (Section 3.3): predict and quantize every point, then save
 *     the quantizer state (unpredictable values), then Huffman-encode the
 *     whole code array, then save the encoder state (the code table).
 *   - Section 3.2, "Quantizer": the linear-scaling quantizer -- equal
 *     consecutive bins of width twice the error bound, the code is the index
 *     of the bin holding the prediction error, out-of-range errors are
 *     unpredictable and stored separately.
 *   - Section 3.2, "Encoder": Huffman coding -- frequencies, greedy tree,
 *     codebook, encode; the tree is saved with the stream.
 *   - Section 6.2, "SZ3-Interp": interpolation predictor (linear and cubic)
 *     with constant coefficients, predicting from already reconstructed
 *     points, followed by the linear-scaling quantizer and Huffman coding.
 *   - Section 6.2, caption of the throughput figure: the relative error bound
 *     is the error bound normalised by the value range.
 *   - Appendix A.3: quantize(data, pred) / recover(pred, code).
 *
 * Where the paper is silent (level structure, stencils at the boundary,
 * tie-breaking, bit order, chunking, stream layout) the oracle implements
 * the readings listed in the design notes of this repository; each function
 * below says which.
 *
 * Arithmetic: every floating-point operation is one IEEE operation in the
 * field's own type T (float or double), round-to-nearest-even, in the order
 * written; the file is compiled with -O2 -ffp-contract=off -fno-fast-math.
 */
#ifndef SZO_H
#define SZO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SZO_F32 = 0, SZO_F64 = 1 };
enum { SZO_ABS = 0, SZO_REL = 1, SZO_PWREL = 2 };
enum { SZO_LINEAR = 0, SZO_CUBIC = 1, SZO_ADAPTIVE = 2, SZO_LORENZO = 3 };
enum {
  SZO_OK = 0,
  SZO_ERR_ARG = -1,
  SZO_ERR_CAPACITY = -3,
  SZO_ERR_CORRUPT = -4,
  SZO_ERR_NOMEM = -6
};

#define SZO_HEADER_BYTES 128
#define SZO_MAX_RADIUS 32768u
#define SZO_MAX_CODE_LEN 64

/* Resolve the error bound into the field type.  ABS: eb = (T)value.
 * REL: eb = (T)(value * ((double)max - (double)min)) over the finite
 * values, 0 if there are none.  *eb_t receives the T value widened to
 * double.  Returns SZO_ERR_ARG if value < 0, is not finite, or the
 * resolved eb is not finite. */
int szo_resolve_eb(const void* x, uint64_t n, int dtype, int eb_mode,
                   double value, double* eb_t);

/* Multilevel interpolation predictor + linear-scaling quantizer over the
 * whole field.  codes: n u16 in flat (row-major) order; recon: n values of
 * type T, the reconstructed field the decompressor will produce. */
int szo_predict_quantize(const void* x, int dtype, int ndim,
                         const uint64_t* dims, const uint8_t* order,
                         int predictor, double eb_t, uint32_t radius,
                         uint16_t* codes, void* recon);

/* Rebuild the field from codes and the unpredictable values (flat order). */
int szo_reconstruct(const uint16_t* codes, const void* unpred,
                    uint64_t n_unpred, int dtype, int ndim,
                    const uint64_t* dims, const uint8_t* order, int predictor,
                    double eb_t, uint32_t radius, void* out);

/* Quantize one value; *code is 0 for unpredictable. */
int szo_quantize_one(int dtype, const void* x, const void* pred, double eb_t,
                     uint32_t radius, uint16_t* code, void* recon);

/* Walk the traversal without data: count visits per point and count stencil
 * reads of points that are not final yet.  visits: n counters. */
int szo_check_traversal(int ndim, const uint64_t* dims, const uint8_t* order,
                        int predictor, uint32_t* visits,
                        uint64_t* early_reads);

int szo_histogram(const uint16_t* codes, uint64_t n, uint32_t nsym,
                  uint64_t* hist);

/* Huffman code lengths by the two-queue greedy merge.  Returns the maximum
 * length (0 when no symbol is used) or a negative status. */
int szo_huffman_lengths(const uint64_t* hist, uint32_t nsym, uint8_t* lens);

/* Canonical codewords from lengths (RFC 1951, section 3.2.2). */
int szo_canonical_codes(const uint8_t* lens, uint32_t nsym,
                        uint64_t* codewords);

/* Sub-chunks per chunk: 1, or 2, 4 or 8 when chunk splits into sub-chunks
 * holding a multiple of max(32, chunk/64) symbols each.  Returns SZO_OK or
 * SZO_ERR_ARG. */
int szo_check_sub(uint32_t chunk, uint32_t sub);

/* Pack symbols chunk by chunk, MSB first into u32 words, each chunk padded
 * to a word.  chunk_words gets ceil(n/chunk) counts; words may be NULL to
 * only count.  sub_bits (may be NULL) gets, per chunk, the bit offset of
 * sub-chunks 1..sub-1 from the chunk's first bit (sub - 1 entries). */
int szo_pack(const uint16_t* codes, uint64_t n, const uint8_t* lens,
             const uint64_t* codewords, uint32_t chunk, uint32_t sub,
             uint32_t* words, uint32_t* chunk_words, uint32_t* sub_bits,
             uint64_t* total_words);

/* Decode n symbols packed by szo_pack; sub_bits (NULL when sub == 1) must
 * match the decoded sub-chunk starts. */
int szo_unpack(const uint32_t* words, uint64_t total_words,
               const uint32_t* chunk_words, uint64_t n, uint32_t chunk,
               uint32_t sub, const uint32_t* sub_bits, const uint8_t* lens,
               uint32_t nsym, uint16_t* codes);

/* The logarithmic preprocessor of the point-wise relative mode (paper
 * Section 3.1 and 3.2 "Preprocessor": the data go to the logarithmic domain
 * and are compressed there with an absolute bound derived from the
 * point-wise relative one).  The maps are written out from their series so
 * that every implementation computes the same bits:
 *   szo_log2(a), a finite and > 0: a = m 2^e with m in [sqrt(1/2), sqrt(2));
 *     log2 a = e + ln(m) / ln 2, ln m = 2 atanh(s), s = (m - 1)/(m + 1),
 *     atanh by its Maclaurin series to s^29 (Horner in s^2);
 *   szo_exp2(y), y finite: y = k + f, k = rint(y), |f| <= 1/2;
 *     2^y = 2^k exp(f ln 2), exp by its Taylor series to t^18 (Horner).
 * szo_pwrel_delta: the log field's absolute bound for a point-wise relative
 * bound eps of a T field: log2((1 + eps)/(1 + 4u)) (1 - 2^-20), u the unit
 * roundoff of T; <= 0 (unusable) when eps is too small for T. */
double szo_log2(double a);
double szo_exp2(double y);
double szo_pwrel_delta(double eps, int dtype);

/* Whole pipeline.  order may be NULL (identity).  *stream is allocated with
 * malloc and must be released with szo_free.  codes_out / recon_out are
 * optional (n entries each). */
int szo_compress(const void* x, int dtype, int ndim, const uint64_t* dims,
                 int eb_mode, double eb, int predictor, uint32_t radius,
                 uint32_t chunk, uint32_t sub, const uint8_t* order,
                 uint8_t** stream, uint64_t* stream_size, uint16_t* codes_out,
                 void* recon_out);

/* Parse, validate and decode a stream.  out holds n values of the stream's
 * type; codes_out is optional. */
int szo_decompress(const uint8_t* stream, uint64_t stream_size, void* out,
                   uint64_t out_bytes, uint16_t* codes_out);

void szo_free(void* p);

#ifdef __cplusplus
}
#endif
#endif
