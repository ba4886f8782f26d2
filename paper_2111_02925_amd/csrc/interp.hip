// Error-bound resolution, multilevel interpolation prediction + linear-scaling
// quantization, and the matching reconstruction, for gfx950.
//
// Paper: SZ3 (arXiv 2111.02925).  Algorithm 1 (Section 3.3) predicts and
// quantizes every point before encoding; SZ3-Interp (Section 6.2) predicts
// each point by constant-coefficient interpolation of already reconstructed
// points; the linear-scaling quantizer (Section 3.2) maps the prediction
// error to the index of a bin of width 2*eb and keeps out-of-range values
// verbatim; recover (Appendix A.3) inverts it.  The range-relative bound is
// the bound normalised by the value range (Section 6.2, throughput figure).
//
// Arithmetic contract: every floating-point step is one IEEE operation in the
// field type T, in a fixed order, with no contraction (-ffp-contract=off) and
// IEEE denormals, so results are reproducible bit for bit by any conforming
// implementation of the same steps.
#include "common.h"
#include "device_math.h"

namespace szg {

// ---------------------------------------------------------------- helpers

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

__global__ void k_meta_init(Meta* m) {
  m->key_min = ~0ull;
  m->key_max = 0;
  m->eb = 0;
  m->twoeb = 0;
  m->inv2eb = 0;
  m->nsym_used = 0;
  m->max_len = 0;
  m->sym_lo = 0xFFFFFFFFu;
  m->sym_hi = 0;
  m->n_unpred = 0;
  m->total_words = 0;
  m->stream_bytes = 0;
  m->status = 0;
  m->hist_far = 0;
}

hipError_t launch_meta_init(Meta* m, hipStream_t st) {
  hipLaunchKernelGGL(k_meta_init, dim3(1), dim3(1), 0, st, m);
  return hipGetLastError();
}

// ------------------------------------------------------- finite min / max
// Order-preserving unsigned keys: flipping the sign bit of non-negative values
// and all bits of negative ones makes unsigned comparison match the order of
// the (finite) floating-point values.

__device__ __forceinline__ uint64_t order_key(float v) {
  uint32_t b = __float_as_uint(v);
  return (b & 0x80000000u) ? (uint64_t)(~b) : (uint64_t)(b | 0x80000000u);
}
__device__ __forceinline__ uint64_t order_key(double v) {
  uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | (1ull << 63));
}
template <typename T>
__device__ __forceinline__ T key_value(uint64_t k);
template <>
__device__ __forceinline__ float key_value<float>(uint64_t k) {
  uint32_t b = (uint32_t)k;
  return __uint_as_float((b & 0x80000000u) ? (b & 0x7FFFFFFFu) : ~b);
}
template <>
__device__ __forceinline__ double key_value<double>(uint64_t k) {
  return __longlong_as_double((long long)((k >> 63) ? (k & ~(1ull << 63)) : ~k));
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ void fold_minmax(T v, uint64_t& lo, uint64_t& hi) {
  if (finite_t(v)) {
    uint64_t k = order_key(v);
    lo = k < lo ? k : lo;
    hi = k > hi ? k : hi;
  }
}

// Grid-stride reduction with 16-byte loads; one 64-bit atomic pair per block.
template <typename T>
__global__ __launch_bounds__(256) void k_minmax(const T* __restrict__ x, uint64_t n, Meta* m) {
  constexpr int V = 16 / sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(V)));
  uint64_t lo = ~0ull, hi = 0;
  const uint64_t nv = n / V;
  const vec_t* xv = reinterpret_cast<const vec_t*>(x);
  const uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  for (; i + 3 * gs < nv; i += 4 * gs) {
    vec_t a = __builtin_nontemporal_load(xv + i);
    vec_t b = __builtin_nontemporal_load(xv + i + gs);
    vec_t c = __builtin_nontemporal_load(xv + i + 2 * gs);
    vec_t d = __builtin_nontemporal_load(xv + i + 3 * gs);
#pragma unroll
    for (int k = 0; k < V; k++) {
      fold_minmax<T>(a[k], lo, hi);
      fold_minmax<T>(b[k], lo, hi);
      fold_minmax<T>(c[k], lo, hi);
      fold_minmax<T>(d[k], lo, hi);
    }
  }
  for (; i < nv; i += gs) {
    vec_t a = xv[i];
#pragma unroll
    for (int k = 0; k < V; k++) fold_minmax<T>(a[k], lo, hi);
  }
  for (uint64_t t = nv * V + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < n; t += gs)
    fold_minmax<T>(x[t], lo, hi);
  lo = wave_min_u64(lo);
  hi = wave_max_u64(hi);
  __shared__ uint64_t slo[4], shi[4];
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    slo[w] = lo;
    shi[w] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); k++) {
      lo = slo[k] < lo ? slo[k] : lo;
      hi = shi[k] > hi ? shi[k] : hi;
    }
    if (lo != ~0ull) {
      atomicMin((unsigned long long*)&m->key_min, (unsigned long long)lo);
      atomicMax((unsigned long long*)&m->key_max, (unsigned long long)hi);
    }
  }
}

hipError_t launch_minmax(const void* x, int dtype, uint64_t n, Meta* m, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 256 * 64 - 1) / (256 * 64);
  if (blocks < 1) blocks = 1;
  if (blocks > 2048) blocks = 2048;
  if (dtype == SZ_F32)
    hipLaunchKernelGGL(k_minmax<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const float*)x, n, m);
  else
    hipLaunchKernelGGL(k_minmax<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const double*)x, n, m);
  return hipGetLastError();
}

// eb in the field type; twoeb and 1/twoeb are derived from it in T.  REL:
// value * (max - min) in double, then rounded to T.
template <typename T>
__global__ void k_resolve_eb(int mode, double value, Meta* m) {
  T eb;
  if (mode == SZ_EB_ABS) {
    eb = (T)value;
  } else if (m->key_min == ~0ull) {
    eb = (T)0;
  } else {
    double mn = (double)key_value<T>(m->key_min);
    double mx = (double)key_value<T>(m->key_max);
    eb = (T)(value * (mx - mn));
  }
  if (!finite_t(eb)) m->status |= kStatusEbNotFinite;
  T twoeb = (T)2 * eb;
  T inv = (T)1 / twoeb;
  m->eb = (double)eb;
  m->twoeb = (double)twoeb;
  m->inv2eb = (double)inv;
}

hipError_t launch_resolve_eb(int dtype, int mode, double value, Meta* m, hipStream_t st) {
  if (dtype == SZ_F32)
    hipLaunchKernelGGL(k_resolve_eb<float>, dim3(1), dim3(1), 0, st, mode, value, m);
  else
    hipLaunchKernelGGL(k_resolve_eb<double>, dim3(1), dim3(1), 0, st, mode, value, m);
  return hipGetLastError();
}

// --------------------------------------------------- generic pass kernels
// One thread per point of a (level, dimension) pass; the points of a pass
// only read points finalised by earlier passes, so they are independent.

struct PassPoint {
  uint64_t f;  // flat index
  uint64_t i;  // coordinate along the pass dimension
};

__device__ __forceinline__ PassPoint pass_point(const PassGeom& g, uint32_t idx) {
  PassPoint p{0, 0};
  for (int e = g.ndim - 1; e >= 0; --e) {
    uint32_t c = idx % g.cnt[e];
    idx /= g.cnt[e];
    uint64_t q = (uint64_t)g.start[e] + (uint64_t)c * g.step[e];
    p.f += q * g.stride[e];
    if (e == g.d) p.i = q;
  }
  return p;
}

template <typename T, int PRED>
__device__ __forceinline__ T pass_predict(const T* v, const PassGeom& g, PassPoint p) {
  const uint64_t s = g.s;
  const uint64_t sd = s * g.stride[g.d];
  const bool has_a = p.i >= 3 * s;
  const bool has_c = p.i + s < g.nd;
  const bool has_e = p.i + 3 * s < g.nd;
  const T b = v[p.f - sd];
  const T c = has_c ? v[p.f + sd] : T(0);
  const bool need_a = has_a && (!has_c || PRED == SZ_INTERP_CUBIC);
  const T a = need_a ? v[p.f - 3 * sd] : T(0);
  const T e = (PRED == SZ_INTERP_CUBIC && has_e) ? v[p.f + 3 * sd] : T(0);
  return interp_predict<T, PRED>(a, b, c, e, has_a, has_c, has_e);
}

template <typename T, int PRED>
__global__ __launch_bounds__(256) void k_pass_compress(const T* __restrict__ x, T* rec,
                                                       uint16_t* codes, PassGeom g,
                                                       const Meta* __restrict__ m, uint32_t R) {
  uint64_t idx = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (idx >= g.total) return;
  const QuantParams<T> q = QuantParams<T>::from_meta(m, R);
  PassPoint p = pass_point(g, (uint32_t)idx);
  T pred = pass_predict<T, PRED>(rec, g, p);
  T r;
  codes[p.f] = (uint16_t)quantize(x[p.f], pred, q, r);
  rec[p.f] = r;
}

template <typename T>
__global__ void k_origin_compress(const T* __restrict__ x, T* rec, uint16_t* codes,
                                  const Meta* __restrict__ m, uint32_t R) {
  const QuantParams<T> q = QuantParams<T>::from_meta(m, R);
  T r;
  codes[0] = (uint16_t)quantize(x[0], T(0), q, r);
  rec[0] = r;
}

hipError_t launch_origin_compress(const void* x, int dtype, void* rec, uint16_t* codes,
                                  const Meta* m, uint32_t radius, hipStream_t st) {
  if (dtype == SZ_F32)
    hipLaunchKernelGGL(k_origin_compress<float>, dim3(1), dim3(1), 0, st, (const float*)x,
                       (float*)rec, codes, m, radius);
  else
    hipLaunchKernelGGL(k_origin_compress<double>, dim3(1), dim3(1), 0, st, (const double*)x,
                       (double*)rec, codes, m, radius);
  return hipGetLastError();
}

hipError_t launch_pass_compress(const void* x, int dtype, int predictor, void* rec,
                                uint16_t* codes, const PassGeom& g, const Meta* m,
                                uint32_t radius, hipStream_t st) {
  if (g.total == 0) return hipSuccess;
  dim3 grid((unsigned)((g.total + 255) / 256)), block(256);
  if (dtype == SZ_F32) {
    if (predictor == SZ_INTERP_CUBIC)
      hipLaunchKernelGGL((k_pass_compress<float, SZ_INTERP_CUBIC>), grid, block, 0, st,
                         (const float*)x, (float*)rec, codes, g, m, radius);
    else
      hipLaunchKernelGGL((k_pass_compress<float, SZ_INTERP_LINEAR>), grid, block, 0, st,
                         (const float*)x, (float*)rec, codes, g, m, radius);
  } else {
    if (predictor == SZ_INTERP_CUBIC)
      hipLaunchKernelGGL((k_pass_compress<double, SZ_INTERP_CUBIC>), grid, block, 0, st,
                         (const double*)x, (double*)rec, codes, g, m, radius);
    else
      hipLaunchKernelGGL((k_pass_compress<double, SZ_INTERP_LINEAR>), grid, block, 0, st,
                         (const double*)x, (double*)rec, codes, g, m, radius);
  }
  return hipGetLastError();
}

// Reconstruction: code 0 keeps the verbatim value already scattered into out
// by the decoder; any other code is recovered from the prediction.
template <typename T, int PRED>
__global__ __launch_bounds__(256) void k_pass_recon(const uint16_t* __restrict__ codes, T* out,
                                                    PassGeom g, T twoeb, uint32_t R) {
  uint64_t idx = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (idx >= g.total) return;
  PassPoint p = pass_point(g, (uint32_t)idx);
  uint32_t code = codes[p.f];
  if (code == 0) return;
  T pred = pass_predict<T, PRED>(out, g, p);
  out[p.f] = recover(pred, twoeb, code, R);
}

template <typename T>
__global__ void k_origin_recon(const uint16_t* __restrict__ codes, T* out, T twoeb, uint32_t R) {
  uint32_t code = codes[0];
  if (code != 0) out[0] = recover(T(0), twoeb, code, R);
}

hipError_t launch_origin_recon(const uint16_t* codes, int dtype, void* out, double eb_t,
                               uint32_t radius, hipStream_t st) {
  if (dtype == SZ_F32) {
    float eb = (float)eb_t;
    hipLaunchKernelGGL(k_origin_recon<float>, dim3(1), dim3(1), 0, st, codes, (float*)out,
                       2.0f * eb, radius);
  } else {
    hipLaunchKernelGGL(k_origin_recon<double>, dim3(1), dim3(1), 0, st, codes, (double*)out,
                       2.0 * eb_t, radius);
  }
  return hipGetLastError();
}

hipError_t launch_pass_recon(const uint16_t* codes, int dtype, int predictor, void* out,
                             const PassGeom& g, double eb_t, uint32_t radius, hipStream_t st) {
  if (g.total == 0) return hipSuccess;
  dim3 grid((unsigned)((g.total + 255) / 256)), block(256);
  if (dtype == SZ_F32) {
    float twoeb = 2.0f * (float)eb_t;
    if (predictor == SZ_INTERP_CUBIC)
      hipLaunchKernelGGL((k_pass_recon<float, SZ_INTERP_CUBIC>), grid, block, 0, st, codes,
                         (float*)out, g, twoeb, radius);
    else
      hipLaunchKernelGGL((k_pass_recon<float, SZ_INTERP_LINEAR>), grid, block, 0, st, codes,
                         (float*)out, g, twoeb, radius);
  } else {
    double twoeb = 2.0 * eb_t;
    if (predictor == SZ_INTERP_CUBIC)
      hipLaunchKernelGGL((k_pass_recon<double, SZ_INTERP_CUBIC>), grid, block, 0, st, codes,
                         (double*)out, g, twoeb, radius);
    else
      hipLaunchKernelGGL((k_pass_recon<double, SZ_INTERP_LINEAR>), grid, block, 0, st, codes,
                         (double*)out, g, twoeb, radius);
  }
  return hipGetLastError();
}

}  // namespace szg
