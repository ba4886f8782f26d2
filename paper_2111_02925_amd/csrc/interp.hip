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

__device__ __forceinline__ void meta_init(Meta* m) {
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
  m->slices_done = 0;
  m->hist_far = 0;
}

// (with nzero > 0, also zero[0 .. nzero), in the same launch)
__global__ void k_meta_init(Meta* m, uint32_t* zero, uint64_t nzero) {
  if (blockIdx.x == 0 && threadIdx.x == 0) meta_init(m);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nzero;
       i += (uint64_t)gridDim.x * blockDim.x)
    zero[i] = 0;
}

hipError_t launch_meta_init(Meta* m, hipStream_t st, uint32_t* zero, uint64_t nzero) {
  if (nzero && !zero) return hipErrorInvalidValue;
  uint64_t blocks = (nzero + 255) / 256;
  blocks = blocks < 1 ? 1 : blocks > 256 ? 256 : blocks;
  hipLaunchKernelGGL(k_meta_init, dim3((unsigned)blocks), dim3(256), 0, st, m, zero, nzero);
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

// A lane keeps its running minimum and maximum as values of T (non-finite
// inputs replaced by the infinity that leaves them unchanged: two selects and
// a min and a max per value); the keys are formed once, for the reductions.
// Which zero is kept when both signs occur does not change max - min.
template <typename T>
__device__ __forceinline__ void fold_minmax(T v, T& lo, T& hi) {
  const bool fin = finite_t(v);
  const T inf = __builtin_inf();
  lo = __builtin_fmin(lo, fin ? v : inf);
  hi = __builtin_fmax(hi, fin ? v : -inf);
}

// Grid-stride reduction with 16-byte loads.  Each workgroup's keys go to its
// pair of part[] (summed by the eb kernel: workgroups that end together
// would otherwise queue on the same two addresses), or with part null, into
// m by one 64-bit atomic pair.  (bid, nblk): this workgroup among the nblk
// that share the field.
template <typename T>
__device__ __forceinline__ void minmax_body(const T* __restrict__ x, uint64_t n, Meta* m,
                                            uint32_t bid, uint32_t nblk, uint64_t* part) {
  constexpr int V = 16 / sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(V)));
  T vlo = __builtin_inf(), vhi = -__builtin_inf();
  const uint64_t nv = n / V;
  const vec_t* xv = reinterpret_cast<const vec_t*>(x);
  const uint64_t gs = (uint64_t)nblk * blockDim.x;
  uint64_t i = bid * (uint64_t)blockDim.x + threadIdx.x;
  for (; i + 3 * gs < nv; i += 4 * gs) {
    vec_t a = __builtin_nontemporal_load(xv + i);
    vec_t b = __builtin_nontemporal_load(xv + i + gs);
    vec_t c = __builtin_nontemporal_load(xv + i + 2 * gs);
    vec_t d = __builtin_nontemporal_load(xv + i + 3 * gs);
#pragma unroll
    for (int k = 0; k < V; k++) {
      fold_minmax<T>(a[k], vlo, vhi);
      fold_minmax<T>(b[k], vlo, vhi);
      fold_minmax<T>(c[k], vlo, vhi);
      fold_minmax<T>(d[k], vlo, vhi);
    }
  }
  for (; i < nv; i += gs) {
    vec_t a = xv[i];
#pragma unroll
    for (int k = 0; k < V; k++) fold_minmax<T>(a[k], vlo, vhi);
  }
  for (uint64_t t = nv * V + bid * (uint64_t)blockDim.x + threadIdx.x; t < n; t += gs)
    fold_minmax<T>(x[t], vlo, vhi);
  // no finite value: the empty keys
  uint64_t lo = vlo <= vhi ? order_key(vlo) : ~0ull;
  uint64_t hi = vlo <= vhi ? order_key(vhi) : 0ull;
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
    if (part) {
      part[2 * bid] = lo;
      part[2 * bid + 1] = hi;
    } else if (lo != ~0ull) {
      atomicMin((unsigned long long*)&m->key_min, (unsigned long long)lo);
      atomicMax((unsigned long long*)&m->key_max, (unsigned long long)hi);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_minmax(const T* __restrict__ x, uint64_t n, Meta* m,
                                                uint64_t* part) {
  minmax_body<T>(x, n, m, blockIdx.x, gridDim.x, part);
}

hipError_t launch_minmax(const void* x, int dtype, uint64_t n, Meta* m, uint64_t* part,
                         hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = minmax_blocks(n);
  if (dtype == SZ_F32)
    hipLaunchKernelGGL(k_minmax<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const float*)x, n, m, part);
  else
    hipLaunchKernelGGL(k_minmax<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const double*)x, n, m, part);
  return hipGetLastError();
}

// eb in the field type; twoeb and 1/twoeb are derived from it in T.  REL:
// value * (max - min) in double, then rounded to T.
template <typename T>
__device__ __forceinline__ void resolve_eb(int mode, double value, Meta* m) {
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

// (nblk > 0: the minimum and maximum keys first, from the nblk pairs of
// part that k_minmax wrote, folded into m's)
template <typename T>
__global__ __launch_bounds__(256) void k_resolve_eb(int mode, double value, Meta* m,
                                                    const uint64_t* __restrict__ part,
                                                    uint32_t nblk) {
  if (nblk) {
    uint64_t lo = ~0ull, hi = 0;
    for (uint32_t i = threadIdx.x; i < nblk; i += blockDim.x) {
      lo = part[2 * i] < lo ? part[2 * i] : lo;
      hi = part[2 * i + 1] > hi ? part[2 * i + 1] : hi;
    }
    lo = wave_min_u64(lo);
    hi = wave_max_u64(hi);
    __shared__ uint64_t slo[4], shi[4];
    const int w = threadIdx.x >> 6;
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
      if (lo < m->key_min) m->key_min = lo;
      if (hi > m->key_max && lo != ~0ull) m->key_max = hi;
    }
  }
  if (threadIdx.x == 0) resolve_eb<T>(mode, value, m);
}

hipError_t launch_resolve_eb(int dtype, int mode, double value, Meta* m, hipStream_t st,
                             const uint64_t* part, uint32_t nblk) {
  if (nblk > kMinmaxBlocks || (nblk && !part)) return hipErrorInvalidValue;
  if (dtype == SZ_F32)
    hipLaunchKernelGGL(k_resolve_eb<float>, dim3(1), dim3(256), 0, st, mode, value, m, part, nblk);
  else
    hipLaunchKernelGGL(k_resolve_eb<double>, dim3(1), dim3(256), 0, st, mode, value, m, part, nblk);
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

// The coarsest levels in one workgroup.  Every point of levels L .. l_stop
// lies on the lattice of stride S = 2^(l_stop - 1) (all coordinates
// multiples of S), which is small (at most kSmallBytes of values and
// codes); as separate launches each level would cost a launch and a few
// dependent round trips to memory for a handful of points.  One workgroup
// loads the lattice into LDS, takes the origin and then the levels' passes
// in the traversal order on the lattice (a barrier after each pass), and
// stores the lattice's codes and values.  On the lattice, stride s becomes
// s / S and extent n_d becomes ceil(n_d / S); every neighbour test
// (i >= 3s, i + s < n_d, i + 3s < n_d) holds on the lattice exactly when it
// holds on the grid, so the per-pass kernels' arithmetic (pass_point,
// pass_predict, quantize / recover) gives their results.  Bit l - 1 of
// `cubic` selects cubic for level l.
constexpr uint32_t kSmallThreads = 1024;

template <typename T, bool RECON>
__device__ __forceinline__ void small_levels_body(const T* __restrict__ x, T* v, uint16_t* codes,
                                                  const SmallGeom& sg, const Meta* __restrict__ m,
                                                  T twoeb_dec, uint32_t R) {
  constexpr uint32_t kCap = kSmallBytes / (sizeof(T) + 2);
  __shared__ T lv[kCap];
  __shared__ uint16_t lc[kCap];
  const uint64_t S = 1ull << (sg.l_stop - 1);
  const int nd = sg.ndim;
  // lattice extents and strides (at most kCap points: 32-bit arithmetic);
  // loops unrolled over kMaxDims so that all of this stays in registers
  uint32_t me[kMaxDims] = {1, 1, 1, 1}, ls[kMaxDims] = {0, 0, 0, 0};
  uint32_t np = 1;
#pragma unroll
  for (int e = kMaxDims - 1; e >= 0; e--) {
    if (e < nd) {
      me[e] = (uint32_t)((sg.dims[e] + S - 1) / S);
      ls[e] = np;
      np *= me[e];
    }
  }
  auto grid_index = [&](uint32_t k) {
    uint64_t f = 0;
#pragma unroll
    for (int e = kMaxDims - 1; e >= 0; e--) {
      if (e < nd) {
        f += (uint64_t)(k % me[e]) * S * sg.stride[e];
        k /= me[e];
      }
    }
    return f;
  };
  // the lattice into LDS, eight loads a lane in flight
  constexpr int kU = 8;
  for (uint32_t k0 = 0; k0 < np; k0 += kU * kSmallThreads) {
    T vv[kU];
    uint16_t cc[kU];
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const uint32_t k = k0 + u * kSmallThreads + threadIdx.x;
      const uint64_t f = k < np ? grid_index(k) : 0;
      vv[u] = RECON ? v[f] : x[f];  // (reconstruction: the verbatim values of code-0 points)
      cc[u] = RECON ? codes[f] : (uint16_t)0;
    }
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const uint32_t k = k0 + u * kSmallThreads + threadIdx.x;
      if (k < np) {
        lv[k] = vv[u];
        if (RECON) lc[k] = cc[u];
      }
    }
  }
  __syncthreads();
  QuantParams<T> q{};
  if (!RECON) q = QuantParams<T>::from_meta(m, R);
  if (threadIdx.x == 0) {  // the origin, predicted as 0
    if (RECON) {
      const uint32_t code = lc[0];
      if (code) lv[0] = recover(T(0), twoeb_dec, code, R);
    } else {
      T r;
      lc[0] = (uint16_t)quantize(lv[0], T(0), q, r);
      lv[0] = r;
    }
  }
  // (compression: lv holds x until a point is visited, then its
  // reconstruction; the stencil reads only visited points)
  for (int l = sg.L; l >= sg.l_stop; l--) {
    const uint32_t sp = (uint32_t)((1ull << (l - 1)) / S);
    const bool cubic = (sg.cubic >> (l - 1)) & 1u;
    for (int j = 0; j < nd; j++) {
      __syncthreads();  // the previous pass (or the origin) is complete
      // the pass along d = order[j] (every lane computes its geometry): d an
      // odd multiple of sp, earlier dimensions of the order multiples of sp,
      // later ones multiples of 2 sp
      const int d = sg.order[j];
      uint32_t cnt[kMaxDims] = {1, 1, 1, 1}, start[kMaxDims] = {0, 0, 0, 0},
               step[kMaxDims] = {1, 1, 1, 1};
      uint32_t total = 1, ext_d = 1, str_d = 0;
#pragma unroll
      for (int e = 0; e < kMaxDims; e++) {
        if (e >= nd) continue;
        start[e] = e == d ? sp : 0u;
        step[e] = (e == d || sg.pos[e] > j) ? 2 * sp : sp;
        cnt[e] = start[e] < me[e] ? (me[e] - start[e] + step[e] - 1) / step[e] : 0u;
        total *= cnt[e];
        if (e == d) {
          ext_d = me[e];
          str_d = ls[e];
        }
      }
      const uint32_t sd = sp * str_d;
      for (uint32_t idx = threadIdx.x; idx < total; idx += kSmallThreads) {
        uint32_t rem = idx, f = 0, i = 0;
#pragma unroll
        for (int e = kMaxDims - 1; e >= 0; e--) {
          if (e < nd) {
            const uint32_t qe = start[e] + (rem % cnt[e]) * step[e];
            rem /= cnt[e];
            f += qe * ls[e];
            if (e == d) i = qe;
          }
        }
        // the stencil as in the per-pass kernels
        const bool has_a = i >= 3 * sp, has_c = i + sp < ext_d, has_e = i + 3 * sp < ext_d;
        const T b = lv[f - sd];
        const T c = has_c ? lv[f + sd] : T(0);
        const T a = has_a && (!has_c || cubic) ? lv[f - 3 * sd] : T(0);
        const T e = cubic && has_e ? lv[f + 3 * sd] : T(0);
        const T pred = cubic ? interp_predict<T, SZ_INTERP_CUBIC>(a, b, c, e, has_a, has_c, has_e)
                             : interp_predict<T, SZ_INTERP_LINEAR>(a, b, c, e, has_a, has_c, has_e);
        if (RECON) {
          const uint32_t code = lc[f];
          if (code) lv[f] = recover(pred, twoeb_dec, code, R);
        } else {
          T r;
          lc[f] = (uint16_t)quantize(lv[f], pred, q, r);
          lv[f] = r;
        }
      }
    }
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < np; k += kSmallThreads) {
    const uint64_t f = grid_index(k);
    v[f] = lv[k];
    if (!RECON) codes[f] = lc[k];
  }
}

template <typename T, bool RECON>
__global__ __launch_bounds__(kSmallThreads) void k_small_levels(
    const T* __restrict__ x, T* v, uint16_t* codes, SmallGeom sg, const Meta* __restrict__ m,
    T twoeb_dec, uint32_t R) {
  small_levels_body<T, RECON>(x, v, codes, sg, m, twoeb_dec, R);
}

// The levels the workgroup takes: from L down to the one with the smallest
// stride S >= 2 whose lattice fits kSmallBytes (l_stop = L + 1: the origin
// only).
SmallGeom plan_small_levels(int ndim, const uint64_t* dims, const uint8_t* order, int L,
                            uint32_t cubic_mask, int tsize) {
  SmallGeom sg{};
  sg.ndim = ndim;
  sg.L = L;
  sg.cubic = cubic_mask;
  uint64_t st = 1;
  for (int e = ndim - 1; e >= 0; e--) {
    sg.dims[e] = dims[e];
    sg.stride[e] = st;
    st *= dims[e];
  }
  for (int j = 0; j < ndim; j++) {
    sg.order[j] = order[j];
    sg.pos[order[j]] = (uint8_t)j;
  }
  const uint64_t cap = kSmallBytes / (uint64_t)(tsize + 2);
  sg.l_stop = L + 1;
  for (int l = L; l >= 2; l--) {
    const uint64_t s = 1ull << (l - 1);
    uint64_t pts = 1;
    for (int e = 0; e < ndim; e++) pts *= (dims[e] + s - 1) / s;
    if (pts > cap) break;
    sg.l_stop = l;
  }
  return sg;
}

hipError_t launch_small_levels_compress(const void* x, int dtype, void* rec, uint16_t* codes,
                                        const SmallGeom& sg, const Meta* m, uint32_t radius,
                                        hipStream_t st) {
  if (dtype == SZ_F32)
    hipLaunchKernelGGL((k_small_levels<float, false>), dim3(1), dim3(kSmallThreads), 0, st,
                       (const float*)x, (float*)rec, codes, sg, m, 0.0f, radius);
  else
    hipLaunchKernelGGL((k_small_levels<double, false>), dim3(1), dim3(kSmallThreads), 0, st,
                       (const double*)x, (double*)rec, codes, sg, m, 0.0, radius);
  return hipGetLastError();
}

hipError_t launch_small_levels_recon(const uint16_t* codes, int dtype, void* out,
                                     const SmallGeom& sg, double eb_t, uint32_t radius,
                                     hipStream_t st) {
  uint16_t* c = const_cast<uint16_t*>(codes);  // (read only in reconstruction)
  if (dtype == SZ_F32)
    hipLaunchKernelGGL((k_small_levels<float, true>), dim3(1), dim3(kSmallThreads), 0, st,
                       nullptr, (float*)out, c, sg, nullptr, 2.0f * (float)eb_t, radius);
  else
    hipLaunchKernelGGL((k_small_levels<double, true>), dim3(1), dim3(kSmallThreads), 0, st,
                       nullptr, (double*)out, c, sg, nullptr, 2.0 * eb_t, radius);
  return hipGetLastError();
}

// Adaptive interpolation: every level's cost under both predictors, from the
// ORIGINAL values at the stencil points (the level's choice is made on the
// host from these sums).  A point's cost under a predictor is the quantizer's
// bin index |k| = rint(|x - pred| / (2 eb)) capped at R (R when not finite;
// with eb = 0, 0 for an exact prediction and R otherwise).  Integer sums, so
// the order of accumulation does not change them.
//
// One launch covers every level: a point q other than the origin belongs to
// level t + 1, t = min over dimensions of ctz(q_e) (ctz(0) counting as
// infinite), and to the pass of that level along the dimension d, last in
// the traversal order, with ctz(q_d) = t (earlier dimensions of the order are
// at multiples of s = 2^t there, later ones at multiples of 2s).
//
// Work units are segments of one row along the last dimension; a lane takes
// pairs of columns (even, odd).  With t_row the fewest trailing zeros among
// the row's other coordinates (d_row that dimension, last in the order):
//  - the odd column is on level 1, along the row when t_row > 0 or the last
//    dimension comes after d_row in the order, else along d_row;
//  - the even column is on level 1 along d_row when t_row = 0, and on a
//    coarser level otherwise (a quarter of the rows in 3-D: 1/8 of the
//    points), where each lane finds its own level and dimension.
// Both columns' stencils are fetched (every load issued before any is used;
// idle lanes read their row's first point) and evaluated by the same code.
// The full estimate gives a unit (up to 256 columns) to one wave, which
// works out its geometry once for up to two pairs a lane, and each wave a
// contiguous run of units; the waves of one XCD (workgroup b on XCD b mod 8)
// take runs of one contiguous eighth of the field, so the rows and planes
// the stencils reach are read by waves of the same XCD at about the same
// time.  Flat indices fit 32 bits (fields hold fewer than 2^32 points).
constexpr uint32_t kEstThreads = 256;
constexpr uint32_t kEstWave = 64;          // lanes of a unit of the full estimate
constexpr uint32_t kEstWaveBlocks = 8192;  // most workgroups of the full estimate
constexpr uint32_t kEstBlocks = 8192;      // most workgroups of the per-order estimate

template <typename T>
__device__ __forceinline__ uint32_t est_cost(T d, T eb, T inv2eb, uint32_t R) {
  if (eb == T(0)) return d == T(0) ? 0u : R;
  const T k = rint_t(fabs_t(d) * inv2eb);
  return k < (T)R ? (uint32_t)k : R;  // (NaN: R)
}

// The stencil of the point at flat index f along a dimension with flat step
// sd (= s x stride), position i and extent nd: which neighbours exist and
// their values (absent ones read the point itself).
template <typename T>
struct EstStencil {
  T x, a, b, c, e;
  bool ha, hc, he;
};
// x[f]; with N (fields of fewer than 2^32 bytes) as a 32-bit byte offset
// from x, which the loads take as a scalar base plus a lane offset.
template <bool N, typename T>
__device__ __forceinline__ T est_ld(const T* __restrict__ x, uint32_t f) {
  if (N) return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(x) + f * (uint32_t)sizeof(T));
  return x[f];
}
template <bool N, typename T>
__device__ __forceinline__ EstStencil<T> est_fetch(const T* __restrict__ x, uint32_t f, uint32_t i,
                                                   uint32_t nd, uint32_t s, uint32_t sd) {
  EstStencil<T> st;
  // i >= s and i < nd; the comparisons avoid 32-bit overflow
  st.ha = ((i - s) >> 1) >= s;                    // i >= 3s
  st.hc = nd - i > s;                             // i + s < nd
  st.he = st.hc && ((nd - i - s - 1) >> 1) >= s;  // i + 3s < nd
  st.x = est_ld<N>(x, f);
  st.b = est_ld<N>(x, f - sd);
  st.c = est_ld<N>(x, st.hc ? f + sd : f);
  st.a = est_ld<N>(x, st.ha ? f - 3 * sd : f);
  st.e = est_ld<N>(x, st.he ? f + 3 * sd : f);
  return st;
}
// Both costs from a fetched stencil.  Where the whole wave is away from the
// ends (both neighbours on each side), the two interior rules alone are
// evaluated.
template <typename T>
__device__ __forceinline__ void est_eval(const EstStencil<T>& st, T eb, T inv2eb, uint32_t R,
                                         uint32_t& cl, uint32_t& cc) {
  T pl, pc;
  if (__builtin_amdgcn_ballot_w64(!(st.ha && st.he)) == 0) {
    pl = (st.b + st.c) * T(0.5);
    pc = (T(9) * (st.b + st.c) - (st.a + st.e)) * T(0.0625);
  } else {
    pl = interp_predict_sel<T, SZ_INTERP_LINEAR>(st.a, st.b, st.c, st.e, st.ha, st.hc, st.he);
    pc = interp_predict_sel<T, SZ_INTERP_CUBIC>(st.a, st.b, st.c, st.e, st.ha, st.hc, st.he);
  }
  cl = est_cost(st.x - pl, eb, inv2eb, R);
  cc = est_cost(st.x - pc, eb, inv2eb, R);
}

// A value of the lane `k` places up (k > 0) or down the wave, by DPP wave
// shifts; lanes without a source get 0 (the callers read theirs instead).
__device__ __forceinline__ uint32_t est_wave_shift(uint32_t v, int k) {
  if (k == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, false);
  if (k == -1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xF, 0xF, false);
  const uint32_t w = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, false);
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x130, 0xF, 0xF, false);  // k == 2
}
__device__ __forceinline__ float est_from_lane(float v, int k) {
  return __uint_as_float(est_wave_shift(__float_as_uint(v), k));
}
__device__ __forceinline__ double est_from_lane(double v, int k) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint64_t lo = est_wave_shift((uint32_t)b, k), hi = est_wave_shift((uint32_t)(b >> 32), k);
  return __longlong_as_double((long long)((hi << 32) | lo));
}
// The odd column co = ce + 1's stencil along the row, in a unit of columns
// [c0, c1) dealt as (even, odd) pairs to consecutive lanes: its neighbours
// are the even columns of this lane and of lanes -1, +1 and +2.  The fetch
// loads the point and those neighbours that no lane of the wave holds (the
// wave's ends, the unit's ends; absent neighbours read the point itself);
// the finish takes the others from the even columns' values xe, moved across
// the wave, once they have arrived.
template <bool N, typename T>
__device__ __forceinline__ EstStencil<T> est_odd_row_fetch(const T* __restrict__ x, uint32_t base,
                                                           uint32_t ce, uint32_t co, bool has_odd,
                                                           uint32_t c0, uint32_t c1, uint32_t ncol) {
  EstStencil<T> so;
  so.ha = has_odd && co >= 3;
  so.hc = has_odd && co + 1 < ncol;
  so.he = so.hc && co + 3 < ncol;
  const uint32_t lane = threadIdx.x & 63;
  const bool c_lane = lane < 63 && ce + 2 < c1, e_lane = lane < 62 && ce + 4 < c1;
  const bool a_lane = lane > 0 && ce >= c0 + 2;
  so.x = est_ld<N>(x, base + co);
  so.c = est_ld<N>(x, base + (!c_lane && so.hc ? co + 1 : co));
  so.e = est_ld<N>(x, base + (!e_lane && so.he ? co + 3 : co));
  so.a = est_ld<N>(x, base + (!a_lane && so.ha ? co - 3 : co));
  return so;
}
template <typename T>
__device__ __forceinline__ void est_odd_row_finish(EstStencil<T>& so, T xe, uint32_t ce, uint32_t c0,
                                                   uint32_t c1) {
  const uint32_t lane = threadIdx.x & 63;
  const bool c_lane = lane < 63 && ce + 2 < c1, e_lane = lane < 62 && ce + 4 < c1;
  const bool a_lane = lane > 0 && ce >= c0 + 2;
  const T c_l = est_from_lane(xe, 1), e_l = est_from_lane(xe, 2), a_l = est_from_lane(xe, -1);
  so.b = xe;
  if (c_lane) so.c = c_l;
  if (e_lane) so.e = e_l;
  if (a_lane) so.a = a_l;
}

// A unit of the estimate: a run of 2 x W x J columns (W lanes, J pairs a
// lane) of the row at coordinates q (all but the last dimension); its
// scalars.  t_row is the
// fewest trailing zeros among q, d_row (place p_row in the order, extent
// n_row, stride s_row) the dimension latest in the order that has them.
struct EstUnit {
  uint32_t base, qrow, srow, nrow, c0, c1;
  int trow, prow;
  bool odd_along_row;
};
template <uint32_t W, int J>
__device__ __forceinline__ EstUnit est_unit_at(const EstGeom& g, const uint8_t (&pos)[kMaxDims],
                                               const uint32_t (&q)[kMaxDims], uint32_t seg) {
  constexpr uint32_t kSeg = 2 * W * J;
  const int last = g.ndim - 1;
  const uint32_t ncol = (uint32_t)g.dims[last];
  EstUnit un;
  un.base = 0;
#pragma unroll
  for (int e = 0; e < kMaxDims - 1; e++)
    if (e < last) un.base += q[e] * (uint32_t)g.stride[e];
  un.trow = 64;
  un.prow = -1;
  un.qrow = un.srow = un.nrow = 0;
#pragma unroll
  for (int e = 0; e < kMaxDims - 1; e++) {
    const int te = q[e] ? __builtin_ctz(q[e]) : 64;
    if (e < last && (te < un.trow || (te == un.trow && (int)pos[e] > un.prow))) {
      un.trow = te;
      un.prow = pos[e];
      un.qrow = q[e];
      un.srow = (uint32_t)g.stride[e];
      un.nrow = (uint32_t)g.dims[e];
    }
  }
  un.c0 = seg * kSeg;
  un.c1 = ncol - un.c0 > kSeg ? un.c0 + kSeg : ncol;
  un.odd_along_row = un.trow > 0 || (int)pos[last] > un.prow;
  return un;
}

// A unit priced for both predictors, every load issued before any is used;
// levels 1 and 2 into the caller's accumulators, coarser ones into the
// block's table sh.  For a row with t_row = 0 the odd column lies on level
// 1, along the row unless d_row comes later in the order, and the even
// column on level 1 along d_row; otherwise the odd column lies on level 1
// along the row, and the even column with t_c trailing zeros on level
// min(t_c, t_row) + 1, along the row when t_c < t_row or t_c = t_row with the
// row later in the order than d_row, else along d_row.  W lanes take a unit.
template <typename T, uint32_t W, int J, bool N>
__device__ __forceinline__ void est_unit(const T* __restrict__ x, const EstGeom& g, int pos_last,
                                         const EstUnit& un, T eb, T inv2eb, uint32_t R,
                                         unsigned long long* sh, uint64_t& acc1l, uint64_t& acc1c,
                                         uint64_t& acc2l, uint64_t& acc2c) {
  const uint32_t ncol = (uint32_t)g.dims[g.ndim - 1];
  const uint32_t base = un.base, rem = un.c1 - un.c0;
  EstStencil<T> se[J], so[J];
  if (un.trow == 0) {
    // (uniform) stencils along d_row at step 1 share the row's neighbour
    // rows: their presence and offsets are the same in every lane (lanes
    // without a point read a point of the unit and are not counted)
    const uint32_t q = un.qrow, sr = un.srow, nr = un.nrow;
    const bool ha = q >= 3, hc = nr - q > 1, he = hc && nr - q > 3;
    const uint32_t ob = base - sr, oc = hc ? base + sr : base, oa = ha ? base - 3 * sr : base;
    const uint32_t oe = he ? base + 3 * sr : base;
#pragma unroll
    for (int j = 0; j < J; j++) {
      const uint32_t o = 2 * (threadIdx.x % W + j * W);
      const bool has_even = o < rem, has_odd = o + 1 < rem;
      const uint32_t ce = has_even ? un.c0 + o : un.c0, co = has_odd ? ce + 1 : ce;
      EstStencil<T>& e = se[j];
      e.ha = ha;
      e.hc = hc;
      e.he = he;
      e.x = est_ld<N>(x, base + ce);
      e.b = est_ld<N>(x, ob + ce);
      e.c = est_ld<N>(x, oc + ce);
      e.a = est_ld<N>(x, oa + ce);
      e.e = est_ld<N>(x, oe + ce);
      if (un.odd_along_row) {
        so[j] = est_odd_row_fetch<N>(x, base, ce, co, has_odd, un.c0, un.c1, ncol);
      } else {
        EstStencil<T>& d = so[j];
        d.ha = ha;
        d.hc = hc;
        d.he = he;
        d.x = est_ld<N>(x, base + co);
        d.b = est_ld<N>(x, ob + co);
        d.c = est_ld<N>(x, oc + co);
        d.a = est_ld<N>(x, oa + co);
        d.e = est_ld<N>(x, oe + co);
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < J; j++) {
      const uint32_t o = 2 * (threadIdx.x % W + j * W);
      const bool has_even = o < rem, has_odd = o + 1 < rem;
      const uint32_t ce = has_even ? un.c0 + o : un.c0, co = has_odd ? ce + 1 : ce;
      const int tc = ce ? __builtin_ctz(ce) : 64;
      const int t = tc < un.trow ? tc : un.trow;
      const bool e_row = tc < un.trow || (tc == un.trow && pos_last > un.prow);
      const uint32_t sp = has_even && t != 64 ? 1u << t : 0u;
      se[j] = est_fetch<N>(x, base + ce, e_row ? ce : un.qrow, e_row ? ncol : un.nrow, sp,
                           e_row ? sp : sp * un.srow);
      // (t_row > 0: the odd column along the row)
      so[j] = est_odd_row_fetch<N>(x, base, ce, co, has_odd, un.c0, un.c1, ncol);
    }
  }
  uint32_t s1l = 0, s1c = 0, s2l = 0, s2c = 0;
#pragma unroll
  for (int j = 0; j < J; j++) {
    const uint32_t o = 2 * (threadIdx.x % W + j * W);
    const bool has_even = o < rem, has_odd = o + 1 < rem;
    const uint32_t ce = has_even ? un.c0 + o : un.c0;
    if (un.odd_along_row) est_odd_row_finish(so[j], se[j].x, ce, un.c0, un.c1);
    uint32_t cl, cc;
    est_eval(so[j], eb, inv2eb, R, cl, cc);
    if (has_odd) {
      s1l += cl;
      s1c += cc;
    }
    est_eval(se[j], eb, inv2eb, R, cl, cc);
    if (un.trow == 0) {  // (uniform) level 1
      if (has_even) {
        s1l += cl;
        s1c += cc;
      }
      continue;
    }
    const int tc = ce ? __builtin_ctz(ce) : 64;
    const int t = tc < un.trow ? tc : un.trow;
    if (has_even && t != 64) {
      if (t == 1) {
        s2l += cl;
        s2c += cc;
      } else {
        atomicAdd(&sh[2 * t], (unsigned long long)cl);
        atomicAdd(&sh[2 * t + 1], (unsigned long long)cc);
      }
    }
  }
  acc1l += s1l;
  acc1c += s1c;
  acc2l += s2l;
  acc2c += s2c;
}

// The block's sums into cost: levels 1 and 2 from every lane's accumulators,
// the coarser levels from the block's table.
__device__ __forceinline__ void est_flush(uint64_t acc1l, uint64_t acc1c, uint64_t acc2l,
                                          uint64_t acc2c, unsigned long long* sh,
                                          unsigned long long* cost) {
  const uint32_t lane = threadIdx.x & 63;
  uint64_t v[4] = {acc1l, acc1c, acc2l, acc2c};
#pragma unroll
  for (int k = 0; k < 4; k++) {
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    if (lane == 0 && v[k]) atomicAdd(&sh[k], (unsigned long long)v[k]);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < 2 * kMaxLevels; i += blockDim.x)
    if (sh[i]) atomicAdd(cost + i, sh[i]);
}

template <typename T, int J, bool N>
__global__ __launch_bounds__(kEstThreads) void k_estimate(const T* __restrict__ x, EstGeom g,
                                                          const uint8_t* __restrict__ pos_dev,
                                                          const Meta* __restrict__ m, uint32_t R,
                                                          unsigned long long* cost) {
  __shared__ unsigned long long sh[2 * kMaxLevels];
  for (uint32_t i = threadIdx.x; i < 2 * kMaxLevels; i += kEstThreads) sh[i] = 0;
  __syncthreads();
  const T eb = (T)m->eb, inv2eb = (T)m->inv2eb;
  const int last = g.ndim - 1;
  uint8_t pos[kMaxDims];  // the order's places: the argument's, or the device's choice
#pragma unroll
  for (int e = 0; e < kMaxDims; e++) pos[e] = pos_dev ? pos_dev[e] : g.pos[e];
  uint64_t acc1l = 0, acc1c = 0, acc2l = 0, acc2c = 0;  // levels 1 and 2
  // every wave takes its own contiguous run of units; the waves of one XCD
  // (workgroup b on XCD b mod 8) take runs of one contiguous eighth, so the
  // rows and planes the stencils reach are read by waves of the same XCD at
  // about the same time
  const uint32_t nx = gridDim.x % 8 == 0 ? 8 : 1;
  const uint32_t wpb = kEstThreads / kEstWave;
  const uint64_t gw = ((uint64_t)(blockIdx.x % nx) * (gridDim.x / nx) + blockIdx.x / nx) * wpb +
                      threadIdx.x / kEstWave;
  const uint64_t nw = (uint64_t)gridDim.x * wpb;
  const uint64_t u0 = g.units * gw / nw, u1 = g.units * (gw + 1) / nw;
  if (u0 < u1) {
    // (wave-uniform; loops unrolled so the geometry stays in scalar
    // registers) the first unit as (row, segment), the row as coordinates
    // q[0..last-1]; then advanced a unit at a time with carries
    uint64_t row = u0 / g.segs;
    uint32_t seg = (uint32_t)(u0 - row * g.segs);
    uint32_t q[kMaxDims] = {0, 0, 0, 0};
    {
      uint64_t r = row;
#pragma unroll
      for (int e = kMaxDims - 2; e >= 0; --e) {
        if (e < last) {
          q[e] = (uint32_t)(r % g.dims[e]);
          r /= g.dims[e];
        }
      }
    }
    for (uint64_t u = u0; u < u1; u++) {
      if (g.sampled == 0 || (g.sampled == 1) == est_row_sampled(row)) {
        const EstUnit un = est_unit_at<kEstWave, J>(g, pos, q, seg);
        est_unit<T, kEstWave, J, N>(x, g, pos[last], un, eb, inv2eb, R, sh, acc1l, acc1c, acc2l,
                                    acc2c);
      }
      if (++seg == g.segs) {
        seg = 0;
        row++;
#pragma unroll
        for (int e = kMaxDims - 2; e >= 0; --e) {
          if (e < last) {
            if (++q[e] < (uint32_t)g.dims[e]) break;
            q[e] = 0;
          }
        }
      }
    }
  }
  est_flush(acc1l, acc1c, acc2l, acc2c, sh, cost);
}

// The sampled estimate of every dimension order in one launch: blockIdx.y
// is the order (its positions in pos[y], its sums at cost + y * per), and
// the units are those of the sampled rows only (rows[], ascending row
// indices), dealt evenly to the blocks.
struct EstOrders {
  uint8_t pos[kMaxOrders][kMaxDims];
};
template <typename T, int J>
__global__ __launch_bounds__(kEstThreads) void k_estimate_orders(const T* __restrict__ x, EstGeom g,
                                                                 EstOrders o,
                                                                 const uint32_t* __restrict__ rows,
                                                                 uint64_t nrows,
                                                                 const Meta* __restrict__ m,
                                                                 uint32_t R, uint64_t per,
                                                                 unsigned long long* cost) {
  __shared__ unsigned long long sh[2 * kMaxLevels];
  for (uint32_t i = threadIdx.x; i < 2 * kMaxLevels; i += kEstThreads) sh[i] = 0;
  __syncthreads();
  const T eb = (T)m->eb, inv2eb = (T)m->inv2eb;
  const int last = g.ndim - 1;
  uint8_t pos[kMaxDims];
#pragma unroll
  for (int e = 0; e < kMaxDims; e++) pos[e] = o.pos[blockIdx.y][e];
  uint64_t acc1l = 0, acc1c = 0, acc2l = 0, acc2c = 0;
  const uint64_t units = nrows * g.segs;
  for (uint64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const uint32_t seg = (uint32_t)(u % g.segs);
    uint64_t r = rows[u / g.segs];
    uint32_t q[kMaxDims] = {0, 0, 0, 0};
#pragma unroll
    for (int e = kMaxDims - 2; e >= 0; --e) {
      if (e < last) {
        q[e] = (uint32_t)(r % g.dims[e]);
        r /= g.dims[e];
      }
    }
    const EstUnit un = est_unit_at<kEstThreads, J>(g, pos, q, seg);
    est_unit<T, kEstThreads, J, false>(x, g, pos[last], un, eb, inv2eb, R, sh, acc1l, acc1c, acc2l,
                                       acc2c);
  }
  est_flush(acc1l, acc1c, acc2l, acc2c, sh, cost + blockIdx.y * per);
}

hipError_t launch_estimate(const void* x, int dtype, const EstGeom& g, const Meta* m,
                           uint32_t radius, uint64_t* cost, hipStream_t st, const uint8_t* pos_dev) {
  if (g.units == 0) return hipSuccess;
  // units of one wave, up to two pairs a lane: a unit is up to 256 columns,
  // whose geometry one wave works out for all of them (four pairs a lane,
  // fewer waves of more registers, ran 3 % slower)
  EstGeom w = g;
  const uint64_t ncol = g.dims[g.ndim - 1];
  w.pairs = ncol <= 2 * kEstWave ? 1 : 2;
  w.segs = (ncol + 2 * kEstWave * w.pairs - 1) / (2 * kEstWave * w.pairs);
  w.units = g.units / g.segs * w.segs;
  const uint64_t wpb = kEstThreads / kEstWave, nb = (w.units + wpb - 1) / wpb;
  dim3 grid((unsigned)(nb < kEstWaveBlocks ? nb : kEstWaveBlocks)), block(kEstThreads);
  auto* c = reinterpret_cast<unsigned long long*>(cost);
  // (32-bit byte offsets when the field is under 4 GiB)
  const uint64_t bytes = g.stride[0] * g.dims[0] * (dtype == SZ_F32 ? 4 : 8);
  const bool narrow = bytes <= 0xFFFFFFFFull;
#define SZG_EST2(T, J, N)                                                                    \
  hipLaunchKernelGGL((k_estimate<T, J, N>), grid, block, 0, st, (const T*)x, w, pos_dev, m, radius, \
                     c)
#define SZG_EST(J)                  \
  do {                              \
    if (dtype == SZ_F32) {          \
      if (narrow)                   \
        SZG_EST2(float, J, true);   \
      else                          \
        SZG_EST2(float, J, false);  \
    } else {                        \
      if (narrow)                   \
        SZG_EST2(double, J, true);  \
      else                          \
        SZG_EST2(double, J, false); \
    }                               \
  } while (0)
  if (w.pairs == 1)
    SZG_EST(1);
  else
    SZG_EST(2);
#undef SZG_EST2
#undef SZG_EST
  return hipGetLastError();
}

// The sampled estimate of every dimension order at once (fields of up to
// three dimensions).  A point p of level t (every coordinate a multiple of
// s = 2^t, at least one an odd multiple) is visited, under a dimension order,
// by the pass of the candidate dimension (coordinate an odd multiple of s)
// that comes last in that order; its stencil along a dimension does not
// depend on the order.  So every point is priced once along each of its
// candidate dimensions, into the bucket (t, candidate set C, dimension d),
// and an order's cost sum for level t + 1 is the sum over C of the bucket of
// C's last dimension in that order (combined on the device by
// k_choose_order).
//
// A row's class is (t_row, R): t_row the fewest trailing zeros among its
// coordinates other than the column, R the dimensions that have them.  A
// column c with t_c trailing zeros holds a point of t = min(t_c, t_row); its
// candidates are the column when t_c <= t_row and R when t_row <= t_c.  So a
// point's buckets are (t_c, {last}) when t_c < t_row (summed over the block
// by level), (t_row, R + {last}) when t_c = t_row and (t_row, R) when
// t_c > t_row (summed by lane while the class repeats: the listed rows come
// grouped by class, and a wave takes a contiguous run of them).
constexpr uint32_t kCandBlocks = 2048;  // most workgroups of the launch
__host__ __device__ inline uint32_t cand_bucket(uint32_t t, uint32_t C, uint32_t d) {
  return ((t * 8 + C) * 3 + d) * 2;
}
__device__ __forceinline__ void cand_add(unsigned long long* sh, uint32_t b, uint64_t l, uint64_t c) {
  const uint32_t lane = threadIdx.x & 63;
  for (int o = 32; o > 0; o >>= 1) {
    l += __shfl_xor(l, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  if (lane == 0) {
    if (l) atomicAdd(&sh[b], (unsigned long long)l);
    if (c) atomicAdd(&sh[b + 1], (unsigned long long)c);
  }
}
// A row class's lane sums: B along R + {last} (index last for the column),
// Q along R.
struct CandSums {
  uint64_t bl[3], bc[3], ql[2], qc[2];
};
__device__ __forceinline__ void cand_flush(unsigned long long* sh, CandSums& a, uint32_t tr,
                                           uint32_t rmask, int last) {
#pragma unroll
  for (int d = 0; d < 3; d++) {
    if (d <= last && (d == last || ((rmask >> d) & 1u)))
      cand_add(sh, cand_bucket(tr, rmask | (1u << last), (uint32_t)d), a.bl[d], a.bc[d]);
    if (d < 2 && d < last && ((rmask >> d) & 1u))
      cand_add(sh, cand_bucket(tr, rmask, (uint32_t)d), a.ql[d], a.qc[d]);
  }
#pragma unroll
  for (int d = 0; d < 3; d++) a.bl[d] = a.bc[d] = 0;
  a.ql[0] = a.qc[0] = a.ql[1] = a.qc[1] = 0;
}
template <typename T, int J, bool N>
__global__ __launch_bounds__(kEstThreads) void k_estimate_cand(const T* __restrict__ x, EstGeom g,
                                                               const uint32_t* __restrict__ rows,
                                                               uint64_t nrows,
                                                               const Meta* __restrict__ m,
                                                               uint32_t R, unsigned long long* bucket) {
  constexpr uint32_t kSeg = 2 * kEstWave * J;  // columns per unit (one wave's)
  __shared__ unsigned long long sh[kCandBuckets];
  for (uint32_t i = threadIdx.x; i < kCandBuckets; i += kEstThreads) sh[i] = 0;
  __syncthreads();
  const T eb = (T)m->eb, inv2eb = (T)m->inv2eb;
  const int last = g.ndim - 1;
  const uint32_t ncol = (uint32_t)g.dims[last];
  uint64_t a0l = 0, a0c = 0, a1l = 0, a1c = 0;  // t_c < t_row, levels 1 and 2
  CandSums sums = {};
  uint32_t held_t = 64, held_r = 0;  // the class sums holds (none yet)
  // every wave takes its own contiguous run of units
  const uint64_t wpb = kEstThreads / kEstWave, nw = (uint64_t)gridDim.x * wpb;
  const uint64_t gw = (uint64_t)blockIdx.x * wpb + threadIdx.x / kEstWave;
  const uint64_t units = nrows * g.segs;
  const uint64_t u0 = units * gw / nw, u1 = units * (gw + 1) / nw;
  for (uint64_t u = u0; u < u1; u++) {
    // (wave-uniform) the unit's row, its coordinates and class
    const uint64_t k = u / g.segs;
    const uint32_t seg = (uint32_t)(u - k * g.segs);
    if (!rows && !est_row_sampled(k)) continue;  // (no list: every row, the sampled ones taken)
    uint64_t r = rows ? rows[k] : k;
    const uint32_t base = (uint32_t)(r * ncol);
    uint32_t q[2] = {0, 0};
#pragma unroll
    for (int e = 1; e >= 0; --e) {
      if (e < last) {
        q[e] = (uint32_t)(r % g.dims[e]);
        r /= g.dims[e];
      }
    }
    uint32_t tr = 64, rmask = 0;
#pragma unroll
    for (int e = 0; e < 2; e++) {
      const uint32_t te = e < last && q[e] ? (uint32_t)__builtin_ctz(q[e]) : 64u;
      if (te < tr) {
        tr = te;
        rmask = 1u << e;
      } else if (te == tr && te != 64) {
        rmask |= 1u << e;
      }
    }
    if (tr != 64 && (tr != held_t || rmask != held_r)) {
      if (held_t != 64) cand_flush(sh, sums, held_t, held_r, last);
      held_t = tr;
      held_r = rmask;
    }
    const uint32_t c0 = seg * kSeg;
    const uint32_t c1 = ncol - c0 > kSeg ? c0 + kSeg : ncol;
    uint32_t s0l = 0, s0c = 0, s1l = 0, s1c = 0;  // this unit's level 1 and 2 sums
    uint32_t ubl[3] = {0, 0, 0}, ubc[3] = {0, 0, 0}, uql[2] = {0, 0}, uqc[2] = {0, 0};
#pragma unroll
    for (int j = 0; j < J; j++) {
      const uint32_t o = 2 * (threadIdx.x % kEstWave + j * kEstWave);
      const uint64_t ce64 = (uint64_t)c0 + o;
      const bool has_even = ce64 < c1, has_odd = ce64 + 1 < c1;
      const uint32_t ce = has_even ? (uint32_t)ce64 : c0, co = has_odd ? ce + 1 : ce;
      const uint32_t tc = ce ? (uint32_t)__builtin_ctz(ce) : 64u;
      // the even column along the row (t_c <= t_row, not the origin) and
      // along R (t_row <= t_c); the odd one along the row, and along R when
      // t_row = 0 -- every load issued before any is used
      const bool e_row = has_even && tc <= tr && tc != 64;
      const bool e_cand = has_even && tr <= tc && tr != 64;
      const uint32_t sr = e_row ? 1u << tc : 0u, sc = e_cand ? 1u << tr : 0u;
      const T xe = est_ld<N>(x, base + ce);
      EstStencil<T> so = est_odd_row_fetch<N>(x, base, ce, co, has_odd, c0, c1, ncol);
      EstStencil<T> ev_row{}, ev_d[2], od_d[2];
      if (tr != 0) ev_row = est_fetch<N>(x, base + ce, ce, ncol, sr, sr);
#pragma unroll
      for (int e = 0; e < 2; e++) {
        if (e < last && ((rmask >> e) & 1u)) {
          ev_d[e] = est_fetch<N>(x, base + ce, q[e], (uint32_t)g.dims[e], sc, sc * (uint32_t)g.stride[e]);
          if (tr == 0)
            od_d[e] = est_fetch<N>(x, base + co, q[e], (uint32_t)g.dims[e], has_odd ? 1u : 0u,
                                has_odd ? (uint32_t)g.stride[e] : 0u);
        }
      }
      est_odd_row_finish(so, xe, ce, c0, c1);
      uint32_t cl, cc;
      est_eval(so, eb, inv2eb, R, cl, cc);
      if (has_odd) {
        if (tr == 0) {
          ubl[last] += cl;
          ubc[last] += cc;
        } else {
          s0l += cl;
          s0c += cc;
        }
      }
      if (tr != 0) {
        est_eval(ev_row, eb, inv2eb, R, cl, cc);
        if (e_row) {
          if (tc == tr) {
            ubl[last] += cl;
            ubc[last] += cc;
          } else if (tc == 1) {
            s1l += cl;
            s1c += cc;
          } else {
            const uint32_t b = cand_bucket(tc, 1u << last, (uint32_t)last);
            atomicAdd(&sh[b], (unsigned long long)cl);
            atomicAdd(&sh[b + 1], (unsigned long long)cc);
          }
        }
      }
#pragma unroll
      for (int e = 0; e < 2; e++) {
        if (e < last && ((rmask >> e) & 1u)) {
          est_eval(ev_d[e], eb, inv2eb, R, cl, cc);
          if (e_cand) {
            if (tc == tr) {
              ubl[e] += cl;
              ubc[e] += cc;
            } else {
              uql[e] += cl;
              uqc[e] += cc;
            }
          }
          if (tr == 0) {
            est_eval(od_d[e], eb, inv2eb, R, cl, cc);
            if (has_odd) {
              ubl[e] += cl;
              ubc[e] += cc;
            }
          }
        }
      }
    }
    a0l += s0l;
    a0c += s0c;
    a1l += s1l;
    a1c += s1c;
#pragma unroll
    for (int d = 0; d < 3; d++) {
      sums.bl[d] += ubl[d];
      sums.bc[d] += ubc[d];
    }
    sums.ql[0] += uql[0];
    sums.qc[0] += uqc[0];
    sums.ql[1] += uql[1];
    sums.qc[1] += uqc[1];
  }
  if (held_t != 64) cand_flush(sh, sums, held_t, held_r, last);
  cand_add(sh, cand_bucket(0, 1u << last, (uint32_t)last), a0l, a0c);
  cand_add(sh, cand_bucket(1, 1u << last, (uint32_t)last), a1l, a1c);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kCandBuckets; i += kEstThreads)
    if (sh[i]) atomicAdd(bucket + i, sh[i]);
}

hipError_t launch_estimate_cand(const void* x, int dtype, const EstGeom& g, const uint32_t* rows,
                                uint64_t nrows, const Meta* m, uint32_t radius, uint64_t* bucket,
                                hipStream_t st) {
  if (g.ndim < 2 || g.ndim > 3) return hipErrorInvalidValue;
  // units of one wave, up to four pairs a lane (as the full estimate's)
  EstGeom w = g;
  const uint64_t ncol = g.dims[g.ndim - 1];
  w.pairs = ncol <= 2 * kEstWave ? 1 : ncol <= 4 * kEstWave ? 2 : 4;
  w.segs = (ncol + 2 * kEstWave * w.pairs - 1) / (2 * kEstWave * w.pairs);
  const uint64_t units = nrows * w.segs, wpb = kEstThreads / kEstWave;
  if (units == 0) return hipSuccess;
  const uint64_t nb = (units + wpb - 1) / wpb;
  dim3 grid((unsigned)(nb < kCandBlocks ? nb : kCandBlocks)), block(kEstThreads);
  auto* c = reinterpret_cast<unsigned long long*>(bucket);
  const uint64_t bytes = g.stride[0] * g.dims[0] * (dtype == SZ_F32 ? 4 : 8);
  const bool narrow = bytes <= 0xFFFFFFFFull;
#define SZG_CAND2(T, J, N)                                                                   \
  hipLaunchKernelGGL((k_estimate_cand<T, J, N>), grid, block, 0, st, (const T*)x, w, rows, nrows, \
                     m, radius, c)
#define SZG_CAND(J)                  \
  do {                               \
    if (dtype == SZ_F32) {           \
      if (narrow)                    \
        SZG_CAND2(float, J, true);   \
      else                           \
        SZG_CAND2(float, J, false);  \
    } else {                         \
      if (narrow)                    \
        SZG_CAND2(double, J, true);  \
      else                           \
        SZG_CAND2(double, J, false); \
    }                                \
  } while (0)
  if (w.pairs == 1)
    SZG_CAND(1);
  else if (w.pairs == 2)
    SZG_CAND(2);
  else
    SZG_CAND(4);
#undef SZG_CAND2
#undef SZG_CAND
  return hipGetLastError();
}

// The class of a row (its coordinates other than the column): the listed
// rows are grouped by it, so that a workgroup's run of rows changes class
// rarely.
uint32_t cand_row_class(int ndim, const uint64_t* dims, uint64_t r) {
  uint32_t tr = 64, rmask = 0;
  for (int e = ndim - 2; e >= 0; --e) {
    const uint64_t qe = r % dims[e];
    r /= dims[e];
    const uint32_t te = qe ? (uint32_t)__builtin_ctzll(qe) : 64u;
    if (te < tr) {
      tr = te;
      rmask = 1u << e;
    } else if (te == tr && te != 64) {
      rmask |= 1u << e;
    }
  }
  return tr * 8 + rmask;
}

// An order's cost sums from the buckets: level t + 1 gathers, for every
// candidate set C, the bucket of C's dimension that comes last in the order.
__device__ __forceinline__ void cand_level(const uint64_t* bucket, int ndim, const uint8_t* pos,
                                           uint32_t t, uint64_t& l, uint64_t& c) {
  l = c = 0;
  for (uint32_t C = 1; C < (1u << ndim); C++) {
    int best = -1;
    for (int d = 0; d < ndim; d++)
      if (((C >> d) & 1u) && (best < 0 || pos[d] > pos[best])) best = d;
    const uint32_t b = cand_bucket(t, C, (uint32_t)best);
    l += bucket[b];
    c += bucket[b + 1];
  }
}

// The order choice on the device: every order's sum over levels 1..L of its
// cheaper cost sum, the least first in the list (orders[k]: the place of
// each dimension); chosen[0] the index, chosen[1..] its places.  With lvl
// non-null, the chosen order's sums over the sampled rows go to lvl (2 per
// level, every level), so that the full estimate need only add the others.
__global__ __launch_bounds__(256) void k_choose_order(const uint64_t* __restrict__ bucket_g, int ndim,
                                                      EstOrders o, uint32_t norders, int L,
                                                      uint8_t* chosen, uint64_t* lvl) {
  __shared__ uint64_t bucket[kCandBuckets];
  __shared__ unsigned long long total[kMaxOrders];
  for (uint32_t i = threadIdx.x; i < kCandBuckets; i += blockDim.x) bucket[i] = bucket_g[i];
  for (uint32_t i = threadIdx.x; i < kMaxOrders; i += blockDim.x) total[i] = 0;
  __syncthreads();
  // a lane per (order, level)
  for (uint32_t i = threadIdx.x; i < norders * (uint32_t)L; i += blockDim.x) {
    const uint32_t k = i / (uint32_t)L, t = i % (uint32_t)L;
    uint64_t l, c;
    cand_level(bucket, ndim, o.pos[k], t, l, c);
    atomicAdd(&total[k], (unsigned long long)(c < l ? c : l));
  }
  __syncthreads();
  __shared__ uint32_t sbi;
  if (threadIdx.x == 0) {
    uint64_t best = ~0ull;
    uint32_t bi = 0;
    for (uint32_t k = 0; k < norders; k++) {
      if (total[k] < best) {
        best = total[k];
        bi = k;
      }
    }
    chosen[0] = (uint8_t)bi;
    for (int d = 0; d < kMaxDims; d++) chosen[1 + d] = o.pos[bi][d];
    sbi = bi;
  }
  __syncthreads();
  if (lvl && threadIdx.x < (uint32_t)kMaxLevels)
    cand_level(bucket, ndim, o.pos[sbi], threadIdx.x, lvl[2 * threadIdx.x], lvl[2 * threadIdx.x + 1]);
}

hipError_t launch_choose_order(const uint64_t* bucket, int ndim, const uint8_t (*orders)[kMaxDims],
                               uint32_t norders, int levels, uint8_t* chosen, uint64_t* lvl,
                               hipStream_t st) {
  if (norders == 0 || norders > (uint32_t)kMaxOrders || ndim < 1 || ndim > 3)
    return hipErrorInvalidValue;
  EstOrders o{};
  for (uint32_t k = 0; k < norders; k++)
    for (int d = 0; d < kMaxDims; d++) o.pos[k][d] = orders[k][d];
  hipLaunchKernelGGL(k_choose_order, dim3(1), dim3(256), 0, st, bucket, ndim, o, norders, levels,
                     chosen, lvl);
  return hipGetLastError();
}

hipError_t launch_estimate_orders(const void* x, int dtype, const EstGeom& g,
                                  const uint8_t (*orders)[kMaxDims], uint32_t norders,
                                  const uint32_t* rows, uint64_t nrows, const Meta* m,
                                  uint32_t radius, uint64_t per, uint64_t* cost, hipStream_t st) {
  const uint64_t units = nrows * g.segs;
  if (units == 0 || norders == 0) return hipSuccess;
  if (norders > (uint32_t)kMaxOrders) return hipErrorInvalidValue;
  EstOrders o{};
  for (uint32_t k = 0; k < norders; k++)
    for (int e = 0; e < kMaxDims; e++) o.pos[k][e] = orders[k][e];
  const uint64_t bx = std::min<uint64_t>(units, std::max<uint64_t>(64, kEstBlocks / norders));
  dim3 grid((unsigned)bx, norders), block(kEstThreads);
  auto* c = reinterpret_cast<unsigned long long*>(cost);
#define SZG_ESTO(J)                                                                               \
  do {                                                                                            \
    if (dtype == SZ_F32)                                                                          \
      hipLaunchKernelGGL((k_estimate_orders<float, J>), grid, block, 0, st, (const float*)x, g, o, \
                         rows, nrows, m, radius, per, c);                                         \
    else                                                                                          \
      hipLaunchKernelGGL((k_estimate_orders<double, J>), grid, block, 0, st, (const double*)x, g,  \
                         o, rows, nrows, m, radius, per, c);                                      \
  } while (0)
  if (g.pairs == 1)
    SZG_ESTO(1);
  else if (g.pairs == 2)
    SZG_ESTO(2);
  else
    SZG_ESTO(4);
#undef SZG_ESTO
  return hipGetLastError();
}

// Units of 512, 1024 or 2048 columns (one, two or four column pairs a lane),
// the smallest that holds a row when one does.
EstGeom make_estimate_geom(int ndim, const uint64_t* dims, const uint8_t* order) {
  EstGeom g{};
  g.ndim = ndim;
  uint64_t st = 1;
  for (int e = ndim - 1; e >= 0; e--) {
    g.dims[e] = dims[e];
    g.stride[e] = st;
    st *= dims[e];
  }
  for (int j = 0; j < ndim; j++) g.pos[order[j]] = (uint8_t)j;
  const uint64_t ncol = dims[ndim - 1];
  g.pairs = ncol <= 2 * kEstThreads ? 1 : ncol <= 4 * kEstThreads ? 2 : 4;
  const uint64_t seg = 2ull * kEstThreads * g.pairs;
  g.segs = ncol ? (ncol + seg - 1) / seg : 0;
  g.units = ncol ? st / ncol * g.segs : 0;
  return g;
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


// ------------------------------------------------------------------ batches
// The same stages for every field of a batch in one launch (batch.hip).

__global__ void k_b_meta_init(const BField* __restrict__ f, uint32_t nf) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nf) meta_init(f[i].m);
}

hipError_t launch_b_meta_init(const BField* f, uint32_t nf, hipStream_t st) {
  if (nf == 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_meta_init, dim3((nf + 255) / 256), dim3(256), 0, st, f, nf);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_b_minmax(BLaunch L) {
  BJob j;
  uint32_t local;
  if (!batch_job(L, j, local)) return;
  const BField& f = L.f[j.field];
  minmax_body<T>(static_cast<const T*>(f.x), f.n, f.m, local, j.nblk, nullptr);
}

hipError_t launch_b_minmax(int dtype, BLaunch L, uint32_t nwg, hipStream_t st) {
  if (nwg == 0) return hipSuccess;
  if (dtype == SZ_F32)
    hipLaunchKernelGGL(k_b_minmax<float>, dim3(nwg), dim3(256), 0, st, L);
  else
    hipLaunchKernelGGL(k_b_minmax<double>, dim3(nwg), dim3(256), 0, st, L);
  return hipGetLastError();
}

__global__ void k_b_resolve_eb(const BField* __restrict__ f, uint32_t nf) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  if (f[i].dtype == SZ_F32)
    resolve_eb<float>(f[i].eb_mode, f[i].eb_value, f[i].m);
  else
    resolve_eb<double>(f[i].eb_mode, f[i].eb_value, f[i].m);
}

hipError_t launch_b_resolve_eb(const BField* f, uint32_t nf, hipStream_t st) {
  if (nf == 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_resolve_eb, dim3((nf + 255) / 256), dim3(256), 0, st, f, nf);
  return hipGetLastError();
}

// one workgroup per field: the origin and the coarsest levels
template <typename T>
__global__ __launch_bounds__(kSmallThreads) void k_b_small_levels(BLaunch L) {
  BJob j;
  uint32_t local;
  if (!batch_job(L, j, local)) return;
  const BField& f = L.f[j.field];
  small_levels_body<T, false>(static_cast<const T*>(f.x), static_cast<T*>(f.rec), f.codes, f.sg,
                              f.m, T(0), f.R);
}

hipError_t launch_b_small_levels(int dtype, BLaunch L, uint32_t nwg, hipStream_t st) {
  if (nwg == 0) return hipSuccess;
  if (dtype == SZ_F32)
    hipLaunchKernelGGL(k_b_small_levels<float>, dim3(nwg), dim3(kSmallThreads), 0, st, L);
  else
    hipLaunchKernelGGL(k_b_small_levels<double>, dim3(nwg), dim3(kSmallThreads), 0, st, L);
  return hipGetLastError();
}

}  // namespace szg
