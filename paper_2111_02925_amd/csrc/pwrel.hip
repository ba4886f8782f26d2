// Point-wise relative error bounds through a logarithmic preprocessor.
//
// Paper: SZ3 (arXiv 2111.02925), Section 3.1 (composing a pipeline from a
// preprocessor and the usual modules) and Section 3.2 "Preprocessor": a
// logarithmic transform turns a point-wise relative bound into an absolute
// one, the data being compressed in the logarithmic domain.
//
// Forward: y = log2|x| as a double field, compressed by the interpolation
// pipeline with the absolute bound delta = log2((1 + eps)/(1 + 4u)) (1 -
// 2^-20) - E, u the unit roundoff of the field type and E the largest
// rounding error of y over the type's normal values (2^-42 for doubles,
// 2^-45 for floats) plus 2^-50 for the rounding of the ratio; the sign bits
// are kept, a
// bit per value, when any is set.  Zeros and values below the smallest
// normal of T go to a level far below every normal value's logarithm and
// come back as signed zeros; infinities map to +inf and NaN to NaN (both
// unpredictable in the log field, hence stored verbatim).  Inverse: x' = +-
// 2^y', clamped to the largest finite T.  With |y - y'| <= delta the bound
// |x - x'| <= eps |x| holds for every normal x: the series below are within
// about one unit in the last place, and the margins in delta cover them, the
// absolute rounding of y at the largest exponents, and the final rounding to
// T.
//
// The two maps are evaluated from their series in a fixed order (no
// contraction), so that every implementation of the same definitions,
// including the one on the host, gives the same bits.
#include "common.h"

namespace szg {

constexpr double kSqrtHalf = 0.70710678118654752440;
constexpr double kInvLn2 = 1.4426950408889634074;
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kLogZero = -1100.0;      // level of zeros and subnormal values
constexpr double kLogZeroBelow = -1050.0; // reconstructed levels below it are zeros

// log2(a) for finite a > 0: a = m 2^e, m in [sqrt(1/2), sqrt(2)); ln m =
// 2 atanh(s), s = (m - 1)/(m + 1), by its Maclaurin series to s^29.
__host__ __device__ inline double pw_log2(double a) {
  int e;
  double m = frexp(a, &e);
  if (m < kSqrtHalf) {
    m = m * 2.0;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
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
  return (double)e + ln_m * kInvLn2;
}

// 2^y for finite |y| <= 1100: y = k + f, k = rint(y); 2^f = exp(f ln 2) by
// its Taylor series to t^18.
__host__ __device__ inline double pw_exp2(double y) {
  const double k = rint(y);
  const double t = (y - k) * kLn2;
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

// The log field's absolute bound: relative margins for the exponential and
// the rounding to T (4u) and for the series of the ratio's logarithm
// (1 - 2^-20); absolute margins for the rounding of y = log2|x| itself, half
// an ulp of |y| with |y| < 2048 for normal doubles (< 256 for floats): 2^-42
// (2^-45), and for the ratio's two roundings in double (below 2^-50).
// Bounds that leave no positive delta are rejected.
double pwrel_delta(double eps, int dtype) {
  if (!(eps > 0.0) || !(eps < 1.0)) return -1.0;
  const double u = dtype == SZ_F64 ? 0x1p-53 : 0x1p-24;
  const double e_abs = (dtype == SZ_F64 ? 0x1p-42 : 0x1p-45) + 0x1p-50;
  const double r = (1.0 + eps) / (1.0 + 4.0 * u);
  if (!(r > 1.0)) return -1.0;
  const double d = pw_log2(r) * (1.0 - 0x1p-20) - e_abs;
  return d > 0.0 ? d : -1.0;
}

template <typename T>
struct PwBits;
template <>
struct PwBits<float> {
  using U = uint32_t;
  static constexpr U kSign = 0x80000000u, kNaN = 0x7FC00000u;
  static constexpr double kMin = 0x1p-126, kMax = 0x1.fffffep+127;
};
template <>
struct PwBits<double> {
  using U = uint64_t;
  static constexpr U kSign = 0x8000000000000000ull, kNaN = 0x7FF8000000000000ull;
  static constexpr double kMin = 0x1p-1022, kMax = 0x1.fffffffffffffp+1023;
};

// y[i] from x[i]; the sign bits of 64 consecutive values form one word
// (lane l of a wave holds value 64 w + l); *any is set when a sign is.
template <typename T>
__global__ __launch_bounds__(256) void k_pwrel_forward(const T* __restrict__ x, double* y,
                                                       uint64_t* signs, uint64_t n,
                                                       uint32_t* any) {
  using B = PwBits<T>;
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t nw = (n + 63) / 64;
  const uint64_t wstride = (uint64_t)gridDim.x * (blockDim.x / 64);
  for (uint64_t w = blockIdx.x * (uint64_t)(blockDim.x / 64) + (threadIdx.x >> 6); w < nw;
       w += wstride) {
    const uint64_t i = 64 * w + lane;
    bool neg = false;
    if (i < n) {
      const T v = x[i];
      typename B::U bits;
      __builtin_memcpy(&bits, &v, sizeof(T));
      neg = (bits & B::kSign) != 0;
      const double a = __builtin_fabs((double)v);
      double r;
      if (__builtin_isnan(a)) {
        const uint64_t nan = 0x7FF8000000000000ull;
        __builtin_memcpy(&r, &nan, 8);
      } else if (__builtin_isinf(a)) {
        r = __builtin_inf();
      } else if (a < B::kMin) {
        r = kLogZero;
      } else {
        r = pw_log2(a);
      }
      y[i] = r;
    }
    const uint64_t word = __ballot(neg);
    if (lane == 0) {
      signs[w] = word;
      if (word) atomicOr(any, 1u);
    }
  }
}

// x'[i] = +- 2^y[i] in T (signs may be null: no sign set).
template <typename T>
__global__ __launch_bounds__(256) void k_pwrel_inverse(const double* __restrict__ y,
                                                       const uint64_t* __restrict__ signs,
                                                       uint64_t n, T* out) {
  using B = PwBits<T>;
  const uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += gs) {
    const double v = y[i];
    typename B::U bits;
    if (__builtin_isnan(v)) {
      bits = B::kNaN;
    } else {
      double r;
      if (v == __builtin_inf())
        r = __builtin_inf();
      else if (v < kLogZeroBelow)
        r = 0.0;
      else if (v > 1100.0)
        r = B::kMax;
      else {
        r = pw_exp2(v);
        if (r > B::kMax) r = B::kMax;
      }
      const T t = (T)r;
      __builtin_memcpy(&bits, &t, sizeof(T));
    }
    if (signs && ((signs[i / 64] >> (i % 64)) & 1ull)) bits |= B::kSign;
    __builtin_memcpy(out + i, &bits, sizeof(T));
  }
}

// The point-wise relative stream from the log stream already in `out`
// (ylen bytes): the sign section at off_signs (zero padding before it) and
// the header fields of the mode.
__global__ __launch_bounds__(256) void k_pwrel_finish(uint8_t* out, uint64_t ylen,
                                                      uint64_t off_signs,
                                                      const uint64_t* __restrict__ signs,
                                                      uint64_t nsw, uint64_t total, double eps,
                                                      uint32_t dtype) {
  const uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t gid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (off_signs) {
    for (uint64_t w = gid; w < nsw; w += gs)
      *reinterpret_cast<uint64_t*>(out + off_signs + 8 * w) = signs[w];
    for (uint64_t b = ylen + gid; b < off_signs; b += gs) out[b] = 0;
  }
  if (gid == 0) {
    out[45] = (uint8_t)SZ_EB_PWREL;
    uint64_t e;
    __builtin_memcpy(&e, &eps, 8);
    for (int k = 0; k < 8; k++) {
      out[48 + k] = (uint8_t)(e >> (8 * k));
      out[96 + k] = (uint8_t)(total >> (8 * k));
      out[112 + k] = (uint8_t)(off_signs >> (8 * k));
    }
    out[104] = (uint8_t)dtype;
    out[105] = off_signs ? 1 : 0;
  }
}

namespace {
unsigned pw_blocks(uint64_t items) {
  uint64_t b = (items + 255) / 256;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (unsigned)b;
}
}  // namespace

hipError_t launch_pwrel_forward(const void* x, int dtype, double* y, uint64_t* signs, uint64_t n,
                                uint32_t* any, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = pw_blocks((n + 63) / 64 * 64);
  if (dtype == SZ_F32)
    hipLaunchKernelGGL(k_pwrel_forward<float>, dim3(blocks), dim3(256), 0, st, (const float*)x, y,
                       signs, n, any);
  else
    hipLaunchKernelGGL(k_pwrel_forward<double>, dim3(blocks), dim3(256), 0, st, (const double*)x,
                       y, signs, n, any);
  return hipGetLastError();
}

hipError_t launch_pwrel_inverse(const double* y, const uint64_t* signs, uint64_t n, int dtype,
                                void* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = pw_blocks(n);
  if (dtype == SZ_F32)
    hipLaunchKernelGGL(k_pwrel_inverse<float>, dim3(blocks), dim3(256), 0, st, y, signs, n,
                       (float*)out);
  else
    hipLaunchKernelGGL(k_pwrel_inverse<double>, dim3(blocks), dim3(256), 0, st, y, signs, n,
                       (double*)out);
  return hipGetLastError();
}

hipError_t launch_pwrel_finish(uint8_t* out, uint64_t ylen, uint64_t off_signs,
                               const uint64_t* signs, uint64_t nsw, uint64_t total, double eps,
                               int dtype, hipStream_t st) {
  const unsigned blocks = pw_blocks(nsw > 64 ? nsw : 64);
  hipLaunchKernelGGL(k_pwrel_finish, dim3(blocks), dim3(256), 0, st, out, ylen, off_signs, signs,
                     nsw, total, eps, (uint32_t)dtype);
  return hipGetLastError();
}

}  // namespace szg
