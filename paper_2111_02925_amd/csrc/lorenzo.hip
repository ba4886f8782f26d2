// The first-order Lorenzo predictor on the device.
//
// Paper: SZ3 (arXiv 2111.02925), Section 3.2 "Predictor" (the Lorenzo
// predictor, which predicts a point from the decompressed values of its
// neighbours) and Section 6.2 (SZ3-LR pairs it with the same linear-scaling
// quantizer and Huffman encoder as SZ3-Interp).
//
// In N dimensions the prediction at q is the sum over the nonempty sets S of
// dimensions of (-1)^(|S|+1) x'(q - e_S), x' the reconstructed values, a
// neighbour outside the grid counting as 0.  The terms are taken as masks
// m = 1 .. 2^N - 1 in increasing order (bit e for dimension e, dimension 0
// the slowest), the m = 1 term first, then each next one added (|S| odd) or
// subtracted (|S| even).  Every reconstruction depends on the ones before it
// through the quantizer, so the points are ordered by wavefronts.
//
// The last three dimensions form a view (A, B, C), C contiguous (leading
// extents 1 for fewer dimensions); a 4-D field is walked one hyperplane
// (index along dimension 0) at a time, each reading the previous one.  The
// view is cut into blocks of BA x BB x BC points, and one launch handles the
// blocks of one block diagonal (bA + bB + bC fixed), whose lower neighbours
// are all finished.  In a block, lane (a, b) walks c, taking point (a, b, c)
// at step t = a + b + c, so each step's points depend only on earlier steps;
// the block's reconstructions live in LDS with a one-point halo on the low
// side of every dimension (the finished neighbours' values, or 0 outside
// the grid), so every term is one LDS read at a constant offset.
#include "common.h"
#include "device_math.h"

namespace szg {

struct LorGeom {
  uint32_t ext[3];  // extents of the view (A, B, C)
  uint64_t sA, sB;  // flat strides of A and B (C is contiguous)
  uint32_t nb[3];   // blocks along A, B, C
  uint32_t diag;    // this launch's block diagonal
  uint64_t off;     // flat offset of the hyperplane
  uint64_t prev;    // flat offset of the previous hyperplane (4-D)
  uint32_t has_prev;
};

// Block shapes: (16, 16, 16) for 3-D f32, (8, 16, 16) for 4-D and f64;
// (1, 256, 16) and (1, 128, 16) for 2-D; (1, 1, 1024) for 1-D.  LDS stays
// within 64 KB.
template <typename T, int N>
struct LorShape;
template <int N>
struct LorShape<float, N> {
  static constexpr int BA = N == 3 ? 16 : N == 4 ? 8 : 1, BB = N >= 3 ? 16 : N == 2 ? 256 : 1,
                       BC = N >= 2 ? 16 : 1024;
};
template <int N>
struct LorShape<double, N> {
  static constexpr int BA = N >= 3 ? 8 : 1, BB = N >= 3 ? 16 : N == 2 ? 128 : 1,
                       BC = N >= 2 ? 16 : 1024;
};

template <int BA, int BB>
struct LorThreads {
  static constexpr int value = BA * BB < 64 ? 64 : BA * BB;
};

template <typename T, int N, bool DEC>
__global__ __launch_bounds__((LorThreads<LorShape<T, N>::BA, LorShape<T, N>::BB>::value)) void
k_lorenzo(const T* __restrict__ x, const uint16_t* __restrict__ codes_in, uint16_t* codes_out,
          T* rec, LorGeom g, const Meta* __restrict__ m, T twoeb_dec, uint32_t R) {
  constexpr int BA = LorShape<T, N>::BA, BB = LorShape<T, N>::BB, BC = LorShape<T, N>::BC;
  constexpr int NT = LorThreads<BA, BB>::value;
  // LDS box with the halo; rows padded to BC + 2 so that the lanes of a step
  // (c = t - a - b) fall in different banks
  constexpr int HA = BA + 1, HB = BB + 1, HC = BC + 2;
  constexpr int NP = N == 4 ? HA * HB * HC : 1;
  __shared__ T Rs[HA * HB * HC];  // reconstructions, halo at index 0 of each dimension
  __shared__ T Ps[NP];            // 4-D: the previous hyperplane, same layout
  __shared__ T Xs[BA * BB * BC];  // inputs (compress) or verbatim values (decompress)
  __shared__ uint16_t Ks[BA * BB * BC];

  const uint32_t bA = blockIdx.x / g.nb[1], bB = blockIdx.x % g.nb[1];
  if (bA + bB > g.diag || g.diag - bA - bB >= g.nb[2]) return;  // (uniform) not on the diagonal
  const uint32_t bC = g.diag - bA - bB;
  const uint32_t a0 = bA * BA, b0 = bB * BB, c0 = bC * BC;
  const int ea = (int)min((uint32_t)BA, g.ext[0] - a0), eb = (int)min((uint32_t)BB, g.ext[1] - b0),
            ec = (int)min((uint32_t)BC, g.ext[2] - c0);
  const int tid = threadIdx.x;
  const T* __restrict__ hp = rec + g.off;  // this hyperplane's reconstructions

  // Fill: every position (ia, ib, ic) of the box with the halo, index 0 for
  // one step back.  A position with a 0 index is halo (the finished
  // neighbour's value, or 0 outside the grid); the others are the block's
  // points (input, or verbatim value and code).  Taken kUnroll positions a
  // lane at a time, loads first, so that they are in flight together.
  constexpr int WB = BB + 1, WC = BC + 1, BOX = (BA + 1) * WB * WC;
  constexpr int kUnroll = 8;
  for (int i0 = 0; i0 < BOX; i0 += kUnroll * NT) {
    T vr[kUnroll], vp[kUnroll];
    uint16_t vk[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; k++) {
      const int i = i0 + k * NT + tid;
      const int ic = i % WC, ib = (i / WC) % WB, ia = i / (WC * WB);
      const bool in_box = i < BOX && ia <= ea && ib <= eb && ic <= ec;
      const int64_t ga = (int64_t)a0 + ia - 1, gb = (int64_t)b0 + ib - 1,
                    gc = (int64_t)c0 + ic - 1;
      const bool inside = in_box && ga >= 0 && gb >= 0 && gc >= 0;
      const uint64_t f = inside ? (uint64_t)ga * g.sA + (uint64_t)gb * g.sB + (uint64_t)gc : 0;
      const bool halo = ia == 0 || ib == 0 || ic == 0;
      vr[k] = T(0);
      vk[k] = 0;
      if (inside) vr[k] = halo ? hp[f] : (DEC ? hp[f] : x[g.off + f]);
      if (DEC && inside && !halo) vk[k] = codes_in[g.off + f];
      vp[k] = T(0);
      if (N == 4 && inside && g.has_prev) vp[k] = rec[g.prev + f];
    }
#pragma unroll
    for (int k = 0; k < kUnroll; k++) {
      const int i = i0 + k * NT + tid;
      const int ic = i % WC, ib = (i / WC) % WB, ia = i / (WC * WB);
      if (!(i < BOX && ia <= ea && ib <= eb && ic <= ec)) continue;
      const int li = (ia * HB + ib) * HC + ic;
      if (ia == 0 || ib == 0 || ic == 0) {
        Rs[li] = vr[k];
      } else {
        const int xi = ((ia - 1) * BB + (ib - 1)) * BC + (ic - 1);
        Xs[xi] = vr[k];
        if (DEC) Ks[xi] = vk[k];
      }
      if (N == 4) Ps[li] = vp[k];
    }
  }
  __syncthreads();

  // compression: the bound resolved on the device; reconstruction: 2 eb
  // from the stream's header
  QuantParams<T> qp{};
  if (!DEC) qp = QuantParams<T>::from_meta(m, R);
  const int a = tid / BB, b = tid % BB;
  const bool lane = tid < BA * BB && a < ea && b < eb;
  for (int t = 0; t < ea + eb + ec - 2; t++) {
    const int c = t - a - b;
    if (lane && c >= 0 && c < ec) {
      const int li = ((a + 1) * HB + (b + 1)) * HC + (c + 1);
      // the terms in mask order; view dimension of real dimension e: N = 4
      // takes dimension 0 from the previous hyperplane
      T acc = T(0);
#pragma unroll
      for (int msk = 1; msk < (1 << N); msk++) {
        int dA = 0, dB = 0, dC = 0, dP = 0;
#pragma unroll
        for (int e = 0; e < N; e++) {
          if (!((msk >> e) & 1)) continue;
          const int v = e + 3 - N;  // view dimension: 0 A, 1 B, 2 C; -1 the hyperplane
          if (v == 0) dA = 1;
          if (v == 1) dB = 1;
          if (v == 2) dC = 1;
          if (v < 0) dP = 1;
        }
        const int o = li - (dA * HB + dB) * HC - dC;
        const T term = dP ? Ps[o] : Rs[o];
        if (msk == 1)
          acc = term;
        else if (__builtin_popcount(msk) & 1)
          acc = acc + term;
        else
          acc = acc - term;
      }
      const int xi = (a * BB + b) * BC + c;
      T r;
      if (DEC) {
        const uint32_t code = Ks[xi];
        r = code ? recover(acc, twoeb_dec, code, R) : Xs[xi];
      } else {
        Ks[xi] = (uint16_t)quantize(Xs[xi], acc, qp, r);
      }
      Rs[li] = r;
    }
    __syncthreads();
  }

  // the block's codes and reconstructions
  for (int i = tid; i < BA * BB * BC; i += NT) {
    const int c = i % BC, b = (i / BC) % BB, a = i / (BC * BB);
    if (a >= ea || b >= eb || c >= ec) continue;
    const uint64_t f =
        g.off + (uint64_t)(a0 + a) * g.sA + (uint64_t)(b0 + b) * g.sB + (uint64_t)(c0 + c);
    rec[f] = Rs[((a + 1) * HB + (b + 1)) * HC + (c + 1)];
    if (!DEC) codes_out[f] = Ks[i];
  }
}

namespace {

template <typename T, int N, bool DEC>
hipError_t lorenzo_run(const T* x, const uint16_t* codes_in, uint16_t* codes_out, T* rec,
                       int ndim, const uint64_t* dims, const Meta* m, T twoeb, uint32_t R,
                       hipStream_t st) {
  using S = LorShape<T, N>;
  constexpr int NT = LorThreads<S::BA, S::BB>::value;
  // the view: the last three dimensions, leading extents 1
  uint64_t v[3] = {1, 1, 1};
  for (int k = 0; k < 3 && k < ndim; k++) v[2 - k] = dims[ndim - 1 - k];
  const uint64_t hyper = ndim == 4 ? dims[0] : 1;
  LorGeom g{};
  for (int k = 0; k < 3; k++) g.ext[k] = (uint32_t)v[k];
  g.sB = v[2];
  g.sA = v[1] * v[2];
  g.nb[0] = (uint32_t)((v[0] + S::BA - 1) / S::BA);
  g.nb[1] = (uint32_t)((v[1] + S::BB - 1) / S::BB);
  g.nb[2] = (uint32_t)((v[2] + S::BC - 1) / S::BC);
  const uint64_t plane = v[0] * v[1] * v[2];
  const unsigned blocks = g.nb[0] * g.nb[1];
  for (uint64_t h = 0; h < hyper; h++) {
    g.off = h * plane;
    g.prev = h ? (h - 1) * plane : 0;
    g.has_prev = h ? 1u : 0u;
    for (uint32_t d = 0; d + 2 < g.nb[0] + g.nb[1] + g.nb[2]; d++) {
      g.diag = d;
      hipLaunchKernelGGL((k_lorenzo<T, N, DEC>), dim3(blocks), dim3(NT), 0, st, x, codes_in,
                         codes_out, rec, g, m, twoeb, R);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

template <typename T, bool DEC>
hipError_t lorenzo_dispatch(const T* x, const uint16_t* codes_in, uint16_t* codes_out, T* rec,
                            int ndim, const uint64_t* dims, const Meta* m, T twoeb, uint32_t R,
                            hipStream_t st) {
  switch (ndim) {
    case 1:
      return lorenzo_run<T, 1, DEC>(x, codes_in, codes_out, rec, ndim, dims, m, twoeb, R, st);
    case 2:
      return lorenzo_run<T, 2, DEC>(x, codes_in, codes_out, rec, ndim, dims, m, twoeb, R, st);
    case 3:
      return lorenzo_run<T, 3, DEC>(x, codes_in, codes_out, rec, ndim, dims, m, twoeb, R, st);
    default:
      return lorenzo_run<T, 4, DEC>(x, codes_in, codes_out, rec, ndim, dims, m, twoeb, R, st);
  }
}

}  // namespace

hipError_t launch_lorenzo_compress(const void* x, int dtype, void* rec, uint16_t* codes, int ndim,
                                   const uint64_t* dims, const Meta* m, uint32_t radius,
                                   hipStream_t st) {
  if (dtype == SZ_F32)
    return lorenzo_dispatch<float, false>((const float*)x, nullptr, codes, (float*)rec, ndim,
                                          dims, m, 0.0f, radius, st);
  return lorenzo_dispatch<double, false>((const double*)x, nullptr, codes, (double*)rec, ndim,
                                         dims, m, 0.0, radius, st);
}

hipError_t launch_lorenzo_recon(const uint16_t* codes, int dtype, void* out, int ndim,
                                const uint64_t* dims, double eb_t, uint32_t radius,
                                hipStream_t st) {
  if (dtype == SZ_F32)
    return lorenzo_dispatch<float, true>(nullptr, codes, nullptr, (float*)out, ndim, dims, nullptr,
                                         2.0f * (float)eb_t, radius, st);
  return lorenzo_dispatch<double, true>(nullptr, codes, nullptr, (double*)out, ndim, dims,
                                        nullptr, 2.0 * eb_t, radius, st);
}

}  // namespace szg
