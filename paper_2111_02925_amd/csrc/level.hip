// Fused level kernels: every pass of one level of the multilevel traversal in
// a single launch, for fields of up to three dimensions.
//
// Paper: SZ3 (arXiv 2111.02925), Section 6.2 (SZ3-Interp): the field is
// predicted level by level from the coarsest stride down to stride 1, and
// inside a level dimension by dimension, each point from already
// reconstructed neighbours along the current dimension; Algorithm 1 runs
// prediction and quantization point by point in that order.
//
// On the lattice of multiples of the level stride s (coordinates in units of
// s, dimensions taken in the pass order a, b, c), the level's points are:
//   pass along a: a odd, b even, c even
//   pass along b: a any, b odd,  c even
//   pass along c: a any, b any,  c odd
// and every stencil reaches +-1 and +-3 lattice units along its dimension.
// A workgroup owns a tile [A0,A1) x [B0,B1) x [C0,C1) and keeps in LDS a box
// that extends it by 3 units along b and c.  It loads the box's coarse points
// (all coordinates even, final from earlier levels), then computes the pass
// along a on the whole box, the pass along b on the box rows of its tile,
// and the pass along c on its tile, synchronising between passes.  Halo
// points are recomputed by every tile that needs them; the arithmetic is the
// same as in the tile that owns them, so the values agree bit for bit.  Only
// points of the tile itself are stored.  A pass along a reads its neighbours
// (coarse points) directly from memory.
#include "common.h"
#include "device_math.h"

namespace szg {

constexpr int kHalo = 3;
constexpr int kLevelThreads = 256;

// Division by a per-tile constant: a float estimate of the quotient corrected
// by one step (exact for dividends below 2^22 times the divisor).
struct FastDiv {
  uint32_t d;
  float inv;
};
__device__ __forceinline__ FastDiv make_div(uint32_t d) { return FastDiv{d, 1.0f / (float)d}; }
__device__ __forceinline__ uint32_t div_mod(uint32_t i, const FastDiv& D, uint32_t& r) {
  uint32_t q = (uint32_t)((float)i * D.inv);
  int32_t rr = (int32_t)(i - q * D.d);
  if (rr < 0) {
    q--;
    rr += (int32_t)D.d;
  } else if (rr >= (int32_t)D.d) {
    q++;
    rr -= (int32_t)D.d;
  }
  r = (uint32_t)rr;
  return q;
}

// The lattice coordinates of one parity (or all) in [lo, hi).
struct Prog {
  uint32_t first, count, step;
};
__device__ __forceinline__ Prog prog_even(uint32_t lo, uint32_t hi) {
  const uint32_t f = (lo + 1) & ~1u;
  return Prog{f, hi > f ? (hi - f + 1) / 2 : 0u, 2};
}
__device__ __forceinline__ Prog prog_odd(uint32_t lo, uint32_t hi) {
  const uint32_t f = lo | 1u;
  return Prog{f, hi > f ? (hi - f + 1) / 2 : 0u, 2};
}
__device__ __forceinline__ Prog prog_all(uint32_t lo, uint32_t hi) {
  return Prog{lo, hi > lo ? hi - lo : 0u, 1};
}

struct Tile {
  uint32_t A0, A1, B0, B1, C0, C1;  // tile
  uint32_t Bo, Be, Co, Ce;          // box along b and c
};

__device__ __forceinline__ Tile tile_of(const LevelGeom& g, uint64_t bid) {
  // XCD-aware order: workgroups are dealt to the 8 dies round-robin, so give
  // each die a contiguous run of tiles (neighbours share halos and coarse
  // points in that die's L2)
  const uint64_t nt = g.ntiles, full = nt & ~7ull;
  uint64_t t = bid;
  if (bid < full) t = (bid & 7) * (full >> 3) + (bid >> 3);
  const uint32_t tc = (uint32_t)(t % g.ntile[2]);
  t /= g.ntile[2];
  const uint32_t tb = (uint32_t)(t % g.ntile[1]);
  const uint32_t ta = (uint32_t)(t / g.ntile[1]);
  Tile T;
  T.A0 = ta * g.tile[0];
  T.B0 = tb * g.tile[1];
  T.C0 = tc * g.tile[2];
  T.A1 = min(T.A0 + g.tile[0], g.ext[0]);
  T.B1 = min(T.B0 + g.tile[1], g.ext[1]);
  T.C1 = min(T.C0 + g.tile[2], g.ext[2]);
  T.Bo = T.B0 >= (uint32_t)kHalo ? T.B0 - kHalo : 0u;
  T.Co = T.C0 >= (uint32_t)kHalo ? T.C0 - kHalo : 0u;
  T.Be = min(T.B1 + kHalo, g.ext[1]);
  T.Ce = min(T.C1 + kHalo, g.ext[2]);
  return T;
}

// The points of one pass inside a tile: a product of three coordinate
// progressions, enumerated with c fastest.
struct StageSet {
  Prog pa, pb, pc;
  FastDiv db, dc;
  uint32_t n;
};
__device__ __forceinline__ StageSet stage_set(Prog pa, Prog pb, Prog pc) {
  StageSet S;
  S.pa = pa;
  S.pb = pb;
  S.pc = pc;
  S.db = make_div(pb.count ? pb.count : 1);
  S.dc = make_div(pc.count ? pc.count : 1);
  S.n = pa.count * pb.count * pc.count;
  return S;
}
__device__ __forceinline__ void stage_coords(const StageSet& S, uint32_t i, uint32_t& qa,
                                             uint32_t& qb, uint32_t& qc) {
  uint32_t jc, jb;
  const uint32_t r = div_mod(i, S.dc, jc);
  const uint32_t ja = div_mod(r, S.db, jb);
  qa = S.pa.first + S.pa.step * ja;
  qb = S.pb.first + S.pb.step * jb;
  qc = S.pc.first + S.pc.step * jc;
}

// Per-point input and step shared by compression and reconstruction.
// Compression: quantize x against the prediction (the value kept is the
// reconstruction).  Reconstruction: recover from the code, or keep the
// verbatim value the decoder already stored for code 0.
template <typename T, bool RECON>
struct PointOp {
  const T* __restrict__ x;
  T* v;
  uint16_t* codes;
  QuantParams<T> q;
  struct In {
    T xv;
    uint32_t code;
  };
  __device__ __forceinline__ In load(uint64_t f) const {
    In in;
    if (RECON) {
      in.xv = T(0);
      in.code = codes[f];
    } else {
      in.xv = x[f];
      in.code = 0;
    }
    return in;
  }
  __device__ __forceinline__ T finish(uint64_t f, T pred, In in, bool own) const {
    if (RECON) {
      return in.code ? recover(pred, q.twoeb, in.code, q.R) : v[f];
    } else {
      T r;
      const uint32_t code = quantize(in.xv, pred, q, r);
      if (own) codes[f] = (uint16_t)code;
      return r;
    }
  }
};

// Points per thread whose memory reads are issued together before any of
// them is used, so that a workgroup keeps many reads in flight.
constexpr int kBatch = 8;

template <typename T, int PRED, bool RECON>
__global__ __launch_bounds__(kLevelThreads) void k_level(const T* __restrict__ x, T* v,
                                                         uint16_t* codes, LevelGeom g,
                                                         const Meta* __restrict__ m, T twoeb,
                                                         uint32_t R, uint32_t flags) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* box = reinterpret_cast<T*>(smem_raw);
  const Tile t = tile_of(g, blockIdx.x);
  const uint32_t BB = g.box_b, BC = g.box_c;
  const uint64_t fa = g.fs[0], fb = g.fs[1], fc = g.fs[2];
  const bool store_v = (flags & kLevelStoreValues) != 0;
  PointOp<T, RECON> op;
  op.x = x;
  op.v = v;
  op.codes = codes;
  if (RECON) {
    op.q.eb = T(0);
    op.q.twoeb = twoeb;
    op.q.inv2eb = T(0);
    op.q.R = R;
  } else {
    op.q = QuantParams<T>::from_meta(m, R);
  }
  using In = typename PointOp<T, RECON>::In;
  auto bidx = [&](uint32_t qa, uint32_t qb, uint32_t qc) {
    return ((qa - t.A0) * BB + (qb - t.Bo)) * BC + (qc - t.Co);
  };
  auto flat = [&](uint32_t qa, uint32_t qb, uint32_t qc) { return qa * fa + qb * fb + qc * fc; };
  const uint32_t tid = threadIdx.x;

  // coarse points of the box (and, when asked, store them back in place so
  // that the tile's rows are written whole)
  {
    const StageSet S = stage_set(prog_even(t.A0, t.A1), prog_even(t.Bo, t.Be), prog_even(t.Co, t.Ce));
    const bool rewrite = (flags & kLevelRewriteCoarse) != 0;
    for (uint32_t i0 = tid; i0 < S.n; i0 += kLevelThreads * kBatch) {
      T val[kBatch];
      uint32_t qa[kBatch], qb[kBatch], qc[kBatch];
#pragma unroll
      for (int k = 0; k < kBatch; k++) {
        const uint32_t i = i0 + k * kLevelThreads;
        if (i < S.n) {
          stage_coords(S, i, qa[k], qb[k], qc[k]);
          val[k] = v[flat(qa[k], qb[k], qc[k])];
        }
      }
#pragma unroll
      for (int k = 0; k < kBatch; k++) {
        const uint32_t i = i0 + k * kLevelThreads;
        if (i < S.n) {
          box[bidx(qa[k], qb[k], qc[k])] = val[k];
          if (rewrite && qb[k] >= t.B0 && qb[k] < t.B1 && qc[k] >= t.C0 && qc[k] < t.C1)
            v[flat(qa[k], qb[k], qc[k])] = val[k];
        }
      }
    }
  }
  __syncthreads();

  // pass along a on the whole box (neighbours are coarse points in memory)
  {
    const StageSet S = stage_set(prog_odd(t.A0, t.A1), prog_even(t.Bo, t.Be), prog_even(t.Co, t.Ce));
    const uint32_t ea = g.ext[0];
    constexpr int KB = kBatch / 2;
    for (uint32_t i0 = tid; i0 < S.n; i0 += kLevelThreads * KB) {
      T na[KB], nb[KB], nc[KB], ne[KB];
      In in[KB];
      uint32_t qa[KB], qb[KB], qc[KB];
#pragma unroll
      for (int k = 0; k < KB; k++) {
        const uint32_t i = i0 + k * kLevelThreads;
        if (i < S.n) {
          stage_coords(S, i, qa[k], qb[k], qc[k]);
          const uint64_t f = flat(qa[k], qb[k], qc[k]);
          const bool has_a = qa[k] >= 3, has_c = qa[k] + 1 < ea, has_e = qa[k] + 3 < ea;
          nb[k] = v[f - fa];
          nc[k] = has_c ? v[f + fa] : T(0);
          const bool need_a = has_a && (!has_c || PRED == SZ_INTERP_CUBIC);
          na[k] = need_a ? v[f - 3 * fa] : T(0);
          ne[k] = (PRED == SZ_INTERP_CUBIC && has_e) ? v[f + 3 * fa] : T(0);
          in[k] = op.load(f);
        }
      }
#pragma unroll
      for (int k = 0; k < KB; k++) {
        const uint32_t i = i0 + k * kLevelThreads;
        if (i < S.n) {
          const uint64_t f = flat(qa[k], qb[k], qc[k]);
          const bool has_a = qa[k] >= 3, has_c = qa[k] + 1 < ea, has_e = qa[k] + 3 < ea;
          const T pred = interp_predict<T, PRED>(na[k], nb[k], nc[k], ne[k], has_a, has_c, has_e);
          const bool own = qb[k] >= t.B0 && qb[k] < t.B1 && qc[k] >= t.C0 && qc[k] < t.C1;
          const T val = op.finish(f, pred, in[k], own);
          box[bidx(qa[k], qb[k], qc[k])] = val;
          if (own && store_v) v[f] = val;
        }
      }
    }
  }
  __syncthreads();

  // pass along b on the tile's rows of the box, then along c on the tile:
  // neighbours come from the box, `step` is the box offset of one unit
  auto lds_pass = [&](const StageSet& S, uint32_t ext, int axis, uint32_t step, bool halo_c) {
    for (uint32_t i0 = tid; i0 < S.n; i0 += kLevelThreads * kBatch) {
      In in[kBatch];
      uint32_t qa[kBatch], qb[kBatch], qc[kBatch];
#pragma unroll
      for (int k = 0; k < kBatch; k++) {
        const uint32_t i = i0 + k * kLevelThreads;
        if (i < S.n) {
          stage_coords(S, i, qa[k], qb[k], qc[k]);
          in[k] = op.load(flat(qa[k], qb[k], qc[k]));
        }
      }
#pragma unroll
      for (int k = 0; k < kBatch; k++) {
        const uint32_t i = i0 + k * kLevelThreads;
        if (i < S.n) {
          const uint32_t q = axis == 1 ? qb[k] : qc[k];
          const uint32_t bk = bidx(qa[k], qb[k], qc[k]);
          const bool has_a = q >= 3, has_c = q + 1 < ext, has_e = q + 3 < ext;
          const T b = box[bk - step];
          const T c = has_c ? box[bk + step] : T(0);
          const bool need_a = has_a && (!has_c || PRED == SZ_INTERP_CUBIC);
          const T a = need_a ? box[bk - 3 * step] : T(0);
          const T e = (PRED == SZ_INTERP_CUBIC && has_e) ? box[bk + 3 * step] : T(0);
          const T pred = interp_predict<T, PRED>(a, b, c, e, has_a, has_c, has_e);
          const bool own = !halo_c || (qc[k] >= t.C0 && qc[k] < t.C1);
          const uint64_t f = flat(qa[k], qb[k], qc[k]);
          const T val = op.finish(f, pred, in[k], own);
          if (halo_c) box[bk] = val;
          if (own && store_v) v[f] = val;
        }
      }
    }
  };
  lds_pass(stage_set(prog_all(t.A0, t.A1), prog_odd(t.B0, t.B1), prog_even(t.Co, t.Ce)), g.ext[1],
           1, BC, true);
  __syncthreads();
  lds_pass(stage_set(prog_all(t.A0, t.A1), prog_all(t.B0, t.B1), prog_odd(t.C0, t.C1)), g.ext[2],
           2, 1, false);
}

// ------------------------------------------------------------------ host side

namespace {
uint32_t ceil_div32(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

uint64_t box_bytes(const uint32_t tile[3], const uint32_t ext[3], int tsize) {
  const uint64_t bb = std::min<uint64_t>(tile[1] + 2 * kHalo, ext[1]);
  const uint64_t bc = std::min<uint64_t>(tile[2] + 2 * kHalo, ext[2]);
  return (uint64_t)tile[0] * bb * bc * tsize;
}
}  // namespace

bool plan_levels(int ndim, const uint64_t* dims, const uint8_t* order, int tsize,
                 const LevelTuning* tune, std::vector<LevelGeom>& out) {
  out.clear();
  if (ndim < 1 || ndim > 3) return false;
  // view as three dimensions with leading extents of 1 (their passes are empty)
  uint64_t V[3], VS[3];
  uint8_t O[3];
  const int lead = 3 - ndim;
  for (int k = 0; k < 3; k++) V[k] = k < lead ? 1 : dims[k - lead];
  VS[2] = 1;
  VS[1] = V[2];
  VS[0] = V[1] * V[2];
  for (int k = 0; k < lead; k++) O[k] = (uint8_t)k;
  for (int j = 0; j < ndim; j++) O[lead + j] = (uint8_t)(lead + order[j]);
  int L = 0;
  for (int d = 0; d < ndim; d++) {
    int l = 0;
    while ((1ull << l) < dims[d]) l++;
    L = std::max(L, l);
  }
  int pc = 0;  // position of the contiguous dimension in the pass order
  for (int j = 0; j < 3; j++)
    if (O[j] == 2) pc = j;
  for (int l = L; l >= 1; l--) {
    const uint64_t s = 1ull << (l - 1);
    LevelGeom g{};
    g.s = (uint32_t)s;
    for (int j = 0; j < 3; j++) {
      g.ext[j] = (uint32_t)((V[O[j]] - 1) / s + 1);
      g.fs[j] = VS[O[j]] * s;
    }
    uint32_t T[3];
    const uint32_t target = tune ? tune->target_points : 4096;
    const uint32_t lds_cap = tune ? tune->lds_bytes : 48 * 1024;
    T[2] = std::min<uint32_t>(g.ext[2], pc == 2 ? (tune ? tune->tile_c : 64) : 16);
    T[1] = std::min<uint32_t>(g.ext[1], tune ? tune->tile_b : 16);
    T[0] = std::min<uint32_t>(g.ext[0], std::max<uint32_t>(1, target / (T[1] * T[2])));
    while ((uint64_t)T[0] * T[1] * T[2] < target && T[1] < g.ext[1])
      T[1] = std::min<uint32_t>(g.ext[1], 2 * T[1]);
    while ((uint64_t)T[0] * T[1] * T[2] < target && T[2] < g.ext[2])
      T[2] = std::min<uint32_t>(g.ext[2], 2 * T[2]);
    while (box_bytes(T, g.ext, tsize) > lds_cap) {
      int big = 0;
      uint64_t bv = 0;
      const uint64_t sz[3] = {T[0], std::min<uint64_t>(T[1] + 2 * kHalo, g.ext[1]),
                              std::min<uint64_t>(T[2] + 2 * kHalo, g.ext[2])};
      for (int j = 0; j < 3; j++)
        if (T[j] > 1 && sz[j] > bv) bv = sz[j], big = j;
      if (T[big] <= 1) return false;
      T[big] = (T[big] + 1) / 2;
    }
    for (int j = 0; j < 3; j++) {
      g.tile[j] = T[j];
      g.ntile[j] = ceil_div32(g.ext[j], T[j]);
    }
    g.box_b = std::min<uint32_t>(T[1] + 2 * kHalo, g.ext[1]);
    g.box_c = std::min<uint32_t>(T[2] + 2 * kHalo, g.ext[2]);
    g.ntiles = (uint64_t)g.ntile[0] * g.ntile[1] * g.ntile[2];
    g.lds = (uint32_t)box_bytes(T, g.ext, tsize);
    out.push_back(g);
  }
  return true;
}

template <typename T, bool RECON>
static hipError_t launch_level_t(const void* x, int predictor, void* v, uint16_t* codes,
                                 const LevelGeom& g, const Meta* m, double eb_t, uint32_t R,
                                 uint32_t flags, hipStream_t st) {
  if (g.ntiles == 0) return hipSuccess;
  if (g.ntiles > 0x7FFFFFFFull) return hipErrorInvalidValue;
  dim3 grid((unsigned)g.ntiles), block(kLevelThreads);
  const T twoeb = RECON ? (T)2 * (T)eb_t : T(0);
  if (predictor == SZ_INTERP_CUBIC)
    hipLaunchKernelGGL((k_level<T, SZ_INTERP_CUBIC, RECON>), grid, block, g.lds, st,
                       (const T*)x, (T*)v, codes, g, m, twoeb, R, flags);
  else
    hipLaunchKernelGGL((k_level<T, SZ_INTERP_LINEAR, RECON>), grid, block, g.lds, st,
                       (const T*)x, (T*)v, codes, g, m, twoeb, R, flags);
  return hipGetLastError();
}

hipError_t launch_level_compress(const void* x, int dtype, int predictor, void* rec,
                                 uint16_t* codes, const LevelGeom& g, const Meta* m,
                                 uint32_t radius, bool store_rec, hipStream_t st) {
  const uint32_t flags = store_rec ? kLevelStoreValues : 0u;
  if (dtype == SZ_F32)
    return launch_level_t<float, false>(x, predictor, rec, codes, g, m, 0.0, radius, flags, st);
  return launch_level_t<double, false>(x, predictor, rec, codes, g, m, 0.0, radius, flags, st);
}

hipError_t launch_level_recon(const uint16_t* codes, int dtype, int predictor, void* out,
                              const LevelGeom& g, double eb_t, uint32_t radius, hipStream_t st) {
  // at stride 1 the tile's coarse points are stored back too, so that whole
  // rows of the output are written by one workgroup
  const uint32_t flags = kLevelStoreValues | (g.s == 1 ? kLevelRewriteCoarse : 0u);
  uint16_t* c = const_cast<uint16_t*>(codes);  // read only when reconstructing
  if (dtype == SZ_F32)
    return launch_level_t<float, true>(nullptr, predictor, out, c, g, nullptr, eb_t, radius,
                                       flags, st);
  return launch_level_t<double, true>(nullptr, predictor, out, c, g, nullptr, eb_t, radius, flags,
                                      st);
}

}  // namespace szg
