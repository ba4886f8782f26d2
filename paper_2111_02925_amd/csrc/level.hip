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
// Points with every coordinate even ("coarse") are final from earlier levels.
//
// Only the pass along a crosses planes of constant a, and it reads coarse
// points only.  So a plane's passes along b and c depend on nothing of the
// level but the plane's own pass along a, and planes can be streamed.  A
// workgroup owns a (b, c) tile of a run of planes and keeps in LDS
//   - the plane's box: the tile extended by 3 units along b and c,
//   - a ring of the coarse grids (b, c even) of four even planes, which the
//     pass along a reads (planes a-3, a-1, a+1, a+3) and even planes take
//     their coarse points from,
//   - the codes of the box (compression).
// Per plane, separated by barriers: fill the box (inputs loaded during the
// previous plane), the pass along a on the whole box (odd planes), the pass
// along b on the tile's rows of the box, the pass along c on the tile, and
// store the tile row by row.  Every input row is read once and whole; halo
// points are recomputed with the same arithmetic as in the tile that owns
// them, so the values agree bit for bit.
//
// Flat indices fit in 32 bits (fields have fewer than 2^32 points).
#include <type_traits>

#include "block_ops.h"
#include "common.h"
#include "device_math.h"

namespace szg {

constexpr int kHalo = 3;
constexpr int kLevelThreads = 256;
constexpr int kLevelWaves = kLevelThreads / 64;
constexpr int kBoxUnits = 12;   // box (row, 64-column chunk) units per wave: 48 per plane
constexpr int kGridUnits = 6;   // coarse-grid units per wave: 24 per plane


// A box slot holds an input before its point is computed: the field value,
// or the quantization code as an integer in the slot's bits.
__device__ __forceinline__ float code_bits(uint32_t c, float) { return __uint_as_float(c); }
__device__ __forceinline__ double code_bits(uint32_t c, double) {
  return __longlong_as_double((long long)c);
}
__device__ __forceinline__ uint32_t bits_code(float v) { return __float_as_uint(v); }
__device__ __forceinline__ uint32_t bits_code(double v) {
  return (uint32_t)__double_as_longlong(v);
}

// Compression: quantize the field value against the prediction (the value
// kept is the reconstruction).  Reconstruction: recover from the code, or
// keep the verbatim value the decoder already stored for code 0 (at flat
// index f(), only evaluated then).
template <typename T, bool RECON, typename FlatFn>
__device__ __forceinline__ T point_step(T slot, T pred, const QuantParams<T>& q, const T* v,
                                        FlatFn f, uint32_t& code) {
  if (RECON) {
    code = bits_code(slot);
    if (code) return recover(pred, q.twoeb, code, q.R);
    // rare: take the read here (an empty asm that uses it), so that the
    // common path never waits on it, nor on the loads in flight before it
    T w = v[f()];
    asm volatile("" : "+v"(w));
    return w;
  } else {
    T r;
    code = quantize(slot, pred, q, r);
    return r;
  }
}

// Interpolation along one dimension at lattice coordinate qd of extent ext;
// get(o, ok) returns the value at offset o in {-3, -1, +1, +3}, reading a
// harmless in-bounds location instead when ok is false.  INTERIOR: every
// stencil point exists (3 <= qd, qd + 3 < ext).  Otherwise every rule is
// evaluated and the right one selected, so lanes never branch on it.
template <typename T, int PRED, bool INTERIOR, typename Get>
__device__ __forceinline__ T predict_at(uint32_t qd, uint32_t ext, Get get) {
  if (INTERIOR) {
    if (PRED == SZ_INTERP_CUBIC)
      return interp_predict<T, PRED>(get(-3, true), get(-1, true), get(1, true), get(3, true),
                                     true, true, true);
    return interp_predict<T, PRED>(T(0), get(-1, true), get(1, true), T(0), true, true, true);
  }
  const bool has_a = qd >= 3, has_c = qd + 1 < ext, has_e = qd + 3 < ext;
  return interp_predict_sel<T, PRED>(get(-3, has_a), get(-1, true), get(1, has_c),
                                     get(3, has_e), has_a, has_c, has_e);
}

// The work item of a workgroup: a (b, c) tile, its box, and a run of planes.
struct Item {
  uint32_t P0, P1;            // planes
  uint32_t B0, B1, C0, C1;    // tile
  uint32_t Bo, Be, Co, Ce;    // box
  uint32_t Bq, Cq;            // first even b and c of the box (coarse-grid origin)
};

__device__ __forceinline__ Item item_of(const LevelGeom& g, uint32_t bid) {
  // XCD-aware order: workgroups are dealt to the 8 dies round-robin, so give
  // each die a contiguous run of items (neighbours share halos in its L2)
  const uint32_t nt = (uint32_t)g.nitems, full = nt & ~7u;
  uint32_t t = bid;
  if (bid < full) t = (bid & 7) * (full >> 3) + (bid >> 3);
  const uint32_t tc = t % g.ntile[2];
  t /= g.ntile[2];
  const uint32_t tb = t % g.ntile[1];
  const uint32_t ta = t / g.ntile[1];
  Item I;
  I.P0 = ta * g.planes;
  I.P1 = min(I.P0 + g.planes, g.ext[0]);
  I.B0 = tb * g.tile[1];
  I.C0 = tc * g.tile[2];
  I.B1 = min(I.B0 + g.tile[1], g.ext[1]);
  I.C1 = min(I.C0 + g.tile[2], g.ext[2]);
  I.Bo = I.B0 >= (uint32_t)kHalo ? I.B0 - kHalo : 0u;
  I.Co = I.C0 >= (uint32_t)kHalo ? I.C0 - kHalo : 0u;
  I.Be = min(I.B1 + kHalo, g.ext[1]);
  I.Ce = min(I.C1 + kHalo, g.ext[2]);
  I.Bq = (I.Bo + 1) & ~1u;
  I.Cq = (I.Co + 1) & ~1u;
  return I;
}

// A wave's units (row, 64-column chunk) of a row set, u = wave + 4k: lane k
// decodes unit k into one word (row | chunk << 16), read back per unit as a
// wave-uniform value.  Columns past the row's end repeat its last column.
__device__ __forceinline__ uint32_t unit_word(uint32_t wave, uint32_t lane, uint32_t nrow,
                                              uint32_t ncc) {
  // units past the last one repeat it: their loads and stores duplicate the
  // last unit's (same addresses, same values), which keeps the loops free of
  // branches
  const uint32_t n = nrow * ncc;
  const uint32_t u = min(wave + kLevelWaves * lane, n - 1);
  return (u / ncc) | (u % ncc) << 16;
}

// Inputs of one plane, held in registers from their loads (issued while the
// previous plane computes) until the box is filled.
template <typename T>
struct PlaneIn {
  T val[kBoxUnits];       // compression: the field's values over the box
  uint32_t raw[kBoxUnits];// codes: all (reconstruction), of coarse rows (compression)
  T grid[kGridUnits];     // rows (b even) of an even plane, for the ring
};

template <typename T, int PRED, bool RECON>
__global__ __launch_bounds__(kLevelThreads) void k_level(const T* __restrict__ x, T* v,
                                                         uint16_t* codes, LevelGeom g,
                                                         const Meta* __restrict__ m, T twoeb,
                                                         uint32_t R, uint32_t flags) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* box = reinterpret_cast<T*>(smem_raw);
  T* ring = reinterpret_cast<T*>(smem_raw + g.box_bytes);
  uint16_t* lcode = reinterpret_cast<uint16_t*>(smem_raw + g.box_bytes + g.ring_bytes);
  const Item I = item_of(g, blockIdx.x);
  const uint32_t BC = g.box_c, RB = g.ring_b, RC = g.ring_c;
  const uint32_t fa = (uint32_t)g.fs[0], fb = (uint32_t)g.fs[1], fc = (uint32_t)g.fs[2];
  const uint32_t ea = g.ext[0];
  const bool store_v = (flags & kLevelStoreValues) != 0;
  QuantParams<T> q;
  if (RECON) {
    q.eb = T(0);
    q.twoeb = twoeb;
    q.inv2eb = T(0);
    q.R = R;
  } else {
    q = QuantParams<T>::from_meta(m, R);
  }
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t nB = I.Be - I.Bo, nC = I.Ce - I.Co, ncc = (nC + 63) >> 6;
  const uint32_t nBq = I.Be > I.Bq ? (I.Be - I.Bq + 1) / 2 : 0u;  // even b rows of the box
  const uint32_t box_units = unit_word(wave, lane, nB, ncc);
  const uint32_t tile_ncc = (I.C1 - I.C0 + 63) >> 6, tile_nunit = (I.B1 - I.B0) * tile_ncc;
  const uint32_t tile_units = unit_word(wave, lane, I.B1 - I.B0, tile_ncc);
  const uint32_t grid_units = unit_word(wave, lane, nBq, ncc);
  auto ring_index = [&](uint32_t e, uint32_t b, uint32_t c) {
    return (((e >> 1) & 3u) * RB + ((b - I.Bq) >> 1)) * RC + ((c - I.Cq) >> 1);
  };
  auto ring_at = [&](uint32_t e, uint32_t b, uint32_t c) -> T& { return ring[ring_index(e, b, c)]; };
  const uint32_t dummy = g.box_b * g.box_c;  // the box's and codes' spare last slot

  // ---- loads of an even plane's coarse rows (b even), all columns
  auto issue_grid = [&](uint32_t e, PlaneIn<T>& in) {
#pragma unroll
    for (int k = 0; k < kGridUnits; k++) {
      const uint32_t w = __builtin_amdgcn_readlane(grid_units, k);
      const uint32_t c = min((w >> 16) * 64 + lane, nC - 1);
      in.grid[k] = v[e * fa + (I.Bq + 2 * (w & 0xFFFF)) * fb + (I.Co + c) * fc];
    }
  };
  auto deposit_grid = [&](uint32_t e, const PlaneIn<T>& in) {
#pragma unroll
    for (int k = 0; k < kGridUnits; k++) {
      const uint32_t w = __builtin_amdgcn_readlane(grid_units, k);
      const uint32_t c = min((w >> 16) * 64 + lane, nC - 1);
      const uint32_t qc = I.Co + c;
      if ((qc & 1u) == 0) ring_at(e, I.Bq + 2 * (w & 0xFFFF), qc) = in.grid[k];
    }
  };
  // ---- loads of plane p's inputs over the box (and the ring's next grid)
  auto issue = [&](uint32_t p, PlaneIn<T>& in) {
    const bool even_p = (p & 1u) == 0;
#pragma unroll
    for (int k = 0; k < kBoxUnits; k++) {
      const uint32_t w = __builtin_amdgcn_readlane(box_units, k);
      const uint32_t c = min((w >> 16) * 64 + lane, nC - 1);
      const uint32_t qb = I.Bo + (w & 0xFFFF);
      const uint32_t f = p * fa + qb * fb + (I.Co + c) * fc;
      if (RECON) {
        in.raw[k] = codes[f];
      } else {
        in.val[k] = x[f];
        // codes of the tile's coarse points, stored back with the tile's
        // rows (a condition on the row: the same for the whole wave)
        if (even_p && (qb & 1u) == 0 && qb >= I.B0 && qb < I.B1) in.raw[k] = codes[f];
      }
    }
    if (!even_p && p + 3 < ea) issue_grid(p + 3, in);
  };
  auto deposit = [&](uint32_t p, const PlaneIn<T>& in) {
    const bool even_p = (p & 1u) == 0;
    if (!even_p && p + 3 < ea) deposit_grid(p + 3, in);
#pragma unroll
    for (int k = 0; k < kBoxUnits; k++) {
      const uint32_t w = __builtin_amdgcn_readlane(box_units, k);
      const uint32_t c = min((w >> 16) * 64 + lane, nC - 1);
      const uint32_t row = w & 0xFFFF, qb = I.Bo + row, qc = I.Co + c;
      const uint32_t slot = row * BC + c;
      const bool coarse = even_p && ((qb | qc) & 1u) == 0;
      // coarse points of an even plane come from the ring (deposited at
      // least one plane earlier); other lanes read ring word 0, so that
      // every lane takes the same path
      const T rv = ring[coarse ? ring_index(p, qb, qc) : 0u];
      box[slot] = coarse ? rv : (RECON ? code_bits(in.raw[k], T(0)) : in.val[k]);
      if (!RECON && even_p && (qb & 1u) == 0 && qb >= I.B0 && qb < I.B1)
        lcode[slot] = (uint16_t)in.raw[k];  // other slots are overwritten when computed
    }
    // every input register is taken here, on every path: left possibly
    // pending, it would make the compiler wait for all loads in flight when
    // the register is next written
#pragma unroll
    for (int k = 0; k < kBoxUnits; k++) {
      asm volatile("" ::"v"(in.val[k]));
      asm volatile("" ::"v"(in.raw[k]));
    }
#pragma unroll
    for (int k = 0; k < kGridUnits; k++) asm volatile("" ::"v"(in.grid[k]));
  };

  // ---- a pass over rows (b) x columns (c) of the plane: slot i = row << lg | col
  auto run_pass = [&](auto interior_tag, auto pass_tag, uint32_t p, uint32_t b_first,
                      uint32_t b_step, uint32_t nrow, uint32_t c_first, uint32_t c_step,
                      uint32_t ncol) {
    constexpr bool IN = decltype(interior_tag)::value;
    constexpr int PASS = decltype(pass_tag)::value;  // 0: along a, 1: along b, 2: along c
    if (nrow == 0 || ncol == 0) return;
    const uint32_t lg = ncol <= 1 ? 0u : 32u - (uint32_t)__builtin_clz(ncol - 1);
    const uint32_t nslot = nrow << lg;
    // Padding slots compute a clamped duplicate of a real point and write it
    // to the spare slot: no lane branches on its slot's validity.
    for (uint32_t i0 = 0; i0 < nslot; i0 += kLevelThreads) {
      const uint32_t i = i0 + tid;
      const uint32_t jc0 = i & ((1u << lg) - 1);
      const bool ok = i < nslot && jc0 < ncol;
      const uint32_t jc = min(jc0, ncol - 1), jr = min(i >> lg, nrow - 1);
      const uint32_t qb = b_first + b_step * jr, qc = c_first + c_step * jc;
      const uint32_t bk = (qb - I.Bo) * BC + (qc - I.Co);
      T pred;
      // (a missing neighbour reads the point's own slot: in bounds, unused)
      if (PASS == 0) {
        // ring slots of planes outside the field hold other planes: unused
        auto get = [&](int o, bool ok) { return ring_at((uint32_t)((int32_t)p + o), qb, qc); };
        pred = predict_at<T, PRED, IN>(p, ea, get);
      } else if (PASS == 1) {
        auto get = [&](int o, bool ok) {
          return box[(uint32_t)((int32_t)bk + (ok ? o * (int32_t)BC : 0))];
        };
        pred = predict_at<T, PRED, IN>(qb, g.ext[1], get);
      } else {
        auto get = [&](int o, bool ok) { return box[(uint32_t)((int32_t)bk + (ok ? o : 0))]; };
        pred = predict_at<T, PRED, IN>(qc, g.ext[2], get);
      }
      uint32_t code;
      const T val = point_step<T, RECON>(box[bk], pred, q, v,
                                         [&] { return p * fa + qb * fb + qc * fc; }, code);
      const uint32_t wk = ok ? bk : dummy;
      box[wk] = val;
      if (!RECON) lcode[wk] = (uint16_t)code;  // halo slots are never stored
    }
  };

  // ---- the ring before the first plane: even planes P0-2, P0, P0+2
  {
    PlaneIn<T> pre;
    for (int d = -2; d <= 2; d += 2) {
      const int e = (int)I.P0 + d;
      if (e < 0 || (uint32_t)e >= ea) continue;
      issue_grid((uint32_t)e, pre);
      deposit_grid((uint32_t)e, pre);
    }
  }
  lds_barrier();

  PlaneIn<T> in;
  issue(I.P0, in);
  const bool int_b = I.B0 >= 3 && I.B1 + 3 <= g.ext[1];
  const bool int_c = I.C0 >= 3 && I.C1 + 3 <= g.ext[2];
  for (uint32_t p = I.P0; p < I.P1; p++) {
    deposit(p, in);
    lds_barrier();
    if (p + 1 < I.P1) issue(p + 1, in);

    // pass along a (odd planes) on the whole box: b, c even
    if (p & 1u) {
      const uint32_t ncol = I.Ce > I.Cq ? (I.Ce - I.Cq + 1) / 2 : 0u;
      if (p >= 3 && p + 3 < ea)
        run_pass(std::true_type{}, std::integral_constant<int, 0>{}, p, I.Bq, 2, nBq, I.Cq, 2, ncol);
      else
        run_pass(std::false_type{}, std::integral_constant<int, 0>{}, p, I.Bq, 2, nBq, I.Cq, 2, ncol);
      lds_barrier();
    }
    // pass along b on the tile's rows of the box: b odd, c even
    {
      const uint32_t b1 = I.B0 | 1u, nb = I.B1 > b1 ? (I.B1 - b1 + 1) / 2 : 0u;
      const uint32_t ncol = I.Ce > I.Cq ? (I.Ce - I.Cq + 1) / 2 : 0u;
      if (int_b)
        run_pass(std::true_type{}, std::integral_constant<int, 1>{}, p, b1, 2, nb, I.Cq, 2, ncol);
      else
        run_pass(std::false_type{}, std::integral_constant<int, 1>{}, p, b1, 2, nb, I.Cq, 2, ncol);
    }
    lds_barrier();
    // pass along c on the tile: c odd
    {
      const uint32_t c1 = I.C0 | 1u, ncol = I.C1 > c1 ? (I.C1 - c1 + 1) / 2 : 0u;
      if (int_c)
        run_pass(std::true_type{}, std::integral_constant<int, 2>{}, p, I.B0, 1, I.B1 - I.B0, c1,
                 2, ncol);
      else
        run_pass(std::false_type{}, std::integral_constant<int, 2>{}, p, I.B0, 1, I.B1 - I.B0, c1,
                 2, ncol);
    }
    lds_barrier();
    // the tile's rows of this plane
    {
      const uint32_t tcn = I.C1 - I.C0;
#pragma unroll
      for (int k = 0; k < kBoxUnits; k++) {
        if ((uint32_t)(wave + kLevelWaves * k) >= tile_nunit) break;  // the same for the wave
        const uint32_t w = __builtin_amdgcn_readlane(tile_units, k);
        const uint32_t c = (w >> 16) * 64 + lane;
        if (c < tcn) {
          const uint32_t qb = I.B0 + (w & 0xFFFF), qc = I.C0 + c;
          const uint32_t f = p * fa + qb * fb + qc * fc;
          const uint32_t bk = (qb - I.Bo) * BC + (qc - I.Co);
          if (!RECON) codes[f] = lcode[bk];
          if (RECON || store_v) v[f] = box[bk];
        }
      }
    }
    lds_barrier();  // the box is refilled next
  }
}


// ------------------------------------------------- boxes of up to 64 columns
// The same schedule with a fixed geometry: box rows are 64 slots apart and
// coarse-grid rows 32, lane l of a wave owns box column l when rows are
// loaded, filled or stored, and wave w owns rows w, w + 4, ...  A pass maps
// the workgroup's threads onto (row, column) once; every further row is a
// fixed slot increment, and the stencil reaches its neighbours through
// constant offsets.  Lanes past the pass's extents compute a clamped
// duplicate and write it to the spare slot.
constexpr uint32_t kPitch = 64;
constexpr uint32_t kRingPitch = 32;
constexpr uint32_t kRowsPerWave = 10;                    // boxes of up to 40 rows
constexpr uint32_t kGridRowsPerWave = (kRowsPerWave + 1) / 2;
constexpr uint32_t kMaxBoxRows64 = kRowsPerWave * kLevelWaves;

template <typename T, bool RECON>
struct RowIn {
  T val[RECON ? 1 : kRowsPerWave];         // compression: the field's values over the box
  uint32_t raw[RECON ? kRowsPerWave : 1];  // reconstruction: the codes over the box
  T grid[kGridRowsPerWave];                // rows (b even) of an even plane, for the ring
};

template <typename T, int PRED, bool RECON>
__device__ __forceinline__ void level64_body(const T* __restrict__ x, T* v, uint16_t* codes,
                                             const LevelGeom& g, const Meta* __restrict__ m,
                                             T twoeb, uint32_t R, uint32_t flags, T* cmp,
                                             uint32_t bid) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* box = reinterpret_cast<T*>(smem_raw);
  T* ring = reinterpret_cast<T*>(smem_raw + g.box_bytes);
  uint16_t* lcode = reinterpret_cast<uint16_t*>(smem_raw + g.box_bytes + g.ring_bytes);
  const Item I = item_of(g, bid);
  const uint32_t ring_slot = g.ring_b * kRingPitch;  // entries per coarse grid
  const uint32_t fa = (uint32_t)g.fs[0], fb = (uint32_t)g.fs[1], fc = (uint32_t)g.fs[2];
  const uint32_t ea = g.ext[0];
  const bool store_c = (flags & kLevelStoreCompact) != 0;
  const bool store_v = (flags & kLevelStoreValues) != 0 || (RECON && !store_c);
  QuantParams<T> q;
  if (RECON) {
    q.eb = T(0);
    q.twoeb = twoeb;
    q.inv2eb = T(0);
    q.R = R;
  } else {
    q = QuantParams<T>::from_meta(m, R);
  }
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t nB = I.Be - I.Bo, nC = I.Ce - I.Co;
  const uint32_t nBq = I.Be > I.Bq ? (I.Be - I.Bq + 1) / 2 : 0u;  // even b rows of the box
  const uint32_t dummy = g.box_b * kPitch;                         // spare slot
  // this lane's box column (clamped to the box) for row-wise work
  const uint32_t lc = min(lane, nC - 1), qc_l = I.Co + lc;
  const uint32_t colf = qc_l * fc;
  const bool col_in = lane < nC, qc_even = (qc_l & 1u) == 0;
  const uint32_t ring_col = (qc_l - I.Cq) >> 1;
  auto grid_base = [&](uint32_t e) { return ((e >> 1) & 3u) * ring_slot; };

  // ---- an even plane's coarse rows (b even) into the ring.  Loads are not
  // branched around (a register loaded on one path only would be waited for
  // where the paths join): rows past the last repeat it.
  auto issue_grid = [&](uint32_t e, RowIn<T, RECON>& in) {
    if (nBq == 0) return;
#pragma unroll
    for (uint32_t k = 0; k < kGridRowsPerWave; k++) {
      const uint32_t j = min(wave + kLevelWaves * k, nBq - 1);
      in.grid[k] = v[e * fa + (I.Bq + 2 * j) * fb + colf];
    }
  };
  auto deposit_grid = [&](uint32_t e, const RowIn<T, RECON>& in) {
#pragma unroll
    for (uint32_t k = 0; k < kGridRowsPerWave; k++) {
      const uint32_t j = wave + kLevelWaves * k;
      if (j < nBq && col_in && qc_even) ring[grid_base(e) + j * kRingPitch + ring_col] = in.grid[k];
    }
  };
  // ---- plane p's inputs over the box (and the ring's next grid)
  auto issue = [&](uint32_t p, RowIn<T, RECON>& in) {
    const bool even_p = (p & 1u) == 0;
#pragma unroll
    for (uint32_t k = 0; k < kRowsPerWave; k++) {
      const uint32_t qb = I.Bo + min(wave + kLevelWaves * k, nB - 1);
      const uint32_t f = p * fa + qb * fb + colf;
      if (RECON)
        in.raw[k] = codes[f];
      else
        in.val[k] = x[f];
    }
    if (!even_p && p + 3 < ea) issue_grid(p + 3, in);
  };
  auto deposit = [&](uint32_t p, const RowIn<T, RECON>& in) {
    const bool even_p = (p & 1u) == 0;
    if (!even_p && p + 3 < ea) deposit_grid(p + 3, in);
    const uint32_t gb = grid_base(p);
#pragma unroll
    for (uint32_t k = 0; k < kRowsPerWave; k++) {
      const uint32_t r = wave + kLevelWaves * k, qb = I.Bo + r;
      if (r < nB) {
        const uint32_t slot = r * kPitch + lane;  // columns past the box are never read
        // coarse points of an even plane come from the ring (deposited at
        // least one plane earlier); other lanes read ring word 0
        const bool coarse = even_p && ((qb | qc_l) & 1u) == 0;
        const T rv = ring[coarse ? gb + ((qb - I.Bq) >> 1) * kRingPitch + ring_col : 0u];
        if (RECON)
          box[slot] = coarse ? rv : code_bits(in.raw[k], T(0));
        else
          box[slot] = coarse ? rv : in.val[k];
      }
    }
    // every input register is taken here, on every path (see PlaneIn)
#pragma unroll
    for (uint32_t k = 0; k < kRowsPerWave; k++) {
      if (RECON)
        asm volatile("" ::"v"(in.raw[k]));
      else
        asm volatile("" ::"v"(in.val[k]));
    }
#pragma unroll
    for (uint32_t k = 0; k < kGridRowsPerWave; k++) asm volatile("" ::"v"(in.grid[k]));
  };

  // ---- a pass over rows qb = b_first + b_step * r (r < nrow) and columns
  // qc = c_first + c_step * j (j < ncol <= 32)
  auto run_pass = [&](auto interior_tag, auto pass_tag, uint32_t p, uint32_t b_first,
                      uint32_t b_step, uint32_t nrow, uint32_t c_first, uint32_t c_step,
                      uint32_t ncol) {
    constexpr bool IN = decltype(interior_tag)::value;
    constexpr int PASS = decltype(pass_tag)::value;  // 0: along a, 1: along b, 2: along c
    if (nrow == 0 || ncol == 0) return;
    const uint32_t lg = ncol <= 1 ? 0u : 32u - (uint32_t)__builtin_clz(ncol - 1);
    const uint32_t rows_per_it = kLevelThreads >> lg;
    const uint32_t jc0 = tid & ((1u << lg) - 1), jc = min(jc0, ncol - 1), jr = tid >> lg;
    const bool col_ok = jc0 < ncol;
    const uint32_t qc = c_first + c_step * jc;
    const uint32_t row0 = b_first - I.Bo;  // box row of r = 0
    uint32_t bk = (row0 + b_step * jr) * kPitch + (qc - I.Co);
    const uint32_t bk_last = (row0 + b_step * (nrow - 1)) * kPitch + (qc - I.Co);
    const uint32_t dbk = rows_per_it * b_step * kPitch;
    // pass along a: the coarse grids of planes p - 3, p - 1, p + 1, p + 3
    // (ring slots of planes outside the field hold other planes: unused)
    uint32_t rk = 0, rk_last = 0, drk = 0, g_m3 = 0, g_m1 = 0, g_p1 = 0, g_p3 = 0;
    if (PASS == 0) {
      rk = ((b_first + b_step * jr - I.Bq) >> 1) * kRingPitch + ((qc - I.Cq) >> 1);
      rk_last = ((b_first + b_step * (nrow - 1) - I.Bq) >> 1) * kRingPitch + ((qc - I.Cq) >> 1);
      drk = rows_per_it * kRingPitch;
      g_m3 = grid_base(p - 3);
      g_m1 = grid_base(p - 1);
      g_p1 = grid_base(p + 1);
      g_p3 = grid_base(p + 3);
    }
    const uint32_t nit = (nrow + rows_per_it - 1) / rows_per_it;
    for (uint32_t it = 0; it < nit; it++) {
      const bool ok = col_ok && bk <= bk_last;
      const uint32_t b = min(bk, bk_last);
      const uint32_t qb = I.Bo + (b >> 6);
      T pred;
      // (a missing neighbour reads the point's own slot: in bounds, unused)
      if (PASS == 0) {
        const uint32_t rr = min(rk, rk_last);
        auto get = [&](int o, bool) {
          return ring[rr + (o == -3 ? g_m3 : o == -1 ? g_m1 : o == 1 ? g_p1 : g_p3)];
        };
        pred = predict_at<T, PRED, IN>(p, ea, get);
      } else if (PASS == 1) {
        auto get = [&](int o, bool okn) {
          return box[(uint32_t)((int32_t)b + (okn ? o * (int32_t)kPitch : 0))];
        };
        pred = predict_at<T, PRED, IN>(qb, g.ext[1], get);
      } else {
        auto get = [&](int o, bool okn) { return box[(uint32_t)((int32_t)b + (okn ? o : 0))]; };
        pred = predict_at<T, PRED, IN>(qc, g.ext[2], get);
      }
      uint32_t code;
      const T val = point_step<T, RECON>(box[b], pred, q, v,
                                         [&] { return p * fa + qb * fb + qc * fc; }, code);
      const uint32_t wk = ok ? b : dummy;
      box[wk] = val;
      if (!RECON) lcode[wk] = (uint16_t)code;  // halo slots are never stored
      bk += dbk;
      if (PASS == 0) rk += drk;
    }
  };

  // ---- the ring before the first plane: even planes P0-2, P0, P0+2
  {
    RowIn<T, RECON> pre;
    for (int d = -2; d <= 2; d += 2) {
      const int e = (int)I.P0 + d;
      if (e < 0 || (uint32_t)e >= ea) continue;
      issue_grid((uint32_t)e, pre);
      deposit_grid((uint32_t)e, pre);
    }
  }
  lds_barrier();

  RowIn<T, RECON> in;
  issue(I.P0, in);
  const bool int_b = I.B0 >= 3 && I.B1 + 3 <= g.ext[1];
  const bool int_c = I.C0 >= 3 && I.C1 + 3 <= g.ext[2];
  const uint32_t tile_rows = I.B1 - I.B0, tcn = I.C1 - I.C0;
  for (uint32_t p = I.P0; p < I.P1; p++) {
    deposit(p, in);
    lds_barrier();
    if (p + 1 < I.P1) issue(p + 1, in);

    // pass along a (odd planes) on the whole box: b, c even
    if (p & 1u) {
      const uint32_t ncol = I.Ce > I.Cq ? (I.Ce - I.Cq + 1) / 2 : 0u;
      if (p >= 3 && p + 3 < ea)
        run_pass(std::true_type{}, std::integral_constant<int, 0>{}, p, I.Bq, 2, nBq, I.Cq, 2, ncol);
      else
        run_pass(std::false_type{}, std::integral_constant<int, 0>{}, p, I.Bq, 2, nBq, I.Cq, 2, ncol);
      lds_barrier();
    }
    // pass along b on the tile's rows of the box: b odd, c even
    {
      const uint32_t b1 = I.B0 | 1u, nb = I.B1 > b1 ? (I.B1 - b1 + 1) / 2 : 0u;
      const uint32_t ncol = I.Ce > I.Cq ? (I.Ce - I.Cq + 1) / 2 : 0u;
      if (int_b)
        run_pass(std::true_type{}, std::integral_constant<int, 1>{}, p, b1, 2, nb, I.Cq, 2, ncol);
      else
        run_pass(std::false_type{}, std::integral_constant<int, 1>{}, p, b1, 2, nb, I.Cq, 2, ncol);
    }
    lds_barrier();
    // pass along c on the tile: c odd
    {
      const uint32_t c1 = I.C0 | 1u, ncol = I.C1 > c1 ? (I.C1 - c1 + 1) / 2 : 0u;
      if (int_c)
        run_pass(std::true_type{}, std::integral_constant<int, 2>{}, p, I.B0, 1, tile_rows, c1, 2,
                 ncol);
      else
        run_pass(std::false_type{}, std::integral_constant<int, 2>{}, p, I.B0, 1, tile_rows, c1,
                 2, ncol);
    }
    lds_barrier();
    // the tile's rows of this plane (compression leaves the codes of coarse
    // points, written at earlier levels, as they are)
    if (lane < tcn) {
      const uint32_t qc = I.C0 + lane, colt = qc * fc;
      const uint32_t bk0 = (I.B0 - I.Bo) * kPitch + (qc - I.Co);
      const bool even_pc = (p & 1u) == 0 && (qc & 1u) == 0;
#pragma unroll
      for (uint32_t k = 0; k < kRowsPerWave; k++) {
        const uint32_t r = wave + kLevelWaves * k;
        if (r < tile_rows) {
          const uint32_t qb = I.B0 + r;
          const uint32_t f = p * fa + qb * fb + colt;
          const uint32_t bk = bk0 + r * kPitch;
          if (!RECON && !(even_pc && (qb & 1u) == 0)) codes[f] = lcode[bk];
          if (store_v) v[f] = box[bk];
          if (store_c) cmp[((size_t)p * g.ext[1] + qb) * g.ext[2] + qc] = box[bk];
        }
      }
    }
    lds_barrier();  // the box is refilled next
  }
}

template <typename T, int PRED, bool RECON>
__global__ __launch_bounds__(kLevelThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_level64(
    const T* __restrict__ x, T* v, uint16_t* codes, LevelGeom g, const Meta* __restrict__ m,
    T twoeb, uint32_t R, uint32_t flags, T* cmp) {
  level64_body<T, PRED, RECON>(x, v, codes, g, m, twoeb, R, flags, cmp, blockIdx.x);
}

// Compression of one level of several fields (a batch): each job is a field's
// level, with its geometry and store flags.
template <typename T, int PRED>
__global__ __launch_bounds__(kLevelThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_b_level64(
    BLaunch L) {
  BJob j;
  uint32_t local;
  if (!batch_job(L, j, local)) return;
  const BField& f = L.f[j.field];
  level64_body<T, PRED, false>(static_cast<const T*>(f.x), static_cast<T*>(f.rec), f.codes, j.g,
                               f.m, T(0), f.R, j.flags, static_cast<T*>(f.cmp), local);
}

// ------------------------------------------------------------------ host side

namespace {
uint32_t ceil_div32(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }
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
  // Without a tuning, a level with few work items under the default tiling
  // (a coarse level of a large field, or a small field) takes shorter (b, c)
  // tiles: more workgroups, more halo work (measured per stride on 512^3:
  // strides 16 and 8 gain a fifth, stride 4 and finer lose).  Tiles never
  // change the bytes.
  const LevelTuning def{2048, 32, 58, 64 * 1024, 1, 0};
  const LevelTuning few{4096, 16, 58, 64 * 1024, 1, 0};
  const LevelTuning fewer{8192, 8, 58, 64 * 1024, 1, 0};
  for (int l = L; l >= 1; l--) {
    const uint64_t s = 1ull << (l - 1);
    const LevelTuning* pick = tune ? tune : &def;
    if (!tune && s >= 8) {
      const uint64_t items32 = (uint64_t)ceil_div32((V[O[1]] - 1) / s + 1, 32) *
                               ceil_div32((V[O[2]] - 1) / s + 1, 58) *
                               ceil_div32((V[O[0]] - 1) / s + 1, 2);
      if (items32 < 64) pick = &fewer;
      else if (items32 < 256) pick = &few;
    }
    const LevelTuning& tu = *pick;
    LevelGeom g{};
    g.s = (uint32_t)s;
    for (int j = 0; j < 3; j++) {
      g.ext[j] = (uint32_t)((V[O[j]] - 1) / s + 1);
      g.fs[j] = VS[O[j]] * s;
    }
    // (b, c) tile: 58 columns make the box rows 64 wide (one unit); a single
    // row (one-dimensional fields) takes as many columns as the units allow
    uint32_t TB = std::min<uint32_t>(g.ext[1], tu.tile_b);
    uint32_t TC = std::min<uint32_t>(g.ext[2], tu.tile_c);
    if (g.ext[1] == 1)
      TC = std::min<uint32_t>(g.ext[2], kBoxUnits * kLevelWaves * 64 - 2 * kHalo);
    auto fits = [&](uint32_t tb, uint32_t tcx) {
      const uint32_t bb = std::min<uint32_t>(tb + 2 * kHalo, g.ext[1]);
      const uint32_t bc = std::min<uint32_t>(tcx + 2 * kHalo, g.ext[2]);
      const uint32_t ncc = (bc + 63) / 64;
      const uint32_t rb = (bb + 1) / 2, rc = (bc + 1) / 2;
      const uint64_t lds = ((uint64_t)(bb * bc + 1) * tsize + 15) / 16 * 16 +
                           ((uint64_t)4 * rb * rc * tsize + 15) / 16 * 16 + (uint64_t)(bb * bc + 1) * 2;
      return (uint64_t)bb * ncc <= (uint64_t)kBoxUnits * kLevelWaves &&
             (uint64_t)rb * ncc <= (uint64_t)kGridUnits * kLevelWaves && lds <= tu.lds_bytes;
    };
    while (!fits(TB, TC)) {
      if (TB > 1)
        TB = (TB + 1) / 2;
      else if (TC > 1)
        TC = (TC + 1) / 2;
      else
        return false;
    }
    g.tile[1] = TB;
    g.tile[2] = TC;
    g.ntile[1] = ceil_div32(g.ext[1], TB);
    g.ntile[2] = ceil_div32(g.ext[2], TC);
    // planes per item: even runs, shortened until there are enough items
    uint32_t P = g.ext[0] > 1 ? std::min<uint32_t>(16, (g.ext[0] + 1) & ~1u) : 1u;
    while (P > 2 && (uint64_t)g.ntile[1] * g.ntile[2] * ceil_div32(g.ext[0], P) < tu.target_points)
      P = std::max<uint32_t>(2, (P / 2 + 1) & ~1u);
    g.planes = P;
    g.tile[0] = P;
    g.ntile[0] = ceil_div32(g.ext[0], P);
    g.box_b = std::min<uint32_t>(TB + 2 * kHalo, g.ext[1]);
    g.box_c = std::min<uint32_t>(TC + 2 * kHalo, g.ext[2]);
    g.ring_b = (g.box_b + 1) / 2;
    g.ring_c = (g.box_c + 1) / 2;
    g.nitems = (uint64_t)g.ntile[0] * g.ntile[1] * g.ntile[2];
    // boxes of up to 64 columns (and kMaxBoxRows64 rows) take the fixed-pitch
    // kernel; the box and the codes carry one spare slot (writes of padding lanes)
    g.pitch64 = g.ext[1] > 1 && g.box_c <= kPitch && g.box_b <= kMaxBoxRows64 ? 1u : 0u;
    const uint32_t bc = g.pitch64 ? kPitch : g.box_c, rc = g.pitch64 ? kRingPitch : g.ring_c;
    g.box_bytes = (uint32_t)(((uint64_t)(g.box_b * bc + 1) * tsize + 15) / 16 * 16);
    g.ring_bytes = (uint32_t)(((uint64_t)4 * g.ring_b * rc * tsize + 15) / 16 * 16);
    g.lds = g.box_bytes + g.ring_bytes + (g.box_b * bc + 1) * 2;
    if (g.nitems > 0x7FFFFFFFull) return false;
    if (tu.fine) plan_fine(g, tsize, tu.fine_rows);
    out.push_back(g);
  }
  return true;
}

template <typename T, bool RECON>
static hipError_t launch_level_t(const void* x, int predictor, void* v, uint16_t* codes,
                                 const LevelGeom& g, const Meta* m, double eb_t, uint32_t R,
                                 uint32_t flags, void* cmp, hipStream_t st) {
  if (g.nitems == 0) return hipSuccess;
  dim3 grid((unsigned)g.nitems), block(kLevelThreads);
  const T twoeb = RECON ? (T)2 * (T)eb_t : T(0);
  const uint32_t lds = RECON ? g.box_bytes + g.ring_bytes : g.lds;
  if (g.pitch64) {
    if (predictor == SZ_INTERP_CUBIC)
      hipLaunchKernelGGL((k_level64<T, SZ_INTERP_CUBIC, RECON>), grid, block, lds, st,
                         (const T*)x, (T*)v, codes, g, m, twoeb, R, flags, (T*)cmp);
    else
      hipLaunchKernelGGL((k_level64<T, SZ_INTERP_LINEAR, RECON>), grid, block, lds, st,
                         (const T*)x, (T*)v, codes, g, m, twoeb, R, flags, (T*)cmp);
  } else if (predictor == SZ_INTERP_CUBIC) {
    hipLaunchKernelGGL((k_level<T, SZ_INTERP_CUBIC, RECON>), grid, block, lds, st, (const T*)x,
                       (T*)v, codes, g, m, twoeb, R, flags);
  } else {
    hipLaunchKernelGGL((k_level<T, SZ_INTERP_LINEAR, RECON>), grid, block, lds, st, (const T*)x,
                       (T*)v, codes, g, m, twoeb, R, flags);
  }
  return hipGetLastError();
}

hipError_t launch_level_compress(const void* x, int dtype, int predictor, void* rec,
                                 uint16_t* codes, const LevelGeom& g, const Meta* m,
                                 uint32_t radius, bool store_rec, void* cmp, hipStream_t st) {
  // (the strip kernel stores no reconstruction: it runs the last level only)
  if (!store_rec && fine_usable(g, dtype, x, rec))
    return launch_fine_compress(x, dtype, predictor, rec, codes, g, m, radius, cmp, st);
  // the stride-2 level with a compact lattice: stored there instead of the field
  const bool compact = cmp && g.s == 2 && g.pitch64;
  const uint32_t flags =
      compact ? kLevelStoreCompact : (store_rec ? kLevelStoreValues : 0u);
  if (dtype == SZ_F32)
    return launch_level_t<float, false>(x, predictor, rec, codes, g, m, 0.0, radius, flags,
                                        compact ? cmp : nullptr, st);
  return launch_level_t<double, false>(x, predictor, rec, codes, g, m, 0.0, radius, flags,
                                       compact ? cmp : nullptr, st);
}

hipError_t launch_b_level(int dtype, int predictor, BLaunch L, uint32_t nwg, uint32_t lds,
                          hipStream_t st) {
  if (nwg == 0) return hipSuccess;
  if (dtype == SZ_F32) {
    if (predictor == SZ_INTERP_CUBIC)
      hipLaunchKernelGGL((k_b_level64<float, SZ_INTERP_CUBIC>), dim3(nwg), dim3(kLevelThreads), lds,
                         st, L);
    else
      hipLaunchKernelGGL((k_b_level64<float, SZ_INTERP_LINEAR>), dim3(nwg), dim3(kLevelThreads),
                         lds, st, L);
  } else {
    if (predictor == SZ_INTERP_CUBIC)
      hipLaunchKernelGGL((k_b_level64<double, SZ_INTERP_CUBIC>), dim3(nwg), dim3(kLevelThreads),
                         lds, st, L);
    else
      hipLaunchKernelGGL((k_b_level64<double, SZ_INTERP_LINEAR>), dim3(nwg), dim3(kLevelThreads),
                         lds, st, L);
  }
  return hipGetLastError();
}

hipError_t launch_level_recon(const uint16_t* codes, int dtype, int predictor, void* out,
                              const LevelGeom& g, double eb_t, uint32_t radius, void* cmp,
                              hipStream_t st) {
  // the tile is stored whole (its coarse points too, unchanged), so that the
  // output rows are written by one workgroup
  if (fine_usable(g, dtype, out, out))
    return launch_fine_recon(codes, dtype, predictor, out, g, eb_t, radius, cmp, st);
  const bool compact = cmp && g.s == 2 && g.pitch64;
  const uint32_t flags = compact ? kLevelStoreCompact : kLevelStoreValues;
  uint16_t* c = const_cast<uint16_t*>(codes);  // only read when reconstructing
  if (dtype == SZ_F32)
    return launch_level_t<float, true>(nullptr, predictor, out, c, g, nullptr, eb_t, radius,
                                       flags, compact ? cmp : nullptr, st);
  return launch_level_t<double, true>(nullptr, predictor, out, c, g, nullptr, eb_t, radius,
                                      flags, compact ? cmp : nullptr, st);
}

}  // namespace szg
