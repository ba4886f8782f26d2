// The finest level (stride 1) of three-dimensional fields as row strips held
// in registers: no LDS box, one barrier per row pair.
//
// Paper: SZ3 (arXiv 2111.02925), Section 6.2 (SZ3-Interp): a level predicts
// its points dimension by dimension, each from reconstructed neighbours at
// +-1 and +-3 along the pass's dimension; Algorithm 1 quantizes point by
// point in that order.  Any schedule that computes every point after the
// points its stencil reads gives the same values; this one is chosen for the
// memory system.
//
// In the level's lattice (dimensions a, b, c in pass order, c contiguous in
// memory) the points are
//   pass along a: a odd, b even, c even  (reads even planes: coarse points)
//   pass along b: a any, b odd,  c even  (reads even rows, same plane)
//   pass along c: a any, b any,  c odd   (reads even columns, same row)
// so the even column of every row is final before the row's pass along c,
// and the even columns of the even rows are final before the pass along b.
//
// A lane owns one (even, odd) column pair; a wave covers 128 columns, and a
// workgroup of up to four waves covers up to 512 (a window).  A workgroup
// takes A consecutive planes and a run of rows, and walks the rows two at a
// time: at step i the even row e = B0 - 2 + 2i and the odd row o = e - 3.
//   even row: even column from the coarse grid (even planes) or the pass
//             along a (odd planes, from the coarse points of planes a +- 1,
//             a +- 3 at the same row and column, read for the A planes and
//             three more around them),
//   odd row:  even column by the pass along b, from the even columns of rows
//             o +- 1, o +- 3 of the same plane (kept in registers: the last
//             four even rows),
//   both:     the odd column by the pass along c, from the even columns of
//             the lane and its neighbours (lanes l - 1, l + 1, l + 2: DPP
//             moves inside the wave, the values at the wave's ends through
//             LDS from the neighbouring waves).
// Rows just outside the run (three even rows) and columns just outside the
// window's owned range are computed with the same arithmetic as by their
// owner and not stored, so the results agree bit for bit.  The loads of the
// next row are in flight while the current one computes.
#include "block_ops.h"
#include "common.h"
#include "device_math.h"

namespace szg {

constexpr uint32_t kFineMaxWaves = 4;
constexpr uint32_t kFineCols = 128;  // columns of one wave

template <typename T>
struct PairOf;
template <>
struct PairOf<float> {
  using type = float2;
};
template <>
struct PairOf<double> {
  using type = double2;
};

// Lane moves across the whole wave: shr gives lane l the value of lane l - 1,
// shl that of lane l + 1; the lane without a source keeps `edge`.
__device__ __forceinline__ int dpp_wave_shr1(int edge, int v) {
  return __builtin_amdgcn_update_dpp(edge, v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_wave_shl1(int edge, int v) {
  return __builtin_amdgcn_update_dpp(edge, v, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ float shr1(float edge, float v) {
  return __int_as_float(dpp_wave_shr1(__float_as_int(edge), __float_as_int(v)));
}
__device__ __forceinline__ float shl1(float edge, float v) {
  return __int_as_float(dpp_wave_shl1(__float_as_int(edge), __float_as_int(v)));
}
__device__ __forceinline__ double shr1(double edge, double v) {
  const long long e = __double_as_longlong(edge), x = __double_as_longlong(v);
  const int lo = dpp_wave_shr1((int)e, (int)x), hi = dpp_wave_shr1((int)(e >> 32), (int)(x >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double shl1(double edge, double v) {
  const long long e = __double_as_longlong(edge), x = __double_as_longlong(v);
  const int lo = dpp_wave_shl1((int)e, (int)x), hi = dpp_wave_shl1((int)(e >> 32), (int)(x >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Stores through buffer resources: a lane that stores nothing gives an
// offset past the buffer's end (the hardware drops the write), so every path
// through the loop issues the same memory instructions and the waits for the
// loads in flight stay exact.  Buffers span less than 2^31 bytes.
constexpr uint32_t kOffNone = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(void* base, uint32_t bytes) {
  // (wave-uniform operands, taken as such: the resource lives in scalar registers)
  const uint64_t b = (uint64_t)base;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  void* p = (void*)(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(p, 0, (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}
__device__ __forceinline__ void store_b16(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v, r, (int)off, 0, 0);
}
__device__ __forceinline__ void store_b32(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)off, 0, 0);
}
__device__ __forceinline__ void store_pair(__amdgpu_buffer_rsrc_t r, uint32_t off, float a, float b) {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  u2 d = {__float_as_uint(a), __float_as_uint(b)};
  __builtin_amdgcn_raw_buffer_store_b64(d, r, (int)off, 0, 0);
}
__device__ __forceinline__ void store_pair(__amdgpu_buffer_rsrc_t r, uint32_t off, double a, double b) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const unsigned long long x = (unsigned long long)__double_as_longlong(a),
                           y = (unsigned long long)__double_as_longlong(b);
  u4 d = {(unsigned)x, (unsigned)(x >> 32), (unsigned)y, (unsigned)(y >> 32)};
  __builtin_amdgcn_raw_buffer_store_b128(d, r, (int)off, 0, 0);
}

// The verbatim value of an unpredictable point (reconstruction), read where
// it is needed: the empty asm takes the load there, so that the common path
// never waits on it.
template <typename T>
__device__ __forceinline__ T verbatim(const T* v, uint32_t f) {
  T w = v[f];
  asm volatile("" : "+v"(w));
  return w;
}

// Column window `win` of a row: its first column Cw and the owned columns
// [O0, O1).  Windows after the first start two columns before the columns
// they own (the pass along c of their first owned column reads column O0 - 2)
// and own all but the last four columns of the window (the last owned column
// reads up to three columns further).
struct Window {
  uint32_t Cw, O0, O1;
};
__host__ __device__ inline Window fine_window(uint32_t win, uint32_t nwin, uint32_t width,
                                              uint32_t E2) {
  Window w;
  w.Cw = win == 0 ? 0u : (width - 4) + (win - 1) * (width - 6) - 2;
  w.O0 = win == 0 ? 0u : w.Cw + 2;
  w.O1 = win + 1 == nwin ? E2 : w.Cw + width - 4;
  return w;
}

template <typename T, int PRED, bool RECON, int A>
__device__ __forceinline__ void fine_body(const T* __restrict__ x, T* v, uint16_t* codes,
                                          const LevelGeom& g, const Meta* __restrict__ m, T twoeb,
                                          uint32_t R, const T* __restrict__ cmp, uint32_t bid) {
  static_assert(A % 2 == 0, "plane groups start on even planes");
  constexpr int NC = A / 2 + 3;  // coarse planes A0 - 2, A0, ..., A0 + A + 2
  using P = typename PairOf<T>::type;
  // the values of lanes 0, 1 and 63 of every wave, for the even and the odd row
  __shared__ T xch[2][kFineMaxWaves][2][3][A];

  const uint32_t E0 = g.ext[0], E1 = g.ext[1], E2 = g.ext[2];
  const uint32_t fa = (uint32_t)g.fs[0], fb = (uint32_t)g.fs[1];
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
  const uint32_t nw = g.f_waves;

  // ---- the work item: XCD-aware order (workgroups are dealt to the 8 dies
  // round-robin; each die takes a contiguous range of items).  Plane groups
  // vary fastest: neighbouring groups read three coarse planes in common, at
  // the same rows at about the same time, so the second read hits the die's L2
  uint32_t t = bid;
  {
    const uint32_t full = g.f_items & ~7u;
    if (t < full) t = (t & 7) * (full >> 3) + (t >> 3);
  }
  const uint32_t at = t % g.f_atiles;
  t /= g.f_atiles;
  const uint32_t run = t % g.f_runs;
  const uint32_t win = t / g.f_runs;
  const Window W = fine_window(win, g.f_wins, kFineCols * nw, E2);
  const uint32_t A0 = at * A;
  const uint32_t B0 = run * g.f_rows, B1 = min(B0 + g.f_rows, E1);

  // ---- this lane's column pair (lanes past the field repeat the last pair)
  const uint32_t wc0 = W.Cw + kFineCols * wave;
  const uint32_t ce_raw = wc0 + 2 * lane;
  const uint32_t ce = min(ce_raw, E2 - 2);
  const bool own_col = ce_raw >= W.O0 && ce_raw < W.O1;
  // the pass along c at column ce + 1 reads ce - 2, ce, ce + 2, ce + 4
  const bool c_has_a = ce >= 2, c_has_c = ce + 2 < E2, c_has_e = ce + 4 < E2;
  const bool c_int = wc0 >= 2 && wc0 + 130 < E2;  // every lane of the wave has all four
  const uint32_t wl = wave > 0 ? wave - 1 : 0u, wr = wave + 1 < nw ? wave + 1 : wave;
  // stores of the plane group, relative to its first plane: up to the end of
  // its last plane's last row (a group's rows lie far apart when the planes
  // are not the field's outer dimension)
  const uint32_t g_na = min(E0 - min(A0, E0), (uint32_t)A);
  const uint32_t g_elems = g_na ? (g_na - 1) * fa + (E1 - 1) * fb + E2 : 0u;
  const uint32_t g_bytes = g_elems * (uint32_t)(RECON ? sizeof(T) : 2);
  const __amdgpu_buffer_rsrc_t out_buf =
      RECON ? buffer_of(v + (size_t)A0 * fa, g_bytes) : buffer_of(codes + (size_t)A0 * fa, g_bytes);

  auto clamp_row = [&](int32_t r) -> uint32_t {
    return (uint32_t)(r < 0 ? 0 : (r >= (int32_t)E1 ? (int32_t)E1 - 1 : r));
  };
  auto clamp_plane = [&](int32_t a) -> uint32_t {
    return (uint32_t)(a < 0 ? 0 : (a >= (int32_t)E0 ? (int32_t)E0 - 1 : a));
  };

  // ---- loads (clamped to the field: values of rows and planes outside it
  // are never used)
  T cv[NC];                           // coarse points of the even row
  P xe[A], xo[A];                     // compression: field values of the even / odd row
  uint32_t ke[A], ko[A];              // reconstruction: code pairs of the even / odd row
  // Rows whose values are not needed still issue their loads (the waits count
  // alike on every path), at an address read by the same step: no traffic.
  // Even rows outside the run feed only the pass along a of odd planes.
  // Coarse points come from the compact stride-2 lattice when the stride-2
  // level stored one (cmp; lattice extents ceil(E/2), the lanes' even columns
  // adjacent there), else from the field (every other column of a line).
  const uint32_t M1 = (E1 + 1) / 2, M2 = (E2 + 1) / 2;
  const T* __restrict__ csrc = cmp ? cmp : v;
  auto issue_even = [&](int32_t e) {
    const uint32_t er = clamp_row(e);
    const uint32_t r = er * fb + ce;
    const bool own = e >= (int32_t)B0 && e < (int32_t)B1;
#pragma unroll
    for (int k = 0; k < NC; k++) {
      const uint32_t a = clamp_plane((int32_t)A0 - 2 + 2 * k);
      const size_t ci = cmp ? ((size_t)(a >> 1) * M1 + (er >> 1)) * M2 + (ce >> 1)
                            : (size_t)(a * fa + r);
      cv[k] = csrc[ci];
    }
#pragma unroll
    for (int j = 0; j < A; j++) {
      const int jj = (j % 2 == 0 && !own) ? j + 1 : j;
      const uint32_t f = clamp_plane((int32_t)(A0 + jj)) * fa + r;
      if (RECON)
        ke[j] = *reinterpret_cast<const uint32_t*>(codes + f);
      else
        xe[j] = *reinterpret_cast<const P*>(x + f);
    }
  };
  // Odd rows outside the run are not needed at all: they read the even row
  // e = o + 3, loaded one step earlier.
  auto issue_odd = [&](int32_t o) {
    const bool own = o >= (int32_t)B0 && o < (int32_t)B1;
    const uint32_t r = clamp_row(own ? o : o + 3) * fb + ce;
#pragma unroll
    for (int j = 0; j < A; j++) {
      const uint32_t f = clamp_plane((int32_t)(A0 + j)) * fa + r;
      if (RECON)
        ko[j] = *reinterpret_cast<const uint32_t*>(codes + f);
      else
        xo[j] = *reinterpret_cast<const P*>(x + f);
    }
  };

  // ---- the even columns of the last four even rows, per plane
  T w0[A], w1[A], w2[A], w3[A];
#pragma unroll
  for (int j = 0; j < A; j++) w0[j] = w1[j] = w2[j] = w3[j] = T(0);

  uint32_t par = 0;
  const uint32_t nit = (B1 - B0 + 1) / 2 + 3;
  // Each step issues the next even row's loads after its even row, and the
  // next odd row's after its odd row, each ahead of a whole half step; the
  // entry mimics a step's order of loads and stores, so that the waits count
  // alike on the first step and the later ones.
  issue_even((int32_t)B0 - 2);
  issue_odd((int32_t)B0 - 5);
#pragma unroll
  for (int j = 0; j < 2 * A; j++) store_b32(out_buf, kOffNone + 4 * j, 0u);
  for (uint32_t i = 0; i < nit; i++) {
    const int32_t e = (int32_t)B0 - 2 + 2 * (int32_t)i, o = e - 3;
    const bool e_in = e >= 0 && e < (int32_t)E1;
    const bool e_own = e >= (int32_t)B0 && e < (int32_t)B1;
    const bool o_own = o >= (int32_t)B0 && o < (int32_t)B1;

    // -- even row: the even column (coarse, or the pass along a)
    T ev[A], xeo[A];
    uint32_t kce[A];  // compression: codes of the even column (odd planes)
#pragma unroll
    for (int j = 0; j < A; j++) {
      ev[j] = T(0);
      xeo[j] = T(0);
      kce[j] = 0;
    }
    if (e_in) {
      const uint32_t fr = (uint32_t)e * fb + ce;
#pragma unroll
      for (int j = 0; j < A; j++) {
        const uint32_t a = A0 + j;
        if (j % 2 == 0) {
          ev[j] = cv[j / 2 + 1];
        } else {
          const int k = (j - 1) / 2;  // planes a - 3, a - 1, a + 1, a + 3
          const bool a_int = a >= 3 && a + 3 < E0;
          const T pred =
              a_int ? interp_predict<T, PRED>(cv[k], cv[k + 1], cv[k + 2], cv[k + 3], true, true, true)
                    : interp_predict_sel<T, PRED>(cv[k], cv[k + 1], cv[k + 2], cv[k + 3], a >= 3,
                                                  a + 1 < E0, a + 3 < E0);
          if (RECON) {
            const uint32_t code = ke[j] & 0xFFFFu;
            ev[j] = code ? recover(pred, q.twoeb, code, q.R)
                         : verbatim(v, clamp_plane((int32_t)a) * fa + fr);
          } else {
            kce[j] = quantize(xe[j].x, pred, q, ev[j]);
          }
        }
        if (RECON)
          kce[j] = ke[j] >> 16;  // the odd column's code
        else
          xeo[j] = xe[j].y;
      }
    }
    // every loaded register is taken here, on every path, before it is
    // loaded again
#pragma unroll
    for (int j = 0; j < A; j++) {
      if (RECON)
        asm volatile("" ::"v"(ke[j]));
      else
        asm volatile("" ::"v"(xe[j].x), "v"(xe[j].y));
    }
#pragma unroll
    for (int k = 0; k < NC; k++) asm volatile("" ::"v"(cv[k]));
    issue_even(e + 2);  // (past the run on the last step: clamped, unused)

    // the window moves to rows e - 6, e - 4, e - 2, e = o - 3, o - 1, o + 1, o + 3
#pragma unroll
    for (int j = 0; j < A; j++) {
      w0[j] = w1[j];
      w1[j] = w2[j];
      w2[j] = w3[j];
      w3[j] = ev[j];
    }

    // -- odd row: the even column by the pass along b
    T ov[A], xoo[A];
    uint32_t kco[A], koo[A];
#pragma unroll
    for (int j = 0; j < A; j++) {
      ov[j] = T(0);
      kco[j] = 0;
      xoo[j] = T(0);
      koo[j] = 0;
    }
    if (o_own) {
      const uint32_t fr = (uint32_t)o * fb + ce;
      const bool ha = o >= 3, hc = o + 1 < (int32_t)E1, he = o + 3 < (int32_t)E1;
      const bool b_int = ha && he;  // (he implies hc)
#pragma unroll
      for (int j = 0; j < A; j++) {
        const T pred = b_int ? interp_predict<T, PRED>(w0[j], w1[j], w2[j], w3[j], true, true, true)
                             : interp_predict_sel<T, PRED>(w0[j], w1[j], w2[j], w3[j], ha, hc, he);
        if (RECON) {
          const uint32_t code = ko[j] & 0xFFFFu;
          ov[j] = code ? recover(pred, q.twoeb, code, q.R)
                       : verbatim(v, clamp_plane((int32_t)(A0 + j)) * fa + fr);
        } else {
          kco[j] = quantize(xo[j].x, pred, q, ov[j]);
        }
        if (RECON)
          koo[j] = ko[j] >> 16;  // the odd column's code
        else
          xoo[j] = xo[j].y;
      }
    }
#pragma unroll
    for (int j = 0; j < A; j++) {
      if (RECON)
        asm volatile("" ::"v"(ko[j]));
      else
        asm volatile("" ::"v"(xo[j].x), "v"(xo[j].y));
    }
    issue_odd(o + 2);  // (past the run on the last step: unused)

    // -- the values at the wave's ends, to and from the neighbouring waves
    if (nw > 1) {
      if (lane <= 1 || lane == 63) {
        const uint32_t slot = lane == 63 ? 2u : lane;
#pragma unroll
        for (int j = 0; j < A; j++) {
          xch[par][wave][0][slot][j] = ev[j];
          xch[par][wave][1][slot][j] = ov[j];
        }
      }
      lds_barrier();
    }

    // -- the pass along c on the odd column of a row (rows outside the run
    // issue as many stores, all dropped: every step issues the same stores)
    auto pass_c = [&](const T (&val)[A], int rsel, int32_t row, bool own_row,
                      const T (&xodd)[A], const uint32_t (&kodd)[A], const uint32_t (&keven)[A],
                      bool even_row) {
      if (!own_row) {
#pragma unroll
        for (int j = 0; j < A; j++) store_b32(out_buf, kOffNone + 4 * j, 0u);
        return;
      }
      const uint32_t fr = clamp_row(row) * fb + ce;
#pragma unroll
      for (int j = 0; j < A; j++) {
        const uint32_t a = A0 + j;
        T Lv = val[j], R0 = val[j], R1 = val[j];
        if (nw > 1) {
          Lv = xch[par][wl][rsel][2][j];
          R0 = xch[par][wr][rsel][0][j];
          R1 = xch[par][wr][rsel][1][j];
        }
        const T left = shr1(Lv, val[j]);
        const T r1 = shl1(R0, val[j]);
        const T r2 = shl1(R1, r1);
        const T pred = c_int ? interp_predict<T, PRED>(left, val[j], r1, r2, true, true, true)
                             : interp_predict_sel<T, PRED>(left, val[j], r1, r2, c_has_a,
                                                           c_has_c, c_has_e);
        const bool store = own_col && a < E0;
        const uint32_t fg = (uint32_t)j * fa + fr;  // relative to the plane group
        if (RECON) {
          const uint32_t code = kodd[j];
          const T val_o = code ? recover(pred, q.twoeb, code, q.R)
                               : verbatim(v, clamp_plane((int32_t)a) * fa + fr + 1);
          store_pair(out_buf, store ? fg * (uint32_t)sizeof(T) : kOffNone, val[j], val_o);
        } else {
          T rec;
          const uint32_t code = quantize(xodd[j], pred, q, rec);
          if (even_row && j % 2 == 0)  // the even column is a coarse point: its code stays
            store_b16(out_buf, store ? 2 * fg + 2 : kOffNone, code);
          else
            store_b32(out_buf, store ? 2 * fg : kOffNone, (keven[j] & 0xFFFFu) | (code << 16));
        }
      }
    };
    pass_c(ev, 0, e, e_own, xeo, kce, kce, true);
    pass_c(ov, 1, o, o_own, xoo, koo, kco, false);
    par ^= 1u;
  }
}

template <typename T, int PRED, bool RECON, int A>
__global__ __launch_bounds__(kFineMaxWaves * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_fine(
    const T* __restrict__ x, T* v, uint16_t* codes, LevelGeom g, const Meta* __restrict__ m,
    T twoeb, uint32_t R, const T* __restrict__ cmp) {
  fine_body<T, PRED, RECON, A>(x, v, codes, g, m, twoeb, R, cmp, blockIdx.x);
}

// The stride-1 level of several fields (a batch) with the same number of
// waves per workgroup: each job is a field's stride-1 level.
template <typename T, int PRED, int A>
__global__ __launch_bounds__(kFineMaxWaves * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_b_fine(
    BLaunch L) {
  BJob j;
  uint32_t local;
  if (!batch_job(L, j, local)) return;
  const BField& f = L.f[j.field];
  fine_body<T, PRED, false, A>(static_cast<const T*>(f.x), static_cast<T*>(f.rec), f.codes, j.g,
                               f.m, T(0), f.R, static_cast<const T*>(f.cmp), local);
}

// ------------------------------------------------------------------ host side

namespace {
uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }
}  // namespace

int fine_planes(int tsize) { return tsize == 4 ? 8 : 4; }

bool plan_fine(LevelGeom& g, int tsize, uint32_t rows) {
  g.fine = 0;
  const uint32_t E0 = g.ext[0], E1 = g.ext[1], E2 = g.ext[2];
  if (g.s != 1 || g.fs[2] != 1 || E0 < 2 || E1 < 2 || E2 < 4 || (E2 & 1u)) return false;
  // a plane group's stores are addressed from its first plane and span less
  // than 2^31 bytes (buffer offsets): from there to the end of its last
  // plane's last row, whichever of the two outer dimensions the planes are
  const uint64_t span = (uint64_t)(fine_planes(tsize) - 1) * g.fs[0] + (uint64_t)(E1 - 1) * g.fs[1] + E2;
  if (span * (uint64_t)tsize >= 0x7FFF0000ull) return false;
  const uint32_t nw = std::min<uint32_t>(kFineMaxWaves, cdiv(E2, kFineCols));
  const uint32_t width = kFineCols * nw;
  uint32_t nwin = 1;
  while (fine_window(nwin - 1, nwin + 1, width, E2).Cw + width < E2) nwin++;
  const uint32_t A = (uint32_t)fine_planes(tsize);
  const uint32_t natiles = cdiv(E0, A);
  // rows per run: the longest (even) run that still gives enough waves
  if (rows == 0) {
    rows = 32;
    while (rows > 8 && (uint64_t)nwin * natiles * cdiv(E1, rows) * nw < 4096) rows /= 2;
  }
  rows = (rows + 1) & ~1u;
  g.f_waves = nw;
  g.f_wins = nwin;
  g.f_atiles = natiles;
  g.f_rows = rows;
  g.f_runs = cdiv(E1, rows);
  const uint64_t items = (uint64_t)nwin * natiles * g.f_runs;
  if (items > 0x7FFFFFFFull) return false;
  g.f_items = (uint32_t)items;
  g.fine = 1;
  return true;
}

template <typename T, bool RECON, int A>
static hipError_t launch_fine_t(const void* x, int predictor, void* v, uint16_t* codes,
                                const LevelGeom& g, const Meta* m, double eb_t, uint32_t R,
                                const void* cmp, hipStream_t st) {
  dim3 grid(g.f_items), block(64 * g.f_waves);
  const T twoeb = RECON ? (T)2 * (T)eb_t : T(0);
  if (predictor == SZ_INTERP_CUBIC)
    hipLaunchKernelGGL((k_fine<T, SZ_INTERP_CUBIC, RECON, A>), grid, block, 0, st, (const T*)x,
                       (T*)v, codes, g, m, twoeb, R, (const T*)cmp);
  else
    hipLaunchKernelGGL((k_fine<T, SZ_INTERP_LINEAR, RECON, A>), grid, block, 0, st, (const T*)x,
                       (T*)v, codes, g, m, twoeb, R, (const T*)cmp);
  return hipGetLastError();
}

bool fine_usable(const LevelGeom& g, int dtype, const void* x, const void* v) {
  if (!g.fine) return false;
  const uintptr_t pair = dtype == SZ_F32 ? 8 : 16;
  return ((uintptr_t)x % pair) == 0 && ((uintptr_t)v % pair) == 0;
}

hipError_t launch_fine_compress(const void* x, int dtype, int predictor, void* rec,
                                uint16_t* codes, const LevelGeom& g, const Meta* m,
                                uint32_t radius, const void* cmp, hipStream_t st) {
  if (g.f_items == 0) return hipSuccess;
  if (dtype == SZ_F32)
    return launch_fine_t<float, false, 8>(x, predictor, rec, codes, g, m, 0.0, radius, cmp, st);
  return launch_fine_t<double, false, 4>(x, predictor, rec, codes, g, m, 0.0, radius, cmp, st);
}

hipError_t launch_b_fine(int dtype, int predictor, uint32_t waves, BLaunch L, uint32_t nwg,
                         hipStream_t st) {
  if (nwg == 0) return hipSuccess;
  dim3 grid(nwg), block(64 * waves);
  if (dtype == SZ_F32) {
    if (predictor == SZ_INTERP_CUBIC)
      hipLaunchKernelGGL((k_b_fine<float, SZ_INTERP_CUBIC, 8>), grid, block, 0, st, L);
    else
      hipLaunchKernelGGL((k_b_fine<float, SZ_INTERP_LINEAR, 8>), grid, block, 0, st, L);
  } else {
    if (predictor == SZ_INTERP_CUBIC)
      hipLaunchKernelGGL((k_b_fine<double, SZ_INTERP_CUBIC, 4>), grid, block, 0, st, L);
    else
      hipLaunchKernelGGL((k_b_fine<double, SZ_INTERP_LINEAR, 4>), grid, block, 0, st, L);
  }
  return hipGetLastError();
}

hipError_t launch_fine_recon(const uint16_t* codes, int dtype, int predictor, void* out,
                             const LevelGeom& g, double eb_t, uint32_t radius, const void* cmp,
                             hipStream_t st) {
  if (g.f_items == 0) return hipSuccess;
  uint16_t* c = const_cast<uint16_t*>(codes);  // only read when reconstructing
  if (dtype == SZ_F32)
    return launch_fine_t<float, true, 8>(nullptr, predictor, out, c, g, nullptr, eb_t, radius,
                                         cmp, st);
  return launch_fine_t<double, true, 4>(nullptr, predictor, out, c, g, nullptr, eb_t, radius,
                                        cmp, st);
}

}  // namespace szg
