// Paired Fourier-domain block products for reciprocal coupling operators.
//
// The free-space Green's function is reciprocal: the coupling from a source
// unknown to a test unknown is unchanged when the two trade places, up to the
// source weights of the discretisation (the patch areas of the point-sampled
// fill).  The generating blocks of Sec. IV-A therefore satisfy
//     T(-d) = W^-1 T(d)^T W          (W diagonal, one weight per unknown),
// and under the circulant embedding of Sec. IV-B the negated offset becomes
// the negated frequency:
//     That[-k] = W^-1 That[k]^T W.
// A reciprocal plan keeps one block per pair {k, -k} (half the Fourier-domain
// store, half the HBM traffic of the block products).  One workgroup per pair
// streams That[k] once and forms both products of the pair:
//     yh[k]  = That[k] xh[k]
//     yh[-k] = W^-1 That[k]^T (W xh[-k])
// Self-paired frequencies (2k = 0 modulo the padded lengths) form only the
// first.
//
// Both precisions run on the matrix cores (v_mfma_f32_16x16x4f32,
// v_mfma_f64_16x16x4f64) on the real embedding of the complex products: for
// an A operand of 16 rows x 4 k-slots the slots are (source index pair,
// real / imaginary part), and the B operand columns are the real parts
// (columns r < NRT) and imaginary parts (NRT <= column < 2 NRT) of NRT
// outputs:
//     part 0 (re M): B = [ xr | xi ],   part 1 (im M): B = [ -xi | xr ].
// A pass takes NRW = 4, 8 or 16 right-hand sides, in NCT = 1 or 2 such
// B tiles of NRT = min(NRW, 8) right-hand sides.  The two instructions share
// their A and B layouts (lane l: A[l % 16][l / 16], B[l / 16][l % 16]); the
// result rows differ: lane l, register e holds row 4 (l / 16) + e in FP32 and
// row l / 16 + 4 e in FP64.
//
// Wavefront w owns u tiles w, w + 4, ... (ntw <= TPW of them) and visits the
// v tiles in nt steps, v tile (q + w) mod nt at step q, so that the four
// wavefronts are on four different v tiles at every step.  For tile (t, v) it
// runs 8 MFMAs per B tile of the first product (A = the tile with rows u,
// read straight from HBM in the lane order of the store) into the tile's row
// accumulator, and 8 of the transposed product (A = the tile transposed,
// staged through LDS) into the v tile's column sums, which the wavefront adds
// into one LDS buffer at the end of the step (plain loads and stores: no other
// wavefront touches that v tile during the step); a barrier closes each step.  So
// every column sum receives its four addends in a fixed order (that of the
// steps), every row sum its v tiles in a fixed order, and the bits of every
// output are the same whatever the wavefront timing and whichever columns
// share the pass.  The column sums take the place of W xh[-k] once its values
// are in registers (OVL), where the LDS would otherwise cost a workgroup per
// CU.
//
// The blocks are read non-temporally with buffer loads; each wavefront keeps
// one tile in flight per u tile it owns, and the next request is
// unconditional (a visit index past the end re-reads the last tile) so that
// every wait covers only the oldest tile.  The row sums are staged in LDS at
// the end and both products leave as coalesced non-temporal stores.
#include "internal.h"

namespace emsurf {
namespace {

constexpr int PNT = 256;  // threads per workgroup
// Transposed staging of one wavefront: one tile of 16 rows of 32 values (a
// wavefront's LDS operations complete in order, so the next tile's writes
// cannot overtake the reads of the current one, and one stage suffices).
// The rows carry 16 bytes of padding, or (SWZ) their 16-byte chunks are
// permuted by a key of the row instead, where the LDS has no room for the
// padding; either way the 16-byte reads of one instruction (rows 0..15 at
// the same place) start on distinct banks.
template <typename T, bool SWZ> constexpr int pair_row_vals() { return SWZ ? 32 : 32 + 16 / (int)sizeof(T); }
template <typename T, bool SWZ> constexpr int pair_stage_vals() { return 16 * pair_row_vals<T, SWZ>(); }
// 16 right-hand sides per pass: the staging without padding
constexpr bool pair_swz(int nrw) { return nrw > 8; }

// Wavefronts per SIMD that the LDS of a workgroup leaves room for at the
// sizes each instance serves (FP32 up to 3 u tiles and 8 right-hand sides:
// four workgroups per CU; FP64 beyond 3 u tiles: one), as the register budget
template <typename T> constexpr int pair_min_waves(int tpw, int nrw) {
  return sizeof(T) == 4 ? (tpw <= 3 && nrw <= 8 ? 4 : 2) : (tpw <= 3 ? 2 : 1);
}

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef double d4v __attribute__((ext_vector_type(4)));

// per-precision pieces: 16-byte chunk type, values per chunk, accumulator
// type, the MFMA and the result row of (lane, register)
template <typename T> struct Mf;
template <> struct Mf<float> {
  using C = f4v;          // one 16-byte chunk
  using Acc = f4v;        // 16 x 16 result, 4 values per lane
  using V2 = float2;
  static constexpr int CH = 4;
  __device__ static Acc mfma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int l, int e) { return 4 * (l >> 4) + e; }
};
template <> struct Mf<double> {
  using C = d2v;
  using Acc = d4v;
  using V2 = double2;
  static constexpr int CH = 2;
  __device__ static Acc mfma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int e) { return (l >> 4) + 4 * e; }
};

template <typename C>
__device__ __forceinline__ C ld_chunk(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff) {
  return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 2));
}

// Column sums and row sums in LDS: [np][2 NRW], right-hand side r, part p at
// column (r / NRT) 2 NRT + p NRT + r % NRT; the columns of row v are permuted
// by XOR with v, so that the output loop (consecutive v per lane, one column)
// does not hit one bank
template <int NRW> __device__ __forceinline__ int sum_idx(int v, int col) {
  return v * 2 * NRW + (col ^ (v & (2 * NRW - 1)));
}
template <int NRW> __device__ __forceinline__ int sum_col(int r, int p) {
  constexpr int NRT = NRW > 8 ? 8 : NRW;
  return (r / NRT) * 2 * NRT + p * NRT + r % NRT;
}

// T = float or double; TPW u tiles per wavefront at most; NRW right-hand
// sides per pass (4, 8, or 16 in FP32).  B2R keeps the B operands of the
// transposed product in registers for the whole block (else they are rebuilt
// from LDS for every tile).  OVL (needs B2R): the column sums overlay
// W xh[-k].
template <typename T, int TPW, int NRW, bool B2R, bool OVL>
__global__ void __launch_bounds__(PNT, pair_min_waves<T>(TPW, NRW)) pair_mfma_kernel(
    const T* __restrict__ That, const int2* __restrict__ pairs, const T* __restrict__ w, const T* __restrict__ winv,
    const typename Mf<T>::V2* __restrict__ xh, typename Mf<T>::V2* __restrict__ yh, int n, int nrhs, int r0, int nr) {
  using M = Mf<T>;
  using C = typename M::C;
  using Acc = typename M::Acc;
  using V2 = typename M::V2;
  constexpr int CH = M::CH, NCH = 8 / CH;   // chunks per lane per tile
  constexpr int NCT = NRW > 8 ? 2 : 1;      // B tiles
  constexpr int NRT = NRW / NCT;            // right-hand sides per B tile
  constexpr bool SWZ = pair_swz(NRW);
  constexpr int TROW = pair_row_vals<T, SWZ>();
  constexpr int TILE_BYTES = 2 * PAIR_TILE * PAIR_TILE * (int)sizeof(T);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nt = pair_tiles(n), np = nt * PAIR_TILE;
  const int tid = (int)threadIdx.x;
  T* xs = reinterpret_cast<T*>(smem_raw);  // [np][NRW][2]: xh[k]; row sums at the end
  T* xt = xs + np * NRW * 2;               // [np][NRW][2]: W xh[-k]
  T* zs = OVL ? xt : xt + np * NRW * 2;    // column sums
  T* tiles = xt + np * NRW * 2 * (OVL ? 1 : 2);   // [4 waves][16 rows][TROW]
  const long long slot = blockIdx.x;
  const int2 pr = pairs[slot];
  const long long k = pr.x, kb = pr.y;
  const bool self = k == kb;
  const int l = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ntw = (nt - wv + 3) / 4;  // u tiles of this wavefront (<= TPW)
  const long long blk = (long long)nt * nt * 2 * PAIR_TILE * PAIR_TILE;  // reals
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(That + slot * blk), (short)0, (int)(blk * (long long)sizeof(T)), 0x00020000);
  const unsigned voff = (unsigned)(l * 16);   // chunk m of this lane sits 1024 m bytes on
  // this wavefront's tiles are stored contiguously in visiting order
  // it = q * ntw + ta (u tile wv + 4 ta, step q)
  const int nvisit = ntw * nt, wbase_tile = pair_wave_base(nt, wv);
  // visit it, clamped to the wavefront's tiles (a wavefront without tiles
  // reads the block's first tile and uses none of it)
  auto visit_off = [&](int it) {
    if (it > nvisit - 1) it = nvisit - 1;
    if (it < 0) it = 0;
    return nvisit > 0 ? (wbase_tile + it) * TILE_BYTES : 0;
  };
  // one tile in flight per u tile of the wavefront: while tile (q, ta) is
  // used, the tiles of the rest of step q and of step q + 1 up to ta - 1 are
  // on their way (every slot is requested, whatever ntw: see the sweep)
  C buf[TPW][NCH];
#pragma unroll
  for (int ta = 0; ta < TPW; ++ta)
#pragma unroll
    for (int m = 0; m < NCH; ++m) buf[ta][m] = ld_chunk<C>(rs, voff + 1024 * m, visit_off(ta));
  const V2* x0 = xh + k * (long long)nrhs * n + (long long)r0 * n;
  const V2* x1 = xh + kb * (long long)nrhs * n + (long long)r0 * n;
  for (int e = tid; e < np * NRW; e += PNT) {
    const int r = e / np, v = e - r * np;
    V2 a{0, 0}, b{0, 0};
    if (r < nr && v < n) {
      a = x0[(long long)r * n + v];
      const V2 c = x1[(long long)r * n + v];
      b = V2{w[v] * c.x, w[v] * c.y};
    }
    xs[(v * NRW + r) * 2] = a.x;
    xs[(v * NRW + r) * 2 + 1] = a.y;
    xt[(v * NRW + r) * 2] = b.x;
    xt[(v * NRW + r) * 2 + 1] = b.y;
  }
  if constexpr (!OVL)
    for (int e = tid; e < np * 2 * NRW; e += PNT) zs[e] = T(0);
  __syncthreads();
  // lane roles: k-slot kk = l / 16 -> (pair offset off, part); column jj = l % 16
  const int kk = l >> 4, jj = l & 15, off = kk >> 1, part = kk & 1, a16 = l & 15;
  const bool jre = jj < NRT, jok = jj < 2 * NRT;
  const int rjt = jre ? jj : (jok ? jj - NRT : 0);
  // B operand value of B tile c at source index idx
  auto bval = [&](const T* x, int idx, int c) {
    const int rj = c * NRT + rjt;
    const T xr = x[(idx * NRW + rj) * 2], xi = x[(idx * NRW + rj) * 2 + 1];
    const T val = part == 0 ? (jre ? xr : xi) : (jre ? -xi : xr);
    return jok ? val : T(0);
  };
  constexpr int NB2 = B2R ? TPW : 1;
  T b2[NB2][NCT][8];
#pragma unroll
  for (int ta = 0; ta < NB2; ++ta)
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int s = 0; s < 8; ++s)
        b2[ta][c][s] = B2R && ta < ntw ? bval(xt, (wv + 4 * ta) * PAIR_TILE + 2 * s + off, c) : T(0);
  if constexpr (OVL) {
    // xt becomes the column-sum buffer
    __syncthreads();
    for (int e = tid; e < np * 2 * NRW; e += PNT) zs[e] = T(0);
    __syncthreads();
  }
  Acc acc[TPW][NCT];
#pragma unroll
  for (int ta = 0; ta < TPW; ++ta)
#pragma unroll
    for (int c = 0; c < NCT; ++c) acc[ta][c] = Acc{};
  // transposed staging: value s of this lane, entry (u = a16, v = 2 s + off, part), goes to
  // row v, place (part * 2 + u % 2) * 8 + u / 2; lane l then reads its 8 transposed operands
  // (u = 2 s + off, v = a16, part) as 8 consecutive values of row a16 (with SWZ, the 16-byte
  // chunks of row v permuted by XOR with (v % 8) ^ (v / 8 % 2))
  T* Tw = tiles + wv * pair_stage_vals<T, SWZ>();
  const int wplace = (part * 2 + (a16 & 1)) * 8 + (a16 >> 1);
  const int wbase = off * TROW + wplace;
  auto wpos = [&](int s) {
    if constexpr (SWZ) {
      const int v = 2 * s + off, key = (v & 7) ^ ((v >> 3) & 1);
      return v * TROW + ((wplace / CH) ^ key) * CH + wplace % CH;
    } else {
      return 2 * s * TROW + wbase;
    }
  };
  const int rplace = (part * 2 + off) * 8;
  const int rkey = (a16 & 7) ^ ((a16 >> 3) & 1);
  auto rpos = [&](int m) {
    if constexpr (SWZ)
      return a16 * TROW + ((rplace / CH + m) ^ rkey) * CH;
    else
      return a16 * TROW + rplace + m * CH;
  };
  // v tile of step q for this wavefront
  auto vtile = [&](int q) { return (q + wv) % nt; };
  // B operands of the first product for the v tile of step q, built one step ahead
  T b1n[NCT][8];
#pragma unroll
  for (int c = 0; c < NCT; ++c)
#pragma unroll
    for (int s = 0; s < 8; ++s) b1n[c][s] = bval(xs, vtile(0) * PAIR_TILE + 2 * s + off, c);
  for (int q = 0; q < nt; ++q) {
    const int vq = vtile(q);
    T b1[NCT][8];
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int s = 0; s < 8; ++s) b1[c][s] = b1n[c][s];
    const int vn = vtile(q + 1 < nt ? q + 1 : q);
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int s = 0; s < 8; ++s) b1n[c][s] = bval(xs, vn * PAIR_TILE + 2 * s + off, c);
    Acc zq[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) zq[c] = Acc{};
#pragma unroll
    for (int ta = 0; ta < TPW; ++ta) {
      const bool live = ta < ntw;
      C cr[NCH];
      if (live) {
#pragma unroll
        for (int s = 0; s < 8; ++s) Tw[wpos(s)] = buf[ta][s / CH][s % CH];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int m = 0; m < NCH; ++m) cr[m] = *reinterpret_cast<const C*>(Tw + rpos(m));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
          for (int c = 0; c < NCT; ++c) acc[ta][c] = M::mfma(buf[ta][s / CH][s % CH], b1[c][s], acc[ta][c]);
        __builtin_amdgcn_sched_barrier(0);
      }
      // the slot's registers are free: request its tile of step q + 1 (every
      // slot requests one, whatever ntw, so that each wait covers exactly
      // the oldest tile; a slot past ntw repeats the request before it)
      const int noff = visit_off((q + 1) * ntw + (live ? ta : ntw - 1));
#pragma unroll
      for (int m = 0; m < NCH; ++m) buf[ta][m] = ld_chunk<C>(rs, voff + 1024 * m, noff);
      if (live) {
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
          for (int c = 0; c < NCT; ++c) {
            const T bt = B2R ? b2[B2R ? ta : 0][c][s] : bval(xt, (wv + 4 * ta) * PAIR_TILE + 2 * s + off, c);
            zq[c] = M::mfma(cr[s / CH][s % CH], bt, zq[c]);
          }
      }
    }
    if (!self && ntw > 0) {
      // the v tile is this wavefront's alone during the step: a plain
      // read, add and write (LDS float atomics are far slower).  FP32 rows
      // 4 (l / 16) + e: the four lane groups start at register (e + l / 16)
      // % 4, so that one access touches four rows that are not a multiple
      // of the bank count apart
      int zi[NCT][4];
      T zo[NCT][4];
#pragma unroll
      for (int c = 0; c < NCT; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int er = sizeof(T) == 4 ? (e + kk) & 3 : e;
          zi[c][e] = sum_idx<NRW>(vq * PAIR_TILE + M::row(l, er), c * 2 * NRT + jj);
          zo[c][e] = jok ? zs[zi[c][e]] : T(0);
        }
#pragma unroll
      for (int c = 0; c < NCT; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int er = sizeof(T) == 4 ? (e + kk) & 3 : e;
          const T val = er == 0 ? zq[c][0] : er == 1 ? zq[c][1] : er == 2 ? zq[c][2] : zq[c][3];
          if (jok) zs[zi[c][e]] = zo[c][e] + val;
        }
    }
    // the next step's adds to this v tile come from another wavefront
    __syncthreads();
  }
  // outputs: the row sums are staged in LDS over the spectral columns of
  // xh[k] (no longer read once every wavefront is past its loop), in the
  // layout of the column sums, and both products leave as coalesced
  // non-temporal stores of 16 bytes per lane
  T* ys = xs;  // [np][2 NRW]: row sums (yh[k])
#pragma unroll
  for (int ta = 0; ta < TPW; ++ta) {
    if (ta < ntw) {
#pragma unroll
      for (int c = 0; c < NCT; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int u = (wv + 4 * ta) * PAIR_TILE + M::row(l, e);
          if (jok) ys[sum_idx<NRW>(u, c * 2 * NRT + jj)] = acc[ta][c][e];
        }
    }
  }
  __syncthreads();
  V2* y0 = yh + k * (long long)nrhs * n + (long long)r0 * n;
  V2* y1 = yh + kb * (long long)nrhs * n + (long long)r0 * n;
  if constexpr (sizeof(T) == 8) {
    for (int e = tid; e < nr * n; e += PNT) {
      const int r = e / n, v = e - r * n;
      const int cr0 = sum_idx<NRW>(v, sum_col<NRW>(r, 0)), ci0 = sum_idx<NRW>(v, sum_col<NRW>(r, 1));
      __builtin_nontemporal_store(d2v{ys[cr0], ys[ci0]}, reinterpret_cast<d2v*>(y0 + e));
      if (!self) {
        const double wi = winv[v];
        __builtin_nontemporal_store(d2v{zs[cr0] * wi, zs[ci0] * wi}, reinterpret_cast<d2v*>(y1 + e));
      }
    }
  } else {
    if ((n & 1) == 0) {
      // two complex values per 16-byte store
      for (int e2 = tid; e2 < nr * n / 2; e2 += PNT) {
        const int e = 2 * e2, r = e / n, v = e - r * n;   // v + 1 < n in the same row r
        const int colr = sum_col<NRW>(r, 0), coli = sum_col<NRW>(r, 1);
        const int a0 = sum_idx<NRW>(v, colr), a1 = sum_idx<NRW>(v, coli);
        const int b0 = sum_idx<NRW>(v + 1, colr), b1 = sum_idx<NRW>(v + 1, coli);
        __builtin_nontemporal_store(f4v{ys[a0], ys[a1], ys[b0], ys[b1]}, reinterpret_cast<f4v*>(y0 + e));
        if (!self) {
          const float w0 = winv[v], w1 = winv[v + 1];
          __builtin_nontemporal_store(f4v{zs[a0] * w0, zs[a1] * w0, zs[b0] * w1, zs[b1] * w1},
                                      reinterpret_cast<f4v*>(y1 + e));
        }
      }
    } else {
      for (int e = tid; e < nr * n; e += PNT) {
        const int r = e / n, v = e - r * n;
        const int cr0 = sum_idx<NRW>(v, sum_col<NRW>(r, 0)), ci0 = sum_idx<NRW>(v, sum_col<NRW>(r, 1));
        y0[e] = V2{ys[cr0], ys[ci0]};
        if (!self) y1[e] = V2{zs[cr0] * winv[v], zs[ci0] * winv[v]};
      }
    }
  }
}

// FP64 B operands of the transposed product stay in registers for at most 2 u
// tiles per wavefront; beyond that they are rebuilt from LDS per tile
template <typename T> constexpr bool pair_b2r(int tpw) { return sizeof(T) == 4 || tpw <= 2; }

// LDS of a workgroup: spectral inputs xh[k] and W xh[-k], the column sums
// (over W xh[-k] when ovl), the transposed staging
template <typename T>
size_t pair_lds_bytes(int n, int nrw, bool ovl) {
  const int np = pair_tiles(n) * PAIR_TILE;
  const int stage = pair_swz(nrw) ? pair_stage_vals<T, true>() : pair_stage_vals<T, false>();
  return (size_t)(np * nrw * 2 * (ovl ? 2 : 3) + 4 * stage) * sizeof(T);
}

constexpr size_t CU_LDS = 160 * 1024;
constexpr int PAIR16_TPW_MAX = 5;
// LDS of one workgroup at most 160 KB
constexpr size_t PAIR_LDS_MAX = CU_LDS;

// Overlay the column sums where their own region would leave fewer
// workgroups per CU (by LDS; a workgroup has one wavefront per SIMD, and at
// most 4 per CU fit the registers of the matrix-core forms here), or where
// the workgroup would not fit otherwise
template <typename T>
bool pair_overlay(int n, int nrw) {
  if (!pair_b2r<T>((pair_tiles(n) + 3) / 4)) return false;
  auto wgs = [](size_t b) { const size_t w = CU_LDS / b; return w < 4 ? w : (size_t)4; };
  return wgs(pair_lds_bytes<T>(n, nrw, false)) < wgs(pair_lds_bytes<T>(n, nrw, true));
}

template <typename T, int TPW, int NRW>
void launch_mfma_pair(const void* That, const void* pairs, const void* w, const void* winv, const void* xh, void* yh,
                      int n, int nrhs, int r0, int nr, int64_t Ps, hipStream_t s) {
  using V2 = typename Mf<T>::V2;
  // FP64 B operands of many u tiles would not fit the registers
  constexpr bool B2R = pair_b2r<T>(TPW);
  const bool ovl = pair_overlay<T>(n, NRW);
  const size_t shm = pair_lds_bytes<T>(n, NRW, ovl);
  if (ovl) {
    if constexpr (B2R)
      hipLaunchKernelGGL((pair_mfma_kernel<T, TPW, NRW, B2R, true>), dim3((unsigned)Ps), dim3(PNT), shm, s,
                         static_cast<const T*>(That), static_cast<const int2*>(pairs), static_cast<const T*>(w),
                         static_cast<const T*>(winv), static_cast<const V2*>(xh), static_cast<V2*>(yh), n, nrhs, r0,
                         nr);
    else
      EMS_CHECK_ARG(false, "internal: column-sum overlay without register B operands");
  } else {
    hipLaunchKernelGGL((pair_mfma_kernel<T, TPW, NRW, B2R, false>), dim3((unsigned)Ps), dim3(PNT), shm, s,
                       static_cast<const T*>(That), static_cast<const int2*>(pairs), static_cast<const T*>(w),
                       static_cast<const T*>(winv), static_cast<const V2*>(xh), static_cast<V2*>(yh), n, nrhs, r0, nr);
  }
}

template <typename T, int TPW>
void launch_mfma_pair_tpw(int nrw, const void* That, const void* pairs, const void* w, const void* winv,
                          const void* xh, void* yh, int n, int nrhs, int r0, int nr, int64_t Ps, hipStream_t s) {
  if (nrw == 4) {
    launch_mfma_pair<T, TPW, 4>(That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s);
  } else if (nrw == 8) {
    launch_mfma_pair<T, TPW, 8>(That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s);
  } else {
    if constexpr (sizeof(T) == 4 && TPW <= PAIR16_TPW_MAX)
      launch_mfma_pair<T, TPW, 16>(That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s);
    else
      EMS_CHECK_ARG(false, "internal: 16 right-hand sides per pass are FP32 only, n_eq <= 320");
  }
}

// Right-hand sides per pass: 4 for at most 4 (less LDS, more workgroups per
// CU); else 8, or 16 in FP32 above 8 (up to 5 u tiles per wavefront, n_eq <=
// 320, whose registers fit two wavefronts per SIMD), wherever the workgroup
// fits the LDS
template <typename T>
int pair_nrw(int n, int nrhs) {
  auto fits = [&](int nrw) { return pair_lds_bytes<T>(n, nrw, pair_overlay<T>(n, nrw)) <= PAIR_LDS_MAX; };
  if (nrhs <= 4 || !fits(8)) return 4;
  if (sizeof(T) == 4 && nrhs > 8 && (pair_tiles(n) + 3) / 4 <= PAIR16_TPW_MAX && fits(16)) return 16;
  return 8;
}

template <typename T>
void launch_pair_typed(const void* That, const void* pairs, const void* w, const void* winv, const void* xh, void* yh,
                       int n, int nrhs, int64_t Ps, hipStream_t s) {
  const int tpw = (pair_tiles(n) + 3) / 4;
  const int nrw = pair_nrw<T>(n, nrhs);
  EMS_CHECK_ARG(pair_lds_bytes<T>(n, nrw, pair_overlay<T>(n, nrw)) <= PAIR_LDS_MAX,
                "internal: paired product LDS too large");
  for (int r0 = 0; r0 < nrhs; r0 += nrw) {
    const int nr = nrhs - r0 < nrw ? nrhs - r0 : nrw;
    switch (tpw) {
      case 1: launch_mfma_pair_tpw<T, 1>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      case 2: launch_mfma_pair_tpw<T, 2>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      case 3: launch_mfma_pair_tpw<T, 3>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      case 4: launch_mfma_pair_tpw<T, 4>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      case 5: launch_mfma_pair_tpw<T, 5>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      case 6: launch_mfma_pair_tpw<T, 6>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      case 7: launch_mfma_pair_tpw<T, 7>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      default: launch_mfma_pair_tpw<T, 8>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
    }
  }
}

}  // namespace

void launch_block_product_pair(Cx t, const void* That, const void* pairs, const void* w, const void* winv,
                               const void* xh, void* yh, int n, int nrhs, int64_t Ps, hipStream_t s) {
  EMS_CHECK_ARG(n >= 1 && n <= 512, "paired block product supports 1 <= n_eq <= 512");
  EMS_CHECK_ARG(nrhs >= 1 && nrhs <= 64, "paired block product supports 1 <= nrhs <= 64");
  EMS_CHECK_ARG(Ps >= 1 && Ps <= 0x7fffffffLL, "pair count out of range");
  if (t == Cx::C128)
    launch_pair_typed<double>(That, pairs, w, winv, xh, yh, n, nrhs, Ps, s);
  else
    launch_pair_typed<float>(That, pairs, w, winv, xh, yh, n, nrhs, Ps, s);
  EMS_LAUNCH_CHECK();
}

void spectrum_pairs(int Lx, int Ly, std::vector<int>& pairs, std::vector<int>& slot_of) {
  const int64_t P = (int64_t)Lx * Ly;
  pairs.clear();
  slot_of.assign((size_t)P, -1);
  for (int ky = 0; ky < Ly; ++ky)
    for (int kx = 0; kx < Lx; ++kx) {
      const int k = ky * Lx + kx;
      const int kb = ((Ly - ky) % Ly) * Lx + (Lx - kx) % Lx;
      if (k <= kb) {
        slot_of[(size_t)k] = (int)(pairs.size() / 2);
        pairs.push_back(k);
        pairs.push_back(kb);
      }
    }
}

}  // namespace emsurf
