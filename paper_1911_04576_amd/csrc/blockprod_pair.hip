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
// (columns r < NR) and imaginary parts (NR <= column < 2 NR) of the outputs:
//     part 0 (re M): B = [ xr | xi ],   part 1 (im M): B = [ -xi | xr ].
// Wavefront w owns u tiles w, w + 4, ... (TPW of them) and visits every v
// tile; for tile (t, q) it runs 8 MFMAs of the first product (A = the tile
// with rows u, read straight from HBM in the lane order of the store) into
// the tile's row accumulator, and 8 of the transposed product (A = the tile
// transposed, staged through LDS) into the v tile's column sums, which are
// added into LDS once per v tile.  Wavefronts 0 and 1 add into one column-sum
// buffer and wavefronts 2 and 3 into another: with two addends per entry the
// LDS float addition gives the same bits in either order (0 + a = a, and
// a + b = b + a), and the two buffers are added in a fixed order at the end,
// so every output has one rounding sequence whatever the wavefront timing.
// The second buffer has a region of its own, or (OVL, where that region would
// cost a workgroup per CU) takes the place of W xh[-k] once its values are in
// registers, which costs two more barriers per workgroup.
// Up to 8 right-hand sides per pass
// (2 NR <= 16 MFMA columns).  The two instructions share their A and B
// layouts (lane l: A[l % 16][l / 16], B[l / 16][l % 16]); the result rows
// differ: lane l, register e holds row 4 (l / 16) + e in FP32 and row
// l / 16 + 4 e in FP64.
//
// The blocks are read non-temporally with buffer loads; two tiles are in
// flight per wavefront and the next request is unconditional (a visit index
// past the end re-reads the last tile) so that every wait covers only the
// older stage.  The row sums are staged in LDS at the end and both products
// leave as coalesced non-temporal stores.
#include "internal.h"

namespace emsurf {
namespace {

constexpr int PNT = 256;  // threads per workgroup
// LDS stages of the transposed staging per wavefront: two in FP32; one in
// FP64, which brings a workgroup at n_eq 192 and 4 RHS under 54 KB, so that
// three fit a CU (a wavefront's LDS operations complete in order, so the next
// tile's writes cannot overtake the reads of the current one)
template <typename T> constexpr int pair_stages() { return sizeof(T) == 8 ? 1 : 2; }

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

// T = float or double; TPW u tiles per wavefront; NRW right-hand sides per
// pass (4 or 8: the MFMA columns used, 2 NRW of 16).  B2R keeps the B
// operands of the transposed product in registers for the whole block (else
// they are rebuilt from LDS for every tile).  OVL (needs B2R): the second
// column-sum buffer overlays W xh[-k].
template <typename T, int TPW, int NRW, bool B2R, bool OVL>
__global__ void __launch_bounds__(PNT, 2) pair_mfma_kernel(const T* __restrict__ That, const int2* __restrict__ pairs,
                                                           const T* __restrict__ w, const T* __restrict__ winv,
                                                           const typename Mf<T>::V2* __restrict__ xh,
                                                           typename Mf<T>::V2* __restrict__ yh, int n, int nrhs, int r0,
                                                           int nr) {
  using M = Mf<T>;
  using C = typename M::C;
  using Acc = typename M::Acc;
  using V2 = typename M::V2;
  constexpr int CH = M::CH, NCH = 8 / CH;   // chunks per lane per tile
  constexpr int TILE_BYTES = 2 * PAIR_TILE * PAIR_TILE * (int)sizeof(T);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nt = pair_tiles(n), np = nt * PAIR_TILE;
  T* xs = reinterpret_cast<T*>(smem_raw);  // [np][NRW][2]: xh[k]; row sums at the end
  T* xt = xs + np * NRW * 2;               // [np][NRW][2]: W xh[-k]
  T* zs = xt + np * NRW * 2;               // [np][2 NRW]: column sums of wavefronts 0, 1
  // column sums of wavefronts 2, 3
  T* zs2 = OVL ? xt : zs + np * 2 * NRW;
  T* tiles = zs + np * 2 * NRW * (OVL ? 1 : 2);   // [4 waves][stages][512]
  const long long slot = blockIdx.x;
  const int2 pr = pairs[slot];
  const long long k = pr.x, kb = pr.y;
  const bool self = k == kb;
  const int l = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ntw = (nt - wv + 3) / 4;  // u tiles of this wavefront (<= TPW)
  const long long blk = (long long)nt * nt * 2 * PAIR_TILE * PAIR_TILE;  // reals
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(That + slot * blk), (short)0, (int)(blk * (long long)sizeof(T)), 0x00020000);
  const unsigned voff = (unsigned)(l * 16);   // chunk m of this lane sits 1024 m bytes on
  // this wavefront's tiles are stored contiguously in visiting order
  // it = q * ntw + ta (u tile wv + 4 ta, v tile q)
  const int nvisit = ntw * nt, wbase_tile = pair_wave_base(nt, wv);
  auto visit_off = [&](int it) {
    if (it > nvisit - 1) it = nvisit - 1;
    return (wbase_tile + it) * TILE_BYTES;
  };
  // two tiles in flight: p (current) and nx (next)
  C p[NCH], nx[NCH];
#pragma unroll
  for (int m = 0; m < NCH; ++m) {
    p[m] = C{};
    nx[m] = C{};
  }
  if (ntw > 0) {
#pragma unroll
    for (int m = 0; m < NCH; ++m) {
      p[m] = ld_chunk<C>(rs, voff + 1024 * m, visit_off(0));
      nx[m] = ld_chunk<C>(rs, voff + 1024 * m, visit_off(1));
    }
  }
  const V2* x0 = xh + k * (long long)nrhs * n + (long long)r0 * n;
  const V2* x1 = xh + kb * (long long)nrhs * n + (long long)r0 * n;
  for (int e = threadIdx.x; e < np * NRW; e += PNT) {
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
  for (int e = threadIdx.x; e < np * 2 * NRW; e += PNT) zs[e] = T(0);
  if constexpr (!OVL)
    for (int e = threadIdx.x; e < np * 2 * NRW; e += PNT) zs2[e] = T(0);
  __syncthreads();
  // lane roles: k-slot kk = l / 16 -> (pair offset off, part); column jj = l % 16
  const int kk = l >> 4, jj = l & 15, off = kk >> 1, part = kk & 1, a16 = l & 15;
  const bool jre = jj < NRW, jok = jj < 2 * NRW;
  const int rj = jre ? jj : (jok ? jj - NRW : 0);
  auto bval = [&](const T* x, int idx) {
    const T xr = x[(idx * NRW + rj) * 2], xi = x[(idx * NRW + rj) * 2 + 1];
    const T val = part == 0 ? (jre ? xr : xi) : (jre ? -xi : xr);
    return jok ? val : T(0);
  };
  constexpr int NB2 = B2R ? TPW : 1;
  T b2[NB2][8];
#pragma unroll
  for (int ta = 0; ta < NB2; ++ta)
#pragma unroll
    for (int s = 0; s < 8; ++s) b2[ta][s] = B2R && ta < ntw ? bval(xt, (wv + 4 * ta) * PAIR_TILE + 2 * s + off) : T(0);
  if constexpr (OVL) {
    // xt becomes the second column-sum buffer
    __syncthreads();
    for (int e = threadIdx.x; e < np * 2 * NRW; e += PNT) zs2[e] = T(0);
    __syncthreads();
  }
  Acc acc[TPW];
#pragma unroll
  for (int ta = 0; ta < TPW; ++ta) acc[ta] = Acc{};
  // transposed staging: value s of this lane, entry (u = a16, v = 2 s + off, part), goes to
  // ((v * 2 + part) * 2 + u % 2) * 8 + u / 2; lane l then reads its 8 transposed operands
  // (u = 2 s + off, v = a16, part) as 8 consecutive values
  const int wbase = (part * 2 + (a16 & 1)) * 8 + (a16 >> 1);
  const int rbase = ((a16 * 2 + part) * 2 + off) * 8;
  constexpr int NSTG = pair_stages<T>();
  T* tw = tiles + wv * NSTG * 512;
  int stage = 0;
  // B operands of the first product for v tile q, built one v tile ahead
  T b1n[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) b1n[s] = bval(xs, 2 * s + off);
  for (int q = 0; q < nt; ++q) {
    T b1[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) b1[s] = b1n[s];
    const int qn = q + 1 < nt ? q + 1 : q;
#pragma unroll
    for (int s = 0; s < 8; ++s) b1n[s] = bval(xs, qn * PAIR_TILE + 2 * s + off);
    Acc zq{};
#pragma unroll
    for (int ta = 0; ta < TPW; ++ta) {
      if (ta < ntw) {
        T a1[8];
#pragma unroll
        for (int m = 0; m < NCH; ++m)
#pragma unroll
          for (int c = 0; c < CH; ++c) a1[m * CH + c] = p[m][c];
        T* Tw = tw + stage * 512;
#pragma unroll
        for (int s = 0; s < 8; ++s) Tw[(2 * s + off) * 32 + wbase] = a1[s];
        __builtin_amdgcn_wave_barrier();
        C cr[NCH];
#pragma unroll
        for (int m = 0; m < NCH; ++m) cr[m] = *reinterpret_cast<const C*>(Tw + rbase + m * CH);
        const int noff = visit_off(q * ntw + ta + 2);
#pragma unroll
        for (int m = 0; m < NCH; ++m) {
          p[m] = nx[m];
          nx[m] = ld_chunk<C>(rs, voff + 1024 * m, noff);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < 8; ++s) acc[ta] = M::mfma(a1[s], b1[s], acc[ta]);
        __builtin_amdgcn_sched_barrier(0);
        T bt[8];
#pragma unroll
        for (int s = 0; s < 8; ++s)
          bt[s] = B2R ? b2[B2R ? ta : 0][s] : bval(xt, (wv + 4 * ta) * PAIR_TILE + 2 * s + off);
#pragma unroll
        for (int m = 0; m < NCH; ++m)
#pragma unroll
          for (int c = 0; c < CH; ++c) zq = M::mfma(cr[m][c], bt[m * CH + c], zq);
        stage = NSTG == 2 ? stage ^ 1 : 0;
      }
    }
    if (!self && ntw > 0) {
      T* zd = wv < 2 ? zs : zs2;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (jok) atomicAdd(&zd[(q * PAIR_TILE + M::row(l, e)) * 2 * NRW + jj], zq[e]);
    }
  }
  // outputs: the row sums are staged in LDS over the spectral columns of
  // xh[k] (no longer read once every wavefront is past its loop), in the
  // layout of the column sums, and both products leave as coalesced
  // non-temporal stores of 16 bytes per lane
  __syncthreads();
  T* ys = xs;  // [np][2 NRW]: row sums (yh[k])
#pragma unroll
  for (int ta = 0; ta < TPW; ++ta) {
    if (ta < ntw) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int u = (wv + 4 * ta) * PAIR_TILE + M::row(l, e);
        if (jok) ys[u * 2 * NRW + jj] = acc[ta][e];
      }
    }
  }
  __syncthreads();
  V2* y0 = yh + k * (long long)nrhs * n + (long long)r0 * n;
  V2* y1 = yh + kb * (long long)nrhs * n + (long long)r0 * n;
  if constexpr (sizeof(T) == 8) {
    for (int e = threadIdx.x; e < nr * n; e += PNT) {
      const int r = e / n, v = e - r * n;
      const int c0 = v * 2 * NRW + r;
      __builtin_nontemporal_store(d2v{ys[c0], ys[c0 + NRW]}, reinterpret_cast<d2v*>(y0 + e));
      if (!self) {
        const double wi = winv[v];
        __builtin_nontemporal_store(d2v{(zs[c0] + zs2[c0]) * wi, (zs[c0 + NRW] + zs2[c0 + NRW]) * wi},
                                    reinterpret_cast<d2v*>(y1 + e));
      }
    }
  } else {
    if ((n & 1) == 0) {
      // two complex values per 16-byte store
      for (int e2 = threadIdx.x; e2 < nr * n / 2; e2 += PNT) {
        const int e = 2 * e2, r = e / n, v = e - r * n;   // v + 1 < n in the same row r
        const int c0 = v * 2 * NRW + r, c1 = c0 + 2 * NRW;
        const f4v a = {ys[c0], ys[c0 + NRW], ys[c1], ys[c1 + NRW]};
        __builtin_nontemporal_store(a, reinterpret_cast<f4v*>(y0 + e));
        if (!self) {
          const float w0 = winv[v], w1 = winv[v + 1];
          const f4v b = {(zs[c0] + zs2[c0]) * w0, (zs[c0 + NRW] + zs2[c0 + NRW]) * w0, (zs[c1] + zs2[c1]) * w1,
                         (zs[c1 + NRW] + zs2[c1 + NRW]) * w1};
          __builtin_nontemporal_store(b, reinterpret_cast<f4v*>(y1 + e));
        }
      }
    } else {
      for (int e = threadIdx.x; e < nr * n; e += PNT) {
        const int r = e / n, v = e - r * n;
        const int c0 = v * 2 * NRW + r;
        y0[e] = V2{ys[c0], ys[c0 + NRW]};
        if (!self) y1[e] = V2{(zs[c0] + zs2[c0]) * winv[v], (zs[c0 + NRW] + zs2[c0 + NRW]) * winv[v]};
      }
    }
  }
}

// FP64 B operands of the transposed product stay in registers for at most 2 u
// tiles per wavefront; beyond that they are rebuilt from LDS per tile
template <typename T> constexpr bool pair_b2r(int tpw) { return sizeof(T) == 4 || tpw <= 2; }

// LDS of a workgroup: spectral inputs xh[k] and W xh[-k], two column-sum
// buffers (one of them over W xh[-k] when ovl), the transposed staging
template <typename T>
size_t pair_lds_bytes(int n, int nrw, bool ovl) {
  const int np = pair_tiles(n) * PAIR_TILE;
  return (size_t)(np * nrw * 2 * (ovl ? 3 : 4) + 4 * pair_stages<T>() * 512) * sizeof(T);
}

constexpr size_t CU_LDS = 160 * 1024;

// Overlay the second column-sum buffer only where its own region would leave
// fewer workgroups per CU (by LDS; a workgroup has one wavefront per SIMD,
// and at most 4 per CU fit the registers of the matrix-core forms here).
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
  } else {
    hipLaunchKernelGGL((pair_mfma_kernel<T, TPW, NRW, B2R, false>), dim3((unsigned)Ps), dim3(PNT), shm, s,
                       static_cast<const T*>(That), static_cast<const int2*>(pairs), static_cast<const T*>(w),
                       static_cast<const T*>(winv), static_cast<const V2*>(xh), static_cast<V2*>(yh), n, nrhs, r0, nr);
  }
}

template <typename T, int TPW>
void launch_mfma_pair_tpw(int nrw, const void* That, const void* pairs, const void* w, const void* winv,
                          const void* xh, void* yh, int n, int nrhs, int r0, int nr, int64_t Ps, hipStream_t s) {
  if (nrw == 4)
    launch_mfma_pair<T, TPW, 4>(That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s);
  else
    launch_mfma_pair<T, TPW, 8>(That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s);
}

// LDS of one workgroup at most 160 KB
constexpr size_t PAIR_LDS_MAX = 160 * 1024;

template <typename T>
void launch_pair_typed(const void* That, const void* pairs, const void* w, const void* winv, const void* xh, void* yh,
                       int n, int nrhs, int64_t Ps, hipStream_t s) {
  const int tpw = (pair_tiles(n) + 3) / 4;
  // 4-wide passes for at most 4 right-hand sides (less LDS, more workgroups
  // per CU), and wherever 8-wide ones would not fit the LDS
  const int nrw = nrhs <= 4 || pair_lds_bytes<T>(n, 8, pair_overlay<T>(n, 8)) > PAIR_LDS_MAX ? 4 : 8;
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
