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
// FP32 (pair_f32_kernel): each half-wavefront owns one block row at a time,
// its 32 lanes the columns c + 32 j.  The row sums of the first product are
// reduced across the half-wavefront (DPP row rotations, then one swizzle)
// and stored once per row; each lane keeps the column sums of the transposed
// product (CC x NR complex) in registers and adds them into LDS at the end.
// The store is tiled in exactly the order the wavefronts read it: tiles of
// 8 rows x 32 columns, each load instruction of a wavefront reads 512
// contiguous bytes (two tile rows) and a block row step one contiguous run.
//
// FP64 (pair_gemv_kernel): 4 row lanes g by 64 column lanes c; lane (g, c)
// owns rows u = g + 4 i and columns v = c + 64 j of row panels of 4 rows
// (entry (u, v) at ((u / 4) n + v) 4 + u % 4); row sums are added into LDS
// with atomics after each row.  A lane column v >= n (n not a multiple of
// 64) reads an entry of the next panel: xh[k] is zero-padded there and that
// column sum is never stored, so it contributes nothing for a finite block.
//
// Both read the blocks non-temporally with buffer loads (offsets past the
// block read zero) and request the next row before multiplying the current
// one; the requests are unconditional (a row index past the end re-reads the
// last row) so that every wait covers only the older stage.
#include <utility>

#include "internal.h"

namespace emsurf {
namespace {

template <typename V> struct Real;
template <> struct Real<float2> { using T = float; };
template <> struct Real<double2> { using T = double; };

__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename V> __device__ __forceinline__ V ld_elem(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff);
template <> __device__ __forceinline__ float2 ld_elem<float2>(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff) {
  auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 2);
  float2 f;
  __builtin_memcpy(&f, &v, sizeof(f));
  return f;
}
template <> __device__ __forceinline__ double2 ld_elem<double2>(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff) {
  auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 2);
  double2 d;
  __builtin_memcpy(&d, &v, sizeof(d));
  return d;
}

constexpr int PNT = 256;  // threads per workgroup
// FP64 kernel: row lanes (= panel height) and column lanes
template <typename V> constexpr int pair_g() { return PAIR_PANEL_FP64; }
template <typename V> constexpr int pair_cs() { return PNT / pair_g<V>(); }

// the CC elements of block row i owned by this lane: columns c + PCS j
template <typename V, int CC>
__device__ __forceinline__ void pair_fetch(V (&a)[CC], __amdgpu_buffer_rsrc_t rs, unsigned voff, int i, int n) {
  constexpr int PG = pair_g<V>(), PCS = pair_cs<V>();
#pragma unroll
  for (int j = 0; j < CC; ++j) a[j] = ld_elem<V>(rs, voff, ((i * n + PCS * j) * PG) * (int)sizeof(V));
}

// One block row: row sums of the first product into LDS, column sums of the
// transposed product into registers.
template <typename V, int CC, int NR, typename T>
__device__ __forceinline__ void pair_row(const V (&a)[CC], int i, int g, int c, int n, const V* __restrict__ xs,
                                         const V* __restrict__ xt, T* __restrict__ ys, T (&zr)[CC][NR],
                                         T (&zi)[CC][NR]) {
  constexpr int PG = pair_g<V>(), PCS = pair_cs<V>();
  const int u = g + PG * i;
  V xr[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) xr[r] = xt[u * NR + r];
  T yr[NR], yi[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) { yr[r] = 0; yi[r] = 0; }
#pragma unroll
  for (int j = 0; j < CC; ++j) {
    const V av = a[j];
    const V* xc = xs + (c + PCS * j) * NR;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const V xv = xc[r];
      yr[r] = fma_r(av.x, xv.x, yr[r]);
      yr[r] = fma_r(-av.y, xv.y, yr[r]);
      yi[r] = fma_r(av.x, xv.y, yi[r]);
      yi[r] = fma_r(av.y, xv.x, yi[r]);
      zr[j][r] = fma_r(av.x, xr[r].x, zr[j][r]);
      zr[j][r] = fma_r(-av.y, xr[r].y, zr[j][r]);
      zi[j][r] = fma_r(av.x, xr[r].y, zi[j][r]);
      zi[j][r] = fma_r(av.y, xr[r].x, zi[j][r]);
    }
  }
  if (u < n) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      atomicAdd(ys + 2 * (r * n + u), yr[r]);
      atomicAdd(ys + 2 * (r * n + u) + 1, yi[r]);
    }
  }
}

// CC columns per lane (PCS CC >= n); NR right-hand sides per pass, nr <= NR
// of them valid.  Register budget: 3 wavefronts per SIMD.

template <typename V, int CC, int NR>
__global__ void __launch_bounds__(PNT, 3) pair_gemv_kernel(const V* __restrict__ That, const int2* __restrict__ pairs,
                                                       const typename Real<V>::T* __restrict__ w,
                                                       const typename Real<V>::T* __restrict__ winv,
                                                       const V* __restrict__ xh, V* __restrict__ yh, int n, int nrhs,
                                                       int r0, int nr) {
  using T = typename Real<V>::T;
  constexpr int PG = pair_g<V>(), PCS = pair_cs<V>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int RR = (n + PG - 1) / PG;
  const int rows_pad = PG * RR, cols_pad = PCS * CC;
  V* xs = reinterpret_cast<V*>(smem_raw);           // [cols_pad][NR]: xh[k]
  V* xt = xs + cols_pad * NR;                       // [rows_pad][NR]: W xh[-k]
  T* ys = reinterpret_cast<T*>(xt + rows_pad * NR); // [NR][n][2]: row sums (yh[k])
  T* zs = ys + 2 * NR * n;                          // [NR][n][2]: column sums (W yh[-k])
  const long long slot = blockIdx.x;
  const int2 pr = pairs[slot];
  const long long k = pr.x, kb = pr.y;
  const bool self = k == kb;
  const int g = threadIdx.x % PG, c = threadIdx.x / PG;
  const long long blk = (long long)rows_pad * n;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(That + slot * blk), (short)0, (int)(blk * (long long)sizeof(V)), 0x00020000);
  const unsigned voff = (unsigned)((c * PG + g) * (int)sizeof(V));
  V a0[CC], a1[CC];
  pair_fetch<V, CC>(a0, rs, voff, 0, n);
  const V* x0 = xh + k * (long long)nrhs * n + (long long)r0 * n;
  const V* x1 = xh + kb * (long long)nrhs * n + (long long)r0 * n;
  for (int e = threadIdx.x; e < NR * cols_pad; e += PNT) {
    const int r = e / cols_pad, v = e - r * cols_pad;
    xs[v * NR + r] = (r < nr && v < n) ? x0[(long long)r * n + v] : V{0, 0};
  }
  for (int e = threadIdx.x; e < NR * rows_pad; e += PNT) {
    const int r = e / rows_pad, u = e - r * rows_pad;
    V val{0, 0};
    if (r < nr && u < n) {
      const V x = x1[(long long)r * n + u];
      val = V{w[u] * x.x, w[u] * x.y};
    }
    xt[u * NR + r] = val;
  }
  for (int e = threadIdx.x; e < 4 * NR * n; e += PNT) ys[e] = 0;  // ys and zs
  __syncthreads();
  T zr[CC][NR], zi[CC][NR];
#pragma unroll
  for (int j = 0; j < CC; ++j)
#pragma unroll
    for (int r = 0; r < NR; ++r) { zr[j][r] = 0; zi[j][r] = 0; }
  // two register stages used alternately; the next row is requested before
  // the current one is multiplied.  The requests are unconditional (a row
  // index past the end re-reads the last row, a cache hit) so that every
  // wait before a multiply covers only the older stage.
  for (int i = 0; i < RR; i += 2) {
    pair_fetch<V, CC>(a1, rs, voff, i + 1 < RR ? i + 1 : RR - 1, n);
    __builtin_amdgcn_sched_barrier(0);
    pair_row<V, CC, NR>(a0, i, g, c, n, xs, xt, ys, zr, zi);
    pair_fetch<V, CC>(a0, rs, voff, i + 2 < RR ? i + 2 : RR - 1, n);
    __builtin_amdgcn_sched_barrier(0);
    if (i + 1 < RR) pair_row<V, CC, NR>(a1, i + 1, g, c, n, xs, xt, ys, zr, zi);
  }
  if (!self) {
#pragma unroll
    for (int j = 0; j < CC; ++j) {
      const int v = c + PCS * j;
      if (v < n) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          atomicAdd(zs + 2 * (r * n + v), zr[j][r]);
          atomicAdd(zs + 2 * (r * n + v) + 1, zi[j][r]);
        }
      }
    }
  }
  __syncthreads();
  V* y0 = yh + k * (long long)nrhs * n + (long long)r0 * n;
  for (int e = threadIdx.x; e < nr * n; e += PNT) y0[e] = V{ys[2 * e], ys[2 * e + 1]};
  if (!self) {
    V* y1 = yh + kb * (long long)nrhs * n + (long long)r0 * n;
    for (int e = threadIdx.x; e < nr * n; e += PNT) {
      const int v = e % n;
      y1[e] = V{zs[2 * e] * winv[v], zs[2 * e + 1] * winv[v]};
    }
  }
}

template <typename V, int CC, int NR>
void launch_pair(const void* That, const void* pairs, const void* w, const void* winv, const void* xh, void* yh, int n,
                 int nrhs, int r0, int nr, int64_t Ps, hipStream_t s) {
  using T = typename Real<V>::T;
  constexpr int PG = pair_g<V>(), PCS = pair_cs<V>();
  const int rows_pad = (n + PG - 1) / PG * PG;
  const size_t shm = (size_t)(PCS * CC + rows_pad) * NR * sizeof(V) + (size_t)4 * NR * n * sizeof(T);
  hipLaunchKernelGGL((pair_gemv_kernel<V, CC, NR>), dim3((unsigned)Ps), dim3(PNT), shm, s,
                     static_cast<const V*>(That), static_cast<const int2*>(pairs), static_cast<const T*>(w),
                     static_cast<const T*>(winv), static_cast<const V*>(xh), static_cast<V*>(yh), n, nrhs, r0, nr);
}

// ---- FP32: matrix cores (v_mfma_f32_16x16x4f32)
//
// Real embedding of the complex products: for an A operand of 16 rows x 4
// k-slots the slots are (source index pair, real / imaginary part), and the B
// operand columns are the real parts (columns r < NR) and imaginary parts
// (NR <= column < 2 NR) of the outputs:
//     part 0 (re M): B = [ xr | xi ],   part 1 (im M): B = [ -xi | xr ].
// Wavefront w owns u tiles w, w + 4, ... (TPW of them) and visits every v tile;
// for tile (t, q) it runs 8 MFMAs of the first product (A = the tile with rows
// u, read straight from HBM in the lane order of the store) into the tile's
// row accumulator, and 8 of the transposed product (A = the tile transposed,
// staged through LDS) into the v tile's column sums, which are added into
// LDS once per v tile.  Up to 8 right-hand sides per pass (2 NR <= 16 MFMA
// columns).

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4v ld_tile(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff) {
  return __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 2));
}

// TPW u tiles per wavefront; NRW right-hand sides per pass (4 or 8: the
// MFMA columns used, 2 NRW of 16)
template <int TPW, int NRW>
__global__ void __launch_bounds__(PNT, 2) pair_f32_kernel(const float* __restrict__ That, const int2* __restrict__ pairs,
                                                          const float* __restrict__ w, const float* __restrict__ winv,
                                                          const float2* __restrict__ xh, float2* __restrict__ yh, int n,
                                                          int nrhs, int r0, int nr) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nt = pair_tiles(n), np = nt * PAIR_TILE;
  float* xs = reinterpret_cast<float*>(smem_raw);  // [np][NRW][2]: xh[k]
  float* xt = xs + np * NRW * 2;                 // [np][NRW][2]: W xh[-k]
  float* zs = xt + np * NRW * 2;                 // [np][2 NRW]: column sums
  float* tiles = zs + np * 2 * NRW;              // [4 waves][2 stages][512]
  const long long slot = blockIdx.x;
  const int2 pr = pairs[slot];
  const long long k = pr.x, kb = pr.y;
  const bool self = k == kb;
  const int l = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ntw = (nt - wv + 3) / 4;  // u tiles of this wavefront (<= TPW)
  const long long blk = (long long)nt * nt * 2 * PAIR_TILE * PAIR_TILE;  // floats
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(That + slot * blk), (short)0, (int)(blk * (long long)sizeof(float)), 0x00020000);
  const unsigned voff = (unsigned)(l * 16);   // registers 0-3; registers 4-7 sit 1024 bytes on
  // this wavefront's tiles are stored contiguously in visiting order
  // it = q * ntw + ta (u tile wv + 4 ta, v tile q)
  const int nvisit = ntw * nt, wbase_tile = pair_wave_base(nt, wv);
  auto visit_off = [&](int it) {
    if (it > nvisit - 1) it = nvisit - 1;
    return (wbase_tile + it) * (2 * PAIR_TILE * PAIR_TILE * 4);
  };
  // two tiles in flight: p (current) and nx (next)
  f4v p0{0, 0, 0, 0}, p1{0, 0, 0, 0}, nx0{0, 0, 0, 0}, nx1{0, 0, 0, 0};
  if (ntw > 0) {
    p0 = ld_tile(rs, voff, visit_off(0));
    p1 = ld_tile(rs, voff + 1024, visit_off(0));
    nx0 = ld_tile(rs, voff, visit_off(1));
    nx1 = ld_tile(rs, voff + 1024, visit_off(1));
  }
  const float2* x0 = xh + k * (long long)nrhs * n + (long long)r0 * n;
  const float2* x1 = xh + kb * (long long)nrhs * n + (long long)r0 * n;
  for (int e = threadIdx.x; e < np * NRW; e += PNT) {
    const int r = e / np, v = e - r * np;
    float2 a{0, 0}, b{0, 0};
    if (r < nr && v < n) {
      a = x0[(long long)r * n + v];
      const float2 c = x1[(long long)r * n + v];
      b = float2{w[v] * c.x, w[v] * c.y};
    }
    xs[(v * NRW + r) * 2] = a.x;
    xs[(v * NRW + r) * 2 + 1] = a.y;
    xt[(v * NRW + r) * 2] = b.x;
    xt[(v * NRW + r) * 2 + 1] = b.y;
  }
  for (int e = threadIdx.x; e < np * 2 * NRW; e += PNT) zs[e] = 0.f;
  __syncthreads();
  // lane roles: k-slot kk = l / 16 -> (pair offset off, part); column jj = l % 16
  const int kk = l >> 4, jj = l & 15, off = kk >> 1, part = kk & 1, a16 = l & 15;
  const bool jre = jj < NRW, jok = jj < 2 * NRW;
  const int rj = jre ? jj : (jok ? jj - NRW : 0);
  auto bval = [&](const float* x, int idx) {
    const float xr = x[(idx * NRW + rj) * 2], xi = x[(idx * NRW + rj) * 2 + 1];
    const float val = part == 0 ? (jre ? xr : xi) : (jre ? -xi : xr);
    return jok ? val : 0.f;
  };
  float b2[TPW][8];
#pragma unroll
  for (int ta = 0; ta < TPW; ++ta)
#pragma unroll
    for (int s = 0; s < 8; ++s) b2[ta][s] = ta < ntw ? bval(xt, (wv + 4 * ta) * PAIR_TILE + 2 * s + off) : 0.f;
  f4v acc[TPW];
#pragma unroll
  for (int ta = 0; ta < TPW; ++ta) acc[ta] = f4v{0, 0, 0, 0};
  // transposed staging: value s of this lane, entry (u = a16, v = 2 s + off, part), goes to
  // ((v * 2 + part) * 2 + u % 2) * 8 + u / 2; lane l then reads its 8 transposed operands
  // (u = 2 s + off, v = a16, part) as 8 consecutive floats
  const int wbase = (part * 2 + (a16 & 1)) * 8 + (a16 >> 1);
  const int rbase = ((a16 * 2 + part) * 2 + off) * 8;
  float* tw = tiles + wv * 2 * 512;
  int stage = 0;
  // B operands of the first product for v tile q, built one v tile ahead
  float b1n[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) b1n[s] = bval(xs, 2 * s + off);
  for (int q = 0; q < nt; ++q) {
    float b1[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) b1[s] = b1n[s];
    const int qn = q + 1 < nt ? q + 1 : q;
#pragma unroll
    for (int s = 0; s < 8; ++s) b1n[s] = bval(xs, qn * PAIR_TILE + 2 * s + off);
    f4v zq{0, 0, 0, 0};
#pragma unroll
    for (int ta = 0; ta < TPW; ++ta) {
      if (ta < ntw) {
        const float a1[8] = {p0[0], p0[1], p0[2], p0[3], p1[0], p1[1], p1[2], p1[3]};
        float* T = tw + stage * 512;
#pragma unroll
        for (int s = 0; s < 8; ++s) T[(2 * s + off) * 32 + wbase] = a1[s];
        __builtin_amdgcn_wave_barrier();
        const f4v c0 = *reinterpret_cast<const f4v*>(T + rbase), c1 = *reinterpret_cast<const f4v*>(T + rbase + 4);
        const int noff = visit_off(q * ntw + ta + 2);
        p0 = nx0;
        p1 = nx1;
        nx0 = ld_tile(rs, voff, noff);
        nx1 = ld_tile(rs, voff + 1024, noff);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < 8; ++s) acc[ta] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[s], b1[s], acc[ta], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        const float a2[8] = {c0[0], c0[1], c0[2], c0[3], c1[0], c1[1], c1[2], c1[3]};
#pragma unroll
        for (int s = 0; s < 8; ++s) zq = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[s], b2[ta][s], zq, 0, 0, 0);
        stage ^= 1;
      }
    }
    // D layout: register e of lane l holds row 4 (l / 16) + e, column l % 16
    if (!self && ntw > 0) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (jok) atomicAdd(&zs[(q * PAIR_TILE + 4 * (l >> 4) + e) * 2 * NRW + jj], zq[e]);
    }
  }
  // outputs: the row sums are staged in LDS over the spectral columns of
  // xh[k] (no longer read once every wavefront is past its loop), in the
  // layout of the column sums, and both products leave as coalesced
  // non-temporal stores, two complex values per 16-byte store when n is even
  __syncthreads();
  float* ys = xs;  // [np][2 NRW]: row sums (yh[k])
#pragma unroll
  for (int ta = 0; ta < TPW; ++ta) {
    if (ta < ntw) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int u = (wv + 4 * ta) * PAIR_TILE + 4 * (l >> 4) + e;
        if (jok) ys[u * 2 * NRW + jj] = acc[ta][e];
      }
    }
  }
  __syncthreads();
  float2* y0 = yh + k * (long long)nrhs * n + (long long)r0 * n;
  float2* y1 = yh + kb * (long long)nrhs * n + (long long)r0 * n;
  if ((n & 1) == 0) {
    for (int e2 = threadIdx.x; e2 < nr * n / 2; e2 += PNT) {
      const int e = 2 * e2, r = e / n, v = e - r * n;   // v + 1 < n in the same row r
      const int c0 = v * 2 * NRW + r, c1 = c0 + 2 * NRW;
      const f4v a = {ys[c0], ys[c0 + NRW], ys[c1], ys[c1 + NRW]};
      __builtin_nontemporal_store(a, reinterpret_cast<f4v*>(y0 + e));
      if (!self) {
        const float w0 = winv[v], w1 = winv[v + 1];
        const f4v b = {zs[c0] * w0, zs[c0 + NRW] * w0, zs[c1] * w1, zs[c1 + NRW] * w1};
        __builtin_nontemporal_store(b, reinterpret_cast<f4v*>(y1 + e));
      }
    }
  } else {
    for (int e = threadIdx.x; e < nr * n; e += PNT) {
      const int r = e / n, v = e - r * n;
      const int c0 = v * 2 * NRW + r;
      y0[e] = float2{ys[c0], ys[c0 + NRW]};
      if (!self) y1[e] = float2{zs[c0] * winv[v], zs[c0 + NRW] * winv[v]};
    }
  }
}

template <int TPW, int NRW>
void launch_f32(const void* That, const void* pairs, const void* w, const void* winv, const void* xh, void* yh, int n,
                int nrhs, int r0, int nr, int64_t Ps, hipStream_t s) {
  const int np = pair_tiles(n) * PAIR_TILE;
  const size_t shm = (size_t)(np * NRW * 2 * 3 + 4 * 2 * 512) * sizeof(float);
  hipLaunchKernelGGL((pair_f32_kernel<TPW, NRW>), dim3((unsigned)Ps), dim3(PNT), shm, s, static_cast<const float*>(That),
                     static_cast<const int2*>(pairs), static_cast<const float*>(w), static_cast<const float*>(winv),
                     static_cast<const float2*>(xh), static_cast<float2*>(yh), n, nrhs, r0, nr);
}

template <int TPW>
void launch_f32_tpw(int nrw, const void* That, const void* pairs, const void* w, const void* winv, const void* xh,
                    void* yh, int n, int nrhs, int r0, int nr, int64_t Ps, hipStream_t s) {
  if (nrw == 4)
    launch_f32<TPW, 4>(That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s);
  else
    launch_f32<TPW, 8>(That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s);
}

void launch_pair_f32(const void* That, const void* pairs, const void* w, const void* winv, const void* xh, void* yh,
                     int n, int nrhs, int64_t Ps, hipStream_t s) {
  const int tpw = (pair_tiles(n) + 3) / 4;
  // 4-wide passes for at most 4 right-hand sides (less LDS, more workgroups per CU)
  const int nrw = nrhs <= 4 ? 4 : 8;
  for (int r0 = 0; r0 < nrhs; r0 += nrw) {
    const int nr = nrhs - r0 < nrw ? nrhs - r0 : nrw;
    switch (tpw) {
      case 1: launch_f32_tpw<1>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      case 2: launch_f32_tpw<2>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      case 3: launch_f32_tpw<3>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      case 4: launch_f32_tpw<4>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      case 5: launch_f32_tpw<5>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      case 6: launch_f32_tpw<6>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      case 7: launch_f32_tpw<7>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      default: launch_f32_tpw<8>(nrw, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
    }
  }
}

// ---- FP64: row panels of 4 rows, atomics for the row sums

// Columns per lane (64 CC >= n).  The transposed product keeps CC x NR
// complex accumulators per lane; NR is capped so that CC NR <= 12.
inline int pair_cc64(int n) { return n <= 192 ? 3 : n <= 384 ? 6 : 8; }

template <int CC>
void launch_pair_cc64(int NR, const void* That, const void* pairs, const void* w, const void* winv, const void* xh,
                      void* yh, int n, int nrhs, int r0, int nr, int64_t Ps, hipStream_t s) {
  switch (NR) {
    case 1: launch_pair<double2, CC, 1>(That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
    case 2: if constexpr (2 * CC <= 12) launch_pair<double2, CC, 2>(That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
    default: if constexpr (4 * CC <= 12) launch_pair<double2, CC, 4>(That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
  }
}

void launch_pair_f64(const void* That, const void* pairs, const void* w, const void* winv, const void* xh, void* yh,
                     int n, int nrhs, int64_t Ps, hipStream_t s) {
  const int CC = pair_cc64(n);
  int NR = 1;
  while (NR < nrhs && NR * 2 <= 4 && CC * NR * 2 <= 12) NR *= 2;
  for (int r0 = 0; r0 < nrhs; r0 += NR) {
    const int nr = nrhs - r0 < NR ? nrhs - r0 : NR;
    switch (CC) {
      case 3: launch_pair_cc64<3>(NR, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      case 6: launch_pair_cc64<6>(NR, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
      default: launch_pair_cc64<8>(NR, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
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
    launch_pair_f64(That, pairs, w, winv, xh, yh, n, nrhs, Ps, s);
  else
    launch_pair_f32(That, pairs, w, winv, xh, yh, n, nrhs, Ps, s);
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
