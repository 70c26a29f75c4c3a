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

// ---- FP32: half-wavefront rows

template <int K> __device__ __forceinline__ float dpp_ror(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x120 + K, 0xF, 0xF, false));
}
// sum over the 32 lanes of a half-wavefront, returned in every lane: rotations
// by 8, 4, 2, 1 within each 16-lane row, then the two rows exchanged
__device__ __forceinline__ float half_wave_sum(float v) {
  v += dpp_ror<8>(v);
  v += dpp_ror<4>(v);
  v += dpp_ror<2>(v);
  v += dpp_ror<1>(v);
  return v + __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), 0x401F));
}

// CC column tiles (32 CC >= n, CC = ceil(n / 32)); NR right-hand sides per
// pass, nr <= NR of them valid.  LDS: W xh[-k] as [rows_pad][NR], xh[k] as NR
// planes of 32 CC, row sums and column sums as [NR][n][2].
template <int CC, int NR>
__global__ void __launch_bounds__(PNT, 4) pair_f32_kernel(const float2* __restrict__ That, const int2* __restrict__ pairs,
                                                          const float* __restrict__ w, const float* __restrict__ winv,
                                                          const float2* __restrict__ xh, float2* __restrict__ yh, int n,
                                                          int nrhs, int r0, int nr) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int RR = (n + PAIR_TILE_ROWS - 1) / PAIR_TILE_ROWS, rows_pad = PAIR_TILE_ROWS * RR;
  constexpr int cols_pad = PAIR_TILE_COLS * CC;
  float2* xt = reinterpret_cast<float2*>(smem_raw);        // [rows_pad][NR]: W xh[-k]
  float2* xs = xt + rows_pad * NR;                         // [NR][cols_pad]: xh[k]
  float* ys = reinterpret_cast<float*>(xs + NR * cols_pad);  // [NR][n][2]: yh[k]
  float* zs = ys + 2 * NR * n;                             // [NR][n][2]: W yh[-k]
  const long long slot = blockIdx.x;
  const int2 pr = pairs[slot];
  const long long k = pr.x, kb = pr.y;
  const bool self = k == kb;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, c = lane & 31, g = 2 * wv + (lane >> 5);
  const long long blk = (long long)rows_pad * cols_pad;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(That + slot * blk), (short)0, (int)(blk * (long long)sizeof(float2)), 0x00020000);
  // a wavefront's 64 lanes read tile rows 2 wv and 2 wv + 1: 512 contiguous bytes
  const unsigned voff = (unsigned)((64 * wv + lane) * (int)sizeof(float2));
  auto fetch = [&](float2 (&a)[CC], int i) {
#pragma unroll
    for (int j = 0; j < CC; ++j) a[j] = ld_elem<float2>(rs, voff, (i * CC + j) * (PAIR_TILE_ROWS * PAIR_TILE_COLS * 8));
  };
  float2 a0[CC], a1[CC];
  fetch(a0, 0);
  const float2* x0 = xh + k * (long long)nrhs * n + (long long)r0 * n;
  const float2* x1 = xh + kb * (long long)nrhs * n + (long long)r0 * n;
  for (int e = threadIdx.x; e < NR * cols_pad; e += PNT) {
    const int r = e / cols_pad, v = e - r * cols_pad;
    xs[e] = (r < nr && v < n) ? x0[(long long)r * n + v] : float2{0, 0};
  }
  for (int e = threadIdx.x; e < NR * rows_pad; e += PNT) {
    const int r = e / rows_pad, u = e - r * rows_pad;
    float2 val{0, 0};
    if (r < nr && u < n) {
      const float2 x = x1[(long long)r * n + u];
      val = float2{w[u] * x.x, w[u] * x.y};
    }
    xt[u * NR + r] = val;
  }
  for (int e = threadIdx.x; e < 4 * NR * n; e += PNT) ys[e] = 0;  // ys and zs
  __syncthreads();
  float zr[CC][NR], zi[CC][NR];
#pragma unroll
  for (int j = 0; j < CC; ++j)
#pragma unroll
    for (int r = 0; r < NR; ++r) { zr[j][r] = 0; zi[j][r] = 0; }
  auto row = [&](const float2 (&a)[CC], int i) {
    const int u = g + PAIR_TILE_ROWS * i;
    float2 xr[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) xr[r] = xt[u * NR + r];
    float yr[NR], yi[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) { yr[r] = 0; yi[r] = 0; }
#pragma unroll
    for (int j = 0; j < CC; ++j) {
      const float2 av = a[j];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const float2 x = xs[r * cols_pad + c + PAIR_TILE_COLS * j];
        yr[r] = fma_r(av.x, x.x, yr[r]);
        yr[r] = fma_r(-av.y, x.y, yr[r]);
        yi[r] = fma_r(av.x, x.y, yi[r]);
        yi[r] = fma_r(av.y, x.x, yi[r]);
        zr[j][r] = fma_r(av.x, xr[r].x, zr[j][r]);
        zr[j][r] = fma_r(-av.y, xr[r].y, zr[j][r]);
        zi[j][r] = fma_r(av.x, xr[r].y, zi[j][r]);
        zi[j][r] = fma_r(av.y, xr[r].x, zi[j][r]);
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      yr[r] = half_wave_sum(yr[r]);
      yi[r] = half_wave_sum(yi[r]);
    }
    if (c == 0 && u < n) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        ys[2 * (r * n + u)] = yr[r];
        ys[2 * (r * n + u) + 1] = yi[r];
      }
    }
  };
  for (int i = 0; i < RR; i += 2) {
    fetch(a1, i + 1 < RR ? i + 1 : RR - 1);
    __builtin_amdgcn_sched_barrier(0);
    row(a0, i);
    fetch(a0, i + 2 < RR ? i + 2 : RR - 1);
    __builtin_amdgcn_sched_barrier(0);
    if (i + 1 < RR) row(a1, i + 1);
  }
  if (!self) {
#pragma unroll
    for (int j = 0; j < CC; ++j) {
      const int v = c + PAIR_TILE_COLS * j;
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
  float2* y0 = yh + k * (long long)nrhs * n + (long long)r0 * n;
  for (int e = threadIdx.x; e < nr * n; e += PNT) y0[e] = float2{ys[2 * e], ys[2 * e + 1]};
  if (!self) {
    float2* y1 = yh + kb * (long long)nrhs * n + (long long)r0 * n;
    for (int e = threadIdx.x; e < nr * n; e += PNT) {
      const int v = e % n;
      y1[e] = float2{zs[2 * e] * winv[v], zs[2 * e + 1] * winv[v]};
    }
  }
}

template <int CC, int NR>
void launch_f32(const void* That, const void* pairs, const void* w, const void* winv, const void* xh, void* yh, int n,
                int nrhs, int r0, int nr, int64_t Ps, hipStream_t s) {
  const int rows_pad = (n + PAIR_TILE_ROWS - 1) / PAIR_TILE_ROWS * PAIR_TILE_ROWS;
  const size_t shm = (size_t)(rows_pad + PAIR_TILE_COLS * CC) * NR * sizeof(float2) + (size_t)4 * NR * n * sizeof(float);
  hipLaunchKernelGGL((pair_f32_kernel<CC, NR>), dim3((unsigned)Ps), dim3(PNT), shm, s,
                     static_cast<const float2*>(That), static_cast<const int2*>(pairs), static_cast<const float*>(w),
                     static_cast<const float*>(winv), static_cast<const float2*>(xh), static_cast<float2*>(yh), n, nrhs,
                     r0, nr);
}

// FP32 right-hand sides per pass: column sums take CC x NR complex registers,
// at most 24
constexpr int f32_nr_max(int CC) { return CC <= 2 ? 8 : CC <= 6 ? 4 : CC <= 12 ? 2 : 1; }

template <int CC>
void launch_f32_cc(int NR, const void* That, const void* pairs, const void* w, const void* winv, const void* xh,
                   void* yh, int n, int nrhs, int r0, int nr, int64_t Ps, hipStream_t s) {
  switch (NR) {
    case 1: launch_f32<CC, 1>(That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
    case 2: if constexpr (f32_nr_max(CC) >= 2) launch_f32<CC, 2>(That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
    case 4: if constexpr (f32_nr_max(CC) >= 4) launch_f32<CC, 4>(That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
    default: if constexpr (f32_nr_max(CC) >= 8) launch_f32<CC, 8>(That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s); break;
  }
}

template <int... C>
void launch_f32_dispatch(std::integer_sequence<int, C...>, int CC, int NR, const void* That, const void* pairs,
                         const void* w, const void* winv, const void* xh, void* yh, int n, int nrhs, int r0, int nr,
                         int64_t Ps, hipStream_t s) {
  ((CC == C + 1 ? launch_f32_cc<C + 1>(NR, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr, Ps, s) : void()), ...);
}

void launch_pair_f32(const void* That, const void* pairs, const void* w, const void* winv, const void* xh, void* yh,
                     int n, int nrhs, int64_t Ps, hipStream_t s) {
  const int CC = pair_col_tiles(n);
  int NR = 1;
  while (NR < nrhs && NR * 2 <= f32_nr_max(CC)) NR *= 2;
  for (int r0 = 0; r0 < nrhs; r0 += NR) {
    const int nr = nrhs - r0 < NR ? nrhs - r0 : NR;
    launch_f32_dispatch(std::make_integer_sequence<int, 16>{}, CC, NR, That, pairs, w, winv, xh, yh, n, nrhs, r0, nr,
                        Ps, s);
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
