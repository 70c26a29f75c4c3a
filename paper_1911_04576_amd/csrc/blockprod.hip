// Fourier-domain block products of the FFT-accelerated coupling apply
// (Sec. IV-B): after the forward transforms every frequency k holds an n x n
// block T^(k) and the n x nrhs spectral columns of x; the sum over source
// unknowns v ("four 1-D FFTs" for two local bases, i.e. accumulation in the
// Fourier domain) is a small complex matrix product per frequency:
//     yh[k][r][u] = sum_v That[k](u, v) xh[k][r][v].
//
// This is HBM-bound for few right-hand sides (each block is used once per
// apply), so the kernel is built to stream That exactly once at full
// bandwidth: one workgroup per frequency, one lane per row u, the block stored
// column-major ([k][v][u]) so that a wavefront's load of a column is one
// contiguous run; the spectral columns xh[k] sit in LDS and are read as
// broadcasts; That is loaded with non-temporal hints since it is never reused
// within an apply.  Input and output spectra are distinct buffers, so large
// right-hand-side counts may be processed in several passes.
#include "internal.h"

namespace emsurf {
namespace {

template <typename V> struct Real;
template <> struct Real<float2> { using T = float; };
template <> struct Real<double2> { using T = double; };

template <typename V> __device__ __forceinline__ V ld_nt(const V* p);
template <> __device__ __forceinline__ double2 ld_nt<double2>(const double2* p) {
  return double2{__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y)};
}
template <> __device__ __forceinline__ float2 ld_nt<float2>(const float2* p) {
  // one 64-bit load
  const unsigned long long* q = reinterpret_cast<const unsigned long long*>(p);
  unsigned long long v = __builtin_nontemporal_load(q);
  float2 r;
  __builtin_memcpy(&r, &v, sizeof(r));
  return r;
}

// NR: right-hand sides handled per pass (compile time); nr <= NR valid ones.
template <typename V, int NR>
__global__ void __launch_bounds__(512) block_gemv_kernel(const V* __restrict__ That, const V* __restrict__ xh, V* __restrict__ yh, int n,
                                                         int nrhs, int r0, int nr) {
  using T = typename Real<V>::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* xs = reinterpret_cast<V*>(smem_raw);  // [v][NR]
  const long long k = blockIdx.x;
  const V* xk = xh + k * (long long)nrhs * n + (long long)r0 * n;
  for (int i = threadIdx.x; i < NR * n; i += blockDim.x) {
    const int r = i / n, v = i - r * n;
    xs[v * NR + r] = (r < nr) ? xk[(long long)r * n + v] : V{0, 0};
  }
  __syncthreads();
  const int u = threadIdx.x;
  if (u >= n) return;
  T ar[NR], ai[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) { ar[r] = 0; ai[r] = 0; }
  const V* A = That + k * (long long)n * n + u;
  int v = 0;
  constexpr int U = 8;
  for (; v + U <= n; v += U) {
    V a[U];
#pragma unroll
    for (int j = 0; j < U; ++j) a[j] = ld_nt(A + (long long)(v + j) * n);
#pragma unroll
    for (int j = 0; j < U; ++j) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const V x = xs[(v + j) * NR + r];
        ar[r] += a[j].x * x.x - a[j].y * x.y;
        ai[r] += a[j].x * x.y + a[j].y * x.x;
      }
    }
  }
  for (; v < n; ++v) {
    const V a = ld_nt(A + (long long)v * n);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const V x = xs[v * NR + r];
      ar[r] += a.x * x.x - a.y * x.y;
      ai[r] += a.x * x.y + a.y * x.x;
    }
  }
  V* yk = yh + k * (long long)nrhs * n + (long long)r0 * n;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (r < nr) yk[(long long)r * n + u] = V{ar[r], ai[r]};
}

template <typename V, int NR>
void launch_nr(const void* That, const void* xh, void* yh, int n, int nrhs, int r0, int nr, int64_t P,
               hipStream_t s) {
  const int threads = ((n + 63) / 64) * 64;
  const size_t shm = (size_t)n * NR * sizeof(V);
  hipLaunchKernelGGL((block_gemv_kernel<V, NR>), dim3((unsigned)P), dim3(threads), shm, s,
                     static_cast<const V*>(That), static_cast<const V*>(xh), static_cast<V*>(yh), n, nrhs, r0, nr);
}

template <typename V>
void launch_t(const void* That, const void* xh, void* yh, int n, int nrhs, int64_t P, hipStream_t s) {
  // Right-hand sides per pass: bounded by 64 KB of LDS for the spectral columns
  // and by the accumulator registers (16 FP64 / 32 FP32 complex per lane).
  int cap = (int)(65536 / ((size_t)n * sizeof(V)));
  const int reg_cap = sizeof(V) == 16 ? 16 : 32;
  if (cap > reg_cap) cap = reg_cap;
  int NR = 1;
  while (NR < nrhs && NR * 2 <= cap) NR *= 2;
  for (int r0 = 0; r0 < nrhs; r0 += NR) {
    const int nr = nrhs - r0 < NR ? nrhs - r0 : NR;
    switch (NR) {
      case 1: launch_nr<V, 1>(That, xh, yh, n, nrhs, r0, nr, P, s); break;
      case 2: launch_nr<V, 2>(That, xh, yh, n, nrhs, r0, nr, P, s); break;
      case 4: launch_nr<V, 4>(That, xh, yh, n, nrhs, r0, nr, P, s); break;
      case 8: launch_nr<V, 8>(That, xh, yh, n, nrhs, r0, nr, P, s); break;
      case 16: launch_nr<V, 16>(That, xh, yh, n, nrhs, r0, nr, P, s); break;
      default: launch_nr<V, 32>(That, xh, yh, n, nrhs, r0, nr, P, s); break;
    }
  }
}

// ----------------------------------------------------------------------------- MFMA path
// Many right-hand sides make each frequency a small dense GEMM.  The complex
// product y = A x is the real product of the interleaved block (n x 2n real,
// column index 2v + re/im) with the 2n x 2nrhs real embedding of x:
//   [Re y_r] = sum_v Ar Br - Ai Bi,   [Im y_r] = sum_v Ar Bi + Ai Br,
// run on v_mfma_f32_32x32x2f32.  A lane supplies A[row][k] for one row of a
// 32-row tile and one of two block columns per instruction; with the
// column-major store ([v][u]) the wave's load of two columns x 32 rows is two
// contiguous 256-byte runs, fed straight from HBM into operand registers
// (double-buffered, non-temporal).  Each wave owns TPW row tiles (one group;
// at most 4 waves) and 16 right-hand sides; the spectral columns sit in LDS
// (rows padded to spread banks) and the outputs are staged through the same
// LDS for coalesced stores once every wave is done reading it.
typedef float floatx16 __attribute__((ext_vector_type(16)));

// 8-byte non-temporal buffer load (out-of-range offsets read zero)
__device__ __forceinline__ float2 ld_buf(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff) {
  auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 2);
  float2 f;
  __builtin_memcpy(&f, &v, sizeof(f));
  return f;
}

template <int TPW, int U>
__global__ void __launch_bounds__(256) block_mfma_kernel(const float2* __restrict__ That,
                                                         const float2* __restrict__ xh, float2* __restrict__ yh,
                                                         int n, int nrhs, int r0, int nr) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2* xs = reinterpret_cast<float2*>(smem_raw);     // [16][n + 1]
  constexpr int NR = 16;
  const int ld = n + 1;
  const long long k = blockIdx.x;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int jl = lane & 31;
  const int ntile = n >> 5;
  const int rsel = jl >> 1;
  const bool dimag = (jl & 1) != 0;
  int tile[TPW];
  bool tv[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    tile[i] = wave * TPW + i;
    tv[i] = tile[i] < ntile;
  }
  floatx16 acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[i][e] = 0.f;
  // The frequency's block is read through a buffer resource: a uniform base,
  // per-lane byte offsets that stay fixed (column h, row tile*32 + jl; a tile
  // past the end re-reads tile 0 and its results are dropped) and a uniform
  // per-step offset, which keeps address arithmetic out of the vector registers.
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(That + k * (long long)n * n), (short)0, n * n * (int)sizeof(float2), 0x00020000);
  unsigned aoff[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) aoff[i] = (unsigned)((h * n + (tv[i] ? tile[i] * 32 : 0) + jl) * sizeof(float2));
  const int step_bytes = 2 * n * (int)sizeof(float2);   // two block columns
  // first block columns are requested before the spectral columns are staged,
  // so the two latencies overlap
  float2 acur[U][TPW], anxt[U][TPW];
#pragma unroll
  for (int st = 0; st < U; ++st)
#pragma unroll
    for (int i = 0; i < TPW; ++i) acur[st][i] = ld_buf(rs, aoff[i], st * step_bytes);
  const float2* xk = xh + k * (long long)nrhs * n + (long long)r0 * n;
  for (int i = threadIdx.x; i < NR * n; i += blockDim.x) {
    const int r = i / n, v = i - r * n;
    xs[r * ld + v] = (r < nr) ? xk[(long long)r * n + v] : float2{0.f, 0.f};
  }
  __syncthreads();
  for (int v0 = 0; v0 < n; v0 += 2 * U) {
    // the last prefetch runs past the block: buffer loads out of range read 0
#pragma unroll
    for (int st = 0; st < U; ++st)
#pragma unroll
      for (int i = 0; i < TPW; ++i) anxt[st][i] = ld_buf(rs, aoff[i], (v0 / 2 + U + st) * step_bytes);
    // keep the prefetch ahead of this step's MFMAs
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int st = 0; st < U; ++st) {
      const int v = v0 + 2 * st + h;
      const float2 xv = xs[rsel * ld + v];
      const float bre = dimag ? xv.y : xv.x;
      const float bim = dimag ? xv.x : -xv.y;
#pragma unroll
      for (int i = 0; i < TPW; ++i) acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(acur[st][i].x, bre, acc[i], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < TPW; ++i) acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(acur[st][i].y, bim, acc[i], 0, 0, 0);
    }
#pragma unroll
    for (int st = 0; st < U; ++st)
#pragma unroll
      for (int i = 0; i < TPW; ++i) acur[st][i] = anxt[st][i];
  }
  // stage outputs in LDS as [r][u] complex, then store the frequency's panel
  __syncthreads();
  float* ysf = reinterpret_cast<float*>(xs);
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    if (!tv[i]) continue;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int u = tile[i] * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
      ysf[2 * (rsel * ld + u) + (dimag ? 1 : 0)] = acc[i][e];
    }
  }
  __syncthreads();
  float2* yk = yh + k * (long long)nrhs * n + (long long)r0 * n;
  for (int i = threadIdx.x; i < nr * n; i += blockDim.x) {
    const int r = i / n, u = i - r * n;
    yk[(long long)r * n + u] = xs[r * ld + u];
  }
}

// row-tile groups (= wavefronts) for TPW tiles per wave
inline int mfma_waves(int n, int tpw) { return (n / 32 + tpw - 1) / tpw; }

template <int TPW, int U>
void launch_mfma(const void* That, const void* xh, void* yh, int n, int nrhs, int r0, int nr, int64_t P,
                 hipStream_t s) {
  const int waves = mfma_waves(n, TPW);
  EMS_CHECK_ARG(waves >= 1 && waves <= 4, "MFMA variant needs at most 4 wavefronts per frequency");
  EMS_CHECK_ARG((n / 2) % U == 0, "MFMA variant needs n_eq / 2 divisible by its prefetch depth");
  const size_t shm = (size_t)16 * (n + 1) * sizeof(float2);
  EMS_CHECK_ARG(shm <= 65536, "MFMA variant needs n_eq <= 480");
  hipLaunchKernelGGL((block_mfma_kernel<TPW, U>), dim3((unsigned)P), dim3(64 * waves), shm, s,
                     static_cast<const float2*>(That), static_cast<const float2*>(xh), static_cast<float2*>(yh), n,
                     nrhs, r0, nr);
}

}  // namespace

bool block_mfma_supported(int n, int nrhs) { return n % 32 == 0 && n >= 32 && n <= 480 && nrhs >= 1; }

// variant 1..4: k = variant row tiles per wave, 4 K steps prefetched;
// variant 5..8: k = variant - 4 row tiles per wave, 6 (n_eq % 96 == 0) or 8
// K steps prefetched
static int variant_tiles(int variant) { return variant <= BP_MFMA_T4 ? variant : variant - BP_MFMA_T4; }

bool block_variant_supported(int variant, int n, int nrhs) {
  if (variant == BP_GEMV) return true;
  if (variant < BP_MFMA_T1 || variant >= BP_NVARIANTS || !block_mfma_supported(n, nrhs)) return false;
  return mfma_waves(n, variant_tiles(variant)) <= 4;
}

void launch_block_product_variant(Cx t, int variant, const void* That, const void* xh, void* yh, int n, int nrhs,
                                  int64_t P, hipStream_t s) {
  EMS_CHECK_ARG(n >= 1 && n <= 512, "block product supports 1 <= n_eq <= 512");
  EMS_CHECK_ARG(nrhs >= 1 && nrhs <= 64, "block product supports 1 <= nrhs <= 64");
  EMS_CHECK_ARG(P >= 1 && P <= 0x7fffffffLL, "frequency count out of range");
  if (t == Cx::C128 || !block_variant_supported(variant, n, nrhs) || variant == BP_GEMV) {
    if (t == Cx::C128)
      launch_t<double2>(That, xh, yh, n, nrhs, P, s);
    else
      launch_t<float2>(That, xh, yh, n, nrhs, P, s);
  } else {
    // 16 right-hand sides per pass
    for (int r0 = 0; r0 < nrhs; r0 += 16) {
      const int nr = nrhs - r0 < 16 ? nrhs - r0 : 16;
      switch (variant) {
        case BP_MFMA_T1: launch_mfma<1, 4>(That, xh, yh, n, nrhs, r0, nr, P, s); break;
        case BP_MFMA_T2: launch_mfma<2, 4>(That, xh, yh, n, nrhs, r0, nr, P, s); break;
        case BP_MFMA_T3: launch_mfma<3, 4>(That, xh, yh, n, nrhs, r0, nr, P, s); break;
        case BP_MFMA_T4: launch_mfma<4, 4>(That, xh, yh, n, nrhs, r0, nr, P, s); break;
        // deep prefetch: 6 steps when n_eq / 2 is a multiple of 6, else 8
        case BP_MFMA_T1D:
          if (n % 96 == 0) launch_mfma<1, 6>(That, xh, yh, n, nrhs, r0, nr, P, s);
          else launch_mfma<1, 8>(That, xh, yh, n, nrhs, r0, nr, P, s);
          break;
        case BP_MFMA_T2D:
          if (n % 96 == 0) launch_mfma<2, 6>(That, xh, yh, n, nrhs, r0, nr, P, s);
          else launch_mfma<2, 8>(That, xh, yh, n, nrhs, r0, nr, P, s);
          break;
        case BP_MFMA_T3D:
          if (n % 96 == 0) launch_mfma<3, 6>(That, xh, yh, n, nrhs, r0, nr, P, s);
          else launch_mfma<3, 8>(That, xh, yh, n, nrhs, r0, nr, P, s);
          break;
        default:
          if (n % 96 == 0) launch_mfma<4, 6>(That, xh, yh, n, nrhs, r0, nr, P, s);
          else launch_mfma<4, 8>(That, xh, yh, n, nrhs, r0, nr, P, s);
          break;
      }
    }
  }
  EMS_LAUNCH_CHECK();
}

void launch_block_product(Cx t, const void* That, const void* xh, void* yh, int n, int nrhs, int64_t P,
                          hipStream_t s) {
  launch_block_product_variant(t, BP_GEMV, That, xh, yh, n, nrhs, P, s);
}

}  // namespace emsurf
