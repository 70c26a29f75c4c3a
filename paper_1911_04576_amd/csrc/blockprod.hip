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
// right-hand-side counts may be processed in several passes.  The FP32
// many-right-hand-side form on the matrix cores is in blockprod_mfma.hip;
// launch_block_product_variant below chooses between them.
#include "internal.h"

namespace emsurf {
namespace {

template <typename V> struct Real;
template <> struct Real<float2> { using T = float; };
template <> struct Real<double2> { using T = double; };

__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Non-temporal buffer loads of one complex entry: a uniform resource for the
// frequency's block, a per-lane byte offset (the row) and a uniform per-column
// offset, so that stepping through the columns costs no vector instructions.
// Callers keep every offset inside the block.
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
template <typename V> __device__ __forceinline__ V ld_col(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff);
template <> __device__ __forceinline__ float2 ld_col<float2>(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff) {
  auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 2);
  float2 f;
  __builtin_memcpy(&f, &v, sizeof(f));
  return f;
}
template <> __device__ __forceinline__ double2 ld_col<double2>(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff) {
  auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 2);
  double2 d;
  __builtin_memcpy(&d, &v, sizeof(d));
  return d;
}

// U consecutive block columns c0 .. c0+U-1 (indices clamped to the block with a
// uniform min: a stage past the end re-reads column n - 1)
template <typename V, int U>
__device__ __forceinline__ void gemv_fetch(V (&a)[U], __amdgpu_buffer_rsrc_t rs, unsigned voff, int c0, int n,
                                           int col_bytes) {
#pragma unroll
  for (int j = 0; j < U; ++j) {
    const int c = c0 + j < n ? c0 + j : n - 1;
    a[j] = ld_col<V>(rs, voff, c * col_bytes);
  }
}

// acc_r += sum_j a[j] * x[j][r], complex, as four real FMAs per term
template <typename V, int NR, int U, typename T>
__device__ __forceinline__ void gemv_stage_mac(const V (&a)[U], const V* __restrict__ x, T (&ar)[NR], T (&ai)[NR]) {
#pragma unroll
  for (int j = 0; j < U; ++j) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const V xv = x[j * NR + r];
      ar[r] = fma_r(a[j].x, xv.x, ar[r]);
      ar[r] = fma_r(-a[j].y, xv.y, ar[r]);
      ai[r] = fma_r(a[j].x, xv.y, ai[r]);
      ai[r] = fma_r(a[j].y, xv.x, ai[r]);
    }
  }
}

// Copy cnt complex values from LDS to global with non-temporal 16-byte stores
// (the output panel of a frequency is one contiguous run); an FP32 run that
// starts on an odd element falls back to 8-byte stores.
__device__ __forceinline__ void store_run(float2* __restrict__ dst, const float2* __restrict__ src, int cnt) {
  if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
    const int pairs = cnt >> 1;
    for (int i = threadIdx.x; i < pairs; i += blockDim.x)
      __builtin_nontemporal_store(reinterpret_cast<const fvec4*>(src)[i], reinterpret_cast<fvec4*>(dst) + i);
    if ((cnt & 1) && threadIdx.x == 0) dst[cnt - 1] = src[cnt - 1];
  } else {
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) dst[i] = src[i];
  }
}
__device__ __forceinline__ void store_run(double2* __restrict__ dst, const double2* __restrict__ src, int cnt) {
  for (int i = threadIdx.x; i < cnt; i += blockDim.x)
    __builtin_nontemporal_store(reinterpret_cast<const dvec2*>(src)[i], reinterpret_cast<dvec2*>(dst) + i);
}

// NR: right-hand sides handled per pass (compile time); nr <= NR valid ones.
// U: block columns per pipeline stage; U columns are in flight while the
// previous U are multiplied.  LDS holds the spectral columns as xs[v][NR] for
// v < npad = n rounded up to U (rows past n zero) and afterwards stages the
// outputs as [r][u] for contiguous stores.
template <typename V, int NR, int U>
__global__ void __launch_bounds__(512) block_gemv_kernel(const V* __restrict__ That, const V* __restrict__ xh, V* __restrict__ yh, int n,
                                                         int nrhs, int r0, int nr) {
  using T = typename Real<V>::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* xs = reinterpret_cast<V*>(smem_raw);  // [npad][NR], later [nr][n]
  const long long k = blockIdx.x;
  const int npad = (n + U - 1) / U * U;
  const int u = threadIdx.x;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(That + k * (long long)n * n), (short)0, n * n * (int)sizeof(V), 0x00020000);
  // lanes past the last row stream row n - 1 and store nothing
  const unsigned voff = (unsigned)((u < n ? u : n - 1) * (int)sizeof(V));
  const int col_bytes = n * (int)sizeof(V);
  // the first columns are requested before the spectral columns are staged
  V acur[U], anxt[U];
  gemv_fetch<V, U>(acur, rs, voff, 0, n, col_bytes);
  const V* xk = xh + k * (long long)nrhs * n + (long long)r0 * n;
  for (int i = threadIdx.x; i < NR * npad; i += blockDim.x) {
    const int r = i / npad, v = i - r * npad;
    xs[v * NR + r] = (r < nr && v < n) ? xk[(long long)r * n + v] : V{0, 0};
  }
  __syncthreads();
  T ar[NR], ai[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) { ar[r] = 0; ai[r] = 0; }
  // two register stages used alternately (no copies between them)
  for (int v0 = 0; v0 < npad; v0 += 2 * U) {
    gemv_fetch<V, U>(anxt, rs, voff, v0 + U, n, col_bytes);
    __builtin_amdgcn_sched_barrier(0);
    gemv_stage_mac<V, NR, U>(acur, xs + v0 * NR, ar, ai);
    gemv_fetch<V, U>(acur, rs, voff, v0 + 2 * U, n, col_bytes);
    __builtin_amdgcn_sched_barrier(0);
    if (v0 + U < npad) gemv_stage_mac<V, NR, U>(anxt, xs + (v0 + U) * NR, ar, ai);
  }
  __syncthreads();
  if (u < n) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (r < nr) xs[r * n + u] = V{ar[r], ai[r]};
  }
  __syncthreads();
  store_run(yh + k * (long long)nrhs * n + (long long)r0 * n, xs, nr * n);
}

// columns per pipeline stage: deep for few right-hand sides (more bytes in
// flight per lane), shallower when accumulators already take the registers
template <typename V, int NR> constexpr int gemv_stage() {
  return sizeof(V) == 8 ? (NR <= 8 ? 8 : 4) : (NR <= 4 ? 4 : 2);
}

template <typename V, int NR>
void launch_nr(const void* That, const void* xh, void* yh, int n, int nrhs, int r0, int nr, int64_t P,
               hipStream_t s) {
  constexpr int U = gemv_stage<V, NR>();
  const int threads = ((n + 63) / 64) * 64;
  const int npad = (n + U - 1) / U * U;
  const size_t shm = (size_t)npad * NR * sizeof(V);
  hipLaunchKernelGGL((block_gemv_kernel<V, NR, U>), dim3((unsigned)P), dim3(threads), shm, s,
                     static_cast<const V*>(That), static_cast<const V*>(xh), static_cast<V*>(yh), n, nrhs, r0, nr);
}

template <typename V>
void launch_t(const void* That, const void* xh, void* yh, int n, int nrhs, int64_t P, hipStream_t s) {
  // Right-hand sides per pass: bounded by 64 KB of LDS for the spectral columns
  // (n rounded up to the pipeline stage) and by the accumulator registers
  // (16 FP64 / 32 FP32 complex per lane).
  int cap = (int)(65536 / ((size_t)(n + 7) * sizeof(V)));
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

}  // namespace

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
    launch_block_mfma(variant, That, xh, yh, n, nrhs, P, s);
  }
  EMS_LAUNCH_CHECK();
}

void launch_block_product(Cx t, const void* That, const void* xh, void* yh, int n, int nrhs, int64_t P,
                          hipStream_t s) {
  launch_block_product_variant(t, BP_GEMV, That, xh, yh, n, nrhs, P, s);
}

}  // namespace emsurf
