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

}  // namespace

void launch_block_product(Cx t, const void* That, const void* xh, void* yh, int n, int nrhs, int64_t P,
                          hipStream_t s) {
  EMS_CHECK_ARG(n >= 1 && n <= 512, "block product supports 1 <= n_eq <= 512");
  EMS_CHECK_ARG(nrhs >= 1 && nrhs <= 64, "block product supports 1 <= nrhs <= 64");
  EMS_CHECK_ARG(P >= 1 && P <= 0x7fffffffLL, "frequency count out of range");
  if (t == Cx::C128)
    launch_t<double2>(That, xh, yh, n, nrhs, P, s);
  else
    launch_t<float2>(That, xh, yh, n, nrhs, P, s);
  EMS_LAUNCH_CHECK();
}

}  // namespace emsurf
