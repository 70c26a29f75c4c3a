// Fourier-domain products of the structured outer operator (eq. (blockZo);
// Sec. IV-B: the discretised L and K operators, scaled by constants, multiply
// blocks of x; Sec. IV-C: only L and K are stored).  Per frequency k the store
// holds the stacked n x n_h matrix [L^(k); K^(k)] column-major ([k][v][L|K][u],
// n = 2 n_h), and
//     yJ = a L xJ + b K xM,      yM = c K xJ + e L xM,
// with xJ / xM the J and M halves of the frequency's spectral column.  This is
// the lane-per-row streaming product of the dense path on a rectangular
// block with twice the right-hand sides ([L; K] [xJ xM]), followed by the
// combination with the four constants, so every stored entry serves two
// products per right-hand side and the store is half the size of dense blocks.
//
// One workgroup per frequency, lane u < n owns row u of [L; K]; columns
// stream through a buffer resource, U in flight while the previous U are
// multiplied; LDS holds the operands xs[v][2 NR] (xJ of every right-hand side,
// then xM) and afterwards the partial products for the combination, whose
// results leave with non-temporal 16-byte stores.
#include "internal.h"

namespace emsurf {
namespace {

template <typename V> struct RealOf;
template <> struct RealOf<float2> { using T = float; };
template <> struct RealOf<double2> { using T = double; };

__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

// one complex entry through the frequency's buffer resource (non-temporal);
// callers keep every offset inside the record
template <typename V> __device__ __forceinline__ V ld_lk(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff);
template <> __device__ __forceinline__ float2 ld_lk<float2>(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff) {
  auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 2);
  float2 f;
  __builtin_memcpy(&f, &v, sizeof(f));
  return f;
}
template <> __device__ __forceinline__ double2 ld_lk<double2>(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff) {
  auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 2);
  double2 d;
  __builtin_memcpy(&d, &v, sizeof(d));
  return d;
}

// complex y += a * x as four real FMAs
template <typename V, typename T>
__device__ __forceinline__ void cmac(T& yr, T& yi, const V a, const V x) {
  yr = fmar(a.x, x.x, yr);
  yr = fmar(-a.y, x.y, yr);
  yi = fmar(a.x, x.y, yi);
  yi = fmar(a.y, x.x, yi);
}

// U columns c0 .. c0+U-1 of the stacked block (indices clamped to the block
// with a uniform min: a stage past the end re-reads column n_h - 1)
template <typename V, int U>
__device__ __forceinline__ void lk_fetch(V (&a)[U], __amdgpu_buffer_rsrc_t rs, unsigned voff, int c0, int nh,
                                         int col_bytes) {
#pragma unroll
  for (int j = 0; j < U; ++j) {
    const int c = c0 + j < nh ? c0 + j : nh - 1;
    a[j] = ld_lk<V>(rs, voff, c * col_bytes);
  }
}

template <typename V, int Q, int U, typename T>
__device__ __forceinline__ void lk_stage(const V (&a)[U], const V* __restrict__ xs, T (&pr)[Q], T (&pi)[Q]) {
#pragma unroll
  for (int j = 0; j < U; ++j) {
#pragma unroll
    for (int q = 0; q < Q; ++q) cmac(pr[q], pi[q], a[j], xs[j * Q + q]);
  }
}

struct Coef4 {
  double2 a, b, c, e;
};

// constant times a complex value, in the value's precision
template <typename V>
__device__ __forceinline__ V cmul(const double2 s, const V x) {
  using T = typename RealOf<V>::T;
  const T sr = (T)s.x, si = (T)s.y;
  return V{sr * x.x - si * x.y, sr * x.y + si * x.x};
}
template <typename V> __device__ __forceinline__ V cadd(const V a, const V b) { return V{a.x + b.x, a.y + b.y}; }

// outputs e in [0, cnt) of a contiguous run computed by f(e), written with
// non-temporal 16-byte stores (FP32 pairs: the run starts on an even element
// and cnt is even because n_eq is even)
template <typename F>
__device__ __forceinline__ void store_pairs(float2* __restrict__ dst, int cnt, F&& f) {
  for (int i = threadIdx.x; i < cnt / 2; i += blockDim.x) {
    const float2 p0 = f(2 * i), p1 = f(2 * i + 1);
    const fvec4 v = {p0.x, p0.y, p1.x, p1.y};
    __builtin_nontemporal_store(v, reinterpret_cast<fvec4*>(dst + 2 * i));
  }
}
template <typename F>
__device__ __forceinline__ void store_pairs(double2* __restrict__ dst, int cnt, F&& f) {
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const double2 p = f(i);
    const dvec2 v = {p.x, p.y};
    __builtin_nontemporal_store(v, reinterpret_cast<dvec2*>(dst + i));
  }
}

// NR right-hand sides per pass (nr <= NR valid).  LDS: operands xs[npad][2 NR]
// (rows v >= n_h zero), then the partial products P[2 NR][n].
template <typename V, int NR, int U>
__global__ void __launch_bounds__(512) block_lk_kernel(const V* __restrict__ That, const V* __restrict__ xh,
                                                       V* __restrict__ yh, int nh, int nrhs, int r0, int nr,
                                                       Coef4 cf) {
  using T = typename RealOf<V>::T;
  constexpr int Q = 2 * NR;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* xs = reinterpret_cast<V*>(smem_raw);
  const long long k = blockIdx.x;
  const int n = 2 * nh;
  const int npad = (nh + U - 1) / U * U;
  const int u = threadIdx.x;
  const long long rec = (long long)n * nh;   // entries per frequency
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(That + k * rec), (short)0, (int)(rec * (long long)sizeof(V)), 0x00020000);
  // lanes past the last row stream row n - 1 and store nothing
  const unsigned voff = (unsigned)((u < n ? u : n - 1) * (int)sizeof(V));
  const int col_bytes = n * (int)sizeof(V);
  // the first columns are requested before the operands are staged
  V A0[U], A1[U];
  lk_fetch<V, U>(A0, rs, voff, 0, nh, col_bytes);
  const V* xk = xh + k * (long long)nrhs * n + (long long)r0 * n;
  for (int i = threadIdx.x; i < Q * npad; i += blockDim.x) {
    const int q = i / npad, v = i - q * npad;
    const int r = q < NR ? q : q - NR;
    V val{0, 0};
    if (r < nr && v < nh) val = xk[(long long)r * n + (q < NR ? 0 : nh) + v];
    xs[v * Q + q] = val;
  }
  __syncthreads();
  T pr[Q], pi[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) { pr[q] = 0; pi[q] = 0; }
  // two register stages used alternately
  for (int v0 = 0; v0 < npad; v0 += 2 * U) {
    lk_fetch<V, U>(A1, rs, voff, v0 + U, nh, col_bytes);
    __builtin_amdgcn_sched_barrier(0);
    lk_stage<V, Q, U>(A0, xs + v0 * Q, pr, pi);
    lk_fetch<V, U>(A0, rs, voff, v0 + 2 * U, nh, col_bytes);
    __builtin_amdgcn_sched_barrier(0);
    if (v0 + U < npad) lk_stage<V, Q, U>(A1, xs + (v0 + U) * Q, pr, pi);
  }
  // partial products: row u < n_h holds (L xJ, L xM), row n_h + u (K xJ, K xM)
  __syncthreads();
  if (u < n) {
#pragma unroll
    for (int q = 0; q < Q; ++q) xs[q * n + u] = V{pr[q], pi[q]};
  }
  __syncthreads();
  // yJ[u] = a (L xJ)[u] + b (K xM)[u],  yM[u] = c (K xJ)[u] + e (L xM)[u]
  V* yk = yh + k * (long long)nrhs * n + (long long)r0 * n;
  auto out = [&](int e) -> V {
    const int r = e / n, w = e - r * n;
    if (w < nh) return cadd(cmul(cf.a, xs[r * n + w]), cmul(cf.b, xs[(NR + r) * n + nh + w]));
    const int uu = w - nh;
    return cadd(cmul(cf.c, xs[r * n + nh + uu]), cmul(cf.e, xs[(NR + r) * n + uu]));
  };
  store_pairs(yk, nr * n, out);
}

// columns per pipeline stage, as for the dense product with 2 NR right-hand sides
template <typename V, int NR> constexpr int lk_stage_cols() {
  return sizeof(V) == 8 ? (NR <= 4 ? 8 : 4) : (NR <= 2 ? 4 : 2);
}

template <typename V, int NR>
void launch_lk_nr(const void* That, const void* xh, void* yh, int nh, int nrhs, int r0, int nr, int64_t P,
                  const Coef4& cf, hipStream_t s) {
  constexpr int U = lk_stage_cols<V, NR>();
  const int n = 2 * nh;
  const int threads = ((n + 63) / 64) * 64;
  const int npad = (nh + U - 1) / U * U;
  size_t shm = (size_t)npad * 2 * NR * sizeof(V);
  const size_t part = (size_t)2 * NR * n * sizeof(V);
  if (part > shm) shm = part;
  hipLaunchKernelGGL((block_lk_kernel<V, NR, U>), dim3((unsigned)P), dim3(threads), shm, s,
                     static_cast<const V*>(That), static_cast<const V*>(xh), static_cast<V*>(yh), nh, nrhs, r0, nr,
                     cf);
}

template <typename V>
void launch_lk_t(const void* That, const void* xh, void* yh, int nh, int nrhs, int64_t P, const Coef4& cf,
                 hipStream_t s) {
  // right-hand sides per pass: 64 KB of LDS for the partial products
  // (2 NR x n_eq, the larger of the two uses) and the accumulator registers
  // (2 complex per right-hand side per lane)
  int cap = (int)(65536 / ((size_t)4 * (nh + 7) * sizeof(V)));
  const int reg_cap = sizeof(V) == 16 ? 8 : 16;
  if (cap > reg_cap) cap = reg_cap;
  EMS_CHECK_ARG(cap >= 1, "structured block product: n_eq too large for the LDS staging");
  int NR = 1;
  while (NR < nrhs && NR * 2 <= cap) NR *= 2;
  for (int r0 = 0; r0 < nrhs; r0 += NR) {
    const int nr = nrhs - r0 < NR ? nrhs - r0 : NR;
    switch (NR) {
      case 1: launch_lk_nr<V, 1>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s); break;
      case 2: launch_lk_nr<V, 2>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s); break;
      case 4: launch_lk_nr<V, 4>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s); break;
      case 8: launch_lk_nr<V, 8>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s); break;
      default: launch_lk_nr<V, 16>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s); break;
    }
  }
}

}  // namespace

void launch_block_product_lk(Cx t, int variant, const void* That, const void* xh, void* yh, int nh, int nrhs,
                             int64_t P, const double* coef, hipStream_t s) {
  EMS_CHECK_ARG(nh >= 1 && nh <= 256, "structured block product supports 1 <= n_eq / 2 <= 256");
  EMS_CHECK_ARG(nrhs >= 1 && nrhs <= 64, "block product supports 1 <= nrhs <= 64");
  EMS_CHECK_ARG(P >= 1 && P <= 0x7fffffffLL, "frequency count out of range");
  const Coef4 cf{{coef[0], coef[1]}, {coef[2], coef[3]}, {coef[4], coef[5]}, {coef[6], coef[7]}};
  if (t == Cx::C128)
    launch_lk_t<double2>(That, xh, yh, nh, nrhs, P, cf, s);
  else if (variant != BP_GEMV && block_variant_supported_lk(variant, 2 * nh, nrhs))
    launch_block_mfma_lk(variant, That, xh, yh, nh, nrhs, P, coef, s);
  else
    launch_lk_t<float2>(That, xh, yh, nh, nrhs, P, cf, s);
  EMS_LAUNCH_CHECK();
}

}  // namespace emsurf
