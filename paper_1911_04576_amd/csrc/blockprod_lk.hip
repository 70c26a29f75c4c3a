// Fourier-domain products of the structured outer operator (eq. (blockZo);
// Sec. IV-B: the discretised L and K operators, scaled by constants, multiply
// blocks of x; Sec. IV-C: only L and K are stored).  Per frequency k the store
// holds L^(k) and K^(k), n_h x n_h each, column-major ([k][L, K][v][u]), and
//     yJ = a L xJ + b K xM,      yM = c K xJ + e L xM,
// with xJ / xM the J and M halves (n_h each) of the frequency's spectral
// column.  Every stored entry is used twice per right-hand side, so the
// product reads half the bytes of a dense n_eq x n_eq block for the same
// arithmetic.
//
// Layout of the work: one workgroup per frequency; lane u < n_h owns row u of
// L and K and both outputs; L and K columns stream through a buffer resource
// (U columns of each in flight while the previous U are multiplied).  LDS
// holds, per source column v and right-hand side r, the four scaled operands
// (a xJ, b xM, c xJ, e xM) and afterwards stages the output panel for
// non-temporal 16-byte stores.
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

// U columns c0 .. c0+U-1 of L (offset 0) and K (offset n_h^2 entries); column
// indices past the block are clamped with a uniform min (values unused)
template <typename V, int U>
__device__ __forceinline__ void lk_fetch(V (&aL)[U], V (&aK)[U], __amdgpu_buffer_rsrc_t rs, unsigned voff, int c0,
                                         int nh, int col_bytes, int k_bytes) {
#pragma unroll
  for (int j = 0; j < U; ++j) {
    const int c = c0 + j < nh ? c0 + j : nh - 1;
    aL[j] = ld_lk<V>(rs, voff, c * col_bytes);
    aK[j] = ld_lk<V>(rs, voff, k_bytes + c * col_bytes);
  }
}

template <typename V, int NR, int U, typename T>
__device__ __forceinline__ void lk_stage(const V (&aL)[U], const V (&aK)[U], const V* __restrict__ xs,
                                         T (&jr)[NR], T (&ji)[NR], T (&mr)[NR], T (&mi)[NR]) {
#pragma unroll
  for (int j = 0; j < U; ++j) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const V* q = xs + (j * NR + r) * 4;
      cmac(jr[r], ji[r], aL[j], q[0]);   // a L xJ
      cmac(jr[r], ji[r], aK[j], q[1]);   // b K xM
      cmac(mr[r], mi[r], aK[j], q[2]);   // c K xJ
      cmac(mr[r], mi[r], aL[j], q[3]);   // e L xM
    }
  }
}

__device__ __forceinline__ void store_panel(float2* __restrict__ dst, const float2* __restrict__ src, int cnt) {
  if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
    const int pairs = cnt >> 1;
    for (int i = threadIdx.x; i < pairs; i += blockDim.x)
      __builtin_nontemporal_store(reinterpret_cast<const fvec4*>(src)[i], reinterpret_cast<fvec4*>(dst) + i);
    if ((cnt & 1) && threadIdx.x == 0) dst[cnt - 1] = src[cnt - 1];
  } else {
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) dst[i] = src[i];
  }
}
__device__ __forceinline__ void store_panel(double2* __restrict__ dst, const double2* __restrict__ src, int cnt) {
  for (int i = threadIdx.x; i < cnt; i += blockDim.x)
    __builtin_nontemporal_store(reinterpret_cast<const dvec2*>(src)[i], reinterpret_cast<dvec2*>(dst) + i);
}

struct Coef4 {
  double2 a, b, c, e;
};

template <typename V>
__device__ __forceinline__ V cmul(const double2 s, const V x) {
  using T = typename RealOf<V>::T;
  return V{(T)(s.x * (double)x.x - s.y * (double)x.y), (T)(s.x * (double)x.y + s.y * (double)x.x)};
}

// NR right-hand sides per pass (nr <= NR valid); LDS: xs[npad][NR][4], rows
// v >= n_h zero, later the output panel [nr][2 n_h].
template <typename V, int NR, int U>
__global__ void __launch_bounds__(512) block_lk_kernel(const V* __restrict__ That, const V* __restrict__ xh,
                                                       V* __restrict__ yh, int nh, int nrhs, int r0, int nr,
                                                       Coef4 cf) {
  using T = typename RealOf<V>::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* xs = reinterpret_cast<V*>(smem_raw);
  const long long k = blockIdx.x;
  const int n = 2 * nh;
  const int npad = (nh + U - 1) / U * U;
  const int u = threadIdx.x;
  const long long rec = 2LL * nh * nh;   // entries per frequency
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(That + k * rec), (short)0, (int)(rec * (long long)sizeof(V)), 0x00020000);
  const unsigned voff = (unsigned)((u < nh ? u : nh - 1) * (int)sizeof(V));
  const int col_bytes = nh * (int)sizeof(V);
  const int k_bytes = nh * nh * (int)sizeof(V);
  V L0[U], K0[U], L1[U], K1[U];
  lk_fetch<V, U>(L0, K0, rs, voff, 0, nh, col_bytes, k_bytes);
  // scaled operands per (v, r)
  const V* xk = xh + k * (long long)nrhs * n + (long long)r0 * n;
  for (int i = threadIdx.x; i < NR * npad; i += blockDim.x) {
    const int r = i / npad, v = i - r * npad;
    V xJ{0, 0}, xM{0, 0};
    if (r < nr && v < nh) {
      xJ = xk[(long long)r * n + v];
      xM = xk[(long long)r * n + nh + v];
    }
    V* q = xs + (v * NR + r) * 4;
    q[0] = cmul(cf.a, xJ);
    q[1] = cmul(cf.b, xM);
    q[2] = cmul(cf.c, xJ);
    q[3] = cmul(cf.e, xM);
  }
  __syncthreads();
  T jr[NR], ji[NR], mr[NR], mi[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) { jr[r] = 0; ji[r] = 0; mr[r] = 0; mi[r] = 0; }
  for (int v0 = 0; v0 < npad; v0 += 2 * U) {
    lk_fetch<V, U>(L1, K1, rs, voff, v0 + U, nh, col_bytes, k_bytes);
    __builtin_amdgcn_sched_barrier(0);
    lk_stage<V, NR, U>(L0, K0, xs + v0 * NR * 4, jr, ji, mr, mi);
    lk_fetch<V, U>(L0, K0, rs, voff, v0 + 2 * U, nh, col_bytes, k_bytes);
    __builtin_amdgcn_sched_barrier(0);
    if (v0 + U < npad) lk_stage<V, NR, U>(L1, K1, xs + (v0 + U) * NR * 4, jr, ji, mr, mi);
  }
  __syncthreads();
  if (u < nh) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r < nr) {
        xs[r * n + u] = V{jr[r], ji[r]};
        xs[r * n + nh + u] = V{mr[r], mi[r]};
      }
    }
  }
  __syncthreads();
  store_panel(yh + k * (long long)nrhs * n + (long long)r0 * n, xs, nr * n);
}

template <typename V, int NR> constexpr int lk_stage_cols() {
  return sizeof(V) == 8 ? (NR <= 4 ? 4 : 2) : 2;
}

template <typename V, int NR>
void launch_lk_nr(const void* That, const void* xh, void* yh, int nh, int nrhs, int r0, int nr, int64_t P,
                  const Coef4& cf, hipStream_t s) {
  constexpr int U = lk_stage_cols<V, NR>();
  const int threads = ((nh + 63) / 64) * 64;
  const int npad = (nh + U - 1) / U * U;
  size_t shm = (size_t)npad * NR * 4 * sizeof(V);
  const size_t out = (size_t)nr * 2 * nh * sizeof(V);
  if (out > shm) shm = out;
  hipLaunchKernelGGL((block_lk_kernel<V, NR, U>), dim3((unsigned)P), dim3(threads), shm, s,
                     static_cast<const V*>(That), static_cast<const V*>(xh), static_cast<V*>(yh), nh, nrhs, r0, nr,
                     cf);
}

template <typename V>
void launch_lk_t(const void* That, const void* xh, void* yh, int nh, int nrhs, int64_t P, const Coef4& cf,
                 hipStream_t s) {
  // right-hand sides per pass: 64 KB of LDS for the scaled operands and the
  // accumulator registers (4 complex per right-hand side per lane)
  int cap = (int)(65536 / ((size_t)(nh + 3) * 4 * sizeof(V)));
  const int reg_cap = sizeof(V) == 16 ? 4 : 8;
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
      default: launch_lk_nr<V, 8>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s); break;
    }
  }
}

}  // namespace

void launch_block_product_lk(Cx t, const void* That, const void* xh, void* yh, int nh, int nrhs, int64_t P,
                             const double* coef, hipStream_t s) {
  EMS_CHECK_ARG(nh >= 1 && nh <= 256, "structured block product supports 1 <= n_eq / 2 <= 256");
  EMS_CHECK_ARG(nrhs >= 1 && nrhs <= 64, "block product supports 1 <= nrhs <= 64");
  EMS_CHECK_ARG(P >= 1 && P <= 0x7fffffffLL, "frequency count out of range");
  const Coef4 cf{{coef[0], coef[1]}, {coef[2], coef[3]}, {coef[4], coef[5]}, {coef[6], coef[7]}};
  if (t == Cx::C128)
    launch_lk_t<double2>(That, xh, yh, nh, nrhs, P, cf, s);
  else
    launch_lk_t<float2>(That, xh, yh, nh, nrhs, P, cf, s);
  EMS_LAUNCH_CHECK();
}

}  // namespace emsurf
