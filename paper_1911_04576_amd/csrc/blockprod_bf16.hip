// Fourier-domain block products in split BF16 on the matrix cores: the
// per-frequency product of Sec. IV-B,
//     yh[k][r][u] = sum_v That[k](u, v) xh[k][r][v],
// with both operands split into two bfloat16 halves, a = a_hi + a_lo
// (a_hi = bf16(a), a_lo = bf16(a - a_hi), each rounded to nearest even), and
//     a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi
// accumulated in FP32 (three products; the dropped a_lo b_lo is below
// 2^-16 |a b|).  The one-product form keeps a_hi b_hi only and reads the hi
// plane alone.  The spectral input stays FP32 (the FFTs are FP32); its split
// is formed in registers as the operands are built.
//
// Operand flow (v_mfma_f32_32x32x16_bf16 on the real embedding of the
// complex product, as the FP32 kernel in blockprod_mfma.hip):
//   D[u][(r, re)] = sum_v Ar xr - Ai xi,   D[u][(r, im)] = sum_v Ar xi + Ai xr,
// K index (v, part).  A lane of a 32-row tile holds 8 consecutive K values,
// i.e. both parts of four consecutive source columns of one row; the store
// keeps exactly those 16 bytes together: per frequency a hi plane then a lo
// plane, each with entry (u, v) part p at bf16 index ((v / 4) n + u) 8 +
// (v % 4) 2 + p.  A wave's load for one row tile and one K step (8 source
// columns) is then two contiguous 512-byte runs.  Each wave owns TPW row
// tiles and 16 right-hand sides; the spectral columns of all n_eq sources sit
// in LDS; outputs are staged through LDS for coalesced stores as in the FP32
// kernel.
#include "internal.h"

namespace emsurf {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// 16-byte non-temporal buffer load; callers keep every offset inside the buffer
__device__ __forceinline__ bf16x8 ld_b16x8(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff) {
  auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 2);
  bf16x8 r;
  __builtin_memcpy(&r, &v, sizeof(r));
  return r;
}

template <int TPW, int U, bool LO>
__global__ void __launch_bounds__(256) block_bf16_kernel(const unsigned char* __restrict__ Tb,
                                                         const float2* __restrict__ xh, float2* __restrict__ yh,
                                                         int n, int nrhs, int r0, int nr) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2* xs = reinterpret_cast<float2*>(smem_raw);   // [16][n + 2], later [8][n + 1]
  constexpr int NR = 16;
  const int ld = n + 2;           // even, so a lane's four columns start on 16 bytes
  const int ldo = n + 1;
  const long long k = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
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
  // one plane is n^2 complex entries x 2 parts x 2 bytes; the resource covers
  // the planes this form reads
  const int plane = 4 * n * n;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(Tb + k * 2LL * plane), (short)0, LO ? 2 * plane : plane, 0x00020000);
  unsigned aoff[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) aoff[i] = (unsigned)((h * n + (tv[i] ? tile[i] * 32 : 0) + jl) * 16);
  const int step_bytes = 2 * n * 16;   // one K step: source columns 8g .. 8g + 7
  const int nsteps = n / 8;
  bf16x8 ahi[U][TPW], alo[U][TPW], nhi[U][TPW], nlo[U][TPW];
#pragma unroll
  for (int st = 0; st < U; ++st)
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      ahi[st][i] = ld_b16x8(rs, aoff[i], st * step_bytes);
      if (LO) alo[st][i] = ld_b16x8(rs, aoff[i], plane + st * step_bytes);
    }
  const float2* xk = xh + k * (long long)nrhs * n + (long long)r0 * n;
  for (int i = threadIdx.x; i < NR * n; i += blockDim.x) {
    const int r = i / n, v = i - r * n;
    xs[r * ld + v] = (r < nr) ? xk[(long long)r * n + v] : float2{0.f, 0.f};
  }
  __syncthreads();
  for (int g0 = 0; g0 < nsteps; g0 += U) {
    // prefetch the next U steps; past the end the step index is clamped to the
    // last one (a uniform min), so every load stays inside the block
#pragma unroll
    for (int st = 0; st < U; ++st) {
      const int g = g0 + U + st < nsteps - 1 ? g0 + U + st : nsteps - 1;
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        nhi[st][i] = ld_b16x8(rs, aoff[i], g * step_bytes);
        if (LO) nlo[st][i] = ld_b16x8(rs, aoff[i], plane + g * step_bytes);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int st = 0; st < U; ++st) {
      // B operand: K values 8h .. 8h + 7 of step g = parts of source columns
      // 8g + 4h .. 8g + 4h + 3 for column (rsel, re/im) of the embedding
      const fvec4* xp = reinterpret_cast<const fvec4*>(xs + rsel * ld + 8 * (g0 + st) + 4 * h);
      const fvec4 x01 = xp[0], x23 = xp[1];
      const float xv[8] = {x01[0], x01[1], x01[2], x01[3], x23[0], x23[1], x23[2], x23[3]};
      bf16x8 bhi, blo;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float re = xv[2 * c], im = xv[2 * c + 1];
        const float b0 = dimag ? im : re;
        const float b1 = dimag ? re : -im;
        bhi[2 * c] = (__bf16)b0;
        bhi[2 * c + 1] = (__bf16)b1;
        if (LO) {
          blo[2 * c] = (__bf16)(b0 - (float)bhi[2 * c]);
          blo[2 * c + 1] = (__bf16)(b1 - (float)bhi[2 * c + 1]);
        }
      }
#pragma unroll
      for (int i = 0; i < TPW; ++i) acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[st][i], bhi, acc[i], 0, 0, 0);
      if (LO) {
#pragma unroll
        for (int i = 0; i < TPW; ++i)
          acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[st][i], blo, acc[i], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < TPW; ++i)
          acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[st][i], bhi, acc[i], 0, 0, 0);
      }
    }
#pragma unroll
    for (int st = 0; st < U; ++st)
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        ahi[st][i] = nhi[st][i];
        if (LO) alo[st][i] = nlo[st][i];
      }
  }
  // outputs in two halves of eight right-hand sides, staged [r][u] in LDS,
  // then 16-byte non-temporal stores of element pairs (n_eq is even)
  float* ysf = reinterpret_cast<float*>(xs);
  float2* yk = yh + k * (long long)nrhs * n + (long long)r0 * n;
  for (int half = 0; half < 2; ++half) {
    const int rlo = 8 * half;
    const int cnt = nr - rlo < 8 ? nr - rlo : 8;
    if (cnt <= 0) break;
    __syncthreads();
    if ((rsel >> 3) == half) {
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        if (!tv[i]) continue;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int u = tile[i] * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
          ysf[2 * ((rsel - rlo) * ldo + u) + (dimag ? 1 : 0)] = acc[i][e];
        }
      }
    }
    __syncthreads();
    float2* yo = yk + (long long)rlo * n;
    for (int i = threadIdx.x; i < cnt * n / 2; i += blockDim.x) {
      const int e = 2 * i;
      const int r = e / n, u = e - r * n;
      const float2 p0 = xs[r * ldo + u], p1 = xs[r * ldo + u + 1];
      const fvec4 v = {p0.x, p0.y, p1.x, p1.y};
      __builtin_nontemporal_store(v, reinterpret_cast<fvec4*>(yo + e));
    }
  }
}

inline int bf16_waves(int n, int tpw) { return (n / 32 + tpw - 1) / tpw; }

template <int TPW, int U, bool LO>
void launch_bf16(const void* Tb, const void* xh, void* yh, int n, int nrhs, int r0, int nr, int64_t P,
                 hipStream_t s) {
  const int waves = bf16_waves(n, TPW);
  const size_t shm = (size_t)16 * (n + 2) * sizeof(float2);
  hipLaunchKernelGGL((block_bf16_kernel<TPW, U, LO>), dim3((unsigned)P), dim3(64 * waves), shm, s,
                     static_cast<const unsigned char*>(Tb), static_cast<const float2*>(xh), static_cast<float2*>(yh),
                     n, nrhs, r0, nr);
}

template <bool LO>
void launch_bf16_form(const void* Tb, const void* xh, void* yh, int n, int nrhs, int r0, int nr, int64_t P,
                      hipStream_t s) {
  // fewest row tiles per wave that keep a frequency within 4 wavefronts
  const int ntile = n / 32;
  if (ntile <= 4) launch_bf16<1, 2, LO>(Tb, xh, yh, n, nrhs, r0, nr, P, s);
  else if (ntile <= 8) launch_bf16<2, 2, LO>(Tb, xh, yh, n, nrhs, r0, nr, P, s);
  else if (ntile <= 12) launch_bf16<3, 2, LO>(Tb, xh, yh, n, nrhs, r0, nr, P, s);
  else launch_bf16<4, 2, LO>(Tb, xh, yh, n, nrhs, r0, nr, P, s);
}

}  // namespace

bool block_bf16_supported(int n) { return n % 32 == 0 && n >= 32 && n <= 480; }

void launch_block_bf16(int split, const void* Tb, const void* xh, void* yh, int n, int nrhs, int64_t P,
                       hipStream_t s) {
  EMS_CHECK_ARG(split == 1 || split == 3, "split-BF16 product needs one or three products");
  EMS_CHECK_ARG(block_bf16_supported(n), "split-BF16 product needs n_eq a multiple of 32 in [32, 480]");
  EMS_CHECK_ARG(nrhs >= 1, "nrhs must be >= 1");
  for (int r0 = 0; r0 < nrhs; r0 += 16) {
    const int nr = nrhs - r0 < 16 ? nrhs - r0 : 16;
    if (split == 3) launch_bf16_form<true>(Tb, xh, yh, n, nrhs, r0, nr, P, s);
    else launch_bf16_form<false>(Tb, xh, yh, n, nrhs, r0, nr, P, s);
  }
  EMS_LAUNCH_CHECK();
}

}  // namespace emsurf
