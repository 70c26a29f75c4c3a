// Fourier-domain block products on the matrix cores (Sec. IV-B): the
// many-right-hand-side form of the per-frequency product
//     yh[k][r][u] = sum_v That[k](u, v) xh[k][r][v]
// in FP32.  The few-right-hand-side GEMV form and the dispatch between the two
// live in blockprod.hip.
#include "internal.h"

namespace emsurf {
namespace {

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
typedef float fvec4 __attribute__((ext_vector_type(4)));

// 8-byte non-temporal buffer load; callers keep every offset inside the buffer
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
  float2* xs = reinterpret_cast<float2*>(smem_raw);     // [16][n/2 + 1], then [8][n + 1]
  constexpr int NR = 16;
  const int hn = n / 2;
  const int ld = hn + 1;          // spectral columns: one half of the source index at a time
  const int ldo = n + 1;          // outputs: eight right-hand sides at a time
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
  // spectral columns of source indices [base, base + n/2) into LDS
  auto stage = [&](int base) {
    for (int i = threadIdx.x; i < NR * hn; i += blockDim.x) {
      const int r = i / hn, v = i - r * hn;
      xs[r * ld + v] = (r < nr) ? xk[(long long)r * n + base + v] : float2{0.f, 0.f};
    }
  };
  const int last_step = n / 2 - 1;
  // column pairs of source indices [vstart, vend), spectral columns in LDS
  // starting at source index vbase
  auto sweep = [&](int vstart, int vend, int vbase) {
    for (int v0 = vstart; v0 < vend; v0 += 2 * U) {
      // the final prefetch would run past the block: its step index is clamped
      // to the last column pair (a uniform min), so every load stays inside the
      // block whatever the hardware range check covers; those values are unused
#pragma unroll
      for (int st = 0; st < U; ++st) {
        const int step = v0 / 2 + U + st < last_step ? v0 / 2 + U + st : last_step;
#pragma unroll
        for (int i = 0; i < TPW; ++i) anxt[st][i] = ld_buf(rs, aoff[i], step * step_bytes);
      }
      // keep the prefetch ahead of this step's MFMAs
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int st = 0; st < U; ++st) {
        const float2 xv = xs[rsel * ld + (v0 - vbase) + 2 * st + h];
        const float bre = dimag ? xv.y : xv.x;
        const float bim = dimag ? xv.x : -xv.y;
#pragma unroll
        for (int i = 0; i < TPW; ++i)
          acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(acur[st][i].x, bre, acc[i], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < TPW; ++i)
          acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(acur[st][i].y, bim, acc[i], 0, 0, 0);
      }
#pragma unroll
      for (int st = 0; st < U; ++st)
#pragma unroll
        for (int i = 0; i < TPW; ++i) acur[st][i] = anxt[st][i];
    }
  };
  // first half of the source index, then the second (n/2 is a multiple of
  // 2U, so each half is a whole number of loop steps)
  stage(0);
  __syncthreads();
  sweep(0, hn, 0);
  __syncthreads();
  stage(hn);
  __syncthreads();
  sweep(hn, n, hn);
  // outputs in two halves of eight right-hand sides: stage [r][u] complex in
  // LDS, then non-temporal 16-byte stores of element pairs (the run of a
  // right-hand side starts on an even element because n_eq is even)
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

// row-tile groups (= wavefronts) for TPW tiles per wave
inline int mfma_waves(int n, int tpw) { return (n / 32 + tpw - 1) / tpw; }

template <int TPW, int U>
void launch_mfma(const void* That, const void* xh, void* yh, int n, int nrhs, int r0, int nr, int64_t P,
                 hipStream_t s) {
  const int waves = mfma_waves(n, TPW);
  EMS_CHECK_ARG(waves >= 1 && waves <= 4, "MFMA variant needs at most 4 wavefronts per frequency");
  EMS_CHECK_ARG((n / 2) % (2 * U) == 0, "MFMA variant needs n_eq / 2 divisible by twice its prefetch depth");
  const size_t a = (size_t)16 * (n / 2 + 1) * sizeof(float2), b = (size_t)8 * (n + 1) * sizeof(float2);
  const size_t shm = a > b ? a : b;
  EMS_CHECK_ARG(shm <= 65536, "MFMA variant needs n_eq <= 480");
  hipLaunchKernelGGL((block_mfma_kernel<TPW, U>), dim3((unsigned)P), dim3(64 * waves), shm, s,
                     static_cast<const float2*>(That), static_cast<const float2*>(xh), static_cast<float2*>(yh), n,
                     nrhs, r0, nr);
}

// ----------------------------------------------------------------------------- structured form
// The structured outer operator (eq. (blockZo); the store holds per frequency
// the stacked n x n_h matrix [L; K] column-major, n = 2 n_h) on the matrix
// cores: the same operand flow as above with two B blocks per step, xJ and xM
// of 16 right-hand sides, so that every streamed tile of [L; K] serves both:
// P_J = [L; K] xJ and P_M = [L; K] xM in two accumulator sets.  The epilogue
// forms yJ = a L xJ + b K xM and yM = c K xJ + e L xM: P_J goes to LDS, each
// lane combines it with its own P_M entry (its re/im partner comes from the
// neighbouring lane), and the results are staged for the coalesced stores.
struct CoefLK {
  float ar, ai, br, bi, cr, ci, er, ei;
};

template <int TPW, int U>
__global__ void __launch_bounds__(256) block_mfma_lk_kernel(const float2* __restrict__ That,
                                                            const float2* __restrict__ xh, float2* __restrict__ yh,
                                                            int nh, int nrhs, int r0, int nr, CoefLK cf) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2* xs = reinterpret_cast<float2*>(smem_raw);     // operands [2][16][nh + 1], later [16][n + 1]
  constexpr int NR = 16;
  const int n = 2 * nh;
  const int ldx = nh + 1, ldo = n + 1;
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
  floatx16 accJ[TPW], accM[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) { accJ[i][e] = 0.f; accM[i][e] = 0.f; }
  const long long rec = (long long)n * nh;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(That + k * rec), (short)0, (int)(rec * (long long)sizeof(float2)), 0x00020000);
  unsigned aoff[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) aoff[i] = (unsigned)((h * n + (tv[i] ? tile[i] * 32 : 0) + jl) * sizeof(float2));
  const int step_bytes = 2 * n * (int)sizeof(float2);   // two columns of [L; K]
  float2 acur[U][TPW], anxt[U][TPW];
#pragma unroll
  for (int st = 0; st < U; ++st)
#pragma unroll
    for (int i = 0; i < TPW; ++i) acur[st][i] = ld_buf(rs, aoff[i], st * step_bytes);
  const float2* xk = xh + k * (long long)nrhs * n + (long long)r0 * n;
  for (int i = threadIdx.x; i < 2 * NR * nh; i += blockDim.x) {
    const int qr = i / nh, v = i - qr * nh;
    const int q = qr / NR, r = qr - q * NR;
    xs[qr * ldx + v] = (r < nr) ? xk[(long long)r * n + q * nh + v] : float2{0.f, 0.f};
  }
  __syncthreads();
  const int last_step = nh / 2 - 1;
  for (int v0 = 0; v0 < nh; v0 += 2 * U) {
    // clamped prefetch of the next U column pairs (values past the block unused)
#pragma unroll
    for (int st = 0; st < U; ++st) {
      const int step = v0 / 2 + U + st < last_step ? v0 / 2 + U + st : last_step;
#pragma unroll
      for (int i = 0; i < TPW; ++i) anxt[st][i] = ld_buf(rs, aoff[i], step * step_bytes);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int st = 0; st < U; ++st) {
      const int v = v0 + 2 * st + h;
      const float2 xj = xs[rsel * ldx + v];
      const float2 xm = xs[(NR + rsel) * ldx + v];
      const float bjre = dimag ? xj.y : xj.x, bjim = dimag ? xj.x : -xj.y;
      const float bmre = dimag ? xm.y : xm.x, bmim = dimag ? xm.x : -xm.y;
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        accJ[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(acur[st][i].x, bjre, accJ[i], 0, 0, 0);
        accM[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(acur[st][i].x, bmre, accM[i], 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        accJ[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(acur[st][i].y, bjim, accJ[i], 0, 0, 0);
        accM[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(acur[st][i].y, bmim, accM[i], 0, 0, 0);
      }
    }
#pragma unroll
    for (int st = 0; st < U; ++st)
#pragma unroll
      for (int i = 0; i < TPW; ++i) acur[st][i] = anxt[st][i];
  }
  // P_J to LDS as [r][w] complex (w = row of [L; K])
  __syncthreads();
  float* ysf = reinterpret_cast<float*>(xs);
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    if (!tv[i]) continue;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int w = tile[i] * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
      ysf[2 * (rsel * ldo + w) + (dimag ? 1 : 0)] = accJ[i][e];
    }
  }
  __syncthreads();
  // this lane's component of: yJ[w - n_h] = a P_J[w - n_h] + b P_M[w]   (w >= n_h, K rows)
  //                           yM[w]       = c P_J[n_h + w] + e P_M[w]   (w <  n_h, L rows)
  float outv[TPW][16];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const float own = accM[i][e];
      const float other = __shfl_xor(own, 1);
      const float pmr = dimag ? other : own, pmi = dimag ? own : other;
      const int w = (tv[i] ? tile[i] * 32 : 0) + 8 * (e >> 2) + 4 * h + (e & 3);
      const bool krow = w >= nh;
      const int wj = krow ? w - nh : nh + w;
      const float pjr = ysf[2 * (rsel * ldo + wj)], pji = ysf[2 * (rsel * ldo + wj) + 1];
      const float c1r = krow ? cf.ar : cf.cr, c1i = krow ? cf.ai : cf.ci;
      const float c2r = krow ? cf.br : cf.er, c2i = krow ? cf.bi : cf.ei;
      outv[i][e] = dimag ? (c1r * pji + c1i * pjr + c2r * pmi + c2i * pmr)
                         : (c1r * pjr - c1i * pji + c2r * pmr - c2i * pmi);
    }
  }
  __syncthreads();
  // stage [r][position] with position w - n_h (yJ) or n_h + w (yM)
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    if (!tv[i]) continue;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int w = tile[i] * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
      const int pos = w >= nh ? w - nh : nh + w;
      ysf[2 * (rsel * ldo + pos) + (dimag ? 1 : 0)] = outv[i][e];
    }
  }
  __syncthreads();
  float2* yk = yh + k * (long long)nrhs * n + (long long)r0 * n;
  for (int i = threadIdx.x; i < nr * n / 2; i += blockDim.x) {
    const int e = 2 * i;
    const int r = e / n, u = e - r * n;
    const float2 p0 = xs[r * ldo + u], p1 = xs[r * ldo + u + 1];
    const fvec4 v = {p0.x, p0.y, p1.x, p1.y};
    __builtin_nontemporal_store(v, reinterpret_cast<fvec4*>(yk + e));
  }
}

size_t lk_mfma_lds(int nh) {
  const size_t a = (size_t)2 * 16 * (nh + 1) * sizeof(float2);
  const size_t b = (size_t)16 * (2 * nh + 1) * sizeof(float2);
  return a > b ? a : b;
}

template <int TPW, int U>
void launch_mfma_lk(const void* That, const void* xh, void* yh, int nh, int nrhs, int r0, int nr, int64_t P,
                    const CoefLK& cf, hipStream_t s) {
  const int n = 2 * nh;
  const int waves = mfma_waves(n, TPW);
  EMS_CHECK_ARG(waves >= 1 && waves <= 4, "MFMA variant needs at most 4 wavefronts per frequency");
  EMS_CHECK_ARG((nh / 2) % U == 0, "MFMA variant needs n_h / 2 divisible by its prefetch depth");
  const size_t shm = lk_mfma_lds(nh);
  EMS_CHECK_ARG(shm <= 65536, "structured MFMA variant needs n_eq <= 480");
  hipLaunchKernelGGL((block_mfma_lk_kernel<TPW, U>), dim3((unsigned)P), dim3(64 * waves), shm, s,
                     static_cast<const float2*>(That), static_cast<const float2*>(xh), static_cast<float2*>(yh), nh,
                     nrhs, r0, nr, cf);
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

void launch_block_mfma(int variant, const void* That, const void* xh, void* yh, int n, int nrhs, int64_t P,
                       hipStream_t s) {
  EMS_CHECK_ARG(block_variant_supported(variant, n, nrhs) && variant != BP_GEMV, "unsupported MFMA variant");
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


bool block_variant_supported_lk(int variant, int n, int nrhs) {
  if (variant == BP_GEMV) return true;
  if (variant < BP_MFMA_T1 || variant >= BP_NVARIANTS || !block_mfma_supported(n, nrhs)) return false;
  return mfma_waves(n, variant_tiles(variant)) <= 4 && lk_mfma_lds(n / 2) <= 65536;
}

void launch_block_mfma_lk(int variant, const void* That, const void* xh, void* yh, int nh, int nrhs, int64_t P,
                          const double* coef, hipStream_t s) {
  const int n = 2 * nh;
  EMS_CHECK_ARG(block_variant_supported_lk(variant, n, nrhs) && variant != BP_GEMV, "unsupported MFMA variant");
  const CoefLK cf{(float)coef[0], (float)coef[1], (float)coef[2], (float)coef[3],
                  (float)coef[4], (float)coef[5], (float)coef[6], (float)coef[7]};
  // deep prefetch: 6 column pairs when n_h / 2 is a multiple of 6, else 8
  const bool six = (nh / 2) % 6 == 0;
  for (int r0 = 0; r0 < nrhs; r0 += 16) {
    const int nr = nrhs - r0 < 16 ? nrhs - r0 : 16;
    switch (variant) {
      case BP_MFMA_T1: launch_mfma_lk<1, 4>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s); break;
      case BP_MFMA_T2: launch_mfma_lk<2, 4>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s); break;
      case BP_MFMA_T3: launch_mfma_lk<3, 4>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s); break;
      case BP_MFMA_T4: launch_mfma_lk<4, 4>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s); break;
      case BP_MFMA_T1D:
        if (six) launch_mfma_lk<1, 6>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s);
        else launch_mfma_lk<1, 8>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s);
        break;
      case BP_MFMA_T2D:
        if (six) launch_mfma_lk<2, 6>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s);
        else launch_mfma_lk<2, 8>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s);
        break;
      case BP_MFMA_T3D:
        if (six) launch_mfma_lk<3, 6>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s);
        else launch_mfma_lk<3, 8>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s);
        break;
      default:
        if (six) launch_mfma_lk<4, 6>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s);
        else launch_mfma_lk<4, 8>(That, xh, yh, nh, nrhs, r0, nr, P, cf, s);
        break;
    }
  }
}
}  // namespace emsurf
