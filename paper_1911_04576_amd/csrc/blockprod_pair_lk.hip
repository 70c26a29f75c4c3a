// Paired Fourier-domain products of the structured outer operator
// (eq. (blockZo): T(d) = [[a L(d), b K(d)], [c K(d), e L(d)]]) on a reciprocal
// store.  The discretised L and K operators are reciprocal one by one,
//     L(-d) = D^-1 L(d)^T D,   K(-d) = D^-1 K(d)^T D   (D: source weights),
// so one record [L | K] (n_h x 2 n_h) per frequency pair {k, -k} serves
//     yJ[k]  = a L xJ + b K xM,              yM[k]  = c K xJ + e L xM,
//     yJ[-k] = D^-1 (a L^T D xJ + b K^T D xM),  yM[-k] = D^-1 (c K^T D xJ + e L^T D xM),
// with L, K the Fourier-domain blocks at k and x the spectra at k or -k.
//
// Each right-hand side becomes two columns of one product with [L | K]: at k
// the record multiplies (a xJ ; b xM) and (e xM ; c xJ), which gives yJ and
// yM directly; at -k its transpose multiplies D xJ and D xM, and the four
// halves of the two results combine into yJ and yM.  Four right-hand sides
// fill the 16 columns of v_mfma_*_16x16x4 (real and imaginary parts of 8
// virtual columns).  The operand flow follows the dense paired product
// (blockprod_pair.hip), oriented the other way: wavefront w owns column
// tiles w, w + 4, ... and walks every row tile under each, so the transposed
// product's column sums are complete within the wavefront (plain stores) and
// the first product's row sums, kept in registers for all row tiles, are
// added across the four wavefronts once per workgroup.  LDS float atomics
// per column tile (the dense kernel's scheme) cost 1.5 ms here at 128 x 128.
#include "internal.h"

namespace emsurf {
namespace {

constexpr int LNT = 256;   // threads per workgroup
constexpr int LNV = 8;     // virtual columns per pass (4 right-hand sides)

typedef float lk_f4v __attribute__((ext_vector_type(4)));
typedef double lk_d2v __attribute__((ext_vector_type(2)));
typedef double lk_d4v __attribute__((ext_vector_type(4)));

template <typename T> struct LkMf;
template <> struct LkMf<float> {
  using C = lk_f4v;
  using Acc = lk_f4v;
  using V2 = float2;
  static constexpr int CH = 4;
  static constexpr int STAGES = 2;
  // column-sum row stride: rows 4 (l / 16) + e of one store instruction fall
  // 4 rows apart, and a stride of 20 floats puts their 16 columns in 64
  // distinct banks (with 16 they would share 16 banks four ways)
  static constexpr int ZST = 20;
  __device__ static Acc mfma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int l, int e) { return 4 * (l >> 4) + e; }
};
template <> struct LkMf<double> {
  using C = lk_d2v;
  using Acc = lk_d4v;
  using V2 = double2;
  static constexpr int CH = 2;
  static constexpr int STAGES = 1;
  static constexpr int ZST = 16;   // 4 consecutive rows of 16 doubles: two passes of 64 banks
  __device__ static Acc mfma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int e) { return (l >> 4) + 4 * e; }
};

template <typename C>
__device__ __forceinline__ C lk_ld_chunk(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff) {
  return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 2));
}

template <typename T> struct LkCoef {
  T ar, ai, br, bi, cr, ci, er, ei;
};

// T = float or double; NTR = ceil(n_h / 16) row tiles (the row sums of all of
// them stay in registers); nr <= 4 right-hand sides from r0.
template <typename T, int NTR>
__global__ void __launch_bounds__(LNT, 2) pair_lk_kernel(const T* __restrict__ That, const int2* __restrict__ pairs,
                                                         const T* __restrict__ w, const T* __restrict__ winv,
                                                         const typename LkMf<T>::V2* __restrict__ xh,
                                                         typename LkMf<T>::V2* __restrict__ yh, int nh, int nrhs,
                                                         int r0, int nr, LkCoef<T> cf) {
  using M = LkMf<T>;
  using C = typename M::C;
  using Acc = typename M::Acc;
  using V2 = typename M::V2;
  constexpr int CH = M::CH, NCH = 8 / CH, NSTG = M::STAGES, ZST = M::ZST;
  constexpr int TILE_BYTES = 2 * PAIR_TILE * PAIR_TILE * (int)sizeof(T);
  constexpr int NTC = 2 * NTR, NP = NTR * PAIR_TILE, NPC = 2 * NP;
  constexpr int QPW = (NTC + 3) / 4;   // column tiles of wavefront 0
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = 2 * nh;
  // region A: xs, xt and the staging tiles during the walk, the four
  // wavefronts' row sums after it; then the column sums
  T* xs = reinterpret_cast<T*>(smem_raw);   // [NPC][8][2]: (a xJ ; b xM), (e xM ; c xJ) at k
  T* xt = xs + NPC * LNV * 2;               // [NP][8][2]: D xJ, D xM at -k
  T* tiles = xt + NP * LNV * 2;             // [4 waves][stages][512]
  T* part = xs;                             // [4 waves][NP][16] after the walk
  constexpr int AREG = (NPC + NP) * LNV * 2 + 4 * NSTG * 512 > 4 * NP * 2 * LNV
                           ? (NPC + NP) * LNV * 2 + 4 * NSTG * 512 : 4 * NP * 2 * LNV;
  T* zs = xs + AREG;                        // [NPC][ZST]: column sums of the transposed product
  const long long slot = blockIdx.x;
  const int2 pr = pairs[slot];
  const long long k = pr.x, kb = pr.y;
  const bool self = k == kb;
  const int l = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nqw = (NTC - wv + 3) / 4;   // column tiles of this wavefront
  const long long blk = (long long)NTR * NTC * 2 * PAIR_TILE * PAIR_TILE;   // reals
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(That + slot * blk), (short)0, (int)(blk * (long long)sizeof(T)), 0x00020000);
  const unsigned voff = (unsigned)(l * 16);
  // this wavefront's tiles, contiguous in visiting order it = qa NTR + t
  const int nvisit = nqw * NTR;
  int wbase_tile = 0;
  for (int x = 0; x < wv; ++x) wbase_tile += (NTC - x + 3) / 4 * NTR;
  auto visit_off = [&](int it) {
    if (it > nvisit - 1) it = nvisit - 1;
    return (wbase_tile + it) * TILE_BYTES;
  };
  C p[NCH], nx[NCH];
#pragma unroll
  for (int m = 0; m < NCH; ++m) {
    p[m] = C{};
    nx[m] = C{};
  }
  if (nqw > 0) {
#pragma unroll
    for (int m = 0; m < NCH; ++m) {
      p[m] = lk_ld_chunk<C>(rs, voff + 1024 * m, visit_off(0));
      nx[m] = lk_ld_chunk<C>(rs, voff + 1024 * m, visit_off(1));
    }
  }
  const V2* x0 = xh + k * (long long)nrhs * n + (long long)r0 * n;
  const V2* x1 = xh + kb * (long long)nrhs * n + (long long)r0 * n;
  auto cmul = [](T ar, T ai, V2 x) { return V2{ar * x.x - ai * x.y, ar * x.y + ai * x.x}; };
  // columns of [L | K]: L half v' = v < NP, K half v' = NP + v
  for (int e = threadIdx.x; e < NPC * 4; e += LNT) {
    const int r = e / NPC, vp = e - r * NPC;
    const int half = vp >= NP ? 1 : 0, v = vp - half * NP;
    V2 c0{0, 0}, c1{0, 0};
    if (r < nr && v < nh) {
      const V2 xj = x0[(long long)r * n + v], xm = x0[(long long)r * n + nh + v];
      if (half == 0) {
        c0 = cmul(cf.ar, cf.ai, xj);
        c1 = cmul(cf.er, cf.ei, xm);
      } else {
        c0 = cmul(cf.br, cf.bi, xm);
        c1 = cmul(cf.cr, cf.ci, xj);
      }
    }
    xs[(vp * LNV + 2 * r) * 2] = c0.x;
    xs[(vp * LNV + 2 * r) * 2 + 1] = c0.y;
    xs[(vp * LNV + 2 * r + 1) * 2] = c1.x;
    xs[(vp * LNV + 2 * r + 1) * 2 + 1] = c1.y;
  }
  for (int e = threadIdx.x; e < NP * 4; e += LNT) {
    const int r = e / NP, u = e - r * NP;
    V2 c0{0, 0}, c1{0, 0};
    if (r < nr && u < nh) {
      const V2 xj = x1[(long long)r * n + u], xm = x1[(long long)r * n + nh + u];
      c0 = V2{w[u] * xj.x, w[u] * xj.y};
      c1 = V2{w[u] * xm.x, w[u] * xm.y};
    }
    xt[(u * LNV + 2 * r) * 2] = c0.x;
    xt[(u * LNV + 2 * r) * 2 + 1] = c0.y;
    xt[(u * LNV + 2 * r + 1) * 2] = c1.x;
    xt[(u * LNV + 2 * r + 1) * 2 + 1] = c1.y;
  }
  __syncthreads();
  // lane roles: k-slot kk = l / 16 -> (pair offset off, part); column jj = l % 16:
  // real part of virtual column jj (jj < 8) or imaginary part of jj - 8
  const int kk = l >> 4, jj = l & 15, off = kk >> 1, part_ = kk & 1, a16 = l & 15;
  const bool jre = jj < LNV;
  const int rj = jj & (LNV - 1);
  auto bval = [&](const T* x, int idx) {
    const T xr = x[(idx * LNV + rj) * 2], xi = x[(idx * LNV + rj) * 2 + 1];
    return part_ == 0 ? (jre ? xr : xi) : (jre ? -xi : xr);
  };
  Acc acc[NTR];
#pragma unroll
  for (int t = 0; t < NTR; ++t) acc[t] = Acc{};
  // transposed staging as in the dense paired product
  const int wbase = (part_ * 2 + (a16 & 1)) * 8 + (a16 >> 1);
  const int rbase = ((a16 * 2 + part_) * 2 + off) * 8;
  T* tw = tiles + wv * NSTG * 512;
  int stage = 0, it = 0;
  for (int qa = 0; qa < QPW; ++qa) {
    if (qa >= nqw) break;
    const int q = wv + 4 * qa;
    T b1[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) b1[s] = bval(xs, q * PAIR_TILE + 2 * s + off);
    Acc zq{};
#pragma unroll
    for (int t = 0; t < NTR; ++t, ++it) {
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
      const int noff = visit_off(it + 2);
#pragma unroll
      for (int m = 0; m < NCH; ++m) {
        p[m] = nx[m];
        nx[m] = lk_ld_chunk<C>(rs, voff + 1024 * m, noff);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int s = 0; s < 8; ++s) acc[t] = M::mfma(a1[s], b1[s], acc[t]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int m = 0; m < NCH; ++m)
#pragma unroll
        for (int c = 0; c < CH; ++c) zq = M::mfma(cr[m][c], bval(xt, t * PAIR_TILE + 2 * (m * CH + c) + off), zq);
      stage = NSTG == 2 ? stage ^ 1 : 0;
    }
    // the column sums of tile column q are complete: plain stores
#pragma unroll
    for (int e = 0; e < 4; ++e) zs[(q * PAIR_TILE + M::row(l, e)) * ZST + jj] = zq[e];
  }
  // row sums of the first product: each wavefront's partial sums to LDS,
  // added across the four at the output
  __syncthreads();
#pragma unroll
  for (int t = 0; t < NTR; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) part[(wv * NP + t * PAIR_TILE + M::row(l, e)) * 2 * LNV + jj] = acc[t][e];
  __syncthreads();
  // virtual column j of row i of a [..][16] array: (re, im) = (a[i][j], a[i][8 + j])
  V2* y0 = yh + k * (long long)nrhs * n + (long long)r0 * n;
  V2* y1 = yh + kb * (long long)nrhs * n + (long long)r0 * n;
  for (int e = threadIdx.x; e < nr * nh; e += LNT) {
    const int r = e / nh, u = e - r * nh;
    T jr = 0, ji = 0, mr = 0, mi = 0;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const T* yr = part + (x * NP + u) * 2 * LNV;
      jr += yr[2 * r];
      ji += yr[LNV + 2 * r];
      mr += yr[2 * r + 1];
      mi += yr[LNV + 2 * r + 1];
    }
    y0[(long long)r * n + u] = V2{jr, ji};         // yJ[k]
    y0[(long long)r * n + nh + u] = V2{mr, mi};    // yM[k]
    if (!self) {
      // halves of the transposed products: L^T D xJ, K^T D xJ (column 2r),
      // L^T D xM, K^T D xM (column 2r + 1)
      const T* zl = zs + u * ZST;
      const T* zk = zs + (NP + u) * ZST;
      const T ljr = zl[2 * r], lji = zl[LNV + 2 * r], kjr = zk[2 * r], kji = zk[LNV + 2 * r];
      const T lmr = zl[2 * r + 1], lmi = zl[LNV + 2 * r + 1], kmr = zk[2 * r + 1], kmi = zk[LNV + 2 * r + 1];
      const T di = winv[u];
      const T tjr = cf.ar * ljr - cf.ai * lji + cf.br * kmr - cf.bi * kmi;
      const T tji = cf.ar * lji + cf.ai * ljr + cf.br * kmi + cf.bi * kmr;
      const T tmr = cf.cr * kjr - cf.ci * kji + cf.er * lmr - cf.ei * lmi;
      const T tmi = cf.cr * kji + cf.ci * kjr + cf.er * lmi + cf.ei * lmr;
      y1[(long long)r * n + u] = V2{di * tjr, di * tji};         // yJ[-k]
      y1[(long long)r * n + nh + u] = V2{di * tmr, di * tmi};    // yM[-k]
    }
  }
}

template <typename T>
size_t pair_lk_lds_bytes(int nh) {
  const int np = pair_tiles(nh) * PAIR_TILE, npc = 2 * np;
  const size_t a = (size_t)(npc + np) * LNV * 2 + 4 * LkMf<T>::STAGES * 512, b = (size_t)4 * np * 2 * LNV;
  return ((a > b ? a : b) + (size_t)npc * LkMf<T>::ZST) * sizeof(T);
}

template <typename T, int NTR>
void launch_lk_pair(const void* That, const void* pairs, const void* w, const void* winv, const void* xh, void* yh,
                    int nh, int nrhs, int r0, int nr, int64_t Ps, const LkCoef<T>& cf, hipStream_t s) {
  using V2 = typename LkMf<T>::V2;
  hipLaunchKernelGGL((pair_lk_kernel<T, NTR>), dim3((unsigned)Ps), dim3(LNT), pair_lk_lds_bytes<T>(nh), s,
                     static_cast<const T*>(That), static_cast<const int2*>(pairs), static_cast<const T*>(w),
                     static_cast<const T*>(winv), static_cast<const V2*>(xh), static_cast<V2*>(yh), nh, nrhs, r0, nr,
                     cf);
}

template <typename T>
void launch_lk_typed(const void* That, const void* pairs, const void* w, const void* winv, const void* xh, void* yh,
                     int nh, int nrhs, int64_t Ps, const double* coef, hipStream_t s) {
  EMS_CHECK_ARG(pair_lk_lds_bytes<T>(nh) <= 160 * 1024, "structured paired product: n_eq too large for the LDS");
  const LkCoef<T> cf{(T)coef[0], (T)coef[1], (T)coef[2], (T)coef[3], (T)coef[4], (T)coef[5], (T)coef[6], (T)coef[7]};
  const int ntr = pair_tiles(nh);
  for (int r0 = 0; r0 < nrhs; r0 += 4) {
    const int nr = nrhs - r0 < 4 ? nrhs - r0 : 4;
#define EMS_LK_CASE(N)                                                                  \
  case N:                                                                               \
    launch_lk_pair<T, N>(That, pairs, w, winv, xh, yh, nh, nrhs, r0, nr, Ps, cf, s);   \
    break;
    switch (ntr) {
      EMS_LK_CASE(1) EMS_LK_CASE(2) EMS_LK_CASE(3) EMS_LK_CASE(4) EMS_LK_CASE(5) EMS_LK_CASE(6) EMS_LK_CASE(7)
      EMS_LK_CASE(8) EMS_LK_CASE(9) EMS_LK_CASE(10) EMS_LK_CASE(11) EMS_LK_CASE(12) EMS_LK_CASE(13) EMS_LK_CASE(14)
      default: EMS_CHECK_ARG(false, "structured paired product supports n_eq <= 416");
    }
#undef EMS_LK_CASE
  }
}

}  // namespace

void launch_block_product_pair_lk(Cx t, const void* That, const void* pairs, const void* w, const void* winv,
                                  const void* xh, void* yh, int nh, int nrhs, int64_t Ps, const double* coef,
                                  hipStream_t s) {
  EMS_CHECK_ARG(nh >= 1 && nh <= 256, "structured paired product supports 2 <= n_eq <= 512");
  EMS_CHECK_ARG(nrhs >= 1 && nrhs <= 64, "structured paired product supports 1 <= nrhs <= 64");
  EMS_CHECK_ARG(Ps >= 1 && Ps <= 0x7fffffffLL, "pair count out of range");
  if (t == Cx::C128)
    launch_lk_typed<double>(That, pairs, w, winv, xh, yh, nh, nrhs, Ps, coef, s);
  else
    launch_lk_typed<float>(That, pairs, w, winv, xh, yh, nh, nrhs, Ps, coef, s);
  EMS_LAUNCH_CHECK();
}

}  // namespace emsurf
