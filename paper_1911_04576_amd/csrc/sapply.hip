// Block-diagonal macromodel apply (Sec. III-A, eq. (Zmacromodel_Array)):
// every element m multiplies its own n-vector by the n x n macromodel of its
// cell type (Sec. II-D: one macromodel per unique cell).  Elements are grouped
// by type so that one type's macromodel tile is staged in LDS once and reused
// across up to TC elements: the apply becomes a grouped complex GEMM
// (rows u, columns = elements of one type) with an optional fused
// "y = x - S t" epilogue used by the operator A = I - S T.
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace emsurf {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));

template <typename V> struct Real;
template <> struct Real<float2> { using T = float; };
template <> struct Real<double2> { using T = double; };

template <typename VO, typename VI> __device__ __forceinline__ VO cvt(VI a) {
  using R = typename Real<VO>::T;
  return VO{static_cast<R>(a.x), static_cast<R>(a.y)};
}

constexpr int TU = 64;   // rows per tile
constexpr int TC = 32;   // elements per tile
constexpr int TK = 16;   // reduction chunk

// grid: x = tile index * nrhs + r, y = row block
template <typename VS, typename VT, typename VX>
__global__ void __launch_bounds__(256) apply_S_kernel(const VS* __restrict__ S, const int* __restrict__ elem_sorted,
                                                      const int* __restrict__ tiles, int n, int M, int nrhs,
                                                      const VT* __restrict__ t, const VX* __restrict__ x_axpy,
                                                      VX* __restrict__ y) {
  using R = typename Real<VS>::T;
  __shared__ VS As[TK][TU + 1];
  __shared__ VS Bs[TK][TC + 1];
  const int tile = blockIdx.x / nrhs;
  const int r = blockIdx.x - tile * nrhs;
  const int type = tiles[3 * tile + 0];
  const int start = tiles[3 * tile + 1];
  const int count = tiles[3 * tile + 2];
  const int u0 = blockIdx.y * TU;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const VS* St = S + (long long)type * n * n;
  const VT* tr = t + (long long)r * M * n;
  R accr[4][2], acci[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) { accr[i][j] = 0; acci[i][j] = 0; }
  // element handled by this thread when loading B
  for (int v0 = 0; v0 < n; v0 += TK) {
    // A tile: rows u0..u0+63, cols v0..v0+15  (4 per thread)
#pragma unroll
    for (int rep = 0; rep < 4; ++rep) {
      const int uu = (tid >> 4) + 16 * rep;
      const int vv = tid & 15;
      const int u = u0 + uu, v = v0 + vv;
      As[vv][uu] = (u < n && v < n) ? St[(long long)u * n + v] : VS{0, 0};
    }
    // B tile: elements 0..31 of the tile, v0..v0+15 (2 per thread)
#pragma unroll
    for (int rep = 0; rep < 2; ++rep) {
      const int cc = (tid >> 4) + 16 * rep;
      const int vv = tid & 15;
      const int v = v0 + vv;
      VS val{0, 0};
      if (cc < count && v < n) {
        const int m = elem_sorted[start + cc];
        val = cvt<VS>(tr[(long long)m * n + v]);
      }
      Bs[vv][cc] = val;
    }
    __syncthreads();
#pragma unroll
    for (int vv = 0; vv < TK; ++vv) {
      VS a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[vv][tx + 16 * i];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[vv][ty + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          accr[i][j] += a[i].x * b[j].x - a[i].y * b[j].y;
          acci[i][j] += a[i].x * b[j].y + a[i].y * b[j].x;
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int cc = ty + 16 * j;
    if (cc >= count) continue;
    const int m = elem_sorted[start + cc];
    const long long base = (long long)r * M * n + (long long)m * n;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int u = u0 + tx + 16 * i;
      if (u >= n) continue;
      VX out;
      if (x_axpy) {
        const VX xv = x_axpy[base + u];
        out = VX{xv.x - static_cast<decltype(xv.x)>(accr[i][j]), xv.y - static_cast<decltype(xv.x)>(acci[i][j])};
      } else {
        out = cvt<VX>(VS{accr[i][j], acci[i][j]});
      }
      y[base + u] = out;
    }
  }
}

template <typename VS, typename VT, typename VX>
void launch_typed(const void* S, const TypeTiles& tl, int n, int M, int nrhs, const void* t, const void* x,
                  void* y, hipStream_t s) {
  dim3 grid((unsigned)(tl.n_tiles * nrhs), (unsigned)((n + TU - 1) / TU));
  hipLaunchKernelGGL((apply_S_kernel<VS, VT, VX>), grid, dim3(256), 0, s, static_cast<const VS*>(S),
                     tl.elem_sorted.as<const int>(), tl.tiles.as<const int>(), n, M, nrhs,
                     static_cast<const VT*>(t), static_cast<const VX*>(x), static_cast<VX*>(y));
}

// ----------------------------------------------------------------------------- matrix-core apply
// The grouped product y[col][u] = sum_v S[u][v] t[col][v] of one type on the
// matrix cores (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64), in the real
// embedding of the complex product: A = the t columns (16 columns x 4
// k-slots, slot kk = (half h = kk / 2, part p = kk % 2) of 8 source indices
// v = 16 vt + 8 h + s for MFMA s), B = the macromodel with the signs of the
// complex product folded in (16 output columns = 8 rows u x (re, im)):
//     out re: p = 0 -> Sr[u][v], p = 1 -> -Si[u][v]
//     out im: p = 0 -> Si[u][v], p = 1 ->  Sr[u][v]
// so D[col][(u, q)] is part q of (S t)[col][u].  B comes packed once per plan
// in the lane order of the instruction (below); A is staged per 16-index
// k-tile through LDS from the plain [r][m][v] vectors.
template <typename T> struct SM;
template <> struct SM<float> {
  using V2 = float2;
  using C = f4;
  using Acc = f4;
  __device__ static Acc mfma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int l, int e) { return 4 * (l >> 4) + e; }
};
template <> struct SM<double> {
  using V2 = double2;
  using C = d2;
  using Acc = d4;
  __device__ static Acc mfma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int e) { return (l >> 4) + 4 * e; }
};

constexpr int SA_THREADS = 256;
constexpr int SA_UT = 8;      // row tiles of 8 per workgroup (64 rows)
// columns per workgroup: two wavefronts across, CTW column tiles of 16 each
template <int CTW> constexpr int sa_cols() { return 32 * CTW; }

__host__ __device__ inline int s_row_tiles(int n) { return (n + 7) / 8; }
__host__ __device__ inline int s_k_tiles(int n) { return (n + 15) / 16; }

// Packed layout per type: blocks (ut, vt) of 512 reals, ut = u / 8 outer,
// vt = v / 16 inner; within a block, value s of lane L = 16 kk + j (k-slot
// kk, output column j = (u % 8) + 8 q) at (s / CH) 64 CH + L CH + s % CH,
// CH = 16 / (bytes of a real), so that each 16-byte load instruction of a
// wavefront reads 1024 contiguous bytes.  Zero beyond n.
template <typename T>
__global__ void pack_S_kernel(const double2* __restrict__ S, T* __restrict__ out, int n, int n_types) {
  constexpr int CH = 16 / (int)sizeof(T);
  const int nut = s_row_tiles(n), nvt = s_k_tiles(n);
  const long long total = (long long)n_types * nut * nvt * 512;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long blk = i / 512;
    const int w = (int)(i - blk * 512);
    const int sc = w / (64 * CH), rem = w - sc * 64 * CH, L = rem / CH, s = sc * CH + rem % CH;
    const int type = (int)(blk / ((long long)nut * nvt));
    const int r2 = (int)(blk - (long long)type * nut * nvt), ut = r2 / nvt, vt = r2 - (r2 / nvt) * nvt;
    const int kk = L >> 4, j = L & 15, h = kk >> 1, p = kk & 1, q = j >> 3;
    const int u = ut * 8 + (j & 7), v = vt * 16 + h * 8 + s;
    double val = 0.0;
    if (u < n && v < n) {
      const double2 a = S[((long long)type * n + u) * n + v];
      val = q == 0 ? (p == 0 ? a.x : -a.y) : (p == 0 ? a.y : a.x);
    }
    out[i] = static_cast<T>(val);
  }
}

// Work items w = (type tile * nub + row block) * ncb + column block, in type
// order.  Workgroups go to the 8 XCDs in turn (workgroup b to XCD b % 8), so
// XCD x takes the contiguous items [x per, (x + 1) per): the workgroups an
// XCD holds at a time share a few macromodel slices in its L2.  Wavefront
// (wc, wu) = (w % 2, w / 2) takes column tiles CTW wc .. CTW wc + CTW - 1 and
// row tiles 4 wu .. 4 wu + 3 of the item.
template <typename T, typename VX, int CTW>
__global__ void __launch_bounds__(SA_THREADS, sizeof(T) == 8 ? 3 : 2) apply_S_mfma_kernel(
    const T* __restrict__ Sp, const int* __restrict__ elem_sorted, const int* __restrict__ tiles, int n, int M,
    int nrhs, int ncb, int nub, int items, int per, const typename SM<T>::V2* __restrict__ t,
    const VX* __restrict__ x_axpy, VX* __restrict__ y) {
  using V2 = typename SM<T>::V2;
  using C = typename SM<T>::C;
  using Acc = typename SM<T>::Acc;
  using R = typename Real<VX>::T;
  constexpr int CH = 16 / (int)sizeof(T), NCH = 8 / CH;
  constexpr int NCOL = sa_cols<CTW>(), NAC = (NCOL + 63) / 64;   // columns staged per thread
  constexpr int NBC = SA_UT * 512 / CH / SA_THREADS;   // macromodel chunks staged per thread
  // a k-tile of the vectors in A-lane order and of the packed macromodels;
  // two buffers: the next k-tile is staged while the current one is used.
  // At the end the same memory holds the output tile, rows of YROW values
  // (64 rows u x (re, im) and padding: the rows start 16 banks apart)
  // (FP64 keeps one macromodel buffer: 48 KB of LDS, three workgroups per CU,
  // for a second barrier per k-tile)
  constexpr int NB = sizeof(T) == 8 ? 1 : 2;
  constexpr int AS = 2 * CTW * 512, BS = SA_UT * 512;
  constexpr int YROW = sizeof(T) == 4 ? 132 : 144;
  constexpr int LDS_T = 2 * AS + NB * BS > NCOL * YROW ? 2 * AS + NB * BS : NCOL * YROW;
  __shared__ __align__(16) T lds[LDS_T];
  auto As = [&](int bf) { return lds + bf * AS; };
  auto Bs = [&](int bf) { return lds + 2 * AS + (NB == 2 ? bf : 0) * BS; };
  const int w = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (w >= items) return;   // the whole workgroup: no barrier reached
  const int cb = w % ncb, tub = w / ncb, tile = tub / nub, ub = tub - tile * nub;
  const int type = tiles[3 * tile], start = tiles[3 * tile + 1], count = tiles[3 * tile + 2];
  const int ncols = nrhs * count, col0 = cb * NCOL;
  if (col0 >= ncols) return;   // the whole workgroup: no barrier reached
  const int nut = s_row_tiles(n), nvt = s_k_tiles(n);
  const int ut0 = ub * SA_UT;
  const T* St = Sp + (long long)type * nut * nvt * 512;
  const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6, wc = wv & 1, wu = wv >> 1;
  // A staging: columns ac + 64 g of the block, source indices 4 aq .. 4 aq + 3 of the k-tile
  const int ac = tid >> 2, aq = tid & 3;
  // Element indices of the block's columns: the input columns of this
  // thread's A staging (NAC) and the output chunks' columns (NXC), loaded
  // at a clamped index without conditions and all before the first is used
  // (the compiler barrier keeps them from sinking into the conditional
  // blocks that use them, where each would cost a wait of its own)
  constexpr int XC = 16 / (2 * (int)sizeof(R)), CPC = 64 / XC, NXC = NCOL * CPC / SA_THREADS;
  int el_a[NAC], el_x[NXC];
#pragma unroll
  for (int g = 0; g < NAC; ++g) {
    const int acol = col0 + ac + 64 * g;
    const bool ok = ac + 64 * g < NCOL && acol < ncols;
    el_a[g] = elem_sorted[start + (ok ? acol % count : 0)];
  }
#pragma unroll
  for (int k = 0; k < NXC; ++k) {
    const int col = col0 + (tid + SA_THREADS * k) / CPC;
    el_x[k] = elem_sorted[start + (col < ncols ? col % count : 0)];
  }
  asm volatile("" ::: "memory");
  const V2* tcol[NAC];
#pragma unroll
  for (int g = 0; g < NAC; ++g) {
    const int acol = col0 + ac + 64 * g;
    const bool ok = ac + 64 * g < NCOL && acol < ncols;
    tcol[g] = ok ? t + ((long long)(acol / count) * M + el_a[g]) * n : nullptr;
  }
  V2 an[NAC][4];
  auto load_a = [&](int vt) {
#pragma unroll
    for (int g = 0; g < NAC; ++g)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int v = vt * 16 + 4 * aq + i;
        an[g][i] = (tcol[g] != nullptr && v < n) ? tcol[g][v] : V2{0, 0};
      }
  };
  // the workgroup's SA_UT row tiles of the packed macromodels (zero past n)
  C bn[NBC];
  auto load_b = [&](int vt) {
#pragma unroll
    for (int j = 0; j < NBC; ++j) {
      const int ci = tid + SA_THREADS * j, bu = ci / (512 / CH), wi = ci - bu * (512 / CH);
      bn[j] = ut0 + bu < nut ? *reinterpret_cast<const C*>(St + ((long long)(ut0 + bu) * nvt + vt) * 512 + wi * CH)
                             : C{};
    }
  };
  // A-lane position of this thread's values: lane (2 h + p) 16 + ac % 16 of column tile ac / 16 + 4 g
  const int ah = aq >> 1, as0 = 4 * (aq & 1), act = ac >> 4, a16 = ac & 15;
  Acc acc[CTW][4];
#pragma unroll
  for (int i = 0; i < CTW; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = Acc{};
  R* yr = reinterpret_cast<R*>(y);
  const R* xr = reinterpret_cast<const R*>(x_axpy);
  // stage the k-tile held in an and bn into LDS buffer bf (whose previous
  // contents every wavefront has used: a barrier lies between)
  auto stage = [&](int bf) {
#pragma unroll
    for (int g = 0; g < NAC; ++g)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        if (ac + 64 * g >= NCOL) break;
        const int L = (2 * ah + p) * 16 + a16;
        T* dst = As(bf) + (act + 4 * g) * 512;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int s = as0 + i;
          dst[(s / CH) * 64 * CH + L * CH + s % CH] = p == 0 ? an[g][i].x : an[g][i].y;
        }
      }
#pragma unroll
    for (int j = 0; j < NBC; ++j) *reinterpret_cast<C*>(Bs(bf) + (tid + SA_THREADS * j) * CH) = bn[j];
  };
  // the products of the k-tile staged in buffer bf
  auto products = [&](int bf) {
    C a[CTW][NCH], b[4][NCH];
#pragma unroll
    for (int i = 0; i < CTW; ++i)
#pragma unroll
      for (int m = 0; m < NCH; ++m)
        a[i][m] = *reinterpret_cast<const C*>(As(bf) + (CTW * wc + i) * 512 + m * 64 * CH + l * CH);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int m = 0; m < NCH; ++m)
        b[j][m] = *reinterpret_cast<const C*>(Bs(bf) + (4 * wu + j) * 512 + m * 64 * CH + l * CH);
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int i = 0; i < CTW; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = SM<T>::mfma(a[i][s / CH][s % CH], b[j][s / CH][s % CH], acc[i][j]);
  };
  // Output chunks of 16 bytes (XC complex values of x and y): chunk k of
  // this thread is column c = k-th chunk / (64 / XC), rows 8 ut0 + XC (chunk
  // % (64 / XC)) + 0 .. XC - 1.  Whole chunks where n allows 16-byte access
  // (n even for FP32 vectors); value by value otherwise.
  using XV = typename std::conditional<sizeof(R) == 4, f4, d2>::type;
  const bool whole = XC == 1 || (n & 1) == 0;
  // twice the vector offset (in reals) of the column of each chunk, -1 past the block's columns
  long long colbase[NXC];
#pragma unroll
  for (int k = 0; k < NXC; ++k) {
    const int col = col0 + (tid + SA_THREADS * k) / CPC;
    colbase[k] = col < ncols ? 2 * (((long long)(col / count) * M + el_x[k]) * n) : -1;
  }
  // the vectors of the fused y = x - S t, requested before the last products
  XV xv[NXC];
  auto load_x = [&]() {
    if (!xr) return;
#pragma unroll
    for (int k = 0; k < NXC; ++k) {
      const int ch = tid + SA_THREADS * k, c = ch / CPC, u = 8 * ut0 + XC * (ch - c * CPC);
      const long long b = colbase[k];
      xv[k] = XV{};
      if (b >= 0 && whole && u + XC <= n) {
        xv[k] = *reinterpret_cast<const XV*>(xr + b + 2 * u);
      } else if (b >= 0) {
#pragma unroll
        for (int z = 0; z < 2 * XC; ++z)
          if (u + z / 2 < n) xv[k][z] = xr[b + 2 * u + z];
      }
    }
  };
  load_a(0);
  load_b(0);
  stage(0);
  __syncthreads();
  for (int vt = 0; vt + 1 < nvt; ++vt) {
    load_a(vt + 1);   // the next k-tile is on its way during the products
    load_b(vt + 1);
    products(vt & 1);
    if constexpr (NB == 1) __syncthreads();   // (one buffer: every read of it precedes the next fill)
    stage((vt + 1) & 1);
    __syncthreads();
  }
  load_x();
  products((nvt - 1) & 1);
  // the output tile through LDS: every wavefront is past its last reads first
  __syncthreads();
  {
    const int jj = l & 15, q = jj >> 3;
#pragma unroll
    for (int i = 0; i < CTW; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = 16 * (CTW * wc + i) + SM<T>::row(l, e);
#pragma unroll
        for (int j = 0; j < 4; ++j) lds[c * YROW + 2 * (8 * (4 * wu + j) + (jj & 7)) + q] = acc[i][j][e];
      }
  }
  __syncthreads();
  // (the loads of x all complete here, once: the stores below sit in
  // conditional blocks, and a load still counted as pending at each block's
  // join would cost a wait for every store before it)
  __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
  for (int k = 0; k < NXC; ++k) {
    const int ch = tid + SA_THREADS * k, c = ch / CPC, ul = XC * (ch - c * CPC), u = 8 * ut0 + ul;
    const long long b = colbase[k];
    if (b < 0 || u >= n) continue;
    XV v;
#pragma unroll
    for (int z = 0; z < 2 * XC; ++z) v[z] = static_cast<R>(lds[c * YROW + 2 * ul + z]);
    if (xr) v = xv[k] - v;
    if (whole && u + XC <= n) {
      *reinterpret_cast<XV*>(yr + b + 2 * u) = v;
    } else {
#pragma unroll
      for (int z = 0; z < 2 * XC; ++z)
        if (u + z / 2 < n) yr[b + 2 * u + z] = v[z];
    }
  }
}

template <typename T, typename VX, int CTW = sizeof(T) == 4 ? 2 : 1>
void launch_mfma_typed(const void* Sp, const TypeTiles& tl, int n, int M, int nrhs, const void* t, const void* x,
                       void* y, hipStream_t s) {
  const int ncb = (nrhs * TC + sa_cols<CTW>() - 1) / sa_cols<CTW>();
  const int nub = (s_row_tiles(n) + SA_UT - 1) / SA_UT;
  const long long items = (long long)tl.n_tiles * ncb * nub;
  EMS_CHECK_ARG(items + 8 <= 0x7fffffffLL, "too many macromodel tiles");
  const int per = (int)((items + 7) / 8);
  hipLaunchKernelGGL((apply_S_mfma_kernel<T, VX, CTW>), dim3((unsigned)(8 * per)), dim3(SA_THREADS), 0, s,
                     static_cast<const T*>(Sp), tl.elem_sorted.as<const int>(), tl.tiles.as<const int>(), n, M, nrhs,
                     ncb, nub, (int)items, per,
                     static_cast<const typename SM<T>::V2*>(t), static_cast<const VX*>(x), static_cast<VX*>(y));
}

}  // namespace

int apply_S_tile_cols() { return TC; }

size_t packed_S_reals(int n, int n_types) { return (size_t)n_types * s_row_tiles(n) * s_k_tiles(n) * 512; }

void launch_pack_S(Cx t, const void* S64, void* out, int n, int n_types, hipStream_t s) {
  const long long total = (long long)packed_S_reals(n, n_types);
  const unsigned blocks = (unsigned)std::min<long long>((total + 255) / 256, 65536);
  if (t == Cx::C128)
    hipLaunchKernelGGL(pack_S_kernel<double>, dim3(blocks), dim3(256), 0, s, static_cast<const double2*>(S64),
                       static_cast<double*>(out), n, n_types);
  else
    hipLaunchKernelGGL(pack_S_kernel<float>, dim3(blocks), dim3(256), 0, s, static_cast<const double2*>(S64),
                       static_cast<float*>(out), n, n_types);
  EMS_LAUNCH_CHECK();
}

void launch_apply_S_packed(Cx tc, Cx txy, const void* Sp, const TypeTiles& tiles, int n, int M, int nrhs,
                           const void* t, const void* x_axpy, void* y, hipStream_t s) {
  if (tc == Cx::C128) {
    EMS_CHECK_ARG(txy == Cx::C128, "FP64 macromodel apply needs FP64 vectors");
    launch_mfma_typed<double, double2>(Sp, tiles, n, M, nrhs, t, x_axpy, y, s);
  } else if (txy == Cx::C64) {
    launch_mfma_typed<float, float2>(Sp, tiles, n, M, nrhs, t, x_axpy, y, s);
  } else {
    launch_mfma_typed<float, double2>(Sp, tiles, n, M, nrhs, t, x_axpy, y, s);
  }
  EMS_LAUNCH_CHECK();
}

void launch_apply_S(Cx ts, Cx tt, Cx txy, const void* S, const TypeTiles& tiles, int n, int M, int nrhs,
                    const void* t, const void* x_axpy, void* y, hipStream_t s) {
  EMS_CHECK_ARG((long long)tiles.n_tiles * nrhs <= 0x7fffffffLL, "too many macromodel tiles");
  if (ts == Cx::C128) {
    EMS_CHECK_ARG(tt == Cx::C128 && txy == Cx::C128, "FP64 macromodel apply needs FP64 vectors");
    launch_typed<double2, double2, double2>(S, tiles, n, M, nrhs, t, x_axpy, y, s);
  } else if (tt == Cx::C64 && txy == Cx::C64) {
    launch_typed<float2, float2, float2>(S, tiles, n, M, nrhs, t, x_axpy, y, s);
  } else if (tt == Cx::C64 && txy == Cx::C128) {
    launch_typed<float2, float2, double2>(S, tiles, n, M, nrhs, t, x_axpy, y, s);
  } else {
    EMS_CHECK_ARG(false, "unsupported macromodel apply type combination");
  }
  EMS_LAUNCH_CHECK();
}

}  // namespace emsurf
