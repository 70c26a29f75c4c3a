// Block-diagonal macromodel apply (Sec. III-A, eq. (Zmacromodel_Array)):
// every element m multiplies its own n-vector by the n x n macromodel of its
// cell type (Sec. II-D: one macromodel per unique cell).  Elements are grouped
// by type so that one type's macromodel tile is staged in LDS once and reused
// across up to TC elements: the apply becomes a grouped complex GEMM
// (rows u, columns = elements of one type) with an optional fused
// "y = x - S t" epilogue used by the operator A = I - S T.
#include "internal.h"

namespace emsurf {
namespace {

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

}  // namespace

int apply_S_tile_cols() { return TC; }

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
