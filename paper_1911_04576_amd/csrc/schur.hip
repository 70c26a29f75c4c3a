// Macromodel generation for unique cells (Sec. II-D, eq. (Zmacromodel)): the
// interior unknowns of a cell are eliminated with the Schur complement
//     Z~ = Z_eq,eq - Z_eq,int Z_int,int^-1 Z_int,eq,
// which takes an LU factorisation of Z_int,int; cells are independent.  The
// operator of the solve then needs S = -(Z~ + Z_self)^-1 (block-Jacobi form
// of Sec. III-C).
//
// Both steps are one operation, the partial elimination of the leading K x K
// block of an N x N matrix, after which the trailing block holds
// A22 - A21 A11^-1 A12:
//   step 1: [[Z_int,int, Z_int,eq], [Z_eq,int, Z_eq,eq]], K = n_int  ->  Z~
//   step 2: [[Z~ + Z_self, I], [I, 0]],                  K = n_eq   ->  -(Z~ + Z_self)^-1 = S
// The elimination is right-looking and blocked (blocks of two 32-column
// panels, a lookahead of one block on a second stream) with partial pivoting
// among the leading rows (trailing rows never move, so the trailing block is
// exactly the Schur complement); every matrix of the batch (one per cell
// type) runs in the same launches, and the trailing updates spread over many
// workgroups per matrix.  FP64 complex throughout; row-major storage, matrix
// b at A + b N^2.
#include <vector>

#include <hip/hip_ext.h>

#include "internal.h"

namespace emsurf {
namespace {

constexpr int PANEL = 32;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ double2 csub_mul(double2 c, double2 a, double2 b) {
  // c - a b with fused multiply-adds
  return double2{__builtin_fma(-a.x, b.x, __builtin_fma(a.y, b.y, c.x)),
                 __builtin_fma(-a.x, b.y, __builtin_fma(-a.y, b.x, c.y))};
}
__device__ __forceinline__ double2 cinv(double2 a) {
  const double rd = 1.0 / (a.x * a.x + a.y * a.y);
  return double2{a.x * rd, -a.y * rd};
}

// Panel columns [k0, k0 + kb) over rows [k0, N): pivot, swap (panel columns
// only), multipliers, update inside the panel.  One workgroup of 512 threads
// per matrix.
// info[b] receives 1 + the first column whose pivot candidates are all zero.
__global__ void __launch_bounds__(512) panel_kernel(double2* __restrict__ A, int N, int K, int k0, int kb,
                                                    int* __restrict__ piv, int* __restrict__ info) {
  const int b = blockIdx.x;
  double2* M = A + (long long)b * N * N;
  __shared__ double best_v[512];
  __shared__ int best_i[512];
  __shared__ double2 prow[PANEL];
  for (int kk = k0; kk < k0 + kb; ++kk) {
    // pivot: largest |a|^2 among the leading rows [kk, K), first index on ties
    double bv = -1.0;
    int bi = kk;
    for (int i = kk + threadIdx.x; i < K; i += blockDim.x) {
      const double2 a = M[(long long)i * N + kk];
      const double v = a.x * a.x + a.y * a.y;
      if (v > bv) { bv = v; bi = i; }
    }
    best_v[threadIdx.x] = bv;
    best_i[threadIdx.x] = bi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        const double ov = best_v[threadIdx.x + s];
        const int oi = best_i[threadIdx.x + s];
        if (ov > best_v[threadIdx.x] || (ov == best_v[threadIdx.x] && oi < best_i[threadIdx.x])) {
          best_v[threadIdx.x] = ov;
          best_i[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    const int p = best_i[0];
    const bool singular = !(best_v[0] > 0.0);
    if (threadIdx.x == 0) {
      piv[(long long)b * K + kk] = p;
      if (singular && info[b] == 0) info[b] = kk + 1;
    }
    // swap rows kk and p in the panel columns, keep the pivot row segment
    for (int j = k0 + threadIdx.x; j < k0 + kb; j += blockDim.x) {
      const double2 t = M[(long long)p * N + j];
      if (p != kk) M[(long long)p * N + j] = M[(long long)kk * N + j];
      M[(long long)kk * N + j] = t;
      prow[j - k0] = t;
    }
    __syncthreads();
    const double2 inv = singular ? double2{0.0, 0.0} : cinv(prow[kk - k0]);
    for (int i = kk + 1 + threadIdx.x; i < N; i += blockDim.x) {
      double2* row = M + (long long)i * N;
      row[kk] = cmul(row[kk], inv);
    }
    __syncthreads();
    // rank-1 update of the rest of the panel, one (row, column) pair per thread
    const int w = k0 + kb - kk - 1;
    if (w > 0) {
      const long long pairs = (long long)(N - kk - 1) * w;
      for (long long t = threadIdx.x; t < pairs; t += blockDim.x) {
        const int i = kk + 1 + (int)(t / w);
        const int j = kk + 1 + (int)(t - (long long)(i - kk - 1) * w);
        double2* row = M + (long long)i * N;
        row[j] = csub_mul(row[j], row[kk], prow[j - k0]);
      }
    }
    __syncthreads();
  }
}

// Lane value moved by DPP within rows of 16 lanes (quad permutes, row
// rotations); a double moves as its two halves
template <int CTRL> __device__ __forceinline__ double dpp_d(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL> __device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ void argmax_take(double& v, int& idx, double ov, int oi) {
  // (bitwise operators: no short-circuit branches)
  const bool take = (ov > v) | ((ov == v) & (oi < idx));
  v = take ? ov : v;
  idx = take ? oi : idx;
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
// The same as a DPP move that only the rows in RM take (the other rows keep
// their value): the row broadcasts of 64-lane reductions
template <int CTRL, int RM> __device__ __forceinline__ double bcast_dpp_d(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, RM, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, RM, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
// (largest v, first index on ties) over the 64 lanes, as wavefront-uniform
// values: quad exchanges 1 and 2 and row rotations 4 and 8 by DPP leave each
// row of 16 lanes with its own result; row_bcast:15 then brings lane 15 of
// rows 0 and 2 into rows 1 and 3, row_bcast:31 lane 31 into rows 2 and 3, so
// that row 3 holds the result of all four, read from lane 63 (the order
// does not matter: the rule is a maximum over (v, -index))
__device__ __forceinline__ void wave_argmax(double& v, int& idx) {
  argmax_take(v, idx, dpp_d<0xB1>(v), dpp_i<0xB1>(idx));   // quad_perm [1,0,3,2]
  argmax_take(v, idx, dpp_d<0x4E>(v), dpp_i<0x4E>(idx));   // quad_perm [2,3,0,1]
  argmax_take(v, idx, dpp_d<0x124>(v), dpp_i<0x124>(idx)); // row_ror 4
  argmax_take(v, idx, dpp_d<0x128>(v), dpp_i<0x128>(idx)); // row_ror 8
  argmax_take(v, idx, bcast_dpp_d<0x142, 0xA>(v), __builtin_amdgcn_update_dpp(idx, idx, 0x142, 0xA, 0xF, false));
  argmax_take(v, idx, bcast_dpp_d<0x143, 0xC>(v), __builtin_amdgcn_update_dpp(idx, idx, 0x143, 0xC, 0xF, false));
  v = readlane_d(v, 63);
  idx = __builtin_amdgcn_readlane(idx, 63);
}

// The same panel with the rows in registers, for N - k0 <= NT * RPT: NT
// threads, thread t owning rows k0 + t, k0 + t + NT, ... (RPT of them; few
// wavefronts keep the per-column barriers and reductions short).  The
// panel's columns go in sub-blocks of PSB: a sub-block is staged through
// LDS with coalesced loads and stores (rows [c0, N)), held in registers, its
// columns are factorised there (pivot by a reduction over the thread's rows,
// a wavefront reduction and one over the NT / 64 wavefronts in LDS, row
// exchange through LDS), and the columns outside it then take the
// sub-block's row swaps at once (the panel's others, the lw columns left of
// the panel and the rw columns right of it), and the columns to its right
// (the panel's and the rw beyond) its U rows (L11^-1 A12 by one wavefront)
// and one rank-PSB update, so that the panel makes one pass through memory
// per sub-block instead of one per column.  Same pivots (largest |a|^2
// among rows [kk, K), first index on ties), same singular flags.
constexpr int PSB = 8;
template <int NT, int RPT>
__global__ void __launch_bounds__(NT) panel_reg_kernel(double2* __restrict__ A, int N, int K, int k0, int kb, int lw,
                                                            int rw, int* __restrict__ piv, int* __restrict__ info) {
  const int b = blockIdx.x;
  double2* M = A + (long long)b * N * N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double rv[2][NT / 64];
  __shared__ int ri[2][NT / 64];
  __shared__ double2 cand[2][NT / 64][PSB];   // each wavefront's best candidate row
  __shared__ double2 krow[2][PSB];                 // row col, which the pivot row displaces
  __shared__ double2 U[PSB][2 * PANEL];    // the sub-block's U rows over the columns to its right
  __shared__ int spv[PSB];                 // the sub-block's pivot rows
  extern __shared__ double2 sub[];         // [N - c0][PSB]: the sub-block, rows c0 ..
  auto rowof = [&](int q) { return k0 + tid + NT * q; };
  int first_singular = -1;   // the same in every thread
  for (int sb0 = 0; sb0 < kb; sb0 += PSB) {
    const int sbw = kb - sb0 < PSB ? kb - sb0 : PSB;
    const int c0 = k0 + sb0, rc0 = sb0 + sbw;   // rc0: first panel column to the right (panel-relative)
    // rows above c0 keep their values in this sub-block (U rows of the panel)
    // (every load of the sub-block is issued before the first is used:
    // nsub <= RPT * NT * PSB)
    const int nsub = (N - c0) * PSB;
    {
      double2 st[RPT * PSB];
#pragma unroll
      for (int j = 0; j < RPT * PSB; ++j) {
        const int e = tid + NT * j, c = e & (PSB - 1);
        st[j] = (e < nsub && c < sbw) ? M[(long long)(c0 + (e / PSB)) * N + k0 + sb0 + c] : double2{0.0, 0.0};
      }
#pragma unroll
      for (int j = 0; j < RPT * PSB; ++j) {
        const int e = tid + NT * j;
        if (e < nsub) sub[e] = st[j];
      }
    }
    __syncthreads();
    double2 r[RPT][PSB];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int rr = rowof(q);
#pragma unroll
      for (int c = 0; c < PSB; ++c) r[q][c] = (rr >= c0 && rr < N) ? sub[(rr - c0) * PSB + c] : double2{0.0, 0.0};
    }
#pragma unroll
    for (int kk = 0; kk < PSB; ++kk) {
      if (kk >= sbw) break;
      const int col = k0 + sb0 + kk;
      // pivot: largest |a|^2 among rows [col, K), first index on ties
      double v = -1.0;
      int idx = tid;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int rr = rowof(q);
        const double vq = (rr >= col && rr < K) ? r[q][kk].x * r[q][kk].x + r[q][kk].y * r[q][kk].y : -1.0;
        argmax_take(v, idx, vq, rr);
      }
      wave_argmax(v, idx);
      // one barrier per column: before it each wavefront publishes its best
      // candidate (value, row, and the row's sub-block values), and the owner
      // of row col publishes that row; the slots alternate with the column's
      // parity, so the next column's writes cannot meet this column's reads
      const int par = kk & 1;
      if (lane == 0) {
        rv[par][wave] = v;
        ri[par][wave] = idx;
      }
      const int qc = (col - k0) / NT;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        if (rowof(q) == idx && v >= 0.0)
#pragma unroll
          for (int c = 0; c < PSB; ++c) cand[par][wave][c] = r[q][c];
        if (q == qc && tid == (col - k0) % NT)
#pragma unroll
          for (int c = 0; c < PSB; ++c) krow[par][c] = r[q][c];
      }
      __syncthreads();
      // the wavefronts' candidates: lane w (w < NT / 64) of every row of 16
      // lanes takes wavefront w's, the others an empty one that never wins;
      // four DPP steps leave every lane with the best, read as uniform values
      double bv;
      int p;
      {
        const int w = lane & 15;
        double cv = w < NT / 64 ? rv[par][w < NT / 64 ? w : 0] : -2.0;
        int ci = w < NT / 64 ? ri[par][w < NT / 64 ? w : 0] : 0x7fffffff;
        argmax_take(cv, ci, dpp_d<0xB1>(cv), dpp_i<0xB1>(ci));
        argmax_take(cv, ci, dpp_d<0x4E>(cv), dpp_i<0x4E>(ci));
        argmax_take(cv, ci, dpp_d<0x124>(cv), dpp_i<0x124>(ci));
        argmax_take(cv, ci, dpp_d<0x128>(cv), dpp_i<0x128>(ci));
        bv = readlane_d(cv, 0);
        p = __builtin_amdgcn_readlane(ci, 0);
      }
      const int pw = ((p - k0) % NT) / 64;   // the wavefront that holds row p
      const double2* prow = cand[par][pw];   // the pivot row over the sub-block
      const bool singular = !(bv > 0.0);
      if (singular && first_singular < 0) first_singular = col;
      if (tid == 0) spv[kk] = p;
      // exchange rows col and p in this sub-block (the other panel columns
      // take the sub-block's swaps together after it: no memory operation
      // inside the column loop, whose barrier would wait for it)
      if (p != col) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          if (rowof(q) == col) {
#pragma unroll
            for (int c = 0; c < PSB; ++c) r[q][c] = prow[c];
          } else if (rowof(q) == p) {
#pragma unroll
            for (int c = 0; c < PSB; ++c) r[q][c] = krow[par][c];
          }
        }
      }
      // multipliers and the rank-1 update inside the sub-block
      const double2 inv = singular ? double2{0.0, 0.0} : cinv(prow[kk]);
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int rr = rowof(q);
        if (rr < N && rr > col) {
          const double2 mlt = cmul(r[q][kk], inv);
          r[q][kk] = mlt;
#pragma unroll
          for (int c = 0; c < PSB; ++c)
            if (c > kk && c < sbw) r[q][c] = csub_mul(r[q][c], mlt, prow[c]);
        }
      }
    }
    // the sub-block back to memory through LDS
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int rr = rowof(q);
      if (rr >= c0 && rr < N)
#pragma unroll
        for (int c = 0; c < PSB; ++c) sub[(rr - c0) * PSB + c] = r[q][c];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RPT * PSB; ++j) {
      const int e = tid + NT * j, c = e & (PSB - 1);
      if (e < nsub && c < sbw) M[(long long)(c0 + (e / PSB)) * N + k0 + sb0 + c] = sub[e];
    }
    // the sub-block's swaps on the other panel columns, and on the lw
    // columns left of the panel, at once: (slot x, column k0 - lw + c)
    // writes row X (c0 + x / 2, or the pivot row of column x / 2) with the
    // value the swap sequence brings to it, the value that row sigma(X) held
    // before, sigma the swaps applied in reverse order
    {
      constexpr int H = (2 * PSB * 2 * PANEL + NT - 1) / NT;
      int Xs[H], srcs[H];
      double2 mv[H];
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int e = tid + NT * h, x = e / (2 * PANEL), c = e % (2 * PANEL);
        Xs[h] = -1;
        srcs[h] = -1;
        mv[h] = double2{0.0, 0.0};
        if (x < 2 * sbw && c < lw + kb + rw && (c < lw + sb0 || c >= lw + sb0 + sbw)) {
          const int X = (x & 1) ? spv[x >> 1] : c0 + (x >> 1);
          int src = X;
          for (int i = sbw - 1; i >= 0; --i) {
            const int pi = spv[i];
            if (src == c0 + i)
              src = pi;
            else if (src == pi)
              src = c0 + i;
          }
          if (src != X) {
            Xs[h] = X;
            srcs[h] = src;
            mv[h] = M[(long long)src * N + k0 - lw + c];
          }
        }
      }
      __syncthreads();   // every value is read before any is written
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int c = (tid + NT * h) % (2 * PANEL);
        if (Xs[h] >= 0) M[(long long)Xs[h] * N + k0 - lw + c] = mv[h];
      }
      if (tid < sbw) piv[(long long)b * K + c0 + tid] = spv[tid];
    }
    if (rc0 < kb + rw) {
      // (the sub-block's unit lower factor: rows 0 .. sbw - 1 of sub)
      __syncthreads();
      // U rows c0 .. c0 + sbw - 1 over the columns to the right: forward
      // substitution with the unit lower L11, one lane per column
      if (wave == 0 && rc0 + lane < kb + rw) {
        const int c = rc0 + lane;
        double2 x[PSB];
#pragma unroll
        for (int i = 0; i < PSB; ++i) x[i] = i < sbw ? M[(long long)(c0 + i) * N + k0 + c] : double2{0.0, 0.0};
#pragma unroll
        for (int i = 0; i < PSB; ++i) {
          if (i >= sbw) break;
          double2 vv = x[i];
#pragma unroll
          for (int j = 0; j < PSB; ++j)
            if (j < i) vv = csub_mul(vv, sub[i * PSB + j], x[j]);
          x[i] = vv;
          U[i][c] = vv;
          M[(long long)(c0 + i) * N + k0 + c] = vv;
        }
      }
      __syncthreads();
      // rank-sbw update of the columns to the right for the rows below the
      // sub-block: a thread keeps one column's U values in registers and
      // walks rows rofs, rofs + rstep, ... (consecutive threads on
      // consecutive columns of a row, the row's multipliers from LDS), with
      // UB rows' requests in flight at once
      constexpr int UB = NT >= 1024 ? 4 : 16;   // (fewer registers for the larger workgroup)
      const int nrc = kb + rw - rc0, rstep = NT / nrc, nrow = N - c0 - sbw;
      const int rofs = tid / nrc, c = rc0 + tid % nrc;
      if (rofs < rstep) {
        double2 u[PSB];
#pragma unroll
        for (int i = 0; i < PSB; ++i) u[i] = i < sbw ? U[i][c] : double2{0.0, 0.0};
        for (int rb = rofs; rb < nrow; rb += UB * rstep) {
          double2 vv[UB];
#pragma unroll
          for (int z = 0; z < UB; ++z) {
            const int rl = rb + z * rstep;
            vv[z] = rl < nrow ? M[(long long)(c0 + sbw + rl) * N + k0 + c] : double2{0.0, 0.0};
          }
          // (u[i] is zero for i >= sbw: an element's eight multipliers are
          // read without conditions, together)
#pragma unroll
          for (int z = 0; z < UB; ++z) {
            const int rl = rb + z * rstep;
            if (rl < nrow) {
              double2 w = vv[z];
#pragma unroll
              for (int i = 0; i < PSB; ++i) w = csub_mul(w, sub[(sbw + rl) * PSB + i], u[i]);
              M[(long long)(c0 + sbw + rl) * N + k0 + c] = w;
            }
          }
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0 && first_singular >= 0 && info[b] == 0) info[b] = first_singular + 1;
}

// Columns [cb, ce) right of the block (cb >= k0 + kb): the block's row
// swaps, then U12 = L11^-1 A12 (unit lower triangular L11 of the block).
// STP lanes per column (a row of 16 lanes, or a quad), lane g holding rows
// g, g + STP, ... of it.  The
// swaps are composed before any memory is touched: only the block rows and
// the pivot rows move, and after the swap sequence row X holds what row
// sigma(X) held before, sigma the swaps applied in reverse order; a column
// is read once for those rows and written once.  The substitution goes by
// columns of L11: the owner of x[l] broadcasts it to the column's lanes by
// DPP (row_newbcast, or a quad permute) and each lane updates its own rows
// below l.
template <int CTRL> __device__ __forceinline__ double2 dpp_d2(double2 v) {
  return double2{dpp_d<CTRL>(v.x), dpp_d<CTRL>(v.y)};
}
__device__ __forceinline__ double2 row_bcast(double2 v, int src) {
  switch (src) {   // (src is a constant where this is called)
    case 0: return dpp_d2<0x150>(v);
    case 1: return dpp_d2<0x151>(v);
    case 2: return dpp_d2<0x152>(v);
    case 3: return dpp_d2<0x153>(v);
    case 4: return dpp_d2<0x154>(v);
    case 5: return dpp_d2<0x155>(v);
    case 6: return dpp_d2<0x156>(v);
    case 7: return dpp_d2<0x157>(v);
    case 8: return dpp_d2<0x158>(v);
    case 9: return dpp_d2<0x159>(v);
    case 10: return dpp_d2<0x15A>(v);
    case 11: return dpp_d2<0x15B>(v);
    case 12: return dpp_d2<0x15C>(v);
    case 13: return dpp_d2<0x15D>(v);
    case 14: return dpp_d2<0x15E>(v);
    default: return dpp_d2<0x15F>(v);
  }
}
__device__ __forceinline__ double2 quad_bcast(double2 v, int src) {
  switch (src) {   // (src is a constant where this is called)
    case 0: return dpp_d2<0x00>(v);   // quad_perm [0,0,0,0]
    case 1: return dpp_d2<0x55>(v);   // quad_perm [1,1,1,1]
    case 2: return dpp_d2<0xAA>(v);   // quad_perm [2,2,2,2]
    default: return dpp_d2<0xFF>(v);  // quad_perm [3,3,3,3]
  }
}
constexpr int SWT = 256;   // threads per workgroup
// W: the largest block width kb it takes (32 or 64: one panel, or two
// panels taken as one block); STP: threads per column (16 where few columns
// are to be done and the work should spread over many workgroups, 4 where
// there are many and the per-workgroup set-up should be shared by more)
template <int W, int STP>
__global__ void __launch_bounds__(SWT) swap_trsm_kernel(double2* __restrict__ A, int N, int K, int k0, int kb, int cb,
                                                        int ce, const int* __restrict__ piv) {
  constexpr int NTH = SWT, STC = SWT / STP, STR = W / STP;   // threads, columns, rows per thread
  const int b = blockIdx.y;
  double2* M = A + (long long)b * N * N;
  __shared__ double2 L[W][W + 1];
  __shared__ int pv[W], Xs[2 * W], Ss[2 * W];
  const int tid = threadIdx.x, g = tid & (STP - 1);
  {
    // every load of L11 is issued before the first is used (kb^2 <= W^2)
    double2 lv[W * W / NTH];
#pragma unroll
    for (int q = 0; q < W * W / NTH; ++q) {
      const int t = tid + NTH * q, i = t / kb, l = t - i * kb;
      lv[q] = t < kb * kb ? M[(long long)(k0 + i) * N + k0 + l] : double2{0.0, 0.0};
    }
#pragma unroll
    for (int q = 0; q < W * W / NTH; ++q) {
      const int t = tid + NTH * q, i = t / kb, l = t - i * kb;
      if (t < kb * kb) L[i][l] = lv[q];
    }
  }
  if (tid < kb) pv[tid] = piv[(long long)b * K + k0 + tid];
  __syncthreads();
  // slot t < kb: block row k0 + t; slot kb + i: the pivot row of column k0 + i
  if (tid < 2 * kb) {
    const int X = tid < kb ? k0 + tid : pv[tid - kb];
    int src = X;
#pragma unroll
    for (int i = W - 1; i >= 0; --i) {
      if (i < kb) {
        const int pi = pv[i];
        src = src == k0 + i ? pi : (src == pi ? k0 + i : src);
      }
    }
    Xs[tid] = X;
    Ss[tid] = src;
  }
  __syncthreads();
  const int j = cb + blockIdx.x * STC + tid / STP;
  const bool live = j < ce;
  const int jc = live ? j : cb;   // (a column in range for the idle threads' addresses)
  double2 x[STR], y[STR];
#pragma unroll
  for (int m = 0; m < STR; ++m) {
    const int i = g + STP * m;
    x[m] = double2{0.0, 0.0};
    y[m] = double2{0.0, 0.0};
    if (live && i < kb) {
      x[m] = M[(long long)Ss[i] * N + jc];
      if (Xs[kb + i] >= k0 + kb) y[m] = M[(long long)Ss[kb + i] * N + jc];
    }
  }
  // every read of the column (by its 16 threads) completes before its
  // writes; a pivot row named by several columns gets the same value from
  // each slot
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < STR; ++m) {
    const int i = g + STP * m;
    if (live && i < kb && Xs[kb + i] >= k0 + kb && Ss[kb + i] != Xs[kb + i])
      M[(long long)Xs[kb + i] * N + jc] = y[m];
  }
#pragma clang loop unroll(full)
  for (int l = 0; l < W - 1; ++l) {
    if (l < kb) {
      const double2 xl = STP == 16 ? row_bcast(x[l / STP], l % STP) : quad_bcast(x[l / STP], l % STP);
      // (rows g + 16 m below l: m >= l / 16)
#pragma clang loop unroll(full)
      for (int m = l / STP; m < STR; ++m) {
        const int i = g + STP * m;
        if (i > l && i < kb) x[m] = csub_mul(x[m], L[i][l], xl);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < STR; ++m) {
    const int i = g + STP * m;
    if (live && i < kb) M[(long long)(k0 + i) * N + jc] = x[m];
  }
}

// Trailing update A22 -= L21 U12 over rows [k0 + kb, N) and columns [cb, ce)
// (kb <= 64 columns of the block, in chunks of 32) on the matrix cores (v_mfma_f64_16x16x4f64): 64 x 64
// output tiles, 4 wavefronts of 2 x 2 tiles of 16 x 16.  The complex
// product in two real ones that share the B operand: k-slot kk = (source
// pair offset h = kk / 2, part p = kk % 2) of l = 2 s + h for MFMA s,
//     B = part p of U12[l][col],
//     A_re = p = 0 ? Re L21[row][l] : -Im L21[row][l]  -> Re (L21 U12)
//     A_im = p = 0 ? Im L21[row][l] :  Re L21[row][l]  -> Im (L21 U12)
// L21 and U12 are staged through LDS; the tile of A22 is read before the
// products and written after them.
constexpr int UT = 64;
constexpr int ULP = PANEL + 1;   // L rows padded: the 16 rows of a read start on distinct banks
// One 64 x 64 tile of the update by 256 threads (Ls, Us: this tile's LDS);
// every thread of the workgroup calls it, live or not (it holds barriers).
template <int ROUNDS>
__device__ __forceinline__ void update_tile(double2* __restrict__ M, int N, int k0, int kb, int ce, int r0, int c0,
                                            bool live, double2* __restrict__ Ls, double2* __restrict__ Us, int tid) {
  typedef double d4v __attribute__((ext_vector_type(4)));
  const int l = tid & 63, wv = tid >> 6, wr = wv & 1, wc = wv >> 1;
  // this lane's outputs: tile (rt, ct), register e -> row (l / 16) + 4 e, column l % 16
  const int jj = l & 15, qrow = l >> 4;
  double2 cv[2][2][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = r0 + 32 * wr + 16 * rt + qrow + 4 * e, gc = c0 + 32 * wc + 16 * ct + jj;
        cv[rt][ct][e] = (live && gi < N && gc < ce) ? M[(long long)gi * N + gc] : double2{0.0, 0.0};
      }
  d4v dre[2][2], dim[2][2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      dre[rt][ct] = d4v{0, 0, 0, 0};
      dim[rt][ct] = d4v{0, 0, 0, 0};
    }
  const int kk = l >> 4, h = kk >> 1, p = kk & 1, i16 = l & 15;
  // the block's columns in chunks of PANEL through LDS
  for (int kc = 0; kc < kb; kc += PANEL) {
    const int kw = kb - kc < PANEL ? kb - kc : PANEL;
    if (kc > 0) __syncthreads();   // the previous chunk's reads precede this fill
    // (the loads of a round are all issued before its first LDS store, so
    // that they are in flight together; ROUNDS > 1 holds fewer registers)
    constexpr int PER = UT * PANEL / 256 / ROUNDS;
#pragma unroll
    for (int rd = 0; rd < ROUNDS; ++rd) {
      double2 lv[PER], uv[PER];
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int e = tid + 256 * (rd * PER + j);
        const int i = e / PANEL, ll = e - i * PANEL;   // L: row i, column ll
        const int gi = r0 + i;
        lv[j] = (live && gi < N && ll < kw) ? M[(long long)gi * N + k0 + kc + ll] : double2{0.0, 0.0};
        const int lu = e / UT, cc = e - lu * UT;       // U: row lu, column cc
        const int gc = c0 + cc;
        uv[j] = (live && gc < ce && lu < kw) ? M[(long long)(k0 + kc + lu) * N + gc] : double2{0.0, 0.0};
      }
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int e = tid + 256 * (rd * PER + j);
        const int i = e / PANEL, ll = e - i * PANEL;
        Ls[i * ULP + ll] = lv[j];
        const int lu = e / UT, cc = e - lu * UT;
        Us[lu * UT + cc] = uv[j];
      }
    }
    __syncthreads();
    if (live) {
      const int ns = (kw + 1) / 2;
      for (int s = 0; s < ns; ++s) {
        const int ll = 2 * s + h;
        double are[2], aim[2], bb[2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          const double2 Lv = Ls[(32 * wr + 16 * rt + i16) * ULP + ll];
          are[rt] = p == 0 ? Lv.x : -Lv.y;
          aim[rt] = p == 0 ? Lv.y : Lv.x;
        }
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const double2 Uv = Us[ll * UT + 32 * wc + 16 * ct + jj];
          bb[ct] = p == 0 ? Uv.x : Uv.y;
        }
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) {
            dre[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[rt], bb[ct], dre[rt][ct], 0, 0, 0);
            dim[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim[rt], bb[ct], dim[rt][ct], 0, 0, 0);
          }
      }
    }
  }
  if (!live) return;
  // (the tile's loads all complete here, once: the stores below sit in
  // conditional blocks, and a load still counted as pending at each block's
  // join would otherwise cost a wait for every store before it)
  __builtin_amdgcn_s_waitcnt(0);
  const bool full = r0 + UT <= N && c0 + UT <= ce;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = r0 + 32 * wr + 16 * rt + qrow + 4 * e, gc = c0 + 32 * wc + 16 * ct + jj;
        const double2 o{cv[rt][ct][e].x - dre[rt][ct][e], cv[rt][ct][e].y - dim[rt][ct][e]};
        if (full) {
          M[(long long)gi * N + gc] = o;
        } else if (gi < N && gc < ce) {
          M[(long long)gi * N + gc] = o;
        }
      }
}

__global__ void __launch_bounds__(256, 2) update_mfma_kernel(double2* __restrict__ A, int N, int k0, int kb, int cb,
                                                               int ce) {
  __shared__ double2 Ls[UT * ULP];     // [row][l]
  __shared__ double2 Us[PANEL * UT];   // [l][col]
  update_tile<1>(A + (long long)blockIdx.z * N * N, N, k0, kb, ce, k0 + kb + blockIdx.y * UT, cb + blockIdx.x * UT,
                 true, Ls, Us, threadIdx.x);
}

// The same update by a persistent grid for the far columns of the lookahead:
// workgroups of 512 threads, two halves of 256 with a tile each and LDS of
// their own (133 KB in all, so that a CU holds at most one workgroup).  With a
// grid of (CUs - 2 panel workgroups' worth) the update never occupies every
// CU, and the next block's panels and near-column kernels, whose workgroups
// each need a CU to themselves, start on the ones it leaves instead of
// waiting for it to drain.  A tile's work is a sequence of phases, for each
// chunk of 32 block columns a load phase (the chunk of L21 and U12 into LDS,
// with the tile of A22 into registers before the first) and a product phase
// (the matrix-core products; the tile's stores after the last).  The second
// half runs its sequence one phase behind the first, with a barrier after
// every phase, so that while one half waits for its loads the other keeps the
// matrix cores busy.  Each half walks tiles 2 (blockIdx.x + i gridDim.x) +
// half, matrix-major, row tile, then column tile.
__global__ void __launch_bounds__(512) update_persist_kernel(double2* __restrict__ A, int N, int k0, int kb, int cb,
                                                             int ce, int nrt, int nct, int T) {
  typedef double d4v __attribute__((ext_vector_type(4)));
  __shared__ double2 Lsh[2][UT * ULP];
  __shared__ double2 Ush[2][PANEL * UT];
  const int half = threadIdx.x >> 8, tid = threadIdx.x & 255;
  double2* Ls = Lsh[half];
  double2* Us = Ush[half];
  const int l = tid & 63, wv = tid >> 6, wr = wv & 1, wc = wv >> 1;
  const int jj = l & 15, qrow = l >> 4;
  const int kk = l >> 4, h = kk >> 1, p = kk & 1, i16 = l & 15;
  const int ntiles = nct * nrt * T, npairs = (ntiles + 1) / 2;
  const int nch = (kb + PANEL - 1) / PANEL;
  const int ntile_half = blockIdx.x < npairs ? (npairs - (int)blockIdx.x + (int)gridDim.x - 1) / (int)gridDim.x : 0;
  const int nphase = 2 * nch * ntile_half;
  double2 cv[2][2][4];
  d4v dre[2][2], dim[2][2];
  // (the same count of steps, and so of barriers, in both halves)
  for (int step = 0; step <= nphase; ++step) {
    const int ph = step - half;   // this half's phase
    if (ph >= 0 && ph < nphase) {
      const int i = ph / (2 * nch), w = ph - i * (2 * nch), c = w >> 1;
      const int t = 2 * ((int)blockIdx.x + i * (int)gridDim.x) + half;
      const bool live = t < ntiles;
      const int tt = live ? t : 0;
      const int ct = tt % nct, rtl = (tt / nct) % nrt, b = tt / (nct * nrt);
      double2* M = A + (long long)b * N * N;
      const int r0 = k0 + kb + rtl * UT, c0 = cb + ct * UT;
      const int kc = c * PANEL, kw = kb - kc < PANEL ? kb - kc : PANEL;
      if ((w & 1) == 0) {
        // load phase
        if (c == 0) {
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct2 = 0; ct2 < 2; ++ct2) {
              dre[rt][ct2] = d4v{0, 0, 0, 0};
              dim[rt][ct2] = d4v{0, 0, 0, 0};
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int gi = r0 + 32 * wr + 16 * rt + qrow + 4 * e, gc = c0 + 32 * wc + 16 * ct2 + jj;
                cv[rt][ct2][e] = (live && gi < N && gc < ce) ? M[(long long)gi * N + gc] : double2{0.0, 0.0};
              }
            }
        }
        constexpr int ROUNDS = 2, PER = UT * PANEL / 256 / ROUNDS;
#pragma unroll
        for (int rd = 0; rd < ROUNDS; ++rd) {
          double2 lv[PER], uv[PER];
#pragma unroll
          for (int j = 0; j < PER; ++j) {
            const int e = tid + 256 * (rd * PER + j);
            const int ii = e / PANEL, ll = e - ii * PANEL;
            const int gi = r0 + ii;
            lv[j] = (live && gi < N && ll < kw) ? M[(long long)gi * N + k0 + kc + ll] : double2{0.0, 0.0};
            const int lu = e / UT, cc = e - lu * UT;
            const int gc = c0 + cc;
            uv[j] = (live && gc < ce && lu < kw) ? M[(long long)(k0 + kc + lu) * N + gc] : double2{0.0, 0.0};
          }
#pragma unroll
          for (int j = 0; j < PER; ++j) {
            const int e = tid + 256 * (rd * PER + j);
            const int ii = e / PANEL, ll = e - ii * PANEL;
            Ls[ii * ULP + ll] = lv[j];
            const int lu = e / UT, cc = e - lu * UT;
            Us[lu * UT + cc] = uv[j];
          }
        }
      } else if (live) {
        // product phase
        const int ns = (kw + 1) / 2;
        for (int s2 = 0; s2 < ns; ++s2) {
          const int ll = 2 * s2 + h;
          double are[2], aim[2], bb[2];
#pragma unroll
          for (int rt = 0; rt < 2; ++rt) {
            const double2 Lv = Ls[(32 * wr + 16 * rt + i16) * ULP + ll];
            are[rt] = p == 0 ? Lv.x : -Lv.y;
            aim[rt] = p == 0 ? Lv.y : Lv.x;
          }
#pragma unroll
          for (int ct2 = 0; ct2 < 2; ++ct2) {
            const double2 Uv = Us[ll * UT + 32 * wc + 16 * ct2 + jj];
            bb[ct2] = p == 0 ? Uv.x : Uv.y;
          }
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct2 = 0; ct2 < 2; ++ct2) {
              dre[rt][ct2] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[rt], bb[ct2], dre[rt][ct2], 0, 0, 0);
              dim[rt][ct2] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim[rt], bb[ct2], dim[rt][ct2], 0, 0, 0);
            }
        }
        if (c == nch - 1) {
          __builtin_amdgcn_s_waitcnt(0);   // (once, not at every conditional store below)
          const bool full = r0 + UT <= N && c0 + UT <= ce;
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct2 = 0; ct2 < 2; ++ct2)
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int gi = r0 + 32 * wr + 16 * rt + qrow + 4 * e, gc = c0 + 32 * wc + 16 * ct2 + jj;
                const double2 o{cv[rt][ct2][e].x - dre[rt][ct2][e], cv[rt][ct2][e].y - dim[rt][ct2][e]};
                if (full) {
                  M[(long long)gi * N + gc] = o;
                } else if (gi < N && gc < ce) {
                  M[(long long)gi * N + gc] = o;
                }
              }
        }
      }
    }
    __syncthreads();
  }
}

// A1[t] = [[Z_int,int, Z_int,eq], [Z_eq,int, Z_eq,eq]] from Z[t] = [[Z_eq,eq, ...]]
__global__ void interior_first_kernel(const double2* __restrict__ Z, int n, int m, int T,
                                      double2* __restrict__ A) {
  const int N = n + m;
  const long long total = (long long)T * N * N;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long t = e / ((long long)N * N);
    const int r = (int)(e - t * N * N);
    const int i = r / N, j = r - i * N;
    const int si = i < m ? n + i : i - m;
    const int sj = j < m ? n + j : j - m;
    A[e] = Z[t * N * N + (long long)si * N + sj];
  }
}

// A2[t] = [[Zt[t] + Z_self, I], [I, 0]] (2n x 2n), Zt read from the trailing
// block of A1 (row stride N1, offset m)
__global__ void inverse_setup_kernel(const double2* __restrict__ A1, int N1, int m, const double2* __restrict__ Zself,
                                     int n, int T, double2* __restrict__ A2) {
  const int N2 = 2 * n;
  const long long total = (long long)T * N2 * N2;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long t = e / ((long long)N2 * N2);
    const int r = (int)(e - t * N2 * N2);
    const int i = r / N2, j = r - i * N2;
    double2 v{0.0, 0.0};
    if (i < n && j < n) {
      v = A1[t * N1 * N1 + (long long)(m + i) * N1 + (m + j)];
      if (Zself) {
        const double2 s = Zself[(long long)i * n + j];
        v.x += s.x;
        v.y += s.y;
      }
    } else if ((i < n && j == i + n) || (i >= n && j == i - n)) {
      v = double2{1.0, 0.0};
    }
    A2[e] = v;
  }
}

// out[t][i][j] = A[t][off + i][off + j] (trailing n x n block)
__global__ void trailing_copy_kernel(const double2* __restrict__ A, int N, int off, int n, int T,
                                     double2* __restrict__ out) {
  const long long total = (long long)T * n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long t = e / ((long long)n * n);
    const int r = (int)(e - t * n * n);
    const int i = r / n, j = r - i * n;
    out[e] = A[t * N * N + (long long)(off + i) * N + (off + j)];
  }
}

unsigned grid1(long long total) {
  long long g = (total + 255) / 256;
  if (g > 65536LL * 4) g = 65536LL * 4;
  return (unsigned)(g < 1 ? 1 : g);
}

// A second stream per device for the lookahead of the elimination below,
// created once (default priority, non-blocking) and kept until the process
// ends; calls that share it only queue behind each other on it, each with
// events of its own.
hipStream_t lookahead_stream() {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  EMS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams.find(dev);
  if (it != streams.end()) return it->second;
  hipStream_t a = nullptr;
  EMS_HIP(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
  streams[dev] = a;
  return a;
}

struct EventPair {
  hipEvent_t panel = nullptr, rest = nullptr;
  EventPair() {
    EMS_HIP(hipEventCreateWithFlags(&panel, hipEventDisableTiming));
    EMS_HIP(hipEventCreateWithFlags(&rest, hipEventDisableTiming));
  }
  ~EventPair() {
    if (panel) (void)hipEventDestroy(panel);
    if (rest) (void)hipEventDestroy(rest);
  }
  EventPair(const EventPair&) = delete;
  EventPair& operator=(const EventPair&) = delete;
};

// Leading K x K elimination of T matrices N x N at A (see the file header),
// in blocks of two panels (one where the panel kernel cannot hold the rows):
// the block's first panel, then the second panel's columns take its swaps,
// U12 and update, then the second panel (whose swaps also reach the first
// panel's columns), and the columns right of the block take the block's
// swaps, U12 = L11^-1 A12 with its 64 x 64 unit lower L11 and one rank-64
// update.  Lookahead of one block: the next block's columns are updated on
// the caller's stream and the next block starts at once, while the columns
// beyond are updated on a second stream (their update, the largest kernel of
// the step, runs beside the next block's panels, which hold one workgroup
// per matrix).  Before it touches those columns the caller's stream waits
// for the second one.  On return all work is on the caller's stream.
void eliminate(double2* A, int N, int K, int T, int* piv, int* info, hipStream_t s) {
  hipStream_t aux = lookahead_stream();
  EventPair ev;
  bool rest_pending = false;
  int cus = 0, dev = 0;
  EMS_HIP(hipGetDevice(&dev));
  EMS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  // far columns: a persistent grid that leaves 2 T CUs free, the panels'
  // and as many again for the near columns' kernels that run beside it
  const int persist_grid = (T <= 64 && cus - 2 * T >= 64) ? cus - 2 * T : 0;
  auto panel = [&](int k0, int kb, int lw, int rw, hipEvent_t stop) {
    const int rows = N - k0;
    const uint32_t shm = (uint32_t)((size_t)rows * PSB * sizeof(double2));
    // (the sub-block staging holds rows * PSB values in LDS; one row per
    // thread: 512 threads up to 512 rows, 1024 beyond, where the larger
    // workgroup beat 768 threads and 512 with two rows each)
    if (rows <= 512)
      hipExtLaunchKernelGGL((panel_reg_kernel<512, 1>), dim3((unsigned)T), dim3(512), shm, s, nullptr, stop, 0u, A, N,
                            K, k0, kb, lw, rw, piv, info);
    else if (rows <= 1024)
      hipExtLaunchKernelGGL((panel_reg_kernel<1024, 1>), dim3((unsigned)T), dim3(1024), shm, s, nullptr, stop, 0u, A, N,
                            K, k0, kb, lw, rw, piv, info);
    else   // (lw == rw == 0 here: blocks of one panel)
      hipExtLaunchKernelGGL(panel_kernel, dim3((unsigned)T), dim3(512), 0u, s, nullptr, stop, 0u, A, N, K, k0, kb, piv, info);
  };
  auto swap_trsm = [&](hipStream_t st, int k0, int kb, int cb, int ce) {
    // (16 lanes per column up to 128 columns, 4 beyond)
    const bool few = ce - cb <= 128;
    const int stc = few ? SWT / 16 : SWT / 4;
    const dim3 grid((unsigned)((ce - cb + stc - 1) / stc), (unsigned)T);
    if (kb <= PANEL && few)
      hipLaunchKernelGGL((swap_trsm_kernel<PANEL, 16>), grid, dim3(SWT), 0, st, A, N, K, k0, kb, cb, ce, piv);
    else if (kb <= PANEL)
      hipLaunchKernelGGL((swap_trsm_kernel<PANEL, 4>), grid, dim3(SWT), 0, st, A, N, K, k0, kb, cb, ce, piv);
    else if (few)
      hipLaunchKernelGGL((swap_trsm_kernel<2 * PANEL, 16>), grid, dim3(SWT), 0, st, A, N, K, k0, kb, cb, ce, piv);
    else
      hipLaunchKernelGGL((swap_trsm_kernel<2 * PANEL, 4>), grid, dim3(SWT), 0, st, A, N, K, k0, kb, cb, ce, piv);
  };
  auto update = [&](hipStream_t st, int k0, int kb, int cb, int ce, bool far, hipEvent_t stop) {
    const int rt = (N - k0 - kb + UT - 1) / UT, ct = (ce - cb + UT - 1) / UT;
    const long long pairs = ((long long)rt * ct * T + 1) / 2;
    if (far && persist_grid > 0)
      hipExtLaunchKernelGGL(update_persist_kernel, dim3((unsigned)(pairs < persist_grid ? pairs : persist_grid)),
                            dim3(512), 0u, st, nullptr, stop, 0u, A, N, k0, kb, cb, ce, rt, ct, T);
    else
      hipExtLaunchKernelGGL(update_mfma_kernel, dim3((unsigned)ct, (unsigned)rt, (unsigned)T), dim3(256), 0u, st, nullptr,
                            stop, 0u, A, N, k0, kb, cb, ce);
  };
  auto block_width = [&](int k0) {
    const int w = N - k0 <= 1024 ? 2 * PANEL : PANEL;
    return K - k0 < w ? K - k0 : w;
  };
  for (int k0 = 0; k0 < K;) {
    const int ob = block_width(k0), ka = ob < PANEL ? ob : PANEL;
    const int c1 = k0 + ob;
    const int nb = c1 < K ? block_width(c1) : 0;   // width of the next block (0 after the last)
    const int c2 = nb > 0 ? c1 + nb : N;
    // the far columns [c2, N) go to the second stream, after this block's
    // panels (and, in its own order, after the previous step's far columns)
    const bool far = c1 < N && c2 < N;
    // the first panel also takes the second panel's columns through its
    // swaps, U rows and in-panel updates; the second panel's swaps also
    // reach the first panel's columns.  The events between the streams
    // complete with the kernels before them (extended launches with a stop
    // event), so that the caller's stream carries no marker of its own
    panel(k0, ka, 0, ob - ka, far && ob == ka ? ev.panel : nullptr);
    if (ob > ka) panel(k0 + ka, ob - ka, ka, 0, far ? ev.panel : nullptr);
    EMS_LAUNCH_CHECK();
    if (c1 >= N) break;   // (no trailing columns: K == N)
    // the previous step's far columns, [c1, N), are final on the second stream
    if (rest_pending) EMS_HIP(hipStreamWaitEvent(s, ev.rest, 0));
    rest_pending = false;
    if (far) {
      EMS_HIP(hipStreamWaitEvent(aux, ev.panel, 0));
      swap_trsm(aux, k0, ob, c2, N);
    }
    swap_trsm(s, k0, ob, c1, c2);
    update(s, k0, ob, c1, c2, false, nullptr);
    EMS_LAUNCH_CHECK();
    if (far) {
      // the far update follows the far swap at once and runs beside the near
      // columns' update and the next block's panels (its persistent grid
      // leaves them CUs); waiting for the near update as well took an event
      // on the caller's stream per block, which cost more than the near
      // update gains from having the device to itself
      update(aux, k0, ob, c2, N, true, ev.rest);
      EMS_LAUNCH_CHECK();
      rest_pending = true;
    }
    k0 = c1;
  }
  if (rest_pending) EMS_HIP(hipStreamWaitEvent(s, ev.rest, 0));
}

}  // namespace

void schur_eliminate(double2* A, int N, int K, int T, int* piv, int* info, hipStream_t s) {
  eliminate(A, N, K, T, piv, info, s);
}

}  // namespace emsurf

using namespace emsurf;

extern "C" emsurf_status emsurf_macromodels(int32_t n_types, int32_t n_eq, int32_t n_int, const void* Z_dev,
                                            const void* Zself_dev, void* S_dev, void* Zt_dev, void* stream) {
  try {
    EMS_CHECK_ARG(n_types >= 1 && n_types <= 4096, "n_types must be in [1, 4096]");
    EMS_CHECK_ARG(n_eq >= 1 && n_eq <= 512, "n_eq must be in [1, 512]");
    EMS_CHECK_ARG(n_int >= 0 && n_int <= 4096, "n_int must be in [0, 4096]");
    EMS_CHECK_ARG(Z_dev != nullptr && S_dev != nullptr, "Z_dev and S_dev must be non-NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int n = n_eq, m = n_int, N1 = n + m, N2 = 2 * n, T = n_types;
    // one allocation for the call: A1, A2, the pivots, and the two steps'
    // singular flags (kept apart, read once at the end)
    const int Kmax = m > n ? m : n;
    const size_t b_a1 = (size_t)T * N1 * N1 * 16, b_a2 = (size_t)T * N2 * N2 * 16;
    const size_t b_piv = ((size_t)T * (Kmax > 0 ? Kmax : 1) * 4 + 255) / 256 * 256;
    DevBuf ws(b_a1 + b_a2 + b_piv + (size_t)2 * T * 4);
    double2* A1 = static_cast<double2*>(ws.p);
    double2* A2 = reinterpret_cast<double2*>(static_cast<char*>(ws.p) + b_a1);
    int* piv = reinterpret_cast<int*>(static_cast<char*>(ws.p) + b_a1 + b_a2);
    int* info = piv + b_piv / 4;   // [2][T]
    EMS_HIP(hipMemsetAsync(info, 0, (size_t)2 * T * 4, s));
    hipLaunchKernelGGL(interior_first_kernel, dim3(grid1((long long)T * N1 * N1)), dim3(256), 0, s,
                       static_cast<const double2*>(Z_dev), n, m, T, A1);
    EMS_LAUNCH_CHECK();
    if (m > 0) eliminate(A1, N1, m, T, piv, info, s);
    if (Zt_dev) {
      hipLaunchKernelGGL(trailing_copy_kernel, dim3(grid1((long long)T * n * n)), dim3(256), 0, s, A1, N1, m, n, T,
                         static_cast<double2*>(Zt_dev));
      EMS_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(inverse_setup_kernel, dim3(grid1((long long)T * N2 * N2)), dim3(256), 0, s, A1, N1, m,
                       static_cast<const double2*>(Zself_dev), n, T, A2);
    EMS_LAUNCH_CHECK();
    eliminate(A2, N2, n, T, piv, info + T, s);
    hipLaunchKernelGGL(trailing_copy_kernel, dim3(grid1((long long)T * n * n)), dim3(256), 0, s, A2, N2, n, n, T,
                       static_cast<double2*>(S_dev));
    EMS_LAUNCH_CHECK();
    std::vector<int> flags(2 * (size_t)T);
    EMS_HIP(hipMemcpyAsync(flags.data(), info, (size_t)2 * T * 4, hipMemcpyDeviceToHost, s));
    EMS_HIP(hipStreamSynchronize(s));
    const int* info1 = flags.data();
    const int* info2 = flags.data() + T;
    for (int t = 0; t < T; ++t) {
      if (info1[t]) {
        set_error("cell type " + std::to_string(t) + ": interior block Z_int,int is singular");
        throw Err{EMSURF_ERR_ARG};
      }
      if (info2[t]) {
        set_error("cell type " + std::to_string(t) + ": Z~ + Z_self is singular");
        throw Err{EMSURF_ERR_ARG};
      }
    }
    return EMSURF_OK;
  } catch (...) {
    return current_exception_status();
  }
}
