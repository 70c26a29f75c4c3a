// Plan-time kernels: circulant embedding of the coupling blocks (Sec. IV-B,
// eq. (LJV3): block T(d) goes to padded slot d mod L on each lattice axis, all
// other slots stay zero), the synthetic point-sampled coupling fills (dense
// blocks, or the L and K operators of the structured form), and the
// scatter of transformed kernel columns into the resident Fourier-domain
// store (FP64 and/or FP32 rounded to nearest).
//
// The padded kernel chunk holds columns c in [c0, c0 + nc) of the per-frequency
// batch, c = v*n + u (source v, test u) for dense blocks and
// c = v*n + part*n_h + u for the structured form (the stacked n x n_h matrix
// [L; K], part 0 = L, 1 = K), as a dense [Ly][Lx][nc] array, so that after the
// 2-D transform every frequency's record is stored column-major.
#include "internal.h"
#include "green.h"

namespace emsurf {
namespace {

// Caller blocks hold `parts` square nb x nb matrices per offset, row-major
// (row = test, column = source): parts = 1, nb = n_eq for dense blocks;
// parts = 2 (L then K), nb = n_h for the structured operator.  The kernel
// columns are those of the stacked (parts * nb) x nb matrix, column-major:
// c = v * (parts * nb) + part * nb + u.
__global__ void pad_blocks_kernel(const double2* __restrict__ Tb, int nx, int ny, int nb, int parts, int Lx, int Ly,
                                  long long c0, long long nc, int vperm, double2* __restrict__ K) {
  const long long total = (long long)Ly * Lx * nc;
  const long long nbb = (long long)nb * nb;
  // 32-bit index arithmetic: a chunk holds fewer than 2^31 entries (host check)
  const int ncc = (int)nc;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < (int)total; i += gridDim.x * blockDim.x) {
    const int sxy = i / ncc, j = i - sxy * ncc;
    const int sy = sxy / Lx, sx = sxy - sy * Lx;
    bool okx, oky;
    const int dx = slot_to_offset(sx, Lx, nx, &okx);
    const int dy = slot_to_offset(sy, Ly, ny, &oky);
    double2 val{0.0, 0.0};
    if (okx && oky) {
      const int c = (int)c0 + j;
      const int rows = parts * nb;
      const int vp = c / rows;
      const int w = c - vp * rows;
      const int part = w / nb, u = w - part * nb;
      const int v = vperm ? pair_fill_v(vp, nb) : vp;
      const long long blk = (long long)(dy + ny - 1) * (2 * nx - 1) + (dx + nx - 1);
      val = Tb[(blk * parts + part) * nbb + (long long)u * nb + v];
    }
    K[i] = val;
  }
}

// Structured fill (outer EFIE/MFIE operators, Sec. III-B), local index 2p + a:
//   part 0: L = A_q t_pa . (I + grad grad / k^2) g(R) . t_qb
//   part 1: K = A_q t_pa . (grad g(R) x t_qb)
// with R = rho_p - rho_q + pitch (dx, dy, 0) and g = exp(-jkR)/(4 pi R); the
// radial derivatives g' = -(jk + 1/R) g and g'' = ((jk + 1/R)^2 + 1/R^2) g
// give grad g = g' Rhat and grad grad g = g'' Rhat Rhat + (g'/R)(I - Rhat Rhat).
__device__ __forceinline__ double2 lk_entry(const double* __restrict__ rho, const double* __restrict__ area,
                                            const double* __restrict__ tan, double pitch, double k, int dx,
                                            int dy, int part, int u, int v) {
  if (dx == 0 && dy == 0) return double2{0.0, 0.0};
  const int p = u >> 1, a = u & 1, q = v >> 1, b = v & 1;
  const double* tp = tan + (p * 2 + a) * 3;
  const double* tq = tan + (q * 2 + b) * 3;
  const double ex = rho[3 * p + 0] - rho[3 * q + 0] + pitch * dx;
  const double ey = rho[3 * p + 1] - rho[3 * q + 1] + pitch * dy;
  const double ez = rho[3 * p + 2] - rho[3 * q + 2];
  const double R = sqrt(ex * ex + ey * ey + ez * ez);
  const double iR = 1.0 / R;
  const double hx = ex * iR, hy = ey * iR, hz = ez * iR;
  double sn, cs;
  sincos(k * R, &sn, &cs);
  const double g0 = iR / (4.0 * 3.14159265358979323846);
  const double gr = g0 * cs, gi = -g0 * sn;                         // g
  // g' = -(1/R + jk) g
  const double g1r = -(iR * gr - k * gi), g1i = -(iR * gi + k * gr);
  const double Aq = area[q];
  if (part == 1) {
    // t_p . (Rhat x t_q)
    const double cx = hy * tq[2] - hz * tq[1], cy = hz * tq[0] - hx * tq[2], cz = hx * tq[1] - hy * tq[0];
    const double trip = tp[0] * cx + tp[1] * cy + tp[2] * cz;
    return double2{Aq * trip * g1r, Aq * trip * g1i};
  }
  // g'' = ((1/R + jk)^2 + 1/R^2) g = (2/R^2 - k^2 + 2jk/R) g
  const double wr = 2.0 * iR * iR - k * k, wi = 2.0 * k * iR;
  const double g2r = wr * gr - wi * gi, g2i = wr * gi + wi * gr;
  const double ik2 = 1.0 / (k * k);
  const double isor = gr + g1r * iR * ik2, isoi = gi + g1i * iR * ik2;     // g + g'/(k^2 R)
  const double radr = (g2r - g1r * iR) * ik2, radi = (g2i - g1i * iR) * ik2;  // (g'' - g'/R)/k^2
  const double tt = tp[0] * tq[0] + tp[1] * tq[1] + tp[2] * tq[2];
  const double pr = (tp[0] * hx + tp[1] * hy + tp[2] * hz) * (tq[0] * hx + tq[1] * hy + tq[2] * hz);
  return double2{Aq * (isor * tt + radr * pr), Aq * (isoi * tt + radi * pr)};
}

// Green fill of one chunk of kernel columns [c0, c0 + nc).  Work item
// (lattice slot, column, patch p): the entries of rows u = 2 p + a (J) and
// 2 P + 2 p + a (M), a = 0, 1, share R and exp(-jkR) (only the half with the
// column's own current type is nonzero), so a thread evaluates the Green's
// function once and writes its 4 entries, two adjacent pairs, coalesced over
// p.  The value of each entry is green_entry's.
__global__ void green_padded_kernel(const double* __restrict__ rho, const double* __restrict__ area,
                                    const double* __restrict__ tan, int P, double pitch, double k, int nx, int ny,
                                    int Lx, int Ly, long long c0, long long nc, int vperm,
                                    double2* __restrict__ K) {
  const int n = 4 * P;
  const int cb = (int)c0, ce = (int)(c0 + nc);   // host: fits 31 bits
  const int vpa = cb / n, ncol = (ce - 1) / n - vpa + 1;
  const int total = Lx * Ly * ncol * P;        // host: fits 31 bits
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int p = i % P, rest = i / P;
    const int cl = rest % ncol, sxy = rest / ncol;
    const int sy = sxy / Lx, sx = sxy - sy * Lx;
    const int vp = vpa + cl;
    const int v = vperm ? pair_fill_v(vp, n) : vp;
    bool okx, oky;
    const int dx = slot_to_offset(sx, Lx, nx, &okx);
    const int dy = slot_to_offset(sy, Ly, ny, &oky);
    double2 e[2][2] = {{{0.0, 0.0}, {0.0, 0.0}}, {{0.0, 0.0}, {0.0, 0.0}}};   // [current type][a]
    const int hv = v / (2 * P), lv = v - hv * 2 * P;
    const int q = lv >> 1, b = lv & 1;
    if (okx && oky && !(dx == 0 && dy == 0)) {
      const double* tq = tan + (q * 2 + b) * 3;
      double dots[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const double* tp = tan + (p * 2 + a) * 3;
        dots[a] = tp[0] * tq[0] + tp[1] * tq[1] + tp[2] * tq[2];
      }
      if (dots[0] != 0.0 || dots[1] != 0.0) {
        const double ex = rho[3 * p + 0] - rho[3 * q + 0] + pitch * dx;
        const double ey = rho[3 * p + 1] - rho[3 * q + 1] + pitch * dy;
        const double ez = rho[3 * p + 2] - rho[3 * q + 2];
        const double R = sqrt(ex * ex + ey * ey + ez * ez);
        const double2 gq = area_green(R, area[q], k);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          if (dots[a] != 0.0) e[hv][a] = double2{dots[a] * gq.x, dots[a] * gq.y};
        }
      }
    }
    const long long kb = (long long)sxy * nc - c0;   // K index of column index c: kb + c
    const int c_u0 = vp * n;                          // column index of (u = 0, this v)
#pragma unroll
    for (int hu = 0; hu < 2; ++hu)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int c = c_u0 + hu * 2 * P + 2 * p + a;
        if (c >= cb && c < ce) K[kb + c] = e[hu][a];
      }
  }
}

__global__ void green_blocks_kernel(const double* __restrict__ rho, const double* __restrict__ area,
                                    const double* __restrict__ tan, int P, double pitch, double k, int nx, int ny,
                                    double2* __restrict__ Tb) {
  const int n = 4 * P;
  const long long total = (long long)(2 * ny - 1) * (2 * nx - 1) * n * n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long nn = (long long)n * n;
    const long long blk = i / nn;
    const int rem = (int)(i - blk * nn);
    const int u = rem / n, v = rem - u * n;
    const int dx = (int)(blk % (2 * nx - 1)) - (nx - 1);
    const int dy = (int)(blk / (2 * nx - 1)) - (ny - 1);
    Tb[i] = green_entry(rho, area, tan, P, pitch, k, dx, dy, u, v);
  }
}

__global__ void lk_padded_kernel(const double* __restrict__ rho, const double* __restrict__ area,
                                 const double* __restrict__ tan, int P, double pitch, double k, int nx, int ny,
                                 int Lx, int Ly, long long c0, long long nc, double2* __restrict__ K) {
  const int nh = 2 * P;
  const long long total = (long long)Ly * Lx * nc;
  // 32-bit index arithmetic: a chunk holds fewer than 2^31 entries (host check)
  const int ncc = (int)nc;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < (int)total; i += gridDim.x * blockDim.x) {
    const int sxy = i / ncc, j = i - sxy * ncc;
    const int sy = sxy / Lx, sx = sxy - sy * Lx;
    bool okx, oky;
    const int dx = slot_to_offset(sx, Lx, nx, &okx);
    const int dy = slot_to_offset(sy, Ly, ny, &oky);
    double2 val{0.0, 0.0};
    if (okx && oky) {
      const int c = (int)c0 + j;
      const int v = c / (2 * nh);
      const int w = c - v * 2 * nh;
      const int part = w / nh, u = w - part * nh;
      val = lk_entry(rho, area, tan, pitch, k, dx, dy, part, u, v);
    }
    K[i] = val;
  }
}

__global__ void lk_blocks_kernel(const double* __restrict__ rho, const double* __restrict__ area,
                                 const double* __restrict__ tan, int P, double pitch, double k, int nx, int ny,
                                 double2* __restrict__ Tb) {
  const int nh = 2 * P;
  const long long nhh = (long long)nh * nh;
  const long long total = (long long)(2 * ny - 1) * (2 * nx - 1) * 2 * nhh;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long blk = i / (2 * nhh);
    const long long r2 = i - blk * 2 * nhh;
    const int part = (int)(r2 / nhh);
    const int rem = (int)(r2 - part * nhh);
    const int u = rem / nh, v = rem - u * nh;
    const int dx = (int)(blk % (2 * nx - 1)) - (nx - 1);
    const int dy = (int)(blk / (2 * nx - 1)) - (ny - 1);
    Tb[i] = lk_entry(rho, area, tan, pitch, k, dx, dy, part, u, v);
  }
}

__global__ void store_chunk_kernel(const double2* __restrict__ Kc, long long P, long long nn, long long c0,
                                   long long nc, const int* __restrict__ slot_of, int n, int nh, int vperm,
                                   int uperm, double2* __restrict__ t64, float2* __restrict__ t32,
                                   __bf16* __restrict__ t16) {
  const long long total = P * nc;
  const long long blk = nh > 0 ? lkpair_block_entries(nh) : pair_block_entries(n);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long kf = i / nc, j = i - kf * nc;
    if (!slot_of) {
      // output-ordered: column c0 + j of the store; with the Green row order its
      // value sits at the row's position in the same column of the chunk
      const long long dst = kf * nn + c0 + j;
      double2 v;
      if (uperm) {
        const long long col = c0 + j;
        const int cv = (int)(col / n), u = (int)(col - (long long)cv * n);
        v = Kc[kf * nc + (long long)cv * n + green_fill_up(u, n / 4) - c0];
      } else {
        v = Kc[i];
      }
      if (t64) t64[dst] = v;
      if (t32) t32[dst] = float2{(float)v.x, (float)v.y};
      if (t16) {
        // split of the FP32-rounded entry: hi = bf16(a), lo = bf16(a - hi),
        // both round to nearest even (a - hi is exact in FP32)
        const long long col = c0 + j;
        const int cv = (int)(col / n), u = (int)(col - (long long)cv * n);
        __bf16* hi = t16 + kf * 4 * nn;
        __bf16* lo = hi + 2 * nn;
        const float parts[2] = {(float)v.x, (float)v.y};
        for (int pp = 0; pp < 2; ++pp) {
          const __bf16 hv = (__bf16)parts[pp];
          const long long o = bf16_offset(n, u, cv, pp);
          hi[o] = hv;
          lo[o] = (__bf16)(parts[pp] - (float)hv);
        }
      }
      continue;
    }
    const double2 v = Kc[i];
    const long long slot = slot_of[kf];
    if (slot < 0) continue;
    const long long col = c0 + j;
    int u, cv, half = 0;
    if (nh > 0) {
      // structured record: column v (2 n_h) + half n_h + u
      cv = (int)(col / (2 * nh));
      const int rem = (int)(col - (long long)cv * 2 * nh);
      half = rem / nh;
      u = rem - half * nh;
    } else {
      cv = (int)(col / n);
      u = (int)(col - (long long)cv * n);
      if (vperm) cv = pair_fill_v(cv, n);
      if (uperm) u = green_fill_u(u, n / 4);
    }
    if (t64) {
      double* d = reinterpret_cast<double*>(t64) + slot * blk * 2;
      d[nh > 0 ? lkpair_value_offset(nh, u, cv, half, 0, 2) : pair_value_offset(n, u, cv, 0, 2)] = v.x;
      d[nh > 0 ? lkpair_value_offset(nh, u, cv, half, 1, 2) : pair_value_offset(n, u, cv, 1, 2)] = v.y;
    }
    if (t32) {
      float* f = reinterpret_cast<float*>(t32) + slot * blk * 2;
      f[nh > 0 ? lkpair_value_offset(nh, u, cv, half, 0, 4) : pair_value_offset(n, u, cv, 0, 4)] = (float)v.x;
      f[nh > 0 ? lkpair_value_offset(nh, u, cv, half, 1, 4) : pair_value_offset(n, u, cv, 1, 4)] = (float)v.y;
    }
  }
}

// Dense reciprocal store of one chunk filled in the pair_fill_v order (c0 and
// the chunk width are multiples of 4 n_eq columns, or the chunk ends the
// block).  Work item (stored pair slot, quad of 4 column positions, u), the
// slot's frequency from the pair list (k, -k): the 4
// positions of a quad of a full group of 8 are v, v + 2, v + 4, v + 6, whose
// values of one part are one 16-byte piece of an FP32 tile (two of an FP64
// tile), written whole; consecutive u write consecutive pieces.  Quads at a
// ragged edge write their values one by one.
__global__ void store_pair_chunk_kernel(const double2* __restrict__ Kc, int Ps, int c0, int nc, int nq,
                                        const int* __restrict__ pairs, int n, int uperm, double* __restrict__ t64,
                                        float* __restrict__ t32) {
  const int total = Ps * nq * n;   // host: fits 31 bits
  const long long blk2 = 2LL * pair_block_entries(n);   // reals per stored block
  const int pos0 = c0 / n, pend = (c0 + nc) / n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int u = i % n, rest = i / n;
    const int qd = rest % nq, slot = rest / nq;
    const int kf = pairs[2 * slot];
    const int vp0 = pos0 + 4 * qd;
    const int cnt = pend - vp0 < 4 ? pend - vp0 : 4;
    int v[4];
    double2 x[4];
    const int up = uperm ? green_fill_up(u, n / 4) : u;   // position of row u in its column
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[j] = j < cnt ? pair_fill_v(vp0 + j, n) : 0;
      x[j] = j < cnt ? Kc[(long long)kf * nc + (long long)(vp0 + j - pos0) * n + up] : double2{0.0, 0.0};
    }
    const bool whole = cnt == 4 && (v[0] & 6) == 0 && v[1] == v[0] + 2 && v[2] == v[0] + 4 && v[3] == v[0] + 6;
    if (t64) {
      double* d = t64 + slot * blk2;
      if (whole) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const double2 a = p == 0 ? double2{x[0].x, x[1].x} : double2{x[0].y, x[1].y};
          const double2 b = p == 0 ? double2{x[2].x, x[3].x} : double2{x[2].y, x[3].y};
          *reinterpret_cast<double2*>(d + pair_value_offset(n, u, v[0], p, 2)) = a;
          *reinterpret_cast<double2*>(d + pair_value_offset(n, u, v[2], p, 2)) = b;
        }
      } else {
        for (int j = 0; j < cnt; ++j) {
          d[pair_value_offset(n, u, v[j], 0, 2)] = x[j].x;
          d[pair_value_offset(n, u, v[j], 1, 2)] = x[j].y;
        }
      }
    }
    if (t32) {
      float* f = t32 + slot * blk2;
      if (whole) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const float4 a = p == 0 ? float4{(float)x[0].x, (float)x[1].x, (float)x[2].x, (float)x[3].x}
                                  : float4{(float)x[0].y, (float)x[1].y, (float)x[2].y, (float)x[3].y};
          *reinterpret_cast<float4*>(f + pair_value_offset(n, u, v[0], p, 4)) = a;
        }
      } else {
        for (int j = 0; j < cnt; ++j) {
          f[pair_value_offset(n, u, v[j], 0, 4)] = (float)x[j].x;
          f[pair_value_offset(n, u, v[j], 1, 4)] = (float)x[j].y;
        }
      }
    }
  }
}

// Reciprocity check of caller blocks (parts n x n matrices per offset):
// out[0] = max |X(-d)[u][v] - X(d)[v][u] w[v] / w[u]| over every part X,
// out[1] = max |X(d)[u][v]| (non-negative doubles combined as their bit
// patterns, which order like the values).
__global__ void __launch_bounds__(256) recip_check_kernel(const double2* __restrict__ T, int nx, int ny, int n,
                                                          int parts, const double* __restrict__ w,
                                                          unsigned long long* __restrict__ out) {
  const long long nn = (long long)n * n;
  const int wx = 2 * nx - 1, wy = 2 * ny - 1;
  const long long total = (long long)wx * wy * parts * nn;
  double dmax = 0.0, mmax = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long bp = e / nn;   // block * parts + part
    const int r = (int)(e - bp * nn);
    const int u = r / n, v = r - u * n;
    const long long blk = bp / parts;
    const int part = (int)(bp - blk * parts);
    const int dyi = (int)(blk / wx), dxi = (int)(blk - (long long)dyi * wx);
    const long long mirror = (long long)(wy - 1 - dyi) * wx + (wx - 1 - dxi);
    const double2 a = T[e];
    const double2 b = T[(mirror * parts + part) * nn + (long long)v * n + u];
    const double f = w[v] / w[u];
    const double dx = a.x - b.x * f, dy = a.y - b.y * f;
    const double d = sqrt(dx * dx + dy * dy), m = sqrt(a.x * a.x + a.y * a.y);
    dmax = (d > dmax || d != d) ? d : dmax;
    mmax = (m > mmax || m != m) ? m : mmax;
  }
  __shared__ double sd[256], sm[256];
  sd[threadIdx.x] = dmax;
  sm[threadIdx.x] = mmax;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      const double o = sd[threadIdx.x + st], q = sm[threadIdx.x + st];
      if (o > sd[threadIdx.x] || o != o) sd[threadIdx.x] = o;
      if (q > sm[threadIdx.x] || q != q) sm[threadIdx.x] = q;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(out, (unsigned long long)__double_as_longlong(sd[0]));
    atomicMax(out + 1, (unsigned long long)__double_as_longlong(sm[0]));
  }
}

template <typename VI, typename VO>
__global__ void convert_kernel(const VI* __restrict__ in, VO* __restrict__ out, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const VI a = in[i];
    out[i] = VO{static_cast<decltype(out[0].x)>(a.x), static_cast<decltype(out[0].x)>(a.y)};
  }
}

unsigned grid_for(long long total, int threads) {
  long long g = (total + threads - 1) / threads;
  if (g > 65536LL * 8) g = 65536LL * 8;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

void launch_pad_blocks(const void* T_blocks_dev, int nx, int ny, int nb, int parts, int Lx, int Ly, int64_t c0,
                       int64_t nc, int vperm, void* K, hipStream_t s) {
  EMS_CHECK_ARG(!vperm || parts == 1, "internal: the pair column order is for dense blocks");
  const long long total = (long long)Ly * Lx * nc;
  EMS_CHECK_ARG(total < (1LL << 31) && c0 + nc < (1LL << 31), "internal: fill chunk exceeds 32-bit indices");
  hipLaunchKernelGGL(pad_blocks_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s,
                     static_cast<const double2*>(T_blocks_dev), nx, ny, nb, parts, Lx, Ly, (long long)c0,
                     (long long)nc, vperm, static_cast<double2*>(K));
  EMS_LAUNCH_CHECK();
}

void launch_green_padded(const GreenGeomDev& g, int nx, int ny, int Lx, int Ly, int64_t c0, int64_t nc, int vperm,
                         void* K, hipStream_t s) {
  const int64_t n = 4LL * g.n_patch;
  const int64_t ncol = (c0 + nc - 1) / n - c0 / n + 1;
  const long long total = (long long)Ly * Lx * ncol * g.n_patch;
  EMS_CHECK_ARG(nc >= 1 && total < (1LL << 31) && c0 + nc < (1LL << 31), "internal: fill chunk exceeds 32-bit indices");
  hipLaunchKernelGGL(green_padded_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, g.rho.as<const double>(),
                     g.area.as<const double>(), g.tan.as<const double>(), g.n_patch, g.pitch, g.k, nx, ny, Lx, Ly,
                     (long long)c0, (long long)nc, vperm, static_cast<double2*>(K));
  EMS_LAUNCH_CHECK();
}

void launch_lk_padded(const GreenGeomDev& g, int nx, int ny, int Lx, int Ly, int64_t c0, int64_t nc, void* K,
                      hipStream_t s) {
  const long long total = (long long)Ly * Lx * nc;
  EMS_CHECK_ARG(total < (1LL << 31) && c0 + nc < (1LL << 31), "internal: fill chunk exceeds 32-bit indices");
  hipLaunchKernelGGL(lk_padded_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, g.rho.as<const double>(),
                     g.area.as<const double>(), g.tan.as<const double>(), g.n_patch, g.pitch, g.k, nx, ny, Lx, Ly,
                     (long long)c0, (long long)nc, static_cast<double2*>(K));
  EMS_LAUNCH_CHECK();
}

void launch_lk_blocks(const GreenGeomDev& g, int nx, int ny, void* LK_blocks, hipStream_t s) {
  const long long nh = 2LL * g.n_patch;
  const long long total = (long long)(2 * ny - 1) * (2 * nx - 1) * 2 * nh * nh;
  hipLaunchKernelGGL(lk_blocks_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, g.rho.as<const double>(),
                     g.area.as<const double>(), g.tan.as<const double>(), g.n_patch, g.pitch, g.k, nx, ny,
                     static_cast<double2*>(LK_blocks));
  EMS_LAUNCH_CHECK();
}

void launch_green_blocks(const GreenGeomDev& g, int nx, int ny, void* T_blocks, hipStream_t s) {
  const long long n = 4LL * g.n_patch;
  const long long total = (long long)(2 * ny - 1) * (2 * nx - 1) * n * n;
  hipLaunchKernelGGL(green_blocks_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, g.rho.as<const double>(),
                     g.area.as<const double>(), g.tan.as<const double>(), g.n_patch, g.pitch, g.k, nx, ny,
                     static_cast<double2*>(T_blocks));
  EMS_LAUNCH_CHECK();
}

void launch_store_chunk(const void* Kc, int64_t P, int64_t nn, int64_t c0, int64_t nc, const int* slot_of,
                        const int* pairs, int64_t Ps, int n, int nh, int vperm, int uperm, void* that64,
                        void* that32, void* that16, hipStream_t s) {
  EMS_CHECK_ARG(!uperm || (nh == 0 && n % 4 == 0 && c0 % n == 0 && (nc % n == 0 || c0 + nc == nn)),
                "internal: the Green row order is for dense point-sampled blocks in whole-column chunks");
  EMS_CHECK_ARG(!(that16 && slot_of), "internal: the split-BF16 store has no reciprocal layout");
  EMS_CHECK_ARG(!vperm || (slot_of && pairs && nh == 0), "internal: the pair column order is for dense reciprocal stores");
  if (vperm) {
    EMS_CHECK_ARG(c0 % (4 * n) == 0 && nc % n == 0 && (nc % (4 * n) == 0 || c0 + nc == nn),
                  "internal: pair-order chunks must be whole multiples of 4 n_eq columns");
    const int64_t nq = (nc / n + 3) / 4;
    const int64_t total = Ps * nq * n;
    EMS_CHECK_ARG(Ps >= 1 && Ps <= P && total < (1LL << 31) && c0 + nc < (1LL << 31),
                  "internal: pair-order chunk too large");
    hipLaunchKernelGGL(store_pair_chunk_kernel, dim3(grid_for((long long)total, 256)), dim3(256), 0, s,
                       static_cast<const double2*>(Kc), (int)Ps, (int)c0, (int)nc, (int)nq, pairs, n, uperm,
                       static_cast<double*>(that64), static_cast<float*>(that32));
    EMS_LAUNCH_CHECK();
    return;
  }
  hipLaunchKernelGGL(store_chunk_kernel, dim3(grid_for((long long)P * nc, 256)), dim3(256), 0, s,
                     static_cast<const double2*>(Kc), (long long)P, (long long)nn, (long long)c0, (long long)nc,
                     slot_of, n, nh, vperm, uperm, static_cast<double2*>(that64), static_cast<float2*>(that32),
                     static_cast<__bf16*>(that16));
  EMS_LAUNCH_CHECK();
}

void launch_recip_check(const void* T_blocks_dev, int nx, int ny, int n, int parts, const double* w_dev, double* out,
                        hipStream_t s) {
  EMS_HIP(hipMemsetAsync(out, 0, 2 * sizeof(double), s));
  const long long total = (long long)(2 * nx - 1) * (2 * ny - 1) * parts * n * n;
  long long g = (total + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(recip_check_kernel, dim3((unsigned)g), dim3(256), 0, s, static_cast<const double2*>(T_blocks_dev),
                     nx, ny, n, parts, w_dev, reinterpret_cast<unsigned long long*>(out));
  EMS_LAUNCH_CHECK();
}

void launch_convert(Cx tin, Cx tout, const void* in, void* out, int64_t n, hipStream_t s) {
  const unsigned g = grid_for(n, 256);
  if (tin == Cx::C128 && tout == Cx::C64)
    hipLaunchKernelGGL((convert_kernel<double2, float2>), dim3(g), dim3(256), 0, s,
                       static_cast<const double2*>(in), static_cast<float2*>(out), (long long)n);
  else if (tin == Cx::C64 && tout == Cx::C128)
    hipLaunchKernelGGL((convert_kernel<float2, double2>), dim3(g), dim3(256), 0, s,
                       static_cast<const float2*>(in), static_cast<double2*>(out), (long long)n);
  else if (tin == Cx::C128)
    hipLaunchKernelGGL((convert_kernel<double2, double2>), dim3(g), dim3(256), 0, s,
                       static_cast<const double2*>(in), static_cast<double2*>(out), (long long)n);
  else
    hipLaunchKernelGGL((convert_kernel<float2, float2>), dim3(g), dim3(256), 0, s,
                       static_cast<const float2*>(in), static_cast<float2*>(out), (long long)n);
  EMS_LAUNCH_CHECK();
}

}  // namespace emsurf
