// Near-field right preconditioner (Sec. IV-A, eq. (final_precond)).
//
// The paper preconditions its final system on the right with P, the part of
// the system matrix whose entries couple basis functions closer than
// Delta_NF, and applies P^-1 through an LU factorisation of that sparse
// matrix.  In the block-Jacobi form solved here, A = I - S T (S the
// per-element macromodels, which hold the exact inverse of each element's
// self block, T the mutual coupling with T(0) = 0), the same construction is
//
//     P = I - S T_NF,   T_NF(d)[u][v] = T(d)[u][v] if |r_u - r_v + pitch d| < Delta_NF, else 0,
//
// with r_u the centre of the patch of unknown u.  For the box lattices of the
// paper Delta_NF (lambda/10 .. lambda/6) reaches adjacent elements only, so
// T_NF lives on the 8 neighbour offsets.  P is factored per tile of
// tile_x x tile_y elements (block Jacobi over tiles: the near-field couplings
// between tiles are dropped; a tile covering the lattice is the paper's P).
//
// On a tile, T_NF couples only the unknowns Q that have a near partner in
// another element of the tile (facing side patches, a fraction of n_eq), so
// with C = T_NF restricted to Q x Q and S_QQ the rows and columns Q of the
// element macromodels,
//     P x = y  <=>  (I - S_QQ C) x_Q = y_Q,   x = y + S E_Q C x_Q,
// and P^-1 y = y + S E_Q G y_Q with G = C (I - S_QQ C)^-1 (|Q| x |Q| per tile).
// G is formed on the device by the partial elimination of the augmented
// matrix [[R, I], [C, 0]] (R = I - S_QQ C), whose trailing block is -C R^-1 = -G.
// An apply gathers y_Q, multiplies by -G (one workgroup per tile), scatters
// the result t into a vector that is zero off Q, and ends with the
// macromodel apply x = y - S t.  Everything is FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "internal.h"

struct emsurf_precond_s {
  emsurf_plan plan = nullptr;
  int tx = 1, ty = 1, ntx = 0, nty = 0, ntiles = 0, nq = 0;
  int64_t near_entries = 0;
  double delta = 0, build_ms = 0;
  emsurf::DevBuf qidx;   // int [ntiles][nq]: global unknown m n_eq + u, -1 for padding
  emsurf::DevBuf qpos;   // int [ntiles][tx ty][n_eq]: position in Q of (element slot, u), -1 if not in Q
  emsurf::DevBuf G;      // c128 [ntiles][nq][nq]: -G, entry (i, j) at j nq + i
  emsurf::DevBuf t;      // c128 [max_rhs][M][n_eq]: scattered -G y_Q
  size_t bytes() const { return qidx.bytes + qpos.bytes + G.bytes + t.bytes; }
};

namespace emsurf {
namespace {

__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {
  return double2{__builtin_fma(a.x, b.x, __builtin_fma(-a.y, b.y, c.x)), __builtin_fma(a.x, b.y, __builtin_fma(a.y, b.x, c.y))};
}

struct TileGeo {
  int nx, ny, n, nq, tx, ntx;
};

// near-field coupling C(i, j) between Q entries qi (test) and qj (source) of one tile
__device__ double2 near_entry(int qi, int qj, const TileGeo& g, const unsigned char* __restrict__ mask,
                              const double2* __restrict__ Tn) {
  if (qi < 0 || qj < 0) return double2{0, 0};
  const int mi = qi / g.n, ui = qi - mi * g.n, mj = qj / g.n, uj = qj - mj * g.n;
  if (mi == mj) return double2{0, 0};
  const int dy = mi / g.nx - mj / g.nx, dx = mi % g.nx - mj % g.nx;
  if (dy < -1 || dy > 1 || dx < -1 || dx > 1) return double2{0, 0};   // not adjacent: no near pair
  const long long o = ((long long)((dy + 1) * 3 + dx + 1) * g.n + ui) * g.n + uj;
  return mask[o] ? Tn[o] : double2{0, 0};
}

// Augmented matrices [[R, I], [C, 0]] (row-major, 2 nq square) of tiles
// [t0, t0 + nb): R = I - S_QQ C, the sum running over the Q entries k of row
// i's own element (segment seg[i] = [k0, k1)).
__global__ void build_aug_kernel(TileGeo g, int t0, int nb, const int* __restrict__ qidx, const int2* __restrict__ seg,
                                 const int* __restrict__ etype, const double2* __restrict__ S,
                                 const unsigned char* __restrict__ mask, const double2* __restrict__ Tn,
                                 double2* __restrict__ A) {
  const int N = 2 * g.nq;
  const long long total = (long long)nb * N * N;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(e / ((long long)N * N));
    const int rem = (int)(e - (long long)b * N * N), i = rem / N, j = rem - i * N;
    const long long t = t0 + b;
    const int* q = qidx + t * g.nq;
    double2 v{0, 0};
    if (i < g.nq && j < g.nq) {
      const int qi = q[i];
      if (qi < 0) {
        v = double2{i == j ? 1.0 : 0.0, 0};
      } else {
        const int m = qi / g.n, ui = qi - m * g.n;
        const double2* Sr = S + ((long long)etype[m] * g.n + ui) * g.n;
        const int2 sg = seg[t * g.nq + i];
        double2 acc{0, 0};
        for (int k = sg.x; k < sg.y; ++k) {
          const int qk = q[k];
          acc = cfma(Sr[qk - m * g.n], near_entry(qk, q[j], g, mask, Tn), acc);
        }
        v = double2{(i == j ? 1.0 : 0.0) - acc.x, -acc.y};
      }
    } else if (i < g.nq) {
      v = double2{i == j - g.nq ? 1.0 : 0.0, 0};
    } else if (j < g.nq) {
      v = near_entry(q[i - g.nq], q[j], g, mask, Tn);
    }
    A[e] = v;
  }
}

// trailing block (-G) of the eliminated augmented matrices into the store,
// transposed: entry (i, j) at j nq + i
__global__ void store_g_kernel(int nq, int t0, int nb, const double2* __restrict__ A, double2* __restrict__ G) {
  const int N = 2 * nq;
  const long long total = (long long)nb * nq * nq;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(e / ((long long)nq * nq));
    const int rem = (int)(e - (long long)b * nq * nq), j = rem / nq, i = rem - j * nq;
    G[(long long)(t0 + b) * nq * nq + rem] = A[(long long)b * N * N + (long long)(nq + i) * N + nq + j];
  }
}

constexpr int PC_THREADS = 256;
constexpr int PC_RC = 4;   // right-hand sides per pass over a tile's G

// t = scatter(-G y_Q) over the tile's elements (zero off Q); one workgroup per tile
__global__ void __launch_bounds__(PC_THREADS) pc_tile_kernel(TileGeo g, int ty, int nrhs, long long N,
                                                             const int* __restrict__ qidx,
                                                             const int* __restrict__ qpos,
                                                             const double2* __restrict__ G,
                                                             const double2* __restrict__ y, double2* __restrict__ t) {
  extern __shared__ double2 pc_lds[];
  double2* yq = pc_lds;                 // [PC_RC][nq]
  double2* zq = pc_lds + PC_RC * g.nq;  // [PC_RC][nq]
  const long long tile = blockIdx.x;
  const int tyi = (int)(tile / g.ntx), txi = (int)(tile - (long long)tyi * g.ntx);
  const int* q = qidx + tile * g.nq;
  const double2* Gt = G + tile * (long long)g.nq * g.nq;
  const int slots = g.tx * ty;
  for (int r0 = 0; r0 < nrhs; r0 += PC_RC) {
    const int rc = nrhs - r0 < PC_RC ? nrhs - r0 : PC_RC;
    for (int e = threadIdx.x; e < PC_RC * g.nq; e += PC_THREADS) {
      const int r = e / g.nq, j = e - r * g.nq;
      const int qj = q[j];
      yq[e] = (r < rc && qj >= 0) ? y[(long long)(r0 + r) * N + qj] : double2{0, 0};
    }
    __syncthreads();
    for (int i = threadIdx.x; i < g.nq; i += PC_THREADS) {
      double2 acc[PC_RC];
#pragma unroll
      for (int r = 0; r < PC_RC; ++r) acc[r] = double2{0, 0};
      for (int j = 0; j < g.nq; ++j) {
        const double2 gij = Gt[(long long)j * g.nq + i];
#pragma unroll
        for (int r = 0; r < PC_RC; ++r) acc[r] = cfma(gij, yq[r * g.nq + j], acc[r]);
      }
#pragma unroll
      for (int r = 0; r < PC_RC; ++r) zq[r * g.nq + i] = acc[r];
    }
    __syncthreads();
    const long long span = (long long)slots * g.n;
    for (long long e = threadIdx.x; e < (long long)rc * span; e += PC_THREADS) {
      const int r = (int)(e / span);
      const int rem = (int)(e - (long long)r * span), sl = rem / g.n, u = rem - sl * g.n;
      const int iy = tyi * ty + sl / g.tx, ix = txi * g.tx + sl % g.tx;
      if (iy >= g.ny || ix >= g.nx) continue;
      const int p = qpos[(tile * slots + sl) * g.n + u];
      t[(long long)(r0 + r) * N + ((long long)iy * g.nx + ix) * g.n + u] = p >= 0 ? zq[r * g.nq + p] : double2{0, 0};
    }
    __syncthreads();
  }
}

unsigned grid_for(long long total) {
  long long b = (total + 255) / 256;
  if (b > 65535LL * 32) b = 65535LL * 32;
  return (unsigned)std::max<long long>(1, b);
}

}  // namespace

void precond_apply(emsurf_precond pc, int nrhs, const void* y, void* x, hipStream_t s) {
  emsurf_plan p = pc->plan;
  const int n = p->d.n_eq;
  const long long N = (long long)p->M * n;
  EMS_CHECK_ARG(nrhs >= 1 && nrhs <= p->d.max_rhs, "nrhs must be in [1, max_rhs]");
  if (pc->nq == 0) {   // no near pair: P = I
    if (x != y) EMS_HIP(hipMemcpyAsync(x, y, (size_t)nrhs * N * 16, hipMemcpyDeviceToDevice, s));
    return;
  }
  EMS_CHECK_ARG(x != y, "the preconditioner apply needs distinct y and x");
  const TileGeo g{p->d.nx, p->d.ny, n, pc->nq, pc->tx, pc->ntx};
  const size_t shm = (size_t)2 * PC_RC * pc->nq * sizeof(double2);
  hipLaunchKernelGGL(pc_tile_kernel, dim3((unsigned)pc->ntiles), dim3(PC_THREADS), shm, s, g, pc->ty, nrhs, N,
                     pc->qidx.as<const int>(), pc->qpos.as<const int>(), pc->G.as<const double2>(),
                     static_cast<const double2*>(y), pc->t.as<double2>());
  EMS_LAUNCH_CHECK();
  apply_S_plan(p, Cx::C128, Cx::C128, nrhs, pc->t.p, y, x, s);
}

emsurf_plan precond_plan(emsurf_precond pc) { return pc->plan; }

}  // namespace emsurf

using namespace emsurf;

namespace {

// element types of the plan, recovered from its type tiles
std::vector<int> plan_types(emsurf_plan p, hipStream_t s) {
  std::vector<int> sorted(p->M), tl((size_t)p->tiles.n_tiles * 3), et(p->M, -1);
  EMS_HIP(hipMemcpyAsync(sorted.data(), p->tiles.elem_sorted.p, sorted.size() * 4, hipMemcpyDeviceToHost, s));
  EMS_HIP(hipMemcpyAsync(tl.data(), p->tiles.tiles.p, tl.size() * 4, hipMemcpyDeviceToHost, s));
  EMS_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < p->tiles.n_tiles; ++i)
    for (int c = 0; c < tl[3 * i + 2]; ++c) et[sorted[tl[3 * i + 1] + c]] = tl[3 * i];
  return et;
}

}  // namespace

extern "C" {

emsurf_status emsurf_precond_create(emsurf_plan plan, const emsurf_geom* geom, double delta_nf, int32_t tile_x,
                                    int32_t tile_y, const void* T_near, void* stream, emsurf_precond* out) {
  emsurf_precond pc = nullptr;
  emsurf_status st = guarded_call([&] {
    const auto t_start = std::chrono::steady_clock::now();
    EMS_CHECK_ARG(plan != nullptr && out != nullptr && geom != nullptr, "plan, geom and out must be non-NULL");
    EMS_CHECK_ARG(plan->S64.p != nullptr, "plan has no FP64 macromodels");
    EMS_CHECK_ARG(std::isfinite(delta_nf) && delta_nf >= 0, "delta_nf must be finite and >= 0");
    EMS_CHECK_ARG(tile_x >= 1 && tile_y >= 1 && (int64_t)tile_x * tile_y <= 64,
                  "tile_x, tile_y must be >= 1 with tile_x tile_y <= 64");
    EMS_CHECK_ARG(geom->rho != nullptr && geom->n_patch >= 1 && 4 * geom->n_patch == plan->d.n_eq,
                  "geom must describe the plan's boxes (n_eq = 4 n_patch)");
    EMS_CHECK_ARG(std::isfinite(geom->pitch) && geom->pitch > 0, "pitch must be > 0");
    EMS_CHECK_ARG(plan->d.form == EMSURF_T_DENSE, "the near-field preconditioner needs dense coupling blocks");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int n = plan->d.n_eq, nx = plan->d.nx, ny = plan->d.ny, P = geom->n_patch;
    const int tx = std::min<int>(tile_x, nx), ty = std::min<int>(tile_y, ny);
    // near pairs per neighbour offset d = (test element) - (source element)
    auto near = [&](int p, int q, int dy, int dx) {
      const double ax = geom->rho[3 * p] - geom->rho[3 * q] + geom->pitch * dx;
      const double ay = geom->rho[3 * p + 1] - geom->rho[3 * q + 1] + geom->pitch * dy;
      const double az = geom->rho[3 * p + 2] - geom->rho[3 * q + 2];
      return std::sqrt(ax * ax + ay * ay + az * az) < delta_nf;
    };
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx) {
        if (std::max(std::abs(dy), std::abs(dx)) != 2) continue;
        for (int p = 0; p < P; ++p)
          for (int q = 0; q < P; ++q)
            EMS_CHECK_ARG(!near(p, q, dy, dx),
                          "delta_nf reaches elements two lattice steps apart; only adjacent elements are supported");
      }
    std::vector<unsigned char> mask((size_t)9 * n * n, 0);
    std::vector<unsigned char> rowany((size_t)9 * n, 0), colany((size_t)9 * n, 0);
    int64_t near_entries = 0;
    auto pu = [&](int u) { return (u % (2 * P)) / 2; };
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (dy == 0 && dx == 0) continue;
        const int o = (dy + 1) * 3 + dx + 1;
        for (int u = 0; u < n; ++u)
          for (int v = 0; v < n; ++v)
            if (near(pu(u), pu(v), dy, dx)) {
              mask[((size_t)o * n + u) * n + v] = 1;
              rowany[(size_t)o * n + u] = 1;
              colany[(size_t)o * n + v] = 1;
              ++near_entries;
            }
      }
    pc = new emsurf_precond_s();
    pc->plan = plan;
    pc->tx = tx;
    pc->ty = ty;
    pc->delta = delta_nf;
    pc->near_entries = near_entries;
    pc->ntx = (nx + tx - 1) / tx;
    pc->nty = (ny + ty - 1) / ty;
    pc->ntiles = pc->ntx * pc->nty;
    const int slots = tx * ty;
    // Q of every tile: element slots in order, unknowns ascending
    std::vector<std::vector<int>> tq(pc->ntiles);
    std::vector<int> qpos((size_t)pc->ntiles * slots * n, -1);
    int nq = 0;
    for (int t = 0; t < pc->ntiles; ++t) {
      const int iy0 = (t / pc->ntx) * ty, ix0 = (t % pc->ntx) * tx;
      for (int sl = 0; sl < slots; ++sl) {
        const int iy = iy0 + sl / tx, ix = ix0 + sl % tx;
        if (iy >= ny || ix >= nx) continue;
        for (int u = 0; u < n; ++u) {
          bool inq = false;
          for (int sl2 = 0; sl2 < slots && !inq; ++sl2) {
            const int jy = iy0 + sl2 / tx, jx = ix0 + sl2 % tx;
            if (sl2 == sl || jy >= ny || jx >= nx) continue;
            const int dy = iy - jy, dx = ix - jx;
            if (std::abs(dy) > 1 || std::abs(dx) > 1) continue;
            inq = rowany[(size_t)((dy + 1) * 3 + dx + 1) * n + u] || colany[(size_t)((1 - dy) * 3 + 1 - dx) * n + u];
          }
          if (inq) {
            qpos[((size_t)t * slots + sl) * n + u] = (int)tq[t].size();
            tq[t].push_back((iy * nx + ix) * n + u);
          }
        }
      }
      nq = std::max<int>(nq, (int)tq[t].size());
    }
    pc->nq = nq;
    pc->t.alloc((size_t)plan->d.max_rhs * plan->M * n * 16);
    if (nq > 0) {
      EMS_CHECK_ARG(nq <= 1024, "more than 1024 near-field unknowns in one tile: use smaller tiles");
      std::vector<int> qidx((size_t)pc->ntiles * nq, -1);
      std::vector<int> seg((size_t)pc->ntiles * nq * 2, 0);
      for (int t = 0; t < pc->ntiles; ++t) {
        const int c = (int)tq[t].size();
        for (int i = 0; i < c; ++i) qidx[(size_t)t * nq + i] = tq[t][i];
        for (int i = 0; i < c;) {
          int k = i;
          while (k < c && tq[t][k] / n == tq[t][i] / n) ++k;
          for (int a = i; a < k; ++a) {
            seg[((size_t)t * nq + a) * 2] = i;
            seg[((size_t)t * nq + a) * 2 + 1] = k;
          }
          i = k;
        }
      }
      pc->qidx.alloc(qidx.size() * 4);
      pc->qpos.alloc(qpos.size() * 4);
      EMS_HIP(hipMemcpyAsync(pc->qidx.p, qidx.data(), qidx.size() * 4, hipMemcpyHostToDevice, s));
      EMS_HIP(hipMemcpyAsync(pc->qpos.p, qpos.data(), qpos.size() * 4, hipMemcpyHostToDevice, s));
      DevBuf seg_d(seg.size() * 4), mask_d(mask.size()), Tn((size_t)9 * n * n * 16), et_d((size_t)plan->M * 4);
      EMS_HIP(hipMemcpyAsync(seg_d.p, seg.data(), seg.size() * 4, hipMemcpyHostToDevice, s));
      EMS_HIP(hipMemcpyAsync(mask_d.p, mask.data(), mask.size(), hipMemcpyHostToDevice, s));
      const std::vector<int> et = plan_types(plan, s);
      EMS_HIP(hipMemcpyAsync(et_d.p, et.data(), et.size() * 4, hipMemcpyHostToDevice, s));
      if (T_near) {
        EMS_HIP(hipMemcpyAsync(Tn.p, T_near, Tn.bytes, hipMemcpyHostToDevice, s));
      } else {
        GreenGeomDev gd;
        upload_geom(geom, gd);
        launch_green_blocks(gd, 2, 2, Tn.p, s);
        EMS_HIP(hipStreamSynchronize(s));
      }
      pc->G.alloc((size_t)pc->ntiles * nq * nq * 16);
      // augmented matrices in batches of at most 512 MB
      const int N2 = 2 * nq;
      const int batch = (int)std::max<int64_t>(1, std::min<int64_t>(pc->ntiles, (512ll << 20) / ((int64_t)N2 * N2 * 16)));
      DevBuf A((size_t)batch * N2 * N2 * 16), piv((size_t)batch * nq * 4), info((size_t)batch * 4);
      const TileGeo g{nx, ny, n, nq, tx, pc->ntx};
      std::vector<int> hinfo(batch);
      for (int t0 = 0; t0 < pc->ntiles; t0 += batch) {
        const int nb = std::min(batch, pc->ntiles - t0);
        hipLaunchKernelGGL(build_aug_kernel, dim3(grid_for((long long)nb * N2 * N2)), dim3(256), 0, s, g, t0, nb,
                           pc->qidx.as<const int>(), seg_d.as<const int2>(), et_d.as<const int>(),
                           plan->S64.as<const double2>(), mask_d.as<const unsigned char>(),
                           Tn.as<const double2>(), A.as<double2>());
        EMS_LAUNCH_CHECK();
        EMS_HIP(hipMemsetAsync(info.p, 0, (size_t)nb * 4, s));
        schur_eliminate(A.as<double2>(), N2, nq, nb, piv.as<int>(), info.as<int>(), s);
        hipLaunchKernelGGL(store_g_kernel, dim3(grid_for((long long)nb * nq * nq)), dim3(256), 0, s, nq, t0, nb,
                           A.as<const double2>(), pc->G.as<double2>());
        EMS_LAUNCH_CHECK();
        EMS_HIP(hipMemcpyAsync(hinfo.data(), info.p, (size_t)nb * 4, hipMemcpyDeviceToHost, s));
        EMS_HIP(hipStreamSynchronize(s));
        for (int b = 0; b < nb; ++b)
          if (hinfo[b]) {
            set_error("near-field block of tile " + std::to_string(t0 + b) + " is singular");
            throw Err{EMSURF_ERR_ARG};
          }
      }
    }
    EMS_HIP(hipStreamSynchronize(s));
    pc->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  });
  if (st != EMSURF_OK) {
    delete pc;
    return st;
  }
  *out = pc;
  return EMSURF_OK;
}

emsurf_status emsurf_precond_apply(emsurf_precond pc, int32_t nrhs, const void* y_dev, void* x_dev, void* stream) {
  return guarded_call([&] {
    EMS_CHECK_ARG(pc != nullptr && y_dev != nullptr && x_dev != nullptr, "pc, y and x must be non-NULL");
    precond_apply(pc, nrhs, y_dev, x_dev, static_cast<hipStream_t>(stream));
  });
}

emsurf_status emsurf_precond_query(emsurf_precond pc, emsurf_precond_stats* out) {
  return guarded_call([&] {
    EMS_CHECK_ARG(pc != nullptr && out != nullptr, "pc and out must be non-NULL");
    out->n_tiles = pc->ntiles;
    out->nq_max = pc->nq;
    out->near_entries = pc->near_entries;
    out->bytes = pc->bytes();
    out->build_ms = pc->build_ms;
  });
}

void emsurf_precond_destroy(emsurf_precond pc) {
  if (!pc) return;
  (void)hipDeviceSynchronize();
  delete pc;
}

}  // extern "C"
