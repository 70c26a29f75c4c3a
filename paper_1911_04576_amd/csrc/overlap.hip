// Touching fictitious surfaces (Sec. III-D, eqs. (connections_IUI), (final)).
//
// When the lattice pitch equals the box edge, a face of each box coincides
// with a face of its neighbour and its currents are expanded twice.  The
// paper keeps one set of unknowns, Y = U_o Y~, and solves
// U_o^T [Z_eq + Z_o] U_o Y~ = U_o^T V.  With the point-sampled patches:
//   * a patch of element m + (1, 0) or m + (0, 1) whose centre coincides with
//     a patch of m is a duplicate; the tangential fields are continuous across
//     the shared face while the outward normals are opposite, so its currents
//     are x' = -sum_a (t'_b . t_a) x_a (both J and M), the face staying with m;
//   * with a ground plane under every box (the bottom faces on PEC), the
//     tangential electric field vanishes there and the bottom faces' M
//     unknowns leave the system;
//   * U_o's columns are the remaining unknowns in increasing full index.
// The paper's Z_eq + Z_o is D + T in the block-Jacobi form used elsewhere,
// D = -S^-1 per cell type, so the reduced operator is
//     A~ x~ = U_o^T (T U_o x~ - S^-1 U_o x~).
// U_o is stored by rows (full unknowns, at most two entries) for the
// expansion and by columns (unique unknowns, preimages in a fixed order) for
// U_o^T, so both are gathers and every sum has one order.
#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

#include "internal.h"

struct emsurf_overlap_s {
  emsurf_plan plan = nullptr;
  int64_t N = 0, Nt = 0;
  emsurf::DevBuf rptr, ridx, rval;   // U_o rows: int [N + 1], int / double [nnz]
  emsurf::DevBuf cptr, cidx, cval;   // U_o columns (U_o^T rows): int [Nt + 1], int / double [nnz]
  emsurf::DevBuf Sinv;               // c128 [n_types][n_eq][n_eq], S^-1 row-major
  emsurf::DevBuf w1, w2, w3;         // c128 [max_rhs][N] each
  size_t bytes() const {
    return rptr.bytes + ridx.bytes + rval.bytes + cptr.bytes + cidx.bytes + cval.bytes + Sinv.bytes + w1.bytes +
           w2.bytes + w3.bytes;
  }
};

namespace emsurf {
namespace {

// out[r][i] = sum over the entries e of row i of val[e] in[r][idx[e]]
__global__ void csr_gather_kernel(const int* __restrict__ ptr, const int* __restrict__ idx,
                                  const double* __restrict__ val, long long rows, long long cols, int nrhs,
                                  const double2* __restrict__ in, double2* __restrict__ out) {
  const long long total = rows * nrhs;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long r = t / rows, i = t - r * rows;
    double2 acc{0.0, 0.0};
    for (int e = ptr[i]; e < ptr[i + 1]; ++e) {
      const double2 v = in[r * cols + idx[e]];
      acc.x += val[e] * v.x;
      acc.y += val[e] * v.y;
    }
    out[t] = acc;
  }
}

// augmented [[S, I], [-I, 0]] per type: eliminating S leaves 0 + I S^-1 I = S^-1
__global__ void inv_setup_kernel(const double2* __restrict__ S, int n, int T, double2* __restrict__ A) {
  const int N = 2 * n;
  const long long total = (long long)T * N * N;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(e / ((long long)N * N));
    const int rem = (int)(e - (long long)t * N * N), i = rem / N, j = rem - i * N;
    double2 v{0.0, 0.0};
    if (i < n && j < n) v = S[((long long)t * n + i) * n + j];
    else if (i < n && j - n == i) v = double2{1.0, 0.0};
    else if (i >= n && j == i - n) v = double2{-1.0, 0.0};
    A[e] = v;
  }
}

__global__ void trailing_kernel(const double2* __restrict__ A, int n, int T, double2* __restrict__ out) {
  const int N = 2 * n;
  const long long total = (long long)T * n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(e / ((long long)n * n));
    const int rem = (int)(e - (long long)t * n * n), i = rem / n, j = rem - i * n;
    out[e] = A[(long long)t * N * N + (long long)(n + i) * N + n + j];
  }
}

unsigned grid_of(long long total) {
  long long b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)std::max<long long>(1, b);
}

void gather(const DevBuf& ptr, const DevBuf& idx, const DevBuf& val, long long rows, long long cols, int nrhs,
            const void* in, void* out, hipStream_t s) {
  hipLaunchKernelGGL(csr_gather_kernel, dim3(grid_of(rows * nrhs)), dim3(256), 0, s, ptr.as<const int>(),
                     idx.as<const int>(), val.as<const double>(), rows, cols, nrhs, static_cast<const double2*>(in),
                     static_cast<double2*>(out));
  EMS_LAUNCH_CHECK();
}

}  // namespace
}  // namespace emsurf

using namespace emsurf;

extern "C" {

emsurf_status emsurf_overlap_create(emsurf_plan plan, const emsurf_geom* geom, int32_t ground_plane, void* stream,
                                    emsurf_overlap* out) {
  emsurf_overlap ov = nullptr;
  emsurf_status st = guarded_call([&] {
    EMS_CHECK_ARG(plan != nullptr && geom != nullptr && out != nullptr, "plan, geom and out must be non-NULL");
    EMS_CHECK_ARG(plan->S64.p != nullptr && plan->that64.p != nullptr,
                  "the reduced operator needs the plan's FP64 store and macromodels");
    EMS_CHECK_ARG(plan->d.form == EMSURF_T_DENSE, "touching boxes need dense coupling blocks");
    EMS_CHECK_ARG(geom->rho && geom->tan && geom->area && geom->n_patch >= 1 && 4 * geom->n_patch == plan->d.n_eq,
                  "geom must describe the plan's boxes (n_eq = 4 n_patch)");
    EMS_CHECK_ARG(std::isfinite(geom->pitch) && geom->pitch > 0, "pitch must be > 0");
    EMS_CHECK_ARG(ground_plane == 0 || ground_plane == 1, "ground_plane must be 0 or 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int P = geom->n_patch, n = 4 * P, nx = plan->d.nx, ny = plan->d.ny;
    const int64_t N = (int64_t)nx * ny * n;
    EMS_CHECK_ARG(N < (1LL << 31), "too many unknowns");
    const double* rho = geom->rho;
    const double* tn = geom->tan;
    // coincident patch pairs within one lattice step: patch q of the +x (+y)
    // neighbour sits on patch p of the element
    std::vector<int> twin_x(P, -1), twin_y(P, -1);   // p -> q
    for (int q = 0; q < P; ++q)
      for (int p = 0; p < P; ++p) {
        for (int ax = 0; ax < 2; ++ax) {
          const double ex = rho[3 * q] + (ax == 0 ? geom->pitch : 0.0) - rho[3 * p];
          const double ey = rho[3 * q + 1] + (ax == 1 ? geom->pitch : 0.0) - rho[3 * p + 1];
          const double ez = rho[3 * q + 2] - rho[3 * p + 2];
          if (ex * ex + ey * ey + ez * ez <= 1e-18 * geom->area[q]) (ax == 0 ? twin_x : twin_y)[q] = p;
        }
      }
    // bottom faces (lowest centres, horizontal tangents) for the ground plane
    double zmin = rho[2];
    for (int p = 1; p < P; ++p) zmin = std::min(zmin, rho[3 * p + 2]);
    std::vector<char> bottom(P, 0);
    for (int p = 0; p < P; ++p)
      bottom[p] = ground_plane && std::fabs(rho[3 * p + 2] - zmin) <= 1e-9 && std::fabs(tn[6 * p + 2]) <= 1e-12 &&
                  std::fabs(tn[6 * p + 5]) <= 1e-12;
    // row entries of U_o: a unique unknown maps to itself; a duplicate to the
    // (negated, tangent-projected) unknowns of the patch it sits on
    std::vector<int64_t> uniq(N, -1);
    std::vector<char> dup(N, 0), gone(N, 0);
    for (int64_t m = 0; m < nx * ny; ++m) {
      const int ix = (int)(m % nx), iy = (int)(m / nx);
      for (int u = 0; u < n; ++u) {
        const int tau = u / (2 * P), p = (u % (2 * P)) / 2;
        if (tau == 1 && bottom[p]) gone[m * n + u] = 1;
        if ((ix > 0 && twin_x[p] >= 0) || (iy > 0 && twin_y[p] >= 0)) dup[m * n + u] = 1;
      }
    }
    int64_t Nt = 0;
    for (int64_t i = 0; i < N; ++i)
      if (!dup[i] && !gone[i]) uniq[i] = Nt++;
    std::vector<int> rptr(N + 1, 0), ridx;
    std::vector<double> rval;
    for (int64_t i = 0; i < N; ++i) {
      if (!gone[i]) {
        if (!dup[i]) {
          ridx.push_back((int)uniq[i]);
          rval.push_back(1.0);
        } else {
          const int64_t m = i / n;
          const int u = (int)(i % n), tau = u / (2 * P), q = (u % (2 * P)) / 2, b = u % 2;
          const int ix = (int)(m % nx);
          const bool along_x = ix > 0 && twin_x[q] >= 0;
          const int p = along_x ? twin_x[q] : twin_y[q];
          const int64_t mo = along_x ? m - 1 : m - nx;
          for (int a = 0; a < 2; ++a) {
            const double c = -(tn[(q * 2 + b) * 3] * tn[(p * 2 + a) * 3] + tn[(q * 2 + b) * 3 + 1] * tn[(p * 2 + a) * 3 + 1] +
                               tn[(q * 2 + b) * 3 + 2] * tn[(p * 2 + a) * 3 + 2]);
            const int64_t j = mo * n + tau * 2 * P + 2 * p + a;
            EMS_CHECK_ARG(!dup[j], "a shared face's kept patch is itself a duplicate");
            if (c != 0.0 && !gone[j]) {
              ridx.push_back((int)uniq[j]);
              rval.push_back(c);
            }
          }
        }
      }
      rptr[i + 1] = (int)ridx.size();
    }
    // columns: preimages of each unique unknown in increasing full index
    std::vector<int> cnt(Nt + 1, 0);
    for (size_t e = 0; e < ridx.size(); ++e) ++cnt[ridx[e] + 1];
    for (int64_t j = 0; j < Nt; ++j) cnt[j + 1] += cnt[j];
    std::vector<int> cptr(cnt), cidx(ridx.size()), fill(cnt.begin(), cnt.end() - 1);
    std::vector<double> cval(ridx.size());
    for (int64_t i = 0; i < N; ++i)
      for (int e = rptr[i]; e < rptr[i + 1]; ++e) {
        const int j = ridx[e];
        cidx[fill[j]] = (int)i;
        cval[fill[j]] = rval[e];
        ++fill[j];
      }
    ov = new emsurf_overlap_s();
    ov->plan = plan;
    ov->N = N;
    ov->Nt = Nt;
    auto up = [&](DevBuf& d, const void* h, size_t bytes) {
      d.alloc(std::max<size_t>(bytes, 4));
      if (bytes) EMS_HIP(hipMemcpyAsync(d.p, h, bytes, hipMemcpyHostToDevice, s));
    };
    up(ov->rptr, rptr.data(), rptr.size() * 4);
    up(ov->ridx, ridx.data(), ridx.size() * 4);
    up(ov->rval, rval.data(), rval.size() * 8);
    up(ov->cptr, cptr.data(), cptr.size() * 4);
    up(ov->cidx, cidx.data(), cidx.size() * 4);
    up(ov->cval, cval.data(), cval.size() * 8);
    // S^-1 per type by the partial elimination of [[S, I], [-I, 0]]
    const int T = plan->d.n_types;
    DevBuf A((size_t)T * 4 * n * n * 16), piv((size_t)T * n * 4), info((size_t)T * 4);
    hipLaunchKernelGGL(inv_setup_kernel, dim3(grid_of((long long)T * 4 * n * n)), dim3(256), 0, s,
                       plan->S64.as<const double2>(), n, T, A.as<double2>());
    EMS_LAUNCH_CHECK();
    EMS_HIP(hipMemsetAsync(info.p, 0, info.bytes, s));
    schur_eliminate(A.as<double2>(), 2 * n, n, T, piv.as<int>(), info.as<int>(), s);
    ov->Sinv.alloc((size_t)T * n * n * 16);
    hipLaunchKernelGGL(trailing_kernel, dim3(grid_of((long long)T * n * n)), dim3(256), 0, s, A.as<const double2>(), n,
                       T, ov->Sinv.as<double2>());
    EMS_LAUNCH_CHECK();
    std::vector<int> hinfo(T);
    EMS_HIP(hipMemcpyAsync(hinfo.data(), info.p, (size_t)T * 4, hipMemcpyDeviceToHost, s));
    EMS_HIP(hipStreamSynchronize(s));
    for (int t = 0; t < T; ++t)
      if (hinfo[t]) {
        set_error("macromodel of cell type " + std::to_string(t) + " is singular (no D = -S^-1)");
        throw Err{EMSURF_ERR_ARG};
      }
    const size_t vb = (size_t)plan->d.max_rhs * N * 16;
    ov->w1.alloc(vb);
    ov->w2.alloc(vb);
    ov->w3.alloc(vb);
  });
  if (st != EMSURF_OK) {
    delete ov;
    return st;
  }
  *out = ov;
  return EMSURF_OK;
}

emsurf_status emsurf_overlap_query(emsurf_overlap ov, int64_t* n_full, int64_t* n_unique, size_t* bytes) {
  return guarded_call([&] {
    EMS_CHECK_ARG(ov != nullptr, "overlap is NULL");
    if (n_full) *n_full = ov->N;
    if (n_unique) *n_unique = ov->Nt;
    if (bytes) *bytes = ov->bytes();
  });
}

emsurf_status emsurf_overlap_expand(emsurf_overlap ov, int32_t nrhs, const void* xt_dev, void* x_dev, void* stream) {
  return guarded_call([&] {
    EMS_CHECK_ARG(ov != nullptr && xt_dev && x_dev && xt_dev != x_dev, "overlap, xt and x must be non-NULL and distinct");
    EMS_CHECK_ARG(nrhs >= 1 && nrhs <= 64, "nrhs must be in [1, 64]");
    gather(ov->rptr, ov->ridx, ov->rval, ov->N, ov->Nt, nrhs, xt_dev, x_dev, static_cast<hipStream_t>(stream));
  });
}

emsurf_status emsurf_overlap_reduce(emsurf_overlap ov, int32_t nrhs, const void* y_dev, void* yt_dev, void* stream) {
  return guarded_call([&] {
    EMS_CHECK_ARG(ov != nullptr && y_dev && yt_dev && y_dev != yt_dev, "overlap, y and yt must be non-NULL and distinct");
    EMS_CHECK_ARG(nrhs >= 1 && nrhs <= 64, "nrhs must be in [1, 64]");
    gather(ov->cptr, ov->cidx, ov->cval, ov->Nt, ov->N, nrhs, y_dev, yt_dev, static_cast<hipStream_t>(stream));
  });
}

emsurf_status emsurf_apply_reduced(emsurf_overlap ov, int32_t nrhs, const void* xt_dev, void* yt_dev, void* stream) {
  return guarded_call([&] {
    EMS_CHECK_ARG(ov != nullptr && xt_dev && yt_dev && xt_dev != yt_dev, "overlap, xt and yt must be non-NULL and distinct");
    emsurf_plan p = ov->plan;
    EMS_CHECK_ARG(nrhs >= 1 && nrhs <= p->d.max_rhs, "nrhs must be in [1, max_rhs]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    gather(ov->rptr, ov->ridx, ov->rval, ov->N, ov->Nt, nrhs, xt_dev, ov->w1.p, s);            // x = U_o x~
    apply_T_typed(p, Cx::C128, Cx::C128, Cx::C128, nrhs, ov->w1.p, ov->w2.p, s);               // T x
    launch_apply_S(Cx::C128, Cx::C128, Cx::C128, ov->Sinv.p, p->tiles, p->d.n_eq, p->M, nrhs, ov->w1.p, ov->w2.p,
                   ov->w3.p, s);                                                                // T x - S^-1 x
    gather(ov->cptr, ov->cidx, ov->cval, ov->Nt, ov->N, nrhs, ov->w3.p, yt_dev, s);            // U_o^T
  });
}

void emsurf_overlap_destroy(emsurf_overlap ov) {
  if (!ov) return;
  (void)hipDeviceSynchronize();
  delete ov;
}

}  // extern "C"
