// Far field radiated by the equivalent currents of every box (Sec. II-A: the
// equivalent J and M on a fictitious surface radiate the exterior field;
// Sec. III: they are the solved unknowns).  With the point-sampled currents of
// the coupling fill (patch q of element m carries J = sum_a xJ t_qa at
// rho_q + pitch (ix, iy, 0), M likewise) and eta = 1,
//     E_theta = N . theta^ + L . phi^,   E_phi = N . phi^ - L . theta^,
//     N = sum A_q J e^{jk rhat . r'},    L = sum A_q M e^{jk rhat . r'}
// (common factor -jk e^{-jkr}/(4 pi r) dropped).  At the direction cosines of
// the bins of an Lu x Lv lattice DFT, k pitch u = 2 pi p' / Lu (p' the signed
// bin), the sum over elements is the zero-padded 2-D DFT with kernel
// e^{+j 2 pi (p ix / Lu + q iy / Lv)} of the lattice data: two Stockham
// passes of sign +1 (the passes of the coupling apply), then one projection
// per bin over the patches of a box.
#include <cmath>
#include <vector>

#include "internal.h"

namespace emsurf {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// One thread per (bin q, bin p, right-hand side r).  X[q][p][r][u] holds the
// lattice DFT of the unknowns; E[r][q][p][2] receives (E_theta, E_phi), zero
// outside the visible region u^2 + v^2 < 1.  wsign = +1 for the upper half
// space (w = cos(theta) >= 0), -1 for the lower one.
__global__ void far_field_kernel(const double2* __restrict__ X, const double* __restrict__ rho,
                                 const double* __restrict__ area, const double* __restrict__ tan, int P, double pitch,
                                 double k, int Lu, int Lv, int nrhs, double wsign, double2* __restrict__ E) {
  const long long total = (long long)Lv * Lu * nrhs;
  const int n = 4 * P;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(t % nrhs);
    const long long bin = t / nrhs;
    const int p = (int)(bin % Lu), q = (int)(bin / Lu);
    const int ps = p < (Lu + 1) / 2 ? p : p - Lu;
    const int qs = q < (Lv + 1) / 2 ? q : q - Lv;
    const double u = 2.0 * 3.14159265358979323846 * ps / (Lu * k * pitch);
    const double v = 2.0 * 3.14159265358979323846 * qs / (Lv * k * pitch);
    double2* out = E + (((long long)r * Lv + q) * Lu + p) * 2;
    const double s2 = u * u + v * v;
    if (!(s2 < 1.0)) {
      out[0] = double2{0.0, 0.0};
      out[1] = double2{0.0, 0.0};
      continue;
    }
    const double w = wsign * sqrt(1.0 - s2), st = sqrt(s2);
    const double cp = st > 0.0 ? u / st : 1.0, sp = st > 0.0 ? v / st : 0.0;
    const double th[3] = {w * cp, w * sp, -st};
    const double ph[3] = {-sp, cp, 0.0};
    const double2* xb = X + (bin * nrhs + r) * n;
    double2 N[3] = {{0, 0}, {0, 0}, {0, 0}}, L[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int i = 0; i < P; ++i) {
      double sn, cs;
      sincos(k * (u * rho[3 * i] + v * rho[3 * i + 1] + w * rho[3 * i + 2]), &sn, &cs);
      const double2 ph_i{area[i] * cs, area[i] * sn};
      const double2 j0 = cmul(ph_i, xb[2 * i]), j1 = cmul(ph_i, xb[2 * i + 1]);
      const double2 m0 = cmul(ph_i, xb[2 * P + 2 * i]), m1 = cmul(ph_i, xb[2 * P + 2 * i + 1]);
      const double* t0 = tan + 6 * i;
      const double* t1 = t0 + 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        N[c].x += j0.x * t0[c] + j1.x * t1[c];
        N[c].y += j0.y * t0[c] + j1.y * t1[c];
        L[c].x += m0.x * t0[c] + m1.x * t1[c];
        L[c].y += m0.y * t0[c] + m1.y * t1[c];
      }
    }
    double2 et{0, 0}, ep{0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      et.x += N[c].x * th[c] + L[c].x * ph[c];
      et.y += N[c].y * th[c] + L[c].y * ph[c];
      ep.x += N[c].x * ph[c] - L[c].x * th[c];
      ep.y += N[c].y * ph[c] - L[c].y * th[c];
    }
    out[0] = et;
    out[1] = ep;
  }
}

// Radiation intensity U = |E_theta|^2 + |E_phi|^2 weighted by the solid angle
// of its bin, du dv / |w|, summed per right-hand side over both half spaces:
// one workgroup per (right-hand side, slice of bins), a fixed-order tree in
// LDS, partial sums written per workgroup (the host adds them in order).
constexpr int DIR_THREADS = 256;
__global__ void __launch_bounds__(DIR_THREADS) power_partial_kernel(const double2* __restrict__ Eu,
                                                                    const double2* __restrict__ El, int Lu, int Lv,
                                                                    double pitch, double k, int slices,
                                                                    double* __restrict__ partial) {
  __shared__ double red[DIR_THREADS];
  const int r = blockIdx.y, sl = blockIdx.x;
  const long long bins = (long long)Lu * Lv;
  const long long per = (bins + slices - 1) / slices;
  const long long b0 = sl * per, b1 = b0 + per < bins ? b0 + per : bins;
  const double pi = 3.14159265358979323846;
  const double dudv = (2.0 * pi / (Lu * k * pitch)) * (2.0 * pi / (Lv * k * pitch));
  double acc = 0.0;
  for (long long b = b0 + threadIdx.x; b < b1; b += DIR_THREADS) {
    const int p = (int)(b % Lu), q = (int)(b / Lu);
    const int ps = p < (Lu + 1) / 2 ? p : p - Lu;
    const int qs = q < (Lv + 1) / 2 ? q : q - Lv;
    const double u = 2.0 * pi * ps / (Lu * k * pitch), v = 2.0 * pi * qs / (Lv * k * pitch);
    const double s2 = u * u + v * v;
    if (!(s2 < 1.0)) continue;
    const double2* eu = Eu + ((long long)r * bins + b) * 2;
    const double2* el = El + ((long long)r * bins + b) * 2;
    const double U = eu[0].x * eu[0].x + eu[0].y * eu[0].y + eu[1].x * eu[1].x + eu[1].y * eu[1].y +
                     el[0].x * el[0].x + el[0].y * el[0].y + el[1].x * el[1].x + el[1].y * el[1].y;
    acc += U * dudv / sqrt(1.0 - s2);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = DIR_THREADS / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(long long)r * slices + sl] = red[0];
}

// D[r][h][q][p] = 4 pi U / P_rad[r] (zero outside the visible region)
__global__ void directivity_kernel(const double2* __restrict__ Eu, const double2* __restrict__ El, int Lu, int Lv,
                                   int nrhs, const double* __restrict__ prad, double* __restrict__ D) {
  const long long bins = (long long)Lu * Lv, total = (long long)nrhs * 2 * bins;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long b = t % bins;
    const int h = (int)((t / bins) % 2), r = (int)(t / (2 * bins));
    const double2* e = (h == 0 ? Eu : El) + ((long long)r * bins + b) * 2;
    const double U = e[0].x * e[0].x + e[0].y * e[0].y + e[1].x * e[1].x + e[1].y * e[1].y;
    D[t] = 4.0 * 3.14159265358979323846 * U / prad[r];
  }
}

// Lattice DFT of the unknowns (sign +1) into X[q][p][r][u]; W is the
// half-transformed workspace
void lattice_dft(const GreenGeomDev& g, int nx, int ny, int nrhs, int Lu, int Lv, const void* x_dev, void* W, void* X,
                 hipStream_t s) {
  const int n = 4 * g.n_patch;
  const int64_t B = (int64_t)nrhs * n, M = (int64_t)nx * ny;
  FftPass fx;
  fx.L = Lu; fx.n_in = nx; fx.n_out = Lu; fx.batch = n;
  fx.n_lines = nrhs * ny; fx.nl0 = ny;
  fx.in_s1 = M * n; fx.in_s0 = (int64_t)nx * n; fx.in_pt = n;
  fx.out_s1 = n; fx.out_s0 = (int64_t)Lu * B; fx.out_pt = B;
  fx.sign = +1;
  launch_fft_pass(fx, Cx::C128, Cx::C128, Cx::C128, x_dev, W, twiddle_table(Lu, Cx::C128), s);
  FftPass fy;
  fy.L = Lv; fy.n_in = ny; fy.n_out = Lv; fy.batch = (int)B;
  fy.n_lines = Lu; fy.nl0 = Lu;
  fy.in_s0 = B; fy.in_pt = (int64_t)Lu * B;
  fy.out_s0 = B; fy.out_pt = (int64_t)Lu * B;
  fy.sign = +1;
  launch_fft_pass(fy, Cx::C128, Cx::C128, Cx::C128, W, X, twiddle_table(Lv, Cx::C128), s);
}

void project(const GreenGeomDev& g, const void* X, int Lu, int Lv, int nrhs, double wsign, void* E, hipStream_t s) {
  const long long total = (long long)Lv * Lu * nrhs;
  long long grid = (total + 255) / 256;
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(far_field_kernel, dim3((unsigned)grid), dim3(256), 0, s, static_cast<const double2*>(X),
                     g.rho.as<const double>(), g.area.as<const double>(), g.tan.as<const double>(), g.n_patch,
                     g.pitch, g.k, Lu, Lv, nrhs, wsign, static_cast<double2*>(E));
  EMS_LAUNCH_CHECK();
}

void check_far_args(const emsurf_geom* geom, int32_t nx, int32_t ny, int32_t nrhs, int32_t Lu, int32_t Lv) {
  EMS_CHECK_ARG(nx >= 1 && ny >= 1 && nx <= 1024 && ny <= 1024, "lattice sizes must be in [1, 1024]");
  EMS_CHECK_ARG(nrhs >= 1 && nrhs <= 64, "nrhs must be in [1, 64]");
  EMS_CHECK_ARG(fft_length_supported(Lu) && fft_length_supported(Lv) && Lu >= nx && Lv >= ny,
                "Lu, Lv must be supported FFT lengths (2^a <= 1024 or 3 * 2^a <= 768) with Lu >= nx, Lv >= ny");
  EMS_CHECK_ARG(geom != nullptr && geom->k > 0, "the far field needs a wavenumber k > 0");
}

}  // namespace
}  // namespace emsurf

using namespace emsurf;

extern "C" emsurf_status emsurf_far_field(const emsurf_geom* geom, int32_t nx, int32_t ny, int32_t nrhs, int32_t Lu,
                                          int32_t Lv, const void* x_dev, void* E_dev, void* stream) {
  try {
    EMS_CHECK_ARG(x_dev != nullptr && E_dev != nullptr, "x_dev and E_dev must be non-NULL");
    check_far_args(geom, nx, ny, nrhs, Lu, Lv);
    hipStream_t s = static_cast<hipStream_t>(stream);
    GreenGeomDev g;
    upload_geom(geom, g);
    const int64_t B = (int64_t)nrhs * 4 * g.n_patch;
    DevBuf W((size_t)ny * Lu * B * 16), X((size_t)Lv * Lu * B * 16);
    lattice_dft(g, nx, ny, nrhs, Lu, Lv, x_dev, W.p, X.p, s);
    project(g, X.p, Lu, Lv, nrhs, 1.0, E_dev, s);
    // the workspaces and geometry are freed on return
    EMS_HIP(hipStreamSynchronize(s));
    return EMSURF_OK;
  } catch (...) {
    return current_exception_status();
  }
}

extern "C" emsurf_status emsurf_directivity(const emsurf_geom* geom, int32_t nx, int32_t ny, int32_t nrhs, int32_t Lu,
                                            int32_t Lv, const void* x_dev, void* D_dev, double* prad_host,
                                            void* stream) {
  try {
    EMS_CHECK_ARG(x_dev != nullptr && D_dev != nullptr, "x_dev and D_dev must be non-NULL");
    check_far_args(geom, nx, ny, nrhs, Lu, Lv);
    hipStream_t s = static_cast<hipStream_t>(stream);
    GreenGeomDev g;
    upload_geom(geom, g);
    const int64_t B = (int64_t)nrhs * 4 * g.n_patch, bins = (int64_t)Lu * Lv;
    DevBuf W((size_t)ny * Lu * B * 16), X((size_t)Lv * Lu * B * 16);
    DevBuf Eu((size_t)nrhs * bins * 32), El((size_t)nrhs * bins * 32);
    lattice_dft(g, nx, ny, nrhs, Lu, Lv, x_dev, W.p, X.p, s);
    project(g, X.p, Lu, Lv, nrhs, 1.0, Eu.p, s);
    project(g, X.p, Lu, Lv, nrhs, -1.0, El.p, s);
    const int slices = 64;
    DevBuf part((size_t)nrhs * slices * 8), prad((size_t)nrhs * 8);
    hipLaunchKernelGGL(power_partial_kernel, dim3(slices, (unsigned)nrhs), dim3(DIR_THREADS), 0, s,
                       Eu.as<const double2>(), El.as<const double2>(), Lu, Lv, g.pitch, g.k, slices,
                       part.as<double>());
    EMS_LAUNCH_CHECK();
    std::vector<double> hp((size_t)nrhs * slices), pr(nrhs, 0.0);
    EMS_HIP(hipMemcpyAsync(hp.data(), part.p, hp.size() * 8, hipMemcpyDeviceToHost, s));
    EMS_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < nrhs; ++r) {
      for (int sl = 0; sl < slices; ++sl) pr[r] += hp[(size_t)r * slices + sl];
      EMS_CHECK_ARG(pr[r] > 0 && std::isfinite(pr[r]), "the currents radiate no power (zero or non-finite x)");
    }
    EMS_HIP(hipMemcpyAsync(prad.p, pr.data(), (size_t)nrhs * 8, hipMemcpyHostToDevice, s));
    const long long total = (long long)nrhs * 2 * bins;
    long long grid = (total + 255) / 256;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(directivity_kernel, dim3((unsigned)grid), dim3(256), 0, s, Eu.as<const double2>(),
                       El.as<const double2>(), Lu, Lv, nrhs, prad.as<const double>(), static_cast<double*>(D_dev));
    EMS_LAUNCH_CHECK();
    EMS_HIP(hipStreamSynchronize(s));
    if (prad_host)
      for (int r = 0; r < nrhs; ++r) prad_host[r] = pr[r];
    return EMSURF_OK;
  } catch (...) {
    return current_exception_status();
  }
}
