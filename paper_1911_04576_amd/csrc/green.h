// Device pieces of the point-sampled coupling fill (Sec. III-B, with the
// circulant embedding of Sec. IV-B): the lattice offset held by a padded slot,
// and one entry of the synthetic dense block T(d).  Shared by the plan fill
// kernels and the kernel FFT's generating first pass.
#pragma once
#include <hip/hip_runtime.h>

namespace emsurf {

// padded slot s of an axis of length L holds offset s (s < N) or s - L
// (s > L - N); the slots between stay zero
__device__ __forceinline__ int slot_to_offset(int s, int L, int N, bool* ok) {
  if (s <= N - 1) { *ok = true; return s; }
  if (s >= L - (N - 1)) { *ok = true; return s - L; }
  *ok = false;
  return 0;
}

// T(d)[(tau,p,a),(tau',q,b)] = delta(tau,tau') (t_pa . t_qb) A_q exp(-jkR)/(4 pi R),
// R = |rho_p - rho_q + pitch (dx, dy, 0)|, T(0) = 0.
__device__ __forceinline__ double2 green_entry(const double* __restrict__ rho, const double* __restrict__ area,
                                               const double* __restrict__ tan, int P, double pitch, double k,
                                               int dx, int dy, int u, int v) {
  if (dx == 0 && dy == 0) return double2{0.0, 0.0};
  const int hu = u / (2 * P), hv = v / (2 * P);
  if (hu != hv) return double2{0.0, 0.0};
  const int lu = u - hu * 2 * P, lv = v - hv * 2 * P;
  const int p = lu >> 1, a = lu & 1, q = lv >> 1, b = lv & 1;
  const double* tp = tan + (p * 2 + a) * 3;
  const double* tq = tan + (q * 2 + b) * 3;
  const double dot = tp[0] * tq[0] + tp[1] * tq[1] + tp[2] * tq[2];
  if (dot == 0.0) return double2{0.0, 0.0};
  const double ex = rho[3 * p + 0] - rho[3 * q + 0] + pitch * dx;
  const double ey = rho[3 * p + 1] - rho[3 * q + 1] + pitch * dy;
  const double ez = rho[3 * p + 2] - rho[3 * q + 2];
  const double R = sqrt(ex * ex + ey * ey + ez * ez);
  double sn, cs;
  sincos(k * R, &sn, &cs);
  const double w = dot * area[q] / (4.0 * 3.14159265358979323846 * R);
  return double2{w * cs, -w * sn};
}

}  // namespace emsurf
