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

// A exp(-jkR) / (4 pi R), the Green's function weighted by the source patch
// area.  A test point on the centre of the source patch (touching boxes share
// a face, Sec. III-D) takes the average over a square source patch of that
// area instead: (4 a ln(1 + sqrt 2) - j k a^2) / (4 pi), a = sqrt(A) (the
// static part integrated over the square, plus the first term of
// (exp(-jkR) - 1) / (4 pi R)).
__device__ __forceinline__ double2 area_green(double R, double A, double k) {
  const double inv4pi = 0.25 / 3.14159265358979323846;
  if (R * R <= 1e-18 * A) return double2{4.0 * sqrt(A) * 0.88137358701954302523 * inv4pi, -k * A * inv4pi};
  double sn, cs;
  sincos(k * R, &sn, &cs);
  const double w = A * inv4pi / R;
  return double2{w * cs, -w * sn};
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
  const double2 g = area_green(R, area[q], k);
  return double2{dot * g.x, dot * g.y};
}

}  // namespace emsurf
