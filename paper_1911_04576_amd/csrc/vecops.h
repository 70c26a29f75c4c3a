// Launchers of the GMRES vector kernels (vecops.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace emsurf {
// One item of a pointer-list launch (device memory).  Meaning per kernel:
//   copy:   dst = scale * (b ? b - a : a)
//   dot:    a = basis (nv vectors of length N, contiguous), dst = w
//   update: a = basis, dst = w (w -= basis * coefficients from the reduction buffer)
//   axpy:   a = basis, b = coefficients (nv complex), dst = x (x += basis * y)
struct VecItem {
  const void* a;
  const void* b;
  void* dst;
  double scale;
  int nv;
  int pad;
};
void launch_copy_list(const VecItem* items_dev, int nq, long long N, hipStream_t s);
// red[q][off + l] = basis_l^H w (l < nv_q), red[q][off + nv_q].x = ||w||^2; ns >= max nv_q + 1
void launch_dot_list(const VecItem* items_dev, int nq, int ns, long long N, void* partial, int nblk, void* red,
                     int rstride, int off, hipStream_t s);
void launch_update_list(const VecItem* items_dev, int nq, long long N, const void* red, int rstride, int off,
                        hipStream_t s);
void launch_axpy_list(const VecItem* items_dev, int nq, long long N, hipStream_t s);
int dot_blocks(long long N);
// red[r][off + l] = V_l^H w (l < nv), red[r][off + nv].x = ||w||^2 ; partial: [nrhs][nblk][nv+1] scratch
void launch_dot(const void* V, long long vstride, int nv, const void* w, long long N, int nrhs, void* partial,
                int nblk, void* red, int rstride, int off, hipStream_t s);
// w -= sum_l V_l red[r][off + l]
void launch_update(const void* V, long long vstride, int nv, const void* red, int rstride, int off, void* w,
                   long long N, int nrhs, hipStream_t s);
// y[r] = x[r] * sc[r] (sc: device doubles)
void launch_scale(const void* x, const void* sc, void* y, long long N, int nrhs, hipStream_t s);
// x[r] += sum_{l<nv} V_l[r] y[r][l]
void launch_axpy_basis(const void* V, long long vstride, int nv, const void* y, int ystride, void* x, long long N,
                       int nrhs, hipStream_t s);
// out[r] = mask[r] ? a[r] - b[r] : 0   (mask may be NULL)
void launch_sub(const void* a, const void* b, const int* mask, void* out, long long N, int nrhs, hipStream_t s);
void launch_add(void* x, const void* d, long long total, hipStream_t s);
// flag[r] set to 0 if b[r] has a non-finite entry (flag must be preset to 1)
void launch_finite(const void* b, long long N, int nrhs, int* flag, hipStream_t s);
}  // namespace emsurf
