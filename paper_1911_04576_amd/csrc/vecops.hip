// FP64 vector kernels of the batched GMRES solve (Sec. IV-A): Gram-Schmidt
// inner products against the Arnoldi basis, basis updates, norms, scalings
// and the solution update x += V y.  Vectors are c128 [nrhs][N]; the basis is
// [(m+1)][nrhs][N].  Reductions are two-stage and atomic-free (per-block
// partials, then a fixed-order sum), so results are bitwise reproducible and
// a right-hand side's numbers never depend on the other right-hand sides.
#include "internal.h"
#include "vecops.h"

namespace emsurf {
namespace {

constexpr int NT = 256;
constexpr int EPT = 8;                  // elements per thread per block chunk
constexpr int CHUNK = NT * EPT;

__device__ __forceinline__ double2 block_sum(double2 v, double2* sh) {
  // wave reduction then across the 4 waves of the block
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double2 r{0, 0};
  if (threadIdx.x == 0) {
    for (int i = 0; i < NT / 64; ++i) { r.x += sh[i].x; r.y += sh[i].y; }
  }
  __syncthreads();
  return r;
}

// partial[r][blk][l] = sum_chunk conj(V_l[r][i]) w[r][i] (l < nv); slot nv holds sum |w|^2.
__global__ void __launch_bounds__(NT) dot_kernel(const double2* __restrict__ V, long long vstride, int nv,
                                                 const double2* __restrict__ w, long long N, int nrhs,
                                                 double2* __restrict__ partial, int nblk) {
  __shared__ double2 sh[NT / 64];
  const int r = blockIdx.y;
  const int blk = blockIdx.x;
  const double2* wr = w + (long long)r * N;
  double2 wv[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const long long i = (long long)blk * CHUNK + e * NT + threadIdx.x;
    wv[e] = i < N ? wr[i] : double2{0, 0};
  }
  // whole vector may need several passes of the grid
  double2* out = partial + ((long long)r * nblk + blk) * (nv + 1);
  for (int l = 0; l < nv; ++l) {
    const double2* vr = V + l * vstride + (long long)r * N;
    double2 acc{0, 0};
    for (long long base = (long long)blk * CHUNK; base < N; base += (long long)nblk * CHUNK) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const long long i = base + e * NT + threadIdx.x;
        if (i < N) {
          const double2 a = vr[i];
          const double2 b = (base == (long long)blk * CHUNK) ? wv[e] : wr[i];
          acc.x += a.x * b.x + a.y * b.y;
          acc.y += a.x * b.y - a.y * b.x;
        }
      }
    }
    const double2 s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[l] = s;
  }
  double2 acc{0, 0};
  for (long long base = (long long)blk * CHUNK; base < N; base += (long long)nblk * CHUNK) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const long long i = base + e * NT + threadIdx.x;
      if (i < N) {
        const double2 b = (base == (long long)blk * CHUNK) ? wv[e] : wr[i];
        acc.x += b.x * b.x + b.y * b.y;
      }
    }
  }
  const double2 s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[nv] = s;
}

// red[r*rstride + off + l] = sum_blk partial[r][blk][l], l < ns (fixed order);
// grid (ns, nrhs)
__global__ void __launch_bounds__(NT) reduce_kernel(const double2* __restrict__ partial, int nblk, int ns,
                                                    double2* __restrict__ red, int rstride, int off) {
  __shared__ double2 sh[NT / 64];
  const int l = blockIdx.x, r = blockIdx.y;
  double2 acc{0, 0};
  for (int b = threadIdx.x; b < nblk; b += NT) {
    const double2 v = partial[((long long)r * nblk + b) * ns + l];
    acc.x += v.x;
    acc.y += v.y;
  }
  const double2 t = block_sum(acc, sh);
  if (threadIdx.x == 0) red[(long long)r * rstride + off + l] = t;
}

// w[r][i] -= sum_l V_l[r][i] c[r][l], c read from red[r*rstride + off + l]
__global__ void __launch_bounds__(NT) update_kernel(const double2* __restrict__ V, long long vstride, int nv,
                                                    const double2* __restrict__ red, int rstride, int off,
                                                    double2* __restrict__ w, long long N) {
  const int r = blockIdx.y;
  const double2* c = red + (long long)r * rstride + off;
  double2* wr = w + (long long)r * N;
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < N; i += (long long)gridDim.x * NT) {
    double2 acc = wr[i];
    for (int l = 0; l < nv; ++l) {
      const double2 a = V[l * vstride + (long long)r * N + i];
      const double2 h = c[l];
      acc.x -= a.x * h.x - a.y * h.y;
      acc.y -= a.x * h.y + a.y * h.x;
    }
    wr[i] = acc;
  }
}

// y[r][i] = x[r][i] * s[r]
__global__ void scale_kernel(const double2* __restrict__ x, const double* __restrict__ s, double2* __restrict__ y,
                             long long N) {
  const int r = blockIdx.y;
  const double f = s[r];
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < N; i += (long long)gridDim.x * NT) {
    const double2 a = x[(long long)r * N + i];
    y[(long long)r * N + i] = double2{a.x * f, a.y * f};
  }
}

// x[r][i] += sum_{l<nv} V_l[r][i] y[r][l]   (y: [nrhs][ystride])
__global__ void axpy_basis_kernel(const double2* __restrict__ V, long long vstride, int nv,
                                  const double2* __restrict__ y, int ystride, double2* __restrict__ x, long long N) {
  const int r = blockIdx.y;
  const double2* c = y + (long long)r * ystride;
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < N; i += (long long)gridDim.x * NT) {
    double2 acc = x[(long long)r * N + i];
    for (int l = 0; l < nv; ++l) {
      const double2 a = V[l * vstride + (long long)r * N + i];
      const double2 h = c[l];
      acc.x += a.x * h.x - a.y * h.y;
      acc.y += a.x * h.y + a.y * h.x;
    }
    x[(long long)r * N + i] = acc;
  }
}

// out[r][i] = mask[r] ? a[r][i] - b[r][i] : 0
__global__ void sub_kernel(const double2* __restrict__ a, const double2* __restrict__ b,
                           const int* __restrict__ mask, double2* __restrict__ out, long long N) {
  const int r = blockIdx.y;
  const bool on = mask == nullptr || mask[r] != 0;
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < N; i += (long long)gridDim.x * NT) {
    const long long j = (long long)r * N + i;
    out[j] = on ? double2{a[j].x - b[j].x, a[j].y - b[j].y} : double2{0, 0};
  }
}

// x[r][i] += d[r][i]
__global__ void add_kernel(double2* __restrict__ x, const double2* __restrict__ d, long long total) {
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < total; i += (long long)gridDim.x * NT) {
    x[i].x += d[i].x;
    x[i].y += d[i].y;
  }
}

// every entry finite?  flag[r] = 0 if any entry of b[r] is not finite
__global__ void finite_kernel(const double2* __restrict__ b, long long N, int* __restrict__ flag) {
  const int r = blockIdx.y;
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < N; i += (long long)gridDim.x * NT) {
    const double2 v = b[(long long)r * N + i];
    if (!isfinite(v.x) || !isfinite(v.y)) flag[r] = 0;
  }
}

unsigned stream_blocks(long long N) {
  long long g = (N + NT - 1) / NT;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

int dot_blocks(long long N) {
  long long b = (N + CHUNK - 1) / CHUNK;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

void launch_dot(const void* V, long long vstride, int nv, const void* w, long long N, int nrhs, void* partial,
                int nblk, void* red, int rstride, int off, hipStream_t s) {
  hipLaunchKernelGGL(dot_kernel, dim3(nblk, nrhs), dim3(NT), 0, s, static_cast<const double2*>(V), vstride, nv,
                     static_cast<const double2*>(w), N, nrhs, static_cast<double2*>(partial), nblk);
  EMS_LAUNCH_CHECK();
  hipLaunchKernelGGL(reduce_kernel, dim3(nv + 1, nrhs), dim3(NT), 0, s, static_cast<const double2*>(partial), nblk,
                     nv + 1, static_cast<double2*>(red), rstride, off);
  EMS_LAUNCH_CHECK();
}

void launch_update(const void* V, long long vstride, int nv, const void* red, int rstride, int off, void* w,
                   long long N, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(update_kernel, dim3(stream_blocks(N), nrhs), dim3(NT), 0, s, static_cast<const double2*>(V),
                     vstride, nv, static_cast<const double2*>(red), rstride, off, static_cast<double2*>(w), N);
  EMS_LAUNCH_CHECK();
}

void launch_scale(const void* x, const void* sc, void* y, long long N, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(stream_blocks(N), nrhs), dim3(NT), 0, s, static_cast<const double2*>(x),
                     static_cast<const double*>(sc), static_cast<double2*>(y), N);
  EMS_LAUNCH_CHECK();
}

void launch_axpy_basis(const void* V, long long vstride, int nv, const void* y, int ystride, void* x, long long N,
                       int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(axpy_basis_kernel, dim3(stream_blocks(N), nrhs), dim3(NT), 0, s,
                     static_cast<const double2*>(V), vstride, nv, static_cast<const double2*>(y), ystride,
                     static_cast<double2*>(x), N);
  EMS_LAUNCH_CHECK();
}

void launch_sub(const void* a, const void* b, const int* mask, void* out, long long N, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(sub_kernel, dim3(stream_blocks(N), nrhs), dim3(NT), 0, s, static_cast<const double2*>(a),
                     static_cast<const double2*>(b), mask, static_cast<double2*>(out), N);
  EMS_LAUNCH_CHECK();
}

void launch_add(void* x, const void* d, long long total, hipStream_t s) {
  hipLaunchKernelGGL(add_kernel, dim3(stream_blocks(total)), dim3(NT), 0, s, static_cast<double2*>(x),
                     static_cast<const double2*>(d), total);
  EMS_LAUNCH_CHECK();
}

void launch_finite(const void* b, long long N, int nrhs, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(finite_kernel, dim3(stream_blocks(N), nrhs), dim3(NT), 0, s, static_cast<const double2*>(b), N,
                     flag);
  EMS_LAUNCH_CHECK();
}

}  // namespace emsurf

// ----------------------------------------------------------------------------- pointer-list forms
// Continuous batching runs one kernel over a list of independent vectors that
// live at arbitrary places (each slot's own Krylov basis); item q of a list
// carries its own pointers and sizes.  Same arithmetic per item as above, so a
// slot's numbers do not depend on which other slots share the launch.
namespace emsurf {
namespace {

__global__ void copy_list_kernel(const VecItem* __restrict__ items, long long N) {
  const VecItem it = items[blockIdx.y];
  const double2* a = reinterpret_cast<const double2*>(it.a);
  const double2* b = reinterpret_cast<const double2*>(it.b);
  double2* d = reinterpret_cast<double2*>(it.dst);
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < N; i += (long long)gridDim.x * NT) {
    double2 v = a[i];
    if (b) { v.x = b[i].x - v.x; v.y = b[i].y - v.y; }   // dst = b - a
    if (it.scale != 1.0) { v.x *= it.scale; v.y *= it.scale; }
    d[i] = v;
  }
}

// partial[q][blk][l] = sum conj(basis_l) w (l < nv_q), slot nv_q: sum |w|^2; layout stride ns
__global__ void __launch_bounds__(NT) dot_list_kernel(const VecItem* __restrict__ items, long long N, int ns,
                                                      double2* __restrict__ partial, int nblk) {
  __shared__ double2 sh[NT / 64];
  const VecItem it = items[blockIdx.y];
  const int blk = blockIdx.x;
  const double2* V = reinterpret_cast<const double2*>(it.a);
  const double2* w = reinterpret_cast<const double2*>(it.dst);
  double2* out = partial + ((long long)blockIdx.y * nblk + blk) * ns;
  for (int l = 0; l <= it.nv; ++l) {
    double2 acc{0, 0};
    for (long long base = (long long)blk * CHUNK; base < N; base += (long long)nblk * CHUNK) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const long long i = base + e * NT + threadIdx.x;
        if (i < N) {
          const double2 b = w[i];
          if (l < it.nv) {
            const double2 a = V[(long long)l * N + i];
            acc.x += a.x * b.x + a.y * b.y;
            acc.y += a.x * b.y - a.y * b.x;
          } else {
            acc.x += b.x * b.x + b.y * b.y;
          }
        }
      }
    }
    const double2 s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[l] = s;
  }
}

// red[q][off + l] = sum_blk partial[q][blk][l], l < ns; grid (ns, nq)
__global__ void __launch_bounds__(NT) reduce_list_kernel(const double2* __restrict__ partial, int nblk, int ns,
                                                         double2* __restrict__ red, int rstride, int off) {
  __shared__ double2 sh[NT / 64];
  const int l = blockIdx.x, q = blockIdx.y;
  double2 acc{0, 0};
  for (int b = threadIdx.x; b < nblk; b += NT) {
    const double2 v = partial[((long long)q * nblk + b) * ns + l];
    acc.x += v.x;
    acc.y += v.y;
  }
  const double2 t = block_sum(acc, sh);
  if (threadIdx.x == 0) red[(long long)q * rstride + off + l] = t;
}

// w -= sum_{l < nv} basis_l red[q][off + l]
__global__ void __launch_bounds__(NT) update_list_kernel(const VecItem* __restrict__ items, long long N,
                                                         const double2* __restrict__ red, int rstride, int off) {
  const VecItem it = items[blockIdx.y];
  const double2* V = reinterpret_cast<const double2*>(it.a);
  double2* w = reinterpret_cast<double2*>(it.dst);
  const double2* c = red + (long long)blockIdx.y * rstride + off;
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < N; i += (long long)gridDim.x * NT) {
    double2 acc = w[i];
    for (int l = 0; l < it.nv; ++l) {
      const double2 a = V[(long long)l * N + i];
      const double2 h = c[l];
      acc.x -= a.x * h.x - a.y * h.y;
      acc.y -= a.x * h.y + a.y * h.x;
    }
    w[i] = acc;
  }
}

// x += sum_{l < nv} basis_l y_l, y = items[q].coef[0..nv)
__global__ void axpy_list_kernel(const VecItem* __restrict__ items, long long N) {
  const VecItem it = items[blockIdx.y];
  const double2* V = reinterpret_cast<const double2*>(it.a);
  const double2* y = reinterpret_cast<const double2*>(it.b);
  double2* x = reinterpret_cast<double2*>(it.dst);
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < N; i += (long long)gridDim.x * NT) {
    double2 acc = x[i];
    for (int l = 0; l < it.nv; ++l) {
      const double2 a = V[(long long)l * N + i];
      const double2 h = y[l];
      acc.x += a.x * h.x - a.y * h.y;
      acc.y += a.x * h.y + a.y * h.x;
    }
    x[i] = acc;
  }
}

}  // namespace

void launch_copy_list(const VecItem* items_dev, int nq, long long N, hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(copy_list_kernel, dim3(stream_blocks(N), nq), dim3(NT), 0, s, items_dev, N);
  EMS_LAUNCH_CHECK();
}

void launch_dot_list(const VecItem* items_dev, int nq, int ns, long long N, void* partial, int nblk, void* red,
                     int rstride, int off, hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(dot_list_kernel, dim3(nblk, nq), dim3(NT), 0, s, items_dev, N, ns,
                     static_cast<double2*>(partial), nblk);
  EMS_LAUNCH_CHECK();
  hipLaunchKernelGGL(reduce_list_kernel, dim3(ns, nq), dim3(NT), 0, s, static_cast<const double2*>(partial), nblk,
                     ns, static_cast<double2*>(red), rstride, off);
  EMS_LAUNCH_CHECK();
}

void launch_update_list(const VecItem* items_dev, int nq, long long N, const void* red, int rstride, int off,
                        hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(update_list_kernel, dim3(stream_blocks(N), nq), dim3(NT), 0, s, items_dev, N,
                     static_cast<const double2*>(red), rstride, off);
  EMS_LAUNCH_CHECK();
}

void launch_axpy_list(const VecItem* items_dev, int nq, long long N, hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(axpy_list_kernel, dim3(stream_blocks(N), nq), dim3(NT), 0, s, items_dev, N);
  EMS_LAUNCH_CHECK();
}

}  // namespace emsurf
