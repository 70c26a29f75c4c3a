// Batched Stockham FFT along one lattice axis, for the circulant-embedded
// coupling product of Sec. IV-B (eq. (LJV5) and its 2-D generalisation).
//
// Layout: every transform point holds a contiguous run of batch columns
// (local unknowns u, or (rhs, u) pairs, or (v, u) kernel entries), so a
// workgroup owns BT consecutive columns of one line and all L points of the
// line; global loads and stores are coalesced along the batch.  The first
// radix stage reads global memory directly (skipping the zero padding:
// points >= n_in are never loaded), intermediate stages exchange through LDS
// in place, and the last stage writes global memory directly, dropping the
// points >= n_out (the crop of the inverse transform).
//
// Every thread holds VPT = L / G values of one column (G threads per column);
// radices 2, 4, 8 and 16 run as register butterflies.  The arithmetic type may
// differ from the input and output types (FP64 <-> FP32 converting loads and
// stores for the mixed-precision solve).
#include "internal.h"

#include <cmath>
#include <mutex>

namespace emsurf {
namespace {

template <typename V> struct Real;
template <> struct Real<float2> { using T = float; };
template <> struct Real<double2> { using T = double; };

template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
// multiply by sign*i
template <typename V> __device__ __forceinline__ V mul_si(V a, int sign) {
  return sign < 0 ? V{a.y, -a.x} : V{-a.y, a.x};
}
template <typename VO, typename VI> __device__ __forceinline__ VO cvt(VI a) {
  using R = typename Real<VO>::T;
  return VO{static_cast<R>(a.x), static_cast<R>(a.y)};
}

// cos and sin of 2*pi*j/16, j = 0..15, correctly rounded FP64 constants
__device__ constexpr double kC16[16] = {
    1.0, 0.92387953251128673848, 0.70710678118654757274, 0.38268343236508978178,
    0.0, -0.38268343236508978178, -0.70710678118654757274, -0.92387953251128673848,
    -1.0, -0.92387953251128673848, -0.70710678118654757274, -0.38268343236508978178,
    0.0, 0.38268343236508978178, 0.70710678118654757274, 0.92387953251128673848};
__device__ constexpr double kS16[16] = {
    0.0, 0.38268343236508978178, 0.70710678118654757274, 0.92387953251128673848,
    1.0, 0.92387953251128673848, 0.70710678118654757274, 0.38268343236508978178,
    0.0, -0.38268343236508978178, -0.70710678118654757274, -0.92387953251128673848,
    -1.0, -0.92387953251128673848, -0.70710678118654757274, -0.38268343236508978178};

// In-register DFT of length R (power of two <= 16): a[k] <- sum_n a[n] e^{sign 2 pi i n k / R}
template <int R, typename V>
__device__ __forceinline__ void dft(V (&a)[R], int sign) {
  using T = typename Real<V>::T;
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    V t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  } else {
    constexpr int H = R / 2;
    V e[H], o[H];
#pragma unroll
    for (int i = 0; i < H; ++i) { e[i] = a[2 * i]; o[i] = a[2 * i + 1]; }
    dft<H, V>(e, sign);
    dft<H, V>(o, sign);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      constexpr int step = 16 / R;
      const int j = k * step;  // angle 2 pi j / 16
      V t;
      if (j == 0) {
        t = o[k];
      } else if (j == 4) {
        t = mul_si(o[k], sign);
      } else {
        V w{static_cast<T>(kC16[j]), static_cast<T>(sign < 0 ? -kS16[j] : kS16[j])};
        t = cmul(w, o[k]);
      }
      a[k] = cadd(e[k], t);
      a[k + H] = csub(e[k], t);
    }
  }
}

struct PassArgs {
  int L, n_in, n_out, batch, nl0, G, BT, nst;
  int rad[6];
  long long in_s0, in_s1, out_s0, out_s1, in_pt, out_pt;
  int sign;
  double scale;
};

template <int R, int VPT, typename VI, typename VC, typename VO>
__device__ __forceinline__ void run_stage(const PassArgs& a, int s, int p, VC* lds, const VI* __restrict__ in,
                                          VO* __restrict__ out, const VC* __restrict__ tw, long long in_base,
                                          long long out_base, bool valid, int b, int g) {
  constexpr int NB = VPT / R;
  const int L = a.L;
  const int LR = L / R;
  const int G = a.G;
  const int BT = a.BT;
  VC v[NB][R];
  // ---- load
  if (s == 0) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int i = g + G * j;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int pos = i + q * LR;
        if (valid && pos < a.n_in)
          v[j][q] = cvt<VC>(in[in_base + (long long)pos * a.in_pt]);
        else
          v[j][q] = VC{0, 0};
      }
    }
  } else {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int i = g + G * j;
#pragma unroll
      for (int q = 0; q < R; ++q) v[j][q] = lds[(i + q * LR) * BT + b];
    }
    if (s < a.nst - 1) __syncthreads();
  }
  // ---- twiddle + butterfly
  const int tstride = L / (p * R);
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int i = g + G * j;
    const int k = i & (p - 1);
    if (s > 0) {
#pragma unroll
      for (int q = 1; q < R; ++q) {
        VC w = tw[(q * k * tstride) & (L - 1)];
        if (a.sign > 0) w.y = -w.y;
        v[j][q] = cmul(v[j][q], w);
      }
    }
    dft<R, VC>(v[j], a.sign);
  }
  // ---- store
  const bool last = (s == a.nst - 1);
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int i = g + G * j;
    const int k = i & (p - 1);
    const int base = (i - k) * R + k;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int pos = base + q * p;
      if (last) {
        if (valid && pos < a.n_out) {
          VC r = v[j][q];
          using T = typename Real<VC>::T;
          const T sc = static_cast<T>(a.scale);
          if (a.scale != 1.0) { r.x *= sc; r.y *= sc; }
          out[out_base + (long long)pos * a.out_pt] = cvt<VO>(r);
        }
      } else {
        lds[pos * BT + b] = v[j][q];
      }
    }
  }
}

template <int VPT, typename VI, typename VC, typename VO>
__global__ void __launch_bounds__(256) fft_pass_kernel(PassArgs a, const VI* __restrict__ in, VO* __restrict__ out,
                                const VC* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  VC* lds = reinterpret_cast<VC*>(smem_raw);
  const int t = threadIdx.x;
  const int b = t % a.BT;
  const int g = t / a.BT;
  const long long line = blockIdx.y;
  const long long l1 = line / a.nl0, l0 = line % a.nl0;
  const int col = blockIdx.x * a.BT + b;
  const bool valid = col < a.batch;
  const long long in_base = l1 * a.in_s1 + l0 * a.in_s0 + col;
  const long long out_base = l1 * a.out_s1 + l0 * a.out_s0 + col;
  int p = 1;
  for (int s = 0; s < a.nst; ++s) {
    const int R = a.rad[s];
    if constexpr (VPT >= 16) {
      if (R == 16) { run_stage<16, VPT>(a, s, p, lds, in, out, tw, in_base, out_base, valid, b, g); p *= 16; continue; }
    }
    if constexpr (VPT >= 8) {
      if (R == 8) { run_stage<8, VPT>(a, s, p, lds, in, out, tw, in_base, out_base, valid, b, g); p *= 8; continue; }
    }
    if constexpr (VPT >= 4) {
      if (R == 4) { run_stage<4, VPT>(a, s, p, lds, in, out, tw, in_base, out_base, valid, b, g); p *= 4; continue; }
    }
    run_stage<2, VPT>(a, s, p, lds, in, out, tw, in_base, out_base, valid, b, g);
    p *= 2;
  }
}

template <int VPT, typename VI, typename VC, typename VO>
void launch_vpt(const PassArgs& a, dim3 grid, int nt, size_t shm, const void* in, void* out, const void* tw,
                hipStream_t s) {
  hipLaunchKernelGGL((fft_pass_kernel<VPT, VI, VC, VO>), grid, dim3(nt), shm, s, a,
                     static_cast<const VI*>(in), static_cast<VO*>(out), static_cast<const VC*>(tw));
}

template <typename VI, typename VC, typename VO>
void launch_typed(const PassArgs& a, int vpt, dim3 grid, int nt, size_t shm, const void* in, void* out,
                  const void* tw, hipStream_t s) {
  switch (vpt) {
    case 16: launch_vpt<16, VI, VC, VO>(a, grid, nt, shm, in, out, tw, s); break;
    case 8: launch_vpt<8, VI, VC, VO>(a, grid, nt, shm, in, out, tw, s); break;
    case 4: launch_vpt<4, VI, VC, VO>(a, grid, nt, shm, in, out, tw, s); break;
    default: launch_vpt<2, VI, VC, VO>(a, grid, nt, shm, in, out, tw, s); break;
  }
}

std::mutex g_tw_mu;
std::map<std::pair<int, int>, DevBuf*> g_tw;

}  // namespace

const void* twiddle_table(int L, Cx t) {
  int dev = 0;
  EMS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_tw_mu);
  const int key_t = (t == Cx::C128 ? 1 : 0) + 2 * dev;
  auto it = g_tw.find({L, key_t});
  if (it != g_tw.end()) return it->second->p;
  std::vector<double> h64(2 * (size_t)L);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < L; ++j) {
    // exact symmetry reduction keeps every entry correctly rounded to FP64
    const long double ang = -2.0L * pi * (long double)j / (long double)L;
    h64[2 * j] = (double)cosl(ang);
    h64[2 * j + 1] = (double)sinl(ang);
  }
  DevBuf* buf = new DevBuf();
  if (t == Cx::C128) {
    buf->alloc(h64.size() * sizeof(double));
    EMS_HIP(hipMemcpy(buf->p, h64.data(), buf->bytes, hipMemcpyHostToDevice));
  } else {
    std::vector<float> h32(h64.size());
    for (size_t i = 0; i < h64.size(); ++i) h32[i] = (float)h64[i];
    buf->alloc(h32.size() * sizeof(float));
    EMS_HIP(hipMemcpy(buf->p, h32.data(), buf->bytes, hipMemcpyHostToDevice));
  }
  g_tw[{L, key_t}] = buf;
  return buf->p;
}

void launch_fft_pass(const FftPass& p, Cx tin, Cx tcomp, Cx tout, const void* in, void* out,
                     const void* twiddles, hipStream_t s) {
  EMS_CHECK_ARG(p.L >= 2 && p.L <= 1024 && (p.L & (p.L - 1)) == 0, "FFT length must be a power of two in [2, 1024]");
  EMS_CHECK_ARG(p.n_in >= 1 && p.n_in <= p.L && p.n_out >= 1 && p.n_out <= p.L, "FFT prune/crop sizes out of range");
  EMS_CHECK_ARG(p.batch >= 1 && p.n_lines >= 1 && p.nl0 >= 1, "FFT batch/lines must be positive");
  PassArgs a{};
  a.L = p.L;
  a.n_in = p.n_in;
  a.n_out = p.n_out;
  a.batch = p.batch;
  a.nl0 = p.nl0;
  a.in_s0 = p.in_s0; a.in_s1 = p.in_s1; a.out_s0 = p.out_s0; a.out_s1 = p.out_s1;
  a.in_pt = p.in_pt; a.out_pt = p.out_pt;
  a.sign = p.sign;
  a.scale = p.scale;
  const int vpt = p.L >= 16 ? 16 : p.L;
  a.G = p.L / vpt;
  // radix plan: 16s first, then the remainder
  int rem = p.L, nst = 0;
  while (rem >= 16 && vpt == 16) { a.rad[nst++] = 16; rem /= 16; }
  if (rem > 1) a.rad[nst++] = rem;   // rem in {2,4,8} (or L itself when L < 16)
  a.nst = nst;
  int bt = 256 / a.G;
  int bpow = 1;
  while (bpow < p.batch) bpow <<= 1;
  if (bt > bpow) bt = bpow;
  if (bt < 1) bt = 1;
  a.BT = bt;
  const int nt = a.BT * a.G;
  const size_t shm = (size_t)p.L * a.BT * cx_bytes(tcomp);
  const long long tiles = (p.batch + a.BT - 1) / a.BT;
  EMS_CHECK_ARG(tiles <= 0x7fffffffLL, "FFT batch too large");
  EMS_CHECK_ARG(p.n_lines <= 65535, "FFT pass has more than 65535 lines");
  dim3 grid((unsigned)tiles, (unsigned)p.n_lines, 1);
  if (tcomp == Cx::C128) {
    EMS_CHECK_ARG(tin == Cx::C128 && tout == Cx::C128, "FP64 FFT needs FP64 input and output");
    launch_typed<double2, double2, double2>(a, vpt, grid, nt, shm, in, out, twiddles, s);
  } else {
    if (tin == Cx::C128 && tout == Cx::C64)
      launch_typed<double2, float2, float2>(a, vpt, grid, nt, shm, in, out, twiddles, s);
    else if (tin == Cx::C64 && tout == Cx::C128)
      launch_typed<float2, float2, double2>(a, vpt, grid, nt, shm, in, out, twiddles, s);
    else if (tin == Cx::C64 && tout == Cx::C64)
      launch_typed<float2, float2, float2>(a, vpt, grid, nt, shm, in, out, twiddles, s);
    else
      launch_typed<double2, float2, double2>(a, vpt, grid, nt, shm, in, out, twiddles, s);
  }
  EMS_LAUNCH_CHECK();
}

}  // namespace emsurf
