// Ring DFT kernels: the longitude step of the SHT (the "2 pi * FFT_1D_R2C
// along W, then keep m < mmax" of Alg. 1) and its inverse.
//
// Design (gfx950):
//  * A workgroup owns one ring pair (k, nlat-1-k) for `fg` fields.  The two
//    real rings of a field are packed as one complex sequence z = u_k + i u_k'
//    (the mirrored ring), so one complex FFT of length nlon yields both real
//    spectra, and the pair is exactly what the equatorial fold of the
//    Legendre step needs: S = X_k + X_k' and A = X_k - X_k'.
//  * The complex FFT is a mixed-radix (4, 2, 3, 5) Stockham autosort in LDS
//    (ping-pong buffers, no bit reversal), each thread doing radix-R
//    butterflies in registers with twiddles from a float32 table built in
//    float64 on the host.
//  * Grid rows are read / written as contiguous nlon-float runs; the
//    workspace is written / read as fg*8-byte runs per (m, parity, ring).
#include "internal.h"

namespace sht {
namespace {

struct DftArgs {
  int nlat, nlon, lmax, mmax, nk, F, kpad, npad, fg;
  int nstages;
  int radix[kMaxRadices];
  float c_rest;
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by +i (sg = +1) or -i (sg = -1)
__device__ __forceinline__ float2 mul_i(float2 a, float sg) { return make_float2(-sg * a.y, sg * a.x); }

// In-register DFT of length R: A_s = sum_q a_q e^{sg 2 pi i q s / R}.
template <int R>
__device__ __forceinline__ void codelet(float2* a, float sg);

template <>
__device__ __forceinline__ void codelet<2>(float2* a, float) {
  const float2 t = a[1];
  a[1] = csub(a[0], t);
  a[0] = cadd(a[0], t);
}

template <>
__device__ __forceinline__ void codelet<4>(float2* a, float sg) {
  const float2 s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
  const float2 s13 = cadd(a[1], a[3]), d13 = mul_i(csub(a[1], a[3]), sg);
  a[0] = cadd(s02, s13);
  a[2] = csub(s02, s13);
  a[1] = cadd(d02, d13);
  a[3] = csub(d02, d13);
}

template <>
__device__ __forceinline__ void codelet<3>(float2* a, float sg) {
  const float h = 0.86602540378443864676f;  // sin(2 pi / 3)
  const float2 t = cadd(a[1], a[2]);
  const float2 d = mul_i(cscale(csub(a[1], a[2]), h), sg);
  const float2 b = make_float2(a[0].x - 0.5f * t.x, a[0].y - 0.5f * t.y);
  a[0] = cadd(a[0], t);
  a[1] = cadd(b, d);
  a[2] = csub(b, d);
}

template <>
__device__ __forceinline__ void codelet<5>(float2* a, float sg) {
  const float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
  const float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
  const float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
  const float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
  const float2 t1 = cadd(a[1], a[4]), d1 = csub(a[1], a[4]);
  const float2 t2 = cadd(a[2], a[3]), d2 = csub(a[2], a[3]);
  const float2 r1 = make_float2(a[0].x + c1 * t1.x + c2 * t2.x, a[0].y + c1 * t1.y + c2 * t2.y);
  const float2 r2 = make_float2(a[0].x + c2 * t1.x + c1 * t2.x, a[0].y + c2 * t1.y + c1 * t2.y);
  const float2 i1 = mul_i(make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y), sg);
  const float2 i2 = mul_i(make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y), sg);
  a[0] = make_float2(a[0].x + t1.x + t2.x, a[0].y + t1.y + t2.y);
  a[1] = cadd(r1, i1);
  a[4] = csub(r1, i1);
  a[2] = cadd(r2, i2);
  a[3] = csub(r2, i2);
}

// One radix-R Stockham butterfly: inputs src[tt + q*nb], twiddled by
// w^(q*kk) with w = e^{sg 2 pi i / (p R)}, outputs dst[(tt-kk)*R + kk + q*p].
template <int R>
__device__ __forceinline__ void butterfly(const float2* __restrict__ src, float2* __restrict__ dst,
                                          int tt, int nb, int kk, int p, int tstride,
                                          const float2* __restrict__ tw, float sg) {
  float2 a[R];
#pragma unroll
  for (int q = 0; q < R; ++q) a[q] = src[tt + q * nb];
  if (kk != 0) {
#pragma unroll
    for (int q = 1; q < R; ++q) {
      float2 w = tw[q * kk * tstride];
      w.y *= sg < 0.f ? 1.f : -1.f;  // table holds e^{-2 pi i j / N}
      a[q] = cmul(a[q], w);
    }
  }
  codelet<R>(a, sg);
  const int ob = (tt - kk) * R + kk;
#pragma unroll
  for (int q = 0; q < R; ++q) dst[ob + q * p] = a[q];
}

// fg independent complex FFTs of length N held in LDS at src (fg * N
// entries); returns the buffer holding the result.  sg = -1: forward.
__device__ float2* fft_lds(float2* src, float2* dst, const DftArgs& a, const float2* __restrict__ tw,
                           float sg) {
  const int N = a.nlon;
  int p = 1;
  for (int s = 0; s < a.nstages; ++s) {
    const int R = a.radix[s];
    const int nb = N / R;
    const int tstride = N / (p * R);
    const int total = a.fg * nb;
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
      const int f = t / nb;
      const int tt = t - f * nb;
      const int kk = tt % p;
      const float2* in = src + f * N;
      float2* out = dst + f * N;
      switch (R) {
        case 4: butterfly<4>(in, out, tt, nb, kk, p, tstride, tw, sg); break;
        case 2: butterfly<2>(in, out, tt, nb, kk, p, tstride, tw, sg); break;
        case 3: butterfly<3>(in, out, tt, nb, kk, p, tstride, tw, sg); break;
        default: butterfly<5>(in, out, tt, nb, kk, p, tstride, tw, sg); break;
      }
    }
    __syncthreads();
    float2* t = src;
    src = dst;
    dst = t;
    p *= R;
  }
  return src;
}

__global__ __launch_bounds__(256) void dft_forward_kernel(DftArgs a, const float* __restrict__ x,
                                                          float* __restrict__ W,
                                                          const float2* __restrict__ tw,
                                                          const float* __restrict__ ring_scale) {
  extern __shared__ float2 lds[];
  const int N = a.nlon;
  float2* b0 = lds;
  float2* b1 = lds + a.fg * N;
  const int kk = blockIdx.x;
  const int ks = a.nlat - 1 - kk;
  const bool eq = (ks == kk);
  const int f0 = blockIdx.y * a.fg;
  for (int idx = threadIdx.x; idx < a.fg * N; idx += blockDim.x) {
    const int f = idx / N;
    const int j = idx - f * N;
    const int fi = f0 + f;
    float re = 0.f, im = 0.f;
    if (fi < a.F) {
      re = x[(static_cast<size_t>(fi) * a.nlat + kk) * N + j];
      if (!eq) im = x[(static_cast<size_t>(fi) * a.nlat + ks) * N + j];
    }
    b0[idx] = make_float2(re, im);
  }
  __syncthreads();
  const float2* Z = fft_lds(b0, b1, a, tw, -1.f);
  const float sc = ring_scale[kk];
  for (int idx = threadIdx.x; idx < a.fg * a.mmax; idx += blockDim.x) {
    const int f = idx % a.fg;
    const int m = idx / a.fg;
    const int fi = f0 + f;
    if (fi >= a.F) continue;
    const float2 zm = Z[f * N + m];
    const float2 zr = Z[f * N + (m == 0 ? 0 : N - m)];
    // spectra of the two packed real rings
    const float2 xn = make_float2(0.5f * (zm.x + zr.x), 0.5f * (zm.y - zr.y));
    const float2 xs = make_float2(0.5f * (zm.y + zr.y), -0.5f * (zm.x - zr.x));
    float2 S, A;
    if (eq) {
      S = cscale(xn, sc);
      A = make_float2(0.f, 0.f);
    } else {
      S = cscale(cadd(xn, xs), sc);
      A = cscale(csub(xn, xs), sc);
    }
    if (m == 0) {
      S.y = 0.f;
      A.y = 0.f;
    }
    const size_t col = 2 * static_cast<size_t>(fi);
    const size_t r0 = (static_cast<size_t>(2 * m) * a.kpad + kk) * a.npad + col;
    const size_t r1 = (static_cast<size_t>(2 * m + 1) * a.kpad + kk) * a.npad + col;
    *reinterpret_cast<float2*>(W + r0) = S;
    *reinterpret_cast<float2*>(W + r1) = A;
  }
}

__global__ __launch_bounds__(256) void dft_inverse_kernel(DftArgs a, const float* __restrict__ W,
                                                          float* __restrict__ x,
                                                          const float2* __restrict__ tw,
                                                          const float* __restrict__ ring_scale) {
  extern __shared__ float2 lds[];
  const int N = a.nlon;
  float2* b0 = lds;
  float2* b1 = lds + a.fg * N;
  const int kk = blockIdx.x;
  const int ks = a.nlat - 1 - kk;
  const bool eq = (ks == kk);
  const int f0 = blockIdx.y * a.fg;
  for (int idx = threadIdx.x; idx < a.fg * N; idx += blockDim.x) b0[idx] = make_float2(0.f, 0.f);
  __syncthreads();
  const float h = 0.5f * a.c_rest;
  for (int idx = threadIdx.x; idx < a.fg * a.mmax; idx += blockDim.x) {
    const int f = idx % a.fg;
    const int m = idx / a.fg;
    const int fi = f0 + f;
    if (fi >= a.F) continue;
    const size_t col = 2 * static_cast<size_t>(fi);
    const float2 E = *reinterpret_cast<const float2*>(W + (static_cast<size_t>(2 * m) * a.kpad + kk) * a.npad + col);
    // order m has odd-parity degrees only when l = m + 1 < lmax; otherwise
    // the synthesis never writes that plane and it must read as zero
    const float2 O = (m + 1 < a.lmax)
        ? *reinterpret_cast<const float2*>(W + (static_cast<size_t>(2 * m + 1) * a.kpad + kk) * a.npad + col)
        : make_float2(0.f, 0.f);
    const float2 yn = cadd(E, O);
    const float2 ys = eq ? make_float2(0.f, 0.f) : csub(E, O);
    if (m == 0) {
      b0[f * N] = make_float2(yn.x, ys.x);
    } else {
      const float2 hn = cscale(yn, h), hs = cscale(ys, h);
      b0[f * N + m] = make_float2(hn.x - hs.y, hn.y + hs.x);
      b0[f * N + N - m] = make_float2(hn.x + hs.y, -hn.y + hs.x);
    }
  }
  __syncthreads();
  const float2* Z = fft_lds(b0, b1, a, tw, 1.f);
  const float sc = ring_scale[kk];
  for (int idx = threadIdx.x; idx < a.fg * N; idx += blockDim.x) {
    const int f = idx / N;
    const int j = idx - f * N;
    const int fi = f0 + f;
    if (fi >= a.F) continue;
    const float2 z = Z[idx];
    x[(static_cast<size_t>(fi) * a.nlat + kk) * N + j] = z.x * sc;
    if (!eq) x[(static_cast<size_t>(fi) * a.nlat + ks) * N + j] = z.y * sc;
  }
}

int pick_fg(int n, int F) {
  // two ping-pong buffers of fg * n complex floats within 64 KiB of LDS
  int fg = 65536 / (16 * n);
  if (fg > 16) fg = 16;
  if (fg > F) fg = F;
  if (fg < 1) fg = 1;
  return fg;
}

DftArgs make_args(const SegGeom& g, const DftPlan& dp) {
  DftArgs a{};
  a.nlat = g.nlat;
  a.nlon = g.nlon;
  a.lmax = g.lmax;
  a.mmax = g.mmax;
  a.nk = g.nk;
  a.F = g.F;
  a.kpad = g.kpad;
  a.npad = g.npad;
  a.fg = pick_fg(g.nlon, g.F);
  a.nstages = dp.nstages;
  for (int i = 0; i < kMaxRadices; ++i) a.radix[i] = dp.radix[i];
  return a;
}

}  // namespace

bool make_dft_plan(int n, DftPlan* p) {
  p->n = n;
  p->nstages = 0;
  int r = n;
  const int order[4] = {4, 2, 3, 5};
  for (int i = 0; i < 4; ++i) {
    while (r % order[i] == 0) {
      if (p->nstages >= kMaxRadices) return false;
      p->radix[p->nstages++] = order[i];
      r /= order[i];
    }
  }
  for (int i = p->nstages; i < kMaxRadices; ++i) p->radix[i] = 1;
  return r == 1;
}

hipError_t launch_dft_forward(const SegGeom& g, const DftPlan& dp, const float* x, float* W,
                              const float2* tw, const float* ring_scale, hipStream_t st) {
  DftArgs a = make_args(g, dp);
  dim3 grid(g.nk, (g.F + a.fg - 1) / a.fg);
  const size_t lds = 2 * static_cast<size_t>(a.fg) * g.nlon * sizeof(float2);
  hipLaunchKernelGGL(dft_forward_kernel, grid, dim3(256), lds, st, a, x, W, tw, ring_scale);
  return hipGetLastError();
}

hipError_t launch_dft_inverse(const SegGeom& g, const DftPlan& dp, const float* W, float* x,
                              const float2* tw, const float* ring_scale, float c_rest,
                              hipStream_t st) {
  DftArgs a = make_args(g, dp);
  a.c_rest = c_rest;
  dim3 grid(g.nk, (g.F + a.fg - 1) / a.fg);
  const size_t lds = 2 * static_cast<size_t>(a.fg) * g.nlon * sizeof(float2);
  hipLaunchKernelGGL(dft_inverse_kernel, grid, dim3(256), lds, st, a, W, x, tw, ring_scale);
  return hipGetLastError();
}

}  // namespace sht
