// Ring DFT kernels: the longitude step of the SHT (the "2 pi * FFT_1D_R2C
// along W, then keep m < mmax" of Alg. 1) and its inverse.
//
// Design (gfx950):
//  * A workgroup owns one ring pair (k, nlat-1-k) for 4 fields.  The two
//    real rings of a field are packed as one complex sequence z = u_k + i u_k'
//    (the mirrored ring), so one complex FFT of length nlon yields both real
//    spectra, and the pair is exactly what the equatorial fold of the
//    Legendre step needs: S = X_k + X_k' and A = X_k - X_k'.
//  * The complex FFT is a Stockham autosort in LDS.  For the grid widths of
//    the 0.25/0.5/1 degree and small test grids (1440, 720, 360, 64) it runs
//    three (two) in-place passes of radix 9/10/16-type butterflies, each a
//    composite DFT held in registers; other widths 2^a 3^b 5^c take a
//    runtime-radix (2, 3, 4, 5) ping-pong path.
//  * Workspace layout W[m][p][g][k][16]: g = group of 8 fields, 16 floats =
//    (re, im) of those fields.  A workgroup writes / reads 32-byte runs; the
//    block order is remapped so that the workgroups completing one 128-byte
//    line run together on the same XCD (which merges them in its L2).
#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "kernel_common.h"

namespace sht {
namespace {

constexpr int FGW = 4;     // fields per workgroup
constexpr int NT = 512;    // threads per workgroup

struct DftArgs {
  int nlat, nlon, lmax, mmax, nk, F, kpad, G;
  long long wslab;         // floats per (m, parity) slab of W
  int nitems;              // G * nk * 2 workgroup items
  int nstages;
  const int* radix;        // the segment's radix plan (device memory)
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

// cos / sin of 2 pi e / R for the composite radices (e < R).
template <int R>
__device__ __forceinline__ float root_cos(int e);
template <int R>
__device__ __forceinline__ float root_sin(int e);

#define SHT_ROOTS(R, ...)                                                    \
  template <>                                                                \
  __device__ __forceinline__ float root_cos<R>(int e) {                      \
    constexpr float c[R] = {__VA_ARGS__};                                    \
    return c[e];                                                             \
  }
SHT_ROOTS(8, 1.f, 0.70710678118654752f, 0.f, -0.70710678118654752f, -1.f, -0.70710678118654752f, 0.f,
          0.70710678118654752f)
SHT_ROOTS(9, 1.f, 0.76604444311897804f, 0.17364817766693035f, -0.5f, -0.93969262078590838f,
          -0.93969262078590838f, -0.5f, 0.17364817766693035f, 0.76604444311897804f)
SHT_ROOTS(10, 1.f, 0.80901699437494742f, 0.30901699437494742f, -0.30901699437494742f, -0.80901699437494742f,
          -1.f, -0.80901699437494742f, -0.30901699437494742f, 0.30901699437494742f, 0.80901699437494742f)
SHT_ROOTS(16, 1.f, 0.92387953251128676f, 0.70710678118654752f, 0.38268343236508977f, 0.f,
          -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128676f, -1.f, -0.92387953251128676f,
          -0.70710678118654752f, -0.38268343236508977f, 0.f, 0.38268343236508977f, 0.70710678118654752f,
          0.92387953251128676f)
#undef SHT_ROOTS
// sin(2 pi e / R) = cos(2 pi (e - R/4) / R) for R divisible by 4; listed
// explicitly for the odd-quarter radices.
template <>
__device__ __forceinline__ float root_sin<8>(int e) {
  constexpr float s[8] = {0.f, 0.70710678118654752f, 1.f, 0.70710678118654752f, 0.f, -0.70710678118654752f, -1.f,
                          -0.70710678118654752f};
  return s[e];
}
template <>
__device__ __forceinline__ float root_sin<9>(int e) {
  constexpr float s[9] = {0.f, 0.64278760968653933f, 0.98480775301220806f, 0.86602540378443865f,
                          0.34202014332566873f, -0.34202014332566873f, -0.86602540378443865f,
                          -0.98480775301220806f, -0.64278760968653933f};
  return s[e];
}
template <>
__device__ __forceinline__ float root_sin<10>(int e) {
  constexpr float s[10] = {0.f, 0.58778525229247313f, 0.95105651629515357f, 0.95105651629515357f,
                           0.58778525229247313f, 0.f, -0.58778525229247313f, -0.95105651629515357f,
                           -0.95105651629515357f, -0.58778525229247313f};
  return s[e];
}
template <>
__device__ __forceinline__ float root_sin<16>(int e) {
  constexpr float s[16] = {0.f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128676f, 1.f,
                           0.92387953251128676f, 0.70710678118654752f, 0.38268343236508977f, 0.f,
                           -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128676f, -1.f,
                           -0.92387953251128676f, -0.70710678118654752f, -0.38268343236508977f};
  return s[e];
}

// In-register DFT of length R: A_s = sum_q a_q e^{sg 2 pi i q s / R}.
template <int R>
struct Codelet;

template <>
struct Codelet<2> {
  __device__ static __forceinline__ void run(float2* a, float) {
    const float2 t = a[1];
    a[1] = csub(a[0], t);
    a[0] = cadd(a[0], t);
  }
};

template <>
struct Codelet<4> {
  __device__ static __forceinline__ void run(float2* a, float sg) {
    const float2 s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
    const float2 s13 = cadd(a[1], a[3]), d13 = mul_i(csub(a[1], a[3]), sg);
    a[0] = cadd(s02, s13);
    a[2] = csub(s02, s13);
    a[1] = cadd(d02, d13);
    a[3] = csub(d02, d13);
  }
};

template <>
struct Codelet<3> {
  __device__ static __forceinline__ void run(float2* a, float sg) {
    const float h = 0.86602540378443864676f;  // sin(2 pi / 3)
    const float2 t = cadd(a[1], a[2]);
    const float2 d = mul_i(cscale(csub(a[1], a[2]), h), sg);
    const float2 b = make_float2(a[0].x - 0.5f * t.x, a[0].y - 0.5f * t.y);
    a[0] = cadd(a[0], t);
    a[1] = cadd(b, d);
    a[2] = csub(b, d);
  }
};

template <>
struct Codelet<5> {
  __device__ static __forceinline__ void run(float2* a, float sg) {
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
};

// Composite R = R1 * R2 (Cooley-Tukey in registers): inputs n = R2 n1 + n2,
// outputs k = k1 + R1 k2, inner twiddles e^{sg 2 pi i n2 k1 / R}.
template <int R1, int R2>
struct Composite {
  __device__ static __forceinline__ void run(float2* a, float sg) {
    constexpr int R = R1 * R2;
    float2 t[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      float2 u[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) u[n1] = a[R2 * n1 + n2];
      Codelet<R1>::run(u, sg);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) {
        const int e = (n2 * k1) % R;
        if (e == 0) {
          t[n2 * R1 + k1] = u[k1];
        } else {
          t[n2 * R1 + k1] = cmul(u[k1], make_float2(root_cos<R>(e), sg * root_sin<R>(e)));
        }
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      float2 u[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) u[n2] = t[n2 * R1 + k1];
      Codelet<R2>::run(u, sg);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) a[k1 + R1 * k2] = u[k2];
    }
  }
};

template <>
struct Codelet<8> : Composite<2, 4> {};
template <>
struct Codelet<9> : Composite<3, 3> {};
template <>
struct Codelet<10> : Composite<2, 5> {};
template <>
struct Codelet<16> : Composite<4, 4> {};

// Twiddles e^{-2 pi i e / N} from a two-level table in LDS: T1[i] =
// w^{32 i} (i < ceil(N/32)) followed by T2[j] = w^j (j < 32), both copied
// from the float64-rounded global table; w^e = T1[e / 32] T2[e % 32].  The
// FFT passes read them from LDS instead of issuing a chain of dependent
// global loads per butterfly.
__host__ __device__ constexpr int twiddle_lds_entries(int n) { return (n + 31) / 32 + 32; }
__device__ __forceinline__ void load_twiddles(float2* ltw, int n, const float2* __restrict__ tw) {
  const int n1 = (n + 31) / 32;
  for (int i = threadIdx.x; i < n1 + 32; i += blockDim.x) ltw[i] = i < n1 ? tw[32 * i] : tw[(i - n1) % n];
}
__device__ __forceinline__ float2 twiddle(const float2* ltw, int n, int e) {
  const int n1 = (n + 31) / 32;
  return cmul(ltw[e >> 5], ltw[n1 + (e & 31)]);
}

// One in-place Stockham pass of radix R over FGW sequences of length N held
// in LDS; P is the product of the radices of the earlier passes.  Every
// thread first gathers the inputs of all its butterflies into registers,
// then (after a barrier) overwrites the buffer with their outputs.
template <int N, int R, int P>
__device__ __forceinline__ void pass_inplace(float2* buf, const float2* ltw, float sg) {
  constexpr int NB = N / R;
  constexpr int TOT = FGW * NB;
  constexpr int PER = (TOT + NT - 1) / NT;
  constexpr int TS = N / (P * R);
  float2 v[PER][R];
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int bi = threadIdx.x + b * NT;
    if (bi < TOT) {
      const int f = bi / NB;
      const int t = bi - f * NB;
#pragma unroll
      for (int q = 0; q < R; ++q) v[b][q] = buf[f * N + t + q * NB];
    }
  }
  lds_barrier();
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int bi = threadIdx.x + b * NT;
    if (bi < TOT) {
      const int f = bi / NB;
      const int t = bi - f * NB;
      const int k = t % P;
      if (P > 1 && k != 0) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          float2 w = twiddle(ltw, N, q * k * TS);
          if (sg > 0.f) w.y = -w.y;  // table holds e^{-2 pi i j / N}
          v[b][q] = cmul(v[b][q], w);
        }
      }
      Codelet<R>::run(v[b], sg);
      const int ob = f * N + (t - k) * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) buf[ob + q * P] = v[b][q];
    }
  }
  lds_barrier();
}

template <int N_, int R1, int R2, int R3>
struct FastFFT {
  static constexpr int N = N_;
  static constexpr int kLdsComplex = FGW * N;  // single in-place buffer
  // twiddle table in LDS right after the FFT buffer
  static constexpr size_t kLdsBytes = (static_cast<size_t>(kLdsComplex) + twiddle_lds_entries(N)) * sizeof(float2);
  __device__ static __forceinline__ void prepare(float2* buf, const DftArgs&, const float2* __restrict__ tw) {
    load_twiddles(buf + kLdsComplex, N, tw);
  }
  __device__ static __forceinline__ float2* run(float2* buf, const DftArgs&, const float2* __restrict__,
                                                float sg) {
    static_assert(R1 * R2 * R3 == N, "radix plan");
    const float2* ltw = buf + kLdsComplex;
    pass_inplace<N, R1, 1>(buf, ltw, sg);
    pass_inplace<N, R2, R1>(buf, ltw, sg);
    if constexpr (R3 > 1) pass_inplace<N, R3, R1 * R2>(buf, ltw, sg);
    return buf;
  }
};

// Ring width fixed at compile time (FastFFT), or 0 (GenericFFT).
template <class T, class = void>
struct fixed_width : std::integral_constant<int, 0> {};
template <class T>
struct fixed_width<T, std::void_t<decltype(T::N)>> : std::integral_constant<int, T::N> {};

// Runtime radices (4, 2, 3, 5), ping-pong buffers: any N = 2^a 3^b 5^c.
template <int R>
__device__ __forceinline__ void pingpong_bfly(const float2* __restrict__ src, float2* __restrict__ dst, int tt,
                                              int nb, int kk, int p, int tstride, const float2* __restrict__ tw,
                                              float sg) {
  float2 a[R];
#pragma unroll
  for (int q = 0; q < R; ++q) a[q] = src[tt + q * nb];
  if (kk != 0) {
#pragma unroll
    for (int q = 1; q < R; ++q) {
      float2 w = tw[q * kk * tstride];
      if (sg > 0.f) w.y = -w.y;
      a[q] = cmul(a[q], w);
    }
  }
  Codelet<R>::run(a, sg);
  const int ob = (tt - kk) * R + kk;
#pragma unroll
  for (int q = 0; q < R; ++q) dst[ob + q * p] = a[q];
}

struct GenericFFT {
  __device__ static __forceinline__ void prepare(float2*, const DftArgs&, const float2* __restrict__) {}
  __device__ static float2* run(float2* src, const DftArgs& a, const float2* __restrict__ tw, float sg) {
    const int N = a.nlon;
    float2* dst = src + FGW * N;
    int p = 1;
    for (int s = 0; s < a.nstages; ++s) {
      const int R = a.radix[s];
      const int nb = N / R;
      const int tstride = N / (p * R);
      const int total = FGW * nb;
      for (int t = threadIdx.x; t < total; t += NT) {
        const int f = t / nb;
        const int tt = t - f * nb;
        const int kk = tt % p;
        const float2* in = src + f * N;
        float2* out = dst + f * N;
        switch (R) {
          case 4: pingpong_bfly<4>(in, out, tt, nb, kk, p, tstride, tw, sg); break;
          case 2: pingpong_bfly<2>(in, out, tt, nb, kk, p, tstride, tw, sg); break;
          case 3: pingpong_bfly<3>(in, out, tt, nb, kk, p, tstride, tw, sg); break;
          default: pingpong_bfly<5>(in, out, tt, nb, kk, p, tstride, tw, sg); break;
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
};

// Item (field group g, ring pair kk, half hh) of a segment, numbered in the
// order (g, kk, hh); the four items that complete a 128-byte line of W are
// consecutive.
struct Item {
  int g, kk, hh;
  bool valid;
};
__device__ __forceinline__ Item item_of(const DftArgs& a, int local) {
  Item it;
  const int two_nk = 2 * a.nk;
  it.g = local / two_nk;
  const int rem = local - it.g * two_nk;
  it.kk = rem >> 1;
  it.hh = rem & 1;
  it.valid = 8 * it.g + 4 * it.hh < a.F;
  return it;
}

__device__ __forceinline__ size_t wrow(const DftArgs& a, int m, int p, int g, int kk) {
  return static_cast<size_t>(2 * m + p) * a.wslab + (static_cast<size_t>(g) * a.kpad + kk) * 16;
}

template <class FFT>
__device__ __forceinline__ void dft_forward_body(const DftArgs& a, const Item& it, const float* __restrict__ x,
                                                 float* __restrict__ W, const float2* __restrict__ tw,
                                                 const float* __restrict__ ring_scale, float2* lds,
                                                 float* __restrict__ zonal) {
  const int N = a.nlon;
  const int kk = it.kk;
  const int ks = a.nlat - 1 - kk;
  const bool eq = (ks == kk);
  const int f0 = 8 * it.g + 4 * it.hh;
  FFT::prepare(lds, a, tw);
  // load 4 fields x 2 rings, packed as complex (north, mirrored ring)
  const int nq = N / 4;
  constexpr int NF = fixed_width<FFT>::value;
  if constexpr (NF > 0 && NF % 4 == 0) {
    // every load of the thread is issued before the first LDS store, so the
    // workgroup waits for one memory round trip, not one per iteration
    constexpr int NQ = NF / 4, TOT = FGW * NQ, PER = (TOT + NT - 1) / NT;
    float4 vn[PER], vs[PER];
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int idx = threadIdx.x + b * NT;
      const int fl = idx / NQ;
      const int j = 4 * (idx - fl * NQ);
      const int fi = f0 + fl;
      vn[b] = make_float4(0.f, 0.f, 0.f, 0.f);
      vs[b] = vn[b];
      if (idx < TOT && fi < a.F) {
        vn[b] = *reinterpret_cast<const float4*>(x + (static_cast<size_t>(fi) * a.nlat + kk) * NF + j);
        if (!eq) vs[b] = *reinterpret_cast<const float4*>(x + (static_cast<size_t>(fi) * a.nlat + ks) * NF + j);
      }
    }
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int idx = threadIdx.x + b * NT;
      if (idx < TOT) {
        const int fl = idx / NQ;
        const int j = 4 * (idx - fl * NQ);
        float2* d = lds + fl * NF + j;
        d[0] = make_float2(vn[b].x, vs[b].x);
        d[1] = make_float2(vn[b].y, vs[b].y);
        d[2] = make_float2(vn[b].z, vs[b].z);
        d[3] = make_float2(vn[b].w, vs[b].w);
      }
    }
  } else if ((N & 3) == 0) {
    for (int idx = threadIdx.x; idx < FGW * nq; idx += NT) {
      const int fl = idx / nq;
      const int j = 4 * (idx - fl * nq);
      const int fi = f0 + fl;
      float4 vn = make_float4(0.f, 0.f, 0.f, 0.f), vs = vn;
      if (fi < a.F) {
        vn = *reinterpret_cast<const float4*>(x + (static_cast<size_t>(fi) * a.nlat + kk) * N + j);
        if (!eq) vs = *reinterpret_cast<const float4*>(x + (static_cast<size_t>(fi) * a.nlat + ks) * N + j);
      }
      float2* d = lds + fl * N + j;
      d[0] = make_float2(vn.x, vs.x);
      d[1] = make_float2(vn.y, vs.y);
      d[2] = make_float2(vn.z, vs.z);
      d[3] = make_float2(vn.w, vs.w);
    }
  } else {
    for (int idx = threadIdx.x; idx < FGW * N; idx += NT) {
      const int fl = idx / N;
      const int j = idx - fl * N;
      const int fi = f0 + fl;
      float re = 0.f, im = 0.f;
      if (fi < a.F) {
        re = x[(static_cast<size_t>(fi) * a.nlat + kk) * N + j];
        if (!eq) im = x[(static_cast<size_t>(fi) * a.nlat + ks) * N + j];
      }
      lds[idx] = make_float2(re, im);
    }
  }
  __syncthreads();
  const float2* Z = FFT::run(lds, a, tw, -1.f);
  const float sc = ring_scale[kk];
  if (zonal) {
    // zonal power spectra of the two rings: sc |X|^2 with the zonal scale
    for (int m = threadIdx.x; m < a.mmax; m += NT) {
#pragma unroll
      for (int fl = 0; fl < FGW; ++fl) {
        const int fi = f0 + fl;
        if (fi >= a.F) continue;
        const float2 zm = Z[fl * N + m];
        const float2 zr = Z[fl * N + (m == 0 ? 0 : N - m)];
        const float2 xn = make_float2(0.5f * (zm.x + zr.x), 0.5f * (zm.y - zr.y));
        const float2 xs = make_float2(0.5f * (zm.y + zr.y), -0.5f * (zm.x - zr.x));
        zonal[(static_cast<size_t>(fi) * a.nlat + kk) * a.mmax + m] = sc * (xn.x * xn.x + xn.y * xn.y);
        if (!eq) zonal[(static_cast<size_t>(fi) * a.nlat + ks) * a.mmax + m] = sc * (xs.x * xs.x + xs.y * xs.y);
      }
    }
    return;
  }
  for (int m = threadIdx.x; m < a.mmax; m += NT) {
    float Sv[8], Av[8];
#pragma unroll
    for (int fl = 0; fl < FGW; ++fl) {
      const float2 zm = Z[fl * N + m];
      const float2 zr = Z[fl * N + (m == 0 ? 0 : N - m)];
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
      Sv[2 * fl] = S.x;
      Sv[2 * fl + 1] = S.y;
      Av[2 * fl] = A.x;
      Av[2 * fl + 1] = A.y;
    }
    float4* ps = reinterpret_cast<float4*>(W + wrow(a, m, 0, it.g, kk) + 8 * it.hh);
    float4* pa = reinterpret_cast<float4*>(W + wrow(a, m, 1, it.g, kk) + 8 * it.hh);
    ps[0] = make_float4(Sv[0], Sv[1], Sv[2], Sv[3]);
    ps[1] = make_float4(Sv[4], Sv[5], Sv[6], Sv[7]);
    pa[0] = make_float4(Av[0], Av[1], Av[2], Av[3]);
    pa[1] = make_float4(Av[4], Av[5], Av[6], Av[7]);
  }
}

template <class FFT>
__device__ __forceinline__ void dft_inverse_body(const DftArgs& a, const Item& it, const float* __restrict__ W,
                                                 float* __restrict__ x, const float2* __restrict__ tw,
                                                 const float* __restrict__ ring_scale, float2* lds) {
  const int N = a.nlon;
  const int kk = it.kk;
  const int ks = a.nlat - 1 - kk;
  const bool eq = (ks == kk);
  const int f0 = 8 * it.g + 4 * it.hh;
  FFT::prepare(lds, a, tw);
  const float h = 0.5f * a.c_rest;
  // E = W[m][0], O = W[m][1] of this item's 4 fields -> spectra of the two
  // rings, placed at bins m and N - m of the packed sequence
  auto place = [&](int m, float4 e0, float4 e1, float4 o0, float4 o1) {
    const float Ev[8] = {e0.x, e0.y, e0.z, e0.w, e1.x, e1.y, e1.z, e1.w};
    const float Ov[8] = {o0.x, o0.y, o0.z, o0.w, o1.x, o1.y, o1.z, o1.w};
#pragma unroll
    for (int fl = 0; fl < FGW; ++fl) {
      const float2 E = make_float2(Ev[2 * fl], Ev[2 * fl + 1]);
      const float2 O = make_float2(Ov[2 * fl], Ov[2 * fl + 1]);
      const float2 yn = cadd(E, O);
      const float2 ys = eq ? make_float2(0.f, 0.f) : csub(E, O);
      if (m == 0) {
        lds[fl * N] = make_float2(yn.x, ys.x);
      } else {
        const float2 hn = cscale(yn, h), hs = cscale(ys, h);
        lds[fl * N + m] = make_float2(hn.x - hs.y, hn.y + hs.x);
        lds[fl * N + N - m] = make_float2(hn.x + hs.y, -hn.y + hs.x);
      }
    }
  };
  // order m has odd-parity degrees only when m + 1 < lmax
  auto load = [&](int m, float4& e0, float4& e1, float4& o0, float4& o1) {
    const float4* pe = reinterpret_cast<const float4*>(W + wrow(a, m, 0, it.g, kk) + 8 * it.hh);
    e0 = pe[0];
    e1 = pe[1];
    o0 = make_float4(0.f, 0.f, 0.f, 0.f);
    o1 = o0;
    if (m + 1 < a.lmax) {
      const float4* po = reinterpret_cast<const float4*>(W + wrow(a, m, 1, it.g, kk) + 8 * it.hh);
      o0 = po[0];
      o1 = po[1];
    }
  };
  constexpr int NF = fixed_width<FFT>::value;
  if constexpr (NF > 0) {
    // all loads of the thread first (m < mmax <= NF / 2), then the zero
    // fill of the buffer, then the stores of the loaded bins
    constexpr int PER = (NF / 2 + NT - 1) / NT;
    float4 e0[PER], e1[PER], o0[PER], o1[PER];
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int m = threadIdx.x + b * NT;
      if (m < a.mmax) load(m, e0[b], e1[b], o0[b], o1[b]);
    }
    for (int idx = threadIdx.x; idx < FGW * N; idx += NT) lds[idx] = make_float2(0.f, 0.f);
    lds_barrier();
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int m = threadIdx.x + b * NT;
      if (m < a.mmax) place(m, e0[b], e1[b], o0[b], o1[b]);
    }
  } else {
    for (int idx = threadIdx.x; idx < FGW * N; idx += NT) lds[idx] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int m = threadIdx.x; m < a.mmax; m += NT) {
      float4 e0, e1, o0, o1;
      load(m, e0, e1, o0, o1);
      place(m, e0, e1, o0, o1);
    }
  }
  __syncthreads();
  const float2* Z = FFT::run(lds, a, tw, 1.f);
  const float sc = ring_scale[kk];
  const int nq = N / 4;
  if ((N & 3) == 0) {
    for (int idx = threadIdx.x; idx < FGW * nq; idx += NT) {
      const int fl = idx / nq;
      const int j = 4 * (idx - fl * nq);
      const int fi = f0 + fl;
      if (fi >= a.F) continue;
      const float2* z = Z + fl * N + j;
      const float2 z0 = z[0], z1 = z[1], z2 = z[2], z3 = z[3];
      *reinterpret_cast<float4*>(x + (static_cast<size_t>(fi) * a.nlat + kk) * N + j) =
          make_float4(z0.x * sc, z1.x * sc, z2.x * sc, z3.x * sc);
      if (!eq)
        *reinterpret_cast<float4*>(x + (static_cast<size_t>(fi) * a.nlat + ks) * N + j) =
            make_float4(z0.y * sc, z1.y * sc, z2.y * sc, z3.y * sc);
    }
  } else {
    for (int idx = threadIdx.x; idx < FGW * N; idx += NT) {
      const int fl = idx / N;
      const int j = idx - fl * N;
      const int fi = f0 + fl;
      if (fi >= a.F) continue;
      const float2 z = Z[idx];
      x[(static_cast<size_t>(fi) * a.nlat + kk) * N + j] = z.x * sc;
      if (!eq) x[(static_cast<size_t>(fi) * a.nlat + ks) * N + j] = z.y * sc;
    }
  }
}

__device__ __forceinline__ DftArgs seg_args(const SegDev& sd, float c_rest) {
  DftArgs a;
  a.nlat = sd.g.nlat;
  a.nlon = sd.g.nlon;
  a.lmax = sd.g.lmax;
  a.mmax = sd.g.mmax;
  a.nk = sd.g.nk;
  a.F = sd.g.F;
  a.kpad = sd.g.kpad;
  a.G = sd.g.groups;
  a.wslab = sd.g.wslab;
  a.nitems = sd.dft_items;
  a.nstages = sd.nstages;
  a.radix = sd.radix;
  a.c_rest = c_rest;
  return a;
}

using F1440 = FastFFT<1440, 9, 10, 16>;
using F720 = FastFFT<720, 9, 5, 16>;
using F360 = FastFFT<360, 9, 5, 8>;
using F64 = FastFFT<64, 4, 16, 1>;

// Batched kernels: the items of all segments are numbered consecutively
// (segment s owns [dft_begin, dft_begin + dft_items)); each XCD (workgroup b
// runs on XCD b % 8) receives one contiguous slice of that numbering.
__device__ __forceinline__ int batched_slot(int total) {
  const int per = (total + 7) / 8;
  return (blockIdx.x % 8) * per + blockIdx.x / 8;
}
__device__ __forceinline__ int segment_of(const SegDev* __restrict__ segs, int nseg, int slot) {
  int s = 0;
  while (s + 1 < nseg && slot >= segs[s + 1].dft_begin) ++s;
  return s;
}

// mode 0: unit ring scale, 1: (2 pi / nlon) w_k, 2: zonal PSD into `zonal`
__global__ __launch_bounds__(NT) void dft_forward_batched(const SegDev* __restrict__ segs, int nseg, int total,
                                                          const float* __restrict__ x, int mode,
                                                          float* __restrict__ zonal) {
  extern __shared__ float2 lds[];
  const int slot = batched_slot(total);
  if (slot >= total) return;
  const SegDev& sd = segs[segment_of(segs, nseg, slot)];
  const DftArgs a = seg_args(sd, 1.f);
  const Item it = item_of(a, slot - sd.dft_begin);
  if (!it.valid) return;
  const float* xs = x + sd.grid_off;
  const float* scale = mode == 1 ? sd.scale_sht : mode == 2 ? sd.scale_zonal : sd.scale_one;
  float* zs = mode == 2 ? zonal : nullptr;
  switch (sd.g.nlon) {
    case 1440: dft_forward_body<F1440>(a, it, xs, sd.work, sd.tw, scale, lds, zs); break;
    case 720: dft_forward_body<F720>(a, it, xs, sd.work, sd.tw, scale, lds, zs); break;
    case 360: dft_forward_body<F360>(a, it, xs, sd.work, sd.tw, scale, lds, zs); break;
    case 64: dft_forward_body<F64>(a, it, xs, sd.work, sd.tw, scale, lds, zs); break;
    default: dft_forward_body<GenericFFT>(a, it, xs, sd.work, sd.tw, scale, lds, zs); break;
  }
}

__global__ __launch_bounds__(NT) void dft_inverse_batched(const SegDev* __restrict__ segs, int nseg, int total,
                                                          float* __restrict__ x, int sht_scale, float c_rest) {
  extern __shared__ float2 lds[];
  const int slot = batched_slot(total);
  if (slot >= total) return;
  const SegDev& sd = segs[segment_of(segs, nseg, slot)];
  const DftArgs a = seg_args(sd, c_rest);
  const Item it = item_of(a, slot - sd.dft_begin);
  if (!it.valid) return;
  float* xs = x + sd.grid_off;
  const float* scale = sht_scale ? sd.scale_sht : sd.scale_one;
  switch (sd.g.nlon) {
    case 1440: dft_inverse_body<F1440>(a, it, sd.work, xs, sd.tw, scale, lds); break;
    case 720: dft_inverse_body<F720>(a, it, sd.work, xs, sd.tw, scale, lds); break;
    case 360: dft_inverse_body<F360>(a, it, sd.work, xs, sd.tw, scale, lds); break;
    case 64: dft_inverse_body<F64>(a, it, sd.work, xs, sd.tw, scale, lds); break;
    default: dft_inverse_body<GenericFFT>(a, it, sd.work, xs, sd.tw, scale, lds); break;
  }
}

hipError_t prepare_lds(const void* k, size_t lds_bytes) {
  if (lds_bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes));
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

size_t dft_lds_bytes(int nlon) {
  switch (nlon) {
    case 1440: return F1440::kLdsBytes;
    case 720: return F720::kLdsBytes;
    case 360: return F360::kLdsBytes;
    case 64: return F64::kLdsBytes;
    default: return 2 * static_cast<size_t>(FGW) * nlon * sizeof(float2);
  }
}

hipError_t prepare_dft_kernels(size_t lds_bytes) {
  hipError_t e = prepare_lds(reinterpret_cast<const void*>(dft_forward_batched), lds_bytes);
  if (e == hipSuccess) e = prepare_lds(reinterpret_cast<const void*>(dft_inverse_batched), lds_bytes);
  return e;
}

hipError_t launch_dft_forward_batched(const BatchArgs& b, const float* x, bool sht_scale, hipStream_t st) {
  const unsigned blocks = static_cast<unsigned>((b.dft_total + 7) / 8 * 8);
  hipLaunchKernelGGL(dft_forward_batched, dim3(blocks), dim3(NT), b.dft_lds, st, b.segs, b.nseg, b.dft_total, x,
                     sht_scale ? 1 : 0, static_cast<float*>(nullptr));
  return hipGetLastError();
}

hipError_t launch_zonal_psd(const BatchArgs& b, const float* x, float* out, hipStream_t st) {
  const unsigned blocks = static_cast<unsigned>((b.dft_total + 7) / 8 * 8);
  hipLaunchKernelGGL(dft_forward_batched, dim3(blocks), dim3(NT), b.dft_lds, st, b.segs, b.nseg, b.dft_total, x, 2,
                     out);
  return hipGetLastError();
}

hipError_t launch_dft_inverse_batched(const BatchArgs& b, float* x, bool sht_scale, float c_rest, hipStream_t st) {
  const unsigned blocks = static_cast<unsigned>((b.dft_total + 7) / 8 * 8);
  hipLaunchKernelGGL(dft_inverse_batched, dim3(blocks), dim3(NT), b.dft_lds, st, b.segs, b.nseg, b.dft_total, x,
                     sht_scale ? 1 : 0, c_rest);
  return hipGetLastError();
}

}  // namespace sht
