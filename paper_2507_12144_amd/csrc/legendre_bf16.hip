// bf16 forms of the Legendre contraction (the per-order-m contraction of
// Alg. 1 and its synthesis counterpart of eq. isht) on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16, float32 accumulation).
//
// Precision forms.  The table is read as NP bf16 planes (rounded to nearest
// even from the float64 recurrence: hi = bf16(v), then the residuals); the
// data (folded DFT output, or spectrum) are split the same way in float32
// when they are loaded.  With a = sum_i a_i, b = sum_j b_j the kernels form
//   NP = 1: a_0 b_0                                   (plain bf16)
//   NP = 2: a_0 b_0 + a_0 b_1 + a_1 b_0               (split bf16)
//   NP = 3: all a_i b_j with i + j < 3 (six products) (three-term split)
// i.e. every product whose magnitude is above the representation error of
// the split.  The correction products of the analysis go into their own
// accumulator, added to the leading one at the end of each output block.
//
// Structure as in the float32 kernels: one workgroup per (m, column chunk),
// wave (p, j) owns parity p and one 16-column field group; the table is
// streamed from L2 in MFMA fragment order (16 bytes a lane per plane and
// step), no LDS, no barriers.  A step is K = 32 contraction values.
#include "bf16.h"
#include "internal.h"
#include "kernel_common.h"

namespace sht {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// Split 8 float32 values into NP bf16 planes (residuals in float32).
template <int NP>
__device__ __forceinline__ void split8(const float* v, bf16x8* out) {
  u16x8 bits[NP];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float r = v[e];
#pragma unroll
    for (int pl = 0; pl < NP; ++pl) {
      const uint16_t b = bf16_rn_from_float(r);
      bits[pl][e] = b;
      r -= bf16_bits_to_float(b);
    }
  }
#pragma unroll
  for (int pl = 0; pl < NP; ++pl) out[pl] = __builtin_bit_cast(bf16x8, bits[pl]);
}

// Products of order below NP between split operands a and b.
template <int NP>
__device__ __forceinline__ void products(const bf16x8* a, const bf16x8* b, floatx4& main, floatx4& corr) {
  main = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], main, 0, 0, 0);
  if constexpr (NP >= 2) {
    corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], corr, 0, 0, 0);
    corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], corr, 0, 0, 0);
  }
  if constexpr (NP >= 3) {
    corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], corr, 0, 0, 0);
    corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], corr, 0, 0, 0);
    corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], corr, 0, 0, 0);
  }
}

// Analysis.  Contraction index k of a wave's K slice = lk * KPAD/4 + 8t + e
// for lane group lk, step t and element e of the 8-value operand.
template <int NCB, int KS, int NP>
__global__ __launch_bounds__(128 * NCB) void analysis_bf16_kernel(LegArgs a, const int2* __restrict__ work,
                                                                  int per, const float* __restrict__ W,
                                                                  float2* __restrict__ y, float c_rest) {
  constexpr int NTH = 128 * NCB;
  constexpr int KPAD = 4 * KS;
  constexpr int Q = KPAD / 4;
  constexpr int T8 = KPAD / 32;  // steps per 16-row block
  constexpr int D = ring_depth(T8, NP >= 3 ? 3 : 4);
  const int2 wk = take_work(work, per);
  const int m = wk.x, c = wk.y;
  if (m < 0) return;
  const SegGeom& g = a.g;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = wave / NCB, j = wave - p * NCB;
  const int cb = c * NCB + j;
  const int li = lane & 15, lk = lane >> 4;
  if (cb < g.groups) {
    bf16x8 xs[T8][NP];
    {
      const float* Wp = W + (static_cast<size_t>(2 * m + p) * g.groups + cb) * KPAD * 16 + li;
#pragma unroll
      for (int t = 0; t < T8; ++t) {
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = Wp[(lk * Q + 8 * t + e) * 16];
        split8<NP>(v, xs[t]);
      }
    }
    const int n0 = (g.lmax - m + 1) >> 1;
    const int nb32 = (n0 + 31) >> 5;
    const int np = p ? (g.lmax - m) >> 1 : n0;
    const int nbp = (np + 15) >> 4;
    const int last = nbp > 0 ? nbp * T8 - 1 : 0;  // clamp: prefetches never leave the table
    const bf16x8* A = reinterpret_cast<const bf16x8*>(static_cast<const uint16_t*>(a.tab_ana) + a.tab_off[m]) +
                      static_cast<size_t>(p * 2 * nb32) * T8 * NP * 64 + lane;
    const float ms = (m == 0) ? 1.f : c_rest;
    float* yf = reinterpret_cast<float*>(y);
    const int f = 8 * cb + (li >> 1);
    const bool fok = f < g.F;
    bf16x8 ring[D][NP];
#pragma unroll
    for (int u = 0; u < D; ++u)
#pragma unroll
      for (int pl = 0; pl < NP; ++pl) ring[u][pl] = A[(static_cast<size_t>(min(u, last)) * NP + pl) * 64];
    for (int ib = 0; ib < nbp; ++ib) {
      floatx4 main = {0.f, 0.f, 0.f, 0.f}, corr = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < T8; ++t) {
        bf16x8 av[NP];
#pragma unroll
        for (int pl = 0; pl < NP; ++pl) av[pl] = ring[t % D][pl];
        const int q = min(ib * T8 + t + D, last);
#pragma unroll
        for (int pl = 0; pl < NP; ++pl) ring[t % D][pl] = A[(static_cast<size_t>(q) * NP + pl) * 64];
        products<NP>(av, xs[t], main, corr);
      }
      if (fok) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * ib + 4 * lk + r;
          if (i < np) {
            const int l = m + p + 2 * i;
            yf[((static_cast<size_t>(f) * g.lmax + l) * g.mmax + m) * 2 + (li & 1)] = (main[r] + corr[r]) * ms;
          }
        }
      }
    }
  }
  // zeros of the spectrum: degree l = m, orders m+1 .. mmax-1 of this
  // chunk's fields (contiguous runs; together the workgroups of all m cover
  // every entry l < m')
  if (m < g.lmax) {
    const int fbeg = 8 * NCB * c;
    const int fend = min(g.F, fbeg + 8 * NCB);
    const int run = g.mmax - 1 - m;
    for (int ff = fbeg; ff < fend; ++ff) {
      float2* row = y + (static_cast<size_t>(ff) * g.lmax + m) * g.mmax + m + 1;
      for (int e = threadIdx.x; e < run; e += NTH) row[e] = make_float2(0.f, 0.f);
    }
  }
}

// Synthesis.  Contraction rows i = 32 ib + 8 lk + e of the wave's parity;
// output ring k = (MFMA row) * KR + rb.
template <int NCB, int KS, int NP>
__global__ __launch_bounds__(128 * NCB) void synthesis_bf16_kernel(LegArgs a, const int2* __restrict__ work,
                                                                   int per, const float2* __restrict__ y,
                                                                   float* __restrict__ W) {
  constexpr int KPAD = 4 * KS;
  constexpr int KR = KPAD / 16;  // 16-ring output blocks = steps per 32-row block
  constexpr int D = ring_depth(KR, NP >= 3 ? 3 : 4);
  const int2 wk = take_work(work, per);
  const int m = wk.x, c = wk.y;
  if (m < 0) return;
  const SegGeom& g = a.g;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = wave / NCB, j = wave - p * NCB;
  const int cb = c * NCB + j;
  if (cb >= g.groups) return;
  const int li = lane & 15, lk = lane >> 4;
  const int n0 = (g.lmax - m + 1) >> 1;
  const int nb32 = (n0 + 31) >> 5;
  const int np = p ? (g.lmax - m) >> 1 : n0;
  const int nbp = (np + 31) >> 5;
  const int last = nbp > 0 ? nbp * KR - 1 : 0;  // clamp: prefetches never leave the table
  const bf16x8* A = reinterpret_cast<const bf16x8*>(static_cast<const uint16_t*>(a.tab_syn) + a.tab_off[m]) +
                    static_cast<size_t>(p * nb32) * KR * NP * 64 + lane;
  // B operand of lane (li, lk) for block ib: re (li even) or im (li odd) of
  // field 8 cb + li/2 at degrees l = m + p + 2 (32 ib + 8 lk + e), e < 8
  const float* yf = reinterpret_cast<const float*>(y);
  const int f = 8 * cb + (li >> 1);
  const bool fok = f < g.F;
  const size_t fbase = (static_cast<size_t>(fok ? f : 0) * g.lmax) * g.mmax;
  float bn[8];
  auto bload = [&](int ib) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int i = 32 * ib + 8 * lk + e;
      const bool ok = fok && i < np;
      const int l = ok ? m + p + 2 * i : m;
      const float v = yf[(fbase + static_cast<size_t>(l) * g.mmax + m) * 2 + (li & 1)];
      bn[e] = ok ? v : 0.f;
    }
  };
  floatx4 acc[KR];
#pragma unroll
  for (int rb = 0; rb < KR; ++rb) acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
  bf16x8 ring[D][NP];
#pragma unroll
  for (int u = 0; u < D; ++u)
#pragma unroll
    for (int pl = 0; pl < NP; ++pl) ring[u][pl] = A[(static_cast<size_t>(min(u, last)) * NP + pl) * 64];
  bload(0);
  for (int ib = 0; ib < nbp; ++ib) {
    bf16x8 bv[NP];
    split8<NP>(bn, bv);
    if (ib + 1 < nbp) bload(ib + 1);
#pragma unroll
    for (int rb = 0; rb < KR; ++rb) {
      bf16x8 av[NP];
#pragma unroll
      for (int pl = 0; pl < NP; ++pl) av[pl] = ring[rb % D][pl];
      const int q = min(ib * KR + rb + D, last);
#pragma unroll
      for (int pl = 0; pl < NP; ++pl) ring[rb % D][pl] = A[(static_cast<size_t>(q) * NP + pl) * 64];
      products<NP>(av, bv, acc[rb], acc[rb]);
    }
  }
  float* Wp = W + (static_cast<size_t>(2 * m + p) * g.groups + cb) * KPAD * 16;
#pragma unroll
  for (int rb = 0; rb < KR; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) Wp[((4 * lk + r) * KR + rb) * 16 + li] = acc[rb][r];
}

template <int NCB, int KS, int NP>
hipError_t launch3(bool analysis, const LegArgs& a, const void* in, void* out, float c_rest, hipStream_t st) {
  if (analysis) {
    hipLaunchKernelGGL((analysis_bf16_kernel<NCB, KS, NP>), dim3(8 * a.work_per), dim3(128 * NCB), 0, st, a,
                       a.work, a.work_per, static_cast<const float*>(in), static_cast<float2*>(out), c_rest);
  } else {
    hipLaunchKernelGGL((synthesis_bf16_kernel<NCB, KS, NP>), dim3(8 * a.work_per), dim3(128 * NCB), 0, st, a,
                       a.work, a.work_per, static_cast<const float2*>(in), static_cast<float*>(out));
  }
  return hipGetLastError();
}

template <int NCB, int KS>
hipError_t by_np(bool analysis, int planes, const LegArgs& a, const void* in, void* out, float c_rest,
                 hipStream_t st) {
  switch (planes) {
    case 1: return launch3<NCB, KS, 1>(analysis, a, in, out, c_rest, st);
    case 2: return launch3<NCB, KS, 2>(analysis, a, in, out, c_rest, st);
    case 3: return launch3<NCB, KS, 3>(analysis, a, in, out, c_rest, st);
    default: return hipErrorInvalidValue;
  }
}

template <int NCB>
hipError_t by_ks(bool analysis, int planes, const LegArgs& a, const void* in, void* out, float c_rest,
                 hipStream_t st) {
  switch (a.g.kpad / 4) {
    case 16: return by_np<NCB, 16>(analysis, planes, a, in, out, c_rest, st);
    case 32: return by_np<NCB, 32>(analysis, planes, a, in, out, c_rest, st);
    case 48: return by_np<NCB, 48>(analysis, planes, a, in, out, c_rest, st);
    case 64: return by_np<NCB, 64>(analysis, planes, a, in, out, c_rest, st);
    case 96: return by_np<NCB, 96>(analysis, planes, a, in, out, c_rest, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t dispatch(bool analysis, int planes, const LegArgs& a, const void* in, void* out, float c_rest,
                    hipStream_t st) {
  switch (a.ncb) {
    case 1: return by_ks<1>(analysis, planes, a, in, out, c_rest, st);
    case 2: return by_ks<2>(analysis, planes, a, in, out, c_rest, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_legendre_analysis_bf16(const LegArgs& a, int planes, const float* W, float2* y, float c_rest,
                                         hipStream_t stream) {
  return dispatch(true, planes, a, W, y, c_rest, stream);
}

hipError_t launch_legendre_synthesis_bf16(const LegArgs& a, int planes, const float2* y, float* W,
                                          hipStream_t stream) {
  return dispatch(false, planes, a, y, W, 1.f, stream);
}

}  // namespace sht
