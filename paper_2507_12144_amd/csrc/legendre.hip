// Legendre contraction kernels: the per-order-m dense contraction of Alg. 1
// (xc_{bclm} = sum_k L_{mlk} x_{bckm}) and its synthesis counterpart
// (eq. isht), on CDNA4 matrix cores (v_mfma_f32_16x16x4_f32).
//
// Folded form.  With nodes symmetric about the equator,
// P^_l^m(-x) = (-1)^(l+m) P^_l^m(x), so for each m the degrees split by
// parity p = (l - m) & 1 and only the northern rings k < nk are needed:
//   analysis : u^[l] = sum_{k<nk} P^_l^m(x_k) (p == 0 ? S_k : A_k)
//   synthesis: E_k = sum_{p=0 rows} P^ u^,  O_k = sum_{p=1 rows} P^ u^,
//              north ring = E + O, mirrored ring = E - O
// which halves the multiply-adds.  S, A, E, O live in the workspace
// W[m][p][g][k][16] (g = group of 8 fields, 16 = their re/im).
//
// Streaming design.  The Legendre table is stored in MFMA fragment order
// (see the table kernel), so every wave streams its own A operands straight
// from L2 as contiguous 1 KiB loads, several in flight in a register ring,
// with no LDS staging and no barriers: waves never wait for each other.
// One workgroup per (m, column chunk of NCB field groups), 2*NCB waves;
// wave (p, j) owns parity p and field group c*NCB + j (one 16-column MFMA
// block).  The NCB waves of one parity read the same table lines (L1 hits),
// the chunks of one m run together on one XCD (L2 hits).
//  * analysis: the wave keeps its whole K = kpad slice of S or A in VGPRs
//    (read once from HBM); each 16-row block of its parity is one 16 x 16
//    output block, written to the spectrum.
//  * synthesis: the wave keeps its whole kpad x 16 output block in VGPRs;
//    the spectrum values (B operands) are read one row block ahead.
// Workgroups are dealt to XCDs in chunks of 16 consecutive m so that each
// XCD gets a balanced share of the triangle and the 8-byte accesses of
// neighbouring m to the spectral tensor (m fastest) meet in its L2.
#include "internal.h"
#include "kernel_common.h"

namespace sht {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
// native 4-float vector (HIP's float4 is a struct; its copies do not stay in
// VGPRs)
typedef float v4f __attribute__((ext_vector_type(4)));

// Analysis.  Contraction index k of a wave's K slice = lk * KS + 4t + q for
// lane group lk, step t and component q of the 16-byte operand.
template <int NCB, int KS>
__global__ __launch_bounds__(128 * NCB) void analysis_kernel(LegArgs a, const int2* __restrict__ work, int per,
                                                             const float* __restrict__ W, float2* __restrict__ y,
                                                             float c_rest) {
  constexpr int NTH = 128 * NCB;
  constexpr int KPAD = 4 * KS;
  constexpr int T4 = KS / 4;  // 16-byte operand loads per row block
  constexpr int D = ring_depth(T4);
  const int2 wk = take_work(work, per);
  const int m = wk.x, c = wk.y;
  if (m < 0) return;
  const SegGeom& g = a.g;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = wave / NCB, j = wave - p * NCB;
  const int cb = c * NCB + j;
  const int li = lane & 15, lk = lane >> 4;
  if (cb < g.groups) {
    float xr[KS];
    {
      const float* Wp = W + (static_cast<size_t>(2 * m + p) * g.groups + cb) * KPAD * 16 + lk * KS * 16 + li;
#pragma unroll
      for (int s = 0; s < KS; ++s) xr[s] = Wp[16 * s];
    }
    const int n0 = (g.lmax - m + 1) >> 1;
    const int nb = (n0 + 15) >> 4;
    const int np = p ? (g.lmax - m) >> 1 : n0;
    const int nbp = (np + 15) >> 4;
    const int last = nbp > 0 ? nbp * T4 - 1 : 0;  // clamp: prefetches never leave the table
    const v4f* A = reinterpret_cast<const v4f*>(static_cast<const float*>(a.tab_ana) + a.tab_off[m]) + static_cast<size_t>(p * nb) * T4 * 64 + lane;
    const float ms = (m == 0) ? 1.f : c_rest;
    float* yf = reinterpret_cast<float*>(y);
    const int f = 8 * cb + (li >> 1);
    const bool fok = f < g.F;
    v4f ring[D];
#pragma unroll
    for (int u = 0; u < D; ++u) ring[u] = A[static_cast<size_t>(min(u, last)) * 64];
    for (int ib = 0; ib < nbp; ++ib) {
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < T4; ++t) {
        const v4f av = ring[t % D];
        const int q = ib * T4 + t + D;
        ring[t % D] = A[static_cast<size_t>(min(q, last)) * 64];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, xr[4 * t + 0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, xr[4 * t + 1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, xr[4 * t + 2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, xr[4 * t + 3], acc, 0, 0, 0);
      }
      if (fok) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * ib + 4 * lk + r;
          if (i < np) {
            const int l = m + p + 2 * i;
            yf[((static_cast<size_t>(f) * g.lmax + l) * g.mmax + m) * 2 + (li & 1)] = acc[r] * ms;
          }
        }
      }
    }
  }
  // the entries l < m of this chunk's fields are zero
  const int fbeg = 8 * NCB * c;
  const int fend = min(g.F, fbeg + 8 * NCB);
  const int nf = fend - fbeg;
  for (int e = threadIdx.x; e < m * nf; e += NTH) {
    const int l = e / nf;
    const int ff = fbeg + (e - l * nf);
    y[(static_cast<size_t>(ff) * g.lmax + l) * g.mmax + m] = make_float2(0.f, 0.f);
  }
}

// Synthesis.  Output ring k of a wave's block = li * KR + 4t + q for MFMA row
// li, step t and component q; contraction row i = 16 ib + 4 s + lk.
template <int NCB, int KS>
__global__ __launch_bounds__(128 * NCB) void synthesis_kernel(LegArgs a, const int2* __restrict__ work, int per,
                                                              const float2* __restrict__ y, float* __restrict__ W) {
  constexpr int KPAD = 4 * KS;
  constexpr int KR = KPAD / 16;  // 16-ring output blocks
  constexpr int T4 = KR / 4;     // 16-byte operand loads per substep
  constexpr int STEPS = 4 * T4;  // operand loads per row block
  constexpr int D = ring_depth(STEPS);
  static_assert(KR % 4 == 0, "KR");
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
  const int nb = (n0 + 15) >> 4;
  const int np = p ? (g.lmax - m) >> 1 : n0;
  const int nbp = (np + 15) >> 4;
  const int last = nbp > 0 ? nbp * STEPS - 1 : 0;  // clamp: prefetches never leave the table
  const v4f* A = reinterpret_cast<const v4f*>(static_cast<const float*>(a.tab_syn) + a.tab_off[m]) + static_cast<size_t>(p * nb) * STEPS * 64 + lane;
  // B operand of lane (li, lk) at substep s of row block ib: re (li even) or
  // im (li odd) of field 8 cb + li/2 at degree l = m + p + 2 (16 ib + 4 s + lk)
  const float* yf = reinterpret_cast<const float*>(y);
  const int f = 8 * cb + (li >> 1);
  const bool fok = f < g.F;
  const size_t fbase = (static_cast<size_t>(fok ? f : 0) * g.lmax) * g.mmax;
  auto bload = [&](int ib, int s) {
    const int i = 16 * ib + 4 * s + lk;
    const bool ok = fok && i < np;
    const int l = ok ? m + p + 2 * i : m;
    const float v = yf[(fbase + static_cast<size_t>(l) * g.mmax + m) * 2 + (li & 1)];
    return ok ? v : 0.f;
  };
  floatx4 acc[KR];
#pragma unroll
  for (int rb = 0; rb < KR; ++rb) acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
  v4f ring[D];
#pragma unroll
  for (int u = 0; u < D; ++u) ring[u] = A[static_cast<size_t>(min(u, last)) * 64];
  float bn[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) bn[s] = bload(0, s);
  for (int ib = 0; ib < nbp; ++ib) {
    float bc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) bc[s] = bn[s];
    if (ib + 1 < nbp) {
#pragma unroll
      for (int s = 0; s < 4; ++s) bn[s] = bload(ib + 1, s);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int t = 0; t < T4; ++t) {
        const int st = s * T4 + t;
        const v4f av = ring[st % D];
        const int q = ib * STEPS + st + D;
        ring[st % D] = A[static_cast<size_t>(min(q, last)) * 64];
        acc[4 * t + 0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bc[s], acc[4 * t + 0], 0, 0, 0);
        acc[4 * t + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bc[s], acc[4 * t + 1], 0, 0, 0);
        acc[4 * t + 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bc[s], acc[4 * t + 2], 0, 0, 0);
        acc[4 * t + 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bc[s], acc[4 * t + 3], 0, 0, 0);
      }
    }
  }
  float* Wp = W + (static_cast<size_t>(2 * m + p) * g.groups + cb) * KPAD * 16;
  // acc[4t + q][r] is output row 4 lk + r, ring k = (4 lk + r) * KR + 4 t + q
#pragma unroll
  for (int t = 0; t < T4; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) Wp[((4 * lk + r) * KR + 4 * t + q) * 16 + li] = acc[4 * t + q][r];
}

template <int NCB, int KS>
hipError_t launch_pair(bool analysis, const LegArgs& a, const void* in, void* out, float c_rest, hipStream_t st) {
  if (analysis) {
    const unsigned blocks = static_cast<unsigned>(8 * a.work_per);
    hipLaunchKernelGGL((analysis_kernel<NCB, KS>), dim3(blocks), dim3(128 * NCB), 0, st, a, a.work, a.work_per,
                       static_cast<const float*>(in), static_cast<float2*>(out), c_rest);
  } else {
    const unsigned blocks = static_cast<unsigned>(8 * a.work_syn_per);
    hipLaunchKernelGGL((synthesis_kernel<NCB, KS>), dim3(blocks), dim3(128 * NCB), 0, st, a, a.work_syn,
                       a.work_syn_per, static_cast<const float2*>(in), static_cast<float*>(out));
  }
  return hipGetLastError();
}

template <int NCB>
hipError_t by_ks(bool analysis, const LegArgs& a, const void* in, void* out, float c_rest, hipStream_t st) {
  switch (a.g.kpad / 4) {
    case 16: return launch_pair<NCB, 16>(analysis, a, in, out, c_rest, st);
    case 32: return launch_pair<NCB, 32>(analysis, a, in, out, c_rest, st);
    case 48: return launch_pair<NCB, 48>(analysis, a, in, out, c_rest, st);
    case 64: return launch_pair<NCB, 64>(analysis, a, in, out, c_rest, st);
    case 96: return launch_pair<NCB, 96>(analysis, a, in, out, c_rest, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t dispatch(bool analysis, const LegArgs& a, Storage st, const void* in, void* out, float c_rest,
                    hipStream_t stream) {
  if (st != Storage::F32) return hipErrorNotSupported;
  switch (a.ncb) {
    case 1: return by_ks<1>(analysis, a, in, out, c_rest, stream);
    case 3: return by_ks<3>(analysis, a, in, out, c_rest, stream);
    case 4: return by_ks<4>(analysis, a, in, out, c_rest, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int legendre_ring_pad(int nk) {
  const int ks[] = {16, 32, 48, 64, 96};
  for (int k : ks)
    if (4 * k >= nk) return 4 * k;
  return -1;
}

int legendre_ncb(int groups) {
  if (groups >= 4 && groups % 4 == 0) return 4;
  if (groups >= 3 && groups % 3 == 0) return 3;
  if (groups >= 8) return 4;
  return 1;
}

hipError_t launch_legendre_analysis(const LegArgs& a, Storage st, const float* W, float2* y, float c_rest,
                                    hipStream_t stream) {
  return dispatch(true, a, st, W, y, c_rest, stream);
}

hipError_t launch_legendre_synthesis(const LegArgs& a, Storage st, const float2* y, float* W,
                                     hipStream_t stream) {
  return dispatch(false, a, st, y, W, 1.f, stream);
}

}  // namespace sht
