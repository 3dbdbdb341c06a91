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
// which halves both the table and the multiply-adds.  S, A, E, O live in the
// workspace W[m][p][g][k][16] (g = group of 8 fields, 16 = their re/im).
//
// Work decomposition.  One workgroup per (m, column chunk of NCB groups),
// 2*NCB waves; wave (p, j) owns parity p and field group c*NCB + j, i.e. one
// 16-column MFMA block.
//  * analysis: the wave keeps its whole K = kpad slice of S or A in VGPRs
//    (read once from HBM) and streams the table through LDS in 16-row tiles
//    of both parities; each tile is one 16 x 16 output block per wave.
//  * synthesis: the wave keeps its whole kpad x 16 output block in VGPRs and
//    streams table tiles and 16-degree slices of the spectrum through LDS.
// Workgroups are dealt to XCDs in chunks of 16 consecutive m so that each
// XCD gets a balanced share of the triangle and the 8-byte accesses of
// neighbouring m to the spectral tensor (m fastest) meet in its L2.
#include "internal.h"

namespace sht {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
// native 4-float vector for register staging and 128-bit LDS / global
// accesses (HIP's float4 is a struct and its copies do not stay in VGPRs)
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int TR = 16;  // table rows per parity per LDS tile

__device__ __forceinline__ int2 take_work(const int2* __restrict__ work, int per) {
  const int slot = (blockIdx.x % 8) * per + blockIdx.x / 8;
  return work[slot];
}

// One pipeline stage of the table: rows [16 ib, 16 ib + 16) of both parity
// blocks of order m, restricted to the ring half [h KH, h KH + KH).  It is
// fetched into registers one stage ahead (4 float4 per thread for the
// 384-ring grids) and written to an LDS buffer Pt[2][16][KH + 4] after the
// current stage's MFMAs; the pipeline needs one barrier per stage.
template <int KPAD, int NTH>
struct HalfTile {
  static constexpr int KH = KPAD / 2;
  static constexpr int Q = KH / 4;  // float4 per half row
  static constexpr int PITCH = KH + 4;
  static constexpr int N4 = 2 * TR * Q;
  static constexpr int PER = (N4 + NTH - 1) / NTH;
  static constexpr int FULL = N4 / NTH;
  static constexpr int LDS = 2 * TR * PITCH;  // floats per buffer
  __device__ static __forceinline__ int goff(int rows_pad, int ib, int h, int e) {
    const int pp = e / (TR * Q);
    const int rem = e - pp * TR * Q;
    const int r = rem / Q;
    const int q = rem - r * Q;
    return (pp * rows_pad + TR * ib + r) * KPAD + h * KH + 4 * q;
  }
  __device__ static __forceinline__ int loff(int e) {
    const int pp = e / (TR * Q);
    const int rem = e - pp * TR * Q;
    const int r = rem / Q;
    const int q = rem - r * Q;
    return (pp * TR + r) * PITCH + 4 * q;
  }
};
// fetch / store of a HalfTile stage through the register array V[PER]
#define SHT_TILE_FETCH(V, T0, ROWS_PAD, IB, H)                                                      \
  _Pragma("unroll") for (int u_ = 0; u_ < Tile::PER; ++u_) {                                        \
    const int e_ = threadIdx.x + u_ * NTH;                                                          \
    if (u_ < Tile::FULL || e_ < Tile::N4)                                                           \
      V[u_] = *reinterpret_cast<const v4f*>((T0) + Tile::goff((ROWS_PAD), (IB), (H), e_));          \
  }
#define SHT_TILE_STORE(V, PT)                                                                       \
  _Pragma("unroll") for (int u_ = 0; u_ < Tile::PER; ++u_) {                                        \
    const int e_ = threadIdx.x + u_ * NTH;                                                          \
    if (u_ < Tile::FULL || e_ < Tile::N4) *reinterpret_cast<v4f*>((PT) + Tile::loff(e_)) = V[u_];    \
  }

// Analysis.  A wave's K = KPAD contraction is split into two ring halves of
// KSH = KS/2 substeps; within half h, substep s' and lane group lk cover ring
// k = h KH + lk KSH + s', so that one 128-bit LDS read yields the A operands
// of four consecutive substeps.  Pipeline stages are (16-row tile ib, half h).
template <int NCB, int KS>
__global__ __launch_bounds__(128 * NCB, 3) void analysis_kernel(LegArgs a, const int2* __restrict__ work, int per,
                                                                const float* __restrict__ W,
                                                                float2* __restrict__ y, float c_rest) {
  constexpr int NTH = 128 * NCB;
  constexpr int KPAD = 4 * KS;
  constexpr int KSH = KS / 2;
  using Tile = HalfTile<KPAD, NTH>;
  constexpr int PITCH = Tile::PITCH;
  static_assert(KSH % 4 == 0, "KS");
  __shared__ __attribute__((aligned(16))) float Pt[2 * Tile::LDS];
  const int2 wk = take_work(work, per);
  const int m = wk.x, c = wk.y;
  if (m < 0) return;
  const SegGeom& g = a.g;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = wave / NCB, j = wave - p * NCB;
  const int cb = c * NCB + j;
  const bool active = cb < g.groups;
  const int li = lane & 15, lk = lane >> 4;
  float xr[KS];
  if (active) {
    const float* Wp = W + (static_cast<size_t>(2 * m + p) * g.groups + cb) * KPAD * 16;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k = (s / KSH) * Tile::KH + lk * KSH + (s % KSH);
      xr[s] = Wp[k * 16 + li];
    }
  }
  const int n0 = (g.lmax - m + 1) >> 1;
  const int np = p ? (g.lmax - m) >> 1 : n0;
  const int nblk = (n0 + TR - 1) / TR;
  const int nst = 2 * nblk;
  const float* T0 = static_cast<const float*>(a.table) + static_cast<size_t>(a.row_off[m]) * KPAD;
  const int rows_pad = a.rows_pad[m];
  const float ms = (m == 0) ? 1.f : c_rest;
  float* yf = reinterpret_cast<float*>(y);
  const int f = 8 * cb + (li >> 1);
  v4f tv[Tile::PER];
  SHT_TILE_FETCH(tv, T0, rows_pad, 0, 0);
  SHT_TILE_STORE(tv, Pt);
  __syncthreads();
  SHT_TILE_FETCH(tv, T0, rows_pad, 0, 1);
  const bool work_rows = active;
  for (int ib = 0; ib < nblk; ++ib) {
    const bool mine = work_rows && TR * ib < np;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int st = 2 * ib + h;
      if (mine) {
        const v4f* Pr = reinterpret_cast<const v4f*>(Pt + h * Tile::LDS + (p * TR + li) * PITCH + lk * KSH);
        v4f cur = Pr[0];
#pragma unroll
        for (int t = 0; t < KSH / 4; ++t) {
          const v4f nxt = (t + 1 < KSH / 4) ? Pr[t + 1] : cur;
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(cur.x, xr[h * KSH + 4 * t + 0], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(cur.y, xr[h * KSH + 4 * t + 1], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(cur.z, xr[h * KSH + 4 * t + 2], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(cur.w, xr[h * KSH + 4 * t + 3], acc, 0, 0, 0);
          cur = nxt;
        }
      }
      if (st + 1 < nst) SHT_TILE_STORE(tv, Pt + (1 - h) * Tile::LDS);
      __syncthreads();
      if (st + 2 < nst) SHT_TILE_FETCH(tv, T0, rows_pad, ib + 1, h);
    }
    if (mine && f < g.F) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = TR * ib + 4 * lk + r;
        if (i < np) {
          const int l = m + p + 2 * i;
          yf[((static_cast<size_t>(f) * g.lmax + l) * g.mmax + m) * 2 + (li & 1)] = acc[r] * ms;
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

// Synthesis.  A workgroup owns ring half kh of order m for one column chunk;
// output ring k = kh KH + i KR + rb of a wave's block (MFMA row i, row block
// rb) so that one 128-bit LDS read yields the A operands of four consecutive
// row blocks.  Pipeline stages are 16-degree tiles of both parities.
template <int NCB, int KS>
__global__ __launch_bounds__(128 * NCB, 3) void synthesis_kernel(LegArgs a, const int2* __restrict__ work, int per,
                                                                 const float2* __restrict__ y,
                                                                 float* __restrict__ W) {
  constexpr int NTH = 128 * NCB;
  constexpr int KPAD = 4 * KS;
  using Tile = HalfTile<KPAD, NTH>;
  constexpr int KH = Tile::KH;
  constexpr int KR = KH / 16;  // 16-ring output blocks of the half
  static_assert(KR % 4 == 0, "KR");
  constexpr int PITCH = Tile::PITCH;
  constexpr int NF = 8 * NCB;       // fields of the chunk
  constexpr int BPITCH = 2 * NF + 4;
  constexpr int BLDS = 2 * TR * BPITCH;
  constexpr int NB = 2 * TR * NF;   // spectral values per stage
  constexpr int BPER = (NB + NTH - 1) / NTH;
  __shared__ __attribute__((aligned(16))) float Pt[2 * Tile::LDS];
  __shared__ __attribute__((aligned(16))) float Bt[2 * BLDS];
  const int2 wk = take_work(work, per);
  const int m = wk.x;
  if (m < 0) return;
  const int c = wk.y >> 1, kh = wk.y & 1;
  const SegGeom& g = a.g;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = wave / NCB, j = wave - p * NCB;
  const int cb = c * NCB + j;
  const bool active = cb < g.groups;
  const int n0 = (g.lmax - m + 1) >> 1;
  const int n1 = (g.lmax - m) >> 1;
  const int np = p ? n1 : n0;
  const int nblk = (n0 + TR - 1) / TR;
  const float* T0 = static_cast<const float*>(a.table) + static_cast<size_t>(a.row_off[m]) * KPAD;
  const int rows_pad = a.rows_pad[m];
  const int li = lane & 15, lk = lane >> 4;
  const int fbeg = NF * c;
  // 16 degrees of each parity x this chunk's fields, gathered from the
  // spectral tensor (m fastest)
  float2 bv_reg[BPER];
#define SHT_FETCH_B(IB)                                                                       \
  _Pragma("unroll") for (int u = 0; u < BPER; ++u) {                                          \
    const int e = threadIdx.x + u * NTH;                                                      \
    float2 v = make_float2(0.f, 0.f);                                                         \
    if (e < NB) {                                                                             \
      const int pp = e / (TR * NF);                                                           \
      const int rem = e - pp * TR * NF;                                                       \
      const int r = rem / NF;                                                                 \
      const int fl = rem - r * NF;                                                            \
      const int i = TR * (IB) + r;                                                            \
      const int ff = fbeg + fl;                                                               \
      if (i < (pp ? n1 : n0) && ff < g.F)                                                     \
        v = y[(static_cast<size_t>(ff) * g.lmax + m + pp + 2 * i) * g.mmax + m];              \
    }                                                                                         \
    bv_reg[u] = v;                                                                            \
  }
#define SHT_STORE_B(B)                                                                        \
  _Pragma("unroll") for (int u = 0; u < BPER; ++u) {                                          \
    const int e = threadIdx.x + u * NTH;                                                      \
    if (e < NB) {                                                                             \
      const int pp = e / (TR * NF);                                                           \
      const int rem = e - pp * TR * NF;                                                       \
      const int r = rem / NF;                                                                 \
      const int fl = rem - r * NF;                                                            \
      *reinterpret_cast<float2*>((B) + (pp * TR + r) * BPITCH + 2 * fl) = bv_reg[u];          \
    }                                                                                         \
  }
  floatx4 acc[KR];
#pragma unroll
  for (int rb = 0; rb < KR; ++rb) acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
  v4f tv[Tile::PER];
  SHT_TILE_FETCH(tv, T0, rows_pad, 0, kh);
  SHT_FETCH_B(0);
  SHT_TILE_STORE(tv, Pt);
  SHT_STORE_B(Bt);
  __syncthreads();
  if (nblk > 1) {
    SHT_TILE_FETCH(tv, T0, rows_pad, 1, kh);
    SHT_FETCH_B(1);
  }
  constexpr int NQ = 4 * (KR / 4);
  for (int ib = 0; ib < nblk; ++ib) {
    const float* Pb = Pt + (ib & 1) * Tile::LDS;
    const float* Bb = Bt + (ib & 1) * BLDS;
    if (active && TR * ib < np) {
      // flattened schedule q = (substep s, 4-block group t): one 128-bit A
      // read and four MFMAs per step, A reads issued two steps ahead
      const float* Pbase = Pb + (p * TR + lk) * PITCH + li * KR;
      float bvs[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) bvs[s] = Bb[(p * TR + 4 * s + lk) * BPITCH + 16 * j + li];
      v4f ring[3];
      ring[0] = reinterpret_cast<const v4f*>(Pbase)[0];
      ring[1] = reinterpret_cast<const v4f*>(Pbase + 4 * (1 / (KR / 4)) * PITCH)[1 % (KR / 4)];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (q + 2 < NQ) {
          const int s2 = (q + 2) / (KR / 4), t2 = (q + 2) - s2 * (KR / 4);
          ring[(q + 2) % 3] = reinterpret_cast<const v4f*>(Pbase + 4 * s2 * PITCH)[t2];
        }
        const int s = q / (KR / 4), t = q - s * (KR / 4);
        const v4f av = ring[q % 3];
        acc[4 * t + 0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bvs[s], acc[4 * t + 0], 0, 0, 0);
        acc[4 * t + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bvs[s], acc[4 * t + 1], 0, 0, 0);
        acc[4 * t + 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bvs[s], acc[4 * t + 2], 0, 0, 0);
        acc[4 * t + 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bvs[s], acc[4 * t + 3], 0, 0, 0);
      }
    }
    if (ib + 1 < nblk) {
      SHT_TILE_STORE(tv, Pt + ((ib + 1) & 1) * Tile::LDS);
      SHT_STORE_B(Bt + ((ib + 1) & 1) * BLDS);
    }
    __syncthreads();
    if (ib + 2 < nblk) {
      SHT_TILE_FETCH(tv, T0, rows_pad, ib + 2, kh);
      SHT_FETCH_B(ib + 2);
    }
  }
#undef SHT_FETCH_B
#undef SHT_STORE_B
#undef SHT_TILE_FETCH
#undef SHT_TILE_STORE
  if (active) {
    float* Wp = W + (static_cast<size_t>(2 * m + p) * g.groups + cb) * KPAD * 16 + static_cast<size_t>(kh) * KH * 16;
#pragma unroll
    for (int rb = 0; rb < KR; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) Wp[((4 * lk + r) * KR + rb) * 16 + li] = acc[rb][r];
  }
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
    case 32: return launch_pair<NCB, 32>(analysis, a, in, out, c_rest, st);
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
  const int ks[] = {32, 64, 96};
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
