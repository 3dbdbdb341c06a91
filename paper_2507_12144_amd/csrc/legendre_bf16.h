// bf16 forms of the Legendre contraction (the per-order-m contraction of
// Alg. 1 and its synthesis counterpart of eq. isht) on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16, float32 accumulation).
//
// Precision forms.  The table is stored as NP bf16 planes (rounded to
// nearest even from the float64 recurrence: hi = bf16(v), then the
// residuals); the data (folded DFT output, or spectrum) are split the same
// way in float32 when they arrive.  With a = sum_i a_i, b = sum_j b_j the
// kernels form
//   NP = 1: a_0 b_0                                   (plain bf16)
//   NP = 2: a_0 b_0 + a_0 b_1 + a_1 b_0               (split bf16)
//   NP = 3: all a_i b_j with i + j < 3 (six products) (three-term split)
// i.e. every product whose magnitude is above the representation error of
// the split.  The correction products of the analysis go into their own
// accumulator, added to the leading one at the end of each output block.
//
// Structure as in the float32 kernels: one workgroup of four waves per
// (segment, m, chunk of two field groups), wave (p, j) owns parity p and one
// 16-column field group; the table pieces (1 KiB: one plane of one K = 32
// step of a 16-row block, 16 bytes a lane) flow through a ring of three LDS
// buffers filled by asynchronous global->LDS copies, each stage carrying SS
// steps x NP planes for both parities.  Analysis: the wave's K slice of S or
// A arrives through the ring first and is split into planes in VGPRs.
// Synthesis: 32-row blocks (K = 32), the spectrum values of the next block
// are loaded one block ahead and split when their block starts.
#pragma once

#include "bf16.h"
#include "internal.h"
#include "kernel_common.h"

namespace sht {
namespace bf16p {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
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

// Steps per stage: the largest divisor of the steps of a row block whose
// NP planes fit in 8 pieces.
constexpr int steps_per_stage(int steps, int np) {
  for (int ss = steps; ss > 1; --ss)
    if (steps % ss == 0 && ss * np <= 8) return ss;
  return 1;
}

// Stage geometry: steps of K = 32 per row block, SS steps (SC = SS * NP
// pieces per parity) per stage, PARTS stages per row block; NST stages
// unrolled into straight-line code (lmax <= 2 kpad; larger lmax goes round
// an outer loop), a multiple of the period of buffer (stage % 3) and part.
template <int STEPS, int NP, int MAXBLK>
struct Geo {
  static constexpr int SS = steps_per_stage(STEPS, NP);
  static constexpr int SC = SS * NP;
  static constexpr int PARTS = STEPS / SS;
  static constexpr int LPW = (2 * SC + 3) / 4;  // copies per wave and stage (4 waves)
  static constexpr int PERIOD = (PARTS % 3 == 0) ? PARTS : 3 * PARTS;
  static constexpr int NST = ((PARTS * MAXBLK + PERIOD - 1) / PERIOD) * PERIOD;
  static_assert(2 * SC <= 16, "stage buffer");
};

// Copy stage st (row block st / PARTS, part st % PARTS) of both parities:
// piece e < 2 SC of the stage is parity e / SC, piece e % SC; pieces are
// 512 bf16 (1 KiB), blk_pieces per row block, par_blocks row blocks per
// parity region.  Stages past the last row block re-read the last one.
template <int SC, int LPW, int PARTS>
__device__ __forceinline__ void issue_stage(v4f* B, const uint16_t* __restrict__ tab, int par_blocks, int nb,
                                            int blk_pieces, int st, int wave, int lane) {
  const int ib = min(st / PARTS, nb - 1), h = st - (st / PARTS) * PARTS;
#pragma unroll
  for (int i = 0; i < LPW; ++i) {
    const int e = min(wave + i * 4, 2 * SC - 1);
    const int pp = e >= SC ? 1 : 0;
    const int t = e - pp * SC;
    const uint16_t* src =
        tab + (static_cast<size_t>(pp * par_blocks + ib) * blk_pieces + h * SC + t) * 512 + lane * 8;
    __builtin_amdgcn_global_load_lds(src, B + (pp * SC + t) * 64, 16, 0, 0);
  }
}

__device__ __forceinline__ bf16x8 as_bf16x8(v4f v) { return __builtin_bit_cast(bf16x8, v); }

// Analysis.  Contraction index k of a wave's K slice = lk * KS + 8t + e for
// lane group lk, step t (K = 32: 8 values a lane) and element e.
template <int KS, int NP>
__device__ __forceinline__ void analysis_body(const SegDev& sd, int m, int c, float2* __restrict__ y, float c_rest,
                                              v4f* b0, v4f* b1, v4f* b2) {
  constexpr int T8 = KS / 8;  // steps per 16-row block
  using G = Geo<T8, NP, KS / 4>;
  constexpr int SC = G::SC, SS = G::SS, LPW = G::LPW, PARTS = G::PARTS;
  constexpr int KPAD = 4 * KS;
  constexpr int XS = KS / 16;  // stages of S / A (16 rings per lane group)
  const SegGeom& g = sd.g;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = wave >> 1, j = wave & 1;
  const int cb = c * 2 + j;
  const bool active = cb < g.groups;
  const int li = lane & 15, lk = lane >> 4;
  const int n0 = (g.lmax - m + 1) >> 1;
  const int nb = (n0 + 15) >> 4;          // 16-row blocks of parity 0
  const int nb32 = (n0 + 31) >> 5;        // the table holds 2 nb32 per parity
  const int np = p ? (g.lmax - m) >> 1 : n0;
  const int nbp = (np + 15) >> 4;
  const int nst = PARTS * nb;
  const uint16_t* tab = static_cast<const uint16_t*>(sd.tab_ana) + sd.tab_off[m];
  const float* Wg = sd.work + (static_cast<size_t>(2 * m + p) * g.groups + (active ? cb : 0)) * KPAD * 16;
  const float ms = (m == 0) ? 1.f : c_rest;
  float* yf = reinterpret_cast<float*>(y);
  const int f = 8 * cb + (li >> 1);
  const bool fok = active && f < g.F;
  if (nb > 0) {
    bf16x8 xs[T8][NP];
    // stage u < XS: rings lk * KS + 16u .. +15 of every lane group of every
    // wave (piece 4 wave + lk); table stage s follows as stage XS + s
    auto issue_x = [&](v4f* B, int u) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        __builtin_amdgcn_global_load_lds(Wg + (q * KS + 16 * u) * 16 + lane * 4, B + (4 * wave + q) * 64, 16, 0, 0);
    };
    issue_x(b0, 0);
    if constexpr (XS > 1)
      issue_x(b1, 1);
    else
      issue_stage<SC, LPW, PARTS>(b1, tab, 2 * nb32, nb, T8 * NP, 0, wave, lane);
    unrolled<0, XS>([&](auto u_c) {
      constexpr int u = decltype(u_c)::value;
      v4f* cur = ring_buf<u>(b0, b1, b2);
      v4f* nxt = ring_buf<u + 2>(b0, b1, b2);
      __builtin_amdgcn_s_waitcnt(vm_wait(u + 1 < XS ? 4 : LPW));
      stage_barrier();
      if constexpr (u + 2 < XS)
        issue_x(nxt, u + 2);
      else
        issue_stage<SC, LPW, PARTS>(nxt, tab, 2 * nb32, nb, T8 * NP, u + 2 - XS, wave, lane);
      const float* xb = reinterpret_cast<const float*>(cur) + (4 * wave + lk) * 256 + li;
      float v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = xb[16 * r];
      split8<NP>(v, xs[2 * u]);
      split8<NP>(v + 8, xs[2 * u + 1]);
      return true;
    });
    floatx4 main = {0.f, 0.f, 0.f, 0.f}, corr = main;
    for (int st0 = 0; st0 < nst; st0 += G::NST) {
      unrolled<0, G::NST>([&](auto su_c) {
        constexpr int su = decltype(su_c)::value;
        constexpr int part = su % PARTS;
        const int st = st0 + su;
        if (st >= nst) return false;
        v4f* cur = ring_buf<su + XS>(b0, b1, b2);
        v4f* nxt = ring_buf<su + XS + 2>(b0, b1, b2);
        __builtin_amdgcn_s_waitcnt(vm_wait(LPW));
        stage_barrier();
        issue_stage<SC, LPW, PARTS>(nxt, tab, 2 * nb32, nb, T8 * NP, st + 2, wave, lane);
        const int ib = st / PARTS;
        if (active && ib < nbp) {
#pragma unroll
          for (int s = 0; s < SS; ++s) {
            bf16x8 av[NP];
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) av[pl] = as_bf16x8(cur[(p * SC + s * NP + pl) * 64 + lane]);
            products<NP>(av, xs[part * SS + s], main, corr);
          }
          if constexpr (part == PARTS - 1) {
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
            main = floatx4{0.f, 0.f, 0.f, 0.f};
            corr = main;
          }
        }
        return true;
      });
    }
    // no copy may still be writing this workgroup's LDS when it ends
    __builtin_amdgcn_s_waitcnt(vm_wait(0));
  }
  // zeros of the spectrum: degree l = m, orders m+1 .. mmax-1 of this
  // chunk's fields (contiguous runs; the orders together cover every l < m')
  if (m < g.lmax) {
    const int fbeg = 16 * c;
    const int fend = min(g.F, fbeg + 16);
    const int run = g.mmax - 1 - m;
    for (int ff = fbeg; ff < fend; ++ff) {
      float2* row = y + (static_cast<size_t>(ff) * g.lmax + m) * g.mmax + m + 1;
      for (int e = threadIdx.x; e < run; e += 256) row[e] = make_float2(0.f, 0.f);
    }
  }
}

// Synthesis.  Contraction rows i = 32 ib + 8 lk + e of the wave's parity;
// output ring k = (MFMA row) * KR + rb for step rb of a 32-row block.
template <int KS, int NP>
__device__ __forceinline__ void synthesis_body(const SegDev& sd, int m, int c, const float2* __restrict__ y,
                                               v4f* b0, v4f* b1, v4f* b2) {
  constexpr int KPAD = 4 * KS;
  constexpr int KR = KPAD / 16;  // steps (16-ring output blocks) per 32-row block
  using G = Geo<KR, NP, KS / 8>;
  constexpr int SC = G::SC, SS = G::SS, LPW = G::LPW, PARTS = G::PARTS;
  constexpr int NB = 8;  // B loads per lane and row block
  const SegGeom& g = sd.g;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = wave >> 1, j = wave & 1;
  const int cb = c * 2 + j;
  const bool active = cb < g.groups;
  const int li = lane & 15, lk = lane >> 4;
  const int n0 = (g.lmax - m + 1) >> 1;
  const int nb32 = (n0 + 31) >> 5;
  const int np = p ? (g.lmax - m) >> 1 : n0;
  const int nbp = (np + 31) >> 5;
  const int nst = PARTS * nb32;
  const uint16_t* tab = static_cast<const uint16_t*>(sd.tab_syn) + sd.tab_off[m];
  // B operand of lane (li, lk) for block ib: re (li even) or im (li odd) of
  // field 8 cb + li/2 at degrees l = m + p + 2 (32 ib + 8 lk + e), e < 8.
  // Rows past the parity's last degree read degree m instead (their table
  // rows are zero); lanes of fields past F read field 0 (never read back).
  const float* yf = reinterpret_cast<const float*>(y);
  const int f = 8 * cb + (li >> 1);
  const bool fok = active && f < g.F;
  const size_t fbase = (static_cast<size_t>(fok ? f : 0) * g.lmax) * g.mmax;
  float bn[NB];
  auto bload = [&](int ib) {
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int i = 32 * ib + 8 * lk + e;
      const int l = i < np ? m + p + 2 * i : m;
      bn[e] = yf[(fbase + static_cast<size_t>(l) * g.mmax + m) * 2 + (li & 1)];
    }
  };
  floatx4 acc[KR];
#pragma unroll
  for (int rb = 0; rb < KR; ++rb) acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
  if (nb32 > 0) {
    // Stage u issues the copies of stage u+2 and then, when it opens a row
    // block, the B loads of the next one; the prologue plays stages -2 and
    // -1 the same way (B loads of row block 0 first when neither opens a
    // block).  The loads issued after the copies of stage s are those of
    // stage s+1 and the B loads of stages s-2 and s-1 that open blocks.
    constexpr int pm2 = ((-2 % PARTS) + PARTS) % PARTS, pm1 = PARTS - 1;
    if constexpr (pm2 != 0 && pm1 != 0) {
      bload(0);
      asm volatile("" ::: "memory");
    }
    issue_stage<SC, LPW, PARTS>(b0, tab, nb32, nb32, KR * NP, 0, wave, lane);
    if constexpr (pm2 == 0) {
      asm volatile("" ::: "memory");
      bload(0);
      asm volatile("" ::: "memory");
    }
    issue_stage<SC, LPW, PARTS>(b1, tab, nb32, nb32, KR * NP, 1, wave, lane);
    if constexpr (pm1 == 0) {
      asm volatile("" ::: "memory");
      bload(0);
      asm volatile("" ::: "memory");
    }
    bf16x8 bv[NP];
    for (int st0 = 0; st0 < nst; st0 += G::NST) {
      unrolled<0, G::NST>([&](auto su_c) {
        constexpr int su = decltype(su_c)::value;
        constexpr int part = su % PARTS;
        const int st = st0 + su;
        if (st >= nst) return false;
        v4f* cur = ring_buf<su>(b0, b1, b2);
        v4f* nxt = ring_buf<su + 2>(b0, b1, b2);
        constexpr int q2 = (part + 2 * PARTS - 2) % PARTS, q1 = (part + PARTS - 1) % PARTS;
        __builtin_amdgcn_s_waitcnt(vm_wait(LPW + NB * ((q2 == 0 ? 1 : 0) + (q1 == 0 ? 1 : 0))));
        stage_barrier();
        const int ib = st / PARTS;
        if constexpr (part == 0) split8<NP>(bn, bv);
        issue_stage<SC, LPW, PARTS>(nxt, tab, nb32, nb32, KR * NP, st + 2, wave, lane);
        if constexpr (part == 0) {
          asm volatile("" ::: "memory");
          bload(ib + 1);
          asm volatile("" ::: "memory");
        }
        if (active && ib < nbp) {
#pragma unroll
          for (int s = 0; s < SS; ++s) {
            bf16x8 av[NP];
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) av[pl] = as_bf16x8(cur[(p * SC + s * NP + pl) * 64 + lane]);
            products<NP>(av, bv, acc[part * SS + s], acc[part * SS + s]);
          }
        }
        return true;
      });
    }
    __builtin_amdgcn_s_waitcnt(vm_wait(0));
  }
  if (!active) return;
  float* Wp = sd.work + (static_cast<size_t>(2 * m + p) * g.groups + cb) * KPAD * 16;
#pragma unroll
  for (int rb = 0; rb < KR; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) Wp[((4 * lk + r) * KR + rb) * 16 + li] = acc[rb][r];
}

// Waves per SIMD the kernels are compiled for: 3 (168 VGPRs) holds the
// one-plane operands; the split forms keep NP planes of the data in VGPRs
// (up to 144 of them at 384 rings) and get 256.
constexpr int waves_per_eu(int np) { return np == 1 ? 3 : 2; }

// Batched kernels of one plane count (items {m, (segment << 16) | chunk}).
template <int NP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(waves_per_eu(NP)))) void analysis_batched(
    const SegDev* __restrict__ segs, const int2* __restrict__ work, int per, float2* __restrict__ y, float c_rest) {
  __shared__ v4f b0[16 * 64], b1[16 * 64], b2[16 * 64];
  const int2 wk = take_work(work, per);
  if (wk.x < 0) return;
  const SegDev& sd = segs[wk.y >> 16];
  const int m = wk.x, c = wk.y & 0xffff;
  float2* ys = y + sd.spec_off;
  switch (sd.g.kpad) {
    case 64: analysis_body<16, NP>(sd, m, c, ys, c_rest, b0, b1, b2); break;
    case 128: analysis_body<32, NP>(sd, m, c, ys, c_rest, b0, b1, b2); break;
    case 192: analysis_body<48, NP>(sd, m, c, ys, c_rest, b0, b1, b2); break;
    case 256: analysis_body<64, NP>(sd, m, c, ys, c_rest, b0, b1, b2); break;
    default: analysis_body<96, NP>(sd, m, c, ys, c_rest, b0, b1, b2); break;
  }
}

template <int NP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(waves_per_eu(NP)))) void synthesis_batched(
    const SegDev* __restrict__ segs, const int2* __restrict__ work, int per, const float2* __restrict__ y) {
  __shared__ v4f b0[16 * 64], b1[16 * 64], b2[16 * 64];
  const int2 wk = take_work(work, per);
  if (wk.x < 0) return;
  const SegDev& sd = segs[wk.y >> 16];
  const int m = wk.x, c = wk.y & 0xffff;
  const float2* ys = y + sd.spec_off;
  switch (sd.g.kpad) {
    case 64: synthesis_body<16, NP>(sd, m, c, ys, b0, b1, b2); break;
    case 128: synthesis_body<32, NP>(sd, m, c, ys, b0, b1, b2); break;
    case 192: synthesis_body<48, NP>(sd, m, c, ys, b0, b1, b2); break;
    case 256: synthesis_body<64, NP>(sd, m, c, ys, b0, b1, b2); break;
    default: synthesis_body<96, NP>(sd, m, c, ys, b0, b1, b2); break;
  }
}

template <int NP>
hipError_t launch_batched(bool analysis, const BatchArgs& b, const void* in, void* out, float c_rest,
                          hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(8 * b.work_per));
  if (analysis)
    hipLaunchKernelGGL(analysis_batched<NP>, grid, dim3(256), 0, st, b.segs, b.work, b.work_per,
                       static_cast<float2*>(out), c_rest);
  else
    hipLaunchKernelGGL(synthesis_batched<NP>, grid, dim3(256), 0, st, b.segs, b.work, b.work_per,
                       static_cast<const float2*>(in));
  return hipGetLastError();
}

extern template hipError_t launch_batched<1>(bool, const BatchArgs&, const void*, void*, float, hipStream_t);
extern template hipError_t launch_batched<2>(bool, const BatchArgs&, const void*, void*, float, hipStream_t);
extern template hipError_t launch_batched<3>(bool, const BatchArgs&, const void*, void*, float, hipStream_t);

}  // namespace bf16p
}  // namespace sht
