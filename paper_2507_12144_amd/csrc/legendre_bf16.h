// bf16 forms of the Legendre contraction (the per-order-m contraction of
// Alg. 1 and its synthesis counterpart of eq. isht) on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16, float32 accumulation).
//
// Precision forms.  The table is stored as NP bf16 planes (rounded to
// nearest even from the float64 recurrence: hi = bf16(v), then the
// residuals); the data (folded DFT output, or spectrum) are split into ND
// planes in float32 in VGPRs when they arrive, ND = 1 for plain bf16 and 3
// otherwise (a third data plane costs no memory traffic).  With
// a = sum_i a_i (table), b = sum_j b_j (data) the kernels form every
// product a_i b_j with i < NP, j < ND and i + j < ND:
//   NP = 1: a_0 b_0                                        (plain bf16)
//   NP = 2: a_0 b_0 + a_0 b_1 + a_1 b_0 + a_0 b_2 + a_1 b_1 (split bf16)
//   NP = 3: all a_i b_j with i + j < 3 (six products)      (three-term split)
// For NP = 2 the only error term left above float32 rounding is the
// representation error of the two-plane table (at most 2^-16 relative,
// about 2^-18 on average), so the data's own split and the dropped a_1 b_1
// product no longer add to it.  The correction products of the analysis go
// into their own accumulator, added to the leading one at the end of each
// output block.
//
// Structure as in the float32 kernels: one workgroup of four waves per
// (segment, m, chunk of two field groups), wave (p, j) owns parity p and one
// 16-column field group; the table pieces (1 KiB: one plane of one K = 32
// step of a 16-row block, 16 bytes a lane) flow through a ring of 16 KiB LDS
// buffers filled by asynchronous global->LDS copies, each stage carrying SS
// steps x NP planes for both parities.  Analysis: five buffers (four stages
// in flight); the wave's K slice of S or A arrives through the ring first
// and is split into planes in VGPRs.  Synthesis: four buffers and a
// spectrum slot; 32-row blocks (K = 32), the spectrum values of the next
// block arrive by 4-byte copies during the current one and are split when
// their block starts.
#pragma once

#include "bf16.h"
#include "internal.h"
#include "kernel_common.h"
#include "stage_waits.h"

namespace sht {
namespace bf16p {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// Split 8 float32 values into NP bf16 planes (residuals in float32, exact).
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

// Data planes of the form with NP table planes.
constexpr int data_planes(int np) { return np == 1 ? 1 : 3; }

// Products a_i b_j (i < NP, j < ND, i + j < ND) between the split table a
// and the split data b.
template <int NP, int ND>
__device__ __forceinline__ void products(const bf16x8* a, const bf16x8* b, floatx4& main, floatx4& corr) {
  main = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], main, 0, 0, 0);
  if constexpr (ND >= 2) {
    corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], corr, 0, 0, 0);
    if constexpr (NP >= 2) corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], corr, 0, 0, 0);
  }
  if constexpr (ND >= 3) {
    corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], corr, 0, 0, 0);
    if constexpr (NP >= 2) corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], corr, 0, 0, 0);
    if constexpr (NP >= 3) corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], corr, 0, 0, 0);
  }
}

// Steps per stage: the largest divisor of the steps of a row block whose
// NP planes fit in 8 pieces and that leaves at least min_parts stages per
// row block.
constexpr int steps_per_stage(int steps, int np, int min_parts) {
  for (int ss = steps; ss > 1; --ss)
    if (steps % ss == 0 && ss * np <= 8 && steps / ss >= min_parts) return ss;
  return 1;
}

// Stage geometry: steps of K = 32 per row block, SS steps (SC = SS * NP
// pieces per parity) per stage, PARTS stages per row block; NST stages
// unrolled into straight-line code (lmax <= 2 kpad; larger lmax goes round
// an outer loop), a multiple of the period of buffer (stage % NBUF) and
// part.
constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }
template <int STEPS, int NP, int MAXBLK, int NBUF, int MIN_PARTS = 1>
struct Geo {
  static constexpr int SS = steps_per_stage(STEPS, NP, MIN_PARTS);
  static constexpr int SC = SS * NP;
  static constexpr int PARTS = STEPS / SS;
  static constexpr int LPW = (2 * SC + 3) / 4;  // copies per wave and stage (4 waves)
  static constexpr int PERIOD = PARTS / gcd_c(PARTS, NBUF) * NBUF;
  static constexpr int NST = ((PARTS * MAXBLK + PERIOD - 1) / PERIOD) * PERIOD;
  static_assert(2 * SC <= 16, "stage buffer");
};

// Buffers of the LDS ring: NBUF stages of 16 pieces (16 KiB); stage g
// lives in buffer g % NBUF and is copied NBUF - 1 stages ahead.
template <int G, int NBUF>
__device__ __forceinline__ v4f* rbuf(v4f* ring) {
  return ring + (G % NBUF) * 16 * 64;
}

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
// lane group lk, step t (K = 32: 8 values a lane) and element e.  Global
// stage g < XS brings rings 16g .. 16g+15 of every lane group's K slice of
// S or A (each wave its own four pieces); stage XS + s is table stage s.
template <int KS, int NP, int NBUF, bool STG>
__device__ __forceinline__ void analysis_body(const SegDev& sd, int m, int c, float2* __restrict__ y, float c_rest,
                                              v4f* ring) {
  constexpr int T8 = KS / 8;  // steps per 16-row block
  using G = Geo<T8, NP, KS / 4, NBUF>;
  constexpr int SC = G::SC, SS = G::SS, LPW = G::LPW, PARTS = G::PARTS;
  constexpr int KPAD = 4 * KS;
  constexpr int XS = KS / 16;
  constexpr int D = NBUF - 1;  // stages in flight
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
  const float* Wg =
      sd.work + static_cast<size_t>(2 * m + p) * g.wslab + static_cast<size_t>(active ? cb : 0) * KPAD * 16;
  const float ms = (m == 0) ? 1.f : c_rest;
  gfloat* yf = as_global(reinterpret_cast<float*>(y));
  const int f = 8 * cb + (li >> 1);
  const bool fok = active && f < g.F;
  // this wave's staging tiles, addressed before the pipeline starts: read
  // inside it, the offset would be reloaded after every stage barrier (a
  // global load whose wait also drains the table copies in flight)
  gfloat* const ystg_out =
      as_global(sd.ystage + sd.ystage_off[m] + (static_cast<size_t>(p) * g.groups + (active ? cb : 0)) * nb * 256);
  if (nb > 0) {
    constexpr int ND = data_planes(NP);
    bf16x8 xs[T8][ND];
    auto issue = [&](auto g_c, int tab_st) {
      constexpr int gs = decltype(g_c)::value;
      v4f* B = rbuf<gs, NBUF>(ring);
      if constexpr (gs < XS) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          __builtin_amdgcn_global_load_lds(Wg + (q * KS + 16 * gs) * 16 + lane * 4, B + (4 * wave + q) * 64, 16, 0,
                                           0);
      } else {
        issue_stage<SC, LPW, PARTS>(B, tab, 2 * nb32, nb, T8 * NP, tab_st, wave, lane);
      }
    };
    unrolled<0, D>([&](auto g_c) {
      issue(g_c, decltype(g_c)::value - XS);
      return true;
    });
    unrolled<0, XS>([&](auto u_c) {
      constexpr int u = decltype(u_c)::value;
      __builtin_amdgcn_s_waitcnt(vm_lds_wait(waits::analysis_behind(XS, LPW, D, u)));
      stage_barrier();
      issue(std::integral_constant<int, u + D>{}, u + D - XS);
      const float* xb = reinterpret_cast<const float*>(rbuf<u, NBUF>(ring)) + (4 * wave + lk) * 256 + li;
      float v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = xb[16 * r];
      split8<ND>(v, xs[2 * u]);
      split8<ND>(v + 8, xs[2 * u + 1]);
      debug_stage_end();
      return true;
    });
    floatx4 main = {0.f, 0.f, 0.f, 0.f}, corr = main;
    for (int st0 = 0; st0 < nst; st0 += G::NST) {
      unrolled<0, G::NST>([&](auto su_c) {
        constexpr int su = decltype(su_c)::value;
        constexpr int part = su % PARTS;
        const int st = st0 + su;
        if (st >= nst) return false;
        __builtin_amdgcn_s_waitcnt(vm_lds_wait(waits::analysis_behind(XS, LPW, D, XS + su)));
        stage_barrier();
        issue(std::integral_constant<int, XS + su + D>{}, st + D);
        const v4f* cur = rbuf<XS + su, NBUF>(ring);
        const int ib = st / PARTS;
        if (active && ib < nbp) {
#pragma unroll
          for (int s = 0; s < SS; ++s) {
            bf16x8 av[NP];
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) av[pl] = as_bf16x8(cur[(p * SC + s * NP + pl) * 64 + lane]);
            products<NP, ND>(av, xs[part * SS + s], main, corr);
          }
          if constexpr (part == PARTS - 1) {
            if constexpr (STG) {
              // the 16 x 16 tile, contiguous, into the order-major staging buffer
              gfloat* dst = ystg_out + static_cast<size_t>(ib) * 256;
#pragma unroll
              for (int r = 0; r < 4; ++r) dst[(4 * lk + r) * 16 + li] = (main[r] + corr[r]) * ms;
            } else {
              // lane pairs (li, li ^ 1) hold re and im of one field: the
              // even lane stores both (8 bytes)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const float v = main[r] + corr[r];
                const float other = __shfl_xor(v, 1, 64);
                const int i = 16 * ib + 4 * lk + r;
                if (fok && (li & 1) == 0 && i < np) {
                  const int l = m + p + 2 * i;
                  *reinterpret_cast<gfloat2*>(yf + ((static_cast<size_t>(f) * g.lmax + l) * g.mmax + m) * 2) =
                      v2f_t{v * ms, other * ms};
                }
              }
            }
            main = floatx4{0.f, 0.f, 0.f, 0.f};
            corr = main;
          }
        }
        debug_stage_end();
        return true;
      });
    }
    // no copy may still be writing this workgroup's LDS when it ends
    __builtin_amdgcn_s_waitcnt(vm_wait(0));
  }
  // zeros of the spectrum: degree l = m, orders m+1 .. mmax-1 of this
  // chunk's fields (contiguous runs; the orders together cover every l < m';
  // staged: the transpose writes them)
  if (!STG && m < g.lmax) {
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
// output ring k = (MFMA row) * KR + rb for step rb of a 32-row block.  The
// spectrum values of a row block (the B operand: 8 per lane) arrive by
// 4-byte global->LDS copies into one slot of 2 KiB per wave (value e of
// lane l at float 64 e + l): all loads in flight are LDS copies, so every
// wait is one of the counted waits below.
template <int KS, int NP, int NBUF, bool STG>
__device__ __forceinline__ void synthesis_body(const SegDev& sd, int m, int c, const float2* __restrict__ y,
                                               v4f* ring, float* spec) {
  constexpr int KPAD = 4 * KS;
  constexpr int KR = KPAD / 16;  // steps (16-ring output blocks) per 32-row block
  using G = Geo<KR, NP, KS / 8, NBUF, 2>;
  constexpr int SC = G::SC, SS = G::SS, LPW = G::LPW, PARTS = G::PARTS;
  static_assert(PARTS >= 2, "the spectrum slot is refilled at part 1");
  constexpr int NB = 8;  // spectrum copies per wave and row block
  constexpr int D = NBUF - 1;
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
  float* wspec = spec + wave * 64 * NB;
  // Staged input: the same values from the order-major staging tiles (rows
  // past the parity's last degree from row 0 of parity 0, degree m).
  const int nbs = (((g.lmax - m + 1) >> 1) + 15) >> 4;
  const float* ystg = sd.ystage + sd.ystage_off[m];
  const int cbs = active ? cb : 0;
  auto spec_copy = [&](int ib) {
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int i = 32 * ib + 8 * lk + e;
      if constexpr (STG) {
        const bool in = i < np;
        const float* src = ystg + ((static_cast<size_t>(in ? p : 0) * g.groups + cbs) * nbs) * 256 +
                           static_cast<size_t>(in ? i : 0) * 16 + li;
        __builtin_amdgcn_global_load_lds(src, wspec + 64 * e, 4, 0, 0);
      } else {
        const int l = i < np ? m + p + 2 * i : m;
        __builtin_amdgcn_global_load_lds(yf + (fbase + static_cast<size_t>(l) * g.mmax + m) * 2 + (li & 1),
                                         wspec + 64 * e, 4, 0, 0);
      }
    }
  };
  floatx4 acc[KR];
#pragma unroll
  for (int rb = 0; rb < KR; ++rb) acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
  if (nb32 > 0) {
    // The prologue plays stages -D .. -1 as the loop does (the table copies
    // of stage v+D and the spectrum of row block 0 where v is at part 1, in
    // the loop's order); when none of them is at part 1, row block 0's
    // spectrum goes first.
    constexpr bool SF = waits::spec_first(PARTS);
    if constexpr (PARTS > D + 1) spec_copy(0);
    unrolled<0, D>([&](auto i_c) {
      constexpr int i = decltype(i_c)::value;
      constexpr bool at1 = (((i - D) % PARTS) + PARTS) % PARTS == 1;
      if constexpr (SF && at1) spec_copy(0);
      issue_stage<SC, LPW, PARTS>(rbuf<i, NBUF>(ring), tab, nb32, nb32, KR * NP, i, wave, lane);
      if constexpr (!SF && at1) spec_copy(0);
      return true;
    });
    constexpr int ND = data_planes(NP);
    bf16x8 bv[ND];
    for (int st0 = 0; st0 < nst; st0 += G::NST) {
      unrolled<0, G::NST>([&](auto su_c) {
        constexpr int su = decltype(su_c)::value;
        constexpr int part = su % PARTS;
        const int st = st0 + su;
        if (st >= nst) return false;
        __builtin_amdgcn_s_waitcnt(vm_lds_wait(waits::synthesis_behind(PARTS, LPW, D, NB, su)));
        stage_barrier();
        const int ib = st / PARTS;
        if constexpr (part == 0) {
          float bn[NB];
#pragma unroll
          for (int e = 0; e < NB; ++e) bn[e] = wspec[64 * e + lane];
          split8<ND>(bn, bv);
        }
        if constexpr (SF && part == 1) spec_copy(ib + 1);
        issue_stage<SC, LPW, PARTS>(rbuf<su + D, NBUF>(ring), tab, nb32, nb32, KR * NP, st + D, wave, lane);
        if constexpr (!SF && part == 1) spec_copy(ib + 1);
        const v4f* cur = rbuf<su, NBUF>(ring);
        if (active && ib < nbp) {
#pragma unroll
          for (int s = 0; s < SS; ++s) {
            bf16x8 av[NP];
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) av[pl] = as_bf16x8(cur[(p * SC + s * NP + pl) * 64 + lane]);
            products<NP, ND>(av, bv, acc[part * SS + s], acc[part * SS + s]);
          }
        }
        debug_stage_end();
        return true;
      });
    }
    __builtin_amdgcn_s_waitcnt(vm_wait(0));
  }
  if (!active) return;
  float* Wp = sd.work + static_cast<size_t>(2 * m + p) * g.wslab + static_cast<size_t>(cb) * KPAD * 16;
#pragma unroll
  for (int rb = 0; rb < KR; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) Wp[((4 * lk + r) * KR + rb) * 16 + li] = acc[rb][r];
}

// LDS ring depth and waves per SIMD: five 16 KiB buffers (four stages in
// flight) take half of the CU's 160 KiB, so two workgroups share a CU and
// each wave may use 256 VGPRs (the split forms keep three planes of the data
// in VGPRs, 144 of them at 384 rings).
constexpr int kRingBuffers = 5;
// Synthesis: four buffers plus the 8 KiB spectrum slot.
constexpr int kSynBuffers = 4;

// Batched kernels of one plane count (items {m, (segment << 16) | chunk}).
template <int NP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void analysis_batched(
    const SegDev* __restrict__ segs, const int2* __restrict__ work, int per, float2* __restrict__ y, float c_rest,
    int staged) {
  __shared__ v4f ring[kRingBuffers * 16 * 64];
  const int2 wk = take_work(work, per);
  if (wk.x < 0) return;
  const SegDev& sd = segs[wk.y >> 16];
  const int m = wk.x, c = wk.y & 0xffff;
  float2* ys = y + sd.spec_off;
  constexpr int R = kRingBuffers;
  // the output path is a compile-time choice, as in the float32 kernels
  auto body = [&](auto ks_c) {
    constexpr int KS = decltype(ks_c)::value;
    if (staged & 1)
      analysis_body<KS, NP, R, true>(sd, m, c, ys, c_rest, ring);
    else
      analysis_body<KS, NP, R, false>(sd, m, c, ys, c_rest, ring);
  };
  switch (sd.g.kpad) {
    case 64: body(std::integral_constant<int, 16>{}); break;
    case 128: body(std::integral_constant<int, 32>{}); break;
    case 192: body(std::integral_constant<int, 48>{}); break;
    case 256: body(std::integral_constant<int, 64>{}); break;
    default: body(std::integral_constant<int, 96>{}); break;
  }
}

template <int NP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void synthesis_batched(
    const SegDev* __restrict__ segs, const int2* __restrict__ work, int per, const float2* __restrict__ y,
    int staged) {
  // one LDS variable for the ring and the spectrum slot: the compiler then
  // leaves the copies to the counted waits instead of waiting for the
  // newest copy into a variable before every read of it
  __shared__ v4f lds[kSynBuffers * 16 * 64 + 4 * 64 * 8 / 4];
  v4f* ring = lds;
  float* spec = reinterpret_cast<float*>(lds + kSynBuffers * 16 * 64);
  const int2 wk = take_work(work, per);
  if (wk.x < 0) return;
  const SegDev& sd = segs[wk.y >> 16];
  const int m = wk.x, c = wk.y & 0xffff;
  const float2* ys = y + sd.spec_off;
  constexpr int R = kSynBuffers;
  // the input source is a compile-time choice, as in the float32 kernels
  auto body = [&](auto ks_c) {
    constexpr int KS = decltype(ks_c)::value;
    if (staged & 2)
      synthesis_body<KS, NP, R, true>(sd, m, c, ys, ring, spec);
    else
      synthesis_body<KS, NP, R, false>(sd, m, c, ys, ring, spec);
  };
  switch (sd.g.kpad) {
    case 64: body(std::integral_constant<int, 16>{}); break;
    case 128: body(std::integral_constant<int, 32>{}); break;
    case 192: body(std::integral_constant<int, 48>{}); break;
    case 256: body(std::integral_constant<int, 64>{}); break;
    default: body(std::integral_constant<int, 96>{}); break;
  }
}

// Launches of one plane count and direction, each explicitly instantiated
// in a translation unit of its own (legendre_bf16_np{1,2,3}_{ana,syn}.hip),
// so that the six compile in parallel.
template <int NP>
hipError_t launch_analysis(const BatchArgs& b, float2* y, float c_rest, hipStream_t st) {
  hipLaunchKernelGGL(analysis_batched<NP>, dim3(static_cast<unsigned>(8 * b.work_per)), dim3(256), 0, st, b.segs,
                     b.work, b.work_per, y, c_rest, b.staged);
  return hipGetLastError();
}

template <int NP>
hipError_t launch_synthesis(const BatchArgs& b, const float2* y, hipStream_t st) {
  hipLaunchKernelGGL(synthesis_batched<NP>, dim3(static_cast<unsigned>(8 * b.work_per)), dim3(256), 0, st, b.segs,
                     b.work, b.work_per, y, b.staged);
  return hipGetLastError();
}

extern template hipError_t launch_analysis<1>(const BatchArgs&, float2*, float, hipStream_t);
extern template hipError_t launch_analysis<2>(const BatchArgs&, float2*, float, hipStream_t);
extern template hipError_t launch_analysis<3>(const BatchArgs&, float2*, float, hipStream_t);
extern template hipError_t launch_synthesis<1>(const BatchArgs&, const float2*, hipStream_t);
extern template hipError_t launch_synthesis<2>(const BatchArgs&, const float2*, hipStream_t);
extern template hipError_t launch_synthesis<3>(const BatchArgs&, const float2*, hipStream_t);

}  // namespace bf16p
}  // namespace sht
