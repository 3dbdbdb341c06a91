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
// Pipelined design.  The Legendre table is stored in MFMA fragment order
// (see the table kernel): a wave's A operands of four consecutive MFMA steps
// are one contiguous 1 KiB piece, 16 bytes a lane.  One workgroup per (m,
// column chunk of NCB field groups) has 2*NCB waves; wave (p, j) owns parity
// p and field group c*NCB + j (one 16-column MFMA block).  The table is
// consumed in stages of a half or a third of a 16-row block for both
// parities that pass through a ring of three LDS buffers, filled by
// asynchronous global->LDS copies (global_load_lds_dwordx4) that the waves
// share out: while the waves multiply stage s, the copies of stages s+1 and
// s+2 are in flight, and no operand passes through VGPRs on its way to LDS.
// The NCB waves of one parity read each piece from LDS.
//  * analysis: the wave keeps its whole K = kpad slice of S or A in VGPRs
//    (read once from HBM); each 16-row block of its parity is one 16 x 16
//    output block, written to the spectrum.
//  * synthesis: the wave keeps its whole kpad x 16 output block in VGPRs;
//    the spectrum values (B operands) are read one row block ahead.
// Occupancy.  At kpad = 384 a wave needs about 160 VGPRs, so a SIMD holds
// three.  Workgroups of four waves (NCB = 2) put one wave on each SIMD, so
// three workgroups share a CU (3 x 48 KiB of LDS); a workgroup of six waves
// would take two wave slots on every SIMD and leave room for no second one.
#pragma once

#include <type_traits>

#include "internal.h"
#include "kernel_common.h"
#include "stage_waits.h"

namespace sht {
namespace fp32k {

typedef float floatx4 __attribute__((ext_vector_type(4)));
// native 4-float vector (HIP's float4 is a struct; its copies do not stay in
// VGPRs)
typedef float v4f __attribute__((ext_vector_type(4)));

// Stage geometry shared by both kernels.  A row block and parity hold T4
// pieces of 1 KiB; a stage takes SC = T4 / PARTS of them for each parity.
// The 2*NCB waves issue LPW copies each per stage (the last piece is
// repeated when 2*SC is not a multiple of the wave count: identical bytes).
template <int NCB, int KS>
struct Stages {
  static constexpr int T4 = KS / 4;
  static constexpr int PARTS = (T4 % 3 == 0) ? 3 : 2;
  static constexpr int SC = T4 / PARTS;
  static constexpr int NW = 2 * NCB;
  static constexpr int LPW = (2 * SC + NW - 1) / NW;
  static constexpr int NTH = 64 * NW;
  // stages unrolled into straight-line code: enough for lmax <= 2 kpad, a
  // multiple of the period after which buffer (stage % 3) and part repeat;
  // larger lmax goes round an outer loop.  Straight-line code lets the
  // compiler prove which buffer each copy writes, so it adds no waits of its
  // own beyond the ones written here.
  static constexpr int PERIOD = PARTS == 3 ? 3 : 6;
  static constexpr int NST = ((PARTS * T4 + PERIOD - 1) / PERIOD) * PERIOD;
  // Analysis: the waves' K slices of S / A come through the same ring
  // first, in XS stages that carry 16 rings of every lane group of every
  // wave (4 pieces of 1 KiB per wave), when a buffer holds them.
  static constexpr bool XSTREAM = (2 * SC >= 4 * NW) && (KS % 16 == 0);
  static constexpr int XS = XSTREAM ? KS / 16 : 0;
  static constexpr int LPWX = 4;
};

// Copy stage st (row block st / PARTS, part st % PARTS) of both parity
// tables into LDS buffer B.  Stages past the last row block re-read the
// last one (into a buffer that is never read).
template <int SC, int NW, int LPW, int PARTS, int T4>
__device__ __forceinline__ void issue_stage(v4f* B, const float* __restrict__ tab, int nb, int st, int wave,
                                            int lane) {
  const int ib = min(st / PARTS, nb - 1), h = st - (st / PARTS) * PARTS;
#pragma unroll
  for (int i = 0; i < LPW; ++i) {
    const int e = min(wave + i * NW, 2 * SC - 1);
    const int pp = e >= SC ? 1 : 0;
    const int t = e - pp * SC;
    const float* src = tab + (static_cast<size_t>(pp * nb + ib) * T4 + h * SC + t) * 256 + lane * 4;
    __builtin_amdgcn_global_load_lds(src, B + (pp * SC + t) * 64, 16, 0, 0);
  }
}

// Analysis.  Contraction index k of a wave's K slice = lk * KS + 4t + q for
// lane group lk, piece t of the row block and component q.
template <int NCB, int KS, bool STG>
__device__ __forceinline__ void analysis_body(const SegDev& sd, int m, int c, const float* __restrict__ W,
                                              float2* __restrict__ y, float c_rest, v4f* b0, v4f* b1,
                                              v4f* b2) {
  using S = Stages<NCB, KS>;
  constexpr int SC = S::SC, NW = S::NW, LPW = S::LPW, NTH = S::NTH, PARTS = S::PARTS, T4 = S::T4;
  constexpr int KPAD = 4 * KS;
  const SegGeom& g = sd.g;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = wave / NCB, j = wave - p * NCB;
  const int cb = c * NCB + j;
  const bool active = cb < g.groups;
  const int li = lane & 15, lk = lane >> 4;
  const int n0 = (g.lmax - m + 1) >> 1;
  const int nb = (n0 + 15) >> 4;
  const int np = p ? (g.lmax - m) >> 1 : n0;
  const int nbp = (np + 15) >> 4;
  const int nst = PARTS * nb;
  const float* tab = static_cast<const float*>(sd.tab_ana) + sd.tab_off[m];
  float xr[KS];
  // this wave's K slice: S or A of its parity and field group (idle waves,
  // past the last field group, read group 0 and never use it)
  const float* Wg = W + static_cast<size_t>(2 * m + p) * g.wslab + static_cast<size_t>(active ? cb : 0) * KPAD * 16;
  if constexpr (!S::XSTREAM) {
#pragma unroll
    for (int s = 0; s < KS; ++s) xr[s] = Wg[(lk * KS + s) * 16 + li];
  }
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
    // Every stage issues the copies of stage s+2, past the end too, so that
    // each wave always has the copies of one stage in flight behind the ones
    // it waits for (waits::analysis_behind: four while S / A streams in, LPW
    // for the table stages).
    constexpr int XS = S::XS;
    if constexpr (S::XSTREAM) {
      // Stage u < XS: every wave copies rings lk * KS + 16u .. +15 of its
      // slice (1 KiB, contiguous in W) for each lane group lk into piece
      // 4 wave + lk of the buffer, then reads its 16 values of xr from there.
      // Table stage s follows as stage XS + s.
      auto issue_x = [&](v4f* B, int u) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          __builtin_amdgcn_global_load_lds(Wg + (q * KS + 16 * u) * 16 + lane * 4, B + (4 * wave + q) * 64, 16, 0, 0);
      };
      issue_x(b0, 0);
      if constexpr (XS > 1)
        issue_x(b1, 1);
      else
        issue_stage<SC, NW, LPW, PARTS, T4>(b1, tab, nb, 0, wave, lane);
      unrolled<0, XS>([&](auto u_c) {
        constexpr int u = decltype(u_c)::value;
        v4f* cur = ring_buf<u>(b0, b1, b2);
        v4f* nxt = ring_buf<u + 2>(b0, b1, b2);
        __builtin_amdgcn_s_waitcnt(vm_lds_wait(waits::analysis_behind(XS, LPW, 2, u)));
        stage_barrier();
        if constexpr (u + 2 < XS)
          issue_x(nxt, u + 2);
        else
          issue_stage<SC, NW, LPW, PARTS, T4>(nxt, tab, nb, u + 2 - XS, wave, lane);
        const float* xb = reinterpret_cast<const float*>(cur) + (4 * wave + lk) * 256 + li;
#pragma unroll
        for (int r = 0; r < 16; ++r) xr[16 * u + r] = xb[16 * r];
        debug_stage_end();
        return true;
      });
    } else {
      issue_stage<SC, NW, LPW, PARTS, T4>(b0, tab, nb, 0, wave, lane);
      issue_stage<SC, NW, LPW, PARTS, T4>(b1, tab, nb, 1, wave, lane);
    }
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int st0 = 0; st0 < nst; st0 += S::NST) {
      unrolled<0, S::NST>([&](auto su_c) {
        constexpr int su = decltype(su_c)::value;
        constexpr int part = su % PARTS;
        const int st = st0 + su;
        if (st >= nst) return false;
        v4f* cur = ring_buf<su + XS>(b0, b1, b2);
        v4f* nxt = ring_buf<su + XS + 2>(b0, b1, b2);
        __builtin_amdgcn_s_waitcnt(vm_lds_wait(waits::analysis_behind(XS, LPW, 2, XS + su)));
        stage_barrier();
        issue_stage<SC, NW, LPW, PARTS, T4>(nxt, tab, nb, st + 2, wave, lane);
        const int ib = st / PARTS;
        if (active && ib < nbp) {
#pragma unroll
          for (int t = 0; t < SC; ++t) {
            const v4f av = cur[(p * SC + t) * 64 + lane];
            constexpr int kb = 4 * part * SC;
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, xr[kb + 4 * t + 0], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, xr[kb + 4 * t + 1], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, xr[kb + 4 * t + 2], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, xr[kb + 4 * t + 3], acc, 0, 0, 0);
          }
          if constexpr (part == PARTS - 1) {
            if constexpr (STG) {
              // the 16 x 16 tile, contiguous, into the order-major staging
              // buffer (rows past the parity's last degree hold zeros)
              gfloat* dst = ystg_out + static_cast<size_t>(ib) * 256;
#pragma unroll
              for (int r = 0; r < 4; ++r) dst[(4 * lk + r) * 16 + li] = acc[r] * ms;
            } else {
              // lane pairs (li, li ^ 1) hold re and im of one field: the
              // even lane stores both (8 bytes)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const float other = __shfl_xor(acc[r], 1, 64);
                const int i = 16 * ib + 4 * lk + r;
                if (fok && (li & 1) == 0 && i < np) {
                  const int l = m + p + 2 * i;
                  *reinterpret_cast<gfloat2*>(yf + ((static_cast<size_t>(f) * g.lmax + l) * g.mmax + m) * 2) =
                      v2f_t{acc[r] * ms, other * ms};
                }
              }
            }
            acc = floatx4{0.f, 0.f, 0.f, 0.f};
          }
        }
        debug_stage_end();
        return true;
      });
    }
    // no copy may still be writing this workgroup's LDS when it ends
    __builtin_amdgcn_s_waitcnt(vm_wait(0));
  }
  // Zeros of the spectrum (entries l < m'): this workgroup writes those of
  // degree l = m for its fields, y[f][m][m+1 .. mmax-1], one contiguous run
  // per field, instead of the scattered column y[f][0 .. m-1][m].  (Staged:
  // the transpose writes them.)
  if (!STG && m < g.lmax) {
    const int fbeg = 8 * NCB * c;
    const int fend = min(g.F, fbeg + 8 * NCB);
    const int run = g.mmax - 1 - m;
    for (int ff = fbeg; ff < fend; ++ff) {
      float2* row = y + (static_cast<size_t>(ff) * g.lmax + m) * g.mmax + m + 1;
      for (int e = threadIdx.x; e < run; e += NTH) row[e] = make_float2(0.f, 0.f);
    }
  }
}

// Synthesis.  Output ring k of a wave's block = li * KR + 4t + q for MFMA row
// li, piece t of a substep and component q; contraction row i = 16 ib + 4 s
// + lk.  Piece e of a row block is substep e / (KR/4), piece e % (KR/4).
template <int NCB, int KS, bool STG>
__device__ __forceinline__ void synthesis_body(const SegDev& sd, int m, int c, const float2* __restrict__ y,
                                               float* __restrict__ W, v4f* b0, v4f* b1, v4f* b2, float* spec) {
  using S = Stages<NCB, KS>;
  constexpr int SC = S::SC, NW = S::NW, LPW = S::LPW, PARTS = S::PARTS, T4 = S::T4;
  constexpr int KPAD = 4 * KS;
  constexpr int KR = KPAD / 16;  // 16-ring output blocks
  constexpr int TS = KR / 4;     // pieces per substep
  static_assert(KR % 4 == 0 && 4 * TS == T4, "stage geometry");
  const SegGeom& g = sd.g;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = wave / NCB, j = wave - p * NCB;
  const int cb = c * NCB + j;
  const bool active = cb < g.groups;
  const int li = lane & 15, lk = lane >> 4;
  const int n0 = (g.lmax - m + 1) >> 1;
  const int nb = (n0 + 15) >> 4;
  const int np = p ? (g.lmax - m) >> 1 : n0;
  const int nbp = (np + 15) >> 4;
  const int nst = PARTS * nb;
  const float* tab = static_cast<const float*>(sd.tab_syn) + sd.tab_off[m];
  // B operand of lane (li, lk) at substep s of row block ib: re (li even) or
  // im (li odd) of field 8 cb + li/2 at degree l = m + p + 2 (16 ib + 4 s + lk).
  // Rows past the parity's last degree read degree m instead: their table
  // rows are zero, so they add nothing (the value is finite whenever the
  // field's own values are).  Lanes of fields past F read field 0; those
  // columns of the workspace are never read back.
  // The four values of a row block arrive by 4-byte global->LDS copies in
  // the wave's 1 KiB of the spectrum slot (value s of lane l at float
  // 64 s + l), refilled at part 1 of every row block for the next one: no
  // load into VGPRs is in flight beside the copies, so the compiler waits
  // only for what a read needs.
  const float* yf = reinterpret_cast<const float*>(y);
  const int f = 8 * cb + (li >> 1);
  const bool fok = active && f < g.F;
  const size_t fbase = (static_cast<size_t>(fok ? f : 0) * g.lmax) * g.mmax;
  float* wspec = spec + wave * 256;
  // Staged input: the same values from the order-major staging tiles
  // (row i of parity p, column li of group cb: 64 contiguous bytes per
  // four lanes' rows), rows past the parity's last degree from row 0 of
  // parity 0 (degree m).
  const int nbs = (((g.lmax - m + 1) >> 1) + 15) >> 4;
  const float* ystg = sd.ystage + sd.ystage_off[m];
  const int cbs = active ? cb : 0;
  auto spec_copy = [&](int ib) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int i = 16 * ib + 4 * s + lk;
      if constexpr (STG) {
        const bool in = i < np;
        const float* src = ystg + ((static_cast<size_t>(in ? p : 0) * g.groups + cbs) * nbs) * 256 +
                           static_cast<size_t>(in ? i : 0) * 16 + li;
        __builtin_amdgcn_global_load_lds(src, wspec + 64 * s, 4, 0, 0);
      } else {
        const int l = i < np ? m + p + 2 * i : m;
        __builtin_amdgcn_global_load_lds(yf + (fbase + static_cast<size_t>(l) * g.mmax + m) * 2 + (li & 1),
                                         wspec + 64 * s, 4, 0, 0);
      }
    }
  };
  floatx4 acc[KR];
#pragma unroll
  for (int rb = 0; rb < KR; ++rb) acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
  if (nb > 0) {
    // Stage u issues the table copies of stage u+2 and, at part 1, the
    // spectrum copies of the next row block (4 per wave), in the order
    // waits::spec_first gives; waits::synthesis_behind counts the copies each
    // stage may leave in flight.  The prologue plays stages -2 and -1 the
    // same way (stage -2 is at part 1 with three parts, stage -1 with two).
    static_assert(PARTS == 2 || PARTS == 3, "spectrum refill at part 1");
    constexpr bool SF = waits::spec_first(PARTS);
    issue_stage<SC, NW, LPW, PARTS, T4>(b0, tab, nb, 0, wave, lane);
    spec_copy(0);
    issue_stage<SC, NW, LPW, PARTS, T4>(b1, tab, nb, 1, wave, lane);
    float bc[4];
    for (int st0 = 0; st0 < nst; st0 += S::NST) {
      unrolled<0, S::NST>([&](auto su_c) {
        constexpr int su = decltype(su_c)::value;
        constexpr int part = su % PARTS;
        const int st = st0 + su;
        if (st >= nst) return false;
        v4f* cur = ring_buf<su>(b0, b1, b2);
        v4f* nxt = ring_buf<su + 2>(b0, b1, b2);
        __builtin_amdgcn_s_waitcnt(vm_lds_wait(waits::synthesis_behind(PARTS, LPW, 2, 4, su)));
        stage_barrier();
        const int ib = st / PARTS;
        if constexpr (part == 0) {
#pragma unroll
          for (int q = 0; q < 4; ++q) bc[q] = wspec[64 * q + lane];
        }
        if constexpr (SF && part == 1) spec_copy(ib + 1);
        issue_stage<SC, NW, LPW, PARTS, T4>(nxt, tab, nb, st + 2, wave, lane);
        if constexpr (!SF && part == 1) spec_copy(ib + 1);
        if (active && ib < nbp) {
#pragma unroll
          for (int tt = 0; tt < SC; ++tt) {
            const int e = part * SC + tt;
            const int s = e / TS, t = e - s * TS;
            const v4f av = cur[(p * SC + tt) * 64 + lane];
            const float bv = bc[s];
            acc[4 * t + 0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv, acc[4 * t + 0], 0, 0, 0);
            acc[4 * t + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv, acc[4 * t + 1], 0, 0, 0);
            acc[4 * t + 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv, acc[4 * t + 2], 0, 0, 0);
            acc[4 * t + 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv, acc[4 * t + 3], 0, 0, 0);
          }
        }
        debug_stage_end();
        return true;
      });
    }
    __builtin_amdgcn_s_waitcnt(vm_wait(0));
  }
  if (!active) return;
  float* Wp = W + static_cast<size_t>(2 * m + p) * g.wslab + static_cast<size_t>(cb) * KPAD * 16;
  // acc[4t + q][r] is output row 4 lk + r, ring k = (4 lk + r) * KR + 4 t + q
#pragma unroll
  for (int t = 0; t < TS; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) Wp[((4 * lk + r) * KR + 4 * t + q) * 16 + li] = acc[4 * t + q][r];
}

// Largest stage buffer of the instantiated geometries (pieces of 64 v4f);
// the stage geometry depends on the ring padding only, not on NCB.
constexpr int kMaxStagePieces = 2 * Stages<2, 96>::SC;
static_assert(2 * Stages<2, 64>::SC <= kMaxStagePieces && 2 * Stages<2, 48>::SC <= kMaxStagePieces,
              "stage buffer size");

// Batched kernels, one instantiation per NCB (field groups per workgroup,
// 2 NCB waves): a workgroup takes its item {m, (segment << 16) | chunk}
// from the plan-wide work list and runs the body specialised for the
// segment's ring padding.  The three LDS buffers are declared here (three
// distinct variables, so that the compiler can tell the copies into one
// from the reads of another) and sized for the largest geometry.
template <int NCB>
__global__ __launch_bounds__(128 * NCB) __attribute__((amdgpu_waves_per_eu(3))) void analysis_batched(
    const SegDev* __restrict__ segs, const int2* __restrict__ work, int per, float2* __restrict__ y, float c_rest,
    int staged) {
  __shared__ v4f b0[kMaxStagePieces * 64], b1[kMaxStagePieces * 64], b2[kMaxStagePieces * 64];
  const int2 wk = take_work(work, per);
  if (wk.x < 0) return;
  const SegDev& sd = segs[wk.y >> 16];
  const int m = wk.x, c = wk.y & 0xffff;
  float2* ys = y + sd.spec_off;
  // the output path is a compile-time choice (as in the synthesis): with a
  // run-time branch the compiler spilled the scaled results around it
  auto body = [&](auto ks_c) {
    constexpr int KS = decltype(ks_c)::value;
    if (staged & 1)
      analysis_body<NCB, KS, true>(sd, m, c, sd.work, ys, c_rest, b0, b1, b2);
    else
      analysis_body<NCB, KS, false>(sd, m, c, sd.work, ys, c_rest, b0, b1, b2);
  };
  switch (sd.g.kpad) {
    case 64: body(std::integral_constant<int, 16>{}); break;
    case 128: body(std::integral_constant<int, 32>{}); break;
    case 192: body(std::integral_constant<int, 48>{}); break;
    case 256: body(std::integral_constant<int, 64>{}); break;
    default: body(std::integral_constant<int, 96>{}); break;
  }
}

template <int NCB>
__global__ __launch_bounds__(128 * NCB) __attribute__((amdgpu_waves_per_eu(3))) void synthesis_batched(
    const SegDev* __restrict__ segs, const int2* __restrict__ work, int per, const float2* __restrict__ y,
    int staged) {
  __shared__ v4f b0[kMaxStagePieces * 64], b1[kMaxStagePieces * 64], b2[kMaxStagePieces * 64];
  __shared__ float spec[2 * NCB * 256];  // spectrum slot: 1 KiB per wave
  const int2 wk = take_work(work, per);
  if (wk.x < 0) return;
  const SegDev& sd = segs[wk.y >> 16];
  const int m = wk.x, c = wk.y & 0xffff;
  const float2* ys = y + sd.spec_off;
  // the input source is a compile-time choice: a run-time branch in the
  // copy loop costs the direct form about a tenth of its time
  auto body = [&](auto ks_c) {
    constexpr int KS = decltype(ks_c)::value;
    if (staged & 2)
      synthesis_body<NCB, KS, true>(sd, m, c, ys, sd.work, b0, b1, b2, spec);
    else
      synthesis_body<NCB, KS, false>(sd, m, c, ys, sd.work, b0, b1, b2, spec);
  };
  switch (sd.g.kpad) {
    case 64: body(std::integral_constant<int, 16>{}); break;
    case 128: body(std::integral_constant<int, 32>{}); break;
    case 192: body(std::integral_constant<int, 48>{}); break;
    case 256: body(std::integral_constant<int, 64>{}); break;
    default: body(std::integral_constant<int, 96>{}); break;
  }
}

// Launch of the NCB instantiation (explicitly instantiated in
// legendre_ncb{2,3,4}.hip, one translation unit each, compiled in parallel).
template <int NCB>
hipError_t launch_ncb(bool analysis, const BatchArgs& b, const float2* in, float2* out, float c_rest,
                      hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(8 * b.work_per)), block(128 * NCB);
  if (analysis)
    hipLaunchKernelGGL(analysis_batched<NCB>, grid, block, 0, st, b.segs, b.work, b.work_per, out, c_rest, b.staged);
  else
    hipLaunchKernelGGL(synthesis_batched<NCB>, grid, block, 0, st, b.segs, b.work, b.work_per, in, b.staged);
  return hipGetLastError();
}

extern template hipError_t launch_ncb<2>(bool, const BatchArgs&, const float2*, float2*, float, hipStream_t);
extern template hipError_t launch_ncb<3>(bool, const BatchArgs&, const float2*, float2*, float, hipStream_t);
extern template hipError_t launch_ncb<4>(bool, const BatchArgs&, const float2*, float2*, float, hipStream_t);

}  // namespace fp32k
}  // namespace sht
