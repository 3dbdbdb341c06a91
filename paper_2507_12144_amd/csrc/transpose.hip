// Spectrum transpose for the staged analysis.
//
// The Legendre analysis produces, for one order m and 8 fields, 16-degree
// tiles of the spectrum.  Written straight into the caller's layout
// y[f][l][m] (m fastest) every tile touches 128 different cache lines with
// 8 bytes each, and the scattered stores cost a quarter (float32) to a
// third (bf16 forms) of the analysis kernel.  In the staged mode the
// analysis writes each tile contiguously to an order-major staging buffer
//   Y'[m][p][g][ib][16 rows][16 floats]   (row i = 16 ib + r: degree
//                                          l = m + p + 2 i; 16 floats: the
//                                          8 fields of group g, re/im)
// and this kernel moves it to y in full lines, writing the zeros of l < m as
// well.  A workgroup takes one (segment, field group, 16 degrees, 32 orders)
// tile: it reads, for each order, the contiguous staging rows of the tile's
// degrees (both parities), transposes them in LDS, and writes 8 fields x
// 16 degrees of 32 consecutive orders (256 contiguous bytes each).
// HBM-bound: the staged spectrum read once (m <= l only) and the whole
// spectrum written once.
#include "internal.h"

namespace sht {
namespace {

constexpr int TL = 16;   // degrees per tile
constexpr int TM = 32;   // orders per tile
constexpr int NTR = 256; // threads

__device__ __forceinline__ int segment_of_tile(const SegDev* __restrict__ segs, int nseg, int t) {
  int s = 0;
  while (s + 1 < nseg && t >= segs[s + 1].tr_begin) ++s;
  return s;
}

// The staging offsets of the tile's orders, read once into LDS (the first
// TM threads; orders past mmax get 0 and are never used).
__device__ __forceinline__ void load_offsets(const SegDev& sd, int m0, long long* off) {
  if (threadIdx.x < TM) {
    const int m = m0 + static_cast<int>(threadIdx.x);
    off[threadIdx.x] = m < sd.g.mmax ? sd.ystage_off[m] : 0;
  }
}

// Staging row of (order m0 + mi, parity par, row `row`) of the tile at
// degree l0: the degree it holds and its float offset (valid when
// m < mmax, l < lmax and l >= m).
struct StageRow {
  int l, mi;
  bool ok;
  long long at;
};
__device__ __forceinline__ StageRow stage_row(const SegGeom& g, const long long* off, int gi, int l0, int m0,
                                              int idx) {
  StageRow r;
  const int q = idx & 3;
  const int row = (idx >> 2) & 7;
  const int par = (idx >> 5) & 1;
  r.mi = idx >> 6;
  const int m = m0 + r.mi;
  // the row-th degree of parity par in [l0, l0 + 16)
  r.l = l0 + ((m + par - l0) & 1) + 2 * row;
  r.ok = m < g.mmax && r.l < g.lmax && r.l >= m;
  const int i = (r.l - m) >> 1;
  const int nbm = (((g.lmax - m + 1) >> 1) + 15) >> 4;
  r.at = off[r.mi] + ((static_cast<long long>(par) * g.groups + gi) * nbm) * 256 + static_cast<long long>(i) * 16 +
         4 * q;
  return r;
}

constexpr int kLoads = TM * 2 * 8 * 4 / NTR;  // float4 staging loads per thread
constexpr int kPairs = 8 * TL * (TM / 2) / NTR;  // spectrum float2 pairs per thread
static_assert(kLoads * NTR == TM * 2 * 8 * 4 && kPairs * NTR == 8 * TL * (TM / 2), "tile geometry");

__global__ __launch_bounds__(NTR) void spectrum_transpose_kernel(const SegDev* __restrict__ segs, int nseg,
                                                                 int total, float2* __restrict__ y) {
  __shared__ float2 T[8][TL][TM + 1];  // [field][degree][order]
  __shared__ long long off[TM];
  const int t = blockIdx.x;
  if (t >= total) return;
  const SegDev& sd = segs[segment_of_tile(segs, nseg, t)];
  const SegGeom& g = sd.g;
  const int lt = (g.lmax + TL - 1) / TL, mt = (g.mmax + TM - 1) / TM;
  int loc = t - sd.tr_begin;
  const int gi = loc / (lt * mt);
  loc -= gi * lt * mt;
  const int l0 = (loc / mt) * TL, m0 = (loc % mt) * TM;
  float2* ys = y + sd.spec_off;
  const int F = g.F;
  if (m0 <= l0 + TL - 1) {
    load_offsets(sd, m0, off);
    __syncthreads();
    // load: (order, parity) pairs of the tile, 8 staging rows each (the
    // degrees l0 .. l0+15 of that parity), 4 float4 per 64-byte row; every
    // load of the thread is issued before the first LDS store
    float4 v[kLoads];
#pragma unroll
    for (int it = 0; it < kLoads; ++it) {
      const StageRow r = stage_row(g, off, gi, l0, m0, static_cast<int>(threadIdx.x) + it * NTR);
      v[it] = r.ok ? *reinterpret_cast<const float4*>(sd.ystage + r.at) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int it = 0; it < kLoads; ++it) {
      const int idx = static_cast<int>(threadIdx.x) + it * NTR;
      const int q = idx & 3, mi = idx >> 6;
      const int li = l0 + (((m0 + mi) + ((idx >> 5) & 1) - l0) & 1) + 2 * ((idx >> 2) & 7) - l0;
      if (li < TL) {
        T[2 * q][li][mi] = make_float2(v[it].x, v[it].y);
        T[2 * q + 1][li][mi] = make_float2(v[it].z, v[it].w);
      }
    }
  } else {
    for (int idx = threadIdx.x; idx < 8 * TL * TM; idx += NTR) (&T[0][0][0])[(idx / TM) * (TM + 1) + idx % TM] =
        make_float2(0.f, 0.f);
  }
  __syncthreads();
  // write: y[f][l][m0 .. m0+31] for the group's 8 fields and 16 degrees
#pragma unroll
  for (int it = 0; it < kPairs; ++it) {
    const int idx = static_cast<int>(threadIdx.x) + it * NTR;
    const int q = idx % (TM / 2);
    const int li = (idx / (TM / 2)) % TL;
    const int fl = idx / (TL * TM / 2);
    const int f = 8 * gi + fl, l = l0 + li, m = m0 + 2 * q;
    if (f >= F || l >= g.lmax || m >= g.mmax) continue;
    float2* dst = ys + (static_cast<size_t>(f) * g.lmax + l) * g.mmax + m;
    const float2 a = T[fl][li][2 * q], b = T[fl][li][2 * q + 1];
    if (m + 1 < g.mmax && ((reinterpret_cast<size_t>(dst) & 15) == 0)) {
      *reinterpret_cast<float4*>(dst) = make_float4(a.x, a.y, b.x, b.y);
    } else {
      dst[0] = a;
      if (m + 1 < g.mmax) dst[1] = b;
    }
  }
}

// The reverse move for the staged synthesis input: y[f][l][m] (live entries
// m <= l) into the order-major tiles Y' that the synthesis then reads as
// contiguous rows instead of gathering 4-byte values from the m-fastest
// spectrum.  Same tiling; tiles with no live entry do nothing; rows of
// degrees past lmax are not written (the synthesis never reads them).
__global__ __launch_bounds__(NTR) void spectrum_stage_kernel(const SegDev* __restrict__ segs, int nseg, int total,
                                                             const float2* __restrict__ y) {
  __shared__ float2 T[8][TL][TM + 1];  // [field][degree][order]
  __shared__ long long off[TM];
  const int t = blockIdx.x;
  if (t >= total) return;
  const SegDev& sd = segs[segment_of_tile(segs, nseg, t)];
  const SegGeom& g = sd.g;
  const int lt = (g.lmax + TL - 1) / TL, mt = (g.mmax + TM - 1) / TM;
  int loc = t - sd.tr_begin;
  const int gi = loc / (lt * mt);
  loc -= gi * lt * mt;
  const int l0 = (loc / mt) * TL, m0 = (loc % mt) * TM;
  if (m0 > l0 + TL - 1) return;  // every order of the tile is above every degree
  const float2* ys = y + sd.spec_off;
  // load y[f][l][m0 .. m0+31] of the group's fields (zeros for fields past F,
  // orders past mmax and degrees past lmax), every load before the first
  // LDS store
  float2 a[kPairs], b[kPairs];
#pragma unroll
  for (int it = 0; it < kPairs; ++it) {
    const int idx = static_cast<int>(threadIdx.x) + it * NTR;
    const int q = idx % (TM / 2);
    const int li = (idx / (TM / 2)) % TL;
    const int fl = idx / (TL * TM / 2);
    const int f = 8 * gi + fl, l = l0 + li, m = m0 + 2 * q;
    a[it] = make_float2(0.f, 0.f);
    b[it] = a[it];
    if (f < g.F && l < g.lmax && m < g.mmax) {
      const float2* src = ys + (static_cast<size_t>(f) * g.lmax + l) * g.mmax + m;
      if (m + 1 < g.mmax && ((reinterpret_cast<size_t>(src) & 15) == 0)) {
        const float4 w = *reinterpret_cast<const float4*>(src);
        a[it] = make_float2(w.x, w.y);
        b[it] = make_float2(w.z, w.w);
      } else {
        a[it] = src[0];
        if (m + 1 < g.mmax) b[it] = src[1];
      }
    }
  }
  load_offsets(sd, m0, off);  // needed by the stores only
#pragma unroll
  for (int it = 0; it < kPairs; ++it) {
    const int idx = static_cast<int>(threadIdx.x) + it * NTR;
    const int q = idx % (TM / 2);
    const int li = (idx / (TM / 2)) % TL;
    const int fl = idx / (TL * TM / 2);
    T[fl][li][2 * q] = a[it];
    T[fl][li][2 * q + 1] = b[it];
  }
  __syncthreads();
  // write the staging rows: (order, parity) pairs, 8 rows of 16 floats each
#pragma unroll
  for (int it = 0; it < kLoads; ++it) {
    const int idx = static_cast<int>(threadIdx.x) + it * NTR;
    const StageRow r = stage_row(g, off, gi, l0, m0, idx);
    if (!r.ok) continue;
    const int q = idx & 3;
    const int li = r.l - l0;
    const float2 u = T[2 * q][li][r.mi], w = T[2 * q + 1][li][r.mi];
    *reinterpret_cast<float4*>(sd.ystage + r.at) = make_float4(u.x, u.y, w.x, w.y);
  }
}

}  // namespace

hipError_t launch_spectrum_stage(const BatchArgs& b, const float2* y, hipStream_t st) {
  hipLaunchKernelGGL(spectrum_stage_kernel, dim3(static_cast<unsigned>(b.tr_total)), dim3(NTR), 0, st, b.segs,
                     b.nseg, b.tr_total, y);
  return hipGetLastError();
}

int spectrum_transpose_tiles(const SegGeom& g) {
  return g.groups * ((g.lmax + TL - 1) / TL) * ((g.mmax + TM - 1) / TM);
}

hipError_t launch_spectrum_transpose(const BatchArgs& b, float2* y, hipStream_t st) {
  hipLaunchKernelGGL(spectrum_transpose_kernel, dim3(static_cast<unsigned>(b.tr_total)), dim3(NTR), 0, st, b.segs,
                     b.nseg, b.tr_total, y);
  return hipGetLastError();
}

}  // namespace sht
