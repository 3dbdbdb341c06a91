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

__global__ __launch_bounds__(NTR) void spectrum_transpose_kernel(const SegDev* __restrict__ segs, int nseg,
                                                                 int total, float2* __restrict__ y) {
  __shared__ float2 T[8][TL][TM + 1];  // [field][degree][order]
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
    // load: (order, parity) pairs of the tile, 8 staging rows each (the
    // degrees l0 .. l0+15 of that parity), 4 float4 per 64-byte row
    for (int idx = threadIdx.x; idx < TM * 2 * 8 * 4; idx += NTR) {
      const int q = idx & 3;
      const int row = (idx >> 2) & 7;
      const int par = (idx >> 5) & 1;
      const int mi = idx >> 6;
      const int m = m0 + mi;
      // degree of this row: the row-th degree of parity par in [l0, l0 + 16)
      const int first = l0 + ((m + par - l0) & 1);
      const int l = first + 2 * row;
      const int li = l - l0;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (m < g.mmax && l < g.lmax && l >= m) {
        const int i = (l - m) >> 1;
        const int nbm = (((g.lmax - m + 1) >> 1) + 15) >> 4;
        const float* src = sd.ystage + sd.ystage_off[m] +
                           ((static_cast<size_t>(par) * g.groups + gi) * nbm) * 256 + static_cast<size_t>(i) * 16 +
                           4 * q;
        v = *reinterpret_cast<const float4*>(src);
      }
      if (li < TL) {
        T[2 * q][li][mi] = make_float2(v.x, v.y);
        T[2 * q + 1][li][mi] = make_float2(v.z, v.w);
      }
    }
  } else {
    for (int idx = threadIdx.x; idx < 8 * TL * TM; idx += NTR) (&T[0][0][0])[(idx / TM) * (TM + 1) + idx % TM] =
        make_float2(0.f, 0.f);
  }
  __syncthreads();
  // write: y[f][l][m0 .. m0+31] for the group's 8 fields and 16 degrees
  for (int idx = threadIdx.x; idx < 8 * TL * (TM / 2); idx += NTR) {
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
  // orders past mmax and degrees past lmax)
  for (int idx = threadIdx.x; idx < 8 * TL * (TM / 2); idx += NTR) {
    const int q = idx % (TM / 2);
    const int li = (idx / (TM / 2)) % TL;
    const int fl = idx / (TL * TM / 2);
    const int f = 8 * gi + fl, l = l0 + li, m = m0 + 2 * q;
    float2 a = make_float2(0.f, 0.f), b = a;
    if (f < g.F && l < g.lmax && m < g.mmax) {
      const float2* src = ys + (static_cast<size_t>(f) * g.lmax + l) * g.mmax + m;
      a = src[0];
      if (m + 1 < g.mmax) b = src[1];
    }
    T[fl][li][2 * q] = a;
    T[fl][li][2 * q + 1] = b;
  }
  __syncthreads();
  // write the staging rows: (order, parity) pairs, 8 rows of 16 floats each
  for (int idx = threadIdx.x; idx < TM * 2 * 8 * 4; idx += NTR) {
    const int q = idx & 3;
    const int row = (idx >> 2) & 7;
    const int par = (idx >> 5) & 1;
    const int mi = idx >> 6;
    const int m = m0 + mi;
    const int first = l0 + ((m + par - l0) & 1);
    const int l = first + 2 * row;
    if (m >= g.mmax || l >= g.lmax || l < m) continue;
    const int li = l - l0;
    const int i = (l - m) >> 1;
    const int nbm = (((g.lmax - m + 1) >> 1) + 15) >> 4;
    float* dst = sd.ystage + sd.ystage_off[m] + ((static_cast<size_t>(par) * g.groups + gi) * nbm) * 256 +
                 static_cast<size_t>(i) * 16 + 4 * q;
    const float2 a = T[2 * q][li][mi], b = T[2 * q + 1][li][mi];
    *reinterpret_cast<float4*>(dst) = make_float4(a.x, a.y, b.x, b.y);
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
