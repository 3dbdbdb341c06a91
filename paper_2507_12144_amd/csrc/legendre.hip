// Legendre contraction kernels: the per-order-m dense contraction of Alg. 1
// (xc_{bclm} = sum_k L_{mlk} x_{bckm}) and its synthesis counterpart
// (eq. isht), on CDNA4 matrix cores.
//
// Folded form.  With nodes symmetric about the equator,
// P^_l^m(-x) = (-1)^(l+m) P^_l^m(x), so for each m the degrees split by
// parity p = (l - m) & 1 and only the northern rings k < nk are needed:
//   analysis : u^[l] = sum_{k<nk} P^_l^m(x_k) (p == 0 ? S_k : A_k)
//   synthesis: E_k = sum_{p=0 rows} P^ u^,  O_k = sum_{p=1 rows} P^ u^,
//              north ring = E + O, mirrored ring = E - O
// which halves both the table and the multiply-adds.  S, A, E, O live in the
// workspace W[m][p][k][col] written / read by the ring DFT kernels; col
// = 2 f + (re, im), so each m is a real GEMM with N = 2F columns.
#include "internal.h"

namespace sht {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64;   // output rows per workgroup
constexpr int TN = 64;   // output columns per workgroup
constexpr int TK = 16;   // contraction step staged in LDS

__device__ __forceinline__ int parity_rows(int lmax, int m, int p) {
  return p == 0 ? (lmax - m + 1) / 2 : (lmax - m) / 2;
}

// 256 threads = 4 waves in a 2 x 2 arrangement; each wave owns a 32 x 32
// sub-tile made of 2 x 2 blocks of v_mfma_f32_16x16x4_f32.
// MFMA operand layout (wave64): A[i][k] from lane i + 16k, B[k][j] from
// lane j + 16k, D[i][j] in lane j + 16 (i / 4), register i % 4.
__global__ __launch_bounds__(256) void analysis_f32_kernel(LegArgs a, const float* __restrict__ W,
                                                           float2* __restrict__ y, float c_rest) {
  __shared__ float sA[TM][TK + 1];
  __shared__ float sB[TK][TN + 4];
  const int4 t = a.tiles[blockIdx.x];
  const int m = t.x, p = t.y, r0 = t.z;
  const int n0 = blockIdx.y * TN;
  const SegGeom& g = a.g;
  const float* A = static_cast<const float*>(a.table) +
                   static_cast<size_t>(a.row_off[m] + static_cast<int64_t>(p) * a.rows_pad[m] + r0) * g.kpad;
  const float* B = W + static_cast<size_t>(2 * m + p) * g.kpad * g.npad + n0;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < g.kpad; k0 += TK) {
    {
      const int r = tid >> 2, c = (tid & 3) * 4;
      const float4 v = *reinterpret_cast<const float4*>(A + static_cast<size_t>(r) * g.kpad + k0 + c);
      sA[r][c] = v.x; sA[r][c + 1] = v.y; sA[r][c + 2] = v.z; sA[r][c + 3] = v.w;
    }
    {
      const int r = tid >> 4, c = (tid & 15) * 4;
      const float4 v = *reinterpret_cast<const float4*>(B + static_cast<size_t>(k0 + r) * g.npad + c);
      sB[r][c] = v.x; sB[r][c + 1] = v.y; sB[r][c + 2] = v.z; sB[r][c + 3] = v.w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      float av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = sA[32 * wr + 16 * i + li][kk + lk];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = sB[kk + lk][32 * wc + 16 * j + li];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  const float ms = (m == 0) ? 1.f : c_rest;
  float* yf = reinterpret_cast<float*>(y);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 32 * wr + 16 * i + 4 * lk + r;
        const int col = 32 * wc + 16 * j + li;
        const int l = m + p + 2 * (r0 + row);
        const int n = n0 + col;
        if (l < g.lmax && n < 2 * g.F) {
          const int f = n >> 1;
          yf[((static_cast<size_t>(f) * g.lmax + l) * g.mmax + m) * 2 + (n & 1)] = acc[i][j][r] * ms;
        }
      }
}

__global__ __launch_bounds__(256) void synthesis_f32_kernel(LegArgs a, const float2* __restrict__ y,
                                                            float* __restrict__ W) {
  __shared__ float sA[TK][TM + 4];  // [i][k]
  __shared__ float sB[TK][TN + 4];  // [i][col]
  const int4 t = a.tiles[blockIdx.x];
  const int m = t.x, p = t.y, k0t = t.z;
  const int n0 = blockIdx.y * TN;
  const SegGeom& g = a.g;
  const int np = parity_rows(g.lmax, m, p);
  const int K = (np + TK - 1) / TK * TK;
  const float* A = static_cast<const float*>(a.table) +
                   static_cast<size_t>(a.row_off[m] + static_cast<int64_t>(p) * a.rows_pad[m]) * g.kpad + k0t;
  const float* yf = reinterpret_cast<const float*>(y);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int i0 = 0; i0 < K; i0 += TK) {
    {
      const int r = tid >> 4, c = (tid & 15) * 4;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (k0t + c < g.kpad) v = *reinterpret_cast<const float4*>(A + static_cast<size_t>(i0 + r) * g.kpad + c);
      sA[r][c] = v.x; sA[r][c + 1] = v.y; sA[r][c + 2] = v.z; sA[r][c + 3] = v.w;
    }
    {
      const int r = tid >> 4, c = (tid & 15) * 4;
      const int i = i0 + r;
      const int l = m + p + 2 * i;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int n = n0 + c + q;
        float v = 0.f;
        if (i < np && n < 2 * g.F) {
          const int f = n >> 1;
          v = yf[((static_cast<size_t>(f) * g.lmax + l) * g.mmax + m) * 2 + (n & 1)];
        }
        sB[r][c + q] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      float av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = sA[kk + lk][32 * wr + 16 * i + li];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = sB[kk + lk][32 * wc + 16 * j + li];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  float* out = W + static_cast<size_t>(2 * m + p) * g.kpad * g.npad;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 32 * wr + 16 * i + 4 * lk + r;
        const int col = 32 * wc + 16 * j + li;
        const int k = k0t + row;
        if (k < g.kpad) out[static_cast<size_t>(k) * g.npad + n0 + col] = acc[i][j][r];
      }
}

__global__ void zero_upper_kernel(int F, int lmax, int mmax, float2* __restrict__ y) {
  const size_t total = static_cast<size_t>(F) * lmax * mmax;
  for (size_t idx = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; idx < total;
       idx += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int m = static_cast<int>(idx % mmax);
    const int l = static_cast<int>((idx / mmax) % lmax);
    if (l < m) y[idx] = make_float2(0.f, 0.f);
  }
}

}  // namespace

hipError_t launch_legendre_analysis(const LegArgs& a, Storage st, const float* W, float2* y,
                                    float c_rest, hipStream_t stream) {
  if (st != Storage::F32) return hipErrorNotSupported;
  dim3 grid(a.ntiles, (2 * a.g.F + TN - 1) / TN);
  hipLaunchKernelGGL(analysis_f32_kernel, grid, dim3(256), 0, stream, a, W, y, c_rest);
  return hipGetLastError();
}

hipError_t launch_legendre_synthesis(const LegArgs& a, Storage st, const float2* y, float* W,
                                     hipStream_t stream) {
  if (st != Storage::F32) return hipErrorNotSupported;
  dim3 grid(a.ntiles, (2 * a.g.F + TN - 1) / TN);
  hipLaunchKernelGGL(synthesis_f32_kernel, grid, dim3(256), 0, stream, a, y, W);
  return hipGetLastError();
}

hipError_t launch_zero_upper(const SegGeom& g, float2* y, hipStream_t stream) {
  const size_t total = static_cast<size_t>(g.F) * g.lmax * g.mmax;
  size_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(zero_upper_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, g.F,
                     g.lmax, g.mmax, y);
  return hipGetLastError();
}

}  // namespace sht
