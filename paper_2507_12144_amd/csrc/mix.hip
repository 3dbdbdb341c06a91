// Per-degree complex channel mix: out[b,c',l,m] = sum_c W[l,c',c] in[b,c,l,m]
// (adjoint: conj(W[l,c,c'])), the multi-channel per-degree filter of the
// spectral convolution (App. B.4, eq. s2_spectral_conv: the filter depends on
// l only, never on m).
//
// For each degree l this is a complex GEMM  W_l (C x C) @ X_l (C x B*(l+1)),
// columns (b, m) with m <= min(l, mmax-1).  A workgroup computes a 64 x 64
// output tile through 16-deep LDS-staged slices on the FP32 matrix cores
// (ComplexTile).
#include "internal.h"

namespace sht {
namespace {

constexpr int MT = 64, NT = 64, KT = 16;  // output tile and K slice

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Workgroup -> (degree l, tile) with every tile of a degree on one XCD (the
// hardware deals workgroup b to XCD b % 8), so that the operands of degree l
// are fetched into one L2: degree l goes to XCD l % 8 (the work of a degree
// grows with l, so this balances the XCDs), its T tiles run consecutively
// there.  The grid has 8 * ceil(lmax / 8) * T workgroups.
struct DegreeTile {
  int l, tile;
  __device__ __forceinline__ DegreeTile(int T) {
    const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
    l = xcd + 8 * (slot / T);
    tile = slot % T;
  }
};

// Complex 64 x 64 output tile on the FP32 matrix cores
// (v_mfma_f32_16x16x4_f32): wave w owns the 32 x 32 sub-tile at rows
// 32 (w / 2), columns 32 (w % 2), i.e. 2 x 2 blocks of 16 x 16; per 4-deep
// step of the K slice a block takes four real products,
// re += a_re b_re - a_im b_im and im += a_re b_im + a_im b_re.  Lane
// (li = lane % 16, lk = lane / 16) supplies A[row li][k lk] and B[k lk][col
// li] and receives C[row 4 lk + r][col li], r < 4.
struct ComplexTile {
  floatx4 re[2][2], im[2][2];
  __device__ __forceinline__ void zero() {
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) re[i][j] = im[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  // sA[k][p], sB[k][q]: the current K slice of the two operands
  __device__ __forceinline__ void step(const float2 (*sA)[MT + 1], const float2 (*sB)[NT + 1]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int pr = (wave >> 1) * 32, qc = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int k4 = 0; k4 < KT; k4 += 4) {
      float2 a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = sA[k4 + lk][pr + 16 * t + li];
        b[t] = sB[k4 + lk][qc + 16 * t + li];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].x, b[j].x, re[i][j], 0, 0, 0);
          re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[i].y, b[j].y, re[i][j], 0, 0, 0);
          im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].x, b[j].y, im[i][j], 0, 0, 0);
          im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].y, b[j].x, im[i][j], 0, 0, 0);
        }
    }
  }
  // f(p, q, value) for every output of this lane (p, q within the tile)
  template <class F>
  __device__ __forceinline__ void store(F&& f) const {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int pr = (wave >> 1) * 32, qc = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int r = 0; r < 4; ++r)
          f(pr + 16 * i + 4 * lk + r, qc + 16 * j + li, make_float2(re[i][j][r], im[i][j][r]));
  }
};

__global__ __launch_bounds__(256) void channel_mix_kernel(int B, int C, int lmax, int mmax,
                                                          const float2* __restrict__ W,
                                                          const float2* __restrict__ in,
                                                          float2* __restrict__ out, int adjoint) {
  __shared__ float2 sW[KT][MT + 1];
  __shared__ float2 sX[KT][NT + 1];
  const int tx = (B * mmax + NT - 1) / NT, ty = (C + MT - 1) / MT;
  const DegreeTile dt(tx * ty);
  const int l = dt.l;
  if (l >= lmax) return;
  const int mcount = (l + 1 < mmax) ? l + 1 : mmax;  // orders m <= l
  const int ncols = B * mcount;
  const int c0 = (dt.tile / tx) * MT;   // output channel tile
  const int j0 = (dt.tile % tx) * NT;   // (b, m) column tile
  if (j0 >= ncols) return;
  const int tid = threadIdx.x;
  ComplexTile acc;
  acc.zero();
  const size_t wl = static_cast<size_t>(l) * C * C;
  // The slice k0 .. k0+KT-1 of both operands, PER values a thread, held in
  // registers: the next slice's loads are in flight while the matrix cores
  // work on the current one.
  constexpr int PER = KT * MT / 256;
  static_assert(KT * MT == KT * NT && KT * MT % 256 == 0, "slice split");
  float2 pw[PER], px[PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      // consecutive threads on consecutive addresses: along c for W_l,
      // along c' for W_l^H
      const int kk = adjoint ? e / MT : e % KT, i = adjoint ? e % MT : e / KT;
      const int co = c0 + i, ci = k0 + kk;
      float2 v = make_float2(0.f, 0.f);
      if (co < C && ci < C) {
        if (adjoint) {
          v = W[wl + static_cast<size_t>(ci) * C + co];
          v.y = -v.y;
        } else {
          v = W[wl + static_cast<size_t>(co) * C + ci];
        }
      }
      pw[q] = v;
      const int xk = e / NT, j = e % NT;
      const int col = j0 + j, xi = k0 + xk;
      float2 u = make_float2(0.f, 0.f);
      if (col < ncols && xi < C) {
        const int b = col / mcount, m = col % mcount;
        u = in[((static_cast<size_t>(b) * C + xi) * lmax + l) * mmax + m];
      }
      px[q] = u;
    }
  };
  auto place = [&]() {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      const int kk = adjoint ? e / MT : e % KT, i = adjoint ? e % MT : e / KT;
      sW[kk][i] = pw[q];
      sX[e / NT][e % NT] = px[q];
    }
  };
  load(0);
  for (int k0 = 0; k0 < C; k0 += KT) {
    place();
    __syncthreads();
    if (k0 + KT < C) load(k0 + KT);
    acc.step(sW, sX);
    __syncthreads();
  }
  acc.store([&](int pi, int qi, float2 v) {
    const int co = c0 + pi, col = j0 + qi;
    if (co < C && col < ncols) {
      const int b = col / mcount, m = col % mcount;
      out[((static_cast<size_t>(b) * C + co) * lmax + l) * mmax + m] = v;
    }
  });
}

// out[b, c, l, m] = 0 for m > l (the part the mix kernel never writes).
// Grid: x = spectral row (b, c, l), y = 256-order slice; 32-bit indices.
__global__ __launch_bounds__(256) void mix_zero_kernel(int lmax, int mmax, float2* __restrict__ out) {
  const int row = static_cast<int>(blockIdx.x);
  const int m = static_cast<int>(blockIdx.y) * 256 + static_cast<int>(threadIdx.x);
  const int l = row % lmax;
  if (m > l && m < mmax) out[static_cast<long long>(row) * mmax + m] = make_float2(0.f, 0.f);
}

// Weight gradient of the mix: dW[l, c', c] = sum_{b, m <= l} g[b, c', l, m]
// conj(x[b, c, l, m]), per degree the complex GEMM G_l (C x K) X_l^H (K x C)
// over the K = B * (l + 1) columns (b, m) with m <= min(l, mmax - 1).  A
// workgroup computes a 64 x 64 tile (rows c', columns c) through 16-deep
// LDS-staged slices of K on the matrix cores (ComplexTile).  The
// slices are loaded with consecutive threads on consecutive orders m.
__global__ __launch_bounds__(256) void mix_weight_grad_kernel(int B, int C, int lmax, int mmax,
                                                              const float2* __restrict__ g,
                                                              const float2* __restrict__ x,
                                                              float2* __restrict__ dW) {
  __shared__ float2 sG[KT][MT + 1];
  __shared__ float2 sX[KT][NT + 1];
  const int tq = (C + NT - 1) / NT, tr = (C + MT - 1) / MT;
  const DegreeTile dt(tq * tr);
  const int l = dt.l;
  if (l >= lmax) return;
  const int mcount = (l + 1 < mmax) ? l + 1 : mmax;
  const int K = B * mcount;
  const int r0 = (dt.tile / tq) * MT;  // output rows c'
  const int q0 = (dt.tile % tq) * NT;  // output columns c
  const int tid = threadIdx.x;
  ComplexTile acc;
  acc.zero();
  // slices held in registers, the next one loading during the current
  // one's matrix-core work (as in the mix kernel)
  constexpr int PER = KT * MT / 256;
  float2 pg[PER], px[PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      const int i = e / KT, kk = e % KT;  // consecutive threads: consecutive k
      const int k = k0 + kk;
      const int b = k / mcount, m = k - (k / mcount) * mcount;
      float2 vg = make_float2(0.f, 0.f), vx = vg;
      if (k < K) {
        if (r0 + i < C) vg = g[((static_cast<size_t>(b) * C + r0 + i) * lmax + l) * mmax + m];
        if (q0 + i < C) vx = x[((static_cast<size_t>(b) * C + q0 + i) * lmax + l) * mmax + m];
      }
      pg[q] = vg;
      px[q] = make_float2(vx.x, -vx.y);  // B = X^H
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += KT) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      sG[e % KT][e / KT] = pg[q];
      sX[e % KT][e / KT] = px[q];
    }
    __syncthreads();
    if (k0 + KT < K) load(k0 + KT);
    acc.step(sG, sX);
    __syncthreads();
  }
  const size_t wl = static_cast<size_t>(l) * C * C;
  acc.store([&](int pi, int qi, float2 v) {
    const int co = r0 + pi, ci = q0 + qi;
    if (co < C && ci < C) dW[wl + static_cast<size_t>(co) * C + ci] = v;
  });
}

// Isotropic per-channel filter, the single-channel form of eq.
// s2_spectral_conv: out[b,c,l,m] = k[c,l] in[b,c,l,m] (adjoint: conj(k)),
// 0 for m > l.  Elementwise and HBM-bound: one thread per coefficient,
// consecutive threads on consecutive m.
// Grid: x = spectral row (b, c, l), y = 256-order slice; 32-bit indices.
__global__ __launch_bounds__(256) void isotropic_filter_kernel(int C, int lmax, int mmax,
                                                               const float2* __restrict__ k,
                                                               const float2* __restrict__ in,
                                                               float2* __restrict__ out, int adjoint) {
  const int row = static_cast<int>(blockIdx.x);
  const int m = static_cast<int>(blockIdx.y) * 256 + static_cast<int>(threadIdx.x);
  if (m >= mmax) return;
  const int f = row / lmax;
  const int l = row - f * lmax;
  const int c = f % C;
  const long long i = static_cast<long long>(row) * mmax + m;
  if (m > l) {
    out[i] = make_float2(0.f, 0.f);
    return;
  }
  const float2 kv = k[static_cast<long long>(c) * lmax + l];
  const float ki = adjoint ? -kv.y : kv.y;
  const float2 x = in[i];
  out[i] = make_float2(kv.x * x.x - ki * x.y, kv.x * x.y + ki * x.x);
}

// Filter gradient dk[c,l] = sum_b sum_{m <= min(l, mmax-1)} g conj(x): one
// wave per (c, l); lanes over m, members in order, a fixed-order wave sum.
__global__ __launch_bounds__(256) void isotropic_filter_grad_kernel(int B, int C, int lmax, int mmax,
                                                                    const float2* __restrict__ g,
                                                                    const float2* __restrict__ x,
                                                                    float2* __restrict__ dk) {
  const int lane = threadIdx.x & 63;
  const long long row = static_cast<long long>(blockIdx.x) * 4 + (threadIdx.x >> 6);  // c * lmax + l
  if (row >= static_cast<long long>(C) * lmax) return;
  const int l = static_cast<int>(row % lmax);
  const int mend = min(l + 1, mmax);
  float re = 0.f, im = 0.f;
  for (int b = 0; b < B; ++b) {
    const long long base = (static_cast<long long>(b) * C * lmax + row) * mmax;
    for (int m = lane; m < mend; m += 64) {
      const float2 gv = g[base + m], xv = x[base + m];
      re += gv.x * xv.x + gv.y * xv.y;
      im += gv.y * xv.x - gv.x * xv.y;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (lane == 0) dk[row] = make_float2(re, im);
}

}  // namespace

hipError_t launch_channel_mix_weight_grad(int batch, int channels, int lmax, int mmax, const float2* g,
                                          const float2* x, float2* dW, hipStream_t stream) {
  static_assert(MT == NT, "square tiles: the slice loader shares its index for rows and columns");
  const long long tiles = static_cast<long long>((channels + NT - 1) / NT) * ((channels + MT - 1) / MT);
  const long long blocks = 8LL * ((lmax + 7) / 8) * tiles;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(blocks));
  hipLaunchKernelGGL(mix_weight_grad_kernel, grid, dim3(256), 0, stream, batch, channels, lmax, mmax, g, x, dW);
  return hipGetLastError();
}

hipError_t launch_channel_mix(int batch, int channels, int lmax, int mmax, const float2* W,
                              const float2* in, float2* out, int adjoint, hipStream_t stream) {
  const long long tiles = static_cast<long long>((batch * mmax + NT - 1) / NT) * ((channels + MT - 1) / MT);
  const long long mix_blocks = 8LL * ((lmax + 7) / 8) * tiles;
  if (mix_blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(mix_blocks));
  hipLaunchKernelGGL(channel_mix_kernel, grid, dim3(256), 0, stream, batch, channels, lmax, mmax, W, in,
                     out, adjoint);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long rows = static_cast<long long>(batch) * channels * lmax;
  if (rows > 0x7fffffffLL) return hipErrorInvalidValue;
  if (rows == 0 || mmax <= 0) return hipSuccess;
  const dim3 zgrid(static_cast<unsigned>(rows), static_cast<unsigned>((mmax + 255) / 256));
  hipLaunchKernelGGL(mix_zero_kernel, zgrid, dim3(256), 0, stream, lmax, mmax, out);
  return hipGetLastError();
}

}  // namespace sht

namespace sht {

hipError_t launch_isotropic_filter(int batch, int channels, int lmax, int mmax, const float2* k, const float2* in,
                                   float2* out, int adjoint, hipStream_t stream) {
  const long long rows = static_cast<long long>(batch) * channels * lmax;
  if (rows > 0x7fffffffLL) return hipErrorInvalidValue;
  if (rows == 0 || mmax <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>(rows), static_cast<unsigned>((mmax + 255) / 256));
  hipLaunchKernelGGL(isotropic_filter_kernel, grid, dim3(256), 0, stream, channels, lmax, mmax, k, in, out,
                     adjoint);
  return hipGetLastError();
}

hipError_t launch_isotropic_filter_grad(int batch, int channels, int lmax, int mmax, const float2* g,
                                        const float2* x, float2* dk, hipStream_t stream) {
  const long long rows = static_cast<long long>(channels) * lmax;
  hipLaunchKernelGGL(isotropic_filter_grad_kernel, dim3(static_cast<unsigned>((rows + 3) / 4)), dim3(256), 0, stream,
                     batch, channels, lmax, mmax, g, x, dk);
  return hipGetLastError();
}

}  // namespace sht
