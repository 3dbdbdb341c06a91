// Ensemble scores and spectra of the transform's outputs:
//  * the angular power spectral density of App. F.7 (eq. psd),
//    PSD(l) = sum_{|m| <= l} |u^_l^m|^2 = sum_{m <= l} c_m |u^_l^m|^2 over the
//    stored orders (c_0 = 1, c_m = 2, the real-field symmetry);
//  * the ensemble CRPS of App. D.4 in its spread-skill form
//    (eq. spread_skill_crps, or eq. fair_spread_skill_crps), summed with the
//    weights of the spectral loss term of App. E.1 (eq. spectral_loss:
//    degrees 1 <= l <= l_hi, orders m <= l with multiplicity c_m, real and
//    imaginary parts as two real marginals) or of the spatial loss term
//    (eq. spatial_loss: quadrature weights (2 pi / nlon) w_k / (4 pi)), and
//    its gradient with respect to every member.
//
// All of these are HBM-bound streams over the spectra or grids: one
// workgroup per row (a (channel, degree) row of the spectrum or a
// (channel, ring) row of the grid), threads over the contiguous last index,
// each thread holding the N member values of its element in VGPRs.  Sums are
// taken in a fixed order (per thread, then a fixed tree in LDS, then per
// channel over the rows in order), so results are bitwise reproducible.
#include <mutex>

#include "internal.h"

namespace sht {
namespace {

constexpr int kRowThreads = 256;

// Scratch of the allocation-free CRPS entry point: the per-row sums, in a
// file-scope device array that every GPU the library runs on holds from
// module load to process end.  Host code uses the per-device address from
// hipGetSymbolAddress, never the array's name.
constexpr size_t kStaticScratchFloats = size_t(1) << 18;  // 1 MiB
static __device__ __align__(256) float scratch[kStaticScratchFloats];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
float* g_scratch_ptr[kMaxDevices] = {};

// Fixed-order sum of one value per thread of a 256-thread workgroup.
__device__ __forceinline__ float block_sum(float v, float* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = kRowThreads / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

// One wave per (field, degree) row of the spectrum.
__global__ __launch_bounds__(256) void psd_kernel(const float2* __restrict__ y, long long rows, int lmax, int mmax,
                                                  float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const long long row = static_cast<long long>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const int l = static_cast<int>(row % lmax);
  const int mend = min(l + 1, mmax);
  const float2* r = y + row * mmax;
  float acc = 0.f;
  for (int m = lane; m < mend; m += 64) {
    const float2 v = r[m];
    acc += (m == 0 ? 1.f : 2.f) * (v.x * v.x + v.y * v.y);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) out[row] = acc;
}

// Spread-skill CRPS of one real marginal: v[0..n) members, obs.  With
// g != nullptr also its derivative per member (times `scale`).
template <int NMAX>
__device__ __forceinline__ float crps_one(const float* v, int n, float obs, float inv_n, float inv_pair,
                                          float* g) {
  float skill = 0.f, spread = 0.f;
#pragma unroll
  for (int e = 0; e < NMAX; ++e) {
    if (e < n) {
      skill += fabsf(v[e] - obs);
      float se = 0.f;
#pragma unroll
      for (int i = 0; i < NMAX; ++i)
        if (i < n) se += fabsf(v[e] - v[i]);
      spread += se;
      if (g) {
        float sg = 0.f;
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
          if (i < n) {
            const float d = v[e] - v[i];
            sg += (d > 0.f) ? 1.f : (d < 0.f ? -1.f : 0.f);
          }
        }
        const float d0 = v[e] - obs;
        g[e] = ((d0 > 0.f) ? inv_n : (d0 < 0.f ? -inv_n : 0.f)) - sg * inv_pair;
      }
    }
  }
  // pairs enter as sum_e sum_i |v_e - v_i| / (2 D): D = N^2 or N (N - 1)
  return skill * inv_n - 0.5f * spread * inv_pair;
}

struct CrpsArgs {
  const float* ens;    // [N][C][rows][cols] elements (float2 for spectra)
  const float* obs;    // [C][rows][cols]
  float* grad;         // like ens, or nullptr
  float* partial;      // [C][rows]
  int n, C, rows, cols, parts;
  long long member_stride;  // elements between members
  float inv_n, inv_pair;
  // weights: spectral (parts == 2): c_m for 1 <= l <= l_hi, m <= l;
  // spatial (parts == 1): ring_w[k] for every j
  int l_hi;
  const float* ring_w;
};

__device__ __forceinline__ float element_weight(const CrpsArgs& a, int row, int col) {
  if (a.parts == 2) return (row >= 1 && row <= a.l_hi && col <= row) ? (col == 0 ? 1.f : 2.f) : 0.f;
  return a.ring_w[row];
}

template <int NMAX, bool SPECTRAL>
__global__ __launch_bounds__(kRowThreads) void crps_rows_kernel(CrpsArgs a) {
  __shared__ float red[kRowThreads];
  const int c = blockIdx.y, row = blockIdx.x;
  const long long base = (static_cast<long long>(c) * a.rows + row) * a.cols;  // elements
  float acc = 0.f;
  for (int col = threadIdx.x; col < a.cols; col += kRowThreads) {
    const float w = element_weight(a, row, col);
    const long long el = base + col;
    if (w == 0.f) {
      if (a.grad) {
        if constexpr (SPECTRAL) {
          for (int e = 0; e < a.n; ++e)
            reinterpret_cast<float2*>(a.grad)[el + e * a.member_stride] = make_float2(0.f, 0.f);
        } else {
          for (int e = 0; e < a.n; ++e) a.grad[el + e * a.member_stride] = 0.f;
        }
      }
      continue;
    }
    float g0[NMAX], g1[NMAX];
    if constexpr (SPECTRAL) {
      // real and imaginary parts as two real marginals
      const float2* ens = reinterpret_cast<const float2*>(a.ens);
      float vr[NMAX], vi[NMAX];
#pragma unroll
      for (int e = 0; e < NMAX; ++e) {
        const float2 t = (e < a.n) ? ens[el + e * a.member_stride] : make_float2(0.f, 0.f);
        vr[e] = t.x;
        vi[e] = t.y;
      }
      const float2 o = reinterpret_cast<const float2*>(a.obs)[el];
      acc += w * (crps_one<NMAX>(vr, a.n, o.x, a.inv_n, a.inv_pair, a.grad ? g0 : nullptr) +
                  crps_one<NMAX>(vi, a.n, o.y, a.inv_n, a.inv_pair, a.grad ? g1 : nullptr));
      if (a.grad) {
        float2* gr = reinterpret_cast<float2*>(a.grad);
#pragma unroll
        for (int e = 0; e < NMAX; ++e)
          if (e < a.n) gr[el + e * a.member_stride] = make_float2(w * g0[e], w * g1[e]);
      }
    } else {
      float v[NMAX];
#pragma unroll
      for (int e = 0; e < NMAX; ++e) v[e] = (e < a.n) ? a.ens[el + e * a.member_stride] : 0.f;
      acc += w * crps_one<NMAX>(v, a.n, a.obs[el], a.inv_n, a.inv_pair, a.grad ? g0 : nullptr);
      if (a.grad) {
#pragma unroll
        for (int e = 0; e < NMAX; ++e)
          if (e < a.n) a.grad[el + e * a.member_stride] = w * g0[e];
      }
    }
  }
  const float s = block_sum(acc, red);
  if (threadIdx.x == 0) a.partial[static_cast<long long>(c) * a.rows + row] = s;
}

// loss[c] = sum over rows of partial[c][row], in row order per thread and a
// fixed tree across threads.
__global__ __launch_bounds__(kRowThreads) void crps_finish_kernel(const float* __restrict__ partial, int rows,
                                                                  float* __restrict__ loss) {
  __shared__ float red[kRowThreads];
  const int c = blockIdx.x;
  float acc = 0.f;
  for (int r = threadIdx.x; r < rows; r += kRowThreads) acc += partial[static_cast<long long>(c) * rows + r];
  const float s = block_sum(acc, red);
  if (threadIdx.x == 0) loss[c] = s;
}

}  // namespace

hipError_t launch_psd(const float2* y, long long F, int lmax, int mmax, float* out, hipStream_t st) {
  const long long rows = F * lmax;
  const unsigned blocks = static_cast<unsigned>((rows + 3) / 4);
  hipLaunchKernelGGL(psd_kernel, dim3(blocks), dim3(256), 0, st, y, rows, lmax, mmax, out);
  return hipGetLastError();
}

int crps_max_members() { return 64; }

size_t crps_static_scratch_floats() { return kStaticScratchFloats; }

hipError_t crps_static_scratch(float** out) {
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_crps(const CrpsShape& s, const float* ens, const float* obs, const float* ring_w, bool fair,
                       float* partial, float* loss, float* grad, hipStream_t st) {
  CrpsArgs a;
  a.ens = ens;
  a.obs = obs;
  a.grad = grad;
  a.partial = partial;
  a.n = s.members;
  a.C = s.channels;
  a.rows = s.rows;
  a.cols = s.cols;
  a.parts = s.spectral ? 2 : 1;
  a.member_stride = static_cast<long long>(s.channels) * s.rows * s.cols;
  a.inv_n = 1.f / static_cast<float>(s.members);
  const double pair = fair ? static_cast<double>(s.members) * (s.members - 1) : static_cast<double>(s.members) * s.members;
  a.inv_pair = static_cast<float>(1.0 / pair);
  a.l_hi = s.l_hi;
  a.ring_w = ring_w;
  const dim3 grid(static_cast<unsigned>(s.rows), static_cast<unsigned>(s.channels));
  const dim3 blk(kRowThreads);
  if (s.spectral) {
    if (s.members <= 2) hipLaunchKernelGGL((crps_rows_kernel<2, true>), grid, blk, 0, st, a);
    else if (s.members <= 4) hipLaunchKernelGGL((crps_rows_kernel<4, true>), grid, blk, 0, st, a);
    else if (s.members <= 8) hipLaunchKernelGGL((crps_rows_kernel<8, true>), grid, blk, 0, st, a);
    else if (s.members <= 16) hipLaunchKernelGGL((crps_rows_kernel<16, true>), grid, blk, 0, st, a);
    else if (s.members <= 32) hipLaunchKernelGGL((crps_rows_kernel<32, true>), grid, blk, 0, st, a);
    else hipLaunchKernelGGL((crps_rows_kernel<64, true>), grid, blk, 0, st, a);
  } else {
    if (s.members <= 2) hipLaunchKernelGGL((crps_rows_kernel<2, false>), grid, blk, 0, st, a);
    else if (s.members <= 4) hipLaunchKernelGGL((crps_rows_kernel<4, false>), grid, blk, 0, st, a);
    else if (s.members <= 8) hipLaunchKernelGGL((crps_rows_kernel<8, false>), grid, blk, 0, st, a);
    else if (s.members <= 16) hipLaunchKernelGGL((crps_rows_kernel<16, false>), grid, blk, 0, st, a);
    else if (s.members <= 32) hipLaunchKernelGGL((crps_rows_kernel<32, false>), grid, blk, 0, st, a);
    else hipLaunchKernelGGL((crps_rows_kernel<64, false>), grid, blk, 0, st, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(crps_finish_kernel, dim3(static_cast<unsigned>(s.channels)), dim3(kRowThreads), 0, st, partial,
                     s.rows, loss);
  return hipGetLastError();
}

}  // namespace sht
