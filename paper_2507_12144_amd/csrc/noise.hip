// Spherical diffusion noise (App. B.7, eq. spherical_diffusion): one AR(1)
// step per call on the spectral coefficients,
//   a_n = phi a_{n-1} + sigma_l eta,   eta from Philox4x64-10 + Box-Muller,
// followed (on the host side of the library) by the ISHT to the grid.
//
// Random numbers.  Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011), a
// counter-based generator: ten rounds of
//   (x0, x1, x2, x3) -> (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0))
// with the key bumped by the Weyl constants after every round.  Coefficient
// (f, l, m) (flat index i = (f lmax + l) mmax + m) of step n takes counter
// (i, n, 0, 0) and key (seed, 0), so every thread draws its own numbers
// with no state and the stream does not depend on the launch shape.  The
// first two outputs give u = (x >> 11) 2^-53 and the Box-Muller pair
// sqrt(-2 ln(1 - u0)) (cos 2 pi u1, sin 2 pi u1), the functions evaluated in
// float32 (the float64 library functions made the kernel slower than the
// ISHT that follows it).
//
// Coefficients of a real field (m >= 0 stored): sigma_l (eta_re + i eta_im)
// for m >= 1 and sqrt(2) sigma_l eta_re for m = 0, so E|a_l^m|^2 = 2 sigma_l^2
// for every order (isotropy) and, with the paper's F_0, the stationary
// point-wise variance is sigma^2.  Degree 0 and entries l < m stay 0.  Step 0
// draws the stationary start a_0 = draw / sqrt(1 - phi^2).
//
// One thread per coefficient; the update is computed in float64 from the
// float32 state and rounded once.  Bound: the Philox rounds (64-bit
// multiplies) and the Box-Muller functions on the vector ALU, not HBM
// (8 bytes read and written per coefficient).
#include "internal.h"

namespace sht {
namespace {

constexpr unsigned long long kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
constexpr unsigned long long kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;

struct U64x4 {
  unsigned long long v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(unsigned long long c0, unsigned long long c1, unsigned long long c2,
                                               unsigned long long c3, unsigned long long k0, unsigned long long k1) {
  U64x4 x{{c0, c1, c2, c3}};
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const unsigned long long hi0 = __umul64hi(kM0, x.v[0]), lo0 = kM0 * x.v[0];
    const unsigned long long hi1 = __umul64hi(kM1, x.v[2]), lo1 = kM1 * x.v[2];
    x.v[0] = hi1 ^ x.v[1] ^ k0;
    x.v[1] = lo1;
    x.v[2] = hi0 ^ x.v[3] ^ k1;
    x.v[3] = lo0;
    k0 += kW0;
    k1 += kW1;
  }
  return x;
}

// Grid: x = spectral row (f, l) of the batch, y = 256-order slice of the
// row; all index arithmetic in 32 bits (64-bit divisions are emulated and
// cost more than the generator).
__global__ __launch_bounds__(256) void noise_step_kernel(int channels, int lmax, int mmax,
                                                         const double* __restrict__ sigma_l,
                                                         const double* __restrict__ phi, unsigned long long seed,
                                                         unsigned long long step, float2* __restrict__ y) {
  const int row = static_cast<int>(blockIdx.x);
  const int m = static_cast<int>(blockIdx.y) * 256 + static_cast<int>(threadIdx.x);
  if (m >= mmax) return;
  const int f = row / lmax;
  const int l = row - f * lmax;
  const int c = f % channels;
  const long long i = static_cast<long long>(row) * mmax + m;
  if (l < 1 || m > l) {
    y[i] = make_float2(0.f, 0.f);
    return;
  }
  const U64x4 x = philox4x64_10(static_cast<unsigned long long>(i), step, 0ull, 0ull, seed, 0ull);
  // 53-bit uniforms; the Box-Muller functions in float32 (correctly rounded
  // to ~1 ulp: the draws differ from a float64 evaluation by ~1e-7 relative)
  const double u0 = static_cast<double>(x.v[0] >> 11) * 0x1.0p-53;
  const double u1 = static_cast<double>(x.v[1] >> 11) * 0x1.0p-53;
  const float r = sqrtf(-2.f * logf(static_cast<float>(1.0 - u0)));
  float sn, cs;
  sincospif(static_cast<float>(2.0 * u1), &sn, &cs);
  const double er = static_cast<double>(r * cs), ei = static_cast<double>(r * sn);
  const double s = sigma_l[static_cast<long long>(c) * lmax + l];
  const double ph = phi[c];
  double dr, di;
  if (m == 0) {
    dr = (1.4142135623730951 * er) * s;
    di = 0.0;
  } else {
    dr = s * er;
    di = s * ei;
  }
  double nr, ni;
  if (step == 0) {
    const double q = sqrt(1.0 - ph * ph);
    nr = dr / q;
    ni = di / q;
  } else {
    const float2 o = y[i];
    nr = ph * static_cast<double>(o.x) + dr;
    ni = ph * static_cast<double>(o.y) + di;
  }
  y[i] = make_float2(static_cast<float>(nr), static_cast<float>(ni));
}

}  // namespace

hipError_t launch_noise_step(int batch, int channels, int lmax, int mmax, const double* sigma_l, const double* phi,
                             unsigned long long seed, unsigned long long step, float2* y, hipStream_t st) {
  const long long rows = static_cast<long long>(batch) * channels * lmax;
  if (rows > 0x7fffffffLL) return hipErrorInvalidValue;
  if (rows == 0 || mmax <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>(rows), static_cast<unsigned>((mmax + 255) / 256));
  hipLaunchKernelGGL(noise_step_kernel, grid, dim3(256), 0, st, channels, lmax, mmax, sigma_l, phi, seed, step, y);
  return hipGetLastError();
}

}  // namespace sht
