// Plan-time float64 kernels: latitude nodes and quadrature weights (App. B.1)
// and the table of orthonormal associated Legendre functions by their
// three-term recurrence (App. B.3, eq. spherical_harmonics).  These are the
// only float64 kernels; every operation of the transforms themselves is
// float32 (or bf16 on the matrix cores).
#include "internal.h"
#include "bf16.h"

namespace sht {
namespace {

constexpr double kPi = 3.14159265358979323846;

// Legendre polynomial P_n and P_{n-1} at x by the Bonnet recurrence.
__device__ void legendre_pn(int n, double x, double* pn, double* pn1) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { *pn = 1.0; *pn1 = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;
  *pn1 = p0;
}

// One thread per ring.  Nodes are generated for the northern half and
// mirrored, so x_{nlat-1-k} = -x_k exactly and the equator (odd nlat) has
// x = 0 exactly; the equatorial fold of the contraction relies on this.
__global__ void grid_kernel(int nlat, int kind, double* __restrict__ xo, double* __restrict__ so,
                            double* __restrict__ wo) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nlat) return;
  const int kn = (k < nlat - 1 - k) ? k : nlat - 1 - k;  // northern mirror index
  const bool south = kn != k;
  const bool equator = (2 * kn == nlat - 1);
  double x, s, w;
  if (kind == 1) {
    // Gauss-Legendre: Newton on P_nlat from the asymptotic guess.
    x = cos(kPi * (kn + 0.75) / (nlat + 0.5));
    for (int it = 0; it < 100; ++it) {
      double pn, pn1;
      legendre_pn(nlat, x, &pn, &pn1);
      const double dp = nlat * (pn1 - x * pn) / ((1.0 - x) * (1.0 + x));
      const double dx = pn / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    if (equator) x = 0.0;
    double pn, pn1;
    legendre_pn(nlat, x, &pn, &pn1);
    const double dp = nlat * (pn1 - x * pn) / ((1.0 - x) * (1.0 + x));
    w = 2.0 / ((1.0 - x) * (1.0 + x) * dp * dp);
    s = sqrt((1.0 - x) * (1.0 + x));
  } else {
    // Pole-inclusive equiangular grid: t_k = pi k / (nlat - 1).
    const int N = nlat - 1;
    const double t = static_cast<double>(kn) / N;
    x = equator ? 0.0 : cospi(t);
    s = sinpi(t);
    if (kind == 2) {
      w = (kPi / N) * s;  // sin(t) dt
    } else {
      // Clenshaw-Curtis: w_k = (c_k/N)(1 - sum_j b_j cos(2 j t_k)/(4 j^2 - 1)),
      // the exact integral of the degree-N Chebyshev interpolant.
      double acc = 1.0;
      for (int j = 1; 2 * j <= N; ++j) {
        const double b = (2 * j == N) ? 1.0 : 2.0;
        // cos(2 j t_k) = cospi(2 j kn / N), argument reduced exactly mod 2N
        const long long r = (2LL * j * kn) % (2LL * N);
        acc -= b * cospi(static_cast<double>(r) / N) / (4.0 * j * j - 1.0);
      }
      const double c = (kn == 0) ? 1.0 : 2.0;
      w = c * acc / N;
    }
  }
  xo[k] = south ? -x : x;
  so[k] = s;
  wo[k] = w;
}

// Legendre table in MFMA fragment order.  One thread per (ring k < nk,
// order m) runs the float64 recurrence of eq. spherical_harmonics
//   P^_0^0 = 1/sqrt(4 pi),  P^_m^m = -sqrt((2m+1)/(2m)) sin t P^_{m-1}^{m-1}
//   P^_{m+1}^m = sqrt(2m+3) x P^_m^m
//   P^_l^m = a_lm (x P^_{l-1}^m - b_lm P^_{l-2}^m)
//   a_lm = sqrt((4l^2-1)/(l^2-m^2)),  b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1))
// and rounds every value once to float32.  Degree l of order m has parity
// p = (l-m) & 1 and row i = (l-m) >> 1 of its parity block; rows come in
// blocks of 16 (ib = i / 16).  Each value is written to two tables, laid
// out so that a wave of the contraction kernels reads its MFMA A operands
// of four consecutive steps as one contiguous 1 KiB load (16 bytes a lane):
//  * analysis  (A[i][k], lane = 16 lk + li holds row li, k = lk*KS + 4t + q):
//      off[m] + ((p*nb + ib)*(KS/4) + t)*256 + (16 lk + li)*4 + q
//  * synthesis (A[k][i], lane = 16 lk + li holds i = 4s + lk, k = li*KR + 4t + q):
//      off[m] + (((p*nb + ib)*4 + s)*(KR/4) + t)*256 + (16 lk + li)*4 + q
// with KS = kpad/4, KR = kpad/16 and nb = ceil(ceil((lmax-m)/2) / 16).
// Values too small for float64 flush to zero; none of them can grow back to
// a significant size before l = 768 on the supported grids.
__global__ void frag_table_kernel(SegGeom g, const double* __restrict__ xs, const double* __restrict__ ss,
                                  const int64_t* __restrict__ off, float* __restrict__ ta,
                                  float* __restrict__ tsyn) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (k >= g.nk || m >= g.mmax) return;
  const int KS = g.kpad / 4, KR = g.kpad / 16;
  const int nb = (((g.lmax - m + 1) >> 1) + 15) / 16;
  const size_t base = static_cast<size_t>(off[m]);
  // position of ring k inside the two fragment layouts
  const int a_lk = k / KS, a_rem = k - a_lk * KS, a_t = a_rem >> 2, a_q = a_rem & 3;
  const int s_li = k / KR, s_rem = k - s_li * KR, s_t = s_rem >> 2, s_q = s_rem & 3;
  auto put = [&](int l, double v) {
    const int d = l - m;
    const int p = d & 1, i = d >> 1, ib = i >> 4, li = i & 15;
    const float f = __double2float_rn(v);
    const size_t blk = static_cast<size_t>(p * nb + ib);
    ta[base + (blk * (KS / 4) + a_t) * 256 + (16 * a_lk + li) * 4 + a_q] = f;
    const int s = li >> 2, lk = li & 3;
    tsyn[base + ((blk * 4 + s) * (KR / 4) + s_t) * 256 + (16 * lk + s_li) * 4 + s_q] = f;
  };
  const double x = xs[k];
  const double sn = ss[k];
  double pmm = 1.0 / sqrt(4.0 * kPi);
  for (int i = 1; i <= m; ++i) pmm = -sqrt((2.0 * i + 1.0) / (2.0 * i)) * sn * pmm;
  if (m >= g.lmax) return;
  put(m, pmm);
  if (m + 1 >= g.lmax) return;
  double p2 = pmm;
  double p1 = sqrt(2.0 * m + 3.0) * x * pmm;
  put(m + 1, p1);
  const double mm = static_cast<double>(m) * m;
  for (int l = m + 2; l < g.lmax; ++l) {
    const double dl = l;
    const double a = sqrt((4.0 * dl * dl - 1.0) / (dl * dl - mm));
    const double b = sqrt(((dl - 1.0) * (dl - 1.0) - mm) / (4.0 * (dl - 1.0) * (dl - 1.0) - 1.0));
    const double p = a * (x * p1 - b * p2);
    p2 = p1;
    p1 = p;
    put(l, p);
  }
}

// bf16 planes of the same table for the bf16 matrix-core kernels
// (v_mfma_f32_16x16x32_bf16: a lane holds 8 consecutive K values).  Each
// float64 value v is split into NP bf16 planes, each rounded to nearest-even
// from the float64 residual: hi = bf16(v), next = bf16(v - hi), ...  Rows
// come in 32-row blocks per parity (nb32 = ceil(ceil((lmax-m)/2) / 32)); per
// plane and step a wave reads 64 lanes x 8 values = 1 KiB:
//  * analysis  (16-row sub-blocks, lane 16 lk + li holds row li,
//    k = lk*KPAD/4 + 8t + e):
//      off[m] + ((blk16*T8 + t)*NP + plane)*512 + (16 lk + li)*8 + e
//  * synthesis (lane 16 lk + li holds i = 8 lk + e of the 32-row block,
//    ring k = li*KR + rb):
//      off[m] + ((blk32*KR + rb)*NP + plane)*512 + (16 lk + li)*8 + e
// with T8 = kpad/32 and KR = kpad/16.
template <int NP>
__global__ void frag_table_bf16_kernel(SegGeom g, const double* __restrict__ xs, const double* __restrict__ ss,
                                       const int64_t* __restrict__ off, uint16_t* __restrict__ ta,
                                       uint16_t* __restrict__ tsyn) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (k >= g.nk || m >= g.mmax) return;
  const int Q = g.kpad / 4, T8 = g.kpad / 32, KR = g.kpad / 16;
  const int nb32 = (((g.lmax - m + 1) >> 1) + 31) / 32;
  const size_t base = static_cast<size_t>(off[m]);
  const int a_lk = k / Q, a_rem = k - a_lk * Q, a_t = a_rem >> 3, a_e = a_rem & 7;
  const int s_li = k / KR, s_rb = k - s_li * KR;
  auto put = [&](int l, double v) {
    const int d = l - m;
    const int p = d & 1, i = d >> 1;
    const size_t blk16 = static_cast<size_t>(p * 2 * nb32 + (i >> 4));
    const int li = i & 15;
    const size_t blk32 = static_cast<size_t>(p * nb32 + (i >> 5));
    const int il = i & 31, lk = il >> 3, e = il & 7;
    double r = v;
#pragma unroll
    for (int pl = 0; pl < NP; ++pl) {
      const uint16_t b = bf16_rn_from_double(r);
      r -= bf16_bits_to_double(b);
      ta[base + ((blk16 * T8 + a_t) * NP + pl) * 512 + (16 * a_lk + li) * 8 + a_e] = b;
      tsyn[base + ((blk32 * KR + s_rb) * NP + pl) * 512 + (16 * lk + s_li) * 8 + e] = b;
    }
  };
  const double x = xs[k];
  const double sn = ss[k];
  double pmm = 1.0 / sqrt(4.0 * kPi);
  for (int i = 1; i <= m; ++i) pmm = -sqrt((2.0 * i + 1.0) / (2.0 * i)) * sn * pmm;
  if (m >= g.lmax) return;
  put(m, pmm);
  if (m + 1 >= g.lmax) return;
  double p2 = pmm;
  double p1 = sqrt(2.0 * m + 3.0) * x * pmm;
  put(m + 1, p1);
  const double mm = static_cast<double>(m) * m;
  for (int l = m + 2; l < g.lmax; ++l) {
    const double dl = l;
    const double a = sqrt((4.0 * dl * dl - 1.0) / (dl * dl - mm));
    const double b = sqrt(((dl - 1.0) * (dl - 1.0) - mm) / (4.0 * (dl - 1.0) * (dl - 1.0) - 1.0));
    const double p = a * (x * p1 - b * p2);
    p2 = p1;
    p1 = p;
    put(l, p);
  }
}

}  // namespace

hipError_t launch_grid(int nlat, int kind, double* x, double* s, double* w, hipStream_t st) {
  const int threads = 64;
  hipLaunchKernelGGL(grid_kernel, dim3((nlat + threads - 1) / threads), dim3(threads), 0, st, nlat,
                     kind, x, s, w);
  return hipGetLastError();
}

hipError_t launch_frag_table(const SegGeom& g, const double* x, const double* s, const int64_t* off, float* ta,
                             float* tsyn, hipStream_t stream) {
  hipLaunchKernelGGL(frag_table_kernel, dim3((g.nk + 63) / 64, g.mmax), dim3(64), 0, stream, g, x, s, off, ta, tsyn);
  return hipGetLastError();
}

hipError_t launch_frag_table_bf16(const SegGeom& g, int planes, const double* x, const double* s,
                                  const int64_t* off, uint16_t* ta, uint16_t* tsyn, hipStream_t stream) {
  const dim3 grid((g.nk + 63) / 64, g.mmax);
  switch (planes) {
    case 1: hipLaunchKernelGGL(frag_table_bf16_kernel<1>, grid, dim3(64), 0, stream, g, x, s, off, ta, tsyn); break;
    case 2: hipLaunchKernelGGL(frag_table_bf16_kernel<2>, grid, dim3(64), 0, stream, g, x, s, off, ta, tsyn); break;
    case 3: hipLaunchKernelGGL(frag_table_bf16_kernel<3>, grid, dim3(64), 0, stream, g, x, s, off, ta, tsyn); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sht
