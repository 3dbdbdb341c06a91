// Plan-time float64 kernels: latitude nodes and quadrature weights (App. B.1)
// and the folded table of orthonormal associated Legendre functions
// (App. B.3, eq. spherical_harmonics).  These are the only float64 kernels
// of the library; everything on the transform path is float32 / bf16.
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

template <int PLANES>
__device__ inline void store_bf16_planes(uint16_t* t, size_t idx, size_t plane_stride, double v) {
  double r = v;
#pragma unroll
  for (int p = 0; p < PLANES; ++p) {
    const uint16_t b = bf16_rn_from_double(r);
    t[idx + p * plane_stride] = b;
    r -= bf16_bits_to_double(b);  // exact in float64
  }
}

// One thread per (ring k < nk, order m).  The recurrence in l runs in
// float64 and every value is rounded once to the storage form:
//   P^_m^m     = -sqrt((2m+1)/(2m)) sin t P^_{m-1}^{m-1},  P^_0^0 = 1/sqrt(4 pi)
//   P^_{m+1}^m = sqrt(2m+3) x P^_m^m
//   P^_l^m     = a_lm (x P^_{l-1}^m - b_lm P^_{l-2}^m)
//   a_lm = sqrt((4l^2-1)/(l^2-m^2)), b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1))
// Row of (m, l): row_off[m] + ((l-m)&1) * rows_pad[m] + (l-m)/2.
template <int MODE>  // 0: f32, 1..3: bf16 planes
__global__ void table_kernel(SegGeom g, const double* __restrict__ xs, const double* __restrict__ ss,
                             const int64_t* __restrict__ row_off, const int* __restrict__ rows_pad,
                             void* __restrict__ table, size_t plane_stride) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (k >= g.nk || m >= g.mmax) return;
  const double x = xs[k];
  const double s = ss[k];
  double pmm = 1.0 / sqrt(4.0 * kPi);
  for (int i = 1; i <= m; ++i) pmm = -sqrt((2.0 * i + 1.0) / (2.0 * i)) * s * pmm;
  const int64_t base = row_off[m];
  const int rp = rows_pad[m];
  auto put = [&](int l, double v) {
    const int d = l - m;
    const size_t idx = static_cast<size_t>(base + (d & 1) * rp + (d >> 1)) * g.kpad + k;
    if constexpr (MODE == 0) {
      static_cast<float*>(table)[idx] = __double2float_rn(v);
    } else {
      store_bf16_planes<MODE>(static_cast<uint16_t*>(table), idx, plane_stride, v);
    }
  };
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

hipError_t launch_table(const SegGeom& g, const double* x, const double* s, const int64_t* row_off,
                        const int* rows_pad, Storage st, void* table, size_t plane_stride,
                        hipStream_t stream) {
  const int threads = 64;
  dim3 grid((g.nk + threads - 1) / threads, g.mmax);
  switch (st) {
    case Storage::F32:
      hipLaunchKernelGGL(table_kernel<0>, grid, dim3(threads), 0, stream, g, x, s, row_off, rows_pad,
                         table, plane_stride);
      break;
    case Storage::BF16:
      hipLaunchKernelGGL(table_kernel<1>, grid, dim3(threads), 0, stream, g, x, s, row_off, rows_pad,
                         table, plane_stride);
      break;
    case Storage::BF16X2:
      hipLaunchKernelGGL(table_kernel<2>, grid, dim3(threads), 0, stream, g, x, s, row_off, rows_pad,
                         table, plane_stride);
      break;
    case Storage::BF16X3:
      hipLaunchKernelGGL(table_kernel<3>, grid, dim3(threads), 0, stream, g, x, s, row_off, rows_pad,
                         table, plane_stride);
      break;
  }
  return hipGetLastError();
}

}  // namespace sht
