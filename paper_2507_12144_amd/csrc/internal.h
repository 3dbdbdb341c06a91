// Internal declarations shared by the host plan code and the kernel files of
// libsht.so.  Not part of the public ABI (include/sht.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace sht {

// Longest ring DFT supported (LDS budget of the DFT kernels).
constexpr int kMaxNlon = 2048;
// Most northern rings (incl. the equator) the contraction kernels hold.
constexpr int kMaxRings = 384;
constexpr int kMaxRadices = 16;

// Storage of the Legendre table / data operands of the contraction.
enum class Storage : int { F32 = 0, BF16 = 1, BF16X2 = 2, BF16X3 = 3 };

// Geometry of one segment as the kernels see it.
// Padding after every (m, parity) slab of the workspace W (floats).  The
// ring DFTs write and read W at a stride of one slab pair per order m; an
// unpadded slab is a multiple of 16 KiB (kpad * 64 bytes per field group),
// so the 64 orders of a wave would all fall on the same offset modulo
// 16 KiB.  256 bytes of padding spread them.
constexpr long long kWorkPad = 64;

struct SegGeom {
  int nlat, nlon, lmax, mmax;
  int F;          // fields = batch * channels
  int nk;         // northern rings incl. the equator: (nlat + 1) / 2
  int kpad;       // nk rounded up to a ring count the contraction kernels hold
  int groups;     // field groups of 8: ceil(F / 8)
  long long wslab;  // floats of one (m, parity) slab of the workspace W:
                    // groups * kpad * 16 plus kWorkPad
  bool has_equator;  // nlat odd
};

// ---- grid_table.hip ----------------------------------------------------
// Nodes x_k, sin t_k and latitude weights w_k (float64, nlat each).
hipError_t launch_grid(int nlat, int kind, double* x, double* s, double* w, hipStream_t st);
// Legendre table (float64 recurrence, float32 values) in the fragment
// orders of the analysis (ta) and synthesis (tsyn) kernels; off[m] is the
// first float of order m in both tables.
hipError_t launch_frag_table(const SegGeom& g, const double* x, const double* s, const int64_t* off, float* ta,
                             float* tsyn, hipStream_t stream);
// The same table as `planes` bf16 planes (hi, [mid,] lo) in the fragment
// orders of the bf16 kernels; off[m] counts bf16 elements.
hipError_t launch_frag_table_bf16(const SegGeom& g, int planes, const double* x, const double* s,
                                  const int64_t* off, uint16_t* ta, uint16_t* tsyn, hipStream_t stream);

// ---- dft.hip -------------------------------------------------------------
struct DftPlan {
  int n;                       // nlon
  int nstages;
  int radix[kMaxRadices];
};
bool make_dft_plan(int n, DftPlan* p);


// ---- batched launches ----------------------------------------------------
// Per-segment arguments of the batched kernels (an array in device memory;
// one launch per transform stage covers every segment of a plan).
struct SegDev {
  SegGeom g;
  const void* tab_ana;     // Legendre table, analysis fragment order
  const void* tab_syn;     // Legendre table, synthesis fragment order
  const int64_t* tab_off;  // [mmax] first element of order m
  float* work;             // workspace W[m][p][g][k][16] of the segment
  const float* scale_sht;  // (2 pi / nlon) w_k
  const float* scale_one;  // 1
  const float* scale_zonal;  // 2 pi sin(t_k) (2 pi / nlon)^2
  const float2* tw;        // e^{-2 pi i j / nlon}
  long long grid_off;      // first float of the segment in grid buffers
  long long spec_off;      // first complex of the segment in spectral buffers
  int dft_begin;           // first DFT item of the segment (plan-wide numbering)
  int dft_items;           // 2 * groups * nk
  float* ystage;           // staged analysis output Y'[m][p][g][ib][16][16]
  const int64_t* ystage_off;  // [mmax] first float of order m in ystage
  int tr_begin;            // first spectrum-transpose tile (plan-wide numbering)
  int nstages;             // DFT radix plan (generic widths)
  int radix[kMaxRadices];
};
// Plan-wide work of the batched kernels.  Legendre items {m, (segment << 16)
// | column chunk}, 8 XCD slices of per entries padded with {-1, -1}.
struct BatchArgs {
  const SegDev* segs;
  int nseg;
  const int2* work;
  int work_per;
  int dft_total;           // DFT items of all segments
  size_t dft_lds;          // dynamic LDS of the batched DFT kernels
  int ncb;                 // field groups per column chunk (workgroup) of the Legendre kernels
  int staged;              // bit 0: the analysis writes tiles to ystage, then the spectrum transpose
                           // runs; bit 1: the spectrum is staged first and the synthesis reads ystage
  int tr_total;            // spectrum-transpose tiles of all segments
};
// Field groups per column chunk of the bf16 Legendre kernels (the float32
// kernels take BatchArgs::ncb, see legendre_ncb_supported).
constexpr int kBatchNcb = 2;
// Dynamic LDS the DFT kernels need for ring width nlon; prepare_dft_kernels
// raises the batched kernels' dynamic-LDS limit to lds_bytes (call once per
// plan, outside any stream capture).
size_t dft_lds_bytes(int nlon);
hipError_t prepare_dft_kernels(size_t lds_bytes);
// Forward ring DFT of every segment's ring pairs (k, nlat-1-k), k < nk,
// multiplied by the ring scale (sht_scale: (2 pi / nlon) w_k, else 1),
// folded into symmetric/antisymmetric parts and written to the segment's
// workspace W[m][p][g][k][16] (field f = 8g + i at floats 2i, 2i+1).
// Inverse: reads E = W[m][0], O = W[m][1], north = E + O, south = E - O,
// synthesises sum_m c_m Re(Y e^{i m p}) with c_0 = 1, c_m = c_rest, scales
// ring k and writes the grid tensor.  x is the plan-wide grid buffer.
hipError_t launch_dft_forward_batched(const BatchArgs& b, const float* x, bool sht_scale, hipStream_t st);
// Zonal power spectral density (App. F.7, eq. zonal_psd) of every ring of a
// single-segment plan: the forward ring DFT with its epilogue writing
// out[f][k][m] = 2 pi sin(t_k) |(2 pi / nlon) sum_j x[f][k][j] e^{-2 pi i j m / nlon}|^2
// for m < mmax instead of the folded spectrum.
hipError_t launch_zonal_psd(const BatchArgs& b, const float* x, float* out, hipStream_t st);
hipError_t launch_dft_inverse_batched(const BatchArgs& b, float* x, bool sht_scale, float c_rest, hipStream_t st);
// Batched float32 Legendre steps (y is the plan-wide spectral buffer):
// analysis y[f][l][m] = mscale_m sum_k P^_l^m(x_k) W[m][p][g][k][..]
// (p = (l - m) & 1, mscale_0 = 1, mscale_m = c_rest; 0 for l < m);
// synthesis W[m][p][g][k][..] = sum_{l = m + p + 2i < lmax} P^_l^m(x_k) y[f][l][m].
hipError_t launch_legendre_analysis_batched(const BatchArgs& b, float2* y, float c_rest, hipStream_t st);
hipError_t launch_legendre_synthesis_batched(const BatchArgs& b, const float2* y, hipStream_t st);

// ---- legendre.hip --------------------------------------------------------
// Ring padding the contraction kernels support for nk rings (-1: none).
int legendre_ring_pad(int nk);
// Field groups per workgroup the float32 contraction kernels are built for.
bool legendre_ncb_supported(int ncb);
// bf16 forms (legendre_bf16*.hip): the contract of the batched float32
// steps, with the table stored as `planes` bf16 planes.
hipError_t launch_legendre_analysis_bf16_batched(const BatchArgs& b, int planes, float2* y, float c_rest,
                                                 hipStream_t st);
hipError_t launch_legendre_synthesis_bf16_batched(const BatchArgs& b, int planes, const float2* y, hipStream_t st);

// ---- transpose.hip -------------------------------------------------------
// Tiles of the spectrum transpose for one segment, and the transpose of every
// segment's staged analysis output Y' into the spectral buffer y (writes the
// whole spectrum, zeros for l < m included).
int spectrum_transpose_tiles(const SegGeom& g);
hipError_t launch_spectrum_transpose(const BatchArgs& b, float2* y, hipStream_t st);
// The reverse: the live entries of y into the staging tiles, which the
// synthesis reads when BatchArgs::staged has bit 1 set.
hipError_t launch_spectrum_stage(const BatchArgs& b, const float2* y, hipStream_t st);

// ---- scores.hip ----------------------------------------------------------
// Angular PSD (App. F.7, eq. psd): out[f][l] = sum_{m <= min(l, mmax-1)} c_m |y[f][l][m]|^2.
hipError_t launch_psd(const float2* y, long long F, int lmax, int mmax, float* out, hipStream_t st);
// Ensemble CRPS loss terms (App. D.4, App. E.1).  Spectral: rows = lmax,
// cols = mmax, complex elements, weights c_m for 1 <= l <= l_hi, m <= l.
// Spatial: rows = nlat, cols = nlon, real elements, weight ring_w[k].
struct CrpsShape {
  bool spectral;
  int members, channels, rows, cols, l_hi;
};
int crps_max_members();
// The allocation-free form's scratch: a static device array (floats) and its
// address on the current device (looked up once per device).
size_t crps_static_scratch_floats();
hipError_t crps_static_scratch(float** out);
// loss[c] (float, channels entries) and, with grad != nullptr, the gradient
// with respect to every member; partial: channels * rows floats of scratch.
hipError_t launch_crps(const CrpsShape& s, const float* ens, const float* obs, const float* ring_w, bool fair,
                       float* partial, float* loss, float* grad, hipStream_t st);

// ---- noise.hip -----------------------------------------------------------
// One step of the spherical diffusion process (App. B.7, eq.
// spherical_diffusion) on the coefficients y[b][c][l][m] (complex64,
// in place): Philox4x64-10 normals at counter (index, step, 0, 0), key
// (seed, 0); sigma_l[c][l] and phi[c] in float64.  step == 0 draws the
// stationary start.
hipError_t launch_noise_step(int batch, int channels, int lmax, int mmax, const double* sigma_l, const double* phi,
                             unsigned long long seed, unsigned long long step, float2* y, hipStream_t st);

// ---- peak.hip ------------------------------------------------------------
// kind 0: HBM copy of `size` bytes (result bytes/s, read + written);
// kind 1 / 2: FP32 / BF16 matrix-core loop of `size` iterations (flop/s).
hipError_t measure_peak(int kind, size_t size, double* result, hipStream_t st);

// ---- mix.hip -------------------------------------------------------------
// dW[l][c'][c] = sum_{b, m <= min(l, mmax-1)} g[b][c'][l][m] conj(x[b][c][l][m])
hipError_t launch_channel_mix_weight_grad(int batch, int channels, int lmax, int mmax, const float2* g,
                                          const float2* x, float2* dW, hipStream_t stream);
hipError_t launch_channel_mix(int batch, int channels, int lmax, int mmax, const float2* W,
                              const float2* in, float2* out, int adjoint, hipStream_t stream);
// out[b][c][l][m] = k[c][l] in[b][c][l][m] (adjoint: conj(k)), 0 for m > l;
// dk[c][l] = sum_{b, m <= min(l, mmax-1)} g conj(x).
hipError_t launch_isotropic_filter(int batch, int channels, int lmax, int mmax, const float2* k, const float2* in,
                                   float2* out, int adjoint, hipStream_t stream);
hipError_t launch_isotropic_filter_grad(int batch, int channels, int lmax, int mmax, const float2* g,
                                        const float2* x, float2* dk, hipStream_t stream);

}  // namespace sht
