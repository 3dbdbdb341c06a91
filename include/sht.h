/*
 * sht.h -- C ABI of the MI355X (gfx950) real spherical harmonic transform
 * library (libsht.so).
 *
 * The operation is the real SHT pair of App. B.3 of "FourCastNet 3"
 * (arXiv 2507.12144): analysis (eq. sht) as a ring DFT along longitude
 * followed by a quadrature-weighted contraction with orthonormal associated
 * Legendre functions per order m (the decomposition described after
 * eq. spherical_harmonics and written out in Alg. 1), and synthesis
 * (eq. isht) running the same two steps in reverse, plus the exact adjoints
 * of both.  The grids are those of App. B.1.
 *
 * Conventions (all functions):
 *  - lmax and mmax are counts: degrees l < lmax, orders m < mmax (the mode
 *    truncation xf[..., :mmax] and the mmax x lmax x H tensor L of Alg. 1).
 *    1 <= mmax <= lmax and 2*mmax <= nlon (the Nyquist bin is never used).
 *  - Grid tensors (x, gx): float32 [batch][channels][nlat][nlon], C order
 *    (B x C x H x W of Alg. 1).  Rings run from the north pole southwards;
 *    longitude j is at 2*pi*j/nlon.
 *  - Spectral tensors (y, gy): complex64 stored as interleaved float32
 *    (re, im), [batch][channels][lmax][mmax], m fastest
 *    (B x C x lmax x mmax of Alg. 1).  Only m >= 0 is stored.
 *  - sht_forward writes 0 for l < m and an exactly zero imaginary part for
 *    m = 0; isht_forward and sht_backward ignore those entries of their input.
 *  - The DFT carries the longitude quadrature 2*pi/nlon (the "2 pi *
 *    FFT_1D_R2C" step of Alg. 1); the ISHT weights order m >= 1 by 2 (real
 *    fields: u^_l^{-m} = (-1)^m conj(u^_l^m)).
 *  - All tensors are DEVICE pointers owned by the caller.  In/out buffers
 *    must not alias.  With several descriptors (the batching form) each
 *    buffer is the concatenation of the segments in descriptor order, each
 *    segment starting at a multiple of 64 elements; use sht_plan_segment for
 *    the element offsets and sht_plan_sizes for the totals.
 *  - Calls enqueue work on hip_stream (NULL: the plan's own stream) and
 *    return without waiting.  A kernel fault surfaces as SHT_ERR_HIP on a
 *    later call or on the caller's synchronisation.  One stream at a time
 *    per plan: concurrent calls on one plan from different streams race on
 *    the plan's workspace.
 *  - Results are bitwise reproducible for a fixed plan.
 *  - Argument checks run on the host before any HIP call; no C++ exception
 *    crosses this interface.  On failure, sht_last_error() returns a
 *    thread-local description.
 */
#ifndef SHT_MI355X_H
#define SHT_MI355X_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SHT_OK = 0,
    SHT_ERR_INVALID_ARG = 1,   /* null pointer, bad size, unknown enum        */
    SHT_ERR_UNSUPPORTED = 2,   /* valid but not implemented: a prime factor
                                  > 5 in nlon, nlon > 2048, nlat > 768,
                                  batch * channels > 2^20                    */
    SHT_ERR_OUT_OF_MEMORY = 3, /* a device allocation failed                 */
    SHT_ERR_HIP = 4,           /* a HIP runtime call failed                  */
    SHT_ERR_INTERNAL = 5
} sht_status;

/* Latitude grids (App. B.1). */
typedef enum {
    SHT_GRID_EQUIANGULAR = 0,           /* t_k = pi k/(nlat-1), both poles on the
                                           grid; Clenshaw-Curtis weights (footnote
                                           to eq. latlon_quad_weights)             */
    SHT_GRID_GAUSS = 1,                 /* Gauss-Legendre nodes and weights        */
    SHT_GRID_EQUIANGULAR_TRAPEZOID = 2  /* as 0 with sin(t) dt weights
                                           (eq. latlon_quad_weights)               */
} sht_grid;

/* Arithmetic of the Legendre contraction.  The ring DFT is float32 in all
 * forms; the Legendre table is always produced by a float64 recurrence and
 * rounded (to nearest even) to the storage form. */
typedef enum {
    SHT_PREC_FP32 = 0,   /* float32 table and data, float32 MFMA            */
    SHT_PREC_BF16 = 1,   /* bfloat16 table and data, bf16 MFMA, fp32 accum   */
    SHT_PREC_BF16X2 = 2, /* split bf16: the table stored as hi + lo bf16
                            planes (hi = bf16(v), lo = bf16(v - hi)), the
                            data split in registers into three bf16 terms
                            d0 + d1 + d2; products t0 d0 + t0 d1 + t1 d0 +
                            t0 d2 + t1 d1, fp32 accumulate               */
    SHT_PREC_BF16X3 = 3  /* three-term bf16 split of the table and data,
                            the six products of order < 3, fp32 accumulate  */
} sht_precision;

/* One transform shape: batch x channels fields on an nlat x nlon grid. */
typedef struct {
    int nlat, nlon, lmax, mmax;
    sht_grid grid;
    int batch, channels;
} sht_desc;

typedef struct sht_plan_s* sht_plan_t;

/* Create a plan for ndesc >= 1 shapes (ndesc > 1: the batching form, in
 * which every call transforms all segments).  Builds the nodes, weights and
 * the Legendre table on the device in float64 (App. B.1, eq.
 * spherical_harmonics), allocates the workspace, and leaves the plan bound to
 * the current HIP device.  hip_stream: the stream used for plan-time work and
 * as the default stream of later calls (NULL: the null stream).
 * *out is set to NULL on failure; a failed build frees everything it had
 * allocated.  Test hook: with SHT_TEST_FAIL_ALLOC=n in the environment the
 * n-th device allocation of the call fails (SHT_ERR_OUT_OF_MEMORY).
 * Environment: SHT_AUTOTUNE=1 runs sht_plan_tune on the new plan (cache
 * file from SHT_TUNE_CACHE, if set); SHT_DEBUG=1 makes every call
 * synchronise its stream after each kernel it launches (outside stream
 * capture), so a kernel fault is reported as SHT_ERR_HIP by that call. */
sht_status sht_plan(sht_plan_t* out, const sht_desc* descs, int ndesc,
                    sht_precision prec, void* hip_stream);

/* Synchronise the plan's stream and free everything the plan owns.
 * NULL is accepted and ignored.  SHT_ERR_INVALID_ARG (nothing freed) while
 * graphs (sht_graph_create) or noise generators (sht_noise_create) of the
 * plan still exist. */
sht_status sht_plan_destroy(sht_plan_t plan);

/* Element offsets of segment i inside the concatenated grid buffer (float32
 * elements) and spectral buffer (complex elements). */
sht_status sht_plan_segment(sht_plan_t plan, int i, size_t* grid_offset,
                            size_t* spec_offset);

/* Total number of grid (float32) and spectral (complex) elements over all
 * segments: the sizes the caller allocates. */
sht_status sht_plan_sizes(sht_plan_t plan, size_t* grid_elems, size_t* spec_elems);

/* Copy segment i's nodes x_k = cos(t_k) and latitude weights w_k (float64,
 * nlat each, north to south; sum(w) approximates 2) to HOST arrays. */
sht_status sht_plan_grid(sht_plan_t plan, int i, double* x_host, double* w_host);

/* Forward SHT (eq. sht on the grid):
 *   y[l,m] = sum_k sum_j (2 pi/nlon) w_k x[k,j] P^_l^m(x_k) e^{-2 pi i j m/nlon}
 * x: float32 grid tensor (device, read), y: complex64 spectral tensor
 * (device, written in full). */
sht_status sht_forward(sht_plan_t plan, const float* x, void* y, void* hip_stream);

/* Inverse SHT (eq. isht for real fields):
 *   x[k,j] = sum_{m<mmax} c_m Re(e^{2 pi i j m/nlon} sum_{l=m}^{lmax-1} P^_l^m(x_k) y[l,m]),
 *   c_0 = 1, c_m = 2.
 * y: spectral tensor (device, read), x: grid tensor (device, written). */
sht_status isht_forward(sht_plan_t plan, const void* y, float* x, void* hip_stream);

/* Adjoint of sht_forward under the real inner product Re sum conj(a) b
 * (PyTorch's complex-gradient convention):
 *   gx[k,j] = (2 pi/nlon) w_k sum_m Re(e^{2 pi i j m/nlon} sum_l P^_l^m(x_k) gy[l,m])
 * with weight 1 for every m.  gy: spectral (device, read), gx: grid
 * (device, written). */
sht_status sht_backward(sht_plan_t plan, const void* gy, float* gx, void* hip_stream);

/* Adjoint of isht_forward:
 *   gy[l,m] = c_m sum_k P^_l^m(x_k) sum_j gx[k,j] e^{-2 pi i j m/nlon}  (l >= m), 0 for l < m.
 * gx: grid (device, read), gy: spectral (device, written in full). */
sht_status isht_backward(sht_plan_t plan, const float* gx, void* gy, void* hip_stream);

/* Per-degree complex channel mix, a multi-channel form of the spectral
 * convolution of App. B.4 (eq. s2_spectral_conv), for a plan with one
 * segment:  out[b,c',l,m] = sum_c W[l,c',c] in[b,c,l,m]  (adjoint != 0: uses
 * conj(W[l,c,c']) instead, i.e. W_l^H).  W: complex64 [lmax][channels]
 * [channels] (device), in/out: spectral tensors of the plan's shape (device,
 * must not alias).  Entries l < m of out are written as 0. */
sht_status sht_channel_mix(sht_plan_t plan, const void* W, const void* in, void* out,
                           int adjoint, void* hip_stream);

/* Weight gradient of sht_channel_mix (plan with one segment): for a real
 * loss L of y = sht_channel_mix(W, x), given g = dL/dRe y + i dL/dIm y,
 *   dW[l,c',c] = sum_b sum_{m <= min(l, mmax-1)} g[b,c',l,m] conj(x[b,c,l,m]),
 * which is dL/dRe W + i dL/dIm W (the gradient of the spectral-convolution
 * weights, App. B.4 eq. s2_spectral_conv; PyTorch's complex convention).
 * g, x: spectral tensors of the plan's shape (device, read); dW: complex64
 * [lmax][channels][channels] (device, written in full; must alias neither
 * input).  Timed as kind 5 (channel mix). */
sht_status sht_channel_mix_weight_grad(sht_plan_t plan, const void* g, const void* x, void* dW,
                                       void* hip_stream);

/* Angular power spectral density (App. F.7, eq. psd) of a spectrum of a
 * single-segment plan: out[b][c][l] = sum over |m| <= l of |y_l^m|^2 =
 * sum_{m <= min(l, mmax-1)} c_m |y[b][c][l][m]|^2 with c_0 = 1, c_m = 2 (real
 * fields, u^_l^{-m} = (-1)^m conj(u^_l^m)).  y: spectral tensor (device,
 * read); out: float32 [batch][channels][lmax] (device, written).  Timed as
 * kind 6 (scores). */
sht_status sht_psd(sht_plan_t plan, const void* y, float* out, void* hip_stream);

/* Zonal power spectral density (App. F.7, eq. zonal_psd) at every ring of a
 * single-segment plan's grid tensor:
 *   out[b][c][k][m] = 2 pi sin(t_k) |(2 pi/nlon) sum_j x[b][c][k][j] e^{-2 pi i j m/nlon}|^2,
 * m < mmax.  x: grid tensor (device, read); out: float32
 * [batch][channels][nlat][mmax] (device, written; must not alias x).  One
 * launch of the ring DFT with a zonal epilogue.  Timed as kind 6. */
sht_status sht_zonal_psd(sht_plan_t plan, const float* x, float* out, void* hip_stream);

/* Spectral CRPS loss term (App. E.1, eq. spectral_loss) of an ensemble
 * against an observation, single-segment plan whose batch is the ensemble
 * (N = batch members, 1 <= N <= 64; N >= 2 for the fair form):
 *   loss[c] = sum_{1 <= l <= l_hi} sum_{m <= l} c_m (CRPS(Re) + CRPS(Im))
 * with CRPS over the N members in the spread-skill form (App. D.4, eq.
 * spread_skill_crps; fair != 0: eq. fair_spread_skill_crps), c_0 = 1,
 * c_m = 2 (the orders -m of real fields), real and imaginary parts as two
 * real marginals.  l_hi <= 0 selects min(lmax - 1, nlat / 2), the paper's
 * range.  ens: spectral tensor of the plan [N][C][lmax][mmax] (device);
 * obs: complex64 [C][lmax][mmax] (device); loss: float32 [C] (device,
 * written); grad: NULL, or complex64 like ens (device, written in full)
 * receiving d(sum_c loss[c])/dRe + i d/dIm with |.|' = sign(.), sign(0) = 0
 * (PyTorch's complex convention, ready for sht_backward).  Row sums go
 * through plan-owned scratch: calls on one plan must not overlap.  Results
 * are bitwise reproducible (fixed summation order).  Timed as kind 6. */
sht_status sht_spectral_crps(sht_plan_t plan, const void* ens, const void* obs, int fair, int l_hi, float* loss,
                             void* grad, void* hip_stream);

/* Allocation-free form of sht_spectral_crps, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): no plan -- the shape comes from
 * *desc (batch = the N ensemble members) -- and the per-row sums go to a
 * static device array of the library (1 MiB on every GPU the library runs
 * on, held until the process ends) instead of plan-owned scratch.  Limits:
 * channels * lmax <= 262144, 1 <= batch <= 64 (batch >= 2 when fair).
 * Calls no hipMalloc or hipFree.  All calls on one GPU share that array:
 * calls that overlap in time on one GPU race.  Arguments, outputs and
 * errors as for sht_spectral_crps (SHT_ERR_UNSUPPORTED beyond the limits,
 * checked before any HIP call); the outputs equal sht_spectral_crps's. */
sht_status sht_spectral_crps_noalloc(const sht_desc* desc, const void* ens, const void* obs, int fair, int l_hi,
                                     float* loss, void* grad, void* hip_stream);

/* Spatial CRPS loss term (App. E.1, eq. spatial_loss): the point-wise CRPS
 * of the N = batch members averaged over the sphere,
 *   loss[c] = (1/4 pi) sum_k sum_j (2 pi/nlon) w_k CRPS_kj,
 * ens: grid tensor of the plan [N][C][nlat][nlon] (device); obs: float32
 * [C][nlat][nlon] (device); loss, grad as for sht_spectral_crps (grad:
 * float32 like ens).  Timed as kind 6. */
sht_status sht_spatial_crps(sht_plan_t plan, const float* ens, const float* obs, int fair, float* loss, float* grad,
                            void* hip_stream);

/* Spherical diffusion noise (App. B.7, eq. spherical_diffusion): for every
 * member b and channel c of a single-segment plan an AR(1) process of
 * spectral coefficients
 *   a_n = phi_c a_{n-1} + sigma_{c,l} eta,  phi_c = e^{-lambda_c},
 *   sigma_{c,l} = F_0 e^{-k_T,c l (l+1) / 2},
 *   F_0 = sigma_c sqrt(2 pi (1 - phi_c^2) / sum_{0 < l < lmax} (2l+1) e^{-k_T,c l (l+1)}),
 * with eta standard normal per coefficient (Philox4x64-10 counter (flat
 * coefficient index, step, 0, 0), key (seed, 0); 53-bit uniforms, the
 * Box-Muller functions in float32):
 * sigma_l (eta_re + i eta_im) for m >= 1, sqrt(2) sigma_l eta_re for m = 0,
 * degree 0 and l < m zero, so the stationary point-wise variance is
 * sigma_c^2.  sht_noise_create: kT, lambda, sigma are HOST arrays of
 * `channels` doubles (k_T > 0, lambda > 0, sigma >= 0); the generator keeps
 * a step counter starting at 0 and refers to the plan (destroy it first).
 * sht_noise_step: state is the plan's spectral tensor (device, read and
 * written in place; ignored at step 0, which draws the stationary start);
 * with z != NULL the ISHT of the new state is written to z (grid tensor,
 * device).  Advances the counter.  sht_noise_set_step sets the counter
 * (restart from a saved state).  Timed as kind 7 (noise). */
typedef struct sht_noise_s* sht_noise_t;
sht_status sht_noise_create(sht_plan_t plan, const double* kT, const double* lambda, const double* sigma,
                            unsigned long long seed, sht_noise_t* out);
sht_status sht_noise_step(sht_noise_t noise, void* state, float* z, void* hip_stream);
sht_status sht_noise_set_step(sht_noise_t noise, unsigned long long step);
sht_status sht_noise_destroy(sht_noise_t noise);

/* Isotropic spectral filter, the spectral convolution of App. B.4 (eq.
 * s2_spectral_conv: (u * k)^_l^m = u^_l^m k^_l^0) with one filter per
 * channel, for a plan with one segment:
 *   out[b,c,l,m] = k[c,l] in[b,c,l,m]   (adjoint != 0: conj(k[c,l])),
 * entries m > l written as 0.  k: complex64 [channels][lmax] (device);
 * in/out: spectral tensors of the plan's shape (device, must not alias).
 * Timed as kind 5. */
sht_status sht_isotropic_filter(sht_plan_t plan, const void* k, const void* in, void* out, int adjoint,
                                void* hip_stream);

/* Filter gradient of sht_isotropic_filter: for a real loss of
 * y = filter(k, x) with g = dL/dRe y + i dL/dIm y,
 *   dk[c,l] = sum_b sum_{m <= min(l, mmax-1)} g[b,c,l,m] conj(x[b,c,l,m])
 * (PyTorch's complex convention).  g, x: spectral tensors (device, read);
 * dk: complex64 [channels][lmax] (device, written in full).  Fixed
 * summation order.  Timed as kind 5. */
sht_status sht_isotropic_filter_grad(sht_plan_t plan, const void* g, const void* x, void* dk, void* hip_stream);

/* Machine-peak microbenchmarks (diagnostics) for quoting roofline
 * fractions against measured rather than datasheet peaks.  kind 0: HBM, a
 * streaming copy between two library-allocated buffers of `size` bytes
 * (multiple of 16), *result = bytes read + written per second; kind 1:
 * FP32 matrix cores (v_mfma_f32_16x16x4_f32), kind 2: BF16 matrix cores
 * (v_mfma_f32_16x16x32_bf16), `size` iterations of eight independent
 * accumulators in 2048 four-wave workgroups, *result = flop/s.  One timed
 * launch after a warm-up; synchronises hip_stream. */
sht_status sht_measure_peak(int kind, size_t size, double* result, void* hip_stream);

/* Kernel timing (diagnostics).  With enable != 0 every later call on the
 * plan records a pair of HIP events on the call's stream around each kernel
 * it launches.  sht_plan_timing_read waits for the recorded events, adds the
 * elapsed milliseconds and launch counts per kernel kind into ms[i] and
 * counts[i] for i < nkinds (kinds: 0 ring DFT forward, 1 ring DFT inverse,
 * 2 Legendre analysis, 3 Legendre synthesis, 4 zero fill, 5 channel mix,
 * 6 scores and spectra, 7 noise, 8 spectrum transpose of the staged
 * analysis output, 9 staging of the synthesis input), then forgets them.
 * Host arrays; nkinds <= SHT_TIMING_KINDS. */
#define SHT_TIMING_KINDS 10
sht_status sht_plan_timing(sht_plan_t plan, int enable);
sht_status sht_plan_timing_read(sht_plan_t plan, double* ms, long long* counts, int nkinds);

/* Captured sequences (the batching form's replay path).  sht_graph_create
 * records nops transforms of the plan -- ops[i] = SHT_OP_*, reading
 * inputs[i] and writing outputs[i] (device buffers with the layouts of the
 * corresponding entry points, owned by the caller and kept alive and in
 * place while the graph exists) -- into a HIP graph by stream capture on a
 * stream of the library's own, and instantiates it.  Nothing is launched
 * at creation.  sht_graph_launch enqueues one replay of the whole sequence
 * on hip_stream (NULL: the plan's stream) and returns without waiting;
 * replays on one plan must not overlap in time (they share the plan's
 * workspace).  Kernel timing is not recorded inside graphs.  The graph
 * refers to the plan: destroy every graph before its plan.  The captured
 * work allocates nothing and contains no memset nodes.  sht_graph_destroy
 * waits for the graph's last replay (an event recorded by sht_graph_launch),
 * not for other work on the device, then frees the graph.
 * Errors: SHT_ERR_INVALID_ARG (NULL plan/graph/arrays/buffers, nops outside
 * [1, 64], unknown op, an input equal to its output), SHT_ERR_HIP (capture
 * or instantiation failed). */
typedef struct sht_graph_s* sht_graph_t;
typedef enum { SHT_OP_SHT = 0, SHT_OP_ISHT = 1, SHT_OP_SHT_T = 2, SHT_OP_ISHT_T = 3 } sht_op;
sht_status sht_graph_create(sht_plan_t plan, int nops, const sht_op* ops, const void* const* inputs,
                            void* const* outputs, sht_graph_t* out);
sht_status sht_graph_launch(sht_graph_t graph, void* hip_stream);
sht_status sht_graph_destroy(sht_graph_t graph);

/* Autotuner.  The work decomposition of a plan has free parameters that do
 * not change any result bit: whether the analysis output and the synthesis
 * input pass through order-major tiles (see sht_plan_set_schedule), the field
 * groups (of 8 fields) per workgroup of the float32 Legendre kernels (2, 3
 * or 4; the bf16 forms always take 2),
 * the orders per scheduling chunk of the Legendre work list (4, 8, 16, 32)
 * and how chunks are dealt to the 8 XCDs (largest-first to the least-loaded
 * XCD, or round robin).  sht_plan_tune times SHT -> ISHT -> ISHT^T -> SHT^T
 * passes per candidate (the fastest of five, after one warm-up pass) on
 * library-allocated synthetic buffers, requires every candidate's four
 * outputs to equal the default candidate's bit for bit (parity), keeps the
 * fastest (a candidate must beat the one kept by 1 %), and returns
 * its index in *chosen and its time in *best_ms (either may be NULL).  With
 * cache_path != NULL the choice is looked up first in that text file under a
 * key of (gfx arch, descriptors, precision, candidate-list version) and
 * appended to it after a measurement; a cached choice is applied without
 * timing (*best_ms = -1).  Synchronises the plan's stream.  Errors:
 * SHT_ERR_INVALID_ARG (NULL plan, graphs of the plan exist),
 * SHT_ERR_OUT_OF_MEMORY, SHT_ERR_HIP, SHT_ERR_INTERNAL (a candidate's
 * outputs differ from the default's). */
sht_status sht_plan_tune(sht_plan_t plan, const char* cache_path, int* chosen, double* best_ms);

/* Set the schedule explicitly (chunk: orders per chunk, 1..64; policy: 0
 * least-loaded XCD, 1 round robin; ncb: field groups per workgroup of the
 * float32 kernels, 2..4, ignored by the bf16 forms; staged, a bit mask:
 * bit 0 = the analysis writes order-major tiles to plan-owned staging and a
 * transpose kernel writes the spectrum in full lines (else the analysis
 * stores into the spectrum directly), bit 1 = the synthesis input is first
 * copied into those order-major tiles and read from there (else gathered
 * from the spectrum directly)), or read the one in use.  Results do not change.
 * A new plan starts at chunk 8, policy 0, ncb 2 and staged 3, except
 * float32 plans whose segments all have fewer than 256 fields: staged 1.
 * SHT_ERR_INVALID_ARG while graphs of the plan exist (they hold the old work
 * list). */
sht_status sht_plan_set_schedule(sht_plan_t plan, int chunk, int policy, int ncb, int staged);
sht_status sht_plan_get_schedule(sht_plan_t plan, int* chunk, int* policy, int* ncb, int* staged);

const char* sht_status_string(sht_status s);
const char* sht_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SHT_MI355X_H */
