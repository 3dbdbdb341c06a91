/* Host-side sanitizer driver for the C ABI (include/sht.h).
 *
 * Built with AddressSanitizer on the host code only (the library's host
 * side in libsht_asan.so and this program; the GPU kernels are the release
 * ones), it walks the ABI and reports any unexpected status:
 *   cpu  -- every argument check that fails before the first HIP call
 *           (no GPU needed);
 *   gpu [cache [repeat]]
 *        -- full plans on the GPU (repeated `repeat` times): every transform, the schedules and
 *           staging modes, the tuner with its cache file, timing, graphs,
 *           the channel mix, filter, spectra, CRPS and noise entry points,
 *           the allocation-free CRPS, and plan builds with the n-th device
 *           allocation failing (SHT_TEST_FAIL_ALLOC), each of which must
 *           return SHT_ERR_OUT_OF_MEMORY and free what it had allocated.
 * AddressSanitizer reports any out-of-bounds access or use after free in
 * the host code; LeakSanitizer, at exit, any host allocation left behind.
 * Exit status 0 when every call returned what it should. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sht.h"

static int failures = 0;

static void expect(sht_status got, sht_status want, const char* what) {
  if (got != want) {
    fprintf(stderr, "FAIL %s: status %d (%s), expected %d: %s\n", what, (int)got, sht_status_string(got), (int)want,
            sht_last_error());
    ++failures;
  }
}

static int cpu_checks(void) {
  sht_plan_t p = NULL;
  sht_desc ok = {33, 64, 17, 17, SHT_GRID_EQUIANGULAR, 1, 3};
  sht_desc bad = ok;
  bad.nlat = 1;
  expect(sht_plan(&p, &bad, 1, SHT_PREC_FP32, NULL), SHT_ERR_INVALID_ARG, "nlat < 2");
  bad = ok;
  bad.lmax = 0;
  expect(sht_plan(&p, &bad, 1, SHT_PREC_FP32, NULL), SHT_ERR_INVALID_ARG, "lmax 0");
  bad = ok;
  bad.mmax = ok.lmax + 1;
  expect(sht_plan(&p, &bad, 1, SHT_PREC_FP32, NULL), SHT_ERR_INVALID_ARG, "mmax > lmax");
  bad = ok;
  bad.channels = 0;
  expect(sht_plan(&p, &bad, 1, SHT_PREC_FP32, NULL), SHT_ERR_INVALID_ARG, "channels 0");
  bad = ok;
  bad.grid = (sht_grid)7;
  expect(sht_plan(&p, &bad, 1, SHT_PREC_FP32, NULL), SHT_ERR_INVALID_ARG, "grid 7");
  expect(sht_plan(&p, &ok, 1, (sht_precision)9, NULL), SHT_ERR_INVALID_ARG, "precision 9");
  expect(sht_plan(NULL, &ok, 1, SHT_PREC_FP32, NULL), SHT_ERR_INVALID_ARG, "out NULL");
  expect(sht_plan(&p, NULL, 1, SHT_PREC_FP32, NULL), SHT_ERR_INVALID_ARG, "descs NULL");
  expect(sht_plan(&p, &ok, 0, SHT_PREC_FP32, NULL), SHT_ERR_INVALID_ARG, "ndesc 0");
  if (p != NULL) {
    fprintf(stderr, "FAIL a failed sht_plan wrote a plan\n");
    ++failures;
  }
  expect(sht_plan_destroy(NULL), SHT_OK, "destroy NULL");
  expect(sht_forward(NULL, NULL, NULL, NULL), SHT_ERR_INVALID_ARG, "sht_forward NULL plan");
  expect(isht_backward(NULL, NULL, NULL, NULL), SHT_ERR_INVALID_ARG, "isht_backward NULL plan");
  expect(sht_plan_tune(NULL, NULL, NULL, NULL), SHT_ERR_INVALID_ARG, "tune NULL plan");
  expect(sht_plan_set_schedule(NULL, 8, 0, 2, 0), SHT_ERR_INVALID_ARG, "set_schedule NULL plan");
  expect(sht_graph_destroy(NULL), SHT_OK, "graph destroy NULL");
  expect(sht_noise_destroy(NULL), SHT_OK, "noise destroy NULL");
  float loss = 0.f;
  expect(sht_spectral_crps_noalloc(NULL, NULL, NULL, 0, 0, &loss, NULL, NULL), SHT_ERR_INVALID_ARG,
         "noalloc NULL desc");
  for (int s = 0; s <= 5; ++s)
    if (sht_status_string((sht_status)s) == NULL || strlen(sht_status_string((sht_status)s)) == 0) {
      fprintf(stderr, "FAIL status string %d\n", s);
      ++failures;
    }
  double r = 0.0;
  expect(sht_measure_peak(7, 1, &r, NULL), SHT_ERR_INVALID_ARG, "measure_peak kind 7");
  expect(sht_measure_peak(0, 15, &r, NULL), SHT_ERR_INVALID_ARG, "measure_peak size");
  sht_desc many = ok;
  many.nlon = 7 * 64;
  expect(sht_plan(&p, &many, 1, SHT_PREC_FP32, NULL), SHT_ERR_UNSUPPORTED, "nlon with a prime factor 7");
  /* an error message longer than any buffer a caller would guess */
  sht_desc two[2] = {ok, ok};
  two[1].mmax = 40;
  expect(sht_plan(&p, two, 2, SHT_PREC_FP32, NULL), SHT_ERR_INVALID_ARG, "second desc mmax > lmax");
  if (strstr(sht_last_error(), "desc 1") == NULL) {
    fprintf(stderr, "FAIL last error does not name desc 1: %s\n", sht_last_error());
    ++failures;
  }
  return failures;
}

/* ---------------------------------------------------------------- GPU */

static void* dev_buf(size_t bytes, unsigned seed) {
  void* d = NULL;
  if (hipMalloc(&d, bytes) != hipSuccess) {
    fprintf(stderr, "FAIL hipMalloc %zu\n", bytes);
    exit(2);
  }
  size_t n = bytes / sizeof(float);
  float* h = (float*)malloc(n * sizeof(float));
  unsigned x = seed * 2654435761u + 1u;
  for (size_t i = 0; i < n; ++i) {
    x = x * 1664525u + 1013904223u;
    h[i] = (float)((x >> 8) & 0xffff) / 65536.0f - 0.5f;
  }
  (void)hipMemcpy(d, h, n * sizeof(float), hipMemcpyHostToDevice);
  free(h);
  return d;
}

static void transforms(sht_plan_t p, const char* tag) {
  size_t ge = 0, se = 0;
  expect(sht_plan_sizes(p, &ge, &se), SHT_OK, "sizes");
  float* x = (float*)dev_buf(ge * 4, 1);
  void* y = dev_buf(se * 8, 2);
  float* gx = (float*)dev_buf(ge * 4, 3);
  void* gy = dev_buf(se * 8, 4);
  char what[128];
  snprintf(what, sizeof what, "%s transforms", tag);
  expect(sht_forward(p, x, y, NULL), SHT_OK, what);
  expect(isht_forward(p, y, gx, NULL), SHT_OK, what);
  expect(isht_backward(p, gx, gy, NULL), SHT_OK, what);
  expect(sht_backward(p, gy, x, NULL), SHT_OK, what);
  for (int staged = 0; staged < 4; ++staged)
    for (int ncb = 2; ncb <= 4; ++ncb) {
      expect(sht_plan_set_schedule(p, 8, staged & 1, ncb, staged), SHT_OK, "set_schedule");
      expect(sht_forward(p, x, y, NULL), SHT_OK, "sht under schedule");
      expect(isht_forward(p, y, gx, NULL), SHT_OK, "isht under schedule");
    }
  int c = 0, pol = 0, n = 0, st = 0;
  expect(sht_plan_get_schedule(p, &c, &pol, &n, &st), SHT_OK, "get_schedule");
  expect(sht_plan_set_schedule(p, 0, 0, 2, 0), SHT_ERR_INVALID_ARG, "chunk 0");
  expect(sht_plan_set_schedule(p, 8, 0, 2, 4), SHT_ERR_INVALID_ARG, "staged 4");
  expect(sht_forward(p, NULL, y, NULL), SHT_ERR_INVALID_ARG, "sht NULL input");
  expect(sht_plan_timing(p, 1), SHT_OK, "timing on");
  expect(sht_forward(p, x, y, NULL), SHT_OK, "timed sht");
  double ms[SHT_TIMING_KINDS];
  long long cnt[SHT_TIMING_KINDS];
  expect(sht_plan_timing_read(p, ms, cnt, SHT_TIMING_KINDS), SHT_OK, "timing read");
  expect(sht_plan_timing_read(p, ms, cnt, SHT_TIMING_KINDS + 1), SHT_ERR_INVALID_ARG, "timing read nkinds");
  expect(sht_plan_timing(p, 0), SHT_OK, "timing off");
  /* graph of the fwd+bwd chain; the plan cannot go while it exists */
  sht_op ops[4] = {SHT_OP_SHT, SHT_OP_ISHT, SHT_OP_ISHT_T, SHT_OP_SHT_T};
  const void* ins[4] = {x, y, gx, gy};
  void* outs[4] = {y, gx, gy, x};
  sht_graph_t g = NULL;
  expect(sht_graph_create(p, 4, ops, ins, outs, &g), SHT_OK, "graph create");
  expect(sht_graph_launch(g, NULL), SHT_OK, "graph launch");
  expect(sht_graph_launch(g, NULL), SHT_OK, "graph launch again");
  expect(sht_plan_set_schedule(p, 8, 0, 2, 0), SHT_ERR_INVALID_ARG, "set_schedule with a graph");
  expect(sht_graph_destroy(g), SHT_OK, "graph destroy");
  (void)hipDeviceSynchronize();
  hipFree(x);
  hipFree(y);
  hipFree(gx);
  hipFree(gy);
}

static int gpu_checks(const char* cache) {
  /* single-segment float32 and multi-segment split-bf16 plans */
  sht_plan_t a = NULL, b = NULL;
  sht_desc da = {33, 64, 17, 17, SHT_GRID_EQUIANGULAR, 1, 3};
  sht_desc db[2] = {{65, 128, 64, 41, SHT_GRID_EQUIANGULAR, 2, 3}, {90, 180, 90, 90, SHT_GRID_GAUSS, 1, 20}};
  expect(sht_plan(&a, &da, 1, SHT_PREC_FP32, NULL), SHT_OK, "plan fp32");
  expect(sht_plan(&b, db, 2, SHT_PREC_BF16X2, NULL), SHT_OK, "plan bf16x2");
  if (failures) return failures;
  size_t go = 0, so = 0;
  expect(sht_plan_segment(b, 1, &go, &so), SHT_OK, "segment 1");
  expect(sht_plan_segment(b, 2, &go, &so), SHT_ERR_INVALID_ARG, "segment 2");
  double xk[90], wk[90];
  expect(sht_plan_grid(b, 1, xk, wk), SHT_OK, "grid");
  transforms(a, "fp32");
  transforms(b, "bf16x2");
  int chosen = -1;
  double best = 0.0;
  expect(sht_plan_tune(a, cache, &chosen, &best), SHT_OK, "tune");
  expect(sht_plan_tune(a, cache, &chosen, &best), SHT_OK, "tune cached");
  expect(sht_plan_destroy(a), SHT_OK, "destroy fp32");
  expect(sht_plan_destroy(b), SHT_OK, "destroy bf16x2");

  /* the block and score entry points on one Gauss plan */
  const int B = 2, C = 8, L = 40;
  sht_desc dc = {42, 80, L, L, SHT_GRID_GAUSS, B, C};
  sht_plan_t p = NULL;
  expect(sht_plan(&p, &dc, 1, SHT_PREC_FP32, NULL), SHT_OK, "plan block");
  if (failures) return failures;
  size_t ge = 0, se = 0;
  expect(sht_plan_sizes(p, &ge, &se), SHT_OK, "sizes");
  void* W = dev_buf((size_t)L * C * C * 8, 5);
  void* y = dev_buf(se * 8, 6);
  void* y2 = dev_buf(se * 8, 7);
  void* dW = dev_buf((size_t)L * C * C * 8, 8);
  void* k = dev_buf((size_t)C * L * 8, 9);
  void* dk = dev_buf((size_t)C * L * 8, 10);
  float* x = (float*)dev_buf(ge * 4, 11);
  float* outf = (float*)dev_buf((size_t)B * C * 42 * L * 4 + ge * 4, 12);
  float* gxf = (float*)dev_buf(ge * 4, 14);
  void* g2 = dev_buf(se * 8, 15);
  float* loss = (float*)dev_buf(C * 4, 13);
  expect(sht_channel_mix(p, W, y, y2, 0, NULL), SHT_OK, "mix");
  expect(sht_channel_mix(p, W, y, y2, 1, NULL), SHT_OK, "mix adjoint");
  expect(sht_channel_mix_weight_grad(p, y, y2, dW, NULL), SHT_OK, "mix dW");
  expect(sht_isotropic_filter(p, k, y, y2, 0, NULL), SHT_OK, "filter");
  expect(sht_isotropic_filter_grad(p, y, y2, dk, NULL), SHT_OK, "filter grad");
  expect(sht_psd(p, y, outf, NULL), SHT_OK, "psd");
  expect(sht_zonal_psd(p, x, outf, NULL), SHT_OK, "zonal psd");
  /* the ensemble is the plan's batch; the observation one member's worth */
  expect(sht_spectral_crps(p, y, y2, 0, 0, loss, NULL, NULL), SHT_OK, "spectral crps");
  expect(sht_spectral_crps(p, y, y2, 1, 10, loss, g2, NULL), SHT_OK, "spectral crps grad");
  expect(sht_spectral_crps(p, y, y2, 0, 0, loss, y2, NULL), SHT_ERR_INVALID_ARG, "crps grad aliasing obs");
  expect(sht_spatial_crps(p, x, outf, 1, loss, gxf, NULL), SHT_OK, "spatial crps");
  expect(sht_spectral_crps_noalloc(&dc, y, y2, 0, 0, loss, NULL, NULL), SHT_OK, "noalloc crps");
  sht_desc huge = dc;
  huge.channels = 1 << 16;
  expect(sht_spectral_crps_noalloc(&huge, y, y2, 0, 0, loss, NULL, NULL), SHT_ERR_UNSUPPORTED, "noalloc oversized");
  double kT[8], lam[8], sig[8];
  for (int i = 0; i < C; ++i) {
    kT[i] = 1e-4 * (i + 1);
    lam[i] = 1.0;
    sig[i] = 0.5 + 0.1 * i;
  }
  sht_noise_t nz = NULL;
  expect(sht_noise_create(p, kT, lam, sig, 7, &nz), SHT_OK, "noise create");
  expect(sht_noise_step(nz, y, x, NULL), SHT_OK, "noise step 0");
  expect(sht_noise_step(nz, y, x, NULL), SHT_OK, "noise step 1");
  expect(sht_noise_set_step(nz, 0), SHT_OK, "noise set step");
  expect(sht_noise_destroy(nz), SHT_OK, "noise destroy");
  (void)hipDeviceSynchronize();
  expect(sht_plan_destroy(p), SHT_OK, "destroy block plan");
  hipFree(W);
  hipFree(y);
  hipFree(y2);
  hipFree(dW);
  hipFree(k);
  hipFree(dk);
  hipFree(x);
  hipFree(outf);
  hipFree(gxf);
  hipFree(g2);
  hipFree(loss);

  /* every device allocation of a plan build failing in turn */
  int built = 0;
  for (int n = 1; n <= 200 && !built; ++n) {
    char v[16];
    snprintf(v, sizeof v, "%d", n);
    setenv("SHT_TEST_FAIL_ALLOC", v, 1);
    sht_plan_t q = NULL;
    sht_status s = sht_plan(&q, db, 2, SHT_PREC_BF16X2, NULL);
    unsetenv("SHT_TEST_FAIL_ALLOC");
    if (s == SHT_OK) {
      built = 1;
      expect(sht_plan_destroy(q), SHT_OK, "destroy after fail-alloc loop");
    } else {
      expect(s, SHT_ERR_OUT_OF_MEMORY, "failing allocation");
      if (q != NULL) {
        fprintf(stderr, "FAIL a failed plan build wrote a plan\n");
        ++failures;
      }
    }
  }
  if (!built) {
    fprintf(stderr, "FAIL the plan never built in the fail-alloc loop\n");
    ++failures;
  }
  return failures;
}

int main(int argc, char** argv) {
  const int gpu = argc > 1 && strcmp(argv[1], "gpu") == 0;
  const int repeat = argc > 3 ? atoi(argv[3]) : 1;
  cpu_checks();
  for (int r = 0; gpu && r < repeat; ++r) gpu_checks(argc > 2 ? argv[2] : NULL);
  printf("%s checks: %d failure(s)\n", gpu ? "cpu+gpu" : "cpu", failures);
  fflush(stdout);  /* LeakSanitizer's report at exit ends the process without flushing */
  return failures ? 1 : 0;
}
