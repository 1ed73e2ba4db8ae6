/*
 * A plain C11 client of the renderer's C ABI (include/vrn.h), with no Python
 * and no C++: it builds a tiny field in C, renders it through vrn_render and
 * checks the result against the compositing closed form (Sec. 4.1, Eq. 2),
 * then serves the same camera through the serving engine (vrn_server_*) and
 * checks that every served result has the direct render's bits.
 *
 * The field has all-zero hash tables, MLP weights and biases, so every
 * evaluated sample has density exp(0) = 1 and color sigmoid(0) = 1/2.  With
 * n evaluated samples of step dt a pixel's transmittance is exp(-n dt), so
 * alpha = 1 - exp(-n dt) and each color channel is alpha / 2.
 *
 * Exit status: 0 = every check passed, 1 = a check failed, 2 = a HIP or
 * library call failed unexpectedly, 3 = no GPU (vrn_create reported
 * VRN_ERR_DEVICE; the header compiled and the library linked and loaded).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "vrn.h"

#define W 8
#define H 8
#define L 2
#define LOG2_T 4
#define BANDS 1
#define G 4

static int fail_call(const char* what, vrn_status s) {
  fprintf(stderr, "%s failed: %d (%s)\n", what, (int)s, vrn_last_error());
  return 2;
}

int main(void) {
  vrn_ctx* ctx = NULL;
  vrn_status s = vrn_create(0, 0, &ctx);
  if (s == VRN_ERR_DEVICE) {
    printf("no GPU: %s\n", vrn_last_error());
    return 3;
  }
  if (s != VRN_OK) return fail_call("vrn_create", s);

  /* field: 2 levels of T = 16 entries, zero tables and MLP, G^3 all occupied */
  const uint32_t T = 1u << LOG2_T, nsh = BANDS * BANDS;
  const size_t n_weights = (size_t)(2 * L) * 64 + 64 + 64 * 16 + 16 + (size_t)(15 + nsh) * 64 + 64 +
                           64 * 64 + 64 + 64 * 3 + 3;
  float* tables = calloc((size_t)L * T * 2, sizeof(float));
  float* weights = calloc(n_weights, sizeof(float));
  uint32_t occ[(G * G * G + 31) / 32];
  memset(occ, 0xFF, sizeof(occ));
  const uint32_t level_res[L] = {2, 3};
  vrn_field_desc d;
  memset(&d, 0, sizeof(d));
  d.n_levels = L;
  d.log2_T = LOG2_T;
  d.n_feat = 2;
  d.level_res = level_res;
  d.hash_primes[0] = 1u;
  d.hash_primes[1] = 2654435761u;
  d.hash_primes[2] = 805459861u;
  d.base_res = 2.0f;
  d.growth = 1.5f;
  d.table_dtype = VRN_F32;
  d.tables = tables;
  d.mlp_in = 2 * L;
  d.mlp_hidden = 64;
  d.geo_out = 16;
  d.sh_bands = BANDS;
  d.weights = weights;
  d.occ_res = G;
  d.occ_bits = occ;
  d.extent = 1.0f;
  d.dt = 0.0625f;
  d.max_samples = 64;
  d.t_min = 1e-4f;
  d.lod_radius_scale = 1.0f;
  vrn_field_id fid = 0;
  if ((s = vrn_load_field(ctx, &d, &fid)) != VRN_OK) return fail_call("vrn_load_field", s);
  free(tables);
  free(weights);

  /* one camera 1 unit in front of the cube, looking along +z */
  vrn_camera cam;
  memset(&cam, 0, sizeof(cam));
  cam.c2w[0] = cam.c2w[5] = cam.c2w[10] = 1.0f;
  cam.c2w[3] = 0.5f;
  cam.c2w[7] = 0.5f;
  cam.c2w[11] = -1.0f;
  cam.fx = cam.fy = 8.0f;
  cam.cx = W / 2.0f;
  cam.cy = H / 2.0f;
  cam.row_begin = 0;
  cam.row_end = H;

  float* d_rgba = NULL;
  uint32_t* d_n = NULL;
  if (hipMalloc((void**)&d_rgba, sizeof(float) * 4 * W * H) != hipSuccess ||
      hipMalloc((void**)&d_n, sizeof(uint32_t) * W * H) != hipSuccess) {
    fprintf(stderr, "hipMalloc failed\n");
    return 2;
  }
  vrn_render_opts opts;
  memset(&opts, 0, sizeof(opts));
  opts.compute = VRN_F32;
  opts.output = VRN_OUT_PQ;
  if ((s = vrn_render(ctx, fid, &cam, 1, W, H, &opts, d_rgba, d_n, NULL, 0, NULL)) != VRN_OK)
    return fail_call("vrn_render", s);
  float rgba[4 * W * H];
  uint32_t n[W * H];
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(rgba, d_rgba, sizeof(rgba), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(n, d_n, sizeof(n), hipMemcpyDeviceToHost) != hipSuccess) {
    fprintf(stderr, "device copy failed\n");
    return 2;
  }

  int bad = 0, hit = 0;
  for (int p = 0; p < W * H; ++p) {
    const double a = 1.0 - exp(-(double)n[p] * (double)d.dt);
    hit += n[p] > 0;
    if (fabs(rgba[4 * p + 3] - a) > 1e-5) ++bad;
    for (int c = 0; c < 3; ++c)
      if (fabs(rgba[4 * p + c] - 0.5 * a) > 1e-5) ++bad;
  }
  /* host-side validation: no camera is an invalid argument, nothing enqueued */
  s = vrn_render(ctx, fid, &cam, 0, W, H, &opts, d_rgba, d_n, NULL, 0, NULL);
  const int err_ok = s == VRN_ERR_INVALID_ARG && strlen(vrn_last_error()) > 0;

  /* the serving engine: the same camera served (graphs, merged launches,
   * an engine-owned arena) gives the direct render's bits */
  vrn_server_opts so;
  memset(&so, 0, sizeof(so));
  so.n_slots = 2;
  so.max_batch = 4;
  so.use_graphs = 1;
  so.render = opts;
  so.arena_bytes = 1u << 20;
  vrn_server* sv = NULL;
  if ((s = vrn_server_create(ctx, &so, &sv)) != VRN_OK) return fail_call("vrn_server_create", s);
  if ((s = vrn_server_prepare(sv, fid, 1, W, H)) != VRN_OK) return fail_call("vrn_server_prepare", s);
  enum { NREQ = 6 };
  uint64_t ids[NREQ];
  for (int i = 0; i < NREQ; ++i) {
    vrn_request_opts ro;
    memset(&ro, 0, sizeof(ro));
    ro.flags = (i == NREQ - 1) ? VRN_SERVE_RELEASE_ON_DONE : 0u;
    if ((s = vrn_server_submit(sv, fid, &cam, 1, W, H, &ro, &ids[i])) != VRN_OK)
      return fail_call("vrn_server_submit", s);
  }
  if ((s = vrn_server_hold(sv, 0)) != VRN_OK) return fail_call("vrn_server_hold", s);
  if ((s = vrn_server_drain(sv, 60.0)) != VRN_OK) return fail_call("vrn_server_drain", s);
  int served_bad = 0;
  float srgba[4 * W * H];
  for (int i = 0; i < NREQ; ++i) {
    vrn_served out;
    if ((s = vrn_server_wait(sv, ids[i], 10.0, &out)) != VRN_OK) return fail_call("vrn_server_wait", s);
    if (out.status != VRN_OK || !(out.t_done >= out.t_launch && out.t_launch >= out.t_arrival)) ++served_bad;
    if (i == NREQ - 1) {
      served_bad += out.d_rgba != NULL; /* returned to its ring at completion */
    } else if (out.d_rgba == NULL ||
               hipMemcpy(srgba, out.d_rgba, sizeof(srgba), hipMemcpyDeviceToHost) != hipSuccess ||
               memcmp(srgba, rgba, sizeof(srgba)) != 0) {
      ++served_bad;
    }
  }
  /* the engine's buffers pin the field */
  const int pinned_ok = vrn_unload_field(ctx, fid) == VRN_ERR_BUSY;
  for (int i = 0; i < NREQ; ++i)
    if ((s = vrn_server_release(sv, ids[i])) != VRN_OK) return fail_call("vrn_server_release", s);
  vrn_serve_stats st;
  if ((s = vrn_server_stats(sv, &st)) != VRN_OK) return fail_call("vrn_server_stats", s);
  if (st.completed != NREQ || st.held_bytes != 0 || st.requests != 0) ++served_bad;
  if ((s = vrn_server_evict(sv, 0)) != VRN_OK) return fail_call("vrn_server_evict", s);
  vrn_server_destroy(sv);

  hipFree(d_rgba);
  hipFree(d_n);
  if ((s = vrn_unload_field(ctx, fid)) != VRN_OK) return fail_call("vrn_unload_field", s);
  vrn_destroy(ctx);
  printf("pixels with samples %d of %d, mismatches %d, error path %s, served mismatches %d, pin %s\n", hit,
         W * H, bad, err_ok ? "ok" : "wrong", served_bad, pinned_ok ? "ok" : "wrong");
  return (bad == 0 && hit == W * H && err_ok && served_bad == 0 && pinned_ok) ? 0 : 1;
}
