/*
 * Host-side argument validation of the C ABI (include/vrn.h) driven from C,
 * meant to run against a library whose host code is built with AddressSanitizer
 * and UndefinedBehaviorSanitizer.  No GPU is needed: every call here is refused
 * on the host (a NULL context, or invalid arguments checked before the context),
 * which covers the validation code at the edges of its ranges (largest sizes,
 * overflow-prone products, non-finite values, NULL arrays).
 *
 * Exit status: 0 = every call returned the expected status, 1 = a mismatch.
 * A sanitizer report aborts the process with a non-zero status of its own.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "vrn.h"

static int failures = 0;

static void expect(const char* what, vrn_status got, vrn_status want) {
  if (got != want) {
    fprintf(stderr, "%s: got %d, want %d (%s)\n", what, (int)got, (int)want, vrn_last_error());
    ++failures;
  }
}

static vrn_camera camera(void) {
  vrn_camera c;
  memset(&c, 0, sizeof(c));
  c.c2w[0] = c.c2w[5] = c.c2w[10] = 1.0f;
  c.fx = c.fy = 100.0f;
  c.cx = c.cy = 50.0f;
  c.row_begin = 0;
  c.row_end = 100;
  return c;
}

int main(void) {
  /* cameras: every check at the edge of its range */
  vrn_camera cams[VRN_MAX_CAMS + 1];
  for (int i = 0; i <= VRN_MAX_CAMS; ++i) cams[i] = camera();
  expect("valid camera", vrn_check_cameras(cams, 1, 100, 100), VRN_OK);
  expect("17 cameras", vrn_check_cameras(cams, VRN_MAX_CAMS + 1, 100, 100), VRN_ERR_INVALID_ARG);
  expect("no camera", vrn_check_cameras(cams, 0, 100, 100), VRN_ERR_INVALID_ARG);
  expect("NULL cameras", vrn_check_cameras(NULL, 1, 100, 100), VRN_ERR_INVALID_ARG);
  cams[0].row_end = 16384;
  expect("largest frame, 16 cameras of 16384 x 8192", vrn_check_cameras(cams, 16, 16384, 8192),
         VRN_ERR_INVALID_ARG); /* row_end above H */
  for (int i = 0; i < 16; ++i) cams[i].row_end = 8192;
  expect("largest call, 2^31 pixels", vrn_check_cameras(cams, 16, 16384, 8192), VRN_OK);
  expect("one row more than 2^31 pixels", vrn_check_cameras(cams, 16, 16384, 8193), VRN_ERR_INVALID_ARG);
  expect("width above 16384", vrn_check_cameras(cams, 1, 16385, 8192), VRN_ERR_INVALID_ARG);
  expect("largest 32-bit sizes", vrn_check_cameras(cams, 16, 0xFFFFFFFFu, 0xFFFFFFFFu), VRN_ERR_INVALID_ARG);
  cams[1] = camera();
  cams[1].c2w[3] = NAN;
  expect("NaN position", vrn_check_cameras(cams + 1, 1, 100, 100), VRN_ERR_INVALID_ARG);
  cams[1] = camera();
  cams[1].fy = INFINITY;
  expect("infinite focal length", vrn_check_cameras(cams + 1, 1, 100, 100), VRN_ERR_INVALID_ARG);
  cams[1] = camera();
  cams[1].c2w[10] = 0.0f; /* rank-2 rotation */
  expect("degenerate rotation", vrn_check_cameras(cams + 1, 1, 100, 100), VRN_ERR_INVALID_ARG);
  cams[1] = camera();
  cams[1].c2w[0] = cams[1].c2w[5] = cams[1].c2w[10] = 3.0e38f; /* determinant overflows FP32 */
  expect("huge rotation entries", vrn_check_cameras(cams + 1, 1, 100, 100), VRN_OK);

  /* renders refused before any device work */
  cams[0] = camera();
  vrn_render_opts opts;
  memset(&opts, 0, sizeof(opts));
  expect("render, NULL context", vrn_render(NULL, 1, cams, 1, 100, 100, &opts, NULL, NULL, NULL, 0, NULL),
         VRN_ERR_INVALID_ARG);
  expect("render, 2^32 - 1 cameras",
         vrn_render(NULL, 1, cams, 0xFFFFFFFFu, 100, 100, &opts, NULL, NULL, NULL, 0, NULL), VRN_ERR_INVALID_ARG);
  expect("device-camera render, NULL context",
         vrn_render_device_cams(NULL, 1, cams, 1, 100, 100, &opts, NULL, NULL, NULL, 0, NULL), VRN_ERR_INVALID_ARG);

  /* field descriptors: each check, with a NULL context (checked after the descriptor) */
  const uint32_t level_res[2] = {2, 3};
  float tables[2 * 16 * 2];
  float weights[8192];
  uint32_t occ[2];
  memset(tables, 0, sizeof(tables));
  memset(weights, 0, sizeof(weights));
  memset(occ, 0xFF, sizeof(occ));
  vrn_field_desc d;
  memset(&d, 0, sizeof(d));
  d.n_levels = 2;
  d.log2_T = 4;
  d.n_feat = 2;
  d.level_res = level_res;
  d.hash_primes[0] = 1u;
  d.hash_primes[1] = 2654435761u;
  d.hash_primes[2] = 805459861u;
  d.base_res = 2.0f;
  d.growth = 1.5f;
  d.table_dtype = VRN_F32;
  d.tables = tables;
  d.mlp_in = 4;
  d.mlp_hidden = 64;
  d.geo_out = 16;
  d.sh_bands = 1;
  d.weights = weights;
  d.occ_res = 4;
  d.occ_bits = occ;
  d.extent = 1.0f;
  d.dt = 0.0625f;
  d.max_samples = 64;
  d.t_min = 1e-4f;
  d.lod_radius_scale = 1.0f;
  vrn_field_id fid = 0;
  expect("valid descriptor, NULL context", vrn_load_field(NULL, &d, &fid), VRN_ERR_INVALID_ARG);
  expect("NULL descriptor", vrn_load_field(NULL, NULL, &fid), VRN_ERR_INVALID_ARG);
  vrn_field_desc b = d;
  b.n_levels = 0xFFFFFFFFu;
  expect("2^32 - 1 levels", vrn_load_field(NULL, &b, &fid), VRN_ERR_UNSUPPORTED);
  b = d;
  b.log2_T = 0xFFFFFFFFu;
  expect("log2_T 2^32 - 1", vrn_load_field(NULL, &b, &fid), VRN_ERR_UNSUPPORTED);
  b = d;
  b.occ_res = 0xFFFFFFFFu;
  expect("occupancy 2^32 - 1", vrn_load_field(NULL, &b, &fid), VRN_ERR_UNSUPPORTED);
  b = d;
  b.mlp_in = 0xFFFFFFFFu;
  expect("mlp_in 2^32 - 1", vrn_load_field(NULL, &b, &fid), VRN_ERR_INVALID_ARG);
  b = d;
  b.sh_bands = 0xFFFFFFFFu;
  expect("sh_bands 2^32 - 1", vrn_load_field(NULL, &b, &fid), VRN_ERR_UNSUPPORTED);
  b = d;
  b.dt = NAN;
  expect("NaN dt", vrn_load_field(NULL, &b, &fid), VRN_ERR_INVALID_ARG);
  b = d;
  b.aabb_min[1] = -INFINITY;
  expect("infinite AABB", vrn_load_field(NULL, &b, &fid), VRN_ERR_INVALID_ARG);
  b = d;
  b.table_dtype = (vrn_dtype)12345;
  expect("unknown table dtype", vrn_load_field(NULL, &b, &fid), VRN_ERR_UNSUPPORTED);
  b = d;
  b.contraction = 1;
  b.aabb_min[0] = b.aabb_min[1] = b.aabb_min[2] = -2.0f;
  b.extent = 4.0f;
  b.radius = 1.0f;
  b.step_growth = 0.01f;
  b.max_lattice = 0xFFFFFFFFu;
  expect("sample table of 2^32 - 1 entries", vrn_load_field(NULL, &b, &fid), VRN_ERR_INVALID_ARG);
  b.max_lattice = 65536;
  expect("contracted field, NULL context", vrn_load_field(NULL, &b, &fid), VRN_ERR_INVALID_ARG);
  b = d;
  b.lod_enable = 1;
  b.growth = NAN;
  expect("NaN growth", vrn_load_field(NULL, &b, &fid), VRN_ERR_INVALID_ARG);

  /* stage entry points and queries with a NULL context */
  uint64_t bytes = 0;
  vrn_stats st;
  expect("workspace bytes", vrn_workspace_bytes(NULL, &bytes), VRN_ERR_INVALID_ARG);
  expect("field bytes", vrn_field_bytes(NULL, 1, &bytes), VRN_ERR_INVALID_ARG);
  expect("unload", vrn_unload_field(NULL, 1), VRN_ERR_INVALID_ARG);
  expect("stats", vrn_read_stats(NULL, NULL, &st, NULL), VRN_ERR_INVALID_ARG);
  expect("encode", vrn_encode(NULL, 1, NULL, NULL, NULL, 0xFFFFFFFFu, NULL, NULL), VRN_ERR_INVALID_ARG);
  expect("mlp", vrn_mlp(NULL, 1, NULL, NULL, 0xFFFFFFFFu, VRN_F16, NULL, NULL, NULL), VRN_ERR_INVALID_ARG);
  expect("prune", vrn_prune_grid(NULL, 1, 0.5f, 4, VRN_F16, NULL, NULL, NULL), VRN_ERR_INVALID_ARG);
  expect("set occupancy", vrn_set_occupancy(NULL, 1, NULL, NULL), VRN_ERR_INVALID_ARG);
  vrn_destroy(NULL);

  /* serving engine: NULL handles and options out of range */
  vrn_server* sv = NULL;
  vrn_server_opts so;
  memset(&so, 0, sizeof(so));
  so.n_slots = 2;
  so.max_batch = 4;
  so.arena_bytes = 1u << 20;
  expect("server, NULL context", vrn_server_create(NULL, &so, &sv), VRN_ERR_INVALID_ARG);
  uint64_t rid = 0;
  vrn_served served;
  vrn_serve_stats sst;
  expect("submit, NULL server", vrn_server_submit(NULL, 1, cams, 1, 100, 100, NULL, &rid), VRN_ERR_INVALID_ARG);
  expect("wait, NULL server", vrn_server_wait(NULL, 1, 0.0, &served), VRN_ERR_INVALID_ARG);
  expect("hold, NULL server", vrn_server_hold(NULL, 1), VRN_ERR_INVALID_ARG);
  expect("prepare, NULL server", vrn_server_prepare(NULL, 1, 1, 100, 100), VRN_ERR_INVALID_ARG);
  expect("release, NULL server", vrn_server_release(NULL, 1), VRN_ERR_INVALID_ARG);
  expect("cancel, NULL server", vrn_server_cancel(NULL, 1), VRN_ERR_INVALID_ARG);
  expect("drain, NULL server", vrn_server_drain(NULL, 0.0), VRN_ERR_INVALID_ARG);
  expect("evict, NULL server", vrn_server_evict(NULL, 0), VRN_ERR_INVALID_ARG);
  expect("server stats, NULL server", vrn_server_stats(NULL, &sst), VRN_ERR_INVALID_ARG);
  vrn_server_destroy(NULL);
  if (!(vrn_server_clock() > 0.0)) {
    printf("MISMATCH server clock\n");
    ++failures;
  }

  printf("%d mismatches\n", failures);
  return failures == 0 ? 0 : 1;
}
