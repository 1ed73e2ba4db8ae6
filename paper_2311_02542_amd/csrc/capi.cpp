// C ABI of the renderer (include/vrn.h): host validation, field residency,
// MFMA weight layout, workspaces and launches.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace vrn;

namespace {

thread_local std::string g_err;

// roctx ranges around the entry points, so a marker trace (rocprofv3
// --marker-trace) shows which call enqueued which kernels.  The marker
// library is opened at run time; without it the ranges cost nothing.
struct RoctxApi {
  int (*push)(const char*) = nullptr;
  int (*pop)() = nullptr;
  RoctxApi() {
    void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) return;
    push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
    pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
    if (!push || !pop) push = nullptr, pop = nullptr;
  }
};

const RoctxApi& roctx() {
  static const RoctxApi api;
  return api;
}

struct Range {
  explicit Range(const char* name) {
    if (roctx().push) roctx().push(name);
  }
  ~Range() {
    if (roctx().pop) roctx().pop();
  }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

vrn_status fail(vrn_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

vrn_status hip_fail(hipError_t e, const char* what) {
  return fail(VRN_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

struct Field {
  FieldDev dev{};
  std::vector<void*> allocs;
  uint64_t bytes = 0;
  std::vector<hipEvent_t> events;  // renders in flight
  // renders of the allocation-free entry point in flight: one event, made
  // at load time and re-recorded by every such render (those renders share
  // one scratch array, so the caller serialises them on the device)
  hipEvent_t noalloc_ev = nullptr;
  // output buffers of serving engines whose graphs render this field
  int pins = 0;
};


}  // namespace

struct vrn_ctx {
  int device = 0;
  uint64_t budget = 0;
  uint64_t used = 0;
  int n_cu = 0;
  std::mutex mu;
  std::map<uint32_t, Field*> fields;
  uint32_t next_id = 1;
  void* ws = nullptr;  // the context's own workspace
  void* scratch = nullptr;  // this device's scratch array (vrn_render_noalloc)
};

namespace {

bool finite(float v) { return std::isfinite(v); }

// ---- MFMA weight layout (mirrors the lane mapping documented in device.hpp)
// Input index feeding element e of lane group g, per layer; -1 = zero weight.
int in_index(int layer, int g, int e, int L, int nsh) {
  switch (layer) {
    case 0: {  // density layer 1: features of levels g + 4 (e >> 1)
      const int lev = g + 4 * (e >> 1);
      return lev < L ? 2 * lev + (e & 1) : -1;
    }
    case 2: {  // color layer 1: density outputs 4 g + e (output 0 = density), then SH g + 4 i
      if (e < 4) {
        const int o = 4 * g + e;
        return o >= 1 ? o - 1 : -1;
      }
      const int c = g + 4 * (e - 4);
      return c < nsh ? 15 + c : -1;
    }
    default:  // hidden-to-hidden layers: unit 16 (e >> 2) + 4 g + (e & 3)
      return 16 * (e >> 2) + 4 * g + (e & 3);
  }
}

uint16_t f16_bits(float f) {
  _Float16 h = (_Float16)f;
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}

uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

float bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

void arrange_weights(const float* W, int L, int nsh, std::vector<float>& w32, std::vector<uint16_t>& w16,
                     std::vector<uint16_t>& wbf, std::vector<uint16_t>& wx3, std::vector<float>& bias) {
  const int din = 2 * L, cin = 15 + nsh;
  // offsets into the concatenated host weights
  const float* W1 = W;
  const float* b1 = W1 + din * 64;
  const float* W2 = b1 + 64;
  const float* b2 = W2 + 64 * 16;
  const float* W3 = b2 + 16;
  const float* b3 = W3 + cin * 64;
  const float* W4 = b3 + 64;
  const float* b4 = W4 + 64 * 64;
  const float* W5 = b4 + 64;
  const float* b5 = W5 + 64 * 3;
  struct Layer { const float* w; int n_in, n_out, n_ot, n_k, off; };
  const Layer layers[5] = {{W1, din, 64, 4, 8, kW32_D1}, {W2, 64, 16, 1, 16, kW32_D2},
                           {W3, cin, 64, 4, 8, kW32_C1}, {W4, 64, 64, 4, 16, kW32_C2},
                           {W5, 64, 3, 1, 16, kW32_C3}};
  w32.assign(kW32Total, 0.0f);
  w16.assign(kW16Total, 0);
  wbf.assign(kW16Total, 0);
  wx3.assign(3 * (size_t)kW16Total, 0);
  for (int li = 0; li < 5; ++li) {
    const Layer& Ly = layers[li];
    for (int ot = 0; ot < Ly.n_ot; ++ot)
      for (int s = 0; s < Ly.n_k; ++s)
        for (int lane = 0; lane < 64; ++lane) {
          const int g = lane >> 4, out = 16 * ot + (lane & 15);
          const int in = in_index(li, g, s, L, nsh);
          const float v = (in >= 0 && in < Ly.n_in && out < Ly.n_out) ? Ly.w[in * Ly.n_out + out] : 0.0f;
          w32[Ly.off + ((ot * (Ly.n_k / 4) + s / 4) * 64 + lane) * 4 + (s % 4)] = v;
          const int s2 = s >> 3, j = s & 7;
          const size_t o16 = Ly.off + ((size_t)(ot * (Ly.n_k / 8) + s2) * 64 + lane) * 8 + j;
          w16[o16] = f16_bits(v);
          wbf[o16] = bf16_bits(v);
          // the FP32 weight as the exact sum of three BF16 parts (VRN_F32X):
          // each part rounds the residual of the previous ones
          float r = v;
          for (int k = 0; k < 3; ++k) {
            const uint16_t b = bf16_bits(r);
            wx3[(size_t)k * kW16Total + o16] = b;
            r -= bf16_value(b);
          }
        }
  }
  bias.assign(kBiasTotal, 0.0f);
  for (int i = 0; i < 64; ++i) {
    bias[kB1 + i] = b1[i];
    bias[kB3 + i] = b3[i];
    bias[kB4 + i] = b4[i];
  }
  for (int i = 0; i < 16; ++i) bias[kB2 + i] = b2[i];
  for (int i = 0; i < 3; ++i) bias[kB5 + i] = b5[i];
}

uint64_t weight_count(int L, int nsh) {
  const uint64_t din = 2 * L, cin = 15 + nsh;
  return din * 64 + 64 + 64 * 16 + 16 + cin * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3;
}

vrn_status validate_desc(const vrn_field_desc* d) {
  if (!d) return fail(VRN_ERR_INVALID_ARG, "field descriptor is NULL");
  if (d->n_feat != 2) return fail(VRN_ERR_UNSUPPORTED, "only F = 2 features per entry are supported");
  if (d->n_levels < 1 || d->n_levels > (uint32_t)kMaxLevels)
    return fail(VRN_ERR_UNSUPPORTED, "n_levels must be 1..16");
  if (d->log2_T < 4 || d->log2_T > 24) return fail(VRN_ERR_UNSUPPORTED, "log2_T must be 4..24");
  if (!d->level_res || !d->tables || !d->weights || !d->occ_bits)
    return fail(VRN_ERR_INVALID_ARG, "NULL level_res / tables / weights / occ_bits");
  if (d->table_dtype != VRN_F32 && d->table_dtype != VRN_F16)
    return fail(VRN_ERR_UNSUPPORTED, "table_dtype must be VRN_F32 or VRN_F16");
  if (d->mlp_in != 2 * d->n_levels) return fail(VRN_ERR_INVALID_ARG, "mlp_in must equal 2 * n_levels");
  if (d->mlp_hidden != 64) return fail(VRN_ERR_UNSUPPORTED, "mlp_hidden must be 64");
  if (d->geo_out != 16) return fail(VRN_ERR_UNSUPPORTED, "geo_out must be 16");
  if (d->sh_bands < 1 || d->sh_bands > 4) return fail(VRN_ERR_UNSUPPORTED, "sh_bands must be 1..4");
  if (d->occ_res < 1 || d->occ_res > 1024) return fail(VRN_ERR_UNSUPPORTED, "occ_res must be 1..1024");
  for (uint32_t l = 0; l < d->n_levels; ++l)
    if (d->level_res[l] < 1 || d->level_res[l] > (1u << 20))
      return fail(VRN_ERR_INVALID_ARG, "level_res must be 1..2^20");
  for (int a = 0; a < 3; ++a)
    if (!finite(d->aabb_min[a])) return fail(VRN_ERR_INVALID_ARG, "aabb_min not finite");
  if (!finite(d->extent) || !(d->extent > 0.0f)) return fail(VRN_ERR_INVALID_ARG, "extent must be > 0");
  if (!finite(d->dt) || !(d->dt > 0.0f)) return fail(VRN_ERR_INVALID_ARG, "dt must be > 0");
  if (d->max_samples < 1) return fail(VRN_ERR_INVALID_ARG, "max_samples must be >= 1");
  if (!finite(d->t_min) || d->t_min < 0.0f || d->t_min >= 1.0f)
    return fail(VRN_ERR_INVALID_ARG, "t_min must be in [0, 1)");
  if (d->contraction != 0 && d->contraction != 1) return fail(VRN_ERR_INVALID_ARG, "contraction must be 0 or 1");
  if (!finite(d->step_growth) || d->step_growth < 0.0f || d->step_growth >= 1.0f)
    return fail(VRN_ERR_INVALID_ARG, "step_growth must be in [0, 1)");
  if (d->contraction) {
    for (int a = 0; a < 3; ++a)
      if (!finite(d->center[a]) || d->aabb_min[a] != -2.0f)
        return fail(VRN_ERR_INVALID_ARG, "contracted fields need a finite center and aabb_min = -2");
    if (d->extent != 4.0f) return fail(VRN_ERR_INVALID_ARG, "contracted fields need extent = 4");
    if (!finite(d->radius) || !(d->radius > 0.0f)) return fail(VRN_ERR_INVALID_ARG, "radius must be > 0");
  }
  if ((d->contraction || d->step_growth > 0.0f) && (d->max_lattice < 1 || d->max_lattice > 65536))
    return fail(VRN_ERR_INVALID_ARG, "max_lattice must be 1..65536 when a sample table is used");
  if (d->lod_enable) {
    if (!finite(d->base_res) || !(d->base_res > 0.0f)) return fail(VRN_ERR_INVALID_ARG, "base_res must be > 0");
    if (!finite(d->growth) || !(d->growth > 1.0f)) return fail(VRN_ERR_INVALID_ARG, "growth must be > 1");
    if (!finite(d->lod_bias)) return fail(VRN_ERR_INVALID_ARG, "lod_bias not finite");
    if (!finite(d->lod_radius_scale) || !(d->lod_radius_scale > 0.0f))
      return fail(VRN_ERR_INVALID_ARG, "lod_radius_scale must be > 0");
  }
  return VRN_OK;
}

vrn_status check_cams(const vrn_camera* cams, uint32_t n_cams, uint32_t W, uint32_t H) {
  if (!cams) return fail(VRN_ERR_INVALID_ARG, "cameras are NULL");
  if (n_cams < 1 || n_cams > (uint32_t)kMaxCams) return fail(VRN_ERR_INVALID_ARG, "n_cams must be 1..16");
  if (W < 1 || H < 1 || W > 16384 || H > 16384) return fail(VRN_ERR_INVALID_ARG, "W and H must be 1..16384");
  if ((uint64_t)n_cams * W * H > (1ull << 31)) return fail(VRN_ERR_INVALID_ARG, "too many pixels in one call");
  for (uint32_t c = 0; c < n_cams; ++c) {
    const vrn_camera& k = cams[c];
    for (int i = 0; i < 12; ++i)
      if (!finite(k.c2w[i])) return fail(VRN_ERR_INVALID_ARG, "camera pose is not finite");
    if (!finite(k.fx) || !finite(k.fy) || !finite(k.cx) || !finite(k.cy) || !(k.fx > 0.0f) || !(k.fy > 0.0f))
      return fail(VRN_ERR_INVALID_ARG, "camera intrinsics must be finite with fx, fy > 0");
    const float* R = k.c2w;
    const double det = (double)R[0] * ((double)R[5] * R[10] - (double)R[6] * R[9]) -
                       (double)R[1] * ((double)R[4] * R[10] - (double)R[6] * R[8]) +
                       (double)R[2] * ((double)R[4] * R[9] - (double)R[5] * R[8]);
    if (!(std::fabs(det) > 1e-6)) return fail(VRN_ERR_INVALID_ARG, "camera rotation is degenerate");
    if (!(k.row_begin < k.row_end) || k.row_end > H)
      return fail(VRN_ERR_INVALID_ARG, "camera rows must satisfy row_begin < row_end <= H");
  }
  return VRN_OK;
}

Field* find_field(vrn_ctx* ctx, vrn_field_id id) {
  auto it = ctx->fields.find(id);
  return it == ctx->fields.end() ? nullptr : it->second;
}

template <typename T>
hipError_t upload(Field* f, const T* host, size_t count, T** out) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(count * sizeof(T), 16));
  if (e != hipSuccess) return e;
  f->allocs.push_back(p);
  f->bytes += count * sizeof(T);
  e = hipMemcpy(p, host, count * sizeof(T), hipMemcpyHostToDevice);
  *out = static_cast<T*>(p);
  return e;
}

// device memory the kernels fill themselves (no host copy)
template <typename T>
hipError_t alloc_only(Field* f, size_t count, T** out) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(count * sizeof(T), 16));
  if (e != hipSuccess) return e;
  f->allocs.push_back(p);
  f->bytes += count * sizeof(T);
  *out = static_cast<T*>(p);
  return hipSuccess;
}

void free_field(Field* f) {
  for (hipEvent_t ev : f->events) hipEventDestroy(ev);
  if (f->noalloc_ev) hipEventDestroy(f->noalloc_ev);
  for (void* p : f->allocs) hipFree(p);
  delete f;
}

void track(Field* f, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  hipEvent_t ev = nullptr;
  for (hipEvent_t e : f->events)
    if (hipEventQuery(e) == hipSuccess) {
      ev = e;
      break;
    }
  if (!ev) {
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return;
    f->events.push_back(ev);
  }
  hipEventRecord(ev, s);
}

vrn_status check_opts(const vrn_render_opts* opts) {
  if (opts && opts->compute != VRN_F32 && opts->compute != VRN_F16 && opts->compute != VRN_BF16 &&
      opts->compute != VRN_F32X)
    return fail(VRN_ERR_INVALID_ARG, "opts.compute must be VRN_F32, VRN_F16, VRN_BF16 or VRN_F32X");
  if (opts && (opts->output < VRN_OUT_PQ || opts->output > VRN_OUT_SRGB))
    return fail(VRN_ERR_INVALID_ARG, "opts.output must be VRN_OUT_PQ, VRN_OUT_LINEAR or VRN_OUT_SRGB");
  if (opts && (!finite(opts->exposure_ev) || std::fabs(opts->exposure_ev) > 64.0f))
    return fail(VRN_ERR_INVALID_ARG, "opts.exposure_ev must be finite, |ev| <= 64");
  return VRN_OK;
}

vrn_status do_render(vrn_ctx* ctx, Field* f, const vrn_camera* d_cams, uint32_t n_cams, uint32_t W,
                     uint32_t H, const vrn_render_opts* opts, float* d_rgba, uint32_t* d_nsamples, void* ws,
                     hipStream_t s, bool noalloc = false) {
  RenderArgs a{};
  a.F = f->dev;
  a.cams = d_cams;
  a.n_cams = n_cams;
  a.W = W;
  a.H = H;
  a.rgba = d_rgba;
  a.nsamples = d_nsamples;
  a.ws = static_cast<uint8_t*>(ws);
  a.output = opts ? opts->output : VRN_OUT_PQ;
  a.exposure = opts ? std::exp2(opts->exposure_ev) : 1.0f;
  a.budget = (opts && opts->march_budget) ? opts->march_budget : 256u;
  const int compute = opts ? (int)opts->compute : 0;
  const uint64_t rays = (uint64_t)n_cams * W * H;
  const uint64_t bt = (uint64_t)render_block_threads(compute);
  const uint64_t want = (rays + bt - 1) / bt;
  const uint64_t cap = (uint64_t)ctx->n_cu * render_blocks_per_cu(f->dev, compute);
  const int grid = (int)std::max<uint64_t>(1, std::min(want, cap));
  hipError_t e = launch_render(a, compute, grid, s);
  if (e != hipSuccess) return hip_fail(e, "render launch");
  if (!noalloc) {
    track(f, s);
  } else {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
      hipEventRecord(f->noalloc_ev, s);
  }
  return VRN_OK;
}

}  // namespace

namespace vrn {

vrn_status set_error(vrn_status s, const char* msg) { return fail(s, msg); }

int ctx_device(const vrn_ctx* ctx) { return ctx->device; }

vrn_status field_pin(vrn_ctx* ctx, vrn_field_id field, int delta) {
  std::lock_guard<std::mutex> lock(ctx->mu);
  Field* f = find_field(ctx, field);
  if (!f) return fail(VRN_ERR_NOT_FOUND, "unknown field id");
  f->pins += delta;
  return VRN_OK;
}

}  // namespace vrn

extern "C" {

const char* vrn_last_error(void) { return g_err.c_str(); }

vrn_status vrn_create(int device, uint64_t hbm_budget_bytes, vrn_ctx** out) {
  if (!out) return fail(VRN_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return fail(VRN_ERR_DEVICE, "no HIP device available");
  if (device < 0 || device >= n) return fail(VRN_ERR_DEVICE, "device ordinal out of range");
  if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  vrn_ctx* ctx = new vrn_ctx();
  ctx->device = device;
  ctx->budget = hbm_budget_bytes;
  ctx->n_cu = prop.multiProcessorCount;
  if ((e = hipMalloc(&ctx->ws, kWsBytes)) != hipSuccess) {
    delete ctx;
    return fail(VRN_ERR_OUT_OF_MEMORY, "workspace allocation failed");
  }
  if ((e = hipMemset(ctx->ws, 0, kWsBytes)) != hipSuccess) {
    hipFree(ctx->ws);
    delete ctx;
    return hip_fail(e, "workspace init");
  }
  // the scratch array of vrn_render_noalloc: its address on this device
  // (taken once per device, with the device current)
  if ((e = scratch_address(device, &ctx->scratch)) != hipSuccess) {
    hipFree(ctx->ws);
    delete ctx;
    return hip_fail(e, "scratch address");
  }
  *out = ctx;
  return VRN_OK;
}

void vrn_destroy(vrn_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  for (auto& kv : ctx->fields) free_field(kv.second);
  if (ctx->ws) hipFree(ctx->ws);
  delete ctx;
}

vrn_status vrn_load_field(vrn_ctx* ctx, const vrn_field_desc* d, vrn_field_id* out) {
  Range range("vrn_load_field");
  vrn_status st = validate_desc(d);
  if (st != VRN_OK) return st;
  if (!ctx || !out) return fail(VRN_ERR_INVALID_ARG, "ctx or out is NULL");
  std::lock_guard<std::mutex> lock(ctx->mu);
  const uint32_t L = d->n_levels, G = d->occ_res, nsh = d->sh_bands * d->sh_bands;
  const uint64_t T = 1ull << d->log2_T;
  const uint64_t n_tab = (uint64_t)L * T * 2;
  // finite tables and weights (LOD-skipped levels count as zeros only if finite)
  if (d->table_dtype == VRN_F32) {
    const float* t = static_cast<const float*>(d->tables);
    for (uint64_t i = 0; i < n_tab; ++i)
      if (!finite(t[i])) return fail(VRN_ERR_INVALID_ARG, "hash tables contain non-finite values");
  } else {
    const uint16_t* t = static_cast<const uint16_t*>(d->tables);
    for (uint64_t i = 0; i < n_tab; ++i)
      if ((t[i] & 0x7C00u) == 0x7C00u) return fail(VRN_ERR_INVALID_ARG, "hash tables contain non-finite values");
  }
  const uint64_t nw = weight_count((int)L, (int)nsh);
  for (uint64_t i = 0; i < nw; ++i)
    if (!finite(d->weights[i])) return fail(VRN_ERR_INVALID_ARG, "MLP weights contain non-finite values");

  // occupancy: 4x4x4 bricks (one 64-bit word each) and a coarse grid of
  // <= 32^3 blocks (2^cshift cells, a multiple of the brick) for LDS
  const uint32_t Gb = (G + 3) / 4;
  uint32_t cshift = 2;
  while (((G + (1u << cshift) - 1) >> cshift) > 32u) ++cshift;
  const uint32_t Gc = (G + (1u << cshift) - 1) >> cshift;
  const uint64_t n_fine = (uint64_t)G * G * G, n_words = (n_fine + 31) / 32;
  std::vector<unsigned long long> bricks((size_t)Gb * Gb * Gb, 0ull);
  std::vector<uint32_t> coarse(((uint64_t)Gc * Gc * Gc + 31) / 32, 0u);
  for (uint64_t w = 0; w < n_words; ++w) {
    uint32_t word = d->occ_bits[w];
    while (word) {
      const int b = __builtin_ctz(word);
      word &= word - 1;
      const uint64_t i = w * 32 + (uint64_t)b;
      if (i >= n_fine) break;
      const uint32_t x = (uint32_t)(i % G), y = (uint32_t)((i / G) % G), z = (uint32_t)(i / ((uint64_t)G * G));
      const uint64_t bi = (x >> 2) + (uint64_t)Gb * ((y >> 2) + (uint64_t)Gb * (z >> 2));
      bricks[bi] |= 1ull << ((x & 3) + 4 * (y & 3) + 16 * (z & 3));
      const uint64_t ci = (x >> cshift) + (uint64_t)Gc * ((y >> cshift) + (uint64_t)Gc * (z >> cshift));
      coarse[ci >> 5] |= 1u << (ci & 31);
    }
  }
  // the coarse grid dilated by one block: empty only where the block and all
  // 26 neighbours are empty (long empty runs are walked block by block)
  std::vector<uint32_t> coarse_dil(coarse.size(), 0u);
  for (uint32_t cz = 0; cz < Gc; ++cz)
    for (uint32_t cy = 0; cy < Gc; ++cy)
      for (uint32_t cx = 0; cx < Gc; ++cx) {
        bool any = false;
        for (int dz = -1; dz <= 1 && !any; ++dz)
          for (int dy = -1; dy <= 1 && !any; ++dy)
            for (int dx = -1; dx <= 1 && !any; ++dx) {
              const int x = (int)cx + dx, y = (int)cy + dy, z = (int)cz + dz;
              if (x < 0 || y < 0 || z < 0 || x >= (int)Gc || y >= (int)Gc || z >= (int)Gc) continue;
              const uint64_t ci = (uint64_t)x + (uint64_t)Gc * ((uint64_t)y + (uint64_t)Gc * (uint64_t)z);
              any = (coarse[ci >> 5] >> (ci & 31)) & 1u;
            }
        if (any) {
          const uint64_t ci = (uint64_t)cx + (uint64_t)Gc * ((uint64_t)cy + (uint64_t)Gc * (uint64_t)cz);
          coarse_dil[ci >> 5] |= 1u << (ci & 31);
        }
      }
  std::vector<float> w32, bias;
  std::vector<uint16_t> w16, wbf, wx3;
  arrange_weights(d->weights, (int)L, (int)nsh, w32, w16, wbf, wx3, bias);
  std::vector<LevelDev> lv(L);
  for (uint32_t l = 0; l < L; ++l) {
    const uint64_t N = d->level_res[l], s = N + 1;
    LevelDev& P = lv[l];
    const uint32_t esize = d->table_dtype == VRN_F16 ? 4u : 8u;   // one entry: two features
    P.top = (float)(N - 1);
    P.dense = (s * s * s <= T) ? 1u : 0u;
    P.bx = (P.dense ? 1u : d->hash_primes[0]) * esize;
    P.by = (P.dense ? (uint32_t)s : d->hash_primes[1]) * esize;
    P.bz = (P.dense ? (uint32_t)(s * s) : d->hash_primes[2]) * esize;
    const double S = (double)N / (double)d->extent;
    P.s_hi = (float)S;
    P.base = (uint32_t)((uint64_t)l * T * esize);
    P.below_n = std::nextafter((float)N, 0.0f);
    P.s64 = S;
    P.top64 = (double)(N - 1);
  }
  // canonical FP32 sample table (same recurrence, same rounding, as the oracle)
  const bool use_table = d->contraction || d->step_growth > 0.0f;
  std::vector<float> lat;
  if (use_table) {
    lat.resize((size_t)d->max_lattice + 1);
    volatile float t = 0.5f * d->dt;   // volatile: every step rounded to FP32
    lat[0] = t;
    for (uint32_t k = 0; k < d->max_lattice; ++k) {
      const float g = d->step_growth * t;
      t = t + (g > d->dt ? g : d->dt);
      lat[k + 1] = t;
    }
  }
  const uint64_t tab_bytes = n_tab * (d->table_dtype == VRN_F16 ? 2 : 4);
  const uint64_t need = tab_bytes + bricks.size() * 8 + coarse.size() * 8 + (w32.size() + bias.size()) * 4 +
                        (w16.size() + wbf.size() + wx3.size()) * 2 + lv.size() * sizeof(LevelDev) + lat.size() * 4 +
                        bricks.size() * 4 + 256;
  if (ctx->budget && ctx->used + need > ctx->budget)
    return fail(VRN_ERR_BUDGET, "loading the field would exceed the HBM budget");

  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  Field* f = new Field();
  FieldDev& F = f->dev;
  uint8_t* tab = nullptr;
  LevelDev* dlv = nullptr;
  unsigned long long* dbr = nullptr;
  uint32_t *dco = nullptr, *dcd = nullptr;
  float *dw32 = nullptr, *dbias = nullptr, *dlat = nullptr;
  uint32_t *dlist = nullptr, *dcount = nullptr;
  const std::vector<uint32_t> zeros(64, 0u);
  uint16_t *dw16 = nullptr, *dwbf = nullptr, *dwx3 = nullptr;
  if ((e = upload(f, static_cast<const uint8_t*>(d->tables), tab_bytes, &tab)) ||
      (e = upload(f, lv.data(), lv.size(), &dlv)) || (e = upload(f, bricks.data(), bricks.size(), &dbr)) ||
      (e = upload(f, coarse.data(), coarse.size(), &dco)) ||
      (e = upload(f, coarse_dil.data(), coarse_dil.size(), &dcd)) || (e = upload(f, w32.data(), w32.size(), &dw32)) ||
      (e = upload(f, w16.data(), w16.size(), &dw16)) || (e = upload(f, wbf.data(), wbf.size(), &dwbf)) ||
      (e = upload(f, wx3.data(), wx3.size(), &dwx3)) ||
      (e = upload(f, bias.data(), bias.size(), &dbias)) ||
      (use_table && (e = upload(f, lat.data(), lat.size(), &dlat))) ||
      (e = alloc_only(f, bricks.size(), &dlist)) || (e = upload(f, zeros.data(), zeros.size(), &dcount)) ||
      (e = hipEventCreateWithFlags(&f->noalloc_ev, hipEventDisableTiming))) {
    free_field(f);
    return e == hipErrorOutOfMemory ? fail(VRN_ERR_OUT_OF_MEMORY, "device allocation failed")
                                    : hip_fail(e, "field upload");
  }
  F.tables = tab;
  F.levels = dlv;
  F.bricks = dbr;
  F.coarse = dco;
  F.coarse_dil = dcd;
  F.brick_list = dlist;
  F.brick_count = dcount;
  F.w32 = dw32;
  F.w16 = dw16;
  F.wbf = dwbf;
  F.wx3 = dwx3;
  F.bias = dbias;
  F.L = L;
  F.log2T = d->log2_T;
  F.Tmask = (uint32_t)(T - 1);
  F.table_f16 = d->table_dtype == VRN_F16;
  F.bmask = F.Tmask * (F.table_f16 ? 4u : 8u);
  F.G = G;
  F.Gb = Gb;
  F.Gc = Gc;
  F.cshift = cshift;
  F.nsh = nsh;
  for (int a = 0; a < 3; ++a) F.amin[a] = d->aabb_min[a];
  F.cs = (float)((double)G / (double)d->extent);
  F.dt = d->dt;
  F.inv_dt = (float)(1.0 / (double)d->dt);
  F.inv_cs = (float)((double)d->extent / (double)G);
  F.t_min = d->t_min;
  F.extent = d->extent;
  F.max_samples = d->max_samples;
  F.lod = d->lod_enable ? 1 : 0;
  F.inv_ln_f = d->lod_enable ? (float)(1.0 / std::log((double)d->growth)) : 0.0f;
  F.lod_c = d->lod_enable ? (float)std::log(2.0 * (double)d->base_res / (double)d->extent) : 0.0f;
  F.lod_bias = d->lod_bias;
  F.lod_radius_scale = d->lod_enable ? d->lod_radius_scale : 1.0f;
  F.d1_ksteps = L > 8 ? 8u : 4u;
  F.lat = dlat;
  F.lat_K = use_table ? d->max_lattice : 0u;
  // the table's shape, for the search guess: steps of dt while step_growth
  // t_k <= dt, growth by (1 + step_growth) per step after
  F.step_growth = d->step_growth;
  F.lat_tsw = INFINITY;
  F.lat_ksw = 0.0f;
  F.lat_inv_log = 0.0f;
  if (use_table && d->step_growth > 0.0f) {
    for (uint32_t k = 0; k < d->max_lattice; ++k) {
      const float g = d->step_growth * lat[k];
      if (g > d->dt) {
        F.lat_tsw = lat[k];
        F.lat_ksw = (float)k;
        break;
      }
    }
    F.lat_inv_log = (float)(1.0 / std::log1p((double)d->step_growth));
  }
  F.contract = d->contraction;
  for (int a = 0; a < 3; ++a) F.center[a] = d->center[a];
  F.radius = d->contraction ? d->radius : 1.0f;
  F.inv_radius = d->contraction ? (float)(1.0 / (double)d->radius) : 1.0f;
  F.lod_c2 = d->lod_enable ? (float)std::log(2.0 * (double)d->base_res) : 0.0f;
  F.dense_mask = 0;
  for (uint32_t l = 0; l < L; ++l) F.dense_mask |= lv[l].dense << l;
  F.c1_ksteps = 8u;
  const vrn_field_id id = ctx->next_id++;
  ctx->fields[id] = f;
  ctx->used += f->bytes;
  *out = id;
  return VRN_OK;
}

vrn_status vrn_unload_field(vrn_ctx* ctx, vrn_field_id field) {
  Range range("vrn_unload_field");
  if (!ctx) return fail(VRN_ERR_INVALID_ARG, "ctx is NULL");
  std::lock_guard<std::mutex> lock(ctx->mu);
  Field* f = find_field(ctx, field);
  if (!f) return fail(VRN_ERR_NOT_FOUND, "unknown field id");
  hipSetDevice(ctx->device);
  for (hipEvent_t ev : f->events)
    if (hipEventQuery(ev) == hipErrorNotReady) return fail(VRN_ERR_BUSY, "field has renders in flight");
  if (hipEventQuery(f->noalloc_ev) == hipErrorNotReady) return fail(VRN_ERR_BUSY, "field has renders in flight");
  if (f->pins > 0) return fail(VRN_ERR_BUSY, "a serving engine holds output buffers of this field");
  ctx->used -= f->bytes;
  ctx->fields.erase(field);
  free_field(f);
  return VRN_OK;
}

vrn_status vrn_field_bytes(vrn_ctx* ctx, vrn_field_id field, uint64_t* out) {
  if (!ctx || !out) return fail(VRN_ERR_INVALID_ARG, "ctx or out is NULL");
  std::lock_guard<std::mutex> lock(ctx->mu);
  Field* f = find_field(ctx, field);
  if (!f) return fail(VRN_ERR_NOT_FOUND, "unknown field id");
  *out = f->bytes;
  return VRN_OK;
}

vrn_status vrn_workspace_bytes(vrn_ctx* ctx, uint64_t* out) {
  if (!ctx || !out) return fail(VRN_ERR_INVALID_ARG, "ctx or out is NULL");
  *out = kWsBytes;
  return VRN_OK;
}

vrn_status vrn_render_bytes(vrn_ctx* ctx, vrn_field_id field, uint32_t n_cams, uint32_t W, uint32_t H,
                            const vrn_render_opts* opts, uint64_t* out) {
  if (!ctx || !out) return fail(VRN_ERR_INVALID_ARG, "ctx or out is NULL");
  if (n_cams < 1 || n_cams > (uint32_t)kMaxCams || W < 1 || H < 1 || W > 16384 || H > 16384 ||
      (uint64_t)n_cams * W * H > (1ull << 31))
    return fail(VRN_ERR_INVALID_ARG, "n_cams must be 1..16 and W, H 1..16384 (at most 2^31 pixels)");
  vrn_status st = check_opts(opts);
  if (st != VRN_OK) return st;
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (!find_field(ctx, field)) return fail(VRN_ERR_NOT_FOUND, "unknown field id");
  // every path writes the same outputs: RGBA float4 and a uint32 count per pixel
  *out = (uint64_t)kWsBytes + (uint64_t)n_cams * W * H * (4 * sizeof(float) + sizeof(uint32_t));
  return VRN_OK;
}

vrn_status vrn_workspace_init(vrn_ctx* ctx, void* ws, uint64_t bytes, void* stream) {
  Range range("vrn_workspace_init");
  if (!ctx || !ws) return fail(VRN_ERR_INVALID_ARG, "ctx or workspace is NULL");
  if (bytes < (uint64_t)kWsBytes) return fail(VRN_ERR_INVALID_ARG, "workspace too small");
  std::lock_guard<std::mutex> lock(ctx->mu);
  hipSetDevice(ctx->device);
  hipError_t e = launch_zero(ws, kWsBytes, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? VRN_OK : hip_fail(e, "workspace init");
}

vrn_status vrn_check_cameras(const vrn_camera* cams, uint32_t n_cams, uint32_t W, uint32_t H) {
  return check_cams(cams, n_cams, W, H);
}

static vrn_status render_common(vrn_ctx* ctx, vrn_field_id field, const vrn_camera* cams, bool cams_dev,
                                uint32_t n_cams, uint32_t W, uint32_t H, const vrn_render_opts* opts,
                                float* d_rgba, uint32_t* d_nsamples, void* ws, uint64_t ws_bytes,
                                void* stream) {
  Range range(cams_dev ? "vrn_render_device_cams" : "vrn_render");
  if (!cams) return fail(VRN_ERR_INVALID_ARG, "cameras are NULL");
  vrn_status st = cams_dev ? VRN_OK : check_cams(cams, n_cams, W, H);
  if (st != VRN_OK) return st;
  if (!ctx) return fail(VRN_ERR_INVALID_ARG, "ctx is NULL");
  if (!d_rgba) return fail(VRN_ERR_INVALID_ARG, "d_rgba is NULL");
  if (cams_dev && (n_cams < 1 || n_cams > (uint32_t)kMaxCams || W < 1 || H < 1 || W > 16384 || H > 16384 ||
                   (uint64_t)n_cams * W * H > (1ull << 31)))
    return fail(VRN_ERR_INVALID_ARG, "n_cams must be 1..16 and W, H 1..16384");
  if ((st = check_opts(opts)) != VRN_OK) return st;
  if (ws && ws_bytes < (uint64_t)kWsBytes) return fail(VRN_ERR_INVALID_ARG, "workspace too small");
  std::lock_guard<std::mutex> lock(ctx->mu);
  Field* f = find_field(ctx, field);
  if (!f) return fail(VRN_ERR_NOT_FOUND, "unknown field id");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  void* w = ws ? ws : ctx->ws;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const vrn_camera* d_cams = cams;
  if (!cams_dev) {
    uint8_t* slot = static_cast<uint8_t*>(w) + kWsCams;
    e = hipMemcpyAsync(slot, cams, n_cams * sizeof(vrn_camera), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "camera upload");
    d_cams = reinterpret_cast<const vrn_camera*>(slot);
  }
  return do_render(ctx, f, d_cams, n_cams, W, H, opts, d_rgba, d_nsamples, w, s);
}

vrn_status vrn_render(vrn_ctx* ctx, vrn_field_id field, const vrn_camera* cams, uint32_t n_cams, uint32_t W,
                      uint32_t H, const vrn_render_opts* opts, float* d_rgba, uint32_t* d_nsamples,
                      void* d_workspace, uint64_t workspace_bytes, void* hip_stream) {
  return render_common(ctx, field, cams, false, n_cams, W, H, opts, d_rgba, d_nsamples, d_workspace,
                       workspace_bytes, hip_stream);
}

vrn_status vrn_render_device_cams(vrn_ctx* ctx, vrn_field_id field, const vrn_camera* d_cams, uint32_t n_cams,
                                  uint32_t W, uint32_t H, const vrn_render_opts* opts, float* d_rgba,
                                  uint32_t* d_nsamples, void* d_workspace, uint64_t workspace_bytes,
                                  void* hip_stream) {
  return render_common(ctx, field, d_cams, true, n_cams, W, H, opts, d_rgba, d_nsamples, d_workspace,
                       workspace_bytes, hip_stream);
}

vrn_status vrn_render_noalloc(vrn_ctx* ctx, vrn_field_id field, const vrn_camera* d_cams, uint32_t n_cams,
                              uint32_t W, uint32_t H, const vrn_render_opts* opts, float* d_rgba,
                              uint32_t* d_nsamples, void* hip_stream) {
  if (!ctx) return fail(VRN_ERR_INVALID_ARG, "ctx is NULL");
  if (!d_cams) return fail(VRN_ERR_INVALID_ARG, "cameras are NULL");
  if (!d_rgba) return fail(VRN_ERR_INVALID_ARG, "d_rgba is NULL");
  // the scratch holds the counters of one render of any size; requests
  // beyond the render limits are refused before anything is enqueued
  if (n_cams < 1 || n_cams > (uint32_t)kMaxCams)
    return fail(VRN_ERR_INVALID_ARG, "n_cams must be 1..16 (the scratch serves one render of at most 16 cameras)");
  if (W < 1 || H < 1 || W > 16384 || H > 16384 || (uint64_t)n_cams * W * H > (1ull << 31))
    return fail(VRN_ERR_INVALID_ARG, "W and H must be 1..16384 with at most 2^31 pixels in one call");
  vrn_status st = check_opts(opts);
  if (st != VRN_OK) return st;
  std::lock_guard<std::mutex> lock(ctx->mu);
  Field* f = find_field(ctx, field);
  if (!f) return fail(VRN_ERR_NOT_FOUND, "unknown field id");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // counters start at zero: a fill kernel, not a memset (safe under capture)
  if ((e = launch_zero(ctx->scratch, kScratchBytes, s)) != hipSuccess) return hip_fail(e, "scratch clear");
  return do_render(ctx, f, d_cams, n_cams, W, H, opts, d_rgba, d_nsamples, ctx->scratch, s, true);
}

vrn_status vrn_read_stats(vrn_ctx* ctx, const void* ws, vrn_stats* out, void* stream) {
  if (!ctx || !out) return fail(VRN_ERR_INVALID_ARG, "ctx or out is NULL");
  std::lock_guard<std::mutex> lock(ctx->mu);
  hipSetDevice(ctx->device);
  const uint8_t* w = static_cast<const uint8_t*>(ws ? ws : ctx->ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint64_t v[6];
  hipError_t e = hipMemcpyAsync(v, w + kWsStats, sizeof(v), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "stats read");
  out->rays = v[0];
  out->samples = v[1];
  out->level_fetches = v[2];
  out->march_steps = v[3];
  out->rounds = v[4];
  out->tiles = v[5];
  return VRN_OK;
}

vrn_status vrn_rays(vrn_ctx* ctx, const vrn_camera* cams, uint32_t n_cams, uint32_t W, uint32_t H,
                    float scale, float* d_o, float* d_d, float* d_r, void* stream) {
  Range range("vrn_rays");
  if (!ctx || !d_o || !d_d || !d_r) return fail(VRN_ERR_INVALID_ARG, "NULL argument");
  vrn_status st = check_cams(cams, n_cams, W, H);
  if (st != VRN_OK) return st;
  if (!finite(scale) || !(scale > 0.0f)) return fail(VRN_ERR_INVALID_ARG, "scale must be > 0");
  std::lock_guard<std::mutex> lock(ctx->mu);
  hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t* slot = static_cast<uint8_t*>(ctx->ws) + kWsCams;
  hipError_t e = hipMemcpyAsync(slot, cams, n_cams * sizeof(vrn_camera), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_rays(reinterpret_cast<const vrn_camera*>(slot), n_cams, W, H, scale, d_o, d_d, d_r, s);
  return e == hipSuccess ? VRN_OK : hip_fail(e, "rays");
}

vrn_status vrn_march(vrn_ctx* ctx, vrn_field_id field, const vrn_camera* cams, uint32_t n_cams, uint32_t W,
                     uint32_t H, uint32_t* d_klist, uint32_t max_k, uint32_t* d_count, void* stream) {
  Range range("vrn_march");
  if (!ctx || !d_count || (max_k > 0 && !d_klist)) return fail(VRN_ERR_INVALID_ARG, "NULL argument");
  vrn_status st = check_cams(cams, n_cams, W, H);
  if (st != VRN_OK) return st;
  std::lock_guard<std::mutex> lock(ctx->mu);
  Field* f = find_field(ctx, field);
  if (!f) return fail(VRN_ERR_NOT_FOUND, "unknown field id");
  hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t* slot = static_cast<uint8_t*>(ctx->ws) + kWsCams;
  hipError_t e = hipMemcpyAsync(slot, cams, n_cams * sizeof(vrn_camera), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_march(f->dev, reinterpret_cast<const vrn_camera*>(slot), n_cams, W, H, d_klist, max_k, d_count, s);
  if (e != hipSuccess) return hip_fail(e, "march");
  track(f, s);
  return VRN_OK;
}

vrn_status vrn_encode(vrn_ctx* ctx, vrn_field_id field, const float* d_xyz, const float* d_t, const float* d_r,
                      uint32_t n, float* d_feat, void* stream) {
  Range range("vrn_encode");
  if (!ctx || !d_xyz || !d_feat) return fail(VRN_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lock(ctx->mu);
  Field* f = find_field(ctx, field);
  if (!f) return fail(VRN_ERR_NOT_FOUND, "unknown field id");
  if (f->dev.lod && (!d_t || !d_r)) return fail(VRN_ERR_INVALID_ARG, "LOD fields need d_t and d_r");
  if (n == 0) return VRN_OK;
  hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_encode(f->dev, d_xyz, d_t, d_r, n, d_feat, s);
  if (e != hipSuccess) return hip_fail(e, "encode");
  track(f, s);
  return VRN_OK;
}

vrn_status vrn_mlp(vrn_ctx* ctx, vrn_field_id field, const float* d_feat, const float* d_dir, uint32_t n,
                   vrn_dtype compute, float* d_sigma, float* d_rgb, void* stream) {
  Range range("vrn_mlp");
  if (!ctx || !d_feat || !d_dir || !d_sigma || !d_rgb) return fail(VRN_ERR_INVALID_ARG, "NULL argument");
  if (compute != VRN_F32 && compute != VRN_F16 && compute != VRN_BF16 && compute != VRN_F32X)
    return fail(VRN_ERR_INVALID_ARG, "compute must be VRN_F32, VRN_F16, VRN_BF16 or VRN_F32X");
  std::lock_guard<std::mutex> lock(ctx->mu);
  Field* f = find_field(ctx, field);
  if (!f) return fail(VRN_ERR_NOT_FOUND, "unknown field id");
  if (n == 0) return VRN_OK;
  hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_mlp(f->dev, d_feat, d_dir, n, (int)compute, d_sigma, d_rgb, s);
  if (e != hipSuccess) return hip_fail(e, "mlp");
  track(f, s);
  return VRN_OK;
}

vrn_status vrn_prune_grid(vrn_ctx* ctx, vrn_field_id field, float alpha, uint32_t points_per_voxel,
                          vrn_dtype compute, uint32_t* d_bits_out, float* d_max_opacity, void* stream) {
  Range range("vrn_prune_grid");
  if (!ctx || !d_bits_out) return fail(VRN_ERR_INVALID_ARG, "ctx or d_bits_out is NULL");
  if (!finite(alpha) || alpha < 0.0f || alpha > 1.0f) return fail(VRN_ERR_INVALID_ARG, "alpha must be in [0, 1]");
  if (points_per_voxel != 4 && points_per_voxel != 1 && points_per_voxel != 8 && points_per_voxel != 27 &&
      points_per_voxel != 64)
    return fail(VRN_ERR_UNSUPPORTED, "points_per_voxel must be 4 or a cube 1, 8, 27, 64");
  if (compute != VRN_F32 && compute != VRN_F16 && compute != VRN_BF16 && compute != VRN_F32X)
    return fail(VRN_ERR_INVALID_ARG, "compute must be VRN_F32, VRN_F16, VRN_BF16 or VRN_F32X");
  std::lock_guard<std::mutex> lock(ctx->mu);
  Field* f = find_field(ctx, field);
  if (!f) return fail(VRN_ERR_NOT_FOUND, "unknown field id");
  hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_prune(f->dev, alpha, points_per_voxel, (int)compute, d_bits_out, d_max_opacity, ctx->n_cu, s);
  if (e != hipSuccess) return hip_fail(e, "prune");
  track(f, s);
  return VRN_OK;
}

vrn_status vrn_debug_counters(vrn_ctx* ctx, uint64_t out[6], int reset) {
  if (!ctx || !out) return fail(VRN_ERR_INVALID_ARG, "ctx or out is NULL");
  std::lock_guard<std::mutex> lock(ctx->mu);
  hipSetDevice(ctx->device);
  hipError_t e = hipDeviceSynchronize();
  unsigned long long v[kDbgSlots] = {};
  if (e == hipSuccess) e = debug_counters(v, reset != 0);
  if (e == hipErrorNotSupported) return fail(VRN_ERR_UNSUPPORTED, "library built without VRN_DEBUG_CHECKS");
  if (e != hipSuccess) return hip_fail(e, "debug counters");
  for (int i = 0; i < kDbgSlots; ++i) out[i] = v[i];
  return VRN_OK;
}

vrn_status vrn_phase_cycles(vrn_ctx* ctx, uint64_t out[6], int reset) {
  if (!ctx || !out) return fail(VRN_ERR_INVALID_ARG, "ctx or out is NULL");
  std::lock_guard<std::mutex> lock(ctx->mu);
  hipSetDevice(ctx->device);
  hipError_t e = hipDeviceSynchronize();
  unsigned long long v[kPhaseSlots] = {};
  if (e == hipSuccess) e = phase_cycles(v, reset != 0);
  if (e == hipErrorNotSupported) return fail(VRN_ERR_UNSUPPORTED, "library built without VRN_PHASE_TIMING");
  if (e != hipSuccess) return hip_fail(e, "phase cycles");
  for (int i = 0; i < kPhaseSlots; ++i) out[i] = v[i];
  return VRN_OK;
}

vrn_status vrn_set_occupancy(vrn_ctx* ctx, vrn_field_id field, const uint32_t* d_bits, void* stream) {
  Range range("vrn_set_occupancy");
  if (!ctx || !d_bits) return fail(VRN_ERR_INVALID_ARG, "ctx or d_bits is NULL");
  std::lock_guard<std::mutex> lock(ctx->mu);
  Field* f = find_field(ctx, field);
  if (!f) return fail(VRN_ERR_NOT_FOUND, "unknown field id");
  hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_set_occupancy(f->dev, d_bits, s);
  if (e != hipSuccess) return hip_fail(e, "set occupancy");
  track(f, s);
  return VRN_OK;
}

}  // extern "C"
