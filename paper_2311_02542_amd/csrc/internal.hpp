// Internal host/device structures shared by the kernels and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vrn.h"

namespace vrn {

constexpr int kMaxLevels = 16;
constexpr int kMaxCams = VRN_MAX_CAMS;
constexpr int kQueues = 8;          // one ray queue per XCD
constexpr int kTile = 8;            // rays are issued in 8x8 pixel tiles
constexpr int kBlock = 256;         // threads per render block (4 waves)
// The FP32-MLP render kernel runs blocks of 16 waves, one block per CU: its
// 40 KiB of weights in LDS are shared by all of them, which leaves room for
// every ray's 16 SH values in FP32 (64 KiB) at the 4 waves/SIMD its registers
// allow.
constexpr int kBlockF32 = 1024;
inline int render_block_threads(int compute) { return (compute == 0 || compute == 3) ? kBlockF32 : kBlock; }
constexpr int kHidden = 64;
constexpr int kCoarseWords = 1024;  // <= 32^3 bits of coarse occupancy in LDS
constexpr int kMlpBatch = 1;        // 16-sample tiles per 16-bit MLP call (weights read once per call)

// MFMA fragment layout of the MLP weights (see mlp_tile in device.hpp).
// FP32: [layer][out_tile][kstep/4][lane][4]; FP16/BF16: [layer][out_tile][kstep][lane][8].
constexpr int kW32_D1 = 0, kW32_D2 = 2048, kW32_C1 = 3072, kW32_C2 = 5120, kW32_C3 = 9216;
constexpr int kW32Total = 10240;    // floats
constexpr int kW16_D1 = 0, kW16_D2 = 2048, kW16_C1 = 3072, kW16_C2 = 5120, kW16_C3 = 9216;
constexpr int kW16Total = 10240;    // 16-bit values
// biases: b1[64] b2[16] b3[64] b4[64] b5[16 (3 used)]
constexpr int kB1 = 0, kB2 = 64, kB3 = 80, kB4 = 144, kB5 = 208, kBiasTotal = 224;

struct LevelDev {
  float top;         // N - 1: the largest base corner (N + 1 lattice points per axis)
  uint32_t dense;    // 1: index = x + y s + z s^2 with s = N + 1
  uint32_t bx, by, bz;  // per-axis multipliers times the entry size in bytes: (1, s, s^2) dense,
                        // hash primes otherwise (products taken mod 2^32)
  float s_hi;        // N / extent in FP32 (16-bit paths)
  uint32_t base;     // byte offset of the level's table
  float below_n;     // largest float below N (clamp of the lattice coordinate, 16-bit paths)
  double s64;        // N / extent in FP64 (FP32 paths)
  double top64;      // N - 1 in FP64
};
static_assert(sizeof(LevelDev) == 48, "LevelDev is three 16-byte LDS rows");

struct FieldDev {
  const void* tables;        // [L][T][2] fp32 or fp16
  const LevelDev* levels;    // [L]
  const unsigned long long* bricks;  // Gb^3 bricks of 4x4x4 cells, bit (x&3) + 4 (y&3) + 16 (z&3)
  const uint32_t* coarse;    // Gc^3 bits (Gc <= 32), block = 2^cshift cells; staged in LDS
  const uint32_t* coarse_dil;  // Gc^3 bits: 1 if the block or one of its 26 neighbours has an
                               // occupied cell; staged in LDS after the coarse grid
  const float* w32;          // kW32Total
  const uint16_t* w16;       // kW16Total fp16 bits
  const uint16_t* wbf;       // kW16Total bf16 bits
  const uint16_t* wx3;       // [3][kW16Total] bf16 bits: the exact three-part split of the FP32 weights
  const float* bias;         // kBiasTotal
  uint32_t L, log2T, Tmask, table_f16;
  uint32_t bmask;            // Tmask times the entry size in bytes (hash mask on byte offsets)
  uint32_t G, Gb, Gc, cshift, nsh;
  float amin[3], cs;         // cs = fp32(G / extent)
  float dt, t_min, extent, inv_ln_f;
  float inv_dt, inv_cs;      // approximate reciprocals for skip estimates
  uint32_t max_samples;
  int32_t lod;
  float lod_c;               // ln(2 s / extent)
  float lod_bias, lod_radius_scale;
  uint32_t dense_mask;       // bit l set: level l is stored densely
  // table lattice / contraction (GEO = 1 kernels)
  const float* lat;          // t_0 .. t_K (K + 1 entries), canonical FP32
  uint32_t lat_K;            // number of lattice samples
  float step_growth;         // table recurrence t_{k+1} = t_k + max(dt, step_growth t_k)
  float lat_tsw;             // first table entry whose step is the growth term (inf: none)
  float lat_ksw;             // its index
  float lat_inv_log;         // 1 / ln(1 + step_growth)
  int32_t contract;          // L-infinity contraction on
  float center[3], inv_radius, radius;
  float lod_c2;              // ln(2 s): LOD constant when the footprint is already normalised
  uint32_t d1_ksteps;        // FP32 k-steps of the first density layer
  uint32_t c1_ksteps;        // FP32 k-steps of the first color layer
  // grid pruning: the non-empty bricks, listed on the device by each
  // vrn_prune_grid call ([Gb^3] entries, count in its own 256-byte block)
  uint32_t* brick_list;
  uint32_t* brick_count;
};

// Workspace layout (bytes).  Counters are spaced 64 B apart.
constexpr int kWsQueue = 0;        // kQueues x u32 at stride 16 u32
constexpr int kWsDone = 512;       // u32 blocks-finished counter
constexpr int kWsStats = 576;      // 6 x u64: rays, samples, level fetches, march steps, rounds, tiles
constexpr int kWsCams = 640;       // kMaxCams x vrn_camera
constexpr int kWsBytes = 4096;
// The allocation-free entry point keeps a render's counters (queues, done,
// stats: everything below kWsCams) in a file-scope device array of this size.
constexpr int kScratchBytes = 1024;
static_assert(kScratchBytes >= kWsCams, "scratch holds every counter of a workspace");

struct RenderArgs {
  FieldDev F;
  const vrn_camera* cams;    // device
  uint32_t n_cams, W, H;
  float* rgba;               // [n_cams][H][W][4]
  uint32_t* nsamples;        // nullable
  uint8_t* ws;               // workspace
  int32_t output;            // vrn_output
  float exposure;            // 2^exposure_ev (VRN_OUT_SRGB)
  uint32_t budget;           // march steps per round
};

// launchers (kernels.hip)
// Debug builds (-DVRN_DEBUG_CHECKS) count, instead of trapping on, hash-table
// offsets outside their level, brick and coarse-grid indices outside the
// grid, framebuffer writes outside the frame and NaN features or MLP
// outputs; vrn_debug_counters reads the counts.  Release builds compile none
// of it.
enum DebugSlot { kDbgTableOffset = 0, kDbgBrick, kDbgCoarse, kDbgPixel, kDbgFeature, kDbgMlpNaN, kDbgSlots };
#ifdef VRN_DEBUG_CHECKS
extern __device__ unsigned long long vrn_debug_counts[kDbgSlots];
#define VRN_DEBUG_COUNT(cond, slot)                                 \
  do {                                                              \
    if (cond) atomicAdd(&vrn_debug_counts[(slot)], 1ull);           \
  } while (0)
#else
#define VRN_DEBUG_COUNT(cond, slot) \
  do {                              \
  } while (0)
#endif
// Copy (and optionally zero) the debug counters; hipErrorNotSupported in
// release builds.
hipError_t debug_counters(unsigned long long out[kDbgSlots], bool reset);

// Phase-timing builds (-DVRN_PHASE_TIMING) sum, over the waves of every
// render, the shader clocks (s_memtime) each wave spends in each step of its
// rounds; vrn_phase_cycles reads the sums.  Other builds compile none of it.
enum PhaseSlot { kPhRefill = 0, kPhMarch, kPhEncode, kPhMlp, kPhReturn, kPhComposite, kPhaseSlots };
hipError_t phase_cycles(unsigned long long out[kPhaseSlots], bool reset);

hipError_t launch_render(const RenderArgs& a, int compute, int grid, hipStream_t s);
int render_blocks_per_cu(const FieldDev& F, int compute);
hipError_t launch_zero(void* p, uint64_t bytes, hipStream_t s);
// Device address of the allocation-free entry point's scratch array on
// `device`, which must be current: taken (and the array cleared) on the first
// call per device, then returned from a per-device cache.
hipError_t scratch_address(int device, void** out);
hipError_t launch_rays(const vrn_camera* d_cams, uint32_t n_cams, uint32_t W, uint32_t H,
                       float scale, float* o, float* d, float* r, hipStream_t s);
hipError_t launch_march(const FieldDev& F, const vrn_camera* d_cams, uint32_t n_cams, uint32_t W,
                        uint32_t H, uint32_t* klist, uint32_t max_k, uint32_t* count, hipStream_t s);
hipError_t launch_encode(const FieldDev& F, const float* xyz, const float* t, const float* r,
                         uint32_t n, float* feat, hipStream_t s);
hipError_t launch_prune(const FieldDev& F, float alpha, uint32_t npts, int compute, uint32_t* bits_out,
                        float* max_op, int n_cu, hipStream_t s);
hipError_t launch_set_occupancy(const FieldDev& F, const uint32_t* bits, hipStream_t s);
hipError_t launch_mlp(const FieldDev& F, const float* feat, const float* dir, uint32_t n,
                      int compute, float* sigma, float* rgb, hipStream_t s);

// Shared by the C ABI (capi.cpp) with the serving engine (server.cpp).
// set_error records vrn_last_error() for this thread and returns s.
vrn_status set_error(vrn_status s, const char* msg);
int ctx_device(const vrn_ctx* ctx);
// Pin (delta = +1) or unpin (-1) a resident field: vrn_unload_field refuses
// a pinned field, whose device pointers live on in captured graphs.
vrn_status field_pin(vrn_ctx* ctx, vrn_field_id field, int delta);

}  // namespace vrn
