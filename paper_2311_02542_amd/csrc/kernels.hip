// Kernels of the renderer hot path and their launchers.
//
// render_kernel is the whole per-ray path in one launch (the paper's
// single-kernel interleave of ray marching, hash sampling and MLPs, Sec. 5):
// persistent waves own 64 rays each (one per lane); every round a wave
//   1. refills lanes whose ray finished from a per-XCD queue of 8x8 pixel
//      tiles (XCD-aware: block b works the image slice of XCD b % 8 first,
//      so each XCD's L2 sees one coherent region of the frame);
//   2. marches every ray to its next occupied lattice sample (bounded
//      number of lattice tests per round, coarse empty blocks skipped);
//   3. compacts the lanes that found a sample into 16-sample tiles and, per
//      tile, encodes the hash grid (4 lanes per sample, levels interleaved
//      so LOD-skipped fine levels idle all lane groups equally) and runs the
//      density and color MLPs on MFMA with the activations in registers;
//   4. composites in FP32 and retires rays at T < t_min, at the sample cap
//      or when the march leaves the grid, writing RGBA and sample counts.
// Counters in the workspace return to zero when the last block finishes, so
// the launch needs no memset and can be replayed from a HIP graph.
#include <map>
#include <mutex>
#include <type_traits>

#include "device.hpp"

namespace vrn {

#ifdef VRN_DEBUG_CHECKS
__device__ unsigned long long vrn_debug_counts[kDbgSlots];
#endif

constexpr uint32_t kNone = 0xFFFFFFFFu;

#ifdef VRN_PHASE_TIMING
__device__ unsigned long long vrn_phase_cycles[kPhaseSlots];
#define VRN_PHASE_START()                              \
  unsigned long long ph_[kPhaseSlots] = {};            \
  unsigned long long tph_ = __builtin_amdgcn_s_memtime()
#define VRN_PHASE(slot)                                               \
  do {                                                                \
    const unsigned long long tn_ = __builtin_amdgcn_s_memtime();     \
    ph_[(slot)] += tn_ - tph_;                                        \
    tph_ = tn_;                                                       \
  } while (0)
#define VRN_PHASE_FLUSH()                                                                  \
  do {                                                                                     \
    if (lane_id() == 0)                                                                    \
      for (int i_ = 0; i_ < kPhaseSlots; ++i_) atomicAdd(&vrn_phase_cycles[i_], ph_[i_]); \
  } while (0)
#else
#define VRN_PHASE_START() \
  do {                    \
  } while (0)
#define VRN_PHASE(slot) \
  do {                  \
  } while (0)
#define VRN_PHASE_FLUSH() \
  do {                    \
  } while (0)
#endif

// exp for compositing: the FP32 path keeps the library expf; the 16-bit
// paths, whose inputs carry FP16 rounding already, use the hardware
// exponential (one multiply and v_exp_f32).
template <bool FAST>
__device__ __forceinline__ float comp_exp(float z) {
  if constexpr (FAST) return __expf(z);
  else return expf(z);
}

template <bool FAST>
__device__ __forceinline__ float sigmoidf(float z) { return __builtin_amdgcn_rcpf(1.0f + comp_exp<FAST>(-z)); }

// MLP arithmetic of a compute mode: 0 FP32 MFMA, 1 FP16, 2 BF16, 3 FP32 by
// split BF16 (VRN_F32X).  Modes 0 and 3 share everything but the MLP: the
// FP32 encode, FP32 SH values and the library exp in compositing.
template <int MODE>
constexpr bool kF32Class = MODE == 0 || MODE == 3;

// Bytes of the split weights of mode 3 in LDS: three BF16 parts, then the
// FP32 fragments of the color output layer (run on the VALU).
constexpr int kX3Bytes = 3 * kW16Total * 2;

template <int MODE>
struct WeightSmem {
  static constexpr int kBytes =
      (MODE == 0) ? kW32Total * 4 : (MODE == 3 ? kX3Bytes + (kW32Total - kW32_C3) * 4 : kW16Total * 2);
};

template <int MODE>
__device__ __forceinline__ const uint4* weight_src(const FieldDev& F) {
  if constexpr (MODE == 0) return reinterpret_cast<const uint4*>(F.w32);
  else if constexpr (MODE == 1) return reinterpret_cast<const uint4*>(F.w16);
  else if constexpr (MODE == 2) return reinterpret_cast<const uint4*>(F.wbf);
  else return reinterpret_cast<const uint4*>(F.wx3);
}

template <int MODE>
__device__ __forceinline__ void load_weights(const FieldDev& F, uint8_t* s_w, float* s_b) {
  const uint4* src = weight_src<MODE>(F);
  uint4* dst = reinterpret_cast<uint4*>(s_w);
  constexpr int kMain = MODE == 3 ? kX3Bytes : WeightSmem<MODE>::kBytes;
  for (int i = threadIdx.x; i < kMain / 16; i += blockDim.x) dst[i] = src[i];
  if constexpr (MODE == 3) {
    const uint4* c3 = reinterpret_cast<const uint4*>(F.w32 + kW32_C3);
    for (int i = threadIdx.x; i < (kW32Total - kW32_C3) / 4; i += blockDim.x) dst[kX3Bytes / 16 + i] = c3[i];
  }
  for (int i = threadIdx.x; i < kBiasTotal; i += blockDim.x) s_b[i] = F.bias[i];
}

template <int MODE>
__device__ __forceinline__ void run_mlp(const uint8_t* s_w, const float* s_b, const FieldDev& F,
                                        const float feat[8], const float shs[4], int lane, float& o0,
                                        float lg[3]) {
  if constexpr (MODE == 0)
    mlp_tile_f32(reinterpret_cast<const float4*>(s_w), s_b, F.d1_ksteps / 4, feat, shs, lane, o0, lg);
  else if constexpr (MODE == 3)
    mlp_tile_x3(reinterpret_cast<const uint4*>(s_w), reinterpret_cast<const float4*>(s_w + kX3Bytes), s_b, feat,
                shs, lane, o0, lg);
  else
    mlp_tile_16<MODE == 2>(reinterpret_cast<const uint4*>(s_w), s_b, feat, Half8<MODE == 2>::pack4(shs), lane,
                           o0, lg);
}

// Stage the coarse occupancy grid and its dilation into LDS ([kCoarseWords]
// words each).
__device__ __forceinline__ void load_coarse(const FieldDev& F, uint32_t* s_coarse) {
  const uint32_t words = (F.Gc * F.Gc * F.Gc + 31u) / 32u;
  for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) {
    s_coarse[i] = F.coarse[i];
    s_coarse[kCoarseWords + i] = F.coarse_dil[i];
  }
}

// The lane that owns compacted sample s = 16 t + (lane & 15), from the
// wave's slot table in LDS.
__device__ __forceinline__ int tile_source(const uint32_t* s_slot_w, int ns, int t, int lane, bool& act) {
  const int s = t * 16 + (lane & 15);
  act = s < ns;
  return act ? (int)s_slot_w[s] : lane;
}

// Gather a compacted sample's position and LOD level from its owner lane and
// encode it (4 lanes per sample, one level group each).
template <bool TAB16, bool PRECISE>
__device__ __forceinline__ void tile_encode(const FieldDev& F, const LevelDev* s_lv, __amdgpu_buffer_rsrc_t tab,
                                            int src, bool act, int lane, const float sx[3], float slst,
                                            float feat[8], uint32_t& fetches) {
  const float px[3] = {shfl_f(sx[0], src), shfl_f(sx[1], src), shfl_f(sx[2], src)};
  const float lstar = shfl_f(slst, src);
  encode_point<TAB16, PRECISE>(F, s_lv, tab, px, lstar, act, lane >> 4, feat, fetches);
}

// Per-ray SH values in FP32 for the FP32 path, laid out [lane][group g][i]
// with c = g + 4 i: a tile's lane group reads its four values in one 16-byte
// LDS load instead of evaluating all 16 polynomials of its sample's ray.
__device__ __forceinline__ void store_ray_sh_f32(const FieldDev& F, const Ray& r, float4* s_sh_lane) {
  float s[16];
  sh_basis16(r.dx, r.dy, r.dz, s);
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = (uint32_t)(g + 4 * i) < F.nsh ? s[g + 4 * i] : 0.0f;
    s_sh_lane[g] = make_float4(v[0], v[1], v[2], v[3]);
  }
}

// Per-ray SH values in the MFMA element type, laid out [lane][group g][c = g + 4 i].
template <bool BF>
__device__ __forceinline__ void store_ray_sh(const FieldDev& F, const Ray& r, uint2* s_sh_lane) {
  float s[16];
  sh_basis16(r.dx, r.dy, r.dz, s);
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = (uint32_t)(g + 4 * i) < F.nsh ? s[g + 4 * i] : 0.0f;
    s_sh_lane[g] = Half8<BF>::pack4(v);
  }
}

// Waves per SIMD the 16-bit kernels are compiled for (register budget
// 512 / waves).  4 measured fastest on the stereo C4 frame; 3 would let two
// tiles share each weight read but loses the latency cover of a fourth wave.
#ifndef VRN_WAVES16
#define VRN_WAVES16 4
#endif

template <bool TAB16, int MODE, int GEO>
__global__ __launch_bounds__(kF32Class<MODE> ? kBlockF32 : kBlock, kF32Class<MODE> ? 4 : VRN_WAVES16) void render_kernel(
    RenderArgs A) {
  constexpr int kThreads = kF32Class<MODE> ? kBlockF32 : kBlock;
  __shared__ __align__(16) uint8_t s_w[WeightSmem<MODE>::kBytes];
  __shared__ float s_b[kBiasTotal];
  __shared__ LevelDev s_lv[kMaxLevels];
  __shared__ uint32_t s_coarse[2 * kCoarseWords];
  __shared__ uint32_t s_off[kMaxCams + 1];
  __shared__ uint32_t s_rb[kMaxCams], s_re[kMaxCams];
  __shared__ uint32_t s_stats[6];
  // per-ray SH values: FP32 [lane][g] float4 (FP32 path) or packed 16-bit [lane][g] uint2
  __shared__ __align__(16) uint8_t s_sh_raw[kThreads * 4 * (kF32Class<MODE> ? 16 : 8)];
  uint2* s_sh = reinterpret_cast<uint2*>(s_sh_raw);
  float4* s_sh4 = reinterpret_cast<float4*>(s_sh_raw);
  __shared__ uint32_t s_slot[kThreads];

  const FieldDev& F = A.F;
  const __amdgpu_buffer_rsrc_t tab = table_rsrc(F);
  load_weights<MODE>(F, s_w, s_b);
  load_coarse(F, s_coarse);
  if (threadIdx.x < F.L) s_lv[threadIdx.x] = F.levels[threadIdx.x];
  if (threadIdx.x < 6) s_stats[threadIdx.x] = 0;
  const uint32_t tx = (A.W + kTile - 1) / kTile;
  const float inv_tx = 1.0f / (float)tx;
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (uint32_t c = 0; c < A.n_cams; ++c) {
      const uint32_t rb = min(A.cams[c].row_begin, A.H);
      const uint32_t re = min(max(A.cams[c].row_end, rb), A.H);
      s_off[c] = acc;
      s_rb[c] = rb;
      s_re[c] = re;
      acc += tx * ((re - rb + kTile - 1) / kTile) * (kTile * kTile);
    }
    s_off[A.n_cams] = acc;
  }
  __syncthreads();

  const int lane = lane_id();
  const uint32_t n_tiles = s_off[A.n_cams] / (kTile * kTile);
  uint32_t* ctrl = reinterpret_cast<uint32_t*>(A.ws + kWsQueue);
  int q = (int)(blockIdx.x % kQueues);
  int q_tried = 0;
  bool out_of_work = false;

  Ray r;
  r.k = 0;
  r.k_hi = -1;
  r.lr = 0.0f;
  r.brick = -1;
  r.blo = r.bhi = 0u;
  r.delta = 0.0f;
  r.ox = r.oy = r.oz = r.dx = r.dy = r.dz = 0.0f;
  uint32_t pix = kNone, n = 0;
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
  uint32_t st_steps = 0, st_fetch = 0, st_samples = 0, st_rays = 0, st_rounds = 0, st_tiles = 0;

  VRN_PHASE_START();
  auto retire = [&]() {
    float4 v = make_float4(cr, cg, cb, 1.0f - T);
    if (A.output != VRN_OUT_PQ) {
      v.x = pq_to_linear(v.x);
      v.y = pq_to_linear(v.y);
      v.z = pq_to_linear(v.z);
      if (A.output == VRN_OUT_SRGB) {
        v.x = srgb_oetf(v.x * A.exposure);
        v.y = srgb_oetf(v.y * A.exposure);
        v.z = srgb_oetf(v.z * A.exposure);
      }
    }
    VRN_DEBUG_COUNT((uint64_t)pix >= (uint64_t)A.n_cams * A.H * A.W, kDbgPixel);
    reinterpret_cast<float4*>(A.rgba)[pix] = v;
    if (A.nsamples) A.nsamples[pix] = n;
    ++st_rays;
    pix = kNone;
  };

  while (true) {
    // keep LDS reads of weights inside the loop (hoisting would pin the
    // weights in registers and drop occupancy to one wave per SIMD)
    asm volatile("" ::: "memory");
    VRN_PHASE(kPhComposite);
    // ---- 1. refill lanes that have no ray -------------------------------
    while (!out_of_work) {
      const uint64_t need = __ballot(pix == kNone);
      if (need == 0) break;
      const int cnt = __popcll(need);
      const int leader = __ffsll((unsigned long long)need) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(&ctrl[q * 16], (uint32_t)cnt);
      base = (uint32_t)shfl_i((int)base, leader);
      const uint32_t qb = (uint32_t)((uint64_t)n_tiles * q / kQueues) * (kTile * kTile);
      const uint32_t qe = (uint32_t)((uint64_t)n_tiles * (q + 1) / kQueues) * (kTile * kTile);
      if (pix == kNone) {
        const int rank = __popcll(need & ((1ull << lane) - 1ull));
        const uint32_t id = qb + base + (uint32_t)rank;
        if (id < qe) {
          uint32_t c = 0;
          while (c + 1 < A.n_cams && id >= s_off[c + 1]) ++c;
          const uint32_t local = id - s_off[c];
          const uint32_t tile = local / (kTile * kTile), within = local % (kTile * kTile);
          // tile / tx without an integer division: float quotient, then an
          // exact integer correction (tile < 2^24)
          uint32_t ty = (uint32_t)((float)tile * inv_tx);
          if (ty * tx > tile) --ty;
          else if ((ty + 1) * tx <= tile) ++ty;
          const uint32_t col = (tile - ty * tx) * kTile + within % kTile;
          const uint32_t row = s_rb[c] + ty * kTile + within / kTile;
          if (col < A.W && row < s_re[c]) {
            setup_ray<GEO>(F, A.cams[c], col, row, r);
            if constexpr (!kF32Class<MODE>) store_ray_sh<MODE == 2>(F, r, &s_sh[threadIdx.x * 4]);
            else store_ray_sh_f32(F, r, &s_sh4[threadIdx.x * 4]);
            pix = (c * A.H + row) * A.W + col;
            T = 1.0f;
            cr = cg = cb = 0.0f;
            n = 0;
          }
        }
      }
      if (qb + base + (uint32_t)cnt >= qe) {
        q = (q + 1) % kQueues;
        if (++q_tried >= kQueues) out_of_work = true;
      }
    }
    VRN_PHASE(kPhRefill);
    if (__ballot(pix != kNone) == 0) break;
    __builtin_amdgcn_wave_barrier();

    // ---- 2. march to the next evaluated sample ---------------------------
    int mres = 0;
    float st = 0.0f, sx[3] = {0.0f, 0.0f, 0.0f}, slst = 0.0f, sdt = F.dt;
    if (pix != kNone) {
      mres = march_next<GEO>(F, s_coarse, r, A.budget, st_steps, st, sx);
      if (mres == 2) retire();
      if (mres == 1) {
        if (F.lod) slst = (GEO == 1 && F.contract) ? level_star_contracted(F, r, st, sx) : level_star(F, st, r.lr);
        sdt = sample_step<GEO>(F, st);
      }
    }
    const bool has = mres == 1;
    const uint64_t m = __ballot(has);
    const int ns = __popcll(m);
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    const int nt = (ns + 15) >> 4;
    const int wave_base = (threadIdx.x >> 6) << 6;
    if (has) s_slot[wave_base + rank] = (uint32_t)lane;
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
      ++st_rounds;
      st_tiles += (uint32_t)nt;
    }

    VRN_PHASE(kPhMarch);
    // ---- 3. encode + MLP of the compacted samples -------------------------
    float so0 = 0.0f, sl0 = 0.0f, sl1 = 0.0f, sl2 = 0.0f;
    if constexpr (kF32Class<MODE>) {
      for (int t = 0; t < nt; ++t) {
        asm volatile("" ::: "memory");
        bool act;
        const int src = tile_source(&s_slot[wave_base], ns, t, lane, act);
        float feat[8], shs[4];
        tile_encode<TAB16, true>(F, s_lv, tab, src, act, lane, sx, slst, feat, st_fetch);
        {
          const float4 v = s_sh4[(wave_base + src) * 4 + (lane >> 4)];
          shs[0] = v.x;
          shs[1] = v.y;
          shs[2] = v.z;
          shs[3] = v.w;
        }
        VRN_PHASE(kPhEncode);
        float o0, lg[3];
        run_mlp<MODE>(s_w, s_b, F, feat, shs, lane, o0, lg);
        VRN_PHASE(kPhMlp);
        const int from = rank & 15;
        const float a0 = shfl_f(o0, from), a1 = shfl_f(lg[0], from);
        const float a2 = shfl_f(lg[1], from), a3 = shfl_f(lg[2], from);
        if (has && (rank >> 4) == t) {
          so0 = a0;
          sl0 = a1;
          sl1 = a2;
          sl2 = a3;
        }
        VRN_PHASE(kPhReturn);
      }
    } else {
      typedef Half8<MODE == 2> H;
      for (int t0 = 0; t0 < nt; t0 += kMlpBatch) {
        asm volatile("" ::: "memory");
        const int cnt = min(kMlpBatch, nt - t0);
        typename H::vec xin[kMlpBatch];
        uint2 shh[kMlpBatch];
#pragma unroll
        for (int t = 0; t < kMlpBatch; ++t)
          if (t < cnt) {
            bool act;
            const int src = tile_source(&s_slot[wave_base], ns, t0 + t, lane, act);
            if constexpr (TAB16 && MODE == 1) {
              const float px[3] = {shfl_f(sx[0], src), shfl_f(sx[1], src), shfl_f(sx[2], src)};
              uint32_t hf[4];
              encode_point_h2(F, s_lv, tab, px, shfl_f(slst, src), act, lane >> 4, hf, st_fetch);
              const uint4 u = make_uint4(hf[0], hf[1], hf[2], hf[3]);
              __builtin_memcpy(&xin[t], &u, 16);
            } else {
              float feat[8];
              tile_encode<TAB16, false>(F, s_lv, tab, src, act, lane, sx, slst, feat, st_fetch);
              xin[t] = H::pack(feat);
            }
            shh[t] = s_sh[(wave_base + src) * 4 + (lane >> 4)];
          }
        VRN_PHASE(kPhEncode);
        float o0[kMlpBatch], lg[kMlpBatch][3];
        // The 16-bit MFMA chain co-executes with other waves' VALU and gather
        // issue, so the batch runs at raised issue priority: its dependent
        // MFMAs then start as soon as their inputs are ready (0.5 % faster on
        // the stereo frame).  The FP32 MFMA does not co-execute and the FP32
        // path keeps the default priority (there the raise measured slower).
        __builtin_amdgcn_s_setprio(2);
        mlp_batch_16<MODE == 2, kMlpBatch>(reinterpret_cast<const uint4*>(s_w), s_b, cnt, xin, shh, lane, o0, lg);
        __builtin_amdgcn_s_setprio(0);
        VRN_PHASE(kPhMlp);
        const int from = rank & 15;
#pragma unroll
        for (int t = 0; t < kMlpBatch; ++t)
          if (t < cnt) {
            const float a0 = shfl_f(o0[t], from), a1 = shfl_f(lg[t][0], from);
            const float a2 = shfl_f(lg[t][1], from), a3 = shfl_f(lg[t][2], from);
            if (has && (rank >> 4) == t0 + t) {
              so0 = a0;
              sl0 = a1;
              sl1 = a2;
              sl2 = a3;
            }
          }
        VRN_PHASE(kPhReturn);
      }
    }

    // ---- 4. composite (FP32), terminate --------------------------------
    if (has) {
      VRN_DEBUG_COUNT(so0 != so0 || sl0 != sl0 || sl1 != sl1 || sl2 != sl2, kDbgMlpNaN);
      constexpr bool kFast = !kF32Class<MODE>;
      const float sd = comp_exp<kFast>(so0) * sdt;
      const float trans = comp_exp<kFast>(-sd);
      const float wgt = T * (1.0f - trans);
      cr = fmaf(wgt, sigmoidf<kFast>(sl0), cr);
      cg = fmaf(wgt, sigmoidf<kFast>(sl1), cg);
      cb = fmaf(wgt, sigmoidf<kFast>(sl2), cb);
      T = T * trans;
      ++n;
      ++st_samples;
      if (T < F.t_min || n >= F.max_samples) retire();
    }
  }

  VRN_PHASE(kPhRefill);
  VRN_PHASE_FLUSH();
  atomicAdd(&s_stats[0], st_rays);
  atomicAdd(&s_stats[1], st_samples);
  atomicAdd(&s_stats[2], st_fetch);
  atomicAdd(&s_stats[3], st_steps);
  atomicAdd(&s_stats[4], st_rounds);
  atomicAdd(&s_stats[5], st_tiles);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long* stats = reinterpret_cast<unsigned long long*>(A.ws + kWsStats);
    for (int i = 0; i < 6; ++i) atomicAdd(&stats[i], (unsigned long long)s_stats[i]);
    __threadfence();
    uint32_t* done = reinterpret_cast<uint32_t*>(A.ws + kWsDone);
    if (atomicAdd(done, 1u) == gridDim.x - 1) {
      for (int i = 0; i < kQueues; ++i) atomicExch(&ctrl[i * 16], 0u);
      atomicExch(done, 0u);
      __threadfence();
    }
  }
}

// ---------------------------------------------------------------------------
// stage kernels
// ---------------------------------------------------------------------------

__global__ void zero_kernel(uint32_t* p, uint64_t n_words) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_words;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void rays_kernel(const vrn_camera* cams, uint32_t n_cams, uint32_t W, uint32_t H, float scale,
                            float* o, float* d, float* rr) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= (uint64_t)n_cams * W * H) return;
  const uint32_t c = (uint32_t)(i / ((uint64_t)W * H));
  const uint32_t rem = (uint32_t)(i % ((uint64_t)W * H));
  const uint32_t row = rem / W, col = rem % W;
  float w[3], nn, dd[3];
  canonical_ray(cams[c], col, row, w, nn, dd);
  for (int a = 0; a < 3; ++a) {
    o[3 * i + a] = cams[c].c2w[4 * a + 3];
    d[3 * i + a] = dd[a];
  }
  rr[i] = cone_pitch(cams[c], w, nn, scale);
}

template <int GEO>
__global__ void march_kernel(FieldDev F, const vrn_camera* cams, uint32_t n_cams, uint32_t W, uint32_t H,
                             uint32_t* klist, uint32_t max_k, uint32_t* count) {
  __shared__ uint32_t s_coarse[2 * kCoarseWords];
  load_coarse(F, s_coarse);
  __syncthreads();
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= (uint64_t)n_cams * W * H) return;
  const uint32_t c = (uint32_t)(i / ((uint64_t)W * H));
  const uint32_t rem = (uint32_t)(i % ((uint64_t)W * H));
  Ray r;
  setup_ray<GEO>(F, cams[c], rem % W, rem / W, r);
  uint32_t cnt = 0, steps = 0;
  float st, sx[3];
  while (cnt < F.max_samples) {
    if (march_next<GEO>(F, s_coarse, r, 0x40000000u, steps, st, sx) != 1) break;
    if (cnt < max_k) klist[i * max_k + cnt] = (uint32_t)(r.k - 1);
    ++cnt;
  }
  count[i] = cnt;
}

template <bool TAB16>
__global__ __launch_bounds__(kBlock) void encode_kernel(FieldDev F, const float* xyz, const float* tt,
                                                        const float* rr, uint32_t n, float* feat) {
  __shared__ LevelDev s_lv[kMaxLevels];
  if (threadIdx.x < F.L) s_lv[threadIdx.x] = F.levels[threadIdx.x];
  __syncthreads();
  const int lane = lane_id(), g = lane >> 4;
  const uint64_t p = (blockIdx.x * (uint64_t)(kBlock / 64) + threadIdx.x / 64) * 16 + (lane & 15);
  const bool act = p < n;
  float x[3] = {0.0f, 0.0f, 0.0f}, lstar = 0.0f;
  if (act) {
    for (int a = 0; a < 3; ++a) x[a] = xyz[3 * p + a];
    if (F.lod) lstar = level_star(F, tt[p], logf(rr[p]) + F.lod_c);
  }
  float f[8];
  uint32_t fetches = 0;
  encode_point<TAB16, true>(F, s_lv, table_rsrc(F), x, lstar, act, g, f, fetches);
  if (!act) return;
  for (int j = 0; j < 4; ++j) {
    const int lev = g + 4 * j;
    if (lev < (int)F.L) {
      feat[p * (2 * F.L) + 2 * lev] = f[2 * j];
      feat[p * (2 * F.L) + 2 * lev + 1] = f[2 * j + 1];
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void mlp_kernel(FieldDev F, const float* feat, const float* dir,
                                                     uint32_t n, float* sigma, float* rgb) {
  __shared__ __align__(16) uint8_t s_w[WeightSmem<MODE>::kBytes];
  __shared__ float s_b[kBiasTotal];
  load_weights<MODE>(F, s_w, s_b);
  __syncthreads();
  const int lane = lane_id(), g = lane >> 4;
  const uint64_t p = (blockIdx.x * (uint64_t)(kBlock / 64) + threadIdx.x / 64) * 16 + (lane & 15);
  const bool act = p < n;
  float f[8], shs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int e = 0; e < 8; ++e) {
    const int lev = g + 4 * (e >> 1);
    f[e] = (act && lev < (int)F.L) ? feat[p * (2 * F.L) + 2 * lev + (e & 1)] : 0.0f;
  }
  const float dx = act ? dir[3 * p] : 0.0f, dy = act ? dir[3 * p + 1] : 0.0f,
              dz = act ? dir[3 * p + 2] : 0.0f;
  sh_select(F, dx, dy, dz, g, shs);
  float o0, lg[3];
  run_mlp<MODE>(s_w, s_b, F, f, shs, lane, o0, lg);
  if (act && g == 0) {
    sigma[p] = expf(o0);
    rgb[3 * p] = sigmoidf<false>(lg[0]);
    rgb[3 * p + 1] = sigmoidf<false>(lg[1]);
    rgb[3 * p + 2] = sigmoidf<false>(lg[2]);
  }
}

// ---------------------------------------------------------------------------
// grid pruning (Sec. 4.3, App. C): max opacity over points inside each
// occupied voxel, threshold alpha; pruning only clears bits.
//
// Three launches: (1) the output bits start as the field's occupancy (and
// the maximum opacity of every unoccupied voxel as NaN); (2) the non-empty
// 4x4x4 bricks are listed; (3) persistent waves walk that list (wave w takes
// entries w, w + n_waves, ...), queue each brick's occupied voxels in LDS,
// and evaluate them 64 voxels at a time -- 16-sample MFMA tiles of the
// voxels' points through the same encode and density layers as the
// renderer -- then clear the bits of voxels below alpha.  Only occupied
// voxels cost work, and the weights are staged once per resident block.
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool cell_occupied(const FieldDev& F, uint32_t x, uint32_t y, uint32_t z) {
  const uint32_t b = (x >> 2) + F.Gb * ((y >> 2) + F.Gb * (z >> 2));
  const unsigned long long w = F.bricks[b];
  return (w >> ((x & 3) + 4 * (y & 3) + 16 * (z & 3))) & 1ull;
}

// offsets of point i inside a voxel: 4 = tetrahedral corners of the 2x2x2
// sub-lattice at {1/4, 3/4}; otherwise a p^3 grid at (i + 1/2) / p
__device__ __forceinline__ float voxel_offset(uint32_t npts, uint32_t p, uint32_t i, int axis) {
  if (npts == 4) {
    const float q = 0.25f, t = 0.75f;
    const float tab[4][3] = {{q, q, q}, {t, t, q}, {t, q, t}, {q, t, t}};
    return tab[i & 3][axis];
  }
  const uint32_t c = axis == 0 ? i % p : (axis == 1 ? (i / p) % p : i / (p * p));
  return ((float)c + 0.5f) / (float)p;
}

// (1) one thread per 32-bit output word (G^3 < 2^31, so 32-bit indices)
__global__ void prune_init_kernel(FieldDev F, uint32_t* bits_out, float* max_op) {
  const uint32_t G = F.G;
  const uint32_t n = G * G * G;
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= (n + 31u) / 32u) return;
  const uint32_t i0 = w * 32u;
  uint32_t x = i0 % G, y = (i0 / G) % G, z = i0 / (G * G);
  if ((G & 31u) == 0u && !max_op) {
    // the word is one row of 32 cells at fixed (y, z): 4 cells from each of
    // 8 bricks, taken from the brick words directly
    const uint32_t shift = 4u * (y & 3u) + 16u * (z & 3u);
    const uint32_t b0 = (x >> 2) + F.Gb * ((y >> 2) + F.Gb * (z >> 2));
    uint32_t out = 0u;
#pragma unroll
    for (uint32_t k = 0; k < 8u; ++k) out |= (uint32_t)((F.bricks[b0 + k] >> shift) & 0xFull) << (4u * k);
    bits_out[w] = out;
    return;
  }
  uint32_t out = 0u;
  for (uint32_t j = 0; j < 32u && i0 + j < n; ++j) {
    if (cell_occupied(F, x, y, z)) out |= 1u << j;
    else if (max_op) max_op[i0 + j] = __builtin_nanf("");
    if (++x == G) {
      x = 0;
      if (++y == G) {
        y = 0;
        ++z;
      }
    }
  }
  bits_out[w] = out;
}

// (2) indices of the non-empty bricks, in any order (count zeroed before)
__global__ void brick_list_kernel(FieldDev F, uint32_t* list, uint32_t* count) {
  const uint32_t nb = F.Gb * F.Gb * F.Gb;
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  const bool nz = b < nb && F.bricks[b] != 0ull;
  const uint64_t m = __ballot(nz);
  if (m == 0) return;
  const int lane = lane_id();
  const int leader = __ffsll((unsigned long long)m) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(m));
  base = (uint32_t)shfl_i((int)base, leader);
  if (nz) list[base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = b;
}

// Density layers only (the pruning pass needs sigma, not color), in the
// renderer's fragment layout.  Lanes 0..15 return the density pre-activation
// o0 of samples 0..15.
__device__ __forceinline__ float density_tile_f32(const float4* __restrict__ sw, const float* __restrict__ sb,
                                                  uint32_t d1_groups, const float feat[8], int lane) {
  const int g = lane >> 4;
  v4f h[4];
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) h[ot] = bias_acc(sb, kB1 + 16 * ot, g);
#pragma unroll
  for (int s4 = 0; s4 < 2; ++s4) {
    if ((uint32_t)s4 < d1_groups) {
#pragma unroll
      for (int ot = 0; ot < 4; ++ot) {
        const float4 w = sw[kW32_D1 / 4 + (ot * 2 + s4) * 64 + lane];
        h[ot] = mfma_f32(w.x, feat[4 * s4 + 0], h[ot]);
        h[ot] = mfma_f32(w.y, feat[4 * s4 + 1], h[ot]);
        h[ot] = mfma_f32(w.z, feat[4 * s4 + 2], h[ot]);
        h[ot] = mfma_f32(w.w, feat[4 * s4 + 3], h[ot]);
      }
    }
  }
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) h[ot] = relu4(h[ot]);
  v4f o = zero4();
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const float4 w = sw[kW32_D2 / 4 + it * 64 + lane];
    o = mfma_f32(w.x, h[it][0], o);
    o = mfma_f32(w.y, h[it][1], o);
    o = mfma_f32(w.z, h[it][2], o);
    o = mfma_f32(w.w, h[it][3], o);
  }
  return o[0] + sb[kB2 + 4 * g];
}

template <bool BF>
__device__ __forceinline__ float density_tile_16(const uint4* __restrict__ sw, const float* __restrict__ sb,
                                                 const float feat[8], int lane) {
  typedef Half8<BF> H;
  typedef typename H::vec vec;
  const int g = lane >> 4;
  auto wfrag = [&](int off16, int idx) -> vec {
    const uint4 u = sw[off16 / 8 + idx * 64 + lane];
    vec v;
    __builtin_memcpy(&v, &u, 16);
    return v;
  };
  const vec xin = H::pack(feat);
  vec hp[2];
#pragma unroll
  for (int pair = 0; pair < 2; ++pair) {
    const v4f a = H::mfma(wfrag(kW16_D1, 2 * pair), xin, bias_acc(sb, kB1 + 32 * pair, g));
    const v4f b = H::mfma(wfrag(kW16_D1, 2 * pair + 1), xin, bias_acc(sb, kB1 + 32 * pair + 16, g));
    const float hv[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    hp[pair] = H::relu_pack(hv);
  }
  const v4f o = H::mfma(wfrag(kW16_D2, 1), hp[1], H::mfma(wfrag(kW16_D2, 0), hp[0], bias_acc(sb, kB2, g)));
  return o[0];
}

// Density layers by split BF16 (mode 3): the D1 and D2 fragments of each
// of the three parts, staged [part][kW16_C1].
__device__ __forceinline__ float density_tile_x3(const uint4* __restrict__ sw3, const float* __restrict__ sb,
                                                 const float feat[8], int lane) {
  const int g = lane >> 4;
  const Bf3 xin = split_bf3(feat);
  float hv[16];
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) {
    const v4f h = relu4(mfma_bf3(wfrag_bf3(sw3, kW16_C1, kW16_D1, ot, lane), xin, bias_acc(sb, kB1 + 16 * ot, g)));
#pragma unroll
    for (int r = 0; r < 4; ++r) hv[4 * ot + r] = h[r];
  }
  v4f o = mfma_bf3(wfrag_bf3(sw3, kW16_C1, kW16_D2, 0, lane), split_bf3(hv), zero4());
  o = mfma_bf3(wfrag_bf3(sw3, kW16_C1, kW16_D2, 1, lane), split_bf3(hv + 8), o);
  return o[0] + sb[kB2 + 4 * g];
}

// The density-layer weights (D1 and D2) are the first kW32_C1 / kW16_C1
// elements of each weight form (of each of the three parts in mode 3).
template <int MODE>
struct DensitySmem {
  static constexpr int kBytes = (MODE == 0) ? kW32_C1 * 4 : (MODE == 3 ? 3 * kW16_C1 * 2 : kW16_C1 * 2);
};

constexpr int kPruneQueue = 128;   // per-wave voxel queue: < 64 carried + one brick

// (3) persistent pruning waves over the brick list.  TET: 4 points per voxel.
template <bool TAB16, int MODE, bool TET>
__global__ __launch_bounds__(kBlock) void prune_kernel(FieldDev F, float alpha, uint32_t npts, uint32_t p,
                                                      const uint32_t* list, const uint32_t* count,
                                                      uint32_t* bits_out, float* max_op) {
  __shared__ __align__(16) uint8_t s_w[DensitySmem<MODE>::kBytes];
  __shared__ float s_b[kBiasTotal];
  __shared__ LevelDev s_lv[kMaxLevels];
  __shared__ uint32_t s_q[kBlock / 64][kPruneQueue];
  __shared__ uint32_t s_max[kBlock / 64][64];
  {
    const uint4* src = weight_src<MODE>(F);
    uint4* dst = reinterpret_cast<uint4*>(s_w);
    if constexpr (MODE == 3) {
      constexpr int kPart = kW16_C1 * 2 / 16;   // uint4 per part
      for (int i = threadIdx.x; i < 3 * kPart; i += blockDim.x)
        dst[i] = src[(i / kPart) * (kW16Total * 2 / 16) + i % kPart];
    } else {
      for (int i = threadIdx.x; i < DensitySmem<MODE>::kBytes / 16; i += blockDim.x) dst[i] = src[i];
    }
    for (int i = threadIdx.x; i < kBiasTotal; i += blockDim.x) s_b[i] = F.bias[i];
    if (threadIdx.x < F.L) s_lv[threadIdx.x] = F.levels[threadIdx.x];
  }
  __syncthreads();
  const __amdgpu_buffer_rsrc_t tab = table_rsrc(F);
  const int lane = lane_id(), g = lane >> 4, wv = threadIdx.x >> 6;
  uint32_t* q = s_q[wv];
  uint32_t* mx = s_max[wv];
  const uint32_t n_list = *count;
  const uint32_t n_waves = gridDim.x * (kBlock / 64);
  const uint32_t G = F.G, Gb = F.Gb;
  const float cell = F.inv_cs;
  int qn = 0;
  for (uint32_t i = blockIdx.x * (kBlock / 64) + (uint32_t)wv;; i += n_waves) {
    const bool more = i < n_list;
    if (more) {
      // queue the occupied voxels of one brick, packed x | y << 10 | z << 20
      const uint32_t b = list[i];
      const unsigned long long w = F.bricks[b];
      const uint32_t bx = b % Gb, by = (b / Gb) % Gb, bz = b / (Gb * Gb);
      if ((w >> lane) & 1ull) {
        const int rank = __popcll(w & ((1ull << lane) - 1ull));
        const uint32_t x = 4u * bx + ((uint32_t)lane & 3u), y = 4u * by + (((uint32_t)lane >> 2) & 3u),
                       z = 4u * bz + ((uint32_t)lane >> 4);
        q[qn + rank] = x | (y << 10) | (z << 20);
      }
      qn += __popcll(w);
    }
    __builtin_amdgcn_wave_barrier();
    while (qn >= 64 || (!more && qn > 0)) {
      asm volatile("" ::: "memory");
      const int V = qn < 64 ? qn : 64;
      mx[lane] = 0u;
      __builtin_amdgcn_wave_barrier();
      const int ns = V * (int)npts;
      for (int t = 0; t * 16 < ns; ++t) {
        asm volatile("" ::: "memory");
        const int s = t * 16 + (lane & 15);
        const bool act = s < ns;
        int vr = 0;
        uint32_t pi = 0;
        if (act) {
          if constexpr (TET) {
            vr = s >> 2;
            pi = (uint32_t)s & 3u;
          } else {
            vr = s / (int)npts;
            pi = (uint32_t)(s - vr * (int)npts);
          }
        }
        const uint32_t c = q[vr];
        const uint32_t cc[3] = {c & 1023u, (c >> 10) & 1023u, c >> 20};
        float x[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) x[a] = F.amin[a] + ((float)cc[a] + voxel_offset(npts, p, pi, a)) * cell;
        float feat[8];
        uint32_t fetches = 0;
        // every level weighs 1 (no ray, no LOD): L* above the finest level
        encode_point<TAB16, kF32Class<MODE>>(F, s_lv, tab, x, 1.0e9f, act, g, feat, fetches);
        float o0;
        if constexpr (MODE == 0)
          o0 = density_tile_f32(reinterpret_cast<const float4*>(s_w), s_b, F.d1_ksteps / 4, feat, lane);
        else if constexpr (MODE == 3)
          o0 = density_tile_x3(reinterpret_cast<const uint4*>(s_w), s_b, feat, lane);
        else
          o0 = density_tile_16<MODE == 2>(reinterpret_cast<const uint4*>(s_w), s_b, feat, lane);
        if (act && g == 0) {
          float op = 1.0f - expf(-expf(o0) * F.dt);
          // a NaN opacity (16-bit activations that overflowed) keeps the voxel
          if (!(op == op)) op = 1.0f;
          atomicMax(&mx[vr], __float_as_uint(fmaxf(op, 0.0f)));
        }
      }
      __builtin_amdgcn_wave_barrier();
      if (lane < V) {
        const uint32_t c = q[lane];
        const uint32_t idx = (c & 1023u) + G * (((c >> 10) & 1023u) + G * (c >> 20));
        const float m = __uint_as_float(mx[lane]);
        if (!(m >= alpha)) atomicAnd(&bits_out[idx >> 5], ~(1u << (idx & 31u)));
        if (max_op) max_op[idx] = m;
      }
      // drop the V evaluated voxels from the front of the queue
      const uint32_t tail = lane + V < qn ? q[lane + V] : 0u;
      __builtin_amdgcn_wave_barrier();
      if (lane + V < qn) q[lane] = tail;
      __builtin_amdgcn_wave_barrier();
      qn -= V;
    }
    if (!more) break;
  }
}

// Rebuild a resident field's bricks and coarse grid from linear bits.
__global__ void bricks_from_bits_kernel(FieldDev F, unsigned long long* bricks, const uint32_t* bits) {
  const uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t nb = (uint64_t)F.Gb * F.Gb * F.Gb;
  if (b >= nb) return;
  const uint32_t bx = (uint32_t)(b % F.Gb), by = (uint32_t)((b / F.Gb) % F.Gb), bz = (uint32_t)(b / ((uint64_t)F.Gb * F.Gb));
  unsigned long long w = 0ull;
  for (uint32_t i = 0; i < 64; ++i) {
    const uint32_t x = 4 * bx + (i & 3), y = 4 * by + ((i >> 2) & 3), z = 4 * bz + (i >> 4);
    if (x < F.G && y < F.G && z < F.G) {
      const uint64_t idx = x + (uint64_t)F.G * (y + (uint64_t)F.G * z);
      if ((bits[idx >> 5] >> (idx & 31)) & 1u) w |= 1ull << i;
    }
  }
  bricks[b] = w;
}

__global__ void coarse_from_bricks_kernel(FieldDev F, uint32_t* coarse) {
  const uint32_t word = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nc = F.Gc * F.Gc * F.Gc;
  if (word >= (nc + 31) / 32) return;
  const uint32_t per = 1u << (F.cshift - 2);   // bricks per coarse block and axis
  uint32_t out = 0u;
  for (uint32_t j = 0; j < 32; ++j) {
    const uint32_t c = word * 32 + j;
    if (c >= nc) break;
    const uint32_t cx = c % F.Gc, cy = (c / F.Gc) % F.Gc, cz = c / (F.Gc * F.Gc);
    bool any = false;
    for (uint32_t k = 0; k < per * per * per && !any; ++k) {
      const uint32_t bx = cx * per + k % per, by = cy * per + (k / per) % per, bz = cz * per + k / (per * per);
      if (bx < F.Gb && by < F.Gb && bz < F.Gb) any = F.bricks[bx + F.Gb * (by + F.Gb * bz)] != 0ull;
    }
    if (any) out |= 1u << j;
  }
  coarse[word] = out;
}

__global__ void dilate_coarse_kernel(FieldDev F, uint32_t* dil) {
  const uint32_t word = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t Gc = F.Gc, nc = Gc * Gc * Gc;
  if (word >= (nc + 31) / 32) return;
  uint32_t out = 0u;
  for (uint32_t j = 0; j < 32; ++j) {
    const uint32_t c = word * 32 + j;
    if (c >= nc) break;
    const int cx = (int)(c % Gc), cy = (int)((c / Gc) % Gc), cz = (int)(c / (Gc * Gc));
    bool any = false;
    for (int k = 0; k < 27 && !any; ++k) {
      const int x = cx + k % 3 - 1, y = cy + (k / 3) % 3 - 1, z = cz + k / 9 - 1;
      if (x < 0 || y < 0 || z < 0 || x >= (int)Gc || y >= (int)Gc || z >= (int)Gc) continue;
      const uint32_t i = (uint32_t)x + Gc * ((uint32_t)y + Gc * (uint32_t)z);
      any = (F.coarse[i >> 5] >> (i & 31u)) & 1u;
    }
    if (any) out |= 1u << j;
  }
  dil[word] = out;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <bool TAB16, int MODE, int GEO>
static int blocks_per_cu_impl() {
  static int cached = -1;
  if (cached < 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, render_kernel<TAB16, MODE, GEO>,
                                                     render_block_threads(MODE), 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    cached = nb;
  }
  return cached;
}

template <int GEO>
static int blocks_per_cu_geo(int table_f16, int compute) {
  if (table_f16) {
    if (compute == 0) return blocks_per_cu_impl<true, 0, GEO>();
    if (compute == 1) return blocks_per_cu_impl<true, 1, GEO>();
    if (compute == 3) return blocks_per_cu_impl<true, 3, GEO>();
    return blocks_per_cu_impl<true, 2, GEO>();
  }
  if (compute == 0) return blocks_per_cu_impl<false, 0, GEO>();
  if (compute == 1) return blocks_per_cu_impl<false, 1, GEO>();
  if (compute == 3) return blocks_per_cu_impl<false, 3, GEO>();
  return blocks_per_cu_impl<false, 2, GEO>();
}

int render_blocks_per_cu(const FieldDev& F, int compute) {
  return F.lat ? blocks_per_cu_geo<1>(F.table_f16, compute) : blocks_per_cu_geo<0>(F.table_f16, compute);
}

template <int GEO>
static void launch_render_geo(const RenderArgs& a, int compute, dim3 gr, dim3 bl, hipStream_t s) {
  if (a.F.table_f16) {
    if (compute == 0) hipLaunchKernelGGL((render_kernel<true, 0, GEO>), gr, bl, 0, s, a);
    else if (compute == 1) hipLaunchKernelGGL((render_kernel<true, 1, GEO>), gr, bl, 0, s, a);
    else if (compute == 3) hipLaunchKernelGGL((render_kernel<true, 3, GEO>), gr, bl, 0, s, a);
    else hipLaunchKernelGGL((render_kernel<true, 2, GEO>), gr, bl, 0, s, a);
  } else {
    if (compute == 0) hipLaunchKernelGGL((render_kernel<false, 0, GEO>), gr, bl, 0, s, a);
    else if (compute == 1) hipLaunchKernelGGL((render_kernel<false, 1, GEO>), gr, bl, 0, s, a);
    else if (compute == 3) hipLaunchKernelGGL((render_kernel<false, 3, GEO>), gr, bl, 0, s, a);
    else hipLaunchKernelGGL((render_kernel<false, 2, GEO>), gr, bl, 0, s, a);
  }
}

hipError_t launch_render(const RenderArgs& a, int compute, int grid, hipStream_t s) {
  const dim3 gr(grid), bl(render_block_threads(compute));
  if (a.F.lat) launch_render_geo<1>(a, compute, gr, bl, s);
  else launch_render_geo<0>(a, compute, gr, bl, s);
  return hipGetLastError();
}

template <bool TAB16, int MODE, bool TET>
static void launch_prune_impl(const FieldDev& F, float alpha, uint32_t npts, uint32_t p, const uint32_t* list,
                              const uint32_t* count, uint32_t* bits_out, float* max_op, int n_cu, hipStream_t s) {
  static int per_cu = -1;
  if (per_cu < 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, prune_kernel<TAB16, MODE, TET>, kBlock, 0) !=
            hipSuccess || nb < 1)
      nb = 1;
    per_cu = nb;
  }
  hipLaunchKernelGGL((prune_kernel<TAB16, MODE, TET>), dim3((unsigned)(per_cu * n_cu)), dim3(kBlock), 0, s, F,
                     alpha, npts, p, list, count, bits_out, max_op);
}

template <bool TAB16, int MODE>
static void launch_prune_mode(const FieldDev& F, float alpha, uint32_t npts, uint32_t p, const uint32_t* list,
                              const uint32_t* count, uint32_t* bits_out, float* max_op, int n_cu, hipStream_t s) {
  if (npts == 4) launch_prune_impl<TAB16, MODE, true>(F, alpha, npts, p, list, count, bits_out, max_op, n_cu, s);
  else launch_prune_impl<TAB16, MODE, false>(F, alpha, npts, p, list, count, bits_out, max_op, n_cu, s);
}

hipError_t launch_prune(const FieldDev& F, float alpha, uint32_t npts, int compute, uint32_t* bits_out,
                        float* max_op, int n_cu, hipStream_t s) {
  uint32_t p = 1;
  while ((p + 1) * (p + 1) * (p + 1) <= npts) ++p;
  const uint32_t n = F.G * F.G * F.G;
  const uint32_t words = (n + 31u) / 32u;
  hipLaunchKernelGGL(prune_init_kernel, dim3((words + 255u) / 256u), dim3(256), 0, s, F, bits_out, max_op);
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, F.brick_count, (uint64_t)1);
  const uint32_t nb = F.Gb * F.Gb * F.Gb;
  hipLaunchKernelGGL(brick_list_kernel, dim3((nb + 255u) / 256u), dim3(256), 0, s, F, F.brick_list,
                     F.brick_count);
  const uint32_t* list = F.brick_list;
  const uint32_t* cnt = F.brick_count;
  if (F.table_f16) {
    if (compute == 0) launch_prune_mode<true, 0>(F, alpha, npts, p, list, cnt, bits_out, max_op, n_cu, s);
    else if (compute == 1) launch_prune_mode<true, 1>(F, alpha, npts, p, list, cnt, bits_out, max_op, n_cu, s);
    else if (compute == 3) launch_prune_mode<true, 3>(F, alpha, npts, p, list, cnt, bits_out, max_op, n_cu, s);
    else launch_prune_mode<true, 2>(F, alpha, npts, p, list, cnt, bits_out, max_op, n_cu, s);
  } else {
    if (compute == 0) launch_prune_mode<false, 0>(F, alpha, npts, p, list, cnt, bits_out, max_op, n_cu, s);
    else if (compute == 1) launch_prune_mode<false, 1>(F, alpha, npts, p, list, cnt, bits_out, max_op, n_cu, s);
    else if (compute == 3) launch_prune_mode<false, 3>(F, alpha, npts, p, list, cnt, bits_out, max_op, n_cu, s);
    else launch_prune_mode<false, 2>(F, alpha, npts, p, list, cnt, bits_out, max_op, n_cu, s);
  }
  return hipGetLastError();
}

hipError_t launch_set_occupancy(const FieldDev& F, const uint32_t* bits, hipStream_t s) {
  const uint64_t nb = (uint64_t)F.Gb * F.Gb * F.Gb;
  hipLaunchKernelGGL(bricks_from_bits_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, F,
                     const_cast<unsigned long long*>(F.bricks), bits);
  const uint32_t words = (F.Gc * F.Gc * F.Gc + 31) / 32;
  hipLaunchKernelGGL(coarse_from_bricks_kernel, dim3((words + 255) / 256), dim3(256), 0, s, F,
                     const_cast<uint32_t*>(F.coarse));
  hipLaunchKernelGGL(dilate_coarse_kernel, dim3((words + 255) / 256), dim3(256), 0, s, F,
                     const_cast<uint32_t*>(F.coarse_dil));
  return hipGetLastError();
}

hipError_t phase_cycles(unsigned long long out[kPhaseSlots], bool reset) {
#ifdef VRN_PHASE_TIMING
  hipError_t e = hipMemcpyFromSymbol(out, HIP_SYMBOL(vrn_phase_cycles), sizeof(unsigned long long) * kPhaseSlots);
  if (e == hipSuccess && reset) {
    const unsigned long long zero[kPhaseSlots] = {};
    e = hipMemcpyToSymbol(HIP_SYMBOL(vrn_phase_cycles), zero, sizeof(zero));
  }
  return e;
#else
  (void)out;
  (void)reset;
  return hipErrorNotSupported;
#endif
}

hipError_t debug_counters(unsigned long long out[kDbgSlots], bool reset) {
#ifdef VRN_DEBUG_CHECKS
  hipError_t e = hipMemcpyFromSymbol(out, HIP_SYMBOL(vrn_debug_counts), sizeof(unsigned long long) * kDbgSlots);
  if (e == hipSuccess && reset) {
    const unsigned long long zero[kDbgSlots] = {};
    e = hipMemcpyToSymbol(HIP_SYMBOL(vrn_debug_counts), zero, sizeof(zero));
  }
  return e;
#else
  (void)out;
  (void)reset;
  return hipErrorNotSupported;
#endif
}

// ---------------------------------------------------------------------------
// scratch of the allocation-free render entry point (vrn_render_noalloc):
// the queue, blocks-done and statistics counters of one render, laid out as
// a workspace.  Every device the library runs on holds its own copy until
// the process ends.  Host code must never pass `scratch` itself to a kernel
// (in host code it is a stand-in, not a device address): it passes the
// address scratch_address() returns for the current device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device ordinal -> that device's copy of `scratch`
}  // namespace

hipError_t scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  // first call on this device (the caller made it current): take the
  // array's device address and clear the array once
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  if ((e = launch_zero(p, kScratchBytes, nullptr)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) return e;
  g_scratch_ptr.emplace(device, p);
  *out = p;
  return hipSuccess;
}

hipError_t launch_zero(void* p, uint64_t bytes, hipStream_t s) {
  const uint64_t words = bytes / 4;
  const int grid = (int)std::min<uint64_t>((words + 255) / 256, 1024);
  hipLaunchKernelGGL(zero_kernel, dim3(std::max(grid, 1)), dim3(256), 0, s,
                     reinterpret_cast<uint32_t*>(p), words);
  return hipGetLastError();
}

hipError_t launch_rays(const vrn_camera* d_cams, uint32_t n_cams, uint32_t W, uint32_t H, float scale,
                       float* o, float* d, float* r, hipStream_t s) {
  const uint64_t n = (uint64_t)n_cams * W * H;
  hipLaunchKernelGGL(rays_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d_cams, n_cams, W, H,
                     scale, o, d, r);
  return hipGetLastError();
}

hipError_t launch_march(const FieldDev& F, const vrn_camera* d_cams, uint32_t n_cams, uint32_t W,
                        uint32_t H, uint32_t* klist, uint32_t max_k, uint32_t* count, hipStream_t s) {
  const uint64_t n = (uint64_t)n_cams * W * H;
  if (F.lat)
    hipLaunchKernelGGL(march_kernel<1>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, F, d_cams, n_cams, W,
                       H, klist, max_k, count);
  else
    hipLaunchKernelGGL(march_kernel<0>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, F, d_cams, n_cams, W,
                       H, klist, max_k, count);
  return hipGetLastError();
}

hipError_t launch_encode(const FieldDev& F, const float* xyz, const float* t, const float* r, uint32_t n,
                         float* feat, hipStream_t s) {
  const uint64_t per_block = (kBlock / 64) * 16;
  const dim3 gr((unsigned)(((uint64_t)n + per_block - 1) / per_block)), bl(kBlock);
  if (F.table_f16) hipLaunchKernelGGL((encode_kernel<true>), gr, bl, 0, s, F, xyz, t, r, n, feat);
  else hipLaunchKernelGGL((encode_kernel<false>), gr, bl, 0, s, F, xyz, t, r, n, feat);
  return hipGetLastError();
}

hipError_t launch_mlp(const FieldDev& F, const float* feat, const float* dir, uint32_t n, int compute,
                      float* sigma, float* rgb, hipStream_t s) {
  const uint64_t per_block = (kBlock / 64) * 16;
  const dim3 gr((unsigned)(((uint64_t)n + per_block - 1) / per_block)), bl(kBlock);
  if (compute == 0) hipLaunchKernelGGL((mlp_kernel<0>), gr, bl, 0, s, F, feat, dir, n, sigma, rgb);
  else if (compute == 1) hipLaunchKernelGGL((mlp_kernel<1>), gr, bl, 0, s, F, feat, dir, n, sigma, rgb);
  else if (compute == 3) hipLaunchKernelGGL((mlp_kernel<3>), gr, bl, 0, s, F, feat, dir, n, sigma, rgb);
  else hipLaunchKernelGGL((mlp_kernel<2>), gr, bl, 0, s, F, feat, dir, n, sigma, rgb);
  return hipGetLastError();
}

}  // namespace vrn
