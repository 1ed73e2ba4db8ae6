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
#include <type_traits>

#include "device.hpp"

namespace vrn {

constexpr uint32_t kNone = 0xFFFFFFFFu;

__device__ __forceinline__ float sigmoidf(float z) { return __builtin_amdgcn_rcpf(1.0f + expf(-z)); }

template <int MODE>
struct WeightSmem {
  static constexpr int kBytes = (MODE == 0) ? kW32Total * 4 : kW16Total * 2;
};

template <int MODE>
__device__ __forceinline__ const uint4* weight_src(const FieldDev& F) {
  if constexpr (MODE == 0) return reinterpret_cast<const uint4*>(F.w32);
  else if constexpr (MODE == 1) return reinterpret_cast<const uint4*>(F.w16);
  else return reinterpret_cast<const uint4*>(F.wbf);
}

template <int MODE>
__device__ __forceinline__ void load_weights(const FieldDev& F, uint8_t* s_w, float* s_b) {
  const uint4* src = weight_src<MODE>(F);
  uint4* dst = reinterpret_cast<uint4*>(s_w);
  for (int i = threadIdx.x; i < WeightSmem<MODE>::kBytes / 16; i += blockDim.x) dst[i] = src[i];
  for (int i = threadIdx.x; i < kBiasTotal; i += blockDim.x) s_b[i] = F.bias[i];
}

template <int MODE>
__device__ __forceinline__ void run_mlp(const uint8_t* s_w, const float* s_b, const FieldDev& F,
                                        const float feat[8], const float shs[4], int lane, float& o0,
                                        float lg[3]) {
  if constexpr (MODE == 0)
    mlp_tile_f32(reinterpret_cast<const float4*>(s_w), s_b, F.d1_ksteps / 4, feat, shs, lane, o0, lg);
  else
    mlp_tile_16<MODE == 2>(reinterpret_cast<const uint4*>(s_w), s_b, feat, Half8<MODE == 2>::pack4(shs), lane,
                           o0, lg);
}

// Stage the coarse occupancy grid into LDS.
__device__ __forceinline__ void load_coarse(const FieldDev& F, uint32_t* s_coarse) {
  const uint32_t words = (F.Gc * F.Gc * F.Gc + 31u) / 32u;
  for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) s_coarse[i] = F.coarse[i];
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

template <bool TAB16, int MODE>
__global__ __launch_bounds__(kBlock, MODE == 0 ? 3 : 4) void render_kernel(RenderArgs A) {
  __shared__ __align__(16) uint8_t s_w[WeightSmem<MODE>::kBytes];
  __shared__ float s_b[kBiasTotal];
  __shared__ LevelDev s_lv[kMaxLevels];
  __shared__ uint32_t s_coarse[kCoarseWords];
  __shared__ uint32_t s_off[kMaxCams + 1];
  __shared__ uint32_t s_rb[kMaxCams], s_re[kMaxCams];
  __shared__ uint32_t s_stats[6];
  __shared__ uint2 s_sh[MODE == 0 ? 1 : kBlock * 4];
  __shared__ uint32_t s_slot[kBlock];

  const FieldDev& F = A.F;
  const __amdgpu_buffer_rsrc_t tab = table_rsrc(F);
  load_weights<MODE>(F, s_w, s_b);
  load_coarse(F, s_coarse);
  if (threadIdx.x < F.L) s_lv[threadIdx.x] = F.levels[threadIdx.x];
  if (threadIdx.x < 6) s_stats[threadIdx.x] = 0;
  const uint32_t tx = (A.W + kTile - 1) / kTile;
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

  auto retire = [&]() {
    float4 v = make_float4(cr, cg, cb, 1.0f - T);
    if (A.linear_hdr) {
      v.x = pq_to_linear(v.x);
      v.y = pq_to_linear(v.y);
      v.z = pq_to_linear(v.z);
    }
    reinterpret_cast<float4*>(A.rgba)[pix] = v;
    if (A.nsamples) A.nsamples[pix] = n;
    ++st_rays;
    pix = kNone;
  };

  while (true) {
    // keep LDS reads of weights inside the loop (hoisting would pin the
    // weights in registers and drop occupancy to one wave per SIMD)
    asm volatile("" ::: "memory");
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
          const uint32_t col = (tile % tx) * kTile + within % kTile;
          const uint32_t row = s_rb[c] + (tile / tx) * kTile + within / kTile;
          if (col < A.W && row < s_re[c]) {
            setup_ray(F, A.cams[c], col, row, r);
            if constexpr (MODE != 0) store_ray_sh<MODE == 2>(F, r, &s_sh[threadIdx.x * 4]);
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
    if (__ballot(pix != kNone) == 0) break;
    __builtin_amdgcn_wave_barrier();

    // ---- 2. march to the next evaluated sample ---------------------------
    int mres = 0;
    float st = 0.0f, sx[3] = {0.0f, 0.0f, 0.0f}, slst = 0.0f;
    if (pix != kNone) {
      mres = march_next(F, s_coarse, r, A.budget, st_steps, st, sx);
      if (mres == 2) retire();
      if (mres == 1 && F.lod) slst = level_star(F, st, r.lr);
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

    // ---- 3. encode + MLP of the compacted samples -------------------------
    float so0 = 0.0f, sl0 = 0.0f, sl1 = 0.0f, sl2 = 0.0f;
    if constexpr (MODE == 0) {
      for (int t = 0; t < nt; ++t) {
        asm volatile("" ::: "memory");
        bool act;
        const int src = tile_source(&s_slot[wave_base], ns, t, lane, act);
        float feat[8], shs[4];
        tile_encode<TAB16, true>(F, s_lv, tab, src, act, lane, sx, slst, feat, st_fetch);
        sh_select(F, shfl_f(r.dx, src), shfl_f(r.dy, src), shfl_f(r.dz, src), lane >> 4, shs);
        float o0, lg[3];
        mlp_tile_f32(reinterpret_cast<const float4*>(s_w), s_b, F.d1_ksteps / 4, feat, shs, lane, o0, lg);
        const int from = rank & 15;
        const float a0 = shfl_f(o0, from), a1 = shfl_f(lg[0], from);
        const float a2 = shfl_f(lg[1], from), a3 = shfl_f(lg[2], from);
        if (has && (rank >> 4) == t) {
          so0 = a0;
          sl0 = a1;
          sl1 = a2;
          sl2 = a3;
        }
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
            float feat[8];
            tile_encode<TAB16, false>(F, s_lv, tab, src, act, lane, sx, slst, feat, st_fetch);
            xin[t] = H::pack(feat);
            shh[t] = s_sh[(wave_base + src) * 4 + (lane >> 4)];
          }
        float o0[kMlpBatch], lg[kMlpBatch][3];
        mlp_batch_16<MODE == 2, kMlpBatch>(reinterpret_cast<const uint4*>(s_w), s_b, cnt, xin, shh, lane, o0, lg);
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
      }
    }

    // ---- 4. composite (FP32), terminate --------------------------------
    if (has) {
      const float sd = expf(so0) * F.dt;
      const float trans = expf(-sd);
      const float wgt = T * (1.0f - trans);
      cr = fmaf(wgt, sigmoidf(sl0), cr);
      cg = fmaf(wgt, sigmoidf(sl1), cg);
      cb = fmaf(wgt, sigmoidf(sl2), cb);
      T = T * trans;
      ++n;
      ++st_samples;
      if (T < F.t_min || n >= F.max_samples) retire();
    }
  }

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

__global__ void march_kernel(FieldDev F, const vrn_camera* cams, uint32_t n_cams, uint32_t W, uint32_t H,
                             uint32_t* klist, uint32_t max_k, uint32_t* count) {
  __shared__ uint32_t s_coarse[kCoarseWords];
  load_coarse(F, s_coarse);
  __syncthreads();
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= (uint64_t)n_cams * W * H) return;
  const uint32_t c = (uint32_t)(i / ((uint64_t)W * H));
  const uint32_t rem = (uint32_t)(i % ((uint64_t)W * H));
  Ray r;
  setup_ray(F, cams[c], rem % W, rem / W, r);
  uint32_t cnt = 0, steps = 0;
  float st, sx[3];
  while (cnt < F.max_samples) {
    if (march_next(F, s_coarse, r, 0x40000000u, steps, st, sx) != 1) break;
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
    rgb[3 * p] = sigmoidf(lg[0]);
    rgb[3 * p + 1] = sigmoidf(lg[1]);
    rgb[3 * p + 2] = sigmoidf(lg[2]);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <bool TAB16, int MODE>
static int blocks_per_cu_impl() {
  static int cached = -1;
  if (cached < 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, render_kernel<TAB16, MODE>, kBlock, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    cached = nb;
  }
  return cached;
}

int render_blocks_per_cu(int table_f16, int compute) {
  if (table_f16) {
    if (compute == 0) return blocks_per_cu_impl<true, 0>();
    if (compute == 1) return blocks_per_cu_impl<true, 1>();
    return blocks_per_cu_impl<true, 2>();
  }
  if (compute == 0) return blocks_per_cu_impl<false, 0>();
  if (compute == 1) return blocks_per_cu_impl<false, 1>();
  return blocks_per_cu_impl<false, 2>();
}

hipError_t launch_render(const RenderArgs& a, int compute, int grid, hipStream_t s) {
  const dim3 gr(grid), bl(kBlock);
  if (a.F.table_f16) {
    if (compute == 0) hipLaunchKernelGGL((render_kernel<true, 0>), gr, bl, 0, s, a);
    else if (compute == 1) hipLaunchKernelGGL((render_kernel<true, 1>), gr, bl, 0, s, a);
    else hipLaunchKernelGGL((render_kernel<true, 2>), gr, bl, 0, s, a);
  } else {
    if (compute == 0) hipLaunchKernelGGL((render_kernel<false, 0>), gr, bl, 0, s, a);
    else if (compute == 1) hipLaunchKernelGGL((render_kernel<false, 1>), gr, bl, 0, s, a);
    else hipLaunchKernelGGL((render_kernel<false, 2>), gr, bl, 0, s, a);
  }
  return hipGetLastError();
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
  hipLaunchKernelGGL(march_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, F, d_cams, n_cams, W,
                     H, klist, max_k, count);
  return hipGetLastError();
}

hipError_t launch_encode(const FieldDev& F, const float* xyz, const float* t, const float* r, uint32_t n,
                         float* feat, hipStream_t s) {
  const uint32_t per_block = (kBlock / 64) * 16;
  const dim3 gr((n + per_block - 1) / per_block), bl(kBlock);
  if (F.table_f16) hipLaunchKernelGGL((encode_kernel<true>), gr, bl, 0, s, F, xyz, t, r, n, feat);
  else hipLaunchKernelGGL((encode_kernel<false>), gr, bl, 0, s, F, xyz, t, r, n, feat);
  return hipGetLastError();
}

hipError_t launch_mlp(const FieldDev& F, const float* feat, const float* dir, uint32_t n, int compute,
                      float* sigma, float* rgb, hipStream_t s) {
  const uint32_t per_block = (kBlock / 64) * 16;
  const dim3 gr((n + per_block - 1) / per_block), bl(kBlock);
  if (compute == 0) hipLaunchKernelGGL((mlp_kernel<0>), gr, bl, 0, s, F, feat, dir, n, sigma, rgb);
  else if (compute == 1) hipLaunchKernelGGL((mlp_kernel<1>), gr, bl, 0, s, F, feat, dir, n, sigma, rgb);
  else hipLaunchKernelGGL((mlp_kernel<2>), gr, bl, 0, s, F, feat, dir, n, sigma, rgb);
  return hipGetLastError();
}

}  // namespace vrn
