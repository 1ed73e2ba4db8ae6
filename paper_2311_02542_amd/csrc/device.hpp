// Device functions of the renderer hot path (gfx950, wave64).
//
// Every function here is used both by the fused render kernel and by the
// single-stage kernels behind vrn_rays / vrn_march / vrn_encode / vrn_mlp,
// so stage parity tests exercise the exact code that renders frames.
//
// The translation unit is compiled with -ffp-contract=off: the ray and
// lattice geometry below is the canonical FP32 operation sequence (each
// product and sum rounded on its own), which is what makes occupancy cell
// decisions reproducible bit for bit.  Fused multiply-adds are written
// explicitly (fmaf) only where the math wants them.
#pragma once

#include <type_traits>

#include "internal.hpp"

namespace vrn {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ float shfl_f(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
__device__ __forceinline__ int shfl_i(int v, int src) {
  return __builtin_amdgcn_ds_bpermute(src << 2, v);
}

// ---------------------------------------------------------------------------
// Rays (Sec. 4.2.1 cone footprint; pinhole, OpenCV axes, pixel centres +0.5)
// ---------------------------------------------------------------------------

struct Ray {
  float ox, oy, oz, dx, dy, dz;
  float lr;      // ln(r) + ln(2 s / extent): log of the LOD footprint per unit t
  float delta;   // block-skip margin in cell units (bounds FP32 rounding of q)
  int k, k_hi;   // lattice cursor and last lattice index worth testing
  int brick;     // index of the 4x4x4 brick whose bits are cached below (-1: none)
  uint32_t blo, bhi;
  float nx, ny, nz;  // right neighbour's direction (contracted LOD footprint)
};

// Canonical FP32 direction: a = ((i + .5) - cx) / fx, b = ((j + .5) - cy) / fy,
// w = (R[:,0] a + R[:,1] b) + R[:,2], d = w / sqrt((wx wx + wy wy) + wz wz).
__device__ __forceinline__ void canonical_ray(const vrn_camera& c, uint32_t col, uint32_t row,
                                              float w[3], float& n, float d[3]) {
  const float a = (((float)col + 0.5f) - c.cx) / c.fx;
  const float b = (((float)row + 0.5f) - c.cy) / c.fy;
#pragma unroll
  for (int r = 0; r < 3; ++r) w[r] = (c.c2w[4 * r] * a + c.c2w[4 * r + 1] * b) + c.c2w[4 * r + 2];
  n = sqrtf((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]);
#pragma unroll
  for (int r = 0; r < 3; ++r) d[r] = w[r] / n;
}

// Base radius at unit distance: chord between the unit directions of this
// pixel and its right neighbour, 2 sin(theta / 2), evaluated without
// cancellation: sin(theta) = |w x v| / (|w| |w + v|) with v = R[:,0] / fx.
__device__ __forceinline__ float cone_pitch(const vrn_camera& c, const float w[3], float n, float scale) {
  // continuous quantity (it only places the LOD weights): hardware
  // reciprocal / square root are accurate to ~1 ulp, far below what matters
  const float ifx = __builtin_amdgcn_rcpf(c.fx);
  const float v[3] = {c.c2w[0] * ifx, c.c2w[4] * ifx, c.c2w[8] * ifx};
  const float e[3] = {w[0] + v[0], w[1] + v[1], w[2] + v[2]};
  const float cx = w[1] * v[2] - w[2] * v[1];
  const float cy = w[2] * v[0] - w[0] * v[2];
  const float cz = w[0] * v[1] - w[1] * v[0];
  const float inv = __builtin_amdgcn_rcpf(n * __builtin_amdgcn_sqrtf(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]));
  const float sn = __builtin_amdgcn_sqrtf(cx * cx + cy * cy + cz * cz) * inv;
  const float cs = (w[0] * e[0] + w[1] * e[1] + w[2] * e[2]) * inv;
  return scale * sn * __builtin_amdgcn_rsqf(0.5f * (1.0f + cs));
}

// Number of lattice samples k < K whose canonical table entry t_k is <= t.
// The table's shape gives a guess -- steps of dt up to t_sw, then growth by
// (1 + g) per step -- that the FP32 recurrence departs from by a fraction
// of a step on the tables used here; a walk over neighbouring entries (two
// independent loads per step) makes it exact, and a binary search takes
// over if the walk runs long.  The plain binary search costs ~log2 K
// dependent loads on every skip of the march.
__device__ __forceinline__ int table_count_le(const FieldDev& F, float t) {
  const int K = (int)F.lat_K;
  if (!(t >= F.lat[0])) return 0;   // NaN included
  if (t >= F.lat[K - 1]) return K;
  // the count is in [1, K - 1]: t_{c-1} <= t < t_c
  const float kf = t < F.lat_tsw ? (t - 0.5f * F.dt) * F.inv_dt
                                 : F.lat_ksw + __logf(t / F.lat_tsw) * F.lat_inv_log;
  int c = (int)fminf(fmaxf(kf + 1.0f, 1.0f), (float)(K - 1));
  for (int i = 0; i < 6; ++i) {
    const float a = F.lat[c - 1], b = F.lat[c];
    if (a > t) --c;
    else if (b <= t) ++c;
    else return c;
  }
  int lo = 1, hi = K - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (F.lat[mid] <= t) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Lattice range [k_lo, k_hi] worth testing.  A canonical FP32 sample
// position strays from the exact point o + t d by less than
// 2^-22 (|o| + t + |aabb_min| + 2 extent) (every op rounds once), so no sample
// outside the slab interval of the cube grown by c0 + c1 t per side, with
// c = 2^-18 (16 times that bound, which also covers the rounding of this
// FP32 evaluation, reciprocals included), can pass the cell test.  The range is that interval,
// padded by two samples on each side; the canonical per-sample test alone
// decides membership.  With a sample table the interval is mapped through
// the table; contracted fields keep every table sample (all of space lies in
// the cube).
template <int GEO>
__device__ __forceinline__ void lattice_range(const FieldDev& F, Ray& r) {
  const float o[3] = {r.ox, r.oy, r.oz};
  const float d[3] = {r.dx, r.dy, r.dz};
  const float kmax = 16777000.0f;  // keep k < 2^24 (k + 0.5 exact in FP32)
  if (GEO == 1 && F.contract) {
    r.k = 0;
    r.k_hi = (int)F.lat_K - 1;
    const float M = (fmaxf(fabsf(o[0] - F.center[0]), fmaxf(fabsf(o[1] - F.center[1]), fabsf(o[2] - F.center[2]))) +
                     F.lat[F.lat_K - 1]) * F.inv_radius + 2.0f;
    r.delta = ldexpf(F.cs * M + (float)F.G + 1.0f, -20);
    return;
  }
  const float amax = fmaxf(fabsf(F.amin[0]), fmaxf(fabsf(F.amin[1]), fabsf(F.amin[2])));
  const float omax = fmaxf(fabsf(o[0]), fmaxf(fabsf(o[1]), fabsf(o[2])));
  const float c1 = 0x1p-18f;
  const float c0 = c1 * (omax + amax + 2.0f * F.extent);
  float tlo = 0.0f, thi = 3.0e38f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // lower face: t (d + c1) >= amin - c0 - o
    // (hardware reciprocals: their ~1 ulp is far inside the margin)
    const float al = d[a] + c1, bl = (F.amin[a] - c0) - o[a];
    const float rl = bl * __builtin_amdgcn_rcpf(al);
    if (al > 0.0f) tlo = fmaxf(tlo, rl);
    else if (al < 0.0f) thi = fminf(thi, rl);
    else if (bl > 0.0f) thi = -1.0f;
    // upper face: t (d - c1) <= amin + extent + c0 - o
    const float ah = d[a] - c1, bh = ((F.amin[a] + F.extent) + c0) - o[a];
    const float rh = bh * __builtin_amdgcn_rcpf(ah);
    if (ah > 0.0f) thi = fminf(thi, rh);
    else if (ah < 0.0f) tlo = fmaxf(tlo, rh);
    else if (bh < 0.0f) thi = -1.0f;
  }
  const bool miss = !(thi >= tlo);
  if constexpr (GEO == 0) {
    const float klo = floorf(tlo * F.inv_dt - 0.5f) - 2.0f;
    const float khi = ceilf(fminf(thi * F.inv_dt, kmax) - 0.5f) + 2.0f;
    if (miss || klo > kmax) {
      r.k = 0;
      r.k_hi = -1;
    } else {
      r.k = (int)fmaxf(klo, 0.0f);
      r.k_hi = (int)fminf(khi, kmax);
    }
  } else {
    if (miss) {
      r.k = 0;
      r.k_hi = -1;
    } else {
      r.k = max(table_count_le(F, tlo) - 2, 0);
      r.k_hi = min(table_count_le(F, thi) + 1, (int)F.lat_K - 1);
    }
  }
  const float tcap = GEO == 0 ? kmax * F.dt : F.lat[F.lat_K - 1];
  const float M = omax + fminf(fmaxf(thi, 0.0f), tcap) + amax;
  r.delta = ldexpf(F.cs * M + (float)F.G + 1.0f, -20);
}

template <int GEO>
__device__ __forceinline__ void setup_ray(const FieldDev& F, const vrn_camera& c, uint32_t col,
                                          uint32_t row, Ray& r) {
  float w[3], n, d[3];
  canonical_ray(c, col, row, w, n, d);
  r.ox = c.c2w[3];
  r.oy = c.c2w[7];
  r.oz = c.c2w[11];
  r.dx = d[0];
  r.dy = d[1];
  r.dz = d[2];
  r.lr = F.lod ? __logf(cone_pitch(c, w, n, F.lod_radius_scale)) + F.lod_c : 0.0f;
  r.nx = r.ny = r.nz = 0.0f;
  if (GEO == 1 && F.contract && F.lod) {
    float w2[3], n2, d2[3];
    canonical_ray(c, col + 1, row, w2, n2, d2);
    r.nx = d2[0];
    r.ny = d2[1];
    r.nz = d2[2];
  }
  r.brick = -1;
  r.blo = r.bhi = 0u;
  lattice_range<GEO>(F, r);
}

// ---------------------------------------------------------------------------
// Occupancy march (Sec. 4.3)
// ---------------------------------------------------------------------------

// Canonical L-infinity contraction of a world point, in place: u = (x - c)
// * inv_radius, m = max |u|, y = u if m <= 1 else u * ((2 - 1/m) * (1/m)).
__device__ __forceinline__ void contract_point(const FieldDev& F, float x[3]) {
  const float u[3] = {(x[0] - F.center[0]) * F.inv_radius, (x[1] - F.center[1]) * F.inv_radius,
                      (x[2] - F.center[2]) * F.inv_radius};
  const float m = fmaxf(fmaxf(fabsf(u[0]), fabsf(u[1])), fabsf(u[2]));
  if (m <= 1.0f) {
    x[0] = u[0];
    x[1] = u[1];
    x[2] = u[2];
  } else {
    const float im = 1.0f / m;
    const float s = (2.0f - im) * im;
    x[0] = u[0] * s;
    x[1] = u[1] * s;
    x[2] = u[2] * s;
  }
}

// The table entry after t: the same FP32 recurrence, in the same operation
// order, that built the table on the host (t_{k+1} = t_k + max(dt, g t_k)),
// so table_next(t_k) equals t_{k+1} bit for bit.
__device__ __forceinline__ float table_next(const FieldDev& F, float t) {
  const float g = F.step_growth * t;
  return t + fmaxf(g, F.dt);  // both operands positive and finite
}

// Canonical position of the lattice sample at parameter t: x = o + t d
// (contracted for unbounded fields), q = (x - amin) cs.
template <int GEO>
__device__ __forceinline__ void lattice_pos(const FieldDev& F, const Ray& r, float t, float x[3], float q[3]) {
  x[0] = r.ox + t * r.dx;
  x[1] = r.oy + t * r.dy;
  x[2] = r.oz + t * r.dz;
  if constexpr (GEO == 1) {
    if (F.contract) contract_point(F, x);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) q[a] = (x[a] - F.amin[a]) * F.cs;
}

// Canonical lattice sample k: t = (k + .5) dt (or the FP32 table entry).
template <int GEO>
__device__ __forceinline__ void lattice_q(const FieldDev& F, const Ray& r, int k, float& t, float x[3],
                                          float q[3]) {
  if constexpr (GEO == 0) t = ((float)k + 0.5f) * F.dt;
  else t = F.lat[k];
  lattice_pos<GEO>(F, r, t, x, q);
}

// floor(q) with q clamped to [-1, G] first (no integer overflow far outside
// the grid; q is never NaN), the floor and the conversion in one instruction.
// (A med3 clamp would save one more, but costs the FP32X kernel scratch
// spills.)
__device__ __forceinline__ int cell_of(float q, int G) {
  const float c = fminf(fmaxf(q, -1.0f), (float)G);
  int i;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(i) : "v"(c));
  return i;
}

// x + n (y + n z) for the coarse-block and brick grids (n <= 256, indices
// below 2^24): 24-bit multiplies issue at the full rate, where a 32-bit
// multiply-add would take the quarter-rate 64-bit form.
__device__ __forceinline__ uint32_t mad_u24(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t d;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}
__device__ __forceinline__ uint32_t grid_index(uint32_t x, uint32_t y, uint32_t z, uint32_t n) {
  return mad_u24(n, mad_u24(n, z, y), x);
}

__device__ __forceinline__ bool bit_set(const uint32_t* bits, uint32_t idx) {
  return (bits[idx >> 5] >> (idx & 31u)) & 1u;
}

// Contracted fields, outside the unit L-inf ball: the canonical samples lie
// on the image of the straight ray under C.  Over a stretch [t_a, t_b] on
// which one axis i dominates u at both ends, with the same sign and
// |u_i| > 1, it dominates throughout (|u_j| - |u_i| is convex in t and
// |u_i| linear), so y_i = sign (2 - 1/|u_i|) is monotone, and y_j = a b with
// a = 2 - 1/|u_i| in (1, 2) and b = u_j / |u_i| both monotone: the products
// of their end values bound y_j.  CurveStart holds the start of a stretch
// (sample r.k); curve_bound returns the box, in cell units, that holds the
// curve from there to sample kb, or false when the dominance condition
// fails.  Canonical sample positions lie within FP32 error (far below a
// hundredth of a cell) of the curve.
struct CurveStart {
  float b[3], s, a;  // b = u / m at the start (the dominant axis' entry is unused)
  int axis;
};

__device__ __forceinline__ void curve_u(const FieldDev& F, const Ray& r, float t, float u[3]) {
  u[0] = (r.ox + t * r.dx - F.center[0]) * F.inv_radius;
  u[1] = (r.oy + t * r.dy - F.center[1]) * F.inv_radius;
  u[2] = (r.oz + t * r.dz - F.center[2]) * F.inv_radius;
}

__device__ __forceinline__ void curve_dominant(const float u[3], int& axis, float& m) {
  const float ax = fabsf(u[0]), ay = fabsf(u[1]), az = fabsf(u[2]);
  axis = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
  m = fmaxf(ax, fmaxf(ay, az));
}

// False when sample r.k lies in the unit ball (no curve bound applies).
__device__ __forceinline__ bool curve_start(const FieldDev& F, const Ray& r, CurveStart& c) {
  float u[3], m;
  curve_u(F, r, F.lat[r.k], u);
  curve_dominant(u, c.axis, m);
  c.s = c.axis == 0 ? u[0] : (c.axis == 1 ? u[1] : u[2]);
  c.a = 2.0f - 1.0f / m;
#pragma unroll
  for (int a = 0; a < 3; ++a) c.b[a] = a == c.axis ? 0.0f : u[a] / m;
  return m > 1.0f;
}

__device__ __forceinline__ bool curve_bound(const FieldDev& F, const Ray& r, const CurveStart& c, int kb,
                                            float qlo[3], float qhi[3]) {
  const float g4 = 0.25f * (float)F.G;
  float ub[3];
  curve_u(F, r, F.lat[kb], ub);
  int ib;
  float mb;
  curve_dominant(ub, ib, mb);
  const float sb = ib == 0 ? ub[0] : (ib == 1 ? ub[1] : ub[2]);
  if (ib != c.axis || (c.s > 0.0f) != (sb > 0.0f) || !(mb > 1.0f)) return false;
  const float ab = 2.0f - 1.0f / mb;
  const float alo = fminf(c.a, ab), ahi = fmaxf(c.a, ab);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float lo, hi;
    if (a == c.axis) {
      lo = c.s > 0.0f ? alo : -ahi;
      hi = c.s > 0.0f ? ahi : -alo;
    } else {
      const float ba = c.b[a], bb = ub[a] / mb;
      const float blo = fminf(ba, bb), bhi = fmaxf(ba, bb);
      lo = fminf(fminf(alo * blo, alo * bhi), fminf(ahi * blo, ahi * bhi));
      hi = fmaxf(fmaxf(alo * blo, alo * bhi), fmaxf(ahi * blo, ahi * bhi));
    }
    qlo[a] = (lo + 2.0f) * g4;
    qhi[a] = (hi + 2.0f) * g4;
  }
  return true;
}

// Jump past the lattice samples that stay inside the empty box of `size`
// cells with corner o (cell units), shrunk by delta.  The jump is taken only
// when the current sample (q) and the landing sample both lie in the shrunk
// box: by convexity every lattice sample in between lies in it too, and
// delta >= twice the FP32 error of q, so no sample whose canonical cell is
// occupied is ever passed.  Beyond the unit ball of a contracted field the
// samples follow a curve: there a doubling search takes the farthest
// r.k + 2^j (j >= 1) whose curve box, padded by a hundredth of a cell, lies
// in the shrunk box.  Returns true if r.k moved.
template <int GEO>
__device__ __forceinline__ bool skip_box(const FieldDev& F, Ray& r, const float q[3], int ox, int oy, int oz,
                                         float size, float& t_land) {
  const float lo[3] = {ox * size + r.delta, oy * size + r.delta, oz * size + r.delta};
  const float hi[3] = {(ox + 1) * size - r.delta, (oy + 1) * size - r.delta, (oz + 1) * size - r.delta};
  if (!(q[0] >= lo[0] && q[0] <= hi[0] && q[1] >= lo[1] && q[1] <= hi[1] && q[2] >= lo[2] && q[2] <= hi[2]))
    return false;
  if (GEO == 1 && F.contract) {
    // only boxes inside the identity region (|u|inf <= 1: q in [G/4, 3G/4])
    // map straight segments to straight segments
    const float a = 0.25f * (float)F.G, b = 0.75f * (float)F.G;
    if (!(ox * size >= a && oy * size >= a && oz * size >= a && (ox + 1) * size <= b && (oy + 1) * size <= b &&
          (oz + 1) * size <= b)) {
      CurveStart c;
      if (!curve_start(F, r, c)) return false;
      int best = r.k;
      for (int step = 2; step < (1 << 20); step *= 2) {
        const int kb = min(r.k + step, r.k_hi);
        if (kb <= best) break;
        float ql[3], qh[3];
        if (!curve_bound(F, r, c, kb, ql, qh)) break;
        if (!(ql[0] - 0.01f >= lo[0] && qh[0] + 0.01f <= hi[0] && ql[1] - 0.01f >= lo[1] && qh[1] + 0.01f <= hi[1] &&
              ql[2] - 0.01f >= lo[2] && qh[2] + 0.01f <= hi[2]))
          break;
        best = kb;
        if (kb == r.k_hi) break;
      }
      if (best < r.k + 2) return false;
      r.k = best + 1;
      return true;
    }
  }
  // approximate exit parameter (reciprocals need not be exact: the landing
  // sample is re-tested with the canonical arithmetic below)
  const float o[3] = {r.ox, r.oy, r.oz};
  const float d[3] = {r.dx, r.dy, r.dz};
  float te = 3.0e38f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float bq = signbit(d[a]) ? lo[a] : hi[a];
    float xb = bq * F.inv_cs + F.amin[a];
    if (GEO == 1 && F.contract) xb = xb * F.radius + F.center[a];
    te = fminf(te, (xb - o[a]) * __builtin_amdgcn_rcpf(d[a]));
  }
  int kb;
  if constexpr (GEO == 0) {
    const float kbf = fminf(floorf(te * F.inv_dt - 0.5f), (float)r.k_hi);
    if (!(kbf >= (float)r.k + 2.0f)) return false;
    kb = (int)kbf;
  } else {
    kb = min(table_count_le(F, te) - 1, r.k_hi);
    if (kb < r.k + 2) return false;
  }
#pragma unroll
  for (int tries = 0; tries < 2; ++tries, --kb) {
    float t2, x2[3], q2[3];
    lattice_q<GEO>(F, r, kb, t2, x2, q2);
    if (q2[0] >= lo[0] && q2[0] <= hi[0] && q2[1] >= lo[1] && q2[1] <= hi[1] && q2[2] >= lo[2] &&
        q2[2] <= hi[2]) {
      r.k = kb + 1;
      t_land = t2;
      return true;
    }
  }
  return false;
}

// Walk the coarse grid from block (bx, by, bz) along a straight ray through
// consecutive blocks whose dilated bit is clear (the block and its 26
// neighbours hold no occupied cell) and lie in [blo, bhi] on every axis,
// and return the ray parameter where the walk leaves the last such block.
// The ray in cell units is qo + t dq.  Every point within one block width of
// a clear block lies in an empty block.  The walk and the canonical sample
// positions both deviate from the exact ray by far less than a block, so
// every lattice sample with t up to the returned value (rounded either way)
// has an empty cell.
__device__ __forceinline__ float coarse_run(const FieldDev& F, const uint32_t* dil, const float qo[3],
                                            const float dq[3], int bx, int by, int bz, int blo, int bhi) {
  const float cb = (float)(1u << F.cshift);
  const int Gc = (int)F.Gc;
  const int b0[3] = {bx, by, bz};
  float tm[3], td[3];
  int st[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float inv = __builtin_amdgcn_rcpf(dq[a]);
    st[a] = dq[a] > 0.0f ? 1 : (dq[a] < 0.0f ? -1 : 0);
    tm[a] = st[a] == 0 ? 3.0e38f : ((float)(b0[a] + (st[a] > 0)) * cb - qo[a]) * inv;
    td[a] = st[a] == 0 ? 3.0e38f : cb * fabsf(inv);
  }
  int x = bx, y = by, z = bz;
  float tx = tm[0], ty = tm[1], tz = tm[2];
  float t_exit = 0.0f;
  for (int it = 0; it < 3 * Gc; ++it) {
    const bool ax = tx <= ty && tx <= tz;
    const bool ay = !ax && ty <= tz;
    const bool az = !ax && !ay;
    t_exit = ax ? tx : (ay ? ty : tz);
    x += ax ? st[0] : 0;
    y += ay ? st[1] : 0;
    z += az ? st[2] : 0;
    if (x < blo || y < blo || z < blo || x > bhi || y > bhi || z > bhi) break;
    if (bit_set(dil, grid_index((uint32_t)x, (uint32_t)y, (uint32_t)z, (uint32_t)Gc))) break;
    tx += ax ? td[0] : 0.0f;
    ty += ay ? td[1] : 0.0f;
    tz += az ? td[2] : 0.0f;
  }
  return t_exit;
}

// When every coarse block touched by the curve's box from r.k to a sample
// (padded by a hundredth of a cell) is clear, every sample of that stretch
// has an empty cell.  A doubling search returns the farthest lattice index
// r.k + 2^j whose stretch from r.k passes (r.k itself when none does).
__device__ __forceinline__ int contracted_run(const FieldDev& F, const uint32_t* dil, const Ray& r) {
  const float inv_cb = 1.0f / (float)(1u << F.cshift);
  const int Gc = (int)F.Gc;
  CurveStart c;
  if (!curve_start(F, r, c)) return r.k;
  // does the stretch [r.k, kb] stay in clear blocks?
  auto stretch_clear = [&](int kb) -> bool {
    float ql[3], qh[3];
    if (!curve_bound(F, r, c, kb, ql, qh)) return false;
    int b0[3], b1[3];
    bool fits = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      b0[a] = (int)floorf((ql[a] - 0.01f) * inv_cb);
      b1[a] = (int)floorf((qh[a] + 0.01f) * inv_cb);
      fits = fits && b0[a] >= 0 && b1[a] < Gc && b1[a] - b0[a] <= 1;
    }
    if (!fits) return false;
    bool clear = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int x = b0[0] + (k & 1), y = b0[1] + ((k >> 1) & 1), z = b0[2] + (k >> 2);
      if (x <= b1[0] && y <= b1[1] && z <= b1[2])
        clear = clear && !bit_set(dil, grid_index((uint32_t)x, (uint32_t)y, (uint32_t)z, (uint32_t)Gc));
    }
    return clear;
  };
  // gallop: double the stretch while it stays clear (a finer search past the
  // first failure costs more probes than it saves lattice tests)
  int best = r.k;
  for (int step = 1; step < (1 << 20); step *= 2) {
    const int kb = min(r.k + step, r.k_hi);
    if (kb <= best || !stretch_clear(kb)) break;
    best = kb;
    if (kb == r.k_hi) break;
  }
  return best;
}

// Advance to the next evaluated sample within `budget` lattice tests.
// Returns 1 (sample found; st, sx are its canonical t and x), 0 (budget used
// up) or 2 (ray exhausted).  Occupancy is tested hierarchically: the coarse
// grid (blocks of 2^cshift cells, in LDS), then the 4x4x4 brick (one 64-bit
// load, kept in registers while the ray stays in the brick), then the cell
// bit.  A sample in a clear block (dilated bit 0) jumps to the end of the
// run of clear blocks: along the straight ray for bounded fields and inside
// the unit ball of contracted ones (coarse_run), along bounds of the curved
// image beyond it (contracted_run).  Other empty coarse blocks and empty
// bricks are skipped with skip_box.  `coarse` holds the coarse grid and,
// kCoarseWords later, its dilation.
template <int GEO>
__device__ __forceinline__ int march_next(const FieldDev& F, const uint32_t* coarse, Ray& r, uint32_t budget,
                                          uint32_t& steps, float& st, float sx[3]) {
  const int G = (int)F.G;
  // sample-table lattices: the parameter of sample r.k is carried from the
  // previous test (tk, valid while kt == r.k) by the table's own
  // recurrence, so stepping and box skips read no table entry
  int kt = -1;
  float tk = 0.0f;
  for (uint32_t it = 0; it < budget; ++it) {
    if (r.k > r.k_hi) return 2;
    ++steps;
    float t, x[3], q[3];
    if constexpr (GEO == 0) {
      lattice_q<GEO>(F, r, r.k, t, x, q);
    } else {
      t = kt == r.k ? tk : F.lat[r.k];
      lattice_pos<GEO>(F, r, t, x, q);
    }
    const int cx = cell_of(q[0], G), cy = cell_of(q[1], G), cz = cell_of(q[2], G);
    // empty box to try to jump over: the cell's block of 2^bsh cells (-1: none)
    int bsh = -1;
    if ((unsigned)cx < (unsigned)G && (unsigned)cy < (unsigned)G && (unsigned)cz < (unsigned)G) {
      const int bx = cx >> F.cshift, by = cy >> F.cshift, bz = cz >> F.cshift;
      const uint32_t ci = grid_index((uint32_t)bx, (uint32_t)by, (uint32_t)bz, F.Gc);
      VRN_DEBUG_COUNT(ci >= F.Gc * F.Gc * F.Gc, kDbgCoarse);
      if (!bit_set(coarse, ci)) {
        if (!bit_set(coarse + kCoarseWords, ci)) {
          // a clear block starts a run of empty blocks: jump to its end
          int kb = r.k;
          // straight walks: bounded fields, and blocks wholly inside the unit
          // ball of contracted ones (q in [G/4, 3G/4], where C is the
          // identity); beyond it the curved image of the ray is bounded
          // piecewise (contracted_run)
          float qo[3], dq[3];
          int blo = 0, bhi = (int)F.Gc - 1;
          bool walk = true;
          if (GEO == 1 && F.contract) {
            const int ilo = (int)(F.G >> (2 + F.cshift)), ihi = (int)((3 * F.G) >> (2 + F.cshift)) - 1;
            walk = bx >= ilo && by >= ilo && bz >= ilo && bx <= ihi && by <= ihi && bz <= ihi &&
                   (ilo << F.cshift) == (int)(F.G >> 2) && ((ihi + 1) << F.cshift) == (int)((3 * F.G) >> 2);
            blo = ilo;
            bhi = ihi;
            const float s = F.inv_radius * 0.25f * (float)F.G;
            qo[0] = (r.ox - F.center[0]) * s + 0.5f * (float)F.G;
            qo[1] = (r.oy - F.center[1]) * s + 0.5f * (float)F.G;
            qo[2] = (r.oz - F.center[2]) * s + 0.5f * (float)F.G;
            dq[0] = r.dx * s;
            dq[1] = r.dy * s;
            dq[2] = r.dz * s;
          } else {
            qo[0] = (r.ox - F.amin[0]) * F.cs;
            qo[1] = (r.oy - F.amin[1]) * F.cs;
            qo[2] = (r.oz - F.amin[2]) * F.cs;
            dq[0] = r.dx * F.cs;
            dq[1] = r.dy * F.cs;
            dq[2] = r.dz * F.cs;
          }
          if (walk) {
            const float te = coarse_run(F, coarse + kCoarseWords, qo, dq, bx, by, bz, blo, bhi);
            if constexpr (GEO == 0) kb = (int)fminf(floorf(te * F.inv_dt - 0.5f), (float)r.k_hi);
            else kb = min(table_count_le(F, te) - 1, r.k_hi);
          } else if (GEO == 1 && F.contract) {
            kb = contracted_run(F, coarse + kCoarseWords, r);
          }
          if (kb > r.k) {
            r.k = kb + 1;
            continue;
          }
        }
        bsh = (int)F.cshift;
      } else {
        const int kx = cx >> 2, ky = cy >> 2, kz = cz >> 2;
        const int brick = (int)grid_index((uint32_t)kx, (uint32_t)ky, (uint32_t)kz, F.Gb);
        if (brick != r.brick) {
          VRN_DEBUG_COUNT((uint32_t)brick >= F.Gb * F.Gb * F.Gb, kDbgBrick);
          const unsigned long long b = F.bricks[brick];
          r.brick = brick;
          r.blo = (uint32_t)b;
          r.bhi = (uint32_t)(b >> 32);
        }
        if ((r.blo | r.bhi) == 0u) {
          bsh = 2;
        } else {
          const uint32_t bit = (uint32_t)((cx & 3) | ((cy & 3) << 2) | ((cz & 3) << 4));
          const unsigned long long bits = ((unsigned long long)r.bhi << 32) | r.blo;
          if ((bits >> bit) & 1ull) {
            st = t;
            sx[0] = x[0];
            sx[1] = x[1];
            sx[2] = x[2];
            r.k++;
            return 1;
          }
        }
      }
    }
    float t_land = 0.0f;   // table entries are > 0: 0 means not known
    const bool moved =
        bsh >= 0 && skip_box<GEO>(F, r, q, cx >> bsh, cy >> bsh, cz >> bsh, (float)(1 << bsh), t_land);
    if constexpr (GEO == 1) {
      // the next test's parameter: the successor of this one, or of the
      // landing sample of a straight skip (r.k is then already past it);
      // after a curve skip the next test reads the table
      if (!moved) {
        tk = table_next(F, t);
        kt = r.k + 1;
      } else if (t_land > 0.0f) {
        tk = table_next(F, t_land);
        kt = r.k;
      } else {
        kt = -1;
      }
    }
    if (!moved) r.k++;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Hash encoding with LOD (Sec. 4 after iNGP; Sec. 4.2.1 Eq. 3; App. D)
// ---------------------------------------------------------------------------

// Base lattice corner and fraction of p = u S in FP64 (u = x - aabb_min,
// exact in FP64 for FP32 x; S = N / extent rounded once), so the fraction
// is accurate to one FP32 rounding even at 2e4-cell levels, where an FP32 p
// would carry an error of 1e-3 cells.  FP64 multiply, floor, min/max and
// conversions issue at the FP32 rate on CDNA.  The corner is clamped to
// [0, N-1] with the fraction carrying the rest (p = N gives the last cell
// with fraction 1).
__device__ __forceinline__ uint32_t base_corner_f64(double u, double s, double top, float& fr) {
  const double p = u * s;
  const double ip = fmin(fmax(floor(p), 0.0), top);
  fr = (float)(p - ip);
  return (uint32_t)ip;
}

// Buffer resource over the whole [L][T][2] table (32-bit byte offsets;
// out-of-range offsets read as zero instead of faulting).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t table_rsrc(const FieldDev& F) {
  const uint32_t bytes = (F.L * (F.Tmask + 1u)) * (F.table_f16 ? 4u : 8u);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(F.tables), 0, (int)bytes, 0x00020000);
}

// Base corner and fraction from a plain FP32 p = u * S (the 16-bit paths,
// whose error budget is far above the rounding of p).  p is clamped to
// [0, below_n], so p = N yields the last cell with fraction 1 - ulp(N).
__device__ __forceinline__ uint32_t base_corner_fast(float u, float shi, float below_n, float& fr) {
  const float p = __builtin_amdgcn_fmed3f(u * shi, 0.0f, below_n);
  fr = __builtin_amdgcn_fractf(p);
  return (uint32_t)p;
}

// Byte offsets of the 8 corners of the cell with base corner i0 (corner c:
// +1 on x if c & 1, on y if c & 2, on z if c & 4).  Dense levels index
// x + y s + z s^2; hashed levels take (x pi_x ^ y pi_y ^ z pi_z) mod T (the
// iNGP hash).  The multipliers carry the entry size, so the mask is applied
// in bytes, and the level's base offset is a multiple of the level size, so
// it can be OR-ed into the masked hash.  grp (bit g: level g + 4j of lane
// group g is dense) is wave-uniform: a set of four levels that is all hashed
// or all dense takes one formula.
__device__ __forceinline__ void corner_offsets(const FieldDev& F, const LevelDev& P, uint32_t grp,
                                               const uint32_t i0[3], uint32_t off[8]) {
  const uint32_t hx0 = i0[0] * P.bx, hx1 = hx0 + P.bx;
  const uint32_t hy0 = i0[1] * P.by, hy1 = hy0 + P.by;
  const uint32_t hz0 = i0[2] * P.bz, hz1 = hz0 + P.bz;
  const uint32_t m = F.bmask;
  if (grp == 0u) {
    const uint32_t x0 = (hx0 & m) | P.base, x1 = (hx1 & m) | P.base;
    const uint32_t y0 = hy0 & m, y1 = hy1 & m, z0 = hz0 & m, z1 = hz1 & m;
#pragma unroll
    for (int c = 0; c < 8; ++c) off[c] = ((c & 1) ? x1 : x0) ^ ((c & 2) ? y1 : y0) ^ ((c & 4) ? z1 : z0);
  } else if (grp == 0xFu) {
    const uint32_t x0 = hx0 + P.base, x1 = hx1 + P.base;
#pragma unroll
    for (int c = 0; c < 8; ++c) off[c] = ((c & 1) ? x1 : x0) + ((c & 2) ? hy1 : hy0) + ((c & 4) ? hz1 : hz0);
  } else {
    // both formulas, then a bitwise select by the lane's level (no branches)
    const uint32_t dm = 0u - P.dense;  // all ones for a dense level
    const uint32_t xb0 = hx0 + P.base, xb1 = hx1 + P.base;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const uint32_t a = (c & 1) ? hx1 : hx0, b = (c & 2) ? hy1 : hy0, e = (c & 4) ? hz1 : hz0;
      const uint32_t od = ((c & 1) ? xb1 : xb0) + b + e;
      const uint32_t oh = ((a ^ b ^ e) & m) | P.base;
      off[c] = (od & dm) | (oh & ~dm);
    }
  }
}

// Lane (sample, level group g) encodes levels g, g+4, g+8, g+12 of one point.
// Levels with LOD weight 0 are not fetched.  feat[2j + f] = level g + 4j,
// feature f.  dense_mask (bit l: level l is stored densely) lets a group of
// four levels that is all hashed (or all dense) use one index formula.
// PRECISE selects the FP64 lattice coordinate (FP32 paths and the encode
// stage entry point).
template <bool TAB16, bool PRECISE>
__device__ __forceinline__ void encode_point(const FieldDev& F, const LevelDev* lv, __amdgpu_buffer_rsrc_t tab,
                                             const float x[3], float lstar, bool active, int g, float feat[8],
                                             uint32_t& fetches) {
  float uh[3];
  double ud[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if constexpr (PRECISE) ud[a] = (double)x[a] - (double)F.amin[a];
    else uh[a] = x[a] - F.amin[a];
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    feat[2 * j] = 0.0f;
    feat[2 * j + 1] = 0.0f;
    const int lev = g + 4 * j;
    if (!active || lev >= (int)F.L) continue;
    const float w = F.lod ? __builtin_amdgcn_fmed3f(lstar + 1.0f - (float)lev, 0.0f, 1.0f) : 1.0f;
    if (!(w > 0.0f)) continue;
    const LevelDev P = lv[lev];
    float fr[3];
    uint32_t i0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if constexpr (PRECISE) i0[a] = base_corner_f64(ud[a], P.s64, P.top64, fr[a]);
      else i0[a] = base_corner_fast(uh[a], P.s_hi, P.below_n, fr[a]);
    }
    uint32_t off[8];
    corner_offsets(F, P, (F.dense_mask >> (4 * j)) & 0xFu, i0, off);
#ifdef VRN_DEBUG_CHECKS
#pragma unroll
    for (int c = 0; c < 8; ++c)
      VRN_DEBUG_COUNT(off[c] - P.base >= (F.Tmask + 1u) * (F.table_f16 ? 4u : 8u), kDbgTableOffset);
#endif
    float v0[8], v1[8];
    if (TAB16) {
      uint32_t raw[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) raw[c] = __builtin_amdgcn_raw_buffer_load_b32(tab, (int)off[c], 0, 0);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        v0[c] = (float)__builtin_bit_cast(_Float16, (uint16_t)(raw[c] & 0xFFFFu));
        v1[c] = (float)__builtin_bit_cast(_Float16, (uint16_t)(raw[c] >> 16));
      }
    } else {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const auto raw = __builtin_amdgcn_raw_buffer_load_b64(tab, (int)off[c], 0, 0);
        v0[c] = __builtin_bit_cast(float, (uint32_t)raw[0]);
        v1[c] = __builtin_bit_cast(float, (uint32_t)raw[1]);
      }
    }
    const float wx[2] = {1.0f - fr[0], fr[0]};
    const float wy[2] = {1.0f - fr[1], fr[1]};
    const float wz[2] = {1.0f - fr[2], fr[2]};
    float acc0 = 0.0f, acc1 = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const float wc = (wx[c & 1] * wy[(c >> 1) & 1]) * wz[c >> 2];
      acc0 = fmaf(wc, v0[c], acc0);
      acc1 = fmaf(wc, v1[c], acc1);
    }
    feat[2 * j] = w * acc0;
    feat[2 * j + 1] = w * acc1;
    VRN_DEBUG_COUNT(feat[2 * j] != feat[2 * j] || feat[2 * j + 1] != feat[2 * j + 1], kDbgFeature);
    ++fetches;
  }
}

// FP16-table encode for the 16-bit MLP paths: same addresses and gathers as
// encode_point, but the trilinear interpolation runs as seven packed FP16
// lerps over both features at once (fractions and LOD weight rounded to
// FP16), and the result stays packed: hfeat[j] = (f0, f1) of level g + 4j,
// the layout the FP16 MFMA operand takes.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ half2_t h2_splat(float v) {
  return __builtin_bit_cast(half2_t, __builtin_amdgcn_cvt_pkrtz(v, v));
}
__device__ __forceinline__ half2_t h2_lerp(half2_t a, half2_t b, half2_t f) {
  return __builtin_elementwise_fma(f, b - a, a);
}

__device__ __forceinline__ void encode_point_h2(const FieldDev& F, const LevelDev* lv, __amdgpu_buffer_rsrc_t tab,
                                                const float x[3], float lstar, bool active, int g,
                                                uint32_t hfeat[4], uint32_t& fetches) {
  float uh[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) uh[a] = x[a] - F.amin[a];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    hfeat[j] = 0u;
    const int lev = g + 4 * j;
    if (!active || lev >= (int)F.L) continue;
    const float w = F.lod ? __builtin_amdgcn_fmed3f(lstar + 1.0f - (float)lev, 0.0f, 1.0f) : 1.0f;
    if (!(w > 0.0f)) continue;
    const LevelDev P = lv[lev];
    float fr[3];
    uint32_t i0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) i0[a] = base_corner_fast(uh[a], P.s_hi, P.below_n, fr[a]);
    uint32_t off[8];
    corner_offsets(F, P, (F.dense_mask >> (4 * j)) & 0xFu, i0, off);
#ifdef VRN_DEBUG_CHECKS
#pragma unroll
    for (int c = 0; c < 8; ++c)
      VRN_DEBUG_COUNT(off[c] - P.base >= (F.Tmask + 1u) * (F.table_f16 ? 4u : 8u), kDbgTableOffset);
#endif
    half2_t v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c)
      v[c] = __builtin_bit_cast(half2_t, __builtin_amdgcn_raw_buffer_load_b32(tab, (int)off[c], 0, 0));
    const half2_t fx = h2_splat(fr[0]), fy = h2_splat(fr[1]), fz = h2_splat(fr[2]);
    const half2_t e00 = h2_lerp(v[0], v[1], fx), e10 = h2_lerp(v[2], v[3], fx);
    const half2_t e01 = h2_lerp(v[4], v[5], fx), e11 = h2_lerp(v[6], v[7], fx);
    const half2_t e0 = h2_lerp(e00, e10, fy), e1 = h2_lerp(e01, e11, fy);
    hfeat[j] = __builtin_bit_cast(uint32_t, h2_lerp(e0, e1, fz) * h2_splat(w));
#ifdef VRN_DEBUG_CHECKS
    {
      const half2_t hv = __builtin_bit_cast(half2_t, hfeat[j]);
      VRN_DEBUG_COUNT(hv[0] != hv[0] || hv[1] != hv[1], kDbgFeature);
    }
#endif
    ++fetches;
  }
}

// Step length of the lattice sample at parameter t (uniform lattice, or
// the FP32 table: t_{k+1} - t_k, with t_{k+1} from the table's recurrence).
template <int GEO>
__device__ __forceinline__ float sample_step(const FieldDev& F, float t) {
  if constexpr (GEO == 0) return F.dt;
  else return table_next(F, t) - t;
}

// L* of a sample of a contracted field: the footprint is the distance between
// the corresponding points of this ray and its right neighbour in contracted
// space (Sec. 4.2.1), in normalised units (the cube edge is 4).
__device__ __forceinline__ float level_star_contracted(const FieldDev& F, const Ray& r, float t, const float y[3]) {
  float yn[3] = {r.ox + t * r.nx, r.oy + t * r.ny, r.oz + t * r.nz};
  contract_point(F, yn);
  const float dx = yn[0] - y[0], dy = yn[1] - y[1], dz = yn[2] - y[2];
  const float rhat = F.lod_radius_scale * 0.25f * __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz);
  return fmaxf(-(__logf(rhat) + F.lod_c2) * F.inv_ln_f + F.lod_bias, 0.0f);
}

// Optimal LOD level L* = -log_f(2 s r_hat) + bias, clamped at 0 (Sec. 4.2.1-2),
// with r_hat = t r / extent and lr = ln(r) + ln(2 s / extent).
__device__ __forceinline__ float level_star(const FieldDev& F, float t, float lr) {
  return fmaxf(-(__logf(t) + lr) * F.inv_ln_f + F.lod_bias, 0.0f);
}

// ---------------------------------------------------------------------------
// Direction encoding: real SH, bands 0..3, no Condon-Shortley phase,
// order (l, m = -l..l).  Constants from the closed-form polynomials.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void sh_basis16(float x, float y, float z, float s[16]) {
  const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, yz = y * z, xz = x * z;
  s[0] = 0.28209479177387814f;
  s[1] = 0.4886025119029199f * y;
  s[2] = 0.4886025119029199f * z;
  s[3] = 0.4886025119029199f * x;
  s[4] = 1.0925484305920792f * xy;
  s[5] = 1.0925484305920792f * yz;
  s[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);
  s[7] = 1.0925484305920792f * xz;
  s[8] = 0.5462742152960396f * (xx - yy);
  s[9] = 0.5900435899266435f * y * (3.0f * xx - yy);
  s[10] = 2.890611442640554f * xy * z;
  s[11] = 0.4570457994644658f * y * (5.0f * zz - 1.0f);
  s[12] = 0.3731763325901154f * z * (5.0f * zz - 3.0f);
  s[13] = 0.4570457994644658f * x * (5.0f * zz - 1.0f);
  s[14] = 1.445305721320277f * z * (xx - yy);
  s[15] = 0.5900435899266435f * x * (xx - 3.0f * yy);
}

// The SH values lane group g feeds to the first color layer: c = g + 4 i.
__device__ __forceinline__ void sh_select(const FieldDev& F, float x, float y, float z, int g, float out[4]) {
  float s[16];
  sh_basis16(x, y, z, s);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float v = g == 0 ? s[4 * i] : g == 1 ? s[4 * i + 1] : g == 2 ? s[4 * i + 2] : s[4 * i + 3];
    out[i] = (uint32_t)(g + 4 * i) < F.nsh ? v : 0.0f;
  }
}

// ---------------------------------------------------------------------------
// MLPs on MFMA (Sec. 5: fused, in-register small MLPs; Sec. 6: 64 wide).
//
// One call evaluates 16 samples.  Every layer computes D^T = W^T X^T with
// 16x16 output tiles: lane l holds output (4 (l >> 4) + r) of sample
// (l & 15) in accumulator register r.  Because the MFMA contraction is
// invariant under any permutation of k that A and B share, that accumulator
// layout is used directly as the B operand of the next layer -- lane group
// g = l >> 4 contributes hidden units {16 t + 4 g + r} -- and the host lays
// the weight fragments out in the same order.  No activation ever leaves
// the registers.  The first layer's B operand is the lane's own encoded
// features (levels g + 4 j); the first color layer's is the lane's density
// outputs 4 g + r (output 0, the density, meets zero weights) followed by
// the SH values g + 4 i.
// Result: lanes 0..15 hold o0 (density pre-activation) and the three color
// logits of samples 0..15.
// ---------------------------------------------------------------------------

__device__ __forceinline__ v4f mfma_f32(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ v4f zero4() {
  v4f z;
  z[0] = z[1] = z[2] = z[3] = 0.0f;
  return z;
}

// The density output bias is added after the MFMA accumulation: it is large
// (several units) next to the products, and adding it last rounds it once.
__device__ __forceinline__ v4f add_bias4(v4f v, const float* sb, int base, int g) {
  v4f r;
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = v[i] + sb[base + 4 * g + i];
  return r;
}

// Hidden layers start the FP32 accumulator at the bias (one 16-byte LDS read,
// no adds); so do all layers of the 16-bit paths.
__device__ __forceinline__ v4f bias_acc(const float* sb, int base, int g) {
  const float4 b = *reinterpret_cast<const float4*>(sb + base + 4 * g);
  v4f r;
  r[0] = b.x;
  r[1] = b.y;
  r[2] = b.z;
  r[3] = b.w;
  return r;
}

// ReLU as one median-of-three (fmaxf would also canonicalise its input)
__device__ __forceinline__ v4f relu4(v4f v) {
  v4f r;
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = __builtin_amdgcn_fmed3f(v[i], 0.0f, 3.0e38f);
  return r;
}

// FP32 path: v_mfma_f32_16x16x4_f32, weights as float4 = 4 consecutive k-steps.
__device__ __forceinline__ void mlp_tile_f32(const float4* __restrict__ sw, const float* __restrict__ sb,
                                             uint32_t d1_groups, const float feat[8],
                                             const float shs[4], int lane, float& o0, float lg[3]) {
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
  o = add_bias4(o, sb, kB2, g);
  v4f c1[4];
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) {
    c1[ot] = bias_acc(sb, kB3 + 16 * ot, g);
    const float4 w0 = sw[kW32_C1 / 4 + (ot * 2 + 0) * 64 + lane];
    c1[ot] = mfma_f32(w0.x, o[0], c1[ot]);
    c1[ot] = mfma_f32(w0.y, o[1], c1[ot]);
    c1[ot] = mfma_f32(w0.z, o[2], c1[ot]);
    c1[ot] = mfma_f32(w0.w, o[3], c1[ot]);
    const float4 w1 = sw[kW32_C1 / 4 + (ot * 2 + 1) * 64 + lane];
    c1[ot] = mfma_f32(w1.x, shs[0], c1[ot]);
    c1[ot] = mfma_f32(w1.y, shs[1], c1[ot]);
    c1[ot] = mfma_f32(w1.z, shs[2], c1[ot]);
    c1[ot] = mfma_f32(w1.w, shs[3], c1[ot]);
  }
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) c1[ot] = relu4(c1[ot]);
  v4f c2[4];
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) {
    c2[ot] = bias_acc(sb, kB4 + 16 * ot, g);
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const float4 w = sw[kW32_C2 / 4 + (ot * 4 + it) * 64 + lane];
      c2[ot] = mfma_f32(w.x, c1[it][0], c2[ot]);
      c2[ot] = mfma_f32(w.y, c1[it][1], c2[ot]);
      c2[ot] = mfma_f32(w.z, c1[it][2], c2[ot]);
      c2[ot] = mfma_f32(w.w, c1[it][3], c2[ot]);
    }
  }
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) c2[ot] = relu4(c2[ot]);
  // color output layer (64 -> 3) on the VALU: 13 of the 16 MFMA output rows
  // would be padding.  Lane (s, g) holds hidden units 16 it + 4 g + r of
  // sample s; the weights W5[16 it + 4 g + r][c] sit in the C3 fragments of
  // lanes 16 g + c.  Each lane dots its 16 units, then the four lane groups
  // of a sample are summed.
  float p[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int it = 0; it < 4; ++it)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float4 w = sw[kW32_C3 / 4 + it * 64 + 16 * g + c];
      p[c] = fmaf(w.x, c2[it][0], p[c]);
      p[c] = fmaf(w.y, c2[it][1], p[c]);
      p[c] = fmaf(w.z, c2[it][2], p[c]);
      p[c] = fmaf(w.w, c2[it][3], p[c]);
    }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    p[c] += __shfl_xor(p[c], 16);
    p[c] += __shfl_xor(p[c], 32);
    lg[c] = p[c] + sb[kB5 + c];
  }
  o0 = o[0];
}

// 16-bit paths: v_mfma_f32_16x16x32_{f16,bf16}; 8 k-values per lane per step.
template <bool BF>
struct Half8 {
  typedef typename std::conditional<BF, v8bf, v8h>::type vec;
  // eight FP32 values rounded to the element type (nearest even)
  __device__ static __forceinline__ vec pack(const float* v) {
    vec r;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if constexpr (BF) r[i] = (__bf16)v[i];
      else r[i] = (_Float16)v[i];
    }
    return r;
  }
  // ReLU of eight FP32 values, rounded to the element type.  Rounding is
  // monotone and maps 0 to 0, so relu(round(x)) = round(relu(x)); the FP16
  // form rounds first and takes the maximum two lanes at a time.
  __device__ static __forceinline__ vec relu_pack(const float* v) {
    if constexpr (BF) {
      float c[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) c[i] = __builtin_amdgcn_fmed3f(v[i], 0.0f, 3.0e38f);
      return pack(c);
    } else {
      typedef _Float16 h2 __attribute__((ext_vector_type(2)));
      const h2 zero = {(_Float16)0.0f, (_Float16)0.0f};
      uint32_t w[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const h2 h = {(_Float16)v[2 * i], (_Float16)v[2 * i + 1]};
        w[i] = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(h, zero));
      }
      vec r;
      __builtin_memcpy(&r, w, 16);
      return r;
    }
  }
  __device__ static __forceinline__ uint16_t bits(float f) {
    if constexpr (BF) return __builtin_bit_cast(uint16_t, (__bf16)f);
    else return __builtin_bit_cast(uint16_t, (_Float16)f);
  }
  // four values rounded to the element type, packed two per 32-bit word
  __device__ static __forceinline__ uint2 pack4(const float* v) {
    return make_uint2((uint32_t)bits(v[0]) | ((uint32_t)bits(v[1]) << 16),
                      (uint32_t)bits(v[2]) | ((uint32_t)bits(v[3]) << 16));
  }
  // first four elements from floats, last four already packed
  __device__ static __forceinline__ vec pack4_raw(const float* v, uint2 raw) {
    const uint2 lo = pack4(v);
    const uint4 u = make_uint4(lo.x, lo.y, raw.x, raw.y);
    vec r;
    __builtin_memcpy(&r, &u, 16);
    return r;
  }
  __device__ static __forceinline__ v4f mfma(vec a, vec b, v4f c) {
    if constexpr (BF) return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <bool BF>
__device__ __forceinline__ void mlp_tile_16(const uint4* __restrict__ sw, const float* __restrict__ sb,
                                            const float feat[8], uint2 shh, int lane, float& o0, float lg[3]) {
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
  v4f h[4];
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) h[ot] = add_bias4(H::mfma(wfrag(kW16_D1, ot), xin, zero4()), sb, kB1 + 16 * ot, g);
  float hv[16];
#pragma unroll
  for (int ot = 0; ot < 4; ++ot)
#pragma unroll
    for (int r = 0; r < 4; ++r) hv[4 * ot + r] = h[ot][r];
  v4f o = zero4();
  o = H::mfma(wfrag(kW16_D2, 0), H::relu_pack(hv), o);
  o = H::mfma(wfrag(kW16_D2, 1), H::relu_pack(hv + 8), o);
  o = add_bias4(o, sb, kB2, g);
  const float oo[4] = {o[0], o[1], o[2], o[3]};
  const vec cv = H::pack4_raw(oo, shh);
  v4f c1[4];
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) c1[ot] = add_bias4(H::mfma(wfrag(kW16_C1, ot), cv, zero4()), sb, kB3 + 16 * ot, g);
#pragma unroll
  for (int ot = 0; ot < 4; ++ot)
#pragma unroll
    for (int r = 0; r < 4; ++r) hv[4 * ot + r] = c1[ot][r];
  const vec a0 = H::relu_pack(hv), a1 = H::relu_pack(hv + 8);
  v4f c2[4];
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) {
    c2[ot] = zero4();
    c2[ot] = H::mfma(wfrag(kW16_C2, ot * 2 + 0), a0, c2[ot]);
    c2[ot] = H::mfma(wfrag(kW16_C2, ot * 2 + 1), a1, c2[ot]);
    c2[ot] = add_bias4(c2[ot], sb, kB4 + 16 * ot, g);
  }
#pragma unroll
  for (int ot = 0; ot < 4; ++ot)
#pragma unroll
    for (int r = 0; r < 4; ++r) hv[4 * ot + r] = c2[ot][r];
  v4f c3 = zero4();
  c3 = H::mfma(wfrag(kW16_C3, 0), H::relu_pack(hv), c3);
  c3 = H::mfma(wfrag(kW16_C3, 1), H::relu_pack(hv + 8), c3);
  c3 = add_bias4(c3, sb, kB5, g);
  o0 = o[0];
  lg[0] = c3[0];
  lg[1] = c3[1];
  lg[2] = c3[2];
}

// The 16-bit MLPs over up to four 16-sample tiles at once: every weight
// fragment is read from LDS once per call and applied to all tiles, so LDS
// traffic for weights falls by the number of tiles.  nt is wave-uniform.
template <bool BF, int NB>
__device__ __forceinline__ void mlp_batch_16(const uint4* __restrict__ sw, const float* __restrict__ sb, int nt,
                                             const typename Half8<BF>::vec xin[NB], const uint2 shh[NB],
                                             int lane, float o0[NB], float lg[NB][3]) {
  typedef Half8<BF> H;
  typedef typename H::vec vec;
  const int g = lane >> 4;
  auto wfrag = [&](int off16, int idx) -> vec {
    const uint4 u = sw[off16 / 8 + idx * 64 + lane];
    vec v;
    __builtin_memcpy(&v, &u, 16);
    return v;
  };
  // one 64-wide hidden layer fed by a single 32-deep B operand per tile;
  // output tiles are produced in pairs so only packed halves stay live
  auto layer_k32 = [&](int off16, int boff, const vec* in, vec out[NB][2]) {
#pragma unroll
    for (int pair = 0; pair < 2; ++pair) {
      const vec w0 = wfrag(off16, 2 * pair), w1 = wfrag(off16, 2 * pair + 1);
#pragma unroll
      for (int t = 0; t < NB; ++t)
        if (t < nt) {
          const v4f a = H::mfma(w0, in[t], bias_acc(sb, boff + 32 * pair, g));
          const v4f b = H::mfma(w1, in[t], bias_acc(sb, boff + 32 * pair + 16, g));
          const float hv[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
          out[t][pair] = H::relu_pack(hv);
        }
    }
  };
  vec hp[NB][2];
  layer_k32(kW16_D1, kB1, xin, hp);
  v4f o[NB];
  {
    const vec w0 = wfrag(kW16_D2, 0), w1 = wfrag(kW16_D2, 1);
#pragma unroll
    for (int t = 0; t < NB; ++t)
      if (t < nt) o[t] = H::mfma(w1, hp[t][1], H::mfma(w0, hp[t][0], bias_acc(sb, kB2, g)));
  }
  vec cv[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t)
    if (t < nt) {
      const float oo[4] = {o[t][0], o[t][1], o[t][2], o[t][3]};
      cv[t] = H::pack4_raw(oo, shh[t]);
    }
  vec c1p[NB][2];
  layer_k32(kW16_C1, kB3, cv, c1p);
  vec c2p[NB][2];
#pragma unroll
  for (int pair = 0; pair < 2; ++pair) {
    const vec wa0 = wfrag(kW16_C2, 4 * pair + 0), wa1 = wfrag(kW16_C2, 4 * pair + 1);
    const vec wb0 = wfrag(kW16_C2, 4 * pair + 2), wb1 = wfrag(kW16_C2, 4 * pair + 3);
#pragma unroll
    for (int t = 0; t < NB; ++t)
      if (t < nt) {
        const v4f a = H::mfma(wa1, c1p[t][1], H::mfma(wa0, c1p[t][0], bias_acc(sb, kB4 + 32 * pair, g)));
        const v4f b = H::mfma(wb1, c1p[t][1], H::mfma(wb0, c1p[t][0], bias_acc(sb, kB4 + 32 * pair + 16, g)));
        const float hv[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
        c2p[t][pair] = H::relu_pack(hv);
      }
  }
  v4f c3[NB];
  {
    const vec w0 = wfrag(kW16_C3, 0), w1 = wfrag(kW16_C3, 1);
#pragma unroll
    for (int t = 0; t < NB; ++t)
      if (t < nt) c3[t] = H::mfma(w1, c2p[t][1], H::mfma(w0, c2p[t][0], bias_acc(sb, kB5, g)));
  }
#pragma unroll
  for (int t = 0; t < NB; ++t)
    if (t < nt) {
      o0[t] = o[t][0];
      lg[t][0] = c3[t][0];
      lg[t][1] = c3[t][1];
      lg[t][2] = c3[t][2];
    }
}

// ---------------------------------------------------------------------------
// FP32-accurate MLP on the BF16 MFMA (VRN_F32X).  Every FP32 operand is the
// exact sum of three BF16 parts, x = x0 + x1 + x2: each part is the
// residual of the previous ones rounded to the nearest BF16.  The residuals
// are exact in FP32 (Sterbenz), and the last holds at most 7 significant
// bits, so it is exact in BF16 too.  A product x w keeps the six part
// products whose orders sum to at most 2; the dropped ones (x1 w2, x2 w1,
// x2 w2) total about 2^-26 |x w|, below FP32's own rounding of the product.
// BF16 products are exact in FP32 and the MFMA accumulates in FP32, so the
// layer matches FP32 arithmetic to within its rounding, at the BF16 MFMA
// rate (six 16x16x32 steps in place of eight 16x16x4 FP32 ones per 32-deep
// step), and the BF16 MFMA co-executes with VALU work where the FP32 one
// does not.  Weights are split on the host into the BF16 fragment layout:
// [part][kW16Total].
// ---------------------------------------------------------------------------
struct Bf3 {
  v8bf p[3];
};

__device__ __forceinline__ Bf3 split_bf3(const float* v) {
  Bf3 s;
  float r[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = v[i];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const __bf16 b = (__bf16)r[i];
      s.p[k][i] = b;
      if (k < 2) r[i] = r[i] - (float)b;
    }
  return s;
}

__device__ __forceinline__ v4f mfma_bf16(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// c + W x over one 32-deep step, the smallest part products first.
__device__ __forceinline__ v4f mfma_bf3(const Bf3& w, const Bf3& x, v4f c) {
  c = mfma_bf16(w.p[1], x.p[1], c);
  c = mfma_bf16(w.p[2], x.p[0], c);
  c = mfma_bf16(w.p[0], x.p[2], c);
  c = mfma_bf16(w.p[1], x.p[0], c);
  c = mfma_bf16(w.p[0], x.p[1], c);
  return mfma_bf16(w.p[0], x.p[0], c);
}

// The three parts of weight fragment idx of a layer (offset off16 in the
// BF16 fragment layout; the parts lie `stride` 16-bit values apart).
__device__ __forceinline__ Bf3 wfrag_bf3(const uint4* __restrict__ sw3, int stride, int off16, int idx, int lane) {
  Bf3 w;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint4 u = sw3[(k * stride + off16) / 8 + idx * 64 + lane];
    __builtin_memcpy(&w.p[k], &u, 16);
  }
  return w;
}

// The same layers, in the same register layouts, as mlp_tile_f32; the
// color output layer (64 -> 3) runs on the VALU in FP32 from the FP32 C3
// fragments (sw_c3 = the kW32_C3 block).
__device__ __forceinline__ void mlp_tile_x3(const uint4* __restrict__ sw3, const float4* __restrict__ sw_c3,
                                            const float* __restrict__ sb, const float feat[8], const float shs[4],
                                            int lane, float& o0, float lg[3]) {
  const int g = lane >> 4;
  const Bf3 xin = split_bf3(feat);
  float hv[16];
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) {
    const v4f h = relu4(mfma_bf3(wfrag_bf3(sw3, kW16Total, kW16_D1, ot, lane), xin, bias_acc(sb, kB1 + 16 * ot, g)));
#pragma unroll
    for (int r = 0; r < 4; ++r) hv[4 * ot + r] = h[r];
  }
  v4f o = mfma_bf3(wfrag_bf3(sw3, kW16Total, kW16_D2, 0, lane), split_bf3(hv), zero4());
  o = mfma_bf3(wfrag_bf3(sw3, kW16Total, kW16_D2, 1, lane), split_bf3(hv + 8), o);
  o = add_bias4(o, sb, kB2, g);
  const float cin[8] = {o[0], o[1], o[2], o[3], shs[0], shs[1], shs[2], shs[3]};
  const Bf3 cv = split_bf3(cin);
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) {
    const v4f c = relu4(mfma_bf3(wfrag_bf3(sw3, kW16Total, kW16_C1, ot, lane), cv, bias_acc(sb, kB3 + 16 * ot, g)));
#pragma unroll
    for (int r = 0; r < 4; ++r) hv[4 * ot + r] = c[r];
  }
  const Bf3 a0 = split_bf3(hv), a1 = split_bf3(hv + 8);
  v4f c2[4];
#pragma unroll
  for (int ot = 0; ot < 4; ++ot) {
    const v4f c = mfma_bf3(wfrag_bf3(sw3, kW16Total, kW16_C2, 2 * ot, lane), a0, bias_acc(sb, kB4 + 16 * ot, g));
    c2[ot] = relu4(mfma_bf3(wfrag_bf3(sw3, kW16Total, kW16_C2, 2 * ot + 1, lane), a1, c));
  }
  float p[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int it = 0; it < 4; ++it)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float4 w = sw_c3[it * 64 + 16 * g + c];
      p[c] = fmaf(w.x, c2[it][0], p[c]);
      p[c] = fmaf(w.y, c2[it][1], p[c]);
      p[c] = fmaf(w.z, c2[it][2], p[c]);
      p[c] = fmaf(w.w, c2[it][3], p[c]);
    }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    p[c] += __shfl_xor(p[c], 16);
    p[c] += __shfl_xor(p[c], 32);
    lg[c] = p[c] + sb[kB5 + c];
  }
  o0 = o[0];
}

// ---------------------------------------------------------------------------
// PQ decode (Sec. 4.1, algebraic inverse of Eq. 1), linear 1 = 100 cd/m^2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float pq_to_linear(float e) {
  const float m1 = 1305.0f / 8192.0f, m2 = 2523.0f / 32.0f;
  const float c1 = 107.0f / 128.0f, c2 = 2413.0f / 128.0f, c3 = 2392.0f / 128.0f;
  const float ep = powf(fmaxf(e, 0.0f), 1.0f / m2);
  const float y = powf(fmaxf(ep - c1, 0.0f) / (c2 - c3 * ep), 1.0f / m1);
  return 100.0f * y;
}

// sRGB transfer (IEC 61966-2-1) of a linear value clipped to [0, 1].
__device__ __forceinline__ float srgb_oetf(float v) {
  v = __builtin_amdgcn_fmed3f(v, 0.0f, 1.0f);
  return v <= 0.0031308f ? 12.92f * v : 1.055f * powf(v, 1.0f / 2.4f) - 0.055f;
}

}  // namespace vrn
