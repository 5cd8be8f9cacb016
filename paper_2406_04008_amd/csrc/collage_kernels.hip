// HIP kernels (gfx950, wave64) of the image-space collage hot path.
//
// One epoch is a short chain of launches with grids fixed by the scene:
//   k_transform  one wave per item: eq. 2 applied to the outline in double precision; float edge
//                records for the scan and double edge records for the per-pixel evaluation, both
//                relative to the item's origin; the pixel box of the item's coverage support; the
//                outline orientation.  (Within a multi-epoch call the update kernel does this for the
//                next epoch.)
//   k_bin        one workgroup per screen tile: the layout's items whose support box meets the tile,
//                in item order; each (tile, item) is a work unit, the box clipped to the tile, packed
//                row by row into 64-pixel chunks, stored in the layout's unit pool without gaps (a
//                tile's first unit is the number of the layout's units in earlier tiles, summed from
//                each item's tile span).  Clears the tile's coverage accumulators.  (Large scenes:
//                k_rowbin first lists each tile row's items and its first unit.)
//   k_scan       one workgroup: prefix sums of the tiles' work costs and chunk counts (up to
//                kScanInCoverTiles tiles every coverage workgroup computes them itself instead).
//   k_cover      persistent waves, each taking an equal share of the pass's cost (split at chunk
//                granularity); per unit the wave stages the item's edge records in LDS, and per chunk
//                every lane scans them in float32 for its pixel's nearest edge and crossing parity,
//                then evaluates the signed distance and the coverage in double precision and adds
//                them to S and S_pad as 2^-40 fixed point with 64-bit integer atomics (exact, so the
//                result does not depend on the order of the work).  Backward calls keep a 2-byte
//                nearest-edge code per (chunk, lane).
//   k_pixel      one workgroup per 32 x 32 pixel tile: S, S_pad, the loss terms (summed per tile in a
//                fixed order) and dLoss/dS, dLoss/dS_pad per pixel; with the uniform term on, also the
//                tile's window occupancies from a summed-area table of the tile and its halo.
//   k_unif_grad  (uniform term on) the same tiles: the term's share of dLoss/dS from window sums of
//                the pixels' active-window bits.
//   k_adjoint    persistent waves again: per chunk, the gradient terms of its pixels (double), summed
//                per piece of a unit (the chunks of the unit in one wave's share) and added into the
//                unit's head partials in 2^-30 fixed point with 64-bit integer atomics (each pixel's
//                terms rounded first, so every sum is exact).
//   k_vgrad,     (outline-vertex gradients only) the adjoint's walk once more, adding each pixel's
//   k_vfinal     d sd / d(end points of its nearest edge) into per-vertex fixed-point sums, then back
//                through eq. 2 per vertex.
//   k_finalize   one wave per item (two or four items per workgroup) sums its units' head partials in
//                a fixed order (gradient, then the optional Adam update and the next epoch's
//                transform); one workgroup per layout sums the loss blocks in a fixed order.
// Bulk outputs that later kernels read are written with nontemporal stores.  Results are bitwise
// reproducible.
#include "collage_internal.h"

#include <hip/hip_ext.h>

#include <math.h>

#include <mutex>

namespace collage {

template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

// Read-only data that a kernel never writes: loads with wave-uniform addresses go through the scalar
// cache and land in SGPRs (one load serves all 64 lanes).
template <typename T>
__device__ __forceinline__ cptr<T> konst(const T *p) {
  return (cptr<T>)(p);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uniform_ll(long long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ int4 load_box(cptr<BinRec> p, int i) {
  cptr<int> q = (cptr<int>)(p + i);
  return make_int4(q[0], q[1], q[2], q[3]);
}

// v moved between lanes by the DPP control CTRL (rows outside ROW_MASK and lanes whose source is out of
// the row read 0); the two 32-bit halves move separately.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v, unsigned long long old = 0ull) {
  const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)old, (int)(unsigned)v, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(old >> 32), (int)(unsigned)(v >> 32), CTRL, ROW_MASK,
                                             0xf, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned dpp_u32(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, false);
}

// Inclusive prefix sum over the 64 lanes of a wave: Hillis-Steele within each row of 16 lanes
// (row_shr 1, 2, 4, 8), then the last lane of row 0 / 2 added into row 1 / 3 (row_bcast 15) and the last
// lane of row 1 into rows 2 and 3 (row_bcast 31).
__device__ __forceinline__ unsigned long long wave_incl_scan_u64(unsigned long long v) {
  v += dpp_u64<0x111, 0xf>(v);
  v += dpp_u64<0x112, 0xf>(v);
  v += dpp_u64<0x114, 0xf>(v);
  v += dpp_u64<0x118, 0xf>(v);
  v += dpp_u64<0x142, 0xa>(v);
  v += dpp_u64<0x143, 0xc>(v);
  return v;
}

// Sum over the 64 lanes of a wave in a fixed order (the scan pattern of wave_incl_scan_u64 with double
// additions; the total ends in lane 63 and is broadcast from there).  Every lane must be active.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += __longlong_as_double((long long)dpp_u64<0x111, 0xf>((unsigned long long)__double_as_longlong(v)));
  v += __longlong_as_double((long long)dpp_u64<0x112, 0xf>((unsigned long long)__double_as_longlong(v)));
  v += __longlong_as_double((long long)dpp_u64<0x114, 0xf>((unsigned long long)__double_as_longlong(v)));
  v += __longlong_as_double((long long)dpp_u64<0x118, 0xf>((unsigned long long)__double_as_longlong(v)));
  v += __longlong_as_double((long long)dpp_u64<0x142, 0xa>((unsigned long long)__double_as_longlong(v)));
  v += __longlong_as_double((long long)dpp_u64<0x143, 0xc>((unsigned long long)__double_as_longlong(v)));
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)bits, 63);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)bits >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The sum over a wave's 64 lanes (every lane active), broadcast to all of them.
__device__ __forceinline__ double wave_sum(double v) { return wave_sum_dpp(v); }

// DPP controls whose source lane always exists: the partner across lane bit 0 or bit 1 within a quad
// (quad permutations [1,0,3,2] and [2,3,0,1]), and rotations by 4 and 8 lanes within a row of 16.
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E, kRowRor4 = 0x124, kRowRor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return __longlong_as_double((long long)dpp_u64<CTRL, 0xf>(b, b));
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The value of lane l ^ 16 (ROWS = 16) or l ^ 32 (ROWS = 32) in registers: v_permlane16_swap exchanges
// the odd rows of 16 lanes of its first operand with the even rows of its second, v_permlane32_swap the
// upper half of the first with the lower half of the second, so with x in both the partner's value is
// in one of the two results.  (No LDS round trip, unlike a shuffle.)
template <int ROWS>
__device__ __forceinline__ unsigned xor_rows_u32(unsigned x) {
  const bool upper = ((threadIdx.x & 63) & ROWS) != 0;
  if constexpr (ROWS == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return upper ? r[0] : r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return upper ? r[0] : r[1];
  }
}

template <int ROWS>
__device__ __forceinline__ double xor_rows_f64(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = xor_rows_u32<ROWS>((unsigned)b), hi = xor_rows_u32<ROWS>((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Wave sums of several values at once (every lane active), in a fixed order.  Each lane gives half of
// its values to the partner across lane bit 0 and adds the other half from it, then the same across
// bit 1, so that from there on it sums a quarter of the values: over the 16 lanes of the same quad
// position, by two rotations within each row of 16 and two exchanges across rows.  Four values cost
// about a quarter of the instructions of four full reductions.
// wave_sum4: lane l ends with the total of component comp = 2 (l & 1) + ((l >> 1) & 1) of (x, y, z, w)
// (lanes 0, 1, 2, 3 hold x, z, y, w).
__device__ __forceinline__ double wave_sum4(double4 v, int &comp) {
  const int lane = threadIdx.x & 63;
  const bool o1 = (lane & 1) != 0, o2 = (lane & 2) != 0;
  double k0 = o1 ? v.z : v.x, k1 = o1 ? v.w : v.y;  // kept: (x, y) on even lanes, (z, w) on odd ones
  k0 += dpp_f64<kQuadXor1>(o1 ? v.x : v.z);          // the partner's share of what this lane keeps
  k1 += dpp_f64<kQuadXor1>(o1 ? v.y : v.w);
  double m = o2 ? k1 : k0;
  m += dpp_f64<kQuadXor2>(o2 ? k0 : k1);
  m += dpp_f64<kRowRor4>(m);
  m += dpp_f64<kRowRor8>(m);
  m += xor_rows_f64<16>(m);
  m += xor_rows_f64<32>(m);
  comp = (o1 ? 2 : 0) + (o2 ? 1 : 0);
  return m;
}

// wave_sum8: lane l ends with the totals of components c0 = 4 (l & 1) + 2 ((l >> 1) & 1) and c0 + 1 of v
// (lanes 0-3 hold all eight).
__device__ __forceinline__ double2 wave_sum8(const double (&v)[8], int &c0) {
  const int lane = threadIdx.x & 63;
  const bool o1 = (lane & 1) != 0, o2 = (lane & 2) != 0;
  double k[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    k[i] = o1 ? v[i + 4] : v[i];
    k[i] += dpp_f64<kQuadXor1>(o1 ? v[i] : v[i + 4]);
  }
  double m0 = o2 ? k[2] : k[0], m1 = o2 ? k[3] : k[1];
  m0 += dpp_f64<kQuadXor2>(o2 ? k[0] : k[2]);
  m1 += dpp_f64<kQuadXor2>(o2 ? k[1] : k[3]);
  m0 += dpp_f64<kRowRor4>(m0);
  m1 += dpp_f64<kRowRor4>(m1);
  m0 += dpp_f64<kRowRor8>(m0);
  m1 += dpp_f64<kRowRor8>(m1);
  m0 += xor_rows_f64<16>(m0);
  m1 += xor_rows_f64<16>(m1);
  m0 += xor_rows_f64<32>(m0);
  m1 += xor_rows_f64<32>(m1);
  c0 = (o1 ? 4 : 0) + (o2 ? 2 : 0);
  return make_double2(m0, m1);
}

__device__ __forceinline__ unsigned long long readlane63_u64(unsigned long long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

// Inclusive prefix sum of 32-bit values over the wave (the DPP pattern of wave_incl_scan_u64).
__device__ __forceinline__ unsigned wave_incl_scan_u32(unsigned v) {
  v += dpp_u32<0x111, 0xf>(v);
  v += dpp_u32<0x112, 0xf>(v);
  v += dpp_u32<0x114, 0xf>(v);
  v += dpp_u32<0x118, 0xf>(v);
  v += dpp_u32<0x142, 0xa>(v);
  v += dpp_u32<0x143, 0xc>(v);
  return v;
}

// Sum over the wave's lanes (every lane active), broadcast.
__device__ __forceinline__ long long wave_sum_ll(long long v) {
  return (long long)readlane63_u64(wave_incl_scan_u64((unsigned long long)v));
}

// Minimum and maximum over the wave's lanes (every lane active), broadcast: the scan pattern with the
// operation's identity moved into lanes without a source.
template <bool MAX>
__device__ __forceinline__ double wave_extreme(double x) {
  const unsigned long long id = (unsigned long long)__double_as_longlong(MAX ? -INFINITY : INFINITY);
  unsigned long long v = (unsigned long long)__double_as_longlong(x);
#define COLLAGE_EXT_STEP(CTRL, MASK)                                                      \
  {                                                                                       \
    const double o = __longlong_as_double((long long)dpp_u64<CTRL, MASK>(v, id));         \
    const double c = __longlong_as_double((long long)v);                                  \
    v = (unsigned long long)__double_as_longlong(MAX ? fmax(c, o) : fmin(c, o));          \
  }
  COLLAGE_EXT_STEP(0x111, 0xf)
  COLLAGE_EXT_STEP(0x112, 0xf)
  COLLAGE_EXT_STEP(0x114, 0xf)
  COLLAGE_EXT_STEP(0x118, 0xf)
  COLLAGE_EXT_STEP(0x142, 0xa)
  COLLAGE_EXT_STEP(0x143, 0xc)
#undef COLLAGE_EXT_STEP
  return __longlong_as_double((long long)readlane63_u64(v));
}

__device__ __forceinline__ double wave_min(double v) { return wave_extreme<false>(v); }
__device__ __forceinline__ double wave_max(double v) { return wave_extreme<true>(v); }

// The bias corrections 1 - beta^t of step t, computed in one place for every caller so that all update
// paths round them alike.  beta^t by binary powering in double (at most 2 log2 t + 2 products, so a
// relative error below 1e-14): 1 - beta^t then rounds to the float nearest the exact value except in
// rare near-halfway cases, with a dependent chain far shorter than a general float power function.
__device__ __forceinline__ float2 adam_bias_of(const KArgs &a, int32_t t) {
  double p1 = 1.0, p2 = 1.0, b1 = (double)a.beta1, b2 = (double)a.beta2;
  for (unsigned n = t > 0 ? (unsigned)t : 0u; n != 0u; n >>= 1) {
    if (n & 1u) {
      p1 *= b1;
      p2 *= b2;
    }
    b1 *= b1;
    b2 *= b2;
  }
  return make_float2((float)(1.0 - p1), (float)(1.0 - p2));
}

__device__ __forceinline__ int layout_of_shape(cptr<LayoutRec> L, int B, int sid) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (L[mid].shape_begin <= sid)
      lo = mid;
    else
      hi = mid - 1;
  }
  // skip empty layouts that share shape_begin with the one that really holds sid
  while (lo < B - 1 && L[lo].shape_end <= sid) ++lo;
  return lo;
}

__device__ __forceinline__ int layout_of_tile(cptr<LayoutRec> L, int B, int tile) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (L[mid].tile_off <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------------------------------------
// k_transform: eq. 2 for every vertex, edge records, support box, orientation.
// ------------------------------------------------------------------------------------------------
// Nontemporal (streaming) vector stores for bulk outputs that later kernels read, mostly from other XCDs:
// the lines leave this XCD's L2 as they are written instead of being written back when the kernel
// ends (measured: update kernel 8.3 -> 7.5 us, per-pixel pass 6.9 -> 6.1 us, binning 5.5 -> 5.3 us).
typedef float nt_f32x4 __attribute__((ext_vector_type(4)));
typedef double nt_f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned long long nt_u64x2 __attribute__((ext_vector_type(2)));
static_assert(sizeof(EdgeRec) == 2 * sizeof(nt_f32x4) && sizeof(EdgeD) == 3 * sizeof(nt_f64x2), "record sizes");

__device__ __forceinline__ void stream_store(EdgeRec *dst, const EdgeRec &r) {
  const nt_f32x4 *src = reinterpret_cast<const nt_f32x4 *>(&r);
  nt_f32x4 *d = reinterpret_cast<nt_f32x4 *>(dst);
  __builtin_nontemporal_store(src[0], d);
  __builtin_nontemporal_store(src[1], d + 1);
}

__device__ __forceinline__ void stream_store(EdgeD *dst, const EdgeD &r) {
  const nt_f64x2 *src = reinterpret_cast<const nt_f64x2 *>(&r);
  nt_f64x2 *d = reinterpret_cast<nt_f64x2 *>(dst);
#pragma unroll
  for (int i = 0; i < 3; ++i) __builtin_nontemporal_store(src[i], d + i);
}

// 1 / x for a positive normal double: the hardware estimate and two Newton steps (each doubles the
// correct bits; the result is within an ulp or two of the quotient, at a third of the instructions of a
// correctly rounded division).
__device__ __forceinline__ double rcp_refined(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

__device__ __forceinline__ void place_vertex(double c, double sn, double s, double k, float2 v, double &x, double &y) {
  const double sx = s * (double)v.x, sy = s * (double)v.y;
  x = k * (c * sx - sn * sy);
  y = k * (sn * sx + c * sy);
}

// What the transform of an item reads besides its parameters: loaded ahead of the parameters where
// those come out of the same kernel (the update), so that the loads overlap the work before it.
constexpr int kTransformPre = 2;  // edges per lane loaded ahead (items of up to 128 edges)
struct TransformPre {
  int v0, n, ec;
  float wst;                        // stroke half-width, 0 for a closed item
  float2 va[kTransformPre], vb[kTransformPre];  // end points of edges lane + 64 r
};

__device__ __forceinline__ int transform_edge_end(bool open, int n, int m) {
  // an open item has edges between consecutive vertices only (a single vertex: one point edge)
  return open ? min(m + 1, n - 1) : (m + 1 == n ? 0 : m + 1);
}

// What lanes past an item's last edge, and items without a stroke array, load (global memory, like the
// arrays they stand in for, so that the loads stay plain global loads).
__device__ float2 kNoVertex = {0.0f, 0.0f};
__device__ float kNoFloat = 0.0f;

// The loads are unconditional (lanes without an edge read kNoVertex), so that nothing consumes their
// results before the caller does.
__device__ __forceinline__ TransformPre transform_preload(const KArgs &a, int sid, int lane) {
  TransformPre t;
  t.v0 = a.vert_off[sid];
  t.n = a.vert_off[sid + 1] - t.v0;
  t.wst = *(a.stroke ? a.stroke + sid : &kNoFloat);
  const bool open = t.wst > 0.0f;
  t.ec = open ? (t.n > 1 ? t.n - 1 : t.n) : t.n;
  const float2 *V = reinterpret_cast<const float2 *>(a.verts) + t.v0;
#pragma unroll
  for (int r = 0; r < kTransformPre; ++r) {
    const int m = lane + 64 * r;
    const bool has = m < t.ec;
    t.va[r] = *(has ? V + m : &kNoVertex);
    t.vb[r] = *(has ? V + transform_edge_end(open, t.n, m) : &kNoVertex);
  }
  return t;
}

// An empty asm statement that takes the preloaded vertices as read and rewritten: the compiler cannot
// move their conversions ahead of it, so the loads stay in flight through the work in between.
__device__ __forceinline__ void transform_hold(TransformPre &t) {
#pragma unroll
  for (int r = 0; r < kTransformPre; ++r)
    asm volatile("" : "+v"(t.va[r].x), "+v"(t.va[r].y), "+v"(t.vb[r].x), "+v"(t.vb[r].y));
}

// One wave transforms item sid with parameters p (the same in every lane).
__device__ void transform_item(const KArgs &a, int sid, int lane, float4 p, const TransformPre &tp) {
  cptr<LayoutRec> LS = konst(a.layouts);
  const int b = layout_of_shape(LS, a.num_layouts, sid);
  const double k = (double)LS[b].k;
  const int W = LS[b].W, H = LS[b].H;
  const int v0 = tp.v0, n = tp.n, ec = tp.ec;
  const bool finite = isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(p.w);
  double sn, c;
  sincos(finite ? (double)p.z : 0.0, &sn, &c);
  const double s = finite ? (double)p.w : 1.0;
  const double cx = k * (double)p.x, cy = k * (double)p.y;
  const float2 *V = reinterpret_cast<const float2 *>(a.verts) + v0;
  if (a.vacc)
    for (int m = lane; m < 2 * n; m += 64) a.vacc[2 * v0 + m] = 0ull;
  const float wst = tp.wst;
  const bool open = wst > 0.0f;
  double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY, area2 = 0.0;
  for (int r = 0, m = lane; m < ec; ++r, m += 64) {
    float2 va, vb;
    static_assert(kTransformPre == 2, "the preloaded edges are picked by r == 0 / r == 1");
    if (r < kTransformPre) {
      va = r == 0 ? tp.va[0] : tp.va[1];
      vb = r == 0 ? tp.vb[0] : tp.vb[1];
    } else {
      va = V[m];
      vb = V[transform_edge_end(open, n, m)];
    }
    double ax, ay, bx, by;
    place_vertex(c, sn, s, k, va, ax, ay);
    place_vertex(c, sn, s, k, vb, bx, by);
    const double ex = bx - ax, ey = by - ay;
    const double ee = ex * ex + ey * ey;
    const double inv = ee > 0.0 ? 1.0 / ee : 0.0;
    EdgeRec er;
    er.ax = (float)ax;
    er.ay = (float)ay;
    er.exs = (float)(ex * inv);
    er.eys = (float)(ey * inv);
    er.ex = (float)ex;
    er.ey = (float)ey;
    er.by = (float)by;  // equals the next edge's ay: the same double rounded the same way
    er.slope = ey != 0.0 ? (float)(ex / ey) : 0.0f;
    stream_store(a.edges + v0 + m, er);
    EdgeD rd;
    rd.ax = ax;
    rd.ay = ay;
    rd.ex = ex;
    rd.ey = ey;
    rd.inv_ee = inv;
    rd.inv_len = sqrt(inv);
    stream_store(a.edges_d + v0 + m, rd);
    mnx = fmin(mnx, fmin(ax, bx));
    mxx = fmax(mxx, fmax(ax, bx));
    mny = fmin(mny, fmin(ay, by));
    mxy = fmax(mxy, fmax(ay, by));
    area2 += ax * by - bx * ay;
  }
  mnx = wave_min(mnx);
  mny = wave_min(mny);
  mxx = wave_max(mxx);
  mxy = wave_max(mxy);
  area2 = wave_sum(area2);
  // stroke radius of an open item: the half-width transformed with the item, and its derivative in s
  const double sw = open ? k * fabs(s) * (double)wst : 0.0;
  const double sw_ds = open ? k * (double)wst * (s > 0.0 ? 1.0 : (s < 0.0 ? -1.0 : 0.0)) : 0.0;
  if (lane == 0) {
    const double ext = (double)a.r_cut + fmax((double)a.r_pad, 0.0) + sw;
    int4 box = make_int4(1, 1, 0, 0);  // empty
    if (n > 0 && finite) {
      // pixel centres i + 1/2 in [cx + mnx - ext, cx + mxx + ext] (widened by 1e-6 px against
      // rounding): a pixel farther than ext from the vertex box is farther than ext from the outline,
      // where both alpha and alpha_pad are cut to zero
      double fx0 = ceil(cx + mnx - ext - 0.5 - 1e-6), fx1 = floor(cx + mxx + ext - 0.5 + 1e-6);
      double fy0 = ceil(cy + mny - ext - 0.5 - 1e-6), fy1 = floor(cy + mxy + ext - 0.5 + 1e-6);
      fx0 = fmax(fx0, 0.0);
      fy0 = fmax(fy0, 0.0);
      fx1 = fmin(fx1, (double)(W - 1));
      fy1 = fmin(fy1, (double)(H - 1));
      if (fx0 <= fx1 && fy0 <= fy1) box = make_int4((int)fx0, (int)fy0, (int)fx1, (int)fy1);
    }
    BinRec br;
    br.box = box;
    br.eo = v0;
    br.ecnv = ec | (n << 16);
    br.flags = (open ? kUnitOpen : 0) | (area2 >= 0.0 ? 0 : kUnitClockwise);
    br.s = p.w;
    br.cx = cx;
    br.cy = cy;
    a.bins[sid] = br;
    ShapeRec sr;
    sr.cx = cx;
    sr.cy = cy;
    sr.k = (float)k;
    sr.s = p.w;
    sr.orient = area2 >= 0.0 ? 1.0f : -1.0f;
    sr.edge_off = v0;
    sr.edge_cnt = ec;
    sr.layout = b;
    sr.bad = finite ? 0 : 1;
    sr.open = open ? 1 : 0;
    sr.sw = sw;
    sr.sw_ds = sw_ds;
    sr.kc = k * c;
    sr.ks = k * sn;
    a.shapes[sid] = sr;
  }
}

__global__ __launch_bounds__(256) void k_transform(KArgs a) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (blockIdx.x == 0 && threadIdx.x < kStatusWords) a.status[threadIdx.x] = 0;
  const int sid = blockIdx.x * 4 + wave;
  if (sid >= a.num_shapes) return;
  transform_item(a, sid, lane, reinterpret_cast<const float4 *>(a.params)[sid], transform_preload(a, sid, lane));
}

// ------------------------------------------------------------------------------------------------
// The float32 edge scan (the hot inner loop): nearest edge and crossing parity.
// ------------------------------------------------------------------------------------------------
// Two consecutive edge records (16 floats), loaded with one scalar-cache load into SGPRs.
typedef float f32x16 __attribute__((ext_vector_type(16), aligned(4)));
typedef const __attribute__((address_space(4))) f32x16 *cptr16;

struct Edge2 {
  f32x16 v;
};

__device__ __forceinline__ Edge2 load_edge2(cptr<float> F, int e) {
  Edge2 r;
  r.v = *(cptr16)(F + 8 * e);
  return r;
}

// One edge of the scan: squared distance (tracked minimum and its index) and the crossing test.
// r0..r7 = ax, ay, exs, eys, ex, ey, by, slope.
__device__ __forceinline__ void scan_one(float ax, float ay, float exs, float eys, float ex, float ey, float by,
                                         float slope, int e, float rx, float ry, float &best, int &idx, bool &par) {
  const float wx = rx - ax, wy = ry - ay;
  const float s = fmaf(wx, exs, wy * eys);
  const float u = __builtin_amdgcn_fmed3f(s, 0.0f, 1.0f);
  const float qx = fmaf(-u, ex, wx), qy = fmaf(-u, ey, wy);
  const float d2 = fmaf(qx, qx, qy * qy);
  if (d2 < best) {
    best = d2;
    idx = e;
  }
  const bool c1 = ay > ry, c2 = by > ry;
  const bool xt = wx < wy * slope;
  par ^= ((c1 != c2) && xt);
}

// Nearest edge (lowest index among equal float distances) of one item, and the even-odd parity of
// the crossings of the ray from the pixel towards +x (half-open rule on the vertex ordinates).
// Edge records are fetched two pairs ahead of their use so that the scalar-load latency overlaps the
// arithmetic; the fetch may run up to four records past the item's last edge (the edge array is
// padded by four records).
__device__ __forceinline__ void edge_scan(cptr<EdgeRec> E, int cnt, float rx, float ry, int &bi, bool &par) {
  cptr<float> F = (cptr<float>)E;
  float best = INFINITY;
  int idx = 0;
  bool pr = false;
  Edge2 cur = load_edge2(F, 0);
  Edge2 nxt = load_edge2(F, 2);
  int e = 0;
  for (; e + 2 <= cnt; e += 2) {
    const Edge2 nn = load_edge2(F, e + 4);
    scan_one(cur.v[0], cur.v[1], cur.v[2], cur.v[3], cur.v[4], cur.v[5], cur.v[6], cur.v[7], e, rx, ry, best, idx, pr);
    scan_one(cur.v[8], cur.v[9], cur.v[10], cur.v[11], cur.v[12], cur.v[13], cur.v[14], cur.v[15], e + 1, rx, ry, best,
             idx, pr);
    cur = nxt;
    nxt = nn;
  }
  if (e < cnt)
    scan_one(cur.v[0], cur.v[1], cur.v[2], cur.v[3], cur.v[4], cur.v[5], cur.v[6], cur.v[7], e, rx, ry, best, idx, pr);
  bi = idx;
  par = pr;
}

// Signed distance (double) from (rx, ry) to edge e; u is the clamped parameter of the nearest point
// and (qx, qy) = p - nearest point.
struct PairD {
  double sd, d, u, qx, qy;
  double inv_d;  // 1 / d (0 at d = 0)
};

__device__ __forceinline__ void pair_d2(const EdgeD &e, double rx, double ry, double &d2, double &u, double &qx,
                                        double &qy) {
  const double wx = rx - e.ax, wy = ry - e.ay;
  u = fmin(fmax((wx * e.ex + wy * e.ey) * e.inv_ee, 0.0), 1.0);
  qx = wx - u * e.ex;
  qy = wy - u * e.ey;
  d2 = qx * qx + qy * qy;
}

// The distance in double; its reciprocal (the unit normal (p - q) / d at an end point) from the hardware
// estimate refined twice, which is within an ulp or two of the quotient.  (A float32 distance was tried:
// its error of a few 1e-7, amplified by the cancellation between the pixels of an item, took config 1's
// gradients past the 1e-4 bar.)
__device__ __forceinline__ PairD pair_eval(const EdgeD &e, double rx, double ry, bool par) {
  PairD r;
  double d2;
  pair_d2(e, rx, ry, d2, r.u, r.qx, r.qy);
  r.d = sqrt(d2);
  r.inv_d = r.d > 0.0 ? rcp_refined(r.d) : 0.0;
  r.sd = par ? r.d : -r.d;
  return r;
}

// The float scan can order two edges wrongly only when their squared distances agree to float
// precision.  Away from the (measure-zero) medial axes that happens only between neighbouring edges
// (near the boundary between a vertex's fan and an edge's perpendicular strip), where the choice does
// not change the distance much but does tilt the gradient direction.  So the nearest edge is decided
// again in double among the scan's choice and its two neighbours (lowest index on exact ties).
struct Nearest {
  int e;                 // the nearest edge
  double d2, u, qx, qy;  // its squared distance, clamped parameter and p - nearest point
};

__device__ __forceinline__ Nearest nearest_refined(const EdgeD *E, int ec, int bi, double rx, double ry) {
  const int lo = bi == 0 ? ec - 1 : bi - 1, hi = bi + 1 == ec ? 0 : bi + 1;
  int c0 = lo, c1 = bi, c2 = hi;
  // visit in increasing index so that strict '<' keeps the lowest index on ties
  if (c0 > c1) {
    const int t = c0;
    c0 = c1;
    c1 = t;
  }
  if (c1 > c2) {
    const int t = c1;
    c1 = c2;
    c2 = t;
  }
  if (c0 > c1) {
    const int t = c0;
    c0 = c1;
    c1 = t;
  }
  Nearest n;
  pair_d2(E[c0], rx, ry, n.d2, n.u, n.qx, n.qy);
  n.e = c0;
  double d2, u, qx, qy;
  if (c1 != c0) {
    pair_d2(E[c1], rx, ry, d2, u, qx, qy);
    if (d2 < n.d2) n = Nearest{c1, d2, u, qx, qy};
  }
  if (c2 != c1) {
    pair_d2(E[c2], rx, ry, d2, u, qx, qy);
    if (d2 < n.d2) n = Nearest{c2, d2, u, qx, qy};
  }
  return n;
}

// e^(-sd / tau) in double, for the range the coverage uses (sd >= -(r_cut + r_pad), so the result is at
// most e^((r_cut + r_pad) / tau)): 2^y with y = -sd log2(e) / tau split into an integer n and a fraction
// f in [-1/2, 1/2]; 2^f = e^g with g = f ln 2, |g| <= 0.347, by the Taylor series of e^g to degree 9
// (remainder below 1e-11 of the value), then scaled by 2^n.  Fewer instructions and registers than the
// library exponential, which also handles the whole double range.
__device__ __forceinline__ double exp_neg_tau(const KArgs &a, double sd) {
  constexpr double kLn2 = 0.6931471805599453;
  const double y = -sd * a.log2e_inv_tau;
  const double n = rint(y);
  const double g = (y - n) * kLn2;
  double p = 1.0 / 362880.0;
  p = fma(p, g, 1.0 / 40320.0);
  p = fma(p, g, 1.0 / 5040.0);
  p = fma(p, g, 1.0 / 720.0);
  p = fma(p, g, 1.0 / 120.0);
  p = fma(p, g, 1.0 / 24.0);
  p = fma(p, g, 1.0 / 6.0);
  p = fma(p, g, 0.5);
  p = fma(p, g, 1.0);
  p = fma(p, g, 1.0);
  return ldexp(p, (int)n);
}

// alpha and alpha_pad of one (pixel, item) from its signed distance, in double with one exponential:
// for x = sd / tau, e^-(x + r_pad / tau) = e^-x pad_factor.  Wherever either is not cut to zero,
// x >= -(r_cut + r_pad) / tau, so e^-x does not overflow and 1 + E is a normal number >= 1.  Double
// matters here: near convergence an item's gradient is a small remainder of its pixels' contributions,
// and alpha carried in float32 (errors of 1e-7 to 1e-6 from the float exponential) moved config 1's
// gradients at some layouts by more than 1e-4 of their size through dLoss/dS.
__device__ __forceinline__ void coverage_pair(const KArgs &a, double sd, double &al, double &alp) {
  al = alp = 0.0;
  if (sd + (double)a.r_pad < -(double)a.r_cut) return;
  const double E = exp_neg_tau(a, sd);
  if (sd >= -(double)a.r_cut) al = rcp_refined(1.0 + E);
  alp = rcp_refined(1.0 + E * a.pad_factor);
}

// omega = G dalpha/dsd + G_pad dalpha_pad/dsd of one (pixel, item), from one exponential: with
// E = e^-x (x = sd / tau), sigma'(x) = E / (1 + E)^2, free of cancellation at both ends of the range used
// (x >= -(r_cut + r_pad) / tau), where E <= e^((r_cut + max(r_pad, 0)) / tau) and E / (1 + E)^2 <= 1/4.
// In double for the reason given at coverage_pair: in float32 its errors of a few 1e-7 were amplified by
// the cancellation between an item's pixels beyond the gradient's 1e-4 bar at converged layouts.
__device__ __forceinline__ double adjoint_omega(const KArgs &a, double sd, double G, double Gp) {
  double dal = 0.0, dalp = 0.0;
  if (sd + (double)a.r_pad >= -(double)a.r_cut) {
    const double E = exp_neg_tau(a, sd), Ep = E * a.pad_factor;
    const double r = rcp_refined(1.0 + E), rp = rcp_refined(1.0 + Ep);
    if (sd >= -(double)a.r_cut) dal = E * r * r * a.inv_tau_d;
    dalp = Ep * rp * rp * a.inv_tau_d;
  }
  return G * dal + Gp * dalp;
}

// n = grad_p sd of one (pixel, item) at a pixel off the outline (q.d > 0).  Nearest point inside the edge:
// the unit edge normal, oriented (inside ? +1 : -1) times the side of the edge the pixel is on; within
// 1e-4 px of the edge the float parity is not reliable, but the product of the two is the outline
// orientation.  Nearest point at an end point: (p - q) / d, signed by the parity.
__device__ __forceinline__ void adjoint_normal(const EdgeD &e, const PairD &q, bool par, float orient, bool open,
                                               double &nx, double &ny) {
  if (q.u > 0.0 && q.u < 1.0) {
    const double il = e.inv_len;
    double sg = (double)orient;
    if (q.d >= 1e-4 || open) {
      const double side = q.qy * e.ex - q.qx * e.ey;
      sg = (par == (side > 0.0)) ? 1.0 : -1.0;
    }
    nx = -e.ey * il * sg;
    ny = e.ex * il * sg;
  } else {
    const double id = par ? q.inv_d : -q.inv_d;
    nx = q.qx * id;
    ny = q.qy * id;
  }
}

// The scale terms need d q' / d s for the nearest point q' = a' + u (b' - a') of the nearest edge,
// k R(theta) (v_a + u (v_b - v_a)) with v the item-frame vertices.  Since q' - k t = s k R(theta) (...),
// that is (r - q) / s, with r = p - k t and q = p - q' (no extra loads); for |s| < kScaleFloor, where the
// quotient loses its digits, it is formed from the vertices (V: the item's, bi: the edge, nv: vertices).
struct ScaleDeriv {
  double inv_s;  // 1 / s, or 0 for |s| < kScaleFloor
  double kc, ks; // k R(theta) (used when inv_s = 0)
  const float2 *V;
  int bi, nv;
  bool open;
};

__device__ __forceinline__ void unscaled_point(const ScaleDeriv &sd, const PairD &q, double rx, double ry,
                                               double &ux, double &uy) {
  if (sd.inv_s != 0.0) {
    ux = (rx - q.qx) * sd.inv_s;
    uy = (ry - q.qy) * sd.inv_s;
    return;
  }
  const int ib = sd.open ? min(sd.bi + 1, sd.nv - 1) : (sd.bi + 1 == sd.nv ? 0 : sd.bi + 1);
  const float2 va = sd.V[sd.bi], vb = sd.V[ib];
  const double vx = (double)va.x + q.u * ((double)vb.x - (double)va.x);
  const double vy = (double)va.y + q.u * ((double)vb.y - (double)va.y);
  ux = sd.kc * vx - sd.ks * vy;
  uy = sd.ks * vx + sd.kc * vy;
}

// Adjoint terms of one (pixel, item): omega * d sd / d(t, theta, s), up to the factor -k of the
// translation terms applied by the finalize kernel.
// For an open item (sw_ds != 0 or open) q.sd = sw - d, par is false (the gradient of -d), and the
// stroke radius adds d sd / d s = sw_ds.
__device__ __forceinline__ double4 adjoint_terms(const KArgs &a, const EdgeD &e, const PairD &q, double rx, double ry,
                                                 bool par, float orient, double G, double Gp, bool open,
                                                 double sw_ds, const ScaleDeriv &sdv) {
  const double om = adjoint_omega(a, q.sd, G, Gp);
  double4 t = make_double4(0.0, 0.0, 0.0, 0.0);
  if (om == 0.0) return t;
  const double stroke_term = open ? om * sw_ds : 0.0;
  t.w = stroke_term;
  if (q.d == 0.0) return t;
  double nx, ny;
  adjoint_normal(e, q, par, orient, open, nx, ny);
  t.x = om * nx;
  t.y = om * ny;
  t.z = om * (nx * ry - ny * rx);
  // d sd / d s = -n . (d q' / d s): the nearest point of the unscaled outline
  double ux, uy;
  unscaled_point(sdv, q, rx, ry, ux, uy);
  t.w = stroke_term - om * (nx * ux + ny * uy);
  return t;
}

// ------------------------------------------------------------------------------------------------
// Unit numbering.  An item's support box meets the screen tiles [tx0, tx0 + tw) x [ty0, ty0 + th) of its
// layout (the box lies on the canvas, so these are floor divisions; tw = th = 0 for an empty box), and
// each of those (tile, item) pairs is one work unit.  A layout's units are numbered twice, both times
// without gaps from the layout's first pool entry: in row-major tile order and, within a tile, in item
// order (the tile lists and unit records); and in item order and, within an item, in row-major order
// of its tiles (the per-item map read by the update).  A tile's first unit is then the number of the
// layout's units in earlier tiles, and an item's first map entry the number of units of earlier items:
// sums over the items of closed forms in their tile spans, so binning needs no counters and no
// separate scan, and the layout needs room for its units only.
// ------------------------------------------------------------------------------------------------
struct TileSpan {
  int tx0, ty0, tw, th;
};

template <int T>
__device__ __forceinline__ TileSpan tile_span(int4 bb) {
  TileSpan t = {0, 0, 0, 0};
  if (bb.x <= bb.z && bb.y <= bb.w) {
    t.tx0 = bb.x / T;
    t.ty0 = bb.y / T;
    t.tw = bb.z / T - t.tx0 + 1;
    t.th = bb.w / T - t.ty0 + 1;
  }
  return t;
}

// The item's units in the tile rows before row tyi.
__device__ __forceinline__ long long units_in_rows_before(const TileSpan &t, int tyi) {
  return (long long)min(max(tyi - t.ty0, 0), t.th) * t.tw;
}

// The item's units before tile (txi, tyi) in row-major tile order; with in_row_only, only those in
// row tyi (the rows before are counted per row by the row pass).
__device__ __forceinline__ long long units_before_tile(const TileSpan &t, int txi, int tyi, bool in_row_only) {
  const bool in_row = tyi >= t.ty0 && tyi < t.ty0 + t.th;
  return (in_row_only ? 0ll : units_in_rows_before(t, tyi)) + (in_row ? min(max(txi - t.tx0, 0), t.tw) : 0);
}

// Work units are the (tile, item) pairs of the per-tile lists, in tile order and slot order.  A unit
// covers the rectangle where the item's support box meets the tile, packed row by row into chunks of
// 64 pixels (one pixel per lane).  A chunk costs (edges + kEpilogueCost + its share of kUnitCost) in the
// coverage pass and 1 in the adjoint pass.  Chunks are numbered through the whole pass in unit order
// (the same numbering in both passes: it indexes the nearest-edge codes kept between them and the
// adjoint partials).
//
// The persistent wave w of W processes the chunks whose cost interval [p, p + c) ends in
// (B_w, B_{w+1}], where B_w = ceil(w * total / W) and p is the chunk's cost prefix.  It finds the tile
// holding B_w, then the unit within it, by 64-way searches over their prefix sums (one probe per lane
// and step) and walks from there; a unit may be split between consecutive waves.  Every wave gets the
// same work to within one chunk, and no counter is shared between waves.
struct Walk {
  int tile, slot, count;   // current unit = slot `slot` of tile `tile` (which has `count` units)
  int W, x0, y0;           // canvas width and origin of the tile
  int64_t pix_off, list_base;
  long long p, end;        // cost prefix of the current unit (in this pass); end of the wave's range
  long long q0;            // first chunk of the tile
  const long long *Q;      // [tiles + 1] chunk prefix of the tiles (LDS or global)
  const int2 *C;           // [tiles] units and first pool entry per tile (LDS), or null: tile_units
  int4 aux;                // (chunks, cost per chunk, chunks and cost of the tile's earlier units) of the unit
  int jlo, jhi;            // the wave's chunks [jlo, jhi) of the current unit
  bool adj;
};

__device__ __forceinline__ int4 load_aux(const KArgs &a, int64_t i) {
  cptr<int> r = (cptr<int>)(konst(a.entry_aux) + i);
  return make_int4(r[0], r[1], r[2], r[3]);
}

__device__ __forceinline__ void walk_tile(const KArgs &a, Walk &w, int T) {
  cptr<LayoutRec> LS = konst(a.layouts);
  const int b = layout_of_tile(LS, a.num_layouts, w.tile);
  w.W = LS[b].W;
  const int ntx = LS[b].ntx;
  const int lt = w.tile - LS[b].tile_off;
  const int tyi = lt / ntx;
  w.x0 = (lt - tyi * ntx) * T;
  w.y0 = tyi * T;
  w.pix_off = LS[b].pix_off;
  int2 tu;
  if (w.C != nullptr) {
    tu = w.C[w.tile];
    tu.x = uniform(tu.x);
    tu.y = uniform(tu.y);
  } else {
    cptr<int> r = (cptr<int>)(konst(a.tile_units) + w.tile);
    tu = make_int2(r[0], r[1]);
  }
  w.count = tu.x;
  w.list_base = tu.y;
  w.q0 = uniform_ll(w.Q[w.tile]);
}

__device__ __forceinline__ int chunk_cost(const Walk &w) { return w.adj ? 1 : w.aux.y; }

// Moves to the next unit that exists and has work (skipping empty tiles and, should one occur, a unit
// without pixels) and loads its record; returns false past the last tile.
__device__ __forceinline__ bool walk_settle(const KArgs &a, Walk &w, int T) {
  for (;;) {
    while (w.slot >= w.count) {
      if (++w.tile >= a.total_tiles) return false;
      w.slot = 0;
      walk_tile(a, w, T);
    }
    w.aux = load_aux(a, w.list_base + w.slot);
    if (w.aux.x > 0) return true;
    ++w.slot;
  }
}

// The wave's chunks of the current unit: those ending in (b0, end] (b0 <= p for every unit after the
// first).
__device__ __forceinline__ void walk_range(Walk &w, long long b0) {
  const long long c = chunk_cost(w);
  w.jlo = b0 > w.p ? (int)((b0 - w.p) / c) : 0;
  const long long hi = (w.end - w.p) / c;
  w.jhi = hi < (long long)w.aux.x ? (int)hi : w.aux.x;
}

// The last index i in [0, n) with val(i) <= x, for a nondecreasing val with val(0) <= x, found by the
// whole wave: each round loads 64 evenly spaced candidates of the remaining range at once (one vector
// load instead of a chain of dependent ones) and keeps the segment after the last candidate <= x.
template <class F>
__device__ __forceinline__ int wave_last_le(int n, long long x, F val) {
  const int lane = threadIdx.x & 63;
  int lo = 0, len = n;
  while (len > 1) {
    const int step = (len + 63) >> 6;
    const int i = lo + lane * step;
    const bool ok = i < lo + len && val(i) <= x;
    const int k = 63 - __clzll(__ballot(ok));  // lane 0 (i = lo) always qualifies
    const int end = lo + len;
    lo += k * step;
    len = min(step, end - lo);
  }
  return uniform(lo);
}

// The last unit i in [0, n) of a tile (n >= 1) whose prefix within the tile (entry_aux .z: chunks, for the
// adjoint passes; .w: cost, for the coverage pass) is <= x, found as wave_last_le finds it, with that
// unit's entry_aux: the last round loads consecutive entries, so the winner's whole record is in one
// lane and needs no second load.
__device__ __forceinline__ int unit_search(const int4 *X, int n, long long x, bool adj, int4 &aux) {
  const int lane = threadIdx.x & 63;
  int lo = 0, len = n;
  for (;;) {
    const int step = (len + 63) >> 6;
    const int i = lo + lane * step;
    const bool valid = i < lo + len;
    int4 v = make_int4(0, 0, 0, 0);
    if (valid) v = X[i];
    const bool ok = valid && (long long)(adj ? v.z : v.w) <= x;
    const int k = 63 - __clzll(__ballot(ok));  // lane 0 (i = lo) always qualifies
    if (step == 1) {
      aux = make_int4(__builtin_amdgcn_readlane(v.x, k), __builtin_amdgcn_readlane(v.y, k),
                      __builtin_amdgcn_readlane(v.z, k), __builtin_amdgcn_readlane(v.w, k));
      return uniform(lo + k);
    }
    const int end = lo + len;
    lo += k * step;
    len = min(step, end - lo);
  }
}

// Where wave g's share of a pass of total cost tot begins.  Waves with a higher index are dispatched
// later and, the SIMDs issuing for their oldest waves first, progress more slowly: measured on the
// coverage pass at 512^2 with equal shares, the last eighth of the waves ended 14 us after the first
// eighth.  The coverage pass therefore tapers the shares linearly with the wave index, the last wave's
// share (1 - taper) times the first's, with the scene's taper (KArgs::cover_taper: larger for items
// with more edges, whose chunks keep a wave busy longer).  The adjoint pass, whose waves were measured
// not to gain, keeps equal shares.

__device__ __forceinline__ long long share_bound(long long tot, int g, int nwaves, double taper) {
  if (g >= nwaves) return tot;
  if (taper == 0.0) return ((long long)g * tot + nwaves - 1) / nwaves;
  const double x = (double)g / (double)nwaves;
  return (long long)ceil((double)tot * (x - 0.5 * taper * x * x) / (1.0 - 0.5 * taper));
}

// First piece of persistent wave gw: returns false when the wave has no work.
// P: [tiles + 1] prefix of the pass's tile costs (chunks for the adjoint passes); Q: the chunk prefix;
// C: the tiles' unit counts and first pool entries in LDS, or null (global).
__device__ __forceinline__ bool walk_begin(const KArgs &a, Walk &w, int gw, int nwaves, bool adj, int T,
                                           const long long *P, const long long *Q, const int2 *C) {
  const long long tot = uniform_ll(P[a.total_tiles]);
  w.Q = Q;
  w.C = C;
  w.adj = adj;
  if (tot <= 0) return false;
  const long long b0 = share_bound(tot, gw, nwaves, adj ? 0.0 : a.cover_taper);
  w.end = share_bound(tot, gw + 1, nwaves, adj ? 0.0 : a.cover_taper);
  if (b0 >= tot || w.end <= b0) return false;
  // the last tile whose prefix is <= b0 (it has work: a tile without any would share its prefix with
  // the next one), then the last of its units whose prefix within the tile is <= b0 (units' prefixes
  // grow strictly: every unit covers at least one pixel)
  w.tile = wave_last_le(a.total_tiles, b0, [&](int i) { return P[i]; });
  w.p = uniform_ll(P[w.tile]);
  walk_tile(a, w, T);
  w.slot = 0;
  bool have = false;  // w.aux holds the record of the unit at w.slot
  if (w.count > 0) {
    w.slot = unit_search(a.entry_aux + w.list_base, w.count, b0 - w.p, adj, w.aux);
    w.p += adj ? w.aux.z : w.aux.w;
    have = true;
  }
  // (the search leaves nothing to skip; the loop only guards the invariant)
  for (;;) {
    if (!have && !walk_settle(a, w, T)) return false;
    have = false;
    const long long c = (long long)w.aux.x * chunk_cost(w);
    if (w.p + c > b0) break;
    w.p += c;
    ++w.slot;
  }
  walk_range(w, b0);
  return w.jhi > w.jlo;
}

// Advances to the wave's next piece; returns false when the wave is done.
__device__ __forceinline__ bool walk_next(const KArgs &a, Walk &w, int T) {
  if (w.jhi < w.aux.x) return false;  // the rest of this unit belongs to the next wave
  w.p += (long long)w.aux.x * chunk_cost(w);
  ++w.slot;
  if (!walk_settle(a, w, T)) return false;
  walk_range(w, w.p);
  return w.jhi > 0;
}

// First chunk (in the pass numbering) of the current unit.
__device__ __forceinline__ long long walk_chunk0(const Walk &w) { return w.q0 + w.aux.z; }

// The rectangle of a unit: the item's support box clipped to the tile (never empty for a listed item).
struct Rect {
  int x0, y0, w, n;
};

__device__ __forceinline__ Rect unit_rect(int4 bb, int tx0, int ty0, int T) {
  Rect r;
  r.x0 = max(bb.x, tx0);
  r.y0 = max(bb.y, ty0);
  r.w = min(bb.z, tx0 + T - 1) - r.x0 + 1;
  r.n = r.w * (min(bb.w, ty0 + T - 1) - r.y0 + 1);
  return r;
}

// The wave index is wave-uniform; readfirstlane tells the compiler so, which keeps the work walk in SGPRs
// and its loads on the scalar cache.
__device__ __forceinline__ int global_wave() { return uniform((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6))); }

// ------------------------------------------------------------------------------------------------
// k_rowbin: per tile row of a layout, the ordered list of items whose support box meets the row band
// (large scenes: the tiles then test only their row's items instead of every item of the layout), and
// the number of the layout's units in earlier rows (-1 when the layout has more units than its pool
// holds).  The first row's workgroup also numbers the items' map entries.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ int layout_of_row(cptr<LayoutRec> L, int B, int row) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (L[mid].row_off <= row)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <int T>
__global__ __launch_bounds__(256) void k_rowbin(KArgs a) {
  constexpr int NW = 4;
  __shared__ long long s_w[NW][2];  // per wave: its hits, its candidates' units
  const int row = blockIdx.x, tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  cptr<LayoutRec> LS = konst(a.layouts);
  const int b = layout_of_row(LS, a.num_layouts, row);
  const int tyi = row - LS[b].row_off;
  const int sb = LS[b].shape_begin, se = LS[b].shape_end, nb = se - sb;
  const int y0 = tyi * T, y1 = y0 + T - 1;
  const bool first_row = tyi == 0;
  const int64_t pool0 = LS[b].list_off;
  int32_t *out = a.row_list + LS[b].row_list_off + (int64_t)tyi * nb;
  int n = 0;
  long long before = 0, carry = 0;  // per thread: units in earlier rows; block: units of earlier items
  for (int base = sb; base < se; base += 256) {
    const int sid = base + tid;
    TileSpan t = {0, 0, 0, 0};
    bool hit = false;
    if (sid < se) {
      const int4 bb = load_box(konst(a.bins), sid);
      // the box lies on the canvas: it meets the row band where its y range does
      hit = bb.x <= bb.z && bb.y <= bb.w && !(bb.y > y1 || bb.w < y0);
      t = tile_span<T>(bb);
    }
    const long long nu = (long long)t.tw * t.th;
    before += units_in_rows_before(t, tyi);
    const unsigned long long m = __ballot(hit);
    const unsigned long long us = wave_incl_scan_u64((unsigned long long)nu);
    if (l == 63) {
      s_w[w][0] = __popcll(m);
      s_w[w][1] = (long long)us;
    }
    __syncthreads();
    int off = n, tot = n;
    long long uoff = carry, utot = carry;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const int cj = (int)s_w[j][0];
      const long long uj = s_w[j][1];
      if (j < w) {
        off += cj;
        uoff += uj;
      }
      tot += cj;
      utot += uj;
    }
    if (hit) out[off + __popcll(m & ((1ull << l) - 1ull))] = sid;
    // first map entry of the item (replaced by -1 below if the layout's units do not fit)
    if (first_row && sid < se) a.item_base[sid] = (int32_t)(pool0 + uoff + (long long)us - nu);
    n = tot;
    carry = utot;
    __syncthreads();
  }
  before = wave_sum_ll(before);
  if (l == 0) s_w[w][0] = before;
  __syncthreads();
  long long rb = 0;
#pragma unroll
  for (int j = 0; j < NW; ++j) rb += s_w[j][0];
  const bool fits = carry <= (long long)LS[b].unit_cap;
  if (tid == 0) {
    a.row_count[row] = n;
    a.row_base[row] = fits ? rb : -1ll;
    if (first_row && !fits) atomicAdd(&a.status[COLLAGE_STATUS_UNIT_OVERFLOW], 1);
  }
  if (first_row && !fits)
    for (int sid = sb + tid; sid < se; sid += 256) a.item_base[sid] = -1;
}

// Whether an item's support box meets the T x T tile at (x0, y0); an item wholly off its canvas has an
// empty box (x1 < x0) and is binned nowhere.
__device__ __forceinline__ bool box_meets_tile(int4 bb, int x0, int y0, int T) {
  return bb.x <= bb.z && bb.y <= bb.w && !(bb.x > x0 + T - 1 || bb.z < x0 || bb.y > y0 + T - 1 || bb.w < y0);
}

// ------------------------------------------------------------------------------------------------
// k_bin: per tile, the ordered item list and one work unit per (tile, item), from the tile's first unit
// on; without the row pass, the first tile of each layout also numbers the items' map entries.
// ------------------------------------------------------------------------------------------------
// Candidates a binning thread loads per pass: two when every item of the layout is a candidate (a pass
// then holds 512 of them; four measured slower), one after the row pass, whose rows list few items
// (half the registers, so more of a large grid's workgroups are resident at once).

// Workgroups per screen tile: 64 x 64 and 128 x 128 tiles spread the clearing of their accumulators
// over 4 and 16 (only the first bins), so that it is not left to a fraction of the compute units.
template <int T>
constexpr int kBinParts = T >= 128 ? 16 : (T >= 64 ? 4 : 1);

template <int T, int K>
__global__ __launch_bounds__(T *T < 256 ? T *T : 256) void k_bin(KArgs a) {
  constexpr int NT = T * T < 256 ? T * T : 256, NW = NT / 64, ZP = kBinParts<T>;
  __shared__ long long s_w[NW][2];  // counting pass, per wave: units before the tile, units
  // main passes, per candidate index k and wave: hits, units of the candidates; per wave: units before
  // the tile
  __shared__ int s_h[K][NW];
  __shared__ int s_u[K][NW], s_b[NW];
  // the first kMaxBinChunk units' chunks and cost, for the prefix pass below (later units of a tile that
  // lists more items are read back from global memory)
  __shared__ int s_uch[kMaxBinChunk], s_ucost[kMaxBinChunk];
  const int tile = blockIdx.x / ZP, part = blockIdx.x % ZP, tid = threadIdx.x;
  cptr<LayoutRec> LS = konst(a.layouts);
  const int b = layout_of_tile(LS, a.num_layouts, tile);
  const int W = LS[b].W, H = LS[b].H, ntx = LS[b].ntx;
  const int sb = LS[b].shape_begin, se = LS[b].shape_end, nb = se - sb;
  const int lt = tile - LS[b].tile_off, tyi = lt / ntx, txi = lt - tyi * ntx;
  const int x0 = txi * T, y0 = tyi * T;
  const int64_t pool0 = LS[b].list_off;
  for (int q = part * (T * T / ZP) + tid; q < (part + 1) * (T * T / ZP); q += NT) {
    const int pxi = x0 + q % T, pyi = y0 + q / T;
    if (pxi < W && pyi < H) {
      const int64_t pix = LS[b].pix_off + (int64_t)pyi * W + pxi;
      __builtin_nontemporal_store((nt_u64x2){0ull, 0ull}, reinterpret_cast<nt_u64x2 *>(a.acc + 2 * pix));
    }
  }
  if (part != 0) return;
  // candidates: every item of the layout, or the items listed for the tile's row.  Each thread loads its
  // candidates' whole bin records with the boxes it tests, so that a hit's unit record needs no further
  // load: the thread writes it at the item's slot in the tile list.
  const bool rowbin = a.rowbin != 0;
  const int32_t *src = rowbin ? a.row_list + LS[b].row_list_off + (int64_t)tyi * nb : nullptr;
  const int c0 = rowbin ? 0 : sb, c1 = rowbin ? a.row_count[LS[b].row_off + tyi] : se;
  const long long row_before = rowbin ? a.row_base[LS[b].row_off + tyi] : 0ll;  // -1: the layout overflows
  const int w = tid >> 6, l = tid & 63;
  // the tile's first unit (after the layout's units in earlier tiles) and the layout's units: from the
  // first pass of candidates when one pass holds them all, else from a counting pass first
  long long before = 0, layout_units = 0;
  const bool one_pass = c1 - c0 <= K * NT;
  if (!one_pass) {
    long long bt = 0, lu = 0;
    for (int pos = c0 + tid; pos < c1; pos += NT) {
      const TileSpan t = tile_span<T>(load_box(konst(a.bins), src ? src[pos] : pos));
      bt += units_before_tile(t, txi, tyi, rowbin);
      lu += (long long)t.tw * t.th;
    }
    bt = wave_sum_ll(bt);
    lu = wave_sum_ll(lu);
    if (l == 0) {
      s_w[w][0] = bt;
      s_w[w][1] = lu;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      before += s_w[j][0];
      layout_units += s_w[j][1];
    }
    __syncthreads();
  }
  bool fits = true;
  int64_t list_base = pool0;
  int slots = 0;
  int ucarry = 0;  // units of the candidates of earlier passes (in item order without the row pass)
  long long my_cost = 0, my_quads = 0;  // coverage cost and chunks of the tile's units
  // K candidates per thread and pass, candidate k of thread tid at base + k NT + tid (coalesced loads);
  // slots and map entries follow the candidate order.  The pass counts units in 32 bits: without the row
  // pass a layout has at most tiles x items <= kRowBinTests units, and with it the units before the tile
  // in its row are used only when the layout fits its pool (< 2^31 units).
  for (int base = c0; base < c1; base += K * NT) {
    BinRec br[K];
    int sid[K], ib[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int pos = base + k * NT + tid;
      sid[k] = pos < c1 ? (src ? src[pos] : pos) : 0;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      ib[k] = 0;
      if (base + k * NT + tid < c1) {
        br[k] = a.bins[sid[k]];
        if (rowbin) ib[k] = a.item_base[sid[k]];
      } else {
        br[k].box = make_int4(1, 1, 0, 0);
      }
    }
    unsigned long long m[K];
    int nu[K], us[K], bt = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const TileSpan t = tile_span<T>(br[k].box);
      m[k] = __ballot(box_meets_tile(br[k].box, x0, y0, T));
      nu[k] = t.tw * t.th;
      us[k] = rowbin ? 0 : (int)wave_incl_scan_u32((unsigned)nu[k]);
      bt += (int)units_before_tile(t, txi, tyi, rowbin);
    }
    bt = __builtin_amdgcn_readlane((int)wave_incl_scan_u32((unsigned)bt), 63);
    if (l == 63) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        s_h[k][w] = __popcll(m[k]);
        s_u[k][w] = us[k];
      }
      s_b[w] = bt;
    }
    __syncthreads();
    // per candidate: hits and units of the candidates before it; block totals
    int hoff[K];
    int uoff[K];
    int htot = slots, utot = ucarry, btot = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      hoff[k] = htot;
      uoff[k] = utot;
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const int hj = s_h[k][j];
        const int uj = s_u[k][j];
        if (j < w) {
          hoff[k] += hj;
          uoff[k] += uj;
        }
        htot += hj;
        utot += uj;
      }
    }
#pragma unroll
    for (int j = 0; j < NW; ++j) btot += s_b[j];
    if (base == c0) {
      if (one_pass) {
        before = btot;
        layout_units = utot;
      }
      // rows: the row pass checked the layout's units against its pool; otherwise this tile sees them all
      fits = rowbin ? row_before >= 0 : layout_units <= (long long)LS[b].unit_cap;
      list_base = pool0 + (rowbin ? row_before : 0ll) + before;
    }
    const unsigned long long below = (1ull << l) - 1ull;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const TileSpan t = tile_span<T>(br[k].box);
      // the item's first map entry
      const int64_t item0 = rowbin ? (int64_t)ib[k] : pool0 + (uoff[k] + us[k] - nu[k]);
      if (!rowbin && lt == 0 && base + k * NT + tid < c1) a.item_base[sid[k]] = fits ? (int32_t)item0 : -1;
      if (((m[k] >> l) & 1ull) && fits) {
        const int slot = hoff[k] + __popcll(m[k] & below);
        const Rect r = unit_rect(br[k].box, x0, y0, T);
        const int chunks = (r.n + 63) >> 6;
        const int ec = br[k].ecnv & 0xffff;
        const int head = (int)(item0 + (int64_t)(tyi - t.ty0) * t.tw + (txi - t.tx0));
        UnitRec u;
        u.eo = br[k].eo;
        u.ecnv = br[k].ecnv;
        u.flags = br[k].flags;
        u.head = head;
        u.xy = r.x0 | (r.y0 << 16);
        u.wn = r.w | (r.n << 16);
        u.sid = sid[k];
        u.s = br[k].s;
        u.cx = br[k].cx;
        u.cy = br[k].cy;
        a.units[list_base + slot] = u;
        a.tile_list[list_base + slot] = sid[k];
        const int cpc = ec + kEpilogueCost + (kUnitCost + chunks - 1) / chunks;
        a.entry_aux[list_base + slot] = make_int4(chunks, cpc, 0, 0);
        // the unit's head partials start at zero (the adjoint adds its pieces)
        ulonglong2 *hp = reinterpret_cast<ulonglong2 *>(a.head + 4 * (int64_t)head);
        hp[0] = make_ulonglong2(0ull, 0ull);
        hp[1] = make_ulonglong2(0ull, 0ull);
        if (slot < kMaxBinChunk) {
          s_uch[slot] = chunks;
          s_ucost[slot] = chunks * cpc;
        }
        my_cost += (long long)chunks * cpc;
        my_quads += chunks;
      }
    }
    slots = htot;
    ucarry = utot;
    __syncthreads();
  }
  if (!fits) {
    slots = 0;
    if (tid == 0 && !rowbin && lt == 0) atomicAdd(&a.status[COLLAGE_STATUS_UNIT_OVERFLOW], 1);
  }
  // chunks and coverage cost of the tile's earlier units, per unit (first wave, 64 units at a time)
  if (tid < 64) {
    int run = 0, run_cost = 0;
    for (int base = 0; base < slots; base += 64) {
      const int j = base + tid;
      int c = 0, k = 0;
      if (j < slots) {
        if (j < kMaxBinChunk) {
          c = s_uch[j];
          k = s_ucost[j];
        } else {
          const int4 ax = a.entry_aux[list_base + j];
          c = ax.x;
          k = ax.x * ax.y;
        }
      }
      const int x = (int)wave_incl_scan_u32((unsigned)c), y = (int)wave_incl_scan_u32((unsigned)k);
      if (j < slots) {
        a.entry_aux[list_base + j].z = run + x - c;
        a.entry_aux[list_base + j].w = run_cost + y - k;
      }
      run += __builtin_amdgcn_readlane(x, 63);
      run_cost += __builtin_amdgcn_readlane(y, 63);
    }
  }
  // tile totals of the unit costs (for the work partition of the persistent kernels)
  my_cost = wave_sum_ll(my_cost);
  my_quads = wave_sum_ll(my_quads);
  __shared__ long long s_red[NW][2];
  if ((tid & 63) == 0) {
    s_red[tid >> 6][0] = my_cost;
    s_red[tid >> 6][1] = my_quads;
  }
  __syncthreads();
  if (tid == 0) {
    long long c = 0, q = 0;
    for (int j = 0; j < NW; ++j) {
      c += s_red[j][0];
      q += s_red[j][1];
    }
    a.tile_units[tile] = make_int2(slots, fits ? (int32_t)list_base : 0);
    a.tile_cost[tile] = make_int2((int)c, (int)q);
  }
}

// ------------------------------------------------------------------------------------------------
// k_scan: one workgroup.  Prefix sums over the tiles of the coverage cost and of the chunk count (the
// work partition of the persistent kernels): every thread owns a contiguous run of tiles.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ long long block_exclusive_scan(long long v, long long *s_w, long long &total) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  long long x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long y = __shfl_up(x, o, 64);
    if (l >= o) x += y;
  }
  if (l == 63) s_w[w] = x;
  __syncthreads();
  long long off = 0, tot = 0;
  for (int j = 0; j < 16; ++j) {
    if (j < w) off += s_w[j];
    tot += s_w[j];
  }
  __syncthreads();
  total = tot;
  return off + x - v;
}

// The chunk counts of the pass in the status words (one thread writes them once per epoch).
__device__ __forceinline__ void publish_chunk_status(const KArgs &a, long long chunks) {
  const long long beyond = chunks > a.code_cap ? chunks - a.code_cap : 0;
  a.status[COLLAGE_STATUS_CHUNKS] = (int32_t)min(chunks, (long long)INT32_MAX);
  a.status[COLLAGE_STATUS_RESCANNED] = a.keep_codes ? (int32_t)min(beyond, (long long)INT32_MAX) : 0;
}

__global__ __launch_bounds__(1024) void k_scan(KArgs a) {
  __shared__ long long s_w[16];
  const int tid = threadIdx.x;
  const int nt = a.total_tiles;
  const int per = (nt + 1023) / 1024, t0 = min(tid * per, nt), t1 = min(t0 + per, nt);
  // the thread's run of tiles, eight loads in flight at a time
  long long cc = 0, cq = 0;
  for (int t = t0; t < t1; t += 8) {
    int2 c[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) c[j] = t + j < t1 ? a.tile_cost[t + j] : make_int2(0, 0);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      cc += c[j].x;
      cq += c[j].y;
    }
  }
  long long tot_c, tot_q;
  long long pc = block_exclusive_scan(cc, s_w, tot_c);
  long long pq = block_exclusive_scan(cq, s_w, tot_q);
  long long *prc = a.tile_pre, *prq = a.tile_pre + (nt + 1);
  for (int t = t0; t < t1; t += 8) {
    int2 c[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) c[j] = t + j < t1 ? a.tile_cost[t + j] : make_int2(0, 0);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (t + j < t1) {
        prc[t + j] = pc;
        prq[t + j] = pq;
      }
      pc += c[j].x;
      pq += c[j].y;
    }
  }
  if (tid == 0) {
    prc[nt] = tot_c;
    prq[nt] = tot_q;
    if (a.step_inc != nullptr) a.step_inc[0] = a.step_inc[0] + 1;
    publish_chunk_status(a, tot_q);
  }
}

// ------------------------------------------------------------------------------------------------
// The scan from LDS.  A wave stages the edges of its current item in its own LDS slice (items with more
// than kStageEdges edges go through in segments), packed to kEdgeFloats floats per edge, then every lane
// reads each group of four edges with kEdgeFloats broadcast 16-byte LDS loads.  LDS loads of a wave
// complete in order, so the next records can be in flight while the current ones are used, which the
// scalar cache could not sustain (most of its edge fetches missed).  The parity of the crossings is kept
// as wave-wide lane masks in scalar registers.  An edge's crossing needs the ordinate tests of both its
// end points: that of its b is the next edge's a (the same float), so each edge's crossing is folded in
// when the next edge is read (the last edge's b is vertex 0).
// ------------------------------------------------------------------------------------------------
// Per staged edge: a_x, a_y, e_x / |e|^2, e_y / |e|^2, e_x, e_y, e_x / e_y (b_y is the next edge's a_y).
// Measured at 512^2 with 500 items: 37.9 us per coverage pass against 39.7 us for the 8 floats of the
// global record, and 40.6 us for 6 floats with the crossing decided by the sign of a cross product
// (one more VALU operation per edge for a quarter fewer LDS bytes).
constexpr int kEdgeFloats = 7;
// float4 slots per wave: kStageEdges packed edges and one group of four of read-ahead
constexpr int kStageSlots = kEdgeFloats * (kStageEdges / 4 + 1);

__device__ __forceinline__ void stage_edges(const EdgeRec *E, int ne, float4 *dst, int lane) {
  float *D = reinterpret_cast<float *>(dst);
  const float4 *src = reinterpret_cast<const float4 *>(E);
  for (int i = lane; i < ne; i += 64) {
    const float4 r0 = src[2 * i], r1 = src[2 * i + 1];
    float *d = D + kEdgeFloats * i;
    d[0] = r0.x;
    d[1] = r0.y;
    d[2] = r0.z;
    d[3] = r0.w;
    d[4] = r1.x;
    d[5] = r1.y;
    d[6] = r1.w;
  }
  __builtin_amdgcn_wave_barrier();
}

struct ScanState {
  unsigned best;            // bits of the smallest squared distance so far (see scan_group)
  int grp;                  // first edge of the earliest group of four edges that holds it
  unsigned long long par;   // lanes with an odd number of crossings so far
  unsigned long long up;    // lanes with a_y > r_y for the last edge read
  unsigned long long left;  // the last edge's x-intercept test, for lanes whose row it may cross
  unsigned long long up0;   // lanes with a_y > r_y for edge 0 (b of the last edge)
};

// S: the staged edges from edge 0 (float index 1 is a_y of edge 0).
__device__ __forceinline__ void scan_start(ScanState &st, const float4 *S, float ry) {
  st.best = __float_as_uint(INFINITY);
  st.grp = 0;
  st.par = 0ull;
  st.up = 0ull;
  st.left = 0ull;
  st.up0 = __ballot(S[0].y > ry);
}

// Squared distance (float) from (rx, ry) to the edge (a_x, a_y) + u (e_x, e_y), u clamped to [0, 1], with
// (e_xs, e_ys) = e / |e|^2.  The scan and the re-decision of the nearest edge both use this one sequence,
// so they produce the same bits.
__device__ __forceinline__ float edge_d2(float ax, float ay, float exs, float eys, float ex, float ey, float rx,
                                         float ry) {
  const float wx = rx - ax, wy = ry - ay;
  const float t = fmaf(wx, exs, wy * eys);
  const float u = __builtin_amdgcn_fmed3f(t, 0.0f, 1.0f);
  const float qx = fmaf(-u, ex, wx), qy = fmaf(-u, ey, wy);
  return fmaf(qx, qx, qy * qy);
}

// One staged edge f[0..kEdgeFloats): its squared distance; the crossing of the previous edge (whose b_y is
// this edge's a_y) folded into the parity; this edge's x-intercept test, r_x - a_x < (r_y - a_y) e_x / e_y,
// kept for the next edge.
__device__ __forceinline__ float scan_edge(const float *f, float rx, float ry, ScanState &st) {
  const float wx = rx - f[0], wy = ry - f[1];
  const float t = fmaf(wx, f[2], wy * f[3]);
  const float u = __builtin_amdgcn_fmed3f(t, 0.0f, 1.0f);
  const float qx = fmaf(-u, f[4], wx), qy = fmaf(-u, f[5], wy);
  const float d2 = fmaf(qx, qx, qy * qy);
  const unsigned long long up = __ballot(wy < 0.0f);  // a_y > r_y (the subtraction's sign is exact)
  st.par ^= (st.up ^ up) & st.left;
  st.left = __ballot(wx < wy * f[6]);
  st.up = up;
  return d2;
}

// The last edge's crossing (its b is vertex 0).
__device__ __forceinline__ void scan_finish(ScanState &st) { st.par ^= (st.up ^ st.up0) & st.left; }

// The minimum of a group of four edges (first edge e) enters the running minimum; strict comparison,
// so the earliest group holding the minimum is kept.  Squared distances are never negative, so their
// bit patterns order as unsigned integers (NaN above +inf: never chosen, as with fminf), which needs
// no canonicalization of the running value.
__device__ __forceinline__ void scan_group(float d0, float d1, float d2, float d3, int e, ScanState &st) {
  const unsigned g = min(min(__float_as_uint(d0), __float_as_uint(d1)), min(__float_as_uint(d2), __float_as_uint(d3)));
  st.grp = g < st.best ? e : st.grp;
  st.best = min(st.best, g);
}

// Edges [0, ne) of the staged slice S, numbered from ebase.  Each step loads a group of four edges
// (kEdgeFloats slots) at once and evaluates them as they arrive; the other waves of the SIMD cover the
// remaining latency.  Reads up to one group past ne.
__device__ __forceinline__ void scan_lds(const float4 *S, int ne, int ebase, float rx, float ry, ScanState &st) {
  int e = 0;
  for (; e + 4 <= ne; e += 4) {
    const float4 *R = S + (kEdgeFloats * e) / 4;
    float f[4 * kEdgeFloats];
#pragma unroll
    for (int k = 0; k < kEdgeFloats; ++k) {
      const float4 r = R[k];
      f[4 * k] = r.x;
      f[4 * k + 1] = r.y;
      f[4 * k + 2] = r.z;
      f[4 * k + 3] = r.w;
    }
    const float d0 = scan_edge(f, rx, ry, st);
    const float d1 = scan_edge(f + kEdgeFloats, rx, ry, st);
    const float d2 = scan_edge(f + 2 * kEdgeFloats, rx, ry, st);
    const float d3 = scan_edge(f + 3 * kEdgeFloats, rx, ry, st);
    scan_group(d0, d1, d2, d3, ebase + e, st);
  }
  if (e < ne) {
    const float4 *R = S + (kEdgeFloats * e) / 4;
    float f[4 * kEdgeFloats];
#pragma unroll
    for (int k = 0; k < kEdgeFloats; ++k) {
      const float4 r = R[k];
      f[4 * k] = r.x;
      f[4 * k + 1] = r.y;
      f[4 * k + 2] = r.z;
      f[4 * k + 3] = r.w;
    }
    const float d0 = scan_edge(f, rx, ry, st);
    const float d1 = e + 1 < ne ? scan_edge(f + kEdgeFloats, rx, ry, st) : INFINITY;
    const float d2 = e + 2 < ne ? scan_edge(f + 2 * kEdgeFloats, rx, ry, st) : INFINITY;
    scan_group(d0, d1, d2, INFINITY, ebase + e, st);
  }
}

// The nearest edge within the winning group: the first of its edges (at most four, up to ec) whose
// recomputed squared distance equals the scan's minimum, i.e. the first edge of the whole outline that
// attains it.  From the staged slice (S, packed) or from the item's global records (E).
__device__ __forceinline__ int scan_resolve_lds(const float4 *S, int grp, int ec, float rx, float ry, unsigned best) {
  const float *D = reinterpret_cast<const float *>(S);
  int bi = grp;
  for (int j = min(grp + 3, ec - 1); j >= grp; --j) {
    const float *f = D + kEdgeFloats * j;
    if (__float_as_uint(edge_d2(f[0], f[1], f[2], f[3], f[4], f[5], rx, ry)) == best) bi = j;
  }
  return bi;
}

__device__ __forceinline__ int scan_resolve_global(const EdgeRec *E, int grp, int ec, float rx, float ry,
                                                   unsigned best) {
  int bi = grp;
  for (int j = min(grp + 3, ec - 1); j >= grp; --j) {
    const EdgeRec &r = E[j];
    if (__float_as_uint(edge_d2(r.ax, r.ay, r.exs, r.eys, r.ex, r.ey, rx, ry)) == best) bi = j;
  }
  return bi;
}

// Nearest edge and inside flag of the lane's pixel over all ec edges of the item at E.  When the item
// has at most kStageEdges edges they must already be staged in S; otherwise they are staged here.
__device__ __forceinline__ void scan_item(const EdgeRec *E, int ec, bool staged, float4 *S, int lane, float rx,
                                          float ry, int &bi, bool &par) {
  ScanState st;
  if (staged) {
    scan_start(st, S, ry);
    scan_lds(S, ec, 0, rx, ry, st);
    bi = scan_resolve_lds(S, st.grp, ec, rx, ry, st.best);
  } else {
    for (int e0 = 0; e0 < ec; e0 += kStageEdges) {
      const int ne = min(kStageEdges, ec - e0);
      stage_edges(E + e0, ne, S, lane);
      if (e0 == 0) scan_start(st, S, ry);
      scan_lds(S, ne, e0, rx, ry, st);
    }
    bi = scan_resolve_global(E, st.grp, ec, rx, ry, st.best);
  }
  scan_finish(st);
  par = ((st.par >> lane) & 1ull) != 0ull;
}

// Pixel of `lane` in chunk j of a unit rectangle (in = false past the rectangle's last pixel; the
// lane then computes on the rectangle's first pixel and its results are discarded).
__device__ __forceinline__ void chunk_pixel(const Rect &r, int j, int lane, int &px, int &py, bool &in) {
  const int i = j * 64 + lane;
  in = i < r.n;
  const int ly = in ? i / r.w : 0;
  px = r.x0 + (in ? i - ly * r.w : 0);
  py = r.y0 + ly;
}

// The same pixels for consecutive chunks without a division per chunk: the next chunk is 64 pixels
// further along the rectangle's rows, i.e. 64 / w rows and 64 mod w columns, with one carry.
struct ChunkPix {
  int i, lx, ly;  // the lane's index in the rectangle and its column and row there
  int dx, dy;     // per chunk (wave-uniform)
};

__device__ __forceinline__ ChunkPix chunk_start(const Rect &r, int j, int lane) {
  ChunkPix c;
  c.i = j * 64 + lane;
  c.ly = c.i / r.w;
  c.lx = c.i - c.ly * r.w;
  c.dy = uniform(64 / r.w);
  c.dx = 64 - c.dy * r.w;
  return c;
}

__device__ __forceinline__ void chunk_step(ChunkPix &c, const Rect &r) {
  c.i += 64;
  c.lx += c.dx;
  c.ly += c.dy;
  if (c.lx >= r.w) {
    c.lx -= r.w;
    ++c.ly;
  }
}

// The pixel of the iterator's chunk, as chunk_pixel gives it.
__device__ __forceinline__ void chunk_at(const ChunkPix &c, const Rect &r, int &px, int &py, bool &in) {
  in = c.i < r.n;
  px = r.x0 + (in ? c.lx : 0);
  py = r.y0 + (in ? c.ly : 0);
}

// A unit record as the persistent passes use it (scalar loads and unpacking).  The float scan takes each
// pixel's position relative to the double origin, computed in double and rounded once.
struct UnitView {
  Rect r;
  int eo, ec, nv, head;
  bool open;
  float orient;
  double cx, cy;
  double sw, sw_ds;  // an open item's stroke radius and its derivative in s (0 for a closed item)
  double inv_s;      // 1 / s (0 when |s| < kScaleFloor)
  double kc, ks;     // k R(theta), loaded only when |s| < kScaleFloor
};

// A unit record by scalar loads (U wave-uniform).
__device__ __forceinline__ UnitRec load_unit(cptr<UnitRec> U) {
  UnitRec u;
  u.eo = U->eo;
  u.ecnv = U->ecnv;
  u.flags = U->flags;
  u.head = U->head;
  u.xy = U->xy;
  u.wn = U->wn;
  u.sid = U->sid;
  u.s = U->s;
  u.cx = U->cx;
  u.cy = U->cy;
  return u;
}

__device__ __forceinline__ UnitView unit_view(const KArgs &a, const UnitRec &U) {
  UnitView v;
  const int xy = U.xy, wn = U.wn, ecnv = U.ecnv, fl = U.flags;
  v.r.x0 = xy & 0xffff;
  v.r.y0 = xy >> 16;
  v.r.w = wn & 0xffff;
  v.r.n = wn >> 16;
  v.eo = U.eo;
  v.ec = ecnv & 0xffff;
  v.nv = ecnv >> 16;
  v.head = U.head;
  v.open = (fl & kUnitOpen) != 0;
  v.orient = (fl & kUnitClockwise) ? -1.0f : 1.0f;
  v.cx = U.cx;
  v.cy = U.cy;
  v.sw = 0.0;
  v.sw_ds = 0.0;
  cptr<ShapeRec> SR = konst(a.shapes) + U.sid;
  if (v.open) {
    v.sw = SR->sw;
    v.sw_ds = SR->sw_ds;
  }
  const double s = (double)U.s;
  v.inv_s = 0.0;
  v.kc = 0.0;
  v.ks = 0.0;
  if (fabs(s) >= kScaleFloor) {
    v.inv_s = 1.0 / s;
  } else {
    v.kc = SR->kc;
    v.ks = SR->ks;
  }
  return v;
}

// Exclusive prefix sums of the tiles' coverage costs (pc) and chunks (pq), [tiles + 1] each, for at most
// kScanInCoverTiles tiles, by one 256-thread workgroup into LDS (two tiles per thread, DPP wave scans).
// Workgroup 0 also writes them to tile_pre for the later passes and advances the Adam step counter,
// which the scan kernel does otherwise.
__device__ void cover_tile_scan(const KArgs &a, long long *pc, long long *pq, int2 *cnt) {
  __shared__ unsigned long long s_w[2][4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nt = a.total_tiles, t0 = 2 * tid;
  const int2 c0 = t0 < nt ? a.tile_cost[t0] : make_int2(0, 0);
  const int2 c1 = t0 + 1 < nt ? a.tile_cost[t0 + 1] : make_int2(0, 0);
  if (t0 < nt) cnt[t0] = a.tile_units[t0];
  if (t0 + 1 < nt) cnt[t0 + 1] = a.tile_units[t0 + 1];
  const unsigned long long vc = (unsigned long long)c0.x + (unsigned long long)c1.x;
  const unsigned long long vq = (unsigned long long)c0.y + (unsigned long long)c1.y;
  const unsigned long long xc = wave_incl_scan_u64(vc), xq = wave_incl_scan_u64(vq);
  if (lane == 63) {
    s_w[0][w] = xc;
    s_w[1][w] = xq;
  }
  __syncthreads();
  unsigned long long oc = 0, oq = 0, tc = 0, tq = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (j < w) {
      oc += s_w[0][j];
      oq += s_w[1][j];
    }
    tc += s_w[0][j];
    tq += s_w[1][j];
  }
  const long long ec = (long long)(oc + xc - vc), eq = (long long)(oq + xq - vq);
  if (t0 < nt) {
    pc[t0] = ec;
    pq[t0] = eq;
  }
  if (t0 + 1 < nt) {
    pc[t0 + 1] = ec + c0.x;
    pq[t0 + 1] = eq + c0.y;
  }
  if (tid == 0) {
    pc[nt] = (long long)tc;
    pq[nt] = (long long)tq;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int t = tid; t <= nt; t += 256) {
      a.tile_pre[t] = pc[t];
      a.tile_pre[nt + 1 + t] = pq[t];
    }
    if (tid == 0) {
      if (a.step_inc != nullptr) a.step_inc[0] = a.step_inc[0] + 1;
      publish_chunk_status(a, (long long)tq);
    }
  }
}

// ------------------------------------------------------------------------------------------------
// k_cover: coverage of every (unit, pixel) into the fixed-point accumulators.
// ------------------------------------------------------------------------------------------------
// The persistent kernels assume that all their workgroups are resident at once (kPersistWaves waves
// per workgroup, k*BlocksPerCU workgroups per CU): the second launch bound keeps that many waves per
// SIMD within the register file.
template <int T>
__global__ __launch_bounds__(256, kCoverBlocksPerCU) void k_cover(KArgs a) {
  __shared__ float4 s_stage[kPersistWaves][kStageSlots];
  const int lane = threadIdx.x & 63;
  float4 *S = s_stage[threadIdx.x >> 6];
  const int gw = global_wave();
  const int nwaves = gridDim.x * (blockDim.x >> 6);
  Walk wk;
  // the tiles' cost and chunk prefixes: computed here in LDS by every workgroup for small scenes (no
  // separate scan launch; workgroup 0 publishes them for the later passes), else from the scan kernel
  __shared__ long long s_pre[2][kScanInCoverTiles + 1];
  __shared__ int2 s_cnt[kScanInCoverTiles];
  const long long *P = a.tile_pre, *Q = a.tile_pre + (a.total_tiles + 1);
  const int2 *C = nullptr;
  if (a.scan_in_cover) {
    cover_tile_scan(a, s_pre[0], s_pre[1], s_cnt);
    P = s_pre[0];
    Q = s_pre[1];
    C = s_cnt;
  }
  bool ok = walk_begin(a, wk, gw, nwaves, false, T, P, Q, C);
  for (; ok; ok = walk_next(a, wk, T)) {
    cptr<UnitRec> U = konst(a.units) + (wk.list_base + wk.slot);
    const UnitView uv = unit_view(a, load_unit(U));
    const Rect r = uv.r;
    const long long q = walk_chunk0(wk);
    const int eo = uv.eo, ec = uv.ec;
    const double cx = uv.cx, cy = uv.cy;
    const bool open = uv.open;
    const double sw = uv.sw;
    const bool staged = ec <= kStageEdges;
    if (staged) stage_edges(a.edges + eo, ec, S, lane);
    ChunkPix it = chunk_start(r, wk.jlo, lane);
    for (int j = wk.jlo; j < wk.jhi; ++j, chunk_step(it, r)) {
      int pxi, pyi;
      bool in;
      chunk_at(it, r, pxi, pyi, in);
      int bi = 0;
      bool par = false;
      // the pixel relative to the item's origin, in double, and rounded once for the float scan
      const double rx = pxi + 0.5 - cx, ry = pyi + 0.5 - cy;
      scan_item(a.edges + eo, ec, staged, S, lane, (float)rx, (float)ry, bi, par);
      if (ec > 0) {
        const Nearest nr = nearest_refined(a.edges_d + eo, ec, bi, rx, ry);
        bi = nr.e;
        if (in) {
          const double d = sqrt(nr.d2);
          double al, alp;
          coverage_pair(a, open ? sw - d : (par ? d : -d), al, alp);
          const int64_t pix = wk.pix_off + (int64_t)pyi * wk.W + pxi;
          if (al > 0.0) atomicAdd(&a.acc[2 * pix], (unsigned long long)llrint(al * kFixScale));
          if (alp > 0.0) atomicAdd(&a.acc[2 * pix + 1], (unsigned long long)llrint(alp * kFixScale));
        }
      }
      if (a.keep_codes && q + j < a.code_cap) a.codes[(q + j) * 64 + lane] = (uint16_t)(bi | (par ? 0x8000 : 0));
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Per-pixel pass and the uniform term.  Both work on kPixTile x kPixTile pixel tiles of a layout, one
// pixel per thread.
//
// The uniform term (Sec. 4.2, eq. 7).  With O = min(S, 1) and windows of 5 + 6 j pixels (radius
// 2 + 3 j, j < kUniWindows) clipped to the canvas, A_j(p) is the sum of O over the window around p;
//   L_unif = sum_j (b_j / b_0) sum_p M(p) relu(1 - A_j(p)),
//   dL_unif/dS(q) = -1(S(q) < 1) sum_j (b_j / b_0) sum_{p : q in window_j(p)} M(p) 1(A_j(p) < 1).
// A tile and a halo of the largest radius go into LDS in the 2^-40 fixed point of the coverage
// accumulators and become a summed-area table, from which every window sum is four lookups.  The sums
// are integers, so A_j is exact given the accumulated S and neither the A_j < 1 decisions nor the
// results depend on an order of summation.
// ------------------------------------------------------------------------------------------------
constexpr int kPixWaves = kPixThreads / 64;
constexpr int kUniReg = kPixTile + 2 * kUniHalo;  // region edge: tile + halo on both sides
constexpr int kUniPitch = kUniReg + 1;            // table row pitch (row 0 and column 0 hold zeros)
constexpr int kUniBand = (kUniReg + kPixWaves - 1) / kPixWaves;  // region rows per wave
static_assert(kPixTile * kPixTile == kPixThreads, "one pixel per thread");
static_assert(kUniHalo == 2 + 3 * (kUniWindows - 1), "halo must be the largest window radius");
static_assert(kUniReg <= 64, "a region row must fit one wave");

__device__ __forceinline__ int uni_radius(int j) { return 2 + 3 * j; }
__device__ __forceinline__ double uni_weight(int j) { return (5.0 + 6.0 * j) / 5.0; }

struct PixTile {
  int b, W, H;
  int x0, y0;  // pixel of the tile's top-left corner
  int64_t pix_off;
};

__device__ __forceinline__ PixTile pix_tile(cptr<LayoutRec> L, int B, int blk) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (L[mid].ptile_off <= blk)
      lo = mid;
    else
      hi = mid - 1;
  }
  PixTile u;
  u.b = lo;
  u.W = L[lo].W;
  u.H = L[lo].H;
  const int ntx = (u.W + kPixTile - 1) / kPixTile;
  const int t = blk - L[lo].ptile_off;
  const int ty = t / ntx;
  u.y0 = ty * kPixTile;
  u.x0 = (t - ty * ntx) * kPixTile;
  u.pix_off = L[lo].pix_off;
  return u;
}

// The pixel of region cell (rx, ry) (0 <= rx, ry < kUniReg), or -1 off the canvas or the region.
__device__ __forceinline__ int64_t uni_cell_pixel(const PixTile &u, int rx, int ry) {
  const int gx = u.x0 - kUniHalo + rx, gy = u.y0 - kUniHalo + ry;
  if (rx >= kUniReg || ry >= kUniReg || gx < 0 || gx >= u.W || gy < 0 || gy >= u.H) return -1;
  return u.pix_off + (int64_t)gy * u.W + gx;
}

// Zeroes row 0 and column 0 of NCH tables.
template <int NCH>
__device__ __forceinline__ void uni_zero_border(unsigned long long *T) {
  for (int i = threadIdx.x; i < NCH * kUniPitch; i += kPixThreads) {
    unsigned long long *t = T + (i / kUniPitch) * kUniPitch * kUniPitch;
    const int k = i % kUniPitch;
    t[k] = 0ull;
    t[k * kUniPitch] = 0ull;
  }
}

// Summed-area tables of NCH sets of region values v[c] (wave w holds rows w kUniBand + i in v[c][i],
// lane = column; zero at lanes and rows outside the region) into T + c kUniPitch^2:
// T[(ry + 1) kUniPitch + rx + 1] = sum of the values at rows <= ry, columns <= rx.  Row prefix sums are
// wave scans, column sums run down each wave's band in registers and are then offset by the totals of
// the bands above.  Two barriers: band totals are exchanged after the first (so every read of T before
// the call is complete when T is rewritten), and T is complete after the second.
template <int NCH>
__device__ void sat_build(unsigned long long *T, unsigned long long *band_tot,
                          unsigned long long (&v)[NCH][kUniBand]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned long long col[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) col[c] = 0ull;
#pragma unroll
  for (int i = 0; i < kUniBand; ++i) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      col[c] += wave_incl_scan_u64(v[c][i]);
      v[c][i] = col[c];
    }
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c) band_tot[(c * kPixWaves + w) * 64 + lane] = col[c];
  __syncthreads();
  if (lane < kUniReg) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      // every band total is loaded (issued together), those of the bands above are added
      unsigned long long off = 0ull;
#pragma unroll
      for (int q = 0; q < kPixWaves; ++q) {
        const unsigned long long t = band_tot[(c * kPixWaves + q) * 64 + lane];
        off += q < w ? t : 0ull;
      }
#pragma unroll
      for (int i = 0; i < kUniBand; ++i) {
        const int ry = w * kUniBand + i;
        if (ry < kUniReg) T[c * kUniPitch * kUniPitch + (ry + 1) * kUniPitch + lane + 1] = v[c][i] + off;
      }
    }
  }
  __syncthreads();
}

// Sum of the values in the window of radius r around region cell (cx, cy) (0-based region coordinates).
// Unsigned wrap-around cancels in the four-corner difference, so the result is exact whenever the
// window sum itself fits.
__device__ __forceinline__ unsigned long long sat_box(const unsigned long long *T, int cx, int cy, int r) {
  const int xa = cx - r, xb = cx + r + 1, ya = (cy - r) * kUniPitch, yb = (cy + r + 1) * kUniPitch;
  return ((T[yb + xb] - T[ya + xb]) - T[yb + xa]) + T[ya + xa];
}

// k_pixel: S, S_pad, the loss terms (summed per tile) and dLoss/dS, dLoss/dS_pad of the per-pixel
// terms.  UNI (uniform weight != 0): also the A_j of the tile's pixels, the uniform term, and for the
// gradient the bits M != 0 and A_j < 1 that k_unif_grad needs.  The first tile of each layout also adds
// the object-space downward force over the layout's items (their transforms are final for this epoch).
template <bool GRAD, bool UNI>
__global__ __launch_bounds__(UNI ? kPixThreads : 256) void k_pixel(KArgs a) {
  // without the uniform term a workgroup of 256 threads takes the tile, four pixels per thread with
  // all their loads in flight together (1024 threads of one pixel each were 0.3 us slower at 512^2);
  // the window pass needs one thread per pixel (16 waves)
  constexpr int NT = UNI ? kPixThreads : 256, PX = kPixTile * kPixTile / NT, NW = NT / 64;
  __shared__ double s_loss[NW][kLossTerms];
  __shared__ unsigned long long T[UNI ? kUniPitch * kUniPitch : 1];
  __shared__ unsigned long long band_tot[UNI ? kPixWaves * 64 : 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  cptr<LayoutRec> LS = konst(a.layouts);
  const PixTile u = pix_tile(LS, a.num_layouts, blockIdx.x);
  bool mine[PX];
  int64_t pix[PX];
  unsigned long long s0[PX], s1[PX];
  float mk[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    const int i = tid + NT * k, px = u.x0 + i % kPixTile, py = u.y0 + i / kPixTile;
    mine[k] = px < u.W && py < u.H;
    pix[k] = u.pix_off + (int64_t)py * u.W + px;
    s0[k] = s1[k] = 0ull;
    mk[k] = 0.0f;
    if (mine[k]) {
      s0[k] = a.acc[2 * pix[k]];
      s1[k] = a.acc[2 * pix[k] + 1];
      mk[k] = a.mask[pix[k]];
    }
  }
  unsigned long long v[1][kUniBand];
  if (UNI) {
    uni_zero_border<1>(T);
#pragma unroll
    for (int i = 0; i < kUniBand; ++i) {
      const int64_t q = uni_cell_pixel(u, lane, w * kUniBand + i);
      v[0][i] = q >= 0 ? a.acc[2 * q] : 0ull;
    }
  }
  // weights, with the 1 / (W H) of the image-mismatch terms when asked for
  const double nu = a.area_mean ? 1.0 / ((double)u.W * (double)u.H) : 1.0;
  double wt[kLossTerms];
#pragma unroll
  for (int t = 0; t < kLossTerms; ++t)
    wt[t] = (double)a.w[t] * ((t <= 3 || t == 6) ? nu : 1.0);
  double c_ov = wt[0], c_c = wt[1], c_f = wt[2], c_p = wt[3], c_d = wt[4], c_w = wt[6], c_cen = wt[7];
  if (GRAD && a.dloss) {
    const float *dl = a.dloss + kLossTerms * u.b;
    c_ov *= (double)dl[0];
    c_c *= (double)dl[1];
    c_f *= (double)dl[2];
    c_p *= (double)dl[3];
    c_d *= (double)dl[4];
    c_w *= (double)dl[6];
    c_cen *= (double)dl[7];
  }
  double term[kLossTerms];
#pragma unroll
  for (int t = 0; t < kLossTerms; ++t) term[t] = 0.0;
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    if (!mine[k]) continue;
    const int i = tid + NT * k, px = u.x0 + i % kPixTile, py = u.y0 + i / kPixTile;
    const double S = (double)s0[k] * kFixInv, Sp = (double)s1[k] * kFixInv, M = (double)mk[k];
    if (a.cov_out) a.cov_out[pix[k]] = (float)S;
    if (a.cov_pad_out) a.cov_pad_out[pix[k]] = (float)Sp;
    const double yinv = (double)u.H - (py + 0.5);
    const double ov = fmax(S - 1.0, 0.0), un = fmax(1.0 - S, 0.0), pv = fmax(Sp - 1.0, 0.0);
    // the terms that a scene leaves at weight 0 (uniform branches) are neither summed nor differentiated
    const bool on_w = a.w[6] != 0.0f, on_cen = a.w[7] != 0.0f;
    const double O = fmin(S, 1.0), Wp = kWmseIn * M + kWmseOut * (1.0 - M);
    double dist = 0.0;
    if (on_cen) {
      const double cx = (px + 0.5) - 0.5 * u.W, cy = (py + 0.5) - 0.5 * u.H;
      dist = sqrt(cx * cx + cy * cy);
    }
    term[0] += ov * ov;
    term[1] += S * (1.0 - M);
    term[2] += M * (un * un);
    term[3] += pv * pv;
    term[4] += S * yinv;
    if (on_w) term[6] += Wp * ((M - O) * (M - O));
    if (on_cen) term[7] += S * dist;
    if (GRAD) {
      double G = 2.0 * c_ov * ov + c_c * (1.0 - M) - 2.0 * c_f * (M * un) + c_d * yinv;
      if (on_w && S < 1.0) G -= 2.0 * c_w * (Wp * (M - S));
      if (on_cen) G += c_cen * dist;
      const double Gp = 2.0 * c_p * pv;
      __builtin_nontemporal_store((nt_f64x2){G, Gp}, reinterpret_cast<nt_f64x2 *>(a.gbuf + pix[k]));
    }
  }
  if (UNI) {
#pragma unroll
    for (int i = 0; i < kUniBand; ++i) v[0][i] = v[0][i] < kFixOne ? v[0][i] : kFixOne;
    sat_build<1>(T, band_tot, v);
    const int ox = tid % kPixTile, oy = tid / kPixTile;
    unsigned bits = 0;
    if (mine[0] && mk[0] != 0.0f) {
#pragma unroll
      for (int j = 0; j < kUniWindows; ++j) {
        const unsigned long long box = sat_box(T, ox + kUniHalo, oy + kUniHalo, uni_radius(j));
        if (box < kFixOne) {
          bits |= 1u << j;
          term[5] += uni_weight(j) * ((double)mk[0] * ((double)(kFixOne - box) * kFixInv));
        }
      }
    }
    if (GRAD && mine[0]) a.uflags[pix[0]] = (uint8_t)bits;
  }
  if (blockIdx.x == LS[u.b].ptile_off) {
    // the first tile of each layout counts the layout's items whose parameters are not finite into the
    // status word (zeroed by this call's transform kernel)
    int bad = 0;
    for (int q = LS[u.b].shape_begin + tid; q < LS[u.b].shape_end; q += NT) bad += a.shapes[q].bad;
    if (bad != 0) atomicAdd(&a.status[COLLAGE_STATUS_NONFINITE], bad);
  }
  if (a.write_loss) {
    if (a.w[8] != 0.0f && blockIdx.x == LS[u.b].ptile_off) {
      cptr<ShapeRec> SR = konst(a.shapes);
      for (int q = LS[u.b].shape_begin + tid; q < LS[u.b].shape_end; q += NT) term[8] += (double)u.H - SR[q].cy;
    }
    // a term with weight 0 is 0; terms 0-7 are summed together, term 8 (only the first tile of a layout
    // has it) on its own when its weight is not 0 (the branch is the same for the whole grid)
    static_assert(kLossTerms == 9, "loss terms");
    double v8[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v8[t] = a.w[t] != 0.0f ? wt[t] * term[t] : 0.0;
    int c0;
    const double2 r8 = wave_sum8(v8, c0);
    if (lane < 4) {
      s_loss[w][c0] = r8.x;
      s_loss[w][c0 + 1] = r8.y;
    }
    const double s8 = a.w[8] != 0.0f ? wave_sum(wt[8] * term[8]) : 0.0;
    if (lane == 0) s_loss[w][8] = s8;
    __syncthreads();
    if (tid < kLossTerms) {
      double s = 0.0;
      for (int q = 0; q < NW; ++q) s += s_loss[q][tid];
      a.block_loss[(int64_t)blockIdx.x * kLossTerms + tid] = s;
    }
  }
}

// k_unif_grad: for each window size j, the window sums of F_j = M 1(A_j < 1) (the pixels whose window_j
// contains q are those in q's own window_j), weighted and added into dLoss/dS where S < 1.
// A tile whose region has a binary mask (every M 0 or 1) counts the flags: the four counts, at most
// kUniReg^2 < 2^16 each, travel as 16-bit fields of one 64-bit value through one table (a field's window
// sum never carries into the next, so each count is exact).  Otherwise the four tables hold M in 2^-40
// fixed point.
constexpr int kUniField = 16;
static_assert(kUniReg * kUniReg < (1 << kUniField) && kUniWindows * kUniField <= 64, "flag counts must fit");

__global__ __launch_bounds__(kPixThreads) void k_unif_grad(KArgs a) {
  __shared__ unsigned long long T[kUniWindows * kUniPitch * kUniPitch];
  __shared__ unsigned long long band_tot[kUniWindows * kPixWaves * 64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const PixTile u = pix_tile(konst(a.layouts), a.num_layouts, blockIdx.x);
  const double cu = (double)a.w[5] * (a.dloss ? (double)a.dloss[kLossTerms * u.b + 5] : 1.0);
  if (cu == 0.0) return;  // the same for every thread of the block
  const int ox = tid % kPixTile, oy = tid / kPixTile;
  const int px = u.x0 + ox, py = u.y0 + oy;
  const int64_t pix = u.pix_off + (int64_t)py * u.W + px;
  // S < 1 at the thread's own pixel (only there does O = min(S, 1) pass a gradient); its dLoss/dS
  // is fetched now, with the other loads
  const bool mine = px < u.W && py < u.H && a.acc[2 * pix] < kFixOne;
  const double g0 = mine ? a.gbuf[pix].x : 0.0;
  unsigned fl[kUniBand];
  float mk[kUniBand];
  bool binary = true;
#pragma unroll
  for (int i = 0; i < kUniBand; ++i) {
    const int64_t q = uni_cell_pixel(u, lane, w * kUniBand + i);
    fl[i] = 0u;
    mk[i] = 0.0f;
    if (q >= 0) {
      fl[i] = a.uflags[q];
      mk[i] = a.mask[q];
    }
    binary = binary && (fl[i] == 0u || mk[i] == 1.0f);
  }
  uni_zero_border<kUniWindows>(T);
  double g = 0.0;
  if (__syncthreads_and(binary)) {
    unsigned long long v[1][kUniBand];
#pragma unroll
    for (int i = 0; i < kUniBand; ++i) {
      unsigned long long x = 0ull;
#pragma unroll
      for (int j = 0; j < kUniWindows; ++j) x |= (unsigned long long)((fl[i] >> j) & 1u) << (kUniField * j);
      v[0][i] = x;
    }
    sat_build<1>(T, band_tot, v);
#pragma unroll
    for (int j = 0; j < kUniWindows; ++j) {
      const unsigned long long box = sat_box(T, ox + kUniHalo, oy + kUniHalo, uni_radius(j));
      g += uni_weight(j) * (double)((box >> (kUniField * j)) & ((1ull << kUniField) - 1ull));
    }
  } else {
    unsigned long long v[kUniWindows][kUniBand];
#pragma unroll
    for (int i = 0; i < kUniBand; ++i) {
      const unsigned long long m = fl[i] ? (unsigned long long)llrint((double)mk[i] * kFixScale) : 0ull;
#pragma unroll
      for (int j = 0; j < kUniWindows; ++j) v[j][i] = ((fl[i] >> j) & 1u) ? m : 0ull;
    }
    sat_build<kUniWindows>(T, band_tot, v);
#pragma unroll
    for (int j = 0; j < kUniWindows; ++j)
      g += uni_weight(j) *
           (double)(long long)sat_box(T + j * kUniPitch * kUniPitch, ox + kUniHalo, oy + kUniHalo, uni_radius(j));
    g *= kFixInv;
  }
  if (mine && g != 0.0) a.gbuf[pix].x = g0 - cu * g;
}

// The head partials of a unit.  Every pixel's four gradient terms are rounded to multiples of 2^-30
// (kept as integer-valued doubles, rint(ldexp(x, 30)): two instructions and no constant registers), so
// that every later sum is a sum of integers, exact while below 2^53: the per-lane sums over a piece's chunks (the chunks of the unit in one wave's
// share), the piece's wave sum, and, as 64-bit integers added with atomics, the unit's total over its
// pieces.  The totals thus depend neither on the order of the pieces nor on where the work partition
// cuts the unit (a batch of layouts and each layout on its own give the same bits).  A piece whose sums
// reach 2^23 in magnitude (2^53 units), in any lane or in total, or are not finite, is left out and
// counted in the status word COLLAGE_STATUS_GRAD_RANGE; a unit has at most 16 pieces, so its totals stay
// below 2^57 units.
constexpr int kHeadBits = 30;                      // units of 2^-30
constexpr double kHeadLimit = 9007199254740992.0;  // 2^53 units

__device__ __forceinline__ double head_round(double x) { return rint(ldexp(x, kHeadBits)); }

__device__ __forceinline__ void head_accumulate(double4 &acc, const double4 &t) {
  acc.x += head_round(t.x);
  acc.y += head_round(t.y);
  acc.z += head_round(t.z);
  acc.w += head_round(t.w);
}

// The piece's per-lane sums acc (integer-valued, units of 2^-30) into the unit's head partials.  Every
// lane must be active.
__device__ __forceinline__ void piece_to_head(const KArgs &a, int head, double4 acc) {
  const int lane = threadIdx.x & 63;
  const bool lane_ok = fabs(acc.x) + fabs(acc.y) + fabs(acc.z) + fabs(acc.w) < kHeadLimit;
  const bool all_ok = __ballot(!lane_ok) == 0ull;
  int comp;
  const double tot = wave_sum4(acc, comp);
  if (lane < 4) {
    if (!all_ok || !(fabs(tot) < kHeadLimit)) {
      if (lane == 0) atomicAdd(&a.status[COLLAGE_STATUS_GRAD_RANGE], 1);
    } else if (tot != 0.0) {
      atomicAdd(a.head + 4 * (int64_t)head + comp, (unsigned long long)(long long)tot);
    }
  }
}

// ------------------------------------------------------------------------------------------------
// k_adjoint: per unit, the gradient terms of its pixels reduced per piece and added into the unit's head
// partials.
// ------------------------------------------------------------------------------------------------
template <int T>
__global__ __launch_bounds__(256, kAdjointBlocksPerCU) void k_adjoint(KArgs a) {
  __shared__ float4 s_stage[kPersistWaves][kStageSlots];
  const int lane = threadIdx.x & 63;
  float4 *S = s_stage[threadIdx.x >> 6];
  const int gw = global_wave();
  const int nwaves = gridDim.x * (blockDim.x >> 6);
  Walk wk;
  const long long *Qg = a.tile_pre + (a.total_tiles + 1);
  bool ok = walk_begin(a, wk, gw, nwaves, true, T, Qg, Qg, nullptr);
  for (; ok; ok = walk_next(a, wk, T)) {
    const UnitView uv = unit_view(a, load_unit(konst(a.units) + (wk.list_base + wk.slot)));
    const Rect r = uv.r;
    const long long q = walk_chunk0(wk);
    const int eo = uv.eo, ec = uv.ec;
    const float orient = uv.orient;
    const double cx = uv.cx, cy = uv.cy;
    const bool open = uv.open;
    const double sw = uv.sw, sw_ds = uv.sw_ds;
    // (a binned item has at least one edge: an item without vertices has an empty support box)
    const bool staged = ec <= kStageEdges;
    ScaleDeriv sdv = {uv.inv_s, uv.kc, uv.ks, reinterpret_cast<const float2 *>(a.verts) + eo, 0, uv.nv, open};
    double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);  // the lane's rounded terms (units of 2^-30)
    if (q + wk.jhi <= a.code_cap) {
      // every chunk of the piece has its nearest-edge codes: a three-stage pipeline over the chunks
      // (codes two chunks ahead, the edge record and dLoss/dS one chunk ahead), since each chunk's
      // loads depend on its codes and the wave has nothing else to cover their latency
      const uint16_t *C = a.codes + q * 64 + lane;
      const int j0 = wk.jlo, j1 = wk.jhi;
      unsigned c_cur = C[(int64_t)j0 * 64];
      unsigned c_nxt = j0 + 1 < j1 ? C[(int64_t)(j0 + 1) * 64] : 0u;
      int px, py;
      bool in;
      chunk_pixel(r, j0, lane, px, py, in);
      EdgeD e_cur = a.edges_d[eo + (int)(c_cur & 0x7fffu)];
      double2 g_cur = a.gbuf[wk.pix_off + (int64_t)py * wk.W + px];
      for (int j = j0; j < j1; ++j) {
        const unsigned c_far = j + 2 < j1 ? C[(int64_t)(j + 2) * 64] : 0u;
        int pn_x = px, pn_y = py;
        bool in_n = false;
        EdgeD e_nxt = e_cur;
        double2 g_nxt = g_cur;
        if (j + 1 < j1) {
          chunk_pixel(r, j + 1, lane, pn_x, pn_y, in_n);
          e_nxt = a.edges_d[eo + (int)(c_nxt & 0x7fffu)];
          g_nxt = a.gbuf[wk.pix_off + (int64_t)pn_y * wk.W + pn_x];
        }
        if (in) {
          const double rx = px + 0.5 - cx, ry = py + 0.5 - cy;
          const bool par = !open && (c_cur & 0x8000u) != 0u;
          PairD pr = pair_eval(e_cur, rx, ry, par);
          if (open) pr.sd = sw - pr.d;
          sdv.bi = (int)(c_cur & 0x7fffu);
          head_accumulate(acc, adjoint_terms(a, e_cur, pr, rx, ry, par, orient, g_cur.x, g_cur.y, open, sw_ds, sdv));
        }
        c_cur = c_nxt;
        c_nxt = c_far;
        e_cur = e_nxt;
        g_cur = g_nxt;
        px = pn_x;
        py = pn_y;
        in = in_n;
      }
    } else {
      if (staged) stage_edges(a.edges + eo, ec, S, lane);
      for (int j = wk.jlo; j < wk.jhi; ++j) {
        int pxi, pyi;
        bool in;
        chunk_pixel(r, j, lane, pxi, pyi, in);
        const double rx = pxi + 0.5 - cx, ry = pyi + 0.5 - cy;
        int bi = 0;
        bool par = false;
        if (q + j < a.code_cap) {
          const unsigned code = a.codes[(q + j) * 64 + lane];
          bi = (int)(code & 0x7fffu);
          par = (code & 0x8000u) != 0u;
        } else {
          scan_item(a.edges + eo, ec, staged, S, lane, (float)rx, (float)ry, bi, par);
          bi = nearest_refined(a.edges_d + eo, ec, bi, rx, ry).e;
        }
        if (in) {
          const int64_t pix = wk.pix_off + (int64_t)pyi * wk.W + pxi;
          const double2 g = a.gbuf[pix];
          const EdgeD e = a.edges_d[eo + bi];
          if (open) par = false;
          PairD pr = pair_eval(e, rx, ry, par);
          if (open) pr.sd = sw - pr.d;
          sdv.bi = bi;
          head_accumulate(acc, adjoint_terms(a, e, pr, rx, ry, par, orient, g.x, g.y, open, sw_ds, sdv));
        }
      }
    }
    piece_to_head(a, uv.head, acc);
  }
}

// ------------------------------------------------------------------------------------------------
// Outline (control-point) gradients (Sec. 3 "Vector Representation": the control points are fitted by
// differentiable rendering).  k_vgrad walks the adjoint's units; per pixel the nearest point
// q' = a' + u (b' - a') of the nearest edge moves with its two end points, d sd / d a' = -n (1 - u) and
// d sd / d b' = -n u, and omega times those is added into the end points' accumulators (level frame,
// 2^-32 fixed point, so the sums do not depend on the order of the atomics).  k_vfinal maps each vertex
// sum back through eq. 2 (dv'/dv = k s R(theta)).
// ------------------------------------------------------------------------------------------------
constexpr double kVertFix = 4294967296.0;  // 2^32

__device__ __forceinline__ void vert_add(unsigned long long *acc, double x) {
  if (x != 0.0) atomicAdd(acc, (unsigned long long)llrint(x * kVertFix));
}

constexpr int kVertLds = 128;  // items with up to this many vertices gather a unit piece's sums in LDS

template <int T>
__global__ __launch_bounds__(256, kAdjointBlocksPerCU) void k_vgrad(KArgs a) {
  __shared__ float4 s_stage[kPersistWaves][kStageSlots];
  __shared__ unsigned long long s_vacc[kPersistWaves][2 * kVertLds];
  const int lane = threadIdx.x & 63;
  float4 *S = s_stage[threadIdx.x >> 6];
  unsigned long long *L = s_vacc[threadIdx.x >> 6];
  const int gw = global_wave();
  const int nwaves = gridDim.x * (blockDim.x >> 6);
  Walk wk;
  const long long *Qg = a.tile_pre + (a.total_tiles + 1);
  for (bool ok = walk_begin(a, wk, gw, nwaves, true, T, Qg, Qg, nullptr); ok; ok = walk_next(a, wk, T)) {
    const UnitView uv = unit_view(a, load_unit(konst(a.units) + (wk.list_base + wk.slot)));
    const Rect r = uv.r;
    const long long q = walk_chunk0(wk);
    const int eo = uv.eo, ec = uv.ec, nv = uv.nv;
    const float orient = uv.orient;
    const double cx = uv.cx, cy = uv.cy;
    const bool open = uv.open;
    const double sw = uv.sw;
    const bool staged = ec <= kStageEdges;
    // small items: the piece's vertex sums gather in the wave's LDS (64-bit integer atomics, so the
    // order does not matter), then one global atomic per vertex and component; large items add directly
    const bool gather = nv <= kVertLds;
    unsigned long long *acc = gather ? L : a.vacc + 2 * eo;
    if (gather)
      for (int m = lane; m < 2 * nv; m += 64) L[m] = 0ull;
    if (staged && q + wk.jhi > a.code_cap) stage_edges(a.edges + eo, ec, S, lane);
    for (int j = wk.jlo; j < wk.jhi; ++j) {
      int pxi, pyi;
      bool in;
      chunk_pixel(r, j, lane, pxi, pyi, in);
      const double rx = pxi + 0.5 - cx, ry = pyi + 0.5 - cy;
      int bi = 0;
      bool par = false;
      if (q + j < a.code_cap) {
        const unsigned code = a.codes[(q + j) * 64 + lane];
        bi = (int)(code & 0x7fffu);
        par = (code & 0x8000u) != 0u;
      } else {
        scan_item(a.edges + eo, ec, staged, S, lane, (float)rx, (float)ry, bi, par);
        bi = nearest_refined(a.edges_d + eo, ec, bi, rx, ry).e;
      }
      if (in) {
        const double2 g = a.gbuf[wk.pix_off + (int64_t)pyi * wk.W + pxi];
        const EdgeD e = a.edges_d[eo + bi];
        if (open) par = false;
        PairD pr = pair_eval(e, rx, ry, par);
        if (open) pr.sd = sw - pr.d;
        const double om = adjoint_omega(a, pr.sd, g.x, g.y);
        if (om != 0.0 && pr.d != 0.0) {
          double nx, ny;
          adjoint_normal(e, pr, par, orient, open, nx, ny);
          const int ib = open ? min(bi + 1, nv - 1) : (bi + 1 == nv ? 0 : bi + 1);
          const double fa = -om * (1.0 - pr.u), fb = -om * pr.u;
          vert_add(&acc[2 * bi], fa * nx);
          vert_add(&acc[2 * bi + 1], fa * ny);
          vert_add(&acc[2 * ib], fb * nx);
          vert_add(&acc[2 * ib + 1], fb * ny);
        }
      }
    }
    if (gather) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      for (int m = lane; m < 2 * nv; m += 64) {
        const unsigned long long x = L[m];
        if (x != 0ull) atomicAdd(&a.vacc[2 * eo + m], x);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

// One wave per item: dL/dv = (k s R(theta))^T dL/dv' for each of its vertices (NaN for an item with a
// non-finite parameter).
__global__ __launch_bounds__(256) void k_vfinal(KArgs a) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sid = blockIdx.x * 4 + wave;
  if (sid >= a.num_shapes) return;
  const int v0 = a.vert_off[sid], n = a.vert_off[sid + 1] - v0;
  const float4 p = reinterpret_cast<const float4 *>(a.params)[sid];
  const bool bad = konst(a.shapes)[sid].bad != 0;
  const double ks = (double)konst(a.shapes)[sid].k * (double)p.w;
  double sn = 0.0, c = 1.0;
  if (!bad) sincos((double)p.z, &sn, &c);
  for (int m = lane; m < n; m += 64) {
    const double gx = (double)(long long)a.vacc[2 * (v0 + m)] / kVertFix;
    const double gy = (double)(long long)a.vacc[2 * (v0 + m) + 1] / kVertFix;
    float2 out = make_float2((float)(ks * (c * gx + sn * gy)), (float)(ks * (-sn * gx + c * gy)));
    if (bad) out = make_float2(NAN, NAN);
    reinterpret_cast<float2 *>(a.grad_verts_out)[v0 + m] = out;
  }
}

// ------------------------------------------------------------------------------------------------
// k_finalize: per-item gradient (fixed tile order) + optional Adam; per-layout loss.
// ------------------------------------------------------------------------------------------------
// The parameters, moments and rim radius an Adam step of item sid reads (loaded ahead of the gradient).
struct AdamIn {
  float4 p, m, v;
  float rho;
  float bc1, bc2;  // bias corrections 1 - beta1^t, 1 - beta2^t of the step t (already incremented)
};


// bias: the step's bias corrections (adam_bias_of), computed by the caller or loaded.
__device__ __forceinline__ AdamIn adam_load(const KArgs &a, int sid, float2 bias) {
  AdamIn r;
  r.p = reinterpret_cast<const float4 *>(a.param_io)[sid];
  r.m = reinterpret_cast<const float4 *>(a.adam_m)[sid];
  r.v = reinterpret_cast<const float4 *>(a.adam_v)[sid];
  r.rho = *(a.rho ? a.rho + sid : &kNoFloat);
  r.bc1 = bias.x;
  r.bc2 = bias.y;
  return r;
}

__device__ __forceinline__ float4 adam_update(const KArgs &a, int sid, float4 g, float k, const AdamIn &in) {
  const float bc1 = in.bc1, bc2 = in.bc2;
  const float lr_t = a.lr_px / k;
  const float lr_r = in.rho > 0.0f ? a.lr_px / (k * in.rho) : 0.0f;
  const float gg[4] = {g.x, g.y, g.z, g.w};
  const float lr[4] = {lr_t, lr_t, lr_r, lr_r};
  float pp[4] = {in.p.x, in.p.y, in.p.z, in.p.w}, mm[4] = {in.m.x, in.m.y, in.m.z, in.m.w};
  float vv[4] = {in.v.x, in.v.y, in.v.z, in.v.w};
  const float sqbc2 = sqrtf(bc2);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    mm[j] = a.beta1 * mm[j] + (1.0f - a.beta1) * gg[j];
    vv[j] = a.beta2 * vv[j] + (1.0f - a.beta2) * gg[j] * gg[j];
    const float denom = sqrtf(vv[j]) / sqbc2 + a.eps;
    pp[j] = pp[j] - (lr[j] / bc1) * mm[j] / denom;
  }
  reinterpret_cast<float4 *>(a.param_io)[sid] = make_float4(pp[0], pp[1], pp[2], pp[3]);
  reinterpret_cast<float4 *>(a.adam_m)[sid] = make_float4(mm[0], mm[1], mm[2], mm[3]);
  reinterpret_cast<float4 *>(a.adam_v)[sid] = make_float4(vv[0], vv[1], vv[2], vv[3]);
  return make_float4(pp[0], pp[1], pp[2], pp[3]);
}

// ADAM: update the parameters; XFORM (with ADAM): transform the items with the updated parameters.
// The loads of the update and of the transform are issued first and consumed last, so that they are in
// flight while the gradient is gathered.  per: items per workgroup (its first per waves take one each).
template <int T, bool ADAM, bool XFORM>
__device__ void finalize_grad(const KArgs &a, int per) {
  constexpr bool do_adam = ADAM, do_transform = ADAM && XFORM;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (wave >= per) return;
  const int sid = blockIdx.x * per + wave;
  if (sid >= a.num_shapes) return;
  cptr<ShapeRec> SR = konst(a.shapes);
  cptr<LayoutRec> LS = konst(a.layouts);
  const int b = a.num_layouts == 1 ? 0 : uniform(SR[sid].layout);  // scalar: the layout's fields are scalar loads
  const float k = LS[b].k;
  const int4 bb = load_box(konst(a.bins), sid);
  const int item0 = konst(a.item_base)[sid];  // the item's first map entry (-1: its layout's units did not fit)
  const int bad = a.shapes[sid].bad;  // loaded with the others, consumed by lane 0 at the end
  AdamIn ain;
  // every lane (one request): no branch around the loads
  if constexpr (do_adam) ain = adam_load(a, sid, make_float2(0.0f, 0.0f));
  int32_t t_step = 0;
  if constexpr (do_adam) t_step = uniform(a.step[0]);
  TransformPre tp;
  if constexpr (do_transform) tp = transform_preload(a, sid, lane);
  double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);
  if (bb.x <= bb.z && bb.y <= bb.w && item0 >= 0) {
    // every tile that the support box meets lists the item: its units' head partials are the item's map
    // entries [item0, item0 + tiles of its span), one per lane, each converted to double and added in
    // a fixed order
    const int nt = (bb.z / T - bb.x / T + 1) * (bb.w / T - bb.y / T + 1);
    const ulonglong2 *H = reinterpret_cast<const ulonglong2 *>(a.head + 4 * (int64_t)item0);
    for (int j = lane; j < nt; j += 64) {
      const ulonglong2 h0 = H[2 * j], h1 = H[2 * j + 1];
      acc.x += ldexp((double)(long long)h0.x, -kHeadBits);
      acc.y += ldexp((double)(long long)h0.y, -kHeadBits);
      acc.z += ldexp((double)(long long)h1.x, -kHeadBits);
      acc.w += ldexp((double)(long long)h1.y, -kHeadBits);
    }
  }
  {
    int comp;
    const double t = wave_sum4(acc, comp);
    acc = make_double4(readlane_f64(t, 0), readlane_f64(t, 2), readlane_f64(t, 1), readlane_f64(t, 3));
  }
  float4 pn = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (lane == 0) {
    // the object-space downward force adds d(H - k t_y)/dt_y = -k per unit of its weight
    const double c_od = (double)a.w[8] * (a.dloss ? (double)a.dloss[kLossTerms * b + 8] : 1.0);
    float4 g = make_float4((float)(-(double)k * acc.x), (float)(-(double)k * (acc.y + c_od)), (float)acc.z, (float)acc.w);
    if (bad != 0) g = make_float4(NAN, NAN, NAN, NAN);
    if (a.grad_out) reinterpret_cast<float4 *>(a.grad_out)[sid] = g;
    if constexpr (do_adam) {
      const float2 bias = adam_bias_of(a, t_step);
      ain.bc1 = bias.x;
      ain.bc2 = bias.y;
      pn = adam_update(a, sid, g, k, ain);
    }
  }
  if constexpr (do_transform) {
    // the next epoch of the same call starts from the updated parameters: transform them now
    pn.x = __shfl(pn.x, 0, 64);
    pn.y = __shfl(pn.y, 0, 64);
    pn.z = __shfl(pn.z, 0, 64);
    pn.w = __shfl(pn.w, 0, 64);
    transform_hold(tp);
    transform_item(a, sid, lane, pn, tp);
  }
}

// The loss sums of layout b over its pixel tiles in one fixed order for any workgroup size (128 or 256
// threads): 256 virtual lanes, lane v summing tiles v, v + 256, ..., then each group of 64 virtual lanes
// by a wave sum, then the four groups in order.
__device__ void finalize_loss(const KArgs &a, int b) {
  __shared__ double s_part[4][kLossTerms];
  const int lane = threadIdx.x & 63;
  cptr<LayoutRec> LS = konst(a.layouts);
  const int p0 = LS[b].ptile_off;
  const int np = ((LS[b].W + kPixTile - 1) / kPixTile) * ((LS[b].H + kPixTile - 1) / kPixTile);
  for (int vb = 0; vb < 256; vb += blockDim.x) {
    const int v = vb + threadIdx.x;
    double s[kLossTerms];
#pragma unroll
    for (int t = 0; t < kLossTerms; ++t) s[t] = 0.0;
    // four tiles' loads in flight at a time, added in tile order
    int j = v;
    for (; j + 3 * 256 < np; j += 4 * 256) {
      double r[4][kLossTerms];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double *bl = a.block_loss + (int64_t)(p0 + j + i * 256) * kLossTerms;
#pragma unroll
        for (int t = 0; t < kLossTerms; ++t) r[i][t] = bl[t];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int t = 0; t < kLossTerms; ++t) s[t] += r[i][t];
    }
    for (; j < np; j += 256) {
      const double *bl = a.block_loss + (int64_t)(p0 + j) * kLossTerms;
#pragma unroll
      for (int t = 0; t < kLossTerms; ++t) s[t] += bl[t];
    }
#pragma unroll
    for (int t = 0; t < kLossTerms; ++t) {
      const double w = wave_sum(s[t]);
      if (lane == 0) s_part[v >> 6][t] = w;
    }
  }
  __syncthreads();
  if (threadIdx.x < kLossTerms) {
    const int t = threadIdx.x;
    const double v = ((s_part[0][t] + s_part[1][t]) + s_part[2][t]) + s_part[3][t];
    a.loss_out[kLossTerms * b + t] = (float)v;
  }
}

template <int T>
__global__ __launch_bounds__(256) void k_finalize(KArgs a, int grad_blocks, int flags, int per) {
  if ((int)blockIdx.x < grad_blocks) {
    if (flags & 4)
      finalize_grad<T, true, true>(a, per);
    else if (flags & 1)
      finalize_grad<T, true, false>(a, per);
    else
      finalize_grad<T, false, false>(a, per);
  } else if (flags & 2) {
    finalize_loss(a, blockIdx.x - grad_blocks);
  }
}

__global__ void k_step_inc(int32_t *step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) step[0] = step[0] + 1;
}

// Zeroes the Adam moments and the step counter (a kernel rather than a memset, so that it can sit in a
// captured graph).
__global__ __launch_bounds__(256) void k_adam_reset(float *m, float *v, int32_t *step, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    m[i] = 0.0f;
    v[i] = 0.0f;
  }
  if (i == 0) step[0] = 0;
}

__global__ __launch_bounds__(256) void k_adam(KArgs a) {
  const int sid = blockIdx.x * 256 + threadIdx.x;
  if (sid >= a.num_shapes) return;
  cptr<LayoutRec> LS = konst(a.layouts);
  const int b = layout_of_shape(LS, a.num_layouts, sid);
  const float4 g = reinterpret_cast<const float4 *>(a.grad_out)[sid];
  adam_update(a, sid, g, LS[b].k, adam_load(a, sid, adam_bias_of(a, a.step[0])));
}

// ------------------------------------------------------------------------------------------------
// k_render: per-item coverage images (tests and small scenes).
// ------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_render(KArgs a, int first, float *alpha, float *alpha_pad) {
  const int q = first + blockIdx.y;
  cptr<LayoutRec> LS = konst(a.layouts);
  cptr<ShapeRec> SR = konst(a.shapes);
  const int b = uniform(SR[q].layout);
  const int W = LS[b].W, H = LS[b].H;
  // output offset: images of items first..q-1, each of its own layout's size
  int64_t off = 0;
  for (int c = 0; c < a.num_layouts; ++c) {
    const int lo = max(LS[c].shape_begin, first), hi = min(LS[c].shape_end, q);
    if (hi > lo) off += (int64_t)(hi - lo) * LS[c].W * LS[c].H;
  }
  const int pix = blockIdx.x * 256 + threadIdx.x;
  if (pix >= W * H) return;
  const int pxi = pix % W, pyi = pix / W;
  const int4 bb = load_box(konst(a.bins), q);
  float al = 0.0f, alp = 0.0f;
  const int eo = SR[q].edge_off, ec = SR[q].edge_cnt;
  if (ec > 0 && pxi >= bb.x && pxi <= bb.z && pyi >= bb.y && pyi <= bb.w) {
    int bi;
    bool par;
    const double rx = pxi + 0.5 - SR[q].cx, ry = pyi + 0.5 - SR[q].cy;
    edge_scan(konst(a.edges) + eo, ec, (float)rx, (float)ry, bi, par);
    const Nearest nr = nearest_refined(a.edges_d + eo, ec, bi, rx, ry);
    const double d = sqrt(nr.d2);
    double ad, apd;
    coverage_pair(a, SR[q].open ? SR[q].sw - d : (par ? d : -d), ad, apd);
    al = (float)ad;
    alp = (float)apd;
  }
  alpha[off + pix] = al;
  if (alpha_pad) alpha_pad[off + pix] = alp;
}

// ------------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------------
hipError_t launch_transform(const KArgs &a, hipStream_t st) {
  const int blocks = a.num_shapes > 0 ? (a.num_shapes + 3) / 4 : 1;
  hipLaunchKernelGGL(k_transform, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Every tile-size dependent kernel is instantiated for T = 8, 16 and 32; the scene fixes T.
#define COLLAGE_TILE_DISPATCH(T_, STMT)                                                               \
  switch (a.tile) {                                                                                  \
    case 8: {                                                                                        \
      constexpr int T_ = 8;                                                                          \
      STMT;                                                                                          \
    } break;                                                                                         \
    case 32: {                                                                                       \
      constexpr int T_ = 32;                                                                         \
      STMT;                                                                                          \
    } break;                                                                                         \
    case 64: {                                                                                       \
      constexpr int T_ = 64;                                                                         \
      STMT;                                                                                          \
    } break;                                                                                         \
    case 128: {                                                                                      \
      constexpr int T_ = 128;                                                                        \
      STMT;                                                                                          \
    } break;                                                                                         \
    default: {                                                                                       \
      constexpr int T_ = 16;                                                                         \
      STMT;                                                                                          \
    } break;                                                                                         \
  }

hipError_t launch_bin(const KArgs &a, hipStream_t st) {
  if (a.total_tiles <= 0) return hipSuccess;
  if (a.rowbin) COLLAGE_TILE_DISPATCH(T, hipLaunchKernelGGL(k_rowbin<T>, dim3(a.total_rows), dim3(256), 0, st, a));
  if (a.rowbin) {
    COLLAGE_TILE_DISPATCH(T, hipLaunchKernelGGL((k_bin<T, 1>), dim3(a.total_tiles * kBinParts<T>),
                                                dim3(T * T < 256 ? T * T : 256), 0, st, a));
  } else {
    COLLAGE_TILE_DISPATCH(T, hipLaunchKernelGGL((k_bin<T, 2>), dim3(a.total_tiles * kBinParts<T>),
                                                dim3(T * T < 256 ? T * T : 256), 0, st, a));
  }
  return hipGetLastError();
}

hipError_t launch_scan(const KArgs &a, hipStream_t st) {
  if (a.scan_in_cover) return hipSuccess;  // the coverage kernel computes the prefixes itself
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_cover(const KArgs &a, hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop) {
  if (ev_start) {
    // the events are timestamped with the dispatch itself (kernel start and end)
    COLLAGE_TILE_DISPATCH(T, hipExtLaunchKernelGGL(k_cover<T>, dim3(a.cover_grid), dim3(256), 0, st, ev_start,
                                                   ev_stop, 0, a));
  } else {
    COLLAGE_TILE_DISPATCH(T, hipLaunchKernelGGL(k_cover<T>, dim3(a.cover_grid), dim3(256), 0, st, a));
  }
  return hipGetLastError();
}

hipError_t launch_pixel(const KArgs &a, bool grad, hipStream_t st) {
  if (a.total_ptiles <= 0) return hipSuccess;
  const dim3 g(a.total_ptiles), b_uni(kPixThreads), b_plain(256);
  if (a.w[5] != 0.0f) {
    if (grad)
      hipLaunchKernelGGL((k_pixel<true, true>), g, b_uni, 0, st, a);
    else
      hipLaunchKernelGGL((k_pixel<false, true>), g, b_uni, 0, st, a);
  } else {
    if (grad)
      hipLaunchKernelGGL((k_pixel<true, false>), g, b_plain, 0, st, a);
    else
      hipLaunchKernelGGL((k_pixel<false, false>), g, b_plain, 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_uniform_grad(const KArgs &a, hipStream_t st) {
  if (a.w[5] == 0.0f || a.total_ptiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unif_grad, dim3(a.total_ptiles), dim3(kPixThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_vertex_grad(const KArgs &a, hipStream_t st) {
  COLLAGE_TILE_DISPATCH(T, hipLaunchKernelGGL(k_vgrad<T>, dim3(a.adjoint_grid), dim3(256), 0, st, a));
  if (a.num_shapes > 0) hipLaunchKernelGGL(k_vfinal, dim3((a.num_shapes + 3) / 4), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_adjoint(const KArgs &a, hipStream_t st) {
  COLLAGE_TILE_DISPATCH(T, hipLaunchKernelGGL(k_adjoint<T>, dim3(a.adjoint_grid), dim3(256), 0, st, a));
  return hipGetLastError();
}

hipError_t launch_finalize(const KArgs &a, bool do_grad, bool do_loss, bool do_adam, hipStream_t st,
                           bool do_transform) {
  // each item's gradient is a short chain of dependent loads: with fewer than 2048 items, two items
  // per workgroup spread the chains over twice the compute units (the workgroups keep 256 threads for
  // the per-layout loss sums, the other waves of a gradient workgroup exit at once)
  const int per = a.num_shapes >= 2048 ? 4 : 2;
  const int gb = do_grad ? (a.num_shapes + per - 1) / per : 0;
  const int lb = do_loss ? a.num_layouts : 0;
  if (gb + lb == 0) return hipSuccess;
  const int flags = (do_adam ? 1 : 0) | (do_loss ? 2 : 0) | (do_adam && do_transform ? 4 : 0);
  COLLAGE_TILE_DISPATCH(T, hipLaunchKernelGGL(k_finalize<T>, dim3(gb + lb), dim3(256), 0, st, a, gb, flags, per));
  return hipGetLastError();
}

hipError_t launch_adam_only(const KArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, st, const_cast<int32_t *>(a.step));
  if (a.num_shapes > 0) hipLaunchKernelGGL(k_adam, dim3((a.num_shapes + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// The static scratch of the allocation-free entry point: a workspace of kStaticScratchBytes that every
// GPU the library runs on holds from the module's load until the process ends.  In host code the
// array's name stands for a host-side shadow, not the device copy: only the address that
// hipGetSymbolAddress returns, per device, may be passed to kernels or copies.
// ------------------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(void **out) {
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (addr[dev] == nullptr) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr || reinterpret_cast<uintptr_t>(p) % 256 != 0) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

hipError_t launch_adam_reset(float *m, float *v, int32_t *step, int num_shapes, hipStream_t st) {
  const int n = 4 * num_shapes;
  hipLaunchKernelGGL(k_adam_reset, dim3(n > 0 ? (n + 255) / 256 : 1), dim3(256), 0, st, m, v, step, n);
  return hipGetLastError();
}

hipError_t launch_render(const KArgs &a, int first, int count, float *alpha, float *alpha_pad, int max_pixels,
                         hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_render, dim3((max_pixels + 255) / 256, count), dim3(256), 0, st, a, first, alpha, alpha_pad);
  return hipGetLastError();
}

}  // namespace collage
