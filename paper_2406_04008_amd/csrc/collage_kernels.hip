// HIP kernels (gfx950, wave64) of the image-space collage hot path.
//
// One call is a short chain of launches with grids fixed by the scene:
//   k_transform  one wave per item: eq. 2 applied to the outline (in double precision), float edge
//                records for the scan and double edge records for the per-pixel evaluation, both
//                relative to the item's origin, the pixel box of the item's coverage support and the
//                outline orientation.  Also clears the work counters.
//   k_bin        one workgroup per screen tile: the layout's items whose support box meets the tile,
//                in item order (LDS list copied to the workspace); every (tile, item) becomes one
//                work unit with a mask of the tile's 8 x 8 quadrants the item touches.  Clears the
//                tile's coverage accumulators.
//   k_cover      persistent waves pull work units from a global counter (so heavy and light regions
//                balance across the whole chip); per unit and pixel: float32 scan of the item's edges
//                (records read through the scalar cache, shared by the wave) for the nearest edge and
//                the even-odd parity, then the signed distance to that edge and the coverage in double
//                precision, added to the pixel's S and S_pad as 2^-40 fixed point with 64-bit integer
//                atomics (exact, so the result does not depend on the order of the units).  Adjoint
//                calls keep a 2-byte nearest-edge code per (unit, pixel).
//   k_pixel      one thread per pixel: S, S_pad, the five loss terms (summed per tile in a fixed order)
//                and dLoss/dS, dLoss/dS_pad.
//   k_adjoint    persistent waves again: per unit, the gradient terms of its pixels (double) reduced to
//                one partial per (tile, item).
//   k_finalize   one wave per item sums its tiles' partials in a fixed order (gradient, then the
//                optional Adam update); one workgroup per layout sums its tiles' loss partials.
// Results are deterministic.
#include "collage_internal.h"

#include <math.h>

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

__device__ __forceinline__ int4 load_box(cptr<int4> p, int i) {
  cptr<int> q = (cptr<int>)(p + i);
  return make_int4(q[0], q[1], q[2], q[3]);
}

__device__ __forceinline__ int2 load_pair(cptr<int2> p, int64_t i) {
  cptr<int> q = (cptr<int>)(p + i);
  return make_int2(q[0], q[1]);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Logistic function and its derivative, a = 1 / (1 + e^-x) and da/dx = a (1 - a), both from
// t = e^-|x| so that neither loses precision when a is close to 0 or 1.
__device__ __forceinline__ void sigmoid_d(double x, double &a, double &da) {
  const double t = exp(-fabs(x));
  const double r = 1.0 / (1.0 + t);
  a = x >= 0.0 ? r : t * r;
  da = t * r * r;
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
__device__ __forceinline__ void place_vertex(double c, double sn, double s, double k, float2 v, double &x, double &y) {
  const double sx = s * (double)v.x, sy = s * (double)v.y;
  x = k * (c * sx - sn * sy);
  y = k * (sn * sx + c * sy);
}

__global__ __launch_bounds__(256) void k_transform(KArgs a) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (blockIdx.x == 0 && threadIdx.x < CNT_WORDS) a.counters[threadIdx.x] = 0;
  if (a.step_inc != nullptr && blockIdx.x == 0 && threadIdx.x == 0) a.step_inc[0] = a.step_inc[0] + 1;
  const int sid = blockIdx.x * 4 + wave;
  if (sid >= a.num_shapes) return;
  cptr<LayoutRec> LS = konst(a.layouts);
  const int b = layout_of_shape(LS, a.num_layouts, sid);
  const double k = (double)LS[b].k;
  const int W = LS[b].W, H = LS[b].H;
  const float4 p = reinterpret_cast<const float4 *>(a.params)[sid];
  const int v0 = a.vert_off[sid];
  const int n = a.vert_off[sid + 1] - v0;
  const bool finite = isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(p.w);
  double sn, c;
  sincos(finite ? (double)p.z : 0.0, &sn, &c);
  const double s = finite ? (double)p.w : 1.0;
  const double cx = k * (double)p.x, cy = k * (double)p.y;
  const float2 *V = reinterpret_cast<const float2 *>(a.verts) + v0;
  double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY, area2 = 0.0;
  for (int m = lane; m < n; m += 64) {
    double ax, ay, bx, by;
    place_vertex(c, sn, s, k, V[m], ax, ay);
    place_vertex(c, sn, s, k, V[m + 1 == n ? 0 : m + 1], bx, by);
    const double ex = bx - ax, ey = by - ay;
    const double ee = ex * ex + ey * ey;
    const double inv = ee > 0.0 ? 1.0 / ee : 0.0;
    EdgeRec r;
    r.ax = (float)ax;
    r.ay = (float)ay;
    r.exs = (float)(ex * inv);
    r.eys = (float)(ey * inv);
    r.ex = (float)ex;
    r.ey = (float)ey;
    r.by = (float)by;  // equals the next edge's ay: the same double rounded the same way
    r.slope = ey != 0.0 ? (float)(ex / ey) : 0.0f;
    a.edges[v0 + m] = r;
    EdgeD rd;
    rd.ax = ax;
    rd.ay = ay;
    rd.ex = ex;
    rd.ey = ey;
    rd.inv_ee = inv;
    // d v' / d s = k R(theta) v for both end points (exact also when s = 0)
    {
      const float2 va = V[m], vb = V[m + 1 == n ? 0 : m + 1];
      rd.kra_x = k * (c * (double)va.x - sn * (double)va.y);
      rd.kra_y = k * (sn * (double)va.x + c * (double)va.y);
      rd.kre_x = k * (c * (double)vb.x - sn * (double)vb.y) - rd.kra_x;
      rd.kre_y = k * (sn * (double)vb.x + c * (double)vb.y) - rd.kra_y;
    }
    a.edges_d[v0 + m] = rd;
    mnx = fmin(mnx, ax);
    mxx = fmax(mxx, ax);
    mny = fmin(mny, ay);
    mxy = fmax(mxy, ay);
    area2 += ax * by - bx * ay;
  }
  mnx = wave_min(mnx);
  mny = wave_min(mny);
  mxx = wave_max(mxx);
  mxy = wave_max(mxy);
  area2 = wave_sum(area2);
  if (lane == 0) {
    const double ext = (double)a.r_cut + fmax((double)a.r_pad, 0.0);
    int4 box = make_int4(1, 1, 0, 0);  // empty
    if (n > 0 && finite) {
      // pixel centres i + 1/2 in [cx + mnx - ext, cx + mxx + ext], widened by one pixel
      double fx0 = floor(cx + mnx - ext - 0.5) - 1.0, fx1 = ceil(cx + mxx + ext - 0.5) + 1.0;
      double fy0 = floor(cy + mny - ext - 0.5) - 1.0, fy1 = ceil(cy + mxy + ext - 0.5) + 1.0;
      fx0 = fmax(fx0, 0.0);
      fy0 = fmax(fy0, 0.0);
      fx1 = fmin(fx1, (double)(W - 1));
      fy1 = fmin(fy1, (double)(H - 1));
      if (fx0 <= fx1 && fy0 <= fy1) box = make_int4((int)fx0, (int)fy0, (int)fx1, (int)fy1);
    }
    a.bbox[sid] = box;
    ShapeRec sr;
    sr.cx = cx;
    sr.cy = cy;
    sr.cxf = (float)cx;
    sr.cyf = (float)cy;
    sr.k = (float)k;
    sr.s = p.w;
    sr.orient = area2 >= 0.0 ? 1.0f : -1.0f;
    sr.edge_off = v0;
    sr.edge_cnt = n;
    sr.layout = b;
    sr.bad = finite ? 0 : 1;
    sr.pad = 0;
    a.shapes[sid] = sr;
  }
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
};

__device__ __forceinline__ void pair_d2(const EdgeD &e, double rx, double ry, double &d2, double &u, double &qx,
                                        double &qy) {
  const double wx = rx - e.ax, wy = ry - e.ay;
  u = fmin(fmax((wx * e.ex + wy * e.ey) * e.inv_ee, 0.0), 1.0);
  qx = wx - u * e.ex;
  qy = wy - u * e.ey;
  d2 = qx * qx + qy * qy;
}

__device__ __forceinline__ PairD pair_eval(const EdgeD &e, double rx, double ry, bool par) {
  PairD r;
  double d2;
  pair_d2(e, rx, ry, d2, r.u, r.qx, r.qy);
  r.d = sqrt(d2);
  r.sd = par ? r.d : -r.d;
  return r;
}

// The float scan can order two edges wrongly only when their squared distances agree to float
// precision.  Away from the (measure-zero) medial axes that happens only between neighbouring edges
// (near the boundary between a vertex's fan and an edge's perpendicular strip), where the choice does
// not change the distance much but does tilt the gradient direction.  So the nearest edge is decided
// again in double among the scan's choice and its two neighbours (lowest index on exact ties).
__device__ __forceinline__ int nearest_refined(const EdgeD *E, int ec, int bi, double rx, double ry) {
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
  double d2, u, qx, qy;
  pair_d2(E[c0], rx, ry, d2, u, qx, qy);
  int best = c0;
  double bd = d2;
  if (c1 != c0) {
    pair_d2(E[c1], rx, ry, d2, u, qx, qy);
    if (d2 < bd) {
      bd = d2;
      best = c1;
    }
  }
  if (c2 != c1) {
    pair_d2(E[c2], rx, ry, d2, u, qx, qy);
    if (d2 < bd) best = c2;
  }
  return best;
}

// Coverage of one item at one pixel from its signed distance: alpha, alpha_pad (0 past the cut-off).
__device__ __forceinline__ void coverage(const KArgs &a, double sd, double &al, double &dal, double &alp,
                                         double &dalp) {
  const double inv_tau = 1.0 / (double)a.tau;
  al = dal = alp = dalp = 0.0;
  if (sd >= -(double)a.r_cut) sigmoid_d(sd * inv_tau, al, dal);
  if (sd + (double)a.r_pad >= -(double)a.r_cut) sigmoid_d((sd + (double)a.r_pad) * inv_tau, alp, dalp);
  dal *= inv_tau;
  dalp *= inv_tau;
}

// Adjoint terms of one (pixel, item): omega * d sd / d(t, theta, s), up to the factor -k of the
// translation terms applied by the finalize kernel.  omega = G dalpha/dsd + G_pad dalpha_pad/dsd.
__device__ __forceinline__ double4 adjoint_terms(const KArgs &a, const EdgeD &e, const PairD &q, double rx, double ry,
                                                 bool par, float orient, double G, double Gp) {
  double al, dal, alp, dalp;
  coverage(a, q.sd, al, dal, alp, dalp);
  const double om = G * dal + Gp * dalp;
  double4 t = make_double4(0.0, 0.0, 0.0, 0.0);
  if (om == 0.0 || q.d == 0.0) return t;
  double nx, ny;
  if (q.u > 0.0 && q.u < 1.0) {
    // nearest point inside the edge: grad sd is the unit edge normal, oriented (inside ? +1 : -1)
    // times the side of the edge the pixel is on; within 1e-4 px of the edge the float parity is
    // not reliable, but the product of the two is the outline orientation
    const double il = sqrt(e.inv_ee);
    double sg = (double)orient;
    if (q.d >= 1e-4) {
      const double side = q.qy * e.ex - q.qx * e.ey;
      sg = (par == (side > 0.0)) ? 1.0 : -1.0;
    }
    nx = -e.ey * il * sg;
    ny = e.ex * il * sg;
  } else {
    const double id = (par ? 1.0 : -1.0) / q.d;
    nx = q.qx * id;
    ny = q.qy * id;
  }
  t.x = om * nx;
  t.y = om * ny;
  t.z = om * (nx * ry - ny * rx);
  // d sd / d s = -n . (k R (v_a + u (v_b - v_a))): the nearest point of the unscaled outline
  t.w = -om * (nx * (e.kra_x + q.u * e.kre_x) + ny * (e.kra_y + q.u * e.kre_y));
  return t;
}

// Bins items [cb, ce) of a layout whose support box meets the tile rectangle, in item order.
template <int NT>
__device__ int bin_chunk(const KArgs &a, int cb, int ce, int x0, int y0, int x1, int y1, int *s_list, int *s_wcnt,
                         int32_t *glist) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  int count = 0;
  for (int base = cb; base < ce; base += NT) {
    const int sid = base + tid;
    bool hit = false;
    if (sid < ce) {
      const int4 bb = a.bbox[sid];
      hit = !(bb.x > x1 || bb.z < x0 || bb.y > y1 || bb.w < y0);
    }
    const unsigned long long m = __ballot(hit);
    const int before = __popcll(m & ((1ull << l) - 1ull));
    if (l == 0) s_wcnt[w] = __popcll(m);
    __syncthreads();
    int off = count, tot = count;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const int cj = s_wcnt[j];
      if (j < w) off += cj;
      tot += cj;
    }
    if (hit) {
      s_list[off + before] = sid;
      if (glist) glist[off + before] = sid;
    }
    count = tot;
    __syncthreads();
  }
  return count;
}

// Work units are the (tile, item) pairs of the per-tile lists, in tile order and slot order.  Each
// has a cost (coverage: quadrants x (edges + 16); adjoint: 64 x quadrants).  The persistent wave w of
// W waves processes the units whose cost interval [p, p + c) ends in (B_w, B_{w+1}], where
// B_w = ceil(w * total / W) and p is the unit's cost prefix: it finds the tile holding B_w by binary
// search over the tile prefix sums and walks from there.  Every wave gets the same amount of work to
// within one unit, and no counter is shared between waves.
struct Walk {
  int tile, slot, count;   // current unit = slot `slot` of tile `tile` (which has `count` units)
  int layout, W, H, x0, y0;
  int64_t pix_off, list_base;
  long long p, end;        // cost prefix of the current unit; the wave stops at units ending past `end`
  bool adj;
};

__device__ __forceinline__ void walk_tile(const KArgs &a, Walk &w, int T) {
  cptr<LayoutRec> LS = konst(a.layouts);
  w.layout = layout_of_tile(LS, a.num_layouts, w.tile);
  w.W = LS[w.layout].W;
  w.H = LS[w.layout].H;
  const int ntx = LS[w.layout].ntx;
  const int nb = LS[w.layout].shape_end - LS[w.layout].shape_begin;
  const int lt = w.tile - LS[w.layout].tile_off;
  const int tyi = lt / ntx;
  w.x0 = (lt - tyi * ntx) * T;
  w.y0 = tyi * T;
  w.pix_off = LS[w.layout].pix_off;
  w.list_base = LS[w.layout].list_off + (int64_t)lt * nb;
  w.count = konst(a.tile_count)[w.tile];
}

__device__ __forceinline__ long long unit_cost(const Walk &w, int2 aux) {
  return w.adj ? 64ll * __popc(aux.x) : (long long)aux.y;
}

// Moves to the next unit that exists (skipping empty tiles); returns false past the last tile.
__device__ __forceinline__ bool walk_settle(const KArgs &a, Walk &w, int T) {
  while (w.slot >= w.count) {
    if (++w.tile >= a.total_tiles) return false;
    w.slot = 0;
    walk_tile(a, w, T);
  }
  return true;
}

// First unit of persistent wave gw: returns false when the wave has no work.
__device__ __forceinline__ bool walk_begin(const KArgs &a, Walk &w, int gw, int nwaves, bool adj, int T) {
  const long long *pre = a.tile_pre + (adj ? a.total_tiles + 1 : 0);
  cptr<long long> P = konst(pre);
  const long long tot = P[a.total_tiles];
  w.adj = adj;
  if (tot <= 0) return false;
  const long long b0 = ((long long)gw * tot + nwaves - 1) / nwaves;
  w.end = ((long long)(gw + 1) * tot + nwaves - 1) / nwaves;
  if (b0 >= tot) return false;
  int lo = 0, hi = a.total_tiles - 1;  // last tile with pre <= b0
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (P[mid] <= b0)
      lo = mid;
    else
      hi = mid - 1;
  }
  w.tile = lo;
  w.slot = 0;
  w.p = P[lo];
  walk_tile(a, w, T);
  // skip the units that end at or before b0 (they belong to earlier waves)
  for (;;) {
    if (!walk_settle(a, w, T)) return false;
    const long long c = unit_cost(w, load_pair(konst(a.entry_aux), w.list_base + w.slot));
    if (w.p + c > b0) break;
    w.p += c;
    ++w.slot;
  }
  // wave 0 also takes any zero-cost units in front of its first unit (there are none: every unit
  // covers at least one quadrant); the current unit is this wave's iff it ends by w.end
  return w.p + unit_cost(w, load_pair(konst(a.entry_aux), w.list_base + w.slot)) <= w.end;
}

// Advances to the next unit of the wave; returns false when the wave is done.
__device__ __forceinline__ bool walk_next(const KArgs &a, Walk &w, int T) {
  w.p += unit_cost(w, load_pair(konst(a.entry_aux), w.list_base + w.slot));
  ++w.slot;
  if (!walk_settle(a, w, T)) return false;
  return w.p + unit_cost(w, load_pair(konst(a.entry_aux), w.list_base + w.slot)) <= w.end;
}

// The unit the walk is on.
struct Unit {
  int slot, mask, item, W, H, x0, y0, u;
  int64_t pix_off, entry;
};

__device__ __forceinline__ Unit walk_unit(const KArgs &a, const Walk &w) {
  Unit r;
  r.slot = w.slot;
  r.entry = w.list_base + w.slot;
  r.mask = load_pair(konst(a.entry_aux), r.entry).x;
  r.item = konst(a.tile_list)[r.entry];
  r.W = w.W;
  r.H = w.H;
  r.x0 = w.x0;
  r.y0 = w.y0;
  r.pix_off = w.pix_off;
  return r;
}

// The wave index is wave-uniform; readfirstlane tells the compiler so, which keeps the work walk in SGPRs
// and its loads on the scalar cache.
__device__ __forceinline__ int global_wave() { return uniform((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6))); }

// ------------------------------------------------------------------------------------------------
// k_bin: per tile, the ordered item list and one work unit per (tile, item).
// ------------------------------------------------------------------------------------------------
template <int T>
__global__ __launch_bounds__(T *T) void k_bin(KArgs a) {
  constexpr int NT = T * T, NW = NT / 64, QPR = T / 8, Q = QPR * QPR;
  __shared__ int s_list[kMaxBinChunk];
  __shared__ int s_wcnt[NW];
  const int tile = blockIdx.x, tid = threadIdx.x;
  cptr<LayoutRec> LS = konst(a.layouts);
  const int b = layout_of_tile(LS, a.num_layouts, tile);
  const int W = LS[b].W, H = LS[b].H, ntx = LS[b].ntx;
  const int sb = LS[b].shape_begin, se = LS[b].shape_end, nb = se - sb;
  const int lt = tile - LS[b].tile_off, tyi = lt / ntx, txi = lt - tyi * ntx;
  const int x0 = txi * T, y0 = tyi * T;
  const int64_t list_base = LS[b].list_off + (int64_t)lt * nb;
  {
    const int pxi = x0 + tid % T, pyi = y0 + tid / T;
    if (pxi < W && pyi < H) {
      const int64_t pix = LS[b].pix_off + (int64_t)pyi * W + pxi;
      a.acc[2 * pix] = 0ull;
      a.acc[2 * pix + 1] = 0ull;
    }
  }
  int slots = 0;
  long long my_cost = 0, my_quads = 0;
  for (int cb = sb; cb < se; cb += a.bin_chunk) {
    const int ce = min(cb + a.bin_chunk, se);
    const int cnt = bin_chunk<NT>(a, cb, ce, x0, y0, x0 + T - 1, y0 + T - 1, s_list, s_wcnt, a.tile_list + list_base + slots);
    for (int q = tid; q < cnt; q += NT) {
      const int4 bb = a.bbox[s_list[q]];
      int mask = 0;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const int qx0 = x0 + 8 * (k % QPR), qy0 = y0 + 8 * (k / QPR);
        if (!(bb.x > qx0 + 7 || bb.z < qx0 || bb.y > qy0 + 7 || bb.w < qy0)) mask |= 1 << k;
      }
      const int nq = __popc(mask);
      const int cost = nq * (a.shapes[s_list[q]].edge_cnt + 16);
      a.entry_aux[list_base + slots + q] = make_int2(mask, cost);
      my_cost += cost;
      my_quads += nq;
    }
    slots += cnt;
    __syncthreads();
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
    a.tile_count[tile] = slots;
    a.tile_cost[tile] = make_int2((int)c, (int)(64 * q));
  }
}

// ------------------------------------------------------------------------------------------------
// k_scan: one workgroup.  Unit numbering (prefix of the tile counts), prefix sums of the unit costs
// and the first unit of every persistent wave.  Every thread owns a contiguous segment: one pass to
// sum it, one block scan of the 1024 sums, one pass to write.
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

__global__ __launch_bounds__(1024) void k_scan(KArgs a) {
  __shared__ long long s_w[16];
  const int tid = threadIdx.x;
  const int nt = a.total_tiles;
  const int per = (nt + 1023) / 1024, t0 = min(tid * per, nt), t1 = min(t0 + per, nt);
  long long cnt = 0, cc = 0, ca = 0;
  for (int t = t0; t < t1; ++t) {
    cnt += a.tile_count[t];
    const int2 c = a.tile_cost[t];
    cc += c.x;
    ca += c.y;
  }
  long long nunits, tot_c, tot_a;
  long long u = block_exclusive_scan(cnt, s_w, nunits);
  long long pc = block_exclusive_scan(cc, s_w, tot_c);
  long long pa = block_exclusive_scan(ca, s_w, tot_a);
  long long *prc = a.tile_pre, *pra = a.tile_pre + (nt + 1);
  for (int t = t0; t < t1; ++t) {
    a.tile_unit[t] = (int)u;
    prc[t] = pc;
    pra[t] = pa;
    const int2 c = a.tile_cost[t];
    u += a.tile_count[t];
    pc += c.x;
    pa += c.y;
  }
  if (tid == 0) {
    a.tile_unit[nt] = (int)nunits;
    prc[nt] = tot_c;
    pra[nt] = tot_a;
  }
}

// ------------------------------------------------------------------------------------------------
// k_cover: coverage of every (unit, pixel) into the fixed-point accumulators.
// ------------------------------------------------------------------------------------------------
template <int T>
__global__ __launch_bounds__(256) void k_cover(KArgs a) {
  constexpr int QPR = T / 8, Q = QPR * QPR;
  const int lane = threadIdx.x & 63;
  cptr<ShapeRec> SR = konst(a.shapes);
  cptr<EdgeRec> ED = konst(a.edges);
  const int gw = global_wave();
  const int nwaves = gridDim.x * (blockDim.x >> 6);
  Walk wk;
  for (bool ok = walk_begin(a, wk, gw, nwaves, false, T); ok; ok = walk_next(a, wk, T)) {
    const Unit un = walk_unit(a, wk);
    const int u = uniform(konst(a.tile_unit)[wk.tile]) + wk.slot;
    const int eo = SR[un.item].edge_off, ec = SR[un.item].edge_cnt;
    const float cxf = SR[un.item].cxf, cyf = SR[un.item].cyf;
    const double cx = SR[un.item].cx, cy = SR[un.item].cy;
    const bool keep = a.keep_codes && u < a.code_cap;
    for (int k = 0; k < Q; ++k) {
      if (!((un.mask >> k) & 1)) continue;
      const int pxi = un.x0 + 8 * (k % QPR) + (lane & 7), pyi = un.y0 + 8 * (k / QPR) + (lane >> 3);
      int bi = 0;
      bool par = false;
      edge_scan(ED + eo, ec, pxi + 0.5f - cxf, pyi + 0.5f - cyf, bi, par);
      if (ec > 0) {
        const double rx = pxi + 0.5 - cx, ry = pyi + 0.5 - cy;
        bi = nearest_refined(a.edges_d + eo, ec, bi, rx, ry);
        if (pxi < un.W && pyi < un.H) {
          const PairD pr = pair_eval(a.edges_d[eo + bi], rx, ry, par);
          double al, dal, alp, dalp;
          coverage(a, pr.sd, al, dal, alp, dalp);
          const int64_t pix = un.pix_off + (int64_t)pyi * un.W + pxi;
          if (al > 0.0) atomicAdd(&a.acc[2 * pix], (unsigned long long)llrint(al * kFixScale));
          if (alp > 0.0) atomicAdd(&a.acc[2 * pix + 1], (unsigned long long)llrint(alp * kFixScale));
        }
      }
      if (keep) a.codes[((int64_t)u * Q + k) * 64 + lane] = (uint16_t)(bi | (par ? 0x8000 : 0));
    }
  }
}

// ------------------------------------------------------------------------------------------------
// k_pixel: S, S_pad, loss terms (per tile) and dLoss/dS, dLoss/dS_pad per pixel.
// ------------------------------------------------------------------------------------------------
template <int T, bool GRAD>
__global__ __launch_bounds__(T *T) void k_pixel(KArgs a) {
  constexpr int NT = T * T, NW = NT / 64;
  __shared__ double s_loss[NW][5];
  const int tile = blockIdx.x, tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  cptr<LayoutRec> LS = konst(a.layouts);
  const int b = layout_of_tile(LS, a.num_layouts, tile);
  const int W = LS[b].W, H = LS[b].H, ntx = LS[b].ntx;
  const int lt = tile - LS[b].tile_off, tyi = lt / ntx, txi = lt - tyi * ntx;
  const int pxi = txi * T + tid % T, pyi = tyi * T + tid / T;
  const bool valid = pxi < W && pyi < H;
  const int64_t pix = LS[b].pix_off + (int64_t)pyi * W + pxi;
  double S = 0.0, Sp = 0.0, M = 0.0;
  if (valid) {
    S = (double)a.acc[2 * pix] * kFixInv;
    Sp = (double)a.acc[2 * pix + 1] * kFixInv;
    M = (double)a.mask[pix];
    if (a.cov_out) a.cov_out[pix] = (float)S;
    if (a.cov_pad_out) a.cov_pad_out[pix] = (float)Sp;
  }
  const double yinv = (double)H - (pyi + 0.5);
  const double ov = fmax(S - 1.0, 0.0), un = fmax(1.0 - S, 0.0), pv = fmax(Sp - 1.0, 0.0);
  if (a.write_loss) {
    double term[5];
    term[0] = valid ? (double)a.w[0] * (ov * ov) : 0.0;
    term[1] = valid ? (double)a.w[1] * (S * (1.0 - M)) : 0.0;
    term[2] = valid ? (double)a.w[2] * (M * (un * un)) : 0.0;
    term[3] = valid ? (double)a.w[3] * (pv * pv) : 0.0;
    term[4] = valid ? (double)a.w[4] * (S * yinv) : 0.0;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      const double v = wave_sum(term[t]);
      if (l == 0) s_loss[w][t] = v;
    }
    __syncthreads();
    if (tid < 5) {
      double v = s_loss[0][tid];
      for (int j = 1; j < NW; ++j) v += s_loss[j][tid];
      a.tile_loss[(int64_t)tile * 5 + tid] = v;
    }
  }
  if (GRAD && valid) {
    double c_ov = a.w[0], c_c = a.w[1], c_f = a.w[2], c_p = a.w[3], c_d = a.w[4];
    if (a.dloss) {
      c_ov *= (double)a.dloss[5 * b + 0];
      c_c *= (double)a.dloss[5 * b + 1];
      c_f *= (double)a.dloss[5 * b + 2];
      c_p *= (double)a.dloss[5 * b + 3];
      c_d *= (double)a.dloss[5 * b + 4];
    }
    const double G = 2.0 * c_ov * ov + c_c * (1.0 - M) - 2.0 * c_f * (M * un) + c_d * yinv;
    const double Gp = 2.0 * c_p * pv;
    a.gbuf[pix] = make_double2(G, Gp);
  }
}

// ------------------------------------------------------------------------------------------------
// k_adjoint: per unit, the gradient terms of its pixels reduced to one partial per (tile, item).
// ------------------------------------------------------------------------------------------------
template <int T>
__global__ __launch_bounds__(256) void k_adjoint(KArgs a) {
  constexpr int QPR = T / 8, Q = QPR * QPR;
  const int lane = threadIdx.x & 63;
  cptr<ShapeRec> SR = konst(a.shapes);
  cptr<EdgeRec> ED = konst(a.edges);
  const int gw = global_wave();
  const int nwaves = gridDim.x * (blockDim.x >> 6);
  Walk wk;
  for (bool ok = walk_begin(a, wk, gw, nwaves, true, T); ok; ok = walk_next(a, wk, T)) {
    const Unit un = walk_unit(a, wk);
    const int u = uniform(konst(a.tile_unit)[wk.tile]) + wk.slot;
    const int eo = SR[un.item].edge_off, ec = SR[un.item].edge_cnt;
    const float cxf = SR[un.item].cxf, cyf = SR[un.item].cyf, orient = SR[un.item].orient;
    const double cx = SR[un.item].cx, cy = SR[un.item].cy;
    const bool cached = u < a.code_cap;
    double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);
    for (int k = 0; k < Q; ++k) {
      if (!((un.mask >> k) & 1)) continue;
      const int pxi = un.x0 + 8 * (k % QPR) + (lane & 7), pyi = un.y0 + 8 * (k / QPR) + (lane >> 3);
      const double rx = pxi + 0.5 - cx, ry = pyi + 0.5 - cy;
      int bi;
      bool par;
      if (cached) {
        const unsigned code = a.codes[((int64_t)u * Q + k) * 64 + lane];
        bi = (int)(code & 0x7fffu);
        par = (code & 0x8000u) != 0u;
      } else {
        edge_scan(ED + eo, ec, pxi + 0.5f - cxf, pyi + 0.5f - cyf, bi, par);
        if (ec > 0) bi = nearest_refined(a.edges_d + eo, ec, bi, rx, ry);
      }
      if (ec > 0 && pxi < un.W && pyi < un.H) {
        const int64_t pix = un.pix_off + (int64_t)pyi * un.W + pxi;
        const double2 g = a.gbuf[pix];
        const EdgeD e = a.edges_d[eo + bi];
        const PairD pr = pair_eval(e, rx, ry, par);
        const double4 t = adjoint_terms(a, e, pr, rx, ry, par, orient, g.x, g.y);
        acc.x += t.x;
        acc.y += t.y;
        acc.z += t.z;
        acc.w += t.w;
      }
    }
    acc.x = wave_sum(acc.x);
    acc.y = wave_sum(acc.y);
    acc.z = wave_sum(acc.z);
    acc.w = wave_sum(acc.w);
    if (lane == 0) a.partial[un.entry] = acc;
  }
}

// ------------------------------------------------------------------------------------------------
// k_finalize: per-item gradient (fixed tile order) + optional Adam; per-layout loss.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ void adam_update(const KArgs &a, int sid, float4 g, float k) {
  const float t = (float)a.step[0];
  const float bc1 = 1.0f - powf(a.beta1, t), bc2 = 1.0f - powf(a.beta2, t);
  const float rho = a.rho ? a.rho[sid] : 0.0f;
  const float lr_t = a.lr_px / k;
  const float lr_r = rho > 0.0f ? a.lr_px / (k * rho) : 0.0f;
  const float gg[4] = {g.x, g.y, g.z, g.w};
  const float lr[4] = {lr_t, lr_t, lr_r, lr_r};
  float4 *P = reinterpret_cast<float4 *>(a.param_io);
  float4 *Mv = reinterpret_cast<float4 *>(a.adam_m);
  float4 *Vv = reinterpret_cast<float4 *>(a.adam_v);
  const float4 p4 = P[sid], m4 = Mv[sid], v4 = Vv[sid];
  float pp[4] = {p4.x, p4.y, p4.z, p4.w}, mm[4] = {m4.x, m4.y, m4.z, m4.w}, vv[4] = {v4.x, v4.y, v4.z, v4.w};
  const float sqbc2 = sqrtf(bc2);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    mm[j] = a.beta1 * mm[j] + (1.0f - a.beta1) * gg[j];
    vv[j] = a.beta2 * vv[j] + (1.0f - a.beta2) * gg[j] * gg[j];
    const float denom = sqrtf(vv[j]) / sqbc2 + a.eps;
    pp[j] = pp[j] - (lr[j] / bc1) * mm[j] / denom;
  }
  P[sid] = make_float4(pp[0], pp[1], pp[2], pp[3]);
  Mv[sid] = make_float4(mm[0], mm[1], mm[2], mm[3]);
  Vv[sid] = make_float4(vv[0], vv[1], vv[2], vv[3]);
}

template <int T>
__device__ void finalize_grad(const KArgs &a, bool do_adam) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sid = blockIdx.x * 4 + wave;
  if (sid >= a.num_shapes) return;
  cptr<ShapeRec> SR = konst(a.shapes);
  cptr<LayoutRec> LS = konst(a.layouts);
  const int b = SR[sid].layout;
  const float k = SR[sid].k;
  const int4 bb = load_box(konst(a.bbox), sid);
  const int ntx = LS[b].ntx, nb = LS[b].shape_end - LS[b].shape_begin;
  const int tile_off = LS[b].tile_off;
  const int64_t list_off = LS[b].list_off;
  double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);
  if (bb.x <= bb.z && bb.y <= bb.w) {
    const int tx0 = bb.x / T, tx1 = bb.z / T, ty0 = bb.y / T, ty1 = bb.w / T;
    const int tw = tx1 - tx0 + 1, nt = tw * (ty1 - ty0 + 1);
    for (int j = lane; j < nt; j += 64) {
      const int ty = ty0 + j / tw, tx = tx0 + j % tw;
      const int lt = ty * ntx + tx;
      const int cnt = a.tile_count[tile_off + lt];
      const int32_t *list = a.tile_list + list_off + (int64_t)lt * nb;
      int lo = 0, hi = cnt - 1, slot = -1;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = list[mid];
        if (v == sid) {
          slot = mid;
          break;
        }
        if (v < sid)
          lo = mid + 1;
        else
          hi = mid - 1;
      }
      if (slot >= 0) {
        const double4 v = a.partial[list_off + (int64_t)lt * nb + slot];
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
        acc.w += v.w;
      }
    }
  }
  acc.x = wave_sum(acc.x);
  acc.y = wave_sum(acc.y);
  acc.z = wave_sum(acc.z);
  acc.w = wave_sum(acc.w);
  if (lane == 0) {
    float4 g = make_float4((float)(-(double)k * acc.x), (float)(-(double)k * acc.y), (float)acc.z, (float)acc.w);
    if (SR[sid].bad != 0) g = make_float4(NAN, NAN, NAN, NAN);
    if (a.grad_out) reinterpret_cast<float4 *>(a.grad_out)[sid] = g;
    if (do_adam) adam_update(a, sid, g, k);
  }
}

__device__ void finalize_loss(const KArgs &a, int b) {
  __shared__ double s_part[4][5];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  cptr<LayoutRec> LS = konst(a.layouts);
  const int t0 = LS[b].tile_off, nt = LS[b].ntx * LS[b].nty;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < nt; j += 256) {
    const double *tl = a.tile_loss + (int64_t)(t0 + j) * 5;
#pragma unroll
    for (int t = 0; t < 5; ++t) s[t] += tl[t];
  }
#pragma unroll
  for (int t = 0; t < 5; ++t) {
    const double v = wave_sum(s[t]);
    if (lane == 0) s_part[wave][t] = v;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    const int t = threadIdx.x;
    const double v = ((s_part[0][t] + s_part[1][t]) + s_part[2][t]) + s_part[3][t];
    a.loss_out[5 * b + t] = (float)v;
  }
}

template <int T>
__global__ __launch_bounds__(256) void k_finalize(KArgs a, int grad_blocks, int do_adam, int do_loss) {
  if ((int)blockIdx.x < grad_blocks) {
    finalize_grad<T>(a, do_adam != 0);
  } else if (do_loss) {
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
  adam_update(a, sid, g, LS[b].k);
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
  const int4 bb = load_box(konst(a.bbox), q);
  double al = 0.0, alp = 0.0;
  const int eo = SR[q].edge_off, ec = SR[q].edge_cnt;
  if (ec > 0 && pxi >= bb.x && pxi <= bb.z && pyi >= bb.y && pyi <= bb.w) {
    int bi;
    bool par;
    edge_scan(konst(a.edges) + eo, ec, pxi + 0.5f - SR[q].cxf, pyi + 0.5f - SR[q].cyf, bi, par);
    const double rx = pxi + 0.5 - SR[q].cx, ry = pyi + 0.5 - SR[q].cy;
    bi = nearest_refined(a.edges_d + eo, ec, bi, rx, ry);
    const PairD pr = pair_eval(a.edges_d[eo + bi], rx, ry, par);
    double dal, dalp;
    coverage(a, pr.sd, al, dal, alp, dalp);
  }
  alpha[off + pix] = (float)al;
  if (alpha_pad) alpha_pad[off + pix] = (float)alp;
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
    default: {                                                                                       \
      constexpr int T_ = 16;                                                                         \
      STMT;                                                                                          \
    } break;                                                                                         \
  }

hipError_t launch_bin(const KArgs &a, hipStream_t st) {
  if (a.total_tiles <= 0) return hipSuccess;
  COLLAGE_TILE_DISPATCH(T, hipLaunchKernelGGL(k_bin<T>, dim3(a.total_tiles), dim3(T * T), 0, st, a));
  return hipGetLastError();
}

hipError_t launch_scan(const KArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_cover(const KArgs &a, hipStream_t st) {
  COLLAGE_TILE_DISPATCH(T, hipLaunchKernelGGL(k_cover<T>, dim3(a.persist_grid), dim3(256), 0, st, a));
  return hipGetLastError();
}

hipError_t launch_pixel(const KArgs &a, bool grad, hipStream_t st) {
  if (a.total_tiles <= 0) return hipSuccess;
  const dim3 g(a.total_tiles);
  if (grad) {
    COLLAGE_TILE_DISPATCH(T, hipLaunchKernelGGL((k_pixel<T, true>), g, dim3(T * T), 0, st, a));
  } else {
    COLLAGE_TILE_DISPATCH(T, hipLaunchKernelGGL((k_pixel<T, false>), g, dim3(T * T), 0, st, a));
  }
  return hipGetLastError();
}

hipError_t launch_adjoint(const KArgs &a, hipStream_t st) {
  COLLAGE_TILE_DISPATCH(T, hipLaunchKernelGGL(k_adjoint<T>, dim3(a.persist_grid), dim3(256), 0, st, a));
  return hipGetLastError();
}

hipError_t launch_finalize(const KArgs &a, bool do_grad, bool do_loss, bool do_adam, hipStream_t st) {
  const int gb = do_grad ? (a.num_shapes + 3) / 4 : 0;
  const int lb = do_loss ? a.num_layouts : 0;
  if (gb + lb == 0) return hipSuccess;
  COLLAGE_TILE_DISPATCH(T, hipLaunchKernelGGL(k_finalize<T>, dim3(gb + lb), dim3(256), 0, st, a, gb, do_adam ? 1 : 0,
                                              do_loss ? 1 : 0));
  return hipGetLastError();
}

hipError_t launch_adam_only(const KArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, st, const_cast<int32_t *>(a.step));
  if (a.num_shapes > 0) hipLaunchKernelGGL(k_adam, dim3((a.num_shapes + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
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
