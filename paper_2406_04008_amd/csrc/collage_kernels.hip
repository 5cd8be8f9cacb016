// HIP kernels (gfx950, wave64) of the image-space collage hot path.
//
// Per call the work is split into three launches with grids fixed by the scene:
//   k_transform  one wave per item: eq. 2 applied to the outline (in double precision), float edge
//                records for the scan and double edge records for the per-pixel evaluation, both
//                relative to the item's origin, the pixel box of the item's coverage support and the
//                outline orientation.
//   k_tiles      one workgroup per screen tile: bins the layout's items whose support box meets the
//                tile (ordered by item index, kept in LDS); for every pixel and binned item, scans the
//                item's edges in float32 (edge records read through the scalar cache, shared by the
//                whole wave) for the nearest edge and the even-odd parity, then evaluates the signed
//                distance to that one edge, the coverage and (adjoint calls) the gradient terms in
//                double precision; accumulates S and S_pad, the loss terms and dLoss/dS per pixel, and
//                reduces the adjoint of every pixel per item into one partial per (tile, item) -- no
//                atomics.  The nearest-edge index found by the coverage pass is kept in LDS for the
//                adjoint pass (items beyond the LDS depth are rescanned).
//   k_finalize   one wave per item sums its tiles' partials in a fixed order (gradient, then the
//                optional Adam update); one workgroup per layout sums its tiles' loss partials in a
//                fixed order.
// Results are deterministic (no atomics, fixed reduction orders).
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

__device__ __forceinline__ double wave_sum(double v) {
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
// Nearest edge (lowest index among equal float distances) of one item, and the even-odd parity of
// the crossings of the ray from the pixel towards +x (half-open rule on the vertex ordinates).
__device__ __forceinline__ void edge_scan(cptr<EdgeRec> E, int cnt, float rx, float ry, int &bi, bool &par) {
  float best = INFINITY;
  int idx = 0;
  bool pr = false;
#pragma unroll 2
  for (int e = 0; e < cnt; ++e) {
    const float ax = E[e].ax, ay = E[e].ay, exs = E[e].exs, eys = E[e].eys;
    const float ex = E[e].ex, ey = E[e].ey, by = E[e].by, slope = E[e].slope;
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
    pr ^= ((c1 != c2) && xt);
  }
  bi = idx;
  par = pr;
}

// Signed distance (double) from (rx, ry) to edge e; u is the clamped parameter of the nearest point
// and (qx, qy) = p - nearest point.
struct PairD {
  double sd, d, u, qx, qy;
};

__device__ __forceinline__ PairD pair_eval(const EdgeD &e, double rx, double ry, bool par) {
  const double wx = rx - e.ax, wy = ry - e.ay;
  const double ee = e.ex * e.ex + e.ey * e.ey;
  double u = 0.0;
  if (ee > 0.0) u = fmin(fmax((wx * e.ex + wy * e.ey) / ee, 0.0), 1.0);
  PairD r;
  r.qx = wx - u * e.ex;
  r.qy = wy - u * e.ey;
  r.d = sqrt(r.qx * r.qx + r.qy * r.qy);
  r.sd = par ? r.d : -r.d;
  r.u = u;
  return r;
}

// The float scan can order two edges wrongly only when their squared distances agree to float
// precision.  Away from the (measure-zero) medial axes that happens only between neighbouring edges
// (near the boundary between a vertex's fan and an edge's perpendicular strip), where the choice does
// not change the distance much but does tilt the gradient direction.  So the nearest edge is decided
// again in double among the scan's choice and its two neighbours (lowest index on exact ties).
__device__ __forceinline__ PairD nearest_refined(const EdgeD *E, int ec, int bi, double rx, double ry, bool par,
                                                 int &best) {
  const int lo = bi == 0 ? ec - 1 : bi - 1, hi = bi + 1 == ec ? 0 : bi + 1;
  int cand[3] = {lo, bi, hi};
  // visit in increasing index so that strict '<' keeps the lowest index on ties
  if (cand[0] > cand[1]) {
    const int t = cand[0];
    cand[0] = cand[1];
    cand[1] = t;
  }
  if (cand[1] > cand[2]) {
    const int t = cand[1];
    cand[1] = cand[2];
    cand[2] = t;
  }
  if (cand[0] > cand[1]) {
    const int t = cand[0];
    cand[0] = cand[1];
    cand[1] = t;
  }
  PairD r = pair_eval(E[cand[0]], rx, ry, par);
  best = cand[0];
#pragma unroll
  for (int j = 1; j < 3; ++j) {
    if (cand[j] == cand[j - 1]) continue;
    const PairD c = pair_eval(E[cand[j]], rx, ry, par);
    if (c.d < r.d) {
      r = c;
      best = cand[j];
    }
  }
  return r;
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

// Adjoint terms of one (pixel, item): omega * d sd / d(t, theta, s), up to the per-item factors
// (-k for t, 1/s for s) applied by the finalize kernel.  omega = G dalpha/dsd + G_pad dalpha_pad/dsd.
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
    const double il = 1.0 / sqrt(e.ex * e.ex + e.ey * e.ey);
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
  t.w = om * (q.sd - (nx * rx + ny * ry));
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

// ------------------------------------------------------------------------------------------------
// k_tiles: one workgroup per T x T screen tile, one thread per pixel, one wave per 8 x 8 quadrant.
// ADJ = false: coverage and loss.  ADJ = true: also the adjoint (gradient partials).
// ------------------------------------------------------------------------------------------------
template <int T, bool ADJ>
__global__ __launch_bounds__(T *T) void k_tiles(KArgs a) {
  constexpr int NT = T * T;
  constexpr int NW = NT / 64;
  constexpr int QPR = T / 8;
  constexpr int CS = ADJ ? kMaxCacheSlots : 1;
  __shared__ int s_list[kMaxBinChunk];
  __shared__ int s_wcnt[NW];
  __shared__ unsigned short s_cache[CS][NT];
  __shared__ double4 s_red[NW][64];
  __shared__ double s_loss[NW][5];

  const int tile = blockIdx.x;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  cptr<LayoutRec> LS = konst(a.layouts);
  const int b = layout_of_tile(LS, a.num_layouts, tile);
  const int W = LS[b].W, H = LS[b].H, ntx = LS[b].ntx;
  const int sb = LS[b].shape_begin, se = LS[b].shape_end;
  const int nb = se - sb;
  const int64_t pix_off = LS[b].pix_off, list_off = LS[b].list_off;
  const int lt = tile - LS[b].tile_off;
  const int tyi = lt / ntx, txi = lt - tyi * ntx;
  const int x0 = txi * T, y0 = tyi * T;
  const int wbx0 = x0 + 8 * (w % QPR), wby0 = y0 + 8 * (w / QPR);
  const int wbx1 = wbx0 + 7, wby1 = wby0 + 7;
  const int pxi = wbx0 + (l & 7), pyi = wby0 + (l >> 3);
  const bool valid = pxi < W && pyi < H;
  const float px = pxi + 0.5f, py = pyi + 0.5f;
  const double pxd = pxi + 0.5, pyd = pyi + 0.5;
  const int64_t pix = pix_off + (int64_t)pyi * W + pxi;
  const int64_t list_base = list_off + (int64_t)lt * nb;
  const int chunk = a.bin_chunk;
  const int nchunks = (nb + chunk - 1) / chunk;
  const int cache_slots = ADJ ? a.cache_slots : 0;
  cptr<int4> BB = konst(a.bbox);
  cptr<ShapeRec> SR = konst(a.shapes);
  cptr<EdgeRec> ED = konst(a.edges);

  // ---- binning + coverage --------------------------------------------------------------------
  double S = 0.0, Sp = 0.0;
  int slots = 0, last_cnt = 0;
  for (int cb = sb; cb < se; cb += chunk) {
    const int ce = min(cb + chunk, se);
    const int cnt =
        bin_chunk<NT>(a, cb, ce, x0, y0, x0 + T - 1, y0 + T - 1, s_list, s_wcnt, a.tile_list + list_base + slots);
    last_cnt = cnt;
    for (int q = 0; q < cnt; ++q) {
      const int sid = uniform(s_list[q]);
      const int4 bb = load_box(BB, sid);
      if (bb.x > wbx1 || bb.z < wbx0 || bb.y > wby1 || bb.w < wby0) continue;
      const int eo = SR[sid].edge_off, ec = SR[sid].edge_cnt;
      int bi;
      bool par;
      edge_scan(ED + eo, ec, px - SR[sid].cxf, py - SR[sid].cyf, bi, par);
      if (ec > 0) {
        int be;
        const PairD pr = nearest_refined(a.edges_d + eo, ec, bi, pxd - SR[sid].cx, pyd - SR[sid].cy, par, be);
        double al, dal, alp, dalp;
        coverage(a, pr.sd, al, dal, alp, dalp);
        S += al;
        Sp += alp;
      }
      if (ADJ) {
        const int slot = slots + q;
        if (slot < cache_slots) s_cache[slot < CS ? slot : 0][tid] = (unsigned short)(bi | (par ? 0x8000 : 0));
      }
    }
    slots += cnt;
    __syncthreads();
  }
  if (tid == 0) a.tile_count[tile] = slots;

  // ---- per-pixel loss terms and dLoss/dS -----------------------------------------------------
  const double M = valid ? (double)a.mask[pix] : 0.0;
  const double yinv = (double)H - pyd;
  const double ov = fmax(S - 1.0, 0.0), un = fmax(1.0 - S, 0.0), pv = fmax(Sp - 1.0, 0.0);
  if (valid && a.cov_out) a.cov_out[pix] = (float)S;
  if (valid && a.cov_pad_out) a.cov_pad_out[pix] = (float)Sp;
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
  if (!ADJ) return;

  double c_ov = a.w[0], c_c = a.w[1], c_f = a.w[2], c_p = a.w[3], c_d = a.w[4];
  if (a.dloss) {
    c_ov *= (double)a.dloss[5 * b + 0];
    c_c *= (double)a.dloss[5 * b + 1];
    c_f *= (double)a.dloss[5 * b + 2];
    c_p *= (double)a.dloss[5 * b + 3];
    c_d *= (double)a.dloss[5 * b + 4];
  }
  double G = 0.0, Gp = 0.0;
  if (valid) {
    G = 2.0 * c_ov * ov + c_c * (1.0 - M) - 2.0 * c_f * (M * un) + c_d * yinv;
    Gp = 2.0 * c_p * pv;
  }

  // ---- adjoint: per (tile, item) partial gradient ----------------------------------------------
  int slot0 = 0;
  for (int cb = sb; cb < se; cb += chunk) {
    const int ce = min(cb + chunk, se);
    int cnt = last_cnt;
    if (nchunks > 1) cnt = bin_chunk<NT>(a, cb, ce, x0, y0, x0 + T - 1, y0 + T - 1, s_list, s_wcnt, nullptr);
    for (int g0 = 0; g0 < cnt; g0 += 64) {
      const int gn = min(64, cnt - g0);
      for (int q = g0; q < g0 + gn; ++q) {
        const int sid = uniform(s_list[q]);
        const int4 bb = load_box(BB, sid);
        double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);
        if (!(bb.x > wbx1 || bb.z < wbx0 || bb.y > wby1 || bb.w < wby0)) {
          const int eo = SR[sid].edge_off, ec = SR[sid].edge_cnt;
          const int slot = slot0 + q;
          int bi;
          bool par;
          if (slot < cache_slots) {
            const unsigned code = s_cache[slot < CS ? slot : 0][tid];
            bi = (int)(code & 0x7fffu);
            par = (code & 0x8000u) != 0u;
          } else {
            edge_scan(ED + eo, ec, px - SR[sid].cxf, py - SR[sid].cyf, bi, par);
          }
          double4 t = make_double4(0.0, 0.0, 0.0, 0.0);
          if (ec > 0) {
            const double rx = pxd - SR[sid].cx, ry = pyd - SR[sid].cy;
            int be;
            const PairD pr = nearest_refined(a.edges_d + eo, ec, bi, rx, ry, par, be);
            t = adjoint_terms(a, a.edges_d[eo + be], pr, rx, ry, par, SR[sid].orient, G, Gp);
          }
          acc.x = wave_sum(t.x);
          acc.y = wave_sum(t.y);
          acc.z = wave_sum(t.z);
          acc.w = wave_sum(t.w);
        }
        if (NW == 1) {
          if (l == 0) a.tile_partial[list_base + slot0 + q] = acc;
        } else {
          if (l == 0) s_red[w][q - g0] = acc;
        }
      }
      if (NW > 1) {
        __syncthreads();
        if (tid < gn) {
          double4 s = s_red[0][tid];
          for (int j = 1; j < NW; ++j) {
            const double4 v = s_red[j][tid];
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
          }
          a.tile_partial[list_base + slot0 + g0 + tid] = s;
        }
        __syncthreads();
      }
    }
    slot0 += cnt;
    if (nchunks > 1) __syncthreads();
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
  const float k = SR[sid].k, s = SR[sid].s;
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
        const double4 v = a.tile_partial[list_off + (int64_t)lt * nb + slot];
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
    float4 g = make_float4((float)(-(double)k * acc.x), (float)(-(double)k * acc.y), (float)acc.z,
                           (float)(acc.w / (double)s));
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
    int be;
    const PairD pr = nearest_refined(a.edges_d + eo, ec, bi, pxi + 0.5 - SR[q].cx, pyi + 0.5 - SR[q].cy, par, be);
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
  const int blocks = (a.num_shapes + 3) / 4;
  if (blocks > 0) {
    hipLaunchKernelGGL(k_transform, dim3(blocks), dim3(256), 0, st, a);
  } else if (a.step_inc) {
    hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, st, a.step_inc);
  }
  return hipGetLastError();
}

hipError_t launch_tiles(const KArgs &a, bool adjoint, hipStream_t st) {
  if (a.total_tiles <= 0) return hipSuccess;
  const dim3 grid(a.total_tiles);
  if (a.tile == 8) {
    if (adjoint)
      hipLaunchKernelGGL((k_tiles<8, true>), grid, dim3(64), 0, st, a);
    else
      hipLaunchKernelGGL((k_tiles<8, false>), grid, dim3(64), 0, st, a);
  } else {
    if (adjoint)
      hipLaunchKernelGGL((k_tiles<16, true>), grid, dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL((k_tiles<16, false>), grid, dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const KArgs &a, bool do_grad, bool do_loss, bool do_adam, hipStream_t st) {
  const int gb = do_grad ? (a.num_shapes + 3) / 4 : 0;
  const int lb = do_loss ? a.num_layouts : 0;
  if (gb + lb == 0) return hipSuccess;
  if (a.tile == 8)
    hipLaunchKernelGGL(k_finalize<8>, dim3(gb + lb), dim3(256), 0, st, a, gb, do_adam ? 1 : 0, do_loss ? 1 : 0);
  else
    hipLaunchKernelGGL(k_finalize<16>, dim3(gb + lb), dim3(256), 0, st, a, gb, do_adam ? 1 : 0, do_loss ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_adam_only(const KArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, st, const_cast<int32_t *>(a.step));
  if (a.num_shapes > 0) hipLaunchKernelGGL(k_adam, dim3((a.num_shapes + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_render(const KArgs &a, int first, int count, const int64_t *, float *alpha, float *alpha_pad,
                         int max_pixels, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_render, dim3((max_pixels + 255) / 256, count), dim3(256), 0, st, a, first, alpha, alpha_pad);
  return hipGetLastError();
}

}  // namespace collage
