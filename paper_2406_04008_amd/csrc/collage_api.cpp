// Host side of the C ABI declared in include/collage.h: argument validation, workspace planning,
// kernel dispatch and hipGraph capture.  No compute happens here.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <limits>
#include <vector>

#include "collage.h"
#include "collage_internal.h"

using namespace collage;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(COLLAGE_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct collage_scene {
  int32_t B = 0, N = 0, V = 0;
  int32_t tile = kDefaultTile;
  int64_t code_cap = 0;
  int64_t chunk_cap = 0;
  int32_t bin_chunk = kDefaultBinChunk;
  int32_t cover_grid = 1, adjoint_grid = 1;
  double cover_taper = 0.25;  // set at creation from the items' vertex counts
  uint32_t flags = 0;
  std::vector<LayoutRec> layouts;
  std::vector<int32_t> vert_off;
  const float *verts = nullptr, *rho = nullptr, *mask = nullptr, *stroke = nullptr;
  float tau = 0.5f, r_cut = 8.0f, r_pad = 0.0f;
  float w[kLossTerms] = {1, 1, 1, 0, 0, 0, 0, 0, 0};
  int64_t total_pixels = 0, total_tiles = 0, list_total = 0, total_ptiles = 0, total_rows = 0, row_list_total = 0;
  int32_t max_canvas = 0;
  // device tables owned by the scene
  LayoutRec *d_layouts = nullptr;
  int32_t *d_vert_off = nullptr;
  // workspace layout
  int64_t unit_pool = 0;  // units of all layouts' pools
  size_t off_ibase = 0, off_rbase = 0;
  size_t off_status = 0, off_shapes = 0, off_bins = 0, off_edges = 0, off_edges_d = 0, off_count = 0, off_loss = 0,
         off_list = 0, off_rcount = 0, off_rlist = 0, off_aux = 0, off_tcost = 0, off_tpre = 0, off_head = 0, off_acc = 0,
         off_gbuf = 0, off_codes = 0, off_uflags = 0, off_vacc = 0, off_units = 0;
  size_t ws_bytes = 0;
};

struct collage_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct collage_timer {
  std::vector<hipEvent_t> start, stop;
  int32_t recorded = 0;  // pairs recorded by the last collage_iterate_n call
};

namespace {

// A layout's default unit pool holds four times the units of its items at twice their rim radius, at
// least this many (and never more than every item in every tile).
constexpr int64_t kMinUnitCapacity = 65536;

// Per layout, the units of its items at twice their rim radius: per item, the screen tiles that a support
// box of side 2 (k 2 (rho + w) + r_cut + r_pad) + 2 px can meet, at most the layout's tiles (rho: the
// largest vertex radius, w: the stroke half-width, both canonical px, read from the device arrays).
int unit_bounds(const collage_scene_desc *d, const collage_scene *s, std::vector<int64_t> &bound) {
  bound.assign(s->B, 0);
  if (s->N == 0) return COLLAGE_OK;
  std::vector<float> v(2 * (size_t)s->V), w(s->N, 0.0f);
  hipError_t e = hipSuccess;
  if (s->V > 0) e = hipMemcpy(v.data(), d->verts, sizeof(float) * v.size(), hipMemcpyDeviceToHost);
  if (e == hipSuccess && d->stroke) e = hipMemcpy(w.data(), d->stroke, sizeof(float) * w.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(verts, stroke) for the unit capacity");
  const double ext = (double)d->r_cut + std::max(0.0, (double)d->r_pad);
  for (int b = 0; b < s->B; ++b) {
    const LayoutRec &L = s->layouts[b];
    const int64_t tiles_b = (int64_t)L.ntx * L.nty;
    for (int i = L.shape_begin; i < L.shape_end; ++i) {
      double rho = 0.0;
      for (int m = s->vert_off[i]; m < s->vert_off[i + 1]; ++m)
        rho = std::max(rho, std::sqrt((double)v[2 * m] * v[2 * m] + (double)v[2 * m + 1] * v[2 * m + 1]));
      const double side = 2.0 * ((double)L.k * 2.0 * (rho + std::max(0.0f, w[i])) + ext) + 2.0;
      const double per_axis = std::ceil(side / s->tile) + 1.0;
      bound[b] += std::min<int64_t>(tiles_b, (int64_t)std::min(per_axis * per_axis, 1e12));
    }
  }
  return COLLAGE_OK;
}

// The coverage pass's taper (the share of its last wave is 1 - taper times the first's) from the mean
// number of vertices per item, which is about the edges a chunk scans: the longer a chunk keeps a wave
// busy, the further the waves that the SIMDs issue last fall behind.  Measured best: 0.25 for 2,000
// polylines of 7.5 vertices (2048^2), 0.5 for the 64-layout batch (49), 0.8 for the 500 Bezier items
// of 80 (512^2 and 1024^2); a linear ramp between them.
constexpr double kMinCoverTaper = 0.25, kMaxCoverTaper = 0.8;

double cover_taper_of(const std::vector<int32_t> &vert_off) {
  const size_t n = vert_off.size() > 0 ? vert_off.size() - 1 : 0;
  if (n == 0) return kMinCoverTaper;
  const double mean_v = (double)(vert_off[n] - vert_off[0]) / (double)n;
  return std::min(kMaxCoverTaper, std::max(kMinCoverTaper, kMinCoverTaper + 0.0075 * (mean_v - 8.0)));
}

int validate_desc(const collage_scene_desc *d) {
  if (!d) return fail(COLLAGE_ERR_INVALID, "desc is NULL");
  if (d->num_layouts < 1) return fail(COLLAGE_ERR_INVALID, "num_layouts must be >= 1 (got %d)", d->num_layouts);
  if (d->num_shapes < 0 || d->num_verts < 0) return fail(COLLAGE_ERR_INVALID, "negative num_shapes or num_verts");
  if (!d->layout_width || !d->layout_height || !d->layout_scale || !d->layout_shapes || !d->vert_offset)
    return fail(COLLAGE_ERR_INVALID, "a host layout or offset array is NULL");
  for (int b = 0; b < d->num_layouts; ++b) {
    if (d->layout_width[b] < 1 || d->layout_width[b] > 32768 || d->layout_height[b] < 1 ||
        d->layout_height[b] > 32768)
      return fail(COLLAGE_ERR_INVALID, "layout %d: canvas %dx%d outside 1..32768", b, d->layout_width[b],
                  d->layout_height[b]);
    if (!(d->layout_scale[b] > 0.0f) || !std::isfinite(d->layout_scale[b]))
      return fail(COLLAGE_ERR_INVALID, "layout %d: scale must be finite and > 0", b);
  }
  if (d->layout_shapes[0] != 0) return fail(COLLAGE_ERR_INVALID, "layout_shapes[0] must be 0");
  for (int b = 0; b < d->num_layouts; ++b)
    if (d->layout_shapes[b + 1] < d->layout_shapes[b])
      return fail(COLLAGE_ERR_INVALID, "layout_shapes must be nondecreasing (at %d)", b);
  if (d->layout_shapes[d->num_layouts] != d->num_shapes)
    return fail(COLLAGE_ERR_SIZE, "layout_shapes[B] = %d but num_shapes = %d", d->layout_shapes[d->num_layouts],
                d->num_shapes);
  if (d->vert_offset[0] != 0) return fail(COLLAGE_ERR_INVALID, "vert_offset[0] must be 0");
  for (int i = 0; i < d->num_shapes; ++i) {
    const int n = d->vert_offset[i + 1] - d->vert_offset[i];
    if (n < 0) return fail(COLLAGE_ERR_INVALID, "vert_offset must be nondecreasing (at item %d)", i);
    if (n > kMaxVertsPerItem) return fail(COLLAGE_ERR_INVALID, "item %d has %d vertices (max %d)", i, n, kMaxVertsPerItem);
  }
  if (d->vert_offset[d->num_shapes] != d->num_verts)
    return fail(COLLAGE_ERR_SIZE, "vert_offset[N] = %d but num_verts = %d", d->vert_offset[d->num_shapes], d->num_verts);
  if (d->num_verts > 0 && !d->verts) return fail(COLLAGE_ERR_INVALID, "verts is NULL");
  if (!d->mask) return fail(COLLAGE_ERR_INVALID, "mask is NULL");
  if (!(d->tau > 0.0f) || !std::isfinite(d->tau)) return fail(COLLAGE_ERR_INVALID, "tau must be finite and > 0");
  if (!(d->r_cut >= 0.0f) || !std::isfinite(d->r_cut)) return fail(COLLAGE_ERR_INVALID, "r_cut must be finite and >= 0");
  if (!(d->r_pad >= 0.0f) || !std::isfinite(d->r_pad)) return fail(COLLAGE_ERR_INVALID, "r_pad must be finite and >= 0");
  const float ws[kLossTerms] = {d->w_overlap, d->w_contain, d->w_fill, d->w_pad, d->w_down,
                                d->w_uniform, d->w_wmse, d->w_centre, d->w_objdown};
  for (float x : ws)
    if (!std::isfinite(x)) return fail(COLLAGE_ERR_INVALID, "loss weights must be finite");
  if (d->tile != 0 && d->tile != 8 && d->tile != 16 && d->tile != 32 && d->tile != 64 && d->tile != 128)
    return fail(COLLAGE_ERR_UNSUPPORTED, "tile must be 0, 8, 16, 32, 64 or 128 (got %d)", d->tile);
  if (d->code_capacity < -1) return fail(COLLAGE_ERR_INVALID, "code_capacity must be -1 or >= 0");
  if (d->unit_capacity < -1) return fail(COLLAGE_ERR_INVALID, "unit_capacity must be -1, 0 or > 0");
  if (d->bin_chunk < 0 || d->bin_chunk > kMaxBinChunk)
    return fail(COLLAGE_ERR_INVALID, "bin_chunk must be 0..%d", kMaxBinChunk);
  if (d->flags & ~(uint32_t)COLLAGE_FLAG_AREA_MEAN) return fail(COLLAGE_ERR_UNSUPPORTED, "unknown flags 0x%x", d->flags);
  return COLLAGE_OK;
}

KArgs base_args(const collage_scene *s, void *ws) {
  KArgs a;
  std::memset(&a, 0, sizeof(a));
  char *w = static_cast<char *>(ws);
  a.layouts = s->d_layouts;
  a.num_layouts = s->B;
  a.num_shapes = s->N;
  a.total_tiles = (int32_t)s->total_tiles;
  a.total_ptiles = (int32_t)s->total_ptiles;
  a.total_rows = (int32_t)s->total_rows;
  a.rowbin = s->list_total > kRowBinTests ? 1 : 0;
  a.scan_in_cover = s->total_tiles <= kScanInCoverTiles ? 1 : 0;
  a.tile = s->tile;
  a.bin_chunk = s->bin_chunk;
  a.item_base = reinterpret_cast<int32_t *>(w + s->off_ibase);
  a.row_base = reinterpret_cast<long long *>(w + s->off_rbase);
  a.chunk_cap = s->chunk_cap;
  a.code_cap = s->code_cap;
  a.cover_grid = s->cover_grid;
  a.cover_taper = s->cover_taper;
  a.adjoint_grid = s->adjoint_grid;
  a.vert_off = s->d_vert_off;
  a.verts = s->verts;
  a.rho = s->rho;
  a.mask = s->mask;
  a.stroke = s->stroke;
  a.status = reinterpret_cast<int32_t *>(w + s->off_status);
  a.shapes = reinterpret_cast<ShapeRec *>(w + s->off_shapes);
  a.bins = reinterpret_cast<BinRec *>(w + s->off_bins);
  a.edges = reinterpret_cast<EdgeRec *>(w + s->off_edges);
  a.edges_d = reinterpret_cast<EdgeD *>(w + s->off_edges_d);
  a.tile_units = reinterpret_cast<int2 *>(w + s->off_count);
  a.block_loss = reinterpret_cast<double *>(w + s->off_loss);
  a.tile_list = reinterpret_cast<int32_t *>(w + s->off_list);
  a.row_count = reinterpret_cast<int32_t *>(w + s->off_rcount);
  a.row_list = reinterpret_cast<int32_t *>(w + s->off_rlist);
  a.entry_aux = reinterpret_cast<int4 *>(w + s->off_aux);
  a.units = reinterpret_cast<UnitRec *>(w + s->off_units);
  a.tile_cost = reinterpret_cast<int2 *>(w + s->off_tcost);
  a.tile_pre = reinterpret_cast<long long *>(w + s->off_tpre);
  a.head = reinterpret_cast<unsigned long long *>(w + s->off_head);
  a.acc = reinterpret_cast<unsigned long long *>(w + s->off_acc);
  a.gbuf = reinterpret_cast<double2 *>(w + s->off_gbuf);
  a.codes = reinterpret_cast<uint16_t *>(w + s->off_codes);
  a.uflags = reinterpret_cast<uint8_t *>(w + s->off_uflags);
  a.tau = s->tau;
  a.inv_tau = 1.0f / s->tau;
  a.r_cut = s->r_cut;
  a.r_pad = s->r_pad;
  a.inv_tau_d = 1.0 / (double)s->tau;
  a.log2e_inv_tau = 1.4426950408889634 / (double)s->tau;
  a.pad_factor = std::exp(-(double)s->r_pad / (double)s->tau);
  for (int i = 0; i < kLossTerms; ++i) a.w[i] = s->w[i];
  a.area_mean = (s->flags & COLLAGE_FLAG_AREA_MEAN) ? 1 : 0;
  return a;
}

int check_ws(const collage_scene *s, void *ws, size_t bytes) {
  if (!ws) return fail(COLLAGE_ERR_WORKSPACE, "workspace is NULL");
  if (bytes < s->ws_bytes)
    return fail(COLLAGE_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", bytes, s->ws_bytes);
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(COLLAGE_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  return COLLAGE_OK;
}

int check_adam(float lr, float b1, float b2, float eps) {
  if (!std::isfinite(lr) || lr < 0.0f) return fail(COLLAGE_ERR_INVALID, "lr_px must be finite and >= 0");
  if (!(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f)) return fail(COLLAGE_ERR_INVALID, "betas must be in [0, 1)");
  if (!(eps > 0.0f) || !std::isfinite(eps)) return fail(COLLAGE_ERR_INVALID, "eps must be finite and > 0");
  return COLLAGE_OK;
}

}  // namespace

extern "C" {

const char *collage_last_error(void) { return g_err; }

const char *collage_version(void) { return "collage-mi355x 0.1 (gfx950)"; }

int collage_scene_create(const collage_scene_desc *desc, collage_scene **out) {
  if (!out) return fail(COLLAGE_ERR_INVALID, "out is NULL");
  *out = nullptr;
  int rc = validate_desc(desc);
  if (rc) return rc;
  collage_scene *s = new (std::nothrow) collage_scene();
  if (!s) return fail(COLLAGE_ERR_INVALID, "out of host memory");
  s->B = desc->num_layouts;
  s->N = desc->num_shapes;
  s->V = desc->num_verts;
  s->tile = desc->tile == 0 ? kDefaultTile : desc->tile;

  s->bin_chunk = desc->bin_chunk == 0 ? kDefaultBinChunk : desc->bin_chunk;
  s->flags = desc->flags;
  s->verts = desc->verts;
  s->rho = desc->rho;
  s->mask = desc->mask;
  s->stroke = desc->stroke;
  s->tau = desc->tau;
  s->r_cut = desc->r_cut;
  s->r_pad = desc->r_pad;
  s->w[0] = desc->w_overlap;
  s->w[1] = desc->w_contain;
  s->w[2] = desc->w_fill;
  s->w[3] = desc->w_pad;
  s->w[4] = desc->w_down;
  s->w[5] = desc->w_uniform;
  s->w[6] = desc->w_wmse;
  s->w[7] = desc->w_centre;
  s->w[8] = desc->w_objdown;
  s->vert_off.assign(desc->vert_offset, desc->vert_offset + s->N + 1);
  s->layouts.resize(s->B);
  int64_t pix = 0, tiles = 0, list = 0, ptiles = 0, rows = 0, rlist = 0;
  for (int b = 0; b < s->B; ++b) {
    LayoutRec &L = s->layouts[b];
    std::memset(&L, 0, sizeof(L));
    L.W = desc->layout_width[b];
    L.H = desc->layout_height[b];
    L.ntx = (L.W + s->tile - 1) / s->tile;
    L.nty = (L.H + s->tile - 1) / s->tile;
    L.tile_off = (int32_t)tiles;
    L.shape_begin = desc->layout_shapes[b];
    L.shape_end = desc->layout_shapes[b + 1];
    L.pix_off = pix;
    L.k = desc->layout_scale[b];
    L.ptile_off = (int32_t)ptiles;
    L.row_off = (int32_t)rows;
    L.row_list_off = rlist;
    rows += L.nty;
    rlist += (int64_t)L.nty * (L.shape_end - L.shape_begin);
    ptiles += (int64_t)((L.W + kPixTile - 1) / kPixTile) * ((L.H + kPixTile - 1) / kPixTile);
    pix += (int64_t)L.W * L.H;
    tiles += (int64_t)L.ntx * L.nty;
    list += (int64_t)L.ntx * L.nty * (L.shape_end - L.shape_begin);
    if (L.W * L.H > s->max_canvas) s->max_canvas = L.W * L.H;
  }
  if (tiles > (int64_t)0x7fffffff || ptiles > (int64_t)0x7fffffff) {
    delete s;
    return fail(COLLAGE_ERR_INVALID, "too many screen tiles");
  }
  s->total_pixels = pix;
  s->total_tiles = tiles;
  s->total_ptiles = ptiles;
  s->total_rows = rows;
  s->row_list_total = rlist;
  s->list_total = list;
  // every (tile, item) pair whose support box meets the tile is one work unit; each layout's units live in
  // a pool of its own, sized by unit_capacity: every item in every tile (-1), the bound above (0), or the
  // given count (at most every item in every tile)
  std::vector<int64_t> bound;
  if (desc->unit_capacity == 0) {
    rc = unit_bounds(desc, s, bound);
    if (rc) {
      delete s;
      return rc;
    }
  }
  int64_t pool = 0;
  for (int b = 0; b < s->B; ++b) {
    LayoutRec &L = s->layouts[b];
    const int64_t dense = (int64_t)L.ntx * L.nty * (L.shape_end - L.shape_begin);
    int64_t cap = dense;
    if (desc->unit_capacity > 0)
      cap = std::min<int64_t>(dense, desc->unit_capacity);
    else if (desc->unit_capacity == 0)
      cap = std::min<int64_t>(dense, std::max<int64_t>(4 * bound[b], kMinUnitCapacity));
    if (cap > (int64_t)0x7fffffff) {
      delete s;
      return fail(COLLAGE_ERR_INVALID, "layout %d: %lld units exceed a pool's limit of 2^31 - 1; set unit_capacity", b,
                  (long long)cap);
    }
    L.list_off = pool;
    L.unit_cap = (int32_t)cap;
    pool += cap;
  }
  if (pool > (int64_t)0x7fffffff) {
    delete s;
    return fail(COLLAGE_ERR_INVALID, "the unit pools (%lld units) exceed 2^31 - 1 entries; set unit_capacity",
                (long long)pool);
  }
  s->unit_pool = std::max<int64_t>(pool, 1);
  // nearest-edge codes: one per lane of every 64-pixel chunk of the pass; a unit has at most
  // tile^2 / 64 chunks.  Default: four items per pixel on average (units beyond it are rescanned).
  const int64_t max_chunks = s->unit_pool * (int64_t)((s->tile * s->tile + 63) / 64);
  s->chunk_cap = max_chunks;
  int64_t code_cap = desc->code_capacity;
  if (code_cap < 0) code_cap = std::max<int64_t>(65536, 4 * ((pix + 63) / 64));
  s->code_cap = std::min<int64_t>(code_cap, max_chunks);
  size_t off = 0;
  s->off_status = off;
  off = align256(off + sizeof(int32_t) * kStatusWords);
  s->off_ibase = off;
  off = align256(off + sizeof(int32_t) * (size_t)s->N);
  s->off_rbase = off;
  off = align256(off + sizeof(long long) * (size_t)rows);
  s->off_shapes = off;
  off = align256(off + sizeof(ShapeRec) * (size_t)s->N);
  s->off_bins = off;
  off = align256(off + sizeof(BinRec) * (size_t)s->N);
  s->off_edges = off;
  off = align256(off + sizeof(EdgeRec) * ((size_t)s->V + kEdgePad));
  s->off_edges_d = off;
  off = align256(off + sizeof(EdgeD) * (size_t)s->V);
  s->off_count = off;
  off = align256(off + sizeof(int2) * (size_t)tiles);
  s->off_loss = off;
  off = align256(off + sizeof(double) * kLossTerms * (size_t)ptiles);
  s->off_uflags = off;
  off = align256(off + (size_t)pix);
  s->off_vacc = off;
  off = align256(off + 2 * sizeof(unsigned long long) * (size_t)s->V);
  s->off_list = off;
  off = align256(off + sizeof(int32_t) * (size_t)s->unit_pool);
  s->off_rcount = off;
  off = align256(off + sizeof(int32_t) * (size_t)rows);
  s->off_rlist = off;
  off = align256(off + sizeof(int32_t) * (size_t)(list > kRowBinTests ? rlist : 0));
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  s->cover_grid = cus * kCoverBlocksPerCU;
  s->cover_taper = cover_taper_of(s->vert_off);
  s->adjoint_grid = cus * kAdjointBlocksPerCU;
  s->off_aux = off;
  off = align256(off + sizeof(int4) * (size_t)s->unit_pool);
  s->off_units = off;
  off = align256(off + sizeof(UnitRec) * (size_t)s->unit_pool);
  s->off_tcost = off;
  off = align256(off + sizeof(int2) * (size_t)tiles);
  s->off_tpre = off;
  off = align256(off + sizeof(long long) * 2 * ((size_t)tiles + 1));
  s->off_head = off;
  off = align256(off + 4 * sizeof(unsigned long long) * (size_t)s->unit_pool);
  s->off_acc = off;
  off = align256(off + 2 * sizeof(unsigned long long) * (size_t)pix);
  s->off_gbuf = off;
  off = align256(off + sizeof(double2) * (size_t)pix);
  s->off_codes = off;
  off = align256(off + sizeof(uint16_t) * 64 * (size_t)s->code_cap);
  s->ws_bytes = off + 256;

  hipError_t e = hipMalloc(&s->d_layouts, sizeof(LayoutRec) * s->B);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipMalloc(layouts)");
  }
  e = hipMalloc(&s->d_vert_off, sizeof(int32_t) * (s->N + 1));
  if (e == hipSuccess) e = hipMemcpy(s->d_layouts, s->layouts.data(), sizeof(LayoutRec) * s->B, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->d_vert_off, s->vert_off.data(), sizeof(int32_t) * (s->N + 1), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    collage_scene_destroy(s);
    return hip_fail(e, "scene device tables");
  }
  *out = s;
  return COLLAGE_OK;
}

void collage_scene_destroy(collage_scene *s) {
  if (!s) return;
  if (s->d_layouts) (void)hipFree(s->d_layouts);
  if (s->d_vert_off) (void)hipFree(s->d_vert_off);
  delete s;
}

int collage_workspace_size(const collage_scene *s, size_t *bytes) {
  if (!s || !bytes) return fail(COLLAGE_ERR_INVALID, "scene or bytes is NULL");
  *bytes = s->ws_bytes;
  return COLLAGE_OK;
}

int collage_read_status(const collage_scene *s, const void *ws, size_t ws_bytes, int32_t *status, void *stream) {
  if (!s || !status) return fail(COLLAGE_ERR_INVALID, "scene or status is NULL");
  int rc = check_ws(s, const_cast<void *>(ws), ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const char *w = static_cast<const char *>(ws) + s->off_status;
  hipError_t e = hipMemcpyAsync(status, w, sizeof(int32_t) * kStatusWords, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? COLLAGE_OK : hip_fail(e, "collage_read_status");
}

int collage_scene_info(const collage_scene *s, int64_t *num_pixels, int64_t *num_tiles) {
  if (!s) return fail(COLLAGE_ERR_INVALID, "scene is NULL");
  if (num_pixels) *num_pixels = s->total_pixels;
  if (num_tiles) *num_tiles = s->total_tiles;
  return COLLAGE_OK;
}

int collage_forward(const collage_scene *s, const float *params, float *cov, float *cov_pad, float *loss, void *ws,
                    size_t ws_bytes, void *stream) {
  if (!s) return fail(COLLAGE_ERR_INVALID, "scene is NULL");
  if ((!params && s->N > 0) || !loss) return fail(COLLAGE_ERR_INVALID, "params or loss is NULL");
  int rc = check_ws(s, ws, ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KArgs a = base_args(s, ws);
  a.params = params;
  a.cov_out = cov;
  a.cov_pad_out = cov_pad;
  a.loss_out = loss;
  a.write_loss = 1;
  hipError_t e = launch_transform(a, st);
  if (e == hipSuccess) e = launch_bin(a, st);
  if (e == hipSuccess) e = launch_scan(a, st);
  if (e == hipSuccess) e = launch_cover(a, st);
  if (e == hipSuccess) e = launch_pixel(a, false, st);
  if (e == hipSuccess) e = launch_finalize(a, false, true, false, st);
  return e == hipSuccess ? COLLAGE_OK : hip_fail(e, "collage_forward launch");
}

int collage_backward(const collage_scene *s, const float *params, const float *dloss, float *grad, void *ws,
                     size_t ws_bytes, void *stream) {
  if (!s) return fail(COLLAGE_ERR_INVALID, "scene is NULL");
  if (!dloss) return fail(COLLAGE_ERR_INVALID, "dloss is NULL");
  if (s->N > 0 && (!params || !grad)) return fail(COLLAGE_ERR_INVALID, "params or grad is NULL");
  int rc = check_ws(s, ws, ws_bytes);
  if (rc) return rc;
  if (s->N == 0) return COLLAGE_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KArgs a = base_args(s, ws);
  a.params = params;
  a.dloss = dloss;
  a.grad_out = grad;
  a.keep_codes = 1;
  hipError_t e = launch_transform(a, st);
  if (e == hipSuccess) e = launch_bin(a, st);
  if (e == hipSuccess) e = launch_scan(a, st);
  if (e == hipSuccess) e = launch_cover(a, st);
  if (e == hipSuccess) e = launch_pixel(a, true, st);
  if (e == hipSuccess) e = launch_uniform_grad(a, st);
  if (e == hipSuccess) e = launch_adjoint(a, st);
  if (e == hipSuccess) e = launch_finalize(a, true, false, false, st);
  return e == hipSuccess ? COLLAGE_OK : hip_fail(e, "collage_backward launch");
}

int collage_backward_vertices(const collage_scene *s, const float *params, const float *dloss, float *grad,
                              float *grad_verts, void *ws, size_t ws_bytes, void *stream) {
  if (!s) return fail(COLLAGE_ERR_INVALID, "scene is NULL");
  if (!dloss) return fail(COLLAGE_ERR_INVALID, "dloss is NULL");
  if (s->N > 0 && (!params || (s->V > 0 && !grad_verts)))
    return fail(COLLAGE_ERR_INVALID, "params or grad_verts is NULL");
  int rc = check_ws(s, ws, ws_bytes);
  if (rc) return rc;
  if (s->N == 0) return COLLAGE_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KArgs a = base_args(s, ws);
  a.params = params;
  a.dloss = dloss;
  a.grad_out = grad;
  a.grad_verts_out = grad_verts;
  a.vacc = reinterpret_cast<unsigned long long *>(static_cast<char *>(ws) + s->off_vacc);
  a.keep_codes = 1;
  hipError_t e = launch_transform(a, st);
  if (e == hipSuccess) e = launch_bin(a, st);
  if (e == hipSuccess) e = launch_scan(a, st);
  if (e == hipSuccess) e = launch_cover(a, st);
  if (e == hipSuccess) e = launch_pixel(a, true, st);
  if (e == hipSuccess) e = launch_uniform_grad(a, st);
  if (e == hipSuccess && grad) e = launch_adjoint(a, st);
  if (e == hipSuccess && grad) e = launch_finalize(a, true, false, false, st);
  if (e == hipSuccess) e = launch_vertex_grad(a, st);
  return e == hipSuccess ? COLLAGE_OK : hip_fail(e, "collage_backward_vertices launch");
}

int collage_forward_backward_static(const collage_scene *s, const float *params, float *cov, float *cov_pad,
                                    float *loss, float *grad, void *stream) {
  if (!s) return fail(COLLAGE_ERR_INVALID, "scene is NULL");
  if (s->ws_bytes > kStaticScratchBytes)
    return fail(COLLAGE_ERR_WORKSPACE,
                "the scene needs a workspace of %zu bytes, more than the %zu bytes of the static scratch; use "
                "collage_forward_backward with a workspace",
                s->ws_bytes, kStaticScratchBytes);
  if (!loss || (s->N > 0 && (!params || !grad))) return fail(COLLAGE_ERR_INVALID, "params, loss or grad is NULL");
  void *ws = nullptr;
  hipError_t e = static_scratch(&ws);
  if (e != hipSuccess) return hip_fail(e, "static scratch (hipGetSymbolAddress)");
  return collage_forward_backward(s, params, cov, cov_pad, loss, grad, ws, kStaticScratchBytes, stream);
}

int collage_forward_backward(const collage_scene *s, const float *params, float *cov, float *cov_pad, float *loss,
                             float *grad, void *ws, size_t ws_bytes, void *stream) {
  if (!s) return fail(COLLAGE_ERR_INVALID, "scene is NULL");
  if (!loss || (s->N > 0 && (!params || !grad))) return fail(COLLAGE_ERR_INVALID, "params, loss or grad is NULL");
  int rc = check_ws(s, ws, ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KArgs a = base_args(s, ws);
  a.params = params;
  a.cov_out = cov;
  a.cov_pad_out = cov_pad;
  a.loss_out = loss;
  a.grad_out = grad;
  a.write_loss = 1;
  a.keep_codes = 1;
  hipError_t e = launch_transform(a, st);
  if (e == hipSuccess) e = launch_bin(a, st);
  if (e == hipSuccess) e = launch_scan(a, st);
  if (e == hipSuccess) e = launch_cover(a, st);
  if (e == hipSuccess) e = launch_pixel(a, true, st);
  if (e == hipSuccess) e = launch_uniform_grad(a, st);
  if (e == hipSuccess) e = launch_adjoint(a, st);
  if (e == hipSuccess) e = launch_finalize(a, true, true, false, st);
  return e == hipSuccess ? COLLAGE_OK : hip_fail(e, "collage_forward_backward launch");
}

int collage_step(const collage_scene *s, float *params, const float *grad, float *m, float *v, int32_t *step,
                 float lr_px, float beta1, float beta2, float eps, void *stream) {
  if (!s) return fail(COLLAGE_ERR_INVALID, "scene is NULL");
  if (!step || (s->N > 0 && (!params || !grad || !m || !v))) return fail(COLLAGE_ERR_INVALID, "a step buffer is NULL");
  if (s->N > 0 && !s->rho) return fail(COLLAGE_ERR_INVALID, "the scene has no rho (needed by the update)");
  int rc = check_adam(lr_px, beta1, beta2, eps);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KArgs a = base_args(s, nullptr);
  a.grad_out = const_cast<float *>(grad);
  a.param_io = params;
  a.adam_m = m;
  a.adam_v = v;
  a.step = step;
  a.lr_px = lr_px;
  a.beta1 = beta1;
  a.beta2 = beta2;
  a.eps = eps;
  hipError_t e = launch_adam_only(a, st);
  return e == hipSuccess ? COLLAGE_OK : hip_fail(e, "collage_step launch");
}

}  // extern "C"

namespace {

// n consecutive epochs (forward, loss, backward, Adam).  Only the first epoch launches the transform
// kernel: the update kernel of every other epoch transforms the items with their new parameters.
// With a timer of c pairs, the coverage kernels of epochs 0, d, 2d, ... (d = ceil(n / c)) are timestamped,
// pair j around epoch j d: a spread sample of the call's launches when c < n, every launch otherwise.
int iterate_impl(const collage_scene *s, float *params, float *cov, float *cov_pad, float *loss, float *grad, float *m,
                 float *v, int32_t *step, float lr_px, float beta1, float beta2, float eps, void *ws, size_t ws_bytes,
                 void *stream, int32_t n, collage_timer *timer) {
  if (!s) return fail(COLLAGE_ERR_INVALID, "scene is NULL");
  if (!loss || !step || (s->N > 0 && (!params || !grad || !m || !v)))
    return fail(COLLAGE_ERR_INVALID, "an iterate buffer is NULL");
  if (s->N > 0 && !s->rho) return fail(COLLAGE_ERR_INVALID, "the scene has no rho (needed by the update)");
  if (n < 1 || n > 65536) return fail(COLLAGE_ERR_INVALID, "epochs must be 1..65536 (got %d)", n);
  int rc = check_adam(lr_px, beta1, beta2, eps);
  if (rc) return rc;
  rc = check_ws(s, ws, ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KArgs a = base_args(s, ws);
  a.params = params;
  a.cov_out = cov;
  a.cov_pad_out = cov_pad;
  a.loss_out = loss;
  a.grad_out = grad;
  a.param_io = params;
  a.adam_m = m;
  a.adam_v = v;
  a.step = step;
  a.step_inc = step;
  a.lr_px = lr_px;
  a.beta1 = beta1;
  a.beta2 = beta2;
  a.eps = eps;
  a.write_loss = 1;
  a.keep_codes = 1;
  const int32_t stride = timer ? (int32_t)((n + (int64_t)timer->start.size() - 1) / (int64_t)timer->start.size()) : 1;
  if (timer) timer->recorded = (n + stride - 1) / stride;
  hipError_t e = launch_transform(a, st);
  for (int32_t i = 0; i < n && e == hipSuccess; ++i) {
    const bool stamp = timer && i % stride == 0;
    e = launch_bin(a, st);
    if (e == hipSuccess) e = launch_scan(a, st);
    if (e == hipSuccess)
      e = launch_cover(a, st, stamp ? timer->start[i / stride] : nullptr, stamp ? timer->stop[i / stride] : nullptr);
    if (e == hipSuccess) e = launch_pixel(a, true, st);
    if (e == hipSuccess) e = launch_uniform_grad(a, st);
    if (e == hipSuccess) e = launch_adjoint(a, st);
    if (e == hipSuccess) e = launch_finalize(a, true, true, true, st, i + 1 < n);
  }
  return e == hipSuccess ? COLLAGE_OK : hip_fail(e, "collage_iterate launch");
}

}  // namespace

extern "C" {

int collage_iterate(const collage_scene *s, float *params, float *cov, float *cov_pad, float *loss, float *grad, float *m,
                    float *v, int32_t *step, float lr_px, float beta1, float beta2, float eps, void *ws,
                    size_t ws_bytes, void *stream) {
  return iterate_impl(s, params, cov, cov_pad, loss, grad, m, v, step, lr_px, beta1, beta2, eps, ws, ws_bytes, stream,
                      1, nullptr);
}

int collage_iterate_n(const collage_scene *s, float *params, float *cov, float *cov_pad, float *loss, float *grad,
                      float *m, float *v, int32_t *step, float lr_px, float beta1, float beta2, float eps, void *ws,
                      size_t ws_bytes, int32_t epochs, collage_timer *timer, void *stream) {
  return iterate_impl(s, params, cov, cov_pad, loss, grad, m, v, step, lr_px, beta1, beta2, eps, ws, ws_bytes, stream,
                      epochs, timer);
}

int collage_timer_create(int32_t count, collage_timer **out) {
  if (!out) return fail(COLLAGE_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (count < 1 || count > 65536) return fail(COLLAGE_ERR_INVALID, "count must be 1..65536");
  collage_timer *t = new (std::nothrow) collage_timer();
  if (!t) return fail(COLLAGE_ERR_INVALID, "out of host memory");
  t->start.assign(count, nullptr);
  t->stop.assign(count, nullptr);
  for (int i = 0; i < count; ++i) {
    hipError_t e = hipEventCreate(&t->start[i]);
    if (e == hipSuccess) e = hipEventCreate(&t->stop[i]);
    if (e != hipSuccess) {
      collage_timer_destroy(t);
      return hip_fail(e, "hipEventCreate");
    }
  }
  *out = t;
  return COLLAGE_OK;
}

int collage_timer_elapsed(collage_timer *t, float *ms) {
  if (!t || !ms) return fail(COLLAGE_ERR_INVALID, "timer or ms is NULL");
  for (size_t i = 0; i < t->start.size(); ++i) {
    if ((int64_t)i >= t->recorded) {
      ms[i] = std::numeric_limits<float>::quiet_NaN();
      continue;
    }
    hipError_t e = hipEventSynchronize(t->stop[i]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms[i], t->start[i], t->stop[i]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
  }
  return COLLAGE_OK;
}

void collage_timer_destroy(collage_timer *t) {
  if (!t) return;
  for (auto e : t->start)
    if (e) (void)hipEventDestroy(e);
  for (auto e : t->stop)
    if (e) (void)hipEventDestroy(e);
  delete t;
}

int collage_render_shapes(const collage_scene *s, const float *params, int32_t first, int32_t count, float *alpha,
                          float *alpha_pad, void *ws, size_t ws_bytes, void *stream) {
  if (!s) return fail(COLLAGE_ERR_INVALID, "scene is NULL");
  if (first < 0 || count < 0 || first + count > s->N)
    return fail(COLLAGE_ERR_SIZE, "items [%d, %d) outside [0, %d)", first, first + count, s->N);
  if (count > 65535) return fail(COLLAGE_ERR_SIZE, "at most 65535 items per render call");
  if (count > 0 && (!params || !alpha)) return fail(COLLAGE_ERR_INVALID, "params or alpha is NULL");
  int rc = check_ws(s, ws, ws_bytes);
  if (rc) return rc;
  if (count == 0) return COLLAGE_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KArgs a = base_args(s, ws);
  a.params = params;
  hipError_t e = launch_transform(a, st);
  if (e == hipSuccess) e = launch_render(a, first, count, alpha, alpha_pad, s->max_canvas, st);
  return e == hipSuccess ? COLLAGE_OK : hip_fail(e, "collage_render_shapes launch");
}

int collage_graph_create(const collage_scene *s, float *params, float *cov, float *cov_pad, float *loss, float *grad,
                         float *m, float *v, int32_t *step, float lr_px, float beta1, float beta2, float eps, void *ws,
                         size_t ws_bytes, int32_t replays_per_launch, uint32_t graph_flags, void *stream,
                         collage_graph **out) {
  if (!out) return fail(COLLAGE_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!stream) return fail(COLLAGE_ERR_INVALID, "graph capture needs a non-NULL stream");
  if (replays_per_launch < 1 || replays_per_launch > 4096)
    return fail(COLLAGE_ERR_INVALID, "replays_per_launch must be 1..4096");
  if (graph_flags & ~(uint32_t)COLLAGE_GRAPH_RESET_ADAM) return fail(COLLAGE_ERR_UNSUPPORTED, "unknown graph flag");
  if (!s) return fail(COLLAGE_ERR_INVALID, "scene is NULL");
  if ((graph_flags & COLLAGE_GRAPH_RESET_ADAM) && (!step || (s->N > 0 && (!m || !v))))
    return fail(COLLAGE_ERR_INVALID, "m, v or step is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  int rc = COLLAGE_OK;
  if (graph_flags & COLLAGE_GRAPH_RESET_ADAM) {
    e = launch_adam_reset(m, v, step, s->N, st);
    if (e != hipSuccess) rc = hip_fail(e, "adam reset launch");
  }
  if (rc == COLLAGE_OK)
    rc = iterate_impl(s, params, cov, cov_pad, loss, grad, m, v, step, lr_px, beta1, beta2, eps, ws, ws_bytes, stream,
                      replays_per_launch, nullptr);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(st, &g);
  if (rc != COLLAGE_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(e, "hipGraphInstantiate");
  }
  collage_graph *cg = new (std::nothrow) collage_graph();
  if (!cg) {
    (void)hipGraphExecDestroy(ex);
    (void)hipGraphDestroy(g);
    return fail(COLLAGE_ERR_INVALID, "out of host memory");
  }
  cg->graph = g;
  cg->exec = ex;
  *out = cg;
  return COLLAGE_OK;
}

int collage_adam_reset(const collage_scene *s, float *m, float *v, int32_t *step, void *stream) {
  if (!s) return fail(COLLAGE_ERR_INVALID, "scene is NULL");
  if (!step || (s->N > 0 && (!m || !v))) return fail(COLLAGE_ERR_INVALID, "m, v or step is NULL");
  hipError_t e = launch_adam_reset(m, v, step, s->N, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? COLLAGE_OK : hip_fail(e, "adam reset launch");
}

int collage_graph_launch(collage_graph *g, int32_t count, void *stream) {
  if (!g || count < 0) return fail(COLLAGE_ERR_INVALID, "graph is NULL or count < 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int i = 0; i < count; ++i) {
    hipError_t e = hipGraphLaunch(g->exec, st);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  }
  return COLLAGE_OK;
}

void collage_graph_destroy(collage_graph *g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

}  // extern "C"
