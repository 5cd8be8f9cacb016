// Internal types shared by the HIP kernels and the host side of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "collage.h"

namespace collage {

// One layout of a batch at one level (device copy built at scene creation).
struct alignas(16) LayoutRec {
  int32_t W, H;         // canvas size, level px
  int32_t ntx, nty;     // screen tiles per row / column
  int32_t tile_off;     // first global tile index
  int32_t shape_begin;  // item range [shape_begin, shape_end)
  int32_t shape_end;
  int32_t ptile_off;    // first kPixTile x kPixTile pixel tile of the layout (per-pixel and window passes)
  int64_t pix_off;      // first pixel in packed images
  int64_t list_off;     // first entry of this layout's unit pool (tile lists, unit records, per-item map)
  float k;              // level scale
  int32_t row_off;      // first global tile row of the layout
  int64_t row_list_off; // first entry of this layout's per-row item lists (capacity: items per row)
  int32_t unit_cap;     // units this layout's pool holds
};

// Per item, written by the transform kernel every call.
struct alignas(16) ShapeRec {
  double cx, cy;     // k * t, level px (the item's origin on the canvas), double
  float k;           // level scale of the item's layout
  float s;           // uniform scale parameter
  float orient;      // +1 if the outline is counter-clockwise in (x, y) coordinates, -1 otherwise
  int32_t edge_off;  // first edge record (= first vertex of the item)
  int32_t edge_cnt;  // edges of the item: its vertices (closed), one fewer (open, at least 1)
  int32_t layout;
  int32_t bad;       // 1 if a parameter is not finite (the item is skipped, its gradient is NaN)
  int32_t open;      // 1: open polyline, sd = sw - d; 0: closed outline, sd = +-d (even-odd)
  double sw;         // open: stroke radius k |s| w in level px
  double sw_ds;      // open: d sw / d s = k w sign(s)
  double kc, ks;     // k cos(theta), k sin(theta): k R(theta), for d v' / d s of items with |s| < kScaleFloor
};

// Per item, written by the transform kernel beside its ShapeRec: what binning reads of each candidate
// item, in one 48-byte record (the support box it tests, and the fields of the unit records it writes).
struct alignas(16) BinRec {
  int4 box;        // inclusive pixel box x0, y0, x1, y1 of the coverage support (empty: x1 < x0)
  int32_t eo;      // first edge record (= first vertex)
  int32_t ecnv;    // edges (bits 0-15) and vertices (bits 16-31)
  int32_t flags;   // kUnitOpen, kUnitClockwise
  float s;         // scale parameter
  double cx, cy;   // the item's origin k t, level px
};
static_assert(sizeof(BinRec) == 48, "bin record size");

// One (tile, item) work unit as the persistent passes read it, written by the binning kernel beside the
// unit's list entry: a wave loads one record per unit instead of the list entry and then the item's.
// 48 bytes: the small fields are packed (vertex and edge counts <= 32767, canvas coordinates <= 32767,
// the rectangle's width <= 128 and its pixel count <= 16384: at most one tile).
struct alignas(16) UnitRec {
  int32_t eo;      // the item's first edge record (= first vertex)
  int32_t ecnv;    // edges (bits 0-15) and vertices (bits 16-31) of the item
  int32_t flags;   // kUnitOpen: open polyline; kUnitClockwise: the outline's orientation is clockwise
  int32_t head;    // the unit's entry of the per-item map: where the adjoint's sums go
  int32_t xy;      // the unit rectangle (the item's support box clipped to the tile): x0 | y0 << 16
  int32_t wn;      // its width | its pixel count << 16 (w x n / w px)
  int32_t sid;     // the item (an open item's stroke radius is read from its ShapeRec)
  float s;         // the item's scale parameter
  double cx, cy;   // the item's origin (double; the scan uses it rounded to float)
};
constexpr int32_t kUnitOpen = 1;
constexpr int32_t kUnitClockwise = 2;
static_assert(sizeof(UnitRec) == 48, "unit record size");

// Per edge (a, b) of an item, in level px relative to the item's origin (cx, cy).
// b is stored explicitly so that the half-open crossing test compares every vertex with the same
// float value from both edges that share it.
struct alignas(16) EdgeRec {
  float ax, ay;   // a
  float exs, eys; // (b - a) / |b - a|^2  (0 for a degenerate edge)
  float ex, ey;   // b - a
  float by;       // b.y
  float slope;    // ex / ey (0 when ey = 0: such an edge never crosses a pixel row)
};

// The same edge in double precision: used once per (pixel, item) to evaluate the signed distance
// to the nearest edge found by the float scan, and everything downstream of it.
struct alignas(16) EdgeD {
  double ax, ay;
  double ex, ey;
  double inv_ee;        // 1 / |b - a|^2 (0 for a degenerate edge)
  double inv_len;       // 1 / |b - a| = sqrt(inv_ee) (0 for a degenerate edge): the unit normal's scale
};
// Below this |s| the adjoint takes d v' / d s = k R(theta) v from the item-frame vertices instead of from
// the transformed nearest point divided by s (whose digits cancel as s goes to 0).
constexpr double kScaleFloor = 1e-6;

// Status words at the start of the workspace (COLLAGE_STATUS_* of collage.h), zeroed by the transform
// kernel, which every compute call launches first.
constexpr int kStatusWords = COLLAGE_STATUS_WORDS;
constexpr int kPersistWaves = 4;      // waves per workgroup of the persistent kernels
constexpr int kCoverBlocksPerCU = 6;  // resident workgroups per CU: coverage kernel (7 and 8 measured slower)
constexpr int kAdjointBlocksPerCU = 4;  // and adjoint kernel (5 measured no faster)

// Kernel arguments (one struct, passed by value).
struct KArgs {
  const LayoutRec *layouts;
  int32_t num_layouts;
  int32_t num_shapes;
  int32_t total_tiles;
  int32_t total_ptiles;  // pixel tiles over all layouts
  int32_t tile;          // tile edge in px (8, 16, 32, 64 or 128)
  int32_t bin_chunk;     // items binned per pass
  int32_t *item_base;    // [N] each item's first per-item map entry, -1 when its layout's units did not
                         // fit its pool (written by binning)
  long long *row_base;   // [rows] the layout's units in earlier tile rows, -1 when they do not fit its
                         // pool (written by the row pass)
  int64_t chunk_cap;     // upper bound of the number of 64-pixel chunks of a pass (bounds the code capacity)
  int64_t code_cap;      // 64-pixel chunks whose nearest-edge codes are kept between the coverage and
                         // adjoint passes (the first code_cap chunks of the pass)
  int32_t cover_grid;    // workgroups of the persistent coverage kernel (all resident at once)
  double cover_taper;    // the coverage pass's last wave gets (1 - cover_taper) times the first's share
  int32_t adjoint_grid;  // and of the persistent adjoint kernel
  const int32_t *vert_off;
  const float *verts;
  const float *rho;
  const float *mask;
  const float *stroke;   // [N] stroke half-width (canonical px), or null (every item closed)
  const float *params;
  // transform outputs
  ShapeRec *shapes;
  BinRec *bins;          // [N] support box and unit fields of each item
  EdgeRec *edges;
  EdgeD *edges_d;
  // binning outputs
  int32_t *status;       // [kStatusWords] device status words (workspace offset 0)
  int2 *tile_units;      // [tiles] each tile's units and its first pool entry
  int32_t *tile_list;    // pool: each tile's items, in item order, from its first pool entry on
  int32_t rowbin;        // 1: items are first binned per tile row (k_rowbin), tiles scan their row's list
  int32_t scan_in_cover; // 1: the coverage kernel computes the tile prefixes (no scan launch)
  int32_t total_rows;    // tile rows over all layouts
  int32_t *row_count;    // [rows] items whose support box meets the row band
  int32_t *row_list;     // per layout [tile rows][items]: those items, in item order
  UnitRec *units;        // pool, beside tile_list: each unit's record
  int4 *entry_aux;       // pool, beside tile_list: (64-pixel chunks, coverage cost per chunk,
                         // chunks of the tile's earlier units, coverage cost of the tile's earlier units)
  int2 *tile_cost;       // [tiles] summed coverage cost and chunks of the tile's units
  long long *tile_pre;   // [2][tiles + 1] exclusive prefix sums of the tile costs and of the tile chunks
  uint16_t *codes;       // [code_cap * 64] per chunk and lane: nearest edge (15 bits) | inside << 15
  // accumulators
  unsigned long long *acc;  // [pixels][2] fixed-point S and S_pad (2^-40 units)
  double2 *gbuf;            // [pixels] dLoss/dS, dLoss/dS_pad
  unsigned long long *head;  // [pool][4] per-item map: per item from item_base[item] on, per tile of its
                             // span in row-major order, its unit's adjoint sums (n_x, n_y, theta, scale
                             // terms) in 2^-30 fixed point (zeroed by binning, added by the adjoint)
  double *block_loss;       // per pixel tile: the kLossTerms weighted loss-term sums
  uint8_t *uflags;          // [pixels] bit j: M != 0 and A_j < 1 (the uniform term's active windows)
  unsigned long long *vacc; // [V][2] outline-vertex adjoint sums, level frame, 2^-32 fixed point; null
                            // unless vertex gradients are asked for (the transform kernel zeroes them)
  float *grad_verts_out;    // [V,2] dLoss/d(vertex) in the item frame
  int32_t *step_inc;        // incremented once per epoch by the scan kernel when not null
  // images
  float *cov_out;
  float *cov_pad_out;
  const float *dloss;    // [B,kLossTerms] or null (= 1)
  int32_t write_loss;    // tile loss partials are written (forward and fused calls)
  int32_t keep_codes;    // the coverage pass stores nearest-edge codes (adjoint calls)
  // constants
  float tau, inv_tau, r_cut, r_pad;
  double inv_tau_d;      // 1 / tau
  double log2e_inv_tau;  // log2(e) / tau
  double pad_factor;     // e^(-r_pad / tau)
  float w[9];            // overlap, contain, fill, pad, down, uniform, wmse, centre, objdown
  int32_t area_mean;     // 1: overlap, contain, fill, pad and wmse are divided by the layout's W * H
  // finalize / Adam
  float *loss_out;
  float *grad_out;
  float *param_io;
  float *adam_m;
  float *adam_v;
  const int32_t *step;
  float lr_px, beta1, beta2, eps;
};

// Launchers (collage_kernels.hip).  Each returns hipGetLastError() of its launches.
hipError_t launch_transform(const KArgs &a, hipStream_t st);
hipError_t launch_bin(const KArgs &a, hipStream_t st);  // (with the row pass first when a.rowbin)
hipError_t launch_scan(const KArgs &a, hipStream_t st);
// ev_start / ev_stop (both or neither): HIP events timestamped at the kernel's start and end
hipError_t launch_cover(const KArgs &a, hipStream_t st, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
hipError_t launch_pixel(const KArgs &a, bool grad, hipStream_t st);
hipError_t launch_adjoint(const KArgs &a, hipStream_t st);
// dLoss/d(outline vertices) into a.grad_verts_out (needs a.vacc, zeroed by this call's transform, and
// the codes and dLoss/dS of this call's coverage and per-pixel passes)
hipError_t launch_vertex_grad(const KArgs &a, hipStream_t st);
// the uniform term's share of dLoss/dS, added into gbuf after launch_pixel(grad = true) (nothing is
// launched when its weight is 0)
hipError_t launch_uniform_grad(const KArgs &a, hipStream_t st);
// do_transform: after the update, transform every item with its new parameters (the next epoch of the
// same call then needs no transform launch)
hipError_t launch_finalize(const KArgs &a, bool do_grad, bool do_loss, bool do_adam, hipStream_t st,
                           bool do_transform = false);
hipError_t launch_adam_reset(float *m, float *v, int32_t *step, int num_shapes, hipStream_t st);
hipError_t launch_adam_only(const KArgs &a, hipStream_t st);
// The calling thread's current device's copy of the library's static scratch array (kStaticScratchBytes,
// 256-byte aligned), found with hipGetSymbolAddress on the first request per device and kept.
hipError_t static_scratch(void **out);
constexpr size_t kStaticScratchBytes = COLLAGE_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
hipError_t launch_render(const KArgs &a, int first, int count, float *alpha, float *alpha_pad, int max_pixels,
                         hipStream_t st);

constexpr int kDefaultTile = 16;
constexpr int kDefaultBinChunk = 1024;
constexpr int kMaxBinChunk = 1024;
constexpr int kEdgePad = 4;  // edge records past the last item that the scalar-cache scan may fetch
constexpr int kStageEdges = 128;   // edge records a wave stages in LDS at a time (4 KiB)
constexpr int kScanInCoverTiles = 448;  // up to this many tiles the coverage kernel scans them itself (LDS: 6 resident workgroups per CU)
constexpr int64_t kRowBinTests = 1 << 21;  // box tests (tiles x items) above which the row pass is used
constexpr int kLossTerms = 9;   // overlap, contain, fill, pad, down, uniform, wmse, centre, objdown
constexpr double kWmseIn = 1.0;    // eq. 5 penalty inside the container
constexpr double kWmseOut = 100.0; // and outside
constexpr int kUniWindows = 4;  // window sizes 5 + 6 j of the uniform term
constexpr int kUniHalo = 11;    // largest window radius (2 + 3 (kUniWindows - 1))
constexpr int kPixTile = 32;    // pixel tile edge of the per-pixel and window passes
constexpr int kPixThreads = kPixTile * kPixTile;  // their workgroup: one thread per pixel
constexpr int kEpilogueCost = 32;  // per-pixel work after the scan, in edge evaluations (work partition)
constexpr int kUnitCost = 128;     // per-unit setup (records, edge staging), spread over the unit's chunks
constexpr int kMaxVertsPerItem = 32767;
constexpr double kFixScale = 1099511627776.0;  // 2^40: fixed-point scale of the coverage accumulators
constexpr double kFixInv = 1.0 / 1099511627776.0;
constexpr unsigned long long kFixOne = 1ull << 40;  // 1.0 in that fixed point

}  // namespace collage
