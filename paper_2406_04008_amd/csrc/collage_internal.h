// Internal types shared by the HIP kernels and the host side of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace collage {

// One layout of a batch at one level (device copy built at scene creation).
struct alignas(16) LayoutRec {
  int32_t W, H;         // canvas size, level px
  int32_t ntx, nty;     // screen tiles per row / column
  int32_t tile_off;     // first global tile index
  int32_t shape_begin;  // item range [shape_begin, shape_end)
  int32_t shape_end;
  int32_t pad0;
  int64_t pix_off;      // first pixel in packed images
  int64_t list_off;     // first entry of this layout's per-tile item lists (capacity: items of the layout per tile)
  float k;              // level scale
  float pad1, pad2, pad3;
};

// Per item, written by the transform kernel every call.
struct alignas(16) ShapeRec {
  double cx, cy;     // k * t, level px (the item's origin on the canvas), double
  float cxf, cyf;    // the same, rounded to float for the edge scan
  float k;           // level scale of the item's layout
  float s;           // uniform scale parameter
  float orient;      // +1 if the outline is counter-clockwise in (x, y) coordinates, -1 otherwise
  int32_t edge_off;  // first edge record (= first vertex of the item)
  int32_t edge_cnt;  // edges (= vertices) of the item
  int32_t layout;
  int32_t bad;       // 1 if a parameter is not finite (the item is skipped, its gradient is NaN)
  int32_t pad;
};

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
};

// Kernel arguments (one struct, passed by value).
struct KArgs {
  const LayoutRec *layouts;
  int32_t num_layouts;
  int32_t num_shapes;
  int32_t total_tiles;
  int32_t tile;          // tile edge in px
  int32_t cache_slots;   // on-chip nearest-edge cache depth (fused call)
  int32_t bin_chunk;     // items binned per pass
  const int32_t *vert_off;
  const float *verts;
  const float *rho;
  const float *mask;
  const float *params;
  // transform outputs
  ShapeRec *shapes;
  int4 *bbox;            // inclusive pixel box x0, y0, x1, y1 (empty: x1 < x0)
  EdgeRec *edges;
  EdgeD *edges_d;
  // per-tile outputs
  int32_t *tile_count;
  int32_t *tile_list;
  double4 *tile_partial; // per (tile, slot): sums of the per-pixel adjoint terms (n_x, n_y, theta, scale)
  double *tile_loss;     // per tile: the 5 loss-term sums
  uint32_t *status;
  int32_t *step_inc;     // incremented once by the transform kernel when not null
  // images
  float *cov_out;
  float *cov_pad_out;
  const float *dloss;    // [B,5] or null (= 1)
  int32_t write_loss;    // tile loss partials are written (forward and fused calls)
  // constants
  float tau, inv_tau, r_cut, r_pad;
  float w[5];
  // finalize / Adam
  float *loss_out;
  float *grad_out;
  float *param_io;
  float *adam_m;
  float *adam_v;
  const int32_t *step;
  float lr_px, beta1, beta2, eps;
  // work queue (batched form)
  int32_t *queue_counter;
  const int32_t *queue_order;
  int32_t use_queue;
  int32_t queue_grid;
};



// Launchers (collage_kernels.hip).  Each returns hipGetLastError() of its launches.
hipError_t launch_transform(const KArgs &a, hipStream_t st);
hipError_t launch_tiles(const KArgs &a, bool adjoint, hipStream_t st);
hipError_t launch_finalize(const KArgs &a, bool do_grad, bool do_loss, bool do_adam, hipStream_t st);
hipError_t launch_adam_only(const KArgs &a, hipStream_t st);
hipError_t launch_render(const KArgs &a, int first, int count, const int64_t *out_off_dev, float *alpha,
                         float *alpha_pad, int max_pixels, hipStream_t st);

constexpr int kDefaultTile = 16;
constexpr int kDefaultCacheSlots = 48;
constexpr int kMaxCacheSlots = 64;
constexpr int kDefaultBinChunk = 2048;
constexpr int kMaxBinChunk = 2048;
constexpr int kMaxVertsPerItem = 32767;

}  // namespace collage
