/*
 * collage.h -- C ABI of the MI355X (gfx950) image-space collage hot path.
 *
 * The operations are those of "Image-Space Collage and Packing with Differentiable Rendering"
 * (arXiv 2406.04008):
 *   - the collage problem of Sec. 3 ("Collage Problem"): items G_i with a translation t_i, a rotation
 *     r_i and a scale s_i each, arranged in a container C;
 *   - the per-epoch pipeline of Sec. 4 (Fig. 2): transform every item (eq. 2), rasterize the items
 *     differentiably into a w x h image, evaluate image-space losses against the container image
 *     (eq. 3, Sec. 4.2), back-propagate to (t, r, s) and update them (eq. 4);
 *   - the coarse-to-fine resolution schedule of Sec. 4.3, driven by the caller level by level.
 *
 * Conventions shared by every entry point
 *   - Pixel (i, j), i the column and j the row, has centre (i + 1/2, j + 1/2) in level pixels; y points
 *     down; images are row-major.  A level has scale k (level px per canonical px).
 *   - Item parameters are float32 [N,4] rows (t_x, t_y, theta, s): translation in canonical px,
 *     rotation in radians about the item's local origin, uniform scale.  Transformed vertex:
 *     v' = k * (R(theta) * (s * v) + t).
 *   - Coverage of item i at pixel p: alpha = sigmoid(sd / tau) where sd is the Euclidean signed
 *     distance from p to the item's closed outline (positive inside, even-odd rule), set to 0 once
 *     sd < -r_cut; padded coverage alpha_pad = sigmoid((sd + r_pad) / tau), 0 once sd + r_pad < -r_cut.
 *     S = sum_i alpha_i and S_pad = sum_i alpha_pad_i per pixel of a layout.
 *   - Loss terms per layout, in this order (weighted by the scene's weights):
 *       [0] overlap  w_overlap * sum_p relu(S - 1)^2
 *       [1] contain  w_contain * sum_p S (1 - M)
 *       [2] fill     w_fill    * sum_p M relu(1 - S)^2
 *       [3] pad      w_pad     * sum_p relu(S_pad - 1)^2
 *       [4] down     w_down    * sum_p S (H - y_p)
 *       [5] uniform  w_uniform * sum_j (b_j / 5) sum_p M relu(1 - A_j(p))           (Sec. 4.2, eq. 7)
 *       [6] wmse     w_wmse    * sum_p W(p) (M - min(S, 1))^2                        (Sec. 4.2, eq. 5)
 *       [7] centre   w_centre  * sum_p S |p - c|, c = (W/2, H/2) the canvas centre   (Sec. 5, central force)
 *       [8] objdown  w_objdown * sum_i (H - y_i), y_i = k t_y,i the item's origin   (Sec. 5, downward force
 *                                                                 on the items themselves, object space)
 *     M is the container mask (1 inside), the complement of the paper's container image I_C.  For the
 *     uniform term, b_j = 5 + 6 j (j = 0..3) and A_j(p) is the sum of min(S, 1) over the b_j x b_j
 *     window centred on p, clipped to the canvas: it charges container pixels with no item nearby,
 *     the more the larger the empty window.  Its gradient with respect to S is
 *     -1(S(q) < 1) sum_j (b_j / 5) sum_{p: q in window_j(p)} M(p) 1(A_j(p) < 1) (relu'(0) = 0).  The
 *     window sums are exact integer sums of S in 2^-40 fixed point, so the A_j < 1 decisions depend
 *     only on the accumulated S.  In [6], W(p) = 1 M + 100 (1 - M): the penalty mask of eq. 5 (1 inside
 *     the container, 100 outside) and 1 - min(S, 1) the black-and-white rendering of the items; its
 *     gradient is -2 W (M - S) where S < 1.  With COLLAGE_FLAG_AREA_MEAN, terms [0]-[3] and [6] of a
 *     layout are divided by its W * H (the 1 / (w h) of eqs. 5 and 6).  Terms with weight 0 cost no
 *     reduction and are reported as 0.
 *   - All buffers passed to compute calls are DEVICE memory owned by the caller, float32 unless stated,
 *     contiguous.  Packed images hold the layouts one after another, layout b starting at pixel
 *     sum_{c<b} W_c * H_c.  Calls are asynchronous on `stream` (a hipStream_t; NULL = default stream)
 *     and never synchronize the host.
 *   - Return value: COLLAGE_OK or a negative code; argument errors are detected on the host before any
 *     launch, and collage_last_error() then describes the failure (thread-local).
 *   - Results are deterministic: the same inputs give bitwise the same outputs on the same device.
 *   - Precision: the nearest edge of every (pixel, item) is found by a float32 scan of the item's
 *     edges and re-decided among its neighbours in double precision; the distance to it is evaluated
 *     in double, the coverage alpha, alpha_pad from it in float32 (a few 1e-7), summed exactly in
 *     2^-40 fixed point; the loss sums and the gradient terms are double (the gradient's logistic
 *     factor sigma'(sd / tau) / tau in float32, a relative error of a few 1e-7); outputs are float32.
 */
#ifndef COLLAGE_H_
#define COLLAGE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define COLLAGE_OK 0
#define COLLAGE_ERR_INVALID (-1)     /* null pointer, out-of-range value, inconsistent offsets */
#define COLLAGE_ERR_SIZE (-2)        /* a size or count does not match the scene */
#define COLLAGE_ERR_WORKSPACE (-3)   /* workspace missing or smaller than collage_workspace_size() */
#define COLLAGE_ERR_HIP (-4)         /* a HIP runtime call or kernel launch failed */
#define COLLAGE_ERR_UNSUPPORTED (-5) /* unknown flag or tile size */

/* collage_scene_desc.flags: divide the image-mismatch loss terms by the canvas area (eqs. 5, 6) */
#define COLLAGE_FLAG_AREA_MEAN 1u

/*
 * Device status words: COLLAGE_STATUS_WORDS int32 values at offset 0 of the workspace, zeroed at the
 * start of every call that takes a workspace and written by its kernels (never read by the library).
 *   [COLLAGE_STATUS_NONFINITE]  (epoch, item) pairs of the call whose parameters were not all finite:
 *                               such an item is skipped by the coverage (it covers no pixel) and its
 *                               gradient is NaN.  Counted by every call that evaluates the losses or the
 *                               gradient (not by collage_render_shapes).
 *   [COLLAGE_STATUS_CHUNKS]     64-pixel chunks of (screen tile, item) work in the coverage pass of the
 *                               call's last epoch (the units of work of the rasterization).
 *   [COLLAGE_STATUS_RESCANNED]  of those, the chunks whose nearest edges the adjoint found by scanning
 *                               the edges again, beyond the scene's code capacity (0 without a backward).
 *   [COLLAGE_STATUS_UNIT_OVERFLOW] (epoch, layout) pairs of the call whose work units did not fit the
 *                               layout's unit capacity.  Such a layout lists no units in that epoch: its
 *                               coverage is 0 and its items' gradients are 0, so the call's results are
 *                               not valid and the scene must be created with a larger unit_capacity.
 *   [COLLAGE_STATUS_GRAD_RANGE] pieces of the adjoint (the chunks of one work unit that one wave sums)
 *                               whose gradient sums were not finite or reached 2^23 in magnitude, the
 *                               range of the exact 2^-30 fixed-point sums: they are left out of the
 *                               gradient, so the call's gradients are not valid.
 * The other words are reserved (0).  collage_read_status copies them to the host.
 */
#define COLLAGE_STATUS_NONFINITE 0
#define COLLAGE_STATUS_CHUNKS 1
#define COLLAGE_STATUS_RESCANNED 2
#define COLLAGE_STATUS_UNIT_OVERFLOW 3
#define COLLAGE_STATUS_GRAD_RANGE 4
#define COLLAGE_STATUS_WORDS 8


typedef struct collage_scene collage_scene; /* opaque host handle */

/*
 * Description of a batch of B independent layouts (one level of the schedule).  Host arrays are
 * copied by collage_scene_create; device pointers are borrowed and must stay valid while the scene
 * is used.
 */
typedef struct collage_scene_desc {
  int32_t num_layouts;          /* B >= 1 */
  int32_t num_shapes;           /* N >= 0, items of all layouts */
  int32_t num_verts;            /* V >= 0, outline vertices of all items */
  const int32_t *layout_width;  /* host [B], canvas width in level px, 1..32768 */
  const int32_t *layout_height; /* host [B], canvas height in level px, 1..32768 */
  const float *layout_scale;    /* host [B], k > 0 */
  const int32_t *layout_shapes; /* host [B+1], item ranges: [0] = 0, nondecreasing, [B] = N */
  const int32_t *vert_offset;   /* host [N+1], vertex ranges: [0] = 0, nondecreasing, [N] = V;
                                   at most 32767 vertices per item */
  const float *verts;           /* device [V,2], outlines in the item frame (canonical px); for a
                                   closed item edge m joins vertex m and vertex m+1 (the last joins
                                   the first), for an open item only consecutive vertices are joined */
  const float *rho;             /* device [N], rim radius of each item (canonical px); used only by
                                   the update (rotation and scale learning rates); may be NULL */
  const float *mask;            /* device, packed [sum W*H] container masks in [0, 1] */
  const float *stroke;          /* device [N], stroke half-width w of each item (canonical px): 0 for
                                   a closed outline (signed distance positive inside, even-odd rule),
                                   > 0 for an open polyline thickened by a disk of radius w and
                                   transformed with the item (signed distance k |s| w - d); NULL =
                                   every item closed */
  float tau;                    /* sigmoid temperature, level px, > 0 */
  float r_cut;                  /* coverage cut-off, level px, >= 0 */
  float r_pad;                  /* padding offset, level px, >= 0 */
  float w_overlap, w_contain, w_fill, w_pad, w_down; /* loss weights, finite */
  float w_uniform;              /* weight of the uniform term, finite; 0 = the term is skipped (no
                                   launches) and reported as 0 */
  float w_wmse, w_centre, w_objdown; /* weights of terms [6]-[8], finite */
  int32_t tile;                 /* screen tile edge in px: 8, 16, 32, 64 or 128; 0 = default (16) */
  int32_t code_capacity;        /* 64-pixel chunks of (tile, item) work whose nearest-edge codes (2 bytes
                                   per pixel) are kept between the coverage and adjoint passes; the
                                   adjoint rescans the edges of later chunks.  -1 = default (four
                                   items per pixel on average, at least 65536 chunks); 0 = always
                                   rescan */
  int32_t bin_chunk;            /* 0..1024, accepted and not used: binning tests each candidate item once and
                                   writes its unit from the testing thread, with no item list in LDS */
  uint32_t flags;               /* 0 or COLLAGE_FLAG_AREA_MEAN; other bits are rejected */
  int32_t unit_capacity;        /* (screen tile, item) work units the workspace holds per layout and epoch,
                                   one per item and tile its support box meets (100 bytes each).
                                   0 = default: every item in every tile of the layout, or, when less, four
                                   times the units of its items at twice their rim radius (read from verts
                                   and stroke at creation), at least 65536; -1 = every item in every tile
                                   (never overflows); > 0 = that many (at most every item in every tile).
                                   An epoch in which a layout needs more is counted in
                                   COLLAGE_STATUS_UNIT_OVERFLOW; -2 and below are rejected */
} collage_scene_desc;

/*
 * The collage problem of Sec. 3 ("Collage Problem") at one level of the schedule of Sec. 4.3: B
 * containers C_b, each with its items G_i (outlines in their own frames, vertex arrays), the level
 * scale k_b, and the loss constants of Sec. 4.2.  Validates `desc` (COLLAGE_ERR_INVALID,
 * COLLAGE_ERR_SIZE or COLLAGE_ERR_UNSUPPORTED, nothing allocated), copies its host arrays and
 * allocates the scene's two small device tables (layout records, vertex offsets: the only device
 * memory the library allocates, COLLAGE_ERR_HIP if that fails).  On success *out owns them until
 * collage_scene_destroy (NULL is ignored).  Device pointers of `desc` stay borrowed.
 */
int collage_scene_create(const collage_scene_desc *desc, collage_scene **out);
void collage_scene_destroy(collage_scene *scene);

/*
 * Bytes of device workspace the compute calls need for this scene: the per-epoch intermediates of
 * Fig. 2 (transformed edges of eq. 2, per-tile item lists, the coverage sums S and S_pad, dLoss/dS, the
 * adjoint partials) and the status words at offset 0.  The caller allocates it (256-byte aligned) and
 * owns it; calls on one workspace must not overlap.  COLLAGE_ERR_INVALID for NULL arguments.
 */
int collage_workspace_size(const collage_scene *scene, size_t *bytes);

/* Copies the COLLAGE_STATUS_WORDS status words of `workspace` to the host array `status`, after the work
 * queued on `stream` (this call waits for the stream).  COLLAGE_ERR_INVALID for NULL arguments,
 * COLLAGE_ERR_WORKSPACE for a workspace smaller than the scene's, COLLAGE_ERR_HIP if the copy fails. */
int collage_read_status(const collage_scene *scene, const void *workspace, size_t workspace_bytes, int32_t *status,
                        void *stream);

/* Number of pixels over all layouts (length of packed images) and of screen tiles. */
int collage_scene_info(const collage_scene *scene, int64_t *num_pixels, int64_t *num_tiles);

/*
 * Forward pass (Sec. 4, eqs. 2-3): coverage sums and the weighted loss terms.
 *   params  [N,4]        item parameters
 *   cov     [pixels]     S, written (may be NULL)
 *   cov_pad [pixels]     S_pad, written (may be NULL)
 *   loss    [B,9]        weighted loss terms, written
 */
int collage_forward(const collage_scene *scene, const float *params, float *cov, float *cov_pad, float *loss,
                    void *workspace, size_t workspace_bytes, void *stream);

/*
 * Backward pass (the gradient used by eq. 4): d(sum_b sum_t dloss[b,t] * loss[b,t]) / d params.
 * Recomputes the coverage and every pixel's nearest edge from params (no per-pixel, per-item
 * intermediates are stored between calls, and no image from the forward pass is needed).
 *   dloss [B,9]  upstream gradient of each loss term
 *   grad  [N,4]  overwritten
 */
int collage_backward(const collage_scene *scene, const float *params, const float *dloss, float *grad,
                     void *workspace, size_t workspace_bytes, void *stream);

/*
 * Gradient with respect to the outline vertices (Sec. 3 "Vector Representation": the items' control
 * points are fitted to their silhouettes by differentiable rendering), together with the parameter
 * gradient of collage_backward.  Each pixel's signed distance moves with the two end points of its
 * nearest edge (weights 1 - u and u of the nearest point); the sums go back through eq. 2
 * (dv'/dv = k s R(theta)).  Term [8] does not depend on the vertices.
 *   dloss      [B,9]  upstream gradient of each loss term
 *   grad       [N,4]  overwritten, or NULL (then only the vertex gradient is computed)
 *   grad_verts [V,2]  overwritten: dLoss/d(vertex) in the item frame, canonical px; NaN for the
 *                     vertices of an item with a non-finite parameter
 * The vertex sums are accumulated in 2^-32 fixed point (deterministic; a sum must stay below 2^31 in
 * magnitude).
 */
int collage_backward_vertices(const collage_scene *scene, const float *params, const float *dloss, float *grad,
                              float *grad_verts, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Forward and backward of the total loss sum_b sum_t loss[b,t] in one pass over the pixels
 * (dloss = 1).  Outputs as in collage_forward plus grad [N,4] (overwritten).
 */
int collage_forward_backward(const collage_scene *scene, const float *params, float *cov, float *cov_pad,
                             float *loss, float *grad, void *workspace, size_t workspace_bytes, void *stream);

/*
 * collage_forward_backward for callers that cannot allocate device memory (code under hipGraph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same computation and outputs, with the
 * library's own static scratch (COLLAGE_STATIC_SCRATCH_BYTES, 256-byte aligned, one copy per GPU, held
 * from the library's first use on that GPU until the process ends) in place of a workspace.  No
 * device memory is allocated or freed.  The first call on a device looks up that device's copy
 * (hipGetSymbolAddress); later calls reuse it.  Every call on a GPU shares its scratch: calls that
 * overlap on one GPU (other streams, other threads) race and give undefined results; the scratch keeps
 * the last call's contents, and every call initializes what it reads.
 * Errors: those of collage_forward_backward, and COLLAGE_ERR_WORKSPACE (checked before any launch) when
 * collage_workspace_size of the scene exceeds COLLAGE_STATIC_SCRATCH_BYTES.
 */
#define COLLAGE_STATIC_SCRATCH_BYTES (64u << 20)
int collage_forward_backward_static(const collage_scene *scene, const float *params, float *cov, float *cov_pad,
                                    float *loss, float *grad, void *stream);

/*
 * Adam update of the parameters (eq. 4 with Adam moments, bias-corrected, no weight decay).
 * step is a device int32 counter: this call uses t = *step + 1 and stores it back.  Learning rates:
 * lr_px / k for t_x, t_y (lr_px level px per step); lr_px / (k * rho_i) for theta and s (the item's
 * rim moves by lr_px level px).  m, v [N,4] are the moment buffers (zero before the first step).
 */
int collage_step(const collage_scene *scene, float *params, const float *grad, float *m, float *v, int32_t *step,
                 float lr_px, float beta1, float beta2, float eps, void *stream);

/*
 * One optimization epoch of Fig. 2: forward, loss, backward and the Adam update of collage_step,
 * in kernel launches with fixed grids (safe to capture in a hipGraph and replay).
 * cov / cov_pad may be NULL.  loss [B,9] and grad [N,4] receive this epoch's values (before the update).
 */
int collage_iterate(const collage_scene *scene, float *params, float *cov, float *cov_pad, float *loss, float *grad,
                    float *m, float *v, int32_t *step, float lr_px, float beta1, float beta2, float eps,
                    void *workspace, size_t workspace_bytes, void *stream);

/*
 * Per-item coverage images of the differentiable rasterization (Sec. 3 "Differentiable Rendering"; the
 * alpha of the conventions above) for items [first, first + count): alpha and (optionally) alpha_pad,
 * each image the size of the item's layout canvas (row-major), written one after another.  For tests
 * and small scenes: the losses themselves never need per-item images.  COLLAGE_ERR_SIZE for a range
 * outside [0, N) or more than 65535 items, COLLAGE_ERR_INVALID for NULL params or alpha.
 */
int collage_render_shapes(const collage_scene *scene, const float *params, int32_t first, int32_t count, float *alpha,
                          float *alpha_pad, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Event timer: `count` pairs of HIP events (timing enabled).  collage_iterate_n timestamps the coverage
 * kernel of epochs 0, d, 2d, ... with d = ceil(epochs / count): every epoch when count >= epochs, else a
 * spread sample (each stamped launch costs a few microseconds of stream time, so a sample keeps the
 * timed work close to an untimed call).  collage_timer_elapsed waits for the events and writes `count`
 * durations in milliseconds: those of the pairs the last collage_iterate_n call recorded, then NaN.
 */
typedef struct collage_timer collage_timer;
int collage_timer_create(int32_t count, collage_timer **out);
int collage_timer_elapsed(collage_timer *timer, float *ms);
void collage_timer_destroy(collage_timer *timer);

/*
 * `epochs` (1..65536) consecutive collage_iterate epochs in one call, on `stream`.  Equivalent to that
 * many collage_iterate calls; loss, grad and the optional images are those of the last epoch.  Within
 * the call, the update of each epoch also transforms the items for the next one (one launch fewer per
 * epoch).  With a non-NULL `timer` of c pairs, pair j is timestamped with the start and the end of the
 * coverage kernel of epoch j d, d = ceil(epochs / c).  Errors: those of collage_iterate.
 */
int collage_iterate_n(const collage_scene *scene, float *params, float *cov, float *cov_pad, float *loss, float *grad,
                      float *m, float *v, int32_t *step, float lr_px, float beta1, float beta2, float eps,
                      void *workspace, size_t workspace_bytes, int32_t epochs, collage_timer *timer, void *stream);

/*
 * Start of a level of the coarse-to-fine schedule (Sec. 4.3; the optimizer state is not carried
 * across levels, since the loss changes scale with the pixel count): zeroes m[N,4], v[N,4] and the
 * device step counter with a kernel on `stream`.  Returns COLLAGE_ERR_INVALID for NULL buffers.
 */
int collage_adam_reset(const collage_scene *scene, float *m, float *v, int32_t *step, void *stream);

/* graph_flags of collage_graph_create */
#define COLLAGE_GRAPH_RESET_ADAM 1u /* the graph begins with collage_adam_reset */

/*
 * hipGraph of `replays_per_launch` (1..4096) consecutive collage_iterate epochs captured on `stream`
 * (which must not be the NULL stream), preceded by the Adam reset when graph_flags has
 * COLLAGE_GRAPH_RESET_ADAM: one launch of such a graph runs a whole level of the coarse-to-fine
 * schedule.  The graph keeps the buffer addresses it was captured with; the caller keeps them alive and
 * unmoved while the graph exists.  collage_graph_launch replays it `count` times on `stream`.
 * Unknown graph flags give COLLAGE_ERR_UNSUPPORTED; argument errors are those of collage_iterate.
 */
typedef struct collage_graph collage_graph;
int collage_graph_create(const collage_scene *scene, float *params, float *cov, float *cov_pad, float *loss,
                         float *grad, float *m, float *v, int32_t *step, float lr_px, float beta1, float beta2,
                         float eps, void *workspace, size_t workspace_bytes, int32_t replays_per_launch,
                         uint32_t graph_flags, void *stream, collage_graph **out);
int collage_graph_launch(collage_graph *graph, int32_t count, void *stream);
void collage_graph_destroy(collage_graph *graph);

/* Thread-local description of the last non-zero return on this thread. */
const char *collage_last_error(void);

/* Library version string. */
const char *collage_version(void);

#ifdef __cplusplus
}
#endif

#endif /* COLLAGE_H_ */
