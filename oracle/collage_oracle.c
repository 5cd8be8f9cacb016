/*
 * collage_oracle.c -- plain FP64 CPU oracle of the image-space collage hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or helper with the HIP path.
 *
 * What it computes, for every layout b of a batch and every pixel centre p = (i + 1/2, j + 1/2)
 * (level pixels, y down), following the paper:
 *
 *   - Rigid transform of each item (Sec. 4, eq. 2 with a uniform scale as in Sec. 5 "Data
 *     Visualization"):  v' = k * (R(theta) * (s * v) + t), k = level scale, rotation about the item's
 *     area centroid (the local origin).
 *   - Soft rasterization (Sec. 3 "Differentiable Rendering": an anti-aliased, continuous scene
 *     function).  Reading used here: per item a coverage alpha = sigmoid(sd / tau), where sd is the
 *     Euclidean signed distance to the closed outline (positive inside by the even-odd rule), with a
 *     hard zero once sd < -r_cut; a padded coverage alpha_pad = sigmoid((sd + r_pad) / tau) with the
 *     same cut-off on sd + r_pad.  S = sum_i alpha_i, S_pad = sum_i alpha_pad_i.
 *     An open item (stroke half-width w > 0) is the polyline through its vertices (no closing
 *     segment) thickened by a disk of radius w, transformed with the item: sd = k |s| w - d, where d
 *     is the distance to the polyline.
 *   - Image-space losses (Sec. 4.2, eqs. for containment and non-overlap, in their differentiable
 *     reading) plus padding and the downward force of Sec. 5 ("Force Attraction"):
 *        L_ov   = sum_p relu(S - 1)^2           L_cont = sum_p S (1 - M)
 *        L_fill = sum_p M relu(1 - S)^2         L_pad  = sum_p relu(S_pad - 1)^2
 *        L_down = sum_p S (H - y_p)
 *     and the uniform loss of Sec. 4.2 (eq. 7), read as: O = min(S, 1); for bandwidths
 *     b_j = 5 + 6 j (j < NUNI), A_j(p) = sum of O over the b_j x b_j window centred on p (clipped to
 *     the canvas);  L_unif = sum_j (b_j / b_0) sum_p M(p) relu(1 - A_j(p))  -- container pixels with
 *     no item within the window, larger windows weighted more;
 *     the weighted mean square error of Sec. 4.2 (eq. 5) between the black-and-white rendering
 *     1 - O and the container image 1 - M, with penalty 1 inside the container and 100 outside:
 *        L_wmse = sum_p W(p) (M - O)^2,  W = WMSE_IN M + WMSE_OUT (1 - M);
 *     and the force terms of Sec. 5 ("Force Attraction"): a central force towards the canvas centre c,
 *        L_centre = sum_p S |p - c|,
 *     and a downward force on the items themselves (object space), with y_i = k t_y,i the item origin,
 *        L_objdown = sum_i (H - y_i).
 *     reported weighted: loss[b][term] = w_term * L_term (NTERMS terms per layout); with area_mean the
 *     image-mismatch terms (overlap, contain, fill, pad, wmse) are divided by W * H, the 1 / (w h) of
 *     eqs. 5 and 6.
 *   - The gradient of sum_b sum_term dloss[b][term] * loss[b][term] with respect to every item's
 *     (t_x, t_y, theta, s) (Sec. 4, eq. 4 needs dL/dt, dL/dr, dL/ds), by the chain rule through the
 *     two end points of each pixel's nearest edge and then through eq. 2.
 *   - Adam on those gradients (the update of eq. 4 with Adam's moment estimates).
 *
 * All arithmetic is double precision; inputs are float32 values widened exactly.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define NTERMS 9 /* loss terms per layout */
#define WMSE_IN 1.0    /* eq. 5 penalty inside the container */
#define WMSE_OUT 100.0 /* and outside */
#define NUNI 4   /* window sizes of the uniform loss */

static int uni_radius(int j) { return 2 + 3 * j; }                     /* window (2 r + 1) = 5 + 6 j */
static double uni_weight(int j) { return (5.0 + 6.0 * j) / 5.0; }     /* b_j / b_0 */

typedef struct {
  int32_t B;                /* layouts */
  int32_t N;                /* items (all layouts) */
  int32_t V;                /* outline vertices (all items) */
  const int32_t *width;     /* [B] canvas width, level px */
  const int32_t *height;    /* [B] canvas height, level px */
  const double *scale;      /* [B] k */
  const int32_t *shape_off; /* [B+1] item ranges */
  const int32_t *vert_off;  /* [N+1] vertex ranges */
  const double *verts;      /* [V*2] local frame, canonical px */
  const double *mask;       /* packed masks, layout b at pixel offset sum_{c<b} W_c*H_c */
  double tau, r_cut, r_pad;
  double w[9];              /* overlap, contain, fill, pad, down, uniform, wmse, centre, objdown */
  int32_t use_cutoff;       /* 1: hard zero below -r_cut (the definition); 0: no cut-off */
  int32_t use_bbox;         /* 1: skip pixels provably beyond the cut-off support (needs use_cutoff) */
  const double *stroke;     /* [N] stroke half-width, canonical px (> 0: open polyline), or NULL */
  int32_t area_mean;        /* 1: overlap, contain, fill, pad and wmse are divided by W * H */
} oracle_scene;

/* 1 / (W H) for the image-mismatch terms when area_mean is set, else 1. */
static double term_norm(const oracle_scene *sc, int b, int t) {
  if (!sc->area_mean) return 1.0;
  if (t == 0 || t == 1 || t == 2 || t == 3 || t == 6) return 1.0 / ((double)sc->width[b] * sc->height[b]);
  return 1.0;
}

static int64_t pixel_offset(const oracle_scene *sc, int b) {
  int64_t off = 0;
  for (int c = 0; c < b; ++c) off += (int64_t)sc->width[c] * sc->height[c];
  return off;
}

static int layout_of(const oracle_scene *sc, int i) {
  for (int b = 0; b < sc->B; ++b)
    if (i >= sc->shape_off[b] && i < sc->shape_off[b + 1]) return b;
  return -1;
}

/* eq. 2: transformed vertices of item i in level pixels. */
static void transform_item(const oracle_scene *sc, const double *params, int i, double k, double *out) {
  const double tx = params[4 * i + 0], ty = params[4 * i + 1];
  const double th = params[4 * i + 2], s = params[4 * i + 3];
  const double c = cos(th), sn = sin(th);
  for (int m = sc->vert_off[i]; m < sc->vert_off[i + 1]; ++m) {
    const double x = s * sc->verts[2 * m], y = s * sc->verts[2 * m + 1];
    out[2 * (m - sc->vert_off[i]) + 0] = k * (c * x - sn * y + tx);
    out[2 * (m - sc->vert_off[i]) + 1] = k * (sn * x + c * y + ty);
  }
}

typedef struct {
  double sd;     /* signed distance, + inside */
  double d;      /* unsigned distance */
  int edge;      /* nearest edge (lowest index on exact ties) */
  double u;      /* clamped parameter of the nearest point on that edge */
  double qx, qy; /* nearest point */
  int inside;
} sd_result;

/* Euclidean distance to the closed polygon and even-odd inside test with the half-open rule. */
static sd_result signed_distance(double px, double py, const double *P, int n) {
  sd_result r;
  double best = INFINITY;
  int best_m = 0;
  double best_u = 0.0;
  int inside = 0;
  for (int m = 0; m < n; ++m) {
    const double ax = P[2 * m], ay = P[2 * m + 1];
    const int mn = (m + 1 == n) ? 0 : m + 1;
    const double bx = P[2 * mn], by = P[2 * mn + 1];
    const double ex = bx - ax, ey = by - ay;
    const double ee = ex * ex + ey * ey;
    double u = 0.0;
    if (ee > 0.0) {
      u = ((px - ax) * ex + (py - ay) * ey) / ee;
      if (u < 0.0) u = 0.0;
      if (u > 1.0) u = 1.0;
    }
    const double qx = ax + u * ex, qy = ay + u * ey;
    const double d2 = (px - qx) * (px - qx) + (py - qy) * (py - qy);
    if (d2 < best) {
      best = d2;
      best_m = m;
      best_u = u;
    }
    if ((ay > py) != (by > py)) {
      const double xc = ax + (py - ay) * ex / ey;
      if (px < xc) inside = !inside;
    }
  }
  r.d = sqrt(best);
  r.sd = inside ? r.d : -r.d;
  r.edge = best_m;
  r.u = best_u;
  {
    const double ax = P[2 * best_m], ay = P[2 * best_m + 1];
    const int mn = (best_m + 1 == n) ? 0 : best_m + 1;
    r.qx = ax + best_u * (P[2 * mn] - ax);
    r.qy = ay + best_u * (P[2 * mn + 1] - ay);
  }
  r.inside = inside;
  return r;
}

/* Euclidean distance to the open polyline P[0], ..., P[n-1] (segments m -> m + 1; one point if n = 1). */
static sd_result polyline_distance(double px, double py, const double *P, int n) {
  sd_result r;
  double best = INFINITY;
  int best_m = 0;
  double best_u = 0.0;
  const int ns = n > 1 ? n - 1 : 1;
  for (int m = 0; m < ns; ++m) {
    const double ax = P[2 * m], ay = P[2 * m + 1];
    const int mn = n > 1 ? m + 1 : m;
    const double ex = P[2 * mn] - ax, ey = P[2 * mn + 1] - ay;
    const double ee = ex * ex + ey * ey;
    double u = 0.0;
    if (ee > 0.0) {
      u = ((px - ax) * ex + (py - ay) * ey) / ee;
      if (u < 0.0) u = 0.0;
      if (u > 1.0) u = 1.0;
    }
    const double qx = ax + u * ex, qy = ay + u * ey;
    const double d2 = (px - qx) * (px - qx) + (py - qy) * (py - qy);
    if (d2 < best) {
      best = d2;
      best_m = m;
      best_u = u;
      r.qx = qx;
      r.qy = qy;
    }
  }
  r.d = sqrt(best);
  r.sd = -r.d;
  r.edge = best_m;
  r.u = best_u;
  r.inside = 0;
  return r;
}

static int is_open(const oracle_scene *sc, int q) { return sc->stroke && sc->stroke[q] > 0.0; }

/* Stroke radius of item q in level px: the half-width transformed with the item, k |s| w. */
static double stroke_radius(const oracle_scene *sc, const double *params, int q, double k) {
  return is_open(sc, q) ? k * fabs(params[4 * q + 3]) * sc->stroke[q] : 0.0;
}

/* Signed distance of pixel (px, py) for item q with transformed vertices P (n of them). */
static sd_result item_distance(const oracle_scene *sc, const double *params, int q, double k, double px, double py,
                               const double *P, int n) {
  if (!is_open(sc, q)) return signed_distance(px, py, P, n);
  sd_result r = polyline_distance(px, py, P, n);
  r.sd = stroke_radius(sc, params, q, k) - r.d;
  return r;
}

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* Derivative of the logistic function, sigma'(x) = sigma(x) (1 - sigma(x)), written as
 * e^-|x| / (1 + e^-|x|)^2 (the same function; no cancellation when sigma(x) is close to 1). */
static double sigmoid_prime(double x) {
  const double t = exp(-fabs(x));
  return t / ((1.0 + t) * (1.0 + t));
}

/* Coverage of one item at one pixel and its derivative with respect to sd. */
static void coverage(const oracle_scene *sc, double sd, double *a, double *da, double *ap, double *dap) {
  const double x = sd / sc->tau, xp = (sd + sc->r_pad) / sc->tau;
  if (sc->use_cutoff && sd < -sc->r_cut) {
    *a = 0.0;
    *da = 0.0;
  } else {
    *a = sigmoid(x);
    *da = sigmoid_prime(x) / sc->tau;
  }
  if (sc->use_cutoff && sd + sc->r_pad < -sc->r_cut) {
    *ap = 0.0;
    *dap = 0.0;
  } else {
    *ap = sigmoid(xp);
    *dap = sigmoid_prime(xp) / sc->tau;
  }
}

/* Pixel index range that can receive non-zero coverage from polygon P (cut-off on), inclusive. */
static void support_box(const oracle_scene *sc, const double *P, int n, double extra, int W, int H, int *x0, int *y0,
                        int *x1, int *y1) {
  double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
  for (int m = 0; m < n; ++m) {
    if (P[2 * m] < mnx) mnx = P[2 * m];
    if (P[2 * m] > mxx) mxx = P[2 * m];
    if (P[2 * m + 1] < mny) mny = P[2 * m + 1];
    if (P[2 * m + 1] > mxy) mxy = P[2 * m + 1];
  }
  const double ext = sc->r_cut + (sc->r_pad > 0.0 ? sc->r_pad : 0.0) + extra + 1.0;
  double fx0 = floor(mnx - ext - 0.5), fx1 = ceil(mxx + ext - 0.5);
  double fy0 = floor(mny - ext - 0.5), fy1 = ceil(mxy + ext - 0.5);
  if (fx0 < 0) fx0 = 0;
  if (fy0 < 0) fy0 = 0;
  if (fx1 > W - 1) fx1 = W - 1;
  if (fy1 > H - 1) fy1 = H - 1;
  if (!(fx0 <= fx1) || !(fy0 <= fy1) || n == 0) {
    *x0 = 1;
    *x1 = 0;
    *y0 = 1;
    *y1 = 0;
    return;
  }
  *x0 = (int)fx0;
  *x1 = (int)fx1;
  *y0 = (int)fy0;
  *y1 = (int)fy1;
}

typedef struct {
  double *P;             /* transformed vertices of all items, [V*2] */
  int *box;              /* [N*4] x0, y0, x1, y1 */
  const double *params;  /* [N*4] the parameters they were transformed with */
} prepared;

static void prepare(const oracle_scene *sc, const double *params, prepared *pr) {
  pr->params = params;
  pr->P = (double *)malloc(sizeof(double) * 2 * (sc->V > 0 ? sc->V : 1));
  pr->box = (int *)malloc(sizeof(int) * 4 * (sc->N > 0 ? sc->N : 1));
  for (int b = 0; b < sc->B; ++b) {
    for (int i = sc->shape_off[b]; i < sc->shape_off[b + 1]; ++i) {
      const int n = sc->vert_off[i + 1] - sc->vert_off[i];
      double *P = pr->P + 2 * sc->vert_off[i];
      transform_item(sc, params, i, sc->scale[b], P);
      if (sc->use_bbox && sc->use_cutoff) {
        support_box(sc, P, n, stroke_radius(sc, params, i, sc->scale[b]), sc->width[b], sc->height[b],
                    &pr->box[4 * i], &pr->box[4 * i + 1], &pr->box[4 * i + 2], &pr->box[4 * i + 3]);
      } else {
        pr->box[4 * i] = 0;
        pr->box[4 * i + 1] = 0;
        pr->box[4 * i + 2] = sc->width[b] - 1;
        pr->box[4 * i + 3] = sc->height[b] - 1;
      }
    }
  }
}

static void release(prepared *pr) {
  free(pr->P);
  free(pr->box);
}

static int in_box(const int *bx, int i, int j) { return i >= bx[0] && i <= bx[2] && j >= bx[1] && j <= bx[3]; }

/* A_j(p): sum of min(S, 1) over the window of radius r around pixel (i, j), clipped to the canvas. */
static double window_occupancy(const double *S, int W, int H, int i, int j, int r) {
  double a = 0.0;
  for (int y = j - r; y <= j + r; ++y) {
    if (y < 0 || y >= H) continue;
    for (int x = i - r; x <= i + r; ++x) {
      if (x < 0 || x >= W) continue;
      const double s = S[(int64_t)y * W + x];
      a += s < 1.0 ? s : 1.0;
    }
  }
  return a;
}

/* Unweighted uniform loss of layout b with coverage sums S (the layout's own image). */
static double uniform_loss(const oracle_scene *sc, int b, const double *S) {
  const int W = sc->width[b], H = sc->height[b];
  const double *M = sc->mask ? sc->mask + pixel_offset(sc, b) : NULL;
  double tot = 0.0;
  for (int q = 0; q < NUNI; ++q) {
    double *rows = (double *)calloc((size_t)(H > 0 ? H : 1), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int j = 0; j < H; ++j) {
      double acc = 0.0;
      for (int i = 0; i < W; ++i) {
        const double m = M ? M[(int64_t)j * W + i] : 0.0;
        if (m == 0.0) continue;
        const double a = window_occupancy(S, W, H, i, j, uni_radius(q));
        if (a < 1.0) acc += m * (1.0 - a);
      }
      rows[j] = acc;
    }
    double t = 0.0;
    for (int j = 0; j < H; ++j) t += rows[j];
    free(rows);
    tot += uni_weight(q) * t;
  }
  return tot;
}

/* dL_unif/dS of layout b, added (times c) into G: at pixel q,
 *   -1(S(q) < 1) sum_j (b_j / b_0) sum over pixels p whose window contains q of M(p) 1(A_j(p) < 1). */
static void uniform_grad(const oracle_scene *sc, int b, const double *S, double c, double *G) {
  const int W = sc->width[b], H = sc->height[b];
  const double *M = sc->mask ? sc->mask + pixel_offset(sc, b) : NULL;
  if (!M || c == 0.0) return;
  double *F = (double *)malloc(sizeof(double) * (size_t)W * H);
  for (int q = 0; q < NUNI; ++q) {
    const int r = uni_radius(q);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < H; ++j)
      for (int i = 0; i < W; ++i) {
        const double m = M[(int64_t)j * W + i];
        F[(int64_t)j * W + i] = (m != 0.0 && window_occupancy(S, W, H, i, j, r) < 1.0) ? m : 0.0;
      }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < H; ++j)
      for (int i = 0; i < W; ++i) {
        if (!(S[(int64_t)j * W + i] < 1.0)) continue;
        double f = 0.0;  /* the window is symmetric: p's window contains q iff q's contains p */
        for (int y = j - r; y <= j + r; ++y) {
          if (y < 0 || y >= H) continue;
          for (int x = i - r; x <= i + r; ++x)
            if (x >= 0 && x < W) f += F[(int64_t)y * W + x];
        }
        G[(int64_t)j * W + i] -= c * uni_weight(q) * f;
      }
  }
  free(F);
}

/* S and S_pad for all layouts (packed), and the weighted loss terms [B*NTERMS]. */
static void forward_impl(const oracle_scene *sc, const prepared *pr, double *S, double *Sp, double *loss) {
  for (int b = 0; b < sc->B; ++b) {
    const int W = sc->width[b], H = sc->height[b];
    const int64_t off = pixel_offset(sc, b);
    /* per-row partial sums, added in row order afterwards, so the result does not depend on threads */
    double *rows = (double *)calloc((size_t)7 * (H > 0 ? H : 1), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int j = 0; j < H; ++j) {
      double lo = 0, lc = 0, lf = 0, lp = 0, ld = 0, lw = 0, lcen = 0;
      for (int i = 0; i < W; ++i) {
        const double px = i + 0.5, py = j + 0.5;
        double s = 0.0, spad = 0.0;
        for (int q = sc->shape_off[b]; q < sc->shape_off[b + 1]; ++q) {
          if (!in_box(pr->box + 4 * q, i, j)) continue;
          const int n = sc->vert_off[q + 1] - sc->vert_off[q];
          if (n == 0) continue;
          const sd_result r = item_distance(sc, pr->params, q, sc->scale[b], px, py, pr->P + 2 * sc->vert_off[q], n);
          double a, da, ap, dap;
          coverage(sc, r.sd, &a, &da, &ap, &dap);
          s += a;
          spad += ap;
        }
        const int64_t idx = off + (int64_t)j * W + i;
        if (S) S[idx] = s;
        if (Sp) Sp[idx] = spad;
        const double M = sc->mask ? sc->mask[idx] : 0.0;
        const double ov = s > 1.0 ? s - 1.0 : 0.0;
        const double un = s < 1.0 ? 1.0 - s : 0.0;
        const double pv = spad > 1.0 ? spad - 1.0 : 0.0;
        lo += ov * ov;
        lc += s * (1.0 - M);
        lf += M * un * un;
        lp += pv * pv;
        ld += s * (H - py);
        const double O = s < 1.0 ? s : 1.0;
        const double Wp = WMSE_IN * M + WMSE_OUT * (1.0 - M);
        lw += Wp * (M - O) * (M - O);
        const double cx = px - 0.5 * W, cy = py - 0.5 * H;
        lcen += s * sqrt(cx * cx + cy * cy);
      }
      rows[7 * j + 0] = lo;
      rows[7 * j + 1] = lc;
      rows[7 * j + 2] = lf;
      rows[7 * j + 3] = lp;
      rows[7 * j + 4] = ld;
      rows[7 * j + 5] = lw;
      rows[7 * j + 6] = lcen;
    }
    double lo = 0, lc = 0, lf = 0, lp = 0, ld = 0, lw = 0, lcen = 0;
    for (int j = 0; j < H; ++j) {
      lo += rows[7 * j + 0];
      lc += rows[7 * j + 1];
      lf += rows[7 * j + 2];
      lp += rows[7 * j + 3];
      ld += rows[7 * j + 4];
      lw += rows[7 * j + 5];
      lcen += rows[7 * j + 6];
    }
    free(rows);
    if (loss) {
      /* object-space downward force: the item origins' heights above the bottom edge */
      double lod = 0.0;
      for (int q = sc->shape_off[b]; q < sc->shape_off[b + 1]; ++q) lod += H - sc->scale[b] * pr->params[4 * q + 1];
      loss[NTERMS * b + 0] = sc->w[0] * term_norm(sc, b, 0) * lo;
      loss[NTERMS * b + 1] = sc->w[1] * term_norm(sc, b, 1) * lc;
      loss[NTERMS * b + 2] = sc->w[2] * term_norm(sc, b, 2) * lf;
      loss[NTERMS * b + 3] = sc->w[3] * term_norm(sc, b, 3) * lp;
      loss[NTERMS * b + 4] = sc->w[4] * ld;
      loss[NTERMS * b + 5] = sc->w[5] != 0.0 && S ? sc->w[5] * uniform_loss(sc, b, S + off) : 0.0;
      loss[NTERMS * b + 6] = sc->w[6] * term_norm(sc, b, 6) * lw;
      loss[NTERMS * b + 7] = sc->w[7] * lcen;
      loss[NTERMS * b + 8] = sc->w[8] * lod;
    }
  }
}

int oracle_forward(const oracle_scene *sc, const double *params, double *S, double *Sp, double *loss) {
  if (!sc || !params) return -1;
  if (sc->use_bbox && !sc->use_cutoff) return -1;
  prepared pr;
  prepare(sc, params, &pr);
  double *Stmp = NULL;
  if (!S && loss && sc->w[5] != 0.0) {
    const int64_t total = pixel_offset(sc, sc->B);
    Stmp = (double *)malloc(sizeof(double) * (total > 0 ? total : 1));
    S = Stmp;
  }
  forward_impl(sc, &pr, S, Sp, loss);
  free(Stmp);
  release(&pr);
  return 0;
}

/* Per-item coverage images alpha (and alpha_pad) for items [first, first+count), each on its own
 * layout's canvas, written consecutively. */
int oracle_render(const oracle_scene *sc, const double *params, int first, int count, double *alpha, double *alpha_pad) {
  if (!sc || !params || first < 0 || count < 0 || first + count > sc->N) return -1;
  prepared pr;
  prepare(sc, params, &pr);
  int64_t out = 0;
  for (int q = first; q < first + count; ++q) {
    const int b = layout_of(sc, q);
    const int W = sc->width[b], H = sc->height[b];
    const int n = sc->vert_off[q + 1] - sc->vert_off[q];
#pragma omp parallel for schedule(static)
    for (int j = 0; j < H; ++j) {
      for (int i = 0; i < W; ++i) {
        double a = 0.0, ap = 0.0, da, dap;
        if (n > 0 && in_box(pr.box + 4 * q, i, j)) {
          const sd_result r = item_distance(sc, params, q, sc->scale[b], i + 0.5, j + 0.5, pr.P + 2 * sc->vert_off[q], n);
          coverage(sc, r.sd, &a, &da, &ap, &dap);
        }
        if (alpha) alpha[out + (int64_t)j * W + i] = a;
        if (alpha_pad) alpha_pad[out + (int64_t)j * W + i] = ap;
      }
    }
    out += (int64_t)W * H;
  }
  release(&pr);
  return 0;
}

/* Signed distances of items [first, first+count) at every pixel (for tests of the geometry). */
int oracle_signed_distance(const oracle_scene *sc, const double *params, int first, int count, double *sd,
                           int32_t *edge) {
  if (!sc || !params || first < 0 || count < 0 || first + count > sc->N) return -1;
  oracle_scene full = *sc;
  full.use_bbox = 0;
  prepared pr;
  prepare(&full, params, &pr);
  int64_t out = 0;
  for (int q = first; q < first + count; ++q) {
    const int b = layout_of(sc, q);
    const int W = sc->width[b], H = sc->height[b];
    const int n = sc->vert_off[q + 1] - sc->vert_off[q];
    for (int j = 0; j < H; ++j)
      for (int i = 0; i < W; ++i) {
        sd_result r;
        if (n > 0) {
          r = item_distance(sc, params, q, sc->scale[b], i + 0.5, j + 0.5, pr.P + 2 * sc->vert_off[q], n);
        } else {
          r.sd = -INFINITY;
          r.edge = -1;
        }
        sd[out + (int64_t)j * W + i] = r.sd;
        if (edge) edge[out + (int64_t)j * W + i] = r.edge;
      }
    out += (int64_t)W * H;
  }
  release(&pr);
  return 0;
}

/*
 * Gradient of sum_b sum_t dloss[b,t] * loss[b,t] with respect to params [N*4].
 *
 * dLoss/dS(p) and dLoss/dS_pad(p) follow from the loss definitions (relu'(0) = 0, and the uniform
 * term's min(S, 1) has derivative 1(S < 1)).  Each item's
 * contribution at pixel p is omega * dsd/dparam, omega = G * dalpha/dsd + G_pad * dalpha_pad/dsd.
 * dsd/dparam is taken through the vertices: for the nearest point q = a + u (b - a) on the nearest
 * edge (a, b), with g = (p - q)/|p - q| and sign +1 inside / -1 outside (always -1 for an open
 * item, whose sd = k |s| w - d also has the direct term d sd / ds = k w sign(s)),
 *     dsd/da = -sign (1 - u) g,  dsd/db = -sign u g          (0 < u < 1)
 *     dsd/da = -sign g (u = 0),  dsd/db = -sign g (u = 1)    (nearest point is an end point)
 * and through eq. 2, v' = k (R(theta) s v + t):
 *     dv'/dt = k I,   dv'/dtheta = k s R'(theta) v,   dv'/ds = k R(theta) v.
 * A pixel centre lying exactly on the outline (|p - q| = 0) contributes nothing.
 */
/* dLoss/dS and dLoss/dS_pad per pixel (G, Gp) of sum_b sum_t dloss[b][t] loss[b][t], from the coverage
 * sums S, S_pad of the prepared items (the derivative of each term of the forward pass). */
static void dloss_images(const oracle_scene *sc, const prepared *pr, const double *dloss, double *S, double *Sp,
                         double *G, double *Gp) {
  forward_impl(sc, pr, S, Sp, NULL);
  for (int b = 0; b < sc->B; ++b) {
    const int W = sc->width[b], H = sc->height[b];
    const int64_t off = pixel_offset(sc, b);
    const double c_ov = dloss[NTERMS * b + 0] * sc->w[0] * term_norm(sc, b, 0);
    const double c_c = dloss[NTERMS * b + 1] * sc->w[1] * term_norm(sc, b, 1);
    const double c_f = dloss[NTERMS * b + 2] * sc->w[2] * term_norm(sc, b, 2);
    const double c_p = dloss[NTERMS * b + 3] * sc->w[3] * term_norm(sc, b, 3);
    const double c_d = dloss[NTERMS * b + 4] * sc->w[4];
    const double c_w = dloss[NTERMS * b + 6] * sc->w[6] * term_norm(sc, b, 6);
    const double c_cen = dloss[NTERMS * b + 7] * sc->w[7];
    for (int j = 0; j < H; ++j)
      for (int i = 0; i < W; ++i) {
        const int64_t idx = off + (int64_t)j * W + i;
        const double s = S[idx], sp = Sp[idx];
        const double M = sc->mask ? sc->mask[idx] : 0.0;
        const double ov = s > 1.0 ? s - 1.0 : 0.0;
        const double un = s < 1.0 ? 1.0 - s : 0.0;
        const double pv = sp > 1.0 ? sp - 1.0 : 0.0;
        G[idx] = 2.0 * c_ov * ov + c_c * (1.0 - M) - 2.0 * c_f * M * un + c_d * (H - (j + 0.5));
        /* d/dS of W (M - min(S, 1))^2 */
        if (s < 1.0) G[idx] -= 2.0 * c_w * (WMSE_IN * M + WMSE_OUT * (1.0 - M)) * (M - s);
        const double cx = i + 0.5 - 0.5 * W, cy = j + 0.5 - 0.5 * H;
        G[idx] += c_cen * sqrt(cx * cx + cy * cy);
        Gp[idx] = 2.0 * c_p * pv;
      }
    uniform_grad(sc, b, S + off, dloss[NTERMS * b + 5] * sc->w[5], G + off);
  }
}

/* The terms one pixel (px, py) adds to item q's gradient g[4] and, with gv, to its outline vertices: with r
 * the pixel's distance result for the item (nearest edge, clamped parameter, nearest point, inside flag)
 * and G, Gp dLoss/dS and dLoss/dS_pad at the pixel, omega = G dalpha/dsd + Gp dalpha_pad/dsd times dsd with
 * respect to the two end points of the nearest edge, then through eq. 2.  (c, sn: cos, sin of theta.) */
static void pixel_terms(const oracle_scene *sc, int q, double k, int n, double c, double sn, double s, int open,
                        double px, double py, const sd_result *r, double G, double Gp, double *g, double *gv) {
  double a, da, ap, dap;
  coverage(sc, r->sd, &a, &da, &ap, &dap);
  const double omega = G * da + Gp * dap;
  if (omega == 0.0) return;
  /* an open item's stroke radius k |s| w grows with |s| */
  if (open) g[3] += omega * k * sc->stroke[q] * (s > 0.0 ? 1.0 : (s < 0.0 ? -1.0 : 0.0));
  if (r->d == 0.0) return;
  const double sgn = r->inside ? 1.0 : -1.0;
  const double gx = (px - r->qx) / r->d, gy = (py - r->qy) / r->d;
  /* dsd/d(vertex) for the two end points of the nearest edge */
  double wa, wb;
  if (r->u <= 0.0) {
    wa = 1.0;
    wb = 0.0;
  } else if (r->u >= 1.0) {
    wa = 0.0;
    wb = 1.0;
  } else {
    wa = 1.0 - r->u;
    wb = r->u;
  }
  const int ma = r->edge, mb = open ? (n > 1 ? r->edge + 1 : r->edge) : ((r->edge + 1 == n) ? 0 : r->edge + 1);
  const int vm[2] = {ma, mb};
  const double wv[2] = {wa, wb};
  for (int e = 0; e < 2; ++e) {
    if (wv[e] == 0.0) continue;
    const double dvx = -sgn * wv[e] * gx, dvy = -sgn * wv[e] * gy; /* dsd/dv' */
    const double lx = sc->verts[2 * (sc->vert_off[q] + vm[e])];
    const double ly = sc->verts[2 * (sc->vert_off[q] + vm[e]) + 1];
    /* dv'/dt = k I */
    g[0] += omega * dvx * k;
    g[1] += omega * dvy * k;
    /* dv'/dtheta = k s R'(theta) v,  R' = [[-sin, -cos], [cos, -sin]] */
    const double rtx = k * s * (-sn * lx - c * ly), rty = k * s * (c * lx - sn * ly);
    g[2] += omega * (dvx * rtx + dvy * rty);
    /* dv'/ds = k R(theta) v */
    const double rsx = k * (c * lx - sn * ly), rsy = k * (sn * lx + c * ly);
    g[3] += omega * (dvx * rsx + dvy * rsy);
    /* dv'/dv = k s R(theta) */
    if (gv) {
      gv[2 * vm[e] + 0] += omega * k * s * (c * dvx + sn * dvy);
      gv[2 * vm[e] + 1] += omega * k * s * (-sn * dvx + c * dvy);
    }
  }
}

int oracle_backward_full(const oracle_scene *sc, const double *params, const double *dloss, double *grad,
                         double *grad_verts);

int oracle_backward(const oracle_scene *sc, const double *params, const double *dloss, double *grad) {
  return oracle_backward_full(sc, params, dloss, grad, NULL);
}

/*
 * As oracle_backward, and (grad_verts not NULL) the gradient with respect to every item's outline
 * vertices in its own frame, [V*2] canonical px (Sec. 3 "Vector Representation": the outline control
 * points are fitted by differentiable rendering): each pixel's dsd/dv' of the two end points of its
 * nearest edge, mapped back through eq. 2, dv'/dv = k s R(theta):  dL/dv = omega (k s R)^T dsd/dv'.
 */
int oracle_backward_full(const oracle_scene *sc, const double *params, const double *dloss, double *grad,
                         double *grad_verts) {
  if (!sc || !params || !dloss || !grad) return -1;
  if (sc->use_bbox && !sc->use_cutoff) return -1;
  prepared pr;
  prepare(sc, params, &pr);
  int64_t total = pixel_offset(sc, sc->B);
  double *S = (double *)malloc(sizeof(double) * (total > 0 ? total : 1));
  double *Sp = (double *)malloc(sizeof(double) * (total > 0 ? total : 1));
  double *G = (double *)malloc(sizeof(double) * (total > 0 ? total : 1));
  double *Gp = (double *)malloc(sizeof(double) * (total > 0 ? total : 1));
  dloss_images(sc, &pr, dloss, S, Sp, G, Gp);
  for (int b = 0; b < sc->B; ++b) {
    const int W = sc->width[b];
    const int64_t off = pixel_offset(sc, b);
    const double k = sc->scale[b];
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = sc->shape_off[b]; q < sc->shape_off[b + 1]; ++q) {
      const int n = sc->vert_off[q + 1] - sc->vert_off[q];
      double g[4] = {0, 0, 0, 0};
      double *gv = grad_verts ? grad_verts + 2 * sc->vert_off[q] : NULL;
      if (gv)
        for (int m = 0; m < 2 * n; ++m) gv[m] = 0.0;
      if (n > 0) {
        const double *P = pr.P + 2 * sc->vert_off[q];
        const double th = params[4 * q + 2], s = params[4 * q + 3];
        const double c = cos(th), sn = sin(th);
        const int *bx = pr.box + 4 * q;
        const int open = is_open(sc, q);
        for (int j = bx[1]; j <= bx[3]; ++j)
          for (int i = bx[0]; i <= bx[2]; ++i) {
            const int64_t idx = off + (int64_t)j * W + i;
            const double px = i + 0.5, py = j + 0.5;
            const sd_result r = item_distance(sc, params, q, k, px, py, P, n);
            pixel_terms(sc, q, k, n, c, sn, s, open, px, py, &r, G[idx], Gp[idx], g, gv);
          }
      }
      /* object-space downward force: d(H - k t_y)/dt_y = -k */
      g[1] -= dloss[NTERMS * b + 8] * sc->w[8] * k;
      for (int e = 0; e < 4; ++e) grad[4 * q + e] = g[e];
    }
  }
  free(S);
  free(Sp);
  free(G);
  free(Gp);
  release(&pr);
  return 0;
}

/* Pixel (px, py)'s distance result for item q if edge m were its nearest edge: the clamped parameter,
 * nearest point and distance on edge m, with the inside flag of the full test kept. */
static sd_result edge_distance(const oracle_scene *sc, const double *params, int q, double k, double px, double py,
                               const double *P, int n, int m, int inside) {
  const int open = is_open(sc, q);
  const int mn = open ? (n > 1 ? m + 1 : m) : ((m + 1 == n) ? 0 : m + 1);
  const double ax = P[2 * m], ay = P[2 * m + 1];
  const double ex = P[2 * mn] - ax, ey = P[2 * mn + 1] - ay;
  const double ee = ex * ex + ey * ey;
  double u = 0.0;
  if (ee > 0.0) {
    u = ((px - ax) * ex + (py - ay) * ey) / ee;
    if (u < 0.0) u = 0.0;
    if (u > 1.0) u = 1.0;
  }
  sd_result r;
  r.qx = ax + u * ex;
  r.qy = ay + u * ey;
  r.d = sqrt((px - r.qx) * (px - r.qx) + (py - r.qy) * (py - r.qy));
  r.edge = m;
  r.u = u;
  r.inside = open ? 0 : inside;
  r.sd = open ? stroke_radius(sc, params, q, k) - r.d : (inside ? r.d : -r.d);
  return r;
}

/*
 * Gradient terms that hang on a nearest-edge decision finer than a given resolution.  Where an edge that
 * is not a neighbour of a pixel's nearest edge lies within delta(p) = delta_abs + delta_rel |p - k t| of
 * the nearest distance, an evaluation whose distances carry errors up to delta(p) may take that edge, and
 * the pixel's terms then come from that edge's nearest point and normal (the loss has a kink there: the
 * pixel sits on a medial axis of the outline to that resolution).  bound[4 q + c] sums, over item q's
 * pixels, the largest change |terms(rival) - terms(nearest)| of component c over such rivals; it is 0 for
 * an item with no such pixel.  The neighbours of the nearest edge are excluded because they share its end
 * points: where one of them ties, both give the same nearest point.
 */
int oracle_nearest_ambiguity(const oracle_scene *sc, const double *params, const double *dloss, double delta_abs,
                             double delta_rel, double *bound) {
  if (!sc || !params || !dloss || !bound) return -1;
  if (sc->use_bbox && !sc->use_cutoff) return -1;
  prepared pr;
  prepare(sc, params, &pr);
  int64_t total = pixel_offset(sc, sc->B);
  double *S = (double *)malloc(sizeof(double) * (total > 0 ? total : 1));
  double *Sp = (double *)malloc(sizeof(double) * (total > 0 ? total : 1));
  double *G = (double *)malloc(sizeof(double) * (total > 0 ? total : 1));
  double *Gp = (double *)malloc(sizeof(double) * (total > 0 ? total : 1));
  dloss_images(sc, &pr, dloss, S, Sp, G, Gp);
  for (int b = 0; b < sc->B; ++b) {
    const int W = sc->width[b];
    const int64_t off = pixel_offset(sc, b);
    const double k = sc->scale[b];
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = sc->shape_off[b]; q < sc->shape_off[b + 1]; ++q) {
      double acc[4] = {0, 0, 0, 0};
      const int n = sc->vert_off[q + 1] - sc->vert_off[q];
      const int open = is_open(sc, q);
      const int ne = open ? (n > 1 ? n - 1 : 1) : n;
      if (ne > 3) {
        const double *P = pr.P + 2 * sc->vert_off[q];
        const double th = params[4 * q + 2], s = params[4 * q + 3];
        const double c = cos(th), sn = sin(th);
        const double ox = k * params[4 * q + 0], oy = k * params[4 * q + 1];
        const int *bx = pr.box + 4 * q;
        for (int j = bx[1]; j <= bx[3]; ++j)
          for (int i = bx[0]; i <= bx[2]; ++i) {
            const int64_t idx = off + (int64_t)j * W + i;
            const double px = i + 0.5, py = j + 0.5;
            const sd_result r = item_distance(sc, params, q, k, px, py, P, n);
            const double delta = delta_abs + delta_rel * sqrt((px - ox) * (px - ox) + (py - oy) * (py - oy));
            double base[4] = {0, 0, 0, 0}, worst[4] = {0, 0, 0, 0};
            int have_base = 0;
            for (int m = 0; m < ne; ++m) {
              const int dm = m > r.edge ? m - r.edge : r.edge - m;
              if (dm <= 1 || (!open && dm == ne - 1)) continue;
              const sd_result rm = edge_distance(sc, params, q, k, px, py, P, n, m, r.inside);
              if (!(rm.d <= r.d + delta)) continue;
              if (!have_base) {
                pixel_terms(sc, q, k, n, c, sn, s, open, px, py, &r, G[idx], Gp[idx], base, NULL);
                have_base = 1;
              }
              double t[4] = {0, 0, 0, 0};
              pixel_terms(sc, q, k, n, c, sn, s, open, px, py, &rm, G[idx], Gp[idx], t, NULL);
              for (int e = 0; e < 4; ++e) {
                const double dv = fabs(t[e] - base[e]);
                if (dv > worst[e]) worst[e] = dv;
              }
            }
            for (int e = 0; e < 4; ++e) acc[e] += worst[e];
          }
      }
      for (int e = 0; e < 4; ++e) bound[4 * q + e] = acc[e];
    }
  }
  free(S);
  free(Sp);
  free(G);
  free(Gp);
  release(&pr);
  return 0;
}

/*
 * One Adam step (moment estimates with bias correction, no weight decay) on n parameters with a
 * per-parameter learning rate.  t is the 1-based step number after this update.
 */
int oracle_adam(int n, double *param, const double *grad, double *m, double *v, int t, const double *lr,
                double beta1, double beta2, double eps) {
  if (n < 0 || t < 1) return -1;
  const double bc1 = 1.0 - pow(beta1, t), bc2 = 1.0 - pow(beta2, t);
  for (int i = 0; i < n; ++i) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
    const double mhat = m[i] / bc1, vhat = v[i] / bc2;
    param[i] -= lr[i] * mhat / (sqrt(vhat) + eps);
  }
  return 0;
}

/*
 * Per-parameter learning rates of the collage update: translations move lr_px level pixels per step
 * (lr_px / k canonical px); rotation and scale move the item's rim (radius rho_i canonical px) by
 * lr_px level pixels: lr = lr_px / (k * rho_i).
 */
int oracle_collage_lr(const oracle_scene *sc, const double *rho, double lr_px, double *lr) {
  for (int b = 0; b < sc->B; ++b) {
    const double k = sc->scale[b];
    for (int i = sc->shape_off[b]; i < sc->shape_off[b + 1]; ++i) {
      lr[4 * i + 0] = lr_px / k;
      lr[4 * i + 1] = lr_px / k;
      lr[4 * i + 2] = rho[i] > 0.0 ? lr_px / (k * rho[i]) : 0.0;
      lr[4 * i + 3] = rho[i] > 0.0 ? lr_px / (k * rho[i]) : 0.0;
    }
  }
  return 0;
}

/*
 * Quality metrics of Sec. 6 ("Metrics of Collage Quality"), on hard rasters: pixel p is covered by
 * item i when sd_i(p) >= 0, and lies in the target shape when M(p) >= 1/2.  Per layout b, with T the
 * number of target pixels,
 *   out[3 b + 0]  LC = (covered pixels in the target) / T             (layout coverage)
 *   out[3 b + 1]  OO = (pixels covered by two or more items) / T      (object overlap)
 *   out[3 b + 2]  EA = (covered pixels outside the target) / T        (exceeding area)
 * (all 0 for a layout without target pixels).  counts (may be NULL) receives per layout
 * [4 b + 0..3] = T, covered in the target, overlap pixels, covered outside the target.
 * Test tooling: the metrics of a finished layout.
 */
int oracle_quality(const oracle_scene *sc, const double *params, double *out, int64_t *counts) {
  if (!sc || !params || !out) return -1;
  if (sc->use_bbox && !sc->use_cutoff) return -1;
  prepared pr;
  prepare(sc, params, &pr);
  for (int b = 0; b < sc->B; ++b) {
    const int W = sc->width[b], H = sc->height[b];
    const int64_t off = pixel_offset(sc, b);
    int64_t target = 0, in_cov = 0, overlap = 0, out_cov = 0;
    for (int j = 0; j < H; ++j)
      for (int i = 0; i < W; ++i) {
        int n_cov = 0;
        for (int q = sc->shape_off[b]; q < sc->shape_off[b + 1]; ++q) {
          const int n = sc->vert_off[q + 1] - sc->vert_off[q];
          if (n == 0 || !in_box(pr.box + 4 * q, i, j)) continue;
          const sd_result r = item_distance(sc, params, q, sc->scale[b], i + 0.5, j + 0.5, pr.P + 2 * sc->vert_off[q], n);
          if (r.sd >= 0.0) ++n_cov;
        }
        const int in_target = sc->mask ? sc->mask[off + (int64_t)j * W + i] >= 0.5 : 0;
        target += in_target;
        if (n_cov >= 1 && in_target) ++in_cov;
        if (n_cov >= 1 && !in_target) ++out_cov;
        if (n_cov >= 2) ++overlap;
      }
    const double T = (double)target;
    out[3 * b + 0] = target > 0 ? (double)in_cov / T : 0.0;
    out[3 * b + 1] = target > 0 ? (double)overlap / T : 0.0;
    out[3 * b + 2] = target > 0 ? (double)out_cov / T : 0.0;
    if (counts) {
      counts[4 * b + 0] = target;
      counts[4 * b + 1] = in_cov;
      counts[4 * b + 2] = overlap;
      counts[4 * b + 3] = out_cov;
    }
  }
  release(&pr);
  return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
