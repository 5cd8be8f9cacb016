/*
 * sanitize_check.c -- drives every entry point of the FP64 oracle once on a small scene, for a build
 * under AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure only).
 *
 * The scene: two layouts (23 x 17 and 9 x 30 pixels); a square, a triangle, an open three-vertex
 * polyline, an item without vertices and a one-vertex open item; one item partly off its canvas;
 * every loss term on, including the uniform term and the 1 / (w h) normalisation.  Prints "ok" and
 * returns 0 when every call succeeds and every result is finite.
 */
#include "collage_oracle.c"

#include <stdio.h>

static int all_finite(const double *x, int n) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(x[i])) return 0;
  return 1;
}

int main(void) {
  const int32_t width[2] = {23, 9}, height[2] = {17, 30};
  const double scale[2] = {1.0, 0.75};
  const int32_t shape_off[3] = {0, 3, 5};
  /* square (4), triangle (3), open polyline (3); layout 1: no vertices, one-vertex open item */
  const int32_t vert_off[6] = {0, 4, 7, 10, 10, 11};
  const double verts[22] = {-3, -3, 3, -3, 3, 3, -3, 3,   /* square */
                            0, -4, 3.5, 2, -3.5, 2,       /* triangle */
                            -4, 0, 0, 3, 4, -1,           /* open polyline */
                            0, 0};                        /* one-vertex open item */
  const double stroke[5] = {0, 0, 1.2, 0, 0.8};
  double mask[23 * 17 + 9 * 30];
  for (int i = 0; i < 23 * 17 + 9 * 30; ++i) mask[i] = (i % 7) < 4 ? 1.0 : (i % 7 == 4 ? 0.5 : 0.0);
  const double params[20] = {8.2, 7.1, 0.3, 1.1,  15.6, 9.9, 1.7, 0.9,  -1.4, 12.3, 2.2, 1.3,
                             4.1, 11.0, 0.0, 1.0,  5.3, 21.7, 0.4, 1.0};
  oracle_scene sc;
  memset(&sc, 0, sizeof(sc));
  sc.B = 2;
  sc.N = 5;
  sc.V = 11;
  sc.width = width;
  sc.height = height;
  sc.scale = scale;
  sc.shape_off = shape_off;
  sc.vert_off = vert_off;
  sc.verts = verts;
  sc.mask = mask;
  sc.tau = 0.5;
  sc.r_cut = 8.0;
  sc.r_pad = 2.0;
  const double w[9] = {1.0, 1.0, 1.0, 1.0, 1e-3, 0.5, 2.0, 3e-3, 0.25};
  memcpy(sc.w, w, sizeof(w));
  sc.use_cutoff = 1;
  sc.use_bbox = 1;
  sc.stroke = stroke;
  sc.area_mean = 1;
  const int npix = 23 * 17 + 9 * 30;
  double S[23 * 17 + 9 * 30], Sp[23 * 17 + 9 * 30], loss[18], dloss[18], grad[20], gv[22];
  double alpha[3 * 23 * 17 + 2 * 9 * 30], alpha_pad[3 * 23 * 17 + 2 * 9 * 30], sd[3 * 23 * 17 + 2 * 9 * 30];
  int32_t edge[3 * 23 * 17 + 2 * 9 * 30];
  double quality[6], lr[20], p[20], m[20], v[20], amb[20], rho[5] = {4.3, 4.1, 5.2, 0.0, 0.8};
  int64_t counts[8];
  for (int i = 0; i < 18; ++i) dloss[i] = 0.5 + 0.1 * i;
  int rc = 0;
  rc |= oracle_forward(&sc, params, S, Sp, loss);
  rc |= oracle_backward(&sc, params, dloss, grad);
  rc |= oracle_backward_full(&sc, params, dloss, grad, gv);
  rc |= oracle_nearest_ambiguity(&sc, params, dloss, 1e-3, 1e-3, amb);
  rc |= oracle_render(&sc, params, 0, 5, alpha, alpha_pad);
  rc |= oracle_signed_distance(&sc, params, 0, 5, sd, edge);
  rc |= oracle_quality(&sc, params, quality, counts);
  rc |= oracle_collage_lr(&sc, rho, 0.5, lr);
  memcpy(p, params, sizeof(p));
  memset(m, 0, sizeof(m));
  memset(v, 0, sizeof(v));
  rc |= oracle_adam(20, p, grad, m, v, 1, lr, 0.9, 0.999, 1e-8);
  sc.use_bbox = 0;
  sc.use_cutoff = 0;
  rc |= oracle_forward(&sc, params, S, Sp, loss);
  if (rc != 0) {
    printf("error %d\n", rc);
    return 1;
  }
  if (!all_finite(S, npix) || !all_finite(Sp, npix) || !all_finite(loss, 18) || !all_finite(grad, 20) ||
      !all_finite(gv, 22) || !all_finite(quality, 6) || !all_finite(p, 20) || !all_finite(amb, 20)) {
    printf("non-finite result\n");
    return 1;
  }
  printf("ok\n");
  return 0;
}
