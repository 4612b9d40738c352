/*
 * oracle.c -- plain CPU FP64 reference for the box-code volume potential.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
 * benchmark's CPU-baseline leg may load this code.  It shares nothing with the
 * HIP library: no headers, tables, constants or helpers.
 *
 * What it computes (section 3, eq. volumeint3 and the definition of the
 * piecewise polynomial approximation f~ in section 3.1; gradient as the second
 * volume integral of section 3.2, eq. volumeint3x):
 *
 *     V(x)  = sum over leaves B of  int_B G(x - y) f~_B(y) dy,
 *     dV(x) = sum over leaves B of  int_B grad_x G(x - y) f~_B(y) dy,
 *
 * with G(r) = log|r| / (2 pi) (the sign that makes Laplacian(V) = f, as in
 * eq. poisson1 and eq. volumeint1), and f~_B the degree-(n-1) tensor
 * polynomial through the leaf's samples at first-kind Chebyshev nodes.
 * This is the plain definition, summed directly over every (target, leaf)
 * pair; no expansions and no tables.
 *
 * Quadrature, per (target x, square S of width w -- a leaf or a quarter of one
 * -- at distance d from x):
 *   - d >= w/2: tensor Gauss-Legendre q x q on S, q chosen from d/w so that
 *     the Bernstein-ellipse estimate of the error is below 1e-17 relative.
 *   - w/16 <= d < w/2: the four quarters of S, each treated the same way.
 *   - d < w/16 (x inside S or just outside): polar coordinates about x.  S is
 *     the signed sum of the four
 *     triangles (x, corner_k, corner_k+1), each parametrised by the angle
 *     from the normal to its edge line (so the ray length p/cos(phi) keeps
 *     full relative precision when x is close to that line).  Along each ray the source is a
 *     polynomial of degree <= 2(n-1) in the radius, so the radial integrals
 *     are done exactly: Gauss-Legendre for rho^1 and rho^0 weights and a
 *     Gauss rule for the weight -log t for the logarithmic part.  The angle
 *     is integrated by adaptive bisection with Gauss-Legendre panels until
 *     the panel and its two halves agree to 1e-15 of the leaf's scale
 *     (the same absolute tolerance on every panel, at most 30 bisections).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXN 32
#define OR_MAXQ 48
#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------ rules */
static void gauss_legendre(int q, double *x, double *w) {
  /* Newton iteration on the Legendre three-term recurrence; nodes on [-1,1]. */
  for (int i = 0; i < q; ++i) {
    double z = cos(OR_PI * (i + 0.75) / (q + 0.5)), pp = 1.0, p1 = 1.0, p2 = 0.0;
    for (int it = 0; it < 100; ++it) {
      p1 = 1.0; p2 = 0.0;
      for (int j = 1; j <= q; ++j) {
        double p3 = p2; p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = q * (z * p1 - p2) / (z * z - 1.0);
      double z1 = z;
      z = z1 - p1 / pp;
      if (fabs(z - z1) < 1e-16) break;
    }
    p1 = 1.0; p2 = 0.0;
    for (int j = 1; j <= q; ++j) {
      double p3 = p2; p2 = p1;
      p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
    }
    pp = q * (z * p1 - p2) / (z * z - 1.0);
    x[q - 1 - i] = z;          /* ascending order */
    w[q - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

typedef struct {
  int n;                        /* nodes per side */
  double coef[OR_MAXN * OR_MAXN];  /* Chebyshev coefficients c[b][a] (b along y) */
  double x0, y0, w;             /* lower-left corner and width */
  double fscale;                /* max |sample|, for tolerances */
} leaf_t;

/* Chebyshev coefficients of the tensor interpolant through first-kind nodes,
 * by the discrete orthogonality of T_a at those nodes (explicit cosine sums). */
static void cheb_coeffs(int n, const double *f, double *c) {
  double T[OR_MAXN][OR_MAXN];   /* T[a][j] = T_a(xi_j), xi_j = -cos((2j+1)pi/2n) */
  for (int a = 0; a < n; ++a)
    for (int j = 0; j < n; ++j) {
      double theta = OR_PI - (2.0 * j + 1.0) * OR_PI / (2.0 * n);   /* xi_j = cos(theta) */
      T[a][j] = cos(a * theta);
    }
  for (int b = 0; b < n; ++b)
    for (int a = 0; a < n; ++a) {
      double s = 0.0;
      for (int j2 = 0; j2 < n; ++j2)
        for (int j1 = 0; j1 < n; ++j1) s += f[j2 * n + j1] * T[a][j1] * T[b][j2];
      double wa = (a == 0 ? 1.0 : 2.0) / n, wb = (b == 0 ? 1.0 : 2.0) / n;
      c[b * n + a] = wa * wb * s;
    }
}

static inline void cheb_values(int n, double t, double *T) {
  T[0] = 1.0;
  if (n > 1) T[1] = t;
  for (int a = 2; a < n; ++a) T[a] = 2.0 * t * T[a - 1] - T[a - 2];
}

/* f~ at a physical point (may lie outside the leaf: the polynomial extends). */
static inline double ftilde(const leaf_t *L, double x, double y) {
  int n = L->n;
  double Tx[OR_MAXN], Ty[OR_MAXN];
  double ex = 2.0 * (x - L->x0) / L->w - 1.0, ey = 2.0 * (y - L->y0) / L->w - 1.0;
  cheb_values(n, ex, Tx);
  cheb_values(n, ey, Ty);
  double s = 0.0;
  for (int b = 0; b < n; ++b) {
    double r = 0.0;
    for (int a = 0; a < n; ++a) r += L->coef[b * n + a] * Tx[a];
    s += r * Ty[b];
  }
  return s;
}

typedef struct {
  int nr;                       /* radial rule size */
  const double *gt, *gw;        /* Gauss-Legendre on [0,1] */
  const double *lt, *lw;        /* Gauss rule for weight -log t on [0,1] */
} radial_t;

/* ------------------------------------------------------------ near field */
typedef struct {
  const leaf_t *L;
  const radial_t *R;
  double x, y;                  /* target */
  double p;                     /* distance from the target to the edge line */
  double mx, my, ex, ey;        /* unit normal towards the edge line, unit edge direction */
} ray_ctx;

/* Integrand in the angle phi measured from the normal m: contributions to
 * (V, Gx, Gy) of the ray x + rho (cos(phi) m + sin(phi) e), 0 <= rho <= p/cos(phi). */
static void ray(const ray_ctx *c, double phi, double out[3]) {
  double cp = cos(phi), sp = sin(phi);
  double dx = cp * c->mx + sp * c->ex, dy = cp * c->my + sp * c->ey;
  double Rr = c->p / cp;
  const radial_t *R = c->R;
  double s1 = 0.0, s0 = 0.0, sl = 0.0;
  for (int i = 0; i < R->nr; ++i) {
    double rho = Rr * R->gt[i];
    double ph = ftilde(c->L, c->x + rho * dx, c->y + rho * dy);
    s1 += R->gw[i] * R->gt[i] * ph;       /* int_0^1 t phi(Rt) dt      */
    s0 += R->gw[i] * ph;                  /* int_0^1 phi(Rt) dt        */
    double rl = Rr * R->lt[i];
    double pl = ftilde(c->L, c->x + rl * dx, c->y + rl * dy);
    sl += R->lw[i] * R->lt[i] * pl;       /* int_0^1 (-log t) t phi dt */
  }
  /* int_0^R log(rho) phi(rho) rho drho = R^2 log R * s1 - R^2 * sl */
  out[0] = (Rr * Rr * log(Rr) * s1 - Rr * Rr * sl) / (2.0 * OR_PI);
  /* grad_x G(x - y) = (x - y) / (2 pi |x - y|^2) = -d / (2 pi rho) */
  out[1] = -dx * Rr * s0 / (2.0 * OR_PI);
  out[2] = -dy * Rr * s0 / (2.0 * OR_PI);
}

typedef struct { int q; double x[OR_MAXQ], w[OR_MAXQ]; } gl_t;

static void panel(const ray_ctx *c, const gl_t *g, double a, double b, double out[3]) {
  double m = 0.5 * (a + b), h = 0.5 * (b - a), v[3];
  out[0] = out[1] = out[2] = 0.0;
  for (int i = 0; i < g->q; ++i) {
    ray(c, m + h * g->x[i], v);
    out[0] += g->w[i] * v[0]; out[1] += g->w[i] * v[1]; out[2] += g->w[i] * v[2];
  }
  out[0] *= h; out[1] *= h; out[2] *= h;
}

static void adapt(const ray_ctx *c, const gl_t *g, double a, double b, const double whole[3],
                  const double tol[3], int depth, double out[3]) {
  double m = 0.5 * (a + b), l[3], r[3];
  panel(c, g, a, m, l);
  panel(c, g, m, b, r);
  int ok = depth >= 30;
  if (!ok) {
    ok = 1;
    for (int k = 0; k < 3; ++k)
      if (fabs(l[k] + r[k] - whole[k]) > tol[k]) ok = 0;
  }
  if (ok) {
    for (int k = 0; k < 3; ++k) out[k] = l[k] + r[k];
    return;
  }
  double lo[3], ro[3];
  adapt(c, g, a, m, l, tol, depth + 1, lo);
  adapt(c, g, m, b, r, tol, depth + 1, ro);
  for (int k = 0; k < 3; ++k) out[k] = lo[k] + ro[k];
}

/* The square is the signed sum of the triangles (x, A, B) over its
 * counter-clockwise edges A -> B; each triangle is integrated in polar
 * coordinates about x, the angle measured from the normal to the edge line. */
static void near_square(const leaf_t *L, const radial_t *R, const gl_t *g, double sx0, double sy0, double sw,
                        double x, double y, double out[3]) {
  double cx[4] = {sx0, sx0 + sw, sx0 + sw, sx0};
  double cy[4] = {sy0, sy0, sy0 + sw, sy0 + sw};     /* counter-clockwise */
  double tol[3];
  double fs = L->fscale > 0.0 ? L->fscale : 1.0;
  tol[0] = 1e-15 * fs * sw * sw * (1.0 + fabs(log(sw)));
  tol[1] = tol[2] = 1e-15 * fs * sw;
  out[0] = out[1] = out[2] = 0.0;
  for (int k = 0; k < 4; ++k) {
    double Ax = cx[k], Ay = cy[k], Bx = cx[(k + 1) & 3], By = cy[(k + 1) & 3];
    double el = hypot(Bx - Ax, By - Ay);
    double ex = (Bx - Ax) / el, ey = (By - Ay) / el;     /* exact for axis-aligned edges */
    double nx = ey, ny = -ex;                           /* outward normal */
    double ps = (Ax - x) * nx + (Ay - y) * ny;          /* signed distance to the edge line */
    if (fabs(ps) < 1e-15 * sw) continue;                /* degenerate triangle: zero area */
    double sg = ps > 0.0 ? 1.0 : -1.0;
    double tA = (Ax - x) * ex + (Ay - y) * ey, tB = (Bx - x) * ex + (By - y) * ey;
    ray_ctx c = {L, R, x, y, fabs(ps), sg * nx, sg * ny, ex, ey};
    double pa = atan2(tA, c.p), pb = atan2(tB, c.p);
    double whole[3], res[3];
    panel(&c, g, pa, pb, whole);
    adapt(&c, g, pa, pb, whole, tol, 0, res);
    out[0] += sg * res[0]; out[1] += sg * res[1]; out[2] += sg * res[2];
  }
}

/* ------------------------------------------------------------- far field */
static void far_square(const leaf_t *L, const gl_t *g, double sx0, double sy0, double sw, double x, double y,
                       double out[3]) {
  int n = L->n, q = g->q;
  double Tq[OR_MAXQ][OR_MAXN], Ty[OR_MAXQ][OR_MAXN], Gm[OR_MAXN][OR_MAXQ];
  double r = 0.5 * sw, xc = sx0 + r, yc = sy0 + r;
  /* Chebyshev values at the Gauss points of the square, in the leaf's coordinates */
  for (int a = 0; a < q; ++a) {
    cheb_values(n, 2.0 * (xc + r * g->x[a] - L->x0) / L->w - 1.0, Tq[a]);
    cheb_values(n, 2.0 * (yc + r * g->x[a] - L->y0) / L->w - 1.0, Ty[a]);
  }
  /* Gm[b][a] = sum_i c[b][i] T_i(x_a) */
  for (int b = 0; b < n; ++b)
    for (int a = 0; a < q; ++a) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += L->coef[b * n + i] * Tq[a][i];
      Gm[b][a] = s;
    }
  double sv = 0.0, sx = 0.0, sy = 0.0;
  for (int bb = 0; bb < q; ++bb) {
    double yy = yc + r * g->x[bb];
    for (int a = 0; a < q; ++a) {
      double fv = 0.0;
      for (int b = 0; b < n; ++b) fv += Gm[b][a] * Ty[bb][b];
      double xx = xc + r * g->x[a];
      double dx = x - xx, dy = y - yy, r2 = dx * dx + dy * dy;
      double wt = g->w[a] * g->w[bb] * fv;
      sv += wt * 0.5 * log(r2);
      sx += wt * dx / r2;
      sy += wt * dy / r2;
    }
  }
  double jac = r * r / (2.0 * OR_PI);
  out[0] = sv * jac; out[1] = sx * jac; out[2] = sy * jac;
}

static int far_order(int n, double d, double w) {
  /* Worst 1D slice: a pole at distance d off the middle of a panel of
   * half-width w/2 gives a Bernstein ellipse rho = b + sqrt(b^2 + 1), b = 2d/w. */
  double b = 2.0 * d / w, rho = b + sqrt(b * b + 1.0);
  int q = (int)ceil((17.0 / log10(rho) + n - 1) / 2.0) + 1;
  if (q < n + 1) q = n + 1;
  if (q > OR_MAXQ) q = OR_MAXQ;
  return q;
}

static double sq_dist(double sx0, double sy0, double sw, double x, double y) {
  double dx = 0.0, dy = 0.0;
  if (x < sx0) dx = sx0 - x; else if (x > sx0 + sw) dx = x - sx0 - sw;
  if (y < sy0) dy = sy0 - y; else if (y > sy0 + sw) dy = y - sy0 - sw;
  return hypot(dx, dy);
}

/* Integral over the square [sx0, sx0+sw] x [sy0, sy0+sw] (part of leaf L):
 * tensor rule when the target is at least sw/2 away; polar when it lies inside
 * or within sw/16 (the signed triangles then nearly do not cancel); otherwise
 * the four quarters, so that a target outside the square never meets the large
 * cancelling triangles of a distant polar decomposition. */
static void square(const leaf_t *L, const radial_t *R, const gl_t *gth, const gl_t *rules, double sx0,
                   double sy0, double sw, double x, double y, double out[3]) {
  double d = sq_dist(sx0, sy0, sw, x, y);
  if (d >= 0.5 * sw) {
    far_square(L, &rules[far_order(L->n, d, sw)], sx0, sy0, sw, x, y, out);
  } else if (d < sw / 16.0) {
    near_square(L, R, gth, sx0, sy0, sw, x, y, out);
  } else {
    double h = 0.5 * sw, o[3];
    out[0] = out[1] = out[2] = 0.0;
    for (int k = 0; k < 4; ++k) {
      square(L, R, gth, rules, sx0 + (k & 1) * h, sy0 + (k >> 1) * h, h, x, y, o);
      out[0] += o[0]; out[1] += o[1]; out[2] += o[2];
    }
  }
}

/* ------------------------------------------------------------------- API */
/*
 * Volume potential and gradient of the piecewise polynomial source at
 * arbitrary targets.  Returns 0 on success, -1 on a bad argument.
 *   n           nodes per side (2..32)
 *   cx,cy,width root box
 *   nleaf, level, ix, iy   leaf boxes
 *   f           [nleaf][n][n] samples, x index fastest
 *   use         [nleaf] or NULL: 0 excludes a leaf as a source
 *   ntgt, tx, ty  targets
 *   nr, gt, gw  Gauss-Legendre rule on [0,1] with nr >= n points
 *   lt, lw      Gauss rule for the weight -log t on [0,1], nr points
 *   V, Gx, Gy   outputs [ntgt]
 */
int oracle_volume(int n, double cx, double cy, double width, int nleaf, const int *level,
                  const int *ix, const int *iy, const double *f, const unsigned char *use,
                  int ntgt, const double *tx, const double *ty, int nr, const double *gt,
                  const double *gw, const double *lt, const double *lw, double *V, double *Gx,
                  double *Gy, int nthreads) {
  if (n < 2 || n > OR_MAXN || nleaf < 0 || ntgt < 0 || nr < n) return -1;
  leaf_t *L = (leaf_t *)malloc(sizeof(leaf_t) * (nleaf > 0 ? nleaf : 1));
  if (!L) return -1;
  for (int i = 0; i < nleaf; ++i) {
    double h = ldexp(width, -level[i]);
    L[i].n = n;
    L[i].w = h;
    L[i].x0 = cx - 0.5 * width + ix[i] * h;
    L[i].y0 = cy - 0.5 * width + iy[i] * h;
    cheb_coeffs(n, f + (size_t)i * n * n, L[i].coef);
    double m = 0.0;
    for (int k = 0; k < n * n; ++k) m = fmax(m, fabs(f[(size_t)i * n * n + k]));
    L[i].fscale = m;
  }
  gl_t rules[OR_MAXQ + 1];
  for (int q = 1; q <= OR_MAXQ; ++q) { rules[q].q = q; gauss_legendre(q, rules[q].x, rules[q].w); }
  gl_t gth;
  gth.q = 12;
  gauss_legendre(12, gth.x, gth.w);
  radial_t R = {nr, gt, gw, lt, lw};
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
  for (int t = 0; t < ntgt; ++t) {
    double x = tx[t], y = ty[t], sv = 0.0, sx = 0.0, sy = 0.0, o[3];
    for (int i = 0; i < nleaf; ++i) {
      if (use && !use[i]) continue;
      square(&L[i], &R, &gth, rules, L[i].x0, L[i].y0, L[i].w, x, y, o);
      sv += o[0]; sx += o[1]; sy += o[2];
    }
    V[t] = sv; Gx[t] = sx; Gy[t] = sy;
  }
  free(L);
  return 0;
}

/* Exact integral of f~ over each leaf (tensor Gauss-Legendre, exact for the
 * polynomial), used by the Gauss-law checks. */
int oracle_leaf_mass(int n, double width, int nleaf, const int *level, const double *f,
                     double *mass) {
  if (n < 2 || n > OR_MAXN) return -1;
  gl_t g;
  g.q = n;
  gauss_legendre(n, g.x, g.w);
  for (int i = 0; i < nleaf; ++i) {
    leaf_t L;
    L.n = n; L.w = ldexp(width, -level[i]); L.x0 = 0.0; L.y0 = 0.0;
    cheb_coeffs(n, f + (size_t)i * n * n, L.coef);
    double s = 0.0, r = 0.5 * L.w;
    for (int b = 0; b < n; ++b)
      for (int a = 0; a < n; ++a) s += g.w[a] * g.w[b] * ftilde(&L, r + r * g.x[a], r + r * g.x[b]);
    mass[i] = s * r * r;
  }
  return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
