// Host FP64 construction of the unit-box operators of the box code.
//
// Everything here is expressed for a target box of unit width centred at the
// origin; the device kernels apply the per-level scalings.  With y = c + h v,
//   log|x - y| = log h + log|xi - v|,  dy = h^2 dv,
// so a near interaction contributes h^2 T f + (h^2 log h / 2pi) (W . f) to V and
// h D f to grad V (the precomputed-table scheme of section 3.1, last
// paragraph, and the gradient tables of section 3.2).  Far-field operators are
// the complex multipole/local expansions of the logarithmic kernel, written
// for coefficients scaled by powers of the box width so that they do not
// depend on the level (the expansions behind Phi_j in section 3.1).
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <thread>

#include "bx_internal.h"

namespace bx {
namespace {

const double kPi = 3.14159265358979323846;
typedef std::complex<double> cd;
typedef std::complex<long double> cld;

struct Rule {
  std::vector<double> x, w;
};

// Gauss-Legendre nodes/weights on [-1,1]: Newton on P_q from Chebyshev-like guesses.
Rule gauss(int q) {
  Rule r;
  r.x.resize(q);
  r.w.resize(q);
  for (int i = 0; i < q; ++i) {
    long double z = std::cos(kPi * (4.0 * i + 3.0) / (4.0 * q + 2.0));
    long double dp = 1;
    for (int it = 0; it < 60; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= q; ++k) {
        long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (q == 1) { p1 = z; p0 = 1; }
      dp = q * (z * p1 - p0) / (z * z - 1);
      long double dz = p1 / dp;
      z -= dz;
      if (std::fabs((double)dz) < 1e-19) break;
    }
    r.x[q - 1 - i] = (double)z;
    r.w[q - 1 - i] = (double)(2 / ((1 - z * z) * dp * dp));
  }
  return r;
}

// First-kind Chebyshev nodes (increasing) and their barycentric weights.
struct Basis {
  int n;
  std::vector<double> x, bw;
  explicit Basis(int n_) : n(n_), x(n_), bw(n_) {
    for (int j = 0; j < n; ++j) {
      double th = (2.0 * j + 1.0) * kPi / (2.0 * n);
      x[j] = -std::cos(th);
      bw[j] = ((n - 1 - j) % 2 ? -1.0 : 1.0) * std::sin(th);
    }
  }
  // values of the n Lagrange polynomials at t (barycentric formula)
  void eval(double t, double *out) const {
    for (int j = 0; j < n; ++j)
      if (t == x[j]) {
        for (int k = 0; k < n; ++k) out[k] = (k == j);
        return;
      }
    double s = 0;
    for (int j = 0; j < n; ++j) {
      out[j] = bw[j] / (t - x[j]);
      s += out[j];
    }
    for (int j = 0; j < n; ++j) out[j] /= s;
  }
};

// A quadrature point: position, offset from the target (kept separately so that
// points very close to the target keep their distance), weight.
struct QPt {
  double x, y, ox, oy, w;
};

// Tensor Gauss rule on a rectangle.
void emit_rect(std::vector<QPt> &pts, const Rule &g, double x0, double x1, double y0, double y1) {
  double hx = 0.5 * (x1 - x0), hy = 0.5 * (y1 - y0), mx = 0.5 * (x0 + x1), my = 0.5 * (y0 + y1);
  int q = (int)g.x.size();
  for (int b = 0; b < q; ++b)
    for (int a = 0; a < q; ++a) {
      double x = mx + hx * g.x[a], y = my + hy * g.x[b];
      pts.push_back({x, y, 0.0, 0.0, hx * hy * g.w[a] * g.w[b]});
    }
}

void set_offsets(std::vector<QPt> &pts, size_t from, double px, double py) {
  for (size_t i = from; i < pts.size(); ++i) {
    pts[i].ox = pts[i].x - px;
    pts[i].oy = pts[i].y - py;
  }
}

double rect_dist(double px, double py, double x0, double x1, double y0, double y1) {
  double dx = px < x0 ? x0 - px : (px > x1 ? px - x1 : 0.0);
  double dy = py < y0 ? y0 - py : (py > y1 ? py - y1 : 0.0);
  return std::hypot(dx, dy);
}

// Rectangle not containing the target: split until every piece is at least
// its own longer side away from the target, then a tensor Gauss rule.
void subdivide(std::vector<QPt> &pts, const Rule &g, double px, double py, double x0, double x1, double y0,
               double y1, int depth) {
  double wx = x1 - x0, wy = y1 - y0, side = std::max(wx, wy);
  if (rect_dist(px, py, x0, x1, y0, y1) >= side || depth > 60) {
    emit_rect(pts, g, x0, x1, y0, y1);
    return;
  }
  if (wx > 1.5 * wy) {
    double m = 0.5 * (x0 + x1);
    subdivide(pts, g, px, py, x0, m, y0, y1, depth + 1);
    subdivide(pts, g, px, py, m, x1, y0, y1, depth + 1);
  } else if (wy > 1.5 * wx) {
    double m = 0.5 * (y0 + y1);
    subdivide(pts, g, px, py, x0, x1, y0, m, depth + 1);
    subdivide(pts, g, px, py, x0, x1, m, y1, depth + 1);
  } else {
    double mx = 0.5 * (x0 + x1), my = 0.5 * (y0 + y1);
    subdivide(pts, g, px, py, x0, mx, y0, my, depth + 1);
    subdivide(pts, g, px, py, mx, x1, y0, my, depth + 1);
    subdivide(pts, g, px, py, x0, mx, my, y1, depth + 1);
    subdivide(pts, g, px, py, mx, x1, my, y1, depth + 1);
  }
}

// Square [0,s]^2 in the quadrant (sx, sy) with the target at its corner:
// Duffy map of its two triangles, (u,t) -> s u (1, t) and s u (t, 1), Jacobian
// s^2 u.  In u the log kernel leaves u log u, integrated on the geometrically
// graded pieces [2^-k-1, 2^-k]; in t the integrand is smooth.
void emit_corner(std::vector<QPt> &pts, const Rule &gu, const Rule &gt, double px, double py, double s,
                 double sx, double sy) {
  const int K = 44;
  for (int tri = 0; tri < 2; ++tri)
    for (int k = 0; k <= K; ++k) {
      double ua = k == K ? 0.0 : std::ldexp(1.0, -k - 1), ub = std::ldexp(1.0, -k);
      double hu = 0.5 * (ub - ua), mu = 0.5 * (ua + ub);
      for (size_t i = 0; i < gu.x.size(); ++i) {
        double u = mu + hu * gu.x[i], wu = hu * gu.w[i];
        for (size_t j = 0; j < gt.x.size(); ++j) {
          double t = 0.5 + 0.5 * gt.x[j], wt = 0.5 * gt.w[j];
          double a = s * u, b = s * u * t;
          double X = tri == 0 ? a : b, Y = tri == 0 ? b : a;
          pts.push_back({px + sx * X, py + sy * Y, sx * X, sy * Y, s * s * u * wu * wt});
        }
      }
    }
}

// Quadrature points for the integral over the square (cx, cy, w) seen from (px, py).
void near_points(std::vector<QPt> &pts, const Rule &g, const Rule &gu, const Rule &gt, double px, double py,
                 double cx, double cy, double w) {
  double x0 = cx - 0.5 * w, x1 = cx + 0.5 * w, y0 = cy - 0.5 * w, y1 = cy + 0.5 * w;
  if (!(px > x0 && px < x1 && py > y0 && py < y1)) {
    subdivide(pts, g, px, py, x0, x1, y0, y1, 0);
    set_offsets(pts, 0, px, py);
    return;
  }
  // split at the target into four rectangles with the target at a corner
  const double ext[4][2] = {{x1 - px, y1 - py}, {px - x0, y1 - py}, {x1 - px, py - y0}, {px - x0, py - y0}};
  const double sg[4][2] = {{1, 1}, {-1, 1}, {1, -1}, {-1, -1}};
  for (int q = 0; q < 4; ++q) {
    double a = ext[q][0], b = ext[q][1], s = std::min(a, b), sx = sg[q][0], sy = sg[q][1];
    emit_corner(pts, gu, gt, px, py, s, sx, sy);
    size_t from = pts.size();
    if (a > s) {  // strip beside the corner square, along x
      double xa = px + sx * s, xb = px + sx * a, ya = py, yb = py + sy * b;
      subdivide(pts, g, px, py, std::min(xa, xb), std::max(xa, xb), std::min(ya, yb), std::max(ya, yb), 0);
    } else if (b > s) {
      double xa = px, xb = px + sx * a, ya = py + sy * s, yb = py + sy * b;
      subdivide(pts, g, px, py, std::min(xa, xb), std::max(xa, xb), std::min(ya, yb), std::max(ya, yb), 0);
    }
    set_offsets(pts, from, px, py);
  }
}

double binom(int a, int b) {  // C(a, b) as a double (b <= a)
  if (b < 0 || b > a) return 0.0;
  long double r = 1;
  for (int i = 1; i <= b; ++i) r = r * (a - b + i) / i;
  return (double)r;
}

}  // namespace

void u_configs(Rel out[NCFG_U]) {
  int c = 0;
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) out[c++] = {(double)dx, (double)dy, 1.0};
  for (int q = 0; q < 4; ++q) {
    int cx = q & 1, cy = q >> 1, ex = cx ? 1 : -1, ey = cy ? 1 : -1;
    const int e[3][2] = {{ex, 0}, {0, ey}, {ex, ey}};
    for (int t = 0; t < 3; ++t)
      out[c++] = {2.0 * e[t][0] - (cx - 0.5), 2.0 * e[t][1] - (cy - 0.5), 2.0};
  }
  for (int b = -1; b <= 2; ++b)
    for (int a = -1; a <= 2; ++a) {
      if (a >= 0 && a <= 1 && b >= 0 && b <= 1) continue;
      out[c++] = {(a + 0.5) / 2 - 0.5, (b + 0.5) / 2 - 0.5, 0.5};
    }
}

void wx_positions(int a[NCFG_W], int b[NCFG_W]) {
  int c = 0;
  for (int j = -2; j <= 3; ++j)
    for (int i = -2; i <= 3; ++i) {
      if (i >= -1 && i <= 2 && j >= -1 && j <= 2) continue;
      a[c] = i;
      b[c] = j;
      ++c;
    }
}

int build_tables(Tables &T, int n, int p, double tol, int nthreads) {
  (void)tol;
  const int P = n * n, nt = p + 1, KP = (nt + 15) / 16 * 16, MR = (3 * P + 1 + 15) / 16 * 16;
  T.n = n; T.P = P; T.p = p; T.nt = nt; T.KP = KP; T.MR = MR;
  Basis B(n);

  // unit-box weights W_j = int over [-1/2,1/2]^2 of L_j
  {
    Rule g = gauss(n);
    std::vector<double> w1(n, 0.0), L(n);
    for (int i = 0; i < n; ++i) {
      B.eval(g.x[i], L.data());
      for (int j = 0; j < n; ++j) w1[j] += g.w[i] * L[j];
    }
    T.wq.assign(P, 0.0);
    for (int j2 = 0; j2 < n; ++j2)
      for (int j1 = 0; j1 < n; ++j1) T.wq[j2 * n + j1] = 0.25 * w1[j1] * w1[j2];
  }

  // ------------------------------------------------------------ near tables
  Rel cfg[NCFG_U];
  u_configs(cfg);
  T.near_.assign((size_t)NCFG_U * MR * P, 0.0);
  {
    const Rule g = gauss(n + 16), gu = gauss(n + 12), gt = gauss(n + 16);
    int nth = nthreads > 0 ? nthreads : (int)std::max(1u, std::thread::hardware_concurrency());
    auto work = [&](int tid) {
      std::vector<QPt> pts;
      std::vector<double> L1(n), L2(n), accV(P), acc1(P), acc2(P);
      for (int job = tid; job < NCFG_U * P; job += nth) {
        int c = job / P, i = job % P;
        double px = 0.5 * B.x[i % n], py = 0.5 * B.x[i / n];
        pts.clear();
        near_points(pts, g, gu, gt, px, py, cfg[c].cx, cfg[c].cy, cfg[c].w);
        std::fill(accV.begin(), accV.end(), 0.0);
        std::fill(acc1.begin(), acc1.end(), 0.0);
        std::fill(acc2.begin(), acc2.end(), 0.0);
        double hs = 0.5 * cfg[c].w;
        for (const QPt &q : pts) {
          double dx = -q.ox, dy = -q.oy, r2 = dx * dx + dy * dy;
          double kv = q.w * 0.5 * std::log(r2) / (2 * kPi), k1 = q.w * dx / (r2 * 2 * kPi),
                 k2 = q.w * dy / (r2 * 2 * kPi);
          B.eval((q.x - cfg[c].cx) / hs, L1.data());
          B.eval((q.y - cfg[c].cy) / hs, L2.data());
          for (int j2 = 0; j2 < n; ++j2) {
            double a = L2[j2];
            for (int j1 = 0; j1 < n; ++j1) {
              double l = a * L1[j1];
              accV[j2 * n + j1] += kv * l;
              acc1[j2 * n + j1] += k1 * l;
              acc2[j2 * n + j1] += k2 * l;
            }
          }
        }
        double *Tc = &T.near_[(size_t)c * MR * P];
        for (int j = 0; j < P; ++j) {
          Tc[(size_t)i * P + j] = accV[j];
          Tc[(size_t)(P + i) * P + j] = acc1[j];
          Tc[(size_t)(2 * P + i) * P + j] = acc2[j];
        }
        if (i == 0)
          for (int j = 0; j < P; ++j) Tc[(size_t)(3 * P) * P + j] = cfg[c].w * cfg[c].w * T.wq[j];
      }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t) th.emplace_back(work, t);
    for (auto &t : th) t.join();
  }

  // ------------------------------------------------------------------- P2M
  // a~_0 = h^2 int f~ dv, a~_k = -(h^2/k) int f~(v) v^k dv, v = (y - c)/h complex.
  T.p2m.assign((size_t)2 * KP * P, 0.0);
  {
    Rule g = gauss((n + p) / 2 + 2);
    std::vector<double> L1(n), L2(n);
    for (size_t b = 0; b < g.x.size(); ++b)
      for (size_t a = 0; a < g.x.size(); ++a) {
        double v1 = 0.5 * g.x[a], v2 = 0.5 * g.x[b], w = 0.25 * g.w[a] * g.w[b];
        B.eval(g.x[a], L1.data());
        B.eval(g.x[b], L2.data());
        cd v(v1, v2), vk(1, 0);
        for (int k = 0; k < nt; ++k) {
          cd c = k == 0 ? cd(1, 0) : -vk / (double)k;
          for (int j2 = 0; j2 < n; ++j2)
            for (int j1 = 0; j1 < n; ++j1) {
              double l = w * L1[j1] * L2[j2];
              T.p2m[(size_t)k * P + j2 * n + j1] += l * c.real();
              T.p2m[(size_t)(KP + k) * P + j2 * n + j1] += l * c.imag();
            }
          vk *= v;
        }
      }
  }

  // ------------------------------------------------------------- M2M, L2L
  T.m2m.assign((size_t)4 * nt * nt * 2, 0.0);
  T.l2l.assign((size_t)4 * nt * nt * 2, 0.0);
  for (int c = 0; c < 4; ++c) {
    cld w((c & 1) - 0.5L, (c >> 1) - 0.5L);   // child centre - parent centre, in child widths
    std::vector<cld> wp(nt + 1);
    wp[0] = 1;
    for (int k = 1; k <= nt; ++k) wp[k] = wp[k - 1] * w;
    double *M = &T.m2m[(size_t)c * nt * nt * 2], *Lm = &T.l2l[(size_t)c * nt * nt * 2];
    for (int l = 0; l < nt; ++l) {
      for (int k = 0; k < nt; ++k) {
        cld v = 0;
        if (l == 0 && k == 0) v = 1;
        else if (k == 0) v = -std::pow(w / 2.0L, l) / (long double)l;
        else if (k <= l) v = (long double)binom(l - 1, k - 1) * wp[l - k] * std::ldexp(1.0L, -l);
        M[((size_t)l * nt + k) * 2] = (double)v.real();
        M[((size_t)l * nt + k) * 2 + 1] = (double)v.imag();
        // L2L: child m from parent l: C(l, m) w^(l-m) 2^-l, here row m = l_, column = k_
        cld u = 0;
        int m = l, lp = k;
        if (lp >= m) u = (long double)binom(lp, m) * wp[lp - m] * std::ldexp(1.0L, -lp);
        Lm[((size_t)m * nt + lp) * 2] = (double)u.real();
        Lm[((size_t)m * nt + lp) * 2 + 1] = (double)u.imag();
      }
    }
  }

  // ------------------------------------------------------------------ M2L
  // b~_l = (d/2)^-l sum_k H[l][k] y_k + [l = 0] a_0 (log h + log|d|),
  // y_0 = a_0, y_k = a~_k (-d/2)^-k, H[l][k] = C(k+l-1, k-1) 2^-(k+l),
  // H[l][0] = -2^-l / l (l >= 1), H[0][0] = 0.
  T.H.assign((size_t)KP * KP, 0.0);
  for (int l = 0; l < nt; ++l)
    for (int k = 0; k < nt; ++k) {
      double v = 0;
      if (k >= 1) v = binom(k + l - 1, k - 1) * std::ldexp(1.0, -(k + l));
      else if (l >= 1) v = -std::ldexp(1.0, -l) / l;
      T.H[(size_t)l * KP + k] = v;
    }
  T.pw_src.assign((size_t)NOFF * KP * 2, 0.0);
  T.pw_tgt.assign((size_t)NOFF * KP * 2, 0.0);
  T.logd.assign(NOFF, 0.0);
  for (int o = 0; o < NOFF; ++o) {
    int dx = o % 7 - 3, dy = o / 7 - 3;
    if (std::max(std::abs(dx), std::abs(dy)) < 2) continue;
    cld h(dx / 2.0L, dy / 2.0L), is = -1.0L / h, it = 1.0L / h, ps = 1, pt = 1;
    for (int k = 0; k < nt; ++k) {
      T.pw_src[((size_t)o * KP + k) * 2] = (double)ps.real();
      T.pw_src[((size_t)o * KP + k) * 2 + 1] = (double)ps.imag();
      T.pw_tgt[((size_t)o * KP + k) * 2] = (double)pt.real();
      T.pw_tgt[((size_t)o * KP + k) * 2 + 1] = (double)pt.imag();
      ps *= is;
      pt *= it;
    }
    T.logd[o] = 0.5 * std::log((double)(dx * dx + dy * dy));
  }

  // ------------------------------------------------------------------ L2T
  // V = Re psi / 2pi, d1 V - i d2 V = psi' / 2pi, psi(z) = sum b~_l u^l, u = (z - c)/h.
  T.l2t.assign((size_t)3 * P * 2 * KP, 0.0);
  for (int i = 0; i < P; ++i) {
    cld u(0.5L * B.x[i % n], 0.5L * B.x[i / n]), up = 1, um = 0;
    double *RV = &T.l2t[(size_t)i * 2 * KP], *R1 = &T.l2t[(size_t)(P + i) * 2 * KP],
           *R2 = &T.l2t[(size_t)(2 * P + i) * 2 * KP];
    for (int l = 0; l < nt; ++l) {  // up = u^l, um = u^(l-1)
      RV[l] = (double)(up.real() / (2 * kPi));
      RV[KP + l] = (double)(-up.imag() / (2 * kPi));
      if (l >= 1) {
        R1[l] = (double)(l * um.real() / (2 * kPi));
        R1[KP + l] = (double)(-l * um.imag() / (2 * kPi));
        R2[l] = (double)(-l * um.imag() / (2 * kPi));
        R2[KP + l] = (double)(-l * um.real() / (2 * kPi));
      }
      um = up;
      up *= u;
    }
  }

  // -------------------------------------------------------------- M2T (W)
  // phi(z) = a_0 log(z - c_s) + sum a~_k e^-k, e = (z - c_s)/h_s, h_s = h/2;
  // the a_0 log h_s term and the 1/h_s of the gradient are applied at run time.
  int pa[NCFG_W], pb[NCFG_W];
  wx_positions(pa, pb);
  T.m2t.assign((size_t)NCFG_W * 3 * P * 2 * KP, 0.0);
  for (int c = 0; c < NCFG_W; ++c) {
    long double scx = (pa[c] + 0.5L) / 2 - 0.5L, scy = (pb[c] + 0.5L) / 2 - 0.5L;
    for (int i = 0; i < P; ++i) {
      cld e(2.0L * (0.5L * B.x[i % n] - scx), 2.0L * (0.5L * B.x[i / n] - scy));
      cld ie = 1.0L / e, pk = ie;   // pk = e^-k
      double *RV = &T.m2t[(((size_t)c * 3 * P) + i) * 2 * KP];
      double *R1 = &T.m2t[(((size_t)c * 3 * P) + P + i) * 2 * KP];
      double *R2 = &T.m2t[(((size_t)c * 3 * P) + 2 * P + i) * 2 * KP];
      RV[0] = (double)(std::log(std::abs(e)) / (2 * kPi));
      R1[0] = (double)(ie.real() / (2 * kPi));
      R2[0] = (double)(-ie.imag() / (2 * kPi));
      for (int k = 1; k < nt; ++k) {
        cld pk1 = pk * ie;   // e^-(k+1)
        RV[k] = (double)(pk.real() / (2 * kPi));
        RV[KP + k] = (double)(-pk.imag() / (2 * kPi));
        R1[k] = (double)(-k * pk1.real() / (2 * kPi));
        R1[KP + k] = (double)(k * pk1.imag() / (2 * kPi));
        R2[k] = (double)(k * pk1.imag() / (2 * kPi));
        R2[KP + k] = (double)(k * pk1.real() / (2 * kPi));
        pk = pk1;
      }
    }
  }

  // -------------------------------------------------------------- P2L (X)
  // b~_0 = h^2 [4 int f~ log|d + 2v| dv] + h^2 log h (4 W.f),
  // b~_l = -(4 h^2 / l) int f~(v) (d + 2v)^-l dv, d = (c_C - c_t)/h.
  T.p2l.assign((size_t)NCFG_X * 2 * KP * P, 0.0);
  {
    Rule g = gauss(24);
    std::vector<double> L1(n), L2(n);
    const int S = 4;   // 4 x 4 composite panels over the unit source box
    for (int c = 0; c < NCFG_X; ++c) {
      long double d1 = 0.5L - pa[c], d2 = 0.5L - pb[c];
      double *R = &T.p2l[(size_t)c * 2 * KP * P];
      for (int sj = 0; sj < S; ++sj)
        for (int si = 0; si < S; ++si)
          for (size_t b = 0; b < g.x.size(); ++b)
            for (size_t a = 0; a < g.x.size(); ++a) {
              double v1 = -0.5 + (si + 0.5 + 0.5 * g.x[a]) / S, v2 = -0.5 + (sj + 0.5 + 0.5 * g.x[b]) / S;
              double w = g.w[a] * g.w[b] * 0.25 / (S * S);
              B.eval(2 * v1, L1.data());
              B.eval(2 * v2, L2.data());
              cld z(d1 + 2.0L * v1, d2 + 2.0L * v2), iz = 1.0L / z, pz = iz;
              std::vector<cd> gl(nt);
              gl[0] = cd((double)(4.0L * std::log(std::abs(z))), 0.0);
              for (int l = 1; l < nt; ++l) {
                gl[l] = cd((double)(-4.0L / l * pz.real()), (double)(-4.0L / l * pz.imag()));
                pz *= iz;
              }
              for (int j2 = 0; j2 < n; ++j2)
                for (int j1 = 0; j1 < n; ++j1) {
                  double lw = w * L1[j1] * L2[j2];
                  for (int l = 0; l < nt; ++l) {
                    R[(size_t)l * P + j2 * n + j1] += lw * gl[l].real();
                    R[(size_t)(KP + l) * P + j2 * n + j1] += lw * gl[l].imag();
                  }
                }
            }
    }
  }
  return BX_OK;
}

LeafFragLayout leaf_frag_layout(int n, int p) {
  LeafFragLayout L;
  const int P = n * n, KP = (p + 1 + 15) / 16 * 16;
  L.MTR = (3 * P / 16 + 3) / 4 * 4;                // padded to whole groups of 4 row tiles
  // chunk width: a divisor of both K = P (near tables) and K = 2 KP (expansions)
  L.KC = P == 16 ? 16 : (P == 64 && (2 * KP) % 64 == 0 ? 64 : 32);
  L.KMAX = std::max(P, 2 * KP);
  L.near0 = 0;
  L.near_step = (int64_t)L.MTR * P * 16;           // MTR tiles x K/4 steps x 64 lanes
  L.l2t = L.near0 + NCFG_U * L.near_step;
  L.w_step = (int64_t)L.MTR * 2 * KP * 16;
  L.w0 = L.l2t + L.w_step;
  L.total = L.w0 + NCFG_W * L.w_step;
  return L;
}

namespace {
// Append the MFMA A fragments of a rows x K matrix (element (i, k) = a(i, k)),
// row tiles of 16, K in chunks of KC, within a chunk k = (lane / 16) * KSC + ks.
template <class F>
void append_frag_chunked(std::vector<double> &out, int MT, int K, int KC, F a, bool permute_rows = false) {
  const int NC = K / KC, KSC = KC / 4;
  for (int mt = 0; mt < MT; ++mt)
    for (int c = 0; c < NC; ++c)
      for (int ks = 0; ks < KSC; ++ks)
        for (int lane = 0; lane < 64; ++lane) {
          const int m = lane & 15, row = permute_rows ? 4 * (m % 4) + m / 4 : m;
          out.push_back(a(mt * 16 + row, c * KC + (lane >> 4) * KSC + ks));
        }
}
template <class F>
void append_frag(std::vector<double> &out, int MT, int K, F a) {
  append_frag_chunked(out, MT, K, K, a);
}
}  // namespace

void build_leaf_frag(const Tables &T, std::vector<double> &out, std::vector<double> &mass) {
  const LeafFragLayout L = leaf_frag_layout(T.n, T.p);
  const int P = T.P, KP = T.KP, MR = T.MR, K2 = 2 * KP;
  out.clear();
  out.reserve(L.total);
  mass.assign((size_t)(NCFG_U + 1 + NCFG_W) * L.KMAX, 0.0);
  for (int c = 0; c < NCFG_U; ++c) {
    const double *A = &T.near_[(size_t)c * MR * P];
    append_frag_chunked(out, L.MTR, P, L.KC, [&](int i, int k) { return i < 3 * P ? A[(size_t)i * P + k] : 0.0; },
                        true);
    for (int k = 0; k < P; ++k) mass[(size_t)c * L.KMAX + k] = A[(size_t)3 * P * P + k];
  }
  // expansion columns are stored interleaved (Re b_m, Im b_m) as in device memory
  append_frag_chunked(out, L.MTR, K2, L.KC, [&](int i, int k) {
    return i < 3 * P ? T.l2t[(size_t)i * K2 + (k & 1) * KP + k / 2] : 0.0;
  }, true);
  // W: V rows carry log|e| - log 2 in the a_0 column (log(h/2) = log h - log 2, the
  // log h part comes through the mass weight on a_0), gradient rows are doubled (1/(h/2)).
  const double log2_2pi = std::log(2.0) / (2 * 3.14159265358979323846);
  for (int c = 0; c < NCFG_W; ++c) {
    const double *A = &T.m2t[(size_t)c * 3 * P * K2];
    append_frag_chunked(out, L.MTR, K2, L.KC, [&](int i, int k) {
      if (i >= 3 * P) return 0.0;
      double v = A[(size_t)i * K2 + (k & 1) * KP + k / 2];
      if (i < P && k == 0) v -= log2_2pi;
      if (i >= P) v *= 2.0;
      return v;
    }, true);
    mass[(size_t)(NCFG_U + 1 + c) * L.KMAX + 0] = 1.0;
  }
}

void build_split_tables(const Tables &T, SplitTables &S) {
  const int P = T.P, MR = T.MR, R = 3 * P, MTR = R / 16, NCH = P / 64;
  Rel cfg[NCFG_U];
  u_configs(cfg);
  S.cfg_w2.resize(NCFG_U);
  for (int c = 0; c < NCFG_U; ++c) S.cfg_w2[c] = cfg[c].w * cfg[c].w;
  auto X = [&](int c, int r, int k) { return T.near_[((size_t)c * MR + r) * P + k]; };
  // row scales 2^E_r with max |x| <= 2^E_r * 127.5/128, so that the leading
  // rounded slice stays within [-127, 127]
  S.row_scale.assign(R, 1.0);
  for (int r = 0; r < R; ++r) {
    double m = 0.0;
    for (int c = 0; c < NCFG_U; ++c)
      for (int k = 0; k < P; ++k) m = std::max(m, std::fabs(X(c, r, k)));
    if (m == 0.0) continue;
    int e;
    const double fr = std::frexp(m, &e);
    if (fr * 128.0 >= 127.5) ++e;
    S.row_scale[r] = std::ldexp(1.0, e);
  }
  // slices: x / 2^E_r = sum_a t_a 2^-7(a+1) + residual, t_a = nearest integers
  // (|t_0| <= 127, |t_a| <= 64 after), and for each row the sums over all
  // configurations and k of |t_a|, of |x - X_s| and of |X_s| (X_s: s slices)
  std::vector<double> sum_t((size_t)R * SPLIT_SMAX, 0.0), sum_res((size_t)R * (SPLIT_SMAX + 1), 0.0),
      sum_abs((size_t)R * (SPLIT_SMAX + 1), 0.0);
  S.a.assign((size_t)NCFG_U * SPLIT_SMAX * MTR * NCH * 64 * 16, 0);
  for (int c = 0; c < NCFG_U; ++c)
    for (int r = 0; r < R; ++r)
      for (int k = 0; k < P; ++k) {
        const double x = X(c, r, k), E = S.row_scale[r];
        double v = x / E, approx = 0.0;
        const int mt = r / 16, i = r % 16, ch = k / 64, kk = k % 64, lane = i + 16 * (kk / 16), e = kk % 16;
        for (int a = 0; a < SPLIT_SMAX; ++a) {
          const double sc = v * 128.0, t = std::nearbyint(sc);
          v = sc - t;
          S.a[(((((size_t)c * SPLIT_SMAX + a) * MTR + mt) * NCH + ch) * 64 + lane) * 16 + e] = (int8_t)t;
          sum_t[(size_t)r * SPLIT_SMAX + a] += std::fabs(t);
          approx += t * std::ldexp(E, -7 * (a + 1));
          sum_res[(size_t)r * (SPLIT_SMAX + 1) + a + 1] += std::fabs(x - approx);
          sum_abs[(size_t)r * (SPLIT_SMAX + 1) + a + 1] += std::fabs(approx);
        }
      }
  // error bound per slice count s, for samples |y| < 1 rounded to s slices the
  // same way: table residual + sample residual (<= 2^-7s / 2 per sample) + the
  // dropped pairs a + b >= s (a, b < s; |s_0| <= 127, |s_b| <= 64 after)
  S.err_v.assign(SPLIT_SMAX + 1, 0.0);
  S.err_d.assign(SPLIT_SMAX + 1, 0.0);
  for (int sn = 1; sn <= SPLIT_SMAX; ++sn)
    for (int r = 0; r < R; ++r) {
      double e = sum_res[(size_t)r * (SPLIT_SMAX + 1) + sn] +
                 sum_abs[(size_t)r * (SPLIT_SMAX + 1) + sn] * 0.5 * std::ldexp(1.0, -7 * sn);
      for (int a = 0; a < sn; ++a)
        for (int b = sn - a; b < sn; ++b)
          e += sum_t[(size_t)r * SPLIT_SMAX + a] * std::ldexp(S.row_scale[r], -7 * (a + 1)) * (b == 0 ? 127.0 : 64.0) *
               std::ldexp(1.0, -7 * (b + 1));
      double &dst = r < P ? S.err_v[sn] : S.err_d[sn];
      dst = std::max(dst, e);
    }
}

int split_slices(const SplitTables &S, int level, double tol, bool grad_rows) {
  // the sample scale 2^Ef is at most 2 (128/127.5) max |f|; values carry h^2,
  // gradients h (h = 2^-level of the root width)
  const double h = std::ldexp(1.0, -level), fs = 2.0 * 128.0 / 127.5;
  for (int sn = 1; sn <= SPLIT_SG; ++sn) {
    const double e = (grad_rows ? h * S.err_d[sn] : h * h * S.err_v[sn]) * fs;
    if (e <= tol) return sn;
  }
  return 0;
}

void build_p2m_frag(const Tables &T, std::vector<double> &out) {
  out.clear();
  append_frag(out, 2 * T.KP / 16, T.P, [&](int i, int k) { return T.p2m[(size_t)i * T.P + k]; });
}

// Real form of a complex coefficient map on interleaved (Re, Im) vectors.
static double cplx_entry(double orr, double oi, int po, int pi) {
  return po == pi ? orr : (po == 0 ? -oi : oi);
}

void build_m2m_frag(const Tables &T, std::vector<double> &out) {
  const int R = 2 * T.KP, nt = T.nt;
  out.clear();
  for (int c = 0; c < 4; ++c)
    append_frag(out, R / 16, R, [&](int o, int i) {
      const int l = o / 2, kk = i / 2;
      if (l >= nt || kk >= nt) return 0.0;
      const double *op = &T.m2m[(((size_t)c * nt + l) * nt + kk) * 2];
      return cplx_entry(op[0], op[1], o & 1, i & 1);
    });
}

void build_l2l_frag(const Tables &T, std::vector<double> &out) {
  const int R = 2 * T.KP, nt = T.nt;
  out.clear();
  for (int c = 0; c < 4; ++c)
    append_frag(out, R / 16, R, [&](int o, int i) {
      const int m = o / 2, l = i / 2;
      if (m >= nt || l >= nt) return 0.0;
      const double *op = &T.l2l[(((size_t)c * nt + m) * nt + l) * 2];
      return cplx_entry(op[0], op[1], o & 1, i & 1);
    });
}

void build_p2l_frag(const Tables &T, std::vector<double> &out) {
  const int R = 2 * T.KP, KP = T.KP, P = T.P;
  out.clear();
  for (int c = 0; c < NCFG_X; ++c)
    append_frag(out, (R + 16) / 16, P, [&](int o, int j) {
      if (o < R) return T.p2l[((size_t)c * 2 * KP + (o & 1) * KP + o / 2) * P + j];
      return o == R ? 4.0 * T.wq[j] : 0.0;
    });
}

uint64_t tables_checksum(const Tables &T) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const std::vector<double> &v) {
    const unsigned char *p = (const unsigned char *)v.data();
    for (size_t i = 0; i < v.size() * sizeof(double); ++i) h = (h ^ p[i]) * 1099511628211ull;
  };
  mix(T.wq); mix(T.near_); mix(T.p2m); mix(T.m2m); mix(T.l2l); mix(T.H);
  mix(T.pw_src); mix(T.pw_tgt); mix(T.logd); mix(T.l2t); mix(T.m2t); mix(T.p2l);
  return h;
}

namespace {
const uint32_t kMagic = 0x42584654u;   // table file tag
const uint32_t kVersion = 1;
std::vector<std::vector<double> *> fields(Tables &T) {
  return {&T.wq, &T.near_, &T.p2m, &T.m2m, &T.l2l, &T.H, &T.pw_src, &T.pw_tgt, &T.logd, &T.l2t, &T.m2t, &T.p2l};
}
}  // namespace

bool save_tables(const Tables &T, const std::string &path) {
  std::string tmp = path + ".tmp";
  std::ofstream f(tmp, std::ios::binary);
  if (!f) return false;
  uint32_t hdr[4] = {kMagic, kVersion, (uint32_t)T.n, (uint32_t)T.p};
  f.write((const char *)hdr, sizeof hdr);
  for (auto *v : fields(const_cast<Tables &>(T))) {
    uint64_t m = v->size();
    f.write((const char *)&m, 8);
    f.write((const char *)v->data(), m * sizeof(double));
  }
  uint64_t cs = tables_checksum(T);
  f.write((const char *)&cs, 8);
  f.close();
  if (!f) return false;
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}

bool load_tables(Tables &T, const std::string &path, int n, int p) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  uint32_t hdr[4];
  f.read((char *)hdr, sizeof hdr);
  if (!f || hdr[0] != kMagic || hdr[1] != kVersion || (int)hdr[2] != n || (int)hdr[3] != p) return false;
  Tables R;
  R.n = n; R.P = n * n; R.p = p; R.nt = p + 1; R.KP = (R.nt + 15) / 16 * 16;
  R.MR = (3 * R.P + 1 + 15) / 16 * 16;
  for (auto *v : fields(R)) {
    uint64_t m = 0;
    f.read((char *)&m, 8);
    if (!f || m > (uint64_t)1 << 32) return false;
    v->resize(m);
    f.read((char *)v->data(), m * sizeof(double));
    if (!f) return false;
  }
  uint64_t cs = 0;
  f.read((char *)&cs, 8);
  if (!f || cs != tables_checksum(R)) return false;
  if (R.near_.size() != (size_t)NCFG_U * R.MR * R.P || R.p2m.size() != (size_t)2 * R.KP * R.P) return false;
  T = std::move(R);
  return true;
}

}  // namespace bx
