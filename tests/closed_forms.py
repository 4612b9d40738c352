"""Closed-form potentials used as pins (derived from the mathematics, not from the code under test).

G(r) = log|r| / (2 pi).

* Constant source on a rectangle: V(x) = (1/2pi) int log|x-y| dy over [x0,x1]x[y0,y1].
  With u = y1 - x1, v = y2 - x2 the mixed antiderivative of log(u^2+v^2)/2 is
  F(u,v)/2 with F = u v (log(u^2+v^2) - 3) + u^2 atan(v/u) + v^2 atan(u/v), so
  V = (1/4pi) sum over corners of +-F (inclusion-exclusion).  For the gradient,
  dV/dx1 = -(1/2pi) int u/(u^2+v^2), whose mixed antiderivative is
  H(u,v) = u atan(v/u) + (v/2) log(u^2+v^2).
* Radial Gaussian f = exp(-r^2/s^2) on the whole plane:
  V(r) = (s^2/2) log r + (s^2/4) E1(r^2/s^2),  V'(r) = (s^2 / 2r) (1 - exp(-r^2/s^2)).
"""
import numpy as np
from scipy.special import exp1


def _F(u, v):
    return u * v * (np.log(u * u + v * v) - 3.0) + u * u * np.arctan(v / u) + v * v * np.arctan(u / v)


def _H(u, v):
    return u * np.arctan(v / u) + 0.5 * v * np.log(u * u + v * v)


def const_rect(x, y, x0, x1, y0, y1):
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    V = np.zeros_like(x)
    gx = np.zeros_like(x)
    gy = np.zeros_like(x)
    for yy, sy in ((y1, 1.0), (y0, -1.0)):
        for xx, sx in ((x1, 1.0), (x0, -1.0)):
            u, v, s = xx - x, yy - y, sx * sy
            V += s * _F(u, v) / (4.0 * np.pi)
            gx -= s * _H(u, v) / (2.0 * np.pi)
            gy -= s * _H(v, u) / (2.0 * np.pi)
    return V, gx, gy


def radial_gaussian(x, y, s, cx=0.0, cy=0.0):
    dx = np.asarray(x, float) - cx
    dy = np.asarray(y, float) - cy
    r2 = dx * dx + dy * dy
    r = np.sqrt(r2)
    V = 0.25 * s * s * np.log(r2) + 0.25 * s * s * exp1(r2 / (s * s))
    dVdr_over_r = 0.5 * s * s * (-np.expm1(-r2 / (s * s))) / r2
    return V, dVdr_over_r * dx, dVdr_over_r * dy
