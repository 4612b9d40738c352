"""CPU FP64 oracle for the box-code volume potential (test infrastructure).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  It shares no code with the HIP library.

It computes, at arbitrary targets x, the plain definition (section 3,
eq. volumeint3, with the piecewise polynomial f~ of section 3.1 and the
gradient integral eq. volumeint3x):

    V(x) = sum_B int_B G(x-y) f~_B(y) dy,   grad V(x) = sum_B int_B grad G(x-y) f~_B(y) dy,
    G(r) = log|r| / (2 pi),

summing every leaf directly (see oracle.c for the quadrature).  The nodes at
which the samples live are the oracle's own first-kind Chebyshev points.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from math import comb

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (OpenMP) into liboracle.so next to it."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_volume.restype = ctypes.c_int
        lib.oracle_volume.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, ip, ip, ip, dp, ctypes.c_void_p, ctypes.c_int, dp, dp,
                                      ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, ctypes.c_int]
        lib.oracle_leaf_mass.restype = ctypes.c_int
        lib.oracle_leaf_mass.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ip, dp, dp]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


# ------------------------------------------------------------------ rules
def cheb_nodes(n: int) -> np.ndarray:
    """First-kind Chebyshev points -cos((2j+1) pi / 2n), increasing."""
    j = np.arange(n)
    return -np.cos((2 * j + 1) * np.pi / (2 * n))


def gauss_legendre01(q: int):
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_log01(q: int):
    """q-point Gauss rule for int_0^1 (-log t) g(t) dt (exact for degree 2q-1).

    Recurrence coefficients by the modified Chebyshev algorithm from the
    modified moments int_0^1 -log(t) P_k(2t-1) dt = 1 (k=0), (-1)^k/(k(k+1))
    (k>=1), taken with respect to the monic shifted Legendre polynomials;
    nodes and weights by the Golub-Welsch eigenvalue method.
    """
    N = q
    nu = np.zeros(2 * N)
    for k in range(2 * N):
        m = 1.0 if k == 0 else (-1.0) ** k / (k * (k + 1.0))
        nu[k] = m / comb(2 * k, k)                 # monic normalisation
    a = np.full(2 * N, 0.5)
    b = np.array([0.0] + [l * l / (4.0 * (4.0 * l * l - 1.0)) for l in range(1, 2 * N)])
    alpha = np.zeros(N)
    beta = np.zeros(N)
    sig_prev = np.zeros(2 * N + 1)
    sig = nu.copy()
    alpha[0] = a[0] + nu[1] / nu[0]
    beta[0] = nu[0]
    for k in range(1, N):
        new = np.zeros(2 * N)
        for l in range(k, 2 * N - k):
            new[l] = (sig[l + 1] - (alpha[k - 1] - a[l]) * sig[l] - beta[k - 1] * sig_prev[l]
                      + b[l] * sig[l - 1])
        alpha[k] = a[k] + new[k + 1] / new[k] - sig[k] / sig[k - 1]
        beta[k] = new[k] / sig[k - 1]
        sig_prev, sig = sig, new
    J = np.diag(alpha) + np.diag(np.sqrt(beta[1:]), 1) + np.diag(np.sqrt(beta[1:]), -1)
    t, V = np.linalg.eigh(J)
    w = beta[0] * V[0, :] ** 2
    return t, w


# ------------------------------------------------------------------ trees
def leaf_nodes(level, ix, iy, n, cx=0.0, cy=0.0, width=1.0):
    """Coordinates of each leaf's nodes, [N_L, n, n] each, x index fastest."""
    level = np.asarray(level, np.int64)
    h = width * np.ldexp(1.0, -level)
    x0 = cx - 0.5 * width + np.asarray(ix) * h
    y0 = cy - 0.5 * width + np.asarray(iy) * h
    xi = cheb_nodes(n)
    X = (x0 + 0.5 * h)[:, None, None] + 0.5 * h[:, None, None] * xi[None, None, :] + 0.0 * xi[None, :, None]
    Y = (y0 + 0.5 * h)[:, None, None] + 0.5 * h[:, None, None] * xi[None, :, None] + 0.0 * xi[None, None, :]
    return X, Y


def volume(level, ix, iy, f, tx, ty, n=None, cx=0.0, cy=0.0, width=1.0, use=None, threads=0):
    """V, dV/dx1, dV/dx2 of the piecewise polynomial source at targets (tx, ty)."""
    lib = _load()
    f = np.ascontiguousarray(f, np.float64)
    nleaf = f.shape[0]
    if n is None:
        n = f.shape[1]
    lv = np.ascontiguousarray(level, np.int32)
    xs = np.ascontiguousarray(ix, np.int32)
    ys = np.ascontiguousarray(iy, np.int32)
    tx = np.ascontiguousarray(np.ravel(tx), np.float64)
    ty = np.ascontiguousarray(np.ravel(ty), np.float64)
    nr = n + 2
    gt, gw = gauss_legendre01(nr)
    lt, lw = gauss_log01(nr)
    gt, gw, lt, lw = (np.ascontiguousarray(v) for v in (gt, gw, lt, lw))
    V = np.zeros(tx.size)
    Gx = np.zeros(tx.size)
    Gy = np.zeros(tx.size)
    usep = None
    if use is not None:
        use = np.ascontiguousarray(use, np.uint8)
        usep = use.ctypes.data
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ipp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    rc = lib.oracle_volume(int(n), float(cx), float(cy), float(width), int(nleaf), ipp(lv), ipp(xs),
                           ipp(ys), dp(f), usep, int(tx.size), dp(tx), dp(ty), int(nr), dp(gt), dp(gw),
                           dp(lt), dp(lw), dp(V), dp(Gx), dp(Gy), int(threads))
    if rc != 0:
        raise ValueError("oracle_volume: bad arguments")
    return V, Gx, Gy


def volume_at_nodes(level, ix, iy, f, leaves=None, n=None, cx=0.0, cy=0.0, width=1.0, use=None,
                    threads=0):
    """Oracle at every node of the given leaves (all by default): arrays [k, n, n]."""
    f = np.asarray(f)
    if n is None:
        n = f.shape[1]
    X, Y = leaf_nodes(level, ix, iy, n, cx, cy, width)
    if leaves is not None:
        X, Y = X[leaves], Y[leaves]
    V, Gx, Gy = volume(level, ix, iy, f, X.ravel(), Y.ravel(), n, cx, cy, width, use, threads)
    shp = X.shape
    return V.reshape(shp), Gx.reshape(shp), Gy.reshape(shp)


def leaf_mass(level, f, width=1.0):
    """Exact integral of f~ over each leaf."""
    lib = _load()
    f = np.ascontiguousarray(f, np.float64)
    lv = np.ascontiguousarray(level, np.int32)
    out = np.zeros(f.shape[0])
    rc = lib.oracle_leaf_mass(int(f.shape[1]), float(width), int(f.shape[0]),
                              lv.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                              f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError("oracle_leaf_mass: bad arguments")
    return out


def num_threads() -> int:
    return int(_load().oracle_num_threads())
