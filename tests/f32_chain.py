"""Float32 evaluations of the Harris chain in numpy, in several summation orders.

Test code only: every numpy operation on float32 arrays rounds once to nearest, so these
are honest float32 evaluations (no FMA, no wider intermediates).  They exercise the
oracle's rounding-error bound, which must hold for every evaluation order a kernel may use.
"""
from __future__ import annotations

import numpy as np

F = np.float32


def shifted(A, dx, dy):
    """A(x+dx, y+dy) with clamped indices (the closest pixel inside)."""
    H, W = A.shape
    yy = np.clip(np.arange(H) + dy, 0, H - 1)
    xx = np.clip(np.arange(W) + dx, 0, W - 1)
    return A[yy][:, xx]


def sobel(X, order):
    """(Ix, Iy) with s = (1,2,1), d = (-1,0,1): nine terms summed in row-major order ("dir"),
    reversed ("rev"), or separably (smooth across, then difference: "sep")."""
    if order == "sep":
        V = shifted(X, 0, -1) + F(2) * X + shifted(X, 0, 1)
        Hs = shifted(X, -1, 0) + F(2) * X + shifted(X, 1, 0)
        return shifted(V, 1, 0) - shifted(V, -1, 0), shifted(Hs, 0, 1) - shifted(Hs, 0, -1)
    s, d = (1, 2, 1), (-1, 0, 1)
    tx, ty = [], []
    for j in (-1, 0, 1):
        for i in (-1, 0, 1):
            p = shifted(X, i, j)
            tx.append(F(s[j + 1] * d[i + 1]) * p)
            ty.append(F(d[j + 1] * s[i + 1]) * p)
    if order == "rev":
        tx, ty = tx[::-1], ty[::-1]
    ix, iy = np.zeros_like(X), np.zeros_like(X)
    for a, b in zip(tx, ty):
        ix = ix + a
        iy = iy + b
    return ix, iy


def window(A, g, order):
    """sum g_j g_i A(x+i, y+j): with float32 weights g_j * g_i in row-major ("dir") or reversed
    ("rev") order, or as a row pass followed by a column pass ("sep")."""
    rg = (len(g) - 1) // 2
    if order == "sep":
        Hs = np.zeros_like(A)
        for i in range(-rg, rg + 1):
            Hs = Hs + g[i + rg] * shifted(A, i, 0)
        S = np.zeros_like(A)
        for j in range(-rg, rg + 1):
            S = S + g[j + rg] * shifted(Hs, 0, j)
        return S
    idx = [(j, i) for j in range(-rg, rg + 1) for i in range(-rg, rg + 1)]
    if order == "rev":
        idx = idx[::-1]
    S = np.zeros_like(A)
    for j, i in idx:
        S = S + (g[j + rg] * g[i + rg]) * shifted(A, i, j)
    return S


def harris32(X, g, k, sobel_order="dir", window_order="dir", response_order=0):
    X, g, k = np.asarray(X, F), np.asarray(g, F), F(k)
    ix, iy = sobel(X, sobel_order)
    A, B, C = ix * ix, iy * iy, ix * iy
    sxx, syy, sxy = window(A, g, window_order), window(B, g, window_order), window(C, g, window_order)
    tr = sxx + syy
    if response_order == 0:
        return (sxx * syy - sxy * sxy) - k * tr * tr
    return sxx * syy - (sxy * sxy + (k * tr) * tr)


ORDERS = [(so, wo, ro) for so in ("dir", "sep", "rev") for wo in ("dir", "sep", "rev") for ro in (0, 1)]
