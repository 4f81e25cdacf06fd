"""Closed forms and brute-force references that pin the oracle.

None of these calls the oracle or repeats its loops: they compute the same
mathematical objects by independent routes.

* Uniform diffusivity: one explicit sub-step of the 7-point scheme moves the
  unit mass like a lazy random walk (stay with probability 1 - 6*lam, step to
  each of the six neighbours with probability lam).  After n sub-steps the
  free-space kernel is a multinomial mixture of products of 1-D +-1 walks:

     G_n(a,b,c) = sum_{mx+my+mz <= n} n! / ((n-m)! mx! my! mz!)
                  (1-6 lam)^(n-m) (2 lam)^m  w_mx(a) w_my(b) w_mz(c)

  with m = mx+my+mz and w_k(a) = C(k, (k+a)/2) 2^-k (0 if |a| > k or the
  parities differ).  A move that would cross a no-flux wall leaves the mass in
  place, which is the method of images: fold every axis position p onto a box of
  length L by y = p mod 2L, y >= L -> 2L-1-y.  Folding is linear and acts per
  axis, so the box kernel is the same mixture of the folded 1-D walks.

* Tiny domains: the whole-domain operator A = I + (weighted graph Laplacian) as
  a dense matrix, and P = A^n by repeated matrix products (float or exact
  rationals).
"""
from __future__ import annotations

from fractions import Fraction
from math import comb, lgamma, log, exp

import numpy as np


def walk_1d(k: int, L: int, pos: int) -> np.ndarray:
    """Distribution of a k-move +-1 walk started at ``pos`` in a box of length
    L with reflecting (stay-in-place) walls, by image folding."""
    out = np.zeros(L)
    for j in range(k + 1):                  # j moves to the right
        a = 2 * j - k
        p = pos + a
        y = p % (2 * L)
        if y >= L:
            y = 2 * L - 1 - y
        out[y] += comb(k, j) * 2.0 ** (-k)
    return out


def uniform_box_kernel(n: int, lam: float, box, src) -> np.ndarray:
    """Kernel after n sub-steps of uniform lam in a box (bz, by, bx) with the
    unit source at src = (z, y, x); reflecting walls on all sides."""
    bz, by, bx = box
    sz, sy, sx = src
    fx = np.array([walk_1d(k, bx, sx) for k in range(n + 1)])      # [n+1, bx]
    fy = np.array([walk_1d(k, by, sy) for k in range(n + 1)])
    fz = np.array([walk_1d(k, bz, sz) for k in range(n + 1)])
    C = np.zeros((n + 1, n + 1, n + 1))
    stay = 1.0 - 6.0 * lam
    for mx in range(n + 1):
        for my in range(n + 1 - mx):
            for mz in range(n + 1 - mx - my):
                m = mx + my + mz
                lc = (lgamma(n + 1) - lgamma(n - m + 1) - lgamma(mx + 1) - lgamma(my + 1)
                      - lgamma(mz + 1))
                term = m * log(2.0 * lam)
                if n - m > 0:
                    if stay <= 0.0:
                        continue
                    term += (n - m) * log(stay)
                C[mx, my, mz] = exp(lc + term)
    return np.einsum("abc,ai,bj,ck->kji", C, fx, fy, fz, optimize=True)


def uniform_line_kernel(n: int, lam: float, L: int, pos: int) -> np.ndarray:
    """Exact 1-D case: an L x 1 x 1 domain.  Each sub-step stays with
    probability 1 - 2 lam and moves +-1 with probability lam each."""
    out = np.zeros(L)
    for k in range(n + 1):
        out += comb(n, k) * (1.0 - 2.0 * lam) ** (n - k) * (2.0 * lam) ** k * walk_1d(k, L, pos)
    return out


def two_cell(n: int, d1: float, d2: float, dt: float, h: float):
    """Two face-adjacent cells with diffusivities d1, d2; unit source in cell 1.
    The mass difference decays by (1 - 2 lam) per sub-step, lam being the
    harmonic-mean face coefficient.  Returns (G_1, G_2)."""
    if d1 > 0 and d2 > 0:
        lam = (2.0 * d1 * d2 / (d1 + d2)) * dt / (h * h)
    else:
        lam = 0.0
    q = (1.0 - 2.0 * lam) ** n
    return 0.5 * (1.0 + q), 0.5 * (1.0 - q)


def dense_operator(label, d_phase, dt, h, exact=False):
    """Whole-domain one-sub-step operator as a dense matrix (column j = where
    the mass of cell j goes).  Built from the face list of the grid."""
    label = np.asarray(label)
    nz, ny, nx = label.shape
    N = label.size
    one = Fraction(1) if exact else 1.0
    A = [[0 * one for _ in range(N)] for _ in range(N)] if exact else np.zeros((N, N))
    dts = Fraction(dt) if exact else dt
    hh = Fraction(h) * Fraction(h) if exact else h * h

    def idx(x, y, z):
        return (z * ny + y) * nx + x

    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                i = idx(x, y, z)
                for (x2, y2, z2) in ((x + 1, y, z), (x, y + 1, z), (x, y, z + 1)):
                    if x2 >= nx or y2 >= ny or z2 >= nz:
                        continue
                    j = idx(x2, y2, z2)
                    da = d_phase[label[z, y, x]]
                    db = d_phase[label[z2, y2, x2]]
                    if exact:
                        da, db = Fraction(da), Fraction(db)
                    if da > 0 and db > 0:
                        lam = (2 * da * db / (da + db)) * dts / hh
                    else:
                        lam = 0 * one
                    A[i][j] += lam
                    A[j][i] += lam
                    A[i][i] -= lam
                    A[j][j] -= lam
    for i in range(N):
        A[i][i] += one
    return A


def matpow_exact(A, n):
    N = len(A)
    R = [[Fraction(int(i == j)) for j in range(N)] for i in range(N)]
    for _ in range(n):
        R = [[sum(R[i][k] * A[k][j] for k in range(N) if A[k][j] != 0) for j in range(N)]
             for i in range(N)]
    return R
