"""Helpers for the oracle pin tests: golden-file parsing and small numpy
utilities that view the canonical DoF layout as a d-dimensional array.

Canonical layout (shared with the GPU library's ABI): dof = cell * n^d + node,
cell lexicographic over the d cell indices and node lexicographic over the d
node indices, dimension 1 fastest in both.
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def golden_gl():
    out = {}
    env = {"sqrt": np.sqrt}
    for line in golden_lines("gauss_lobatto.txt"):
        k, pts, wts = [s.strip() for s in line.split("|")]
        out[int(k)] = (np.array([eval(p, env) for p in pts.split(",")], dtype=float),
                       np.array([eval(w, env) for w in wts.split(",")], dtype=float))
    return out


def golden_lsrk():
    A, B, C = [], [], []
    for line in golden_lines("lsrk45_ck1994.txt"):
        _, a, b, c = line.split()
        A.append(Fraction(a))
        B.append(Fraction(b))
        C.append(Fraction(c))
    return A, B, C


def butcher_from_2n(A, B):
    """Butcher tableau (a, b, c) of a 2N-storage scheme
    du_s = A_s du_{s-1} + dt F(Y_s), u_s = u_{s-1} + B_s du_s, Y_{s+1} = u_s.
    Stage s+1 input: Y_{s+1} = u_0 + sum_r k_r sum_{s'=r}^{s} B_s' prod_{m=r+1}^{s'} A_m."""
    S = len(A)
    a = [[Fraction(0)] * S for _ in range(S + 1)]
    for s in range(1, S + 1):          # row s gives Y_{s+1} (row S gives b)
        for r in range(1, s + 1):
            tot = Fraction(0)
            for sp in range(r, s + 1):
                prod = Fraction(1)
                for m in range(r + 1, sp + 1):
                    prod *= A[m - 1]
                tot += B[sp - 1] * prod
            a[s][r - 1] = tot
    b = a[S]
    amat = a[:S]
    c = [sum(row) for row in amat]
    return amat, b, c


def grid_view(u, cells, n):
    """Reshape a canonical DoF vector to (C_d, ..., C_1, n_d, ..., n_1)."""
    d = len(cells)
    return np.asarray(u).reshape(tuple(reversed(cells)) + (n,) * d)


def cell_axis(d, j):
    """Array axis of the cell index of dimension j (0-based) in grid_view."""
    return d - 1 - j


def node_axis(d, j):
    return 2 * d - 1 - j


def weights_view(w, h, d):
    """W_i = prod_j h_j w_{i_j} as an (n,)*d array in node-axis order."""
    W = np.ones((len(w),) * d)
    for j in range(d):
        shape = [1] * d
        shape[d - 1 - j] = len(w)
        W = W * (h[j] * np.asarray(w)).reshape(shape)
    return W


def integrate(P, u):
    """sum_i W_i u_i over the whole mesh using the golden-checked GL weights."""
    import oracle
    xi, w = oracle.gl_rule(P.k)
    h = [(P.hi[j] - P.lo[j]) / P.cells[j] for j in range(P.d)]
    W = weights_view(w, h, P.d)
    g = grid_view(u, P.cells, P.n)
    return float((g * W).sum())
