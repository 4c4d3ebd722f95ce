"""Deslauriers-Dubuc wavelet-collocation first derivative (section 2.3, the
derivative formula with support j-2p+1 .. j+2p-1 and error O(dx^2p)).

ORACLE - test infrastructure only.  Nothing in the product path may import it.

The interpolant u^N(x) = sum_k u_k psi((x - x_k)/dx) uses the DD interpolating
scaling function psi of order 2p.  Its derivative at a grid point is

    (D u)_i = (1/dx) sum_k u_k psi'(i - k),

so the stencil is the vector of values d_n = psi'(n) at the integers.  They
follow from the two-scale (refinement) relation of psi,

    psi(x) = sum_n h_n psi(2x - n),   h_0 = 1,  h_{2j+1} = L_{-j}(1/2),

where L_k are the Lagrange weights of the 2p nodes -p+1..p at the midpoint 1/2
(p = 2: 9/16 and -1/16).  Differentiating gives d_n = 2 sum_k h_k d_{2n-k}: the
stencil is the eigenvector of the refinement matrix for eigenvalue 1/2,
normalised by the first-moment condition sum_k k psi'(-k) = 1 (linear functions
are reproduced).  Nothing here hard-codes the resulting numbers.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def dd_filter(p: int) -> dict:
    """Two-scale coefficients h_n of the order-2p DD interpolating function."""
    nodes = list(range(-p + 1, p + 1))
    half = Fraction(1, 2)
    h = {0: Fraction(1)}
    for j in range(-p, p):
        node = -j
        if node not in nodes:
            continue
        wgt = Fraction(1)
        for m in nodes:
            if m != node:
                wgt *= (half - m) / Fraction(node - m)
        h[2 * j + 1] = wgt
    return h


def _solve_exact(rows, rhs):
    """Consistent linear system over the rationals (Gauss-Jordan elimination
    with exact Fractions); returns the unique solution."""
    n = len(rows[0])
    A = [list(r) + [b] for r, b in zip(rows, rhs)]
    piv_row = 0
    cols = []
    for c in range(n):
        r = next((i for i in range(piv_row, len(A)) if A[i][c] != 0), None)
        if r is None:
            continue
        A[piv_row], A[r] = A[r], A[piv_row]
        pv = A[piv_row][c]
        A[piv_row] = [x / pv for x in A[piv_row]]
        for i in range(len(A)):
            if i != piv_row and A[i][c] != 0:
                f = A[i][c]
                A[i] = [x - f * y for x, y in zip(A[i], A[piv_row])]
        cols.append(c)
        piv_row += 1
    if len(cols) != n:
        raise ValueError("refinement system does not fix the stencil")
    for i in range(piv_row, len(A)):
        if A[i][n] != 0:
            raise ValueError("refinement system is inconsistent")
    return [A[i][n] for i in range(n)]


def derivative_values(p: int = 2, exact: bool = False) -> dict:
    """psi'(n) for integer n with |n| <= 2p-2 (zero outside), from the
    eigen-relation d_n = 2 sum_k h_k d_{2n-k} plus the moment condition,
    solved exactly over the rationals."""
    h = dd_filter(p)
    M = 2 * p - 2                      # psi has support [-(2p-1), 2p-1]; psi' vanishes at the ends
    idx = list(range(-M, M + 1))
    rows, rhs = [], []
    for n in idx:                      # (2A - I) d = 0
        rows.append([2 * h.get(2 * n - m, Fraction(0)) - (1 if m == n else 0) for m in idx])
        rhs.append(Fraction(0))
    rows.append([Fraction(-m) for m in idx])   # sum_k k psi'(-k) = 1 with m = -k
    rhs.append(Fraction(1))
    d = _solve_exact(rows, rhs)
    if exact:
        return {n: d[a] for a, n in enumerate(idx)}
    return {n: float(d[a]) for a, n in enumerate(idx)}


def stencil(p: int = 2):
    """Offsets m and weights c_m with (D u)_i = (1/dx) sum_m c_m u_{i+m}."""
    d = derivative_values(p)
    offs = sorted(d.keys())
    return offs, np.array([d[-m] for m in offs])


_CACHE = {}


def _coef(p):
    if p not in _CACHE:
        _CACHE[p] = stencil(p)
    return _CACHE[p]


def deriv(a: np.ndarray, axis: int, h: float, p: int = 2) -> np.ndarray:
    """Apply D along ``axis`` of a ghost-extended array.  Entries whose stencil
    would leave the array are NaN, so any use of an undefined value shows up."""
    offs, c = _coef(p)
    M = max(offs)
    out = np.full(a.shape, np.nan, dtype=np.result_type(a.dtype, np.float64))
    n = a.shape[axis]
    if n <= 2 * M:
        return out
    acc = np.zeros_like(np.take(a, range(M, n - M), axis=axis))
    for m, cm in zip(offs, c):
        if cm == 0.0:
            continue
        acc = acc + cm * np.take(a, range(M + m, n - M + m), axis=axis)
    sl = [slice(None)] * a.ndim
    sl[axis] = slice(M, n - M)
    out[tuple(sl)] = acc / h
    return out
