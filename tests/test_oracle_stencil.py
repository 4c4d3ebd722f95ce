"""Pins of the oracle's derivative stencil against textbook facts (section 2.3:
DD interpolation, exactness on low-degree polynomials, order 2p, filtering of the
2-dx mode).  No GPU."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import stencil as ST

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_filter():
    out = {}
    for line in open(os.path.join(GOLD, "dd_filter_p2.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, a, b = line.split()
        out[int(n)] = Fraction(int(a), int(b))
    return out


def test_dd_filter_matches_textbook_coefficients():
    assert ST.dd_filter(2) == _read_filter()


def test_p2_stencil_is_the_fourth_order_central_difference():
    d = ST.derivative_values(2, exact=True)
    # psi'(n): D u_i = sum_k u_k psi'(i-k)/dx  =>  coefficient of u_{i+1} is psi'(-1)
    assert d == {-2: Fraction(-1, 12), -1: Fraction(2, 3), 0: Fraction(0),
                 1: Fraction(-2, 3), 2: Fraction(1, 12)}


@pytest.mark.parametrize("p", [2, 3])
def test_polynomial_exactness_and_antisymmetry(p):
    """The paper promises exactness for polynomials of degree 2p-1; the centred
    stencil is in fact exact up to degree 2p."""
    offs, c = ST.stencil(p)
    assert np.allclose(c, -c[::-1], atol=0, rtol=0)
    x = np.arange(-20, 21) * 0.37 + 1.3
    h = 0.37
    for k in range(0, 2 * p + 1):
        a = x ** k
        d = ST.deriv(a[None, :], 1, h, p)[0]
        ok = ~np.isnan(d)
        exact = k * x ** (k - 1) if k else np.zeros_like(x)
        assert np.allclose(d[ok], exact[ok], rtol=1e-11, atol=1e-9), k
    # degree 2p+1 is not reproduced
    a = x ** (2 * p + 1)
    d = ST.deriv(a[None, :], 1, h, p)[0]
    ok = ~np.isnan(d)
    assert not np.allclose(d[ok], (2 * p + 1) * x[ok] ** (2 * p), rtol=1e-9)


@pytest.mark.parametrize("p", [2, 3])
def test_order_of_accuracy(p):
    errs = []
    for n in (32, 64, 128):
        h = 2 * np.pi / n
        x = np.arange(-8, n + 8) * h
        d = ST.deriv(np.sin(x)[None, :], 1, h, p)[0]
        ok = ~np.isnan(d)
        errs.append(np.abs(d[ok] - np.cos(x[ok])).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2 * p - 0.1), rates


def test_modified_wavenumber_and_nyquist_filter():
    """D exp(ikx) = i k~ exp(ikx), k~ dx = (4/3) sin(k dx) - (1/6) sin(2 k dx);
    the 2-dx mode (k dx = pi) is annihilated."""
    n, h = 64, 1.0
    x = np.arange(-8, n + 8) * h
    for kh in (0.3, 1.0, 1.797, 2.5, np.pi):
        e = np.exp(1j * kh * x / h)
        d = ST.deriv(e[None, :], 1, h, 2)[0]
        ok = ~np.isnan(d)
        kt = (4.0 / 3.0) * np.sin(kh) - (1.0 / 6.0) * np.sin(2 * kh)
        assert np.allclose(d[ok], 1j * kt * e[ok] / h, atol=1e-13)
    alt = (-1.0) ** np.arange(x.size)
    d = ST.deriv(alt[None, :], 1, h, 2)[0]
    assert np.abs(d[~np.isnan(d)]).max() < 1e-14


def test_p3_stencil_coefficients():
    d = ST.derivative_values(3, exact=True)
    assert d[-1] == Fraction(272, 365) and d[-2] == Fraction(-53, 365)
    assert d[-3] == Fraction(16, 1095) and d[-4] == Fraction(1, 2920)
