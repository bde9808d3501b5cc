"""Pins of the oracle's finite-difference weights (textbook closed forms and exactness)."""
import numpy as np
import pytest

from oracle.fd import diff_matrix, fornberg, window_start


def test_centred_sixth_order_first_derivative_closed_form():
    w = fornberg(0.0, np.arange(-3, 4, dtype=float), 1)[:, 1]
    ref = np.array([-1 / 60, 3 / 20, -3 / 4, 0.0, 3 / 4, -3 / 20, 1 / 60])
    assert np.allclose(w, ref, rtol=0, atol=1e-15)


def test_three_point_stencils_closed_form():
    w = fornberg(0.0, [-1.0, 0.0, 1.0], 2)
    assert np.allclose(w[:, 1], [-0.5, 0.0, 0.5], atol=1e-15)
    assert np.allclose(w[:, 2], [1.0, -2.0, 1.0], atol=1e-15)


@pytest.mark.parametrize("width,deriv", [(7, 1), (3, 1), (3, 2), (5, 1)])
def test_every_window_exact_on_monomials(width, deriv):
    npts, h = 12, 0.37
    D = diff_matrix(npts, h, deriv, width, periodic=False).toarray()
    x = np.arange(npts) * h
    for p in range(width):
        f = x ** p
        if deriv == 1:
            exact = p * x ** (p - 1) if p >= 1 else np.zeros(npts)
        else:
            exact = p * (p - 1) * x ** (p - 2) if p >= 2 else np.zeros(npts)
        assert np.allclose(D @ f, exact, rtol=1e-9, atol=1e-9), (width, deriv, p)
    # rows of a derivative operator annihilate constants
    assert np.allclose(D.sum(axis=1), 0.0, atol=1e-12)


def test_window_start_stays_inside():
    for npts in (7, 8, 20):
        for i in range(npts):
            s = window_start(i, npts, 7)
            assert 0 <= s <= i <= s + 6 < npts
            if 3 <= i < npts - 3:
                assert s == i - 3


def test_periodic_sixth_order_convergence():
    errs = []
    for n in (16, 32, 64):
        h = 2 * np.pi / n
        x = np.arange(n) * h
        D = diff_matrix(n, h, 1, 7, periodic=True)
        errs.append(np.abs(D @ np.sin(x) - np.cos(x)).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 5.8), rates
