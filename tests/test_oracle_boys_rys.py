"""Pins of the oracle's Boys values and Rys rule (eq. 5) against mathematics
that the oracle does not use: closed forms, a library special function,
direct quadrature of the defining integral and the large-T Hermite limit."""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle as O


def boys_by_quadrature(m, T, n=400):
    """F_m(T) = int_0^1 t^(2m) exp(-T t^2) dt by Gauss-Legendre on [0,1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    t = 0.5 * (x + 1.0)
    return 0.5 * np.sum(w * t ** (2 * m) * np.exp(-T * t * t))


@pytest.mark.parametrize("m", range(0, 20))
def test_boys_at_zero(m):
    assert O.boys(m, 0.0)[m] == pytest.approx(1.0 / (2 * m + 1), rel=1e-16, abs=0)


@pytest.mark.parametrize("T", [1e-12, 1e-3, 0.5, 3.0, 11.0, 29.99, 30.01, 44.0, 120.0, 900.0])
def test_boys_f0_erf(T):
    F0 = O.boys(0, T)[0]
    ref = 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
    assert F0 == pytest.approx(ref, rel=2e-15)


@pytest.mark.parametrize("T", [0.0, 0.2, 2.0, 9.0, 25.0, 31.0, 60.0])
def test_boys_hypergeometric(T):
    F = O.boys(16, T)
    for m in range(17):
        ref = sp.hyp1f1(m + 0.5, m + 1.5, -T) / (2 * m + 1)
        assert F[m] == pytest.approx(ref, rel=5e-14), m


@pytest.mark.parametrize("T", [0.05, 1.7, 8.0, 28.0, 33.0])
def test_boys_quadrature_of_definition(T):
    F = O.boys(12, T)
    for m in range(13):
        assert F[m] == pytest.approx(boys_by_quadrature(m, T), rel=1e-13), m


@pytest.mark.parametrize("T", [150.0, 400.0, 2000.0])
def test_boys_large_T_asymptotic(T):
    # F_m(T) -> (2m-1)!! / 2^(m+1) sqrt(pi / T^(2m+1)); the correction is O(exp(-T))
    F = O.boys(10, T)
    for m in range(11):
        dfact = 1.0
        for k in range(2 * m - 1, 0, -2):
            dfact *= k
        ref = dfact / 2 ** (m + 1) * math.sqrt(math.pi / T ** (2 * m + 1))
        assert F[m] == pytest.approx(ref, rel=1e-14), m


def test_boys_recursion_identities():
    for T in [0.3, 5.0, 29.0, 31.0, 70.0]:
        F = O.boys(14, T)
        e = math.exp(-T)
        for m in range(14):
            # downward relation 2T F_{m+1} + exp(-T) = (2m+1) F_m
            assert 2 * T * F[m + 1] + e == pytest.approx((2 * m + 1) * F[m], rel=1e-14)


@pytest.mark.parametrize("n", range(1, 9))
@pytest.mark.parametrize("T", [0.0, 0.4, 3.0, 15.0, 29.5, 35.0, 100.0])
def test_rys_moments(n, T):
    """sum_mu w_mu u_mu^k = F_k(T), k = 0..2n-1, with F_k from direct quadrature."""
    u, w = O.rys_rule(n, T)
    assert np.all(u > 0) and np.all(u < 1) and np.all(w > 0)
    for k in range(2 * n):
        ref = boys_by_quadrature(k, T, n=600) if T < 40 else \
            sp.hyp1f1(k + 0.5, k + 1.5, -T) / (2 * k + 1)
        assert np.sum(w * u ** k) == pytest.approx(ref, rel=1e-12), k


@pytest.mark.parametrize("T", [0.0, 1.0, 20.0, 50.0])
def test_rys_one_point_closed_form(T):
    u, w = O.rys_rule(1, T)
    F = [boys_by_quadrature(m, T, n=600) for m in (0, 1)] if T < 40 else \
        [sp.hyp1f1(m + 0.5, m + 1.5, -T) / (2 * m + 1) for m in (0, 1)]
    assert w[0] == pytest.approx(F[0], rel=1e-14)
    assert u[0] == pytest.approx(F[1] / F[0], rel=1e-13)


@pytest.mark.parametrize("n", range(1, 8))
def test_rys_large_T_hermite_limit(n):
    """For T -> inf the measure exp(-T t^2) on [0,1] becomes the half-line
    Hermite weight: u_mu -> x_j^2 / T, w_mu -> h_j / sqrt(T), x_j the positive
    nodes of the 2n-point Gauss-Hermite rule."""
    T = 1.0e5
    x, h = np.polynomial.hermite.hermgauss(2 * n)
    pos = x > 0
    u_ref = np.sort(x[pos] ** 2 / T)
    order = np.argsort(x[pos] ** 2)
    w_ref = (h[pos] / math.sqrt(T))[order]
    u, w = O.rys_rule(n, T)
    assert np.allclose(u, u_ref, rtol=1e-12, atol=0)
    assert np.allclose(w, w_ref, rtol=1e-12, atol=0)


@pytest.mark.parametrize("L", range(0, 5))
@pytest.mark.parametrize("alpha", [0.1, 1.5, 37.0, 4000.0])
def test_normalisation_axis_aligned(L, alpha):
    """N(alpha,L)^2 * int x^(2L) exp(-2 alpha r^2) d^3r = 1 (eq. 1, Kenny08
    convention), the integral done by Gauss-Hermite quadrature."""
    N = O.norm(alpha, L)
    y, h = np.polynomial.hermite.hermgauss(40)
    s = 1.0 / math.sqrt(2 * alpha)
    ix = np.sum(h * (y * s) ** (2 * L)) * s
    i1 = np.sum(h) * s
    assert N * N * ix * i1 * i1 == pytest.approx(1.0, rel=1e-13)
