"""Pins for the oracle's tables and pair-potential step (CPU only).

Each check compares the oracle against something other than itself: exact
polynomial integration, numpy's Gauss-Legendre routine, independent
quadrature of the defining integrals, a radial Fourier-Bessel transform, and
the secular equation of a rank-1 potential.
"""
import math

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss
from scipy import integrate

import oracle.wpcd as W
from inputs import YAM_BETA, YAM_KAPPA, YAM_LAMBDA, YUK_RANGES


@pytest.mark.parametrize("n", [1, 2, 3, 8, 16, 20, 33])
def test_gauss_legendre_exactness(n):
    x, w = W.gauss_legendre(n)
    assert np.all(np.diff(x) > 0)
    np.testing.assert_allclose(x, -x[::-1], atol=1e-15)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 2e-14
    xr, wr = leggauss(n)
    np.testing.assert_allclose(x, xr, atol=3e-16)
    np.testing.assert_allclose(w, wr, rtol=0, atol=3e-15)


def test_edges():
    for n in (3, 12, 40, 150):
        e = W.cheb_edges(n, 10.0)
        assert e[0] == 0.0 and e[-1] == 10.0
        assert np.all(np.diff(e) > 0)
        # spacing grows monotonically away from zero (dense near 0)
        assert np.all(np.diff(np.diff(e)) > 0)
    e = W.cheb_edges(6, 3.0)
    assert abs(e[4] - 1.5) < 1e-15  # 1 - cos(pi/3) = 1/2


def test_free_energies():
    p = W.cheb_edges(10, 10.0)
    eps = W.free_energies(p)
    for i in range(10):
        val = integrate.quad(lambda x: x * x, p[i], p[i + 1])[0] / (p[i + 1] - p[i])
        assert abs(eps[i] - val) <= 1e-13 * val


def test_yamaguchi_matrix_vs_quadrature():
    p = W.cheb_edges(12, 10.0)
    v = W.yamaguchi_v(p, YAM_LAMBDA, YAM_BETA)
    g = lambda x: 1.0 / (x * x + YAM_BETA ** 2)
    for i, k in [(0, 0), (3, 7), (11, 2)]:
        gi = integrate.quad(lambda x: x * g(x), p[i], p[i + 1], epsabs=0, epsrel=1e-13)[0]
        gk = integrate.quad(lambda x: x * g(x), p[k], p[k + 1], epsabs=0, epsrel=1e-13)[0]
        ref = YAM_LAMBDA * gi * gk / math.sqrt((p[i + 1] - p[i]) * (p[k + 1] - p[k]))
        assert abs(v[i, k] - ref) <= 1e-12 * abs(ref)


def test_yamaguchi_strength_binds_at_kappa():
    # 1 = -lam int_0^inf p^2 g^2 / (p^2 + kappa^2) dp with g = 1/(p^2+beta^2)
    f = lambda x: x * x / ((x * x + YAM_BETA ** 2) ** 2 * (x * x + YAM_KAPPA ** 2))
    val = integrate.quad(f, 0, np.inf, epsabs=0, epsrel=1e-13)[0]
    assert abs(-YAM_LAMBDA * val - 1.0) < 1e-12


def test_yukawa_kernel_normalisation():
    """v(p,p') = (2/pi) int r^2 dr j0(pr) V(r) j0(p'r) for V = s e^{-mu r}/r;
    the oracle's closed form in the bins must equal the bin integral of it."""
    s, mu = -1.3, 1.0
    p, pp = 0.7, 1.9
    f = lambda r: (2.0 / math.pi) * math.sin(p * r) * math.sin(pp * r) / (p * pp) * s * math.exp(-mu * r) / r
    vk = integrate.quad(f, 0, 60, limit=400, epsabs=1e-15, epsrel=1e-13)[0]
    closed = s / (2 * math.pi * p * pp) * math.log(((p + pp) ** 2 + mu ** 2) / ((p - pp) ** 2 + mu ** 2))
    assert abs(vk - closed) < 1e-10 * abs(closed)
    # bin integral of p p' v(p,p') against the Phi closed form
    edges = np.array([0.0, 0.3, 0.8, 1.5, 2.5])
    V = W.yukawa_v_swave(edges, s, mu)
    for i, k in [(0, 0), (1, 3), (2, 2), (3, 1)]:
        g = lambda y, x: s / (2 * math.pi) * math.log(((x + y) ** 2 + mu ** 2) / ((x - y) ** 2 + mu ** 2))
        val = integrate.dblquad(g, edges[i], edges[i + 1], edges[k], edges[k + 1],
                                epsabs=0, epsrel=1e-12)[0]
        ref = val / math.sqrt((edges[i + 1] - edges[i]) * (edges[k + 1] - edges[k]))
        assert abs(V[i, k] - ref) <= 1e-10 * abs(ref)


@pytest.mark.parametrize("l", [0, 1, 2, 4])
def test_legendre_q_vs_neumann_integral(l):
    # Q_l(z) = 1/2 int_{-1}^{1} P_l(t) / (z - t) dt
    from numpy.polynomial.legendre import Legendre
    Pl = Legendre.basis(l)
    for z in [1.05, 1.7, 2.0, 3.5, 40.0]:
        ref = 0.5 * integrate.quad(lambda t: Pl(t) / (z - t), -1, 1, epsabs=0, epsrel=1e-13,
                                   limit=200)[0]
        got = W.legendre_q(l, np.array([z]))[0]
        # the integral cancels for large z: allow round-off on its scale 1/z
        assert abs(got - ref) <= 1e-11 * abs(ref) + 1e-14 / z
    # large z: Q_l(z) = l!/(2l+1)!! z^-(l+1) [1 + (l+1)(l+2)/(2(2l+3)) z^-2 + O(z^-4)]
    z = 1e4
    dfact = math.prod(range(1, 2 * l + 2, 2))
    ref = math.factorial(l) / dfact * z ** -(l + 1) * (1 + (l + 1) * (l + 2) / (2 * (2 * l + 3)) / z ** 2)
    assert abs(W.legendre_q(l, np.array([z]))[0] - ref) <= 1e-14 * ref


def test_yukawa_d_wave_matrix_vs_dblquad():
    edges = np.array([0.0, 0.3, 0.8, 1.5, 2.5])
    s, mu, l = -2.0, 1.0, 2
    V = W.yukawa_v(edges, s, mu, l)
    for i, k in [(0, 0), (1, 3), (2, 2)]:
        g = lambda y, x: s / math.pi * W.legendre_q(l, np.array([(x * x + y * y + mu * mu) / (2 * x * y)]))[0]
        val = integrate.dblquad(g, edges[i], edges[i + 1], edges[k], edges[k + 1],
                                epsabs=0, epsrel=1e-11)[0]
        ref = val / math.sqrt((edges[i + 1] - edges[i]) * (edges[k + 1] - edges[k]))
        assert abs(V[i, k] - ref) <= 1e-8 * abs(ref)


def test_yamaguchi_spectrum_secular_equation():
    """Rank-1 v = lam gamma gamma^T: every eigenvalue e of diag(eps) + v solves
    1 = lam sum_i gamma_i^2 / (e - eps_i)."""
    p = W.cheb_edges(30, 10.0)
    eps = W.free_energies(p)
    d = np.diff(p)
    gam = np.log((p[1:] ** 2 + 1.0) / (p[:-1] ** 2 + 1.0)) / (2 * np.sqrt(d))
    e, O = W.pair_diag(p, W.yamaguchi_v(p, YAM_LAMBDA, YAM_BETA))
    for ek in e:
        f = YAM_LAMBDA * np.sum(gam ** 2 / (ek - eps))
        assert abs(f - 1.0) < 1e-9
    # eigenvalues interlace the free energies, exactly one bound state
    assert e[0] < 0 < e[1]
    assert np.all(e[1:] > eps[:-1]) and np.all(e[1:] < eps[1:] + 1e-12)
    # O orthogonal, rows eigenvectors, sign rule
    np.testing.assert_allclose(O @ O.T, np.eye(30), atol=1e-13)
    h = np.diag(eps) + W.yamaguchi_v(p, YAM_LAMBDA, YAM_BETA)
    np.testing.assert_allclose(O.T @ np.diag(e) @ O, h, atol=1e-12)
    for k in range(30):
        m = np.argmax(np.abs(O[k]))
        assert O[k, m] > 0


def test_pair_binding_converges_to_target():
    prev = None
    for n in (20, 40, 80):
        p = W.cheb_edges(n, 10.0)
        e, _ = W.pair_diag(p, W.yamaguchi_v(p, YAM_LAMBDA, YAM_BETA))
        # variational from above; the cutoff at p = 10 leaves ~3e-4
        assert e[0] > -0.1
        if prev is not None:
            assert e[0] < prev
        prev = e[0]
    assert abs(prev + 0.1) < 1.5e-3


def test_strength_fit():
    p = W.cheb_edges(40, 10.0)
    s = W.fit_strength(p, YUK_RANGES, -0.1)
    v = sum(W.yukawa_v_swave(p, -s, mu) for mu in YUK_RANGES)
    e, _ = W.pair_diag(p, v)
    assert abs(e[0] + 0.1) < 1e-12
    assert e[1] > 0
