"""Pins for the oracle's energy-dependent steps (CPU only).

* the bin resolvent against direct quadrature of its defining integral;
* three independent solves of the same discrete equation agree: dense LU,
  GMRES, and the paper's iterations summed by Pade approximants;
* below breakup |S| = 1 holds exactly for any real P0, O, v (Sherman-Morrison
  on the single open channel), which ties the resolvent's imaginary part to
  the amplitude normalisation of Sec. III.B;
* above breakup the elastic inelasticity eta = |S| stays <= 1;
* the breakup pseudostate elements S_k0 (same column of U, Sec. III.B): for a
  real symmetric operator in place of P V1 the open-channel S-matrix of the
  discrete equation is exactly unitary (K-matrix argument below), so
  |S_00|^2 + sum_k |S_k0|^2 = 1 holds to rounding -- which fails for a wrong
  flux factor rho_k, a wrong on-shell bin j_k or a wrong (channel, k, j)
  index of the breakup element;
* the converged elastic S-matrix below breakup approaches the textbook
  separable-potential solution as the grid is refined (on-shell momentum
  kept at the same relative place in its bin);
* the three-body bound state of the homogeneous equation converges, as the
  grid is refined, to the textbook Nystrom solution of the separable
  three-boson equation with the same cutoffs (separable_ref.py), which shares
  nothing with the wave-packet formulation.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle.wpcd as W
from inputs import C1, YAM_BETA, YAM_LAMBDA, YUK_RANGES
from separable_ref import Separable


def _yamaguchi_system(n, n_gx=16):
    p = W.cheb_edges(n, 10.0)
    pot = W.Potential("yamaguchi", (YAM_LAMBDA,), (YAM_BETA,))
    return W.build_system(p, p.copy(), 0, [(0, 0)], 8, n_gx, pot)


@pytest.fixture(scope="module")
def c1():
    return _yamaguchi_system(C1["n_p"])


def test_resolvent_bin_vs_quadrature():
    qlo, qhi, qmax = 0.7, 1.1, 10.0
    for E, ek in [(0.5, -0.1), (0.2, 0.05), (-0.3, -0.1), (0.5, 0.9)]:
        g = W.resolvent_bin(E, ek, qlo, qhi, qmax)
        s = E - ek
        if s > 0 and qlo < math.sqrt(4 * s / 3) < qhi:
            qs = math.sqrt(4 * s / 3)
            # PV by scipy's Cauchy weight: 1/(s - 3/4 q^2) = -(4/3)/((q-qs)(q+qs))
            pv = integrate.quad(lambda q: -(4.0 / 3.0) / (q + qs), qlo, qhi, weight="cauchy",
                                wvar=qs, epsabs=0, epsrel=1e-13)[0]
            im = -math.pi * (4.0 / 3.0) / (2 * qs)
            ref = complex(pv, im) / (qhi - qlo)
        else:
            ref = integrate.quad(lambda q: 1.0 / (s - 0.75 * q * q), qlo, qhi, epsabs=0,
                                 epsrel=1e-13)[0] / (qhi - qlo)
        assert abs(g - ref) <= 1e-11 * abs(ref), (E, ek, g, ref)
    with pytest.raises(W.OnEdge):
        W.resolvent_bin(0.75 * 0.7 ** 2 - 0.1, -0.1, 0.7, 1.1, 10.0)


def test_solvers_agree_c1(c1):
    E = C1["energies"][0]
    idx = W.entrance(c1, E)[3]
    u_lu = W.solve_lu(c1, E)
    u_gm, its, res = W.solve_gmres(c1, E)
    assert res < 1e-12
    u_pd, diff = W.solve_pade(c1, E)
    assert abs(u_gm[idx] - u_lu[idx]) <= 1e-11 * abs(u_lu[idx])
    assert np.linalg.norm(u_gm - u_lu) <= 1e-10 * np.linalg.norm(u_lu)
    assert abs(u_pd - u_lu[idx]) <= 1e-8 * abs(u_lu[idx])


@pytest.mark.parametrize("E", [-0.08, -0.05, -0.02])
def test_unitarity_below_breakup(c1, E):
    u, _, _ = W.solve_gmres(c1, E)
    a = W.amplitudes(c1, E, u)
    assert abs(abs(a.S) - 1.0) < 1e-12
    assert a.breakup == []


def test_unitarity_below_breakup_yukawa():
    p = W.cheb_edges(30, 10.0)
    s = W.fit_strength(p, YUK_RANGES, -0.1)
    pot = W.Potential("yukawa", (-s, -s), YUK_RANGES)
    sysm = W.build_system(p, p.copy(), 0, [(0, 0)], 8, 20, pot)
    assert abs(sysm.eps[0][0] + 0.1) < 1e-12
    for E in (-0.06, -0.01):
        u, _, res = W.solve_gmres(sysm, E)
        assert res < 1e-12
        a = W.amplitudes(sysm, E, u)
        assert abs(abs(a.S) - 1.0) < 1e-12


@pytest.mark.parametrize("E", [0.05, 0.5, 2.0])
def test_inelasticity_bounded_above_breakup(c1, E):
    u, _, res = W.solve_gmres(c1, E)
    assert res < 1e-12
    a = W.amplitudes(c1, E, u)
    assert a.eta <= 1.0 + 1e-12
    assert len(a.breakup) > 0


def test_bound_state_converges_to_separable_reference():
    ref = Separable(YAM_LAMBDA, YAM_BETA, 10.0, 10.0)
    e3_ref = ref.bound_state(-5.0)
    errs = []
    for n in (20, 40, 80):
        sysm = _yamaguchi_system(n)
        e3 = W.bound_state(sysm, -3.0, sysm.eps[0][0] - 1e-4, tol=1e-9)
        errs.append(e3 - e3_ref)
    # variational-like approach from above, roughly second order in 1/N
    assert all(e > 0 for e in errs)
    assert errs[1] < 0.4 * errs[0] and errs[2] < 0.4 * errs[1]
    assert abs(errs[2]) < 5e-3 * abs(e3_ref)


def test_pair_threshold_matches_separable_reference():
    ref = Separable(YAM_LAMBDA, YAM_BETA, 10.0, 10.0)
    e0 = [_yamaguchi_system(n).eps[0][0] for n in (20, 40, 80)]
    errs = [e - ref.eb for e in e0]
    assert errs[0] > errs[1] > errs[2] > 0
    assert errs[2] < 1e-2 * abs(ref.eb) and errs[2] < 0.4 * errs[1]


def _open_channel_unitarity(sysm, E, seed):
    """Solve (1 - A G1) u = A e0 with a random real symmetric A of the
    system's size and the oracle's resolvent, then form the amplitudes with
    the oracle's formulas.  With G1 = G_R + i sum_o g_o e_o e_o^T over the
    open channels o (g_o = -pi rho_o) and K_R = (1 - A G_R)^-1 A (real and
    symmetric when A is), the open block of u is K (1 - i g K)^-1 e0, so the
    matrix S = 1 - 2 pi i rho^(1/2) U rho^(1/2) of the open channels is
    (1 - i k)(1 + i k)^-1 with k = (-g)^(1/2) K (-g)^(1/2) real symmetric:
    unitary.  Returns (|S_00|^2 + sum_k |S_k0|^2, amplitude)."""
    rng = np.random.default_rng(seed)
    M = sysm.M
    R = rng.normal(size=(M, M))
    A = 0.2 * (R + R.T) / math.sqrt(M)
    G = W.resolvent(sysm, E).ravel()
    idx = W.entrance(sysm, E)[3]
    e0 = np.zeros(M)
    e0[idx] = 1.0
    u = np.linalg.solve(np.eye(M) - A * G[None, :], A @ e0)
    a = W.amplitudes(sysm, E, u)
    return abs(a.S) ** 2 + sum(abs(s) ** 2 for (_, _, _, s) in a.breakup), a


@pytest.mark.parametrize("E", [0.3, 1.2, 2.5])
def test_breakup_elements_exact_unitarity_symmetric_operator(E):
    sysm = _yamaguchi_system(14)
    total, a = _open_channel_unitarity(sysm, E, 11)
    assert len(a.breakup) >= 2
    assert abs(total - 1.0) < 1e-12, total
    # flux really goes into the breakup elements
    assert sum(abs(s) ** 2 for (_, _, _, s) in a.breakup) > 1e-3


def test_breakup_elements_exact_unitarity_three_channels():
    """The same with the three L = 2+ channels (entrance (l, lam) = (0, 2)):
    the open pseudostates of all three channels enter the sum, so the
    channel part of the breakup element's index is checked too."""
    p = W.cheb_edges(8, 6.0)
    q = W.cheb_edges(9, 6.0)
    pot = W.Potential("yukawa", (-1.2, -1.2), YUK_RANGES)
    sysm = W.build_system(p, q, 2, [(0, 2), (2, 0), (2, 2)], 4, 8, pot, with_p0=False)
    for E in (0.4, 1.5):
        total, a = _open_channel_unitarity(sysm, E, 5)
        assert {c for (c, _, _, _) in a.breakup} == {0, 1, 2}
        assert abs(total - 1.0) < 1e-12, (E, total)
        assert sum(abs(s) ** 2 for (_, _, _, s) in a.breakup) > 1e-3


@pytest.mark.parametrize("q_target", [0.15, 0.26, 0.32])
def test_elastic_S_converges_to_separable_reference(q_target):
    """Below breakup, with the on-shell momentum q0 at 30% of its bin for
    each grid (so the on-shell bin's principal-value part is alike), the
    wave-packet S-matrix approaches the Nystrom solution of the separable
    three-boson equation at the same q0 (same cutoffs) as N = 40 -> 80 ->
    120; phases are compared through S itself (no branch of arg)."""
    ref = Separable(YAM_LAMBDA, YAM_BETA, 10.0, 10.0)
    errs = []
    for n in (40, 80, 120):
        sysm = _yamaguchi_system(n)
        p = sysm.q
        j = int(np.searchsorted(p, q_target) - 1)
        q0 = p[j] + 0.3 * (p[j + 1] - p[j])
        E = sysm.eps[0][0] + 0.75 * q0 * q0
        assert E < 0.0
        u, _, res = W.solve_gmres(sysm, E)
        assert res < 1e-12
        a = W.amplitudes(sysm, E, u)
        errs.append(abs(a.S - ref.elastic(ref.eb + 0.75 * q0 * q0)))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 0.07, errs
