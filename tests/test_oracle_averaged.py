"""Pins for the oracle's energy-averaged channel resolvent (Sec. II.C: the
resolvent eigenvalues averaged over the on-shell energy interval, carried
over to the three-body channel resolvent) and the amplitudes built on it
(CPU only).

* the averaged eigenvalue against two quadratures of its definition: the
  average over E of the bin resolvent at E (itself pinned against its
  defining integral), and the q integral of the E-integrated kernel; across
  bins below, across and above the energy shell;
* it reduces to the bin resolvent at E as the energy interval shrinks;
* below breakup |S| = 1 exactly with the averaged flux factor rho0 = 1/D,
  and for a real symmetric operator the open-channel S-matrix (elastic state
  plus every pseudostate bin whose shell overlaps the energy interval, with
  rho = overlap / (D dq)) is exactly unitary -- which fails for a wrong
  overlap, flux factor or index;
* all energies of one on-shell bin give the same amplitudes (the histogram
  form of the averaged solution);
* the averaged elastic S-matrix approaches the separable reference
  monotonically as the grid is refined (on-shell momentum at the centre of
  its bin), closer than the unaveraged one.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle.wpcd as W
from inputs import YAM_BETA, YAM_LAMBDA, YUK_RANGES
from separable_ref import Separable

CASES = [
    # (E1, E2, eps_k, qlo, qhi): shell below, across, above, inside the bin
    (0.10, 0.25, -0.1, 0.2, 0.45),
    (0.10, 0.25, -0.1, 0.55, 0.70),
    (0.10, 0.25, -0.1, 0.62, 0.63),
    (0.10, 0.25, 0.05, 0.0, 0.3),
    (0.10, 0.25, 0.40, 0.5, 0.9),
    (-0.30, -0.20, -0.1, 0.1, 0.7),
    (-0.05, 0.02, 0.0, 0.0, 0.25),
    (0.5, 0.9, 0.1, 0.7, 0.75),
]


def _unaveraged(E, ek, qlo, qhi):
    # the bin resolvent at E without the on-edge guard (a measure-zero set
    # of E inside the E integral)
    return W.resolvent_bin(E, ek, qlo, qhi, 1e-300)


@pytest.mark.parametrize("case", CASES)
def test_averaged_resolvent_is_the_energy_average(case):
    E1, E2, ek, qlo, qhi = case
    g = W.resolvent_bin_avg(E1, E2, ek, qlo, qhi)
    pts = [ek + 0.75 * qlo * qlo, ek + 0.75 * qhi * qhi]
    pts = [x for x in pts if E1 < x < E2]
    re = integrate.quad(lambda E: _unaveraged(E, ek, qlo, qhi).real, E1, E2, points=pts or None,
                        epsabs=0, epsrel=1e-12, limit=400)[0]
    im = integrate.quad(lambda E: _unaveraged(E, ek, qlo, qhi).imag, E1, E2, points=pts or None,
                        epsabs=0, epsrel=1e-12, limit=400)[0]
    ref = complex(re, im) / (E2 - E1)
    assert abs(g - ref) <= 1e-9 * abs(ref), (g, ref)
    # the q integral of the E-integrated kernel: ln|E2 - c| - ln|E1 - c|
    s1, s2 = E1 - ek, E2 - ek
    qs = [math.sqrt(4 * s / 3) for s in (s1, s2) if s > 0 and qlo < math.sqrt(4 * s / 3) < qhi]
    f = lambda q: math.log(abs(s2 - 0.75 * q * q)) - math.log(abs(s1 - 0.75 * q * q))
    re2 = integrate.quad(f, qlo, qhi, points=qs or None, epsabs=0, epsrel=1e-13, limit=400)[0]
    assert abs(g.real - re2 / ((E2 - E1) * (qhi - qlo))) <= 1e-10 * abs(g), (g, re2)


def test_averaged_resolvent_narrow_interval_limit():
    """As the energy interval shrinks around E, the average tends to the
    bin resolvent at E (first order in the width)."""
    for E, ek, qlo, qhi in [(0.2, -0.1, 0.55, 0.7), (0.2, 0.05, 0.1, 0.3), (-0.3, -0.1, 0.1, 0.7)]:
        g0 = W.resolvent_bin(E, ek, qlo, qhi, 10.0)
        errs = []
        for h in (1e-2, 1e-3, 1e-4):
            g = W.resolvent_bin_avg(E - h, E + h, ek, qlo, qhi)
            errs.append(abs(g - g0))
        assert errs[0] > errs[1] > errs[2]
        assert errs[2] < 1e-5 * abs(g0)


def _yamaguchi_system(n, n_gx=16):
    p = W.cheb_edges(n, 10.0)
    pot = W.Potential("yamaguchi", (YAM_LAMBDA,), (YAM_BETA,))
    return W.build_system(p, p.copy(), 0, [(0, 0)], 8, n_gx, pot)


def test_averaged_unitarity_below_breakup():
    """|S| = 1 with the averaged resolvent when no pseudostate shell but the
    elastic one meets the on-shell energy interval."""
    p20 = W.cheb_edges(20, 10.0)
    s20 = W.fit_strength(p20, YUK_RANGES, -0.1)
    for sysm in (_yamaguchi_system(24),
                 W.build_system(p20, p20.copy(), 0, [(0, 0)], 8, 16,
                                W.Potential("yukawa", (-s20, -s20), YUK_RANGES))):
        assert sysm.eps[0][0] < -0.05
        e2 = min(e for e in sysm.eps[0] if e > sysm.eps[0][0])
        n_checked = 0
        for E in np.linspace(sysm.eps[0][0] + 0.01, min(0.0, e2) - 1e-3, 6):
            E1, E2 = W.energy_bin(sysm, E)
            if E2 >= e2:
                continue
            u, _, res = W.solve_gmres(sysm, E, averaged=True)
            assert res < 1e-12
            a = W.amplitudes(sysm, E, u, averaged=True)
            assert a.breakup == []
            assert abs(abs(a.S) - 1.0) < 1e-12, (E, a.S)
            n_checked += 1
        assert n_checked >= 3


def _open_channel_unitarity_avg(sysm, E, seed):
    rng = np.random.default_rng(seed)
    M = sysm.M
    R = rng.normal(size=(M, M))
    A = 0.2 * (R + R.T) / math.sqrt(M)
    G = W.resolvent(sysm, E, averaged=True).ravel()
    idx = W.entrance(sysm, E)[3]
    e0 = np.zeros(M)
    e0[idx] = 1.0
    u = np.linalg.solve(np.eye(M) - A * G[None, :], A @ e0)
    a = W.amplitudes(sysm, E, u, averaged=True)
    return abs(a.S) ** 2 + sum(abs(s) ** 2 for (_, _, _, s) in a.breakup), a


@pytest.mark.parametrize("E", [0.3, 1.2])
def test_averaged_breakup_exact_unitarity_symmetric_operator(E):
    sysm = _yamaguchi_system(14)
    total, a = _open_channel_unitarity_avg(sysm, E, 11)
    assert abs(total - 1.0) < 1e-12, total
    # several bins of one pseudostate take part, and the distribution sums them
    ks = [k for (_, k, _, _) in a.breakup]
    assert len(ks) > len(set(ks))
    assert abs(sum(d[3] for d in a.breakup_dist)
               - sum(abs(s) ** 2 for (_, _, _, s) in a.breakup)) < 1e-14
    assert sum(abs(s) ** 2 for (_, _, _, s) in a.breakup) > 1e-3


def test_averaged_breakup_exact_unitarity_three_channels():
    p = W.cheb_edges(8, 6.0)
    q = W.cheb_edges(9, 6.0)
    pot = W.Potential("yukawa", (-1.2, -1.2), YUK_RANGES)
    sysm = W.build_system(p, q, 2, [(0, 2), (2, 0), (2, 2)], 4, 8, pot, with_p0=False)
    for E in (0.4, 1.5):
        total, a = _open_channel_unitarity_avg(sysm, E, 5)
        assert {c for (c, _, _, _) in a.breakup} == {0, 1, 2}
        assert abs(total - 1.0) < 1e-12, (E, total)


def test_averaged_amplitudes_constant_on_an_energy_bin():
    sysm = _yamaguchi_system(20)
    E1, E2 = W.energy_bin(sysm, 0.5)
    res = []
    for t in (0.1, 0.5, 0.9):
        E = E1 + t * (E2 - E1)
        u, _, _ = W.solve_gmres(sysm, E, averaged=True)
        res.append(W.amplitudes(sysm, E, u, averaged=True).S)
    assert abs(res[0] - res[1]) < 1e-12 and abs(res[1] - res[2]) < 1e-12


@pytest.mark.parametrize("q_target", [0.15, 0.26])
def test_averaged_elastic_S_converges_to_separable_reference(q_target):
    """Below breakup, with q0 at the centre of its bin, the averaged elastic
    S-matrix approaches the Nystrom solution of the separable three-boson
    equation monotonically as N = 40 -> 80 -> 120, and at N = 120 it is
    closer to it than the unaveraged one (whose bin-position error stays)."""
    ref = Separable(YAM_LAMBDA, YAM_BETA, 10.0, 10.0)
    d_avg, d_un = [], []
    for n in (40, 80, 120):
        sysm = _yamaguchi_system(n)
        q = sysm.q
        j = int(np.searchsorted(q, q_target) - 1)
        q0 = 0.5 * (q[j] + q[j + 1])
        E = sysm.eps[0][0] + 0.75 * q0 * q0
        assert E < 0.0
        Sr = ref.elastic(ref.eb + 0.75 * q0 * q0)
        ua, _, _ = W.solve_gmres(sysm, E, averaged=True)
        uu, _, _ = W.solve_gmres(sysm, E)
        d_avg.append(abs(W.amplitudes(sysm, E, ua, averaged=True).S - Sr))
        d_un.append(abs(W.amplitudes(sysm, E, uu).S - Sr))
    assert d_avg[0] > d_avg[1] > d_avg[2], d_avg
    assert d_avg[2] < 0.02 and d_avg[2] < d_un[2], (d_avg, d_un)
