"""Oracle pins for three nucleons in pair s-waves (Sec. III.B eq.(gal) with
the spin-isospin coefficients; Sec. V.A).  CPU only."""
import math

import numpy as np
import pytest

import oracle.wpcd as W
import oracle.nucleons as N
from inputs import YUK_RANGES, NUC_DOUBLET, NUC_QUARTET, NUC_SINGLET_MULT


def test_clebsch_textbook_values():
    r2 = 1.0 / math.sqrt(2.0)
    assert N.clebsch(0.5, 0.5, 0.5, -0.5, 0, 0) == pytest.approx(r2, abs=1e-15)
    assert N.clebsch(0.5, -0.5, 0.5, 0.5, 0, 0) == pytest.approx(-r2, abs=1e-15)
    assert N.clebsch(0.5, 0.5, 0.5, -0.5, 1, 0) == pytest.approx(r2, abs=1e-15)
    assert N.clebsch(0.5, 0.5, 0.5, 0.5, 1, 1) == pytest.approx(1.0, abs=1e-15)
    # spin 1 x 1/2 -> 1/2: <1 1, 1/2 -1/2 | 1/2 1/2> = sqrt(2/3),
    # <1 0, 1/2 1/2 | 1/2 1/2> = -sqrt(1/3)
    assert N.clebsch(1, 1, 0.5, -0.5, 0.5, 0.5) == pytest.approx(math.sqrt(2 / 3), abs=1e-15)
    assert N.clebsch(1, 0, 0.5, 0.5, 0.5, 0.5) == pytest.approx(-math.sqrt(1 / 3), abs=1e-15)
    assert N.clebsch(1, 1, 0.5, 0.5, 1.5, 1.5) == pytest.approx(1.0, abs=1e-15)


def test_coupled_states_orthonormal():
    for S2, chans in ((1, [0, 1]), (3, [1])):
        v = [N.coupled_state(s, S2 / 2, S2 / 2) for s in chans]
        G = np.array([[a @ b for b in v] for a in v])
        assert np.allclose(G, np.eye(len(v)), atol=1e-14)


def test_recoupling_is_fixed_by_the_symmetric_group():
    """The spin-isospin part of C + C^2 is 2 on the totally antisymmetric
    spin-isospin state (which pairs with the symmetric space state) and -1
    on the mixed-symmetry ones (the two-dimensional irrep: the cyclic
    permutation has eigenvalues exp(+-2 pi i/3)); so g = (C + C^2)/2 has
    eigenvalues {1, -1/2} in the doublet and -1/2 in the quartet (totally
    symmetric spin times the mixed isospin doublet), for every M_S, M_T."""
    for ms, mt in ((1, 1), (-1, 1), (1, -1), (-1, -1)):
        g = N.recoupling(1, NUC_DOUBLET, two_MS=ms, two_MT=mt)
        assert np.allclose(g, g.T, atol=1e-14)
        assert np.allclose(np.sort(np.linalg.eigvalsh(g)), [-0.5, 1.0], atol=1e-14)
    for ms in (3, 1, -1, -3):
        g = N.recoupling(3, NUC_QUARTET, two_MS=ms)
        assert g.shape == (1, 1) and abs(g[0, 0] + 0.5) < 1e-14


def _pot(p):
    s = W.fit_strength(p, YUK_RANGES, -0.1)
    return W.Potential("yukawa", (-s, -s), YUK_RANGES)


def test_equal_pair_forces_split_into_boson_kernels():
    """With the same pair potential in both channels the doublet kernel is
    the boson kernel on g's eigenvectors: its spectrum below the pair
    threshold is that of K_boson together with that of -K_boson / 2."""
    p = W.cheb_edges(10, 10.0)
    pot = _pot(p)
    bos = W.build_system(p, p.copy(), 0, [(0, 0)], 8, 16, pot)
    nuc = N.build_system_nucleons(p, p.copy(), 1, NUC_DOUBLET, 8, 16, pot)
    for E in (-1.0, -0.3, -0.12):
        Kb = W.dense_K(bos, W.resolvent(bos, E).real)
        Kn = W.dense_K(nuc, W.resolvent(nuc, E).real)
        eb = np.sort_complex(np.concatenate([np.linalg.eigvals(Kb), np.linalg.eigvals(-0.5 * Kb)]))
        en = np.sort_complex(np.linalg.eigvals(Kn))
        scale = np.abs(eb).max()
        assert np.allclose(en.real, eb.real, atol=1e-10 * scale)
        assert np.allclose(en.imag, eb.imag, atol=1e-10 * scale)
    # hence the same three-body bound state (the spatially symmetric one)
    e_b = W.bound_state(bos, -3.0, -0.1 - 1e-4, tol=1e-10)
    e_n = W.bound_state(nuc, -3.0, -0.1 - 1e-4, tol=1e-10)
    assert abs(e_b - e_n) < 1e-8 * abs(e_b)


def _nucleons(n, two_S):
    p = W.cheb_edges(n, 10.0)
    pot = _pot(p)
    if two_S == 1:
        return N.build_system_nucleons(p, p.copy(), 1, NUC_DOUBLET, 8, 16, pot,
                                       [[1.0, 1.0], list(NUC_SINGLET_MULT)])
    return N.build_system_nucleons(p, p.copy(), 3, NUC_QUARTET, 8, 16, pot)


@pytest.mark.parametrize("two_S", [1, 3])
def test_unitarity_below_breakup(two_S):
    sysm = _nucleons(20, two_S)
    assert abs(sysm.eps[0][0] + 0.1) < 1e-12          # the deuteron channel
    if two_S == 1:
        assert sysm.eps[1][0] > 0.0                     # no bound 1S0 pair
    for E in (-0.07, -0.02):
        u, _, res = W.solve_gmres(sysm, E)
        assert res < 1e-12
        a = W.amplitudes(sysm, E, u)
        assert abs(abs(a.S) - 1.0) < 1e-12
        assert a.breakup == []


def test_quartet_has_no_three_body_bound_state():
    sysm = _nucleons(20, 3)
    for E in (-3.0, -1.0, -0.3, -0.1 - 1e-3):
        assert W.kernel_top_eig(sysm, E) < 1.0


@pytest.mark.parametrize("E", [-0.05, 0.3, 1.5])
def test_equal_pair_forces_amplitudes_from_boson_solves(E):
    """With one pair potential in every channel, P0 = g (x) P0_boson and the
    pair waves coincide, so on g's eigenvectors w (g w = lambda w) the
    equation splits into boson equations with the kernel lambda K_boson.
    The entrance element of the solution is then
        U = sum_lambda lambda (w . e_0)^2 [(1 - lambda K_b)^-1 b_b]_idx
    (doublet: lambda = 1 and -1/2, weights 1/2 each; quartet: the channel
    alone, lambda = -1/2), at any energy."""
    p = W.cheb_edges(12, 10.0)
    pot = _pot(p)
    bos = W.build_system(p, p.copy(), 0, [(0, 0)], 8, 16, pot)
    a0, j0, q0, idx = W.entrance(bos, E)
    Kb = W.dense_K(bos, W.resolvent(bos, E))
    bb = W.rhs(bos, idx)
    M = bos.M

    def ub(lam):
        return np.linalg.solve(np.eye(M) - lam * Kb, bb)[idx]

    for two_S, chans, expect in ((1, NUC_DOUBLET, 0.5 * ub(1.0) - 0.25 * ub(-0.5)),
                                 (3, NUC_QUARTET, -0.5 * ub(-0.5))):
        nuc = N.build_system_nucleons(p, p.copy(), two_S, chans, 8, 16, pot)
        u = W.solve_lu(nuc, E)
        assert W.entrance(nuc, E)[3] == idx
        assert abs(u[idx] - expect) <= 1e-10 * abs(expect)


def test_breakup_elements_exact_unitarity_two_pair_waves():
    """Exact unitarity of the open-channel S-matrix for a random real
    symmetric operator in place of A (see test_oracle_solve): with the
    doublet's two channels and their different pair waves, the open
    pseudostates of both channels enter the flux sum, each at its own
    pair energies."""
    p = W.cheb_edges(9, 8.0)
    pot = _pot(p)
    sysm = N.build_system_nucleons(p, p.copy(), 1, NUC_DOUBLET, 4, 8, pot,
                                   [[1.0, 1.0], list(NUC_SINGLET_MULT)])
    rng = np.random.default_rng(7)
    M = sysm.M
    R = rng.normal(size=(M, M))
    A = 0.2 * (R + R.T) / math.sqrt(M)
    for E in (0.4, 1.5):
        G = W.resolvent(sysm, E).ravel()
        idx = W.entrance(sysm, E)[3]
        e0 = np.zeros(M)
        e0[idx] = 1.0
        u = np.linalg.solve(np.eye(M) - A * G[None, :], A @ e0)
        a = W.amplitudes(sysm, E, u)
        total = abs(a.S) ** 2 + sum(abs(s) ** 2 for (_, _, _, s) in a.breakup)
        assert {c for (c, _, _, _) in a.breakup} == {0, 1}
        assert abs(total - 1.0) < 1e-12, (E, total)
