"""Pins for the oracle's Feshbach major/minor channel reduction (CPU only).

* the coarse lattice of the Chebyshev edge family is a sub-lattice of the
  fine one (every r-th edge), and the coarse packets built from the fine
  ones are orthonormal (R R^T = 1);
* with no coarsening the effective-kernel solution equals the unreduced
  solve of the whole system;
* the coarse-coarse elements obtained from the fine ones converge, as the
  quadrature is refined, to the elements computed directly on the coarse
  lattice; the fine-coarse elements agree with a Monte Carlo of the
  six-dimensional overlap between a fine cell and a coarse cell;
* the reduced P0 is symmetric; |S| = 1 below breakup; with a random real
  symmetric operator the elastic and breakup elements (minor channels on the
  coarse lattice included) conserve flux exactly;
* the effective-kernel form agrees with a direct solve of the coupled
  reduced system (a check of the partition).
"""
import math

import numpy as np
import pytest

import oracle.feshbach as F
import oracle.wpcd as W
from inputs import TOY_P, TOY_Q, YUK_RANGES

L2_CHANS = [(0, 2), (2, 0), (2, 2)]


def _pot(s):
    return W.Potential("yukawa", (-s, -s), YUK_RANGES)


@pytest.mark.parametrize("n,r", [(12, 2), (12, 3), (150, 2), (300, 3), (40, 4)])
def test_coarse_edges_are_every_rth_edge(n, r):
    fine = W.cheb_edges(n, 10.0)
    coarse = W.cheb_edges(n // r, 10.0)
    assert np.max(np.abs(fine[::r] - coarse)) <= 4e-15 * 10.0


def test_restriction_rows_orthonormal():
    sysm = W.build_system(W.cheb_edges(8, 6.0), W.cheb_edges(6, 6.0), 2, L2_CHANS, 4, 8,
                          _pot(1.5))
    R = F.restriction(sysm, 1, 2, 3)
    assert R.shape == (8 * 6 + 2 * 4 * 2, 3 * 8 * 6)
    RRt = (R @ R.T).toarray()
    assert np.max(np.abs(RRt - np.eye(R.shape[0]))) < 1e-15
    # each fine cell of a minor channel feeds exactly one coarse cell
    assert np.all(np.diff(R.tocsc().indptr) == 1)


@pytest.mark.parametrize("n_major", [1, 2])
def test_no_coarsening_equals_unreduced_solve(n_major):
    sysm = W.build_system(W.cheb_edges(7, 6.0), W.cheb_edges(8, 6.0), 2, L2_CHANS, 4, 8,
                          _pot(2.0))
    red = F.build_reduced(sysm, n_major, 1, 1)
    e0 = sysm.eps[0][0]
    for E in (e0 + 0.05, 0.4, 1.5):
        u = W.solve_lu(sysm, E)
        ur = F.solve_effective(red, E)
        assert np.max(np.abs(ur - u)) <= 1e-10 * np.max(np.abs(u)), E
        a, ar = W.amplitudes(sysm, E, u), F.amplitudes(red, E, ur)
        assert abs(ar.U00 - a.U00) <= 1e-10 * abs(a.U00)
        assert len(ar.breakup) == len(a.breakup)
        for x, y in zip(sorted(a.breakup, key=lambda t: t[:3]), sorted(ar.breakup, key=lambda t: t[:3])):
            assert x[:3] == y[:3] and abs(x[3] - y[3]) <= 1e-10


@pytest.mark.parametrize("rp,rq", [(1, 2), (2, 1), (2, 2)])
def test_coarse_elements_converge_to_direct_quadrature(rp, rq):
    """Two s-wave channels (L = 0) on the toy grid, the second minor: its
    block of the reduced P0 against P0 computed on the coarse lattice
    itself, for 8, 16 and 32 Gauss points per q bin and cosine interval."""
    p, q = np.array(TOY_P), np.array(TOY_Q)
    ncell = (p.size - 1) * (q.size - 1)
    errs = []
    for ng in (8, 16, 32):
        full = W.build_system(p, q, 0, [(0, 0), (0, 0)], ng, ng, _pot(2.0))
        red = F.build_reduced(full, 1, rp, rq)
        direct = W.build_system(p[::rp].copy(), q[::rq].copy(), 0, [(0, 0)], ng, ng, _pot(2.0))
        Pd = direct.P0_matrix().toarray()
        Pr = red.P0.toarray()[ncell:, ncell:]
        errs.append(np.max(np.abs(Pr - Pd)) / np.max(np.abs(Pd)))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 2e-3, errs


def test_coarse_multichannel_block_converges():
    """The same for the two d-wave channels of the L = 2 set."""
    p, q = np.array(TOY_P), np.array(TOY_Q)
    ncell = (p.size - 1) * (q.size - 1)
    errs = []
    for ng in (8, 24):
        full = W.build_system(p, q, 2, L2_CHANS, ng, ng, _pot(2.0))
        red = F.build_reduced(full, 1, 2, 2)
        direct = W.build_system(p[::2].copy(), q[::2].copy(), 2, L2_CHANS[1:], ng, ng, _pot(2.0))
        Pd = direct.P0_matrix().toarray()
        Pr = red.P0.toarray()[ncell:, ncell:]
        errs.append(np.max(np.abs(Pr - Pd)) / np.max(np.abs(Pd)))
    assert errs[1] < 0.5 * errs[0] and errs[1] < 3e-3, errs


def _mc_mixed(pr, qr, pc, qc, cells, n, rng):
    """Estimator of <X_ij|P|X_IJ> between cell (i, j) of the lattice (pr, qr)
    and cell (I, J) of the lattice (pc, qc): sample p, q uniformly in the
    first cell with isotropic directions, map to Jacobi sets 2 and 3 and test
    membership in the second cell (unit-weight packets)."""
    i, j, I, J = cells
    pa = rng.uniform(pr[i], pr[i + 1], n)
    qa = rng.uniform(qr[j], qr[j + 1], n)

    def unit(k):
        v = rng.normal(size=(k, 3))
        return v / np.linalg.norm(v, axis=1)[:, None]

    pv = pa[:, None] * unit(n)
    qv = qa[:, None] * unit(n)
    tot = np.zeros(n)
    for p2v, q2v in ((-0.5 * pv - 0.75 * qv, pv - 0.5 * qv), (-0.5 * pv + 0.75 * qv, -pv - 0.5 * qv)):
        p2 = np.linalg.norm(p2v, axis=1)
        q2 = np.linalg.norm(q2v, axis=1)
        inside = (p2 >= pc[I]) & (p2 < pc[I + 1]) & (q2 >= qc[J]) & (q2 < qc[J + 1])
        tot += np.where(inside, pa * qa / np.maximum(p2 * q2, 1e-300), 0.0)
    scale = math.sqrt((pr[i + 1] - pr[i]) * (qr[j + 1] - qr[j]) /
                      ((pc[I + 1] - pc[I]) * (qc[J + 1] - qc[J])))
    est = tot * scale
    return est.mean(), est.std() / math.sqrt(n)


@pytest.mark.parametrize("cells", [(1, 1, 0, 0), (2, 1, 0, 1), (1, 2, 1, 0)])
def test_fine_coarse_element_monte_carlo(cells):
    """A major (fine) row and a minor (coarse) column of the reduced P0."""
    p, q = np.array(TOY_P), np.array(TOY_Q)
    full = W.build_system(p, q, 0, [(0, 0), (0, 0)], 40, 40, _pot(2.0))
    red = F.build_reduced(full, 1, 2, 2)
    i, j, I, J = cells
    ncell = 16
    row, col = j * 4 + i, ncell + J * 2 + I
    val = red.P0[row, col]
    assert val > 1e-3
    assert abs(red.P0[col, row] - val) < 1e-14
    rng = np.random.default_rng(31 + 5 * i + 7 * j + 11 * I + 13 * J)
    pc, qc = p[::2].copy(), q[::2].copy()
    vals = [_mc_mixed(p, q, pc, qc, cells, 400_000, rng) for _ in range(6)]
    est = np.mean([v[0] for v in vals])
    err = math.sqrt(np.sum([v[1] ** 2 for v in vals])) / len(vals)
    assert abs(est - val) < 4.5 * err + 1e-3 * val, (est, err, val)


def test_reduced_p0_symmetric_and_structure():
    sysm = W.build_system(W.cheb_edges(8, 6.0), W.cheb_edges(9, 6.0), 2, L2_CHANS, 4, 8,
                          _pot(1.5))
    red = F.build_reduced(sysm, 1, 2, 3)
    d = (red.P0 - red.P0.T).tocsr()
    assert (abs(d).max() if d.nnz else 0.0) < 1e-14 * abs(red.P0).max()
    # the structure is the union of the fine patterns; the product above
    # drops the entries that sum to exact zeros (channel blocks that vanish
    # for a cell pair), so its pattern lies inside the union
    ptr, col = F.structure(red)
    rows = np.repeat(np.arange(ptr.size - 1), np.diff(ptr))
    assert set(zip(*red.P0.nonzero())) <= set(zip(rows.tolist(), col.tolist()))
    v = F.values_on(red, ptr, col)
    assert np.count_nonzero(v) == red.P0.nnz


def test_reduced_unitarity_below_breakup():
    sysm = W.build_system(W.cheb_edges(10, 6.0), W.cheb_edges(10, 6.0), 2, L2_CHANS, 4, 8,
                          _pot(2.0))
    red = F.build_reduced(sysm, 1, 2, 2)
    e0 = sysm.eps[0][0]
    for E in (e0 + 0.02, e0 + 0.2):
        assert E < min(red.minor.eps[w][0] for w in red.minor.eps)
        a = F.amplitudes(red, E, F.solve_effective(red, E))
        assert abs(abs(a.S) - 1.0) < 1e-12
        assert a.breakup == []


@pytest.mark.parametrize("E", [0.4, 1.5])
def test_reduced_breakup_exact_unitarity_symmetric_operator(E):
    """As for the unreduced system: with a random real symmetric operator in
    place of A and the reduced resolvent, |S_00|^2 + sum |S_k0|^2 = 1 over
    the open states of the fine and the coarse channels alike."""
    sysm = W.build_system(W.cheb_edges(8, 6.0), W.cheb_edges(9, 6.0), 2, L2_CHANS, 4, 8,
                          _pot(1.5), with_p0=False)
    sysm.row_ptr = np.zeros(sysm.Np * sysm.Nq + 1, dtype=np.int64)
    sysm.col = np.zeros(0, dtype=np.int32)
    sysm.val = np.zeros((0, 3, 3))
    red = F.build_reduced(sysm, 1, 2, 3)
    rng = np.random.default_rng(7)
    M = red.M
    Rn = rng.normal(size=(M, M))
    A = 0.2 * (Rn + Rn.T) / math.sqrt(M)
    G = F.resolvent(red, E)
    idx = F.entrance(red, E)[3]
    e0 = np.zeros(M)
    e0[idx] = 1.0
    u = np.linalg.solve(np.eye(M) - A * G[None, :], A @ e0)
    a = F.amplitudes(red, E, u)
    assert {c for (c, _, _, _) in a.breakup} == {0, 1, 2}
    total = abs(a.S) ** 2 + sum(abs(s) ** 2 for (_, _, _, s) in a.breakup)
    assert abs(total - 1.0) < 1e-12, total


def test_effective_kernel_equals_coupled_solve():
    sysm = W.build_system(W.cheb_edges(8, 6.0), W.cheb_edges(8, 6.0), 2, L2_CHANS, 4, 8,
                          _pot(2.0))
    red = F.build_reduced(sysm, 1, 2, 2)
    for E in (0.3, 1.2):
        for averaged in (False, True):
            G = F.resolvent(red, E, averaged)
            idx = F.entrance(red, E)[3]
            rhs = np.zeros(red.M)
            rhs[idx] = 1.0
            b = F.apply_A(red, rhs)
            u, its, res = W.gmres(lambda y: y - F.apply_A(red, G * y), b, tol=1e-13)
            ur = F.solve_effective(red, E, averaged)
            assert np.max(np.abs(u - ur)) <= 1e-10 * np.max(np.abs(ur)), (E, averaged)
