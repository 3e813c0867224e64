"""Pins for the oracle's lattice permutation matrix P0 (CPU only).

* Monte Carlo of the six-dimensional overlap <X_ij | P | X_i'j'> sampled in
  Jacobi set 1 and mapped to sets 2 and 3 -- independent of the delta-function
  reduction, the cosine clipping and the Gauss rule;
* the s-wave cosine integral against its closed form
  int dx/(pi1 pi2) = (2/(q q')) ln(pi1 + pi2) |_{x_lo}^{x_hi};
* symmetry and non-negativity of the s-wave P0;
* the pre-selection is a necessary condition: every pair it drops evaluates
  to exactly zero under the rule;
* the angular coupling G: 1 in the s-wave, the Legendre addition theorem for
  L = 0, the exchange symmetry G_ab(q,q',x) = G_ba(q',q,x), its bipolar-
  harmonic definition evaluated with scipy's spherical harmonics (l, lam up
  to 4), and the node-shared evaluation of the quadrature against the
  single-pair routine;
* multichannel elements (L = 2+, five channels with l, lam up to 4) against a
  Monte Carlo of the six-dimensional overlap with bipolar harmonics.
"""
import math

import numpy as np
import pytest
from numpy.polynomial.legendre import Legendre

import oracle.wpcd as W
from inputs import C1, TOY_P, TOY_Q


def _mc_swave(p, q, i, j, i2, j2, n, rng):
    """Estimator of <X_ij|P|X_i'j'>: sample p in D_i, q in D_j uniformly and
    isotropic directions; map to the two other Jacobi sets."""
    pa = rng.uniform(p[i], p[i + 1], n)
    qa = rng.uniform(q[j], q[j + 1], n)

    def unit(k):
        v = rng.normal(size=(k, 3))
        return v / np.linalg.norm(v, axis=1)[:, None]

    pv = pa[:, None] * unit(n)
    qv = qa[:, None] * unit(n)
    total = np.zeros(n)
    for p2v, q2v in ((-0.5 * pv - 0.75 * qv, pv - 0.5 * qv),     # set 2
                     (-0.5 * pv + 0.75 * qv, -pv - 0.5 * qv)):   # set 3
        p2 = np.linalg.norm(p2v, axis=1)
        q2 = np.linalg.norm(q2v, axis=1)
        inside = (p2 >= p[i2]) & (p2 < p[i2 + 1]) & (q2 >= q[j2]) & (q2 < q[j2 + 1])
        total += np.where(inside, pa * qa / np.maximum(p2 * q2, 1e-300), 0.0)
    di, dj = p[i + 1] - p[i], q[j + 1] - q[j]
    d2i, d2j = p[i2 + 1] - p[i2], q[j2 + 1] - q[j2]
    est = total * math.sqrt(di * dj / (d2i * d2j))
    return est.mean(), est.std() / math.sqrt(n)


def _elem(p, q, i, j, i2, j2, n_gq, n_gx):
    np_ = p.size - 1
    return W.p0_pairs(p, q, n_gq, n_gx, 0, [(0, 0)],
                      np.array([j * np_ + i]), np.array([j2 * np_ + i2]))[0, 0, 0]


@pytest.mark.parametrize("cells", [(1, 1, 1, 1), (2, 1, 1, 2), (0, 1, 1, 0), (2, 2, 1, 3), (2, 0, 0, 2),
                                   (0, 0, 0, 0)])
def test_p0_element_monte_carlo(cells):
    p, q = np.array(TOY_P), np.array(TOY_Q)
    i, j, i2, j2 = cells
    rule = _elem(p, q, i, j, i2, j2, 8, 16)
    fine = _elem(p, q, i, j, i2, j2, 64, 64)
    rng = np.random.default_rng(1508 + 7 * i + 13 * j + 17 * i2 + 19 * j2)
    est, err = 0.0, 0.0
    batches = 8
    vals = [_mc_swave(p, q, i, j, i2, j2, 500_000, rng) for _ in range(batches)]
    est = np.mean([v[0] for v in vals])
    err = math.sqrt(np.sum([v[1] ** 2 for v in vals])) / batches
    assert fine > 0.0
    assert abs(est - fine) < 4.5 * err + 1e-4 * fine, (est, err, fine)
    # the 8 x 8 x 16 rule is a quadrature of the same integral
    assert abs(rule - fine) < 2e-2 * fine, (rule, fine)


def test_p0_rule_converges_with_nodes():
    p, q = np.array(TOY_P), np.array(TOY_Q)
    ref = _elem(p, q, 2, 1, 1, 2, 96, 96)
    errs = [abs(_elem(p, q, 2, 1, 1, 2, n, n) - ref) for n in (4, 8, 16, 32)]
    assert errs[-1] < errs[0] and errs[-1] < 1e-3 * ref


def test_swave_cosine_integral_closed_form():
    """With one Gauss point per q bin (the bin midpoints, weight 2) the element
    is (dq dq')^(1/2) (d d')^(-1/2) q q' int dx/(pi1 pi2)."""
    p = W.cheb_edges(12, 10.0)
    q = W.cheb_edges(12, 10.0)
    checked = 0
    ptr, col = W.preselect(p, q)
    cand = []
    for r in (12 * 6 + 5, 12 * 4 + 7, 12 * 8 + 8, 12 * 9 + 3, 12 * 2 + 6):
        for c in col[ptr[r]:ptr[r + 1]][::3]:
            cand.append((r % 12, r // 12, int(c) % 12, int(c) // 12))
    for (i, j, i2, j2) in cand:
        if min(i, i2) < 2:
            continue
        qa = 0.5 * (q[j] + q[j + 1]); qb = 0.5 * (q[j2] + q[j2 + 1])
        A = qb * qb + 0.25 * qa * qa; C = qa * qa + 0.25 * qb * qb; B = qa * qb
        xlo = max(-1.0, (p[i] ** 2 - A) / B, (p[i2] ** 2 - C) / B)
        xhi = min(1.0, (p[i + 1] ** 2 - A) / B, (p[i2 + 1] ** 2 - C) / B)
        if xhi <= xlo:
            continue
        f = lambda x: math.log(math.sqrt(A + B * x) + math.sqrt(C + B * x))
        exact = 2.0 / B * (f(xhi) - f(xlo))
        pref = math.sqrt((q[j + 1] - q[j]) * (q[j2 + 1] - q[j2])
                         / ((p[i + 1] - p[i]) * (p[i2 + 1] - p[i2]))) * qa * qb
        for nx, tol in ((16, 1e-9), (40, 1e-13)):
            got = _elem(p, q, i, j, i2, j2, 1, nx) / pref
            assert abs(got - exact) <= tol * exact, (nx, got, exact)
        checked += 1
    assert checked >= 6


def test_swave_cosine_integral_closed_form_lowest_bins():
    """The same closed form for every selected cell pair with a p bin at
    p = 0 or next to it (i or i' in {0, 1}), where pi1 or pi2 reaches zero
    inside the cosine interval and the integrand has an inverse-square-root
    end point: the mapped Gauss rule converges more slowly there, so the
    bound is looser at 16 points and 1e-10 only at 64."""
    n = 12
    p = W.cheb_edges(n, 10.0)
    q = W.cheb_edges(n, 10.0)
    ptr, col = W.preselect(p, q)
    checked = 0
    worst16 = 0.0
    for r in range(n * n):
        i, j = r % n, r // n
        for c in col[ptr[r]:ptr[r + 1]]:
            i2, j2 = int(c) % n, int(c) // n
            if min(i, i2) >= 2:
                continue
            qa = 0.5 * (q[j] + q[j + 1]); qb = 0.5 * (q[j2] + q[j2 + 1])
            A = qb * qb + 0.25 * qa * qa; C = qa * qa + 0.25 * qb * qb; B = qa * qb
            xlo = max(-1.0, (p[i] ** 2 - A) / B, (p[i2] ** 2 - C) / B)
            xhi = min(1.0, (p[i + 1] ** 2 - A) / B, (p[i2 + 1] ** 2 - C) / B)
            if xhi <= xlo:
                continue
            f = lambda x: math.log(math.sqrt(max(A + B * x, 0.0)) + math.sqrt(max(C + B * x, 0.0)))
            exact = 2.0 / B * (f(xhi) - f(xlo))
            pref = math.sqrt((q[j + 1] - q[j]) * (q[j2 + 1] - q[j2])
                             / ((p[i + 1] - p[i]) * (p[i2 + 1] - p[i2]))) * qa * qb
            e16 = abs(_elem(p, q, i, j, i2, j2, 1, 16) / pref - exact) / exact
            e64 = abs(_elem(p, q, i, j, i2, j2, 1, 64) / pref - exact) / exact
            worst16 = max(worst16, e16)
            assert e16 <= 1e-3, (i, j, i2, j2, e16)
            assert e64 <= 1e-10, (i, j, i2, j2, e64)
            checked += 1
    assert checked >= 30
    # the p = 0 end point is really met: the 16-point rule is visibly worse
    assert worst16 > 1e-6


def test_p0_symmetric_nonnegative_c1():
    p = W.cheb_edges(C1["n_p"], C1["p_max"])
    q = W.cheb_edges(C1["n_q"], C1["q_max"])
    ptr, col = W.preselect(p, q)
    ncell = (p.size - 1) * (q.size - 1)
    rows = np.repeat(np.arange(ncell, dtype=np.int64), np.diff(ptr))
    val = W.p0_pairs(p, q, C1["n_gq"], C1["n_gx"], 0, [(0, 0)], rows, col)[:, 0, 0]
    import scipy.sparse as sp
    P = sp.csr_matrix((val, col, ptr), shape=(ncell, ncell))
    # structure symmetric exactly, values up to rounding order
    Sfull = sp.csr_matrix((np.ones_like(val), col, ptr), shape=(ncell, ncell))
    assert (Sfull - Sfull.T).nnz == 0
    assert abs(P - P.T).max() <= 1e-14 * abs(P).max()
    assert val.min() >= 0.0
    assert int(ptr[-1]) == 53105
    # the selected pairs are mostly nonzero under the rule
    assert np.count_nonzero(val) > 0.9 * val.size


@pytest.mark.parametrize("n", [6, 11])
def test_preselection_is_necessary(n):
    """Evaluate the rule on every cell pair of a small grid: nothing outside
    the selected structure is nonzero."""
    p = W.cheb_edges(n, 10.0)
    q = W.cheb_edges(n + 1, 7.0)
    ncell = n * (n + 1)
    rows = np.repeat(np.arange(ncell, dtype=np.int64), ncell)
    cols = np.tile(np.arange(ncell, dtype=np.int32), ncell)
    val = W.p0_pairs(p, q, 8, 16, 0, [(0, 0)], rows, cols)[:, 0, 0].reshape(ncell, ncell)
    ptr, col = W.preselect(p, q)
    mask = np.zeros((ncell, ncell), dtype=bool)
    for r in range(ncell):
        mask[r, col[ptr[r]:ptr[r + 1]]] = True
    assert np.all(val[~mask] == 0.0)
    assert np.count_nonzero(val[mask]) > 0.8 * mask.sum()
    # a single-pair query agrees with the brute-force structure
    for r in (0, ncell // 2, ncell - 1):
        i, j = r % n, r // n
        for c in range(ncell):
            assert W.lib().orc_is_selected(W._p(p, W.ctypes.c_double), W._p(q, W.ctypes.c_double),
                                           i, j, c % n, c // n) == int(mask[r, c])


def test_geom_G_swave_is_one():
    for (q, q2, x) in [(0.3, 1.7, -0.4), (2.0, 0.1, 0.99), (1.0, 1.0, 0.0)]:
        assert abs(W.geom_G(0, (0, 0), (0, 0), q, q2, x) - 1.0) < 1e-14


@pytest.mark.parametrize("ll", [(0, 2), (2, 0), (2, 2), (4, 2)])
def test_geom_G_L0_addition_theorem(ll):
    """For L = 0 the bipolar harmonic is (-1)^l sqrt(2l+1)/(4 pi) P_l(a.b), so
    G = (-1)^(l+l') sqrt((2l+1)(2l'+1)) P_l(pi1^.q^) P_l'(pi2^.q'^)."""
    l, l2 = ll
    for (q, q2, x) in [(0.3, 1.7, -0.4), (2.0, 0.7, 0.6), (1.0, 1.3, -0.9)]:
        s = math.sqrt(1 - x * x)
        qv = np.array([q * s, 0, q * x]); q2v = np.array([0, 0, q2])
        pi1 = q2v + 0.5 * qv; pi2 = -(qv + 0.5 * q2v)
        c1 = pi1 @ qv / (np.linalg.norm(pi1) * q)
        c2 = pi2 @ q2v / (np.linalg.norm(pi2) * q2)
        ref = (-1) ** (l + l2) * math.sqrt((2 * l + 1) * (2 * l2 + 1)) \
            * Legendre.basis(l)(c1) * Legendre.basis(l2)(c2)
        got = W.geom_G(0, (l, l), (l2, l2), q, q2, x)
        assert abs(got - ref) < 1e-12 * max(1.0, abs(ref))


def test_geom_G_exchange_symmetry():
    chans = [(0, 2), (2, 0), (2, 2)]
    for a in chans:
        for b in chans:
            for (q, q2, x) in [(0.3, 1.7, -0.4), (2.0, 0.7, 0.6)]:
                g1 = W.geom_G(2, a, b, q, q2, x)
                g2 = W.geom_G(2, b, a, q2, q, x)
                assert abs(g1 - g2) < 1e-12 * max(1.0, abs(g1))


def test_structure_regression_fixture():
    import hashlib
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "structure.json")) as f:
        gold = json.load(f)
    g = gold["40x40"]
    p = W.cheb_edges(g["n_p"], g["p_max"])
    ptr, col = W.preselect(p, W.cheb_edges(g["n_q"], g["q_max"]))
    h = hashlib.sha256()
    h.update(ptr.astype("<i8").tobytes())
    h.update(col.astype("<i4").tobytes())
    assert int(ptr[-1]) == g["nnz_cells"]
    assert h.hexdigest() == g["sha256_rowptr_i64_col_i32"]


def _cg_py(j1, m1, j2, m2, J, M):
    """Clebsch-Gordan coefficient from the Racah formula (test-side copy)."""
    f = math.factorial
    if m1 + m2 != M or abs(m1) > j1 or abs(m2) > j2 or abs(M) > J or not abs(j1 - j2) <= J <= j1 + j2:
        return 0.0
    pre = math.sqrt((2 * J + 1) * f(J + j1 - j2) * f(J - j1 + j2) * f(j1 + j2 - J) / f(j1 + j2 + J + 1))
    pre *= math.sqrt(f(J + M) * f(J - M) * f(j1 - m1) * f(j1 + m1) * f(j2 - m2) * f(j2 + m2))
    s = 0.0
    for k in range(0, j1 + j2 + J + 1):
        args = (j1 + j2 - J - k, j1 - m1 - k, j2 + m2 - k, J - j2 + m1 + k, J - j1 - m2 + k)
        if min(args) < 0:
            continue
        s += (-1) ** k / (f(k) * f(args[0]) * f(args[1]) * f(args[2]) * f(args[3]) * f(args[4]))
    return pre * s


def _ylm(l, m, v):
    from scipy.special import sph_harm_y
    r = np.linalg.norm(v, axis=1)
    theta = np.arccos(np.clip(v[:, 2] / r, -1, 1))
    phi = np.arctan2(v[:, 1], v[:, 0])
    return sph_harm_y(l, m, theta, phi)


def _bip(L, M, l, lam, a, b):
    out = np.zeros(a.shape[0], dtype=complex)
    for m in range(-l, l + 1):
        mu = M - m
        if abs(mu) > lam:
            continue
        c = _cg_py(l, m, lam, mu, L, M)
        if c:
            out += c * _ylm(l, m, a) * _ylm(lam, mu, b)
    return out


def _mc_channel(p, q, cells, L, M, ch1, ch2, n, rng):
    i, j, i2, j2 = cells
    pa = rng.uniform(p[i], p[i + 1], n)
    qa = rng.uniform(q[j], q[j + 1], n)

    def unit(k):
        v = rng.normal(size=(k, 3))
        return v / np.linalg.norm(v, axis=1)[:, None]

    pv = pa[:, None] * unit(n)
    qv = qa[:, None] * unit(n)
    left = np.conj(_bip(L, M, ch1[0], ch1[1], pv, qv))
    total = np.zeros(n, dtype=complex)
    for p2v, q2v in ((-0.5 * pv - 0.75 * qv, pv - 0.5 * qv), (-0.5 * pv + 0.75 * qv, -pv - 0.5 * qv)):
        p2 = np.linalg.norm(p2v, axis=1)
        q2 = np.linalg.norm(q2v, axis=1)
        inside = (p2 >= p[i2]) & (p2 < p[i2 + 1]) & (q2 >= q[j2]) & (q2 < q[j2 + 1])
        right = _bip(L, M, ch2[0], ch2[1], p2v, q2v)
        total += np.where(inside, pa * qa / np.maximum(p2 * q2, 1e-300) * right, 0.0)
    d = math.sqrt((p[i + 1] - p[i]) * (q[j + 1] - q[j]) / ((p[i2 + 1] - p[i2]) * (q[j2 + 1] - q[j2])))
    est = (4 * math.pi) ** 2 * d * (left * total).real
    return est.mean(), est.std() / math.sqrt(n)


@pytest.mark.parametrize("pair", [((0, 2), (0, 2)), ((0, 2), (2, 0)), ((2, 2), (2, 0)), ((2, 2), (2, 2)),
                                  ((2, 4), (4, 2)), ((4, 2), (0, 2)), ((2, 4), (2, 2))])
def test_multichannel_element_monte_carlo(pair):
    """L = 2+ channel pair of one cell pair against a Monte Carlo of the
    six-dimensional overlap with bipolar harmonics (two values of M); the
    element is computed in the five-channel set, so the node-shared
    coupling of the quadrature is checked for l or lam = 4 as well."""
    p, q = np.array(TOY_P), np.array(TOY_Q)
    cells = (1, 1, 1, 2)
    chans = FIVE_CH
    a, b = chans.index(pair[0]), chans.index(pair[1])
    fine = W.p0_pairs(p, q, 48, 48, 2, chans, np.array([1 * 4 + 1]), np.array([2 * 4 + 1]))[0, a, b]
    assert abs(fine) > 1e-3
    rng = np.random.default_rng(99 + 3 * a + b)
    for M in (0, 1):
        vals = [_mc_channel(p, q, cells, 2, M, pair[0], pair[1], 400_000, rng) for _ in range(5)]
        est = np.mean([v[0] for v in vals])
        err = math.sqrt(np.sum([v[1] ** 2 for v in vals])) / len(vals)
        assert abs(est - fine) < 4.5 * err + 2e-3 * abs(fine), (M, est, err, fine)


def test_multichannel_block_symmetry():
    p = W.cheb_edges(8, 6.0)
    q = W.cheb_edges(9, 6.0)
    ch = [(0, 2), (2, 0), (2, 2)]
    ptr, col = W.preselect(p, q)
    ncell = 72
    rows = np.repeat(np.arange(ncell, dtype=np.int64), np.diff(ptr))
    vals = W.p0_pairs(p, q, 8, 16, 2, ch, rows, col)
    import scipy.sparse as sp
    R, C, V = [], [], []
    for a in range(3):
        for b in range(3):
            R.append(rows + a * ncell)
            C.append(col.astype(np.int64) + b * ncell)
            V.append(vals[:, a, b])
    P = sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))), shape=(3 * ncell,) * 2)
    assert abs(P - P.T).max() <= 1e-13 * abs(P).max()


FIVE_CH = [(0, 2), (2, 0), (2, 2), (2, 4), (4, 2)]


def _nodes(seed, n):
    rng = np.random.default_rng(seed)
    return [(rng.uniform(0.05, 4.0), rng.uniform(0.05, 4.0), rng.uniform(-1.0, 1.0)) for _ in range(n)] \
        + [(0.8, 1.3, 1.0), (1.1, 0.4, -1.0), (0.6, 1.2, 0.0)]


@pytest.mark.parametrize("L,chans", [(2, FIVE_CH), (0, [(0, 0), (2, 2), (4, 4)]),
                                     (4, [(0, 4), (4, 0), (2, 2), (2, 4), (4, 2), (4, 4)])])
def test_geom_G_node_shared_equals_pair_routine(L, chans):
    """The node-shared evaluation of G used inside the element quadrature
    (all channel pairs at once from one set of spherical harmonics) equals
    the single-pair routine for every channel pair, including l or lam = 4."""
    for (qq, q2, x) in _nodes(31 + L, 12):
        tab = W.geom_G_table(L, chans, qq, q2, x)
        for a, ca in enumerate(chans):
            for b, cb in enumerate(chans):
                g = W.geom_G(L, ca, cb, qq, q2, x)
                assert abs(tab[a, b] - g) <= 1e-13 * max(1.0, abs(g)), (ca, cb, qq, q2, x)


def _G_scipy(L, ca, cb, qq, q2, x):
    """16 pi^2/(2L+1) sum_M conj(Y^{LM}_{l lam}(pi1^, q^)) Y^{LM}_{l' lam'}(pi2^, q'^) at the
    canonical geometry, from scipy's spherical harmonics and the test-side
    Clebsch-Gordan coefficients."""
    s = math.sqrt((1.0 - x) * (1.0 + x))
    qv = np.array([[qq * s, 0.0, qq * x]]); q2v = np.array([[0.0, 0.0, q2]])
    pi1 = q2v + 0.5 * qv; pi2 = -(qv + 0.5 * q2v)
    acc = 0.0
    for M in range(-L, L + 1):
        acc += (np.conj(_bip(L, M, ca[0], ca[1], pi1, qv)) * _bip(L, M, cb[0], cb[1], pi2, q2v))[0]
    return 16.0 * math.pi ** 2 / (2 * L + 1) * acc.real


def test_geom_G_five_channels_vs_scipy_harmonics():
    """G for every pair of the five L = 2+ channels (l, lam up to 4) against
    an evaluation of its bipolar-harmonic definition with scipy's spherical
    harmonics, which shares nothing with the oracle's Legendre recursion."""
    for (qq, q2, x) in _nodes(7, 6):
        for ca in FIVE_CH:
            for cb in FIVE_CH:
                g = W.geom_G(2, ca, cb, qq, q2, x)
                ref = _G_scipy(2, ca, cb, qq, q2, x)
                assert abs(g - ref) <= 1e-11 * max(1.0, abs(ref)), (ca, cb, qq, q2, x, g, ref)
