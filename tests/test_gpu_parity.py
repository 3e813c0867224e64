"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars: structure (row_ptr, col) bit-exact; FP64 values and amplitudes within
1e-10 relative; FP32-compensated values within the bound derived in the
design notes (a few FP32 ulps on every element); run-to-run determinism.
"""
import math
import sys

import numpy as np
import pytest

import oracle.wpcd as O
from inputs import C1, C2, TOY_P, TOY_Q, YAM_BETA, YAM_LAMBDA, YUK_RANGES

pytestmark = pytest.mark.gpu

YAM = dict(kind="yamaguchi", strength=[YAM_LAMBDA], range=[YAM_BETA])
ENERGIES = (-0.08, -0.05, -0.02, 0.05, 0.2, 0.5, 1.0, 2.0)
FP32_REL = 2e-6     # per-element relative bound for the FP32-compensated path


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_1508_07441_amd as P
    return P


@pytest.fixture(scope="module")
def ctx(P):
    c = P.Context(0)
    yield c
    c.close()


def _oracle_values(p, q, ngq, ngx, ptr, col):
    rows = np.repeat(np.arange(ptr.size - 1, dtype=np.int64), np.diff(ptr))
    return O.p0_pairs(p, q, ngq, ngx, 0, [(0, 0)], rows, col)[:, 0, 0]


def _check_structure_and_values(ctx, P, p, q, ngq, ngx, label):
    say(f"[{label}] build_p FP64 n_p={p.size-1} n_q={q.size-1} ngq={ngq} ngx={ngx}")
    nnz = ctx.build_p(P.WPCD_FP64)
    rp, col, val = ctx.get_p()
    ptr_o, col_o = O.preselect(p, q)
    assert nnz == int(ptr_o[-1])
    assert np.array_equal(rp, ptr_o)
    assert np.array_equal(col, col_o)
    vo = _oracle_values(p, q, ngq, ngx, ptr_o, col_o)
    v = val[:, 0, 0]
    scale = np.abs(vo).max() if vo.size else 1.0
    err = np.abs(v - vo)
    assert np.all(err <= 1e-10 * np.abs(vo) + 1e-14 * scale), float(np.max(err / (np.abs(vo) + scale * 1e-14)))
    say(f"[{label}] FP64 max rel err {np.max(err / np.maximum(np.abs(vo), 1e-300 + 1e-14 * scale)):.2e}")
    say(f"[{label}] build_p MIXED")
    ctx.build_p(P.WPCD_MIXED)
    rp2, col2, val2 = ctx.get_p()
    assert np.array_equal(rp2, ptr_o) and np.array_equal(col2, col_o)
    e32 = np.abs(val2[:, 0, 0] - vo)
    rel32 = np.max(e32 / np.maximum(np.abs(vo), 1e-30 + 1e-7 * scale)) if vo.size else 0.0
    say(f"[{label}] FP32 max rel err {rel32:.2e}")
    assert np.all(e32 <= FP32_REL * np.abs(vo) + 1e-7 * scale * 1e-3)
    return vo


def test_c1_p0_parity(ctx, P):
    n = C1["n_p"]
    ctx.build_basis(n, n, 10.0, 10.0, C1["n_gq"], C1["n_gx"], potential=YAM)
    p = O.cheb_edges(n, 10.0)
    _check_structure_and_values(ctx, P, p, p.copy(), C1["n_gq"], C1["n_gx"], "C1")


@pytest.mark.parametrize("shape", [(37, 23, 8.0, 6.0, 5, 7), (2, 2, 1.0, 1.0, 8, 16),
                                   (64, 65, 10.0, 10.0, 3, 20), (17, 40, 10.0, 10.0, 9, 4)])
def test_ragged_grids_p0_parity(ctx, P, shape):
    n_p, n_q, pm, qm, ngq, ngx = shape
    ctx.build_basis(n_p, n_q, pm, qm, ngq, ngx, potential=YAM)
    p, q = O.cheb_edges(n_p, pm), O.cheb_edges(n_q, qm)
    _check_structure_and_values(ctx, P, p, q, ngq, ngx, f"ragged{shape}")


def test_explicit_edges_p0_parity(ctx, P):
    p, q = np.array(TOY_P), np.array(TOY_Q)
    ctx.build_basis(4, 4, 0, 0, 8, 16, potential=YAM, p_edges=p, q_edges=q)
    _check_structure_and_values(ctx, P, p, q, 8, 16, "toy")


def test_c2_structure_full_size(ctx, P):
    """Full 150 x 150 structure against the oracle's committed digest."""
    import hashlib
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "structure.json")) as f:
        g = json.load(f)["150x150"]
    say("[C2] structure")
    ctx.build_basis(150, 150, 10.0, 10.0, 8, 20, potential=YAM)
    nnz = ctx.build_p(P.WPCD_FP64)
    rp, col, val = ctx.get_p()
    h = hashlib.sha256()
    h.update(rp.astype("<i8").tobytes())
    h.update(col.astype("<i4").tobytes())
    assert nnz == g["nnz_cells"]
    assert h.hexdigest() == g["sha256_rowptr_i64_col_i32"]
    # sampled rows of values, oracle element by element: the FP64 elements,
    # then the FP32-compensated ones of the bench's element kernel (8-point
    # q rule, 20-point cosine rule) on the same rows
    say("[C2] build_p MIXED")
    ctx.build_p(P.WPCD_MIXED)
    _, _, val32 = ctx.get_p()
    rng = np.random.default_rng(7)
    rows = np.sort(rng.choice(150 * 150, 120, replace=False))
    p = O.cheb_edges(150, 10.0)
    worst = 0.0
    for r in rows[:120]:
        cols = col[rp[r]:rp[r + 1]]
        vo = O.p0_pairs(p, p, 8, 20, 0, [(0, 0)], np.full(cols.size, r, dtype=np.int64), cols)[:, 0, 0]
        v = val[rp[r]:rp[r + 1], 0, 0]
        sc = max(np.abs(vo).max(), 1e-300) if vo.size else 1.0
        assert np.all(np.abs(v - vo) <= 1e-10 * np.abs(vo) + 1e-14 * sc)
        v32 = val32[rp[r]:rp[r + 1], 0, 0]
        assert np.all(np.abs(v32 - vo) <= FP32_REL * np.abs(vo) + 1e-10 * sc), r
        if vo.size:
            worst = max(worst, float(np.max(np.abs(v32 - vo) / np.maximum(np.abs(vo), 1e-10 * sc))))
    say(f"[C2] FP32 elements on 120 sampled rows: max rel err {worst:.2e}")


@pytest.mark.parametrize("shape", [(100, 150), (128, 256), (200, 170)])
def test_structure_scan_paths(ctx, P, shape):
    """Row pointers when the scan runs in one tile of 16384 rows (ragged),
    in exactly two, and in three with a ragged last one: every row pointer
    nondecreasing from 0, and sampled rows' column lists equal the oracle's
    brute-force ones (rows at the tile seams included)."""
    n_p, n_q = shape
    say(f"[scan] {n_p}x{n_q} rows={n_p * n_q}")
    ctx.build_basis(n_p, n_q, 10.0, 10.0, 8, 16, potential=YAM)
    nnz = ctx.build_p(P.WPCD_MIXED)
    rp, col, _ = ctx.get_p(values=False)
    assert rp[0] == 0 and rp[-1] == nnz and np.all(np.diff(rp) >= 0)
    p, q = O.cheb_edges(n_p, 10.0), O.cheb_edges(n_q, 10.0)
    rng = np.random.default_rng(11)
    seams = [t * 16384 + d for t in (1, 2) for d in (-1, 0, 1) if 0 <= t * 16384 + d < n_p * n_q]
    rows = np.unique(np.concatenate([np.array([0, 1, n_p * n_q - 1] + seams, dtype=np.int64),
                                     rng.choice(n_p * n_q, 40, replace=False)]))
    ptr_o, col_o = O.preselect(p, q, rows)
    for k, r in enumerate(rows):
        assert np.array_equal(col[rp[r]:rp[r + 1]], col_o[ptr_o[k]:ptr_o[k + 1]]), r


def test_determinism(ctx, P):
    ctx.build_basis(40, 40, 10.0, 10.0, 8, 16, potential=YAM)
    for prec in (P.WPCD_FP64, P.WPCD_MIXED):
        say(f"[det] prec={prec}")
        ctx.build_p(prec)
        a = ctx.get_p()
        ctx.build_p(prec)
        b = ctx.get_p()
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_pair_spectrum_parity(ctx, P):
    n = 40
    ctx.build_basis(n, n, 10.0, 10.0, 8, 16, potential=YAM)
    eps, Og, _ = ctx.pair_spectrum(0)
    p = O.cheb_edges(n, 10.0)
    e_o, O_o = O.pair_diag(p, O.yamaguchi_v(p, YAM_LAMBDA, YAM_BETA))
    assert np.max(np.abs(eps - e_o)) <= 1e-12 * np.abs(e_o).max()
    # rows are eigenvectors with the same sign rule; compare up to FP64 noise
    assert np.max(np.abs(Og - O_o)) < 1e-9
    np.testing.assert_allclose(Og @ Og.T, np.eye(n), atol=1e-12)


@pytest.mark.parametrize("n,l", [(37, 0), (40, 2), (150, 0), (161, 0), (161, 2)])
def test_pair_spectrum_yukawa(ctx, P, n, l):
    """Pair spectrum of a two-range Yukawa sum against the oracle: odd and
    even sizes, both Jacobi paths (one workgroup up to 160 bins, block-cyclic
    above), s and d waves.  Eigenvectors to FP64 noise scaled by the
    eigenvalue gap (the condition number of each vector)."""
    pot = dict(kind="yukawa", strength=[-1.3, -0.8], range=list(YUK_RANGES))
    chans = [(0, 0)] if l == 0 else [(0, 2), (2, 0), (2, 2)]
    say(f"[pair] n={n} l={l}")
    ctx.build_basis(n, n, 10.0, 10.0, 8, 16, channels=chans, L=0 if l == 0 else 2, potential=pot)
    eps, Og, _ = ctx.pair_spectrum(l)
    p = O.cheb_edges(n, 10.0)
    v = sum(O.yukawa_v(p, s_, mu, l) for s_, mu in zip(pot["strength"], pot["range"]))
    e_o, O_o = O.pair_diag(p, v)
    scale = np.abs(e_o).max()
    # the s-wave oracle integrates the potential in closed form, the library by
    # 24-point Gauss quadrature: agreement to ~1e-12
    assert np.max(np.abs(eps - e_o)) <= 1e-11 * scale
    gap = np.full(n, np.inf)
    d = np.diff(e_o)
    gap[:-1] = np.minimum(gap[:-1], d)
    gap[1:] = np.minimum(gap[1:], d)
    err = np.abs(Og - O_o).max(axis=1)
    assert np.all(err <= 1e-12 * scale / gap + 1e-9), float(np.max(err * gap / scale))
    np.testing.assert_allclose(Og @ Og.T, np.eye(n), atol=1e-12)


def _oracle_system_yam(n, ngx):
    p = O.cheb_edges(n, 10.0)
    pot = O.Potential("yamaguchi", (YAM_LAMBDA,), (YAM_BETA,))
    return O.build_system(p, p.copy(), 0, [(0, 0)], 8, ngx, pot)


def test_c1_amplitudes_fp64(ctx, P):
    n = C1["n_p"]
    ctx.build_basis(n, n, 10.0, 10.0, 8, C1["n_gx"], potential=YAM)
    ctx.build_p(P.WPCD_FP64)
    say("[C1] solve FP64")
    res = ctx.solve(ENERGIES, P.WPCD_FP64)
    sysm = _oracle_system_yam(n, C1["n_gx"])
    for r, E in zip(res, ENERGIES):
        assert r.status == P.WPCD_OK, (E, P.STATUS_NAMES[r.status])
        u, _, _ = O.solve_gmres(sysm, E)
        a = O.amplitudes(sysm, E, u)
        U = complex(r.U_re, r.U_im)
        assert abs(U - a.U00) <= 1e-10 * abs(a.U00), (E, U, a.U00)
        assert abs(complex(r.S_re, r.S_im) - a.S) <= 1e-10
        if E < 0:
            assert abs(math.hypot(r.S_re, r.S_im) - 1.0) < 1e-12
        else:
            assert r.eta <= 1.0 + 1e-12
        assert r.residual < 1e-11


def test_c1_breakup_parity(ctx, P):
    n = C1["n_p"]
    ctx.build_basis(n, n, 10.0, 10.0, 8, C1["n_gx"], potential=YAM)
    ctx.build_p(P.WPCD_FP64)
    E = 0.5
    res, br = ctx.solve([E], P.WPCD_FP64, want_breakup=True)
    sysm = _oracle_system_yam(n, C1["n_gx"])
    u, _, _ = O.solve_gmres(sysm, E)
    a = O.amplitudes(sysm, E, u)
    assert res[0].n_open == len(a.breakup)
    got = {(int(r[0]), int(r[1]), int(r[2])): complex(r[3], r[4]) for r in br[0]}
    for (ch, k, jk, S) in a.breakup:
        assert abs(got[(ch, k, jk)] - S) <= 1e-10 * max(abs(S), 1e-3)


def test_status_codes(ctx, P):
    n = 40
    ctx.build_basis(n, n, 10.0, 10.0, 8, 16, potential=YAM)
    ctx.build_p(P.WPCD_FP64)
    eps, _, _ = ctx.pair_spectrum(0, want_O=False)
    q = O.cheb_edges(n, 10.0)
    e_edge = eps[0] + 0.75 * q[10] ** 2
    res = ctx.solve([eps[0] - 0.01, eps[0], float("nan"), 80.0, e_edge, 0.5], P.WPCD_FP64)
    st = [r.status for r in res]
    assert st[0] == P.WPCD_E_BELOW_THRESHOLD
    assert st[1] == P.WPCD_E_BELOW_THRESHOLD
    assert st[2] == P.WPCD_E_INVALID
    assert st[3] == P.WPCD_E_INVALID
    assert st[4] == P.WPCD_E_ON_EDGE
    assert st[5] == P.WPCD_OK
    # an empty energy list is a valid call with no results
    assert ctx.solve([], P.WPCD_FP64) == []
    # state errors
    c2 = P.Context(0)
    with pytest.raises(P.WpcdError) as ei:
        c2.build_p(P.WPCD_FP64)
    assert ei.value.status == P.WPCD_E_STATE
    c2.close()


def test_c2_full_fp64_and_mixed(ctx, P):
    """Bench configuration: Yukawa sum fitted to a pair level at -0.1,
    150 x 150 bins, 20-point cosine rule, 8 energies."""
    n = C2["n_p"]
    pot = dict(kind="yukawa", strength=[-1.0, -1.0], range=list(YUK_RANGES), fit_e2=-0.1)
    say("[C2] build_basis with fit")
    ctx.build_basis(n, n, 10.0, 10.0, 8, C2["n_gx"], potential=pot)
    eps, _, scale = ctx.pair_spectrum(0, want_O=False)
    p = O.cheb_edges(n, 10.0)
    s_o = O.fit_strength(p, YUK_RANGES, -0.1)
    assert abs(scale - s_o) <= 1e-10 * s_o
    assert abs(eps[0] + 0.1) < 1e-12
    opot = O.Potential("yukawa", (-s_o, -s_o), YUK_RANGES)
    sysm = O.build_system(p, p.copy(), 0, [(0, 0)], 8, C2["n_gx"], opot)
    ctx.build_p(P.WPCD_FP64)
    say("[C2] solve FP64")
    res = ctx.solve(C2["energies"], P.WPCD_FP64)
    ref = {}
    for r, E in zip(res, C2["energies"]):
        assert r.status == P.WPCD_OK, (E, P.STATUS_NAMES[r.status])
        u, _, _ = O.solve_gmres(sysm, E)
        a = O.amplitudes(sysm, E, u)
        ref[E] = a.U00
        U = complex(r.U_re, r.U_im)
        assert abs(U - a.U00) <= 1e-10 * abs(a.U00), (E, U, a.U00)
    say("[C2] build_p MIXED + solve")
    ctx.build_p(P.WPCD_MIXED)
    res2 = ctx.solve(C2["energies"], P.WPCD_MIXED)
    worst = 0.0
    for r, E in zip(res2, C2["energies"]):
        assert r.status == P.WPCD_OK
        U = complex(r.U_re, r.U_im)
        worst = max(worst, abs(U - ref[E]) / abs(ref[E]))
    say(f"[C2] mixed max rel amplitude error vs FP64 oracle: {worst:.3e}")
    assert worst <= 1e-6     # the mixed tier's amplitude gate
    say("[C2] solve MIXED_REFINE")
    res3 = ctx.solve(C2["energies"], P.WPCD_MIXED_REFINE)
    worst = 0.0
    for r, E in zip(res3, C2["energies"]):
        assert r.status == P.WPCD_OK and r.residual <= 1e-8
        U = complex(r.U_re, r.U_im)
        worst = max(worst, abs(U - ref[E]) / abs(ref[E]))
    say(f"[C2] mixed+refine max rel amplitude error vs FP64 oracle: {worst:.3e}")
    assert worst <= 1e-6
    say("[C2] solve MIXED_BF16")
    res4 = ctx.solve(C2["energies"], P.WPCD_MIXED_BF16)
    worst = 0.0
    for r, E in zip(res4, C2["energies"]):
        assert r.status == P.WPCD_OK and r.residual <= 1e-8
        U = complex(r.U_re, r.U_im)
        worst = max(worst, abs(U - ref[E]) / abs(ref[E]))
    say(f"[C2] mixed+BF16 max rel amplitude error vs FP64 oracle: {worst:.3e}, "
        f"iterations {[r.iters for r in res4]}")
    assert worst <= 1e-6


# ------------------------------------------------------------ multichannel
L2_CHANS = [(0, 2), (2, 0), (2, 2)]


def _yuk_pot(scale=1.0):
    return dict(kind="yukawa", strength=[-scale, -scale], range=list(YUK_RANGES))


@pytest.mark.parametrize("shape", [(12, 12, 8.0, 8.0, 8, 16), (10, 13, 6.0, 7.0, 5, 9)])
def test_multichannel_p0_parity(ctx, P, shape):
    n_p, n_q, pm, qm, ngq, ngx = shape
    say(f"[mc{shape}] build_p FP64")
    ctx.build_basis(n_p, n_q, pm, qm, ngq, ngx, channels=L2_CHANS, L=2, potential=_yuk_pot(2.0))
    nnz = ctx.build_p(P.WPCD_FP64)
    rp, col, val = ctx.get_p()
    p, q = O.cheb_edges(n_p, pm), O.cheb_edges(n_q, qm)
    ptr_o, col_o = O.preselect(p, q)
    assert np.array_equal(rp, ptr_o) and np.array_equal(col, col_o)
    rows = np.repeat(np.arange(n_p * n_q, dtype=np.int64), np.diff(ptr_o))
    vo = O.p0_pairs(p, q, ngq, ngx, 2, L2_CHANS, rows, col_o)
    scale = np.abs(vo).max()
    err = np.abs(val - vo)
    assert np.all(err <= 1e-10 * np.abs(vo) + 1e-13 * scale), float(err.max() / scale)
    say(f"[mc{shape}] build_p MIXED")
    ctx.build_p(P.WPCD_MIXED)
    _, _, v32 = ctx.get_p()
    assert np.all(np.abs(v32 - vo) <= 1e-6 * np.abs(vo) + 1e-7 * scale)


L2_CHANS5 = [(0, 2), (2, 0), (2, 2), (2, 4), (4, 2)]


def test_five_channel_p0_and_amplitudes(ctx, P):
    """Channels up to l = 4, lambda = 4 (coupling polynomials of degree 6,
    the general element kernel, the 5-channel block SpMM) against the
    oracle, FP64 and FP32 values and FP64 amplitudes."""
    n = 10
    ctx.build_basis(n, n, 8.0, 8.0, 8, 12, channels=L2_CHANS5, L=2, potential=_yuk_pot(2.0))
    say("[mc5] build_p FP64")
    ctx.build_p(P.WPCD_FP64)
    rp, col, val = ctx.get_p()
    p = O.cheb_edges(n, 8.0)
    ptr_o, col_o = O.preselect(p, p.copy())
    assert np.array_equal(rp, ptr_o) and np.array_equal(col, col_o)
    rows = np.repeat(np.arange(n * n, dtype=np.int64), np.diff(ptr_o))
    vo = O.p0_pairs(p, p.copy(), 8, 12, 2, L2_CHANS5, rows, col_o)
    scale = np.abs(vo).max()
    err = np.abs(val - vo)
    assert np.all(err <= 1e-10 * np.abs(vo) + 1e-13 * scale), float(err.max() / scale)
    say("[mc5] solve FP64")
    energies = [0.1, 0.9]
    res = ctx.solve(energies, P.WPCD_FP64)
    pot = O.Potential("yukawa", (-2.0, -2.0), YUK_RANGES)
    sysm = O.build_system(p, p.copy(), 2, L2_CHANS5, 8, 12, pot)
    for r, E in zip(res, energies):
        assert r.status == P.WPCD_OK, (E, P.STATUS_NAMES[r.status])
        u, _, _ = O.solve_gmres(sysm, E)
        a = O.amplitudes(sysm, E, u)
        U = complex(r.U_re, r.U_im)
        assert abs(U - a.U00) <= 1e-10 * abs(a.U00), (E, U, a.U00)
    say("[mc5] build_p MIXED")
    ctx.build_p(P.WPCD_MIXED)
    _, _, v32 = ctx.get_p()
    assert np.all(np.abs(v32 - vo) <= 1e-6 * np.abs(vo) + 1e-7 * scale)


def test_multichannel_amplitudes_fp64(ctx, P):
    n = 16
    scale = 2.0
    ctx.build_basis(n, n, 8.0, 8.0, 8, 16, channels=L2_CHANS, L=2, potential=_yuk_pot(scale))
    ctx.build_p(P.WPCD_FP64)
    energies = [-0.3, 0.2, 0.8]
    eps0, _, _ = ctx.pair_spectrum(0, want_O=False)
    assert eps0[0] < energies[0]
    say("[mc16] solve FP64")
    res = ctx.solve(energies, P.WPCD_FP64, want_breakup=False)
    p = O.cheb_edges(n, 8.0)
    pot = O.Potential("yukawa", (-scale, -scale), YUK_RANGES)
    sysm = O.build_system(p, p.copy(), 2, L2_CHANS, 8, 16, pot)
    assert np.max(np.abs(sysm.eps[0] - eps0)) < 1e-11 * np.abs(sysm.eps[0]).max()
    for r, E in zip(res, energies):
        assert r.status == P.WPCD_OK, (E, P.STATUS_NAMES[r.status])
        u, _, _ = O.solve_gmres(sysm, E)
        a = O.amplitudes(sysm, E, u)
        U = complex(r.U_re, r.U_im)
        assert abs(U - a.U00) <= 1e-10 * abs(a.U00), (E, U, a.U00)
        if E < 0:
            assert abs(math.hypot(r.S_re, r.S_im) - 1.0) < 1e-12
    # the mixed tiers on the same system (block products of three channels on
    # the FP32 and BF16 matrix cores): the 1e-6 amplitude gate
    refs = {E: O.amplitudes(sysm, E, O.solve_gmres(sysm, E)[0]).U00 for E in energies}
    ctx.build_p(P.WPCD_MIXED)
    for prec in (P.WPCD_MIXED, P.WPCD_MIXED_REFINE, P.WPCD_MIXED_BF16):
        say(f"[mc16] solve precision {prec}")
        for r, E in zip(ctx.solve(energies, prec), energies):
            assert r.status == P.WPCD_OK and r.residual <= 1e-8, (prec, E)
            U = complex(r.U_re, r.U_im)
            assert abs(U - refs[E]) <= 1e-6 * abs(refs[E]), (prec, E, U, refs[E])


def test_c3_structure_and_sampled_values(ctx, P):
    """300 x 300 bins, three L = 2+ channels (270,000 basis): structure against
    the oracle's digest; sampled cell-pair blocks element by element."""
    import hashlib
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "structure.json")) as f:
        g = json.load(f)["300x300"]
    say("[C3] build_basis + build_p FP64")
    ctx.build_basis(300, 300, 10.0, 10.0, 8, 20, channels=L2_CHANS, L=2, potential=_yuk_pot(1.5))
    nnz = ctx.build_p(P.WPCD_FP64)
    assert nnz == g["nnz_cells"]
    rp, col, val = ctx.get_p()
    h = hashlib.sha256()
    h.update(rp.astype("<i8").tobytes())
    h.update(col.astype("<i4").tobytes())
    assert h.hexdigest() == g["sha256_rowptr_i64_col_i32"]
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(nnz, 400, replace=False))
    rows = np.searchsorted(rp, idx, side="right") - 1
    p = O.cheb_edges(300, 10.0)
    vo = O.p0_pairs(p, p.copy(), 8, 20, 2, L2_CHANS, rows.astype(np.int64), col[idx])
    scale = np.abs(val).max()
    assert np.all(np.abs(val[idx] - vo) <= 1e-10 * np.abs(vo) + 1e-13 * scale)
    # the FP32 elements of the 270k basis's own kernel (moments of the
    # coupling polynomials, 20-point cosine rule) on the same blocks
    say("[C3] build_p MIXED")
    assert ctx.build_p(P.WPCD_MIXED) == nnz
    _, _, v32 = ctx.get_p()
    err = np.abs(v32[idx] - vo)
    say(f"[C3] FP32 blocks: max err / scale {err.max() / scale:.2e}")
    assert np.all(err <= 1e-6 * np.abs(vo) + 1e-7 * scale)


def _oracle_l2_system(n, ngx, e2=-0.1):
    """The oracle's 3-channel L = 2+ system on an n x n grid (Yukawa sum
    fitted to a pair level at e2), P0 computed once."""
    p = O.cheb_edges(n, 10.0)
    s_o = O.fit_strength(p, YUK_RANGES, e2)
    sysm = O.build_system(p, p.copy(), 2, L2_CHANS, 8, ngx,
                          O.Potential("yukawa", (-s_o, -s_o), YUK_RANGES), with_p0=False)
    sysm.row_ptr, sysm.col = O.preselect(p, p.copy())
    rows = np.repeat(np.arange(n * n, dtype=np.int64), np.diff(sysm.row_ptr))
    sysm.val = O.p0_pairs(p, p.copy(), 8, ngx, 2, L2_CHANS, rows, sysm.col)
    return sysm


def test_three_channel_rule_of_the_270k_basis(ctx, P):
    """The 270k basis's quadrature rule (8 q points, 20 cosine points) and
    channels on a 40 x 40 grid (4,800 basis states): every FP32 element of
    its kernel against the oracle, and the amplitudes of all four precision
    tiers against the oracle's (FP64 1e-10, mixed tiers 1e-6)."""
    n = 40
    fit = dict(kind="yukawa", strength=[-1.0, -1.0], range=list(YUK_RANGES), fit_e2=-0.1)
    say("[mc40] oracle system")
    sysm = _oracle_l2_system(n, 20)
    vo = sysm.val
    scale = np.abs(vo).max()
    ctx.build_basis(n, n, 10.0, 10.0, 8, 20, channels=L2_CHANS, L=2, potential=fit)
    say("[mc40] build_p MIXED")
    nnz = ctx.build_p(P.WPCD_MIXED)
    rp, col, v32 = ctx.get_p()
    assert nnz == int(sysm.row_ptr[-1])
    assert np.array_equal(rp, sysm.row_ptr) and np.array_equal(col, sysm.col)
    err = np.abs(v32 - vo)
    say(f"[mc40] FP32 elements: max err / scale {err.max() / scale:.2e}")
    assert np.all(err <= 1e-6 * np.abs(vo) + 1e-7 * scale)
    energies = [-0.05, 0.5, 1.5]
    refs = {}
    for E in energies:
        u, _, _ = O.solve_gmres(sysm, E)
        refs[E] = O.amplitudes(sysm, E, u).U00
    for prec in (P.WPCD_MIXED, P.WPCD_MIXED_REFINE, P.WPCD_MIXED_BF16):
        say(f"[mc40] solve precision {prec}")
        for r, E in zip(ctx.solve(energies, prec), energies):
            assert r.status == P.WPCD_OK, (prec, E, P.STATUS_NAMES[r.status])
            U = complex(r.U_re, r.U_im)
            say(f"[mc40]   E={E}: rel err {abs(U - refs[E]) / abs(refs[E]):.2e}, {r.iters} it")
            assert abs(U - refs[E]) <= 1e-6 * abs(refs[E]), (prec, E, U, refs[E])
    say("[mc40] build_p FP64 + solve")
    ctx.build_p(P.WPCD_FP64)
    for r, E in zip(ctx.solve(energies, P.WPCD_FP64), energies):
        assert r.status == P.WPCD_OK
        U = complex(r.U_re, r.U_im)
        assert abs(U - refs[E]) <= 1e-10 * abs(refs[E]), (E, U, refs[E])


def test_three_channel_fp32_elements_full_grid(ctx, P):
    """Every FP32 element of a ragged-size 3-channel grid with the 270k
    basis's rule (n_q = 8, n_x = 20) against the oracle."""
    n_p, n_q = 23, 27
    ctx.build_basis(n_p, n_q, 9.0, 11.0, 8, 20, channels=L2_CHANS, L=2, potential=_yuk_pot(1.3))
    say("[mc23x27] build_p MIXED")
    nnz = ctx.build_p(P.WPCD_MIXED)
    rp, col, v32 = ctx.get_p()
    p, q = O.cheb_edges(n_p, 9.0), O.cheb_edges(n_q, 11.0)
    ptr_o, col_o = O.preselect(p, q)
    assert nnz == int(ptr_o[-1]) and np.array_equal(rp, ptr_o) and np.array_equal(col, col_o)
    rows = np.repeat(np.arange(n_p * n_q, dtype=np.int64), np.diff(ptr_o))
    vo = O.p0_pairs(p, q, 8, 20, 2, L2_CHANS, rows, col_o)
    scale = np.abs(vo).max()
    err = np.abs(v32 - vo)
    say(f"[mc23x27] FP32 elements: max err / scale {err.max() / scale:.2e}")
    assert np.all(err <= 1e-6 * np.abs(vo) + 1e-7 * scale)


def test_err_vs_fp64_matches_true_error(ctx, P):
    """The per-amplitude error estimate of the mixed tiers (one FP64
    refinement step's correction) against the true difference from the
    oracle's amplitude, at 8 energies below and above breakup on a 60 x 60
    s-wave grid with the bench's rule; NaN when not asked for; tiny in
    FP64."""
    n = 60
    fit = dict(kind="yukawa", strength=[-1.0, -1.0], range=list(YUK_RANGES), fit_e2=-0.1)
    ctx.build_basis(n, n, 10.0, 10.0, 8, 20, potential=fit)
    p = O.cheb_edges(n, 10.0)
    s_o = O.fit_strength(p, YUK_RANGES, -0.1)
    sysm = O.build_system(p, p.copy(), 0, [(0, 0)], 8, 20,
                          O.Potential("yukawa", (-s_o, -s_o), YUK_RANGES))
    ref = {E: O.amplitudes(sysm, E, O.solve_gmres(sysm, E)[0]).U00 for E in ENERGIES}
    ctx.build_p(P.WPCD_MIXED)
    assert all(math.isnan(r.err_vs_fp64) for r in ctx.solve(ENERGIES, P.WPCD_MIXED))
    for prec in (P.WPCD_MIXED, P.WPCD_MIXED_REFINE, P.WPCD_MIXED_BF16):
        say(f"[err] precision {prec}")
        for r in ctx.solve(ENERGIES, prec, err_est=True):
            assert r.status == P.WPCD_OK
            true = abs(complex(r.U_re, r.U_im) - ref[r.E]) / abs(ref[r.E])
            say(f"[err]   E={r.E:+.2f}: reported {r.err_vs_fp64:.3e} true {true:.3e}")
            assert abs(r.err_vs_fp64 - true) <= 0.05 * true + 2e-10, (prec, r.E)
    ctx.build_p(P.WPCD_FP64)
    for r in ctx.solve(ENERGIES, P.WPCD_FP64, err_est=True):
        assert r.status == P.WPCD_OK and r.err_vs_fp64 < 1e-10, (r.E, r.err_vs_fp64)


def _check_averaged(ctx, P, sysm, energies, label, prec, tol):
    """Amplitudes and the breakup distribution with the energy-averaged
    resolvent against the oracle's."""
    res, dist = ctx.solve(energies, prec, resolvent=P.WPCD_RESOLVENT_AVERAGED,
                          want_breakup=P.WPCD_BREAKUP_DIST)
    for r, rows, E in zip(res, dist, energies):
        assert r.status == P.WPCD_OK, (label, E, P.STATUS_NAMES[r.status])
        u, _, _ = O.solve_gmres(sysm, E, averaged=True)
        a = O.amplitudes(sysm, E, u, averaged=True)
        U = complex(r.U_re, r.U_im)
        assert abs(U - a.U00) <= tol * abs(a.U00), (label, E, U, a.U00)
        assert abs(complex(r.S_re, r.S_im) - a.S) <= tol * 10, (label, E)
        assert len(rows) == len(a.breakup_dist), (label, E, len(rows), len(a.breakup_dist))
        pmax = max([d[3] for d in a.breakup_dist], default=0.0)
        for g, o in zip(rows, a.breakup_dist):
            assert (int(g[0]), int(g[1]), int(g[4])) == (o[0], o[1], o[4]), (label, E, g, o)
            assert abs(g[2] - o[2]) <= 1e-12 * max(1.0, abs(o[2]))
            assert abs(g[3] - o[3]) <= tol * max(o[3], 1e-3 * pmax), (label, E, g[3], o[3])
        say(f"[{label}] E={E:+.3f}: |S|={abs(a.S):.12f} delta={math.degrees(a.delta):+.4f} deg, "
            f"{len(rows)} pseudostates open, sum P={sum(d[3] for d in a.breakup_dist):.4e}")
    return res


def test_averaged_resolvent_parity(ctx, P):
    """The energy-averaged channel resolvent (Sec. II.C): FP64 amplitudes and
    breakup distributions against the oracle's (1e-10) on an s-wave grid and
    a three-channel L = 2+ grid, the mixed tier within 1e-6; |S| = 1 below
    breakup; all energies of one bin alike; elements are refused with it."""
    n = 24
    ctx.build_basis(n, n, 10.0, 10.0, 8, 16, potential=YAM)
    ctx.build_p(P.WPCD_FP64)
    sysm = _oracle_system_yam(n, 16)
    energies = [-0.09, -0.04, 0.05, 0.3, 0.8, 1.7]
    say("[avg24] FP64")
    res = _check_averaged(ctx, P, sysm, energies, "avg24", P.WPCD_FP64, 1e-10)
    for r in res[:2]:
        assert abs(math.hypot(r.S_re, r.S_im) - 1.0) < 1e-12
    # histogram form: another energy of the same bin gives the same amplitude
    E1, E2 = O.energy_bin(sysm, 0.3)
    r2 = ctx.solve([E1 + 0.9 * (E2 - E1)], P.WPCD_FP64, resolvent=P.WPCD_RESOLVENT_AVERAGED)[0]
    assert abs(complex(r2.U_re, r2.U_im) - complex(res[3].U_re, res[3].U_im)) <= 1e-11 * abs(
        complex(res[3].U_re, res[3].U_im))
    # the distribution also with the resolvent at E (one bin per pseudostate)
    _, dist_e = ctx.solve([0.8], P.WPCD_FP64, want_breakup=P.WPCD_BREAKUP_DIST)
    a = O.amplitudes(sysm, 0.8, O.solve_gmres(sysm, 0.8)[0])
    assert len(dist_e[0]) == len(a.breakup_dist)
    for g, o in zip(dist_e[0], a.breakup_dist):
        assert int(g[4]) == 1 and abs(g[3] - o[3]) <= 1e-10 * max(o[3], 1e-12)
    with pytest.raises(P.WpcdError) as ei:
        ctx.solve([0.8], P.WPCD_FP64, resolvent=P.WPCD_RESOLVENT_AVERAGED,
                  want_breakup=P.WPCD_BREAKUP_ELEMENTS)
    assert ei.value.status == P.WPCD_E_INVALID
    say("[avg24] mixed")
    ctx.build_p(P.WPCD_MIXED)
    _check_averaged(ctx, P, sysm, energies, "avg24-mixed", P.WPCD_MIXED, 1e-6)
    # three channels
    nc = 12
    ctx.build_basis(nc, nc, 8.0, 8.0, 8, 16, channels=L2_CHANS, L=2, potential=_yuk_pot(2.0))
    ctx.build_p(P.WPCD_FP64)
    p = O.cheb_edges(nc, 8.0)
    sys3 = O.build_system(p, p.copy(), 2, L2_CHANS, 8, 16,
                          O.Potential("yukawa", (-2.0, -2.0), YUK_RANGES))
    say("[avg3ch] FP64")
    _check_averaged(ctx, P, sys3, [0.2, 0.9, 1.6], "avg3ch", P.WPCD_FP64, 1e-10)


def test_max_grid_1024(ctx, P):
    """The largest grid the library takes, 1024 x 1024 bins (cell indices up
    to 2^20 - 1, ~7e8 cell pairs, int64 offsets): sampled rows' columns and
    sampled FP32 elements against the oracle, and |S| = 1 below breakup (a
    property of the discrete equations at any size)."""
    n = 1024
    say("[max] build_basis 1024 x 1024")
    ctx.build_basis(n, n, 10.0, 10.0, 8, 16, potential=YAM)
    say("[max] build_p MIXED")
    nnz = ctx.build_p(P.WPCD_MIXED)
    say(f"[max] nnz={nnz}")
    rp, col, val = ctx.get_p()
    assert rp[0] == 0 and rp[-1] == nnz and np.all(np.diff(rp) >= 0)
    p = O.cheb_edges(n, 10.0)
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([[0, n * n - 1], rng.choice(n * n, 24, replace=False)]))
    ptr_o, col_o = O.preselect(p, p, rows)
    for k, r in enumerate(rows):
        assert np.array_equal(col[rp[r]:rp[r + 1]], col_o[ptr_o[k]:ptr_o[k + 1]]), r
    idx = np.sort(rng.choice(nnz, 300, replace=False))
    idx[-1] = nnz - 1
    r_idx = np.searchsorted(rp, idx, side="right") - 1
    vo = O.p0_pairs(p, p.copy(), 8, 16, 0, [(0, 0)], r_idx.astype(np.int64), col[idx])[:, 0, 0]
    scale = np.abs(val).max()
    assert np.all(np.abs(val[idx, 0, 0] - vo) <= FP32_REL * np.abs(vo) + 1e-7 * scale * 1e-3)
    del col, val
    say("[max] solve MIXED at E = -0.05")
    r = ctx.solve([-0.05], P.WPCD_MIXED)[0]
    assert r.status == P.WPCD_OK
    assert abs(abs(complex(r.S_re, r.S_im)) - 1.0) <= 1e-7


def test_repeat_builds_on_same_edges(ctx, P):
    """A build on the bin edges of the previous build (whose nonzero count
    then sizes the buffers before the new count is known) gives the same
    structure and values; a build on other edges in between, and the build
    after it, match the oracle's structure."""
    pa, qa = O.cheb_edges(40, 10.0), O.cheb_edges(44, 10.0)
    pb, qb = O.cheb_edges(37, 10.0), O.cheb_edges(29, 10.0)
    runs = []
    for p, q, tag in ((pa, qa, "a"), (pa, qa, "a again"), (pb, qb, "b"), (pa, qa, "a after b"),
                      (pa, qa, "a repeated")):
        ctx.build_basis(p.size - 1, q.size - 1, 10.0, 10.0, 8, 16, potential=YAM)
        say(f"[repeat builds] {tag}")
        for prec in (P.WPCD_MIXED, P.WPCD_FP64):
            nnz = ctx.build_p(prec)
            rp, col, val = ctx.get_p()
            ptr_o, col_o = O.preselect(p, q)
            assert nnz == int(ptr_o[-1]) == int(rp[-1])
            assert np.array_equal(rp, ptr_o) and np.array_equal(col, col_o)
            runs.append((tag[0], prec, val.copy()))
    for tag in "ab":
        for prec in (P.WPCD_MIXED, P.WPCD_FP64):
            vals = [v for t, pr, v in runs if t == tag and pr == prec]
            assert all(np.array_equal(v, vals[0]) for v in vals[1:])


# ------------------------------------------------------------- autotuning
def test_autotune_candidates_agree(ctx, P):
    """Every candidate launch shape (forced) and the measured choice give the
    amplitudes of the heuristic choice to rounding."""
    n = 24
    pot = dict(kind="yukawa", strength=[-1.0, -1.0], range=list(YUK_RANGES), fit_e2=-0.1)
    ctx.build_basis(n, n, 10.0, 10.0, 8, 16, channels=L2_CHANS, L=2, potential=pot)
    ctx.build_p(P.WPCD_FP64)
    E = [-0.05, 0.3, 1.1]
    ctx.set_autotune(P.WPCD_TUNE_HEURISTIC)
    ref = ctx.solve(E, P.WPCD_FP64)
    for mode in [P.WPCD_TUNE_FORCE + i for i in range(8)] + [P.WPCD_TUNE_MEASURE]:
        say(f"[tune] mode {mode}")
        ctx.set_autotune(mode)
        res = ctx.solve(E, P.WPCD_FP64)
        for a, b in zip(ref, res):
            assert b.status == P.WPCD_OK
            Ua, Ub = complex(a.U_re, a.U_im), complex(b.U_re, b.U_im)
            assert abs(Ua - Ub) <= 1e-12 * abs(Ua)
    ent = ctx.autotune()
    assert {e["name"] for e in ent} == {"block_apply", "vector_rows", "spmm"}
    for e in ent:
        assert 0 <= e["choice"] < e["n_candidates"] and e["us"] > 0.0
    ctx.set_autotune(P.WPCD_TUNE_HEURISTIC)


@pytest.mark.parametrize("chans", ["s", "L2"])
def test_tiled_spmm_ragged_grid(ctx, P, chans):
    """Every SpMM variant (forced in turn; the last ones visit the rows in
    lattice tiles) on a grid whose sides are not multiples of the tile and
    whose cell count is not a multiple of 8 (padding workgroups) gives the
    amplitudes of the plain launch to rounding."""
    np_, nq = 37, 43                     # 1591 cells
    if chans == "s":
        ctx.build_basis(np_, nq, 10.0, 10.0, 8, 16, potential=YAM)
    else:
        pot = dict(kind="yukawa", strength=[-1.0, -1.0], range=list(YUK_RANGES), fit_e2=-0.1)
        ctx.build_basis(np_, nq, 10.0, 10.0, 8, 16, channels=L2_CHANS, L=2, potential=pot)
    E = [-0.05, 0.4, 1.3]
    for prec in (P.WPCD_FP64, P.WPCD_MIXED):
        ctx.build_p(prec)
        ctx.set_autotune(P.WPCD_TUNE_FORCE)
        say(f"[tiled spmm] {chans} prec={prec} force 0")
        ref = ctx.solve(E, prec)
        for f in range(1, 8):                          # clamped past the last candidate
            ctx.set_autotune(P.WPCD_TUNE_FORCE + f)
            say(f"[tiled spmm] {chans} prec={prec} force {f}")
            res = ctx.solve(E, prec)
            for a, b in zip(ref, res):
                assert a.status == P.WPCD_OK and b.status == P.WPCD_OK
                Ua, Ub = complex(a.U_re, a.U_im), complex(b.U_re, b.U_im)
                assert abs(Ua - Ub) <= 1e-10 * abs(Ua)
    ctx.set_autotune(P.WPCD_TUNE_HEURISTIC)


def test_element_kernel_variants_identical(ctx, P):
    """The s-wave element kernel's launch variants (4 or 8 cell pairs per
    wavefront round; capped grid with several rounds per workgroup, or one
    round per workgroup) give bit-identical P values."""
    ctx.build_basis(80, 80, 10.0, 10.0, 8, 20, potential=YAM)
    for prec in (P.WPCD_FP64, P.WPCD_MIXED):
        ctx.set_autotune(P.WPCD_TUNE_FORCE)
        say(f"[elem variants] prec={prec} force 0")
        nnz = ctx.build_p(prec)
        assert nnz > 4 * 4 * 8192 * 2    # several rounds per workgroup
        ref = ctx.get_p()[2]
        for mode in [P.WPCD_TUNE_FORCE + i for i in (1, 2, 3)] + [P.WPCD_TUNE_MEASURE]:
            say(f"[elem variants] prec={prec} mode {mode}")
            ctx.set_autotune(mode)
            ctx.build_p(prec)
            assert np.array_equal(ctx.get_p()[2], ref)
        ent = [e for e in ctx.autotune() if e["name"] == "p0_elem"]
        assert len(ent) == 1 and ent[0]["n_candidates"] == 4 and ent[0]["us"] > 0.0
    ctx.set_autotune(P.WPCD_TUNE_HEURISTIC)


def test_graph_replays_match_eager(ctx, P):
    """Captured iteration graphs replayed over several solves, with other
    (eager and captured) work and synchronisations in between, give the
    eager launches' results bit for bit."""
    n = 24
    pot = dict(kind="yukawa", strength=[-1.0, -1.0], range=list(YUK_RANGES), fit_e2=-0.1)
    ctx.build_basis(n, n, 10.0, 10.0, 8, 16, channels=L2_CHANS, L=2, potential=pot)
    ctx.build_p(P.WPCD_FP64)
    EA = [-0.05, 0.2, 0.6, 1.1, 1.7]
    EB = [0.35, 0.9]
    ctx.set_graphs(False)
    refA = ctx.solve(EA, P.WPCD_FP64)
    refB = ctx.solve(EB, P.WPCD_FP64)
    ctx.set_graphs(True)
    for rep in range(3):
        say(f"[graphs] replay {rep}")
        for E, ref in ((EA, refA), (EB, refB)):
            res = ctx.solve(E, P.WPCD_FP64)
            ctx.synchronize()
            for a, b in zip(ref, res):
                assert b.status == P.WPCD_OK
                assert (a.U_re, a.U_im, a.iters) == (b.U_re, b.U_im, b.iters)
        ctx.pair_spectrum(0, want_O=False)   # eager work between replays


def test_solve_multi_uneven_systems(P):
    """Three systems of different size and channel count solved at once
    give the results of solving them one by one, and those equal the
    oracle's amplitudes."""
    yuk = dict(kind="yukawa", strength=[-1.0, -1.0], range=list(YUK_RANGES), fit_e2=-0.1)
    specs = [(16, [(0, 0)], 0, YAM, [0.1, 0.7]),
             (22, [(0, 2), (2, 0)], 2, yuk, [-0.05, 0.3, 0.9, 1.4]),
             (18, L2_CHANS, 2, yuk, [0.2, 1.1, 1.9])]
    ctxs = []
    for n, ch, L, pot, _ in specs:
        c = P.Context(0)
        c.build_basis(n, n, 10.0, 10.0, 8, 16, channels=ch, L=L, potential=pot)
        c.build_p(P.WPCD_FP64)
        ctxs.append(c)
    say("[multi] one by one")
    seq = [c.solve(sp[4], P.WPCD_FP64) for c, sp in zip(ctxs, specs)]
    for rep in range(2):
        say(f"[multi] together {rep}")
        res = P.wpcd_solve_multi([c.h for c in ctxs], [sp[4] for sp in specs], P.WPCD_FP64)
        for a_list, b_list in zip(seq, res):
            for a, b in zip(a_list, b_list):
                assert b.status == a.status == P.WPCD_OK
                assert (a.U_re, a.U_im, a.iters) == (b.U_re, b.U_im, b.iters)
    # and every system's amplitudes equal the oracle's
    for (n, ch, L, pot, Es), rs in zip(specs, seq):
        p = O.cheb_edges(n, 10.0)
        if pot is YAM:
            opot = O.Potential("yamaguchi", (YAM_LAMBDA,), (YAM_BETA,))
        else:
            s_o = O.fit_strength(p, YUK_RANGES, -0.1)
            opot = O.Potential("yukawa", (-s_o, -s_o), YUK_RANGES)
        sysm = O.build_system(p, p.copy(), L, ch, 8, 16, opot)
        for r, E in zip(rs, Es):
            a = O.amplitudes(sysm, E, O.solve_gmres(sysm, E)[0])
            U = complex(r.U_re, r.U_im)
            assert abs(U - a.U00) <= 1e-10 * abs(a.U00), (n, E, U, a.U00)
    with pytest.raises(P.WpcdError):
        P.wpcd_solve_multi([ctxs[0].h, ctxs[0].h], [[0.1], [0.2]], P.WPCD_FP64)
    for c in ctxs:
        c.close()


def test_save_load_p_and_device_energies(ctx, P, tmp_path):
    """A saved P0 loads into a context with the same basis (not another one)
    and solves identically; device-resident energies give the host results."""
    import ctypes
    n = 24
    ctx.build_basis(n, n, 10.0, 10.0, 8, 16, potential=YAM)
    nnz = ctx.build_p(P.WPCD_FP64)
    E = [0.05, 0.6]
    ref = ctx.solve(E, P.WPCD_FP64)
    path = str(tmp_path / "p0.bin")
    ctx.save_p(path)
    c2 = P.Context(0)
    c2.build_basis(n, n, 10.0, 10.0, 8, 16, potential=YAM)
    assert c2.load_p(path) == nnz
    res = c2.solve(E, P.WPCD_FP64)
    for a, b in zip(ref, res):
        assert (a.U_re, a.U_im) == (b.U_re, b.U_im)
    c3 = P.Context(0)
    c3.build_basis(n + 1, n, 10.0, 10.0, 8, 16, potential=YAM)
    with pytest.raises(P.WpcdError) as ei:
        c3.load_p(path)
    assert ei.value.status == P.WPCD_E_INVALID
    # device-resident energies and results
    hip = ctypes.CDLL("libamdhip64.so")
    dE, dR = ctypes.c_void_p(), ctypes.c_void_p()
    nb = ctypes.sizeof(P.wpcd_energy_result) * len(E)
    assert hip.hipMalloc(ctypes.byref(dE), ctypes.c_size_t(8 * len(E))) == 0
    assert hip.hipMalloc(ctypes.byref(dR), ctypes.c_size_t(nb)) == 0
    hE = (ctypes.c_double * len(E))(*E)
    assert hip.hipMemcpy(dE, hE, ctypes.c_size_t(8 * len(E)), 1) == 0
    P.wpcd_solve_dev(c2.h, dE.value, len(E), dR.value, P.WPCD_FP64)
    hR = (P.wpcd_energy_result * len(E))()
    assert hip.hipMemcpy(hR, dR, ctypes.c_size_t(nb), 2) == 0
    for a, b in zip(ref, hR):
        assert (a.U_re, a.U_im, a.status) == (b.U_re, b.U_im, b.status)
    hip.hipFree(dE)
    hip.hipFree(dR)
    c2.close()
    c3.close()


def test_bound_state_parity(ctx, P):
    """E3 of the homogeneous equation (Arnoldi on K(E) on the GPU, largest
    real Ritz value = 1) against the oracle's (ARPACK, bisection) on the
    40 x 40 Yamaguchi grid; a bracket without a sign change is an error."""
    n = 40
    ctx.build_basis(n, n, 10.0, 10.0, 8, 16, potential=YAM)
    ctx.build_p(P.WPCD_FP64)
    eps, _, _ = ctx.pair_spectrum(0, want_O=False)
    say("[E3] GPU bound state")
    e3 = ctx.bound_state(-3.0, eps[0] - 1e-4)
    sysm = _oracle_system_yam(n, 16)
    e3_o = O.bound_state(sysm, -3.0, sysm.eps[0][0] - 1e-4, tol=1e-11)
    say(f"[E3] GPU {e3:.12f} oracle {e3_o:.12f}")
    assert abs(e3 - e3_o) <= 1e-9 * abs(e3_o)
    with pytest.raises(P.WpcdError) as ei:
        ctx.bound_state(-3.0, -2.0)
    assert ei.value.status == P.WPCD_E_INVALID
