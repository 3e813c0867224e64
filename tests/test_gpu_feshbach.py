"""GPU parity of the Feshbach major/minor channel reduction (Sec. V.B)
through the C ABI against the FP64 oracle (oracle.feshbach).

Bars: the reduced structure bit-exact; FP64 values within 1e-12 of the
largest (a different summation order of the same sums); FP64 amplitudes
within 1e-10 relative; the mixed tiers within 1e-6.  At the 300 x 300
three-channel size, sampled reduced rows are rebuilt by the oracle cell
pair by cell pair.
"""
import math
import sys

import numpy as np
import pytest

import oracle.feshbach as F
import oracle.wpcd as O
from inputs import YUK_RANGES

pytestmark = pytest.mark.gpu

L2_CHANS = [(0, 2), (2, 0), (2, 2)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_1508_07441_amd as P
    return P


def _pot(scale):
    return dict(kind="yukawa", strength=[-scale, -scale], range=list(YUK_RANGES))


def _opot(scale):
    return O.Potential("yukawa", (-scale, -scale), YUK_RANGES)


def _pair(P, n_p, n_q, pm, qm, ngq, ngx, scale, prec, chans=L2_CHANS):
    full = P.Context(0)
    full.build_basis(n_p, n_q, pm, qm, ngq, ngx, channels=chans, L=2, potential=_pot(scale))
    full.build_p(prec)
    return full


CASES = [  # n_p, n_q, p_max, q_max, n_gq, n_gx, n_major, r_p, r_q
    (12, 10, 8.0, 8.0, 8, 12, 1, 2, 2),
    (12, 10, 7.0, 9.0, 5, 9, 2, 3, 2),
    (9, 12, 8.0, 8.0, 8, 16, 1, 3, 4),
]


@pytest.mark.parametrize("case", CASES)
def test_reduced_structure_and_values(P, case):
    n_p, n_q, pm, qm, ngq, ngx, nmaj, rp, rq = case
    say(f"[fesh] structure {case}")
    full = _pair(P, n_p, n_q, pm, qm, ngq, ngx, 2.0, P.WPCD_FP64)
    red = P.Context(0)
    try:
        nnz = red.build_reduced(full, nmaj, rp, rq, P.WPCD_FP64)
        ptr, col, val = red.get_p()
        sysm = O.build_system(O.cheb_edges(n_p, pm), O.cheb_edges(n_q, qm), 2, L2_CHANS, ngq, ngx,
                              _opot(2.0))
        ro = F.build_reduced(sysm, nmaj, rp, rq)
        ptr_o, col_o = F.structure(ro)
        assert nnz == int(ptr_o[-1])
        assert np.array_equal(ptr, ptr_o)
        assert np.array_equal(col, col_o)
        vo = F.values_on(ro, ptr_o, col_o)
        scale = np.abs(vo).max()
        assert np.max(np.abs(val - vo)) <= 1e-12 * scale, float(np.max(np.abs(val - vo)) / scale)
        # the same build again: identical bits
        red.build_reduced(full, nmaj, rp, rq, P.WPCD_FP64)
        _, _, val2 = red.get_p()
        assert np.array_equal(val, val2)
        # the pair spectrum of the major waves is the full system's
        e_red, _, _ = red.pair_spectrum(0, want_O=False)
        e_full, _, _ = full.pair_spectrum(0, want_O=False)
        assert np.array_equal(e_red, e_full)
    finally:
        red.close()
        full.close()


def _oracle_red(n_p, n_q, pm, qm, ngq, ngx, scale, nmaj, rp, rq):
    sysm = O.build_system(O.cheb_edges(n_p, pm), O.cheb_edges(n_q, qm), 2, L2_CHANS, ngq, ngx,
                          _opot(scale))
    return F.build_reduced(sysm, nmaj, rp, rq)


@pytest.mark.parametrize("averaged", [False, True])
def test_reduced_amplitudes_fp64_and_breakup(P, averaged):
    n_p, n_q, pm, qm, ngq, ngx, nmaj, rp, rq = 12, 10, 8.0, 8.0, 8, 12, 1, 2, 2
    scale = 2.0
    say(f"[fesh] amplitudes FP64 averaged={averaged}")
    full = _pair(P, n_p, n_q, pm, qm, ngq, ngx, scale, P.WPCD_FP64)
    red = P.Context(0)
    try:
        red.build_reduced(full, nmaj, rp, rq, P.WPCD_FP64)
        ro = _oracle_red(n_p, n_q, pm, qm, ngq, ngx, scale, nmaj, rp, rq)
        e0 = ro.major.eps[0][0]
        energies = [e0 + 0.05, 0.3, 1.1, 2.2]
        mode = P.WPCD_BREAKUP_DIST if averaged else P.WPCD_BREAKUP_ELEMENTS
        res, brs = red.solve(energies, P.WPCD_FP64, want_breakup=mode,
                             resolvent=P.WPCD_RESOLVENT_AVERAGED if averaged else 0)
        for r, br, E in zip(res, brs, energies):
            assert r.status == P.WPCD_OK, (E, P.STATUS_NAMES[r.status])
            u = F.solve_effective(ro, E, averaged)
            a = F.amplitudes(ro, E, u, averaged)
            U = complex(r.U_re, r.U_im)
            assert abs(U - a.U00) <= 1e-10 * abs(a.U00), (E, U, a.U00)
            if averaged:
                want = sorted((c, k, tot) for (c, k, _, tot, _) in a.breakup_dist)
                got = sorted((int(x[0]), int(x[1]), x[3]) for x in br)
                assert [w[:2] for w in want] == [g[:2] for g in got]
                for w, g in zip(want, got):
                    assert abs(w[2] - g[2]) <= 1e-10 * max(1e-3, w[2])
            else:
                want = {(c, k, j): s for (c, k, j, s) in a.breakup}
                got = {(int(x[0]), int(x[1]), int(x[2])): complex(x[3], x[4]) for x in br}
                assert set(want) == set(got), E
                smax = max([abs(v) for v in want.values()] + [1e-30])
                for key, v in want.items():
                    assert abs(got[key] - v) <= 1e-10 * smax, (E, key)
                if E < min(ro.minor.eps[w][0] for w in ro.minor.eps) and E < ro.major.eps[0][1]:
                    assert abs(math.hypot(r.S_re, r.S_im) - 1.0) < 1e-12
            if E > 0:
                # the minor (coarse) channels take part in the breakup
                assert any(int(x[0]) >= nmaj for x in br), E
    finally:
        red.close()
        full.close()


def test_reduced_mixed_tiers(P):
    n_p, n_q, pm, qm, ngq, ngx, nmaj, rp, rq = 12, 10, 8.0, 8.0, 8, 12, 1, 2, 2
    scale = 2.0
    say("[fesh] mixed tiers")
    full = _pair(P, n_p, n_q, pm, qm, ngq, ngx, scale, P.WPCD_MIXED)
    red = P.Context(0)
    try:
        red.build_reduced(full, nmaj, rp, rq, P.WPCD_MIXED)
        ro = _oracle_red(n_p, n_q, pm, qm, ngq, ngx, scale, nmaj, rp, rq)
        energies = [ro.major.eps[0][0] + 0.05, 0.3, 1.1]
        refs = {E: F.amplitudes(ro, E, F.solve_effective(ro, E)).U00 for E in energies}
        for prec in (P.WPCD_MIXED, P.WPCD_MIXED_REFINE, P.WPCD_MIXED_BF16):
            say(f"[fesh] mixed precision {prec}")
            for r, E in zip(red.solve(energies, prec), energies):
                assert r.status == P.WPCD_OK, (prec, E, P.STATUS_NAMES[r.status])
                U = complex(r.U_re, r.U_im)
                assert abs(U - refs[E]) <= 1e-6 * abs(refs[E]), (prec, E, U, refs[E])
        # an FP64 solve needs an FP64 reduction
        with pytest.raises(P.WpcdError):
            red.solve(energies[:1], P.WPCD_FP64)
    finally:
        red.close()
        full.close()


def test_reduced_spmm_variants(P):
    """Every SpMM candidate of the reduced system's scalar CSR (plain,
    XCD-contiguous, LDS-staged, pipelined), forced in turn: the same
    amplitudes to rounding."""
    n_p, n_q, pm, qm, ngq, ngx, nmaj, rp, rq = 12, 10, 8.0, 8.0, 8, 12, 1, 2, 2
    full = _pair(P, n_p, n_q, pm, qm, ngq, ngx, 2.0, P.WPCD_FP64)
    red = P.Context(0)
    try:
        red.build_reduced(full, nmaj, rp, rq, P.WPCD_FP64)
        E = [0.3, 1.1]
        red.set_autotune(P.WPCD_TUNE_FORCE)
        ref = red.solve(E, P.WPCD_FP64)
        for f in range(1, 6):
            say(f"[fesh] spmm force {f}")
            red.set_autotune(P.WPCD_TUNE_FORCE + f)
            for a, b in zip(ref, red.solve(E, P.WPCD_FP64)):
                assert a.status == P.WPCD_OK and b.status == P.WPCD_OK
                Ua, Ub = complex(a.U_re, a.U_im), complex(b.U_re, b.U_im)
                assert abs(Ua - Ub) <= 1e-12 * abs(Ua), (f, Ua, Ub)
    finally:
        red.close()
        full.close()


def test_reduced_sampled_rows_300(P):
    """300 x 300 bins, three L = 2+ channels, the d-wave channels coarsened
    2 x 2: sampled rows of the reduced P0 (fine and coarse) against the
    oracle's cell-pair elements summed with the packet weights."""
    n, ngq, ngx, nmaj, rp, rq = 300, 8, 20, 1, 2, 2
    say("[fesh] 300 x 300 reduced build")
    full = _pair(P, n, n, 10.0, 10.0, ngq, ngx, 1.5, P.WPCD_FP64)
    red = P.Context(0)
    try:
        nnz = red.build_reduced(full, nmaj, rp, rq, P.WPCD_FP64)
        ptr, col, val = red.get_p()
        assert ptr[-1] == nnz and np.all(np.diff(ptr) > 0)
        p = O.cheb_edges(n, 10.0)
        pc, ap, wp = F.coarse_bins(p, rp)
        ncell, nc = n * n, (n // rp) * (n // rq)
        nch = 3
        rng = np.random.default_rng(2024)
        fine_rows = rng.choice(ncell, 3, replace=False)
        coarse_rows = rng.choice(nc, 3, replace=False)
        samples = [(0, int(R)) for R in fine_rows] + [(1 + int(a), int(I)) for a, I in
                                                   zip(rng.integers(0, 2, 3), coarse_rows)]
        for ch, cell in samples:
            if ch < nmaj:
                r = ch * ncell + cell
                src = [(cell, 1.0)]
            else:
                r = nmaj * ncell + (ch - nmaj) * nc + cell
                J, I = divmod(cell, n // rp)
                src = [((J * rq + dj) * n + I * rp + di, wp[J * rq + dj] * wp[I * rp + di])
                       for dj in range(rq) for di in range(rp)]
            rows = np.array([s for s, _ in src], dtype=np.int64)
            rptr, rcol = O.preselect(p, p.copy(), rows)
            want = {}
            for t, (R, w) in enumerate(src):
                cols = rcol[rptr[t]:rptr[t + 1]]
                vals = O.p0_pairs(p, p.copy(), ngq, ngx, 2, L2_CHANS,
                                  np.full(cols.size, R, dtype=np.int64), cols)
                for C, blk in zip(cols.tolist(), vals):
                    jc, ic = divmod(C, n)
                    for b in range(nch):
                        if b < nmaj:
                            key, wc = b * ncell + C, 1.0
                        else:
                            key = nmaj * ncell + (b - nmaj) * nc + (jc // rq) * (n // rp) + ic // rp
                            wc = wp[jc] * wp[ic]
                        want[key] = want.get(key, 0.0) + w * wc * blk[ch, b]
            keys = sorted(want)
            got_c = col[ptr[r]:ptr[r + 1]]
            got_v = val[ptr[r]:ptr[r + 1]]
            assert np.array_equal(got_c, np.array(keys, dtype=np.int32)), (ch, cell)
            wv = np.array([want[k] for k in keys])
            assert np.max(np.abs(got_v - wv)) <= 1e-10 * np.abs(wv).max(), (ch, cell)
            say(f"[fesh] row channel {ch} cell {cell}: {len(keys)} entries ok")
    finally:
        red.close()
        full.close()


def test_reduced_errors(P):
    full = _pair(P, 12, 10, 8.0, 8.0, 8, 12, 2.0, P.WPCD_FP64)
    red = P.Context(0)
    other = P.Context(0)
    try:
        for args in ((0, 2, 2), (3, 2, 2), (1, 5, 2), (1, 2, 3), (1, 12, 1)):
            with pytest.raises(P.WpcdError) as e:
                red.build_reduced(full, *args)
            assert e.value.status == P.WPCD_E_INVALID, args
        with pytest.raises(P.WpcdError) as e:
            red.build_reduced(full, 1, 2, 2, P.WPCD_MIXED_BF16)
        assert e.value.status == P.WPCD_E_INVALID
        # the entrance channel (0, 2) listed second: n_major = 1 leaves it minor
        other.build_basis(12, 10, 8.0, 8.0, 8, 12, channels=[(2, 0), (0, 2), (2, 2)], L=2,
                          potential=_pot(2.0))
        other.build_p(P.WPCD_FP64)
        with pytest.raises(P.WpcdError) as e:
            red.build_reduced(other, 1, 2, 2)
        assert e.value.status == P.WPCD_E_INVALID
        red.build_reduced(full, 1, 2, 2)
        for call in (lambda: red.build_p(P.WPCD_FP64), lambda: red.set_potential(_pot(1.0)),
                     lambda: red.set_multipliers([1.0, 1.0]), lambda: red.bound_state(-1.0, -0.5)):
            with pytest.raises(P.WpcdError) as e:
                call()
            assert e.value.status == P.WPCD_E_STATE
        # a reduced system cannot be reduced again
        with pytest.raises(P.WpcdError) as e:
            other.build_reduced(red, 1, 2, 2)
        assert e.value.status == P.WPCD_E_INVALID
        # full stays usable and may go away: red keeps what it needs
        full.close()
        r = red.solve([0.4], P.WPCD_FP64)[0]
        assert r.status == P.WPCD_OK
        # a new basis makes red an ordinary context again
        red.build_basis(12, 10, 8.0, 8.0, 8, 12, channels=L2_CHANS, L=2, potential=_pot(2.0))
        red.build_p(P.WPCD_FP64)
        assert red.solve([0.4], P.WPCD_FP64)[0].status == P.WPCD_OK
    finally:
        other.close()
        red.close()
        full.close()


def test_reduced_lockstep_error_estimate_and_given_start(P):
    """A reduced system in lockstep with its own full system gives the bits
    of the one-by-one solves; the mixed tier's error estimate against the
    FP64 values of the reduced P0 matches the measured difference; its own
    FP64 solution given as the start vector leaves nothing to iterate."""
    n_p, n_q, pm, qm, ngq, ngx, nmaj, rp, rq = 12, 10, 8.0, 8.0, 8, 12, 1, 2, 2
    full = _pair(P, n_p, n_q, pm, qm, ngq, ngx, 2.0, P.WPCD_MIXED)
    red = P.Context(0)
    red64 = P.Context(0)
    try:
        red.build_reduced(full, nmaj, rp, rq, P.WPCD_MIXED)
        red64.build_reduced(full, nmaj, rp, rq, P.WPCD_FP64)
        Es = [[0.3, 1.1, -0.2], [0.5, 1.7]]
        alone = [red.solve(Es[0], P.WPCD_MIXED), full.solve(Es[1], P.WPCD_MIXED)]
        say("[fesh] lockstep with the full system")
        together = P.wpcd_solve_multi([red.h, full.h], Es, P.WPCD_MIXED)
        for ra, rt in zip(alone, together):
            for a, t in zip(ra, rt):
                assert a.status == t.status == P.WPCD_OK
                assert (a.U_re, a.U_im) == (t.U_re, t.U_im)
        say("[fesh] error estimate")
        est = red.solve(Es[0], P.WPCD_MIXED, err_est=True)
        ref = red64.solve(Es[0], P.WPCD_FP64)
        for a, b in zip(est, ref):
            Ua, Ub = complex(a.U_re, a.U_im), complex(b.U_re, b.U_im)
            d = abs(Ua - Ub) / abs(Ub)
            assert d < 1e-6 and a.err_vs_fp64 < 1e-6
            assert abs(a.err_vs_fp64 - d) <= 0.05 * d + 2e-10, (a.err_vs_fp64, d)
        say("[fesh] given start vector")
        M = red.red_rows
        assert M == nmaj * n_p * n_q + 2 * (n_p // rp) * (n_q // rq)
        # a zero proposal over the reduced layout is judged useless and the
        # solve is the plain one
        first = red64.solve([0.7], P.WPCD_FP64)[0]
        x0 = np.zeros((1, M), dtype=np.complex128)
        r = red64.solve([0.7], P.WPCD_FP64, warm_start=P.WPCD_WARM_GIVEN, x0=x0)[0]
        assert r.status == P.WPCD_OK and r.warm == 0
        # a start vector of the unreduced system's length is refused
        with pytest.raises(ValueError):
            red64.solve([0.7], P.WPCD_FP64, warm_start=P.WPCD_WARM_GIVEN,
                        x0=np.zeros((1, 3 * n_p * n_q), dtype=np.complex128))
        assert (r.U_re, r.U_im) == (first.U_re, first.U_im)
    finally:
        red64.close()
        red.close()
        full.close()


def test_reduced_two_major_channels_uneven_coarsening(P):
    """Two major channels ((0,2) and (2,0) on the 12 x 10 lattice) and one
    minor ((2,2) on bins of 3 x 2 fine bins): FP64 amplitudes and breakup
    elements against the oracle's effective-kernel solution."""
    n_p, n_q, pm, qm, ngq, ngx, nmaj, rp, rq = 12, 10, 7.0, 9.0, 5, 9, 2, 3, 2
    scale = 2.0
    full = _pair(P, n_p, n_q, pm, qm, ngq, ngx, scale, P.WPCD_FP64)
    red = P.Context(0)
    try:
        red.build_reduced(full, nmaj, rp, rq, P.WPCD_FP64)
        assert red.red_rows == 2 * n_p * n_q + (n_p // rp) * (n_q // rq)
        ro = _oracle_red(n_p, n_q, pm, qm, ngq, ngx, scale, nmaj, rp, rq)
        energies = [ro.major.eps[0][0] + 0.05, 0.6, 1.8]
        say("[fesh] two major channels")
        res, brs = red.solve(energies, P.WPCD_FP64, want_breakup=P.WPCD_BREAKUP_ELEMENTS)
        for r, br, E in zip(res, brs, energies):
            assert r.status == P.WPCD_OK, (E, P.STATUS_NAMES[r.status])
            a = F.amplitudes(ro, E, F.solve_effective(ro, E))
            U = complex(r.U_re, r.U_im)
            assert abs(U - a.U00) <= 1e-10 * abs(a.U00), (E, U, a.U00)
            want = {(c, k, j): s for (c, k, j, s) in a.breakup}
            got = {(int(x[0]), int(x[1]), int(x[2])): complex(x[3], x[4]) for x in br}
            assert set(want) == set(got), E
            smax = max([abs(v) for v in want.values()] + [1e-30])
            for key, v in want.items():
                assert abs(got[key] - v) <= 1e-10 * smax, (E, key)
    finally:
        red.close()
        full.close()


def test_reduced_sweep_and_fp64_fallback(P, tmp_path):
    """The journaled sweep and the mixed tier's FP64 fallback on a reduced
    system: an interrupted sweep resumes to the bits of the batch-by-batch
    solves; a fallback bound below the FP32 error gives the amplitudes of
    the reduced system built in FP64."""
    full = _pair(P, 12, 10, 8.0, 8.0, 8, 12, 2.0, P.WPCD_MIXED)
    red = P.Context(0)
    red64 = P.Context(0)
    try:
        red.build_reduced(full, 1, 2, 2, P.WPCD_MIXED)
        red64.build_reduced(full, 1, 2, 2, P.WPCD_FP64)
        E = [0.3, 0.7, 1.1, 1.7, -0.2]
        ref = []
        for k in range(0, len(E), 2):
            ref += red.solve(E[k:k + 2], P.WPCD_MIXED)
        path = str(tmp_path / "red.wj")
        say("[fesh] sweep, interrupted and resumed")
        _, n_done, _ = red.sweep(E, 2, P.WPCD_MIXED, journal=path, max_batches=1)
        assert n_done == 2
        res, n_done, n_res = red.sweep(E, 2, P.WPCD_MIXED, journal=path)
        assert (n_done, n_res) == (len(E), 2)
        for a, b in zip(res, ref):
            assert (a.status, a.iters, a.U_re, a.U_im) == (b.status, b.iters, b.U_re, b.U_im)
        say("[fesh] FP64 fallback")
        fb = red.solve(E, P.WPCD_MIXED, err_est=True, fallback_tol=1e-13)
        r64 = red64.solve(E, P.WPCD_FP64)
        n_ok = 0
        for a, b in zip(fb, r64):
            assert a.status == b.status
            if b.status != P.WPCD_OK:
                continue
            n_ok += 1
            Ua, Ub = complex(a.U_re, a.U_im), complex(b.U_re, b.U_im)
            assert a.fallback == 1 and abs(Ua - Ub) <= 1e-12 * abs(Ub), (Ua, Ub)
        assert n_ok >= 4
    finally:
        red64.close()
        red.close()
        full.close()
