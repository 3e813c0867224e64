"""GPU: the mixed tiers' FP64 fallback (opts.fallback_tol) through the C ABI.

After a mixed solve, the energies that did not converge, or whose estimated
amplitude error (err_vs_fp64) is above the bound, are solved again on the
FP64 P0 values of the same structure.  Checked: a loose bound changes
nothing; a bound below the FP32 error re-solves every energy, and the
results then equal an FP64 build's solve (and the oracle to 1e-10),
breakup rows and a caller-given start included; a solve cut off by the
iteration cap is re-solved; energies with other statuses are left alone;
the FP64 tier ignores the option.
"""
import sys

import numpy as np
import pytest

import oracle.wpcd as O
from inputs import YAM_BETA, YAM_LAMBDA

pytestmark = pytest.mark.gpu

YAM = dict(kind="yamaguchi", strength=[YAM_LAMBDA], range=[YAM_BETA])
N = 40
ENERGIES = (-0.09, -0.05, -0.2, 0.05, 0.5, 1.0, 2.0)   # -0.2: below the threshold
SKIP = 2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_1508_07441_amd as P
    return P


@pytest.fixture(scope="module")
def mixed(P):
    c = P.Context(0)
    c.build_basis(N, N, 10.0, 10.0, 8, 16, potential=YAM)
    c.build_p(P.WPCD_MIXED)
    yield c
    c.close()


@pytest.fixture(scope="module")
def fp64(P):
    c = P.Context(0)
    c.build_basis(N, N, 10.0, 10.0, 8, 16, potential=YAM)
    c.build_p(P.WPCD_FP64)
    yield c
    c.close()


def _U(r):
    return complex(r.U_re, r.U_im)


def test_loose_bound_changes_nothing(mixed, P):
    say("[fallback] mixed, loose bound")
    a = mixed.solve(ENERGIES, P.WPCD_MIXED, err_est=True)
    b = mixed.solve(ENERGIES, P.WPCD_MIXED, err_est=True, fallback_tol=1e-3)
    for x, y in zip(a, b):
        assert y.fallback == 0
        assert (x.status, x.iters, _U(x)) == (y.status, y.iters, _U(y))
    assert b[SKIP].status == P.WPCD_E_BELOW_THRESHOLD
    assert max(r.err_vs_fp64 for k, r in enumerate(b) if k != SKIP) < 1e-5


def test_tight_bound_gives_the_fp64_solve(mixed, fp64, P):
    say("[fallback] mixed, bound below the FP32 error")
    res = mixed.solve(ENERGIES, P.WPCD_MIXED, err_est=True, fallback_tol=1e-13)
    ref = fp64.solve(ENERGIES, P.WPCD_FP64)
    for k, (r, f) in enumerate(zip(res, ref)):
        if k == SKIP:
            assert r.status == P.WPCD_E_BELOW_THRESHOLD and r.fallback == 0
            continue
        assert r.status == P.WPCD_OK and r.fallback == 1, (k, r.status, r.fallback)
        assert abs(_U(r) - _U(f)) <= 1e-12 * abs(_U(f)), (ENERGIES[k], _U(r), _U(f))
        assert r.err_vs_fp64 < 1e-10
    p = O.cheb_edges(N, 10.0)
    sysm = O.build_system(p, p.copy(), 0, [(0, 0)], 8, 16,
                          O.Potential("yamaguchi", (YAM_LAMBDA,), (YAM_BETA,)))
    for k in (0, 5):
        a = O.amplitudes(sysm, ENERGIES[k], O.solve_gmres(sysm, ENERGIES[k])[0])
        assert abs(_U(res[k]) - a.U00) <= 1e-10 * abs(a.U00)
    # the mixed results themselves are unchanged afterwards
    again = mixed.solve(ENERGIES, P.WPCD_MIXED, err_est=True)
    assert all(r.fallback == 0 for r in again)


def test_breakup_rows_and_given_start(mixed, fp64, P):
    E = [0.5, 1.0, 2.0]
    say("[fallback] breakup rows")
    res, br = mixed.solve(E, P.WPCD_MIXED, want_breakup=True, err_est=True, fallback_tol=1e-13)
    ref, brf = fp64.solve(E, P.WPCD_FP64, want_breakup=True)
    for r, f, rows, rows_f in zip(res, ref, br, brf):
        assert r.fallback == 1 and r.n_open == f.n_open and r.n_open > 0
        assert np.array_equal(rows[:, :3], rows_f[:, :3])
        assert np.max(np.abs(rows[:, 3:] - rows_f[:, 3:])) <= 1e-10
    say("[fallback] caller-given start")
    M = mixed.basis_rows()
    rng = np.random.default_rng(5)
    x0 = 1e-3 * (rng.normal(size=(len(E), M)) + 1j * rng.normal(size=(len(E), M)))
    res = mixed.solve(E, P.WPCD_MIXED, warm_start=P.WPCD_WARM_GIVEN, x0=x0, err_est=True,
                      fallback_tol=1e-13)
    for r, f in zip(res, ref):
        assert r.fallback == 1 and r.status == P.WPCD_OK
        assert abs(_U(r) - _U(f)) <= 1e-10 * abs(_U(f))


def test_iteration_cap_triggers_the_fallback(mixed, P):
    say("[fallback] iteration cap")
    res = mixed.solve(ENERGIES, P.WPCD_MIXED, max_iter=2, fallback_tol=1e-6)
    for k, r in enumerate(res):
        if k == SKIP:
            assert r.fallback == 0
            continue
        # the FP64 solve is held to the same cap, so it stops short as well
        assert r.fallback == 1 and r.status == P.WPCD_E_NOT_CONVERGED


def test_fp64_tier_ignores_the_option(fp64, P):
    res = fp64.solve(ENERGIES, P.WPCD_FP64, err_est=True, fallback_tol=1e-30)
    assert all(r.fallback == 0 for r in res)


def test_stagnation_stops_the_solve(mixed, fp64, P):
    """A tolerance below the rounding floor cannot be met: the solve stops
    after two restart cycles that do not halve the true residual, instead of
    spending the whole iteration cap, with the converged amplitudes."""
    E = [0.05, 0.5, 2.0]
    say("[stagnation] FP64, tolerance below the rounding floor")
    ref = fp64.solve(E, P.WPCD_FP64)
    res = fp64.solve(E, P.WPCD_FP64, tol=1e-30, max_iter=4000)
    for r, f in zip(res, ref):
        assert r.status == P.WPCD_E_STAGNATED, P.STATUS_NAMES[r.status]
        assert r.iters < 400 and r.residual < 1e-13, (r.iters, r.residual)
        assert abs(_U(r) - _U(f)) <= 1e-11 * abs(_U(f))
    say("[stagnation] mixed with the FP64 fallback")
    res = mixed.solve(E, P.WPCD_MIXED, tol=1e-30, max_iter=4000, fallback_tol=1e-6)
    for r, f in zip(res, ref):
        assert r.fallback == 1 and r.status == P.WPCD_E_STAGNATED
        assert abs(_U(r) - _U(f)) <= 1e-11 * abs(_U(f))
