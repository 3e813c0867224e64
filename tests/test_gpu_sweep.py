"""GPU: the journaled energy sweep (wpcd_sweep) through the C ABI.

P0 is energy independent (Sec. III.B), so a sweep builds it once and solves
batches of energies; the journal lets an interrupted sweep resume from its
last completed batch.  Checked: the sweep equals wpcd_solve over the same
batches bit for bit and the oracle to 1e-10; an interrupted sweep resumes
where it stopped and ends with the uninterrupted results; a torn or damaged
tail of the journal is dropped and solved again; a journal of another sweep,
or a file that is not a journal, is refused.
"""
import os
import sys

import numpy as np
import pytest

import oracle.wpcd as O
from inputs import YAM_BETA, YAM_LAMBDA

pytestmark = pytest.mark.gpu

YAM = dict(kind="yamaguchi", strength=[YAM_LAMBDA], range=[YAM_BETA])
N = 40
BATCH = 3
FIELDS = ("E", "q0", "j0", "status", "iters", "n_open", "U_re", "U_im", "A_re", "A_im", "S_re",
          "S_im", "delta", "eta", "residual", "warm", "r0")
REC = 16 + 128 * BATCH   # bytes of one full batch record in the journal


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
    c.build_basis(N, N, 10.0, 10.0, 8, 16, potential=YAM)
    c.build_p(P.WPCD_FP64)
    yield c
    c.close()


@pytest.fixture(scope="module")
def energies(ctx):
    eps = ctx.pair_spectrum(0, want_O=False)[0]
    E = list(np.linspace(-0.09, 2.0, 10))
    E.insert(4, float(eps[0]) - 0.01)   # below the two-body threshold: a status, journaled too
    return np.array(E)


def _same(a, b):
    for f in FIELDS:
        x, y = getattr(a, f), getattr(b, f)
        assert x == y or (x != x and y != y), (f, x, y)


def _reference(ctx, P, E):
    out = []
    for k in range(0, E.size, BATCH):
        out += ctx.solve(E[k:k + BATCH], P.WPCD_FP64)
    return out


def test_sweep_equals_batched_solve_and_oracle(ctx, P, energies):
    say(f"[sweep] {energies.size} energies, batch {BATCH}, no journal")
    res, n_done, n_res = ctx.sweep(energies, BATCH, P.WPCD_FP64)
    assert (n_done, n_res) == (energies.size, 0)
    ref = _reference(ctx, P, energies)
    for a, b in zip(res, ref):
        _same(a, b)
    assert res[4].status == P.WPCD_E_BELOW_THRESHOLD
    p = O.cheb_edges(N, 10.0)
    sysm = O.build_system(p, p.copy(), 0, [(0, 0)], 8, 16,
                          O.Potential("yamaguchi", (YAM_LAMBDA,), (YAM_BETA,)))
    for k in (0, 7, 10):
        E = float(energies[k])
        assert res[k].status == P.WPCD_OK
        a = O.amplitudes(sysm, E, O.solve_gmres(sysm, E)[0])
        U = complex(res[k].U_re, res[k].U_im)
        assert abs(U - a.U00) <= 1e-10 * abs(a.U00), (E, U, a.U00)


def test_sweep_resumes_after_interruption(ctx, P, energies, tmp_path):
    path = str(tmp_path / "sweep.wj")
    ref = _reference(ctx, P, energies)
    say("[sweep] journal: first two batches")
    res, n_done, n_res = ctx.sweep(energies, BATCH, P.WPCD_FP64, journal=path, max_batches=2)
    assert (n_done, n_res) == (2 * BATCH, 0)
    for a, b in zip(res[:n_done], ref):
        _same(a, b)
    for r, E in zip(res[n_done:], energies[n_done:]):
        assert r.status == P.WPCD_E_STATE and r.E == E
    size2 = os.path.getsize(path)
    assert size2 == 32 + 8 * energies.size + 2 * REC
    say("[sweep] journal: resume")
    res, n_done, n_res = ctx.sweep(energies, BATCH, P.WPCD_FP64, journal=path)
    assert (n_done, n_res) == (energies.size, 2 * BATCH)
    for a, b in zip(res, ref):
        _same(a, b)
    full = os.path.getsize(path)
    say("[sweep] journal: complete, nothing left to solve")
    res, n_done, n_res = ctx.sweep(energies, BATCH, P.WPCD_FP64, journal=path)
    assert (n_done, n_res) == (energies.size, energies.size)
    for a, b in zip(res, ref):
        _same(a, b)
    assert os.path.getsize(path) == full


def test_sweep_torn_and_damaged_journal(ctx, P, energies, tmp_path):
    path = str(tmp_path / "sweep.wj")
    ref = _reference(ctx, P, energies)
    ctx.sweep(energies, BATCH, P.WPCD_FP64, journal=path)
    full = os.path.getsize(path)
    say("[sweep] torn last record")
    with open(path, "r+b") as f:
        f.truncate(full - 50)
    res, n_done, n_res = ctx.sweep(energies, BATCH, P.WPCD_FP64, journal=path)
    nb = -(-energies.size // BATCH)
    assert (n_done, n_res) == (energies.size, (nb - 1) * BATCH)
    for a, b in zip(res, ref):
        _same(a, b)
    assert os.path.getsize(path) == full
    say("[sweep] damaged second record")
    head = 32 + 8 * energies.size
    with open(path, "r+b") as f:
        f.seek(head + REC + 16 + 48)   # inside the results of batch 1
        b = f.read(1)
        f.seek(-1, os.SEEK_CUR)
        f.write(bytes([b[0] ^ 0x40]))
    res, n_done, n_res = ctx.sweep(energies, BATCH, P.WPCD_FP64, journal=path)
    assert (n_done, n_res) == (energies.size, BATCH)
    for a, b in zip(res, ref):
        _same(a, b)
    assert os.path.getsize(path) == full


def test_sweep_refuses_other_journals(ctx, P, energies, tmp_path):
    path = str(tmp_path / "sweep.wj")
    ctx.sweep(energies, BATCH, P.WPCD_FP64, journal=path, max_batches=1)
    other = energies.copy()
    other[-1] += 1e-12
    for kw in (dict(energies=other, batch=BATCH, precision=P.WPCD_FP64),
               dict(energies=energies, batch=BATCH + 1, precision=P.WPCD_FP64),
               dict(energies=energies, batch=BATCH, precision=P.WPCD_FP64, tol=1e-8)):
        with pytest.raises(P.WpcdError) as e:
            ctx.sweep(journal=path, **kw)
        assert e.value.status == P.WPCD_E_INVALID
    say("[sweep] potential changed")
    ctx.set_multipliers([1.01])
    try:
        with pytest.raises(P.WpcdError) as e:
            ctx.sweep(energies, BATCH, P.WPCD_FP64, journal=path)
        assert e.value.status == P.WPCD_E_INVALID
    finally:
        ctx.set_multipliers([1.0])
    junk = str(tmp_path / "junk.bin")
    with open(junk, "wb") as f:
        f.write(os.urandom(256))
    with pytest.raises(P.WpcdError) as e:
        ctx.sweep(energies, BATCH, P.WPCD_FP64, journal=junk)
    assert e.value.status == P.WPCD_E_INVALID
    # a file that cannot be opened for reading and writing, and a folder,
    # are refused and left as they are
    locked = tmp_path / "locked.wj"
    locked.write_bytes(b"x" * 64)
    os.chmod(locked, 0o200)
    try:
        for j in (str(locked), str(tmp_path)):
            with pytest.raises(P.WpcdError) as e:
                ctx.sweep(energies, BATCH, P.WPCD_FP64, journal=j)
            assert e.value.status == P.WPCD_E_INVALID
    finally:
        os.chmod(locked, 0o600)
    assert locked.read_bytes() == b"x" * 64
    with pytest.raises(P.WpcdError) as e:
        ctx.sweep(energies, 0, P.WPCD_FP64)
    assert e.value.status == P.WPCD_E_INVALID
    with pytest.raises(P.WpcdError) as e:
        ctx.sweep(energies, BATCH, P.WPCD_FP64, warm_start=P.WPCD_WARM_GIVEN)
    assert e.value.status == P.WPCD_E_INVALID
    # the journal is still good after the refusals
    res, n_done, n_res = ctx.sweep(energies, BATCH, P.WPCD_FP64, journal=path)
    assert (n_done, n_res) == (energies.size, BATCH)
    assert ctx.sweep([], BATCH, P.WPCD_FP64)[1:] == (0, 0)
