"""Host sanitizer run of the oracle's C part (CPU only).

``oracle/sanitize_check.c`` and ``oracle/wpcd_oracle.c`` are compiled with
AddressSanitizer and UndefinedBehaviorSanitizer (every report fatal) and
run over a 6 x 5 Chebyshev lattice: every Gauss-Legendre order, the
pre-selection of all rows, the angular coupling and the P0 blocks of the
s-wave and of the three-channel L = 2 set.  The run must end cleanly, and
its printed results must equal those of the library the tests load
(``liborc.so``, built without sanitizers).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle.wpcd as W

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")
L2_CHANS = [(0, 2), (2, 0), (2, 2)]


@pytest.fixture(scope="module")
def run(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("san") / "sanitize_check")
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall",
           "-Wno-unknown-pragmas", "-o", exe, os.path.join(ORACLE, "sanitize_check.c"),
           os.path.join(ORACLE, "wpcd_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "ERROR: AddressSanitizer" not in res.stderr
    recs = {}
    for line in res.stdout.splitlines():
        f = line.split()
        recs.setdefault(f[0], []).append(f[1:])
    return recs


def test_sanitized_run_gauss_legendre(run):
    assert len(run["gl"]) == 256
    for n, sx, sw in run["gl"]:
        x, w = W.gauss_legendre(int(n))
        ax = aw = 0.0
        for xv, wv in zip(x.tolist(), w.tolist()):   # the program's summation order
            ax += abs(xv)
            aw += wv
        assert float(sx) == ax and float(sw) == aw


def test_sanitized_run_preselection(run):
    p, q = W.cheb_edges(6, 6.0), W.cheb_edges(5, 6.0)
    assert [float(e[1]) for e in run["edges"]] == p.tolist()
    ptr, col = W.preselect(p, q)
    assert len(run["row"]) == 30
    for r, rec in enumerate(run["row"]):
        assert int(rec[0]) == r and int(rec[1]) == ptr[r + 1] - ptr[r]
        assert [int(c) for c in rec[2:]] == col[ptr[r]:ptr[r + 1]].tolist()


def test_sanitized_run_coupling(run):
    nodes = [(0.7, 1.3, -0.4), (2.0, 0.5, 0.9), (1.1, 1.1, 1.0)]
    G = [float(r[3]) for r in run["G"]]
    T = [float(r[0]) for r in run["T"]]
    k = 0
    for qv, q2, x in nodes:
        tab = W.geom_G_table(2, L2_CHANS, qv, q2, x).ravel()
        for a in range(3):
            for b in range(3):
                assert G[k] == W.geom_G(2, L2_CHANS[a], L2_CHANS[b], qv, q2, x)
                assert T[k] == tab[3 * a + b]
                k += 1


def test_sanitized_run_p0_blocks(run):
    p, q = W.cheb_edges(6, 6.0), W.cheb_edges(5, 6.0)
    ptr, col = W.preselect(p, q)
    rows = np.repeat(np.arange(30), np.diff(ptr))
    vs = W.p0_pairs(p, q, 4, 8, 0, [(0, 0)], rows, col).ravel()
    vm = W.p0_pairs(p, q, 4, 8, 2, L2_CHANS, rows, col).reshape(-1)
    s = np.array([float(r[1]) for r in run["s"]])
    m = np.array([float(r[2]) for r in run["m"]])
    assert s.size == col.size and m.size == 9 * col.size
    # a different optimisation level may round differently in the last bits
    assert np.max(np.abs(s - vs)) <= 1e-14 * np.max(np.abs(vs))
    assert np.max(np.abs(m - vm)) <= 1e-14 * np.max(np.abs(vm))
