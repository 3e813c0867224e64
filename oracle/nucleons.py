"""Three nucleons in s-wave pair channels (the oracle side).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module; it shares no code
with the HIP library.

The permutation kernel of eq.(gal) carries algebraic coefficients that
couple the spin-angular channels (Sec. III.B; Sec. V.A for the nucleon
case).  With pair s-waves (l = lam = 0) only its spin-isospin part is left:
channel a = (pair spin s_a, pair isospin t_a), s_a + t_a odd (the pair is
antisymmetric), three-body spin S and isospin T = 1/2.  Both cyclic
permutations of the three particles give the same s-wave space kernel,
half of the boson one, so the nucleon P0 is the boson (s-wave) P0 times

    g_ab = 1/2 (<a| C_sigma C_tau |b> + <a| C_sigma^2 C_tau^2 |b>),

C the cyclic permutation 1 -> 2 -> 3 -> 1 acting on spins and isospins.
Here g is computed by brute force: the coupled three-particle states
|(s_23, 1/2_1) S M> are built as vectors over the 8 product states from
Clebsch-Gordan coefficients (Racah's closed form) and C as an explicit
8 x 8 permutation matrix.  Each channel has its own pair potential (the
common one with per-term strength multipliers), hence its own pair wave.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import wpcd as W


def clebsch(j1, m1, j2, m2, J, M) -> float:
    """<j1 m1 j2 m2 | J M> by Racah's closed form (half-integers as floats)."""
    if abs(m1 + m2 - M) > 1e-9 or J < abs(j1 - j2) - 1e-9 or J > j1 + j2 + 1e-9:
        return 0.0
    if abs(m1) > j1 + 1e-9 or abs(m2) > j2 + 1e-9 or abs(M) > J + 1e-9:
        return 0.0

    def f(x):
        return math.factorial(int(round(x)))

    pre = math.sqrt((2 * J + 1) * f(J + j1 - j2) * f(J - j1 + j2) * f(j1 + j2 - J)
                    / f(j1 + j2 + J + 1))
    pre *= math.sqrt(f(J + M) * f(J - M) * f(j1 - m1) * f(j1 + m1) * f(j2 - m2) * f(j2 + m2))
    tot = 0.0
    for k in range(0, int(round(j1 + j2 + J)) + 2):
        d = [k, j1 + j2 - J - k, j1 - m1 - k, j2 + m2 - k, J - j2 + m1 + k, J - j1 - m2 + k]
        if min(d) < -1e-9:
            continue
        tot += (-1) ** k / np.prod([f(x) for x in d])
    return pre * tot


_HALF = (0.5, -0.5)


def coupled_state(s: int, S: float, MS: float) -> np.ndarray:
    """|(s_23, 1/2_1) S MS> over the product states |m1 m2 m3> (index
    m = +1/2 -> 0, -1/2 -> 1; particle 1 slowest)."""
    out = np.zeros((2, 2, 2))
    for ms in range(-s, s + 1):
        for i1, m1 in enumerate(_HALF):
            c1 = clebsch(s, ms, 0.5, m1, S, MS)
            if c1 == 0.0:
                continue
            for i2, m2 in enumerate(_HALF):
                for i3, m3 in enumerate(_HALF):
                    out[i1, i2, i3] += c1 * clebsch(0.5, m2, 0.5, m3, s, ms)
    return out.ravel()


def cyclic() -> np.ndarray:
    """8 x 8 matrix of the cyclic permutation taking particle i's state to
    particle (i + 1) mod 3."""
    P = np.zeros((8, 8))
    for idx in itertools.product(range(2), repeat=3):
        dst = [0, 0, 0]
        for i in range(3):
            dst[(i + 1) % 3] = idx[i]
        P[np.ravel_multi_index(dst, (2, 2, 2)), np.ravel_multi_index(idx, (2, 2, 2))] = 1.0
    return P


def recoupling(two_S: int, chans, two_T: int = 1, two_MS=None, two_MT=None) -> np.ndarray:
    """g_ab for channels chans = [(s, t), ...] (see the module docstring)."""
    S, T = two_S / 2.0, two_T / 2.0
    MS = S if two_MS is None else two_MS / 2.0
    MT = T if two_MT is None else two_MT / 2.0
    C = cyclic()
    C2 = C @ C
    CC, CC2 = np.kron(C, C), np.kron(C2, C2)
    vec = [np.kron(coupled_state(s, S, MS), coupled_state(t, T, MT)) for s, t in chans]
    n = len(chans)
    g = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            g[a, b] = 0.5 * (vec[a] @ CC @ vec[b] + vec[a] @ CC2 @ vec[b])
    return g


def build_system_nucleons(p, q, two_S: int, chans, n_gq: int, n_gx: int, pot: W.Potential,
                          mult=None) -> W.System:
    """Nucleon system on the grid (p, q): channels chans = [(s, t), ...],
    the first (s, t) = (1, 0) (the deuteron channel, the entrance channel);
    channel a's pair potential is pot with its term strengths times
    mult[a] (default 1)."""
    chans = [tuple(c) for c in chans]
    assert chans[0] == (1, 0), "channel 0 must be the deuteron channel (s, t) = (1, 0)"
    for s, t in chans:
        assert (s + t) % 2 == 1 and s in (0, 1) and t in (0, 1), "s-wave pairs need s + t odd"
        assert two_S in (1, 3) and (two_S == 1 or s == 1), "S = 3/2 needs s = 1"
    n = len(chans)
    mult = [[1.0] * len(pot.strengths)] * n if mult is None else mult
    sysm = W.System(p=p, q=q, L=0, chans=[(0, 0)] * n, n_gq=n_gq, n_gx=n_gx, pot=pot)
    sysm.wave = list(range(n))
    for a in range(n):
        pa = W.Potential(pot.kind, tuple(s * m for s, m in zip(pot.strengths, mult[a])),
                         pot.ranges)
        v = pa.matrix(p, 0)
        e, O = W.pair_diag(p, v)
        sysm.eps[a], sysm.O[a], sysm.v[a] = e, O, v
    sysm.row_ptr, sysm.col = W.preselect(p, q)
    rows = np.repeat(np.arange(sysm.Np * sysm.Nq, dtype=np.int64), np.diff(sysm.row_ptr))
    v0 = W.p0_pairs(p, q, n_gq, n_gx, 0, [(0, 0)], rows, sysm.col)[:, 0, 0]
    g = recoupling(two_S, chans)
    sysm.val = v0[:, None, None] * g[None, :, :]
    sysm.g = g
    return sysm
