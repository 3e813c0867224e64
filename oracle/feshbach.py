"""Feshbach major/minor channel reduction (Sec. V.B) on the CPU, in FP64.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It builds on
``oracle.wpcd`` (the unreduced system) and shares no code with the library.

Sec. V.B proposes, for systems with many channels, to split the channels
into major and minor ones, to carry the minor channels into the kernel of
the major subspace as an effective interaction that holds the resolvent of
the minor subspace, and to describe the minor channels with a much smaller
basis than the major ones.  Readings taken here (the paper gives no
formulas):

* Reduced minor basis.  The minor channels keep the free wave-packet
  construction on a coarser lattice whose cells are unions of r_p x r_q
  fine cells: every r_p-th p edge and every r_q-th q edge.  With unit-weight
  packets (B_i = d_i) the packet of a union of bins is
  sum_i sqrt(d_i / D) |x_i>, D = sum_i d_i, so every element of P0 that
  involves a coarse cell is the same combination of fine elements (the
  element is an integral over the two cells, eqs.(perm),(gal)): the reduced
  lattice matrix is R P0 R^T with R the identity on the major channels and
  these weights on the minor ones.
* The minor channels' pair Hamiltonian is diagonalised on the coarse p bins
  (eq.(exp_z), the same potential); their channel resolvent uses the coarse
  spectator bins (Sec. II.D).
* The solution in the major subspace is that of the effective-kernel
  equation
      (1 - K_MM - K_Mm (1 - K_mm)^-1 K_mM) U_M = b_M + K_Mm (1 - K_mm)^-1 b_m,
  with K and b the reduced system's kernel and driving term partitioned
  into major (M) and minor (m) rows and columns; the minor components are
  U_m = (1 - K_mm)^-1 (b_m + K_mM U_M).

Layout of the reduced channel basis: the major channels on the fine
lattice, (a*Nq + j)*Np + k as in the unreduced system, then the minor
channels on the coarse lattice from row M_F = n_major*Nq*Np on, with the
same ordering over (minor channel, coarse j, coarse k).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import wpcd as W


def coarse_bins(edges, r: int):
    """Edges of the coarse lattice (every r-th edge), the coarse bin of each
    fine bin, and the packet weights sqrt(d_i / D) of the fine bins."""
    edges = np.asarray(edges, dtype=float)
    n = edges.size - 1
    if r < 1 or n % r:
        raise ValueError("the coarsening factor must divide the bin count")
    ce = edges[::r].copy()
    agg = np.arange(n) // r
    d, D = np.diff(edges), np.diff(ce)
    return ce, agg, np.sqrt(d / D[agg])


@dataclass
class Reduced:
    full: W.System      # the unreduced system (fine lattice, every channel)
    n_major: int
    rp: int
    rq: int
    major: W.System     # fine lattice, the major channels (pair waves only)
    minor: W.System     # coarse lattice, the minor channels (pair waves only)
    R: sp.csr_matrix    # reduced lattice cells x unreduced lattice cells
    P0: sp.csr_matrix   # R P0 R^T over the reduced lattice cells

    @property
    def M_F(self):
        return self.major.M

    @property
    def M_C(self):
        return self.minor.M

    @property
    def M(self):
        return self.M_F + self.M_C


def restriction(full: W.System, n_major: int, rp: int, rq: int):
    """R over the lattice-cell index (channel, j, i): identity rows for the
    major channels, weights sqrt(d_i dq_j / (D_I DQ_J)) from each fine cell
    (j, i) into its coarse cell (j / r_q, i / r_p) for the minor ones."""
    _, ap, wp = coarse_bins(full.p, rp)
    _, aq, wq = coarse_bins(full.q, rq)
    Np, Nq = full.Np, full.Nq
    Npc, Nqc = Np // rp, Nq // rq
    ncell, nccell = Np * Nq, Npc * Nqc
    nch = len(full.chans)
    jj, ii = np.divmod(np.arange(ncell), Np)
    coarse = aq[jj] * Npc + ap[ii]
    w = wq[jj] * wp[ii]
    rows, cols, vals = [], [], []
    for a in range(nch):
        src = a * ncell + np.arange(ncell)
        if a < n_major:
            rows.append(src)
            vals.append(np.ones(ncell))
        else:
            rows.append(n_major * ncell + (a - n_major) * nccell + coarse)
            vals.append(w)
        cols.append(src)
    shape = (n_major * ncell + (nch - n_major) * nccell, nch * ncell)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=shape)


def build_reduced(full: W.System, n_major: int, rp: int, rq: int) -> Reduced:
    """The reduced system of `full` with channels [0, n_major) major and the
    rest minor on the lattice coarsened by (rp, rq)."""
    nch = len(full.chans)
    if not 1 <= n_major < nch:
        raise ValueError("need at least one major and one minor channel")
    pc, _, _ = coarse_bins(full.p, rp)
    qc, _, _ = coarse_bins(full.q, rq)
    major = W.build_system(full.p, full.q, full.L, full.chans[:n_major], full.n_gq, full.n_gx,
                           full.pot, with_p0=False)
    minor = W.build_system(pc, qc, full.L, full.chans[n_major:], full.n_gq, full.n_gx,
                           full.pot, with_p0=False)
    R = restriction(full, n_major, rp, rq)
    P0 = (R @ full.P0_matrix() @ R.T).tocsr()
    P0.sort_indices()
    return Reduced(full, n_major, rp, rq, major, minor, R, P0)


def structure(red: Reduced):
    """(row_ptr, col) of the reduced P0: every cell pair that some pair of
    its fine cells holds (the union of the patterns, whatever the values)."""
    pat = red.full.P0_matrix().copy()
    pat.data = np.ones_like(pat.data)
    Rp = red.R.copy()
    Rp.data = np.ones_like(Rp.data)
    S = (Rp @ pat @ Rp.T).tocsr()
    S.sort_indices()
    return S.indptr.astype(np.int64), S.indices.astype(np.int32)


def values_on(red: Reduced, ptr, col):
    """Reduced P0 values at the entries of the structure (ptr, col), zero
    where R P0 R^T holds none."""
    rows = np.repeat(np.arange(ptr.size - 1), np.diff(ptr))
    return np.asarray(red.P0[rows, col.astype(np.int64)]).ravel()


# ------------------------------------------------------------ the kernel
def _energy_bin(red: Reduced, E: float):
    return W.energy_bin(red.major, E)


def _resolvent_part(sysm: W.System, E: float, ebin):
    G = np.zeros((len(sysm.chans), sysm.Nq, sysm.Np), dtype=complex)
    qmax = sysm.q[-1]
    for a in range(len(sysm.chans)):
        eps = sysm.eps[sysm.wkey(a)]
        for j in range(sysm.Nq):
            for k in range(sysm.Np):
                if ebin is None:
                    G[a, j, k] = W.resolvent_bin(E, eps[k], sysm.q[j], sysm.q[j + 1], qmax)
                else:
                    G[a, j, k] = W.resolvent_bin_avg(ebin[0], ebin[1], eps[k], sysm.q[j],
                                                     sysm.q[j + 1])
    return G.ravel()


def resolvent(red: Reduced, E: float, averaged: bool = False):
    """Diagonal of G1 over the reduced basis: fine spectator bins for the
    major channels, coarse ones for the minor channels; averaged over the
    entrance's on-shell energy bin when asked."""
    ebin = _energy_bin(red, E) if averaged else None
    return np.concatenate([_resolvent_part(red.major, E, ebin),
                           _resolvent_part(red.minor, E, ebin)])


def apply_A(red: Reduced, y):
    """A y = O P0 V~ y over the reduced basis (eq.(kernel)), each part with
    its own pair waves."""
    F = red.M_F
    nM, nm = red.n_major, len(red.minor.chans)
    yF = y[:F].reshape(nM, red.major.Nq, red.major.Np)
    yC = y[F:].reshape(nm, red.minor.Nq, red.minor.Np)
    vtF = {w: red.major.v[w] @ red.major.O[w].T for w in red.major.v}
    vtC = {w: red.minor.v[w] @ red.minor.O[w].T for w in red.minor.v}
    t = np.concatenate([W._blockwise(red.major, yF, vtF).ravel(),
                        W._blockwise(red.minor, yC, vtC).ravel()])
    t = red.P0 @ t
    return np.concatenate([W._blockwise(red.major, t[:F].reshape(yF.shape), red.major.O).ravel(),
                           W._blockwise(red.minor, t[F:].reshape(yC.shape), red.minor.O).ravel()])


def entrance(red: Reduced, E: float):
    """The incident state lies in the major subspace (fine lattice)."""
    return W.entrance(red.major, E)


def solve_effective(red: Reduced, E: float, averaged: bool = False):
    """Dense solve through the effective kernel of the major subspace (see
    the module docstring); returns the whole reduced solution [U_M, U_m]."""
    a0, j0, q0, idx = entrance(red, E)
    G = resolvent(red, E, averaged)
    M, F = red.M, red.M_F
    A = np.empty((M, M))
    e = np.zeros(M)
    for c in range(M):
        e[:] = 0.0
        e[c] = 1.0
        A[:, c] = apply_A(red, e).real
    K = A * G[None, :]
    b = A[:, idx].astype(complex)
    KMM, KMm, KmM, Kmm = K[:F, :F], K[:F, F:], K[F:, :F], K[F:, F:]
    one_m = np.eye(M - F) - Kmm
    Y = np.linalg.solve(one_m, np.column_stack([KmM, b[F:]]))
    Keff = KMM + KMm @ Y[:, :F]
    beff = b[:F] + KMm @ Y[:, F]
    uM = np.linalg.solve(np.eye(F) - Keff, beff)
    um = np.linalg.solve(one_m, b[F:] + KmM @ uM)
    return np.concatenate([uM, um])


def amplitudes(red: Reduced, E: float, u, averaged: bool = False):
    """Elastic amplitude and breakup elements of the reduced solution, as
    in ``oracle.wpcd.amplitudes``: the major channels' states on the fine
    lattice, the minor channels' pseudostates and spectator bins on the
    coarse one (channel numbers over the whole channel list)."""
    F = red.M_F
    a = W.amplitudes(red.major, E, u[:F], averaged)
    _, j0, q0, _ = entrance(red, E)
    dq0 = red.major.q[j0 + 1] - red.major.q[j0]
    if averaged:
        E1, E2 = _energy_bin(red, E)
        D = E2 - E1
        rho0 = 1.0 / D
    else:
        rho0 = 2.0 / (3.0 * q0 * dq0)
    mn = red.minor
    dq = mn.q[1:] - mn.q[:-1]
    br, dist = list(a.breakup), list(a.breakup_dist)
    for am in range(len(mn.chans)):
        for k, ek in enumerate(mn.eps[mn.wkey(am)]):
            states = []
            if averaged:
                for j in range(mn.Nq):
                    ov = W.shell_overlap(E1 - ek, E2 - ek, mn.q[j], mn.q[j + 1])
                    if ov > 0.0:
                        states.append((j, ov / (D * dq[j])))
            elif ek < E:
                qk = math.sqrt(4.0 * (E - ek) / 3.0)
                jk = int(np.searchsorted(mn.q, qk) - 1)
                if 0 <= jk < mn.Nq:
                    states.append((jk, 2.0 / (3.0 * qk * dq[jk])))
            if not states:
                continue
            tot = 0.0
            for j, rk in states:
                Sk = -2j * math.pi * math.sqrt(rk * rho0) * u[F + (am * mn.Nq + j) * mn.Np + k]
                br.append((red.n_major + am, k, j, Sk))
                tot += abs(Sk) ** 2
            dist.append((red.n_major + am, k, float(ek), tot, len(states)))
    a.breakup, a.breakup_dist = br, dist
    return a
