"""Textbook reference for three identical spinless bosons with a rank-1
separable s-wave pair interaction v = lam |g><g|, g(p) = 1/(p^2 + beta^2).

Test infrastructure, independent of both the oracle and the HIP library.
With the pair t-matrix t(z) = |g> tau(z) <g|, the AGS equation for the
elastic amplitude reduces to a one-dimensional integral equation in the
spectator momentum (the classic Amado-Lovelace form):

    X(q) = Z(q, q0) + int_0^Q q'^2 dq' Z(q, q') tau(E - 3/4 q'^2) X(q'),
    Z(q, q') = int_{-1}^{1} dx g(pi1) g(pi2) / (E - q^2 - q'^2 - q q' x),
    1/tau(z) = 1/lam - int_0^Pmax p^2 g(p)^2 / (z - p^2) dp,

with hbar = m = 1 and the same momentum cutoffs as the wave-packet grid.
The on-shell amplitude is n_b^2 X(q0) with n_b^2 the residue of tau at the
pair binding energy; S = 1 - 2 pi i (2 q0 / 3) n_b^2 X(q0).  The bound
state is the energy at which the homogeneous kernel has eigenvalue 1.
Solved by Nystrom on Gauss-Legendre grids, with the pole at q0 subtracted
(Haftel-Tabakin).
"""
import math

import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy.optimize import brentq


class Separable:
    def __init__(self, lam, beta, pmax, qmax, n_p=400, n_x=64):
        self.lam, self.beta, self.pmax, self.qmax = lam, beta, pmax, qmax
        # pair integrals on [0, pmax], nodes clustered at small p
        t, w = leggauss(n_p)
        u = 0.5 * (t + 1.0)
        self.pp = pmax * u ** 2
        self.pw = pmax * 2.0 * u * 0.5 * w
        self.xx, self.xw = leggauss(n_x)
        self.eb = brentq(lambda z: self.tau_inv(z), -50.0, -1e-9, xtol=1e-15, rtol=1e-15)
        g2 = self.g(self.pp) ** 2
        self.nb2 = 1.0 / np.sum(self.pw * self.pp ** 2 * g2 / (self.pp ** 2 - self.eb) ** 2)

    def g(self, p):
        return 1.0 / (p * p + self.beta ** 2)

    def tau_inv(self, z):
        """1/tau(z) for real z < 0."""
        g2 = self.g(self.pp) ** 2
        return 1.0 / self.lam + np.sum(self.pw * self.pp ** 2 * g2 / (self.pp ** 2 - z))

    def Z(self, E, q, qp):
        q = np.asarray(q)[:, None, None]
        qp = np.asarray(qp)[None, :, None]
        x = self.xx[None, None, :]
        pi1 = np.sqrt(qp ** 2 + q ** 2 / 4 + q * qp * x)
        pi2 = np.sqrt(q ** 2 + qp ** 2 / 4 + q * qp * x)
        f = self.g(pi1) * self.g(pi2) / (E - q ** 2 - qp ** 2 - q * qp * x)
        return np.sum(f * self.xw, axis=-1)

    def _grid(self, n, a, b):
        t, w = leggauss(n)
        return 0.5 * (b - a) * t + 0.5 * (b + a), 0.5 * (b - a) * w

    def top_eig(self, E, n=96):
        """Largest real eigenvalue of the homogeneous kernel at E < eb."""
        q1, w1 = self._grid(n // 2, 0.0, 1.0)
        q2, w2 = self._grid(n // 2, 1.0, self.qmax)
        q = np.concatenate([q1, q2]); w = np.concatenate([w1, w2])
        tau = np.array([1.0 / self.tau_inv(E - 0.75 * qq * qq) for qq in q])
        K = self.Z(E, q, q) * (w * q * q * tau)[None, :]
        return float(np.max(np.linalg.eigvals(K).real))

    def bound_state(self, e_lo, e_hi=None):
        e_hi = self.eb - 1e-6 if e_hi is None else e_hi
        return brentq(lambda e: self.top_eig(e) - 1.0, e_lo, e_hi, xtol=1e-13)

    def elastic(self, E, n=96):
        """S-matrix below breakup (eb < E < 0)."""
        assert self.eb < E < 0
        q0 = math.sqrt(4.0 * (E - self.eb) / 3.0)
        qa, wa = self._grid(n // 2, 0.0, q0)
        qb, wb = self._grid(n // 2, q0, self.qmax)
        q = np.concatenate([qa, qb]); w = np.concatenate([wa, wb])
        # tau(E - 3/4 q^2) = (4/3) nb2 that(q) / (q0^2 - q^2), that(q0) = 1
        z = E - 0.75 * q * q
        tau = np.array([1.0 / self.tau_inv(zz) for zz in z])
        that = tau * 0.75 * (q0 ** 2 - q ** 2) / self.nb2
        Q = self.qmax
        c0 = -np.sum(w / (q0 ** 2 - q ** 2)) + (math.log((Q + q0) / (Q - q0)) - 1j * math.pi) / (2 * q0)
        qq = np.concatenate([q, [q0]])
        Zm = self.Z(E, qq, qq)
        n1 = q.size
        kern = np.zeros((n1 + 1, n1 + 1), dtype=complex)
        kern[:, :n1] = Zm[:, :n1] * ((4.0 / 3.0) * self.nb2 * w * q * q * that / (q0 ** 2 - q * q))[None, :]
        kern[:, n1] = Zm[:, n1] * (4.0 / 3.0) * self.nb2 * q0 * q0 * c0
        X = np.linalg.solve(np.eye(n1 + 1) - kern, Zm[:, n1].astype(complex))
        U = self.nb2 * X[n1]
        S = 1.0 - 2j * math.pi * (2.0 * q0 / 3.0) * U
        return S
