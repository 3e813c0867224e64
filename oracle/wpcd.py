"""FP64 CPU oracle for the WPCD three-body hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library: the lattice element and pre-selection live in
``wpcd_oracle.c`` (compiled to ``liborc.so``), the rest is plain numpy/scipy.

The steps follow the paper (Pomerantsev, Kukulin, Rubtsova, Sakhiev,
"Fast GPU-based calculations in few-body quantum scattering"):

1. free wave-packet bins and Gauss tables (Sec. II.B, eq.(ip); Sec. II.D);
2. pair potential in the free WP basis (eq.(vpot)), pair Hamiltonian
   h1 = h0 + v diagonalised to give the rotation O (eq.(exp_z));
3. pre-selection of the nonzero lattice elements (Sec. IV.B);
4. the lattice permutation matrix P0 (eqs.(perm),(gal));
5. the channel resolvent G1 (Sec. II.D, diagonal in the channel WP basis),
   at E or averaged over E's on-shell energy bin (Sec. II.C);
6. the factored kernel K = O P0 V~ G1 with V~ = O^T V1 (eq.(kernel));
7. the matrix Faddeev equation U = P V1 + P V1 G1 U (eq.(m_pvg)) for the
   on-shell column, by dense LU, by GMRES, and by the paper's iterations
   summed with Pade approximants (Sec. III.C);
8. the elastic amplitude from the diagonal element of U (Sec. III.B) and the
   breakup pseudostate elements from the same column.

Conventions (readings of points the paper leaves open):
* hbar = m = 1, so the pair kinetic energy is p^2 and the spectator's 3/4 q^2.
* free WPs with unit weight: <p|x_i> = theta(p in D_i) / (p sqrt d_i) in the
  p^2 dp measure, i.e. B_i = d_i.  This normalisation is the one for which
  the amplitude formula of Sec. III.B, A = 2m/(3 q0) U / d_j0, gives an
  exactly unitary S-matrix below breakup.
* bins are 0-based, bin i = [p[i], p[i+1]]; the channel-basis index of
  (channel a, spectator bin j, pair state k) is (a*Nq + j)*Np + k.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    """Load liborc.so (built by oracle/build.py)."""
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liborc.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        L.orc_cheb_edges.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.orc_is_selected.argtypes = [dp, dp] + [ctypes.c_int] * 4
        L.orc_preselect_counts.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, i64p,
                                           ctypes.c_int64, i64p]
        L.orc_preselect_cols.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, i64p,
                                         ctypes.c_int64, i64p, i32p]
        L.orc_geom_G.argtypes = [ctypes.c_int] * 5 + [ctypes.c_double] * 3
        L.orc_geom_G.restype = ctypes.c_double
        L.orc_geom_G_table.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip] + [ctypes.c_double] * 3 + [dp]
        L.orc_p0_pairs.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ip,
                                   i64p, i32p, ctypes.c_int64, dp]
        _LIB = L
    return _LIB


def _p(a, t):
    # the C routines index the buffer densely: a strided view would be read
    # as the wrong values
    if not a.flags.c_contiguous:
        raise ValueError("arrays passed to the C oracle must be contiguous")
    return a.ctypes.data_as(ctypes.POINTER(t))


# ---------------------------------------------------------------- tables
def gauss_legendre(n: int):
    """n-point Gauss-Legendre nodes (ascending) and weights on [-1, 1]."""
    x = np.zeros(n)
    w = np.zeros(n)
    if lib().orc_gauss_legendre(n, _p(x, ctypes.c_double), _p(w, ctypes.c_double)):
        raise ValueError("bad Gauss order")
    return x, w


def cheb_edges(n: int, vmax: float):
    """Edges vmax (1 - cos(pi k / 2n)), k = 0..n (dense near zero)."""
    e = np.zeros(n + 1)
    lib().orc_cheb_edges(n, float(vmax), _p(e, ctypes.c_double))
    return e


def free_energies(p):
    """Diagonal of h0 = p^2 in the free WP basis: (1/d_i) int_{D_i} p^2 dp."""
    a, b = p[:-1], p[1:]
    return (a * a + a * b + b * b) / 3.0


# ------------------------------------------------------- pair potential
def yamaguchi_lambda(beta: float, kappa: float) -> float:
    """Strength giving a pair bound state at -kappa^2 for v = lam g g,
    g = 1/(p^2 + beta^2): 1 = -lam int p^2 g^2/(p^2+kappa^2) dp."""
    return -4.0 * beta * (beta + kappa) ** 2 / math.pi


def yamaguchi_v(p, lam: float, beta: float):
    """eq.(vpot) for v(p,p') = lam g(p) g(p'): v_ii' = lam gamma_i gamma_i',
    gamma_i = d_i^(-1/2) int_{D_i} p g(p) dp."""
    a, b = p[:-1], p[1:]
    d = b - a
    gam = np.log((b * b + beta * beta) / (a * a + beta * beta)) / (2.0 * np.sqrt(d))
    return lam * np.outer(gam, gam)


def _phi(u, mu):
    """Second antiderivative of ln(u^2 + mu^2)."""
    return 0.5 * (u * u - mu * mu) * np.log(u * u + mu * mu) - 1.5 * u * u \
        + 2.0 * mu * u * np.arctan(u / mu)


def yukawa_v_swave(p, s: float, mu: float):
    """eq.(vpot) in the s-wave for V(r) = s exp(-mu r)/r:
    v(p,p') = s/(2 pi p p') ln(((p+p')^2+mu^2)/((p-p')^2+mu^2)), integrated in
    closed form over the two bins."""
    a, b = p[:-1], p[1:]
    d = b - a
    A = a[:, None]; B = b[:, None]; C = a[None, :]; D = b[None, :]
    plus = _phi(B + D, mu) - _phi(B + C, mu) - _phi(A + D, mu) + _phi(A + C, mu)
    minus = _phi(B - C, mu) - _phi(B - D, mu) - _phi(A - C, mu) + _phi(A - D, mu)
    return s / (2.0 * math.pi) * (plus - minus) / np.sqrt(np.outer(d, d))


def legendre_q(l: int, z):
    """Legendre function of the second kind Q_l(z), z > 1.  Closed form for
    z < 2, hypergeometric series in 1/z^2 for z >= 2 (no cancellation)."""
    z = np.asarray(z, dtype=float)
    out = np.empty_like(z)
    small = z < 2.0
    zs = z[small]
    q0 = 0.5 * np.log((zs + 1.0) / (zs - 1.0))
    if l == 0:
        out[small] = q0
    else:
        qm, qc = q0, zs * q0 - 1.0
        for k in range(1, l):
            qm, qc = qc, ((2 * k + 1) * zs * qc - k * qm) / (k + 1)
        out[small] = qc
    zl = z[~small]
    if zl.size:
        # Q_l(z) = sqrt(pi) l! / (Gamma(l+3/2) (2z)^(l+1)) 2F1((l+1)/2, (l+2)/2; l+3/2; 1/z^2)
        a1, a2, c = (l + 1) / 2.0, (l + 2) / 2.0, l + 1.5
        w = 1.0 / (zl * zl)
        term = np.ones_like(zl)
        ssum = np.ones_like(zl)
        for n in range(200):
            term = term * (a1 + n) * (a2 + n) / ((c + n) * (n + 1)) * w
            ssum = ssum + term
            if np.all(np.abs(term) < 1e-18 * np.abs(ssum)):
                break
        pref = math.sqrt(math.pi) * math.factorial(l) / math.gamma(l + 1.5)
        out[~small] = pref * ssum / (2.0 * zl) ** (l + 1)
    return out


def yukawa_v(p, s: float, mu: float, l: int, n_gauss: int = 24):
    """eq.(vpot) for V(r) = s exp(-mu r)/r in pair wave l by Gauss quadrature:
    v_ii' = (d_i d_i')^(-1/2) int int dp dp' (s/pi) Q_l((p^2+p'^2+mu^2)/(2pp'))."""
    if l == 0:
        return yukawa_v_swave(p, s, mu)
    x, w = gauss_legendre(n_gauss)
    a, b = p[:-1], p[1:]
    d = b - a
    nodes = (0.5 * (a + b))[:, None] + (0.5 * d)[:, None] * x[None, :]
    wts = (0.5 * d)[:, None] * w[None, :]
    P1 = nodes[:, :, None, None]
    P2 = nodes[None, None, :, :]
    z = (P1 * P1 + P2 * P2 + mu * mu) / (2.0 * P1 * P2)
    f = s / math.pi * legendre_q(l, z.ravel()).reshape(z.shape)
    v = np.einsum("ia,iajb,jb->ij", wts, f, wts)
    return v / np.sqrt(np.outer(d, d))


@dataclass
class Potential:
    """Pair potential: kind 'yamaguchi' (s-wave, params lam, beta) or
    'yukawa' (sum of s_k exp(-mu_k r)/r, acting in every pair wave)."""
    kind: str
    strengths: tuple
    ranges: tuple

    def matrix(self, p, l: int):
        if self.kind == "yamaguchi":
            if l != 0:
                return np.zeros((p.size - 1, p.size - 1))
            return yamaguchi_v(p, self.strengths[0], self.ranges[0])
        v = np.zeros((p.size - 1, p.size - 1))
        for s, mu in zip(self.strengths, self.ranges):
            v += yukawa_v(p, s, mu, l)
        return v


def pair_diag(p, v):
    """Diagonalise h1 = diag(eps) + v in the free WP basis (eq.(exp_z)).
    Returns eps* ascending and O with rows = eigenvectors, sign fixed so the
    largest-magnitude component is positive (first index on ties)."""
    h = np.diag(free_energies(p)) + v
    e, vec = np.linalg.eigh(h)
    O = vec.T.copy()
    for k in range(O.shape[0]):
        m = int(np.argmax(np.abs(O[k])))
        if O[k, m] < 0:
            O[k] = -O[k]
    return e, O


def fit_strength(p, ranges, e_target: float, lo: float = 0.0, hi: float = 50.0,
                 iters: int = 200):
    """Bisection on s so that V = -s sum_k exp(-mu_k r)/r has its lowest
    s-wave pair level at e_target in this basis."""
    eps = free_energies(p)
    unit = sum(yukawa_v_swave(p, -1.0, mu) for mu in ranges)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        e0 = np.linalg.eigvalsh(np.diag(eps) + mid * unit)[0]
        if e0 > e_target:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-15 * hi:
            break
    return 0.5 * (lo + hi)


# ------------------------------------------------------------- P0 build
def preselect(p, q, rows=None):
    """Brute-force pre-selection over every column.  Returns (row_ptr, col)
    for the listed cell rows (all rows when None); cols ascending."""
    np_, nq_ = p.size - 1, q.size - 1
    if rows is None:
        rows = np.arange(np_ * nq_, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cnt = np.zeros(rows.size, dtype=np.int64)
    L = lib()
    L.orc_preselect_counts(np_, nq_, _p(p, ctypes.c_double), _p(q, ctypes.c_double),
                           _p(rows, ctypes.c_int64), rows.size, _p(cnt, ctypes.c_int64))
    ptr = np.zeros(rows.size + 1, dtype=np.int64)
    np.cumsum(cnt, out=ptr[1:])
    col = np.zeros(int(ptr[-1]), dtype=np.int32)
    L.orc_preselect_cols(np_, nq_, _p(p, ctypes.c_double), _p(q, ctypes.c_double),
                         _p(rows, ctypes.c_int64), rows.size, _p(ptr, ctypes.c_int64),
                         _p(col, ctypes.c_int32))
    return ptr, col


def p0_pairs(p, q, n_gq, n_gx, L, chans, rows, cols):
    """P0 blocks (n_ch x n_ch, row-channel major) for cell pairs (rows[t], cols[t])."""
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    nch = len(chans)
    la = np.array([c[0] for c in chans], dtype=np.intc)
    lb = np.array([c[1] for c in chans], dtype=np.intc)
    out = np.zeros(rows.size * nch * nch)
    lib().orc_p0_pairs(p.size - 1, q.size - 1, _p(p, ctypes.c_double), _p(q, ctypes.c_double),
                       n_gq, n_gx, L, nch, _p(la, ctypes.c_int), _p(lb, ctypes.c_int),
                       _p(rows, ctypes.c_int64), _p(cols, ctypes.c_int32), rows.size,
                       _p(out, ctypes.c_double))
    return out.reshape(rows.size, nch, nch)


def geom_G(L, a, b, q, q2, x):
    """Angular coupling G^L_{a,b}(q, q', x) for channels a = (l, lam), b."""
    return lib().orc_geom_G(L, a[0], a[1], b[0], b[1], float(q), float(q2), float(x))


def geom_G_table(L, chans, q, q2, x):
    """All channel pairs of G at one node by the node-shared routine of the
    element quadrature: array (nch, nch), rows = first channel."""
    nch = len(chans)
    la = np.array([c[0] for c in chans], dtype=np.intc)
    lb = np.array([c[1] for c in chans], dtype=np.intc)
    out = np.zeros(nch * nch)
    if lib().orc_geom_G_table(L, nch, _p(la, ctypes.c_int), _p(lb, ctypes.c_int), float(q),
                              float(q2), float(x), _p(out, ctypes.c_double)):
        raise ValueError("channel set outside the supported sizes")
    return out.reshape(nch, nch)


# --------------------------------------------------------------- system
@dataclass
class System:
    """Everything the energy-dependent steps need (steps 1-2 of Sec. III.C)."""
    p: np.ndarray
    q: np.ndarray
    L: int
    chans: list
    n_gq: int
    n_gx: int
    pot: Potential
    eps: dict = field(default_factory=dict)     # l -> eps* (ascending)
    O: dict = field(default_factory=dict)       # l -> O (rows eigenvectors)
    v: dict = field(default_factory=dict)       # l -> v matrix
    row_ptr: np.ndarray = None
    col: np.ndarray = None
    val: np.ndarray = None                      # (nnz, nch, nch)
    _P0: object = None
    # pair wave of each channel (key into eps, O, v); None: the channel's l
    wave: list = None

    def wkey(self, a: int):
        """Key of channel a's pair wave in eps, O and v."""
        return self.chans[a][0] if self.wave is None else self.wave[a]

    @property
    def Np(self):
        return self.p.size - 1

    @property
    def Nq(self):
        return self.q.size - 1

    @property
    def M(self):
        return len(self.chans) * self.Np * self.Nq

    def P0_matrix(self):
        """P0 as a scipy CSR matrix over (channel, j, i)."""
        if self._P0 is None:
            nch, ncell = len(self.chans), self.Np * self.Nq
            rows = np.repeat(np.arange(ncell), np.diff(self.row_ptr))
            R, C, V = [], [], []
            for a in range(nch):
                for b in range(nch):
                    R.append(rows + a * ncell)
                    C.append(self.col.astype(np.int64) + b * ncell)
                    V.append(self.val[:, a, b])
            self._P0 = sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))),
                                     shape=(nch * ncell, nch * ncell))
        return self._P0


def build_system(p, q, L, chans, n_gq, n_gx, pot: Potential, with_p0=True) -> System:
    s = System(p=p, q=q, L=L, chans=list(chans), n_gq=n_gq, n_gx=n_gx, pot=pot)
    for l in sorted({c[0] for c in chans}):
        v = pot.matrix(p, l)
        e, O = pair_diag(p, v)
        s.eps[l], s.O[l], s.v[l] = e, O, v
    if with_p0:
        s.row_ptr, s.col = preselect(p, q)
        rows = np.repeat(np.arange(s.Np * s.Nq, dtype=np.int64), np.diff(s.row_ptr))
        s.val = p0_pairs(p, q, n_gq, n_gx, L, chans, rows, s.col)
    return s


# ------------------------------------------------------------ resolvent
class OnEdge(ValueError):
    pass


def resolvent_bin(E: float, eps_k: float, qlo: float, qhi: float, qmax: float):
    """(1/dq) int_{qlo}^{qhi} dq / (E - eps_k - 3/4 q^2 + i0)."""
    s = E - eps_k
    dq = qhi - qlo
    if s > 0.0:
        qs = math.sqrt(4.0 * s / 3.0)
        if abs(qs - qlo) < 1e-12 * qmax or abs(qs - qhi) < 1e-12 * qmax:
            raise OnEdge("on-shell momentum on a bin edge")
        f = lambda x: math.log((qs + x) / abs(qs - x))
        re = 2.0 / (3.0 * qs * dq) * (f(qhi) - f(qlo))
        im = -2.0 * math.pi / (3.0 * qs * dq) if (qlo < qs < qhi) else 0.0
        return complex(re, im)
    if s < 0.0:
        ka = math.sqrt(-4.0 * s / 3.0)
        return complex(-4.0 / (3.0 * ka * dq) * (math.atan(qhi / ka) - math.atan(qlo / ka)), 0.0)
    raise OnEdge("zero spectator energy")


def log_integral(s: float, qa: float, qb: float) -> float:
    """F(s) = int_qa^qb ln|s - 3/4 q^2| dq in closed form (b = sqrt(3)/2):
    s > 0, a = sqrt(s): [((b q - a)(ln|b q - a| - 1) + (a + b q)(ln(a + b q) - 1)) / b];
    s < 0, k = sqrt(-s): [q ln(k^2 + b^2 q^2) - 2 q + (2 k / b) atan(b q / k)];
    s = 0: [2 q (ln(b q) - 1)]."""
    b = math.sqrt(3.0) / 2.0

    def tlogt(t):
        return t * (math.log(abs(t)) - 1.0) if t != 0.0 else 0.0

    def prim(q):
        if s > 0.0:
            a = math.sqrt(s)
            return (tlogt(b * q - a) + tlogt(a + b * q)) / b
        if s < 0.0:
            kap = math.sqrt(-s)
            return q * math.log(-s + 0.75 * q * q) - 2.0 * q + 2.0 * kap / b * math.atan(b * q / kap)
        return 2.0 * tlogt(b * q) / b if q > 0.0 else 0.0

    return prim(qb) - prim(qa)


def shell_overlap(s1: float, s2: float, qa: float, qb: float) -> float:
    """Length of {q in [qa, qb] : s1 < 3/4 q^2 < s2}."""
    if s2 <= 0.0:
        return 0.0
    q1 = math.sqrt(4.0 * s1 / 3.0) if s1 > 0.0 else 0.0
    q2 = math.sqrt(4.0 * s2 / 3.0)
    return max(0.0, min(qb, q2) - max(qa, q1))


def resolvent_bin_avg(E1: float, E2: float, eps_k: float, qlo: float, qhi: float):
    """The channel resolvent eigenvalue averaged over the on-shell energy
    interval [E1, E2] (Sec. II.C, the bin average of g_0i(E) carried over
    to the three-body channel resolvent):
      (1/(D dq)) int_{E1}^{E2} dE int_{qlo}^{qhi} dq / (E - eps_k - 3/4 q^2 + i0),
    D = E2 - E1, dq = qhi - qlo.  The E integral is ln|E2 - c| - ln|E1 - c|
    - i pi [E1 < c < E2] with c = eps_k + 3/4 q^2; the q integral of the logs
    is log_integral, that of the step the overlap length."""
    D, dq = E2 - E1, qhi - qlo
    s1, s2 = E1 - eps_k, E2 - eps_k
    re = (log_integral(s2, qlo, qhi) - log_integral(s1, qlo, qhi)) / (D * dq)
    im = -math.pi * shell_overlap(s1, s2, qlo, qhi) / (D * dq)
    return complex(re, im)


def energy_bin(sysm: System, E: float):
    """On-shell energy interval of E for the averaged resolvent: the
    energies eps*_0 + 3/4 q^2 over the entrance spectator bin j0 that holds
    q0 (every E in it gives the same averaged kernel and amplitudes)."""
    a0, j0, q0, idx = entrance(sysm, E)
    eb = sysm.eps[sysm.wkey(a0)][0]
    return eb + 0.75 * sysm.q[j0] ** 2, eb + 0.75 * sysm.q[j0 + 1] ** 2


def resolvent(sysm: System, E: float, averaged: bool = False):
    """Diagonal of G1(E) in the channel WP basis, shape (nch, Nq, Np); with
    averaged, each eigenvalue averaged over E's on-shell energy bin."""
    G = np.zeros((len(sysm.chans), sysm.Nq, sysm.Np), dtype=complex)
    qmax = sysm.q[-1]
    if averaged:
        E1, E2 = energy_bin(sysm, E)
    for a in range(len(sysm.chans)):
        eps = sysm.eps[sysm.wkey(a)]
        for j in range(sysm.Nq):
            for k in range(sysm.Np):
                if averaged:
                    G[a, j, k] = resolvent_bin_avg(E1, E2, eps[k], sysm.q[j], sysm.q[j + 1])
                else:
                    G[a, j, k] = resolvent_bin(E, eps[k], sysm.q[j], sysm.q[j + 1], qmax)
    return G


# --------------------------------------------------------------- kernel
def _blockwise(sysm: System, y, mats):
    """Apply a per-channel N x N matrix to the pair index of y (nch, Nq, Np)."""
    out = np.empty_like(y)
    for a in range(len(sysm.chans)):
        out[a] = y[a] @ mats[sysm.wkey(a)].T
    return out


def apply_A(sysm: System, y):
    """A y = O P0 V~ y, with V~ = O^T (O v O^T) = v O^T per pair wave (eq.(kernel))."""
    y = y.reshape(len(sysm.chans), sysm.Nq, sysm.Np)
    vt = {w: sysm.v[w] @ sysm.O[w].T for w in sysm.v}
    y2 = _blockwise(sysm, y, vt)
    y3 = (sysm.P0_matrix() @ y2.ravel()).reshape(y.shape)
    return _blockwise(sysm, y3, sysm.O).ravel()


def apply_K(sysm: System, G, y):
    """K y = O P0 V~ G1 y (eq.(kernel))."""
    return apply_A(sysm, G.ravel() * y)


def entrance(sysm: System, E: float):
    """Incident state e0: channel with l = 0, lam = L; pair bound state k = 0;
    spectator bin j0 holding q0 = sqrt(4 (E - eps*_0) / 3)."""
    a0 = [i for i, c in enumerate(sysm.chans) if c[0] == 0 and c[1] == sysm.L]
    if not a0:
        raise ValueError("no entrance channel (l=0, lam=L)")
    a0 = a0[0]
    eb = sysm.eps[sysm.wkey(a0)][0]
    if E <= eb:
        raise ValueError("energy below the two-body threshold")
    q0 = math.sqrt(4.0 * (E - eb) / 3.0)
    j0 = int(np.searchsorted(sysm.q, q0) - 1)
    if j0 < 0 or j0 >= sysm.Nq:
        raise ValueError("q0 outside the spectator grid")
    idx = (a0 * sysm.Nq + j0) * sysm.Np + 0
    return a0, j0, q0, idx


def rhs(sysm: System, idx: int):
    """b = A e0 = P V1 e0 (the driving term of eq.(m_pvg))."""
    e = np.zeros(sysm.M, dtype=complex)
    e[idx] = 1.0
    return apply_A(sysm, e)


# --------------------------------------------------------------- solvers
def dense_K(sysm: System, G):
    """Dense K = A G1 (small systems only)."""
    M = sysm.M
    A = np.empty((M, M))
    eye = np.zeros(M)
    for c in range(M):
        eye[:] = 0.0
        eye[c] = 1.0
        A[:, c] = apply_A(sysm, eye).real
    return A * G.ravel()[None, :]


def solve_lu(sysm: System, E: float):
    """Dense complex LU solve of (1 - K) u = A e0."""
    a0, j0, q0, idx = entrance(sysm, E)
    G = resolvent(sysm, E)
    K = dense_K(sysm, G)
    b = rhs(sysm, idx)
    return np.linalg.solve(np.eye(sysm.M) - K, b)


def gmres(matvec, b, tol=1e-13, m=50, max_restarts=200, x0=None):
    """Restarted GMRES(m), modified Gram-Schmidt Arnoldi, least-squares by
    numpy.lstsq.  Returns (x, iterations, relative residual)."""
    n = b.size
    x = np.zeros(n, dtype=complex) if x0 is None else x0.astype(complex).copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, 0.0
    its = 0
    for _ in range(max_restarts):
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta <= tol * bn:
            return x, its, beta / bn
        V = np.zeros((m + 1, n), dtype=complex)
        H = np.zeros((m + 1, m), dtype=complex)
        V[0] = r / beta
        k_done = 0
        y = None
        for k in range(m):
            w = matvec(V[k])
            its += 1
            for i in range(k + 1):
                H[i, k] = np.vdot(V[i], w)
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] != 0.0:
                V[k + 1] = w / H[k + 1, k]
            e1 = np.zeros(k + 2, dtype=complex)
            e1[0] = beta
            y = np.linalg.lstsq(H[:k + 2, :k + 1], e1, rcond=None)[0]
            res = np.linalg.norm(e1 - H[:k + 2, :k + 1] @ y)
            k_done = k + 1
            if res <= tol * bn or H[k + 1, k] == 0.0:
                break
        x = x + V[:k_done].T @ y
    r = b - matvec(x)
    return x, its, np.linalg.norm(r) / bn


def solve_gmres(sysm: System, E: float, tol=1e-13, m=50, averaged=False):
    a0, j0, q0, idx = entrance(sysm, E)
    G = resolvent(sysm, E, averaged)
    b = rhs(sysm, idx)
    u, its, res = gmres(lambda y: y - apply_K(sysm, G, y), b, tol=tol, m=m)
    return u, its, res


def wynn_epsilon(s):
    """Wynn's epsilon algorithm on the scalar sequence s; returns the list
    of diagonal values eps_{2k}^{(0)} (the [k/k] Pade approximants)."""
    n = len(s)
    prev = [0.0 + 0.0j] * (n + 1)    # eps_{-1}
    cur = list(s)                    # eps_0
    diag = [cur[0]]
    for k in range(1, n):
        nxt = []
        for i in range(len(cur) - 1):
            d = cur[i + 1] - cur[i]
            if d == 0:
                return diag
            nxt.append(prev[i + 1] + 1.0 / d)
        prev, cur = cur, nxt
        if k % 2 == 0 and cur:
            diag.append(cur[0])
    return diag


def solve_pade(sysm: System, E: float, n_terms: int = 80, tol: float = 1e-12):
    """The paper's route (Sec. III.C): iterate u_{n+1} = K u_n from u_0 = b,
    form the partial sums of the on-shell component and sum them with
    diagonal Pade approximants (Wynn epsilon).  Stops when two successive
    diagonal approximants agree to tol, or returns the approximant at the
    smallest successive change once round-off makes them wander (the terms
    grow like |lambda_max(K)|^n above the three-body bound state).
    Returns (on-shell U, last successive change)."""
    a0, j0, q0, idx = entrance(sysm, E)
    G = resolvent(sysm, E)
    u = rhs(sysm, idx)
    partial, acc = [], 0.0 + 0.0j
    for n in range(n_terms):
        acc += u[idx]
        partial.append(acc)
        u = apply_K(sysm, G, u)
    d = wynn_epsilon(partial)
    best, best_diff = d[-1], float("inf")
    for k in range(1, len(d)):
        diff = abs(d[k] - d[k - 1])
        if diff < best_diff:
            best, best_diff = d[k], diff
        if diff <= tol * abs(d[k]):
            return d[k], diff
    return best, best_diff


# ------------------------------------------------------------ amplitudes
@dataclass
class Amplitude:
    E: float
    q0: float
    j0: int
    U00: complex
    A: complex
    S: complex
    delta: float
    eta: float
    breakup: list   # (channel, k, j, S_(k j)0)
    breakup_dist: list = None   # (channel, k, eps*_k, sum_j |S_(k j)0|^2, bins)


def amplitudes(sysm: System, E: float, u, averaged: bool = False):
    """Elastic amplitude A = rho0 U00 with rho0 = 2/(3 q0 dq_j0) (Sec.
    III.B with m = 1), S = 1 - 2 pi i A; breakup elements
    S_(kj)0 = -2 pi i sqrt(rho_kj rho_0) u_(kj) of every open channel state,
    rho = -Im G1 / pi: the pseudostate's on-shell bin with rho = 2/(3 q dq)
    for the resolvent at E; for the averaged resolvent every bin j whose
    shell overlaps the on-shell energy bin [E1, E2], rho = overlap / (D dq),
    and rho0 = 1 / D (the elastic state's whole bin).  breakup_dist sums
    |S|^2 over the bins of each pseudostate: the breakup distribution over
    the pair energy eps*_k."""
    a0, j0, q0, idx = entrance(sysm, E)
    dq = sysm.q[1:] - sysm.q[:-1]
    if averaged:
        E1, E2 = energy_bin(sysm, E)
        D = E2 - E1
        rho0 = 1.0 / D
    else:
        rho0 = 2.0 / (3.0 * q0 * dq[j0])
    U00 = u[idx]
    A = rho0 * U00
    S = 1.0 - 2j * math.pi * A
    br, dist = [], []
    for a in range(len(sysm.chans)):
        for k, ek in enumerate(sysm.eps[sysm.wkey(a)]):
            if a == a0 and k == 0:
                continue
            states = []
            if averaged:
                for j in range(sysm.Nq):
                    ov = shell_overlap(E1 - ek, E2 - ek, sysm.q[j], sysm.q[j + 1])
                    if ov > 0.0:
                        states.append((j, ov / (D * dq[j])))
            elif ek < E:
                qk = math.sqrt(4.0 * (E - ek) / 3.0)
                jk = int(np.searchsorted(sysm.q, qk) - 1)
                if 0 <= jk < sysm.Nq:
                    states.append((jk, 2.0 / (3.0 * qk * dq[jk])))
            if not states:
                continue
            tot = 0.0
            for j, rk in states:
                Sk = -2j * math.pi * math.sqrt(rk * rho0) * u[(a * sysm.Nq + j) * sysm.Np + k]
                br.append((a, k, j, Sk))
                tot += abs(Sk) ** 2
            dist.append((a, k, float(ek), tot, len(states)))
    d = 0.5 * math.atan2(S.imag, S.real)
    return Amplitude(E, q0, j0, U00, A, S, d, abs(S), br, dist)


# ----------------------------------------------------------- bound state
def kernel_top_eig(sysm: System, E: float):
    """Largest real eigenvalue of the real kernel K(E) for E below the
    two-body threshold (homogeneous form of eq.(m_pvg))."""
    import scipy.sparse.linalg as sla
    G = resolvent(sysm, E).real.ravel()
    op = sla.LinearOperator((sysm.M, sysm.M), matvec=lambda y: apply_A(sysm, G * y).real,
                            dtype=float)
    vals = sla.eigs(op, k=4, which="LR", return_eigenvectors=False, tol=1e-12)
    return float(np.max(vals.real))


def bound_state(sysm: System, e_lo: float, e_hi: float, tol=1e-10):
    """Three-body bound state: E with top eigenvalue of K(E) equal to 1,
    by bisection on [e_lo, e_hi] (both below the pair threshold)."""
    f_lo = kernel_top_eig(sysm, e_lo) - 1.0
    f_hi = kernel_top_eig(sysm, e_hi) - 1.0
    if f_lo * f_hi > 0:
        raise ValueError("no sign change of lambda_max - 1 on the bracket")
    for _ in range(100):
        mid = 0.5 * (e_lo + e_hi)
        fm = kernel_top_eig(sysm, mid) - 1.0
        if fm * f_lo > 0:
            e_lo, f_lo = mid, fm
        else:
            e_hi, f_hi = mid, fm
        if e_hi - e_lo < tol * abs(mid):
            break
    return 0.5 * (e_lo + e_hi)
