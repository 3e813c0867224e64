"""FP64 CPU oracle of the paper's model matrix fills (Sec. IV.A).

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): only ``tests/`` and
``bench.py``'s ``cpu_baseline`` leg may use it.  It shares no code with the
HIP library.

Two element formulas over random u_ij, w_ij in [0, 1):
* eq.(Atrig): A(i, j) = sum_{k=1..K} (sin^k(u_ij) + cos^k(w_ij));
* eq.(Agau):  A(i, j) = sum_{k=1..K} int_{u_ij}^{w_ij} (sin^k t + cos^k t) dt,
  each integral by the 48-point Gauss-Legendre rule;
and the sparse variant eq.(Acond): the element is kept where u_ij <= alpha
and is zero elsewhere.

Random numbers: the counter-based form of splitmix64 (Steele, Lea, Flood
2014): output n of the stream started at `seed` is mix(seed + (n + 1) g),
g = 0x9E3779B97F4A7C15, u = (x >> 11) 2^-53; u_ij is output 2 (i M + j) and
w_ij output 2 (i M + j) + 1.  This module takes them from the seeded input
module of the tests (``inputs.uniforms``), which computes the same stream.
"""
import numpy as np

from inputs import uniforms


def model_inputs(seed: int, M: int):
    """u, w as M x M arrays (row i, column j)."""
    x = np.array(uniforms(seed, 2 * M * M)).reshape(M * M, 2)
    return x[:, 0].reshape(M, M), x[:, 1].reshape(M, M)


def trig_elements(u, w, K: int):
    """eq.(Atrig), elementwise on arrays u, w."""
    s, c = np.sin(u), np.cos(w)
    out = np.zeros_like(u)
    for k in range(1, K + 1):
        out += s ** k + c ** k
    return out


def gauss_elements(u, w, K: int, n_gauss: int = 48):
    """eq.(Agau): sum over k of the n_gauss-point Gauss-Legendre rule of
    sin^k t + cos^k t on [u, w] (numpy's Legendre nodes and weights)."""
    x, wt = np.polynomial.legendre.leggauss(n_gauss)
    half, mid = 0.5 * (w - u), 0.5 * (w + u)
    out = np.zeros_like(u)
    for xg, wg in zip(x, wt):
        t = mid + half * xg
        s, c = np.sin(t), np.cos(t)
        f = np.zeros_like(u)
        for k in range(1, K + 1):
            f += s ** k + c ** k
        out += wg * f
    return half * out


def model_fill(kind: str, M: int, K: int, seed: int, alpha: float = None):
    """The M x M model matrix; with alpha, eq.(Acond)'s sparse form as
    (flat indices i M + j ascending, values)."""
    u, w = model_inputs(seed, M)
    A = trig_elements(u, w, K) if kind == "trig" else gauss_elements(u, w, K)
    if alpha is None:
        return A
    keep = u <= alpha
    idx = np.flatnonzero(keep)
    return idx.astype(np.int64), A.ravel()[idx]
