"""Pins for the oracle of the model matrix fills (Sec. IV.A, eqs.(Atrig),
(Agau), (Acond)); CPU only.

* the counter-based random numbers equal the sequential splitmix64 stream;
* eq.(Agau) with K = 1 and K = 2 against closed forms: the integral of
  sin + cos is (cos u - cos w) + (sin w - sin u), and that of sin^2 + cos^2 is
  w - u; higher K against adaptive quadrature;
* eq.(Atrig) against a direct evaluation with powers for a few elements;
* eq.(Acond) keeps exactly the elements with u <= alpha, a fraction close
  to alpha.
"""
import math

import numpy as np
from scipy import integrate

import oracle.model as MD
from inputs import splitmix64, SEED


def test_counter_based_stream_is_splitmix64():
    s = SEED
    seq = []
    for _ in range(10):
        s, x = splitmix64(s)
        seq.append((x >> 11) * 2.0 ** -53)
    u, w = MD.model_inputs(SEED, 3)
    assert np.array_equal(np.stack([u.ravel(), w.ravel()], 1).ravel()[:10], np.array(seq))


def test_gauss_elements_closed_forms():
    u, w = MD.model_inputs(SEED + 1, 8)
    a1 = MD.gauss_elements(u, w, 1)
    ref1 = (np.cos(u) - np.cos(w)) + (np.sin(w) - np.sin(u))
    assert np.max(np.abs(a1 - ref1)) < 1e-14
    a2 = MD.gauss_elements(u, w, 2)
    ref2 = ref1 + (w - u)
    assert np.max(np.abs(a2 - ref2)) < 1e-14


def test_gauss_elements_vs_adaptive_quadrature():
    u, w = MD.model_inputs(SEED + 2, 4)
    K = 7
    a = MD.gauss_elements(u, w, K)
    for i in range(4):
        for j in range(4):
            f = lambda t: sum(math.sin(t) ** k + math.cos(t) ** k for k in range(1, K + 1))
            ref = integrate.quad(f, u[i, j], w[i, j], epsabs=0, epsrel=1e-13)[0]
            assert abs(a[i, j] - ref) <= 1e-13 * max(1.0, abs(ref))


def test_trig_elements_direct():
    u, w = MD.model_inputs(SEED + 3, 5)
    K = 9
    a = MD.trig_elements(u, w, K)
    for i, j in [(0, 0), (2, 3), (4, 1)]:
        ref = sum(math.pow(math.sin(u[i, j]), k) + math.pow(math.cos(w[i, j]), k)
                  for k in range(1, K + 1))
        assert abs(a[i, j] - ref) <= 1e-13 * abs(ref)


def test_sparse_filter():
    M, alpha = 64, 0.05
    idx, val = MD.model_fill("trig", M, 4, SEED, alpha)
    u, w = MD.model_inputs(SEED, M)
    assert np.array_equal(idx, np.flatnonzero(u <= alpha))
    assert abs(idx.size / M ** 2 - alpha) < 0.01
    dense = MD.model_fill("trig", M, 4, SEED)
    assert np.array_equal(val, dense.ravel()[idx])
