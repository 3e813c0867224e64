"""wpcd_build_p_noalloc through the C ABI: the P0 it writes into caller
device buffers, with its intermediates in the library's fixed device scratch,
equals wpcd_build_p's bit for bit (same kernels), on two calls in a row, the
second on a smaller grid with another channel set and precision; a capacity
below the nonzero count is rejected with the count reported."""
import sys

import numpy as np
import pytest

from inputs import YAM_BETA, YAM_LAMBDA, YUK_RANGES

pytestmark = pytest.mark.gpu

YAM = dict(kind="yamaguchi", strength=[YAM_LAMBDA], range=[YAM_BETA])
YUK = dict(kind="yukawa", strength=[-1.2, -1.2], range=list(YUK_RANGES))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc(P, ctx, prec, cap):
    """Caller-owned device buffers (allocated here, by the caller, with the
    HIP runtime), filled with a marker first; the entry point writes them."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    nrow = ctx.n_p * ctx.n_q
    nv = max(cap, 1) * ctx.n_ch * ctx.n_ch
    vsz = 8 if prec == P.WPCD_FP64 else 4
    sizes = (8 * (nrow + 1), 4 * max(cap, 1), vsz * nv)
    bufs = [ctypes.c_void_p() for _ in sizes]
    try:
        for b, n in zip(bufs, sizes):
            assert hip.hipMalloc(ctypes.byref(b), ctypes.c_size_t(n)) == 0
            assert hip.hipMemset(b, 0xA5, ctypes.c_size_t(n)) == 0
        assert hip.hipDeviceSynchronize() == 0
        st, nnz = P.wpcd_build_p_noalloc(ctx.h, prec, bufs[0].value, bufs[1].value,
                                         bufs[2].value, cap)
        rp = np.zeros(nrow + 1, np.int64)
        col = np.zeros(max(cap, 1), np.int32)
        val = np.zeros(nv, np.float64 if prec == P.WPCD_FP64 else np.float32)
        for b, a in zip(bufs, (rp, col, val)):
            assert hip.hipMemcpy(a.ctypes.data_as(ctypes.c_void_p), b,
                                 ctypes.c_size_t(a.nbytes), 2) == 0
        return st, nnz, rp, col, val
    finally:
        for b in bufs:
            if b.value:
                hip.hipFree(b)


def _same_as_build_p(P, ctx, prec, label):
    say(f"[{label}] wpcd_build_p n_p={ctx.n_p} n_q={ctx.n_q} n_ch={ctx.n_ch} prec={prec}")
    nnz = ctx.build_p(prec)
    rp0, col0, val0 = ctx.get_p()
    say(f"[{label}] wpcd_build_p_noalloc cap={nnz}")
    st, n, rp, col, val = _noalloc(P, ctx, prec, nnz)
    assert st == P.WPCD_OK, P.STATUS_NAMES[st]
    assert n == nnz
    assert np.array_equal(rp, rp0)
    assert np.array_equal(col[:nnz], col0)
    v = val[:nnz * ctx.n_ch * ctx.n_ch].astype(np.float64).reshape(val0.shape)
    assert np.array_equal(v, val0)      # same kernels: identical bits
    say(f"[{label}] identical: nnz={nnz}")
    return nnz


def test_noalloc_matches_build_p_two_calls():
    import paper_1508_07441_amd as P
    ctx = P.Context(0)
    try:
        # first call: 40 x 40 s-wave, FP32-compensated elements
        ctx.build_basis(40, 40, 10.0, 10.0, 8, 16, potential=YAM)
        _same_as_build_p(P, ctx, P.WPCD_MIXED, "40x40 s-wave")
        # second call, smaller: 12 x 12 with the three L = 2+ channels, FP64
        ctx.build_basis(12, 12, 10.0, 10.0, 8, 16, channels=[(0, 2), (2, 0), (2, 2)], L=2,
                        potential=YUK)
        nnz = _same_as_build_p(P, ctx, P.WPCD_FP64, "12x12 3ch")
        # capacity one short: rejected, count reported, no fault
        say("[12x12 3ch] cap = nnz - 1")
        st, n, _, _, _ = _noalloc(P, ctx, P.WPCD_FP64, nnz - 1)
        assert st == P.WPCD_E_INVALID and n == nnz
        # the context's own P0 is untouched and still solves
        r = ctx.solve([0.5], P.WPCD_FP64)[0]
        assert r.status == P.WPCD_OK
    finally:
        ctx.close()
