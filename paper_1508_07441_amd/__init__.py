"""Python binding of libwpcd.so (the MI355X WPCD hot path).

Argument marshalling only: every step runs in the library's HIP kernels.
The functions carry the C ABI's names (include/wpcd.h); ``Context`` is a
small convenience wrapper over them.  If the library has not been built,
importing works but every call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwpcd.so")

WPCD_OK = 0
WPCD_E_INVALID = 1
WPCD_E_NOMEM = 2
WPCD_E_DEVICE = 3
WPCD_E_NOT_CONVERGED = 4
WPCD_E_BELOW_THRESHOLD = 5
WPCD_E_ON_EDGE = 6
WPCD_E_STATE = 7
WPCD_E_STAGNATED = 8
WPCD_FP64 = 0
WPCD_MIXED = 1
WPCD_MIXED_REFINE = 2
WPCD_MIXED_BF16 = 3
WPCD_TIME_PAIR = 1
WPCD_TIME_P0 = 2
WPCD_TIME_SOLVE = 4
WPCD_TIME_PRESELECT = 8
WPCD_TIME_ALL = 15
WPCD_WARM_NONE = 0
WPCD_WARM_LEARNED = 1
WPCD_WARM_GIVEN = 2
WPCD_RESOLVENT_AT_E = 0
WPCD_RESOLVENT_AVERAGED = 1
WPCD_BREAKUP_ELEMENTS = 1
WPCD_BREAKUP_DIST = 2
WPCD_TUNE_HEURISTIC = 0
WPCD_TUNE_MEASURE = 1
WPCD_TUNE_FORCE = 16

STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_NOMEM", 3: "E_DEVICE", 4: "E_NOT_CONVERGED",
                5: "E_BELOW_THRESHOLD", 6: "E_ON_EDGE", 7: "E_STATE", 8: "E_STAGNATED"}

ABI_FUNCTIONS = ("wpcd_create", "wpcd_build_basis", "wpcd_build_basis_nucleons",
                 "wpcd_set_potential", "wpcd_pair_spectrum",
                 "wpcd_build_p", "wpcd_build_p_noalloc", "wpcd_get_p", "wpcd_save_p",
                 "wpcd_load_p", "wpcd_build_reduced", "wpcd_solve",
                 "wpcd_solve_dev", "wpcd_solve_multi", "wpcd_sweep", "wpcd_bound_state",
                 "wpcd_model_fill",
                 "wpcd_set_multipliers",
                 "wpcd_learn_train", "wpcd_mlp_eval", "wpcd_set_autotune",
                 "wpcd_get_autotune", "wpcd_set_graphs", "wpcd_set_timing",
                 "wpcd_get_timing", "wpcd_reset_timing", "wpcd_synchronize", "wpcd_last_error",
                 "wpcd_destroy")


class wpcd_basis_desc(ctypes.Structure):
    _fields_ = [("n_p", ctypes.c_int32), ("n_q", ctypes.c_int32),
                ("p_max", ctypes.c_double), ("q_max", ctypes.c_double),
                ("edge_kind", ctypes.c_int32),
                ("p_edges", ctypes.POINTER(ctypes.c_double)),
                ("q_edges", ctypes.POINTER(ctypes.c_double)),
                ("n_gauss_q", ctypes.c_int32), ("n_gauss_x", ctypes.c_int32),
                ("L", ctypes.c_int32), ("n_ch", ctypes.c_int32),
                ("l", ctypes.POINTER(ctypes.c_int32)), ("lam", ctypes.POINTER(ctypes.c_int32))]


class wpcd_nucleon_desc(ctypes.Structure):
    _fields_ = [("two_S", ctypes.c_int32), ("n_ch", ctypes.c_int32),
                ("s", ctypes.POINTER(ctypes.c_int32)), ("t", ctypes.POINTER(ctypes.c_int32)),
                ("mult", ctypes.POINTER(ctypes.c_double))]


class wpcd_potential_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_terms", ctypes.c_int32),
                ("strength", ctypes.POINTER(ctypes.c_double)),
                ("range", ctypes.POINTER(ctypes.c_double)),
                ("fit_e2", ctypes.c_double)]


class wpcd_solve_opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("krylov_dim", ctypes.c_int32),
                ("tol", ctypes.c_double), ("want_breakup", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("x0", ctypes.POINTER(ctypes.c_double)),
                ("err_est", ctypes.c_int32), ("resolvent", ctypes.c_int32),
                ("fallback_tol", ctypes.c_double)]


class wpcd_energy_result(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("q0", ctypes.c_double),
                ("j0", ctypes.c_int32), ("status", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("n_open", ctypes.c_int32),
                ("U_re", ctypes.c_double), ("U_im", ctypes.c_double),
                ("A_re", ctypes.c_double), ("A_im", ctypes.c_double),
                ("S_re", ctypes.c_double), ("S_im", ctypes.c_double),
                ("delta", ctypes.c_double), ("eta", ctypes.c_double),
                ("residual", ctypes.c_double), ("warm", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("r0", ctypes.c_double),
                ("err_vs_fp64", ctypes.c_double)]


class wpcd_learn_desc(ctypes.Structure):
    _fields_ = [("n_var", ctypes.c_int32), ("n_mult", ctypes.c_int32),
                ("mult", ctypes.POINTER(ctypes.c_double)), ("n_E", ctypes.c_int32),
                ("E", ctypes.POINTER(ctypes.c_double)), ("precision", ctypes.c_int32),
                ("n_basis", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("solve", ctypes.POINTER(wpcd_solve_opts))]


class wpcd_learn_report(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int32), ("plain_iters", ctypes.c_int32),
                ("basis_max_rel_err", ctypes.c_double), ("basis_mean_rel_err", ctypes.c_double),
                ("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("basis_ms", ctypes.c_double),
                ("train_ms", ctypes.c_double)]


class wpcd_tune_entry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("key", ctypes.c_char * 64),
                ("choice", ctypes.c_int32), ("n_candidates", ctypes.c_int32),
                ("us", ctypes.c_double)]


class wpcd_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("total_ms", ctypes.c_double),
                ("launches", ctypes.c_int64)]


class WpcdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libwpcd.so; raise if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1508_07441_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        L.wpcd_create.argtypes = [ctypes.c_int, vp, ctypes.POINTER(vp)]
        L.wpcd_build_basis.argtypes = [vp, ctypes.POINTER(wpcd_basis_desc),
                                       ctypes.POINTER(wpcd_potential_desc)]
        L.wpcd_build_basis_nucleons.argtypes = [vp, ctypes.POINTER(wpcd_basis_desc),
                                                ctypes.POINTER(wpcd_potential_desc),
                                                ctypes.POINTER(wpcd_nucleon_desc)]
        L.wpcd_set_potential.argtypes = [vp, ctypes.POINTER(wpcd_potential_desc)]
        L.wpcd_pair_spectrum.argtypes = [vp, ctypes.c_int32, dp, dp, dp]
        L.wpcd_build_p.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
        L.wpcd_build_p_noalloc.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_int64)]
        L.wpcd_get_p.argtypes = [vp, ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int32), dp]
        L.wpcd_build_reduced.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
        L.wpcd_solve.argtypes = [vp, dp, ctypes.c_int32, ctypes.c_int,
                                 ctypes.POINTER(wpcd_solve_opts),
                                 ctypes.POINTER(wpcd_energy_result), dp]
        fp = ctypes.POINTER(ctypes.c_float)
        L.wpcd_bound_state.argtypes = [vp, ctypes.c_double, ctypes.c_double, dp]
        L.wpcd_model_fill.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                                      ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int64), dp,
                                      ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), dp]
        L.wpcd_save_p.argtypes = [vp, ctypes.c_char_p]
        L.wpcd_load_p.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)]
        L.wpcd_solve_dev.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int,
                                     ctypes.POINTER(wpcd_solve_opts), vp]
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.wpcd_sweep.argtypes = [vp, dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int,
                                 ctypes.POINTER(wpcd_solve_opts), ctypes.c_char_p, ctypes.c_int32,
                                 ctypes.POINTER(wpcd_energy_result), i32p, i32p]
        L.wpcd_solve_multi.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(dp),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.c_int,
                                       ctypes.POINTER(wpcd_solve_opts),
                                       ctypes.POINTER(ctypes.POINTER(wpcd_energy_result)),
                                       ctypes.POINTER(ctypes.c_int)]
        L.wpcd_set_multipliers.argtypes = [vp, dp, ctypes.c_int32]
        L.wpcd_learn_train.argtypes = [vp, ctypes.POINTER(wpcd_learn_desc),
                                       ctypes.POINTER(wpcd_learn_report)]
        L.wpcd_mlp_eval.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, fp,
                                    ctypes.c_int32, fp, fp, fp, fp, dp]
        L.wpcd_set_autotune.argtypes = [vp, ctypes.c_int32]
        L.wpcd_get_autotune.argtypes = [vp, ctypes.POINTER(wpcd_tune_entry), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]
        L.wpcd_set_graphs.argtypes = [vp, ctypes.c_int32]
        L.wpcd_set_timing.argtypes = [vp, ctypes.c_int32]
        L.wpcd_get_timing.argtypes = [vp, ctypes.POINTER(wpcd_kernel_time), ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int32)]
        L.wpcd_reset_timing.argtypes = [vp]
        L.wpcd_synchronize.argtypes = [vp]
        L.wpcd_last_error.argtypes = [vp]
        L.wpcd_last_error.restype = ctypes.c_char_p
        L.wpcd_destroy.argtypes = [vp]
        L.wpcd_destroy.restype = None
        for f in ABI_FUNCTIONS:
            if f not in ("wpcd_last_error", "wpcd_destroy"):
                getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(ctx, st):
    if st != WPCD_OK:
        msg = lib().wpcd_last_error(ctx).decode() if ctx else ""
        raise WpcdError(st, msg)


# ------------------------------------------------------------ ABI names
def wpcd_create(device: int = 0, stream: int | None = None):
    h = ctypes.c_void_p()
    st = lib().wpcd_create(device, ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
    if st != WPCD_OK:
        raise WpcdError(st, "wpcd_create failed")
    return h


def wpcd_build_basis(ctx, n_p, n_q, p_max, q_max, n_gauss_q, n_gauss_x, channels=((0, 0),),
                     L=0, potential=None, p_edges=None, q_edges=None):
    l = np.ascontiguousarray([c[0] for c in channels], dtype=np.int32)
    lam = np.ascontiguousarray([c[1] for c in channels], dtype=np.int32)
    pe = None if p_edges is None else np.ascontiguousarray(p_edges, dtype=np.float64)
    qe = None if q_edges is None else np.ascontiguousarray(q_edges, dtype=np.float64)
    d = wpcd_basis_desc(n_p, n_q, float(p_max), float(q_max), 0 if pe is None else 1,
                        _dp(pe), _dp(qe), n_gauss_q, n_gauss_x, L, len(channels),
                        l.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        lam.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    pd, keep = _pot_desc(potential)
    _check(ctx, lib().wpcd_build_basis(ctx, ctypes.byref(d), ctypes.byref(pd)))
    del keep


def wpcd_build_basis_nucleons(ctx, n_p, n_q, p_max, q_max, n_gauss_q, n_gauss_x, two_S,
                              channels=((1, 0), (0, 1)), potential=None, mult=None,
                              p_edges=None, q_edges=None):
    """channels: (pair spin s, pair isospin t) per channel, (1, 0) first;
    mult: per channel, one strength multiplier per potential term."""
    s_ = np.ascontiguousarray([c[0] for c in channels], dtype=np.int32)
    t_ = np.ascontiguousarray([c[1] for c in channels], dtype=np.int32)
    m_ = None if mult is None else np.ascontiguousarray(mult, dtype=np.float64).ravel()
    pe = None if p_edges is None else np.ascontiguousarray(p_edges, dtype=np.float64)
    qe = None if q_edges is None else np.ascontiguousarray(q_edges, dtype=np.float64)
    d = wpcd_basis_desc(n_p, n_q, float(p_max), float(q_max), 0 if pe is None else 1,
                        _dp(pe), _dp(qe), n_gauss_q, n_gauss_x, 0, 0, None, None)
    nd = wpcd_nucleon_desc(int(two_S), len(channels),
                           s_.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           t_.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(m_))
    pd, keep = _pot_desc(potential)
    _check(ctx, lib().wpcd_build_basis_nucleons(ctx, ctypes.byref(d), ctypes.byref(pd),
                                                ctypes.byref(nd)))
    del keep


def _pot_desc(potential):
    """potential: dict(kind='yamaguchi'|'yukawa', strength=[...], range=[...], fit_e2=None)."""
    kind = {"yamaguchi": 0, "yukawa": 1}[potential["kind"]]
    s = np.ascontiguousarray(potential["strength"], dtype=np.float64)
    r = np.ascontiguousarray(potential["range"], dtype=np.float64)
    fit = potential.get("fit_e2")
    d = wpcd_potential_desc(kind, s.size, _dp(s), _dp(r), math.nan if fit is None else float(fit))
    return d, (s, r)


def wpcd_set_potential(ctx, potential):
    pd, keep = _pot_desc(potential)
    _check(ctx, lib().wpcd_set_potential(ctx, ctypes.byref(pd)))
    del keep


def wpcd_pair_spectrum(ctx, l, n_p, want_O=True):
    eps = np.zeros(n_p)
    O = np.zeros((n_p, n_p)) if want_O else None
    sc = np.zeros(1)
    _check(ctx, lib().wpcd_pair_spectrum(ctx, l, _dp(eps), _dp(O), _dp(sc)))
    return eps, O, float(sc[0])


def wpcd_build_p(ctx, precision=WPCD_FP64):
    n = ctypes.c_int64()
    _check(ctx, lib().wpcd_build_p(ctx, precision, ctypes.byref(n)))
    return n.value


def wpcd_build_p_noalloc(ctx, precision, row_ptr_dev, col_dev, val_dev, cap_nnz):
    """P0 into caller device buffers (integer device addresses), no
    allocation; returns (status, nnz) without raising, so a caller can
    re-size on WPCD_E_INVALID with nnz set."""
    n = ctypes.c_int64(-1)
    st = lib().wpcd_build_p_noalloc(ctx, precision, ctypes.c_void_p(row_ptr_dev),
                                    ctypes.c_void_p(col_dev), ctypes.c_void_p(val_dev),
                                    cap_nnz, ctypes.byref(n))
    return st, n.value


def wpcd_get_p(ctx, n_cells, nnz, n_ch=1, values=True):
    row_ptr = np.zeros(n_cells + 1, dtype=np.int64)
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros(nnz * n_ch * n_ch) if values else None
    _check(ctx, lib().wpcd_get_p(ctx, row_ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(val)))
    if values:
        val = val.reshape(nnz, n_ch, n_ch)
    return row_ptr, col, val


def wpcd_build_reduced(red, full, n_major, r_p, r_q, precision=WPCD_FP64):
    """Feshbach reduction: red becomes the reduced system of full (channels
    [0, n_major) major on full's lattice, the rest on the lattice coarsened
    by r_p x r_q); returns the number of stored entries of its P0."""
    n = ctypes.c_int64(0)
    _check(red, lib().wpcd_build_reduced(red, full, n_major, r_p, r_q, precision,
                                         ctypes.byref(n)))
    return n.value


def _opts(max_iter=0, krylov_dim=0, tol=0.0, want_breakup=False, warm_start=WPCD_WARM_NONE,
          x0=None, err_est=False, resolvent=0, fallback_tol=0.0):
    wb = int(want_breakup) if not isinstance(want_breakup, bool) else (1 if want_breakup else 0)
    return wpcd_solve_opts(max_iter, krylov_dim, tol, wb, warm_start, _dp(x0),
                           1 if err_est else 0, resolvent, fallback_tol)


def wpcd_solve(ctx, energies, precision=WPCD_FP64, max_iter=0, krylov_dim=0, tol=0.0,
               want_breakup=False, n_p=0, n_ch=1, warm_start=WPCD_WARM_NONE, x0=None,
               err_est=False, resolvent=0, fallback_tol=0.0):
    """want_breakup: False, True / WPCD_BREAKUP_ELEMENTS or WPCD_BREAKUP_DIST
    (returns the rows per energy beside the results); resolvent: a
    WPCD_RESOLVENT_* value; x0 (warm_start=WPCD_WARM_GIVEN): complex array
    [n_E][M]; fallback_tol > 0: mixed-tier energies that did not converge or
    whose error estimate exceeds it are solved again in FP64."""
    E = np.ascontiguousarray(energies, dtype=np.float64)
    out = (wpcd_energy_result * max(1, E.size))()
    x0r = None
    if x0 is not None:
        x0c = np.ascontiguousarray(x0, dtype=np.complex128)
        if x0c.ndim != 2 or x0c.shape[0] != E.size:
            raise ValueError("x0 must be [n_E][M] complex")
        x0r = x0c.view(np.float64).reshape(-1)
    opts = _opts(max_iter, krylov_dim, tol, want_breakup, warm_start, x0r, err_est, resolvent,
                 fallback_tol)
    br = np.zeros(E.size * max(1, n_p) * n_ch * 5) if want_breakup else None
    _check(ctx, lib().wpcd_solve(ctx, _dp(E), E.size, precision, ctypes.byref(opts), out,
                                 _dp(br)))
    res = [out[k] for k in range(E.size)]
    if want_breakup:
        brs = []
        for k in range(E.size):
            rows = br.reshape(E.size, -1, 5)[k, :res[k].n_open]
            brs.append(rows.copy())
        return res, brs
    return res


def wpcd_model_fill(ctx, kind, mode, M, K, alpha=1.0, seed=0, precision=WPCD_FP64, cap=None):
    """Model matrix fill (kind 0 trig, 1 Gauss; mode 0 dense, 1 filtered, 2
    selected).  Returns (dense M x M array or (idx, val), GPU ms)."""
    n = ctypes.c_int64()
    ms = np.zeros(1)
    if mode != 2:
        out = np.zeros(M * M)
        _check(ctx, lib().wpcd_model_fill(ctx, kind, mode, M, K, alpha, seed, precision, _dp(out),
                                          None, None, 0, ctypes.byref(n), _dp(ms)))
        return out.reshape(M, M), float(ms[0])
    if cap is None:   # first call counts
        lib().wpcd_model_fill(ctx, kind, mode, M, K, alpha, seed, precision, None, None, None, 0,
                              ctypes.byref(n), _dp(ms))
        cap = n.value
    idx = np.zeros(max(cap, 1), dtype=np.int64)
    val = np.zeros(max(cap, 1))
    _check(ctx, lib().wpcd_model_fill(ctx, kind, mode, M, K, alpha, seed, precision, None,
                                      idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(val),
                                      cap, ctypes.byref(n), _dp(ms)))
    return (idx[:n.value], val[:n.value]), float(ms[0])


def wpcd_bound_state(ctx, e_lo, e_hi):
    e3 = ctypes.c_double()
    _check(ctx, lib().wpcd_bound_state(ctx, float(e_lo), float(e_hi), ctypes.byref(e3)))
    return e3.value


def wpcd_save_p(ctx, path):
    _check(ctx, lib().wpcd_save_p(ctx, os.fsencode(path)))


def wpcd_load_p(ctx, path):
    n = ctypes.c_int64()
    _check(ctx, lib().wpcd_load_p(ctx, os.fsencode(path), ctypes.byref(n)))
    return n.value


def wpcd_solve_dev(ctx, E_dev_ptr, n_E, out_dev_ptr, precision=WPCD_FP64, **kw):
    """Energies and results in device memory (raw device pointers)."""
    opts = _opts(**kw)
    _check(ctx, lib().wpcd_solve_dev(ctx, ctypes.c_void_p(E_dev_ptr), n_E, precision,
                                     ctypes.byref(opts), ctypes.c_void_p(out_dev_ptr)))


def wpcd_sweep(ctx, energies, batch, precision=WPCD_FP64, journal=None, max_batches=0,
               max_iter=0, krylov_dim=0, tol=0.0, warm_start=WPCD_WARM_NONE, err_est=False,
               resolvent=0, fallback_tol=0.0):
    """Energy sweep in batches, resumable through the journal file (None:
    no journal).  Returns (results, n_done, n_resumed): results[k] for
    every energy, valid for k < n_done; n_resumed were read back from the
    journal."""
    E = np.ascontiguousarray(energies, dtype=np.float64)
    out = (wpcd_energy_result * max(1, E.size))()
    opts = _opts(max_iter, krylov_dim, tol, False, warm_start, None, err_est, resolvent,
                 fallback_tol)
    n_done, n_res = ctypes.c_int32(), ctypes.c_int32()
    _check(ctx, lib().wpcd_sweep(ctx, _dp(E), E.size, int(batch), precision, ctypes.byref(opts),
                                 None if journal is None else os.fsencode(journal),
                                 int(max_batches), out, ctypes.byref(n_done), ctypes.byref(n_res)))
    return [out[k] for k in range(E.size)], n_done.value, n_res.value


def wpcd_solve_multi(ctxs, energies, precision=WPCD_FP64, max_iter=0, krylov_dim=0, tol=0.0):
    """Solve several systems at once: ctxs[i] (handles) at energies[i]."""
    n = len(ctxs)
    Es = [np.ascontiguousarray(e, dtype=np.float64) for e in energies]
    outs = [(wpcd_energy_result * max(1, e.size))() for e in Es]
    H = (ctypes.c_void_p * n)(*[c.value if isinstance(c, ctypes.c_void_p) else c for c in ctxs])
    dp = ctypes.POINTER(ctypes.c_double)
    EP = (dp * n)(*[_dp(e) for e in Es])
    NE = (ctypes.c_int32 * n)(*[e.size for e in Es])
    OP = (ctypes.POINTER(wpcd_energy_result) * n)(
        *[ctypes.cast(o, ctypes.POINTER(wpcd_energy_result)) for o in outs])
    st = (ctypes.c_int * n)()
    opts = _opts(max_iter, krylov_dim, tol)
    rc = lib().wpcd_solve_multi(H, n, EP, NE, precision, ctypes.byref(opts), OP, st)
    if rc != WPCD_OK:
        bad = [i for i in range(n) if st[i] != WPCD_OK]
        msg = lib().wpcd_last_error(H[bad[0]]).decode() if bad else ""
        raise WpcdError(rc, msg)
    return [[outs[i][k] for k in range(Es[i].size)] for i in range(n)]


def wpcd_set_multipliers(ctx, mult):
    m = np.ascontiguousarray(mult, dtype=np.float64)
    _check(ctx, lib().wpcd_set_multipliers(ctx, _dp(m), m.size))


def wpcd_learn_train(ctx, mult, energies, precision=WPCD_FP64, n_basis=32, hidden=256,
                     epochs=400, batch=64, lr=2e-3, seed=1508074410, solve_opts=None):
    """mult: [n_var][n_mult]; energies: [n_var][n_E].  Returns the report as a dict."""
    m = np.ascontiguousarray(mult, dtype=np.float64)
    E = np.ascontiguousarray(energies, dtype=np.float64)
    if m.ndim != 2 or E.ndim != 2 or m.shape[0] != E.shape[0]:
        raise ValueError("mult [n_var][n_mult] and energies [n_var][n_E] expected")
    so = _opts(**(solve_opts or {}))
    d = wpcd_learn_desc(m.shape[0], m.shape[1], _dp(m), E.shape[1], _dp(E), precision, n_basis,
                        hidden, epochs, batch, lr, seed, ctypes.pointer(so))
    r = wpcd_learn_report()
    _check(ctx, lib().wpcd_learn_train(ctx, ctypes.byref(d), ctypes.byref(r)))
    return {f: getattr(r, f) for f, _ in r._fields_}


def wpcd_mlp_eval(ctx, n_in, n_hidden, n_out, params, X, T=None, want_grad=True):
    """One forward/backward of the network kernels; returns (Y, grad, loss)."""
    fp = ctypes.POINTER(ctypes.c_float)
    P = np.ascontiguousarray(params, dtype=np.float32)
    Xa = np.ascontiguousarray(X, dtype=np.float32)
    B = Xa.shape[0]
    Ta = None if T is None else np.ascontiguousarray(T, dtype=np.float32)
    Y = np.zeros((B, n_out), dtype=np.float32)
    G = np.zeros(P.size, dtype=np.float32) if (Ta is not None and want_grad) else None
    loss = np.zeros(1) if Ta is not None else None

    def f(a):
        return None if a is None else a.ctypes.data_as(fp)
    _check(ctx, lib().wpcd_mlp_eval(ctx, n_in, n_hidden, n_out, f(P), B, f(Xa), f(Ta), f(Y), f(G),
                                    _dp(loss)))
    return Y, G, (None if loss is None else float(loss[0]))


def wpcd_set_autotune(ctx, mode=WPCD_TUNE_MEASURE):
    _check(ctx, lib().wpcd_set_autotune(ctx, int(mode)))


def wpcd_get_autotune(ctx):
    arr = (wpcd_tune_entry * 64)()
    n = ctypes.c_int32()
    _check(ctx, lib().wpcd_get_autotune(ctx, arr, 64, ctypes.byref(n)))
    return [dict(name=arr[k].name.decode(), key=arr[k].key.decode(), choice=arr[k].choice,
                 n_candidates=arr[k].n_candidates, us=arr[k].us) for k in range(min(n.value, 64))]


def wpcd_set_graphs(ctx, enable=True):
    _check(ctx, lib().wpcd_set_graphs(ctx, 1 if enable else 0))


def wpcd_set_timing(ctx, groups=WPCD_TIME_ALL):
    _check(ctx, lib().wpcd_set_timing(ctx, int(groups)))


def wpcd_get_timing(ctx):
    arr = (wpcd_kernel_time * 64)()
    n = ctypes.c_int32()
    _check(ctx, lib().wpcd_get_timing(ctx, arr, 64, ctypes.byref(n)))
    return {arr[k].name.decode(): (arr[k].total_ms, arr[k].launches) for k in range(min(n.value, 64))}


def wpcd_reset_timing(ctx):
    _check(ctx, lib().wpcd_reset_timing(ctx))


def wpcd_synchronize(ctx):
    _check(ctx, lib().wpcd_synchronize(ctx))


def wpcd_last_error(ctx):
    return lib().wpcd_last_error(ctx).decode()


def wpcd_destroy(ctx):
    if ctx:
        lib().wpcd_destroy(ctx)


class Context:
    """Owns one wpcd_ctx; thin wrapper over the ABI functions above."""

    def __init__(self, device: int = 0, stream: int | None = None):
        self.h = wpcd_create(device, stream)
        self.n_p = self.n_q = self.n_ch = 0
        self.nnz = 0
        self.red_rows = 0   # reduced cells of a reduced system (0: not reduced)

    def build_basis(self, n_p, n_q, p_max=10.0, q_max=10.0, n_gauss_q=8, n_gauss_x=16,
                    channels=((0, 0),), L=0, potential=None, p_edges=None, q_edges=None):
        wpcd_build_basis(self.h, n_p, n_q, p_max, q_max, n_gauss_q, n_gauss_x, channels, L,
                         potential, p_edges, q_edges)
        self.n_p, self.n_q, self.n_ch = n_p, n_q, len(channels)
        self.red_rows = 0

    def build_basis_nucleons(self, n_p, n_q, p_max=10.0, q_max=10.0, n_gauss_q=8, n_gauss_x=16,
                             two_S=1, channels=((1, 0), (0, 1)), potential=None, mult=None,
                             p_edges=None, q_edges=None):
        wpcd_build_basis_nucleons(self.h, n_p, n_q, p_max, q_max, n_gauss_q, n_gauss_x, two_S,
                                  channels, potential, mult, p_edges, q_edges)
        self.n_p, self.n_q, self.n_ch = n_p, n_q, len(channels)
        self.red_rows = 0

    def set_potential(self, potential):
        wpcd_set_potential(self.h, potential)

    def pair_spectrum(self, l=0, want_O=True):
        return wpcd_pair_spectrum(self.h, l, self.n_p, want_O)

    def build_p(self, precision=WPCD_FP64):
        self.nnz = wpcd_build_p(self.h, precision)
        return self.nnz

    def build_reduced(self, full, n_major, r_p, r_q, precision=WPCD_FP64):
        """This context becomes the Feshbach-reduced system of `full` (a
        Context with basis, potential and P0)."""
        self.nnz = wpcd_build_reduced(self.h, full.h, n_major, r_p, r_q, precision)
        self.n_p, self.n_q, self.n_ch = full.n_p, full.n_q, full.n_ch
        self.red_rows = (n_major * full.n_p * full.n_q +
                         (full.n_ch - n_major) * (full.n_p // r_p) * (full.n_q // r_q))
        return self.nnz

    def get_p(self, values=True):
        if self.red_rows:
            rp, col, val = wpcd_get_p(self.h, self.red_rows, self.nnz, 1, values)
            return rp, col, (val.reshape(-1) if values else None)
        return wpcd_get_p(self.h, self.n_p * self.n_q, self.nnz, self.n_ch, values)

    def basis_rows(self):
        """M, the rows of the channel basis (a reduced system: its major
        and minor parts together)."""
        return self.red_rows if self.red_rows else self.n_ch * self.n_q * self.n_p

    def solve(self, energies, precision=WPCD_FP64, **kw):
        x0 = kw.get("x0")
        if x0 is not None and np.shape(x0)[-1] != self.basis_rows():
            raise ValueError(f"x0 rows {np.shape(x0)[-1]} != the basis' {self.basis_rows()}")
        return wpcd_solve(self.h, energies, precision, n_p=self.n_p, n_ch=self.n_ch, **kw)

    def sweep(self, energies, batch, precision=WPCD_FP64, journal=None, max_batches=0, **kw):
        return wpcd_sweep(self.h, energies, batch, precision, journal, max_batches, **kw)

    def bound_state(self, e_lo, e_hi):
        return wpcd_bound_state(self.h, e_lo, e_hi)

    def model_fill(self, kind, mode, M, K, alpha=1.0, seed=0, precision=WPCD_FP64, cap=None):
        return wpcd_model_fill(self.h, kind, mode, M, K, alpha, seed, precision, cap)

    def save_p(self, path):
        wpcd_save_p(self.h, path)

    def load_p(self, path):
        self.nnz = wpcd_load_p(self.h, path)
        return self.nnz

    def set_multipliers(self, mult):
        wpcd_set_multipliers(self.h, mult)

    def learn_train(self, mult, energies, **kw):
        return wpcd_learn_train(self.h, mult, energies, **kw)

    def mlp_eval(self, n_in, n_hidden, n_out, params, X, T=None, want_grad=True):
        return wpcd_mlp_eval(self.h, n_in, n_hidden, n_out, params, X, T, want_grad)

    def set_autotune(self, mode=WPCD_TUNE_MEASURE):
        wpcd_set_autotune(self.h, mode)

    def autotune(self):
        return wpcd_get_autotune(self.h)

    def set_graphs(self, enable=True):
        wpcd_set_graphs(self.h, enable)

    def set_timing(self, groups=WPCD_TIME_ALL):
        wpcd_set_timing(self.h, groups)

    def timing(self):
        return wpcd_get_timing(self.h)

    def reset_timing(self):
        wpcd_reset_timing(self.h)

    def synchronize(self):
        wpcd_synchronize(self.h)

    def close(self):
        if self.h:
            wpcd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
