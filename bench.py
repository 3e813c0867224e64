#!/usr/bin/env python3
"""Benchmark of the WPCD hot path on one MI355X.

Workload (the 150 x 150 s-wave configuration): three identical spinless
bosons, two-range Yukawa-sum pair potential with ranges 1 and 2 and a common
strength fitted once (at setup) so the lowest pair level is -0.1 in the
150-packet basis; 150 p-bins x 150 q-bins, Chebyshev-spaced edges to 10,
8 Gauss points per q bin, 20 on the cosine interval; 8 energies spanning
below and above breakup.

One step = the whole hot path: pair potential + FP64 diagonalisation,
pre-selection + P0 elements (FP32 with compensated sums), resolvent + the
batched GMRES solve at the 8 energies + amplitudes.  Inputs are synthetic
and resident on the GPU when the timed region starts.

Beside the timed steps: the solve per energy in the mixed tier, in the
mixed tier with the learned warm start (trained at setup on 16 potential
variants x 32 energies drawn with splitmix64: strength multipliers
U[0.8, 1.2], energies U[-0.05, 2.0]), in the refine and BF16 tiers and in
FP64, with iterations and the amplitude errors against the FP64 solve; the
oracle's P build on all host threads (cpu_baseline) and on one
(cpu_baseline_1thread, a sample of every 8th cell row).

Prints one JSON line.  value = P-matrix elements (selected cell pairs) per
second of P-build wall time (pre-selection + elements); the whole-step time
and the solve time per energy are reported beside it.
"""
import argparse
import json
import math
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))
from inputs import SEED, learn_draws  # noqa: E402  (seeded draws only)

N = 150
NGQ, NGX = 8, 20
RANGES = (1.0, 2.0)
ENERGIES = (-0.08, -0.05, -0.02, 0.05, 0.2, 0.5, 1.0, 2.0)
LEARN_VARIANTS, LEARN_ENERGIES = 16, 32

# HBM bytes per launch of the roofline kernel (FP32 P0 elements, this
# workload) from two rocprofv3 counter runs, FETCH_SIZE and WRITE_SIZE, each
# scaled by the counter's reading of a plain device copy of known size
# (factors 2.0 and 1.0); valid only for the element-kernel source they were
# taken on (sha256 prefix of csrc/k_p0.hip), reported as null otherwise.
P0_ELEM_F32_TRAFFIC = {"bytes": 5.2080e+07, "k_p0_sha256": "60a4f52ddfd1e805"}

# MI355X published peaks used for the roofline fractions
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def measured_traffic():
    import hashlib
    src = os.path.join(ROOT, "paper_1508_07441_amd", "csrc", "k_p0.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    return P0_ELEM_F32_TRAFFIC["bytes"] if h == P0_ELEM_F32_TRAFFIC["k_p0_sha256"] else None


def algorithmic_flops_per_element(ngq, ngx):
    """Inner cosine rule per (q, q') Gauss pair and node: s = h u_c (1 mul),
    t = t0 + s, u = u0 + s (2 add), t*u (1 mul), rsqrt (1), w*r accumulated
    (1 fma = 2) -> 7 flops; the per-pair limits (~20 flops) and weights
    (3 flops) are added once per pair."""
    return ngq * ngq * (7 * ngx + 23)


def cpu_baseline(sample_stride, threads):
    """The oracle (as it stands) on a bounded sample of the same workload:
    every sample_stride-th cell row of the 150 x 150 grid, brute-force
    pre-selection over all columns plus the FP64 elements of those rows."""
    import numpy as np

    import oracle.wpcd as O
    os.environ.setdefault("OMP_NUM_THREADS", str(threads))
    p = O.cheb_edges(N, 10.0)
    rows = np.arange(0, N * N, sample_stride, dtype=np.int64)
    t0 = time.perf_counter()
    ptr, col = O.preselect(p, p.copy(), rows)
    rr = np.repeat(rows, np.diff(ptr))
    O.p0_pairs(p, p.copy(), NGQ, NGX, 0, [(0, 0)], rr, col)
    dt = time.perf_counter() - t0
    n = int(ptr[-1])
    return {"value": n / dt, "unit": "P-matrix elements/s", "cores": threads, "kind": "oracle",
            "sample": f"every {sample_stride}th of the {N*N} cell rows ({rows.size} rows, {n} "
                      f"cell pairs): brute-force pre-selection + FP64 elements, {dt:.1f} s"}


def cpu_solve_baseline(threads):
    """The oracle's FP64 GMRES (same algorithm class as the GPU solve:
    restarted GMRES on the factored kernel with the sparse P0) on the same
    150 x 150 system at the 8 energies, one after another."""
    import oracle.wpcd as O
    os.environ.setdefault("OMP_NUM_THREADS", str(threads))
    p = O.cheb_edges(N, 10.0)
    s = O.fit_strength(p, RANGES, -0.1)
    sysm = O.build_system(p, p.copy(), 0, [(0, 0)], NGQ, NGX,
                          O.Potential("yukawa", (-s, -s), RANGES))
    t0 = time.perf_counter()
    for E in ENERGIES:
        O.solve_gmres(sysm, E)
    dt = time.perf_counter() - t0
    return {"value": dt / len(ENERGIES), "unit": "s/energy", "cores": threads, "kind": "oracle",
            "sample": f"the {len(ENERGIES)} energies of the workload, FP64 GMRES to 1e-13, "
                      f"{dt:.1f} s"}


def cpu_baseline_one_thread(sample_stride):
    """cpu_baseline with OMP_NUM_THREADS=1, in a child process of this script
    (called before any GPU use, so the child is started from a process that
    has not initialised the GPU)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-only",
                        str(sample_stride)], env=env, capture_output=True, text=True,
                       timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def copy_calibration(nbytes):
    """One device-to-device copy of nbytes by the HIP runtime's copy kernel:
    a kernel of known traffic (nbytes read, nbytes written) for scaling the
    HBM byte counters."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(a), ctypes.c_size_t(nbytes)) == 0
    assert hip.hipMalloc(ctypes.byref(b), ctypes.c_size_t(nbytes)) == 0
    assert hip.hipMemset(a, 1, ctypes.c_size_t(nbytes)) == 0
    assert hip.hipMemcpy(b, a, ctypes.c_size_t(nbytes), 3) == 0   # device to device
    assert hip.hipDeviceSynchronize() == 0
    hip.hipFree(a)
    hip.hipFree(b)
    return {"read": nbytes, "write": nbytes}


def torch_copy_calibration(nbytes):
    """One device-to-device copy of nbytes by torch's elementwise copy kernel
    (ordinary vector loads and stores): a second plain copy kernel of known
    traffic for the byte counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    return {"read": nbytes, "write": nbytes}


def active_pair_fraction(p, q, ngq, rows, cols, stride=64):
    """Fraction of the (q, q') Gauss pairs of the selected cell pairs whose
    clipped cosine interval is not empty (the integrand is evaluated only
    there), on every stride-th nonzero: the same limit expressions as the
    element quadrature, in numpy."""
    import numpy as np
    x, w = np.polynomial.legendre.leggauss(ngq)
    r, c = rows[::stride], cols[::stride]
    npb = p.size - 1
    i, j, i2, j2 = r % npb, r // npb, c % npb, c // npb
    qa = 0.5 * (q[j][:, None] + q[j + 1][:, None]) + 0.5 * (q[j + 1] - q[j])[:, None] * x[None, :]
    qb = 0.5 * (q[j2][:, None] + q[j2 + 1][:, None]) + 0.5 * (q[j2 + 1] - q[j2])[:, None] * x[None, :]
    qa, qb = qa[:, :, None], qb[:, None, :]
    D = 0.75 * (qa - qb) * (qa + qb)
    tlo, thi = (qb - 0.5 * qa) ** 2, (qb + 0.5 * qa) ** 2
    P2 = p * p
    pl1, ph1 = P2[i][:, None, None], P2[i + 1][:, None, None]
    pl2, ph2 = P2[i2][:, None, None], P2[i2 + 1][:, None, None]
    lo = np.maximum(np.maximum(tlo, pl1), pl2 - D)
    hi = np.minimum(np.minimum(thi, ph1), ph2 - D)
    return float(np.mean(hi > lo)), int(r.size)


def solve_kernel_rates(P, ctx, prec, energies, nnz, n, nch):
    """HIP-event times of the solve's kernels in one batched solve (eager
    launches, the library's stream) and what they move or compute per
    launch: the P0 SpMM (P0 stream: values + columns + row pointers read
    once for all batched energies; x gather: one panel row of 2 n_E doubles
    per nonzero and column channel, from L2 / MALL) and the block products
    (2 N^2 N_q n_ch 2 n_E flops each)."""
    ctx.set_timing(P.WPCD_TIME_SOLVE)
    ctx.reset_timing()
    ctx.solve(energies, prec)
    ctx.synchronize()
    tim = ctx.timing()
    ctx.set_timing(0)
    W = 2 * len(energies)
    vsize = 8 if prec == P.WPCD_FP64 else 4
    sp_ms, sp_n = tim["spmm"]
    t_sp = sp_ms / sp_n / 1e3
    p0_bytes = nnz * (nch * nch * vsize + 4) + 8 * (n * n + 1)
    gather = nnz * nch * W * 8
    bl_ms = tim["apply_vt"][0] + tim["apply_o"][0]
    bl_n = tim["apply_vt"][1] + tim["apply_o"][1]
    t_bl = bl_ms / bl_n / 1e3
    flops = 2.0 * n * n * n * nch * W
    return {"spmm": {"us_per_launch": 1e6 * t_sp, "launches": sp_n,
                     "p0_stream_bytes": p0_bytes, "p0_stream_GBps": p0_bytes / t_sp / 1e9,
                     "p0_stream_frac_hbm": p0_bytes / t_sp / 1e9 / PEAK_HBM_GBS,
                     "x_gather_bytes": gather, "x_gather_GBps": gather / t_sp / 1e9},
            "block_product": {"us_per_launch": 1e6 * t_bl, "launches": bl_n, "flops": flops,
                              "TFLOPs": flops / t_bl / 1e12,
                              "frac_fp64_peak": flops / t_bl / 1e12 / PEAK_FP64_VECTOR_TFLOPS}}


def preselect_rate(tim, nnz, n_cells, builds):
    """Pre-selection (count + scan + fill) HIP-event time per build against
    its algorithmic bytes: 4 B column per nonzero + 8 B row pointer per
    row."""
    ms = sum(tim.get(k, (0.0, 1))[0] for k in ("preselect_count", "preselect_scan",
                                                "preselect_fill")) / builds
    nbytes = 4 * nnz + 8 * (n_cells + 1)
    return {"us": 1e3 * ms, "bytes": nbytes, "GBps": nbytes / (ms / 1e3) / 1e9,
            "frac_hbm": nbytes / (ms / 1e3) / 1e9 / PEAK_HBM_GBS}


def c3_measure(P):
    """The 270k-basis case beside the main line: L = 2+ channels (0,2), (2,0),
    (2,2), 300 x 300 bins, the same Yukawa sum fitted to -0.1, 8 energies.
    P build (pre-selection + elements) in the mixed tier, and the batched
    solve per energy in the three tiers with their amplitude error against
    the FP64 solve."""
    ctx = P.Context(0)
    ctx.set_autotune(P.WPCD_TUNE_MEASURE)
    fit = dict(kind="yukawa", strength=[-1.0, -1.0], range=list(RANGES), fit_e2=-0.1)
    chans = [(0, 2), (2, 0), (2, 2)]
    ctx.build_basis(300, 300, 10.0, 10.0, NGQ, NGX, channels=chans, L=2, potential=fit)
    ctx.build_p(P.WPCD_MIXED)
    ctx.synchronize()
    t = time.perf_counter()
    nnz = ctx.build_p(P.WPCD_MIXED)
    ctx.synchronize()
    t_build = time.perf_counter() - t
    ctx.set_timing(P.WPCD_TIME_PRESELECT)
    ctx.reset_timing()
    ctx.build_p(P.WPCD_MIXED)
    ctx.synchronize()
    presel = preselect_rate(ctx.timing(), nnz, 300 * 300, 1)
    ctx.set_timing(0)

    def solve(prec):
        ctx.solve(ENERGIES, prec)            # tune + capture
        best, res = 1e30, None
        for _ in range(2):
            a = time.perf_counter()
            res = ctx.solve(ENERGIES, prec)
            best = min(best, time.perf_counter() - a)
        return best / len(ENERGIES), res

    s_mixed, r_mixed = solve(P.WPCD_MIXED)
    rates_mixed = solve_kernel_rates(P, ctx, P.WPCD_MIXED, ENERGIES, nnz, 300, 3)
    s_refine, r_refine = solve(P.WPCD_MIXED_REFINE)
    s_bf16, r_bf16 = solve(P.WPCD_MIXED_BF16)
    ctx.build_p(P.WPCD_FP64)
    s_fp64, r_fp64 = solve(P.WPCD_FP64)
    rates_fp64 = solve_kernel_rates(P, ctx, P.WPCD_FP64, ENERGIES, nnz, 300, 3)
    ok = [k for k, r in enumerate(r_fp64) if r.status == P.WPCD_OK]

    def err(ra):
        return max(abs(complex(ra[k].U_re, ra[k].U_im) - complex(r_fp64[k].U_re, r_fp64[k].U_im))
                   / abs(complex(r_fp64[k].U_re, r_fp64[k].U_im)) for k in ok)
    fesh = feshbach_measure(P, ctx, nnz, r_fp64, {"mixed": s_mixed, "fp64": s_fp64})
    ctx.close()
    return {"feshbach": fesh,
            "workload": "L=2+ channels (0,2),(2,0),(2,2); 300x300 bins; Yukawa sum fitted to "
                        "-0.1; 8 energies", "basis": 3 * 300 * 300, "nnz_cells": nnz,
            "p_build_mixed_ms": 1e3 * t_build, "p_elements_per_s": nnz / t_build,
            "channel_values_per_s": 9 * nnz / t_build,
            "solve_s_per_energy": {"mixed": s_mixed, "mixed_refine": s_refine,
                                   "mixed_bf16": s_bf16, "fp64": s_fp64},
            "iters_per_energy": {"mixed": sum(r.iters for r in r_mixed) / len(r_mixed),
                                 "mixed_refine": sum(r.iters for r in r_refine) / len(r_refine),
                                 "mixed_bf16": sum(r.iters for r in r_bf16) / len(r_bf16),
                                 "fp64": sum(r.iters for r in r_fp64) / len(r_fp64)},
            "max_rel_amp_err_vs_fp64": {"mixed": err(r_mixed), "mixed_refine": err(r_refine),
                                        "mixed_bf16": err(r_bf16)},
            "preselect": presel,
            "solve_kernels": {"mixed": rates_mixed, "fp64": rates_fp64}}


def feshbach_measure(P, full, nnz_full, r_full, s_full):
    """Feshbach reduction (Sec. V.B) of the 270k system: the entrance
    channel (0,2) major on the 300 x 300 lattice, the d-wave channels (2,0)
    and (2,2) minor on the lattice coarsened r x r (r = 2, 3).  Reduction
    build time, size, solve per energy (mixed, FP64) against the unreduced
    solve, and the elastic amplitudes' relative difference from the
    unreduced FP64 ones (the accuracy the reduction gives up)."""
    out = {"workload": "the 270k system (3 channels, 300x300 bins); major (0,2), minor "
                       "(2,0),(2,2) on the lattice coarsened r x r; 8 energies"}
    ok = [k for k, r in enumerate(r_full) if r.status == P.WPCD_OK]
    for r in (2, 3):
        red = P.Context(0)
        red.set_autotune(P.WPCD_TUNE_MEASURE)
        row = {}
        for prec, label in ((P.WPCD_FP64, "fp64"), (P.WPCD_MIXED, "mixed")):
            red.build_reduced(full, 1, r, r, prec)
            red.synchronize()
            t = time.perf_counter()
            nnz = red.build_reduced(full, 1, r, r, prec)
            red.synchronize()
            row[f"build_ms_{label}"] = 1e3 * (time.perf_counter() - t)
            red.solve(ENERGIES, prec)            # tune + capture
            best, res = 1e30, None
            for _ in range(2):
                a = time.perf_counter()
                res = red.solve(ENERGIES, prec)
                best = min(best, time.perf_counter() - a)
            row.setdefault("solve_s_per_energy", {})[label] = best / len(ENERGIES)
            row.setdefault("iters_per_energy", {})[label] = sum(x.iters for x in res) / len(res)
            row.setdefault("speedup_vs_unreduced", {})[label] = s_full[label] / (best / len(ENERGIES))
            if label == "fp64":
                r_red64 = res
                row["max_rel_amp_diff_vs_unreduced_fp64"] = max(
                    abs(complex(res[k].U_re, res[k].U_im) - complex(r_full[k].U_re, r_full[k].U_im))
                    / abs(complex(r_full[k].U_re, r_full[k].U_im)) for k in ok)
            else:
                row["max_rel_amp_err_mixed_vs_fp64"] = max(
                    abs(complex(res[k].U_re, res[k].U_im) - complex(r_red64[k].U_re, r_red64[k].U_im))
                    / abs(complex(r_red64[k].U_re, r_red64[k].U_im)) for k in ok)
                # the reduced SpMM (scalar CSR over the reduced cells, FP32
                # values): P0 stream and x panel rows gathered per application
                red.set_timing(P.WPCD_TIME_SOLVE)
                red.reset_timing()
                red.solve(ENERGIES, prec)
                red.synchronize()
                sp_ms, sp_n = red.timing()["spmm"]
                red.set_timing(0)
                t_sp = sp_ms / sp_n / 1e3
                p0_bytes = nnz * (4 + 4) + 8 * (red.red_rows + 1)
                gather = nnz * 2 * len(ENERGIES) * 8
                row["spmm_mixed"] = {"us_per_launch": 1e6 * t_sp, "p0_stream_bytes": p0_bytes,
                                     "p0_stream_frac_hbm": p0_bytes / t_sp / 1e9 / PEAK_HBM_GBS,
                                     "x_gather_bytes": gather,
                                     "x_gather_GBps": gather / t_sp / 1e9}
        row["basis"] = red.red_rows
        row["entries"] = nnz
        row["entries_unreduced"] = 9 * nnz_full
        red.close()
        out[f"r{r}"] = row
    return out


def c5_measure(P, n_var, n_e, sweep):
    """Learned warm start on the 270k basis: plain mixed solves of n_var x n_e
    (potential variant, energy) pairs train the network (multipliers
    U[0.8, 1.2], energies U[-0.05, 2.0], splitmix64), then a sweep of `sweep`
    energies uniform in [-0.05, 2.0] at the base potential is solved plainly
    and with the warm start: iterations, time and amplitude agreement."""
    ctx = P.Context(0)
    ctx.set_autotune(P.WPCD_TUNE_MEASURE)
    fit = dict(kind="yukawa", strength=[-1.0, -1.0], range=list(RANGES), fit_e2=-0.1)
    ctx.build_basis(300, 300, 10.0, 10.0, NGQ, NGX, channels=[(0, 2), (2, 0), (2, 2)], L=2,
                    potential=fit)
    ctx.build_p(P.WPCD_MIXED)
    mult, e_train = learn_draws(SEED + 5, n_var, 2, n_e, -0.05, 2.0)
    t = time.perf_counter()
    rep = ctx.learn_train(mult, e_train, precision=P.WPCD_MIXED, n_basis=128, hidden=256,
                          epochs=200, batch=128, seed=SEED)
    t_train = time.perf_counter() - t
    E = [-0.05 + 2.05 * k / (sweep - 1) for k in range(sweep)]
    ctx.solve(E[:32], P.WPCD_MIXED)
    ctx.solve(E[:32], P.WPCD_MIXED, warm_start=P.WPCD_WARM_LEARNED)
    t = time.perf_counter()
    plain = ctx.solve(E, P.WPCD_MIXED)
    t_plain = time.perf_counter() - t
    t = time.perf_counter()
    learned = ctx.solve(E, P.WPCD_MIXED, warm_start=P.WPCD_WARM_LEARNED)
    t_learned = time.perf_counter() - t
    # the same sweep through wpcd_sweep with a journal (batches of 32, each
    # flushed to disk), then its replay from the complete journal
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "sweep.wj")
        t = time.perf_counter()
        journaled, n_done, _ = ctx.sweep(E, 32, P.WPCD_MIXED, journal=path)
        t_journaled = time.perf_counter() - t
        t = time.perf_counter()
        _, _, n_replayed = ctx.sweep(E, 32, P.WPCD_MIXED, journal=path)
        t_replay = time.perf_counter() - t
    same = n_done == sweep and all(
        (journaled[k].status, journaled[k].U_re, journaled[k].U_im)
        == (plain[k].status, plain[k].U_re, plain[k].U_im) for k in range(sweep))
    ok = [k for k in range(sweep) if plain[k].status == P.WPCD_OK]
    err = max(abs(complex(learned[k].U_re, learned[k].U_im) - complex(plain[k].U_re, plain[k].U_im))
              / abs(complex(plain[k].U_re, plain[k].U_im)) for k in ok)
    r0 = sorted(learned[k].r0 for k in ok)
    ctx.close()
    return {"workload": f"270k basis (300x300, L=2+ 3 channels); training {n_var} variants x "
                        f"{n_e} energies, sweep of {sweep} energies",
            "train": {k: rep[k] for k in ("n_samples", "plain_iters", "basis_mean_rel_err",
                                          "basis_max_rel_err", "loss_first", "loss_last")},
            "train_s": t_train, "train_solve_s": rep["solve_ms"] / 1e3,
            "sweep_iters": {"plain": sum(plain[k].iters for k in ok),
                            "learned": sum(learned[k].iters for k in ok)},
            "sweep_s_per_energy": {"plain": t_plain / sweep, "learned": t_learned / sweep},
            "learned_initial_residual_median": r0[len(r0) // 2],
            "max_rel_amp_diff_learned_vs_plain": err,
            "journaled_sweep": {"batch": 32, "s_per_energy": t_journaled / sweep,
                                "replay_s": t_replay, "replayed": n_replayed,
                                "same_results_as_solve": same}}


def nucleon_measure(P):
    """Three nucleons in pair s-waves (Sec. III.B eq.(gal) with spin and
    isospin) on the 150 x 150 grid: 3S1 pair potential = the Yukawa sum
    fitted to -0.1 (the deuteron), 1S0 = the same with both strengths x 0.7
    (unbound); doublet (channels 3S1, 1S0) and quartet (3S1).  P build
    (mixed) and the 8-energy solve (mixed, FP64) per energy, elastic phases."""
    ctx = P.Context(0)
    ctx.set_autotune(P.WPCD_TUNE_MEASURE)
    fit = dict(kind="yukawa", strength=[-1.0, -1.0], range=list(RANGES), fit_e2=-0.1)
    out = {"workload": "3N pair s-waves, 150x150 bins, 3S1 Yukawa sum fitted to -0.1, "
                       "1S0 x 0.7; doublet (3S1, 1S0) and quartet (3S1); 8 energies"}
    for name, two_S, chans, mult in (("doublet", 1, [(1, 0), (0, 1)], [[1.0, 1.0], [0.7, 0.7]]),
                                     ("quartet", 3, [(1, 0)], None)):
        ctx.build_basis_nucleons(N, N, 10.0, 10.0, NGQ, NGX, two_S=two_S, channels=chans,
                                 potential=fit, mult=mult)
        nnz = ctx.build_p(P.WPCD_MIXED)
        ctx.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            ctx.build_p(P.WPCD_MIXED)
        ctx.synchronize()
        t_build = (time.perf_counter() - t) / 3
        row = {"n_ch": len(chans), "nnz_cells": nnz, "p_build_mixed_ms": 1e3 * t_build,
               "channel_values_per_s": len(chans) ** 2 * nnz / t_build}
        for prec, label in ((P.WPCD_MIXED, "mixed"), (P.WPCD_FP64, "fp64")):
            if prec == P.WPCD_FP64:
                ctx.build_p(P.WPCD_FP64)
            ctx.solve(ENERGIES, prec)
            best, res = 1e30, None
            for _ in range(3):
                a = time.perf_counter()
                res = ctx.solve(ENERGIES, prec)
                best = min(best, time.perf_counter() - a)
            row[f"solve_s_per_energy_{label}"] = best / len(ENERGIES)
            row[f"iters_per_energy_{label}"] = sum(r.iters for r in res) / len(res)
            if label == "fp64":
                row["delta_deg"] = [math.degrees(r.delta) for r in res]
                row["eta"] = [r.eta for r in res]
        out[name] = row
    ctx.close()
    return out


def model_fill_measure(P):
    """The paper's model matrix fills (Sec. IV.A): dense, and sparse at
    alpha = 0.01 by filtering inside the dense launch or by selecting the
    kept elements first; GPU time of the fill kernels (HIP events), best of
    three."""
    ctx = P.Context(0)
    out = {}
    for name, kind, M, K in (("trig", 0, 4096, 256), ("gauss", 1, 2048, 16)):
        row = {"M": M, "K": K}
        for label, mode, prec, alpha in (("dense_fp64", 0, P.WPCD_FP64, 1.0),
                                         ("dense_fp32", 0, P.WPCD_MIXED, 1.0),
                                         ("filtered_fp32_alpha0.01", 1, P.WPCD_MIXED, 0.01),
                                         ("selected_fp32_alpha0.01", 2, P.WPCD_MIXED, 0.01)):
            best = 1e30
            for _ in range(3):
                _, ms = ctx.model_fill(kind, mode, M, K, alpha=alpha, seed=SEED, precision=prec)
                best = min(best, ms)
            row[label + "_ms"] = best
        row["elements_per_s_dense_fp32"] = M * M / (row["dense_fp32_ms"] / 1e3)
        row["selected_over_filtered_speedup"] = (row["filtered_fp32_alpha0.01_ms"]
                                                 / row["selected_fp32_alpha0.01_ms"])
        out[name] = row
    ctx.close()
    return out


C4_SYSTEMS = ((100, 1), (150, 2), (200, 3), (250, 4), (300, 5), (400, 1))
C4_L2_CHANNELS = ((0, 2), (2, 0), (2, 2), (2, 4), (4, 2))


def c4_measure(P, n_var, n_e):
    """Uneven systems: (N, n_ch) in C4_SYSTEMS (n_ch = 1: the s-wave L = 0+
    channel; n_ch > 1: the first n_ch L = 2+ channels), the Yukawa sum fitted
    to -0.1 on each grid, n_var potential variants (strength multipliers
    U[0.8, 1.2], splitmix64) x n_e energies -0.05 .. 2.0.  Mixed tier.  The
    systems are solved together (wpcd_solve_multi, one stream each) and one
    after another; (E, variant) pairs at or below the pair threshold are
    reported as such and not counted."""
    fit_t = dict(kind="yukawa", strength=[-1.0, -1.0], range=list(RANGES), fit_e2=-0.1)
    ctxs, build_s = [], []
    for n, nch in C4_SYSTEMS:
        c = P.Context(0)
        c.set_autotune(P.WPCD_TUNE_MEASURE)
        if nch == 1:
            c.build_basis(n, n, 10.0, 10.0, NGQ, NGX, potential=fit_t)
        else:
            c.build_basis(n, n, 10.0, 10.0, NGQ, NGX, channels=list(C4_L2_CHANNELS[:nch]), L=2,
                          potential=fit_t)
        t = time.perf_counter()
        c.build_p(P.WPCD_MIXED)
        c.synchronize()
        build_s.append(time.perf_counter() - t)
        ctxs.append(c)
    mult, _ = learn_draws(SEED + 9, n_var, 2, 0, 0.0, 1.0)
    E = [-0.05 + 2.05 * k / (n_e - 1) for k in range(n_e)]
    # first pass (untimed): launch-shape tuning and graph capture for every
    # batch shape the timed runs meet, alone and in lockstep (a variant can
    # push an energy below its pair threshold, which changes the batch width)
    for v in range(n_var):
        for c in ctxs:
            c.set_multipliers(mult[v])
        P.wpcd_solve_multi([c.h for c in ctxs], [E] * len(ctxs), P.WPCD_MIXED)
        for c in ctxs:
            c.solve(E, P.WPCD_MIXED)
    t_multi = t_seq = 0.0
    ok = 0
    for v in range(n_var):
        for c in ctxs:
            c.set_multipliers(mult[v])
        t = time.perf_counter()
        res = P.wpcd_solve_multi([c.h for c in ctxs], [E] * len(ctxs), P.WPCD_MIXED)
        t_multi += time.perf_counter() - t
        ok += sum(r.status == P.WPCD_OK for rs in res for r in rs)
        t = time.perf_counter()
        for c in ctxs:
            c.solve(E, P.WPCD_MIXED)
        t_seq += time.perf_counter() - t
    for c in ctxs:
        c.close()
    return {"workload": f"{len(C4_SYSTEMS)} systems (N, n_ch) {list(C4_SYSTEMS)}; {n_var} potential "
                        f"variants x {n_e} energies each; mixed tier",
            "p_build_s": dict(zip([f"{n}x{n}/{nch}ch" for n, nch in C4_SYSTEMS], build_s)),
            "solved": ok, "together_s": t_multi, "one_by_one_s": t_seq,
            "solves_per_s_together": ok / t_multi, "solves_per_s_one_by_one": ok / t_seq}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-stride", type=int, default=1)
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--no-learn", action="store_true",
                    help="skip the learned-warm-start leg (short runs under a profiler)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="after the run, one device-to-device copy of this many MiB by the "
                         "HIP runtime's copy kernel, to calibrate HBM byte counters")
    ap.add_argument("--cpu-only", type=int, default=0,
                    help="no GPU: only the oracle baseline on every N-th cell row with this "
                         "process's OMP_NUM_THREADS; prints its JSON (used for the 1-thread "
                         "figure, run as a child before the GPU is touched)")
    ap.add_argument("--c4", type=str, default="6,64",
                    help="uneven systems solved together: VARIANTS,ENERGIES ('' to skip)")
    ap.add_argument("--c5", type=str, default="64,64,256",
                    help="learned warm start on the 270k basis: VARIANTS,ENERGIES,SWEEP "
                         "('' to skip)")
    args = ap.parse_args()
    if args.cpu_only:
        print(json.dumps(cpu_baseline(args.cpu_only, int(os.environ.get("OMP_NUM_THREADS", "1")))),
              flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    # the oracle on one host thread (the paper's speed-up convention), in a
    # child process started before this process touches the GPU
    cpu1 = None
    if rank == 0 and not args.no_cpu_baseline:
        cpu1 = cpu_baseline_one_thread(8 * args.cpu_sample_stride)

    import paper_1508_07441_amd as P

    ctx = P.Context(0)
    # setup (untimed): fit the common strength once
    fit = dict(kind="yukawa", strength=[-1.0, -1.0], range=list(RANGES), fit_e2=-0.1)
    ctx.build_basis(N, N, 10.0, 10.0, NGQ, NGX, potential=fit)
    _, _, scale = ctx.pair_spectrum(0, want_O=False)
    pot = dict(kind="yukawa", strength=[-scale, -scale], range=list(RANGES))

    # launch shapes: time the candidates once per shape (cached in the context)
    ctx.set_autotune(P.WPCD_TUNE_MEASURE)
    pbuild = [0.0]

    def step():
        ctx.build_basis(N, N, 10.0, 10.0, NGQ, NGX, potential=pot)
        t0 = time.perf_counter()
        nnz = ctx.build_p(P.WPCD_MIXED)
        pbuild[0] += time.perf_counter() - t0
        res = ctx.solve(ENERGIES, P.WPCD_MIXED)
        return nnz, res

    for _ in range(args.warmup):
        step()
    ctx.synchronize()
    ctx.set_timing(P.WPCD_TIME_P0)
    ctx.reset_timing()
    pbuild[0] = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nnz, res = step()
    ctx.synchronize()
    t1 = time.perf_counter()
    tim = ctx.timing()
    ctx.set_timing(0)
    wall = t1 - t0

    # pre-selection kernels timed in builds of their own (events only around
    # the element kernel inside the timed steps)
    ctx.build_p(P.WPCD_MIXED)
    ctx.set_timing(P.WPCD_TIME_PRESELECT)
    ctx.reset_timing()
    for _ in range(3):
        ctx.build_p(P.WPCD_MIXED)
    ctx.synchronize()
    presel = preselect_rate(ctx.timing(), nnz, N * N, 3)
    ctx.set_timing(0)

    # solve-only timing (untimed for value): batched 8 energies, mixed and FP64
    def solve_time(prec, reps=3, **kw):
        ts = []
        for _ in range(reps):
            a = time.perf_counter()
            r = ctx.solve(ENERGIES, prec, **kw)
            ts.append(time.perf_counter() - a)
        return min(ts) / len(ENERGIES), r

    s_mixed, r_mixed = solve_time(P.WPCD_MIXED)
    rates_mixed = solve_kernel_rates(P, ctx, P.WPCD_MIXED, ENERGIES, nnz, N, 1)
    # the energy-averaged channel resolvent beside the one at E: elastic
    # phases and inelasticities at the same energies
    solve_time(P.WPCD_MIXED, reps=1, resolvent=P.WPCD_RESOLVENT_AVERAGED)
    s_avg, r_avg = solve_time(P.WPCD_MIXED, resolvent=P.WPCD_RESOLVENT_AVERAGED)
    resolvent_cmp = {
        "energies": list(ENERGIES),
        "delta_deg_at_E": [math.degrees(r.delta) for r in r_mixed],
        "delta_deg_averaged": [math.degrees(r.delta) for r in r_avg],
        "eta_at_E": [r.eta for r in r_mixed], "eta_averaged": [r.eta for r in r_avg],
        "solve_s_per_energy_averaged": s_avg,
        "note": "averaged: channel resolvent eigenvalues averaged over the on-shell energy bin "
                "(histogram amplitudes, flux factor 1/D); mixed tier"}
    # fraction of Gauss pairs with a non-empty cosine interval (sampled)
    import numpy as np
    rp_h, col_h, _ = ctx.get_p(values=False)
    grid = np.array([10.0 * (1.0 - math.cos(math.pi * k / (2 * N))) for k in range(N + 1)])
    grid[0], grid[N] = 0.0, 10.0
    act_frac, act_n = active_pair_fraction(grid, grid, NGQ,
                                           np.repeat(np.arange(N * N), np.diff(rp_h)), col_h)
    solve_time(P.WPCD_MIXED_REFINE, reps=1)     # tune + capture
    s_refine, r_refine = solve_time(P.WPCD_MIXED_REFINE)
    solve_time(P.WPCD_MIXED_BF16, reps=1)
    s_bf16, r_bf16 = solve_time(P.WPCD_MIXED_BF16)
    # learned warm start (mixed): trained on plain mixed solves of potential
    # variants, then the 8 energies at the base potential (a held-out point)
    if not args.no_learn:
        mult, e_train = learn_draws(SEED, LEARN_VARIANTS, 2, LEARN_ENERGIES, -0.05, 2.0)
        t_learn = time.perf_counter()
        rep = ctx.learn_train(mult, e_train, precision=P.WPCD_MIXED, n_basis=64, hidden=256,
                              epochs=300, batch=64, seed=SEED)
        t_learn = time.perf_counter() - t_learn
        s_learned, r_learned = solve_time(P.WPCD_MIXED, warm_start=P.WPCD_WARM_LEARNED)
    else:
        s_learned, r_learned, rep, t_learn = s_mixed, r_mixed, None, 0.0
    # FP64 P-build throughput and FP64 solve beside it
    ctx.build_p(P.WPCD_FP64)          # first FP64 build: launch-shape tuning
    ctx.synchronize()
    ctx.set_timing(P.WPCD_TIME_P0)
    ctx.reset_timing()
    a = time.perf_counter()
    for _ in range(3):
        ctx.build_p(P.WPCD_FP64)
    fp64_build = (time.perf_counter() - a) / 3
    tim64 = ctx.timing()
    ctx.set_timing(0)
    s_fp64, r_fp64 = solve_time(P.WPCD_FP64)
    rates_fp64 = solve_kernel_rates(P, ctx, P.WPCD_FP64, ENERGIES, nnz, N, 1)

    def amp_err(ra):
        return max(abs(complex(x.U_re, x.U_im) - complex(y.U_re, y.U_im)) / abs(complex(y.U_re, y.U_im))
                   for x, y in zip(ra, r_fp64))

    def mean_iters(ra):
        return sum(x.iters for x in ra) / len(ra)

    elem_ms, elem_n = tim.get("p0_elem_f32", (0.0, 1))
    elem_avg_s = elem_ms / max(elem_n, 1) / 1e3
    flops = algorithmic_flops_per_element(NGQ, NGX) * nnz
    achieved = flops / elem_avg_s / 1e12
    e64_ms, e64_n = tim64.get("p0_elem_f64", (0.0, 1))
    out = {
        "metric": "P-matrix elements/s; solve s/energy, mixed+learned vs FP64 at <=1e-6 amp err",
        "value": nnz * args.steps / pbuild[0],
        "unit": "P-matrix elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (P0 elements, compensated sums) + f64 (pair, resolvent, solve)",
        "data": "synthetic",
        "config": {"workload": "s-wave bosons, 2-range Yukawa sum fitted to -0.1; 150x150 bins, "
                               "8x8 q Gauss, 20-pt cosine rule, 8 energies", "nnz_cells": nnz,
                   "basis": N * N, "energies": list(ENERGIES)},
        "solve_s_per_energy": {"mixed": s_mixed, "mixed_learned": s_learned,
                               "mixed_refine": s_refine, "mixed_bf16": s_bf16, "fp64": s_fp64,
                               "mixed_max_rel_amp_err_vs_fp64": amp_err(r_mixed),
                               "mixed_refine_max_rel_amp_err_vs_fp64": amp_err(r_refine),
                               "mixed_bf16_max_rel_amp_err_vs_fp64": amp_err(r_bf16),
                               "mixed_learned_max_rel_amp_err_vs_fp64": amp_err(r_learned),
                               "iters_per_energy": {"mixed": mean_iters(r_mixed),
                                                    "mixed_learned": mean_iters(r_learned),
                                                    "mixed_refine": mean_iters(r_refine),
                                                    "mixed_bf16": mean_iters(r_bf16),
                                                    "fp64": mean_iters(r_fp64)},
                               "learned_initial_residual_median":
                                   sorted(x.r0 for x in r_learned)[len(r_learned) // 2],
                               "fp64_over_mixed_learned": s_fp64 / s_learned},
        "learn": None if rep is None else {
            "train_solves": rep["n_samples"], "basis": 64,
            "basis_mean_rel_err": rep["basis_mean_rel_err"],
            "loss_first": rep["loss_first"], "loss_last": rep["loss_last"], "train_s": t_learn},
        "p_build": {"mixed_ms": 1e3 * pbuild[0] / args.steps, "fp64_ms": 1e3 * fp64_build,
                    "fp64_elements_per_s": nnz / fp64_build,
                    "elem_kernel_f32_ms": 1e3 * elem_avg_s,
                    "elem_kernel_f64_ms": e64_ms / max(e64_n, 1),
                    "preselect_ms": presel["us"] / 1e3, "preselect": presel},
        "solve_kernels": {"mixed": rates_mixed, "fp64": rates_fp64},
        "resolvent_variants": resolvent_cmp,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                     "traffic": measured_traffic(), "kernel": "p0_elem_f32",
                     "flops_per_cell_pair": algorithmic_flops_per_element(NGQ, NGX),
                     "active_pair_frac": act_frac, "active_pair_sample": act_n,
                     "achieved_active": achieved * (23 + 7 * NGX * act_frac) / (23 + 7 * NGX),
                     "note": "achieved counts the cosine rule for all n_q^2 Gauss pairs of every "
                             "cell pair (an upper bound of the useful work); achieved_active "
                             "counts it only for the pairs with a non-empty interval"},
    }
    out["autotune"] = {f'{e["name"]} [{e["key"]}]': e["choice"] for e in ctx.autotune()}
    if not args.no_c3:
        out["c3"] = c3_measure(P)
    out["model_fill"] = model_fill_measure(P)
    out["nucleons"] = nucleon_measure(P)
    if args.c4:
        nv, ne = (int(x) for x in args.c4.split(","))
        out["c4"] = c4_measure(P, nv, ne)
    if args.c5:
        nv, ne, sw = (int(x) for x in args.c5.split(","))
        out["c5"] = c5_measure(P, nv, ne, sw)
    if rank == 0 and not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_stride, threads)
        out["cpu_baseline"]["solve"] = cpu_solve_baseline(threads)
        out["cpu_baseline_1thread"] = cpu1
    ctx.close()
    if args.copy_calib_mb:
        out["copy_calib_bytes"] = copy_calibration(args.copy_calib_mb << 20)
        out["torch_copy_calib_bytes"] = torch_copy_calibration(args.copy_calib_mb << 20)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
