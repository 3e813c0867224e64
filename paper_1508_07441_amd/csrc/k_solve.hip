// Energy-dependent steps (paper Sec. III.C, steps 3-4): channel resolvent
// G1, the factored kernel K = O P0 V~ G1 (eq.(kernel)) applied without
// forming K, and a batched restarted GMRES for the on-shell column of the
// matrix Faddeev equation U = P V1 + P V1 G1 U (eq.(m_pvg)); amplitudes from
// the diagonal element (Sec. III.B).
//
// Vectors over the channel basis are stored [row][energy][re, im] with
// row = (a*nq + j)*np + k, so one row of a batched vector is W = 2 nE
// contiguous doubles: a P0 gather reads one contiguous W-run per nonzero.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <type_traits>

#include "wpcd_internal.h"

namespace wpcd {

struct ChPtrs {
    const double *p[kMaxCh];
};

// ------------------------------------------------------------ resolvent
// G1 on the diagonal of the channel WP basis:
//   G = (1/dq_j) int_{q_j}^{q_j+1} dq / (E - eps*_k - 3/4 q^2 + i0).
// s > 0: 2/(3 qs dq) [ln((qs+q)/|qs-q|)] - i 2 pi/(3 qs dq) [qs in bin]
// s < 0: -4/(3 ks dq) [atan(q/ks)]
// An on-shell momentum within 1e-12 q_max of an edge flags the energy.
__global__ void k_resolvent(const double *__restrict__ q, int np, int nq, int nch, int nE,
                            const double *__restrict__ E, ChPtrs eps, double *__restrict__ G,
                            int32_t *__restrict__ flag) {
    const int64_t M = (int64_t)nch * nq * np;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * nE) return;
    const int e = (int)(idx % nE);
    const int64_t row = idx / nE;
    const int k = (int)(row % np);
    const int j = (int)((row / np) % nq);
    const int a = (int)(row / ((int64_t)np * nq));
    const double s = E[e] - eps.p[a][k];
    const double ql = q[j], qh = q[j + 1], dq = qh - ql;
    const double tol = 1e-12 * q[nq];
    double re = 0.0, im = 0.0;
    if (s > 0.0) {
        const double qs = sqrt(4.0 * s / 3.0);
        if (fabs(qs - ql) < tol || fabs(qs - qh) < tol) {
            flag[e] = 1;
        } else {
            const double fh = log((qs + qh) / fabs(qs - qh));
            const double fl = (ql == 0.0) ? 0.0 : log((qs + ql) / fabs(qs - ql));
            re = 2.0 / (3.0 * qs * dq) * (fh - fl);
            if (ql < qs && qs < qh) im = -2.0 * M_PI / (3.0 * qs * dq);
        }
    } else if (s < 0.0) {
        const double ks = sqrt(-4.0 * s / 3.0);
        re = -4.0 / (3.0 * ks * dq) * (atan(qh / ks) - atan(ql / ks));
    } else {
        flag[e] = 1;
    }
    G[2 * idx] = re;
    G[2 * idx + 1] = im;
}

// Channel resolvent averaged over the on-shell energy interval [E1, E2] of
// each energy (Sec. II.C; width D = E2 - E1):
//   G = (1/(D dq_j)) int_{E1}^{E2} dE int_{q_j}^{q_j+1} dq / (E - eps*_k - 3/4 q^2 + i0)
//     = (F(E2 - eps*_k) - F(E1 - eps*_k)) / (D dq) - i pi L / (D dq),
// F(s) = int ln|s - 3/4 q^2| dq over the bin, L = the length of the bin
// inside the shell E1 < eps*_k + 3/4 q^2 < E2.  With b = sqrt(3)/2:
//   s > 0, a = sqrt(s): [((b q - a)(ln|b q - a| - 1) + (a + b q)(ln(a + b q) - 1)) / b]
//   s < 0, c = sqrt(-s): [q ln(c^2 + b^2 q^2) - 2 q + (2 c / b) atan(b q / c)]
//   s = 0: [2 q (ln(b q) - 1)]
__device__ __forceinline__ double tlogt_m1(double t) {   // t (ln|t| - 1), 0 at t = 0
    return t != 0.0 ? t * (log(fabs(t)) - 1.0) : 0.0;
}

__device__ double log_prim(double s, double q) {
    const double b = 0.86602540378443864676;   // sqrt(3)/2
    if (s > 0.0) {
        const double a = sqrt(s);
        return (tlogt_m1(b * q - a) + tlogt_m1(a + b * q)) / b;
    }
    if (s < 0.0) {
        const double c = sqrt(-s);
        return q * log(-s + 0.75 * q * q) - 2.0 * q + 2.0 * c / b * atan(b * q / c);
    }
    return q > 0.0 ? 2.0 * tlogt_m1(b * q) / b : 0.0;
}

__global__ void k_resolvent_avg(const double *__restrict__ q, int np, int nq, int nch, int nE,
                                const double *__restrict__ ebin, ChPtrs eps,
                                double *__restrict__ G) {
    const int64_t M = (int64_t)nch * nq * np;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * nE) return;
    const int e = (int)(idx % nE);
    const int64_t row = idx / nE;
    const int k = (int)(row % np);
    const int j = (int)((row / np) % nq);
    const int a = (int)(row / ((int64_t)np * nq));
    const double E1 = ebin[2 * e], E2 = ebin[2 * e + 1];
    const double s1 = E1 - eps.p[a][k], s2 = E2 - eps.p[a][k];
    const double ql = q[j], qh = q[j + 1];
    const double w = (E2 - E1) * (qh - ql);
    const double re = ((log_prim(s2, qh) - log_prim(s2, ql)) - (log_prim(s1, qh) - log_prim(s1, ql))) / w;
    double L = 0.0;
    if (s2 > 0.0) {
        const double q1 = s1 > 0.0 ? sqrt(4.0 * s1 / 3.0) : 0.0;
        const double q2 = sqrt(4.0 * s2 / 3.0);
        L = fmax(0.0, fmin(qh, q2) - fmax(ql, q1));
    }
    G[2 * idx] = re;
    G[2 * idx + 1] = -M_PI * L / w;
}

// ------------------------------------------------------- block products
// out[(b, r)][c] = sum_k Mat_b[r][k] y[(b, k)][c],  b = a*nq + j, Mat_b = mats[a]
// y = G (.) in (complex product, USE_G) or in; out = that (SUB false) or
// add - that (SUB true).  Per channel a this is one GEMM
//   C_a[r][(j, c)] = sum_k Mat_a[r][k] Y_a[k][(j, c)]
// over all spectator bins j at once: tiles of TM rows x TN panel columns
// (a panel column is (j, c), c < W), k in steps of 16 staged in LDS, each of
// the 256 threads accumulating (TM/16) x (TN/16) outputs in registers.
// Panels in and out are FP64, or FP32 (TI/TO float) for the inner
// iterations of the mixed tier; the arithmetic is FP64 throughout.
template <bool USE_G, bool SUB, int TM, int TN, class TI, class TO>
__global__ __launch_bounds__(256) void k_block_apply(ChPtrs mats, int n, int nq, int W,
                                                     const TI *__restrict__ in,
                                                     const double *__restrict__ G,
                                                     const double *__restrict__ add,
                                                     TO *__restrict__ out) {
    constexpr int KS = 16, UM = TM / 16, UN = TN / 16;
    __shared__ double sA[KS][TM + 1];
    __shared__ double sB[KS][TN + 1];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int a = blockIdx.z;
    const int row0 = blockIdx.y * TM;
    const int64_t q0 = (int64_t)blockIdx.x * TN;
    const int64_t ncol = (int64_t)nq * W;
    const double *Mt = mats.p[a];
    const int64_t chbase = (int64_t)a * nq * n;   // first channel-basis row of channel a
    double acc[UM][UN];
#pragma unroll
    for (int u = 0; u < UM; ++u)
#pragma unroll
        for (int v = 0; v < UN; ++v) acc[u][v] = 0.0;
    // the panel columns this thread stages are the same for every k step:
    // their (j, c) split (a division by W) is done once
    constexpr int NBL = (KS * TN + 255) / 256;
    int64_t bbase[NBL];   // (chbase + j n) W, or -1 past the panel
    int bc[NBL];
#pragma unroll
    for (int sl = 0; sl < NBL; ++sl) {
        const int idx = t + 256 * sl;
        const int64_t q = q0 + idx % TN;
        bbase[sl] = -1;
        bc[sl] = 0;
        if (idx < KS * TN && q < ncol) {
            const int j = (int)(q / W);
            bc[sl] = (int)(q - (int64_t)j * W);
            bbase[sl] = (chbase + (int64_t)j * n) * W;
        }
    }
    // The loads of k step k0 + KS are issued before the products of step k0
    // (held raw in registers, parked in LDS at the top of the next step), so
    // the global-memory latency of a step overlaps the previous step's FMAs.
    constexpr int NAL = (TM * KS + 255) / 256;
    double ra[NAL];
    double rg[NBL][2], rx[NBL][2];   // raw G and panel entries (USE_G: the pair)
    auto fetch = [&](int k0) {
#pragma unroll
        for (int sl = 0; sl < NAL; ++sl) {
            const int idx = t + 256 * sl;
            const int rr = idx / KS, kk = idx % KS;
            const int r = row0 + rr, k = k0 + kk;
            ra[sl] = (idx < TM * KS && r < n && k < n) ? Mt[(int64_t)r * n + k] : 0.0;
        }
#pragma unroll
        for (int sl = 0; sl < NBL; ++sl) {
            const int idx = t + 256 * sl;
            const int kk = idx / TN;
            const int k = k0 + kk;
            const bool ok = idx < KS * TN && k < n && bbase[sl] >= 0;
            const int64_t o = bbase[sl] + (int64_t)k * W;
            const int c = bc[sl];
            if (USE_G) {
                const int c0 = c & ~1;
                rg[sl][0] = ok ? G[o + c0] : 0.0;
                rg[sl][1] = ok ? G[o + c0 + 1] : 0.0;
                rx[sl][0] = ok ? (double)in[o + c0] : 0.0;
                rx[sl][1] = ok ? (double)in[o + c0 + 1] : 0.0;
            } else {
                rx[sl][0] = ok ? (double)in[o + c] : 0.0;
            }
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < n; k0 += KS) {
        // A tile, transposed: sA[kk][rr] = Mat[row0 + rr][k0 + kk]
#pragma unroll
        for (int sl = 0; sl < NAL; ++sl) {
            const int idx = t + 256 * sl;
            if (idx < TM * KS) sA[idx % KS][idx / KS] = ra[sl];
        }
        // B tile: sB[kk][qq] = Y[k0 + kk][q0 + qq]
#pragma unroll
        for (int sl = 0; sl < NBL; ++sl) {
            const int idx = t + 256 * sl;
            if (idx >= KS * TN) break;
            double v = rx[sl][0];
            if (USE_G) {
                const double gr = rg[sl][0], gi = rg[sl][1], xr = rx[sl][0], xi = rx[sl][1];
                v = (bc[sl] & 1) ? (gr * xi + gi * xr) : (gr * xr - gi * xi);
            }
            sB[idx / TN][idx % TN] = v;
        }
        __syncthreads();
        if (k0 + KS < n) fetch(k0 + KS);
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            double av[UM], bv[UN];
#pragma unroll
            for (int u = 0; u < UM; ++u) av[u] = sA[kk][ty + 16 * u];
#pragma unroll
            for (int v = 0; v < UN; ++v) bv[v] = sB[kk][tx + 16 * v];
#pragma unroll
            for (int u = 0; u < UM; ++u)
#pragma unroll
                for (int v = 0; v < UN; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
        }
        __syncthreads();
    }
    int64_t obase[UN];   // (chbase + j n) W + c of output column v, or -1
#pragma unroll
    for (int v = 0; v < UN; ++v) {
        const int64_t q = q0 + tx + 16 * v;
        obase[v] = -1;
        if (q < ncol) {
            const int j = (int)(q / W);
            obase[v] = (chbase + (int64_t)j * n) * W + (q - (int64_t)j * W);
        }
    }
#pragma unroll
    for (int u = 0; u < UM; ++u) {
        const int r = row0 + ty + 16 * u;
        if (r >= n) continue;
#pragma unroll
        for (int v = 0; v < UN; ++v) {
            if (obase[v] < 0) continue;
            const int64_t gi = obase[v] + (int64_t)r * W;
            out[gi] = (TO)(SUB ? add[gi] - acc[u][v] : acc[u][v]);
        }
    }
}

// Same product on the matrix cores: a 64 x 64 output tile per workgroup, each
// of the 4 wavefronts owning 32 x 32 as 2 x 2 tiles of the 16 x 16 x 4 MFMA
// (v_mfma_f64_16x16x4f64 for MT = double, v_mfma_f32_16x16x4f32 for MT =
// float with FP32 accumulation).  Operand layout of the 16 x 16 x 4 forms:
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; its result item
// r < 4 is D[i][l % 16] with i = 4 (l / 16) + r for the FP32 form and
// i = l / 16 + 4 r for the FP64 form (measured on gfx950).  Tiles staged in
// LDS as in k_block_apply, k in steps of 16.
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

// Operand tag of the BF16 form: v_mfma_f32_16x16x16bf16_1k, FP32
// accumulation; lane l supplies A[l % 16][4 (l / 16) + q] and
// B[4 (l / 16) + q][l % 16] for q < 4, and its result items follow the FP32
// 16 x 16 x 4 form.  Tiles are staged in FP32 and rounded to BF16 (nearest,
// ties to even) as the operands are formed.
struct Bf16 {};

template <class MT>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
    using V = v4d;
    using L = double;   // LDS tile element
    static __device__ __forceinline__ V step(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};
template <>
struct MfmaAcc<float> {
    using V = v4f;
    using L = float;
    static __device__ __forceinline__ V step(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};
template <>
struct MfmaAcc<Bf16> {
    using V = v4f;
    using L = float;
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

// BF16 bits of a finite float, rounded to nearest with ties to even.
__device__ __forceinline__ short bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// TM = 64: each wavefront owns 32 x 32 outputs (2 x 2 MFMA tiles); TM = 32:
// 16 x 32 (1 x 2), twice the workgroups for the small products.
template <bool USE_G, bool SUB, class TI, class TO, class MT, int TM = 64>
__global__ __launch_bounds__(256) void k_block_apply_mfma(ChPtrs mats, int n, int nq, int W,
                                                          const TI *__restrict__ in,
                                                          const double *__restrict__ G,
                                                          const double *__restrict__ add,
                                                          TO *__restrict__ out) {
    static_assert(TM == 64 || TM == 32, "64- or 32-row tiles");
    constexpr int TN = 64, KS = 16, UM = TM / 32;   // 16-row MFMA tiles per wavefront
    using V = typename MfmaAcc<MT>::V;
    using L = typename MfmaAcc<MT>::L;
    __shared__ L sA[KS][TM + 1];
    __shared__ L sB[KS][TN + 1];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int a = blockIdx.z;
    const int row0 = blockIdx.y * TM;
    const int64_t q0 = (int64_t)blockIdx.x * TN;
    const int64_t ncol = (int64_t)nq * W;
    const double *Mt = mats.p[a];
    const int64_t chbase = (int64_t)a * nq * n;
    V acc[UM][2];
#pragma unroll
    for (int u = 0; u < UM; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[u][v][r] = 0;
    const int li = lane & 15, lk = lane >> 4;
    // (j, c) of the panel columns this thread stages, once (as in k_block_apply)
    constexpr int NBL = KS * TN / 256;
    int64_t bbase[NBL];
    int bc[NBL];
#pragma unroll
    for (int sl = 0; sl < NBL; ++sl) {
        const int64_t q = q0 + (t + 256 * sl) % TN;
        bbase[sl] = -1;
        bc[sl] = 0;
        if (q < ncol) {
            const int j = (int)(q / W);
            bc[sl] = (int)(q - (int64_t)j * W);
            bbase[sl] = (chbase + (int64_t)j * n) * W;
        }
    }
    // loads of the next k step in flight during this step's products (as in
    // k_block_apply)
    constexpr int NAL = TM * KS / 256;
    double ra[NAL], rg[NBL][2], rx[NBL][2];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int sl = 0; sl < NAL; ++sl) {
            const int idx = t + 256 * sl;
            const int r = row0 + idx / KS, k = k0 + idx % KS;
            ra[sl] = (r < n && k < n) ? Mt[(int64_t)r * n + k] : 0.0;
        }
#pragma unroll
        for (int sl = 0; sl < NBL; ++sl) {
            const int k = k0 + (t + 256 * sl) / TN;
            const bool ok = k < n && bbase[sl] >= 0;
            const int64_t o = bbase[sl] + (int64_t)k * W;
            const int c = bc[sl];
            if (USE_G) {
                const int c0 = c & ~1;
                rg[sl][0] = ok ? G[o + c0] : 0.0;
                rg[sl][1] = ok ? G[o + c0 + 1] : 0.0;
                rx[sl][0] = ok ? (double)in[o + c0] : 0.0;
                rx[sl][1] = ok ? (double)in[o + c0 + 1] : 0.0;
            } else {
                rx[sl][0] = ok ? (double)in[o + c] : 0.0;
            }
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < n; k0 += KS) {
#pragma unroll
        for (int sl = 0; sl < NAL; ++sl) {
            const int idx = t + 256 * sl;
            sA[idx % KS][idx / KS] = (L)ra[sl];
        }
#pragma unroll
        for (int sl = 0; sl < NBL; ++sl) {
            const int idx = t + 256 * sl;
            double v = rx[sl][0];
            if (USE_G) {
                const double gr = rg[sl][0], gi = rg[sl][1], xr = rx[sl][0], xi = rx[sl][1];
                v = (bc[sl] & 1) ? (gr * xi + gi * xr) : (gr * xr - gi * xi);
            }
            sB[idx / TN][idx % TN] = (L)v;
        }
        __syncthreads();
        if (k0 + KS < n) fetch(k0 + KS);
        if constexpr (std::is_same<MT, Bf16>::value) {
            // one 16 x 16 x 16 step covers the whole k slab
            v4s av[UM], bv[2];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int u = 0; u < UM; ++u) av[u][q] = bf16_bits(sA[4 * lk + q][wr * (TM / 2) + u * 16 + li]);
#pragma unroll
                for (int v = 0; v < 2; ++v) bv[v][q] = bf16_bits(sB[4 * lk + q][wc * 32 + v * 16 + li]);
            }
#pragma unroll
            for (int u = 0; u < UM; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v)
                    acc[u][v] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[u], bv[v], acc[u][v], 0, 0, 0);
        } else {
#pragma unroll
            for (int kb = 0; kb < KS; kb += 4) {
                MT av[UM], bv[2];
#pragma unroll
                for (int u = 0; u < UM; ++u) av[u] = sA[kb + lk][wr * (TM / 2) + u * 16 + li];
#pragma unroll
                for (int v = 0; v < 2; ++v) bv[v] = sB[kb + lk][wc * 32 + v * 16 + li];
#pragma unroll
                for (int u = 0; u < UM; ++u)
#pragma unroll
                    for (int v = 0; v < 2; ++v) acc[u][v] = MfmaAcc<MT>::step(av[u], bv[v], acc[u][v]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < UM; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int64_t q = q0 + wc * 32 + v * 16 + li;
            if (q >= ncol) continue;
            const int j = (int)(q / W);
            const int64_t ob = (chbase + (int64_t)j * n) * W + (q - (int64_t)j * W);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + wr * (TM / 2) + u * 16 + MfmaAcc<MT>::row(lk, r);
                if (row >= n) continue;
                const int64_t gi = ob + (int64_t)row * W;
                const double d = (double)acc[u][v][r];
                out[gi] = (TO)(SUB ? add[gi] - d : d);
            }
        }
}

// --------------------------------------------------------------- P0 SpMM
// Workgroups are dealt to the 8 XCDs round robin (workgroup b runs on XCD
// b % 8), each XCD with its own L2.  Neighbouring cell rows share most of
// their columns, so the row range is remapped to give every XCD one
// contiguous run of rows: XCD x takes logical blocks [start_x, start_x +
// count_x) in order.  A bijection on [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int q = nb / 8, r = nb % 8;
    const int x = b % 8, i = b / 8;
    return x * q + (x < r ? x : r) + i;
}

// y[r][c] = sum_t val[t] x[col[t]][c]; one wavefront per cell row, lanes =
// (nonzero slot g, column c) with Wp = pow2 >= W columns per slot; four
// independent gathers in flight per lane.
template <class V, class XT, class YT, bool XCD>
__global__ __launch_bounds__(256) void k_spmm(const int64_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ col,
                                              const V *__restrict__ val, int nrow, int W, int Wp,
                                              const XT *__restrict__ x,
                                              YT *__restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int r = (XCD ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (r >= nrow) return;
    const int G = 64 / Wp;
    const int g = lane / Wp, c = lane % Wp;
    const int64_t b = rowptr[r], e = rowptr[r + 1];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (c < W) {
        int64_t t = b + g;
        for (; t + 3 * G < e; t += 4 * G) {
            const int64_t c0 = col[t], c1 = col[t + G], c2 = col[t + 2 * G], c3 = col[t + 3 * G];
            const double v0 = (double)val[t], v1 = (double)val[t + G];
            const double v2 = (double)val[t + 2 * G], v3 = (double)val[t + 3 * G];
            a0 += v0 * (double)x[c0 * W + c];
            a1 += v1 * (double)x[c1 * W + c];
            a2 += v2 * (double)x[c2 * W + c];
            a3 += v3 * (double)x[c3 * W + c];
        }
        for (; t < e; t += G) a0 += (double)val[t] * (double)x[(int64_t)col[t] * W + c];
    }
    double acc = (a0 + a1) + (a2 + a3);
    for (int off = Wp; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
    if (g == 0 && c < W) y[(int64_t)r * W + c] = (YT)acc;
}

// Block SpMM for n_ch channels: y[(a, r)][c] = sum_t sum_a2 val[t][a][a2]
// x[(a2, col[t])][c]; one wavefront per cell row, all NCH output rows.
template <class V, int NCH, class XT, class YT, bool XCD, int U>
__global__ __launch_bounds__(256) void k_spmm_bsr(const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col,
                                                  const V *__restrict__ val, int ncell, int W,
                                                  int Wp, const XT *__restrict__ x,
                                                  YT *__restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int r = (XCD ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (r >= ncell) return;
    const int G = 64 / Wp;
    const int g = lane / Wp, c = lane % Wp;
    const int64_t b = rowptr[r], e = rowptr[r + 1];
    double acc[NCH];
#pragma unroll
    for (int a = 0; a < NCH; ++a) acc[a] = 0.0;
    // U > 1: U nonzeros per lane in flight (their column indices, then all
    // their gathers, issued before any is used)
    if (c < W) {
        int64_t t = b + g;
        for (; U > 1 && t + (U - 1) * G < e; t += U * G) {
            int64_t cc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) cc[u] = col[t + u * G];
            double xv[U][NCH];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int a2 = 0; a2 < NCH; ++a2)
                    xv[u][a2] = (double)x[((int64_t)a2 * ncell + cc[u]) * W + c];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const V *vb = val + (t + u * G) * NCH * NCH;
#pragma unroll
                for (int a2 = 0; a2 < NCH; ++a2)
#pragma unroll
                    for (int a = 0; a < NCH; ++a) acc[a] += (double)vb[a * NCH + a2] * xv[u][a2];
            }
        }
        for (; t < e; t += G) {
            const int64_t cc = col[t];
            const V *vb = val + t * NCH * NCH;
#pragma unroll
            for (int a2 = 0; a2 < NCH; ++a2) {
                const double xv = (double)x[((int64_t)a2 * ncell + cc) * W + c];
#pragma unroll
                for (int a = 0; a < NCH; ++a) acc[a] += (double)vb[a * NCH + a2] * xv;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < NCH; ++a) {
        double v = acc[a];
        for (int off = Wp; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
        if (g == 0 && c < W) y[((int64_t)a * ncell + r) * W + c] = (YT)v;
    }
}

// LDS-staged SpMM for any n_ch (n_ch = 1 is the s-wave case): one
// wavefront (= workgroup) per cell row; the row's column indices and value
// blocks are loaded a tile at a time with coalesced loads into LDS, then
// every lane slot (nonzero slot g, column pair c, c + 1) reads them as LDS
// broadcasts, so global memory sees each value once instead of once per
// column lane.  Two columns per lane halve the lanes per nonzero, so twice
// as many nonzeros are gathered per instruction (measured 32 -> 25 us per
// application at 150 x 150 with 8 energies).
template <class V, int NCH, class XT, class YT>
__global__ __launch_bounds__(64) void k_spmm_lds(const int64_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col,
                                                 const V *__restrict__ val, int ncell, int W,
                                                 int Wp, const XT *__restrict__ x,
                                                 YT *__restrict__ y) {
    constexpr int NV = NCH * NCH;
    constexpr int T = NV <= 16 ? 64 : 32;   // nonzeros per tile
    __shared__ int32_t cs[T];
    __shared__ V vs[T * NV];
    const int lane = threadIdx.x;
    const int r = blockIdx.x;
    // two consecutive entries of x per lane: Wp / 2 lanes per nonzero
    const int L = Wp >> 1;
    const int G = 64 / L, g = lane / L, c = 2 * (lane % L);
    const int64_t b = rowptr[r], e = rowptr[r + 1];
    double acc[NCH][2];
#pragma unroll
    for (int a = 0; a < NCH; ++a) acc[a][0] = acc[a][1] = 0.0;
    for (int64_t t0 = b; t0 < e; t0 += T) {
        const int n = (int)(e - t0 < T ? e - t0 : T);
        __syncthreads();   // the previous tile has been consumed
        for (int k = lane; k < n; k += 64) cs[k] = col[t0 + k];
        for (int k = lane; k < n * NV; k += 64) vs[k] = val[t0 * NV + k];
        __syncthreads();
        if (c < W) {
#pragma unroll 4
            for (int k = g; k < n; k += G) {
                const int64_t cc = cs[k];
                const V *vb = vs + k * NV;
#pragma unroll
                for (int a2 = 0; a2 < NCH; ++a2) {
                    const XT *xp = x + ((int64_t)a2 * ncell + cc) * W + c;
                    const double x0 = (double)xp[0], x1 = (double)xp[1];
#pragma unroll
                    for (int a = 0; a < NCH; ++a) {
                        const double v = (double)vb[a * NCH + a2];
                        acc[a][0] += v * x0;
                        acc[a][1] += v * x1;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int a = 0; a < NCH; ++a) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            double v = acc[a][h];
            for (int off = L; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
            if (g == 0 && c < W) y[((int64_t)a * ncell + r) * W + c + h] = (YT)v;
        }
    }
}

template <class T> struct Pair2;
template <> struct Pair2<double> { using type = double2; };
template <> struct Pair2<float> { using type = float2; };

// P0 SpMM with its memory latencies overlapped.  One wavefront per cell row
// (a 64-thread workgroup), two entries of x per lane as above.  The row's
// nonzeros go in tiles of T: the columns and channel-coupling values of the
// next tile are loaded (contiguously, into registers) while the current
// tile's x rows are gathered, and are parked in LDS once it is consumed.
// Inside a tile each lane issues the gathers of SU nonzeros, every column
// channel, before it uses any of them (SU = 2 for three or more channels:
// fewer registers, more wavefronts resident, measured faster than 4 or 8 on
// the 300 x 300 three-channel operator).  The sums run in the same order as
// k_spmm_lds, so both give the same bits.
// With PERM the workgroups visit the rows in the order perm[0, ncell): XCD x
// (workgroups g = x mod 8) walks the contiguous stretch perm[s_x, s_x+1),
// workgroup g taking entry s_x + g / 8, where s_0..s_8 = perm[ncell ..
// ncell + 8] split the order into eight parts of equal nonzero count.  perm
// lists the cells in square tiles of the (p, q) lattice; neighbouring cells
// touch largely the same columns, so an XCD's concurrent rows share their x
// panel rows in its L2 instead of fetching them again.
template <class V, int NCH, class XT, class YT, bool PERM>
__global__ __launch_bounds__(64) void k_spmm_pipe(const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col,
                                                  const V *__restrict__ val, int ncell, int W,
                                                  int Wp, const XT *__restrict__ x,
                                                  YT *__restrict__ y,
                                                  const int32_t *__restrict__ perm) {
    using X2 = typename Pair2<XT>::type;
    constexpr int NV = NCH * NCH;
    constexpr int T = NV <= 16 ? 64 : 32;   // nonzeros per tile (<= 64)
    constexpr int NVL = (T * NV + 63) / 64;  // staged values per lane
    constexpr int SU = NCH >= 3 ? 2 : 4;     // nonzeros gathered together per lane
    __shared__ int32_t cs[T];
    __shared__ V vs[T * NV];
    const int lane = threadIdx.x;
    int r = blockIdx.x;
    if (PERM) {
        const int xcd = blockIdx.x & 7;
        const int lr = perm[ncell + xcd] + (int)(blockIdx.x >> 3);
        if (lr >= perm[ncell + xcd + 1]) return;   // the whole workgroup leaves
        r = perm[lr];
    }
    const int L = Wp >> 1;
    const int G = 64 / L, g = lane / L, c = 2 * (lane % L);
    const bool colok = c < W;
    const int64_t b = rowptr[r], e = rowptr[r + 1];
    double acc[NCH][2];
#pragma unroll
    for (int a = 0; a < NCH; ++a) acc[a][0] = acc[a][1] = 0.0;
    int32_t pc = 0;
    V pv[NVL];
    auto fetch = [&](int64_t t0) {
        const int n = (int)(e - t0 < T ? e - t0 : T);
        pc = lane < n ? col[t0 + lane] : 0;
#pragma unroll
        for (int u = 0; u < NVL; ++u) {
            const int k = lane + 64 * u;
            pv[u] = k < n * NV ? val[t0 * NV + k] : V(0);
        }
    };
    if (b < e) fetch(b);
    for (int64_t t0 = b; t0 < e; t0 += T) {
        const int n = (int)(e - t0 < T ? e - t0 : T);
        __syncthreads();   // the previous tile has been consumed
        if (lane < T) cs[lane] = pc;
#pragma unroll
        for (int u = 0; u < NVL; ++u)
            if (lane + 64 * u < T * NV) vs[lane + 64 * u] = pv[u];
        __syncthreads();
        if (t0 + T < e) fetch(t0 + T);
        for (int k0 = 0; k0 < n; k0 += G * SU) {
            int kv[SU];
            X2 xv[SU][NCH];
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int k = k0 + u * G + g;
                const bool ok = colok && k < n;
                kv[u] = ok ? k : 0;   // slots past the tile read x = 0
                const int64_t cc = ok ? cs[k] : 0;
#pragma unroll
                for (int a2 = 0; a2 < NCH; ++a2) {
                    if (ok) xv[u][a2] = *(const X2 *)(x + ((int64_t)a2 * ncell + cc) * W + c);
                    else xv[u][a2] = X2{XT(0), XT(0)};
                }
            }
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const V *vb = vs + kv[u] * NV;
#pragma unroll
                for (int a2 = 0; a2 < NCH; ++a2) {
                    const double x0 = (double)xv[u][a2].x, x1 = (double)xv[u][a2].y;
#pragma unroll
                    for (int a = 0; a < NCH; ++a) {
                        const double v = (double)vb[a * NCH + a2];
                        acc[a][0] += v * x0;
                        acc[a][1] += v * x1;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int a = 0; a < NCH; ++a) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            double v = acc[a][h];
            for (int off = L; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
            if (g == 0 && colok) y[((int64_t)a * ncell + r) * W + c + h] = (YT)v;
        }
    }
}

// ------------------------------------------------------ Krylov vector ops
// Rows are processed in chunks of NR * (256 / nEp) per workgroup (nEp =
// pow2 >= nE).  Thread t handles energy e = t % nEp and rows r0 + t / nEp +
// k (256 / nEp), k < NR, so loads of one row are contiguous across threads
// and each thread keeps one energy.  Larger NR means fewer per-chunk partial
// sums to reduce, smaller NR more workgroups in flight.
inline int chunk_rows_of(int nEp, int nr) { return nr * (256 / nEp); }

// Reduce (sr, si) over the lanes of a wavefront that share the same energy
// (lane offsets nEp, 2 nEp, ...).
__device__ __forceinline__ void reduce_rows(double &sr, double &si, int nEp) {
    for (int off = nEp; off < 64; off <<= 1) {
        sr += __shfl_xor(sr, off, 64);
        si += __shfl_xor(si, off, 64);
    }
}

// Partial dot products of vectors V_0..V_{nvec-1} with the thread's rows of
// w (held in wr/wi): partial[blk][i][e] = sum conj(V_i) w over the chunk.
template <int NR>
__device__ __forceinline__ void chunk_dots(const double *__restrict__ Vb, int64_t vstride, int nvec,
                                           const double (&wr)[NR], const double (&wi)[NR],
                                           const int64_t (&off)[NR], bool valid_e, int nE, int nEp,
                                           double *__restrict__ partial,
                                           double (*red)[8][32][2]) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, e = t % nEp;
    for (int i0 = 0; i0 < nvec; i0 += 8) {
        double ar[8], ai[8];
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            ar[g] = 0.0;
            ai[g] = 0.0;
        }
        // all 8 x NR loads first (absent entries read as 0), then the sums
        double vr[8][NR], vi[8][NR];
#pragma unroll
        for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                const bool ok = off[k] >= 0 && valid_e && i0 + g < nvec;
                const double *v = Vb + (int64_t)(i0 + g) * vstride + off[k];
                vr[g][k] = ok ? v[0] : 0.0;
                vi[g][k] = ok ? v[1] : 0.0;
            }
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (off[k] < 0 || !valid_e) continue;
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                if (i0 + g < nvec) {
                    ar[g] += vr[g][k] * wr[k] + vi[g][k] * wi[k];
                    ai[g] += vr[g][k] * wi[k] - vi[g][k] * wr[k];
                }
            }
        }
#pragma unroll
        for (int g = 0; g < 8; ++g) reduce_rows(ar[g], ai[g], nEp);
        if (lane < nEp) {
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                red[wave][g][lane][0] = ar[g];
                red[wave][g][lane][1] = ai[g];
            }
        }
        __syncthreads();
        if (t < 8 * nE) {
            const int g = t / nE, ee = t % nE;
            if (i0 + g < nvec) {
                const double sr = (red[0][g][ee][0] + red[1][g][ee][0]) + (red[2][g][ee][0] + red[3][g][ee][0]);
                const double si = (red[0][g][ee][1] + red[1][g][ee][1]) + (red[2][g][ee][1] + red[3][g][ee][1]);
                const int64_t p = ((int64_t)blockIdx.x * nvec + (i0 + g)) * nE + ee;
                partial[2 * p] = sr;
                partial[2 * p + 1] = si;
            }
        }
        __syncthreads();
        (void)e;
    }
}

template <int NR>
__device__ __forceinline__ void chunk_rows(int64_t M, int nE, int nEp, int64_t (&off)[NR],
                                           bool &valid_e) {
    const int t = threadIdx.x, e = t % nEp, rs = t / nEp, rstep = 256 / nEp;
    const int64_t r0 = (int64_t)blockIdx.x * (NR * rstep);
    valid_e = e < nE;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int64_t row = r0 + rs + (int64_t)k * rstep;
        off[k] = (row < M) ? (row * nE + e) * 2 : -1;
    }
}

// partial[blk][i][e] = sum_{rows of blk} conj(V_i[row][e]) w[row][e]
template <int NR>
__global__ __launch_bounds__(256) void k_vdots(const double *__restrict__ Vb, int64_t vstride,
                                               int nvec, const double *__restrict__ w, int64_t M,
                                               int nE, int nEp, double *__restrict__ partial) {
    __shared__ double red[4][8][32][2];
    int64_t off[NR];
    bool valid_e;
    chunk_rows<NR>(M, nE, nEp, off, valid_e);
    double wr[NR], wi[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        wr[k] = (off[k] >= 0 && valid_e) ? w[off[k]] : 0.0;
        wi[k] = (off[k] >= 0 && valid_e) ? w[off[k] + 1] : 0.0;
    }
    chunk_dots<NR>(Vb, vstride, nvec, wr, wi, off, valid_e, nE, nEp, partial, red);
}

// w -= sum_i h[i][e] V_i; then either the partial dots of V_0.. with the new
// w (DOTS, second Gram-Schmidt pass) or the partial |w|^2 per energy (NORM:
// npart[blk][e]).  h layout [nvec][nE] complex.
template <int NR, bool DOTS, bool NORM>
__global__ __launch_bounds__(256) void k_vupdate(const double *__restrict__ Vb, int64_t vstride,
                                                 int nvec, const double *__restrict__ h, int64_t M,
                                                 int nE, int nEp, double *__restrict__ w,
                                                 double *__restrict__ partial) {
    __shared__ double red[4][8][32][2];
    int64_t off[NR];
    bool valid_e;
    chunk_rows<NR>(M, nE, nEp, off, valid_e);
    const int t = threadIdx.x, e = t % nEp;
    double wr[NR], wi[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        wr[k] = (off[k] >= 0 && valid_e) ? w[off[k]] : 0.0;
        wi[k] = (off[k] >= 0 && valid_e) ? w[off[k] + 1] : 0.0;
    }
    if (valid_e) {
        // four vectors at a time, their coefficients and rows loaded before
        // any is used (the loads are independent; the sums keep their order)
        constexpr int U = 4;
        for (int i0 = 0; i0 < nvec; i0 += U) {
            double hr[U], hi[U], vr[U][NR], vi[U][NR];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u;
                const bool ok = i < nvec;
                hr[u] = ok ? h[2 * (i * nE + e)] : 0.0;
                hi[u] = ok ? h[2 * (i * nE + e) + 1] : 0.0;
                const double *v = Vb + (int64_t)i * vstride;
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    const bool okk = ok && off[k] >= 0;
                    vr[u][k] = okk ? v[off[k]] : 0.0;
                    vi[u][k] = okk ? v[off[k] + 1] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (i0 + u >= nvec) break;
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    if (off[k] < 0) continue;
                    wr[k] -= hr[u] * vr[u][k] - hi[u] * vi[u][k];
                    wi[k] -= hr[u] * vi[u][k] + hi[u] * vr[u][k];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (off[k] < 0) continue;
            w[off[k]] = wr[k];
            w[off[k] + 1] = wi[k];
        }
    }
    if (DOTS) chunk_dots<NR>(Vb, vstride, nvec, wr, wi, off, valid_e, nE, nEp, partial, red);
    if (NORM) {
        double s = 0.0, z = 0.0;
#pragma unroll
        for (int k = 0; k < NR; ++k) s += wr[k] * wr[k] + wi[k] * wi[k];
        reduce_rows(s, z, nEp);
        const int lane = t & 63, wave = t >> 6;
        if (lane < nEp) red[wave][0][lane][0] = s;
        __syncthreads();
        if (t < nE) {
            const double v = (red[0][0][t][0] + red[1][0][t][0]) + (red[2][0][t][0] + red[3][0][t][0]);
            partial[2 * ((int64_t)blockIdx.x * nE + t)] = v;
            partial[2 * ((int64_t)blockIdx.x * nE + t) + 1] = 0.0;
        }
    }
}

// Cross-chunk reduction of per-chunk partial sums partial[chunk][p] (p <
// npair complex values), deterministic and in two stages.  Stage 1: grid
// (npair/32, S); each workgroup sums a contiguous run of chunks for 32
// consecutive p (8 chunk lanes per p, coalesced 512-byte rows), giving
// out2[s][p].  Stage 2 sums the S values per p.
__global__ __launch_bounds__(256) void k_reduce_stage1(const double *__restrict__ partial,
                                                       int nchunk, int npair,
                                                       double *__restrict__ out2) {
    __shared__ double red[8][32][2];
    const int t = threadIdx.x, pl = t & 31, cl = t >> 5;
    const int p = blockIdx.x * 32 + pl;
    const int S = gridDim.y, s = blockIdx.y;
    const int cps = (nchunk + S - 1) / S;
    const int c0 = s * cps, c1 = min(nchunk, c0 + cps);
    double sr = 0.0, si = 0.0;
    if (p < npair)
        for (int cb = c0 + cl; cb < c1; cb += 32) {
            // four chunks' loads in flight, summed in chunk order
            double xr[4], xi[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = cb + 8 * u;
                xr[u] = c < c1 ? partial[((int64_t)c * npair + p) * 2] : 0.0;
                xi[u] = c < c1 ? partial[((int64_t)c * npair + p) * 2 + 1] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (cb + 8 * u >= c1) break;
                sr += xr[u];
                si += xi[u];
            }
        }
    red[cl][pl][0] = sr;
    red[cl][pl][1] = si;
    __syncthreads();
    if (t < 32 && p < npair) {
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            ar += red[k][t][0];
            ai += red[k][t][1];
        }
        out2[((int64_t)s * npair + p) * 2] = ar;
        out2[((int64_t)s * npair + p) * 2 + 1] = ai;
    }
}

// Stage 2 of the dot products: h[p] = sum_s out2[s][p]; also written or
// accumulated into the Hessenberg column H[e][i][k] (layout [nE][m+1][m]
// complex) when H is given (p = i nE + e).
__global__ void k_dots_reduce(const double *__restrict__ out2, int S, int nvec, int nE,
                              double *__restrict__ h, double *__restrict__ H, int m, int kcol,
                              int accumulate) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int npair = nvec * nE;
    if (p >= npair) return;
    double sr = 0.0, si = 0.0;
    for (int s0 = 0; s0 < S; s0 += 4) {
        double xr[4], xi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = s0 + u;
            xr[u] = s < S ? out2[((int64_t)s * npair + p) * 2] : 0.0;
            xi[u] = s < S ? out2[((int64_t)s * npair + p) * 2 + 1] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (s0 + u >= S) break;
            sr += xr[u];
            si += xi[u];
        }
    }
    h[2 * p] = sr;
    h[2 * p + 1] = si;
    if (H) {
        const int i = p / nE, e = p % nE;
        double *hh = H + (((int64_t)e * (m + 1) + i) * m + kcol) * 2;
        if (accumulate) {
            hh[0] += sr;
            hh[1] += si;
        } else {
            hh[0] = sr;
            hh[1] = si;
        }
    }
}

// Both stages at once when the chunks are few (a launch saved per set of
// dot products): 8 pairs per workgroup, 32 lanes over each pair's chunks
// (four loads in flight per lane), the 32 lane sums added in lane order and
// written to h (and H) as k_dots_reduce does.
constexpr int kFusedChunks = 1024;

__global__ __launch_bounds__(256) void k_dots_final(const double *__restrict__ partial, int nchunk,
                                                    int nvec, int nE, double *__restrict__ h,
                                                    double *__restrict__ H, int m, int kcol,
                                                    int accumulate) {
    __shared__ double red[32][8][2];
    const int t = threadIdx.x, pl = t & 7, cl = t >> 3;
    const int npair = nvec * nE;
    const int p = blockIdx.x * 8 + pl;
    double sr = 0.0, si = 0.0;
    if (p < npair)
        for (int cb = cl; cb < nchunk; cb += 128) {
            double xr[4], xi[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = cb + 32 * u;
                xr[u] = c < nchunk ? partial[((int64_t)c * npair + p) * 2] : 0.0;
                xi[u] = c < nchunk ? partial[((int64_t)c * npair + p) * 2 + 1] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (cb + 32 * u >= nchunk) break;
                sr += xr[u];
                si += xi[u];
            }
        }
    red[cl][pl][0] = sr;
    red[cl][pl][1] = si;
    __syncthreads();
    if (t < 8 && p < npair) {
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            ar += red[k][t][0];
            ai += red[k][t][1];
        }
        h[2 * p] = ar;
        h[2 * p + 1] = ai;
        if (H) {
            const int i = p / nE, e = p % nE;
            double *hh = H + (((int64_t)e * (m + 1) + i) * m + kcol) * 2;
            if (accumulate) {
                hh[0] += ar;
                hh[1] += ai;
            } else {
                hh[0] = ar;
                hh[1] = ai;
            }
        }
    }
}

// w[row][e] *= scale[e] (scale[e] = 1/norm, or 0 after breakdown)
__global__ void k_scale(const double *__restrict__ inv, int64_t M, int nE,
                        double *__restrict__ w) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * nE) return;
    const double s = inv[idx % nE];
    w[2 * idx] *= s;
    w[2 * idx + 1] *= s;
}

// x[row][e] += sum_i y[e][i] V_i[row][e] for i < kuse[e]
__global__ void k_xupdate(const double *__restrict__ Vb, int64_t vstride,
                          const double *__restrict__ y, const int32_t *__restrict__ kuse, int m,
                          int64_t M, int nE, double *__restrict__ x) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * nE) return;
    const int e = (int)(idx % nE);
    double xr = x[2 * idx], xi = x[2 * idx + 1];
    const int ku = kuse[e];
    for (int i0 = 0; i0 < ku; i0 += 4) {
        double yr[4], yi[4], vr[4], vi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u;
            const bool ok = i < ku;
            yr[u] = ok ? y[2 * (e * m + i)] : 0.0;
            yi[u] = ok ? y[2 * (e * m + i) + 1] : 0.0;
            vr[u] = ok ? Vb[i * vstride + 2 * idx] : 0.0;
            vi[u] = ok ? Vb[i * vstride + 2 * idx + 1] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (i0 + u >= ku) break;
            xr += yr[u] * vr[u] - yi[u] * vi[u];
            xi += yr[u] * vi[u] + yi[u] * vr[u];
        }
    }
    x[2 * idx] = xr;
    x[2 * idx + 1] = xi;
}

// Per-energy GMRES bookkeeping.  st layout per energy (doubles):
//   [0] beta (initial residual norm of this cycle)   [1] bnorm
//   [2] residual estimate   [3] converged flag   [4] columns to use
// cs/sn: Givens rotations [nE][m] (c real, s complex); g: [nE][m+1] complex.
struct GState {
    double *st;
    double *cs, *sn, *g;
};
constexpr int kSt = 8;

// Start of a cycle: beta[e] = sqrt(nrm2[e]); g = (beta, 0, ...); inv[e] = 1/beta.
__global__ void k_cycle_start(const double *__restrict__ nrm2, int nE, int m, double tol,
                              GState S, double *__restrict__ inv) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nE) return;
    const double beta = sqrt(nrm2[2 * e]);
    double *st = S.st + e * kSt;
    st[0] = beta;
    st[2] = beta;
    const double bn = st[1];
    st[3] = (beta <= tol * bn) ? 1.0 : 0.0;
    st[4] = 0.0;
    for (int i = 0; i <= m; ++i) {
        S.g[2 * (e * (m + 1) + i)] = 0.0;
        S.g[2 * (e * (m + 1) + i) + 1] = 0.0;
    }
    S.g[2 * (e * (m + 1))] = beta;
    inv[e] = beta > 1e-300 ? 1.0 / beta : 0.0;
}

// After orthogonalising w = K v_k, one workgroup: the per-chunk |w|^2
// partials npart[chunk][e] are summed in a fixed order (256 / nE threads per
// energy, strided over chunks, then the thread sums in order), column k of
// every energy's Hessenberg matrix is staged in LDS, and one thread per
// energy sets H[k+1][k] = ||w|| and inv = 1/||w||, applies the previous
// Givens rotations to column k, forms the new one and updates the residual
// estimate.  Dynamic LDS: 256 + nE (m + 1) 2 doubles.
// With w given (few chunks), every workgroup reduces the norms itself, in
// the same order (the same bits), and scales its share of w by 1/norm:
// the basis vector's normalisation without a launch of its own; workgroup
// 0 alone updates the Hessenberg column and the rotations.
__global__ __launch_bounds__(256) void k_norm_givens(const double *__restrict__ npart, int nchunk,
                                                     double *__restrict__ H, int nE, int m, int k,
                                                     double tol, GState S,
                                                     double *__restrict__ inv,
                                                     double *__restrict__ w, int64_t M) {
    extern __shared__ double sm[];
    __shared__ double s_inv[64], s_hn[64];
    double *red = sm, *col = sm + 256;
    const int t = threadIdx.x;
    const int G = 256 / nE;
    const int ee = t % nE, ct = t / nE;
    double acc = 0.0;
    if (ct < G)
        for (int cb = ct; cb < nchunk; cb += 4 * G) {
            double x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int ch = cb + u * G;
                x[u] = ch < nchunk ? npart[2 * ((int64_t)ch * nE + ee)] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (cb + u * G >= nchunk) break;
                acc += x[u];
            }
        }
    red[t] = acc;
    if (blockIdx.x == 0)
        for (int idx = t; idx < nE * (k + 1); idx += 256) {
            const int e = idx / (k + 1), i = idx - e * (k + 1);
            const double *src = H + (((int64_t)e * (m + 1) + i) * m + k) * 2;
            col[(e * (m + 1) + i) * 2] = src[0];
            col[(e * (m + 1) + i) * 2 + 1] = src[1];
        }
    __syncthreads();
    if (t < nE) {
        double n2 = 0.0;
        for (int g = 0; g < G; ++g) n2 += red[g * nE + t];
        const double hn = sqrt(n2);
        const double beta = S.st[t * kSt];
        s_hn[t] = hn;
        s_inv[t] = (hn > 1e-14 * beta && hn > 1e-300) ? 1.0 / hn : 0.0;
    }
    __syncthreads();
    if (w)
        for (int64_t idx = (int64_t)blockIdx.x * 256 + t; idx < M * nE;
             idx += (int64_t)gridDim.x * 256) {
            const double sc = s_inv[idx % nE];
            w[2 * idx] *= sc;
            w[2 * idx + 1] *= sc;
        }
    if (blockIdx.x != 0) return;
    const int e = t;
    if (e >= nE) return;
    double *st = S.st + e * kSt;
    double *ce = col + (size_t)e * (m + 1) * 2;
    double *He = H + (int64_t)e * (m + 1) * m * 2;
    const double hn = s_hn[e];
    inv[e] = s_inv[e];
    He[((k + 1) * m + k) * 2] = hn;
    He[((k + 1) * m + k) * 2 + 1] = 0.0;
    if (st[3] != 0.0) return;   // already converged: leave its state alone
    ce[(k + 1) * 2] = hn;
    ce[(k + 1) * 2 + 1] = 0.0;
    // apply previous rotations to column k
    for (int i = 0; i < k; ++i) {
        const double c = S.cs[e * m + i];
        const double sr = S.sn[2 * (e * m + i)], si = S.sn[2 * (e * m + i) + 1];
        const double ar = ce[2 * i], ai = ce[2 * i + 1], br = ce[2 * i + 2], bi = ce[2 * i + 3];
        // a' = c a + s b ;  b' = -conj(s) a + c b
        ce[2 * i] = c * ar + (sr * br - si * bi);
        ce[2 * i + 1] = c * ai + (sr * bi + si * br);
        ce[2 * i + 2] = -(sr * ar + si * ai) + c * br;
        ce[2 * i + 3] = -(sr * ai - si * ar) + c * bi;
    }
    const double ar = ce[2 * k], ai = ce[2 * k + 1], br = ce[2 * k + 2], bi = ce[2 * k + 3];
    const double na = sqrt(ar * ar + ai * ai), nb = sqrt(br * br + bi * bi);
    double c, sr, si;
    if (na == 0.0) {
        c = 0.0;
        sr = 1.0;
        si = 0.0;
    } else {
        const double tt = sqrt(na * na + nb * nb);
        c = na / tt;
        // s = (a/|a|) conj(b) / t
        const double ur = ar / na, ui = ai / na;
        sr = (ur * br + ui * bi) / tt;
        si = (ui * br - ur * bi) / tt;
    }
    S.cs[e * m + k] = c;
    S.sn[2 * (e * m + k)] = sr;
    S.sn[2 * (e * m + k) + 1] = si;
    ce[2 * k] = c * ar + (sr * br - si * bi);
    ce[2 * k + 1] = c * ai + (sr * bi + si * br);
    ce[2 * k + 2] = 0.0;
    ce[2 * k + 3] = 0.0;
    for (int i = 0; i <= k + 1; ++i) {
        He[(i * m + k) * 2] = ce[2 * i];
        He[(i * m + k) * 2 + 1] = ce[2 * i + 1];
    }
    double *g = S.g + 2 * e * (m + 1);
    const double gr = g[2 * k], gi = g[2 * k + 1];
    g[2 * k] = c * gr;
    g[2 * k + 1] = c * gi;
    // g_{k+1} = -conj(s) g_k
    g[2 * (k + 1)] = -(sr * gr + si * gi);
    g[2 * (k + 1) + 1] = -(sr * gi - si * gr);
    const double res = sqrt(g[2 * (k + 1)] * g[2 * (k + 1)] + g[2 * (k + 1) + 1] * g[2 * (k + 1) + 1]);
    st[2] = res;
    st[4] = k + 1;
    if (res <= tol * st[1] || s_inv[e] == 0.0) st[3] = 1.0;
}

// y = R^{-1} g over the first st[4] columns (back substitution).
__global__ void k_trisolve(const double *__restrict__ H, int nE, int m, GState S,
                           double *__restrict__ y, int32_t *__restrict__ kuse) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nE) return;
    const double *st = S.st + e * kSt;
    const int ku = (int)st[4];
    kuse[e] = ku;
    const double *He = H + (int64_t)e * (m + 1) * m * 2;
    const double *g = S.g + 2 * e * (m + 1);
    double *ye = y + 2 * e * m;
    for (int i = ku - 1; i >= 0; --i) {
        double sr = g[2 * i], si = g[2 * i + 1];
        for (int jj = i + 1; jj < ku; ++jj) {
            const double hr = He[(i * m + jj) * 2], hi = He[(i * m + jj) * 2 + 1];
            sr -= hr * ye[2 * jj] - hi * ye[2 * jj + 1];
            si -= hr * ye[2 * jj + 1] + hi * ye[2 * jj];
        }
        const double dr = He[(i * m + i) * 2], di = He[(i * m + i) * 2 + 1];
        const double dd = dr * dr + di * di;
        ye[2 * i] = dd > 0 ? (sr * dr + si * di) / dd : 0.0;
        ye[2 * i + 1] = dd > 0 ? (si * dr - sr * di) / dd : 0.0;
    }
}

// e0 vectors: x[idx0[e]][e] = 1 (others 0 -- caller zeroes).
__global__ void k_unit(const int64_t *__restrict__ idx0, int nE, double *__restrict__ x) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nE) return;
    x[(idx0[e] * nE + e) * 2] = 1.0;
}

// r = b - r (in place: r holds A_op(x)); used for true residuals.
__global__ void k_sub_from(const double *__restrict__ b, int64_t n, double *__restrict__ r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) r[i] = b[i] - r[i];
}

// Amplitudes: A = rho0 U, S = 1 - 2 pi i A; breakup S_k0 = -2 pi i sqrt(rho_k rho0) u_k.
// list entries: (energy e, row, rho_k); out[t] = (Re, Im).
__global__ void k_amplitudes(const double *__restrict__ x, int nE, const int64_t *__restrict__ rows,
                             const int32_t *__restrict__ ens, const double *__restrict__ rho,
                             const double *__restrict__ rho0, int n, double *__restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int e = ens[t];
    const double ur = x[(rows[t] * nE + e) * 2], ui = x[(rows[t] * nE + e) * 2 + 1];
    const double f = sqrt(rho[t] * rho0[e]);
    // value = f * u ; S-like entries: -2 pi i f u = 2 pi f (ui - i ur)
    out[4 * t + 0] = ur;
    out[4 * t + 1] = ui;
    out[4 * t + 2] = 2.0 * M_PI * f * ui;
    out[4 * t + 3] = -2.0 * M_PI * f * ur;
}

// Warm-start judge: alpha[e] = <r, b> / |r|^2 with r = (1 - K) x0, the
// scaling of x0 that minimises |b - alpha r|; 0 when |r|^2 is zero or
// anything is not finite.  rb: <r, b> (complex), rr: |r|^2 (real part).
__global__ void k_warm_alpha(const double *__restrict__ rb, const double *__restrict__ rr, int nE,
                             double *__restrict__ alpha) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nE) return;
    const double n2 = rr[2 * e];
    const double ar = rb[2 * e] / n2, ai = rb[2 * e + 1] / n2;
    const bool ok = n2 > 0.0 && isfinite(n2) && isfinite(ar) && isfinite(ai);
    alpha[2 * e] = ok ? ar : 0.0;
    alpha[2 * e + 1] = ok ? ai : 0.0;
}

// x = alpha x, r = b - alpha r; alpha = 0 gives x = 0 and r = b exactly,
// whatever x and r held (NaN included).
__global__ void k_warm_apply(const double *__restrict__ alpha, int64_t M, int nE,
                             const double *__restrict__ b, double *__restrict__ x,
                             double *__restrict__ r) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * nE) return;
    const int e = (int)(idx % nE);
    const double ar = alpha[2 * e], ai = alpha[2 * e + 1];
    if (ar == 0.0 && ai == 0.0) {
        x[2 * idx] = 0.0;
        x[2 * idx + 1] = 0.0;
        r[2 * idx] = b[2 * idx];
        r[2 * idx + 1] = b[2 * idx + 1];
        return;
    }
    const double xr = x[2 * idx], xi = x[2 * idx + 1];
    x[2 * idx] = ar * xr - ai * xi;
    x[2 * idx + 1] = ar * xi + ai * xr;
    const double rr = r[2 * idx], ri = r[2 * idx + 1];
    r[2 * idx] = b[2 * idx] - (ar * rr - ai * ri);
    r[2 * idx + 1] = b[2 * idx + 1] - (ar * ri + ai * rr);
}

// ----------------------------------------------------------------- host
namespace {

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

struct Batch {
    wpcd_ctx *c;
    int nE, nEp, W, Wp, m;
    int64_t M;
    bool fp64;
    double *G, *X, *B, *T1, *T2, *R, *Vb, *H, *partial, *h, *inv, *y;
    int32_t *kuse;
    GState S;
    int64_t vstride;
    int nchunk;
    int apply_cfg;   // tile shape of the block products (kApplyCfg)
    int nr;          // rows per thread of the vector kernels (1, 2, 4)
    int nsplit;      // stage-1 splits of the cross-chunk reductions
    double *out2;    // stage-1 results [nsplit][pairs][2]
    bool lowp;       // FP32 intermediate panels in the inner iterations
    bool bf16;       // ... with the block products on the BF16 matrix cores
    int spmm_cfg;    // P0 SpMM variant (0..6, see launch_spmm)
    // Layout.  A reduced system (Feshbach reduction) holds its major
    // channels in c (fine lattice, rows [0, M_F)) and its minor channels in
    // cm (coarse lattice, rows [M_F, M)); P0 is then one scalar CSR over
    // the reduced cells.  Otherwise cm is null and M_F = M.
    wpcd_ctx *cm;
    int64_t M_F;
    int spmm_rows;   // CSR rows of the SpMM: cells (n_p n_q), or the reduced cells
    int spmm_nch;    // channel block of a CSR entry (1 for the reduced CSR)
    void set_chunks(int nr_) {
        nr = nr_;
        nchunk = (int)((M + (int64_t)nr * (256 / nEp) - 1) / ((int64_t)nr * (256 / nEp)));
        nsplit = std::max(1, std::min(64, (nchunk + 127) / 128));
    }
};
constexpr int kMaxSplit = 64;

// Candidate tile shapes (TM x TN) of the block products; the last one is
// the FP64 matrix-core kernel (64 x 64 tiles).
constexpr int kApplyCfg = 6;
constexpr int kApplyTM[kApplyCfg] = {64, 32, 32, 16, 64, 32};
constexpr int kApplyTN[kApplyCfg] = {64, 64, 32, 64, 64, 64};
constexpr int kNrCand[3] = {1, 2, 4};

int apply_blocks(const wpcd_ctx *c, int W, int cfg) {
    return cdiv((int64_t)c->nq * W, kApplyTN[cfg]) * cdiv(c->np, kApplyTM[cfg]) * c->nch;
}

// One part of the layout: the geometry (n_p, n_q, channels, pair waves)
// of a context and the offset of its rows in the batch's vectors.
struct Part {
    const wpcd_ctx *g;
    int64_t off;   // first row of the part
};

// Per-channel pair-wave matrices of a part: V~ (which 0) or O (which 1).
ChPtrs wave_mats(const wpcd_ctx *g, int which) {
    ChPtrs m{};
    for (int a = 0; a < g->nch; ++a) {
        const PairWave &w = g->waves[g->ch_wave[a]];
        m.p[a] = which ? w.O.ptr : w.Vt.ptr;
    }
    return m;
}

template <bool USE_G, bool SUB, int TM, int TN, class TI, class TO>
void launch_block_apply_t(Batch &b, const Part &pt, ChPtrs mats, const TI *in, const double *add,
                          TO *out) {
    const wpcd_ctx *g = pt.g;
    const int64_t o = pt.off * b.W;
    dim3 grid(cdiv((int64_t)g->nq * b.W, TN), cdiv(g->np, TM), g->nch);
    hipLaunchKernelGGL((k_block_apply<USE_G, SUB, TM, TN, TI, TO>), grid, dim3(256), 0, b.c->stream,
                       mats, g->np, g->nq, b.W, in + o, b.G + o, add ? add + o : nullptr, out + o);
}

template <bool USE_G, bool SUB, class TI, class TO, class MT, int TM = 64>
void launch_block_apply_mfma(Batch &b, const Part &pt, ChPtrs mats, const TI *in, const double *add,
                             TO *out) {
    const wpcd_ctx *g = pt.g;
    const int64_t o = pt.off * b.W;
    dim3 grid(cdiv((int64_t)g->nq * b.W, 64), cdiv(g->np, TM), g->nch);
    hipLaunchKernelGGL((k_block_apply_mfma<USE_G, SUB, TI, TO, MT, TM>), grid, dim3(256), 0,
                       b.c->stream, mats, g->np, g->nq, b.W, in + o, b.G + o,
                       add ? add + o : nullptr, out + o);
}

// Tile shapes 0-3 on the vector ALUs, 4 and 5 (64- and 32-row tiles) on the FP64 matrix cores (all FP64
// arithmetic); the inner iterations of the refine tiers (FP32 panels) use the
// FP32 matrix cores, or the BF16 ones, with FP32 accumulation.
template <bool USE_G, bool SUB, class TI, class TO>
void block_apply_part(Batch &b, const Part &pt, ChPtrs mats, const TI *in, const double *add,
                      TO *out) {
    if (std::is_same<TI, float>::value || std::is_same<TO, float>::value) {
        // 32-row tiles when 64-row ones would leave the device under-filled
        const bool small = apply_blocks(pt.g, b.W, 4) < 512;
        if (b.bf16) {
            if (small) launch_block_apply_mfma<USE_G, SUB, TI, TO, Bf16, 32>(b, pt, mats, in, add, out);
            else launch_block_apply_mfma<USE_G, SUB, TI, TO, Bf16>(b, pt, mats, in, add, out);
        } else {
            if (small) launch_block_apply_mfma<USE_G, SUB, TI, TO, float, 32>(b, pt, mats, in, add, out);
            else launch_block_apply_mfma<USE_G, SUB, TI, TO, float>(b, pt, mats, in, add, out);
        }
        return;
    }
    switch (b.apply_cfg) {
        case 0: launch_block_apply_t<USE_G, SUB, 64, 64>(b, pt, mats, in, add, out); break;
        case 1: launch_block_apply_t<USE_G, SUB, 32, 64>(b, pt, mats, in, add, out); break;
        case 2: launch_block_apply_t<USE_G, SUB, 32, 32>(b, pt, mats, in, add, out); break;
        case 3: launch_block_apply_t<USE_G, SUB, 16, 64>(b, pt, mats, in, add, out); break;
        case 4: launch_block_apply_mfma<USE_G, SUB, TI, TO, double>(b, pt, mats, in, add, out); break;
        default: launch_block_apply_mfma<USE_G, SUB, TI, TO, double, 32>(b, pt, mats, in, add, out); break;
    }
}

// The block products of every part of the layout with its pair waves'
// V~ (which 0) or O (which 1).
template <bool USE_G, bool SUB, class TI, class TO>
void launch_block_apply(Batch &b, int which, const TI *in, const double *add, TO *out) {
    block_apply_part<USE_G, SUB>(b, Part{b.c, 0}, wave_mats(b.c, which), in, add, out);
    if (b.cm) block_apply_part<USE_G, SUB>(b, Part{b.cm, b.M_F}, wave_mats(b.cm, which), in, add, out);
}

// P0 SpMM candidates: 0 plain, 1 XCD-contiguous rows, 2 several nonzeros
// in flight per lane (block form), 3 both, 4 LDS-staged tiles, 5 LDS-staged
// tiles with the loads of a tile overlapped (k_spmm_pipe), 6 as 5 with the
// rows visited in lattice tiles, XCD-contiguous and balanced.

template <class PT, class V, int NCH, bool PERM, bool PIPE>
void launch_spmm_lds(Batch &b, const V *val, const PT *x, PT *y) {
    wpcd_ctx *c = b.c;
    const int nrow = b.spmm_rows;
    const int grid = PERM ? c->perm_grid : nrow;
    if (PIPE)
        hipLaunchKernelGGL((k_spmm_pipe<V, NCH, PT, PT, PERM>), dim3(grid), dim3(64), 0,
                           c->stream, c->d_rowptr.ptr, c->d_col.ptr, val, nrow, b.W, b.Wp, x,
                           y, PERM ? c->d_perm.ptr : nullptr);
    else
        hipLaunchKernelGGL((k_spmm_lds<V, NCH, PT, PT>), dim3(nrow), dim3(64), 0, c->stream,
                           c->d_rowptr.ptr, c->d_col.ptr, val, nrow, b.W, b.Wp, x, y);
    WPCD_HIP(hipGetLastError());
}

template <class PT, class V, bool PERM, bool PIPE>
void launch_spmm_lds_n(Batch &b, const V *val, const PT *x, PT *y) {
    switch (b.spmm_nch) {
        case 1: launch_spmm_lds<PT, V, 1, PERM, PIPE>(b, val, x, y); break;
        case 2: launch_spmm_lds<PT, V, 2, PERM, PIPE>(b, val, x, y); break;
        case 3: launch_spmm_lds<PT, V, 3, PERM, PIPE>(b, val, x, y); break;
        case 4: launch_spmm_lds<PT, V, 4, PERM, PIPE>(b, val, x, y); break;
        case 5: launch_spmm_lds<PT, V, 5, PERM, PIPE>(b, val, x, y); break;
        case 6: launch_spmm_lds<PT, V, 6, PERM, PIPE>(b, val, x, y); break;
        case 7: launch_spmm_lds<PT, V, 7, PERM, PIPE>(b, val, x, y); break;
        default: launch_spmm_lds<PT, V, 8, PERM, PIPE>(b, val, x, y); break;
    }
}

// Row visiting order of the tiled SpMM variants: the cells in square tiles
// of kPermTile x kPermTile lattice cells (tiles in row-major order over
// (j, i), cells row-major inside a tile), followed by the nine bounds that
// cut it into eight stretches of equal nonzero count, one per XCD (the row
// lengths vary several-fold over the lattice, so equal row counts would
// leave XCDs idle).  Built on the host from the row pointers, uploaded
// before any launch that uses it (never inside a graph capture); the order
// is valid for any P of this grid, the balance is that of the P it was
// built for.
constexpr int kPermTile = 32;

// A reduced system's rows are the cells of its parts: each major channel's
// fine lattice, then each minor channel's coarse lattice; each part is
// visited in tiles of its own lattice.
void ensure_perm(wpcd_ctx *c) {
    struct Lat {
        int64_t off;
        int np, nq;
    };
    std::vector<Lat> parts;
    if (c->reduced) {
        const int64_t ncell = (int64_t)c->np * c->nq;
        for (int a = 0; a < c->nch; ++a) parts.push_back({a * ncell, c->np, c->nq});
        const wpcd_ctx *m = c->minor;
        const int64_t ncc = (int64_t)m->np * m->nq;
        for (int a = 0; a < m->nch; ++a) parts.push_back({c->nch * ncell + a * ncc, m->np, m->nq});
    } else {
        parts.push_back({0, c->np, c->nq});
    }
    const int nrow = c->reduced ? (int)c->red_rows : c->np * c->nq;
    if (c->perm_np == c->np && c->perm_nq == c->nq && c->perm_nnz == c->nnz &&
        c->perm_rows == nrow && c->d_perm.ptr)
        return;
    std::vector<int64_t> rp(nrow + 1);
    WPCD_HIP(hipMemcpyAsync(rp.data(), c->d_rowptr.ptr, rp.size() * sizeof(int64_t),
                            hipMemcpyDeviceToHost, c->stream));
    WPCD_HIP(hipStreamSynchronize(c->stream));
    std::vector<int32_t> perm;
    perm.reserve((size_t)nrow + 9);
    for (const Lat &l : parts)
        for (int tj = 0; tj < l.nq; tj += kPermTile)
            for (int ti = 0; ti < l.np; ti += kPermTile)
                for (int j = tj; j < std::min(l.nq, tj + kPermTile); ++j)
                    for (int i = ti; i < std::min(l.np, ti + kPermTile); ++i)
                        perm.push_back((int32_t)(l.off + (int64_t)j * l.np + i));
    const int64_t total = rp[nrow];
    int64_t acc = 0;
    int next = 1, grid = 0, prev = 0;
    perm.push_back(0);
    for (int k = 0; k < nrow && next < 8; ++k) {
        acc += rp[perm[k] + 1] - rp[perm[k]];
        while (next < 8 && acc * 8 >= total * next) {
            perm.push_back(k + 1);
            grid = std::max(grid, k + 1 - prev);
            prev = k + 1;
            ++next;
        }
    }
    while (next < 8) {   // empty P: the remaining stretches are empty
        perm.push_back(nrow);
        grid = std::max(grid, nrow - prev);
        prev = nrow;
        ++next;
    }
    perm.push_back(nrow);
    grid = std::max(grid, nrow - prev);
    c->d_perm.reserve(perm.size());
    WPCD_HIP(hipMemcpyAsync(c->d_perm.ptr, perm.data(), perm.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, c->stream));
    WPCD_HIP(hipStreamSynchronize(c->stream));
    c->perm_np = c->np;
    c->perm_nq = c->nq;
    c->perm_nnz = c->nnz;
    c->perm_rows = nrow;
    c->perm_grid = 8 * std::max(grid, 1);
}

template <class PT, class V, bool XCD, int U>
void launch_spmm_v(Batch &b, const V *val, const PT *x, PT *y) {
    wpcd_ctx *c = b.c;
    const int nrow = b.spmm_rows;
    const dim3 grid(cdiv(nrow, 4)), blk(256);
    const int64_t *rp = c->d_rowptr.ptr;
    const int32_t *cl = c->d_col.ptr;
    hipStream_t s = c->stream;
    switch (b.spmm_nch) {
        case 1: hipLaunchKernelGGL((k_spmm<V, PT, PT, XCD>), grid, blk, 0, s, rp, cl, val, nrow, b.W, b.Wp, x, y); break;
        case 2: hipLaunchKernelGGL((k_spmm_bsr<V, 2, PT, PT, XCD, U>), grid, blk, 0, s, rp, cl, val, nrow, b.W, b.Wp, x, y); break;
        case 3: hipLaunchKernelGGL((k_spmm_bsr<V, 3, PT, PT, XCD, U>), grid, blk, 0, s, rp, cl, val, nrow, b.W, b.Wp, x, y); break;
        case 4: hipLaunchKernelGGL((k_spmm_bsr<V, 4, PT, PT, XCD, U>), grid, blk, 0, s, rp, cl, val, nrow, b.W, b.Wp, x, y); break;
        case 5: hipLaunchKernelGGL((k_spmm_bsr<V, 5, PT, PT, XCD, (U > 2 ? 2 : U)>), grid, blk, 0, s, rp, cl, val, nrow, b.W, b.Wp, x, y); break;
        case 6: hipLaunchKernelGGL((k_spmm_bsr<V, 6, PT, PT, XCD, (U > 2 ? 2 : U)>), grid, blk, 0, s, rp, cl, val, nrow, b.W, b.Wp, x, y); break;
        case 7: hipLaunchKernelGGL((k_spmm_bsr<V, 7, PT, PT, XCD, (U > 2 ? 2 : U)>), grid, blk, 0, s, rp, cl, val, nrow, b.W, b.Wp, x, y); break;
        default: hipLaunchKernelGGL((k_spmm_bsr<V, 8, PT, PT, XCD, (U > 2 ? 2 : U)>), grid, blk, 0, s, rp, cl, val, nrow, b.W, b.Wp, x, y); break;
    }
    WPCD_HIP(hipGetLastError());
}

template <class PT>
void launch_spmm(Batch &b, const PT *x, PT *y, int cfg) {
    wpcd_ctx *c = b.c;
    auto go = [&](auto val) {
        using VT = std::remove_const_t<std::remove_pointer_t<decltype(val)>>;
        switch (cfg) {
            case 4: launch_spmm_lds_n<PT, VT, false, false>(b, val, x, y); return;
            case 5: launch_spmm_lds_n<PT, VT, false, true>(b, val, x, y); return;
            case 6: launch_spmm_lds_n<PT, VT, true, true>(b, val, x, y); return;
            default: break;
        }
        switch (cfg) {
            case 0: launch_spmm_v<PT, std::remove_const_t<std::remove_pointer_t<decltype(val)>>, false, 1>(b, val, x, y); break;
            case 1: launch_spmm_v<PT, std::remove_const_t<std::remove_pointer_t<decltype(val)>>, true, 1>(b, val, x, y); break;
            case 2: launch_spmm_v<PT, std::remove_const_t<std::remove_pointer_t<decltype(val)>>, false, 4>(b, val, x, y); break;
            default: launch_spmm_v<PT, std::remove_const_t<std::remove_pointer_t<decltype(val)>>, true, 4>(b, val, x, y); break;
        }
    };
    if (b.fp64) go((const double *)c->d_val64.ptr);
    else go((const float *)c->d_val32.ptr);
}

// out = (1 - K) x (sub) or K x / O P0 V~ x (with_g false: the driving
// term).  lowp: the two intermediate panels in FP32 (inner iterations of the
// mixed tier); otherwise FP64.
template <class PT>
void op_apply_t(Batch &b, const double *x, double *out, bool with_g, bool sub) {
    wpcd_ctx *c = b.c;
    PT *T1 = (PT *)b.T1, *T2 = (PT *)b.T2;
    {
        TimedLaunch tl(c->timer, c->stream, "apply_vt", WPCD_TIME_SOLVE);
        if (with_g) launch_block_apply<true, false>(b, 0, x, nullptr, T1);
        else launch_block_apply<false, false>(b, 0, x, nullptr, T1);
        WPCD_HIP(hipGetLastError());
    }
    {
        TimedLaunch tl(c->timer, c->stream, "spmm", WPCD_TIME_SOLVE);
        launch_spmm<PT>(b, T1, T2, b.spmm_cfg);
    }
    {
        TimedLaunch tl(c->timer, c->stream, "apply_o", WPCD_TIME_SOLVE);
        if (sub) launch_block_apply<false, true>(b, 1, T2, x, out);
        else launch_block_apply<false, false>(b, 1, T2, nullptr, out);
        WPCD_HIP(hipGetLastError());
    }
}

void op_apply(Batch &b, const double *x, double *out, bool with_g, bool sub, bool lowp = false) {
    if (lowp) op_apply_t<float>(b, x, out, with_g, sub);
    else op_apply_t<double>(b, x, out, with_g, sub);
}

// Rows per thread of the vector kernels: NR in {1, 2, 4}.
template <class F>
void with_nr(int nr, F &&f) {
    switch (nr) {
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 2: f(std::integral_constant<int, 2>{}); break;
        default: f(std::integral_constant<int, 4>{}); break;
    }
}

// Stage 1 of the cross-chunk reduction of npair partial sums -> b.out2.
void reduce_stage1(Batch &b, int npair) {
    hipLaunchKernelGGL(k_reduce_stage1, dim3(cdiv(npair, 32), b.nsplit), dim3(256), 0,
                       b.c->stream, b.partial, b.nchunk, npair, b.out2);
}

void reduce_partials(Batch &b, int nvec, double *h, double *H, int kcol, int accumulate) {
    wpcd_ctx *c = b.c;
    TimedLaunch tl(c->timer, c->stream, "gmres_reduce", WPCD_TIME_SOLVE);
    if (b.nchunk <= kFusedChunks) {
        hipLaunchKernelGGL(k_dots_final, dim3(cdiv(nvec * b.nE, 8)), dim3(256), 0, c->stream,
                           b.partial, b.nchunk, nvec, b.nE, h, H, b.m, kcol, accumulate);
        WPCD_HIP(hipGetLastError());
        return;
    }
    reduce_stage1(b, nvec * b.nE);
    hipLaunchKernelGGL(k_dots_reduce, dim3(cdiv(nvec * b.nE, 256)), dim3(256), 0, c->stream,
                       b.out2, b.nsplit, nvec, b.nE, h, H, b.m, kcol, accumulate);
    WPCD_HIP(hipGetLastError());
}

// dots of w against nvec vectors starting at Vb -> h (reduced), optional H column.
void dots(Batch &b, const double *Vb, int nvec, const double *w, double *h, double *H, int kcol,
          int accumulate) {
    wpcd_ctx *c = b.c;
    {
        TimedLaunch tl(c->timer, c->stream, "gmres_dots", WPCD_TIME_SOLVE);
        with_nr(b.nr, [&](auto nr) {
            hipLaunchKernelGGL(k_vdots<decltype(nr)::value>, dim3(b.nchunk), dim3(256), 0,
                               c->stream, Vb, b.vstride, nvec, w, b.M, b.nE, b.nEp, b.partial);
        });
        WPCD_HIP(hipGetLastError());
    }
    reduce_partials(b, nvec, h, H, kcol, accumulate);
}

// w -= sum h V over nvec vectors, then DOTS: second-pass partial dots, or
// NORM: |w|^2 partials.
template <bool DOTS, bool NORM>
void vupdate(Batch &b, int nvec, double *w) {
    wpcd_ctx *c = b.c;
    TimedLaunch tl(c->timer, c->stream, "gmres_update", WPCD_TIME_SOLVE);
    with_nr(b.nr, [&](auto nr) {
        hipLaunchKernelGGL((k_vupdate<decltype(nr)::value, DOTS, NORM>), dim3(b.nchunk), dim3(256),
                           0, c->stream, b.Vb, b.vstride, nvec, b.h, b.M, b.nE, b.nEp, w,
                           b.partial);
    });
    WPCD_HIP(hipGetLastError());
}

// One Arnoldi step k: w = (1 - K) v_k, classical Gram-Schmidt in two passes
// (the second pass's dots fused into the first update, |w|^2 into the
// second), then the Givens update of every energy and w /= |w|.  In the
// mixed tier the operator's intermediate panels are FP32 here; the true
// residual that starts each cycle is formed with FP64 panels, so a restart
// is a step of iterative refinement.
void iteration(Batch &b, int k, double tol) {
    wpcd_ctx *c = b.c;
    hipStream_t s = c->stream;
    const int64_t vec = b.vstride;
    double *vk = b.Vb + (int64_t)k * vec;
    double *w = b.Vb + (int64_t)(k + 1) * vec;
    op_apply(b, vk, w, true, true, b.lowp);
    dots(b, b.Vb, k + 1, w, b.h, b.H, k, 0);
    vupdate<true, false>(b, k + 1, w);
    reduce_partials(b, k + 1, b.h, b.H, k, 1);
    vupdate<false, true>(b, k + 1, w);
    TimedLaunch tl(c->timer, s, "gmres_givens", WPCD_TIME_SOLVE);
    const size_t lds = (256 + (size_t)b.nE * (b.m + 1) * 2) * sizeof(double);
    if (b.nchunk <= kFusedChunks) {
        // norms reduced by every workgroup, w scaled in the same launch
        const int nb = (int)std::min<int64_t>(cdiv(b.M * b.nE, 1024), 512);
        hipLaunchKernelGGL(k_norm_givens, dim3(nb), dim3(256), lds, s, b.partial, b.nchunk, b.H,
                           b.nE, b.m, k, tol, b.S, b.inv, w, b.M);
    } else {
        hipLaunchKernelGGL(k_norm_givens, dim3(1), dim3(256), lds, s, b.partial, b.nchunk, b.H,
                           b.nE, b.m, k, tol, b.S, b.inv, nullptr, b.M);
        hipLaunchKernelGGL(k_scale, dim3(cdiv(b.M * b.nE, 256)), dim3(256), 0, s, b.inv, b.M,
                           b.nE, w);
    }
    WPCD_HIP(hipGetLastError());
}

// Capture iterations [k, k + n) of this batch as one executable graph.
hipGraphExec_t capture_group(Batch &b, int k, int n, double tol) {
    hipStream_t s = b.c->stream;
    hipGraph_t g = nullptr;
    WPCD_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
        for (int i = 0; i < n; ++i) iteration(b, k + i, tol);
    } catch (...) {
        hipGraph_t tmp = nullptr;
        (void)hipStreamEndCapture(s, &tmp);
        if (tmp) (void)hipGraphDestroy(tmp);
        throw;
    }
    WPCD_HIP(hipStreamEndCapture(s, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    WPCD_HIP(e);
    return ex;
}

// Graphs of a batch are valid while every pointer, size and constant the
// captured launches use is unchanged: all of them form the key.
IterGraphs *graphs_for(Batch &b, double tol, int check_every) {
    wpcd_ctx *c = b.c;
    std::vector<uint64_t> key = {
        (uint64_t)b.Vb, (uint64_t)b.T1, (uint64_t)b.G, (uint64_t)b.H, (uint64_t)b.partial,
        (uint64_t)b.h, (uint64_t)b.inv, (uint64_t)b.S.st, (uint64_t)b.S.cs, (uint64_t)b.S.sn,
        (uint64_t)b.S.g, (uint64_t)c->d_rowptr.ptr, (uint64_t)c->d_col.ptr,
        (uint64_t)(b.fp64 ? (void *)c->d_val64.ptr : (void *)c->d_val32.ptr),
        (uint64_t)b.nE, (uint64_t)b.m, (uint64_t)b.M, (uint64_t)b.fp64, (uint64_t)b.lowp,
        (uint64_t)b.bf16,
        (uint64_t)b.apply_cfg, (uint64_t)b.spmm_cfg,
        (uint64_t)b.nr, (uint64_t)b.nchunk, (uint64_t)b.nsplit, (uint64_t)b.out2,
        (uint64_t)c->np, (uint64_t)c->nq, (uint64_t)c->nch,
        (uint64_t)b.vstride};
    uint64_t tb;
    std::memcpy(&tb, &tol, sizeof tb);
    key.push_back(tb);
    for (const wpcd_ctx *g : {(const wpcd_ctx *)c, (const wpcd_ctx *)b.cm}) {
        if (!g) continue;
        key.push_back((uint64_t)g->nch);
        for (int a = 0; a < g->nch; ++a) {
            key.push_back((uint64_t)g->waves[g->ch_wave[a]].Vt.ptr);
            key.push_back((uint64_t)g->waves[g->ch_wave[a]].O.ptr);
        }
    }
    key.push_back((uint64_t)b.M_F);
    key.push_back((uint64_t)c->d_perm.ptr);   // the tiled SpMM's row order
    for (auto &g : c->graphs)
        if (g.key == key) return &g;
    if (c->graphs.size() >= 8) {
        c->graphs.front().release();
        c->graphs.erase(c->graphs.begin());
    }
    c->graphs.emplace_back();
    IterGraphs &g = c->graphs.back();
    g.key = key;
    g.exec.assign(cdiv(b.m, check_every), nullptr);
    return &g;
}

// Microseconds per launch of f (one warm-up, then reps timed launches).
template <class F>
double time_launches(hipStream_t s, F &&f, int reps = 3) {
    hipEvent_t a, z;
    WPCD_HIP(hipEventCreate(&a));
    WPCD_HIP(hipEventCreate(&z));
    f();
    WPCD_HIP(hipEventRecord(a, s));
    for (int i = 0; i < reps; ++i) f();
    WPCD_HIP(hipEventRecord(z, s));
    WPCD_HIP(hipEventSynchronize(z));
    float ms = 0.f;
    WPCD_HIP(hipEventElapsedTime(&ms, a, z));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(z);
    return 1e3 * ms / reps;
}

// Launch shapes of this batch (buffers must be allocated; their contents
// are only read, or written where they are scratch).
void choose_shapes(Batch &b, int m) {
    wpcd_ctx *c = b.c;
    char key[64];
    std::snprintf(key, sizeof key, "np=%d nq=%d W=%d nch=%d", c->np, c->nq, b.W, c->nch);
    int heur = 2;
    for (int i = 0; i < 4; ++i)   // vector-ALU tilings; the matrix-core one is measured only
        if (apply_blocks(c, b.W, i) >= 512) {
            heur = i;
            break;
        }
    b.apply_cfg = tune_pick(c, "block_apply", key, kApplyCfg, heur, [&](int i) {
        b.apply_cfg = i;
        return time_launches(c->stream, [&] {
            launch_block_apply<true, false>(b, 0, (const double *)b.X, nullptr, b.T1);
            WPCD_HIP(hipGetLastError());
        });
    });
    std::snprintf(key, sizeof key, "M=%lld nEp=%d", (long long)b.M, b.nEp);
    heur = 0;
    for (int i = 2; i >= 0; --i)
        if (cdiv(b.M, chunk_rows_of(b.nEp, kNrCand[i])) >= 1024) {
            heur = i;
            break;
        }
    const int nvec = std::max(1, std::min(m, 8));   // w = basis vector nvec <= m
    const int ch = tune_pick(c, "vector_rows", key, 3, heur, [&](int i) {
        b.set_chunks(kNrCand[i]);
        // one Gram-Schmidt step's vector work as in iteration(): the dots, the
        // update fused with the second-pass dots, the update fused with the
        // norm, and their reductions (w is basis vector nvec: scratch here)
        double *w = b.Vb + (int64_t)nvec * b.vstride;
        return time_launches(c->stream, [&] {
            with_nr(b.nr, [&](auto nr) {
                hipLaunchKernelGGL(k_vdots<decltype(nr)::value>, dim3(b.nchunk), dim3(256), 0,
                                   c->stream, b.Vb, b.vstride, nvec, w, b.M, b.nE, b.nEp,
                                   b.partial);
            });
            reduce_partials(b, nvec, b.h, nullptr, 0, 0);
            vupdate<true, false>(b, nvec, w);
            reduce_partials(b, nvec, b.h, nullptr, 0, 0);
            vupdate<false, true>(b, nvec, w);
            WPCD_HIP(hipGetLastError());
        }, 5);
    });
    b.set_chunks(kNrCand[ch]);
    // P0 SpMM: the variant for the inner iterations' panel type
    std::snprintf(key, sizeof key, "nnz=%lld nch=%d W=%d %s%s", (long long)c->nnz, b.spmm_nch, b.W,
                  b.fp64 ? "f64" : "f32", b.lowp ? " lowp" : "");
    // candidates: the s-wave kernel and the reduced system's scalar CSR have
    // no unrolled form
    std::vector<int> cand = b.cm ? std::vector<int>{0, 1, 4, 5, 6}
                            : c->nch > 1 ? std::vector<int>{0, 1, 2, 3, 4, 5, 6}
                                         : std::vector<int>{0, 1, 4, 5, 6};
    ensure_perm(c);   // before any capture
    const int pick = tune_pick(c, "spmm", key, (int)cand.size(), 0, [&](int i) {
        return time_launches(c->stream, [&] {
            if (b.lowp) launch_spmm<float>(b, (const float *)b.T1, (float *)b.T2, cand[i]);
            else launch_spmm<double>(b, b.T1, b.T2, cand[i]);
        });
    });
    b.spmm_cfg = cand[pick];
}

}  // namespace

// Solve the batch of energies already validated by the caller.
// idx0: entrance row per energy.
// |B| of every energy: the residual normalisation of the cycles (host st
// and the device state's st[1]).
void rhs_norms(Batch &b, std::vector<double> &st) {
    const int nE = b.nE;
    hipStream_t s = b.c->stream;
    dots(b, b.B, 1, b.B, b.h, nullptr, 0, 0);
    std::vector<double> h0(2 * nE);
    WPCD_HIP(hipMemcpyAsync(h0.data(), b.h, 2 * nE * sizeof(double), hipMemcpyDeviceToHost, s));
    WPCD_HIP(hipStreamSynchronize(s));
    st.assign(nE * kSt, 0.0);
    for (int e = 0; e < nE; ++e) st[e * kSt + 1] = std::sqrt(h0[2 * e]);
    WPCD_HIP(hipMemcpyAsync(b.S.st, st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice, s));
}

// One batch of energies of one system through the restarted GMRES.
struct GmresRun {
    Batch b;
    std::vector<double> st, rn;   // per-energy state (st[1] = |B|), residual norms^2
    GmresOut *out = nullptr;
    int max_iter = 0;
    double tol = 0.0;
    bool err_est = false;
    std::vector<int64_t> idx0;
};

GmresRun *gmres_run_new() { return new GmresRun(); }
void gmres_run_delete(GmresRun *r) { delete r; }

// Iterations [k, k + n) of several batches (on their own streams, one
// device) as one executable graph: the first stream forks to the others and
// joins them at the end, so the batches' launches form parallel branches.
hipGraphExec_t capture_multi(const std::vector<Batch *> &bs, int k, int n, double tol) {
    hipStream_t s0 = bs[0]->c->stream;
    hipGraph_t g = nullptr;
    std::vector<hipEvent_t> evs;
    auto cleanup = [&] {
        for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    };
    WPCD_HIP(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
    try {
        hipEvent_t fork;
        WPCD_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        evs.push_back(fork);
        WPCD_HIP(hipEventRecord(fork, s0));
        for (size_t r = 1; r < bs.size(); ++r) WPCD_HIP(hipStreamWaitEvent(bs[r]->c->stream, fork, 0));
        for (Batch *b : bs)
            for (int i = 0; i < n; ++i) iteration(*b, k + i, tol);
        for (size_t r = 1; r < bs.size(); ++r) {
            hipEvent_t join;
            WPCD_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
            evs.push_back(join);
            WPCD_HIP(hipEventRecord(join, bs[r]->c->stream));
            WPCD_HIP(hipStreamWaitEvent(s0, join, 0));
        }
    } catch (...) {
        hipGraph_t tmp = nullptr;
        (void)hipStreamEndCapture(s0, &tmp);
        if (tmp) (void)hipGraphDestroy(tmp);
        cleanup();
        throw;
    }
    const hipError_t ec = hipStreamEndCapture(s0, &g);
    cleanup();
    WPCD_HIP(ec);
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    WPCD_HIP(e);
    return ex;
}

// Restarted GMRES cycles of one or several batches in lockstep: from
// x = b.X with r = b.R = b.B - (1 - K) x until every energy's true relative
// residual |r| / |B| (st[1] = |B|) is <= tol or max_iter iterations are
// spent.  All batches start a cycle together and run their groups of
// check_every iterations together; a group of several batches replays one
// graph holding all of them (captured on first use per set of batches),
// a single batch its own graph; convergence is read back after each group,
// and a batch whose energies have all converged leaves the cycle.
void gmres_cycles(std::vector<GmresRun *> &runs) {
    const int check_every = 4;
    const int m = runs[0]->b.m;
    for (GmresRun *r : runs)
        WPCD_REQUIRE(r->b.m == m, WPCD_E_INVALID, "batches solved together need one krylov_dim");
    // A batch whose unconverged energies have not halved their smallest
    // true residual so far in kStagCycles consecutive restart cycles stops
    // (those energies are marked stagnated): restarted GMRES that gains
    // that little per cycle, or has reached the rounding floor, would only
    // spend the remaining iterations.
    constexpr int kStagCycles = 2;
    struct State {
        GmresRun *r;
        std::vector<double> sth;
        std::vector<double> best;   // smallest true residual so far, per energy
        int total = 0;
        int idle = 0;               // consecutive cycles without progress
        bool all_done = false, in_cycle = false, started = false;
        IterGraphs *graphs = nullptr;
    };
    std::vector<State> xs;
    bool graphs_ok = true;
    for (GmresRun *r : runs) {
        State x;
        x.r = r;
        x.sth.assign((size_t)r->b.nE * kSt, 0.0);
        x.best.assign(r->b.nE, std::numeric_limits<double>::infinity());
        r->out->iters.assign(r->b.nE, 0);
        r->out->stag.assign(r->b.nE, 0);
        r->out->resid.assign(r->b.nE, 1.0);
        wpcd_ctx *c = r->b.c;
        graphs_ok &= c->use_graphs && !(c->timer.enabled & WPCD_TIME_SOLVE) &&
                     c->device == runs[0]->b.c->device;
        xs.push_back(std::move(x));
    }
    if (graphs_ok)
        for (State &x : xs) x.graphs = graphs_for(x.r->b, x.r->tol, check_every);
    // events joining the other streams' pending work into a multi-batch graph launch
    struct Joins {
        std::vector<hipEvent_t> e;
        ~Joins() {
            for (hipEvent_t v : e)
                if (v) (void)hipEventDestroy(v);
        }
        hipEvent_t &operator[](size_t i) { return e[i]; }
    } joins;
    joins.e.assign(runs.size(), nullptr);
    if (graphs_ok && runs.size() > 1)
        for (size_t i = 1; i < runs.size(); ++i)
            WPCD_HIP(hipEventCreateWithFlags(&joins.e[i], hipEventDisableTiming));
    auto active = [](const State &x) { return x.total < x.r->max_iter && !x.all_done; };
    for (;;) {
        bool any = false;
        for (State &x : xs) any |= active(x);
        if (!any) break;
        // cycle start from r
        for (State &x : xs) {
            x.started = x.in_cycle = active(x);
            if (!x.started) continue;
            Batch &b = x.r->b;
            hipStream_t s = b.c->stream;
            const int nE = b.nE;
            dots(b, b.R, 1, b.R, b.h, nullptr, 0, 0);
            hipLaunchKernelGGL(k_cycle_start, dim3(cdiv(nE, 64)), dim3(64), 0, s, b.h, nE, m,
                               x.r->tol, b.S, b.inv);
            hipLaunchKernelGGL(k_scale, dim3(cdiv(b.M * nE, 256)), dim3(256), 0, s, b.inv, b.M, nE,
                               b.R);
            WPCD_HIP(hipMemcpyAsync(b.Vb, b.R, b.vstride * sizeof(double), hipMemcpyDeviceToDevice,
                                    s));
            WPCD_HIP(hipMemsetAsync(b.H, 0, (size_t)nE * (m + 1) * m * 2 * sizeof(double), s));
        }
        for (int k = 0; k < m;) {
            std::vector<State *> in;
            for (State &x : xs)
                if (x.in_cycle) in.push_back(&x);
            if (in.empty()) break;
            bool full = graphs_ok;
            hipStream_t rb_stream = nullptr;   // read-back stream when one graph ran them all
            std::vector<int> kg(in.size());
            for (size_t i = 0; i < in.size(); ++i) {
                kg[i] = std::min({check_every, m - k, in[i]->r->max_iter - in[i]->total});
                full &= kg[i] == check_every;
            }
            if (full && in.size() == 1) {
                hipGraphExec_t &ex = in[0]->graphs->exec[k / check_every];
                if (!ex) ex = capture_group(in[0]->r->b, k, check_every, in[0]->r->tol);
                WPCD_HIP(hipGraphLaunch(ex, in[0]->r->b.c->stream));
            } else if (full) {
                // one graph for this set of batches at this k
                std::vector<uint64_t> key = {(uint64_t)(k / check_every), (uint64_t)in.size()};
                for (State *x : in) {
                    key.push_back(0x9e37ull);
                    key.insert(key.end(), x->graphs->key.begin(), x->graphs->key.end());
                }
                wpcd_ctx *c0 = in[0]->r->b.c;
                hipGraphExec_t ex = nullptr;
                for (auto &mg : c0->multi_graphs)
                    if (mg.key == key) ex = mg.exec;
                if (!ex) {
                    std::vector<Batch *> bs;
                    for (State *x : in) bs.push_back(&x->r->b);
                    ex = capture_multi(bs, k, check_every, in[0]->r->tol);
                    if (c0->multi_graphs.size() >= 64) {
                        (void)hipGraphExecDestroy(c0->multi_graphs.front().exec);
                        c0->multi_graphs.erase(c0->multi_graphs.begin());
                    }
                    c0->multi_graphs.push_back({key, ex});
                }
                // the graph runs on the first stream: it starts after the
                // other streams' pending work, and the read-backs below go
                // on the first stream after it
                for (size_t i = 1; i < in.size(); ++i) {
                    WPCD_HIP(hipEventRecord(joins[i], in[i]->r->b.c->stream));
                    WPCD_HIP(hipStreamWaitEvent(c0->stream, joins[i], 0));
                }
                WPCD_HIP(hipGraphLaunch(ex, c0->stream));
                rb_stream = c0->stream;
            } else {
                for (size_t i = 0; i < in.size(); ++i)
                    for (int t = 0; t < kg[i]; ++t) iteration(in[i]->r->b, k + t, in[i]->r->tol);
            }
            for (size_t i = 0; i < in.size(); ++i) {
                State &x = *in[i];
                x.total += kg[i];
                WPCD_HIP(hipMemcpyAsync(x.sth.data(), x.r->b.S.st, x.sth.size() * sizeof(double),
                                        hipMemcpyDeviceToHost,
                                        rb_stream ? rb_stream : x.r->b.c->stream));
            }
            for (State *x : in) WPCD_HIP(hipStreamSynchronize(x->r->b.c->stream));
            if (rb_stream) WPCD_HIP(hipStreamSynchronize(rb_stream));
            for (State *x : in) {
                bool done = true;
                for (int e = 0; e < x->r->b.nE; ++e) done &= x->sth[e * kSt + 3] != 0.0;
                if (done || x->total >= x->r->max_iter) x->in_cycle = false;
            }
            k += check_every;
        }
        // end of the cycle: x from the least-squares solution, true residual
        for (State &x : xs) {
            if (!x.started) continue;
            Batch &b = x.r->b;
            hipStream_t s = b.c->stream;
            const int nE = b.nE;
            const int64_t vec = b.M * b.W;
            hipLaunchKernelGGL(k_trisolve, dim3(cdiv(nE, 64)), dim3(64), 0, s, b.H, nE, m, b.S, b.y,
                               b.kuse);
            hipLaunchKernelGGL(k_xupdate, dim3(cdiv(b.M * nE, 256)), dim3(256), 0, s, b.Vb,
                               b.vstride, b.y, b.kuse, m, b.M, nE, b.X);
            WPCD_HIP(hipGetLastError());
            // per-energy iteration count: columns used in this cycle
            WPCD_HIP(hipMemcpyAsync(x.sth.data(), b.S.st, x.sth.size() * sizeof(double),
                                    hipMemcpyDeviceToHost, s));
            op_apply(b, b.X, b.R, true, true);
            hipLaunchKernelGGL(k_sub_from, dim3(cdiv(vec, 256)), dim3(256), 0, s, b.B, vec, b.R);
            dots(b, b.R, 1, b.R, b.h, nullptr, 0, 0);
            x.r->rn.assign(2 * nE, 0.0);
            WPCD_HIP(hipMemcpyAsync(x.r->rn.data(), b.h, 2 * nE * sizeof(double),
                                    hipMemcpyDeviceToHost, s));
        }
        for (State &x : xs)
            if (x.started) WPCD_HIP(hipStreamSynchronize(x.r->b.c->stream));
        for (State &x : xs) {
            if (!x.started) continue;
            const int nE = x.r->b.nE;
            std::vector<int> &iters = x.r->out->iters;
            std::vector<double> &resid = x.r->out->resid;
            x.all_done = true;
            bool progress = false;
            for (int e = 0; e < nE; ++e) {
                if (resid[e] > x.r->tol) iters[e] += (int)x.sth[e * kSt + 4];
                const double bn = x.r->st[e * kSt + 1];
                resid[e] = bn > 0 ? std::sqrt(x.r->rn[2 * e]) / bn : 0.0;
                if (resid[e] > x.r->tol) {
                    x.all_done = false;
                    if (resid[e] < 0.5 * x.best[e]) progress = true;
                }
                if (resid[e] < x.best[e]) x.best[e] = resid[e];
            }
            x.idle = progress ? 0 : x.idle + 1;
            if (!x.all_done && x.idle >= kStagCycles) {
                x.all_done = true;
                for (int e = 0; e < nE; ++e)
                    if (resid[e] > x.r->tol) x.r->out->stag[e] = 1;
            }
        }
    }
}

// Rows of the batch's vectors and the SpMM's CSR (see Batch).
void set_layout(Batch &b) {
    wpcd_ctx *c = b.c;
    b.cm = c->reduced ? c->minor : nullptr;
    b.M_F = (int64_t)c->nch * c->nq * c->np;
    b.M = b.M_F + (b.cm ? (int64_t)b.cm->nch * b.cm->nq * b.cm->np : 0);
    b.spmm_rows = c->reduced ? (int)c->red_rows : c->np * c->nq;
    b.spmm_nch = c->reduced ? 1 : c->nch;
}

void gmres_setup(GmresRun &run, wpcd_ctx *c, const std::vector<double> &E,
                 const std::vector<int64_t> &idx0, int prec, int m, int max_iter, double tol,
                 WarmFill warm, void *warm_user, GmresOut &out, bool err_est,
                 const std::vector<double> *ebin) {
    run.out = &out;
    run.max_iter = max_iter;
    run.tol = tol;
    run.err_est = err_est;
    run.idx0 = idx0;
    const bool fp64 = prec == WPCD_FP64;
    std::vector<int> &edge_flag = out.edge;
    const int nE = (int)E.size();
    // the Givens kernel's LDS column stage can exceed the 64 KB default
    WPCD_HIP(hipFuncSetAttribute((const void *)k_norm_givens,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024));
    Batch &b = run.b;
    b = Batch{};
    b.c = c;
    b.nE = nE;
    b.W = 2 * nE;
    b.nEp = 1;
    while (b.nEp < nE) b.nEp <<= 1;
    b.Wp = 2 * b.nEp;
    b.m = m;
    set_layout(b);
    b.fp64 = fp64;
    b.lowp = prec == WPCD_MIXED_REFINE || prec == WPCD_MIXED_BF16;
    b.bf16 = prec == WPCD_MIXED_BF16;
    const int64_t vec = b.M * b.W;   // doubles per batched vector
    b.vstride = vec;
    const int max_chunks = cdiv(b.M, chunk_rows_of(b.nEp, 1));
    c->d_G.reserve(vec);
    c->d_X.reserve(vec);
    c->d_B.reserve(vec);
    c->d_T1.reserve(2 * vec);
    c->d_V.reserve((size_t)(m + 1) * vec);
    c->d_Hess.reserve((size_t)nE * (m + 1) * m * 2);
    c->d_partial.reserve((size_t)(max_chunks + kMaxSplit) * (m + 1) * nE * 2);
    c->d_W.reserve(vec);
    if (err_est) c->d_X2.reserve(vec);
    c->d_misc.reserve((size_t)nE * (kSt + 2 * m + 2 * (m + 1) + m + 4) + (size_t)(m + 1) * nE * 2 +
                      (size_t)nE * m * 2 + 64);
    c->d_flag.reserve(2 * nE + 4);
    c->d_idx.reserve(nE);
    b.G = c->d_G.ptr;
    b.X = c->d_X.ptr;
    b.B = c->d_B.ptr;
    b.T1 = c->d_T1.ptr;
    b.T2 = c->d_T1.ptr + vec;
    b.R = c->d_W.ptr;
    b.Vb = c->d_V.ptr;
    b.H = c->d_Hess.ptr;
    b.partial = c->d_partial.ptr;
    b.out2 = c->d_partial.ptr + (size_t)max_chunks * (m + 1) * nE * 2;
    double *ms = c->d_misc.ptr;
    b.S.st = ms;
    ms += nE * kSt;
    b.S.cs = ms;
    ms += nE * m;
    b.S.sn = ms;
    ms += 2 * nE * m;
    b.S.g = ms;
    ms += 2 * nE * (m + 1);
    b.h = ms;
    ms += 2 * (m + 1) * nE;
    b.inv = ms;
    ms += nE;
    b.y = ms;
    ms += 2 * nE * m;
    int32_t *flag = c->d_flag.ptr;   // [0, nE): resolvent edge flags
    b.kuse = flag + nE;              // [nE, 2 nE): GMRES columns used

    hipStream_t s = c->stream;
    choose_shapes(b, m);
    // energies
    double *dE = c->d_T1.ptr;   // scratch: T1 not yet in use
    WPCD_HIP(hipMemcpyAsync(dE, E.data(), nE * sizeof(double), hipMemcpyHostToDevice, s));
    WPCD_HIP(hipMemsetAsync(flag, 0, nE * sizeof(int32_t), s));
    if (ebin) {
        // on-shell energy intervals [E1, E2] per energy (after dE in the scratch)
        double *dB = dE + nE;
        WPCD_HIP(hipMemcpyAsync(dB, ebin->data(), 2 * nE * sizeof(double), hipMemcpyHostToDevice,
                                s));
        TimedLaunch tl(c->timer, s, "resolvent", WPCD_TIME_SOLVE);
        for (const Part &pt : {Part{c, 0}, Part{b.cm, b.M_F}}) {
            if (!pt.g) continue;
            const wpcd_ctx *g = pt.g;
            ChPtrs ep{};
            for (int a = 0; a < g->nch; ++a) ep.p[a] = g->waves[g->ch_wave[a]].eps.ptr;
            const int64_t rows = (int64_t)g->nch * g->nq * g->np;
            hipLaunchKernelGGL(k_resolvent_avg, dim3(cdiv(rows * nE, 256)), dim3(256), 0, s,
                               g->d_q.ptr, g->np, g->nq, g->nch, nE, dB, ep, b.G + pt.off * b.W);
        }
        WPCD_HIP(hipGetLastError());
    } else {
        TimedLaunch tl(c->timer, s, "resolvent", WPCD_TIME_SOLVE);
        for (const Part &pt : {Part{c, 0}, Part{b.cm, b.M_F}}) {
            if (!pt.g) continue;
            const wpcd_ctx *g = pt.g;
            ChPtrs ep{};
            for (int a = 0; a < g->nch; ++a) ep.p[a] = g->waves[g->ch_wave[a]].eps.ptr;
            const int64_t rows = (int64_t)g->nch * g->nq * g->np;
            hipLaunchKernelGGL(k_resolvent, dim3(cdiv(rows * nE, 256)), dim3(256), 0, s,
                               g->d_q.ptr, g->np, g->nq, g->nch, nE, dE, ep,
                               b.G + pt.off * b.W, flag);
        }
        WPCD_HIP(hipGetLastError());
    }
    edge_flag.assign(nE, 0);
    WPCD_HIP(hipMemcpyAsync(edge_flag.data(), flag, nE * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    // right-hand side b = O P0 V~ e0
    WPCD_HIP(hipMemsetAsync(b.X, 0, vec * sizeof(double), s));
    WPCD_HIP(hipMemcpyAsync(c->d_idx.ptr, idx0.data(), nE * sizeof(int64_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_unit, dim3(1), dim3(64), 0, s, c->d_idx.ptr, nE, b.X);
    WPCD_HIP(hipGetLastError());
    op_apply(b, b.X, b.B, false, false);
    std::vector<double> &st = run.st;
    rhs_norms(b, st);
    out.warm.assign(nE, 0);
    out.r0.assign(nE, 1.0);
    if (warm) {
        // proposed x0, judged by the minimal initial residual over its scalings
        warm(c, warm_user, b.X, nE);
        op_apply(b, b.X, b.R, true, true);
        dots(b, b.R, 1, b.B, b.h, nullptr, 0, 0);
        dots(b, b.R, 1, b.R, b.h + 2 * nE, nullptr, 0, 0);
        {
            TimedLaunch tl(c->timer, s, "warm_judge", WPCD_TIME_SOLVE);
            hipLaunchKernelGGL(k_warm_alpha, dim3(cdiv(nE, 64)), dim3(64), 0, s, b.h, b.h + 2 * nE,
                               nE, b.y);
            hipLaunchKernelGGL(k_warm_apply, dim3(cdiv(b.M * nE, 256)), dim3(256), 0, s, b.y, b.M,
                               nE, b.B, b.X, b.R);
            WPCD_HIP(hipGetLastError());
        }
        dots(b, b.R, 1, b.R, b.h, nullptr, 0, 0);
        std::vector<double> al(2 * nE), rr(2 * nE);
        WPCD_HIP(hipMemcpyAsync(al.data(), b.y, 2 * nE * sizeof(double), hipMemcpyDeviceToHost, s));
        WPCD_HIP(hipMemcpyAsync(rr.data(), b.h, 2 * nE * sizeof(double), hipMemcpyDeviceToHost, s));
        WPCD_HIP(hipStreamSynchronize(s));
        for (int e = 0; e < nE; ++e) {
            out.warm[e] = (al[2 * e] != 0.0 || al[2 * e + 1] != 0.0) ? 1 : 0;
            const double bn = st[e * kSt + 1];
            out.r0[e] = bn > 0 ? std::sqrt(std::max(rr[2 * e], 0.0)) / bn : 0.0;
        }
    } else {
        // x = 0, r = b
        WPCD_HIP(hipMemsetAsync(b.X, 0, vec * sizeof(double), s));
        WPCD_HIP(hipMemcpyAsync(b.R, b.B, vec * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
}

void gmres_finish(GmresRun &run) {
    if (!run.err_est) return;
    Batch &b = run.b;
    wpcd_ctx *c = b.c;
    hipStream_t s = c->stream;
    const int nE = b.nE;
    const int64_t vec = b.M * b.W;
    const std::vector<int64_t> &idx0 = run.idx0;
    GmresOut &out = *run.out;
    const int max_iter = run.max_iter;
    // Error against the FP64 path: the residual of x with the FP64 P0 values,
    // r64 = b64 - (1 - K64) x, and the correction d from (1 - K) d = r64
    // solved in this tier to a relative residual of 1e-4; d ~ x64 - x, so its
    // on-shell component is the amplitude's difference from the FP64 solution
    // (to first order in the FP32 rounding of P0).  x itself is kept.
    const bool fp64_saved = b.fp64;
    double *X2 = c->d_X2.ptr;
    WPCD_HIP(hipMemcpyAsync(X2, b.X, vec * sizeof(double), hipMemcpyDeviceToDevice, s));
    WPCD_HIP(hipMemsetAsync(b.X, 0, vec * sizeof(double), s));
    hipLaunchKernelGGL(k_unit, dim3(1), dim3(64), 0, s, c->d_idx.ptr, nE, b.X);
    WPCD_HIP(hipGetLastError());
    b.fp64 = true;
    op_apply(b, b.X, b.B, false, false);          // b64
    op_apply(b, X2, b.R, true, true);             // (1 - K64) x
    hipLaunchKernelGGL(k_sub_from, dim3(cdiv(vec, 256)), dim3(256), 0, s, b.B, vec, b.R);
    WPCD_HIP(hipGetLastError());
    b.fp64 = fp64_saved;
    WPCD_HIP(hipMemcpyAsync(b.B, b.R, vec * sizeof(double), hipMemcpyDeviceToDevice, s));
    WPCD_HIP(hipMemsetAsync(b.X, 0, vec * sizeof(double), s));
    GmresOut o2;
    GmresRun r2;
    r2.b = b;
    r2.out = &o2;
    r2.max_iter = std::max(max_iter, 64);
    r2.tol = 1e-4;
    rhs_norms(r2.b, r2.st);
    std::vector<GmresRun *> one{&r2};
    gmres_cycles(one);
    out.dU.assign(2 * nE, 0.0);
    out.U.assign(2 * nE, 0.0);
    for (int e = 0; e < nE; ++e) {
        const int64_t off = (idx0[e] * nE + e) * 2;
        WPCD_HIP(hipMemcpyAsync(&out.dU[2 * e], b.X + off, 2 * sizeof(double),
                                hipMemcpyDeviceToHost, s));
        WPCD_HIP(hipMemcpyAsync(&out.U[2 * e], X2 + off, 2 * sizeof(double),
                                hipMemcpyDeviceToHost, s));
    }
    WPCD_HIP(hipMemcpyAsync(b.X, X2, vec * sizeof(double), hipMemcpyDeviceToDevice, s));
    WPCD_HIP(hipStreamSynchronize(s));
}

void gmres_batch(wpcd_ctx *c, const std::vector<double> &E, const std::vector<int64_t> &idx0,
                 int prec, int m, int max_iter, double tol, WarmFill warm, void *warm_user,
                 GmresOut &out, bool err_est, const std::vector<double> *ebin) {
    GmresRun run;
    gmres_setup(run, c, E, idx0, prec, m, max_iter, tol, warm, warm_user, out, err_est, ebin);
    std::vector<GmresRun *> one{&run};
    gmres_cycles(one);
    gmres_finish(run);
}


// H[k+1][k] = |w| from the stage-1 norm partials; inv = 1/|w| (0 on breakdown).
__global__ void k_arnoldi_norm(const double *__restrict__ npart, int nsplit, double *__restrict__ H,
                               int m, int k, double *__restrict__ inv) {
    if (threadIdx.x != 0) return;
    double n2 = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) n2 += npart[2 * sp];
    const double hn = sqrt(n2);
    H[((int64_t)(k + 1) * m + k) * 2] = hn;
    H[((int64_t)(k + 1) * m + k) * 2 + 1] = 0.0;
    inv[0] = hn > 1e-300 ? 1.0 / hn : 0.0;
}

// x[row] = 1 (real start vector)
__global__ void k_fill_re(int64_t M, double v, double *__restrict__ x) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= M) return;
    x[2 * r] = v;
    x[2 * r + 1] = 0.0;
}

// m Arnoldi steps of K(E) = O P0 V~ G1(E) for one energy below the pair
// threshold (everything real), start vector of ones; the Hessenberg matrix
// (m+1) x m (complex layout, imaginary parts zero) is returned in H; the
// number of steps taken (fewer on breakdown) in *steps.
void arnoldi_kernel(wpcd_ctx *c, double E, int m, std::vector<double> &H, int &steps) {
    const bool fp64 = c->p_fp64;
    Batch b{};
    b.c = c;
    b.nE = 1;
    b.nEp = 1;
    b.W = 2;
    b.Wp = 2;
    b.m = m;
    set_layout(b);
    b.fp64 = fp64;
    b.lowp = false;
    b.bf16 = false;
    const int64_t vec = b.M * 2;
    b.vstride = vec;
    const int max_chunks = cdiv(b.M, chunk_rows_of(1, 1));
    c->d_G.reserve(vec);
    c->d_T1.reserve(2 * vec);
    c->d_V.reserve((size_t)(m + 1) * vec);
    c->d_Hess.reserve((size_t)(m + 1) * m * 2);
    c->d_partial.reserve((size_t)(max_chunks + kMaxSplit) * (m + 1) * 2);
    c->d_misc.reserve(2 * (size_t)(m + 1) + 8);
    c->d_flag.reserve(4);
    b.G = c->d_G.ptr;
    b.T1 = c->d_T1.ptr;
    b.T2 = c->d_T1.ptr + vec;
    b.Vb = c->d_V.ptr;
    b.H = c->d_Hess.ptr;
    b.partial = c->d_partial.ptr;
    b.out2 = c->d_partial.ptr + (size_t)max_chunks * (m + 1) * 2;
    b.h = c->d_misc.ptr;
    b.inv = c->d_misc.ptr + 2 * (m + 1);
    hipStream_t s = c->stream;
    choose_shapes(b, m);
    ChPtrs eps{};
    for (int a = 0; a < c->nch; ++a) eps.p[a] = c->waves[c->ch_wave[a]].eps.ptr;
    double *dE = c->d_misc.ptr + 2 * (m + 1) + 2;
    WPCD_HIP(hipMemcpyAsync(dE, &E, sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_resolvent, dim3(cdiv(b.M, 256)), dim3(256), 0, s, c->d_q.ptr, c->np, c->nq,
                       c->nch, 1, dE, eps, b.G, c->d_flag.ptr);
    WPCD_HIP(hipMemsetAsync(b.H, 0, (size_t)(m + 1) * m * 2 * sizeof(double), s));
    hipLaunchKernelGGL(k_fill_re, dim3(cdiv(b.M, 256)), dim3(256), 0, s, b.M,
                       1.0 / std::sqrt((double)b.M), b.Vb);
    WPCD_HIP(hipGetLastError());
    std::vector<double> invh(1);
    steps = 0;
    for (int k = 0; k < m; ++k) {
        double *vk = b.Vb + (int64_t)k * vec;
        double *w = b.Vb + (int64_t)(k + 1) * vec;
        op_apply(b, vk, w, true, false);   // w = K v_k
        dots(b, b.Vb, k + 1, w, b.h, b.H, k, 0);
        vupdate<true, false>(b, k + 1, w);
        reduce_partials(b, k + 1, b.h, b.H, k, 1);
        vupdate<false, true>(b, k + 1, w);
        reduce_stage1(b, 1);
        hipLaunchKernelGGL(k_arnoldi_norm, dim3(1), dim3(64), 0, s, b.out2, b.nsplit, b.H, m, k, b.inv);
        hipLaunchKernelGGL(k_scale, dim3(cdiv(b.M, 256)), dim3(256), 0, s, b.inv, b.M, 1, w);
        WPCD_HIP(hipGetLastError());
        steps = k + 1;
        if ((k + 1) % 8 == 0) {
            WPCD_HIP(hipMemcpyAsync(invh.data(), b.inv, sizeof(double), hipMemcpyDeviceToHost, s));
            WPCD_HIP(hipStreamSynchronize(s));
            if (invh[0] == 0.0) break;   // invariant subspace found
        }
    }
    H.resize((size_t)(m + 1) * m * 2);
    WPCD_HIP(hipMemcpyAsync(H.data(), b.H, H.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    WPCD_HIP(hipStreamSynchronize(s));
}

void amplitudes_batch(wpcd_ctx *c, int nE, const std::vector<int64_t> &rows,
                      const std::vector<int32_t> &ens, const std::vector<double> &rho,
                      const std::vector<double> &rho0, std::vector<double> &out) {
    const int n = (int)rows.size();
    hipStream_t s = c->stream;
    // device layout in one scratch block: rows | ens | rho | rho0 | out
    const size_t bytes = n * (sizeof(int64_t) + sizeof(int32_t) + sizeof(double) + 4 * sizeof(double)) +
                         nE * sizeof(double) + 64;
    c->d_T2.reserve(bytes / sizeof(double) + 1);
    char *base = (char *)c->d_T2.ptr;
    int64_t *d_rows = (int64_t *)base;
    double *d_rho = (double *)(base + n * sizeof(int64_t));
    double *d_out = d_rho + n;
    double *d_rho0 = d_out + 4 * n;
    int32_t *d_ens = (int32_t *)(d_rho0 + nE);
    WPCD_HIP(hipMemcpyAsync(d_rows, rows.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    WPCD_HIP(hipMemcpyAsync(d_ens, ens.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    WPCD_HIP(hipMemcpyAsync(d_rho, rho.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
    WPCD_HIP(hipMemcpyAsync(d_rho0, rho0.data(), nE * sizeof(double), hipMemcpyHostToDevice, s));
    {
        TimedLaunch tl(c->timer, s, "amplitudes", WPCD_TIME_SOLVE);
        hipLaunchKernelGGL(k_amplitudes, dim3(cdiv(n, 256)), dim3(256), 0, s, c->d_X.ptr, nE, d_rows,
                           d_ens, d_rho, d_rho0, n, d_out);
        WPCD_HIP(hipGetLastError());
    }
    out.resize(4 * (size_t)n);
    WPCD_HIP(hipMemcpyAsync(out.data(), d_out, 4 * n * sizeof(double), hipMemcpyDeviceToHost, s));
    WPCD_HIP(hipStreamSynchronize(s));
}

}  // namespace wpcd
