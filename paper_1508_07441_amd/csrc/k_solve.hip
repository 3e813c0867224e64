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
#include <cstring>

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

// ------------------------------------------------------- block products
// out[(b, r)][c] = sum_k Mat_b[r][k] y[(b, k)][c],  b = a*nq + j, Mat_b = mats[a]
// y = G (.) in (complex product, USE_G) or in; out = that (SUB false) or
// add - that (SUB true).  Tiles of 32 rows x W columns, k in steps of 32.
constexpr int kTR = 32, kTK = 32;

template <bool USE_G, bool SUB>
__global__ __launch_bounds__(256) void k_block_apply(ChPtrs mats, int n, int nq, int W,
                                                     const double *__restrict__ in,
                                                     const double *__restrict__ G,
                                                     const double *__restrict__ add,
                                                     double *__restrict__ out) {
    __shared__ double sM[kTR][kTK + 1];
    __shared__ double sX[kTK][64 + 1];
    const int t = threadIdx.x;
    const int blk = blockIdx.y;
    const int row0 = blockIdx.x * kTR;
    const double *Mt = mats.p[blk / nq];
    const int64_t base = (int64_t)blk * n;   // first channel-basis row of this block
    const int nout = kTR * W;
    double acc[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[s] = 0.0;
    for (int k0 = 0; k0 < n; k0 += kTK) {
        for (int idx = t; idx < kTR * kTK; idx += 256) {
            int rr = idx / kTK, kk = idx % kTK;
            int r = row0 + rr, k = k0 + kk;
            sM[rr][kk] = (r < n && k < n) ? Mt[(int64_t)r * n + k] : 0.0;
        }
        for (int idx = t; idx < kTK * W; idx += 256) {
            int kk = idx / W, cc = idx % W;
            int k = k0 + kk;
            double v = 0.0;
            if (k < n) {
                const int64_t o = (base + k) * W;
                if (USE_G) {
                    const int c0 = cc & ~1;
                    const double gr = G[o + c0], gi = G[o + c0 + 1];
                    const double xr = in[o + c0], xi = in[o + c0 + 1];
                    v = (cc & 1) ? (gr * xi + gi * xr) : (gr * xr - gi * xi);
                } else {
                    v = in[o + cc];
                }
            }
            sX[kk][cc] = v;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int o = t + 256 * s;
            if (o < nout) {
                const int rr = o / W, cc = o % W;
                double a = acc[s];
#pragma unroll 8
                for (int kk = 0; kk < kTK; ++kk) a += sM[rr][kk] * sX[kk][cc];
                acc[s] = a;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int o = t + 256 * s;
        if (o < nout) {
            const int rr = o / W, cc = o % W;
            const int r = row0 + rr;
            if (r < n) {
                const int64_t gi = (base + r) * W + cc;
                out[gi] = SUB ? add[gi] - acc[s] : acc[s];
            }
        }
    }
}

// --------------------------------------------------------------- P0 SpMM
// y[r][c] = sum_t val[t] x[col[t]][c]; one wavefront per cell row, lanes =
// (nonzero slot g, column c) with Wp = pow2 >= W columns per slot.
template <class V>
__global__ __launch_bounds__(256) void k_spmm(const int64_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ col,
                                              const V *__restrict__ val, int nrow, int W, int Wp,
                                              const double *__restrict__ x,
                                              double *__restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nrow) return;
    const int G = 64 / Wp;
    const int g = lane / Wp, c = lane % Wp;
    const int64_t b = rowptr[r], e = rowptr[r + 1];
    double acc = 0.0;
    if (c < W)
        for (int64_t t = b + g; t < e; t += G) acc += (double)val[t] * x[(int64_t)col[t] * W + c];
    for (int off = Wp; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
    if (g == 0 && c < W) y[(int64_t)r * W + c] = acc;
}

// ----------------------------------------------------------- GMRES parts
// partial[chunk][i][e] = sum_{rows in chunk} conj(V_i[row][e]) w[row][e]
constexpr int kDotRows = 64;

__global__ __launch_bounds__(256) void k_dots(const double *__restrict__ Vb, int64_t vstride,
                                              int nvec, const double *__restrict__ w, int64_t M,
                                              int nE, double *__restrict__ partial) {
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kDotRows;
    const int64_t r1 = r0 + kDotRows < M ? r0 + kDotRows : M;
    const int npair = nvec * nE;
    for (int p = t; p < npair; p += 256) {
        const int i = p / nE, e = p % nE;
        const double *v = Vb + i * vstride;
        double sr = 0.0, si = 0.0;
        for (int64_t r = r0; r < r1; ++r) {
            const int64_t o = (r * nE + e) * 2;
            const double vr = v[o], vi = v[o + 1], wr = w[o], wi = w[o + 1];
            sr += vr * wr + vi * wi;
            si += vr * wi - vi * wr;
        }
        partial[((int64_t)blockIdx.x * npair + p) * 2] = sr;
        partial[((int64_t)blockIdx.x * npair + p) * 2 + 1] = si;
    }
}

// h[p] = sum_chunks partial[chunk][p] (one wavefront per pair p); also
// written/accumulated into the Hessenberg column H[e][i][k] (layout
// [nE][m+1][m] complex) when H is given.
__global__ __launch_bounds__(256) void k_dots_reduce(const double *__restrict__ partial, int nchunk,
                                                     int nvec, int nE, double *__restrict__ h,
                                                     double *__restrict__ H, int m, int kcol,
                                                     int accumulate) {
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int npair = nvec * nE;
    if (p >= npair) return;
    double sr = 0.0, si = 0.0;
    for (int c = lane; c < nchunk; c += 64) {
        sr += partial[((int64_t)c * npair + p) * 2];
        si += partial[((int64_t)c * npair + p) * 2 + 1];
    }
    for (int off = 32; off > 0; off >>= 1) {
        sr += __shfl_xor(sr, off, 64);
        si += __shfl_xor(si, off, 64);
    }
    if (lane != 0) return;
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

// w[row][e] -= sum_i h[i][e] V_i[row][e]
__global__ void k_update(const double *__restrict__ Vb, int64_t vstride, int nvec,
                         const double *__restrict__ h, int64_t M, int nE,
                         double *__restrict__ w) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * nE) return;
    const int e = (int)(idx % nE);
    double wr = w[2 * idx], wi = w[2 * idx + 1];
    for (int i = 0; i < nvec; ++i) {
        const double hr = h[2 * (i * nE + e)], hi = h[2 * (i * nE + e) + 1];
        const double vr = Vb[i * vstride + 2 * idx], vi = Vb[i * vstride + 2 * idx + 1];
        wr -= hr * vr - hi * vi;
        wi -= hr * vi + hi * vr;
    }
    w[2 * idx] = wr;
    w[2 * idx + 1] = wi;
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
    for (int i = 0; i < ku; ++i) {
        const double yr = y[2 * (e * m + i)], yi = y[2 * (e * m + i) + 1];
        const double vr = Vb[i * vstride + 2 * idx], vi = Vb[i * vstride + 2 * idx + 1];
        xr += yr * vr - yi * vi;
        xi += yr * vi + yi * vr;
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

// After orthogonalising w = K v_k: H[k+1][k] = ||w||; inv = 1/||w||; Givens.
__global__ void k_givens(const double *__restrict__ nrm2, double *__restrict__ H, int nE, int m,
                         int k, double tol, GState S, double *__restrict__ inv) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nE) return;
    double *st = S.st + e * kSt;
    double *He = H + (int64_t)e * (m + 1) * m * 2;
    auto Hr = [&](int i) -> double & { return He[(i * m + k) * 2]; };
    auto Hi = [&](int i) -> double & { return He[(i * m + k) * 2 + 1]; };
    const double hn = sqrt(nrm2[2 * e]);
    Hr(k + 1) = hn;
    Hi(k + 1) = 0.0;
    const double beta = st[0];
    inv[e] = (hn > 1e-14 * beta && hn > 1e-300) ? 1.0 / hn : 0.0;
    if (st[3] != 0.0) return;   // already converged: leave its state alone
    // apply previous rotations to column k
    for (int i = 0; i < k; ++i) {
        const double c = S.cs[e * m + i];
        const double sr = S.sn[2 * (e * m + i)], si = S.sn[2 * (e * m + i) + 1];
        const double ar = Hr(i), ai = Hi(i), br = Hr(i + 1), bi = Hi(i + 1);
        // a' = c a + s b ;  b' = -conj(s) a + c b
        Hr(i) = c * ar + (sr * br - si * bi);
        Hi(i) = c * ai + (sr * bi + si * br);
        Hr(i + 1) = -(sr * ar + si * ai) + c * br;
        Hi(i + 1) = -(sr * ai - si * ar) + c * bi;
    }
    const double ar = Hr(k), ai = Hi(k), br = Hr(k + 1), bi = Hi(k + 1);
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
    Hr(k) = c * ar + (sr * br - si * bi);
    Hi(k) = c * ai + (sr * bi + si * br);
    Hr(k + 1) = 0.0;
    Hi(k + 1) = 0.0;
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
    if (res <= tol * st[1] || inv[e] == 0.0) st[3] = 1.0;
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

// ----------------------------------------------------------------- host
namespace {

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

struct Batch {
    wpcd_ctx *c;
    int nE, W, Wp, m;
    int64_t M;
    bool fp64;
    double *G, *X, *B, *T1, *T2, *R, *Vb, *H, *partial, *h, *inv, *y;
    int32_t *kuse;
    GState S;
    int64_t vstride;
    int nchunk;
};

void op_apply(Batch &b, const double *x, double *out, bool with_g, bool sub) {
    wpcd_ctx *c = b.c;
    ChPtrs vt{}, oo{};
    for (int a = 0; a < c->nch; ++a) {
        vt.p[a] = c->waves[c->ch_wave[a]].Vt.ptr;
        oo.p[a] = c->waves[c->ch_wave[a]].O.ptr;
    }
    const int n = c->np;
    dim3 grid(cdiv(n, kTR), c->nch * c->nq);
    {
        TimedLaunch tl(c->timer, c->stream, "apply_vt", WPCD_TIME_SOLVE);
        if (with_g)
            hipLaunchKernelGGL((k_block_apply<true, false>), grid, dim3(256), 0, c->stream, vt, n,
                               c->nq, b.W, x, b.G, nullptr, b.T1);
        else
            hipLaunchKernelGGL((k_block_apply<false, false>), grid, dim3(256), 0, c->stream, vt, n,
                               c->nq, b.W, x, nullptr, nullptr, b.T1);
        WPCD_HIP(hipGetLastError());
    }
    {
        const int nrow = c->np * c->nq;
        TimedLaunch tl(c->timer, c->stream, "spmm", WPCD_TIME_SOLVE);
        if (b.fp64)
            hipLaunchKernelGGL(k_spmm<double>, dim3(cdiv(nrow, 4)), dim3(256), 0, c->stream,
                               c->d_rowptr.ptr, c->d_col.ptr, c->d_val64.ptr, nrow, b.W, b.Wp,
                               b.T1, b.T2);
        else
            hipLaunchKernelGGL(k_spmm<float>, dim3(cdiv(nrow, 4)), dim3(256), 0, c->stream,
                               c->d_rowptr.ptr, c->d_col.ptr, c->d_val32.ptr, nrow, b.W, b.Wp,
                               b.T1, b.T2);
        WPCD_HIP(hipGetLastError());
    }
    {
        TimedLaunch tl(c->timer, c->stream, "apply_o", WPCD_TIME_SOLVE);
        if (sub)
            hipLaunchKernelGGL((k_block_apply<false, true>), grid, dim3(256), 0, c->stream, oo, n,
                               c->nq, b.W, b.T2, nullptr, x, out);
        else
            hipLaunchKernelGGL((k_block_apply<false, false>), grid, dim3(256), 0, c->stream, oo, n,
                               c->nq, b.W, b.T2, nullptr, nullptr, out);
        WPCD_HIP(hipGetLastError());
    }
}

// nrm2/dots of w against nvec vectors starting at Vb -> h (reduced), optional H column.
void dots(Batch &b, const double *Vb, int nvec, const double *w, double *h, double *H, int kcol,
          int accumulate) {
    wpcd_ctx *c = b.c;
    {
        TimedLaunch tl(c->timer, c->stream, "gmres_dots", WPCD_TIME_SOLVE);
        hipLaunchKernelGGL(k_dots, dim3(b.nchunk), dim3(256), 0, c->stream, Vb, b.vstride, nvec, w,
                           b.M, b.nE, b.partial);
        WPCD_HIP(hipGetLastError());
    }
    {
        TimedLaunch tl(c->timer, c->stream, "gmres_reduce", WPCD_TIME_SOLVE);
        hipLaunchKernelGGL(k_dots_reduce, dim3(cdiv(nvec * b.nE, 4)), dim3(256), 0, c->stream,
                           b.partial, b.nchunk, nvec, b.nE, h, H, b.m, kcol, accumulate);
        WPCD_HIP(hipGetLastError());
    }
}

}  // namespace

// Solve the batch of energies already validated by the caller.
// idx0/rho0: entrance row and flux factor per energy.  Returns iterations
// and relative residual per energy in iters/resid.
void gmres_batch(wpcd_ctx *c, const std::vector<double> &E, const std::vector<int64_t> &idx0,
                 bool fp64, int m, int max_iter, double tol, std::vector<int> &iters,
                 std::vector<double> &resid, std::vector<int> &edge_flag) {
    const int nE = (int)E.size();
    Batch b{};
    b.c = c;
    b.nE = nE;
    b.W = 2 * nE;
    b.Wp = 1;
    while (b.Wp < b.W) b.Wp <<= 1;
    b.m = m;
    b.M = (int64_t)c->nch * c->nq * c->np;
    b.fp64 = fp64;
    const int64_t vec = b.M * b.W;   // doubles per batched vector
    b.vstride = vec;
    b.nchunk = cdiv(b.M, kDotRows);
    c->d_G.reserve(vec);
    c->d_X.reserve(vec);
    c->d_B.reserve(vec);
    c->d_T1.reserve(2 * vec);
    c->d_V.reserve((size_t)(m + 1) * vec);
    c->d_Hess.reserve((size_t)nE * (m + 1) * m * 2);
    c->d_partial.reserve((size_t)b.nchunk * (m + 1) * nE * 2);
    c->d_W.reserve(vec);
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
    // energies
    double *dE = c->d_T1.ptr;   // scratch: T1 not yet in use
    WPCD_HIP(hipMemcpyAsync(dE, E.data(), nE * sizeof(double), hipMemcpyHostToDevice, s));
    WPCD_HIP(hipMemsetAsync(flag, 0, nE * sizeof(int32_t), s));
    ChPtrs eps{};
    for (int a = 0; a < c->nch; ++a) eps.p[a] = c->waves[c->ch_wave[a]].eps.ptr;
    {
        TimedLaunch tl(c->timer, s, "resolvent", WPCD_TIME_SOLVE);
        hipLaunchKernelGGL(k_resolvent, dim3(cdiv(b.M * nE, 256)), dim3(256), 0, s, c->d_q.ptr,
                           c->np, c->nq, c->nch, nE, dE, eps, b.G, flag);
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
    // ||b||
    dots(b, b.B, 1, b.B, b.h, nullptr, 0, 0);
    // st[1] = ||b||: copy via host (small)
    std::vector<double> h0(2 * nE);
    WPCD_HIP(hipMemcpyAsync(h0.data(), b.h, 2 * nE * sizeof(double), hipMemcpyDeviceToHost, s));
    WPCD_HIP(hipStreamSynchronize(s));
    std::vector<double> st(nE * kSt, 0.0);
    for (int e = 0; e < nE; ++e) st[e * kSt + 1] = std::sqrt(h0[2 * e]);
    WPCD_HIP(hipMemcpyAsync(b.S.st, st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice, s));
    // x = 0, r = b
    WPCD_HIP(hipMemsetAsync(b.X, 0, vec * sizeof(double), s));
    WPCD_HIP(hipMemcpyAsync(b.R, b.B, vec * sizeof(double), hipMemcpyDeviceToDevice, s));

    iters.assign(nE, 0);
    resid.assign(nE, 1.0);
    int total = 0;
    std::vector<double> sth(nE * kSt);
    const int check_every = 4;
    bool all_done = false;
    while (total < max_iter && !all_done) {
        // cycle start from r
        dots(b, b.R, 1, b.R, b.h, nullptr, 0, 0);
        hipLaunchKernelGGL(k_cycle_start, dim3(cdiv(nE, 64)), dim3(64), 0, s, b.h, nE, m, tol, b.S,
                           b.inv);
        hipLaunchKernelGGL(k_scale, dim3(cdiv(b.M * nE, 256)), dim3(256), 0, s, b.inv, b.M, nE, b.R);
        WPCD_HIP(hipMemcpyAsync(b.Vb, b.R, vec * sizeof(double), hipMemcpyDeviceToDevice, s));
        WPCD_HIP(hipMemsetAsync(b.H, 0, (size_t)nE * (m + 1) * m * 2 * sizeof(double), s));
        int k = 0;
        for (; k < m && total < max_iter; ++k) {
            double *vk = b.Vb + (int64_t)k * vec;
            double *w = b.Vb + (int64_t)(k + 1) * vec;
            op_apply(b, vk, w, true, true);
            for (int pass = 0; pass < 2; ++pass) {
                dots(b, b.Vb, k + 1, w, b.h, b.H, k, pass);
                TimedLaunch tl(c->timer, s, "gmres_update", WPCD_TIME_SOLVE);
                hipLaunchKernelGGL(k_update, dim3(cdiv(b.M * nE, 256)), dim3(256), 0, s, b.Vb,
                                   b.vstride, k + 1, b.h, b.M, nE, w);
                WPCD_HIP(hipGetLastError());
            }
            dots(b, w, 1, w, b.h, nullptr, 0, 0);
            hipLaunchKernelGGL(k_givens, dim3(cdiv(nE, 64)), dim3(64), 0, s, b.h, b.H, nE, m, k, tol,
                               b.S, b.inv);
            hipLaunchKernelGGL(k_scale, dim3(cdiv(b.M * nE, 256)), dim3(256), 0, s, b.inv, b.M, nE, w);
            WPCD_HIP(hipGetLastError());
            ++total;
            if ((k + 1) % check_every == 0 || k + 1 == m) {
                WPCD_HIP(hipMemcpyAsync(sth.data(), b.S.st, sth.size() * sizeof(double),
                                        hipMemcpyDeviceToHost, s));
                WPCD_HIP(hipStreamSynchronize(s));
                bool done = true;
                for (int e = 0; e < nE; ++e) done &= sth[e * kSt + 3] != 0.0;
                if (done) {
                    ++k;
                    break;
                }
            }
        }
        hipLaunchKernelGGL(k_trisolve, dim3(cdiv(nE, 64)), dim3(64), 0, s, b.H, nE, m, b.S, b.y,
                           b.kuse);
        hipLaunchKernelGGL(k_xupdate, dim3(cdiv(b.M * nE, 256)), dim3(256), 0, s, b.Vb, b.vstride,
                           b.y, b.kuse, m, b.M, nE, b.X);
        WPCD_HIP(hipGetLastError());
        // per-energy iteration count: columns used in this cycle
        WPCD_HIP(hipMemcpyAsync(sth.data(), b.S.st, sth.size() * sizeof(double),
                                hipMemcpyDeviceToHost, s));
        // true residual r = b - (1 - K) x
        op_apply(b, b.X, b.R, true, true);
        hipLaunchKernelGGL(k_sub_from, dim3(cdiv(vec, 256)), dim3(256), 0, s, b.B, vec, b.R);
        dots(b, b.R, 1, b.R, b.h, nullptr, 0, 0);
        std::vector<double> rn(2 * nE);
        WPCD_HIP(hipMemcpyAsync(rn.data(), b.h, 2 * nE * sizeof(double), hipMemcpyDeviceToHost, s));
        WPCD_HIP(hipStreamSynchronize(s));
        all_done = true;
        for (int e = 0; e < nE; ++e) {
            if (resid[e] > tol) iters[e] += (int)sth[e * kSt + 4];
            const double bn = st[e * kSt + 1];
            resid[e] = bn > 0 ? std::sqrt(rn[2 * e]) / bn : 0.0;
            if (resid[e] > tol) all_done = false;
        }
        (void)k;
    }
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
