// Reduced basis of the learned warm start: snapshot storage, a greedy
// orthonormal basis built from the snapshots by classical Gram-Schmidt with
// reorthogonalisation, and the lift of predicted coefficients to an initial
// vector of the solve.  Not part of the paper's method.
//
// Snapshots and basis vectors are complex FP32 ([vector][M][2]); every dot
// product accumulates in FP64.  The initial vector only has to be close to
// the solution, not exact: the solve corrects it to full precision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "wpcd_internal.h"

namespace wpcd {

// snaps[(first + t) M + row] = x[row][which[t]] (batch layout, nE energies)
__global__ void k_snap_store(const double *__restrict__ x, int nE, const int32_t *__restrict__ which,
                             int nsel, int64_t M, float *__restrict__ snaps, int64_t first) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * nsel) return;
    const int t = (int)(idx / M);
    const int64_t row = idx % M;
    const int e = which[t];
    const double *src = x + (row * nE + e) * 2;
    float *dst = snaps + ((first + t) * M + row) * 2;
    dst[0] = (float)src[0];
    dst[1] = (float)src[1];
}

// partial[split][i] = sum over the split's rows of conj(A_i[r]) x[r]
// (or |A_i[r]|^2 when NORM).  Grid (nvec, nsplit).
template <bool NORM>
__global__ __launch_bounds__(256) void k_cdots(const float *__restrict__ A, int64_t lda,
                                               const float *__restrict__ x, int64_t M,
                                               int64_t rows_per_split, double *__restrict__ partial,
                                               int nvec) {
    __shared__ double red[2][4];
    const int i = blockIdx.x, split = blockIdx.y;
    const int64_t r0 = (int64_t)split * rows_per_split;
    const int64_t r1 = (r0 + rows_per_split < M) ? r0 + rows_per_split : M;
    const float *a = A + (int64_t)i * lda * 2;
    double sr = 0.0, si = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        const double ar = a[2 * r], ai = a[2 * r + 1];
        if (NORM) {
            sr += ar * ar + ai * ai;
        } else {
            const double xr = x[2 * r], xi = x[2 * r + 1];
            sr += ar * xr + ai * xi;
            si += ar * xi - ai * xr;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        sr += __shfl_xor(sr, off, 64);
        si += __shfl_xor(si, off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = sr;
        red[1][wave] = si;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t p = (int64_t)split * nvec + i;
        partial[2 * p] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        partial[2 * p + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
}

// v[r] -= sum_k d[k] Phi_k[r]
__global__ void k_basis_sub(const float *__restrict__ phi, int nk, int64_t M,
                            const double *__restrict__ d, float *__restrict__ v) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= M) return;
    double vr = v[2 * r], vi = v[2 * r + 1];
    for (int k = 0; k < nk; ++k) {
        const double pr = phi[((int64_t)k * M + r) * 2], pi = phi[((int64_t)k * M + r) * 2 + 1];
        vr -= d[2 * k] * pr - d[2 * k + 1] * pi;
        vi -= d[2 * k] * pi + d[2 * k + 1] * pr;
    }
    v[2 * r] = (float)vr;
    v[2 * r + 1] = (float)vi;
}

__global__ void k_cscale(const float *__restrict__ v, int64_t M, double s, float *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= M) return;
    out[2 * r] = (float)(s * v[2 * r]);
    out[2 * r + 1] = (float)(s * v[2 * r + 1]);
}

// x[row][e] = scale sum_k Phi_k[row] (y[e][2k] + i y[e][2k+1]); y staged in LDS.
__global__ __launch_bounds__(256) void k_lift(const float *__restrict__ phi, int K, int64_t M,
                                              const float *__restrict__ y, int nE, double scale,
                                              double *__restrict__ x) {
    extern __shared__ float ys[];
    for (int t = threadIdx.x; t < nE * 2 * K; t += 256) ys[t] = y[t];
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= M) return;
    for (int e0 = 0; e0 < nE; e0 += 8) {
        float ar[8] = {}, ai[8] = {};
        for (int k = 0; k < K; ++k) {
            const float pr = phi[((int64_t)k * M + r) * 2], pi = phi[((int64_t)k * M + r) * 2 + 1];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (e0 + u < nE) {
                    const float yr = ys[(e0 + u) * 2 * K + 2 * k], yi = ys[(e0 + u) * 2 * K + 2 * k + 1];
                    ar[u] = fmaf(pr, yr, fmaf(-pi, yi, ar[u]));
                    ai[u] = fmaf(pr, yi, fmaf(pi, yr, ai[u]));
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (e0 + u < nE) {
                x[(r * nE + e0 + u) * 2] = scale * ar[u];
                x[(r * nE + e0 + u) * 2 + 1] = scale * ai[u];
            }
        }
    }
}

// x[row][e] = src[e][row] (complex)
__global__ void k_interleave(const double *__restrict__ src, int nE, int64_t M,
                             double *__restrict__ x) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * nE) return;
    const int64_t row = idx / nE;
    const int e = (int)(idx % nE);
    x[2 * idx] = src[((int64_t)e * M + row) * 2];
    x[2 * idx + 1] = src[((int64_t)e * M + row) * 2 + 1];
}

// ------------------------------------------------------------------ host
static inline int gdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

void learn_snap_store(wpcd_ctx *c, float *snaps, int64_t first, const double *x, int nE,
                      const std::vector<int> &which) {
    const int nsel = (int)which.size();
    if (nsel == 0) return;
    const int64_t M = (int64_t)c->nch * c->nq * c->np;
    std::vector<int32_t> w(which.begin(), which.end());
    c->learned.sel.reserve(nsel);
    int32_t *dw = c->learned.sel.ptr;
    WPCD_HIP(hipMemcpyAsync(dw, w.data(), nsel * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_snap_store, dim3(gdiv(M * nsel, 256)), dim3(256), 0, c->stream, x, nE, dw,
                       nsel, M, snaps, first);
    WPCD_HIP(hipGetLastError());
    WPCD_HIP(hipStreamSynchronize(c->stream));
}

namespace {

// out[i] = <A_i, x> (or |A_i|^2) for i < nvec, reduced on the host.
void cdots(wpcd_ctx *c, const float *A, int nvec, const float *x, int64_t M, bool norm,
           DBuf<double> &partial, std::vector<double> &out) {
    out.assign(2 * (size_t)nvec, 0.0);
    if (nvec == 0) return;
    int nsplit = std::max(1, std::min(64, 1024 / nvec));
    nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(nsplit, M / 4096));
    const int64_t rps = (M + nsplit - 1) / nsplit;
    partial.reserve(2 * (size_t)nsplit * nvec);
    dim3 grid(nvec, nsplit);
    if (norm)
        hipLaunchKernelGGL(k_cdots<true>, grid, dim3(256), 0, c->stream, A, M, x, M, rps,
                           partial.ptr, nvec);
    else
        hipLaunchKernelGGL(k_cdots<false>, grid, dim3(256), 0, c->stream, A, M, x, M, rps,
                           partial.ptr, nvec);
    WPCD_HIP(hipGetLastError());
    std::vector<double> h(2 * (size_t)nsplit * nvec);
    WPCD_HIP(hipMemcpyAsync(h.data(), partial.ptr, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
    WPCD_HIP(hipStreamSynchronize(c->stream));
    for (int s = 0; s < nsplit; ++s)
        for (int i = 0; i < nvec; ++i) {
            out[2 * i] += h[2 * ((size_t)s * nvec + i)];
            out[2 * i + 1] += h[2 * ((size_t)s * nvec + i) + 1];
        }
}

}  // namespace

// Greedy reduced basis: repeatedly take the snapshot worst represented (in
// relative norm) by the current basis, orthogonalise it (two Gram-Schmidt
// passes) and normalise it.  coef[k][i] = <Phi_k, S_i> (complex, [K][n][2]).
// Stops early when every snapshot is represented to 1e-7 (FP32 snapshots);
// the basis size then shrinks (c->learned.K).
void learn_build_basis(wpcd_ctx *c, const float *snaps, int n, int K, std::vector<double> &coef,
                       double &max_err, double &mean_err) {
    Learned &L = c->learned;
    const int64_t M = (int64_t)c->nch * c->nq * c->np;
    L.M = M;
    L.phi.reserve((size_t)K * M * 2);
    DBuf<double> partial, dd;
    DBuf<float> v;
    v.reserve(2 * (size_t)M);
    dd.reserve(2 * (size_t)K);
    std::vector<double> ns, res(n), d, cc;
    cdots(c, snaps, n, nullptr, M, true, partial, ns);
    for (int i = 0; i < n; ++i) res[i] = ns[2 * i];
    coef.assign(2 * (size_t)K * n, 0.0);
    int k = 0;
    for (; k < K; ++k) {
        int best = -1;
        double bv = 0.0;
        for (int i = 0; i < n; ++i) {
            const double rel = ns[2 * i] > 0 ? res[i] / ns[2 * i] : 0.0;
            if (rel > bv) {
                bv = rel;
                best = i;
            }
        }
        if (best < 0 || bv < 1e-14) break;
        WPCD_HIP(hipMemcpyAsync(v.ptr, snaps + (int64_t)best * M * 2, M * 2 * sizeof(float),
                                hipMemcpyDeviceToDevice, c->stream));
        for (int pass = 0; pass < 2 && k > 0; ++pass) {
            cdots(c, L.phi.ptr, k, v.ptr, M, false, partial, d);
            WPCD_HIP(hipMemcpyAsync(dd.ptr, d.data(), d.size() * sizeof(double),
                                    hipMemcpyHostToDevice, c->stream));
            hipLaunchKernelGGL(k_basis_sub, dim3(gdiv(M, 256)), dim3(256), 0, c->stream, L.phi.ptr,
                               k, M, dd.ptr, v.ptr);
            WPCD_HIP(hipGetLastError());
        }
        std::vector<double> nv;
        cdots(c, v.ptr, 1, nullptr, M, true, partial, nv);
        const double nrm = std::sqrt(nv[0]);
        if (!(nrm > 1e-7 * std::sqrt(ns[2 * best]))) {
            res[best] = 0.0;   // numerically inside the span already
            --k;
            continue;
        }
        float *phik = L.phi.ptr + (int64_t)k * M * 2;
        hipLaunchKernelGGL(k_cscale, dim3(gdiv(M, 256)), dim3(256), 0, c->stream, v.ptr, M,
                           1.0 / nrm, phik);
        WPCD_HIP(hipGetLastError());
        // <S_i, Phi_k> for all snapshots; the coefficient is its conjugate
        cdots(c, snaps, n, phik, M, false, partial, cc);
        for (int i = 0; i < n; ++i) {
            const double cr = cc[2 * i], ci = -cc[2 * i + 1];
            coef[2 * ((size_t)k * n + i)] = cr;
            coef[2 * ((size_t)k * n + i) + 1] = ci;
            res[i] -= cr * cr + ci * ci;
        }
    }
    L.K = k;
    coef.resize(2 * (size_t)k * n);
    max_err = 0.0;
    mean_err = 0.0;
    for (int i = 0; i < n; ++i) {
        const double e = ns[2 * i] > 0 ? std::sqrt(std::max(res[i], 0.0) / ns[2 * i]) : 0.0;
        max_err = std::max(max_err, e);
        mean_err += e / n;
    }
    partial.release();
    dd.release();
    v.release();
}

void learn_interleave(wpcd_ctx *c, const double *src, int nE, int64_t M, double *x) {
    hipLaunchKernelGGL(k_interleave, dim3(gdiv(M * nE, 256)), dim3(256), 0, c->stream, src, nE, M, x);
    WPCD_HIP(hipGetLastError());
}

void learn_lift(wpcd_ctx *c, const float *y, int nE, double *x) {
    Learned &L = c->learned;
    const size_t lds = (size_t)nE * 2 * L.K * sizeof(float);
    WPCD_REQUIRE(lds <= 64 * 1024, WPCD_E_INVALID, "warm-start batch too large");
    TimedLaunch tl(c->timer, c->stream, "learn_lift", WPCD_TIME_SOLVE);
    hipLaunchKernelGGL(k_lift, dim3(gdiv(L.M, 256)), dim3(256), lds, c->stream, L.phi.ptr, L.K, L.M,
                       y, nE, L.coef_scale, x);
    WPCD_HIP(hipGetLastError());
}

}  // namespace wpcd
