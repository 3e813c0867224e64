// Pair-wave setup on the GPU (paper Sec. II.B-C): potential matrix in the
// free wave-packet basis (eq.(vpot)) and the FP64 diagonalisation of the pair
// Hamiltonian h1 = h0 + v that gives the rotation O (eq.(exp_z)).
#include <hip/hip_runtime.h>

#include <cmath>

#include "wpcd_internal.h"

namespace wpcd {

// Gauss points for the potential quadrature (set by the API from the host
// Golub-Welsch table); npot <= 32.
struct PotQuad {
    double x[32], w[32];
    int n;
};

// Legendre function of the second kind Q_l(z), z > 1, given z - 1 and z + 1
// in factored form so that neither is formed by cancellation:
//   zp1 = ((a+b)^2 + mu^2) / (2ab),  zm1 = ((a-b)^2 + mu^2) / (2ab).
__device__ double legendre_q_dev(int l, double z, double zp1, double zm1) {
    double q0 = 0.5 * log(zp1 / zm1);
    if (l == 0) return q0;
    if (z < 1.5) {
        double qm = q0, qc = z * q0 - 1.0;
        for (int k = 1; k < l; ++k) {
            double qn = ((2 * k + 1) * z * qc - k * qm) / (k + 1);
            qm = qc;
            qc = qn;
        }
        return qc;
    }
    // Q_l(z) = l!/(2l+1)!! z^-(l+1) sum_n ((l+1)/2)_n ((l+2)/2)_n / ((l+3/2)_n n!) z^-2n
    double c = 1.0;
    for (int k = 1; k <= l; ++k) c *= (double)k / (double)(2 * k + 1);
    double w = 1.0 / (z * z), term = 1.0, sum = 1.0;
    double a1 = 0.5 * (l + 1), a2 = 0.5 * (l + 2), cc = l + 1.5;
    for (int n = 0; n < 400; ++n) {
        term *= (a1 + n) * (a2 + n) / ((cc + n) * (n + 1)) * w;
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    double zl = z;
    for (int k = 0; k < l; ++k) zl *= z;
    return c * sum / zl;
}

// v[i][k] = (d_i d_k)^(-1/2) int_{D_i} int_{D_k} dp dp' p p' v_l(p, p').
// kind 0: Yamaguchi lam g(p) g(p'), g = 1/(p^2 + beta^2) (l = 0 only).
// kind 1: sum_t s_t exp(-mu_t r)/r -> p p' v_l = (s/pi) Q_l(z).
__global__ void k_potential(const double *__restrict__ p, int n, int l, int kind, int nterms,
                            const double *__restrict__ s, const double *__restrict__ mu,
                            PotQuad qd, double scale, double *__restrict__ v) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    int i = idx / n, k = idx % n;
    double ai = p[i], bi = p[i + 1], ak = p[k], bk = p[k + 1];
    double mi = 0.5 * (ai + bi), hi = 0.5 * (bi - ai);
    double mk = 0.5 * (ak + bk), hk = 0.5 * (bk - ak);
    double acc = 0.0;
    if (kind == 0) {
        if (l == 0) {
            double beta2 = mu[0] * mu[0];
            double gi = 0.0, gk = 0.0;
            for (int a = 0; a < qd.n; ++a) {
                double x1 = mi + hi * qd.x[a];
                double x2 = mk + hk * qd.x[a];
                gi += qd.w[a] * x1 / (x1 * x1 + beta2);
                gk += qd.w[a] * x2 / (x2 * x2 + beta2);
            }
            acc = s[0] * (hi * gi) * (hk * gk);
        }
    } else {
        for (int t = 0; t < nterms; ++t) {
            double m2 = mu[t] * mu[t];
            double st = 0.0;
            for (int a = 0; a < qd.n; ++a) {
                double x1 = mi + hi * qd.x[a];
                double inner = 0.0;
                for (int b = 0; b < qd.n; ++b) {
                    double x2 = mk + hk * qd.x[b];
                    double den = 2.0 * x1 * x2;
                    double sp = (x1 + x2) * (x1 + x2) + m2;
                    double sm = (x1 - x2) * (x1 - x2) + m2;
                    double z = (x1 * x1 + x2 * x2 + m2) / den;
                    inner += qd.w[b] * legendre_q_dev(l, z, sp / den, sm / den);
                }
                st += qd.w[a] * inner;
            }
            acc += s[t] / M_PI * st * hi * hk;
        }
    }
    v[idx] = scale * acc / sqrt((bi - ai) * (bk - ak));
}

// ---------------------------------------------------------- eigensolver
// h1 is made positive definite by a shift sigma (Gershgorin), then
// diagonalised by one-sided (Hestenes) Jacobi: the columns of W = h1 + sigma
// are rotated pairwise until mutually orthogonal.  Since W = Q Lambda' Q^T,
// the final columns are Q Lambda': eigenvalue = column norm - sigma,
// eigenvector = normalised column.  Column pairs are visited block-cyclically:
// each workgroup holds two blocks of b columns in LDS and sweeps every pair
// among them; one launch per round of a round-robin tournament over blocks.

// Tournament pairing of P players (P even) in round r: pair k.
__device__ __forceinline__ void tourney(int P, int r, int k, int &a, int &b) {
    if (k == 0) {
        a = r;
        b = P - 1;
    } else {
        a = (r + k) % (P - 1);
        b = (r - k + (P - 1)) % (P - 1);
    }
}

// W = h1 (symmetric, so row- and column-major coincide); rowlo[i] =
// Gershgorin lower bound of row i.
__global__ void k_h1_gersh(const double *__restrict__ p, const double *__restrict__ v, int n,
                           double *__restrict__ W, double *__restrict__ rowlo) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = p[i], b = p[i + 1];
    double off = 0.0, d = 0.0;
    for (int k = 0; k < n; ++k) {
        double x = v[(int64_t)i * n + k];
        if (k == i) {
            x += (a * a + a * b + b * b) / 3.0;
            d = x;
        } else {
            off += fabs(x);
        }
        W[(int64_t)i * n + k] = x;
    }
    rowlo[i] = d - off;
}

// sigma = max(0, 1 - min_i rowlo[i]); W += sigma I.  One workgroup.
__global__ __launch_bounds__(256) void k_shift(double *__restrict__ W, int n,
                                               const double *__restrict__ rowlo,
                                               double *__restrict__ sigma_out) {
    __shared__ double red[256];
    double m = 1e300;
    for (int i = threadIdx.x; i < n; i += 256) m = fmin(m, rowlo[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    const double sigma = red[0] < 1.0 ? 1.0 - red[0] : 0.0;
    for (int i = threadIdx.x; i < n; i += 256) W[(int64_t)i * n + i] += sigma;
    if (threadIdx.x == 0) *sigma_out = sigma;
}

// Wavefront sum broadcast to all lanes, by DPP: row_shr 1, 2, 4, 8 leave each
// 16-lane row's sum in its lane 15; row_bcast 15 and 31 carry the row sums up
// to lane 63, which is then read as a scalar.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wsum(double v) {
    v += dpp_move<0x111, 0xf>(v);   // row_shr:1
    v += dpp_move<0x112, 0xf>(v);   // row_shr:2
    v += dpp_move<0x114, 0xf>(v);   // row_shr:4
    v += dpp_move<0x118, 0xf>(v);   // row_shr:8
    v += dpp_move<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Yukawa-sum potential matrix, one wavefront per element of the upper
// triangle (i <= k; the lower triangle is its mirror): the lanes split the
// n_gauss^2 quadrature points of the cell pair (8 x 8 lane grid, strided),
// then a wavefront sum.  Same integrand as k_potential.
__global__ __launch_bounds__(256) void k_potential_yukawa(const double *__restrict__ p, int n,
                                                          int l, int nterms,
                                                          const double *__restrict__ s,
                                                          const double *__restrict__ mu,
                                                          PotQuad qd, double scale,
                                                          double *__restrict__ v) {
    const int lane = threadIdx.x & 63;
    const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= (int64_t)n * n) return;   // uniform per wavefront
    const int i = (int)(e / n), k = (int)(e - (int64_t)i * n);
    if (k < i) return;
    const double ai = p[i], bi = p[i + 1], ak = p[k], bk = p[k + 1];
    const double mi = 0.5 * (ai + bi), hi = 0.5 * (bi - ai);
    const double mk = 0.5 * (ak + bk), hk = 0.5 * (bk - ak);
    const int a0 = lane >> 3, b0 = lane & 7;
    double acc = 0.0;
    for (int t = 0; t < nterms; ++t) {
        const double m2 = mu[t] * mu[t];
        double st = 0.0;
        for (int a = a0; a < qd.n; a += 8) {
            const double x1 = mi + hi * qd.x[a];
            for (int b = b0; b < qd.n; b += 8) {
                const double x2 = mk + hk * qd.x[b];
                const double den = 2.0 * x1 * x2;
                const double sp = (x1 + x2) * (x1 + x2) + m2;
                const double sm = (x1 - x2) * (x1 - x2) + m2;
                const double z = (x1 * x1 + x2 * x2 + m2) / den;
                st += (qd.w[a] * qd.w[b]) * legendre_q_dev(l, z, sp / den, sm / den);
            }
        }
        acc += s[t] / M_PI * wsum(st) * hi * hk;
    }
    if (lane == 0) {
        const double val = scale * acc / sqrt((bi - ai) * (bk - ak));
        v[(int64_t)i * n + k] = val;
        v[(int64_t)k * n + i] = val;
    }
}

// One tournament round over blocks: workgroup s takes block pair (I, J),
// loads the 2b columns into LDS, rotates every pair among them once (2b - 1
// inner rounds of b disjoint pairs, one wavefront per pair, the pair's
// columns held in registers: NPL elements per lane), writes them back.
// rotated[sweep] is set if any pair was rotated (|w_x.w_y| > tol |w_x||w_y|).
template <int NPL>
__global__ __launch_bounds__(1024) void k_jacobi_blocks(double *__restrict__ W, int n, int b,
                                                        int NB, int r, double tol,
                                                        int *__restrict__ rotated, int sweep) {
    extern __shared__ double sW[];   // [2b][n]
    int I, J;
    tourney(NB, r, blockIdx.x, I, J);
    const int P = 2 * b;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int idx = tid; idx < P * n; idx += blockDim.x) {
        const int lc = idx / n, e = idx % n;
        const int gc = lc < b ? I * b + lc : J * b + (lc - b);
        sW[idx] = gc < n ? W[(int64_t)gc * n + e] : 0.0;
    }
    __syncthreads();
    int any = 0;
    for (int rr = 0; rr < P - 1; ++rr) {
        if (wave < b) {
            int x, y;
            tourney(P, rr, wave, x, y);
            const int gx = x < b ? I * b + x : J * b + (x - b);
            const int gy = y < b ? I * b + y : J * b + (y - b);
            if (gx < n && gy < n) {
                double wx[NPL], wy[NPL];
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int u = 0; u < NPL; ++u) {
                    const int e = lane + 64 * u;
                    wx[u] = e < n ? sW[x * n + e] : 0.0;
                    wy[u] = e < n ? sW[y * n + e] : 0.0;
                    al += wx[u] * wx[u];
                    be += wy[u] * wy[u];
                    ga += wx[u] * wy[u];
                }
                al = wsum(al);
                be = wsum(be);
                ga = wsum(ga);
                if (fabs(ga) > tol * sqrt(al * be)) {
                    const double ze = (be - al) / (2.0 * ga);
                    const double t = (ze >= 0 ? 1.0 : -1.0) / (fabs(ze) + sqrt(1.0 + ze * ze));
                    const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
#pragma unroll
                    for (int u = 0; u < NPL; ++u) {
                        const int e = lane + 64 * u;
                        if (e < n) {
                            sW[x * n + e] = c * wx[u] - sn * wy[u];
                            sW[y * n + e] = sn * wx[u] + c * wy[u];
                        }
                    }
                    any = 1;
                }
            }
        }
        __syncthreads();
    }
    for (int idx = tid; idx < P * n; idx += blockDim.x) {
        const int lc = idx / n, e = idx % n;
        const int gc = lc < b ? I * b + lc : J * b + (lc - b);
        if (gc < n) W[(int64_t)gc * n + e] = sW[idx];
    }
    if (any) rotated[sweep] = 1;
}

// Sum over the 8 lanes of an aligned group (half-row mirror, quad reverse,
// quad swap); the result in every lane of the group.
__device__ __forceinline__ double gsum8(double v) {
    v += dpp_move<0x141, 0xf>(v);   // row_half_mirror
    v += dpp_move<0x1B, 0xf>(v);    // quad_perm [3, 2, 1, 0]
    v += dpp_move<0xB1, 0xf>(v);    // quad_perm [1, 0, 3, 2]
    return v;
}

// Whole one-sided Jacobi in one workgroup, for n <= 8 EPL (EPL <= 20): group g of 8
// lanes holds two columns (A, B) in registers, element u + 8 r in lane u,
// slot r.  Column pairs follow the odd-even transposition ordering over
// positions 0 .. 2P - 1 (P = ceil(n / 2) groups): in even rounds group g
// rotates the columns at positions (2g, 2g + 1), in odd rounds those at
// (2g + 1, 2g + 2) (group P - 1 idle), and each rotated pair trades places,
// so every pair meets once in 2P rounds.  In registers this means one column
// per group moves per round, through an LDS mailbox: after an even round B
// comes from group g + 1 (group P - 1 then swaps A and B), after an odd round
// A comes from group g - 1 (indices mod P).  Sweeps repeat until a sweep
// rotates nothing (workgroup vote) or max_sweeps; status[0] = sweeps done,
// status[1] = 1 if converged.
// One round of k_jacobi_wg for group g (ODD: the odd positions' pairing):
// rotate the held pair if it is active and not yet orthogonal, then pass
// the moving column (with its squared norm) on through the mailbox.  The
// squared norms nA, nB are carried through the rotations and recomputed at
// the start of every sweep; only the overlap is a fresh dot product.
template <int EPL, bool ODD>
__device__ __forceinline__ void jacobi_round(double (&A)[EPL], double (&B)[EPL], double &nA,
                                             double &nB, int &idA, int &idB, double *mail,
                                             double *mail_n, int *mail_id, int g, int u, int P,
                                             double tol2, int &any, int &big) {
    double ga = 0.0;
#pragma unroll
    for (int r = 0; r < EPL; ++r) ga += A[r] * B[r];
    ga = gsum8(ga);
    const bool active = ODD ? g < P - 1 : g < P;
    if (active && ga * ga > tol2 * (nA * nB)) {
        // an overlap above 1e-8 (relative) may leave more than rounding after
        // its rotation and the rest of the sweep
        if (ga * ga > 1e-16 * (nA * nB)) big = 1;
        // The angle only sets how much of the pair's overlap this rotation
        // removes, so it is formed in FP32 (|ze| < 1e17 here: the norms
        // differ by < 1e3 and |ga| > tol |A||B|) with hardware reciprocal
        // and square root; the rotation built from it, c = (1 + t^2)^(-1/2)
        // and s = t c, is orthogonal to FP64 rounding, and convergence is
        // judged on FP64 overlaps.
        const float ze = (float)(nB - nA) * __builtin_amdgcn_rcpf((float)(2.0 * ga));
        const float rt = __builtin_amdgcn_rcpf(fabsf(ze) + __builtin_amdgcn_sqrtf(fmaf(ze, ze, 1.f)));
        const double t = (double)(ze >= 0.f ? rt : -rt);
        const double x = 1.0 + t * t;
        double c = rsqrt(x);
        c = c * (1.5 - 0.5 * x * c * c);   // one Newton step: c to FP64 rounding
        const double sn = t * c;
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
            const double xa = A[r], yb = B[r];
            A[r] = c * xa - sn * yb;
            B[r] = sn * xa + c * yb;
        }
        const double cc = c * c, ss = sn * sn, cs2 = 2.0 * c * sn * ga;
        const double a2 = cc * nA + ss * nB - cs2, b2 = ss * nA + cc * nB + cs2;
        nA = a2;
        nB = b2;
        any = 1;
    }
    // mailbox slot r of group g at mail[r][g][u]; at most 4 EPL groups
    constexpr int stride = 32 * EPL;
    double *mine = mail + g * 8 + u;
#pragma unroll
    for (int r = 0; r < EPL; ++r) mine[r * stride] = ODD ? A[r] : B[r];
    if (u == 0) {
        mail_id[g] = ODD ? idA : idB;
        mail_n[g] = ODD ? nA : nB;
    }
    __syncthreads();
    if (g < P) {
        const int src = ODD ? (g == 0 ? P - 1 : g - 1) : (g + 1 == P ? 0 : g + 1);
        const double *from = mail + src * 8 + u;
        if (ODD) {
#pragma unroll
            for (int r = 0; r < EPL; ++r) A[r] = from[r * stride];
            idA = mail_id[src];
            nA = mail_n[src];
        } else {
#pragma unroll
            for (int r = 0; r < EPL; ++r) B[r] = from[r * stride];
            idB = mail_id[src];
            nB = mail_n[src];
            if (g == P - 1) {
#pragma unroll
                for (int r = 0; r < EPL; ++r) {
                    const double xa = A[r];
                    A[r] = B[r];
                    B[r] = xa;
                }
                const int xi = idA;
                idA = idB;
                idB = xi;
                const double xn = nA;
                nA = nB;
                nB = xn;
            }
        }
    }
    __syncthreads();
}

template <int EPL>
__global__ __launch_bounds__(768) void k_jacobi_wg(double *__restrict__ W, int n, double tol,
                                                    int max_sweeps, int *__restrict__ status) {
    // [EPL][4 EPL][8] column doubles, then norms [4 EPL], then ids [4 EPL]
    // (P = ceil(n / 2) <= 4 EPL groups; blockDim = 8 ceil(P / 8) * 8)
    extern __shared__ double mail[];
    const int tid = threadIdx.x, u = tid & 7, g = tid >> 3;
    const int P = (n + 1) >> 1;
    double *mail_n = mail + EPL * 32 * EPL;
    int *mail_id = (int *)(mail_n + 4 * EPL);
    double A[EPL], B[EPL];
    int idA = 2 * g, idB = 2 * g + 1;
#pragma unroll
    for (int r = 0; r < EPL; ++r) {
        const int e = u + 8 * r;
        A[r] = (idA < n && e < n) ? W[(int64_t)idA * n + e] : 0.0;
        B[r] = (idB < n && e < n) ? W[(int64_t)idB * n + e] : 0.0;
    }
    const double tol2 = tol * tol;
    int sweep = 0, converged = 0;
    while (sweep < max_sweeps) {
        double nA = 0.0, nB = 0.0;
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
            nA += A[r] * A[r];
            nB += B[r] * B[r];
        }
        nA = gsum8(nA);
        nB = gsum8(nB);
        int any = 0, big = 0;
        // 2P rounds: even and odd alternate
        for (int rd = 0; rd < P; ++rd) {
            jacobi_round<EPL, false>(A, B, nA, nB, idA, idB, mail, mail_n, mail_id, g, u, P, tol2,
                                     any, big);
            jacobi_round<EPL, true>(A, B, nA, nB, idA, idB, mail, mail_n, mail_id, g, u, P, tol2,
                                    any, big);
        }
        ++sweep;
        // Done when the sweep rotated nothing, or when every overlap it met
        // was below 1e-8 of the column norms: the one-sided Jacobi then
        // converges quadratically, so what its rotations leave (and what
        // they induce in other pairs) is of the order of the squares, below
        // 1e-16 < tol, and a further sweep would only confirm it.
        if (!__syncthreads_or(any) || !__syncthreads_or(big)) {
            converged = 1;
            break;
        }
    }
    if (g < P) {
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
            const int e = u + 8 * r;
            if (e < n) {
                if (idA < n) W[(int64_t)idA * n + e] = A[r];
                if (idB < n) W[(int64_t)idB * n + e] = B[r];
            }
        }
    }
    if (tid == 0) {
        status[0] = sweep;
        status[1] = converged;
    }
}

// Column norms: lam'[k] = |w_k|, eps[k] = lam'[k] - sigma.
__global__ void k_colnorm(const double *__restrict__ W, int n, const double *__restrict__ sigma,
                          double *__restrict__ nrm, double *__restrict__ ev) {
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (k >= n) return;
    double s = 0.0;
    for (int e = lane; e < n; e += 64) {
        const double x = W[(int64_t)k * n + e];
        s += x * x;
    }
    s = wsum(s);
    if (lane == 0) {
        nrm[k] = sqrt(s);
        ev[k] = sqrt(s) - sigma[0];
    }
}

// Ascending order + sign rule: eps[rank] = ev[k]; O[rank][:] = w_k / |w_k|
// with the largest-magnitude component made positive (lowest index on ties).
__global__ void k_eig_sort(const double *__restrict__ W, const double *__restrict__ nrm,
                           const double *__restrict__ ev, int n, int want_vectors,
                           double *__restrict__ eps, double *__restrict__ O) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double ek = ev[k];
    int rank = 0;
    for (int m = 0; m < n; ++m) {
        const double em = ev[m];
        rank += (em < ek) || (em == ek && m < k);
    }
    eps[rank] = ek;
    if (!want_vectors) return;
    double big = -1.0, sgn = 1.0;
    const double *w = W + (int64_t)k * n;
    for (int r = 0; r < n; ++r) {
        const double x = w[r];
        if (fabs(x) > big) {
            big = fabs(x);
            sgn = x < 0 ? -1.0 : 1.0;
        }
    }
    const double f = sgn / nrm[k];
    for (int r = 0; r < n; ++r) O[(int64_t)rank * n + r] = f * w[r];
}

// Vt = v O^T  (Vt[i][k] = sum_m v[i][m] O[k][m])
__global__ void k_vt(const double *__restrict__ v, const double *__restrict__ O, int n,
                     double *__restrict__ Vt) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    int i = idx / n, k = idx % n;
    double acc = 0.0;
    for (int m = 0; m < n; ++m) acc += v[i * n + m] * O[k * n + m];
    Vt[idx] = acc;
}

// ------------------------------------------------------------------ host
static PotQuad pot_quad(wpcd_ctx *c) {
    PotQuad q{};
    std::vector<double> x, w;
    gauss_legendre_gw(24, x, w);
    q.n = 24;
    for (int a = 0; a < 24; ++a) {
        q.x[a] = x[a];
        q.w[a] = w[a];
    }
    (void)c;
    return q;
}

void launch_potential(wpcd_ctx *c, int wave, double *v_out) {
    int n = c->np;
    int l = c->waves[wave].l;
    int nt = (int)c->pot_s.size();
    DBuf<double> &ms = c->d_pot;
    ms.reserve(2 * 16);
    std::vector<double> host(32, 0.0);
    const std::vector<double> &wm = c->waves[wave].mult;   // per-wave multipliers (nucleons)
    for (int t = 0; t < nt; ++t) {
        host[t] = c->pot_s[t] * (t < (int)wm.size() ? wm[t] : 1.0);
        host[16 + t] = c->pot_mu[t];
    }
    WPCD_HIP(hipMemcpyAsync(ms.ptr, host.data(), 32 * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
    PotQuad qd = pot_quad(c);
    TimedLaunch tl(c->timer, c->stream, "potential", WPCD_TIME_PAIR);
    if (c->pot_kind == 0) {
        // separable: one thread per element
        int threads = 256, blocks = (n * n + threads - 1) / threads;
        hipLaunchKernelGGL(k_potential, dim3(blocks), dim3(threads), 0, c->stream, c->d_p.ptr, n,
                           l, c->pot_kind, nt, ms.ptr, ms.ptr + 16, qd, c->pot_scale, v_out);
    } else {
        const int64_t waves = (int64_t)n * n;
        hipLaunchKernelGGL(k_potential_yukawa, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0,
                           c->stream, c->d_p.ptr, n, l, nt, ms.ptr, ms.ptr + 16, qd, c->pot_scale,
                           v_out);
    }
    WPCD_HIP(hipGetLastError());
}

// Largest elements per lane of the one-workgroup Jacobi (n <= 160).
constexpr int kWgMaxEpl = 20;

void pair_diagonalise(wpcd_ctx *c, int wave, bool want_vectors) {
    const int n = c->np;
    PairWave &pw = c->waves[wave];
    constexpr int kMaxSweeps = 40;
    // workspace: W [n*n] | rowlo [n] | nrm [n] | ev [n] | sigma [1]
    c->d_jac.reserve((size_t)n * n + 3 * (size_t)n + 8);
    c->d_flag.reserve(kMaxSweeps + 4);
    double *W = c->d_jac.ptr, *rowlo = W + (size_t)n * n, *nrm = rowlo + n, *ev = nrm + n,
           *sigma = ev + n;
    int *rot = c->d_flag.ptr;
    hipStream_t s = c->stream;
    {
        TimedLaunch tl(c->timer, s, "h1", WPCD_TIME_PAIR);
        hipLaunchKernelGGL(k_h1_gersh, dim3((n + 255) / 256), dim3(256), 0, s, c->d_p.ptr, pw.v.ptr,
                           n, W, rowlo);
        hipLaunchKernelGGL(k_shift, dim3(1), dim3(256), 0, s, W, n, rowlo, sigma);
        WPCD_HIP(hipGetLastError());
    }
    const double tol = 2.2e-16 * (double)n;
    if (n <= 8 * kWgMaxEpl) {
        // whole Jacobi in one workgroup, columns in registers
        const int need = (n + 7) / 8;
        const int epl = need <= 4 ? 4 : need <= 8 ? 8 : need <= 12 ? 12 : need <= 16 ? 16 : 20;
        const int P = (n + 1) / 2, Ppad = (P + 7) / 8 * 8;
        const size_t lds = (size_t)epl * 32 * epl * sizeof(double) +
                           (size_t)4 * epl * (sizeof(double) + sizeof(int));
        auto go = [&](auto kern) {
            WPCD_HIP(hipFuncSetAttribute((const void *)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            TimedLaunch tl(c->timer, s, "jacobi_sweep", WPCD_TIME_PAIR);
            hipLaunchKernelGGL(kern, dim3(1), dim3(Ppad * 8), lds, s, W, n, tol, kMaxSweeps, rot);
            WPCD_HIP(hipGetLastError());
        };
        switch (epl) {
            case 4: go(k_jacobi_wg<4>); break;
            case 8: go(k_jacobi_wg<8>); break;
            case 12: go(k_jacobi_wg<12>); break;
            case 16: go(k_jacobi_wg<16>); break;
            default: go(k_jacobi_wg<20>); break;
        }
        int st[2] = {0, 0};
        WPCD_HIP(hipMemcpyAsync(st, rot, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
        WPCD_HIP(hipStreamSynchronize(s));
        WPCD_REQUIRE(st[1] == 1, WPCD_E_NOT_CONVERGED, "pair diagonalisation did not converge");
    } else {
        // block-cyclic Jacobi over workgroups, one launch per tournament round
        const int b = (2 * 16 * n * (int)sizeof(double) <= 150 * 1024) ? 16 : 8;
        const int nbr = (n + b - 1) / b;
        const int NB = nbr + (nbr & 1);
        const size_t lds = (size_t)2 * b * n * sizeof(double);
        WPCD_HIP(hipMemsetAsync(rot, 0, kMaxSweeps * sizeof(int), s));
        const int npl = (n + 63) / 64;
        auto kern = npl <= 2 ? k_jacobi_blocks<2>
                  : npl <= 4 ? k_jacobi_blocks<4>
                  : npl <= 8 ? k_jacobi_blocks<8>
                             : k_jacobi_blocks<16>;
        WPCD_HIP(hipFuncSetAttribute((const void *)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        int sweep = 0;
        bool converged = false;
        for (; sweep < kMaxSweeps && !converged; ++sweep) {
            {
                TimedLaunch tl(c->timer, s, "jacobi_sweep", WPCD_TIME_PAIR);
                for (int r = 0; r < NB - 1; ++r)
                    hipLaunchKernelGGL(kern, dim3(NB / 2), dim3(64 * b), lds, s, W, n, b, NB, r,
                                       tol, rot, sweep);
                WPCD_HIP(hipGetLastError());
            }
            int flag = 1;
            WPCD_HIP(hipMemcpyAsync(&flag, rot + sweep, sizeof(int), hipMemcpyDeviceToHost, s));
            WPCD_HIP(hipStreamSynchronize(s));
            converged = (flag == 0);
        }
        WPCD_REQUIRE(converged, WPCD_E_NOT_CONVERGED, "pair diagonalisation did not converge");
    }
    {
        TimedLaunch tl(c->timer, s, "eig_finish", WPCD_TIME_PAIR);
        hipLaunchKernelGGL(k_colnorm, dim3((n + 3) / 4), dim3(256), 0, s, W, n, sigma, nrm, ev);
        hipLaunchKernelGGL(k_eig_sort, dim3((n + 255) / 256), dim3(256), 0, s, W, nrm, ev, n,
                           want_vectors ? 1 : 0, pw.eps.ptr, pw.O.ptr);
        WPCD_HIP(hipGetLastError());
    }
    pw.h_eps.resize(n);
    WPCD_HIP(hipMemcpyAsync(pw.h_eps.data(), pw.eps.ptr, n * sizeof(double), hipMemcpyDeviceToHost, s));
    WPCD_HIP(hipStreamSynchronize(s));
}

void launch_vt(wpcd_ctx *c, int wave) {
    int n = c->np;
    PairWave &pw = c->waves[wave];
    int threads = 256, blocks = (n * n + threads - 1) / threads;
    TimedLaunch tl(c->timer, c->stream, "vt", WPCD_TIME_PAIR);
    hipLaunchKernelGGL(k_vt, dim3(blocks), dim3(threads), 0, c->stream, pw.v.ptr, pw.O.ptr, n,
                       pw.Vt.ptr);
    WPCD_HIP(hipGetLastError());
}

}  // namespace wpcd
