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
    for (int t = 0; t < nt; ++t) {
        host[t] = c->pot_s[t];
        host[16 + t] = c->pot_mu[t];
    }
    WPCD_HIP(hipMemcpyAsync(ms.ptr, host.data(), 32 * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
    PotQuad qd = pot_quad(c);
    int threads = 256, blocks = (n * n + threads - 1) / threads;
    TimedLaunch tl(c->timer, c->stream, "potential", WPCD_TIME_PAIR);
    hipLaunchKernelGGL(k_potential, dim3(blocks), dim3(threads), 0, c->stream, c->d_p.ptr, n, l,
                       c->pot_kind, nt, ms.ptr, ms.ptr + 16, qd, c->pot_scale, v_out);
    WPCD_HIP(hipGetLastError());
}

void pair_diagonalise(wpcd_ctx *c, int wave, bool want_vectors) {
    const int n = c->np;
    PairWave &pw = c->waves[wave];
    constexpr int kMaxSweeps = 40;
    const int b = (2 * 16 * n * (int)sizeof(double) <= 150 * 1024) ? 16 : 8;
    const int nbr = (n + b - 1) / b;
    const int NB = nbr + (nbr & 1);
    const size_t lds = (size_t)2 * b * n * sizeof(double);
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
    WPCD_HIP(hipMemsetAsync(rot, 0, kMaxSweeps * sizeof(int), s));
    const int npl = (n + 63) / 64;
    auto kern = npl <= 2 ? k_jacobi_blocks<2>
              : npl <= 4 ? k_jacobi_blocks<4>
              : npl <= 8 ? k_jacobi_blocks<8>
                         : k_jacobi_blocks<16>;
    WPCD_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 160 * 1024));
    const double tol = 2.2e-16 * (double)n;
    int sweep = 0;
    bool converged = false;
    for (; sweep < kMaxSweeps && !converged; ++sweep) {
        {
            TimedLaunch tl(c->timer, s, "jacobi_sweep", WPCD_TIME_PAIR);
            for (int r = 0; r < NB - 1; ++r)
                hipLaunchKernelGGL(kern, dim3(NB / 2), dim3(64 * b), lds, s, W, n, b, NB, r, tol,
                                   rot, sweep);
            WPCD_HIP(hipGetLastError());
        }
        int flag = 1;
        WPCD_HIP(hipMemcpyAsync(&flag, rot + sweep, sizeof(int), hipMemcpyDeviceToHost, s));
        WPCD_HIP(hipStreamSynchronize(s));
        converged = (flag == 0);
    }
    WPCD_REQUIRE(converged, WPCD_E_NOT_CONVERGED, "pair diagonalisation did not converge");
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
