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

// Parallel-ordered cyclic Jacobi on one workgroup.  A (n x n, row-major,
// symmetric) is overwritten: on exit its diagonal holds the eigenvalues and
// V (n x n) the eigenvectors as columns (A0 = V diag V^T).  Each round of the
// round-robin tournament rotates n/2 disjoint index pairs at once: the
// columns of A and V are rotated first, then the rows of A.
constexpr int kJacThreads = 1024;

__global__ __launch_bounds__(kJacThreads) void k_jacobi(double *__restrict__ A,
                                                         double *__restrict__ V, int n,
                                                         int want_vectors, int max_sweeps,
                                                         int *__restrict__ sweeps_out) {
    const int nn = n + (n & 1);   // even number of tournament players
    const int npairs = nn / 2;
    __shared__ int s_p[512], s_q[512];
    __shared__ double s_c[512], s_s[512];
    __shared__ int s_rot;
    const int tid = threadIdx.x;
    if (want_vectors)
        for (int idx = tid; idx < n * n; idx += blockDim.x) V[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
    __syncthreads();
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int r = 0; r < nn - 1; ++r) {
            for (int k = tid; k < npairs; k += blockDim.x) {
                int a, b;
                if (k == 0) {
                    a = r;
                    b = nn - 1;
                } else {
                    a = (r + k) % (nn - 1);
                    b = (r - k + (nn - 1)) % (nn - 1);
                }
                int pp = a < b ? a : b, qq = a < b ? b : a;
                double c = 1.0, sn = 0.0;
                if (qq < n) {
                    double app = A[pp * n + pp], aqq = A[qq * n + qq], apq = A[pp * n + qq];
                    if (fabs(apq) > 1e-280 && fabs(apq) > 2.2e-16 * sqrt(fabs(app * aqq))) {
                        double th = (aqq - app) / (2.0 * apq);
                        double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
                        c = 1.0 / sqrt(1.0 + t * t);
                        sn = t * c;
                        s_rot = 1;
                    }
                }
                s_p[k] = pp;
                s_q[k] = qq;
                s_c[k] = c;
                s_s[k] = sn;
            }
            __syncthreads();
            // columns: A <- A J, V <- V J
            for (int idx = tid; idx < npairs * n; idx += blockDim.x) {
                int k = idx / n, row = idx % n;
                double c = s_c[k], sn = s_s[k];
                if (sn == 0.0) continue;
                int pp = s_p[k], qq = s_q[k];
                double x = A[row * n + pp], y = A[row * n + qq];
                A[row * n + pp] = c * x - sn * y;
                A[row * n + qq] = sn * x + c * y;
                if (want_vectors) {
                    x = V[row * n + pp];
                    y = V[row * n + qq];
                    V[row * n + pp] = c * x - sn * y;
                    V[row * n + qq] = sn * x + c * y;
                }
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int idx = tid; idx < npairs * n; idx += blockDim.x) {
                int k = idx / n, col = idx % n;
                double c = s_c[k], sn = s_s[k];
                if (sn == 0.0) continue;
                int pp = s_p[k], qq = s_q[k];
                double x = A[pp * n + col], y = A[qq * n + col];
                A[pp * n + col] = c * x - sn * y;
                A[qq * n + col] = sn * x + c * y;
            }
            __syncthreads();
            for (int k = tid; k < npairs; k += blockDim.x) {
                if (s_s[k] != 0.0) {
                    int pp = s_p[k], qq = s_q[k];
                    A[pp * n + qq] = 0.0;
                    A[qq * n + pp] = 0.0;
                }
            }
            __syncthreads();
        }
        int done = (s_rot == 0);
        __syncthreads();
        if (done) break;
    }
    if (tid == 0) *sweeps_out = sweep;
}

// Ascending order + sign rule: eps[rank] = A[k][k]; O[rank][:] = V[:, k]
// with the largest-magnitude component made positive (lowest index on ties).
__global__ void k_eig_sort(const double *__restrict__ A, const double *__restrict__ V, int n,
                           int want_vectors, double *__restrict__ eps, double *__restrict__ O) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double ek = A[k * n + k];
    int rank = 0;
    for (int m = 0; m < n; ++m) {
        double em = A[m * n + m];
        rank += (em < ek) || (em == ek && m < k);
    }
    eps[rank] = ek;
    if (!want_vectors) return;
    double big = -1.0, sgn = 1.0;
    for (int r = 0; r < n; ++r) {
        double x = V[r * n + k];
        if (fabs(x) > big) {
            big = fabs(x);
            sgn = x < 0 ? -1.0 : 1.0;
        }
    }
    for (int r = 0; r < n; ++r) O[(int64_t)rank * n + r] = sgn * V[r * n + k];
}

// A = diag(eps0) + v
__global__ void k_h1(const double *__restrict__ p, const double *__restrict__ v, int n,
                     double *__restrict__ A) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    int i = idx / n, k = idx % n;
    double x = v[idx];
    if (i == k) {
        double a = p[i], b = p[i + 1];
        x += (a * a + a * b + b * b) / 3.0;
    }
    A[idx] = x;
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
    int n = c->np;
    PairWave &pw = c->waves[wave];
    c->d_jac.reserve((size_t)2 * n * n);
    c->d_flag.reserve(4);
    double *A = c->d_jac.ptr, *V = c->d_jac.ptr + (size_t)n * n;
    int threads = 256, blocks = (n * n + threads - 1) / threads;
    {
        TimedLaunch tl(c->timer, c->stream, "h1", WPCD_TIME_PAIR);
        hipLaunchKernelGGL(k_h1, dim3(blocks), dim3(threads), 0, c->stream, c->d_p.ptr, pw.v.ptr,
                           n, A);
        WPCD_HIP(hipGetLastError());
    }
    {
        TimedLaunch tl(c->timer, c->stream, "jacobi", WPCD_TIME_PAIR);
        hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(kJacThreads), 0, c->stream, A, V, n,
                           want_vectors ? 1 : 0, 40, c->d_flag.ptr);
        WPCD_HIP(hipGetLastError());
    }
    {
        TimedLaunch tl(c->timer, c->stream, "eig_sort", WPCD_TIME_PAIR);
        hipLaunchKernelGGL(k_eig_sort, dim3((n + 255) / 256), dim3(256), 0, c->stream, A, V, n,
                           want_vectors ? 1 : 0, pw.eps.ptr, pw.O.ptr);
        WPCD_HIP(hipGetLastError());
    }
    pw.h_eps.resize(n);
    WPCD_HIP(hipMemcpyAsync(pw.h_eps.data(), pw.eps.ptr, n * sizeof(double),
                            hipMemcpyDeviceToHost, c->stream));
    int sweeps = 0;
    WPCD_HIP(hipMemcpyAsync(&sweeps, c->d_flag.ptr, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    WPCD_HIP(hipStreamSynchronize(c->stream));
    WPCD_REQUIRE(sweeps < 40, WPCD_E_NOT_CONVERGED, "pair diagonalisation did not converge");
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
