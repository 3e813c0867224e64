// Angular coupling of the permutation kernel for spinless bosons in the
// partial-wave basis |p q (l lam) L> (paper Sec. III.B, eq.(gal): algebraic
// coupling coefficients times angular functions of the rotated momenta).
//
// For channels a = (l, lam), a' = (l', lam') the kernel carries
//   G(q, q', x) = 16 pi^2/(2L+1) sum_M Ybip^{LM}_{l lam}(pi1^, q^)^* Ybip^{LM}_{l' lam'}(pi2^, q'^)
// with pi1 = q' + q/2 and pi2 = -(q + q'/2) at relative cosine x.  The
// product N = G pi1^l pi2^l' q^lam q'^lam' is a rotation-invariant
// polynomial, homogeneous of degree D = l + lam + l' + lam' in the
// components of q and q', hence a polynomial in q^2, q'^2 and y = q q' x:
//   N = sum_{a + b + c = D/2} C_abc (q^2)^a (q'^2)^b y^c.
// Here G is evaluated in long double from Clebsch-Gordan coefficients and
// spherical harmonics built from the explicit Legendre expansion, and the
// C_abc are fitted by least squares on points where the polynomial is exact;
// the GPU then evaluates N and divides by the powers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <vector>

#include "wpcd_internal.h"

namespace wpcd {
namespace {

using ld = long double;
using cld = std::complex<long double>;

ld lfact(int n) {
    ld f = 1.0L;
    for (int k = 2; k <= n; ++k) f *= k;
    return f;
}

ld binom(int n, int k) {
    if (k < 0 || k > n) return 0.0L;
    return lfact(n) / (lfact(k) * lfact(n - k));
}

// <j1 m1 j2 m2 | J M> from the Wigner 3j symbol (Racah's closed form).
ld clebsch(int j1, int m1, int j2, int m2, int J, int M) {
    if (m1 + m2 != M || std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(M) > J) return 0.0L;
    if (J < std::abs(j1 - j2) || J > j1 + j2) return 0.0L;
    // 3j (j1 j2 J; m1 m2 -M)
    const int m3 = -M;
    ld tri = lfact(j1 + j2 - J) * lfact(j1 - j2 + J) * lfact(-j1 + j2 + J) / lfact(j1 + j2 + J + 1);
    ld pre = std::sqrt(tri * lfact(j1 + m1) * lfact(j1 - m1) * lfact(j2 + m2) * lfact(j2 - m2) *
                       lfact(J + m3) * lfact(J - m3));
    ld sum = 0.0L;
    for (int k = 0; k < 64; ++k) {
        const int d1 = k, d2 = J - j2 + k + m1, d3 = J - j1 + k - m2, d4 = j1 + j2 - J - k,
                  d5 = j1 - k - m1, d6 = j2 - k + m2;
        if (d2 < 0 || d3 < 0) continue;
        if (d4 < 0 || d5 < 0 || d6 < 0) break;
        const ld term = 1.0L / (lfact(d1) * lfact(d2) * lfact(d3) * lfact(d4) * lfact(d5) * lfact(d6));
        sum += (k % 2) ? -term : term;
    }
    ld w3j = ((j1 - j2 - m3) % 2 != 0 ? -1.0L : 1.0L) * pre * sum;
    // <j1 m1 j2 m2|J M> = (-1)^(j1 - j2 + M) sqrt(2J+1) 3j(j1 j2 J; m1 m2 -M)
    const int ph = j1 - j2 + M;
    return ((ph % 2 != 0) ? -1.0L : 1.0L) * std::sqrt(2.0L * J + 1.0L) * w3j;
}

// Associated Legendre P_l^m(x), m >= 0, Condon-Shortley phase, from the
// explicit expansion P_l(x) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k,l) x^(l-2k)
// differentiated m times.
ld assoc_legendre(int l, int m, ld x) {
    ld d = 0.0L;
    for (int k = 0; 2 * k <= l; ++k) {
        const int p = l - 2 * k;
        if (p < m) continue;
        ld c = ((k % 2) ? -1.0L : 1.0L) * binom(l, k) * binom(2 * l - 2 * k, l);
        // d^m/dx^m x^p = p!/(p-m)! x^(p-m)
        c *= lfact(p) / lfact(p - m);
        d += c * std::pow(x, (ld)(p - m));
    }
    d /= std::pow(2.0L, (ld)l);
    const ld s = std::sqrt(std::max((ld)0.0L, (1.0L - x) * (1.0L + x)));
    return ((m % 2) ? -1.0L : 1.0L) * std::pow(s, (ld)m) * d;
}

cld sph_harm(int l, int m, ld vx, ld vy, ld vz) {
    const ld r = std::sqrt(vx * vx + vy * vy + vz * vz);
    const ld ct = r > 0 ? vz / r : 1.0L;
    const ld phi = std::atan2(vy, vx);
    const int am = std::abs(m);
    const ld nrm = std::sqrt((2.0L * l + 1.0L) / (4.0L * 3.14159265358979323846264338327950288L) *
                             lfact(l - am) / lfact(l + am));
    cld y = nrm * assoc_legendre(l, am, ct) * std::exp(cld(0.0L, am * phi));
    if (m < 0) y = ((am % 2) ? -1.0L : 1.0L) * std::conj(y);
    return y;
}

cld bipolar(int L, int M, int l, int lam, const ld *a, const ld *b) {
    cld s = 0.0L;
    for (int m = -l; m <= l; ++m) {
        const int m2 = M - m;
        if (std::abs(m2) > lam) continue;
        const ld c = clebsch(l, m, lam, m2, L, M);
        if (c == 0.0L) continue;
        s += c * sph_harm(l, m, a[0], a[1], a[2]) * sph_harm(lam, m2, b[0], b[1], b[2]);
    }
    return s;
}

// G at the canonical geometry q' = q' z^, q = q (sqrt(1-x^2), 0, x).
ld coupling_G(int L, int l, int lam, int l2, int lam2, ld q, ld q2, ld x) {
    const ld s = std::sqrt((1.0L - x) * (1.0L + x));
    const ld qv[3] = {q * s, 0.0L, q * x}, q2v[3] = {0.0L, 0.0L, q2};
    const ld p1[3] = {q2v[0] + 0.5L * qv[0], 0.0L, q2v[2] + 0.5L * qv[2]};
    const ld p2[3] = {-(qv[0] + 0.5L * q2v[0]), 0.0L, -(qv[2] + 0.5L * q2v[2])};
    cld acc = 0.0L;
    for (int M = -L; M <= L; ++M)
        acc += std::conj(bipolar(L, M, l, lam, p1, qv)) * bipolar(L, M, l2, lam2, p2, q2v);
    return 16.0L * 3.14159265358979323846264338327950288L * 3.14159265358979323846264338327950288L /
           (2.0L * L + 1.0L) * acc.real();
}

}  // namespace

// Fill the coefficient table for all channel pairs (row channel a, column
// channel a2, pair index a * nch + a2).  Layout: pairs[p] gives d = D/2,
// the half powers l/2, l'/2, lam/2, lam'/2 and the offset into coef, where
// coefficients are stored for c = 0..d, a = 0..d-c (b = d - c - a).
void coupling_tables(int L, int nch, const int *l, const int *lam, std::vector<McPair> &pairs,
                     std::vector<double> &coef) {
    pairs.assign(nch * nch, McPair{});
    coef.clear();
    for (int a1 = 0; a1 < nch; ++a1)
        for (int a2 = 0; a2 < nch; ++a2) {
            McPair &P = pairs[a1 * nch + a2];
            const int D = l[a1] + lam[a1] + l[a2] + lam[a2];
            const int d = D / 2;
            P.d = d;
            P.hl = l[a1] / 2;
            P.hl2 = l[a2] / 2;
            P.hlam = lam[a1] / 2;
            P.hlam2 = lam[a2] / 2;
            P.off = (int)coef.size();
            // unknowns (c, a): index order c major
            std::vector<std::pair<int, int>> idx;
            for (int c = 0; c <= d; ++c)
                for (int a = 0; a <= d - c; ++a) idx.push_back({c, a});
            const int nu = (int)idx.size();
            // sample points
            const ld qs[] = {0.55L, 0.9L, 1.3L, 1.85L, 2.4L};
            const ld xs[] = {-0.85L, -0.45L, -0.1L, 0.3L, 0.65L, 0.92L};
            std::vector<std::vector<ld>> A;
            std::vector<ld> rhs;
            for (ld q : qs)
                for (ld q2 : qs)
                    for (ld x : xs) {
                        const ld G = coupling_G(L, l[a1], lam[a1], l[a2], lam[a2], q, q2, x);
                        const ld t = q2 * q2 + 0.25L * q * q + q * q2 * x;
                        const ld u = q * q + 0.25L * q2 * q2 + q * q2 * x;
                        const ld Nv = G * std::pow(t, (ld)P.hl) * std::pow(u, (ld)P.hl2) *
                                      std::pow(q * q, (ld)P.hlam) * std::pow(q2 * q2, (ld)P.hlam2);
                        std::vector<ld> row(nu);
                        const ld y = q * q2 * x;
                        for (int k = 0; k < nu; ++k) {
                            const int c = idx[k].first, a = idx[k].second, bb = d - c - a;
                            row[k] = std::pow(q * q, (ld)a) * std::pow(q2 * q2, (ld)bb) * std::pow(y, (ld)c);
                        }
                        A.push_back(row);
                        rhs.push_back(Nv);
                    }
            // normal equations (small, long double), Gaussian elimination with pivoting
            std::vector<std::vector<ld>> NtN(nu, std::vector<ld>(nu + 1, 0.0L));
            for (size_t r = 0; r < A.size(); ++r)
                for (int i = 0; i < nu; ++i) {
                    for (int j = 0; j < nu; ++j) NtN[i][j] += A[r][i] * A[r][j];
                    NtN[i][nu] += A[r][i] * rhs[r];
                }
            for (int i = 0; i < nu; ++i) {
                int piv = i;
                for (int r = i + 1; r < nu; ++r)
                    if (std::fabs(NtN[r][i]) > std::fabs(NtN[piv][i])) piv = r;
                std::swap(NtN[i], NtN[piv]);
                WPCD_REQUIRE(std::fabs(NtN[i][i]) > 0, WPCD_E_INVALID, "coupling fit singular");
                for (int r = 0; r < nu; ++r) {
                    if (r == i) continue;
                    const ld f = NtN[r][i] / NtN[i][i];
                    for (int j = i; j <= nu; ++j) NtN[r][j] -= f * NtN[i][j];
                }
            }
            std::vector<ld> sol(nu);
            for (int i = 0; i < nu; ++i) sol[i] = NtN[i][nu] / NtN[i][i];
            // residual check: the polynomial must reproduce the samples
            ld worst = 0.0L, scale = 0.0L;
            for (size_t r = 0; r < A.size(); ++r) {
                ld v = 0.0L;
                for (int k = 0; k < nu; ++k) v += A[r][k] * sol[k];
                worst = std::max(worst, std::fabs(v - rhs[r]));
                scale = std::max(scale, std::fabs(rhs[r]));
            }
            WPCD_REQUIRE(worst <= 1e-13L * std::max(scale, (ld)1.0L), WPCD_E_INVALID,
                         "coupling polynomial fit failed");
            for (int k = 0; k < nu; ++k) coef.push_back((double)sol[k]);
        }
}

}  // namespace wpcd
