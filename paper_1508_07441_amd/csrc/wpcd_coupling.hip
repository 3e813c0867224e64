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
#include <map>
#include <mutex>
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

namespace {
ld ylm_norm(int l, int am) {
    return std::sqrt((2.0L * l + 1.0L) / (4.0L * 3.14159265358979323846264338327950288L) *
                     lfact(l - am) / lfact(l + am));
}
// Y_lm = ylm_norm(l,|m|) P_l^|m|(cos theta) e^{i|m| phi} for m >= 0 and
// (-1)^m times the conjugate for m < 0; with phi in {0, pi} all are real.
ld ylm_sign(int m, int azimuth_sign) {
    const int am = std::abs(m);
    ld s = (m < 0 && (am % 2)) ? -1.0L : 1.0L;
    if (azimuth_sign < 0 && (am % 2)) s = -s;
    return s;
}
}  // namespace

// Direct form of G for every channel pair at the canonical geometry
// (q' along z, q in the xz plane at cosine x): pi1 = q' + q/2 has a
// non-negative x component (azimuth 0), q too, pi2 = -(q + q'/2) a
// non-positive one (azimuth pi), and Y_lam' mu(z) = delta_mu0
// sqrt((2 lam' + 1)/(4 pi)).  Hence
//   G = sum_{M, m1} coef P_l^|m1|(c1) P_lam^|M-m1|(x) P_l'^|M|(c2),
// c1, c2 the polar cosines of pi1, pi2, with every constant in coef.  The
// terms are validated against coupling_G (long double) at sample points.
static void coupling_terms_compute(int L, int nch, const int *l, const int *lam,
                                   std::vector<McTerm> &terms, std::vector<int> &first) {
    terms.clear();
    first.assign(nch * nch + 1, 0);
    const ld pi = 3.14159265358979323846264338327950288L;
    for (int a1 = 0; a1 < nch; ++a1)
        for (int a2 = 0; a2 < nch; ++a2) {
            const int p = a1 * nch + a2;
            first[p] = (int)terms.size();
            const int la = l[a1], lb = lam[a1], lc = l[a2], ld2 = lam[a2];
            for (int M = -L; M <= L; ++M) {
                if (std::abs(M) > lc) continue;
                const ld cg2 = clebsch(lc, M, ld2, 0, L, M);
                if (cg2 == 0.0L) continue;
                for (int m1 = -la; m1 <= la; ++m1) {
                    const int m2 = M - m1;
                    if (std::abs(m2) > lb) continue;
                    const ld cg1 = clebsch(la, m1, lb, m2, L, M);
                    if (cg1 == 0.0L) continue;
                    const ld c = 16.0L * pi * pi / (2.0L * L + 1.0L) * cg1 * cg2 *
                                 std::sqrt((2.0L * ld2 + 1.0L) / (4.0L * pi)) *
                                 ylm_norm(la, std::abs(m1)) * ylm_sign(m1, +1) *
                                 ylm_norm(lb, std::abs(m2)) * ylm_sign(m2, +1) *
                                 ylm_norm(lc, std::abs(M)) * ylm_sign(M, -1);
                    McTerm T;
                    T.coef = (double)c;
                    T.i1 = la * (la + 1) / 2 + std::abs(m1);
                    T.iq = lb * (lb + 1) / 2 + std::abs(m2);
                    T.i2 = lc * (lc + 1) / 2 + std::abs(M);
                    terms.push_back(T);
                }
            }
            // validation against the bipolar-harmonic evaluation
            const ld qs[] = {0.6L, 1.4L, 2.3L}, xs[] = {-0.8L, -0.2L, 0.35L, 0.9L};
            ld worst = 0.0L, scale = 0.0L;
            for (ld q : qs)
                for (ld q2 : qs)
                    for (ld x : xs) {
                        const ld G = coupling_G(L, la, lb, lc, ld2, q, q2, x);
                        const ld sx = std::sqrt((1.0L - x) * (1.0L + x));
                        const ld p1x = 0.5L * q * sx, p1z = q2 + 0.5L * q * x;
                        const ld p2x = -q * sx, p2z = -(q * x + 0.5L * q2);
                        const ld c1 = p1z / std::sqrt(p1x * p1x + p1z * p1z);
                        const ld c2 = p2z / std::sqrt(p2x * p2x + p2z * p2z);
                        ld v = 0.0L;
                        for (int k = first[p]; k < (int)terms.size(); ++k) {
                            const McTerm &T = terms[k];
                            auto P = [&](int idx, ld cc) {
                                int ll = 0;
                                while ((ll + 1) * (ll + 2) / 2 <= idx) ++ll;
                                return assoc_legendre(ll, idx - ll * (ll + 1) / 2, cc);
                            };
                            v += (ld)T.coef * P(T.i1, c1) * P(T.iq, x) * P(T.i2, c2);
                        }
                        worst = std::max(worst, std::fabs(v - G));
                        scale = std::max(scale, std::fabs(G));
                    }
            WPCD_REQUIRE(worst <= 1e-13L * std::max(scale, (ld)1.0L), WPCD_E_INVALID,
                         "direct coupling terms do not reproduce the coupling");
        }
    first[nch * nch] = (int)terms.size();
}

// Fill the coefficient table for all channel pairs (row channel a, column
// channel a2, pair index a * nch + a2).  Layout: pairs[p] gives d = D/2,
// the half powers l/2, l'/2, lam/2, lam'/2 and the offset into coef, where
// coefficients are stored for c = 0..d, a = 0..d-c (b = d - c - a).
static void coupling_tables_compute(int L, int nch, const int *l, const int *lam,
                                    std::vector<McPair> &pairs, std::vector<double> &coef) {
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
            // unknowns (c, a): index order c major.  The monomial
            // (q^2)^a (q'^2)^b y^c is q^(2a+c) q'^(2b+c) x^c; N carries the
            // factor q^lam q'^lam', so terms with 2a + c < lam or 2b + c < lam'
            // are exactly zero.  They are left out of the fit: a rounding-size
            // coefficient there would be amplified by 1/q^lam on the nodes
            // near q = 0.
            std::vector<std::pair<int, int>> idx, all;
            for (int c = 0; c <= d; ++c)
                for (int a = 0; a <= d - c; ++a) {
                    all.push_back({c, a});
                    const int b = d - c - a;
                    if (2 * a + c >= lam[a1] && 2 * b + c >= lam[a2]) idx.push_back({c, a});
                }
            const int nu = (int)idx.size();
            // sample points: for fixed (q, q') the polynomial has degree d <= 8
            // in y = q q' x, so at least d + 1 distinct cosines are needed
            // (12 here); the homogeneous (q^2, q'^2) parts of degree <= 8 need
            // >= 9 distinct ratios q^2/q'^2 (the 6 x 6 grid gives 31)
            const ld qs[] = {0.55L, 0.9L, 1.3L, 1.85L, 2.4L, 3.1L};
            const ld xs[] = {-0.97L, -0.85L, -0.68L, -0.45L, -0.27L, -0.1L,
                             0.08L,  0.3L,   0.47L,  0.65L,  0.81L,  0.92L};
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
            // and off the samples (an underdetermined fit interpolates the
            // samples but not the function)
            {
                const ld vq[] = {0.7L, 1.15L, 2.05L, 2.7L};
                const ld vx[] = {-0.91L, -0.33L, 0.17L, 0.59L, 0.88L};
                ld vworst = 0.0L, vscale = 0.0L;
                for (ld q : vq)
                    for (ld q2 : vq)
                        for (ld x : vx) {
                            const ld G = coupling_G(L, l[a1], lam[a1], l[a2], lam[a2], q, q2, x);
                            const ld t = q2 * q2 + 0.25L * q * q + q * q2 * x;
                            const ld u = q * q + 0.25L * q2 * q2 + q * q2 * x;
                            const ld Nv = G * std::pow(t, (ld)P.hl) * std::pow(u, (ld)P.hl2) *
                                          std::pow(q * q, (ld)P.hlam) *
                                          std::pow(q2 * q2, (ld)P.hlam2);
                            const ld y = q * q2 * x;
                            ld v = 0.0L;
                            for (int k = 0; k < nu; ++k) {
                                const int c = idx[k].first, a = idx[k].second, bb = d - c - a;
                                v += sol[k] * std::pow(q * q, (ld)a) * std::pow(q2 * q2, (ld)bb) *
                                     std::pow(y, (ld)c);
                            }
                            vworst = std::max(vworst, std::fabs(v - Nv));
                            vscale = std::max(vscale, std::fabs(Nv));
                        }
                WPCD_REQUIRE(vworst <= 1e-12L * std::max(vscale, (ld)1.0L), WPCD_E_INVALID,
                             "coupling polynomial does not reproduce the coupling off the fit points");
            }
            // stored for every (c, a) of the full layout, zeros included
            for (const auto &ca : all) {
                ld v = 0.0L;
                for (int k = 0; k < nu; ++k)
                    if (idx[k] == ca) v = sol[k];
                coef.push_back((double)v);
            }
        }
}

// ---- three nucleons, pair s-waves (Sec. III.B eq.(gal) with spin and
// isospin; Sec. V.A).  Arguments of the 6j symbols are given doubled (2j),
// so half-integers stay integers.
namespace {

// Triangle coefficient Delta(a b c) of doubled arguments.
ld tri_delta(int a2, int b2, int c2) {
    return std::sqrt(lfact((a2 + b2 - c2) / 2) * lfact((a2 - b2 + c2) / 2) *
                     lfact((-a2 + b2 + c2) / 2) / lfact((a2 + b2 + c2) / 2 + 1));
}

bool triad(int a2, int b2, int c2) {
    return c2 >= std::abs(a2 - b2) && c2 <= a2 + b2 && (a2 + b2 + c2) % 2 == 0;
}

// Wigner 6j symbol {j1 j2 j3; j4 j5 j6} by Racah's sum (doubled arguments).
ld sixj2(int j1, int j2, int j3, int j4, int j5, int j6) {
    if (!triad(j1, j2, j3) || !triad(j1, j5, j6) || !triad(j4, j2, j6) || !triad(j4, j5, j3))
        return 0.0L;
    const ld pre = tri_delta(j1, j2, j3) * tri_delta(j1, j5, j6) * tri_delta(j4, j2, j6) *
                   tri_delta(j4, j5, j3);
    const int a1 = (j1 + j2 + j3) / 2, a2 = (j1 + j5 + j6) / 2, a3 = (j4 + j2 + j6) / 2,
              a4 = (j4 + j5 + j3) / 2;
    const int b1 = (j1 + j2 + j4 + j5) / 2, b2 = (j2 + j3 + j5 + j6) / 2,
              b3 = (j3 + j1 + j6 + j4) / 2;
    const int tmin = std::max(std::max(a1, a2), std::max(a3, a4));
    const int tmax = std::min(b1, std::min(b2, b3));
    ld sum = 0.0L;
    for (int t = tmin; t <= tmax; ++t) {
        const ld term = lfact(t + 1) / (lfact(t - a1) * lfact(t - a2) * lfact(t - a3) *
                                        lfact(t - a4) * lfact(b1 - t) * lfact(b2 - t) *
                                        lfact(b3 - t));
        sum += (t % 2 ? -term : term);
    }
    return pre * sum;
}

// <(x_a 1/2) X | C | (x_b 1/2) X> for two spins 1/2 of the pair (2, 3)
// coupled to x and the third to X (2X = two_X): the cyclic permutation of
// the three particles between recoupled states,
//   (-1)^(x_b) sqrt((2 x_a + 1)(2 x_b + 1)) {1/2 1/2 x_b; 1/2 X x_a}.
ld cyclic_recoupling(int xa, int xb, int two_X) {
    const ld v = std::sqrt((ld)((2 * xa + 1) * (2 * xb + 1))) *
                 sixj2(1, 1, 2 * xb, 1, two_X, 2 * xa);
    return (xb % 2) ? -v : v;
}
}  // namespace

// g_ab = (1/2)(sigma_ab tau_ab + sigma_ba tau_ba) for channels a = (s_a,
// t_a): spin part with total 2S = two_S, isospin part with total 1/2; the
// second term is the other cyclic permutation (the inverse, whose matrix is
// the transpose).  Stored as McPair entries of degree 0 with one
// coefficient each, so the multichannel element kernels multiply the
// s-wave integrand by g_ab.
void nucleon_tables(int two_S, int nch, const int *s, const int *t, std::vector<McPair> &pairs,
                    std::vector<double> &coef, std::vector<double> &g) {
    pairs.assign(nch * nch, McPair{});
    coef.assign(nch * nch, 0.0);
    g.assign(nch * nch, 0.0);
    for (int a = 0; a < nch; ++a)
        for (int b = 0; b < nch; ++b) {
            const ld sab = cyclic_recoupling(s[a], s[b], two_S), sba = cyclic_recoupling(s[b], s[a], two_S);
            const ld tab = cyclic_recoupling(t[a], t[b], 1), tba = cyclic_recoupling(t[b], t[a], 1);
            const double v = (double)(0.5L * (sab * tab + sba * tba));
            McPair &P = pairs[a * nch + b];
            P.d = 0;
            P.hl = P.hl2 = P.hlam = P.hlam2 = 0;
            P.off = a * nch + b;
            coef[a * nch + b] = v;
            g[a * nch + b] = v;
        }
}

// Both are pure functions of (L, channels): computed once per process for
// each channel set and shared.
static std::vector<int> channel_key(int L, int nch, const int *l, const int *lam) {
    std::vector<int> k{L, nch};
    for (int a = 0; a < nch; ++a) {
        k.push_back(l[a]);
        k.push_back(lam[a]);
    }
    return k;
}

void coupling_tables(int L, int nch, const int *l, const int *lam, std::vector<McPair> &pairs,
                     std::vector<double> &coef) {
    static std::mutex mu;
    static std::map<std::vector<int>, std::pair<std::vector<McPair>, std::vector<double>>> memo;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = channel_key(L, nch, l, lam);
    auto it = memo.find(key);
    if (it == memo.end()) {
        std::vector<McPair> pr;
        std::vector<double> cf;
        coupling_tables_compute(L, nch, l, lam, pr, cf);
        it = memo.emplace(key, std::make_pair(std::move(pr), std::move(cf))).first;
    }
    pairs = it->second.first;
    coef = it->second.second;
}

void coupling_terms(int L, int nch, const int *l, const int *lam, std::vector<McTerm> &terms,
                    std::vector<int> &first) {
    static std::mutex mu;
    static std::map<std::vector<int>, std::pair<std::vector<McTerm>, std::vector<int>>> memo;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = channel_key(L, nch, l, lam);
    auto it = memo.find(key);
    if (it == memo.end()) {
        std::vector<McTerm> tm;
        std::vector<int> fi;
        coupling_terms_compute(L, nch, l, lam, tm, fi);
        it = memo.emplace(key, std::make_pair(std::move(tm), std::move(fi))).first;
    }
    terms = it->second.first;
    first = it->second.second;
}

}  // namespace wpcd
