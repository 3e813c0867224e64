/*
 * FP64 CPU oracle for the lattice matrix P0 of the particle-permutation
 * operator in the three-body free wave-packet basis.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liborc.so, which
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load.  The product library never links, includes or calls it,
 * and shares no code with it.
 *
 * What is computed (paper: Sec. II.D "Three-body wave-packet basis",
 * eq.(xij); Sec. III.B, eqs.(perm) and (gal)):
 *
 *   P0[(a j i),(a' j' i')] = <X_ij^a | P | X_i'j'^a'>,  P = P12 P23 + P13 P23,
 *
 * with free wave packets of unit weight, <p|x_i> = theta(p in D_i)/(p sqrt d_i)
 * in the p^2 dp measure (eqs.(ip),(theta_p) with f = 1, normalisation
 * B_i = d_i = width of the bin).  After the delta functions of the
 * permutation kernel are used, each element is a triple integral over the
 * two spectator momenta q, q' and the cosine x between them, with limits
 * that vary with (q, q'):
 *
 *   P0 = (d_i d_i' dq_j dq_j')^(-1/2) Int_Dj dq Int_Dj' dq' q q'
 *                 Int_{x_lo}^{x_hi} dx  G(q,q',x) / (pi1 pi2),
 *   pi1^2 = q'^2 + q^2/4 + q q' x,   pi2^2 = q^2 + q'^2/4 + q q' x,
 *
 * x restricted to [-1,1], pi1 in D_i and pi2 in D_i'.  G = 1 in the s-wave
 * (both permutation terms contribute 1/2).  For l, lambda > 0 G is the
 * angular coupling function, evaluated here directly from Clebsch-Gordan
 * coefficients and spherical harmonics (eq.(gal): coupling coefficients
 * times Legendre-type angular functions).
 *
 * Quadrature rule (the paper only states "a double integral with variable
 * limits"; the reading taken is): n_q-point Gauss-Legendre on each q bin,
 * n_x-point Gauss-Legendre mapped onto the clipped cosine interval.  The
 * cosine interval is parametrised by the pair energy t = pi1^2 = A + B x,
 * an affine map, so the mapped Gauss points are the same points; doing it
 * in t keeps pi1^2 and pi2^2 free of cancellation near p = 0.
 *
 * Pre-selection (Sec. IV.B; the criterion is not given in the paper): a
 * cell pair is kept when the cell energy ranges overlap and the range of
 * pi1 (resp. pi2) over the two q bins meets D_i (resp. D_i').  This is a
 * necessary condition for a nonzero element.  It is evaluated here by brute
 * force over every cell pair, using only IEEE add/sub/mul/compare on
 * host-computed tables.
 *
 * Indexing: bins are 0-based, bin i = [p[i], p[i+1]].  Row index
 * r = (a*Nq + j)*Np + i (i fastest), column likewise.
 *
 * Build with -ffp-contract=off so that the table expressions are rounded
 * exactly as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <complex.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ */
/* Legendre P_n(z) and P_{n-1}(z) by the three-term recurrence. */
static void orc_legendre(int n, long double z, long double *pn, long double *pnm1)
{
    long double a = 1.0L, b = z; /* P_0, P_1 */
    if (n == 0) { *pn = 1.0L; *pnm1 = 0.0L; return; }
    for (int m = 2; m <= n; ++m) {
        long double c = ((2.0L * m - 1.0L) * z * b - (m - 1.0L) * a) / m;
        a = b; b = c;
    }
    *pn = b; *pnm1 = a;
}

/* Gauss-Legendre nodes and weights on [-1,1] by Newton iteration on P_n,
 * w = 2 / ((1 - z^2) P_n'(z)^2), carried out in long double so that the
 * values rounded to double are (almost always) the correctly rounded ones.
 * Nodes ascending.  Returns 0 on success. */
int orc_gauss_legendre(int n, double *x, double *w)
{
    if (n < 1 || n > 256) return 1;
    for (int k = 0; k < (n + 1) / 2; ++k) {
        long double z = cosl(3.14159265358979323846264338327950288L * (k + 0.75L) / (n + 0.5L));
        long double pn, pm, dp;
        for (int it = 0; it < 100; ++it) {
            orc_legendre(n, z, &pn, &pm);
            dp = n * (pm - z * pn) / (1.0L - z * z);
            long double dz = pn / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        orc_legendre(n, z, &pn, &pm);
        dp = n * (pm - z * pn) / (1.0L - z * z);
        long double wk = 2.0L / ((1.0L - z * z) * dp * dp);
        x[n - 1 - k] = (double)z;  w[n - 1 - k] = (double)wk;
        x[k] = -(double)z;         w[k] = (double)wk;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
    return 0;
}

/* Bin edges e[k] = vmax (1 - cos(pi k / (2 n))), k = 0..n: dense near 0.
 * The end points are set to exactly 0 and vmax. */
void orc_cheb_edges(int n, double vmax, double *e)
{
    for (int k = 1; k < n; ++k)
        e[k] = vmax * (1.0 - cos((M_PI * (double)k) / (2.0 * (double)n)));
    e[0] = 0.0;
    e[n] = vmax;
}

/* ------------------------------------------------------------------ */
/* Pre-selection predicate for cell (i,j) against cell (i2,j2). */
static int orc_selected(const double *p, const double *q, int i, int j, int i2, int j2)
{
    double elo1 = p[i] * p[i] + 0.75 * (q[j] * q[j]);
    double ehi1 = p[i + 1] * p[i + 1] + 0.75 * (q[j + 1] * q[j + 1]);
    double elo2 = p[i2] * p[i2] + 0.75 * (q[j2] * q[j2]);
    double ehi2 = p[i2 + 1] * p[i2 + 1] + 0.75 * (q[j2 + 1] * q[j2 + 1]);
    /* energy conservation p^2 + 3/4 q^2 = p'^2 + 3/4 q'^2 */
    if (!(ehi2 > elo1 && ehi1 > elo2)) return 0;
    /* pi1 = |q' + q/2| ranges over [max(0, q'lo - qhi/2, qlo/2 - q'hi), q'hi + qhi/2] */
    double hj_lo = 0.5 * q[j], hj_hi = 0.5 * q[j + 1];
    double hj2_lo = 0.5 * q[j2], hj2_hi = 0.5 * q[j2 + 1];
    double d1 = 0.0, a;
    a = q[j2] - hj_hi;   if (a > d1) d1 = a;
    a = hj_lo - q[j2 + 1]; if (a > d1) d1 = a;
    if (!(p[i + 1] > d1 && p[i] < q[j2 + 1] + hj_hi)) return 0;
    /* pi2 = |q + q'/2| */
    double d2 = 0.0;
    a = q[j] - hj2_hi;   if (a > d2) d2 = a;
    a = hj2_lo - q[j + 1]; if (a > d2) d2 = a;
    if (!(p[i2 + 1] > d2 && p[i2] < q[j + 1] + hj2_hi)) return 0;
    return 1;
}

int orc_is_selected(const double *p, const double *q, int i, int j, int i2, int j2)
{
    return orc_selected(p, q, i, j, i2, j2);
}

/* Row counts by brute force over all columns: cnt[r] for the n_rows rows
 * listed in rows[] (cell-level rows r = j*np + i).  Channel-independent. */
void orc_preselect_counts(int np, int nq, const double *p, const double *q,
                          const int64_t *rows, int64_t n_rows, int64_t *cnt)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_rows; ++t) {
        int64_t r = rows[t];
        int i = (int)(r % np), j = (int)(r / np);
        int64_t c = 0;
        for (int j2 = 0; j2 < nq; ++j2)
            for (int i2 = 0; i2 < np; ++i2)
                c += orc_selected(p, q, i, j, i2, j2);
        cnt[t] = c;
    }
}

/* Column lists (ascending, c = j2*np + i2) for the listed rows; out_ptr[t]
 * is the offset of row t's list in col (caller computed it from counts). */
void orc_preselect_cols(int np, int nq, const double *p, const double *q,
                        const int64_t *rows, int64_t n_rows, const int64_t *out_ptr,
                        int32_t *col)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_rows; ++t) {
        int64_t r = rows[t];
        int i = (int)(r % np), j = (int)(r / np);
        int64_t o = out_ptr[t];
        for (int j2 = 0; j2 < nq; ++j2)
            for (int i2 = 0; i2 < np; ++i2)
                if (orc_selected(p, q, i, j, i2, j2)) col[o++] = (int32_t)(j2 * np + i2);
    }
}

/* ------------------------------------------------------------------ */
/* Angular coupling G^L_{(l lam),(l2 lam2)}(q, q2, x) for spinless bosons.
 *
 * G = (16 pi^2 / (2L+1)) sum_M  Ybip^{LM}_{l lam}(pi1^, q^)^*  Ybip^{LM}_{l2 lam2}(pi2^, q2^)
 * Ybip^{LM}_{l lam}(a, b) = sum_m <l m lam M-m | L M> Y_lm(a) Y_{lam,M-m}(b)
 *
 * evaluated at q2 = q2 z^, q = q (sqrt(1-x^2), 0, x), pi1 = q2 + q/2,
 * pi2 = -(q + q2/2).  The factor 16 pi^2/(2L+1) = 2 (both permutation
 * terms, equal for even l) x 8 pi^2 (integral over the directions of q and
 * q2 at fixed relative angle) / (2L+1) (average over M).  In the s-wave
 * G = 1.                                                               */

static double orc_fact(int n) { double f = 1.0; for (int k = 2; k <= n; ++k) f *= k; return f; }

/* Clebsch-Gordan <j1 m1 j2 m2 | J M> by the Racah formula (integer spins). */
static double orc_cg(int j1, int m1, int j2, int m2, int J, int M)
{
    if (m1 + m2 != M) return 0.0;
    if (abs(m1) > j1 || abs(m2) > j2 || abs(M) > J) return 0.0;
    if (J < abs(j1 - j2) || J > j1 + j2) return 0.0;
    double pre = sqrt((2.0 * J + 1.0) * orc_fact(J + j1 - j2) * orc_fact(J - j1 + j2) *
                      orc_fact(j1 + j2 - J) / orc_fact(j1 + j2 + J + 1));
    pre *= sqrt(orc_fact(J + M) * orc_fact(J - M) * orc_fact(j1 - m1) * orc_fact(j1 + m1) *
                orc_fact(j2 - m2) * orc_fact(j2 + m2));
    double s = 0.0;
    for (int k = 0; k <= j1 + j2 + J; ++k) {
        int a1 = j1 + j2 - J - k, a2 = j1 - m1 - k, a3 = j2 + m2 - k;
        int a4 = J - j2 + m1 + k, a5 = J - j1 - m2 + k;
        if (a1 < 0 || a2 < 0 || a3 < 0 || a4 < 0 || a5 < 0) continue;
        double term = 1.0 / (orc_fact(k) * orc_fact(a1) * orc_fact(a2) * orc_fact(a3) *
                             orc_fact(a4) * orc_fact(a5));
        s += (k % 2 ? -term : term);
    }
    return pre * s;
}

/* Associated Legendre P_l^m(x), m >= 0, with the Condon-Shortley phase. */
static double orc_plm(int l, int m, double x)
{
    double pmm = 1.0;
    if (m > 0) {
        double s = sqrt((1.0 - x) * (1.0 + x)), f = 1.0;
        for (int k = 1; k <= m; ++k) { pmm *= -f * s; f += 2.0; }
    }
    if (l == m) return pmm;
    double pmmp1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pmmp1;
    double pll = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pll = (x * (2.0 * ll - 1.0) * pmmp1 - (ll + m - 1.0) * pmm) / (ll - m);
        pmm = pmmp1; pmmp1 = pll;
    }
    return pll;
}

/* Spherical harmonic Y_lm of the direction of the vector (vx, vy, vz). */
static double complex orc_ylm(int l, int m, double vx, double vy, double vz)
{
    double r = sqrt(vx * vx + vy * vy + vz * vz);
    double ct = (r > 0.0) ? vz / r : 1.0;
    if (ct > 1.0) ct = 1.0;
    if (ct < -1.0) ct = -1.0;
    double phi = atan2(vy, vx);
    int am = abs(m);
    double nrm = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * orc_fact(l - am) / orc_fact(l + am));
    double complex y = nrm * orc_plm(l, am, ct) * cexp(I * am * phi);
    if (m < 0) y = ((am % 2) ? -1.0 : 1.0) * conj(y);
    return y;
}

static double complex orc_bipolar(int L, int M, int l, int lam,
                                  const double *a, const double *b)
{
    double complex s = 0.0;
    for (int m = -l; m <= l; ++m) {
        int m2 = M - m;
        if (abs(m2) > lam) continue;
        double c = orc_cg(l, m, lam, m2, L, M);
        if (c == 0.0) continue;
        s += c * orc_ylm(l, m, a[0], a[1], a[2]) * orc_ylm(lam, m2, b[0], b[1], b[2]);
    }
    return s;
}

double orc_geom_G(int L, int l, int lam, int l2, int lam2, double q, double q2, double x)
{
    double s = sqrt((1.0 - x) * (1.0 + x));
    double qv[3] = { q * s, 0.0, q * x };
    double q2v[3] = { 0.0, 0.0, q2 };
    double pi1[3] = { q2v[0] + 0.5 * qv[0], 0.0, q2v[2] + 0.5 * qv[2] };
    double pi2[3] = { -(qv[0] + 0.5 * q2v[0]), 0.0, -(qv[2] + 0.5 * q2v[2]) };
    double complex acc = 0.0;
    for (int M = -L; M <= L; ++M)
        acc += conj(orc_bipolar(L, M, l, lam, pi1, qv)) * orc_bipolar(L, M, l2, lam2, pi2, q2v);
    return 16.0 * M_PI * M_PI / (2.0 * L + 1.0) * creal(acc);
}

/* All channel pairs of G at one node: G[a*nch + a2].  Same formula as
 * orc_geom_G; the spherical harmonics of the four directions are computed
 * once per node and shared by the pairs, the Clebsch-Gordan coefficients
 * come from the caller's table cg[a][M+L][m+l] = <l m lam M-m | L M>.    */
#define ORC_LMAX 4
static void orc_geom_G_all(int L, int nch, const int *l, const int *lam, const double *cg,
                           double q, double q2, double x, double *G)
{
    double s = sqrt((1.0 - x) * (1.0 + x));
    double qv[3] = { q * s, 0.0, q * x };
    double q2v[3] = { 0.0, 0.0, q2 };
    double pi1[3] = { q2v[0] + 0.5 * qv[0], 0.0, q2v[2] + 0.5 * qv[2] };
    double pi2[3] = { -(qv[0] + 0.5 * q2v[0]), 0.0, -(qv[2] + 0.5 * q2v[2]) };
    /* Y[dir][l][m + ORC_LMAX] for dir = pi1, q, pi2, q2 */
    double complex Y[4][ORC_LMAX + 1][2 * ORC_LMAX + 1];
    const double *dirs[4] = { pi1, qv, pi2, q2v };
    for (int d = 0; d < 4; ++d)
        for (int ll = 0; ll <= ORC_LMAX; ++ll)
            for (int m = -ll; m <= ll; ++m)
                Y[d][ll][m + ORC_LMAX] = orc_ylm(ll, m, dirs[d][0], dirs[d][1], dirs[d][2]);
    const int W = 2 * ORC_LMAX + 1, WM = 2 * 8 + 1;
    for (int a = 0; a < nch; ++a)
        for (int a2 = 0; a2 < nch; ++a2) {
            double complex acc = 0.0;
            for (int M = -L; M <= L; ++M) {
                double complex b1 = 0.0, b2 = 0.0;
                for (int m = -l[a]; m <= l[a]; ++m) {
                    int mu = M - m;
                    if (abs(mu) > lam[a]) continue;
                    b1 += cg[(a * WM + (M + L)) * W + (m + ORC_LMAX)] *
                          Y[0][l[a]][m + ORC_LMAX] * Y[1][lam[a]][mu + ORC_LMAX];
                }
                for (int m = -l[a2]; m <= l[a2]; ++m) {
                    int mu = M - m;
                    if (abs(mu) > lam[a2]) continue;
                    b2 += cg[(a2 * WM + (M + L)) * W + (m + ORC_LMAX)] *
                          Y[2][l[a2]][m + ORC_LMAX] * Y[3][lam[a2]][mu + ORC_LMAX];
                }
                acc += conj(b1) * b2;
            }
            G[a * nch + a2] = 16.0 * M_PI * M_PI / (2.0 * L + 1.0) * creal(acc);
        }
}

/* Clebsch-Gordan table of a channel list for orc_geom_G_all:
 * cg[a][M + L][m + LMAX] = <l_a m lam_a M-m | L M> (zero where |m| > l_a). */
static void orc_cg_table(int L, int nch, const int *l, const int *lam, double *cg)
{
    for (int a = 0; a < nch; ++a)
        for (int M = -L; M <= L; ++M)
            for (int m = -ORC_LMAX; m <= ORC_LMAX; ++m)
                cg[(a * 17 + (M + L)) * (2 * ORC_LMAX + 1) + (m + ORC_LMAX)] =
                    (abs(m) <= l[a]) ? orc_cg(l[a], m, lam[a], M - m, L, M) : 0.0;
}

/* Every channel pair of G at one node through the node-shared routine the
 * element quadrature uses (exported so the tests can compare it with
 * orc_geom_G pair by pair).  G[a*nch + a2]; returns 0, or 1 for sizes
 * outside nch <= 8, L <= 8, l, lam <= 4.                                 */
int orc_geom_G_table(int L, int nch, const int *l, const int *lam, double q, double q2,
                     double x, double *G)
{
    if (nch < 1 || nch > 8 || L < 0 || L > 8) return 1;
    for (int a = 0; a < nch; ++a)
        if (l[a] < 0 || l[a] > ORC_LMAX || lam[a] < 0 || lam[a] > ORC_LMAX) return 1;
    double cg[8 * 17 * (2 * ORC_LMAX + 1)];
    orc_cg_table(L, nch, l, lam, cg);
    orc_geom_G_all(L, nch, l, lam, cg, q, q2, x, G);
    return 0;
}

/* ------------------------------------------------------------------ */
/* One cell-pair block of P0: out[a*nch + a2] for channel rows a, columns a2.
 * i, j: row cell; i2, j2: column cell (0-based bins).
 * gq/wq: n_q Gauss points on [-1,1]; gx/wx: n_x Gauss points on [-1,1].
 * L, l[], lam[]: three-body total orbital momentum and channel list.       */
void orc_p0_block(const double *p, const double *q, int i, int j, int i2, int j2,
                  int nq_pts, const double *gq, const double *wq,
                  int nx_pts, const double *gx, const double *wx,
                  int L, int nch, const int *l, const int *lam, double *out)
{
    double dp1 = p[i + 1] - p[i], dp2 = p[i2 + 1] - p[i2];
    double dq1 = q[j + 1] - q[j], dq2 = q[j2 + 1] - q[j2];
    double qm1 = 0.5 * (q[j + 1] + q[j]), qh1 = 0.5 * dq1;
    double qm2 = 0.5 * (q[j2 + 1] + q[j2]), qh2 = 0.5 * dq2;
    int swave = (nch == 1 && L == 0 && l[0] == 0 && lam[0] == 0);
    for (int c = 0; c < nch * nch; ++c) out[c] = 0.0;
    /* Clebsch-Gordan table per channel: cg[a][M + L][m + LMAX] */
    double cg[8 * 17 * (2 * ORC_LMAX + 1)];
    double Gn[64];
    if (!swave) orc_cg_table(L, nch, l, lam, cg);

    for (int a = 0; a < nq_pts; ++a) {
        double qa = qm1 + qh1 * gq[a];
        double wa = qh1 * wq[a];
        for (int b = 0; b < nq_pts; ++b) {
            double qb = qm2 + qh2 * gq[b];
            double wb = qh2 * wq[b];
            /* pi1^2 = A + B x, pi2^2 = C + B x, x in [-1, 1] */
            double A = qb * qb + 0.25 * qa * qa;
            double B = qa * qb;
            /* at x = -1 and x = +1: pi1 = |q' -+ q/2|, pi2 = |q -+ q'/2|; the
             * squares are formed directly (no cancellation near q' = q/2) */
            double tlo = (qb - 0.5 * qa) * (qb - 0.5 * qa), thi = (qb + 0.5 * qa) * (qb + 0.5 * qa);
            double ulo = (qa - 0.5 * qb) * (qa - 0.5 * qb), uhi = (qa + 0.5 * qb) * (qa + 0.5 * qb);
            /* pi1 in [p_i, p_{i+1}] */
            double p1l = p[i] * p[i], p1h = p[i + 1] * p[i + 1];
            double p2l = p[i2] * p[i2], p2h = p[i2 + 1] * p[i2 + 1];
            /* convert each constraint to both variables: u - t = D */
            double D = 0.75 * (qa - qb) * (qa + qb); /* = 3/4 (q^2 - q'^2) */
            double lo_t = tlo, hi_t = thi;
            if (p1l > lo_t) lo_t = p1l;
            if (p2l - D > lo_t) lo_t = p2l - D;
            if (p1h < hi_t) hi_t = p1h;
            if (p2h - D < hi_t) hi_t = p2h - D;
            double lo_u = ulo, hi_u = uhi;
            if (p2l > lo_u) lo_u = p2l;
            if (p1l + D > lo_u) lo_u = p1l + D;
            if (p2h < hi_u) hi_u = p2h;
            if (p1h + D < hi_u) hi_u = p1h + D;
            if (!(hi_t > lo_t)) continue;
            double ht = 0.5 * (hi_t - lo_t);
            double hu = 0.5 * (hi_u - lo_u);
            double h = 0.5 * (ht + hu); /* equal up to rounding */
            /* dx = dt / B, and the q q' in the measure cancels 1/B */
            for (int c = 0; c < nx_pts; ++c) {
                double s = h * (1.0 + gx[c]);
                double t = lo_t + s;   /* pi1^2 */
                double u = lo_u + s;   /* pi2^2 */
                double f = wx[c] * h / sqrt(t * u);
                if (swave) {
                    out[0] += wa * wb * f;
                } else {
                    double x = (t - A) / B;
                    if (x > 1.0) x = 1.0;
                    if (x < -1.0) x = -1.0;
                    orc_geom_G_all(L, nch, l, lam, cg, qa, qb, x, Gn);
                    for (int cab = 0; cab < nch * nch; ++cab)
                        out[cab] += wa * wb * f * Gn[cab];
                }
            }
        }
    }
    double nrm = 1.0 / sqrt(dp1 * dp2 * dq1 * dq2);
    for (int c = 0; c < nch * nch; ++c) out[c] *= nrm;
}

/* P0 values for a list of cell pairs (rows[t], cols[t]); out has nch*nch
 * values per pair (row channel major).                                    */
void orc_p0_pairs(int np, int nqb, const double *p, const double *q,
                  int nq_pts, int nx_pts, int L, int nch, const int *l, const int *lam,
                  const int64_t *rows, const int32_t *cols, int64_t n_pairs, double *out)
{
    double gq[256], wq[256], gx[256], wx[256];
    orc_gauss_legendre(nq_pts, gq, wq);
    orc_gauss_legendre(nx_pts, gx, wx);
    (void)nqb;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < n_pairs; ++t) {
        int64_t r = rows[t];
        int32_t c = cols[t];
        int i = (int)(r % np), j = (int)(r / np);
        int i2 = (int)(c % np), j2 = (int)(c / np);
        orc_p0_block(p, q, i, j, i2, j2, nq_pts, gq, wq, nx_pts, gx, wx, L, nch, l, lam,
                     out + t * (int64_t)nch * nch);
    }
}
