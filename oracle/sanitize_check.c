/* Host sanitizer run of the oracle's C part.  TEST INFRASTRUCTURE ONLY.
 *
 * Built together with wpcd_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer (no recovery) by the CPU test suite, this
 * program walks every exported routine over a small Chebyshev lattice --
 * Gauss-Legendre rules of every supported order, the bin edges, the brute-
 * force pre-selection of all cell rows (counts and column lists), the
 * angular coupling (single pairs and node tables) and the P0 cell-pair
 * blocks of the s-wave and of the three-channel L = 2 set (Sec. III.B
 * eqs.(perm),(gal)) -- and prints every result, so that the test can also
 * compare them with the same routines of the normally built library.
 *
 * Output, one record a line:
 *   gl <n> <sum of |x|> <sum of w>
 *   edges <k> <e_k>
 *   row <r> <count> ; col <c>      (the selected columns of each row)
 *   G <L> <a> <b> <value>          (pairs of the L = 2 set at fixed nodes)
 *   T <value>                      (the node table of the same set)
 *   s <t> <value>                  (s-wave P0 element of selected pair t)
 *   m <t> <k> <value>              (L = 2 block entry k of selected pair t)
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_gauss_legendre(int n, double *x, double *w);
void orc_cheb_edges(int n, double vmax, double *e);
int orc_is_selected(const double *p, const double *q, int i, int j, int i2, int j2);
void orc_preselect_counts(int np, int nq, const double *p, const double *q,
                          const int64_t *rows, int64_t n_rows, int64_t *cnt);
void orc_preselect_cols(int np, int nq, const double *p, const double *q,
                        const int64_t *rows, int64_t n_rows, const int64_t *out_ptr,
                        int32_t *col);
double orc_geom_G(int L, int l, int lam, int l2, int lam2, double q, double q2, double x);
int orc_geom_G_table(int L, int nch, const int *l, const int *lam, double q, double q2,
                     double x, double *G);
void orc_p0_pairs(int np, int nqb, const double *p, const double *q,
                  int nq_pts, int nx_pts, int L, int nch, const int *l, const int *lam,
                  const int64_t *rows, const int32_t *cols, int64_t n_pairs, double *out);

enum { NP = 6, NQ = 5, NGQ = 4, NGX = 8 };

static void *xmalloc(size_t n)
{
    void *v = malloc(n ? n : 1);
    if (!v) { fprintf(stderr, "out of memory\n"); exit(2); }
    return v;
}

int main(void)
{
    /* every rule order the element routines accept */
    for (int n = 1; n <= 256; ++n) {
        double *x = xmalloc(sizeof(double) * n), *w = xmalloc(sizeof(double) * n);
        if (orc_gauss_legendre(n, x, w)) return 3;
        double sx = 0.0, sw = 0.0;
        for (int k = 0; k < n; ++k) { sx += x[k] < 0 ? -x[k] : x[k]; sw += w[k]; }
        printf("gl %d %.17g %.17g\n", n, sx, sw);
        free(x);
        free(w);
    }
    double p[NP + 1], q[NQ + 1];
    orc_cheb_edges(NP, 6.0, p);
    orc_cheb_edges(NQ, 6.0, q);
    for (int k = 0; k <= NP; ++k) printf("edges %d %.17g\n", k, p[k]);

    /* pre-selection of every cell row */
    const int64_t nrow = (int64_t)NP * NQ;
    int64_t *rows = xmalloc(sizeof(int64_t) * nrow), *cnt = xmalloc(sizeof(int64_t) * nrow);
    int64_t *ptr = xmalloc(sizeof(int64_t) * (nrow + 1));
    for (int64_t r = 0; r < nrow; ++r) rows[r] = r;
    orc_preselect_counts(NP, NQ, p, q, rows, nrow, cnt);
    ptr[0] = 0;
    for (int64_t r = 0; r < nrow; ++r) ptr[r + 1] = ptr[r] + cnt[r];
    const int64_t nnz = ptr[nrow];
    int32_t *col = xmalloc(sizeof(int32_t) * nnz);
    orc_preselect_cols(NP, NQ, p, q, rows, nrow, ptr, col);
    int64_t *prow = xmalloc(sizeof(int64_t) * nnz);
    for (int64_t r = 0; r < nrow; ++r) {
        printf("row %lld %lld", (long long)r, (long long)cnt[r]);
        for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
            prow[e] = r;
            if (!orc_is_selected(p, q, (int)(r % NP), (int)(r / NP), col[e] % NP, col[e] / NP))
                return 4;
            printf(" %d", col[e]);
        }
        printf("\n");
    }

    /* angular coupling of the L = 2 set */
    const int l[3] = {0, 2, 2}, lam[3] = {2, 0, 2};
    const double nodes[3][3] = {{0.7, 1.3, -0.4}, {2.0, 0.5, 0.9}, {1.1, 1.1, 1.0}};
    double T[9];
    for (int n = 0; n < 3; ++n) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                printf("G 2 %d %d %.17g\n", a, b,
                       orc_geom_G(2, l[a], lam[a], l[b], lam[b], nodes[n][0], nodes[n][1],
                                  nodes[n][2]));
        if (orc_geom_G_table(2, 3, l, lam, nodes[n][0], nodes[n][1], nodes[n][2], T)) return 5;
        for (int k = 0; k < 9; ++k) printf("T %.17g\n", T[k]);
    }

    /* P0 cell-pair blocks of every selected pair */
    const int l0[1] = {0}, lam0[1] = {0};
    double *vs = xmalloc(sizeof(double) * nnz), *vm = xmalloc(sizeof(double) * 9 * nnz);
    orc_p0_pairs(NP, NQ, p, q, NGQ, NGX, 0, 1, l0, lam0, prow, col, nnz, vs);
    orc_p0_pairs(NP, NQ, p, q, NGQ, NGX, 2, 3, l, lam, prow, col, nnz, vm);
    for (int64_t t = 0; t < nnz; ++t) {
        printf("s %lld %.17g\n", (long long)t, vs[t]);
        for (int k = 0; k < 9; ++k) printf("m %lld %d %.17g\n", (long long)t, k, vm[9 * t + k]);
    }
    free(rows);
    free(cnt);
    free(ptr);
    free(col);
    free(prow);
    free(vs);
    free(vm);
    return 0;
}
