/*
 * wpcd.h -- C ABI of libwpcd.so, the MI355X (gfx950) implementation of the
 * hot path of the wave-packet continuum discretization (WPCD) method for
 * three-body Faddeev scattering (Pomerantsev, Kukulin, Rubtsova, Sakhiev,
 * "Fast GPU-based calculations in few-body quantum scattering").
 *
 * The calls follow the paper's four-step scheme (Sec. III.C): process the
 * input (bases, pair potential, pair diagonalisation), build the lattice
 * permutation matrix P0, then for each energy build the channel resolvent
 * and solve the matrix Faddeev equation for the on-shell amplitudes.
 *
 * Conventions used throughout:
 *  - Units hbar = m = 1: pair kinetic energy p^2, spectator energy 3/4 q^2.
 *  - Free wave packets have unit weight (eqs.(ip),(theta_p) with f = 1).
 *  - Bins are 0-based: bin i is [p[i], p[i+1]].  A lattice cell (i, j) has
 *    cell index j*n_p + i.  The channel-basis index of (channel a,
 *    spectator bin j, pair state k) is (a*n_q + j)*n_p + k.
 *  - All host pointers are owned by the caller and are only read or written
 *    during the call.  The context owns every device allocation.
 *  - Every call returns a wpcd_status; no C++ exception crosses the ABI.
 *    On an error, outputs are left untouched and wpcd_last_error() holds a
 *    message.  A context is not thread-safe: use one per host thread.
 */
#ifndef WPCD_H
#define WPCD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wpcd_ctx wpcd_ctx;

typedef enum {
    WPCD_OK = 0,
    WPCD_E_INVALID = 1,          /* bad argument or unsupported size */
    WPCD_E_NOMEM = 2,            /* device or host allocation failed */
    WPCD_E_DEVICE = 3,           /* a HIP runtime call failed */
    WPCD_E_NOT_CONVERGED = 4,    /* iterative solve hit max_iter (per energy) */
    WPCD_E_BELOW_THRESHOLD = 5,  /* E at or below the two-body threshold (per energy) */
    WPCD_E_ON_EDGE = 6,          /* an on-shell momentum sits on a bin edge (per energy) */
    WPCD_E_STATE = 7,            /* calls made out of order */
    WPCD_E_STAGNATED = 8         /* iterative solve stopped: two restart cycles
                                    without halving the smallest true residual
                                    (per energy) */
} wpcd_status;

typedef enum {
    WPCD_FP64 = 0,          /* FP64 everywhere */
    WPCD_MIXED = 1,         /* P0 accumulated in FP32 with compensated sums */
    WPCD_MIXED_REFINE = 2,  /* wpcd_solve only, on a WPCD_MIXED P0: the two
                               intermediate panels of the kernel product are
                               FP32 inside the Krylov iterations; each restart
                               forms the true residual with FP64 panels
                               (iterative refinement) */
    WPCD_MIXED_BF16 = 3     /* wpcd_solve only, on a WPCD_MIXED P0: as
                               WPCD_MIXED_REFINE, with the two block products
                               of the inner iterations (V~ and O, Sec. III.B
                               eq.(perm_z)) on the BF16 matrix cores with FP32
                               accumulation */
} wpcd_precision;

/* Lattice basis (Sec. II.D, eq.(xij); channels eq.(si)).
 * edge_kind 0: edges x_k = x_max (1 - cos(pi k / (2 n))) for 0 < k < n,
 *              x_0 = 0 and x_n = x_max exactly.
 * edge_kind 1: p_edges[n_p+1] and q_edges[n_q+1] given (strictly increasing,
 *              first edge >= 0); p_max/q_max are then ignored.
 * n_gauss_q: Gauss-Legendre points per q bin (1..16) for the P0 quadrature.
 * n_gauss_x: Gauss-Legendre points on the clipped cosine interval (1..64).
 * L: total orbital momentum; n_ch channels (l[a], lam[a]) with even l.
 * Limits: 2 <= n_p, n_q <= 1024; 1 <= n_ch <= 8; l, lam <= 4.            */
typedef struct {
    int32_t n_p, n_q;
    double p_max, q_max;
    int32_t edge_kind;
    const double *p_edges, *q_edges;
    int32_t n_gauss_q, n_gauss_x;
    int32_t L, n_ch;
    const int32_t *l, *lam;
} wpcd_basis_desc;

/* Pair potential (eq.(vpot)).
 * kind 0: rank-1 Yamaguchi v = strength[0] g g, g = 1/(p^2 + range[0]^2),
 *         s-wave only (zero in l > 0).
 * kind 1: sum over n_terms of strength[k] exp(-range[k] r)/r, in every pair
 *         wave l.
 * fit_e2: if not NaN (kind 1 only), all strengths are scaled by one common
 *         positive factor chosen so that the lowest l = 0 pair level equals
 *         fit_e2 in this basis.                                          */
typedef struct {
    int32_t kind;
    int32_t n_terms;
    const double *strength, *range;
    double fit_e2;
} wpcd_potential_desc;

/* Initial vector of the iterative solve.  The paper starts from zero (or
 * sums the Neumann series); the warm starts are an addition of this library
 * and never change what the solve converges to: the proposed vector x0 is
 * replaced by alpha x0 with the complex alpha that minimises the initial
 * residual |b - alpha (1 - K) x0| (alpha = 0, i.e. the zero start, when the
 * proposal is useless or not finite), and the usual residual test ends the
 * solve.                                                                 */
#define WPCD_WARM_NONE 0     /* zero initial vector */
#define WPCD_WARM_LEARNED 1  /* reduced-basis vector proposed by the network of wpcd_learn_train */
#define WPCD_WARM_GIVEN 2    /* caller's x0 */

/* Iterative solve options.  max_iter: total Krylov iterations per energy
 * (default 400 when <= 0); krylov_dim: GMRES restart length (default 48,
 * max 128); tol: relative residual target (default 1e-12 for WPCD_FP64,
 * 1e-9 for the mixed tiers, whose FP32 P0 values already perturb the
 * operator at the 1e-7 level).  want_breakup:
 * fill breakup_out in wpcd_solve.  warm_start: a WPCD_WARM_* value; x0
 * (WPCD_WARM_GIVEN only): host array [n_E][M][2] of (re, im) doubles in
 * channel-basis order, M = n_ch*n_q*n_p (a reduced system: its major and
 * minor rows, see wpcd_build_reduced).  err_est: nonzero to fill
 * err_vs_fp64 of every result (see wpcd_energy_result); this needs the P0
 * values in FP64 as well, which the first such call computes on the
 * existing structure and keeps (8 B per channel value).
 * resolvent: WPCD_RESOLVENT_AT_E (default, 0) projects the channel
 * resolvent on every channel state at the energy E; WPCD_RESOLVENT_AVERAGED
 * averages each eigenvalue over E's on-shell energy interval (Sec. II.C),
 * [eps*_1 + 3/4 q_j0^2, eps*_1 + 3/4 q_(j0+1)^2] of width D, the energies of
 * the entrance spectator bin j0 holding q0:
 *   (1/(D dq_j)) int dE int dq / (E - eps*_k - 3/4 q^2 + i0)   (closed form).
 * All energies of one bin then give the same amplitudes (histogram form);
 * the elastic flux factor is 1/D (A = U / D) and every pseudostate bin whose
 * shell eps*_k + 3/4 q^2 meets the interval is an open breakup state with
 * flux factor (its length inside the shell) / (D dq_j).
 * fallback_tol (mixed tiers of wpcd_solve, wpcd_solve_dev and wpcd_sweep;
 * 0 or less: off): after the mixed solve, every energy that did not
 * converge (WPCD_E_NOT_CONVERGED or WPCD_E_STAGNATED), or (with err_est)
 * whose err_vs_fp64 is above fallback_tol or
 * not finite, is solved again on the FP64 P0 values of the same structure
 * (computed and kept as for err_est) with the FP64 solve's default
 * tolerance unless tol is given, and its result replaces the mixed one
 * (result field fallback = 1; err_vs_fp64 then measures the FP64 solve's
 * remaining error).  With err_est this bounds each returned amplitude's
 * estimated error by fallback_tol.                                        */
#define WPCD_RESOLVENT_AT_E 0
#define WPCD_RESOLVENT_AVERAGED 1
/* want_breakup values */
#define WPCD_BREAKUP_ELEMENTS 1   /* rows (channel, k, j, Re S, Im S) per open state (resolvent at E only) */
#define WPCD_BREAKUP_DIST 2       /* rows (channel, k, eps*_k, sum_j |S|^2, bins) per pseudostate */
typedef struct {
    int32_t max_iter;
    int32_t krylov_dim;
    double tol;
    int32_t want_breakup;
    int32_t warm_start;
    const double *x0;
    int32_t err_est;
    int32_t resolvent;
    double fallback_tol;
} wpcd_solve_opts;

/* Per-energy result.  status is a wpcd_status value for this energy.
 * U = on-shell element of the transition matrix, A = (2/(3 q0)) U / dq_j0
 * (A = U / D with the averaged resolvent), S = 1 - 2 pi i A (Sec. III.B,
 * m = 1), delta = arg(S)/2, eta = |S|.
 * n_open: rows written to breakup_out for this energy (open breakup states
 * with WPCD_BREAKUP_ELEMENTS or none asked, pseudostates with open bins with
 * WPCD_BREAKUP_DIST).
 * warm: 1 if a warm start was kept (alpha != 0); r0: relative residual of
 * the initial vector (1 for the zero start).  fallback: 1 if this energy
 * was solved again in FP64 (opts.fallback_tol).
 * err_vs_fp64 (opts.err_est set, else NaN): |U - U64| / |U|, the relative
 * difference of this amplitude from the FP64 path's (FP64 P0 values, FP64
 * solve), estimated as the on-shell component of the correction d of one
 * step of iterative refinement: r64 = b64 - (1 - K64) u with the FP64 P0,
 * (1 - K) d = r64 solved in this tier to 1e-4.  Exact to first order in the
 * FP32 rounding of P0 (and in the solver's residual); the returned U is not
 * corrected.  For WPCD_FP64 it measures the solver's remaining error.      */
typedef struct {
    double E, q0;
    int32_t j0, status, iters, n_open;
    double U_re, U_im, A_re, A_im, S_re, S_im;
    double delta, eta, residual;
    int32_t warm, fallback;
    double r0;
    double err_vs_fp64;
} wpcd_energy_result;

/* Training of the learned warm start (not part of the paper's method).
 * For each of n_var potential variants the strengths of the current
 * potential are multiplied term by term by mult[v][0..n_mult) (n_mult =
 * the potential's n_terms), the pair waves are re-diagonalised (P0 is
 * potential independent and is kept), and the energies E[v][0..n_E) are
 * solved from the zero start in `precision` with `solve` options.  The
 * converged solutions are snapshots: a greedy reduced basis of n_basis
 * orthonormal vectors is built from them, and a multilayer perceptron
 * (three tanh hidden layers of `hidden` units, BF16 weights, FP32
 * accumulation, Adam) is trained to map the features (E, on-shell
 * momentum and its position on the spectator grid, entrance channel,
 * multipliers) to the snapshot coefficients.
 * The multipliers are restored to 1 at the end.  Limits: n_basis 1..128,
 * hidden 16..512, n_mult = n_terms, all multipliers finite and > 0.      */
typedef struct {
    int32_t n_var, n_mult;
    const double *mult;      /* [n_var][n_mult] */
    int32_t n_E;
    const double *E;         /* [n_var][n_E] */
    int32_t precision;       /* wpcd_precision of the training solves */
    int32_t n_basis;         /* reduced-basis size */
    int32_t hidden;          /* hidden width (default 256 when <= 0) */
    int32_t epochs;          /* passes over the samples (default 400) */
    int32_t batch;           /* minibatch size (default 64) */
    double lr;               /* Adam step size (default 2e-3), cosine decay to lr/20 */
    uint64_t seed;           /* weight initialisation and minibatch order */
    const wpcd_solve_opts *solve;   /* may be NULL */
} wpcd_learn_desc;

typedef struct {
    int32_t n_samples;       /* converged solves that entered the training set */
    int32_t plain_iters;     /* Krylov iterations of those solves, summed */
    double basis_max_rel_err;   /* max over samples of |u - Phi Phi^H u| / |u| */
    double basis_mean_rel_err;
    double loss_first, loss_last;   /* training loss of the first / last epoch */
    double solve_ms, basis_ms, train_ms;
} wpcd_learn_report;

/* Per-kernel timing (milliseconds summed over launches since the last
 * reset, measured with HIP events on the stream the kernels run on).    */
typedef struct {
    char name[32];
    double total_ms;
    int64_t launches;
} wpcd_kernel_time;

/* Create a context on HIP device `device`.  hip_stream is a hipStream_t to
 * launch on (NULL: the context creates its own).  The stream is not owned
 * when passed in.  Errors: WPCD_E_INVALID, WPCD_E_DEVICE.               */
wpcd_status wpcd_create(int device, void *hip_stream, wpcd_ctx **out);

/* Step 1 of Sec. III.C: bin edges and Gauss tables (host, FP64, uploaded),
 * pair-potential matrices in the free WP basis (eq.(vpot)) and the FP64
 * diagonalisation of h1 = h0 + v for every pair wave used (eq.(exp_z)),
 * both on the GPU.  O has rows = eigenvectors, eigenvalues ascending, sign
 * chosen so the largest-magnitude component is positive.  Invalidates any
 * P0 built for a different grid.  Errors: WPCD_E_INVALID, WPCD_E_NOMEM,
 * WPCD_E_DEVICE.                                                         */
wpcd_status wpcd_build_basis(wpcd_ctx *ctx, const wpcd_basis_desc *basis,
                             const wpcd_potential_desc *pot);

/* Three nucleons with pair interactions in s-waves only (Sec. III.B,
 * eq.(gal) with the spin and isospin of the nucleons; the paper's
 * realistic case of Sec. V.A couples many more channels).  Channel a has
 * pair spin s[a] and pair isospin t[a], l = lam = 0, with s + t odd (the
 * pair antisymmetric): (1, 0) is 3S1, (0, 1) is 1S0; channel 0 must be
 * (1, 0), whose pair bound state (the deuteron) is the entrance state.
 * two_S = 1 (three-body spin 1/2, channels (1, 0) and optionally (0, 1))
 * or 3 (spin 3/2, channel (1, 0) only); three-body isospin 1/2.  The
 * permutation kernel between channels a and b is the s-wave one times
 *   g_ab = (1/2) (sigma_ab tau_ab + sigma_ba tau_ba),
 *   sigma_ab = (-1)^(s_b) sqrt((2 s_a + 1)(2 s_b + 1)) {1/2 1/2 s_b; 1/2 S s_a},
 * tau_ab the same with t and total isospin 1/2 (the cyclic permutation of
 * the three nucleons between recoupled spin and isospin states; 6j symbols
 * by Racah's sum): g = [[1/4, -3/4], [-3/4, 1/4]] for the doublet, -1/2 for
 * the quartet.  Channel a's pair potential is pot with strength term k
 * times mult[a * pot->n_terms + k] (mult NULL: 1); pot->fit_e2 fits the
 * common scale on channel 0.  basis gives the grid and the quadratures
 * (its n_ch, L, l and lam are not read).  wpcd_pair_spectrum's l then
 * selects the channel.  Errors: WPCD_E_INVALID for the conditions above. */
typedef struct {
    int32_t two_S;
    int32_t n_ch;
    const int32_t *s, *t;
    const double *mult;
} wpcd_nucleon_desc;
wpcd_status wpcd_build_basis_nucleons(wpcd_ctx *ctx, const wpcd_basis_desc *basis,
                                      const wpcd_potential_desc *pot,
                                      const wpcd_nucleon_desc *nuc);

/* Replace only the pair potential (the grid and any built P0 stay valid,
 * since P0 does not depend on the potential -- Sec. III.C).              */
wpcd_status wpcd_set_potential(wpcd_ctx *ctx, const wpcd_potential_desc *pot);

/* Copy out the pair spectrum of wave l: eps_out[n_p] and, if O_out is not
 * NULL, O_out[n_p*n_p] (row-major, rows = eigenvectors).  Also reports the
 * fitted strength scale (1 if no fit) in *scale_out if not NULL.
 * Errors: WPCD_E_STATE (no basis), WPCD_E_INVALID (l not used).          */
wpcd_status wpcd_pair_spectrum(wpcd_ctx *ctx, int32_t l, double *eps_out, double *O_out,
                               double *scale_out);

/* Step 2 of Sec. III.C (Sec. IV.B-C, eqs.(perm),(gal)): pre-select the
 * nonzero cell pairs of P0 and compute them.  Structure: CSR over cells,
 * row_ptr int64[n_p*n_q+1], col int32[nnz] ascending (bit-exact, from IEEE
 * add/compare on FP64 tables).  Values: n_ch*n_ch per cell pair (row
 * channel major), FP64 (WPCD_FP64) or FP32 with compensated sums
 * (WPCD_MIXED).  *nnz_cells_out receives the number of cell pairs.
 * Errors: WPCD_E_STATE, WPCD_E_NOMEM, WPCD_E_DEVICE.                      */
wpcd_status wpcd_build_p(wpcd_ctx *ctx, wpcd_precision prec, int64_t *nnz_cells_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * P0 as wpcd_build_p (same kernels, same bits), written into the caller's
 * device buffers, with no hipMalloc, hipFree or other allocation.
 *   row_ptr  device int64[n_p*n_q + 1]          (written)
 *   col      device int32[cap_nnz]               (first nnz written)
 *   val      device float[cap_nnz*n_ch*n_ch] for WPCD_MIXED or
 *            double[cap_nnz*n_ch*n_ch] for WPCD_FP64 (first nnz blocks written)
 * *nnz_cells_out (may be NULL) receives the number of cell pairs once the
 * pre-selection has counted them, also when cap_nnz is too small.  The
 * context's own P0 (wpcd_build_p's) is neither used nor changed, so this
 * does not enable wpcd_solve.  The intermediates (row counts, per-tile
 * totals, row lookup tables of the element kernels) live in one fixed
 * device array of WPCD_NOALLOC_SCRATCH_BYTES per GPU, taken at wpcd_create
 * and held until the process ends; it needs 512 B + 4 n_p n_q B +
 * 1.07 nnz B (about 21 MB for 300 x 300 bins with 19.2 million cell
 * pairs).  Every call on one GPU, from any context or thread, shares that
 * array: calls that overlap in time on one GPU race and must be
 * serialised by the caller.  Nothing in the array needs to start at zero.
 * Launch shapes are the cached or heuristic choices (no timing launches),
 * and per-kernel timing is off during the call.  Returns when the values
 * are written (the context's stream is synchronised).
 * Errors: WPCD_E_STATE (no basis), WPCD_E_INVALID (NULL pointer, bad
 * precision, nnz > cap_nnz, or the grid or nnz beyond the fixed scratch),
 * WPCD_E_DEVICE.                                                        */
#define WPCD_NOALLOC_SCRATCH_BYTES (32ll << 20)
wpcd_status wpcd_build_p_noalloc(wpcd_ctx *ctx, wpcd_precision prec, int64_t *row_ptr,
                                 int32_t *col, void *val, int64_t cap_nnz,
                                 int64_t *nnz_cells_out);

/* Copy P0 to caller buffers: row_ptr[n_p*n_q+1], col[nnz], val[nnz*n_ch*n_ch]
 * (FP64; FP32 values are widened).  Any pointer may be NULL to skip it.
 * Errors: WPCD_E_STATE (no P0).                                          */
wpcd_status wpcd_get_p(wpcd_ctx *ctx, int64_t *row_ptr, int32_t *col, double *val);

/* Feshbach major/minor channel reduction (Sec. V.B): turn `red` into a
 * reduced system of `full`.  Channels [0, n_major) of full are the major
 * ones and keep full's lattice; the others are minor and are described on
 * the coarse lattice of every r_p-th p edge and every r_q-th q edge (bins
 * that are unions of r_p x r_q fine cells).  The reading: with unit-weight
 * packets the packet of a union of bins is sum_i sqrt(d_i / D) |x_i>, so
 * every P0 element involving a coarse cell is that combination of full's
 * fine elements (exact for the element as an integral over the cells); the
 * minor channels' pair Hamiltonians are diagonalised on the coarse p bins
 * with full's potential and their channel resolvent uses the coarse
 * spectator bins.  wpcd_solve on `red` then solves the coupled reduced
 * system, whose major components are the solution of the effective-kernel
 * equation of the major subspace,
 *   (1 - K_MM - K_Mm (1 - K_mm)^-1 K_mM) u_M = b_M + K_Mm (1 - K_mm)^-1 b_m.
 * red: a context from wpcd_create on full's device (any basis or P0 it held
 * is dropped).  full: basis, potential and P0 built (boson channels); if
 * its P0 is a WPCD_MIXED build, its FP64 values are computed once on the
 * same structure and kept in full.  The entrance channel (l = 0, lam = L)
 * must be major.  prec: WPCD_FP64 (solve red with WPCD_FP64) or WPCD_MIXED
 * (FP32 copies of the reduced values for the mixed tiers; the FP64 ones
 * are kept as well).  *nnz_out (may be NULL) receives the number of stored
 * entries.  Layout of red's channel basis (x0, breakup rows): the major
 * channels as in full, (a n_q + j) n_p + k, then from row n_major n_q n_p
 * on the minor channels over (a', coarse j, pair state k of the coarse
 * pair basis); breakup rows carry channel numbers over full's channel
 * list, with j and k on the coarse lattice for minor channels; breakup_out
 * needs n_p*n_ch*5 doubles per energy with full's n_p and n_ch.
 * wpcd_get_p on red copies the reduced P0: row_ptr[R + 1] over the R
 * reduced cells (n_major n_p n_q fine ones, then (n_ch - n_major)
 * (n_p/r_p)(n_q/r_q) coarse ones, channel major), columns ascending,
 * one value per entry.  wpcd_pair_spectrum reports red's major waves.
 * Not available on red: wpcd_build_p (and _noalloc), wpcd_save_p,
 * wpcd_load_p, wpcd_set_potential, wpcd_set_multipliers, wpcd_bound_state,
 * wpcd_learn_train (WPCD_E_STATE); wpcd_build_basis makes red an ordinary
 * context again.  full may be changed or destroyed afterwards.  The build
 * keeps each coarse cell's column sets in one workgroup's LDS: lattices up
 * to about 250,000 fine cells.  Errors: WPCD_E_INVALID (the conditions
 * above), WPCD_E_STATE, WPCD_E_NOMEM, WPCD_E_DEVICE.                      */
wpcd_status wpcd_build_reduced(wpcd_ctx *red, wpcd_ctx *full, int32_t n_major, int32_t r_p,
                               int32_t r_q, wpcd_precision prec, int64_t *nnz_out);

/* Steps 3-4 of Sec. III.C for n_E energies at once: channel resolvent G1
 * (FP64, diagonal in the channel WP basis), the factored kernel
 * K = O P0 V~ G1 (eq.(kernel)) applied on the GPU, and a batched restarted
 * GMRES solve of (1 - K) u = O P0 V~ e0 for the on-shell column of
 * eq.(m_pvg).  out[n_E] receives the amplitudes.  breakup_out, if not NULL
 * and opts->want_breakup is set, receives per energy (at offset
 * e*n_p*n_ch*5 doubles) up to n_p*n_ch rows of 5 doubles, row count in
 * n_open: WPCD_BREAKUP_ELEMENTS, (channel, k, j_k, Re S_k0, Im S_k0) with
 * S_k0 = -2 pi i sqrt(rho_k rho_0) u_k (Sec. III.B, breakup as transitions to
 * the pair's discretised continuum); WPCD_BREAKUP_DIST, the breakup
 * distribution over the pair energy, (channel, k, eps*_k, sum over the
 * pseudostate's open bins of |S|^2, number of those bins).
 * Per-energy failures are reported in out[e].status and do not abort the
 * batch.  prec selects the P0 values used (FP64 requires an FP64 build,
 * WPCD_MIXED, WPCD_MIXED_REFINE and WPCD_MIXED_BF16 a mixed one).
 * Errors: WPCD_E_STATE, WPCD_E_INVALID, WPCD_E_NOMEM, WPCD_E_DEVICE.      */
wpcd_status wpcd_solve(wpcd_ctx *ctx, const double *E, int32_t n_E, wpcd_precision prec,
                       const wpcd_solve_opts *opts, wpcd_energy_result *out,
                       double *breakup_out);

/* wpcd_solve with the energies E_dev[n_E] in device memory and the
 * results written to device memory out_dev[n_E] (no breakup rows), on the
 * context's stream.  The energy bookkeeping (threshold, on-shell bin) runs
 * on the host, so the call copies the energies in and synchronises.
 * Errors: as wpcd_solve.                                                  */
wpcd_status wpcd_solve_dev(wpcd_ctx *ctx, const double *E_dev, int32_t n_E, wpcd_precision prec,
                           const wpcd_solve_opts *opts, wpcd_energy_result *out_dev);

/* Energy sweep in batches with a journal of the completed ones, so that an
 * interrupted sweep resumes from the last completed batch.  P0 does not
 * depend on the energy (Sec. III.B), so one built (or loaded) P0 serves
 * the whole sweep.  The energies E[n_E] are solved in batches of `batch`
 * (the last one shorter; a batch is one wpcd_solve call), in order.
 * journal: path of the journal file, or NULL for none.  A missing or empty
 * file is created with a header (the sweep's energies, batch, precision and
 * a fingerprint of what fixes the results: basis, bin edges, reduction, P0
 * precision and size, potential and multipliers (also those of each pair
 * wave of a nucleon basis), solve options, the learned
 * model's shape and scalings when it proposes the start); a journal of the
 * same sweep is replayed: its complete batch records (each checked by a
 * hash) fill out[] and are not solved again, and a torn or damaged tail is
 * cut off.  Each batch solved here is appended and flushed to disk before
 * the next one starts.  max_batches > 0 solves at most that many batches
 * in this call (0: all).  out[n_E]: the results of every energy done (the
 * first *n_done_out); energies not reached have status WPCD_E_STATE.
 * *n_resumed_out (may be NULL): energies taken from the journal.  No
 * breakup rows; opts->want_breakup is ignored; warm_start must not be
 * WPCD_WARM_GIVEN.  Results equal those of wpcd_solve over the same batches.
 * A journal is used by one call at a time.
 * Errors: WPCD_E_INVALID (NULL arrays, batch < 1, WPCD_WARM_GIVEN, a
 * journal of another sweep or not a journal, the file cannot be created,
 * trimmed or written), and those of wpcd_solve.                           */
wpcd_status wpcd_sweep(wpcd_ctx *ctx, const double *E, int32_t n_E, int32_t batch,
                       wpcd_precision prec, const wpcd_solve_opts *opts, const char *journal,
                       int32_t max_batches, wpcd_energy_result *out, int32_t *n_done_out,
                       int32_t *n_resumed_out);

/* Save the built P0 (structure, values in the precision it was built in)
 * with the grid signature (sizes, Gauss orders, channels, bin edges) to a
 * binary file; load it into a context whose basis has the same signature
 * (P0 is potential independent, so it can be reused across potentials and
 * runs); *nnz_cells_out (may be NULL) receives the number of cell pairs.
 * Errors: WPCD_E_STATE (no P0 / no basis), WPCD_E_INVALID (file cannot be
 * opened, written or read, other signature, inconsistent data).          */
wpcd_status wpcd_save_p(wpcd_ctx *ctx, const char *path);
wpcd_status wpcd_load_p(wpcd_ctx *ctx, const char *path, int64_t *nnz_cells_out);

/* The paper's model matrix fills (Sec. IV.A), a micro-benchmark of filling
 * a matrix of costly elements on the GPU, dense and sparse:
 *   kind 0, eq.(Atrig): A(i,j) = sum_{k=1..K} (sin^k u_ij + cos^k w_ij);
 *   kind 1, eq.(Agau):  A(i,j) = sum_{k=1..K} int_{u_ij}^{w_ij} (sin^k t + cos^k t) dt,
 *                       by the 48-point Gauss-Legendre rule;
 * u_ij, w_ij = outputs 2(i M + j) and 2(i M + j) + 1 of the splitmix64
 * stream of `seed` (counter form mix(seed + (n+1) 0x9E3779B97F4A7C15),
 * u = (x >> 11) 2^-53).  mode 0: every element, one thread each (the
 * paper's M^2 threads), into dense_out[M*M] (row major, may be NULL);
 * mode 1, eq.(Acond) by filtering in the same launch: elements with
 * u_ij > alpha are zero and not evaluated; mode 2, eq.(Acond) with the kept
 * elements selected first (ballot compaction, ascending flat index
 * i M + j) and then evaluated with every lane busy: idx_out[cap] and
 * val_out[cap] (may be NULL), *nnz_out = the number kept (also when it
 * exceeds cap, which returns WPCD_E_INVALID).  prec WPCD_FP64 or WPCD_MIXED
 * (FP32 arithmetic); values are returned as doubles.  *ms_out: GPU time of
 * the fill's kernels (HIP events on the context's stream).  Limits:
 * M <= 8192, K <= 4096.  Errors: WPCD_E_INVALID, WPCD_E_NOMEM,
 * WPCD_E_DEVICE.                                                         */
wpcd_status wpcd_model_fill(wpcd_ctx *ctx, int32_t kind, int32_t mode, int32_t M, int32_t K,
                            double alpha, uint64_t seed, wpcd_precision prec, double *dense_out,
                            int64_t *idx_out, double *val_out, int64_t cap, int64_t *nnz_out,
                            double *ms_out);

/* Three-body bound state of the homogeneous equation u = K(E) u (eq.(m_pvg)
 * without the driving term): the energy in [e_lo, e_hi] (below the lowest
 * pair level, where K is real) at which the largest real eigenvalue of K(E)
 * equals 1.  The eigenvalue is the largest real Ritz value of 64 Arnoldi
 * steps of K(E) on the GPU (eigenvalues of the small Hessenberg matrix on
 * the host); E by bisection to 1e-12 relative.  Errors: WPCD_E_STATE,
 * WPCD_E_INVALID (no sign change on the bracket), WPCD_E_BELOW_THRESHOLD
 * (bracket not below the pair level).                                    */
wpcd_status wpcd_bound_state(wpcd_ctx *ctx, double e_lo, double e_hi, double *e3_out);

/* wpcd_solve for n_sys independent systems at once (uneven sizes and
 * channel sets allowed): system i is solved in context ctxs[i] at energies
 * E[i][0..n_E[i]) into out[i][0..n_E[i]) (no breakup rows).  Contexts on one
 * device are solved in lockstep by one host thread: the systems' batches of
 * energies start their GMRES cycles together, and every group of iterations
 * of all of them is replayed as one captured HIP graph (each system's
 * launches a branch on its own context's stream), with one convergence
 * read-back per group; a system whose energies have converged leaves the
 * cycle (a graph of the remaining ones is captured on first use).  Contexts
 * on several devices are driven by one host thread each.  The contexts must
 * be distinct (a context is not thread-safe) and share the Krylov
 * dimension (one opts).  status_out[i] (may be
 * NULL) receives each system's call status; the return value is the first
 * non-OK one.  opts is shared by all systems, so opts->warm_start may not
 * be WPCD_WARM_GIVEN (one x0 cannot match systems of different sizes).
 * Errors: WPCD_E_INVALID (NULL arrays, repeated context, WPCD_WARM_GIVEN). */
wpcd_status wpcd_solve_multi(wpcd_ctx *const *ctxs, int32_t n_sys, const double *const *E,
                             const int32_t *n_E, wpcd_precision prec, const wpcd_solve_opts *opts,
                             wpcd_energy_result *const *out, wpcd_status *status_out);

/* Multiply the strengths of the current potential term by term by
 * mult[0..n_mult) (n_mult = n_terms; the multipliers are relative to the
 * potential given last) and re-diagonalise the pair waves; P0 stays valid.
 * These multipliers are features of the learned warm start.
 * Errors: WPCD_E_STATE, WPCD_E_INVALID.                                   */
wpcd_status wpcd_set_multipliers(wpcd_ctx *ctx, const double *mult, int32_t n_mult);

/* Build the learned warm start (see wpcd_learn_desc); report may be NULL.
 * Errors: WPCD_E_STATE (no P0), WPCD_E_INVALID, WPCD_E_NOMEM (snapshots
 * take n_var*n_E*M*8 bytes of device memory), WPCD_E_DEVICE.             */
wpcd_status wpcd_learn_train(wpcd_ctx *ctx, const wpcd_learn_desc *desc,
                             wpcd_learn_report *report);

/* One forward and backward pass of the warm-start network's kernels on
 * caller data, for checking them.  params: FP32 [W1 b1 W2 b2 W3 b3 W4 b4],
 * W_l row-major (out x in), layer widths n_in -> n_hidden (x3) -> n_out;
 * the weights are rounded to BF16 as in training (biases stay FP32).
 * X[batch][n_in], T[batch][n_out].  Outputs (any may be NULL): Y[batch]
 * [n_out], grad (same layout as params) of loss = sum (Y - T)^2 / batch,
 * *loss_out.  Does not touch a trained model.  Errors: WPCD_E_INVALID.   */
wpcd_status wpcd_mlp_eval(wpcd_ctx *ctx, int32_t n_in, int32_t n_hidden, int32_t n_out,
                          const float *params, int32_t batch, const float *X, const float *T,
                          float *Y_out, float *grad_out, double *loss_out);

/* Launch shapes (tile sizes of the block products, rows per workgroup of
 * the Krylov vector kernels) are chosen per problem shape:
 * WPCD_TUNE_HEURISTIC (default): fixed rules from the number of workgroups;
 * WPCD_TUNE_MEASURE: the first solve of each shape times every candidate on
 * the live buffers (a few launches) and keeps the fastest for the life of
 * the context; WPCD_TUNE_FORCE + i: candidate i everywhere (clamped), for
 * tests.  Changing the mode clears the decisions.  wpcd_get_autotune lists
 * them (up to n entries, count in *n_out).  Results agree between choices
 * to rounding (the block products bit for bit).                          */
#define WPCD_TUNE_HEURISTIC 0
#define WPCD_TUNE_MEASURE 1
#define WPCD_TUNE_FORCE 16
typedef struct {
    char name[32];
    char key[64];
    int32_t choice, n_candidates;
    double us;   /* measured time of the choice, 0 when not measured */
} wpcd_tune_entry;
wpcd_status wpcd_set_autotune(wpcd_ctx *ctx, int32_t mode);
wpcd_status wpcd_get_autotune(wpcd_ctx *ctx, wpcd_tune_entry *out, int32_t n, int32_t *n_out);

/* Replay of captured HIP graphs for the solve's iterations (default on):
 * each group of four GMRES iterations of a batch shape is captured once
 * and then launched as one graph; results are identical to the eager
 * launches, which are used instead while solve-kernel timing is on or
 * after wpcd_set_graphs(ctx, 0).  Clears the captured graphs.            */
wpcd_status wpcd_set_graphs(wpcd_ctx *ctx, int32_t enable);

/* Kernel timing with HIP events recorded on the context's stream around
 * each launch.  enable is a bit mask of kernel groups: WPCD_TIME_PAIR (pair
 * potential and diagonalisation), WPCD_TIME_P0 (P0 element kernels),
 * WPCD_TIME_SOLVE (resolvent, kernel products, GMRES), WPCD_TIME_PRESELECT
 * (pre-selection count, scan and fill); 0 turns timing off.
 * wpcd_get_timing copies the accumulated table (up to n entries, count in
 * *n_out); wpcd_reset_timing clears it.                                  */
#define WPCD_TIME_PAIR 1
#define WPCD_TIME_P0 2
#define WPCD_TIME_SOLVE 4
#define WPCD_TIME_PRESELECT 8
wpcd_status wpcd_set_timing(wpcd_ctx *ctx, int32_t enable);
wpcd_status wpcd_get_timing(wpcd_ctx *ctx, wpcd_kernel_time *out, int32_t n, int32_t *n_out);
wpcd_status wpcd_reset_timing(wpcd_ctx *ctx);

/* Wait for all work the context queued.                                  */
wpcd_status wpcd_synchronize(wpcd_ctx *ctx);

/* Message for the last error on this context (never NULL).              */
const char *wpcd_last_error(const wpcd_ctx *ctx);

/* Release the context and all its device memory.  NULL is ignored.       */
void wpcd_destroy(wpcd_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* WPCD_H */
