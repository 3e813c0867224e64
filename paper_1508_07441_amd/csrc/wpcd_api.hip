// C ABI of libwpcd: context, host tables, orchestration of the GPU steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cerrno>
#include <chrono>
#include <complex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include <unistd.h>

#include "wpcd_internal.h"

namespace wpcd {

// ------------------------------------------------------------ timing
int Timer::id_of(const char *name) {
    for (size_t i = 0; i < names.size(); ++i)
        if (names[i] == name) return (int)i;
    names.emplace_back(name);
    total_ms.push_back(0.0);
    launches.push_back(0);
    return (int)names.size() - 1;
}

hipEvent_t Timer::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    WPCD_HIP(hipEventCreate(&e));
    return e;
}

void Timer::begin(hipStream_t s, const char *name, Pending &p) {
    p.id = id_of(name);
    p.a = get();
    p.b = get();
    WPCD_HIP(hipEventRecord(p.a, s));
}

void Timer::end(hipStream_t s, Pending &p) {
    (void)hipEventRecord(p.b, s);
    pending.push_back(p);
}

void Timer::collect() {
    for (auto &p : pending) {
        float ms = 0.f;
        WPCD_HIP(hipEventSynchronize(p.b));
        WPCD_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        total_ms[p.id] += ms;
        launches[p.id] += 1;
        pool.push_back(p.a);
        pool.push_back(p.b);
    }
    pending.clear();
}

void Timer::reset() {
    collect();
    for (auto &t : total_ms) t = 0.0;
    for (auto &l : launches) l = 0;
}

void Timer::release() {
    for (auto &p : pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    pending.clear();
    for (auto e : pool) (void)hipEventDestroy(e);
    pool.clear();
}

// ------------------------------------------------------- Gauss tables
// Golub-Welsch: the nodes are the eigenvalues of the symmetric tridiagonal
// Jacobi matrix of the Legendre recurrence (zero diagonal, off-diagonal
// k / sqrt(4k^2 - 1)); weight = 2 (first eigenvector component)^2.  The
// eigenproblem is solved by cyclic Jacobi rotations on the dense n x n
// matrix; nodes are then polished by Newton steps in long double and the
// weights recomputed from P_n'.
static void gauss_legendre_compute(int n, std::vector<double> &x, std::vector<double> &w) {
    std::vector<long double> J((size_t)n * n, 0.0L), V((size_t)n * n, 0.0L);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0L;
    for (int k = 1; k < n; ++k) {
        long double b = k / std::sqrt(4.0L * k * k - 1.0L);
        J[(size_t)(k - 1) * n + k] = b;
        J[(size_t)k * n + k - 1] = b;
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        long double off = 0.0L;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += J[(size_t)p * n + q] * J[(size_t)p * n + q];
        if (off < 1e-40L) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                long double apq = J[(size_t)p * n + q];
                if (std::fabs(apq) < 1e-300L) continue;
                long double th = (J[(size_t)q * n + q] - J[(size_t)p * n + p]) / (2.0L * apq);
                long double t = (th >= 0 ? 1.0L : -1.0L) / (std::fabs(th) + std::sqrt(1.0L + th * th));
                long double c = 1.0L / std::sqrt(1.0L + t * t), s = t * c;
                for (int r = 0; r < n; ++r) {
                    long double a = J[(size_t)r * n + p], bq = J[(size_t)r * n + q];
                    J[(size_t)r * n + p] = c * a - s * bq;
                    J[(size_t)r * n + q] = s * a + c * bq;
                }
                for (int r = 0; r < n; ++r) {
                    long double a = J[(size_t)p * n + r], bq = J[(size_t)q * n + r];
                    J[(size_t)p * n + r] = c * a - s * bq;
                    J[(size_t)q * n + r] = s * a + c * bq;
                }
                for (int r = 0; r < n; ++r) {
                    long double a = V[(size_t)r * n + p], bq = V[(size_t)r * n + q];
                    V[(size_t)r * n + p] = c * a - s * bq;
                    V[(size_t)r * n + q] = s * a + c * bq;
                }
            }
    }
    std::vector<std::pair<long double, long double>> nw(n);
    for (int k = 0; k < n; ++k) nw[k] = {J[(size_t)k * n + k], 2.0L * V[k] * V[k]};
    std::sort(nw.begin(), nw.end());
    x.resize(n);
    w.resize(n);
    for (int k = 0; k < n; ++k) {
        long double z = nw[k].first, dp = 0.0L;
        for (int it = 0; it < 3; ++it) {
            long double p0 = 1.0L, p1 = z;
            for (int mm = 2; mm <= n; ++mm) {
                long double p2 = ((2 * mm - 1) * z * p1 - (mm - 1) * p0) / mm;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) {
                p1 = z;
                p0 = 1.0L;
            }
            dp = n * (p0 - z * p1) / (1.0L - z * z);
            z -= p1 / dp;
        }
        long double p0 = 1.0L, p1 = z;
        for (int mm = 2; mm <= n; ++mm) {
            long double p2 = ((2 * mm - 1) * z * p1 - (mm - 1) * p0) / mm;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) {
            p1 = z;
            p0 = 1.0L;
        }
        dp = n * (p0 - z * p1) / (1.0L - z * z);
        x[k] = (double)z;
        w[k] = (double)(2.0L / ((1.0L - z * z) * dp * dp));
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

// The rule of each order is computed once per process and shared.
void gauss_legendre_gw(int n, std::vector<double> &x, std::vector<double> &w) {
    static std::mutex mu;
    static std::map<int, std::pair<std::vector<double>, std::vector<double>>> rules;
    std::lock_guard<std::mutex> lock(mu);
    auto it = rules.find(n);
    if (it == rules.end()) {
        std::vector<double> xs, ws;
        gauss_legendre_compute(n, xs, ws);
        it = rules.emplace(n, std::make_pair(std::move(xs), std::move(ws))).first;
    }
    x = it->second.first;
    w = it->second.second;
}

template <class T>
static void upload(DBuf<T> &d, const std::vector<T> &h, hipStream_t s) {
    d.reserve(h.size());
    WPCD_HIP(hipMemcpyAsync(d.ptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Edges x_k = x_max (1 - cos(pi k / (2n))), ends exactly 0 and x_max.
static std::vector<double> cheb_edges(int n, double vmax) {
    std::vector<double> e(n + 1);
    for (int k = 1; k < n; ++k) e[k] = vmax * (1.0 - std::cos((M_PI * (double)k) / (2.0 * (double)n)));
    e[0] = 0.0;
    e[n] = vmax;
    return e;
}

static void upload_tables(wpcd_ctx *c) {
    const int np = c->np, nq = c->nq;
    hipStream_t s = c->stream;
    std::vector<double> P2(np + 1), Q34(nq + 1), H(nq + 1), rp(np), rq(nq);
    for (int k = 0; k <= np; ++k) P2[k] = c->p[k] * c->p[k];
    for (int k = 0; k <= nq; ++k) {
        Q34[k] = 0.75 * (c->q[k] * c->q[k]);
        H[k] = 0.5 * c->q[k];
    }
    for (int k = 0; k < np; ++k) rp[k] = 1.0 / std::sqrt(c->p[k + 1] - c->p[k]);
    for (int k = 0; k < nq; ++k) rq[k] = 1.0 / std::sqrt(c->q[k + 1] - c->q[k]);
    std::vector<double> qn((size_t)nq * c->ngq), qw((size_t)nq * c->ngq);
    for (int j = 0; j < nq; ++j) {
        const double m = 0.5 * (c->q[j] + c->q[j + 1]), h = 0.5 * (c->q[j + 1] - c->q[j]);
        for (int a = 0; a < c->ngq; ++a) {
            qn[(size_t)j * c->ngq + a] = m + h * c->gq[a];
            qw[(size_t)j * c->ngq + a] = h * c->wq[a];
        }
    }
    std::vector<double> ux(c->ngx), wx(c->ngx);
    std::vector<float> uxf(c->ngx), wxf(c->ngx);
    for (int k = 0; k < c->ngx; ++k) {
        ux[k] = 1.0 + c->gx[k];
        wx[k] = c->wx[k];
        uxf[k] = (float)ux[k];
        wxf[k] = (float)wx[k];
    }
    upload(c->d_p, c->p, s);
    upload(c->d_q, c->q, s);
    upload(c->d_P2, P2, s);
    upload(c->d_Q34, Q34, s);
    upload(c->d_H, H, s);
    upload(c->d_rsd_p, rp, s);
    upload(c->d_rsd_q, rq, s);
    upload(c->d_qnode, qn, s);
    upload(c->d_qwt, qw, s);
    upload(c->d_ux, ux, s);
    upload(c->d_wx, wx, s);
    upload(c->d_uxf, uxf, s);
    upload(c->d_wxf, wxf, s);
    WPCD_HIP(hipStreamSynchronize(s));
}

static void set_potential_desc(wpcd_ctx *c, const wpcd_potential_desc *pot) {
    WPCD_REQUIRE(pot, WPCD_E_INVALID, "potential descriptor is NULL");
    WPCD_REQUIRE(pot->kind == 0 || pot->kind == 1, WPCD_E_INVALID, "potential kind must be 0 or 1");
    WPCD_REQUIRE(pot->n_terms >= 1 && pot->n_terms <= 16, WPCD_E_INVALID, "n_terms must be 1..16");
    WPCD_REQUIRE(pot->strength && pot->range, WPCD_E_INVALID, "strength/range NULL");
    if (pot->kind == 0) WPCD_REQUIRE(pot->n_terms == 1, WPCD_E_INVALID, "Yamaguchi takes one term");
    for (int t = 0; t < pot->n_terms; ++t) {
        WPCD_REQUIRE(std::isfinite(pot->strength[t]) && std::isfinite(pot->range[t]) &&
                         pot->range[t] > 0.0,
                     WPCD_E_INVALID, "potential parameters must be finite with range > 0");
    }
    c->pot_kind = pot->kind;
    c->pot_s.assign(pot->strength, pot->strength + pot->n_terms);
    c->pot_base = c->pot_s;
    c->pot_mult.assign(pot->n_terms, 1.0);
    c->pot_mu.assign(pot->range, pot->range + pot->n_terms);
    c->pot_scale = 1.0;
}

static void diagonalise_all(wpcd_ctx *c) {
    const int n = c->np;
    for (int w = 0; w < c->n_waves; ++w) {
        PairWave &pw = c->waves[w];
        pw.v.reserve((size_t)n * n);
        pw.O.reserve((size_t)n * n);
        pw.Vt.reserve((size_t)n * n);
        pw.eps.reserve(n);
        launch_potential(c, w, pw.v.ptr);
        pair_diagonalise(c, w, true);
        launch_vt(c, w);
    }
    WPCD_HIP(hipStreamSynchronize(c->stream));
}

// Common positive scale of all strengths so that the lowest l = 0 level is
// `target`: safeguarded Newton on sigma with the Hellmann-Feynman slope
// d eps0 / d sigma = z0^T v_unit z0 (host arithmetic on copied vectors).
static void fit_scale(wpcd_ctx *c, double target) {
    int w0 = -1;   // the first l = 0 wave (for nucleons the deuteron channel's)
    for (int w = c->n_waves - 1; w >= 0; --w)
        if (c->waves[w].l == 0) w0 = w;
    WPCD_REQUIRE(w0 >= 0, WPCD_E_INVALID, "strength fit needs an l = 0 channel");
    const int n = c->np;
    PairWave &pw = c->waves[w0];
    pw.v.reserve((size_t)n * n);
    pw.O.reserve((size_t)n * n);
    pw.Vt.reserve((size_t)n * n);
    pw.eps.reserve(n);
    std::vector<double> vu((size_t)n * n), z(n);
    c->pot_scale = 1.0;
    launch_potential(c, w0, pw.v.ptr);
    WPCD_HIP(hipMemcpyAsync(vu.data(), pw.v.ptr, vu.size() * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
    WPCD_HIP(hipStreamSynchronize(c->stream));
    auto eval = [&](double sig, double &e0, double &slope) {
        c->pot_scale = sig;
        launch_potential(c, w0, pw.v.ptr);
        pair_diagonalise(c, w0, true);
        WPCD_HIP(hipMemcpyAsync(z.data(), pw.O.ptr, n * sizeof(double), hipMemcpyDeviceToHost,
                                c->stream));
        WPCD_HIP(hipStreamSynchronize(c->stream));
        e0 = pw.h_eps[0];
        double s = 0.0;
        for (int i = 0; i < n; ++i) {
            double r = 0.0;
            for (int k = 0; k < n; ++k) r += vu[(size_t)i * n + k] * z[k];
            s += z[i] * r;
        }
        slope = s;
    };
    double lo = 0.0, hi = 1.0, e0 = 0.0, sl = 0.0;
    // bracket: eps0(lo) > target >= eps0(hi)
    for (int it = 0; it < 60; ++it) {
        eval(hi, e0, sl);
        if (e0 <= target) break;
        lo = hi;
        hi *= 2.0;
        WPCD_REQUIRE(it < 59, WPCD_E_INVALID, "strength fit: no bound state reachable");
    }
    double sig = hi;
    for (int it = 0; it < 100; ++it) {
        eval(sig, e0, sl);
        double f = e0 - target;
        if (f > 0) lo = sig;
        else hi = sig;
        if (std::fabs(f) <= 1e-14 * std::fabs(target) || hi - lo <= 1e-15 * hi) break;
        double nx = (sl != 0.0) ? sig - f / sl : 0.5 * (lo + hi);
        if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
        sig = nx;
    }
    c->pot_scale = sig;
}

static void set_multipliers(wpcd_ctx *c, const double *mult, int n) {
    WPCD_REQUIRE(mult, WPCD_E_INVALID, "multipliers NULL");
    WPCD_REQUIRE(n == (int)c->pot_base.size(), WPCD_E_INVALID,
                 "one multiplier per potential term is required");
    for (int k = 0; k < n; ++k)
        WPCD_REQUIRE(std::isfinite(mult[k]) && mult[k] > 0.0, WPCD_E_INVALID,
                     "multipliers must be finite and > 0");
    for (int k = 0; k < n; ++k) {
        c->pot_mult[k] = mult[k];
        c->pot_s[k] = c->pot_base[k] * mult[k];
    }
    c->has_pot = false;
    diagonalise_all(c);
    c->has_pot = true;
}

static void build_pair_waves(wpcd_ctx *c, const wpcd_potential_desc *pot) {
    set_potential_desc(c, pot);
    if (!std::isnan(pot->fit_e2)) {
        WPCD_REQUIRE(pot->kind == 1, WPCD_E_INVALID, "fit_e2 applies to the Yukawa sum only");
        fit_scale(c, pot->fit_e2);
    }
    diagonalise_all(c);
    c->has_pot = true;
}

// Features of one energy for the warm-start network: E, on-shell momentum,
// its position on the spectator grid (bin index plus fraction, and the
// fraction alone: the driving term changes with the bin), the entrance
// channel and the potential multipliers.
static int learn_features(const wpcd_ctx *c, double E, double q0, int j0, int a0, double *f) {
    const double frac = (q0 - c->q[j0]) / (c->q[j0 + 1] - c->q[j0]);
    f[0] = E;
    f[1] = q0;
    f[2] = j0 + frac;
    f[3] = frac;
    f[4] = a0;
    const int nm = (int)c->pot_mult.size();
    for (int k = 0; k < nm; ++k) f[5 + k] = c->pot_mult[k];
    return 5 + nm;
}

// Converged solutions collected for training.
struct Collect {
    float *snaps = nullptr;
    int64_t n = 0, cap = 0;
    std::vector<double> feat;   // [n][nfeat]
    int nfeat = 0;
    int64_t iters = 0;
};

// Initial vectors for one GMRES batch.
struct WarmCtx {
    int kind = WPCD_WARM_NONE;
    std::vector<float> feat;               // learned: normalised features [nb][nfeat]
    std::vector<const double *> given;     // given: caller vector per energy
};

// Rows of the channel basis: for a reduced system its major part (this
// context's lattice) and then its minor part (the coarse lattice).
static int64_t basis_rows(const wpcd_ctx *c) {
    int64_t M = (int64_t)c->nch * c->nq * c->np;
    if (c->reduced && c->minor) M += (int64_t)c->minor->nch * c->minor->nq * c->minor->np;
    return M;
}

static int total_channels(const wpcd_ctx *c) {
    return c->nch + (c->reduced && c->minor ? c->minor->nch : 0);
}

static void warm_fill(wpcd_ctx *c, void *user, double *x, int nE) {
    WarmCtx &w = *(WarmCtx *)user;
    const int64_t M = basis_rows(c);
    if (w.kind == WPCD_WARM_LEARNED) {
        Learned &L = c->learned;
        L.feat.reserve(w.feat.size());
        WPCD_HIP(hipMemcpyAsync(L.feat.ptr, w.feat.data(), w.feat.size() * sizeof(float),
                                hipMemcpyHostToDevice, c->stream));
        const float *y = mlp_forward(L.mlp, c->stream, c->timer, L.feat.ptr, nE);
        learn_lift(c, y, nE, x);
    } else {
        // stage the caller's vectors in the residual buffer (free until the
        // judge overwrites it), then interleave them into the batch layout
        double *stage = c->d_W.ptr;
        for (int e = 0; e < nE; ++e)
            WPCD_HIP(hipMemcpyAsync(stage + (int64_t)e * M * 2, w.given[e], M * 2 * sizeof(double),
                                    hipMemcpyHostToDevice, c->stream));
        learn_interleave(c, stage, nE, M, x);
    }
}

// Steps 3-4 for a list of energies; collect, if given, receives the
// converged solutions and their features.
// One wpcd_solve call's work on one context, in steps, so that several
// systems' batches can iterate in lockstep (wpcd_solve_multi): plan (checks,
// energies, on-shell bins), then per batch of up to kBatch energies
// begin_batch (GMRES set-up), gmres_cycles over the batches, end_batch
// (error estimate, amplitudes), and finish (results out).
struct SolveJob {
    static constexpr int kBatch = 32;
    wpcd_ctx *c = nullptr;
    const double *E = nullptr;
    int n_E = 0;
    wpcd_precision prec = WPCD_FP64;
    const wpcd_solve_opts *opts = nullptr;
    wpcd_energy_result *out = nullptr;
    double *breakup_out = nullptr;
    Collect *collect = nullptr;
    bool values64 = false;   // FP64 tier on the FP64 values kept beside a mixed build
    // plan
    int m = 48, max_iter = 400;
    double tol = 0.0;
    int want_breakup = 0, warm_kind = WPCD_WARM_NONE;
    bool err_est = false, averaged = false;
    int64_t M = 0;
    int64_t bstride = 0;   // doubles per energy in breakup_out
    int a0 = -1;
    double eb = 0.0, qmax = 0.0;
    std::vector<wpcd_energy_result> res;
    std::vector<int> active;
    std::vector<int64_t> idx0v;
    std::vector<double> rho0v, ebinv;
    // current batch
    size_t b0 = 0;
    int nb = 0;
    std::vector<double> Eb, rho0, ebin;
    std::vector<int64_t> idx0;
    WarmCtx wc;
    GmresOut go;
    std::unique_ptr<GmresRun, void (*)(GmresRun *)> run{nullptr, gmres_run_delete};

    size_t n_batches() const { return (active.size() + kBatch - 1) / kBatch; }

    void plan() {
        WPCD_REQUIRE(c->has_basis && c->has_pot && c->has_p, WPCD_E_STATE,
                     "build_basis and build_p must come first");
        WPCD_REQUIRE(E && out && n_E >= 0, WPCD_E_INVALID, "E/out NULL or n_E < 0");
        WPCD_REQUIRE(prec == WPCD_FP64 || prec == WPCD_MIXED || prec == WPCD_MIXED_REFINE ||
                         prec == WPCD_MIXED_BF16,
                     WPCD_E_INVALID, "bad precision");
        WPCD_REQUIRE(prec != WPCD_FP64 || c->p_fp64 || (values64 && c->has_val64), WPCD_E_STATE,
                     "FP64 solve needs an FP64 P0 build");
        WPCD_REQUIRE(prec == WPCD_FP64 || !c->p_fp64, WPCD_E_STATE, "mixed solve needs a mixed P0 build");
        m = 48;
        max_iter = 400;
        // FP32 storage of P0 perturbs the operator at the 1e-7 level: a mixed
        // solve gains nothing below 1e-9
        tol = prec == WPCD_FP64 ? 1e-12 : 1e-9;
        want_breakup = 0;
        warm_kind = WPCD_WARM_NONE;
        err_est = false;
        int rmode = WPCD_RESOLVENT_AT_E;
        if (opts) {
            if (opts->krylov_dim > 0) m = opts->krylov_dim;
            if (opts->max_iter > 0) max_iter = opts->max_iter;
            if (opts->tol > 0) tol = opts->tol;
            want_breakup = opts->want_breakup;
            warm_kind = opts->warm_start;
            err_est = opts->err_est != 0;
            rmode = opts->resolvent;
        }
        WPCD_REQUIRE(rmode == WPCD_RESOLVENT_AT_E || rmode == WPCD_RESOLVENT_AVERAGED, WPCD_E_INVALID,
                     "resolvent must be a WPCD_RESOLVENT_* value");
        WPCD_REQUIRE(want_breakup >= 0 && want_breakup <= WPCD_BREAKUP_DIST, WPCD_E_INVALID,
                     "want_breakup must be 0, WPCD_BREAKUP_ELEMENTS or WPCD_BREAKUP_DIST");
        WPCD_REQUIRE(!(rmode == WPCD_RESOLVENT_AVERAGED && want_breakup == WPCD_BREAKUP_ELEMENTS),
                     WPCD_E_INVALID,
                     "breakup elements need the resolvent at E (a pseudostate has several open "
                     "bins with the averaged one): ask for WPCD_BREAKUP_DIST");
        averaged = rmode == WPCD_RESOLVENT_AVERAGED;
        WPCD_REQUIRE(m >= 2 && m <= 128, WPCD_E_INVALID, "krylov_dim must be 2..128");
        WPCD_REQUIRE(warm_kind >= WPCD_WARM_NONE && warm_kind <= WPCD_WARM_GIVEN, WPCD_E_INVALID,
                     "warm_start must be a WPCD_WARM_* value");
        M = basis_rows(c);
        bstride = (int64_t)c->np * total_channels(c) * 5;
        if (warm_kind == WPCD_WARM_GIVEN) WPCD_REQUIRE(opts->x0, WPCD_E_INVALID, "x0 is NULL");
        if (warm_kind == WPCD_WARM_LEARNED)
            WPCD_REQUIRE(c->learned.ready && c->learned.M == M &&
                             c->learned.n_mult == (int)c->pot_mult.size(),
                         WPCD_E_STATE, "no learned warm start for this basis and potential");
        // entrance channel: l = 0, lam = L
        a0 = -1;
        for (int a = 0; a < c->nch; ++a)
            if (c->ch_l[a] == 0 && c->ch_lam[a] == c->L) {
                a0 = a;
                break;
            }
        WPCD_REQUIRE(a0 >= 0, WPCD_E_INVALID, "no entrance channel (l = 0, lam = L)");
        eb = c->waves[c->ch_wave[a0]].h_eps[0];
        qmax = c->q[c->nq];
        res.assign(n_E, wpcd_energy_result{});
        for (int e = 0; e < n_E; ++e) {
            wpcd_energy_result &r = res[e];
            std::memset(&r, 0, sizeof(r));
            r.E = E[e];
            r.status = WPCD_OK;
            r.r0 = 1.0;
            r.err_vs_fp64 = std::numeric_limits<double>::quiet_NaN();
            if (!std::isfinite(E[e])) {
                r.status = WPCD_E_INVALID;
                continue;
            }
            if (E[e] <= eb) {
                r.status = WPCD_E_BELOW_THRESHOLD;
                continue;
            }
            const double q0 = std::sqrt(4.0 * (E[e] - eb) / 3.0);
            r.q0 = q0;
            if (q0 >= qmax) {
                r.status = WPCD_E_INVALID;
                continue;
            }
            const int j0 = (int)(std::upper_bound(c->q.begin(), c->q.end(), q0) - c->q.begin()) - 1;
            r.j0 = j0;
            active.push_back(e);
            idx0v.push_back(((int64_t)a0 * c->nq + j0) * c->np);
            if (averaged) {
                // on-shell energy interval: the energies of the entrance bin j0
                const double e1 = eb + 0.75 * c->q[j0] * c->q[j0], e2 = eb + 0.75 * c->q[j0 + 1] * c->q[j0 + 1];
                ebinv.push_back(e1);
                ebinv.push_back(e2);
                rho0v.push_back(1.0 / (e2 - e1));
            } else {
                rho0v.push_back(2.0 / (3.0 * q0 * (c->q[j0 + 1] - c->q[j0])));
            }
        }
        // the error estimate needs the FP64 P0 values on the same structure
        if (err_est && !c->has_val64 && !active.empty()) {
            build_values(c, true);
            c->has_val64 = true;
        }
    }

    void begin_batch(size_t t) {
        b0 = t * kBatch;
        nb = (int)std::min(active.size() - b0, (size_t)kBatch);
        Eb.assign(nb, 0.0);
        rho0.assign(nb, 0.0);
        ebin.clear();
        idx0.assign(nb, 0);
        for (int t = 0; t < nb; ++t) {
            Eb[t] = E[active[b0 + t]];
            idx0[t] = idx0v[b0 + t];
            rho0[t] = rho0v[b0 + t];
            if (averaged) {
                ebin.push_back(ebinv[2 * (b0 + t)]);
                ebin.push_back(ebinv[2 * (b0 + t) + 1]);
            }
        }
        wc = WarmCtx{};
        wc.kind = warm_kind;
        if (warm_kind == WPCD_WARM_LEARNED) {
            const Learned &L = c->learned;
            double f[kMaxFeat];
            for (int t = 0; t < nb; ++t) {
                const int e = active[b0 + t];
                learn_features(c, Eb[t], res[e].q0, res[e].j0, a0, f);
                for (int k = 0; k < L.nfeat; ++k)
                    wc.feat.push_back((float)((f[k] - L.feat_mu[k]) / L.feat_sd[k]));
            }
        } else if (warm_kind == WPCD_WARM_GIVEN) {
            for (int t = 0; t < nb; ++t) wc.given.push_back(opts->x0 + (size_t)active[b0 + t] * M * 2);
        }
        go = GmresOut{};
        run.reset(gmres_run_new());
        gmres_setup(*run, c, Eb, idx0, prec, m, max_iter, tol,
                    warm_kind == WPCD_WARM_NONE ? nullptr : warm_fill, &wc, go, err_est,
                    averaged ? &ebin : nullptr);
    }

    void end_batch() {
        gmres_finish(*run);
        // amplitude list: elastic first, then open breakup pseudostates
        std::vector<int64_t> rows;
        std::vector<int32_t> ens;
        std::vector<double> rho;
        std::vector<int> first_br(nb), n_br(nb);
        for (int t = 0; t < nb; ++t) {
            rows.push_back(idx0[t]);
            ens.push_back(t);
            rho.push_back(rho0[t]);
        }
        // open breakup states: the pseudostate's on-shell bin (resolvent at
        // E, rho = 2/(3 q dq)), or every bin whose shell eps + 3/4 q^2 meets
        // the on-shell energy interval (averaged, rho = overlap / (D dq)).
        // A reduced system's minor channels follow its major ones, on their
        // own (coarse) lattice and with their own pair states.
        std::vector<int> r_ch, r_k, r_j;
        std::vector<double> r_eps;
        for (int t = 0; t < nb; ++t) {
            r_ch.push_back(-1);
            r_k.push_back(0);
            r_j.push_back(0);
            r_eps.push_back(0.0);
        }
        for (int t = 0; t < nb; ++t) {
            first_br[t] = (int)rows.size();
            n_br[t] = 0;
            int64_t off = 0;
            int a_base = 0;
            for (const wpcd_ctx *g : {(const wpcd_ctx *)c, (const wpcd_ctx *)c->minor}) {
                if (!g) continue;
                const std::vector<double> &qg = g->q;
                auto push = [&](int a, int k, int j, double rh, double ek) {
                    rows.push_back(off + ((int64_t)a * g->nq + j) * g->np + k);
                    ens.push_back(t);
                    rho.push_back(rh);
                    r_ch.push_back(a_base + a);
                    r_k.push_back(k);
                    r_j.push_back(j);
                    r_eps.push_back(ek);
                    ++n_br[t];
                };
                for (int a = 0; a < g->nch; ++a) {
                    const std::vector<double> &ev = g->waves[g->ch_wave[a]].h_eps;
                    for (int k = 0; k < g->np; ++k) {
                        if (g == c && a == a0 && k == 0) continue;
                        if (averaged) {
                            const double e1 = ebin[2 * t], e2 = ebin[2 * t + 1], D = e2 - e1;
                            const double s1 = e1 - ev[k], s2 = e2 - ev[k];
                            if (!(s2 > 0.0)) continue;
                            const double q1 = s1 > 0.0 ? std::sqrt(4.0 * s1 / 3.0) : 0.0;
                            const double q2 = std::sqrt(4.0 * s2 / 3.0);
                            int j = (int)(std::upper_bound(qg.begin(), qg.end(), q1) - qg.begin()) - 1;
                            for (j = std::max(j, 0); j < g->nq && qg[j] < q2; ++j) {
                                const double ov = std::min(qg[j + 1], q2) - std::max(qg[j], q1);
                                if (!(ov > 0.0)) continue;
                                push(a, k, j, ov / (D * (qg[j + 1] - qg[j])), ev[k]);
                            }
                            continue;
                        }
                        if (!(ev[k] < Eb[t])) continue;
                        const double qk = std::sqrt(4.0 * (Eb[t] - ev[k]) / 3.0);
                        if (qk >= qmax) continue;
                        const int jk =
                            (int)(std::upper_bound(qg.begin(), qg.end(), qk) - qg.begin()) - 1;
                        push(a, k, jk, 2.0 / (3.0 * qk * (qg[jk + 1] - qg[jk])), ev[k]);
                    }
                }
                off += (int64_t)g->nch * g->nq * g->np;
                a_base += g->nch;
            }
        }
        std::vector<double> amp;
        amplitudes_batch(c, nb, rows, ens, rho, rho0, amp);
        std::vector<int> ok;
        for (int t = 0; t < nb; ++t) {
            const int e = active[b0 + t];
            wpcd_energy_result &r = res[e];
            r.iters = go.iters[t];
            r.residual = go.resid[t];
            r.warm = go.warm[t];
            r.r0 = go.r0[t];
            if (go.edge[t]) {
                r.status = WPCD_E_ON_EDGE;
                continue;
            }
            if (!(go.resid[t] <= tol * 10.0))
                r.status = go.stag[t] ? WPCD_E_STAGNATED : WPCD_E_NOT_CONVERGED;
            r.U_re = amp[4 * t];
            r.U_im = amp[4 * t + 1];
            r.A_re = rho0[t] * r.U_re;
            r.A_im = rho0[t] * r.U_im;
            r.S_re = 1.0 + amp[4 * t + 2];
            r.S_im = amp[4 * t + 3];
            r.delta = 0.5 * std::atan2(r.S_im, r.S_re);
            r.eta = std::hypot(r.S_re, r.S_im);
            r.n_open = n_br[t];   // open channel states (elements); distribution rows below
            if (err_est) {
                const double du = std::hypot(go.dU[2 * t], go.dU[2 * t + 1]);
                const double u = std::hypot(go.U[2 * t], go.U[2 * t + 1]);
                r.err_vs_fp64 = u > 0.0 ? du / u : std::numeric_limits<double>::quiet_NaN();
            }
            if (r.status == WPCD_OK) ok.push_back(t);
            if (breakup_out && want_breakup == WPCD_BREAKUP_ELEMENTS) {
                double *dst = breakup_out + (size_t)e * bstride;
                for (int u = 0; u < n_br[t]; ++u) {
                    const int row = first_br[t] + u;
                    dst[5 * u + 0] = r_ch[row];
                    dst[5 * u + 1] = r_k[row];
                    dst[5 * u + 2] = r_j[row];
                    dst[5 * u + 3] = amp[4 * row + 2];
                    dst[5 * u + 4] = amp[4 * row + 3];
                }
            } else if (want_breakup == WPCD_BREAKUP_DIST) {
                // one row per pseudostate with open bins, in row order
                // (channel major, then k): summed |S|^2 over its bins
                double *dst = breakup_out ? breakup_out + (size_t)e * bstride : nullptr;
                int nd = 0;
                for (int u = 0; u < n_br[t];) {
                    const int row0 = first_br[t] + u;
                    const int a = r_ch[row0], k = r_k[row0];
                    double ptot = 0.0;
                    int nbin = 0;
                    for (; u < n_br[t]; ++u, ++nbin) {
                        const int row = first_br[t] + u;
                        if (r_ch[row] != a || r_k[row] != k) break;
                        ptot += amp[4 * row + 2] * amp[4 * row + 2] + amp[4 * row + 3] * amp[4 * row + 3];
                    }
                    if (dst) {
                        dst[5 * nd + 0] = a;
                        dst[5 * nd + 1] = k;
                        dst[5 * nd + 2] = r_eps[row0];
                        dst[5 * nd + 3] = ptot;
                        dst[5 * nd + 4] = nbin;
                    }
                    ++nd;
                }
                r.n_open = nd;
            }
        }
        if (collect && !ok.empty()) {
            WPCD_REQUIRE(collect->n + (int64_t)ok.size() <= collect->cap, WPCD_E_INVALID,
                         "snapshot store full");
            learn_snap_store(c, collect->snaps, collect->n, c->d_X.ptr, nb, ok);
            double f[kMaxFeat];
            for (int t : ok) {
                const int e = active[b0 + t];
                collect->nfeat = learn_features(c, Eb[t], res[e].q0, res[e].j0, a0, f);
                collect->feat.insert(collect->feat.end(), f, f + collect->nfeat);
                collect->iters += go.iters[t];
            }
            collect->n += (int64_t)ok.size();
        }
    }

    void finish() {
        for (int e = 0; e < n_E; ++e) out[e] = res[e];
    }
};

static void run_job(SolveJob &j) {
    j.plan();
    for (size_t t = 0; t < j.n_batches(); ++t) {
        j.begin_batch(t);
        std::vector<GmresRun *> one{j.run.get()};
        gmres_cycles(one);
        j.end_batch();
    }
    j.finish();
}

static void solve_impl(wpcd_ctx *c, const double *E, int n_E, wpcd_precision prec,
                       const wpcd_solve_opts *opts, wpcd_energy_result *out, double *breakup_out,
                       Collect *collect) {
    SolveJob j;
    j.c = c;
    j.E = E;
    j.n_E = n_E;
    j.prec = prec;
    j.opts = opts;
    j.out = out;
    j.breakup_out = breakup_out;
    j.collect = collect;
    run_job(j);
    if (!opts || !(opts->fallback_tol > 0.0) || prec == WPCD_FP64 || collect) return;
    // FP64 fallback: the energies the mixed tier did not converge, or whose
    // error estimate is above the bound (or not finite), solved again on
    // the FP64 values of the same structure
    std::vector<int> redo;
    for (int e = 0; e < n_E; ++e) {
        const wpcd_energy_result &r = out[e];
        if (r.status == WPCD_E_NOT_CONVERGED || r.status == WPCD_E_STAGNATED ||
            (r.status == WPCD_OK && j.err_est && !(r.err_vs_fp64 <= opts->fallback_tol)))
            redo.push_back(e);
    }
    if (redo.empty()) return;
    if (!c->p_fp64 && !c->has_val64) {
        build_values(c, true);
        c->has_val64 = true;
    }
    const int n2 = (int)redo.size();
    std::vector<double> E2(n2), x02;
    for (int k = 0; k < n2; ++k) E2[k] = E[redo[k]];
    wpcd_solve_opts o2 = *opts;
    o2.fallback_tol = 0.0;
    if (o2.warm_start == WPCD_WARM_GIVEN) {   // the chosen energies' rows of x0
        const size_t row = (size_t)j.M * 2;
        x02.resize((size_t)n2 * row);
        for (int k = 0; k < n2; ++k)
            std::memcpy(x02.data() + k * row, opts->x0 + (size_t)redo[k] * row, row * sizeof(double));
        o2.x0 = x02.data();
    }
    std::vector<wpcd_energy_result> out2(n2);
    std::vector<double> br2(breakup_out && j.want_breakup ? (size_t)n2 * j.bstride : 0);
    SolveJob j2;
    j2.c = c;
    j2.E = E2.data();
    j2.n_E = n2;
    j2.prec = WPCD_FP64;
    j2.opts = &o2;
    j2.out = out2.data();
    j2.breakup_out = br2.empty() ? nullptr : br2.data();
    j2.values64 = true;
    run_job(j2);
    for (int k = 0; k < n2; ++k) {
        out[redo[k]] = out2[k];
        out[redo[k]].fallback = 1;
        if (!br2.empty())
            std::memcpy(breakup_out + (size_t)redo[k] * j.bstride, br2.data() + (size_t)k * j.bstride,
                        (size_t)j.bstride * sizeof(double));
    }
}

static uint64_t splitmix_next(uint64_t &st) {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Training of the learned warm start (see wpcd_learn_desc).
static void learn_train(wpcd_ctx *c, const wpcd_learn_desc *d, wpcd_learn_report *rep) {
    WPCD_REQUIRE(c->has_basis && c->has_pot && c->has_p, WPCD_E_STATE,
                 "build_basis and build_p must come first");
    WPCD_REQUIRE(d, WPCD_E_INVALID, "learn descriptor is NULL");
    const int nm = (int)c->pot_base.size();
    WPCD_REQUIRE(d->n_var >= 1 && d->n_E >= 1 && d->mult && d->E, WPCD_E_INVALID,
                 "need n_var >= 1, n_E >= 1, mult and E");
    WPCD_REQUIRE(d->n_mult == nm, WPCD_E_INVALID, "n_mult must equal the potential's n_terms");
    WPCD_REQUIRE(d->n_basis >= 1 && d->n_basis <= 128, WPCD_E_INVALID, "n_basis must be 1..128");
    const int hidden = d->hidden > 0 ? d->hidden : 256;
    WPCD_REQUIRE(hidden >= 16 && hidden <= 512, WPCD_E_INVALID, "hidden must be 16..512");
    const int epochs = d->epochs > 0 ? d->epochs : 400;
    const int bsz_req = d->batch > 0 ? d->batch : 64;
    const double lr = d->lr > 0 ? d->lr : 2e-3;
    WPCD_REQUIRE(std::isfinite(lr), WPCD_E_INVALID, "lr must be finite");
    WPCD_REQUIRE(d->precision == WPCD_FP64 || d->precision == WPCD_MIXED, WPCD_E_INVALID,
                 "bad precision");
    for (int64_t k = 0; k < (int64_t)d->n_var * nm; ++k)
        WPCD_REQUIRE(std::isfinite(d->mult[k]) && d->mult[k] > 0.0, WPCD_E_INVALID,
                     "multipliers must be finite and > 0");
    hipStream_t s = c->stream;
    Learned &L = c->learned;
    L.release();
    const int64_t M = (int64_t)c->nch * c->nq * c->np;
    wpcd_solve_opts so{};
    if (d->solve) so = *d->solve;
    so.warm_start = WPCD_WARM_NONE;
    so.x0 = nullptr;
    so.want_breakup = 0;

    // 1. plain solves over the variants; converged solutions become snapshots
    auto t0 = std::chrono::steady_clock::now();
    DBuf<float> snaps;
    Collect col;
    col.cap = (int64_t)d->n_var * d->n_E;
    snaps.reserve((size_t)col.cap * M * 2);
    col.snaps = snaps.ptr;
    std::vector<wpcd_energy_result> res(d->n_E);
    const std::vector<double> ones(nm, 1.0);
    try {
        for (int v = 0; v < d->n_var; ++v) {
            set_multipliers(c, d->mult + (size_t)v * nm, nm);
            solve_impl(c, d->E + (size_t)v * d->n_E, d->n_E, (wpcd_precision)d->precision, &so,
                       res.data(), nullptr, &col);
        }
    } catch (...) {
        set_multipliers(c, ones.data(), nm);
        throw;
    }
    set_multipliers(c, ones.data(), nm);
    const double solve_ms = ms_since(t0);
    const int n = (int)col.n;
    WPCD_REQUIRE(n >= 1, WPCD_E_INVALID, "no training solve converged");

    // 2. greedy reduced basis and the coefficient targets
    t0 = std::chrono::steady_clock::now();
    std::vector<double> coef;
    double max_err = 0.0, mean_err = 0.0;
    learn_build_basis(c, snaps.ptr, n, std::min(d->n_basis, n), coef, max_err, mean_err);
    snaps.release();
    const int K = L.K;
    WPCD_REQUIRE(K >= 1, WPCD_E_INVALID, "empty reduced basis");
    const double basis_ms = ms_since(t0);

    // 3. network: normalised features -> coefficients / coef_scale
    t0 = std::chrono::steady_clock::now();
    const int nf = col.nfeat;
    L.nfeat = nf;
    L.n_mult = nm;
    for (int k = 0; k < nf; ++k) {
        double mu = 0.0, sd = 0.0;
        for (int i = 0; i < n; ++i) mu += col.feat[(size_t)i * nf + k] / n;
        for (int i = 0; i < n; ++i) {
            const double dv = col.feat[(size_t)i * nf + k] - mu;
            sd += dv * dv / n;
        }
        sd = std::sqrt(sd);
        L.feat_mu[k] = mu;
        L.feat_sd[k] = sd > 1e-12 * std::max(1.0, std::fabs(mu)) ? sd : 1.0;
    }
    double c2 = 0.0;
    for (double x : coef) c2 += x * x;
    L.coef_scale = c2 > 0 ? std::sqrt(c2 / coef.size()) : 1.0;
    const int nout = 2 * K;
    std::vector<float> Xh((size_t)n * nf), Th((size_t)n * nout);
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < nf; ++k)
            Xh[(size_t)i * nf + k] = (float)((col.feat[(size_t)i * nf + k] - L.feat_mu[k]) / L.feat_sd[k]);
        for (int k = 0; k < K; ++k) {
            Th[(size_t)i * nout + 2 * k] = (float)(coef[2 * ((size_t)k * n + i)] / L.coef_scale);
            Th[(size_t)i * nout + 2 * k + 1] = (float)(coef[2 * ((size_t)k * n + i) + 1] / L.coef_scale);
        }
    }
    DBuf<float> dX, dT, bX, bT;
    DBuf<int32_t> dperm;
    dX.reserve(Xh.size());
    dT.reserve(Th.size());
    const int bsz = std::min(bsz_req, n);
    bX.reserve((size_t)bsz * nf);
    bT.reserve((size_t)bsz * nout);
    dperm.reserve(n);
    WPCD_HIP(hipMemcpyAsync(dX.ptr, Xh.data(), Xh.size() * sizeof(float), hipMemcpyHostToDevice, s));
    WPCD_HIP(hipMemcpyAsync(dT.ptr, Th.data(), Th.size() * sizeof(float), hipMemcpyHostToDevice, s));
    Mlp &net = L.mlp;
    mlp_init(net, s, nf, hidden, nout, d->seed);
    const double loss_first = mlp_loss_grad(net, s, c->timer, dX.ptr, dT.ptr, n, true);
    std::vector<int32_t> perm(n);
    uint64_t st = d->seed ^ 0x5DEECE66Dull;
    const int nbatch = (n + bsz - 1) / bsz;
    const int64_t total_steps = (int64_t)epochs * nbatch;
    int64_t step = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int i = n - 1; i > 0; --i) {
            const int j = (int)(splitmix_next(st) % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        WPCD_HIP(hipMemcpyAsync(dperm.ptr, perm.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
        for (int bi = 0; bi < nbatch; ++bi, ++step) {
            const int first = bi * bsz, cnt = std::min(bsz, n - first);
            mlp_gather(s, dX.ptr, nf, dperm.ptr + first, cnt, bX.ptr);
            mlp_gather(s, dT.ptr, nout, dperm.ptr + first, cnt, bT.ptr);
            mlp_loss_grad(net, s, c->timer, bX.ptr, bT.ptr, cnt, false);
            const double lr_min = lr / 20.0;
            const double lr_t =
                lr_min + 0.5 * (lr - lr_min) * (1.0 + std::cos(M_PI * (double)step / (double)total_steps));
            mlp_adam_step(net, s, c->timer, (float)lr_t);
        }
        // the minibatch order of the next epoch is uploaded only after this
        // epoch's gathers have run
        WPCD_HIP(hipStreamSynchronize(s));
    }
    const double loss_last = mlp_loss_grad(net, s, c->timer, dX.ptr, dT.ptr, n, true);
    dX.release();
    dT.release();
    bX.release();
    bT.release();
    dperm.release();
    L.ready = true;
    const double train_ms = ms_since(t0);
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->n_samples = n;
        rep->plain_iters = (int32_t)col.iters;
        rep->basis_max_rel_err = max_err;
        rep->basis_mean_rel_err = mean_err;
        rep->loss_first = loss_first;
        rep->loss_last = loss_last;
        rep->solve_ms = solve_ms;
        rep->basis_ms = basis_ms;
        rep->train_ms = train_ms;
    }
}

// One forward and backward pass on caller data with a temporary network.
static void mlp_eval(wpcd_ctx *c, int nin, int nh, int nout, const float *params, int B,
                     const float *X, const float *T, float *Y_out, float *grad_out,
                     double *loss_out) {
    WPCD_REQUIRE(nin >= 1 && nin <= 4096 && nh >= 1 && nh <= 4096 && nout >= 1 && nout <= 4096 &&
                     B >= 1 && B <= 65536,
                 WPCD_E_INVALID, "network sizes out of range");
    WPCD_REQUIRE(params && X, WPCD_E_INVALID, "params/X NULL");
    WPCD_REQUIRE(T || (!grad_out && !loss_out), WPCD_E_INVALID, "gradients and loss need T");
    hipStream_t s = c->stream;
    Mlp net;
    net.nin = nin;
    net.nh = nh;
    net.nout = nout;
    DBuf<float> dX, dT;
    try {
        mlp_set_weights(net, s, params);
        dX.reserve((size_t)B * nin);
        WPCD_HIP(hipMemcpyAsync(dX.ptr, X, (size_t)B * nin * sizeof(float), hipMemcpyHostToDevice, s));
        const float *Y = mlp_forward(net, s, c->timer, dX.ptr, B);
        if (Y_out)
            WPCD_HIP(hipMemcpyAsync(Y_out, Y, (size_t)B * nout * sizeof(float), hipMemcpyDeviceToHost, s));
        WPCD_HIP(hipStreamSynchronize(s));
        if (T) {
            dT.reserve((size_t)B * nout);
            WPCD_HIP(hipMemcpyAsync(dT.ptr, T, (size_t)B * nout * sizeof(float), hipMemcpyHostToDevice, s));
            const double loss = mlp_loss_grad(net, s, c->timer, dX.ptr, dT.ptr, B, true);
            if (grad_out)
                WPCD_HIP(hipMemcpyAsync(grad_out, net.grad.ptr, net.n_params() * sizeof(float),
                                        hipMemcpyDeviceToHost, s));
            WPCD_HIP(hipStreamSynchronize(s));
            if (loss_out) *loss_out = loss;
        }
    } catch (...) {
        (void)hipStreamSynchronize(s);
        net.release();
        dX.release();
        dT.release();
        throw;
    }
    net.release();
    dX.release();
    dT.release();
}

}  // namespace wpcd

using namespace wpcd;

// ---- fixed device scratch of wpcd_build_p_noalloc
// The intermediates of that call (row counts, per-tile totals, row hints and
// row-start marks of the element kernels) live in one file-scope device
// array of WPCD_NOALLOC_SCRATCH_BYTES per device, so the call allocates
// nothing.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address is taken once per device with
// hipGetSymbolAddress (in wpcd_create, with that device current) and only
// that address is used.
static __device__ __align__(256) unsigned char scratch[WPCD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device `dev` (looked
// up once per device).  Returns a HIP error code.
hipError_t scratch_setup(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (g_scratch_ptr[dev]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<unsigned char *>(ptr);
    return hipSuccess;
}

unsigned char *scratch_of(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return dev >= 0 && dev < kMaxDevices ? g_scratch_ptr[dev] : nullptr;
}
}  // namespace

template <class F>
static wpcd_status guarded(wpcd_ctx *c, F &&f) {
    if (!c) return WPCD_E_INVALID;
    try {
        WPCD_HIP(hipSetDevice(c->device));
        f();
        c->err.clear();
        return WPCD_OK;
    } catch (const Error &e) {
        c->err = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        c->err = e.what();
        return WPCD_E_NOMEM;
    } catch (...) {
        c->err = "unknown error";
        return WPCD_E_DEVICE;
    }
}

extern "C" {

wpcd_status wpcd_create(int device, void *hip_stream, wpcd_ctx **out) {
    if (!out) return WPCD_E_INVALID;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return WPCD_E_DEVICE;
    if (device < 0 || device >= ndev) return WPCD_E_INVALID;
    wpcd_ctx *c = new (std::nothrow) wpcd_ctx();
    if (!c) return WPCD_E_NOMEM;
    c->device = device;
    if (hipSetDevice(device) != hipSuccess || scratch_setup(device) != hipSuccess) {
        delete c;
        return WPCD_E_DEVICE;
    }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return WPCD_E_DEVICE;
        }
        c->own_stream = true;
    }
    *out = c;
    return WPCD_OK;
}

// Basis set-up shared by the boson and the nucleon entry points.  nuc:
// three nucleons in pair s-waves (channels from nuc; the channel arrays of
// b are not read), else spinless bosons with b's channels.
static void build_basis_impl(wpcd_ctx *c, const wpcd_basis_desc *b, const wpcd_potential_desc *pot,
                             const wpcd_nucleon_desc *nuc, bool with_waves = true) {
    WPCD_REQUIRE(b, WPCD_E_INVALID, "basis descriptor is NULL");
    WPCD_REQUIRE(pot || !with_waves, WPCD_E_INVALID, "potential descriptor is NULL");
    WPCD_REQUIRE(b->n_p >= 2 && b->n_p <= 1024 && b->n_q >= 2 && b->n_q <= 1024,
                 WPCD_E_INVALID, "n_p, n_q must be in 2..1024");
    WPCD_REQUIRE(b->n_gauss_q >= 1 && b->n_gauss_q <= kMaxGq, WPCD_E_INVALID,
                 "n_gauss_q must be 1..16");
    WPCD_REQUIRE(b->n_gauss_x >= 1 && b->n_gauss_x <= kMaxGx, WPCD_E_INVALID,
                 "n_gauss_x must be 1..64");
    // channels: (l, lam) per channel, and for nucleons (s, t) and the
    // pair wave of each channel (its own, with its strength multipliers)
    int nch, L;
    std::vector<int> ch_l, ch_lam, ch_s, ch_t;
    std::vector<int> waves;   // l of each pair wave
    std::vector<int> ch_wave;
    if (nuc) {
        WPCD_REQUIRE(nuc->two_S == 1 || nuc->two_S == 3, WPCD_E_INVALID, "two_S must be 1 or 3");
        WPCD_REQUIRE(nuc->n_ch >= 1 && nuc->n_ch <= 2, WPCD_E_INVALID,
                     "nucleon pair s-waves have 1 or 2 channels");
        WPCD_REQUIRE(nuc->s && nuc->t, WPCD_E_INVALID, "channel arrays NULL");
        nch = nuc->n_ch;
        L = 0;
        for (int a = 0; a < nch; ++a) {
            const int sa = nuc->s[a], ta = nuc->t[a];
            WPCD_REQUIRE((sa == 1 && ta == 0) || (sa == 0 && ta == 1), WPCD_E_INVALID,
                         "pair s-wave channels are (s, t) = (1, 0) or (0, 1)");
            WPCD_REQUIRE(nuc->two_S == 1 || sa == 1, WPCD_E_INVALID,
                         "three-body spin 3/2 needs pair spin 1");
            for (int b2 = 0; b2 < a; ++b2)
                WPCD_REQUIRE(nuc->s[b2] != sa, WPCD_E_INVALID, "repeated channel");
            ch_l.push_back(0);
            ch_lam.push_back(0);
            ch_s.push_back(sa);
            ch_t.push_back(ta);
            waves.push_back(0);
            ch_wave.push_back(a);
        }
        WPCD_REQUIRE(ch_s[0] == 1, WPCD_E_INVALID,
                     "channel 0 must be the deuteron channel (s, t) = (1, 0)");
        WPCD_REQUIRE(pot, WPCD_E_INVALID, "potential descriptor is NULL");
        WPCD_REQUIRE(!nuc->mult || pot->n_terms >= 1, WPCD_E_INVALID, "bad n_terms");
        if (nuc->mult)
            for (int k = 0; k < nch * pot->n_terms; ++k)
                WPCD_REQUIRE(std::isfinite(nuc->mult[k]) && nuc->mult[k] >= 0.0, WPCD_E_INVALID,
                             "strength multipliers must be finite and >= 0");
    } else {
        WPCD_REQUIRE(b->n_ch >= 1 && b->n_ch <= kMaxCh, WPCD_E_INVALID, "n_ch must be 1..8");
        WPCD_REQUIRE(b->l && b->lam, WPCD_E_INVALID, "channel arrays NULL");
        WPCD_REQUIRE(b->L >= 0 && b->L <= 8, WPCD_E_INVALID, "L must be 0..8");
        nch = b->n_ch;
        L = b->L;
        for (int a = 0; a < nch; ++a) {
            const int l = b->l[a], lam = b->lam[a];
            WPCD_REQUIRE(l >= 0 && l <= 4 && lam >= 0 && lam <= kMaxLam && l % 2 == 0,
                         WPCD_E_INVALID, "channels need even l <= 4 and lam <= 4");
            WPCD_REQUIRE(std::abs(l - lam) <= L && L <= l + lam && (l + lam - L) % 2 == 0,
                         WPCD_E_INVALID, "channel (l, lam) cannot couple to L with parity (-1)^L");
            if (std::find(waves.begin(), waves.end(), l) == waves.end()) waves.push_back(l);
            ch_l.push_back(l);
            ch_lam.push_back(lam);
            ch_s.push_back(0);
            ch_t.push_back(0);
            ch_wave.push_back((int)(std::find(waves.begin(), waves.end(), l) - waves.begin()));
        }
    }
    WPCD_REQUIRE((int)waves.size() <= kMaxWaves, WPCD_E_INVALID, "too many pair waves");
    const int two_S = nuc ? nuc->two_S : 0;
    std::vector<double> p, q;
    if (b->edge_kind == 0) {
        WPCD_REQUIRE(b->p_max > 0 && b->q_max > 0 && std::isfinite(b->p_max) &&
                         std::isfinite(b->q_max),
                     WPCD_E_INVALID, "p_max, q_max must be positive");
        p = cheb_edges(b->n_p, b->p_max);
        q = cheb_edges(b->n_q, b->q_max);
    } else if (b->edge_kind == 1) {
        WPCD_REQUIRE(b->p_edges && b->q_edges, WPCD_E_INVALID, "explicit edges NULL");
        p.assign(b->p_edges, b->p_edges + b->n_p + 1);
        q.assign(b->q_edges, b->q_edges + b->n_q + 1);
        WPCD_REQUIRE(p[0] >= 0 && q[0] >= 0, WPCD_E_INVALID, "edges must start >= 0");
        for (int k = 0; k < b->n_p; ++k)
            WPCD_REQUIRE(p[k + 1] > p[k] && std::isfinite(p[k + 1]), WPCD_E_INVALID,
                         "p edges must increase");
        for (int k = 0; k < b->n_q; ++k)
            WPCD_REQUIRE(q[k + 1] > q[k] && std::isfinite(q[k + 1]), WPCD_E_INVALID,
                         "q edges must increase");
    } else {
        throw Error{WPCD_E_INVALID, "edge_kind must be 0 or 1"};
    }
    bool same_grid = c->has_basis && c->np == b->n_p && c->nq == b->n_q && c->p == p &&
                     c->q == q && c->ngq == b->n_gauss_q && c->ngx == b->n_gauss_x &&
                     c->L == L && c->nch == nch && c->nuc_two_S == two_S;
    for (int a = 0; same_grid && a < nch; ++a)
        same_grid = c->ch_l[a] == ch_l[a] && c->ch_lam[a] == ch_lam[a] &&
                    c->ch_s[a] == ch_s[a] && c->ch_t[a] == ch_t[a];
    c->has_basis = false;
    c->learned.release();
    c->has_pot = false;
    if (!same_grid) {
        c->has_p = false;
        c->has_val64 = false;
    }
    c->np = b->n_p;
    c->nq = b->n_q;
    c->ngq = b->n_gauss_q;
    c->ngx = b->n_gauss_x;
    c->L = L;
    c->nch = nch;
    c->nuc_two_S = two_S;
    c->p = p;
    c->q = q;
    gauss_legendre_gw(c->ngq, c->gq, c->wq);
    gauss_legendre_gw(c->ngx, c->gx, c->wx);
    c->n_waves = (int)waves.size();
    for (int w = 0; w < c->n_waves; ++w) {
        c->waves[w].l = waves[w];
        c->waves[w].mult.clear();
        if (nuc && nuc->mult)
            c->waves[w].mult.assign(nuc->mult + (size_t)w * pot->n_terms,
                                    nuc->mult + (size_t)(w + 1) * pot->n_terms);
    }
    for (int a = 0; a < c->nch; ++a) {
        c->ch_l[a] = ch_l[a];
        c->ch_lam[a] = ch_lam[a];
        c->ch_s[a] = ch_s[a];
        c->ch_t[a] = ch_t[a];
        c->ch_wave[a] = ch_wave[a];
    }
    upload_tables(c);
    // s-wave element kernel only for the single boson channel; nucleon
    // channels take the multichannel kernels with degree-0 couplings g_ab
    c->swave = !nuc && (c->nch == 1 && c->L == 0 && c->ch_l[0] == 0 && c->ch_lam[0] == 0);
    // angular coupling: the fitted polynomial for l, lam <= 2 (validated
    // and fast), the direct bipolar-harmonic terms beyond
    c->mc_direct = false;
    for (int a = 0; a < c->nch; ++a)
        if (c->ch_l[a] > 2 || c->ch_lam[a] > 2) c->mc_direct = true;
    c->mc_pairs.clear();
    c->mc_deg = 0;
    c->nuc_g.clear();
    if (nuc) {
        std::vector<double> coef;
        nucleon_tables(two_S, c->nch, c->ch_s, c->ch_t, c->mc_pairs, coef, c->nuc_g);
        upload(c->d_mcoef, coef, c->stream);
    } else if (!c->mc_direct) {
        std::vector<double> coef;
        coupling_tables(c->L, c->nch, c->ch_l, c->ch_lam, c->mc_pairs, coef);
        for (auto &pp : c->mc_pairs) c->mc_deg = std::max(c->mc_deg, pp.d);
        upload(c->d_mcoef, coef, c->stream);
    } else {
        std::vector<McTerm> terms;
        std::vector<int> first;
        coupling_terms(c->L, c->nch, c->ch_l, c->ch_lam, terms, first);
        upload(c->d_mterms, terms, c->stream);
        upload(c->d_mterm_first, first, c->stream);
    }
    WPCD_HIP(hipStreamSynchronize(c->stream));
    c->has_basis = true;
    if (with_waves) build_pair_waves(c, pot);
}

// Every device buffer of a context (and of its reduced system's minor
// part); the context itself and its stream stay.
static void release_all(wpcd_ctx *c);

// A reduced system becomes an ordinary context again (no P0, no minor part).
static void drop_reduction(wpcd_ctx *c) {
    if (!c->reduced && !c->minor) return;
    if (c->minor) {
        release_all(c->minor);
        delete c->minor;
        c->minor = nullptr;
    }
    c->reduced = false;
    c->red_rows = 0;
    c->has_p = false;
    c->has_val64 = false;
    c->pred_nnz = -1;
    for (auto &g : c->graphs) g.release();
    c->graphs.clear();
    for (auto &g : c->multi_graphs) (void)hipGraphExecDestroy(g.exec);
    c->multi_graphs.clear();
}

#define WPCD_NOT_REDUCED(c)                                                                \
    WPCD_REQUIRE(!(c)->reduced, WPCD_E_STATE,                                             \
                 "not available on a reduced system (build a basis to reuse the context)")

wpcd_status wpcd_build_basis(wpcd_ctx *c, const wpcd_basis_desc *b, const wpcd_potential_desc *pot) {
    return guarded(c, [&] {
        drop_reduction(c);
        build_basis_impl(c, b, pot, nullptr);
    });
}

// The potential of `src` (kind, strengths with their multipliers, ranges,
// fitted scale) on `c`'s pair waves, diagonalised on c's lattice.
static void copy_potential(const wpcd_ctx *src, wpcd_ctx *c) {
    c->pot_kind = src->pot_kind;
    c->pot_s = src->pot_s;
    c->pot_base = src->pot_base;
    c->pot_mult = src->pot_mult;
    c->pot_mu = src->pot_mu;
    c->pot_scale = src->pot_scale;
    c->has_pot = false;
    diagonalise_all(c);
    c->has_pot = true;
}

// The pair waves of `src` on `c` (the same lattice and potential): each of
// c's waves copied from src's wave of the same l, no diagonalisation.
static void copy_waves(const wpcd_ctx *src, wpcd_ctx *c) {
    const int n = c->np;
    c->pot_kind = src->pot_kind;
    c->pot_s = src->pot_s;
    c->pot_base = src->pot_base;
    c->pot_mult = src->pot_mult;
    c->pot_mu = src->pot_mu;
    c->pot_scale = src->pot_scale;
    for (int w = 0; w < c->n_waves; ++w) {
        int ws = -1;
        for (int k = 0; k < src->n_waves; ++k)
            if (src->waves[k].l == c->waves[w].l) ws = k;
        WPCD_REQUIRE(ws >= 0, WPCD_E_STATE, "pair wave missing in the full system");
        const PairWave &a = src->waves[ws];
        PairWave &b = c->waves[w];
        b.v.reserve((size_t)n * n);
        b.O.reserve((size_t)n * n);
        b.Vt.reserve((size_t)n * n);
        b.eps.reserve(n);
        const size_t nn = (size_t)n * n * sizeof(double);
        WPCD_HIP(hipMemcpyAsync(b.v.ptr, a.v.ptr, nn, hipMemcpyDeviceToDevice, c->stream));
        WPCD_HIP(hipMemcpyAsync(b.O.ptr, a.O.ptr, nn, hipMemcpyDeviceToDevice, c->stream));
        WPCD_HIP(hipMemcpyAsync(b.Vt.ptr, a.Vt.ptr, nn, hipMemcpyDeviceToDevice, c->stream));
        WPCD_HIP(hipMemcpyAsync(b.eps.ptr, a.eps.ptr, n * sizeof(double), hipMemcpyDeviceToDevice,
                                c->stream));
        b.h_eps = a.h_eps;
    }
    WPCD_HIP(hipStreamSynchronize(c->stream));
    c->has_pot = true;
}

// Feshbach reduction (Sec. V.B): see wpcd_build_reduced in the header.
static void build_reduced(wpcd_ctx *red, wpcd_ctx *full, int nmaj, int cp, int cq,
                          wpcd_precision prec) {
    WPCD_REQUIRE(full && full != red, WPCD_E_INVALID, "full is NULL or the reduced context itself");
    WPCD_REQUIRE(!full->reduced, WPCD_E_INVALID, "full is itself a reduced system");
    WPCD_REQUIRE(full->has_basis && full->has_pot && full->has_p, WPCD_E_STATE,
                 "the full system needs its basis, potential and P0");
    WPCD_REQUIRE(full->device == red->device, WPCD_E_INVALID, "contexts on different devices");
    WPCD_REQUIRE(full->nuc_two_S == 0, WPCD_E_INVALID, "the reduction takes boson channel sets");
    WPCD_REQUIRE(nmaj >= 1 && nmaj < full->nch, WPCD_E_INVALID,
                 "n_major must leave at least one major and one minor channel");
    WPCD_REQUIRE(cp >= 1 && cq >= 1 && full->np % cp == 0 && full->nq % cq == 0 &&
                     full->np / cp >= 2 && full->nq / cq >= 2,
                 WPCD_E_INVALID, "r_p, r_q must divide n_p, n_q and leave at least 2 bins");
    WPCD_REQUIRE(prec == WPCD_FP64 || prec == WPCD_MIXED, WPCD_E_INVALID,
                 "precision must be WPCD_FP64 or WPCD_MIXED");
    bool entrance = false;
    for (int a = 0; a < nmaj; ++a) entrance |= full->ch_l[a] == 0 && full->ch_lam[a] == full->L;
    WPCD_REQUIRE(entrance, WPCD_E_INVALID, "the entrance channel (l = 0, lam = L) must be major");
    // the unreduced values in FP64 (computed once on the existing structure)
    if (!full->p_fp64 && !full->has_val64) {
        build_values(full, true);
        full->has_val64 = true;
    }
    WPCD_HIP(hipStreamSynchronize(full->stream));
    drop_reduction(red);
    red->learned.release();
    // major part: this context, the full system's lattice and major channels
    wpcd_basis_desc bd{};
    bd.n_p = full->np;
    bd.n_q = full->nq;
    bd.edge_kind = 1;
    bd.p_edges = full->p.data();
    bd.q_edges = full->q.data();
    bd.n_gauss_q = full->ngq;
    bd.n_gauss_x = full->ngx;
    bd.L = full->L;
    bd.n_ch = nmaj;
    bd.l = full->ch_l;
    bd.lam = full->ch_lam;
    build_basis_impl(red, &bd, nullptr, nullptr, false);
    copy_waves(full, red);
    // minor part: every cp-th p edge and cq-th q edge, the minor channels
    wpcd_ctx *m = new wpcd_ctx();
    m->device = red->device;
    m->stream = red->stream;
    m->own_stream = false;
    red->minor = m;
    std::vector<double> pc, qc;
    for (int k = 0; k <= full->np; k += cp) pc.push_back(full->p[k]);
    for (int k = 0; k <= full->nq; k += cq) qc.push_back(full->q[k]);
    wpcd_basis_desc bm = bd;
    bm.n_p = full->np / cp;
    bm.n_q = full->nq / cq;
    bm.p_edges = pc.data();
    bm.q_edges = qc.data();
    bm.n_ch = full->nch - nmaj;
    bm.l = full->ch_l + nmaj;
    bm.lam = full->ch_lam + nmaj;
    build_basis_impl(m, &bm, nullptr, nullptr, false);
    copy_potential(full, m);
    // P0 of the reduced cells
    reduce_p0(full, red, nmaj, cp, cq, full->d_val64.ptr, prec == WPCD_MIXED);
    red->reduced = true;
    red->red_cp = cp;
    red->red_cq = cq;
    red->red_rows = (int64_t)nmaj * full->np * full->nq + (int64_t)m->nch * m->np * m->nq;
    red->has_p = true;
    red->p_fp64 = prec == WPCD_FP64;
    red->has_val64 = true;
    red->pred_nnz = -1;
}

wpcd_status wpcd_build_reduced(wpcd_ctx *red, wpcd_ctx *full, int32_t n_major, int32_t r_p,
                               int32_t r_q, wpcd_precision prec, int64_t *nnz_out) {
    return guarded(red, [&] {
        build_reduced(red, full, n_major, r_p, r_q, prec);
        if (nnz_out) *nnz_out = red->nnz;
    });
}

wpcd_status wpcd_build_basis_nucleons(wpcd_ctx *c, const wpcd_basis_desc *b,
                                      const wpcd_potential_desc *pot,
                                      const wpcd_nucleon_desc *nuc) {
    return guarded(c, [&] {
        WPCD_REQUIRE(nuc, WPCD_E_INVALID, "nucleon descriptor is NULL");
        drop_reduction(c);
        build_basis_impl(c, b, pot, nuc);
    });
}

wpcd_status wpcd_set_potential(wpcd_ctx *c, const wpcd_potential_desc *pot) {
    return guarded(c, [&] {
        WPCD_REQUIRE(c->has_basis, WPCD_E_STATE, "wpcd_build_basis must come first");
        WPCD_NOT_REDUCED(c);
        c->has_pot = false;
        build_pair_waves(c, pot);
    });
}

wpcd_status wpcd_pair_spectrum(wpcd_ctx *c, int32_t l, double *eps_out, double *O_out,
                               double *scale_out) {
    return guarded(c, [&] {
        WPCD_REQUIRE(c->has_basis && c->has_pot, WPCD_E_STATE, "no basis/potential");
        int w = -1;
        if (c->nuc_two_S) {
            WPCD_REQUIRE(l >= 0 && l < c->nch, WPCD_E_INVALID, "channel index out of range");
            w = c->ch_wave[l];
        } else {
            for (int k = 0; k < c->n_waves; ++k)
                if (c->waves[k].l == l) w = k;
        }
        WPCD_REQUIRE(w >= 0, WPCD_E_INVALID, "pair wave l not used by the channels");
        const int n = c->np;
        if (eps_out)
            WPCD_HIP(hipMemcpyAsync(eps_out, c->waves[w].eps.ptr, n * sizeof(double),
                                    hipMemcpyDeviceToHost, c->stream));
        if (O_out)
            WPCD_HIP(hipMemcpyAsync(O_out, c->waves[w].O.ptr, (size_t)n * n * sizeof(double),
                                    hipMemcpyDeviceToHost, c->stream));
        WPCD_HIP(hipStreamSynchronize(c->stream));
        if (scale_out) *scale_out = c->pot_scale;
    });
}

wpcd_status wpcd_build_p_noalloc(wpcd_ctx *c, wpcd_precision prec, int64_t *row_ptr,
                                 int32_t *col, void *val, int64_t cap_nnz, int64_t *nnz_out) {
    return guarded(c, [&] {
        WPCD_REQUIRE(c->has_basis, WPCD_E_STATE, "wpcd_build_basis must come first");
        WPCD_NOT_REDUCED(c);
        WPCD_REQUIRE(prec == WPCD_FP64 || prec == WPCD_MIXED, WPCD_E_INVALID, "bad precision");
        WPCD_REQUIRE(row_ptr && col && val && cap_nnz >= 0, WPCD_E_INVALID,
                     "row_ptr, col and val must be device pointers and cap_nnz >= 0");
        unsigned char *base = scratch_of(c->device);
        WPCD_REQUIRE(base, WPCD_E_STATE, "no scratch address for this device");
        // scratch layout: per-tile totals | row counts | row hints | row starts
        const int64_t nrow = (int64_t)c->np * c->nq;
        const int64_t off_cnt = 256 * ((kMaxScanTiles * 8 + 255) / 256);
        const int64_t off_hint = off_cnt + 256 * ((4 * nrow + 255) / 256);
        WPCD_REQUIRE(off_hint <= WPCD_NOALLOC_SCRATCH_BYTES, WPCD_E_INVALID,
                     "grid too large for the fixed scratch");
        // timing events are not created here
        const int timing = c->timer.enabled;
        c->timer.enabled = 0;
        struct Restore {
            wpcd_ctx *c;
            int t;
            ~Restore() { c->timer.enabled = t; }
        } restore{c, timing};
        int32_t *cnt = reinterpret_cast<int32_t *>(base + off_cnt);
        int64_t *tsum = reinterpret_cast<int64_t *>(base);
        const int64_t nnz = structure_rows(c, cnt, row_ptr, tsum);
        if (nnz_out) *nnz_out = nnz;
        const int64_t off_rs = off_hint + 256 * ((4 * hint_len(nnz) + 255) / 256);
        WPCD_REQUIRE(nnz <= cap_nnz, WPCD_E_INVALID,
                     "P0 has " + std::to_string(nnz) + " nonzero cells, cap_nnz is " +
                         std::to_string(cap_nnz));
        WPCD_REQUIRE(off_rs + nnz <= WPCD_NOALLOC_SCRATCH_BYTES, WPCD_E_INVALID,
                     "P0 too large for the fixed scratch (" + std::to_string(nnz) +
                         " nonzero cells)");
        int32_t *hint = reinterpret_cast<int32_t *>(base + off_hint);
        uint8_t *rstart = reinterpret_cast<uint8_t *>(base + off_rs);
        structure_fill(c, cnt, tsum, row_ptr, col, hint, rstart, nnz);
        const bool fp64 = prec == WPCD_FP64;
        values_into(c, fp64, row_ptr, col, hint, rstart, nnz, fp64 ? (double *)val : nullptr,
                    fp64 ? nullptr : (float *)val, false, false);
        WPCD_HIP(hipStreamSynchronize(c->stream));
    });
}

wpcd_status wpcd_model_fill(wpcd_ctx *c, int32_t kind, int32_t mode, int32_t M, int32_t K,
                            double alpha, uint64_t seed, wpcd_precision prec, double *dense_out,
                            int64_t *idx_out, double *val_out, int64_t cap, int64_t *nnz_out,
                            double *ms_out) {
    return guarded(c, [&] {
        WPCD_REQUIRE(kind == 0 || kind == 1, WPCD_E_INVALID, "kind must be 0 (trig) or 1 (Gauss)");
        WPCD_REQUIRE(mode >= 0 && mode <= 2, WPCD_E_INVALID, "mode must be 0, 1 or 2");
        WPCD_REQUIRE(M >= 1 && M <= 8192 && K >= 1 && K <= 4096, WPCD_E_INVALID,
                     "need 1 <= M <= 8192 and 1 <= K <= 4096");
        WPCD_REQUIRE(prec == WPCD_FP64 || prec == WPCD_MIXED, WPCD_E_INVALID,
                     "precision must be WPCD_FP64 or WPCD_MIXED (FP32)");
        WPCD_REQUIRE(mode != 2 || cap >= 0, WPCD_E_INVALID, "cap < 0");
        WPCD_REQUIRE(std::isfinite(alpha), WPCD_E_INVALID, "alpha not finite");
        ModelRequest r{kind, mode, M, K, alpha, seed, prec == WPCD_FP64, dense_out, idx_out, val_out,
                       cap};
        ModelResult res{};
        model_fill(c, r, res);
        if (nnz_out) *nnz_out = res.nnz;
        if (ms_out) *ms_out = res.ms;
        WPCD_REQUIRE(mode != 2 || res.nnz <= cap, WPCD_E_INVALID,
                     "selected elements (" + std::to_string(res.nnz) + ") exceed cap");
    });
}

wpcd_status wpcd_build_p(wpcd_ctx *c, wpcd_precision prec, int64_t *nnz_out) {
    return guarded(c, [&] {
        WPCD_REQUIRE(c->has_basis, WPCD_E_STATE, "wpcd_build_basis must come first");
        WPCD_NOT_REDUCED(c);
        WPCD_REQUIRE(prec == WPCD_FP64 || prec == WPCD_MIXED, WPCD_E_INVALID, "bad precision");
        c->has_p = false;
        c->has_val64 = false;
        if (!c->h_nnz) {
            void *h = nullptr;
            if (hipHostMalloc(&h, sizeof(int64_t)) == hipSuccess) c->h_nnz = (int64_t *)h;
            else (void)hipGetLastError();   // no pinned word: every build waits for its count
        }
        build_structure(c);
        build_values(c, prec == WPCD_FP64);
        structure_count_copy(c);
        WPCD_HIP(hipStreamSynchronize(c->stream));
        if (c->nnz_check && *c->h_nnz != c->nnz) {
            // the count differs from the last build's on the same edges:
            // build again on the waiting path
            c->pred_nnz = -1;
            build_structure(c);
            build_values(c, prec == WPCD_FP64);
            WPCD_HIP(hipStreamSynchronize(c->stream));
        }
        c->nnz_check = false;
        c->pred_nnz = c->nnz;
        c->pred_p = c->p;
        c->pred_q = c->q;
        c->has_p = true;
        c->p_fp64 = prec == WPCD_FP64;
        c->has_val64 = c->p_fp64;
        if (nnz_out) *nnz_out = c->nnz;
    });
}

wpcd_status wpcd_get_p(wpcd_ctx *c, int64_t *row_ptr, int32_t *col, double *val) {
    return guarded(c, [&] {
        WPCD_REQUIRE(c->has_p, WPCD_E_STATE, "no P0 built");
        // a reduced system: one value per entry over its reduced cells
        const int64_t nrow = c->reduced ? c->red_rows : (int64_t)c->np * c->nq;
        const int64_t nv = c->reduced ? c->nnz : c->nnz * c->nch * c->nch;
        if (row_ptr)
            WPCD_HIP(hipMemcpyAsync(row_ptr, c->d_rowptr.ptr, (nrow + 1) * sizeof(int64_t),
                                    hipMemcpyDeviceToHost, c->stream));
        if (col)
            WPCD_HIP(hipMemcpyAsync(col, c->d_col.ptr, c->nnz * sizeof(int32_t),
                                    hipMemcpyDeviceToHost, c->stream));
        if (val) {
            if (c->p_fp64) {
                WPCD_HIP(hipMemcpyAsync(val, c->d_val64.ptr, nv * sizeof(double),
                                        hipMemcpyDeviceToHost, c->stream));
            } else {
                std::vector<float> tmp(nv);
                WPCD_HIP(hipMemcpyAsync(tmp.data(), c->d_val32.ptr, nv * sizeof(float),
                                        hipMemcpyDeviceToHost, c->stream));
                WPCD_HIP(hipStreamSynchronize(c->stream));
                for (int64_t k = 0; k < nv; ++k) val[k] = tmp[k];
            }
        }
        WPCD_HIP(hipStreamSynchronize(c->stream));
    });
}

wpcd_status wpcd_solve(wpcd_ctx *c, const double *E, int32_t n_E, wpcd_precision prec,
                       const wpcd_solve_opts *opts, wpcd_energy_result *out, double *breakup_out) {
    return guarded(c, [&] { solve_impl(c, E, n_E, prec, opts, out, breakup_out, nullptr); });
}

extern "C++" {  // C++ helpers inside the C-linkage block
namespace {
using cd = std::complex<double>;

// Eigenvalues of an n x n upper Hessenberg matrix A (row major) by the
// shifted QR algorithm with Wilkinson shifts and deflation (complex).
std::vector<cd> hessenberg_eigs(std::vector<cd> A, int n) {
    auto at = [&](int i, int j) -> cd & { return A[(size_t)i * n + j]; };
    std::vector<cd> ev;
    int hi = n - 1, iter = 0;
    while (hi >= 0) {
        if (hi == 0) {
            ev.push_back(at(0, 0));
            break;
        }
        int l = hi;
        for (; l > 0; --l) {
            const double sc = std::abs(at(l - 1, l - 1)) + std::abs(at(l, l));
            if (std::abs(at(l, l - 1)) <= 1e-15 * (sc > 0 ? sc : 1.0)) {
                at(l, l - 1) = 0.0;
                break;
            }
        }
        if (l == hi) {
            ev.push_back(at(hi, hi));
            --hi;
            iter = 0;
            continue;
        }
        WPCD_REQUIRE(++iter <= 200, WPCD_E_NOT_CONVERGED, "Hessenberg QR did not converge");
        const cd a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
        const cd tr2 = 0.5 * (a + d), disc = std::sqrt(tr2 * tr2 - (a * d - b * c));
        cd mu = std::abs(tr2 + disc - d) < std::abs(tr2 - disc - d) ? tr2 + disc : tr2 - disc;
        if (iter % 11 == 10) mu += std::abs(at(hi, hi - 1));   // exceptional shift
        for (int k = l; k <= hi; ++k) at(k, k) -= mu;
        std::vector<double> cs;
        std::vector<cd> sn;
        for (int k = l; k < hi; ++k) {
            // G = [[c, s], [-conj(s), c]] with G [x; y] = [r; 0]
            const cd x = at(k, k), y = at(k + 1, k);
            const double r = std::sqrt(std::norm(x) + std::norm(y));
            double cc = 1.0;
            cd ss = 0.0;
            if (r > 0) {
                cc = std::abs(x) / r;
                ss = (std::abs(x) > 0 ? x / std::abs(x) : cd(1.0, 0.0)) * std::conj(y) / r;
            }
            for (int j = k; j < n; ++j) {
                const cd t1 = at(k, j), t2 = at(k + 1, j);
                at(k, j) = cc * t1 + ss * t2;
                at(k + 1, j) = -std::conj(ss) * t1 + cc * t2;
            }
            cs.push_back(cc);
            sn.push_back(ss);
        }
        for (int k = l; k < hi; ++k) {   // times G^H from the right
            const double cc = cs[k - l];
            const cd ss = sn[k - l];
            for (int i = 0; i <= std::min(k + 2, hi); ++i) {
                const cd t1 = at(i, k), t2 = at(i, k + 1);
                at(i, k) = cc * t1 + std::conj(ss) * t2;
                at(i, k + 1) = -ss * t1 + cc * t2;
            }
        }
        for (int k = l; k <= hi; ++k) at(k, k) += mu;
    }
    return ev;
}

// Largest real part of the Ritz values of K(E) from m Arnoldi steps.
double kernel_top_ritz(wpcd_ctx *c, double E, int m) {
    std::vector<double> H;
    int n = 0;
    arnoldi_kernel(c, E, m, H, n);
    WPCD_REQUIRE(n >= 1, WPCD_E_DEVICE, "Arnoldi produced no step");
    std::vector<cd> A((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = cd(H[((size_t)i * m + j) * 2], H[((size_t)i * m + j) * 2 + 1]);
    double best = -1e300;
    for (const cd &v : hessenberg_eigs(A, n)) best = std::max(best, v.real());
    return best;
}
}  // namespace
}  // extern "C++"

wpcd_status wpcd_bound_state(wpcd_ctx *c, double e_lo, double e_hi, double *e3_out) {
    return guarded(c, [&] {
        WPCD_REQUIRE(c->has_basis && c->has_pot && c->has_p, WPCD_E_STATE,
                     "build_basis and build_p must come first");
        WPCD_NOT_REDUCED(c);
        WPCD_REQUIRE(e3_out && std::isfinite(e_lo) && std::isfinite(e_hi) && e_lo < e_hi,
                     WPCD_E_INVALID, "need e_lo < e_hi and e3_out");
        double eb = 1e300;
        for (int a = 0; a < c->nch; ++a) eb = std::min(eb, c->waves[c->ch_wave[a]].h_eps[0]);
        WPCD_REQUIRE(e_hi < eb, WPCD_E_BELOW_THRESHOLD,
                     "the bracket must lie below the lowest pair level");
        const int m = 64;
        double f_lo = kernel_top_ritz(c, e_lo, m) - 1.0, f_hi = kernel_top_ritz(c, e_hi, m) - 1.0;
        WPCD_REQUIRE(f_lo * f_hi <= 0.0, WPCD_E_INVALID,
                     "no sign change of (largest eigenvalue of K) - 1 on the bracket");
        double mid = 0.5 * (e_lo + e_hi);
        for (int it = 0; it < 100 && e_hi - e_lo > 1e-12 * std::fabs(mid); ++it) {
            mid = 0.5 * (e_lo + e_hi);
            const double fm = kernel_top_ritz(c, mid, m) - 1.0;
            if (fm * f_lo > 0) {
                e_lo = mid;
                f_lo = fm;
            } else {
                e_hi = mid;
                f_hi = fm;
            }
        }
        *e3_out = 0.5 * (e_lo + e_hi);
    });
}

wpcd_status wpcd_solve_dev(wpcd_ctx *c, const double *E_dev, int32_t n_E, wpcd_precision prec,
                           const wpcd_solve_opts *opts, wpcd_energy_result *out_dev) {
    return guarded(c, [&] {
        WPCD_REQUIRE(E_dev && out_dev && n_E >= 0, WPCD_E_INVALID, "E_dev/out_dev NULL or n_E < 0");
        std::vector<double> E(n_E);
        std::vector<wpcd_energy_result> out(n_E);
        if (n_E)
            WPCD_HIP(hipMemcpyAsync(E.data(), E_dev, n_E * sizeof(double), hipMemcpyDeviceToHost,
                                    c->stream));
        WPCD_HIP(hipStreamSynchronize(c->stream));
        solve_impl(c, E.data(), n_E, prec, opts, out.data(), nullptr, nullptr);
        if (n_E)
            WPCD_HIP(hipMemcpyAsync(out_dev, out.data(), n_E * sizeof(wpcd_energy_result),
                                    hipMemcpyHostToDevice, c->stream));
        WPCD_HIP(hipStreamSynchronize(c->stream));
    });
}

// ---- P0 file: header (magic, version, grid signature), edges, CSR, values
namespace {
constexpr char kP0Magic[8] = {'W', 'P', 'C', 'D', 'P', '0', '\0', '\1'};

struct P0Header {
    char magic[8];
    int32_t version, np, nq, ngq, ngx, L, nch, fp64;
    int32_t l[kMaxCh], lam[kMaxCh];
    int64_t nnz;
};

P0Header p0_header(const wpcd_ctx *c) {
    P0Header h{};
    std::memcpy(h.magic, kP0Magic, 8);
    h.version = 2;   // 2: no per-nonzero row array
    h.np = c->np;
    h.nq = c->nq;
    h.ngq = c->ngq;
    h.ngx = c->ngx;
    h.L = c->L;
    h.nch = c->nch;
    h.fp64 = c->p_fp64 ? 1 : 0;
    for (int a = 0; a < c->nch; ++a) {
        // nucleon channels are coded as l = 100 + 10 s + t, lam = 100 + 2S
        h.l[a] = c->nuc_two_S ? 100 + 10 * c->ch_s[a] + c->ch_t[a] : c->ch_l[a];
        h.lam[a] = c->nuc_two_S ? 100 + c->nuc_two_S : c->ch_lam[a];
    }
    h.nnz = c->nnz;
    return h;
}

struct File {
    FILE *f;
    explicit File(FILE *f_) : f(f_) {}
    ~File() {
        if (f) std::fclose(f);
    }
};
}  // namespace

wpcd_status wpcd_save_p(wpcd_ctx *c, const char *path) {
    return guarded(c, [&] {
        WPCD_REQUIRE(path, WPCD_E_INVALID, "path is NULL");
        WPCD_REQUIRE(c->has_p, WPCD_E_STATE, "no P0 built");
        WPCD_NOT_REDUCED(c);
        const P0Header h = p0_header(c);
        const int64_t nrow = (int64_t)c->np * c->nq, nv = c->nnz * c->nch * c->nch;
        std::vector<int64_t> rp(nrow + 1);
        std::vector<int32_t> col(c->nnz);
        std::vector<char> val(nv * (c->p_fp64 ? 8 : 4));
        WPCD_HIP(hipMemcpyAsync(rp.data(), c->d_rowptr.ptr, rp.size() * 8, hipMemcpyDeviceToHost, c->stream));
        WPCD_HIP(hipMemcpyAsync(col.data(), c->d_col.ptr, col.size() * 4, hipMemcpyDeviceToHost, c->stream));
        WPCD_HIP(hipMemcpyAsync(val.data(), c->p_fp64 ? (void *)c->d_val64.ptr : (void *)c->d_val32.ptr,
                                val.size(), hipMemcpyDeviceToHost, c->stream));
        WPCD_HIP(hipStreamSynchronize(c->stream));
        File f(std::fopen(path, "wb"));
        WPCD_REQUIRE(f.f, WPCD_E_INVALID, std::string("cannot open for writing: ") + path);
        bool ok = std::fwrite(&h, sizeof h, 1, f.f) == 1 &&
                  std::fwrite(c->p.data(), 8, c->p.size(), f.f) == c->p.size() &&
                  std::fwrite(c->q.data(), 8, c->q.size(), f.f) == c->q.size() &&
                  std::fwrite(rp.data(), 8, rp.size(), f.f) == rp.size() &&
                  std::fwrite(col.data(), 4, col.size(), f.f) == col.size() &&
                  std::fwrite(val.data(), 1, val.size(), f.f) == val.size();
        ok = (std::fclose(f.f) == 0) && ok;
        f.f = nullptr;
        WPCD_REQUIRE(ok, WPCD_E_INVALID, std::string("write failed: ") + path);
    });
}

wpcd_status wpcd_load_p(wpcd_ctx *c, const char *path, int64_t *nnz_out) {
    return guarded(c, [&] {
        WPCD_REQUIRE(path, WPCD_E_INVALID, "path is NULL");
        WPCD_REQUIRE(c->has_basis, WPCD_E_STATE, "wpcd_build_basis must come first");
        WPCD_NOT_REDUCED(c);
        File f(std::fopen(path, "rb"));
        WPCD_REQUIRE(f.f, WPCD_E_INVALID, std::string("cannot open: ") + path);
        P0Header h{};
        WPCD_REQUIRE(std::fread(&h, sizeof h, 1, f.f) == 1 && std::memcmp(h.magic, kP0Magic, 8) == 0 &&
                         h.version == 2,
                     WPCD_E_INVALID, "not a P0 file of this library");
        P0Header mine = p0_header(c);
        bool same = h.np == mine.np && h.nq == mine.nq && h.ngq == mine.ngq && h.ngx == mine.ngx &&
                    h.L == mine.L && h.nch == mine.nch;
        for (int a = 0; same && a < h.nch; ++a) same = h.l[a] == mine.l[a] && h.lam[a] == mine.lam[a];
        WPCD_REQUIRE(same, WPCD_E_INVALID, "P0 file was built for another basis");
        std::vector<double> p(c->p.size()), q(c->q.size());
        WPCD_REQUIRE(std::fread(p.data(), 8, p.size(), f.f) == p.size() &&
                         std::fread(q.data(), 8, q.size(), f.f) == q.size() && p == c->p && q == c->q,
                     WPCD_E_INVALID, "P0 file was built on other bin edges");
        WPCD_REQUIRE(h.nnz >= 0 && h.nnz < ((int64_t)1 << 40), WPCD_E_INVALID, "bad nonzero count");
        const int64_t nrow = (int64_t)c->np * c->nq, nv = h.nnz * c->nch * c->nch;
        std::vector<int64_t> rp(nrow + 1);
        std::vector<int32_t> col(h.nnz);
        std::vector<char> val(nv * (h.fp64 ? 8 : 4));
        WPCD_REQUIRE(std::fread(rp.data(), 8, rp.size(), f.f) == rp.size() &&
                         std::fread(col.data(), 4, col.size(), f.f) == col.size() &&
                         std::fread(val.data(), 1, val.size(), f.f) == val.size(),
                     WPCD_E_INVALID, "P0 file is truncated");
        WPCD_REQUIRE(rp[0] == 0 && rp[nrow] == h.nnz, WPCD_E_INVALID, "P0 file: inconsistent row pointers");
        for (int64_t r = 0; r < nrow; ++r)
            WPCD_REQUIRE(rp[r] <= rp[r + 1], WPCD_E_INVALID, "P0 file: row pointers not monotone");
        for (int64_t k = 0; k < h.nnz; ++k)
            WPCD_REQUIRE(col[k] >= 0 && col[k] < nrow, WPCD_E_INVALID,
                         "P0 file: index out of range");
        c->has_p = false;
        // row hints of the element kernels: the row of every 64th nonzero
        std::vector<int32_t> hint(wpcd::hint_len(h.nnz), 0);
        std::vector<uint8_t> rstart(h.nnz, 0);
        for (int64_t r = 0; r < nrow; ++r) {
            if (rp[r] < rp[r + 1]) rstart[rp[r]] = (r > 0 && rp[r - 1] == rp[r]) ? 2 : 1;
            for (int64_t e = (rp[r] + 63) / 64 * 64; e < rp[r + 1]; e += 64) hint[e / 64] = (int32_t)r;
        }
        c->d_rowptr.reserve(nrow + 1);
        c->d_col.reserve(h.nnz);
        c->d_hint.reserve(hint.size());
        c->d_rstart.reserve(h.nnz);
        WPCD_HIP(hipMemcpyAsync(c->d_hint.ptr, hint.data(), hint.size() * 4, hipMemcpyHostToDevice, c->stream));
        WPCD_HIP(hipMemcpyAsync(c->d_rstart.ptr, rstart.data(), rstart.size(), hipMemcpyHostToDevice, c->stream));
        WPCD_HIP(hipMemcpyAsync(c->d_rowptr.ptr, rp.data(), rp.size() * 8, hipMemcpyHostToDevice, c->stream));
        WPCD_HIP(hipMemcpyAsync(c->d_col.ptr, col.data(), col.size() * 4, hipMemcpyHostToDevice, c->stream));
        if (h.fp64) {
            c->d_val64.reserve(nv);
            WPCD_HIP(hipMemcpyAsync(c->d_val64.ptr, val.data(), val.size(), hipMemcpyHostToDevice, c->stream));
        } else {
            c->d_val32.reserve(nv);
            WPCD_HIP(hipMemcpyAsync(c->d_val32.ptr, val.data(), val.size(), hipMemcpyHostToDevice, c->stream));
        }
        WPCD_HIP(hipStreamSynchronize(c->stream));
        c->nnz = h.nnz;
        c->p_fp64 = h.fp64 != 0;
        c->has_val64 = c->p_fp64;
        c->has_p = true;
        if (nnz_out) *nnz_out = h.nnz;
    });
}

// ---- energy sweep with a journal of completed batches
extern "C++" {
namespace {
constexpr char kSweepMagic[8] = {'W', 'P', 'C', 'D', 'S', 'W', 'P', '\1'};

struct SweepHeader {
    char magic[8];
    int32_t version, n_E, batch, prec;
    uint64_t fingerprint;
};

struct SweepRecord {
    int32_t index, count;
    uint64_t check;   // FNV-1a of the record's results
};

// 64-bit FNV-1a (offset basis and prime as published for the hash).
struct Fnv {
    uint64_t h = 14695981039346656037ull;
    void bytes(const void *p, size_t n) {
        const unsigned char *b = static_cast<const unsigned char *>(p);
        for (size_t k = 0; k < n; ++k) {
            h ^= b[k];
            h *= 1099511628211ull;
        }
    }
    template <class T>
    void val(T v) {
        bytes(&v, sizeof v);
    }
    template <class T>
    void vec(const std::vector<T> &v) {
        val<uint64_t>(v.size());
        bytes(v.data(), v.size() * sizeof(T));
    }
};

// What fixes the results of a sweep: the basis (grid, channels, edges, the
// reduction), the P0 build (its precision and size), the potential with its
// multipliers, the solve options, the learned model's shape and scalings
// when it proposes the start, and the energies.
uint64_t sweep_fingerprint(const wpcd_ctx *c, wpcd_precision prec, const wpcd_solve_opts &o,
                           const double *E, int n_E, int batch) {
    Fnv f;
    for (const wpcd_ctx *x : {c, (const wpcd_ctx *)c->minor}) {
        if (!x) continue;
        const P0Header h = p0_header(x);
        for (int32_t v : {h.np, h.nq, h.ngq, h.ngx, h.L, h.nch}) f.val(v);
        for (int a = 0; a < h.nch; ++a) {
            f.val(h.l[a]);
            f.val(h.lam[a]);
        }
        f.vec(x->p);
        f.vec(x->q);
    }
    f.val<int32_t>(c->p_fp64);
    f.val(c->nnz);
    f.val<int32_t>(c->reduced);
    f.val(c->red_cp);
    f.val(c->red_cq);
    f.val(c->pot_kind);
    f.vec(c->pot_s);
    f.vec(c->pot_mu);
    f.val(c->pot_scale);
    f.val(c->n_waves);
    for (int w = 0; w < c->n_waves; ++w) {   // per-wave strength multipliers (nucleons)
        f.val(c->waves[w].l);
        f.vec(c->waves[w].mult);
    }
    f.val<int32_t>(prec);
    for (int32_t v : {o.max_iter, o.krylov_dim, o.warm_start, o.err_est, o.resolvent}) f.val(v);
    f.val(o.tol);
    f.val(o.fallback_tol);
    if (o.warm_start == WPCD_WARM_LEARNED) {
        const wpcd::Learned &l = c->learned;
        f.val<int32_t>(l.ready);
        f.val(l.K);
        f.val(l.nfeat);
        f.val(l.M);
        f.bytes(l.feat_mu, sizeof l.feat_mu);
        f.bytes(l.feat_sd, sizeof l.feat_sd);
        f.val(l.coef_scale);
    }
    f.val(n_E);
    f.val(batch);
    f.bytes(E, (size_t)n_E * sizeof(double));
    return f.h;
}

uint64_t record_check(const wpcd_energy_result *r, int n) {
    Fnv f;
    f.bytes(r, (size_t)n * sizeof *r);
    return f.h;
}

bool write_all(FILE *f, const void *p, size_t n) { return n == 0 || std::fwrite(p, 1, n, f) == n; }

bool read_all(FILE *f, void *p, size_t n) { return n == 0 || std::fread(p, 1, n, f) == n; }

// Data of the journal on disk before the call returns.
bool flush_to_disk(FILE *f) { return std::fflush(f) == 0 && fsync(fileno(f)) == 0; }
}  // namespace
}  // extern "C++"

wpcd_status wpcd_sweep(wpcd_ctx *c, const double *E, int32_t n_E, int32_t batch,
                       wpcd_precision prec, const wpcd_solve_opts *opts, const char *journal,
                       int32_t max_batches, wpcd_energy_result *out, int32_t *n_done_out,
                       int32_t *n_resumed_out) {
    return guarded(c, [&] {
        WPCD_REQUIRE(E && out && n_E >= 0 && batch >= 1, WPCD_E_INVALID,
                     "E/out NULL, n_E < 0 or batch < 1");
        batch = std::min(batch, std::max(n_E, 1));
        wpcd_solve_opts o{};
        if (opts) o = *opts;
        WPCD_REQUIRE(o.warm_start != WPCD_WARM_GIVEN && !o.x0, WPCD_E_INVALID,
                     "a sweep takes no caller-given start vector");
        o.want_breakup = 0;
        o.x0 = nullptr;
        const int nb = (n_E + batch - 1) / batch;
        auto count_of = [&](int b) { return std::min(batch, n_E - b * batch); };
        int done = 0;   // batches complete (from the journal, then solved here)
        File f(nullptr);
        if (journal) {
            SweepHeader h{};
            std::memcpy(h.magic, kSweepMagic, 8);
            h.version = 1;
            h.n_E = n_E;
            h.batch = batch;
            h.prec = prec;
            h.fingerprint = sweep_fingerprint(c, prec, o, E, n_E, batch);
            errno = 0;
            f.f = std::fopen(journal, "r+b");
            // only a missing file is created (one that cannot be opened for
            // reading and writing is not replaced)
            WPCD_REQUIRE(f.f || errno == ENOENT, WPCD_E_INVALID,
                         std::string("cannot open journal: ") + journal);
            SweepHeader g{};
            const bool fresh = !f.f || std::fread(&g, 1, sizeof g, f.f) == 0;
            if (fresh) {   // a new journal (or an empty file)
                if (f.f) std::fclose(f.f);
                f.f = std::fopen(journal, "w+b");
                WPCD_REQUIRE(f.f, WPCD_E_INVALID, std::string("cannot create journal: ") + journal);
                WPCD_REQUIRE(write_all(f.f, &h, sizeof h) &&
                                 write_all(f.f, E, (size_t)n_E * sizeof(double)) && flush_to_disk(f.f),
                             WPCD_E_INVALID, std::string("journal write failed: ") + journal);
            } else {
                WPCD_REQUIRE(std::memcmp(g.magic, kSweepMagic, 8) == 0 && g.version == 1,
                             WPCD_E_INVALID, "not a sweep journal of this library");
                std::vector<double> Ej(n_E);
                WPCD_REQUIRE(g.n_E == n_E && g.batch == batch && g.prec == prec &&
                                 g.fingerprint == h.fingerprint &&
                                 read_all(f.f, Ej.data(), Ej.size() * sizeof(double)) &&
                                 std::memcmp(Ej.data(), E, Ej.size() * sizeof(double)) == 0,
                             WPCD_E_INVALID,
                             "the journal belongs to another sweep (energies, batch, precision, "
                             "basis, potential or options differ)");
                long good = std::ftell(f.f);
                // complete records in batch order; a torn or damaged tail
                // (an interrupted write) ends the replay and is cut off
                while (done < nb) {
                    SweepRecord r{};
                    const int n = count_of(done);
                    wpcd_energy_result *dst = out + (size_t)done * batch;
                    if (!read_all(f.f, &r, sizeof r) || r.index != done || r.count != n ||
                        !read_all(f.f, dst, (size_t)n * sizeof *dst) || record_check(dst, n) != r.check)
                        break;
                    ++done;
                    good = std::ftell(f.f);
                }
                WPCD_REQUIRE(good >= 0 && std::fflush(f.f) == 0 && ftruncate(fileno(f.f), good) == 0 &&
                                 std::fseek(f.f, good, SEEK_SET) == 0,
                             WPCD_E_INVALID, std::string("cannot trim journal: ") + journal);
            }
        }
        const int resumed = done;
        const int stop = max_batches > 0 ? std::min(nb, done + max_batches) : nb;
        for (; done < stop; ++done) {
            const int n = count_of(done);
            wpcd_energy_result *dst = out + (size_t)done * batch;
            solve_impl(c, E + (size_t)done * batch, n, prec, &o, dst, nullptr, nullptr);
            if (f.f) {
                const SweepRecord r{done, n, record_check(dst, n)};
                WPCD_REQUIRE(write_all(f.f, &r, sizeof r) && write_all(f.f, dst, (size_t)n * sizeof *dst) &&
                                 flush_to_disk(f.f),
                             WPCD_E_INVALID, std::string("journal write failed: ") + journal);
            }
        }
        const int n_done = std::min(n_E, done * batch);
        for (int k = n_done; k < n_E; ++k) {   // not reached in this call
            out[k] = wpcd_energy_result{};
            out[k].E = E[k];
            out[k].status = WPCD_E_STATE;
        }
        if (n_done_out) *n_done_out = n_done;
        if (n_resumed_out) *n_resumed_out = std::min(n_E, resumed * batch);
    });
}

wpcd_status wpcd_solve_multi(wpcd_ctx *const *ctxs, int32_t n_sys, const double *const *E,
                             const int32_t *n_E, wpcd_precision prec, const wpcd_solve_opts *opts,
                             wpcd_energy_result *const *out, wpcd_status *status_out) {
    if (!ctxs || !E || !n_E || !out || n_sys < 0) return WPCD_E_INVALID;
    // one opts for systems of different sizes: a caller-given x0 cannot fit them all
    if (opts && opts->warm_start == WPCD_WARM_GIVEN) return WPCD_E_INVALID;
    for (int i = 0; i < n_sys; ++i) {
        if (!ctxs[i]) return WPCD_E_INVALID;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return WPCD_E_INVALID;   // a context is not thread-safe
    }
    std::vector<wpcd_status> st(n_sys, WPCD_OK);
    bool one_device = true;
    for (int i = 1; i < n_sys; ++i) one_device &= ctxs[i]->device == ctxs[0]->device;
    if (!one_device) {
        // systems on several devices: one host thread per system
        std::vector<std::thread> th;
        th.reserve(n_sys);
        for (int i = 0; i < n_sys; ++i)
            th.emplace_back([&, i] { st[i] = wpcd_solve(ctxs[i], E[i], n_E[i], prec, opts, out[i], nullptr); });
        for (auto &t : th) t.join();
    } else {
        // one device: the systems' batches iterate in lockstep, and each group
        // of iterations of all of them is one captured graph (gmres_cycles)
        std::vector<SolveJob> jobs(n_sys);
        auto step = [&](int i, auto &&f) {
            if (st[i] != WPCD_OK) return;
            const wpcd_status r = guarded(ctxs[i], f);
            st[i] = r;
        };
        for (int i = 0; i < n_sys; ++i) {
            SolveJob &j = jobs[i];
            j.c = ctxs[i];
            j.E = E[i];
            j.n_E = n_E[i];
            j.prec = prec;
            j.opts = opts;
            j.out = out[i];
            step(i, [&] { j.plan(); });
        }
        size_t nbt = 0;
        for (int i = 0; i < n_sys; ++i)
            if (st[i] == WPCD_OK) nbt = std::max(nbt, jobs[i].n_batches());
        for (size_t t = 0; t < nbt; ++t) {
            std::vector<GmresRun *> runs;
            std::vector<int> who;
            for (int i = 0; i < n_sys; ++i) {
                if (st[i] != WPCD_OK || t >= jobs[i].n_batches()) continue;
                step(i, [&] { jobs[i].begin_batch(t); });
                if (st[i] != WPCD_OK) continue;
                runs.push_back(jobs[i].run.get());
                who.push_back(i);
            }
            if (runs.empty()) continue;
            const wpcd_status r = guarded(ctxs[who[0]], [&] { gmres_cycles(runs); });
            if (r != WPCD_OK)
                for (int i : who) {
                    st[i] = r;
                    ctxs[i]->err = ctxs[who[0]]->err;
                }
            for (int i : who) step(i, [&] { jobs[i].end_batch(); });
        }
        for (int i = 0; i < n_sys; ++i) step(i, [&] { jobs[i].finish(); });
    }
    wpcd_status first = WPCD_OK;
    for (int i = 0; i < n_sys; ++i) {
        if (status_out) status_out[i] = st[i];
        if (first == WPCD_OK) first = st[i];
    }
    return first;
}

wpcd_status wpcd_set_multipliers(wpcd_ctx *c, const double *mult, int32_t n_mult) {
    return guarded(c, [&] {
        WPCD_REQUIRE(c->has_basis && c->has_pot, WPCD_E_STATE, "no basis/potential");
        WPCD_NOT_REDUCED(c);
        set_multipliers(c, mult, n_mult);
    });
}

wpcd_status wpcd_learn_train(wpcd_ctx *c, const wpcd_learn_desc *desc, wpcd_learn_report *report) {
    return guarded(c, [&] {
        WPCD_NOT_REDUCED(c);
        learn_train(c, desc, report);
    });
}

wpcd_status wpcd_mlp_eval(wpcd_ctx *c, int32_t n_in, int32_t n_hidden, int32_t n_out,
                          const float *params, int32_t batch, const float *X, const float *T,
                          float *Y_out, float *grad_out, double *loss_out) {
    return guarded(c, [&] { mlp_eval(c, n_in, n_hidden, n_out, params, batch, X, T, Y_out, grad_out, loss_out); });
}

wpcd_status wpcd_set_autotune(wpcd_ctx *c, int32_t mode) {
    return guarded(c, [&] {
        WPCD_REQUIRE(mode == WPCD_TUNE_HEURISTIC || mode == WPCD_TUNE_MEASURE ||
                         (mode >= WPCD_TUNE_FORCE && mode < WPCD_TUNE_FORCE + 64),
                     WPCD_E_INVALID, "unknown autotune mode");
        c->tune.mode = mode;
        c->tune.entries.clear();
    });
}

wpcd_status wpcd_get_autotune(wpcd_ctx *c, wpcd_tune_entry *out, int32_t n, int32_t *n_out) {
    return guarded(c, [&] {
        const int cnt = (int)c->tune.entries.size();
        for (int k = 0; k < cnt && k < n && out; ++k) {
            const auto &e = c->tune.entries[k];
            std::memset(&out[k], 0, sizeof(out[k]));
            std::snprintf(out[k].name, sizeof(out[k].name), "%s", e.name.c_str());
            std::snprintf(out[k].key, sizeof(out[k].key), "%s", e.key.c_str());
            out[k].choice = e.choice;
            out[k].n_candidates = e.n_cand;
            out[k].us = e.us;
        }
        if (n_out) *n_out = cnt;
    });
}

wpcd_status wpcd_set_graphs(wpcd_ctx *c, int32_t enable) {
    return guarded(c, [&] {
        WPCD_HIP(hipStreamSynchronize(c->stream));
        c->use_graphs = enable != 0;
        for (auto &g : c->graphs) g.release();
        c->graphs.clear();
        for (auto &g : c->multi_graphs) (void)hipGraphExecDestroy(g.exec);
        c->multi_graphs.clear();
    });
}

wpcd_status wpcd_set_timing(wpcd_ctx *c, int32_t enable) {
    return guarded(c, [&] {
        c->timer.collect();
        c->timer.enabled = enable;
    });
}

wpcd_status wpcd_get_timing(wpcd_ctx *c, wpcd_kernel_time *out, int32_t n, int32_t *n_out) {
    return guarded(c, [&] {
        c->timer.collect();
        const int cnt = (int)c->timer.names.size();
        for (int k = 0; k < cnt && k < n; ++k) {
            std::memset(&out[k], 0, sizeof(out[k]));
            std::snprintf(out[k].name, sizeof(out[k].name), "%s", c->timer.names[k].c_str());
            out[k].total_ms = c->timer.total_ms[k];
            out[k].launches = c->timer.launches[k];
        }
        if (n_out) *n_out = cnt;
    });
}

wpcd_status wpcd_reset_timing(wpcd_ctx *c) {
    return guarded(c, [&] { c->timer.reset(); });
}

wpcd_status wpcd_synchronize(wpcd_ctx *c) {
    return guarded(c, [&] { WPCD_HIP(hipStreamSynchronize(c->stream)); });
}

const char *wpcd_last_error(const wpcd_ctx *c) {
    if (!c) return "null context";
    return c->err.c_str();
}

static void release_all(wpcd_ctx *c) {
    if (c->minor) {
        release_all(c->minor);
        delete c->minor;
        c->minor = nullptr;
    }
    if (c->h_nnz) (void)hipHostFree(c->h_nnz);
    c->h_nnz = nullptr;
    c->timer.release();
    c->d_p.release();
    c->d_q.release();
    c->d_P2.release();
    c->d_Q34.release();
    c->d_H.release();
    c->d_rsd_p.release();
    c->d_rsd_q.release();
    c->d_qnode.release();
    c->d_qwt.release();
    c->d_ux.release();
    c->d_wx.release();
    c->d_uxf.release();
    c->d_wxf.release();
    for (auto &w : c->waves) {
        w.v.release();
        w.O.release();
        w.eps.release();
        w.Vt.release();
    }
    c->d_rowptr.release();
    c->d_col.release();
    c->d_cnt.release();
    c->d_hint.release();
    c->d_rstart.release();
    c->d_perm.release();
    c->d_nuc64.release();
    c->d_nuc32.release();
    c->d_tsum.release();
    c->d_val64.release();
    c->d_val32.release();
    c->d_G.release();
    c->d_X.release();
    c->d_B.release();
    c->d_W.release();
    c->d_T1.release();
    c->d_T2.release();
    c->d_V.release();
    c->d_Hess.release();
    c->d_partial.release();
    c->d_misc.release();
    c->d_idx.release();
    c->d_jac.release();
    c->d_flag.release();
    c->learned.release();
    for (auto &g : c->graphs) g.release();
    c->graphs.clear();
    for (auto &g : c->multi_graphs) (void)hipGraphExecDestroy(g.exec);
    c->multi_graphs.clear();
    c->d_pot.release();
    c->d_mcoef.release();
    c->d_mterms.release();
    c->d_mterm_first.release();
}

void wpcd_destroy(wpcd_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    release_all(c);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"
