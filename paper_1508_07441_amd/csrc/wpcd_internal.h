// Internal declarations of libwpcd (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/wpcd.h"

namespace wpcd {

constexpr int kMaxCh = 8;
constexpr int kMaxWaves = 3;      // distinct even pair waves l = 0, 2, 4
constexpr int kMaxGq = 16;
constexpr int kMaxGx = 64;
constexpr int kMaxLam = 4;

struct Error {
    wpcd_status code;
    std::string msg;
};

#define WPCD_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            throw ::wpcd::Error{WPCD_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define WPCD_REQUIRE(cond, code, msg)                                                    \
    do {                                                                                 \
        if (!(cond)) throw ::wpcd::Error{(code), (msg)};                                 \
    } while (0)

// Device buffer that grows on demand and is freed with the context.
template <class T>
struct DBuf {
    T *ptr = nullptr;
    size_t cap = 0;
    void reserve(size_t n) {
        if (n <= cap) return;
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        cap = 0;
        hipError_t e = hipMalloc(&ptr, sizeof(T) * (n ? n : 1));
        if (e != hipSuccess) {
            ptr = nullptr;
            throw Error{WPCD_E_NOMEM, "hipMalloc of " + std::to_string(sizeof(T) * n) + " bytes failed"};
        }
        cap = n;
    }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        cap = 0;
    }
};

struct Timer {
    struct Pending {
        int id;
        hipEvent_t a, b;
    };
    int enabled = 0;   // bit mask of WPCD_TIME_* groups
    std::vector<std::string> names;
    std::vector<double> total_ms;
    std::vector<int64_t> launches;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    int id_of(const char *name);
    hipEvent_t get();
    void begin(hipStream_t s, const char *name, Pending &p);
    void end(hipStream_t s, Pending &p);
    void collect();
    void reset();
    void release();
};

// Scope guard that brackets one kernel launch with timing events.
struct TimedLaunch {
    Timer &t;
    hipStream_t s;
    Timer::Pending p{};
    bool on;
    TimedLaunch(Timer &t_, hipStream_t s_, const char *name, int group)
        : t(t_), s(s_), on((t_.enabled & group) != 0) {
        if (on) t.begin(s, name, p);
    }
    ~TimedLaunch() {
        if (on) t.end(s, p);
    }
};

// Coupling polynomial of one channel pair: degree d = (l+lam+l'+lam')/2,
// half powers of the divisor t^(l/2) u^(l'/2) (q^2)^(lam/2) (q'^2)^(lam'/2),
// offset of its coefficients (c major, then a) in the coefficient table.
struct McPair {
    int d, hl, hl2, hlam, hlam2, off;
};

// One term of the direct angular coupling: coef times the associated
// Legendre values with table indices i = l (l + 1)/2 + |m| at the polar
// cosines of pi1 (i1), of q (iq) and of pi2 (i2).
struct McTerm {
    double coef;
    int i1, iq, i2, pad;
};

struct PairWave {
    int l = 0;
    std::vector<double> mult;     // per-term strength multipliers of this wave (empty: 1)
    DBuf<double> v, O, eps, Vt;   // v, O (rows eigenvectors), eps* ascending, Vt = v O^T
    std::vector<double> h_eps;    // host copy of eps*
};

// Multilayer perceptron x -> tanh(W1 x + b1) -> tanh(W2 . + b2) ->
// tanh(W3 . + b3) -> W4 . + b4.  FP32 master parameters [W1 b1 .. W4 b4]
// (W row-major out x in), BF16 copies of the weights for the products.
struct Mlp {
    int nin = 0, nh = 0, nout = 0;
    int step = 0;
    bool ready = false;
    int din(int l) const { return l == 0 ? nin : nh; }
    int dout(int l) const { return l == 3 ? nout : nh; }
    int64_t n_params() const;
    int64_t w_off(int l) const;
    DBuf<float> w32, am, av, grad, act, dact, rowloss;
    DBuf<uint16_t> w16;
    void release() {
        w32.release();
        am.release();
        av.release();
        grad.release();
        act.release();
        dact.release();
        rowloss.release();
        w16.release();
        ready = false;
    }
};

// Learned warm start: reduced basis Phi (K orthonormal complex FP32 vectors
// of length M, [K][M][2]) and the network mapping normalised features to
// coefficients in Phi (scaled by 1/coef_scale).
constexpr int kMaxFeat = 5 + 16;
struct Learned {
    bool ready = false;
    int K = 0, nfeat = 0, n_mult = 0;
    int64_t M = 0;
    double feat_mu[kMaxFeat] = {}, feat_sd[kMaxFeat] = {};
    double coef_scale = 1.0;
    DBuf<float> phi;
    Mlp mlp;
    DBuf<float> feat, y;   // inference scratch
    DBuf<int32_t> sel;     // snapshot selection list
    void release() {
        phi.release();
        mlp.release();
        feat.release();
        y.release();
        sel.release();
        ready = false;
    }
};

// Launch-shape decisions of the context, keyed by kernel family and
// problem shape (see wpcd_set_autotune).
struct Tuning {
    int mode = 0;
    struct Entry {
        std::string name, key;
        int choice, n_cand;
        double us;   // measured time of the choice (0: heuristic or forced)
    };
    std::vector<Entry> entries;
};

// Executable graphs of the GMRES iteration groups of one batch shape.
// Graph of one group of iterations of several batches (key: the batches'
// graph keys and the group's first iteration).
struct MultiGraph {
    std::vector<uint64_t> key;
    hipGraphExec_t exec;
};

struct IterGraphs {
    std::vector<uint64_t> key;
    std::vector<hipGraphExec_t> exec;
    void release() {
        for (auto &e : exec)
            if (e) (void)hipGraphExecDestroy(e);
        exec.clear();
    }
};

}  // namespace wpcd

struct wpcd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    wpcd::Timer timer;

    // ---- basis
    bool has_basis = false;
    int np = 0, nq = 0, ngq = 0, ngx = 0, L = 0, nch = 0;
    int ch_l[wpcd::kMaxCh] = {}, ch_lam[wpcd::kMaxCh] = {};
    // three nucleons in pair s-waves: 2S (1 or 3; 0 for bosons), the pair
    // spin and isospin of each channel, and the coefficients g_ab
    int nuc_two_S = 0;
    int ch_s[wpcd::kMaxCh] = {}, ch_t[wpcd::kMaxCh] = {};
    std::vector<double> nuc_g;
    wpcd::DBuf<double> d_nuc64;          // s-wave values before the channel spread
    wpcd::DBuf<float> d_nuc32;
    int ch_wave[wpcd::kMaxCh] = {};     // channel -> index into waves
    std::vector<double> p, q;           // host edges
    std::vector<double> gq, wq, gx, wx; // host Gauss tables on [-1, 1]
    wpcd::DBuf<double> d_p, d_q, d_P2, d_Q34, d_H, d_rsd_p, d_rsd_q;
    wpcd::DBuf<double> d_qnode, d_qwt, d_ux, d_wx;
    wpcd::DBuf<float> d_uxf, d_wxf;

    bool swave = true;                  // single (0,0) channel with L = 0: G = 1
    std::vector<wpcd::McPair> mc_pairs; // coupling polynomials per channel pair
    int mc_deg = 0;                     // largest d over the pairs
    wpcd::DBuf<double> d_mcoef;
    wpcd::DBuf<wpcd::McTerm> d_mterms;  // direct coupling terms
    wpcd::DBuf<int> d_mterm_first;      // first term of each channel pair [NP + 1]
    bool mc_direct = false;             // general channel sets: direct evaluation

    // ---- potential / pair waves
    bool has_pot = false;
    int pot_kind = 0;
    std::vector<double> pot_s, pot_mu;
    wpcd::DBuf<double> d_pot;           // strengths [16] | ranges [16]
    double pot_scale = 1.0;
    std::vector<double> pot_base;       // strengths as given; pot_s = pot_base * mult
    std::vector<double> pot_mult;
    int n_waves = 0;
    wpcd::PairWave waves[wpcd::kMaxWaves];

    // ---- P0
    bool has_p = false;
    bool p_fp64 = false;     // P0 built in FP64 (else FP32 values in d_val32)
    bool has_val64 = false;  // d_val64 holds the FP64 values of the current structure
    int64_t nnz = 0;
    // the nonzero count of the last completed build and its bin edges (the
    // structure depends on them alone); h_nnz: pinned word the deferred
    // count is copied to; nnz_check: this build's count awaits that check
    int64_t pred_nnz = -1;
    std::vector<double> pred_p, pred_q;
    int64_t *h_nnz = nullptr;
    bool nnz_check = false;
    wpcd::DBuf<int64_t> d_rowptr;
    wpcd::DBuf<int32_t> d_col, d_cnt, d_hint;   // columns, row counts, row hints (one per 64 nonzeros)
    wpcd::DBuf<int64_t> d_tsum;                  // pre-selection scan: per-tile totals
    wpcd::DBuf<uint8_t> d_rstart;                // 1 where a nonzero starts its row
    wpcd::DBuf<int32_t> d_perm;                  // SpMM row order in lattice tiles
    int perm_np = 0, perm_nq = 0;                // grid d_perm was built for
    int perm_rows = 0;                           // rows it orders (reduced cells for a reduced system)
    int64_t perm_nnz = -1;                       // nonzero count it was balanced for
    int perm_grid = 0;                           // workgroups of a tiled SpMM launch
    wpcd::DBuf<double> d_val64;
    wpcd::DBuf<float> d_val32;

    // ---- solve workspace
    wpcd::DBuf<double> d_G, d_X, d_X2, d_B, d_W, d_T1, d_T2, d_V, d_Hess, d_partial, d_misc;
    wpcd::DBuf<int64_t> d_idx;
    wpcd::DBuf<double> d_jac;   // Jacobi workspace (A and V per wave)
    wpcd::DBuf<int32_t> d_flag;

    // ---- learned warm start
    wpcd::Learned learned;

    // ---- Feshbach reduction: this context is a reduced system whose major
    // channels are its own channels (fine lattice) and whose minor channels
    // live in `minor` (coarse lattice, every red_cp-th p edge and red_cq-th
    // q edge, the same potential; owned, on this context's stream).  Its P0
    // (d_rowptr, d_col, d_val64 and, for a mixed build, d_val32) is one
    // scalar CSR over the red_rows reduced cells.
    bool reduced = false;
    wpcd_ctx *minor = nullptr;
    int red_cp = 1, red_cq = 1;
    int64_t red_rows = 0;

    // ---- launch-shape autotuning, captured iteration graphs
    wpcd::Tuning tune;
    bool use_graphs = true;
    std::vector<wpcd::IterGraphs> graphs;
    std::vector<wpcd::MultiGraph> multi_graphs;   // lockstep groups led by this context
};

namespace wpcd {

// Gauss-Legendre nodes (ascending) and weights on [-1, 1] by the Golub-Welsch
// eigenvalue method, polished by Newton steps in long double (host).
void gauss_legendre_gw(int n, std::vector<double> &x, std::vector<double> &w);

// Coupling polynomial coefficients for all channel pairs (host, long double fit).
void coupling_tables(int L, int nch, const int *l, const int *lam, std::vector<McPair> &pairs,
                     std::vector<double> &coef);
void coupling_terms(int L, int nch, const int *l, const int *lam, std::vector<McTerm> &terms,
                    std::vector<int> &first);
// Three nucleons in pair s-waves: the spin-isospin coefficients g_ab of the
// permutation kernel (row-major nch x nch) and their degree-0 coupling
// tables for the multichannel element kernels.
void nucleon_tables(int two_S, int nch, const int *s, const int *t, std::vector<McPair> &pairs,
                    std::vector<double> &coef, std::vector<double> &g);

// ---- kernel launchers (defined in the .hip files)
void launch_potential(wpcd_ctx *c, int wave, double *v_out);
void pair_diagonalise(wpcd_ctx *c, int wave, bool want_vectors);
void launch_vt(wpcd_ctx *c, int wave);

// Model matrix fills of Sec. IV.A (k_model.hip).
struct ModelRequest {
    int kind, mode, M, K;   // kind 0 eq.(Atrig), 1 eq.(Agau); mode 0 dense, 1 filtered, 2 selected
    double alpha;
    uint64_t seed;
    bool fp64;
    double *dense_out;      // host [M*M] (modes 0, 1) or NULL
    int64_t *idx_out;       // host [cap] (mode 2) or NULL
    double *val_out;        // host [cap] (mode 2) or NULL
    int64_t cap;
};
struct ModelResult {
    int64_t nnz;
    double ms;
};
void model_fill(wpcd_ctx *c, const ModelRequest &r, ModelResult &res);

void build_structure(wpcd_ctx *c);   // a3: counts, scan, fill (sets c->nnz)
// Feshbach reduction (k_reduce.hip): the reduced P0 of `red` (major
// channels [0, nmaj) of `full` on its lattice, the rest on the lattice
// coarsened by cp x cq) from full's structure and FP64 values d_val64, into
// red->d_rowptr, d_col, d_val64 (and d_val32 with keep32); sets red->nnz.
void reduce_p0(wpcd_ctx *full, wpcd_ctx *red, int nmaj, int cp, int cq, const double *d_val64,
               bool keep32);
void build_values(wpcd_ctx *c, bool fp64);
// The same into given device buffers: row counts cnt[n_p n_q] and row_ptr
// [n_p n_q + 1] (returns nnz), columns col[nnz], values val64 or val32
// [nnz][n_ch][n_ch].
// Row counts cnt[n_p n_q], row_ptr[n_p n_q + 1], per-tile totals
// tsum[kMaxScanTiles]; returns nnz.  The fill then writes col[nnz], the
// final row_ptr and the row lookup tables of the element kernels,
// hint[hint_len(nnz)] and rstart[nnz].
constexpr int kMaxScanTiles = 64;   // tiles of 16384 rows: n_p n_q <= 2^20
inline int64_t hint_len(int64_t nnz) { return (nnz + 63) / 64 + 1; }
int scan_tiles(int nrow);
int64_t structure_rows(wpcd_ctx *c, int32_t *cnt, int64_t *row_ptr, int64_t *tsum);
void structure_count_copy(wpcd_ctx *c);
void structure_fill(wpcd_ctx *c, const int32_t *cnt, const int64_t *tsum, int64_t *row_ptr,
                    int32_t *col, int32_t *hint, uint8_t *rstart, int64_t cap);
// nuc_spread: nucleon channels from one s-wave value per cell pair in a
// scratch array of the context (false: the multichannel kernels, no
// allocation)
void values_into(wpcd_ctx *c, bool fp64, const int64_t *row_ptr, const int32_t *col,
                 const int32_t *hint, const uint8_t *rstart, int64_t nnz, double *val64,
                 float *val32, bool measure, bool nuc_spread);

// Pick candidate 0..n_cand-1 for (name, key): forced, cached, heuristic
// (heur) or measured (measure(i) returns microseconds), by c->tune.mode.
template <class Measure>
int tune_pick(wpcd_ctx *c, const char *name, const std::string &key, int n_cand, int heur,
              Measure &&measure, bool allow_measure = true) {
    Tuning &T = c->tune;
    if (T.mode >= WPCD_TUNE_FORCE) return std::min(T.mode - WPCD_TUNE_FORCE, n_cand - 1);
    for (const auto &e : T.entries)
        if (e.name == name && e.key == key) return e.choice;
    if (!allow_measure) return heur;   // not recorded: a later call may still measure
    int best = heur;
    double best_us = 0.0;
    if (T.mode == WPCD_TUNE_MEASURE) {
        best_us = 1e300;
        for (int i = 0; i < n_cand; ++i) {
            const double us = measure(i);
            if (us < best_us) {
                best_us = us;
                best = i;
            }
        }
    }
    T.entries.push_back({name, key, best, n_cand, best_us});
    return best;
}

// Batched GMRES over energies (k_solve.hip).  warm: fills the initial
// vector in the batch layout x[row][e][2] (called after b is formed), or
// empty for the zero start.  Per energy: iterations, final relative
// residual, resolvent edge flag, warm start kept, initial relative residual.
struct GmresOut {
    std::vector<int> iters, edge, warm;
    std::vector<int> stag;   // stopped on stagnation (see gmres_cycles)
    std::vector<double> resid, r0;
    std::vector<double> U, dU;   // err_est: on-shell x and its FP64 correction, [nE][2]
};
using WarmFill = void (*)(wpcd_ctx *c, void *user, double *x, int nE);
void gmres_batch(wpcd_ctx *c, const std::vector<double> &E, const std::vector<int64_t> &idx0,
                 int prec, int m, int max_iter, double tol, WarmFill warm, void *warm_user,
                 GmresOut &out, bool err_est = false,
                 const std::vector<double> *ebin = nullptr);   // [nE][2]: averaged resolvent
// The same in three parts, so that batches of several systems can iterate in
// lockstep: set up (resolvent, driving term, initial vector), restarted
// cycles of one or several runs together, finish (error estimate).
struct GmresRun;
GmresRun *gmres_run_new();
void gmres_run_delete(GmresRun *r);
void gmres_setup(GmresRun &run, wpcd_ctx *c, const std::vector<double> &E,
                 const std::vector<int64_t> &idx0, int prec, int m, int max_iter, double tol,
                 WarmFill warm, void *warm_user, GmresOut &out, bool err_est,
                 const std::vector<double> *ebin);
void gmres_cycles(std::vector<GmresRun *> &runs);
void gmres_finish(GmresRun &run);
void arnoldi_kernel(wpcd_ctx *c, double E, int m, std::vector<double> &H, int &steps);
void amplitudes_batch(wpcd_ctx *c, int nE, const std::vector<int64_t> &rows,
                      const std::vector<int32_t> &ens, const std::vector<double> &rho,
                      const std::vector<double> &rho0, std::vector<double> &out);

// Network kernels (k_mlp.hip).  X, T, Y on the device; parameters in m.
void mlp_init(Mlp &m, hipStream_t s, int nin, int nh, int nout, uint64_t seed);
void mlp_set_weights(Mlp &m, hipStream_t s, const float *w_host);
float *mlp_forward(Mlp &m, hipStream_t s, Timer &t, const float *X, int B);
// Gradients into m.grad; returns the loss if want_loss (synchronises), else 0.
double mlp_loss_grad(Mlp &m, hipStream_t s, Timer &t, const float *X, const float *T, int B,
                     bool want_loss);
void mlp_adam_step(Mlp &m, hipStream_t s, Timer &t, float lr);
void mlp_gather(hipStream_t s, const float *src, int ncol, const int32_t *idx, int n, float *dst);

// Learned warm start (wpcd_learn.hip).
void learn_snap_store(wpcd_ctx *c, float *snaps, int64_t first, const double *x, int nE,
                      const std::vector<int> &which);
void learn_build_basis(wpcd_ctx *c, const float *snaps, int n, int K, std::vector<double> &coef,
                       double &max_err, double &mean_err);
void learn_lift(wpcd_ctx *c, const float *y, int nE, double *x);
void learn_interleave(wpcd_ctx *c, const double *src, int nE, int64_t M, double *x);

}  // namespace wpcd
