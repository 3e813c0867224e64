// Lattice permutation matrix P0 (paper Sec. III.B eqs.(perm),(gal); GPU
// scheme Sec. IV.B-C): pre-selection of the nonzero cell pairs, compaction
// into CSR, and the cell-overlap quadrature for each selected pair.
//
// Structure kernels use only IEEE add/sub/compare on FP64 tables computed on
// the host (p, q, p^2, 3/4 q^2, q/2), so the selected set is bit-exact.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>

#include <cmath>
#include <type_traits>

#include "wpcd_internal.h"

#pragma clang fp contract(off)

namespace wpcd {

struct GridView {
    const double *p, *q, *P2, *Q34, *H;   // p[np+1], q[nq+1], p^2, 3/4 q^2, q/2
    int np, nq;
};

// First index k in [lo, hi) with f(k) true for a monotone predicate
// (false ... false true ... true); returns hi if none.
template <class F>
__device__ __forceinline__ int first_true(int lo, int hi, F f) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (f(mid)) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// The same first index in [0, n) by binary lifting with a step count that
// depends on n only (top = the largest power of two <= n, the same in every
// lane), so the loop control stays scalar however the lanes' answers differ:
// k grows by s whenever f(k + s - 1) is false, keeping f false below k.
template <class F>
__device__ __forceinline__ int first_true_lift(int n, int top, F f) {
    int k = 0;
    for (int s = top; s > 0; s >>= 1) {
        const int t = k + s;
        if (t <= n && !f(t - 1)) k = t;
    }
    return k;
}

__device__ __forceinline__ int pow2_floor(int n) { return n > 0 ? 1 << (31 - __clz(n)) : 0; }

// First index k in [0, n) with f(k) true for a monotone predicate that is
// the same in every lane (n if none): each step tests 64 points spread over
// the current interval, one per lane, and a ballot keeps the sub-interval
// holding the first true one (two steps for n <= 4096).
template <class F>
__device__ __forceinline__ int first_true_wave(int n, F f) {
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = n;   // answer in [lo, hi]; points >= hi count as true
    while (hi > lo) {
        const int step = (hi - lo + 63) >> 6;
        const int k = lo + lane * step;          // tested point of this lane
        const bool t = k >= hi || f(k);
        const unsigned long long m = __builtin_amdgcn_ballot_w64(t);
        // lane c = the first true point; the answer is in (point c - 1,
        // point c] (none true: beyond lane 63's point)
        const int c = m ? (int)__builtin_ctzll(m) : 64;
        const int nlo = c == 0 ? lo : lo + (c - 1) * step + 1;
        const int nhi = c == 64 ? hi : min(lo + c * step, hi);
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// Row cell (i, j): |q' + q/2| over q in bin j and q' in bin j2 reaches D_i
// when p[i+1] > max(0, q[j2] - H[j+1], H[j] - q[j2+1]) and
// p[i] < q[j2+1] + H[j+1].  Each of the three comparisons is monotone in j2,
// so the column spectator bins that pass form one interval [J0, J1).  (On
// the Chebyshev grids about a fifth of all j2 pass, and every passing j2 but
// a few holds a selected cell.)
__device__ __forceinline__ void row_bins(const GridView &g, int i, int j, int &J0, int &J1) {
    const double pi1 = g.p[i + 1], pi0 = g.p[i], hj = g.H[j], hj1 = g.H[j + 1];
    const int n = g.nq;
    J1 = first_true_wave(n, [&](int k) { return !(pi1 > g.q[k] - hj1); });
    const int b2 = first_true_wave(n, [&](int k) { return pi1 > hj - g.q[k + 1]; });
    const int b3 = first_true_wave(n, [&](int k) { return pi0 < g.q[k + 1] + hj1; });
    J0 = b2 > b3 ? b2 : b3;
    if (J1 < J0) J1 = J0;
}

// Column range [lo, hi) of row cell (i, j) in a passing column spectator bin
// j2: the intersection of four monotone conditions on i2,
//   la: first i2 with  P2[i2+1] + Q34[j2+1] >  P2[i] + Q34[j]  (energy ranges)
//   hb: first i2 with !(P2[i+1] + Q34[j+1] >  P2[i2] + Q34[j2])
//   lc: first i2 with  p[i2+1] > max(0, q[j] - H[j2+1], H[j2] - q[j+1])
//                                              (|q + q'/2| can reach D_i2)
//   hd: first i2 with !(p[i2] < q[j+1] + H[j2+1])
// Two lanes share a j2: the even one finds la and lc (the lower end), the
// odd one hb and hd (the upper end), both with the same instructions: the
// energy search is "first k with P2[k + o] + a > b" (even: o = 1, strict;
// odd: o = 0, b = the row's upper energy, "!(b > x)" read as x >= b) and the
// pi2 search "first k with p[k + o] > b" (or >= b) likewise.  col_pair
// returns [lo, hi) in the even lane (hi == lo in the odd one).  Every
// comparison is the same IEEE expression as in the predicate above, so the
// selected set is the same bit for bit.
__device__ __forceinline__ void col_pair(const GridView &g, int i, int j, int j2, bool on,
                                         int &lo, int &hi) {
    const bool upper = threadIdx.x & 1;
    int e1 = 0, e2 = 0;
    if (on) {
        double a, d2 = 0.0;
        a = g.q[j] - g.H[j2 + 1];
        if (a > d2) d2 = a;
        a = g.H[j2] - g.q[j + 1];
        if (a > d2) d2 = a;
        const double pmax2 = g.q[j + 1] + g.H[j2 + 1];
        const int o = upper ? 0 : 1;
        const double ea = upper ? g.Q34[j2] : g.Q34[j2 + 1];
        const double eb = upper ? g.P2[i + 1] + g.Q34[j + 1] : g.P2[i] + g.Q34[j];
        const double pb = upper ? pmax2 : d2;
        const int n = g.np, top = pow2_floor(n);
        const double *P2o = g.P2 + o, *po = g.p + o;
        e1 = first_true_lift(n, top, [&](int k) {
            const double x = P2o[k] + ea;
            return upper ? x >= eb : x > eb;
        });
        e2 = first_true_lift(n, top, [&](int k) {
            const double x = po[k];
            return upper ? x >= pb : x > pb;
        });
    }
    const int v = upper ? (e1 < e2 ? e1 : e2) : (e1 > e2 ? e1 : e2);   // hi or lo
    const int w = __shfl_xor(v, 1, 64);
    lo = upper ? 0 : v;
    hi = upper ? 0 : (w > v ? w : v);
}

// Grid tables staged in LDS (p, P2: np + 1; q, Q34, H: nq + 1 doubles).
__device__ __forceinline__ GridView stage_grid(const GridView &g, double *sm) {
    GridView l;
    l.np = g.np;
    l.nq = g.nq;
    double *p = sm, *P2 = p + g.np + 1, *q = P2 + g.np + 1, *Q34 = q + g.nq + 1,
           *H = Q34 + g.nq + 1;
    for (int k = threadIdx.x; k <= g.np; k += blockDim.x) {
        p[k] = g.p[k];
        P2[k] = g.P2[k];
    }
    for (int k = threadIdx.x; k <= g.nq; k += blockDim.x) {
        q[k] = g.q[k];
        Q34[k] = g.Q34[k];
        H[k] = g.H[k];
    }
    __syncthreads();
    l.p = p;
    l.P2 = P2;
    l.q = q;
    l.Q34 = Q34;
    l.H = H;
    return l;
}

__device__ __forceinline__ int wave_isum(int v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// cnt[row] = selected cells of the row.  One wavefront per row cell (cell
// index j np + i), lanes over the row's passing column spectator bins.  No
// barrier after the table staging, so wavefronts past the last row may
// leave early.
__global__ __launch_bounds__(256) void k_count(GridView g0, int32_t *__restrict__ cnt) {
    extern __shared__ double sgrid[];
    const GridView g = stage_grid(g0, sgrid);
    const int lane = threadIdx.x & 63;
    const int nrow = g.np * g.nq;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int row = blockIdx.x * 4 + wv; row < nrow; row += gridDim.x * 4) {
        const int j = row / g.np, i = row - j * g.np;
        int J0, J1;
        row_bins(g, i, j, J0, J1);
        int c = 0;
        for (int jc = J0; jc < J1; jc += 32) {
            const int j2 = jc + (lane >> 1);
            int lo, hi;
            col_pair(g, i, j, j2, j2 < J1, lo, hi);
            c += hi - lo;
        }
        c = wave_isum(c);
        if (lane == 0) cnt[row] = c;
    }
}

// Prefix sums of cnt[0..n) per tile of 16384 rows, one workgroup of 1024
// threads per tile: row_ptr[k] = exclusive sum within k's tile, tsum[t] =
// the tile's total (the fill kernel adds the sums of the earlier tiles).
// Each thread sums 16 consecutive counts (stored with one pad word per 16 so
// the 64 lanes of a wavefront hit distinct banks); the 1024 segment sums are
// scanned by shuffles and across the 16 wavefronts; row_ptr is written
// coalesced.
constexpr int kScanTile = 16384, kScanSeg = 16;

__global__ __launch_bounds__(1024) void k_scan(const int32_t *__restrict__ cnt, int n,
                                               int64_t *__restrict__ row_ptr,
                                               int64_t *__restrict__ tsum) {
    __shared__ int32_t sc[kScanTile + kScanTile / kScanSeg];
    __shared__ int64_t wtot[16];
    __shared__ int64_t segbase[1024];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    auto pos = [](int k) { return k + k / kScanSeg; };
    const int t0 = blockIdx.x * kScanTile;
    const int m = min(kScanTile, n - t0);
    for (int k = tid; k < kScanTile; k += 1024) sc[pos(k)] = k < m ? cnt[t0 + k] : 0;
    __syncthreads();
    int32_t run = 0;
    const int b = tid * kScanSeg;
#pragma unroll
    for (int k = 0; k < kScanSeg; ++k) {
        const int32_t v = sc[pos(b + k)];
        sc[pos(b + k)] = run;   // offset within the segment
        run += v;
    }
    int64_t incl = run;
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wtot[wv] = incl;
    __syncthreads();
    int64_t wbase = 0, ttot = 0;
    for (int w = 0; w < 16; ++w) {
        const int64_t x = wtot[w];
        if (w < wv) wbase += x;
        ttot += x;
    }
    segbase[tid] = wbase + incl - run;
    __syncthreads();
    for (int k = tid; k < m; k += 1024) row_ptr[t0 + k] = segbase[k / kScanSeg] + sc[pos(k)];
    if (tid == 0) tsum[blockIdx.x] = ttot;
}

// Column indices c = j2 np + i2 of every row, ascending, from the same
// ranges as k_count (recomputed).  One wavefront per row: the row's start is
// its in-tile offset from k_scan plus the totals of the earlier tiles,
// written back as the final row_ptr[row] (and row_ptr[nrow] by the last
// row).  Each lane writes its own range's columns one after another (the
// lanes' runs are adjacent, so a store instruction covers a few consecutive
// cache lines).  Row lookup tables for the element kernels: hint[e / 64] =
// the row of nonzero e for every e divisible by 64, and rstart[e] = 1 where
// nonzero e is the first of its row (2 if the row before it is empty), else
// 0; the row of any e is then hint[e / 64] plus the row starts after e's
// block start up to e.
__global__ __launch_bounds__(256) void k_fill(GridView g0, const int32_t *__restrict__ cnt,
                                              const int64_t *__restrict__ tsum,
                                              int64_t *__restrict__ row_ptr,
                                              int32_t *__restrict__ col,
                                              int32_t *__restrict__ hint,
                                              uint8_t *__restrict__ rstart, int64_t cap) {
    extern __shared__ double sgrid[];
    const GridView g = stage_grid(g0, sgrid);
    const int lane = threadIdx.x & 63;
    const int nrow = g.np * g.nq;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int row = blockIdx.x * 4 + wv; row < nrow; row += gridDim.x * 4) {
        const int j = row / g.np, i = row - j * g.np;
        // sum of the earlier tiles' totals (at most 64 tiles)
        const int tile = row / kScanTile;
        int64_t tb = lane < tile ? tsum[lane] : 0;
        for (int off = 32; off > 0; off >>= 1) tb += __shfl_xor(tb, off, 64);
        const int64_t first = row_ptr[row] + tb;
        if (lane == 0) row_ptr[row] = first;
        // row-start mark of the row's first nonzero: 2 after an empty row
        const uint8_t mark = (row > 0 && cnt[row - 1] == 0) ? 2 : 1;
        int64_t base = first;
        int J0, J1;
        row_bins(g, i, j, J0, J1);
        for (int jc = J0; jc < J1; jc += 32) {
            const int j2 = jc + (lane >> 1);
            int lo, hi;
            col_pair(g, i, j, j2, j2 < J1, lo, hi);
            const int cn = hi - lo;
            int incl = cn;
            for (int off = 1; off < 64; off <<= 1) {
                const int v = __shfl_up(incl, off, 64);
                if (lane >= off) incl += v;
            }
            int64_t pos = base + (incl - cn);
            for (int i2 = lo; i2 < hi && pos < cap; ++i2, ++pos) {
                col[pos] = j2 * g.np + i2;
                rstart[pos] = pos == first ? mark : 0;
                if ((pos & 63) == 0) hint[pos >> 6] = row;
            }
            base += __shfl(incl, 63, 64);
        }
        if (row == nrow - 1 && lane == 0) row_ptr[nrow] = base;
    }
}

// Row r of nonzero e (row_ptr[r] <= e < row_ptr[r + 1]; e is the same in
// every lane and e < row_ptr[nrow]), by a 64-way search over row_ptr: each
// step compares 64 boundaries spread evenly over the current row interval
// with e (a ballot; row_ptr is nondecreasing, so the true lanes are a
// prefix) and keeps the sub-interval that brackets e.  Three steps up to
// 262144 rows, four up to 2^24.
__device__ __forceinline__ int row_of(const int64_t *__restrict__ row_ptr, int nrow, int64_t e) {
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = nrow;   // row_ptr[lo] <= e < row_ptr[hi]
    while (hi - lo > 1) {
        const int step = (hi - lo + 63) >> 6;
        const int b = lo + (lane + 1) * step;
        const bool le = b < hi && row_ptr[b] <= e;
        const int cnt = (int)__popcll(__builtin_amdgcn_ballot_w64(le));
        lo += cnt * step;
        hi = min(hi, lo + step);
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// Rows of nonzeros in the 64-nonzero block of e (wave-uniform e <
// row_ptr[nrow]): the block's first row from hint, and a ballot of the
// rstart marks of the block's 64 nonzeros (one byte per lane, the same load
// for every lane).  A row is the first row plus the row starts after the
// block start up to e.  A mark of 2 (an empty row skipped) makes exact()
// false up to that point; the caller then searches row_ptr.
struct BlockRows {
    int r0;
    int64_t b0;
    unsigned long long starts, gaps;
    __device__ __forceinline__ void start(const int32_t *hint, const uint8_t *rstart, int64_t nnz,
                                          int64_t e) {
        const int64_t m = e >> 6;
        b0 = m << 6;
        r0 = __builtin_amdgcn_readfirstlane(hint[m]);
        const int64_t pos = b0 + (threadIdx.x & 63);
        const int v = pos < nnz ? rstart[pos] : 0;
        starts = __builtin_amdgcn_ballot_w64(v != 0) & ~1ull;
        gaps = __builtin_amdgcn_ballot_w64(v > 1) & ~1ull;
    }
    // nonzeros b0 .. e of the block
    __device__ __forceinline__ unsigned long long upto(int64_t e) const {
        return ~0ull >> (63 - (int)(e - b0));
    }
    __device__ __forceinline__ bool exact(int64_t e) const { return (gaps & upto(e)) == 0; }
    __device__ __forceinline__ int row(int64_t e) const {
        return r0 + (int)__popcll(starts & upto(e));
    }
};

// The element quadrature below may contract into FMAs.
#pragma clang fp contract(fast)

// ------------------------------------------------------------ element
// P0 element of cell pair (i, j) x (i2, j2), s-wave:
//   (d_i d_i2 dq_j dq_j2)^(-1/2) sum_{a,b} wq_a wq_b  int dt / sqrt(t u)
// with t = pi1^2 in [t_lo, t_hi] (the clipped cosine interval mapped by the
// affine t = q'^2 + q^2/4 + q q' x; the q q' of the measure cancels dx = dt/(q q'))
// and u = pi2^2 = t + 3/4 (q^2 - q'^2).  Lane = (a, b) Gauss pair.
struct ElemTables {
    const double *P2;      // p^2 [np+1]
    const double *rsd_p;   // 1/sqrt(d_i) [np]
    const double *rsd_q;   // 1/sqrt(dq_j) [nq]
    const double *qnode;   // [nq][ngq] Gauss points in each q bin
    const double *qwt;     // [nq][ngq] weights * half width
    const double *ux;      // 1 + t_c [ngx]
    const double *wx;      // w_c [ngx]
    const float *uxf, *wxf;
    int np, ngq, ngx;
    uint32_t np_magic;     // ceil(2^32 / np): r / np = umulhi(r, np_magic) for r < 2^20
    int nrow;              // cells n_p n_q (rows of row_ptr)
    const int32_t *hint;   // hint[e / 64]: row of nonzero e, e divisible by 64
    const uint8_t *rstart; // rstart[e]: nonzero e starts its row (1; 2 after an empty row)
};

// (i, j) of a cell index r = j np + i (r < 2^20, np <= 1024): the quotient
// by multiply-high is exact because r (np_magic - 2^32/np) / 2^32 < 2^-12 is
// below the gap 1/np between r/np and the next integer.
__device__ __forceinline__ void cell_ij(const ElemTables &T, uint32_t r, int &i, int &j) {
    j = (int)__umulhi(r, T.np_magic);
    i = (int)r - j * T.np;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Neumaier two-sum accumulation in FP32.
struct Comp32 {
    float s = 0.f, c = 0.f;
    __device__ __forceinline__ void add(float x) {
        float t = s + x;
        if (fabsf(s) >= fabsf(x)) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
    }
};

// Parts of the limits that depend only on the Gauss pair (q, q2).
struct QLim {
    double t_lo, t_hi, u_lo, u_hi, D;
};

__device__ __forceinline__ QLim q_limits(double q, double q2) {
    // Limits are rounded exactly as written (no FMA contraction): where a
    // limit is formed by cancellation (p^2 - D with D ~ p^2) the element is
    // ill-conditioned and must round the same way as the reference formula.
#pragma clang fp contract(off)
    // cosine -1 / +1 give pi1 = |q2 -+ q/2| and pi2 = |q -+ q2/2|: squares
    // formed directly, and u - t = D = 3/4 (q^2 - q2^2) as a product, so no
    // limit is formed by cancellation.
    const double m1 = q2 - 0.5 * q, p1 = q2 + 0.5 * q;
    const double m2 = q - 0.5 * q2, p2 = q + 0.5 * q2;
    QLim L;
    L.D = 0.75 * (q - q2) * (q + q2);
    L.t_lo = m1 * m1;
    L.t_hi = p1 * p1;
    L.u_lo = m2 * m2;
    L.u_hi = p2 * p2;
    return L;
}

// Clipped interval of t = pi1^2 (and u = pi2^2 = t + D) for pair bins i, i2.
__device__ __forceinline__ void bin_limits(const ElemTables &T, int i, int i2, const QLim &L,
                                           double &lo_t, double &lo_u, double &h) {
#pragma clang fp contract(off)
    const double pl1 = T.P2[i], ph1 = T.P2[i + 1];
    const double pl2 = T.P2[i2], ph2 = T.P2[i2 + 1];
    lo_t = fmax(fmax(L.t_lo, pl1), pl2 - L.D);
    double hi_t = fmin(fmin(L.t_hi, ph1), ph2 - L.D);
    lo_u = fmax(fmax(L.u_lo, pl2), pl1 + L.D);
    double hi_u = fmin(fmin(L.u_hi, ph2), ph1 + L.D);
    h = (hi_t > lo_t) ? 0.25 * ((hi_t - lo_t) + (hi_u - lo_u)) : 0.0;
}

__device__ __forceinline__ void lane_limits(const ElemTables &T, int i, int i2, double q, double q2,
                                            double &lo_t, double &lo_u, double &h) {
    bin_limits(T, i, i2, q_limits(q, q2), lo_t, lo_u, h);
}

// bin_limits split by what each part depends on: the row bin i (with the
// Gauss pair) and the column bin i2.  max and min are exact, so the
// regrouped limits equal bin_limits' bit for bit.
struct RowLim {
    double A1, B1, A2, B2;   // t: [A1, B1] before the column bin; u: [A2, B2]
};

__device__ __forceinline__ RowLim row_limits(const ElemTables &T, int i, const QLim &L) {
#pragma clang fp contract(off)
    const double pl1 = T.P2[i], ph1 = T.P2[i + 1];
    RowLim R;
    R.A1 = fmax(L.t_lo, pl1);
    R.B1 = fmin(L.t_hi, ph1);
    R.A2 = fmax(L.u_lo, pl1 + L.D);
    R.B2 = fmin(L.u_hi, ph1 + L.D);
    return R;
}

// Returns whether the lane's interval is open (h > 0 as in bin_limits); h
// is meaningful only then.
__device__ __forceinline__ bool cell_limits(const ElemTables &T, int i2, const QLim &L,
                                            const RowLim &R, double &lo_t, double &lo_u,
                                            double &h) {
#pragma clang fp contract(off)
    const double pl2 = T.P2[i2], ph2 = T.P2[i2 + 1];
    lo_t = fmax(R.A1, pl2 - L.D);
    const double hi_t = fmin(R.B1, ph2 - L.D);
    lo_u = fmax(R.A2, pl2);
    const double hi_u = fmin(R.B2, ph2);
    const double dt = hi_t - lo_t;
    h = 0.25 * (dt + (hi_u - lo_u));
    // hi_t > lo_t and h > 0 as one comparison (dt > 0 exactly when hi_t > lo_t)
    return fmin(dt, h) > 0.0;
}

__global__ __launch_bounds__(256) void k_p0_swave_f64(ElemTables T,
                                                      const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col, int64_t nnz,
                                                      double *__restrict__ val) {
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int npair = T.ngq * T.ngq;
    for (int64_t e = wave0; e < nnz; e += nwaves) {
        BlockRows br{};
        br.start(T.hint, T.rstart, nnz, e);
        const int r = br.exact(e) ? br.row(e) : row_of(row_ptr, T.nrow, e), c = col[e];
        const int i = r % T.np, j = r / T.np, i2 = c % T.np, j2 = c / T.np;
        double acc = 0.0;
        for (int pr = lane; pr < npair; pr += 64) {
            const int a = pr / T.ngq, b = pr - a * T.ngq;
            const double q = T.qnode[j * T.ngq + a], q2 = T.qnode[j2 * T.ngq + b];
            double lo_t, lo_u, h;
            lane_limits(T, i, i2, q, q2, lo_t, lo_u, h);
            if (h > 0.0) {
                double s = 0.0;
                for (int k = 0; k < T.ngx; ++k) {
                    const double sk = h * T.ux[k];
                    s += T.wx[k] * rsqrt((lo_t + sk) * (lo_u + sk));
                }
                acc += T.qwt[j * T.ngq + a] * T.qwt[j2 * T.ngq + b] * h * s;
            }
        }
        acc = wave_sum(acc);
        if (lane == 0) val[e] = acc * (T.rsd_p[i] * T.rsd_p[i2]) * (T.rsd_q[j] * T.rsd_q[j2]);
    }
}

__global__ __launch_bounds__(256) void k_p0_swave_f32(ElemTables T,
                                                      const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col, int64_t nnz,
                                                      float *__restrict__ val) {
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int npair = T.ngq * T.ngq;
    for (int64_t e = wave0; e < nnz; e += nwaves) {
        BlockRows br{};
        br.start(T.hint, T.rstart, nnz, e);
        const int r = br.exact(e) ? br.row(e) : row_of(row_ptr, T.nrow, e), c = col[e];
        const int i = r % T.np, j = r / T.np, i2 = c % T.np, j2 = c / T.np;
        Comp32 acc;
        for (int pr = lane; pr < npair; pr += 64) {
            const int a = pr / T.ngq, b = pr - a * T.ngq;
            const double q = T.qnode[j * T.ngq + a], q2 = T.qnode[j2 * T.ngq + b];
            double lo_t, lo_u, h;
            lane_limits(T, i, i2, q, q2, lo_t, lo_u, h);
            if (h > 0.0) {
                const float tf = (float)lo_t, uf = (float)lo_u, hf = (float)h;
                Comp32 s;
                for (int k = 0; k < T.ngx; ++k) {
                    const float sk = hf * T.uxf[k];
                    s.add(T.wxf[k] * rsqrtf((tf + sk) * (uf + sk)));
                }
                const float wab = (float)(T.qwt[j * T.ngq + a] * T.qwt[j2 * T.ngq + b] * h);
                acc.add(wab * s.s);
                acc.add(wab * s.c);
            }
        }
        // compensated wavefront reduction of (s, c) pairs
        float s = acc.s, cc = acc.c;
        for (int off = 32; off > 0; off >>= 1) {
            float so = __shfl_xor(s, off, 64), co = __shfl_xor(cc, off, 64);
            float t = s + so;
            float bp = t - s;
            float err = (s - (t - bp)) + (so - bp);
            s = t;
            cc = cc + co + err;
        }
        if (lane == 0)
            val[e] = (float)(((double)s + (double)cc) * (T.rsd_p[i] * T.rsd_p[i2]) *
                             (T.rsd_q[j] * T.rsd_q[j2]));
    }
}

// ------------------------------------------------- compacted element kernel
// For the 8-point q rule (64 Gauss pairs per cell pair).  About half of the
// (q, q') pairs of a cell pair have an empty cosine interval, so a wavefront
// first evaluates the limits of EC cell pairs x 64 Gauss pairs, compacts
// the non-empty ones into an LDS queue (ballot + popcount, order preserved),
// then every lane integrates one queued interval at a time with the cosine
// rule fully unrolled, and finally each cell pair is reduced over its slots
// (FP32: (hi, lo) pairs combined with TwoSum).  Deterministic: the queue
// order and the reduction order depend only on the inputs.

struct NodeTab {
    double ux[kMaxGx], wx[kMaxGx];
    float uxf[kMaxGx], wxf[kMaxGx];
};

__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    const float bp = s - a;
    e = (a - (s - bp)) + (b - bp);
}

// Interval sum over the cosine rule in FP32.  With A = t0 u0 and B = t0 + u0
// (all terms positive, so no cancellation) the node product is
// (t0 + s)(u0 + s) = A + s (B + s): one add and one FMA per node.  (The
// two-FMA Horner form of inner_f64 measures slower here.)
template <int NGX>
__device__ __forceinline__ void inner_f32(const NodeTab &N, int ngx, float lt, float lu, float h,
                                          float &s0, float &s1) {
    s0 = 0.f;
    s1 = 0.f;
    const float A = lt * lu, B = lt + lu;
    if (NGX > 0) {
#pragma unroll
        for (int k = 0; k < NGX; k += 2) {
            const float sa = h * N.uxf[k];
            s0 = fmaf(N.wxf[k], __builtin_amdgcn_rsqf(fmaf(sa, B + sa, A)), s0);
            if (k + 1 < NGX) {
                const float sb = h * N.uxf[k + 1];
                s1 = fmaf(N.wxf[k + 1], __builtin_amdgcn_rsqf(fmaf(sb, B + sb, A)), s1);
            }
        }
    } else {
        for (int k = 0; k < ngx; ++k) {
            const float sa = h * N.uxf[k];
            const float v = N.wxf[k] * __builtin_amdgcn_rsqf(fmaf(sa, B + sa, A));
            if (k & 1) s1 += v;
            else s0 += v;
        }
    }
}

// 1/sqrt(x) in FP64: FP32 seed (v_rsq_f32, ~1 ulp of FP32) refined by two
// Newton-Raphson steps y <- y (3 - x y^2) / 2, each squaring the relative
// error (2^-23 -> 2^-45 -> below FP64 rounding).  Arguments here are
// products of squared momenta, well inside the FP32 normal range.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = (double)__builtin_amdgcn_rsqf((float)x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}

template <int NGX>
__device__ __forceinline__ double inner_f64(const NodeTab &N, int ngx, double lt, double lu,
                                            double h) {
    double s = 0.0;
    const double A = lt * lu, B = lt + lu;   // (t0 + s)(u0 + s) = A + s (B + s)
    if (NGX > 0) {
        // = A + (beta + gamma x_k) x_k, beta = h B, gamma = h^2 (all terms
        // positive): two FMAs per node with the node constant x_k
        const double beta = h * B, gamma = h * h;
#pragma unroll
        for (int k = 0; k < NGX; ++k)
            s = fma(N.wx[k], rsqrt_nr(fma(fma(gamma, N.ux[k], beta), N.ux[k], A)), s);
    } else {
        for (int k = 0; k < ngx; ++k) {
            const double sk = h * N.ux[k];
            s = fma(N.wx[k], rsqrt_nr(fma(sk, B + sk, A)), s);
        }
    }
    return s;
}

// FP64 value of lane (permuted within its row of 16) by a DPP move of both
// halves; every lane must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over aligned groups of G lanes (G = 16, 8 or 4), the result in every
// lane of the group: row mirror (lane i with 15 - i), half-row mirror
// (i with 7 - i), quad reverse, quad swap.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    static_assert(G == 16 || G == 8 || G == 4, "group of 4, 8 or 16 lanes");
    if (G == 16) v += dpp_f64<0x140>(v);
    if (G >= 8) v += dpp_f64<0x141>(v);
    v += dpp_f64<0x1B>(v);   // quad_perm [3, 2, 1, 0]
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    return v;
}

// Per-wavefront LDS of the compacted kernel: the queued intervals (t0, u0,
// half-length, Gauss weight, destination sum slot) and the per-slot sums.
template <class R, int EC>
struct ElemQueue {
    R lt[EC * 64], lu[EC * 64], h[EC * 64], w[EC * 64];
    R s_hi[EC * 64];
    float s_lo[EC * 64];
    uint16_t dst[EC * 64];   // k * 64 + rank: cell pair k of the round, lane rank
};

// Sums over the 64 lanes of one wavefront of the NP values each lane has
// stored in red[p][lane], the wavefront's own LDS block (no other wavefront
// touches it, and a wavefront's LDS accesses are performed in order): lane
// 4 p + x (x < 4) sums the quarter x of value p, then the quad is combined
// by DPP.  Returns the sum of value p in lanes 4 p .. 4 p + 3 (p < NP); a
// fixed order.  The caller brackets its stores with wave barriers.
template <int NP>
__device__ __forceinline__ double wave_sums(double (*red)[64], int lane) {
    static_assert(NP <= 16, "at most 16 values");
    __builtin_amdgcn_wave_barrier();
    const int p = lane >> 2, x = lane & 3;
    double s = 0.0;
    if (p < NP) {
#pragma unroll
        for (int r = 0; r < 16; ++r) s += red[p][x * 16 + r];
    }
    s += dpp_f64<0xB1>(s);   // quad_perm [1, 0, 3, 2]
    s += dpp_f64<0x4E>(s);   // quad_perm [2, 3, 0, 1]
    __builtin_amdgcn_wave_barrier();
    return s;
}

template <bool F32, int NGX, int EC>
__global__ __launch_bounds__(256) void k_p0_swave_c(ElemTables T, NodeTab N,
                                                    const int64_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col, int64_t nnz,
                                                    double *__restrict__ val64,
                                                    float *__restrict__ val32) {
    using R = typename std::conditional<F32, float, double>::type;
    constexpr int kEC = EC;   // cell pairs per wavefront per round
    // one block per wavefront: members at fixed offsets from one base, so a
    // queue slot is one address plus immediate offsets
    __shared__ ElemQueue<R, kEC> Qs[4];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    ElemQueue<R, kEC> &Q = Qs[w];
    const int a = lane >> 3, b = lane & 7;
    const int64_t nch = (nnz + kEC - 1) / kEC;
    for (int64_t it = 0;; ++it) {
        const int64_t cbase = (it * gridDim.x + blockIdx.x) * 4;
        if (cbase >= nch) break;   // uniform across the workgroup
        const int64_t chunk = cbase + w;
        // phase 1: limits of kEC cell pairs, compaction into the queue
        int total = 0;
        // cell pairs in this wavefront's round (wave-uniform; 0 past the end)
        const int nrem = chunk < nch ? (int)std::min<int64_t>(nnz - chunk * kEC, kEC) : 0;
        // consecutive cell pairs of a row mostly share the spectator bins
        // (j, j2): their Gauss-pair parts of the limits are kept, and the
        // row-bin parts while the row is the same too.  The normalisation
        // (d_i d_i2 dq_j dq_j2)^(-1/2) is folded into the Gauss weight the
        // same way (wq: Gauss pair and spectator bins, wr: times the row bin).
        int pj = -1, pj2 = -1, pi = -1;
        // rows of the round: the first by a search over row_ptr, the others
        // by a ballot over the next 64 row boundaries (a new search only if
        // the round crosses all of them)
        const int64_t e0 = chunk * kEC;
        int rows[kEC];
        if (nrem > 0) {
            // a round never crosses a 64-nonzero block (kEC divides 64)
            BlockRows br{};
            br.start(T.hint, T.rstart, nnz, e0);
            if (br.exact(e0 + nrem - 1)) {
#pragma unroll
                for (int k = 0; k < kEC; ++k) rows[k] = br.row(e0 + k);
            } else {
#pragma unroll
                for (int k = 0; k < kEC; ++k) rows[k] = row_of(row_ptr, T.nrow, e0 + k);
            }
        }
        QLim QL{};
        RowLim RL{};
        double wq = 0.0, wr = 0.0;
#pragma unroll
        for (int k = 0; k < kEC; ++k) {
            unsigned long long m = 0;
            if (k < nrem) {
                // the cell pair is the same for the whole wavefront
                const int64_t e = e0 + k;
                int i, j, i2, j2;
                cell_ij(T, (uint32_t)rows[k], i, j);
                cell_ij(T, (uint32_t)__builtin_amdgcn_readfirstlane(col[e]), i2, j2);
                if (j != pj || j2 != pj2) {
                    // uniform bases (scalar registers) plus the lane's node offset
                    const double *qn = T.qnode + j * 8, *qn2 = T.qnode + j2 * 8;
                    const double *qw = T.qwt + j * 8, *qw2 = T.qwt + j2 * 8;
                    QL = q_limits(qn[a], qn2[b]);
                    wq = (qw[a] * qw2[b]) * (T.rsd_q[j] * T.rsd_q[j2]);
                    pj = j;
                    pj2 = j2;
                    pi = -1;
                }
                if (i != pi) {
                    RL = row_limits(T, i, QL);
                    wr = wq * T.rsd_p[i];
                    pi = i;
                }
                double lo_t, lo_u, h;
                const bool act = cell_limits(T, i2, QL, RL, lo_t, lo_u, h);
                m = __builtin_amdgcn_ballot_w64(act);
                if (act) {
                    const int rank = (int)__builtin_amdgcn_mbcnt_hi(
                        (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                    const int slot = total + rank;
                    Q.lt[slot] = (R)lo_t;
                    Q.lu[slot] = (R)lo_u;
                    Q.h[slot] = (R)h;
                    Q.w[slot] = (R)(h * (wr * T.rsd_p[i2]));
                    Q.dst[slot] = (uint16_t)(k * 64 + rank);   // sum slot of this interval
                }
            }
            total += __popcll(m);
            Q.s_hi[k * 64 + lane] = (R)0;
            Q.s_lo[k * 64 + lane] = 0.f;
        }
        __syncthreads();
        // phase 2: one queued interval per lane
        for (int base = 0; base < total; base += 64) {
            const int t = base + lane;
            if (t < total) {
                const int d = Q.dst[t];
                if (F32) {
                    float s0, s1, hi, lo;
                    inner_f32<NGX>(N, T.ngx, (float)Q.lt[t], (float)Q.lu[t], (float)Q.h[t], s0, s1);
                    two_sum(s0, s1, hi, lo);
                    const float wf = (float)Q.w[t];
                    const float p = hi * wf;
                    const float ep = fmaf(hi, wf, -p);
                    Q.s_hi[d] = (R)p;
                    Q.s_lo[d] = fmaf(lo, wf, ep);
                } else {
                    Q.s_hi[d] = (R)(Q.w[t] * inner_f64<NGX>(N, T.ngx, (double)Q.lt[t],
                                                              (double)Q.lu[t], (double)Q.h[t]));
                }
            }
        }
        __syncthreads();
        // phase 3: each cell pair's 64 slots summed in FP64 by 16 lanes (slots
        // m, m + 16, m + 32, m + 48; conflict-free LDS rows), then across the
        // 16 lanes by DPP; each slot's (hi, lo) pair is summed in FP64 first.
        // Four cell pairs per step, so every kEC gives the same order; exact
        // enough to make the order immaterial at FP32 output precision.
        static_assert(kEC % 4 == 0, "cell pairs per round: a multiple of 4");
#pragma unroll
        for (int hf = 0; hf < kEC / 4; ++hf) {
            const int k = hf * 4 + (lane >> 4), m = lane & 15;
            auto slot = [&](int t) {
                return F32 ? (double)Q.s_hi[k * 64 + t] + (double)Q.s_lo[k * 64 + t]
                           : (double)Q.s_hi[k * 64 + t];
            };
            double sv = slot(m);
            sv += slot(m + 16);
            sv += slot(m + 32);
            sv += slot(m + 48);
            sv = group_sum<16>(sv);
            if (m == 0 && k < nrem) {
                const int64_t e = chunk * kEC + k;
                if (F32) val32[e] = (float)sv;
                else val64[e] = sv;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------ multichannel elements
// Cell pair block of P0 for n_ch channels: the s-wave integrand 1/(pi1 pi2)
// times the angular coupling G_aa'(q, q', x) = N_aa'(q^2, q'^2, y) /
// (t^(l/2) u^(l'/2) (q^2)^(lam/2) (q'^2)^(lam'/2)), y = q q' x = t - q'^2 - q^2/4,
// with N the coupling polynomial (coefficients from coupling_tables).
// One wavefront per cell pair, lanes = (q, q') Gauss pairs; FP64 arithmetic
// (the polynomial cancels near pi1 -> 0 and needs the range); values are
// stored in FP64 or rounded once to FP32.
struct McTab {
    McPair p[kMaxCh * kMaxCh];
    int npair;
};

__device__ __forceinline__ double ipow_h(double v, int h) {
    return h == 0 ? 1.0 : (h == 1 ? v : (h == 2 ? v * v : v * v * v * v));
}

// Coefficients D_c (c = 0..min(d, DEG)) of one channel pair's coupling
// polynomial in y for fixed (q, q'):
//   D_c = sum_{a <= d - c} coef[a] (q^2)^a (q'^2)^(d - c - a)
// (coef: block c of the pair's table, blocks of d - c + 1 entries), as
// (q'^2)^(d - c) H_c(r) with H_c the same polynomial in r = q^2 / q'^2 by
// Horner; rb = 1 / q'^2.  Entries with c > d are zero.
template <int DEG>
__device__ __forceinline__ void coupling_coeffs(const double *__restrict__ coef, int off, int d,
                                                double a2, double b2, double rb,
                                                double (&D)[DEG + 1]) {
    const double r = a2 * rb;
    double w = 1.0;   // (q'^2)^(d - c)
    for (int k = 0; k < d; ++k) w *= b2;
    int o = off;
#pragma unroll
    for (int c = 0; c <= DEG; ++c) {
        D[c] = 0.0;
        if (c <= d) {
            const int n = d - c;
            double hh = coef[o + n];
            for (int aa = n - 1; aa >= 0; --aa) hh = fma(hh, r, coef[o + aa]);
            D[c] = w * hh;
            w *= rb;
            o += n + 1;
        }
    }
}

template <int NP, int DEG>
__device__ __forceinline__ void mc_lane_fast(const McTab &Mt, const double *__restrict__ coef,
                                             const NodeTab &N, int ngx, double q, double q2,
                                             double lo_t, double lo_u, double h, double (&acc)[NP]) {
    const double a2 = q * q, b2 = q2 * q2, A = b2 + 0.25 * a2;
    // q, q' are interior Gauss nodes (> 0): two reciprocals serve every
    // channel pair's divisor (q^2)^(lam/2) (q'^2)^(lam'/2)
    const double ra = 1.0 / a2, rb = 1.0 / b2;
    double Dc[NP][DEG + 1];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const McPair P = Mt.p[p];
        const double rden = ipow_h(ra, P.hlam) * ipow_h(rb, P.hlam2);
        double D[DEG + 1];
        coupling_coeffs<DEG>(coef, P.off, P.d, a2, b2, rb, D);
#pragma unroll
        for (int c = 0; c <= DEG; ++c) Dc[p][c] = D[c] * rden;
        acc[p] = 0.0;
    }
    for (int k = 0; k < ngx; ++k) {
        const double sk = h * N.ux[k];
        const double t = lo_t + sk, u = lo_u + sk;
        const double rt = rsqrt_nr(t), ru = rsqrt_nr(u);
        const double base = N.wx[k] * rt * ru, it = rt * rt, iu = ru * ru;
        const double y = t - A;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            double nv = Dc[p][DEG];
#pragma unroll
            for (int c = DEG - 1; c >= 0; --c) nv = fma(nv, y, Dc[p][c]);
            acc[p] = fma(base * ipow_h(it, Mt.p[p].hl) * ipow_h(iu, Mt.p[p].hl2), nv, acc[p]);
        }
    }
}

template <int NP, int DEG>
__global__ __launch_bounds__(256) void k_p0_mc(ElemTables T, NodeTab N, McTab Mt,
                                               const double *__restrict__ coef,
                                               const int64_t *__restrict__ row_ptr,
                                               const int32_t *__restrict__ col, int64_t nnz,
                                               double *__restrict__ val64, float *__restrict__ val32) {
    __shared__ double red[4][NP][64];
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int npair_q = T.ngq * T.ngq;
    for (int64_t e = wave0; e < nnz; e += nwaves) {
        BlockRows br{};
        br.start(T.hint, T.rstart, nnz, e);
        const int r = br.exact(e) ? br.row(e) : row_of(row_ptr, T.nrow, e), c = col[e];
        const int i = r % T.np, j = r / T.np, i2 = c % T.np, j2 = c / T.np;
        double tot[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) tot[p] = 0.0;
        for (int pr = lane; pr < npair_q; pr += 64) {
            const int a = pr / T.ngq, b = pr - a * T.ngq;
            const double q = T.qnode[j * T.ngq + a], q2 = T.qnode[j2 * T.ngq + b];
            double lo_t, lo_u, h;
            lane_limits(T, i, i2, q, q2, lo_t, lo_u, h);
            if (h > 0.0) {
                double acc[NP];
                mc_lane_fast<NP, DEG>(Mt, coef, N, T.ngx, q, q2, lo_t, lo_u, h, acc);
                const double wab = T.qwt[j * T.ngq + a] * T.qwt[j2 * T.ngq + b] * h;
#pragma unroll
                for (int p = 0; p < NP; ++p) tot[p] = fma(wab, acc[p], tot[p]);
            }
        }
        const double nrm = (T.rsd_p[i] * T.rsd_p[i2]) * (T.rsd_q[j] * T.rsd_q[j2]);
        double(*rw)[64] = red[threadIdx.x >> 6];
#pragma unroll
        for (int p = 0; p < NP; ++p) rw[p][lane] = tot[p];
        const double v = wave_sums<NP>(rw, lane);
        if ((lane & 3) == 0 && (lane >> 2) < NP) {
            const int p = lane >> 2;
            if (val64) val64[e * NP + p] = v * nrm;
            else val32[e * NP + p] = (float)(v * nrm);
        }
    }
}

// Same block by moments.  The node weight of channel pair p is
// g_k t^-hl u^-hl2 with g_k = w_k / sqrt(t u), and its polynomial is
// sum_c D_pc y^c with D_pc depending only on (q, q'); so
//   sum_k g_k t^-hl u^-hl2 N_p(y_k) = sum_c D_pc M_{(hl,hl2), c},
//   M_{(h1,h2), c} = sum_k g_k t^-h1 u^-h2 y_k^c,
// and per node only the (HMAX+1)^2 x (DEG+1) moments are accumulated; the
// NP polynomials are applied once per (q, q') pair.  A reordering of the
// same sums (used for FP32 output).  NEWTON: refinement steps of the FP32
// reciprocal square root (1 for FP32 output: 2^-45 relative).
template <int NEWTON>
__device__ __forceinline__ double rsqrt_n(double x) {
    double y = (double)__builtin_amdgcn_rsqf((float)x);
    const double hx = 0.5 * x;
#pragma unroll
    for (int it = 0; it < NEWTON; ++it) y = y * fma(-hx * y, y, 1.5);
    return y;
}

template <int NP, int HMAX, int DEG, int NGX, bool F32OUT>
__global__ __launch_bounds__(256) void k_p0_mcm(ElemTables T, NodeTab N, McTab Mt,
                                                const double *__restrict__ coef,
                                                const int64_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ col, int64_t nnz,
                                                double *__restrict__ val64,
                                                float *__restrict__ val32) {
    constexpr int NG = (HMAX + 1) * (HMAX + 1);
    __shared__ double red[4][NP][64];
    const int lane = threadIdx.x & 63;
    const int a = lane >> 3, b = lane & 7;
    const int64_t wave0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t e = wave0; e < nnz; e += nwaves) {
        int i, j, i2, j2;
        BlockRows br{};
        br.start(T.hint, T.rstart, nnz, e);
        cell_ij(T, (uint32_t)(br.exact(e) ? br.row(e) : row_of(row_ptr, T.nrow, e)), i, j);
        cell_ij(T, (uint32_t)__builtin_amdgcn_readfirstlane(col[e]), i2, j2);
        const double q = T.qnode[j * 8 + a], q2 = T.qnode[j2 * 8 + b];
        double lo_t, lo_u, h;
        lane_limits(T, i, i2, q, q2, lo_t, lo_u, h);
        const bool act = h > 0.0;
        const double a2 = q * q, b2 = q2 * q2, A = b2 + 0.25 * a2;
        const double ra = 1.0 / a2, rb = 1.0 / b2;   // interior nodes: q, q' > 0
        double M[NG][DEG + 1];
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int c = 0; c <= DEG; ++c) M[g][c] = 0.0;
        if (act) {
#pragma unroll
            for (int k = 0; k < NGX; ++k) {
                const double sk = h * N.ux[k];
                const double t = lo_t + sk, u = lo_u + sk;
                const double rt = rsqrt_n<F32OUT ? 1 : 2>(t), ru = rsqrt_n<F32OUT ? 1 : 2>(u);
                const double it = rt * rt, iu = ru * ru, y = t - A;
                double gt = N.wx[k] * rt * ru;
                double gg[NG];
#pragma unroll
                for (int h1 = 0; h1 <= HMAX; ++h1) {
                    double gu = gt;
#pragma unroll
                    for (int h2 = 0; h2 <= HMAX; ++h2) {
                        gg[h1 * (HMAX + 1) + h2] = gu;
                        gu *= iu;
                    }
                    gt *= it;
                }
                double yc = 1.0;
#pragma unroll
                for (int c = 0; c <= DEG; ++c) {
#pragma unroll
                    for (int g = 0; g < NG; ++g) M[g][c] = fma(gg[g], yc, M[g][c]);
                    yc *= y;
                }
            }
        }
        const double wab = act ? T.qwt[j * 8 + a] * T.qwt[j2 * 8 + b] * h : 0.0;
        const double nrm = (T.rsd_p[i] * T.rsd_p[i2]) * (T.rsd_q[j] * T.rsd_q[j2]);
        double(*rw)[64] = red[threadIdx.x >> 6];
        for (int p = 0; p < NP; ++p) {
            const McPair P = Mt.p[p];
            const int g = P.hl * (HMAX + 1) + P.hl2;
            double v = 0.0;
            if (act) {
                double D[DEG + 1];
                coupling_coeffs<DEG>(coef, P.off, P.d, a2, b2, rb, D);
                // g is the same for the whole wavefront: a scalar branch picks
                // the moment row (D_c = 0 for c > d adds exact zeros)
#pragma unroll
                for (int gi = 0; gi < NG; ++gi) {
                    if (g != gi) continue;
#pragma unroll
                    for (int c = 0; c <= DEG; ++c) v = fma(D[c], M[gi][c], v);
                }
                v = wab * v * (ipow_h(ra, P.hlam) * ipow_h(rb, P.hlam2));
            }
            rw[p][lane] = v;
        }
        const double v = wave_sums<NP>(rw, lane);
        if ((lane & 3) == 0 && (lane >> 2) < NP) {
            const int p = lane >> 2;
            if (F32OUT) val32[e * NP + p] = (float)(v * nrm);
            else val64[e * NP + p] = v * nrm;
        }
    }
}

// General channel sets (l or lam up to 4): the coupling evaluated directly
// at every node from bipolar harmonics, as the sum of host-tabulated terms
// coef P_l^|m1|(c1) P_lam^|M-m1|(cq) P_l'^|M|(c2) (coupling_terms), with the
// polar cosines of pi1, q and pi2 taken from their vectors at the node's
// cosine x = (t - A) / (q q').  No power of t, u or q is divided out, so the
// evaluation stays accurate where pi1, pi2 or q is small.  One wavefront per
// cell pair; each lane keeps its associated Legendre values (l <= 4, index
// l (l + 1)/2 + m) in its own LDS column; channel pairs in chunks of 16.
__device__ __forceinline__ void legendre_col(double c, double (*Pt)[64], int lane) {
    const double s = sqrt(fmax(0.0, (1.0 - c) * (1.0 + c)));
    double pmm = 1.0;   // P_m^m = (-1)^m (2m - 1)!! s^m
#pragma unroll
    for (int m = 0; m <= 4; ++m) {
        if (m > 0) pmm *= -(2.0 * m - 1.0) * s;
        Pt[m * (m + 1) / 2 + m][lane] = pmm;
        if (m < 4) {
            double p1 = c * (2.0 * m + 1.0) * pmm;   // P_{m+1}^m
            Pt[(m + 1) * (m + 2) / 2 + m][lane] = p1;
            double p0 = pmm;
#pragma unroll
            for (int l = m + 2; l <= 4; ++l) {
                const double pl = (c * (2.0 * l - 1.0) * p1 - (l + m - 1.0) * p0) / (l - m);
                Pt[l * (l + 1) / 2 + m][lane] = pl;
                p0 = p1;
                p1 = pl;
            }
        }
    }
}

__device__ __forceinline__ double dir_cos(double vx, double vz) {
    const double r = sqrt(vx * vx + vz * vz);
    const double c = r > 0.0 ? vz / r : 1.0;
    return fmin(1.0, fmax(-1.0, c));
}

__global__ __launch_bounds__(64) void k_p0_mc_direct(ElemTables T, NodeTab N,
                                                     const McTerm *__restrict__ terms,
                                                     const int *__restrict__ first, int NP,
                                                     const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, int64_t nnz,
                                                     double *__restrict__ val64,
                                                     float *__restrict__ val32) {
    constexpr int PC = 16;
    __shared__ double P1[15][64], Pq[15][64], P2[15][64];
    const int lane = threadIdx.x;
    const int npair_q = T.ngq * T.ngq;
    for (int64_t e = blockIdx.x; e < nnz; e += gridDim.x) {
        int i, j, i2, j2;
        BlockRows br{};
        br.start(T.hint, T.rstart, nnz, e);
        cell_ij(T, (uint32_t)(br.exact(e) ? br.row(e) : row_of(row_ptr, T.nrow, e)), i, j);
        cell_ij(T, (uint32_t)__builtin_amdgcn_readfirstlane(col[e]), i2, j2);
        const double nrm = (T.rsd_p[i] * T.rsd_p[i2]) * (T.rsd_q[j] * T.rsd_q[j2]);
        for (int p0 = 0; p0 < NP; p0 += PC) {
            double tot[PC];
#pragma unroll
            for (int sx = 0; sx < PC; ++sx) tot[sx] = 0.0;
            for (int pr = lane; pr < npair_q; pr += 64) {
                const int a = pr / T.ngq, b = pr - a * T.ngq;
                const double q = T.qnode[j * T.ngq + a], q2 = T.qnode[j2 * T.ngq + b];
                double lo_t, lo_u, h;
                lane_limits(T, i, i2, q, q2, lo_t, lo_u, h);
                if (!(h > 0.0)) continue;
                const double A = q2 * q2 + 0.25 * q * q, B = q * q2;
                const double wab = T.qwt[j * T.ngq + a] * T.qwt[j2 * T.ngq + b] * h;
                double acc[PC];
#pragma unroll
                for (int sx = 0; sx < PC; ++sx) acc[sx] = 0.0;
                for (int k = 0; k < T.ngx; ++k) {
                    const double sk = h * N.ux[k];
                    const double t = lo_t + sk, u = lo_u + sk;
                    const double base = N.wx[k] / sqrt(t * u);
                    const double x = fmin(1.0, fmax(-1.0, (t - A) / B));
                    const double sn = sqrt((1.0 - x) * (1.0 + x));
                    legendre_col(dir_cos(0.5 * q * sn, q2 + 0.5 * q * x), P1, lane);
                    legendre_col(dir_cos(q * sn, q * x), Pq, lane);
                    legendre_col(dir_cos(-q * sn, -(q * x + 0.5 * q2)), P2, lane);
#pragma unroll
                    for (int sx = 0; sx < PC; ++sx) {
                        const int p = p0 + sx;
                        if (p >= NP) break;
                        double g = 0.0;
                        for (int tt = first[p]; tt < first[p + 1]; ++tt) {
                            const McTerm Tm = terms[tt];
                            g = fma(Tm.coef * P1[Tm.i1][lane], Pq[Tm.iq][lane] * P2[Tm.i2][lane], g);
                        }
                        acc[sx] = fma(base, g, acc[sx]);
                    }
                }
#pragma unroll
                for (int sx = 0; sx < PC; ++sx) tot[sx] = fma(wab, acc[sx], tot[sx]);
            }
#pragma unroll
            for (int sx = 0; sx < PC; ++sx) {
                const int p = p0 + sx;
                const double v = wave_sum(tot[sx]);
                if (lane == 0 && p < NP) {
                    if (val64) val64[e * NP + p] = v * nrm;
                    else val32[e * NP + p] = (float)(v * nrm);
                }
            }
        }
    }
}


// ------------------------------------------------------------------ host
static GridView grid_view(wpcd_ctx *c) {
    return GridView{c->d_p.ptr, c->d_q.ptr, c->d_P2.ptr, c->d_Q34.ptr, c->d_H.ptr, c->np, c->nq};
}

static size_t grid_lds(const wpcd_ctx *c) {
    return (size_t)(2 * (c->np + 1) + 3 * (c->nq + 1)) * sizeof(double);
}

// Grid of the row kernels: each workgroup stages the grid tables once and
// takes rows with a stride.
static int structure_blocks(const wpcd_ctx *c) { return std::min((c->np * c->nq + 3) / 4, 2048); }

int scan_tiles(int nrow) { return (nrow + kScanTile - 1) / kScanTile; }

// Count and scan kernels of the pre-selection (no host wait).
static void structure_count_scan(wpcd_ctx *c, int32_t *cnt, int64_t *row_ptr, int64_t *tsum) {
    const int nrow = c->np * c->nq;
    const int nt = scan_tiles(nrow);
    {
        TimedLaunch tl(c->timer, c->stream, "preselect_count", WPCD_TIME_PRESELECT);
        hipLaunchKernelGGL(k_count, dim3(structure_blocks(c)), dim3(256), grid_lds(c), c->stream,
                           grid_view(c), cnt);
        WPCD_HIP(hipGetLastError());
    }
    {
        TimedLaunch tl(c->timer, c->stream, "preselect_scan", WPCD_TIME_PRESELECT);
        hipLaunchKernelGGL(k_scan, dim3(nt), dim3(1024), 0, c->stream, cnt, nrow, row_ptr, tsum);
        WPCD_HIP(hipGetLastError());
    }
}

int64_t structure_rows(wpcd_ctx *c, int32_t *cnt, int64_t *row_ptr, int64_t *tsum) {
    const int nt = scan_tiles(c->np * c->nq);
    structure_count_scan(c, cnt, row_ptr, tsum);
    int64_t ts[kMaxScanTiles];
    WPCD_HIP(hipMemcpyAsync(ts, tsum, nt * sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    WPCD_HIP(hipStreamSynchronize(c->stream));
    int64_t nnz = 0;
    for (int t = 0; t < nt; ++t) nnz += ts[t];
    WPCD_REQUIRE(nnz >= 0 && nnz < ((int64_t)1 << 40), WPCD_E_DEVICE, "bad nonzero count");
    return nnz;
}

void structure_fill(wpcd_ctx *c, const int32_t *cnt, const int64_t *tsum, int64_t *row_ptr,
                    int32_t *col, int32_t *hint, uint8_t *rstart, int64_t cap) {
    TimedLaunch tl(c->timer, c->stream, "preselect_fill", WPCD_TIME_PRESELECT);
    hipLaunchKernelGGL(k_fill, dim3(structure_blocks(c)), dim3(256), grid_lds(c), c->stream,
                       grid_view(c), cnt, tsum, row_ptr, col, hint, rstart, cap);
    WPCD_HIP(hipGetLastError());
}

// The structure depends on the bin edges alone.  When they equal those of
// the last completed build, that build's nonzero count sizes the buffers
// and the element launch, and the count, scan and fill kernels run without
// the host waiting for their total in between; the total the fill writes
// (row_ptr[nrow]) is copied to pinned host memory on the stream and
// compared once the build has finished (nnz_check, copied by
// structure_count_copy after the element launch), and a mismatch rebuilds
// on the waiting path.  The fill never writes past the buffers either way.
void build_structure(wpcd_ctx *c) {
    const int nrow = c->np * c->nq;
    c->d_cnt.reserve(nrow);
    c->d_tsum.reserve(kMaxScanTiles);
    c->d_rowptr.reserve((size_t)nrow + 1);
    c->nnz_check = c->pred_nnz >= 0 && c->h_nnz && c->pred_p == c->p && c->pred_q == c->q;
    int64_t nnz;
    if (c->nnz_check) {
        structure_count_scan(c, c->d_cnt.ptr, c->d_rowptr.ptr, c->d_tsum.ptr);
        nnz = c->pred_nnz;
    } else {
        nnz = structure_rows(c, c->d_cnt.ptr, c->d_rowptr.ptr, c->d_tsum.ptr);
    }
    c->nnz = nnz;
    c->d_col.reserve(nnz);
    c->d_hint.reserve(hint_len(nnz));
    c->d_rstart.reserve(nnz);
    structure_fill(c, c->d_cnt.ptr, c->d_tsum.ptr, c->d_rowptr.ptr, c->d_col.ptr, c->d_hint.ptr,
                   c->d_rstart.ptr, nnz);
}

// The copy of the deferred count (after the element launch, so it does not
// sit between the fill and the elements on the stream).
void structure_count_copy(wpcd_ctx *c) {
    if (c->nnz_check)
        WPCD_HIP(hipMemcpyAsync(c->h_nnz, c->d_rowptr.ptr + (int64_t)c->np * c->nq,
                                sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
}

// Microseconds per launch of f (one warm-up, then two timed launches).
template <class F>
static double time_launches_p0(hipStream_t s, F &&f) {
    hipEvent_t a, z;
    WPCD_HIP(hipEventCreate(&a));
    WPCD_HIP(hipEventCreate(&z));
    f();
    WPCD_HIP(hipEventRecord(a, s));
    f();
    f();
    WPCD_HIP(hipEventRecord(z, s));
    WPCD_HIP(hipEventSynchronize(z));
    float ms = 0.f;
    WPCD_HIP(hipEventElapsedTime(&ms, a, z));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(z);
    return 1e3 * ms / 2;
}

// Where the elements are written: the structure and the value array (FP64
// or FP32, one of them non-null).
struct P0Dst {
    const int64_t *row_ptr;
    const int32_t *col;
    int64_t nnz;
    double *val64;
    float *val32;
};

template <bool F32, int EC>
static void launch_compacted_ec(wpcd_ctx *c, const ElemTables &T, const NodeTab &N,
                                const P0Dst &D, int64_t max_blocks) {
    const int64_t nchunk = (D.nnz + EC - 1) / EC;
    const int64_t want = (nchunk + 3) / 4;
    const int blocks = (int)(want < max_blocks ? want : max_blocks);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, c->stream, T, N, D.row_ptr, D.col,
                           D.nnz, D.val64, D.val32);
    };
    switch (c->ngx) {
        case 16: go(k_p0_swave_c<F32, 16, EC>); break;
        case 20: go(k_p0_swave_c<F32, 20, EC>); break;
        case 24: go(k_p0_swave_c<F32, 24, EC>); break;
        case 32: go(k_p0_swave_c<F32, 32, EC>); break;
        default: go(k_p0_swave_c<F32, 0, EC>); break;
    }
    WPCD_HIP(hipGetLastError());
}

// Launch variants: cell pairs per round (4 or 8: more pairs fill the
// integration passes better, fewer use less LDS per wavefront) and the grid
// (at most 8192 workgroups looping over rounds, or one round per workgroup,
// which lets the dispatcher balance the load).  All give identical values.
struct ElemVariant {
    int ec;
    int64_t max_blocks;
};
// (one round per workgroup up to 2^23 workgroups: the grid's thread count
// must stay below 2^32)
constexpr ElemVariant kElemVariants[4] = {{4, 8192}, {8, 8192}, {4, 1 << 23}, {8, 1 << 23}};

template <bool F32>
static void launch_compacted(wpcd_ctx *c, const ElemTables &T, const NodeTab &N,
                             const P0Dst &D, int v) {
    const ElemVariant ev = kElemVariants[v];
    if (ev.ec == 8) launch_compacted_ec<F32, 8>(c, T, N, D, ev.max_blocks);
    else launch_compacted_ec<F32, 4>(c, T, N, D, ev.max_blocks);
}

// Element values of the structure (row_ptr, col) into val64 or val32.
// measure: the launch shape of the s-wave kernel may be timed on first use
// (otherwise a cached choice or the heuristic one is taken).
// Nucleon channel blocks from the s-wave values: out[e][p] = g_p v[e]
// (p = a n_ch + b; the g_p are exact binary fractions).
struct NucG {
    double g[kMaxCh * kMaxCh];
};

template <class T>
__global__ __launch_bounds__(256) void k_spread_g(const T *__restrict__ v, int64_t nnz, int NP,
                                                  NucG G, T *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nnz * NP) return;
    const int64_t e = i / NP;
    out[i] = (T)(G.g[i - e * NP] * (double)v[e]);
}

static void swave_values(wpcd_ctx *c, const ElemTables &T, bool fp64, const P0Dst &D,
                         bool measure);

void values_into(wpcd_ctx *c, bool fp64, const int64_t *row_ptr, const int32_t *col,
                 const int32_t *hint, const uint8_t *rstart, int64_t nnz, double *val64,
                 float *val32, bool measure, bool nuc_spread) {
    ElemTables T{c->d_P2.ptr, c->d_rsd_p.ptr, c->d_rsd_q.ptr, c->d_qnode.ptr, c->d_qwt.ptr,
                 c->d_ux.ptr,  c->d_wx.ptr,    c->d_uxf.ptr,   c->d_wxf.ptr,   c->np,
                 c->ngq,       c->ngx,
                 (uint32_t)(((1ull << 32) + (uint64_t)c->np - 1) / (uint64_t)c->np),
                 c->np * c->nq, hint, rstart};
    const int NP = c->nch * c->nch;
    const P0Dst D{row_ptr, col, nnz, fp64 ? val64 : nullptr, fp64 ? nullptr : val32};
    if (nnz == 0) return;
    if (c->nuc_two_S && nuc_spread) {
        // nucleon pair s-waves: every channel block is the s-wave element
        // times g_ab, so the s-wave kernel computes it once per cell pair
        // into a scratch array and a spreading pass writes the blocks
        NucG G{};
        for (int p = 0; p < NP; ++p) G.g[p] = c->nuc_g[p];
        const unsigned blocks = (unsigned)((nnz * NP + 255) / 256);
        if (fp64) {
            c->d_nuc64.reserve(nnz);
            swave_values(c, T, true, P0Dst{row_ptr, col, nnz, c->d_nuc64.ptr, nullptr}, measure);
            hipLaunchKernelGGL(k_spread_g<double>, dim3(blocks), dim3(256), 0, c->stream,
                               c->d_nuc64.ptr, nnz, NP, G, val64);
        } else {
            c->d_nuc32.reserve(nnz);
            swave_values(c, T, false, P0Dst{row_ptr, col, nnz, nullptr, c->d_nuc32.ptr}, measure);
            hipLaunchKernelGGL(k_spread_g<float>, dim3(blocks), dim3(256), 0, c->stream,
                               c->d_nuc32.ptr, nnz, NP, G, val32);
        }
        WPCD_HIP(hipGetLastError());
        return;
    }
    if (!c->swave) {
        NodeTab N{};
        for (int k = 0; k < c->ngx; ++k) {
            N.ux[k] = 1.0 + c->gx[k];
            N.wx[k] = c->wx[k];
        }
        McTab Mt{};
        Mt.npair = NP;
        if (!c->mc_direct)
            for (int p = 0; p < NP; ++p) Mt.p[p] = c->mc_pairs[p];
        const int64_t want = (nnz + 3) / 4;
        const int blocks = (int)(want < 65536 ? want : 65536);
        double *v64 = D.val64;
        float *v32 = D.val32;
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, c->stream, T, N, Mt,
                               c->d_mcoef.ptr, row_ptr, col, nnz, v64, v32);
        };
        TimedLaunch tl(c->timer, c->stream, fp64 ? "p0_elem_mc_f64" : "p0_elem_mc_f32",
                       WPCD_TIME_P0);
        int hmax = 0;
        for (int p = 0; p < NP; ++p) hmax = std::max(hmax, std::max(Mt.p[p].hl, Mt.p[p].hl2));
        // moments only for FP32 output: summing D_c M_c cancels more than the
        // node-by-node polynomial (a few 1e-13 of the largest element on
        // near-zero elements), which the FP64 tier does not accept
        const bool mom = !fp64 && !c->mc_direct && c->ngq == 8 && hmax <= 1 && c->mc_deg <= 4 &&
                         (NP == 1 || NP == 4 || NP == 9) &&
                         (c->ngx == 16 || c->ngx == 20 || c->ngx == 24 || c->ngx == 32);
        if (mom) {
            auto by_ngx = [&](auto np_c, auto f32_c) {
                constexpr int NPc = decltype(np_c)::value;
                constexpr bool F = decltype(f32_c)::value;
                switch (c->ngx) {
                    case 16: go(k_p0_mcm<NPc, 1, 4, 16, F>); break;
                    case 20: go(k_p0_mcm<NPc, 1, 4, 20, F>); break;
                    case 24: go(k_p0_mcm<NPc, 1, 4, 24, F>); break;
                    default: go(k_p0_mcm<NPc, 1, 4, 32, F>); break;
                }
            };
            if (NP == 1) by_ngx(std::integral_constant<int, 1>{}, std::true_type{});
            else if (NP == 4) by_ngx(std::integral_constant<int, 4>{}, std::true_type{});
            else by_ngx(std::integral_constant<int, 9>{}, std::true_type{});
        } else if (!c->mc_direct && c->mc_deg <= 4 && NP == 1) go(k_p0_mc<1, 4>);
        else if (!c->mc_direct && c->mc_deg <= 4 && NP == 4) go(k_p0_mc<4, 4>);
        else if (!c->mc_direct && c->mc_deg <= 4 && NP == 9) go(k_p0_mc<9, 4>);
        else {
            const int dblocks = (int)(nnz < 262144 ? nnz : 262144);
            hipLaunchKernelGGL(k_p0_mc_direct, dim3(dblocks), dim3(64), 0, c->stream, T, N,
                               c->d_mterms.ptr, c->d_mterm_first.ptr, NP, row_ptr, col, nnz,
                               v64, v32);
        }
        WPCD_HIP(hipGetLastError());
        return;
    }
    swave_values(c, T, fp64, D, measure);
}

// The s-wave element values of every cell pair into D (one value each).
static void swave_values(wpcd_ctx *c, const ElemTables &T, bool fp64, const P0Dst &D,
                         bool measure) {
    const int64_t nnz = D.nnz;
    const int64_t *row_ptr = D.row_ptr;
    const int32_t *col = D.col;
    if (c->ngq == 8) {
        NodeTab N{};
        for (int k = 0; k < c->ngx; ++k) {
            N.ux[k] = 1.0 + c->gx[k];
            N.wx[k] = c->wx[k];
            N.uxf[k] = (float)N.ux[k];
            N.wxf[k] = (float)N.wx[k];
        }
        char key[64];
        std::snprintf(key, sizeof key, "nnz=%lld ngx=%d %s", (long long)nnz, c->ngx,
                      fp64 ? "f64" : "f32");
        const int v = tune_pick(c, "p0_elem", key, 4, 0, [&](int i) {
            return time_launches_p0(c->stream, [&] {
                if (fp64) launch_compacted<false>(c, T, N, D, i);
                else launch_compacted<true>(c, T, N, D, i);
            });
        }, measure);
        if (fp64) {
            TimedLaunch tl(c->timer, c->stream, "p0_elem_f64", WPCD_TIME_P0);
            launch_compacted<false>(c, T, N, D, v);
        } else {
            TimedLaunch tl(c->timer, c->stream, "p0_elem_f32", WPCD_TIME_P0);
            launch_compacted<true>(c, T, N, D, v);
        }
        WPCD_HIP(hipGetLastError());
        return;
    }
    // general Gauss order: one wavefront per cell pair, lanes = (a, b)
    int64_t want = (nnz + 3) / 4;
    int blocks = (int)(want < 65536 ? want : 65536);
    if (fp64) {
        TimedLaunch tl(c->timer, c->stream, "p0_elem_f64", WPCD_TIME_P0);
        hipLaunchKernelGGL(k_p0_swave_f64, dim3(blocks), dim3(256), 0, c->stream, T, row_ptr, col,
                           nnz, D.val64);
        WPCD_HIP(hipGetLastError());
    } else {
        TimedLaunch tl(c->timer, c->stream, "p0_elem_f32", WPCD_TIME_P0);
        hipLaunchKernelGGL(k_p0_swave_f32, dim3(blocks), dim3(256), 0, c->stream, T, row_ptr, col,
                           nnz, D.val32);
        WPCD_HIP(hipGetLastError());
    }
}

void build_values(wpcd_ctx *c, bool fp64) {
    const int64_t nv = c->nnz * c->nch * c->nch;
    if (fp64) c->d_val64.reserve(nv);
    else c->d_val32.reserve(nv);
    values_into(c, fp64, c->d_rowptr.ptr, c->d_col.ptr, c->d_hint.ptr, c->d_rstart.ptr, c->nnz,
                c->d_val64.ptr, c->d_val32.ptr, true, true);
}

}  // namespace wpcd
