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

// Column range [lo, hi) of row cell (i, j) within column spectator bin j2.
// Selection (a necessary condition for a nonzero element): the two cells'
// energy ranges p^2 + 3/4 q^2 overlap, |q' + q/2| can fall in D_i, and
// |q + q'/2| can fall in D_i'.
__device__ __forceinline__ void col_range(const GridView &g, int i, int j, int j2, int &lo,
                                          int &hi) {
    lo = 0;
    hi = 0;
    // pi1 = |q' + q/2| over q in bin j, q' in bin j2
    double d1 = 0.0, a;
    a = g.q[j2] - g.H[j + 1];
    if (a > d1) d1 = a;
    a = g.H[j] - g.q[j2 + 1];
    if (a > d1) d1 = a;
    if (!(g.p[i + 1] > d1 && g.p[i] < g.q[j2 + 1] + g.H[j + 1])) return;
    const double elo = g.P2[i] + g.Q34[j];
    const double ehi = g.P2[i + 1] + g.Q34[j + 1];
    const double q34lo = g.Q34[j2], q34hi = g.Q34[j2 + 1];
    double d2 = 0.0;
    a = g.q[j] - g.H[j2 + 1];
    if (a > d2) d2 = a;
    a = g.H[j2] - g.q[j + 1];
    if (a > d2) d2 = a;
    const double pmax2 = g.q[j + 1] + g.H[j2 + 1];
    const int n = g.np;
    // i2 >= first with  P2[i2+1] + Q34[j2+1] > elo
    int la = first_true(0, n, [&](int k) { return g.P2[k + 1] + q34hi > elo; });
    // i2 >= first with  p[i2+1] > d2
    int lc = first_true(0, n, [&](int k) { return g.p[k + 1] > d2; });
    // i2 <  first with  !(ehi > P2[i2] + Q34[j2])
    int hb = first_true(0, n, [&](int k) { return !(ehi > g.P2[k] + q34lo); });
    // i2 <  first with  !(p[i2] < pmax2)
    int hd = first_true(0, n, [&](int k) { return !(g.p[k] < pmax2); });
    lo = la > lc ? la : lc;
    hi = hb < hd ? hb : hd;
    if (hi < lo) hi = lo;
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

// One wavefront per row cell (rows strided over the grid); lanes sweep the
// column spectator bins.  cnt[row] = selected cells of the row; ranges[row]
// [j2] = lo | hi << 16 (the column range of bin j2, n_p < 2^16).
__global__ __launch_bounds__(256) void k_count(GridView g0, int32_t *__restrict__ cnt,
                                               uint32_t *__restrict__ ranges) {
    extern __shared__ double sgrid[];
    const GridView g = stage_grid(g0, sgrid);
    const int lane = threadIdx.x & 63;
    const int nrow = g.np * g.nq;
    for (int row = blockIdx.x * 4 + (threadIdx.x >> 6); row < nrow; row += gridDim.x * 4) {
        const int i = row % g.np, j = row / g.np;
        int c = 0;
        for (int j2 = lane; j2 < g.nq; j2 += 64) {
            int lo, hi;
            col_range(g, i, j, j2, lo, hi);
            c += hi - lo;
            ranges[(int64_t)row * g.nq + j2] = (uint32_t)lo | ((uint32_t)hi << 16);
        }
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
        if (lane == 0) cnt[row] = c;
    }
}

// Exclusive prefix sum of cnt[0..n) into row_ptr[0..n] for n <= 32768, one
// workgroup with the counts in LDS: each thread sums a contiguous segment,
// the 1024 segment sums are scanned, then row_ptr is written coalesced from
// segment bases and in-segment offsets.
__global__ __launch_bounds__(1024) void k_scan_lds(const int32_t *__restrict__ cnt, int n,
                                                   int64_t *__restrict__ row_ptr) {
    __shared__ int32_t sc[32768];
    __shared__ int64_t base[1024];
    const int tid = threadIdx.x;
    for (int k = tid; k < n; k += 1024) sc[k] = cnt[k];
    __syncthreads();
    const int per = (n + 1023) / 1024;
    const int beg = min(tid * per, n), end = min(beg + per, n);
    int32_t run = 0;
    for (int k = beg; k < end; ++k) {
        const int32_t v = sc[k];
        sc[k] = run;   // offset within the segment (< 2^31: per * 2^20 cells)
        run += v;
    }
    // inclusive scan of the 1024 segment sums: within each wavefront by
    // shuffles, then across the 16 wavefront totals
    __shared__ int64_t wtot[16];
    const int lane = tid & 63, wv = tid >> 6;
    int64_t incl = run;
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wtot[wv] = incl;
    __syncthreads();
    if (wv == 0) {
        int64_t t = lane < 16 ? wtot[lane] : 0;
        for (int off = 1; off < 16; off <<= 1) {
            const int64_t v = __shfl_up(t, off, 64);
            if (lane >= off) t += v;
        }
        if (lane < 16) wtot[lane] = t;
    }
    __syncthreads();
    base[tid] = incl + (wv ? wtot[wv - 1] : 0);
    __syncthreads();
    // base[t] is now the inclusive sum of segments 0..t
    for (int k = tid; k < n; k += 1024) {
        const int sgm = k / per;
        row_ptr[k] = (sgm ? base[sgm - 1] : 0) + sc[k];
    }
    if (tid == 0) row_ptr[n] = base[1023];
}

// Exclusive prefix sum of cnt[0..n) into row_ptr[0..n], one workgroup.
__global__ __launch_bounds__(1024) void k_scan(const int32_t *__restrict__ cnt, int n,
                                               int64_t *__restrict__ row_ptr) {
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int beg = tid * per;
    const int end = min(beg + per, n);
    int64_t s = 0;
    for (int k = beg; k < end; ++k) s += cnt[k];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = tid ? part[tid - 1] : 0;
    for (int k = beg; k < end; ++k) {
        row_ptr[k] = run;
        run += cnt[k];
    }
    if (tid == 1023) row_ptr[n] = part[1023];
}

// One wavefront per row cell (rows strided over the grid, the same number
// of passes for every wavefront): the column ranges from k_count ->
// coalesced column writes in ascending order (column index c = j2*np + i2).
__global__ __launch_bounds__(256) void k_fill(int np, int nq, const uint32_t *__restrict__ ranges,
                                              const int64_t *__restrict__ row_ptr,
                                              int32_t *__restrict__ col,
                                              int32_t *__restrict__ rowidx) {
    __shared__ int s_off[4][65];
    __shared__ int s_lo[4][64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int nrow = np * nq;
    const int stride = gridDim.x * 4;
    const int passes = (nrow + stride - 1) / stride;
    for (int ps = 0; ps < passes; ++ps) {
        const int row = ps * stride + blockIdx.x * 4 + w;
        const bool valid = row < nrow;
        int64_t base = valid ? row_ptr[row] : 0;
        for (int j0 = 0; j0 < nq; j0 += 64) {
            const int j2 = j0 + lane;
            int lo = 0, c = 0;
            if (valid && j2 < nq) {
                const uint32_t rg = ranges[(int64_t)row * nq + j2];
                lo = (int)(rg & 0xffffu);
                c = (int)(rg >> 16) - lo;
            }
            // inclusive scan across the wavefront
            int incl = c;
            for (int off = 1; off < 64; off <<= 1) {
                int v = __shfl_up(incl, off, 64);
                if (lane >= off) incl += v;
            }
            s_off[w][lane + 1] = incl;
            if (lane == 0) s_off[w][0] = 0;
            s_lo[w][lane] = lo;
            __syncthreads();
            const int total = s_off[w][64];
            for (int t = lane; t < total; t += 64) {
                // owner lane: last k with s_off[k] <= t
                int a = 0, b = 63;
                while (a < b) {
                    int m = (a + b + 1) >> 1;
                    if (s_off[w][m] <= t) a = m;
                    else b = m - 1;
                }
                int i2 = s_lo[w][a] + (t - s_off[w][a]);
                col[base + t] = (j0 + a) * np + i2;
                rowidx[base + t] = row;
            }
            base += total;
            __syncthreads();
        }
    }
}

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
                                                      const int32_t *__restrict__ rowidx,
                                                      const int32_t *__restrict__ col, int64_t nnz,
                                                      double *__restrict__ val) {
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int npair = T.ngq * T.ngq;
    for (int64_t e = wave0; e < nnz; e += nwaves) {
        const int r = rowidx[e], c = col[e];
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
                                                      const int32_t *__restrict__ rowidx,
                                                      const int32_t *__restrict__ col, int64_t nnz,
                                                      float *__restrict__ val) {
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int npair = T.ngq * T.ngq;
    for (int64_t e = wave0; e < nnz; e += nwaves) {
        const int r = rowidx[e], c = col[e];
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
                                                    const int32_t *__restrict__ rowidx,
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
        QLim QL{};
        RowLim RL{};
        double wq = 0.0, wr = 0.0;
#pragma unroll
        for (int k = 0; k < kEC; ++k) {
            unsigned long long m = 0;
            if (k < nrem) {
                // the cell pair is the same for the whole wavefront
                const int64_t e = chunk * kEC + k;
                int i, j, i2, j2;
                cell_ij(T, (uint32_t)__builtin_amdgcn_readfirstlane(rowidx[e]), i, j);
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
                                               const int32_t *__restrict__ rowidx,
                                               const int32_t *__restrict__ col, int64_t nnz,
                                               double *__restrict__ val64, float *__restrict__ val32) {
    __shared__ double red[4][NP][64];
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int npair_q = T.ngq * T.ngq;
    for (int64_t e = wave0; e < nnz; e += nwaves) {
        const int r = rowidx[e], c = col[e];
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
                                                const int32_t *__restrict__ rowidx,
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
        cell_ij(T, (uint32_t)__builtin_amdgcn_readfirstlane(rowidx[e]), i, j);
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
                                                     const int32_t *__restrict__ rowidx,
                                                     const int32_t *__restrict__ col, int64_t nnz,
                                                     double *__restrict__ val64,
                                                     float *__restrict__ val32) {
    constexpr int PC = 16;
    __shared__ double P1[15][64], Pq[15][64], P2[15][64];
    const int lane = threadIdx.x;
    const int npair_q = T.ngq * T.ngq;
    for (int64_t e = blockIdx.x; e < nnz; e += gridDim.x) {
        int i, j, i2, j2;
        cell_ij(T, (uint32_t)__builtin_amdgcn_readfirstlane(rowidx[e]), i, j);
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

void build_structure(wpcd_ctx *c) {
    const int nrow = c->np * c->nq;
    GridView g = grid_view(c);
    c->d_cnt.reserve(nrow);
    c->d_rowptr.reserve((size_t)nrow + 1);
    c->d_ranges.reserve((size_t)nrow * c->nq);
    const int blocks = std::min((nrow + 3) / 4, 2048);
    const size_t lds = (size_t)(2 * (c->np + 1) + 3 * (c->nq + 1)) * sizeof(double);
    {
        TimedLaunch tl(c->timer, c->stream, "preselect_count", WPCD_TIME_P0);
        hipLaunchKernelGGL(k_count, dim3(blocks), dim3(256), lds, c->stream, g, c->d_cnt.ptr,
                           c->d_ranges.ptr);
        WPCD_HIP(hipGetLastError());
    }
    {
        TimedLaunch tl(c->timer, c->stream, "preselect_scan", WPCD_TIME_P0);
        if (nrow <= 32768)
            hipLaunchKernelGGL(k_scan_lds, dim3(1), dim3(1024), 0, c->stream, c->d_cnt.ptr, nrow,
                               c->d_rowptr.ptr);
        else
            hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, c->stream, c->d_cnt.ptr, nrow,
                               c->d_rowptr.ptr);
        WPCD_HIP(hipGetLastError());
    }
    int64_t nnz = 0;
    WPCD_HIP(hipMemcpyAsync(&nnz, c->d_rowptr.ptr + nrow, sizeof(int64_t), hipMemcpyDeviceToHost,
                            c->stream));
    WPCD_HIP(hipStreamSynchronize(c->stream));
    WPCD_REQUIRE(nnz >= 0 && nnz < ((int64_t)1 << 40), WPCD_E_DEVICE, "bad nonzero count");
    c->nnz = nnz;
    c->d_col.reserve(nnz);
    c->d_rowidx.reserve(nnz);
    {
        TimedLaunch tl(c->timer, c->stream, "preselect_fill", WPCD_TIME_P0);
        hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, c->stream, c->np, c->nq,
                           c->d_ranges.ptr, c->d_rowptr.ptr, c->d_col.ptr, c->d_rowidx.ptr);
        WPCD_HIP(hipGetLastError());
    }
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

template <bool F32, int EC>
static void launch_compacted_ec(wpcd_ctx *c, const ElemTables &T, const NodeTab &N,
                                int64_t max_blocks) {
    const int64_t nchunk = (c->nnz + EC - 1) / EC;
    const int64_t want = (nchunk + 3) / 4;
    const int blocks = (int)(want < max_blocks ? want : max_blocks);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, c->stream, T, N, c->d_rowidx.ptr,
                           c->d_col.ptr, c->nnz, c->d_val64.ptr, c->d_val32.ptr);
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
static void launch_compacted(wpcd_ctx *c, const ElemTables &T, const NodeTab &N, int v) {
    const ElemVariant ev = kElemVariants[v];
    if (ev.ec == 8) launch_compacted_ec<F32, 8>(c, T, N, ev.max_blocks);
    else launch_compacted_ec<F32, 4>(c, T, N, ev.max_blocks);
}

void build_values(wpcd_ctx *c, bool fp64) {
    ElemTables T{c->d_P2.ptr, c->d_rsd_p.ptr, c->d_rsd_q.ptr, c->d_qnode.ptr, c->d_qwt.ptr,
                 c->d_ux.ptr,  c->d_wx.ptr,    c->d_uxf.ptr,   c->d_wxf.ptr,   c->np,
                 c->ngq,       c->ngx,
                 (uint32_t)(((1ull << 32) + (uint64_t)c->np - 1) / (uint64_t)c->np)};
    const int64_t nnz = c->nnz;
    const int NP = c->nch * c->nch;
    if (fp64) c->d_val64.reserve(nnz * NP);
    else c->d_val32.reserve(nnz * NP);
    if (nnz == 0) return;
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
        double *v64 = fp64 ? c->d_val64.ptr : nullptr;
        float *v32 = fp64 ? nullptr : c->d_val32.ptr;
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, c->stream, T, N, Mt,
                               c->d_mcoef.ptr, c->d_rowidx.ptr, c->d_col.ptr, nnz, v64, v32);
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
                               c->d_mterms.ptr, c->d_mterm_first.ptr, NP, c->d_rowidx.ptr,
                               c->d_col.ptr, nnz, v64, v32);
        }
        WPCD_HIP(hipGetLastError());
        return;
    }
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
                if (fp64) launch_compacted<false>(c, T, N, i);
                else launch_compacted<true>(c, T, N, i);
            });
        });
        if (fp64) {
            TimedLaunch tl(c->timer, c->stream, "p0_elem_f64", WPCD_TIME_P0);
            launch_compacted<false>(c, T, N, v);
        } else {
            TimedLaunch tl(c->timer, c->stream, "p0_elem_f32", WPCD_TIME_P0);
            launch_compacted<true>(c, T, N, v);
        }
        WPCD_HIP(hipGetLastError());
        return;
    }
    // general Gauss order: one wavefront per cell pair, lanes = (a, b)
    int64_t want = (nnz + 3) / 4;
    int blocks = (int)(want < 65536 ? want : 65536);
    if (fp64) {
        TimedLaunch tl(c->timer, c->stream, "p0_elem_f64", WPCD_TIME_P0);
        hipLaunchKernelGGL(k_p0_swave_f64, dim3(blocks), dim3(256), 0, c->stream, T,
                           c->d_rowidx.ptr, c->d_col.ptr, nnz, c->d_val64.ptr);
        WPCD_HIP(hipGetLastError());
    } else {
        TimedLaunch tl(c->timer, c->stream, "p0_elem_f32", WPCD_TIME_P0);
        hipLaunchKernelGGL(k_p0_swave_f32, dim3(blocks), dim3(256), 0, c->stream, T,
                           c->d_rowidx.ptr, c->d_col.ptr, nnz, c->d_val32.ptr);
        WPCD_HIP(hipGetLastError());
    }
}

}  // namespace wpcd
