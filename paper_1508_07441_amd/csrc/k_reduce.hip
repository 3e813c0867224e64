// Feshbach major/minor channel reduction (Sec. V.B): the lattice matrix P0
// of a reduced channel basis, built from the P0 of the unreduced one.
//
// The minor channels are described on a coarse lattice whose cells are
// unions of r_p x r_q fine cells (every r_p-th p edge, every r_q-th q edge).
// With unit-weight packets the packet of a union of bins is
// sum_i sqrt(d_i / D) |x_i>, so an element of P0 that involves a coarse cell
// is the same combination of fine elements (the element is an integral over
// the two cells, eqs.(perm),(gal)):
//   P0_red = R P0 R^T,  R = identity on the major channels, the weights
//   w(j, i) = sqrt(dq_j / DQ_J) sqrt(dp_i / DP_I) on the minor ones.
// Rows and columns of P0_red are the cells of the reduced basis: the major
// channels' fine cells (a ncell + j n_p + i), then the minor channels'
// coarse cells (n_major ncell + a' nccell + J n_pc + I).  It is stored as
// one scalar CSR (one value per entry) with the columns ascending.
//
// The pattern of a cell pair does not depend on the channel pair, so the
// work is organised per pattern cell: a fine cell (the rows of every major
// channel at that cell) or a coarse cell (the rows of every minor channel).
// One workgroup per pattern cell marks the fine columns (coarse cells only:
// the union over its fine rows) and the coarse columns its fine rows reach
// in LDS bitmaps; the count pass stores their sizes, the fill pass ranks
// them and accumulates the values in LDS, then writes its rows.
// Accumulation order is fixed: source fine rows in order, and within a row
// the columns by their offset inside their coarse cell, one offset per
// phase, so that no two contributions to one slot meet in a phase and
// every entry is summed in the same order on every run.
#include "wpcd_internal.h"

#include <cmath>

namespace wpcd {
namespace {

struct RedGeom {
    const int64_t *rp;   // unreduced row_ptr [ncell + 1]
    const int32_t *col;  // unreduced columns (fine cells)
    const double *val;   // unreduced values [nnz][nch][nch]
    const double *wp;    // packet weight of each fine p bin in its coarse bin [np]
    const double *wq;    // the same for the q bins [nq]
    int np, nq, cp, cq, npc;
    int nch, nmaj;
    int ncell, nccell;
    int wF, wC;          // bitmap words over the fine and the coarse cells
};

__device__ __forceinline__ int coarse_of(const RedGeom &g, int C) {
    const int jc = C / g.np, ic = C - jc * g.np;
    return (jc / g.cq) * g.npc + ic / g.cp;
}

// Fine row k of pattern cell x (0 <= k < cp*cq for a coarse cell).
__device__ __forceinline__ int source_row(const RedGeom &g, bool coarse, int cell, int k,
                                          double &w) {
    if (!coarse) {
        w = 1.0;
        return cell;
    }
    const int J = cell / g.npc, I = cell - J * g.npc;
    const int j = J * g.cq + k / g.cp, i = I * g.cp + k % g.cp;
    w = g.wq[j] * g.wp[i];
    return j * g.np + i;
}

// Exclusive prefix popcounts of n bitmap words into pre (256 threads).
__device__ void word_prefix(const uint32_t *bm, int n, int32_t *pre, int32_t *part) {
    const int t = threadIdx.x;
    const int per = (n + 255) / 256;
    const int w0 = min(n, t * per), w1 = min(n, w0 + per);
    int s = 0;
    for (int w = w0; w < w1; ++w) s += __popc(bm[w]);
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int k = 0; k < 256; ++k) {
            const int v = part[k];
            part[k] = run;
            run += v;
        }
        part[256] = run;
    }
    __syncthreads();
    s = part[t];
    for (int w = w0; w < w1; ++w) {
        pre[w] = s;
        s += __popc(bm[w]);
    }
}

// Cells [x0, x0 + gridDim.x) of the pattern-cell list (fine cells first,
// then coarse ones).  Count pass (FILL false): nF[x], nC[x] = sizes of the
// fine and coarse column sets.  Fill pass: rows of the cell into the
// reduced CSR (rrp, rcol, rval); nF, nC are read.
template <bool FILL>
__global__ __launch_bounds__(256) void k_reduce_p0(RedGeom g, int x0, int32_t *__restrict__ nF,
                                                   int32_t *__restrict__ nC,
                                                   const int64_t *__restrict__ rrp,
                                                   int32_t *__restrict__ rcol,
                                                   double *__restrict__ rval) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int32_t part[257];
    __shared__ int32_t red_n[2];
    const int t = threadIdx.x;
    const int x = x0 + (int)blockIdx.x;
    const bool coarse = x >= g.ncell;
    const int cell = coarse ? x - g.ncell : x;
    const int nsrc = coarse ? g.cp * g.cq : 1;
    const int wFu = coarse ? g.wF : 0;
    uint32_t *bmF = (uint32_t *)lds_raw;
    uint32_t *bmC = bmF + wFu;
    for (int w = t; w < wFu + g.wC; w += 256) bmF[w] = 0u;
    __syncthreads();
    for (int k = 0; k < nsrc; ++k) {
        double w;
        const int R = source_row(g, coarse, cell, k, w);
        for (int64_t e = g.rp[R] + t; e < g.rp[R + 1]; e += 256) {
            const int C = g.col[e];
            const int cc = coarse_of(g, C);
            atomicOr(&bmC[cc >> 5], 1u << (cc & 31));
            if (coarse) atomicOr(&bmF[C >> 5], 1u << (C & 31));
        }
    }
    __syncthreads();
    if (!FILL) {
        if (t < 2) red_n[t] = 0;
        __syncthreads();
        int sf = 0, sc = 0;
        for (int w = t; w < wFu; w += 256) sf += __popc(bmF[w]);
        for (int w = t; w < g.wC; w += 256) sc += __popc(bmC[w]);
        if (sf) atomicAdd(&red_n[0], sf);
        if (sc) atomicAdd(&red_n[1], sc);
        __syncthreads();
        if (t == 0) {
            nF[x] = coarse ? red_n[0] : (int32_t)(g.rp[cell + 1] - g.rp[cell]);
            nC[x] = red_n[1];
        }
        return;
    }
    const int nf = nF[x], nc = nC[x];
    const int nmin = g.nch - g.nmaj;
    const int nrows = coarse ? nmin : g.nmaj;
    int32_t *preF = (int32_t *)(bmC + g.wC);
    int32_t *preC = preF + wFu;
    int32_t *setF = preC + g.wC;   // coarse cells only
    int32_t *setC = setF + (coarse ? nf : 0);
    size_t off = (size_t)((unsigned char *)(setC + nc) - lds_raw);
    off = (off + 7) & ~(size_t)7;
    double *accF = (double *)(lds_raw + off);
    double *accC = accF + (size_t)nrows * g.nmaj * nf;
    const int nacc = nrows * (g.nmaj * nf + nmin * nc);
    if (coarse) word_prefix(bmF, g.wF, preF, part);
    __syncthreads();
    word_prefix(bmC, g.wC, preC, part);
    for (int k = t; k < nacc; k += 256) accF[k] = 0.0;
    __syncthreads();
    // the sorted column sets
    for (int w = t; w < wFu; w += 256) {
        uint32_t b = bmF[w];
        int p = preF[w];
        while (b) {
            const int s = __ffs(b) - 1;
            setF[p++] = w * 32 + s;
            b &= b - 1;
        }
    }
    for (int w = t; w < g.wC; w += 256) {
        uint32_t b = bmC[w];
        int p = preC[w];
        while (b) {
            const int s = __ffs(b) - 1;
            setC[p++] = w * 32 + s;
            b &= b - 1;
        }
    }
    // accumulation, one (source row, offset in the coarse cell) per phase
    const int noff = g.cp * g.cq;
    for (int k = 0; k < nsrc; ++k) {
        double wr;
        const int R = source_row(g, coarse, cell, k, wr);
        const int64_t e0 = g.rp[R], e1 = g.rp[R + 1];
        for (int o = 0; o < noff; ++o) {
            __syncthreads();
            for (int64_t e = e0 + t; e < e1; e += 256) {
                const int C = g.col[e];
                const int jc = C / g.np, ic = C - jc * g.np;
                if ((jc % g.cq) * g.cp + ic % g.cp != o) continue;
                int fpos;
                if (coarse) {
                    const uint32_t m = bmF[C >> 5] & ((1u << (C & 31)) - 1u);
                    fpos = preF[C >> 5] + __popc(m);
                } else {
                    fpos = (int)(e - e0);
                }
                const int cc = (jc / g.cq) * g.npc + ic / g.cp;
                const int cpos = preC[cc >> 5] + __popc(bmC[cc >> 5] & ((1u << (cc & 31)) - 1u));
                const double wc = wr * g.wq[jc] * g.wp[ic];
                for (int ar = 0; ar < nrows; ++ar) {
                    const int a = coarse ? g.nmaj + ar : ar;
                    const double *v = g.val + ((size_t)e * g.nch + a) * g.nch;
                    for (int b = 0; b < g.nmaj; ++b)
                        accF[((size_t)ar * g.nmaj + b) * nf + fpos] += wr * v[b];
                    for (int b = 0; b < nmin; ++b)
                        accC[((size_t)ar * nmin + b) * nc + cpos] += wc * v[g.nmaj + b];
                }
            }
        }
    }
    __syncthreads();
    const int64_t mf = (int64_t)g.nmaj * g.ncell;
    for (int ar = 0; ar < nrows; ++ar) {
        const int64_t r = coarse ? mf + (int64_t)ar * g.nccell + cell : (int64_t)ar * g.ncell + cell;
        const int64_t base = rrp[r];
        for (int k = t; k < g.nmaj * nf; k += 256) {
            const int b = k / nf, s = k - b * nf;
            const int C = coarse ? setF[s] : g.col[g.rp[cell] + s];
            rcol[base + k] = b * g.ncell + C;
            rval[base + k] = accF[((size_t)ar * g.nmaj + b) * nf + s];
        }
        const int64_t base2 = base + (int64_t)g.nmaj * nf;
        for (int k = t; k < nmin * nc; k += 256) {
            const int b = k / nc, s = k - b * nc;
            rcol[base2 + k] = (int32_t)(mf + (int64_t)b * g.nccell + setC[s]);
            rval[base2 + k] = accC[((size_t)ar * nmin + b) * nc + s];
        }
    }
}

// Row lengths of the reduced CSR from the per-cell set sizes.
__global__ void k_reduce_rows(const int32_t *__restrict__ nF, const int32_t *__restrict__ nC,
                              int ncell, int nccell, int nmaj, int nmin, int64_t nrow,
                              int32_t *__restrict__ cnt) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrow) return;
    const int64_t mf = (int64_t)nmaj * ncell;
    const int x = r < mf ? (int)(r % ncell) : ncell + (int)((r - mf) % nccell);
    cnt[r] = nmaj * nF[x] + nmin * nC[x];
}

// Exclusive scan of n row lengths into row_ptr[n + 1] (one workgroup of
// 1024 threads, each a contiguous run of rows).
__global__ __launch_bounds__(1024) void k_reduce_scan(const int32_t *__restrict__ cnt, int64_t n,
                                                      int64_t *__restrict__ row_ptr) {
    __shared__ int64_t part[1025];
    const int t = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t r0 = min(n, (int64_t)t * per), r1 = min(n, r0 + per);
    int64_t s = 0;
    for (int64_t r = r0; r < r1; r += 8) {   // eight loads in flight
        int32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = r + u < r1 ? cnt[r + u] : 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    s = t ? part[t - 1] : 0;
    for (int64_t r = r0; r < r1; r += 8) {
        int32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = r + u < r1 ? cnt[r + u] : 0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (r + u < r1) {
                row_ptr[r + u] = s;
                s += v[u];
            }
    }
    if (t == 1023) row_ptr[n] = part[1023];
}

__global__ void k_to_f32(const double *__restrict__ v, int64_t n, float *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = (float)v[k];
}

// Device scratch freed when it leaves scope (also on an error).
template <class T>
struct TmpBuf : DBuf<T> {
    ~TmpBuf() { this->release(); }
};

// Dynamic LDS of the fill pass for a cell with column sets of nf and nc.
size_t fill_lds(const RedGeom &g, bool coarse, int nf, int nc) {
    const int wFu = coarse ? g.wF : 0;
    const int nmin = g.nch - g.nmaj;
    const int nrows = coarse ? nmin : g.nmaj;
    size_t b = (size_t)4 * (2 * (wFu + g.wC) + (coarse ? nf : 0) + nc);
    b = (b + 7) & ~(size_t)7;
    return b + (size_t)8 * nrows * ((size_t)g.nmaj * nf + (size_t)nmin * nc);
}

}  // namespace

constexpr size_t kReduceLdsMax = 160 * 1024 - 2 * 1024;   // beside the static arrays

void reduce_p0(wpcd_ctx *full, wpcd_ctx *red, int nmaj, int cp, int cq, const double *d_val64,
               bool keep32) {
    hipStream_t s = red->stream;
    RedGeom g{};
    g.np = full->np;
    g.nq = full->nq;
    g.cp = cp;
    g.cq = cq;
    g.npc = full->np / cp;
    g.nch = full->nch;
    g.nmaj = nmaj;
    g.ncell = full->np * full->nq;
    g.nccell = (full->np / cp) * (full->nq / cq);
    g.wF = (g.ncell + 31) / 32;
    g.wC = (g.nccell + 31) / 32;
    WPCD_REQUIRE((size_t)4 * 2 * (g.wF + g.wC) <= kReduceLdsMax / 2, WPCD_E_INVALID,
                 "lattice too large for the reduction's LDS bitmaps");
    // packet weights of the fine bins in their coarse bins
    std::vector<double> wp(g.np), wq(g.nq);
    for (int i = 0; i < g.np; ++i) {
        const int I = i / cp;
        wp[i] = std::sqrt((full->p[i + 1] - full->p[i]) / (full->p[(I + 1) * cp] - full->p[I * cp]));
    }
    for (int j = 0; j < g.nq; ++j) {
        const int J = j / cq;
        wq[j] = std::sqrt((full->q[j + 1] - full->q[j]) / (full->q[(J + 1) * cq] - full->q[J * cq]));
    }
    TmpBuf<double> dw;
    dw.reserve(g.np + g.nq);
    WPCD_HIP(hipMemcpyAsync(dw.ptr, wp.data(), g.np * sizeof(double), hipMemcpyHostToDevice, s));
    WPCD_HIP(hipMemcpyAsync(dw.ptr + g.np, wq.data(), g.nq * sizeof(double),
                            hipMemcpyHostToDevice, s));
    g.rp = full->d_rowptr.ptr;
    g.col = full->d_col.ptr;
    g.val = d_val64;
    g.wp = dw.ptr;
    g.wq = dw.ptr + g.np;
    const int ncx = g.ncell + g.nccell;
    const int nmin = g.nch - nmaj;
    const int64_t nrow = (int64_t)nmaj * g.ncell + (int64_t)nmin * g.nccell;
    TmpBuf<int32_t> dn, dcnt;
    dn.reserve(2 * (size_t)ncx);
    dcnt.reserve(nrow);
    int32_t *nF = dn.ptr, *nC = dn.ptr + ncx;
    const size_t bm_fine = (size_t)4 * g.wC, bm_coarse = (size_t)4 * (g.wF + g.wC);
    WPCD_HIP(hipFuncSetAttribute((const void *)k_reduce_p0<false>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bm_coarse));
    {
        TimedLaunch tl(red->timer, s, "reduce_count", WPCD_TIME_P0);
        hipLaunchKernelGGL(k_reduce_p0<false>, dim3(g.ncell), dim3(256), bm_fine, s, g, 0, nF, nC,
                           nullptr, nullptr, nullptr);
        hipLaunchKernelGGL(k_reduce_p0<false>, dim3(g.nccell), dim3(256), bm_coarse, s, g, g.ncell,
                           nF, nC, nullptr, nullptr, nullptr);
        WPCD_HIP(hipGetLastError());
    }
    // LDS of the fill pass: the largest cell of each kind
    std::vector<int32_t> hn(2 * (size_t)ncx);
    WPCD_HIP(hipMemcpyAsync(hn.data(), dn.ptr, hn.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                            s));
    red->d_rowptr.reserve(nrow + 1);
    {
        TimedLaunch tl(red->timer, s, "reduce_scan", WPCD_TIME_P0);
        hipLaunchKernelGGL(k_reduce_rows, dim3((unsigned)((nrow + 255) / 256)), dim3(256), 0, s, nF,
                           nC, g.ncell, g.nccell, nmaj, nmin, nrow, dcnt.ptr);
        hipLaunchKernelGGL(k_reduce_scan, dim3(1), dim3(1024), 0, s, dcnt.ptr, nrow,
                           red->d_rowptr.ptr);
        WPCD_HIP(hipGetLastError());
    }
    int64_t nnz = 0;
    WPCD_HIP(hipMemcpyAsync(&nnz, red->d_rowptr.ptr + nrow, sizeof(int64_t),
                            hipMemcpyDeviceToHost, s));
    WPCD_HIP(hipStreamSynchronize(s));
    WPCD_REQUIRE(nnz < ((int64_t)1 << 31), WPCD_E_INVALID, "reduced P0 exceeds 2^31 entries");
    size_t lf = 0, lc = 0;
    for (int x = 0; x < g.ncell; ++x) lf = std::max(lf, fill_lds(g, false, hn[x], hn[ncx + x]));
    for (int x = g.ncell; x < ncx; ++x) lc = std::max(lc, fill_lds(g, true, hn[x], hn[ncx + x]));
    WPCD_REQUIRE(lf <= kReduceLdsMax && lc <= kReduceLdsMax, WPCD_E_INVALID,
                 "a reduced row set exceeds one workgroup's LDS");
    WPCD_HIP(hipFuncSetAttribute((const void *)k_reduce_p0<true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)std::max(lf, lc)));
    red->d_col.reserve(nnz);
    red->d_val64.reserve(nnz);
    {
        TimedLaunch tl(red->timer, s, "reduce_fill", WPCD_TIME_P0);
        hipLaunchKernelGGL(k_reduce_p0<true>, dim3(g.ncell), dim3(256), lf, s, g, 0, nF, nC,
                           red->d_rowptr.ptr, red->d_col.ptr, red->d_val64.ptr);
        hipLaunchKernelGGL(k_reduce_p0<true>, dim3(g.nccell), dim3(256), lc, s, g, g.ncell, nF, nC,
                           red->d_rowptr.ptr, red->d_col.ptr, red->d_val64.ptr);
        WPCD_HIP(hipGetLastError());
    }
    if (keep32) {
        red->d_val32.reserve(nnz);
        hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s,
                           red->d_val64.ptr, nnz, red->d_val32.ptr);
        WPCD_HIP(hipGetLastError());
    }
    WPCD_HIP(hipStreamSynchronize(s));
    red->nnz = nnz;
}

}  // namespace wpcd
