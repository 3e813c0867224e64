// Model matrix fills of Sec. IV.A: a micro-benchmark of filling a matrix
// whose elements are costly, dense (one thread per element, the paper's
// scheme) and sparse (eq.(Acond)), the latter either by filtering inside the
// dense launch or by selecting the kept elements first and evaluating only
// those with every lane busy.
//   eq.(Atrig): A(i, j) = sum_{k=1..K} (sin^k u_ij + cos^k w_ij)
//   eq.(Agau):  A(i, j) = sum_{k=1..K} int_{u_ij}^{w_ij} (sin^k t + cos^k t) dt,
//               48-point Gauss-Legendre
//   eq.(Acond): the element is kept where u_ij <= alpha, zero elsewhere.
// u_ij and w_ij are outputs 2 (i M + j) and 2 (i M + j) + 1 of the
// splitmix64 stream of `seed` (Steele, Lea, Flood 2014), computed in the
// counter-based form mix(seed + (n + 1) g), u = (x >> 11) 2^-53.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <vector>

#include "wpcd_internal.h"

namespace wpcd {

constexpr int kModelGauss = 48;

struct ModelTab {
    double x[kModelGauss], w[kModelGauss];   // Gauss-Legendre nodes (ascending) and weights
    float xf[kModelGauss], wf[kModelGauss];
};

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double model_uniform(uint64_t seed, uint64_t n) {
    return (double)(mix64(seed + (n + 1) * 0x9E3779B97F4A7C15ull) >> 11) * 0x1.0p-53;
}

// sum_{k=1..K} (a^k + b^k) by running products, in T
template <class T>
__device__ __forceinline__ T power_sum(T a, T b, int K) {
    T pa = a, pb = b, acc = (T)0;
    for (int k = 0; k < K; ++k) {
        acc += pa + pb;
        pa *= a;
        pb *= b;
    }
    return acc;
}

template <class T>
__device__ __forceinline__ T model_element(int kind, double u, double w, int K, const ModelTab &G) {
    if (kind == 0) return power_sum<T>((T)sin((T)u), (T)cos((T)w), K);
    const T half = (T)(0.5 * (w - u)), mid = (T)(0.5 * (w + u));
    T acc = (T)0;
    for (int g = 0; g < kModelGauss; ++g) {
        const T xg = sizeof(T) == 8 ? (T)G.x[g] : (T)G.xf[g];
        const T wg = sizeof(T) == 8 ? (T)G.w[g] : (T)G.wf[g];
        const T t = mid + half * xg;
        acc += wg * power_sum<T>((T)sin(t), (T)cos(t), K);
    }
    return half * acc;
}

// Dense fill, one thread per element; with filter (eq.(Acond)) the elements
// with u > alpha are written as zero without being evaluated.
template <class T, bool FILTER>
__global__ __launch_bounds__(256) void k_model_dense(int kind, int M, int K, uint64_t seed,
                                                     double alpha, ModelTab G,
                                                     T *__restrict__ out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)M * M) return;
    const double u = model_uniform(seed, 2 * (uint64_t)n), w = model_uniform(seed, 2 * (uint64_t)n + 1);
    if (FILTER && !(u <= alpha)) {
        out[n] = (T)0;
        return;
    }
    out[n] = model_element<T>(kind, u, w, K, G);
}

// Selection: segments of kModelSeg consecutive flat indices, one wavefront
// each (64 indices per step).  Count pass, then (after an exclusive scan of
// the counts) the write pass puts the kept indices in ascending order.
constexpr int kModelSeg = 1024;

template <bool WRITE>
__global__ __launch_bounds__(256) void k_model_select(int M, uint64_t seed, double alpha,
                                                      int32_t *__restrict__ cnt,
                                                      const int64_t *__restrict__ off,
                                                      int64_t *__restrict__ idx) {
    const int lane = threadIdx.x & 63;
    const int64_t seg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t total = (int64_t)M * M;
    const int64_t b0 = seg * kModelSeg;
    if (b0 >= total) return;
    int64_t pos = WRITE ? off[seg] : 0;
    int c = 0;
    for (int s = 0; s < kModelSeg; s += 64) {
        const int64_t n = b0 + s + lane;
        const bool keep = n < total && model_uniform(seed, 2 * (uint64_t)n) <= alpha;
        const unsigned long long m = __builtin_amdgcn_ballot_w64(keep);
        if (WRITE && keep) {
            const int rank = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            idx[pos + rank] = n;
        }
        pos += __popcll(m);
        c += __popcll(m);
    }
    if (!WRITE && lane == 0) cnt[seg] = c;
}

// Exclusive prefix sums of n counts (one workgroup; n <= 1024 * 64).
__global__ __launch_bounds__(1024) void k_model_scan(const int32_t *__restrict__ cnt, int n,
                                                     int64_t *__restrict__ off) {
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int beg = min(tid * per, n), end = min(beg + per, n);
    int64_t s = 0;
    for (int k = beg; k < end; ++k) s += cnt[k];
    part[tid] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = tid ? part[tid - 1] : 0;
    for (int k = beg; k < end; ++k) {
        off[k] = run;
        run += cnt[k];
    }
    if (tid == 1023) off[n] = part[1023];
}

// Evaluation of the selected elements, one thread each.
template <class T>
__global__ __launch_bounds__(256) void k_model_sparse(int kind, int K, uint64_t seed, ModelTab G,
                                                      const int64_t *__restrict__ idx, int64_t nnz,
                                                      T *__restrict__ val) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const uint64_t n = (uint64_t)idx[e];
    val[e] = model_element<T>(kind, model_uniform(seed, 2 * n), model_uniform(seed, 2 * n + 1), K, G);
}

void model_fill(wpcd_ctx *c, const ModelRequest &r, ModelResult &res) {
    hipStream_t s = c->stream;
    const int64_t total = (int64_t)r.M * r.M;
    ModelTab G{};
    std::vector<double> gx, gw;
    gauss_legendre_gw(kModelGauss, gx, gw);
    for (int g = 0; g < kModelGauss; ++g) {
        G.x[g] = gx[g];
        G.w[g] = gw[g];
        G.xf[g] = (float)gx[g];
        G.wf[g] = (float)gw[g];
    }
    hipEvent_t ev0, ev1;
    WPCD_HIP(hipEventCreate(&ev0));
    WPCD_HIP(hipEventCreate(&ev1));
    struct Events {
        hipEvent_t a, b;
        ~Events() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } evs{ev0, ev1};
    const size_t vsz = r.fp64 ? 8 : 4;
    res.nnz = total;
    if (r.mode != 2) {
        c->d_misc.reserve((size_t)(total * vsz + 7) / 8);
        void *out = c->d_misc.ptr;
        const dim3 grid((unsigned)((total + 255) / 256));
        WPCD_HIP(hipEventRecord(ev0, s));
        auto go = [&](auto t, auto filt) {
            using T = decltype(t);
            constexpr bool F = decltype(filt)::value;
            hipLaunchKernelGGL((k_model_dense<T, F>), grid, dim3(256), 0, s, r.kind, r.M, r.K,
                               r.seed, r.alpha, G, (T *)out);
        };
        if (r.fp64) {
            if (r.mode == 1) go(0.0, std::true_type{});
            else go(0.0, std::false_type{});
        } else {
            if (r.mode == 1) go(0.f, std::true_type{});
            else go(0.f, std::false_type{});
        }
        WPCD_HIP(hipGetLastError());
        WPCD_HIP(hipEventRecord(ev1, s));
        WPCD_HIP(hipEventSynchronize(ev1));
        float ms = 0.f;
        WPCD_HIP(hipEventElapsedTime(&ms, ev0, ev1));
        res.ms = ms;
        if (r.dense_out) {
            if (r.fp64) {
                WPCD_HIP(hipMemcpy(r.dense_out, out, total * 8, hipMemcpyDeviceToHost));
            } else {
                std::vector<float> h(total);
                WPCD_HIP(hipMemcpy(h.data(), out, total * 4, hipMemcpyDeviceToHost));
                for (int64_t n = 0; n < total; ++n) r.dense_out[n] = h[n];
            }
        }
        return;
    }
    // pre-selected: count, scan, select, evaluate
    const int64_t nseg = (total + kModelSeg - 1) / kModelSeg;
    WPCD_REQUIRE(nseg <= 1024 * 64, WPCD_E_INVALID, "matrix too large for the selection scan");
    c->d_cnt.reserve(nseg);
    c->d_tsum.reserve(nseg + 1);
    const dim3 sgrid((unsigned)((nseg + 3) / 4));
    WPCD_HIP(hipEventRecord(ev0, s));
    hipLaunchKernelGGL((k_model_select<false>), sgrid, dim3(256), 0, s, r.M, r.seed, r.alpha,
                       c->d_cnt.ptr, nullptr, nullptr);
    hipLaunchKernelGGL(k_model_scan, dim3(1), dim3(1024), 0, s, c->d_cnt.ptr, (int)nseg,
                       c->d_tsum.ptr);
    WPCD_HIP(hipGetLastError());
    int64_t nnz = 0;
    WPCD_HIP(hipMemcpyAsync(&nnz, c->d_tsum.ptr + nseg, 8, hipMemcpyDeviceToHost, s));
    WPCD_HIP(hipStreamSynchronize(s));
    res.nnz = nnz;
    // selected indices (8 B) then values, in one buffer
    c->d_misc.reserve((size_t)nnz * 2 + 1);
    int64_t *idx = (int64_t *)c->d_misc.ptr;
    void *val = c->d_misc.ptr + nnz;
    hipLaunchKernelGGL((k_model_select<true>), sgrid, dim3(256), 0, s, r.M, r.seed, r.alpha,
                       nullptr, c->d_tsum.ptr, idx);
    const dim3 egrid((unsigned)((nnz + 255) / 256 + (nnz == 0)));
    if (r.fp64)
        hipLaunchKernelGGL((k_model_sparse<double>), egrid, dim3(256), 0, s, r.kind, r.K, r.seed, G,
                           idx, nnz, (double *)val);
    else
        hipLaunchKernelGGL((k_model_sparse<float>), egrid, dim3(256), 0, s, r.kind, r.K, r.seed, G,
                           idx, nnz, (float *)val);
    WPCD_HIP(hipGetLastError());
    WPCD_HIP(hipEventRecord(ev1, s));
    WPCD_HIP(hipEventSynchronize(ev1));
    float ms = 0.f;
    WPCD_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    res.ms = ms;
    if (nnz > r.cap) return;   // the caller reads nnz and calls again
    if (r.idx_out) WPCD_HIP(hipMemcpy(r.idx_out, idx, nnz * 8, hipMemcpyDeviceToHost));
    if (r.val_out) {
        if (r.fp64) {
            WPCD_HIP(hipMemcpy(r.val_out, val, nnz * 8, hipMemcpyDeviceToHost));
        } else {
            std::vector<float> h(nnz);
            WPCD_HIP(hipMemcpy(h.data(), val, nnz * 4, hipMemcpyDeviceToHost));
            for (int64_t e = 0; e < nnz; ++e) r.val_out[e] = h[e];
        }
    }
}

}  // namespace wpcd
