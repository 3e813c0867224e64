// Warm-start network for the solve: a multilayer perceptron (tanh hidden
// layers, linear output) with BF16 weights and FP32 accumulation, trained by
// Adam on solutions of the plain solve.  Forward and backward passes are
// strided tiled GEMMs plus elementwise kernels.  This is not part of the
// paper's method: it only proposes the initial vector of the Krylov solve,
// whose residual decides whether the proposal is kept.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "wpcd_internal.h"

namespace wpcd {

__device__ __forceinline__ float bf16_to_f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }

__device__ __forceinline__ uint16_t f_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even (finite inputs)
    return (uint16_t)(u >> 16);
}

template <class T>
__device__ __forceinline__ float ld_f(const T *p, int64_t i);
template <>
__device__ __forceinline__ float ld_f<float>(const float *p, int64_t i) {
    return p[i];
}
template <>
__device__ __forceinline__ float ld_f<uint16_t>(const uint16_t *p, int64_t i) {
    return bf16_to_f(p[i]);
}

// C[m][n] = sum_k A[m*sam + k*sak] B[n*sbn + k*sbk]  (+ bias[n], tanh)
// Tiles 64 x 64, k-step 16; 256 threads, 4 x 4 outputs each.
enum { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_TANH = 2 };

template <class TA, class TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const TA *__restrict__ A,
                                              int64_t sam, int64_t sak, const TB *__restrict__ B,
                                              int64_t sbn, int64_t sbk,
                                              const float *__restrict__ bias,
                                              float *__restrict__ C, int64_t ldc) {
    __shared__ float sA[16][64 + 1], sB[16][64 + 1];
    const int t = threadIdx.x;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int tm = (t / 16) * 4, tn = (t % 16) * 4;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int idx = t; idx < 16 * 64; idx += 256) {
            const int kk = idx / 64, r = idx % 64;
            const int m = m0 + r, n = n0 + r, k = k0 + kk;
            sA[kk][r] = (m < M && k < K) ? ld_f<TA>(A, (int64_t)m * sam + (int64_t)k * sak) : 0.f;
            sB[kk][r] = (n < N && k < K) ? ld_f<TB>(B, (int64_t)n * sbn + (int64_t)k * sbk) : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = sA[kk][tm + u];
                b[u] = sB[kk][tn + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(a[u], b[v], acc[u][v]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int m = m0 + tm + u, n = n0 + tn + v;
            if (m < M && n < N) {
                float x = acc[u][v];
                if (EPI != EPI_NONE) x += bias[n];
                if (EPI == EPI_BIAS_TANH) x = tanhf(x);
                C[(int64_t)m * ldc + n] = x;
            }
        }
}

// dZ = dH (1 - H^2)
__global__ void k_tanh_bwd(const float *__restrict__ H, float *__restrict__ dH, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dH[i] *= (1.f - H[i] * H[i]);
}

// dY = 2 (Y - T) / B; per-row partial of the squared error.
__global__ void k_mse(const float *__restrict__ Y, const float *__restrict__ T, int B, int nout,
                      float *__restrict__ dY, float *__restrict__ rowloss) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float s = 0.f;
    for (int o = 0; o < nout; ++o) {
        const float d = Y[(int64_t)b * nout + o] - T[(int64_t)b * nout + o];
        s += d * d;
        dY[(int64_t)b * nout + o] = 2.f * d / (float)B;
    }
    rowloss[b] = s;
}

// db[n] = sum_b dZ[b][n]
__global__ void k_colsum(const float *__restrict__ dZ, int B, int N, float *__restrict__ db) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += dZ[(int64_t)b * N + n];
    db[n] = s;
}

// Adam on the FP32 master copy; refresh the BF16 weights.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, uint16_t *__restrict__ w16, int64_t n, float lr,
                       float b1, float b2, float c1, float c2, float eps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    w16[i] = f_to_bf16(wi);
}

// dst[i][:] = src[idx[i]][:]
__global__ void k_gather_rows(const float *__restrict__ src, int ncol, const int32_t *__restrict__ idx,
                              int n, float *__restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * ncol) return;
    const int i = (int)(t / ncol), k = (int)(t % ncol);
    dst[t] = src[(int64_t)idx[i] * ncol + k];
}

__global__ void k_to_bf16(const float *__restrict__ w, uint16_t *__restrict__ w16, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w16[i] = f_to_bf16(w[i]);
}

// ------------------------------------------------------------------ host
static inline int gdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

int64_t Mlp::n_params() const {
    int64_t n = 0;
    for (int l = 0; l < 4; ++l) n += (int64_t)dout(l) * din(l) + dout(l);
    return n;
}

int64_t Mlp::w_off(int l) const {
    int64_t o = 0;
    for (int k = 0; k < l; ++k) o += (int64_t)dout(k) * din(k) + dout(k);
    return o;
}

// A is FP32 activations, B either BF16 weights or FP32 activations.
static void gemm_launch(hipStream_t s, int epi, bool b_bf16, int M, int N, int K, const float *A,
                        int64_t sam, int64_t sak, const void *B, int64_t sbn, int64_t sbk,
                        const float *bias, float *C, int64_t ldc) {
    if (M <= 0 || N <= 0) return;
    dim3 grid(gdiv(N, 64), gdiv(M, 64));
    if (b_bf16) {
        const uint16_t *Bw = (const uint16_t *)B;
        if (epi == EPI_NONE)
            hipLaunchKernelGGL((k_gemm<float, uint16_t, EPI_NONE>), grid, dim3(256), 0, s, M, N, K, A,
                               sam, sak, Bw, sbn, sbk, bias, C, ldc);
        else if (epi == EPI_BIAS)
            hipLaunchKernelGGL((k_gemm<float, uint16_t, EPI_BIAS>), grid, dim3(256), 0, s, M, N, K, A,
                               sam, sak, Bw, sbn, sbk, bias, C, ldc);
        else
            hipLaunchKernelGGL((k_gemm<float, uint16_t, EPI_BIAS_TANH>), grid, dim3(256), 0, s, M, N,
                               K, A, sam, sak, Bw, sbn, sbk, bias, C, ldc);
    } else {
        hipLaunchKernelGGL((k_gemm<float, float, EPI_NONE>), grid, dim3(256), 0, s, M, N, K, A, sam,
                           sak, (const float *)B, sbn, sbk, bias, C, ldc);
    }
    WPCD_HIP(hipGetLastError());
}

// Glorot-uniform weights, zero biases; counter-based generator (splitmix64).
void mlp_init(Mlp &m, hipStream_t s, int nin, int nh, int nout, uint64_t seed) {
    m.nin = nin;
    m.nh = nh;
    m.nout = nout;
    std::vector<float> w(m.n_params(), 0.f);
    uint64_t st = seed;
    auto next = [&]() {
        st += 0x9E3779B97F4A7C15ull;
        uint64_t z = st;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    };
    for (int l = 0; l < 4; ++l) {
        const double a = std::sqrt(6.0 / (m.din(l) + m.dout(l)));
        float *W = w.data() + m.w_off(l);
        for (int64_t k = 0; k < (int64_t)m.dout(l) * m.din(l); ++k)
            W[k] = (float)((2.0 * next() - 1.0) * a);
    }
    mlp_set_weights(m, s, w.data());
}

void mlp_set_weights(Mlp &m, hipStream_t s, const float *w) {
    const int64_t np = m.n_params();
    m.w32.reserve(np);
    m.w16.reserve(np);
    m.am.reserve(np);
    m.av.reserve(np);
    m.grad.reserve(np);
    WPCD_HIP(hipMemcpyAsync(m.w32.ptr, w, np * sizeof(float), hipMemcpyHostToDevice, s));
    WPCD_HIP(hipMemsetAsync(m.am.ptr, 0, np * sizeof(float), s));
    WPCD_HIP(hipMemsetAsync(m.av.ptr, 0, np * sizeof(float), s));
    hipLaunchKernelGGL(k_to_bf16, dim3(gdiv(np, 256)), dim3(256), 0, s, m.w32.ptr, m.w16.ptr, np);
    WPCD_HIP(hipGetLastError());
    m.step = 0;
    m.ready = true;
}

// Activation buffer: input [B][nin], then the outputs of the four layers.
static float *act_ptr(Mlp &m, int B, int layer) {
    int64_t o = 0;
    for (int l = 0; l < layer; ++l) o += (int64_t)B * (l == 0 ? m.nin : m.nh);
    return m.act.ptr + o;
}

float *mlp_forward(Mlp &m, hipStream_t s, Timer &t, const float *X, int B) {
    WPCD_REQUIRE(m.ready, WPCD_E_STATE, "network has no weights");
    m.act.reserve((size_t)B * ((int64_t)m.nin + 3 * m.nh + m.nout));
    m.dact.reserve((size_t)B * (3 * m.nh + m.nout));
    m.rowloss.reserve(B);
    WPCD_HIP(hipMemcpyAsync(act_ptr(m, B, 0), X, (size_t)B * m.nin * sizeof(float),
                            hipMemcpyDeviceToDevice, s));
    TimedLaunch tl(t, s, "mlp_forward", WPCD_TIME_SOLVE);
    for (int l = 0; l < 4; ++l) {
        const int64_t wo = m.w_off(l);
        const float *bias = m.w32.ptr + wo + (int64_t)m.dout(l) * m.din(l);
        // Z[b][o] = sum_i H[b][i] W[o][i] + bias[o]
        gemm_launch(s, l < 3 ? EPI_BIAS_TANH : EPI_BIAS, true, B, m.dout(l), m.din(l),
                    act_ptr(m, B, l), m.din(l), 1, m.w16.ptr + wo, m.din(l), 1, bias,
                    act_ptr(m, B, l + 1), m.dout(l));
    }
    return act_ptr(m, B, 4);
}

double mlp_loss_grad(Mlp &m, hipStream_t s, Timer &t, const float *X, const float *T, int B,
                     bool want_loss) {
    const float *Y = mlp_forward(m, s, t, X, B);
    TimedLaunch tl(t, s, "mlp_backward", WPCD_TIME_SOLVE);
    float *dZ = m.dact.ptr + (int64_t)B * 3 * m.nh;   // [B][nout]
    hipLaunchKernelGGL(k_mse, dim3(gdiv(B, 256)), dim3(256), 0, s, Y, T, B, m.nout, dZ,
                       m.rowloss.ptr);
    WPCD_HIP(hipGetLastError());
    for (int l = 3; l >= 0; --l) {
        const int din = m.din(l), dout = m.dout(l);
        const float *H = act_ptr(m, B, l);
        float *gW = m.grad.ptr + m.w_off(l);
        float *gb = gW + (int64_t)dout * din;
        // dW[o][i] = sum_b dZ[b][o] H[b][i]
        gemm_launch(s, EPI_NONE, false, dout, din, B, dZ, 1, dout, H, 1, din, nullptr, gW, din);
        hipLaunchKernelGGL(k_colsum, dim3(gdiv(dout, 256)), dim3(256), 0, s, dZ, B, dout, gb);
        WPCD_HIP(hipGetLastError());
        if (l > 0) {
            float *dH = m.dact.ptr + (int64_t)B * (l - 1) * m.nh;   // [B][nh]
            // dH[b][i] = sum_o dZ[b][o] W[o][i], then times tanh' = 1 - H^2
            gemm_launch(s, EPI_NONE, true, B, din, dout, dZ, dout, 1, m.w16.ptr + m.w_off(l), 1,
                        din, nullptr, dH, din);
            hipLaunchKernelGGL(k_tanh_bwd, dim3(gdiv((int64_t)B * din, 256)), dim3(256), 0, s, H,
                               dH, (int64_t)B * din);
            WPCD_HIP(hipGetLastError());
            dZ = dH;
        }
    }
    if (!want_loss) return 0.0;
    std::vector<float> rl(B);
    WPCD_HIP(hipMemcpyAsync(rl.data(), m.rowloss.ptr, B * sizeof(float), hipMemcpyDeviceToHost, s));
    WPCD_HIP(hipStreamSynchronize(s));
    double loss = 0.0;
    for (float x : rl) loss += x;
    return loss / B;
}

void mlp_gather(hipStream_t s, const float *src, int ncol, const int32_t *idx, int n, float *dst) {
    hipLaunchKernelGGL(k_gather_rows, dim3(gdiv((int64_t)n * ncol, 256)), dim3(256), 0, s, src, ncol,
                       idx, n, dst);
    WPCD_HIP(hipGetLastError());
}

void mlp_adam_step(Mlp &m, hipStream_t s, Timer &t, float lr) {
    const int64_t np = m.n_params();
    m.step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)m.step), c2 = 1.f - std::pow(b2, (float)m.step);
    TimedLaunch tl(t, s, "mlp_adam", WPCD_TIME_SOLVE);
    hipLaunchKernelGGL(k_adam, dim3(gdiv(np, 256)), dim3(256), 0, s, m.w32.ptr, m.grad.ptr, m.am.ptr,
                       m.av.ptr, m.w16.ptr, np, lr, b1, b2, c1, c2, 1e-8f);
    WPCD_HIP(hipGetLastError());
}

}  // namespace wpcd
