// mc_mlp.hip -- the learned initial weight: a 2-64-64-1 tanh network in fp32
// that maps (1/L, e = E/N) to the entropy per site f ~ ln g(E)/N.  Trained on
// converged weights of small lattices (ln g(E) = -ln w(E) + const, because a
// flat histogram means D(E) w(E) = const, Sec. 3.1 of the paper), it proposes
// ln w = -N f for a larger lattice, where the recursion then continues.
//
// Kernels: initialisation, forward, per-sample backward, weight gradients
// (one thread per parameter, fixed summation order: no atomics, so results
// are reproducible), loss, Adam, training targets from a weight, and the
// predicted weight of a lattice size.
#include <cmath>
#include <cstring>

#include "../../include/mc.h"
#include "mc_internal.h"
#include "mc_math.h"

namespace {

constexpr int H = 64;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + H * 2;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H;
constexpr int OFF_B3 = OFF_W3 + H;
constexpr int N_PARAMS = OFF_B3 + 1;
constexpr uint32_t kDomMlp = 3u;  // random-word domain of the initial parameters

// workspace layout (floats): act [n][2H] (h1 | h2), dact [n][2H] (dz1 | dz2),
// y [n], dy [n], scalars [4] (loss, weight sum)
size_t ws_floats(int n) { return (size_t)n * 4 * H + 2 * (size_t)n + 4; }

struct Ws {
    float *act, *dact, *y, *dy, *scal;
};

Ws carve(void *w, int n) {
    float *f = (float *)w;
    Ws s;
    s.act = f;
    s.dact = s.act + (size_t)n * 2 * H;
    s.y = s.dact + (size_t)n * 2 * H;
    s.dy = s.y + n;
    s.scal = s.dy + n;
    return s;
}

// Glorot-uniform weights from Philox words (domain 3), zero biases.
__global__ void k_mlp_init(float *p, uint32_t seed) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N_PARAMS) return;
    float scale = 0.f;
    if (k < OFF_B1) scale = sqrtf(6.f / (2 + H));
    else if (k >= OFF_W2 && k < OFF_B2) scale = sqrtf(6.f / (H + H));
    else if (k >= OFF_W3 && k < OFF_B3) scale = sqrtf(6.f / (H + 1));
    const uint4 r = mcgpu::philox10(make_uint4((uint32_t)k >> 2, 0u, 0u, kDomMlp), seed, 0u);
    const uint32_t u = mcgpu::word_of(r, (uint32_t)k & 3u);
    const float unit = (float)(u >> 8) * (1.0f / 16777216.0f);  // [0, 1)
    p[k] = scale * (2.f * unit - 1.f);
}

__device__ __forceinline__ void stage_params(const float *p, float *sp) {
    for (int k = threadIdx.x; k < N_PARAMS; k += blockDim.x) sp[k] = p[k];
    __syncthreads();
}

// Forward pass, one sample per thread; parameters staged in LDS (read as
// broadcasts).  Stores h1, h2 when act != nullptr.
__global__ __launch_bounds__(256) void k_mlp_forward(const float *p, const float *x, int n, float *y, float *act) {
    __shared__ float sp[N_PARAMS];
    stage_params(p, sp);
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float x0 = x[2 * s], x1 = x[2 * s + 1];
    float h1[H];
#pragma unroll
    for (int i = 0; i < H; ++i) h1[i] = tanhf(sp[OFF_B1 + i] + sp[OFF_W1 + 2 * i] * x0 + sp[OFF_W1 + 2 * i + 1] * x1);
    float o = sp[OFF_B3];
    for (int j = 0; j < H; ++j) {
        float z = sp[OFF_B2 + j];
#pragma unroll
        for (int i = 0; i < H; ++i) z += sp[OFF_W2 + H * j + i] * h1[i];
        const float h2 = tanhf(z);
        if (act) act[(size_t)s * 2 * H + H + j] = h2;
        o += sp[OFF_W3 + j] * h2;
    }
    if (act)
        for (int i = 0; i < H; ++i) act[(size_t)s * 2 * H + i] = h1[i];
    y[s] = o;
}

// Weighted mean squared error and the weight sum (one block, fixed order).
__global__ __launch_bounds__(256) void k_mlp_loss(const float *y, const float *t, const float *w, int n, float *scal) {
    __shared__ float s_l[256], s_w[256];
    float l = 0.f, ws = 0.f;
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        const float ww = w ? w[s] : 1.f;
        const float r = y[s] - t[s];
        l += ww * r * r;
        ws += ww;
    }
    s_l[threadIdx.x] = l;
    s_w[threadIdx.x] = ws;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            s_l[threadIdx.x] += s_l[threadIdx.x + off];
            s_w[threadIdx.x] += s_w[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        scal[0] = s_l[0] / s_w[0];
        scal[1] = s_w[0];
    }
}

// Per-sample backward: dy = 2 w (y - t) / sum w, dz2 = dy W3 (1 - h2^2),
// dz1 = (W2^T dz2) (1 - h1^2).
__global__ __launch_bounds__(256) void k_mlp_backward(const float *p, const float *t, const float *w, int n,
                                                      const float *scal, const float *y, const float *act,
                                                      float *dact, float *dy) {
    __shared__ float sp[N_PARAMS];
    stage_params(p, sp);
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float g = 2.f * (w ? w[s] : 1.f) * (y[s] - t[s]) / scal[1];
    dy[s] = g;
    const float *a = act + (size_t)s * 2 * H;
    float *d = dact + (size_t)s * 2 * H;
    float d2[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        const float h2 = a[H + j];
        d2[j] = g * sp[OFF_W3 + j] * (1.f - h2 * h2);
        d[H + j] = d2[j];
    }
    for (int i = 0; i < H; ++i) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < H; ++j) acc += d2[j] * sp[OFF_W2 + H * j + i];
        const float h1 = a[i];
        d[i] = acc * (1.f - h1 * h1);
    }
}

// Gradient of every parameter: one wave per parameter.  Lane l sums samples
// l, l + 64, l + 128, ... in order, then the wave adds its 64 partial sums in
// a fixed butterfly, so the result depends on n alone, not on the launch.
// The sample loops are over rows of the activations (2H floats each, held in
// L2 for the sample counts of a training set).
constexpr int kWgradWaves = 4;

__global__ __launch_bounds__(64 * kWgradWaves) void k_mlp_wgrad(const float *x, int n, const float *act,
                                                                const float *dact, const float *dy, float *grad) {
    const int k = blockIdx.x * kWgradWaves + (int)(threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    if (k >= N_PARAMS) return;  // the whole wave leaves together
    float acc = 0.f;
    if (k < OFF_B1) {  // W1[i][c]
        const int i = k >> 1, c = k & 1;
        for (int s = lane; s < n; s += 64) acc += dact[(size_t)s * 2 * H + i] * x[2 * s + c];
    } else if (k < OFF_W2) {  // b1[i]
        const int i = k - OFF_B1;
        for (int s = lane; s < n; s += 64) acc += dact[(size_t)s * 2 * H + i];
    } else if (k < OFF_B2) {  // W2[j][i]
        const int j = (k - OFF_W2) / H, i = (k - OFF_W2) % H;
        for (int s = lane; s < n; s += 64) acc += dact[(size_t)s * 2 * H + H + j] * act[(size_t)s * 2 * H + i];
    } else if (k < OFF_W3) {  // b2[j]
        const int j = k - OFF_B2;
        for (int s = lane; s < n; s += 64) acc += dact[(size_t)s * 2 * H + H + j];
    } else if (k < OFF_B3) {  // W3[j]
        const int j = k - OFF_W3;
        for (int s = lane; s < n; s += 64) acc += dy[s] * act[(size_t)s * 2 * H + H + j];
    } else {  // b3
        for (int s = lane; s < n; s += 64) acc += dy[s];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) grad[k] = acc;
}

// Adam (Kingma & Ba), bias-corrected.
__global__ void k_adam(float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N_PARAMS) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// Centre of bin b as energy per site: level m = b 2^s + (2^s - 1)/2, e = (4m - 2N)/N.
__device__ __forceinline__ double bin_energy(int b, int bin_shift, int N) {
    const double m = (double)(b << bin_shift) + 0.5 * (double)((1 << bin_shift) - 1);
    return (4.0 * m - 2.0 * (double)N) / (double)N;
}

// Inputs and targets of one converged weight: t_b = (-ln w_b + c)/N with c
// fixing sum_b G_b = 2^N, i.e. c = N ln 2 - logsumexp(-ln w).
__global__ __launch_bounds__(256) void k_mlp_targets(const double *lnW, int L, int bin_shift, float *x, float *t) {
    __shared__ double s_r[256];
    const int N = L * L, nb = (N >> bin_shift) + 1;
    double mx = -1e300;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) mx = fmax(mx, -lnW[b]);
    s_r[threadIdx.x] = mx;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s_r[threadIdx.x] = fmax(s_r[threadIdx.x], s_r[threadIdx.x + off]);
        __syncthreads();
    }
    const double m0 = s_r[0];
    __syncthreads();
    double sm = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) sm += exp(-lnW[b] - m0);
    s_r[threadIdx.x] = sm;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s_r[threadIdx.x] += s_r[threadIdx.x + off];
        __syncthreads();
    }
    const double c = (double)N * mcgpu::kLn2Head - (m0 + log(s_r[0]));
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        x[2 * b] = (float)(1.0 / (double)L);
        x[2 * b + 1] = (float)bin_energy(b, bin_shift, N);
        t[b] = (float)((-lnW[b] + c) / (double)N);
    }
}

// Proposed weight of a lattice size: ln w_b = -N f(1/L, e_b).
__global__ __launch_bounds__(256) void k_mlp_predict(const float *p, int L, int bin_shift, double *lnW) {
    __shared__ float sp[N_PARAMS];
    stage_params(p, sp);
    const int N = L * L, nb = (N >> bin_shift) + 1;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const float x0 = (float)(1.0 / (double)L), x1 = (float)bin_energy(b, bin_shift, N);
    float h1[H];
#pragma unroll
    for (int i = 0; i < H; ++i) h1[i] = tanhf(sp[OFF_B1 + i] + sp[OFF_W1 + 2 * i] * x0 + sp[OFF_W1 + 2 * i + 1] * x1);
    float o = sp[OFF_B3];
    for (int j = 0; j < H; ++j) {
        float z = sp[OFF_B2 + j];
#pragma unroll
        for (int i = 0; i < H; ++i) z += sp[OFF_W2 + H * j + i] * h1[i];
        o += sp[OFF_W3 + j] * tanhf(z);
    }
    lnW[b] = -(double)N * (double)o;
}

mc_status mlp_fail(mc_status st, const char *msg) {
    mcgpu::set_last_error(msg);
    return st;
}

#define MLP_HIP(call)                                                 \
    do {                                                              \
        hipError_t e_ = (call);                                       \
        if (e_ != hipSuccess) return mlp_fail(MC_EHIP, #call);        \
    } while (0)

int blocks(int n, int bs) { return (n + bs - 1) / bs; }

mc_status loss_grad(const float *p, const float *x, const float *t, const float *w, int n, float *grad, void *ws,
                    hipStream_t st) {
    Ws s = carve(ws, n);
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks(n, 256)), dim3(256), 0, st, p, x, n, s.y, s.act);
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, st, s.y, t, w, n, s.scal);
    hipLaunchKernelGGL(k_mlp_backward, dim3(blocks(n, 256)), dim3(256), 0, st, p, t, w, n, s.scal, s.y, s.act,
                       s.dact, s.dy);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(blocks(N_PARAMS, kWgradWaves)), dim3(64 * kWgradWaves), 0, st, x, n, s.act,
                       s.dact, s.dy, grad);
    MLP_HIP(hipGetLastError());
    return MC_OK;
}

}  // namespace

extern "C" {

int32_t mc_mlp_n_params(void) { return N_PARAMS; }

size_t mc_mlp_workspace_bytes(int32_t n) { return n < 1 ? 0 : ws_floats(n) * sizeof(float) + N_PARAMS * sizeof(float); }

mc_status mc_mlp_init(float *params_dev, uint32_t seed, void *stream) {
    if (!params_dev) return mlp_fail(MC_EINVAL, "null parameters");
    hipLaunchKernelGGL(k_mlp_init, dim3(blocks(N_PARAMS, 256)), dim3(256), 0, (hipStream_t)stream, params_dev, seed);
    MLP_HIP(hipGetLastError());
    return MC_OK;
}

mc_status mc_mlp_forward(const float *params_dev, const float *x_dev, int32_t n, float *y_dev, void *stream) {
    if (!params_dev || !x_dev || !y_dev || n < 1) return mlp_fail(MC_EINVAL, "bad forward arguments");
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks(n, 256)), dim3(256), 0, (hipStream_t)stream, params_dev, x_dev, n,
                       y_dev, nullptr);
    MLP_HIP(hipGetLastError());
    return MC_OK;
}

mc_status mc_mlp_loss_grad(const float *params_dev, const float *x_dev, const float *t_dev, const float *w_dev,
                           int32_t n, float *grad_dev, float *loss_dev, void *workspace_dev, void *stream) {
    if (!params_dev || !x_dev || !t_dev || !grad_dev || !workspace_dev || n < 1)
        return mlp_fail(MC_EINVAL, "bad loss_grad arguments");
    hipStream_t st = (hipStream_t)stream;
    mc_status r = loss_grad(params_dev, x_dev, t_dev, w_dev, n, grad_dev, workspace_dev, st);
    if (r != MC_OK) return r;
    if (loss_dev) MLP_HIP(hipMemcpyAsync(loss_dev, carve(workspace_dev, n).scal, sizeof(float), hipMemcpyDeviceToDevice, st));
    return MC_OK;
}

mc_status mc_mlp_train(float *params_dev, const float *x_dev, const float *t_dev, const float *w_dev, int32_t n,
                       int32_t steps, float lr, float *adam_dev, int32_t *step_io, float *loss_host,
                       void *workspace_dev, void *stream) {
    if (!params_dev || !x_dev || !t_dev || !adam_dev || !step_io || !workspace_dev || n < 1 || steps < 0 ||
        !(lr > 0.f))
        return mlp_fail(MC_EINVAL, "bad train arguments");
    hipStream_t st = (hipStream_t)stream;
    float *grad = (float *)workspace_dev + ws_floats(n);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int k = 0; k < steps; ++k) {
        mc_status r = loss_grad(params_dev, x_dev, t_dev, w_dev, n, grad, workspace_dev, st);
        if (r != MC_OK) return r;
        const int t = ++(*step_io);
        const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
        hipLaunchKernelGGL(k_adam, dim3(blocks(N_PARAMS, 256)), dim3(256), 0, st, params_dev, grad, adam_dev,
                           adam_dev + N_PARAMS, lr, b1, b2, eps, c1, c2);
        MLP_HIP(hipGetLastError());
    }
    if (loss_host) {
        MLP_HIP(hipMemcpyAsync(loss_host, carve(workspace_dev, n).scal, sizeof(float), hipMemcpyDeviceToHost, st));
        MLP_HIP(hipStreamSynchronize(st));
    }
    return MC_OK;
}

mc_status mc_mlp_targets(const double *lnW_dev, int32_t L, int32_t bin_shift, float *x_dev, float *t_dev,
                         void *stream) {
    if (!lnW_dev || !x_dev || !t_dev || L < 4 || L > 256 || (L & 1) || bin_shift < 0 || bin_shift > 1)
        return mlp_fail(MC_EINVAL, "bad targets arguments");
    hipLaunchKernelGGL(k_mlp_targets, dim3(1), dim3(256), 0, (hipStream_t)stream, lnW_dev, L, bin_shift, x_dev, t_dev);
    MLP_HIP(hipGetLastError());
    return MC_OK;
}

mc_status mc_mlp_predict_weights(const float *params_dev, int32_t L, int32_t bin_shift, double *lnW_dev,
                                 void *stream) {
    if (!params_dev || !lnW_dev || L < 4 || L > 256 || (L & 1) || bin_shift < 0 || bin_shift > 1)
        return mlp_fail(MC_EINVAL, "bad predict arguments");
    const int nb = ((L * L) >> bin_shift) + 1;
    hipLaunchKernelGGL(k_mlp_predict, dim3(blocks(nb, 256)), dim3(256), 0, (hipStream_t)stream, params_dev, L,
                       bin_shift, lnW_dev);
    MLP_HIP(hipGetLastError());
    return MC_OK;
}

}  // extern "C"
