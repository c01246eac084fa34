// Learned Sinkhorn warm start: per-column features of X = G / eps, a
// 4 -> 128 -> 128 -> 1 ReLU network (float32) mapping them to the column
// potential g_j / eps, and its training kernels (forward, backward, Adam).
//
// Features of column j (computed over rows i of X): mean, max, standard
// deviation, log-mean-exp (LSE_i x_ij - log n), each centred by its mean
// over j (potentials are defined up to a constant shift between f and g).
// Parameters are packed as W1[128][4], b1[128], W2[128][128], b2[128],
// W3[128], b3 (17281 floats).
#include <cmath>

#include "common.h"

namespace goat {
namespace {

constexpr int H = 128, NF = 4, SB = 64;   // hidden width, features, samples per block
constexpr int OFF_W1 = 0, OFF_B1 = 512, OFF_W2 = 640, OFF_B2 = 640 + H * H, OFF_W3 = OFF_B2 + H,
              OFF_B3 = OFF_W3 + H, NPARAM = OFF_B3 + 1;
constexpr int kFeatWG = 256;              // row strips of the feature sweep

__device__ inline float wsum(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
__device__ inline double wsum_d(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// ------------------------------------------------------------------ features

struct FeatArgs {
    const float* G;
    int ldg, n, np, rpw, W;
    const float* eps;
    float* part;        // 4 planes [W][np]: mean, M2, max, sum exp(x - max)
    float* F;           // [n][4]
};

// Strip partials per column: Welford mean/M2 and an online max-shifted sum
// of exponentials over the strip's rows.
template <int T, int C>
__global__ __launch_bounds__(T) void feat_strip_kernel(FeatArgs a) {
    const int tid = threadIdx.x, w = blockIdx.x;
    const int r0 = w * a.rpw, r1 = min(a.n, r0 + a.rpw);
    const float inv_eps = 1.0f / *a.eps;
    float mean[C][4], m2[C][4], mx[C][4], ls[C][4];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            mean[c][e] = 0.0f; m2[c][e] = 0.0f; mx[c][e] = -INFINITY; ls[c][e] = 0.0f;
        }
    for (int i = r0; i < r1; ++i) {
        const float invc = 1.0f / (float)(i - r0 + 1);
        const float4* row = reinterpret_cast<const float4*>(a.G + (size_t)i * a.ldg);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j4 = tid + T * c;
            if (4 * j4 >= a.n) continue;
            const float4 g4 = row[j4];
            const float gv[4] = {g4.x, g4.y, g4.z, g4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float x = gv[e] * inv_eps;
                const float d = x - mean[c][e];
                mean[c][e] += d * invc;
                m2[c][e] += d * (x - mean[c][e]);
                const float mnew = fmaxf(mx[c][e], x);
                ls[c][e] = ls[c][e] * expf(mx[c][e] - mnew) + expf(x - mnew);
                mx[c][e] = mnew;
            }
        }
    }
    const size_t plane = (size_t)a.W * a.np;
    float* base = a.part + (size_t)w * a.np;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j4 = tid + T * c;
        if (4 * j4 >= a.np) continue;
        reinterpret_cast<float4*>(base)[j4] = make_float4(mean[c][0], mean[c][1], mean[c][2], mean[c][3]);
        reinterpret_cast<float4*>(base + plane)[j4] = make_float4(m2[c][0], m2[c][1], m2[c][2], m2[c][3]);
        reinterpret_cast<float4*>(base + 2 * plane)[j4] = make_float4(mx[c][0], mx[c][1], mx[c][2], mx[c][3]);
        reinterpret_cast<float4*>(base + 3 * plane)[j4] = make_float4(ls[c][0], ls[c][1], ls[c][2], ls[c][3]);
    }
}

// One thread per column: strips combined in order (Chan's update for the
// mean and M2; the max first, then the rescaled sum of exponentials).
__global__ __launch_bounds__(256) void feat_merge_kernel(FeatArgs a) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    const size_t plane = (size_t)a.W * a.np;
    float cnt = 0.0f, mean = 0.0f, m2 = 0.0f, mx = -INFINITY;
    for (int w = 0; w < a.W; ++w) {
        const int r0 = w * a.rpw, r1 = min(a.n, r0 + a.rpw);
        const float nb = (float)(r1 - r0);
        if (nb <= 0.0f) continue;
        const float mb = a.part[(size_t)w * a.np + j], m2b = a.part[plane + (size_t)w * a.np + j];
        const float tot = cnt + nb;
        const float d = mb - mean;
        mean += d * (nb / tot);
        m2 += m2b + d * d * (cnt * nb / tot);
        cnt = tot;
        mx = fmaxf(mx, a.part[2 * plane + (size_t)w * a.np + j]);
    }
    float s = 0.0f;
    for (int w = 0; w < a.W; ++w) {
        const int r0 = w * a.rpw, r1 = min(a.n, r0 + a.rpw);
        if (r1 <= r0) continue;
        s += a.part[3 * plane + (size_t)w * a.np + j] * expf(a.part[2 * plane + (size_t)w * a.np + j] - mx);
    }
    float* f = a.F + (size_t)j * NF;
    f[0] = mean;
    f[1] = mx;
    f[2] = sqrtf(fmaxf(m2 / cnt, 0.0f));
    f[3] = mx + logf(s) - logf((float)a.n);
}

// Subtracts the mean over columns of each feature (float64 sums, fixed order).
__global__ __launch_bounds__(256) void feat_centre_kernel(int n, float* F) {
    __shared__ double sh[4][4];
    double s[NF] = {0.0, 0.0, 0.0, 0.0};
    for (int j = threadIdx.x; j < n; j += 256)
#pragma unroll
        for (int k = 0; k < NF; ++k) s[k] += F[(size_t)j * NF + k];
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        const double t = wsum_d(s[k]);
        if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = t;
    }
    __syncthreads();
    float mu[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) mu[k] = (float)(((sh[k][0] + sh[k][1]) + (sh[k][2] + sh[k][3])) / n);
    for (int j = threadIdx.x; j < n; j += 256)
#pragma unroll
        for (int k = 0; k < NF; ++k) F[(size_t)j * NF + k] -= mu[k];
}

// ------------------------------------------------------------------ network

// Layer 1 for SB samples into LDS: z1[s][k] (pre-activation). Thread k = hidden unit.
__device__ inline void layer1(const float* Fs, const float* p, float (*z1)[H + 1]) {
    const int k = threadIdx.x;
    const float w0 = p[OFF_W1 + k * NF + 0], w1 = p[OFF_W1 + k * NF + 1];
    const float w2 = p[OFF_W1 + k * NF + 2], w3 = p[OFF_W1 + k * NF + 3], b = p[OFF_B1 + k];
    for (int s = 0; s < SB; ++s) {
        const float* f = Fs + s * NF;
        z1[s][k] = fmaf(w3, f[3], fmaf(w2, f[2], fmaf(w1, f[1], fmaf(w0, f[0], b))));
    }
}

// Layer 2 pre-activation of unit t for every sample, from relu(z1) in LDS.
__device__ inline void layer2(const float* p, const float (*z1)[H + 1], float (&z2)[SB]) {
    const int t = threadIdx.x;
    const float b = p[OFF_B2 + t];
#pragma unroll
    for (int s = 0; s < SB; ++s) z2[s] = b;
    const float* w = p + OFF_W2 + (size_t)t * H;
    for (int k = 0; k < H; ++k) {
        const float wk = w[k];
#pragma unroll
        for (int s = 0; s < SB; ++s) z2[s] = fmaf(wk, fmaxf(z1[s][k], 0.0f), z2[s]);
    }
}

// Output y[s] = W3 . relu(z2[s]) + b3, reduced over the H units (2 waves).
__device__ inline void layer3(const float* p, const float (&z2)[SB], float* ys, float (*red)[SB]) {
    const int t = threadIdx.x;
    const float w3 = p[OFF_W3 + t];
#pragma unroll
    for (int s = 0; s < SB; ++s) {
        const float v = wsum(w3 * fmaxf(z2[s], 0.0f));
        if ((t & 63) == 0) red[t >> 6][s] = v;
    }
    __syncthreads();
    if (t < SB) ys[t] = (red[0][t] + red[1][t]) + p[OFF_B3];
    __syncthreads();
}

__device__ inline void load_features(int N, const float* F, int s0, float* Fs) {
    for (int q = threadIdx.x; q < SB * NF; q += H) {
        const int s = s0 + q / NF;
        Fs[q] = s < N ? F[(size_t)s0 * NF + q] : 0.0f;
    }
    __syncthreads();
}

__global__ __launch_bounds__(H) void mlp_forward_kernel(int N, const float* F, const float* p, float* y) {
    __shared__ float Fs[SB * NF];
    __shared__ float z1[SB][H + 1];
    __shared__ float red[2][SB];
    __shared__ float ys[SB];
    const int s0 = blockIdx.x * SB;
    load_features(N, F, s0, Fs);
    layer1(Fs, p, z1);
    __syncthreads();
    float z2[SB];
    layer2(p, z1, z2);
    layer3(p, z2, ys, red);
    if (threadIdx.x < SB && s0 + threadIdx.x < N) y[s0 + threadIdx.x] = ys[threadIdx.x];
}

// Gradients of L = (1/N) sum_s (y_s - t_s)^2 for one block of SB samples,
// written as one partial per block (the reduction kernel sums them in order).
__global__ __launch_bounds__(H) void mlp_backward_kernel(int N, const float* F, const float* tgt,
                                                         const float* p, float* partial, float* loss_part) {
    __shared__ float Fs[SB * NF];
    __shared__ float z1[SB][H + 1];
    __shared__ float dz2s[SB][H + 1];
    __shared__ float red[2][SB];
    __shared__ float ys[SB];
    __shared__ float dy[SB];
    const int t = threadIdx.x;
    const int s0 = blockIdx.x * SB;
    load_features(N, F, s0, Fs);
    layer1(Fs, p, z1);
    __syncthreads();
    float z2[SB];
    layer2(p, z1, z2);
    layer3(p, z2, ys, red);
    if (t < SB) {
        const bool ok = s0 + t < N;
        const float r = ok ? ys[t] - tgt[s0 + t] : 0.0f;
        dy[t] = ok ? (2.0f / (float)N) * r : 0.0f;
        red[0][t] = r * r;
    }
    __syncthreads();
    float* g = partial + (size_t)blockIdx.x * NPARAM;
    if (t == 0) {
        float l = 0.0f, gb3 = 0.0f;
        for (int s = 0; s < SB; ++s) { l += red[0][s]; gb3 += dy[s]; }
        loss_part[blockIdx.x] = l;
        g[OFF_B3] = gb3;
    }
    // layer 3 and layer 2 (unit t)
    const float w3 = p[OFF_W3 + t];
    float gw3 = 0.0f, gb2 = 0.0f;
#pragma unroll
    for (int s = 0; s < SB; ++s) {
        const float a2 = fmaxf(z2[s], 0.0f);
        gw3 = fmaf(dy[s], a2, gw3);
        const float d = z2[s] > 0.0f ? dy[s] * w3 : 0.0f;
        dz2s[s][t] = d;
        gb2 += d;
    }
    g[OFF_W3 + t] = gw3;
    g[OFF_B2 + t] = gb2;
    __syncthreads();
    // dW2[t][k] = sum_s dz2[s][t] relu(z1[s][k])
    for (int k = 0; k < H; ++k) {
        float acc = 0.0f;
#pragma unroll 8
        for (int s = 0; s < SB; ++s) acc = fmaf(dz2s[s][t], fmaxf(z1[s][k], 0.0f), acc);
        g[OFF_W2 + (size_t)t * H + k] = acc;
    }
    // layer 1, unit k = t: dz1[s][k] = (sum_o dz2[s][o] W2[o][k]) [z1 > 0]
    const int k = t;
    float dz1[SB];
#pragma unroll
    for (int s = 0; s < SB; ++s) dz1[s] = 0.0f;
    for (int o = 0; o < H; ++o) {
        const float w = p[OFF_W2 + (size_t)o * H + k];
#pragma unroll
        for (int s = 0; s < SB; ++s) dz1[s] = fmaf(dz2s[s][o], w, dz1[s]);
    }
    float gw1[NF] = {0.0f, 0.0f, 0.0f, 0.0f}, gb1 = 0.0f;
#pragma unroll
    for (int s = 0; s < SB; ++s) {
        const float d = z1[s][k] > 0.0f ? dz1[s] : 0.0f;
        gb1 += d;
#pragma unroll
        for (int f = 0; f < NF; ++f) gw1[f] = fmaf(d, Fs[s * NF + f], gw1[f]);
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) g[OFF_W1 + k * NF + f] = gw1[f];
    g[OFF_B1 + k] = gb1;
}

__global__ __launch_bounds__(256) void mlp_grad_reduce_kernel(int nblk, const float* partial, const float* loss_part,
                                                              int N, float* grad, float* loss) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < NPARAM) {
        float s = 0.0f;
        for (int b = 0; b < nblk; ++b) s += partial[(size_t)b * NPARAM + q];
        grad[q] = s;
    }
    if (q == 0 && loss) {
        float l = 0.0f;
        for (int b = 0; b < nblk; ++b) l += loss_part[b];
        *loss = l / (float)N;
    }
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(const float* grad, float* p, float* m, float* v,
                                                       float lr, float bc1, float bc2) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= NPARAM) return;
    const float g = grad[q];
    const float mq = 0.9f * m[q] + 0.1f * g;
    const float vq = 0.999f * v[q] + 0.001f * g * g;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / bc1) / (sqrtf(vq / bc2) + 1e-8f);
}

// Column potentials from the network's prediction pred_j ~ g_j / eps:
// v_j = pred_j log2(e) split into grid part and remainder; a non-finite
// prediction leaves that column cold (v_j = 0).
__global__ __launch_bounds__(256) void warm_seed_kernel(int n, const float* pred, const SkCtrl* ctrl,
                                                        float* vg, float* vs) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n || ctrl->done) return;
    const float x = pred[j];
    float r = isfinite(x) ? x * 1.4426950408889634f : 0.0f;
    const float h = ctrl->h;
    const float g = rintf(r / h) * h;
    vg[j] = g;
    vs[j] = r - g;
}

int feat_geometry(int n, int& T, int& C, int& W, int& rpw) {
    const int n4 = (n + 3) / 4;
    T = n < 4096 ? 256 : 512;
    C = (n4 + T - 1) / T;
    const int cs[] = {1, 2, 3, 4, 5, 6, 8, 10};
    int c2 = 0;
    for (int c : cs)
        if (c >= C) { c2 = c; break; }
    if (!c2) return GOAT_ENOTSUP;
    C = c2;
    W = n < kFeatWG ? n : kFeatWG;
    rpw = (n + W - 1) / W;
    W = (n + rpw - 1) / rpw;
    return GOAT_OK;
}

template <int T>
void launch_feat_T(int C, int W, const FeatArgs& a, hipStream_t s) {
    switch (C) {
#define GOAT_F_C(CC) case CC: hipLaunchKernelGGL((feat_strip_kernel<T, CC>), dim3(W), dim3(T), 0, s, a); break;
        GOAT_F_C(1) GOAT_F_C(2) GOAT_F_C(3) GOAT_F_C(4) GOAT_F_C(5) GOAT_F_C(6) GOAT_F_C(8) GOAT_F_C(10)
#undef GOAT_F_C
        default: break;
    }
}

}  // namespace

int mlp_param_count() { return NPARAM; }

size_t mlp_part_bytes(int N) { return (size_t)((N + SB - 1) / SB) * (NPARAM + 1) * 4 + 256; }

int mlp_features(int n, int np, const float* G, int ldg, const float* eps_dev, float* part, float* F,
                 hipStream_t s) {
    int T, C, W, rpw;
    if (feat_geometry(n, T, C, W, rpw)) {
        set_error("goat_mlp_features: n above 20480 is not supported");
        return GOAT_ENOTSUP;
    }
    FeatArgs a{G, ldg, n, np, rpw, W, eps_dev, part, F};
    if (T == 256) launch_feat_T<256>(C, W, a, s);
    else launch_feat_T<512>(C, W, a, s);
    hipLaunchKernelGGL(feat_merge_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(feat_centre_kernel, dim3(1), dim3(256), 0, s, n, F);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int mlp_forward(int N, const float* F, const float* p, float* y, hipStream_t s) {
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((N + SB - 1) / SB), dim3(H), 0, s, N, F, p, y);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int mlp_backward(int N, const float* F, const float* t, const float* p, float* grad, float* loss, void* part,
                 hipStream_t s) {
    const int nblk = (N + SB - 1) / SB;
    float* partial = static_cast<float*>(part);
    float* loss_part = partial + (size_t)nblk * NPARAM;
    hipLaunchKernelGGL(mlp_backward_kernel, dim3(nblk), dim3(H), 0, s, N, F, t, p, partial, loss_part);
    hipLaunchKernelGGL(mlp_grad_reduce_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s, nblk,
                       (const float*)partial, (const float*)loss_part, N, grad, loss);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int mlp_adam(const float* grad, float* p, float* m, float* v, int step, float lr, hipStream_t s) {
    const float bc1 = 1.0f - powf(0.9f, (float)step), bc2 = 1.0f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s, grad, p, m, v, lr, bc1, bc2);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int warm_seed(int n, const float* pred, const SkCtrl* ctrl, float* vg, float* vs, hipStream_t s) {
    hipLaunchKernelGGL(warm_seed_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, pred, ctrl, vg, vs);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

}  // namespace goat
