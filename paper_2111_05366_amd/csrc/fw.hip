// Frank-Wolfe bookkeeping kernels: max|G| for eps, the float64 traces and
// exact step of the line search (Alg. 3 step 3), the update
// P <- P + t (Q - P) with grad f updated by linearity, initial fills and
// the permutation score. Every float64 reduction is two-level with a fixed
// summation order, so results are bitwise reproducible.
#include "common.h"

namespace goat {
namespace {

constexpr int RT = 256;   // threads per reduction block

__device__ inline double wsum_d(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
__device__ inline float wmax_f(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
    return x;
}

// Sum of x over the block in a fixed order (wave shuffles, then waves 0..3).
__device__ inline double block_sum_d(double x, double* sh) {
    x = wsum_d(x);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}
__device__ inline float block_max_f(float x, float* sh) {
    x = wmax_f(x);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    return fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
}

int nblocks_rows(int n) { return n < kRedWG ? n : kRedWG; }

// ------------------------------------------------------------------ absmax

__global__ __launch_bounds__(RT) void absmax_partial_kernel(int n, const float* __restrict__ G, int ldg,
                                                            float* partial) {
    __shared__ float sh[4];
    float m = 0.0f;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const float* row = G + (size_t)i * ldg;
        for (int j = threadIdx.x; j < n; j += RT) m = fmaxf(m, fabsf(row[j]));
    }
    m = block_max_f(m, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ __launch_bounds__(RT) void max_final_kernel(int nb, const float* partial, float* out,
                                                       const double* ls8) {
    if (ls8 && ls8[5] == 0.0) return;   // no update happened: keep the old value
    __shared__ float sh[4];
    float m = 0.0f;
    for (int b = threadIdx.x; b < nb; b += RT) m = fmaxf(m, partial[b]);
    m = block_max_f(m, sh);
    if (threadIdx.x == 0) *out = m;
}

// ------------------------------------------------------------------ traces

// Partial traces per block: <P,GP>, <Q,GQ>, <Q,GP>, ||Q-P||^2 and, with a
// linear term C (seeded problems), <P,C> and <Q,C>.
__global__ __launch_bounds__(RT) void traces_partial_kernel(int n, const float* __restrict__ P,
                                                            const float* __restrict__ Q,
                                                            const float* __restrict__ GP,
                                                            const float* __restrict__ GQ,
                                                            const float* __restrict__ C, int ld,
                                                            double* partial) {
    __shared__ double sh[4];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0, s5 = 0.0;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const size_t o = (size_t)i * ld;
        for (int j = threadIdx.x; j < n; j += RT) {
            const double p = P[o + j], q = Q[o + j], gp = GP[o + j], gq = GQ[o + j];
            s0 += p * gp;
            s1 += q * gq;
            s2 += q * gp;
            const double d = q - p;
            s3 += d * d;
            if (C) {
                const double c = C[o + j];
                s4 += p * c;
                s5 += q * c;
            }
        }
    }
    s0 = block_sum_d(s0, sh);
    s1 = block_sum_d(s1, sh);
    s2 = block_sum_d(s2, sh);
    s3 = block_sum_d(s3, sh);
    s4 = block_sum_d(s4, sh);
    s5 = block_sum_d(s5, sh);
    if (threadIdx.x == 0) {
        double* o = partial + kTraceSlots * (size_t)blockIdx.x;
        o[0] = s0; o[1] = s1; o[2] = s2; o[3] = s3; o[4] = s4; o[5] = s5;
    }
}

// Exact step: with fP = <P,GP>/2, fQ = <Q,GQ>/2, c = <Q,GP>,
// f(P + t(Q-P)) = fP + b t + a t^2, a = fP + fQ - c, b = c - 2 fP.
// With a linear term C (f(X) = <C,X> + q(X), q quadratic) the curvature
// gains <Q - P, C>/2, and f(P) = fP + <P,C>/2, f(Q) = fQ + <Q,C>/2 are
// reported.
__global__ __launch_bounds__(RT) void linesearch_final_kernel(int nb, const double* partial, double* out8) {
    __shared__ double sh[4];
    double s[kTraceSlots];
    for (int k = 0; k < kTraceSlots; ++k) {
        double x = 0.0;
        for (int b = threadIdx.x; b < nb; b += RT) x += partial[kTraceSlots * (size_t)b + k];
        s[k] = block_sum_d(x, sh);
    }
    if (threadIdx.x == 0) {
        const double fP = 0.5 * s[0], fQ = 0.5 * s[1], c = s[2];
        const double a = fP + fQ - c + 0.5 * (s[5] - s[4]), b = c - 2.0 * fP;
        double t;
        if (a < 0.0) {
            t = -b / (2.0 * a);
            t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        } else {
            t = (a + b > 0.0) ? 1.0 : 0.0;
        }
        out8[0] = fP + 0.5 * s[4]; out8[1] = fQ + 0.5 * s[5]; out8[2] = c; out8[3] = a;
        out8[4] = b;  out8[5] = t;  out8[6] = s[3]; out8[7] = 0.0;
    }
}

// ------------------------------------------------------------------ update

__global__ __launch_bounds__(RT) void fw_update_kernel(int n, float* __restrict__ P, const float* __restrict__ Q,
                                                       float* __restrict__ GP, const float* __restrict__ GQ,
                                                       int ld, const double* ls8, float* partial) {
    const double td = ls8[5];
    if (td == 0.0) return;
    const float t = (float)td;
    __shared__ float sh[4];
    float m = 0.0f;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const size_t o = (size_t)i * ld;
        for (int j = threadIdx.x; j < n; j += RT) {
            const float p = P[o + j], q = Q[o + j];
            P[o + j] = fmaf(t, q - p, p);
            const float gp = GP[o + j], gq = GQ[o + j];
            const float g = fmaf(t, gq - gp, gp);
            GP[o + j] = g;
            m = fmaxf(m, fabsf(g));
        }
    }
    m = block_max_f(m, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

// ------------------------------------------------------------------ fills

__global__ __launch_bounds__(RT) void fill_bary_kernel(int n, int np, float* P) {
    const float v = 1.0f / (float)n;
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < np; j += RT) P[(size_t)i * np + j] = (i < n && j < n) ? v : 0.0f;
}

__global__ __launch_bounds__(RT) void copy_pad_kernel(int n, const float* src, int lds, float* dst, int ldd,
                                                      int np) {
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < np; j += RT)
        dst[(size_t)i * ldd + j] = (i < n && j < n) ? src[(size_t)i * lds + j] : 0.0f;
}

__global__ __launch_bounds__(RT) void split_kernel(int n, int np, const float* src, int lds, uint16_t* hi,
                                                   uint16_t* lo) {
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < np; j += RT) {
        const float x = (i < n && j < n) ? src[(size_t)i * lds + j] : 0.0f;
        const uint16_t h = f32_to_bf16_rne(x);
        hi[(size_t)i * np + j] = h;
        lo[(size_t)i * np + j] = f32_to_bf16_rne(x - bf16_to_f32(h));
    }
}

// ------------------------------------------------------------------ score

__global__ __launch_bounds__(RT) void score_partial_kernel(int n, const float* __restrict__ A,
                                                           const float* __restrict__ B, int ld,
                                                           const int32_t* __restrict__ perm, double* partial) {
    __shared__ double sh[4];
    double s = 0.0;
    // indices are clamped so that an invalid permutation cannot read out of bounds
    auto pidx = [n, perm](int k) { const int p = perm[k]; return p < 0 ? 0 : (p >= n ? n - 1 : p); };
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const float* brow = B + (size_t)pidx(i) * ld;
        const float* arow = A + (size_t)i * ld;
        for (int j = threadIdx.x; j < n; j += RT) s += (double)arow[j] * (double)brow[pidx(j)];
    }
    s = block_sum_d(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(RT) void sum_final_kernel(int nb, const double* partial, double* out) {
    __shared__ double sh[4];
    double x = 0.0;
    for (int b = threadIdx.x; b < nb; b += RT) x += partial[b];
    x = block_sum_d(x, sh);
    if (threadIdx.x == 0) *out = x;
}

// Seeded problems: Y[i][j] = X'[o[i]][o[j]] with X' = X (naive) or 2X - 1
// (adopted); rows and columns with o < 0 (dummy vertices) are zero.
__global__ __launch_bounds__(RT) void arrange_kernel(int n, const float* __restrict__ X, int ldx,
                                                     const int* __restrict__ order, int adopted, float* Y,
                                                     int ldy) {
    const int i = blockIdx.x;
    const int oi = order[i];
    for (int j = threadIdx.x; j < n; j += RT) {
        const int oj = order[j];
        float v = 0.0f;
        if (oi >= 0 && oj >= 0) {
            v = X[(size_t)oi * ldx + oj];
            if (adopted) v = 2.0f * v - 1.0f;
        }
        Y[(size_t)i * ldy + j] = v;
    }
}

// dst (prows x pcols, ldd) = the rows x cols block of src (or its
// transpose), zero elsewhere.
__global__ __launch_bounds__(RT) void pack_rect_kernel(const float* __restrict__ src, int ld, int rows, int cols,
                                                       int transpose, float* dst, int ldd, int pcols) {
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < pcols; j += RT) {
        float v = 0.0f;
        if (i < rows && j < cols) v = transpose ? src[(size_t)j * ld + i] : src[(size_t)i * ld + j];
        dst[(size_t)i * ldd + j] = v;
    }
}

__global__ __launch_bounds__(RT) void add_mat_kernel(int n, float* G, const float* __restrict__ C, int ld) {
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < n; j += RT) G[(size_t)i * ld + j] += C[(size_t)i * ld + j];
}

}  // namespace

int launch_absmax(int n, const float* G, int ldg, float* partial, float* out, hipStream_t s) {
    const int nb = nblocks_rows(n);
    hipLaunchKernelGGL(absmax_partial_kernel, dim3(nb), dim3(RT), 0, s, n, G, ldg, partial);
    hipLaunchKernelGGL(max_final_kernel, dim3(1), dim3(RT), 0, s, nb, partial, out, (const double*)nullptr);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int launch_traces(int n, const float* P, const float* Q, const float* GP, const float* GQ, int ld,
                  double* red, double* out8, hipStream_t s, const float* C) {
    const int nb = nblocks_rows(n);
    hipLaunchKernelGGL(traces_partial_kernel, dim3(nb), dim3(RT), 0, s, n, P, Q, GP, GQ, C, ld, red);
    hipLaunchKernelGGL(linesearch_final_kernel, dim3(1), dim3(RT), 0, s, nb, (const double*)red, out8);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int launch_fw_update(int n, float* P, const float* Q, float* GP, const float* GQ, int ld, const double* ls8,
                     float* absmax_partial, float* absmax_out, hipStream_t s) {
    const int nb = nblocks_rows(n);
    hipLaunchKernelGGL(fw_update_kernel, dim3(nb), dim3(RT), 0, s, n, P, Q, GP, GQ, ld, ls8, absmax_partial);
    hipLaunchKernelGGL(max_final_kernel, dim3(1), dim3(RT), 0, s, nb, (const float*)absmax_partial,
                       absmax_out, ls8);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int launch_fill_barycenter(int n, int np, float* P, hipStream_t s) {
    hipLaunchKernelGGL(fill_bary_kernel, dim3(np), dim3(RT), 0, s, n, np, P);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int launch_copy_pad(int n, const float* src, int lds, float* dst, int ldd, int np, hipStream_t s) {
    hipLaunchKernelGGL(copy_pad_kernel, dim3(np), dim3(RT), 0, s, n, src, lds, dst, ldd, np);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int launch_split_bf16(int n, int np, const float* src, int lds, uint16_t* hi, uint16_t* lo, hipStream_t s) {
    hipLaunchKernelGGL(split_kernel, dim3(np), dim3(RT), 0, s, n, np, src, lds, hi, lo);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int launch_score(int n, const float* A, const float* B, int ld, const int32_t* perm, double* red,
                 double* out, hipStream_t s) {
    const int nb = nblocks_rows(n);
    hipLaunchKernelGGL(score_partial_kernel, dim3(nb), dim3(RT), 0, s, n, A, B, ld, perm, red);
    hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(RT), 0, s, nb, (const double*)red, out);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

}  // namespace goat

namespace goat {

namespace {

// Sets *flag when any of the n x n entries (leading dimension ld) is NaN or
// infinite.
__global__ __launch_bounds__(RT) void check_finite_kernel(int n, const float* __restrict__ X, long ld,
                                                          int* flag) {
    bool bad = false;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const float* r = X + (long)i * ld;
        for (int j = threadIdx.x; j < n; j += RT) bad |= !isfinite(r[j]);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

}  // namespace

int launch_check_finite(int n, const float* X, int ld, int* flag, hipStream_t s) {
    if (n < 1) return GOAT_OK;
    hipLaunchKernelGGL(check_finite_kernel, dim3(n < kRedWG ? n : kRedWG), dim3(RT), 0, s, n, X, (long)ld, flag);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int launch_arrange(int n, const float* X, int ldx, const int* order_dev, int adopted, float* Y, int ldy,
                   hipStream_t s) {
    if (n < 1) return GOAT_OK;
    hipLaunchKernelGGL(arrange_kernel, dim3(n), dim3(RT), 0, s, n, X, ldx, order_dev, adopted, Y, ldy);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int launch_pack_rect(const float* src, int ld, int rows, int cols, int transpose, float* dst, int ldd, int prows,
                     int pcols, hipStream_t s) {
    if (prows < 1) return GOAT_OK;
    hipLaunchKernelGGL(pack_rect_kernel, dim3(prows), dim3(RT), 0, s, src, ld, rows, cols, transpose, dst, ldd,
                       pcols);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

// ln U into an np x np buffer (zero padding), and the scalar 1 at one_out:
// the Sinkhorn-Knopp scaling of U is the entropic plan of the cost ln U at
// eps = 1, Q = exp(ln U + f + g) = diag(e^f) U diag(e^g)
__global__ __launch_bounds__(RT) void log_pad_kernel(int n, const float* __restrict__ U, int ldu, float* dst,
                                                     int np, float* one_out) {
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < np; j += RT)
        dst[(size_t)i * np + j] = (i < n && j < n) ? logf(U[(size_t)i * ldu + j]) : 0.0f;
    if (i == 0 && threadIdx.x == 0) *one_out = 1.0f;
}

// P = (J + K) / 2 in place (K doubly stochastic, n x n, ld)
__global__ __launch_bounds__(RT) void half_bary_kernel(int n, float* P, int ld) {
    const float h = 0.5f / (float)n;
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < n; j += RT) P[(size_t)i * ld + j] = fmaf(0.5f, P[(size_t)i * ld + j], h);
}

int launch_log_pad(int n, const float* U, int ldu, float* dst, int np, float* one_out, hipStream_t s) {
    hipLaunchKernelGGL(log_pad_kernel, dim3(np), dim3(RT), 0, s, n, U, ldu, dst, np, one_out);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int launch_half_bary(int n, float* P, int ld, hipStream_t s) {
    hipLaunchKernelGGL(half_bary_kernel, dim3(n), dim3(RT), 0, s, n, P, ld);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int launch_add_mat(int n, float* G, const float* C, int ld, hipStream_t s) {
    if (n < 1) return GOAT_OK;
    hipLaunchKernelGGL(add_mat_kernel, dim3(n), dim3(RT), 0, s, n, G, C, ld);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

}  // namespace goat
