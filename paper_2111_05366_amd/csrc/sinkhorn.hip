// Log-domain Sinkhorn-Knopp scaling for the LOT direction (Alg. 2, with the
// cost negated for the maximisation of Alg. 3 step 2).
//
// Units: potentials in base 2 scaled by 1/eps,
//     u_i = f_i * kappa,  v_j = g_j * kappa,  kappa = log2(e) / eps,
// so Q_ij = 2^(G_ij kappa + u_i + v_j).
//
// Compensated potentials. Each potential is a pair (grid part, remainder):
// the grid part is a multiple of h = 2^(e - 24), where 2^e bounds
// max|G kappa| + 64, and the remainder is small (|r| <= h/2). For an entry
// that matters (exponent near 0) the grid parts satisfy
// |v_grid + u_grid| < 2^e, so their sum is exact in float32, the fma
// G kappa + (v_grid + u_grid) rounds only a small result, and the small
// remainders are added last. This keeps row and column sums accurate to a
// few 1e-7 (a plain float32 potential of magnitude ~48 alone carries ~2e-6
// of rounding), so a 1e-6 marginal tolerance can be certified. The first
// sweep, which shifts by the row maximum, adds v_grid + v_rem once per
// column instead; at n = 10,000 both forms sweep at the same speed.
//
// One iteration = one read of G:
//   row sweep (sk_row_kernel): workgroup w owns a strip of rows. For a row i
//     it forms e_ij = 2^(G_ij kappa + v_j + u_i) for the whole row, S_i =
//     sum_j e_ij (a block reduction), the new potential u_i - log2 S_i, and
//     adds e_ij / S_i (the row-normalised plan) into per-thread column
//     accumulators. S_i is the row sum of the current plan, so |S_i - 1| is
//     the row-marginal error checked by the stop rule.
//   column update (sk_merge_kernel): c_j = sum_w partial_w[j] in a fixed
//     order, v_j <- v_j - log2 c_j, which is
//     g_j = -eps log sum_i exp((G_ij + f_i)/eps) written as a correction.
// The first iteration shifts by the exact row maximum instead of u_i (start
// potentials are arbitrary). Afterwards every term is a column-normalised
// plan entry (<= 1) and S_i, c_j lie in [1/n, n], so no further shift is
// needed.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include <hip/hip_ext.h>

#include "common.h"

namespace goat {

// Compute units of the current device (cached per device).
int cu_count() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        cached[dev] = cus;
    }
    return cached[dev];
}

namespace {

constexpr float kLog2e = 1.4426950408889634f;

// Wave-wide sum / max in a fixed order: butterfly steps xor 16, 8, 4, 2, 1
// inside each 32-lane half (ds_swizzle in bit-mask mode: lane i reads lane
// i ^ m), then the two halves' results combined. The result is uniform.
template <int M>
__device__ inline float swz_xor(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, x), 0x1F | (M << 10)));
}
__device__ inline float wave_sum(float x) {
    x += swz_xor<16>(x);
    x += swz_xor<8>(x);
    x += swz_xor<4>(x);
    x += swz_xor<2>(x);
    x += swz_xor<1>(x);
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 0)) +
           __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 32));
}
__device__ inline float wave_max(float x) {
    x = fmaxf(x, swz_xor<16>(x));
    x = fmaxf(x, swz_xor<8>(x));
    x = fmaxf(x, swz_xor<4>(x));
    x = fmaxf(x, swz_xor<2>(x));
    x = fmaxf(x, swz_xor<1>(x));
    return fmaxf(__builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 0)),
                 __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 32)));
}

// Block-wide sum / max; `red` holds T/64 floats and the callers alternate
// between two such buffers so consecutive reductions need one barrier each.
template <int T>
__device__ inline float block_sum(float x, float* red) {
    x = wave_sum(x);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    float s = 0.0f;
#pragma unroll
    for (int w = 0; w < T / 64; ++w) s += red[w];
    return s;
}
template <int T>
__device__ inline float block_max(float x, float* red) {
    x = wave_max(x);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    float s = -INFINITY;
#pragma unroll
    for (int w = 0; w < T / 64; ++w) s = fmaxf(s, red[w]);
    return s;
}

// 2^x by the hardware instruction. Results below 2^-126 flush to zero: every
// sum formed from these terms is at least 1/n (row and column sums of a
// plan normalised on the other side), so such terms are negligible.
__device__ inline float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// Moves the grid-aligned part of the remainder r into the grid part g.
__device__ inline void renorm(float& g, float& r, float h, float inv_h) {
    const float t = rintf(r * inv_h) * h;
    g += t;
    r -= t;
}

struct SkArgs {
    const float* G;
    int ldg, n, np, rpw;       // rows per workgroup
    int rev;                   // walk the strip's rows last to first
    float* ug; float* us;      // row potentials (grid part, remainder)
    float* ung; float* uns;    // new row potentials of the sweep in flight
    float* vg; float* vs;      // column potentials
    float* colpart;            // [W][np]
    float* errpart;            // [W]
    SkCtrl* ctrl;
    const uint32_t* G24;       // 24-bit copy of G (or null), ld24 words per row
    int ld24;
    int* hdone;                // host-visible copy of ctrl->done (or null)
};

// Four consecutive 24-bit two's-complement values packed little-endian in
// three words (value k occupies bits 24k .. 24k + 23 of the 96-bit group).
struct W3 {
    uint32_t x, y, z;
};
__device__ inline float4 dec24(const W3 w) {
    const int q0 = static_cast<int>(w.x << 8) >> 8;
    const int q1 = static_cast<int>(__builtin_amdgcn_alignbit(w.y, w.x, 24) << 8) >> 8;
    const int q2 = static_cast<int>(__builtin_amdgcn_alignbit(w.z, w.y, 16) << 8) >> 8;
    const int q3 = static_cast<int>(w.z) >> 8;
    return make_float4(static_cast<float>(q0), static_cast<float>(q1), static_cast<float>(q2),
                       static_cast<float>(q3));
}
__device__ inline float4 as_f4(const float4 x) { return x; }
__device__ inline float4 as_f4(const W3 w) { return dec24(w); }

// Thread t of a strip owns the float4 column groups t, t + T, ..., t + (C-1)T.
// VLDS: the column potentials sit in LDS (32 T C bytes) instead of
// registers, leaving room for more strips per compute unit. Rows of a strip
// are walked forwards or backwards (a.rev): alternating the direction
// between iterations re-reads first the rows streamed last.
// Occupancy target: two strips per compute unit (4 waves per SIMD for 512
// threads, 2 for 256), which caps the registers at 128 / 256.
template <int T, int C, bool FIRST, bool PRECISE, bool VLDS, bool Q24>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(T >= 512 ? 4 : 2)))
void sk_row_kernel(SkArgs a) {
    static_assert(!(FIRST && PRECISE), "the first sweep uses the plain form");
    extern __shared__ float4 sv4[];          // [T*C] v (grid parts), then [T*C] remainders if PRECISE
    __shared__ float red[2][T / 64];
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * a.rpw;
    const int r1 = min(a.n, r0 + a.rpw);
    // Q24: G is read as 24-bit integers q with G kappa = q * g24
    const float kappa = Q24 ? a.ctrl->g24 : a.ctrl->kappa;
    const float h = a.ctrl->h, inv_h = 1.0f / h;

    // Prologue: the strip's first row, its potential and the column
    // potentials are all requested before the stop flag is read, so the
    // launch waits for one memory round trip instead of three.
    float errmax = 0.0f;
    const int nrows = r1 - r0;
    // column groups past the row end re-read the last group (in bounds since
    // ld >= 4 ceil(n/4)); their v = -inf makes them contribute exactly 0
    const int n4m1 = ((a.n + 3) >> 2) - 1;
    using XT = typename std::conditional<Q24, W3, float4>::type;
    XT xa[C], xb[C];
#define GOAT_ROW_OF(K) (a.rev ? r1 - 1 - (K) : r0 + (K))
#define GOAT_LOAD_ROW(X, I)                                                                        \
    do {                                                                                           \
        const XT* row_ = Q24 ? reinterpret_cast<const XT*>(a.G24 + (size_t)(I) * a.ld24)           \
                             : reinterpret_cast<const XT*>(a.G + (size_t)(I) * a.ldg);            \
        _Pragma("unroll") for (int c = 0; c < C; ++c) X[c] = row_[min(tid + T * c, n4m1)];        \
    } while (0)
#define GOAT_LOAD_U(U, I)                                                                          \
    do {                                                                                           \
        if (!FIRST) U = make_float2(a.ug[I], a.us[I]);                                             \
    } while (0)
    float2 ua = make_float2(0.0f, 0.0f), ub = ua;
    if (nrows > 0) {
        GOAT_LOAD_ROW(xa, GOAT_ROW_OF(0));
        GOAT_LOAD_U(ua, GOAT_ROW_OF(0));
    }
    // np-sized arrays: one vector load per group inside np, entries past n
    // replaced below
    float4 gld[C], rld[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j4 = tid + T * c;
        gld[c] = make_float4(0.f, 0.f, 0.f, 0.f);
        rld[c] = gld[c];
        if (4 * j4 < a.np) {
            gld[c] = reinterpret_cast<const float4*>(a.vg)[j4];
            rld[c] = reinterpret_cast<const float4*>(a.vs)[j4];
        }
    }
    // the stop flag is read with the loads above in flight (a launch after
    // convergence discards them)
    if (a.ctrl->done) return;
    float4 vgr[VLDS ? 1 : C], vsr[VLDS ? 1 : C];
    float acc[C][4];
    bool live[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j4 = tid + T * c;
        live[c] = 4 * j4 < a.n;
        float g[4], r[4];
        const float4 gl = gld[c], rl = rld[c];
        const float glv[4] = {gl.x, gl.y, gl.z, gl.w}, rlv[4] = {rl.x, rl.y, rl.z, rl.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * j4 + e;
            g[e] = (j < a.n) ? glv[e] : -INFINITY;
            r[e] = (j < a.n) ? rlv[e] : 0.0f;
            if (!PRECISE) { g[e] += r[e]; r[e] = 0.0f; }
            acc[c][e] = 0.0f;
        }
        const float4 g4 = make_float4(g[0], g[1], g[2], g[3]);
        const float4 r4 = make_float4(r[0], r[1], r[2], r[3]);
        if (VLDS) {
            sv4[j4] = g4;
            if (PRECISE) sv4[T * C + j4] = r4;
        } else {
            vgr[VLDS ? 0 : c] = g4;
            vsr[VLDS ? 0 : c] = r4;
        }
    }
    if (VLDS) __syncthreads();
    // One row k held in XC with its potential (u_grid, u_rem) in UC; the next
    // row and its potential are loaded into XN, UN before row k is used, so
    // no row starts with a dependent memory round trip. The row remainder
    // u_rem enters only as the per-row factor 2^u_rem, which cancels in the
    // row-normalised plan: the sweep works with
    // y_ij = G_ij kappa + (v_grid + u_grid) + v_rem and applies 2^u_rem to
    // the row sum for the stop test.
#define GOAT_ROW_STEP(XC, XN, UC, UN, K)                                                           \
    do {                                                                                           \
        const int i = GOAT_ROW_OF(K);                                                              \
        if (VLDS) asm volatile("" ::: "memory");   /* re-read v from LDS every row */              \
        const float ug = FIRST ? 0.0f : UC.x;                                                      \
        const float us = FIRST ? 0.0f : UC.y;                                                      \
        const float uu = ug + us;                                                                  \
        float y[C][4];                                                                             \
        _Pragma("unroll") for (int c = 0; c < C; ++c) {                                            \
            const float4 g4 = VLDS ? sv4[tid + T * c] : vgr[VLDS ? 0 : c];                         \
            const float4 x4 = as_f4(XC[c]);                                                        \
            if (PRECISE) {                                                                         \
                const float4 r4 = VLDS ? sv4[T * C + tid + T * c] : vsr[VLDS ? 0 : c];             \
                y[c][0] = fmaf(x4.x, kappa, g4.x + ug) + r4.x;                                     \
                y[c][1] = fmaf(x4.y, kappa, g4.y + ug) + r4.y;                                     \
                y[c][2] = fmaf(x4.z, kappa, g4.z + ug) + r4.z;                                     \
                y[c][3] = fmaf(x4.w, kappa, g4.w + ug) + r4.w;                                     \
            } else { /* plain: g4 holds v_grid + v_rem */                                          \
                y[c][0] = fmaf(x4.x, kappa, g4.x) + uu;                                            \
                y[c][1] = fmaf(x4.y, kappa, g4.y) + uu;                                            \
                y[c][2] = fmaf(x4.z, kappa, g4.z) + uu;                                            \
                y[c][3] = fmaf(x4.w, kappa, g4.w) + uu;                                            \
            }                                                                                      \
        }                                                                                          \
        /* XC is consumed before the next row's loads are issued: issued     */                    \
        /* earlier, they would share the wait for XC (the wait counter is    */                    \
        /* in order), and the prefetch would no longer overlap the row. The  */                    \
        /* empty asm statements take y as inputs and order the loads after.  */                    \
        _Pragma("unroll") for (int c = 0; c < C; ++c)                                              \
            _Pragma("unroll") for (int e = 0; e < 4; ++e) asm volatile("" ::"v"(y[c][e]));         \
        if ((K) + 1 < nrows) {                                                                     \
            GOAT_LOAD_ROW(XN, GOAT_ROW_OF((K) + 1));                                               \
            GOAT_LOAD_U(UN, GOAT_ROW_OF((K) + 1));                                                 \
        }                                                                                          \
        float shift = 0.0f;                                                                        \
        if (FIRST) {                                                                               \
            float m = -INFINITY;                                                                   \
            _Pragma("unroll") for (int c = 0; c < C; ++c)                                          \
                _Pragma("unroll") for (int e = 0; e < 4; ++e) m = fmaxf(m, y[c][e]);              \
            shift = -block_max<T>(m, red[par]);                                                    \
            par ^= 1;                                                                              \
        }                                                                                          \
        float s = 0.0f;                                                                            \
        _Pragma("unroll") for (int c = 0; c < C; ++c)                                              \
            _Pragma("unroll") for (int e = 0; e < 4; ++e) {                                        \
                y[c][e] = exp2_fast(FIRST ? y[c][e] + shift : y[c][e]);                            \
                s += y[c][e];                                                                      \
            }                                                                                      \
        const float S = block_sum<T>(s, red[par]);   /* row sum without 2^u_rem */                 \
        par ^= 1;                                                                                  \
        const float inv = 1.0f / S;                                                                \
        _Pragma("unroll") for (int c = 0; c < C; ++c)                                              \
            _Pragma("unroll") for (int e = 0; e < 4; ++e) acc[c][e] = fmaf(y[c][e], inv, acc[c][e]); \
        if (!FIRST) errmax = fmaxf(errmax, fabsf((PRECISE ? S * exp2f(us) : S) - 1.0f));           \
        if (tid == 0) {                                                                            \
            /* new row potential: u - log2 S (first sweep: -max - log2 S); the   */                \
            /* compensated sweep's S excludes 2^u_rem, so u_rem drops out there */                 \
            float g_ = FIRST ? rintf(shift * inv_h) * h : ug;                                      \
            float r_ = FIRST ? (shift - g_) - log2f(S) : (PRECISE ? 0.0f : us) - log2f(S);         \
            renorm(g_, r_, h, inv_h);                                                              \
            a.ung[i] = g_;                                                                         \
            a.uns[i] = r_;                                                                         \
        }                                                                                          \
    } while (0)
    int par = 0;
    for (int k = 0; k < nrows; k += 2) {
        GOAT_ROW_STEP(xa, xb, ua, ub, k);
        if (k + 1 >= nrows) break;
        GOAT_ROW_STEP(xb, xa, ub, ua, k + 1);
    }
#undef GOAT_ROW_STEP
#undef GOAT_LOAD_U
#undef GOAT_LOAD_ROW
#undef GOAT_ROW_OF
    float* out = a.colpart + (size_t)blockIdx.x * a.np;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j4 = tid + T * c;
        if (4 * j4 < a.np)
            reinterpret_cast<float4*>(out)[j4] = make_float4(acc[c][0], acc[c][1], acc[c][2], acc[c][3]);
    }
    if (!FIRST) {
        const float m = block_max<T>(errmax, red[par]);
        if (tid == 0) a.errpart[blockIdx.x] = m;
    }
}

// Column update: c_j = sum over strips of the partial column sums, summed in
// a fixed order (strip lane l adds strips l, l + 32, ...; lanes combined in
// order), then v_j <- v_j - log2 c_j and u <- u_new. 256 threads = 8 float4
// column groups (one 128-byte line of a partial row) x 32 strip lanes per
// block, n/32 blocks; L strips per lane (W <= 32 L). With check, the largest
// row-marginal error of the sweep decides convergence first (no update then).
template <int L>
__global__ __launch_bounds__(256) void sk_merge_kernel(SkArgs a, int W, int check) {
    __shared__ float4 part[32][8];
    __shared__ float red[4];
    const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
    // Every load of the kernel is issued before the first one is used: the
    // stop flag, the control scalars, the column partials, the strips'
    // error partials and (threads that write columns) the potentials, so
    // the kernel waits for one memory round trip instead of four. The strip
    // loop has a fixed trip count (loads past W are predicated off), so no
    // lane waits on its loads one at a time. Loads made after convergence
    // are read and discarded.
    const int done = a.ctrl->done;
    const float tol = a.ctrl->tol, h = a.ctrl->h;
    const int cq = tid & 7, sl = tid >> 3;
    const int j4 = blockIdx.x * 8 + cq;
    const bool ok = 4 * j4 < a.n;
    float4 t[L];
    {
        const float4* cp = reinterpret_cast<const float4*>(a.colpart);
        const size_t stride = (size_t)a.np / 4;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int w = sl + 32 * l;
            t[l] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (ok && w < W) t[l] = cp[(size_t)w * stride + j4];
        }
    }
    // error partials: the array holds kSkWG >= 32 L entries, so every lane
    // loads (a predicated load would make the compiler wait for it in its
    // branch); entries past W are masked when the maximum is taken
    float e[L / 8];
#pragma unroll
    for (int l = 0; l < L / 8; ++l) e[l] = a.errpart[tid + 256 * l];
    // potentials of this thread's four columns (np-sized arrays, so the
    // vector loads stay in bounds past n)
    float4 vg4 = make_float4(0.f, 0.f, 0.f, 0.f), vs4 = vg4, ung4 = vg4, uns4 = vg4;
    if (sl == 0 && ok) {
        vg4 = reinterpret_cast<const float4*>(a.vg)[j4];
        vs4 = reinterpret_cast<const float4*>(a.vs)[j4];
        ung4 = reinterpret_cast<const float4*>(a.ung)[j4];
        uns4 = reinterpret_cast<const float4*>(a.uns)[j4];
    }
    // strips added in increasing order (zeros past W leave the sum unchanged)
    float4 acc = t[0];
#pragma unroll
    for (int l = 1; l < L; ++l) {
        acc.x += t[l].x; acc.y += t[l].y; acc.z += t[l].z; acc.w += t[l].w;
    }
    float m = 0.0f;
#pragma unroll
    for (int l = 0; l < L / 8; ++l)
        if (check && tid + 256 * l < W) m = fmaxf(m, e[l]);
    if (done) return;
    if (check) {
        m = wave_max(m);
        if (lane == 0) red[q] = m;
        __syncthreads();
        const float err = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        if (err <= tol) {
            if (blockIdx.x == 0 && tid == 0) {
                a.ctrl->err = err;
                a.ctrl->done = 1;
                if (a.hdone) {
                    *a.hdone = 1;
                    __threadfence_system();
                }
            }
            return;
        }
        if (blockIdx.x == 0 && tid == 0) a.ctrl->err = err;
    }
    part[sl][cq] = acc;
    __syncthreads();
    if (sl == 0 && ok) {
        float4 c = part[0][cq];
#pragma unroll
        for (int l = 1; l < 32; ++l) {
            const float4 t = part[l][cq];
            c.x += t.x; c.y += t.y; c.z += t.z; c.w += t.w;
        }
        const float cc[4] = {c.x, c.y, c.z, c.w};
        const float vgv[4] = {vg4.x, vg4.y, vg4.z, vg4.w};
        const float vsv[4] = {vs4.x, vs4.y, vs4.z, vs4.w};
        const float ungv[4] = {ung4.x, ung4.y, ung4.z, ung4.w};
        const float unsv[4] = {uns4.x, uns4.y, uns4.z, uns4.w};
        const float inv_h = 1.0f / h;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * j4 + e;
            if (j < a.n) {
                float g = vgv[e], r = vsv[e] - log2f(fmaxf(cc[e], 1.17549435e-38f));
                renorm(g, r, h, inv_h);
                a.vg[j] = g;
                a.vs[j] = r;
                a.ug[j] = ungv[e];
                a.us[j] = unsv[e];
            }
        }
    }
    if (blockIdx.x == 0 && tid == 0) a.ctrl->iters += 1;
}

// eps from eps_dev or eps_rel * max|G|; grid step h from max|G| kappa;
// potentials initialised (v from the caller's g when given).
__global__ __launch_bounds__(256) void sk_init_kernel(int n, const float* eps_dev, float eps_rel,
                                                      const float* absmax, const float* g_init,
                                                      float tol, SkArgs a) {
    const float gmax = *absmax;
    const float eps = eps_dev ? *eps_dev : eps_rel * gmax;
    const bool ok = eps > 0.0f && gmax > 0.0f;
    const float kappa = ok ? kLog2e / eps : 0.0f;
    // h = 2^(e - 24) with 2^e >= max|G kappa| + 64
    int e = 0;
    frexpf(gmax * kappa + 64.0f, &e);
    const float h = ldexpf(1.0f, e - 24);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        a.ug[i] = 0.0f;
        a.us[i] = 0.0f;
        float g = 0.0f, r = 0.0f;
        if (g_init && ok) {
            r = g_init[i] * kappa;
            renorm(g, r, h, 1.0f / h);
        }
        a.vg[i] = g;
        a.vs[i] = r;
    }
    if (i == 0) {
        a.ctrl->kappa = kappa;
        a.ctrl->eps = eps;
        a.ctrl->h = h;
        a.ctrl->done = ok ? 0 : 2;
        if (a.hdone) {
            *a.hdone = ok ? 0 : 2;
            __threadfence_system();
        }
        a.ctrl->iters = 0;
        a.ctrl->err = 0.0f;
        a.ctrl->tol = tol;
    }
}

// Q = 2^(G kappa + u_i + v_j) (or J when eps == 0), its largest row-marginal
// error, and optional bf16 hi/lo planes of Q (np stride).
struct FinArgs {
    SkArgs a;
    float* Q; int ldq;
    uint16_t* Qhi; uint16_t* Qlo;
};

template <int T, int C, bool Q24>
__global__ __launch_bounds__(T) void sk_finalize_kernel(FinArgs fa) {
    const SkArgs& a = fa.a;
    __shared__ float red[2][T / 64];
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * a.rpw;
    const int r1 = min(a.n, r0 + a.rpw);
    // Q24: Q is formed from the same 24-bit G the sweeps read
    const float kappa = Q24 ? a.ctrl->g24 : a.ctrl->kappa;
    const bool flat = a.ctrl->done == 2;
    const float jval = 1.0f / (float)a.n;
    using XT = typename std::conditional<Q24, W3, float4>::type;
    // column potentials of this thread's groups, read once for all rows
    float vgl[C][4], vsl[C][4];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * (tid + T * c) + e;
            vgl[c][e] = j < a.n ? a.vg[j] : 0.0f;
            vsl[c][e] = j < a.n ? a.vs[j] : 0.0f;
        }
    // one row of G in flight ahead of the row being written (rows past the
    // strip are not loaded; groups past n read zeros)
    XT xa[C], xb[C];
    float2 ua = make_float2(0.0f, 0.0f), ub = ua;
#define GOAT_FIN_LOAD(X, U, I)                                                                     \
    do {                                                                                           \
        _Pragma("unroll") for (int c = 0; c < C; ++c) {                                            \
            const int j0_ = 4 * (tid + T * c);                                                     \
            if (j0_ < a.n) {                                                                       \
                if constexpr (Q24) X[c] = reinterpret_cast<const W3*>(a.G24 + (size_t)(I) * a.ld24)[j0_ >> 2]; \
                else X[c] = *reinterpret_cast<const float4*>(a.G + (size_t)(I) * a.ldg + j0_);     \
            }                                                                                      \
        }                                                                                          \
        U = make_float2(a.ug[I], a.us[I]);                                                         \
    } while (0)
    float errmax = 0.0f;
    int par = 0;
    if (r0 < r1) GOAT_FIN_LOAD(xa, ua, r0);
#define GOAT_FIN_ROW(XC, XN, UC, UN, I)                                                            \
    do {                                                                                           \
        const float ug = UC.x, us = UC.y;                                                          \
        float q[C][4];                                                                             \
        _Pragma("unroll") for (int c = 0; c < C; ++c) {                                            \
            const int j0 = 4 * (tid + T * c);                                                      \
            float4 g4 = make_float4(0.f, 0.f, 0.f, 0.f);                                           \
            if (j0 < a.n) g4 = as_f4(XC[c]);                                                       \
            const float gv[4] = {g4.x, g4.y, g4.z, g4.w};                                          \
            _Pragma("unroll") for (int e = 0; e < 4; ++e) {                                        \
                const int j = j0 + e;                                                              \
                q[c][e] = 0.0f;                                                                    \
                if (j < a.n)                                                                       \
                    q[c][e] = flat ? jval : exp2f(fmaf(gv[e], kappa, vgl[c][e] + ug) + (vsl[c][e] + us)); \
            }                                                                                      \
        }                                                                                          \
        /* the row is consumed before the next row's loads are issued (the  */                     \
        /* wait counter is in order)                                        */                     \
        _Pragma("unroll") for (int c = 0; c < C; ++c)                                              \
            _Pragma("unroll") for (int e = 0; e < 4; ++e) asm volatile("" ::"v"(q[c][e]));         \
        if ((I) + 1 < r1) GOAT_FIN_LOAD(XN, UN, (I) + 1);                                          \
        float s = 0.0f;                                                                            \
        _Pragma("unroll") for (int c = 0; c < C; ++c) {                                            \
            const int j0 = 4 * (tid + T * c);                                                      \
            if (j0 >= a.np && j0 >= a.n) continue;                                                 \
            _Pragma("unroll") for (int e = 0; e < 4; ++e) s += q[c][e];                            \
            if (fa.Q) {                                                                            \
                float* qrow = fa.Q + (size_t)(I) * fa.ldq;                                         \
                if (j0 + 3 < a.n && (fa.ldq & 3) == 0) {                                           \
                    *reinterpret_cast<float4*>(qrow + j0) = make_float4(q[c][0], q[c][1], q[c][2], q[c][3]); \
                } else {                                                                           \
                    _Pragma("unroll") for (int e = 0; e < 4; ++e)                                  \
                        if (j0 + e < a.n) qrow[j0 + e] = q[c][e];                                  \
                }                                                                                  \
            }                                                                                      \
            if (fa.Qhi && j0 < a.np) {                                                             \
                ushort4 hi, lo;                                                                    \
                uint16_t hv[4], lv[4];                                                             \
                _Pragma("unroll") for (int e = 0; e < 4; ++e) {                                    \
                    hv[e] = f32_to_bf16_rne(q[c][e]);                                              \
                    lv[e] = f32_to_bf16_rne(q[c][e] - bf16_to_f32(hv[e]));                         \
                }                                                                                  \
                hi.x = hv[0]; hi.y = hv[1]; hi.z = hv[2]; hi.w = hv[3];                            \
                lo.x = lv[0]; lo.y = lv[1]; lo.z = lv[2]; lo.w = lv[3];                            \
                *reinterpret_cast<ushort4*>(fa.Qhi + (size_t)(I) * a.np + j0) = hi;                \
                *reinterpret_cast<ushort4*>(fa.Qlo + (size_t)(I) * a.np + j0) = lo;                \
            }                                                                                      \
        }                                                                                          \
        const float S = block_sum<T>(s, red[par]);                                                 \
        par ^= 1;                                                                                  \
        errmax = fmaxf(errmax, fabsf(S - 1.0f));                                                   \
    } while (0)
    for (int i = r0; i < r1; i += 2) {
        GOAT_FIN_ROW(xa, xb, ua, ub, i);
        if (i + 1 >= r1) break;
        GOAT_FIN_ROW(xb, xa, ub, ua, i + 1);
    }
#undef GOAT_FIN_ROW
#undef GOAT_FIN_LOAD
    const float m = block_max<T>(errmax, red[par]);
    if (tid == 0) a.errpart[blockIdx.x] = m;
}

__global__ __launch_bounds__(256) void sk_outputs_kernel(SkArgs a, int W, float* f, float* g,
                                                         int* iters_out, float* err_out,
                                                         float* eps_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const float kappa = a.ctrl->kappa;
    const bool flat = a.ctrl->done == 2;
    if (i < a.n) {
        if (f) f[i] = flat ? 0.0f : (a.ug[i] + a.us[i]) / kappa;
        if (g) g[i] = flat ? 0.0f : (a.vg[i] + a.vs[i]) / kappa;
    }
    if (i == 0) {
        float m = 0.0f;
        for (int w = 0; w < W; ++w) m = fmaxf(m, a.errpart[w]);
        if (err_out) *err_out = m;
        if (iters_out) *iters_out = a.ctrl->iters;
        if (eps_out) *eps_out = a.ctrl->eps;
    }
}

// ---------------------------------------------------------------- dispatch

struct Geometry {
    int T, C, W, rpw;
};

// Strips: below n = 4096, 256 threads and up to 512 strips; from n = 4096,
// 1024 threads (16 waves) and one strip per compute unit, so every strip
// streams many rows and the per-strip prologue (potentials into LDS) and
// epilogue (column partials) are amortised (n = 10,000, when this geometry
// was chosen: 68.6 us per sweep against 81.1 us with 512 x 512 threads).
// GOAT_SK_GEOM="T,W" overrides both (a measurement knob).
constexpr int kSkSmallWG = 512;


Geometry geometry(int n) {
    int env_T = 0, env_W = 0;
    if (const char* e = getenv("GOAT_SK_GEOM")) {
        int t = 0, w = 0;
        if (sscanf(e, "%d,%d", &t, &w) == 2 && (t == 256 || t == 512 || t == 1024) && w >= 1 && w <= kSkWG) {
            env_T = t;
            env_W = w;
        }
    }
    Geometry g;
    const int n4 = (n + 3) / 4;
    const bool large = n >= 4096;
    g.T = large ? 1024 : 256;
    if (env_T > 0 && n4 <= env_T * 16) g.T = env_T;
    g.C = (n4 + g.T - 1) / g.T;
    const int cs[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16};
    for (int c : cs)
        if (c >= g.C) { g.C = c; break; }
    const int wmax = env_W > 0 ? env_W : (large ? std::min(cu_count(), kSkWG) : kSkSmallWG);
    g.W = n < wmax ? n : wmax;
    g.rpw = (n + g.W - 1) / g.W;
    g.W = (n + g.rpw - 1) / g.rpw;
    return g;
}

// LDS for the column potentials: 32 T C bytes; above 64 KB the kernel asks
// for the larger dynamic allocation once, and keeps v in registers if the
// runtime refuses.
template <typename K>
bool allow_lds(K kfn, size_t bytes) {
    if (bytes <= 65536) return true;
    if (bytes > 160 * 1024) return false;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kfn), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes) == hipSuccess;
}

template <int T, int C, bool FIRST, bool PRECISE, bool Q24>
void launch_row_TCPQ(const Geometry& g, const SkArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const size_t lds = (size_t)(PRECISE ? 32 : 16) * T * C;
    static const bool vlds = allow_lds(sk_row_kernel<T, C, FIRST, PRECISE, true, Q24>, lds);
    if (e0) {
        // a sampled launch: the events mark the kernel's own start and end
        if (vlds)
            hipExtLaunchKernelGGL((sk_row_kernel<T, C, FIRST, PRECISE, true, Q24>), dim3(g.W), dim3(T),
                                  (uint32_t)lds, s, e0, e1, 0, a);
        else
            hipExtLaunchKernelGGL((sk_row_kernel<T, C, FIRST, PRECISE, false, Q24>), dim3(g.W), dim3(T), 0, s, e0,
                                  e1, 0, a);
        return;
    }
    if (vlds) hipLaunchKernelGGL((sk_row_kernel<T, C, FIRST, PRECISE, true, Q24>), dim3(g.W), dim3(T), lds, s, a);
    else hipLaunchKernelGGL((sk_row_kernel<T, C, FIRST, PRECISE, false, Q24>), dim3(g.W), dim3(T), 0, s, a);
}

template <int T, int C, bool FIRST, bool PRECISE>
void launch_row_TCP(const Geometry& g, const SkArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (a.G24) launch_row_TCPQ<T, C, FIRST, PRECISE, true>(g, a, s, e0, e1);
    else launch_row_TCPQ<T, C, FIRST, PRECISE, false>(g, a, s, e0, e1);
}

template <int T, bool FIRST>
int launch_row_T(const Geometry& g, const SkArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                 hipEvent_t e1 = nullptr) {
    switch (g.C) {
#define GOAT_SK_C(CC) case CC: launch_row_TCP<T, CC, FIRST, !FIRST>(g, a, s, e0, e1); break;
        GOAT_SK_C(1) GOAT_SK_C(2) GOAT_SK_C(3) GOAT_SK_C(4) GOAT_SK_C(5) GOAT_SK_C(6)
        GOAT_SK_C(8) GOAT_SK_C(10) GOAT_SK_C(12) GOAT_SK_C(16)
#undef GOAT_SK_C
        default: set_error("sinkhorn: unsupported n"); return GOAT_ENOTSUP;
    }
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

template <int T>
int launch_fin_T(const Geometry& g, const FinArgs& fa, hipStream_t s) {
    dim3 grid(g.W), block(T);
    switch (g.C) {
#define GOAT_SK_C(CC)                                                                              \
    case CC:                                                                                       \
        if (fa.a.G24) hipLaunchKernelGGL((sk_finalize_kernel<T, CC, true>), grid, block, 0, s, fa);   \
        else hipLaunchKernelGGL((sk_finalize_kernel<T, CC, false>), grid, block, 0, s, fa);           \
        break;
        GOAT_SK_C(1) GOAT_SK_C(2) GOAT_SK_C(3) GOAT_SK_C(4) GOAT_SK_C(5) GOAT_SK_C(6)
        GOAT_SK_C(8) GOAT_SK_C(10) GOAT_SK_C(12) GOAT_SK_C(16)
#undef GOAT_SK_C
        default: set_error("sinkhorn: unsupported n"); return GOAT_ENOTSUP;
    }
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

SkArgs make_args(int n, int np, const float* G, int ldg, const SkState& st, const Geometry& g) {
    SkArgs a;
    a.G = G;
    a.ldg = ldg;
    a.n = n;
    a.np = np;
    a.rpw = g.rpw;
    a.rev = 0;
    a.ug = st.ug; a.us = st.us;
    a.ung = st.ung; a.uns = st.uns;
    a.vg = st.vg; a.vs = st.vs;
    a.colpart = st.colpart;
    a.errpart = st.errpart;
    a.ctrl = st.ctrl;
    a.G24 = st.g24;
    a.ld24 = st.ld24;
    a.hdone = st.hdone;
    return a;
}

// 24-bit copy of G: one thread per four columns of a row (zero past n)
__global__ __launch_bounds__(256) void pack_g24_kernel(int n, int np, const float* __restrict__ G, int ldg,
                                                       const float* absmax, SkCtrl* ctrl, uint32_t* out, int ld24) {
    const float gmax = *absmax;
    const float qmax = 8388607.0f;                      // 2^23 - 1
    const float s = gmax > 0.0f ? qmax / gmax : 0.0f;
    const int i = blockIdx.y;
    const int j4 = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && j4 == 0) ctrl->g24 = gmax > 0.0f ? ctrl->kappa * (gmax / qmax) : 0.0f;
    if (4 * j4 >= np) return;
    const float* row = G + (size_t)i * ldg;
    int q[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int j = 4 * j4 + e;
        const float x = j < n ? row[j] : 0.0f;
        q[e] = static_cast<int>(fminf(fmaxf(rintf(x * s), -qmax), qmax));
    }
    uint32_t* w = out + (size_t)i * ld24 + 3 * j4;
    w[0] = (static_cast<uint32_t>(q[0]) & 0xFFFFFFu) | (static_cast<uint32_t>(q[1]) << 24);
    w[1] = ((static_cast<uint32_t>(q[1]) >> 8) & 0xFFFFu) | (static_cast<uint32_t>(q[2]) << 16);
    w[2] = ((static_cast<uint32_t>(q[2]) >> 16) & 0xFFu) | (static_cast<uint32_t>(q[3]) << 8);
}

}  // namespace

int sk_prepare(int n, const float* G, int ldg, const float* eps_dev, float eps_rel,
               const float* absmax_dev, const float* g_init, float tol, SkState st, float* fscal,
               double* red, hipStream_t s) {
    (void)red;
    const float* absmax = absmax_dev;
    if (!absmax) {
        int rc = launch_absmax(n, G, ldg, fscal + 16, fscal, s);
        if (rc) return rc;
        absmax = fscal;
    }
    const Geometry g = geometry(n);
    const SkArgs a = make_args(n, pad_n(n), G, ldg, st, g);
    hipLaunchKernelGGL(sk_init_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, eps_dev, eps_rel, absmax,
                       g_init, tol, a);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int sk_pack_g24(int n, int np, const float* G, int ldg, const float* absmax_dev, SkState st, hipStream_t s) {
    if (!st.g24 || st.ld24 < 3 * (np / 4)) {
        set_error("sinkhorn: no 24-bit buffer");
        return GOAT_EINVAL;
    }
    dim3 grid((np / 4 + 255) / 256, n);
    hipLaunchKernelGGL(pack_g24_kernel, grid, dim3(256), 0, s, n, np, G, ldg, absmax_dev, st.ctrl,
                       const_cast<uint32_t*>(st.g24), st.ld24);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int sk_iterate(int n, int np, const float* G, int ldg, SkState st, int first, int check, int iter,
               hipStream_t s, bool sample) {
    const Geometry g = geometry(n);
    SkArgs a = make_args(n, np, G, ldg, st, g);
    a.rev = iter & 1;
    int rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    // only the steady-state (compensated) sweep is sampled
    const bool sampled = sample && !first && prof_sample(0, &e0, &e1);
    if (g.T == 256)
        rc = first ? launch_row_T<256, true>(g, a, s, e0, e1) : launch_row_T<256, false>(g, a, s, e0, e1);
    else if (g.T == 512)
        rc = first ? launch_row_T<512, true>(g, a, s, e0, e1) : launch_row_T<512, false>(g, a, s, e0, e1);
    else
        rc = first ? launch_row_T<1024, true>(g, a, s, e0, e1) : launch_row_T<1024, false>(g, a, s, e0, e1);
    if (sampled && rc == GOAT_OK) prof_commit(0);
    if (rc) return rc;
    const dim3 mgrid((n + 31) / 32), mblock(256);
    if (g.W <= 256) hipLaunchKernelGGL(sk_merge_kernel<8>, mgrid, mblock, 0, s, a, g.W, check);
    else if (g.W <= 512) hipLaunchKernelGGL(sk_merge_kernel<16>, mgrid, mblock, 0, s, a, g.W, check);
    else hipLaunchKernelGGL(sk_merge_kernel<32>, mgrid, mblock, 0, s, a, g.W, check);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int sk_finalize(int n, int np, const float* G, int ldg, SkState st, float* Q, int ldq, uint16_t* Q_hi,
                uint16_t* Q_lo, float* f, float* g, int* iters_out, float* err_out, float* eps_out,
                double* red, hipStream_t s) {
    (void)red;
    const Geometry geo = geometry(n);
    FinArgs fa;
    fa.a = make_args(n, np, G, ldg, st, geo);
    fa.Q = Q;
    fa.ldq = ldq;
    fa.Qhi = Q_hi;
    fa.Qlo = Q_lo;
    int rc = geo.T == 256 ? launch_fin_T<256>(geo, fa, s)
             : (geo.T == 512 ? launch_fin_T<512>(geo, fa, s) : launch_fin_T<1024>(geo, fa, s));
    if (rc) return rc;
    hipLaunchKernelGGL(sk_outputs_kernel, dim3((n + 255) / 256), dim3(256), 0, s, fa.a, geo.W, f, g,
                       iters_out, err_out, eps_out);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

}  // namespace goat
