// Log-domain Sinkhorn-Knopp scaling for the LOT direction (Alg. 2, with the
// cost negated for the maximisation of Alg. 3 step 2).
//
// Internal units: potentials in base 2 scaled by 1/eps,
//     u_i = f_i * kappa,  v_j = g_j * kappa,  kappa = log2(e) / eps,
// so Q_ij = 2^(G_ij kappa + u_i + v_j).
//
// One iteration = one read of G:
//   row pass  (sk_row_kernel):  workgroup w owns a strip of rows. For a row i
//     it forms e_ij = 2^(G_ij kappa + v_j + u_i) for the whole row (held in
//     registers), S_i = sum_j e_ij (a block reduction), the new potential
//     u_i - log2 S_i, and adds e_ij / S_i (the row-normalised plan) into
//     per-thread column accumulators. S_i is the row sum of the current plan,
//     so |S_i - 1| is the row-marginal error checked by the stop rule.
//   merge     (sk_merge_kernel): c_j = sum_w partial_w[j] in fixed order,
//     v_j <- v_j - log2 c_j, which is the column update
//     g_j = -eps log sum_i exp((G_ij + f_i)/eps) written as a correction.
// The first iteration shifts by the exact row maximum instead of u_i (the
// start potentials are arbitrary). Afterwards every term is a column-
// normalised plan entry (<= 1) and S_i, c_j lie in [1/n, n], so no further
// shift is needed.
#include <hip/hip_cooperative_groups.h>

#include <cstdio>
#include <cstdlib>

#include "common.h"

namespace cg = cooperative_groups;

namespace goat {
namespace {

constexpr float kLog2e = 1.4426950408889634f;

__device__ inline float wave_sum(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
__device__ inline float wave_max(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
    return x;
}
__device__ inline double wave_sum_d(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Block-wide sum / max; `red` holds T/64 floats and alternates between two
// halves so consecutive reductions need one barrier each.
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

// G is streamed once per iteration: non-temporal loads when GOAT_SK_NT is
// defined at build time, plain loads otherwise.
#ifdef GOAT_SK_NT
typedef float goat_f4v __attribute__((ext_vector_type(4)));
__device__ inline float4 goat_nt_load(const float4* p) {
    const goat_f4v v = __builtin_nontemporal_load(reinterpret_cast<const goat_f4v*>(p));
    return make_float4(v[0], v[1], v[2], v[3]);
}
#define GOAT_GLOAD(P) goat_nt_load(P)
#else
#define GOAT_GLOAD(P) (*(P))
#endif

struct SkArgs {
    const float* G;
    int ldg, n, np, rpw;       // rows per workgroup
    int rev;                   // walk the strip's rows last to first
    float* u;
    float* unew;
    float* v;
    float* colpart;            // [W][np]
    float* errpart;            // [W]
    SkCtrl* ctrl;
};

// Thread t of a strip owns the float4 column groups t, t + T, ..., t + (C-1)T.
// R rows are processed per step (one block reduction for all R row sums)
// and the next R rows are loaded while the current ones reduce.
// VLDS: the column potentials sit in LDS (16 T C bytes) instead of
// registers, which leaves room for more rows in flight. Rows of a strip are
// walked forwards or backwards (a.rev): alternating the direction between
// iterations re-reads first the rows streamed last, which are the ones still
// held in the memory-side cache when G is larger than it.
template <int T, int R>
__device__ inline void block_sum_r(float (&x)[R], float* red) {
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = wave_sum(x[r]);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) red[r * (T / 64) + (threadIdx.x >> 6)] = x[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float s = 0.0f;
#pragma unroll
        for (int w = 0; w < T / 64; ++w) s += red[r * (T / 64) + w];
        x[r] = s;
    }
}
template <int T, int R>
__device__ inline void block_max_r(float (&x)[R], float* red) {
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = wave_max(x[r]);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) red[r * (T / 64) + (threadIdx.x >> 6)] = x[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float s = -INFINITY;
#pragma unroll
        for (int w = 0; w < T / 64; ++w) s = fmaxf(s, red[r * (T / 64) + w]);
        x[r] = s;
    }
}

template <int T, int C, int R, bool FIRST, bool VLDS>
__global__ __launch_bounds__(T) void sk_row_kernel(SkArgs a) {
    if (a.ctrl->done) return;
    extern __shared__ float4 sv4[];
    __shared__ float red[2][R * (T / 64)];
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * a.rpw;
    const int r1 = min(a.n, r0 + a.rpw);
    const float kappa = a.ctrl->kappa;

    float4 vreg[VLDS ? 1 : C];
    float acc[C][4];
    bool live[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j4 = tid + T * c;
        live[c] = 4 * j4 < a.n;
        float vv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * j4 + e;
            vv[e] = (j < a.n) ? a.v[j] : -INFINITY;
            acc[c][e] = 0.0f;
        }
        const float4 v4 = make_float4(vv[0], vv[1], vv[2], vv[3]);
        if (VLDS) sv4[j4] = v4;
        else vreg[VLDS ? 0 : c] = v4;
    }
    if (VLDS) __syncthreads();
    float errmax = 0.0f;
    const int nrows = r1 - r0;
    auto row_of = [&](int k) { return a.rev ? r1 - 1 - k : r0 + k; };
    float4 x[R][C];
    // rows k0 .. k0+R-1 of the strip into x (rows past the strip read as zero)
#define GOAT_LOAD_ROWS(K0)                                                                          \
    do {                                                                                            \
        _Pragma("unroll") for (int r = 0; r < R; ++r) {                                             \
            const bool ok_ = (K0) + r < nrows;                                                      \
            const float4* row_ = reinterpret_cast<const float4*>(                                   \
                a.G + (size_t)(ok_ ? row_of((K0) + r) : r0) * a.ldg);                               \
            _Pragma("unroll") for (int c = 0; c < C; ++c)                                           \
                x[r][c] = (ok_ && live[c]) ? GOAT_GLOAD(row_ + tid + T * c)                          \
                                           : make_float4(0.f, 0.f, 0.f, 0.f);                        \
        }                                                                                           \
    } while (0)
    if (nrows > 0) GOAT_LOAD_ROWS(0);
    int par = 0;
    for (int k0 = 0; k0 < nrows; k0 += R) {
        // keep the LDS copy of v authoritative: re-read it every step instead
        // of letting the compiler cache it in registers
        if (VLDS) asm volatile("" ::: "memory");
        float y[R][C][4];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float4 v4 = VLDS ? sv4[tid + T * c] : vreg[VLDS ? 0 : c];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                y[r][c][0] = fmaf(x[r][c].x, kappa, v4.x);
                y[r][c][1] = fmaf(x[r][c].y, kappa, v4.y);
                y[r][c][2] = fmaf(x[r][c].z, kappa, v4.z);
                y[r][c][3] = fmaf(x[r][c].w, kappa, v4.w);
            }
        }
        // x is consumed: prefetch the next R rows into it while these reduce
        if (k0 + R < nrows) GOAT_LOAD_ROWS(k0 + R);
        float shift[R], s[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            s[r] = 0.0f;
            const bool ok = k0 + r < nrows;
            if (FIRST) {
                float m = -INFINITY;
#pragma unroll
                for (int c = 0; c < C; ++c)
#pragma unroll
                    for (int e = 0; e < 4; ++e) m = fmaxf(m, y[r][c][e]);
                shift[r] = m;
            } else {
                shift[r] = ok ? a.u[row_of(k0 + r)] : 0.0f;
            }
        }
        if (FIRST) {
            block_max_r<T, R>(shift, red[par]);
            par ^= 1;
#pragma unroll
            for (int r = 0; r < R; ++r) shift[r] = (k0 + r < nrows) ? -shift[r] : 0.0f;
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    y[r][c][e] = exp2f(y[r][c][e] + shift[r]);
                    s[r] += y[r][c][e];
                }
        block_sum_r<T, R>(s, red[par]);
        par ^= 1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (k0 + r >= nrows) break;
            const float inv = 1.0f / s[r];
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[c][e] = fmaf(y[r][c][e], inv, acc[c][e]);
            if (!FIRST) errmax = fmaxf(errmax, fabsf(s[r] - 1.0f));
            if (tid == 0) a.unew[row_of(k0 + r)] = shift[r] - log2f(s[r]);
        }
    }
#undef GOAT_LOAD_ROWS
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

// Whole Sinkhorn solve in one cooperative launch: every workgroup owns a
// row strip (row phase as in sk_row_kernel) and, after a grid barrier, a
// slice of columns (the column update as in sk_merge_kernel, same fixed
// summation order over strips). All workgroups evaluate the stop test on the
// same partials, so they leave the loop together. Iterations k_begin ..
// k_end-1 run; k == 0 is the max-shifted first sweep.
struct SkPersist {
    int k_begin, k_end, W, cpw;
};

template <int T, int C>
__global__ __launch_bounds__(T) void sk_persistent_kernel(SkArgs a, SkPersist pp) {
    if (a.ctrl->done) return;
    cg::grid_group grid = cg::this_grid();
    extern __shared__ float4 sv4[];
    __shared__ float red[2][T / 64];
    __shared__ float mpart[T / 64][64];
    const int tid = threadIdx.x, w = blockIdx.x;
    const int r0 = w * a.rpw;
    const int r1 = min(a.n, r0 + a.rpw);
    const int nrows = max(r1 - r0, 0);
    const float kappa = a.ctrl->kappa;
    const float tol = a.ctrl->tol;
    bool live[C];
#pragma unroll
    for (int c = 0; c < C; ++c) live[c] = 4 * (tid + T * c) < a.n;

    for (int k = pp.k_begin; k < pp.k_end; ++k) {
        const bool first = (k == 0);
        const bool rev = (k & 1) != 0;
        // ---------------- row phase
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j4 = tid + T * c;
            float vv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = 4 * j4 + e;
                vv[e] = (j < a.n) ? a.v[j] : -INFINITY;
            }
            sv4[j4] = make_float4(vv[0], vv[1], vv[2], vv[3]);
        }
        __syncthreads();
        float acc[C][4];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[c][e] = 0.0f;
        float errmax = 0.0f;
        float4 x[C];
        int par = 0;
#define GOAT_ROW_OF(K) (rev ? r1 - 1 - (K) : r0 + (K))
#define GOAT_LOAD_ROW(I)                                                                           \
    do {                                                                                           \
        const float4* row_ = reinterpret_cast<const float4*>(a.G + (size_t)(I) * a.ldg);          \
        _Pragma("unroll") for (int c = 0; c < C; ++c)                                              \
            x[c] = live[c] ? row_[tid + T * c] : make_float4(0.f, 0.f, 0.f, 0.f);                \
    } while (0)
        if (nrows > 0) GOAT_LOAD_ROW(GOAT_ROW_OF(0));
        for (int kk = 0; kk < nrows; ++kk) {
            const int i = GOAT_ROW_OF(kk);
            asm volatile("" ::: "memory");
            float y[C][4];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float4 v4 = sv4[tid + T * c];
                y[c][0] = fmaf(x[c].x, kappa, v4.x);
                y[c][1] = fmaf(x[c].y, kappa, v4.y);
                y[c][2] = fmaf(x[c].z, kappa, v4.z);
                y[c][3] = fmaf(x[c].w, kappa, v4.w);
            }
            if (kk + 1 < nrows) GOAT_LOAD_ROW(GOAT_ROW_OF(kk + 1));
            float shift;
            if (first) {
                float m = -INFINITY;
#pragma unroll
                for (int c = 0; c < C; ++c)
#pragma unroll
                    for (int e = 0; e < 4; ++e) m = fmaxf(m, y[c][e]);
                shift = -block_max<T>(m, red[par]);
                par ^= 1;
            } else {
                shift = a.u[i];
            }
            float s = 0.0f;
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    y[c][e] = exp2f(y[c][e] + shift);
                    s += y[c][e];
                }
            const float S = block_sum<T>(s, red[par]);
            par ^= 1;
            const float inv = 1.0f / S;
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[c][e] = fmaf(y[c][e], inv, acc[c][e]);
            if (!first) errmax = fmaxf(errmax, fabsf(S - 1.0f));
            if (tid == 0) a.unew[i] = shift - log2f(S);
        }
#undef GOAT_LOAD_ROW
#undef GOAT_ROW_OF
        float* out = a.colpart + (size_t)w * a.np;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j4 = tid + T * c;
            if (4 * j4 < a.np)
                reinterpret_cast<float4*>(out)[j4] = make_float4(acc[c][0], acc[c][1], acc[c][2], acc[c][3]);
        }
        {
            const float m = block_max<T>(errmax, red[par]);
            par ^= 1;
            if (tid == 0) a.errpart[w] = m;
        }
        grid.sync();
        // ---------------- column phase
        if (!first) {
            float m = 0.0f;
            for (int q = tid; q < pp.W; q += T) m = fmaxf(m, a.errpart[q]);
            const float err = block_max<T>(m, red[par]);
            par ^= 1;
            if (w == 0 && tid == 0) a.ctrl->err = err;
            if (err <= tol) {
                if (w == 0 && tid == 0) a.ctrl->done = 1;
                break;                           // the same decision in every workgroup
            }
        }
        const int lane = tid & 63, sl = tid >> 6;   // 64 columns x T/64 strip lanes
        const int cbeg = w * pp.cpw, cend = min(a.n, cbeg + pp.cpw);
        for (int cb = cbeg; cb < cend; cb += 64) {
            const int j = cb + lane;
            float part = 0.0f;
            if (j < cend)
                for (int q = sl; q < pp.W; q += T / 64) part += a.colpart[(size_t)q * a.np + j];
            mpart[sl][lane] = part;
            __syncthreads();
            if (sl == 0 && j < cend) {
                float c = mpart[0][lane];
#pragma unroll
                for (int l = 1; l < T / 64; ++l) c += mpart[l][lane];
                a.v[j] -= log2f(fmaxf(c, 1.17549435e-38f));
                a.u[j] = a.unew[j];
            }
            __syncthreads();
        }
        if (w == 0 && tid == 0) a.ctrl->iters += 1;
        grid.sync();
    }
}

// Column update: c_j = sum over strips of the partial column sums, summed in
// a fixed order (strip lane l adds strips l, l + 16, ...; lanes combined in
// order), then v_j <- v_j - log2 c_j and u <- unew. 256 threads = 16 float4
// column groups x 16 strip lanes per block.
__global__ __launch_bounds__(256) void sk_merge_kernel(SkArgs a, int W, int check) {
    if (a.ctrl->done) return;
    __shared__ float4 part[16][16];
    __shared__ float red[4];
    const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
    if (check) {
        float m = 0.0f;
        for (int w = tid; w < W; w += 256) m = fmaxf(m, a.errpart[w]);
        m = wave_max(m);
        if (lane == 0) red[q] = m;
        __syncthreads();
        const float err = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        if (err <= a.ctrl->tol) {
            if (blockIdx.x == 0 && tid == 0) {
                a.ctrl->err = err;
                a.ctrl->done = 1;
            }
            return;
        }
        if (blockIdx.x == 0 && tid == 0) a.ctrl->err = err;
    }
    const int cq = tid & 15, sl = tid >> 4;
    const int j4 = blockIdx.x * 16 + cq;
    const bool ok = 4 * j4 < a.n;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ok) {
        const float4* cp = reinterpret_cast<const float4*>(a.colpart);
        const size_t stride = (size_t)a.np / 4;
#pragma unroll 4
        for (int w = sl; w < W; w += 16) {
            const float4 t = cp[(size_t)w * stride + j4];
            acc.x += t.x; acc.y += t.y; acc.z += t.z; acc.w += t.w;
        }
    }
    part[sl][cq] = acc;
    __syncthreads();
    if (sl == 0 && ok) {
        float4 c = part[0][cq];
#pragma unroll
        for (int l = 1; l < 16; ++l) {
            const float4 t = part[l][cq];
            c.x += t.x; c.y += t.y; c.z += t.z; c.w += t.w;
        }
        const float cc[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * j4 + e;
            if (j < a.n) {
                a.v[j] -= log2f(fmaxf(cc[e], 1.17549435e-38f));
                a.u[j] = a.unew[j];
            }
        }
    }
    if (blockIdx.x == 0 && tid == 0) a.ctrl->iters += 1;
}

// eps from eps_dev or eps_rel * absmax; potentials initialised.
__global__ __launch_bounds__(256) void sk_init_kernel(int n, const float* eps_dev, float eps_rel,
                                                      const float* absmax, const float* g_init,
                                                      float tol, float* u, float* v, SkCtrl* ctrl) {
    const float eps = eps_dev ? *eps_dev : eps_rel * (*absmax);
    const float kappa = eps > 0.0f ? kLog2e / eps : 0.0f;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        u[i] = 0.0f;
        v[i] = (g_init && eps > 0.0f) ? g_init[i] * kappa : 0.0f;
    }
    if (i == 0) {
        ctrl->kappa = kappa;
        ctrl->eps = eps;
        ctrl->done = eps > 0.0f ? 0 : 2;
        ctrl->iters = 0;
        ctrl->err = 0.0f;
        ctrl->tol = tol;
    }
}

// Q = 2^(G kappa + u_i + v_j) (or J when eps == 0), its largest row-marginal
// error, optional bf16 hi/lo planes of Q (np stride), and the potentials in
// natural units.
struct FinArgs {
    SkArgs a;
    float* Q; int ldq;
    uint16_t* Qhi; uint16_t* Qlo;
};

template <int T, int C>
__global__ __launch_bounds__(T) void sk_finalize_kernel(FinArgs fa) {
    const SkArgs& a = fa.a;
    __shared__ float red[2][T / 64];
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * a.rpw;
    const int r1 = min(a.n, r0 + a.rpw);
    const float kappa = a.ctrl->kappa;
    const bool flat = a.ctrl->done == 2;
    const float jval = 1.0f / (float)a.n;
    float vj[C][4];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * (tid + T * c) + e;
            vj[c][e] = (j < a.n) ? a.v[j] : -INFINITY;
        }
    float errmax = 0.0f;
    int par = 0;
    for (int i = r0; i < r1; ++i) {
        const float ui = a.u[i];
        const float* grow = a.G + (size_t)i * a.ldg;
        float s = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j0 = 4 * (tid + T * c);
            if (j0 >= a.np && j0 >= a.n) continue;
            float4 g4 = j0 < a.n ? *reinterpret_cast<const float4*>(grow + j0) : make_float4(0.f, 0.f, 0.f, 0.f);
            float gv[4] = {g4.x, g4.y, g4.z, g4.w};
            float q[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = j0 + e;
                q[e] = (j < a.n) ? (flat ? jval : exp2f(fmaf(gv[e], kappa, vj[c][e]) + ui)) : 0.0f;
                s += q[e];
                if (j < a.n && fa.Q) fa.Q[(size_t)i * fa.ldq + j] = q[e];
                if (fa.Qhi && j < a.np) {
                    const uint16_t h = f32_to_bf16_rne(q[e]);
                    fa.Qhi[(size_t)i * a.np + j] = h;
                    fa.Qlo[(size_t)i * a.np + j] = f32_to_bf16_rne(q[e] - bf16_to_f32(h));
                }
            }
        }
        const float S = block_sum<T>(s, red[par]);
        par ^= 1;
        errmax = fmaxf(errmax, fabsf(S - 1.0f));
    }
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
        if (f) f[i] = flat ? 0.0f : a.u[i] / kappa;
        if (g) g[i] = flat ? 0.0f : a.v[i] / kappa;
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
    int T, C, W, rpw, R;
};

// Threads per strip: 256 below n = 4096, else the smallest of 512 / 1024
// that keeps a row's share per thread at <= 40 columns (register budget
// without spills); beyond n = 20480 the 1024-thread variant is used and
// spills. The number of
// strips W defaults to kSkDefaultWG; GOAT_SK_GEOM="T,W" overrides both (a
// tuning knob for measurements).
constexpr int kSkDefaultWG = 512;

Geometry geometry(int n) {
    int env_T = 0, env_W = 0, env_R = 0;
    if (const char* e = getenv("GOAT_SK_GEOM")) {
        int t = 0, w = 0, r = 1;
        const int got = sscanf(e, "%d,%d,%d", &t, &w, &r);
        if (got >= 2 && (t == 256 || t == 512 || t == 1024) && w >= 1 && w <= kSkWG && (r == 1 || r == 2)) {
            env_T = t;
            env_W = w;
            env_R = r;
        }
    }
    Geometry g;
    const int n4 = (n + 3) / 4;
    // 512 threads from n = 4096 on: measured 2% faster than 256 at n = 10000
    g.T = n < 4096 ? 256 : (n4 <= 512 * 10 ? 512 : 1024);
    if (env_T > 0 && n4 <= env_T * 16) g.T = env_T;
    g.C = (n4 + g.T - 1) / g.T;
    const int cs[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16};
    for (int c : cs)
        if (c >= g.C) { g.C = c; break; }
    const int wmax = env_W > 0 ? env_W : kSkDefaultWG;
    g.W = n < wmax ? n : wmax;
    g.rpw = (n + g.W - 1) / g.W;
    g.W = (n + g.rpw - 1) / g.rpw;
    g.R = env_R > 0 ? env_R : 1;
    return g;
}

template <int T, bool FIRST>
int launch_row_T(const Geometry& g, const SkArgs& a, hipStream_t s) {
    dim3 grid(g.W), block(T);
    const size_t lds = (size_t)16 * T * g.C;
    const bool vlds = lds <= 65536;
    switch (g.C) {
#define GOAT_SK_C(CC)                                                                                     \
    case CC:                                                                                              \
        if (g.R == 2 && CC <= 6) {                                                                        \
            if (vlds) hipLaunchKernelGGL((sk_row_kernel<T, CC, 2, FIRST, true>), grid, block, lds, s, a);    \
            else hipLaunchKernelGGL((sk_row_kernel<T, CC, 2, FIRST, false>), grid, block, 0, s, a);          \
        } else {                                                                                          \
            if (vlds) hipLaunchKernelGGL((sk_row_kernel<T, CC, 1, FIRST, true>), grid, block, lds, s, a);    \
            else hipLaunchKernelGGL((sk_row_kernel<T, CC, 1, FIRST, false>), grid, block, 0, s, a);          \
        }                                                                                                 \
        break;
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
#define GOAT_SK_C(CC) case CC: hipLaunchKernelGGL((sk_finalize_kernel<T, CC>), grid, block, 0, s, fa); break;
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
    a.u = st.u;
    a.unew = st.unew;
    a.v = st.v;
    a.colpart = st.colpart;
    a.errpart = st.errpart;
    a.ctrl = st.ctrl;
    return a;
}

// Cooperative launch of the whole solve; GOAT_ENOTSUP when the shape has no
// persistent variant or the strips cannot all be resident at once.
template <int T, int C>
int launch_persistent_TC(const Geometry& g, SkArgs a, int k_begin, int k_end, hipStream_t s) {
    auto kfn = sk_persistent_kernel<T, C>;
    const size_t lds = (size_t)16 * T * C;
    int per_cu = 0, cus = 0, dev = 0;
    GOAT_HIP(hipGetDevice(&dev));
    GOAT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    GOAT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, T, lds));
    if (per_cu < 1 || (long long)per_cu * cus < g.W) return GOAT_ENOTSUP;
    SkPersist pp;
    pp.k_begin = k_begin;
    pp.k_end = k_end;
    pp.W = g.W;
    pp.cpw = (a.n + g.W - 1) / g.W;
    void* args[] = {&a, &pp};
    GOAT_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kfn), dim3(g.W), dim3(T), args, lds, s));
    return GOAT_OK;
}

template <int T>
int launch_persistent_T(const Geometry& g, const SkArgs& a, int k_begin, int k_end, hipStream_t s) {
    switch (g.C) {
        case 1: return launch_persistent_TC<T, 1>(g, a, k_begin, k_end, s);
        case 2: return launch_persistent_TC<T, 2>(g, a, k_begin, k_end, s);
        case 3: return launch_persistent_TC<T, 3>(g, a, k_begin, k_end, s);
        case 4: return launch_persistent_TC<T, 4>(g, a, k_begin, k_end, s);
        case 5: return launch_persistent_TC<T, 5>(g, a, k_begin, k_end, s);
        case 6: return launch_persistent_TC<T, 6>(g, a, k_begin, k_end, s);
        case 8: return launch_persistent_TC<T, 8>(g, a, k_begin, k_end, s);
        case 10: return launch_persistent_TC<T, 10>(g, a, k_begin, k_end, s);
        default: return GOAT_ENOTSUP;
    }
}

}  // namespace

int sk_prepare(int n, const float* G, int ldg, const float* eps_dev, float eps_rel,
               const float* absmax_dev, const float* g_init, float tol, SkState st, float* fscal,
               double* red, hipStream_t s) {
    (void)red;
    const float* absmax = absmax_dev;
    if (!eps_dev && !absmax) {
        int rc = launch_absmax(n, G, ldg, fscal + 16, fscal, s);
        if (rc) return rc;
        absmax = fscal;
    }
    hipLaunchKernelGGL(sk_init_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, eps_dev, eps_rel,
                       absmax, g_init, tol, st.u, st.v, st.ctrl);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int sk_iterate(int n, int np, const float* G, int ldg, SkState st, int first, int check, int iter,
               hipStream_t s) {
    const Geometry g = geometry(n);
    SkArgs a = make_args(n, np, G, ldg, st, g);
    a.rev = iter & 1;
    int rc;
    prof_begin(0, s);
    if (g.T == 256) rc = first ? launch_row_T<256, true>(g, a, s) : launch_row_T<256, false>(g, a, s);
    else if (g.T == 512) rc = first ? launch_row_T<512, true>(g, a, s) : launch_row_T<512, false>(g, a, s);
    else rc = first ? launch_row_T<1024, true>(g, a, s) : launch_row_T<1024, false>(g, a, s);
    prof_end(0, s);
    if (rc) return rc;
    hipLaunchKernelGGL(sk_merge_kernel, dim3((n + 63) / 64), dim3(256), 0, s, a, g.W, check);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int sk_run_persistent(int n, int np, const float* G, int ldg, SkState st, int k_begin, int k_end,
                      hipStream_t s) {
    // Opt-in (GOAT_SK_PERSISTENT=1): measured slower than one launch pair per
    // iteration on MI355X at n = 10000 (the grid barrier costs more than the
    // two launch gaps it removes).
    const char* e = getenv("GOAT_SK_PERSISTENT");
    if (!e || e[0] != '1') return GOAT_ENOTSUP;
    if (k_end <= k_begin) return GOAT_OK;
    const Geometry g = geometry(n);
    if (g.T > 512 || 16 * g.T * g.C > 65536) return GOAT_ENOTSUP;
    const SkArgs a = make_args(n, np, G, ldg, st, g);
    prof_begin(0, s);
    int rc = g.T == 256 ? launch_persistent_T<256>(g, a, k_begin, k_end, s)
                        : launch_persistent_T<512>(g, a, k_begin, k_end, s);
    prof_end(0, s);
    if (rc == GOAT_ENOTSUP) clear_error();
    return rc;
}

int sk_finalize(int n, int np, const float* G, int ldg, SkState st, float* Q, int ldq,
                uint16_t* Q_hi, uint16_t* Q_lo, float* f, float* g, int* iters_out,
                float* err_out, float* eps_out, double* red, hipStream_t s) {
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
