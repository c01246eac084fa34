// Batched GOAT for many small problems (random-start batches of graph pairs,
// GOAT section, random initialisations): one workgroup solves one
// (pair, start) problem from its start to its last Frank-Wolfe iterate
// (Alg. 3 steps 1-4 repeated), so thousands of problems of uneven size run as
// one persistent launch per size bucket, with no host round trip and no
// grid-wide synchronisation. Phases of a workgroup, separated by barriers:
//   start   P0 = J, or (J + K)/2 with K the Sinkhorn-Knopp scaling of the
//           caller's positive draws U
//   grad    G = A P B^T + A^T P B as two NT products on the fp32 matrix
//           cores: T = [B; B^T] P^T, then G = A T_0^T + A^T T_1^T (symmetric
//           pairs: T = B P^T, G = 2 A T^T); 32 x 32 tiles spread over waves
//   LOT     log-domain Sinkhorn (Alg. 2, maximisation kernel) with the
//           potentials in LDS: per iteration one row sweep that also
//           accumulates the row-normalised plan's column sums, then the
//           column update; the same compensated potentials (grid part +
//           remainder, base 2, scaled by 1/eps) as the single-problem solver
//   Q       Q = exp((G + f + g)/eps), its row-marginal error, and the traces
//           <Q,G_P>, <P,G_P>, ||Q-P||^2 in float64
//   step    G_Q = grad f(Q), <Q,G_Q>, the exact step t (Alg. 3 step 3)
//   update  P += t (Q - P), G_P += t (G_Q - G_P) (grad f is linear), max|G_P|
// Every matrix is np x np (np = n rounded up to 32) with zero padding, so
// the products need no edge handling and padded rows/columns stay zero.
#include <cfloat>
#include <cmath>
#include <cstdio>

#include "batch.h"
#include "common.h"

namespace goat {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr float kL2e = 1.4426950408889634f;

// ---------------------------------------------------------------- reductions

template <int M>
__device__ inline float sxor(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, x), 0x1F | (M << 10)));
}
template <int M>
__device__ inline double sxor(double x) {
    const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_ds_swizzle((int)(unsigned)(v & 0xffffffffull), 0x1F | (M << 10));
    const int hi = __builtin_amdgcn_ds_swizzle((int)(unsigned)(v >> 32), 0x1F | (M << 10));
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

struct OpAdd {
    template <typename V> __device__ V operator()(V a, V b) const { return a + b; }
};
struct OpMax {
    __device__ float operator()(float a, float b) const { return fmaxf(a, b); }
};

// Butterfly over the L-lane group holding this lane (L = 16, 32, 64); every
// lane of the group ends with the same value (the operations commute).
template <int L, typename V, typename Op>
__device__ inline V group_reduce(V x, Op op) {
    x = op(x, sxor<1>(x));
    x = op(x, sxor<2>(x));
    x = op(x, sxor<4>(x));
    x = op(x, sxor<8>(x));
    if (L >= 32) x = op(x, sxor<16>(x));
    if (L >= 64) x = op(x, __shfl_xor(x, 32));
    return x;
}

template <int WAVES>
__device__ inline float wg_max(float x, float* red) {
    x = group_reduce<64>(x, OpMax());
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    float m = red[0];
#pragma unroll
    for (int w = 1; w < WAVES; ++w) m = fmaxf(m, red[w]);
    return m;
}

// three float64 sums at once, fixed order
template <int WAVES>
__device__ inline void wg_sum3(double& a, double& b, double& c, double* red) {
    a = group_reduce<64>(a, OpAdd());
    b = group_reduce<64>(b, OpAdd());
    c = group_reduce<64>(c, OpAdd());
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        const int w = threadIdx.x >> 6;
        red[3 * w] = a;
        red[3 * w + 1] = b;
        red[3 * w + 2] = c;
    }
    __syncthreads();
    a = red[0]; b = red[1]; c = red[2];
#pragma unroll
    for (int w = 1; w < WAVES; ++w) {
        a += red[3 * w];
        b += red[3 * w + 1];
        c += red[3 * w + 2];
    }
}

__device__ inline void renorm(float& g, float& r, float h, float inv_h) {
    const float t = rintf(r * inv_h) * h;
    g += t;
    r -= t;
}

// ---------------------------------------------------------------- products

// C = alpha (X0 Z0^T + X1 Z1^T) over an M x N block with inner size K (all
// multiples of 32, row stride ld). A wave owns a 32 x 32 tile at a time
// (v_mfma_f32_32x32x2f32). Lane l reads 4 consecutive k of row l % 32 for
// both operands; lane halves take k and k + 4, so each instruction pairs
// (k0 + e, k0 + 4 + e) - a permutation of k applied to both operands alike.
template <int WAVES>
__device__ void wg_gemm_nt(const float* X0, const float* Z0, const float* X1, const float* Z1, int M, int N,
                           int K, int ld, float alpha, float* C) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 31, kh = lane >> 5;
    const int tn = N >> 5, tiles = (M >> 5) * tn;
    const int nseg = X1 ? 2 : 1;
    for (int t = wave; t < tiles; t += WAVES) {
        const int i0 = (t / tn) << 5, j0 = (t % tn) << 5;
        f32x16 acc;
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[e] = 0.0f;
        for (int s = 0; s < nseg; ++s) {
            const float* xr = (s ? X1 : X0) + (size_t)(i0 + r) * ld + 4 * kh;
            const float* zr = (s ? Z1 : Z0) + (size_t)(j0 + r) * ld + 4 * kh;
            for (int k0 = 0; k0 < K; k0 += 32) {
                float4 xa[4], za[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    xa[u] = *reinterpret_cast<const float4*>(xr + k0 + 8 * u);
                    za[u] = *reinterpret_cast<const float4*>(zr + k0 + 8 * u);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(xa[u].x, za[u].x, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(xa[u].y, za[u].y, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(xa[u].z, za[u].z, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(xa[u].w, za[u].w, acc, 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = i0 + 8 * (e >> 2) + 4 * kh + (e & 3);
            C[(size_t)i * ld + j0 + r] = alpha * acc[e];
        }
    }
}

// grad f(M) into Gout (np x np) via T
template <int WAVES>
__device__ void wg_grad(const BProb& pr, const float* Mat, float* Gout) {
    const int np = pr.np;
    const bool gen = pr.A1 != nullptr;
    wg_gemm_nt<WAVES>(pr.X1, Mat, nullptr, nullptr, gen ? 2 * np : np, np, np, np, 1.0f, pr.T);
    __syncthreads();
    if (gen)
        wg_gemm_nt<WAVES>(pr.A0, pr.T, pr.A1, pr.T + (size_t)np * np, np, np, np, np, 1.0f, Gout);
    else
        wg_gemm_nt<WAVES>(pr.A0, pr.T, nullptr, nullptr, np, np, np, np, 2.0f, Gout);
    __syncthreads();
}

// ---------------------------------------------------------------- start

// Sinkhorn-Knopp scaling K = diag(r) U diag(c) of a positive n x n matrix
// (r = 1/(U c), c = 1/(U^T r) from c = 1; row sums checked from the second
// sweep), sums in float64; then P = (J + K)/2 over prow x pcol (zero outside
// n x n). r, c, rn: LDS vectors of >= n floats.
template <int NT, int L>
__device__ void sk_start(int n, const float* U, int ldu, float* P, int ldp, int prow, int pcol, float tol,
                         int max_iter, float* r, float* c, float* rn, float* red, int* iters_out,
                         float* err_out) {
    constexpr int WAVES = NT / 64, NG = NT / L;
    const int tid = threadIdx.x, grp = tid / L, q = tid % L;
    for (int j = tid; j < n; j += NT) c[j] = 1.0f;
    __syncthreads();
    float err = INFINITY;
    int it = 0;
    for (;; ++it) {
        float emax = 0.0f;
        for (int i = grp; i < n; i += NG) {
            double s = 0.0;
            const float* ur = U + (size_t)i * ldu;
            for (int j = q; j < n; j += L) s += (double)ur[j] * (double)c[j];
            s = group_reduce<L>(s, OpAdd());
            if (it > 0) emax = fmaxf(emax, (float)fabs((double)r[i] * s - 1.0));
            if (q == 0) rn[i] = (float)(1.0 / s);
        }
        if (it > 0) {
            err = wg_max<WAVES>(emax, red);
            if (err <= tol || it >= max_iter) break;
        } else {
            __syncthreads();
        }
        for (int i = tid; i < n; i += NT) r[i] = rn[i];
        __syncthreads();
        for (int j = tid; j < n; j += NT) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += (double)r[i] * (double)U[(size_t)i * ldu + j];
            c[j] = (float)(1.0 / s);
        }
        __syncthreads();
    }
    const float jn = 1.0f / (float)n;
    for (int i = 0; i < prow; ++i) {
        const float ri = i < n ? r[i] : 0.0f;
        for (int j = tid; j < pcol; j += NT)
            P[(size_t)i * ldp + j] = (i < n && j < n) ? 0.5f * (jn + ri * U[(size_t)i * ldu + j] * c[j]) : 0.0f;
    }
    if (tid == 0) {
        if (iters_out) *iters_out = it;
        if (err_out) *err_out = err;
    }
    __syncthreads();
}

// ---------------------------------------------------------------- the solver

template <int L, int CMAX, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void batch_goat_kernel(BArgs a, int npb) {
    constexpr int NT = WAVES * 64, NG = NT / L;
    const int slot = a.order[blockIdx.x];
    if (slot < 0) return;
    const BProb pr = a.probs[slot];
    const int n = pr.n, np = pr.np;
    extern __shared__ float lds[];
    float* ug = lds;
    float* us = ug + npb;
    float* vg = us + npb;
    float* vs = vg + npb;
    float* ung = vs + npb;
    float* uns = ung + npb;
    float* colacc = uns + npb;   // [NG][npb]
    __shared__ float fred[WAVES];
    __shared__ double dred[3 * WAVES];
    const int tid = threadIdx.x;
    const int grp = tid / L, q = tid % L;
    const int cn = (np + 4 * L - 1) / (4 * L);

    // ---- start
    if (pr.U) {
        sk_start<NT, L>(n, pr.U, pr.ldu, pr.P, np, np, np, a.init_tol, a.init_max, ug, vg, ung, fred, nullptr,
                        nullptr);
    } else {
        const float jn = 1.0f / (float)n;
        for (int idx = tid; idx < np * np; idx += NT) {
            const int i = idx / np, j = idx - i * np;
            pr.P[idx] = (i < n && j < n) ? jn : 0.0f;
        }
        __syncthreads();
    }
    wg_grad<WAVES>(pr, pr.P, pr.GP);
    float gmax = 0.0f;
    {
        float m = 0.0f;
        const float4* g4 = reinterpret_cast<const float4*>(pr.GP);
        for (int k = tid; k < n * np / 4; k += NT) {
            const float4 v = g4[k];
            m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
        gmax = wg_max<WAVES>(m, fred);
    }

    float kap_prev = 0.0f;
    int fw = 0;
    bool stop_fw = false;
    while (fw < a.fw_max && !stop_fw) {
        const float eps = a.eps_rel * gmax;
        const bool flat = !(eps > 0.0f && gmax > 0.0f);
        float kap = 0.0f;
        int sk_it = 0;
        if (!flat) {
            kap = kL2e / eps;
            int e2 = 0;
            frexpf(gmax * kap + 64.0f, &e2);
            const float h = ldexpf(1.0f, e2 - 24), inv_h = 1.0f / h;
            const bool warm = a.warm && kap_prev > 0.0f;
            for (int j = tid; j < npb; j += NT) {
                float g = 0.0f, r = 0.0f;
                if (j < n && warm) {
                    r = (vg[j] + vs[j]) / kap_prev * kap;
                    renorm(g, r, h, inv_h);
                }
                vg[j] = j < n ? g : -INFINITY;
                vs[j] = j < n ? r : 0.0f;
                ug[j] = 0.0f;
                us[j] = 0.0f;
            }
            __syncthreads();
            for (int k = 0; k < a.sk_max; ++k) {
                const bool first = k == 0;
                float4 vgr[CMAX], vsr[CMAX];
                float acc[CMAX][4];
                bool ok[CMAX];
#pragma unroll
                for (int c = 0; c < CMAX; ++c) {
                    const int col = 4 * (q + L * c);
                    ok[c] = c < cn && col < np;
                    vgr[c] = ok[c] ? *reinterpret_cast<const float4*>(vg + col)
                                   : make_float4(-INFINITY, -INFINITY, -INFINITY, -INFINITY);
                    vsr[c] = ok[c] ? *reinterpret_cast<const float4*>(vs + col) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[c][e] = 0.0f;
                }
                float emax = 0.0f;
                for (int i = grp; i < n; i += NG) {
                    const float4* row = reinterpret_cast<const float4*>(pr.GP + (size_t)i * np);
                    float4 x[CMAX];
#pragma unroll
                    for (int c = 0; c < CMAX; ++c)
                        x[c] = ok[c] ? row[q + L * c] : make_float4(0.f, 0.f, 0.f, 0.f);
                    const float ugi = first ? 0.0f : ug[i];
                    float y[CMAX][4];
#pragma unroll
                    for (int c = 0; c < CMAX; ++c) {
                        y[c][0] = fmaf(x[c].x, kap, vgr[c].x + ugi) + vsr[c].x;
                        y[c][1] = fmaf(x[c].y, kap, vgr[c].y + ugi) + vsr[c].y;
                        y[c][2] = fmaf(x[c].z, kap, vgr[c].z + ugi) + vsr[c].z;
                        y[c][3] = fmaf(x[c].w, kap, vgr[c].w + ugi) + vsr[c].w;
                    }
                    float shift = 0.0f;
                    if (first) {
                        float m = -INFINITY;
#pragma unroll
                        for (int c = 0; c < CMAX; ++c)
#pragma unroll
                            for (int e = 0; e < 4; ++e) m = fmaxf(m, y[c][e]);
                        shift = -group_reduce<L>(m, OpMax());
                    }
                    float s = 0.0f;
#pragma unroll
                    for (int c = 0; c < CMAX; ++c)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            y[c][e] = __builtin_amdgcn_exp2f(y[c][e] + shift);
                            s += y[c][e];
                        }
                    const float S = group_reduce<L>(s, OpAdd());
                    const float inv = 1.0f / S;
#pragma unroll
                    for (int c = 0; c < CMAX; ++c)
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc[c][e] = fmaf(y[c][e], inv, acc[c][e]);
                    // the row remainder u_rem is left out of y; it enters the
                    // stop test as the factor 2^u_rem
                    if (!first) emax = fmaxf(emax, fabsf(S * exp2f(us[i]) - 1.0f));
                    if (q == 0) {
                        float g_ = first ? rintf(shift * inv_h) * h : ugi;
                        float r_ = first ? (shift - g_) - log2f(S) : -log2f(S);
                        renorm(g_, r_, h, inv_h);
                        ung[i] = g_;
                        uns[i] = r_;
                    }
                }
                float* my = colacc + (size_t)grp * npb;
#pragma unroll
                for (int c = 0; c < CMAX; ++c)
                    if (ok[c])
                        *reinterpret_cast<float4*>(my + 4 * (q + L * c)) =
                            make_float4(acc[c][0], acc[c][1], acc[c][2], acc[c][3]);
                bool done = false;
                if (!first) {
                    const float err = wg_max<WAVES>(emax, fred);
                    done = err <= a.sk_tol;
                } else {
                    __syncthreads();
                }
                if (done) break;
                for (int j = tid; j < n; j += NT) {
                    float cs = 0.0f;
                    for (int g2 = 0; g2 < NG; ++g2) cs += colacc[(size_t)g2 * npb + j];
                    float g = vg[j], r = vs[j] - log2f(fmaxf(cs, FLT_MIN));
                    renorm(g, r, h, inv_h);
                    vg[j] = g;
                    vs[j] = r;
                }
                for (int i = tid; i < n; i += NT) {
                    ug[i] = ung[i];
                    us[i] = uns[i];
                }
                __syncthreads();
                ++sk_it;
            }
        }

        // ---- Q, its row-marginal error, traces <Q,G_P>, <P,G_P>, ||Q-P||^2
        double tc = 0.0, tp = 0.0, td = 0.0;
        float qerr = 0.0f;
        {
            const float jn = 1.0f / (float)n;
            for (int i = grp; i < n; i += NG) {
                const float4* grow = reinterpret_cast<const float4*>(pr.GP + (size_t)i * np);
                const float4* prow = reinterpret_cast<const float4*>(pr.P + (size_t)i * np);
                float4* qrow = reinterpret_cast<float4*>(pr.Q + (size_t)i * np);
                const float ugi = ug[i], usi = us[i];
                float s = 0.0f;
#pragma unroll
                for (int c = 0; c < CMAX; ++c) {
                    const int c4 = q + L * c;
                    if (!(c < cn && 4 * c4 < np)) continue;
                    const float4 x = grow[c4], p = prow[c4];
                    const float xv[4] = {x.x, x.y, x.z, x.w}, pv[4] = {p.x, p.y, p.z, p.w};
                    float qv[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int j = 4 * c4 + e;
                        if (flat) qv[e] = j < n ? jn : 0.0f;
                        else qv[e] = exp2f(fmaf(xv[e], kap, vg[j] + ugi) + (vs[j] + usi));
                        s += qv[e];
                        tc += (double)qv[e] * xv[e];
                        tp += (double)pv[e] * xv[e];
                        const double d = (double)qv[e] - pv[e];
                        td += d * d;
                    }
                    qrow[c4] = make_float4(qv[0], qv[1], qv[2], qv[3]);
                }
                const float S = group_reduce<L>(s, OpAdd());
                qerr = fmaxf(qerr, fabsf(S - 1.0f));
            }
            __syncthreads();
            qerr = wg_max<WAVES>(qerr, fred);
            wg_sum3<WAVES>(tc, tp, td, dred);
        }

        // ---- G_Q and the exact step
        wg_grad<WAVES>(pr, pr.Q, pr.GQ);
        double fq = 0.0, z1 = 0.0, z2 = 0.0;
        {
            const float4* q4 = reinterpret_cast<const float4*>(pr.Q);
            const float4* g4 = reinterpret_cast<const float4*>(pr.GQ);
            for (int k = tid; k < n * np / 4; k += NT) {
                const float4 x = q4[k], y = g4[k];
                fq += (double)x.x * y.x + (double)x.y * y.y + (double)x.z * y.z + (double)x.w * y.w;
            }
            wg_sum3<WAVES>(fq, z1, z2, dred);
        }
        const double fP = 0.5 * tp, fQ = 0.5 * fq, cc = tc;
        const double qa = fP + fQ - cc, qb = cc - 2.0 * fP;
        double t;
        if (qa < 0.0) {
            t = -qb / (2.0 * qa);
            t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        } else {
            t = (qa + qb > 0.0) ? 1.0 : 0.0;
        }
        if (tid == 0) {
            goat_iter_record rec;
            rec.fP = fP; rec.fQ = fQ; rec.c = cc; rec.a = qa; rec.b = qb; rec.t = t; rec.dist2 = td;
            rec.eps = eps; rec.sk_err = qerr; rec.sk_iters = sk_it; rec.pad = 0;
            pr.hist[fw] = rec;
        }
        ++fw;
        kap_prev = flat ? 0.0f : kap;
        if (t == 0.0 && a.stop_on_stall) break;

        // ---- update
        const float tf = (float)t;
        float m = 0.0f;
        {
            float4* p4 = reinterpret_cast<float4*>(pr.P);
            float4* gp4 = reinterpret_cast<float4*>(pr.GP);
            const float4* q4 = reinterpret_cast<const float4*>(pr.Q);
            const float4* gq4 = reinterpret_cast<const float4*>(pr.GQ);
            for (int k = tid; k < n * np / 4; k += NT) {
                float4 p = p4[k], gp = gp4[k];
                const float4 x = q4[k], y = gq4[k];
                p.x = fmaf(tf, x.x - p.x, p.x); p.y = fmaf(tf, x.y - p.y, p.y);
                p.z = fmaf(tf, x.z - p.z, p.z); p.w = fmaf(tf, x.w - p.w, p.w);
                gp.x = fmaf(tf, y.x - gp.x, gp.x); gp.y = fmaf(tf, y.y - gp.y, gp.y);
                gp.z = fmaf(tf, y.z - gp.z, gp.z); gp.w = fmaf(tf, y.w - gp.w, gp.w);
                p4[k] = p;
                gp4[k] = gp;
                m = fmaxf(m, fmaxf(fmaxf(fabsf(gp.x), fabsf(gp.y)), fmaxf(fabsf(gp.z), fabsf(gp.w))));
            }
        }
        gmax = wg_max<WAVES>(m, fred);
        const double delta = t * sqrt(td) / sqrt((double)n);
        if (a.fw_tol > 0.0f && delta < (double)a.fw_tol) stop_fw = true;
    }
    if (tid == 0) *pr.fw_done = fw;
}

// ---------------------------------------------------------------- helpers

__global__ __launch_bounds__(256) void batch_pack_kernel(const BPack* jobs, int njobs) {
    const BPack jb = jobs[blockIdx.x];
    const int n = jb.n, np = jb.np, ld = jb.ld;
    for (int r = blockIdx.y; r < np; r += gridDim.y) {
        for (int j = threadIdx.x; j < np; j += blockDim.x) {
            const bool in = r < n && j < n;
            jb.A0[(size_t)r * np + j] = in ? jb.A[(size_t)r * ld + j] : 0.0f;
            jb.X1[(size_t)r * np + j] = in ? jb.B[(size_t)r * ld + j] : 0.0f;
            if (jb.general) {
                jb.A1[(size_t)r * np + j] = in ? jb.A[(size_t)j * ld + r] : 0.0f;
                jb.X1[(size_t)(np + r) * np + j] = in ? jb.B[(size_t)j * ld + r] : 0.0f;
            }
        }
    }
}

// tr(A^T Pi B Pi^T) = sum_ij A_ij B_{p_i p_j} per problem, float64
__global__ __launch_bounds__(256) void batch_score_kernel(const BProb* probs, const int32_t* perms,
                                                          const int* off, double* out) {
    const BProb pr = probs[blockIdx.x];
    const int n = pr.n, np = pr.np;
    const int32_t* p = perms + off[blockIdx.x];
    __shared__ double red[4 * 3];
    double s = 0.0;
    for (int idx = threadIdx.x; idx < n * n; idx += 256) {
        const int i = idx / n, j = idx - i * n;
        const float av = pr.A0[(size_t)i * np + j];
        // indices clamped into range; meaningful only for a permutation
        const int pi = min(max(p[i], 0), n - 1), pj = min(max(p[j], 0), n - 1);
        if (av != 0.0f) s += (double)av * pr.X1[(size_t)pi * np + pj];
    }
    double z1 = 0.0, z2 = 0.0;
    wg_sum3<4>(s, z1, z2, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void batch_zero_kernel(float* p, size_t count) {
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x)
        p[k] = 0.0f;
}

// synthetic symmetric 0/1 pair (edge density about 1/8) for autotuning
__device__ inline uint32_t mix32(uint32_t x) {
    x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
    return x;
}
__global__ void batch_synth_kernel(float* A, float* B, int n, int ld, uint32_t seed) {
    const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || j >= n) return;
    const int lo = min(i, j), hi = max(i, j);
    const uint32_t h = mix32(seed ^ mix32((uint32_t)lo * 40503u + (uint32_t)hi));
    A[(size_t)i * ld + j] = (i != j && (h & 7u) == 0u) ? 1.0f : 0.0f;
    B[(size_t)i * ld + j] = (i != j && ((h >> 8) & 7u) == 0u) ? 1.0f : 0.0f;
}

__global__ __launch_bounds__(256) void random_init_kernel(int n, const float* U, int ldu, float* P, int ldp,
                                                          float tol, int max_iter, int* iters, float* err) {
    extern __shared__ float lds[];
    __shared__ float red[4];
    sk_start<256, 16>(n, U, ldu, P, ldp, n, n, tol, max_iter, lds, lds + n, lds + 2 * n, red, iters, err);
}

template <int L, int CMAX, int WAVES>
int launch_shape(int npb, int nblocks, const BArgs& a, hipStream_t st, size_t lds) {
    hipLaunchKernelGGL((batch_goat_kernel<L, CMAX, WAVES>), dim3(nblocks), dim3(WAVES * 64), lds, st, a, npb);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

}  // namespace

size_t batch_lds_bytes(const BShape& s, int npb) {
    const int ng = s.waves * 64 / s.L;
    return (size_t)(6 + ng) * npb * sizeof(float);
}

bool batch_shape_ok(const BShape& s, int npb) {
    if (!(s.L == 16 || s.L == 32 || s.L == 64) || !(s.waves == 4 || s.waves == 8)) return false;
    if (!(s.cmax == 1 || s.cmax == 2 || s.cmax == 4)) return false;
    return 4 * s.L * s.cmax >= npb && batch_lds_bytes(s, npb) <= 65536;
}

int batch_launch(const BShape& s, int npb, int nblocks, const BArgs& a, hipStream_t st) {
    if (!batch_shape_ok(s, npb)) {
        set_error("batch: unsupported kernel shape");
        return GOAT_ENOTSUP;
    }
    if (nblocks == 0) return GOAT_OK;
    const size_t lds = batch_lds_bytes(s, npb);
#define GOAT_B_SHAPE(LL, CC, WW) \
    if (s.L == LL && s.cmax == CC && s.waves == WW) return launch_shape<LL, CC, WW>(npb, nblocks, a, st, lds);
    GOAT_B_SHAPE(16, 1, 4) GOAT_B_SHAPE(16, 2, 4) GOAT_B_SHAPE(16, 4, 4)
    GOAT_B_SHAPE(32, 1, 4) GOAT_B_SHAPE(32, 2, 4) GOAT_B_SHAPE(32, 4, 4)
    GOAT_B_SHAPE(64, 1, 4) GOAT_B_SHAPE(64, 2, 4) GOAT_B_SHAPE(64, 4, 4)
    GOAT_B_SHAPE(16, 1, 8) GOAT_B_SHAPE(16, 2, 8) GOAT_B_SHAPE(16, 4, 8)
    GOAT_B_SHAPE(32, 1, 8) GOAT_B_SHAPE(32, 2, 8) GOAT_B_SHAPE(32, 4, 8)
    GOAT_B_SHAPE(64, 1, 8) GOAT_B_SHAPE(64, 2, 8) GOAT_B_SHAPE(64, 4, 8)
#undef GOAT_B_SHAPE
    set_error("batch: unsupported kernel shape");
    return GOAT_ENOTSUP;
}

int batch_pack_launch(const BPack* jobs_dev, int njobs, int np_max, hipStream_t st) {
    if (njobs == 0) return GOAT_OK;
    hipLaunchKernelGGL(batch_pack_kernel, dim3(njobs, np_max < 64 ? np_max : 64), dim3(256), 0, st, jobs_dev,
                       njobs);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int batch_score_launch(const BProb* probs_dev, int nprob, const int32_t* perms_dev, const int* perm_off_dev,
                       double* out_dev, hipStream_t st) {
    if (nprob == 0) return GOAT_OK;
    hipLaunchKernelGGL(batch_score_kernel, dim3(nprob), dim3(256), 0, st, probs_dev, perms_dev, perm_off_dev,
                       out_dev);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int batch_fill_zero(float* p, size_t count, hipStream_t st) {
    if (count == 0) return GOAT_OK;
    size_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(batch_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, count);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int batch_synth_launch(float* A, float* B, int n, int ld, uint32_t seed, hipStream_t st) {
    hipLaunchKernelGGL(batch_synth_kernel, dim3((n + 255) / 256, n), dim3(256), 0, st, A, B, n, ld, seed);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int random_init_launch(int n, const float* U, int ldu, float* P, int ldp, float tol, int max_iter,
                       int* iters_dev, float* err_dev, hipStream_t st) {
    hipLaunchKernelGGL(random_init_kernel, dim3(1), dim3(256), (size_t)3 * n * sizeof(float), st, n, U, ldu, P,
                       ldp, tol, max_iter, iters_dev, err_dev);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

}  // namespace goat
