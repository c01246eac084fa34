// Soft matching on the device: for each row i of a score matrix (the final
// doubly stochastic iterate P, or a direction Q), the k columns with the
// largest scores, best first (vertex nomination, named in the Discussion as
// the use of the relaxed solution beyond a single assignment).
//
// One 256-thread workgroup per row. Each thread scans the columns
// j = t, t + 256, ... (four at a time with 16-byte loads when the row is
// aligned) and keeps its own top-K in registers, inserted by a fixed chain
// of compare-and-swap, so every index is static and nothing spills. The
// block then takes k rounds of a (score desc, column asc) arg-max over the
// 256 list heads; the winning thread shifts its list by one. A row is read
// once: HBM traffic is rows * cols * 4 bytes plus the output.
#include "batch.h"
#include "common.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <vector>

namespace goat {
namespace {

constexpr int NT = 256;

// a ranks before b: larger score, or equal score and smaller column
__device__ inline bool nom_better(float va, int ca, float vb, int cb) {
    return va > vb || (va == vb && ca < cb);
}

template <int K>
__device__ inline void nom_insert(float (&v)[K], int (&c)[K], float x, int j) {
    if (!nom_better(x, j, v[K - 1], c[K - 1])) return;
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const bool sw = nom_better(x, j, v[s], c[s]);
        const float tv = v[s];
        const int tc = c[s];
        v[s] = sw ? x : tv;
        c[s] = sw ? j : tc;
        x = sw ? tv : x;
        j = sw ? tc : j;
    }
}

template <int K>
__global__ __launch_bounds__(NT) void nominate_kernel(int cols, const float* __restrict__ P, long ldp, int k,
                                                      int vec4, int32_t* __restrict__ idx,
                                                      float* __restrict__ val) {
    __shared__ float wv[NT / 64];
    __shared__ int wc[NT / 64];
    const int t = threadIdx.x;
    const long row = blockIdx.x;
    const float* r = P + row * ldp;
    float v[K];
    int c[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
        v[s] = -INFINITY;
        c[s] = INT_MAX;
    }
    int j0 = 0;
    if (vec4) {
        const int c4 = cols >> 2;
        const float4* r4 = reinterpret_cast<const float4*>(r);
        for (int q = t; q < c4; q += NT) {
            const float4 x = r4[q];
            nom_insert<K>(v, c, x.x, 4 * q);
            nom_insert<K>(v, c, x.y, 4 * q + 1);
            nom_insert<K>(v, c, x.z, 4 * q + 2);
            nom_insert<K>(v, c, x.w, 4 * q + 3);
        }
        j0 = c4 << 2;
    }
    for (int j = j0 + t; j < cols; j += NT) nom_insert<K>(v, c, r[j], j);

    const int lane = t & 63, w = t >> 6;
    for (int round = 0; round < k; ++round) {
        float bv = v[0];
        int bc = c[0];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const float ov = __shfl_xor(bv, o, 64);
            const int oc = __shfl_xor(bc, o, 64);
            if (nom_better(ov, oc, bv, bc)) {
                bv = ov;
                bc = oc;
            }
        }
        if (lane == 0) {
            wv[w] = bv;
            wc[w] = bc;
        }
        __syncthreads();
        bv = wv[0];
        bc = wc[0];
#pragma unroll
        for (int u = 1; u < NT / 64; ++u)
            if (nom_better(wv[u], wc[u], bv, bc)) {
                bv = wv[u];
                bc = wc[u];
            }
        __syncthreads();
        // columns are distinct across threads, so exactly one head matches
        if (c[0] == bc) {
#pragma unroll
            for (int s = 0; s + 1 < K; ++s) {
                v[s] = v[s + 1];
                c[s] = c[s + 1];
            }
            v[K - 1] = -INFINITY;
            c[K - 1] = INT_MAX;
        }
        if (t == 0) {
            // fewer than k comparable scores (NaN rows) leave -1
            idx[row * k + round] = bc == INT_MAX ? -1 : bc;
            if (val) val[row * k + round] = bv;
        }
    }
}

template <int K>
void launch_nom_K(int rows, int cols, const float* P, int ldp, int k, int vec4, int32_t* idx, float* val,
                  hipStream_t s) {
    hipLaunchKernelGGL(nominate_kernel<K>, dim3(rows), dim3(NT), 0, s, cols, P, (long)ldp, k, vec4, idx, val);
}

}  // namespace

int launch_nominate(int rows, int cols, const float* P, int ldp, int k, int32_t* idx, float* val,
                    hipStream_t s) {
    if (rows < 1) return GOAT_OK;
    const int vec4 = (ldp % 4) == 0 && (reinterpret_cast<uintptr_t>(P) % 16) == 0;
    if (k <= 4)
        launch_nom_K<4>(rows, cols, P, ldp, k, vec4, idx, val, s);
    else if (k <= 8)
        launch_nom_K<8>(rows, cols, P, ldp, k, vec4, idx, val, s);
    else if (k <= 16)
        launch_nom_K<16>(rows, cols, P, ldp, k, vec4, idx, val, s);
    else
        launch_nom_K<32>(rows, cols, P, ldp, k, vec4, idx, val, s);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

// ---------------------------------------------------------------- device assignment
//
// Final projection of Alg. 3 on the device: a permutation maximising
// sum_i M[i, perm i], solved by Bertsekas' auction with epsilon scaling:
// parallel (Jacobi) rounds in which every unassigned row bids, and
// sequential (Gauss-Seidel) bids in one workgroup when rounds assign few
// rows.
//
// Scores are first mapped to integers: with 2^(e-1) <= max|M| < 2^e and
// s = R - 1 - e, q_ij = rint(M_ij 2^s) (round half to even; the scaling by
// 2^s is exact, and so is the conversion: a float of magnitude >= 2^24 is an
// integer) and c_ij = q_ij - min q, so 0 <= c_ij <= 2^R. Prices and bids are
// int64 in units of 1 / (n + 1) of c: a final phase with epsilon = 1 unit
// leaves the assignment within n / (n + 1) < 1 of the optimum of c, hence
// optimal for c. R = min(40, 55 - ceil(log2(n + 1))) keeps every scaled cost
// below 2^55; a phase raises no price by more than the cost range plus
// epsilon, so over the ~33 phases (epsilon divided by 3 each time) prices
// stay below the 2^62 guard (a bid past it is reported, not wrapped).
//
// A parallel round: each bidding row records (bid, object) and takes the
// object's atomicMax; a claim pass lets the lowest row among those whose bid
// equals the maximum take the object (atomicMin); the resolve pass hands
// each claimed object over. Everything is integer once c is formed, so the
// result does not depend on the order in which threads run.

namespace {

constexpr int AB = 256;             // threads per block
constexpr long long kBidLimit = 1ll << 62;
constexpr int kNoRow = 0x7fffffff;
constexpr int kSeqThreads = 1024;   // threads of the sequential kernel
constexpr int kPerWave = 4;          // candidates each wave of that kernel contributes
constexpr int kCand = kPerWave * (kSeqThreads / 64);   // candidate slots per row (64: one per lane of a wave)
static_assert(kCand == 64, "wave 0 holds one candidate per lane");

struct AuctionArgs {
    const float* M;
    long ld;
    int n, s, vec4, pad;
    long long qmin;              // min_ij rint(M_ij 2^s)
    long long np1;               // n + 1
    long long* price;            // per object
    long long* best;             // per object: highest bid of the round (0: none)
    int32_t* win;                // per object: lowest row with that bid
    long long* mybid;            // per row: its bid of the round
    int32_t* tgt;                // per row: the object it bid for, or -1
    int32_t* owner;              // row holding object j, or -1
    int32_t* assign;             // object held by row i, or -1
    int* ctl;                    // [0] rows assigned, [1] bid overflow, [2] parallel rounds,
                                 // [3] sequential bids
    const long long* cp;         // precomputed scaled scores (row stride ldc), or null
    long ldc;
    int32_t* cj;                 // per row: candidate columns (kCand slots; -1: empty)
    long long* cc;               // per row: their scaled scores
    long long* thr;              // per row: bound on every other column's value (LLONG_MAX: no list)
};

__device__ inline long long auc_cost(const AuctionArgs& a, float m) {
    const long long q = (long long)rintf(ldexpf(m, a.s));
    return (q - a.qmin) * a.np1;
}

__device__ inline long long auc_value(const AuctionArgs& a, float m, int j) {
    return auc_cost(a, m) - a.price[j];
}

// (v, j) ranks before (w, k): larger value, or equal and smaller column
__device__ inline bool auc_better(long long v, int j, long long w, int k) {
    return v > w || (v == w && j < k);
}

// Columns reach a thread in increasing order, so a value equal to the
// current best never displaces it; selects, no branches.
__device__ inline void auc_push(long long& v1, int& j1, long long& v2, long long v, int j) {
    const bool top = v > v1;
    const long long lo = top ? v1 : v;
    v2 = lo > v2 ? lo : v2;
    v1 = top ? v : v1;
    j1 = top ? j : j1;
}

__device__ inline void auc_merge(long long& v1, int& j1, long long& v2, long long ov1, int oj1, long long ov2) {
    // top two of the union of two disjoint sets, without branches
    const bool b = auc_better(ov1, oj1, v1, j1);
    const long long lo = b ? v1 : ov1;     // the head that lost
    const long long w2 = b ? ov2 : v2;     // the winner's second
    v2 = lo > w2 ? lo : w2;
    v1 = b ? ov1 : v1;
    j1 = b ? oj1 : j1;
}

// Cross-lane moves on the data-parallel primitives (DPP) of the VALU, which
// take a few cycles where a general lane shuffle goes through the LDS unit.
// CTRL: 0xB1 lane ^ 1, 0x4E lane ^ 2 (quad permutations), 0x141 mirror
// within each 8 lanes, 0x140 mirror within each 16 lanes (a row).
template <int CTRL>
__device__ inline int dpp_i(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ inline long long dpp_ll(long long x) {
    const int lo = dpp_i<CTRL>((int)(unsigned long long)x);
    const int hi = dpp_i<CTRL>((int)((unsigned long long)x >> 32));
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ inline long long readlane_ll(long long x, int l) {
    const int lo = __builtin_amdgcn_readlane((int)(unsigned long long)x, l);
    const int hi = __builtin_amdgcn_readlane((int)((unsigned long long)x >> 32), l);
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <int CTRL>
__device__ inline void auc_merge_dpp(long long& v1, int& j1, long long& v2) {
    const long long ov1 = dpp_ll<CTRL>(v1), ov2 = dpp_ll<CTRL>(v2);
    const int oj1 = dpp_i<CTRL>(j1);
    auc_merge(v1, j1, v2, ov1, oj1, ov2);
}

// Top two over each row of 16 lanes (every lane of the row ends with its
// row's result): each step merges the set a lane holds with a disjoint set
// of the same size. The whole wave must be active.
__device__ inline void auc_row_merge(long long& v1, int& j1, long long& v2) {
    auc_merge_dpp<0xB1>(v1, j1, v2);
    auc_merge_dpp<0x4E>(v1, j1, v2);
    auc_merge_dpp<0x141>(v1, j1, v2);
    auc_merge_dpp<0x140>(v1, j1, v2);
}

// Top two over the wave: rows merged, then the four row results read into
// scalar registers and merged there. The result is uniform.
__device__ inline void auc_wave_merge(long long& v1, int& j1, long long& v2) {
    auc_row_merge(v1, j1, v2);
    long long r1 = readlane_ll(v1, 0), r2 = readlane_ll(v2, 0);
    int rj = __builtin_amdgcn_readlane(j1, 0);
#pragma unroll
    for (int r = 1; r < 4; ++r)
        auc_merge(r1, rj, r2, readlane_ll(v1, 16 * r), __builtin_amdgcn_readlane(j1, 16 * r), readlane_ll(v2, 16 * r));
    v1 = r1;
    j1 = rj;
    v2 = r2;
}

// Largest value over each row of 16 lanes / over the wave (uniform).
__device__ inline long long auc_row_max(long long v) {
    long long o = dpp_ll<0xB1>(v);
    v = o > v ? o : v;
    o = dpp_ll<0x4E>(v);
    v = o > v ? o : v;
    o = dpp_ll<0x141>(v);
    v = o > v ? o : v;
    o = dpp_ll<0x140>(v);
    return o > v ? o : v;
}
__device__ inline long long auc_wave_max(long long v) {
    v = auc_row_max(v);
    long long m = readlane_ll(v, 0);
#pragma unroll
    for (int r = 1; r < 4; ++r) {
        const long long o = readlane_ll(v, 16 * r);
        m = o > m ? o : m;
    }
    return m;
}

// This thread's best value (lowest column among equals) and second-best
// value over its columns of row i; thread t takes column quads t, t + NT,
// ... On the aligned path a thread issues the loads of up to four chunks of
// the row and of their prices before it uses any of them.
template <int NT>
__device__ inline void auc_lane_scan(const AuctionArgs& a, int i, long long& v1, int& j1, long long& v2) {
    constexpr int U = 4;
    const int t = threadIdx.x;
    const float* r = a.M + (long)i * a.ld;
    v1 = LLONG_MIN;
    v2 = LLONG_MIN;
    j1 = INT_MAX;
    int j0 = 0;
    if (a.cp) {
        // precomputed scores: rows of ldc (a multiple of 4) int64, 32-byte aligned
        const longlong2* c2 = reinterpret_cast<const longlong2*>(a.cp + (long)i * a.ldc);
        const longlong2* p2 = reinterpret_cast<const longlong2*>(a.price);
        const int c4 = a.n >> 2;
        for (int q0 = t; q0 < c4; q0 += NT * U) {
            longlong2 ca[U], cb[U], pa[U], pb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + u * NT;
                if (q < c4) {
                    ca[u] = c2[2 * q];
                    cb[u] = c2[2 * q + 1];
                    pa[u] = p2[2 * q];
                    pb[u] = p2[2 * q + 1];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + u * NT;
                if (q < c4) {
                    const int j = 4 * q;
                    auc_push(v1, j1, v2, ca[u].x - pa[u].x, j);
                    auc_push(v1, j1, v2, ca[u].y - pa[u].y, j + 1);
                    auc_push(v1, j1, v2, cb[u].x - pb[u].x, j + 2);
                    auc_push(v1, j1, v2, cb[u].y - pb[u].y, j + 3);
                }
            }
        }
        for (int j = (c4 << 2) + t; j < a.n; j += NT) auc_push(v1, j1, v2, a.cp[(long)i * a.ldc + j] - a.price[j], j);
        j0 = a.n;     // every column done
    } else if (a.vec4) {
        const int c4 = a.n >> 2;
        const float4* r4 = reinterpret_cast<const float4*>(r);
        const longlong2* p2 = reinterpret_cast<const longlong2*>(a.price);
        for (int q0 = t; q0 < c4; q0 += NT * U) {
            float4 x[U];
            longlong2 pa[U], pb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + u * NT;
                if (q < c4) {
                    x[u] = r4[q];
                    pa[u] = p2[2 * q];
                    pb[u] = p2[2 * q + 1];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + u * NT;
                if (q < c4) {
                    const int j = 4 * q;
                    auc_push(v1, j1, v2, auc_cost(a, x[u].x) - pa[u].x, j);
                    auc_push(v1, j1, v2, auc_cost(a, x[u].y) - pa[u].y, j + 1);
                    auc_push(v1, j1, v2, auc_cost(a, x[u].z) - pb[u].x, j + 2);
                    auc_push(v1, j1, v2, auc_cost(a, x[u].w) - pb[u].y, j + 3);
                }
            }
        }
        j0 = c4 << 2;
    }
    for (int j = j0 + t; j < a.n; j += NT) auc_push(v1, j1, v2, auc_value(a, r[j], j), j);
}

// Best and second-best value of row i over all columns, reduced over the
// block (NT threads); the result is valid in thread 0.
template <int NT>
__device__ inline void auc_scan_row(const AuctionArgs& a, int i, long long& v1, int& j1, long long& v2,
                                    long long* sv1, long long* sv2, int* sj1) {
    static_assert(NT % 64 == 0 && NT / 64 <= 16, "one row of wave 0 merges the waves");
    const int t = threadIdx.x;
    auc_lane_scan<NT>(a, i, v1, j1, v2);
    auc_wave_merge(v1, j1, v2);
    if ((t & 63) == 0) {
        sv1[t >> 6] = v1;
        sv2[t >> 6] = v2;
        sj1[t >> 6] = j1;
    }
    __syncthreads();
    if (t < 64) {
        // wave 0: lane w takes wave w's result, one row merges them
        v1 = LLONG_MIN;
        v2 = LLONG_MIN;
        j1 = INT_MAX;
        if (t < NT / 64) {
            v1 = sv1[t];
            v2 = sv2[t];
            j1 = sj1[t];
        }
        auc_row_merge(v1, j1, v2);
    }
}

// Full scan of row i by the kSeqThreads threads of the sequential kernel,
// with a refresh of the row's candidate list. Each wave contributes the
// kPerWave best of its threads' maxima (e_1 .. e_k) and the largest value
// outside them (tw: the other threads' maxima and every thread's second
// value). The candidates are the e of all waves; no other column is worth
// more than thr_i = max_w tw, and since prices only rise this stays true
// for the rest of the auction. Writes the list (slot k by lane k of wave
// 0); the row's exact (v1, j1, v2), as auc_scan_row gives them, end in
// thread 0. se / sje: LDS [kPerWave][waves], stw: LDS [waves].
__device__ inline void auc_scan_row_lists(const AuctionArgs& a, int i, long long& v1, int& j1, long long& v2,
                                          long long (*se)[kSeqThreads / 64], int (*sje)[kSeqThreads / 64],
                                          long long* stw) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    long long lv1, lv2;
    int lj1;
    auc_lane_scan<kSeqThreads>(a, i, lv1, lj1, lv2);
    // a column belongs to one thread, so each round's winner is the thread
    // holding its column (threads without columns hold INT_MAX and
    // LLONG_MIN: harmless), which then drops out
    long long cv = lv1;
    int cjj = lj1;
#pragma unroll
    for (int k = 0; k < kPerWave; ++k) {
        long long b = cv, d = LLONG_MIN;
        int bj = cjj;
        auc_wave_merge(b, bj, d);
        if (lane == 0) {
            se[k][w] = b;
            sje[k][w] = bj;
        }
        const bool won = cjj == bj;
        cv = won ? LLONG_MIN : cv;
        cjj = won ? INT_MAX : cjj;
    }
    const long long rest = cv > lv2 ? cv : lv2;
    const long long tw = auc_wave_max(rest);
    if (lane == 0) stw[w] = tw;
    __syncthreads();
    if (w == 0) {
        {
            const int ww = lane / kPerWave, k = lane % kPerWave;
            const long long ev = se[k][ww];
            const int ej = sje[k][ww];
            const bool ok = ej >= 0 && ej < a.n;
            a.cj[(long)i * kCand + lane] = ok ? ej : -1;
            a.cc[(long)i * kCand + lane] = ok ? ev + a.price[ej] : 0;
        }
        // the row's exact result: wave w's top two are e_1 and max(e_2, tw)
        // (e_3 .. e_k are at most e_2), so merging those pairs over the
        // waves gives (v1, j1, v2); lane w takes wave w, one row merges
        long long tw_l = LLONG_MIN;
        v1 = LLONG_MIN;
        v2 = LLONG_MIN;
        j1 = INT_MAX;
        if (lane < kSeqThreads / 64) {
            v1 = se[0][lane];
            j1 = sje[0][lane];
            tw_l = stw[lane];
            v2 = se[1][lane] > tw_l ? se[1][lane] : tw_l;
        }
        auc_row_merge(v1, j1, v2);
        const long long T = auc_row_max(tw_l);
        if (lane == 0) a.thr[i] = T;
    }
}

// Bid of row i from its candidate list alone, by wave 0 (lane k reads slot
// k, the lane that wrote it): the best candidate (lowest column among
// equals) and the second-best candidate value. Exact whenever v1 > thr_i
// and v2 >= thr_i, since no column outside the list is worth more than
// thr_i; the return value says whether that holds (valid in lane 0).
__device__ inline bool auc_try_list(const AuctionArgs& a, int i, long long& v1, int& j1, long long& v2) {
    const int lane = threadIdx.x & 63;
    const long long T = lane == 0 ? a.thr[i] : LLONG_MAX;
    int c = -1;
    long long sc = 0;
    if (lane < kCand) {
        c = a.cj[(long)i * kCand + lane];
        sc = a.cc[(long)i * kCand + lane];
    }
    v1 = LLONG_MIN;
    v2 = LLONG_MIN;
    j1 = INT_MAX;
    if (c >= 0 && c < a.n) {
        v1 = sc - a.price[c];
        j1 = c;
    }
    auc_wave_merge(v1, j1, v2);
    return v1 > T && v2 >= T;
}

// Parallel bids: one workgroup per bidding row; this block's rows are
// blockIdx.x + k * gridDim.x, their assignment flags read in one parallel
// load, AB rows at a time (order within the list does not matter: every bid
// of a round sees the same prices).
__global__ __launch_bounds__(AB) void auction_bid_kernel(AuctionArgs a, long long eps) {
    __shared__ long long sv1[AB / 64], sv2[AB / 64];
    __shared__ int sj1[AB / 64];
    __shared__ int rows[AB];
    __shared__ int cnt;
    if (a.ctl[0] == a.n) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&a.ctl[2], 1);
    const int t = threadIdx.x;
    const int per = (a.n - (int)blockIdx.x + (int)gridDim.x - 1) / (int)gridDim.x;
    for (int base = 0; base < per; base += AB) {
        if (t == 0) cnt = 0;
        __syncthreads();
        const int k = base + t;
        if (k < per) {
            const int i = (int)blockIdx.x + k * (int)gridDim.x;
            if (a.assign[i] < 0) rows[atomicAdd(&cnt, 1)] = i;
        }
        __syncthreads();
        const int m = cnt;
        for (int u = 0; u < m; ++u) {
            const int i = rows[u];
            long long v1, v2;
            int j1;
            auc_scan_row<AB>(a, i, v1, j1, v2, sv1, sv2, sj1);
            if (t == 0) {
                // n >= 2, so both values are real: bid = price + (v1 - v2) + eps
                const long long bid = a.price[j1] + (v1 - v2) + eps;
                if (bid >= kBidLimit) {
                    atomicOr(&a.ctl[1], 1);
                } else {
                    a.mybid[i] = bid;
                    a.tgt[i] = j1;
                    atomicMax(&a.best[j1], bid);
                }
            }
            __syncthreads();
        }
    }
}

// Among the rows whose bid equals their object's maximum, the lowest wins.
__global__ __launch_bounds__(AB) void auction_claim_kernel(AuctionArgs a) {
    const int i = blockIdx.x * AB + threadIdx.x;
    if (i >= a.n) return;
    const int j = a.tgt[i];
    if (j < 0) return;
    a.tgt[i] = -1;
    if (a.mybid[i] == a.best[j]) atomicMin(&a.win[j], i);
}

__global__ __launch_bounds__(AB) void auction_resolve_kernel(AuctionArgs a) {
    const int j = blockIdx.x * AB + threadIdx.x;
    if (j >= a.n) return;
    const int i = a.win[j];
    if (i == kNoRow) return;
    a.win[j] = kNoRow;
    a.price[j] = a.best[j];
    a.best[j] = 0;
    const int old = a.owner[j];
    a.owner[j] = i;
    a.assign[i] = j;
    // the previous owner was assigned at the start of the round, so it made
    // no bid and no other object writes its entry
    if (old >= 0)
        a.assign[old] = -1;
    else
        atomicAdd(&a.ctl[0], 1);
}

// Phase start without a full restart: a row keeps its object when the pair
// still satisfies eps-complementary slackness for the new, smaller eps
// (its value is within eps of the row's best); later price rises only make
// other objects worse, so kept pairs stay valid. Other rows are released.
// ctl[0] counts the kept rows and the int64 at ctl + 8 receives the largest
// slack v1 - va among them (the reset before this kernel zeroed both).
__global__ __launch_bounds__(AB) void auction_keep_kernel(AuctionArgs a, long long eps) {
    __shared__ long long sv[AB / 64];
    const int t = threadIdx.x;
    long long dmax = -1;         // thread 0: largest kept slack of this block's rows
    for (int i = blockIdx.x; i < a.n; i += gridDim.x) {
        const int ja = a.assign[i];
        if (ja < 0) continue;
        const float* r = a.M + (long)i * a.ld;
        long long v1 = LLONG_MIN;
        for (int j = t; j < a.n; j += AB) {
            const long long v = a.cp ? a.cp[(long)i * a.ldc + j] - a.price[j] : auc_value(a, r[j], j);
            v1 = v > v1 ? v : v1;
        }
        v1 = auc_wave_max(v1);
        if ((t & 63) == 0) sv[t >> 6] = v1;
        __syncthreads();
        if (t == 0) {
            for (int w = 1; w < AB / 64; ++w) v1 = sv[w] > v1 ? sv[w] : v1;
            const long long va = a.cp ? a.cp[(long)i * a.ldc + ja] - a.price[ja] : auc_value(a, r[ja], ja);
            if (v1 - va > eps) {
                a.assign[i] = -1;
                a.owner[ja] = -1;
            } else {
                atomicAdd(&a.ctl[0], 1);
                dmax = v1 - va > dmax ? v1 - va : dmax;
            }
        }
        __syncthreads();
    }
    if (t == 0 && dmax >= 0) atomicMax(reinterpret_cast<unsigned long long*>(a.ctl + 8), (unsigned long long)dmax);
}

// Scaled integer scores c'_ij = (rint(M_ij 2^s) - qmin) (n + 1), written once
// so that every later scan reads them instead of converting floats.
__global__ __launch_bounds__(AB) void auction_cost_kernel(AuctionArgs a, long long* __restrict__ cp) {
    for (int i = blockIdx.x; i < a.n; i += gridDim.x) {
        const float* r = a.M + (long)i * a.ld;
        long long* o = cp + (long)i * a.ldc;
        for (int j = threadIdx.x; j < a.n; j += AB) o[j] = auc_cost(a, r[j]);
    }
}

// mode 0: everything (prices to zero); 1: assignments released, prices
// kept; 2: only the assigned-row count (before auction_keep_kernel)
__global__ __launch_bounds__(AB) void auction_reset_kernel(AuctionArgs a, int mode) {
    const int j = blockIdx.x * AB + threadIdx.x;
    if (j == 0) {
        a.ctl[0] = 0;
        *reinterpret_cast<unsigned long long*>(a.ctl + 8) = 0;
        if (mode == 0) {
            a.ctl[1] = 0;
            a.ctl[2] = 0;
            a.ctl[3] = 0;
            a.ctl[4] = 0;
        }
    }
    if (j >= a.n) return;
    if (mode == 0) {
        a.price[j] = 0;
        a.best[j] = 0;
        a.win[j] = kNoRow;
        a.tgt[j] = -1;
        a.thr[j] = LLONG_MAX;
        for (int k = 0; k < kCand; ++k) a.cj[(long)j * kCand + k] = -1;
    }
    if (mode == 2) return;
    a.owner[j] = -1;
    a.assign[j] = -1;
}

// Sequential bidding: when parallel rounds assign few rows each (the tail
// of a phase, or rows that all want the same objects), one 1024-thread
// workgroup takes the bids one after the other (the Gauss-Seidel auction)
// inside one launch instead of three launches per round. The unassigned
// rows form a queue in global memory (capacity n), built in increasing row
// order; an evicted row takes its evictor's place at the head. At most
// `budget` bids per launch, so every launch ends.
constexpr int TB = kSeqThreads;

// LDSST: prices, owners and the assignment live in LDS for the launch
// (16 bytes per vertex, dynamic shared memory), copied in at the start and
// back at the end, so the scan's price reads and the updates of the bidding
// thread stay on the CU.
//
// With `lists`, a bid first tries the row's candidate list (auc_try_list)
// and scans the row only when the list cannot decide it; the scan then
// refreshes the list. Both give the same bid.
template <bool LDSST>
__global__ __launch_bounds__(TB) void auction_seq_kernel(AuctionArgs g, int* __restrict__ q, long long eps,
                                                        long long budget, int lists) {
    extern __shared__ __attribute__((aligned(16))) unsigned char seq_smem[];
    __shared__ int qn, cur, list_hit;
    __shared__ int wcnt[TB / 64];
    __shared__ long long sv1[TB / 64], sv2[TB / 64], stw[TB / 64];
    __shared__ int sj1[TB / 64];
    __shared__ long long se[kPerWave][TB / 64];
    __shared__ int sje[kPerWave][TB / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    AuctionArgs a = g;
    if (LDSST) {
        const int nal = (g.n + 3) & ~3;
        a.price = reinterpret_cast<long long*>(seq_smem);
        a.owner = reinterpret_cast<int32_t*>(seq_smem + (size_t)8 * nal);
        a.assign = a.owner + nal;
        for (int j = t; j < g.n; j += TB) {
            a.price[j] = g.price[j];
            a.owner[j] = g.owner[j];
            a.assign[j] = g.assign[j];
        }
    }
    if (t == 0) qn = 0;
    __syncthreads();
    for (int base = 0; base < a.n; base += TB) {
        const int i = base + t;
        const bool un = i < a.n && a.assign[i] < 0;
        const unsigned long long m = __ballot(un);
        if (lane == 0) wcnt[w] = __popcll(m);
        __syncthreads();
        int off = qn;
        for (int u = 0; u < w; ++u) off += wcnt[u];
        off += __popcll(m & ((1ull << lane) - 1ull));
        if (un) q[off] = i;
        __syncthreads();
        if (t == 0) {
            int tot = 0;
            for (int u = 0; u < TB / 64; ++u) tot += wcnt[u];
            qn += tot;
        }
        __syncthreads();
    }
    if (t == 0 && qn > 0) cur = q[0];
    __syncthreads();
    long long done = 0;
    int hits = 0;
    // lists that decide fewer than a quarter of a window of tries are left
    // aside for the next kListSkip bids (every thread keeps the same count)
    constexpr int kListWindow = 32, kListSkip = 256;
    int tries = 0, wins = 0, skip = 0;
    while (qn > 0 && done < budget) {
        const int i = cur;
        long long v1, v2;
        int j1;
        if (lists && skip == 0) {
            if (w == 0) {
                const bool hit = auc_try_list(a, i, v1, j1, v2);
                if (lane == 0) list_hit = hit;
            }
            __syncthreads();
            const bool hit = list_hit;
            ++tries;
            wins += hit;
            if (tries == kListWindow) {
                if (4 * wins < kListWindow) skip = kListSkip;
                tries = 0;
                wins = 0;
            }
            if (hit) {
                hits += t == 0;
            } else {
                auc_scan_row_lists(a, i, v1, j1, v2, se, sje, stw);
            }
        } else {
            skip -= skip > 0;
            auc_scan_row<TB>(a, i, v1, j1, v2, sv1, sv2, sj1);
        }
        if (t == 0) {
            // both loads issue before either is used
            const long long pj = a.price[j1];
            const int old = a.owner[j1];
            const long long bid = pj + (v1 - v2) + eps;
            if (bid >= kBidLimit) {
                atomicOr(&a.ctl[1], 1);
                qn = 0;
            } else {
                a.owner[j1] = i;
                a.assign[i] = j1;
                a.price[j1] = bid;
                if (old >= 0) {
                    a.assign[old] = -1;
                    q[0] = old;
                    cur = old;
                } else {
                    a.ctl[0] += 1;
                    const int last = q[qn - 1];
                    q[0] = last;
                    cur = last;
                    qn -= 1;
                }
            }
        }
        ++done;
        // thread 0's stores to price, owner and assign are seen by the whole
        // workgroup after the barrier
        __syncthreads();
    }
    if (LDSST) {
        for (int j = t; j < g.n; j += TB) {
            g.price[j] = a.price[j];
            g.owner[j] = a.owner[j];
            g.assign[j] = a.assign[j];
        }
    }
    if (t == 0) {
        a.ctl[3] += (int)done;
        a.ctl[4] += hits;
    }
}

// per block: max |x|, min x, and a flag for non-finite entries
__global__ __launch_bounds__(AB) void auction_range_kernel(int n, const float* __restrict__ M, long ld,
                                                           float* __restrict__ part) {
    __shared__ float sh[3][AB / 64];
    float mx = 0.0f, mn = INFINITY, bad = 0.0f;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const float* r = M + (long)i * ld;
        for (int j = threadIdx.x; j < n; j += AB) {
            const float x = r[j];
            if (!isfinite(x)) bad = 1.0f;
            mx = fmaxf(mx, fabsf(x));
            mn = fminf(mn, x);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmaxf(mx, __shfl_xor(mx, o, 64));
        mn = fminf(mn, __shfl_xor(mn, o, 64));
        bad = fmaxf(bad, __shfl_xor(bad, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = mx;
        sh[1][threadIdx.x >> 6] = mn;
        sh[2][threadIdx.x >> 6] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < AB / 64; ++w) {
            mx = fmaxf(mx, sh[0][w]);
            mn = fminf(mn, sh[1][w]);
            bad = fmaxf(bad, sh[2][w]);
        }
        part[3 * blockIdx.x] = mx;
        part[3 * blockIdx.x + 1] = mn;
        part[3 * blockIdx.x + 2] = bad;
    }
}

constexpr int kRangeWG = 512;
constexpr long long kSeqBudget = 262144;      // bids per sequential launch

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Tuning: GOAT_LAP_TAIL (unassigned rows that switch a phase to sequential
// bids, default 32), GOAT_LAP_RATE (a batch of parallel rounds that assigns
// fewer rows than this per round also switches, default 2), GOAT_LAP_THETA
// (epsilon divisor between phases, default 3), GOAT_LAP_KEEP (0: every
// phase restarts from no assignment; default 1 keeps the pairs that stay
// eps-optimal), GOAT_LAP_BITS (score resolution R, default and maximum 40),
// GOAT_LAP_SEQ_GLOBAL=1 (sequential bids keep their state in global memory),
// GOAT_LAP_LISTS=0 (sequential bids always scan the whole row),
// GOAT_LAP_SKIP_IDLE=0 (run every phase, also those that would keep every
// pair),
// GOAT_LAP_TRACE=1 (per-phase counts on stderr).
struct LapKnobs {
    int tail = 32, theta = 3, trace = 0, keep = 1, rate = 2, seq_global = 0, lists = 1, skip_idle = 1;
};
const LapKnobs& lap_knobs() {
    static const LapKnobs k = [] {
        LapKnobs r;
        if (const char* e = std::getenv("GOAT_LAP_TAIL")) r.tail = std::max(0, std::atoi(e));
        if (const char* e = std::getenv("GOAT_LAP_RATE")) r.rate = std::max(0, std::atoi(e));
        if (const char* e = std::getenv("GOAT_LAP_THETA")) r.theta = std::max(2, std::atoi(e));
        if (const char* e = std::getenv("GOAT_LAP_TRACE")) r.trace = std::atoi(e);
        if (const char* e = std::getenv("GOAT_LAP_KEEP")) r.keep = std::atoi(e) != 0;
        if (const char* e = std::getenv("GOAT_LAP_SEQ_GLOBAL")) r.seq_global = std::atoi(e) != 0;
        if (const char* e = std::getenv("GOAT_LAP_LISTS")) r.lists = std::atoi(e) != 0;
        if (const char* e = std::getenv("GOAT_LAP_SKIP_IDLE")) r.skip_idle = std::atoi(e) != 0;
        return r;
    }();
    return k;
}

// dynamic LDS of the sequential kernel, at most: 160 KB per workgroup less
// 2 KB for its static arrays
constexpr size_t kSeqLdsMax = 160 * 1024 - 2048;

// LDS bytes of the sequential kernel's state for n vertices, or 0 when it
// does not fit (the state then stays in global memory)
size_t seq_lds_bytes(int n) {
    const size_t b = (size_t)16 * ((n + 3) & ~3);
    if (b > kSeqLdsMax || lap_knobs().seq_global) return 0;
    static const bool ok = hipFuncSetAttribute(reinterpret_cast<const void*>(auction_seq_kernel<true>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)kSeqLdsMax) == hipSuccess;
    return ok ? b : 0;
}

}  // namespace

size_t auction_ws_bytes(int n) {
    if (n < 1) return 0;
    return align256((size_t)n * 8) * 4 + align256((size_t)n * 4) * 5 + 256 + align256(kRangeWG * 3 * 4) +
           align256((size_t)n * kCand * 4) + align256((size_t)n * kCand * 8);
}

size_t auction_ws_bytes_fast(int n) {
    if (n < 1) return 0;
    const size_t ldc = (size_t)((n + 3) & ~3);
    return auction_ws_bytes(n) + align256(ldc * n * 8);
}

int auction_resolution_bits(int n) {
    int b = 0;
    while ((1ll << b) < (long long)n + 1) ++b;   // ceil(log2(n + 1))
    int r = 40;
    if (const char* e = std::getenv("GOAT_LAP_BITS")) r = std::max(8, std::min(40, std::atoi(e)));
    return std::min(r, 55 - b);
}

int auction_lap(int n, const float* M, int ld, int32_t* perm_dev, void* ws, size_t ws_bytes, long long max_rounds,
                AuctionStats* st, hipStream_t s) {
    AuctionStats loc{};
    if (n >= (1 << 20) - 1) {
        set_error("goat_lap_device: n too large");
        return GOAT_EINVAL;
    }
    if (ws_bytes < auction_ws_bytes(n)) {
        set_error("goat_lap_device: workspace too small");
        return GOAT_ENOMEM;
    }
    char* base = static_cast<char*>(ws);
    auto take = [&](size_t bytes) {
        char* p = base;
        base += align256(bytes);
        return p;
    };
    AuctionArgs a{};
    a.M = M;
    a.ld = ld;
    a.n = n;
    a.np1 = (long long)n + 1;
    a.vec4 = (ld % 4) == 0 && (reinterpret_cast<uintptr_t>(M) % 16) == 0;
    a.price = reinterpret_cast<long long*>(take((size_t)n * 8));
    a.best = reinterpret_cast<long long*>(take((size_t)n * 8));
    a.mybid = reinterpret_cast<long long*>(take((size_t)n * 8));
    a.win = reinterpret_cast<int32_t*>(take((size_t)n * 4));
    a.tgt = reinterpret_cast<int32_t*>(take((size_t)n * 4));
    a.owner = reinterpret_cast<int32_t*>(take((size_t)n * 4));
    a.assign = reinterpret_cast<int32_t*>(take((size_t)n * 4));
    int* queue = reinterpret_cast<int*>(take((size_t)n * 4));
    a.ctl = reinterpret_cast<int*>(take(256));
    float* part = reinterpret_cast<float*>(take(kRangeWG * 3 * 4));
    a.thr = reinterpret_cast<long long*>(take((size_t)n * 8));
    a.cj = reinterpret_cast<int32_t*>(take((size_t)n * kCand * 4));
    a.cc = reinterpret_cast<long long*>(take((size_t)n * kCand * 8));
    // with room for them, the scaled scores are precomputed once (8 bytes
    // per entry) and every scan reads them
    const long ldc = (n + 3) & ~3;
    long long* cp = ws_bytes >= auction_ws_bytes_fast(n) ? reinterpret_cast<long long*>(take((size_t)ldc * n * 8))
                                                         : nullptr;

    // score range: the quantisation's shift and offset
    const int nb = std::min(n, kRangeWG);
    hipLaunchKernelGGL(auction_range_kernel, dim3(nb), dim3(AB), 0, s, n, M, (long)ld, part);
    GOAT_HIP(hipGetLastError());
    std::vector<float> hp((size_t)nb * 3);
    GOAT_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * 4, hipMemcpyDeviceToHost, s));
    GOAT_HIP(hipStreamSynchronize(s));
    float mx = 0.0f, mn = INFINITY;
    for (int b = 0; b < nb; ++b) {
        if (hp[3 * b + 2] != 0.0f) {
            set_error("goat_lap_device: non-finite entry");
            return GOAT_EINVAL;
        }
        mx = std::max(mx, hp[3 * b]);
        mn = std::min(mn, hp[3 * b + 1]);
    }
    const int R = auction_resolution_bits(n);
    int e = 0;
    if (mx > 0.0f) std::frexp(mx, &e);
    a.s = R - 1 - e;
    // rint is monotone, so min q = q(min M); both are exact in double
    a.qmin = (long long)std::nearbyint(std::ldexp((double)mn, a.s));
    const long long cmax = (long long)std::nearbyint(std::ldexp((double)mx, a.s)) - a.qmin;
    loc.shift = a.s;
    loc.resolution_bits = R;

    const int gr = (n + AB - 1) / AB;
    hipLaunchKernelGGL(auction_reset_kernel, dim3(gr), dim3(AB), 0, s, a, 0);
    GOAT_HIP(hipGetLastError());
    if (n == 1 || cmax == 0) {
        // one vertex, or all scores equal after quantisation: the identity
        // (lowest columns first) is optimal
        std::vector<int32_t> id(n);
        for (int i = 0; i < n; ++i) id[i] = i;
        GOAT_HIP(hipMemcpyAsync(perm_dev, id.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
        GOAT_HIP(hipStreamSynchronize(s));
        if (st) *st = loc;
        return GOAT_OK;
    }
    // bidding grid: one workgroup per row while many bid, a stride loop beyond
    const int gb = std::min(n, 2048);
    if (cp) {
        a.ldc = ldc;
        hipLaunchKernelGGL(auction_cost_kernel, dim3(gb), dim3(AB), 0, s, a, cp);
        GOAT_HIP(hipGetLastError());
        a.cp = cp;
    }
    // sequential bids keep their state in LDS when 16 bytes per vertex fit
    const size_t seq_lds = seq_lds_bytes(n);
    const long long cbig = cmax * a.np1;
    long long eps = std::max(1ll, cbig / 4);
    int ctl[12] = {0};           // device ctl[0..4]; ctl[8..9]: the keep filter's largest slack (int64)
    long long work = 0;          // parallel rounds launched + sequential budgets
    const LapKnobs& kn = lap_knobs();
    int prev_rounds = 0, prev_seq = 0, prev_hits = 0;
    auto tp = std::chrono::steady_clock::now();
    for (;;) {
        ++loc.phases;
        int left = n;
        bool idle = false;       // the phase filter kept every pair: no bid in this phase
        long long slack = 0;
        if (loc.phases > 1) {
            hipLaunchKernelGGL(auction_reset_kernel, dim3(gr), dim3(AB), 0, s, a, kn.keep ? 2 : 1);
            if (kn.keep) hipLaunchKernelGGL(auction_keep_kernel, dim3(gb), dim3(AB), 0, s, a, eps);
            GOAT_HIP(hipGetLastError());
            if (kn.keep) {
                GOAT_HIP(hipMemcpyAsync(ctl, a.ctl, sizeof(ctl), hipMemcpyDeviceToHost, s));
                GOAT_HIP(hipStreamSynchronize(s));
                left = n - ctl[0];
                idle = left == 0;
                std::memcpy(&slack, &ctl[8], sizeof(slack));
            }
        }
        int batch = 4;
        bool seq = false;
        while (left > 0) {
            const bool sequential = seq || left <= kn.tail;
            if (sequential) {
                const long long budget = std::min(kSeqBudget, std::max(1ll, max_rounds - work));
                if (seq_lds)
                    hipLaunchKernelGGL(auction_seq_kernel<true>, dim3(1), dim3(TB), seq_lds, s, a, queue, eps,
                                       budget, kn.lists);
                else
                    hipLaunchKernelGGL(auction_seq_kernel<false>, dim3(1), dim3(TB), 0, s, a, queue, eps, budget,
                                       kn.lists);
                work += budget;
            } else {
                for (int k = 0; k < batch; ++k) {
                    hipLaunchKernelGGL(auction_bid_kernel, dim3(gb), dim3(AB), 0, s, a, eps);
                    hipLaunchKernelGGL(auction_claim_kernel, dim3(gr), dim3(AB), 0, s, a);
                    hipLaunchKernelGGL(auction_resolve_kernel, dim3(gr), dim3(AB), 0, s, a);
                }
                work += batch;
            }
            GOAT_HIP(hipGetLastError());
            GOAT_HIP(hipMemcpyAsync(ctl, a.ctl, sizeof(ctl), hipMemcpyDeviceToHost, s));
            GOAT_HIP(hipStreamSynchronize(s));
            if (ctl[1]) {
                set_error("goat_lap_device: bid overflow");
                return GOAT_ENOTSUP;
            }
            const int now_left = n - ctl[0];
            if (!sequential) {
                // rows that collide on the same objects: bid one by one
                if ((long long)(left - now_left) < (long long)kn.rate * batch) seq = true;
                batch = std::min(batch * 2, 64);
                if (now_left <= 4 * kn.tail) batch = 4;
            }
            left = now_left;
            if (left == 0) break;
            if (work >= max_rounds) {
                set_error("goat_lap_device: round limit reached");
                return GOAT_ENOTSUP;
            }
        }
        if (kn.trace) {
            const auto now = std::chrono::steady_clock::now();
            std::fprintf(stderr, "[lap] phase %d eps %lld: rounds %d, sequential bids %d (list %d), %.2f ms\n",
                         loc.phases, eps, ctl[2] - prev_rounds, ctl[3] - prev_seq, ctl[4] - prev_hits,
                         std::chrono::duration<double, std::milli>(now - tp).count());
            tp = now;
            prev_rounds = ctl[2];
            prev_seq = ctl[3];
            prev_hits = ctl[4];
        }
        if (eps == 1) break;
        eps = std::max(1ll, eps / kn.theta);
        // No bid ran in an idle phase, so prices and slacks are what its
        // filter measured: every later phase whose eps is at least the
        // largest slack would keep every pair and bid nothing. Those phases
        // are counted and passed over.
        if (idle && kn.skip_idle) {
            bool done = false;
            while (slack <= eps) {
                ++loc.phases;
                ++loc.skipped_phases;
                if (eps == 1) {
                    done = true;
                    break;
                }
                eps = std::max(1ll, eps / kn.theta);
            }
            if (done) break;
        }
    }
    loc.rounds = ctl[2];
    loc.tail_bids = ctl[3];
    loc.list_bids = ctl[4];
    loc.rounds_launched = work;
    GOAT_HIP(hipMemcpyAsync(perm_dev, a.assign, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    GOAT_HIP(hipStreamSynchronize(s));
    if (st) *st = loc;
    return GOAT_OK;
}

// ---------------------------------------------------------------- batched assignment
//
// The final assignment of every (pair, start) problem of a batch (n <= 1024)
// on the device: the same integer auction as above (same quantisation, bid
// rule, epsilon schedule and phase-start filter) run by one 64-thread
// workgroup per problem with prices, owners, assignment and the bid queue in
// LDS, bids taken one after the other. A problem stops after `budget` bids;
// its status is then GOAT_ENOTSUP.

namespace {

constexpr int BW = 64;                 // one wave per problem
constexpr int kBatchLapMax = 1024;

__global__ __launch_bounds__(BW) void batch_auction_kernel(const BProb* __restrict__ probs, int proj,
                                                           const int* __restrict__ offs, int32_t* __restrict__ perms,
                                                           int* __restrict__ status, long long budget, int theta,
                                                           int skip_idle) {
    __shared__ long long price[kBatchLapMax];
    __shared__ int owner[kBatchLapMax], assign[kBatchLapMax], queue[kBatchLapMax];
    __shared__ int qn, overflow;
    const int k = blockIdx.x, t = threadIdx.x;
    const BProb& q = probs[k];
    const int n = q.n;
    const long ld = q.np;
    if (n > kBatchLapMax || n < 1) {
        if (t == 0) status[k] = GOAT_EINVAL;
        return;
    }
    const float* M = proj ? q.GP : q.P;
    int32_t* out = perms + offs[k];

    // score range and finiteness
    float mx = 0.0f, mn = INFINITY;
    bool bad = false;
    for (int i = 0; i < n; ++i)
        for (int j = t; j < n; j += BW) {
            const float x = M[i * ld + j];
            bad |= !isfinite(x);
            mx = fmaxf(mx, fabsf(x));
            mn = fminf(mn, x);
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmaxf(mx, __shfl_xor(mx, o, 64));
        mn = fminf(mn, __shfl_xor(mn, o, 64));
    }
    if (__any(bad)) {
        if (t == 0) status[k] = GOAT_EINVAL;
        return;
    }
    // integer scores: the quantisation of auction_lap
    int b = 0;
    while ((1ll << b) < (long long)n + 1) ++b;
    const int R = min(40, 55 - b);
    int e = 0;
    if (mx > 0.0f) frexpf(mx, &e);
    AuctionArgs a{};
    a.M = M;
    a.ld = ld;
    a.n = n;
    a.s = R - 1 - e;
    a.qmin = (long long)rintf(ldexpf(mn, a.s));
    a.np1 = (long long)n + 1;
    a.price = price;
    const long long cmax = (long long)rintf(ldexpf(mx, a.s)) - a.qmin;
    for (int j = t; j < n; j += BW) {
        price[j] = 0;
        owner[j] = -1;
        assign[j] = -1;
    }
    if (t == 0) overflow = 0;
    __syncthreads();
    if (n == 1 || cmax == 0) {
        for (int i = t; i < n; i += BW) out[i] = i;
        if (t == 0) status[k] = 0;
        return;
    }
    long long eps = max(1ll, cmax * a.np1 / 4);
    long long bids = 0;
    __shared__ long long sdmax;
    bool first = true;
    for (;;) {
        // phase start: rows whose pair is no longer eps-optimal are released;
        // sdmax: the largest slack among the kept pairs
        const bool filtered = !first;
        if (filtered) {
            long long dmax = -1;
            for (int i = 0; i < n; ++i) {
                const int ja = assign[i];
                long long v1 = LLONG_MIN;
                for (int j = t; j < n; j += BW) {
                    const long long v = auc_cost(a, M[i * ld + j]) - price[j];
                    v1 = v > v1 ? v : v1;
                }
                v1 = auc_wave_max(v1);
                if (t == 0) {
                    const long long d = v1 - (auc_cost(a, M[i * ld + ja]) - price[ja]);
                    if (d > eps) {
                        assign[i] = -1;
                        owner[ja] = -1;
                    } else {
                        dmax = d > dmax ? d : dmax;
                    }
                }
            }
            if (t == 0) sdmax = dmax;
            __syncthreads();
        }
        first = false;
        if (t == 0) {
            int c = 0;
            for (int i = 0; i < n; ++i)
                if (assign[i] < 0) queue[c++] = i;
            qn = c;
        }
        __syncthreads();
        const int qn0 = qn;
        while (qn > 0 && bids < budget) {
            const int i = queue[0];
            long long v1 = LLONG_MIN, v2 = LLONG_MIN;
            int j1 = INT_MAX;
            for (int j = t; j < n; j += BW) auc_push(v1, j1, v2, auc_cost(a, M[i * ld + j]) - price[j], j);
            auc_wave_merge(v1, j1, v2);
            if (t == 0) {
                // n >= 2, so both values are real. Prices stay far below the
                // limit (c <= 2^40 scaled by n + 1 <= 1025, epsilon at most a
                // quarter of that), but a bid past it would wrap: the
                // problem then fails as in auction_lap
                const long long bid = price[j1] + (v1 - v2) + eps;
                if (bid >= kBidLimit) {
                    overflow = 1;
                    qn = 0;
                } else {
                    const int old = owner[j1];
                    owner[j1] = i;
                    assign[i] = j1;
                    price[j1] = bid;
                    if (old >= 0) {
                        assign[old] = -1;
                        queue[0] = old;
                    } else {
                        queue[0] = queue[qn - 1];
                        qn = qn - 1;
                    }
                }
            }
            ++bids;
            __syncthreads();
        }
        if (qn > 0 || overflow) {
            if (t == 0) status[k] = GOAT_ENOTSUP;
            return;
        }
        // the filter kept every pair (idle = no row was queued): phases whose
        // eps is at least the largest slack would keep every pair too and
        // bid nothing; they are passed over (as in auction_lap)
        const bool idle = filtered && qn0 == 0;
        if (eps == 1) break;
        eps = max(1ll, eps / theta);
        if (idle && skip_idle) {
            const long long d = sdmax;
            bool done = false;
            while (d <= eps) {
                if (eps == 1) {
                    done = true;
                    break;
                }
                eps = max(1ll, eps / theta);
            }
            if (done) break;
        }
    }
    for (int i = t; i < n; i += BW) out[i] = assign[i];
    if (t == 0) status[k] = bids > INT_MAX ? INT_MAX : (int)bids;
}

}  // namespace

int batch_auction_launch(const BProb* probs_dev, int nprob, int proj, const int* offs_dev, int32_t* perms_dev,
                         int* status_dev, long long budget, hipStream_t s) {
    if (nprob < 1) return GOAT_OK;
    hipLaunchKernelGGL(batch_auction_kernel, dim3(nprob), dim3(BW), 0, s, probs_dev, proj, offs_dev, perms_dev,
                       status_dev, budget, lap_knobs().theta, lap_knobs().skip_idle);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

}  // namespace goat
