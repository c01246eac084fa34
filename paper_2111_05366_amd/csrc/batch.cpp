// Host side of the batched solver: workspace plan, XCD-aware problem order,
// graph capture (packing, then one persistent kernel per size bucket as
// parallel graph branches), final assignments on the host, device scoring,
// the choice among starts, and the shape autotuner.
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "batch.h"
#include "common.h"

namespace goat {
namespace {

constexpr int kXcds = 8;          // workgroups are dealt to the 8 XCDs round-robin
constexpr int kMaxDevices = 16;
constexpr float kInitTol = 1e-6f; // Sinkhorn-Knopp scaling of the random starts
constexpr int kInitMax = 1000;

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

BShape shape_for(int L, int waves, int npb) {
    BShape s;
    s.L = L;
    s.waves = waves;
    int c = (npb + 4 * L - 1) / (4 * L);
    s.cmax = c <= 1 ? 1 : (c <= 2 ? 2 : 4);
    return s;
}

// default shapes: row groups as narrow as the bucket allows
BShape default_shape(int b) {
    static const int Ls[kBatchBuckets] = {16, 16, 32, 64, 64};
    return shape_for(Ls[b], 4, kBucketMax[b]);
}

std::mutex g_tune_mu;
BShape g_tuned[kMaxDevices][kBatchBuckets];
bool g_has_tuned[kMaxDevices][kBatchBuckets];

BShape current_shape(int b) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (dev >= 0 && dev < kMaxDevices && g_has_tuned[dev][b]) return g_tuned[dev][b];
    return default_shape(b);
}

struct Plan {
    size_t probs, order_off, jobs, hist, fwd, score, perms, offs, lapst, pairs_mat, probs_mat, total;
    std::vector<size_t> pair_off, prob_off;
    int nprob = 0, total_blocks = 0, sum_n = 0;
    // per bucket: first block in the order array and number of blocks
    int bstart[kBatchBuckets] = {0}, bcount[kBatchBuckets] = {0};
    std::vector<int> order;       // block -> problem
};

bool general_of(const goat_options& o) { return o.symmetric == 0; }

int validate(const goat_pair* pairs, int npairs, int restarts, const goat_options* opt) {
    if (!pairs || npairs < 1 || restarts < 1 || !opt) {
        set_error("goat_batch: bad arguments");
        return GOAT_EINVAL;
    }
    for (int p = 0; p < npairs; ++p) {
        const goat_pair& q = pairs[p];
        if (q.n < 1 || q.n > GOAT_BATCH_NMAX || q.ld < q.n || !q.A || !q.B) {
            set_error("goat_batch: bad pair " + std::to_string(p));
            return GOAT_EINVAL;
        }
    }
    if (!(std::isfinite(opt->eps_rel) && opt->eps_rel > 0.0f) || !(std::isfinite(opt->sk_tol) && opt->sk_tol >= 0.0f) ||
        opt->sk_max < 1 || opt->fw_max < 1 || !(std::isfinite(opt->fw_tol) && opt->fw_tol >= 0.0f) ||
        (opt->proj != 0 && opt->proj != 1) || (opt->lap != 0 && opt->lap != 1)) {
        set_error("goat_batch: bad options");
        return GOAT_EINVAL;
    }
    if (opt->prec != GOAT_PREC_FP32 || opt->warm < 0 || opt->warm > 1 || opt->sk_g24 != 0) {
        set_error("goat_batch: only fp32 products, warm 0/1 and float G (sk_g24 = 0) are supported");
        return GOAT_ENOTSUP;
    }
    return GOAT_OK;
}

Plan make_plan(const goat_pair* pairs, int npairs, int restarts, const goat_options& o) {
    Plan pl;
    const bool gen = general_of(o);
    pl.nprob = npairs * restarts;
    // block order: per bucket, pairs dealt to XCDs by largest remaining work
    // first (restarts of a pair share A, B: same XCD, same L2); each XCD's
    // list runs largest problems first; block b goes to XCD b % 8
    std::vector<std::vector<int>> bucket_pairs(kBatchBuckets);
    for (int p = 0; p < npairs; ++p) bucket_pairs[batch_bucket(batch_pad(pairs[p].n))].push_back(p);
    for (int b = 0; b < kBatchBuckets; ++b) {
        auto& bp = bucket_pairs[b];
        std::stable_sort(bp.begin(), bp.end(), [&](int x, int y) { return pairs[x].n > pairs[y].n; });
        std::vector<std::vector<int>> lists(kXcds);
        std::vector<double> work(kXcds, 0.0);
        for (int p : bp) {
            const int x = (int)(std::min_element(work.begin(), work.end()) - work.begin());
            const double np = batch_pad(pairs[p].n);
            work[x] += np * np * np * restarts;
            for (int r = 0; r < restarts; ++r) lists[x].push_back(p * restarts + r);
        }
        size_t len = 0;
        for (auto& l : lists) len = std::max(len, l.size());
        pl.bstart[b] = (int)pl.order.size();
        pl.bcount[b] = (int)(len * kXcds);
        for (size_t s = 0; s < len; ++s)
            for (int x = 0; x < kXcds; ++x) pl.order.push_back(s < lists[x].size() ? lists[x][s] : -1);
    }
    pl.total_blocks = (int)pl.order.size();
    size_t off = 0;
    pl.probs = off; off = al256(off + sizeof(BProb) * pl.nprob);
    pl.order_off = off; off = al256(off + sizeof(int) * std::max(pl.total_blocks, 1));
    pl.jobs = off; off = al256(off + sizeof(BPack) * npairs);
    pl.hist = off; off = al256(off + sizeof(goat_iter_record) * (size_t)pl.nprob * o.fw_max);
    pl.fwd = off; off = al256(off + sizeof(int) * pl.nprob);
    pl.score = off; off = al256(off + sizeof(double) * pl.nprob);
    for (int p = 0; p < npairs; ++p) pl.sum_n += pairs[p].n;
    pl.perms = off; off = al256(off + sizeof(int32_t) * (size_t)pl.sum_n * restarts);
    pl.offs = off; off = al256(off + sizeof(int) * pl.nprob);
    pl.lapst = off; off = al256(off + sizeof(int) * pl.nprob);
    pl.pairs_mat = off;
    for (int p = 0; p < npairs; ++p) {
        const size_t np = batch_pad(pairs[p].n), m = np * np * sizeof(float);
        pl.pair_off.push_back(off);
        off = al256(off + m * (gen ? 4 : 2));   // A0 (+A1), X1 (1 or 2 blocks)
    }
    pl.probs_mat = off;
    for (int k = 0; k < pl.nprob; ++k) {
        const size_t np = batch_pad(pairs[k / restarts].n), m = np * np * sizeof(float);
        pl.prob_off.push_back(off);
        off = al256(off + m * (gen ? 6 : 5));   // P, Q, GP, GQ, T (1 or 2 blocks)
    }
    pl.total = off;
    return pl;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace
}  // namespace goat

using namespace goat;

struct goat_batch {
    int npairs = 0, restarts = 0, nprob = 0, device = 0;
    goat_options opt;
    std::vector<goat_pair> pairs;
    Plan plan;
    char* ws = nullptr;
    std::vector<BProb> probs;
    BShape shapes[kBatchBuckets];
    int launches = 0;
    hipStream_t s0 = nullptr;
    hipStream_t sb[kBatchBuckets] = {nullptr};
    hipEvent_t ev_fork = nullptr, ev_in = nullptr, ev0 = nullptr, ev1 = nullptr;
    hipEvent_t ev_join[kBatchBuckets] = {nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool launched = false;
    void* hbuf = nullptr;   // pinned staging for the final matrices
    size_t hbuf_bytes = 0;
    long long lap_bids = 0; // device assignments of the last results call: bids summed

    ~goat_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipEvent_t e : {ev_fork, ev_in, ev0, ev1})
            if (e) (void)hipEventDestroy(e);
        for (int b = 0; b < kBatchBuckets; ++b) {
            if (ev_join[b]) (void)hipEventDestroy(ev_join[b]);
            if (sb[b]) (void)hipStreamDestroy(sb[b]);
        }
        if (s0) (void)hipStreamDestroy(s0);
        if (hbuf) (void)hipHostFree(hbuf);
    }
};

namespace {

#define B_HIP(call)                                                                  \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) {                                                      \
            ::goat::set_error(std::string(#call) + ": " + hipGetErrorString(e_));   \
            return GOAT_EHIP;                                                        \
        }                                                                            \
    } while (0)

// capture: pack, fork, one kernel per non-empty bucket, join
int build_graph(goat_batch& b) {
    const Plan& pl = b.plan;
    BArgs a{};
    a.probs = reinterpret_cast<const BProb*>(b.ws + pl.probs);
    a.eps_rel = b.opt.eps_rel;
    a.sk_tol = b.opt.sk_tol;
    a.fw_tol = b.opt.fw_tol;
    a.init_tol = kInitTol;
    a.sk_max = b.opt.sk_max;
    a.fw_max = b.opt.fw_max;
    a.stop_on_stall = b.opt.stop_on_stall;
    a.warm = b.opt.warm;
    a.init_max = kInitMax;
    int np_max = 32;
    for (auto& q : b.pairs) np_max = std::max(np_max, batch_pad(q.n));
    B_HIP(hipStreamBeginCapture(b.s0, hipStreamCaptureModeThreadLocal));
    int rc = batch_pack_launch(reinterpret_cast<const BPack*>(b.ws + pl.jobs), b.npairs, np_max, b.s0);
    b.launches = 1;
    if (rc == GOAT_OK) {
        hipError_t e = hipEventRecord(b.ev_fork, b.s0);
        for (int k = 0; k < kBatchBuckets && rc == GOAT_OK && e == hipSuccess; ++k) {
            if (pl.bcount[k] == 0) continue;
            e = hipStreamWaitEvent(b.sb[k], b.ev_fork, 0);
            if (e != hipSuccess) break;
            BArgs ak = a;
            ak.order = reinterpret_cast<const int*>(b.ws + pl.order_off) + pl.bstart[k];
            rc = batch_launch(b.shapes[k], kBucketMax[k], pl.bcount[k], ak, b.sb[k]);
            if (rc) break;
            ++b.launches;
            e = hipEventRecord(b.ev_join[k], b.sb[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(b.s0, b.ev_join[k], 0);
        }
        if (e != hipSuccess && rc == GOAT_OK) {
            set_error(std::string("goat_batch: capture: ") + hipGetErrorString(e));
            rc = GOAT_EHIP;
        }
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b.s0, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) {
        set_error(std::string("goat_batch: end capture: ") + hipGetErrorString(e));
        return GOAT_EHIP;
    }
    b.graph = g;
    B_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
    return GOAT_OK;
}

int create_impl(const goat_pair* pairs, int npairs, int restarts, const goat_options* opt, void* ws,
                size_t ws_bytes, const BShape* force, goat_batch** out) {
    if (!out) {
        set_error("goat_batch_create: null out");
        return GOAT_EINVAL;
    }
    *out = nullptr;
    int rc = validate(pairs, npairs, restarts, opt);
    if (rc) return rc;
    if (!ws) {
        set_error("goat_batch_create: null workspace");
        return GOAT_EINVAL;
    }
    auto bp = new (std::nothrow) goat_batch;
    if (!bp) {
        set_error("goat_batch_create: out of host memory");
        return GOAT_ENOMEM;
    }
    std::unique_ptr<goat_batch> b(bp);
    b->npairs = npairs;
    b->restarts = restarts;
    b->nprob = npairs * restarts;
    b->opt = *opt;
    b->pairs.assign(pairs, pairs + npairs);
    b->plan = make_plan(pairs, npairs, restarts, *opt);
    const Plan& pl = b->plan;
    if (ws_bytes < pl.total) {
        set_error("goat_batch_create: workspace too small");
        return GOAT_ENOMEM;
    }
    b->ws = static_cast<char*>(ws);
    B_HIP(hipGetDevice(&b->device));
    for (int k = 0; k < kBatchBuckets; ++k) b->shapes[k] = force ? force[k] : current_shape(k);
    const bool gen = general_of(*opt);
    // descriptors
    std::vector<BPack> jobs(npairs);
    for (int p = 0; p < npairs; ++p) {
        const size_t np = batch_pad(pairs[p].n), m = np * np;
        float* base = reinterpret_cast<float*>(b->ws + pl.pair_off[p]);
        BPack& j = jobs[p];
        j.n = pairs[p].n;
        j.np = (int)np;
        j.ld = pairs[p].ld;
        j.general = gen ? 1 : 0;
        j.A = pairs[p].A;
        j.B = pairs[p].B;
        j.A0 = base;
        j.A1 = gen ? base + m : nullptr;
        j.X1 = gen ? base + 2 * m : base + m;
    }
    b->probs.resize(b->nprob);
    std::vector<int> offs(b->nprob);
    int perm_off = 0;
    for (int k = 0; k < b->nprob; ++k) {
        const int p = k / restarts, r = k % restarts;
        const size_t np = batch_pad(pairs[p].n), m = np * np;
        float* base = reinterpret_cast<float*>(b->ws + pl.prob_off[k]);
        BProb& q = b->probs[k];
        q.n = pairs[p].n;
        q.np = (int)np;
        q.pair = p;
        q.restart = r;
        q.A0 = jobs[p].A0;
        q.A1 = jobs[p].A1;
        q.X1 = jobs[p].X1;
        q.U = pairs[p].U ? pairs[p].U + (size_t)r * pairs[p].n * pairs[p].ld : nullptr;
        q.ldu = pairs[p].ld;
        q.pad = 0;
        q.P = base;
        q.Q = base + m;
        q.GP = base + 2 * m;
        q.GQ = base + 3 * m;
        q.T = base + 4 * m;
        q.hist = reinterpret_cast<goat_iter_record*>(b->ws + pl.hist) + (size_t)k * opt->fw_max;
        q.fw_done = reinterpret_cast<int*>(b->ws + pl.fwd) + k;
        offs[k] = perm_off;
        perm_off += q.n;
    }
    B_HIP(hipStreamCreateWithFlags(&b->s0, hipStreamNonBlocking));
    for (int k = 0; k < kBatchBuckets; ++k) {
        B_HIP(hipStreamCreateWithFlags(&b->sb[k], hipStreamNonBlocking));
        B_HIP(hipEventCreateWithFlags(&b->ev_join[k], hipEventDisableTiming));
    }
    B_HIP(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    B_HIP(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    B_HIP(hipEventCreate(&b->ev0));
    B_HIP(hipEventCreate(&b->ev1));
    {
        // adjacency with a NaN or an infinity is refused up front (one flag
        // per pair in the assignment-status array, free until the results)
        int* bad_dev = reinterpret_cast<int*>(b->ws + pl.lapst);
        B_HIP(hipMemsetAsync(bad_dev, 0, sizeof(int) * npairs, b->s0));
        for (int p = 0; p < npairs; ++p) {
            rc = launch_check_finite(pairs[p].n, pairs[p].A, pairs[p].ld, bad_dev + p, b->s0);
            if (!rc) rc = launch_check_finite(pairs[p].n, pairs[p].B, pairs[p].ld, bad_dev + p, b->s0);
            if (rc) return rc;
        }
        std::vector<int> bad(npairs);
        B_HIP(hipMemcpyAsync(bad.data(), bad_dev, sizeof(int) * npairs, hipMemcpyDeviceToHost, b->s0));
        B_HIP(hipStreamSynchronize(b->s0));
        for (int p = 0; p < npairs; ++p)
            if (bad[p]) {
                set_error("goat_batch_create: pair " + std::to_string(p) + " has a non-finite entry");
                return GOAT_EINVAL;
            }
    }
    B_HIP(hipMemcpyAsync(b->ws + pl.probs, b->probs.data(), sizeof(BProb) * b->nprob, hipMemcpyHostToDevice, b->s0));
    if (pl.total_blocks > 0)
        B_HIP(hipMemcpyAsync(b->ws + pl.order_off, pl.order.data(), sizeof(int) * pl.total_blocks,
                             hipMemcpyHostToDevice, b->s0));
    B_HIP(hipMemcpyAsync(b->ws + pl.jobs, jobs.data(), sizeof(BPack) * npairs, hipMemcpyHostToDevice, b->s0));
    B_HIP(hipMemcpyAsync(b->ws + pl.offs, offs.data(), sizeof(int) * b->nprob, hipMemcpyHostToDevice, b->s0));
    // zero every problem matrix once (rows of Q past n are never written)
    rc = batch_fill_zero(reinterpret_cast<float*>(b->ws + pl.probs_mat), (pl.total - pl.probs_mat) / sizeof(float),
                         b->s0);
    if (rc) return rc;
    rc = batch_fill_zero(reinterpret_cast<float*>(b->ws + pl.hist),
                         sizeof(goat_iter_record) * (size_t)b->nprob * opt->fw_max / sizeof(float), b->s0);
    if (rc) return rc;
    B_HIP(hipStreamSynchronize(b->s0));
    rc = build_graph(*b);
    if (rc) return rc;
    *out = b.release();
    return GOAT_OK;
}

}  // namespace

extern "C" {

int goat_batch_workspace_size(const goat_pair* pairs, int npairs, int restarts, const goat_options* opt,
                              size_t* bytes) {
    if (!bytes) {
        set_error("goat_batch_workspace_size: null bytes");
        return GOAT_EINVAL;
    }
    int rc = validate(pairs, npairs, restarts, opt);
    if (rc) return rc;
    *bytes = make_plan(pairs, npairs, restarts, *opt).total;
    return GOAT_OK;
}

int goat_batch_create(const goat_pair* pairs, int npairs, int restarts, const goat_options* opt, void* ws,
                      size_t ws_bytes, goat_batch** out) {
    return create_impl(pairs, npairs, restarts, opt, ws, ws_bytes, nullptr, out);
}

int goat_batch_launch(goat_batch* b, void* stream) {
    if (!b) {
        set_error("goat_batch_launch: null batch");
        return GOAT_EINVAL;
    }
    hipStream_t us = static_cast<hipStream_t>(stream);
    // ordered after the caller's prior work, and the caller's later work after it
    B_HIP(hipEventRecord(b->ev_in, us));
    B_HIP(hipStreamWaitEvent(b->s0, b->ev_in, 0));
    B_HIP(hipEventRecord(b->ev0, b->s0));
    B_HIP(hipGraphLaunch(b->exec, b->s0));
    B_HIP(hipEventRecord(b->ev1, b->s0));
    B_HIP(hipStreamWaitEvent(us, b->ev1, 0));
    b->launched = true;
    return GOAT_OK;
}

// bids per problem before the device assignment reports GOAT_ENOTSUP
constexpr long long kBatchLapBudget = 4000000;

int goat_batch_results(goat_batch* b, int32_t* perm_host, double* score_host, int* best_host, double* all_score_host,
                       goat_iter_record* hist_host, int hist_cap, int* fw_iters_host, goat_batch_stats* stats_host) {
    if (!b || !b->launched) {
        set_error("goat_batch_results: batch not launched");
        return GOAT_EINVAL;
    }
    if (hist_host && hist_cap < 1) {
        set_error("goat_batch_results: hist_cap < 1");
        return GOAT_EINVAL;
    }
    const double t_start = now_ms();
    const Plan& pl = b->plan;
    B_HIP(hipEventSynchronize(b->ev1));
    float ms_graph = 0.0f;
    B_HIP(hipEventElapsedTime(&ms_graph, b->ev0, b->ev1));
    const int R = b->restarts, N = b->nprob, fwm = b->opt.fw_max;
    std::vector<int> fwd(N);
    std::vector<goat_iter_record> hist((size_t)N * fwm);
    B_HIP(hipMemcpy(fwd.data(), b->ws + pl.fwd, sizeof(int) * N, hipMemcpyDeviceToHost));
    B_HIP(hipMemcpy(hist.data(), b->ws + pl.hist, sizeof(goat_iter_record) * hist.size(), hipMemcpyDeviceToHost));

    // final assignment per problem on P_final (proj 0) or grad f(P_final)
    // (proj 1, equal to G_P by linearity); matrices staged through pinned
    // memory in chunks, assignments in parallel over problems
    const double t_lap = now_ms();
    std::vector<int32_t> perms((size_t)pl.sum_n * R);
    std::vector<size_t> poff(N);
    {
        size_t o = 0;
        for (int k = 0; k < N; ++k) {
            poff[k] = o;
            o += b->probs[k].n;
        }
    }
    if (b->opt.lap == 1) {
        // all assignments on the device, written into the batch's perm array
        int rc = batch_auction_launch(reinterpret_cast<const BProb*>(b->ws + pl.probs), N, b->opt.proj,
                                      reinterpret_cast<const int*>(b->ws + pl.offs),
                                      reinterpret_cast<int32_t*>(b->ws + pl.perms),
                                      reinterpret_cast<int*>(b->ws + pl.lapst), kBatchLapBudget, b->s0);
        if (rc) return rc;
        std::vector<int> st(N);
        B_HIP(hipMemcpyAsync(st.data(), b->ws + pl.lapst, sizeof(int) * N, hipMemcpyDeviceToHost, b->s0));
        B_HIP(hipMemcpyAsync(perms.data(), b->ws + pl.perms, sizeof(int32_t) * perms.size(), hipMemcpyDeviceToHost,
                             b->s0));
        B_HIP(hipStreamSynchronize(b->s0));
        b->lap_bids = 0;
        for (int k = 0; k < N; ++k) {
            if (st[k] >= 0) b->lap_bids += st[k];
        }
        for (int k = 0; k < N; ++k)
            if (st[k] < 0) {
                set_error("goat_batch_results: device assignment of problem " + std::to_string(k) +
                          (st[k] == GOAT_ENOTSUP ? " spent its bid budget" : " found a non-finite score"));
                return st[k];
            }
    }
    const size_t chunk_bytes = (size_t)64 << 20;
    if (b->opt.lap != 1 && !b->hbuf) {
        B_HIP(hipHostMalloc(&b->hbuf, chunk_bytes, hipHostMallocDefault));
        b->hbuf_bytes = chunk_bytes;
    }
    int status = GOAT_OK;
    std::string err_msg;
    for (int k0 = (b->opt.lap == 1 ? N : 0); k0 < N && status == GOAT_OK;) {
        size_t used = 0;
        int k1 = k0;
        std::vector<size_t> hoff;
        while (k1 < N) {
            const size_t need = (size_t)b->probs[k1].n * b->probs[k1].n * sizeof(float);
            if (used + need > b->hbuf_bytes && k1 > k0) break;
            hoff.push_back(used);
            used += need;
            ++k1;
        }
        for (int k = k0; k < k1; ++k) {
            const BProb& q = b->probs[k];
            const float* src = b->opt.proj == 1 ? q.GP : q.P;
            B_HIP(hipMemcpy2DAsync(static_cast<char*>(b->hbuf) + hoff[k - k0], (size_t)q.n * sizeof(float), src,
                                   (size_t)q.np * sizeof(float), (size_t)q.n * sizeof(float), q.n,
                                   hipMemcpyDeviceToHost, b->s0));
        }
        B_HIP(hipStreamSynchronize(b->s0));
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = k0; k < k1; ++k) {
            const int n = b->probs[k].n;
            const float* M = reinterpret_cast<const float*>(static_cast<char*>(b->hbuf) + hoff[k - k0]);
            std::vector<double> Md((size_t)n * n);
            for (size_t e = 0; e < Md.size(); ++e) Md[e] = M[e];
            const int rc = lap_max(n, Md.data(), n, perms.data() + poff[k]);
            if (rc) {
#pragma omp critical
                {
                    status = rc;
                    err_msg = "goat_batch_results: assignment of problem " + std::to_string(k) + " failed";
                }
            }
        }
        k0 = k1;
    }
    if (status) {
        set_error(err_msg);
        return status;
    }
    const double ms_lap = now_ms() - t_lap;
    if (b->opt.lap != 1)
        B_HIP(hipMemcpyAsync(b->ws + pl.perms, perms.data(), sizeof(int32_t) * perms.size(), hipMemcpyHostToDevice,
                             b->s0));
    int rc = batch_score_launch(reinterpret_cast<const BProb*>(b->ws + pl.probs), N,
                                reinterpret_cast<const int32_t*>(b->ws + pl.perms),
                                reinterpret_cast<const int*>(b->ws + pl.offs), reinterpret_cast<double*>(b->ws + pl.score),
                                b->s0);
    if (rc) return rc;
    std::vector<double> scores(N);
    B_HIP(hipMemcpyAsync(scores.data(), b->ws + pl.score, sizeof(double) * N, hipMemcpyDeviceToHost, b->s0));
    B_HIP(hipStreamSynchronize(b->s0));

    size_t pair_off = 0;
    for (int p = 0; p < b->npairs; ++p) {
        int best = 0;
        for (int r = 1; r < R; ++r)
            if (scores[(size_t)p * R + r] > scores[(size_t)p * R + best]) best = r;
        const int k = p * R + best, n = b->pairs[p].n;
        if (perm_host) std::memcpy(perm_host + pair_off, perms.data() + poff[k], sizeof(int32_t) * n);
        if (score_host) score_host[p] = scores[k];
        if (best_host) best_host[p] = best;
        pair_off += n;
    }
    if (all_score_host) std::memcpy(all_score_host, scores.data(), sizeof(double) * N);
    if (fw_iters_host) std::memcpy(fw_iters_host, fwd.data(), sizeof(int) * N);
    if (hist_host) {
        for (int k = 0; k < N; ++k)
            for (int f = 0; f < hist_cap; ++f) {
                goat_iter_record& dst = hist_host[(size_t)k * hist_cap + f];
                if (f < fwd[k] && f < fwm) dst = hist[(size_t)k * fwm + f];
                else std::memset(&dst, 0, sizeof(dst));
            }
    }
    if (stats_host) {
        goat_batch_stats st{};
        st.problems = N;
        for (int k = 0; k < N; ++k) {
            st.fw_iters_total += fwd[k];
            for (int f = 0; f < fwd[k] && f < fwm; ++f) {
                const goat_iter_record& r = hist[(size_t)k * fwm + f];
                st.sk_iters_total += r.sk_iters;
                if (r.sk_iters >= b->opt.sk_max) ++st.sk_capped;
            }
        }
        st.launches = b->launches;
        st.ms_graph = ms_graph;
        st.ms_lap = ms_lap;
        st.ms_total = now_ms() - t_start;
        st.lap_bids = b->opt.lap == 1 ? b->lap_bids : 0;
        *stats_host = st;
    }
    return GOAT_OK;
}

int goat_batch_get_P(goat_batch* b, int pair, int restart, float* out, int ld, void* stream) {
    if (!b || pair < 0 || pair >= b->npairs || restart < 0 || restart >= b->restarts || !out) {
        set_error("goat_batch_get_P: bad arguments");
        return GOAT_EINVAL;
    }
    const BProb& q = b->probs[(size_t)pair * b->restarts + restart];
    if (ld < q.n) {
        set_error("goat_batch_get_P: ld < n");
        return GOAT_EINVAL;
    }
    B_HIP(hipMemcpy2DAsync(out, (size_t)ld * sizeof(float), q.P, (size_t)q.np * sizeof(float),
                           (size_t)q.n * sizeof(float), q.n, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
    return GOAT_OK;
}

void goat_batch_destroy(goat_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->s0);
    delete b;
}

size_t goat_random_init_workspace_size(int n) {
    if (n <= GOAT_BATCH_NMAX) return 0;
    const Layout L = make_layout(n, GOAT_PREC_FP32, 1);
    return small_bytes(L) + (size_t)L.np * L.np * sizeof(float);
}

// Up to GOAT_BATCH_NMAX one workgroup scales U in place of LDS. Above, the
// Sinkhorn-Knopp scaling of U is the entropic plan of the cost ln U at
// eps = 1 (Q = diag(e^f) U diag(e^g)), so the LOT sweeps do it: ln U goes
// into the workspace, the sweeps run with the same stop rule (row sums of
// K within tol), and K is written into P before P = (J + K) / 2.
int goat_random_init(int n, const float* U, int ldu, float* P, int ldp, float tol, int max_iter, int* iters_dev,
                     float* err_dev, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (n < 1 || !U || !P || ldu < n || ldp < n || !(tol >= 0.0f) || !std::isfinite(tol) || max_iter < 1) {
        set_error("goat_random_init: bad arguments");
        return GOAT_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n <= GOAT_BATCH_NMAX) return random_init_launch(n, U, ldu, P, ldp, tol, max_iter, iters_dev, err_dev, s);
    if (!ws || ws_bytes < goat_random_init_workspace_size(n)) {
        set_error("goat_random_init: workspace smaller than goat_random_init_workspace_size(n)");
        return GOAT_ENOMEM;
    }
    const Layout L = make_layout(n, GOAT_PREC_FP32, 1);
    Ptrs p = make_ptrs(L, ws);
    float* one = reinterpret_cast<float*>(p.scal + 20);
    int rc = launch_log_pad(n, U, ldu, p.P, L.np, one, s);
    if (!rc) rc = sk_prepare(n, p.P, L.np, one, 0.0f, nullptr, nullptr, tol, p.sk, p.fscal, p.red, s);
    for (int k = 0; !rc && k < max_iter; ++k) rc = sk_iterate(n, L.np, p.P, L.np, p.sk, k == 0, k >= 1, k, s);
    if (!rc)
        rc = sk_finalize(n, L.np, p.P, L.np, p.sk, P, ldp, nullptr, nullptr, nullptr, nullptr, iters_dev, err_dev,
                         nullptr, p.red, s);
    if (!rc) rc = launch_half_bary(n, P, ldp, s);
    return rc;
}

// Each bucket up to n_max: a synthetic batch of 64 pairs x 8 starts at the
// bucket's largest size (fixed work: 1 FW iteration, 16 Sinkhorn sweeps,
// tolerance 0), every feasible shape timed over reps graph launches.
int goat_tune(int n_max, int reps, void* stream) {
    if (n_max < 1 || n_max > GOAT_BATCH_NMAX || reps < 1) {
        set_error("goat_tune: bad arguments");
        return GOAT_EINVAL;
    }
    (void)stream;
    int dev = 0;
    B_HIP(hipGetDevice(&dev));
    if (dev >= kMaxDevices) {
        set_error("goat_tune: device index too large");
        return GOAT_ENOTSUP;
    }
    goat_options o;
    goat_default_options(&o);
    o.fw_max = 1;
    o.sk_max = 16;
    o.sk_tol = 0.0f;
    o.stop_on_stall = 0;
    const int npairs = 64, R = 8;
    for (int bk = 0; bk < kBatchBuckets; ++bk) {
        const int lo = bk == 0 ? 1 : kBucketMax[bk - 1] + 1;
        if (lo > n_max) break;
        const int n = kBucketMax[bk];
        float* AB = nullptr;
        B_HIP(hipMalloc(&AB, (size_t)2 * n * n * sizeof(float)));
        std::unique_ptr<float, void (*)(float*)> ab_guard(AB, [](float* p) { (void)hipFree(p); });
        int rc = batch_synth_launch(AB, AB + (size_t)n * n, n, n, 0x9e3779b9u + bk, nullptr);
        if (rc) return rc;
        B_HIP(hipStreamSynchronize(nullptr));
        std::vector<goat_pair> pairs(npairs);
        for (auto& q : pairs) q = goat_pair{n, n, AB, AB + (size_t)n * n, nullptr};
        const size_t bytes = make_plan(pairs.data(), npairs, R, o).total;
        void* ws = nullptr;
        B_HIP(hipMalloc(&ws, bytes));
        std::unique_ptr<void, void (*)(void*)> ws_guard(ws, [](void* p) { (void)hipFree(p); });
        BShape best = default_shape(bk);
        double best_ms = 1e300;
        for (int L : {16, 32, 64})
            for (int w : {4, 8}) {
                const BShape s = shape_for(L, w, n);
                if (!batch_shape_ok(s, n)) continue;
                BShape force[kBatchBuckets];
                for (int k = 0; k < kBatchBuckets; ++k) force[k] = k == bk ? s : default_shape(k);
                goat_batch* b = nullptr;
                rc = create_impl(pairs.data(), npairs, R, &o, ws, bytes, force, &b);
                if (rc) return rc;
                std::unique_ptr<goat_batch, void (*)(goat_batch*)> bg(b, goat_batch_destroy);
                rc = goat_batch_launch(b, nullptr);   // warm-up
                if (rc) return rc;
                B_HIP(hipEventSynchronize(b->ev1));
                double ms = 0.0;
                for (int r = 0; r < reps; ++r) {
                    rc = goat_batch_launch(b, nullptr);
                    if (rc) return rc;
                    B_HIP(hipEventSynchronize(b->ev1));
                    float m = 0.0f;
                    B_HIP(hipEventElapsedTime(&m, b->ev0, b->ev1));
                    ms += m;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best = s;
                }
            }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[dev][bk] = best;
        g_has_tuned[dev][bk] = true;
    }
    return GOAT_OK;
}

int goat_tune_get(int n, int* lanes_per_row, int* waves) {
    if (n < 1 || n > GOAT_BATCH_NMAX) {
        set_error("goat_tune_get: bad n");
        return GOAT_EINVAL;
    }
    const BShape s = current_shape(batch_bucket(batch_pad(n)));
    if (lanes_per_row) *lanes_per_row = s.L;
    if (waves) *waves = s.waves;
    return GOAT_OK;
}

}  // extern "C"
