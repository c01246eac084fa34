// GOAT end to end (Alg. 3): initialisation, Frank-Wolfe iterations on the
// device and the final host assignment, exposed as goat_solve and as the
// begin / steps / finish triple used to time a fixed number of iterations.
//
// Per iteration, on the caller's stream:
//   1. eps = eps_rel * max|G_P| (the max comes from the previous update)
//   2. LOT: Sinkhorn sweeps on G_P, polled every check_every iterations for
//      the device-side convergence flag; then Q (and its bf16 split)
//   3. G_Q = grad f(Q); by linearity grad f(P + t(Q-P)) = G_P + t(G_Q - G_P),
//      so one gradient product per iteration suffices
//   4. float64 traces -> exact step t (Alg. 3 step 3)
//   5. P <- P + t(Q - P), G_P <- G_P + t(G_Q - G_P), next max|G_P|
// The only host synchronisation per iteration reads back the step scalars.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace goat {

struct Run {
    Layout L;
    Ptrs p;
    GradOps ops;
    goat_options opt;
    hipStream_t s = nullptr;
    const float* A = nullptr;
    const float* B = nullptr;
    int ld = 0;
    const float* lin = nullptr;  // seeded problems: linear term C (np x np), added to every gradient
    int fw = 0;                 // iterations done
    bool stalled = false;
    bool operands_spent = false;  // the device assignment reused G_Q and the packed operands
    double last_ls[8] = {0};
    goat_stats st{};
    void* hbuf = nullptr;       // pinned host scratch
    hipEvent_t ev_poll[2] = {nullptr, nullptr};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::chrono::steady_clock::time_point wall0;
    double loop_ms = 0.0;

    ~Run() {
        if (hbuf) (void)hipHostFree(hbuf);
        for (hipEvent_t e : {ev_poll[0], ev_poll[1], ev0, ev1})
            if (e) (void)hipEventDestroy(e);
    }
};

// Sinkhorn sweeps on G_P: one launch pair per iteration, the device-side
// convergence flag polled every check_every iterations (two chunks in
// flight, so the device never waits for the host).
static int run_sinkhorn_polled(Run& r) {
    const int n = r.L.n, np = r.L.np;
    Ptrs& p = r.p;
    int rc;
    rc = sk_iterate(n, np, p.GP, np, p.sk, 1, 0, 0, r.s);
    if (rc) return rc;
    const int check_every = r.opt.check_every > 0 ? r.opt.check_every : 16;
    // The kernels that set the stop flag also store it in pinned host memory
    // (p.sk.hdone; sk_prepare's init kernel resets it in stream order). After
    // each chunk of sweeps an event is recorded, and the host waits for the
    // previous chunk's event and reads the flag, so one chunk is always
    // queued ahead and no copy enters the stream. A flag read late only
    // costs launches that exit at once.
    const volatile int* hflag = p.sk.hdone;
    int k = 1, chunk = 0;
    bool stop = false;
    while (k < r.opt.sk_max && !stop) {
        const int m = std::min(check_every, r.opt.sk_max - k);
        for (int q = 0; q < m; ++q) {
            rc = sk_iterate(n, np, p.GP, np, p.sk, 0, 1, k + q, r.s);
            if (rc) return rc;
        }
        k += m;
        const int slot = chunk & 1;
        GOAT_HIP(hipEventRecord(r.ev_poll[slot], r.s));
        if (chunk >= 1) {
            GOAT_HIP(hipEventSynchronize(r.ev_poll[slot ^ 1]));
            if (hflag && *hflag) stop = true;
        }
        ++chunk;
    }
    return GOAT_OK;
}

static int run_sinkhorn(Run& r) {
    const int n = r.L.n, np = r.L.np;
    const bool bf = r.opt.prec == GOAT_PREC_BF16X2 || r.opt.prec == GOAT_PREC_BF16X3;
    Ptrs& p = r.p;
    // warm: 1 previous iteration's column potentials; 2 the network every
    // iteration; 3 the network on the first iteration, then as 1
    const bool prev = (r.opt.warm == 1 || r.opt.warm == 3) && r.fw > 0;
    const bool net = r.opt.mlp_params && (r.opt.warm == 2 || (r.opt.warm == 3 && r.fw == 0));
    // eps from the max|G_P| that the previous update (or the start) left in fscal[0]
    int rc = sk_prepare(n, p.GP, np, nullptr, r.opt.eps_rel, p.fscal, prev ? p.g_prev : nullptr, r.opt.sk_tol,
                        p.sk, p.fscal, p.red, r.s);
    if (!rc && p.sk.g24) rc = sk_pack_g24(n, np, p.GP, np, p.fscal, p.sk, r.s);
    if (rc) return rc;
    if (net) {
        rc = mlp_features(n, np, p.GP, np, &p.sk.ctrl->eps, p.sk.colpart, p.feat, r.s);
        if (!rc) rc = mlp_forward(n, p.feat, r.opt.mlp_params, p.pred, r.s);
        if (!rc) rc = warm_seed(n, p.pred, p.sk.ctrl, p.sk.vg, p.sk.vs, r.s);
        if (rc) return rc;
    }
    rc = run_sinkhorn_polled(r);
    if (rc) return rc;
    int* it_dev = reinterpret_cast<int*>(p.scal + 8);
    float* err_dev = reinterpret_cast<float*>(p.scal + 9);
    return sk_finalize(n, np, p.GP, np, p.sk, p.Q, np, bf ? static_cast<uint16_t*>(p.P_hi) : nullptr,
                       bf ? static_cast<uint16_t*>(p.P_lo) : nullptr, nullptr, p.g_prev, it_dev, err_dev,
                       err_dev + 1, p.red, r.s);
}

static int run_step(Run& r, goat_iter_record* rec) {
    const int n = r.L.n, np = r.L.np;
    Ptrs& p = r.p;
    int rc = run_sinkhorn(r);
    if (rc) return rc;
    if (r.opt.prec == GOAT_PREC_FP32) r.ops.P_hi = p.Q;
    if (r.opt.prec == GOAT_PREC_FP8) rc = prep_fp8_operand(r.L, r.ops, p.Q, np, r.s);
    if (!rc) rc = grad_packed(r.L, r.ops, p.GQ, np, np, r.s);
    if (!rc && r.lin) rc = launch_add_mat(n, p.GQ, r.lin, np, r.s);
    if (rc) return rc;
    rc = launch_traces(n, p.P, p.Q, p.GP, p.GQ, np, p.red, p.scal, r.s, r.lin);
    if (!rc) rc = launch_fw_update(n, p.P, p.Q, p.GP, p.GQ, np, p.scal, p.fscal + 16, p.fscal, r.s);
    if (rc) return rc;
    GOAT_HIP(hipMemcpyAsync(r.hbuf, p.scal, 80, hipMemcpyDeviceToHost, r.s));
    GOAT_HIP(hipStreamSynchronize(r.s));
    const char* hb = static_cast<const char*>(r.hbuf);
    double ls[8];
    std::memcpy(ls, hb, sizeof(ls));
    int skit;
    float skerr, eps;
    std::memcpy(&skit, hb + 64, 4);
    std::memcpy(&skerr, hb + 72, 4);
    std::memcpy(&eps, hb + 76, 4);
    std::memcpy(r.last_ls, ls, sizeof(ls));
    r.st.sk_iters_total += skit;
    if (skit >= r.opt.sk_max) r.st.sk_capped += 1;
    if (rec) {
        rec->fP = ls[0]; rec->fQ = ls[1]; rec->c = ls[2]; rec->a = ls[3]; rec->b = ls[4];
        rec->t = ls[5]; rec->dist2 = ls[6]; rec->eps = eps; rec->sk_err = skerr; rec->sk_iters = skit;
        rec->pad = 0;
    }
    r.fw += 1;
    const double t = ls[5];
    const double delta = t * std::sqrt(ls[6]) / std::sqrt((double)n);
    if ((t == 0.0 && r.opt.stop_on_stall) || (r.opt.fw_tol > 0.0f && delta < r.opt.fw_tol)) r.stalled = true;
    return GOAT_OK;
}

}  // namespace goat

using namespace goat;

struct goat_run {
    Run r;
};

extern "C" {

static int run_begin_impl(int n, const float* A, const float* B, int ld, const float* P0,
                          const goat_options* opt_in, void* ws, size_t ws_bytes, void* stream, const float* lin,
                          goat_run** run_out);

int goat_run_begin(int n, const float* A, const float* B, int ld, const float* P0, const goat_options* opt_in,
                   void* ws, size_t ws_bytes, void* stream, goat_run** run_out) {
    return run_begin_impl(n, A, B, ld, P0, opt_in, ws, ws_bytes, stream, nullptr, run_out);
}

}  // extern "C"

// lin: optional linear term (np x np, zero padded) of a seeded problem
static int run_begin_impl(int n, const float* A, const float* B, int ld, const float* P0,
                          const goat_options* opt_in, void* ws, size_t ws_bytes, void* stream, const float* lin,
                          goat_run** run_out) {
    clear_error();
    GOAT_CHECK_ARG(run_out, "null run pointer");
    *run_out = nullptr;
    goat_options opt;
    if (opt_in) opt = *opt_in; else goat_default_options(&opt);
    GOAT_CHECK_ARG(n >= 1, "n < 1");
    GOAT_CHECK_ARG(A && B && ws, "null pointer");
    GOAT_CHECK_ARG(ld >= n, "leading dimension < n");
    GOAT_CHECK_ARG(opt.prec >= GOAT_PREC_FP32 && opt.prec <= GOAT_PREC_FP8, "unknown precision");
    GOAT_CHECK_ARG(std::isfinite(opt.eps_rel) && opt.eps_rel > 0.0f, "eps_rel must be > 0");
    GOAT_CHECK_ARG(std::isfinite(opt.sk_tol) && opt.sk_tol >= 0.0f, "bad sk_tol");
    GOAT_CHECK_ARG(opt.sk_max >= 1 && opt.fw_max >= 1, "sk_max and fw_max must be >= 1");
    GOAT_CHECK_ARG(std::isfinite(opt.fw_tol) && opt.fw_tol >= 0.0f, "bad fw_tol");
    GOAT_CHECK_ARG(opt.warm >= 0 && opt.warm <= 3, "unknown warm-start mode");
    GOAT_CHECK_ARG(opt.lap == 0 || opt.lap == 1, "unknown assignment mode");
    GOAT_CHECK_ARG(opt.warm < 2 || opt.mlp_params, "warm-start network requested without parameters");
    GOAT_CHECK_ARG(opt.sk_g24 == 0 || (opt.sk_g24 == 1 && opt.prec != GOAT_PREC_FP32),
                   "sk_g24 must be 0, or 1 with a mixed precision (its workspace holds the 24-bit copy)");
    const Layout L = make_layout(n, opt.prec, opt.symmetric);
    if (ws_bytes < L.total) { set_error("goat_run_begin: workspace too small"); return GOAT_ENOMEM; }

    goat_run* h = new (std::nothrow) goat_run();
    if (!h) { set_error("goat_run_begin: out of host memory"); return GOAT_ENOMEM; }
    Run& r = h->r;
    r.wall0 = std::chrono::steady_clock::now();
    r.L = L;
    r.p = make_ptrs(L, ws);
    if (opt.sk_g24) {
        r.p.sk.g24 = reinterpret_cast<const uint32_t*>(static_cast<char*>(ws) + L.g24);
        r.p.sk.ld24 = 3 * (L.np / 4);
    }
    r.opt = opt;
    r.s = static_cast<hipStream_t>(stream);
    r.A = A;
    r.B = B;
    r.ld = ld;
    r.lin = lin;
    auto fail = [&](int rc) { delete h; return rc; };
#define RUN_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            set_error(std::string(#call) + ": " + hipGetErrorString(e_));                \
            return fail(GOAT_EHIP);                                                      \
        }                                                                                \
    } while (0)
    RUN_HIP(hipHostMalloc(&r.hbuf, 256, hipHostMallocDefault));
    // the Sinkhorn stop flag, stored by the device (see run_sinkhorn_polled)
    r.p.sk.hdone = reinterpret_cast<int*>(static_cast<char*>(r.hbuf) + 128);
    for (hipEvent_t* e : {&r.ev_poll[0], &r.ev_poll[1], &r.ev0, &r.ev1}) RUN_HIP(hipEventCreate(e));
    Ptrs& p = r.p;
    const int np = L.np;
    RUN_HIP(hipMemsetAsync(ws, 0, L.total, r.s));
    // non-finite adjacency entries are refused up front (the reduction
    // partials are zero here and free until the first iteration)
    int* bad_dev = reinterpret_cast<int*>(p.red);
    int rc = launch_check_finite(n, A, ld, bad_dev, r.s);
    if (!rc) rc = launch_check_finite(n, B, ld, bad_dev, r.s);
    if (rc) return fail(rc);
    RUN_HIP(hipMemcpyAsync(r.hbuf, bad_dev, sizeof(int), hipMemcpyDeviceToHost, r.s));
    RUN_HIP(hipStreamSynchronize(r.s));
    if (*static_cast<int*>(r.hbuf) != 0) {
        set_error("goat_run_begin: A or B has a non-finite entry");
        return fail(GOAT_EINVAL);
    }
    rc = pack_graph(L, A, ld, p.A_hi, p.A_lo, r.s);
    if (!rc) rc = pack_graph(L, B, ld, p.B_hi, p.B_lo, r.s);
    if (!rc) rc = P0 ? launch_copy_pad(n, P0, ld, p.P, np, np, r.s) : launch_fill_barycenter(n, np, p.P, r.s);
    if (rc) return fail(rc);
    r.ops = grad_ops(p);
    if (opt.prec == GOAT_PREC_FP8) {
        rc = prep_fp8_operand(L, r.ops, p.P, np, r.s);
        if (rc) return fail(rc);
    } else if (opt.prec != GOAT_PREC_FP32) {
        rc = launch_split_bf16(n, np, p.P, np, static_cast<uint16_t*>(p.P_hi), static_cast<uint16_t*>(p.P_lo), r.s);
        if (rc) return fail(rc);
    } else {
        r.ops.P_hi = p.P;
    }
    rc = grad_packed(L, r.ops, p.GP, np, np, r.s);
    if (!rc && lin) rc = launch_add_mat(n, p.GP, lin, np, r.s);
    if (!rc) rc = launch_absmax(n, p.GP, np, p.fscal + 16, p.fscal, r.s);
    if (rc) return fail(rc);
    RUN_HIP(hipStreamSynchronize(r.s));
#undef RUN_HIP
    *run_out = h;
    return GOAT_OK;
}

extern "C" {

int goat_run_steps(goat_run* h, int k, goat_iter_record* hist_host, int hist_cap, int* done_out) {
    clear_error();
    GOAT_CHECK_ARG(h, "null run");
    GOAT_CHECK_ARG(k >= 0, "k < 0");
    GOAT_CHECK_ARG(hist_cap >= 0 && (hist_cap == 0 || hist_host), "bad history buffer");
    Run& r = h->r;
    GOAT_CHECK_ARG(!r.operands_spent, "the device assignment of goat_run_finish reused this run's operands");
    int done = 0;
    GOAT_HIP(hipEventRecord(r.ev0, r.s));
    while (done < k && !r.stalled) {
        int rc = run_step(r, done < hist_cap ? &hist_host[done] : nullptr);
        if (rc) return rc;
        ++done;
    }
    GOAT_HIP(hipEventRecord(r.ev1, r.s));
    GOAT_HIP(hipEventSynchronize(r.ev1));
    float ms = 0.0f;
    GOAT_HIP(hipEventElapsedTime(&ms, r.ev0, r.ev1));
    r.loop_ms += ms;
    if (done_out) *done_out = done;
    return GOAT_OK;
}

int goat_run_finish(goat_run* h, int32_t* perm_host, goat_stats* stats_host, float* P_out, int ldp) {
    clear_error();
    GOAT_CHECK_ARG(h && perm_host, "null pointer");
    Run& r = h->r;
    const int n = r.L.n, np = r.L.np;
    GOAT_CHECK_ARG(!P_out || ldp >= n, "leading dimension < n");
    Ptrs& p = r.p;
    r.st.fw_iters = r.fw;
    r.st.ms_loop = r.loop_ms;
    const double t = r.last_ls[5];
    r.st.f_final = r.fw ? r.last_ls[0] + r.last_ls[4] * t + r.last_ls[3] * t * t : 0.0;
    if (P_out)
        GOAT_HIP(hipMemcpy2DAsync(P_out, (size_t)ldp * 4, p.P, (size_t)np * 4, (size_t)n * 4, n,
                                  hipMemcpyDeviceToDevice, r.s));
    if (r.fw == 0) {
        // no iteration ran: f(P0) = <P0, grad f(P0)>/2 is not tracked; report 0
        r.st.f_final = 0.0;
    }
    // final projection (Alg. 3 return line)
    const float* src = r.opt.proj ? p.GP : p.P;
    const auto lap0 = std::chrono::steady_clock::now();
    bool on_device = false;
    if (r.opt.lap == 1) {
        // the direction buffer Q is free once the loop has ended; errors of
        // the device assignment (round cap, bid range) are returned as they
        // are: the host solver runs only when the caller asks for it (lap 0)
        // G_Q and the packed operands after it are free once the loop has
        // ended (the score uses the caller's A and B): room for the
        // precomputed scores; else the direction buffer Q alone
        void* aws = p.GQ;
        size_t aws_bytes = r.L.total - r.L.GQ;
        if (aws_bytes < auction_ws_bytes_fast(n)) {
            aws = p.Q;
            aws_bytes = (size_t)np * np * 4;
        } else {
            r.operands_spent = true;
        }
        if (auction_ws_bytes(n) > aws_bytes) {
            set_error("goat_run_finish: workspace too small for the device assignment");
            return GOAT_ENOMEM;
        }
        int rc = auction_lap(n, src, np, p.perm_dev, aws, aws_bytes, 20000000ll, nullptr, r.s);
        if (rc) return rc;
        on_device = true;
        GOAT_HIP(hipMemcpyAsync(perm_host, p.perm_dev, (size_t)n * 4, hipMemcpyDeviceToHost, r.s));
    } else {
        std::vector<float> hm((size_t)n * n);
        GOAT_HIP(hipMemcpy2DAsync(hm.data(), (size_t)n * 4, src, (size_t)np * 4, (size_t)n * 4, n,
                                  hipMemcpyDeviceToHost, r.s));
        GOAT_HIP(hipStreamSynchronize(r.s));
        std::vector<double> md(hm.begin(), hm.end());
        std::vector<float>().swap(hm);
        int rc = lap_max(n, md.data(), n, perm_host);
        if (rc) return rc;
        GOAT_HIP(hipMemcpyAsync(p.perm_dev, perm_host, (size_t)n * 4, hipMemcpyHostToDevice, r.s));
    }
    GOAT_HIP(hipStreamSynchronize(r.s));
    r.st.lap_device = on_device ? 1 : 0;
    r.st.ms_lap = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - lap0).count();
    int rc = launch_score(n, r.A, r.B, r.ld, p.perm_dev, p.red, p.scal + 10, r.s);
    if (rc) return rc;
    GOAT_HIP(hipMemcpyAsync(r.hbuf, p.scal + 10, 8, hipMemcpyDeviceToHost, r.s));
    GOAT_HIP(hipStreamSynchronize(r.s));
    std::memcpy(&r.st.score, r.hbuf, 8);
    r.st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - r.wall0).count();
    if (stats_host) *stats_host = r.st;
    return GOAT_OK;
}

int goat_run_gradient(goat_run* h, float* G_out, int ldg) {
    clear_error();
    GOAT_CHECK_ARG(h && G_out, "null pointer");
    Run& r = h->r;
    const int n = r.L.n, np = r.L.np;
    GOAT_CHECK_ARG(ldg >= n, "leading dimension < n");
    GOAT_HIP(hipMemcpy2DAsync(G_out, (size_t)ldg * 4, r.p.GP, (size_t)np * 4, (size_t)n * 4, n,
                              hipMemcpyDeviceToDevice, r.s));
    GOAT_HIP(hipStreamSynchronize(r.s));
    return GOAT_OK;
}

int goat_run_direction(goat_run* h, float* Q_out, int ldq) {
    clear_error();
    GOAT_CHECK_ARG(h && Q_out, "null pointer");
    Run& r = h->r;
    const int n = r.L.n, np = r.L.np;
    GOAT_CHECK_ARG(ldq >= n, "leading dimension < n");
    GOAT_CHECK_ARG(r.fw > 0, "no iteration has run yet");
    GOAT_CHECK_ARG(!r.operands_spent, "the device assignment has reused the run's buffers");
    GOAT_HIP(hipMemcpy2DAsync(Q_out, (size_t)ldq * 4, r.p.Q, (size_t)np * 4, (size_t)n * 4, n,
                              hipMemcpyDeviceToDevice, r.s));
    GOAT_HIP(hipStreamSynchronize(r.s));
    return GOAT_OK;
}

int goat_run_set_sinkhorn(goat_run* h, int sk_max, float sk_tol) {
    clear_error();
    GOAT_CHECK_ARG(h, "null run");
    GOAT_CHECK_ARG(sk_max >= 1, "sk_max must be >= 1");
    GOAT_CHECK_ARG(std::isfinite(sk_tol) && sk_tol >= 0.0f, "bad sk_tol");
    h->r.opt.sk_max = sk_max;
    h->r.opt.sk_tol = sk_tol;
    return GOAT_OK;
}

void goat_run_free(goat_run* h) { delete h; }

// ---------------------------------------------------------------- seeded, unequal sizes

// Workspace of a seeded problem: the inner (non-seed) solver's layout, then
// the arranged graphs (n x n), the linear term C (kp x kp), the four packed
// seed blocks (kp x mp), the vertex orders and the full assignment.
struct SeededPlan {
    int n, m, k, kp, mp;
    size_t inner, arrA, arrB, lin, x1, z1, x2, z2, ordA, ordB, pos, total;
};

static SeededPlan seeded_plan(int nA, int nB, int m, int prec, int symmetric) {
    SeededPlan sp{};
    sp.n = std::max(nA, nB);
    sp.m = m;
    sp.k = sp.n - m;
    const int kk = std::max(sp.k, 1);
    sp.kp = pad_n(kk);
    sp.mp = std::max(16, (m + 15) / 16 * 16);
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    size_t o = al(make_layout(kk, prec, symmetric).total);
    sp.inner = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = al(o + bytes); return at; };
    const size_t nn = (size_t)sp.n * sp.n * 4;
    sp.arrA = take(nn);
    sp.arrB = take(nn);
    sp.lin = take((size_t)sp.kp * sp.kp * 4);
    const size_t rect = (size_t)sp.kp * sp.mp * 4;
    sp.x1 = take(rect);
    sp.z1 = take(rect);
    sp.x2 = take(rect);
    sp.z2 = take(rect);
    sp.ordA = take((size_t)sp.n * 4);
    sp.ordB = take((size_t)sp.n * 4);
    sp.pos = take((size_t)sp.n * 4);
    sp.total = o;
    return sp;
}

size_t goat_seeded_workspace_size(int nA, int nB, int m, int prec, int symmetric) {
    if (nA < 1 || nB < 1 || m < 0 || m > std::min(nA, nB) || prec < GOAT_PREC_FP32 || prec > GOAT_PREC_FP8)
        return 0;
    return seeded_plan(nA, nB, m, prec, symmetric).total;
}

int goat_solve_seeded(int nA, const float* A, int lda, int nB, const float* B, int ldb, int m,
                      const int32_t* seeds_A, const int32_t* seeds_B, int pad, const goat_options* opt,
                      int32_t* perm_host, goat_stats* stats_host, goat_iter_record* hist_host, int hist_cap,
                      void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    GOAT_CHECK_ARG(nA >= 1 && nB >= 1, "graph size < 1");
    GOAT_CHECK_ARG(A && B && ws && perm_host, "null pointer");
    GOAT_CHECK_ARG(lda >= nA && ldb >= nB, "leading dimension < n");
    GOAT_CHECK_ARG(m >= 0 && m <= std::min(nA, nB) && (m == 0 || (seeds_A && seeds_B)), "bad seed count");
    GOAT_CHECK_ARG(pad == 0 || pad == 1, "pad must be 0 (naive) or 1 (adopted)");
    GOAT_CHECK_ARG(hist_cap >= 0 && (hist_cap == 0 || hist_host), "bad history buffer");
    goat_options o;
    if (opt) o = *opt; else goat_default_options(&o);
    const SeededPlan sp = seeded_plan(nA, nB, m, o.prec, o.symmetric);
    if (ws_bytes < sp.total) { set_error("goat_solve_seeded: workspace too small"); return GOAT_ENOMEM; }
    // vertex orders: seeds, then the other vertices ascending, then dummies
    const int n = sp.n, k = sp.k;
    std::vector<int> ordA, ordB;
    for (int pass = 0; pass < 2; ++pass) {
        const int nx = pass ? nB : nA;
        const int32_t* seeds = pass ? seeds_B : seeds_A;
        std::vector<char> used(nx, 0);
        std::vector<int>& ord = pass ? ordB : ordA;
        for (int i = 0; i < m; ++i) {
            const int v = seeds[i];
            if (v < 0 || v >= nx || used[v]) {
                set_error("goat_solve_seeded: seeds must be distinct vertices of their graph");
                return GOAT_EINVAL;
            }
            used[v] = 1;
            ord.push_back(v);
        }
        for (int v = 0; v < nx; ++v)
            if (!used[v]) ord.push_back(v);
        while ((int)ord.size() < n) ord.push_back(-1);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* b = static_cast<char*>(ws);
    float* arrA = reinterpret_cast<float*>(b + sp.arrA);
    float* arrB = reinterpret_cast<float*>(b + sp.arrB);
    float* lin = reinterpret_cast<float*>(b + sp.lin);
    int* dA = reinterpret_cast<int*>(b + sp.ordA);
    int* dB = reinterpret_cast<int*>(b + sp.ordB);
    GOAT_HIP(hipMemcpyAsync(dA, ordA.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    GOAT_HIP(hipMemcpyAsync(dB, ordB.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    int rc = launch_arrange(n, A, lda, dA, pad, arrA, n, s);
    if (!rc) rc = launch_arrange(n, B, ldb, dB, pad, arrB, n, s);
    if (rc) return rc;
    std::vector<int> pos(n);
    for (int i = 0; i < m; ++i) pos[i] = i;
    goat_stats st{};
    if (k > 0) {
        // C = A21 B21^T + A12^T B12 on the fp32 matrix cores (zero without seeds)
        GOAT_HIP(hipMemsetAsync(lin, 0, (size_t)sp.kp * sp.kp * 4, s));
        if (m > 0) {
            float* x1 = reinterpret_cast<float*>(b + sp.x1);
            float* z1 = reinterpret_cast<float*>(b + sp.z1);
            float* x2 = reinterpret_cast<float*>(b + sp.x2);
            float* z2 = reinterpret_cast<float*>(b + sp.z2);
            rc = launch_pack_rect(arrA + (size_t)m * n, n, k, m, 0, x1, sp.mp, sp.kp, sp.mp, s);   // A21
            if (!rc) rc = launch_pack_rect(arrB + (size_t)m * n, n, k, m, 0, z1, sp.mp, sp.kp, sp.mp, s);   // B21
            if (!rc) rc = launch_pack_rect(arrA + m, n, k, m, 1, x2, sp.mp, sp.kp, sp.mp, s);   // A12^T
            if (!rc) rc = launch_pack_rect(arrB + m, n, k, m, 1, z2, sp.mp, sp.kp, sp.mp, s);   // B12^T
            if (rc) return rc;
            GemmSegs sg{};
            sg.X[0] = x1; sg.Z[0] = z1;
            sg.X[1] = x2; sg.Z[1] = z2;
            sg.nseg = 2;
            rc = launch_gemm_nt(GEMM_F32, sp.kp, sp.kp, sp.mp, sp.mp, sp.mp, sg, 1.0f, OUT_F32, lin, sp.kp, k, k,
                                nullptr, nullptr, 0, s);
            if (rc) return rc;
        }
        // GOAT on the non-seed block, with C added to every gradient
        goat_run* h = nullptr;
        rc = run_begin_impl(k, arrA + (size_t)m * n + m, arrB + (size_t)m * n + m, n, nullptr, &o, ws,
                            sp.arrA, stream, lin, &h);
        if (rc) return rc;
        rc = goat_run_steps(h, o.fw_max, hist_host, hist_cap, nullptr);
        std::vector<int32_t> inner(k);
        if (!rc) rc = goat_run_finish(h, inner.data(), &st, nullptr, 0);
        goat_run_free(h);
        if (rc) return rc;
        for (int i = 0; i < k; ++i) pos[m + i] = m + inner[i];
    }
    // full assignment in original labels, and its score on the arranged graphs
    for (int i = 0; i < nA; ++i) perm_host[i] = -1;
    for (int i = 0; i < n; ++i)
        if (ordA[i] >= 0) perm_host[ordA[i]] = ordB[pos[i]];
    int* dpos = reinterpret_cast<int*>(b + sp.pos);
    GOAT_HIP(hipMemcpyAsync(dpos, pos.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    Ptrs p = make_ptrs(make_layout(std::max(k, 1), o.prec, o.symmetric), ws);
    rc = launch_score(n, arrA, arrB, n, dpos, p.red, p.scal + 10, s);
    if (rc) return rc;
    double score = 0.0;
    GOAT_HIP(hipMemcpyAsync(&score, p.scal + 10, 8, hipMemcpyDeviceToHost, s));
    GOAT_HIP(hipStreamSynchronize(s));
    st.score = score;
    if (stats_host) *stats_host = st;
    return GOAT_OK;
}

int goat_solve(int n, const float* A, const float* B, int ld, const float* P0, const goat_options* opt,
               int32_t* perm_host, goat_stats* stats_host, goat_iter_record* hist_host, int hist_cap,
               float* P_out, void* ws, size_t ws_bytes, void* stream) {
    goat_options o;
    if (opt) o = *opt; else goat_default_options(&o);
    GOAT_CHECK_ARG(perm_host, "null pointer");
    goat_run* h = nullptr;
    int rc = goat_run_begin(n, A, B, ld, P0, &o, ws, ws_bytes, stream, &h);
    if (rc) return rc;
    rc = goat_run_steps(h, o.fw_max, hist_host, hist_cap, nullptr);
    if (!rc) rc = goat_run_finish(h, perm_host, stats_host, P_out, ld);
    goat_run_free(h);
    return rc;
}

// Workspace of goat_solve_restarts: [goat_solve's][P0, n x ld][the random
// start's], each 256-byte aligned.
static size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

size_t goat_solve_restarts_workspace_size(int n, int ld, int prec, int symmetric) {
    if (n < 1 || ld < n) return 0;
    return align256(goat_workspace_size(n, prec, symmetric)) + align256((size_t)n * ld * sizeof(float)) +
           goat_random_init_workspace_size(n);
}

int goat_solve_restarts(int n, const float* A, const float* B, int ld, const float* U, int ldu, int restarts,
                        const goat_options* opt, int32_t* perm_host, double* scores_host, int* best_host,
                        goat_stats* stats_host, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    goat_options o;
    if (opt) o = *opt; else goat_default_options(&o);
    GOAT_CHECK_ARG(n >= 1 && ld >= n && ldu >= n, "n < 1 or a leading dimension < n");
    GOAT_CHECK_ARG(A && B && U && perm_host && ws, "null pointer");
    GOAT_CHECK_ARG(restarts >= 1, "restarts < 1");
    const size_t need = goat_solve_restarts_workspace_size(n, ld, o.prec, o.symmetric);
    if (ws_bytes < need) {
        set_error("goat_solve_restarts: workspace smaller than goat_solve_restarts_workspace_size");
        return GOAT_ENOMEM;
    }
    char* base = static_cast<char*>(ws);
    const size_t solve_bytes = align256(goat_workspace_size(n, o.prec, o.symmetric));
    float* P0 = reinterpret_cast<float*>(base + solve_bytes);
    char* init_ws = base + solve_bytes + align256((size_t)n * ld * sizeof(float));
    const size_t init_bytes = goat_random_init_workspace_size(n);
    std::vector<int32_t> perm(n);
    double best_score = 0.0;
    int best = -1;
    for (int r = 0; r < restarts; ++r) {
        const float* Ur = U + (size_t)r * n * ldu;
        int rc = goat_random_init(n, Ur, ldu, P0, ld, 1e-6f, 1000, nullptr, nullptr, init_bytes ? init_ws : nullptr,
                                  init_bytes, stream);
        goat_stats st{};
        if (!rc) rc = goat_solve(n, A, B, ld, P0, &o, perm.data(), &st, nullptr, 0, nullptr, ws, solve_bytes, stream);
        if (rc) return rc;
        if (scores_host) scores_host[r] = st.score;
        // the largest score is kept; a tie keeps the earlier start
        if (best < 0 || st.score > best_score) {
            best = r;
            best_score = st.score;
            std::memcpy(perm_host, perm.data(), sizeof(int32_t) * n);
            if (stats_host) *stats_host = st;
        }
    }
    if (best_host) *best_host = best;
    return GOAT_OK;
}

}  // extern "C"
