// C ABI of libgoat: argument checks, workspace layout, and the host drivers
// of the gradient, LOT (Sinkhorn) and line-search calls and of the full
// GOAT Frank-Wolfe loop (Alg. 3).
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"

namespace goat {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

Layout make_layout(int n, int prec, int sym) {
    Layout L;
    L.n = n;
    L.np = pad_n(n);
    L.prec = prec;
    L.sym = sym ? 1 : 0;
    const size_t np = L.np;
    const size_t pl = np * np;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
    // small state first: offsets depend on n only
    L.ctrl = take(256);
    L.pot = take(np * 4 * 6);
    L.errpart = take(kSkWG * 4);
    L.colpart = take((size_t)kSkWG * np * 4);
    L.red = take((size_t)kRedWG * kTraceSlots * 8);
    L.scal = take(64 * 8 + np * 4 * 2);   // scalars, then g_prev[np], perm_dev[np]
    L.fscal = take((16 + kRedWG) * 4);
    L.mlp = take(np * 5 * 4);
    // fp32 solver matrices
    L.P = take(pl * 4);
    L.Q = take(pl * 4);
    L.GP = take(pl * 4);
    L.GQ = take(pl * 4);
    // 24-bit copy of G for the Sinkhorn sweeps (mixed forms only)
    if (prec != GOAT_PREC_FP32) L.g24 = take(pl * 3);
    // packed operands
    const int rows = L.sym ? 1 : 2;
    if (prec == GOAT_PREC_FP8) {
        L.opA = take(pl * rows);                          // E4M3
        L.opB = take(pl * rows);
        L.opP = take(pl * kFp8Terms);                     // term planes of P (or Q)
        L.opY = take(pl * rows * 4 + pl * rows * kFp8Terms);   // fp32 Y^T, then its terms
        L.total = o;
        return L;
    }
    const size_t op_elt = prec == GOAT_PREC_FP32 ? 4 : 2;
    const int op_planes = prec == GOAT_PREC_BF16X3 ? 2 : 1;
    L.opA = take(pl * rows * op_elt * op_planes);
    L.opB = take(pl * rows * op_elt * op_planes);
    L.opP = take(prec == GOAT_PREC_FP32 ? pl * 4 : pl * 2 * 2);
    L.opY = take(prec == GOAT_PREC_FP32 ? pl * rows * 4 : pl * rows * 2 * 2);
    L.total = o;
    return L;
}

size_t small_bytes(const Layout& L) { return L.P; }

// ---------------------------------------------------------------- gradient

// Symmetric: Y^T = B P^T (= (P B)^T) then G = 2 A Y. General: the stacked
// [B; B^T] P^T gives (P B^T)^T and (P B)^T, then
// G = A (P B^T) + A^T (P B) as one product over two k-segments.
// FP8 (0/1 A, B exact in E4M3): the P-side operand and Y^T enter as three
// E4M3 terms each, k-concatenated segments scaled back on the matrix cores.
static int grad_packed_fp8(const Layout& L, const GradOps& o, float* G, int ldg, int m_valid, hipStream_t s) {
    const int np = L.np;
    const size_t pl = (size_t)np * np;
    const int rows = L.sym ? 1 : 2;
    const uint8_t* P8 = static_cast<const uint8_t*>(o.P_hi);
    GemmSegs s1{};
    for (int t = 0; t < kFp8Terms; ++t) {
        s1.X[t] = o.B_hi;
        s1.Z[t] = P8 + t * pl;
        s1.zterm[t] = t;
    }
    s1.nseg = kFp8Terms;
    s1.zmax = o.P_max;
    float* Y = static_cast<float*>(o.Y_hi);
    uint8_t* Y8 = static_cast<uint8_t*>(o.Y_lo);
    int rc = launch_gemm_nt(GEMM_FP8, rows * np, np, np, np, np, s1, 1.0f, OUT_F32, Y, np, rows * np, np, nullptr,
                            nullptr, 0, s);
    if (!rc) rc = launch_absmax_rect(rows * np, np, Y, np, o.max_partial, o.Y_max, s);
    if (!rc) rc = launch_split_fp8(rows * np, np, rows * np, np, Y, np, o.Y_max, Y8, pl * rows, s);
    if (rc) return rc;
    GemmSegs s2{};
    int k = 0;
    for (int h = 0; h < rows; ++h)
        for (int t = 0; t < kFp8Terms; ++t) {
            s2.X[k] = static_cast<const uint8_t*>(o.A_hi) + h * pl;     // A (h=0) or A^T (h=1)
            s2.Z[k] = Y8 + t * pl * rows + h * pl;                     // term t of (P B^T)^T or (P B)^T
            s2.zterm[k] = t;
            ++k;
        }
    s2.nseg = k;
    s2.zmax = o.Y_max;
    return launch_gemm_nt(GEMM_FP8, np, np, np, np, np, s2, L.sym ? 2.0f : 1.0f, OUT_F32, G, ldg, m_valid, m_valid,
                          nullptr, nullptr, 0, s);
}

int prep_fp8_operand(const Layout& L, const GradOps& o, const float* src, int ld, hipStream_t s) {
    float* pmax = const_cast<float*>(o.P_max);
    int rc = launch_absmax_rect(L.n, L.n, src, ld, o.max_partial, pmax, s);
    if (rc) return rc;
    return launch_split_fp8(L.n, L.n, L.np, L.np, src, ld, pmax,
                            static_cast<uint8_t*>(const_cast<void*>(o.P_hi)), (size_t)L.np * L.np, s);
}

int grad_packed(const Layout& L, const GradOps& o, float* G, int ldg, int m_valid, hipStream_t s) {
    if (L.prec == GOAT_PREC_FP8) return grad_packed_fp8(L, o, G, ldg, m_valid, s);
    const int np = L.np;
    const size_t pl = (size_t)np * np;
    const int rows = L.sym ? 1 : 2;
    const bool bf = L.prec != GOAT_PREC_FP32;
    const size_t es = bf ? 2 : 4;
    auto off = [&](const void* p, size_t elems) {
        return static_cast<const void*>(static_cast<const char*>(p) + elems * es);
    };
    GemmSegs s1{}, s2{};
    if (L.prec == GOAT_PREC_FP32) {
        s1.X[0] = o.B_hi; s1.Z[0] = o.P_hi; s1.nseg = 1;
    } else if (L.prec == GOAT_PREC_BF16X2) {
        s1.X[0] = o.B_hi; s1.Z[0] = o.P_hi;
        s1.X[1] = o.B_hi; s1.Z[1] = o.P_lo; s1.nseg = 2;
    } else {
        s1.X[0] = o.B_hi; s1.Z[0] = o.P_hi;
        s1.X[1] = o.B_hi; s1.Z[1] = o.P_lo;
        s1.X[2] = o.B_lo; s1.Z[2] = o.P_hi; s1.nseg = 3;
    }
    int rc = launch_gemm_nt(bf ? GEMM_BF16 : GEMM_F32, rows * np, np, np, np, np, s1, 1.0f, bf ? OUT_BF16_SPLIT : OUT_F32,
                            static_cast<float*>(o.Y_hi), np, rows * np, np,
                            static_cast<uint16_t*>(o.Y_hi), static_cast<uint16_t*>(o.Y_lo), np, s);
    if (rc) return rc;
    // second product: segments over (A-part, Y-part) for each stacked half
    int k = 0;
    for (int h = 0; h < rows; ++h) {
        const size_t ah = (size_t)h * pl;        // A (h=0) or A^T (h=1)
        const size_t yh = (size_t)h * pl;        // (P B^T)^T (h=0) or (P B)^T (h=1)
        if (L.prec == GOAT_PREC_FP32) {
            s2.X[k] = off(o.A_hi, ah); s2.Z[k] = off(o.Y_hi, yh); ++k;
        } else if (L.prec == GOAT_PREC_BF16X2) {
            s2.X[k] = off(o.A_hi, ah); s2.Z[k] = off(o.Y_hi, yh); ++k;
            s2.X[k] = off(o.A_hi, ah); s2.Z[k] = off(o.Y_lo, yh); ++k;
        } else {
            s2.X[k] = off(o.A_hi, ah); s2.Z[k] = off(o.Y_hi, yh); ++k;
            s2.X[k] = off(o.A_hi, ah); s2.Z[k] = off(o.Y_lo, yh); ++k;
            s2.X[k] = off(o.A_lo, ah); s2.Z[k] = off(o.Y_hi, yh); ++k;
        }
    }
    s2.nseg = k;
    return launch_gemm_nt(bf ? GEMM_BF16 : GEMM_F32, np, np, np, np, np, s2, L.sym ? 2.0f : 1.0f, OUT_F32, G, ldg, m_valid,
                          m_valid, nullptr, nullptr, 0, s);
}

Ptrs make_ptrs(const Layout& L, void* ws) {
    Ptrs p{};
    char* b = static_cast<char*>(ws);
    const size_t pl = (size_t)L.np * L.np;
    const int rows = L.sym ? 1 : 2;
    p.base = b;
    p.P = reinterpret_cast<float*>(b + L.P);
    p.Q = reinterpret_cast<float*>(b + L.Q);
    p.GP = reinterpret_cast<float*>(b + L.GP);
    p.GQ = reinterpret_cast<float*>(b + L.GQ);
    if (L.prec == GOAT_PREC_FP8) {
        p.A_hi = b + L.opA;
        p.A_lo = nullptr;
        p.B_hi = b + L.opB;
        p.B_lo = nullptr;
        p.P_hi = b + L.opP;
        p.P_lo = nullptr;
        p.Y_hi = b + L.opY;
        p.Y_lo = b + L.opY + pl * rows * 4;
    } else {
        const size_t op_elt = L.prec == GOAT_PREC_FP32 ? 4 : 2;
        p.A_hi = b + L.opA;
        p.A_lo = b + L.opA + pl * rows * op_elt;
        p.B_hi = b + L.opB;
        p.B_lo = b + L.opB + pl * rows * op_elt;
        p.P_hi = b + L.opP;
        p.P_lo = b + L.opP + pl * 2;
        p.Y_hi = b + L.opY;
        p.Y_lo = b + L.opY + pl * rows * 2;
    }
    p.sk.ctrl = reinterpret_cast<SkCtrl*>(b + L.ctrl);
    float* pot = reinterpret_cast<float*>(b + L.pot);
    p.sk.ug = pot;
    p.sk.us = pot + (size_t)L.np;
    p.sk.ung = pot + 2 * (size_t)L.np;
    p.sk.uns = pot + 3 * (size_t)L.np;
    p.sk.vg = pot + 4 * (size_t)L.np;
    p.sk.vs = pot + 5 * (size_t)L.np;
    p.sk.errpart = reinterpret_cast<float*>(b + L.errpart);
    p.sk.colpart = reinterpret_cast<float*>(b + L.colpart);
    p.red = reinterpret_cast<double*>(b + L.red);
    p.scal = reinterpret_cast<double*>(b + L.scal);
    p.g_prev = reinterpret_cast<float*>(b + L.scal + 64 * 8);
    p.perm_dev = reinterpret_cast<int32_t*>(b + L.scal + 64 * 8 + (size_t)L.np * 4);
    p.fscal = reinterpret_cast<float*>(b + L.fscal);
    p.feat = reinterpret_cast<float*>(b + L.mlp);
    p.pred = p.feat + (size_t)L.np * 4;
    return p;
}

int pack_graph(const Layout& L, const float* X, int ld, void* hi, void* lo, hipStream_t s) {
    const int mode = L.prec == GOAT_PREC_FP32 ? PACK_F32
                     : L.prec == GOAT_PREC_FP8 ? PACK_FP8
                     : (L.prec == GOAT_PREC_BF16X2 ? PACK_BF16 : PACK_BF16_SPLIT);
    const size_t es = L.prec == GOAT_PREC_FP32 ? 4 : (L.prec == GOAT_PREC_FP8 ? 1 : 2);
    const size_t pl = (size_t)L.np * L.np;
    int rc = launch_pack(X, ld, L.n, L.np, 0, mode, hi, lo, s);
    if (rc || L.sym) return rc;
    return launch_pack(X, ld, L.n, L.np, 1, mode, static_cast<char*>(hi) + pl * es,
                       lo ? static_cast<char*>(lo) + pl * es : nullptr, s);
}

GradOps grad_ops(const Ptrs& p) {
    GradOps o;
    o.A_hi = p.A_hi; o.A_lo = p.A_lo; o.B_hi = p.B_hi; o.B_lo = p.B_lo;
    o.P_hi = p.P_hi; o.P_lo = p.P_lo; o.Y_hi = p.Y_hi; o.Y_lo = p.Y_lo;
    // FP8 maxima: fscal[1] (P-side operand), fscal[2] (Y^T); partials at fscal + 16
    o.P_max = p.fscal + 1;
    o.Y_max = p.fscal + 2;
    o.max_partial = p.fscal + 16;
    return o;
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace goat

using namespace goat;

namespace goat {

int sinkhorn_check(int n, const float* G, int ldg, const float* eps_dev, float eps_rel, const float* g, int init,
                   const float* mlp_params, int max_iter, float tol, const float* Q, int ldq) {
    GOAT_CHECK_ARG(n >= 1, "n < 1");
    GOAT_CHECK_ARG(G, "null pointer");
    GOAT_CHECK_ARG(ldg >= n && (!Q || ldq >= n), "leading dimension < n");
    GOAT_CHECK_ARG(init == GOAT_INIT_COLD || (init == GOAT_INIT_G && g) || (init == GOAT_INIT_MLP && mlp_params),
                   "bad init (GOAT_INIT_G needs g, GOAT_INIT_MLP needs mlp_params)");
    GOAT_CHECK_ARG(init != GOAT_INIT_MLP || n <= 20480, "the warm-start network takes n <= 20480");
    GOAT_CHECK_ARG(max_iter >= 0, "max_iter < 0");
    GOAT_CHECK_ARG(std::isfinite(tol) && tol >= 0.0f, "bad tol");
    GOAT_CHECK_ARG(eps_dev || (std::isfinite(eps_rel) && eps_rel > 0.0f), "bad eps_rel");
    return GOAT_OK;
}

bool sinkhorn_needs_repack(const float* G, int ldg, int max_iter) {
    return (ldg % 4) != 0 || !aligned16(G) || ((ldg % 64) != 0 && max_iter >= 8);
}

// The LOT solve of goat_sinkhorn on G (ldg) with the small state at p:
// starting potentials, sweeps (each launch samples the profiler only when
// `sample`), then Q and the outputs.
int sinkhorn_run(int n, const float* G, int ldg, const float* eps_dev, float eps_rel, float* f, float* g, int init,
                 const float* mlp_params, int max_iter, float tol, float* Q, int ldq, int* iters_dev,
                 float* err_dev, float* eps_out, const Ptrs& p, int np, bool sample, hipStream_t s) {
    int rc = sk_prepare(n, G, ldg, eps_dev, eps_rel, nullptr, init == GOAT_INIT_G ? g : nullptr, tol, p.sk,
                        p.fscal, p.red, s);
    if (rc) return rc;
    if (init == GOAT_INIT_MLP) {
        // features of G / eps with the eps just set, the network, then the
        // column potentials (the column partials are scratch until the sweeps)
        rc = mlp_features(n, np, G, ldg, &p.sk.ctrl->eps, p.sk.colpart, p.feat, s);
        if (!rc) rc = mlp_forward(n, p.feat, mlp_params, p.pred, s);
        if (!rc) rc = warm_seed(n, p.pred, p.sk.ctrl, p.sk.vg, p.sk.vs, s);
        if (rc) return rc;
    }
    for (int k = 0; k < max_iter; ++k) {
        rc = sk_iterate(n, np, G, ldg, p.sk, k == 0, k >= 1, k, s, sample);
        if (rc) return rc;
    }
    return sk_finalize(n, np, G, ldg, p.sk, Q, ldq, nullptr, nullptr, f, g, iters_dev, err_dev, eps_out, p.red, s);
}

}  // namespace goat

extern "C" {

int goat_version(void) { return 100; }

const char* goat_last_error(void) { return g_last_error.c_str(); }

size_t goat_workspace_size(int n, int prec, int symmetric) {
    if (n < 1 || prec < GOAT_PREC_FP32 || prec > GOAT_PREC_FP8) return 0;
    return make_layout(n, prec, symmetric).total;
}

void goat_default_options(goat_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->eps_rel = 0.03f;
    opt->sk_tol = 1e-6f;
    opt->sk_max = 1000;
    opt->fw_max = 30;
    opt->fw_tol = 0.0f;
    opt->prec = GOAT_PREC_FP32;
    opt->symmetric = 1;
    opt->proj = 0;
    opt->warm = 0;
    opt->stop_on_stall = 1;
    opt->check_every = 16;
}

int goat_pack(int n, const float* A, const float* B, int ld, int prec, int symmetric, void* ws, size_t ws_bytes,
              void* stream) {
    clear_error();
    GOAT_CHECK_ARG(n >= 1, "n < 1");
    GOAT_CHECK_ARG(A && B && ws, "null pointer");
    GOAT_CHECK_ARG(ld >= n, "leading dimension < n");
    GOAT_CHECK_ARG(prec >= GOAT_PREC_FP32 && prec <= GOAT_PREC_FP8, "unknown precision");
    const Layout L = make_layout(n, prec, symmetric);
    if (ws_bytes < L.total) { set_error("goat_pack: workspace too small"); return GOAT_ENOMEM; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ptrs p = make_ptrs(L, ws);
    int rc = pack_graph(L, A, ld, p.A_hi, p.A_lo, s);
    if (!rc) rc = pack_graph(L, B, ld, p.B_hi, p.B_lo, s);
    return rc;
}

int goat_grad_packed(int n, const float* P, int ldp, float* G, int ldg, int prec, int symmetric, void* ws,
                     size_t ws_bytes, void* stream) {
    clear_error();
    GOAT_CHECK_ARG(n >= 1, "n < 1");
    GOAT_CHECK_ARG(P && G && ws, "null pointer");
    GOAT_CHECK_ARG(ldp >= n && ldg >= n, "leading dimension < n");
    GOAT_CHECK_ARG(prec >= GOAT_PREC_FP32 && prec <= GOAT_PREC_FP8, "unknown precision");
    const Layout L = make_layout(n, prec, symmetric);
    if (ws_bytes < L.total) { set_error("goat_grad_packed: workspace too small"); return GOAT_ENOMEM; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ptrs p = make_ptrs(L, ws);
    int rc;
    if (prec == GOAT_PREC_FP8) rc = prep_fp8_operand(L, grad_ops(p), P, ldp, s);
    else if (prec == GOAT_PREC_FP32) rc = launch_copy_pad(n, P, ldp, static_cast<float*>(p.P_hi), L.np, L.np, s);
    else rc = launch_split_bf16(n, L.np, P, ldp, static_cast<uint16_t*>(p.P_hi), static_cast<uint16_t*>(p.P_lo), s);
    if (rc) return rc;
    return grad_packed(L, grad_ops(p), G, ldg, n, s);
}

int goat_grad(int n, const float* A, const float* B, int ld, const float* P, int ldp, float* G, int ldg,
              int prec, int symmetric, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    GOAT_CHECK_ARG(n >= 1, "n < 1");
    GOAT_CHECK_ARG(A && B && P && G && ws, "null pointer");
    GOAT_CHECK_ARG(ld >= n && ldp >= n && ldg >= n, "leading dimension < n");
    GOAT_CHECK_ARG(prec >= GOAT_PREC_FP32 && prec <= GOAT_PREC_FP8, "unknown precision");
    const Layout L = make_layout(n, prec, symmetric);
    if (ws_bytes < L.total) { set_error("goat_grad: workspace too small"); return GOAT_ENOMEM; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ptrs p = make_ptrs(L, ws);
    int rc = pack_graph(L, A, ld, p.A_hi, p.A_lo, s);
    if (!rc) rc = pack_graph(L, B, ld, p.B_hi, p.B_lo, s);
    if (rc) return rc;
    if (prec == GOAT_PREC_FP8) rc = prep_fp8_operand(L, grad_ops(p), P, ldp, s);
    else if (prec == GOAT_PREC_FP32) rc = launch_copy_pad(n, P, ldp, static_cast<float*>(p.P_hi), L.np, L.np, s);
    else rc = launch_split_bf16(n, L.np, P, ldp, static_cast<uint16_t*>(p.P_hi), static_cast<uint16_t*>(p.P_lo), s);
    if (rc) return rc;
    return grad_packed(L, grad_ops(p), G, ldg, n, s);
}

int goat_sinkhorn(int n, const float* G, int ldg, const float* eps_dev, float eps_rel, float* f, float* g,
                  int init, const float* mlp_params, int max_iter, float tol, float* Q, int ldq, int* iters_dev,
                  float* err_dev, float* eps_out, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    int rc = sinkhorn_check(n, G, ldg, eps_dev, eps_rel, g, init, mlp_params, max_iter, tol, Q, ldq);
    if (rc) return rc;
    GOAT_CHECK_ARG(ws, "null workspace");
    const Layout L = make_layout(n, GOAT_PREC_FP32, 1);
    // rows are swept as float4 and read best at 256-byte alignment: G is
    // copied into the padded layout when it is misaligned for float4, or when
    // its rows are not 256-byte multiples and enough sweeps follow to pay back
    // the copy (one read and one write of G)
    const bool repack = sinkhorn_needs_repack(G, ldg, max_iter);
    const size_t need = small_bytes(L) + (repack ? (size_t)L.np * L.np * 4 : 0);
    if (ws_bytes < need) { set_error("goat_sinkhorn: workspace too small"); return GOAT_ENOMEM; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ptrs p = make_ptrs(L, ws);
    const float* Gk = G;
    int ldk = ldg;
    if (repack) {
        rc = launch_copy_pad(n, G, ldg, p.P, L.np, L.np, s);
        if (rc) return rc;
        Gk = p.P;
        ldk = L.np;
    }
    return sinkhorn_run(n, Gk, ldk, eps_dev, eps_rel, f, g, init, mlp_params, max_iter, tol, Q, ldq, iters_dev,
                        err_dev, eps_out, p, L.np, true, s);
}

int goat_linesearch(int n, const float* P, const float* Q, const float* GP, const float* GQ, int ld,
                    double* out_dev, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    GOAT_CHECK_ARG(n >= 1, "n < 1");
    GOAT_CHECK_ARG(P && Q && GP && GQ && out_dev && ws, "null pointer");
    GOAT_CHECK_ARG(ld >= n, "leading dimension < n");
    const Layout L = make_layout(n, GOAT_PREC_FP32, 1);
    if (ws_bytes < small_bytes(L)) { set_error("goat_linesearch: workspace too small"); return GOAT_ENOMEM; }
    Ptrs p = make_ptrs(L, ws);
    return launch_traces(n, P, Q, GP, GQ, ld, p.red, out_dev, static_cast<hipStream_t>(stream));
}

int goat_lap_max(int n, const double* M_host, int ld, int32_t* perm_host) {
    clear_error();
    return lap_max(n, M_host, ld, perm_host);
}

int goat_score(int n, const float* A, const float* B, int ld, const int32_t* perm_dev, double* out_dev,
               void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    GOAT_CHECK_ARG(n >= 1, "n < 1");
    GOAT_CHECK_ARG(A && B && perm_dev && out_dev && ws, "null pointer");
    GOAT_CHECK_ARG(ld >= n, "leading dimension < n");
    const Layout L = make_layout(n, GOAT_PREC_FP32, 1);
    if (ws_bytes < small_bytes(L)) { set_error("goat_score: workspace too small"); return GOAT_ENOMEM; }
    Ptrs p = make_ptrs(L, ws);
    return launch_score(n, A, B, ld, perm_dev, p.red, out_dev, static_cast<hipStream_t>(stream));
}

size_t goat_lap_device_workspace_size(int n) { return auction_ws_bytes_fast(n); }
size_t goat_lap_device_workspace_min(int n) { return auction_ws_bytes(n); }

int goat_lap_device(int n, const float* M, int ld, int32_t* perm_dev, void* ws, size_t ws_bytes,
                    long long max_rounds, goat_lap_stats* stats, void* stream) {
    clear_error();
    GOAT_CHECK_ARG(n >= 1, "n < 1");
    GOAT_CHECK_ARG(ld >= n, "leading dimension < n");
    GOAT_CHECK_ARG(M && perm_dev && ws, "null pointer");
    return auction_lap(n, M, ld, perm_dev, ws, ws_bytes, max_rounds > 0 ? max_rounds : 20000000ll, stats,
                       static_cast<hipStream_t>(stream));
}

int goat_nominate(int rows, int cols, const float* P, int ldp, int k, int32_t* idx_dev, float* val_dev,
                  void* stream) {
    clear_error();
    GOAT_CHECK_ARG(rows >= 1 && cols >= 1, "rows < 1 or cols < 1");
    GOAT_CHECK_ARG(k >= 1 && k <= cols, "k outside [1, cols]");
    GOAT_CHECK_ARG(k <= GOAT_NOMINATE_KMAX, "k > GOAT_NOMINATE_KMAX");
    GOAT_CHECK_ARG(ldp >= cols, "leading dimension < cols");
    GOAT_CHECK_ARG(P && idx_dev, "null pointer");
    return launch_nominate(rows, cols, P, ldp, k, idx_dev, val_dev, static_cast<hipStream_t>(stream));
}

int goat_mlp_param_count(void) { return mlp_param_count(); }

size_t goat_mlp_workspace_size(int n_samples) {
    return n_samples < 1 ? 0 : mlp_part_bytes(n_samples);
}

int goat_mlp_features(int n, const float* G, int ldg, const float* eps_dev, float* F, void* ws, size_t ws_bytes,
                      void* stream) {
    clear_error();
    GOAT_CHECK_ARG(n >= 1, "n < 1");
    GOAT_CHECK_ARG(G && eps_dev && F && ws, "null pointer");
    GOAT_CHECK_ARG(ldg >= n, "leading dimension < n");
    const Layout L = make_layout(n, GOAT_PREC_FP32, 1);
    const bool repack = (ldg % 4) != 0 || !aligned16(G);
    const size_t need = small_bytes(L) + (repack ? (size_t)L.np * L.np * 4 : 0);
    if (ws_bytes < need) { set_error("goat_mlp_features: workspace too small"); return GOAT_ENOMEM; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ptrs p = make_ptrs(L, ws);
    const float* Gk = G;
    int ldk = ldg;
    if (repack) {
        int rc = launch_copy_pad(n, G, ldg, p.P, L.np, L.np, s);
        if (rc) return rc;
        Gk = p.P;
        ldk = L.np;
    }
    return mlp_features(n, L.np, Gk, ldk, eps_dev, p.sk.colpart, F, s);
}

int goat_mlp_forward(int N, const float* F, const float* params, float* y, void* stream) {
    clear_error();
    GOAT_CHECK_ARG(N >= 1, "N < 1");
    GOAT_CHECK_ARG(F && params && y, "null pointer");
    return mlp_forward(N, F, params, y, static_cast<hipStream_t>(stream));
}

int goat_mlp_backward(int N, const float* F, const float* target, const float* params, float* grad, float* loss_dev,
                      void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    GOAT_CHECK_ARG(N >= 1, "N < 1");
    GOAT_CHECK_ARG(F && target && params && grad && ws, "null pointer");
    if (ws_bytes < mlp_part_bytes(N)) { set_error("goat_mlp_backward: workspace too small"); return GOAT_ENOMEM; }
    return mlp_backward(N, F, target, params, grad, loss_dev, ws, static_cast<hipStream_t>(stream));
}

int goat_mlp_adam(const float* grad, float* params, float* m, float* v, int step, float lr, void* stream) {
    clear_error();
    GOAT_CHECK_ARG(grad && params && m && v, "null pointer");
    GOAT_CHECK_ARG(step >= 1 && std::isfinite(lr) && lr > 0.0f, "step >= 1 and lr > 0 required");
    return mlp_adam(grad, params, m, v, step, lr, static_cast<hipStream_t>(stream));
}

}  // extern "C"
