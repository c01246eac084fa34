// Internal declarations shared by the libgoat translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/goat.h"

namespace goat {

// ---------------------------------------------------------------- errors

void set_error(const std::string& msg);
void clear_error();

#define GOAT_CHECK_ARG(cond, msg)                     \
    do {                                              \
        if (!(cond)) {                                \
            ::goat::set_error(std::string(__func__) + ": " + (msg)); \
            return GOAT_EINVAL;                       \
        }                                             \
    } while (0)

#define GOAT_HIP(call)                                                      \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) {                                             \
            ::goat::set_error(std::string(#call) + ": " + hipGetErrorString(e_)); \
            return GOAT_EHIP;                                               \
        }                                                                   \
    } while (0)

// ---------------------------------------------------------------- sizes

constexpr int kPad = 256;          // internal matrices are np x np, np = ceil(n/kPad)*kPad
constexpr int kSkWG = 1024;        // max row strips (workgroups) of a Sinkhorn sweep
constexpr int kRedWG = 1024;       // max workgroups of a float64 reduction pass

inline int pad_n(int n) { return (n + kPad - 1) / kPad * kPad; }

struct SkCtrl {                    // Sinkhorn control block (device)
    float kappa;                   // log2(e) / eps
    float eps;
    int   done;                    // 1 converged, 2 eps == 0 (Q = J)
    int   iters;                   // completed column updates
    float err;                     // last checked row-marginal error
    float tol;
    float h;                       // grid step of the compensated potentials
    float g24;                     // 24-bit storage of G: G kappa = q * g24
};

// Workspace layout. All internal matrices have leading dimension np.
struct Layout {
    int n = 0, np = 0, prec = 0, sym = 1;
    size_t opA = 0, opB = 0;       // packed A and B ([X; X^T] when general)
    size_t opP = 0;                // packed P-side operand
    size_t opY = 0;                // intermediate product (transposed layout)
    size_t P = 0, Q = 0, GP = 0, GQ = 0;   // solver matrices (fp32)
    size_t g24 = 0;                // 24-bit copy of G_P (np rows of 3 np / 4 words; mixed forms), 0 = none
    size_t pot = 0;                // potentials: ug, us, ung, uns, vg, vs ([np] each)
    size_t colpart = 0, errpart = 0, ctrl = 0;
    size_t red = 0;                // float64 reduction partials
    size_t scal = 0;               // float64 scalars (line search etc.)
    size_t fscal = 0;              // float scalars (absmax, eps)
    size_t mlp = 0;                // warm-start features [np][4] and prediction [np]
    size_t total = 0;
};

Layout make_layout(int n, int prec, int sym);

inline size_t plane_bytes(int np, int rows_mult, int elt) {
    return (size_t)np * np * rows_mult * elt;
}

// ---------------------------------------------------------------- bf16

__host__ __device__ inline uint16_t f32_to_bf16_rne(float x) {
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// OCP FP8 E4M3 (sign, 4 exponent bits with bias 7, 3 mantissa bits; no
// infinities; largest finite 448; subnormals m * 2^-9). Encoding rounds to
// nearest, ties to even, and saturates at +-448; NaN is not produced for
// finite input.
__host__ __device__ inline uint8_t f32_to_e4m3_rne(float x) {
    const uint32_t u = __builtin_bit_cast(uint32_t, x);
    const uint8_t sign = (uint8_t)((u >> 31) << 7);
    const float a = __builtin_fabsf(x);
    if (!(a > 0.0f)) return sign;                       // zero (or NaN: encoded as zero)
    if (a >= 448.0f) return (uint8_t)(sign | 0x7E);     // saturate
    const int E = (int)((u >> 23) & 0xFF) - 127;
    if (E < -6) {                                       // subnormal: m * 2^-9, m = 0..8
        const int m = (int)__builtin_rintf(a * 512.0f);
        return (uint8_t)(sign | (m >= 8 ? 0x08 : m));
    }
    uint32_t q = ((u & 0x7FFFFFu) | 0x800000u) >> 20;   // 1.mmm (4 bits)
    const uint32_t rem = u & 0xFFFFFu, half = 0x80000u;
    if (rem > half || (rem == half && (q & 1u))) ++q;
    int e = E;
    if (q == 16u) { q = 8u; ++e; }
    if (e > 8 || (e == 8 && q > 14u)) return (uint8_t)(sign | 0x7E);
    return (uint8_t)(sign | ((e + 7) << 3) | (q & 7u));
}
__host__ __device__ inline float e4m3_to_f32(uint8_t c) {
    const int e = (c >> 3) & 15, m = c & 7;
    const float v = e == 0 ? (float)m * 0.001953125f : __builtin_ldexpf((float)(8 + m), e - 10);
    return (c & 0x80) ? -v : v;
}
// Power-of-two exponent s with max|x| * 2^s <= 448 (the first FP8 term of a
// split); 0 for an all-zero matrix.
__host__ __device__ inline int fp8_split_exponent(float absmax) {
    if (!(absmax > 0.0f)) return 0;
    int e = 0;
    __builtin_frexpf(448.0f / absmax, &e);              // 448 / absmax in [2^(e-1), 2^e)
    int s = e - 1;
    if (__builtin_ldexpf(absmax, s) > 448.0f) --s;
    return s < -100 ? -100 : (s > 100 ? 100 : s);
}
constexpr int kFp8Terms = 3;       // FP8 terms of a split operand
constexpr int kFp8TermShift = 4;   // term t is scaled by 2^(s + 4 t)

// ---------------------------------------------------------------- launchers

// Operand packing into padded internal planes (pack.hip).
enum PackMode { PACK_F32 = 0, PACK_BF16 = 1, PACK_BF16_SPLIT = 2, PACK_FP8 = 3 };
int launch_pack(const float* src, int ld, int n, int np, int transpose, int mode,
                void* dst_hi, void* dst_lo, hipStream_t s);
// rows x cols block of src (row stride ld) -> max |x| into *out (pack.hip)
int launch_absmax_rect(int rows, int cols, const float* src, int ld, float* partial, float* out,
                       hipStream_t s);
// rows x cols block of src -> kFp8Terms zero-padded E4M3 planes (np columns,
// plane stride plane_bytes): term t = e4m3(r_t 2^(s + 4t)) with r_0 = x,
// r_{t+1} = r_t - term_t 2^-(s + 4t), s = fp8_split_exponent(*absmax)
// (pack.hip). Rows past `rows` up to prow are written as zeros.
int launch_split_fp8(int rows, int cols, int prow, int np, const float* src, int ld, const float* absmax,
                     uint8_t* planes, size_t plane_bytes, hipStream_t s);

// C[i][j] = alpha * sum_s sum_k X_s[i][k] Z_s[j][k]  (gemm.hip)
enum OutMode { OUT_F32 = 0, OUT_BF16_SPLIT = 1 };
enum GemmKind { GEMM_F32 = 0, GEMM_BF16 = 1, GEMM_FP8 = 2 };
constexpr int kMaxSeg = 6;
struct GemmSegs {
    const void* X[kMaxSeg];
    const void* Z[kMaxSeg];
    int nseg;
    // FP8 only: Z_s holds term (zterm[s]) of a split whose exponent follows
    // from *zmax; the product is scaled back by 2^-(s + 4 zterm[s])
    int zterm[kMaxSeg];
    const float* zmax;
};
int launch_gemm_nt(int kind, int M, int N, int K, int ldx, int ldz,
                   const GemmSegs& segs, float alpha,
                   int out_mode, float* C, int ldc, int m_valid, int n_valid,
                   uint16_t* C_hi, uint16_t* C_lo, int ld_split,
                   hipStream_t s);

// Gradient driver on already-packed operands (grad.cpp).
struct GradOps {
    const void* A_hi; const void* A_lo;     // [A; A^T] when general
    const void* B_hi; const void* B_lo;     // [B; B^T] when general
    const void* P_hi; const void* P_lo;     // P-side operand (fp32 in P_hi for FP32;
                                            // FP8: the term planes in P_hi)
    void* Y_hi; void* Y_lo;                 // intermediate (FP8: fp32 in Y_hi, terms in Y_lo)
    const float* P_max;                     // FP8: max |P-side operand| of its split
    float* Y_max;                           // FP8: max |intermediate|
    float* max_partial;                     // FP8: kRedWG floats for the maxima
};
// FP8 form: split an n x n fp32 operand (leading dimension ld) into the
// E4M3 term planes of P_hi, its maximum into P_max (api.cpp).
int prep_fp8_operand(const Layout& L, const GradOps& o, const float* src, int ld, hipStream_t s);
int grad_packed(const Layout& L, const GradOps& ops, float* G, int ldg, int m_valid,
                hipStream_t s);

// Sinkhorn (sinkhorn.hip)
struct SkState {
    float* ug; float* us;          // row potentials: grid part, remainder
    float* ung; float* uns;        // row potentials of the sweep in flight
    float* vg; float* vs;          // column potentials
    float* colpart; float* errpart; SkCtrl* ctrl;
    // optional 24-bit fixed-point copy of G (sk_pack_g24): the sweeps and Q
    // read it instead of the float G when set
    const uint32_t* g24 = nullptr;
    int ld24 = 0;                  // row stride in 32-bit words (3 np / 4)
    // optional host-visible stop flag (pinned host memory): the kernels that
    // set ctrl->done also store it here, so a host loop can poll it after an
    // event without a device-to-host copy
    int* hdone = nullptr;
};
// Writes the 24-bit copy of G into st.g24 (n rows of ld24 words, zero past
// column n): q_ij = rint(G_ij (2^23 - 1) / max|G|), packed four to three
// words, and ctrl->g24 = kappa max|G| / (2^23 - 1) so that G_ij kappa is read
// back as q_ij * g24 (within max|G kappa| 2^-24 of the float value). Runs after
// sk_prepare (kappa known); absmax_dev is the max|G| that sk_prepare used.
int sk_pack_g24(int n, int np, const float* G, int ldg, const float* absmax_dev, SkState st, hipStream_t s);
// eps = *eps_dev if given, else eps_rel * *absmax_dev if given, else
// eps_rel * max|G| computed here (into fscal[0]).
int sk_prepare(int n, const float* G, int ldg, const float* eps_dev, float eps_rel,
               const float* absmax_dev, const float* g_init, float tol, SkState st, float* fscal,
               double* red, hipStream_t s);
// One Sinkhorn iteration (row sweep + column update); iter is its index in
// the solve (row-walk direction alternates with its parity).
// The first iteration shifts by the row maximum with single-float column
// potentials; every later one uses the compensated potentials.
// sample: the launch may take the profiler's sampled events (false: never,
// so the call creates no event)
int sk_iterate(int n, int np, const float* G, int ldg, SkState st, int first, int check, int iter,
               hipStream_t s, bool sample = true);
// Form Q (fp32 and optional bf16 split), its row-marginal error, potentials
// in natural units, and (when P != NULL) the traces <Q,G>, <P,G>, ||Q-P||^2.
int sk_finalize(int n, int np, const float* G, int ldg, SkState st,
                float* Q, int ldq, uint16_t* Q_hi, uint16_t* Q_lo,
                float* f, float* g, int* iters_out, float* err_out, float* eps_out,
                double* red, hipStream_t s);

// Elementwise / reductions (fw.hip)
int launch_absmax(int n, const float* G, int ldg, float* partial, float* out, hipStream_t s);
// Float64 partials per block of the trace pass (kRedWG blocks at most).
constexpr int kTraceSlots = 6;
int launch_traces(int n, const float* P, const float* Q, const float* GP, const float* GQ,
                  int ld, double* red, double* out8, hipStream_t s, const float* C = nullptr);
// Seeded problems (fw.hip): arrangement of a graph by a vertex order (o < 0:
// dummy), rectangular zero-padded packing, and G += C.
int launch_arrange(int n, const float* X, int ldx, const int* order_dev, int adopted, float* Y, int ldy,
                   hipStream_t s);
int launch_pack_rect(const float* src, int ld, int rows, int cols, int transpose, float* dst, int ldd, int prows,
                     int pcols, hipStream_t s);
int launch_add_mat(int n, float* G, const float* C, int ld, hipStream_t s);
int launch_log_pad(int n, const float* U, int ldu, float* dst, int np, float* one_out, hipStream_t s);
int launch_half_bary(int n, float* P, int ld, hipStream_t s);
// atomically ORs 1 into *flag when X (n x n, ld) holds a NaN or an infinity
int launch_check_finite(int n, const float* X, int ld, int* flag, hipStream_t s);
int launch_fw_update(int n, float* P, const float* Q, float* GP, const float* GQ, int ld,
                     const double* ls8, float* absmax_partial, float* absmax_out,
                     hipStream_t s);
int launch_fill_barycenter(int n, int np, float* P, hipStream_t s);
int launch_copy_pad(int n, const float* src, int lds, float* dst, int ldd, int np, hipStream_t s);
int launch_split_bf16(int n, int np, const float* src, int lds, uint16_t* hi, uint16_t* lo,
                      hipStream_t s);
// Final assignment on the device (assign.hip): epsilon-scaling auction on
// the integer-quantised scores; perm_dev receives the row -> column map.
using AuctionStats = goat_lap_stats;
size_t auction_ws_bytes(int n);         // minimum: scores converted in every scan
size_t auction_ws_bytes_fast(int n);    // with the precomputed scores (+ 8 bytes per entry)
int auction_resolution_bits(int n);
int auction_lap(int n, const float* M, int ld, int32_t* perm_dev, void* ws, size_t ws_bytes, long long max_rounds,
                AuctionStats* st, hipStream_t s);

// compute units of the current device, cached per device (sinkhorn.hip)
int cu_count();

// per-row top-k columns of a score matrix, best first (assign.hip)
int launch_nominate(int rows, int cols, const float* P, int ldp, int k, int32_t* idx, float* val,
                    hipStream_t s);
int launch_score(int n, const float* A, const float* B, int ld, const int32_t* perm,
                 double* red, double* out, hipStream_t s);

// Workspace pointers (api.cpp)
struct Ptrs {
    char* base;
    float* P; float* Q; float* GP; float* GQ;
    void* A_hi; void* A_lo; void* B_hi; void* B_lo;
    void* P_hi; void* P_lo; void* Y_hi; void* Y_lo;
    SkState sk;
    double* red; double* scal; float* fscal; float* g_prev; int32_t* perm_dev;
    float* feat; float* pred;
};
size_t small_bytes(const Layout& L);
Ptrs make_ptrs(const Layout& L, void* ws);

// goat_sinkhorn's argument checks, whether G must be repacked into the
// workspace, and the solve itself on a prepared small state (api.cpp)
int sinkhorn_check(int n, const float* G, int ldg, const float* eps_dev, float eps_rel, const float* g, int init,
                   const float* mlp_params, int max_iter, float tol, const float* Q, int ldq);
bool sinkhorn_needs_repack(const float* G, int ldg, int max_iter);
int sinkhorn_run(int n, const float* G, int ldg, const float* eps_dev, float eps_rel, float* f, float* g, int init,
                 const float* mlp_params, int max_iter, float tol, float* Q, int ldq, int* iters_dev,
                 float* err_dev, float* eps_out, const Ptrs& p, int np, bool sample, hipStream_t s);
int pack_graph(const Layout& L, const float* X, int ld, void* hi, void* lo, hipStream_t s);
GradOps grad_ops(const Ptrs& p);

// Sampled per-launch timing (profile.cpp): which = 0 Sinkhorn row sweep,
// 1 gradient product
void prof_begin(int which, hipStream_t s);
void prof_end(int which, hipStream_t s);
// events for a sampled launch to hand to hipExtLaunchKernel (false and null
// events when this launch is not sampled); prof_commit after the launch
bool prof_sample(int which, hipEvent_t* start, hipEvent_t* stop);
void prof_commit(int which);

// Learned warm start (mlp.hip)
int mlp_param_count();
size_t mlp_part_bytes(int N);
int mlp_features(int n, int np, const float* G, int ldg, const float* eps_dev, float* part, float* F,
                 hipStream_t s);
int mlp_forward(int N, const float* F, const float* p, float* y, hipStream_t s);
int mlp_backward(int N, const float* F, const float* t, const float* p, float* grad, float* loss, void* part,
                 hipStream_t s);
int mlp_adam(const float* grad, float* p, float* m, float* v, int step, float lr, hipStream_t s);
int warm_seed(int n, const float* pred, const SkCtrl* ctrl, float* vg, float* vs, hipStream_t s);

// Host linear assignment (lap.cpp)
int lap_max(int n, const double* M, int ld, int32_t* perm);

}  // namespace goat
