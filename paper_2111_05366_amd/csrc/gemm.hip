// Dense "NT" products on the gfx950 matrix cores:
//     C[i][j] = alpha * sum_s sum_k X_s[i][k] * Z_s[j][k]
// X_s and Z_s are row-major with the contraction index contiguous, so both
// MFMA operands are read along k. The segments s concatenate contractions
// (hi/lo precision terms, or the two gradient terms of a general pair).
// Operands are zero-padded internal planes: M, N multiples of 128 and K a
// multiple of the k-tile, so the main loop has no bounds checks.
//
// Block tile 128 x 128, four waves in a 2 x 2 arrangement, each wave a
// 64 x 64 sub-tile made of 2 x 2 MFMA 32x32 blocks. Double-buffered LDS
// stages with register-staged global loads (one barrier per k-tile).
#include "common.h"

namespace goat {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BM = 128, BN = 128;

struct GemmParams {
    const void* X[kMaxSeg];
    const void* Z[kMaxSeg];
    int nseg, K, ldx, ldz;
    float alpha;
    float* C;
    int ldc, m_valid, n_valid;
    uint16_t* Chi;
    uint16_t* Clo;
    int ld_split;
    int tiles_m, tiles_n;
};

// Block -> tile map. Consecutive block ids go to different XCDs (round
// robin); remap so that the blocks of one XCD cover a compact group of
// tiles sharing X rows and Z rows in that XCD's L2.
__device__ inline void tile_of(const GemmParams& p, int& tm, int& tn) {
    const int nb = p.tiles_m * p.tiles_n;
    int b = blockIdx.x;
    if (nb % 8 == 0) {
        const int per = nb / 8;
        b = (b % 8) * per + (b / 8);
    }
    // group-of-8-rows ordering inside the linear range
    const int G = 8;
    const int group = b / (G * p.tiles_n);
    const int first_m = group * G;
    const int gm = min(p.tiles_m - first_m, G);
    const int in = b % (G * p.tiles_n);
    tm = first_m + (in % gm);
    tn = in / gm;
}

template <int OUT>
__device__ inline void store_tile(const GemmParams& p, const f32x16 (&acc)[2][2], int m0, int n0,
                                  int wm, int wn, int lane) {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm * 64 + mi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int col = n0 + wn * 64 + ni * 32 + (lane & 31);
                const float x = p.alpha * acc[mi][ni][r];
                if (OUT == OUT_F32) {
                    if (row < p.m_valid && col < p.n_valid) p.C[(size_t)row * p.ldc + col] = x;
                } else {
                    const uint16_t h = f32_to_bf16_rne(x);
                    const size_t idx = (size_t)row * p.ld_split + col;
                    p.Chi[idx] = h;
                    p.Clo[idx] = f32_to_bf16_rne(x - bf16_to_f32(h));
                }
            }
}

// ------------------------------------------------------------------ bf16

constexpr int BK16 = 64;                 // k-tile (bf16 elements)
constexpr int LD16 = BK16 + 8;           // LDS row stride (bf16 elements), 16 B pad

template <int OUT>
__global__ __launch_bounds__(256) void gemm_nt_bf16_kernel(GemmParams p) {
    __shared__ __attribute__((aligned(16))) uint16_t sA[2][BM * LD16];
    __shared__ __attribute__((aligned(16))) uint16_t sB[2][BN * LD16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_of(p, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int ktiles = p.K / BK16;
    const int total = ktiles * p.nseg;

    f32x16 acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mi][ni][r] = 0.0f;

    uint4 ra[4], rb[4];
    auto gload = [&](int t) {
        const int seg = t / ktiles, kt = t - seg * ktiles;
        const uint16_t* X = static_cast<const uint16_t*>(p.X[seg]) + (size_t)m0 * p.ldx + kt * BK16;
        const uint16_t* Z = static_cast<const uint16_t*>(p.Z[seg]) + (size_t)n0 * p.ldz + kt * BK16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c = tid + 256 * i, row = c >> 3, kc = c & 7;
            ra[i] = *reinterpret_cast<const uint4*>(X + (size_t)row * p.ldx + kc * 8);
            rb[i] = *reinterpret_cast<const uint4*>(Z + (size_t)row * p.ldz + kc * 8);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c = tid + 256 * i, row = c >> 3, kc = c & 7;
            *reinterpret_cast<uint4*>(&sA[buf][row * LD16 + kc * 8]) = ra[i];
            *reinterpret_cast<uint4*>(&sB[buf][row * LD16 + kc * 8]) = rb[i];
        }
    };

    gload(0);
    sstore(0);
    __syncthreads();
    for (int t = 0; t < total; ++t) {
        const int buf = t & 1;
        if (t + 1 < total) gload(t + 1);
#pragma unroll
        for (int ks = 0; ks < BK16 / 16; ++ks) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
                a[mi] = *reinterpret_cast<const bf16x8*>(
                    &sA[buf][(wm * 64 + mi * 32 + (lane & 31)) * LD16 + ks * 16 + (lane >> 5) * 8]);
#pragma unroll
            for (int ni = 0; ni < 2; ++ni)
                b[ni] = *reinterpret_cast<const bf16x8*>(
                    &sB[buf][(wn * 64 + ni * 32 + (lane & 31)) * LD16 + ks * 16 + (lane >> 5) * 8]);
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
        }
        if (t + 1 < total) sstore(buf ^ 1);
        __syncthreads();
    }
    store_tile<OUT>(p, acc, m0, n0, wm, wn, lane);
}

// ------------------------------------------------------------------ fp32

constexpr int BK32 = 16;                 // k-tile (float elements)
constexpr int LD32 = BK32 + 4;           // LDS row stride (floats)

// In LDS each row's k-tile is stored permuted, k -> (k & 1) * 8 + (k >> 1),
// so that the eight values a lane feeds to eight successive 32x32x2 MFMAs
// (k = 2 kk + lane/32) are contiguous.
template <int OUT>
__global__ __launch_bounds__(256) void gemm_nt_f32_kernel(GemmParams p) {
    __shared__ __attribute__((aligned(16))) float sA[2][BM * LD32];
    __shared__ __attribute__((aligned(16))) float sB[2][BN * LD32];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_of(p, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int ktiles = p.K / BK32;
    const int total = ktiles * p.nseg;

    f32x16 acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mi][ni][r] = 0.0f;

    float4 ra[2], rb[2];
    auto gload = [&](int t) {
        const int seg = t / ktiles, kt = t - seg * ktiles;
        const float* X = static_cast<const float*>(p.X[seg]) + (size_t)m0 * p.ldx + kt * BK32;
        const float* Z = static_cast<const float*>(p.Z[seg]) + (size_t)n0 * p.ldz + kt * BK32;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int c = tid + 256 * i, row = c >> 2, kc = c & 3;
            ra[i] = *reinterpret_cast<const float4*>(X + (size_t)row * p.ldx + kc * 4);
            rb[i] = *reinterpret_cast<const float4*>(Z + (size_t)row * p.ldz + kc * 4);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int c = tid + 256 * i, row = c >> 2, kc = c & 3;
            float* a = &sA[buf][row * LD32];
            float* b = &sB[buf][row * LD32];
            *reinterpret_cast<float2*>(a + 2 * kc) = make_float2(ra[i].x, ra[i].z);
            *reinterpret_cast<float2*>(a + 8 + 2 * kc) = make_float2(ra[i].y, ra[i].w);
            *reinterpret_cast<float2*>(b + 2 * kc) = make_float2(rb[i].x, rb[i].z);
            *reinterpret_cast<float2*>(b + 8 + 2 * kc) = make_float2(rb[i].y, rb[i].w);
        }
    };

    gload(0);
    sstore(0);
    __syncthreads();
    for (int t = 0; t < total; ++t) {
        const int buf = t & 1;
        if (t + 1 < total) gload(t + 1);
        float a[2][8], b[2][8];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
            const float* src = &sA[buf][(wm * 64 + mi * 32 + (lane & 31)) * LD32 + (lane >> 5) * 8];
            const float4 lo = *reinterpret_cast<const float4*>(src);
            const float4 hi = *reinterpret_cast<const float4*>(src + 4);
            a[mi][0] = lo.x; a[mi][1] = lo.y; a[mi][2] = lo.z; a[mi][3] = lo.w;
            a[mi][4] = hi.x; a[mi][5] = hi.y; a[mi][6] = hi.z; a[mi][7] = hi.w;
        }
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            const float* src = &sB[buf][(wn * 64 + ni * 32 + (lane & 31)) * LD32 + (lane >> 5) * 8];
            const float4 lo = *reinterpret_cast<const float4*>(src);
            const float4 hi = *reinterpret_cast<const float4*>(src + 4);
            b[ni][0] = lo.x; b[ni][1] = lo.y; b[ni][2] = lo.z; b[ni][3] = lo.w;
            b[ni][4] = hi.x; b[ni][5] = hi.y; b[ni][6] = hi.z; b[ni][7] = hi.w;
        }
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[mi][kk], b[ni][kk], acc[mi][ni], 0, 0, 0);
        if (t + 1 < total) sstore(buf ^ 1);
        __syncthreads();
    }
    store_tile<OUT>(p, acc, m0, n0, wm, wn, lane);
}

}  // namespace

int launch_gemm_nt(int is_bf16, int M, int N, int K, int ldx, int ldz, const GemmSegs& segs,
                   float alpha, int out_mode, float* C, int ldc, int m_valid, int n_valid,
                   uint16_t* C_hi, uint16_t* C_lo, int ld_split, hipStream_t s) {
    if (M % BM || N % BN || K % (is_bf16 ? BK16 : BK32) || segs.nseg < 1 || segs.nseg > kMaxSeg) {
        set_error("launch_gemm_nt: shape not a multiple of the tile or bad segment count");
        return GOAT_EINVAL;
    }
    GemmParams p{};
    for (int i = 0; i < segs.nseg; ++i) {
        p.X[i] = segs.X[i];
        p.Z[i] = segs.Z[i];
    }
    p.nseg = segs.nseg;
    p.K = K;
    p.ldx = ldx;
    p.ldz = ldz;
    p.alpha = alpha;
    p.C = C;
    p.ldc = ldc;
    p.m_valid = m_valid;
    p.n_valid = n_valid;
    p.Chi = C_hi;
    p.Clo = C_lo;
    p.ld_split = ld_split;
    p.tiles_m = M / BM;
    p.tiles_n = N / BN;
    dim3 grid(p.tiles_m * p.tiles_n), block(256);
    prof_begin(1, s);
    if (is_bf16) {
        if (out_mode == OUT_F32) hipLaunchKernelGGL(gemm_nt_bf16_kernel<OUT_F32>, grid, block, 0, s, p);
        else hipLaunchKernelGGL(gemm_nt_bf16_kernel<OUT_BF16_SPLIT>, grid, block, 0, s, p);
    } else {
        if (out_mode == OUT_F32) hipLaunchKernelGGL(gemm_nt_f32_kernel<OUT_F32>, grid, block, 0, s, p);
        else hipLaunchKernelGGL(gemm_nt_f32_kernel<OUT_BF16_SPLIT>, grid, block, 0, s, p);
    }
    prof_end(1, s);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

}  // namespace goat
