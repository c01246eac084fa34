// Dense "NT" products on the gfx950 matrix cores:
//     C[i][j] = alpha * sum_s sum_k X_s[i][k] * Z_s[j][k]
// X_s and Z_s are row-major with the contraction index contiguous, so both
// MFMA operands are read along k. The segments s concatenate contractions
// (hi/lo precision terms, or the two gradient terms of a general pair).
// Operands are zero-padded internal planes: M, N multiples of 128 and K a
// multiple of the k-tile, so the main loop has no bounds checks.
//
// Block tile 128 x 128, four waves in a 2 x 2 arrangement, each wave a
// 64 x 64 sub-tile made of 2 x 2 MFMA 32x32 blocks (fp32 and fp8 products;
// bf16 products use the 256 x 256 eight-wave tile below when the shape is a
// multiple of it). Double-buffered LDS stages with register-staged global
// loads (one barrier per k-tile).
#include <cstdlib>
#include <cstring>

#include "common.h"

namespace goat {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 128, BN = 128;

struct GemmParams {
    const void* X[kMaxSeg];
    const void* Z[kMaxSeg];
    int zterm[kMaxSeg];
    const float* zmax;
    int nseg, K, ldx, ldz;
    float alpha;
    float* C;
    int ldc, m_valid, n_valid;
    uint16_t* Chi;
    uint16_t* Clo;
    int ld_split;
    int tiles_m, tiles_n;
    int m_off;                   // first output row of this launch
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
    const int m0 = p.m_off + tm * BM, n0 = tn * BN;
    const int ktiles = p.K / BK16;
    const int total = ktiles * p.nseg;

    f32x16 acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mi][ni][r] = 0.0f;

    // global -> register staging of one k-tile: 128 rows x 64 bf16 per
    // operand, four 16-byte chunks per thread (row = c / 8, chunk = c % 8)
    uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
    const int lrow = tid >> 3, lkc = (tid & 7) * 8;
#define GOAT_GLOAD16(T)                                                                          \
    do {                                                                                          \
        const int seg_ = (T) / ktiles, kt_ = (T) - seg_ * ktiles;                                 \
        const uint16_t* X_ = static_cast<const uint16_t*>(p.X[seg_]) +                            \
                             (size_t)(m0 + lrow) * p.ldx + kt_ * BK16 + lkc;                     \
        const uint16_t* Z_ = static_cast<const uint16_t*>(p.Z[seg_]) +                            \
                             (size_t)(n0 + lrow) * p.ldz + kt_ * BK16 + lkc;                     \
        const size_t sx_ = (size_t)32 * p.ldx, sz_ = (size_t)32 * p.ldz;                          \
        ra0 = *reinterpret_cast<const uint4*>(X_);                                                \
        ra1 = *reinterpret_cast<const uint4*>(X_ + sx_);                                          \
        ra2 = *reinterpret_cast<const uint4*>(X_ + 2 * sx_);                                      \
        ra3 = *reinterpret_cast<const uint4*>(X_ + 3 * sx_);                                      \
        rb0 = *reinterpret_cast<const uint4*>(Z_);                                                \
        rb1 = *reinterpret_cast<const uint4*>(Z_ + sz_);                                          \
        rb2 = *reinterpret_cast<const uint4*>(Z_ + 2 * sz_);                                      \
        rb3 = *reinterpret_cast<const uint4*>(Z_ + 3 * sz_);                                      \
    } while (0)
#define GOAT_SSTORE16(BUF)                                                                        \
    do {                                                                                          \
        uint16_t* a_ = &sA[BUF][lrow * LD16 + lkc];                                               \
        uint16_t* b_ = &sB[BUF][lrow * LD16 + lkc];                                               \
        *reinterpret_cast<uint4*>(a_) = ra0;                                                      \
        *reinterpret_cast<uint4*>(a_ + 32 * LD16) = ra1;                                          \
        *reinterpret_cast<uint4*>(a_ + 64 * LD16) = ra2;                                          \
        *reinterpret_cast<uint4*>(a_ + 96 * LD16) = ra3;                                          \
        *reinterpret_cast<uint4*>(b_) = rb0;                                                      \
        *reinterpret_cast<uint4*>(b_ + 32 * LD16) = rb1;                                          \
        *reinterpret_cast<uint4*>(b_ + 64 * LD16) = rb2;                                          \
        *reinterpret_cast<uint4*>(b_ + 96 * LD16) = rb3;                                          \
    } while (0)

    GOAT_GLOAD16(0);
    GOAT_SSTORE16(0);
    __syncthreads();
    const int arow = (wm * 64 + (lane & 31)) * LD16 + (lane >> 5) * 8;
    const int brow = (wn * 64 + (lane & 31)) * LD16 + (lane >> 5) * 8;
    for (int t = 0; t < total; ++t) {
        const int buf = t & 1;
        if (t + 1 < total) GOAT_GLOAD16(t + 1);
        const uint16_t* sa = sA[buf];
        const uint16_t* sb = sB[buf];
#pragma unroll
        for (int ks = 0; ks < BK16 / 16; ++ks) {
            const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(sa + arow + ks * 16);
            const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(sa + arow + 32 * LD16 + ks * 16);
            const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(sb + brow + ks * 16);
            const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(sb + brow + 32 * LD16 + ks * 16);
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
        }
        if (t + 1 < total) GOAT_SSTORE16(buf ^ 1);
        __syncthreads();
    }
#undef GOAT_GLOAD16
#undef GOAT_SSTORE16
    store_tile<OUT>(p, acc, m0, n0, wm, wn, lane);
}

// ------------------------------------------------------------------ fp8

// FP8 E4M3 operands (one byte per element), same block and wave tiles as
// the bf16 kernel; a k-tile is 128 bytes = 128 elements, so a stage moves the
// same bytes as a bf16 stage but covers twice the contraction. Each wave
// step is v_mfma_scale_f32_32x32x64_f8f6f4: lane l supplies 32 consecutive k
// of row l % 32 (lane halves take k and k + 32) for both operands, and the
// E8M0 scale of the Z operand undoes segment s's split factor
// 2^(e + 4 zterm[s]) exactly (X operands are exact, scale 2^0).
constexpr int BK8 = 128;                 // k-tile (bytes = elements)
constexpr int LD8 = BK8 + 16;            // LDS row stride (bytes), 16 B pad

template <int OUT>
__global__ __launch_bounds__(256) void gemm_nt_fp8_kernel(GemmParams p) {
    __shared__ __attribute__((aligned(16))) uint8_t sA[2][BM * LD8];
    __shared__ __attribute__((aligned(16))) uint8_t sB[2][BN * LD8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_of(p, tm, tn);
    const int m0 = p.m_off + tm * BM, n0 = tn * BN;
    const int ktiles = p.K / BK8;
    const int total = ktiles * p.nseg;
    const int zexp = fp8_split_exponent(*p.zmax);

    f32x16 acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mi][ni][r] = 0.0f;

    // global -> register staging of one k-tile: 128 rows x 128 bytes per
    // operand, four 16-byte chunks per thread (row = c / 8, chunk = c % 8)
    uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
    const int lrow = tid >> 3, lkc = (tid & 7) * 16;
#define GOAT_GLOAD8(T)                                                                            \
    do {                                                                                          \
        const int seg_ = (T) / ktiles, kt_ = (T) - seg_ * ktiles;                                 \
        const uint8_t* X_ = static_cast<const uint8_t*>(p.X[seg_]) +                              \
                            (size_t)(m0 + lrow) * p.ldx + kt_ * BK8 + lkc;                       \
        const uint8_t* Z_ = static_cast<const uint8_t*>(p.Z[seg_]) +                              \
                            (size_t)(n0 + lrow) * p.ldz + kt_ * BK8 + lkc;                       \
        const size_t sx_ = (size_t)32 * p.ldx, sz_ = (size_t)32 * p.ldz;                          \
        ra0 = *reinterpret_cast<const uint4*>(X_);                                                \
        ra1 = *reinterpret_cast<const uint4*>(X_ + sx_);                                          \
        ra2 = *reinterpret_cast<const uint4*>(X_ + 2 * sx_);                                      \
        ra3 = *reinterpret_cast<const uint4*>(X_ + 3 * sx_);                                      \
        rb0 = *reinterpret_cast<const uint4*>(Z_);                                                \
        rb1 = *reinterpret_cast<const uint4*>(Z_ + sz_);                                          \
        rb2 = *reinterpret_cast<const uint4*>(Z_ + 2 * sz_);                                      \
        rb3 = *reinterpret_cast<const uint4*>(Z_ + 3 * sz_);                                      \
    } while (0)
#define GOAT_SSTORE8(BUF)                                                                         \
    do {                                                                                          \
        uint8_t* a_ = &sA[BUF][lrow * LD8 + lkc];                                                 \
        uint8_t* b_ = &sB[BUF][lrow * LD8 + lkc];                                                 \
        *reinterpret_cast<uint4*>(a_) = ra0;                                                      \
        *reinterpret_cast<uint4*>(a_ + 32 * LD8) = ra1;                                           \
        *reinterpret_cast<uint4*>(a_ + 64 * LD8) = ra2;                                           \
        *reinterpret_cast<uint4*>(a_ + 96 * LD8) = ra3;                                           \
        *reinterpret_cast<uint4*>(b_) = rb0;                                                      \
        *reinterpret_cast<uint4*>(b_ + 32 * LD8) = rb1;                                           \
        *reinterpret_cast<uint4*>(b_ + 64 * LD8) = rb2;                                           \
        *reinterpret_cast<uint4*>(b_ + 96 * LD8) = rb3;                                           \
    } while (0)

    GOAT_GLOAD8(0);
    GOAT_SSTORE8(0);
    __syncthreads();
    const int arow = (wm * 64 + (lane & 31)) * LD8 + (lane >> 5) * 32;
    const int brow = (wn * 64 + (lane & 31)) * LD8 + (lane >> 5) * 32;
    for (int t = 0; t < total; ++t) {
        const int buf = t & 1;
        const int zscale = 127 - zexp - kFp8TermShift * p.zterm[t / ktiles];
        if (t + 1 < total) GOAT_GLOAD8(t + 1);
        const uint8_t* sa = sA[buf];
        const uint8_t* sb = sB[buf];
#pragma unroll
        for (int ks = 0; ks < BK8 / 64; ++ks) {
            const i32x8 a0 = *reinterpret_cast<const i32x8*>(sa + arow + ks * 64);
            const i32x8 a1 = *reinterpret_cast<const i32x8*>(sa + arow + 32 * LD8 + ks * 64);
            const i32x8 b0 = *reinterpret_cast<const i32x8*>(sb + brow + ks * 64);
            const i32x8 b1 = *reinterpret_cast<const i32x8*>(sb + brow + 32 * LD8 + ks * 64);
            acc[0][0] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a0, b0, acc[0][0], 0, 0, 0, 127, 0, zscale);
            acc[0][1] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a0, b1, acc[0][1], 0, 0, 0, 127, 0, zscale);
            acc[1][0] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a1, b0, acc[1][0], 0, 0, 0, 127, 0, zscale);
            acc[1][1] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a1, b1, acc[1][1], 0, 0, 0, 127, 0, zscale);
        }
        if (t + 1 < total) GOAT_SSTORE8(buf ^ 1);
        __syncthreads();
    }
#undef GOAT_GLOAD8
#undef GOAT_SSTORE8
    store_tile<OUT>(p, acc, m0, n0, wm, wn, lane);
}

// FP8 products whose segments come in groups of kFp8Terms = 3 that share X
// and take the three terms of a split Z (segment 3 g + t: X_g, Z term t):
// per 64-wide k slice the tiles X_g, Z_t0, Z_t1, Z_t2 are staged once, so a
// wave reads 8 fragments for 12 MFMAs instead of 12. Tiles are stored
// without padding, the four 16-byte chunks of a row XOR-swizzled with bits
// 2..3 of the row, so the sixteen rows a group of lanes reads at one chunk
// column fall on disjoint banks (a lane's 32-byte fragment is read as two
// chunks). Two stages of 32 KB: two blocks per compute unit.
constexpr int BKF8 = 64;                                              // k slice (bytes)
constexpr size_t kTileF8 = (size_t)BM * BKF8;                         // bytes per operand tile
constexpr size_t kLdsF8 = (size_t)2 * 4 * kTileF8;

__device__ inline int f8_chunk(int r, int c) { return r * BKF8 + ((c ^ ((r >> 2) & 3)) << 4); }

// the 32-byte fragment of row r, k half h (chunks 2h and 2h + 1)
__device__ inline i32x8 f8_frag(const uint8_t* tile, int r, int h) {
    const uint4 lo = *reinterpret_cast<const uint4*>(tile + f8_chunk(r, 2 * h));
    const uint4 hi = *reinterpret_cast<const uint4*>(tile + f8_chunk(r, 2 * h + 1));
    i32x8 v;
    v[0] = (int)lo.x; v[1] = (int)lo.y; v[2] = (int)lo.z; v[3] = (int)lo.w;
    v[4] = (int)hi.x; v[5] = (int)hi.y; v[6] = (int)hi.z; v[7] = (int)hi.w;
    return v;
}

template <int OUT>
__global__ __launch_bounds__(256) void gemm_nt_fp8_f3_kernel(GemmParams p) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smemf8[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_of(p, tm, tn);
    const int m0 = p.m_off + tm * BM, n0 = tn * BN;
    const int ktiles = p.K / BKF8;
    const int total = ktiles * (p.nseg / kFp8Terms);
    const int zexp = fp8_split_exponent(*p.zmax);
    int zscale[kFp8Terms];
#pragma unroll
    for (int t = 0; t < kFp8Terms; ++t) zscale[t] = 127 - zexp - kFp8TermShift * t;

    f32x16 acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mi][ni][r] = 0.0f;

    // staging: 16-byte pieces tid and tid + 256 of each tile, i.e. rows
    // tid / 4 and tid / 4 + 64, piece tid % 4 (bytes 16 (tid % 4) ..)
    const int lrow = tid >> 2, lp = tid & 3;
    const size_t xr0 = (size_t)(m0 + lrow) * p.ldx, xr1 = xr0 + (size_t)64 * p.ldx;
    const size_t zr0 = (size_t)(n0 + lrow) * p.ldz, zr1 = zr0 + (size_t)64 * p.ldz;
    uint4 s0, s1, s2, s3, s4, s5, s6, s7;
#define GOAT_GLOADF8(T)                                                                           \
    do {                                                                                          \
        const int g_ = (T) / ktiles, kt_ = (T) - g_ * ktiles;                                     \
        const size_t k_ = (size_t)kt_ * BKF8 + lp * 16;                                           \
        const uint8_t* X_ = static_cast<const uint8_t*>(p.X[kFp8Terms * g_]);                     \
        const uint8_t* Z0_ = static_cast<const uint8_t*>(p.Z[kFp8Terms * g_]);                    \
        const uint8_t* Z1_ = static_cast<const uint8_t*>(p.Z[kFp8Terms * g_ + 1]);                \
        const uint8_t* Z2_ = static_cast<const uint8_t*>(p.Z[kFp8Terms * g_ + 2]);                \
        s0 = *reinterpret_cast<const uint4*>(X_ + xr0 + k_);                                      \
        s1 = *reinterpret_cast<const uint4*>(X_ + xr1 + k_);                                      \
        s2 = *reinterpret_cast<const uint4*>(Z0_ + zr0 + k_);                                     \
        s3 = *reinterpret_cast<const uint4*>(Z0_ + zr1 + k_);                                     \
        s4 = *reinterpret_cast<const uint4*>(Z1_ + zr0 + k_);                                     \
        s5 = *reinterpret_cast<const uint4*>(Z1_ + zr1 + k_);                                     \
        s6 = *reinterpret_cast<const uint4*>(Z2_ + zr0 + k_);                                     \
        s7 = *reinterpret_cast<const uint4*>(Z2_ + zr1 + k_);                                     \
    } while (0)
    const int so0 = f8_chunk(lrow, lp), so1 = f8_chunk(lrow + 64, lp);
#define GOAT_SSTOREF8(BUF)                                                                        \
    do {                                                                                          \
        uint8_t* b_ = smemf8 + (size_t)(BUF) * 4 * kTileF8;                                       \
        *reinterpret_cast<uint4*>(b_ + so0) = s0;                                                 \
        *reinterpret_cast<uint4*>(b_ + so1) = s1;                                                 \
        *reinterpret_cast<uint4*>(b_ + kTileF8 + so0) = s2;                                       \
        *reinterpret_cast<uint4*>(b_ + kTileF8 + so1) = s3;                                       \
        *reinterpret_cast<uint4*>(b_ + 2 * kTileF8 + so0) = s4;                                   \
        *reinterpret_cast<uint4*>(b_ + 2 * kTileF8 + so1) = s5;                                   \
        *reinterpret_cast<uint4*>(b_ + 3 * kTileF8 + so0) = s6;                                   \
        *reinterpret_cast<uint4*>(b_ + 3 * kTileF8 + so1) = s7;                                   \
    } while (0)

    GOAT_GLOADF8(0);
    GOAT_SSTOREF8(0);
    __syncthreads();
    // fragments: rows wm*64 + 32 i + lane % 32 (X) and wn*64 + 32 i + lane % 32
    // (Z), 32 bytes from half lane / 32 of the slice
    const int ar = wm * 64 + (lane & 31), br = wn * 64 + (lane & 31), hf = lane >> 5;
    for (int t = 0; t < total; ++t) {
        const int buf = t & 1;
        if (t + 1 < total) GOAT_GLOADF8(t + 1);
        const uint8_t* sx = smemf8 + (size_t)buf * 4 * kTileF8;
        i32x8 a[2], b[kFp8Terms][2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = f8_frag(sx, ar + 32 * i, hf);
#pragma unroll
        for (int z = 0; z < kFp8Terms; ++z)
#pragma unroll
            for (int i = 0; i < 2; ++i) b[z][i] = f8_frag(sx + (z + 1) * kTileF8, br + 32 * i, hf);
#pragma unroll
        for (int z = 0; z < kFp8Terms; ++z)
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[mi], b[z][ni], acc[mi][ni], 0, 0,
                                                                                  0, 127, 0, zscale[z]);
        if (t + 1 < total) GOAT_SSTOREF8(buf ^ 1);
        __syncthreads();
    }
#undef GOAT_GLOADF8
#undef GOAT_SSTOREF8
    store_tile<OUT>(p, acc, m0, n0, wm, wn, lane);
}

// ------------------------------------------------------------------ bf16, 256 x 256

// Block tile 256 x 256 with four waves, each owning a 128 x 128 sub-tile
// (4 x 4 MFMA 32x32 blocks: 256 accumulator registers, held in the
// accumulation register file). Per 32-wide k-tile a wave reads 16 KB of
// operands from LDS for 32 MFMAs - half the LDS bytes per MFMA of the
// 128 x 128 tile, whose LDS reads and writes outlast its MFMAs. Two LDS
// stages (80 KB), one barrier per k-tile; the next k-tile's global loads
// (four 16-byte chunks per operand and thread, 64 contiguous bytes per
// row) are in flight during the current tile's MFMAs.
constexpr int BM2 = 256, BN2 = 256, BK2 = 32, LD2 = BK2 + 8;
constexpr size_t kLds256 = (size_t)2 * 2 * BM2 * LD2 * sizeof(uint16_t);

template <int OUT>
__device__ inline void store_tile_256(const GemmParams& p, const f32x16 (&acc)[4][4], int m0, int n0, int wm,
                                      int wn, int lane) {
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm * 128 + mi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int col = n0 + wn * 128 + ni * 32 + (lane & 31);
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

template <int OUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void gemm_nt_bf16_256_kernel(GemmParams p) {
    extern __shared__ __attribute__((aligned(16))) uint16_t smem16[];
    uint16_t* sA = smem16;                       // [2][BM2 * LD2]
    uint16_t* sB = smem16 + 2 * BM2 * LD2;       // [2][BN2 * LD2]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_of(p, tm, tn);
    const int m0 = p.m_off + tm * BM2, n0 = tn * BN2;
    const int ktiles = p.K / BK2;
    const int total = ktiles * p.nseg;

    f32x16 acc[4][4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mi][ni][r] = 0.0f;

    // chunk q of a thread: row tid / 4 + 64 q, bf16 columns (tid % 4) * 8 .. + 7
    // (named registers: an array here ends up in scratch memory)
    uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
    const int lrow = tid >> 2, lkc = (tid & 3) * 8;
#define GOAT_GLOAD256(T)                                                                          \
    do {                                                                                          \
        const int seg_ = (T) / ktiles, kt_ = (T) - seg_ * ktiles;                                 \
        const uint16_t* X_ = static_cast<const uint16_t*>(p.X[seg_]) +                            \
                             (size_t)(m0 + lrow) * p.ldx + kt_ * BK2 + lkc;                      \
        const uint16_t* Z_ = static_cast<const uint16_t*>(p.Z[seg_]) +                            \
                             (size_t)(n0 + lrow) * p.ldz + kt_ * BK2 + lkc;                      \
        const size_t sx_ = (size_t)64 * p.ldx, sz_ = (size_t)64 * p.ldz;                          \
        ra0 = *reinterpret_cast<const uint4*>(X_);                                                \
        ra1 = *reinterpret_cast<const uint4*>(X_ + sx_);                                          \
        ra2 = *reinterpret_cast<const uint4*>(X_ + 2 * sx_);                                      \
        ra3 = *reinterpret_cast<const uint4*>(X_ + 3 * sx_);                                      \
        rb0 = *reinterpret_cast<const uint4*>(Z_);                                                \
        rb1 = *reinterpret_cast<const uint4*>(Z_ + sz_);                                          \
        rb2 = *reinterpret_cast<const uint4*>(Z_ + 2 * sz_);                                      \
        rb3 = *reinterpret_cast<const uint4*>(Z_ + 3 * sz_);                                      \
    } while (0)
#define GOAT_SSTORE256(BUF)                                                                       \
    do {                                                                                          \
        uint16_t* a_ = sA + (BUF) * BM2 * LD2 + lrow * LD2 + lkc;                                 \
        uint16_t* b_ = sB + (BUF) * BN2 * LD2 + lrow * LD2 + lkc;                                 \
        *reinterpret_cast<uint4*>(a_) = ra0;                                                      \
        *reinterpret_cast<uint4*>(a_ + 64 * LD2) = ra1;                                           \
        *reinterpret_cast<uint4*>(a_ + 128 * LD2) = ra2;                                          \
        *reinterpret_cast<uint4*>(a_ + 192 * LD2) = ra3;                                          \
        *reinterpret_cast<uint4*>(b_) = rb0;                                                      \
        *reinterpret_cast<uint4*>(b_ + 64 * LD2) = rb1;                                           \
        *reinterpret_cast<uint4*>(b_ + 128 * LD2) = rb2;                                          \
        *reinterpret_cast<uint4*>(b_ + 192 * LD2) = rb3;                                          \
    } while (0)

    GOAT_GLOAD256(0);
    GOAT_SSTORE256(0);
    __syncthreads();
    const int arow = (wm * 128 + (lane & 31)) * LD2 + (lane >> 5) * 8;
    const int brow = (wn * 128 + (lane & 31)) * LD2 + (lane >> 5) * 8;
    for (int t = 0; t < total; ++t) {
        const int buf = t & 1;
        if (t + 1 < total) GOAT_GLOAD256(t + 1);
        const uint16_t* sa = sA + buf * BM2 * LD2;
        const uint16_t* sb = sB + buf * BN2 * LD2;
#pragma unroll
        for (int ks = 0; ks < BK2 / 16; ++ks) {
            bf16x8 a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = *reinterpret_cast<const bf16x8*>(sa + arow + i * 32 * LD2 + ks * 16);
                b[i] = *reinterpret_cast<const bf16x8*>(sb + brow + i * 32 * LD2 + ks * 16);
            }
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
            // one k-step's operands live at a time (hoisting all of them
            // would push the staging registers out to scratch)
            __builtin_amdgcn_sched_barrier(0);
        }
        if (t + 1 < total) GOAT_SSTORE256(buf ^ 1);
        __syncthreads();
    }
#undef GOAT_GLOAD256
#undef GOAT_SSTORE256
    store_tile_256<OUT>(p, acc, m0, n0, wm, wn, lane);
}

// 256 x 256 tile on eight waves (2 x 4), 128 x 64 per wave: per 16-wide
// k-step a wave reads six 16-byte fragments for eight MFMAs (43.7 flops per
// LDS byte against 32.8 for the 64 x 64 wave tile), and 128 accumulator
// registers leave room for two waves per SIMD. k-tile 64, two LDS stages of
// 72 KB; each thread stages four 16-byte chunks per operand.
constexpr int BM3 = 256, BN3 = 256, BK3 = 64, LD3 = BK3 + 8;
constexpr size_t kLdsW8 = (size_t)2 * 2 * BM3 * LD3 * sizeof(uint16_t);

template <int OUT>
__device__ inline void store_tile_w8(const GemmParams& p, const f32x16 (&acc)[4][2], int m0, int n0, int wm,
                                     int wn, int lane) {
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm * 128 + mi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
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

template <int OUT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void gemm_nt_bf16_w8_kernel(GemmParams p) {
    extern __shared__ __attribute__((aligned(16))) uint16_t smem16w[];
    uint16_t* sA = smem16w;                      // [2][BM3 * LD3]
    uint16_t* sB = smem16w + 2 * BM3 * LD3;      // [2][BN3 * LD3]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 2, wn = wave & 3;
    int tm, tn;
    tile_of(p, tm, tn);
    const int m0 = p.m_off + tm * BM3, n0 = tn * BN3;
    const int ktiles = p.K / BK3;
    const int total = ktiles * p.nseg;

    f32x16 acc[4][2];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mi][ni][r] = 0.0f;

    // chunk q of a thread: row tid / 8 + 64 q, bf16 columns (tid % 8) * 8 .. + 7
    uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
    const int lrow = tid >> 3, lkc = (tid & 7) * 8;
#define GOAT_GLOADW8(T)                                                                           \
    do {                                                                                          \
        const int seg_ = (T) / ktiles, kt_ = (T) - seg_ * ktiles;                                 \
        const uint16_t* X_ = static_cast<const uint16_t*>(p.X[seg_]) +                            \
                             (size_t)(m0 + lrow) * p.ldx + kt_ * BK3 + lkc;                      \
        const uint16_t* Z_ = static_cast<const uint16_t*>(p.Z[seg_]) +                            \
                             (size_t)(n0 + lrow) * p.ldz + kt_ * BK3 + lkc;                      \
        const size_t sx_ = (size_t)64 * p.ldx, sz_ = (size_t)64 * p.ldz;                          \
        ra0 = *reinterpret_cast<const uint4*>(X_);                                                \
        ra1 = *reinterpret_cast<const uint4*>(X_ + sx_);                                          \
        ra2 = *reinterpret_cast<const uint4*>(X_ + 2 * sx_);                                      \
        ra3 = *reinterpret_cast<const uint4*>(X_ + 3 * sx_);                                      \
        rb0 = *reinterpret_cast<const uint4*>(Z_);                                                \
        rb1 = *reinterpret_cast<const uint4*>(Z_ + sz_);                                          \
        rb2 = *reinterpret_cast<const uint4*>(Z_ + 2 * sz_);                                      \
        rb3 = *reinterpret_cast<const uint4*>(Z_ + 3 * sz_);                                      \
    } while (0)
#define GOAT_SSTOREW8(BUF)                                                                        \
    do {                                                                                          \
        uint16_t* a_ = sA + (BUF) * BM3 * LD3 + lrow * LD3 + lkc;                                 \
        uint16_t* b_ = sB + (BUF) * BN3 * LD3 + lrow * LD3 + lkc;                                 \
        *reinterpret_cast<uint4*>(a_) = ra0;                                                      \
        *reinterpret_cast<uint4*>(a_ + 64 * LD3) = ra1;                                           \
        *reinterpret_cast<uint4*>(a_ + 128 * LD3) = ra2;                                          \
        *reinterpret_cast<uint4*>(a_ + 192 * LD3) = ra3;                                          \
        *reinterpret_cast<uint4*>(b_) = rb0;                                                      \
        *reinterpret_cast<uint4*>(b_ + 64 * LD3) = rb1;                                           \
        *reinterpret_cast<uint4*>(b_ + 128 * LD3) = rb2;                                          \
        *reinterpret_cast<uint4*>(b_ + 192 * LD3) = rb3;                                          \
    } while (0)

    GOAT_GLOADW8(0);
    GOAT_SSTOREW8(0);
    __syncthreads();
    const int arow = (wm * 128 + (lane & 31)) * LD3 + (lane >> 5) * 8;
    const int brow = (wn * 64 + (lane & 31)) * LD3 + (lane >> 5) * 8;
    for (int t = 0; t < total; ++t) {
        const int buf = t & 1;
        if (t + 1 < total) GOAT_GLOADW8(t + 1);
        const uint16_t* sa = sA + buf * BM3 * LD3;
        const uint16_t* sb = sB + buf * BN3 * LD3;
#pragma unroll
        for (int ks = 0; ks < BK3 / 16; ++ks) {
            bf16x8 a[4], b[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const bf16x8*>(sa + arow + i * 32 * LD3 + ks * 16);
#pragma unroll
            for (int i = 0; i < 2; ++i) b[i] = *reinterpret_cast<const bf16x8*>(sb + brow + i * 32 * LD3 + ks * 16);
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
        }
        if (t + 1 < total) GOAT_SSTOREW8(buf ^ 1);
        __syncthreads();
    }
#undef GOAT_GLOADW8
#undef GOAT_SSTOREW8
    store_tile_w8<OUT>(p, acc, m0, n0, wm, wn, lane);
}

// Three-segment bf16 products X0 Z0 + X0 Z1 + X2 Z0 (the hi/lo split of
// both operands with the lo x lo term dropped) on the 256 x 256 eight-wave
// tile: the four operand tiles X0, X2, Z0, Z1 of a 32-wide k slice are
// staged once and feed all three segments, so per 16-wide k-step a wave
// reads 12 fragments for 24 MFMAs (18 when the segments run one after the
// other) and a barrier covers 48 MFMAs per wave. Tiles are stored without
// padding, their 16-byte chunks XOR-swizzled with bits 2..3 of the row so
// that the eight rows a group of lanes reads at one chunk column fall on
// disjoint banks. Two stages of 64 KB.
constexpr int BK4 = 32;
constexpr size_t kTileF3 = (size_t)BM3 * BK4;                        // bf16 per operand tile
constexpr size_t kLdsF3 = (size_t)2 * 4 * kTileF3 * sizeof(uint16_t);

__device__ inline int f3_off(int r, int c) { return r * BK4 + ((c ^ ((r >> 2) & 3)) << 3); }

template <int OUT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void gemm_nt_bf16_w8f3_kernel(GemmParams p) {
    extern __shared__ __attribute__((aligned(16))) uint16_t smemf3[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 2, wn = wave & 3;
    int tm, tn;
    tile_of(p, tm, tn);
    const int m0 = p.m_off + tm * BM3, n0 = tn * BN3;
    const int ktiles = p.K / BK4;
    const uint16_t* X0 = static_cast<const uint16_t*>(p.X[0]);
    const uint16_t* X2 = static_cast<const uint16_t*>(p.X[2]);
    const uint16_t* Z0 = static_cast<const uint16_t*>(p.Z[0]);
    const uint16_t* Z1 = static_cast<const uint16_t*>(p.Z[1]);

    f32x16 acc[4][2];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mi][ni][r] = 0.0f;

    // staging: chunks tid and tid + 512 of each tile, i.e. rows tid / 4 and
    // tid / 4 + 128, chunk tid % 4 (eight bf16)
    const int lrow = tid >> 2, lc = tid & 3;
    const size_t xr0 = (size_t)(m0 + lrow) * p.ldx, xr1 = xr0 + (size_t)128 * p.ldx;
    const size_t zr0 = (size_t)(n0 + lrow) * p.ldz, zr1 = zr0 + (size_t)128 * p.ldz;
    uint4 s0, s1, s2, s3, s4, s5, s6, s7;
#define GOAT_GLOADF3(T)                                                                           \
    do {                                                                                          \
        const size_t k_ = (size_t)(T) * BK4 + lc * 8;                                             \
        s0 = *reinterpret_cast<const uint4*>(X0 + xr0 + k_);                                      \
        s1 = *reinterpret_cast<const uint4*>(X0 + xr1 + k_);                                      \
        s2 = *reinterpret_cast<const uint4*>(X2 + xr0 + k_);                                      \
        s3 = *reinterpret_cast<const uint4*>(X2 + xr1 + k_);                                      \
        s4 = *reinterpret_cast<const uint4*>(Z0 + zr0 + k_);                                      \
        s5 = *reinterpret_cast<const uint4*>(Z0 + zr1 + k_);                                      \
        s6 = *reinterpret_cast<const uint4*>(Z1 + zr0 + k_);                                      \
        s7 = *reinterpret_cast<const uint4*>(Z1 + zr1 + k_);                                      \
    } while (0)
    const int so0 = f3_off(lrow, lc), so1 = f3_off(lrow + 128, lc);
#define GOAT_SSTOREF3(BUF)                                                                        \
    do {                                                                                          \
        uint16_t* b_ = smemf3 + (size_t)(BUF) * 4 * kTileF3;                                      \
        *reinterpret_cast<uint4*>(b_ + so0) = s0;                                                 \
        *reinterpret_cast<uint4*>(b_ + so1) = s1;                                                 \
        *reinterpret_cast<uint4*>(b_ + kTileF3 + so0) = s2;                                       \
        *reinterpret_cast<uint4*>(b_ + kTileF3 + so1) = s3;                                       \
        *reinterpret_cast<uint4*>(b_ + 2 * kTileF3 + so0) = s4;                                   \
        *reinterpret_cast<uint4*>(b_ + 2 * kTileF3 + so1) = s5;                                   \
        *reinterpret_cast<uint4*>(b_ + 3 * kTileF3 + so0) = s6;                                   \
        *reinterpret_cast<uint4*>(b_ + 3 * kTileF3 + so1) = s7;                                   \
    } while (0)

    GOAT_GLOADF3(0);
    GOAT_SSTOREF3(0);
    __syncthreads();
    // fragment rows of this lane: X rows wm*128 + 32 i + lane % 32, Z rows
    // wn*64 + 32 i + lane % 32; k chunk 2 ks + lane / 32 of the slice
    const int ar = wm * 128 + (lane & 31), br = wn * 64 + (lane & 31), kh = lane >> 5;
    for (int t = 0; t < ktiles; ++t) {
        const int buf = t & 1;
        if (t + 1 < ktiles) GOAT_GLOADF3(t + 1);
        const uint16_t* sx0 = smemf3 + (size_t)buf * 4 * kTileF3;
        const uint16_t* sx2 = sx0 + kTileF3;
        const uint16_t* sz0 = sx0 + 2 * kTileF3;
        const uint16_t* sz1 = sx0 + 3 * kTileF3;
#pragma unroll
        for (int ks = 0; ks < BK4 / 16; ++ks) {
            const int c = 2 * ks + kh;
            bf16x8 ah[4], al[4], bh[2], bl[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ah[i] = *reinterpret_cast<const bf16x8*>(sx0 + f3_off(ar + 32 * i, c));
                al[i] = *reinterpret_cast<const bf16x8*>(sx2 + f3_off(ar + 32 * i, c));
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                bh[i] = *reinterpret_cast<const bf16x8*>(sz0 + f3_off(br + 32 * i, c));
                bl[i] = *reinterpret_cast<const bf16x8*>(sz1 + f3_off(br + 32 * i, c));
            }
            // segment-major, so consecutive MFMAs on one accumulator are
            // eight apart
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[mi], bh[ni], acc[mi][ni], 0, 0, 0);
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[mi], bl[ni], acc[mi][ni], 0, 0, 0);
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[mi], bh[ni], acc[mi][ni], 0, 0, 0);
        }
        if (t + 1 < ktiles) GOAT_SSTOREF3(buf ^ 1);
        __syncthreads();
    }
#undef GOAT_GLOADF3
#undef GOAT_SSTOREF3
    store_tile_w8<OUT>(p, acc, m0, n0, wm, wn, lane);
}

// The same fusion on the 128 x 128 tile (four waves of 64 x 64): the last
// tile-rows of a large product and every three-segment product below the
// eight-wave shapes. Per 16-wide k-step a wave reads 8 fragments for 12
// MFMAs instead of 12; two stages of 32 KB.
constexpr size_t kTileF3s = (size_t)BM * BK4;                         // bf16 per operand tile
constexpr size_t kLdsF3s = (size_t)2 * 4 * kTileF3s * sizeof(uint16_t);

template <int OUT>
__global__ __launch_bounds__(256) void gemm_nt_bf16_f3_kernel(GemmParams p) {
    extern __shared__ __attribute__((aligned(16))) uint16_t smemf3s[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_of(p, tm, tn);
    const int m0 = p.m_off + tm * BM, n0 = tn * BN;
    const int ktiles = p.K / BK4;
    const uint16_t* X0 = static_cast<const uint16_t*>(p.X[0]);
    const uint16_t* X2 = static_cast<const uint16_t*>(p.X[2]);
    const uint16_t* Z0 = static_cast<const uint16_t*>(p.Z[0]);
    const uint16_t* Z1 = static_cast<const uint16_t*>(p.Z[1]);

    f32x16 acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mi][ni][r] = 0.0f;

    // staging: rows tid / 4 and tid / 4 + 64 of each tile, chunk tid % 4
    const int lrow = tid >> 2, lc = tid & 3;
    const size_t xr0 = (size_t)(m0 + lrow) * p.ldx, xr1 = xr0 + (size_t)64 * p.ldx;
    const size_t zr0 = (size_t)(n0 + lrow) * p.ldz, zr1 = zr0 + (size_t)64 * p.ldz;
    uint4 s0, s1, s2, s3, s4, s5, s6, s7;
#define GOAT_GLOADF3S(T)                                                                          \
    do {                                                                                          \
        const size_t k_ = (size_t)(T) * BK4 + lc * 8;                                             \
        s0 = *reinterpret_cast<const uint4*>(X0 + xr0 + k_);                                      \
        s1 = *reinterpret_cast<const uint4*>(X0 + xr1 + k_);                                      \
        s2 = *reinterpret_cast<const uint4*>(X2 + xr0 + k_);                                      \
        s3 = *reinterpret_cast<const uint4*>(X2 + xr1 + k_);                                      \
        s4 = *reinterpret_cast<const uint4*>(Z0 + zr0 + k_);                                      \
        s5 = *reinterpret_cast<const uint4*>(Z0 + zr1 + k_);                                      \
        s6 = *reinterpret_cast<const uint4*>(Z1 + zr0 + k_);                                      \
        s7 = *reinterpret_cast<const uint4*>(Z1 + zr1 + k_);                                      \
    } while (0)
    const int so0 = f3_off(lrow, lc), so1 = f3_off(lrow + 64, lc);
#define GOAT_SSTOREF3S(BUF)                                                                       \
    do {                                                                                          \
        uint16_t* b_ = smemf3s + (size_t)(BUF) * 4 * kTileF3s;                                    \
        *reinterpret_cast<uint4*>(b_ + so0) = s0;                                                 \
        *reinterpret_cast<uint4*>(b_ + so1) = s1;                                                 \
        *reinterpret_cast<uint4*>(b_ + kTileF3s + so0) = s2;                                      \
        *reinterpret_cast<uint4*>(b_ + kTileF3s + so1) = s3;                                      \
        *reinterpret_cast<uint4*>(b_ + 2 * kTileF3s + so0) = s4;                                  \
        *reinterpret_cast<uint4*>(b_ + 2 * kTileF3s + so1) = s5;                                  \
        *reinterpret_cast<uint4*>(b_ + 3 * kTileF3s + so0) = s6;                                  \
        *reinterpret_cast<uint4*>(b_ + 3 * kTileF3s + so1) = s7;                                  \
    } while (0)

    GOAT_GLOADF3S(0);
    GOAT_SSTOREF3S(0);
    __syncthreads();
    const int ar = wm * 64 + (lane & 31), br = wn * 64 + (lane & 31), kh = lane >> 5;
    for (int t = 0; t < ktiles; ++t) {
        const int buf = t & 1;
        if (t + 1 < ktiles) GOAT_GLOADF3S(t + 1);
        const uint16_t* sx0 = smemf3s + (size_t)buf * 4 * kTileF3s;
        const uint16_t* sx2 = sx0 + kTileF3s;
        const uint16_t* sz0 = sx0 + 2 * kTileF3s;
        const uint16_t* sz1 = sx0 + 3 * kTileF3s;
#pragma unroll
        for (int ks = 0; ks < BK4 / 16; ++ks) {
            const int c = 2 * ks + kh;
            bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                ah[i] = *reinterpret_cast<const bf16x8*>(sx0 + f3_off(ar + 32 * i, c));
                al[i] = *reinterpret_cast<const bf16x8*>(sx2 + f3_off(ar + 32 * i, c));
                bh[i] = *reinterpret_cast<const bf16x8*>(sz0 + f3_off(br + 32 * i, c));
                bl[i] = *reinterpret_cast<const bf16x8*>(sz1 + f3_off(br + 32 * i, c));
            }
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[mi], bh[ni], acc[mi][ni], 0, 0, 0);
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[mi], bl[ni], acc[mi][ni], 0, 0, 0);
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[mi], bh[ni], acc[mi][ni], 0, 0, 0);
        }
        if (t + 1 < ktiles) GOAT_SSTOREF3S(buf ^ 1);
        __syncthreads();
    }
#undef GOAT_GLOADF3S
#undef GOAT_SSTOREF3S
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
    const int m0 = p.m_off + tm * BM, n0 = tn * BN;
    const int ktiles = p.K / BK32;
    const int total = ktiles * p.nseg;

    f32x16 acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mi][ni][r] = 0.0f;

    // global -> register staging of one k-tile: 128 rows x 16 floats per
    // operand, two float4 per thread (row = c / 4, chunk = c % 4)
    float4 ra0, ra1, rb0, rb1;
    const int lrow = tid >> 2, lkc = tid & 3;
#define GOAT_GLOAD32(T)                                                                           \
    do {                                                                                          \
        const int seg_ = (T) / ktiles, kt_ = (T) - seg_ * ktiles;                                 \
        const float* X_ = static_cast<const float*>(p.X[seg_]) + (size_t)(m0 + lrow) * p.ldx +    \
                          kt_ * BK32 + lkc * 4;                                                  \
        const float* Z_ = static_cast<const float*>(p.Z[seg_]) + (size_t)(n0 + lrow) * p.ldz +    \
                          kt_ * BK32 + lkc * 4;                                                  \
        ra0 = *reinterpret_cast<const float4*>(X_);                                               \
        ra1 = *reinterpret_cast<const float4*>(X_ + (size_t)64 * p.ldx);                          \
        rb0 = *reinterpret_cast<const float4*>(Z_);                                               \
        rb1 = *reinterpret_cast<const float4*>(Z_ + (size_t)64 * p.ldz);                          \
    } while (0)
#define GOAT_PUT32(PTR, V)                                                                        \
    do {                                                                                          \
        *reinterpret_cast<float2*>((PTR) + 2 * lkc) = make_float2((V).x, (V).z);                  \
        *reinterpret_cast<float2*>((PTR) + 8 + 2 * lkc) = make_float2((V).y, (V).w);              \
    } while (0)
#define GOAT_SSTORE32(BUF)                                                                        \
    do {                                                                                          \
        float* a_ = &sA[BUF][lrow * LD32];                                                        \
        float* b_ = &sB[BUF][lrow * LD32];                                                        \
        GOAT_PUT32(a_, ra0);                                                                      \
        GOAT_PUT32(a_ + 64 * LD32, ra1);                                                          \
        GOAT_PUT32(b_, rb0);                                                                      \
        GOAT_PUT32(b_ + 64 * LD32, rb1);                                                          \
    } while (0)

    GOAT_GLOAD32(0);
    GOAT_SSTORE32(0);
    __syncthreads();
    const int arow = (wm * 64 + (lane & 31)) * LD32 + (lane >> 5) * 8;
    const int brow = (wn * 64 + (lane & 31)) * LD32 + (lane >> 5) * 8;
    for (int t = 0; t < total; ++t) {
        const int buf = t & 1;
        if (t + 1 < total) GOAT_GLOAD32(t + 1);
        const float* sa = sA[buf];
        const float* sb = sB[buf];
        const float4 a0l = *reinterpret_cast<const float4*>(sa + arow);
        const float4 a0h = *reinterpret_cast<const float4*>(sa + arow + 4);
        const float4 a1l = *reinterpret_cast<const float4*>(sa + arow + 32 * LD32);
        const float4 a1h = *reinterpret_cast<const float4*>(sa + arow + 32 * LD32 + 4);
        const float4 b0l = *reinterpret_cast<const float4*>(sb + brow);
        const float4 b0h = *reinterpret_cast<const float4*>(sb + brow + 4);
        const float4 b1l = *reinterpret_cast<const float4*>(sb + brow + 32 * LD32);
        const float4 b1h = *reinterpret_cast<const float4*>(sb + brow + 32 * LD32 + 4);
        const float a0[8] = {a0l.x, a0l.y, a0l.z, a0l.w, a0h.x, a0h.y, a0h.z, a0h.w};
        const float a1[8] = {a1l.x, a1l.y, a1l.z, a1l.w, a1h.x, a1h.y, a1h.z, a1h.w};
        const float b0[8] = {b0l.x, b0l.y, b0l.z, b0l.w, b0h.x, b0h.y, b0h.z, b0h.w};
        const float b1[8] = {b1l.x, b1l.y, b1l.z, b1l.w, b1h.x, b1h.y, b1h.z, b1h.w};
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[kk], b0[kk], acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[kk], b1[kk], acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[kk], b0[kk], acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[kk], b1[kk], acc[1][1], 0, 0, 0);
        }
        if (t + 1 < total) GOAT_SSTORE32(buf ^ 1);
        __syncthreads();
    }
#undef GOAT_GLOAD32
#undef GOAT_PUT32
#undef GOAT_SSTORE32
    store_tile<OUT>(p, acc, m0, n0, wm, wn, lane);
}

// bf16 products use the 256 x 256 tile on eight waves when the shape allows
// (1034 against 951 TFLOP/s executed for the 128 x 128 tile at n = 10,000;
// the 256 x 256 tile on four waves: 782, one wave per SIMD leaves its LDS and
// global latencies exposed). GOAT_GEMM_TILE = 128 or 256 selects the others
// (a measurement knob). An eight-wave fp8 tile does not fit: its 32-byte
// fragments push the registers past two waves per SIMD (spills; 1071
// against 1735 TFLOP/s).
int tile_choice(int M, int N, int K) {
    // bf16 products: 0: 128 x 128, 1: 256 x 256 on four waves, 2: 256 x 256
    // on eight waves
    static const int want = [] {
        const char* e = getenv("GOAT_GEMM_TILE");
        if (e && std::strcmp(e, "128") == 0) return 0;
        if (e && std::strcmp(e, "256") == 0) return 1;
        return 2;
    }();
    if (want == 0 || M % 256 || N % 256 || K % 64) return 0;
    static const bool lds_ok =
        hipFuncSetAttribute(reinterpret_cast<const void*>(gemm_nt_bf16_256_kernel<OUT_F32>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLds256) == hipSuccess &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(gemm_nt_bf16_256_kernel<OUT_BF16_SPLIT>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLds256) == hipSuccess &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(gemm_nt_bf16_w8_kernel<OUT_F32>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsW8) == hipSuccess &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(gemm_nt_bf16_w8_kernel<OUT_BF16_SPLIT>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsW8) == hipSuccess;
    return lds_ok ? want : 0;
}

// The fused fp8 kernel takes products whose segments come in groups of
// kFp8Terms sharing X, segment kFp8Terms g + t holding term t of Z
// (GOAT_GEMM_F3=0 keeps the segment-by-segment kernel).
bool fused_fp8_ok(const GemmSegs& segs, int K) {
    static const bool on = [] {
        const char* e = getenv("GOAT_GEMM_F3");
        return !(e && std::strcmp(e, "0") == 0);
    }();
    static const bool lds_ok = hipFuncSetAttribute(reinterpret_cast<const void*>(gemm_nt_fp8_f3_kernel<OUT_F32>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)kLdsF8) == hipSuccess;
    if (!on || !lds_ok || K % BKF8 || segs.nseg % kFp8Terms) return false;
    for (int sg = 0; sg < segs.nseg; ++sg)
        if (segs.X[sg] != segs.X[sg - sg % kFp8Terms] || segs.zterm[sg] != sg % kFp8Terms) return false;
    return true;
}

// The fused three-segment kernels take bf16 products whose segments are
// (X0, Z0), (X0, Z1), (X2, Z0), on either tile. GOAT_GEMM_F3=0 keeps the
// segment-by-segment kernels (a measurement knob).
bool fused3_pattern(const GemmSegs& segs, int K) {
    static const bool on = [] {
        const char* e = getenv("GOAT_GEMM_F3");
        return !(e && std::strcmp(e, "0") == 0);
    }();
    return on && segs.nseg == 3 && segs.X[0] == segs.X[1] && segs.Z[0] == segs.Z[2] && K % BK4 == 0;
}

bool fused3_ok(const GemmSegs& segs, int K) {
    static const bool lds_ok =
        hipFuncSetAttribute(reinterpret_cast<const void*>(gemm_nt_bf16_w8f3_kernel<OUT_F32>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsF3) == hipSuccess &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(gemm_nt_bf16_w8f3_kernel<OUT_BF16_SPLIT>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsF3) == hipSuccess;
    return lds_ok && fused3_pattern(segs, K);
}

}  // namespace

int launch_gemm_nt(int kind, int M, int N, int K, int ldx, int ldz, const GemmSegs& segs,
                   float alpha, int out_mode, float* C, int ldc, int m_valid, int n_valid,
                   uint16_t* C_hi, uint16_t* C_lo, int ld_split, hipStream_t s) {
    const bool is_bf16 = kind == GEMM_BF16, is_fp8 = kind == GEMM_FP8;
    const int bk = is_fp8 ? BK8 : (is_bf16 ? BK16 : BK32);
    if (is_fp8 && (!segs.zmax || out_mode != OUT_F32)) {
        set_error("launch_gemm_nt: fp8 products need the split maximum and fp32 output");
        return GOAT_EINVAL;
    }
    if (M % BM || N % BN || K % bk || segs.nseg < 1 || segs.nseg > kMaxSeg) {
        set_error("launch_gemm_nt: shape not a multiple of the tile or bad segment count");
        return GOAT_EINVAL;
    }
    GemmParams p{};
    for (int i = 0; i < segs.nseg; ++i) {
        p.X[i] = segs.X[i];
        p.Z[i] = segs.Z[i];
        p.zterm[i] = segs.zterm[i];
    }
    p.zmax = segs.zmax;
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
    int tile = is_bf16 ? tile_choice(M, N, K) : 0;
    // Eight-wave tiles run one block per compute unit. Whole tile-rows that
    // fill complete rounds go to them; the rows of a last, partial round go
    // to a second launch of the 128 x 128 kernel (four times as many
    // blocks); a product with fewer 256-tiles than compute units runs on
    // 128 x 128 tiles only.
    int rows_big = M;
    if (tile == 2) {
        const int tm2 = M / BM3, tn2 = N / BN3, cus = cu_count();
        const int nb = tm2 * tn2;
        if (nb < cus) {
            tile = 0;
        } else if (nb % cus != 0) {
            rows_big = (nb / cus * cus) / tn2 * BM3;
            if (rows_big == 0) tile = 0;
        }
    }
    p.m_off = 0;
    p.tiles_m = (tile ? rows_big : M) / (tile ? BM2 : BM);
    p.tiles_n = N / (tile ? BN2 : BN);
    dim3 grid(p.tiles_m * p.tiles_n), block(tile == 2 ? 512 : 256);
    prof_begin(1, s);
    if (tile == 2 && rows_big < M) {
        GemmParams q = p;
        q.m_off = rows_big;
        q.tiles_m = (M - rows_big) / BM;
        q.tiles_n = N / BN;
        const dim3 g2(q.tiles_m * q.tiles_n), b2(256);
        if (fused3_pattern(segs, K)) {
            if (out_mode == OUT_F32) hipLaunchKernelGGL(gemm_nt_bf16_f3_kernel<OUT_F32>, g2, b2, kLdsF3s, s, q);
            else hipLaunchKernelGGL(gemm_nt_bf16_f3_kernel<OUT_BF16_SPLIT>, g2, b2, kLdsF3s, s, q);
        } else if (out_mode == OUT_F32) {
            hipLaunchKernelGGL(gemm_nt_bf16_kernel<OUT_F32>, g2, b2, 0, s, q);
        } else {
            hipLaunchKernelGGL(gemm_nt_bf16_kernel<OUT_BF16_SPLIT>, g2, b2, 0, s, q);
        }
    }
    if (is_fp8 && fused_fp8_ok(segs, K)) {
        hipLaunchKernelGGL(gemm_nt_fp8_f3_kernel<OUT_F32>, grid, block, kLdsF8, s, p);
    } else if (is_fp8) {
        hipLaunchKernelGGL(gemm_nt_fp8_kernel<OUT_F32>, grid, block, 0, s, p);
    } else if (tile == 1) {
        if (out_mode == OUT_F32) hipLaunchKernelGGL(gemm_nt_bf16_256_kernel<OUT_F32>, grid, block, kLds256, s, p);
        else hipLaunchKernelGGL(gemm_nt_bf16_256_kernel<OUT_BF16_SPLIT>, grid, block, kLds256, s, p);
    } else if (tile == 2 && fused3_ok(segs, K)) {
        if (out_mode == OUT_F32) hipLaunchKernelGGL(gemm_nt_bf16_w8f3_kernel<OUT_F32>, grid, block, kLdsF3, s, p);
        else hipLaunchKernelGGL(gemm_nt_bf16_w8f3_kernel<OUT_BF16_SPLIT>, grid, block, kLdsF3, s, p);
    } else if (tile == 2) {
        if (out_mode == OUT_F32) hipLaunchKernelGGL(gemm_nt_bf16_w8_kernel<OUT_F32>, grid, block, kLdsW8, s, p);
        else hipLaunchKernelGGL(gemm_nt_bf16_w8_kernel<OUT_BF16_SPLIT>, grid, block, kLdsW8, s, p);
    } else if (is_bf16 && tile == 0 && fused3_pattern(segs, K)) {
        if (out_mode == OUT_F32) hipLaunchKernelGGL(gemm_nt_bf16_f3_kernel<OUT_F32>, grid, block, kLdsF3s, s, p);
        else hipLaunchKernelGGL(gemm_nt_bf16_f3_kernel<OUT_BF16_SPLIT>, grid, block, kLdsF3s, s, p);
    } else if (is_bf16) {
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
