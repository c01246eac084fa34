// Operand packing: caller float32 n x n (leading dimension ld) -> internal
// zero-padded np x np planes, optionally transposed, as float32, bf16, a
// bf16 hi + lo split (hi = bf16(x), lo = bf16(x - hi)), or FP8 E4M3 (for
// operands it represents exactly, such as 0/1 adjacency). Also the FP8
// three-term split of a dense operand and the max |x| it is scaled by.
#include "common.h"

namespace goat {
namespace {

template <int MODE>
__device__ inline void put(void* hi, void* lo, size_t idx, float x) {
    if (MODE == PACK_F32) {
        static_cast<float*>(hi)[idx] = x;
    } else if (MODE == PACK_FP8) {
        static_cast<uint8_t*>(hi)[idx] = f32_to_e4m3_rne(x);
    } else {
        uint16_t h = f32_to_bf16_rne(x);
        static_cast<uint16_t*>(hi)[idx] = h;
        if (MODE == PACK_BF16_SPLIT) static_cast<uint16_t*>(lo)[idx] = f32_to_bf16_rne(x - bf16_to_f32(h));
    }
}

// One 64 x 64 destination tile per block; 256 threads, 16 elements each.
template <int MODE, bool TR>
__global__ __launch_bounds__(256) void pack_kernel(const float* __restrict__ src, int ld, int n,
                                                   int np, void* hi, void* lo) {
    __shared__ float tile[64][65];
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    if (!TR) {
        for (int r = ty; r < 64; r += 4) {
            const int i = r0 + r, j = c0 + tx;
            float x = (i < n && j < n) ? src[(size_t)i * ld + j] : 0.0f;
            put<MODE>(hi, lo, (size_t)i * np + j, x);
        }
    } else {
        // destination (r0 + r, c0 + c) = source (c0 + c, r0 + r)
        for (int r = ty; r < 64; r += 4) {
            const int si = c0 + r, sj = r0 + tx;
            tile[r][tx] = (si < n && sj < n) ? src[(size_t)si * ld + sj] : 0.0f;
        }
        __syncthreads();
        for (int r = ty; r < 64; r += 4) {
            put<MODE>(hi, lo, (size_t)(r0 + r) * np + c0 + tx, tile[tx][r]);
        }
    }
}

constexpr int kRT = 256;

__device__ inline float block_max256(float m, float* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    return fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
}

__global__ __launch_bounds__(kRT) void absmax_rect_kernel(int rows, int cols, const float* __restrict__ src,
                                                          int ld, float* partial) {
    __shared__ float sh[4];
    float m = 0.0f;
    for (int i = blockIdx.x; i < rows; i += gridDim.x) {
        const float* r = src + (size_t)i * ld;
        for (int j = threadIdx.x; j < cols; j += kRT) m = fmaxf(m, fabsf(r[j]));
    }
    m = block_max256(m, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ __launch_bounds__(kRT) void absmax_final_kernel(int nb, const float* partial, float* out) {
    __shared__ float sh[4];
    float m = 0.0f;
    for (int b = threadIdx.x; b < nb; b += kRT) m = fmaxf(m, partial[b]);
    m = block_max256(m, sh);
    if (threadIdx.x == 0) *out = m;
}

// One row per block. The residual of each term is exact in float32 (it is
// the difference of x and a nearby value with 4 significant bits), and the
// factor 16 keeps every term within the E4M3 range.
__global__ __launch_bounds__(kRT) void split_fp8_kernel(int rows, int cols, int np, const float* __restrict__ src,
                                                        int ld, const float* absmax, uint8_t* planes,
                                                        size_t plane_bytes) {
    const int i = blockIdx.x;
    const int s = fp8_split_exponent(*absmax);
    for (int j = threadIdx.x; j < np; j += kRT) {
        float r = (i < rows && j < cols) ? ldexpf(src[(size_t)i * ld + j], s) : 0.0f;
#pragma unroll
        for (int t = 0; t < kFp8Terms; ++t) {
            const uint8_t c = f32_to_e4m3_rne(r);
            planes[(size_t)t * plane_bytes + (size_t)i * np + j] = c;
            r = (r - e4m3_to_f32(c)) * (float)(1 << kFp8TermShift);
        }
    }
}

}  // namespace

int launch_absmax_rect(int rows, int cols, const float* src, int ld, float* partial, float* out, hipStream_t s) {
    const int nb = rows < kRedWG ? (rows > 0 ? rows : 1) : kRedWG;
    hipLaunchKernelGGL(absmax_rect_kernel, dim3(nb), dim3(kRT), 0, s, rows, cols, src, ld, partial);
    hipLaunchKernelGGL(absmax_final_kernel, dim3(1), dim3(kRT), 0, s, nb, (const float*)partial, out);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int launch_split_fp8(int rows, int cols, int prow, int np, const float* src, int ld, const float* absmax,
                     uint8_t* planes, size_t plane_bytes, hipStream_t s) {
    if (prow < rows || np < cols) {
        set_error("launch_split_fp8: padded shape smaller than the block");
        return GOAT_EINVAL;
    }
    hipLaunchKernelGGL(split_fp8_kernel, dim3(prow), dim3(kRT), 0, s, rows, cols, np, src, ld, absmax, planes,
                       plane_bytes);
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

int launch_pack(const float* src, int ld, int n, int np, int transpose, int mode, void* dst_hi,
                void* dst_lo, hipStream_t s) {
    dim3 grid(np / 64, np / 64), block(256);
#define GOAT_PACK_CASE(M, T) \
    hipLaunchKernelGGL((pack_kernel<M, T>), grid, block, 0, s, src, ld, n, np, dst_hi, dst_lo)
    if (mode == PACK_F32) {
        if (transpose) GOAT_PACK_CASE(PACK_F32, true); else GOAT_PACK_CASE(PACK_F32, false);
    } else if (mode == PACK_BF16) {
        if (transpose) GOAT_PACK_CASE(PACK_BF16, true); else GOAT_PACK_CASE(PACK_BF16, false);
    } else if (mode == PACK_FP8) {
        if (transpose) GOAT_PACK_CASE(PACK_FP8, true); else GOAT_PACK_CASE(PACK_FP8, false);
    } else {
        if (transpose) GOAT_PACK_CASE(PACK_BF16_SPLIT, true); else GOAT_PACK_CASE(PACK_BF16_SPLIT, false);
    }
#undef GOAT_PACK_CASE
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

}  // namespace goat
