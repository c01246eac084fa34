// Operand packing: caller float32 n x n (leading dimension ld) -> internal
// zero-padded np x np planes, optionally transposed, as float32, bf16, or a
// bf16 hi + lo split (hi = bf16(x), lo = bf16(x - hi)).
#include "common.h"

namespace goat {
namespace {

template <int MODE>
__device__ inline void put(void* hi, void* lo, size_t idx, float x) {
    if (MODE == PACK_F32) {
        static_cast<float*>(hi)[idx] = x;
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

}  // namespace

int launch_pack(const float* src, int ld, int n, int np, int transpose, int mode, void* dst_hi,
                void* dst_lo, hipStream_t s) {
    dim3 grid(np / 64, np / 64), block(256);
#define GOAT_PACK_CASE(M, T) \
    hipLaunchKernelGGL((pack_kernel<M, T>), grid, block, 0, s, src, ld, n, np, dst_hi, dst_lo)
    if (mode == PACK_F32) {
        if (transpose) GOAT_PACK_CASE(PACK_F32, true); else GOAT_PACK_CASE(PACK_F32, false);
    } else if (mode == PACK_BF16) {
        if (transpose) GOAT_PACK_CASE(PACK_BF16, true); else GOAT_PACK_CASE(PACK_BF16, false);
    } else {
        if (transpose) GOAT_PACK_CASE(PACK_BF16_SPLIT, true); else GOAT_PACK_CASE(PACK_BF16_SPLIT, false);
    }
#undef GOAT_PACK_CASE
    GOAT_HIP(hipGetLastError());
    return GOAT_OK;
}

}  // namespace goat
