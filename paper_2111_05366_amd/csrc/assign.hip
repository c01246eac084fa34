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
#include "common.h"

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

}  // namespace goat
