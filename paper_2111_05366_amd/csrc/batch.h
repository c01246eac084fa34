// Shared host/device declarations of the batched solver.
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

#include "goat.h"

namespace goat {

// One (pair, start) problem. Every matrix is np x np with row stride np and
// zero padding outside the leading n x n block (np = n rounded up to 32).
struct BProb {
    int n, np, pair, restart;
    const float* A0;    // packed A
    const float* A1;    // packed A^T (general pairs) or nullptr (symmetric)
    const float* X1;    // packed B (symmetric) or [B; B^T] (general, 2np x np)
    const float* U;     // caller's start draws (ld ldu) or nullptr: P0 = J
    int ldu, pad;
    float* P;
    float* Q;
    float* GP;
    float* GQ;
    float* T;           // np x np (symmetric) or 2np x np
    goat_iter_record* hist;   // fw_max records
    int* fw_done;             // FW iterations run
};

struct BArgs {
    const BProb* probs;   // device
    const int* order;     // block -> problem index, -1 = idle block
    float eps_rel, sk_tol, fw_tol, init_tol;
    int sk_max, fw_max, stop_on_stall, warm, init_max, pad;
};

// Per-pair packing job: source A, B (ld) into the arena.
struct BPack {
    int n, np, ld, general;
    const float* A;
    const float* B;
    float* A0;
    float* A1;
    float* X1;
};

// lanes per Sinkhorn row, waves per workgroup, float4 column chunks per lane
struct BShape {
    int L, waves, cmax;
};

constexpr int kBatchBuckets = 5;   // np <= 64, 128, 256, 512, 1024
constexpr int kBucketMax[kBatchBuckets] = {64, 128, 256, 512, 1024};
inline int batch_bucket(int np) {
    for (int b = 0; b < kBatchBuckets; ++b)
        if (np <= kBucketMax[b]) return b;
    return -1;
}
inline int batch_pad(int n) { return (n + 31) / 32 * 32; }

// dynamic LDS bytes of the batched kernel for bucket capacity npb
size_t batch_lds_bytes(const BShape& s, int npb);
bool batch_shape_ok(const BShape& s, int npb);
int batch_launch(const BShape& s, int npb, int nblocks, const BArgs& a, hipStream_t st);
int batch_pack_launch(const BPack* jobs_dev, int njobs, int np_max, hipStream_t st);
int batch_score_launch(const BProb* probs_dev, int nprob, const int32_t* perms_dev, const int* perm_off_dev,
                       double* out_dev, hipStream_t st);
int batch_fill_zero(float* p, size_t count, hipStream_t st);
// final assignments of all problems on the device (assign.hip): status_dev[k]
// = bids taken (>= 0), GOAT_EINVAL (non-finite scores) or GOAT_ENOTSUP
// (bid budget spent)
int batch_auction_launch(const BProb* probs_dev, int nprob, int proj, const int* offs_dev, int32_t* perms_dev,
                         int* status_dev, long long budget, hipStream_t s);
int batch_synth_launch(float* A, float* B, int n, int ld, uint32_t seed, hipStream_t st);
int random_init_launch(int n, const float* U, int ldu, float* P, int ldp, float tol, int max_iter,
                       int* iters_dev, float* err_dev, hipStream_t st);

}  // namespace goat
