// sal_batch.h -- per-volume descriptors of the batched kernels (not part of the ABI).
#pragma once

#include "sal_aux.h"

namespace sal {

// partial-sum blocks per volume for the fusion statistics: the same partition as the
// single-volume path, so both reduce in the same order and agree bit for bit
constexpr int kBatchParts = kFuseParts;

struct DcsItem {
    const float* E;
    float* S;
    int64_t Tg, ILg, XLg;
    DcsStencil st;
};

struct FuseItem {
    const float* Sm;
    const float* D;
    const uint8_t* mask;
    int64_t Tg, ILg, XLg, T, IL, XL;
    int s;
    int mode;
    double w0, w1, w2, delta;
    double* W;
    float* S;
    double* part;  // kBatchParts x kStats doubles (adapted weights only)
};

sal_status launch_dcs_batch(const DcsItem* items, const int64_t* first, int n, int64_t blocks, hipStream_t stream);
// The plan's status word: status[0] = members whose W[3] flags an equal-weight fallback,
// status[1] = the lowest such member (-1 if none).
sal_status launch_plan_status(const FuseItem* items, int n, int64_t* status, hipStream_t stream);
sal_status launch_fuse_batch(const FuseItem* items, int n, const int* adapt_list, int nadapt, const int64_t* first,
                             int64_t rows, hipStream_t stream);

}  // namespace sal
