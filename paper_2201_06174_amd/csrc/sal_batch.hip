// sal_batch.hip -- batched center-surround and fusion kernels: one launch covers every
// volume of a plan, each block looking up the volume it serves in a small table.
#include <cstdint>

#include "sal_batch.h"
#include "sal_device.h"

namespace sal {

// last index i with first[i] <= b (first[0] == 0, ascending)
__device__ __forceinline__ int find_item(const int64_t* __restrict__ first, int n, int64_t b) {
    int a = 0, z = n - 1;
    while (a < z) {
        const int m = (a + z + 1) / 2;
        if (first[m] <= b) a = m; else z = m - 1;
    }
    return a;
}

__global__ __launch_bounds__(256) void k_dcs_batch(const DcsItem* __restrict__ items,
                                                   const int64_t* __restrict__ first, int n) {
    const int64_t b = block_id();
    const int a = find_item(first, n, b);
    const DcsItem& it = items[a];
    const int64_t j = (b - first[a]) * blockDim.x + threadIdx.x;
    if (j >= it.Tg * it.ILg * it.XLg) return;
    dcs_point(it.E, it.S, it.Tg, it.ILg, it.XLg, it.st, j);
}

__global__ __launch_bounds__(256) void k_fuse_stats_batch(const FuseItem* __restrict__ items,
                                                          const int* __restrict__ adapt_list) {
    __shared__ double red[256];
    const FuseItem& it = items[adapt_list[blockIdx.x / kBatchParts]];
    const int b = blockIdx.x % kBatchParts;
    const int64_t G = it.Tg * it.ILg * it.XLg;
    fuse_stats_block(it.Sm, it.D, it.mask, G, (int64_t)b * blockDim.x, (int64_t)kBatchParts * blockDim.x,
                     it.part + (int64_t)b * kStats, red);
}

__global__ __launch_bounds__(64) void k_fuse_solve_batch(const FuseItem* __restrict__ items) {
    __shared__ double st[kStats];
    const FuseItem& it = items[blockIdx.x];
    solve_weights(it.part, kBatchParts, it.mode, it.w0, it.w1, it.w2, it.delta, it.W, nullptr, st);
}

__global__ __launch_bounds__(256) void k_combine_batch(const FuseItem* __restrict__ items,
                                                       const int64_t* __restrict__ first, int n, int64_t rows) {
    const int64_t b = block_id();
    if (b >= rows) return;
    const int a = find_item(first, n, b);
    const FuseItem& it = items[a];
    combine_row(it.Sm, it.W, it.Tg, it.ILg, it.XLg, it.IL, it.XL, it.s, b - first[a], it.S);
}

// One block of 256 threads: counts the members whose status word W[3] is set and finds the
// lowest of them (integer reductions in a fixed order).
__global__ __launch_bounds__(256) void k_plan_status(const FuseItem* __restrict__ items, int n,
                                                     int64_t* __restrict__ status) {
    __shared__ int64_t cnt[256], low[256];
    int64_t c = 0, l = INT64_MAX;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (items[i].W[3] != 0.0) {
            c++;
            l = l < i ? l : i;
        }
    cnt[threadIdx.x] = c;
    low[threadIdx.x] = l;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            cnt[threadIdx.x] += cnt[threadIdx.x + w];
            low[threadIdx.x] = low[threadIdx.x] < low[threadIdx.x + w] ? low[threadIdx.x] : low[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        status[0] = cnt[0];
        status[1] = cnt[0] ? low[0] : -1;
    }
}

sal_status launch_plan_status(const FuseItem* items, int n, int64_t* status, hipStream_t stream) {
    hipLaunchKernelGGL(k_plan_status, dim3(1), dim3(256), 0, stream, items, n, status);
    return check_hip(hipGetLastError(), "launch k_plan_status");
}

sal_status launch_dcs_batch(const DcsItem* items, const int64_t* first, int n, int64_t blocks, hipStream_t stream) {
    if (blocks == 0) return SAL_OK;
    if (!wide_grid_fits(blocks, 256)) return fail(SAL_ERR_SHAPE, "batch too large for one launch");
    hipLaunchKernelGGL(k_dcs_batch, wide_grid(blocks, 256), dim3(256), 0, stream, items, first, n);
    return check_hip(hipGetLastError(), "launch k_dcs_batch");
}

sal_status launch_fuse_batch(const FuseItem* items, int n, const int* adapt_list, int nadapt, const int64_t* first,
                             int64_t rows, hipStream_t stream) {
    sal_status st;
    if (nadapt > 0) {
        hipLaunchKernelGGL(k_fuse_stats_batch, dim3((unsigned)(nadapt * kBatchParts)), dim3(256), 0, stream, items,
                           adapt_list);
        if ((st = check_hip(hipGetLastError(), "launch k_fuse_stats_batch"))) return st;
    }
    hipLaunchKernelGGL(k_fuse_solve_batch, dim3((unsigned)n), dim3(64), 0, stream, items);
    if ((st = check_hip(hipGetLastError(), "launch k_fuse_solve_batch"))) return st;
    if (rows == 0) return SAL_OK;
    if (!wide_grid_fits(rows, 256)) return fail(SAL_ERR_SHAPE, "batch too large for one launch");
    hipLaunchKernelGGL(k_combine_batch, wide_grid(rows, 256), dim3(256), 0, stream, items, first, n, rows);
    return check_hip(hipGetLastError(), "launch k_combine_batch");
}

}  // namespace sal
