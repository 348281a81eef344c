// Small kernels of the batch / serving engine. They replace memset and memcpy nodes so that a whole
// batched run can be captured in one hipGraph and replayed.
#include "snk_internal.h"

namespace snk {

namespace {

// Restore every item's contour state from its job's initial state (start of a batched run).
__global__ void reset_items_kernel(const JobDev *jobs, const int2 *items, int n_items, const DevContour *const *init) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    const int2 it = items[i];
    jobs[it.x].st[it.y] = init[it.x][it.y];
}

__global__ void zero_kernel(unsigned long long *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Per job: contours that can still evolve (ACTIVE and below the job's iteration target).
__global__ void count_unfinished_kernel(const JobDev *jobs, const int2 *items, int n_items, int *unfinished) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    const int2 it = items[i];
    const DevContour &c = jobs[it.x].st[it.y];
    if ((c.status & 0x0f) == SNK_ACTIVE && c.iters < jobs[it.x].target) atomicAdd(&unfinished[it.x], 1);
}

}  // namespace

hipError_t launch_reset_items(const JobDev *jobs, const int2 *items, int n_items, const DevContour *const *init,
                              hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(reset_items_kernel, dim3((n_items + 255) / 256), dim3(256), 0, s, jobs, items, n_items, init);
    return hipGetLastError();
}

hipError_t launch_zero(unsigned long long *p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_count_unfinished(const JobDev *jobs, const int2 *items, int n_items, int *unfinished, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(count_unfinished_kernel, dim3((n_items + 255) / 256), dim3(256), 0, s, jobs, items, n_items,
                       unfinished);
    return hipGetLastError();
}

}  // namespace snk
