// Neighbour lists for the soft repulsion between contours (not in the paper: a builder-defined
// extension; the paper's contours are independent during evolution and compete only afterwards).
//
// At the start of each chunk of iterations the centres and radii of all contours are copied into a
// snapshot, and every ACTIVE contour gets the list of live contours (ACTIVE or CONVERGED) whose inner
// sphere overlaps its own: |c_i - c_j| < rho (R_i + R_j). The evolve kernel sums the repulsion of
// the listed snapshot contours at every iteration of the chunk. Candidates are found on a uniform
// grid whose cell is at least 2 rho r_max (so a 3^d neighbourhood holds every partner), and each list
// is kept in ascending contour index, so the order of the sums does not depend on timing.
#include "snk_internal.h"

namespace snk {

namespace {

constexpr int NB_T = 256;

template <int DIM>
__device__ __forceinline__ int cell_of_point(const DevContour &s, const Geometry &g, float cell, const int G[3]) {
    int gi[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const float pa = ((float)s.anc[a] + s.off[a]) * g.h[a];
        gi[a] = min(max((int)floorf(pa / cell), 0), G[a] - 1);
    }
    return (gi[2] * G[1] + gi[1]) * G[0] + gi[0];
}

__device__ __forceinline__ bool is_live(uint8_t status) {
    const int st = status & 0x0f;
    return st == SNK_ACTIVE || st == SNK_CONVERGED;
}

__global__ __launch_bounds__(NB_T) void nb_zero_kernel(NeighbourArgs b) {
    const int i = blockIdx.x * NB_T + threadIdx.x;
    const int G = b.G[0] * b.G[1] * b.G[2];
    if (i <= G) b.cell_start[i] = 0;
    if (i < G) b.cell_fill[i] = 0;
    if (i == 0) *b.overflow = 0;
}

// Snapshot record of contour i (anchor bits and R; offset and live flag) and its grid cell.
template <int DIM>
__global__ __launch_bounds__(NB_T) void nb_snap_kernel(const DevContour *st, int n, Geometry g, NeighbourArgs b) {
    const int i = blockIdx.x * NB_T + threadIdx.x;
    if (i >= n) return;
    const DevContour s = st[i];
    const bool live = is_live(s.status);
    b.snap[2 * i] = make_float4(__int_as_float(s.anc[0]), __int_as_float(s.anc[1]), __int_as_float(s.anc[2]), s.R);
    b.snap[2 * i + 1] = make_float4(s.off[0], s.off[1], s.off[2], live ? 1.0f : 0.0f);
    int cell = -1;
    if (live) {
        cell = cell_of_point<DIM>(s, g, b.cell, b.G);
        atomicAdd(&b.cell_start[cell + 1], 1);
    }
    b.cell_of[i] = cell;
}

// Running sum of the cell counts, in place, by one workgroup (grids here hold at most 2^20 cells).
__global__ __launch_bounds__(1024) void nb_scan_kernel(NeighbourArgs b) {
    __shared__ int part[1024];
    const int G = b.G[0] * b.G[1] * b.G[2];
    const int t = threadIdx.x;
    const int per = (G + 1023) / 1024;
    const int lo = 1 + t * per, hi = min(lo + per, G + 1);
    int sum = 0;
    for (int c = lo; c < hi; ++c) sum += b.cell_start[c];
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = t > 0 ? part[t - 1] : 0;
    for (int c = lo; c < hi; ++c) {
        run += b.cell_start[c];
        b.cell_start[c] = run;
    }
}

__global__ __launch_bounds__(NB_T) void nb_scatter_kernel(int n, NeighbourArgs b) {
    const int i = blockIdx.x * NB_T + threadIdx.x;
    if (i >= n) return;
    const int cell = b.cell_of[i];
    if (cell >= 0) b.items[b.cell_start[cell] + atomicAdd(&b.cell_fill[cell], 1)] = i;
}

// Whether live contour j (snapshot records sj0, sj1) overlaps contour i: |c_i - c_j| < rho (R_i + R_j).
template <int DIM>
__device__ __forceinline__ bool overlaps(const int ai[3], const float oi[3], float Ri, float4 sj0, float4 sj1,
                                         const Geometry &g, float rho) {
    const int aj[3] = {__float_as_int(sj0.x), __float_as_int(sj0.y), __float_as_int(sj0.z)};
    const float oj[3] = {sj1.x, sj1.y, sj1.z};
    float d2 = 0.0f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const float dv = ((float)(ai[a] - aj[a]) + (oi[a] - oj[a])) * g.h[a];
        d2 = fmaf(dv, dv, d2);
    }
    const float span = rho * (Ri + sj0.w);
    return d2 < span * span;
}

// The list of one contour by one lane: the 3^d cells around it, inserting each overlapping j so the
// list stays ascending and keeps the lowest cap indices (more sets the overflow flag).
template <int DIM>
__device__ int list_serial(int i, const int gi[3], const int ai[3], const float oi[3], float Ri, const Geometry &g,
                           float rho, const NeighbourArgs &b, int *list) {
    int count = 0;
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int cx = gi[0] + dx, cy = gi[1] + dy, cz = gi[2] + dz;
                if (cx < 0 || cy < 0 || cz < 0 || cx >= b.G[0] || cy >= b.G[1] || cz >= b.G[2]) continue;
                const int c = (cz * b.G[1] + cy) * b.G[0] + cx;
                for (int q = b.cell_start[c]; q < b.cell_start[c + 1]; ++q) {
                    const int j = b.items[q];
                    if (j == i || !overlaps<DIM>(ai, oi, Ri, b.snap[2 * j], b.snap[2 * j + 1], g, rho)) continue;
                    if (count == b.cap) {
                        atomicOr(b.overflow, 1);
                        if (j > list[count - 1]) continue;
                        --count;   // drop the largest index to keep the lowest cap
                    }
                    int k = count;
                    while (k > 0 && list[k - 1] > j) {
                        list[k] = list[k - 1];
                        --k;
                    }
                    list[k] = j;
                    ++count;
                }
            }
    return count;
}

constexpr int NB_LIST_WAVES = 4;   // contours per workgroup, one wave each
constexpr int NB_BUF = 256;        // matches a wave collects before ranking them

// The list of contour i (ACTIVE only; others get none): live contours j != i with
// |c_i - c_j| < rho (R_i + R_j), ascending j, at most b.cap (more sets the overflow flag). One wave
// per contour: the lanes test a cell's candidates 64 at a time and append the matches to an LDS
// buffer (in whatever order the grid holds them), then each match's rank among all of them gives
// its place, so the list does not depend on that order. A contour with more matches than the buffer
// holds falls back to one lane inserting them one by one (same list).
template <int DIM>
__global__ __launch_bounds__(64 * NB_LIST_WAVES) void nb_list_kernel(int n, Geometry g, float rho, NeighbourArgs b) {
    __shared__ int buf[NB_LIST_WAVES][NB_BUF];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int i = blockIdx.x * NB_LIST_WAVES + w;
    if (i >= n) return;   // whole waves leave; no barrier follows
    int *list = b.nb + (long)i * b.cap;
    const int cell = b.cell_of[i];
    const bool active = cell >= 0 && (b.status ? (b.status[i].status & 0x0f) == SNK_ACTIVE : true);
    if (!active) {
        if (lane == 0) b.nbn[i] = 0;
        return;
    }
    const float4 si0 = b.snap[2 * i], si1 = b.snap[2 * i + 1];
    const int gi[3] = {cell % b.G[0], (cell / b.G[0]) % b.G[1], cell / (b.G[0] * b.G[1])};
    const int ai[3] = {__float_as_int(si0.x), __float_as_int(si0.y), __float_as_int(si0.z)};
    const float oi[3] = {si1.x, si1.y, si1.z};
    int *mine = buf[w];
    int total = 0;
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int cx = gi[0] + dx, cy = gi[1] + dy, cz = gi[2] + dz;
                if (cx < 0 || cy < 0 || cz < 0 || cx >= b.G[0] || cy >= b.G[1] || cz >= b.G[2]) continue;
                const int c = (cz * b.G[1] + cy) * b.G[0] + cx;
                const int q1 = b.cell_start[c + 1];
                for (int q0 = b.cell_start[c]; q0 < q1; q0 += 64) {
                    const int q = q0 + lane;
                    bool hit = false;
                    int j = -1;
                    if (q < q1) {
                        j = b.items[q];
                        hit = j != i && overlaps<DIM>(ai, oi, si0.w, b.snap[2 * j], b.snap[2 * j + 1], g, rho);
                    }
                    const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
                    const int pos = total + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    if (hit && pos < NB_BUF) mine[pos] = j;
                    total += __builtin_popcountll(m);
                }
            }
    int count;
    if (total <= NB_BUF) {
        // the lanes' buffer writes before any lane reads the buffer
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        for (int e = lane; e < total; e += 64) {
            const int j = mine[e];
            int rank = 0;
            for (int k = 0; k < total; ++k) rank += mine[k] < j ? 1 : 0;
            if (rank < b.cap) list[rank] = j;
        }
        count = min(total, b.cap);
        if (total > b.cap && lane == 0) atomicOr(b.overflow, 1);
    } else {
        count = lane == 0 ? list_serial<DIM>(i, gi, ai, oi, si0.w, g, rho, b, list) : 0;
    }
    if (lane == 0) b.nbn[i] = count;
}

}  // namespace

hipError_t launch_neighbours(const DevContour *st, int n, const Geometry &g, int dim, float rho,
                             const NeighbourArgs &b0, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    NeighbourArgs b = b0;
    b.status = st;
    const int G = b.G[0] * b.G[1] * b.G[2];
    const int blocks = (n + NB_T - 1) / NB_T;
    hipLaunchKernelGGL(nb_zero_kernel, dim3((G + 1 + NB_T - 1) / NB_T), dim3(NB_T), 0, s, b);
    if (dim == 2) hipLaunchKernelGGL(nb_snap_kernel<2>, dim3(blocks), dim3(NB_T), 0, s, st, n, g, b);
    else hipLaunchKernelGGL(nb_snap_kernel<3>, dim3(blocks), dim3(NB_T), 0, s, st, n, g, b);
    hipLaunchKernelGGL(nb_scan_kernel, dim3(1), dim3(1024), 0, s, b);
    hipLaunchKernelGGL(nb_scatter_kernel, dim3(blocks), dim3(NB_T), 0, s, n, b);
    const int lblocks = (n + NB_LIST_WAVES - 1) / NB_LIST_WAVES;
    if (dim == 2) hipLaunchKernelGGL(nb_list_kernel<2>, dim3(lblocks), dim3(64 * NB_LIST_WAVES), 0, s, n, g, rho, b);
    else hipLaunchKernelGGL(nb_list_kernel<3>, dim3(lblocks), dim3(64 * NB_LIST_WAVES), 0, s, n, g, rho, b);
    return hipGetLastError();
}

}  // namespace snk
