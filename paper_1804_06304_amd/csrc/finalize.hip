// End of evolution (Results of the paper): exact energy and selection.
//
// Exact energy: one workgroup per contour evaluates Eq. (5) literally over the lattice points within
// R + dR/2 of the centre (clamp-to-edge values outside the volume), times the voxel measure,
// divided by (2R)^d. FP32 terms, FP64 accumulation, fixed-order reduction. Contours still ACTIVE
// become MAXITER here.
//
// Selection: one workgroup per job. Candidates (CONVERGED or MAXITER, E_vox <= E0) are binned on a
// uniform grid with cell >= rho * r_max, so every overlapping pair (|c' - c''| < rho max(R', R''))
// lies in neighbouring cells. Rounds of "accept a candidate whose (E_vox, id) is the smallest among
// its undecided overlapping neighbours and that has no accepted overlapping neighbour; reject a
// candidate with an accepted overlapping neighbour" run until nothing is undecided. An accepted
// neighbour always has the smaller key, and the undecided candidate with the globally smallest key
// is decided in every round, so the result equals the sequential greedy of the paper's competition
// (lower energy survives) taken in ascending (E_vox, id) order.
#include <math.h>

#include "snk_internal.h"

namespace snk {

namespace {

constexpr int SEL_T = 1024;
constexpr int kSelectGridMin = 1024;   // contours above which the plain path bins and decides grid-wide
constexpr int kSelectGridRounds = 6;   // grid-wide decision rounds before the single-workgroup finish

// Threads per contour of the exact energy: a 3D ball holds thousands of lattice points, a disk
// hundreds.
template <int DIM>
constexpr int ev_threads() {
    return DIM == 3 ? 256 : 64;
}

// The weight S of Eq. (5) in FP64: the exact energy sums a few thousand terms once per contour, so
// the distance and weight of each lattice point are formed in double and only the voxel value is
// FP32 (as the smoothed volume is).
template <int DIM>
__device__ __forceinline__ double weight_S(double r, double R, double dR) {
    constexpr double RHO = DIM == 3 ? 0.79370052598409973738 : 0.70710678118654752440;
    const double ain = RHO * R, dr = RHO * dR;
    if (r < ain - 0.5 * dr) return -1.0;
    if (r < ain + 0.5 * dr) return 2.0 * (r - ain) / dr;
    if (r < R - 0.5 * dR) return 1.0;
    if (r < R + 0.5 * dR) return 0.5 - (r - R) / dR;
    return 0.0;
}

template <int DIM>
__device__ void energy_one(const JobParams &p, DevContour *slot, double *e_out, bool finalize = true) {
    constexpr int EV_T = ev_threads<DIM>();
    __shared__ double part[EV_T / 64];
    const int t = threadIdx.x;
    const DevContour s = *slot;
    const Geometry &g = p.g;
    const float R = s.R;
    if (!isfinite(R) || !(R > 0.0f) || !(R <= p.r_hi) || (s.status & 0x0f) == SNK_NONFINITE) {
        if (t == 0) {
            *e_out = NAN;
            if (finalize) slot->e_vox = NAN;
        }
        return;
    }
    const float smax = R + 0.5f * p.dR;
    const double R_d = (double)R, dR_d = (double)p.dR, smax_d = R_d + 0.5 * dR_d;
    int lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        const float ext = smax * g.inv_h[i];
        lo[i] = (int)floorf(s.off[i] - ext) - 1;
        cnt[i] = (int)ceilf(s.off[i] + ext) + 1 - lo[i] + 1;
    }
    const int nn[3] = {g.nx, g.ny, g.nz};
    const int total = cnt[0] * cnt[1] * cnt[2];
    // box coordinates of this thread's first point and the step of EV_T points (no division in
    // the loop)
    int rx = t % cnt[0], ry = (t / cnt[0]) % cnt[1], rz = t / (cnt[0] * cnt[1]);
    const int sx = EV_T % cnt[0], sy = EV_T / cnt[0];
    double acc = 0.0;
    for (int idx = t; idx < total; idx += EV_T) {
        const int rel[3] = {lo[0] + rx, lo[1] + ry, lo[2] + rz};
        rx += sx;
        if (rx >= cnt[0]) {
            rx -= cnt[0];
            ry += 1;
        }
        ry += sy;
        while (ry >= cnt[1]) {
            ry -= cnt[1];
            rz += 1;
        }
        double d2 = 0.0;
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            const double d = ((double)rel[i] - (double)s.off[i]) * (double)g.h[i];
            d2 = fma(d, d, d2);
        }
        const double r = sqrt(d2);
        if (!(r < smax_d)) continue;  // (the step above already advanced the coordinates)
        int k[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < DIM; ++i) k[i] = min(max(s.anc[i] + rel[i], 0), nn[i] - 1);
        const float v = g.J[((long)k[2] * g.ny + k[1]) * g.nx + k[0]];
        acc += weight_S<DIM>(r, R_d, dR_d) * (double)v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((t & 63) == 0) part[t >> 6] = acc;
    __syncthreads();
    if (t == 0) {
        double tot = 0.0;
#pragma unroll
        for (int w = 0; w < EV_T / 64; ++w) tot += part[w];
        const double meas = (double)g.h[0] * g.h[1] * (DIM == 3 ? g.h[2] : 1.0f);
        double norm = 1.0;
        for (int i = 0; i < DIM; ++i) norm *= 2.0 * (double)R;
        const double e = tot * meas / norm;
        *e_out = e;
        if (finalize) {
            DevContour o = s;
            o.e_vox = (float)e;
            if ((o.status & 0x0f) == SNK_ACTIVE) o.status = (uint8_t)((o.status & SNK_CLAMPED) | SNK_MAXITER);
            *slot = o;
        }
    }
}

template <int DIM>
__global__ __launch_bounds__(ev_threads<DIM>()) void energy_vox_kernel(JobParams p, DevContour *st, double *e_vox,
                                                                      int n, int finalize) {
    const int cid = blockIdx.x;
    if (cid < n) energy_one<DIM>(p, st + cid, e_vox + cid, finalize != 0);
}

template <int DIM>
__global__ __launch_bounds__(ev_threads<DIM>()) void energy_vox_batch_kernel(const JobDev *jobs, const int2 *items,
                                                                            int n_items) {
    const int item = blockIdx.x;
    if (item >= n_items) return;
    const int job = __builtin_amdgcn_readfirstlane(items[item].x);
    const int cid = __builtin_amdgcn_readfirstlane(items[item].y);
    const JobDev &j = jobs[job];
    energy_one<DIM>(j.p, j.st + cid, j.e_vox + cid);
}

enum : int { DEC_NONE = 0, DEC_UNDECIDED = 1, DEC_ACCEPT = 2, DEC_REJECT = 3 };

template <int DIM>
__device__ __forceinline__ bool overlaps(const DevContour &x, const DevContour &y, const float h[3]) {
    constexpr float RHO = DIM == 3 ? 0.79370052598409973738f : 0.70710678118654752440f;
    float d2 = 0.0f;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        const float d = ((float)(x.anc[i] - y.anc[i]) + (x.off[i] - y.off[i])) * h[i];
        d2 = fmaf(d, d, d2);
    }
    const float thr = RHO * fmaxf(x.R, y.R);
    return sqrtf(d2) < thr;
}

// Energy that ranks contour i: E_vox for the final selection (mode 0), the last Monte-Carlo
// energy for a culling pass during evolution (mode 1) and for the final selection of star-shaped
// contours (mode 2).
__device__ __forceinline__ double rank_energy(const JobDev &a, int i, const DevContour &s) {
    return a.mode == 0 ? a.e_vox[i] : (double)s.e_mc;
}

// One decision step for contour i (no-op unless undecided): reject if an overlapping neighbour is
// accepted, accept if it has the smallest (E_vox, id) among its undecided overlapping neighbours.
// Decisions of other contours may change concurrently; every decision taken is final and
// correct whatever the interleaving, since a contour is accepted only once every overlapping
// contour with a smaller key has been rejected.
template <int DIM>
__device__ int decide(const JobDev &a, int i) {
    volatile int *dec = a.dec;
    if (dec[i] != DEC_UNDECIDED) return dec[i];
    const Geometry &g = a.p.g;
    const DevContour si = a.st[i];
    const double ei = rank_energy(a, i, si);
    const int cell = a.cell_of[i];
    const int gi[3] = {cell % a.G[0], (cell / a.G[0]) % a.G[1], cell / (a.G[0] * a.G[1])};
    bool accepted_nb = false, minimal = true;
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0) && !accepted_nb; ++dz)
        for (int dy = -1; dy <= 1 && !accepted_nb; ++dy)
            for (int dx = -1; dx <= 1 && !accepted_nb; ++dx) {
                const int cx = gi[0] + dx, cy = gi[1] + dy, cz = gi[2] + dz;
                if (cx < 0 || cy < 0 || cz < 0 || cx >= a.G[0] || cy >= a.G[1] || cz >= a.G[2]) continue;
                const int c = (cz * a.G[1] + cy) * a.G[0] + cx;
                for (int q = a.cell_start[c]; q < a.cell_start[c + 1]; ++q) {
                    const int j = a.items[q];
                    if (j == i) continue;
                    const int dj = dec[j];
                    if (dj == DEC_REJECT) continue;
                    const DevContour sj = a.st[j];
                    if (!overlaps<DIM>(si, sj, g.h)) continue;
                    if (dj == DEC_ACCEPT) {
                        accepted_nb = true;
                        break;
                    }
                    const double ej = rank_energy(a, j, sj);
                    if (ej < ei || (ej == ei && sj.id < si.id)) minimal = false;
                }
            }
    const int d = accepted_nb ? DEC_REJECT : (minimal ? DEC_ACCEPT : DEC_UNDECIDED);
    if (d != DEC_UNDECIDED) dec[i] = d;
    return d;
}

// Candidate flag and grid cell of contour i; counts the cell's members in cell_start[cell + 1].
template <int DIM>
__device__ __forceinline__ void bin_one(const JobDev &a, int i) {
    const Geometry &g = a.p.g;
    const DevContour s = a.st[i];
    const int st = s.status & 0x0f;
    const double e = rank_energy(a, i, s);
    // final selection: stopped contours at or below E0; culling pass: live contours below E0, or all
    // of them during the run's grace period (the host passes a grace above every count then, else 0)
    const bool cand = a.mode != 1 ? (st == SNK_CONVERGED || st == SNK_MAXITER) && isfinite(e) && e <= (double)a.e0
                                  : (st == SNK_ACTIVE || st == SNK_CONVERGED) && isfinite(e) &&
                                        (s.iters < a.grace || e <= (double)a.e_cull);
    // a culling pass without competition keeps every candidate
    a.dec[i] = cand ? (a.mode == 1 && !a.compete ? DEC_ACCEPT : DEC_UNDECIDED) : DEC_NONE;
    int cell = -1;
    if (cand) {
        int gi[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const float pk = ((float)s.anc[k] + s.off[k]) * g.h[k];
            gi[k] = min(max((int)floorf(pk / a.cell), 0), a.G[k] - 1);
        }
        cell = (gi[2] * a.G[1] + gi[1]) * a.G[0] + gi[0];
        atomicAdd(&a.cell_start[cell + 1], 1);
    }
    a.cell_of[i] = cell;
}

// Inclusive running sum of one tile of SEL_T * 8 cell counts cs[base ..] (in place), plus carry: 8
// consecutive cells per thread, a shuffle scan of the thread sums inside each wave, the wave totals
// scanned through LDS (ws: SEL_T / 64 + 1 ints). Returns the tile's total (every thread).
__device__ int scan_tile(int *cs, int G, int base, int carry, int *ws) {
    constexpr int V = 8;
    constexpr int W = SEL_T / 64;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int i0 = base + t * V;
    int v[V];
    int s = 0;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        s += i0 + k < G ? cs[i0 + k] : 0;
        v[k] = s;
    }
    int incl = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    if (lane == 63) ws[w] = incl;
    __syncthreads();
    if (w == 0) {
        const int x = lane < W ? ws[lane] : 0;
        int sc = x;
#pragma unroll
        for (int d = 1; d < W; d <<= 1) {
            const int y = __shfl_up(sc, d, 64);
            if (lane >= d) sc += y;
        }
        if (lane < W) ws[lane] = sc - x;  // exclusive prefix of the wave totals
        if (lane == W - 1) ws[W] = sc;    // tile total
    }
    __syncthreads();
    const int off = carry + ws[w] + (incl - s);
#pragma unroll
    for (int k = 0; k < V; ++k)
        if (i0 + k < G) cs[i0 + k] = v[k] + off;
    const int total = ws[W];
    __syncthreads();
    return total;
}

constexpr int SCAN_TILE = SEL_T * 8;

// Inclusive running sum of the cell counts cell_start[1..G], in place, by one workgroup (tile by
// tile, carrying the total across).
__device__ void scan_cells(const JobDev &a, int G, int *ws) {
    int *cs = a.cell_start + 1;
    int carry = 0;
    for (int base = 0; base < G; base += SCAN_TILE) carry += scan_tile(cs, G, base, carry, ws);
}

__device__ __forceinline__ void scatter_one(const JobDev &a, int i) {
    const int cell = a.cell_of[i];
    if (cell >= 0) {
        const int pos = atomicAdd(&a.cell_fill[cell], 1);
        a.items[a.cell_start[cell] + pos] = i;
    }
}

// Outcome of the decisions for contour i: keep flag (final selection) or retirement (culling pass);
// returns 1 when it counts (kept, or retired).
__device__ __forceinline__ int apply_one(const JobDev &a, int i, int d) {
    if (a.mode != 1) {
        const uint8_t k = d == DEC_ACCEPT ? 1 : 0;
        a.st[i].keep = k;
        return k;
    }
    // culling pass: live contours that lost or are no candidates stop
    const uint8_t s8 = a.st[i].status;
    const int st = s8 & 0x0f;
    if ((st == SNK_ACTIVE || st == SNK_CONVERGED) && d != DEC_ACCEPT) {
        a.st[i].status = (uint8_t)((s8 & SNK_CLAMPED) | SNK_CULLED);
        return 1;
    }
    return 0;
}

// Whole selection of one job by one workgroup. binned: the grid (cell_start, items, cell_of, dec)
// was already built and some decisions may already be taken; then a scan of the decisions decides
// whether the decision loop is needed at all. apply = false leaves the outcome to sel_apply_kernel.
template <int DIM>
__device__ void select_job(const JobDev &a, bool binned, bool apply = true) {
    __shared__ int chunk_sum[SEL_T];
    const int t = threadIdx.x;
    const int n = a.n;
    const int G = a.G[0] * a.G[1] * a.G[2];
    volatile int *dec = a.dec;
    if (!binned) {
        for (int c = t; c <= G; c += SEL_T) a.cell_start[c] = 0;
        for (int c = t; c < G; c += SEL_T) a.cell_fill[c] = 0;
        __syncthreads();
        for (int i = t; i < n; i += SEL_T) bin_one<DIM>(a, i);
        __syncthreads();
        scan_cells(a, G, chunk_sum);
        __syncthreads();
        for (int i = t; i < n; i += SEL_T) scatter_one(a, i);
        __syncthreads();
    }
    bool any = true;
    if (binned) {
        // no decision is written while this scan runs, so plain loads (issued back to back) serve
        const int *dn = a.dec;
        int local = 0;
#pragma unroll 8
        for (int i = t; i < n; i += SEL_T) local |= dn[i] == DEC_UNDECIDED ? 1 : 0;
        any = __syncthreads_or(local) != 0;
    }
    while (any) {
        int local = 0;
        for (int i = t; i < n; i += SEL_T) local |= decide<DIM>(a, i) == DEC_UNDECIDED ? 1 : 0;
        __threadfence_block();
        any = __syncthreads_or(local) != 0;
    }
    if (!apply) return;
    unsigned long long count = 0;
    for (int i = t; i < n; i += SEL_T) count += apply_one(a, i, dec[i]);
    if (count) atomicAdd(a.kept, count);
}

template <int DIM>
__global__ __launch_bounds__(SEL_T) void select_kernel(JobDev j, int binned, int apply) {
    if (j.n > 0) select_job<DIM>(j, binned != 0, apply != 0);
}

template <int DIM>
__global__ __launch_bounds__(SEL_T) void select_batch_kernel(const JobDev *jobs, const int *job_list, int n_jobs) {
    if ((int)blockIdx.x >= n_jobs) return;
    const JobDev &j = jobs[__builtin_amdgcn_readfirstlane(job_list[blockIdx.x])];
    if (j.n > 0) select_job<DIM>(j, false);
}

// Grid-wide selection steps for one job with many contours (the single-workgroup loop above then
// finishes whatever the rounds left undecided).
constexpr int SG_T = 256;

__global__ __launch_bounds__(SG_T) void sel_zero_kernel(JobDev a, int G, int *rounds) {
    const int i = blockIdx.x * SG_T + threadIdx.x;
    if (i <= G) a.cell_start[i] = 0;
    if (i < G) a.cell_fill[i] = 0;
    if (i < 3) rounds[i] = 0;
}

template <int DIM>
__global__ __launch_bounds__(SG_T) void sel_bin_kernel(JobDev a) {
    const int i = blockIdx.x * SG_T + threadIdx.x;
    if (i < a.n) bin_one<DIM>(a, i);
}

__global__ __launch_bounds__(SEL_T) void sel_scan_kernel(JobDev a, int G) {
    __shared__ int chunk_sum[SEL_T];
    scan_cells(a, G, chunk_sum);
}

// The same running sum by one workgroup per tile, for grids of several tiles: (1) each tile's own
// running sum, its total parked in cell_fill[tile] (zero until the scatter counts in it); (2) one
// workgroup turns the totals into each tile's offset; (3) each tile adds its offset and puts the
// zero back in cell_fill[tile].
__global__ __launch_bounds__(SEL_T) void sel_scan_tiles_kernel(JobDev a, int G) {
    __shared__ int ws[SEL_T / 64 + 1];
    const int total = scan_tile(a.cell_start + 1, G, blockIdx.x * SCAN_TILE, 0, ws);
    if (threadIdx.x == 0) a.cell_fill[blockIdx.x] = total;
}

__global__ __launch_bounds__(SEL_T) void sel_scan_totals_kernel(JobDev a, int ntiles) {
    __shared__ int ws[SEL_T / 64 + 1];
    // ntiles <= SEL_T * 8: one tile of totals; inclusive, then shifted to the exclusive offsets
    const int t = threadIdx.x;
    int own[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) own[k] = t * 8 + k < ntiles ? a.cell_fill[t * 8 + k] : 0;
    __syncthreads();
    scan_tile(a.cell_fill, ntiles, 0, 0, ws);
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (t * 8 + k < ntiles) a.cell_fill[t * 8 + k] -= own[k];
}

__global__ __launch_bounds__(SEL_T) void sel_scan_add_kernel(JobDev a, int G) {
    __shared__ int off_sh;
    if (threadIdx.x == 0) {
        off_sh = a.cell_fill[blockIdx.x];
        a.cell_fill[blockIdx.x] = 0;
    }
    __syncthreads();
    const int off = off_sh;
    if (off == 0) return;
    int *cs = a.cell_start + 1;
    const int base = blockIdx.x * SCAN_TILE;
    for (int i = base + (int)threadIdx.x; i < min(base + SCAN_TILE, G); i += SEL_T) cs[i] += off;
}

__global__ __launch_bounds__(SG_T) void sel_scatter_kernel(JobDev a) {
    const int i = blockIdx.x * SG_T + threadIdx.x;
    if (i < a.n) scatter_one(a, i);
}

// Round r: skipped when round r-1 left nothing undecided; counts what it leaves undecided in
// rounds[r % 3] and clears rounds[(r + 1) % 3] for the next round.
template <int DIM>
__global__ __launch_bounds__(SG_T) void sel_round_kernel(JobDev a, int r, int *rounds) {
    if (r > 0 && *(volatile int *)&rounds[(r + 2) % 3] == 0) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) rounds[(r + 1) % 3] = 0;
    const int i = blockIdx.x * SG_T + threadIdx.x;
    int left = 0;
    if (i < a.n) left = decide<DIM>(a, i) == DEC_UNDECIDED ? 1 : 0;
    if (__builtin_amdgcn_ballot_w64(left != 0) != 0 && (threadIdx.x & 63) == 0) atomicAdd(&rounds[r % 3], 1);
}

// The outcome of every decision, grid-wide (after the decisions are complete).
__global__ __launch_bounds__(SG_T) void sel_apply_kernel(JobDev a) {
    const int i = blockIdx.x * SG_T + threadIdx.x;
    const int c = i < a.n ? apply_one(a, i, a.dec[i]) : 0;
    const int total = __syncthreads_count(c);
    if (threadIdx.x == 0 && total) atomicAdd(a.kept, (unsigned long long)total);
}

template <int DIM>
hipError_t select_grid(const JobDev &j, int *rounds, hipStream_t s) {
    const int G = j.G[0] * j.G[1] * j.G[2];
    const int bn = (j.n + SG_T - 1) / SG_T;
    hipLaunchKernelGGL(sel_zero_kernel, dim3((G + 1 + SG_T - 1) / SG_T), dim3(SG_T), 0, s, j, G, rounds);
    hipLaunchKernelGGL(sel_bin_kernel<DIM>, dim3(bn), dim3(SG_T), 0, s, j);
    // one workgroup walks up to three tiles faster than three launches take (about 8 us per tile
    // against about 20 us for the tile, totals and add kernels together)
    const int ntiles = (G + SCAN_TILE - 1) / SCAN_TILE;
    if (ntiles <= 3) {
        hipLaunchKernelGGL(sel_scan_kernel, dim3(1), dim3(SEL_T), 0, s, j, G);
    } else {
        hipLaunchKernelGGL(sel_scan_tiles_kernel, dim3(ntiles), dim3(SEL_T), 0, s, j, G);
        hipLaunchKernelGGL(sel_scan_totals_kernel, dim3(1), dim3(SEL_T), 0, s, j, ntiles);
        hipLaunchKernelGGL(sel_scan_add_kernel, dim3(ntiles), dim3(SEL_T), 0, s, j, G);
    }
    hipLaunchKernelGGL(sel_scatter_kernel, dim3(bn), dim3(SG_T), 0, s, j);
    for (int r = 0; r < kSelectGridRounds; ++r)
        hipLaunchKernelGGL(sel_round_kernel<DIM>, dim3(bn), dim3(SG_T), 0, s, j, r, rounds);
    hipLaunchKernelGGL(select_kernel<DIM>, dim3(1), dim3(SEL_T), 0, s, j, 1, 0);
    hipLaunchKernelGGL(sel_apply_kernel, dim3(bn), dim3(SG_T), 0, s, j);
    return hipGetLastError();
}

}  // namespace

namespace {
__global__ __launch_bounds__(256) void mark_maxiter_kernel(DevContour *st, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n && (st[i].status & 0x0f) == SNK_ACTIVE) st[i].status = (uint8_t)((st[i].status & SNK_CLAMPED) | SNK_MAXITER);
}
}  // namespace

namespace {
__global__ __launch_bounds__(256) void compact_active_kernel(const DevContour *st, int n, int *idx, int *count) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const bool act = i < n && (st[i].status & 0x0f) == SNK_ACTIVE;
    // one atomic per wave: the active lanes take consecutive slots in lane order
    const unsigned long long m = __builtin_amdgcn_ballot_w64(act);
    const int lane = threadIdx.x & 63;
    int base = 0;
    if (lane == 0 && m) base = atomicAdd(count, __popcll(m));
    base = __shfl(base, 0, 64);
    if (act) idx[base + __popcll(m & ((1ull << lane) - 1ull))] = i;
}
}  // namespace

hipError_t launch_compact_active(const DevContour *st, int n, int *idx, int *count, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(compact_active_kernel, dim3((n + 255) / 256), dim3(256), 0, s, st, n, idx, count);
    return hipGetLastError();
}

hipError_t launch_mark_maxiter(DevContour *st, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mark_maxiter_kernel, dim3((n + 255) / 256), dim3(256), 0, s, st, n);
    return hipGetLastError();
}

hipError_t launch_energy_vox(const JobParams &p, DevContour *st, double *e_vox, int n, int dim, bool finalize,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int f = finalize ? 1 : 0;
    if (dim == 2) hipLaunchKernelGGL(energy_vox_kernel<2>, dim3(n), dim3(ev_threads<2>()), 0, s, p, st, e_vox, n, f);
    else hipLaunchKernelGGL(energy_vox_kernel<3>, dim3(n), dim3(ev_threads<3>()), 0, s, p, st, e_vox, n, f);
    return hipGetLastError();
}

hipError_t launch_select(const JobDev &j, int dim, int *rounds, hipStream_t s) {
    if (j.n <= 0) return hipSuccess;
    if (j.n > kSelectGridMin && rounds) return dim == 2 ? select_grid<2>(j, rounds, s) : select_grid<3>(j, rounds, s);
    if (dim == 2) hipLaunchKernelGGL(select_kernel<2>, dim3(1), dim3(SEL_T), 0, s, j, 0, 1);
    else hipLaunchKernelGGL(select_kernel<3>, dim3(1), dim3(SEL_T), 0, s, j, 0, 1);
    return hipGetLastError();
}

hipError_t launch_energy_vox_batch(const JobDev *jobs, const int2 *items, int n_items, int dim, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (dim == 2)
        hipLaunchKernelGGL(energy_vox_batch_kernel<2>, dim3(n_items), dim3(ev_threads<2>()), 0, s, jobs, items, n_items);
    else
        hipLaunchKernelGGL(energy_vox_batch_kernel<3>, dim3(n_items), dim3(ev_threads<3>()), 0, s, jobs, items, n_items);
    return hipGetLastError();
}

hipError_t launch_select_batch(const JobDev *jobs, const int *job_list, int n_jobs, int dim, hipStream_t s) {
    if (n_jobs <= 0) return hipSuccess;
    if (dim == 2) hipLaunchKernelGGL(select_batch_kernel<2>, dim3(n_jobs), dim3(SEL_T), 0, s, jobs, job_list, n_jobs);
    else hipLaunchKernelGGL(select_batch_kernel<3>, dim3(n_jobs), dim3(SEL_T), 0, s, jobs, job_list, n_jobs);
    return hipGetLastError();
}

}  // namespace snk
