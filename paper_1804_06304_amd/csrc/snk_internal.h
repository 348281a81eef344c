// Internal declarations shared by the HIP translation units of libsnk.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "snk.h"

namespace snk {

// Device-resident state of one contour (48 bytes). The centre is held as an integer voxel anchor
// plus an FP32 offset in voxel units, so sample positions are formed from small numbers and keep
// FP32 precision on large images.
struct DevContour {
    int32_t anc[3];    // anchor voxel index per axis
    float off[3];      // offset from the anchor, voxel units
    float R;           // outer radius, physical units
    float e_mc;        // Monte-Carlo energy of the last iteration
    float e_vox;       // exact energy (after finalize)
    int32_t iters;     // iterations evolved so far (n of eps0/sqrt(n))
    uint32_t id;       // Philox stream id
    uint8_t status;    // SNK_* state | SNK_CLAMPED
    uint8_t streak;    // consecutive small steps
    uint8_t keep;      // selected (after finalize)
    uint8_t pad;
};
static_assert(sizeof(DevContour) == 48, "DevContour layout");

struct Geometry {
    const float *J;    // smoothed volume [z][y][x]
    const float4 *Jq;  // the same in the quad layout (J(x,y), J(x+1,y), J(x,y+1), J(x+1,y+1)), or null
    int nx, ny, nz;
    float h[3];
    float inv_h[3];
};

// Per-job constants of the evolution (one volume, one parameter set).
struct JobParams {
    Geometry g;
    const float *dirs;           // D x dim
    int D, M, L;
    uint32_t key0, key1;
    int flags;
    float dR, eps0, r_lo, r_hi, conv_tol;
    int conv_window;
    float in_slope, out_slope;   // 2 / (rho dR) and 1 / dR
    // culling passes without competition applied inside the evolution: after the launch's
    // iterations cull_first, cull_first + cull_every, ... up to cull_last (0-based, cull_first < 0:
    // none) an active contour whose energy is not <= cull_thr retires
    int cull_first = -1, cull_every = 0, cull_last = -1;
    float cull_thr = 0.0f;
};

// snk_params.flags bits.
constexpr int kFlagNoRotation = 1;  // random rotation off (Q = I)
constexpr int kFlagExact = 2;       // exact lattice sums over the ball instead of Monte-Carlo samples
constexpr int kFlagGradI = 4;       // centre force from sum S grad I (Monte-Carlo, whole-wave groups)

// How the evolve kernels read the smoothed volume.
enum VolumeLayout {
    kGlobalPlain = 0,  // FP32 [z][y][x], 64-bit addressing (any size)
    kBufferPlain = 1,  // FP32 [z][y][x] through a buffer descriptor (< 2 GiB, 24-bit strides)
    kBufferQuad = 2,   // quad records through a buffer descriptor (< 2 GiB, 24-bit strides)
    kBufferPair = 3,   // column pairs (J(x,y,z), J(x,y+1,z)) per voxel through a buffer descriptor
                       // (< 2 GiB): one 16-byte load at (x, y, z) fetches the four corners of the
                       // cell's plane z
};

// Layout for a volume: `requested` 0 = automatic (column pairs when they fit: one 16-byte load
// fetches the four corners of a cell's plane, as from the quad records, at half their footprint, so
// more of the volume stays in the caches and the pre-pass writes less; else plain), 1 = plain,
// 2 = quad, 3 = plain with 64-bit addressing, 4 = column pairs. Returns the layout, or -1 if the
// request cannot be met.
inline int volume_layout(int dim, int64_t nx, int64_t ny, int64_t nz, int requested) {
    const int64_t vox = nx * ny * nz;
    const bool strides = nx < (1 << 23) && (dim == 2 || nx * ny < (1 << 23));
    const bool plain_ok = strides && vox * 4 < ((int64_t)1 << 31);
    const bool quad_ok = strides && vox * 16 < ((int64_t)1 << 31) && ny <= 65535 && nz <= 65535;
    const bool pair_ok = strides && vox * 8 < ((int64_t)1 << 31) && ny <= 65535 && nz <= 65535;
    if (requested == 4) return pair_ok ? kBufferPair : -1;
    if (requested == 3) return kGlobalPlain;
    if (requested == 2) return quad_ok ? kBufferQuad : -1;
    if (requested == 1) return plain_ok ? kBufferPlain : kGlobalPlain;
    return pair_ok ? kBufferPair : (plain_ok ? kBufferPlain : kGlobalPlain);
}

// Star-shaped contours: direction tables (antipode, symmetric neighbour graph in CSR form), the
// per-direction radii (n x D) and the smoothing weight.
struct StarArgs {
    const int *anti;        // antipode of each direction
    const uint16_t *nb;     // neighbours of each direction: nb_chunks x 8 entries, 0xffff past the last
    int nb_chunks;
    float *Rk;
    float lambda;
};

struct EvolveArgs {
    JobParams p;
    DevContour *st;
    int n;                       // contours
    int n_iter;
    float *trace;                // n x SNK_TRACE_W or null
    unsigned long long *counter; // contour-iterations evolved
    int tile_cap;                // voxels of the per-contour LDS box (0: corners read from the volume)
    const int *idx;              // contour of each launch slot, n of them (null: slot i is contour i)
    // soft repulsion (kappa > 0): snapshot of every contour, each contour's neighbour list
    const float4 *snap;          // 2 per contour: (anchor bits x3, R), (offset x3, live)
    const int *nb, *nbn;         // nb_cap neighbour indices per contour (ascending), their counts
    int nb_cap;
    float kappa;
};

// Neighbour lists of the soft repulsion (neighbours.hip): a grid of cell >= 2 rho r_max over the live
// contours, then per ACTIVE contour the live contours whose inner sphere overlaps its own.
struct NeighbourArgs {
    float4 *snap;
    int *cell_start, *cell_fill, *items, *cell_of;   // grid: G + 1, G, n, n
    int *nb, *nbn;               // n x cap, n
    int *overflow;               // set when a contour has more than cap neighbours
    int cap;
    int G[3];
    float cell;
    const DevContour *status;
};
hipError_t launch_neighbours(const DevContour *st, int n, const Geometry &g, int dim, float rho,
                             const NeighbourArgs &b, hipStream_t s);

// One job of a batch, resident in device memory.
struct JobDev {
    JobParams p;
    DevContour *st;
    double *e_vox;
    int n;
    int target;                  // iteration count every contour evolves to
    float e0;
    int *cell_start, *cell_fill, *items, *cell_of, *dec;   // selection scratch
    int G[3];
    float cell;
    unsigned long long *kept;    // final selection: contours kept; culling pass: contours retired
    int mode;                    // 0: final selection, 1: culling pass during evolution, 2: final
                                 // selection ranked by the last Monte-Carlo energy (star contours)
    int grace;                   // culling pass: iterations before E_mc > e_cull retires a contour
    float e_cull;                // culling pass: threshold of its candidates (E0 or laxer)
    int compete;                 // culling pass: overlapping candidates compete (else all survive)
};

struct BatchArgs {
    const JobDev *jobs;
    const int2 *items;           // (job, contour)
    int n_items;
    int *queue;                  // work-queue head (persistent launch)
    int chunk;                   // iterations per contour in this launch
    unsigned long long *counter;
    int max_D, max_M;
    int tile_cap;                // voxels of each workgroup's LDS box (0: corners read from the volumes)
};

struct PrepassArgs {
    const void *raw;
    int dtype;
    float *J;
    float4 *Jq;                  // quad layout output, or null
    float2 *Jp;                  // column-pair layout output (2D), or null
    int nx, ny, nz;
    float i_offset, i_scale;
    int rx, ry, rz;              // tap radii per axis (0: axis not smoothed)
    float gx[33], gy[33], gz[33];
};

constexpr int kPrepassTX = 64;
constexpr int kPrepassMaxR = 16;
constexpr size_t kPrepassMaxLds = 65536;

hipError_t launch_prepass(const PrepassArgs &a, hipStream_t s);
bool prepass_lds_limit_ok(int rx, int ry, int rz);
// Pack J into the quad layout (one record per voxel, neighbours clamped at the upper edges).
hipError_t launch_pack_quad(const float *J, float4 *Jq, int nx, int ny, int nz, hipStream_t s);
hipError_t launch_pack_pair(const float *J, float2 *Jp, int nx, int ny, int nz, hipStream_t s);
// lanes: contour group size 16, 32, 64, 128 or 256; unroll: pair-points in flight (1 or 2);
// layout: a VolumeLayout (batched launches and LDS boxes: buffer layouts only). a.tile_cap > 0
// (whole-wave groups, Monte-Carlo sums) stages each contour's ball in an LDS box of that many voxels.
hipError_t launch_evolve(const EvolveArgs &a, int dim, int lanes, int unroll, int layout, bool trace,
                         hipStream_t s);
// a.tile_cap > 0: each workgroup stages its contour's ball in an LDS box of that many voxels.
hipError_t launch_evolve_batch(const BatchArgs &a, int dim, int lanes, int unroll, int layout, bool persistent,
                               int grid, hipStream_t s);
// Workgroups per CU of a batched launch shape (registers and LDS, including a box of tile_cap voxels).
int evolve_batch_max_blocks(int dim, int lanes, int unroll, int layout, int max_M, int tile_cap);
size_t evolve_lds_bytes(int dim, int lanes, int M, int tile_cap);
// Star-shaped contours (one wave per contour, n_radial 16).
hipError_t launch_star(const EvolveArgs &a, const StarArgs &sa, int dim, int lanes, int layout, hipStream_t s);
size_t star_lds_bytes(int dim, int D, int M, int lanes);
// Every direction's radius of contour i set to its R.
hipError_t launch_star_init(const DevContour *st, float *Rk, int n, int D, hipStream_t s);
// Workgroups per CU that registers allow for a launch shape with LDS boxes (0: no such shape).
int evolve_stage_blocks_per_cu(int dim, int lanes, int unroll, int layout);

// Engine helpers (engine_kernels.hip).
hipError_t launch_reset_items(const JobDev *jobs, const int2 *items, int n_items, const DevContour *const *init,
                              hipStream_t s);
hipError_t launch_zero(unsigned long long *p, int n, hipStream_t s);
hipError_t launch_count_unfinished(const JobDev *jobs, const int2 *items, int n_items, int *unfinished, hipStream_t s);
// finalize: contours still ACTIVE become MAXITER and E_vox is stored in the state (else only in
// e_vox).
hipError_t launch_energy_vox(const JobParams &p, DevContour *st, double *e_vox, int n, int dim, bool finalize,
                             hipStream_t s);
// Contours still ACTIVE become MAXITER (the end of evolution without the exact energy).
hipError_t launch_mark_maxiter(DevContour *st, int n, hipStream_t s);
// Indices of the ACTIVE contours among st[0..n-1] into idx, their number into *count (which must be
// zero beforehand); the order of the indices is unspecified.
hipError_t launch_compact_active(const DevContour *st, int n, int *idx, int *count, hipStream_t s);
// rounds: 3 ints of device scratch for the grid-wide rounds (null: one workgroup does everything).
hipError_t launch_select(const JobDev &j, int dim, int *rounds, hipStream_t s);
hipError_t launch_energy_vox_batch(const JobDev *jobs, const int2 *items, int n_items, int dim, hipStream_t s);
hipError_t launch_select_batch(const JobDev *jobs, const int *job_list, int n_jobs, int dim, hipStream_t s);

}  // namespace snk

// Uniform selection grid for one volume (defined in api.hip).
int64_t snk_grid_for(const snk_params &P, int64_t nx, int64_t ny, int64_t nz, int G[3], double *cell_out);
