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
    int buffer_ok;               // volume fits a 32-bit buffer descriptor
};

struct EvolveArgs {
    JobParams p;
    DevContour *st;
    int n;                       // contours
    int n_iter;
    float *trace;                // n x SNK_TRACE_W or null
    unsigned long long *counter; // contour-iterations evolved
    int box_cap;                 // LDS floats for the staged footprint (0: gather from memory)
};

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
    unsigned long long *kept;
};

struct BatchArgs {
    const JobDev *jobs;
    const int2 *items;           // (job, contour)
    int n_items;
    int *queue;                  // work-queue head (persistent launch)
    int chunk;                   // iterations per contour in this launch
    unsigned long long *counter;
    int max_D, max_M;
    int box_cap;                 // LDS floats for the staged footprint (0: gather from memory)
};

struct PrepassArgs {
    const void *raw;
    int dtype;
    float *J;
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
hipError_t launch_evolve(const EvolveArgs &a, int dim, int waves, int unroll, bool trace, hipStream_t s);
hipError_t launch_evolve_batch(const BatchArgs &a, int dim, int waves, int unroll, bool persistent, int grid,
                               hipStream_t s);
int evolve_batch_max_blocks(int dim, int waves, int unroll, int max_D, int max_M, int box_cap);
size_t evolve_lds_bytes(int dim, int waves, int D, int M, int box_cap);
// LDS floats for the staged footprint: `requested` > 0 as given, 0 = automatic (the box of a contour
// of radius about 1.5 r_init, bounded by what fits the workgroup's LDS), < 0 = off.
int evolve_box_cap(int requested, int dim, int waves, int D, int M, const snk_params &P);

// Engine helpers (engine_kernels.hip).
hipError_t launch_reset_items(const JobDev *jobs, const int2 *items, int n_items, const DevContour *const *init,
                              hipStream_t s);
hipError_t launch_zero(unsigned long long *p, int n, hipStream_t s);
hipError_t launch_count_unfinished(const JobDev *jobs, const int2 *items, int n_items, int *unfinished, hipStream_t s);
hipError_t launch_energy_vox(const JobParams &p, DevContour *st, double *e_vox, int n, int dim, hipStream_t s);
hipError_t launch_select(const JobDev &j, int dim, hipStream_t s);
hipError_t launch_energy_vox_batch(const JobDev *jobs, const int2 *items, int n_items, int dim, hipStream_t s);
hipError_t launch_select_batch(const JobDev *jobs, const int *job_list, int n_jobs, int dim, hipStream_t s);

}  // namespace snk

// Uniform selection grid for one volume (defined in api.hip).
int64_t snk_grid_for(const snk_params &P, int64_t nx, int64_t ny, int64_t nz, int G[3], double *cell_out);
