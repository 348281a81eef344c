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

struct EvolveArgs {
    Geometry g;
    const float *dirs;           // D x dim
    DevContour *st;
    int n;                       // contours
    int n_iter;
    int D, M, L;
    uint32_t key0, key1;
    int flags;
    float dR, eps0, r_lo, r_hi, conv_tol;
    int conv_window;
    float *trace;                // n x SNK_TRACE_W or null
    unsigned long long *counter; // contour-iterations evolved
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

struct FinalizeArgs {
    Geometry g;
    DevContour *st;
    double *e_vox;
    int n;
    float dR;
    float e0;
    float r_hi;
    // selection scratch (single-workgroup kernel)
    int *cell_start;     // G + 1
    int *cell_fill;      // G
    int *items;          // n
    int *cell_of;        // n
    int *dec;            // n
    int G[3];
    float cell;          // physical cell size
    unsigned long long *counter;  // survivors
};

constexpr int kPrepassTX = 64;
constexpr int kPrepassMaxR = 16;
constexpr size_t kPrepassMaxLds = 65536;

hipError_t launch_prepass(const PrepassArgs &a, hipStream_t s);
bool prepass_lds_limit_ok(int rx, int ry, int rz);
hipError_t launch_evolve(const EvolveArgs &a, int dim, int waves, int unroll, bool trace, hipStream_t s);
hipError_t launch_energy_vox(const FinalizeArgs &a, int dim, hipStream_t s);
hipError_t launch_select(const FinalizeArgs &a, int dim, hipStream_t s);

}  // namespace snk
