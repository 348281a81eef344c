// Host side of the C ABI declared in include/snk.h: context, device buffers, parameter
// validation, kernel launches on the caller's stream, readback and event timing.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "snk_internal.h"

using snk::DevContour;

struct snk_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    snk_params P{};
    bool have_params = false;
    int lanes = 0;   // lanes per contour (0: automatic)
    int unroll = 0;  // pair-points in flight (0: automatic)
    int layout_req = 0;  // volume layout: 0 automatic, 1 plain, 2 quad
    int tile_req = -1;   // LDS box per contour, voxels: -1 automatic, 0 off
    int cus = 0;         // compute units of the device
    int lds_per_cu = 0;  // LDS bytes per compute unit
    int stage_key = -1, stage_blocks = 0;  // registers-limited workgroups per CU of the last staged shape
    int last_lanes = 0, last_unroll = 0, last_layout = 0, last_tile = 0;  // last evolve launch

    // culling passes of snk_evolve_cull: threshold (NaN: params.e0) and competition
    double cull_thr = NAN;
    int cull_compete = 1;
    // passes applied inside the evolve kernel (every 0: none): pass interval, grace, run length
    int cull_in_every = 0, cull_in_grace = 0, cull_in_end = 0;

    // soft repulsion (kappa 0: off): strength, iterations per neighbour snapshot, buffers
    double repel_kappa = 0.0;
    int repel_every = 1;
    float4 *d_snap = nullptr;
    int *d_nbgrid = nullptr, *d_nbitems = nullptr, *d_rnb = nullptr;
    size_t snap_cap = 0, nbgrid_cap = 0, nbitems_cap = 0, rnb_cap = 0;

    // star-shaped contours (lambda < 0: off)
    double star_lambda = -1.0;
    int *d_anti = nullptr;
    uint16_t *d_nb = nullptr;  // neighbour rows, nb_chunks x 8 entries each, padded with D
    int nb_chunks = 0;
    size_t anti_cap = 0, nb_cap = 0;
    std::vector<float> star_dirs;    // the table the star tables were built from
    float *d_Rk = nullptr;           // n x D radii
    size_t Rk_cap = 0;
    bool Rk_valid = false;
    int layout = snk::kGlobalPlain;  // layout of the current pre-pass output

    std::vector<float> dirs_host;
    float *d_dirs = nullptr;
    size_t dirs_cap = 0;
    int D = 0;

    int64_t nx = 0, ny = 0, nz = 0;
    snk_dtype dtype = SNK_U8;
    const void *raw = nullptr;      // borrowed or owned
    void *raw_owned = nullptr;
    size_t raw_owned_cap = 0;
    float *J = nullptr;
    size_t J_cap = 0;
    float4 *Jq = nullptr;   // quad layout copy of J (when the layout is quad)
    size_t Jq_cap = 0;
    bool have_volume = false;
    bool J_dirty = true;

    int64_t n = 0;
    DevContour *d_st = nullptr;
    double *d_evox = nullptr;
    size_t n_cap = 0, evox_cap = 0;
    float *d_trace = nullptr;
    size_t trace_cap = 0;

    int *d_cell_start = nullptr, *d_cell_fill = nullptr, *d_items = nullptr, *d_cell_of = nullptr,
        *d_dec = nullptr;
    size_t grid_cap = 0, grid_fill_cap = 0, sel_cap = 0;

    unsigned long long *d_counters = nullptr;  // [0] evolved, [1] kept, [2..3] selection round counters
    unsigned char *scratch = nullptr;  // this device's copy of the static selection scratch (no-alloc finalize)
    int *d_live = nullptr;             // snk_evolve_cull: indices of the active contours, then their count
    size_t live_cap = 0;

    // pinned staging of contour records for host <-> device copies; ev_stage marks the end of the
    // last upload from it, which must complete before the buffer is written again
    DevContour *h_stage = nullptr;
    size_t stage_cap = 0;
    hipEvent_t ev_stage = nullptr;
    bool stage_busy = false;

    hipEvent_t ev[6] = {};
    bool ev_pre = false, ev_evo = false, ev_fin = false;
    int64_t evolve_launches = 0;
};

// Scratch of snk_finalize_noalloc, a static device array so that the call allocates nothing: the
// selection counters (kept count and the grid-wide round counters), the cell starts and fills of
// the uniform grid, and the per-contour item, cell and decision arrays. Every device the library
// runs on holds one copy until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for that device (the array's name is a host-side stand-in).
namespace {
constexpr int64_t kNoAllocMaxContours = (int64_t)1 << 17;
constexpr int64_t kNoAllocMaxCells = (int64_t)1 << 19;
constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kNaCounters = 0;                                                   // 4 x u64
constexpr size_t kNaCellStart = 256;                                                // cells + 1 ints
constexpr size_t kNaCellFill = kNaCellStart + align256((kNoAllocMaxCells + 1) * 4); // cells + 1 ints
constexpr size_t kNaItems = kNaCellFill + align256((kNoAllocMaxCells + 1) * 4);     // contours ints
constexpr size_t kNaCellOf = kNaItems + align256(kNoAllocMaxContours * 4);
constexpr size_t kNaDec = kNaCellOf + align256(kNoAllocMaxContours * 4);
constexpr size_t kNoAllocScratchBytes = kNaDec + align256(kNoAllocMaxContours * 4);
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
unsigned char *g_scratch_addr[kMaxDevices] = {};

// The device address of `scratch` on `device` (which must be current), looked up once per device.
hipError_t scratch_address(int device, unsigned char **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}
}  // namespace

namespace {

thread_local std::string g_create_err;

snk_status fail(snk_ctx *c, snk_status code, const std::string &msg) {
    if (c) c->err = msg;
    else g_create_err = msg;
    return code;
}

snk_status hip_fail(snk_ctx *c, hipError_t e, const char *what) {
    return fail(c, SNK_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPTRY(c, call)                                      \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail((c), e_, #call); \
    } while (0)

template <typename T>
snk_status ensure(snk_ctx *c, T **p, size_t *cap, size_t count) {
    if (*cap >= count && *p) return SNK_OK;
    if (*p) {
        hipError_t e = hipFree(*p);
        *p = nullptr;
        *cap = 0;
        if (e != hipSuccess) return hip_fail(c, e, "hipFree");
    }
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return fail(c, SNK_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    *p = static_cast<T *>(q);
    *cap = count;
    return SNK_OK;
}

double rho_of(int dim) { return dim == 3 ? pow(2.0, -1.0 / 3.0) : sqrt(0.5); }

double r_low(const snk_params &p) {
    const double rho = rho_of(p.dim);
    const double geo = p.dR * (1.0 + rho) / (2.0 * (1.0 - rho));
    return std::max(p.r_min, geo);
}

snk_status check_params(snk_ctx *c, const snk_params &p) {
    if (p.dim != 2 && p.dim != 3) return fail(c, SNK_EINVAL, "dim must be 2 or 3");
    for (int i = 0; i < 3; ++i)
        if (!(p.spacing[i] > 0.0) || !isfinite(p.spacing[i])) return fail(c, SNK_EINVAL, "spacing must be > 0");
    if (!(p.sigma_pre >= 0.0)) return fail(c, SNK_EINVAL, "sigma_pre must be >= 0");
    if (!isfinite(p.i_offset) || !isfinite(p.i_scale)) return fail(c, SNK_EINVAL, "i_offset/i_scale not finite");
    if (!(p.dR > 0.0)) return fail(c, SNK_EINVAL, "dR must be > 0");
    if (!(p.eps0 >= 0.0) || !isfinite(p.eps0)) return fail(c, SNK_EINVAL, "eps0 must be finite and >= 0");
    if (!(p.r_max >= r_low(p))) return fail(c, SNK_EINVAL, "r_max below the smallest admissible radius");
    if (p.n_dirs <= 0) return fail(c, SNK_EINVAL, "n_dirs must be > 0");
    if (p.n_rays <= 0 || (p.n_rays & 1)) return fail(c, SNK_EINVAL, "n_rays must be even and > 0");
    if (p.n_radial <= 0) return fail(c, SNK_EINVAL, "n_radial must be > 0");
    if ((int64_t)p.n_rays * p.n_radial > (1 << 20)) return fail(c, SNK_EINVAL, "n_rays*n_radial too large");
    if (!(p.conv_tol >= 0.0) || p.conv_window < 0 || p.conv_window > 255)
        return fail(c, SNK_EINVAL, "conv_tol >= 0 and 0 <= conv_window <= 255 required");
    if (!isfinite(p.e0)) return fail(c, SNK_EINVAL, "e0 not finite");
    if (p.flags & ~(snk::kFlagNoRotation | snk::kFlagExact | snk::kFlagGradI))
        return fail(c, SNK_EINVAL, "unknown flag bits");
    if ((p.flags & snk::kFlagExact) && (p.flags & snk::kFlagGradI))
        return fail(c, SNK_EINVAL, "flags bits 1 (exact sums) and 2 (gradient-form centre force) exclude each other");
    return SNK_OK;
}

bool same_prepass(const snk_params &a, const snk_params &b) {
    return a.dim == b.dim && a.sigma_pre == b.sigma_pre && a.i_offset == b.i_offset && a.i_scale == b.i_scale &&
           a.spacing[0] == b.spacing[0] && a.spacing[1] == b.spacing[1] && a.spacing[2] == b.spacing[2];
}

}  // namespace

// Uniform grid for the selection: cell >= rho * r_max (plus a rounding margin), so overlapping
// pairs sit in neighbouring cells; grown if the grid would exceed 2^22 cells.
int64_t snk_grid_for(const snk_params &P, int64_t nx, int64_t ny, int64_t nz, int G[3], double *cell_out) {
    const double rho = P.dim == 3 ? pow(2.0, -1.0 / 3.0) : sqrt(0.5);
    double cell = rho * P.r_max * 1.01 + 0.01;
    const int64_t nn[3] = {nx, ny, nz};
    int64_t total = 1;
    for (int iter = 0; iter < 64; ++iter) {
        total = 1;
        for (int i = 0; i < 3; ++i) {
            const int64_t gi = i < P.dim ? (int64_t)floor((double)(nn[i] - 1) * P.spacing[i] / cell) + 1 : 1;
            G[i] = (int)gi;
            total *= gi;
        }
        if (total <= ((int64_t)1 << 22)) break;
        cell *= 1.5;
    }
    *cell_out = cell;
    return total;
}

namespace {

snk::Geometry geometry(const snk_ctx *c) {
    snk::Geometry g;
    g.J = c->J;
    // quad records, or the column pairs of a 2D image (8 bytes per pixel in the same buffer)
    g.Jq = (c->layout == snk::kBufferQuad || c->layout == snk::kBufferPair) ? c->Jq : nullptr;
    g.nx = (int)c->nx;
    g.ny = (int)c->ny;
    g.nz = (int)c->nz;
    for (int i = 0; i < 3; ++i) {
        g.h[i] = (float)c->P.spacing[i];
        g.inv_h[i] = (float)(1.0 / c->P.spacing[i]);
    }
    return g;
}

// centre (physical, double) -> anchor + offset (voxel units)
void to_anchor(const snk_ctx *c, const double *cen, DevContour &s) {
    for (int i = 0; i < 3; ++i) {
        if (i >= c->P.dim) {
            s.anc[i] = 0;
            s.off[i] = 0.0f;
            continue;
        }
        const double v = cen[i] / c->P.spacing[i];
        const double a = floor(v + 0.5);
        s.anc[i] = (int32_t)std::max(std::min(a, 2.0e9), -2.0e9);
        s.off[i] = (float)(v - (double)s.anc[i]);
    }
}

bool inside(const snk_ctx *c, const DevContour &s) {
    const int64_t nn[3] = {c->nx, c->ny, c->nz};
    for (int i = 0; i < c->P.dim; ++i) {
        const double v = (double)s.anc[i] + (double)s.off[i];
        if (!(v >= 0.0) || v > (double)(nn[i] - 1)) return false;
    }
    return true;
}

snk_status need(snk_ctx *c, bool vol, bool seeds) {
    if (!c->have_params) return fail(c, SNK_ESTATE, "parameters not set");
    if (vol && !c->have_volume) return fail(c, SNK_ESTATE, "no volume loaded");
    if (seeds && c->n <= 0) return fail(c, SNK_ESTATE, "no seeds loaded");
    return SNK_OK;
}

// The second copy of J that the layout reads (quad records, or the column pairs of a 2D image, in
// one float4 buffer), allocated once.
snk_status ensure_layout_buffer(snk_ctx *c, int layout) {
    const size_t vox = (size_t)(c->nx * c->ny * c->nz);
    if (layout == snk::kBufferQuad) return ensure(c, &c->Jq, &c->Jq_cap, vox);
    if (layout == snk::kBufferPair) return ensure(c, &c->Jq, &c->Jq_cap, (vox + 1) / 2);
    return SNK_OK;
}

snk_status run_prepass(snk_ctx *c) {
    snk::PrepassArgs a{};
    a.raw = c->raw;
    a.dtype = (int)c->dtype;
    a.J = c->J;
    a.nx = (int)c->nx;
    a.ny = (int)c->ny;
    a.nz = (int)c->nz;
    a.i_offset = (float)c->P.i_offset;
    a.i_scale = (float)c->P.i_scale;
    int *rad[3] = {&a.rx, &a.ry, &a.rz};
    float *tap[3] = {a.gx, a.gy, a.gz};
    const int64_t nn[3] = {c->nx, c->ny, c->nz};
    for (int ax = 0; ax < 3; ++ax) {
        const double s = c->P.sigma_pre / c->P.spacing[ax];
        const bool use = s > 0.0 && ax < c->P.dim && nn[ax] > 1;
        const int r = use ? (int)ceil(3.0 * s) : 0;
        if (r > snk::kPrepassMaxR) return fail(c, SNK_EINVAL, "sigma_pre too large for the pre-pass (radius > 16)");
        *rad[ax] = r;
        std::vector<double> g(2 * r + 1);
        double sum = 0.0;
        for (int k = -r; k <= r; ++k) {
            g[k + r] = r ? exp(-(double)k * k / (2.0 * s * s)) : 1.0;
            sum += g[k + r];
        }
        for (int k = 0; k <= 2 * r; ++k) tap[ax][k] = (float)(g[k] / sum);
    }
    if (!snk::prepass_lds_limit_ok(a.rx, a.ry, a.rz))
        return fail(c, SNK_EINVAL, "sigma_pre too large for the pre-pass tile (LDS > 64 KiB)");
    const int layout = snk::volume_layout(c->P.dim, c->nx, c->ny, c->nz, c->layout_req);
    if (layout < 0)
        return fail(c, SNK_EINVAL, "volume too large for the requested layout");
    snk_status lst = ensure_layout_buffer(c, layout);
    if (lst != SNK_OK) return lst;
    a.Jq = layout == snk::kBufferQuad ? c->Jq : nullptr;
    a.Jp = layout == snk::kBufferPair ? reinterpret_cast<float2 *>(c->Jq) : nullptr;
    HIPTRY(c, hipEventRecord(c->ev[0], c->stream));
    HIPTRY(c, snk::launch_prepass(a, c->stream));
    HIPTRY(c, hipEventRecord(c->ev[1], c->stream));
    c->layout = layout;
    c->ev_pre = true;
    c->J_dirty = false;
    return SNK_OK;
}

// Lanes per contour: whole waves with at least two pair-points per lane; sub-wave groups only
// when a contour has fewer pair-points than a wave has lanes.
int pick_lanes(const snk_ctx *c) {
    if (c->lanes > 0) return c->lanes;
    const int64_t pairs = (int64_t)(c->P.n_rays / 2) * c->P.n_radial;
    int g = 256;
    while (g > 64 && 2 * g > pairs) g >>= 1;
    while (g > 16 && g > pairs) g >>= 1;
    return g;
}

snk::JobParams job_params(const snk_ctx *c) {
    snk::JobParams p{};
    p.g = geometry(c);
    p.dirs = c->d_dirs;
    p.D = c->D;
    p.M = c->P.n_rays;
    p.L = c->P.n_radial;
    p.key0 = (uint32_t)(c->P.seed & 0xffffffffu);
    p.key1 = (uint32_t)(c->P.seed >> 32);
    p.flags = c->P.flags;
    p.dR = (float)c->P.dR;
    p.eps0 = (float)c->P.eps0;
    p.r_lo = (float)r_low(c->P);
    p.r_hi = (float)c->P.r_max;
    p.conv_tol = (float)c->P.conv_tol;
    p.conv_window = c->P.conv_window;
    p.in_slope = (float)(2.0 / (rho_of(c->P.dim) * c->P.dR));
    p.out_slope = (float)(1.0 / c->P.dR);
    return p;
}

struct McShape {
    int lanes, unroll, tile;
};

// Launch shape of a Monte-Carlo evolve over `layout`. Explicit knobs are taken as set. The automatic
// LDS box applies when every contour can stay resident at once, ceil(n / CUs) workgroups per CU,
// and there are more than four of them per CU (the common case of one volume with a few thousand
// cells: their footprints overflow the L2, which a handful of contours per CU do not, where
// staging only adds latency): two waves per contour when a contour has at least four pair-points
// per lane of them, else one (unless set), four pair-points in flight with two waves (two if that
// would leave contours waiting, or with one wave), and the largest box whose LDS still leaves room
// for all of them. Otherwise no box and the lane rule of pick_lanes.
McShape mc_shape(snk_ctx *c, int M, int layout) {
    McShape s;
    s.lanes = pick_lanes(c);
    s.unroll = c->unroll > 0 ? c->unroll : (s.lanes >= 64 ? 2 : 1);
    s.tile = 0;
    if (c->tile_req > 0) {
        s.tile = c->tile_req;
        return s;
    }
    if (c->tile_req == 0 || c->n <= 0 || c->cus <= 0 || c->lds_per_cu <= 0) return s;
    if (layout != snk::kBufferQuad && layout != snk::kBufferPlain && !(c->P.dim == 3 && layout == snk::kBufferPair))
        return s;
    const int64_t pairs = (int64_t)(M / 2) * c->P.n_radial;
    const int64_t per_cu = (c->n + c->cus - 1) / c->cus;
    if (per_cu <= 4) return s;
    const int G = c->lanes > 0 ? c->lanes : (pairs >= 512 ? 128 : (pairs >= 128 ? 64 : 0));
    if (G < 64) return s;
    // two-wave groups with at least four pair-points per lane take all four in one pass when the
    // contours still fit at that register count
    int U = c->unroll > 0 ? c->unroll : ((G == 128 && pairs >= 4 * G) ? 4 : 2);
    for (;;) {
        const int key = ((c->P.dim * 512 + G) * 8 + U) * 4 + layout;
        if (key != c->stage_key) {
            c->stage_blocks = snk::evolve_stage_blocks_per_cu(c->P.dim, G, U, layout);
            c->stage_key = key;
        }
        if (per_cu <= c->stage_blocks) break;
        if (c->unroll > 0 || U == 2) return s;
        U = 2;
    }
    const size_t other = snk::evolve_lds_bytes(c->P.dim, G, M, 0);
    // LDS is handed out in 512-byte blocks
    const size_t budget = std::min<size_t>((size_t)c->lds_per_cu / (size_t)per_cu, 65536) & ~(size_t)511;
    if (budget <= other) return s;
    const int tile = (int)std::min<size_t>((budget - other) / 4, 16384) & ~63;
    if (tile < 1024) return s;
    s.lanes = G;
    s.unroll = U;
    s.tile = tile;
    return s;
}

// Re-packs the current J when the requested layout changed after the pre-pass.
snk_status ensure_layout(snk_ctx *c) {
    const int layout = snk::volume_layout(c->P.dim, c->nx, c->ny, c->nz, c->layout_req);
    if (layout < 0)
        return fail(c, SNK_EINVAL, "volume too large for the requested layout");
    if (layout == c->layout) return SNK_OK;
    snk_status st = ensure_layout_buffer(c, layout);
    if (st != SNK_OK) return st;
    if (layout == snk::kBufferQuad)
        HIPTRY(c, snk::launch_pack_quad(c->J, c->Jq, (int)c->nx, (int)c->ny, (int)c->nz, c->stream));
    if (layout == snk::kBufferPair)
        HIPTRY(c, snk::launch_pack_pair(c->J, reinterpret_cast<float2 *>(c->Jq), (int)c->nx, (int)c->ny, (int)c->nz,
                                          c->stream));
    c->layout = layout;
    return SNK_OK;
}

// Direction tables of the star contour from the context's direction table: the opposite direction
// of each (|T_j + T_k| < 1e-4, else SNK_EINVAL), and a symmetric graph: the 6 (3D) or 2 (2D)
// directions of largest dot product with T_k (ties to the lower index), closed under symmetry,
// neighbours in ascending order.
snk_status star_tables(snk_ctx *c) {
    const int dim = c->P.dim, D = c->D;
    if (c->star_dirs == c->dirs_host && c->d_anti) return SNK_OK;
    const std::vector<float> &T = c->dirs_host;
    std::vector<int> anti(D), off(D + 1, 0), idx;
    for (int k = 0; k < D; ++k) {
        int best = -1;
        double bd = 1e30;
        for (int j = 0; j < D; ++j) {
            double e2 = 0.0;
            for (int a = 0; a < dim; ++a) {
                const double t = (double)T[j * dim + a] + (double)T[k * dim + a];
                e2 += t * t;
            }
            if (e2 < bd) {
                bd = e2;
                best = j;
            }
        }
        if (!(sqrt(bd) < 1e-4)) return fail(c, SNK_EINVAL, "star contours need a direction table with antipodes");
        anti[k] = best;
    }
    const int deg = dim == 3 ? 6 : 2;
    std::vector<int> knn((size_t)D * deg, -1);
    std::vector<double> dots(D);
    std::vector<char> used(D);
    for (int k = 0; k < D; ++k) {
        for (int j = 0; j < D; ++j) {
            double dt = 0.0;
            for (int a = 0; a < dim; ++a) dt += (double)T[j * dim + a] * (double)T[k * dim + a];
            dots[j] = dt;
            used[j] = j == k;
        }
        // repeated maximum; dot products within 1e-6 tie and the lower index wins, so a table given
        // in FP32 yields the graph its exact directions define
        for (int t = 0; t < deg && t < D - 1; ++t) {
            int best = -1;
            for (int j = 0; j < D; ++j)
                if (!used[j] && (best < 0 || dots[j] > dots[best] + 1e-6)) best = j;
            used[best] = 1;
            knn[(size_t)k * deg + t] = best;
        }
    }
    for (int k = 0; k < D; ++k) {
        for (int j = 0; j < D; ++j) {
            if (j == k) continue;
            bool edge = false;
            for (int t = 0; t < deg; ++t)
                edge = edge || knn[(size_t)k * deg + t] == j || knn[(size_t)j * deg + t] == k;
            if (edge) idx.push_back(j);
        }
        off[k + 1] = (int)idx.size();
    }
    snk_status st = ensure(c, &c->d_anti, &c->anti_cap, (size_t)D);
    if (st != SNK_OK) return st;
    // rows of whole 16-byte chunks (8 entries, in the order above, padded with the index D, whose
    // radius entry the kernel holds at zero), so the kernel loads a direction's neighbours with
    // independent vector loads and reads every entry without a branch
    if (D >= 0xffff) return fail(c, SNK_EINVAL, "star contours need fewer than 65535 directions");
    int maxdeg = 1;
    for (int k = 0; k < D; ++k) maxdeg = std::max(maxdeg, off[k + 1] - off[k]);
    const int chunks = (maxdeg + 7) / 8;
    std::vector<uint16_t> nb((size_t)D * chunks * 8, (uint16_t)D);
    for (int k = 0; k < D; ++k)
        for (int b = off[k]; b < off[k + 1]; ++b) nb[(size_t)k * chunks * 8 + (b - off[k])] = (uint16_t)idx[b];
    st = ensure(c, &c->d_nb, &c->nb_cap, nb.size());
    if (st != SNK_OK) return st;
    HIPTRY(c, hipMemcpyAsync(c->d_anti, anti.data(), sizeof(int) * D, hipMemcpyHostToDevice, c->stream));
    HIPTRY(c, hipMemcpyAsync(c->d_nb, nb.data(), sizeof(uint16_t) * nb.size(), hipMemcpyHostToDevice, c->stream));
    c->nb_chunks = chunks;
    HIPTRY(c, hipStreamSynchronize(c->stream));
    c->star_dirs = c->dirs_host;
    return SNK_OK;
}

// Per-direction radii of every contour, set tied to its R unless already valid.
snk_status star_radii(snk_ctx *c) {
    snk_status st = ensure(c, &c->d_Rk, &c->Rk_cap, (size_t)std::max<int64_t>(c->n * c->D, 1));
    if (st != SNK_OK) return st;
    if (!c->Rk_valid) {
        HIPTRY(c, snk::launch_star_init(c->d_st, c->d_Rk, (int)c->n, c->D, c->stream));
        c->Rk_valid = true;
    }
    return SNK_OK;
}

snk_status run_star(snk_ctx *c, int32_t n_iter, bool standalone) {
    if (c->P.flags & (snk::kFlagExact | snk::kFlagGradI))
        return fail(c, SNK_EINVAL, "star contours take Monte-Carlo sums with the weight-form centre force");
    if (c->P.n_radial != 16) return fail(c, SNK_EINVAL, "star contours need n_radial = 16");
    // one or two waves per contour (lanes_per_contour 64 or 128; automatic: two)
    const int lanes = c->lanes > 0 ? c->lanes : 128;
    if (lanes != 64 && lanes != 128) return fail(c, SNK_EINVAL, "star contours take 64 or 128 lanes per contour");
    if (snk::star_lds_bytes(c->P.dim, c->D, c->P.n_rays, lanes) > 65536)
        return fail(c, SNK_EINVAL, "n_dirs / n_rays too large for the star kernel's LDS (64 KiB)");
    snk_status st = star_tables(c);
    if (st != SNK_OK) return st;
    st = star_radii(c);
    if (st != SNK_OK) return st;
    snk::EvolveArgs a{};
    a.p = job_params(c);
    a.st = c->d_st;
    a.n = (int)c->n;
    a.n_iter = n_iter;
    a.counter = c->d_counters;
    snk::StarArgs sa{};
    sa.anti = c->d_anti;
    sa.nb = c->d_nb;
    sa.nb_chunks = c->nb_chunks;
    sa.Rk = c->d_Rk;
    sa.lambda = (float)c->star_lambda;
    if (standalone) {
        HIPTRY(c, hipMemsetAsync(c->d_counters, 0, sizeof(unsigned long long), c->stream));
        HIPTRY(c, hipEventRecord(c->ev[2], c->stream));
    }
    const int layout = c->layout;
    HIPTRY(c, snk::launch_star(a, sa, c->P.dim, lanes, layout, c->stream));
    if (standalone) {
        HIPTRY(c, hipEventRecord(c->ev[3], c->stream));
        c->ev_evo = true;
    }
    c->last_lanes = lanes;
    c->last_unroll = 2;
    c->last_layout = layout;
    c->last_tile = 0;
    c->evolve_launches += 1;
    return SNK_OK;
}

// standalone: zero the contour-iteration counter and record the evolve events around the launch
// (off for the chunks of snk_evolve_cull, which brackets the whole call).
constexpr int kNbCap = 64;   // neighbours per contour of the repulsion (one lane each)

// Buffers and grid of the repulsion's neighbour lists for the current contours.
snk_status neighbour_args(snk_ctx *c, snk::NeighbourArgs &b) {
    const double rho = rho_of(c->P.dim);
    double cell = 2.0 * rho * c->P.r_max * 1.01 + 0.01;
    const int64_t nn[3] = {c->nx, c->ny, c->nz};
    int64_t total = 1;
    for (int it = 0; it < 64; ++it) {
        total = 1;
        for (int i = 0; i < 3; ++i) {
            b.G[i] = i < c->P.dim ? (int)(floor((double)(nn[i] - 1) * c->P.spacing[i] / cell) + 1) : 1;
            total *= b.G[i];
        }
        if (total <= ((int64_t)1 << 20)) break;
        cell *= 1.5;
    }
    b.cell = (float)cell;
    const size_t n = (size_t)c->n;
    snk_status st = ensure(c, &c->d_snap, &c->snap_cap, 2 * n);
    if (st != SNK_OK) return st;
    st = ensure(c, &c->d_nbgrid, &c->nbgrid_cap, 2 * (size_t)(total + 1) + 1);
    if (st != SNK_OK) return st;
    st = ensure(c, &c->d_nbitems, &c->nbitems_cap, 3 * n);
    if (st != SNK_OK) return st;
    st = ensure(c, &c->d_rnb, &c->rnb_cap, n * kNbCap);
    if (st != SNK_OK) return st;
    b.snap = c->d_snap;
    b.cell_start = c->d_nbgrid;
    b.cell_fill = c->d_nbgrid + total + 1;
    b.overflow = c->d_nbgrid + 2 * (total + 1);
    b.items = c->d_nbitems;
    b.cell_of = c->d_nbitems + n;
    b.nbn = c->d_nbitems + 2 * n;
    b.nb = c->d_rnb;
    b.cap = kNbCap;
    b.status = c->d_st;
    return SNK_OK;
}

// idx (device, n_launch entries): evolve only those contours (the shape is still chosen for all n).
snk_status run_evolve(snk_ctx *c, int32_t n_iter, bool trace, bool standalone = true, const int *idx = nullptr,
                      int n_launch = -1) {
    if (c->D != c->P.n_dirs) return fail(c, SNK_ESTATE, "direction table size != params.n_dirs");
    if (c->J_dirty) {
        snk_status st = run_prepass(c);
        if (st != SNK_OK) return st;
    }
    snk_status lst = ensure_layout(c);
    if (lst != SNK_OK) return lst;
    if (c->star_lambda >= 0.0) {
        if (trace) return fail(c, SNK_EINVAL, "snk_trace_step does not cover star contours");
        if (c->repel_kappa > 0.0) return fail(c, SNK_EINVAL, "repulsion applies to sphere contours");
        return run_star(c, n_iter, standalone);
    }
    snk::EvolveArgs a{};
    a.p = job_params(c);
    a.p.cull_first = -1;
    if (c->cull_in_every > 0) a.p.cull_thr = (float)(std::isnan(c->cull_thr) ? c->P.e0 : c->cull_thr);
    // the pass points r = every, 2 every, ... of the run with grace <= r < end that fall in the
    // launch's iterations base + 1 .. base + len, as 0-based iterations of the launch
    auto cull_points = [&](int base, int len) {
        a.p.cull_first = -1;
        if (c->cull_in_every <= 0) return;
        const int every = c->cull_in_every;
        const int lo = std::max(base + 1, c->cull_in_grace), hi = std::min(base + len, c->cull_in_end - 1);
        const int first = (lo + every - 1) / every * every;
        if (lo > hi || first > hi) return;
        a.p.cull_first = first - base - 1;
        a.p.cull_every = every;
        a.p.cull_last = hi / every * every - base - 1;
    };
    a.st = c->d_st;
    a.n = idx ? n_launch : (int)c->n;
    a.idx = idx;
    a.n_iter = n_iter;
    a.trace = trace ? c->d_trace : nullptr;
    a.counter = c->d_counters;
    const bool exact = (c->P.flags & snk::kFlagExact) != 0;
    // exact sums read single voxels from J (the plain layout); so does the gradient-form kernel in
    // place of column pairs
    const bool gradi = (c->P.flags & snk::kFlagGradI) != 0;
    int layout = (exact && (c->layout == snk::kBufferQuad || c->layout == snk::kBufferPair)) ||
                         (gradi && c->P.dim == 2 && c->layout == snk::kBufferPair)
                     ? snk::kBufferPlain
                     : c->layout;
    int lanes, unroll;
    if (exact) {
        lanes = c->lanes > 0 ? c->lanes : 256;
        unroll = 1;
    } else {
        const McShape sh = mc_shape(c, a.p.M, layout);
        lanes = sh.lanes;
        unroll = sh.unroll;
        // LDS boxes: whole-wave groups over a buffer layout
        if (sh.tile > 0 && (lanes < 64 || layout == snk::kGlobalPlain))
            return fail(c, SNK_EINVAL, "LDS boxes need lanes_per_contour >= 64 and layout 1, 2 or 4");
        // with a box, the iterations whose ball does not fit read the plain copy
        if (sh.tile > 0 && layout == snk::kBufferPair && c->P.dim == 2) layout = snk::kBufferPlain;
        a.tile_cap = sh.tile;
        if (c->P.flags & snk::kFlagGradI) {
            // gradient-form centre force: whole-wave groups, two pair-points in flight
            if (c->lanes > 0 && c->lanes < 64)
                return fail(c, SNK_EINVAL, "the gradient-form centre force needs lanes_per_contour >= 64");
            if (layout == snk::kGlobalPlain)
                return fail(c, SNK_EINVAL, "the gradient-form centre force needs layout 1, 2 or 4");
            lanes = std::max(lanes, 64);
            unroll = 2;
        }
    }
    const bool repel = c->repel_kappa > 0.0;
    snk::NeighbourArgs nbargs{};
    if (repel) {
        if (lanes < 64) return fail(c, SNK_EINVAL, "repulsion needs lanes_per_contour >= 64");
        snk_status rs = neighbour_args(c, nbargs);
        if (rs != SNK_OK) return rs;
        a.snap = nbargs.snap;
        a.nb = nbargs.nb;
        a.nbn = nbargs.nbn;
        a.nb_cap = kNbCap;
        a.kappa = (float)c->repel_kappa;
    }
    if (snk::evolve_lds_bytes(c->P.dim, lanes, a.p.M, 0) > 65536)
        return fail(c, SNK_EINVAL, "n_rays too large for the evolve kernel's LDS (64 KiB per workgroup)");
    if (snk::evolve_lds_bytes(c->P.dim, lanes, a.p.M, a.tile_cap) > 65536)
        return fail(c, SNK_EINVAL, "LDS box too large (the evolve kernel's LDS is 64 KiB per workgroup)");
    if (standalone) {
        HIPTRY(c, hipMemsetAsync(c->d_counters, 0, sizeof(unsigned long long), c->stream));
        HIPTRY(c, hipEventRecord(c->ev[2], c->stream));
    }
    // A long evolve runs as two launches of half the iterations each: the second one starts only
    // the contours still active, spread over every CU, instead of leaving them on the CUs the
    // first launch gave them (the results are identical: every draw depends on the contour's id
    // and iteration only).
    int parts = (!trace && n_iter >= 64) ? 2 : 1;
    if (repel) {
        // the neighbours' snapshot and lists are rebuilt before every chunk of repel_every iterations
        parts = 0;
        const float rho = (float)rho_of(c->P.dim);
        for (int done = 0; done < n_iter; ++parts) {
            a.n_iter = std::min(c->repel_every, n_iter - done);
            done += a.n_iter;
            HIPTRY(c, snk::launch_neighbours(c->d_st, (int)c->n, geometry(c), c->P.dim, rho, nbargs, c->stream));
            HIPTRY(c, snk::launch_evolve(a, c->P.dim, lanes, unroll, layout, trace, c->stream));
        }
        parts = std::max(parts, 1);
    } else {
        for (int part = 0, done = 0; part < parts; ++part) {
            a.n_iter = (int)((int64_t)n_iter * (part + 1) / parts) - done;
            cull_points(done, a.n_iter);
            done += a.n_iter;
            HIPTRY(c, snk::launch_evolve(a, c->P.dim, lanes, unroll, layout, trace, c->stream));
        }
    }
    c->evolve_launches += parts - 1;
    c->last_lanes = lanes;
    c->last_unroll = exact ? 1 : unroll;
    c->last_layout = layout;
    c->last_tile = a.tile_cap;
    if (standalone) {
        HIPTRY(c, hipEventRecord(c->ev[3], c->stream));
        c->ev_evo = true;
    }
    c->evolve_launches += 1;
    if (repel && n_iter > 0) {
        int over = 0;
        HIPTRY(c, hipMemcpyAsync(&over, nbargs.overflow, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPTRY(c, hipStreamSynchronize(c->stream));
        if (over)
            return fail(c, SNK_ERANGE, "a contour overlapped more than 64 neighbours (repulsion lists truncated)");
    }
    return SNK_OK;
}

// The pinned staging buffer with room for n records, free to write (the last upload from it done).
snk_status stage(snk_ctx *c, size_t n, DevContour **out) {
    if (c->stage_busy) {
        HIPTRY(c, hipEventSynchronize(c->ev_stage));
        c->stage_busy = false;
    }
    if (c->stage_cap < n || !c->h_stage) {
        if (c->h_stage) HIPTRY(c, hipHostFree(c->h_stage));
        c->h_stage = nullptr;
        c->stage_cap = 0;
        void *q = nullptr;
        hipError_t e = hipHostMalloc(&q, std::max<size_t>(n, 1) * sizeof(DevContour), hipHostMallocDefault);
        if (e != hipSuccess) return fail(c, SNK_ENOMEM, std::string("hipHostMalloc: ") + hipGetErrorString(e));
        c->h_stage = static_cast<DevContour *>(q);
        c->stage_cap = n;
    }
    *out = c->h_stage;
    return SNK_OK;
}

// Uploads the first n staged records to the contour state without waiting for the copy: the
// stream orders it before every later launch, and the next use of the staging buffer waits for it.
snk_status upload_stage(snk_ctx *c, size_t n) {
    if (n == 0) return SNK_OK;
    HIPTRY(c, hipMemcpyAsync(c->d_st, c->h_stage, sizeof(DevContour) * n, hipMemcpyHostToDevice, c->stream));
    HIPTRY(c, hipEventRecord(c->ev_stage, c->stream));
    c->stage_busy = true;
    return SNK_OK;
}

snk_status unpack(snk_ctx *c, std::vector<DevContour> &h) {
    DevContour *buf = nullptr;
    snk_status st = stage(c, (size_t)c->n, &buf);
    if (st != SNK_OK) return st;
    if (c->n > 0)
        HIPTRY(c, hipMemcpyAsync(buf, c->d_st, sizeof(DevContour) * c->n, hipMemcpyDeviceToHost, c->stream));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    h.assign(buf, buf + c->n);
    return SNK_OK;
}

void centre_of(const snk_ctx *c, const DevContour &s, double *out) {
    for (int i = 0; i < 3; ++i)
        out[i] = i < c->P.dim ? ((double)s.anc[i] + (double)s.off[i]) * c->P.spacing[i] : 0.0;
}

// Exact energies and the final selection (mode 0), or a culling pass (mode 1) over every contour.
// noalloc: the selection scratch and counters come from the device's static scratch array (checked
// against its limits by the caller) and nothing is allocated.
snk_status run_select(snk_ctx *c, int mode, int grace, bool noalloc = false) {
    snk_status st = SNK_OK;
    snk::JobDev a{};
    a.p = job_params(c);
    a.st = c->d_st;
    a.e_vox = c->d_evox;
    a.n = (int)c->n;
    a.target = 0;
    a.e0 = (float)c->P.e0;
    int G3[3];
    double cell = 0.0;
    const int64_t G = snk_grid_for(c->P, c->nx, c->ny, c->nz, G3, &cell);
    for (int i = 0; i < 3; ++i) a.G[i] = G3[i];
    a.cell = (float)cell;
    a.mode = mode;
    a.grace = grace;
    a.e_cull = (float)(std::isnan(c->cull_thr) ? c->P.e0 : c->cull_thr);
    a.compete = c->cull_compete;
    if (noalloc) {
        if (c->n > kNoAllocMaxContours || G > kNoAllocMaxCells)
            return fail(c, SNK_EINVAL, "snk_finalize_noalloc: more than its maximum contours or grid cells");
        unsigned char *base = c->scratch;
        a.cell_start = reinterpret_cast<int *>(base + kNaCellStart);
        a.cell_fill = reinterpret_cast<int *>(base + kNaCellFill);
        a.items = reinterpret_cast<int *>(base + kNaItems);
        a.cell_of = reinterpret_cast<int *>(base + kNaCellOf);
        a.dec = reinterpret_cast<int *>(base + kNaDec);
        unsigned long long *counters = reinterpret_cast<unsigned long long *>(base + kNaCounters);
        a.kept = counters;
        // a fill kernel, not a memset node, so the call can also be captured in a graph
        HIPTRY(c, snk::launch_zero(counters, 4, c->stream));
        if (mode == 0) HIPTRY(c, snk::launch_energy_vox(a.p, a.st, a.e_vox, a.n, c->P.dim, true, c->stream));
        if (mode == 2) HIPTRY(c, snk::launch_mark_maxiter(a.st, a.n, c->stream));
        HIPTRY(c, snk::launch_select(a, c->P.dim, reinterpret_cast<int *>(counters + 2), c->stream));
        return SNK_OK;
    }
    st = ensure(c, &c->d_cell_start, &c->grid_cap, (size_t)G + 1);
    if (st != SNK_OK) return st;
    st = ensure(c, &c->d_cell_fill, &c->grid_fill_cap, (size_t)G + 1);
    if (st != SNK_OK) return st;
    if (c->sel_cap < (size_t)c->n) {
        for (int **p : {&c->d_items, &c->d_cell_of, &c->d_dec}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
        size_t k1 = 0, k2 = 0, k3 = 0;
        if ((st = ensure(c, &c->d_items, &k1, (size_t)c->n)) != SNK_OK) return st;
        if ((st = ensure(c, &c->d_cell_of, &k2, (size_t)c->n)) != SNK_OK) return st;
        if ((st = ensure(c, &c->d_dec, &k3, (size_t)c->n)) != SNK_OK) return st;
        c->sel_cap = (size_t)c->n;
    }
    a.cell_start = c->d_cell_start;
    a.cell_fill = c->d_cell_fill;
    a.items = c->d_items;
    a.cell_of = c->d_cell_of;
    a.dec = c->d_dec;
    a.kept = c->d_counters + 1;
    HIPTRY(c, hipMemsetAsync(c->d_counters + 1, 0, sizeof(unsigned long long), c->stream));
    // a culling pass ranks by the Monte-Carlo energy the last iteration left in the state
    if (mode == 0) HIPTRY(c, snk::launch_energy_vox(a.p, a.st, a.e_vox, a.n, c->P.dim, true, c->stream));
    if (mode == 2) HIPTRY(c, snk::launch_mark_maxiter(a.st, a.n, c->stream));
    HIPTRY(c, snk::launch_select(a, c->P.dim, reinterpret_cast<int *>(c->d_counters + 2), c->stream));
    return SNK_OK;
}

}  // namespace

extern "C" {

const char *snk_version(void) { return "snk 0.1 (gfx950)"; }

const char *snk_last_error(const snk_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

snk_status snk_create(snk_ctx **out, int device, void *hip_stream) {
    if (!out) return fail(nullptr, SNK_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return fail(nullptr, SNK_EDEVICE, "no HIP device available");
    if (device < 0 || device >= count) return fail(nullptr, SNK_EINVAL, "device index out of range");
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, SNK_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    snk_ctx *c = new (std::nothrow) snk_ctx();
    if (!c) return fail(nullptr, SNK_ENOMEM, "host allocation failed");
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) c->cus = 0;
    if (hipDeviceGetAttribute(&c->lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) !=
        hipSuccess)
        c->lds_per_cu = 0;
    for (auto &ev : c->ev) {
        e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            snk_destroy(c);
            return fail(nullptr, SNK_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
        }
    }
    e = hipEventCreateWithFlags(&c->ev_stage, hipEventDisableTiming);
    if (e != hipSuccess) {
        snk_destroy(c);
        return fail(nullptr, SNK_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
    }
    e = hipMalloc(&c->d_counters, 4 * sizeof(unsigned long long));
    if (e != hipSuccess) {
        snk_destroy(c);
        return fail(nullptr, SNK_ENOMEM, "hipMalloc counters");
    }
    e = scratch_address(device, &c->scratch);
    if (e != hipSuccess) {
        snk_destroy(c);
        return fail(nullptr, SNK_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    *out = c;
    return SNK_OK;
}

snk_status snk_destroy(snk_ctx *c) {
    if (!c) return SNK_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    void *bufs[] = {c->d_dirs, c->raw_owned, c->J, c->Jq, c->d_st, c->d_evox, c->d_trace, c->d_cell_start,
                    c->d_cell_fill, c->d_items, c->d_cell_of, c->d_dec, c->d_counters, c->d_anti, c->d_nb,
                    c->d_Rk, c->d_live, c->d_snap, c->d_nbgrid, c->d_nbitems, c->d_rnb};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    for (auto &ev : c->ev)
        if (ev) (void)hipEventDestroy(ev);
    if (c->ev_stage) (void)hipEventDestroy(c->ev_stage);
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    delete c;
    return SNK_OK;
}

snk_status snk_set_params(snk_ctx *c, const snk_params *p) {
    if (!c || !p) return fail(c, SNK_EINVAL, "NULL argument");
    snk_status st = check_params(c, *p);
    if (st != SNK_OK) return st;
    if (c->have_params && !same_prepass(c->P, *p)) c->J_dirty = true;
    if (c->have_volume && p->dim == 3 && (c->nx < 2 || c->ny < 2 || c->nz < 2))
        return fail(c, SNK_EINVAL, "dim 3 needs >= 2 voxels on every axis");
    c->P = *p;
    c->have_params = true;
    return SNK_OK;
}

snk_status snk_set_launch(snk_ctx *c, int32_t lanes_per_contour, int32_t pairs_in_flight, int32_t layout) {
    if (!c) return fail(c, SNK_EINVAL, "NULL context");
    if (lanes_per_contour != 0 && lanes_per_contour != 16 && lanes_per_contour != 32 && lanes_per_contour != 64 &&
        lanes_per_contour != 128 && lanes_per_contour != 256)
        return fail(c, SNK_EINVAL, "lanes_per_contour must be 0 (auto), 16, 32, 64, 128 or 256");
    if (pairs_in_flight < 0 || pairs_in_flight > 4 || pairs_in_flight == 3)
        return fail(c, SNK_EINVAL, "pairs_in_flight must be 0 (auto), 1, 2 or 4");
    if (layout < 0 || layout > 4)
        return fail(c, SNK_EINVAL,
                    "layout must be 0 (auto), 1 (plain), 2 (quad), 3 (plain, 64-bit addressing) or 4 (column pairs, 2D)");
    c->lanes = lanes_per_contour;
    c->unroll = pairs_in_flight;
    c->layout_req = layout;
    return SNK_OK;
}

snk_status snk_set_tile(snk_ctx *c, int32_t tile_voxels) {
    if (!c) return fail(c, SNK_EINVAL, "NULL context");
    if (tile_voxels < -1 || tile_voxels > 16384)
        return fail(c, SNK_EINVAL, "tile_voxels must be -1 (auto), 0 (off) or at most 16384");
    c->tile_req = tile_voxels;
    return SNK_OK;
}

snk_status snk_set_star(snk_ctx *c, double smooth) {
    if (!c) return fail(c, SNK_EINVAL, "NULL context");
    if (!isfinite(smooth)) return fail(c, SNK_EINVAL, "smooth must be finite");
    c->star_lambda = smooth < 0.0 ? -1.0 : smooth;
    return SNK_OK;
}

snk_status snk_get_star_radii(snk_ctx *c, float *radii, int64_t cap, int64_t *n_out) {
    if (!c || !radii) return fail(c, SNK_EINVAL, "NULL argument");
    snk_status st = need(c, true, true);
    if (st != SNK_OK) return st;
    const int64_t total = c->n * c->D;
    if (n_out) *n_out = total;
    if (cap < total) return fail(c, SNK_ERANGE, "capacity smaller than n x n_dirs");
    (void)hipSetDevice(c->device);
    st = star_radii(c);
    if (st != SNK_OK) return st;
    if (total > 0)
        HIPTRY(c, hipMemcpyAsync(radii, c->d_Rk, sizeof(float) * total, hipMemcpyDeviceToHost, c->stream));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    return SNK_OK;
}

snk_status snk_set_star_radii(snk_ctx *c, const float *radii, int64_t n) {
    if (!c || !radii) return fail(c, SNK_EINVAL, "NULL argument");
    snk_status st = need(c, true, true);
    if (st != SNK_OK) return st;
    if (n != c->n) return fail(c, SNK_EINVAL, "n must equal the number of seeded contours");
    const int64_t total = n * c->D;
    for (int64_t i = 0; i < total; ++i)
        if (!(radii[i] > 0.0f) || !(radii[i] <= (float)c->P.r_max))
            return fail(c, SNK_EINVAL, "star radius outside (0, r_max]");
    (void)hipSetDevice(c->device);
    st = ensure(c, &c->d_Rk, &c->Rk_cap, (size_t)std::max<int64_t>(total, 1));
    if (st != SNK_OK) return st;
    if (total > 0)
        HIPTRY(c, hipMemcpyAsync(c->d_Rk, radii, sizeof(float) * total, hipMemcpyHostToDevice, c->stream));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    c->Rk_valid = true;
    return SNK_OK;
}

snk_status snk_set_directions(snk_ctx *c, const float *dirs, int32_t D) {
    if (!c || !dirs || D <= 0) return fail(c, SNK_EINVAL, "bad direction table");
    snk_status st = need(c, false, false);
    if (st != SNK_OK) return st;
    const int dim = c->P.dim;
    if ((int64_t)D * dim > 12288) return fail(c, SNK_EINVAL, "direction table too large (D * dim > 12288)");
    for (int32_t k = 0; k < D; ++k) {
        double n2 = 0.0;
        for (int i = 0; i < dim; ++i) n2 += (double)dirs[k * dim + i] * dirs[k * dim + i];
        if (!(fabs(n2 - 1.0) < 1e-5)) return fail(c, SNK_EINVAL, "direction table rows must be unit vectors");
    }
    (void)hipSetDevice(c->device);
    st = ensure(c, &c->d_dirs, &c->dirs_cap, (size_t)D * dim);
    if (st != SNK_OK) return st;
    c->dirs_host.assign(dirs, dirs + (size_t)D * dim);
    c->Rk_valid = false;
    HIPTRY(c, hipMemcpyAsync(c->d_dirs, c->dirs_host.data(), sizeof(float) * D * dim, hipMemcpyHostToDevice,
                             c->stream));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    c->D = D;
    return SNK_OK;
}

snk_status snk_load_volume(snk_ctx *c, const void *data, snk_dtype dtype, int64_t nx, int64_t ny, int64_t nz,
                           int on_device) {
    if (!c || !data) return fail(c, SNK_EINVAL, "NULL argument");
    snk_status st = need(c, false, false);
    if (st != SNK_OK) return st;
    if (dtype != SNK_U8 && dtype != SNK_U16 && dtype != SNK_F32) return fail(c, SNK_EINVAL, "bad dtype");
    if (nx < 2 || ny < 2 || nz < 1) return fail(c, SNK_EINVAL, "volume needs nx, ny >= 2 and nz >= 1");
    if (c->P.dim == 3 && nz < 2) return fail(c, SNK_EINVAL, "dim 3 needs nz >= 2");
    if (c->P.dim == 2 && nz != 1) return fail(c, SNK_EINVAL, "dim 2 needs nz == 1");
    if (nx * ny * nz >= (int64_t)1 << 31) return fail(c, SNK_EINVAL, "volume too large (>= 2^31 voxels)");
    (void)hipSetDevice(c->device);
    const size_t vox = (size_t)(nx * ny * nz);
    const size_t esz = dtype == SNK_U8 ? 1 : (dtype == SNK_U16 ? 2 : 4);
    if (on_device) {
        c->raw = data;
    } else {
        st = ensure(c, reinterpret_cast<uint8_t **>(&c->raw_owned), &c->raw_owned_cap, vox * esz);
        if (st != SNK_OK) return st;
        HIPTRY(c, hipMemcpyAsync(c->raw_owned, data, vox * esz, hipMemcpyHostToDevice, c->stream));
        HIPTRY(c, hipStreamSynchronize(c->stream));
        c->raw = c->raw_owned;
    }
    st = ensure(c, &c->J, &c->J_cap, vox);
    if (st != SNK_OK) return st;
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->dtype = dtype;
    c->have_volume = true;
    c->J_dirty = true;
    c->n = 0;  // seeds refer to a volume
    return SNK_OK;
}

snk_status snk_prepass(snk_ctx *c) {
    if (!c) return fail(c, SNK_EINVAL, "NULL context");
    snk_status st = need(c, true, false);
    if (st != SNK_OK) return st;
    (void)hipSetDevice(c->device);
    return run_prepass(c);
}

snk_status snk_load_seeds(snk_ctx *c, const double *centers, const float *r0, const uint32_t *ids, int64_t n) {
    if (!c || (n > 0 && !centers) || n < 0) return fail(c, SNK_EINVAL, "bad seed arguments");
    snk_status st = need(c, true, false);
    if (st != SNK_OK) return st;
    if (n >= (int64_t)1 << 31) return fail(c, SNK_EINVAL, "too many seeds");
    (void)hipSetDevice(c->device);
    DevContour *h = nullptr;
    st = stage(c, (size_t)n, &h);
    if (st != SNK_OK) return st;
    const double lo = r_low(c->P), hi = c->P.r_max;
    for (int64_t i = 0; i < n; ++i) {
        DevContour &s = h[i];
        memset(&s, 0, sizeof(s));
        to_anchor(c, &centers[i * 3], s);
        double R = r0 ? (double)r0[i] : c->P.r_init;
        if (!isfinite(R)) return fail(c, SNK_EINVAL, "initial radius not finite");
        R = std::min(std::max(R, lo), hi);
        s.R = (float)R;
        s.e_mc = 0.0f;
        s.e_vox = 0.0f;
        s.iters = 0;
        s.id = ids ? ids[i] : (uint32_t)i;
        s.status = inside(c, s) ? SNK_ACTIVE : SNK_OUT;
        s.streak = 0;
        s.keep = 0;
    }
    st = ensure(c, &c->d_st, &c->n_cap, (size_t)n);
    if (st != SNK_OK) return st;
    st = ensure(c, &c->d_evox, &c->evox_cap, (size_t)n);
    if (st != SNK_OK) return st;
    st = upload_stage(c, (size_t)n);
    if (st != SNK_OK) return st;
    c->n = n;
    c->Rk_valid = false;
    return SNK_OK;
}

snk_status snk_evolve(snk_ctx *c, int32_t n_iter) {
    if (!c) return fail(c, SNK_EINVAL, "NULL context");
    if (n_iter < 0) return fail(c, SNK_EINVAL, "n_iter must be >= 0");
    snk_status st = need(c, true, false);
    if (st != SNK_OK) return st;
    if (c->n == 0 || n_iter == 0) return SNK_OK;
    (void)hipSetDevice(c->device);
    return run_evolve(c, n_iter, false);
}

snk_status snk_trace_step(snk_ctx *c, float *terms) {
    if (!c || !terms) return fail(c, SNK_EINVAL, "NULL argument");
    snk_status st = need(c, true, true);
    if (st != SNK_OK) return st;
    (void)hipSetDevice(c->device);
    st = ensure(c, &c->d_trace, &c->trace_cap, (size_t)c->n * SNK_TRACE_W);
    if (st != SNK_OK) return st;
    HIPTRY(c, hipMemsetAsync(c->d_trace, 0, sizeof(float) * c->n * SNK_TRACE_W, c->stream));
    st = run_evolve(c, 1, true);
    if (st != SNK_OK) return st;
    HIPTRY(c, hipMemcpyAsync(terms, c->d_trace, sizeof(float) * c->n * SNK_TRACE_W, hipMemcpyDeviceToHost,
                             c->stream));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    return SNK_OK;
}

snk_status snk_finalize(snk_ctx *c) {
    if (!c) return fail(c, SNK_EINVAL, "NULL context");
    snk_status st = need(c, true, false);
    if (st != SNK_OK) return st;
    if (c->n == 0) return SNK_OK;
    (void)hipSetDevice(c->device);
    if (c->J_dirty) {
        st = run_prepass(c);
        if (st != SNK_OK) return st;
    }
    HIPTRY(c, hipEventRecord(c->ev[4], c->stream));
    // star contours rank by their last Monte-Carlo energy (no exact star energy is formed)
    st = run_select(c, c->star_lambda >= 0.0 ? 2 : 0, 0);
    if (st != SNK_OK) return st;
    HIPTRY(c, hipEventRecord(c->ev[5], c->stream));
    c->ev_fin = true;
    return SNK_OK;
}

snk_status snk_finalize_noalloc(snk_ctx *c) {
    if (!c) return fail(c, SNK_EINVAL, "NULL context");
    snk_status st = need(c, true, false);
    if (st != SNK_OK) return st;
    if (c->n == 0) return SNK_OK;
    if (c->J_dirty) return fail(c, SNK_ESTATE, "snk_finalize_noalloc: the pre-pass has not run (snk_prepass or snk_evolve first)");
    if (!c->scratch) return fail(c, SNK_ESTATE, "snk_finalize_noalloc: no scratch address for this device");
    (void)hipSetDevice(c->device);
    HIPTRY(c, hipEventRecord(c->ev[4], c->stream));
    st = run_select(c, c->star_lambda >= 0.0 ? 2 : 0, 0, true);
    if (st != SNK_OK) return st;
    HIPTRY(c, hipEventRecord(c->ev[5], c->stream));
    c->ev_fin = true;
    return SNK_OK;
}

snk_status snk_seed_lattice(snk_ctx *c, double pitch, int64_t *n_out) {
    if (!c) return fail(c, SNK_EINVAL, "NULL context");
    snk_status st = need(c, true, false);
    if (st != SNK_OK) return st;
    if (!(pitch > 0.0)) pitch = sqrt(1.5) * c->P.r_init;
    if (!(pitch > 0.0) || !isfinite(pitch)) return fail(c, SNK_EINVAL, "lattice pitch must be > 0 (or r_init > 0)");
    const int64_t nn[3] = {c->nx, c->ny, c->nz};
    int64_t k[3] = {1, 1, 1};
    double o[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < c->P.dim; ++a) {
        const double ext = (double)(nn[a] - 1) * c->P.spacing[a];
        k[a] = std::max<int64_t>(1, (int64_t)floor(ext / pitch));
        o[a] = 0.5 * (ext - (double)(k[a] - 1) * pitch);
    }
    const int64_t n = k[0] * k[1] * k[2];
    if (n >= ((int64_t)1 << 31)) return fail(c, SNK_EINVAL, "lattice too fine (>= 2^31 contours)");
    std::vector<double> cen((size_t)n * 3);
    int64_t m = 0;
    for (int64_t iz = 0; iz < k[2]; ++iz)
        for (int64_t iy = 0; iy < k[1]; ++iy)
            for (int64_t ix = 0; ix < k[0]; ++ix, ++m) {
                cen[m * 3 + 0] = o[0] + (double)ix * pitch;
                cen[m * 3 + 1] = o[1] + (double)iy * pitch;
                cen[m * 3 + 2] = c->P.dim == 3 ? o[2] + (double)iz * pitch : 0.0;
            }
    if (n_out) *n_out = n;
    return snk_load_seeds(c, cen.data(), nullptr, nullptr, n);
}

snk_status snk_set_repulsion(snk_ctx *c, double kappa, int32_t every) {
    if (!c) return fail(c, SNK_EINVAL, "NULL context");
    if (!(kappa >= 0.0) || !isfinite(kappa) || every < 1)
        return fail(c, SNK_EINVAL, "kappa must be finite and >= 0, every >= 1");
    c->repel_kappa = kappa;
    c->repel_every = every;
    return SNK_OK;
}

snk_status snk_set_cull(snk_ctx *c, double e_cull, int32_t compete) {
    if (!c) return fail(c, SNK_EINVAL, "NULL context");
    if (isinf(e_cull) || (compete != 0 && compete != 1))
        return fail(c, SNK_EINVAL, "e_cull must be finite (NaN: params.e0) and compete 0 or 1");
    c->cull_thr = e_cull;
    c->cull_compete = compete;
    return SNK_OK;
}

snk_status snk_evolve_cull(snk_ctx *c, int32_t n_iter, int32_t cull_every, int32_t grace_iters) {
    if (!c) return fail(c, SNK_EINVAL, "NULL context");
    if (n_iter < 0 || grace_iters < 0 || (n_iter > 0 && cull_every <= 0))
        return fail(c, SNK_EINVAL, "n_iter >= 0, cull_every > 0 and grace_iters >= 0 required");
    snk_status st = need(c, true, false);
    if (st != SNK_OK) return st;
    if (c->n == 0) return SNK_OK;
    (void)hipSetDevice(c->device);
    if (c->J_dirty) {
        st = run_prepass(c);
        if (st != SNK_OK) return st;
    }
    // after each pass the next chunk launches only the contours still active (sphere contours; star
    // contours run every slot), so the dwindling population is not spread over slots that only exit
    const bool compact = c->star_lambda < 0.0;
    if (compact) {
        st = ensure(c, &c->d_live, &c->live_cap, (size_t)c->n + 1);
        if (st != SNK_OK) return st;
    }
    HIPTRY(c, hipMemsetAsync(c->d_counters, 0, sizeof(unsigned long long), c->stream));
    HIPTRY(c, hipEventRecord(c->ev[2], c->stream));
    if (!c->cull_compete && compact && c->repel_kappa <= 0.0 && n_iter > 0) {
        // without competition a pass judges each contour alone, so one evolution applies the
        // passes between its chunks itself (an active contour above the threshold at a pass point
        // retires at once and its workgroup slot goes to the next contour) and one pass at the end
        // judges the rest: the same outcome as chunks and passes, with no relaunches
        c->cull_in_every = cull_every;
        c->cull_in_grace = grace_iters;
        c->cull_in_end = n_iter;
        st = run_evolve(c, n_iter, false, false);
        c->cull_in_every = 0;
        if (st != SNK_OK) return st;
        st = run_select(c, 1, n_iter < grace_iters ? INT32_MAX : 0);
        if (st != SNK_OK) return st;
        HIPTRY(c, hipEventRecord(c->ev[3], c->stream));
        c->ev_evo = true;
        return SNK_OK;
    }
    int32_t done = 0;
    int live = -1;   // active contours after the last pass (-1: every contour, before the first)
    do {
        const int32_t k = std::min(cull_every > 0 ? cull_every : 0, n_iter - done);
        if (k > 0 && live != 0) {
            st = live < 0 ? run_evolve(c, k, false, false) : run_evolve(c, k, false, false, c->d_live, live);
            if (st != SNK_OK) return st;
        }
        // the grace period counts the iterations of this call: until it ends every live contour
        // competes (the pass's age test is passed for all of them), afterwards none is young
        done += k;
        st = run_select(c, 1, done < grace_iters ? INT32_MAX : 0);
        if (st != SNK_OK) return st;
        if (compact && done < n_iter) {
            int *count = c->d_live + c->n;
            HIPTRY(c, hipMemsetAsync(count, 0, sizeof(int), c->stream));
            HIPTRY(c, snk::launch_compact_active(c->d_st, (int)c->n, c->d_live, count, c->stream));
            HIPTRY(c, hipMemcpyAsync(&live, count, sizeof(int), hipMemcpyDeviceToHost, c->stream));
            HIPTRY(c, hipStreamSynchronize(c->stream));
        }
    } while (done < n_iter);
    HIPTRY(c, hipEventRecord(c->ev[3], c->stream));
    c->ev_evo = true;
    return SNK_OK;
}

snk_status snk_read(snk_ctx *c, float *radii, double *centers, float *e_mc, float *e_vox, int32_t *iters,
                    uint8_t *status, uint8_t *keep, int64_t cap, int64_t *n_out) {
    if (!c) return fail(c, SNK_EINVAL, "NULL context");
    if (n_out) *n_out = c->n;
    if (cap < c->n) return fail(c, SNK_ERANGE, "capacity smaller than the number of contours");
    (void)hipSetDevice(c->device);
    std::vector<DevContour> h;
    snk_status st = unpack(c, h);
    if (st != SNK_OK) return st;
    for (int64_t i = 0; i < c->n; ++i) {
        const DevContour &s = h[i];
        if (radii) radii[i] = s.R;
        if (centers) centre_of(c, s, &centers[i * 3]);
        if (e_mc) e_mc[i] = s.e_mc;
        if (e_vox) e_vox[i] = c->star_lambda >= 0.0 ? s.e_mc : s.e_vox;
        if (iters) iters[i] = s.iters;
        if (status) status[i] = s.status;
        if (keep) keep[i] = s.keep;
    }
    return SNK_OK;
}

snk_status snk_get_state(snk_ctx *c, double *centers, float *radii, int32_t *iters, uint8_t *status,
                         uint8_t *streak, int64_t cap, int64_t *n_out) {
    if (!c) return fail(c, SNK_EINVAL, "NULL context");
    if (n_out) *n_out = c->n;
    if (cap < c->n) return fail(c, SNK_ERANGE, "capacity smaller than the number of contours");
    (void)hipSetDevice(c->device);
    std::vector<DevContour> h;
    snk_status st = unpack(c, h);
    if (st != SNK_OK) return st;
    for (int64_t i = 0; i < c->n; ++i) {
        if (centers) centre_of(c, h[i], &centers[i * 3]);
        if (radii) radii[i] = h[i].R;
        if (iters) iters[i] = h[i].iters;
        if (status) status[i] = h[i].status;
        if (streak) streak[i] = h[i].streak;
    }
    return SNK_OK;
}

snk_status snk_set_state(snk_ctx *c, const double *centers, const float *radii, const int32_t *iters,
                         const uint8_t *status, const uint8_t *streak, int64_t n) {
    if (!c || !centers || !radii || !iters || !status) return fail(c, SNK_EINVAL, "NULL argument");
    snk_status st = need(c, true, true);
    if (st != SNK_OK) return st;
    if (n != c->n) return fail(c, SNK_EINVAL, "n must equal the number of seeded contours");
    (void)hipSetDevice(c->device);
    std::vector<DevContour> h;
    st = unpack(c, h);
    if (st != SNK_OK) return st;
    for (int64_t i = 0; i < n; ++i) {
        if (!(radii[i] > 0.0f) || !(radii[i] <= (float)c->P.r_max) || iters[i] < 0)
            return fail(c, SNK_EINVAL, "state radius outside (0, r_max] or negative iteration count");
        if ((status[i] & 0x0f) > SNK_CULLED) return fail(c, SNK_EINVAL, "bad status value");
        to_anchor(c, &centers[i * 3], h[i]);
        h[i].R = radii[i];
        h[i].iters = iters[i];
        h[i].status = status[i];
        h[i].streak = streak ? streak[i] : 0;
        h[i].keep = 0;
    }
    DevContour *buf = nullptr;
    st = stage(c, (size_t)n, &buf);
    if (st != SNK_OK) return st;
    if (n > 0) memcpy(buf, h.data(), sizeof(DevContour) * n);
    st = upload_stage(c, (size_t)n);
    if (st != SNK_OK) return st;
    c->Rk_valid = false;
    return SNK_OK;
}

snk_status snk_read_volume(snk_ctx *c, float *out, int on_device) {
    if (!c || !out) return fail(c, SNK_EINVAL, "NULL argument");
    snk_status st = need(c, true, false);
    if (st != SNK_OK) return st;
    (void)hipSetDevice(c->device);
    if (c->J_dirty) {
        st = run_prepass(c);
        if (st != SNK_OK) return st;
    }
    const size_t bytes = sizeof(float) * (size_t)(c->nx * c->ny * c->nz);
    HIPTRY(c, hipMemcpyAsync(out, c->J, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             c->stream));
    if (!on_device) HIPTRY(c, hipStreamSynchronize(c->stream));
    return SNK_OK;
}

snk_status snk_get_timing(snk_ctx *c, snk_timing *t) {
    if (!c || !t) return fail(c, SNK_EINVAL, "NULL argument");
    (void)hipSetDevice(c->device);
    HIPTRY(c, hipStreamSynchronize(c->stream));
    float ms = 0.0f;
    t->prepass_ms = t->evolve_ms = t->finalize_ms = 0.0;
    if (c->ev_pre) {
        HIPTRY(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        t->prepass_ms = ms;
    }
    if (c->ev_evo) {
        HIPTRY(c, hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
        t->evolve_ms = ms;
    }
    if (c->ev_fin) {
        HIPTRY(c, hipEventElapsedTime(&ms, c->ev[4], c->ev[5]));
        t->finalize_ms = ms;
    }
    unsigned long long cnt = 0;
    HIPTRY(c, hipMemcpy(&cnt, c->d_counters, sizeof(cnt), hipMemcpyDeviceToHost));
    t->evolved = (int64_t)cnt;
    t->evolve_launches = c->evolve_launches;
    t->lanes_per_contour = c->last_lanes;
    t->pairs_in_flight = c->last_unroll;
    t->layout = c->last_layout;
    t->tile_voxels = c->last_tile;
    return SNK_OK;
}

snk_status snk_sync(snk_ctx *c) {
    if (!c) return fail(c, SNK_EINVAL, "NULL context");
    (void)hipSetDevice(c->device);
    HIPTRY(c, hipStreamSynchronize(c->stream));
    return SNK_OK;
}

}  // extern "C"
