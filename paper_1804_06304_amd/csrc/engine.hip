// Host side of the batch / serving engine (snk_engine_* in include/snk.h).
//
// Jobs (one volume + its seeds + parameters) are queued by snk_engine_submit and admitted in FIFO
// order while their device footprint fits the HBM budget. Admitted jobs live in a device job table
// (JobDev); the kernels walk a device list of (job, contour) items, so one launch serves contours of
// many volumes of uneven size and contour count.
//
//  - snk_engine_run (batched): every admitted job is evolved from its seeds to its iteration target
//    and finalised in one captured hipGraph: state reset -> pre-pass per volume -> one evolve launch
//    per launch class (dim, D, M, L) -> exact energy over all items -> selection, one workgroup per
//    job. The graph is replayed while the job set is unchanged. The launch shape of each class
//    (lanes per contour, pair-points in flight, persistent work queue or one workgroup per item) is
//    picked once by timing short trials of every candidate. Every job keeps its volume in column
//    pairs (or quad records, on request) next to the FP32 one; launches read that copy unless the
//    plain layout is forced.
//  - snk_engine_step (served): continuous batching. Newly admitted jobs get their pre-pass and join
//    the running set; every running contour advances by at most `chunk` iterations in one launch
//    per class; jobs whose contours have all stopped are finalised, copied to the host and their
//    device memory returned to the budget. A contour's result does not depend on the mix it runs
//    in: its samples are keyed by (seed, id, iteration) and its sums are reduced in a fixed order.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "snk_internal.h"

using snk::DevContour;
using snk::JobDev;

namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

enum JobState { PENDING, RUNNING, DONE };

struct EJob {
    uint64_t id = 0;
    snk_params P{};
    int64_t nx = 0, ny = 0, nz = 0;
    snk_dtype dtype = SNK_U8;
    size_t raw_bytes = 0;
    std::vector<uint8_t> host_raw;       // copy of a host volume until admission
    const void *borrowed = nullptr;      // device volume passed with on_device = 1
    std::vector<float> dirs;             // D x dim
    std::vector<DevContour> init;        // initial contour states
    int n = 0;
    int n_iter = 0;
    size_t bytes = 0;                    // device footprint (admission estimate)
    size_t charged = 0;                  // capacity of the block it holds, charged to the budget
    JobState state = PENDING;
    int slot = -1;                       // row in the device job table
    // device buffers (one allocation)
    void *block = nullptr;
    const void *d_raw = nullptr;
    float *d_J = nullptr;
    float4 *d_Jq = nullptr;
    float *d_dirs = nullptr;
    DevContour *d_st = nullptr, *d_init = nullptr;
    double *d_evox = nullptr;
    int *d_sel = nullptr;
    int G[3] = {1, 1, 1};
    double cell = 1.0;
    int64_t grid_cells = 1;
    bool prepared = false;               // pre-pass done (served mode)
    std::vector<DevContour> result;
    double t_submit = 0, t_done = 0;
};

struct ClassKey {
    int dim, D, M, L;
    bool operator<(const ClassKey &o) const { return std::tie(dim, D, M, L) < std::tie(o.dim, o.D, o.M, o.L); }
};

struct Launch {
    int lanes = 256, unroll = 1, persistent = 1;
    int grid = 1;       // workgroups of a persistent launch
    int tile = 0;       // LDS box per workgroup, voxels (0: none)
    int per_cu = 0;     // persistent: workgroups per CU (0: as many as registers and LDS allow)
    float trial_ms = 0.0f;  // autotuned: time of the winning trial
    int trials = 0;         // autotuned: shapes timed
};

constexpr int kMaxClasses = 64;            // launch classes per run (one queue head each)
constexpr int kQueueWords = kMaxClasses / 2;  // queue heads are ints, zeroed as 64-bit words

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

double rho_of(int dim) { return dim == 3 ? pow(2.0, -1.0 / 3.0) : sqrt(0.5); }

double r_low(const snk_params &p) {
    const double rho = rho_of(p.dim);
    return std::max(p.r_min, p.dR * (1.0 + rho) / (2.0 * (1.0 - rho)));
}

}  // namespace

struct snk_engine {
    int device = 0;
    hipStream_t stream = nullptr;
    uint64_t budget = 0, in_use = 0;       // in_use: capacity of the blocks held by admitted jobs
    std::multimap<size_t, void *> pool;    // blocks of released jobs, reused before allocating
    uint64_t pooled = 0;
    std::vector<EJob *> staged;            // admitted jobs whose host copies are freed at the next sync
    std::string err;
    uint64_t next_id = 1;
    std::map<uint64_t, EJob *> jobs;     // every job not yet released
    std::deque<uint64_t> pending;        // FIFO of PENDING jobs
    std::vector<uint64_t> done_unpolled;
    int cus = 256;

    // device job table
    JobDev *d_jobs = nullptr;
    DevContour **d_init_ptrs = nullptr;
    int table_cap = 0;
    std::vector<int> free_slots;
    std::vector<JobDev> h_jobs;
    std::vector<DevContour *> h_init_ptrs;

    // item lists and per-launch scratch
    int2 *d_items = nullptr;
    size_t items_cap = 0;
    int *d_joblist = nullptr;
    size_t joblist_cap = 0;
    int *d_unfinished = nullptr;
    unsigned long long *d_counters = nullptr;  // [0] evolved, [1..] queue heads (as int) / kept
    int *d_queues = nullptr;                   // one queue head per launch class
    hipStream_t own_stream = nullptr;          // created when the caller passes the null stream
    int dim = 0;                               // every job of an engine has the same dimension

    // launch shapes
    Launch forced;
    bool force = false;
    int layout = snk::kBufferPair;             // volume layout of every evolve launch
    std::map<ClassKey, Launch> tuned;

    // captured batched run
    hipGraphExec_t graph = nullptr;
    std::vector<uint64_t> graph_jobs;
    int graph_replays = 0;

    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
    double last_ms = 0, last_evolve_ms = 0;
    int64_t last_evolved = 0;
    int64_t submitted = 0, admitted = 0, completed = 0;
    Launch last_launch;
};

namespace {

void unstage(snk_engine *e);

snk_status efail(snk_engine *e, snk_status code, const std::string &m) {
    if (e) e->err = m;
    return code;
}

#define EHIP(e, call)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return efail((e), SNK_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
snk_status grow(snk_engine *e, T **p, size_t *cap, size_t count) {
    if (*p && *cap >= count) return SNK_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    const size_t c = std::max<size_t>(count, 16) * 2;
    if (hipMalloc(p, c * sizeof(T)) != hipSuccess) return efail(e, SNK_ENOMEM, "hipMalloc (engine scratch)");
    *cap = c;
    return SNK_OK;
}

void drop_graph(snk_engine *e) {
    if (e->graph) (void)hipGraphExecDestroy(e->graph);
    e->graph = nullptr;
    e->graph_jobs.clear();
}

snk_status ensure_table(snk_engine *e, int need) {
    if (need <= e->table_cap) return SNK_OK;
    int cap = std::max(64, e->table_cap * 2);
    while (cap < need) cap *= 2;
    JobDev *nj = nullptr;
    DevContour **np = nullptr;
    int *nu = nullptr;
    if (hipMalloc(&nj, sizeof(JobDev) * cap) != hipSuccess || hipMalloc(&np, sizeof(DevContour *) * cap) != hipSuccess ||
        hipMalloc(&nu, sizeof(int) * cap) != hipSuccess)
        return efail(e, SNK_ENOMEM, "hipMalloc (job table)");
    if (e->d_jobs) (void)hipFree(e->d_jobs);
    if (e->d_init_ptrs) (void)hipFree(e->d_init_ptrs);
    if (e->d_unfinished) (void)hipFree(e->d_unfinished);
    e->d_jobs = nj;
    e->d_init_ptrs = np;
    e->d_unfinished = nu;
    for (int s = e->table_cap; s < cap; ++s) e->free_slots.push_back(s);
    std::sort(e->free_slots.begin(), e->free_slots.end(), std::greater<int>());
    e->h_jobs.resize(cap);
    e->h_init_ptrs.resize(cap, nullptr);
    e->table_cap = cap;
    drop_graph(e);
    EHIP(e, hipMemcpyAsync(e->d_jobs, e->h_jobs.data(), sizeof(JobDev) * cap, hipMemcpyHostToDevice, e->stream));
    EHIP(e, hipMemcpyAsync(e->d_init_ptrs, e->h_init_ptrs.data(), sizeof(DevContour *) * cap, hipMemcpyHostToDevice,
                           e->stream));
    EHIP(e, hipStreamSynchronize(e->stream));
    unstage(e);
    return SNK_OK;
}

size_t footprint(const EJob &j, int64_t grid_cells) {
    const size_t vox = (size_t)(j.nx * j.ny * j.nz);
    size_t b = 0;
    if (!j.borrowed) b += align256(j.raw_bytes);
    b += align256(vox * 4);                                    // J
    b += align256(vox * 16);                                   // quad copy of J
    b += align256(j.dirs.size() * 4);
    b += 2 * align256((size_t)std::max(j.n, 1) * sizeof(DevContour));
    b += align256((size_t)std::max(j.n, 1) * 8);               // e_vox
    b += align256(((size_t)grid_cells + 1) * 2 * 4 + (size_t)std::max(j.n, 1) * 3 * 4);   // selection
    return b;
}

snk::JobParams params_of(const EJob &j) {
    snk::JobParams p{};
    p.g.J = j.d_J;
    p.g.Jq = j.d_Jq;
    p.g.nx = (int)j.nx;
    p.g.ny = (int)j.ny;
    p.g.nz = (int)j.nz;
    for (int i = 0; i < 3; ++i) {
        p.g.h[i] = (float)j.P.spacing[i];
        p.g.inv_h[i] = (float)(1.0 / j.P.spacing[i]);
    }
    p.dirs = j.d_dirs;
    p.D = (int)(j.dirs.size() / j.P.dim);
    p.M = j.P.n_rays;
    p.L = j.P.n_radial;
    p.key0 = (uint32_t)(j.P.seed & 0xffffffffu);
    p.key1 = (uint32_t)(j.P.seed >> 32);
    p.flags = j.P.flags;
    p.dR = (float)j.P.dR;
    p.eps0 = (float)j.P.eps0;
    p.r_lo = (float)r_low(j.P);
    p.r_hi = (float)j.P.r_max;
    p.conv_tol = (float)j.P.conv_tol;
    p.conv_window = j.P.conv_window;
    p.in_slope = (float)(2.0 / (rho_of(j.P.dim) * j.P.dR));
    p.out_slope = (float)(1.0 / j.P.dR);
    return p;
}

// A device block of at least `need` bytes for a job: a pooled block up to 25% larger when the budget
// allows, else a new allocation (pooled blocks are freed first while budget or device memory run
// short). Pooled and admitted blocks together stay within the budget.
void *pool_get(snk_engine *e, size_t need, size_t *cap) {
    auto it = e->pool.lower_bound(need);
    if (it != e->pool.end() && it->first <= need + need / 4 && e->in_use + it->first <= e->budget) {
        void *b = it->second;
        *cap = it->first;
        e->pooled -= it->first;
        e->pool.erase(it);
        return b;
    }
    while (!e->pool.empty() && e->in_use + e->pooled + need > e->budget) {
        auto big = std::prev(e->pool.end());
        (void)hipFree(big->second);
        e->pooled -= big->first;
        e->pool.erase(big);
    }
    void *b = nullptr;
    while (hipMalloc(&b, need) != hipSuccess) {
        (void)hipGetLastError();
        if (e->pool.empty()) return nullptr;
        auto big = std::prev(e->pool.end());
        (void)hipFree(big->second);
        e->pooled -= big->first;
        e->pool.erase(big);
    }
    *cap = need;
    return b;
}

void pool_put(snk_engine *e, void *b, size_t cap) {
    e->pool.insert({cap, b});
    e->pooled += cap;
}

void pool_drain(snk_engine *e) {
    for (auto &kv : e->pool) (void)hipFree(kv.second);
    e->pool.clear();
    e->pooled = 0;
}

// Allocate, upload and enter a job into the device table (asynchronously: its host copies stay
// alive until the next synchronisation of the engine's stream).
snk_status admit(snk_engine *e, EJob &j) {
    snk_status st = ensure_table(e, (int)(e->jobs.size() + 1));
    if (st != SNK_OK) return st;
    if (e->free_slots.empty()) return efail(e, SNK_ENOMEM, "job table full");
    const size_t vox = (size_t)(j.nx * j.ny * j.nz);
    const size_t n = (size_t)std::max(j.n, 1);
    size_t off = 0;
    const size_t o_raw = off; if (!j.borrowed) off += align256(j.raw_bytes);
    const size_t o_J = off; off += align256(vox * 4);
    const size_t o_Jq = off; off += align256(vox * 16);
    const size_t o_dirs = off; off += align256(j.dirs.size() * 4);
    const size_t o_st = off; off += align256(n * sizeof(DevContour));
    const size_t o_init = off; off += align256(n * sizeof(DevContour));
    const size_t o_evox = off; off += align256(n * 8);
    const size_t o_sel = off; off += align256(((size_t)j.grid_cells + 1) * 2 * 4 + n * 3 * 4);
    size_t cap = 0;
    j.block = pool_get(e, off, &cap);
    if (!j.block) {
        size_t free_b = 0, total_b = 0;
        (void)hipMemGetInfo(&free_b, &total_b);
        return efail(e, SNK_ENOMEM,
                     "hipMalloc (job buffers): " + std::to_string(off) + " bytes requested, " +
                         std::to_string(e->in_use) + " charged to the budget, " + std::to_string(free_b) +
                         " of " + std::to_string(total_b) + " bytes free on the device");
    }
    char *b = static_cast<char *>(j.block);
    j.d_raw = j.borrowed ? j.borrowed : (const void *)(b + o_raw);
    j.d_J = reinterpret_cast<float *>(b + o_J);
    j.d_Jq = reinterpret_cast<float4 *>(b + o_Jq);
    j.d_dirs = reinterpret_cast<float *>(b + o_dirs);
    j.d_st = reinterpret_cast<DevContour *>(b + o_st);
    j.d_init = reinterpret_cast<DevContour *>(b + o_init);
    j.d_evox = reinterpret_cast<double *>(b + o_evox);
    j.d_sel = reinterpret_cast<int *>(b + o_sel);
    if (!j.borrowed)
        EHIP(e, hipMemcpyAsync(b + o_raw, j.host_raw.data(), j.raw_bytes, hipMemcpyHostToDevice, e->stream));
    EHIP(e, hipMemcpyAsync(j.d_dirs, j.dirs.data(), j.dirs.size() * 4, hipMemcpyHostToDevice, e->stream));
    if (j.n > 0) {
        EHIP(e, hipMemcpyAsync(j.d_init, j.init.data(), sizeof(DevContour) * j.n, hipMemcpyHostToDevice, e->stream));
        EHIP(e, hipMemcpyAsync(j.d_st, j.init.data(), sizeof(DevContour) * j.n, hipMemcpyHostToDevice, e->stream));
    }
    j.slot = e->free_slots.back();
    e->free_slots.pop_back();
    JobDev d{};
    d.p = params_of(j);
    d.st = j.d_st;
    d.e_vox = j.d_evox;
    d.n = j.n;
    d.target = j.n_iter;
    d.e0 = (float)j.P.e0;
    d.e_cull = d.e0;
    d.compete = 1;
    const size_t G1 = (size_t)j.grid_cells + 1;
    d.cell_start = j.d_sel;
    d.cell_fill = j.d_sel + G1;
    d.items = j.d_sel + 2 * G1;
    d.cell_of = d.items + n;
    d.dec = d.cell_of + n;
    for (int i = 0; i < 3; ++i) d.G[i] = j.G[i];
    d.cell = (float)j.cell;
    d.kept = e->d_counters + 1;
    e->h_jobs[j.slot] = d;
    e->h_init_ptrs[j.slot] = j.d_init;
    EHIP(e, hipMemcpyAsync(e->d_jobs + j.slot, &e->h_jobs[j.slot], sizeof(JobDev), hipMemcpyHostToDevice, e->stream));
    EHIP(e, hipMemcpyAsync(e->d_init_ptrs + j.slot, &e->h_init_ptrs[j.slot], sizeof(DevContour *),
                           hipMemcpyHostToDevice, e->stream));
    e->staged.push_back(&j);
    j.state = RUNNING;
    j.charged = cap;
    e->in_use += cap;
    e->admitted += 1;
    return SNK_OK;
}

// After a synchronisation of the engine's stream: drop the host copies of uploaded volumes.
void unstage(snk_engine *e) {
    for (EJob *j : e->staged) {
        j->host_raw.clear();
        j->host_raw.shrink_to_fit();
    }
    e->staged.clear();
}

// Returns a job's device memory and table row; idempotent (a finished job is released when it
// completes and again when the caller releases it), so the budget is credited exactly once.
void release_device(snk_engine *e, EJob &j) {
    if (j.block) {
        pool_put(e, j.block, j.charged);
        j.block = nullptr;
        e->in_use = e->in_use >= j.charged ? e->in_use - j.charged : 0;
    }
    if (j.slot >= 0) {
        e->free_slots.push_back(j.slot);
        j.slot = -1;
    }
}

// Admit pending jobs in FIFO order while they fit.
snk_status admit_pending(snk_engine *e, std::vector<EJob *> &newly) {
    while (!e->pending.empty()) {
        EJob *j = e->jobs[e->pending.front()];
        if (e->in_use + j->bytes > e->budget) break;  // pooled blocks are evicted as needed
        snk_status st = admit(e, *j);
        if (st != SNK_OK) return st;
        newly.push_back(j);
        e->pending.pop_front();
    }
    return SNK_OK;
}

snk_status prepass_job(snk_engine *e, const EJob &j) {
    snk::PrepassArgs a{};
    a.raw = j.d_raw;
    a.dtype = (int)j.dtype;
    a.J = j.d_J;
    // column pairs (8 bytes per voxel) or quad records in the same buffer
    if (e->layout == snk::kBufferPair) a.Jp = reinterpret_cast<float2 *>(j.d_Jq);
    else a.Jq = j.d_Jq;
    a.nx = (int)j.nx;
    a.ny = (int)j.ny;
    a.nz = (int)j.nz;
    a.i_offset = (float)j.P.i_offset;
    a.i_scale = (float)j.P.i_scale;
    int *rad[3] = {&a.rx, &a.ry, &a.rz};
    float *tap[3] = {a.gx, a.gy, a.gz};
    const int64_t nn[3] = {j.nx, j.ny, j.nz};
    for (int ax = 0; ax < 3; ++ax) {
        const double s = j.P.sigma_pre / j.P.spacing[ax];
        const bool use = s > 0.0 && ax < j.P.dim && nn[ax] > 1;
        const int r = use ? (int)ceil(3.0 * s) : 0;
        *rad[ax] = r;
        double g[2 * snk::kPrepassMaxR + 1], sum = 0.0;
        for (int k = -r; k <= r; ++k) {
            g[k + r] = r ? exp(-(double)k * k / (2.0 * s * s)) : 1.0;
            sum += g[k + r];
        }
        for (int k = 0; k <= 2 * r; ++k) tap[ax][k] = (float)(g[k] / sum);
    }
    EHIP(e, snk::launch_prepass(a, e->stream));
    return SNK_OK;
}

// Items of the given jobs grouped by launch class; returns the class boundaries.
struct ItemPlan {
    std::vector<int2> items;
    std::vector<std::pair<ClassKey, std::pair<int, int>>> classes;   // key -> [begin, end)
    std::vector<snk_params> params;                                   // one job's parameters per class
    std::vector<int> joblist;
};

ItemPlan plan_items(const std::vector<EJob *> &js) {
    ItemPlan pl;
    std::map<ClassKey, std::vector<const EJob *>> by;
    for (const EJob *j : js) {
        ClassKey k{j->P.dim, (int)(j->dirs.size() / j->P.dim), j->P.n_rays, j->P.n_radial};
        by[k].push_back(j);
        pl.joblist.push_back(j->slot);
    }
    for (auto &kv : by) {
        const int b = (int)pl.items.size();
        for (const EJob *j : kv.second)
            for (int c = 0; c < j->n; ++c) pl.items.push_back(make_int2(j->slot, c));
        pl.classes.push_back({kv.first, {b, (int)pl.items.size()}});
        pl.params.push_back(kv.second.front()->P);
    }
    return pl;
}

snk_status upload_plan(snk_engine *e, const ItemPlan &pl) {
    snk_status st = grow(e, &e->d_items, &e->items_cap, pl.items.size());
    if (st != SNK_OK) return st;
    st = grow(e, &e->d_joblist, &e->joblist_cap, pl.joblist.size());
    if (st != SNK_OK) return st;
    if (!pl.items.empty())
        EHIP(e, hipMemcpyAsync(e->d_items, pl.items.data(), sizeof(int2) * pl.items.size(), hipMemcpyHostToDevice,
                               e->stream));
    if (!pl.joblist.empty())
        EHIP(e, hipMemcpyAsync(e->d_joblist, pl.joblist.data(), sizeof(int) * pl.joblist.size(),
                               hipMemcpyHostToDevice, e->stream));
    EHIP(e, hipStreamSynchronize(e->stream));
    unstage(e);
    return SNK_OK;
}

snk::BatchArgs batch_args(snk_engine *e, const ClassKey &k, int b, int end, int cls, int chunk, int tile) {
    snk::BatchArgs a{};
    a.tile_cap = tile;
    a.jobs = e->d_jobs;
    a.items = e->d_items + b;
    a.n_items = end - b;
    a.queue = e->d_queues + cls;
    a.chunk = chunk;
    a.counter = e->d_counters;
    a.max_D = k.D;
    a.max_M = k.M;
    return a;
}

int grid_for(snk_engine *e, const ClassKey &k, const Launch &L, int n_items) {
    int per_cu = snk::evolve_batch_max_blocks(k.dim, L.lanes, L.unroll, e->layout, k.M, L.tile);
    if (L.per_cu > 0) per_cu = std::min(per_cu, L.per_cu);
    return std::max(1, std::min(n_items, per_cu * e->cus));
}

// Evolve launches of every class of the plan (queue heads must be zero).
snk_status launch_classes(snk_engine *e, const ItemPlan &pl, int chunk, const std::vector<Launch> &shapes) {
    for (size_t c = 0; c < pl.classes.size(); ++c) {
        const ClassKey &k = pl.classes[c].first;
        const int b = pl.classes[c].second.first, end = pl.classes[c].second.second;
        const Launch &L = shapes[c];
        if (snk::evolve_lds_bytes(k.dim, L.lanes, k.M, L.tile) > 65536)
            return efail(e, SNK_EINVAL, "n_rays too large for this launch shape's LDS");
        snk::BatchArgs a = batch_args(e, k, b, end, (int)c, chunk, L.tile);
        EHIP(e, snk::launch_evolve_batch(a, k.dim, L.lanes, L.unroll, e->layout, L.persistent != 0, L.grid,
                                         e->stream));
        e->last_launch = L;
    }
    return SNK_OK;
}

// Pick the launch shape of each class: forced, cached, or timed on short trials.
snk_status shapes_for(snk_engine *e, const ItemPlan &pl, bool allow_trials, std::vector<Launch> &out) {
    out.clear();
    for (size_t c = 0; c < pl.classes.size(); ++c) {
        const ClassKey &k = pl.classes[c].first;
        const int b = pl.classes[c].second.first, end = pl.classes[c].second.second;
        const int n_items = end - b;
        Launch L{};
        auto it = e->tuned.find(k);
        if (e->force) {
            L = e->forced;
        } else if (it != e->tuned.end()) {
            L = it->second;
        } else if (allow_trials) {
            // every candidate evolves the class's items for a few iterations from their initial
            // state: lanes per contour, pair-points in flight, LDS box capacity (the gather tile),
            // and one workgroup per item or a persistent work queue with all or half of the
            // workgroups per CU that registers and LDS allow (contours per CU)
            const int trial_iters = 10;
            float best_ms = 1e30f;
            int tried = 0;
            for (int g : {64, 128, 256}) {
                for (int u : {1, 2}) {
                    for (int tile : {0, 2048, 4224, 8192}) {
                        if (snk::evolve_lds_bytes(k.dim, g, k.M, tile) > 65536) continue;
                        const int max_cu = snk::evolve_batch_max_blocks(k.dim, g, u, e->layout, k.M, tile);
                        // -1: one workgroup per item; 0: persistent, all it can hold; else that many
                        int cands[3] = {-1, 0, 0};
                        int nc = 2;
                        if (max_cu >= 2) cands[nc++] = max_cu / 2;
                        for (int ci = 0; ci < nc; ++ci) {
                            const int pc = cands[ci];
                            Launch T{g, u, pc >= 0 ? 1 : 0, 1, tile, pc > 0 ? pc : 0};
                            T.grid = grid_for(e, k, T, n_items);
                            EHIP(e, snk::launch_reset_items(e->d_jobs, e->d_items + b, n_items, e->d_init_ptrs,
                                                            e->stream));
                            EHIP(e, snk::launch_zero(reinterpret_cast<unsigned long long *>(e->d_queues), kQueueWords,
                                                     e->stream));
                            snk::BatchArgs a = batch_args(e, k, b, end, (int)c, trial_iters, tile);
                            EHIP(e, hipEventRecord(e->ev0, e->stream));
                            EHIP(e, snk::launch_evolve_batch(a, k.dim, g, u, e->layout, T.persistent != 0, T.grid,
                                                             e->stream));
                            EHIP(e, hipEventRecord(e->ev1, e->stream));
                            EHIP(e, hipEventSynchronize(e->ev1));
                            float ms = 0.0f;
                            EHIP(e, hipEventElapsedTime(&ms, e->ev0, e->ev1));
                            ++tried;
                            if (ms < best_ms) {
                                best_ms = ms;
                                L = T;
                            }
                        }
                    }
                }
            }
            L.trial_ms = best_ms;
            L.trials = tried;
            EHIP(e, snk::launch_reset_items(e->d_jobs, e->d_items + b, n_items, e->d_init_ptrs, e->stream));
            EHIP(e, hipStreamSynchronize(e->stream));
            unstage(e);
            e->tuned[k] = L;
        }
        L.grid = grid_for(e, k, L, n_items);
        out.push_back(L);
    }
    return SNK_OK;
}

}  // namespace

namespace {

snk_status collect(snk_engine *e, const std::vector<EJob *> &js) {
    for (EJob *j : js) {
        j->result.resize((size_t)j->n);
        if (j->n > 0)
            EHIP(e, hipMemcpyAsync(j->result.data(), j->d_st, sizeof(DevContour) * j->n, hipMemcpyDeviceToHost,
                                   e->stream));
    }
    EHIP(e, hipStreamSynchronize(e->stream));
    unstage(e);
    const double t = now_ms();
    for (EJob *j : js) {
        j->state = DONE;
        j->t_done = t;
        e->done_unpolled.push_back(j->id);
        e->completed += 1;
    }
    return SNK_OK;
}

void centre_of(const EJob &j, const DevContour &s, double *out) {
    for (int i = 0; i < 3; ++i)
        out[i] = i < j.P.dim ? ((double)s.anc[i] + (double)s.off[i]) * j.P.spacing[i] : 0.0;
}

}  // namespace

extern "C" {

snk_status snk_engine_create(snk_engine **out, int device, void *hip_stream, uint64_t hbm_budget_bytes) {
    if (!out) return SNK_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return SNK_EDEVICE;
    if (device < 0 || device >= count) return SNK_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return SNK_EDEVICE;
    snk_engine *e = new (std::nothrow) snk_engine();
    if (!e) return SNK_ENOMEM;
    e->device = device;
    e->stream = static_cast<hipStream_t>(hip_stream);
    if (!e->stream) {
        // a captured graph needs a stream other than the null stream
        if (hipStreamCreateWithFlags(&e->own_stream, hipStreamNonBlocking) != hipSuccess) {
            delete e;
            return SNK_EDEVICE;
        }
        e->stream = e->own_stream;
    }
    e->budget = hbm_budget_bytes;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        e->cus = prop.multiProcessorCount;
    if (hipEventCreate(&e->ev0) != hipSuccess || hipEventCreate(&e->ev1) != hipSuccess ||
        hipEventCreate(&e->ev2) != hipSuccess || hipMalloc(&e->d_counters, sizeof(unsigned long long) * 4) != hipSuccess ||
        hipMalloc(&e->d_queues, sizeof(int) * kMaxClasses) != hipSuccess) {
        snk_engine_destroy(e);
        return SNK_EDEVICE;
    }
    if (ensure_table(e, 64) != SNK_OK) {
        snk_engine_destroy(e);
        return SNK_ENOMEM;
    }
    *out = e;
    return SNK_OK;
}

snk_status snk_engine_destroy(snk_engine *e) {
    if (!e) return SNK_OK;
    (void)hipSetDevice(e->device);
    (void)hipStreamSynchronize(e->stream);
    drop_graph(e);
    e->staged.clear();
    for (auto &kv : e->jobs) {
        release_device(e, *kv.second);
        delete kv.second;
    }
    pool_drain(e);
    void *bufs[] = {e->d_jobs, e->d_init_ptrs, e->d_items, e->d_joblist, e->d_unfinished, e->d_counters, e->d_queues};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    for (hipEvent_t ev : {e->ev0, e->ev1, e->ev2})
        if (ev) (void)hipEventDestroy(ev);
    if (e->own_stream) (void)hipStreamDestroy(e->own_stream);
    delete e;
    return SNK_OK;
}

const char *snk_engine_last_error(const snk_engine *e) { return e ? e->err.c_str() : ""; }

snk_status snk_engine_set_launch(snk_engine *e, int32_t lanes_per_contour, int32_t pairs_in_flight,
                                 int32_t persistent, int32_t layout) {
    if (!e) return SNK_EINVAL;
    if (layout < 0 || layout > 2) return efail(e, SNK_EINVAL, "layout in {0,1,2}");
    const int lay = layout == 1 ? snk::kBufferPlain : (layout == 2 ? snk::kBufferQuad : snk::kBufferPair);
    if (lay != e->layout) {
        e->layout = lay;
        e->tuned.clear();
        drop_graph(e);
    }
    if (lanes_per_contour == 0) {
        e->force = false;
        return SNK_OK;
    }
    if ((lanes_per_contour != 64 && lanes_per_contour != 128 && lanes_per_contour != 256) ||
        (pairs_in_flight != 1 && pairs_in_flight != 2) || (persistent != 0 && persistent != 1))
        return efail(e, SNK_EINVAL, "lanes in {0,64,128,256}, pairs_in_flight in {1,2}, persistent in {0,1}");
    e->force = true;
    e->forced = Launch{lanes_per_contour, pairs_in_flight, persistent, 1, 0, 0};
    drop_graph(e);
    return SNK_OK;
}

snk_status snk_engine_set_tile(snk_engine *e, int32_t tile_voxels, int32_t workgroups_per_cu) {
    if (!e) return SNK_EINVAL;
    if (!e->force) return efail(e, SNK_ESTATE, "snk_engine_set_tile applies to a shape forced by snk_engine_set_launch");
    if (tile_voxels < 0 || tile_voxels > 16384 || workgroups_per_cu < 0)
        return efail(e, SNK_EINVAL, "tile_voxels in 0..16384, workgroups_per_cu >= 0");
    e->forced.tile = tile_voxels;
    e->forced.per_cu = workgroups_per_cu;
    drop_graph(e);
    return SNK_OK;
}

snk_status snk_engine_submit(snk_engine *e, const snk_params *p, const float *dirs, int32_t D, const void *vol,
                             snk_dtype dtype, int64_t nx, int64_t ny, int64_t nz, int on_device,
                             const double *centers, const float *r0, const uint32_t *ids, int64_t n,
                             int32_t n_iter, uint64_t *job) {
    if (!e || !p || !dirs || !vol || !job || (n > 0 && !centers) || n < 0 || n_iter < 0)
        return efail(e, SNK_EINVAL, "NULL or negative argument");
    (void)hipSetDevice(e->device);
    const snk_params &P = *p;
    if (P.dim != 2 && P.dim != 3) return efail(e, SNK_EINVAL, "dim must be 2 or 3");
    for (int i = 0; i < 3; ++i)
        if (!(P.spacing[i] > 0.0)) return efail(e, SNK_EINVAL, "spacing must be > 0");
    if (!(P.dR > 0.0) || !(P.r_max >= r_low(P)) || P.n_rays <= 0 || (P.n_rays & 1) || P.n_radial <= 0 ||
        P.n_rays / 2 > 768 || !(P.eps0 >= 0.0) || !(P.sigma_pre >= 0.0) || P.conv_window < 0 || P.conv_window > 255)
        return efail(e, SNK_EINVAL, "invalid parameters");
    if (D <= 0 || D != P.n_dirs || (int64_t)D * P.dim > 12288) return efail(e, SNK_EINVAL, "direction table size");
    // the evolve kernels take |u| <= 1 for granted when they decide that a sample ball lies inside
    // the volume (and skip clamping), so a row that is not a unit vector is refused as in
    // snk_set_directions
    for (int32_t k = 0; k < D; ++k) {
        double n2 = 0.0;
        for (int i = 0; i < P.dim; ++i) n2 += (double)dirs[k * P.dim + i] * dirs[k * P.dim + i];
        if (!(fabs(n2 - 1.0) < 1e-5)) return efail(e, SNK_EINVAL, "direction table rows must be unit vectors");
    }
    if (P.flags & ~snk::kFlagNoRotation)
        return efail(e, SNK_EINVAL, "engine jobs evolve by Monte-Carlo sums (exact lattice sums: snk_evolve)");
    if (e->dim != 0 && P.dim != e->dim) return efail(e, SNK_EINVAL, "all jobs of an engine must have the same dim");
    if (nx < 2 || ny < 2 || nz < 1 || (P.dim == 3 && nz < 2) || (P.dim == 2 && nz != 1))
        return efail(e, SNK_EINVAL, "volume shape");
    if (snk::volume_layout(P.dim, nx, ny, nz, 2) != snk::kBufferQuad)
        return efail(e, SNK_EINVAL, "engine volumes must fit the quad layout (16 B per voxel below 2 GiB)");
    if (n >= ((int64_t)1 << 30)) return efail(e, SNK_EINVAL, "too many seeds");
    for (int ax = 0; ax < 3; ++ax) {
        const double s = P.sigma_pre / P.spacing[ax];
        if (s > 0.0 && ax < P.dim && (int)ceil(3.0 * s) > snk::kPrepassMaxR)
            return efail(e, SNK_EINVAL, "sigma_pre too large for the pre-pass");
    }
    EJob *j = new (std::nothrow) EJob();
    if (!j) return efail(e, SNK_ENOMEM, "host allocation");
    j->id = e->next_id++;
    j->P = P;
    j->nx = nx;
    j->ny = ny;
    j->nz = nz;
    j->dtype = dtype;
    const size_t esz = dtype == SNK_U8 ? 1 : (dtype == SNK_U16 ? 2 : 4);
    j->raw_bytes = (size_t)(nx * ny * nz) * esz;
    if (on_device) {
        j->borrowed = vol;
    } else {
        const uint8_t *src = static_cast<const uint8_t *>(vol);
        j->host_raw.assign(src, src + j->raw_bytes);
    }
    j->dirs.assign(dirs, dirs + (size_t)D * P.dim);
    j->n = (int)n;
    j->n_iter = n_iter;
    j->init.resize((size_t)n);
    const double lo = r_low(P), hi = P.r_max;
    const int64_t nn[3] = {nx, ny, nz};
    for (int64_t i = 0; i < n; ++i) {
        DevContour &s = j->init[i];
        memset(&s, 0, sizeof(s));
        bool inside = true;
        for (int a = 0; a < 3; ++a) {
            if (a >= P.dim) continue;
            const double v = centers[i * 3 + a] / P.spacing[a];
            const double an = floor(v + 0.5);
            s.anc[a] = (int32_t)std::max(std::min(an, 2.0e9), -2.0e9);
            s.off[a] = (float)(v - (double)s.anc[a]);
            const double vv = (double)s.anc[a] + (double)s.off[a];
            if (!(vv >= 0.0) || vv > (double)(nn[a] - 1)) inside = false;
        }
        double R = r0 ? (double)r0[i] : P.r_init;
        if (!isfinite(R)) {
            delete j;
            return efail(e, SNK_EINVAL, "initial radius not finite");
        }
        s.R = (float)std::min(std::max(R, lo), hi);
        s.id = ids ? ids[i] : (uint32_t)i;
        s.status = inside ? SNK_ACTIVE : SNK_OUT;
    }
    j->grid_cells = snk_grid_for(P, nx, ny, nz, j->G, &j->cell);
    j->bytes = footprint(*j, j->grid_cells);
    if (j->bytes > e->budget) {
        delete j;
        return efail(e, SNK_EBUSY, "job exceeds the whole HBM budget");
    }
    j->t_submit = now_ms();
    e->dim = P.dim;
    e->jobs[j->id] = j;
    e->pending.push_back(j->id);
    e->submitted += 1;
    *job = j->id;
    return SNK_OK;
}

snk_status snk_engine_run(snk_engine *e) {
    if (!e) return SNK_EINVAL;
    (void)hipSetDevice(e->device);
    std::vector<EJob *> fresh;
    snk_status st = admit_pending(e, fresh);
    if (st != SNK_OK) return st;
    // the batch: every admitted job (RUNNING or DONE), evolved from its seeds
    std::vector<EJob *> js;
    std::vector<uint64_t> ids;
    for (auto &kv : e->jobs)
        if (kv.second->state != PENDING && kv.second->slot >= 0) {
            js.push_back(kv.second);
            ids.push_back(kv.first);
        }
    if (js.empty()) return SNK_OK;
    ItemPlan pl = plan_items(js);
    if ((int)pl.classes.size() > kMaxClasses) return efail(e, SNK_EINVAL, "too many launch classes");
    const bool same = e->graph && ids == e->graph_jobs;
    if (!same) {
        drop_graph(e);
        st = upload_plan(e, pl);
        if (st != SNK_OK) return st;
        std::vector<Launch> shapes;
        for (EJob *j : js) {
            st = prepass_job(e, *j);
            if (st != SNK_OK) return st;
        }
        st = shapes_for(e, pl, true, shapes);
        if (st != SNK_OK) return st;
        int max_target = 0;
        for (EJob *j : js) max_target = std::max(max_target, j->n_iter);
        hipGraph_t g = nullptr;
        EHIP(e, hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
        bool ok = snk::launch_reset_items(e->d_jobs, e->d_items, (int)pl.items.size(), e->d_init_ptrs, e->stream) ==
                  hipSuccess;
        ok = ok && snk::launch_zero(e->d_counters, 4, e->stream) == hipSuccess;
        ok = ok && snk::launch_zero(reinterpret_cast<unsigned long long *>(e->d_queues), kQueueWords, e->stream) ==
                       hipSuccess;
        for (EJob *j : js) ok = ok && prepass_job(e, *j) == SNK_OK;
        ok = ok && launch_classes(e, pl, max_target, shapes) == SNK_OK;
        ok = ok && snk::launch_energy_vox_batch(e->d_jobs, e->d_items, (int)pl.items.size(), js[0]->P.dim == 2 ? 2 : 3,
                                                e->stream) == hipSuccess;
        ok = ok && snk::launch_select_batch(e->d_jobs, e->d_joblist, (int)pl.joblist.size(), js[0]->P.dim == 2 ? 2 : 3,
                                            e->stream) == hipSuccess;
        hipError_t ce = hipStreamEndCapture(e->stream, &g);
        if (!ok || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return efail(e, SNK_EDEVICE, "graph capture of the batched run failed");
        }
        hipError_t ie = hipGraphInstantiate(&e->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            e->graph = nullptr;
            return efail(e, SNK_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
        }
        e->graph_jobs = ids;
    }
    EHIP(e, hipEventRecord(e->ev0, e->stream));
    EHIP(e, hipGraphLaunch(e->graph, e->stream));
    EHIP(e, hipEventRecord(e->ev1, e->stream));
    e->graph_replays += 1;
    st = collect(e, js);
    if (st != SNK_OK) return st;
    float ms = 0.0f;
    EHIP(e, hipEventElapsedTime(&ms, e->ev0, e->ev1));
    e->last_ms = ms;
    e->last_evolve_ms = 0;
    unsigned long long cnt = 0;
    EHIP(e, hipMemcpy(&cnt, e->d_counters, sizeof(cnt), hipMemcpyDeviceToHost));
    e->last_evolved = (int64_t)cnt;
    return SNK_OK;
}

snk_status snk_engine_step(snk_engine *e, int32_t chunk, int32_t *n_finished) {
    if (!e || chunk <= 0) return SNK_EINVAL;
    (void)hipSetDevice(e->device);
    if (n_finished) *n_finished = 0;
    drop_graph(e);
    std::vector<EJob *> fresh;
    snk_status st = admit_pending(e, fresh);
    if (st != SNK_OK) return st;
    for (EJob *j : fresh) {
        st = prepass_job(e, *j);
        if (st != SNK_OK) return st;
        j->prepared = true;
    }
    std::vector<EJob *> running;
    for (auto &kv : e->jobs)
        if (kv.second->state == RUNNING) running.push_back(kv.second);
    if (running.empty()) return SNK_OK;
    ItemPlan pl = plan_items(running);
    if ((int)pl.classes.size() > kMaxClasses) return efail(e, SNK_EINVAL, "too many launch classes");
    st = upload_plan(e, pl);
    if (st != SNK_OK) return st;
    std::vector<Launch> shapes;
    st = shapes_for(e, pl, false, shapes);
    if (st != SNK_OK) return st;
    EHIP(e, snk::launch_zero(e->d_counters, 4, e->stream));
    EHIP(e, snk::launch_zero(reinterpret_cast<unsigned long long *>(e->d_queues), kQueueWords, e->stream));
    EHIP(e, hipEventRecord(e->ev0, e->stream));
    st = launch_classes(e, pl, chunk, shapes);
    if (st != SNK_OK) return st;
    EHIP(e, hipEventRecord(e->ev1, e->stream));
    // which jobs have stopped?
    EHIP(e, hipMemsetAsync(e->d_unfinished, 0, sizeof(int) * e->table_cap, e->stream));
    EHIP(e, snk::launch_count_unfinished(e->d_jobs, e->d_items, (int)pl.items.size(), e->d_unfinished, e->stream));
    std::vector<int> unfinished((size_t)e->table_cap, 0);
    EHIP(e, hipMemcpyAsync(unfinished.data(), e->d_unfinished, sizeof(int) * e->table_cap, hipMemcpyDeviceToHost,
                           e->stream));
    EHIP(e, hipStreamSynchronize(e->stream));
    unstage(e);
    float ms = 0.0f;
    EHIP(e, hipEventElapsedTime(&ms, e->ev0, e->ev1));
    e->last_evolve_ms = ms;
    unsigned long long cnt = 0;
    EHIP(e, hipMemcpy(&cnt, e->d_counters, sizeof(cnt), hipMemcpyDeviceToHost));
    e->last_evolved = (int64_t)cnt;
    std::vector<EJob *> fin;
    for (EJob *j : running)
        if (unfinished[j->slot] == 0) fin.push_back(j);
    if (fin.empty()) return SNK_OK;
    ItemPlan fp = plan_items(fin);
    st = upload_plan(e, fp);
    if (st != SNK_OK) return st;
    const int dim = fin[0]->P.dim == 2 ? 2 : 3;
    EHIP(e, snk::launch_energy_vox_batch(e->d_jobs, e->d_items, (int)fp.items.size(), dim, e->stream));
    EHIP(e, snk::launch_select_batch(e->d_jobs, e->d_joblist, (int)fp.joblist.size(), dim, e->stream));
    st = collect(e, fin);
    if (st != SNK_OK) return st;
    for (EJob *j : fin) release_device(e, *j);
    if (n_finished) *n_finished = (int32_t)fin.size();
    return SNK_OK;
}

snk_status snk_engine_poll(snk_engine *e, uint64_t *done, int64_t cap, int64_t *n_done) {
    if (!e || !n_done) return SNK_EINVAL;
    const int64_t k = std::min<int64_t>(cap, (int64_t)e->done_unpolled.size());
    for (int64_t i = 0; i < k; ++i)
        if (done) done[i] = e->done_unpolled[i];
    e->done_unpolled.erase(e->done_unpolled.begin(), e->done_unpolled.begin() + k);
    *n_done = k;
    return SNK_OK;
}

snk_status snk_engine_read(snk_engine *e, uint64_t job, float *radii, double *centers, float *e_mc, float *e_vox,
                           int32_t *iters, uint8_t *status, uint8_t *keep, int64_t cap, int64_t *n_out) {
    if (!e) return SNK_EINVAL;
    auto it = e->jobs.find(job);
    if (it == e->jobs.end()) return efail(e, SNK_EINVAL, "unknown job");
    const EJob &j = *it->second;
    if (n_out) *n_out = j.n;
    if (j.state != DONE) return efail(e, SNK_ESTATE, "job not finished");
    if (cap < j.n) return efail(e, SNK_ERANGE, "capacity smaller than the job's contour count");
    for (int i = 0; i < j.n; ++i) {
        const DevContour &s = j.result[i];
        if (radii) radii[i] = s.R;
        if (centers) centre_of(j, s, &centers[i * 3]);
        if (e_mc) e_mc[i] = s.e_mc;
        if (e_vox) e_vox[i] = s.e_vox;
        if (iters) iters[i] = s.iters;
        if (status) status[i] = s.status;
        if (keep) keep[i] = s.keep;
    }
    return SNK_OK;
}

snk_status snk_engine_job_times(snk_engine *e, uint64_t job, double *submit_ms, double *done_ms) {
    if (!e) return SNK_EINVAL;
    auto it = e->jobs.find(job);
    if (it == e->jobs.end()) return efail(e, SNK_EINVAL, "unknown job");
    if (submit_ms) *submit_ms = it->second->t_submit;
    if (done_ms) *done_ms = it->second->t_done;
    return SNK_OK;
}

snk_status snk_engine_release(snk_engine *e, uint64_t job) {
    if (!e) return SNK_EINVAL;
    auto it = e->jobs.find(job);
    if (it == e->jobs.end()) return efail(e, SNK_EINVAL, "unknown job");
    EJob *j = it->second;
    if (j->state == PENDING) e->pending.erase(std::find(e->pending.begin(), e->pending.end(), job));
    (void)hipSetDevice(e->device);
    (void)hipStreamSynchronize(e->stream);
    if (j->slot >= 0 || j->block) drop_graph(e);
    release_device(e, *j);
    delete j;
    e->jobs.erase(it);
    return SNK_OK;
}

snk_status snk_engine_get_stats(snk_engine *e, snk_engine_stats *s) {
    if (!e || !s) return SNK_EINVAL;
    memset(s, 0, sizeof(*s));
    s->submitted = e->submitted;
    s->admitted = e->admitted;
    s->completed = e->completed;
    s->pending = (int64_t)e->pending.size();
    int64_t running = 0;
    for (auto &kv : e->jobs) running += kv.second->state == RUNNING;
    s->running = running;
    s->bytes_in_use = e->in_use;
    s->budget = e->budget;
    s->last_ms = e->last_ms;
    s->last_evolve_ms = e->last_evolve_ms;
    s->last_evolved = e->last_evolved;
    s->lanes_per_contour = e->last_launch.lanes;
    s->pairs_in_flight = e->last_launch.unroll;
    s->persistent = e->last_launch.persistent;
    s->layout = e->layout == snk::kBufferPlain ? 1 : (e->layout == snk::kBufferQuad ? 2 : 0);
    s->graph_replays = e->graph_replays;
    return SNK_OK;
}

snk_status snk_engine_tuned_shapes(snk_engine *e, int32_t *rows, int64_t cap, int64_t *n_out) {
    if (!e) return SNK_EINVAL;
    const int64_t n = (int64_t)e->tuned.size();
    if (n_out) *n_out = n;
    if (!rows) return SNK_OK;
    if (cap < n) return efail(e, SNK_ERANGE, "capacity below the number of tuned classes");
    int64_t i = 0;
    for (const auto &kv : e->tuned) {
        const ClassKey &k = kv.first;
        const Launch &L = kv.second;
        int32_t *r = rows + i * SNK_TUNED_W;
        r[0] = k.dim;
        r[1] = k.D;
        r[2] = k.M;
        r[3] = k.L;
        r[4] = L.lanes;
        r[5] = L.unroll;
        r[6] = L.persistent;
        r[7] = L.per_cu;
        r[8] = L.tile;
        r[9] = (int32_t)lrintf(L.trial_ms * 1000.0f);
        r[10] = L.trials;
        ++i;
    }
    return SNK_OK;
}

}  // extern "C"
