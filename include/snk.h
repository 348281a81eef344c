/*
 * snk.h -- C ABI of the MI355X (gfx950) snakuscule evolution library, libsnk.so.
 *
 * The library evolves many independent 3D (or 2D) snakuscules on one GPU, as in arXiv
 * 1804.06304 ("Three-Dimensional GPU-Accelerated Active Contours for Automated Localization of
 * Cells in Large Images"): load a volume and seed points, set the energy parameters, evolve N
 * gradient-descent iterations with Monte-Carlo integration, then read back radii, centres and
 * energies together with the detected set.
 *
 * Conventions (all entry points):
 *   - Every call returns snk_status; 0 is success. No C++ exception crosses this boundary.
 *     On failure snk_last_error() returns a message; the context stays usable unless the error
 *     is SNK_EDEVICE (a HIP runtime error, whose text is included).
 *   - A context belongs to one host thread at a time.
 *   - Work is enqueued asynchronously on the context's HIP stream. Calls that return data to the
 *     host (snk_read, snk_get_state, snk_trace_step, snk_read_volume with on_device = 0,
 *     snk_get_timing) and snk_sync synchronise that stream before returning.
 *   - Volumes are [z][y][x] with x fastest. Physical coordinates have their origin at the centre
 *     of voxel (0,0,0); voxel (i,j,k) sits at (i*h_x, j*h_y, k*h_z). 2D images are volumes with
 *     nz = 1 and dim = 2; their z coordinate is 0.
 *   - Per-contour arrays are in seed order. Centres cross the ABI as double (n x 3) so that
 *     large images keep sub-voxel precision; the device holds each centre as an integer voxel
 *     anchor plus an FP32 offset.
 *   - Host buffers passed in are read before the call returns; the library keeps no pointer to
 *     them. A device buffer passed with on_device = 1 is borrowed: it must stay valid until the
 *     next snk_sync (or any synchronising call) on that context.
 *   - Device memory for the smoothed volume, contour state and scratch is allocated by the
 *     library (hipMalloc) and freed by snk_destroy.
 */
#ifndef SNK_H
#define SNK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t snk_status;
#define SNK_OK 0
#define SNK_EINVAL (-1)   /* bad argument or parameter                                    */
#define SNK_ENOMEM (-2)   /* device allocation failed                                      */
#define SNK_EDEVICE (-3)  /* HIP runtime error (text in snk_last_error)                    */
#define SNK_ESTATE (-4)   /* call out of order (e.g. evolve before a volume is loaded)      */
#define SNK_EBUSY (-5)    /* admission refused (engine: HBM budget or slots exhausted)      */
#define SNK_ERANGE (-6)   /* output capacity too small; *n_out holds the required count     */

typedef enum { SNK_U8 = 0, SNK_U16 = 1, SNK_F32 = 2 } snk_dtype;

/* Per-contour status byte: low nibble is the state, bit 0x10 is set once R was clamped. */
#define SNK_ACTIVE 0       /* still evolving                                              */
#define SNK_CONVERGED 1    /* froze after conv_window small steps (Results: "they converge") */
#define SNK_MAXITER 2      /* stopped on the iteration limit (set by snk_finalize)          */
#define SNK_OUT 3          /* centre left the volume                                        */
#define SNK_NONFINITE 4    /* state became NaN/Inf                                          */
#define SNK_CULLED 5       /* retired by a culling pass during evolution (snk_evolve_cull)  */
#define SNK_CLAMPED 0x10

/* Parameters of one run. Physical units are x-voxel units.
 *   dim          2 or 3.
 *   spacing      physical step per voxel along x, y, z (anisotropic stacks; Results: voxels are
 *                made isotropic -- here samples live in physical space and map through h).
 *   sigma_pre    low-pass sigma of the pre-pass, physical units; 0 disables it (Sec. II-E).
 *   i_offset, i_scale   image I = (raw - i_offset) * i_scale before the low-pass.
 *   dR           outer ramp width Delta R; the inner ramp is rho*dR (Sec. II-B, Eq. (5)).
 *   eps0         step constant: eps_n = eps0 / sqrt(n) (Eqs. (12)-(15)).
 *   r_min, r_max bounds on R; the lower bound is raised to dR(1+rho)/(2(1-rho)), the smallest
 *                radius at which the four regions of the weight do not overlap.
 *   r_init       initial radius R0 of every seed when snk_load_seeds gets no per-seed radii.
 *   n_dirs       D, rows of the direction table.
 *   n_rays       M, rays per contour-iteration; even (antithetic pairs).
 *   n_radial     L, radial points per ray; a contour-iteration draws M*L points uniform in the
 *                ball of radius R + dR/2 (Sec. II-E).
 *   seed         Philox4x32-10 key (low word, high word).
 *   conv_tol, conv_window   freeze a contour after conv_window consecutive steps with
 *                max(|dR|, |dc|) < conv_tol; conv_window = 0 runs to the iteration limit.
 *   e0           energy threshold of the selection (Results: contours above E0 are removed).
 *   flags        bit 0: do not rotate the direction table (test mode; biased sampling).
 *                bit 1: exact sums: every iteration takes A, B_R, B_c over all lattice points
 *                within R + dR/2 of the centre (the point set of Eq. (5)), times the voxel
 *                measure, instead of the Monte-Carlo estimate: the gradient of the exact discrete
 *                energy, deterministic (no random numbers; n_dirs, n_rays, n_radial and seed are
 *                not used). Plain context path only (snk_engine_submit rejects it).
 *                bit 2: centre force in its image-gradient form: with the sample offsets from the
 *                centre held fixed, E = (2R)^-d * integral over the ball of S(|y|) I(c + y), so
 *                dE/dc = (2R)^-d * integral S(|y|) grad I(c + y); B_c (trace columns 2..4)
 *                becomes (V/N) sum S * grad I, with the gradient of the trilinear interpolant of
 *                the same corners (zero along axes beyond the volume's faces). Same expectation as
 *                the weight form (Eqs. (7)-(10)), every sample contributes instead of only those
 *                in the two ramps; A and B_R are unchanged (not in the paper: a variance-reduction
 *                option). Monte-Carlo only (SNK_EINVAL with bit 1); lanes_per_contour >= 64 and
 *                layout 1, 2 or 4 (two pair-points in flight are used); plain context path only.
 *                Other bits must be zero.
 */
typedef struct snk_params {
    int32_t dim;
    double spacing[3];
    double sigma_pre;
    double i_offset, i_scale;
    double dR;
    double eps0;
    double r_min, r_max, r_init;
    int32_t n_dirs, n_rays, n_radial;
    uint64_t seed;
    double conv_tol;
    int32_t conv_window;
    double e0;
    int32_t flags;
} snk_params;

/* Width of one contour's row written by snk_trace_step. Layout:
 *  0 A = (V/N) sum S*I          1 B_R = (V/N) sum dS/dR * I
 *  2..4 B_c = -(V/N) sum dS/dr * I * u  (x, y, z; z = 0 in 2D; flags bit 2: (V/N) sum S grad I)
 *  5 E_mc = A / (2R)^d          6 dR step = -(eps/2) (B_R - (d/R) A) / (2R)^d  (before clamping)
 *  7..9 dc step = -(eps/2) B_c / (2R)^d                                             (physical)
 *  10 n (iteration number)      11 R before the step       12 eps
 *  13..15 reserved (0). */
#define SNK_TRACE_W 16

typedef struct snk_ctx snk_ctx;

/* Create a context on HIP device `device`, enqueuing on `hip_stream` (a hipStream_t; NULL means
 * the device's null stream). The stream must outlive the context. */
snk_status snk_create(snk_ctx **out, int device, void *hip_stream);

/* Free the context and every device buffer it owns (synchronises its stream first). */
snk_status snk_destroy(snk_ctx *ctx);

/* Validate and store the parameters (copied). Must precede snk_load_seeds. Changing sigma_pre,
 * i_offset, i_scale or spacing after a volume is loaded re-runs the pre-pass at the next evolve. */
snk_status snk_set_params(snk_ctx *ctx, const snk_params *params);

/* Launch shape of the evolution kernel: lanes per contour (0 = automatic; 16 or 32: several
 * contours share one wave64; 64: one wave; 128 or 256: a workgroup of 2 or 4 waves), antithetic
 * pair-points whose gathers one lane issues before consuming them (0 = automatic, 1, 2 or 4; 4 is
 * taken with 64 or 128 lanes and outside snk_trace_step, otherwise it runs as 2), and the
 * layout the kernel reads the smoothed volume from (0 = automatic: column pairs when they fit, else
 * plain; 1 = plain FP32,
 * 2 = quad: one 16-byte record per voxel with its +x, +y, +xy neighbours, 4x the FP32 volume; needs
 * 16 * nx*ny*nz below 2 GiB and ny, nz <= 65535, else SNK_EINVAL at the next evolve; 3 = plain FP32
 * with 64-bit addressing, the path of volumes beyond 2 GiB; 4 = column pairs: (J(x,y,z),
 * J(x,y+1,z)) per voxel, twice the FP32 volume, so one 16-byte load fetches the four corners of a
 * cell's plane; needs 8 * nx*ny*nz below 2 GiB and ny, nz <= 65535, else SNK_EINVAL at the next
 * evolve; the exact sums, and in 2D the gradient-form sums and LDS boxes, read the plain copy
 * instead). Layouts change only how voxels are
 * fetched: results are bit-identical across layouts and across pair-point counts, and depend on
 * lanes_per_contour only through FP32 summation order. */
snk_status snk_set_launch(snk_ctx *ctx, int32_t lanes_per_contour, int32_t pairs_in_flight, int32_t layout);

/* LDS box of the Monte-Carlo evolution (whole-wave launch shapes, layouts 1, 2 and 4): each contour
 * keeps a box of the smoothed volume around its sample ball (Sec. II-E) in on-chip memory, staged
 * with a margin and re-staged only when the ball leaves it, and reads the trilinear corners of its
 * samples from there. tile_voxels = -1: automatic (boxes only when more than four contours per
 * compute unit must stay resident, where their footprints overflow the L2: the largest capacity
 * that keeps them all resident), 0: off (every corner read from the volume), 1..16384: capacity in
 * voxels (4 bytes each). An iteration whose ball does not fit, or
 * reaches the volume's edge, reads the volume. Results are bit-identical with and without the box.
 * SNK_EINVAL if tile_voxels is out of range, or at the next evolve if the box and the kernel's other
 * LDS exceed 64 KiB per workgroup. */
snk_status snk_set_tile(snk_ctx *ctx, int32_t tile_voxels);

/* Star-shaped contours (not in the paper: a builder-defined extension of its sphere). With
 * smooth >= 0 the following evolves give each contour one radius R_k per table direction T_k; the
 * directions stay fixed in space (no random rotation). The energy is the table average of
 * per-direction radial energies, E = (1/D) sum_k (2R_k)^-d omega_d d integral S(s; R_k)
 * I(c + s T_k) s^(d-1) ds (Eq. (5)'s weight and normalisation along each direction; the sphere's
 * energy when every R_k is equal). Each iteration draws the sphere sampler's Philox pairs: pair m
 * picks k, its rays run along +T_k with radius R_k and along -T_k with the radius of the opposite
 * table direction, at the sphere's radial points (R + dR/2)((l + xi)/L)^(1/d). The centre force
 * sums every ray's (Eqs. (7)-(10) along each ray); each sampled direction gets the unbiased
 * estimate g_k of dE/dR_k from its rays. Step: c -= (eps/2) g_c; R_k -= (eps/2) D g_k +
 * min(1, eps smooth / 2) (R_k - mean of its neighbours' radii), from the old radii; the neighbours
 * are the 6 (3D) or 2 (2D) directions nearest to T_k, made symmetric. Clamps, OUT and the stop
 * rule as for the sphere (the move of an iteration is the largest |dR_k| and |dc|); status bit
 * 0x10 when any radius was clamped. snk_read's radius is the mean of the R_k and its e_vox is the
 * last Monte-Carlo energy, which snk_finalize's selection ranks by (overlaps against the mean
 * radius). Needs a direction table with every opposite direction (else SNK_EINVAL at the next
 * evolve), n_radial = 16, and flags bits 1 and 2 clear; runs 64 or 128 lanes per contour (the
 * lanes_per_contour of snk_set_launch; 0: 128; other values SNK_EINVAL at the next evolve), ignores
 * its other knobs and snk_set_tile; snk_trace_step returns SNK_EINVAL. smooth < 0: the sphere
 * (default). Radii start tied at each contour's R after snk_load_seeds, snk_set_state or
 * snk_set_directions. */
snk_status snk_set_star(snk_ctx *ctx, double smooth);

/* Per-direction radii of the star contours, n x n_dirs in seed order (row k = direction k); cap in
 * floats (SNK_ERANGE with *n_out = n * n_dirs if smaller). */
snk_status snk_get_star_radii(snk_ctx *ctx, float *radii, int64_t cap, int64_t *n_out);

/* Replace the per-direction radii (n x n_dirs, each in (0, r_max]); n must equal the seeded count.
 * Call after snk_set_state, which resets them to the tied radius. */
snk_status snk_set_star_radii(snk_ctx *ctx, const float *radii, int64_t n);

/* Direction table: D rows of `dim` floats (host pointer), unit vectors, D * dim <= 12288. D must
 * equal params.n_dirs at evolve time. Sec. II-E: the table's directions, randomly rotated per
 * contour-iteration, carry the Monte-Carlo rays. */
snk_status snk_set_directions(snk_ctx *ctx, const float *dirs, int32_t D);

/* Load a raw volume nx*ny*nz of `dtype` (host pointer copied, or device pointer borrowed when
 * on_device = 1). The pre-pass (Sec. II-E low-pass) runs at the next snk_prepass / snk_evolve.
 * nx*ny*nz must be below 2^31; for dim = 3 every axis needs >= 2 voxels. */
snk_status snk_load_volume(snk_ctx *ctx, const void *data, snk_dtype dtype, int64_t nx, int64_t ny,
                           int64_t nz, int on_device);

/* Run the pre-pass now: J = Gaussian_{sigma_pre/h}((raw - i_offset) * i_scale), separable,
 * taps |k| <= ceil(3 sigma), clamp-to-edge. Enqueued on the stream. */
snk_status snk_prepass(snk_ctx *ctx);

/* Seed n contours (host pointers): centres n x 3 physical (double), optional per-seed initial
 * radii r0 (NULL: params.r_init), optional 32-bit ids (NULL: 0..n-1) that key the Philox
 * streams, so a contour's samples do not depend on its position in the list. Radii are clamped
 * into the bounds; seeds outside the volume start as SNK_OUT. Resets iteration counters. The host
 * arrays are read before the call returns; the upload is enqueued on the stream (from pinned
 * memory, without waiting for it). */
snk_status snk_load_seeds(snk_ctx *ctx, const double *centers, const float *r0, const uint32_t *ids,
                          int64_t n);

/* Run up to n_iter further iterations of every SNK_ACTIVE contour (Eqs. (7)-(15) with
 * Monte-Carlo sums, Sec. II-E); each contour continues its own iteration counter, so
 * evolve(a) then evolve(b) equals evolve(a + b). Runs the pre-pass first if needed. With 64 or
 * more iterations (and no per-iteration trace) the iterations are enqueued as two kernel launches
 * of about half each, which only changes how the still-active contours are spread over the CUs. */
snk_status snk_evolve(snk_ctx *ctx, int32_t n_iter);

/* End of evolution (Results): contours still ACTIVE become SNK_MAXITER; compute the exact
 * Eq. (5) energy E_vox of every contour (sum over the lattice points within R + dR/2, times the
 * voxel measure, clamp-to-edge outside the volume); then select: candidates are CONVERGED or
 * MAXITER with E_vox <= e0, and overlapping candidates (|c' - c''| < rho*max(R', R'')) compete,
 * the lower (E_vox, id) surviving -- identical to sequential greedy in ascending order. */
snk_status snk_finalize(snk_ctx *ctx);

/* snk_finalize for callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc. Same kernels, same results as snk_finalize, but
 * the selection's scratch (grid cells, per-contour items, cells and decisions, counters) lives in a
 * static device array of the library, about 6 MB, that each GPU the library runs on holds until the
 * process ends; the call itself calls no hipMalloc, hipFree or allocating library routine. Limits:
 * at most 131072 contours and 524288 cells of the selection grid (cell edge rho * r_max * 1.01 + 0.01
 * physical, widened until the grid has at most 4,194,304 cells); beyond them SNK_EINVAL and nothing
 * is enqueued. The pre-pass must already have run (snk_prepass, snk_evolve or snk_finalize since the
 * volume or its parameters last changed), else SNK_ESTATE. Every call on one GPU shares that GPU's
 * array and rewrites it before reading it: calls that overlap on one GPU (two streams, two contexts
 * or two threads without ordering between them) race and give undefined selections. */
snk_status snk_finalize_noalloc(snk_ctx *ctx);

/* Unattended workflow (the initial configuration of Sec. II-A / II-B: contours placed on a lattice,
 * neighbours sqrt(1.5) R apart; culling while evolving, the remedy the Conclusion proposes for the
 * work spent on contours that are culled at the end).
 *
 * snk_seed_lattice replaces the seeds with the centres of a cubic (2D: square) lattice of pitch
 * `pitch` (physical units; <= 0: sqrt(1.5) * params.r_init) centred in the volume: per axis
 * k = max(1, floor((n - 1) h / pitch)) points, the first at ((n - 1) h - (k - 1) pitch) / 2, x fastest.
 * Radii params.r_init, ids 0..n-1. *n_out (may be NULL) receives the contour count. */
snk_status snk_seed_lattice(snk_ctx *ctx, double pitch, int64_t *n_out);

/* snk_evolve with a culling pass after every `cull_every` (> 0) iterations and after the last one.
 * A pass ranks the live contours (ACTIVE or CONVERGED) by the Monte-Carlo energy of their last
 * iteration (e_mc of snk_read; the exact energy is left to snk_finalize): candidates are the live
 * contours with a finite energy, all of them while fewer than `grace_iters` iterations of this call
 * have run, afterwards those with e_mc <= the culling threshold (params.e0 unless snk_set_cull
 * sets another; a contour that stopped early is judged like the others once the grace period is
 * over); overlapping candidates compete as in snk_finalize (the lower (e_mc, id) survives) unless
 * snk_set_cull switches the competition off; the losers and the live non-candidates become
 * SNK_CULLED (clamp flag kept) and stop.
 * n_iter = 0 runs one culling pass. Timing (snk_get_timing): evolve_ms covers the evolve launches
 * and the passes; evolved counts every contour-iteration of the call. After each pass the next chunk
 * launches only the contours still active (their indices compacted on the device; star contours
 * launch every slot), which changes where contours run, never their results. Without competition
 * (sphere contours, no repulsion, n_iter > 0) a pass decides each contour alone, so the call runs
 * one evolution that applies the passes between chunks itself (an active contour above the
 * threshold at a pass point retires in the evolve kernel, whose workgroup slot then goes to the
 * next contour) and one pass after it: the same outcome, with no relaunches. */
snk_status snk_evolve_cull(snk_ctx *ctx, int32_t n_iter, int32_t cull_every, int32_t grace_iters);

/* Soft repulsion between neighbouring contours (not in the paper: its contours are independent
 * while they evolve, Sec. II-D, and compete only afterwards). With kappa > 0, contour i descends its
 * energy plus kappa * sum_j w(t_ij), t_ij = |c_i - c_j| / (rho (R_i + R_j)), w(t) = (1 - t)^2 for
 * t < 1 and 0 beyond: the inner spheres (radius rho R, the cell estimates) of overlapping contours
 * push each other apart and shrink. The neighbours (the live contours, ACTIVE or CONVERGED) are held
 * at a snapshot taken every `every` iterations (1: every iteration); the gradient joins the energy's
 * in the step of Eqs. (12)-(15). kappa = 0 (default) is the paper's contour exactly. Applies to
 * snk_evolve, snk_evolve_cull and snk_trace_step on sphere contours with lanes_per_contour >= 64
 * (else SNK_EINVAL at the evolve); a contour overlapping more than 64 neighbours makes the evolve
 * return SNK_ERANGE (its list keeps the 64 lowest indices). Evolving with repulsion synchronises the
 * context's stream at the end of the call. SNK_EINVAL for a negative or non-finite kappa or
 * every < 1. */
snk_status snk_set_repulsion(snk_ctx *ctx, double kappa, int32_t every);

/* Threshold and competition of the culling passes of snk_evolve_cull (the Conclusion's dynamic
 * culling leaves both open). After the grace period a pass's candidates are the live contours with
 * e_mc <= e_cull (NaN, the default: params.e0); a laxer threshold (e.g. e0 / 4) retires only contours
 * still far from being cells, so the final selection (at e0, by the exact energy) loses none of
 * the cells it would find without culling. compete = 1 (default): overlapping candidates compete
 * as in snk_finalize and the losers are retired too; 0: every candidate survives the pass.
 * SNK_EINVAL for an infinite e_cull or compete outside {0, 1}. */
snk_status snk_set_cull(snk_ctx *ctx, double e_cull, int32_t compete);

/* Read back (synchronises). Any output pointer may be NULL. radii, e_mc (last Monte-Carlo
 * energy), e_vox (exact energy, valid after snk_finalize), iters, status, keep (1 = detected
 * cell) are n-long; centers is n x 3 physical (double). If cap < n nothing is written,
 * *n_out = n and SNK_ERANGE is returned. */
snk_status snk_read(snk_ctx *ctx, float *radii, double *centers, float *e_mc, float *e_vox,
                    int32_t *iters, uint8_t *status, uint8_t *keep, int64_t cap, int64_t *n_out);

/* Checkpoint: the full evolving state (centre, radius, iteration counter, status, convergence
 * streak). Same capacity rule as snk_read. */
snk_status snk_get_state(snk_ctx *ctx, double *centers, float *radii, int32_t *iters,
                         uint8_t *status, uint8_t *streak, int64_t cap, int64_t *n_out);

/* Resume / teacher forcing: overwrite the state of the n loaded contours (n must equal the
 * seeded count). streak may be NULL (zeros). Reads the current state back first (synchronises);
 * the upload of the new one is enqueued like snk_load_seeds'. */
snk_status snk_set_state(snk_ctx *ctx, const double *centers, const float *radii, const int32_t *iters,
                         const uint8_t *status, const uint8_t *streak, int64_t n);

/* Parity aid: run exactly one iteration of every ACTIVE contour and write its terms
 * (n x SNK_TRACE_W floats, host pointer; rows of inactive contours are zero). Synchronises. */
snk_status snk_trace_step(snk_ctx *ctx, float *terms);

/* Copy the smoothed FP32 volume J (nx*ny*nz) to `out` (host, or device when on_device = 1). */
snk_status snk_read_volume(snk_ctx *ctx, float *out, int on_device);

/* Kernel timings of the last calls, from HIP events recorded around each launch on the
 * context's stream (synchronises). evolved = contour-iterations run by the last snk_evolve;
 * vertex-updates = evolved * n_rays. */
typedef struct snk_timing {
    double prepass_ms;
    double evolve_ms;
    double finalize_ms;
    int64_t evolved;
    int64_t evolve_launches;
    /* shape of the last evolve launch as resolved from snk_set_launch / snk_set_tile (the automatic
     * shape depends on the contour count, so a contour's FP32 summation order can too) */
    int32_t lanes_per_contour, pairs_in_flight, layout, tile_voxels;
} snk_timing;
snk_status snk_get_timing(snk_ctx *ctx, snk_timing *t);

/* ------------------------------------------------------------------------------------------
 * Engine: many volumes in one launch (batched) and a request loop (served).
 *
 * A job is one volume with its seeds, parameters, direction table and iteration target. Jobs are
 * queued by snk_engine_submit and admitted in FIFO order while their device footprint (raw copy,
 * FP32 volume and its quad copy, contour state, scratch) fits the HBM budget given at creation. Every job of one
 * engine has the same dim; every engine volume must fit the quad layout (16 * nx*ny*nz below 2 GiB,
 * ny, nz <= 65535). Contours evolve exactly as
 * in snk_evolve (Sec. II-D: independent contours), so a job's results do not depend on which other
 * jobs share its launches.
 * ------------------------------------------------------------------------------------------ */
typedef struct snk_engine snk_engine;

typedef struct snk_engine_stats {
    int64_t submitted, admitted, completed, pending, running;
    uint64_t bytes_in_use, budget;
    double last_ms;           /* snk_engine_run: the captured graph's duration (HIP events)      */
    double last_evolve_ms;    /* snk_engine_step: the evolve launches of the step (HIP events)   */
    int64_t last_evolved;     /* contour-iterations run by the last run / step                   */
    int32_t lanes_per_contour, pairs_in_flight, persistent, layout;   /* last evolve launch's shape */
    int32_t graph_replays;
} snk_engine_stats;

/* Create an engine on `device` enqueuing on `hip_stream` (NULL: a private stream). */
snk_status snk_engine_create(snk_engine **out, int device, void *hip_stream, uint64_t hbm_budget_bytes);
snk_status snk_engine_destroy(snk_engine *e);
const char *snk_engine_last_error(const snk_engine *e);

/* Force the evolve launch shape (lanes per contour 64/128/256, pair-points in flight 1/2,
 * persistent 0/1, layout 0 = column pairs / 1 = plain / 2 = quad), or lanes = 0 to pick lanes, pair-points
 * and persistence per launch class (dim, D, M, L) by timing short trials of every shape. */
snk_status snk_engine_set_launch(snk_engine *e, int32_t lanes_per_contour, int32_t pairs_in_flight,
                                 int32_t persistent, int32_t layout);

/* Gather tile and residency of the shape forced by snk_engine_set_launch (SNK_ESTATE if none is
 * forced): each workgroup stages its contour's sample ball in an LDS box of tile_voxels FP32 voxels
 * (0: none; at most 16384, and the workgroup's LDS must stay within 64 KiB, else SNK_EINVAL at the
 * next run or step), re-staged when the ball leaves it, as snk_set_tile does for a context; a
 * persistent launch keeps workgroups_per_cu workgroups per CU (0: as many as registers and LDS
 * allow). Results are identical with and without a box. The autotuner searches both knobs itself. */
snk_status snk_engine_set_tile(snk_engine *e, int32_t tile_voxels, int32_t workgroups_per_cu);

/* Queue a job (arguments as in snk_set_params / snk_set_directions / snk_load_volume /
 * snk_load_seeds; host data is copied, a device volume with on_device = 1 is borrowed until the job
 * completes). n_iter is the job's iteration target. SNK_EBUSY if the job alone exceeds the budget. */
snk_status snk_engine_submit(snk_engine *e, const snk_params *params, const float *dirs, int32_t D,
                             const void *vol, snk_dtype dtype, int64_t nx, int64_t ny, int64_t nz, int on_device,
                             const double *centers, const float *r0, const uint32_t *ids, int64_t n,
                             int32_t n_iter, uint64_t *job);

/* Batched: admit what fits, then evolve every admitted job from its seeds to its target and
 * finalise it (exact energy + selection) in one captured hipGraph, replayed while the job set is
 * unchanged. Synchronises; results are then readable with snk_engine_read. */
snk_status snk_engine_run(snk_engine *e);

/* Served: admit what fits (pre-pass on admission), advance every running contour by up to `chunk`
 * iterations in one launch per launch class, then finalise the jobs whose contours have all stopped,
 * copy their results to the host and return their device memory to the budget. Synchronises.
 * *n_finished (may be NULL) receives the number of jobs completed by this step. */
snk_status snk_engine_step(snk_engine *e, int32_t chunk, int32_t *n_finished);

/* Ids of jobs completed since the last poll (up to cap). */
snk_status snk_engine_poll(snk_engine *e, uint64_t *done, int64_t cap, int64_t *n_done);

/* Results of a completed job (same outputs and capacity rule as snk_read). */
snk_status snk_engine_read(snk_engine *e, uint64_t job, float *radii, double *centers, float *e_mc, float *e_vox,
                           int32_t *iters, uint8_t *status, uint8_t *keep, int64_t cap, int64_t *n_out);

/* Host timestamps (milliseconds, steady clock) of a job's submission and completion. */
snk_status snk_engine_job_times(snk_engine *e, uint64_t job, double *submit_ms, double *done_ms);

/* Forget a job (frees its device memory if still held). */
snk_status snk_engine_release(snk_engine *e, uint64_t job);

snk_status snk_engine_get_stats(snk_engine *e, snk_engine_stats *s);

/* The launch shape the autotuner picked for each launch class so far (rows in class order, a class
 * being (dim, n_dirs, n_rays, n_radial)), SNK_TUNED_W int32 per row:
 *   dim, D, M, L, lanes per contour, pair-points in flight, persistent (0: one workgroup per
 *   contour, 1: a work queue), workgroups per CU of a persistent launch (0: as many as registers and
 *   LDS allow), LDS box capacity in voxels (0: none), the winning trial's time in microseconds, the
 *   number of shapes timed.
 * rows may be NULL (only *n_out, the class count, is written); SNK_ERANGE if cap < the class count.
 * Classes with a forced shape (snk_engine_set_launch) are not tuned and not listed. */
#define SNK_TUNED_W 11
snk_status snk_engine_tuned_shapes(snk_engine *e, int32_t *rows, int64_t cap, int64_t *n_out);

/* Wait for all work enqueued on the context's stream. */
snk_status snk_sync(snk_ctx *ctx);

/* Message of the last failed call on this context ("" if none). NULL ctx: last create error. */
const char *snk_last_error(const snk_ctx *ctx);

/* Library version string. */
const char *snk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SNK_H */
