/*
 * snk_oracle.c -- plain, slow, FP64 CPU oracle of 3D (and 2D) snakuscule evolution.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call this file: it is
 * used by the test suite, by the smoke check and by the CPU-baseline leg of the benchmark. It
 * shares no source with the HIP library (its own Philox, Gaussian, interpolation, weight
 * function, estimator, update and selection); only the synthetic inputs are common.
 *
 * What it computes, in the paper's order (arXiv 1804.06304, "Three-Dimensional GPU-Accelerated
 * Active Contours for Automated Localization of Cells in Large Images"):
 *   - pre-pass: affine intensity map, then a normalised separable Gaussian low-pass
 *     (Sec. II-E, the low-pass filter that makes Monte-Carlo integration well behaved;
 *     Results: images resampled to isotropic pixels -- here the spacing h enters the sampler);
 *   - the discrete energy E(p,q) = ||p - q||^-d * sum_k S(|k - c|) I(k) of Eq. (5)/(6), with the
 *     four-region weight S of Sec. II-B (inner core -1, ramp of width dr = rho*dR, shell +1,
 *     outer ramp of width dR) and rho = 2^(-1/d) (Sec. II-A for d = 2, Sec. II-B for d = 3);
 *   - its gradient in the identifier points p, q (Eqs. (7)-(11)) and the descent step
 *     p <- p - eps dE/dp, q <- q - eps dE/dq with eps = eps0/sqrt(n) (Eqs. (12)-(15)); the same
 *     gradient is also formed in (c, R) coordinates and the two are checked against each other;
 *   - the sums are Monte-Carlo estimates from points uniform in the ball of radius R + dR/2
 *     (Sec. II-E), drawn as randomly rotated table directions in antithetic pairs with
 *     r^d-stratified radial points (one reading of the unspecified sampling pattern);
 *   - optionally (flags bit 1) the same sums taken exactly over every lattice point of the ball of
 *     radius R + dR/2, i.e. the gradient of the discrete energy of Eq. (5) itself, the full
 *     voxel-sum evolution the paper compares its Monte-Carlo estimate with (Sec. II-E);
 *   - optionally (flags bit 2) the centre force in its image-gradient form: with the sample
 *     offsets y = x - c held fixed, E = (2R)^-d * integral S(|y|) I(c + y) dy, so
 *     dE/dc = (2R)^-d * integral S(|y|) grad I(c + y) dy, estimated from the same samples with the
 *     gradient of the trilinear interpolant (zero along axes clamped at the faces). It has the
 *     same expectation as the weight-derivative form of Eqs. (7)-(10) (a variance-reduction
 *     option, not in the paper); the radius force is unchanged;
 *   - star-shaped contours (not in the paper: a builder-defined extension whose radius varies with
 *     the table direction, with a smoothing energy over the direction graph; it reduces to the
 *     sphere when the radii are tied; see the block before orc_star_tables);
 *   - stopping on maximum iterations or convergence, overlap competition with the lower energy
 *     surviving (||c' - c''|| < max(R', R'')*rho), and the energy threshold E0 (Results).
 *
 * Parity pins (see the tests): Philox known-answer vectors; the weight function's zero-mean
 * identity (Sec. II-B); the ideal-blob energy of Eq. (3) and the alpha = d symmetric-slope
 * normalisation of Eq. (4); finite differences of the same-sample estimator against Eqs. (7)-(11);
 * the p,q <-> c,R identity; Monte-Carlo unbiasedness against quadrature; the pre-pass against a
 * library Gaussian filter; exact energy against a brute-force sum; greedy selection on
 * hand-built cases; whole runs settling at the argmin of an independent quadrature of the
 * continuous energy (ball, anisotropic ellipsoid, disk). A single stream's exact trajectory is
 * fixed only by these pieces.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -fPIC -shared snk_oracle.c -o libsnk_oracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_ACTIVE 0
#define ORC_CONVERGED 1
#define ORC_MAXITER 2
#define ORC_OUT 3
#define ORC_NONFINITE 4
#define ORC_CULLED 5       /* retired by a culling pass during evolution */
#define ORC_CLAMPED 0x10

#define ORC_TRACE_W 32
/* Samples within ORC_KINK_REL * s_max of a kink of S are flagged (reading R20): the FP32 kernels
 * place a radial point relative to a kink with an error below about 3.2e-7 * s_max (cube root on the
 * transcendental unit to ~2e-7 relative, one rounding each of s_max and rho * R, a fused offset), so
 * 1.5e-6 leaves a margin near 5. Samples within ORC_FACE_REL * s_max / h_a of a voxel face (the
 * image-gradient centre force) get the wider band, since their position also carries the FP32
 * rotation of the ray direction. */
#define ORC_KINK_REL 1.5e-6
#define ORC_FACE_REL 4e-6
#define ORC_FLAG_NOROT 1   /* flags bit 0: rotation Q = I */
#define ORC_FLAG_EXACT 2   /* flags bit 1: exact lattice sums instead of Monte-Carlo samples */
#define ORC_FLAG_GRADI 4   /* flags bit 2: centre force from the image gradient (Monte-Carlo only) */

static const double ORC_PI = 3.14159265358979323846;

typedef struct {
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
} orc_params;

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3",   */
/* SC'11): ten rounds of two 32x32->64 multiplies with a Weyl-sequence key schedule.           */
/* ------------------------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform on (0,1): (2*(x >> 9) + 1) * 2^-24, exactly representable in FP32 and FP64. */
double orc_uniform(uint32_t x)
{
    return (2.0 * (double)(x >> 9) + 1.0) * 5.9604644775390625e-08; /* 2^-24 */
}

static void philox_at(const orc_params *p, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                      uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------------------------ */
/* geometry constants                                                                         */
/* ------------------------------------------------------------------------------------------ */

/* rho = 2^(-1/d): inner and outer regions of equal measure (Sec. II-A, Sec. II-B). */
static double rho_of(int dim) { return dim == 3 ? pow(2.0, -1.0 / 3.0) : pow(2.0, -0.5); }

/* volume of the unit d-ball */
static double ball_measure(int dim) { return dim == 3 ? 4.0 * ORC_PI / 3.0 : ORC_PI; }

/* Smallest R for which the four regions of S do not overlap: rho R + dr/2 <= R - dR/2. */
double orc_r_geom_min(int dim, double dR)
{
    double rho = rho_of(dim);
    return dR * (1.0 + rho) / (2.0 * (1.0 - rho));
}

static double r_low(const orc_params *p)
{
    double g = orc_r_geom_min(p->dim, p->dR);
    return p->r_min > g ? p->r_min : g;
}

/* ------------------------------------------------------------------------------------------ */
/* Weight function S(r; R) of Eq. (5): four regions -- dynamic inner core (-1), fixed-width     */
/* ramp dr = rho*dR about rho*R, dynamic shell (+1), fixed-width outer ramp dR about R down to  */
/* zero at R + dR/2. Out: S, dS/dr, dS/dR. Half-open intervals: at a kink the right interval.  */
/* ------------------------------------------------------------------------------------------ */
void orc_weight(int dim, double r, double R, double dR, double out[3])
{
    double rho = rho_of(dim);
    double a = rho * R;
    double dr = rho * dR;
    double S, Sr, SR;
    if (r < a - 0.5 * dr) {
        S = -1.0; Sr = 0.0; SR = 0.0;
    } else if (r < a + 0.5 * dr) {
        S = 2.0 * (r - a) / dr; Sr = 2.0 / dr; SR = -2.0 * rho / dr;
    } else if (r < R - 0.5 * dR) {
        S = 1.0; Sr = 0.0; SR = 0.0;
    } else if (r < R + 0.5 * dR) {
        S = 0.5 - (r - R) / dR; Sr = -1.0 / dR; SR = 1.0 / dR;
    } else {
        S = 0.0; Sr = 0.0; SR = 0.0;
    }
    out[0] = S; out[1] = Sr; out[2] = SR;
}

/* S, dS/dr, dS/dR at n radii (out: n x 3). */
void orc_weight_many(int dim, const double *r, int64_t n, double R, double dR, double *out)
{
    for (int64_t i = 0; i < n; ++i) orc_weight(dim, r[i], R, dR, &out[i * 3]);
}

/* ------------------------------------------------------------------------------------------ */
/* pre-pass: J = (raw - i_offset) * i_scale, then a normalised separable Gaussian per axis with */
/* sigma_a = sigma_pre / h_a and taps |k| <= ceil(3 sigma_a), clamp-to-edge (Sec. II-E).        */
/* dtype: 0 = uint8, 1 = uint16, 2 = float32.                                                  */
/* ------------------------------------------------------------------------------------------ */
static double raw_at(const void *raw, int dtype, int64_t i)
{
    if (dtype == 0) return (double)((const uint8_t *)raw)[i];
    if (dtype == 1) return (double)((const uint16_t *)raw)[i];
    return (double)((const float *)raw)[i];
}

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

static void gauss_axis(double *J, int64_t nx, int64_t ny, int64_t nz, int axis, double sigma)
{
    if (!(sigma > 0.0)) return;
    int64_t n_axis = axis == 0 ? nx : (axis == 1 ? ny : nz);
    if (n_axis < 2) return;
    int rad = (int)ceil(3.0 * sigma);
    double *g = (double *)malloc(sizeof(double) * (2 * rad + 1));
    double sum = 0.0;
    for (int k = -rad; k <= rad; ++k) {
        g[k + rad] = exp(-(double)k * (double)k / (2.0 * sigma * sigma));
        sum += g[k + rad];
    }
    for (int k = 0; k < 2 * rad + 1; ++k) g[k] /= sum;
    int64_t stride = axis == 0 ? 1 : (axis == 1 ? nx : nx * ny);
    int64_t n_lines = nx * ny * nz / n_axis;
#pragma omp parallel
    {
        double *line = (double *)malloc(sizeof(double) * n_axis);
#pragma omp for schedule(static)
        for (int64_t li = 0; li < n_lines; ++li) {
            int64_t base;
            if (axis == 0) base = li * nx;
            else if (axis == 1) base = (li / nx) * nx * ny + (li % nx);
            else base = li;
            for (int64_t t = 0; t < n_axis; ++t) line[t] = J[base + t * stride];
            for (int64_t t = 0; t < n_axis; ++t) {
                double acc = 0.0;
                for (int k = -rad; k <= rad; ++k) acc += g[k + rad] * line[clampi(t + k, 0, n_axis - 1)];
                J[base + t * stride] = acc;
            }
        }
        free(line);
    }
    free(g);
}

int orc_prepass(const void *raw, int dtype, int64_t nx, int64_t ny, int64_t nz, const orc_params *p,
                double *J)
{
    int64_t n = nx * ny * nz;
    for (int64_t i = 0; i < n; ++i) J[i] = (raw_at(raw, dtype, i) - p->i_offset) * p->i_scale;
    if (p->sigma_pre > 0.0) {
        gauss_axis(J, nx, ny, nz, 0, p->sigma_pre / p->spacing[0]);
        gauss_axis(J, nx, ny, nz, 1, p->sigma_pre / p->spacing[1]);
        if (p->dim == 3) gauss_axis(J, nx, ny, nz, 2, p->sigma_pre / p->spacing[2]);
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Image value at a non-integer voxel coordinate v: trilinear (bilinear in 2D) interpolation    */
/* with voxel centres at integer coordinates and the coordinate clamped to [0, n_a - 1].       */
/* ------------------------------------------------------------------------------------------ */
static void split_coord(double v, int64_t n, int64_t *i0, int64_t *i1, double *f)
{
    if (n == 1) { *i0 = 0; *i1 = 0; *f = 0.0; return; }
    if (v < 0.0) v = 0.0;
    if (v > (double)(n - 1)) v = (double)(n - 1);
    double fl = floor(v);
    int64_t i = (int64_t)fl;
    if (i > n - 2) i = n - 2;
    *i0 = i; *i1 = i + 1; *f = v - (double)i;
}

double orc_interp(const double *J, int64_t nx, int64_t ny, int64_t nz, int dim, double vx, double vy,
                  double vz)
{
    int64_t x0, x1, y0, y1, z0, z1;
    double fx, fy, fz;
    split_coord(vx, nx, &x0, &x1, &fx);
    split_coord(vy, ny, &y0, &y1, &fy);
    if (dim == 2) { z0 = z1 = 0; fz = 0.0; }
    else split_coord(vz, nz, &z0, &z1, &fz);
    double acc = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? fx : 1.0 - fx) * (dy ? fy : 1.0 - fy) * (dz ? fz : 1.0 - fz);
                if (w == 0.0) continue;
                int64_t xi = dx ? x1 : x0, yi = dy ? y1 : y0, zi = dz ? z1 : z0;
                acc += w * J[(zi * ny + yi) * nx + xi];
            }
    return acc;
}

/* Trilinear (bilinear) value and its gradient with respect to the voxel coordinates, in the cell
 * the value is interpolated from; an axis whose coordinate lies outside [0, n - 1] (clamped to the
 * face) has zero derivative. */
double orc_interp_grad(const double *J, int64_t nx, int64_t ny, int64_t nz, int dim, double vx, double vy,
                       double vz, double g[3])
{
    const double v[3] = {vx, vy, vz};
    const int64_t n[3] = {nx, ny, nz};
    int64_t i0[3], i1[3];
    double f[3];
    int inside[3];
    for (int a = 0; a < 3; ++a) {
        if (a >= dim) { i0[a] = i1[a] = 0; f[a] = 0.0; inside[a] = 0; continue; }
        split_coord(v[a], n[a], &i0[a], &i1[a], &f[a]);
        inside[a] = n[a] > 1 && v[a] >= 0.0 && v[a] <= (double)(n[a] - 1);
    }
    double acc = 0.0;
    g[0] = g[1] = g[2] = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                if (dim == 2 && dz) continue;
                const int d[3] = {dx, dy, dz};
                double w[3];
                for (int a = 0; a < 3; ++a) w[a] = a >= dim ? 1.0 : (d[a] ? f[a] : 1.0 - f[a]);
                int64_t xi = dx ? i1[0] : i0[0], yi = dy ? i1[1] : i0[1], zi = dz ? i1[2] : i0[2];
                const double Jc = J[(zi * ny + yi) * nx + xi];
                acc += w[0] * w[1] * w[2] * Jc;
                for (int a = 0; a < dim; ++a) {
                    /* derivative of the corner's weight along axis a: +1 or -1 times the others */
                    double dw = d[a] ? 1.0 : -1.0;
                    for (int b = 0; b < 3; ++b)
                        if (b != a) dw *= w[b];
                    g[a] += dw * Jc;
                }
            }
    for (int a = 0; a < dim; ++a)
        if (!inside[a]) g[a] = 0.0;
    return acc;
}

/* ------------------------------------------------------------------------------------------ */
/* Random rotation of the direction table for (contour id, iteration n): Philox with counter    */
/* (0, n, id, 0). 3D: Shoemake's uniform unit quaternion (Graphics Gems III, 1992) from three   */
/* uniforms; 2D: angle 2*pi*U. Q is row-major and acts on column vectors. flags bit 0: Q = I.   */
/* ------------------------------------------------------------------------------------------ */
void orc_rotation(const orc_params *p, uint32_t n, uint32_t id, double Q[9])
{
    for (int i = 0; i < 9; ++i) Q[i] = (i % 4 == 0) ? 1.0 : 0.0;
    if (p->flags & ORC_FLAG_NOROT) return;
    uint32_t x[4];
    philox_at(p, 0u, n, id, 0u, x);
    if (p->dim == 2) {
        double th = 2.0 * ORC_PI * orc_uniform(x[0]);
        Q[0] = cos(th); Q[1] = -sin(th);
        Q[3] = sin(th); Q[4] = cos(th);
        return;
    }
    double u1 = orc_uniform(x[0]), u2 = orc_uniform(x[1]), u3 = orc_uniform(x[2]);
    double a = sqrt(1.0 - u1), b = sqrt(u1);
    double t1 = 2.0 * ORC_PI * u2, t2 = 2.0 * ORC_PI * u3;
    double qx = a * sin(t1), qy = a * cos(t1), qz = b * sin(t2), qw = b * cos(t2);
    Q[0] = 1.0 - 2.0 * (qy * qy + qz * qz); Q[1] = 2.0 * (qx * qy - qw * qz); Q[2] = 2.0 * (qx * qz + qw * qy);
    Q[3] = 2.0 * (qx * qy + qw * qz); Q[4] = 1.0 - 2.0 * (qx * qx + qz * qz); Q[5] = 2.0 * (qy * qz - qw * qx);
    Q[6] = 2.0 * (qx * qz - qw * qy); Q[7] = 2.0 * (qy * qz + qw * qx); Q[8] = 1.0 - 2.0 * (qx * qx + qy * qy);
}

/* ------------------------------------------------------------------------------------------ */
/* The sample set of one contour-iteration (Sec. II-E): M rays in M/2 antithetic pairs; pair m  */
/* draws Philox(m, n, id, 1) -> table index k = floor(x0 * D / 2^32) and jitter xi = U(x1); ray  */
/* direction u = Q T[k] (and -u for its partner); radial point l sits at                        */
/* s = s_max * ((l + xi) / L)^(1/d), s_max = R + dR/2. Every point is marginally uniform in the  */
/* ball, so (V/N) * sum f estimates the integral of f over it.                                  */
/* Callback receives (position offset s*u', direction u', radius s).                            */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    const double *J;
    int64_t nx, ny, nz;
    const orc_params *p;
    const double *dirs;
} orc_vol;

typedef struct {
    /* c,R-form sums (unscaled) */
    double A, BR, Bc[3];
    double Aabs, BRabs, Bcabs[3];
    /* p,q-form sums: sum dS/dp_a * I and sum dS/dq_a * I */
    double Sp[3], Sq[3];
    /* kink slack (unscaled) */
    double slBR, slBc[3];
    int n_kink;
    int n_samples;
} orc_sums;

static void accumulate_samples(const orc_vol *vol, const double c[3], double R, uint32_t n, uint32_t id,
                               orc_sums *sm, double *pts, double *vals)
{
    const orc_params *p = vol->p;
    int dim = p->dim;
    double Q[9];
    orc_rotation(p, n, id, Q);
    double smax = R + 0.5 * p->dR;
    double rho = rho_of(dim);
    double a = rho * R, dr = rho * p->dR;
    double kinks[4] = {a - 0.5 * dr, a + 0.5 * dr, R - 0.5 * p->dR, R + 0.5 * p->dR};
    int M = p->n_rays, L = p->n_radial;
    const int gradi = (p->flags & ORC_FLAG_GRADI) != 0;
    memset(sm, 0, sizeof(*sm));
    int idx = 0;
    for (int m = 0; m < M / 2; ++m) {
        uint32_t x[4];
        philox_at(p, (uint32_t)m, n, id, 1u, x);
        uint32_t k = (uint32_t)(((uint64_t)x[0] * (uint64_t)(uint32_t)p->n_dirs) >> 32);
        double xi = orc_uniform(x[1]);
        double t[3] = {0.0, 0.0, 0.0}, u[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < dim; ++i) t[i] = vol->dirs[(int64_t)k * dim + i];
        for (int i = 0; i < dim; ++i) {
            double acc = 0.0;
            for (int j = 0; j < dim; ++j) acc += Q[i * 3 + j] * t[j];
            u[i] = acc;
        }
        for (int sgn = 0; sgn < 2; ++sgn) {
            double us[3];
            for (int i = 0; i < 3; ++i) us[i] = sgn ? -u[i] : u[i];
            for (int l = 0; l < L; ++l) {
                double tau = ((double)l + xi) / (double)L;
                double s = smax * (dim == 3 ? cbrt(tau) : sqrt(tau));
                double pos[3];
                for (int i = 0; i < 3; ++i) pos[i] = c[i] + s * us[i];
                const double vv[3] = {pos[0] / p->spacing[0], pos[1] / p->spacing[1],
                                      dim == 3 ? pos[2] / p->spacing[2] : 0.0};
                double I, gI[3] = {0.0, 0.0, 0.0};
                if (gradi) {
                    double gv[3];
                    I = orc_interp_grad(vol->J, vol->nx, vol->ny, vol->nz, dim, vv[0], vv[1], vv[2], gv);
                    for (int i = 0; i < dim; ++i) gI[i] = gv[i] / p->spacing[i];  /* physical gradient */
                } else {
                    I = orc_interp(vol->J, vol->nx, vol->ny, vol->nz, dim, vv[0], vv[1], vv[2]);
                }
                double w[3];
                orc_weight(dim, s, R, p->dR, w);
                double S = w[0], Sr = w[1], SR = w[2];
                sm->A += S * I;
                sm->Aabs += fabs(S * I);
                sm->BR += SR * I;
                sm->BRabs += fabs(SR * I);
                /* derivative of the integrand with respect to c_a: -Sr u_a I (weight form, the
                 * sample points fixed), or S dI/dx_a (gradient form, the offsets fixed) */
                double dc_int[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < dim; ++i) dc_int[i] = gradi ? S * gI[i] : -Sr * I * us[i];
                for (int i = 0; i < dim; ++i) {
                    sm->Bc[i] += dc_int[i];
                    sm->Bcabs[i] += fabs(dc_int[i]);
                }
                /* Eqs. (7)-(10): c = (p+q)/2, R = (q_x - p_x)/2 along x (Eq. (6)), so
                 * d/dp_a = (d/dc_a) / 2 - [a == x] (d/dR) / 2 and d/dq_a = (d/dc_a) / 2 + [a == x] (d/dR) / 2;
                 * in the weight form dr/dc = -u gives dS/dp_a = -Sr u_a / 2 - SR [a == x] / 2. */
                for (int i = 0; i < dim; ++i) {
                    sm->Sp[i] += 0.5 * dc_int[i] - (i == 0 ? 0.5 * SR * I : 0.0);
                    sm->Sq[i] += 0.5 * dc_int[i] + (i == 0 ? 0.5 * SR * I : 0.0);
                }
                /* gradient form: the normal derivative of the interpolant jumps across voxel faces
                 * (and at the volume's faces); record the jump for samples an FP32 evaluation may
                 * place in the neighbouring cell */
                if (gradi) {
                    for (int a = 0; a < dim; ++a) {
                        const double tol = ORC_FACE_REL * smax / p->spacing[a];
                        if (fabs(vv[a] - nearbyint(vv[a])) <= tol) {
                            double vl[3] = {vv[0], vv[1], vv[2]}, vr[3] = {vv[0], vv[1], vv[2]}, gl[3], gr[3];
                            vl[a] = nearbyint(vv[a]) - 1e-9;
                            vr[a] = nearbyint(vv[a]) + 1e-9;
                            orc_interp_grad(vol->J, vol->nx, vol->ny, vol->nz, dim, vl[0], vl[1], vl[2], gl);
                            orc_interp_grad(vol->J, vol->nx, vol->ny, vol->nz, dim, vr[0], vr[1], vr[2], gr);
                            sm->slBc[a] += fabs(S * (gr[a] - gl[a]) / p->spacing[a]);
                            sm->n_kink += 1;
                        }
                    }
                }
                /* samples within ORC_KINK_REL * s_max of a kink of S: an FP32 evaluation may place
                 * them on the other side; record how much dS/dr and dS/dR could change. */
                for (int kk = 0; kk < 4; ++kk) {
                    if (fabs(s - kinks[kk]) <= ORC_KINK_REL * smax) {
                        double wl[3], wr[3];
                        orc_weight(dim, kinks[kk] - 1e-9 * smax, R, p->dR, wl);
                        orc_weight(dim, kinks[kk] + 1e-9 * smax, R, p->dR, wr);
                        sm->slBR += fabs((wr[2] - wl[2]) * I);
                        if (!gradi)
                            for (int i = 0; i < dim; ++i) sm->slBc[i] += fabs((wr[1] - wl[1]) * I * us[i]);
                        sm->n_kink += 1;
                    }
                }
                if (pts) {
                    for (int i = 0; i < 3; ++i) pts[idx * 3 + i] = pos[i];
                    vals[idx] = I;
                }
                ++idx;
            }
        }
    }
    sm->n_samples = idx;
}

/* Adds one point's terms: weight, derivatives, p,q-form derivatives, magnitudes and kink slack.
 * u: unit vector from the centre to the point (zero at the centre), r its distance. */
static void add_point(const orc_params *p, double r, const double u[3], double I, double R, const double kinks[4],
                      double smax, orc_sums *sm)
{
    int dim = p->dim;
    double w[3];
    orc_weight(dim, r, R, p->dR, w);
    double S = w[0], Sr = w[1], SR = w[2];
    sm->A += S * I;
    sm->Aabs += fabs(S * I);
    sm->BR += SR * I;
    sm->BRabs += fabs(SR * I);
    for (int i = 0; i < dim; ++i) {
        sm->Bc[i] += -Sr * I * u[i];
        sm->Bcabs[i] += fabs(Sr * I * u[i]);
    }
    for (int i = 0; i < dim; ++i) {
        sm->Sp[i] += (-0.5 * Sr * u[i] - (i == 0 ? 0.5 * SR : 0.0)) * I;
        sm->Sq[i] += (-0.5 * Sr * u[i] + (i == 0 ? 0.5 * SR : 0.0)) * I;
    }
    for (int kk = 0; kk < 4; ++kk) {
        if (fabs(r - kinks[kk]) <= ORC_KINK_REL * smax) {
            double wl[3], wr[3];
            orc_weight(dim, kinks[kk] - 1e-9 * smax, R, p->dR, wl);
            orc_weight(dim, kinks[kk] + 1e-9 * smax, R, p->dR, wr);
            sm->slBR += fabs((wr[2] - wl[2]) * I);
            for (int i = 0; i < dim; ++i) sm->slBc[i] += fabs((wr[1] - wl[1]) * I * u[i]);
            sm->n_kink += 1;
        }
    }
}

/* Exact sums (flags bit 1): every lattice point k with |k h - c| < R + dR/2, the point set of
 * Eq. (5), with I(k) = J(k) (clamp-to-edge outside the volume). Multiplied by the voxel measure
 * they are the terms of the exact discrete energy's gradient (the lattice held fixed). */
static void accumulate_lattice(const orc_vol *vol, const double c[3], double R, orc_sums *sm)
{
    const orc_params *p = vol->p;
    int dim = p->dim;
    double smax = R + 0.5 * p->dR;
    double rho = rho_of(dim);
    double a = rho * R, dr = rho * p->dR;
    double kinks[4] = {a - 0.5 * dr, a + 0.5 * dr, R - 0.5 * p->dR, R + 0.5 * p->dR};
    memset(sm, 0, sizeof(*sm));
    int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int i = 0; i < dim; ++i) {
        lo[i] = (int64_t)ceil((c[i] - smax) / p->spacing[i]);
        hi[i] = (int64_t)floor((c[i] + smax) / p->spacing[i]);
    }
    int count = 0;
    for (int64_t kz = lo[2]; kz <= hi[2]; ++kz)
        for (int64_t ky = lo[1]; ky <= hi[1]; ++ky)
            for (int64_t kx = lo[0]; kx <= hi[0]; ++kx) {
                double d[3] = {kx * p->spacing[0] - c[0], ky * p->spacing[1] - c[1],
                               dim == 3 ? kz * p->spacing[2] - c[2] : 0.0};
                double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                if (!(r < smax)) continue;
                double u[3] = {0.0, 0.0, 0.0};
                if (r > 0.0)
                    for (int i = 0; i < dim; ++i) u[i] = d[i] / r;
                double I = vol->J[(clampi(kz, 0, vol->nz - 1) * vol->ny + clampi(ky, 0, vol->ny - 1)) * vol->nx +
                                  clampi(kx, 0, vol->nx - 1)];
                add_point(p, r, u, I, R, kinks, smax, sm);
                ++count;
            }
    sm->n_samples = count;
}

static double voxel_measure(const orc_params *p)
{
    return p->spacing[0] * p->spacing[1] * (p->dim == 3 ? p->spacing[2] : 1.0);
}

/* Sums of one contour-iteration and their scale: exact lattice sums times the voxel measure, or
 * Monte-Carlo sums times V/N. */
static double contour_sums(const orc_vol *vol, const double c[3], double R, uint32_t n, uint32_t id, orc_sums *sm,
                           double *pts, double *vals)
{
    const orc_params *p = vol->p;
    if (p->flags & ORC_FLAG_EXACT) {
        accumulate_lattice(vol, c, R, sm);
        return voxel_measure(p);
    }
    accumulate_samples(vol, c, R, n, id, sm, pts, vals);
    double smax = R + 0.5 * p->dR;
    return ball_measure(p->dim) * pow(smax, p->dim) / (double)sm->n_samples;
}

/* ------------------------------------------------------------------------------------------ */
/* One gradient-descent iteration of one contour (Eqs. (7)-(15)).                               */
/* ------------------------------------------------------------------------------------------ */
/* Repulsion from neighbouring contours (not in the paper; the block before orc_evolve_repel):
 * gradient of the contour's penalty with respect to its centre and radius, and the sums of the
 * magnitudes of the terms (for tolerances). NULL: no repulsion. */
typedef struct {
    double gc[3], gR;
    double gc_abs[3], gR_abs;
} orc_repel;

static int step_contour_r(const orc_vol *vol, double c[3], double *R, int32_t *iter, uint8_t *status,
                          uint8_t *streak, double *e_mc, uint32_t id, double *trace, double *move_out,
                          const orc_repel *rep);

static int step_contour(const orc_vol *vol, double c[3], double *R, int32_t *iter, uint8_t *status,
                        uint8_t *streak, double *e_mc, uint32_t id, double *trace, double *move_out)
{
    return step_contour_r(vol, c, R, iter, status, streak, e_mc, id, trace, move_out, NULL);
}

static int step_contour_r(const orc_vol *vol, double c[3], double *R, int32_t *iter, uint8_t *status,
                          uint8_t *streak, double *e_mc, uint32_t id, double *trace, double *move_out,
                          const orc_repel *rep)
{
    const orc_params *p = vol->p;
    int dim = p->dim;
    int mismatch = 0;
    double Rc = *R;
    uint32_t n = (uint32_t)(*iter + 1);
    *iter = (int32_t)n;
    orc_sums sm;
    double scale = contour_sums(vol, c, Rc, n, id, &sm, NULL, NULL);
    double twoR_d = pow(2.0 * Rc, dim);
    double eps = p->eps0 / sqrt((double)n);

    /* c,R form */
    double A = scale * sm.A, BR = scale * sm.BR, Bc[3] = {0, 0, 0};
    for (int i = 0; i < dim; ++i) Bc[i] = scale * sm.Bc[i];
    double E = A / twoR_d;
    double gR = (BR - (double)dim / Rc * A) / twoR_d;
    double dR_step = -0.5 * eps * gR;
    double dc[3] = {0, 0, 0};
    for (int i = 0; i < dim; ++i) dc[i] = -0.5 * eps * Bc[i] / twoR_d;
    /* repulsion: its gradient joins the energy's, with the same step */
    if (rep) {
        dR_step += -0.5 * eps * rep->gR;
        for (int i = 0; i < dim; ++i) dc[i] += -0.5 * eps * rep->gc[i];
    }

    /* p,q form, literally: p = c - R e_x, q = c + R e_x (Eq. (6)), gamma = (q_x - p_x)^-d (Eq. (11)) */
    double pp[3], qq[3];
    for (int i = 0; i < 3; ++i) { pp[i] = c[i]; qq[i] = c[i]; }
    pp[0] -= Rc; qq[0] += Rc;
    double qmp = qq[0] - pp[0];
    double gamma = 1.0 / pow(qmp, dim);
    double dEdp[3] = {0, 0, 0}, dEdq[3] = {0, 0, 0};
    dEdp[0] = gamma * ((double)dim / qmp * A + scale * sm.Sp[0]);
    dEdq[0] = gamma * (-(double)dim / qmp * A + scale * sm.Sq[0]);
    for (int i = 1; i < dim; ++i) {
        dEdp[i] = gamma * scale * sm.Sp[i];
        dEdq[i] = gamma * scale * sm.Sq[i];
    }
    if (rep) {
        /* c = (p + q)/2, R = (q_x - p_x)/2: d/dp = dc/2 - dR/2 e_x, d/dq = dc/2 + dR/2 e_x */
        for (int i = 0; i < dim; ++i) {
            dEdp[i] += 0.5 * rep->gc[i];
            dEdq[i] += 0.5 * rep->gc[i];
        }
        dEdp[0] -= 0.5 * rep->gR;
        dEdq[0] += 0.5 * rep->gR;
    }
    double pn[3], qn[3];
    for (int i = 0; i < 3; ++i) { pn[i] = pp[i] - eps * dEdp[i]; qn[i] = qq[i] - eps * dEdq[i]; }
    double c_new[3], R_new = 0.5 * (qn[0] - pn[0]);
    for (int i = 0; i < 3; ++i) c_new[i] = 0.5 * (pn[i] + qn[i]);
    /* the two forms must agree */
    double tolR = 1e-9 * (fabs(Rc) + fabs(dR_step)) + 1e-12;
    if (fabs((R_new - Rc) - dR_step) > tolR) mismatch = 1;
    for (int i = 0; i < dim; ++i) {
        double tolc = 1e-9 * (fabs(c[i]) + fabs(dc[i]) + 1.0);
        if (fabs((c_new[i] - c[i]) - dc[i]) > tolc) mismatch = 1;
        if (i > 0 && dEdp[i] != dEdq[i]) mismatch = 1; /* Eqs. (9)-(10): p, q stay aligned */
    }

    if (trace) {
        double Aabs = scale * sm.Aabs, BRabs = scale * sm.BRabs;
        trace[0] = A; trace[1] = BR;
        for (int i = 0; i < 3; ++i) trace[2 + i] = Bc[i];
        trace[5] = Aabs; trace[6] = BRabs;
        for (int i = 0; i < 3; ++i) trace[7 + i] = scale * sm.Bcabs[i];
        trace[10] = E; trace[11] = Aabs / twoR_d;
        trace[12] = dR_step; trace[13] = 0.5 * eps * (BRabs + (double)dim / Rc * Aabs) / twoR_d;
        for (int i = 0; i < 3; ++i) {
            trace[14 + i] = dc[i];
            trace[17 + i] = 0.5 * eps * scale * sm.Bcabs[i] / twoR_d;
        }
        if (rep) {
            trace[13] += 0.5 * eps * rep->gR_abs;
            for (int i = 0; i < dim; ++i) trace[17 + i] += 0.5 * eps * rep->gc_abs[i];
        }
        trace[20] = scale * sm.slBR;
        for (int i = 0; i < 3; ++i) trace[21 + i] = scale * sm.slBc[i];
        trace[24] = 0.5 * eps * scale * sm.slBR / twoR_d;
        for (int i = 0; i < 3; ++i) trace[25 + i] = 0.5 * eps * scale * sm.slBc[i] / twoR_d;
        trace[28] = (double)sm.n_kink;
        trace[29] = (double)n;
        trace[30] = Rc;
        trace[31] = eps;
    }

    /* radius bounds (minimum contour size, Conclusion) */
    double lo = r_low(p), hi = p->r_max;
    uint8_t flag = *status & ORC_CLAMPED;
    if (R_new < lo) { R_new = lo; flag = ORC_CLAMPED; }
    if (R_new > hi) { R_new = hi; flag = ORC_CLAMPED; }
    double move = fabs(R_new - Rc);
    double dcn = 0.0;
    for (int i = 0; i < dim; ++i) dcn += (c_new[i] - c[i]) * (c_new[i] - c[i]);
    dcn = sqrt(dcn);
    if (dcn > move) move = dcn;
    if (move_out) *move_out = move;

    for (int i = 0; i < 3; ++i) c[i] = c_new[i];
    *R = R_new;
    *e_mc = E;
    uint8_t st = ORC_ACTIVE;
    int finite = isfinite(R_new) && isfinite(E);
    for (int i = 0; i < dim; ++i) finite = finite && isfinite(c_new[i]);
    if (!finite) {
        st = ORC_NONFINITE;
    } else {
        for (int i = 0; i < dim; ++i) {
            int64_t na = i == 0 ? vol->nx : (i == 1 ? vol->ny : vol->nz);
            if (c_new[i] < 0.0 || c_new[i] > (double)(na - 1) * p->spacing[i]) st = ORC_OUT;
        }
    }
    if (st == ORC_ACTIVE) {
        if (move < p->conv_tol) *streak = (uint8_t)(*streak < 255 ? *streak + 1 : 255);
        else *streak = 0;
        if (p->conv_window > 0 && *streak >= p->conv_window) st = ORC_CONVERGED;
    }
    *status = (uint8_t)(st | flag);
    return mismatch;
}

/* ------------------------------------------------------------------------------------------ */
/* Soft repulsion between neighbouring contours (not in the paper: a builder-defined extension;  */
/* the paper's contours are independent during evolution, Sec. II-D, and compete only after it).  */
/* Neighbours are held at a snapshot (c_s, R_s) taken at the start of each chunk of iterations.   */
/* Contour i at (c, R) pays kappa * sum over the live snapshot contours j != i of w(t_ij),          */
/*   t_ij = |c - c_j| / (rho (R + R_j)),   w(t) = (1 - t)^2 for t < 1, else 0:                   */
/* its inner sphere (radius rho R, the cell estimate) and each neighbour's overlap exactly when  */
/* t < 1. With the neighbour fixed, dw/dc = -2 (1 - t) (c - c_j) / (|c - c_j| rho (R + R_j)) and   */
/* dw/dR = 2 (1 - t) t / (R + R_j); coincident centres give no centre force. The gradient joins the */
/* energy's in the descent step of Eqs. (12)-(15); kappa = 0 is the paper's contour exactly.      */
/* ------------------------------------------------------------------------------------------ */

/* The repulsion gradient of contour `self` at (c, R) from snapshot contours j in ascending order. */
static void repel_grad(const orc_params *p, int64_t n_s, const double *c_s, const double *R_s,
                       const uint8_t *live_s, int64_t self, const double c[3], double R, double kappa,
                       orc_repel *out)
{
    int dim = p->dim;
    double rho = rho_of(dim);
    memset(out, 0, sizeof(*out));
    for (int64_t j = 0; j < n_s; ++j) {
        if (j == self || !live_s[j]) continue;
        double dv[3] = {0, 0, 0}, d2 = 0.0;
        for (int a = 0; a < dim; ++a) {
            dv[a] = c[a] - c_s[j * 3 + a];
            d2 += dv[a] * dv[a];
        }
        double d = sqrt(d2), span = rho * (R + R_s[j]);
        double t = d / span;
        if (!(t < 1.0)) continue;
        double gR = kappa * 2.0 * (1.0 - t) * t / (R + R_s[j]);
        out->gR += gR;
        out->gR_abs += fabs(gR);
        if (d > 0.0) {
            for (int a = 0; a < dim; ++a) {
                double g = -kappa * 2.0 * (1.0 - t) * dv[a] / (d * span);
                out->gc[a] += g;
                out->gc_abs[a] += fabs(g);
            }
        }
    }
}

/* The penalty kappa * sum_j w(t_ij) of contour `self` at (c, R) (for finite-difference pins). */
double orc_repel_energy(const orc_params *p, int64_t n_s, const double *c_s, const double *R_s,
                        const uint8_t *live_s, int64_t self, const double *c, double R, double kappa)
{
    int dim = p->dim;
    double rho = rho_of(dim), e = 0.0;
    for (int64_t j = 0; j < n_s; ++j) {
        if (j == self || !live_s[j]) continue;
        double d2 = 0.0;
        for (int a = 0; a < dim; ++a) d2 += (c[a] - c_s[j * 3 + a]) * (c[a] - c_s[j * 3 + a]);
        double t = sqrt(d2) / (rho * (R + R_s[j]));
        if (t < 1.0) e += kappa * (1.0 - t) * (1.0 - t);
    }
    return e;
}

/* The repulsion gradient at (c, R) as orc_repel_grad computes it: gc[0..2], gR. */
void orc_repel_grad(const orc_params *p, int64_t n_s, const double *c_s, const double *R_s,
                    const uint8_t *live_s, int64_t self, const double *c, double R, double kappa, double *out4)
{
    orc_repel r;
    repel_grad(p, n_s, c_s, R_s, live_s, self, c, R, kappa, &r);
    for (int a = 0; a < 3; ++a) out4[a] = r.gc[a];
    out4[3] = r.gR;
}

/* Evolve every ACTIVE contour for up to n_iter further iterations with repulsion of strength kappa:
 * in chunks of `every` iterations, each starting from a snapshot of the centres, radii and live
 * flags (ACTIVE or CONVERGED) of all contours; within a chunk each contour steps against that
 * snapshot. trace as in orc_evolve (its step terms include the repulsion). Returns the number of
 * contour-iterations whose p,q and c,R forms disagreed (must be 0). */
int64_t orc_evolve_repel(const double *J, int64_t nx, int64_t ny, int64_t nz, const orc_params *p,
                         const double *dirs, int64_t n, const uint32_t *ids, double *c, double *R,
                         int32_t *iters, uint8_t *status, uint8_t *streak, double *e_mc, int32_t n_iter,
                         int32_t every, double kappa, double *trace, int64_t *evolved)
{
    orc_vol vol = {J, nx, ny, nz, p, dirs};
    int64_t mism = 0, done_all = 0;
    double *c_s = (double *)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    double *R_s = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    uint8_t *live_s = (uint8_t *)malloc(n > 0 ? n : 1);
    if (every < 1) every = 1;
    for (int32_t done = 0; done < n_iter;) {
        int32_t k = n_iter - done < every ? n_iter - done : every;
        for (int64_t i = 0; i < n; ++i) {
            for (int a = 0; a < 3; ++a) c_s[i * 3 + a] = c[i * 3 + a];
            R_s[i] = R[i];
            int st = status[i] & 0x0f;
            live_s[i] = (uint8_t)(st == ORC_ACTIVE || st == ORC_CONVERGED);
        }
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : mism, done_all)
        for (int64_t i = 0; i < n; ++i) {
            for (int32_t it = 0; it < k; ++it) {
                if ((status[i] & 0x0f) != ORC_ACTIVE) break;
                orc_repel rep;
                repel_grad(p, n, c_s, R_s, live_s, i, &c[i * 3], R[i], kappa, &rep);
                mism += step_contour_r(&vol, &c[i * 3], &R[i], &iters[i], &status[i], &streak[i], &e_mc[i],
                                       ids[i], trace ? &trace[i * ORC_TRACE_W] : NULL, NULL, &rep);
                ++done_all;
            }
        }
        done += k;
    }
    free(c_s);
    free(R_s);
    free(live_s);
    if (evolved) *evolved = done_all;
    return mism;
}

/* Clamp of the initial radius R0 into [max(r_min, geometric minimum), r_max]. */
double orc_initial_radius(const orc_params *p, double r0)
{
    double lo = r_low(p);
    if (r0 < lo) r0 = lo;
    if (r0 > p->r_max) r0 = p->r_max;
    return r0;
}

/* Evolve every ACTIVE contour for up to n_iter further iterations. c: n x 3 physical. trace (n x
 * ORC_TRACE_W, may be NULL) receives the terms of the last iteration each contour ran. moves (n x
 * n_iter, may be NULL) receives the move of every step this call ran, max(|R change|, |c change|),
 * the quantity the stop rule compares with conv_tol (steps not run are left untouched). Returns the
 * number of contour-iterations whose p,q and c,R forms disagreed (must be 0). */
int64_t orc_evolve_log(const double *J, int64_t nx, int64_t ny, int64_t nz, const orc_params *p,
                       const double *dirs, int64_t n, const uint32_t *ids, double *c, double *R,
                       int32_t *iters, uint8_t *status, uint8_t *streak, double *e_mc, int32_t n_iter,
                       double *trace, double *moves, int64_t *evolved)
{
    orc_vol vol = {J, nx, ny, nz, p, dirs};
    int64_t mism = 0, done = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : mism, done)
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t it = 0; it < n_iter; ++it) {
            if ((status[i] & 0x0f) != ORC_ACTIVE) break;
            mism += step_contour(&vol, &c[i * 3], &R[i], &iters[i], &status[i], &streak[i], &e_mc[i],
                                 ids[i], trace ? &trace[i * ORC_TRACE_W] : NULL,
                                 moves ? &moves[i * (int64_t)n_iter + it] : NULL);
            done += 1;
        }
    }
    if (evolved) *evolved = done;
    return mism;
}

int64_t orc_evolve(const double *J, int64_t nx, int64_t ny, int64_t nz, const orc_params *p,
                   const double *dirs, int64_t n, const uint32_t *ids, double *c, double *R,
                   int32_t *iters, uint8_t *status, uint8_t *streak, double *e_mc, int32_t n_iter,
                   double *trace, int64_t *evolved)
{
    return orc_evolve_log(J, nx, ny, nz, p, dirs, n, ids, c, R, iters, status, streak, e_mc, n_iter, trace, NULL,
                          evolved);
}

/* Terms of one contour at (c, R) for iteration n without updating it (Monte-Carlo, or exact lattice
 * sums when flags bit 1 is set; pts / vals are filled by the Monte-Carlo form only).
 * out: [A, B_R, Bc_x, Bc_y, Bc_z, scale=V/N, dE/dp (3), dE/dq (3), E, g_R, g_c (3)] (17 values).
 * pts (N x 3) / vals (N) receive the sample positions and interpolated values if non-NULL. */
void orc_mc_terms(const double *J, int64_t nx, int64_t ny, int64_t nz, const orc_params *p,
                  const double *dirs, const double c[3], double R, uint32_t n, uint32_t id, double *out,
                  double *pts, double *vals)
{
    orc_vol vol = {J, nx, ny, nz, p, dirs};
    orc_sums sm;
    double scale = contour_sums(&vol, c, R, n, id, &sm, pts, vals);
    int dim = p->dim;
    double twoR_d = pow(2.0 * R, dim);
    double A = scale * sm.A;
    out[0] = A;
    out[1] = scale * sm.BR;
    for (int i = 0; i < 3; ++i) out[2 + i] = scale * sm.Bc[i];
    out[5] = scale;
    double qmp = 2.0 * R, gamma = 1.0 / pow(qmp, dim);
    for (int i = 0; i < 3; ++i) { out[6 + i] = 0.0; out[9 + i] = 0.0; }
    out[6] = gamma * ((double)dim / qmp * A + scale * sm.Sp[0]);
    out[9] = gamma * (-(double)dim / qmp * A + scale * sm.Sq[0]);
    for (int i = 1; i < dim; ++i) {
        out[6 + i] = gamma * scale * sm.Sp[i];
        out[9 + i] = gamma * scale * sm.Sq[i];
    }
    out[12] = A / twoR_d;
    out[13] = (out[1] - (double)dim / R * A) / twoR_d;
    for (int i = 0; i < 3; ++i) out[14 + i] = out[2 + i] / twoR_d;
}

/* Estimator value with the sample points held fixed: scale * sum S(|x_j - c|; R) I_j / (2R)^d. */
double orc_energy_fixed(int dim, double dR, const double *pts, const double *vals, int64_t N, double scale,
                        const double c[3], double R)
{
    double acc = 0.0;
    for (int64_t j = 0; j < N; ++j) {
        double d2 = 0.0;
        for (int i = 0; i < dim; ++i) d2 += (pts[j * 3 + i] - c[i]) * (pts[j * 3 + i] - c[i]);
        double w[3];
        orc_weight(dim, sqrt(d2), R, dR, w);
        acc += w[0] * vals[j];
    }
    return scale * acc / pow(2.0 * R, dim);
}

/* ------------------------------------------------------------------------------------------ */
/* Exact discrete energy of Eq. (5): sum over every lattice point k with |k*h - c| < R + dR/2 of */
/* S(|k*h - c|; R) J(k), times the voxel measure prod(h), divided by (2R)^d. Lattice points      */
/* outside the volume take the clamp-to-edge value.                                            */
/* ------------------------------------------------------------------------------------------ */
int orc_energy_vox(const double *J, int64_t nx, int64_t ny, int64_t nz, const orc_params *p, int64_t n,
                   const double *c, const double *R, double *e_vox, double *e_abs)
{
    int dim = p->dim;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        double Ri = R[i];
        double smax = Ri + 0.5 * p->dR;
        const double *ci = &c[i * 3];
        int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) {
            lo[a] = (int64_t)ceil((ci[a] - smax) / p->spacing[a]);
            hi[a] = (int64_t)floor((ci[a] + smax) / p->spacing[a]);
        }
        double acc = 0.0, aabs = 0.0;
        for (int64_t kz = lo[2]; kz <= hi[2]; ++kz)
            for (int64_t ky = lo[1]; ky <= hi[1]; ++ky)
                for (int64_t kx = lo[0]; kx <= hi[0]; ++kx) {
                    double dx = kx * p->spacing[0] - ci[0];
                    double dy = ky * p->spacing[1] - ci[1];
                    double dz = dim == 3 ? kz * p->spacing[2] - ci[2] : 0.0;
                    double r = sqrt(dx * dx + dy * dy + dz * dz);
                    if (!(r < smax)) continue;
                    double w[3];
                    orc_weight(dim, r, Ri, p->dR, w);
                    double v = J[(clampi(kz, 0, nz - 1) * ny + clampi(ky, 0, ny - 1)) * nx + clampi(kx, 0, nx - 1)];
                    acc += w[0] * v;
                    aabs += fabs(w[0] * v);
                }
        double meas = p->spacing[0] * p->spacing[1] * (dim == 3 ? p->spacing[2] : 1.0);
        double norm = meas / pow(2.0 * Ri, dim);
        e_vox[i] = acc * norm;
        if (e_abs) e_abs[i] = aabs * norm;
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Selection (Results): candidates are contours that stopped on convergence or maximum          */
/* iterations with E_vox <= E0; overlapping pairs (|c' - c''| < rho * max(R', R'')) compete and  */
/* the lower energy survives. Sequential greedy in ascending (E_vox, id).                      */
/* ------------------------------------------------------------------------------------------ */
typedef struct { double e; uint32_t id; int64_t idx; } orc_key;

static int key_cmp(const void *a, const void *b)
{
    const orc_key *x = (const orc_key *)a, *y = (const orc_key *)b;
    if (x->e < y->e) return -1;
    if (x->e > y->e) return 1;
    if (x->id < y->id) return -1;
    if (x->id > y->id) return 1;
    return 0;
}

int64_t orc_cull(const orc_params *p, int64_t n, const double *c, const double *R, const double *e_vox,
                 const uint8_t *status, const uint32_t *ids, uint8_t *keep)
{
    int dim = p->dim;
    double rho = rho_of(dim);
    orc_key *keys = (orc_key *)malloc(sizeof(orc_key) * (n > 0 ? n : 1));
    int64_t nc = 0;
    for (int64_t i = 0; i < n; ++i) {
        keep[i] = 0;
        int st = status[i] & 0x0f;
        if ((st == ORC_CONVERGED || st == ORC_MAXITER) && isfinite(e_vox[i]) && e_vox[i] <= p->e0) {
            keys[nc].e = e_vox[i]; keys[nc].id = ids[i]; keys[nc].idx = i; ++nc;
        }
    }
    qsort(keys, (size_t)nc, sizeof(orc_key), key_cmp);
    int64_t *acc = (int64_t *)malloc(sizeof(int64_t) * (nc > 0 ? nc : 1));
    int64_t na = 0;
    for (int64_t t = 0; t < nc; ++t) {
        int64_t i = keys[t].idx;
        int ok = 1;
        for (int64_t u = 0; u < na && ok; ++u) {
            int64_t j = acc[u];
            double d2 = 0.0;
            for (int a = 0; a < dim; ++a) d2 += (c[i * 3 + a] - c[j * 3 + a]) * (c[i * 3 + a] - c[j * 3 + a]);
            double rm = R[i] > R[j] ? R[i] : R[j];
            if (sqrt(d2) < rho * rm) ok = 0;
        }
        if (ok) { acc[na++] = i; keep[i] = 1; }
    }
    free(acc);
    free(keys);
    return na;
}

/* Flags contours whose selection outcome could flip under FP32 evaluation: energy within
 * rel_e of E0 or of an overlapping rival's energy, or a pair distance within tol_d of the
 * overlap radius. */
int64_t orc_cull_ambiguity(const orc_params *p, int64_t n, const double *c, const double *R,
                           const double *e_vox, double rel_e, double tol_d, uint8_t *amb)
{
    int dim = p->dim;
    double rho = rho_of(dim);
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) amb[i] = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (fabs(e_vox[i] - p->e0) <= rel_e * fabs(p->e0)) amb[i] = 1;
        for (int64_t j = i + 1; j < n; ++j) {
            double d2 = 0.0;
            for (int a = 0; a < dim; ++a) d2 += (c[i * 3 + a] - c[j * 3 + a]) * (c[i * 3 + a] - c[j * 3 + a]);
            double d = sqrt(d2), thr = rho * (R[i] > R[j] ? R[i] : R[j]);
            if (fabs(d - thr) <= tol_d) { amb[i] = 1; amb[j] = 1; }
            if (d < thr + tol_d) {
                double sc = fabs(e_vox[i]) > fabs(e_vox[j]) ? fabs(e_vox[i]) : fabs(e_vox[j]);
                if (fabs(e_vox[i] - e_vox[j]) <= rel_e * sc) { amb[i] = 1; amb[j] = 1; }
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) cnt += amb[i];
    return cnt;
}

/* Flags contours whose selection outcome two runs of the same contours may legitimately decide
 * differently: the energy lies within tol_e[i] of E0, or, for an overlapping rival j, the energies
 * lie within tol_e[i] + tol_e[j] of each other, or the pair distance lies within
 * tol_d[i] + tol_d[j] of the overlap radius rho * max(R_i, R_j). The tolerances are per contour
 * (e.g. how far the two runs' energies and centres/radii of that contour are apart), so a
 * decision is flagged only when its margin is smaller than the disagreement in the very
 * quantities it compares. Pairs are found by a sweep over x. Returns the count flagged. */
typedef struct { double x; int64_t i; } orc_xkey;

static int xkey_cmp(const void *a, const void *b)
{
    const orc_xkey *x = (const orc_xkey *)a, *y = (const orc_xkey *)b;
    return x->x < y->x ? -1 : (x->x > y->x ? 1 : (x->i < y->i ? -1 : (x->i > y->i)));
}

int64_t orc_cull_ambiguity_tol(const orc_params *p, int64_t n, const double *c, const double *R,
                               const double *e, const double *tol_e, const double *tol_d, uint8_t *amb)
{
    int dim = p->dim;
    double rho = rho_of(dim);
    double rmax = 0.0, tdmax = 0.0;
    orc_xkey *k = (orc_xkey *)malloc(sizeof(orc_xkey) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        amb[i] = 0;
        if (isfinite(e[i]) && fabs(e[i] - p->e0) <= tol_e[i]) amb[i] = 1;
        if (R[i] > rmax) rmax = R[i];
        if (tol_d[i] > tdmax) tdmax = tol_d[i];
        k[i].x = c[i * 3];
        k[i].i = i;
    }
    qsort(k, (size_t)n, sizeof(orc_xkey), xkey_cmp);
    const double reach = rho * rmax + 2.0 * tdmax;
    for (int64_t a = 0; a < n; ++a) {
        int64_t i = k[a].i;
        for (int64_t b = a + 1; b < n && k[b].x - k[a].x <= reach; ++b) {
            int64_t j = k[b].i;
            double d2 = 0.0;
            for (int q = 0; q < dim; ++q) d2 += (c[i * 3 + q] - c[j * 3 + q]) * (c[i * 3 + q] - c[j * 3 + q]);
            double d = sqrt(d2), thr = rho * (R[i] > R[j] ? R[i] : R[j]);
            double td = tol_d[i] + tol_d[j];
            if (fabs(d - thr) <= td) { amb[i] = 1; amb[j] = 1; }
            if (d < thr + td && fabs(e[i] - e[j]) <= tol_e[i] + tol_e[j]) { amb[i] = 1; amb[j] = 1; }
        }
    }
    free(k);
    /* A flagged contour may be kept by one run and not the other, which changes what it suppresses:
     * every candidate that may overlap a flagged contour earlier in the greedy order (smaller
     * (E, id), within the tolerances) is flagged too, in that order, so the flags close over such
     * chains. */
    orc_key *o = (orc_key *)malloc(sizeof(orc_key) * (n > 0 ? n : 1));
    int64_t no = 0;
    for (int64_t i = 0; i < n; ++i)
        if (isfinite(e[i])) { o[no].e = e[i]; o[no].id = (uint32_t)i; o[no].idx = i; ++no; }
    qsort(o, (size_t)no, sizeof(orc_key), key_cmp);
    int64_t *seen = (int64_t *)malloc(sizeof(int64_t) * (no > 0 ? no : 1));   /* flagged, in greedy order */
    int64_t ns = 0;
    for (int64_t a = 0; a < no; ++a) {
        int64_t j = o[a].idx;
        for (int64_t b = 0; b < ns && !amb[j]; ++b) {
            int64_t i = seen[b];
            double d2 = 0.0;
            for (int q = 0; q < dim; ++q) d2 += (c[i * 3 + q] - c[j * 3 + q]) * (c[i * 3 + q] - c[j * 3 + q]);
            double thr = rho * (R[i] > R[j] ? R[i] : R[j]);
            if (sqrt(d2) < thr + tol_d[i] + tol_d[j]) amb[j] = 1;
        }
        if (amb[j]) seen[ns++] = j;
    }
    free(seen);
    free(o);
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) cnt += amb[i];
    return cnt;
}

/* ------------------------------------------------------------------------------------------ */
/* Unattended workflow: a lattice of initial contours (Sec. II-A / II-B figures: neighbours      */
/* sqrt(1.5) R apart) and culling passes during evolution (the dynamic culling the Conclusion    */
/* proposes).                                                                                   */
/* ------------------------------------------------------------------------------------------ */

/* Centres of a cubic (square in 2D) lattice of pitch `pitch` (physical units) centred in the
 * volume: k_a = max(1, floor(extent_a / pitch)) points per axis, extent_a = (n_a - 1) h_a, the first
 * one at (extent_a - (k_a - 1) pitch) / 2. x fastest. Writes up to cap centres (n x 3) and returns
 * the count. */
int64_t orc_lattice_seeds(const orc_params *p, int64_t nx, int64_t ny, int64_t nz, double pitch, double *out,
                          int64_t cap)
{
    int dim = p->dim;
    int64_t nn[3] = {nx, ny, nz}, k[3] = {1, 1, 1};
    double o[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < dim; ++a) {
        double ext = (double)(nn[a] - 1) * p->spacing[a];
        k[a] = (int64_t)floor(ext / pitch);
        if (k[a] < 1) k[a] = 1;
        o[a] = 0.5 * (ext - (double)(k[a] - 1) * pitch);
    }
    int64_t total = k[0] * k[1] * k[2], m = 0;
    for (int64_t iz = 0; iz < k[2]; ++iz)
        for (int64_t iy = 0; iy < k[1]; ++iy)
            for (int64_t ix = 0; ix < k[0]; ++ix) {
                if (m < cap) {
                    out[m * 3 + 0] = o[0] + (double)ix * pitch;
                    out[m * 3 + 1] = o[1] + (double)iy * pitch;
                    out[m * 3 + 2] = dim == 3 ? o[2] + (double)iz * pitch : 0.0;
                }
                ++m;
            }
    return total;
}

/* One culling pass at the current state, ranking live contours (ACTIVE or CONVERGED) by the
 * Monte-Carlo energy of their last iteration (the exact energy stays with the final selection):
 * candidates are the live contours with a finite energy, all of them while the run is young (its
 * grace period, counted in the run's iterations, has not ended), afterwards only those with
 * E_mc <= e_cull (the pass's own threshold: E0, or a laxer value that only retires contours still
 * far from being cells); with compete set, overlapping candidates compete as in the final selection
 * (sequential greedy in ascending (E_mc, id)) and the losers are retired; the live contours that are
 * not candidates are retired too. Retired contours keep their state with status CULLED (clamp flag
 * kept). Returns the number retired. */
int64_t orc_cull_pass_t(const orc_params *p, int64_t n, const double *c, const double *R, const double *e_mc,
                        uint8_t *status, const uint32_t *ids, int32_t young, double e_cull, int32_t compete)
{
    int dim = p->dim;
    double rho = rho_of(dim);
    orc_key *keys = (orc_key *)malloc(sizeof(orc_key) * (n > 0 ? n : 1));
    int64_t nc = 0, retired = 0;
    for (int64_t i = 0; i < n; ++i) {
        int st = status[i] & 0x0f;
        if (st != ORC_ACTIVE && st != ORC_CONVERGED) continue;
        if (isfinite(e_mc[i]) && (young || e_mc[i] <= e_cull)) {
            keys[nc].e = e_mc[i]; keys[nc].id = ids[i]; keys[nc].idx = i; ++nc;
        } else {
            status[i] = (uint8_t)((status[i] & ORC_CLAMPED) | ORC_CULLED);
            ++retired;
        }
    }
    qsort(keys, (size_t)nc, sizeof(orc_key), key_cmp);
    int64_t *acc = (int64_t *)malloc(sizeof(int64_t) * (nc > 0 ? nc : 1));
    int64_t na = 0;
    for (int64_t t = 0; t < nc; ++t) {
        int64_t i = keys[t].idx;
        int ok = 1;
        for (int64_t u = 0; u < na && ok && compete; ++u) {
            int64_t j = acc[u];
            double d2 = 0.0;
            for (int a = 0; a < dim; ++a) d2 += (c[i * 3 + a] - c[j * 3 + a]) * (c[i * 3 + a] - c[j * 3 + a]);
            double rm = R[i] > R[j] ? R[i] : R[j];
            if (sqrt(d2) < rho * rm) ok = 0;
        }
        if (ok) {
            acc[na++] = i;
        } else {
            status[i] = (uint8_t)((status[i] & ORC_CLAMPED) | ORC_CULLED);
            ++retired;
        }
    }
    free(acc);
    free(keys);
    return retired;
}

/* The pass with the final selection's threshold E0 and competition. */
int64_t orc_cull_pass(const orc_params *p, int64_t n, const double *c, const double *R, const double *e_mc,
                      uint8_t *status, const uint32_t *ids, int32_t young)
{
    return orc_cull_pass_t(p, n, c, R, e_mc, status, ids, young, p->e0, 1);
}

/* ------------------------------------------------------------------------------------------ */
/* Star-shaped contours (not in the paper: a builder-defined extension of its sphere). A contour */
/* has one radius R_k per table direction T_k; the directions stay fixed in space (no rotation). */
/* Energy: the table average of per-direction radial energies,                                  */
/*   E = (1/D) sum_k e_k,  e_k = (2 R_k)^-d omega_d d integral_0^inf S(s; R_k) I(c + s T_k) s^(d-1) ds, */
/* which is the sphere's energy (Eq. (5), the direction integral taken as the table average)    */
/* when every R_k equals R. Smoothing over the direction graph: each radius relaxes toward the   */
/* mean m_k of its neighbours' by the fraction min(1, eps lambda / 2) (a Laplacian step whose    */
/* rate is capped, so it stays stable while eps is large).                                      */
/* One iteration draws the sphere sampler's Philox pairs with Q = I: pair m picks k; its rays run */
/* along +T_k with radius R_k and along -T_k with the radius of the antipodal direction; ray     */
/* points s = (R + dR/2) ((l + xi)/L)^(1/d). With the per-point weight                          */
/*   q(R) = (2R)^-d omega_d (R + dR/2)^d / (M L)                                                  */
/* E = sum q S I, g_c = sum q (-dS/dr I u), and for each sampled direction k                     */
/*   g_k = sum over the rays along k of q (B_R,ray - (d / R_k) A_ray),                           */
/* an unbiased estimate of dE/dR_k (a ray picks k with probability 1/D). Step: c -= (eps/2) g_c; */
/* R_k -= (eps/2) D g_k + min(1, eps lambda / 2) (R_k - m_k), all from the old radii: each radius */
/* is stepped as if it were the contour's only one, so tied radii take the sphere's step on      */
/* average (and the smoothing leaves tied radii alone).                                          */
/* ------------------------------------------------------------------------------------------ */

/* Direction tables of the star contour: anti[k] = the direction opposite T_k (|T_j + T_k| <
 * 1e-4, else -1 is returned), and the direction graph: the 6 (3D) or 2 (2D) nearest directions of
 * each (largest dot product; dot products within 1e-6 tie and the lower index wins, so a table
 * rounded to FP32 gives the same graph), made symmetric; N(k) is
 * nb_idx[nb_off[k] .. nb_off[k+1]) in ascending order. Returns the number of entries, or -2 if
 * they exceed cap. */
int32_t orc_star_tables(int dim, const double *dirs, int32_t D, int32_t *anti, int32_t *nb_off, int32_t *nb_idx,
                        int32_t cap)
{
    const int deg = dim == 3 ? 6 : 2;
    for (int32_t k = 0; k < D; ++k) {
        int32_t best = -1;
        double bd = 1e30;
        for (int32_t j = 0; j < D; ++j) {
            double e2 = 0.0;
            for (int a = 0; a < dim; ++a) {
                double t = dirs[j * dim + a] + dirs[k * dim + a];
                e2 += t * t;
            }
            if (e2 < bd) { bd = e2; best = j; }
        }
        if (!(sqrt(bd) < 1e-4)) return -1;
        anti[k] = best;
    }
    /* k-nearest lists */
    int32_t *knn = (int32_t *)malloc(sizeof(int32_t) * (size_t)D * deg);
    for (int32_t k = 0; k < D; ++k) {
        int taken = 0;
        while (taken < deg) {
            int32_t best = -1;
            double bd = -2.0;
            for (int32_t j = 0; j < D; ++j) {
                if (j == k) continue;
                int used = 0;
                for (int t = 0; t < taken; ++t) used |= knn[k * deg + t] == j;
                if (used) continue;
                double dt = 0.0;
                for (int a = 0; a < dim; ++a) dt += dirs[j * dim + a] * dirs[k * dim + a];
                /* dot products within 1e-6 tie (the table's symmetric neighbours); the lower index wins */
                if (best < 0 || dt > bd + 1e-6) { bd = dt; best = j; }
            }
            knn[k * deg + taken++] = best;
        }
    }
    /* symmetric closure, ascending */
    int32_t total = 0;
    nb_off[0] = 0;
    for (int32_t k = 0; k < D; ++k) {
        for (int32_t j = 0; j < D; ++j) {
            if (j == k) continue;
            int edge = 0;
            for (int t = 0; t < deg; ++t) edge |= knn[k * deg + t] == j || knn[j * deg + t] == k;
            if (!edge) continue;
            if (total >= cap) { free(knn); return -2; }
            nb_idx[total++] = j;
        }
        nb_off[k + 1] = total;
    }
    free(knn);
    return total;
}

typedef struct {
    double E, Eabs, gc[3], gcabs[3], gcsl[3];
    double *gk, *gkabs, *gksl;  /* D each */
    int n_kink;
    double *pts, *vals;         /* optional: sample positions (N x 3) and values (N) */
    int32_t *ray_dir;           /* optional: direction whose radius each sample's ray used (N) */
} orc_star_sums;

/* Sums of one star iteration at (c, R_k) for iteration n (see the block comment above). */
static void star_sums(const orc_vol *vol, const int32_t *anti, const double c[3], const double *Rk, uint32_t n,
                      uint32_t id, orc_star_sums *sm)
{
    const orc_params *p = vol->p;
    const int dim = p->dim, M = p->n_rays, L = p->n_radial, D = p->n_dirs;
    const double rho = rho_of(dim);
    sm->E = sm->Eabs = 0.0;
    for (int i = 0; i < 3; ++i) sm->gc[i] = sm->gcabs[i] = sm->gcsl[i] = 0.0;
    for (int k = 0; k < D; ++k) sm->gk[k] = sm->gkabs[k] = sm->gksl[k] = 0.0;
    sm->n_kink = 0;
    for (int m = 0; m < M / 2; ++m) {
        uint32_t x[4];
        philox_at(p, (uint32_t)m, n, id, 1u, x);
        uint32_t k = (uint32_t)(((uint64_t)x[0] * (uint64_t)(uint32_t)D) >> 32);
        double xi = orc_uniform(x[1]);
        double t[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < dim; ++i) t[i] = vol->dirs[(int64_t)k * dim + i];
        for (int sgn = 0; sgn < 2; ++sgn) {
            const int32_t kr = sgn ? anti[k] : (int32_t)k;
            const double R = Rk[kr];
            const double smax = R + 0.5 * p->dR;
            const double q = ball_measure(dim) * pow(smax, dim) / pow(2.0 * R, dim) / ((double)M * (double)L);
            const double a = rho * R, dr = rho * p->dR;
            const double kinks[4] = {a - 0.5 * dr, a + 0.5 * dr, R - 0.5 * p->dR, R + 0.5 * p->dR};
            double us[3];
            for (int i = 0; i < 3; ++i) us[i] = sgn ? -t[i] : t[i];
            double A = 0.0, Aabs = 0.0, BR = 0.0, BRabs = 0.0, slBR = 0.0;
            for (int l = 0; l < L; ++l) {
                double tau = ((double)l + xi) / (double)L;
                double s = smax * (dim == 3 ? cbrt(tau) : sqrt(tau));
                double pos[3];
                for (int i = 0; i < 3; ++i) pos[i] = c[i] + s * us[i];
                double I = orc_interp(vol->J, vol->nx, vol->ny, vol->nz, dim, pos[0] / p->spacing[0],
                                      pos[1] / p->spacing[1], dim == 3 ? pos[2] / p->spacing[2] : 0.0);
                double w[3];
                orc_weight(dim, s, R, p->dR, w);
                A += w[0] * I; Aabs += fabs(w[0] * I);
                BR += w[2] * I; BRabs += fabs(w[2] * I);
                if (sm->pts) {
                    const int64_t idx = ((int64_t)m * 2 + sgn) * L + l;
                    for (int i = 0; i < 3; ++i) sm->pts[idx * 3 + i] = pos[i];
                    sm->vals[idx] = I;
                    sm->ray_dir[idx] = kr;
                }
                sm->E += q * w[0] * I; sm->Eabs += fabs(q * w[0] * I);
                for (int i = 0; i < dim; ++i) {
                    sm->gc[i] += q * (-w[1] * I * us[i]);
                    sm->gcabs[i] += fabs(q * w[1] * I * us[i]);
                }
                for (int kk = 0; kk < 4; ++kk) {
                    if (fabs(s - kinks[kk]) <= ORC_KINK_REL * smax) {
                        double wl[3], wr[3];
                        orc_weight(dim, kinks[kk] - 1e-9 * smax, R, p->dR, wl);
                        orc_weight(dim, kinks[kk] + 1e-9 * smax, R, p->dR, wr);
                        slBR += fabs((wr[2] - wl[2]) * I);
                        for (int i = 0; i < dim; ++i) sm->gcsl[i] += fabs(q * (wr[1] - wl[1]) * I * us[i]);
                        sm->n_kink += 1;
                    }
                }
            }
            sm->gk[kr] += q * (BR - (double)dim / R * A);
            sm->gkabs[kr] += q * (BRabs + (double)dim / R * Aabs);
            sm->gksl[kr] += q * slBR;
        }
    }
}

/* Smoothing fraction of iteration eps. */
static double star_relax(double eps, double lambda)
{
    double f = 0.5 * eps * lambda;
    return f < 1.0 ? f : 1.0;
}

/* Radius steps of one star iteration before clamping:
 * dR_k = -(eps/2) D g_k - min(1, eps lambda / 2) (R_k - m_k). */
static void star_radius_steps(const orc_params *p, const int32_t *nb_off, const int32_t *nb_idx, double lambda,
                              const double *Rk, const orc_star_sums *sm, double eps, double *dRk)
{
    const double f = star_relax(eps, lambda);
    for (int32_t k = 0; k < p->n_dirs; ++k) {
        double sum = 0.0;
        for (int32_t e = nb_off[k]; e < nb_off[k + 1]; ++e) sum += Rk[nb_idx[e]];
        const double mk = nb_off[k + 1] > nb_off[k] ? sum / (double)(nb_off[k + 1] - nb_off[k]) : Rk[k];
        dRk[k] = -0.5 * eps * (double)p->n_dirs * sm->gk[k] - f * (Rk[k] - mk);
    }
}

/* Terms of one star iteration at (c, R_k), iteration n, without updating. out: [E, E_abs,
 * g_c (3), g_c_abs (3), dc (3), dc_abs (3), dc_slack (3), n_kink] (18 values); dRk / dRk_abs /
 * dRk_slack (D each): the radius steps before clamping, their magnitude scale and kink slack. */
void orc_star_step_terms(const double *J, int64_t nx, int64_t ny, int64_t nz, const orc_params *p,
                         const double *dirs, const int32_t *anti, const int32_t *nb_off, const int32_t *nb_idx,
                         double lambda, const double c[3], const double *Rk, uint32_t n, uint32_t id, double *out,
                         double *dRk, double *dRk_abs, double *dRk_slack, double *pts, double *vals,
                         int32_t *ray_dir)
{
    orc_vol vol = {J, nx, ny, nz, p, dirs};
    const int D = p->n_dirs;
    orc_star_sums sm;
    sm.gk = (double *)malloc(sizeof(double) * 3 * (size_t)D);
    sm.gkabs = sm.gk + D;
    sm.gksl = sm.gk + 2 * D;
    sm.pts = pts;
    sm.vals = vals;
    sm.ray_dir = ray_dir;
    star_sums(&vol, anti, c, Rk, n, id, &sm);
    const double eps = p->eps0 / sqrt((double)n);
    out[0] = sm.E; out[1] = sm.Eabs;
    for (int i = 0; i < 3; ++i) {
        out[2 + i] = sm.gc[i]; out[5 + i] = sm.gcabs[i];
        out[8 + i] = -0.5 * eps * sm.gc[i]; out[11 + i] = 0.5 * eps * sm.gcabs[i];
        out[14 + i] = 0.5 * eps * sm.gcsl[i];
    }
    out[17] = (double)sm.n_kink;
    star_radius_steps(p, nb_off, nb_idx, lambda, Rk, &sm, eps, dRk);
    const double f = star_relax(eps, lambda);
    for (int32_t k = 0; k < D; ++k) {
        double mabs = 0.0;
        for (int32_t e = nb_off[k]; e < nb_off[k + 1]; ++e) mabs += fabs(Rk[nb_idx[e]]);
        if (nb_off[k + 1] > nb_off[k]) mabs /= (double)(nb_off[k + 1] - nb_off[k]);
        dRk_abs[k] = 0.5 * eps * (double)D * sm.gkabs[k] + f * (fabs(Rk[k]) + mabs);
        dRk_slack[k] = 0.5 * eps * (double)D * sm.gksl[k];
    }
    free(sm.gk);
}

/* Evolve star contours: c (n x 3 physical), Rk (n x D), Rmean (n, written: the mean of R_k), and
 * the sphere path's per-contour counters; same stop rules, with the move of an iteration the
 * largest of |dR_k| (after clamping) and |dc|. Returns the contour-iterations run. */
int64_t orc_star_evolve(const double *J, int64_t nx, int64_t ny, int64_t nz, const orc_params *p,
                        const double *dirs, const int32_t *anti, const int32_t *nb_off, const int32_t *nb_idx,
                        double lambda, int64_t n, const uint32_t *ids, double *c, double *Rk, double *Rmean,
                        int32_t *iters, uint8_t *status, uint8_t *streak, double *e_mc, int32_t n_iter)
{
    orc_vol vol = {J, nx, ny, nz, p, dirs};
    const int dim = p->dim, D = p->n_dirs;
    int64_t done = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : done)
    for (int64_t i = 0; i < n; ++i) {
        double *R = &Rk[i * D];
        orc_star_sums sm;
        sm.pts = sm.vals = NULL;
        sm.ray_dir = NULL;
        sm.gk = (double *)malloc(sizeof(double) * 4 * (size_t)D);
        sm.gkabs = sm.gk + D;
        sm.gksl = sm.gk + 2 * D;
        double *dR = sm.gk + 3 * D;
        for (int32_t it = 0; it < n_iter; ++it) {
            if ((status[i] & 0x0f) != ORC_ACTIVE) break;
            uint32_t nn = (uint32_t)(iters[i] + 1);
            iters[i] = (int32_t)nn;
            double *ci = &c[i * 3];
            star_sums(&vol, anti, ci, R, nn, ids[i], &sm);
            const double eps = p->eps0 / sqrt((double)nn);
            star_radius_steps(p, nb_off, nb_idx, lambda, R, &sm, eps, dR);
            const double lo = r_low(p), hi = p->r_max;
            uint8_t flag = status[i] & ORC_CLAMPED;
            double move = 0.0, sum = 0.0;
            int finite = isfinite(sm.E);
            for (int32_t k = 0; k < D; ++k) {
                double Rn = R[k] + dR[k];
                if (Rn < lo) { Rn = lo; flag = ORC_CLAMPED; }
                if (Rn > hi) { Rn = hi; flag = ORC_CLAMPED; }
                finite = finite && isfinite(Rn);
                if (fabs(Rn - R[k]) > move) move = fabs(Rn - R[k]);
                R[k] = Rn;
                sum += Rn;
            }
            double dcn = 0.0;
            for (int a = 0; a < dim; ++a) {
                double d = -0.5 * eps * sm.gc[a];
                ci[a] += d;
                dcn += d * d;
                finite = finite && isfinite(ci[a]);
            }
            dcn = sqrt(dcn);
            if (dcn > move) move = dcn;
            Rmean[i] = sum / (double)D;
            e_mc[i] = sm.E;
            uint8_t st = ORC_ACTIVE;
            if (!finite) {
                st = ORC_NONFINITE;
            } else {
                for (int a = 0; a < dim; ++a) {
                    int64_t na = a == 0 ? nx : (a == 1 ? ny : nz);
                    if (ci[a] < 0.0 || ci[a] > (double)(na - 1) * p->spacing[a]) st = ORC_OUT;
                }
            }
            if (st == ORC_ACTIVE) {
                if (move < p->conv_tol) streak[i] = (uint8_t)(streak[i] < 255 ? streak[i] + 1 : 255);
                else streak[i] = 0;
                if (p->conv_window > 0 && streak[i] >= p->conv_window) st = ORC_CONVERGED;
            }
            status[i] = (uint8_t)(st | flag);
            done += 1;
        }
        free(sm.gk);
    }
    return done;
}

/* Threads the parallel loops over contours use from now on (timing only; results do not depend
 * on it: every contour is computed by one thread in a fixed order). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
