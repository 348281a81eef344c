// Evolution kernel: gradient descent of independent snakuscules with Monte-Carlo sums.
//
// One workgroup (WAVES wave64s) owns one contour for all iterations of a call; contours are
// independent during evolution (Sec. II-D), so there is no grid-wide synchronisation. Per
// iteration n the workgroup
//   1. draws the contour's random rotation Q from Philox4x32-10 at counter (0, n, id, 0)
//      (Shoemake's uniform quaternion in 3D, an angle in 2D);
//   2. gives each thread one ray: pair m = ray mod M/2 draws Philox at (m, n, id, 1) -> table row
//      k = floor(x0 * D / 2^32) and jitter xi; rays m and m + M/2 use +u and -u (antithetic);
//   3. samples its radial points s = s_max ((l + xi)/L)^(1/d), s_max = R + dR/2 (uniform in the
//      ball, Sec. II-E), gathers the smoothed volume trilinearly (bilinearly in 2D), evaluates the
//      four-region weight S and its derivatives (Sec. II-B, Eq. (5)) and accumulates
//      A = sum S I, B_R = sum dS/dR I, B_c = -sum dS/dr I u;
//   4. reduces the sums across the workgroup in a fixed order (xor-shuffle butterflies, then the
//      per-wave partials in wave order), so every lane holds bit-identical totals;
//   5. applies the descent step of Eqs. (7)-(15) in (c, R) form: E = A/(2R)^d,
//      dE/dR = (B_R - (d/R) A)/(2R)^d, dE/dc = B_c/(2R)^d, eps = eps0/sqrt(n),
//      dR = -(eps/2) dE/dR, dc = -(eps/2) dE/dc (the p,q steps of Eqs. (12)-(15) mapped through
//      c = (p+q)/2, R = (q_x - p_x)/2), clamps R, re-anchors c, and tests OUT / convergence.
// Every lane runs the identical update, so the state stays in registers across iterations.
#include <math.h>

#include "snk_internal.h"

namespace snk {

namespace {

__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                         uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// (2*(x >> 9) + 1) * 2^-24: exact in FP32, strictly inside (0, 1).
__device__ __forceinline__ float unit_open(uint32_t x) {
    return (float)((x >> 9) * 2u + 1u) * 5.9604644775390625e-08f;
}

template <int DIM>
struct Rot {
    float q[DIM][DIM];
};

template <int DIM>
__device__ __forceinline__ Rot<DIM> draw_rotation(uint32_t n, uint32_t id, uint32_t k0, uint32_t k1, bool off) {
    Rot<DIM> Q;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) Q.q[i][j] = i == j ? 1.0f : 0.0f;
    if (off) return Q;
    uint32_t x[4];
    philox10(0u, n, id, 0u, k0, k1, x);
    if constexpr (DIM == 2) {
        float s, c;
        sincospif(2.0f * unit_open(x[0]), &s, &c);
        Q.q[0][0] = c;
        Q.q[0][1] = -s;
        Q.q[1][0] = s;
        Q.q[1][1] = c;
    } else {
        const float u1 = unit_open(x[0]), u2 = unit_open(x[1]), u3 = unit_open(x[2]);
        const float a = sqrtf(1.0f - u1), b = sqrtf(u1);
        float s1, c1, s2, c2;
        sincospif(2.0f * u2, &s1, &c1);
        sincospif(2.0f * u3, &s2, &c2);
        const float qx = a * s1, qy = a * c1, qz = b * s2, qw = b * c2;
        Q.q[0][0] = 1.0f - 2.0f * (qy * qy + qz * qz);
        Q.q[0][1] = 2.0f * (qx * qy - qw * qz);
        Q.q[0][2] = 2.0f * (qx * qz + qw * qy);
        Q.q[1][0] = 2.0f * (qx * qy + qw * qz);
        Q.q[1][1] = 1.0f - 2.0f * (qx * qx + qz * qz);
        Q.q[1][2] = 2.0f * (qy * qz - qw * qx);
        Q.q[2][0] = 2.0f * (qx * qz - qw * qy);
        Q.q[2][1] = 2.0f * (qy * qz + qw * qx);
        Q.q[2][2] = 1.0f - 2.0f * (qx * qx + qy * qy);
    }
    return Q;
}

// Coordinate split with clamp-to-edge: v = anc + w, clamped to [0, n-1]; returns the lower voxel
// index and the fraction toward the upper one.
__device__ __forceinline__ int split(int anc, float w, int n, float &f) {
    const float fl = floorf(w);
    int i = anc + (int)fl;
    f = w - fl;
    if (i < 0) {
        i = 0;
        f = 0.0f;
    } else if (i > n - 2) {
        i = n - 2;
        f = 1.0f;
    }
    return i;
}

// Two x-adjacent voxels in one 8-byte load (dword-aligned; gfx950 global loads need no 8-byte
// alignment). The pair never crosses the end of a row: split() keeps the lower index <= n - 2.
struct __attribute__((packed, aligned(4))) Pair {
    float lo, hi;
};

__device__ __forceinline__ Pair pair_at(const float *p) { return *reinterpret_cast<const Pair *>(p); }

template <int DIM>
__device__ __forceinline__ float gather(const Geometry &g, const int anc[3], const float w[3]) {
    float fx, fy;
    const int ix = split(anc[0], w[0], g.nx, fx);
    const int iy = split(anc[1], w[1], g.ny, fy);
    if constexpr (DIM == 2) {
        const float *p = g.J + (long)iy * g.nx + ix;
        const Pair r0 = pair_at(p), r1 = pair_at(p + g.nx);
        const float a0 = fmaf(fx, r0.hi - r0.lo, r0.lo);
        const float a1 = fmaf(fx, r1.hi - r1.lo, r1.lo);
        return fmaf(fy, a1 - a0, a0);
    } else {
        float fz;
        const int iz = split(anc[2], w[2], g.nz, fz);
        const long nxy = (long)g.nx * g.ny;
        const float *p = g.J + ((long)iz * g.ny + iy) * g.nx + ix;
        const Pair r00 = pair_at(p), r10 = pair_at(p + g.nx);
        const Pair r01 = pair_at(p + nxy), r11 = pair_at(p + nxy + g.nx);
        const float a00 = fmaf(fx, r00.hi - r00.lo, r00.lo);
        const float a10 = fmaf(fx, r10.hi - r10.lo, r10.lo);
        const float a01 = fmaf(fx, r01.hi - r01.lo, r01.lo);
        const float a11 = fmaf(fx, r11.hi - r11.lo, r11.lo);
        const float b0 = fmaf(fy, a10 - a00, a00);
        const float b1 = fmaf(fy, a11 - a01, a01);
        return fmaf(fz, b1 - b0, b0);
    }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int DIM, int WAVES, bool TRACE>
__global__ __launch_bounds__(64 * WAVES) void evolve_kernel(EvolveArgs a) {
    constexpr int T = 64 * WAVES;
    constexpr int NR = 2 + DIM;  // A, B_R, B_c[DIM]
    constexpr float RHO = DIM == 3 ? 0.79370052598409973738f : 0.70710678118654752440f;
    constexpr float BALL = DIM == 3 ? 4.18879020478639098462f : 3.14159265358979323846f;
    extern __shared__ float lds[];
    float *tdir = lds;                     // D x DIM direction table
    float *red = lds + a.D * DIM;          // [2][WAVES][NR] partial sums

    const int cid = blockIdx.x;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    DevContour s = a.st[cid];
    if ((s.status & 0x0f) != SNK_ACTIVE || a.n_iter <= 0) return;

    for (int i = t; i < a.D * DIM; i += T) tdir[i] = a.dirs[i];
    __syncthreads();

    const Geometry g = a.g;
    int anc[3] = {s.anc[0], s.anc[1], s.anc[2]};
    float off[3] = {s.off[0], s.off[1], s.off[2]};
    float R = s.R;
    int n = s.iters;
    uint8_t status = s.status;
    int streak = s.streak;
    float e_mc = s.e_mc;
    const uint32_t id = s.id;
    const int M = a.M, L = a.L, half = a.M / 2;
    const int NPTS = M * L;
    const float invL = 1.0f / (float)L;
    const float dR = a.dR;
    const float dr = RHO * dR;
    int ran = 0;

    for (int it = 0; it < a.n_iter; ++it) {
        n += 1;
        const float smax = R + 0.5f * dR;
        const float ain = RHO * R;
        const float k0 = ain - 0.5f * dr, k1 = ain + 0.5f * dr;
        const float k2 = R - 0.5f * dR, k3 = R + 0.5f * dR;
        const float in_slope = 2.0f / dr;
        const float out_slope = 1.0f / dR;
        const Rot<DIM> Q = draw_rotation<DIM>((uint32_t)n, id, a.key0, a.key1, (a.flags & 1) != 0);

        float accA = 0.0f, accBR = 0.0f, accB[DIM];
#pragma unroll
        for (int i = 0; i < DIM; ++i) accB[i] = 0.0f;
        int cur_ray = -1;
        float u[DIM];
        float xi = 0.0f, accQ = 0.0f;
#pragma unroll
        for (int i = 0; i < DIM; ++i) u[i] = 0.0f;

        for (int j = t; j < NPTS; j += T) {
            const int ray = j % M;
            const int l = j / M;
            if (ray != cur_ray) {
                if (cur_ray >= 0) {
#pragma unroll
                    for (int i = 0; i < DIM; ++i) accB[i] = fmaf(-accQ, u[i], accB[i]);
                    accQ = 0.0f;
                }
                cur_ray = ray;
                const int m = ray % half;
                uint32_t x[4];
                philox10((uint32_t)m, (uint32_t)n, id, 1u, a.key0, a.key1, x);
                const int k = (int)__umulhi(x[0], (uint32_t)a.D);
                xi = unit_open(x[1]);
                const float sgn = ray < half ? 1.0f : -1.0f;
                float tk[DIM];
#pragma unroll
                for (int i = 0; i < DIM; ++i) tk[i] = tdir[k * DIM + i];
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    float acc = 0.0f;
#pragma unroll
                    for (int jj = 0; jj < DIM; ++jj) acc = fmaf(Q.q[i][jj], tk[jj], acc);
                    u[i] = sgn * acc;
                }
            }
            const float tau = ((float)l + xi) * invL;
            const float rad = smax * (DIM == 3 ? cbrtf(tau) : sqrtf(tau));
            float w[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int i = 0; i < DIM; ++i) w[i] = fmaf(rad * u[i], g.inv_h[i], off[i]);
            const float I = gather<DIM>(g, anc, w);
            float S, Sr, SR;
            if (rad < k0) {
                S = -1.0f; Sr = 0.0f; SR = 0.0f;
            } else if (rad < k1) {
                S = (rad - ain) * in_slope; Sr = in_slope; SR = -RHO * in_slope;
            } else if (rad < k2) {
                S = 1.0f; Sr = 0.0f; SR = 0.0f;
            } else if (rad < k3) {
                S = 0.5f - (rad - R) * out_slope; Sr = -out_slope; SR = out_slope;
            } else {
                S = 0.0f; Sr = 0.0f; SR = 0.0f;
            }
            accA = fmaf(S, I, accA);
            accBR = fmaf(SR, I, accBR);
            accQ = fmaf(Sr, I, accQ);
        }
        if (cur_ray >= 0) {
#pragma unroll
            for (int i = 0; i < DIM; ++i) accB[i] = fmaf(-accQ, u[i], accB[i]);
        }

        float tot[NR];
        tot[0] = wave_sum(accA);
        tot[1] = wave_sum(accBR);
#pragma unroll
        for (int i = 0; i < DIM; ++i) tot[2 + i] = wave_sum(accB[i]);
        if constexpr (WAVES > 1) {
            float *slot = red + (it & 1) * WAVES * NR;
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < NR; ++k) slot[wave * NR + k] = tot[k];
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                float v = slot[k];
#pragma unroll
                for (int ww = 1; ww < WAVES; ++ww) v += slot[ww * NR + k];
                tot[k] = v;
            }
        }

        // descent step, identical in every lane
        float smax_d = smax;
#pragma unroll
        for (int i = 1; i < DIM; ++i) smax_d *= smax;
        const float scale = BALL * smax_d / (float)NPTS;
        const float A = scale * tot[0];
        const float BR = scale * tot[1];
        float twoR_d = 2.0f * R;
#pragma unroll
        for (int i = 1; i < DIM; ++i) twoR_d *= 2.0f * R;
        const float inv_norm = 1.0f / twoR_d;
        const float E = A * inv_norm;
        const float gR = (BR - ((float)DIM / R) * A) * inv_norm;
        const float eps = a.eps0 / sqrtf((float)n);
        const float dRs = -0.5f * eps * gR;
        float dc[3] = {0.0f, 0.0f, 0.0f};
        float dc2 = 0.0f;
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            dc[i] = -0.5f * eps * (scale * tot[2 + i]) * inv_norm;
            dc2 = fmaf(dc[i], dc[i], dc2);
        }
        if (TRACE && t == 0) {
            float *row = a.trace + (long)cid * SNK_TRACE_W;
            row[0] = A;
            row[1] = BR;
            for (int i = 0; i < 3; ++i) row[2 + i] = i < DIM ? scale * tot[2 + i] : 0.0f;
            row[5] = E;
            row[6] = dRs;
            for (int i = 0; i < 3; ++i) row[7 + i] = dc[i];
            row[10] = (float)n;
            row[11] = R;
            row[12] = eps;
            row[13] = row[14] = row[15] = 0.0f;
        }
        float Rn = R + dRs;
        uint8_t flag = status & SNK_CLAMPED;
        if (Rn < a.r_lo) { Rn = a.r_lo; flag = SNK_CLAMPED; }
        if (Rn > a.r_hi) { Rn = a.r_hi; flag = SNK_CLAMPED; }
        const float move = fmaxf(fabsf(Rn - R), sqrtf(dc2));
        R = Rn;
        e_mc = E;
        bool finite = isfinite(Rn) && isfinite(E);
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            off[i] = fmaf(dc[i], g.inv_h[i], off[i]);
            finite = finite && isfinite(off[i]);
        }
        uint8_t st = SNK_ACTIVE;
        if (!finite) {
            st = SNK_NONFINITE;
        } else {
            const int nn[3] = {g.nx, g.ny, g.nz};
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                if (fabsf(off[i]) >= 0.5f) {
                    const float k = rintf(off[i]);
                    anc[i] += (int)k;
                    off[i] -= k;
                }
                if (off[i] < (float)(-anc[i]) || off[i] > (float)(nn[i] - 1 - anc[i])) st = SNK_OUT;
            }
        }
        if (st == SNK_ACTIVE) {
            streak = move < a.conv_tol ? min(streak + 1, 255) : 0;
            if (a.conv_window > 0 && streak >= a.conv_window) st = SNK_CONVERGED;
        }
        status = (uint8_t)(st | flag);
        ++ran;
        if (st != SNK_ACTIVE) break;
    }

    if (t == 0) {
        DevContour o = s;
        for (int i = 0; i < 3; ++i) {
            o.anc[i] = anc[i];
            o.off[i] = off[i];
        }
        o.R = R;
        o.e_mc = e_mc;
        o.iters = n;
        o.status = status;
        o.streak = (uint8_t)streak;
        a.st[cid] = o;
        atomicAdd(a.counter, (unsigned long long)ran);
    }
}

template <int DIM, int WAVES, bool TRACE>
hipError_t launch_t(const EvolveArgs &a, hipStream_t s) {
    const size_t lds = sizeof(float) * ((size_t)a.D * DIM + 2 * WAVES * (2 + DIM));
    hipLaunchKernelGGL((evolve_kernel<DIM, WAVES, TRACE>), dim3(a.n), dim3(64 * WAVES), lds, s, a);
    return hipGetLastError();
}

template <int DIM, bool TRACE>
hipError_t launch_w(const EvolveArgs &a, int waves, hipStream_t s) {
    switch (waves) {
        case 1: return launch_t<DIM, 1, TRACE>(a, s);
        case 2: return launch_t<DIM, 2, TRACE>(a, s);
        case 8: return launch_t<DIM, 8, TRACE>(a, s);
        default: return launch_t<DIM, 4, TRACE>(a, s);
    }
}

}  // namespace

hipError_t launch_evolve(const EvolveArgs &a, int dim, int waves, bool trace, hipStream_t s) {
    if (a.n <= 0 || a.n_iter <= 0) return hipSuccess;
    if (dim == 2) return trace ? launch_w<2, true>(a, waves, s) : launch_w<2, false>(a, waves, s);
    return trace ? launch_w<3, true>(a, waves, s) : launch_w<3, false>(a, waves, s);
}

}  // namespace snk
