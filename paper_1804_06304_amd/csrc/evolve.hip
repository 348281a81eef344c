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

// The loaded corners of one trilinear (bilinear) gather, split from the arithmetic so that a thread
// can issue the loads of several points before it consumes any of them.
template <int DIM>
struct Tap {
    Pair r[DIM == 3 ? 4 : 2];
    float fx, fy, fz;
};

template <int DIM>
__device__ __forceinline__ Tap<DIM> tap_load(const Geometry &g, const int anc[3], const float w[3]) {
    Tap<DIM> tp;
    const int ix = split(anc[0], w[0], g.nx, tp.fx);
    const int iy = split(anc[1], w[1], g.ny, tp.fy);
    if constexpr (DIM == 2) {
        tp.fz = 0.0f;
        const float *p = g.J + (long)iy * g.nx + ix;
        tp.r[0] = pair_at(p);
        tp.r[1] = pair_at(p + g.nx);
    } else {
        const int iz = split(anc[2], w[2], g.nz, tp.fz);
        const long nxy = (long)g.nx * g.ny;
        const float *p = g.J + ((long)iz * g.ny + iy) * g.nx + ix;
        tp.r[0] = pair_at(p);
        tp.r[1] = pair_at(p + g.nx);
        tp.r[2] = pair_at(p + nxy);
        tp.r[3] = pair_at(p + nxy + g.nx);
    }
    return tp;
}

template <int DIM>
__device__ __forceinline__ float tap_value(const Tap<DIM> &tp) {
    const float a0 = fmaf(tp.fx, tp.r[0].hi - tp.r[0].lo, tp.r[0].lo);
    const float a1 = fmaf(tp.fx, tp.r[1].hi - tp.r[1].lo, tp.r[1].lo);
    const float b0 = fmaf(tp.fy, a1 - a0, a0);
    if constexpr (DIM == 2) {
        return b0;
    } else {
        const float a2 = fmaf(tp.fx, tp.r[2].hi - tp.r[2].lo, tp.r[2].lo);
        const float a3 = fmaf(tp.fx, tp.r[3].hi - tp.r[3].lo, tp.r[3].lo);
        const float b1 = fmaf(tp.fy, a3 - a2, a2);
        return fmaf(tp.fz, b1 - b0, b0);
    }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Geometry of the weight S(r; R) for the current R (Sec. II-B, Eq. (5)): inner core -1 up to
// rho R - dr/2, ramp of width dr = rho dR, shell +1 up to R - dR/2, outer ramp of width dR down to 0
// at R + dR/2. Half-open intervals.
template <int DIM>
struct Weight {
    static constexpr float RHO = DIM == 3 ? 0.79370052598409973738f : 0.70710678118654752440f;
    float ain, R, k0, k1, k2, k3, in_slope, out_slope;
    __device__ __forceinline__ Weight(float R_, float dR) {
        const float dr = RHO * dR;
        R = R_;
        ain = RHO * R_;
        k0 = ain - 0.5f * dr;
        k1 = ain + 0.5f * dr;
        k2 = R_ - 0.5f * dR;
        k3 = R_ + 0.5f * dR;
        in_slope = 2.0f / dr;
        out_slope = 1.0f / dR;
    }
    // S, dS/dr, dS/dR at radius r
    __device__ __forceinline__ void eval(float r, float &S, float &Sr, float &SR) const {
        if (r < k0) {
            S = -1.0f; Sr = 0.0f; SR = 0.0f;
        } else if (r < k1) {
            S = (r - ain) * in_slope; Sr = in_slope; SR = -RHO * in_slope;
        } else if (r < k2) {
            S = 1.0f; Sr = 0.0f; SR = 0.0f;
        } else if (r < k3) {
            S = 0.5f - (r - R) * out_slope; Sr = -out_slope; SR = out_slope;
        } else {
            S = 0.0f; Sr = 0.0f; SR = 0.0f;
        }
    }
};

// Direction and radial jitter of ray `ray` (0..M-1) at iteration n: pair m = ray mod M/2 draws
// Philox at (m, n, id, 1); rays m and m + M/2 point along +u and -u.
template <int DIM>
__device__ __forceinline__ void draw_ray(int ray, int half, uint32_t n, uint32_t id, uint32_t k0, uint32_t k1,
                                         int D, const float *tdir, const Rot<DIM> &Q, float u[DIM], float &xi) {
    const int m = ray % half;
    uint32_t x[4];
    philox10((uint32_t)m, n, id, 1u, k0, k1, x);
    const int k = (int)__umulhi(x[0], (uint32_t)D);
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

template <int DIM>
__device__ __forceinline__ float radial(float smax, int l, float xi, float invL) {
    const float tau = ((float)l + xi) * invL;
    return smax * (DIM == 3 ? cbrtf(tau) : sqrtf(tau));
}

// Sums of one thread for one iteration. Fast mapping (M divides T or T divides M): a thread owns
// whole rays and walks their radial points U at a time, issuing all U gathers before using them.
// Otherwise points are taken round-robin.
template <int DIM, int T, int U>
__device__ __forceinline__ void thread_sums(const Geometry &g, const int anc[3], const float off[3],
                                            const Weight<DIM> &wt, float smax, const Rot<DIM> &Q, int M, int L,
                                            uint32_t n, uint32_t id, uint32_t key0, uint32_t key1, int D,
                                            const float *tdir, int t, float &accA, float &accBR,
                                            float accB[DIM]) {
    const int half = M / 2;
    const float invL = 1.0f / (float)L;
    if (M <= T ? (T % M == 0) : (M % T == 0)) {
        const int ray0 = M <= T ? t % M : t;
        const int rstep = M <= T ? M : T;
        const int l0 = M <= T ? t / M : 0;
        const int ls = M <= T ? T / M : 1;
        if (l0 >= L) return;
        for (int ray = ray0; ray < M; ray += rstep) {
            float u[DIM], xi;
            draw_ray<DIM>(ray, half, n, id, key0, key1, D, tdir, Q, u, xi);
            float du[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int i = 0; i < DIM; ++i) du[i] = u[i] * g.inv_h[i];
            float q = 0.0f;
            for (int l = l0; l < L; l += ls * U) {
                Tap<DIM> tp[U];
                float rad[U];
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const int ll = l + ls * k;
                    rad[k] = radial<DIM>(smax, ll < L ? ll : l, xi, invL);
                    float w[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int i = 0; i < DIM; ++i) w[i] = fmaf(rad[k], du[i], off[i]);
                    tp[k] = tap_load<DIM>(g, anc, w);
                }
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    if (l + ls * k < L) {
                        const float I = tap_value<DIM>(tp[k]);
                        float S, Sr, SR;
                        wt.eval(rad[k], S, Sr, SR);
                        accA = fmaf(S, I, accA);
                        accBR = fmaf(SR, I, accBR);
                        q = fmaf(Sr, I, q);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < DIM; ++i) accB[i] = fmaf(-q, u[i], accB[i]);
        }
        return;
    }
    // general mapping
    int cur_ray = -1;
    float u[DIM], xi = 0.0f, q = 0.0f;
#pragma unroll
    for (int i = 0; i < DIM; ++i) u[i] = 0.0f;
    for (int j = t; j < M * L; j += T) {
        const int ray = j % M;
        const int l = j / M;
        if (ray != cur_ray) {
            if (cur_ray >= 0) {
#pragma unroll
                for (int i = 0; i < DIM; ++i) accB[i] = fmaf(-q, u[i], accB[i]);
                q = 0.0f;
            }
            cur_ray = ray;
            draw_ray<DIM>(ray, half, n, id, key0, key1, D, tdir, Q, u, xi);
        }
        const float rad = radial<DIM>(smax, l, xi, invL);
        float w[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < DIM; ++i) w[i] = fmaf(rad * u[i], g.inv_h[i], off[i]);
        const float I = tap_value<DIM>(tap_load<DIM>(g, anc, w));
        float S, Sr, SR;
        wt.eval(rad, S, Sr, SR);
        accA = fmaf(S, I, accA);
        accBR = fmaf(SR, I, accBR);
        q = fmaf(Sr, I, q);
    }
    if (cur_ray >= 0) {
#pragma unroll
        for (int i = 0; i < DIM; ++i) accB[i] = fmaf(-q, u[i], accB[i]);
    }
}

template <int DIM, int WAVES, bool TRACE, int U>
__global__ __launch_bounds__(64 * WAVES) void evolve_kernel(EvolveArgs a) {
    constexpr int T = 64 * WAVES;
    constexpr int NR = 2 + DIM;  // A, B_R, B_c[DIM]
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
    const int NPTS = a.M * a.L;
    const float dR = a.dR;
    int ran = 0;

    for (int it = 0; it < a.n_iter; ++it) {
        n += 1;
        const float smax = R + 0.5f * dR;
        const Weight<DIM> wt(R, dR);
        const Rot<DIM> Q = draw_rotation<DIM>((uint32_t)n, id, a.key0, a.key1, (a.flags & 1) != 0);

        float accA = 0.0f, accBR = 0.0f, accB[DIM];
#pragma unroll
        for (int i = 0; i < DIM; ++i) accB[i] = 0.0f;
        thread_sums<DIM, T, U>(g, anc, off, wt, smax, Q, a.M, a.L, (uint32_t)n, id, a.key0, a.key1, a.D, tdir, t,
                               accA, accBR, accB);

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

template <int DIM, int WAVES, bool TRACE, int U>
hipError_t launch_t(const EvolveArgs &a, hipStream_t s) {
    const size_t lds = sizeof(float) * ((size_t)a.D * DIM + 2 * WAVES * (2 + DIM));
    hipLaunchKernelGGL((evolve_kernel<DIM, WAVES, TRACE, U>), dim3(a.n), dim3(64 * WAVES), lds, s, a);
    return hipGetLastError();
}

// Gathers in flight per thread: `unroll` points at a time (0: as many as the thread has, up to 4).
template <int DIM, int WAVES, bool TRACE>
hipError_t launch_u(const EvolveArgs &a, int unroll, hipStream_t s) {
    constexpr int T = 64 * WAVES;
    int u = unroll;
    if (u <= 0) {
        const int per = a.M <= T ? (a.L + T / a.M - 1) / (T / a.M) : a.L;
        u = per >= 4 ? 4 : (per >= 2 ? 2 : 1);
    }
    if (u >= 4) return launch_t<DIM, WAVES, TRACE, 4>(a, s);
    if (u >= 2) return launch_t<DIM, WAVES, TRACE, 2>(a, s);
    return launch_t<DIM, WAVES, TRACE, 1>(a, s);
}

template <int DIM, bool TRACE>
hipError_t launch_w(const EvolveArgs &a, int waves, int unroll, hipStream_t s) {
    switch (waves) {
        case 1: return launch_u<DIM, 1, TRACE>(a, unroll, s);
        case 2: return launch_u<DIM, 2, TRACE>(a, unroll, s);
        case 8: return launch_u<DIM, 8, TRACE>(a, unroll, s);
        default: return launch_u<DIM, 4, TRACE>(a, unroll, s);
    }
}

}  // namespace

hipError_t launch_evolve(const EvolveArgs &a, int dim, int waves, int unroll, bool trace, hipStream_t s) {
    if (a.n <= 0 || a.n_iter <= 0) return hipSuccess;
    if (dim == 2) return trace ? launch_w<2, true>(a, waves, unroll, s) : launch_w<2, false>(a, waves, unroll, s);
    return trace ? launch_w<3, true>(a, waves, unroll, s) : launch_w<3, false>(a, waves, unroll, s);
}

}  // namespace snk
