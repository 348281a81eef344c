// Evolution kernel: gradient descent of independent snakuscules with Monte-Carlo sums.
//
// One workgroup (WAVES wave64s) owns one contour at a time and runs its iterations back to back;
// contours are independent during evolution (Sec. II-D), so there is no grid-wide
// synchronisation. Per iteration n the workgroup
//   1. takes the contour's random rotation Q(n) (Philox4x32-10 at counter (0, n, id, 0); Shoemake's
//      uniform quaternion in 3D, an angle in 2D) and the ray draws of every antithetic pair m
//      (Philox at (m, n, id, 1) -> table row k = floor(x0 D / 2^32) and jitter xi) from LDS. Both
//      are state-independent, so wave 0 / wave 1 produce them for iteration n+1 while iteration n
//      is still sampling, and the per-iteration barrier publishes them;
//   2. gives each thread whole rays (u = +-Q T[k]) and walks their radial points
//      s = s_max ((l + xi)/L)^(1/d), s_max = R + dR/2 (uniform in the ball, Sec. II-E), issuing the
//      trilinear (bilinear) gathers of U points before consuming them;
//   3. evaluates the four-region weight S (Sec. II-B, Eq. (5)) and accumulates
//      A = sum S I, B_R = sum dS/dR I, B_c = -sum dS/dr I u (the derivatives are constant on the
//      two ramps, so only the ramp sums of I are kept per ray);
//   4. reduces the sums in a fixed order (xor-shuffle butterflies, then the per-wave partials in
//      wave order), so every lane holds bit-identical totals;
//   5. applies the descent step of Eqs. (7)-(15) in (c, R) form: E = A/(2R)^d,
//      dE/dR = (B_R - (d/R) A)/(2R)^d, dE/dc = B_c/(2R)^d, eps = eps0/sqrt(n),
//      dR = -(eps/2) dE/dR, dc = -(eps/2) dE/dc (the p,q steps of Eqs. (12)-(15) mapped through
//      c = (p+q)/2, R = (q_x - p_x)/2), clamps R, re-anchors c, and tests OUT / convergence.
// Every lane runs the identical update, so the state stays in registers across iterations.
//
// Two launches share this routine: one workgroup per contour of a single volume, and a batched
// launch over a device table of (job, contour) items, optionally persistent with a work queue.
#include <math.h>

#include "snk_internal.h"

namespace snk {

namespace {

constexpr uint32_t kBufferWord3 = 0x00020000u;  // raw buffer descriptor, gfx9 family

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

// Rotation Q (row-major, acting on column vectors) of contour `id` at iteration n.
template <int DIM>
__device__ __forceinline__ void rotation(uint32_t n, uint32_t id, uint32_t k0, uint32_t k1, bool off, float Q[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) Q[i] = (i % 4 == 0) ? 1.0f : 0.0f;
    if (off) return;
    uint32_t x[4];
    philox10(0u, n, id, 0u, k0, k1, x);
    if constexpr (DIM == 2) {
        float s, c;
        sincospif(2.0f * unit_open(x[0]), &s, &c);
        Q[0] = c;
        Q[1] = -s;
        Q[3] = s;
        Q[4] = c;
    } else {
        const float u1 = unit_open(x[0]), u2 = unit_open(x[1]), u3 = unit_open(x[2]);
        const float a = sqrtf(1.0f - u1), b = sqrtf(u1);
        float s1, c1, s2, c2;
        sincospif(2.0f * u2, &s1, &c1);
        sincospif(2.0f * u3, &s2, &c2);
        const float qx = a * s1, qy = a * c1, qz = b * s2, qw = b * c2;
        Q[0] = 1.0f - 2.0f * (qy * qy + qz * qz);
        Q[1] = 2.0f * (qx * qy - qw * qz);
        Q[2] = 2.0f * (qx * qz + qw * qy);
        Q[3] = 2.0f * (qx * qy + qw * qz);
        Q[4] = 1.0f - 2.0f * (qx * qx + qz * qz);
        Q[5] = 2.0f * (qy * qz - qw * qx);
        Q[6] = 2.0f * (qx * qz - qw * qy);
        Q[7] = 2.0f * (qy * qz + qw * qx);
        Q[8] = 1.0f - 2.0f * (qx * qx + qy * qy);
    }
}

// LDS layout of one workgroup.
template <int DIM, int WAVES>
struct Smem {
    static constexpr int NR = 2 + DIM;  // A, B_R, B_c[DIM]
    float *tdir;   // D x DIM direction table
    float *rot;    // [2][9] rotation of the current / next iteration
    int *rk;       // [2][MH] table row of each antithetic pair
    float *rxi;    // [2][MH] radial jitter of each pair
    float *red;    // [2][WAVES][NR] per-wave partial sums
    float *box;    // staged footprint of the contour (box_cap floats)
    int MH;
    __device__ __forceinline__ Smem(float *base, int D, int MH_) {
        MH = MH_;
        tdir = base;
        rot = tdir + D * DIM;
        rk = reinterpret_cast<int *>(rot + 18);
        rxi = reinterpret_cast<float *>(rk + 2 * MH);
        red = rxi + 2 * MH;
        box = red + 2 * WAVES * NR;
    }
    static size_t bytes(int D, int MH, int box_cap) {
        return sizeof(float) * ((size_t)D * DIM + 18 + 4 * MH + 2 * WAVES * NR + (size_t)box_cap);
    }
};

// Wave 0 writes Q(n) into slot `par`; wave 1 (wave 0 when alone) writes the pair draws of n.
template <int DIM, int WAVES>
__device__ __forceinline__ void produce(const Smem<DIM, WAVES> &sm, int par, uint32_t n, uint32_t id,
                                        const JobParams &p, int wave, int lane) {
    if (wave == 0) {
        float Q[9];
        rotation<DIM>(n, id, p.key0, p.key1, (p.flags & 1) != 0, Q);
        if (lane < 9) {
            float v = Q[0];
#pragma unroll
            for (int i = 1; i < 9; ++i) v = lane == i ? Q[i] : v;
            sm.rot[par * 9 + lane] = v;
        }
    }
    if (wave == (WAVES > 1 ? 1 : 0)) {
        for (int m = lane; m < sm.MH; m += 64) {
            uint32_t x[4];
            philox10((uint32_t)m, n, id, 1u, p.key0, p.key1, x);
            sm.rk[par * sm.MH + m] = (int)__umulhi(x[0], (uint32_t)p.D);
            sm.rxi[par * sm.MH + m] = unit_open(x[1]);
        }
    }
}

// Two x-adjacent voxels per load (dword-aligned 8-byte loads). The pair never crosses the end of a
// row: the lower index is kept <= n - 2.
struct __attribute__((packed, aligned(4))) Pair {
    float lo, hi;
};

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Volume access: a raw buffer descriptor with the three neighbour offsets (row, plane,
// row + plane) in scalar registers, or plain global loads with 64-bit offsets for volumes beyond
// 2 GiB.
template <int DIM, bool BUF>
struct Vol {
    const float *J;
    __amdgpu_buffer_rsrc_t rsrc;
    int nx, ny, nz, nxy;
    int so[4];    // byte offsets of the x, y, z and y+z neighbour pairs (buffer path)
    long lo[4];   // element offsets of the same (global path)
    __device__ __forceinline__ Vol(const Geometry &g) {
        J = g.J;
        nx = g.nx;
        ny = g.ny;
        nz = g.nz;
        nxy = g.nx * g.ny;
        lo[0] = 0;
        lo[1] = nx;
        lo[2] = (long)nx * ny;
        lo[3] = (long)nx * ny + nx;
        if constexpr (BUF) {
            for (int k = 0; k < 4; ++k) so[k] = (int)(lo[k] * 4);
            const long bytes = (long)nxy * nz * 4;
            rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)g.J, (short)0, (int)bytes, (int)kBufferWord3);
        }
    }
    // idx: element index of the lower corner (< 2^31); k: which neighbour pair
    template <int K>
    __device__ __forceinline__ Pair load(long idx) const {
        if constexpr (BUF) {
            const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rsrc, (int)idx * 4, so[K], 0);
            return Pair{__uint_as_float(v.x), __uint_as_float(v.y)};
        } else {
            return *reinterpret_cast<const Pair *>(J + idx + lo[K]);
        }
    }
};

template <int DIM>
struct Tap {
    Pair r[DIM == 3 ? 4 : 2];
    float fx, fy, fz;
};

// Clamp-to-edge split of v = anc + w into a lower index in [0, n-2] and a fraction. CLAMP = false
// is used only when every sample of the iteration is known to lie inside, where both agree.
template <bool CLAMP>
__device__ __forceinline__ int split(int anc, float w, int n, float &f) {
    const float fl = floorf(w);
    int i = anc + (int)fl;
    f = w - fl;
    if constexpr (CLAMP) {
        if (i < 0) {
            i = 0;
            f = 0.0f;
        } else if (i > n - 2) {
            i = n - 2;
            f = 1.0f;
        }
    }
    return i;
}

template <int DIM, bool BUF, bool CLAMP>
__device__ __forceinline__ Tap<DIM> vol_tap_load(const Vol<DIM, BUF> &v, const int anc[3], const float w[3]) {
    Tap<DIM> tp;
    const int ix = split<CLAMP>(anc[0], w[0], v.nx, tp.fx);
    const int iy = split<CLAMP>(anc[1], w[1], v.ny, tp.fy);
    if constexpr (DIM == 2) {
        tp.fz = 0.0f;
        const long idx = BUF ? (long)(iy * v.nx + ix) : (long)iy * v.nx + ix;
        tp.r[0] = v.template load<0>(idx);
        tp.r[1] = v.template load<1>(idx);
    } else {
        const int iz = split<CLAMP>(anc[2], w[2], v.nz, tp.fz);
        const long idx = BUF ? (long)(iz * v.nxy + iy * v.nx + ix) : ((long)iz * v.ny + iy) * v.nx + ix;
        tp.r[0] = v.template load<0>(idx);
        tp.r[1] = v.template load<1>(idx);
        tp.r[2] = v.template load<2>(idx);
        tp.r[3] = v.template load<3>(idx);
    }
    return tp;
}

template <int DIM, bool CLAMP, bool BUF>
__device__ __forceinline__ Tap<DIM> tap_load(const Vol<DIM, BUF> &v, const int anc[3], const float w[3]) {
    return vol_tap_load<DIM, BUF, CLAMP>(v, anc, w);
}

// The contour's footprint staged in LDS: voxels [lo, lo + n) of the volume, x fastest. Holds exact
// copies of the smoothed volume, so gathers from it equal gathers from memory.
template <int DIM>
struct Box {
    const float *data;
    int lo[3];
    int bx, bxy;
    int n[3];   // volume dimensions (clamp-to-edge happens in volume coordinates)
};

template <int DIM, bool CLAMP>
__device__ __forceinline__ Tap<DIM> tap_load(const Box<DIM> &b, const int anc[3], const float w[3]) {
    Tap<DIM> tp;
    const int ix = split<CLAMP>(anc[0], w[0], b.n[0], tp.fx) - b.lo[0];
    const int iy = split<CLAMP>(anc[1], w[1], b.n[1], tp.fy) - b.lo[1];
    int idx = iy * b.bx + ix;
    if constexpr (DIM == 2) {
        tp.fz = 0.0f;
    } else {
        const int iz = split<CLAMP>(anc[2], w[2], b.n[2], tp.fz) - b.lo[2];
        idx += iz * b.bxy;
    }
    const float *p = b.data + idx;
    tp.r[0] = Pair{p[0], p[1]};
    tp.r[1] = Pair{p[b.bx], p[b.bx + 1]};
    if constexpr (DIM == 3) {
        tp.r[2] = Pair{p[b.bxy], p[b.bxy + 1]};
        tp.r[3] = Pair{p[b.bxy + b.bx], p[b.bxy + b.bx + 1]};
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
// at R + dR/2. Half-open intervals. On the inner ramp dS/dr = is and dS/dR = -rho is; on the outer
// ramp dS/dr = -os and dS/dR = os; elsewhere both are zero.
template <int DIM>
struct Weight {
    static constexpr float RHO = DIM == 3 ? 0.79370052598409973738f : 0.70710678118654752440f;
    float ain, R, k0, k1, k2, k3, is, os;
    __device__ __forceinline__ Weight(float R_, float dR, float is_, float os_) {
        const float dr = RHO * dR;
        R = R_;
        ain = RHO * R_;
        k0 = ain - 0.5f * dr;
        k1 = ain + 0.5f * dr;
        k2 = R_ - 0.5f * dR;
        k3 = R_ + 0.5f * dR;
        is = is_;
        os = os_;
    }
    // S(r); ramp1 / ramp2 = r on the inner / outer ramp
    __device__ __forceinline__ float S(float r, bool &ramp1, bool &ramp2) const {
        ramp1 = r >= k0 && r < k1;
        ramp2 = r >= k2 && r < k3;
        const float sin_ = fminf(fmaxf((r - ain) * is, -1.0f), 1.0f);
        const float sout = fminf(fmaxf(0.5f - (r - R) * os, 0.0f), 1.0f);
        return r < k2 ? sin_ : sout;
    }
};

template <int DIM>
__device__ __forceinline__ float cube_or_square_root(float tau) {
    if constexpr (DIM == 3) {
        // tau in (0, 1), never denormal: 2^(log2(tau)/3) on the transcendental unit
        return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(tau) * 0.333333343267f);
    } else {
        return __builtin_amdgcn_sqrtf(tau);
    }
}

// Sums of one thread for one iteration. Fast mapping (M divides T or T divides M): a thread owns
// whole rays and walks their radial points U at a time, issuing all U gathers before using them.
// Otherwise points are taken round-robin, one at a time.
template <int DIM, int T, int U, bool CLAMP, typename Src>
__device__ __forceinline__ void thread_sums(const Src &vol, const float inv_h[3], const int anc[3],
                                            const float off[3], const Weight<DIM> &wt, float smax, const float Q[9],
                                            const float *tdir, const int *rk, const float *rxi, int M, int L, int t,
                                            float &accA, float &accBR, float accB[DIM]) {
    constexpr float RHO = Weight<DIM>::RHO;
    const int half = M / 2;
    const float invL = 1.0f / (float)L;
    auto direction = [&](int ray, float u[DIM], float &xi) {
        const int m = ray % half;
        const int k = rk[m];
        xi = rxi[m];
        const float sgn = ray < half ? 1.0f : -1.0f;
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            float acc = 0.0f;
#pragma unroll
            for (int j = 0; j < DIM; ++j) acc = fmaf(Q[i * 3 + j], tdir[k * DIM + j], acc);
            u[i] = sgn * acc;
        }
    };
    auto point = [&](float rad, const Tap<DIM> &tp, float &q1, float &q2) {
        const float I = tap_value<DIM>(tp);
        bool r1, r2;
        const float S = wt.S(rad, r1, r2);
        accA = fmaf(S, I, accA);
        q1 += r1 ? I : 0.0f;
        q2 += r2 ? I : 0.0f;
    };
    auto flush = [&](const float u[DIM], float q1, float q2) {
        accBR = fmaf(-RHO * wt.is, q1, fmaf(wt.os, q2, accBR));
        const float g = wt.is * q1 - wt.os * q2;  // sum of dS/dr * I along the ray
#pragma unroll
        for (int i = 0; i < DIM; ++i) accB[i] = fmaf(-g, u[i], accB[i]);
    };
    if (M <= T ? (T % M == 0) : (M % T == 0)) {
        const int ray0 = M <= T ? t % M : t;
        const int rstep = M <= T ? M : T;
        const int l0 = M <= T ? t / M : 0;
        const int ls = M <= T ? T / M : 1;
        if (l0 >= L) return;
        for (int ray = ray0; ray < M; ray += rstep) {
            float u[DIM], xi;
            direction(ray, u, xi);
            float du[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int i = 0; i < DIM; ++i) du[i] = u[i] * inv_h[i];
            float q1 = 0.0f, q2 = 0.0f;
            for (int l = l0; l < L; l += ls * U) {
                Tap<DIM> tp[U];
                float rad[U];
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const int ll = l + ls * k;
                    rad[k] = smax * cube_or_square_root<DIM>(((float)(ll < L ? ll : l) + xi) * invL);
                    float w[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int i = 0; i < DIM; ++i) w[i] = fmaf(rad[k], du[i], off[i]);
                    tp[k] = tap_load<DIM, CLAMP>(vol, anc, w);
                }
#pragma unroll
                for (int k = 0; k < U; ++k)
                    if (l + ls * k < L) point(rad[k], tp[k], q1, q2);
            }
            flush(u, q1, q2);
        }
        return;
    }
    int cur_ray = -1;
    float u[DIM], xi = 0.0f, q1 = 0.0f, q2 = 0.0f;
#pragma unroll
    for (int i = 0; i < DIM; ++i) u[i] = 0.0f;
    for (int j = t; j < M * L; j += T) {
        const int ray = j % M;
        const int l = j / M;
        if (ray != cur_ray) {
            if (cur_ray >= 0) flush(u, q1, q2);
            q1 = q2 = 0.0f;
            cur_ray = ray;
            direction(ray, u, xi);
        }
        const float rad = smax * cube_or_square_root<DIM>(((float)l + xi) * invL);
        float w[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < DIM; ++i) w[i] = fmaf(rad * u[i], inv_h[i], off[i]);
        point(rad, tap_load<DIM, CLAMP>(vol, anc, w), q1, q2);
    }
    if (cur_ray >= 0) flush(u, q1, q2);
}

// Run up to n_iter iterations of one contour, stopping early at iteration `target` or when it
// leaves SNK_ACTIVE. Every thread of the workgroup calls this with the same arguments.
template <int DIM, int WAVES, bool TRACE, int U, bool BUF>
__device__ void run_contour(const JobParams &p, DevContour *slot, int n_iter, int target, float *trace_row,
                            float *lds, int box_cap, unsigned long long *counter) {
    constexpr int T = 64 * WAVES;
    constexpr int NR = Smem<DIM, WAVES>::NR;
    constexpr float BALL = DIM == 3 ? 4.18879020478639098462f : 3.14159265358979323846f;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const DevContour s = *slot;
    const int n0 = __builtin_amdgcn_readfirstlane(s.iters);
    const int budget = min(n_iter, target - n0);
    if ((s.status & 0x0f) != SNK_ACTIVE || budget <= 0) return;

    const Smem<DIM, WAVES> sm(lds, p.D, p.M / 2);
    for (int i = t; i < p.D * DIM; i += T) sm.tdir[i] = p.dirs[i];
    const uint32_t id = __builtin_amdgcn_readfirstlane(s.id);
    produce<DIM, WAVES>(sm, 0, (uint32_t)(n0 + 1), id, p, wave, lane);
    __syncthreads();

    const Vol<DIM, BUF> vol(p.g);
    const float inv_h[3] = {p.g.inv_h[0], p.g.inv_h[1], p.g.inv_h[2]};
    const int nn[3] = {p.g.nx, p.g.ny, p.g.nz};
    int anc[3] = {s.anc[0], s.anc[1], s.anc[2]};
    float off[3] = {s.off[0], s.off[1], s.off[2]};
    float R = s.R;
    int n = n0;
    uint8_t status = s.status;
    int streak = s.streak;
    float e_mc = s.e_mc;
    const float inv_npts = 1.0f / (float)(p.M * p.L);
    const float tol2 = p.conv_tol * p.conv_tol;
    int ran = 0;
    // staged footprint: voxels [b.lo, b.lo + bn) of the volume, valid when `staged`
    Box<DIM> box;
    box.data = sm.box;
    int bn[3] = {1, 1, 1};
    bool staged = false;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        box.lo[i] = 0;
        box.n[i] = nn[i];
    }
    box.bx = box.bxy = 1;
    int margin[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < DIM; ++i) margin[i] = max(1, (int)ceilf(1.5f * inv_h[i]));

    for (int it = 0; it < budget; ++it) {
        n += 1;
        const int par = it & 1;
        const float smax = R + 0.5f * p.dR;
        const Weight<DIM> wt(R, p.dR, p.in_slope, p.out_slope);
        float Q[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) Q[i] = sm.rot[par * 9 + i];
        // clamping can be skipped when the whole sample ball (with a rounding margin) is interior
        bool interior = true;
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            const float ext = fmaf(smax * inv_h[i], 1.0001f, 1e-3f);
            interior = interior && (off[i] - ext > (float)(-anc[i])) && (off[i] + ext < (float)(nn[i] - 1 - anc[i]));
        }
        // voxel range this iteration's gathers touch (corner pairs included), clamped to the volume
        bool use_box = false;
        if (box_cap > 0) {
            int need_lo[3] = {0, 0, 0}, need_hi[3] = {0, 0, 0};
            bool inside = staged;
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                const float ext = fmaf(smax * inv_h[i], 1.0001f, 1e-3f);
                // clamped gathers use index pairs within [0, n-2] + 1, so keep at least one such pair
                need_lo[i] = max(0, min(nn[i] - 2, anc[i] + (int)floorf(off[i] - ext)));
                need_hi[i] = min(nn[i] - 1, max(1, anc[i] + (int)floorf(off[i] + ext) + 1));
                inside = inside && need_lo[i] >= box.lo[i] && need_hi[i] < box.lo[i] + bn[i];
            }
            if (!inside) {
                int lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
                long size = 1;
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    lo[i] = max(0, need_lo[i] - margin[i]);
                    cnt[i] = min(nn[i] - 1, need_hi[i] + margin[i]) - lo[i] + 1;
                    size *= cnt[i];
                }
                staged = size <= box_cap;
                if (staged) {
                    // every wave finished reading the old box before the previous iteration's barrier
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        box.lo[i] = lo[i];
                        bn[i] = cnt[i];
                    }
                    box.bx = cnt[0];
                    box.bxy = cnt[0] * cnt[1];
                    const int rows = cnt[1] * cnt[2];
                    for (int row = wave; row < rows; row += WAVES) {
                        const int y = row % cnt[1], z = row / cnt[1];
                        const float *src = p.g.J + ((long)(lo[2] + z) * nn[1] + (lo[1] + y)) * nn[0] + lo[0];
                        float *dst = sm.box + row * cnt[0];
                        for (int x = lane; x < cnt[0]; x += 64) dst[x] = src[x];
                    }
                    __syncthreads();
                }
            }
            use_box = staged;
        }
        float accA = 0.0f, accBR = 0.0f, accB[DIM];
#pragma unroll
        for (int i = 0; i < DIM; ++i) accB[i] = 0.0f;
        const int *rk = sm.rk + par * sm.MH;
        const float *rxi = sm.rxi + par * sm.MH;
        if (use_box) {
            if (interior)
                thread_sums<DIM, T, U, false>(box, inv_h, anc, off, wt, smax, Q, sm.tdir, rk, rxi, p.M, p.L, t, accA,
                                              accBR, accB);
            else
                thread_sums<DIM, T, U, true>(box, inv_h, anc, off, wt, smax, Q, sm.tdir, rk, rxi, p.M, p.L, t, accA,
                                             accBR, accB);
        } else {
            if (interior)
                thread_sums<DIM, T, U, false>(vol, inv_h, anc, off, wt, smax, Q, sm.tdir, rk, rxi, p.M, p.L, t, accA,
                                              accBR, accB);
            else
                thread_sums<DIM, T, U, true>(vol, inv_h, anc, off, wt, smax, Q, sm.tdir, rk, rxi, p.M, p.L, t, accA,
                                             accBR, accB);
        }
        // draws of the next iteration, published by the barrier below
        if (it + 1 < budget) produce<DIM, WAVES>(sm, 1 - par, (uint32_t)(n + 1), id, p, wave, lane);

        float tot[NR];
        tot[0] = wave_sum(accA);
        tot[1] = wave_sum(accBR);
#pragma unroll
        for (int i = 0; i < DIM; ++i) tot[2 + i] = wave_sum(accB[i]);
        float *slotp = sm.red + par * WAVES * NR;
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < NR; ++k) slotp[wave * NR + k] = tot[k];
        }
        __syncthreads();
        if constexpr (WAVES > 1) {
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                float v = slotp[k];
#pragma unroll
                for (int ww = 1; ww < WAVES; ++ww) v += slotp[ww * NR + k];
                tot[k] = v;
            }
        }

        // descent step, identical in every lane
        float smax_d = smax;
#pragma unroll
        for (int i = 1; i < DIM; ++i) smax_d *= smax;
        const float scale = BALL * smax_d * inv_npts;
        const float A = scale * tot[0];
        const float BR = scale * tot[1];
        const float inv2R = __builtin_amdgcn_rcpf(2.0f * R);
        float inv_norm = inv2R;
#pragma unroll
        for (int i = 1; i < DIM; ++i) inv_norm *= inv2R;
        const float E = A * inv_norm;
        const float gR = (BR - (2.0f * DIM) * inv2R * A) * inv_norm;
        const float eps = p.eps0 * __builtin_amdgcn_rsqf((float)n);
        const float half_eps = 0.5f * eps;
        const float dRs = -half_eps * gR;
        float dc[3] = {0.0f, 0.0f, 0.0f};
        float dc2 = 0.0f;
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            dc[i] = -half_eps * (scale * tot[2 + i]) * inv_norm;
            dc2 = fmaf(dc[i], dc[i], dc2);
        }
        if (TRACE && t == 0) {
            float *row = trace_row;
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
        if (Rn < p.r_lo) { Rn = p.r_lo; flag = SNK_CLAMPED; }
        if (Rn > p.r_hi) { Rn = p.r_hi; flag = SNK_CLAMPED; }
        const float dRe = Rn - R;
        const bool small = dRe * dRe < tol2 && dc2 < tol2;
        R = Rn;
        e_mc = E;
        bool finite = isfinite(Rn) && isfinite(E);
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            off[i] = fmaf(dc[i], inv_h[i], off[i]);
            finite = finite && isfinite(off[i]);
        }
        uint8_t st = SNK_ACTIVE;
        if (!finite) {
            st = SNK_NONFINITE;
        } else {
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
            streak = small ? min(streak + 1, 255) : 0;
            if (p.conv_window > 0 && streak >= p.conv_window) st = SNK_CONVERGED;
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
        *slot = o;
        atomicAdd(counter, (unsigned long long)ran);
    }
}

template <int DIM, int WAVES, bool TRACE, int U, bool BUF>
__global__ __launch_bounds__(64 * WAVES) void evolve_kernel(EvolveArgs a) {
    extern __shared__ float lds[];
    const int cid = blockIdx.x;
    run_contour<DIM, WAVES, TRACE, U, BUF>(a.p, a.st + cid, a.n_iter, 0x7fffffff,
                                           TRACE ? a.trace + (long)cid * SNK_TRACE_W : nullptr, lds, a.box_cap,
                                           a.counter);
}

// Copy of a record that every lane reads at the same address, forced into scalar registers (the
// table lives in memory the kernel also writes, so the compiler would otherwise keep it per lane).
template <typename T>
__device__ __forceinline__ T uniform_copy(const T *src) {
    static_assert(sizeof(T) % 4 == 0, "word-sized record");
    T out;
    const uint32_t *in = reinterpret_cast<const uint32_t *>(src);
    uint32_t *o = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) o[i] = __builtin_amdgcn_readfirstlane(in[i]);
    return out;
}

// Batched launch over (job, contour) items. PERSISTENT: a fixed grid pops items from a device
// work queue until it is exhausted (every workgroup reaches the exit); otherwise one workgroup
// per item.
template <int DIM, int WAVES, int U, bool BUF, bool PERSISTENT>
__global__ __launch_bounds__(64 * WAVES) void evolve_batch_kernel(BatchArgs a) {
    extern __shared__ float lds[];
    __shared__ int item_sh;
    if constexpr (PERSISTENT) {
        for (;;) {
            if (threadIdx.x == 0) item_sh = atomicAdd(a.queue, 1);
            __syncthreads();
            const int item = __builtin_amdgcn_readfirstlane(item_sh);
            __syncthreads();
            if (item >= a.n_items) break;
            const int job = __builtin_amdgcn_readfirstlane(a.items[item].x);
            const int cid = __builtin_amdgcn_readfirstlane(a.items[item].y);
            const JobParams p = uniform_copy(&a.jobs[job].p);
            DevContour *st = uniform_copy(&a.jobs[job].st);
            const int target = __builtin_amdgcn_readfirstlane(a.jobs[job].target);
            run_contour<DIM, WAVES, false, U, BUF>(p, st + cid, a.chunk, target, nullptr, lds, a.box_cap, a.counter);
            __syncthreads();
        }
    } else {
        const int item = blockIdx.x;
        if (item >= a.n_items) return;
        const int job = __builtin_amdgcn_readfirstlane(a.items[item].x);
        const int cid = __builtin_amdgcn_readfirstlane(a.items[item].y);
        const JobParams p = uniform_copy(&a.jobs[job].p);
        DevContour *st = uniform_copy(&a.jobs[job].st);
        const int target = __builtin_amdgcn_readfirstlane(a.jobs[job].target);
        run_contour<DIM, WAVES, false, U, BUF>(p, st + cid, a.chunk, target, nullptr, lds, a.box_cap, a.counter);
    }
}

template <int DIM, int WAVES>
size_t smem_bytes(int D, int M, int box_cap) {
    return Smem<DIM, WAVES>::bytes(D, M / 2, box_cap);
}

template <int DIM, int WAVES, bool TRACE, int U>
hipError_t launch_t(const EvolveArgs &a, hipStream_t s) {
    const size_t lds = smem_bytes<DIM, WAVES>(a.p.D, a.p.M, a.box_cap);
    if (a.p.buffer_ok)
        hipLaunchKernelGGL((evolve_kernel<DIM, WAVES, TRACE, U, true>), dim3(a.n), dim3(64 * WAVES), lds, s, a);
    else
        hipLaunchKernelGGL((evolve_kernel<DIM, WAVES, TRACE, U, false>), dim3(a.n), dim3(64 * WAVES), lds, s, a);
    return hipGetLastError();
}

int pick_unroll(int T, int M, int L, int unroll) {
    if (unroll > 0) return unroll >= 4 ? 4 : (unroll >= 2 ? 2 : 1);
    const int per = M <= T ? (L + T / M - 1) / (T / M) : L;
    return per >= 2 ? 2 : 1;
}

template <int DIM, int WAVES, bool TRACE>
hipError_t launch_u(const EvolveArgs &a, int unroll, hipStream_t s) {
    switch (pick_unroll(64 * WAVES, a.p.M, a.p.L, unroll)) {
        case 4: return launch_t<DIM, WAVES, TRACE, 4>(a, s);
        case 2: return launch_t<DIM, WAVES, TRACE, 2>(a, s);
        default: return launch_t<DIM, WAVES, TRACE, 1>(a, s);
    }
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

template <int DIM, int WAVES, int U, bool PERSISTENT>
hipError_t batch_t(const BatchArgs &a, int grid, hipStream_t s) {
    const size_t lds = smem_bytes<DIM, WAVES>(a.max_D, a.max_M, a.box_cap);
    const int g = PERSISTENT ? grid : a.n_items;
    if (g <= 0) return hipSuccess;
    hipLaunchKernelGGL((evolve_batch_kernel<DIM, WAVES, U, true, PERSISTENT>), dim3(g), dim3(64 * WAVES), lds, s, a);
    return hipGetLastError();
}

template <int DIM, int WAVES, int U>
hipError_t batch_p(const BatchArgs &a, bool persistent, int grid, hipStream_t s) {
    return persistent ? batch_t<DIM, WAVES, U, true>(a, grid, s) : batch_t<DIM, WAVES, U, false>(a, grid, s);
}

template <int DIM, int WAVES>
hipError_t batch_u(const BatchArgs &a, int unroll, bool persistent, int grid, hipStream_t s) {
    switch (unroll >= 4 ? 4 : (unroll >= 2 ? 2 : 1)) {
        case 4: return batch_p<DIM, WAVES, 4>(a, persistent, grid, s);
        case 2: return batch_p<DIM, WAVES, 2>(a, persistent, grid, s);
        default: return batch_p<DIM, WAVES, 1>(a, persistent, grid, s);
    }
}

template <int DIM>
hipError_t batch_w(const BatchArgs &a, int waves, int unroll, bool persistent, int grid, hipStream_t s) {
    switch (waves) {
        case 1: return batch_u<DIM, 1>(a, unroll, persistent, grid, s);
        case 2: return batch_u<DIM, 2>(a, unroll, persistent, grid, s);
        case 8: return batch_u<DIM, 8>(a, unroll, persistent, grid, s);
        default: return batch_u<DIM, 4>(a, unroll, persistent, grid, s);
    }
}

template <int DIM, int WAVES, int U>
int max_blocks_t(int max_D, int max_M, int box_cap) {
    int blocks = 0;
    const size_t lds = smem_bytes<DIM, WAVES>(max_D, max_M, box_cap);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, evolve_batch_kernel<DIM, WAVES, U, true, true>,
                                                     64 * WAVES, lds) != hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

template <int DIM, int WAVES>
int max_blocks_u(int unroll, int max_D, int max_M, int box_cap) {
    switch (unroll >= 4 ? 4 : (unroll >= 2 ? 2 : 1)) {
        case 4: return max_blocks_t<DIM, WAVES, 4>(max_D, max_M, box_cap);
        case 2: return max_blocks_t<DIM, WAVES, 2>(max_D, max_M, box_cap);
        default: return max_blocks_t<DIM, WAVES, 1>(max_D, max_M, box_cap);
    }
}

template <int DIM>
int max_blocks_w(int waves, int unroll, int max_D, int max_M, int box_cap) {
    switch (waves) {
        case 1: return max_blocks_u<DIM, 1>(unroll, max_D, max_M, box_cap);
        case 2: return max_blocks_u<DIM, 2>(unroll, max_D, max_M, box_cap);
        case 8: return max_blocks_u<DIM, 8>(unroll, max_D, max_M, box_cap);
        default: return max_blocks_u<DIM, 4>(unroll, max_D, max_M, box_cap);
    }
}

}  // namespace

hipError_t launch_evolve(const EvolveArgs &a, int dim, int waves, int unroll, bool trace, hipStream_t s) {
    if (a.n <= 0 || a.n_iter <= 0) return hipSuccess;
    if (dim == 2) return trace ? launch_w<2, true>(a, waves, unroll, s) : launch_w<2, false>(a, waves, unroll, s);
    return trace ? launch_w<3, true>(a, waves, unroll, s) : launch_w<3, false>(a, waves, unroll, s);
}

// Batched launches always use buffer loads (every job's volume must fit 2 GiB).
hipError_t launch_evolve_batch(const BatchArgs &a, int dim, int waves, int unroll, bool persistent, int grid,
                               hipStream_t s) {
    if (a.n_items <= 0 || a.chunk <= 0) return hipSuccess;
    if (dim == 2) return batch_w<2>(a, waves, unroll, persistent, grid, s);
    return batch_w<3>(a, waves, unroll, persistent, grid, s);
}

int evolve_batch_max_blocks(int dim, int waves, int unroll, int max_D, int max_M, int box_cap) {
    return dim == 2 ? max_blocks_w<2>(waves, unroll, max_D, max_M, box_cap)
                    : max_blocks_w<3>(waves, unroll, max_D, max_M, box_cap);
}

size_t evolve_lds_bytes(int dim, int waves, int D, int M, int box_cap) {
    const int w = waves == 1 || waves == 2 || waves == 8 ? waves : 4;
    const int nr = 2 + dim;
    return sizeof(float) * ((size_t)D * dim + 18 + 4 * (M / 2) + 2 * w * nr + (size_t)box_cap);
}

int evolve_box_cap(int requested, int dim, int waves, int D, int M, const snk_params &P) {
    if (requested < 0) return 0;
    const size_t limit = 65536;  // dynamic LDS of one workgroup
    const size_t base = evolve_lds_bytes(dim, waves, D, M, 0);
    if (base + 4096 >= limit) return 0;
    const int maxcap = (int)((limit - base) / 4);
    if (requested > 0) return requested < maxcap ? requested : maxcap;
    const double R = P.r_max < 1.5 * P.r_init ? P.r_max : 1.5 * P.r_init;
    const double smax = R + 0.5 * P.dR;
    long size = 1;
    for (int a = 0; a < dim; ++a) {
        const double inv_h = 1.0 / P.spacing[a];
        const int margin = (int)ceil(1.5 * inv_h) > 1 ? (int)ceil(1.5 * inv_h) : 1;
        size *= 2 * (long)ceil(smax * inv_h) + 3 + 2 * margin;
    }
    return size < maxcap ? (int)size : maxcap;
}

}  // namespace snk
