// Evolution kernel: gradient descent of independent snakuscules with Monte-Carlo sums.
//
// A group of G lanes owns one contour and runs its iterations back to back; contours are
// independent during evolution (Sec. II-D), so there is no grid-wide synchronisation. G is 16 or 32
// (several contours share one wave64), 64 (one wave per contour) or 128/256 (a workgroup of 2/4
// waves per contour). Per iteration n the group
//   1. reads, for each antithetic pair m, the ray direction u = Q(n) T[k] already divided by the
//      voxel spacing, and the radial jitter xi. These are state-independent: the Philox4x32-10 draws
//      (rotation Q(n) at counter (0, n, id, 0), Shoemake's uniform quaternion in 3D or an angle in
//      2D; table row k = floor(x0 D / 2^32) and xi from counter (m, n, id, 1)) are produced for a
//      block of K iterations at once by all lanes of the group, one draw per lane, and the
//      rotations are applied in the following iteration, so each costs about 1/K of a draw per lane
//      and iteration;
//   2. walks pair-points (m, l): both rays +u and -u at the common radius
//      s = s_max ((l + xi)/L)^(1/d), s_max = R + dR/2 (uniform in the ball, Sec. II-E), issuing the
//      trilinear (bilinear) gathers of both points before consuming them. The two points share the
//      radius, hence S and its ramp memberships;
//   3. evaluates the four-region weight S (Sec. II-B, Eq. (5)) and accumulates
//      A = sum S I, B_R = sum dS/dR I and B_c = -sum dS/dr I u (per pair: the ramp coefficient times
//      I(+u) + I(-u) for A and B_R, times I(+u) - I(-u) for B_c; B_c is kept in voxel units);
//   4. reduces the sums in a fixed order (DPP row shifts/rotations inside a wave, then per-wave
//      partials in wave order through LDS), so every lane of the group holds identical totals;
//   5. applies the descent step of Eqs. (7)-(15) in (c, R) form: E = A/(2R)^d,
//      dE/dR = (B_R - (d/R) A)/(2R)^d, dE/dc = B_c/(2R)^d, eps = eps0/sqrt(n),
//      dR = -(eps/2) dE/dR, dc = -(eps/2) dE/dc (the p,q steps of Eqs. (12)-(15) mapped through
//      c = (p+q)/2, R = (q_x - p_x)/2), clamps R, re-anchors c, and tests OUT / convergence.
// Every lane of a group runs the identical update, so the state stays in registers.
//
// Volume layouts: plain FP32 [z][y][x] (2^d/2 eight-byte pair loads per point), or "quad": one
// 16-byte record per voxel holding J(x,y), J(x+1,y), J(x,y+1), J(x+1,y+1) of its plane (one 16-byte
// load per point in 2D, two in 3D). Both hold exact copies of the smoothed volume.
//
// Two launches share the per-contour routine: one group per contour of a single volume, and a
// batched launch over a device table of (job, contour) items (one workgroup per item, optionally
// persistent with a work queue).
#include <math.h>

#include "snk_internal.h"

namespace snk {

namespace {

constexpr uint32_t kBufferWord3 = 0x00020000u;  // raw buffer descriptor, gfx9 family

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// The rounds stay a loop: unrolled, the compiler keeps all twenty round keys in scalar registers for
// the whole kernel and spills other uniform values to make room.
__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                         uint32_t k1, uint32_t out[4]) {
#pragma unroll 1
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
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

// Rotation Q (row-major, acting on column vectors) from the Philox words of counter (0, n, id, 0).
// Evaluated operation by operation (no multiply-add contraction), so every kernel instance and build
// rounds it alike.
template <int DIM>
__device__ __forceinline__ void rotation_from(const uint32_t x[4], float Q[9]) {
#pragma clang fp contract(off)
    if constexpr (DIM == 2) {
        float s, c;
        sincospif(2.0f * unit_open(x[0]), &s, &c);
        Q[0] = c;
        Q[1] = -s;
        Q[2] = 0.0f;
        Q[3] = s;
        Q[4] = c;
        Q[5] = 0.0f;
        Q[6] = 0.0f;
        Q[7] = 0.0f;
        Q[8] = 1.0f;
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

// ---------------------------------------------------------------------------------------------
// Group shape and LDS layout
// ---------------------------------------------------------------------------------------------

template <int G>
struct Grp {
    static constexpr int NT = G < 64 ? 64 : G;       // threads per workgroup
    static constexpr int CPB = G < 64 ? 64 / G : 1;  // contours per workgroup
    static constexpr int WAVES = NT / 64;
};

// Iterations per block of draws. A block takes ceil(K (MH + 1) / G) rounds of one draw per lane;
// K is the smallest block size (at least two: the rotation of a block is applied one iteration
// after its draws) whose rounds per iteration come within 30% of the ideal (MH + 1) / G, else the
// one with the fewest rounds per iteration.
__host__ __device__ __forceinline__ int block_iters(int G, int MH) {
    const int per = MH + 1;
    int best = 2;
    float best_cost = 1e30f;
    for (int K = 2; K <= 16; ++K) {
        const float cost = (float)((K * per + G - 1) / G) / (float)K;
        if (cost * (float)G <= 1.3f * (float)per) return K;
        if (cost < best_cost) {
            best_cost = cost;
            best = K;
        }
    }
    return best;
}

// Floats of one contour's draw buffers (two blocks), a multiple of 4.
__host__ __device__ __forceinline__ int draw_floats(int G, int MH) {
    const int K = block_iters(G, MH);
    return 2 * K * (4 * MH + 12);
}

// One contour's draw buffers: for each of 2 blocks x K iterations,
//   pu[m] = (u_x/h_x, u_y/h_y, u_z/h_z, xi) per pair m (between the two phases pu[m].x holds the
//   table row k), rot = Q (9 floats, 12 reserved).
struct Draws {
    float4 *pu;
    float *rot;
    int K, MH;
    __device__ __forceinline__ Draws(float *base, int G, int MH_) {
        MH = MH_;
        K = block_iters(G, MH_);
        pu = reinterpret_cast<float4 *>(base);
        rot = base + 2 * K * 4 * MH;
    }
    __device__ __forceinline__ int slot(int buf, int s) const { return buf * K + s; }
};

// j -> (j / d, j % d) for small j, without an integer division.
__device__ __forceinline__ void divmod_small(int j, int d, float inv_d, int &q, int &r) {
    q = (int)(((float)j + 0.5f) * inv_d);
    r = j - q * d;
    if (r < 0) {
        q -= 1;
        r += d;
    } else if (r >= d) {
        q += 1;
        r -= d;
    }
}

// Phase 1 of block b: the Philox draws of its K iterations (n_first .. n_first + K - 1), one per
// lane: pair draws -> table row k (parked in pu.x) and xi; rotation draws -> Q.
template <int DIM, int G>
__device__ __forceinline__ void draws_phase1(const Draws &d, int buf, uint32_t n_first, uint32_t id,
                                             const JobParams &p, int gl) {
    const int per = d.MH + 1;
    const int total = d.K * per;
    const float inv = 1.0f / (float)per;
    for (int j = gl; j < total; j += G) {
        int s, r;
        divmod_small(j, per, inv, s, r);
        const bool pair = r < d.MH;
        uint32_t x[4];
        philox10(pair ? (uint32_t)r : 0u, n_first + (uint32_t)s, id, pair ? 1u : 0u, p.key0, p.key1, x);
        const int sl = d.slot(buf, s);
        if (pair) {
            d.pu[sl * d.MH + r].x = __int_as_float((int)__umulhi(x[0], (uint32_t)p.D));
            d.pu[sl * d.MH + r].w = unit_open(x[1]);
        } else {
            float Q[9];
            if (p.flags & 1) {
#pragma unroll
                for (int i = 0; i < 9; ++i) Q[i] = (i % 4 == 0) ? 1.0f : 0.0f;
            } else {
                rotation_from<DIM>(x, Q);
            }
#pragma unroll
            for (int i = 0; i < 9; ++i) d.rot[sl * 12 + i] = Q[i];
        }
    }
}

// Phase 2 of block b (one iteration after phase 1): u = Q T[k] / h for every pair of the block.
template <int DIM, int G>
__device__ __forceinline__ void draws_phase2(const Draws &d, int buf, const JobParams &p, int gl) {
    const int total = d.K * d.MH;
    const float inv = 1.0f / (float)d.MH;
    for (int j = gl; j < total; j += G) {
        int s, m;
        divmod_small(j, d.MH, inv, s, m);
        const int sl = d.slot(buf, s);
        float4 &o = d.pu[sl * d.MH + m];
        const int k = __float_as_int(o.x);
        const float *Q = d.rot + sl * 12;
        float t[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < DIM; ++i) t[i] = p.dirs[k * DIM + i];
        float u[3];
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            float acc = 0.0f;
#pragma unroll
            for (int jj = 0; jj < DIM; ++jj) acc = fmaf(Q[i * 3 + jj], t[jj], acc);
            u[i] = acc * p.g.inv_h[i];
        }
        o.x = u[0];
        o.y = u[1];
        o.z = DIM == 3 ? u[2] : 0.0f;
    }
}

// ---------------------------------------------------------------------------------------------
// Reductions (fixed order; every lane of a group ends with identical totals)
// ---------------------------------------------------------------------------------------------

template <int CTRL, int ROWS = 0xf, bool BC = true>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, BC));
}

// Butterfly over the 16 lanes of a DPP row (rotations are symmetric, so all lanes agree bitwise).
__device__ __forceinline__ float row_sum16(float v) {
    v += dpp<0x128>(v);  // row_ror:8
    v += dpp<0x124>(v);  // row_ror:4
    v += dpp<0x122>(v);  // row_ror:2
    v += dpp<0x121>(v);  // row_ror:1
    return v;
}

// Sum of the wave in lane 63 (row shifts, then row broadcasts).
__device__ __forceinline__ float wave_sum_to_63(float v) {
    v += dpp<0x111>(v);             // row_shr:1
    v += dpp<0x112>(v);             // row_shr:2
    v += dpp<0x114>(v);             // row_shr:4
    v += dpp<0x118>(v);             // row_shr:8
    v += dpp<0x142, 0xa, false>(v); // row_bcast:15
    v += dpp<0x143, 0xc, false>(v); // row_bcast:31
    return v;
}

// Maximum of the wave in lane 63 (row shifts, then row broadcasts; values are >= 0 here, so the
// zero filled in by the shifts is harmless).
__device__ __forceinline__ float wave_max_to_63(float v) {
    v = fmaxf(v, dpp<0x111>(v));             // row_shr:1
    v = fmaxf(v, dpp<0x112>(v));             // row_shr:2
    v = fmaxf(v, dpp<0x114>(v));             // row_shr:4
    v = fmaxf(v, dpp<0x118>(v));             // row_shr:8
    v = fmaxf(v, dpp<0x142, 0xa, false>(v)); // row_bcast:15
    v = fmaxf(v, dpp<0x143, 0xc, false>(v)); // row_bcast:31
    return v;
}

// Adds a value's copies in the two halves of the wave (lane i and lane i ^ 32), then in the two rows
// of each half (lane i and lane i ^ 16); both partners add the same two operands in the same order.
__device__ __forceinline__ float cross_row_sum(float x) {
    auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    const float y = __uint_as_float(h[0]) + __uint_as_float(h[1]);   // x[i mod 32] + x[32 + i mod 32]
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(y), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);            // even row + odd row of the half
}

// Totals over the 64 lanes of a wave of NR = 4 or 5 per-lane values, in scalar registers. Values 0..3
// are reduced together: lanes exchange values so that after two quad steps each lane holds the
// quad's sum of one value, j = 2 (lane & 1) + ((lane >> 1) & 1); the row and cross-row steps then
// add the copies of that value (the same value sits in lanes i, i + 4, i + 8, ...). A fifth value
// takes the same row and cross-row steps on its own. The order of every addition is fixed, so the
// totals do not depend on timing.
template <int NR>
__device__ __forceinline__ void wave_sums(const float *v, float *tot) {
    static_assert(NR == 4 || NR == 5, "four or five sums");
    const int lane = __lane_id();
    const bool b0 = (lane & 1) != 0, b1 = (lane & 2) != 0;
    // lane pairs (2i, 2i + 1): the even lane keeps values 0 and 1, the odd one 2 and 3
    const float k0 = b0 ? v[2] : v[0], k1 = b0 ? v[3] : v[1];
    const float s0 = b0 ? v[0] : v[2], s1 = b0 ? v[1] : v[3];
    const float w0 = k0 + dpp<0xB1>(s0);   // quad_perm [1, 0, 3, 2]
    const float w1 = k1 + dpp<0xB1>(s1);
    // lanes i and i ^ 2: keep w_b1, add the partner's copy of the same value
    const float keep = b1 ? w1 : w0, send = b1 ? w0 : w1;
    float x = keep + dpp<0x4E>(send);     // quad_perm [2, 3, 0, 1]
    float z = 0.0f;
    if constexpr (NR == 5) {
        z = v[4] + dpp<0xB1>(v[4]);
        z = z + dpp<0x4E>(z);
    }
    x += dpp<0x128>(x);                   // row_ror:8
    x += dpp<0x124>(x);                   // row_ror:4
    if constexpr (NR == 5) {
        z += dpp<0x128>(z);
        z += dpp<0x124>(z);
    }
    x = cross_row_sum(x);
    // value j's total sits in lane 0 (j = 0), 2 (j = 1), 1 (j = 2), 3 (j = 3)
    tot[0] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
    tot[1] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 2));
    tot[2] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 1));
    tot[3] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 3));
    if constexpr (NR == 5) {
        z = cross_row_sum(z);
        tot[4] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(z)));
    }
}

template <int G>
__device__ __forceinline__ float group_sum_wave(float v) {
    if constexpr (G == 16) {
        return row_sum16(v);
    } else if constexpr (G == 32) {
        v = row_sum16(v);
        return v + __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));  // lane ^ 16
    } else {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_sum_to_63(v)), 63));
    }
}

// ---------------------------------------------------------------------------------------------
// Volume access
// ---------------------------------------------------------------------------------------------

struct __attribute__((packed, aligned(4))) Pair {
    float lo, hi;
};

// The 2^d corner values of one trilinear (bilinear) sample, in the order
// v000 v100 v010 v110 v001 v101 v011 v111.
template <int DIM>
struct Corners {
    float v[DIM == 3 ? 8 : 4];
};

template <int DIM, int LAYOUT>
struct Vol {
    static constexpr bool kSmall = LAYOUT != kGlobalPlain;  // 24-bit index arithmetic
    const float *J;
    __amdgpu_buffer_rsrc_t rsrc;
    int n[3];
    int nx, nxy;
    int so1, so2, so3;  // byte offsets of the neighbour loads (buffer layouts)
    __device__ __forceinline__ Vol(const Geometry &g) {
        n[0] = g.nx;
        n[1] = g.ny;
        n[2] = g.nz;
        nx = g.nx;
        nxy = g.nx * g.ny;
        J = g.J;
        so1 = so2 = so3 = 0;
        if constexpr (LAYOUT == kBufferPlain) {
            so1 = nx * 4;
            so2 = nxy * 4;
            so3 = (nxy + nx) * 4;
            rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)g.J, (short)0, (int)((long)nxy * g.nz * 4),
                                                     (int)kBufferWord3);
        } else if constexpr (LAYOUT == kBufferQuad) {
            so2 = nxy * 16;
            rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)g.Jq, (short)0, (int)((long)nxy * g.nz * 16),
                                                     (int)kBufferWord3);
        } else if constexpr (LAYOUT == kBufferPair) {
            so2 = nxy * 8;
            rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)g.Jq, (short)0, (int)((long)nxy * (DIM == 3 ? g.nz : 1) * 8),
                                                     (int)kBufferWord3);
        }
    }
    // One voxel value (plain layouts).
    __device__ __forceinline__ float load1(long idx) const {
        if constexpr (LAYOUT == kBufferPlain) {
            return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)idx * 4, 0, 0));
        } else if constexpr (LAYOUT == kBufferPair) {
            return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)idx * 8, 0, 0));
        } else {
            return J[idx];
        }
    }
    // Loads the corners of the cell whose lower corner has linear voxel index `idx` (< 2^31 for
    // the buffer layouts).
    __device__ __forceinline__ void load(long idx, Corners<DIM> &c) const {
        if constexpr (LAYOUT == kBufferQuad) {
            const int vo = (int)idx * 16;
            const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(rsrc, vo, 0, 0);
            c.v[0] = __uint_as_float(a.x);
            c.v[1] = __uint_as_float(a.y);
            c.v[2] = __uint_as_float(a.z);
            c.v[3] = __uint_as_float(a.w);
            if constexpr (DIM == 3) {
                const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(rsrc, vo, so2, 0);
                c.v[4] = __uint_as_float(b.x);
                c.v[5] = __uint_as_float(b.y);
                c.v[6] = __uint_as_float(b.z);
                c.v[7] = __uint_as_float(b.w);
            }
        } else if constexpr (LAYOUT == kBufferPair) {
            // (J(x,y), J(x,y+1)) then (J(x+1,y), J(x+1,y+1)), of plane z and then of plane z+1
            const int vo = (int)idx * 8;
            const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(rsrc, vo, 0, 0);
            c.v[0] = __uint_as_float(a.x);
            c.v[2] = __uint_as_float(a.y);
            c.v[1] = __uint_as_float(a.z);
            c.v[3] = __uint_as_float(a.w);
            if constexpr (DIM == 3) {
                const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(rsrc, vo, so2, 0);
                c.v[4] = __uint_as_float(b.x);
                c.v[6] = __uint_as_float(b.y);
                c.v[5] = __uint_as_float(b.z);
                c.v[7] = __uint_as_float(b.w);
            }
        } else if constexpr (LAYOUT == kBufferPlain) {
            const int vo = (int)idx * 4;
            const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(rsrc, vo, 0, 0);
            const u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(rsrc, vo, so1, 0);
            c.v[0] = __uint_as_float(a.x);
            c.v[1] = __uint_as_float(a.y);
            c.v[2] = __uint_as_float(b.x);
            c.v[3] = __uint_as_float(b.y);
            if constexpr (DIM == 3) {
                const u32x2 e = __builtin_amdgcn_raw_buffer_load_b64(rsrc, vo, so2, 0);
                const u32x2 f = __builtin_amdgcn_raw_buffer_load_b64(rsrc, vo, so3, 0);
                c.v[4] = __uint_as_float(e.x);
                c.v[5] = __uint_as_float(e.y);
                c.v[6] = __uint_as_float(f.x);
                c.v[7] = __uint_as_float(f.y);
            }
        } else {
            const float *q = J + idx;
            const Pair a = *reinterpret_cast<const Pair *>(q);
            const Pair b = *reinterpret_cast<const Pair *>(q + nx);
            c.v[0] = a.lo;
            c.v[1] = a.hi;
            c.v[2] = b.lo;
            c.v[3] = b.hi;
            if constexpr (DIM == 3) {
                const Pair e = *reinterpret_cast<const Pair *>(q + nxy);
                const Pair f = *reinterpret_cast<const Pair *>(q + (long)nxy + nx);
                c.v[4] = e.lo;
                c.v[5] = e.hi;
                c.v[6] = f.lo;
                c.v[7] = f.hi;
            }
        }
    }
};

// Corner reads from a box of the smoothed volume staged in LDS (x fastest; nx = box row length,
// nxy = box plane size). Indices are relative to the box, so they stay small.
template <int DIM>
struct TileVol {
    static constexpr bool kSmall = true;
    const float *t;
    int n[3];
    int nx, nxy;
    __device__ __forceinline__ void load(long idx, Corners<DIM> &c) const {
        const float *q = t + (int)idx;
        c.v[0] = q[0];
        c.v[1] = q[1];
        c.v[2] = q[nx];
        c.v[3] = q[nx + 1];
        if constexpr (DIM == 3) {
            const float *r = q + nxy;
            c.v[4] = r[0];
            c.v[5] = r[1];
            c.v[6] = r[nx];
            c.v[7] = r[nx + 1];
        }
    }
};

template <int DIM>
__device__ __forceinline__ float trilerp(const Corners<DIM> &c, const float f[3]) {
    const float a0 = fmaf(f[0], c.v[1] - c.v[0], c.v[0]);
    const float a1 = fmaf(f[0], c.v[3] - c.v[2], c.v[2]);
    const float b0 = fmaf(f[1], a1 - a0, a0);
    if constexpr (DIM == 2) {
        return b0;
    } else {
        const float a2 = fmaf(f[0], c.v[5] - c.v[4], c.v[4]);
        const float a3 = fmaf(f[0], c.v[7] - c.v[6], c.v[6]);
        const float b1 = fmaf(f[1], a3 - a2, a2);
        return fmaf(f[2], b1 - b0, b0);
    }
}

// Trilinear (bilinear) value with the same operations as trilerp, and its gradient with respect to
// the voxel coordinates in the same cell.
template <int DIM>
__device__ __forceinline__ float trilerp_grad(const Corners<DIM> &c, const float f[3], float g[3]) {
    const float d0 = c.v[1] - c.v[0], d1 = c.v[3] - c.v[2];
    const float a0 = fmaf(f[0], d0, c.v[0]);
    const float a1 = fmaf(f[0], d1, c.v[2]);
    const float e0 = a1 - a0;
    const float b0 = fmaf(f[1], e0, a0);
    const float q0 = fmaf(f[1], d1 - d0, d0);
    if constexpr (DIM == 2) {
        g[0] = q0;
        g[1] = e0;
        g[2] = 0.0f;
        return b0;
    } else {
        const float d2 = c.v[5] - c.v[4], d3 = c.v[7] - c.v[6];
        const float a2 = fmaf(f[0], d2, c.v[4]);
        const float a3 = fmaf(f[0], d3, c.v[6]);
        const float e1 = a3 - a2;
        const float b1 = fmaf(f[1], e1, a2);
        const float q1 = fmaf(f[1], d3 - d2, d2);
        const float gz = b1 - b0;
        g[0] = fmaf(f[2], q1 - q0, q0);
        g[1] = fmaf(f[2], e1 - e0, e0);
        g[2] = gz;
        return fmaf(f[2], gz, b0);
    }
}

// Per-contour quantities of one iteration that the sampler reads.
template <int DIM>
struct Frame {
    int anc[3];
    float off[3];
    long base;     // linear index of the anchor voxel
    float smax;
    // weight S(r; R) (Sec. II-B): inner core -1 up to rho R - dr/2, ramp of width dr = rho dR, shell
    // +1 up to R - dR/2, outer ramp of width dR down to 0 at R + dR/2; half-open intervals
    float ain, R;          // centres of the inner and outer ramps
    float hd, hD;          // half widths dr/2 and dR/2
    float is, os;          // ramp slopes 2/dr and 1/dR
    float rho_is;          // rho * is
};

// floor(x) as an integer in one instruction (|x| far below 2^31 here).
__device__ __forceinline__ int floor_to_int(float x) {
    int i;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(i) : "v"(x));
    return i;
}

// Point x = anchor + off + rad * du (voxel units) -> corner index and fractions. CLAMP = false is
// used only when every sample of the iteration is known to lie inside, where both agree. SMALL: the
// row and plane strides fit 24-bit multiplies (buffer layouts).
// out (CLAMP only, may be null): per axis 0.0 where the coordinate lies beyond the volume's faces
// (the clamped interpolant is flat there), else 1.0; the last face itself counts as inside.
template <int DIM, bool CLAMP, bool SMALL>
__device__ __forceinline__ long locate(const Frame<DIM> &fr, const int n[3], int nx, int nxy, const float w[3],
                                       float f[3], float *in = nullptr) {
    if constexpr (!CLAMP) {
        int i[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            i[a] = floor_to_int(w[a]);
            f[a] = __builtin_amdgcn_fractf(w[a]);
        }
        if constexpr (SMALL) {
            int rel = __mul24(i[1], nx) + i[0];
            if constexpr (DIM == 3) rel += __mul24(i[2], nxy);
            return fr.base + rel;
        } else {
            long rel = (long)i[1] * nx + i[0];
            if constexpr (DIM == 3) rel += (long)i[2] * nxy;
            return fr.base + rel;
        }
    } else {
        long idx = 0;
        const long stride[3] = {1, nx, nxy};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const float fl = floorf(w[a]);
            int i = fr.anc[a] + (int)fl;
            float fa = w[a] - fl;
            if (in) in[a] = (i < 0 || i > n[a] - 1 || (i == n[a] - 1 && fa > 0.0f)) ? 0.0f : 1.0f;
            if (i < 0) {
                i = 0;
                fa = 0.0f;
            } else if (i > n[a] - 2) {
                i = n[a] - 2;
                fa = 1.0f;
            }
            f[a] = fa;
            idx += (long)i * stride[a];
        }
        return idx;
    }
}

template <int DIM>
__device__ __forceinline__ float cube_or_square_root(float tau) {
    if constexpr (DIM == 3) {
        // tau in (0, 1), never denormal: 2^(log2(tau)/3) on the transcendental unit
        return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(tau) * 0.333333343267f);
    } else {
        return __builtin_amdgcn_sqrtf(tau);
    }
}

// Sums of one lane for one iteration over pair-points q = gl, gl + G, ... < P (pair m = q / L,
// radial index l = q % L), U pair-points in flight.
// FULL: L divides G and G U divides P, so every pass of every lane holds U valid pair-points, all at
// the lane's radial index l0 (pairs m0 + k G / L), and the passes are uniform: no per-pair-point
// index stepping or validity tests. The arithmetic of each pair-point is the same in both forms.
// GRADI: the centre sums are sum S grad I (voxel-coordinate gradient of the interpolant, zero along
// axes beyond a face) instead of sum -dS/dr I u / h.
template <int DIM, int G, int U, bool CLAMP, bool GRADI = false, bool FULL = false, typename V>
__device__ __forceinline__ void lane_sums(const V &vol, const Frame<DIM> &fr, const float4 *pu,
                                          int P, int L, float invL, int gl, int l0, int m0, int dl, int dm,
                                          float acc[2 + DIM]) {
    int l = l0, m = m0;
    const float lf = (float)l0;
    for (int q = FULL ? 0 : gl; q < P; q += G * U) {
        Corners<DIM> cp[U], cm[U];
        float fp[U][3], fm[U][3], d1s[U], d2s[U];
        float inp[U][3], inm[U][3];
        int mk[U];
        bool ok[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if constexpr (FULL) {
                ok[k] = true;
                mk[k] = m + k * dm;
            } else {
                ok[k] = q + k * G < P;
                mk[k] = ok[k] ? m : 0;
            }
            const float4 d = pu[mk[k]];
            const float tau = ((FULL ? lf : (float)l) + d.w) * invL;
            const float e = cube_or_square_root<DIM>(tau);
            const float rad = fr.smax * e;
            // offsets from the ramp centres, fused explicitly so every instance rounds them alike
            d1s[k] = fmaf(fr.smax, e, -fr.ain);
            d2s[k] = fmaf(fr.smax, e, -fr.R);
            float wp[3] = {0.0f, 0.0f, 0.0f}, wm[3] = {0.0f, 0.0f, 0.0f};
            const float du[3] = {d.x, d.y, d.z};
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                wp[a] = fmaf(rad, du[a], fr.off[a]);
                wm[a] = fmaf(-rad, du[a], fr.off[a]);
            }
            constexpr bool SMALL = V::kSmall;
            const long ip = locate<DIM, CLAMP, SMALL>(fr, vol.n, vol.nx, vol.nxy, wp, fp[k],
                                                      GRADI && CLAMP ? inp[k] : nullptr);
            const long im = locate<DIM, CLAMP, SMALL>(fr, vol.n, vol.nx, vol.nxy, wm, fm[k],
                                                      GRADI && CLAMP ? inm[k] : nullptr);
            vol.load(ip, cp[k]);
            vol.load(im, cm[k]);
            if constexpr (!FULL) {
                l += dl;
                m += dm;
                if (l >= L) {
                    l -= L;
                    m += 1;
                }
            }
        }
        if constexpr (FULL) m += U * dm;
        // branch-free: a pair-point past P (it read pair 0, in bounds) gets zero weights, so its
        // gathers are consumed unconditionally and those of all U pair-points stay in flight
        // together
#pragma unroll
        for (int k = 0; k < U; ++k) {
            float gp[3], gm[3];
            const float Ip = GRADI ? trilerp_grad<DIM>(cp[k], fp[k], gp) : trilerp<DIM>(cp[k], fp[k]);
            const float Im = GRADI ? trilerp_grad<DIM>(cm[k], fm[k], gm) : trilerp<DIM>(cm[k], fm[k]);
            const float d1 = d1s[k], d2 = d2s[k];
            const bool r1 = d1 >= -fr.hd && d1 < fr.hd;   // inner ramp
            const bool r2 = d2 >= -fr.hD && d2 < fr.hD;   // outer ramp
            const float sin_ = __builtin_amdgcn_fmed3f(d1 * fr.is, -1.0f, 1.0f);
            const float sout = __builtin_amdgcn_fmed3f(fmaf(-d2, fr.os, 0.5f), 0.0f, 1.0f);
            // the inner profile is +1 wherever the outer one is below 1 (R >= the geometric
            // minimum keeps the regions disjoint), and vice versa
            const float S = ok[k] ? fminf(sin_, sout) : 0.0f;
            const float cC = ok[k] ? (r1 ? fr.is : (r2 ? -fr.os : 0.0f)) : 0.0f;  // dS/dr on the ramps
            const float cR = ok[k] ? (r1 ? -fr.rho_is : -cC) : 0.0f;               // dS/dR on the ramps
            const float Is = Ip + Im, Id = Ip - Im;
            acc[0] = fmaf(S, Is, acc[0]);
            acc[1] = fmaf(cR, Is, acc[1]);
            if constexpr (GRADI) {
                // both points share the radius, hence S
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    const float gsum = CLAMP ? fmaf(gp[a], inp[k][a], gm[a] * inm[k][a]) : gp[a] + gm[a];
                    acc[2 + a] = fmaf(S, gsum, acc[2 + a]);
                }
            } else {
                const float g = cC * Id;
                const float4 d = pu[mk[k]];
                acc[2] = fmaf(-g, d.x, acc[2]);
                acc[3] = fmaf(-g, d.y, acc[3]);
                if constexpr (DIM == 3) acc[4] = fmaf(-g, d.z, acc[4]);
            }
        }
    }
}

// Exact sums of one lane (flags bit 1): the lattice points of the box around the ball of radius
// s_max, those inside the ball counted (the point set of Eq. (5)), I = J at the voxel itself
// (clamp-to-edge outside the volume when CLAMP). Box points q = gl, gl + G, ..., x fastest; P
// points are evaluated per pass with their loads issued first.
template <int DIM, int G, bool CLAMP, int LAYOUT>
__device__ __forceinline__ void lattice_sums(const Vol<DIM, LAYOUT> &vol, const Frame<DIM> &fr, const float hh[3],
                                             const float inv_h[3], int gl, float acc[2 + DIM]) {
    constexpr int P = 4;
    int lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const float e = fr.smax * inv_h[a];
        lo[a] = (int)ceilf(fr.off[a] - e);
        cnt[a] = (int)floorf(fr.off[a] + e) - lo[a] + 1;
    }
    const int total = cnt[0] * cnt[1] * cnt[2];
    int x = gl % cnt[0], y = (gl / cnt[0]) % cnt[1], z = gl / (cnt[0] * cnt[1]);
    const int sx = G % cnt[0], sy = G / cnt[0];
    const float smax2 = fr.smax * fr.smax;
    for (int q0 = gl; q0 < total; q0 += G * P) {
        float I[P], d[P][3], r2[P];
        bool in[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int j[3] = {lo[0] + x, lo[1] + y, lo[2] + z};
            x += sx;
            if (x >= cnt[0]) {
                x -= cnt[0];
                y += 1;
            }
            y += sy;
            while (y >= cnt[1]) {
                y -= cnt[1];
                z += 1;
            }
            r2[k] = 0.0f;
            d[k][0] = d[k][1] = d[k][2] = 0.0f;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                d[k][a] = ((float)j[a] - fr.off[a]) * hh[a];
                r2[k] = fmaf(d[k][a], d[k][a], r2[k]);
            }
            in[k] = q0 + k * G < total && r2[k] < smax2;
            long idx;
            if constexpr (CLAMP) {
                idx = 0;
                const long stride[3] = {1, vol.nx, vol.nxy};
#pragma unroll
                for (int a = 0; a < DIM; ++a) idx += (long)min(max(fr.anc[a] + j[a], 0), vol.n[a] - 1) * stride[a];
            } else if constexpr (LAYOUT != kGlobalPlain) {
                int rel = __mul24(j[1], vol.nx) + j[0];
                if constexpr (DIM == 3) rel += __mul24(j[2], vol.nxy);
                idx = fr.base + rel;
            } else {
                long rel = (long)j[1] * vol.nx + j[0];
                if constexpr (DIM == 3) rel += (long)j[2] * vol.nxy;
                idx = fr.base + rel;
            }
            I[k] = in[k] ? vol.load1(idx) : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (!in[k]) continue;
            const float r = __builtin_amdgcn_sqrtf(r2[k]);
            const float inv_r = r > 0.0f ? __builtin_amdgcn_rcpf(r) : 0.0f;
            const float d1 = r - fr.ain, d2 = r - fr.R;
            const bool r1 = d1 >= -fr.hd && d1 < fr.hd;   // inner ramp
            const bool ro = d2 >= -fr.hD && d2 < fr.hD;   // outer ramp
            const float sin_ = __builtin_amdgcn_fmed3f(d1 * fr.is, -1.0f, 1.0f);
            const float sout = __builtin_amdgcn_fmed3f(fmaf(-d2, fr.os, 0.5f), 0.0f, 1.0f);
            const float S = fminf(sin_, sout);
            const float cC = r1 ? fr.is : (ro ? -fr.os : 0.0f);
            const float cR = r1 ? -fr.rho_is : -cC;
            acc[0] = fmaf(S, I[k], acc[0]);
            acc[1] = fmaf(cR, I[k], acc[1]);
            const float g = cC * I[k] * inv_r;   // dS/dr I / r; u = d / r
#pragma unroll
            for (int a = 0; a < DIM; ++a) acc[2 + a] = fmaf(-g, d[k][a] * inv_h[a], acc[2 + a]);
        }
    }
}

// ---------------------------------------------------------------------------------------------
// LDS tile of the sample ball
// ---------------------------------------------------------------------------------------------

// A box of the smoothed volume held in LDS by one whole-wave group: voxels lo[a] .. lo[a] + n[a] - 1
// per axis, x fastest (n[2] = 1 in 2D). An iteration whose samples, trilinear corners included,
// all fall inside the box reads its corners from LDS; the box is staged again only when the ball
// leaves it. It is staged with a margin, so a contour that moves and grows slowly keeps its box
// for many iterations, and its corners stop costing scattered global loads.
struct Tile {
    int lo[3], n[3];
    bool valid;
};

constexpr int kTileMargin = 2;  // voxels added on each side of the ball's range, when they fit

// Voxel range lo .. hi per axis that the corners of an iteration's samples can touch (the ball of
// radius s_max around the centre, with the same rounding margin as the interior test).
template <int DIM>
__device__ __forceinline__ void ball_range(const Frame<DIM> &fr, const float inv_h[3], int lo[3], int hi[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = hi[a] = 0;
        if (a < DIM) {
            const float e = fmaf(fr.smax * inv_h[a], 1.0001f, 1e-3f);
            lo[a] = fr.anc[a] + (int)floorf(fr.off[a] - e);
            hi[a] = fr.anc[a] + (int)floorf(fr.off[a] + e) + 1;
        }
    }
}

// New box for the range lo .. hi (inside the volume): the largest margin of kTileMargin .. 0
// voxels per side whose box holds at most `cap` voxels, clamped to the volume. False if even the
// bare range does not fit.
template <int DIM>
__device__ __forceinline__ bool choose_tile(const int lo[3], const int hi[3], const int nvol[3], int cap, Tile &t) {
    for (int m = kTileMargin; m >= 0; --m) {
        int n[3] = {1, 1, 1};
        int size = 1;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            n[a] = min(hi[a] - lo[a] + 1 + 2 * m, nvol[a]);
            size *= n[a];
        }
        if (size <= cap) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                t.n[a] = n[a];
                t.lo[a] = a < DIM ? min(max(lo[a] - m, 0), nvol[a] - n[a]) : 0;
            }
            t.valid = true;
            return true;
        }
    }
    t.valid = false;
    return false;
}

// All G lanes copy the box from the plain FP32 volume into LDS, 8 loads in flight per lane. The
// caller synchronises the group before the box is read.
template <int G>
__device__ __forceinline__ void stage_tile(float *tile, const float *J, int nx, int nxy, const Tile &t, int gl) {
    const int n0 = t.n[0], n1 = t.n[1];
    const int total = n0 * n1 * t.n[2];
    const float *src = J + ((long)t.lo[2] * nxy + (long)t.lo[1] * nx + t.lo[0]);
    // element e = gl + k G of the box -> (x, y, z), advanced by G without a division
    int x = gl % n0, y = (gl / n0) % n1, z = gl / (n0 * n1);
    const int sx = G % n0, sy = G / n0;
    constexpr int B = 8;
    for (int e0 = gl; e0 < total; e0 += B * G) {
        float v[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            v[k] = e0 + k * G < total ? src[(long)z * nxy + y * nx + x] : 0.0f;
            x += sx;
            if (x >= n0) {
                x -= n0;
                y += 1;
            }
            y += sy;
            while (y >= n1) {
                y -= n1;
                z += 1;
            }
        }
#pragma unroll
        for (int k = 0; k < B; ++k)
            if (e0 + k * G < total) tile[e0 + k * G] = v[k];
    }
}

// ---------------------------------------------------------------------------------------------
// Per-contour iteration loop
// ---------------------------------------------------------------------------------------------

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

// A value identical in every lane of a whole-wave group, moved to a scalar register (frees vector
// registers; sub-wave groups keep per-lane values).
template <int G>
__device__ __forceinline__ float uni(float v) {
    if constexpr (G >= 64) return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
    else return v;
}
template <int G>
__device__ __forceinline__ int uni(int v) {
    if constexpr (G >= 64) return __builtin_amdgcn_readfirstlane(v);
    else return v;
}

// Run up to n_iter iterations of the group's contour (slot == nullptr: no contour), stopping early at
// iteration `target` or when it leaves SNK_ACTIVE. All lanes of the workgroup call this; the loop
// and its barriers are workgroup-uniform.
// STAGE (whole-wave groups): iterations whose ball fits a box of tile_cap voxels read their corners
// from an LDS box at lds_tile, the others from the volume in LAYOUT.
// Soft repulsion of one contour (kappa > 0): the snapshot of every contour and this contour's
// neighbour list (cnt indices, ascending).
struct Repel {
    const float4 *snap = nullptr;
    const int *nb = nullptr;
    int cnt = 0;
    float kappa = 0.0f;
};

template <int DIM, int G, int U, bool TRACE, int LAYOUT, bool EXACT = false, bool STAGE = false, bool GRADI = false>
__device__ void run_group(const JobParams &p, DevContour *slot, int n_iter, int target, float *trace_row,
                          float *lds_draws, float *lds_red, unsigned long long *counter, float *lds_tile = nullptr,
                          int tile_cap = 0, const Repel rp = Repel{}) {
    static_assert(!STAGE || (G >= 64 && !EXACT), "LDS boxes are staged by whole-wave Monte-Carlo groups");
    constexpr int NR = 2 + DIM;
    constexpr int WAVES = Grp<G>::WAVES;
    constexpr float RHO = DIM == 3 ? 0.79370052598409973738f : 0.70710678118654752440f;
    constexpr float BALL = DIM == 3 ? 4.18879020478639098462f : 3.14159265358979323846f;
    const int t = threadIdx.x;
    const int gl = G < 64 ? (t & (G - 1)) : t;
    const int lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform (scalar branches)

    DevContour s{};
    s.status = SNK_OUT;
    if (slot) {
        if constexpr (G >= 64) s = uniform_copy(slot);
        else s = *slot;
    }
    const int n0 = s.iters;
    const int budget = ((s.status & 0x0f) == SNK_ACTIVE && slot) ? min(n_iter, target - n0) : 0;
    const int MH = p.M / 2;
    const int P = MH * p.L;
    const Draws dr(lds_draws, G, MH);
    const uint32_t id = s.id;
    const Vol<DIM, LAYOUT> vol(p.g);
    const float inv_h[3] = {p.g.inv_h[0], p.g.inv_h[1], p.g.inv_h[2]};
    const float hh[3] = {p.g.h[0], p.g.h[1], p.g.h[2]};

    if (!EXACT && budget > 0) draws_phase1<DIM, G>(dr, 0, (uint32_t)(n0 + 1), id, p, gl);
    __syncthreads();
    if (!EXACT && budget > 0) draws_phase2<DIM, G>(dr, 0, p, gl);
    __syncthreads();

    // lane's first pair-point and its step
    const int L = p.L;
    const float invL = 1.0f / (float)L;
    const int l0 = gl % L, m0 = gl / L;
    const int dl = G % L, dm = G / L;
    // every lane's passes hold only valid pair-points at one radial index (lane_sums FULL; in 2D:
    // the second copy of the sums loop costs the 3D instances registers they do not have)
    const bool full = DIM == 2 && dl == 0 && P % (G * U) == 0;

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
    int cull_next = p.cull_first;  // this launch's next culling pass point (-1: none)
    Tile tile;
    tile.valid = false;

    for (int it = 0;; ++it) {
        const bool active = it < budget && (status & 0x0f) == SNK_ACTIVE;
        bool any;
        if constexpr (G <= 64) any = __builtin_amdgcn_ballot_w64(active) != 0;
        else any = active;  // identical in every wave of the workgroup
        if (!any) break;
        float acc[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = 0.0f;
        Frame<DIM> fr;
        bool interior = true;
        if (active) {
            const int blk = it / dr.K, sl = it - blk * dr.K;
            if (!EXACT && sl == 0)
                draws_phase1<DIM, G>(dr, (blk + 1) & 1, (uint32_t)(n0 + 1 + (blk + 1) * dr.K), id, p, gl);
            if (!EXACT && sl == 1) draws_phase2<DIM, G>(dr, (blk + 1) & 1, p, gl);

            fr.smax = uni<G>(R + 0.5f * p.dR);
            fr.ain = uni<G>(RHO * R);
            fr.R = R;
            fr.hd = 0.5f * RHO * p.dR;
            fr.hD = 0.5f * p.dR;
            fr.is = p.in_slope;
            fr.os = p.out_slope;
            fr.rho_is = RHO * p.in_slope;
            long base = 0;
            const long stride[3] = {1, vol.nx, vol.nxy};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                fr.anc[a] = anc[a];
                fr.off[a] = off[a];
            }
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                base += (long)anc[a] * stride[a];
                // clamping can be skipped when the whole sample ball (with a rounding margin) is
                // interior
                const float ext = fmaf(fr.smax * inv_h[a], 1.0001f, 1e-3f);
                interior = interior && (off[a] - ext > (float)(-anc[a])) &&
                           (off[a] + ext < (float)(vol.n[a] - 1 - anc[a]));
            }
            fr.base = base;
            if constexpr (EXACT) {
                if (interior)
                    lattice_sums<DIM, G, false, LAYOUT>(vol, fr, hh, inv_h, gl, acc);
                else
                    lattice_sums<DIM, G, true, LAYOUT>(vol, fr, hh, inv_h, gl, acc);
            } else {
                const float4 *pu = dr.pu + dr.slot(blk & 1, sl) * MH;
                bool staged = false;
                if constexpr (STAGE) {
                    if (interior && tile_cap > 0) {
                        int lo[3], hi[3];
                        ball_range<DIM>(fr, inv_h, lo, hi);
                        bool covered = tile.valid;
#pragma unroll
                        for (int a = 0; a < DIM; ++a)
                            covered = covered && lo[a] >= tile.lo[a] && hi[a] < tile.lo[a] + tile.n[a];
                        if (!covered && choose_tile<DIM>(lo, hi, vol.n, tile_cap, tile)) {
                            // the previous iteration's reads of the box ended at its reduction barrier
                            stage_tile<G>(lds_tile, p.g.J, vol.nx, vol.nxy, tile, gl);
                            __syncthreads();
                        }
                        staged = tile.valid;
                    }
                }
                if (staged) {
                    TileVol<DIM> tv;
                    tv.t = lds_tile;
                    tv.n[0] = tile.n[0];
                    tv.n[1] = tile.n[1];
                    tv.n[2] = tile.n[2];
                    tv.nx = tile.n[0];
                    tv.nxy = tile.n[0] * tile.n[1];
                    Frame<DIM> ft = fr;
                    ft.base = (anc[0] - tile.lo[0]) + (anc[1] - tile.lo[1]) * tv.nx;
                    if constexpr (DIM == 3) ft.base += (anc[2] - tile.lo[2]) * tv.nxy;
                    if (full)
                        lane_sums<DIM, G, U, false, GRADI, true>(tv, ft, pu, P, L, invL, gl, l0, m0, dl, dm, acc);
                    else
                        lane_sums<DIM, G, U, false, GRADI>(tv, ft, pu, P, L, invL, gl, l0, m0, dl, dm, acc);
                } else if (interior) {
                    if (full)
                        lane_sums<DIM, G, U, false, GRADI, true>(vol, fr, pu, P, L, invL, gl, l0, m0, dl, dm, acc);
                    else
                        lane_sums<DIM, G, U, false, GRADI>(vol, fr, pu, P, L, invL, gl, l0, m0, dl, dm, acc);
                } else {
                    lane_sums<DIM, G, U, true, GRADI>(vol, fr, pu, P, L, invL, gl, l0, m0, dl, dm, acc);
                }
            }
        }

        // group totals
        float tot[NR];
        if constexpr (G < 64) {
#pragma unroll
            for (int k = 0; k < NR; ++k) tot[k] = group_sum_wave<G>(acc[k]);
        } else if constexpr (G == 64) {
            wave_sums<NR>(acc, tot);
        } else {
            float *red = lds_red + (it & 1) * NR * WAVES;
            float wt[NR];
            wave_sums<NR>(acc, wt);
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < NR; ++k) red[k * WAVES + wave] = wt[k];
            }
            __syncthreads();
            // every wave adds the partials in wave order, so all of them hold the same totals and
            // take the same step below (no second barrier to hand wave 0's result to the others)
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                float v = red[k * WAVES];
#pragma unroll
                for (int w = 1; w < WAVES; ++w) v += red[k * WAVES + w];
                tot[k] = v;
            }
        }
        // gradient form: sum S dI/dv_a (voxel coordinates) -> the units of the weight form's
        // sum -dS/dr I u_a / h_a, i.e. the physical force divided by h_a
        if constexpr (GRADI) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) tot[2 + a] *= inv_h[a] * inv_h[a];
        }

        // descent step, identical in every lane of the group (multi-wave groups: every wave, from the
        // same totals)
        if (active) {
            // no multiply-add contraction in the step: every instance (with or without the optional
            // terms below) rounds it operation by operation, so their results agree bit for bit
#pragma clang fp contract(off)
            n += 1;
            const float smax = fr.smax;
            float smax_d = smax;
#pragma unroll
            for (int i = 1; i < DIM; ++i) smax_d *= smax;
            // Monte-Carlo: V/N; exact: the voxel measure
            const float scale = EXACT ? hh[0] * hh[1] * (DIM == 3 ? hh[2] : 1.0f) : BALL * smax_d * inv_npts;
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
            float dRs = -half_eps * gR;
            const float kc = -half_eps * scale * inv_norm;
            float doff[3] = {0.0f, 0.0f, 0.0f}, dc[3] = {0.0f, 0.0f, 0.0f};
            float dc2 = 0.0f;
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                doff[i] = kc * tot[2 + i];   // voxel units (B_c was accumulated against u / h)
                dc[i] = doff[i] * hh[i];
            }
            if constexpr (G >= 64) {
                if (rp.kappa > 0.0f) {
                    // repulsion of the neighbours' snapshot: lane k takes neighbour k; with t = |c - c_j| /
                    // (rho (R + R_j)) < 1 the penalty (1 - t)^2 has dP/dc = -2 (1 - t) (c - c_j) /
                    // (|c - c_j| rho (R + R_j)) and dP/dR = 2 (1 - t) t / (R + R_j)
                    float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                    if (lane < rp.cnt) {
                        const int j = rp.nb[lane];
                        const float4 s0 = rp.snap[2 * j], s1 = rp.snap[2 * j + 1];
                        const int aj[3] = {__float_as_int(s0.x), __float_as_int(s0.y), __float_as_int(s0.z)};
                        const float oj[3] = {s1.x, s1.y, s1.z};
                        float dv[3] = {0.0f, 0.0f, 0.0f}, d2 = 0.0f;
#pragma unroll
                        for (int a = 0; a < DIM; ++a) {
                            dv[a] = ((float)(anc[a] - aj[a]) + (off[a] - oj[a])) * hh[a];
                            d2 = fmaf(dv[a], dv[a], d2);
                        }
                        const float d = __builtin_amdgcn_sqrtf(d2);
                        const float span = RHO * (R + s0.w);
                        const float t = d / span;
                        if (t < 1.0f) {
                            const float om = 1.0f - t;
                            v[3] = 2.0f * om * t / (R + s0.w);
                            if (d > 0.0f) {
                                const float f = -2.0f * om / (d * span);
#pragma unroll
                                for (int a = 0; a < DIM; ++a) v[a] = f * dv[a];
                            }
                        }
                    }
                    float rt[4];
                    wave_sums<4>(v, rt);
                    const float kr = -half_eps * rp.kappa;
                    dRs = dRs + kr * rt[3];
#pragma unroll
                    for (int i = 0; i < DIM; ++i) {
                        const float dcr = kr * rt[i];
                        dc[i] = dc[i] + dcr;
                        doff[i] = doff[i] + dcr * inv_h[i];
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < DIM; ++i) dc2 = fmaf(dc[i], dc[i], dc2);
            if (TRACE && gl == 0) {
                float *row = trace_row;
                row[0] = A;
                row[1] = BR;
                for (int i = 0; i < 3; ++i) row[2 + i] = i < DIM ? scale * tot[2 + i] * hh[i] : 0.0f;
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
            if (Rn < p.r_lo) {
                Rn = p.r_lo;
                flag = SNK_CLAMPED;
            }
            if (Rn > p.r_hi) {
                Rn = p.r_hi;
                flag = SNK_CLAMPED;
            }
            const float dRe = Rn - R;
            const bool small = dRe * dRe < tol2 && dc2 < tol2;
            R = Rn;
            e_mc = E;
            bool finite = isfinite(Rn) && isfinite(E);
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                off[i] += doff[i];
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
                    if (off[i] < (float)(-anc[i]) || off[i] > (float)(vol.n[i] - 1 - anc[i])) st = SNK_OUT;
                }
            }
            if (st == SNK_ACTIVE) {
                streak = small ? min(streak + 1, 255) : 0;
                if (p.conv_window > 0 && streak >= p.conv_window) st = SNK_CONVERGED;
            }
            // a culling pass without competition judges each contour alone: at the run's pass
            // points an active contour above the threshold retires here and frees its slot at once
            // (the pass after the evolution treats the others as the passes between chunks would)
            if (it == cull_next) {
                // kept a branch (an empty volatile statement cannot be executed speculatively):
                // selects in its place would cost every iteration of every run
                __asm__ volatile("");
                if (st == SNK_ACTIVE && !(E <= p.cull_thr)) st = SNK_CULLED;
                cull_next = cull_next + p.cull_every <= p.cull_last ? cull_next + p.cull_every : -1;
            }
            status = (uint8_t)uni<G>((int)(st | flag));
            streak = uni<G>(streak);
            R = uni<G>(R);
            e_mc = uni<G>(e_mc);
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                off[i] = uni<G>(off[i]);
                anc[i] = uni<G>(anc[i]);
            }
            ++ran;
        }
        if constexpr (G <= 64) __syncthreads();  // orders this iteration's LDS draws before later reads
    }

    if (slot && gl == 0 && budget > 0) {
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

// LDS of one workgroup: draws of each contour it holds, then (multi-wave groups) the reduction
// slots.
template <int DIM, int G>
__host__ __device__ __forceinline__ int lds_floats(int MH) {
    const int per = (draw_floats(G, MH) + 3) & ~3;
    return Grp<G>::CPB * per + (G > 64 ? 2 * (2 + DIM) * Grp<G>::WAVES : 0);
}

// Whole-wave groups with one pair-point in flight fit 64 vector registers: ask for 8 waves per SIMD
// (a full CU of 4-wave groups holds 8 contours). Two-wave groups with four pair-points in flight
// ask for 4 waves per SIMD (128 registers), so 8 contours per CU stay resident.
// STAGE: the workgroup's LDS ends with a box of a.tile_cap voxels. GRADI: centre force in its
// image-gradient form.
template <int DIM, int G, int U, bool TRACE, int LAYOUT, bool EXACT, bool STAGE, bool GRADI>
__global__ __launch_bounds__(Grp<G>::NT, (U == 1 && G >= 64) ? 8 : ((U == 4 && G == 128) ? 4 : 1))
void evolve_kernel(EvolveArgs a) {
    extern __shared__ float lds[];
    const int MH = a.p.M / 2;
    const int per = (draw_floats(G, MH) + 3) & ~3;
    const int sub = G < 64 ? (int)threadIdx.x / G : 0;
    const int k = blockIdx.x * Grp<G>::CPB + sub;
    const int cid = k < a.n ? (a.idx ? a.idx[k] : k) : k;
    DevContour *slot = k < a.n ? a.st + cid : nullptr;
    Repel rp;
    if (G >= 64 && a.kappa > 0.0f && slot) {
        rp.snap = a.snap;
        rp.nb = a.nb + (long)cid * a.nb_cap;
        rp.cnt = __builtin_amdgcn_readfirstlane(a.nbn[cid]);
        rp.kappa = a.kappa;
    }
    run_group<DIM, G, U, TRACE, LAYOUT, EXACT, STAGE, GRADI>(a.p, slot, a.n_iter, 0x7fffffff,
                                                      TRACE && slot ? a.trace + (long)cid * SNK_TRACE_W : nullptr,
                                                      lds + sub * per, lds + Grp<G>::CPB * per, a.counter,
                                                      lds + lds_floats<DIM, G>(MH), STAGE ? a.tile_cap : 0, rp);
}

// Batched launch over (job, contour) items, one workgroup (G >= 64 lanes) per item. PERSISTENT: a
// fixed grid pops items from a device work queue until it is exhausted (every workgroup reaches
// the exit); otherwise one workgroup per item. STAGE: the workgroup's LDS ends with a box of
// a.tile_cap voxels for the contour it is running (restaged for each item).
template <int DIM, int G, int U, int LAYOUT, bool PERSISTENT, bool STAGE>
__global__ __launch_bounds__(G, U == 1 ? 8 : 1) void evolve_batch_kernel(BatchArgs a) {
    static_assert(G >= 64, "batched groups span whole waves");
    extern __shared__ float lds[];
    __shared__ int item_sh;
    const int per = (draw_floats(G, a.max_M / 2) + 3) & ~3;
    for (int round = 0;; ++round) {
        int item;
        if constexpr (PERSISTENT) {
            if (threadIdx.x == 0) item_sh = atomicAdd(a.queue, 1);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(item_sh);
            __syncthreads();
        } else {
            item = round == 0 ? (int)blockIdx.x : a.n_items;
        }
        if (item >= a.n_items) break;
        const int job = __builtin_amdgcn_readfirstlane(a.items[item].x);
        const int cid = __builtin_amdgcn_readfirstlane(a.items[item].y);
        const JobParams p = uniform_copy(&a.jobs[job].p);
        DevContour *st = uniform_copy(&a.jobs[job].st);
        const int target = __builtin_amdgcn_readfirstlane(a.jobs[job].target);
        run_group<DIM, G, U, false, LAYOUT, false, STAGE>(p, st + cid, a.chunk, target, nullptr, lds, lds + per,
                                                         a.counter, lds + lds_floats<DIM, G>(a.max_M / 2),
                                                         STAGE ? a.tile_cap : 0);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------------------------

template <int DIM, int G, int U, bool TRACE, int LAYOUT, bool EXACT = false, bool STAGE = false, bool GRADI = false>
hipError_t launch_t(const EvolveArgs &a, hipStream_t s) {
    const size_t lds = sizeof(float) * ((size_t)lds_floats<DIM, G>(a.p.M / 2) + (STAGE ? (size_t)a.tile_cap : 0));
    const int blocks = (a.n + Grp<G>::CPB - 1) / Grp<G>::CPB;
    hipLaunchKernelGGL((evolve_kernel<DIM, G, U, TRACE, LAYOUT, EXACT, STAGE, GRADI>), dim3(blocks),
                       dim3(Grp<G>::NT), lds, s, a);
    return hipGetLastError();
}

// Gradient-form centre force: whole-wave groups, two pair-points in flight, buffer layouts, with or
// without LDS boxes.
template <int DIM, int G, bool TRACE>
hipError_t launch_gradi_l(const EvolveArgs &a, int layout, hipStream_t s) {
    const bool stage = a.tile_cap > 0;
    if (layout == kBufferQuad)
        return stage ? launch_t<DIM, G, 2, TRACE, kBufferQuad, false, true, true>(a, s)
                     : launch_t<DIM, G, 2, TRACE, kBufferQuad, false, false, true>(a, s);
    if (layout == kBufferPlain)
        return stage ? launch_t<DIM, G, 2, TRACE, kBufferPlain, false, true, true>(a, s)
                     : launch_t<DIM, G, 2, TRACE, kBufferPlain, false, false, true>(a, s);
    if constexpr (DIM == 3)
        if (layout == kBufferPair)
            return stage ? launch_t<DIM, G, 2, TRACE, kBufferPair, false, true, true>(a, s)
                         : launch_t<DIM, G, 2, TRACE, kBufferPair, false, false, true>(a, s);
    return hipErrorInvalidValue;
}

template <int DIM, bool TRACE>
hipError_t launch_gradi_g(const EvolveArgs &a, int lanes, int layout, hipStream_t s) {
    switch (lanes) {
        case 64: return launch_gradi_l<DIM, 64, TRACE>(a, layout, s);
        case 128: return launch_gradi_l<DIM, 128, TRACE>(a, layout, s);
        case 256: return launch_gradi_l<DIM, 256, TRACE>(a, layout, s);
        default: return hipErrorInvalidValue;
    }
}

// Exact lattice sums read single voxels: plain layouts only.
template <int DIM, int G, bool TRACE>
hipError_t launch_exact_l(const EvolveArgs &a, int layout, hipStream_t s) {
    return layout == kGlobalPlain ? launch_t<DIM, G, 1, TRACE, kGlobalPlain, true>(a, s)
                                  : launch_t<DIM, G, 1, TRACE, kBufferPlain, true>(a, s);
}

template <int DIM, bool TRACE>
hipError_t launch_exact_g(const EvolveArgs &a, int lanes, int layout, hipStream_t s) {
    switch (lanes) {
        case 16: return launch_exact_l<DIM, 16, TRACE>(a, layout, s);
        case 32: return launch_exact_l<DIM, 32, TRACE>(a, layout, s);
        case 64: return launch_exact_l<DIM, 64, TRACE>(a, layout, s);
        case 128: return launch_exact_l<DIM, 128, TRACE>(a, layout, s);
        default: return launch_exact_l<DIM, 256, TRACE>(a, layout, s);
    }
}

template <int DIM, int G, int U, bool TRACE>
hipError_t launch_l(const EvolveArgs &a, int layout, hipStream_t s) {
    if constexpr (G >= 64) {
        // LDS boxes, with a buffer layout for the iterations whose ball does not fit
        if (a.tile_cap > 0) {
            if (layout == kBufferQuad) return launch_t<DIM, G, U, TRACE, kBufferQuad, false, true>(a, s);
            if (layout == kBufferPlain) return launch_t<DIM, G, U, TRACE, kBufferPlain, false, true>(a, s);
            if constexpr (DIM == 3)
                if (layout == kBufferPair) return launch_t<DIM, G, U, TRACE, kBufferPair, false, true>(a, s);
            return hipErrorInvalidValue;
        }
    } else {
        if (a.tile_cap > 0) return hipErrorInvalidValue;
    }
    switch (layout) {
        case kBufferPair: return launch_t<DIM, G, U, TRACE, kBufferPair>(a, s);
        case kBufferQuad: return launch_t<DIM, G, U, TRACE, kBufferQuad>(a, s);
        case kBufferPlain: return launch_t<DIM, G, U, TRACE, kBufferPlain>(a, s);
        case kGlobalPlain: return launch_t<DIM, G, U, TRACE, kGlobalPlain>(a, s);
        default: return hipErrorInvalidValue;
    }
}

// Four pair-points in flight: half-wave, one- and two-wave groups, outside the per-iteration trace (there the
// order of a lane's sums is the same as with two, so the trace runs the two-pair-point instance).
template <int DIM, int G, bool TRACE>
hipError_t launch_u(const EvolveArgs &a, int unroll, int layout, hipStream_t s) {
    if constexpr (!TRACE && (G == 32 || G == 64 || G == 128))
        if (unroll >= 4) return launch_l<DIM, G, 4, TRACE>(a, layout, s);
    return unroll >= 2 ? launch_l<DIM, G, 2, TRACE>(a, layout, s) : launch_l<DIM, G, 1, TRACE>(a, layout, s);
}

template <int DIM, bool TRACE>
hipError_t launch_g(const EvolveArgs &a, int lanes, int unroll, int layout, hipStream_t s) {
    switch (lanes) {
        case 16: return launch_u<DIM, 16, TRACE>(a, unroll, layout, s);
        case 32: return launch_u<DIM, 32, TRACE>(a, unroll, layout, s);
        case 64: return launch_u<DIM, 64, TRACE>(a, unroll, layout, s);
        case 128: return launch_u<DIM, 128, TRACE>(a, unroll, layout, s);
        default: return launch_u<DIM, 256, TRACE>(a, unroll, layout, s);
    }
}

template <int DIM, int G, int U, int LAYOUT, bool PERSISTENT, bool STAGE>
hipError_t batch_t(const BatchArgs &a, int grid, hipStream_t s) {
    const size_t lds = sizeof(float) * ((size_t)lds_floats<DIM, G>(a.max_M / 2) + (STAGE ? (size_t)a.tile_cap : 0));
    const int g = PERSISTENT ? grid : a.n_items;
    if (g <= 0) return hipSuccess;
    hipLaunchKernelGGL((evolve_batch_kernel<DIM, G, U, LAYOUT, PERSISTENT, STAGE>), dim3(g), dim3(G), lds, s, a);
    return hipGetLastError();
}

template <int DIM, int G, int U, int LAYOUT, bool PERSISTENT>
hipError_t batch_s(const BatchArgs &a, int grid, hipStream_t s) {
    return a.tile_cap > 0 ? batch_t<DIM, G, U, LAYOUT, PERSISTENT, true>(a, grid, s)
                          : batch_t<DIM, G, U, LAYOUT, PERSISTENT, false>(a, grid, s);
}

template <int DIM, int G, int U, int LAYOUT>
hipError_t batch_p(const BatchArgs &a, bool persistent, int grid, hipStream_t s) {
    return persistent ? batch_s<DIM, G, U, LAYOUT, true>(a, grid, s) : batch_s<DIM, G, U, LAYOUT, false>(a, grid, s);
}

template <int DIM, int G, int U>
hipError_t batch_l(const BatchArgs &a, int layout, bool persistent, int grid, hipStream_t s) {
    if (layout == kBufferPair) return batch_p<DIM, G, U, kBufferPair>(a, persistent, grid, s);
    return layout == kBufferQuad ? batch_p<DIM, G, U, kBufferQuad>(a, persistent, grid, s)
                                 : batch_p<DIM, G, U, kBufferPlain>(a, persistent, grid, s);
}

template <int DIM, int G>
hipError_t batch_u(const BatchArgs &a, int unroll, int layout, bool persistent, int grid, hipStream_t s) {
    return unroll >= 2 ? batch_l<DIM, G, 2>(a, layout, persistent, grid, s)
                       : batch_l<DIM, G, 1>(a, layout, persistent, grid, s);
}

template <int DIM>
hipError_t batch_g(const BatchArgs &a, int lanes, int unroll, int layout, bool persistent, int grid,
                   hipStream_t s) {
    switch (lanes) {
        case 64: return batch_u<DIM, 64>(a, unroll, layout, persistent, grid, s);
        case 128: return batch_u<DIM, 128>(a, unroll, layout, persistent, grid, s);
        default: return batch_u<DIM, 256>(a, unroll, layout, persistent, grid, s);
    }
}

template <int DIM, int G, int U, int LAYOUT, bool STAGE>
int max_blocks_t(int max_M, int tile_cap) {
    int blocks = 0;
    const size_t lds = sizeof(float) * ((size_t)lds_floats<DIM, G>(max_M / 2) + (STAGE ? (size_t)tile_cap : 0));
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, evolve_batch_kernel<DIM, G, U, LAYOUT, true, STAGE>, G,
                                                     lds) != hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

template <int DIM, int G, int U, int LAYOUT>
int max_blocks_s(int max_M, int tile_cap) {
    return tile_cap > 0 ? max_blocks_t<DIM, G, U, LAYOUT, true>(max_M, tile_cap)
                        : max_blocks_t<DIM, G, U, LAYOUT, false>(max_M, 0);
}

template <int DIM, int G>
int max_blocks_u(int unroll, int layout, int max_M, int tile_cap) {
    if (unroll >= 2) {
        if (layout == kBufferPair) return max_blocks_s<DIM, G, 2, kBufferPair>(max_M, tile_cap);
        return layout == kBufferQuad ? max_blocks_s<DIM, G, 2, kBufferQuad>(max_M, tile_cap)
                                     : max_blocks_s<DIM, G, 2, kBufferPlain>(max_M, tile_cap);
    }
    if (layout == kBufferPair) return max_blocks_s<DIM, G, 1, kBufferPair>(max_M, tile_cap);
    return layout == kBufferQuad ? max_blocks_s<DIM, G, 1, kBufferQuad>(max_M, tile_cap)
                                 : max_blocks_s<DIM, G, 1, kBufferPlain>(max_M, tile_cap);
}

template <int DIM>
int max_blocks_g(int lanes, int unroll, int layout, int max_M, int tile_cap) {
    switch (lanes) {
        case 64: return max_blocks_u<DIM, 64>(unroll, layout, max_M, tile_cap);
        case 128: return max_blocks_u<DIM, 128>(unroll, layout, max_M, tile_cap);
        default: return max_blocks_u<DIM, 256>(unroll, layout, max_M, tile_cap);
    }
}

// ---------------------------------------------------------------------------------------------
// Star-shaped contours (builder-defined extension: one radius per table direction)
// ---------------------------------------------------------------------------------------------
//
// One wave per contour. The table directions stay fixed in space (no rotation). Per iteration the
// Philox pair draws pick directions k; each pair's rays run along +T_k with radius R_k and along
// -T_k with the radius of the antipodal direction, with the sphere's radial points
// s = (R + dR/2) ((l + xi)/L)^(1/d) (L = 16: one DPP row of lanes per ray pair). With the per-point
// weight q(R) = (2R)^-d omega_d (R + dR/2)^d / (M L): E = sum q S I, g_c = sum q (-dS/dr I u), and
// every sampled direction k collects g_k = sum over its rays of q (B_R,ray - (d/R_k) A_ray)
// (rays that drew the same direction are summed in ray order by the first of them, so the result
// does not depend on timing). Step: c -= (eps/2) g_c; R_k -= (eps/2) D g_k + min(1, eps lambda / 2)
// (R_k - mean of its graph neighbours), from the old radii (double-buffered in LDS).

template <int DIM>
__host__ __device__ __forceinline__ int star_lds_floats(int D, int M, int NT) {
    const int per = (draw_floats(NT, M / 2) + 3) & ~3;
    return per + 4 * D + 2 + 2 * M + (M / 2) * (2 + DIM) + 8 * (NT / 64);
}

// NT threads per contour (64: one wave; 128: two waves, whose partial sums meet in LDS in wave
// order).
template <int DIM, int LAYOUT, int NT>
__global__ __launch_bounds__(NT, NT == 128 ? 4 : 1) void star_kernel(EvolveArgs a, StarArgs sa) {
    extern __shared__ float lds[];
    constexpr float RHO = DIM == 3 ? 0.79370052598409973738f : 0.70710678118654752440f;
    constexpr float BALL = DIM == 3 ? 4.18879020478639098462f : 3.14159265358979323846f;
    const JobParams &p = a.p;
    const int cid = blockIdx.x;
    if (cid >= a.n) return;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int NW = NT / 64;
    const int D = p.D, M = p.M, MH = M / 2, L = p.L;
    DevContour *slot = a.st + cid;
    DevContour s = uniform_copy(slot);
    const int n0 = s.iters;
    const int budget = (s.status & 0x0f) == SNK_ACTIVE ? a.n_iter : 0;
    const int per = (draw_floats(NT, MH) + 3) & ~3;
    const Draws dr(lds, NT, MH);
    // two radius buffers of D + 1 entries: entry D stays +0, so a neighbour row's padding (index D)
    // reads a zero
    float *Ra = lds + per;
    float *Rb = Ra + D + 1;
    float *gk = Rb + D + 1;
    int *ray_dir = reinterpret_cast<int *>(gk + D);
    float *ray_g = reinterpret_cast<float *>(ray_dir + M);
    // this iteration's ray pairs: direction, antipode, unit vector
    int *rk = reinterpret_cast<int *>(ray_g + M);
    int *rka = rk + MH;
    float *ru = reinterpret_cast<float *>(rka + MH);
    float *red = ru + MH * DIM;  // per-wave partials, 8 per wave
    // lowest ray of each direction this iteration (INT_MAX for none; reset by that ray after use)
    int *own = reinterpret_cast<int *>(red + 8 * NW);
    float *Rg = sa.Rk + (long)cid * D;
    for (int k = t; k < D; k += NT) {
        Ra[k] = Rg[k];
        gk[k] = 0.0f;
        own[k] = 0x7fffffff;
    }
    if (t == 0) {
        Ra[D] = 0.0f;
        Rb[D] = 0.0f;
    }
    const Vol<DIM, LAYOUT> vol(p.g);
    const float inv_h[3] = {p.g.inv_h[0], p.g.inv_h[1], p.g.inv_h[2]};
    const float hh[3] = {p.g.h[0], p.g.h[1], p.g.h[2]};
    const uint32_t id = s.id;
    if (budget > 0) draws_phase1<DIM, NT>(dr, 0, (uint32_t)(n0 + 1), id, p, t);
    __syncthreads();
    // largest radius (interior test) and the clamp flag of the radii
    float rmax = 0.0f;
    for (int k = t; k < D; k += NT) rmax = fmaxf(rmax, Ra[k]);
    rmax = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_max_to_63(rmax)), 63));
    if constexpr (NW > 1) {
        if (lane == 0) red[wave * 8] = rmax;
        __syncthreads();
        rmax = red[0];
        for (int w = 1; w < NW; ++w) rmax = fmaxf(rmax, red[w * 8]);
        __syncthreads();
    }

    int anc[3] = {s.anc[0], s.anc[1], s.anc[2]};
    float off[3] = {s.off[0], s.off[1], s.off[2]};
    float Rmean = s.R;
    int n = n0;
    uint8_t status = s.status;
    int streak = s.streak;
    float e_mc = s.e_mc;
    const float invL = 1.0f / (float)L;
    const float inv_ml = 1.0f / (float)(M * L);
    const float tol2 = p.conv_tol * p.conv_tol;
    const float hd = 0.5f * RHO * p.dR, hD = 0.5f * p.dR;
    int ran = 0;
    float *Rold = Ra, *Rnew = Rb;

    for (int it = 0; it < budget && (status & 0x0f) == SNK_ACTIVE; ++it) {
        const int blk = it / dr.K, sl = it - blk * dr.K;
        if (sl == 0) draws_phase1<DIM, NT>(dr, (blk + 1) & 1, (uint32_t)(n0 + 1 + (blk + 1) * dr.K), id, p, t);
        const float4 *pu = dr.pu + dr.slot(blk & 1, sl) * MH;
        Frame<DIM> fr;
        long base = 0;
        const long stride[3] = {1, vol.nx, vol.nxy};
        bool interior = true;
        const float ext_r = rmax + 0.5f * p.dR;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            fr.anc[ax] = anc[ax];
            fr.off[ax] = off[ax];
        }
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            base += (long)anc[ax] * stride[ax];
            const float ext = fmaf(ext_r * inv_h[ax], 1.0001f, 1e-3f);
            interior = interior && (off[ax] - ext > (float)(-anc[ax])) && (off[ax] + ext < (float)(vol.n[ax] - 1 - anc[ax]));
        }
        fr.base = base;
        // the ray pairs' tables entries, once per iteration (the pair-points below read them from LDS)
        for (int m = t; m < MH; m += NT) {
            const int k = __float_as_int(pu[m].x);
            rk[m] = k;
            rka[m] = sa.anti[k];
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) ru[m * DIM + ax] = p.dirs[k * DIM + ax];
        }
        __syncthreads();
        float accE = 0.0f, accc[3] = {0.0f, 0.0f, 0.0f};
        // pair-points q = t + NT j: pair m = q / 16, radial index l = q % 16 (one DPP row per pair);
        // two of them in flight, consumed in order
        const int PP = MH * L;
        for (int q0 = t; q0 - t < PP; q0 += 2 * NT) {
            Corners<DIM> cr[2][2];
            float fv[2][2][3], Rv[2][2], ev[2], uv[2][3];
            int mv2[2], lv[2], kv[2][2];
            bool on[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int q = q0 + NT * h;
                on[h] = q < PP;
                if (!on[h]) continue;
                const int m = q >> 4, l = q & 15;
                mv2[h] = m;
                lv[h] = l;
                const int k = rk[m], ka = rka[m];
                kv[h][0] = k;
                kv[h][1] = ka;
                float du[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) uv[h][ax] = 0.0f;
#pragma unroll
                for (int ax = 0; ax < DIM; ++ax) {
                    uv[h][ax] = ru[m * DIM + ax];
                    du[ax] = uv[h][ax] * inv_h[ax];
                }
                const float e = cube_or_square_root<DIM>(((float)l + pu[m].w) * invL);
                ev[h] = e;
#pragma unroll
                for (int sg = 0; sg < 2; ++sg) {
                    const float R = Rold[sg ? ka : k];
                    const float smax = R + 0.5f * p.dR;
                    const float rad = smax * e;
                    float w[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int ax = 0; ax < DIM; ++ax) w[ax] = fmaf(sg ? -rad : rad, du[ax], off[ax]);
                    Rv[h][sg] = R;
                    if (interior)
                        vol.load(locate<DIM, false, Vol<DIM, LAYOUT>::kSmall>(fr, vol.n, vol.nx, vol.nxy, w, fv[h][sg]),
                                 cr[h][sg]);
                    else
                        vol.load(locate<DIM, true, Vol<DIM, LAYOUT>::kSmall>(fr, vol.n, vol.nx, vol.nxy, w, fv[h][sg]),
                                 cr[h][sg]);
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (!on[h]) continue;
                const int m = mv2[h], l = lv[h];
                const float e = ev[h];
                float Ival[2], Sv[2], cCv[2], cRv[2], qv[2];
#pragma unroll
                for (int sg = 0; sg < 2; ++sg) {
                    const float R = Rv[h][sg];
                    const float smax = R + 0.5f * p.dR;
                    const float I = trilerp<DIM>(cr[h][sg], fv[h][sg]);
                    const float d1 = fmaf(smax, e, -RHO * R), d2 = fmaf(smax, e, -R);
                    const float is = p.in_slope, os = p.out_slope;
                    const bool r1 = d1 >= -hd && d1 < hd;
                    const bool r2 = d2 >= -hD && d2 < hD;
                    const float sin_ = __builtin_amdgcn_fmed3f(d1 * is, -1.0f, 1.0f);
                    const float sout = __builtin_amdgcn_fmed3f(fmaf(-d2, os, 0.5f), 0.0f, 1.0f);
                    const float inv2R = __builtin_amdgcn_rcpf(2.0f * R);
                    float nrm = inv2R, sm_d = smax;
#pragma unroll
                    for (int i = 1; i < DIM; ++i) {
                        nrm *= inv2R;
                        sm_d *= smax;
                    }
                    Ival[sg] = I;
                    Sv[sg] = fminf(sin_, sout);
                    cCv[sg] = r1 ? is : (r2 ? -os : 0.0f);
                    cRv[sg] = r1 ? -RHO * is : -cCv[sg];
                    qv[sg] = BALL * sm_d * nrm * inv_ml;
                }
#pragma unroll
                for (int sg = 0; sg < 2; ++sg) {
                    const float qI = qv[sg] * Ival[sg];
                    accE = fmaf(Sv[sg], qI, accE);
                    const float gcs = -cCv[sg] * qI * (sg ? -1.0f : 1.0f);
#pragma unroll
                    for (int ax = 0; ax < DIM; ++ax) accc[ax] = fmaf(gcs, uv[h][ax], accc[ax]);
                }
                // per-ray sums over the row's 16 radial points
                float Ap = row_sum16(Sv[0] * Ival[0]), Bp = row_sum16(cRv[0] * Ival[0]);
                float Am = row_sum16(Sv[1] * Ival[1]), Bm = row_sum16(cRv[1] * Ival[1]);
                if (l == 0) {
                    ray_dir[2 * m] = kv[h][0];
                    ray_g[2 * m] = qv[0] * (Bp - ((float)DIM / Rv[h][0]) * Ap);
                    ray_dir[2 * m + 1] = kv[h][1];
                    ray_g[2 * m + 1] = qv[1] * (Bm - ((float)DIM / Rv[h][1]) * Am);
                }
            }
        }
        float E = 0.0f, gc[3] = {0.0f, 0.0f, 0.0f};
        if constexpr (NW == 1) {
            E = group_sum_wave<64>(accE);
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) gc[ax] = group_sum_wave<64>(accc[ax]);
        } else {
            const float wE = wave_sum_to_63(accE);
            float wc[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) wc[ax] = wave_sum_to_63(accc[ax]);
            if (lane == 63) {
                red[wave * 8] = wE;
#pragma unroll
                for (int ax = 0; ax < DIM; ++ax) red[wave * 8 + 1 + ax] = wc[ax];
            }
            __syncthreads();
            E = red[0];
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) gc[ax] = red[1 + ax];
            for (int w = 1; w < NW; ++w) {
                E += red[w * 8];
#pragma unroll
                for (int ax = 0; ax < DIM; ++ax) gc[ax] += red[w * 8 + 1 + ax];
            }
        }
        __syncthreads();
        // sampled directions: the first ray of each direction sums its rays in order (the sum starts
        // at +0, so it is never -0 and adding +0 leaves it unchanged).
        if (M <= 64) {
            // all rays in wave 0: the lowest ray of each direction comes from an LDS minimum; the few
            // later rays of a direction are then added, lowest first, by that direction's first ray
            if (wave == 0) {
                const bool has = lane < M;
                const int dk = has ? ray_dir[lane] : 0;
                const float gr = has ? ray_g[lane] : 0.0f;
                if (has) atomicMin(&own[dk], lane);
                // one wave's LDS operations complete in order: every lane's minimum is in
                const bool first = has && own[dk] == lane;
                float g = 0.0f + gr;
                uint64_t later = __builtin_amdgcn_ballot_w64(has && !first);
                while (later) {
                    const int j = __builtin_amdgcn_readfirstlane(__builtin_ctzll(later));
                    later &= later - 1;
                    const int dj = __builtin_amdgcn_readlane(dk, j);
                    const float gj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(gr), j));
                    if (first && dk == dj) g += gj;
                }
                if (first) {
                    gk[dk] = g;
                    own[dk] = 0x7fffffff;
                }
            }
        } else {
            // Every lane walks all rays, eight at a time with their loads issued together and no branch
            // on the loaded values (a ray of another direction adds +0)
            for (int r = t; r < M; r += NT) {
                const int dk = ray_dir[r];
                bool first = true;
                float g = 0.0f;
                int r2 = 0;
                for (; r2 + 8 <= M; r2 += 8) {
                    int dd[8];
                    float gg[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        dd[u] = ray_dir[r2 + u];
                        gg[u] = ray_g[r2 + u];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const bool same = dd[u] == dk;
                        first = first && !(same && r2 + u < r);
                        g += same && r2 + u >= r ? gg[u] : 0.0f;
                    }
                }
                for (; r2 < M; ++r2) {
                    const bool same = ray_dir[r2] == dk;
                    first = first && !(same && r2 < r);
                    g += same && r2 >= r ? ray_g[r2] : 0.0f;
                }
                if (first) gk[dk] = g;
            }
        }
        __syncthreads();
        n += 1;
        const float eps = p.eps0 * __builtin_amdgcn_rsqf((float)n);
        const float half_eps = 0.5f * eps;
        const float relax = fminf(1.0f, half_eps * sa.lambda);
        float mv = 0.0f, sum = 0.0f, mx = 0.0f;
        int clamped = 0, finite_r = 1;
        // neighbour rows of four directions are loaded before any of them is used; every entry is
        // read without a branch (the padding index D reads +0, which leaves the sum unchanged), so
        // a row's LDS reads are all issued before the first is added
        // (a direction past D loads the last row, unused)
        const uint4 *nbrow = reinterpret_cast<const uint4 *>(sa.nb);
        for (int k0 = t; k0 < D; k0 += 4 * NT) {
            uint4 pre[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) pre[b] = nbrow[min(k0 + NT * b, D - 1) * sa.nb_chunks];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int k = k0 + NT * b;
                if (k < D) {
                    // neighbour mean in the rows' order
                    float ms = 0.0f;
                    int cnt = 0;
                    for (int ch = 0; ch < sa.nb_chunks; ++ch) {
                        const uint4 w = ch == 0 ? pre[b] : nbrow[k * sa.nb_chunks + ch];
                        const uint32_t wv[4] = {w.x, w.y, w.z, w.w};
                        float rv[8];
#pragma unroll
                        for (int t8 = 0; t8 < 8; ++t8) {
                            const uint32_t j = (wv[t8 >> 1] >> (16 * (t8 & 1))) & 0xffffu;
                            rv[t8] = Rold[j];
                            cnt += j != (uint32_t)D;
                        }
#pragma unroll
                        for (int t8 = 0; t8 < 8; ++t8) ms += rv[t8];
                    }
                    const float Rk0 = Rold[k];
                    const float mk = cnt > 0 ? ms / (float)cnt : Rk0;
                    float Rn = Rk0 - half_eps * (float)D * gk[k] - relax * (Rk0 - mk);
                    if (Rn < p.r_lo) {
                        Rn = p.r_lo;
                        clamped = 1;
                    }
                    if (Rn > p.r_hi) {
                        Rn = p.r_hi;
                        clamped = 1;
                    }
                    finite_r = finite_r && isfinite(Rn);
                    mv = fmaxf(mv, fabsf(Rn - Rk0));
                    sum += Rn;
                    mx = fmaxf(mx, Rn);
                    Rnew[k] = Rn;
                    gk[k] = 0.0f;
                }
            }
        }
        mv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_max_to_63(mv)), 63));
        mx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_max_to_63(mx)), 63));
        clamped = __builtin_amdgcn_ballot_w64(clamped != 0) != 0;
        bool fin_r = __builtin_amdgcn_ballot_w64(!finite_r) == 0;
        if constexpr (NW == 1) {
            sum = group_sum_wave<64>(sum);
        } else {
            const float ws = wave_sum_to_63(sum);
            if (lane == 63) {
                red[wave * 8] = mv;
                red[wave * 8 + 1] = mx;
                red[wave * 8 + 2] = ws;
                red[wave * 8 + 3] = clamped ? 1.0f : 0.0f;
                red[wave * 8 + 4] = fin_r ? 1.0f : 0.0f;
            }
            __syncthreads();
            mv = red[0];
            mx = red[1];
            sum = red[2];
            clamped = red[3] != 0.0f;
            fin_r = red[4] != 0.0f;
            for (int w = 1; w < NW; ++w) {
                mv = fmaxf(mv, red[w * 8]);
                mx = fmaxf(mx, red[w * 8 + 1]);
                sum += red[w * 8 + 2];
                clamped = clamped || red[w * 8 + 3] != 0.0f;
                fin_r = fin_r && red[w * 8 + 4] != 0.0f;
            }
        }
        rmax = mx;
        Rmean = sum / (float)D;
        e_mc = E;
        float dc2 = 0.0f;
        bool finite = fin_r && isfinite(E);
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            const float dcp = -half_eps * gc[ax];
            dc2 = fmaf(dcp, dcp, dc2);
            off[ax] += dcp * inv_h[ax];
            finite = finite && isfinite(off[ax]);
        }
        uint8_t flag = (status & SNK_CLAMPED) | (clamped ? SNK_CLAMPED : 0);
        uint8_t st = SNK_ACTIVE;
        if (!finite) {
            st = SNK_NONFINITE;
        } else {
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) {
                if (fabsf(off[ax]) >= 0.5f) {
                    const float kk = rintf(off[ax]);
                    anc[ax] += (int)kk;
                    off[ax] -= kk;
                }
                if (off[ax] < (float)(-anc[ax]) || off[ax] > (float)(vol.n[ax] - 1 - anc[ax])) st = SNK_OUT;
            }
        }
        if (st == SNK_ACTIVE) {
            const bool small = mv * mv < tol2 && dc2 < tol2;
            streak = small ? min(streak + 1, 255) : 0;
            if (p.conv_window > 0 && streak >= p.conv_window) st = SNK_CONVERGED;
        }
        status = (uint8_t)uni<64>((int)(st | flag));
        streak = uni<64>(streak);
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            off[ax] = uni<64>(off[ax]);
            anc[ax] = uni<64>(anc[ax]);
        }
        float *t = Rold;
        Rold = Rnew;
        Rnew = t;
        ++ran;
        // no barrier here: the next iteration first writes the ray tables and the next block's
        // draws, which nothing reads after this iteration's last barrier, and its barrier after
        // the ray tables orders everything else
    }
    if (budget > 0) {
        for (int k = t; k < D; k += NT) Rg[k] = Rold[k];
        if (t == 0) {
            DevContour o = s;
            for (int i = 0; i < 3; ++i) {
                o.anc[i] = anc[i];
                o.off[i] = off[i];
            }
            o.R = Rmean;
            o.e_mc = e_mc;
            o.iters = n;
            o.status = status;
            o.streak = (uint8_t)streak;
            *slot = o;
            atomicAdd(a.counter, (unsigned long long)ran);
        }
    }
}

template <int DIM, int NT>
hipError_t launch_star_t(const EvolveArgs &a, const StarArgs &sa, int layout, hipStream_t s) {
    const size_t lds = sizeof(float) * (size_t)star_lds_floats<DIM>(a.p.D, a.p.M, NT);
    switch (layout) {
        case kBufferQuad:
            hipLaunchKernelGGL((star_kernel<DIM, kBufferQuad, NT>), dim3(a.n), dim3(NT), lds, s, a, sa);
            break;
        case kBufferPair:
            hipLaunchKernelGGL((star_kernel<DIM, kBufferPair, NT>), dim3(a.n), dim3(NT), lds, s, a, sa);
            break;
        case kBufferPlain:
            hipLaunchKernelGGL((star_kernel<DIM, kBufferPlain, NT>), dim3(a.n), dim3(NT), lds, s, a, sa);
            break;
        default:
            hipLaunchKernelGGL((star_kernel<DIM, kGlobalPlain, NT>), dim3(a.n), dim3(NT), lds, s, a, sa);
            break;
    }
    return hipGetLastError();
}

template <int DIM>
hipError_t launch_star_d(const EvolveArgs &a, const StarArgs &sa, int lanes, int layout, hipStream_t s) {
    if (lanes == 128) return launch_star_t<DIM, 128>(a, sa, layout, s);
    if (lanes == 64) return launch_star_t<DIM, 64>(a, sa, layout, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_evolve(const EvolveArgs &a, int dim, int lanes, int unroll, int layout, bool trace,
                         hipStream_t s) {
    if (a.n <= 0 || a.n_iter <= 0) return hipSuccess;
    if (a.p.flags & kFlagGradI) {
        if (a.p.flags & kFlagExact) return hipErrorInvalidValue;
        if (dim == 2) return trace ? launch_gradi_g<2, true>(a, lanes, layout, s) : launch_gradi_g<2, false>(a, lanes, layout, s);
        return trace ? launch_gradi_g<3, true>(a, lanes, layout, s) : launch_gradi_g<3, false>(a, lanes, layout, s);
    }
    if (a.p.flags & kFlagExact) {
        if (layout == kBufferQuad) return hipErrorInvalidValue;
        if (dim == 2) return trace ? launch_exact_g<2, true>(a, lanes, layout, s) : launch_exact_g<2, false>(a, lanes, layout, s);
        return trace ? launch_exact_g<3, true>(a, lanes, layout, s) : launch_exact_g<3, false>(a, lanes, layout, s);
    }
    if (dim == 2)
        return trace ? launch_g<2, true>(a, lanes, unroll, layout, s) : launch_g<2, false>(a, lanes, unroll, layout, s);
    return trace ? launch_g<3, true>(a, lanes, unroll, layout, s) : launch_g<3, false>(a, lanes, unroll, layout, s);
}

hipError_t launch_evolve_batch(const BatchArgs &a, int dim, int lanes, int unroll, int layout, bool persistent,
                               int grid, hipStream_t s) {
    if (a.n_items <= 0 || a.chunk <= 0) return hipSuccess;
    if (layout != kBufferQuad && layout != kBufferPlain && layout != kBufferPair) return hipErrorInvalidValue;
    if (dim == 2) return batch_g<2>(a, lanes, unroll, layout, persistent, grid, s);
    return batch_g<3>(a, lanes, unroll, layout, persistent, grid, s);
}

namespace {
__global__ __launch_bounds__(256) void star_init_kernel(const DevContour *st, float *Rk, int n, int D) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < (long)n * D) Rk[i] = st[i / D].R;
}
}  // namespace

hipError_t launch_star_init(const DevContour *st, float *Rk, int n, int D, hipStream_t s) {
    const long total = (long)n * D;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(star_init_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, st, Rk, n, D);
    return hipGetLastError();
}

hipError_t launch_star(const EvolveArgs &a, const StarArgs &sa, int dim, int lanes, int layout, hipStream_t s) {
    if (a.n <= 0 || a.n_iter <= 0) return hipSuccess;
    return dim == 2 ? launch_star_d<2>(a, sa, lanes, layout, s) : launch_star_d<3>(a, sa, lanes, layout, s);
}

size_t star_lds_bytes(int dim, int D, int M, int lanes) {
    return sizeof(float) * (size_t)(dim == 2 ? star_lds_floats<2>(D, M, lanes) : star_lds_floats<3>(D, M, lanes));
}

int evolve_batch_max_blocks(int dim, int lanes, int unroll, int layout, int max_M, int tile_cap) {
    return dim == 2 ? max_blocks_g<2>(lanes, unroll, layout, max_M, tile_cap)
                    : max_blocks_g<3>(lanes, unroll, layout, max_M, tile_cap);
}

namespace {

template <int DIM, int G, int U>
int stage_blocks_t(int layout) {
    int nb = 0;
    hipError_t e;
    if (layout == kBufferQuad)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, evolve_kernel<DIM, G, U, false, kBufferQuad, false, true, false>, Grp<G>::NT, 0);
    else if (DIM == 3 && layout == kBufferPair)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, evolve_kernel<DIM, G, U, false, DIM == 3 ? kBufferPair : kBufferPlain, false, true, false>,
            Grp<G>::NT, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, evolve_kernel<DIM, G, U, false, kBufferPlain, false, true, false>, Grp<G>::NT, 0);
    return e == hipSuccess ? nb : 0;
}

template <int DIM, int G>
int stage_blocks_u(int unroll, int layout) {
    if constexpr (G == 64 || G == 128)
        if (unroll >= 4) return stage_blocks_t<DIM, G, 4>(layout);
    return unroll >= 2 ? stage_blocks_t<DIM, G, 2>(layout) : stage_blocks_t<DIM, G, 1>(layout);
}

template <int DIM>
int stage_blocks_g(int lanes, int unroll, int layout) {
    switch (lanes) {
        case 64: return stage_blocks_u<DIM, 64>(unroll, layout);
        case 128: return stage_blocks_u<DIM, 128>(unroll, layout);
        case 256: return stage_blocks_u<DIM, 256>(unroll, layout);
        default: return 0;
    }
}

}  // namespace

int evolve_stage_blocks_per_cu(int dim, int lanes, int unroll, int layout) {
    if (layout != kBufferQuad && layout != kBufferPlain && !(dim == 3 && layout == kBufferPair)) return 0;
    return dim == 2 ? stage_blocks_g<2>(lanes, unroll, layout) : stage_blocks_g<3>(lanes, unroll, layout);
}

size_t evolve_lds_bytes(int dim, int lanes, int M, int tile_cap) {
    const int MH = M / 2;
    const int G = lanes;
    const int per = (draw_floats(G, MH) + 3) & ~3;
    const int cpb = G < 64 ? 64 / G : 1;
    const int waves = G > 64 ? G / 64 : 1;
    return sizeof(float) * ((size_t)cpb * per + (G > 64 ? 2 * (2 + dim) * waves : 0) + (size_t)tile_cap);
}

}  // namespace snk
