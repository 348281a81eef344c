// Pre-pass: affine intensity map and separable Gaussian low-pass (the paper's low-pass filter that
// keeps Monte-Carlo integration well behaved, Sec. II-E), clamp-to-edge, raw u8/u16/f32 -> FP32,
// optionally also written in the evolve kernels' quad layout, or (2D) their column-pair layout.
//
// One workgroup evaluates the filters on a 64 x EY (x, y) tile (EY = 16, 8 or 4: the tallest whose
// LDS fits) and marches along a chunk of z; it outputs the first 63 x (EY - 1) of it, the extra
// column and row being the +x / +y neighbours of the quad records, so every phase maps exactly one
// tile column to each lane. Per input plane: stage the plane with its x/y halo in LDS from
// registers that were fetched while the previous plane was filtered (A), filter along x (B), filter
// along y into a ring of 2*rz+1 planes that each thread reads back for the z filter (C, D), then
// write J and the quad records or column pairs of the tile from an LDS copy of the filtered plane
// (E). Each thread
// z-filters only the elements it y-filtered, so with compile-time radii the ring lives in its
// registers (less LDS per workgroup, more workgroups per CU); the generic instance keeps it in LDS.
// Thread-to-element maps use shifts only: no integer division in any loop. HBM traffic: the raw read (halo re-reads mostly hit L2), 4 B of J and 16 B of quad
// records per voxel.
#include <algorithm>

#include "snk_internal.h"

namespace snk {

namespace {

constexpr int EX = kPrepassTX;  // 64 columns evaluated per tile
constexpr int TX = EX - 1;      // 63 output columns (the last evaluated one is the +x neighbour)
constexpr int NT = 256;
constexpr int RS = NT / EX;     // row stride of the thread map (4)

template <typename T>
__device__ __forceinline__ T raw_value(const void *raw, long i) {
    return static_cast<const T *>(raw)[i];
}

// RXY / RZ >= 0: the filter radii are compile-time constants (tap loops unroll, taps live in scalar
// registers); -1: taken from the arguments. EY: evaluated rows per tile. SECOND: also write the quad
// records (1) or the column pairs of a 2D image (2).
template <typename T, int EY, int RXY, int RZ, int SECOND>
__global__ __launch_bounds__(NT) void prepass_kernel(PrepassArgs a, int z_chunk) {
    constexpr int TY = EY - 1;  // output rows (the last evaluated one is the +y neighbour)
    constexpr bool REG_RING = RZ >= 0;
    constexpr int KR = REG_RING ? 2 * RZ + 1 : 1;   // register ring depth
    constexpr int NRT = (EY + RS - 1) / RS;          // y-filtered rows per thread
    constexpr int RMAX = RXY >= 0 ? RXY : kPrepassMaxR;
    constexpr int NRA = (EY + 2 * RMAX + RS - 1) / RS;  // plane rows per thread (upper bound)
    constexpr int NCA = (EX + 2 * RMAX + EX - 1) / EX;  // plane columns per thread (upper bound)
    extern __shared__ float lds[];
    const int rx = RXY >= 0 ? RXY : a.rx;
    const int ry = RXY >= 0 ? RXY : a.ry;
    const int rz = RZ >= 0 ? RZ : a.rz;
    const int PW = EX + 2 * rx;            // plane row width
    const int PH = EY + 2 * ry;            // plane rows
    const int K = 2 * rz + 1;              // ring depth
    float *plane = lds;                    // PH x PW
    float *tmp = plane + PH * PW;          // PH x EX (x-filtered)
    float *ring = tmp + PH * EX;           // K x EY x EX (xy-filtered; generic instance only)
    float *out = ring + (REG_RING ? 0 : K * EY * EX);  // EY x EX (filtered plane)
    // register ring: rr[i][k] = y-filtered row ty + RS i of plane zi - (KR - 1) + k
    float rr[NRT][KR];
#pragma unroll
    for (int i = 0; i < NRT; ++i)
#pragma unroll
        for (int k = 0; k < KR; ++k) rr[i][k] = 0.0f;

    const int x0 = blockIdx.x * TX;
    const int y0 = blockIdx.y * TY;
    const int z0 = blockIdx.z * z_chunk;
    const int z1 = min(a.nz, z0 + z_chunk);
    const int t = threadIdx.x;
    const int tx = t & (EX - 1);           // tile column of this lane in every phase
    const int ty = t >> 6;                 // rows ty, ty + 4, ...
    const long nxy = (long)a.nx * a.ny;
    // output column of this lane: the evaluated +x neighbour column and columns past the volume
    // store the value of the last output column inside it again (a duplicate write of the same
    // value), so every thread issues the same number of stores per plane and waiting for the next
    // plane's loads never has to wait for this plane's stores
    const int xc = min(x0 + min(tx, TX - 1), a.nx - 1);
    const int tc = xc - x0;
    // neighbour column of the quad records, clamped to the last voxel of the volume
    const int cx1 = min(min(xc + 1, a.nx - 1) - x0, EX - 1);

    // raw plane values of this thread (rows ty + 4i, columns tx + 64j), clamp-to-edge. Every load is
    // issued unconditionally (slots past the plane read a clamped, valid address and are never
    // stored), so no branch forces a wait between them and they stay in flight while the current
    // plane is filtered.
    T pre[NRA][NCA];  // raw values: converted only when staged, so nothing waits on the loads earlier
    auto fetch = [&](int zi) {
        const long zoff = (long)min(max(zi, 0), a.nz - 1) * nxy;
#pragma unroll
        for (int i = 0; i < NRA; ++i) {
            const int r = min(ty + RS * i, PH - 1);
            const long yoff = zoff + (long)min(max(y0 + r - ry, 0), a.ny - 1) * a.nx;
#pragma unroll
            for (int j = 0; j < NCA; ++j) {
                const int c = min(tx + EX * j, PW - 1);
                pre[i][j] = raw_value<T>(a.raw, yoff + min(max(x0 + c - rx, 0), a.nx - 1));
            }
        }
    };

    int slot = 0;                          // ring slot of the plane being filtered
    // A: the plane (fetched during the previous plane) into LDS, then fetch the next one (always:
    // past the chunk it re-reads a clamped plane, so every plane issues the same loads)
    auto stage = [&](int zi) {
#pragma unroll
        for (int i = 0; i < NRA; ++i) {
            const int r = ty + RS * i;
            if (r < PH) {
#pragma unroll
                for (int j = 0; j < NCA; ++j) {
                    const int c = tx + EX * j;
                    if (c < PW) plane[r * PW + c] = ((float)pre[i][j] - a.i_offset) * a.i_scale;
                }
            }
        }
        __syncthreads();
        fetch(zi + 1);
    };
    // B: x filter; C: y filter into the ring (each thread later reads back only its own elements)
    auto filter_xy = [&]() {
#pragma unroll
        for (int i = 0; i < NRA; ++i) {
            const int r = ty + RS * i;
            if (r < PH) {
                const float *row = plane + r * PW + tx;
                float acc = 0.0f;
                for (int k = 0; k <= 2 * rx; ++k) acc = fmaf(a.gx[k], row[k], acc);
                tmp[r * EX + tx] = acc;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NRT; ++i) {
            const int r = ty + RS * i;
            if (r < EY) {
                float acc = 0.0f;
                for (int k = 0; k <= 2 * ry; ++k) acc = fmaf(a.gy[k], tmp[(r + k) * EX + tx], acc);
                if constexpr (REG_RING) {
#pragma unroll
                    for (int k = 0; k + 1 < KR; ++k) rr[i][k] = rr[i][k + 1];
                    rr[i][KR - 1] = acc;
                } else {
                    ring[(slot * EY + r) * EX + tx] = acc;
                }
            }
        }
    };

    fetch(z0 - rz);
    // the first 2 rz planes only fill the ring
    int zi = z0 - rz;
    for (; zi < z0 + rz; ++zi) {
        stage(zi);
        filter_xy();
        slot = slot + 1 == K ? 0 : slot + 1;
    }
    for (; zi < z1 + rz; ++zi) {
        stage(zi);
        filter_xy();
        const int zo = zi - rz;
        // D: z filter over planes zo - rz .. zo + rz (oldest ring entry first)
        int s0 = slot + 1;
        if (s0 == K) s0 = 0;
#pragma unroll
        for (int i = 0; i < NRT; ++i) {
            const int r = ty + RS * i;
            if (r < EY) {
                float acc = 0.0f;
                if constexpr (REG_RING) {
#pragma unroll
                    for (int k = 0; k < KR; ++k) acc = fmaf(a.gz[k], rr[i][k], acc);
                } else {
                    int s = s0;
                    for (int k = 0; k < K; ++k) {
                        acc = fmaf(a.gz[k], ring[(s * EY + r) * EX + tx], acc);
                        s = s + 1 == K ? 0 : s + 1;
                    }
                }
                out[r * EX + tx] = acc;
            }
        }
        __syncthreads();
        // E: J and the quad records or column pairs of the tile (rows past the tile or the volume
        // store the last row inside both again)
#pragma unroll
        for (int i = 0; i < (TY + RS - 1) / RS; ++i) {
            const int y = min(y0 + min(ty + RS * i, TY - 1), a.ny - 1);
            const int r = y - y0;
            const int r1 = min(y + 1, a.ny - 1) - y0;
            const long o = zo * nxy + (long)y * a.nx + xc;
            const float v = out[r * EX + tc];
            a.J[o] = v;
            if constexpr (SECOND == 1) {
                // non-temporal: the quad records (4x the volume) are written past the caches, which
                // shortens the pre-pass (0.20 -> 0.17 ms on the slab) and does not slow the evolution
                // that gathers from them
                typedef float f4v __attribute__((ext_vector_type(4)));
                const f4v q = {v, out[r * EX + cx1], out[r1 * EX + tc], out[r1 * EX + cx1]};
                __builtin_nontemporal_store(q, reinterpret_cast<f4v *>(&a.Jq[o]));
            }
            if constexpr (SECOND == 2) a.Jp[o] = make_float2(v, out[r1 * EX + tc]);
        }
        slot = slot + 1 == K ? 0 : slot + 1;
    }
}

// ring_lds: the z ring is held in LDS (generic instance) rather than in registers.
size_t prepass_lds_bytes(int rx, int ry, int rz, int ey, bool ring_lds = true) {
    return sizeof(float) * ((ey + 2 * ry) * (EX + 2 * rx) + (ey + 2 * ry) * EX + (ring_lds ? (2 * rz + 1) * ey * EX : 0) +
                            ey * EX);
}

int prepass_rows(int rx, int ry, int rz) {
    for (int ty : {16, 8, 4})
        if (prepass_lds_bytes(rx, ry, rz, ty) <= kPrepassMaxLds) return ty;
    return 0;
}

template <typename T, int EY, int RXY, int RZ, int SECOND>
hipError_t launch_q(const PrepassArgs &a, hipStream_t s) {
    const int bx = (a.nx + TX - 1) / TX;
    const int by = (a.ny + EY - 2) / (EY - 1);
    const long bxy = (long)bx * by;
    int chunks = 1;
    if (bxy < 2048) chunks = (int)((2048 + bxy - 1) / bxy);
    chunks = std::min(chunks, a.nz);
    int z_chunk = (a.nz + chunks - 1) / chunks;
    z_chunk = std::max(z_chunk, std::min(a.nz, 4));
    const int bz = (a.nz + z_chunk - 1) / z_chunk;
    const size_t lds = prepass_lds_bytes(a.rx, a.ry, a.rz, EY, RZ < 0);
    hipLaunchKernelGGL((prepass_kernel<T, EY, RXY, RZ, SECOND>), dim3(bx, by, bz), dim3(NT), lds, s, a, z_chunk);
    return hipGetLastError();
}

template <typename T, int EY, int RXY, int RZ>
hipError_t launch_ty(const PrepassArgs &a, hipStream_t s) {
    if (a.Jq) return launch_q<T, EY, RXY, RZ, 1>(a, s);
    if (a.Jp) return launch_q<T, EY, RXY, RZ, 2>(a, s);
    return launch_q<T, EY, RXY, RZ, 0>(a, s);
}

// Radii of sigma_pre = 1 on unit (x, y) spacing with z spacing 1, 2 or a 2D image get unrolled
// instances; every other radius set runs the generic one.
template <typename T>
hipError_t launch_t(const PrepassArgs &a, hipStream_t s) {
    const int ey = prepass_rows(a.rx, a.ry, a.rz);
    if (ey == 16 && a.rx == 3 && a.ry == 3) {
        if (a.rz == 2) return launch_ty<T, 16, 3, 2>(a, s);
        if (a.rz == 3) return launch_ty<T, 16, 3, 3>(a, s);
        if (a.rz == 0) return launch_ty<T, 16, 3, 0>(a, s);
    }
    switch (ey) {
        case 16: return launch_ty<T, 16, -1, -1>(a, s);
        case 8: return launch_ty<T, 8, -1, -1>(a, s);
        case 4: return launch_ty<T, 4, -1, -1>(a, s);
        default: return hipErrorInvalidValue;
    }
}

// Quad records of one row segment from an existing J: J(x,y), J(x+1,y), J(x,y+1), J(x+1,y+1) of
// plane z, the neighbours clamped to the last column / row (only cells with x <= nx-2, y <= ny-2 are
// gathered).
__global__ __launch_bounds__(256) void pack_quad_kernel(const float *__restrict__ J, float4 *__restrict__ Jq,
                                                       int nx, int ny, int nz) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int y = blockIdx.y;
    const int z = blockIdx.z;
    if (x >= nx) return;
    const long row = ((long)z * ny + y) * nx;
    const long row1 = ((long)z * ny + min(y + 1, ny - 1)) * nx;
    const int x1 = min(x + 1, nx - 1);
    Jq[row + x] = make_float4(J[row + x], J[row + x1], J[row1 + x], J[row1 + x1]);
}

}  // namespace

hipError_t launch_pack_quad(const float *J, float4 *Jq, int nx, int ny, int nz, hipStream_t s) {
    if (nx <= 0 || ny <= 0 || nz <= 0) return hipSuccess;
    if (ny > 65535 || nz > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pack_quad_kernel, dim3((nx + 255) / 256, ny, nz), dim3(256), 0, s, J, Jq, nx, ny, nz);
    return hipGetLastError();
}

namespace {
// Column pairs of a 2D image: Jp[y][x] = (J[y][x], J[y + 1][x]), the last row paired with itself.
__global__ __launch_bounds__(256) void pack_pair_kernel(const float *__restrict__ J, float2 *__restrict__ Jp,
                                                        int nx, int ny) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int y = blockIdx.y;
    const long plane = (long)blockIdx.z * ny * nx;
    if (x >= nx) return;
    const long row = plane + (long)y * nx, row1 = plane + (long)min(y + 1, ny - 1) * nx;
    Jp[row + x] = make_float2(J[row + x], J[row1 + x]);
}
}  // namespace

hipError_t launch_pack_pair(const float *J, float2 *Jp, int nx, int ny, int nz, hipStream_t s) {
    if (nx <= 0 || ny <= 0 || nz <= 0) return hipSuccess;
    hipLaunchKernelGGL(pack_pair_kernel, dim3((nx + 255) / 256, ny, nz), dim3(256), 0, s, J, Jp, nx, ny);
    return hipGetLastError();
}

bool prepass_lds_limit_ok(int rx, int ry, int rz) { return prepass_rows(rx, ry, rz) != 0; }

hipError_t launch_prepass(const PrepassArgs &a, hipStream_t s) {
    switch (a.dtype) {
        case SNK_U8: return launch_t<uint8_t>(a, s);
        case SNK_U16: return launch_t<uint16_t>(a, s);
        default: return launch_t<float>(a, s);
    }
}

}  // namespace snk
