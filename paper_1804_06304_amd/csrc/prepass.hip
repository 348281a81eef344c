// Pre-pass: affine intensity map and separable Gaussian low-pass (the paper's low-pass filter that
// keeps Monte-Carlo integration well behaved, Sec. II-E), clamp-to-edge, raw u8/u16/f32 -> FP32,
// optionally also written in the evolve kernels' quad layout.
//
// One workgroup evaluates the filters on a 64 x EY (x, y) tile (EY = 16, 8 or 4: the tallest whose
// LDS fits) and marches along a chunk of z; it outputs the first 63 x (EY - 1) of it, the extra
// column and row being the +x / +y neighbours of the quad records, so every phase maps exactly one
// tile column to each lane. Per input plane: stage the plane with its x/y halo in LDS from
// registers that were fetched while the previous plane was filtered (A), filter along x (B), filter
// along y into a ring of 2*rz+1 planes that each thread reads back for the z filter (C, D), then
// write J and the quad records of the tile from an LDS copy of the filtered plane (E).
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
__device__ __forceinline__ float raw_value(const void *raw, long i) {
    return static_cast<float>(static_cast<const T *>(raw)[i]);
}

// RXY / RZ >= 0: the filter radii are compile-time constants (tap loops unroll, taps live in scalar
// registers); -1: taken from the arguments. EY: evaluated rows per tile.
template <typename T, int EY, int RXY, int RZ>
__global__ __launch_bounds__(NT) void prepass_kernel(PrepassArgs a, int z_chunk) {
    constexpr int TY = EY - 1;  // output rows (the last evaluated one is the +y neighbour)
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
    float *ring = tmp + PH * EX;           // K x EY x EX (xy-filtered)
    float *out = ring + K * EY * EX;       // EY x EX (filtered plane)

    const int x0 = blockIdx.x * TX;
    const int y0 = blockIdx.y * TY;
    const int z0 = blockIdx.z * z_chunk;
    const int z1 = min(a.nz, z0 + z_chunk);
    const int t = threadIdx.x;
    const int tx = t & (EX - 1);           // tile column of this lane in every phase
    const int ty = t >> 6;                 // rows ty, ty + 4, ...
    const long nxy = (long)a.nx * a.ny;
    // neighbour column of the quad records, clamped to the last voxel of the volume
    const int cx1 = min(min(x0 + tx + 1, a.nx - 1) - x0, EX - 1);

    // raw plane values of this thread (rows ty + 4i, columns tx + 64j), clamp-to-edge
    float pre[NRA][NCA];
    auto fetch = [&](int zi) {
        const long zoff = (long)min(max(zi, 0), a.nz - 1) * nxy;
#pragma unroll
        for (int i = 0; i < NRA; ++i) {
            const int r = ty + RS * i;
            if (r < PH) {
                const long yoff = zoff + (long)min(max(y0 + r - ry, 0), a.ny - 1) * a.nx;
#pragma unroll
                for (int j = 0; j < NCA; ++j) {
                    const int c = tx + EX * j;
                    if (c < PW) pre[i][j] = raw_value<T>(a.raw, yoff + min(max(x0 + c - rx, 0), a.nx - 1));
                }
            }
        }
    };

    int slot = 0;                          // ring slot of the plane being filtered
    fetch(z0 - rz);
    for (int zi = z0 - rz; zi < z1 + rz; ++zi) {
        // A: the plane (fetched during the previous plane) into LDS, then fetch the next one
#pragma unroll
        for (int i = 0; i < NRA; ++i) {
            const int r = ty + RS * i;
            if (r < PH) {
#pragma unroll
                for (int j = 0; j < NCA; ++j) {
                    const int c = tx + EX * j;
                    if (c < PW) plane[r * PW + c] = (pre[i][j] - a.i_offset) * a.i_scale;
                }
            }
        }
        __syncthreads();
        if (zi + 1 < z1 + rz) fetch(zi + 1);
        // B: x filter
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
        // C: y filter into the ring (each thread later reads back only its own elements)
#pragma unroll
        for (int r = ty; r < EY; r += RS) {
            float acc = 0.0f;
            for (int k = 0; k <= 2 * ry; ++k) acc = fmaf(a.gy[k], tmp[(r + k) * EX + tx], acc);
            ring[(slot * EY + r) * EX + tx] = acc;
        }
        const int zo = zi - rz;
        if (zo >= z0) {
            // D: z filter over planes zo - rz .. zo + rz (ring slots slot - 2rz .. slot, in order)
            int s0 = slot + 1;
            if (s0 == K) s0 = 0;
#pragma unroll
            for (int r = ty; r < EY; r += RS) {
                float acc = 0.0f;
                int s = s0;
                for (int k = 0; k < K; ++k) {
                    acc = fmaf(a.gz[k], ring[(s * EY + r) * EX + tx], acc);
                    s = s + 1 == K ? 0 : s + 1;
                }
                out[r * EX + tx] = acc;
            }
            __syncthreads();
            // E: J and the quad records of the tile
            const int x = x0 + tx;
            if (tx < TX && x < a.nx) {
#pragma unroll
                for (int r = ty; r < TY; r += RS) {
                    const int y = y0 + r;
                    if (y < a.ny) {
                        const int r1 = min(y + 1, a.ny - 1) - y0;
                        const long o = zo * nxy + (long)y * a.nx + x;
                        const float v = out[r * EX + tx];
                        a.J[o] = v;
                        if (a.Jq)
                            a.Jq[o] = make_float4(v, out[r * EX + cx1], out[r1 * EX + tx], out[r1 * EX + cx1]);
                    }
                }
            }
        }
        slot = slot + 1 == K ? 0 : slot + 1;
    }
}

size_t prepass_lds_bytes(int rx, int ry, int rz, int ey) {
    return sizeof(float) * ((ey + 2 * ry) * (EX + 2 * rx) + (ey + 2 * ry) * EX + (2 * rz + 1) * ey * EX + ey * EX);
}

int prepass_rows(int rx, int ry, int rz) {
    for (int ty : {16, 8, 4})
        if (prepass_lds_bytes(rx, ry, rz, ty) <= kPrepassMaxLds) return ty;
    return 0;
}

template <typename T, int EY, int RXY, int RZ>
hipError_t launch_ty(const PrepassArgs &a, hipStream_t s) {
    const int bx = (a.nx + TX - 1) / TX;
    const int by = (a.ny + EY - 2) / (EY - 1);
    const long bxy = (long)bx * by;
    int chunks = 1;
    if (bxy < 2048) chunks = (int)((2048 + bxy - 1) / bxy);
    chunks = std::min(chunks, a.nz);
    int z_chunk = (a.nz + chunks - 1) / chunks;
    z_chunk = std::max(z_chunk, std::min(a.nz, 4));
    const int bz = (a.nz + z_chunk - 1) / z_chunk;
    const size_t lds = prepass_lds_bytes(a.rx, a.ry, a.rz, EY);
    hipLaunchKernelGGL((prepass_kernel<T, EY, RXY, RZ>), dim3(bx, by, bz), dim3(NT), lds, s, a, z_chunk);
    return hipGetLastError();
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

bool prepass_lds_limit_ok(int rx, int ry, int rz) { return prepass_rows(rx, ry, rz) != 0; }

hipError_t launch_prepass(const PrepassArgs &a, hipStream_t s) {
    switch (a.dtype) {
        case SNK_U8: return launch_t<uint8_t>(a, s);
        case SNK_U16: return launch_t<uint16_t>(a, s);
        default: return launch_t<float>(a, s);
    }
}

}  // namespace snk
