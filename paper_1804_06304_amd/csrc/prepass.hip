// Pre-pass: affine intensity map and separable Gaussian low-pass (the paper's low-pass filter that
// keeps Monte-Carlo integration well behaved, Sec. II-E), clamp-to-edge, raw u8/u16/f32 -> FP32.
//
// One workgroup owns a 64 x TY (x, y) output tile (TY = 16, 8 or 4: the tallest whose LDS fits) and
// marches along z. Each input plane is staged
// once into LDS with its x/y halo, filtered along x then y inside LDS, and the xy-filtered values
// go into a per-thread ring of 2*rz+1 planes; the z filter reads that ring. HBM traffic is the raw
// read (plus halo re-reads that mostly hit L2) and one FP32 write per voxel.
#include <algorithm>

#include "snk_internal.h"

namespace snk {

namespace {

constexpr int TX = kPrepassTX;
constexpr int NT = 256;

template <typename T>
__device__ __forceinline__ float raw_value(const void *raw, long i) {
    return static_cast<float>(static_cast<const T *>(raw)[i]);
}

template <typename T, int TY>
__global__ __launch_bounds__(NT) void prepass_kernel(PrepassArgs a, int z_chunk) {
    constexpr int ROWS_PER_THREAD = TX * TY / NT;
    extern __shared__ float lds[];
    const int rx = a.rx, ry = a.ry, rz = a.rz;
    const int PW = TX + 2 * rx;            // plane row width
    const int PH = TY + 2 * ry;            // plane rows
    const int K = 2 * rz + 1;              // ring depth
    float *plane = lds;                    // PH x PW
    float *tmp = plane + PH * PW;          // PH x TX
    float *ring = tmp + PH * TX;           // K x TY x TX

    const int x0 = blockIdx.x * TX;
    const int y0 = blockIdx.y * TY;
    const int z0 = blockIdx.z * z_chunk;
    const int z1 = min(a.nz, z0 + z_chunk);
    const int t = threadIdx.x;
    const int tx = t % TX;
    const int ty = t / TX;                 // 0..3; rows ty, ty+4, ...
    const long nxy = (long)a.nx * a.ny;

    for (int zi = z0 - rz; zi < z1 + rz; ++zi) {
        const int zc = min(max(zi, 0), a.nz - 1);
        const long zoff = zc * nxy;
        for (int idx = t; idx < PH * PW; idx += NT) {
            const int r = idx / PW, c = idx % PW;
            const int y = min(max(y0 + r - ry, 0), a.ny - 1);
            const int x = min(max(x0 + c - rx, 0), a.nx - 1);
            plane[idx] = (raw_value<T>(a.raw, zoff + (long)y * a.nx + x) - a.i_offset) * a.i_scale;
        }
        __syncthreads();
        for (int idx = t; idx < PH * TX; idx += NT) {
            const int r = idx / TX, c = idx % TX;
            const float *row = plane + r * PW + c;
            float acc = 0.0f;
            for (int k = 0; k <= 2 * rx; ++k) acc = fmaf(a.gx[k], row[k], acc);
            tmp[idx] = acc;
        }
        __syncthreads();
        const int slot = (zi - (z0 - rz)) % K;
#pragma unroll
        for (int q = 0; q < ROWS_PER_THREAD; ++q) {
            const int r = ty + 4 * q;
            float acc = 0.0f;
            for (int k = 0; k <= 2 * ry; ++k) acc = fmaf(a.gy[k], tmp[(r + k) * TX + tx], acc);
            ring[(slot * TY + r) * TX + tx] = acc;
        }
        const int zo = zi - rz;
        if (zo >= z0) {
            const int x = x0 + tx;
#pragma unroll
            for (int q = 0; q < ROWS_PER_THREAD; ++q) {
                const int r = ty + 4 * q;
                float acc = 0.0f;
                for (int k = 0; k < K; ++k) {
                    const int s = (zo - z0 + k) % K;
                    acc = fmaf(a.gz[k], ring[(s * TY + r) * TX + tx], acc);
                }
                const int y = y0 + r;
                if (x < a.nx && y < a.ny) a.J[zo * nxy + (long)y * a.nx + x] = acc;
            }
        }
    }
}

size_t prepass_lds_bytes(int rx, int ry, int rz, int ty) {
    return sizeof(float) * ((size_t)(ty + 2 * ry) * (TX + 2 * rx) + (size_t)(ty + 2 * ry) * TX +
                            (size_t)(2 * rz + 1) * ty * TX);
}

int prepass_rows(int rx, int ry, int rz) {
    for (int ty : {16, 8, 4})
        if (prepass_lds_bytes(rx, ry, rz, ty) <= kPrepassMaxLds) return ty;
    return 0;
}

template <typename T, int TY>
hipError_t launch_ty(const PrepassArgs &a, hipStream_t s) {
    const int bx = (a.nx + TX - 1) / TX;
    const int by = (a.ny + TY - 1) / TY;
    const long bxy = (long)bx * by;
    int chunks = 1;
    if (bxy < 2048) chunks = (int)((2048 + bxy - 1) / bxy);
    chunks = std::min(chunks, a.nz);
    int z_chunk = (a.nz + chunks - 1) / chunks;
    z_chunk = std::max(z_chunk, std::min(a.nz, 4));
    const int bz = (a.nz + z_chunk - 1) / z_chunk;
    const size_t lds = prepass_lds_bytes(a.rx, a.ry, a.rz, TY);
    hipLaunchKernelGGL((prepass_kernel<T, TY>), dim3(bx, by, bz), dim3(NT), lds, s, a, z_chunk);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_t(const PrepassArgs &a, hipStream_t s) {
    switch (prepass_rows(a.rx, a.ry, a.rz)) {
        case 16: return launch_ty<T, 16>(a, s);
        case 8: return launch_ty<T, 8>(a, s);
        case 4: return launch_ty<T, 4>(a, s);
        default: return hipErrorInvalidValue;
    }
}

// Quad records of one row segment: J(x,y), J(x+1,y), J(x,y+1), J(x+1,y+1) of plane z, the
// neighbours clamped to the last column / row (only cells with x <= nx-2, y <= ny-2 are gathered).
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
