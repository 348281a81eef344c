// Pre-pass: affine intensity map and separable Gaussian low-pass (the paper's low-pass filter that
// keeps Monte-Carlo integration well behaved, Sec. II-E), clamp-to-edge, raw u8/u16/f32 -> FP32.
//
// One workgroup owns a 64 x 16 (x, y) output tile and marches along z. Each input plane is staged
// once into LDS with its x/y halo, filtered along x then y inside LDS, and the xy-filtered values
// go into a per-thread ring of 2*rz+1 planes; the z filter reads that ring. HBM traffic is the raw
// read (plus halo re-reads that mostly hit L2) and one FP32 write per voxel.
#include <algorithm>

#include "snk_internal.h"

namespace snk {

namespace {

constexpr int TX = kPrepassTX;
constexpr int TY = kPrepassTY;
constexpr int NT = 256;
constexpr int ROWS_PER_THREAD = TX * TY / NT;  // 4

template <typename T>
__device__ __forceinline__ float raw_value(const void *raw, long i) {
    return static_cast<float>(static_cast<const T *>(raw)[i]);
}

template <typename T>
__global__ __launch_bounds__(NT) void prepass_kernel(PrepassArgs a, int z_chunk) {
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
    const int ty = t / TX;                 // 0..3; rows ty, ty+4, ty+8, ty+12
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

}  // namespace

hipError_t launch_prepass(const PrepassArgs &a, hipStream_t s) {
    const int bx = (a.nx + TX - 1) / TX;
    const int by = (a.ny + TY - 1) / TY;
    const long bxy = (long)bx * by;
    int chunks = 1;
    if (bxy < 2048) chunks = (int)((2048 + bxy - 1) / bxy);
    chunks = std::min(chunks, a.nz);
    int z_chunk = (a.nz + chunks - 1) / chunks;
    z_chunk = std::max(z_chunk, std::min(a.nz, 4));
    const int bz = (a.nz + z_chunk - 1) / z_chunk;
    const size_t lds = sizeof(float) * ((size_t)(TY + 2 * a.ry) * (TX + 2 * a.rx) +
                                        (size_t)(TY + 2 * a.ry) * TX + (size_t)(2 * a.rz + 1) * TY * TX);
    dim3 grid(bx, by, bz), block(NT);
    switch (a.dtype) {
        case SNK_U8: hipLaunchKernelGGL(prepass_kernel<uint8_t>, grid, block, lds, s, a, z_chunk); break;
        case SNK_U16: hipLaunchKernelGGL(prepass_kernel<uint16_t>, grid, block, lds, s, a, z_chunk); break;
        default: hipLaunchKernelGGL(prepass_kernel<float>, grid, block, lds, s, a, z_chunk); break;
    }
    return hipGetLastError();
}

}  // namespace snk
