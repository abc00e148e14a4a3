// Batched, strided 2-D transpose through LDS tiles, shared by the layout
// transposes of the host-ingest path and the F-engine's corner turn:
//
//     dst[b * dbs + c * drs + r] = src[b * sbs + r * srs + c]
//
// for r < R, c < C, b < B (elements of E = 4, 8 or 16 bytes).  A 32 x 32 tile
// padded by one element per row: reads run along c and writes along r, 32
// consecutive elements per 32 lanes.
#pragma once
#include <algorithm>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace xc {

constexpr int TP_TILE = 32;

template <typename E>
__global__ __launch_bounds__(256) void transpose_tiles(const E *__restrict__ src, E *__restrict__ dst, int R, int C,
                                                       int64_t srs, int64_t drs, int64_t sbs, int64_t dbs, int64_t b0) {
    __shared__ E tile[TP_TILE][TP_TILE + 1];
    const int64_t b = b0 + blockIdx.z;
    const int c0 = blockIdx.x * TP_TILE, r0 = blockIdx.y * TP_TILE;
    const int tx = threadIdx.x & (TP_TILE - 1), ty = threadIdx.x / TP_TILE;
    const E *in = src + b * sbs;
    E *out = dst + b * dbs;
#pragma unroll
    for (int k = 0; k < TP_TILE; k += 256 / TP_TILE) {
        const int r = r0 + ty + k, c = c0 + tx;
        if (r < R && c < C) tile[ty + k][tx] = in[(int64_t)r * srs + c];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TP_TILE; k += 256 / TP_TILE) {
        const int c = c0 + ty + k, r = r0 + tx;
        if (r < R && c < C) out[(int64_t)c * drs + r] = tile[tx][ty + k];
    }
}

// Launches the transpose for B batches (in chunks of at most 65535 in the
// grid's z dimension); elem_bytes picks E.  R and C must be >= 1.
inline hipError_t launch_transpose_tiles(const void *src, void *dst, int elem_bytes, int R, int C, int64_t srs,
                                         int64_t drs, int64_t sbs, int64_t dbs, int64_t B, hipStream_t stream) {
    const dim3 block(256);
    for (int64_t b0 = 0; b0 < B; b0 += 65535) {
        const dim3 grid((C + TP_TILE - 1) / TP_TILE, (R + TP_TILE - 1) / TP_TILE,
                        (unsigned)std::min<int64_t>(B - b0, 65535));
        switch (elem_bytes) {
        case 16:
            hipLaunchKernelGGL(transpose_tiles<uint4>, grid, block, 0, stream, static_cast<const uint4 *>(src),
                               static_cast<uint4 *>(dst), R, C, srs, drs, sbs, dbs, b0);
            break;
        case 8:
            hipLaunchKernelGGL(transpose_tiles<uint2>, grid, block, 0, stream, static_cast<const uint2 *>(src),
                               static_cast<uint2 *>(dst), R, C, srs, drs, sbs, dbs, b0);
            break;
        default:
            hipLaunchKernelGGL(transpose_tiles<uint32_t>, grid, block, 0, stream,
                               static_cast<const uint32_t *>(src), static_cast<uint32_t *>(dst), R, C, srs, drs, sbs,
                               dbs, b0);
            break;
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace xc
