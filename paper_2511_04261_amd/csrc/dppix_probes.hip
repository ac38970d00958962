// Streaming probes: the practical HBM ceilings the library's kernels are
// measured against (built as libdppix_probes.so, apart from the library).
//
//   dppix_probe_stream  linear copy, read-only and write-only passes over a
//                       buffer, 16-byte non-temporal accesses, one access per
//                       lane (the best case of a pure stream);
//   dppix_probe_tiles   a copy in the forward's shape: frames of rows `pitch`
//                       bytes apart cut into bands of `tile_rows` rows and tiles
//                       of `tile_bytes` bytes per row; a workgroup reads its
//                       whole tile into registers, waits at a barrier, then
//                       writes it (what a tile kernel that must see its whole
//                       tile before writing can do at best).
//
// Both return hipErrorInvalidValue for shapes they do not cover, before any
// launch.  They allocate nothing.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4u g_v4u;

__device__ __forceinline__ v4u ld_nt(const void* p) { return __builtin_nontemporal_load((const g_v4u*)p); }
__device__ __forceinline__ void st_nt(void* p, v4u v) { __builtin_nontemporal_store(v, (g_v4u*)p); }

__global__ __launch_bounds__(256) void k_copy(const uint8_t* src, uint8_t* dst, int64_t n16)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16)
        st_nt(dst + 16 * i, ld_nt(src + 16 * i));
}

// Reads every byte; the xor of what a lane read is written only if it equals
// a value the caller passes and never occurs in its data, so the loads stay.
__global__ __launch_bounds__(256) void k_read(const uint8_t* src, uint32_t* sink, int64_t n16, uint32_t never)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) {
        const v4u v = ld_nt(src + 16 * i);
        const uint32_t x = v.x ^ v.y ^ v.z ^ v.w;
        if (x == never)
            sink[0] = x;
    }
}

__global__ __launch_bounds__(256) void k_write(uint8_t* dst, int64_t n16, uint32_t value)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16)
        st_nt(dst + 16 * i, v4u{value, value, value, value});
}

constexpr int kTileLanes = 256;
constexpr int kTileLoads = 16;   // 16-byte strips one lane holds

// One workgroup per (frame, band, tile); strips of the tile are numbered row
// by row and lane t holds strips t, t + 256, ... (consecutive lanes read
// consecutive strips of a row).
__global__ __launch_bounds__(kTileLanes) void k_tile_copy(const uint8_t* src, uint8_t* dst, int64_t frame_bytes,
                                                          int64_t pitch, int rows, int tile_rows, int row_bytes,
                                                          int tile_bytes, int tiles_per_band, int bands)
{
    const int tid = threadIdx.x;
    const int64_t wg = blockIdx.x;
    const int64_t f = wg / ((int64_t)bands * tiles_per_band);
    const int rest = (int)(wg - f * bands * tiles_per_band);
    const int band = rest / tiles_per_band, tile = rest - band * tiles_per_band;
    const int y0 = band * tile_rows, x0 = tile * tile_bytes;
    const int ty = min(tile_rows, rows - y0), tx = min(tile_bytes, row_bytes - x0);
    const int per_row = tx >> 4;
    const int strips = ty * per_row;
    const uint8_t* s0 = src + f * frame_bytes + (int64_t)y0 * pitch + x0;
    uint8_t* d0 = dst + f * frame_bytes + (int64_t)y0 * pitch + x0;
    v4u w[kTileLoads];
#pragma unroll
    for (int k = 0; k < kTileLoads; ++k) {
        const int q = tid + k * kTileLanes;
        if (q < strips) {
            const int y = q / per_row, x = q - y * per_row;
            w[k] = ld_nt(s0 + (int64_t)y * pitch + 16 * x);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTileLoads; ++k) {
        const int q = tid + k * kTileLanes;
        if (q < strips) {
            const int y = q / per_row, x = q - y * per_row;
            st_nt(d0 + (int64_t)y * pitch + 16 * x, w[k]);
        }
    }
}

}  // namespace

extern "C" {

// mode 0: copy bytes from src to dst; 1: read src; 2: write dst.  bytes: a
// multiple of 16; src and dst 16-byte aligned device buffers of that size
// (dst: 4 bytes at least for mode 1, where it is only written if the data
// contain `never` as the xor of a 16-byte word).
hipError_t dppix_probe_stream(int mode, const void* src, void* dst, int64_t bytes, uint32_t never, hipStream_t s)
{
    if (bytes <= 0 || (bytes & 15) != 0 || mode < 0 || mode > 2 ||
        ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) != 0 ||
        (mode != 2 && src == nullptr) || dst == nullptr)
        return hipErrorInvalidValue;
    const int64_t n16 = bytes >> 4;
    const int64_t grid = (n16 + 255) / 256;
    if (grid > INT32_MAX)
        return hipErrorInvalidValue;
    const uint8_t* sp = static_cast<const uint8_t*>(src);
    uint8_t* dp = static_cast<uint8_t*>(dst);
    if (mode == 0)
        hipLaunchKernelGGL(k_copy, dim3((unsigned)grid), dim3(256), 0, s, sp, dp, n16);
    else if (mode == 1)
        hipLaunchKernelGGL(k_read, dim3((unsigned)grid), dim3(256), 0, s, sp, reinterpret_cast<uint32_t*>(dp), n16,
                           never);
    else
        hipLaunchKernelGGL(k_write, dim3((unsigned)grid), dim3(256), 0, s, dp, n16, 0x5A5A5A5Au);
    return hipGetLastError();
}

// Tile-shaped copy of `frames` frames of `rows` rows, `row_bytes` bytes used
// of each `pitch`-byte row, frames frame_bytes apart in both buffers.
// tile_rows x tile_bytes tiles, at most 256 x 16 strips of 16 bytes each;
// row_bytes, tile_bytes and pitch multiples of 16, buffers 16-byte aligned.
hipError_t dppix_probe_tiles(const void* src, void* dst, int32_t frames, int64_t frame_bytes, int64_t pitch,
                             int32_t rows, int32_t row_bytes, int32_t tile_rows, int32_t tile_bytes, hipStream_t s)
{
    if (src == nullptr || dst == nullptr || frames <= 0 || rows <= 0 || row_bytes <= 0 || tile_rows <= 0 ||
        tile_bytes <= 0 || ((row_bytes | tile_bytes) & 15) != 0 || (pitch & 15) != 0 || pitch < row_bytes ||
        frame_bytes < pitch * (int64_t)rows ||
        ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst) | (uintptr_t)frame_bytes) & 15) != 0 ||
        (int64_t)tile_rows * (tile_bytes / 16) > (int64_t)kTileLanes * kTileLoads)
        return hipErrorInvalidValue;
    const int tiles_per_band = (row_bytes + tile_bytes - 1) / tile_bytes;
    const int bands = (rows + tile_rows - 1) / tile_rows;
    const int64_t grid = (int64_t)frames * bands * tiles_per_band;
    if (grid > INT32_MAX)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tile_copy, dim3((unsigned)grid), dim3(kTileLanes), 0, s, static_cast<const uint8_t*>(src),
                       static_cast<uint8_t*>(dst), frame_bytes, pitch, rows, tile_rows, row_bytes, tile_bytes,
                       tiles_per_band, bands);
    return hipGetLastError();
}

}  // extern "C"
