// dppix_tiles.h — LDS carving of one work tile, shared by the host (to size
// dynamic LDS) and the kernels (to place their buffers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dppix {

constexpr int kRowGroup = 8;   // subgrid rows summed per pass of the u8 forward
constexpr int kRowGroupF = 4;  // subgrid rows summed per pass of the fp32 forward (all channels)

enum TileKind : int {
    kPlan = 0,       // plan unit: mask counts per cell, complex cells per tile
    kFwdU8 = 1,      // forward, uint8 HWC
    kFwdF32 = 2,     // forward, fp32 CHW
    kRecU8 = 3,      // reconstruction, uint8 HWC
    kRecF32 = 4,     // reconstruction, fp32 CHW
    kBwd = 5         // adjoint reduction, fp32 CHW
};

struct LdsPlan {
    uint32_t colsum;  // per padded column (byte or float) of the tile; reused as the expanded output row
    uint32_t cspart;  // per (subcell column, channel) running sum over subcell rows
    uint32_t cidx;    // per cell: index within its class (frame-local)
    uint32_t cflag;   // per cell: 1 = complex
    uint32_t vgs;     // per (cell, channel): value of a simple cell (adjoint: its gradient)
    uint32_t vgc;     // per (subcell row, subcell column, channel): value of a complex subcell (adjoint: gradient)
    uint32_t cxl;     // u8 forward: the tile's complex cells in order (uint16 each)
    uint32_t bytes;
};

__host__ __device__ inline uint32_t al16(uint32_t x) { return (x + 15u) & ~15u; }

// Number of 16-byte strips covering K cells of one padded row of the tile.
__host__ __device__ inline uint32_t tile_strips(int kind, int K, int b, int C)
{
    if (kind == kFwdF32 || kind == kRecF32 || kind == kBwd)
        return (uint32_t)((K * b + 3) / 4);
    return (uint32_t)((K * b * C + 15) / 16);
}

__host__ __device__ inline LdsPlan lds_plan(int kind, int K, int b, int n, int C)
{
    LdsPlan p{};
    const uint32_t nstr = tile_strips(kind, K, b, C);
    uint32_t o = 0;
    p.colsum = o;
    // u8 forward: 16-bit column sums of up to kRowGroup subgrid rows (reused
    // as two expanded output rows); f32 forward: float column sums of every
    // channel for up to kRowGroupF subgrid rows (reused likewise); f32
    // reconstruction: two expanded output rows; adjoint: float column sums
    // like the f32 forward
    if (kind == kFwdU8)
        o += al16(32u * nstr * (uint32_t)(n < kRowGroup ? n : kRowGroup));
    else if (kind == kFwdF32) {
        // float4 column sums per (channel, subgrid row of a group), at least
        // the two expanded output rows of the reconstruction
        const uint32_t rows = (uint32_t)C * (uint32_t)(n < kRowGroupF ? n : kRowGroupF);
        o += al16(16u * nstr * (rows > 2u ? rows : 2u));
    } else if (kind == kBwd) {
        // float4 column sums per (channel, subgrid row of a group), at least
        // the two expanded rows of the gradient broadcast
        const uint32_t rows = (uint32_t)C * (uint32_t)(n < kRowGroupF ? n : kRowGroupF);
        o += al16(16u * nstr * (rows > 2u ? rows : 2u));
    }
    else
        o += al16(32u * nstr);
    p.cspart = o;
    if (kind == kFwdU8)
        o += al16(4u * (uint32_t)(K * n * C));
    else if (kind == kFwdF32 || kind == kBwd)
        o += al16(8u * (uint32_t)(K * n * C));
    p.cidx = o;
    o += al16(4u * (uint32_t)K);
    p.cflag = o;
    o += al16((uint32_t)K);
    p.vgs = o;
    if (kind == kFwdU8 || kind == kRecU8)
        o += al16((uint32_t)(K * C));
    else if (kind == kFwdF32 || kind == kRecF32 || kind == kBwd)
        o += al16(4u * (uint32_t)(K * C));
    p.vgc = o;
    if (kind == kFwdU8 || kind == kRecU8)
        o += al16((uint32_t)(K * n * n * C));
    else if (kind == kFwdF32 || kind == kRecF32 || kind == kBwd)
        o += al16(4u * (uint32_t)(K * n * n * C));
    p.cxl = o;
    if (kind == kFwdU8)
        o += al16(2u * (uint32_t)K);
    p.bytes = o;
    return p;
}

// LDS of one plan unit: a 32-bit mask count per cell of cnb bands x ctx
// tiles of K cells, and a complex-cell count per tile.
__host__ __device__ inline uint32_t plan_lds(int cnb, int ctx, int K)
{
    return 4u * (uint32_t)cnb * (uint32_t)(ctx * K + ctx);
}

}  // namespace dppix
