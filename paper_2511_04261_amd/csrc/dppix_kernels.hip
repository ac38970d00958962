// dppix_kernels.hip — gfx950 kernels of libdppix.
//
// The path is bandwidth-bound: per pixel it reads the image (and, in the plan,
// the mask) once and writes the reconstruction once; the statistics are a few
// percent of that.  Nothing is a dense contraction, so there is no MFMA work.
// Every tile kernel follows one pattern:
//   1. a work item is one 16-byte strip of the tile's padded rows over one
//      (or a few) subgrid rows; it issues all of its row loads, then sums
//      them in registers (two 16-bit lanes per 32-bit register for bytes:
//      255 * 256 rows still fits);
//   2. the column sums go to LDS, where one lane per (subcell column,
//      channel) adds its s_b columns — exact integer sums of every s_b x s_b
//      subcell;
//   3. a coarse cell's sum is the exact total of its n x n subcell sums
//      (Eq. 16-17: b = n * s_b), so simple and complex cells cost the same;
//   4. each released statistic draws one Philox4x32-10 block, turns it into
//      Laplace noise in fp64, clips and rounds once to fp32 (the releases
//      of complex subcells are dealt evenly over the lanes);
//   5. with a fused output, the rounded values are expanded into one padded
//      row in LDS and the strips are stored on the s_b output rows.
// Mirror padding (Algorithm 2 step 4, Algorithm 3 step 3) is never
// materialised: padded rows fold to a source row per row, and padded columns
// fold per byte in the few strips that cross the right edge (which become
// one-row items so their byte loads overlap).  The unpadded mode (Algorithm
// 1) skips those rows and columns and divides by real pixel counts.
#include "dppix_internal.h"
#include "dppix_tiles.h"

#include <math.h>

#include <map>
#include <mutex>
#include <utility>

// Register budget of the u8 forward kernel, as resident waves per SIMD: 4
// leaves 128 VGPRs (no spills with all of a subgrid row's loads in flight).
#ifndef DPPIX_FWD_WAVES_PER_EU
#define DPPIX_FWD_WAVES_PER_EU 4
#endif

namespace dppix {
namespace {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// 16-byte streaming accesses through global (not flat) address space: frame
// pointers come from device tables, so the compiler cannot infer the address
// space, and flat accesses would make every wait cover LDS traffic as well.
typedef __attribute__((address_space(1))) v4u g_v4u;
typedef __attribute__((address_space(1))) v4f g_v4f;
typedef __attribute__((address_space(1))) const uint8_t g_u8;
typedef __attribute__((address_space(1))) uint8_t g_u8w;
typedef __attribute__((address_space(1))) uint16_t g_u16w;
typedef __attribute__((address_space(1))) const float g_f32;
typedef __attribute__((address_space(1))) float g_f32w;

__device__ __forceinline__ v4u ld16_nt(const void* p) { return __builtin_nontemporal_load((const g_v4u*)p); }
__device__ __forceinline__ v4f ld16f_nt(const void* p) { return __builtin_nontemporal_load((const g_v4f*)p); }
__device__ __forceinline__ void st16_nt(void* p, v4u v) { __builtin_nontemporal_store(v, (g_v4u*)p); }
__device__ __forceinline__ void st16f_nt(void* p, v4f v) { __builtin_nontemporal_store(v, (g_v4f*)p); }

// --------------------------------------------------------------------------
// Counter-based noise.  Philox4x32 with ten rounds (Salmon et al., SC'11):
// per round the first and third words are multiplied by two fixed odd
// constants, the high halves of the products are xored with the other two
// words and the round key, and the key advances by two Weyl increments.
// --------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // one 32x32 -> 64-bit product per multiplier gives both halves
        const uint64_t pa = (uint64_t)0xD2511F53u * c.x;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(pb >> 32) ^ c.y ^ k0, (uint32_t)pb, (uint32_t)(pa >> 32) ^ c.w ^ k1, (uint32_t)pa);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Natural log of x in (0, 1] (the Laplace draw's arguments are 2u and
// 2(1-u), never 0, infinite or subnormal), within one ulp: x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), f = m - 1 (exact), s = f / (2 + f), and
// ln(1 + f) = 2 atanh(s) = 2s + sum_{k>=1} 2 s^(2k+1) / (2k+1).  Since
// 2s = f - f^2 / (2 + f), the sum is arranged as f - h + s (h + R) with
// h = f^2 / 2 and R = sum_{k=1..10} 2 z^k / (2k+1), z = s^2 <= 0.0295, so the
// two large terms are exact and the series (truncated below 2^-56 relative)
// only corrects.  ln 2 is split into 42 leading bits (e ln2_hi is exact) and
// the rest.  Against the C library's log on 2e7 such arguments it agrees
// exactly on 93 % and within one ulp on all.
__device__ __forceinline__ double ln_unit(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double R = 2.0 / 21.0;
    R = fma(R, z, 2.0 / 19.0);
    R = fma(R, z, 2.0 / 17.0);
    R = fma(R, z, 2.0 / 15.0);
    R = fma(R, z, 2.0 / 13.0);
    R = fma(R, z, 2.0 / 11.0);
    R = fma(R, z, 2.0 / 9.0);
    R = fma(R, z, 2.0 / 7.0);
    R = fma(R, z, 2.0 / 5.0);
    R = fma(R, z, 2.0 / 3.0);
    R *= z;
    const double h = 0.5 * f * f;
    const double de = (double)e;
    return de * 0x1.62e42fefa3800p-1 - ((h - (s * (h + R) + de * 0x1.ef35793c76730p-45)) - f);
}

// Laplace(0, sigma) sample of one statistic: words 0,1 of the block give a
// uniform u = (2k+1) 2^-53 with k the top 52 bits, inverted through the
// Laplace CDF (Eq. 9) in fp64.
__device__ __forceinline__ double laplace_sample(const FrameRec& F, uint32_t id, int ch, int level, double sigma)
{
    // The key is one frame's, the same in every lane (readfirstlane states
    // that, so it sits in scalar registers at any optimisation level).  The
    // empty asm makes it opaque here, so the ten round keys are recomputed by
    // one scalar add per round instead of being hoisted out of the caller's
    // release loop: there they would take 20 scalar registers the tile
    // kernels do not have, and be spilled to vector lanes and read back by a
    // vector instruction each.
    uint32_t k0 = __builtin_amdgcn_readfirstlane(F.key0), k1 = __builtin_amdgcn_readfirstlane(F.key1);
    asm volatile("" : "+s"(k0), "+s"(k1));
    const uint4 w = philox10(make_uint4(id, (uint32_t)ch | ((uint32_t)level << 8), F.fi0, F.fi1), k0, k1);
    const uint64_t bits = ((uint64_t)w.y << 32) | (uint64_t)w.x;
    const double u = (double)(((bits >> 12) << 1) | 1ull) * 0x1p-53;
    // one log per lane: the two tails differ only in its argument and sign
    const bool lower = u < 0.5;
    const double l = ln_unit(lower ? 2.0 * u : 2.0 * (1.0 - u));
    return lower ? sigma * l : -sigma * l;
}

// Release one statistic: mean = sum / area, plus noise (Eq. 11 scale given by
// the host), clipped to [0, 255] (Algorithm 3 steps 10, 17), one rounding to
// fp32.  pass = the clip did not bind (gradient flows).  inv_area: 1 / area
// when that is exact (area a power of two: the product then equals the
// quotient bit for bit), else 0 (divide).
__device__ __forceinline__ float release(double sum, double area, double inv_area, int noisy, double sigma,
                                         const FrameRec& F, uint32_t id, int ch, int level, uint8_t& pass)
{
    if (area == 0.0) {   // unpadded mode: a subcell with no real pixel releases nothing
        pass = 0;
        return 0.f;
    }
    const double mu = inv_area != 0.0 ? sum * inv_area : sum / area;
    const double z = noisy ? mu + laplace_sample(F, id, ch, level, sigma) : mu;
    pass = (uint8_t)(z >= 0.0 && z <= 255.0);
    const double v = z < 0.0 ? 0.0 : (z > 255.0 ? 255.0 : z);
    return (float)v;
}

__device__ __forceinline__ uint8_t to_u8(float v) { return (uint8_t)rintf(v); }

// Mirror index of padded coordinate x >= 0 into [0, L).
__device__ __forceinline__ int fold(int x, int L, int mode)
{
    if (x < L)
        return x;
    if (mode == 0) {
        if (x < 2 * L)          // first mirror image, the common case
            return 2 * L - 1 - x;
        const int p = 2 * L;
        const int y = x % p;
        return y < L ? y : p - 1 - y;
    }
    if (L == 1)
        return 0;
    if (x < 2 * L - 1)
        return 2 * L - 2 - x;
    const int p = 2 * L - 2;
    const int y = x % p;
    return y < L ? y : p - y;
}

// Unpadded border mode (Algorithm 1): positions past the frame are absent —
// they add nothing to sums or mask counts, and each (sub)cell's mean divides
// by its real pixel count.
constexpr int kPadNone = 2;

// Mirror index of a coordinate in [-1, 2L) for the Sobel stencil: -1 mirrors
// like the frame's own padding, the unpadded mode mirrors like the symmetric one.
__device__ __forceinline__ int edge_fold(int x, int L, int mode)
{
    if (mode == kPadNone)   // the Sobel stencil mirrors like the symmetric mode
        mode = 0;
    if (x < 0)
        return (mode == 0 || L == 1) ? 0 : 1;
    return fold(x, L, mode);
}

// 1 / side^2 when that is exact and every statistic of that side has area
// side^2 (mirror padding, side a power of two), else 0.
__device__ __forceinline__ double exact_inv_area(const FrameRec& F, int side)
{
    return (F.pad != kPadNone && (side & (side - 1)) == 0) ? 1.0 / ((double)side * (double)side) : 0.0;
}

// Real-pixel area of the statistic whose (sub)cell starts at padded (y0, x0)
// with the given side: side^2 when the frame is mirror-padded; h*w real
// pixels in the unpadded mode (0 for a subcell wholly past the frame).
__device__ __forceinline__ double stat_area(const FrameRec& F, int y0, int x0, int side)
{
    if (F.pad != kPadNone)
        return (double)side * (double)side;
    const int h = min(side, F.H - y0), w = min(side, F.W - x0);
    return (h > 0 && w > 0) ? (double)h * (double)w : 0.0;
}

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroup barrier for LDS hand-offs only.  The tile kernels never read
// global memory written by their own workgroup, so outstanding global stores
// (the reconstruction, the store) need not drain at every barrier, which a
// full __syncthreads() would force.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Bytes 1 and 3 of a dword in the low bytes of its two 16-bit halves: one
// byte permute (selector bytes 1, zero, 3, zero) instead of a shift and a mask.
__device__ __forceinline__ uint32_t odd_bytes(uint32_t w) { return __builtin_amdgcn_perm(0u, w, 0x0C030C01u); }

// Add the bytes of one 16-byte strip into 16-bit lane pairs: e[d] holds bytes
// 4d and 4d+2, o[d] bytes 4d+1 and 4d+3.
__device__ __forceinline__ void acc_bytes(const v4u& w, uint32_t (&e)[4], uint32_t (&o)[4])
{
    e[0] += w.x & 0x00FF00FFu; o[0] += odd_bytes(w.x);
    e[1] += w.y & 0x00FF00FFu; o[1] += odd_bytes(w.y);
    e[2] += w.z & 0x00FF00FFu; o[2] += odd_bytes(w.z);
    e[3] += w.w & 0x00FF00FFu; o[3] += odd_bytes(w.w);
}

// Nonzero bytes of a dword as 0/1 bytes.
__device__ __forceinline__ uint32_t nz_bytes(uint32_t w)
{
    return ((((w & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w) >> 7) & 0x01010101u;
}

// Column sums of a strip as 16-bit values in natural byte-column order (a
// subgrid row has at most 256 rows of bytes, so 255 * 256 fits).
__device__ __forceinline__ void store_colsums16(uint16_t* dst, const uint32_t (&e)[4], const uint32_t (&o)[4])
{
    v4u* d4 = reinterpret_cast<v4u*>(dst);
    d4[0] = v4u{(e[0] & 0xFFFFu) | (o[0] << 16), (e[0] >> 16) | (o[0] & 0xFFFF0000u),
                (e[1] & 0xFFFFu) | (o[1] << 16), (e[1] >> 16) | (o[1] & 0xFFFF0000u)};
    d4[1] = v4u{(e[2] & 0xFFFFu) | (o[2] << 16), (e[2] >> 16) | (o[2] & 0xFFFF0000u),
                (e[3] & 0xFFFFu) | (o[3] << 16), (e[3] >> 16) | (o[3] & 0xFFFF0000u)};
}

// Gather one 16-byte strip of a padded row byte by byte: columns past the
// image fold back (mirror; zero in the unpadded mode), bytes past the tile
// end read as zero.  Only the strips that cross the right edge or a
// misaligned row take this path.
template <int C>
__device__ __noinline__ v4u gather_strip_u8(const uint8_t* row, int p0, int tile_end, int W, int pad)
{
    const g_u8* src = (const g_u8*)row;
    // source offsets first (folding branches), then 16 unconditional byte
    // loads issued back to back; bytes past the tile end are masked after
    // (the unpadded mode reads columns past the frame as zero)
    const int end = pad == kPadNone ? min(tile_end, W * C) : tile_end;
    int idx[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int p = p0 + q;
        const int x = p / C, ch = p - x * C;
        idx[q] = p < end ? fold(x, W, pad) * C + ch : 0;
    }
    uint32_t v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        v[q] = src[idx[q]];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        v[q] = p0 + q < end ? v[q] : 0u;
    return v4u{v[0] | (v[1] << 8) | (v[2] << 16) | (v[3] << 24), v[4] | (v[5] << 8) | (v[6] << 16) | (v[7] << 24),
               v[8] | (v[9] << 8) | (v[10] << 16) | (v[11] << 24),
               v[12] | (v[13] << 8) | (v[14] << 16) | (v[15] << 24)};
}

// Cell classes and class-local indices of the tile's cells (wave 0):
// complex cells count from the number of complex cells of the frame before
// the tile, simple cells from the simple ones — row-major order, which is the
// order of the compact store.
// With cxl, also the list of the tile's complex cells in order (cxl[q] = kc
// of the q-th complex cell) and their number in *ncx.
__device__ __forceinline__ void tile_cells(const TileArgs& a, const FrameRec& F, int64_t t, int r, int x0c, int Kt,
                                           uint32_t* cidx, uint8_t* cflag, uint16_t* cxl = nullptr,
                                           uint32_t* ncx = nullptr)
{
    if (threadIdx.x >= 64)
        return;
    const int lane = threadIdx.x;
    uint32_t run_fg = a.tile_fg[t];
    const uint32_t fg0 = run_fg;
    const uint32_t before = (uint32_t)(r * F.GC + x0c);
    uint32_t run_bg = before - run_fg;
    for (int base = 0; base < Kt; base += 64) {
        const int kc = base + lane;
        const bool in = kc < Kt;
        const uint8_t fl = in ? a.flags[F.cell_base + before + kc] : (uint8_t)0;
        const uint64_t m = __ballot(fl != 0);
        const uint64_t below = lane ? (m & (~0ull >> (64 - lane))) : 0ull;
        const uint32_t pc = (uint32_t)__popcll(below);
        if (in) {
            cflag[kc] = fl;
            cidx[kc] = fl ? run_fg + pc : run_bg + (uint32_t)lane - pc;
            if (cxl && fl)
                cxl[run_fg - fg0 + pc] = (uint16_t)kc;
            if (a.cell_index)
                a.cell_index[F.cell_base + before + kc] = cidx[kc];
        }
        const uint32_t nf = (uint32_t)__popcll(m);
        const uint32_t nv = (uint32_t)min(64, Kt - base);
        run_fg += nf;
        run_bg += nv - nf;
    }
    if (ncx && lane == 0)
        *ncx = run_fg - fg0;
}

struct TileCoord {
    int f;
    int64_t t;
    int r, ct;
};

__device__ __forceinline__ TileCoord tile_of(const TileArgs& a, int64_t sched_idx, FrameRec& F)
{
    TileCoord tc;
    // one load: (frame, tile within frame) of this scheduling index
    const int64_t idx = a.sched_offset + sched_idx;
    tc.f = (int)uniform_u32((uint32_t)a.tile_map[2 * idx]);
    const int64_t local = (int64_t)uniform_u32((uint32_t)a.tile_map[2 * idx + 1]);
    F = a.frames[tc.f];
    if (a.noise != nullptr) {
        // this call's noise counters, read at launch time (a replayed graph
        // draws fresh noise once the caller has advanced them)
        const uint64_t key = a.noise[2 * tc.f], ctr = a.noise[2 * tc.f + 1];
        F.key0 = (uint32_t)key;
        F.key1 = (uint32_t)(key >> 32);
        F.fi0 = (uint32_t)ctr;
        F.fi1 = (uint32_t)(ctr >> 32);
    }
    tc.t = F.tile_base + local;
    tc.r = (int)(local / F.TX);
    tc.ct = (int)(local - (int64_t)tc.r * F.TX);
    return tc;
}

// ==========================================================================
// Scans of the plan.
// ==========================================================================
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* wave_tot, T& total)
{
    // inclusive scan inside the wavefront
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    T x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T y = __shfl_up(x, d, 64);
        if (lane >= d)
            x += y;
    }
    if (lane == 63)
        wave_tot[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int i = 0; i < nw; ++i) {
            const T w = wave_tot[i];
            wave_tot[i] = run;
            run += w;
        }
        wave_tot[nw] = run;
    }
    __syncthreads();
    const T excl = x - v + wave_tot[wid];
    total = wave_tot[nw];
    __syncthreads();
    return excl;
}

// Frame-level pass of the scan (k_scan_frames, one workgroup, launched after
// k_scan_tiles): store offsets of every frame (frames concatenated in batch
// order) from the per-frame counts the tile pass wrote, ticket words reset.
__device__ void scan_frames(const TileArgs& a, uint64_t* wave_tot)
{
    uint64_t carry_bg = 0, carry_fg = 0;
    for (int base = 0; base < a.n_frames; base += blockDim.x) {
        const int f = base + threadIdx.x;
        uint64_t vb = 0, vf = 0;
        if (f < a.n_frames) {
            const FrameRec F = a.frames[f];
            vb = a.counts[4 * f] * (uint64_t)F.C;
            vf = a.counts[4 * f + 1] * (uint64_t)F.n * (uint64_t)F.n * (uint64_t)F.C;
        }
        uint64_t tb, tf;
        const uint64_t eb = block_exclusive_scan<uint64_t>(vb, wave_tot, tb);
        const uint64_t ef = block_exclusive_scan<uint64_t>(vf, wave_tot, tf);
        if (f < a.n_frames) {
            a.counts[4 * f + 2] = carry_bg + eb;
            a.counts[4 * f + 3] = carry_fg + ef;
        }
        carry_bg += tb;
        carry_fg += tf;
    }
    if (threadIdx.x < kTicketWords)
        a.ticket[threadIdx.x] = 0;
}

// ==========================================================================
// Plan (Algorithm 3 steps 3-6): classify every cell from the mirror-padded
// mask (k_plan), then scan the complex counts into store offsets (k_scan_prefix,
// or k_scan_tiles and k_scan_frames).
// A plan unit is `cnb` bands x `ctx` tiles of one frame.  Each lane sums one
// 16-byte strip of the mask down up to kPlanRows padded rows with all its
// loads in flight, then hands the strip's column counts to per-cell counters
// in LDS (at most two cells per strip when b >= 16).
// ==========================================================================
constexpr int kPlanRows = 16;   // padded mask rows one lane sums per item
constexpr int kPlanBatch = 8;   // row loads issued back to back

__device__ __forceinline__ v4u nz_strip(const v4u& w)
{
    return v4u{nz_bytes(w.x), nz_bytes(w.y), nz_bytes(w.z), nz_bytes(w.w)};
}

// Column x (0..15) of a strip's packed counts (see acc_bytes).
template <int X>
__device__ __forceinline__ uint32_t col_count(const uint32_t (&e)[4], const uint32_t (&o)[4])
{
    const uint32_t v = (X & 1) ? o[X >> 2] : e[X >> 2];
    return (X & 2) ? (v >> 16) : (v & 0xFFFFu);
}

template <int X>
__device__ __forceinline__ void spread_col(const uint32_t (&e)[4], const uint32_t (&o)[4], uint32_t* cc, int KC,
                                           int b, int& cell, int& next, uint32_t& run)
{
    if (X == next) {
        if (run != 0u && cell < KC)
            atomicAdd(cc + cell, run);
        run = 0u;
        ++cell;
        next += b;
    }
    run += col_count<X>(e, o);
}

// Add the 16 column counts of one strip that starts at padded column p0 of
// the unit to the counters of the cells they fall in.
__device__ __forceinline__ void spread_strip(const uint32_t (&e)[4], const uint32_t (&o)[4], uint32_t* cc, int KC,
                                             int b, int p0)
{
    int cell = p0 / b;
    int next = (cell + 1) * b - p0;
    uint32_t run = 0u;
    spread_col<0>(e, o, cc, KC, b, cell, next, run);
    spread_col<1>(e, o, cc, KC, b, cell, next, run);
    spread_col<2>(e, o, cc, KC, b, cell, next, run);
    spread_col<3>(e, o, cc, KC, b, cell, next, run);
    spread_col<4>(e, o, cc, KC, b, cell, next, run);
    spread_col<5>(e, o, cc, KC, b, cell, next, run);
    spread_col<6>(e, o, cc, KC, b, cell, next, run);
    spread_col<7>(e, o, cc, KC, b, cell, next, run);
    spread_col<8>(e, o, cc, KC, b, cell, next, run);
    spread_col<9>(e, o, cc, KC, b, cell, next, run);
    spread_col<10>(e, o, cc, KC, b, cell, next, run);
    spread_col<11>(e, o, cc, KC, b, cell, next, run);
    spread_col<12>(e, o, cc, KC, b, cell, next, run);
    spread_col<13>(e, o, cc, KC, b, cell, next, run);
    spread_col<14>(e, o, cc, KC, b, cell, next, run);
    spread_col<15>(e, o, cc, KC, b, cell, next, run);
    if (run != 0u && cell < KC)
        atomicAdd(cc + cell, run);
}

// Mask counts of every cell of the unit into cellcnt[j * KCs + kc].
__device__ void plan_count(const TileArgs& a, const FrameRec& F, const uint8_t* mask, int r0, int nb, int c0, int KC,
                           int KCs, uint32_t* cellcnt)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    const int b = F.b, H = F.H, W = F.W, pad = F.pad;
    const int64_t X0 = (int64_t)c0 * b;
    const int WB = KC * b;
    const int nstr = (WB + 15) >> 4;
    const int RI = min(b, kPlanRows);
    const int groups = (b + RI - 1) / RI;
    const int64_t lim = min(X0 + WB, (int64_t)W);
    const bool aligned = ((reinterpret_cast<uintptr_t>(mask) | (uintptr_t)W | (uintptr_t)X0) & 15) == 0;
    // strips [0, nfast) are whole 16-byte vectors inside the frame; the rest
    // (right edge, or every strip of a misaligned mask) are gathered byte by
    // byte, one padded row per item so that their latencies overlap
    const int nfast = aligned ? (int)min((int64_t)nstr, (lim - X0) >> 4) : 0;
    const int nslow = nstr - nfast;
    const int per_band = nfast * groups;
    for (int item = tid; item < nb * per_band; item += NT) {
        const int j = item / per_band;
        const int rem = item - j * per_band;
        const int g = rem / nfast;
        const int st = rem - g * nfast;
        const int64_t p0 = X0 + 16 * st;
        const int row0 = (r0 + j) * b;
        const int k0 = g * RI, k1 = min(b, k0 + RI);
        uint32_t e[4] = {0, 0, 0, 0}, o[4] = {0, 0, 0, 0};
        if (row0 + k1 <= H) {
            // rows inside the frame: no folding
            const uint8_t* col = mask + (int64_t)row0 * W + p0;
            int k = k0;
            for (; k + kPlanBatch <= k1; k += kPlanBatch) {
                v4u w[kPlanBatch];
#pragma unroll
                for (int i = 0; i < kPlanBatch; ++i)
                    w[i] = ld16_nt(col + (int64_t)(k + i) * W);
#pragma unroll
                for (int i = 0; i < kPlanBatch; ++i)
                    acc_bytes(nz_strip(w[i]), e, o);
            }
            if (k < k1) {
                // the last partial batch (b not a multiple of the batch)
                v4u w[kPlanBatch];
#pragma unroll
                for (int i = 0; i < kPlanBatch; ++i)
                    w[i] = k + i < k1 ? ld16_nt(col + (int64_t)(k + i) * W) : v4u{0u, 0u, 0u, 0u};
#pragma unroll
                for (int i = 0; i < kPlanBatch; ++i)
                    acc_bytes(nz_strip(w[i]), e, o);
            }
        } else {
            // bottom border: mirrored rows (absent without padding), still
            // issued a batch at a time so that their latencies overlap
            for (int k = k0; k < k1; k += kPlanBatch) {
                v4u w[kPlanBatch];
#pragma unroll
                for (int i = 0; i < kPlanBatch; ++i) {
                    const int r = row0 + k + i;
                    w[i] = (k + i < k1 && (r < H || pad != kPadNone))
                               ? ld16_nt(mask + (int64_t)fold(r, H, pad) * W + p0)
                               : v4u{0u, 0u, 0u, 0u};
                }
#pragma unroll
                for (int i = 0; i < kPlanBatch; ++i)
                    acc_bytes(nz_strip(w[i]), e, o);
            }
        }
        if ((b & 15) == 0) {
            // b a multiple of 16: the strip lies in one cell, one counter
            // update (a 16-bit half sums at most 8 columns of 16 rows)
            const uint32_t t = (e[0] + e[1] + e[2] + e[3]) + (o[0] + o[1] + o[2] + o[3]);
            const uint32_t cnt = (t & 0xFFFFu) + (t >> 16);
            const int cell = (16 * st) / b;
            if (cnt != 0u && cell < KC)
                atomicAdd(cellcnt + j * KCs + cell, cnt);
        } else {
            spread_strip(e, o, cellcnt + j * KCs, KC, b, 16 * st);
        }
    }
    for (int item = tid; item < nb * b * nslow; item += NT) {
        const int st = nfast + item % nslow;
        const int rest = item / nslow;
        const int k = rest % b, j = rest / b;
        const int64_t p0 = X0 + 16 * st;
        if ((r0 + j) * b + k >= H && pad == kPadNone)
            continue;
        uint32_t e[4] = {0, 0, 0, 0}, o[4] = {0, 0, 0, 0};
        acc_bytes(nz_strip(gather_strip_u8<1>(mask + (int64_t)fold((r0 + j) * b + k, H, pad) * W, (int)p0,
                                              (int)(X0 + WB), W, pad)),
                  e, o);
        spread_strip(e, o, cellcnt + j * KCs, KC, b, 16 * st);
    }
}

// One plan unit: its cell counters cleared, counted by `count(F, f, r0, nb, c0,
// KC, KCs, cellcnt)`, then every cell flagged (count >= tau) and the complex
// cells of every tile counted.
template <typename Count>
__device__ __forceinline__ void plan_unit(const TileArgs& a, uint8_t* lds, Count count)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    const int f = (int)uniform_u32((uint32_t)a.unit_map[2 * (int64_t)blockIdx.x]);
    const int lu = (int)uniform_u32((uint32_t)a.unit_map[2 * (int64_t)blockIdx.x + 1]);
    const FrameRec F = a.frames[f];
    const int chunks = (F.TX + F.ctx - 1) / F.ctx;
    const int band_grp = lu / chunks;
    const int r0 = band_grp * F.cnb;
    const int nb = min(F.cnb, F.GR - r0);
    const int t0 = (lu - band_grp * chunks) * F.ctx;
    const int nt = min(F.ctx, F.TX - t0);
    const int c0 = t0 * F.K;
    const int KC = min(nt * F.K, F.GC - c0);
    const int KCs = F.ctx * F.K;
    uint32_t* cellcnt = reinterpret_cast<uint32_t*>(lds);
    uint32_t* tcnt = cellcnt + F.cnb * KCs;
    for (int i = tid; i < F.cnb * (KCs + F.ctx); i += NT)
        cellcnt[i] = 0u;
    // the store's ticket words start at zero for the scan and later launches
    // of this call sequence (stream order: no earlier launch still uses them)
    if (blockIdx.x == 0 && tid < kTicketWords)
        a.ticket[tid] = 0u;
    lds_barrier();
    count(F, f, r0, nb, c0, KC, KCs, cellcnt);
    lds_barrier();
    for (int i = tid; i < nb * KC; i += NT) {
        const int j = i / KC, kc = i - j * KC;
        // tau = 0 (unpadded mode only): majority of the cell's real pixels
        const uint32_t tau = F.tau > 0 ? (uint32_t)F.tau
                                       : ((uint32_t)stat_area(F, (r0 + j) * F.b, (c0 + kc) * F.b, F.b) + 1u) / 2u;
        const uint8_t fl = (uint8_t)(cellcnt[j * KCs + kc] >= tau);
        a.flags[F.cell_base + (int64_t)(r0 + j) * F.GC + c0 + kc] = fl;
        if (fl)
            atomicAdd(&tcnt[j * F.ctx + kc / F.K], 1u);
    }
    lds_barrier();
    for (int i = tid; i < nb * nt; i += NT) {
        const int j = i / nt, ti = i - j * nt;
        a.tile_cnt[F.tile_base + (int64_t)(r0 + j) * F.TX + t0 + ti] = tcnt[j * F.ctx + ti];
    }
}

__global__ __launch_bounds__(kMaxThreads) void k_plan(TileArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    plan_unit(a, lds, [&](const FrameRec& F, int f, int r0, int nb, int c0, int KC, int KCs, uint32_t* cellcnt) {
        const uint8_t* mask = a.masks ? a.masks[f] : nullptr;
        if (mask != nullptr)
            plan_count(a, F, mask, r0, nb, c0, KC, KCs, cellcnt);
    });
}

// --------------------------------------------------------------------------
// Plan from complexity labels (Sec. VI-A names an edge detector such as the
// Sobel operator as a source of the region mask), in the same pass: a cell's
// count is the number of edge pixels among its b x b mirror-padded
// positions, each position taking the label of the real pixel it folds onto
// (the label dp_pix_edge_mask writes).  No mask is written or read.  The 3x3
// stencil evaluated on the padded grid of channel sums, every coordinate
// folded as the label's border rule folds it (edge_fold), gives exactly the
// label of the folded pixel: a mirror maps the pair of neighbours of a padded
// position onto the pair of neighbours of its image, at most swapped, and a
// swap only flips the sign of Gy.  So each chunk of padded rows and columns is
// staged as channel sums in LDS (one halo row and column on every side) and
// counted without knowing which positions are real.
// --------------------------------------------------------------------------
constexpr int kLabRows = 16;                      // padded rows per chunk (within one band)
constexpr int kLabCols = 512;                     // padded columns per chunk (16 x 512: fastest of 8-32 x 128-1024)
constexpr int kLabPad = 8;                        // LDS columns before column 0 (16-byte aligned rows)
constexpr int kLabStride = kLabCols + 2 * kLabPad;

// Channel sums of 16 consecutive pixels from their 16 C bytes, as eight
// dwords of two 16-bit sums each (pixel 2k low, 2k + 1 high).
template <int C>
__device__ __forceinline__ void pixel_sums16(const v4u (&w)[C], v4u& lo, v4u& hi)
{
    uint32_t d[4 * C];
#pragma unroll
    for (int i = 0; i < C; ++i) {
        d[4 * i + 0] = w[i].x;
        d[4 * i + 1] = w[i].y;
        d[4 * i + 2] = w[i].z;
        d[4 * i + 3] = w[i].w;
    }
    uint32_t pr[8];   // pixel pairs (2k low, 2k + 1 high)
    if constexpr (C == 1) {
        // each byte is its own sum: bytes 0, 1 and 2, 3 of a dword into halves
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            pr[2 * i] = __builtin_amdgcn_perm(0u, d[i], 0x0C010C00u);
            pr[2 * i + 1] = __builtin_amdgcn_perm(0u, d[i], 0x0C030C02u);
        }
    } else if constexpr (C == 2) {
        // a dword is two pixels: (b0 + b1, b2 + b3) as halves
#pragma unroll
        for (int i = 0; i < 8; ++i)
            pr[i] = __builtin_amdgcn_perm(0u, d[i], 0x0C020C00u) + __builtin_amdgcn_perm(0u, d[i], 0x0C030C01u);
    } else if constexpr (C == 3) {
        // three dwords are four pixels: bytes 0-2 | 3-5 | 6-8 | 9-11, each
        // pixel's bytes added by byte dot products with 0/1 weights
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t a = d[3 * i], b = d[3 * i + 1], c = d[3 * i + 2];
            const uint32_t s0 = __builtin_amdgcn_udot4(a, 0x00010101u, 0u, false);
            const uint32_t s1 = __builtin_amdgcn_udot4(b, 0x00000101u, __builtin_amdgcn_udot4(a, 0x01000000u, 0u, false), false);
            const uint32_t s2 = __builtin_amdgcn_udot4(c, 0x00000001u, __builtin_amdgcn_udot4(b, 0x01010000u, 0u, false), false);
            const uint32_t s3 = __builtin_amdgcn_udot4(c, 0x01010100u, 0u, false);
            pr[2 * i] = s0 | (s1 << 16);
            pr[2 * i + 1] = s2 | (s3 << 16);
        }
    } else {
        // a dword is one pixel
#pragma unroll
        for (int i = 0; i < 8; ++i)
            pr[i] = __builtin_amdgcn_udot4(d[2 * i], 0x01010101u, 0u, false) |
                    (__builtin_amdgcn_udot4(d[2 * i + 1], 0x01010101u, 0u, false) << 16);
    }
    lo = v4u{pr[0], pr[1], pr[2], pr[3]};
    hi = v4u{pr[4], pr[5], pr[6], pr[7]};
}

// Channel sums of the staged chunk: staged row yy is padded row py0 - 1 + yy,
// staged column xx padded column px0 + xx (xx = -1 .. cols), each folded into
// the frame as the label's border rule folds it; whole 16-pixel groups inside
// the frame are read as vectors (aligned rows), the rest one pixel at a time.
template <int C>
__device__ __forceinline__ void stage_label_sums(const uint8_t* img, int64_t pitch, int H, int W, int pad, int py0,
                                                 int rows, int px0, int cols, bool aligned, uint16_t* S)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    const int gfast = (aligned && (px0 & 15) == 0) ? max(0, min(cols, W - px0)) >> 4 : 0;
    for (int it = tid; it < (rows + 2) * gfast; it += NT) {
        const int yy = it / gfast, g = it - yy * gfast;
        const int ry = edge_fold(py0 - 1 + yy, H, pad);
        const uint8_t* src = img + (int64_t)ry * pitch + (int64_t)(px0 + 16 * g) * C;
        v4u w[C];
#pragma unroll
        for (int i = 0; i < C; ++i)
            w[i] = ld16_nt(src + 16 * i);
        v4u lo, hi;
        pixel_sums16<C>(w, lo, hi);
        v4u* dst = reinterpret_cast<v4u*>(S + yy * kLabStride + kLabPad + 16 * g);
        dst[0] = lo;
        dst[1] = hi;
    }
    const int nrest = cols + 2 - 16 * gfast;
    for (int it = tid; it < (rows + 2) * nrest; it += NT) {
        const int yy = it / nrest, q = it - yy * nrest;
        const int xx = q == 0 ? -1 : 16 * gfast + q - 1;
        const int ry = edge_fold(py0 - 1 + yy, H, pad);
        const int rx = edge_fold(px0 + xx, W, pad);
        const g_u8* px = (const g_u8*)(img + (int64_t)ry * pitch + (int64_t)rx * C);
        uint32_t sum = 0u;
#pragma unroll
        for (int ch = 0; ch < C; ++ch)
            sum += px[ch];
        S[yy * kLabStride + kLabPad + xx] = (uint16_t)sum;
    }
}

// Sobel labels of the staged column pair (2p, 2p + 1) down rows y0 .. y1 - 1
// of the chunk, the two columns in the 16-bit halves of one register:
// Gx = dx(-1) + 2 dx(0) + dx(+1), Gy = sx(+1) - sx(-1), with
// dx(r) = S[r][+1] - S[r][-1], sx(r) = S[r][-1] + 2 S[r][0] + S[r][+1].
// With S <= 4 * 255 every intermediate fits a signed 16-bit half exactly
// (|Gx|, |Gy| <= 4080), and so does thr - 1 - (|Gx| + |Gy|) for thr <= 16384:
// its sign is the label.  emit(y, d) gets that difference, bit 15 = label of
// column 2p, bit 31 = label of column 2p + 1.  Each row is three dword reads
// (the pair and its two neighbouring pairs, 4-byte aligned).
typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void sobel_row_pair(const uint32_t* r, s16x2& dx, s16x2& sx)
{
    const uint32_t w0 = r[-1], w1 = r[0], w2 = r[1];
    const s16x2 l = __builtin_bit_cast(s16x2, __builtin_amdgcn_alignbit(w1, w0, 16));   // S[-1], S[0]
    const s16x2 c = __builtin_bit_cast(s16x2, w1);                                      // S[0], S[+1]
    const s16x2 rr = __builtin_bit_cast(s16x2, __builtin_amdgcn_alignbit(w2, w1, 16));  // S[+1], S[+2]
    dx = rr - l;
    sx = (l + rr) + (c + c);
}

template <typename Emit>
__device__ __forceinline__ void label_pair(const uint16_t* S, int p, int y0, int y1, int thr, Emit emit)
{
    constexpr int RW = kLabStride / 2;                       // dwords per staged row
    const uint32_t* row = reinterpret_cast<const uint32_t*>(S + kLabPad) + y0 * RW + p;
    const s16x2 t = {(short)(thr - 1), (short)(thr - 1)};
    s16x2 dxa, sxa, dxb, sxb;
    sobel_row_pair(row, dxa, sxa);
    sobel_row_pair(row + RW, dxb, sxb);
    row += 2 * RW;
    for (int y = y0; y < y1; ++y, row += RW) {
        s16x2 dxc, sxc;
        sobel_row_pair(row, dxc, sxc);
        const s16x2 gx = (dxa + dxc) + (dxb + dxb), gy = sxc - sxa;
        const s16x2 mag = __builtin_elementwise_abs(gx) + __builtin_elementwise_abs(gy);
        emit(y, __builtin_bit_cast(uint32_t, t - mag));
        dxa = dxb;
        sxa = sxb;
        dxb = dxc;
        sxb = sxc;
    }
}

// Lanes over the column pairs of a chunk: pairs 0 .. np - 1, and when the
// pairs are fewer than the lanes, the rows split over up to 4 lane groups
// (each group whole waves).  split = this lane's row group (>= splits: idle).
struct PairLanes {
    int step, pl, split, splits, rper;
};

__device__ __forceinline__ PairLanes pair_lanes(int np, int rows)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    const int npr = (np + 63) & ~63;
    PairLanes L;
    L.splits = npr >= NT ? 1 : min(4, NT / npr);
    L.step = L.splits == 1 ? NT : npr;
    L.pl = L.splits == 1 ? tid : tid % npr;
    L.split = L.splits == 1 ? 0 : tid / npr;
    L.rper = (rows + L.splits - 1) / L.splits;
    return L;
}

template <int C>
__device__ void plan_count_labels(const TileArgs& a, const FrameRec& F, const uint8_t* img, int r0, int nb, int c0,
                                  int KC, int KCs, uint32_t* cellcnt, uint16_t* S)
{
    const int b = F.b, H = F.H, W = F.W, pad = F.pad;
    const int64_t pitch = F.pitch;
    const int thr = a.edge_threshold * C;
    const int X0 = c0 * b, XW = KC * b;
    const int R = min(b, kLabRows);
    const bool aligned = ((reinterpret_cast<uintptr_t>(img) | (uintptr_t)pitch) & 15) == 0;
    // b a power of two up to 64: chunks start on cell boundaries and the
    // lanes of one cell add their counts by shuffles first (one LDS atomic
    // per cell and chunk instead of one per lane)
    const bool groups = (b & (b - 1)) == 0 && b <= 64;
    for (int j = 0; j < nb; ++j) {
        const int band0 = (r0 + j) * b;
        for (int k0 = 0; k0 < b; k0 += R) {
            const int rows = min(R, b - k0);
            const int py0 = band0 + k0;
            // unpadded mode: rows past the frame are absent
            const int ylim = pad == kPadNone ? min(rows, H - py0) : rows;
            if (ylim <= 0)
                break;
            for (int cx = 0; cx < XW; cx += kLabCols) {
                const int cols = min(kLabCols, XW - cx);
                const int px0 = X0 + cx;
                stage_label_sums<C>(img, pitch, H, W, pad, py0, rows, px0, cols, aligned, S);
                lds_barrier();
                // a lane per pair of padded columns, down its share of the rows
                const int np = (cols + 1) >> 1;
                const PairLanes L = pair_lanes(np, ylim);
                const int ya = L.split * L.rper, yb = min(ylim, ya + L.rper);
                for (int pb = 0; pb < np; pb += L.step) {
                    const int p = pb + L.pl, x = 2 * p;
                    // valid columns: inside the chunk, and real in the unpadded mode
                    const int xend = pad == kPadNone ? min(cols, W - px0) : cols;
                    const uint32_t vm = (x < xend ? 0x8000u : 0u) | (x + 1 < xend ? 0x80000000u : 0u);
                    uint32_t cnt = 0u, cnt_hi = 0u;
                    if (vm != 0u && L.split < L.splits && ya < yb) {
                        if ((b & 1) == 0)
                            label_pair(S, p, ya, yb, thr, [&](int, uint32_t d) { cnt += __builtin_popcount(d & vm); });
                        else
                            label_pair(S, p, ya, yb, thr, [&](int, uint32_t d) {
                                d &= vm;
                                cnt += (d >> 15) & 1u;
                                cnt_hi += d >> 31;
                            });
                    }
                    // b even: both columns lie in one cell
                    const int cell = (cx + x) / b;
                    if (groups && b >= 2) {
                        for (int m = 1; m < (b >> 1); m <<= 1)
                            cnt += __shfl_xor(cnt, m, 64);
                        if ((L.pl & ((b >> 1) - 1)) == 0 && cnt != 0u && cell < KC)
                            atomicAdd(cellcnt + j * KCs + cell, cnt);
                    } else {
                        if (cnt != 0u && cell < KC)
                            atomicAdd(cellcnt + j * KCs + cell, cnt);
                        const int cell_hi = (cx + x + 1) / b;
                        if (cnt_hi != 0u && cell_hi < KC)
                            atomicAdd(cellcnt + j * KCs + cell_hi, cnt_hi);
                    }
                }
                lds_barrier();
            }
        }
    }
}

// One launch per channel count present in the batch: a workgroup whose unit
// belongs to a frame of another channel count leaves it to that launch (the
// unit's frame decides before anything is written), so each instantiation
// carries one pixel width only.
template <int C>
__global__ __launch_bounds__(kMaxThreads) void k_plan_labels(TileArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ __align__(16) uint16_t S[(kLabRows + 2) * kLabStride];
    const int f0 = (int)uniform_u32((uint32_t)a.unit_map[2 * (int64_t)blockIdx.x]);
    if (a.frames[f0].C != C)
        return;
    plan_unit(a, lds, [&](const FrameRec& F, int f, int r0, int nb, int c0, int KC, int KCs, uint32_t* cellcnt) {
        plan_count_labels<C>(a, F, static_cast<const uint8_t*>(a.images[f]), r0, nb, c0, KC, KCs, cellcnt, S);
    });
}

// Plan of a call without masks (Algorithm 3 with every cell simple): flags
// cleared, no complex cell in any tile, and each frame's counts and offsets
// copied from the table the host derived from the geometry alone.  One
// launch in place of the count and scan passes.
__global__ __launch_bounds__(256) void k_plan_simple(TileArgs a)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 < kTicketWords)
        a.ticket[i0] = 0u;
    for (int64_t i = i0; i < a.total_cells; i += stride)
        a.flags[i] = 0;
    for (int64_t i = i0; i < a.n_tiles; i += stride) {
        a.tile_cnt[i] = 0u;
        a.tile_fg[i] = 0u;
    }
    for (int64_t i = i0; i < 4 * (int64_t)a.n_frames; i += stride)
        a.counts[i] = a.simple_counts[i];
}

// One workgroup per frame: exclusive scan of the per-tile complex counts into
// each tile's count of complex cells before it, and the frame's simple and
// complex cell counts; k_scan_frames, launched next, turns the per-frame
// counts into store offsets.  (Electing a last workgroup here instead needs
// an agent-scope release in every workgroup, an L2 write-back on gfx950: the
// plan call of the 256-frame batch took 3 us longer that way.)
__global__ __launch_bounds__(256) void k_scan_tiles(TileArgs a)
{
    __shared__ uint32_t wave_tot[9];
    const int f = blockIdx.x;
    const FrameRec F = a.frames[f];
    const int64_t nt = (int64_t)F.GR * F.TX;
    uint32_t carry = 0;
    for (int64_t base = 0; base < nt; base += blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const uint32_t v = i < nt ? a.tile_cnt[F.tile_base + i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan<uint32_t>(v, wave_tot, tot);
        if (i < nt)
            a.tile_fg[F.tile_base + i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        const uint64_t cells = (uint64_t)F.GR * F.GC;
        a.counts[4 * f + 0] = cells - carry;
        a.counts[4 * f + 1] = (uint64_t)carry;
    }
}

__global__ __launch_bounds__(256) void k_scan_frames(TileArgs a)
{
    __shared__ uint64_t wave_tot64[9];
    scan_frames(a, wave_tot64);
}

// The scan without a hand-off between workgroups, for batches whose frames
// share C and n (a frame's store size is then a fixed weight times its
// counts) and whose tile counts are few: frames are concatenated, so the
// complex cells of every earlier frame are one prefix of the tile array,
// which workgroup f adds up itself before scanning its own tiles.
__global__ __launch_bounds__(256) void k_scan_prefix(TileArgs a)
{
    __shared__ uint32_t wave_tot[9];
    const int f = blockIdx.x, tid = threadIdx.x, NT = blockDim.x;
    const FrameRec F = a.frames[f];
    const int64_t t0 = F.tile_base;
    const int64_t nt = (int64_t)F.GR * F.TX;
    // tile counts of the earlier frames: 16 bytes a load, all in flight
    const int64_t n4 = t0 >> 2;
    const v4u* c4 = reinterpret_cast<const v4u*>(a.tile_cnt);
    uint32_t part = tid < (int)(t0 & 3) ? a.tile_cnt[4 * n4 + tid] : 0u;
    for (int64_t base = 0; base < n4; base += 8 * (int64_t)NT) {
        v4u w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t i = base + (int64_t)k * NT + tid;
            w[k] = i < n4 ? c4[i] : v4u{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            part += (w[k].x + w[k].y) + (w[k].z + w[k].w);
    }
    uint32_t before;
    block_exclusive_scan<uint32_t>(part, wave_tot, before);
    uint32_t carry = 0;
    for (int64_t base = 0; base < nt; base += NT) {
        const int64_t i = base + tid;
        const uint32_t v = i < nt ? a.tile_cnt[t0 + i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan<uint32_t>(v, wave_tot, tot);
        if (i < nt)
            a.tile_fg[t0 + i] = carry + ex;
        carry += tot;
    }
    if (tid == 0) {
        const uint64_t nf = carry, nb = (uint64_t)F.GR * (uint64_t)F.GC - nf;
        const uint64_t bb = (uint64_t)F.C * ((uint64_t)F.cell_base - before);
        const uint64_t fb = (uint64_t)F.n * (uint64_t)F.n * (uint64_t)F.C * (uint64_t)before;
        a.counts[4 * f + 0] = nb;
        a.counts[4 * f + 1] = nf;
        a.counts[4 * f + 2] = bb;
        a.counts[4 * f + 3] = fb;
    }
    if (f == 0 && tid < kTicketWords)
        a.ticket[tid] = 0;
}

// Complex cells per tile from the store's flags alone (a store that was
// written elsewhere, e.g. decoded from its serialised form), one lane per
// tile; the scan then rebuilds the tile prefixes and the frame counts and
// offsets.  Workgroup 0 clears the ticket words as k_plan does.
__global__ __launch_bounds__(256) void k_tile_count(TileArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x < kTicketWords)
        a.ticket[threadIdx.x] = 0u;
    if (i >= a.n_tiles)
        return;
    const int f = a.tile_map[2 * i];
    const int64_t local = a.tile_map[2 * i + 1];
    const FrameRec F = a.frames[f];
    const int r = (int)(local / F.TX), ct = (int)(local - (int64_t)r * F.TX);
    const int x0c = ct * F.K, Kt = min(F.K, F.GC - x0c);
    const uint8_t* fl = a.flags + F.cell_base + (int64_t)r * F.GC + x0c;
    uint32_t cnt = 0;
    for (int k = 0; k < Kt; ++k)
        cnt += fl[k] != 0;
    a.tile_cnt[F.tile_base + local] = cnt;
}

// Subgrid rows per phase-1 item: with short subgrid rows an item takes
// several, so that every lane has about eight row loads in flight.
__device__ __forceinline__ int rows_per_item(int s) { return s == 2 ? 4 : ((s == 3 || s == 4) ? 2 : 1); }

// Column sums of up to 8 / S consecutive subgrid rows of S rows each (qq of
// them), one 16-byte strip: every load is issued before the first add.
template <int S>
__device__ __forceinline__ void strip_rows_q(const uint8_t* base, uint32_t off, uint32_t upitch, int qq,
                                             uint16_t* dst, int rowbuf)
{
    constexpr int Q = 8 / S;
    uint32_t e[Q][4], o[Q][4];
#pragma unroll
    for (int j = 0; j < Q; ++j)
#pragma unroll
        for (int d = 0; d < 4; ++d)
            e[j][d] = o[j][d] = 0u;
    v4u w[Q * S];
    if (qq == Q) {
        // every row of the item (the common case): no per-load guards
#pragma unroll
        for (int i = 0; i < Q * S; ++i)
            w[i] = ld16_nt(base + (off + (uint32_t)i * upitch));
#pragma unroll
        for (int i = 0; i < Q * S; ++i)
            acc_bytes(w[i], e[i / S], o[i / S]);
#pragma unroll
        for (int j = 0; j < Q; ++j)
            store_colsums16(dst + j * rowbuf, e[j], o[j]);
        return;
    }
#pragma unroll
    for (int i = 0; i < Q * S; ++i)
        if (i < qq * S)
            w[i] = ld16_nt(base + (off + (uint32_t)i * upitch));
#pragma unroll
    for (int i = 0; i < Q * S; ++i)
        if (i < qq * S)
            acc_bytes(w[i], e[i / S], o[i / S]);
#pragma unroll
    for (int j = 0; j < Q; ++j)
        if (j < qq)
            store_colsums16(dst + j * rowbuf, e[j], o[j]);
}

// Column sums of one subgrid row of s padded rows from row0 on, folded into
// the frame (last band), one strip; loads in batches of 4.
__device__ __forceinline__ void strip_rows_fold(const uint8_t* col, int64_t pitch, int row0, int s, int H, int pad,
                                                uint16_t* dst)
{
    uint32_t e[4] = {0, 0, 0, 0}, o[4] = {0, 0, 0, 0};
    if (pad == kPadNone)   // rows past the frame are absent
        s = max(0, min(s, H - row0));
    int k = 0;
    for (; k + 4 <= s; k += 4) {
        v4u w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            w[i] = ld16_nt(col + (int64_t)fold(row0 + k + i, H, pad) * pitch);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            acc_bytes(w[i], e, o);
    }
    for (; k < s; ++k)
        acc_bytes(ld16_nt(col + (int64_t)fold(row0 + k, H, pad) * pitch), e, o);
    store_colsums16(dst, e, o);
}

// Column sums of one subgrid row of s rows, one strip, loads in batches of 8.
__device__ __forceinline__ void strip_rows_1(const uint8_t* base, uint32_t off, uint32_t upitch, int s, uint16_t* dst)
{
    uint32_t e[4] = {0, 0, 0, 0}, o[4] = {0, 0, 0, 0};
    int k = 0;
    for (; k + 8 <= s; k += 8) {
        v4u w[8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            w[i] = ld16_nt(base + (off + (uint32_t)(k + i) * upitch));
#pragma unroll
        for (int i = 0; i < 8; ++i)
            acc_bytes(w[i], e, o);
    }
    for (; k + 4 <= s; k += 4) {
        v4u w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            w[i] = ld16_nt(base + (off + (uint32_t)(k + i) * upitch));
#pragma unroll
        for (int i = 0; i < 4; ++i)
            acc_bytes(w[i], e, o);
    }
    for (; k < s; ++k)
        acc_bytes(ld16_nt(base + (off + (uint32_t)k * upitch)), e, o);
    store_colsums16(dst, e, o);
}

// One padded row of a band's rounded values, expanded in LDS for the row
// stores: subcell column fc (cell fc / n) covers s_b pixels of C bytes from
// byte fc * s_b * C.  When that span is whole dwords, the pixel's C-byte
// pattern is written a dword at a time (for C = 3 it repeats every three
// dwords): a quarter of the LDS writes of one byte per (pixel, channel), and
// no two lanes write into the same dword.
template <int C>
__device__ __forceinline__ void expand_row_u8(uint8_t* exb, int kn, int n, int s, int fr, const uint8_t* cflag,
                                              const uint8_t* vgs, const uint8_t* vgc)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    if (((s * C) & 3) == 0) {
        const int words = (s * C) >> 2;
        for (int fc = tid; fc < kn; fc += NT) {
            const int kc = fc / n;
            const uint8_t* v = cflag[kc] ? vgc + (fr * kn + fc) * C : vgs + kc * C;
            uint32_t pix = 0;   // the pixel's C bytes, first channel lowest
#pragma unroll
            for (int ch = 0; ch < C; ++ch)
                pix |= (uint32_t)v[ch] << (8 * ch);
            uint32_t* d = reinterpret_cast<uint32_t*>(exb + fc * s * C);
            if (C == 3) {
                const uint32_t d0 = pix | (pix << 24), d1 = (pix >> 8) | (pix << 16), d2 = (pix >> 16) | (pix << 8);
                for (int k = 0; k < words; k += 3) {
                    d[k] = d0;
                    d[k + 1] = d1;
                    d[k + 2] = d2;
                }
            } else {
                const uint32_t w = C == 1 ? pix * 0x01010101u : (C == 2 ? pix | (pix << 16) : pix);
                for (int k = 0; k < words; ++k)
                    d[k] = w;
            }
        }
        return;
    }
    for (int j = tid; j < kn * C; j += NT) {
        const int fc = j / C, ch = j - fc * C;
        const int kc = fc / n;
        const uint8_t v = cflag[kc] ? vgc[(fr * kn + fc) * C + ch] : vgs[kc * C + ch];
        uint8_t* e = exb + fc * s * C + ch;
        for (int x = 0; x < s; ++x)
            e[x * C] = v;
    }
}

// Sums per channel of one subcell's s_b packed 16-bit column sums of one
// subgrid row (s_b pixels of C channels, contiguous in LDS).  For even s_b * C
// the span starts on a dword and is read two columns at a time.
template <int C>
__device__ __forceinline__ void subcell_sums(const uint16_t* cp, int s, uint32_t (&S)[C])
{
#pragma unroll
    for (int ch = 0; ch < C; ++ch)
        S[ch] = 0u;
    if (((s * C) & 1) != 0) {
        for (int x = 0; x < s; ++x)
#pragma unroll
            for (int ch = 0; ch < C; ++ch)
                S[ch] += cp[x * C + ch];
        return;
    }
    const uint32_t* w = reinterpret_cast<const uint32_t*>(cp);
    const int dw = (s * C) >> 1;
    if (C == 3) {
        // two pixels per three dwords: (c0 c1) (c2 c0) (c1 c2)
        for (int k = 0; k < dw; k += 3) {
            const uint32_t w0 = w[k], w1 = w[k + 1], w2 = w[k + 2];
            S[0] += (w0 & 0xFFFFu) + (w1 >> 16);
            S[1 % C] += (w0 >> 16) + (w2 & 0xFFFFu);
            S[2 % C] += (w1 & 0xFFFFu) + (w2 >> 16);
        }
    } else if (C == 1) {
        for (int k = 0; k < dw; ++k)
            S[0] += (w[k] & 0xFFFFu) + (w[k] >> 16);
    } else if (C == 2) {
        for (int k = 0; k < dw; ++k) {
            S[0] += w[k] & 0xFFFFu;
            S[1 % C] += w[k] >> 16;
        }
    } else {
        // C = 4: one pixel per two dwords, (c0 c1) (c2 c3)
        for (int k = 0; k < dw; k += 2) {
            S[0] += w[k] & 0xFFFFu;
            S[1 % C] += w[k] >> 16;
            S[2 % C] += w[k + 1] & 0xFFFFu;
            S[3 % C] += w[k + 1] >> 16;
        }
    }
}

// Phase 2a of the u8 forward for even s_b: one lane per subcell column
// adds, for every subgrid row of the group, the subcell's s_b * C packed
// 16-bit column sums (contiguous in LDS: s_b pixels of C channels) read two
// at a time as dwords, into one sum per channel, and keeps the running sums
// over subgrid rows in cspart[fc * C + ch].  (Per-(column, channel) lanes
// would read each 16-bit sum on its own, C lanes into the same dwords.)
// dbg: optional exact subcell sums, row-major over the fine grid from
// dbg_base (first subgrid row of the group, first subcell column of the
// tile), dbg_row fine cells per row.
template <int C>
__device__ __forceinline__ void subcell_sums_pairs(const uint16_t* col16, int rowbuf, int kn, int s, int ng, int fr0,
                                                   uint32_t* cspart, uint32_t* dbg, int64_t dbg_base, int64_t dbg_row)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    for (int fc = tid; fc < kn; fc += NT) {
        uint32_t tot[C];
#pragma unroll
        for (int ch = 0; ch < C; ++ch)
            tot[ch] = fr0 == 0 ? 0u : cspart[fc * C + ch];
        for (int g = 0; g < ng; ++g) {
            uint32_t S[C];
            subcell_sums<C>(col16 + g * rowbuf + fc * s * C, s, S);
#pragma unroll
            for (int ch = 0; ch < C; ++ch) {
                tot[ch] += S[ch];
                if (dbg)
                    dbg[(dbg_base + (int64_t)g * dbg_row + fc) * C + ch] = S[ch];
            }
        }
#pragma unroll
        for (int ch = 0; ch < C; ++ch)
            cspart[fc * C + ch] = tot[ch];
    }
}

// ==========================================================================
// Forward, uint8 HWC (Algorithm 3 steps 7-19, fused steps 11, 18-21).
// ==========================================================================
// DBG: also write the exact sums of every cell and subcell (dp_pix_debug_sums);
// a separate instantiation, so the release kernel carries none of that state.
template <int C, bool DBG>
__device__ void forward_tile_u8(const TileArgs& a, const FrameRec& F, const TileCoord& tc, uint8_t* lds)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    const int b = F.b, s = F.s, n = F.n, H = F.H, W = F.W, pad = F.pad;
    const int r = tc.r;
    const int x0c = tc.ct * F.K;
    const int Kt = min(F.K, F.GC - x0c);
    const int WB = Kt * b * C;
    const int nstr = (WB + 15) >> 4;
    const int64_t X0 = (int64_t)x0c * b * C;
    const int64_t tile_end = X0 + WB;
    const int64_t real_end = (int64_t)W * C;
    const int64_t lim = min(tile_end, real_end);
    const int64_t pitch = F.pitch;
    const uint8_t* img = static_cast<const uint8_t*>(a.images[tc.f]);
    uint8_t* out = a.outs ? static_cast<uint8_t*>(a.outs[tc.f]) : nullptr;
    const bool in_aligned = ((reinterpret_cast<uintptr_t>(img) | (uintptr_t)pitch | (uintptr_t)X0) & 15) == 0;
    // bands without vertical padding address rows by 32-bit offsets from the
    // band's first byte of the tile (uniform base, one offset register)
    const bool band_inside = F.off32 && (r + 1) * b <= H;
    const uint32_t upitch = (uint32_t)pitch;
    const uint8_t* band_in = img + (int64_t)r * b * pitch + X0;

    const LdsPlan L = lds_plan(kFwdU8, F.K, b, n, C);
    uint16_t* col16 = reinterpret_cast<uint16_t*>(lds + L.colsum);
    uint8_t* ex = lds + L.colsum;
    uint32_t* cspart = reinterpret_cast<uint32_t*>(lds + L.cspart);
    uint32_t* cidx = reinterpret_cast<uint32_t*>(lds + L.cidx);
    uint8_t* cflag = lds + L.cflag;
    uint8_t* vgs = lds + L.vgs;
    uint8_t* vgc = lds + L.vgc;
    uint16_t* cxl = reinterpret_cast<uint16_t*>(lds + L.cxl);
    __shared__ uint32_t s_ncx;

    tile_cells(a, F, tc.t, r, x0c, Kt, cidx, cflag, cxl, &s_ncx);
    const uint64_t bg_base = a.counts[4 * tc.f + 2];
    const uint64_t fg_base = a.counts[4 * tc.f + 3];
    const int items = Kt * n * C;
    const int nn = n * n;
    const int rowbuf = 16 * nstr;           // 16-bit column sums of one subgrid row
    const double area_s = (double)s * (double)s, inv_s = exact_inv_area(F, s);

    // ---- subgrid rows, up to kRowGroup at a time: each lane streams its strip
    // down all rows of the group (exact 16-bit column sums per subgrid row,
    // one LDS buffer each), then one lane per (subcell column, channel) adds
    // s_b columns per subgrid row and releases complex subcells ----
    for (int fr0 = 0; fr0 < n; fr0 += kRowGroup) {
        const int ng = min(kRowGroup, n - fr0);
        // Whole-vector strips ([0, nfast)): one item per (q subgrid rows,
        // strip); consecutive lanes read consecutive strips of a row and all
        // q * s_b rows of an item (8 or fewer) are loaded before they are
        // added.  Other strips (right edge, misaligned rows): one padded row
        // per item, added into the column sums with LDS atomics so that their
        // latencies overlap.
        const int nfast = in_aligned ? (int)min((int64_t)nstr, (lim - X0) >> 4) : 0;
        const int nslow = nstr - nfast;
        if (nslow > 0) {
            uint32_t* c32 = reinterpret_cast<uint32_t*>(col16);
            for (int i = tid; i < ng * nslow * 8; i += NT) {
                const int g = i / (nslow * 8);
                c32[(g * rowbuf + 16 * nfast) / 2 + (i - g * nslow * 8)] = 0u;
            }
            lds_barrier();
        }
        const int q = band_inside ? rows_per_item(s) : 1;
        const int ngq = (ng + q - 1) / q;
        for (int it = tid; it < nfast * ngq; it += NT) {
            const int gq = it / nfast;
            const int st = it - gq * nfast;
            const int g0 = gq * q;
            const int qq = min(q, ng - g0);
            uint16_t* dst = col16 + g0 * rowbuf + 16 * st;
            if (!band_inside) {
                // last band: padded rows fold back into the frame
                strip_rows_fold(img + X0 + 16 * st, pitch, r * b + (fr0 + g0) * s, s, H, pad, dst);
                continue;
            }
            // rows inside the frame: 32-bit offsets from the band's first row
            const uint32_t off = (uint32_t)((fr0 + g0) * s) * upitch + 16u * (uint32_t)st;
            switch (q) {
            case 4: strip_rows_q<2>(band_in, off, upitch, qq, dst, rowbuf); break;
            case 2:
                if (s == 4)
                    strip_rows_q<4>(band_in, off, upitch, qq, dst, rowbuf);
                else
                    strip_rows_q<3>(band_in, off, upitch, qq, dst, rowbuf);
                break;
            default: strip_rows_1(band_in, off, upitch, s, dst); break;
            }
        }
        for (int it = tid; it < nslow * ng * s; it += NT) {
            const int st = nfast + it % nslow;
            const int rest = it / nslow;
            const int k = rest % s, g = rest / s;
            const int64_t p0 = X0 + 16 * st;
            if (r * b + (fr0 + g) * s + k >= H && pad == kPadNone)
                continue;
            const uint8_t* rp = img + (int64_t)fold(r * b + (fr0 + g) * s + k, H, pad) * pitch;
            const v4u v = (in_aligned && p0 + 16 <= lim) ? ld16_nt(rp + p0)
                                                         : gather_strip_u8<C>(rp, (int)p0, (int)tile_end, W, pad);
            // column pairs (2m, 2m+1) packed as in store_colsums16; a 16-bit
            // half holds at most 255 * 256, so no carry crosses into the other
            uint32_t* cw = reinterpret_cast<uint32_t*>(col16 + g * rowbuf + 16 * st);
            atomicAdd(cw + 0, (v.x & 0xFFu) | ((v.x & 0xFF00u) << 8));
            atomicAdd(cw + 1, ((v.x >> 16) & 0xFFu) | ((v.x >> 24) << 16));
            atomicAdd(cw + 2, (v.y & 0xFFu) | ((v.y & 0xFF00u) << 8));
            atomicAdd(cw + 3, ((v.y >> 16) & 0xFFu) | ((v.y >> 24) << 16));
            atomicAdd(cw + 4, (v.z & 0xFFu) | ((v.z & 0xFF00u) << 8));
            atomicAdd(cw + 5, ((v.z >> 16) & 0xFFu) | ((v.z >> 24) << 16));
            atomicAdd(cw + 6, (v.w & 0xFFu) | ((v.w & 0xFF00u) << 8));
            atomicAdd(cw + 7, ((v.w >> 16) & 0xFFu) | ((v.w >> 24) << 16));
        }
        // classes and store indices of the tile's cells (wave 0), read while
        // the row loads above are still in flight
        lds_barrier();
        // running sums of every (subcell column, channel) for the coarse cells
        if ((s & 1) == 0) {
            subcell_sums_pairs<C>(col16, rowbuf, Kt * n, s, ng, fr0, cspart, DBG ? a.dbg_fine : nullptr,
                                  F.fine_base + (int64_t)(r * n + fr0) * ((int64_t)F.GC * n) + (int64_t)x0c * n,
                                  (int64_t)F.GC * n);
        } else {
            for (int j = tid; j < items; j += NT) {
                const int fc = j / C, ch = j - fc * C;
                uint32_t total = fr0 == 0 ? 0u : cspart[j];
                for (int g = 0; g < ng; ++g) {
                    const uint16_t* cp = col16 + g * rowbuf + fc * s * C + ch;
                    uint32_t S = 0;
                    for (int x = 0; x < s; ++x)
                        S += cp[x * C];
                    total += S;
                    if (DBG && a.dbg_fine)
                        a.dbg_fine[(F.fine_base + (int64_t)(r * n + fr0 + g) * ((int64_t)F.GC * n) +
                                    (int64_t)x0c * n + fc) * C + ch] = S;
                }
                cspart[j] = total;
            }
        }
        // releases of the complex cells' subcells, spread evenly over the
        // lanes (only complex cells draw noise, so a lane-per-subcell loop
        // would leave the lanes of simple cells idle): one item per (complex
        // cell, subgrid row, subcell column) re-reads the subcell's column
        // sums and releases its C channels
        const int ncx = (int)s_ncx;
        const int per_cx = ng * n;
        for (int it = tid; it < ncx * per_cx; it += NT) {
            const int q = it / per_cx;
            const int rem = it - q * per_cx;
            const int g = rem / n, jj = rem - g * n;
            const int kc = cxl[q];
            const int fc = kc * n + jj, fr = fr0 + g;
            uint32_t S[C];
            subcell_sums<C>(col16 + g * rowbuf + fc * s * C, s, S);
            const uint32_t id = (uint32_t)(r * n + fr) * (uint32_t)(F.GC * n) + (uint32_t)(x0c * n + fc);
            const double area = pad == kPadNone ? stat_area(F, r * b + fr * s, x0c * b + fc * s, s) : area_s;
            const uint64_t at = fg_base + ((uint64_t)cidx[kc] * nn + fr * n + jj) * C;
            uint8_t* vd = vgc + (fr * Kt * n + fc) * C;
            // one channel at a time (unrolled, the C draws would be live at once)
#pragma unroll 1
            for (int ch = 0; ch < C; ++ch) {
                uint32_t Sc = S[0];
#pragma unroll
                for (int k = 1; k < C; ++k)
                    Sc = ch == k ? S[k] : Sc;
                uint8_t pass;
                const float v = release((double)Sc, area, inv_s, F.noise_fg, F.sigma_fg, F, id, ch, 1, pass);
                a.fg[at + ch] = v;
                if (a.clip_fg)
                    a.clip_fg[at + ch] = pass;
                vd[ch] = to_u8(v);
            }
        }
        lds_barrier();
    }

    // ---- simple cells: coarse sum = total of the n*n subcell sums ----
    for (int j = tid; j < Kt * C; j += NT) {
        const int kc = j / C, ch = j - kc * C;
        uint32_t S = 0;
        for (int jj = 0; jj < n; ++jj)
            S += cspart[(kc * n + jj) * C + ch];
        if (DBG && a.dbg_coarse)
            a.dbg_coarse[(F.cell_base + (int64_t)r * F.GC + x0c + kc) * C + ch] = S;
        if (!cflag[kc]) {
            const uint32_t id = (uint32_t)(r * F.GC + x0c + kc);
            uint8_t pass;
            const float v = release((double)S, stat_area(F, r * b, (x0c + kc) * b, b), exact_inv_area(F, b),
                                    F.noise_bg, F.sigma_bg, F, id, ch, 0, pass);
            const uint64_t at = bg_base + (uint64_t)cidx[kc] * C + ch;
            a.bg[at] = v;
            if (a.clip_bg)
                a.clip_bg[at] = pass;
            vgs[kc * C + ch] = to_u8(v);
        }
    }
    if (out == nullptr)
        return;
    lds_barrier();

    // ---- fused reconstruction of the band's real pixels ----
    // The expanded row alternates between two LDS buffers, so one barrier per
    // subgrid row suffices: a buffer is rewritten two rows later, after every
    // lane has passed the barrier that follows its last read.
    const bool out_aligned = ((reinterpret_cast<uintptr_t>(out) | (uintptr_t)pitch | (uintptr_t)X0) & 15) == 0;
    uint8_t* band_out = out + (int64_t)r * b * pitch + X0;
    for (int fr = 0; fr < n; ++fr) {
        uint8_t* exb = ex + (fr & 1) * (16 * nstr);
        expand_row_u8<C>(exb, Kt * n, n, s, fr, cflag, vgs, vgc);
        lds_barrier();
        const int row0 = r * b + fr * s;
        const int rows = min(s, H - row0);
        // items (row part, strip): the s_b rows of a strip are split over
        // `parts` lanes when the tile has fewer strips than lanes
        const int parts = max(1, min(rows, NT / nstr));
        const int per = (rows + parts - 1) / max(parts, 1);
        for (int it = tid; it < nstr * parts; it += NT) {
            const int part = it / nstr;
            const int st = it - part * nstr;
            const int64_t p0 = X0 + 16 * st;
            const int k0 = part * per, k1 = min(rows, k0 + per);
            if (p0 >= lim)
                continue;
            const v4u v = *reinterpret_cast<const v4u*>(exb + 16 * st);
            if (out_aligned && p0 + 16 <= lim) {
                if (F.off32) {
                    const uint32_t off = (uint32_t)(fr * s) * upitch + 16u * (uint32_t)st;
                    for (int k = k0; k < k1; ++k)
                        st16_nt(band_out + (off + (uint32_t)k * upitch), v);
                } else {
                    for (int k = k0; k < k1; ++k)
                        st16_nt(out + (int64_t)(row0 + k) * pitch + p0, v);
                }
            } else {
                const uint8_t* vb = exb + 16 * st;
                for (int k = k0; k < k1; ++k) {
                    g_u8w* op = (g_u8w*)(out + (int64_t)(row0 + k) * pitch);
                    for (int q = 0; q < 16 && p0 + q < lim; ++q)
                        op[p0 + q] = vb[q];
                }
            }
        }
    }
}

// ==========================================================================
// Forward, fp32 CHW.  Column sums in fp32 over at most s_b rows, subcell and
// cell sums in fp64.
// ==========================================================================
// Broadcast of a tile's statistics to its real pixels, fp32 CHW: per
// (channel, subgrid row) one padded row is expanded in LDS (two alternating
// buffers of 4 * nstr floats at `rowbuf`, one barrier per row) and each lane
// stores the s_b rows of one 4-float strip.  vgs / vgc hold the values of the
// simple cells and of the complex subcells (as the fp32 forward lays them out).
__device__ void broadcast_tile_f32(const FrameRec& F, int r, int64_t X0, int64_t lim, int Kt, int nstr,
                                   float* rowbuf, const uint8_t* cflag, const float* vgs, const float* vgc,
                                   float* out)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    const int b = F.b, s = F.s, n = F.n, H = F.H, C = F.C;
    const int kn = Kt * n;
    const int64_t pitch = F.pitch, plane = pitch * H;
    const bool out_aligned = ((reinterpret_cast<uintptr_t>(out) | (uintptr_t)(pitch * 4) | (uintptr_t)(X0 * 4)) & 15) == 0;
    for (int ch = 0; ch < C; ++ch) {
        float* pl = out + plane * ch;
        for (int fr = 0; fr < n; ++fr) {
            float* exf = rowbuf + ((ch * n + fr) & 1) * (4 * nstr);   // two alternating row buffers
            for (int fc = tid; fc < kn; fc += NT) {
                const int kc = fc / n;
                const float v = cflag[kc] ? vgc[(fr * kn + fc) * C + ch] : vgs[kc * C + ch];
                for (int x = 0; x < s; ++x)
                    exf[fc * s + x] = v;
            }
            lds_barrier();
            const int row0 = r * b + fr * s;
            const int rows = min(s, H - row0);
            for (int st = tid; st < nstr; st += NT) {
                const int64_t p0 = X0 + 4 * st;
                if (p0 >= lim)
                    continue;
                const v4f v = reinterpret_cast<const v4f*>(exf)[st];
                if (out_aligned && p0 + 4 <= lim) {
                    for (int k = 0; k < rows; ++k)
                        st16f_nt(pl + (int64_t)(row0 + k) * pitch + p0, v);
                } else {
                    const float vv[4] = {v.x, v.y, v.z, v.w};
                    g_f32w* pg = (g_f32w*)pl;
                    for (int k = 0; k < rows; ++k)
                        for (int q = 0; q < 4 && p0 + q < lim; ++q)
                            pg[(int64_t)(row0 + k) * pitch + p0 + q] = vv[q];
                }
            }
        }
    }
}

__device__ void forward_tile_f32(const TileArgs& a, const FrameRec& F, const TileCoord& tc, uint8_t* lds)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    const int b = F.b, s = F.s, n = F.n, H = F.H, W = F.W, C = F.C, pad = F.pad;
    const int r = tc.r;
    const int x0c = tc.ct * F.K;
    const int Kt = min(F.K, F.GC - x0c);
    const int WB = Kt * b;                 // floats
    const int nstr = (WB + 3) >> 2;
    const int64_t X0 = (int64_t)x0c * b;
    const int64_t tile_end = X0 + WB;
    const int64_t lim = min(tile_end, (int64_t)W);
    const int64_t pitch = F.pitch;
    const int64_t plane = pitch * H;
    const float* img = static_cast<const float*>(a.images[tc.f]);
    float* out = a.outs ? static_cast<float*>(a.outs[tc.f]) : nullptr;
    const bool in_aligned = ((reinterpret_cast<uintptr_t>(img) | (uintptr_t)(pitch * 4) | (uintptr_t)(X0 * 4)) & 15) == 0;

    const double inv_s = exact_inv_area(F, s), inv_b = exact_inv_area(F, b);
    const LdsPlan L = lds_plan(kFwdF32, F.K, b, n, C);
    float* colsum = reinterpret_cast<float*>(lds + L.colsum);
    double* cspart = reinterpret_cast<double*>(lds + L.cspart);
    uint32_t* cidx = reinterpret_cast<uint32_t*>(lds + L.cidx);
    uint8_t* cflag = lds + L.cflag;
    float* vgs = reinterpret_cast<float*>(lds + L.vgs);
    float* vgc = reinterpret_cast<float*>(lds + L.vgc);

    tile_cells(a, F, tc.t, r, x0c, Kt, cidx, cflag);
    const uint64_t bg_base = a.counts[4 * tc.f + 2];
    const uint64_t fg_base = a.counts[4 * tc.f + 3];
    const int nn = n * n;
    const int kn = Kt * n;
    lds_barrier();

    // Subgrid rows in groups of kRowGroupF: one item per (channel, subgrid
    // row, 4-float strip), consecutive lanes on consecutive strips of a row,
    // rows added in order (fp32) with up to four loads in flight; then one
    // lane per (channel, subcell column) adds the s_b column sums (fp64) per
    // subgrid row and releases the complex subcells.
    const int kn4 = 4 * nstr;                 // floats of one row buffer
    for (int fr0 = 0; fr0 < n; fr0 += kRowGroupF) {
        const int ng = min(kRowGroupF, n - fr0);
        for (int it = tid; it < C * ng * nstr; it += NT) {
            const int st = it % nstr;
            const int rest = it / nstr;
            const int g = rest % ng, ch = rest / ng;
            const float* pl = img + plane * ch;
            const int row0 = r * b + (fr0 + g) * s;
            const int64_t p0 = X0 + 4 * st;
            // rows past the frame are absent in the unpadded mode
            const int srows = pad == kPadNone ? max(0, min(s, H - row0)) : s;
            const int64_t cend = pad == kPadNone ? lim : tile_end;
            v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
            if (in_aligned && p0 + 4 <= lim) {
                int k = 0;
                for (; k + 4 <= srows; k += 4) {
                    v4f w[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        w[i] = ld16f_nt(pl + (int64_t)fold(row0 + k + i, H, pad) * pitch + p0);
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        acc += w[i];
                }
                for (; k < srows; ++k)
                    acc += ld16f_nt(pl + (int64_t)fold(row0 + k, H, pad) * pitch + p0);
            } else {
                for (int k = 0; k < srows; ++k) {
                    const g_f32* rk = (const g_f32*)(pl + (int64_t)fold(row0 + k, H, pad) * pitch);
                    float v[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        v[q] = (p0 + q < cend) ? rk[fold((int)(p0 + q), W, pad)] : 0.f;
                    acc.x += v[0]; acc.y += v[1]; acc.z += v[2]; acc.w += v[3];
                }
            }
            reinterpret_cast<v4f*>(colsum)[(ch * ng + g) * nstr + st] = acc;
        }
        lds_barrier();
        for (int j = tid; j < C * kn; j += NT) {
            const int ch = j / kn, fc = j - ch * kn;
            const int kc = fc / n, jj = fc - kc * n;
            const int ci = fc * C + ch;
            double part = fr0 == 0 ? 0.0 : cspart[ci];
            for (int g = 0; g < ng; ++g) {
                const float* cs = colsum + (ch * ng + g) * kn4 + fc * s;
                double S = 0.0;
                for (int x = 0; x < s; ++x)
                    S += (double)cs[x];
                part += S;
                if (cflag[kc]) {
                    const int fr = fr0 + g;
                    const int row0 = r * b + fr * s;
                    const uint32_t id = (uint32_t)(r * n + fr) * (uint32_t)(F.GC * n) + (uint32_t)(x0c * n + fc);
                    uint8_t pass;
                    const float v = release(S, stat_area(F, row0, x0c * b + fc * s, s), inv_s, F.noise_fg,
                                            F.sigma_fg, F, id, ch, 1, pass);
                    const uint64_t at = fg_base + ((uint64_t)cidx[kc] * nn + fr * n + jj) * C + ch;
                    a.fg[at] = v;
                    if (a.clip_fg)
                        a.clip_fg[at] = pass;
                    vgc[(fr * kn + fc) * C + ch] = v;
                }
            }
            cspart[ci] = part;
        }
        lds_barrier();
    }
    for (int j = tid; j < Kt * C; j += NT) {
        const int kc = j / C, ch = j - kc * C;
        if (cflag[kc])
            continue;
        double S = 0.0;
        for (int jj = 0; jj < n; ++jj)
            S += cspart[(kc * n + jj) * C + ch];
        const uint32_t id = (uint32_t)(r * F.GC + x0c + kc);
        uint8_t pass;
        const float v = release(S, stat_area(F, r * b, (x0c + kc) * b, b), inv_b, F.noise_bg, F.sigma_bg, F, id,
                                ch, 0, pass);
        const uint64_t at = bg_base + (uint64_t)cidx[kc] * C + ch;
        a.bg[at] = v;
        if (a.clip_bg)
            a.clip_bg[at] = pass;
        vgs[kc * C + ch] = v;
    }
    if (out == nullptr)
        return;
    lds_barrier();
    broadcast_tile_f32(F, r, X0, lim, Kt, nstr, colsum, cflag, vgs, vgc, out);
}

// Persistent workgroups take tiles from an atomic ticket; the last one out
// resets the ticket for the next launch (no memset, so graphs can replay).
// Each launch covers one group of frames sharing layout and channel count
// (scheduling indices [sched_offset, sched_offset + n_tiles)), so every kernel
// instantiation carries only its own path.
// The tile of this workgroup, for kernels that are never launched as a
// resident grid (the persistent branch would only hold scalar registers).
template <typename Body>
__device__ __forceinline__ void run_one_tile(const TileArgs& a, Body body)
{
    FrameRec F;
    const TileCoord tc = tile_of(a, blockIdx.x, F);
    body(F, tc);
}

template <typename Body>
__device__ __forceinline__ void run_tiles(const TileArgs& a, uint8_t* lds, Body body)
{
    if (!a.persistent) {
        FrameRec F;
        const TileCoord tc = tile_of(a, blockIdx.x, F);
        body(F, tc);
        return;
    }
    __shared__ int64_t s_next;
    for (;;) {
        if (threadIdx.x == 0)
            s_next = (int64_t)atomicAdd(&a.ticket[0], 1u);
        lds_barrier();
        const int64_t idx = s_next;
        if (idx >= a.n_tiles)
            break;
        FrameRec F;
        const TileCoord tc = tile_of(a, idx, F);
        body(F, tc);
        lds_barrier();
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t done = atomicAdd(&a.ticket[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&a.ticket[0], 0u);
            atomicExch(&a.ticket[1], 0u);
        }
    }
}

// Five waves per SIMD: enough resident tiles per CU to keep HBM busy while
// other waves are in their LDS phases (the register budget still fits).
template <int C, bool DBG = false>
__global__ __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(DPPIX_FWD_WAVES_PER_EU))) void
k_forward_u8(TileArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    run_tiles(a, lds, [&](const FrameRec& F, const TileCoord& tc) { forward_tile_u8<C, DBG>(a, F, tc, lds); });
}

__global__ __launch_bounds__(kMaxThreads) void k_forward_f32(TileArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    run_tiles(a, lds, [&](const FrameRec& F, const TileCoord& tc) { forward_tile_f32(a, F, tc, lds); });
}

// ==========================================================================
// Reconstruction from the compact store (Sec. VI-F).
// ==========================================================================
template <int C>
__device__ void reconstruct_tile_u8(const TileArgs& a, const FrameRec& F, const TileCoord& tc, uint8_t* lds)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    const int b = F.b, s = F.s, n = F.n, H = F.H, W = F.W;
    const int r = tc.r;
    const int x0c = tc.ct * F.K;
    const int Kt = min(F.K, F.GC - x0c);
    const int WB = Kt * b * C;
    const int nstr = (WB + 15) >> 4;
    const int64_t X0 = (int64_t)x0c * b * C;
    const int64_t lim = min(X0 + WB, (int64_t)W * C);
    const int64_t pitch = F.pitch;
    uint8_t* out = static_cast<uint8_t*>(a.outs[tc.f]);
    const LdsPlan L = lds_plan(kRecU8, F.K, b, n, C);
    uint8_t* ex = lds + L.colsum;
    uint32_t* cidx = reinterpret_cast<uint32_t*>(lds + L.cidx);
    uint8_t* cflag = lds + L.cflag;
    uint8_t* vgs = lds + L.vgs;
    uint8_t* vgc = lds + L.vgc;
    tile_cells(a, F, tc.t, r, x0c, Kt, cidx, cflag);
    const uint64_t bg_base = a.counts[4 * tc.f + 2];
    const uint64_t fg_base = a.counts[4 * tc.f + 3];
    const int nn = n * n, kn = Kt * n;
    lds_barrier();
    for (int j = tid; j < Kt * C; j += NT) {
        const int kc = j / C, ch = j - kc * C;
        if (!cflag[kc])
            vgs[j] = to_u8(a.bg[bg_base + (uint64_t)cidx[kc] * C + ch]);
    }
    for (int j = tid; j < Kt * nn * C; j += NT) {
        // j = ((fr * kn) + fc) * C + ch
        const int ch = j % C;
        const int q = j / C;
        const int fr = q / kn, fc = q - fr * kn;
        const int kc = fc / n, jj = fc - kc * n;
        if (cflag[kc])
            vgc[j] = to_u8(a.fg[fg_base + ((uint64_t)cidx[kc] * nn + fr * n + jj) * C + ch]);
    }
    lds_barrier();
    const bool out_aligned = ((reinterpret_cast<uintptr_t>(out) | (uintptr_t)pitch | (uintptr_t)X0) & 15) == 0;
    const uint32_t upitch = (uint32_t)pitch;
    uint8_t* band_out = out + (int64_t)r * b * pitch + X0;
    for (int fr = 0; fr < n; ++fr) {
        uint8_t* exb = ex + (fr & 1) * (16 * nstr);   // two alternating row buffers
        expand_row_u8<C>(exb, kn, n, s, fr, cflag, vgs, vgc);
        lds_barrier();
        const int row0 = r * b + fr * s;
        const int rows = min(s, H - row0);
        // items (row part, strip): the s_b rows of a strip are split over
        // `parts` lanes when the tile has fewer strips than lanes
        const int parts = max(1, min(rows, NT / nstr));
        const int per = (rows + parts - 1) / max(parts, 1);
        for (int it = tid; it < nstr * parts; it += NT) {
            const int part = it / nstr;
            const int st = it - part * nstr;
            const int64_t p0 = X0 + 16 * st;
            const int k0 = part * per, k1 = min(rows, k0 + per);
            if (p0 >= lim)
                continue;
            const v4u v = *reinterpret_cast<const v4u*>(exb + 16 * st);
            if (out_aligned && p0 + 16 <= lim) {
                if (F.off32) {
                    const uint32_t off = (uint32_t)(fr * s) * upitch + 16u * (uint32_t)st;
                    for (int k = k0; k < k1; ++k)
                        st16_nt(band_out + (off + (uint32_t)k * upitch), v);
                } else {
                    for (int k = k0; k < k1; ++k)
                        st16_nt(out + (int64_t)(row0 + k) * pitch + p0, v);
                }
            } else {
                const uint8_t* vb = exb + 16 * st;
                for (int k = k0; k < k1; ++k) {
                    g_u8w* op = (g_u8w*)(out + (int64_t)(row0 + k) * pitch);
                    for (int q = 0; q < 16 && p0 + q < lim; ++q)
                        op[p0 + q] = vb[q];
                }
            }
        }
    }
}

__device__ void reconstruct_tile_f32(const TileArgs& a, const FrameRec& F, const TileCoord& tc, uint8_t* lds)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    const int b = F.b, s = F.s, n = F.n, H = F.H, W = F.W, C = F.C;
    const int r = tc.r;
    const int x0c = tc.ct * F.K;
    const int Kt = min(F.K, F.GC - x0c);
    const int WB = Kt * b;
    const int nstr = (WB + 3) >> 2;
    const int64_t X0 = (int64_t)x0c * b;
    const int64_t lim = min(X0 + WB, (int64_t)W);
    const int64_t pitch = F.pitch, plane = pitch * H;
    float* out = static_cast<float*>(a.outs[tc.f]);
    const LdsPlan L = lds_plan(kRecF32, F.K, b, n, C);
    float* exbase = reinterpret_cast<float*>(lds + L.colsum);
    uint32_t* cidx = reinterpret_cast<uint32_t*>(lds + L.cidx);
    uint8_t* cflag = lds + L.cflag;
    float* vgs = reinterpret_cast<float*>(lds + L.vgs);
    float* vgc = reinterpret_cast<float*>(lds + L.vgc);
    tile_cells(a, F, tc.t, r, x0c, Kt, cidx, cflag);
    const uint64_t bg_base = a.counts[4 * tc.f + 2];
    const uint64_t fg_base = a.counts[4 * tc.f + 3];
    const int nn = n * n, kn = Kt * n;
    lds_barrier();
    for (int j = tid; j < Kt * C; j += NT) {
        const int kc = j / C, ch = j - kc * C;
        if (!cflag[kc])
            vgs[j] = a.bg[bg_base + (uint64_t)cidx[kc] * C + ch];
    }
    for (int j = tid; j < Kt * nn * C; j += NT) {
        const int ch = j % C;
        const int q = j / C;
        const int fr = q / kn, fc = q - fr * kn;
        const int kc = fc / n, jj = fc - kc * n;
        if (cflag[kc])
            vgc[j] = a.fg[fg_base + ((uint64_t)cidx[kc] * nn + fr * n + jj) * C + ch];
    }
    lds_barrier();
    const bool out_aligned = ((reinterpret_cast<uintptr_t>(out) | (uintptr_t)(pitch * 4) | (uintptr_t)(X0 * 4)) & 15) == 0;
    for (int ch = 0; ch < C; ++ch) {
        float* pl = out + plane * ch;
        for (int fr = 0; fr < n; ++fr) {
            float* exf = exbase + ((ch * n + fr) & 1) * (4 * nstr);   // two alternating row buffers
            for (int fc = tid; fc < kn; fc += NT) {
                const int kc = fc / n;
                const float v = cflag[kc] ? vgc[(fr * kn + fc) * C + ch] : vgs[kc * C + ch];
                for (int x = 0; x < s; ++x)
                    exf[fc * s + x] = v;
            }
            lds_barrier();
            const int row0 = r * b + fr * s;
            const int rows = min(s, H - row0);
            for (int st = tid; st < nstr; st += NT) {
                const int64_t p0 = X0 + 4 * st;
                if (p0 >= lim)
                    continue;
                const v4f v = reinterpret_cast<const v4f*>(exf)[st];
                if (out_aligned && p0 + 4 <= lim) {
                    for (int k = 0; k < rows; ++k)
                        st16f_nt(pl + (int64_t)(row0 + k) * pitch + p0, v);
                } else {
                    const float vv[4] = {v.x, v.y, v.z, v.w};
                    g_f32w* pg = (g_f32w*)pl;
                    for (int k = 0; k < rows; ++k)
                        for (int q = 0; q < 4 && p0 + q < lim; ++q)
                            pg[(int64_t)(row0 + k) * pitch + p0 + q] = vv[q];
                }
            }
        }
    }
}

template <int C>
__global__ __launch_bounds__(kMaxThreads) void k_reconstruct_u8(TileArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    run_tiles(a, lds, [&](const FrameRec& F, const TileCoord& tc) { reconstruct_tile_u8<C>(a, F, tc, lds); });
}

__global__ __launch_bounds__(kMaxThreads) void k_reconstruct_f32(TileArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    run_tiles(a, lds, [&](const FrameRec& F, const TileCoord& tc) { reconstruct_tile_f32(a, F, tc, lds); });
}

// ==========================================================================
// Adjoint (fp32 CHW).  Per tile: G_k = sum of grad_out over the real pixels
// of statistic k, g_k = pass_k * G_k / area_k (kept in the gradient store for
// the mirror terms), and every real pixel of the tile takes its own g_k.
// Then, only where padding folds onto real pixels: add the g of every padded
// position that folds onto the pixel.
// ==========================================================================
__device__ void backward_reduce_tile(const TileArgs& a, const FrameRec& F, const TileCoord& tc, uint8_t* lds)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    const int b = F.b, s = F.s, n = F.n, H = F.H, W = F.W, C = F.C;
    const int r = tc.r;
    const int x0c = tc.ct * F.K;
    const int Kt = min(F.K, F.GC - x0c);
    const int WB = Kt * b;
    const int nstr = (WB + 3) >> 2;
    const int64_t X0 = (int64_t)x0c * b;
    const int64_t lim = min(X0 + WB, (int64_t)W);
    const int64_t pitch = F.pitch, plane = pitch * H;
    const float* go = a.grad_out[tc.f];
    const bool aligned = ((reinterpret_cast<uintptr_t>(go) | (uintptr_t)(pitch * 4) | (uintptr_t)(X0 * 4)) & 15) == 0;
    const LdsPlan L = lds_plan(kBwd, F.K, b, n, C);
    float* colsum = reinterpret_cast<float*>(lds + L.colsum);
    double* cspart = reinterpret_cast<double*>(lds + L.cspart);
    uint32_t* cidx = reinterpret_cast<uint32_t*>(lds + L.cidx);
    uint8_t* cflag = lds + L.cflag;
    float* vgs = reinterpret_cast<float*>(lds + L.vgs);
    float* vgc = reinterpret_cast<float*>(lds + L.vgc);
    float* gin = a.grad_in ? a.grad_in[tc.f] : nullptr;
    tile_cells(a, F, tc.t, r, x0c, Kt, cidx, cflag);
    const uint64_t bg_base = a.counts[4 * tc.f + 2];
    const uint64_t fg_base = a.counts[4 * tc.f + 3];
    const int nn = n * n, kn = Kt * n;
    lds_barrier();
    // as in the fp32 forward: (channel, subgrid row, strip) items over groups
    // of kRowGroupF subgrid rows, real rows only, in order, then one lane per
    // (channel, subcell column)
    const int kn4 = 4 * nstr;
    for (int fr0 = 0; fr0 < n; fr0 += kRowGroupF) {
        const int ng = min(kRowGroupF, n - fr0);
        for (int it = tid; it < C * ng * nstr; it += NT) {
            const int st = it % nstr;
            const int rest = it / nstr;
            const int g = rest % ng, ch = rest / ng;
            const float* pl = go + plane * ch;
            const int row0 = r * b + (fr0 + g) * s;
            const int rows = max(0, min(s, H - row0));   // real rows only
            const int64_t p0 = X0 + 4 * st;
            v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
            if (aligned && p0 + 4 <= lim) {
                const float* col = pl + (int64_t)row0 * pitch + p0;
                int k = 0;
                for (; k + 4 <= rows; k += 4) {
                    v4f w[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        w[i] = ld16f_nt(col + (int64_t)(k + i) * pitch);
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        acc += w[i];
                }
                for (; k < rows; ++k)
                    acc += ld16f_nt(col + (int64_t)k * pitch);
            } else {
                for (int k = 0; k < rows; ++k) {
                    const g_f32* rk = (const g_f32*)(pl + (int64_t)(row0 + k) * pitch);
                    acc.x += (p0 + 0 < lim) ? rk[p0 + 0] : 0.f;
                    acc.y += (p0 + 1 < lim) ? rk[p0 + 1] : 0.f;
                    acc.z += (p0 + 2 < lim) ? rk[p0 + 2] : 0.f;
                    acc.w += (p0 + 3 < lim) ? rk[p0 + 3] : 0.f;
                }
            }
            reinterpret_cast<v4f*>(colsum)[(ch * ng + g) * nstr + st] = acc;
        }
        lds_barrier();
        for (int j = tid; j < C * kn; j += NT) {
            const int ch = j / kn, fc = j - ch * kn;
            const int kc = fc / n, jj = fc - kc * n;
            const int ci = fc * C + ch;
            double part = fr0 == 0 ? 0.0 : cspart[ci];
            for (int g = 0; g < ng; ++g) {
                const float* cs = colsum + (ch * ng + g) * kn4 + fc * s;
                double G = 0.0;
                for (int x = 0; x < s; ++x)
                    G += (double)cs[x];
                part += G;
                if (cflag[kc]) {
                    const int fr = fr0 + g;
                    const uint64_t at = fg_base + ((uint64_t)cidx[kc] * nn + fr * n + jj) * C + ch;
                    const double area = stat_area(F, r * b + fr * s, x0c * b + fc * s, s);
                    const float gv = (a.clip_fg[at] && area > 0.0) ? (float)(G / area) : 0.f;
                    a.g_fg[at] = gv;
                    vgc[(fr * kn + fc) * C + ch] = gv;
                }
            }
            cspart[ci] = part;
        }
        lds_barrier();
    }
    for (int j = tid; j < Kt * C; j += NT) {
        const int kc = j / C, ch = j - kc * C;
        if (cflag[kc])
            continue;
        double G = 0.0;
        for (int jj = 0; jj < n; ++jj)
            G += cspart[(kc * n + jj) * C + ch];
        const uint64_t at = bg_base + (uint64_t)cidx[kc] * C + ch;
        const float gv = a.clip_bg[at] ? (float)(G / stat_area(F, r * b, (x0c + kc) * b, b)) : 0.f;
        a.g_bg[at] = gv;
        vgs[kc * C + ch] = gv;
    }
    if (gin == nullptr)
        return;
    // every real pixel takes its own statistic's gradient (the mirror terms
    // of pixels near padded borders are added by a later pass)
    lds_barrier();
    broadcast_tile_f32(F, r, X0, lim, Kt, nstr, colsum, cflag, vgs, vgc, gin);
}

__global__ __launch_bounds__(kMaxThreads) void k_backward_reduce(TileArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    run_tiles(a, lds, [&](const FrameRec& F, const TileCoord& tc) { backward_reduce_tile(a, F, tc, lds); });
}

__device__ __forceinline__ float g_at(const TileArgs& a, const FrameRec& F, int f, int y, int x, int ch)
{
    const int b = F.b, s = F.s, n = F.n;
    const int64_t cell = F.cell_base + (int64_t)(y / b) * F.GC + x / b;
    const uint32_t idx = a.cell_index[cell];
    if (!a.flags[cell])
        return a.g_bg[a.counts[4 * f + 2] + (uint64_t)idx * F.C + ch];
    const int i = (y % b) / s, j = (x % b) / s;
    return a.g_fg[a.counts[4 * f + 3] + ((uint64_t)idx * n * n + i * n + j) * F.C + ch];
}

// Mirror terms of the adjoint: a real pixel near the bottom or right border is
// also the source of the padded positions that fold onto it, and collects
// their statistics' gradients too.  Its own statistic's gradient is already in
// grad_in (broadcast by the reduction's tile), so only
// the pixels that have mirror preimages are visited, and only the mirror
// terms are added.  Nothing to do in the unpadded mode.
__device__ void backward_mirror_tile(const TileArgs& a, const FrameRec& F, const TileCoord& tc)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    const int b = F.b, H = F.H, W = F.W, C = F.C, pad = F.pad;
    if (pad == kPadNone)
        return;
    const int x0c = tc.ct * F.K;
    const int Kt = min(F.K, F.GC - x0c);
    const int y0 = tc.r * b, y1 = min(y0 + b, H);
    const int xa = x0c * b, xb = min((x0c + Kt) * b, W);
    if (y0 >= H || xa >= W)
        return;
    const int PR = F.GR * b - H, PC = F.GC * b - W;
    // rows at or above lo_r (columns at or above lo_c) may have mirror preimages
    const int lo_r = (PR > 0) ? ((PR <= H - 1) ? H - 1 - PR : 0) : H;
    const int lo_c = (PC > 0) ? ((PC <= W - 1) ? W - 1 - PC : 0) : W;
    if (y1 <= lo_r && xb <= lo_c)
        return;
    // region A: rows [ra, y1) x columns [xa, xb); region B: rows [y0, rb) x columns [ca, xb)
    const int ra = max(y0, lo_r), rb = min(y1, lo_r), ca = max(xa, lo_c);
    const int wA = xb - xa, wB = xb - ca;
    const int64_t nA = ra < y1 ? (int64_t)(y1 - ra) * wA : 0;
    const int64_t nB = (rb > y0 && wB > 0) ? (int64_t)(rb - y0) * wB : 0;
    const int64_t pitch = F.pitch, plane = pitch * H;
    float* gi = a.grad_in[tc.f];
    for (int ch = 0; ch < C; ++ch) {
        for (int64_t q = tid; q < nA + nB; q += NT) {
            int y, x;
            if (q < nA) {
                y = ra + (int)(q / wA);
                x = xa + (int)(q % wA);
            } else {
                y = y0 + (int)((q - nA) / wB);
                x = ca + (int)((q - nA) % wB);
            }
            float acc = 0.f;
            // padded rows folding onto y, each also with the padded columns folding onto x
            for (int yy = (y >= lo_r ? H : F.GR * b); yy < F.GR * b; ++yy)
                if (fold(yy, H, pad) == y) {
                    acc += g_at(a, F, tc.f, yy, x, ch);
                    for (int xx = (x >= lo_c ? W : F.GC * b); xx < F.GC * b; ++xx)
                        if (fold(xx, W, pad) == x)
                            acc += g_at(a, F, tc.f, yy, xx, ch);
                }
            for (int xx = (x >= lo_c ? W : F.GC * b); xx < F.GC * b; ++xx)
                if (fold(xx, W, pad) == x)
                    acc += g_at(a, F, tc.f, y, xx, ch);
            if (acc != 0.f)
                ((g_f32w*)gi)[plane * ch + (int64_t)y * pitch + x] += acc;
        }
    }
}

__global__ __launch_bounds__(kMaxThreads) void k_backward_mirror(TileArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    run_tiles(a, lds, [&](const FrameRec& F, const TileCoord& tc) { backward_mirror_tile(a, F, tc); });
}

// ==========================================================================
// Complexity label from the image (Sec. VI-A names the Sobel operator as one
// source of the region mask): per real pixel, the 3x3 Sobel responses of the
// channel sum S, with neighbours past the border mirrored; the pixel is an
// edge pixel when |Gx| + |Gy| >= threshold * C.  Each tile's real pixels are
// processed in chunks of up to kLabRows x kLabCols whose channel sums, with a
// one-pixel mirrored halo, are staged in LDS exactly as the plan from labels
// stages them; one lane per column walks down the chunk and writes its mask
// byte of every row.
// ==========================================================================
template <int C>
__device__ void edge_tile(const TileArgs& a, const FrameRec& F, const TileCoord& tc, uint16_t* S)
{
    const int b = F.b, H = F.H, W = F.W, pad = F.pad;
    const int x0c = tc.ct * F.K;
    const int Kt = min(F.K, F.GC - x0c);
    const int y0 = tc.r * b, y1 = min(y0 + b, H);
    const int xa = x0c * b, xb = min((x0c + Kt) * b, W);
    if (y0 >= H || xa >= W)
        return;
    const uint8_t* img = static_cast<const uint8_t*>(a.images[tc.f]);
    uint8_t* out = a.masks_out[tc.f];
    const int64_t pitch = F.pitch;
    const int thr = a.edge_threshold * C;
    const bool aligned = ((reinterpret_cast<uintptr_t>(img) | (uintptr_t)pitch) & 15) == 0;
    for (int cy = y0; cy < y1; cy += kLabRows) {
        const int rows = min(kLabRows, y1 - cy);
        for (int cx = xa; cx < xb; cx += kLabCols) {
            const int cols = min(kLabCols, xb - cx);
            // every pair of the chunk starts on an even byte of the mask
            const bool even = ((reinterpret_cast<uintptr_t>(out) | (uintptr_t)W | (uintptr_t)cx) & 1) == 0;
            stage_label_sums<C>(img, pitch, H, W, pad, cy, rows, cx, cols, aligned, S);
            lds_barrier();
            const int np = (cols + 1) >> 1;
            const PairLanes L = pair_lanes(np, rows);
            const int ya = L.split * L.rper, yb = min(rows, ya + L.rper);
            if (L.split < L.splits && ya < yb) {
                for (int p = L.pl; p < np; p += L.step) {
                    g_u8w* o = (g_u8w*)(out + (int64_t)cy * W + cx + 2 * p);
                    if (2 * p + 1 < cols && even)
                        label_pair(S, p, ya, yb, thr, [&](int y, uint32_t d) {
                            // both labels of the pair in one 16-bit store
                            *(g_u16w*)(o + (int64_t)y * W) = (uint16_t)(((d >> 15) & 1u) | ((d >> 31) << 8));
                        });
                    else if (2 * p + 1 < cols)
                        label_pair(S, p, ya, yb, thr, [&](int y, uint32_t d) {
                            o[(int64_t)y * W] = (uint8_t)((d >> 15) & 1u);
                            o[(int64_t)y * W + 1] = (uint8_t)(d >> 31);
                        });
                    else
                        label_pair(S, p, ya, yb, thr,
                                   [&](int y, uint32_t d) { o[(int64_t)y * W] = (uint8_t)((d >> 15) & 1u); });
                }
            }
            lds_barrier();
        }
    }
}

template <int C>
__global__ __launch_bounds__(kMaxThreads) void k_edge_mask(TileArgs a)
{
    __shared__ __align__(16) uint16_t S[(kLabRows + 2) * kLabStride];
    extern __shared__ __align__(16) uint8_t lds[];
    run_one_tile(a, [&](const FrameRec& F, const TileCoord& tc) { edge_tile<C>(a, F, tc, S); });
}

// ==========================================================================
// Utility metrics of the paper's evaluation (Sec. VII-A): MSE and SSIM
// (Wang et al. 2004; 7 x 7 equal-weight windows fully inside the frame,
// sample covariances, K1 = 0.01, K2 = 0.03, range 255, channels averaged).
// With uint8 inputs every window sum of x, y, x^2, y^2 and xy is an integer,
// so the sums are exact and so are the numerators below; only the final
// ratio is fp64.  Each tile writes its partial sums; k_metrics_reduce adds
// them per frame in tile order (deterministic).
//
// SSIM of a window from its integer sums s0 = sum x, s1 = sum y, s2 = sum x^2,
// s3 = sum y^2, s4 = sum xy over np = 49 pixels: with ux = s0/49, the sample
// variances (49 s2 - s0^2) / (49 * 48) and covariance (49 s4 - s0 s1) / (49 * 48),
// the four factors of SSIM share the denominators 49^2 and 49 * 48, which
// cancel:  SSIM = (A B) / (D E) with
//   A = 2 s0 s1 + 49^2 c1,            B = 2 (49 s4 - s0 s1) + 49 * 48 c2,
//   D = s0^2 + s1^2 + 49^2 c1,        E = 49 (s2 + s3) - s0^2 - s1^2 + 49 * 48 c2,
// every integer part below 2^31.
//
// A tile's window centres are covered in chunks of one lane per (channel,
// pixel) pair and up to kMetRowsMax centre rows; the chunk's rows, with 3
// more on each side, are staged in LDS as one plane per channel (all of them
// inside the frame, since every window is), so that the 7 taps of a window
// row are consecutive bytes: a lane reads them as two words and forms the
// row's five moments with byte dot products.  A lane walks down its column:
// the moments of each new row go into a ring of the last 7 rows in
// registers, and the window sum is updated by the new row minus the row
// that leaves it.
// ==========================================================================
constexpr int kMetRowsMax = 32;                 // window-centre rows per chunk
constexpr int kMetStage = kMetRowsMax + 6;      // staged rows per chunk

// Window-centre pixels per chunk (at most 256 lanes of (channel, pixel)) and
// bytes per staged plane row: a row holds the chunk's pixels and the 6 of the
// windows' reach, starting up to 15 pixels early at a 16-pixel boundary, and
// a lane's three words read past its last tap stay inside it.
template <int C>
struct MetShape {
    static constexpr int kCw = 256 / C;
    static constexpr int kRow = (kCw + 26 + 15) & ~15;
};

template <int C>
struct MetLds {
    alignas(16) uint8_t x[C][kMetStage][MetShape<C>::kRow];
    alignas(16) uint8_t y[C][kMetStage][MetShape<C>::kRow];
    double red[kMaxThreads / 64];
    unsigned long long red_se[kMaxThreads / 64];
};

// Squared differences of the 16 bytes of two 16-byte vectors.
__device__ __forceinline__ uint32_t sq_diff16(const v4u& x, const v4u& y)
{
    uint32_t acc = 0u;
    const uint32_t xs[4] = {x.x, x.y, x.z, x.w}, ys[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int d = (int)((xs[k] >> (8 * q)) & 0xFFu) - (int)((ys[k] >> (8 * q)) & 0xFFu);
            acc += (uint32_t)(d * d);
        }
    return acc;
}

struct Moments {
    uint32_t s[4];   // sum x | sum y << 16, sum x^2, sum y^2, sum xy
};

// The five moments of the 7 taps that start `a` bytes into the word xr[0]
// (and yr[0]) of a plane row: the taps as two words (the second one's top
// byte cleared), byte sums and byte products by 4-way dot products.  The two
// byte sums (at most 7 * 255 each) share a word, and so do their window sums
// (at most 49 * 255): a window update adds and subtracts both at once, and
// neither half carries into the other.
__device__ __forceinline__ Moments row_moments(const uint32_t* xr, const uint32_t* yr, uint32_t a)
{
    const uint32_t x0 = __builtin_amdgcn_alignbyte(xr[1], xr[0], a);
    const uint32_t x1 = __builtin_amdgcn_alignbyte(xr[2], xr[1], a) & 0x00FFFFFFu;
    const uint32_t y0 = __builtin_amdgcn_alignbyte(yr[1], yr[0], a);
    const uint32_t y1 = __builtin_amdgcn_alignbyte(yr[2], yr[1], a) & 0x00FFFFFFu;
    constexpr uint32_t one = 0x01010101u;
    Moments m;
    const uint32_t sx = __builtin_amdgcn_udot4(x1, one, __builtin_amdgcn_udot4(x0, one, 0u, false), false);
    const uint32_t sy = __builtin_amdgcn_udot4(y1, one, __builtin_amdgcn_udot4(y0, one, 0u, false), false);
    m.s[0] = sx | (sy << 16);
    m.s[1] = __builtin_amdgcn_udot4(x1, x1, __builtin_amdgcn_udot4(x0, x0, 0u, false), false);
    m.s[2] = __builtin_amdgcn_udot4(y1, y1, __builtin_amdgcn_udot4(y0, y0, 0u, false), false);
    m.s[3] = __builtin_amdgcn_udot4(x1, y1, __builtin_amdgcn_udot4(x0, y0, 0u, false), false);
    return m;
}

// Every factor of a product here is below 2^24 (s0, s1 <= 49 * 255, s4 and
// s2 + s3 <= 2 * 49 * 255^2), so the 24-bit multiplier forms them exactly at
// full rate.  The quotient: the hardware reciprocal refined by one Newton
// step, which squares its relative error (the mean of the windows is held to
// 1e-9 of the oracle's; the denominator is a normal number of at most 2^62,
// so no scaling is needed), times the numerator.  t[0] packs sum x (low
// half) and sum y (high half), each at most 49 * 255; t[1..3] are sum x^2,
// sum y^2 and sum xy.
__device__ __forceinline__ double ssim_window(const uint32_t (&t)[4])
{
    const double c1 = (0.01 * 255.0) * (0.01 * 255.0), c2 = (0.03 * 255.0) * (0.03 * 255.0);
    const uint32_t s0 = t[0] & 0xFFFFu, s1 = t[0] >> 16;
    const int32_t p01 = (int32_t)__umul24(s0, s1), q = (int32_t)(__umul24(s0, s0) + __umul24(s1, s1));
    const double A = (double)(2 * p01) + 2401.0 * c1;
    const double B = (double)(2 * ((int32_t)__umul24(49u, t[3]) - p01)) + 2352.0 * c2;
    const double D = (double)q + 2401.0 * c1;
    const double E = (double)((int32_t)__umul24(49u, t[1] + t[2]) - q) + 2352.0 * c2;
    const double num = A * B, den = D * E;
    double r = __builtin_amdgcn_rcp(den);
    r = fma(r, fma(-den, r, 1.0), r);
    return num * r;
}

// Sixteen pixels of C interleaved channels (C 16-byte vectors; pixel i's
// channel c at byte C i + c) as C planes of 16 bytes, by byte permutes.
template <int C>
__device__ __forceinline__ void deinterleave16(const v4u (&v)[C], v4u (&p)[C])
{
    uint32_t d[4 * C], o[4 * C];   // o[4 c + j]: pixels 4 j .. 4 j + 3 of channel c
#pragma unroll
    for (int i = 0; i < C; ++i) {
        d[4 * i] = v[i].x;
        d[4 * i + 1] = v[i].y;
        d[4 * i + 2] = v[i].z;
        d[4 * i + 3] = v[i].w;
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if constexpr (C == 1) {
                o[j] = d[j];
            } else if constexpr (C == 2) {
                o[4 * c + j] = __builtin_amdgcn_perm(d[2 * j + 1], d[2 * j], 0x06040200u + 0x01010101u * c);
            } else if constexpr (C == 3) {
                constexpr uint32_t lo[3] = {0x0C060300u, 0x0C070401u, 0x0C0C0502u};
                constexpr uint32_t hi[3] = {0x05020100u, 0x06020100u, 0x07040100u};
                o[4 * c + j] = __builtin_amdgcn_perm(d[3 * j + 2], __builtin_amdgcn_perm(d[3 * j + 1], d[3 * j], lo[c]),
                                                     hi[c]);
            } else {
                const uint32_t sel = 0x0C0C0400u + 0x0101u * c;
                o[4 * c + j] = __builtin_amdgcn_perm(__builtin_amdgcn_perm(d[4 * j + 3], d[4 * j + 2], sel),
                                                     __builtin_amdgcn_perm(d[4 * j + 1], d[4 * j], sel), 0x05040100u);
            }
        }
#pragma unroll
    for (int c = 0; c < C; ++c)
        p[c] = v4u{o[4 * c], o[4 * c + 1], o[4 * c + 2], o[4 * c + 3]};
}

// Stage nrs rows (row k at byte r0 + k * pitch) of the pixels [p0, p0 + np)
// of both frames, all inside the frame's width W, as channel planes: channel
// c of pixel p0 + q in row k goes to L.x[c][k][q].  With 16-byte aligned rows
// (`vec`) and p0 a multiple of 16, the 16-pixel groups that end inside the
// width move as C 16-byte vectors per frame (the last one may stage pixels
// past p0 + np, inside the frame and the plane row); the pixels after them
// move byte by byte.  Loads of a batch of items are all issued before the
// first LDS write.
template <int C>
__device__ __forceinline__ void stage_metrics_planes(const g_u8* X, const g_u8* Y, int64_t pitch, int64_t r0, int p0,
                                                     int np, int nrs, int W, bool vec, MetLds<C>& L)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    const int ngv = vec ? min((np + 15) >> 4, (W - p0) >> 4) : 0;
    const int nv = nrs * ngv;
    // items (frame, row, group): a lane holds one group's C vectors at a time
    for (int it = tid; it < 2 * nv; it += NT) {
        const int fy = it >= nv, r = it - fy * nv;
        const int k = r / ngv, g = r - k * ngv;
        const g_u8* src = fy ? Y : X;
        const int64_t at = r0 + (int64_t)k * pitch + (int64_t)(p0 + 16 * g) * C;
        v4u w[C], pl[C];
#pragma unroll
        for (int c = 0; c < C; ++c)
            w[c] = ld16_nt((const void*)(src + at + 16 * c));
        deinterleave16<C>(w, pl);
        uint8_t(&dst)[C][kMetStage][MetShape<C>::kRow] = fy ? L.y : L.x;
#pragma unroll
        for (int c = 0; c < C; ++c)
            *reinterpret_cast<v4u*>(&dst[c][k][16 * g]) = pl[c];
    }
    const int q0 = 16 * ngv, nb = max(0, np - q0) * C, ns = nrs * nb;
    constexpr int kBb = 4;
    for (int base = 0; base < ns; base += kBb * NT) {
        uint8_t bxv[kBb], byv[kBb];
#pragma unroll
        for (int i = 0; i < kBb; ++i) {
            const int it = base + i * NT + tid;
            if (it < ns) {
                const int k = it / nb, j = it - k * nb;
                const int64_t at = r0 + (int64_t)k * pitch + (int64_t)(p0 + q0) * C + j;
                bxv[i] = X[at];
                byv[i] = Y[at];
            }
        }
#pragma unroll
        for (int i = 0; i < kBb; ++i) {
            const int it = base + i * NT + tid;
            if (it < ns) {
                const int k = it / nb, j = it - k * nb;
                const int q = j / C, c = j - q * C;
                L.x[c][k][q0 + q] = bxv[i];
                L.y[c][k][q0 + q] = byv[i];
            }
        }
    }
}

template <int C>
__device__ void metrics_tile(const TileArgs& a, const FrameRec& F, const TileCoord& tc, MetLds<C>& L)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    const int b = F.b, H = F.H, W = F.W;
    const int x0c = tc.ct * F.K;
    const int Kt = min(F.K, F.GC - x0c);
    const int y0 = tc.r * b, y1 = min(y0 + b, H);
    const int xa = x0c * b, xb = min((x0c + Kt) * b, W);
    const uint8_t* X = static_cast<const uint8_t*>(a.images[tc.f]);
    const uint8_t* Y = static_cast<const uint8_t*>(a.outs[tc.f]);
    const g_u8* Xg = (const g_u8*)X;
    const g_u8* Yg = (const g_u8*)Y;
    const int64_t pitch = F.pitch;
    double ssim_acc = 0.0;
    unsigned long long se = 0;
    // squared error over the tile's real pixels: 16-byte strips where the
    // rows allow, single bytes for the rest
    if (y0 < H && xa < W) {
        const int64_t b0 = (int64_t)xa * C, b1 = (int64_t)xb * C;
        const bool aligned = ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y) | (uintptr_t)pitch |
                               (uintptr_t)b0) & 15) == 0;
        const int nv = aligned ? (int)((b1 - b0) >> 4) : 0;
        const int rows = y1 - y0;
        constexpr int kB = 4;   // items whose loads are all in flight together
        for (int base = 0; base < rows * nv; base += kB * NT) {
            v4u wx[kB], wy[kB];
#pragma unroll
            for (int i = 0; i < kB; ++i) {
                const int it = base + i * NT + tid;
                if (it < rows * nv) {
                    const int yy = it / nv, v = it - yy * nv;
                    const int64_t at = (int64_t)(y0 + yy) * pitch + b0 + 16 * v;
                    wx[i] = ld16_nt(X + at);
                    wy[i] = ld16_nt(Y + at);
                }
            }
#pragma unroll
            for (int i = 0; i < kB; ++i)
                if (base + i * NT + tid < rows * nv)
                    se += sq_diff16(wx[i], wy[i]);
        }
        const int nr = (int)(b1 - b0) - 16 * nv;
        for (int it = tid; it < rows * nr; it += NT) {
            const int yy = it / nr, q = it - yy * nr;
            const int64_t at = (int64_t)(y0 + yy) * pitch + b0 + 16 * nv + q;
            const int d = (int)Xg[at] - (int)Yg[at];
            se += (unsigned long long)(d * d);
        }
    }
    // SSIM windows centred in this tile's real pixels, 3 away from every edge
    const int cy0 = max(y0, 3), cy1 = min(y1, H - 3);
    const int cx0 = max(xa, 3), cx1 = min(xb, W - 3);
    const int CW = min(NT, 256) / C;                  // window-centre pixels per chunk
    constexpr int kRowW = MetShape<C>::kRow / 4;      // words per plane row
    const bool vec = ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y) | (uintptr_t)pitch) & 15) == 0;
    for (int cxb = cx0; cxb < cx1; cxb += CW) {
        const int cw = min(CW, cx1 - cxb);
        const int pa = cxb - 3;                         // first pixel a window of the chunk reads
        const int p0 = vec ? (pa & ~15) : pa;
        const int sh = pa - p0;
        const int np = sh + cw + 6;                     // staged pixels from p0
        const int ch = tid / cw, px = tid - ch * cw;    // this lane's (channel, centre pixel)
        const uint32_t o = (uint32_t)(sh + px);
        for (int cyb = cy0; cyb < cy1; cyb += kMetRowsMax) {
            const int rb = min(kMetRowsMax, cy1 - cyb);
            const int nrs = rb + 6;
            stage_metrics_planes<C>(Xg, Yg, pitch, (int64_t)(cyb - 3) * pitch, p0, np, nrs, W, vec, L);
            lds_barrier();
            if (ch < C) {
                const uint32_t* xr = reinterpret_cast<const uint32_t*>(&L.x[ch][0][0]) + (o >> 2);
                const uint32_t* yr = reinterpret_cast<const uint32_t*>(&L.y[ch][0][0]) + (o >> 2);
                Moments ring[7];
                uint32_t t[4] = {0u, 0u, 0u, 0u};
                for (int k0 = 0; k0 < nrs; k0 += 7) {
#pragma unroll
                    for (int j = 0; j < 7; ++j) {
                        const int k = k0 + j;
                        if (k < nrs) {
                            const Moments h = row_moments(xr + k * kRowW, yr + k * kRowW, o & 3u);
#pragma unroll
                            for (int m = 0; m < 4; ++m)
                                t[m] = (t[m] + h.s[m]) - (k >= 7 ? ring[j].s[m] : 0u);
                            ring[j] = h;
                            if (k >= 6)
                                ssim_acc += ssim_window(t);
                        }
                    }
                }
            }
            lds_barrier();
        }
    }
    // workgroup reduction in a fixed order
    const int lane = tid & 63, wid = tid >> 6;
    for (int d = 32; d > 0; d >>= 1) {
        ssim_acc += __shfl_down(ssim_acc, d, 64);
        se += __shfl_down(se, d, 64);
    }
    if (lane == 0) {
        L.red[wid] = ssim_acc;
        L.red_se[wid] = se;
    }
    lds_barrier();
    if (tid == 0) {
        double tt = 0.0;
        unsigned long long e = 0;
        for (int w = 0; w < (NT + 63) / 64; ++w) {
            tt += L.red[w];
            e += L.red_se[w];
        }
        a.met_partial[2 * tc.t] = tt;
        reinterpret_cast<unsigned long long*>(a.met_partial)[2 * tc.t + 1] = e;
    }
    lds_barrier();
}

template <int C>
__global__ __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(C < 4 ? 5 : 4))) void k_metrics(TileArgs a)
{
    __shared__ MetLds<C> L;
    extern __shared__ __align__(16) uint8_t lds[];
    run_one_tile(a, [&](const FrameRec& F, const TileCoord& tc) { metrics_tile<C>(a, F, tc, L); });
}

// One thread per frame: MSE = sum of squared errors / (H W C); SSIM = sum of
// window values / (windows * C), partials added in tile order.
__global__ void k_metrics_reduce(TileArgs a, double* out)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= a.n_frames)
        return;
    const FrameRec F = a.frames[f];
    double t = 0.0;
    unsigned long long e = 0;
    for (int64_t i = 0; i < (int64_t)F.GR * F.TX; ++i) {
        t += a.met_partial[2 * (F.tile_base + i)];
        e += reinterpret_cast<const unsigned long long*>(a.met_partial)[2 * (F.tile_base + i) + 1];
    }
    const double windows = (double)max(F.H - 6, 0) * (double)max(F.W - 6, 0) * F.C;
    out[2 * f + 0] = (double)e / ((double)F.H * F.W * F.C);
    out[2 * f + 1] = windows > 0 ? t / windows : 0.0;
}

// Advance every frame's Philox counter (frame_index) by `step`: the next
// video step of a captured graph draws fresh noise.
__global__ void k_noise_advance(uint64_t* noise, int32_t n, uint64_t step)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        noise[2 * i + 1] += step;
}

// ==========================================================================
// Diagnostics.
// ==========================================================================
__global__ void k_philox(const uint32_t* in, uint32_t* out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t* p = in + 6 * i;
    const uint4 w = philox10(make_uint4(p[0], p[1], p[2], p[3]), p[4], p[5]);
    out[4 * i + 0] = w.x;
    out[4 * i + 1] = w.y;
    out[4 * i + 2] = w.z;
    out[4 * i + 3] = w.w;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
// Workgroups asking for more than 64 KiB of LDS must opt in per kernel.  The
// limit belongs to the kernel, not to a plan, so it is only ever raised (per
// device, under a lock): a smaller request from one host thread must not
// lower it between another thread's opt-in and its launch.
template <typename K>
hipError_t allow_lds(K kernel, size_t lds)
{
    if (lds <= 65536)
        return hipSuccess;
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, size_t> granted;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    const void* fn = reinterpret_cast<const void*>(kernel);
    std::lock_guard<std::mutex> lock(mu);
    size_t& g = granted[{dev, fn}];
    if (lds <= g)
        return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess)
        g = lds;
    return e;
}

static hipError_t launch_scan(const TileArgs& a, bool prefix_scan, hipStream_t s)
{
    if (prefix_scan)
        hipLaunchKernelGGL(k_scan_prefix, dim3((unsigned)a.n_frames), dim3(256), 0, s, a);
    else {
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)a.n_frames), dim3(256), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_scan_frames, dim3(1), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_plan(const TileArgs& a, int64_t n_units, int threads, size_t lds, bool prefix_scan, hipStream_t s)
{
    if (n_units == 0)
        return hipSuccess;
    if (a.masks == nullptr) {
        const int64_t n = std::max<int64_t>(std::max<int64_t>(a.total_cells, a.n_tiles), 4 * (int64_t)a.n_frames);
        const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
        hipLaunchKernelGGL(k_plan_simple, dim3(grid), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    hipError_t e = allow_lds(k_plan, lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_plan, dim3((unsigned)n_units), dim3(threads), lds, s, a);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return launch_scan(a, prefix_scan, s);
}

template <int C>
static hipError_t launch_plan_labels_c(const TileArgs& a, int64_t n_units, int threads, size_t lds, hipStream_t s)
{
    hipError_t e = allow_lds(k_plan_labels<C>, lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_plan_labels<C>, dim3((unsigned)n_units), dim3(threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_plan_labels(const TileArgs& a, int64_t n_units, int threads, size_t lds, unsigned channel_mask,
                              bool prefix_scan, hipStream_t s)
{
    if (n_units == 0)
        return hipSuccess;
    hipError_t e = hipSuccess;
    if (e == hipSuccess && (channel_mask & 2u))
        e = launch_plan_labels_c<1>(a, n_units, threads, lds, s);
    if (e == hipSuccess && (channel_mask & 4u))
        e = launch_plan_labels_c<2>(a, n_units, threads, lds, s);
    if (e == hipSuccess && (channel_mask & 8u))
        e = launch_plan_labels_c<3>(a, n_units, threads, lds, s);
    if (e == hipSuccess && (channel_mask & 16u))
        e = launch_plan_labels_c<4>(a, n_units, threads, lds, s);
    if (e != hipSuccess)
        return e;
    return launch_scan(a, prefix_scan, s);
}

hipError_t launch_store_index(const TileArgs& a, bool prefix_scan, hipStream_t s)
{
    if (a.n_tiles == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_tile_count, dim3((unsigned)((a.n_tiles + 255) / 256)), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return launch_scan(a, prefix_scan, s);
}

template <typename K>
hipError_t launch_tiles(K kernel, const TileArgs& a, int threads, size_t lds, int grid, hipStream_t s)
{
    if (a.n_tiles == 0)
        return hipSuccess;
    hipError_t e = allow_lds(kernel, lds);
    if (e != hipSuccess)
        return e;
    const unsigned g = a.persistent ? (unsigned)grid : (unsigned)a.n_tiles;
    hipLaunchKernelGGL(kernel, dim3(g), dim3(threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_forward(const TileArgs& a, int layout, int C, int threads, size_t lds, int grid, hipStream_t s)
{
    if (layout == 1)
        return launch_tiles(k_forward_f32, a, threads, lds, grid, s);
    if (a.dbg_coarse != nullptr || a.dbg_fine != nullptr) {
        switch (C) {
        case 1: return launch_tiles(k_forward_u8<1, true>, a, threads, lds, grid, s);
        case 2: return launch_tiles(k_forward_u8<2, true>, a, threads, lds, grid, s);
        case 3: return launch_tiles(k_forward_u8<3, true>, a, threads, lds, grid, s);
        default: return launch_tiles(k_forward_u8<4, true>, a, threads, lds, grid, s);
        }
    }
    switch (C) {
    case 1: return launch_tiles(k_forward_u8<1>, a, threads, lds, grid, s);
    case 2: return launch_tiles(k_forward_u8<2>, a, threads, lds, grid, s);
    case 3: return launch_tiles(k_forward_u8<3>, a, threads, lds, grid, s);
    default: return launch_tiles(k_forward_u8<4>, a, threads, lds, grid, s);
    }
}

hipError_t launch_reconstruct(const TileArgs& a, int layout, int C, int threads, size_t lds, int grid, hipStream_t s)
{
    if (layout == 1)
        return launch_tiles(k_reconstruct_f32, a, threads, lds, grid, s);
    switch (C) {
    case 1: return launch_tiles(k_reconstruct_u8<1>, a, threads, lds, grid, s);
    case 2: return launch_tiles(k_reconstruct_u8<2>, a, threads, lds, grid, s);
    case 3: return launch_tiles(k_reconstruct_u8<3>, a, threads, lds, grid, s);
    default: return launch_tiles(k_reconstruct_u8<4>, a, threads, lds, grid, s);
    }
}

hipError_t launch_backward_reduce(const TileArgs& a, int threads, size_t lds, int grid, hipStream_t s)
{
    return launch_tiles(k_backward_reduce, a, threads, lds, grid, s);
}

hipError_t launch_backward_mirror(const TileArgs& a, int threads, int grid, hipStream_t s)
{
    return launch_tiles(k_backward_mirror, a, threads, 0, grid, s);
}

hipError_t launch_edge_mask(const TileArgs& a, int C, int threads, hipStream_t s)
{
    TileArgs b = a;
    b.persistent = 0;
    switch (C) {
    case 1: return launch_tiles(k_edge_mask<1>, b, threads, 0, (int)b.n_tiles, s);
    case 2: return launch_tiles(k_edge_mask<2>, b, threads, 0, (int)b.n_tiles, s);
    case 3: return launch_tiles(k_edge_mask<3>, b, threads, 0, (int)b.n_tiles, s);
    default: return launch_tiles(k_edge_mask<4>, b, threads, 0, (int)b.n_tiles, s);
    }
}

hipError_t launch_metrics(const TileArgs& a, int C, int threads, hipStream_t s)
{
    TileArgs b = a;
    b.persistent = 0;
    switch (C) {
    case 1: return launch_tiles(k_metrics<1>, b, threads, 0, (int)b.n_tiles, s);
    case 2: return launch_tiles(k_metrics<2>, b, threads, 0, (int)b.n_tiles, s);
    case 3: return launch_tiles(k_metrics<3>, b, threads, 0, (int)b.n_tiles, s);
    default: return launch_tiles(k_metrics<4>, b, threads, 0, (int)b.n_tiles, s);
    }
}

hipError_t launch_metrics_reduce(const TileArgs& a, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_metrics_reduce, dim3((unsigned)((a.n_frames + 63) / 64)), dim3(64), 0, s, a, out);
    return hipGetLastError();
}

hipError_t launch_noise_advance(uint64_t* noise, int32_t n, uint64_t step, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_noise_advance, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, noise, n, step);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t occupancy_forward(int layout, int C, int threads, size_t lds, int* blocks_per_cu)
{
    const void* k;
    if (layout == 1)
        k = reinterpret_cast<const void*>(k_forward_f32);
    else if (C == 1)
        k = reinterpret_cast<const void*>(k_forward_u8<1>);
    else if (C == 2)
        k = reinterpret_cast<const void*>(k_forward_u8<2>);
    else if (C == 3)
        k = reinterpret_cast<const void*>(k_forward_u8<3>);
    else
        k = reinterpret_cast<const void*>(k_forward_u8<4>);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, threads, lds);
}

}  // namespace dppix
