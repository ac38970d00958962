// dppix_internal.h — device-side records and launch interfaces of libdppix.
//
// Layout of the work: every frame is cut into bands of b_bg padded rows (one
// row of grid cells) and each band into tiles of K grid cells.  A tile is the
// unit a workgroup processes (Thm. 3 of the paper: cells are independent, so
// any distribution of cells over processing units is valid).  Tiles are
// numbered frame-major, band-major, left to right — which is also row-major
// cell order, the order of the compact store (Table IV).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dppix {

constexpr int kStrip = 16;             // bytes one lane moves per row (dwordx4)
constexpr int kMaxThreads = 512;
constexpr int kMaxB = 256;             // 255 * 256 rows fits a 16-bit lane sum
constexpr int kMaxGroups = 16;         // launch groups: layout x channels x workgroup size
constexpr int kTicketWords = 2 * kMaxGroups;      // two per launch group (resident-grid tickets)

// One frame as the kernels see it (host computes everything derivable).
struct FrameRec {
    int32_t H, W, C, layout;
    int64_t pitch;            // U8: bytes per row; F32: floats per row
    int32_t b, s, n, pad;     // b_bg, b_fg, n = b/s, pad mode
    int32_t GR, GC, K, TX;    // grid rows/cols, cells per tile, tiles per band
    int32_t tau, noise_bg, noise_fg, off32;    // off32: (b + 1) rows of the frame span < 2^31 bytes
    int32_t cnb, ctx, cunits, pad_;           // plan units: bands, tiles per band, units of the frame
    int64_t cell_base;        // first cell of the frame in batch-wide cell arrays
    int64_t fine_base;        // first subcell in dense fine arrays
    int64_t tile_base;        // first tile
    double sigma_bg, sigma_fg;
    uint32_t key0, key1, fi0, fi1;
};

// Workspace layout of a plan (byte offsets from the bound workspace base):
// tables written once by dp_pix_plan_bind and only read afterwards, so one
// bound plan serves any number of concurrent calls.
struct WsLayout {
    size_t frames;        // FrameRec[n_frames]
    size_t tile_map;      // int32[n_tiles][2]: (frame, tile within frame) per scheduling index
    size_t unit_map;      // int32[n_units][2]: (frame, plan unit within frame), frame-major
    size_t border_map;    // int32[n_border][2]: (frame, tile) of the tiles the adjoint's mirror pass visits
    size_t simple_counts; // uint64[n_frames][4]: store counts of a call without masks (every cell simple)
    size_t total;
};

// Per-call state that travels with a store (byte offsets from store->state):
// what dp_pix_plan (or dp_pix_store_index) derives from the flags beside the
// store's counts, and the ticket words of that call sequence's launches.
struct StateLayout {
    size_t tile_cnt;      // uint32[n_tiles]: complex cells per tile
    size_t tile_fg;       // uint32[n_tiles]: complex cells of the frame before the tile
    size_t counters;      // uint32[kTicketWords]: tickets of persistent launches (two per group)
    size_t total;
};

struct TileArgs {
    const FrameRec* frames;
    const int32_t* tile_map;
    const int32_t* unit_map;
    int32_t n_frames;
    int64_t sched_offset;     // first scheduling index of this launch
    int64_t n_tiles;          // tiles of this launch
    uint32_t* ticket;         // [0]: next tile, [1]: finished workgroups
    int32_t persistent;
    // per-frame pointer tables (device arrays of device pointers)
    const uint8_t* const* masks;
    const uint64_t* simple_counts;   // store counts when no frame has a mask (geometry only)
    int64_t total_cells;             // cells of the whole batch (store flags)
    const void* const* images;
    void* const* outs;
    // products of the plan, held by the caller's store
    uint8_t* flags;           // store flags, 1 = complex cell
    uint64_t* counts;         // store counts: per frame n_bg, n_fg, bg offset, fg offset
    uint32_t* tile_cnt;       // store state: complex cells per tile
    uint32_t* tile_fg;        // store state: complex cells of the frame before the tile
    // per-frame Philox (key, counter) of this call: noise[2f] = seed,
    // noise[2f + 1] = frame_index; NULL: the frame records' own
    const uint64_t* noise;
    // store statistics
    float* bg;
    float* fg;
    uint8_t* clip_bg;
    uint8_t* clip_fg;
    // diagnostics
    uint32_t* dbg_coarse;
    uint32_t* dbg_fine;
    // backward
    const float* const* grad_out;
    float* const* grad_in;
    float* g_bg;              // per-statistic gradient, store layout
    float* g_fg;
    uint32_t* cell_index;     // frame-local store index of every cell
    // complexity label
    uint8_t* const* masks_out;
    int32_t edge_threshold;
    // utility metrics: per tile (SSIM partial sum, squared-error sum)
    double* met_partial;
};

// Host-side launchers (defined in dppix_kernels.hip).
// prefix_scan: every frame has the same C and n and the batch has at most
// kPrefixScanTiles tiles (each workgroup of the scan then re-reads the counts
// of all earlier frames instead of waiting for the others).
constexpr int64_t kPrefixScanTiles = 16384;
hipError_t launch_plan(const TileArgs& a, int64_t n_units, int threads, size_t lds, bool prefix_scan,
                       hipStream_t s);
// Plan from the frames' Sobel labels (edge_threshold, images), then the scan;
// channel_mask: bit C set for every channel count C among the frames.
hipError_t launch_plan_labels(const TileArgs& a, int64_t n_units, int threads, size_t lds, unsigned channel_mask,
                              bool prefix_scan, hipStream_t s);
// Tile counts of complex cells from the store's flags alone, then the scan.
hipError_t launch_store_index(const TileArgs& a, bool prefix_scan, hipStream_t s);
hipError_t launch_forward(const TileArgs& a, int layout, int C, int threads, size_t lds, int grid, hipStream_t s);
hipError_t launch_reconstruct(const TileArgs& a, int layout, int C, int threads, size_t lds, int grid,
                              hipStream_t s);
hipError_t launch_backward_reduce(const TileArgs& a, int threads, size_t lds, int grid, hipStream_t s);
hipError_t launch_backward_mirror(const TileArgs& a, int threads, int grid, hipStream_t s);
hipError_t launch_philox(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s);
hipError_t launch_noise_advance(uint64_t* noise, int32_t n, uint64_t step, hipStream_t s);
hipError_t launch_edge_mask(const TileArgs& a, int C, int threads, hipStream_t s);
hipError_t launch_metrics(const TileArgs& a, int C, int threads, hipStream_t s);
hipError_t launch_metrics_reduce(const TileArgs& a, double* out, hipStream_t s);
hipError_t occupancy_forward(int layout, int C, int threads, size_t lds, int* blocks_per_cu);

}  // namespace dppix
