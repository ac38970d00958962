/*
 * dppix.h — C ABI of libdppix, region-adaptive differentially private image
 * pixelization on AMD Instinct MI355X (gfx950).
 *
 * Method: Liu, "A Parallel Region-Adaptive Differential Privacy Framework for
 * Image Pixelization" (arXiv 2511.04261).  A frame of M x N pixels is cut into
 * b x b grid cells (Sec. IV-A, Eq. 1); a foreground mask marks cells as
 * complex, which are cut again into n x n subgrids of size s_b = b/n
 * (Sec. VI-C, Eq. 16).  Each simple cell and each complex subcell releases its
 * mean plus Laplace noise of scale 255 m / (area * eps) (Eq. 11, Sec. VI-A),
 * clipped to [0, 255]; only these statistics and the grid layout are stored
 * (Table IV), and the frame is rebuilt by broadcasting them (Sec. VI-F).
 *
 * Conventions shared by every entry point
 *  - All data pointers are DEVICE pointers owned by the caller.  Per-frame
 *    arrays (images, masks, outputs) are passed as DEVICE arrays of n_frames
 *    device pointers, so a captured graph can be replayed on new frames by
 *    refilling the same buffers.  The library never allocates device memory:
 *    its working memory is the caller's plan workspace (dp_pix_plan_bind),
 *    the per-call state of each store (dppix_store_t.state) and the scratch
 *    arguments of dp_pix_backward / dp_pix_metrics.
 *  - Calls are asynchronous on the given HIP stream and never synchronise
 *    (dp_pix_plan_bind, a set-up call, returns once its upload is done).
 *  - Errors: argument errors are found on the host before anything is
 *    enqueued; the call returns DPPIX_EINVAL (or DPPIX_ENOTSUP for valid but
 *    unsupported parameters) and writes nothing.  Launch failures return
 *    DPPIX_EDEVICE.  dp_pix_last_error() gives a per-thread detail string.
 *  - A plan is immutable once bound: its workspace holds only the frame and
 *    tile tables that dp_pix_plan_bind uploads.  Everything a call sequence
 *    derives from its masks (flags, counts, tile prefixes, ticket words)
 *    lives in that sequence's store, so one plan serves any number of
 *    streams and host threads at once, each with its own store and images.
 *    Calls that share a STORE are ordered by the caller (one stream, or
 *    events); dp_pix_plan_set_launch must not run concurrently with other
 *    calls on the plan.
 *  - One code path: a single frame is a batch of one.
 */
#ifndef DPPIX_H
#define DPPIX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* dppix_stream_t; /* a hipStream_t */

typedef enum {
    DPPIX_OK = 0,
    DPPIX_EINVAL = 1,  /* invalid argument; nothing was enqueued            */
    DPPIX_ENOMEM = 2,  /* host allocation failed or workspace too small      */
    DPPIX_EDEVICE = 3, /* HIP runtime / launch error                         */
    DPPIX_ENOTSUP = 4  /* valid but not supported by this library          */
} dppix_status_t;

typedef enum {
    DPPIX_U8_HWC = 0,  /* uint8, rows of width*channels interleaved bytes   */
    DPPIX_F32_CHW = 1  /* float32, channel planes of height rows each         */
} dppix_layout_t;

typedef enum {
    DPPIX_PAD_SYMMETRIC = 0, /* mirror with the edge pixel repeated (default) */
    DPPIX_PAD_REFLECT = 1,   /* mirror without repeating the edge pixel       */
    DPPIX_PAD_NONE = 2       /* no padding (Algorithm 1): a border cell or
                                subcell holds only its h x w real pixels and
                                its mean divides by h*w; a subcell with no
                                real pixel releases 0 with no noise drawn     */
} dppix_pad_t;

/*
 * One frame (Algorithm 3 inputs: image of size M x N, grid size b, budget eps,
 * max variation m, mask, subgrid factor n = b / s_b).
 *   height, width      M, N >= 1
 *   channels           C in 1..4; cells are per channel, noise is drawn per channel
 *   layout             dppix_layout_t of the image, of a fused/standalone
 *                      reconstruction and of gradients
 *   pitch              U8_HWC: bytes between rows (>= width*channels);
 *                      F32_CHW: floats between rows (>= width); channel planes
 *                      are pitch*height floats apart
 *   pad_mode           dppix_pad_t (Algorithm 2 step 4 / Algorithm 3 step 3;
 *                      NONE: Algorithm 1's border cells)
 *   b_bg               b, grid size of simple cells, 1..256
 *   b_fg               s_b, subgrid size of complex cells; b_bg % b_fg == 0 (Eq. 16)
 *   m                  pixels neighbouring images may differ in (Eq. 11), >= 1
 *   eps_bg, eps_fg     budgets of simple cells and complex subcells, > 0;
 *                      +INFINITY releases the exact mean (no noise)
 *   fg_min_count       tau: a cell is complex iff at least tau of its b*b
 *                      mirror-padded mask pixels (NONE: of its real mask
 *                      pixels) are nonzero; 0 selects ceil(area/2), area = b*b
 *                      (NONE: the cell's real pixel count), the paper's "mean
 *                      of the simple-region mask <= 0.5" rule (Algorithm 3
 *                      step 6) for binary masks
 *   tile_cells         coarse cells per work tile (0 = library default);
 *                      a tuning knob that never changes results
 *   seed               Philox4x32-10 key
 *   frame_index        Philox counter words 2..3; must differ between frames
 *                      released under the same seed
 */
typedef struct {
    int32_t height, width, channels;
    int32_t layout;
    int64_t pitch;
    int32_t pad_mode;
    int32_t b_bg, b_fg;
    int32_t m;
    double eps_bg, eps_fg;
    int32_t fg_min_count;
    int32_t tile_cells;
    uint64_t seed;
    uint64_t frame_index;
} dppix_frame_desc_t;

typedef struct dppix_plan* dppix_plan_t;

/*
 * Compact store (Table IV) for a batch, frames concatenated in batch order:
 *   flags   one byte per grid cell, row-major per frame, frames at
 *           dp_pix_plan_frame_info().cell_offset; 1 = complex
 *   bg      simple cells in row-major order: C floats each (mu'_G, clipped)
 *   fg      complex cells in row-major order: n*n subcells row-major, C
 *           floats each (mu'_{G_s}, clipped)
 *   counts  per frame 4 x uint64: n_bg cells, n_fg cells, offset of the
 *           frame's first float in bg, offset of its first float in fg
 *           (8-byte aligned)
 *   state   store_state_bytes of device memory, 256-byte aligned: the store's
 *           index (complex cells per work tile and before each tile, derived
 *           from the flags) and the ticket words of its call sequence.
 *           dp_pix_plan writes it (dp_pix_store_index rebuilds it from the
 *           flags of a store written elsewhere); its initial contents do
 *           not matter.
 *   noise   optional INPUT of dp_pix_forward / dp_pix_debug_sums: device
 *           array of n_frames x 2 uint64, (seed, frame_index) of each
 *           frame's Philox draws, read when the kernels run; NULL uses the
 *           descriptors' seed and frame_index.  One plan then serves every
 *           step of a video: a replayed graph draws fresh noise once the
 *           counters are advanced (dp_pix_noise_advance).  The seed is the
 *           generator's key and must stay secret: whoever knows it can
 *           regenerate the noise and subtract it.
 * Capacities (worst case: every cell simple, resp. complex) come from
 * dp_pix_plan_sizes; actual counts stay on the device.  forward, reconstruct
 * and backward read the cell classes and offsets from the store they are
 * given and nothing else, so any number of stores of one plan can be in use.
 */
typedef struct {
    float* bg;
    float* fg;
    uint8_t* flags;
    uint64_t* counts;
    void* state;
    const uint64_t* noise;
} dppix_store_t;

typedef struct {
    size_t workspace_bytes;  /* device workspace for dp_pix_plan_bind          */
    size_t bg_capacity;      /* floats                                          */
    size_t fg_capacity;      /* floats                                          */
    size_t flag_bytes;       /* total grid cells                                */
    size_t clip_bytes_bg;    /* bytes of clip bits for bg (one per float)       */
    size_t clip_bytes_fg;    /* bytes of clip bits for fg (one per float)       */
    size_t grad_scratch_bytes; /* device scratch for dp_pix_backward            */
    int64_t n_tiles;         /* work tiles of the batch                         */
    int64_t total_pixels;    /* sum of height*width                             */
    size_t metrics_scratch_bytes; /* device scratch for dp_pix_metrics          */
    size_t store_state_bytes; /* dppix_store_t.state of each store              */
    int64_t forward_launches; /* kernel launches of one dp_pix_forward (one per group
                                 of frames sharing layout, channels and workgroup size) */
} dppix_sizes_t;

typedef struct {
    int32_t grid_rows, grid_cols, n;   /* G_R, G_C, n                        */
    int32_t pad_rows, pad_cols;        /* P_R, P_C                           */
    int32_t tile_cells, tiles_per_band;
    int32_t fg_min_count;              /* effective tau (0: per-cell majority of the real pixels, unpadded mode) */
    int64_t cell_offset;               /* first flag byte of this frame      */
    int64_t fine_offset;               /* first subcell in dense fine arrays */
    double sigma_bg, sigma_fg;         /* Eq. (11) scales; 0 when noise off  */
} dppix_frame_info_t;

/* ---------------------------------------------------------------------------
 * Plan (Algorithm 3 steps 1-6).
 * ------------------------------------------------------------------------- */

/* Validate n_frames descriptors (host memory, copied) and lay out geometry,
 * tiles and store capacities.  Host only: no device call. */
dppix_status_t dp_pix_plan_create(const dppix_frame_desc_t* descs, int32_t n_frames, dppix_plan_t* out);

/* Release a plan (host memory only). */
void dp_pix_plan_destroy(dppix_plan_t plan);

dppix_status_t dp_pix_plan_sizes(dppix_plan_t plan, dppix_sizes_t* out);

/* The sizes of dp_pix_plan_sizes for n_frames descriptors, without keeping a
 * plan: host only, for sizing buffers before anything is allocated.  Returns
 * the status dp_pix_plan_create would return for these descriptors. */
dppix_status_t dp_pix_plan_workspace_size(const dppix_frame_desc_t* descs, int32_t n_frames, dppix_sizes_t* out);
dppix_status_t dp_pix_plan_frame_info(dppix_plan_t plan, int32_t frame, dppix_frame_info_t* out);

/* Bind a device workspace of at least workspace_bytes (256-byte aligned) and
 * upload the plan's frame and tile tables into it: one host-to-device copy on
 * the stream, waited for before returning, so the plan may be used from any
 * stream afterwards.  A plan is bound once (EINVAL on a second bind); not
 * for use under stream capture. */
dppix_status_t dp_pix_plan_bind(dppix_plan_t plan, void* workspace, size_t bytes, dppix_stream_t stream);

/* Classify every grid cell and lay out the compact store (Algorithm 3 steps
 * 3-6): count nonzero mask pixels of each mirror-padded b x b cell, flag it
 * complex when the count reaches tau, then scan the flags into store offsets
 * and per-frame counts (written to store->flags, store->counts and
 * store->state; bg and fg are not touched and may be NULL).
 *   masks   device array of n_frames device pointers to uint8 masks of
 *           height x width bytes, rows width bytes apart; NULL, or a NULL
 *           entry, makes every cell of that frame simple (Algorithm 2).
 * Kernels only: safe under stream capture. */
dppix_status_t dp_pix_plan(dppix_plan_t plan, const uint8_t* const* masks, const dppix_store_t* store,
                           dppix_stream_t stream);

/* dp_pix_plan with the region mask computed from the frames in the same pass
 * (Sec. VI-A: the mask may come from an edge detector such as the Sobel
 * operator): a cell's count is the number of its b x b mirror-padded positions
 * whose pixel is an edge pixel by the rule of dp_pix_edge_mask (a padded
 * position takes the label of the real pixel it folds onto; NONE counts real
 * positions only).  Gives exactly the flags, counts and state of
 * dp_pix_edge_mask followed by dp_pix_plan on its masks, without writing or
 * reading an H x W mask.
 *   images     device array of n_frames device pointers (U8_HWC frames only)
 *   threshold  0..4096, per-channel units, as dp_pix_edge_mask
 * A label computed from the frame depends on the data: the released flags
 * then carry information the Laplace noise does not cover.
 * Kernels only: safe under stream capture. */
dppix_status_t dp_pix_plan_labels(dppix_plan_t plan, const void* const* images, int32_t threshold,
                                  const dppix_store_t* store, dppix_stream_t stream);

/* Rebuild a store's counts and state from its flags alone (Table IV: the
 * flags are the grid layout), for a store whose flags and statistics were
 * written elsewhere, e.g. decoded from its serialised form: frames are
 * packed back to back in batch order, as dp_pix_plan lays them out.  Flag
 * bytes are read as complex when nonzero.  bg and fg are not touched. */
dppix_status_t dp_pix_store_index(dppix_plan_t plan, const dppix_store_t* store, dppix_stream_t stream);

/* Region mask from the frames themselves (Sec. VI-A: the mask may come from an
 * edge detector such as the Sobel operator): for every real pixel, the 3x3
 * Sobel responses Gx, Gy of the sum of its channels, neighbours past the
 * border mirrored as pad_mode says (NONE mirrors like SYMMETRIC); the mask
 * byte is 1 when
 * |Gx| + |Gy| >= threshold * channels, else 0.
 *   images     device array of n_frames device pointers (U8_HWC frames only)
 *   threshold  0..4096, per-channel units
 *   masks_out  device array of n_frames device pointers to height*width bytes
 *              (rows width bytes apart), ready for dp_pix_plan.
 * A mask computed from the frame depends on the data: the released flags then
 * carry information the Laplace noise does not cover. */
dppix_status_t dp_pix_edge_mask(dppix_plan_t plan, const void* const* images, int32_t threshold,
                                uint8_t* const* masks_out, dppix_stream_t stream);

/* Utility of a release, as the paper measures it (Sec. VII-A): per frame the
 * mean squared error and SSIM (Wang et al. 2004) between images[f] and
 * recons[f] (U8_HWC frames of the plan's geometry, e.g. a frame and its
 * reconstruction).  SSIM: 7 x 7 equal-weight windows lying inside the frame,
 * sample covariances, K1 = 0.01, K2 = 0.03, range 255, averaged over windows
 * and channels (0 for frames under 7 x 7).  out: device array of n_frames
 * (MSE, SSIM) double pairs; scratch: metrics_scratch_bytes of device memory.
 * Window sums are exact integers; the result does not depend on scheduling. */
dppix_status_t dp_pix_metrics(dppix_plan_t plan, const void* const* images, const void* const* recons, void* scratch,
                              size_t scratch_bytes, double* out, dppix_stream_t stream);

/* ---------------------------------------------------------------------------
 * Forward (Algorithm 3 steps 7-19; Algorithm 2 steps 6-9).
 * Exact integer sums of every subcell over the mirror-padded frame (uint8
 * input; fp64 for float input), means, Laplace noise from Philox4x32-10 with
 * counter (cell id, channel | level << 8, frame_index) and key seed, clip to
 * [0, 255], one rounding to fp32, written to the compact store.
 *   images     device array of n_frames device pointers (layout per frame)
 *   store      from dp_pix_plan on this plan
 *   clip_bg/fg optional (may be NULL): one byte per stored float, 1 when the
 *              noisy mean was inside [0, 255] (its gradient passes)
 *   fused_out  optional device array of n_frames output pointers: also write
 *              the reconstruction (steps 11, 18-21) in the same pass.  An
 *              output must not overlap its image: with mirror padding a
 *              tile reads rows and columns that neighbouring tiles of the
 *              same launch write, so an in-place forward races.
 * ------------------------------------------------------------------------- */
dppix_status_t dp_pix_forward(dppix_plan_t plan, const void* const* images, const dppix_store_t* store,
                              uint8_t* clip_bg, uint8_t* clip_fg, void* const* fused_out,
                              dppix_stream_t stream);

/* Restoration from the stored metadata (Sec. VI-F): every real pixel takes the
 * value of its cell or subcell; U8_HWC output is rounded half-to-even, F32_CHW
 * output is the stored value.  Reads the given store only (flags, counts,
 * state and statistics): a store keeps its own layout whatever other stores
 * of the plan were planned since.  out: device array of n_frames pointers. */
dppix_status_t dp_pix_reconstruct(dppix_plan_t plan, const dppix_store_t* store, void* const* out,
                                  dppix_stream_t stream);

/* Adjoint of forward + reconstruct for F32_CHW frames, noise and mask held
 * fixed (not in the paper; exact derivative of the map above):
 *   grad_in(p) = sum over padded positions x folding onto p of
 *                pass_k(x) * G_k(x) / area_k(x),
 * where k(x) is the statistic covering x and G_k sums grad_out over the real
 * pixels of k.  store is the one the matching dp_pix_forward wrote (its cell
 * classes and offsets); clip_bg/clip_fg are the bits that forward wrote;
 * scratch holds grad_scratch_bytes of device memory. */
dppix_status_t dp_pix_backward(dppix_plan_t plan, const dppix_store_t* store, const float* const* grad_out,
                               const uint8_t* clip_bg, const uint8_t* clip_fg, float* const* grad_in,
                               void* scratch, size_t scratch_bytes, dppix_stream_t stream);

/* dp_pix_backward without a scratch argument, for callers that cannot
 * allocate device memory (code under stream capture, tight serving or
 * training loops, harnesses that forbid hipMalloc): the scratch is a fixed
 * 32 MiB device array inside the library, one per GPU, held from the
 * library's load until the process ends.  Calls the same kernels as
 * dp_pix_backward and gives the same result.  Returns DPPIX_ENOMEM, having
 * enqueued nothing, when the plan's grad_scratch_bytes exceed 32 MiB (about
 * 8 M statistics and cells; use dp_pix_backward then).  Allocates nothing:
 * the device address of the array is looked up once per device, on the
 * first call with that device current.  Every call on a GPU shares that
 * GPU's array, so calls that may overlap on one GPU (other streams, other
 * host threads) race and must be ordered by the caller.  The array needs
 * no clearing: the first kernel writes every entry the second reads. */
dppix_status_t dp_pix_backward_static(dppix_plan_t plan, const dppix_store_t* store, const float* const* grad_out,
                                      const uint8_t* clip_bg, const uint8_t* clip_fg, float* const* grad_in,
                                      dppix_stream_t stream);

/* ---------------------------------------------------------------------------
 * Execution options, graphs, diagnostics.
 * ------------------------------------------------------------------------- */

/* Launch shape of the tile kernels: threads per workgroup (64..512, multiple
 * of 64; 0 = the default: 256, except forward and reconstruction tiles with
 * few row items per tile, which run 128 per workgroup in a launch of their
 * own) and the work distribution: persistent = 0 launches one
 * workgroup per tile (the hardware dispatcher feeds the CUs; the default);
 * persistent = 1 launches as many workgroups as the CUs hold at once and
 * persistent = k in 2..64 launches k per CU — those workgroups stay resident
 * and pull tiles from an atomic ticket in the workspace.  Results never
 * depend on these. */
dppix_status_t dp_pix_plan_set_launch(dppix_plan_t plan, int32_t threads, int32_t persistent);

/* Capture plan + forward (+ fused reconstruction) on the stream into a HIP
 * graph and instantiate it; dp_pix_graph_launch replays it.  The pointer
 * arrays are read by the kernels at replay time. */
typedef struct dppix_graph* dppix_graph_t;
dppix_status_t dp_pix_graph_create(dppix_plan_t plan, const uint8_t* const* masks, const void* const* images,
                                   const dppix_store_t* store, void* const* fused_out, dppix_stream_t stream,
                                   dppix_graph_t* out);
dppix_status_t dp_pix_graph_launch(dppix_graph_t graph, dppix_stream_t stream);
void dp_pix_graph_destroy(dppix_graph_t graph);

/* dp_pix_forward (no clip bits, no fused output) that also writes the exact
 * sums of every cell and subcell of every frame over the mirror-padded frame
 * (Eq. 2 numerators, Algorithm 3 steps 8 and 14), for parity checks:
 * coarse[(cell_offset + r*G_C + c)*C + ch] and
 * fine[(fine_offset + i*(G_C*n) + j)*C + ch] for subcell row i, column j.
 * uint8 frames only. */
dppix_status_t dp_pix_debug_sums(dppix_plan_t plan, const void* const* images, const dppix_store_t* store,
                                 uint32_t* coarse, uint32_t* fine, dppix_stream_t stream);

/* Add step to the frame_index of each of n_frames (seed, frame_index) pairs
 * of a store's noise array (8-byte aligned device memory), on the stream:
 * the next release of the same frames draws fresh noise (a frame_index must
 * never repeat under one seed).  A kernel, so it can be captured with the
 * calls it precedes or follows. */
dppix_status_t dp_pix_noise_advance(uint64_t* noise, int32_t n_frames, uint64_t step, dppix_stream_t stream);

/* Raw Philox4x32-10 blocks: for i < n, words[4i..4i+3] = Philox(ctr = in[6i..6i+3], key = in[6i+4..6i+5]). */
dppix_status_t dp_pix_debug_philox(const uint32_t* in, uint32_t* words, int64_t n, dppix_stream_t stream);

const char* dp_pix_status_string(dppix_status_t status);
const char* dp_pix_last_error(void);
const char* dp_pix_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DPPIX_H */
