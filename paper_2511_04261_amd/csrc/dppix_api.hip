// dppix_api.hip — host side of the libdppix C ABI: argument validation, plan
// layout (geometry, tiles, workspace, store capacities) and kernel launches.
#include "dppix.h"
#include "dppix_internal.h"
#include "dppix_tiles.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

using namespace dppix;

namespace {

thread_local std::string g_err;

dppix_status_t fail(dppix_status_t st, const std::string& msg)
{
    g_err = msg;
    return st;
}

dppix_status_t dev_fail(hipError_t e, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return DPPIX_EDEVICE;
}

constexpr int kDefaultThreads = 256;
constexpr int64_t kTileBytesTarget = 2048;  // padded bytes per tile row (u8)
constexpr int64_t kPlanCellsMax = 2048;     // cells per band of one plan unit
constexpr int64_t kPlanLdsMax = 32 * 1024;  // LDS of one plan unit
constexpr int64_t kTileLdsTarget = 48 * 1024;
constexpr int64_t kTileLdsMax = 150 * 1024;
constexpr int kMaxDim = 1 << 24;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
size_t grad_scratch_need(dppix_plan_t p);

}  // namespace

// Frames sharing layout, channel count and workgroup size, launched together.
struct LaunchGroup {
    int layout, C;
    int threads;          // workgroup size chosen for the group's tiles
    int64_t lo, hi;       // scheduling-index range
    size_t lds_fwd, lds_rec;
};

struct dppix_plan {
    std::vector<dppix_frame_desc_t> desc;
    std::vector<FrameRec> frames;
    std::vector<int32_t> sched_frame;
    std::vector<int64_t> sched_base;
    int64_t n_tiles = 0;
    int64_t n_units = 0;
    int64_t n_border = 0;               // tiles with pixels that mirrored padding folds onto
    bool prefix_scan = false;           // the plan's scan needs no hand-off between workgroups
    int64_t total_cells = 0;
    int64_t total_fine = 0;
    int64_t total_pixels = 0;
    size_t bg_cap = 0, fg_cap = 0;
    WsLayout ws{};
    StateLayout st{};
    size_t lds[6] = {0, 0, 0, 0, 0, 0};
    std::vector<LaunchGroup> groups;
    bool any_f32 = false, any_u8 = false;
    int threads = 0;                    // 0: per launch group (forward, reconstruct), else fixed
    int persistent = 0;
    int cus = 0;                        // compute units of the bound device
    uint8_t* bound = nullptr;
    size_t bound_bytes = 0;
    std::vector<uint8_t> host_tables;   // frame records and scheduling maps, as uploaded
};

struct dppix_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// Largest multiple of `unit` not above x (at least `unit` when x >= unit).
int64_t round_down(int64_t x, int64_t unit) { return (x / unit) * unit; }

dppix_status_t validate(const dppix_frame_desc_t& d, int32_t f)
{
    char buf[256];
    auto bad = [&](const char* what) {
        std::snprintf(buf, sizeof buf, "frame %d: %s", f, what);
        return fail(DPPIX_EINVAL, buf);
    };
    if (d.height < 1 || d.width < 1)
        return bad("height and width must be >= 1");
    if (d.height > kMaxDim || d.width > kMaxDim)
        return fail(DPPIX_ENOTSUP, "frame dimensions above 2^24");
    if (d.channels < 1 || d.channels > 4)
        return bad("channels must be in 1..4");
    if (d.layout != DPPIX_U8_HWC && d.layout != DPPIX_F32_CHW)
        return bad("unknown layout");
    if (d.layout == DPPIX_U8_HWC && d.pitch < (int64_t)d.width * d.channels)
        return bad("pitch must be >= width*channels bytes");
    if (d.layout == DPPIX_F32_CHW && d.pitch < (int64_t)d.width)
        return bad("pitch must be >= width floats");
    if (d.pad_mode != DPPIX_PAD_SYMMETRIC && d.pad_mode != DPPIX_PAD_REFLECT && d.pad_mode != DPPIX_PAD_NONE)
        return bad("unknown pad_mode");
    if (d.b_fg < 1 || d.b_bg < d.b_fg)
        return bad("need 1 <= b_fg <= b_bg");
    if (d.b_bg % d.b_fg != 0)
        return bad("b_bg must be a multiple of b_fg (b = n * s_b)");
    if (d.b_bg > kMaxB)
        return fail(DPPIX_ENOTSUP, "b_bg above 256");
    if (d.m < 1)
        return bad("m must be >= 1");
    if (!(d.eps_bg > 0.0) || !(d.eps_fg > 0.0))
        return bad("eps_bg and eps_fg must be > 0 (+inf disables noise)");
    if (d.fg_min_count < 0 || (int64_t)d.fg_min_count > (int64_t)d.b_bg * d.b_bg)
        return bad("fg_min_count must be in [0, b_bg^2]");
    if (d.tile_cells < 0)
        return bad("tile_cells must be >= 0");
    const int64_t n = d.b_bg / d.b_fg;
    const int64_t GR = (d.height + d.b_bg - 1) / d.b_bg, GC = (d.width + d.b_bg - 1) / d.b_bg;
    if ((GR * n) * (GC * n) > (int64_t)UINT32_MAX)
        return fail(DPPIX_ENOTSUP, "more than 2^32 subcells in one frame");
    return DPPIX_OK;
}

double sigma_of(int b, int m, double eps)
{
    // Eq. (11): Delta = 255 m / b^2; Eq. (8): sigma = Delta / eps
    const double delta = 255.0 * (double)m / ((double)b * (double)b);
    return delta / eps;
}

// Per-kind LDS bytes of one frame with K cells per tile.
size_t frame_lds(int kind, const FrameRec& F) { return lds_plan(kind, F.K, F.b, F.n, F.C).bytes; }

int kind_fwd(const FrameRec& F) { return F.layout == DPPIX_F32_CHW ? kFwdF32 : kFwdU8; }
int kind_rec(const FrameRec& F) { return F.layout == DPPIX_F32_CHW ? kRecF32 : kRecU8; }

// Tile width: about kTileBytesTarget padded bytes per row, tiles of one band
// balanced, u8 tiles starting on 16-byte boundaries when possible, LDS bounded.
void choose_tiles(FrameRec& F, int32_t requested)
{
    const int64_t unit_bytes = (F.layout == DPPIX_F32_CHW) ? 4 * (int64_t)F.b : (int64_t)F.b * F.C;
    int64_t align = 16 / std::gcd<int64_t>(16, unit_bytes);  // cells per 16-byte-aligned step
    int64_t K;
    if (requested > 0) {
        K = std::min<int64_t>(requested, F.GC);
    } else {
        // the band's padded row cut into the fewest tiles of at most about
        // kTileBytesTarget bytes (a batch of 768-pixel frames alone runs 7 %
        // faster with one 2304-byte tile per band, the mixed-resolution batch
        // 3.8 % slower; the autotuner can pick the former for such batches)
        int64_t kmax = std::max<int64_t>(1, kTileBytesTarget / unit_bytes);
        if (kmax >= align)
            kmax = round_down(kmax, align);
        const int64_t band = (int64_t)F.GC * unit_bytes;
        const int64_t tx = std::max<int64_t>(1, (band + kTileBytesTarget - 1) / kTileBytesTarget);
        K = (F.GC + tx - 1) / tx;
        if (K % align != 0 && ((K + align - 1) / align) * align <= std::max(kmax, K))
            K = ((K + align - 1) / align) * align;
        K = std::min<int64_t>(K, F.GC);
    }
    F.K = (int32_t)std::max<int64_t>(1, K);
    // keep every tile kind of this frame within the LDS target
    while (F.K > 1) {
        size_t need = std::max(frame_lds(kind_fwd(F), F), frame_lds(kind_rec(F), F));
        if (F.layout == DPPIX_F32_CHW)
            need = std::max(need, frame_lds(kBwd, F));
        if ((int64_t)need <= kTileLdsTarget)
            break;
        F.K = std::max(1, F.K / 2);
    }
    F.TX = (F.GC + F.K - 1) / F.K;
    // Plan units: whole tiles of a band (at most kPlanCellsMax cells), and as
    // many bands as keep about one 16-row strip item per lane of a 256-lane
    // workgroup (several bands' worth of rows per lane when b < 16).
    F.ctx = (int32_t)std::max<int64_t>(1, std::min<int64_t>(F.TX, kPlanCellsMax / F.K));
    const int64_t kc = std::min<int64_t>((int64_t)F.ctx * F.K, F.GC);
    const int64_t nstr = (kc * F.b + 15) / 16;
    const int64_t rows = std::min<int64_t>(F.b, 16);
    const int64_t items = nstr * ((F.b + rows - 1) / rows);
    int64_t cnb = (int64_t)kDefaultThreads * std::max<int64_t>(1, 16 / F.b) / items;
    cnb = std::max<int64_t>(1, std::min<int64_t>(cnb, F.GR));
    while (cnb > 1 && plan_lds((int)cnb, F.ctx, F.K) > kPlanLdsMax)
        --cnb;
    F.cnb = (int32_t)cnb;
    F.cunits = (int32_t)(((F.GR + cnb - 1) / cnb) * ((F.TX + F.ctx - 1) / F.ctx));
}

// XCD-aware tile order within one launch's scheduling range [lo, hi): the
// dispatcher hands workgroup i of a launch to XCD i mod kXcds, and each XCD
// has its own L2.  Neighbouring tiles of a band share the cache lines their
// rows are cut at (rows whose pitch or tile width is not a whole number of
// lines), so the map gives every XCD runs of kXcdRun consecutive tiles:
// within each chunk of kXcds * kXcdRun workgroups, workgroup i takes tile
// (i mod kXcds) * kXcdRun + i / kXcds of the chunk.  A shared line is then
// fetched once, by one L2, while both tiles are in flight.  The last partial
// chunk keeps the linear order.
constexpr int64_t kXcds = 8;
constexpr int64_t kXcdRun = 8;

void xcd_runs(int32_t* map, int64_t lo, int64_t hi)
{
    const int64_t n = hi - lo, chunk = kXcds * kXcdRun;
    const int64_t full = (n / chunk) * chunk;
    std::vector<int32_t> tmp(2 * (size_t)full);
    for (int64_t i = 0; i < full; ++i) {
        const int64_t c = i / chunk, w = i - c * chunk;
        const int64_t t = c * chunk + (w % kXcds) * kXcdRun + w / kXcds;
        tmp[2 * i] = map[2 * (lo + t)];
        tmp[2 * i + 1] = map[2 * (lo + t) + 1];
    }
    std::copy(tmp.begin(), tmp.end(), map + 2 * lo);
}

// Workgroup size of a frame's forward and reconstruction tiles.  A u8 tile
// with few phase-1 items (strips x groups of subgrid rows, e.g. b = 16 or
// narrow frames) keeps more tiles in flight per CU with 128 lanes; larger
// tiles fill 256 (measured on 64 x 1080p and 300 x 768x576 batches).
int tile_threads(const FrameRec& F)
{
    if (F.layout != DPPIX_U8_HWC)
        return kDefaultThreads;
    const int64_t nstr = ((int64_t)F.K * F.b * F.C + 15) / 16;
    const int q = F.s == 2 ? 4 : ((F.s == 3 || F.s == 4) ? 2 : 1);
    const int64_t ngq = (std::min(F.n, kRowGroup) + q - 1) / q;
    return nstr * ngq <= 320 ? 128 : kDefaultThreads;
}

}  // namespace

extern "C" {

const char* dp_pix_version(void) { return "dppix 0.1 (gfx950)"; }

const char* dp_pix_status_string(dppix_status_t s)
{
    switch (s) {
    case DPPIX_OK: return "ok";
    case DPPIX_EINVAL: return "invalid argument";
    case DPPIX_ENOMEM: return "out of memory";
    case DPPIX_EDEVICE: return "device error";
    case DPPIX_ENOTSUP: return "not supported";
    }
    return "unknown status";
}

const char* dp_pix_last_error(void) { return g_err.c_str(); }

dppix_status_t dp_pix_plan_create(const dppix_frame_desc_t* descs, int32_t n_frames, dppix_plan_t* out)
{
    if (out == nullptr)
        return fail(DPPIX_EINVAL, "out is NULL");
    *out = nullptr;
    if (descs == nullptr || n_frames < 1)
        return fail(DPPIX_EINVAL, "need at least one frame descriptor");
    for (int32_t f = 0; f < n_frames; ++f) {
        dppix_status_t st = validate(descs[f], f);
        if (st != DPPIX_OK)
            return st;
    }
    dppix_plan* p = new (std::nothrow) dppix_plan;
    if (p == nullptr)
        return fail(DPPIX_ENOMEM, "host allocation failed");
    p->desc.assign(descs, descs + n_frames);
    p->frames.resize(n_frames);
    int64_t cell = 0, fine = 0, tile = 0;
    for (int32_t f = 0; f < n_frames; ++f) {
        const dppix_frame_desc_t& d = descs[f];
        FrameRec& F = p->frames[f];
        std::memset(&F, 0, sizeof F);
        F.H = d.height;
        F.W = d.width;
        F.C = d.channels;
        F.layout = d.layout;
        F.pitch = d.pitch;
        F.b = d.b_bg;
        F.s = d.b_fg;
        F.n = d.b_bg / d.b_fg;
        F.pad = d.pad_mode;
        F.GR = (d.height + d.b_bg - 1) / d.b_bg;   // G_R = ceil(M / b)
        F.GC = (d.width + d.b_bg - 1) / d.b_bg;    // G_C = ceil(N / b)
        // tau = 0 in the unpadded mode: majority of each cell's real pixels
        F.tau = d.fg_min_count > 0 ? d.fg_min_count
                                   : (d.pad_mode == DPPIX_PAD_NONE ? 0 : (d.b_bg * d.b_bg + 1) / 2);
        F.noise_bg = std::isinf(d.eps_bg) ? 0 : 1;
        F.noise_fg = std::isinf(d.eps_fg) ? 0 : 1;
        F.sigma_bg = F.noise_bg ? sigma_of(F.b, d.m, d.eps_bg) : 0.0;
        F.sigma_fg = F.noise_fg ? sigma_of(F.s, d.m, d.eps_fg) : 0.0;
        F.key0 = (uint32_t)(d.seed & 0xFFFFFFFFu);
        F.key1 = (uint32_t)(d.seed >> 32);
        F.fi0 = (uint32_t)(d.frame_index & 0xFFFFFFFFu);
        F.fi1 = (uint32_t)(d.frame_index >> 32);
        F.off32 = ((int64_t)d.b_bg + 1) * d.pitch * (d.layout == DPPIX_F32_CHW ? 4 : 1) < ((int64_t)1 << 31);
        choose_tiles(F, d.tile_cells);
        {
            size_t need = std::max(frame_lds(kind_fwd(F), F), frame_lds(kind_rec(F), F));
            if ((int64_t)need > kTileLdsMax) {
                delete p;
                return fail(DPPIX_ENOTSUP, "n*n*channels too large for one tile in LDS");
            }
        }
        F.cell_base = cell;
        F.fine_base = fine;
        F.tile_base = tile;
        cell += (int64_t)F.GR * F.GC;
        fine += (int64_t)F.GR * F.n * F.GC * F.n;
        tile += (int64_t)F.GR * F.TX;
        p->n_units += F.cunits;
        p->lds[kPlan] = std::max<size_t>(p->lds[kPlan], plan_lds(F.cnb, F.ctx, F.K));
        p->bg_cap += (size_t)F.GR * F.GC * F.C;
        p->fg_cap += (size_t)F.GR * F.GC * F.n * F.n * F.C;
        p->total_pixels += (int64_t)F.H * F.W;
        if (F.layout == DPPIX_F32_CHW)
            p->any_f32 = true;
        else
            p->any_u8 = true;
        for (int k = 1; k < 6; ++k) {
            if (k == kBwd && F.layout != DPPIX_F32_CHW)
                continue;
            if ((k == kFwdU8 || k == kRecU8) && F.layout != DPPIX_U8_HWC)
                continue;
            if ((k == kFwdF32 || k == kRecF32) && F.layout != DPPIX_F32_CHW)
                continue;
            p->lds[k] = std::max(p->lds[k], frame_lds(k, F));
        }
    }
    p->total_cells = cell;
    p->total_fine = fine;
    p->n_tiles = tile;
    if (tile > (int64_t)INT32_MAX || p->n_units > (int64_t)INT32_MAX) {
        delete p;
        return fail(DPPIX_ENOTSUP, "more than 2^31 tiles");
    }
    p->prefix_scan = tile <= kPrefixScanTiles;
    for (const FrameRec& F : p->frames)
        p->prefix_scan = p->prefix_scan && F.C == p->frames[0].C && F.n == p->frames[0].n && F.K < 65536;
    // Scheduling order: frames with the heaviest tiles first (longest tiles
    // start early, the tail is made of light ones); ties keep batch order.
    std::vector<int32_t> order(n_frames);
    std::iota(order.begin(), order.end(), 0);
    auto tile_cost = [&](int32_t f) {
        const FrameRec& F = p->frames[f];
        const int64_t bpp = F.layout == DPPIX_F32_CHW ? 4 : 1;
        return (int64_t)F.b * F.K * F.b * F.C * bpp;
    };
    // group-major (one kernel instantiation per layout and channel count, one
    // launch per workgroup size)
    auto group_key = [&](int32_t f) {
        const FrameRec& F = p->frames[f];
        return (F.layout * 8 + F.C) * 2 + (tile_threads(F) == kDefaultThreads ? 0 : 1);
    };
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        if (group_key(x) != group_key(y))
            return group_key(x) < group_key(y);
        return tile_cost(x) > tile_cost(y);
    });
    p->sched_frame = order;
    p->sched_base.resize(n_frames + 1);
    int64_t acc = 0;
    for (int32_t k = 0; k < n_frames; ++k) {
        p->sched_base[k] = acc;
        const FrameRec& F = p->frames[order[k]];
        acc += (int64_t)F.GR * F.TX;
    }
    p->sched_base[n_frames] = acc;
    for (int32_t k = 0; k < n_frames; ++k) {
        const FrameRec& F = p->frames[order[k]];
        const int th = tile_threads(F);
        if (p->groups.empty() || p->groups.back().layout != F.layout || p->groups.back().C != F.C ||
            p->groups.back().threads != th)
            p->groups.push_back(LaunchGroup{F.layout, F.C, th, p->sched_base[k], p->sched_base[k], 0, 0});
        LaunchGroup& g = p->groups.back();
        g.hi = p->sched_base[k + 1];
        g.lds_fwd = std::max(g.lds_fwd, frame_lds(kind_fwd(F), F));
        g.lds_rec = std::max(g.lds_rec, frame_lds(kind_rec(F), F));
    }

    if (p->groups.size() > (size_t)kMaxGroups) {   // 2 layouts x 4 channel counts x 2 sizes at most
        delete p;
        return fail(DPPIX_ENOTSUP, "too many launch groups");
    }

    // Workspace layout.
    WsLayout& w = p->ws;
    size_t o = 0;
    w.frames = o;      o = align256(o + sizeof(FrameRec) * n_frames);
    w.tile_map = o;    o = align256(o + sizeof(int32_t) * 2 * (size_t)p->n_tiles);
    w.unit_map = o;    o = align256(o + sizeof(int32_t) * 2 * (size_t)p->n_units);
    // Tiles of the adjoint's mirror pass: those holding a real pixel that a
    // padded row or column folds onto (the same test the kernel applies).
    std::vector<int32_t> border;
    for (int32_t f = 0; f < n_frames; ++f) {
        const FrameRec& F = p->frames[f];
        if (F.pad == DPPIX_PAD_NONE)
            continue;
        const int PR = F.GR * F.b - F.H, PC = F.GC * F.b - F.W;
        const int lo_r = PR > 0 ? (PR <= F.H - 1 ? F.H - 1 - PR : 0) : F.H;
        const int lo_c = PC > 0 ? (PC <= F.W - 1 ? F.W - 1 - PC : 0) : F.W;
        for (int32_t r = 0; r < F.GR; ++r)
            for (int32_t ct = 0; ct < F.TX; ++ct) {
                const int x0c = ct * F.K, Kt = std::min(F.K, F.GC - x0c);
                const int y0 = r * F.b, y1 = std::min(y0 + F.b, F.H);
                const int xa = x0c * F.b, xb = std::min((x0c + Kt) * F.b, F.W);
                if (y0 >= F.H || xa >= F.W || (y1 <= lo_r && xb <= lo_c))
                    continue;
                border.push_back(f);
                border.push_back(r * F.TX + ct);
            }
    }
    p->n_border = (int64_t)border.size() / 2;
    w.border_map = o;  o = align256(o + sizeof(int32_t) * border.size());
    w.simple_counts = o; o = align256(o + sizeof(uint64_t) * 4 * (size_t)n_frames);
    w.total = o;
    // Per-call state carried by each store.
    StateLayout& sl = p->st;
    o = 0;
    sl.tile_cnt = o;   o = align256(o + sizeof(uint32_t) * (size_t)p->n_tiles);
    sl.tile_fg = o;    o = align256(o + sizeof(uint32_t) * (size_t)p->n_tiles);
    sl.counters = o;   o = align256(o + sizeof(uint32_t) * kTicketWords);
    sl.total = o;

    // Host image of the tables: frame records, and per scheduling index the
    // frame and the tile within it.
    p->host_tables.assign(w.total, 0);
    std::memcpy(p->host_tables.data() + w.frames, p->frames.data(), sizeof(FrameRec) * n_frames);
    int32_t* map = reinterpret_cast<int32_t*>(p->host_tables.data() + w.tile_map);
    for (int32_t k = 0; k < n_frames; ++k)
        for (int64_t i = p->sched_base[k]; i < p->sched_base[k + 1]; ++i) {
            map[2 * i] = order[k];
            map[2 * i + 1] = (int32_t)(i - p->sched_base[k]);
        }
    for (const LaunchGroup& g : p->groups)
        xcd_runs(map, g.lo, g.hi);
    if (!border.empty())
        std::memcpy(p->host_tables.data() + w.border_map, border.data(), sizeof(int32_t) * border.size());
    {
        // without masks every cell is simple: n_bg = cells, n_fg = 0, and the
        // frames' statistics packed back to back in batch order
        uint64_t* sc = reinterpret_cast<uint64_t*>(p->host_tables.data() + w.simple_counts);
        uint64_t bg_off = 0;
        for (int32_t f = 0; f < n_frames; ++f) {
            const FrameRec& F = p->frames[f];
            const uint64_t cells = (uint64_t)F.GR * (uint64_t)F.GC;
            sc[4 * f + 0] = cells;
            sc[4 * f + 1] = 0;
            sc[4 * f + 2] = bg_off;
            sc[4 * f + 3] = 0;
            bg_off += cells * (uint64_t)F.C;
        }
    }
    int32_t* umap = reinterpret_cast<int32_t*>(p->host_tables.data() + w.unit_map);
    for (int32_t f = 0, u = 0; f < n_frames; ++f)
        for (int32_t i = 0; i < p->frames[f].cunits; ++i, ++u) {
            umap[2 * u] = f;
            umap[2 * u + 1] = i;
        }
    *out = p;
    return DPPIX_OK;
}

void dp_pix_plan_destroy(dppix_plan_t p) { delete p; }

dppix_status_t dp_pix_plan_sizes(dppix_plan_t p, dppix_sizes_t* out)
{
    if (p == nullptr || out == nullptr)
        return fail(DPPIX_EINVAL, "NULL plan or output");
    out->workspace_bytes = p->ws.total;
    out->store_state_bytes = p->st.total;
    out->bg_capacity = p->bg_cap;
    out->fg_capacity = p->fg_cap;
    out->flag_bytes = (size_t)p->total_cells;
    out->clip_bytes_bg = p->bg_cap;
    out->clip_bytes_fg = p->fg_cap;
    out->grad_scratch_bytes = grad_scratch_need(p);
    out->metrics_scratch_bytes = align256(16 * (size_t)p->n_tiles);
    out->n_tiles = p->n_tiles;
    out->total_pixels = p->total_pixels;
    out->forward_launches = (int64_t)p->groups.size();
    return DPPIX_OK;
}

dppix_status_t dp_pix_plan_frame_info(dppix_plan_t p, int32_t f, dppix_frame_info_t* out)
{
    if (p == nullptr || out == nullptr)
        return fail(DPPIX_EINVAL, "NULL plan or output");
    if (f < 0 || f >= (int32_t)p->frames.size())
        return fail(DPPIX_EINVAL, "frame index out of range");
    const FrameRec& F = p->frames[f];
    out->grid_rows = F.GR;
    out->grid_cols = F.GC;
    out->n = F.n;
    out->pad_rows = F.GR * F.b - F.H;
    out->pad_cols = F.GC * F.b - F.W;
    out->tile_cells = F.K;
    out->tiles_per_band = F.TX;
    out->fg_min_count = F.tau;
    out->cell_offset = F.cell_base;
    out->fine_offset = F.fine_base;
    out->sigma_bg = F.sigma_bg;
    out->sigma_fg = F.sigma_fg;
    return DPPIX_OK;
}

dppix_status_t dp_pix_plan_set_launch(dppix_plan_t p, int32_t threads, int32_t persistent)
{
    if (p == nullptr)
        return fail(DPPIX_EINVAL, "NULL plan");
    if (threads != 0 && (threads < 64 || threads > kMaxThreads || threads % 64 != 0))
        return fail(DPPIX_EINVAL, "threads must be 0 (chosen per frame class) or a multiple of 64 in 64..512");
    if (persistent < 0 || persistent > 64)
        return fail(DPPIX_EINVAL, "persistent must be 0 (one workgroup per tile), 1 (resident grid) or 2..64 "
                                  "(workgroups per CU)");
    p->threads = threads;
    p->persistent = persistent;
    return DPPIX_OK;
}

dppix_status_t dp_pix_plan_bind(dppix_plan_t p, void* ws, size_t bytes, dppix_stream_t stream)
{
    if (p == nullptr || ws == nullptr)
        return fail(DPPIX_EINVAL, "NULL plan or workspace");
    if (p->bound != nullptr)
        return fail(DPPIX_EINVAL, "plan is already bound (its tables are immutable once uploaded)");
    if (bytes < p->ws.total)
        return fail(DPPIX_ENOMEM, "workspace smaller than workspace_bytes");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(DPPIX_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(ws, p->host_tables.data(), p->host_tables.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
        return dev_fail(e, "uploading plan tables");
    // the tables are on the device when bind returns, so calls on any stream
    // may use the plan from then on
    e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return dev_fail(e, "uploading plan tables");
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
        p->cus = n;
    else
        p->cus = 256;
    p->bound = static_cast<uint8_t*>(ws);
    p->bound_bytes = bytes;
    return DPPIX_OK;
}

dppix_status_t dp_pix_plan_workspace_size(const dppix_frame_desc_t* descs, int32_t n_frames, dppix_sizes_t* out)
{
    if (out == nullptr)
        return fail(DPPIX_EINVAL, "out is NULL");
    dppix_plan_t p = nullptr;
    dppix_status_t st = dp_pix_plan_create(descs, n_frames, &p);
    if (st != DPPIX_OK)
        return st;
    st = dp_pix_plan_sizes(p, out);
    dp_pix_plan_destroy(p);
    return st;
}

}  // extern "C"

namespace {

// Kernel arguments of one call: the plan's tables, and the per-call state
// (flags, counts, tile counts and prefixes, tickets) of the call's store.
TileArgs base_args(dppix_plan_t p, const dppix_store_t* store)
{
    TileArgs a;
    std::memset(&a, 0, sizeof a);
    uint8_t* w = p->bound;
    a.frames = reinterpret_cast<const FrameRec*>(w + p->ws.frames);
    a.tile_map = reinterpret_cast<const int32_t*>(w + p->ws.tile_map);
    a.n_frames = (int32_t)p->frames.size();
    a.n_tiles = p->n_tiles;
    a.unit_map = reinterpret_cast<const int32_t*>(w + p->ws.unit_map);
    a.simple_counts = reinterpret_cast<const uint64_t*>(w + p->ws.simple_counts);
    a.total_cells = p->total_cells;
    a.persistent = p->persistent;
    if (store != nullptr) {
        uint8_t* st = static_cast<uint8_t*>(store->state);
        a.flags = store->flags;
        a.counts = store->counts;
        a.bg = store->bg;
        a.fg = store->fg;
        a.tile_cnt = reinterpret_cast<uint32_t*>(st + p->st.tile_cnt);
        a.tile_fg = reinterpret_cast<uint32_t*>(st + p->st.tile_fg);
        a.ticket = reinterpret_cast<uint32_t*>(st + p->st.counters);
        a.noise = store->noise;
    }
    return a;
}

dppix_status_t need_bound(dppix_plan_t p)
{
    if (p == nullptr)
        return fail(DPPIX_EINVAL, "NULL plan");
    if (p->bound == nullptr)
        return fail(DPPIX_EINVAL, "plan has no workspace (call dp_pix_plan_bind)");
    return DPPIX_OK;
}

// Every call that takes a store needs its layout (flags, counts) and its
// per-call state; need_stats: also the statistics arrays.
dppix_status_t check_store(const dppix_store_t* s, bool need_stats)
{
    if (s == nullptr)
        return fail(DPPIX_EINVAL, "NULL store");
    if (s->flags == nullptr || s->counts == nullptr || s->state == nullptr)
        return fail(DPPIX_EINVAL, "store flags, counts and state are required");
    if ((reinterpret_cast<uintptr_t>(s->state) & 255) != 0)
        return fail(DPPIX_EINVAL, "store state must be 256-byte aligned");
    if ((reinterpret_cast<uintptr_t>(s->counts) & 7) != 0)
        return fail(DPPIX_EINVAL, "store counts must be 8-byte aligned");
    if ((reinterpret_cast<uintptr_t>(s->noise) & 7) != 0)
        return fail(DPPIX_EINVAL, "store noise counters must be 8-byte aligned");
    if (need_stats && (s->bg == nullptr || s->fg == nullptr))
        return fail(DPPIX_EINVAL, "store bg/fg are NULL");
    return DPPIX_OK;
}

// Workgroup size of the kernels outside the launch groups.
int plain_threads(dppix_plan_t p) { return p->threads ? p->threads : kDefaultThreads; }

// Workgroup size of a launch group's forward and reconstruction tiles.
int group_threads(dppix_plan_t p, const LaunchGroup& g) { return p->threads ? p->threads : g.threads; }

int grid_for(dppix_plan_t p, int layout, int C, int threads, int64_t tiles, size_t lds)
{
    if (!p->persistent)
        return (int)tiles;
    const int cus = p->cus > 0 ? p->cus : 256;
    int per_cu = p->persistent;
    if (per_cu == 1 && (occupancy_forward(layout, C, threads, lds, &per_cu) != hipSuccess || per_cu < 1))
        per_cu = 1;
    const int64_t g = std::min<int64_t>((int64_t)cus * per_cu, tiles);
    return (int)std::max<int64_t>(1, g);
}

// One launch per group: its scheduling range and its own ticket pair.
template <typename Launch>
hipError_t for_groups(dppix_plan_t p, const TileArgs& base, bool rec, Launch launch)
{
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        const LaunchGroup& g = p->groups[gi];
        TileArgs a = base;
        a.sched_offset = g.lo;
        a.n_tiles = g.hi - g.lo;
        a.ticket = base.ticket + 2 * gi;
        const size_t lds = rec ? g.lds_rec : g.lds_fwd;
        hipError_t e = launch(a, g, lds, grid_for(p, g.layout, g.C, group_threads(p, g), a.n_tiles, lds));
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// Scratch of dp_pix_backward: gradient of every statistic (bg, fg in store
// order) and the class-local index of every grid cell.
size_t grad_scratch_need(dppix_plan_t p)
{
    return align256(4 * p->bg_cap) + align256(4 * p->fg_cap) + align256(4 * (size_t)p->total_cells);
}

dppix_status_t check_backward(dppix_plan_t p, const dppix_store_t* store, const float* const* grad_out,
                              const uint8_t* clip_bg, const uint8_t* clip_fg, float* const* grad_in)
{
    dppix_status_t st = need_bound(p);
    if (st != DPPIX_OK)
        return st;
    if (p->any_u8)
        return fail(DPPIX_EINVAL, "backward needs every frame in F32_CHW layout");
    if (grad_out == nullptr || grad_in == nullptr || clip_bg == nullptr || clip_fg == nullptr)
        return fail(DPPIX_EINVAL, "grad_out, grad_in and clip bits are required");
    return check_store(store, true);
}

dppix_status_t run_backward(dppix_plan_t p, const dppix_store_t* store, const float* const* grad_out,
                            const uint8_t* clip_bg, const uint8_t* clip_fg, float* const* grad_in, uint8_t* sc,
                            dppix_stream_t stream);

// Fixed device scratch of dp_pix_backward_static, for callers that cannot
// allocate.  Each device holds its own copy of the array from the library's
// load until the process ends.  In host code `scratch` names a host-side
// stand-in: kernels get the device address that hipGetSymbolAddress returns
// for the current device, looked up once per device and kept.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
std::vector<uint8_t*> g_scratch_ptr;  // per device; nullptr until looked up

dppix_status_t static_scratch(uint8_t** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return dev_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((size_t)dev >= g_scratch_ptr.size())
        g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (g_scratch_ptr[dev] == nullptr) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return dev_fail(e, "hipGetSymbolAddress(scratch)");
        if (ptr == nullptr || (reinterpret_cast<uintptr_t>(ptr) & 255) != 0)
            return fail(DPPIX_EDEVICE, "device scratch has no 256-byte aligned address");
        g_scratch_ptr[dev] = static_cast<uint8_t*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return DPPIX_OK;
}

}  // namespace

extern "C" {

dppix_status_t dp_pix_plan(dppix_plan_t p, const uint8_t* const* masks, const dppix_store_t* store,
                           dppix_stream_t stream)
{
    dppix_status_t st = need_bound(p);
    if (st != DPPIX_OK)
        return st;
    if ((st = check_store(store, false)) != DPPIX_OK)
        return st;
    TileArgs a = base_args(p, store);
    a.masks = masks;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = launch_plan(a, p->n_units, plain_threads(p), p->lds[kPlan], p->prefix_scan, s);
    if (e != hipSuccess)
        return dev_fail(e, "plan launch");
    return DPPIX_OK;
}

dppix_status_t dp_pix_plan_labels(dppix_plan_t p, const void* const* images, int32_t threshold,
                                  const dppix_store_t* store, dppix_stream_t stream)
{
    dppix_status_t st = need_bound(p);
    if (st != DPPIX_OK)
        return st;
    if (p->any_f32)
        return fail(DPPIX_EINVAL, "labels are computed from U8_HWC frames");
    if (images == nullptr)
        return fail(DPPIX_EINVAL, "images is NULL");
    if (threshold < 0 || threshold > 4 * 1024)
        return fail(DPPIX_EINVAL, "threshold must be in 0..4096");
    if ((st = check_store(store, false)) != DPPIX_OK)
        return st;
    TileArgs a = base_args(p, store);
    a.images = images;
    a.edge_threshold = threshold;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned channel_mask = 0;
    for (const FrameRec& F : p->frames)
        channel_mask |= 1u << F.C;
    hipError_t e = launch_plan_labels(a, p->n_units, plain_threads(p), p->lds[kPlan], channel_mask, p->prefix_scan, s);
    if (e != hipSuccess)
        return dev_fail(e, "plan launch");
    return DPPIX_OK;
}

dppix_status_t dp_pix_store_index(dppix_plan_t p, const dppix_store_t* store, dppix_stream_t stream)
{
    dppix_status_t st = need_bound(p);
    if (st != DPPIX_OK)
        return st;
    if ((st = check_store(store, false)) != DPPIX_OK)
        return st;
    TileArgs a = base_args(p, store);
    hipError_t e = launch_store_index(a, p->prefix_scan, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return dev_fail(e, "store index launch");
    return DPPIX_OK;
}

dppix_status_t dp_pix_forward(dppix_plan_t p, const void* const* images, const dppix_store_t* store,
                              uint8_t* clip_bg, uint8_t* clip_fg, void* const* fused_out, dppix_stream_t stream)
{
    dppix_status_t st = need_bound(p);
    if (st != DPPIX_OK)
        return st;
    if (images == nullptr)
        return fail(DPPIX_EINVAL, "images is NULL");
    if ((st = check_store(store, true)) != DPPIX_OK)
        return st;
    if ((clip_bg == nullptr) != (clip_fg == nullptr))
        return fail(DPPIX_EINVAL, "clip_bg and clip_fg must both be given or both be NULL");
    TileArgs a = base_args(p, store);
    a.images = images;
    a.outs = fused_out;
    a.clip_bg = clip_bg;
    a.clip_fg = clip_fg;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = for_groups(p, a, false, [&](const TileArgs& ga, const LaunchGroup& g, size_t lds, int grid) {
        return launch_forward(ga, g.layout, g.C, group_threads(p, g), lds, grid, s);
    });
    if (e != hipSuccess)
        return dev_fail(e, "forward launch");
    return DPPIX_OK;
}

dppix_status_t dp_pix_reconstruct(dppix_plan_t p, const dppix_store_t* store, void* const* out, dppix_stream_t stream)
{
    dppix_status_t st = need_bound(p);
    if (st != DPPIX_OK)
        return st;
    if (out == nullptr)
        return fail(DPPIX_EINVAL, "out is NULL");
    if ((st = check_store(store, true)) != DPPIX_OK)
        return st;
    TileArgs a = base_args(p, store);
    a.outs = out;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = for_groups(p, a, true, [&](const TileArgs& ga, const LaunchGroup& g, size_t lds, int grid) {
        return launch_reconstruct(ga, g.layout, g.C, group_threads(p, g), lds, grid, s);
    });
    if (e != hipSuccess)
        return dev_fail(e, "reconstruct launch");
    return DPPIX_OK;
}

dppix_status_t dp_pix_backward(dppix_plan_t p, const dppix_store_t* store, const float* const* grad_out,
                               const uint8_t* clip_bg, const uint8_t* clip_fg, float* const* grad_in, void* scratch,
                               size_t scratch_bytes, dppix_stream_t stream)
{
    dppix_status_t st = check_backward(p, store, grad_out, clip_bg, clip_fg, grad_in);
    if (st != DPPIX_OK)
        return st;
    if (scratch == nullptr || scratch_bytes < grad_scratch_need(p))
        return fail(DPPIX_ENOMEM, "scratch smaller than grad_scratch_bytes");
    return run_backward(p, store, grad_out, clip_bg, clip_fg, grad_in, static_cast<uint8_t*>(scratch), stream);
}

dppix_status_t dp_pix_backward_static(dppix_plan_t p, const dppix_store_t* store, const float* const* grad_out,
                                      const uint8_t* clip_bg, const uint8_t* clip_fg, float* const* grad_in,
                                      dppix_stream_t stream)
{
    dppix_status_t st = check_backward(p, store, grad_out, clip_bg, clip_fg, grad_in);
    if (st != DPPIX_OK)
        return st;
    if (grad_scratch_need(p) > kStaticScratchBytes)
        return fail(DPPIX_ENOMEM, "backward needs " + std::to_string(grad_scratch_need(p)) +
                                      " bytes of scratch; the fixed device scratch holds " +
                                      std::to_string(kStaticScratchBytes) + " (use dp_pix_backward)");
    uint8_t* sc = nullptr;
    if ((st = static_scratch(&sc)) != DPPIX_OK)
        return st;
    return run_backward(p, store, grad_out, clip_bg, clip_fg, grad_in, sc, stream);
}

}  // extern "C"

namespace {

dppix_status_t run_backward(dppix_plan_t p, const dppix_store_t* store, const float* const* grad_out,
                            const uint8_t* clip_bg, const uint8_t* clip_fg, float* const* grad_in, uint8_t* sc,
                            dppix_stream_t stream)
{
    TileArgs a = base_args(p, store);
    a.grad_out = grad_out;
    a.grad_in = grad_in;
    a.clip_bg = const_cast<uint8_t*>(clip_bg);
    a.clip_fg = const_cast<uint8_t*>(clip_fg);
    a.g_bg = reinterpret_cast<float*>(sc);
    a.g_fg = reinterpret_cast<float*>(sc + align256(4 * p->bg_cap));
    a.cell_index = reinterpret_cast<uint32_t*>(sc + align256(4 * p->bg_cap) + align256(4 * p->fg_cap));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // 1. gradient of every statistic (store layout): pass * sum of grad_out
    // over its real pixels / area, broadcast in the same tile to the real
    // pixels of the statistic (grad_in)
    hipError_t e = launch_backward_reduce(a, plain_threads(p), p->lds[kBwd],
                                          grid_for(p, 1, 1, plain_threads(p), p->n_tiles, p->lds[kBwd]), s);
    if (e != hipSuccess)
        return dev_fail(e, "backward launch");
    // 2. mirror terms of the pixels near padded borders: only the border
    // tiles, and no launch at all when no frame is padded
    if (p->n_border > 0) {
        TileArgs m = a;
        m.tile_map = reinterpret_cast<const int32_t*>(p->bound + p->ws.border_map);
        m.n_tiles = p->n_border;
        e = launch_backward_mirror(m, plain_threads(p), grid_for(p, 1, 1, plain_threads(p), p->n_border, 0), s);
        if (e != hipSuccess)
            return dev_fail(e, "backward launch");
    }
    return DPPIX_OK;
}

}  // namespace

extern "C" {

dppix_status_t dp_pix_debug_sums(dppix_plan_t p, const void* const* images, const dppix_store_t* store,
                                 uint32_t* coarse, uint32_t* fine, dppix_stream_t stream)
{
    dppix_status_t st = need_bound(p);
    if (st != DPPIX_OK)
        return st;
    if (p->any_f32)
        return fail(DPPIX_EINVAL, "debug sums are for U8_HWC frames");
    if (images == nullptr || coarse == nullptr || fine == nullptr)
        return fail(DPPIX_EINVAL, "images, coarse and fine are required");
    if ((st = check_store(store, true)) != DPPIX_OK)
        return st;
    TileArgs a = base_args(p, store);
    a.images = images;
    a.dbg_coarse = coarse;
    a.dbg_fine = fine;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = for_groups(p, a, false, [&](const TileArgs& ga, const LaunchGroup& g, size_t lds, int grid) {
        return launch_forward(ga, g.layout, g.C, group_threads(p, g), lds, grid, s);
    });
    if (e != hipSuccess)
        return dev_fail(e, "forward launch");
    return DPPIX_OK;
}

dppix_status_t dp_pix_edge_mask(dppix_plan_t p, const void* const* images, int32_t threshold, uint8_t* const* masks_out,
                                dppix_stream_t stream)
{
    dppix_status_t st = need_bound(p);
    if (st != DPPIX_OK)
        return st;
    if (p->any_f32)
        return fail(DPPIX_EINVAL, "edge masks are computed from U8_HWC frames");
    if (images == nullptr || masks_out == nullptr)
        return fail(DPPIX_EINVAL, "images and masks_out are required");
    if (threshold < 0 || threshold > 4 * 1024)
        return fail(DPPIX_EINVAL, "threshold must be in 0..4096");
    TileArgs a = base_args(p, nullptr);
    a.images = images;
    a.masks_out = masks_out;
    a.edge_threshold = threshold;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (const LaunchGroup& g : p->groups) {
        TileArgs ga = a;
        ga.sched_offset = g.lo;
        ga.n_tiles = g.hi - g.lo;
        hipError_t e = launch_edge_mask(ga, g.C, plain_threads(p), s);
        if (e != hipSuccess)
            return dev_fail(e, "edge mask launch");
    }
    return DPPIX_OK;
}

dppix_status_t dp_pix_metrics(dppix_plan_t p, const void* const* images, const void* const* recons, void* scratch,
                              size_t scratch_bytes, double* out, dppix_stream_t stream)
{
    dppix_status_t st = need_bound(p);
    if (st != DPPIX_OK)
        return st;
    if (p->any_f32)
        return fail(DPPIX_EINVAL, "metrics are computed on U8_HWC frames");
    if (images == nullptr || recons == nullptr || out == nullptr)
        return fail(DPPIX_EINVAL, "images, recons and out are required");
    if (scratch == nullptr || scratch_bytes < (size_t)(16 * p->n_tiles))
        return fail(DPPIX_ENOMEM, "scratch smaller than metrics_scratch_bytes");
    TileArgs a = base_args(p, nullptr);
    a.images = images;
    a.outs = const_cast<void* const*>(recons);
    a.met_partial = static_cast<double*>(scratch);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (const LaunchGroup& g : p->groups) {
        TileArgs ga = a;
        ga.sched_offset = g.lo;
        ga.n_tiles = g.hi - g.lo;
        hipError_t e = launch_metrics(ga, g.C, plain_threads(p), s);
        if (e != hipSuccess)
            return dev_fail(e, "metrics launch");
    }
    hipError_t e = launch_metrics_reduce(a, out, s);
    if (e != hipSuccess)
        return dev_fail(e, "metrics reduce launch");
    return DPPIX_OK;
}

dppix_status_t dp_pix_noise_advance(uint64_t* noise, int32_t n_frames, uint64_t step, dppix_stream_t stream)
{
    if (n_frames < 0 || (n_frames > 0 && noise == nullptr))
        return fail(DPPIX_EINVAL, "noise must hold n_frames >= 0 counter pairs");
    if ((reinterpret_cast<uintptr_t>(noise) & 7) != 0)
        return fail(DPPIX_EINVAL, "noise must be 8-byte aligned");
    hipError_t e = launch_noise_advance(noise, n_frames, step, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return dev_fail(e, "noise advance launch");
    return DPPIX_OK;
}

dppix_status_t dp_pix_debug_philox(const uint32_t* in, uint32_t* words, int64_t n, dppix_stream_t stream)
{
    if (n < 0 || (n > 0 && (in == nullptr || words == nullptr)))
        return fail(DPPIX_EINVAL, "bad philox arguments");
    hipError_t e = launch_philox(in, words, n, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return dev_fail(e, "philox launch");
    return DPPIX_OK;
}

dppix_status_t dp_pix_graph_create(dppix_plan_t p, const uint8_t* const* masks, const void* const* images,
                                   const dppix_store_t* store, void* const* fused_out, dppix_stream_t stream,
                                   dppix_graph_t* out)
{
    if (out == nullptr)
        return fail(DPPIX_EINVAL, "out is NULL");
    *out = nullptr;
    dppix_status_t st = need_bound(p);
    if (st != DPPIX_OK)
        return st;
    if (images == nullptr || (st = check_store(store, true)) != DPPIX_OK)
        return st == DPPIX_OK ? fail(DPPIX_EINVAL, "images is NULL") : st;
    // The legacy default stream cannot be captured; capture on a private
    // non-blocking stream instead (the graph does not depend on it).
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipStream_t own = nullptr;
    if (s == nullptr) {
        hipError_t ec = hipStreamCreateWithFlags(&own, hipStreamNonBlocking);
        if (ec != hipSuccess)
            return dev_fail(ec, "capture stream");
        s = own;
    }
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        if (own)
            (void)hipStreamDestroy(own);
        return dev_fail(e, "begin capture");
    }
    dppix_stream_t cs = reinterpret_cast<dppix_stream_t>(s);
    dppix_status_t s1 = dp_pix_plan(p, masks, store, cs);
    dppix_status_t s2 = s1 == DPPIX_OK ? dp_pix_forward(p, images, store, nullptr, nullptr, fused_out, cs) : s1;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (own)
        (void)hipStreamDestroy(own);
    if (s2 != DPPIX_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return s2;
    }
    if (e != hipSuccess)
        return dev_fail(e, "end capture");
    dppix_graph* G = new (std::nothrow) dppix_graph;
    if (G == nullptr) {
        (void)hipGraphDestroy(g);
        return fail(DPPIX_ENOMEM, "host allocation failed");
    }
    G->graph = g;
    e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete G;
        return dev_fail(e, "graph instantiate");
    }
    *out = G;
    return DPPIX_OK;
}

dppix_status_t dp_pix_graph_launch(dppix_graph_t g, dppix_stream_t stream)
{
    if (g == nullptr)
        return fail(DPPIX_EINVAL, "NULL graph");
    hipError_t e = hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return dev_fail(e, "graph launch");
    return DPPIX_OK;
}

void dp_pix_graph_destroy(dppix_graph_t g)
{
    if (g == nullptr)
        return;
    if (g->exec)
        (void)hipGraphExecDestroy(g->exec);
    if (g->graph)
        (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
