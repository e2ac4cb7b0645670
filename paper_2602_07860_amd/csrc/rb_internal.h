// Internal plan shared by the host entry points (rb_api.cpp) and the kernels
// (rb_kernels.hip).  Not part of the public ABI.
#pragma once
#include <cstddef>
#include <algorithm>
#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

#include "motion_blur_raster.h"

namespace rb {

// A tile is tw x th = 64 pixels, one 64-lane wave (lane = th-row * tw + column):
// 8 x 8 by default, 16 x 4 or 4 x 16 on request
constexpr int kWave = 64;
constexpr int kTileWDefault = 8;
constexpr int kMaxTileH = 16;          // rows of the tallest tile shape (4 x 16)
constexpr float kTauDet = 1e-10f;         // |det F(tau)| at or below this: face skipped
constexpr double kTauDetBin = 1e-10;      // the same rule in double, applied when the lists are built
// background adjoint: a term whose weight prod_{m != j}(1 - A_m) A_j is below
// this is left out, and so is a whole (pixel, sub-frame) where the bound
// prod_m (1 - A_m) / min(min_m (1 - A_m), 1/2) on its weights is (the FP64
// reference with the same rule: the vertex gradient moves by ~1e-6)
constexpr float kAdjWMin = 1e-8f;
constexpr int kHdrFaceRange = 1, kHdrBehind = 2, kHdrOverflow = 4, kHdrDetRange = 8;
// deterministic mode: one background task per (chunk, tile) (lists hold
// distinct faces, fewer than RB_MAX_FACES < this)
constexpr int kDetSliceLen = 1 << 24;

// First sub-frame of segment s: the smallest k with floor(k S / (K-1)) >= s,
// i.e. sub-frame t_k = k/(K-1) falls in segment min(floor(t_k S), S-1).
__host__ __device__ inline int seg_first(int s, int K, int S)
{
    if (K <= 1) return s == 0 ? 0 : 1;
    if (s <= 0) return 0;
    long long num = (long long)s * (K - 1);
    return (int)((num + S - 1) / S);
}

// Chunk c = s * CPS + j: the j-th of CPS near-equal runs of segment s's
// sub-frames [k0, k0 + n).
struct Chunk {
    int s, k0, n;
};

__host__ __device__ inline Chunk chunk_info(int c, int K, int S, int CPS)
{
    int s = c / CPS, j = c - s * CPS;
    int klo = seg_first(s, K, S);
    int khi = (s == S - 1) ? K : seg_first(s + 1, K, S);
    int n = khi - klo;
    Chunk ch;
    ch.s = s;
    // j * n <= CPS * K < 2^31 (checked when the plan is made)
    ch.k0 = klo + (j * n) / CPS;
    ch.n = klo + ((j + 1) * n) / CPS - ch.k0;
    return ch;
}

// Per-instance workspace header as laid out on the device (first 256 bytes).
struct DevHeader {
    int32_t error_bits;
    int32_t reserved;
    int64_t list_entries;
    int64_t list_capacity;
    int64_t ntasks;       // background tasks of the current forward
    unsigned long long bwd_task_ctr;   // next background-adjoint task
    uint32_t gmax;        // deterministic mode: bits of max |dL/dI| (non-negative floats order as integers)
    int32_t pad32;
    int64_t pad[2];
};

// The device pass sees an instance's buffers as global-memory pointers, so
// that its loads, stores and atomics compile to global (not flat)
// instructions; the host pass sees plain pointers of the same size.
#if defined(__HIP_DEVICE_COMPILE__)
#define RB_G __attribute__((address_space(1)))
#else
#define RB_G
#endif

struct ViewArgs {
    float m[12];
    float tanf;
};

// One instance as the kernels see it (device memory, written at the start of
// every call).  Every kernel covers all instances of a batch; b_* is the first
// block of this instance in the launch of that kernel.
struct Inst {
    // caller's arrays
    const float RB_G *verts;
    const int32_t RB_G *faces;
    const float RB_G *attrs;
    const float RB_G *model;
    float RB_G *image;
    const float RB_G *grad_image;
    float RB_G *grad_verts;
    float RB_G *grad_attrs;
    // workspace
    DevHeader RB_G *hdr;
    double2 RB_G *kf;         // [S+1][V] keyframe (x, y), kept in double: edge-on (sliver)
                         // faces make barycentrics sensitive to 1e-8 position errors
    float RB_G *kfz;          // [S+1][V] keyframe camera depth
    int32_t RB_G *cnt;        // [2][NC][ntiles] list lengths (fg, bg)
    int64_t RB_G *off;        // [2][NC][ntiles] list starts
    int32_t RB_G *cur;        // [2][NC][ntiles] fill cursors
    int64_t RB_G *bsum;       // scan block sums
    uint32_t RB_G *list;      // entries: face << 8 | sub-frame mask
    int32_t RB_G *vis_id;     // [ntiles][K][64] winner face; -1 uncovered; -4 outside the image
    float RB_G *pix;          // [ntiles][K][NS][64] winner colour, or (sum log2(1 - A), #zero factors, min 1 - A)
    int32_t RB_G *tsl;        // [NC][ntiles] background tasks (list slices) per (chunk, tile)
    int64_t RB_G *toff;       // [NC][ntiles] first task
    int64_t RB_G *tbsum;      // task scan block sums
    uint64_t RB_G *tasks;     // (chunk * ntiles + tile) << 32 | slice
    float RB_G *gkf;          // [S+1][V][2] keyframe gradient
    int32_t RB_G *fgw;        // [NC * ntiles] 1 where the (chunk, tile) has a winner
    int64_t RB_G *gfx;        // deterministic mode: [S+1][V][2] then [V][C] gradient sums in fixed point
    // sizes
    int V, F, C, S, K, W, H, tiles_x, tiles_y, ntiles;
    int tw, th, lw, lh;  // tile width and height in pixels and their log2
    uint64_t rep;        // bit 0 of every tile row: sum over rows r of 2^(tw r)
    int CPS, NC, SL, NS, nfb;
    int seq_bg;          // consecutive items per lane in the background adjoint
    int fgg;             // chunks per wave (at most) in the foreground adjoint
    int bwd_merge;       // background tasks per unit of the background adjoint
    int ntct;            // (chunk, tile) pairs = NC * ntiles
    int det;             // RB_FLAG_DETERMINISTIC
    int nblocks_scan, nblocks_tscan;
    int64_t cap, maxtasks, ncounts;
    float inv_w, inv_h, dmax, halo, neg_log2e_over_delta, inv_delta, invK;
    ViewArgs vw;
    // first block of this instance in each launch
    int b_init, b_proj, b_bin, b_scan1, b_scan3, b_tscan1, b_tscan3, b_fg, b_fgb, b_res, b_bwdinit, b_vtx,
        b_sort, b_detp;
};

// Host plan of one instance.
struct Plan {
    int V, F, C, S, K, W, H;
    float tanf, delta, dmax, halo;
    float view[12];
    int solver;
    int tiles_x, tiles_y, ntiles;
    int tw, th;     // tile shape (pixels)
    int T;          // chunk length (template)
    int CPS;        // chunks per segment
    int NC;         // chunks = S * CPS
    int SL;         // background list entries per task
    int seq_bg;     // consecutive items per lane in the background adjoint
    int fgg;        // chunks per wave (at most) in the foreground adjoint
    int bwd_merge;  // background tasks per unit of the background adjoint
    bool wide;      // background halo of 12 pixels or more (faces reach many pixels of a tile)
    bool det;       // RB_FLAG_DETERMINISTIC
    int NS;         // per (pixel, sub-frame) value slots: colour, or log-sum, zero count, smallest 1 - A
    int nfb;        // binning blocks per chunk
    int64_t cap;    // list capacity (entries)
    int64_t ntct;   // (chunk, tile) pairs = NC * ntiles
    int64_t maxtasks;
    // workspace byte offsets (from the instance's base)
    size_t o_hdr, o_kf, o_kfz, o_cnt, o_off, o_cur, o_bsum, o_list, o_vis_id, o_pix, o_tsl, o_toff, o_tbsum,
        o_tasks, o_gkf, o_fgw, o_gfx, total;
    int64_t ncounts;  // 2 * NC * ntiles
    int64_t nblocks_scan, nblocks_tscan;
};

// Block counts of each launch over a batch.
struct Grids {
    int64_t init, proj, bin, scan1, scan3, tscan1, tscan3, fg, fgb, res, bwdinit, vtx, sort, detp;
};

// Blocks of one instance in each launch (256-thread blocks unless noted).
inline Grids plan_grids(const Plan &p)
{
    auto div = [](int64_t n, int64_t b) { return (n + b - 1) / b; };
    const int64_t ngrad = (int64_t)(p.S + 1) * p.V * 2 + (int64_t)p.V * p.C;
    Grids g;
    g.init = div(p.ncounts, 256);
    g.proj = div((int64_t)(p.S + 1) * p.V + p.F, 256);
    g.bin = (int64_t)p.NC * p.nfb;
    g.scan1 = p.nblocks_scan;
    g.scan3 = div(p.ncounts, 256);
    g.tscan1 = p.nblocks_tscan;
    g.tscan3 = div(p.ntct, 256);
    g.fg = p.ntct;                                                   // one wave per (chunk, tile)
    g.fgb = (int64_t)p.S * div(p.CPS, p.fgg) * p.ntiles;             // one wave per chunk group and tile
    g.res = p.ntiles;
    g.bwdinit = div(ngrad, 256);                                     // also the deterministic finish
    g.vtx = div(p.V, 256);
    g.sort = p.det ? p.ncounts : 0;                                  // one block per bin list
    g.detp = p.det ? div(std::max<int64_t>(ngrad, (int64_t)(p.C + 1) * p.H * p.W), 256) : 0;
    return g;
}

// Host plan of a batch: per-instance plans and where each instance's
// workspace starts; the table of Inst and the task numbering follow them.
struct Batch {
    int n, T, solver;
    bool det;       // RB_FLAG_DETERMINISTIC (batch-wide: one options record)
    int tw;         // tile width (batch-wide)
    bool wide;      // every instance has a wide halo: background kernels built for long item runs
    std::vector<Plan> plans;
    std::vector<size_t> base;
    Grids g;
    size_t o_table, o_tprefix, total;
};

// Per-instance arrays the host entry points pass in.
struct Io {
    const float *verts;
    const int32_t *faces;
    const float *attrs;
    const float *model;
    float *image;
    const float *grad_image;
    float *grad_verts;
    float *grad_attrs;
};

// Optional phase events (benchmark timing); null entries are skipped.
struct PhaseEvents {
    hipEvent_t ev[6];
};

hipError_t launch_forward(const Batch &bt, const std::vector<Io> &io, void *ws, hipStream_t st, const PhaseEvents *pe);
// device address of the library-held workspace on the current device
// (RB_STATIC_SCRATCH_BYTES), looked up on the first call per device
constexpr int kMaxDevices = 64;
hipError_t static_scratch(void **ptr);
hipError_t launch_backward(const Batch &bt, const std::vector<Io> &io, void *ws, hipStream_t st,
                           const PhaseEvents *pe);

}  // namespace rb
