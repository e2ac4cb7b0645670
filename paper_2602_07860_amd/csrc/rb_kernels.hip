// HIP kernels (gfx950) of the motion-blur differentiable rasterizer and the
// launch sequences of its forward and backward passes.
//
// Every kernel covers all instances of a batch (a single render is a batch of
// one); blocks find their instance in a table written by k_set_table.
//
// Forward (launch_forward):
//   k_init, k_project  clear the workspace's counters; project the S+1
//                      keyframes M_s P0 (App. I), (x, y) in double, depth in
//                      float (a nearly edge-on face's barycentrics move by
//                      position error / height, so float32 keyframes would
//                      cost ~1e-5 of the image).
//   k_bin (x2), k_scan1..3
//                      one thread per (face, chunk of at most T sub-frames of
//                      one segment) takes the face's exact box at each of the
//                      chunk's sub-frames and, for every tile (64 pixels:
//                      8x8, 16x4 or 4x16) the union touches, emits
//                      face << 8 | sub-frame mask into the foreground list
//                      (exact box) and the background list (box grown by the
//                      influence radius), leaving out the sub-frames where
//                      the face is degenerate (|det F| <= 1e-10 in double);
//                      counts and fill ranks go through LDS window counters.
//   k_sort_lists       (deterministic mode) sorts every list into face order.
//   k_fg               one 64-lane wave per (chunk, tile), lane = pixel: list
//                      entries are staged in LDS 32 at a time (anchor-local
//                      float32 records) and dealt out as (entry, pixel)
//                      items; coverage by the fast solver (eq 8: quadratic
//                      numerators per (pixel, face, chunk), Horner per
//                      sub-frame) or the per-sub-frame recompute; an LDS
//                      64-bit z-buffer (depth bits, face) picks the winner,
//                      which is shaded (eq 9); visibility and winner colours
//                      go to the per (pixel, sub-frame) records; the
//                      (chunk, tile)'s background tasks are counted.
//   k_tasks, k_tprefix number the background tasks (slices of a list).
//   k_bg               persistent waves over the background tasks: items of
//                      the uncovered (pixel, sub-frame)s accumulate
//                      log2(1 - A) (eqs 10, 13-15, App. B closest point),
//                      the zero factors and the smallest 1 - A in LDS, then
//                      in the records.
//   k_resolve          mean over the K sub-frames (double).
// Backward (launch_backward):
//   k_bwd_init         clears the keyframe and attribute gradients
//                      (k_det_prep: the fixed-point sums of the
//                      deterministic mode and their scale).
//   k_fg_bwd           one wave per (group of chunks of a segment, tile):
//                      gathers the distinct winners from the visibility,
//                      stages them 16 at a time and runs the shading /
//                      barycentric adjoint into an LDS table keyed by vertex.
//   k_bg_bwd           persistent waves over the background tasks, with a
//                      task counter: re-walks the list slices for the
//                      (pixel, sub-frame)s with gradient (leaving out terms
//                      of negligible weight; faces' boxes are grown per tile
//                      row by how far the row's terms can reach under that
//                      rule, not by the full halo) and runs the
//                      closest-point / barycentric adjoint into the vertex
//                      table.
//   k_det_finish       (deterministic mode) fixed-point sums to float.
//   k_kf_to_vertex     maps keyframe gradients through the projection and
//                      the keyframe transforms to the rest vertices.
// The adjoints deal items to lanes in runs (for_runs) so that a lane adds a
// run's contributions to the vertex table once per (lane, entry).
#include <cfloat>
#include <climits>
#include <cstring>
#include <mutex>

#include "rb_internal.h"

namespace rb {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    // consecutive logical blocks (neighbouring tiles) on the same XCD / L2
    int full = (nb / 8) * 8;
    if (b >= full) return b;
    return (b % 8) * (nb / 8) + b / 8;
}

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// 1 - exp(-x) for x >= 0 without cancellation at small x
__device__ __forceinline__ float one_minus_exp_neg(float x, float A)
{
    if (x < 0.0625f) {
        float t = fmaf(-x, 0.2f, 1.0f);
        t = fmaf(-x * 0.25f, t, 1.0f);
        t = fmaf(-x * (1.0f / 3.0f), t, 1.0f);
        t = fmaf(-x * 0.5f, t, 1.0f);
        return x * t;
    }
    return 1.0f - A;
}

// ------------------------------------------------------------ instances
//
// Every kernel covers all instances of a batch (a single render is a batch
// of one).  Instance i owns the blocks [b_X(i), b_X(i+1)) of launch X; a block
// finds its instance by binary search over the (ascending) starts.

template <int Inst::*B>
__device__ __forceinline__ int inst_of(const Inst *__restrict__ tab, int n, int block)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].*B <= block)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// copies a chunk of the instance table (passed by value) to device memory
constexpr int kTabChunk = 8;
struct TabChunk {
    int first, count;
    Inst v[kTabChunk];
};
static_assert(sizeof(TabChunk) <= 4096, "kernel argument size");

__global__ void k_set_table(TabChunk c, Inst *tab)
{
    // plain word copies, one struct per block
    const int i = blockIdx.x;
    if (i >= c.count) return;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&c.v[i]);
    uint32_t *dst = reinterpret_cast<uint32_t *>(&tab[c.first + i]);
    for (int w = threadIdx.x; w < (int)(sizeof(Inst) / 4); w += blockDim.x) dst[w] = src[w];
}

// ------------------------------------------------------------ small kernels

__global__ void k_init(const Inst *__restrict__ tab, int n)
{
    const Inst a = tab[inst_of<&Inst::b_init>(tab, n, blockIdx.x)];
    const int64_t i = (int64_t)(blockIdx.x - a.b_init) * blockDim.x + threadIdx.x;
    if (i == 0) {
        a.hdr->error_bits = 0;
        a.hdr->reserved = 0;
        a.hdr->list_entries = 0;
        a.hdr->list_capacity = a.cap;
        a.hdr->ntasks = 0;
    }
    if (i < a.ncounts) {
        a.cnt[i] = 0;
        a.cur[i] = 0;
    }
}

// clear the keyframe and attribute gradients and the background-adjoint
// task counter
__global__ void k_bwd_init(const Inst *__restrict__ tab, int n)
{
    const Inst a = tab[inst_of<&Inst::b_bwdinit>(tab, n, blockIdx.x)];
    const int64_t i = (int64_t)(blockIdx.x - a.b_bwdinit) * blockDim.x + threadIdx.x;
    if (i == 0) {
        a.hdr->bwd_task_ctr = 0;
        a.hdr->gmax = 0;
    }
    const int64_t n1 = (int64_t)(a.S + 1) * a.V * 2, n2 = (int64_t)a.V * a.C;
    if (i < n1)
        a.gkf[i] = 0.0f;
    else if (i < n1 + n2)
        a.grad_attrs[i - n1] = 0.0f;
}

// Deterministic mode: gradient partial sums are added as 64-bit integers in
// units of 2^-det_shift, det_shift = 32 - e with 2^(e-1) <= max |dL/dI| < 2^e
// (integer addition does not depend on the order the atomics resolve in).
__device__ __forceinline__ int det_shift(const Inst &a)
{
    const float g = __uint_as_float(a.hdr->gmax);
    int e = 0;
    if (g > 0.0f && g <= 3.4028235e38f) (void)frexpf(g, &e);
    return 32 - e;
}

__device__ __forceinline__ void det_add(const Inst &a, int64_t RB_G *acc, double v, int shift)
{
    const double q = rint(ldexp(v, shift));
    if (!(fabs(q) < 0x1p62)) {
        atomicOr(&a.hdr->error_bits, kHdrDetRange);
        return;
    }
    atomicAdd((unsigned long long RB_G *)acc, (unsigned long long)(long long)q);
}

// deterministic mode, before the adjoint: max |dL/dI| (as float bits) and
// cleared fixed-point gradient sums
__global__ void k_det_prep(const Inst *__restrict__ tab, int n)
{
    const Inst a = tab[inst_of<&Inst::b_detp>(tab, n, blockIdx.x)];
    const int64_t i = (int64_t)(blockIdx.x - a.b_detp) * blockDim.x + threadIdx.x;
    const int64_t ngrad = (int64_t)(a.S + 1) * a.V * 2 + (int64_t)a.V * a.C;
    const int64_t nimg = (int64_t)(a.C + 1) * a.H * a.W;
    if (i < ngrad) a.gfx[i] = 0;
    uint32_t b = i < nimg ? __float_as_uint(fabsf(a.grad_image[i])) : 0u;
    // one atomic per wave (unsigned max on the bits orders non-negative
    // floats; a NaN's bits exceed every finite value's)
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) b = max(b, (uint32_t)__shfl_xor((int)b, d));
    if ((threadIdx.x & 63) == 0 && b) atomicMax(&a.hdr->gmax, b);
}

// deterministic mode, after the adjoint: fixed-point sums to the float
// keyframe and attribute gradients (NaN if a sum left the integer range)
__global__ void k_det_finish(const Inst *__restrict__ tab, int n)
{
    const Inst a = tab[inst_of<&Inst::b_bwdinit>(tab, n, blockIdx.x)];
    const int64_t i = (int64_t)(blockIdx.x - a.b_bwdinit) * blockDim.x + threadIdx.x;
    const int64_t n1 = (int64_t)(a.S + 1) * a.V * 2, n2 = (int64_t)a.V * a.C;
    if (i >= n1 + n2) return;
    const bool bad = (a.hdr->error_bits & kHdrDetRange) != 0;
    const float v = bad ? __builtin_nanf("") : (float)ldexp((double)a.gfx[i], -det_shift(a));
    if (i < n1)
        a.gkf[i] = v;
    else
        a.grad_attrs[i - n1] = v;
}

// Keyframe projection (App. I): X = view (M_s P0), x = X.x/(X.z tan), y = X.y/(X.z tan)
__global__ void k_project(const Inst *__restrict__ tab, int n)
{
    const Inst a = tab[inst_of<&Inst::b_proj>(tab, n, blockIdx.x)];
    const int64_t i = (int64_t)(blockIdx.x - a.b_proj) * blockDim.x + threadIdx.x;
    const int V = a.V, F = a.F;
    const int64_t nkf = (int64_t)(a.S + 1) * V;
    const ViewArgs &vw = a.vw;
    if (i < nkf) {
        int s = (int)(i / V), v = (int)(i - (int64_t)s * V);
        const float *m = a.model + (size_t)s * 12;
        double p0 = a.verts[3 * v], p1 = a.verts[3 * v + 1], p2 = a.verts[3 * v + 2];
        double w[3], c[3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            w[r] = (double)m[4 * r] * p0 + (double)m[4 * r + 1] * p1 + (double)m[4 * r + 2] * p2 + (double)m[4 * r + 3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            c[r] = (double)vw.m[4 * r] * w[0] + (double)vw.m[4 * r + 1] * w[1] + (double)vw.m[4 * r + 2] * w[2] +
                   (double)vw.m[4 * r + 3];
        double t = (double)vw.tanf;
        double x = c[0] / (c[2] * t), y = c[1] / (c[2] * t);
        a.kf[i] = make_double2(x, y);
        a.kfz[i] = (float)c[2];
        if (!(c[2] > 1e-6)) atomicOr(&a.hdr->error_bits, kHdrBehind);
    } else if (i < nkf + F) {
        int f = (int)(i - nkf);
        int q0 = a.faces[3 * f], q1 = a.faces[3 * f + 1], q2 = a.faces[3 * f + 2];
        if (q0 < 0 || q0 >= V || q1 < 0 || q1 >= V || q2 < 0 || q2 >= V) atomicOr(&a.hdr->error_bits, kHdrFaceRange);
    }
}

__device__ __forceinline__ void pixel_range(float lo, float hi, float scale, float off, int n, int &a, int &b)
{
    // pixel indices i in [0, n) with centre (2 i + 1 - n)/n inside [lo, hi]
    // (scale = n, off = n - 1 for columns; rows use the mirrored mapping)
    float fa = fmaf(lo, scale, off) * 0.5f - 0.01f;
    float fb = fmaf(hi, scale, off) * 0.5f + 0.01f;
    fa = fminf(fmaxf(fa, -2.0f), (float)n + 1.0f);
    fb = fminf(fmaxf(fb, -2.0f), (float)n + 1.0f);
    a = (int)ceilf(fa);
    b = (int)floorf(fb);
}

// Tile ranges of one face at one sub-frame: foreground (exact box) and
// background (box grown by halo).  Empty ranges come back with lo > hi.
template <int TW>
__device__ __forceinline__ void face_tiles(const float x[3], const float y[3], const Inst &a, float grow,
                                           int &tx0, int &tx1, int &ty0, int &ty1)
{
    float xmin = fminf(x[0], fminf(x[1], x[2])) - grow, xmax = fmaxf(x[0], fmaxf(x[1], x[2])) + grow;
    float ymin = fminf(y[0], fminf(y[1], y[2])) - grow, ymax = fmaxf(y[0], fmaxf(y[1], y[2])) + grow;
    int c0, c1, r0, r1;
    pixel_range(xmin, xmax, (float)a.W, (float)(a.W - 1), a.W, c0, c1);
    // rows: centre v = (H - 2r - 1)/H  ->  r = (H - 1 - v H)/2, decreasing in v
    pixel_range(-ymax, -ymin, (float)a.H, (float)(a.H - 1), a.H, r0, r1);
    c0 = max(c0, 0);
    c1 = min(c1, a.W - 1);
    r0 = max(r0, 0);
    r1 = min(r1, a.H - 1);
    if (c0 > c1 || r0 > r1) {
        tx0 = ty0 = 1;
        tx1 = ty1 = 0;
        return;
    }
    constexpr int TH = kWave / TW;
    tx0 = c0 / TW;
    tx1 = c1 / TW;
    ty0 = r0 / TH;
    ty1 = r1 / TH;
}

// Binning.  A block takes 256 consecutive faces of one chunk; meshes list
// neighbouring faces close together, so the block's tiles form a small
// window.  Per-tile counts are gathered with LDS atomics over that window and
// reach global memory with one atomic per (window tile, list kind); in the
// fill pass each window tile reserves one contiguous range of its list and
// the block's entries go there at LDS-atomic ranks.  A window larger than
// the LDS counters (fast motion: a chunk's faces sweep far) is taken in bands
// of rows; only a window whose single row does not fit uses one global atomic
// per entry.
constexpr int kBinThreads = 256;
constexpr int kBinWin = 2048;   // window counters: 2 list kinds x tiles

struct FaceTiles {
    int ux0, ux1, uy0, uy1;                 // union of the background rects over the chunk
};

template <int T, int TW>
__device__ __forceinline__ bool face_chunk_tiles(const Inst &a, int f, const Chunk &ch, int ftx0[T], int ftx1[T],
                                                 int fty0[T], int fty1[T], int btx0[T], int btx1[T], int bty0[T],
                                                 int bty1[T], FaceTiles &u)
{
    float ax[3], ay[3], bx[3], by[3];
    double2 kp[3], kr[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        int v = clampi(a.faces[3 * f + q], 0, a.V - 1);
        const double2 p = a.kf[(size_t)ch.s * a.V + v];
        const double2 r = a.kf[(size_t)(ch.s + 1) * a.V + v];
        kp[q] = p;
        kr[q] = r;
        ax[q] = (float)p.x;
        ay[q] = (float)p.y;
        bx[q] = (float)(r.x - p.x);
        by[q] = (float)(r.y - p.y);
    }
    u.ux0 = INT_MAX;
    u.ux1 = INT_MIN;
    u.uy0 = INT_MAX;
    u.uy1 = INT_MIN;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        ftx0[j] = fty0[j] = btx0[j] = bty0[j] = 1;
        ftx1[j] = fty1[j] = btx1[j] = bty1[j] = 0;
        if (j < ch.n) {
            int rem = (ch.k0 + j) * a.S - ch.s * (a.K - 1);
            // the skip rule |det F(tau)| <= kTauDet is decided here, in
            // double from the double keyframes: a face that is degenerate at
            // this sub-frame (a repeated vertex, coincident or collinear
            // vertices) gets no entry bit, whatever its float32 determinant
            // in the raster kernels would round to
            {
                const double td = a.K > 1 ? (double)rem / (double)(a.K - 1) : 0.0;
                double xd[3], yd[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    xd[q] = (1.0 - td) * kp[q].x + td * kr[q].x;
                    yd[q] = (1.0 - td) * kp[q].y + td * kr[q].y;
                }
                const double D = (xd[1] - xd[0]) * (yd[2] - yd[0]) - (xd[2] - xd[0]) * (yd[1] - yd[0]);
                if (!(fabs(D) > (double)kTauDetBin)) continue;
            }
            float tau = a.K > 1 ? (float)rem / (float)(a.K - 1) : 0.0f;
            float x[3], y[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                x[q] = fmaf(tau, bx[q], ax[q]);
                y[q] = fmaf(tau, by[q], ay[q]);
            }
            face_tiles<TW>(x, y, a, 0.0f, ftx0[j], ftx1[j], fty0[j], fty1[j]);
            face_tiles<TW>(x, y, a, a.halo, btx0[j], btx1[j], bty0[j], bty1[j]);
            if (btx0[j] <= btx1[j]) {
                u.ux0 = min(u.ux0, btx0[j]);
                u.ux1 = max(u.ux1, btx1[j]);
                u.uy0 = min(u.uy0, bty0[j]);
                u.uy1 = max(u.uy1, bty1[j]);
            }
        }
    }
    return u.ux0 <= u.ux1;
}

// TW: tile width (the tile shape is a batch-wide option)
template <int T, int TW>
__global__ __launch_bounds__(kBinThreads) void k_bin(const Inst *__restrict__ tab, int n, int pass)
{
    __shared__ int lcnt[kBinWin];
    __shared__ int64_t lbase[kBinWin];
    __shared__ int win[4];
    const Inst a = tab[inst_of<&Inst::b_bin>(tab, n, blockIdx.x)];
    const int nfb = a.nfb;
    const int lb = blockIdx.x - a.b_bin;
    const int c = lb / nfb;
    const int f = (lb - c * nfb) * kBinThreads + threadIdx.x;
    const Chunk ch = chunk_info(c, a.K, a.S, a.CPS);
    if (ch.n <= 0) return;   // block-uniform
    int ftx0[T], ftx1[T], fty0[T], fty1[T], btx0[T], btx1[T], bty0[T], bty1[T];
    FaceTiles u;
    const bool has = f < a.F && face_chunk_tiles<T, TW>(a, f, ch, ftx0, ftx1, fty0, fty1, btx0, btx1, bty0, bty1, u);
    if (threadIdx.x == 0) {
        win[0] = INT_MAX;
        win[1] = INT_MIN;
        win[2] = INT_MAX;
        win[3] = INT_MIN;
    }
    __syncthreads();
    if (has) {
        atomicMin(&win[0], u.ux0);
        atomicMax(&win[1], u.ux1);
        atomicMin(&win[2], u.uy0);
        atomicMax(&win[3], u.uy1);
    }
    __syncthreads();
    const int wx0 = win[0], wy0 = win[2];
    const int ww = win[1] - wx0 + 1;
    if (win[0] > win[1]) return;   // no face of the block touches the image (block-uniform)
    auto gidx = [&](int L, int tile) { return ((int64_t)L * a.NC + c) * a.ntiles + tile; };
    const uint32_t fbits = (uint32_t)f << 8;
    // the entries of this thread's face in window rows [y0, y1]:
    // fn(list kind, tile, mask, slot of the tile in the band)
    auto visit = [&](int y0, int y1, int nwt, auto &&fn) {
        if (!has) return;
        for (int ty = max(u.uy0, y0); ty <= min(u.uy1, y1); ++ty) {
            for (int tx = u.ux0; tx <= u.ux1; ++tx) {
                uint32_t fm = 0, bm = 0;
#pragma unroll
                for (int j = 0; j < T; ++j) {
                    if (tx >= ftx0[j] && tx <= ftx1[j] && ty >= fty0[j] && ty <= fty1[j]) fm |= 1u << j;
                    if (tx >= btx0[j] && tx <= btx1[j] && ty >= bty0[j] && ty <= bty1[j]) bm |= 1u << j;
                }
                const int tile = ty * a.tiles_x + tx;
                const int w = (ty - y0) * ww + (tx - wx0);
                if (fm) fn(0, tile, fm, w);
                if (bm) fn(1, tile, bm, nwt + w);
            }
        }
    };
    if (2 * ww > kBinWin) {
        // a window row does not fit in LDS: one global atomic per entry
        if (pass == 0) {
            visit(u.uy0, u.uy1, 0, [&](int L, int tile, uint32_t, int) { atomicAdd(&a.cnt[gidx(L, tile)], 1); });
        } else {
            visit(u.uy0, u.uy1, 0, [&](int L, int tile, uint32_t m, int) {
                const int64_t g = gidx(L, tile);
                const int64_t pos = a.off[g] + atomicAdd(&a.cur[g], 1);
                if (pos < a.cap) a.list[pos] = fbits | m;
            });
        }
        return;
    }
    // bands of window rows whose counters fit in LDS (usually one band)
    const int band = kBinWin / (2 * ww);
    for (int y0 = wy0; y0 <= win[3]; y0 += band) {
        const int y1 = min(win[3], y0 + band - 1);
        const int nwt = ww * (y1 - y0 + 1);
        for (int i = threadIdx.x; i < 2 * nwt; i += kBinThreads) lcnt[i] = 0;
        __syncthreads();
        visit(y0, y1, nwt, [&](int, int, uint32_t, int w) { atomicAdd(&lcnt[w], 1); });
        __syncthreads();
        for (int i = threadIdx.x; i < 2 * nwt; i += kBinThreads) {
            const int n = lcnt[i];
            if (!n) continue;
            const int L = i >= nwt, w = i - L * nwt;
            const int64_t g = gidx(L, (y0 + w / ww) * a.tiles_x + wx0 + w % ww);
            if (pass == 0) {
                atomicAdd(&a.cnt[g], n);
            } else {
                lbase[i] = a.off[g] + atomicAdd(&a.cur[g], n);
                lcnt[i] = 0;
            }
        }
        if (pass == 1) {
            __syncthreads();
            visit(y0, y1, nwt, [&](int, int, uint32_t m, int w) {
                const int64_t pos = lbase[w] + atomicAdd(&lcnt[w], 1);
                if (pos < a.cap) a.list[pos] = fbits | m;
            });
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------- scan
// exclusive prefix sum of n int32 counts into int64 offsets, 3 phases

constexpr int kScanThreads = 1024, kScanPer = 4, kScanBlock = kScanThreads * kScanPer;

__device__ int64_t block_exclusive_scan(int64_t x, int64_t *total)
{
    __shared__ int64_t wsum[kScanThreads / 64];
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        int64_t v = lane < kScanThreads / 64 ? wsum[lane] : 0;
        int64_t vi = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            int64_t y = __shfl_up(vi, d, 64);
            if (lane >= d) vi += y;
        }
        if (lane < kScanThreads / 64) wsum[lane] = vi - v;
        if (lane == kScanThreads / 64 - 1) *total = vi;
    }
    __syncthreads();
    int64_t r = inc - x + wsum[wid];
    __syncthreads();
    return r;
}

// which = 0: bin-list counts (cnt -> off, total to the header's list_entries,
// overflow against the capacity); which = 1: background task counts (tsl ->
// toff, total to the header's ntasks)
struct ScanIo {
    const int32_t *cnt;
    int64_t *off, *bsum, *total;
    int64_t n, nb;
    int first1, first3;
};

__device__ __forceinline__ ScanIo scan_io(const Inst &a, int which)
{
    ScanIo r;
    if (which == 0) {
        r.cnt = a.cnt;
        r.off = a.off;
        r.bsum = a.bsum;
        r.total = &a.hdr->list_entries;
        r.n = a.ncounts;
        r.nb = a.nblocks_scan;
        r.first1 = a.b_scan1;
        r.first3 = a.b_scan3;
    } else {
        r.cnt = a.tsl;
        r.off = a.toff;
        r.bsum = a.tbsum;
        r.total = &a.hdr->ntasks;
        r.n = a.ntct;
        r.nb = a.nblocks_tscan;
        r.first1 = a.b_tscan1;
        r.first3 = a.b_tscan3;
    }
    return r;
}

__global__ __launch_bounds__(kScanThreads) void k_scan1(const Inst *__restrict__ tab, int n, int which)
{
    __shared__ int64_t tot;
    const Inst &a = which == 0 ? tab[inst_of<&Inst::b_scan1>(tab, n, blockIdx.x)]
                               : tab[inst_of<&Inst::b_tscan1>(tab, n, blockIdx.x)];
    const ScanIo io = scan_io(a, which);
    const int blk = blockIdx.x - io.first1;
    int64_t base = (int64_t)blk * kScanBlock + (int64_t)threadIdx.x * kScanPer;
    int64_t v[kScanPer];
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        v[q] = base + q < io.n ? io.cnt[base + q] : 0;
        s += v[q];
    }
    int64_t ex = block_exclusive_scan(s, &tot);
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        if (base + q < io.n) io.off[base + q] = ex;
        ex += v[q];
    }
    if (threadIdx.x == 0) io.bsum[blk] = tot;
}

// block sums -> block offsets, one block per instance; the grand total goes
// to the header (bin lists: overflow bit when it exceeds the capacity)
__global__ __launch_bounds__(kScanThreads) void k_scan2(const Inst *__restrict__ tab, int which)
{
    __shared__ int64_t tot;
    const Inst a = tab[blockIdx.x];
    const ScanIo io = scan_io(a, which);
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < io.nb; b0 += kScanThreads) {
        int64_t i = b0 + threadIdx.x;
        int64_t x = i < io.nb ? io.bsum[i] : 0;
        int64_t ex = block_exclusive_scan(x, &tot);
        if (i < io.nb) io.bsum[i] = ex + carry;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *io.total = carry;
        if (which == 0 && carry > a.cap) atomicOr(&a.hdr->error_bits, kHdrOverflow);
    }
}

__global__ void k_scan3(const Inst *__restrict__ tab, int n, int which)
{
    const Inst &a = which == 0 ? tab[inst_of<&Inst::b_scan3>(tab, n, blockIdx.x)]
                               : tab[inst_of<&Inst::b_tscan3>(tab, n, blockIdx.x)];
    const ScanIo io = scan_io(a, which);
    const int64_t i = (int64_t)(blockIdx.x - io.first3) * blockDim.x + threadIdx.x;
    if (i < io.n) io.off[i] += io.bsum[i / kScanBlock];
}

// ------------------------------------------------- deterministic list order
// Deterministic mode: the binning appends entries in whatever order its
// atomics resolve; sorting each list by entry (face << 8 | mask, faces
// distinct within a list) makes every later pass see the same order.
// Bitonic sorting network in the variant without direction changes: merging
// blocks of size k starts by comparing i with its mirror k - 1 - i in the
// block, then halves the distance.  Positions past the list's end act as
// +infinity and never take part (a compare-exchange keeps the minimum at the
// lower index, so such a pair is a no-op).  Stages whose pairs lie within one
// block of kSortB entries run in LDS; longer lists do the wider stages in
// global memory.  Lists of at most 64 entries are sorted by the block's first
// wave in registers, one entry per lane.

constexpr int kSortThreads = 256, kSortB = 4096;

// compare-exchange over pair q of a stage of distance j (j == 0: the mirror
// step of block size k), indices relative to the buffer
template <class P>
__device__ __forceinline__ void cx_pair(P buf, int64_t q, int64_t k, int64_t j, int64_t len)
{
    int64_t i, pq;
    if (j == 0) {
        const int64_t h = k >> 1, b = q / h, o = q - b * h;
        i = b * k + o;
        pq = b * k + k - 1 - o;
    } else {
        const int64_t b = q / j;
        i = b * 2 * j + (q - b * j);
        pq = i + j;
    }
    if (pq >= len) return;
    const uint32_t x = buf[i], y = buf[pq];
    if (x > y) {
        buf[i] = y;
        buf[pq] = x;
    }
}

// The stages whose compare distance is below 64 stay inside one 64-entry
// chunk of the block: a wave runs them on its chunks in registers (one entry
// per lane, partners through shuffles), with no barrier between stages.
// full: the whole network of block sizes 2 .. 64; else the halving steps
// from distance 32 down to 1.
__device__ __forceinline__ void chunk_pass(uint32_t *sh, int blk, bool full)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int c = w; c < blk / kWave; c += kSortThreads / kWave) {
        uint32_t x = sh[c * kWave + lane];
        auto step = [&](int m) {
            const uint32_t y = (uint32_t)__shfl_xor((int)x, m, kWave);
            x = lane < (lane ^ m) ? min(x, y) : max(x, y);
        };
        if (full) {
#pragma unroll
            for (int k = 2; k <= kWave; k <<= 1) {
                step(k - 1);
#pragma unroll
                for (int m = k >> 2; m >= 1; m >>= 1) step(m);
            }
        } else {
#pragma unroll
            for (int m = kWave / 2; m >= 1; m >>= 1) step(m);
        }
        sh[c * kWave + lane] = x;
    }
}

// LDS pass over block [b0, b0 + blk) of the list (blk a power of two,
// 128 <= blk <= kSortB): the mirror steps of block sizes 2 .. blk, each
// followed by its halving steps, or (full == false) only the halving steps
// from distance blk / 2 down to 1
__device__ __forceinline__ void lds_pass(uint32_t RB_G *L, int64_t len, int64_t b0, int blk, bool full, uint32_t *sh)
{
    const int m = (int)min<int64_t>(blk, len - b0);
    for (int t = threadIdx.x; t < blk; t += kSortThreads) sh[t] = t < m ? L[b0 + t] : 0xffffffffu;
    __syncthreads();
    auto halve_lds = [&](int j) {   // halving steps of distance j .. 64
        for (; j >= kWave; j >>= 1) {
            for (int q = threadIdx.x; q < blk / 2; q += kSortThreads) cx_pair(sh, q, 0, j, blk);
            __syncthreads();
        }
    };
    if (!full) {
        halve_lds(blk >> 1);
        chunk_pass(sh, blk, false);
        __syncthreads();
    } else {
        chunk_pass(sh, blk, true);
        __syncthreads();
        for (int k = 2 * kWave; k <= blk; k <<= 1) {
            for (int q = threadIdx.x; q < blk / 2; q += kSortThreads) cx_pair(sh, q, k, 0, blk);
            __syncthreads();
            halve_lds(k >> 2);
            chunk_pass(sh, blk, false);
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < m; t += kSortThreads) L[b0 + t] = sh[t];
    __syncthreads();
}

// one block per list (foreground and background lists of every chunk and tile)
__global__ __launch_bounds__(kSortThreads) void k_sort_lists(const Inst *__restrict__ tab, int n)
{
    __shared__ uint32_t sh[kSortB];
    const Inst &a = tab[inst_of<&Inst::b_sort>(tab, n, blockIdx.x)];
    const int64_t g = blockIdx.x - a.b_sort;
    const int64_t len = a.cnt[g], beg = a.off[g];
    if (len <= 1 || beg + len > a.cap) return;   // (an overflowed forward is reported, not used)
    uint32_t RB_G *L = a.list + beg;
    if (len <= kWave) {
        // the same network over the 64 lanes; lanes past the end hold the
        // largest value and keep it
        if (threadIdx.x >= kWave) return;
        const int lane = threadIdx.x;
        uint32_t x = lane < len ? L[lane] : 0xffffffffu;
        auto cx = [&](int partner) {
            const uint32_t y = (uint32_t)__shfl((int)x, partner, kWave);
            x = lane < partner ? min(x, y) : max(x, y);
        };
#pragma unroll
        for (int k = 2; k <= kWave; k <<= 1) {
            cx(lane ^ (k - 1));
#pragma unroll
            for (int j = k >> 2; j >= 1; j >>= 1) cx(lane ^ j);
        }
        if (lane < len) L[lane] = x;
        return;
    }
    // network size: the smallest power of two >= len
    int64_t P = 2;
    while (P < len) P <<= 1;
    const int blk = (int)min<int64_t>(P, kSortB);
    // blocks sorted in LDS, then the wider merges
    for (int64_t b0 = 0; b0 < len; b0 += blk) lds_pass(L, len, b0, blk, true, sh);
    for (int64_t k = 2 * (int64_t)kSortB; k <= P; k <<= 1) {
        for (int64_t q = threadIdx.x; q < P / 2; q += kSortThreads) cx_pair(L, q, k, 0, len);
        __syncthreads();
        for (int64_t j = k >> 2; j >= kSortB; j >>= 1) {
            for (int64_t q = threadIdx.x; q < P / 2; q += kSortThreads) cx_pair(L, q, 0, j, len);
            __syncthreads();
        }
        for (int64_t b0 = 0; b0 < len; b0 += kSortB) lds_pass(L, len, b0, kSortB, false, sh);
    }
}

// ----------------------------------------------------------------- raster
//
// Forward, three kernels:
//  * k_fg, one 64-lane wave per (chunk, tile), lane = pixel: z-buffer
//    over the tile's foreground list (eq 9), shading of the winners, and the
//    per-(pixel, sub-frame) records the rest reads: winner (or uncovered),
//    colour, zeroed background accumulators.  It also counts the background
//    tasks of its (chunk, tile): slices of SL background-list entries, none
//    if every in-image pixel is covered at every sub-frame of the chunk.
//  * k_bg, persistent waves (one per resident slot; task t to wave t mod G):
//    soft aggregation (eqs 10, 13-15) of the slice's faces on the uncovered
//    pixels, accumulated in LDS as sum log2(1 - A) (zero factors counted
//    apart) and added to the pixel records.  Splitting the long lists of
//    silhouette tiles into slices keeps every wave's work bounded.
//  * k_resolve, one block per tile: the average over the K sub-frames (four
//    waves over interleaved sub-frames, combined in LDS).
//
// Inside a wave, a list is walked NB entries at a time:
//  * staging: lane e gathers entry e's face indices and double keyframes and
//    forms the entry's float32 coordinates relative to the tile anchor at the
//    chunk's middle time (stored in LDS field-major, so lanes reading different
//    entries hit different banks).  It also forms, per sub-frame of the chunk,
//    the 64-bit mask of tile pixels the entry can reach (its box at that
//    sub-frame; for the background, the pixels within the influence radius of
//    that box; restricted to the pixels still in question) and their union U_e.
//  * items: the batch's work is the set of (entry, pixel) pairs with the pixel
//    in U_e.  An exclusive scan over the entries numbers them and they are
//    dealt out 64 at a time, one per lane, so a face that reaches 3 pixels of
//    the tile costs 3 lane-evaluations instead of 64.  An item carries the
//    sub-frames where its pixel is in the entry's mask; the fast solver's
//    coefficients are formed once per item and evaluated per sub-frame.
//  * foreground items update the LDS z-buffer by a 64-bit atomic min of
//    (depth bits, face index), which keeps the lowest face index on exact
//    depth ties; background items add log2(1 - A) with LDS float atomics,
//    or, when faces reach many pixels, are regrouped by pixel and dealt in
//    per-lane runs that add a pixel's factors up before touching LDS.
//
// Backward, two kernels: k_fg_bwd per (chunk, tile) with a winner stages
// only the faces that win a (pixel, sub-frame) with a colour gradient, found
// from the visibility record; k_bg_bwd over the same background tasks as the
// forward.  Items are dealt in per-lane runs whose gradients add up in
// registers; a vertex-keyed LDS table collects the runs and is added to
// global memory with one atomic per non-zero value when it fills or the work
// unit ends.

constexpr int NCH = RB_MAX_CHANNELS;
constexpr int NB = 32;              // list entries staged per batch
constexpr int kVisOut = -4;         // vis_id of a pixel outside the image
constexpr int kSeqFg = 4;           // consecutive items per lane in the foreground adjoint
constexpr int kSeqBgFwd = 4;        // and in the background forward (grouped by pixel)
// background-forward grid, in multiples of the resident waves: wide-halo
// tasks vary more in cost and gain from finer dealing
constexpr unsigned kBgFwdOversubWide = 32, kBgFwdOversubNarrow = 8;

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

enum { kRecFg = 0, kRecBg = 1, kRecGeom = 2 };

// field offsets of a staged entry (edge i runs from vertex (i+1)%3 to (i+2)%3)
enum {
    R_XC = 0,     // positions at the chunk's middle time tc, minus the tile anchor
    R_YC = 3,
    R_DX = 6,     // segment displacement
    R_DY = 9,
    R_E0X = 12,   // edge i at the segment start
    R_E0Y = 15,
    R_E1X = 18,   // edge i at the segment end
    R_E1Y = 21,
    R_A0 = 24,    // foreground: camera depth at the start; background: 1/|edge i|^2 at the start (0 if degenerate)
    R_A1 = 27,    // foreground: its change over the segment; background: 1/|edge i|^2 at the end
    R_F = 30,     // face index (int bits)
    R_N = 31
};

// An entry in registers.
struct FaceRec {
    float v[R_N - 1];
    int f;
    __device__ float at(int k) const { return v[k]; }
};

// An entry staged in LDS, field-major: field k of entry e at rec[k][e].
// a staged record in LDS, field-major with a stride of NBX entries
template <int NBX>
struct LdsRecN {
    const float *p;
    __device__ float at(int k) const { return p[k * NBX]; }
};

__device__ __forceinline__ void lds_sync()
{
    // LDS operations of one wave execute in order; keep the compiler from
    // moving memory accesses across this point
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
}

// vertex indices of face f (clamped; out-of-range indices are reported by k_project)
__device__ __forceinline__ void face_verts(const Inst &a, int f, int vid[3])
{
#pragma unroll
    for (int q = 0; q < 3; ++q) vid[q] = clampi(a.faces[3 * f + q], 0, a.V - 1);
}

__device__ __forceinline__ void stage_rec(const Inst &a, int f, const int vid[3], int s, double ua, double va,
                                          float tc, int kind, FaceRec &r)
{
    r.f = f;
    double X0[3], Y0[3], X1[3], Y1[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int v = vid[q];
        const double2 p = a.kf[(size_t)s * a.V + v];
        const double2 e = a.kf[(size_t)(s + 1) * a.V + v];
        X0[q] = p.x;
        Y0[q] = p.y;
        X1[q] = e.x;
        Y1[q] = e.y;
        r.v[R_XC + q] = (float)(fma((double)tc, e.x - p.x, p.x) - ua);
        r.v[R_YC + q] = (float)(fma((double)tc, e.y - p.y, p.y) - va);
        r.v[R_DX + q] = (float)(e.x - p.x);
        r.v[R_DY + q] = (float)(e.y - p.y);
        if (kind == kRecFg) {
            const float z0 = a.kfz[(size_t)s * a.V + v], z1 = a.kfz[(size_t)(s + 1) * a.V + v];
            r.v[R_A0 + q] = z0;
            r.v[R_A1 + q] = z1 - z0;
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int j = (i + 1) % 3, k = (i + 2) % 3;
        const double ax = X0[k] - X0[j], ay = Y0[k] - Y0[j], bx = X1[k] - X1[j], by = Y1[k] - Y1[j];
        r.v[R_E0X + i] = (float)ax;
        r.v[R_E0Y + i] = (float)ay;
        r.v[R_E1X + i] = (float)bx;
        r.v[R_E1Y + i] = (float)by;
        if (kind == kRecBg) {
            const float ea = (float)(ax * ax + ay * ay), eb = (float)(bx * bx + by * by);
            r.v[R_A0 + i] = ea > 0.0f ? rcp(ea) : 0.0f;
            r.v[R_A1 + i] = eb > 0.0f ? rcp(eb) : 0.0f;
        }
    }
    if (kind == kRecGeom) {
#pragma unroll
        for (int i = 0; i < 3; ++i) r.v[R_A0 + i] = r.v[R_A1 + i] = 0.0f;
    }
}

// Per-lane barycentric numerators N_i(tau) (w_i = N_i / sum N) at the pixel
// (du, dv) from the anchor; N_i = (v_j - p) x (v_k - v_j) with (i, j, k)
// cyclic, i.e. row i of adj(F) p (eq 7).
//
// FAST (eq 8): under linear motion N_i is a quadratic in the local time, with
// coefficients computed once per (pixel, face, chunk) and evaluated by Horner's
// rule per sub-frame.  The quadratic is expanded about the chunk's middle time
// tc (t' = tau - tc): the same polynomial as the segment-start expansion, but
// built from pixel-to-vertex and edge vectors at tc, which keeps float32
// cancellation small when a segment moves far.
// RECOMPUTE: per sub-frame, lerp the three vertices (eq 5) and take the
// adjugate row products afresh (eqs 2-3).
template <int SOLVER>
struct Bary {
    float c1[3], c2[3], c3[3];
    template <class R>
    __device__ __forceinline__ void setup(const R &r, float tc, float du, float dv)
    {
        if (SOLVER == RB_SOLVER_FAST) {
            float ax[3], ay[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                ax[q] = r.at(R_XC + q) - du;
                ay[q] = r.at(R_YC + q) - dv;
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int j = (i + 1) % 3;
                const float e0x = r.at(R_E0X + i), e0y = r.at(R_E0Y + i);
                const float dex = r.at(R_E1X + i) - e0x, dey = r.at(R_E1Y + i) - e0y;
                const float ecx = fmaf(tc, dex, e0x), ecy = fmaf(tc, dey, e0y);
                const float djx = r.at(R_DX + j), djy = r.at(R_DY + j);
                c1[i] = fmaf(djx, dey, -djy * dex);
                c2[i] = fmaf(ax[j], dey, -ay[j] * dex) + fmaf(djx, ecy, -djy * ecx);
                c3[i] = fmaf(ax[j], ecy, -ay[j] * ecx);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                c1[i] = r.at(R_XC + i) - du;
                c2[i] = r.at(R_YC + i) - dv;
                c3[i] = 0.0f;
            }
        }
    }
    template <class R>
    __device__ __forceinline__ void eval(const R &r, float t, float N[3]) const
    {
        // t = tau - tc
        if (SOLVER == RB_SOLVER_FAST) {
#pragma unroll
            for (int i = 0; i < 3; ++i) N[i] = fmaf(fmaf(c1[i], t, c2[i]), t, c3[i]);
        } else {
            float xt[3], yt[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                xt[i] = fmaf(t, r.at(R_DX + i), c1[i]);
                yt[i] = fmaf(t, r.at(R_DY + i), c2[i]);
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int j = (i + 1) % 3, k = (i + 2) % 3;
                N[i] = fmaf(xt[j], yt[k], -xt[k] * yt[j]);
            }
        }
    }
};

// Background term of one (pixel, face, sub-frame): closest point of the
// keyframe triangle F(X) to q = F(X) w by the three clamped edge projections
// of App. B (edges (0,1), (1,2), (2,0), first wins ties; eq 13), mapped to
// the sub-frame (eq 14): d = |p - F(tau) w*|^2.
struct BgEval {
    float w[3];
    float rx, ry;             // q - v_be in F(X)
    float sr, sg;             // raw and clamped edge parameter
    float psx, psy, d;        // closest point at tau (anchor-local) and squared distance
    int be;                   // chosen edge: vertices be and (be+1)%3
};

// keyframe X positions (anchor-local) and edges; closest-point edge e of
// F(X) (from vertex e to e+1) is the entry's edge (e+2)%3
struct KEdges {
    float Ex[3], Ey[3], iee[3], kx[3], ky[3];
};

template <class R>
__device__ __forceinline__ void kedges(const R &r, int X, float tc, KEdges &k)
{
    const float tx = (X ? 1.0f : 0.0f) - tc;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        k.kx[q] = fmaf(tx, r.at(R_DX + q), r.at(R_XC + q));
        k.ky[q] = fmaf(tx, r.at(R_DY + q), r.at(R_YC + q));
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int i = (e + 2) % 3, b = (e + 1) % 3;
        k.Ex[e] = k.kx[b] - k.kx[e];
        k.Ey[e] = k.ky[b] - k.ky[e];
        k.iee[e] = X ? r.at(R_A1 + i) : r.at(R_A0 + i);
    }
}

template <class R>
__device__ __forceinline__ void bg_eval(const R &r, const KEdges &k, float tc, float tau, int X, const float N[3],
                                        float invD, float du, float dv, BgEval &b)
{
#pragma unroll
    for (int i = 0; i < 3; ++i) b.w[i] = N[i] * invD;
    const float *Ex = k.Ex, *Ey = k.Ey, *iee = k.iee, *kx = k.kx, *ky = k.ky;
    // q = F(X) w = p + (X - tau) sum_i w_i dv_i (linear motion, sum w = 1):
    // exact at the keyframes and under translation, and free of the
    // |w| * |edge| rounding of sum_i w_i v_i(X) when the face is nearly
    // edge-on at tau (|w| large)
    const float mX = (X ? 1.0f : 0.0f) - tau;
    const float d0x = r.at(R_DX), d0y = r.at(R_DY);
    const float sx = fmaf(b.w[1], r.at(R_DX + 1) - d0x, fmaf(b.w[2], r.at(R_DX + 2) - d0x, d0x));
    const float sy = fmaf(b.w[1], r.at(R_DY + 1) - d0y, fmaf(b.w[2], r.at(R_DY + 2) - d0y, d0y));
    const float qx = fmaf(mX, sx, du), qy = fmaf(mX, sy, dv);
    float best = FLT_MAX;
    b.be = 0;
    b.sr = 0.0f;
    b.sg = 0.0f;
    b.rx = 0.0f;
    b.ry = 0.0f;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const float rx = qx - kx[e], ry = qy - ky[e];
        const float sr = fmaf(rx, Ex[e], ry * Ey[e]) * iee[e];
        const float sg = __builtin_amdgcn_fmed3f(sr, 0.0f, 1.0f);
        const float hx = fmaf(-sg, Ex[e], rx), hy = fmaf(-sg, Ey[e], ry);
        const float dist = fmaf(hx, hx, hy * hy);
        const bool better = dist < best || e == 0;
        best = better ? dist : best;
        b.be = better ? e : b.be;
        b.sr = better ? sr : b.sr;
        b.sg = better ? sg : b.sg;
        b.rx = better ? rx : b.rx;
        b.ry = better ? ry : b.ry;
    }
    const float t = tau - tc;
    float xt[3], yt[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        xt[q] = fmaf(t, r.at(R_DX + q), r.at(R_XC + q));
        yt[q] = fmaf(t, r.at(R_DY + q), r.at(R_YC + q));
    }
    const float xa = b.be == 0 ? xt[0] : (b.be == 1 ? xt[1] : xt[2]);
    const float ya = b.be == 0 ? yt[0] : (b.be == 1 ? yt[1] : yt[2]);
    const float xb = b.be == 0 ? xt[1] : (b.be == 1 ? xt[2] : xt[0]);
    const float yb = b.be == 0 ? yt[1] : (b.be == 1 ? yt[2] : yt[0]);
    b.psx = fmaf(b.sg, xb - xa, xa);
    b.psy = fmaf(b.sg, yb - ya, ya);
    const float ddx = b.psx - du, ddy = b.psy - dv;
    b.d = fmaf(ddx, ddx, ddy * ddy);
}

// log2(1 - A) with A = exp(-x): series in A for small A, log of the
// cancellation-free 1 - A otherwise
__device__ __forceinline__ float log2_one_minus(float A, float om)
{
    if (A < 0.015625f) {
        float s = fmaf(A, 0.2f, 0.25f);
        s = fmaf(A, s, 1.0f / 3.0f);
        s = fmaf(A, s, 0.5f);
        s = fmaf(A, s, 1.0f);
        return -A * s * 1.4426950408889634f;
    }
    return __log2f(om);
}

// pixel p of a tile (bit tw * row + column) relative to the tile anchor, which
// lies between the 4 centre pixels; exact for W, H powers of 2
// (TWS: the tile width when known at compile time, 0 when read from a)
template <int TWS = 0>
__device__ __forceinline__ float pix_du(const Inst &a, int p)
{
    const int tw = TWS ? TWS : a.tw;
    return (float)(2 * (p & (tw - 1)) - (tw - 1)) * a.inv_w;
}
template <int TWS = 0>
__device__ __forceinline__ float pix_dv(const Inst &a, int p)
{
    const int th = TWS ? kWave / TWS : a.th, lw = TWS ? __builtin_ctz(TWS) : a.lw;
    return (float)((th - 1) - 2 * (p >> lw)) * a.inv_h;
}

// image pixel of lane `lane` in tile (tx, ty)
__device__ __forceinline__ void tile_pixel(const Inst &a, int tx, int ty, int lane, int &px, int &py)
{
    px = (tx << a.lw) + (lane & (a.tw - 1));
    py = (ty << a.lh) + (lane >> a.lw);
}

struct TileCtx {
    int c, tile, px, py;
    bool inimg;
    double ua, va;   // tile anchor in normalized coordinates
    float du, dv;    // this lane's pixel centre relative to the anchor
    Chunk ck;
};

__device__ __forceinline__ void tile_ctx(const Inst &a, int ct, TileCtx &g)
{
    const int lane = threadIdx.x & 63;
    g.c = ct / a.ntiles;
    g.tile = ct - g.c * a.ntiles;
    const int tx = g.tile % a.tiles_x, ty = g.tile / a.tiles_x;
    tile_pixel(a, tx, ty, lane, g.px, g.py);
    g.inimg = g.px < a.W && g.py < a.H;
    g.ua = (double)(2 * a.tw * tx + a.tw - a.W) / (double)a.W;
    g.va = (double)(a.H - 2 * a.th * ty - a.th) / (double)a.H;
    g.du = pix_du(a, lane);
    g.dv = pix_dv(a, lane);
    g.ck = chunk_info(g.c, a.K, a.S, a.CPS);
}

// local time of sub-frame j of a chunk and whether eq 13 takes the segment's
// end keyframe (tau > 1/2, decided in integers)
__device__ __forceinline__ float chunk_tau(const Inst &a, const Chunk &ch, int j, int &X)
{
    const int rem = (ch.k0 + j) * a.S - ch.s * (a.K - 1);
    X = 2 * rem > a.K - 1 ? 1 : 0;
    return a.K > 1 ? (float)rem / (float)(a.K - 1) : 0.0f;
}

template <int T>
__device__ __forceinline__ void chunk_taus(const Inst &a, const Chunk &ch, float tau[T], uint32_t &xbits)
{
    xbits = 0;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        int X;
        tau[j] = chunk_tau(a, ch, j, X);
        if (j < ch.n && X) xbits |= 1u << j;
    }
}

// middle local time of a chunk: the expansion point of the fast solver
template <int T>
__device__ __forceinline__ float chunk_centre(const float tau[T], int n)
{
    float last = tau[0];
#pragma unroll
    for (int j = 1; j < T; ++j)
        if (j < n) last = tau[j];
    return 0.5f * (tau[0] + last);
}

// record index of pixel lane, sub-frame k of a tile
__device__ __forceinline__ size_t vis_index(const Inst &a, int tile, int k, int lane)
{
    return ((size_t)tile * a.K + k) * kWave + lane;
}
__device__ __forceinline__ size_t pix_index(const Inst &a, int tile, int k, int slot, int lane)
{
    return (((size_t)tile * a.K + k) * a.NS + slot) * kWave + lane;
}

// ------------------------------------------------------------ item machinery

// mask of the tile pixels whose centres lie in [x0 - g, x1 + g] x [y0 - g, y1 + g]
// (anchor-local; bit = TW * row + column), with a margin of 0.05 pixel so that
// the box never cuts off a pixel the exact test would accept
template <int TW>
__device__ __forceinline__ uint64_t rect_mask_t(float x0, float x1, float y0, float y1, float g, float W, float H)
{
    constexpr int TH = kWave / TW;
    constexpr uint64_t REP = ~0ull / ((1ull << TW) - 1ull);   // bit 0 of every row
    // column c has centre du = (2c - (TW-1))/W, row r has dv = ((TH-1) - 2r)/H
    const float ca = fmaf(x0 - g, W, (float)(TW - 1)) * 0.5f - 0.05f, cb = fmaf(x1 + g, W, (float)(TW - 1)) * 0.5f + 0.05f;
    const float ra = ((float)(TH - 1) - (y1 + g) * H) * 0.5f - 0.05f, rb = ((float)(TH - 1) - (y0 - g) * H) * 0.5f + 0.05f;
    const int c0 = max((int)ceilf(fmaxf(ca, -1.0f)), 0), c1 = min((int)floorf(fminf(cb, (float)TW)), TW - 1);
    const int r0 = max((int)ceilf(fmaxf(ra, -1.0f)), 0), r1 = min((int)floorf(fminf(rb, (float)TH)), TH - 1);
    if (c0 > c1 || r0 > r1) return 0ull;
    const uint64_t row = (uint64_t)(((2u << (c1 - c0)) - 1u) << c0);
    const uint64_t hi = r1 == TH - 1 ? ~0ull : ((1ull << (TW * (r1 + 1))) - 1ull);
    const uint64_t lo = (1ull << (TW * r0)) - 1ull;
    return (row * REP) & hi & ~lo;
}

// mask of the tile pixels whose centres lie within distance g of the box
// [x0, x1] x [y0, y1] (anchor-local), with a margin of 0.05 pixel: a superset
// of the pixels within distance g of a triangle inside the box, i.e. of the
// pixels the background term can reach (the box grown by g, corners rounded)
// (g2r: the squared distance per tile row instead of g * g, when given)
template <int TW>
__device__ __forceinline__ uint64_t disc_mask_t(float x0, float x1, float y0, float y1, float g, float W, float H,
                                                const float *g2r = nullptr)
{
    constexpr int TH = kWave / TW;
    const float ih = rcp(H), my = 0.1f * ih, gg = g * g;
    uint64_t m = 0;
#pragma unroll
    for (int r = 0; r < TH; ++r) {
        // row r has centre dv = ((TH-1) - 2r)/H
        const float v = (float)(TH - 1 - 2 * r) * ih;
        const float dy = fmaxf(fmaxf(y0 - v, v - y1) - my, 0.0f);
        const float h2 = fmaf(-dy, dy, g2r ? g2r[r] : gg);
        const float hx = sqrtf(fmaxf(h2, 0.0f));
        const float ca = fmaf(x0 - hx, W, (float)(TW - 1)) * 0.5f - 0.05f, cb = fmaf(x1 + hx, W, (float)(TW - 1)) * 0.5f + 0.05f;
        const int c0 = max((int)ceilf(fmaxf(ca, -1.0f)), 0), c1 = min((int)floorf(fminf(cb, (float)TW)), TW - 1);
        const uint32_t row = (h2 >= 0.0f && c0 <= c1) ? (((2u << (c1 - c0)) - 1u) << c0) : 0u;
        m |= (uint64_t)row << (TW * r);
    }
    return m;
}

// the same for 16 x 4 and 4 x 16 tiles (shape in run-time values): the
// rectangle in closed form, the rounded box row by row
__device__ __forceinline__ uint64_t rect_mask_any(const Inst &a, float x0, float x1, float y0, float y1, float g)
{
    const int tw = a.tw, th = a.th;
    const float W = (float)a.W, H = (float)a.H, cw = (float)(tw - 1), ch = (float)(th - 1);
    const float ca = fmaf(x0 - g, W, cw) * 0.5f - 0.05f, cb = fmaf(x1 + g, W, cw) * 0.5f + 0.05f;
    const float ra = (ch - (y1 + g) * H) * 0.5f - 0.05f, rb = (ch - (y0 - g) * H) * 0.5f + 0.05f;
    const int c0 = max((int)ceilf(fmaxf(ca, -1.0f)), 0), c1 = min((int)floorf(fminf(cb, (float)tw)), tw - 1);
    const int r0 = max((int)ceilf(fmaxf(ra, -1.0f)), 0), r1 = min((int)floorf(fminf(rb, (float)th)), th - 1);
    if (c0 > c1 || r0 > r1) return 0ull;
    const uint64_t row = (uint64_t)(((2u << (c1 - c0)) - 1u) << c0);
    const uint64_t hi = r1 == th - 1 ? ~0ull : ((1ull << (tw * (r1 + 1))) - 1ull);
    const uint64_t lo = (1ull << (tw * r0)) - 1ull;
    return (row * a.rep) & hi & ~lo;
}

__device__ __forceinline__ uint64_t disc_mask_any(const Inst &a, float x0, float x1, float y0, float y1, float g,
                                                  const float *g2r = nullptr)
{
    const int tw = a.tw, th = a.th;
    const float W = (float)a.W, cw = (float)(tw - 1), ih = rcp((float)a.H), my = 0.1f * ih, gg = g * g;
    uint64_t m = 0;
    for (int r = 0; r < th; ++r) {
        const float v = (float)(th - 1 - 2 * r) * ih;   // row r's centre
        const float dy = fmaxf(fmaxf(y0 - v, v - y1) - my, 0.0f);
        const float h2 = fmaf(-dy, dy, g2r ? g2r[r] : gg);
        if (h2 < 0.0f) continue;
        const float hx = sqrtf(h2);
        const float ca = fmaf(x0 - hx, W, cw) * 0.5f - 0.05f, cb = fmaf(x1 + hx, W, cw) * 0.5f + 0.05f;
        const int c0 = max((int)ceilf(fmaxf(ca, -1.0f)), 0), c1 = min((int)floorf(fminf(cb, (float)tw)), tw - 1);
        if (c0 <= c1) m |= (uint64_t)(((2u << (c1 - c0)) - 1u) << c0) << (tw * r);
    }
    return m;
}

// the masks for the instance's tile shape (a wave-uniform choice; TWS == 8:
// the kernel is built for 8 x 8 tiles)
template <int TWS = 0>
__device__ __forceinline__ uint64_t tile_mask(const Inst &a, bool disc, float x0, float x1, float y0, float y1, float g,
                                              const float *g2r = nullptr)
{
    const float W = (float)a.W, H = (float)a.H;
    const bool t8 = TWS == 8 || a.tw == 8;
    if (disc) return t8 ? disc_mask_t<8>(x0, x1, y0, y1, g, W, H, g2r) : disc_mask_any(a, x0, x1, y0, y1, g, g2r);
    return t8 ? rect_mask_t<8>(x0, x1, y0, y1, g, W, H) : rect_mask_any(a, x0, x1, y0, y1, g);
}

// position of the r-th set bit (r < popcount(m))
__device__ __forceinline__ int select64(uint64_t m, int r)
{
    uint32_t x = (uint32_t)m;
    int base = 0;
    int c = __popc(x);
    if (r >= c) {
        r -= c;
        x = (uint32_t)(m >> 32);
        base = 32;
    }
    c = __popc(x & 0xffffu);
    if (r >= c) {
        r -= c;
        x >>= 16;
        base += 16;
    }
    c = __popc(x & 0xffu);
    if (r >= c) {
        r -= c;
        x >>= 8;
        base += 8;
    }
    c = __popc(x & 0xfu);
    if (r >= c) {
        r -= c;
        x >>= 4;
        base += 4;
    }
    c = __popc(x & 0x3u);
    if (r >= c) {
        r -= c;
        x >>= 2;
        base += 2;
    }
    return base + (r >= (int)(x & 1u) ? 1 : 0);
}

__device__ __forceinline__ int wave_incl_scan(int x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

__device__ __forceinline__ int lane_rank(uint64_t bal)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
}

// Item bookkeeping shared by the forward and backward walks (NBX entries
// staged per batch).
template <int T, int NBX = NB>
struct ItemShared {
    float rec[R_N][NBX];  // staged entries, field-major
    uint64_t m[T][NBX];   // per sub-frame and entry: pixels to evaluate
    uint64_t U[NBX];      // union over the sub-frames
    int pre[NBX + 1];     // number of the entry's first item (entry nb: the batch's item count)
    int ne[NBX];          // entries with at least one item, in order
    uint8_t flag[kWave];
};

template <int T, int NBX>
__device__ __forceinline__ LdsRecN<NBX> lds_rec(ItemShared<T, NBX> &sh, int e)
{
    return LdsRecN<NBX>{&sh.rec[0][e]};
}

template <int T, int NBX>
__device__ __forceinline__ void store_rec(ItemShared<T, NBX> &sh, int e, const FaceRec &r)
{
#pragma unroll
    for (int k = 0; k < R_N - 1; ++k) sh.rec[k][e] = r.v[k];
    sh.rec[R_F][e] = __int_as_float(r.f);
}

// A batch's list entries and their faces' vertex indices, loaded one batch
// ahead so that staging waits for one level of gathers instead of three.
struct Pref {
    uint32_t ent;
    int v[3];
};

__device__ __forceinline__ Pref prefetch(const Inst &a, int64_t first, int nb)
{
    const int lane = threadIdx.x & 63;
    Pref pf;
    pf.ent = 0;
    pf.v[0] = pf.v[1] = pf.v[2] = 0;
    if (lane < nb) {
        pf.ent = a.list[first + lane];
        face_verts(a, (int)(pf.ent >> 8), pf.v);
    }
    return pf;
}

// Stage a batch of nb list entries (one per lane) with their per-sub-frame
// pixel masks; allow[j] is the set of pixels in question at sub-frame j (0 for
// sub-frames outside the chunk).  Returns the number of items; cnt / pre are
// the lane's entry's item count and first item.  Optionally also stages the
// vertex attributes (at) and vertex indices (vids).  With reach, background
// boxes are grown row by row by reach[j][row] (squared) instead of by grow.
template <int T, int TWS = 0>
__device__ __forceinline__ int stage_items(const Inst &a, ItemShared<T> &sh, const Pref &pf, int nb, int s,
                                           const TileCtx &g, float tc, const float tau[T], int kind, float grow,
                                           const uint64_t allow[T], float (*at)[NB], int (*vids)[3], int &cnt,
                                           int &pre, const float (*reach)[kMaxTileH] = nullptr)
{
    const int lane = threadIdx.x & 63;
    lds_sync();
    cnt = 0;
    if (lane < nb) {
        const uint32_t ent = pf.ent;
        const int *vid = pf.v;
        FaceRec r;
        stage_rec(a, (int)(ent >> 8), vid, s, g.ua, g.va, tc, kind, r);
        uint64_t U = 0;
#pragma unroll
        for (int j = 0; j < T; ++j) {
            uint64_t mj = 0;
            if (((ent >> j) & 1u) && allow[j]) {
                const float t = tau[j] - tc;
                float x0 = FLT_MAX, x1 = -FLT_MAX, y0 = FLT_MAX, y1 = -FLT_MAX;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const float xt = fmaf(t, r.v[R_DX + q], r.v[R_XC + q]);
                    const float yt = fmaf(t, r.v[R_DY + q], r.v[R_YC + q]);
                    x0 = fminf(x0, xt);
                    x1 = fmaxf(x1, xt);
                    y0 = fminf(y0, yt);
                    y1 = fmaxf(y1, yt);
                }
                mj = tile_mask<TWS>(a, kind == kRecBg, x0, x1, y0, y1, grow, reach ? reach[j] : nullptr) &
                     allow[j];
            }
            sh.m[j][lane] = mj;
            U |= mj;
        }
        store_rec(sh, lane, r);
        sh.U[lane] = U;
        if (at) {
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int c = 0; c < NCH; ++c) at[q * NCH + c][lane] = c < a.C ? a.attrs[(size_t)vid[q] * a.C + c] : 0.0f;
        }
        if (vids) {
#pragma unroll
            for (int q = 0; q < 3; ++q) vids[lane][q] = vid[q];
        }
        cnt = __popcll(U);
    }
    const int incl = wave_incl_scan(cnt);
    pre = incl - cnt;
    const uint64_t bal = __ballot(cnt > 0);
    if (lane <= nb) sh.pre[lane] = pre;
    if (cnt > 0) sh.ne[lane_rank(bal)] = lane;
    lds_sync();
    return __shfl(incl, 63, 64);
}

// Deal the batch's items out 64 at a time: fn(entry, pixel) on one lane each.
template <int T, class Fn>
__device__ __forceinline__ void for_items(ItemShared<T> &sh, int total, int cnt, int pre, Fn &&fn)
{
    const int lane = threadIdx.x & 63;
    const uint64_t upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    for (int rb = 0; rb < total; rb += kWave) {
        sh.flag[lane] = 0;
        lds_sync();
        // entries whose first item falls in this round (distinct positions)
        if (cnt > 0 && pre >= rb && pre < rb + kWave) sh.flag[pre - rb] = 1;
        const int c0 = __popcll(__ballot(cnt > 0 && pre <= rb)) - 1;
        lds_sync();
        const uint64_t B = __ballot(sh.flag[lane] != 0);
        if (rb + lane < total) {
            const int e = sh.ne[c0 + __popcll(B & upto & ~1ull)];
            const int p = select64(sh.U[e], rb + lane - sh.pre[e]);
            fn(e, p);
        }
        lds_sync();
    }
}


// Deal a batch's items out M consecutive ones per lane (64 M per round).
// Items are grouped by key (a staged entry, or a pixel): key k owns items
// kpre[k] .. kpre[k+1] - 1, one per set bit of kmask[k] in increasing order.
// item(k, b) runs for each item of the lane's range in order and flush(k)
// after the lane's last item of key k, so a lane's accumulators hold one key
// at a time and reach shared memory once per (lane, key) rather than once
// per item: far fewer LDS atomics, and far fewer lanes adding to the same
// address at once.  pre is kpre[lane] (the item count past the last key).
template <class Fi, class Ff>
__device__ __forceinline__ void for_runs(int M, int total, int pre, const int *kpre, const uint64_t *kmask, Fi &&item,
                                         Ff &&flush)
{
    const int lane = threadIdx.x & 63;
    for (int rb = 0; rb < total; rb += kWave * M) {
        const int i0 = rb + lane * M;
        // key holding item i0: the last key whose first item is <= i0
        int L = 0;
#pragma unroll
        for (int st = 32; st >= 1; st >>= 1) {
            const int v = __shfl(pre, L + st, 64);
            if (v <= i0) L += st;
        }
        if (i0 < total) {
            const int i1 = min(i0 + M, total);
            int k = L;
            int end = kpre[k + 1];
            uint64_t rem = kmask[k];
            int b = select64(rem, i0 - kpre[k]);
            rem = b == 63 ? 0ull : rem & (~0ull << (b + 1));
            for (int i = i0;;) {
                item(k, b);
                if (++i == i1) break;
                if (i == end) {
                    flush(k);
                    // the next key with items (one exists: i < total)
                    do {
                        ++k;
                    } while (kpre[k + 1] == kpre[k]);
                    end = kpre[k + 1];
                    rem = kmask[k];
                }
                b = __builtin_ctzll(rem);
                rem &= rem - 1ull;
            }
            flush(k);
        }
    }
}


// next task of a persistent kernel (wave-uniform)
__device__ __forceinline__ int64_t next_task(unsigned long long *ctr)
{
    unsigned long long t = 0;
    if ((threadIdx.x & 63) == 0) t = atomicAdd(ctr, 1ull);
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)t, 0, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(t >> 32), 0, 64);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// --------------------------------------------------------- forward: k_fg

template <int T>
struct FgShared {
    ItemShared<T> it;
    unsigned long long zb[T][kWave];   // depth bits << 32 | face
};

// foreground item: coverage (eqs 1-3 / 8) and depth test (eq 9) per sub-frame
template <int T, int SOLVER, int TWS>
__device__ __forceinline__ void fg_item(const Inst &a, FgShared<T> &sh, int e, int p, const float tau[T],
                                        float tc)
{
    const auto r = lds_rec(sh.it, e);
    const float du = pix_du<TWS>(a, p), dv = pix_dv<TWS>(a, p);
    Bary<SOLVER> bc;
    bc.setup(r, tc, du, dv);
    const unsigned long long f = (uint32_t)__float_as_int(r.at(R_F));
#pragma unroll
    for (int j = 0; j < T; ++j) {
        if (!((sh.it.m[j][e] >> p) & 1ull)) continue;
        float N[3];
        bc.eval(r, tau[j] - tc, N);
        const float D = N[0] + N[1] + N[2];
        if (!(fabsf(D) > kTauDet)) continue;
        const bool cov = D > 0.0f ? fminf(N[0], fminf(N[1], N[2])) >= 0.0f : fmaxf(N[0], fmaxf(N[1], N[2])) <= 0.0f;
        if (!cov) continue;
        float zt[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) zt[q] = fmaf(tau[j], r.at(R_A1 + q), r.at(R_A0 + q));
        const float z = fmaf(N[0], zt[0], fmaf(N[1], zt[1], N[2] * zt[2])) * rcp(D);
        // z > 0 (all vertices in front of the camera), so its bits order like its value
        atomicMin(&sh.zb[j][p], ((unsigned long long)__float_as_uint(z) << 32) | f);
    }
}

// colour of the winning face at this lane's pixel: barycentric interpolation
// of the vertex attributes (eq 9), from the same float32 record the depth
// test used (r) and the attributes at[q * NCH + c]
template <int SOLVER, class R, class A>
__device__ __forceinline__ void shade(const R &r, const A &at, float tc, float tau, const TileCtx &g, float rgb[NCH])
{
    Bary<SOLVER> bc;
    bc.setup(r, tc, g.du, g.dv);
    float N[3];
    bc.eval(r, tau - tc, N);
    const float invD = rcp(N[0] + N[1] + N[2]);
    const float w0 = N[0] * invD, w1 = N[1] * invD, w2 = N[2] * invD;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) rgb[ch] = fmaf(w0, at(0 * NCH + ch), fmaf(w1, at(1 * NCH + ch), w2 * at(2 * NCH + ch)));
}

// the winner's record is no longer staged: gather it
template <int SOLVER>
__device__ __forceinline__ void shade_gather(const Inst &a, int f, int s, const TileCtx &g, float tc, float tau,
                                             float rgb[NCH])
{
    int vid[3];
    face_verts(a, f, vid);
    FaceRec r;
    stage_rec(a, f, vid, s, g.ua, g.va, tc, kRecGeom, r);
    shade<SOLVER>(r, [&](int k) { const int q = k / NCH, c = k - q * NCH; return c < a.C ? a.attrs[(size_t)vid[q] * a.C + c] : 0.0f; },
                  tc, tau, g, rgb);
}

// TWS: 8 for a batch of 8 x 8 tiles (constant pixel offsets and masks), 0
// for the other tile shapes
template <int T, int SOLVER, int TWS>
__global__ __launch_bounds__(64) void k_fg(const Inst *__restrict__ tab, int n)
{
    __shared__ FgShared<T> sh;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const Inst a = tab[inst_of<&Inst::b_fg>(tab, n, lb)];
    const int ct = lb - a.b_fg;
    const int lane = threadIdx.x & 63;
    TileCtx g;
    tile_ctx(a, ct, g);
    const Chunk &ck = g.ck;
    if ((a.hdr->error_bits & kHdrOverflow) || ck.n <= 0) {
        if (lane == 0) {
            a.tsl[ct] = 0;
            a.fgw[ct] = 0;
        }
        return;
    }
    const uint64_t inimg = __ballot(g.inimg);
    float tau[T];
    uint32_t xbits;
    chunk_taus<T>(a, ck, tau, xbits);
    const float tc = chunk_centre<T>(tau, ck.n);
    uint64_t allow[T];
#pragma unroll
    for (int j = 0; j < T; ++j) {
        allow[j] = j < ck.n ? inimg : 0ull;
        sh.zb[j][lane] = ~0ull;
    }
    // foreground list of (chunk, tile)
    const int64_t beg = a.off[ct];
    const int n_e = a.cnt[ct];
    for (int base = 0; base < n_e; base += NB) {
        const int nb = min(NB, n_e - base);
        int cnt, pre;
        const int total = stage_items<T, TWS>(a, sh.it, prefetch(a, beg + base, nb), nb, ck.s, g, tc, tau, kRecFg, 0.0f,
                                         allow, nullptr, nullptr, cnt, pre);
        for_items<T>(sh.it, total, cnt, pre, [&](int e, int p) { fg_item<T, SOLVER, TWS>(a, sh, e, p, tau, tc); });
    }
    lds_sync();
    bool anyunc = false, anycov = false;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        if (j >= ck.n) continue;
        const int k = ck.k0 + j;
        const unsigned long long key = sh.zb[j][lane];
        const int zid = key == ~0ull ? -1 : (int)(uint32_t)key;
        anyunc = anyunc || __ballot(g.inimg && zid < 0) != 0ull;
        anycov = anycov || __ballot(g.inimg && zid >= 0) != 0ull;
        float rgb[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) rgb[ch] = 0.0f;
        if (g.inimg && zid >= 0) shade_gather<SOLVER>(a, zid, ck.s, g, tc, tau[j], rgb);
        a.vis_id[vis_index(a, g.tile, k, lane)] = g.inimg ? zid : kVisOut;
        // colour of a covered pixel; the background accumulators start at 0
        // (log-sum, zero count) and 1 (smallest non-zero 1 - A)
        const bool bgpix = !(g.inimg && zid >= 0);
        for (int sl = 0; sl < a.NS; ++sl) {
            float v = bgpix && sl == 2 ? 1.0f : 0.0f;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                if (ch == sl) v = rgb[ch];
            a.pix[pix_index(a, g.tile, k, sl, lane)] = v;
        }
    }
    if (lane == 0) {
        const int n_bg = a.cnt[(int64_t)a.NC * a.ntiles + ct];
        a.tsl[ct] = anyunc ? (n_bg + a.SL - 1) / a.SL : 0;
        // whether the (chunk, tile) has a winner, for the foreground adjoint
        a.fgw[ct] = anycov ? 1 : 0;
    }
}

// write the task list: tasks[toff[ct] + i] = (ct, i), i < tsl[ct]
__global__ void k_tasks(const Inst *__restrict__ tab, int n)
{
    const Inst a = tab[inst_of<&Inst::b_tscan3>(tab, n, blockIdx.x)];
    const int64_t ct = (int64_t)(blockIdx.x - a.b_tscan3) * blockDim.x + threadIdx.x;
    if (ct >= a.ntct) return;
    const int m = a.tsl[ct];
    const int64_t o = a.toff[ct];
    for (int i = 0; i < m; ++i)
        if (o + i < a.maxtasks) a.tasks[o + i] = ((uint64_t)ct << 32) | (uint32_t)i;
}

// first background task of every instance in the batch's task numbering
__global__ void k_tprefix(const Inst *__restrict__ tab, int n, int64_t *__restrict__ tprefix)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t s = 0;
    for (int i = 0; i < n; ++i) {
        tprefix[i] = s;
        const Inst a = tab[i];
        if (!(a.hdr->error_bits & kHdrOverflow)) s += min(a.hdr->ntasks, a.maxtasks);
    }
    tprefix[n] = s;
}

// instance owning batch task t (tprefix ascending, t < tprefix[n])
__device__ __forceinline__ int task_inst(const int64_t *__restrict__ tprefix, int n, int64_t t)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tprefix[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// --------------------------------------------------------- forward: k_bg

template <int T>
struct BgShared {
    ItemShared<T> it;
    double lsum[T][kWave];  // sum of log2(1 - A) over non-zero factors (hundreds of
                            // factors per pixel near a silhouette: summed in double)
    int nz[T][kWave];       // number of zero factors (A == 1)
    unsigned omin[T][kWave];  // smallest non-zero factor 1 - A below 1/2, else 1 (float bits; min on
                              // the bits orders non-negative floats)
    int ppre[kWave + 1];    // items regrouped by pixel: first item of each pixel
    uint64_t pe[kWave];     // and its staged entries
};

// background item: eqs 10, 13-15, accumulated as log2(1 - A) per sub-frame
// of the chunk, with the zero factors (A == 1) counted: into ls / nz (ACC)
// or straight into the LDS sums
// (xk: the keyframe X shared by every sub-frame of the chunk, or -1)
template <int T, int SOLVER, bool ACC>
__device__ __forceinline__ void bg_item_fwd(const Inst &a, BgShared<T> &sh, int e, int p, const float tau[T],
                                            uint32_t xbits, int xk, float tc, double (&ls)[T], int (&nz)[T],
                                            float (&om_lo)[T])
{
    const auto r = lds_rec(sh.it, e);
    const float du = pix_du(a, p), dv = pix_dv(a, p);
    Bary<SOLVER> bc;
    bc.setup(r, tc, du, dv);
    KEdges ke;
    if (xk >= 0) kedges(r, xk, tc, ke);
#pragma unroll
    for (int j = 0; j < T; ++j) {
        if (!((sh.it.m[j][e] >> p) & 1ull)) continue;
        float N[3];
        bc.eval(r, tau[j] - tc, N);
        const float D = N[0] + N[1] + N[2];
        if (!(fabsf(D) > kTauDet)) continue;
        const int X = (xbits >> j) & 1u;
        if (xk < 0) kedges(r, X, tc, ke);
        BgEval b;
        bg_eval(r, ke, tc, tau[j], X, N, rcp(D), du, dv, b);
        if (!(b.d <= a.dmax)) continue;
        const float A = exp2f(b.d * a.neg_log2e_over_delta);
        const float om = one_minus_exp_neg(b.d * a.inv_delta, A);
        if (ACC) {
            if (om > 0.0f) {
                ls[j] += (double)log2_one_minus(A, om);
                if (om < 0.5f) om_lo[j] = fminf(om_lo[j], om);
            } else {
                ++nz[j];
            }
        } else {
            if (om > 0.0f) {
                atomicAdd(&sh.lsum[j][p], (double)log2_one_minus(A, om));
                if (om < 0.5f) atomicMin(&sh.omin[j][p], __float_as_uint(om));
            } else {
                atomicAdd(&sh.nz[j][p], 1);
            }
        }
    }
}

// RUNS: items grouped by pixel in per-lane runs (wide halo) or dealt one per
// lane in entry order
template <int T, int SOLVER, bool RUNS>
__global__ __launch_bounds__(64, 4) void k_bg(const Inst *__restrict__ tab, int n, const int64_t *__restrict__ tprefix)
{
    __shared__ BgShared<T> sh;
    const int lane = threadIdx.x & 63;
    // batch task tb goes to wave tb mod G; the instance record is loaded once
    // per (wave, instance)
    const int64_t G = gridDim.x;
    for (int ii = 0; ii < n; ++ii) {
        const int64_t lo = tprefix[ii], hi = tprefix[ii + 1];
        int64_t tb = lo + (((int64_t)blockIdx.x - lo) % G + G) % G;
        if (tb >= hi) continue;
        const Inst &a = tab[ii];
    for (; tb < hi; tb += G) {
        const int64_t t = tb - lo;
        const uint64_t task = a.tasks[t];
        const int ct = (int)(task >> 32);
        const int slice = (int)(uint32_t)task;
        TileCtx g;
        tile_ctx(a, ct, g);
        const Chunk &ck = g.ck;
        float tau[T];
        uint32_t xbits;
        chunk_taus<T>(a, ck, tau, xbits);
        const float tc = chunk_centre<T>(tau, ck.n);
        // keyframe X of every sub-frame of the chunk, when they share one
        const int xk = xbits == 0u ? 0 : (xbits == (1u << ck.n) - 1u ? 1 : -1);
        uint64_t unc[T];
        lds_sync();
#pragma unroll
        for (int j = 0; j < T; ++j) {
            const int vid = j < ck.n ? a.vis_id[vis_index(a, g.tile, ck.k0 + j, lane)] : kVisOut;
            unc[j] = __ballot(vid == -1);
            sh.lsum[j][lane] = 0.0;
            sh.nz[j][lane] = 0;
            sh.omin[j][lane] = __float_as_uint(1.0f);
        }
        const int64_t idx = (int64_t)a.NC * a.ntiles + ct;
        const int64_t beg = a.off[idx];
        const int n_e = a.cnt[idx];
        const int e0 = slice * a.SL, e1 = min(n_e, e0 + a.SL);
        Pref pf = prefetch(a, beg + e0, min(NB, e1 - e0));
        for (int base = e0; base < e1; base += NB) {
            const int nb = min(NB, e1 - base);
            const Pref cur = pf;
            if (base + NB < e1) pf = prefetch(a, beg + base + NB, min(NB, e1 - base - NB));
            int cnt, pre;
            const int total =
                stage_items<T>(a, sh.it, cur, nb, ck.s, g, tc, tau, kRecBg, a.halo, unc, nullptr, nullptr, cnt, pre);
            if (!RUNS) {
                // items in entry order, one per lane, each adding its factors
                // to LDS (few lanes share a pixel: best when faces reach few
                // pixels)
                double ls[T];
                int nzc[T];
                float oml[T];
                for_items<T>(sh.it, total, cnt, pre, [&](int e, int p) {
                    bg_item_fwd<T, SOLVER, false>(a, sh, e, p, tau, xbits, xk, tc, ls, nzc, oml);
                });
                continue;
            }
            // regroup the items by pixel: a lane's run then adds up one
            // pixel's factors over several faces before touching LDS (best
            // when faces reach many pixels, so that a pixel has many items)
            uint64_t pe = 0;
            for (int e = 0; e < nb; ++e) pe |= ((sh.it.U[e] >> lane) & 1ull) << e;
            const int cp = __popcll(pe);
            const int inclp = wave_incl_scan(cp);
            sh.pe[lane] = pe;
            sh.ppre[lane] = inclp - cp;
            if (lane == kWave - 1) sh.ppre[kWave] = inclp;
            lds_sync();
            double ls[T];
            int nzc[T];
            float oml[T];
#pragma unroll
            for (int j = 0; j < T; ++j) {
                ls[j] = 0.0;
                nzc[j] = 0;
                oml[j] = 1.0f;
            }
            for_runs(
                kSeqBgFwd, total, inclp - cp, sh.ppre, sh.pe,
                [&](int p, int e) { bg_item_fwd<T, SOLVER, true>(a, sh, e, p, tau, xbits, xk, tc, ls, nzc, oml); },
                [&](int p) {
#pragma unroll
                    for (int j = 0; j < T; ++j) {
                        if (ls[j] != 0.0) atomicAdd(&sh.lsum[j][p], ls[j]);
                        if (nzc[j]) atomicAdd(&sh.nz[j][p], nzc[j]);
                        if (oml[j] < 1.0f) atomicMin(&sh.omin[j][p], __float_as_uint(oml[j]));
                        ls[j] = 0.0;
                        nzc[j] = 0;
                        oml[j] = 1.0f;
                    }
                });
            lds_sync();
        }
        lds_sync();
#pragma unroll
        for (int j = 0; j < T; ++j) {
            if (!((unc[j] >> lane) & 1ull)) continue;
            const float ls = (float)sh.lsum[j][lane];
            const int nz = sh.nz[j][lane];
            const unsigned om = sh.omin[j][lane];
            if (ls != 0.0f) unsafeAtomicAdd(&a.pix[pix_index(a, g.tile, ck.k0 + j, 0, lane)], ls);
            if (nz) atomicAdd((int *)&a.pix[pix_index(a, g.tile, ck.k0 + j, 1, lane)], nz);
            if (om < __float_as_uint(1.0f)) atomicMin((unsigned *)&a.pix[pix_index(a, g.tile, ck.k0 + j, 2, lane)], om);
        }
    }
    }
}

// ---------------------------------------------------- forward: k_resolve

// image = mean over the K sub-frames of the winner's colour (premultiplied,
// alpha 1) or, where uncovered, alpha = 1 - prod (1 - A) (eq 15)
constexpr int kResWaves = 4;   // waves per tile in the resolve (interleaved sub-frames)

__global__ __launch_bounds__(64 * kResWaves) void k_resolve(const Inst *__restrict__ tab, int n)
{
    __shared__ double part[kResWaves - 1][NCH + 1][kWave];
    const Inst &a = tab[inst_of<&Inst::b_res>(tab, n, blockIdx.x)];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int tile = blockIdx.x - a.b_res;
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    int px, py;
    tile_pixel(a, tx, ty, lane, px, py);
    const bool in = px < a.W && py < a.H;
    // wave w sums sub-frames w, w + kResWaves, ... in double
    double acc[NCH + 1];
#pragma unroll
    for (int ch = 0; ch <= NCH; ++ch) acc[ch] = 0.0;
    if (in) {
        // the record's slots are loaded with the visibility, not after it,
        // so that a sub-frame waits for one round of loads, not two (a
        // background pixel reads the slots past its two as well)
        const int nl = max(a.C, 2);
#pragma unroll 2
        for (int k = w; k < a.K; k += kResWaves) {
            const int vid = a.vis_id[vis_index(a, tile, k, lane)];
            float v[NCH];
#pragma unroll
            for (int sl = 0; sl < NCH; ++sl) v[sl] = sl < nl ? a.pix[pix_index(a, tile, k, sl, lane)] : 0.0f;
            if (vid >= 0) {
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch)
                    if (ch < a.C) acc[ch] += (double)v[ch];
                acc[NCH] += 1.0;
            } else {
                const int nz = __float_as_int(v[1]);
                acc[NCH] += nz > 0 ? 1.0 : (double)(1.0f - exp2f(v[0]));
            }
        }
    }
    if (w > 0) {
#pragma unroll
        for (int ch = 0; ch <= NCH; ++ch) part[w - 1][ch][lane] = acc[ch];
    }
    __syncthreads();
    if (w > 0 || !in) return;
#pragma unroll
    for (int q = 0; q < kResWaves - 1; ++q)
#pragma unroll
        for (int ch = 0; ch <= NCH; ++ch) acc[ch] += part[q][ch][lane];
    float *__restrict__ image = a.image;
    const bool bad = (a.hdr->error_bits & kHdrOverflow) != 0;
    const double invK = 1.0 / (double)a.K;
    const size_t plane = (size_t)a.H * a.W, at = (size_t)py * a.W + px;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
        if (ch < a.C) image[ch * plane + at] = bad ? __builtin_nanf("") : (float)(acc[ch] * invK);
    image[a.C * plane + at] = bad ? __builtin_nanf("") : (float)(acc[NCH] * invK);
}

// ---------------------------------------------------------------- adjoint



// Gradient accumulation.  Item contributions go to an LDS table keyed by
// vertex (open addressing): per vertex, dL/d(x, y) at the chunk's two
// keyframes and, in the foreground, dL/d(attributes).  Neighbouring faces
// share vertices, so the table reaches global memory with one atomic per
// (vertex, value) when it fills up or the task ends, instead of one per
// (face, vertex, value).
// V: the accumulator type (double tables measured faster in the foreground
// adjoint; in the background adjoint their LDS would cost occupancy)
template <int NV, int NS, class V = float>
struct VTab {
    static_assert((NS & (NS - 1)) == 0 && NS >= 64 && NS <= 1024, "slot count");
    static constexpr int kSlots = NS;
    static constexpr int kLoad = NS * 3 / 4;   // flush before a batch could push the table past this
    static constexpr int kShift = NS == 64 ? 26 : NS == 128 ? 25 : NS == 256 ? 24 : NS == 512 ? 23 : 22;
    int key[NS];               // vertex index, -1 = empty
    V g[NV][NS];               // 0-3: keyframe s (x, y), keyframe s + 1 (x, y); 4+: attributes
};

template <int NV, int NS, class V>
__device__ __forceinline__ void vt_clear(VTab<NV, NS, V> &vt)
{
    const int lane = threadIdx.x & 63;
    for (int i = lane; i < NS; i += kWave) {
        vt.key[i] = -1;
#pragma unroll
        for (int k = 0; k < NV; ++k) vt.g[k][i] = V(0);
    }
}

template <int NS>
__device__ __forceinline__ int hash_vertex(int v)
{
    return (int)(((uint32_t)v * 2654435761u) >> VTab<1, NS>::kShift);
}

__device__ __forceinline__ int wave_sum_int(int x)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// Replace the staged entries' vertex indices vs[e][q] (e < nb) by their table
// slots, inserting new vertices; returns the number of new keys.  The caller
// keeps the table below kLoad of its NS slots, so a free slot is always found.
template <int NV, int NS, class V>
__device__ __forceinline__ int vt_bind(VTab<NV, NS, V> &vt, int (*vs)[3], int nb)
{
    const int lane = threadIdx.x & 63;
    int fresh = 0;
    lds_sync();
    if (lane < nb) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int v = vs[lane][q];
            int h = hash_vertex<NS>(v), slot = -1;
            for (int probe = 0; probe < NS; ++probe) {
                const int old = atomicCAS(&vt.key[h], -1, v);
                if (old == -1 || old == v) {
                    slot = h;
                    fresh += old == -1 ? 1 : 0;
                    break;
                }
                h = (h + 1) & (NS - 1);
            }
            vs[lane][q] = slot;
        }
    }
    lds_sync();
    return wave_sum_int(fresh);
}

template <int NV, int NS, class V>
__device__ __forceinline__ void vt_add(VTab<NV, NS, V> &vt, int slot, int k, float v)
{
    if (v != 0.0f && slot >= 0) atomicAdd(&vt.g[k][slot], (V)v);
}

// Add the table to the keyframe (and attribute) gradients and clear it.
template <int NV, int NS, class V>
__device__ __forceinline__ void vt_flush(VTab<NV, NS, V> &vt, int s, const Inst &a)
{
    const int lane = threadIdx.x & 63;
    const int shift = a.det ? det_shift(a) : 0;
    const int64_t n1 = (int64_t)(a.S + 1) * a.V * 2;
    lds_sync();
    for (int i = lane; i < NS; i += kWave) {
        const int v = vt.key[i];
        if (v < 0) continue;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const size_t at = ((size_t)(s + (k >> 1)) * a.V + v) * 2 + (k & 1);
            if (a.det) {
                if (vt.g[k][i] != V(0)) det_add(a, a.gfx + at, (double)vt.g[k][i], shift);
            } else {
                const float g = (float)vt.g[k][i];
                if (g != 0.0f) unsafeAtomicAdd(a.gkf + at, g);
            }
            vt.g[k][i] = V(0);
        }
#pragma unroll
        for (int c = 0; c < NV - 4; ++c) {
            if (c < a.C) {
                const size_t at = (size_t)v * a.C + c;
                if (a.det) {
                    if (vt.g[4 + c][i] != V(0)) det_add(a, a.gfx + n1 + at, (double)vt.g[4 + c][i], shift);
                } else {
                    const float g = (float)vt.g[4 + c][i];
                    if (g != 0.0f) unsafeAtomicAdd(a.grad_attrs + at, g);
                }
            }
            vt.g[4 + c][i] = V(0);
        }
        vt.key[i] = -1;
    }
    lds_sync();
}

// ------------------------------------------------------- backward: k_fg_bwd

// winning faces staged per batch in the foreground adjoint: half the list
// walk's batch, which keeps the wave's LDS near 9 KB (16 waves per compute
// unit) with a 64-slot vertex table that one batch cannot overfill
constexpr int NBF = 16;

template <int T>
struct FgBwdShared {
    ItemShared<T, NBF> it;    // staged winning faces, their (pixel, sub-frame) masks and items
    float at[3 * NCH][NBF];   // their vertex attributes
    int vslot[NBF][3];        // their vertices: index, then vertex-table slot
    VTab<4 + NCH, 64, double> vt;    // at most 3 NBF new vertices per batch
    float gI[NCH][kWave];     // dL/dcolour of each pixel, already divided by K
};

// Foreground adjoint of one item (pixel p of staged face e, at every
// sub-frame of the chunk where e wins p): colour = sum_i w_i c_i, dL/dw
// through the static solve (dw = -F^-1 dF w), dL/dc_i = w_i dL/dcolour.
// Adds to acc: per vertex q, dL/d(x_s, y_s, x_s+1, y_s+1) at 4 q and
// dL/d(attributes) at 12 + NCH q.
template <int T, int SOLVER>
__device__ __forceinline__ void fg_item_bwd(const Inst &a, FgBwdShared<T> &sh, int e, int p, const float tau[T],
                                            float tc, float (&acc)[12 + 3 * NCH])
{
    const auto r = lds_rec(sh.it, e);
    const float du = pix_du(a, p), dv = pix_dv(a, p);
    float gI[NCH], gw[3], ws[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) gI[ch] = sh.gI[ch][p];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        gw[q] = 0.0f;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) gw[q] = fmaf(gI[ch], sh.at[q * NCH + ch][e], gw[q]);
    }
    Bary<SOLVER> bc;
    bc.setup(r, tc, du, dv);
#pragma unroll
    for (int j = 0; j < T; ++j) {
        if (!((sh.it.m[j][e] >> p) & 1ull)) continue;
        const float t = tau[j] - tc;
        float N[3];
        bc.eval(r, t, N);
        const float invD = rcp(N[0] + N[1] + N[2]);
        const float w[3] = {N[0] * invD, N[1] * invD, N[2] * invD};
        float xt[3], yt[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            xt[q] = fmaf(t, r.at(R_DX + q), r.at(R_XC + q));
            yt[q] = fmaf(t, r.at(R_DY + q), r.at(R_YC + q));
        }
        const float gxs = fmaf(gw[0], yt[1] - yt[2], fmaf(gw[1], yt[2] - yt[0], gw[2] * (yt[0] - yt[1]))) * invD;
        const float gys = fmaf(gw[0], xt[2] - xt[1], fmaf(gw[1], xt[0] - xt[2], gw[2] * (xt[1] - xt[0]))) * invD;
        const float t1 = tau[j], t0 = 1.0f - tau[j];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const float gx = -w[q] * gxs, gy = -w[q] * gys;
            acc[q * 4 + 0] = fmaf(t0, gx, acc[q * 4 + 0]);
            acc[q * 4 + 1] = fmaf(t0, gy, acc[q * 4 + 1]);
            acc[q * 4 + 2] = fmaf(t1, gx, acc[q * 4 + 2]);
            acc[q * 4 + 3] = fmaf(t1, gy, acc[q * 4 + 3]);
            ws[q] += w[q];
        }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) acc[12 + q * NCH + ch] = fmaf(ws[q], gI[ch], acc[12 + q * NCH + ch]);
}

template <int T, int SOLVER>
__global__ __launch_bounds__(64) void k_fg_bwd(const Inst *__restrict__ tab, int n)
{
    __shared__ FgBwdShared<T> sh;
    // one wave per (group of up to a.fgg consecutive chunks of one segment,
    // tile): the chunks share the keyframe pair, so one vertex table (and
    // one flush) serves them, and the tile's colour gradient is loaded once;
    // groups stay short so that the chunks' latencies are not all serialized
    // in one wave
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const Inst &a = tab[inst_of<&Inst::b_fgb>(tab, n, lb)];
    const int gti = lb - a.b_fgb;
    const int grp = gti / a.ntiles, tile = gti - grp * a.ntiles;
    const int gps = (a.CPS + a.fgg - 1) / a.fgg;   // groups per segment
    const int seg = grp / gps, gi = grp - seg * gps;
    const int lane = threadIdx.x & 63;
    if (a.hdr->error_bits & kHdrOverflow) return;
    const int c0 = seg * a.CPS + gi * a.fgg, c1 = min(c0 + a.fgg, (seg + 1) * a.CPS);
    bool any = false;
    for (int c = c0; c < c1 && !any; ++c) any = a.fgw[(int64_t)c * a.ntiles + tile] != 0;
    if (!any) return;   // no chunk of the segment has a winner here
    // the tile's colour gradient: loaded here, stored to LDS once the first
    // chunk's visibility loads are in flight too
    float gIr[NCH];
    bool gcol = false, gstored = false;
    {
        const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
        int px, py;
        tile_pixel(a, tx, ty, lane, px, py);
        const bool inimg = px < a.W && py < a.H;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
            gIr[ch] = inimg && ch < a.C ? a.grad_image[((size_t)ch * a.H + py) * a.W + px] * a.invK : 0.0f;
    }
    vt_clear(sh.vt);
    int used = 0;
    for (int c = c0; c < c1; ++c) {
        const int ct = c * a.ntiles + tile;
        if (!a.fgw[ct]) continue;
        TileCtx g;
        tile_ctx(a, ct, g);
        const Chunk &ck = g.ck;
        if (ck.n <= 0) continue;
        // (pixel, sub-frame) pairs with a winner and a colour gradient
        int vid[T];
        uint64_t pend[T];
        bool anyfg = false;
#pragma unroll
        for (int j = 0; j < T; ++j) vid[j] = j < ck.n ? a.vis_id[vis_index(a, g.tile, ck.k0 + j, lane)] : kVisOut;
        if (!gstored) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                sh.gI[ch][lane] = gIr[ch];
                gcol = gcol || gIr[ch] != 0.0f;
            }
            gstored = true;
        }
#pragma unroll
        for (int j = 0; j < T; ++j) {
            pend[j] = __ballot(gcol && vid[j] >= 0);
            anyfg = anyfg || pend[j] != 0ull;
        }
        if (!anyfg) continue;
        float tau[T];
        uint32_t xbits;
        chunk_taus<T>(a, ck, tau, xbits);
        const float tc = chunk_centre<T>(tau, ck.n);

        // Only the winning faces are staged (the list is not walked): the first
        // pending pair's face becomes the next entry and takes every pending pair
        // of that face, as its per-sub-frame pixel masks; a batch of NBF entries
        // (or the last one) is staged and its items (entry, pixel) are run.
        uint64_t mown[T];         // masks of entry `lane` of the batch being gathered
#pragma unroll
        for (int j = 0; j < T; ++j) mown[j] = 0ull;
        int sel = 0;              // its face
        int ne = 0;
        for (;;) {
            int j0 = -1, v0 = 0;
#pragma unroll
            for (int j = 0; j < T; ++j)
                if (j0 < 0 && pend[j] != 0ull) {
                    j0 = j;
                    v0 = vid[j];
                }
            if (j0 >= 0) {
                uint64_t pm = 0;
#pragma unroll
                for (int j = 0; j < T; ++j)
                    if (j == j0) pm = pend[j];
                const int f = __shfl(v0, __builtin_ctzll(pm), 64);
#pragma unroll
                for (int j = 0; j < T; ++j) {
                    const uint64_t hit = __ballot(((pend[j] >> lane) & 1ull) && vid[j] == f);
                    pend[j] &= ~hit;
                    if (lane == ne) mown[j] = hit;
                }
                if (lane == ne) sel = f;
                ++ne;
            }
            if (ne == NBF || (j0 < 0 && ne > 0)) {
                if (used + 3 * ne > sh.vt.kLoad) {
                    vt_flush(sh.vt, ck.s, a);
                    used = 0;
                }
                lds_sync();
                int cnt = 0;
                if (lane < ne) {
                    int vq[3];
                    face_verts(a, sel, vq);
                    FaceRec r;
                    stage_rec(a, sel, vq, ck.s, g.ua, g.va, tc, kRecGeom, r);
                    store_rec(sh.it, lane, r);
                    uint64_t U = 0;
#pragma unroll
                    for (int j = 0; j < T; ++j) {
                        sh.it.m[j][lane] = mown[j];
                        U |= mown[j];
                    }
                    sh.it.U[lane] = U;
                    cnt = __popcll(U);
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        sh.vslot[lane][q] = vq[q];
#pragma unroll
                        for (int ch = 0; ch < NCH; ++ch)
                            sh.at[q * NCH + ch][lane] = ch < a.C ? a.attrs[(size_t)vq[q] * a.C + ch] : 0.0f;
                    }
                }
                const int incl = wave_incl_scan(cnt);
                const int pre = incl - cnt;
                if (lane <= ne) sh.it.pre[lane] = pre;
                const int total = __shfl(incl, 63, 64);
                used += vt_bind(sh.vt, sh.vslot, ne);
                float acc[12 + 3 * NCH];
#pragma unroll
                for (int k = 0; k < 12 + 3 * NCH; ++k) acc[k] = 0.0f;
                for_runs(
                    kSeqFg, total, pre, sh.it.pre, sh.it.U, [&](int e, int p) { fg_item_bwd<T, SOLVER>(a, sh, e, p, tau, tc, acc); },
                    [&](int e) {
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            const int slot = sh.vslot[e][q];
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                vt_add(sh.vt, slot, k, acc[q * 4 + k]);
                                acc[q * 4 + k] = 0.0f;
                            }
#pragma unroll
                            for (int ch = 0; ch < NCH; ++ch) {
                                vt_add(sh.vt, slot, 4 + ch, acc[12 + q * NCH + ch]);
                                acc[12 + q * NCH + ch] = 0.0f;
                            }
                        }
                    });
                lds_sync();
#pragma unroll
                for (int j = 0; j < T; ++j) mown[j] = 0ull;
                ne = 0;
            }
            if (j0 < 0) break;
        }
    }
    vt_flush(sh.vt, seg, a);
}

// ------------------------------------------------------- backward: k_bg_bwd

template <int T>
struct BgBwdShared {
    ItemShared<T> it;
    int vslot[NB][3];         // staged entries' vertices: index, then vertex-table slot
    VTab<4, 128> vt;
    float P[T][kWave];        // forward product over the non-zero factors if there is none
                              // of A == 1; minus the product if there is one; -0 if more
    float gal[kWave];         // dL/dalpha of each pixel, already divided by K
    float reach[T][kMaxTileH];  // per tile row: squared reach of its pixels' terms (-1: none)
};

// Background adjoint of one item: dalpha/dA_j = prod_{m != j}(1 - A_m),
// dA/dd = -A/delta, then the chain through d = |p - p*|^2, the closest point
// (edge parameter where unclamped), q = F(X) w and w(tau) (dw = -F^-1 dF w).
// Adds dL/d(keyframe s, s+1 positions) of the entry's vertices to gK
// (vertex q: x_s, y_s, x_s+1, y_s+1 at 4 q).
template <int T, int SOLVER>
__device__ __forceinline__ void bg_item_bwd(const Inst &a, BgBwdShared<T> &sh, int e, int p,
                                            const float tau[T], uint32_t xbits, float tc, float (&gK)[12])
{
    const auto r = lds_rec(sh.it, e);
    const float du = pix_du(a, p), dv = pix_dv(a, p);
    const float galpha = sh.gal[p];
    Bary<SOLVER> bc;
    bc.setup(r, tc, du, dv);
    KEdges ke;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        if (!((sh.it.m[j][e] >> p) & 1ull)) continue;
        const float t = tau[j] - tc;
        float N[3];
        bc.eval(r, t, N);
        const float D = N[0] + N[1] + N[2];
        if (!(fabsf(D) > kTauDet)) continue;
        const float invD = rcp(D);
        const int X = (xbits >> j) & 1u;
        kedges(r, X, tc, ke);
        BgEval b;
        bg_eval(r, ke, tc, tau[j], X, N, invD, du, dv, b);
        if (!(b.d <= a.dmax)) continue;
        const float A = exp2f(b.d * a.neg_log2e_over_delta);
        const float om = one_minus_exp_neg(b.d * a.inv_delta, A);
        // product over the other factors: the item's own factor divided out,
        // or the product of the rest when the item holds the one zero factor
        const float P = sh.P[j][p];
        const float Pe = !signbit(P) ? P * rcp(om) : (om > 0.0f ? 0.0f : -P);
        // a term of weight prod_{m != j}(1 - A_m) A_j below kAdjWMin is left out
        if (!(Pe * A >= kAdjWMin)) continue;
        const float gd = -galpha * Pe * A * a.inv_delta;
        const float gpx = 2.0f * gd * (b.psx - du), gpy = 2.0f * gd * (b.psy - dv);
        float xt[3], yt[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            xt[q] = fmaf(t, r.at(R_DX + q), r.at(R_XC + q));
            yt[q] = fmaf(t, r.at(R_DY + q), r.at(R_YC + q));
        }
        // per-vertex gradient at tau (gt) and at keyframe X (gk)
        float gtx[3], gty[3], gkx[3], gky[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const float wq = b.be == q ? 1.0f - b.sg : (b.be == (q + 2) % 3 ? b.sg : 0.0f);
            gtx[q] = wq * gpx;
            gty[q] = wq * gpy;
            gkx[q] = 0.0f;
            gky[q] = 0.0f;
        }
        const bool interior = !(b.sr < 0.0f) && !(b.sr > 1.0f);
        if (interior) {
            const int ea = b.be;
            const float *Ex = ke.Ex, *Ey = ke.Ey, *iee3 = ke.iee;
            const float exs = ea == 0 ? Ex[0] : (ea == 1 ? Ex[1] : Ex[2]);
            const float eys = ea == 0 ? Ey[0] : (ea == 1 ? Ey[1] : Ey[2]);
            const float iee = ea == 0 ? iee3[0] : (ea == 1 ? iee3[1] : iee3[2]);
            // edge ea+2 (from vertex ea+2 back to ea): v_{ea+2} - v_ea = -E_{ea+2}
            const float e2x = ea == 0 ? Ex[2] : (ea == 1 ? Ex[0] : Ex[1]);
            const float e2y = ea == 0 ? Ey[2] : (ea == 1 ? Ey[0] : Ey[1]);
            const float xa = ea == 0 ? xt[0] : (ea == 1 ? xt[1] : xt[2]);
            const float ya = ea == 0 ? yt[0] : (ea == 1 ? yt[1] : yt[2]);
            const float xb = ea == 0 ? xt[1] : (ea == 1 ? xt[2] : xt[0]);
            const float yb = ea == 0 ? yt[1] : (ea == 1 ? yt[2] : yt[0]);
            const float gsig = fmaf(gpx, xb - xa, gpy * (yb - ya));
            const float rx = b.rx, ry = b.ry;
            const float grx = gsig * exs * iee, gry = gsig * eys * iee;
            const float gex = gsig * fmaf(-2.0f * b.sr, exs, rx) * iee;
            const float gey = gsig * fmaf(-2.0f * b.sr, eys, ry) * iee;
            // dL/dw_i = g_r . (v_i - v_ea): 0, E_ea, -E_{ea+2} for i = ea, ea+1, ea+2
            const float g1 = fmaf(grx, exs, gry * eys), g2 = -fmaf(grx, e2x, gry * e2y);
            float gwq[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const bool isa = ea == q, isb = ea == (q + 2) % 3;
                gkx[q] = fmaf(b.w[q], grx, isa ? -grx - gex : (isb ? gex : 0.0f));
                gky[q] = fmaf(b.w[q], gry, isa ? -gry - gey : (isb ? gey : 0.0f));
                gwq[q] = isa ? 0.0f : (isb ? g1 : g2);
            }
            const float gxs = fmaf(gwq[0], yt[1] - yt[2], fmaf(gwq[1], yt[2] - yt[0], gwq[2] * (yt[0] - yt[1]))) * invD;
            const float gys = fmaf(gwq[0], xt[2] - xt[1], fmaf(gwq[1], xt[0] - xt[2], gwq[2] * (xt[1] - xt[0]))) * invD;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                gtx[q] = fmaf(-b.w[q], gxs, gtx[q]);
                gty[q] = fmaf(-b.w[q], gys, gty[q]);
            }
        }
        const float t1 = tau[j], t0 = 1.0f - tau[j];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            gK[q * 4 + 0] += fmaf(t0, gtx[q], X ? 0.0f : gkx[q]);
            gK[q * 4 + 1] += fmaf(t0, gty[q], X ? 0.0f : gky[q]);
            gK[q * 4 + 2] += fmaf(t1, gtx[q], X ? gkx[q] : 0.0f);
            gK[q * 4 + 3] += fmaf(t1, gty[q], X ? gky[q] : 0.0f);
        }
    }
}

// WPS: waves per SIMD the register allocation targets.  4 spills some
// registers but hides more latency, which pays off when faces reach many
// pixels (long item runs); 3 is better otherwise.
template <int T, int SOLVER, int WPS>
__global__ __launch_bounds__(64, WPS) void k_bg_bwd(const Inst *__restrict__ tab, int n)
{
    __shared__ BgBwdShared<T> sh;
    const int lane = threadIdx.x & 63;
    vt_clear(sh.vt);
    // tasks vary more in cost here than in the forward (pixels without
    // gradient drop out), so waves take them from a counter per instance,
    // moving through the instances in order.  A wave takes a unit of
    // bwd_merge consecutive tasks and runs the consecutive slices of one
    // (chunk, tile) among them as one range: fewer visibility reads, table
    // flushes and counter atomics where faces reach few pixels.
    for (int ii = 0; ii < n; ++ii) {
        const Inst &a = tab[ii];
        if (a.hdr->error_bits & kHdrOverflow) continue;
        const int64_t ntasks = min(a.hdr->ntasks, a.maxtasks);
        const int MB = a.bwd_merge;
        const int64_t nunits = (ntasks + MB - 1) / MB;
        const float halo2 = a.halo * a.halo, reach_pad = 1e-3f / a.inv_delta + 1e-8f;
    for (;;) {
        const int64_t u = next_task(&a.hdr->bwd_task_ctr);
        if (u >= nunits) break;
        const int64_t tend = min(u * MB + MB, ntasks);
    for (int64_t t = u * MB; t < tend;) {
        const uint64_t task = a.tasks[t];
        const int ct = (int)(task >> 32);
        const int slice = (int)(uint32_t)task;
        int64_t t2 = t + 1;
        while (t2 < tend && (int)(a.tasks[t2] >> 32) == ct) ++t2;
        const int nsl = (int)(t2 - t);
        t = t2;
        TileCtx g;
        tile_ctx(a, ct, g);
        const Chunk &ck = g.ck;
        const float gal = g.inimg ? a.grad_image[((size_t)a.C * a.H + g.py) * a.W + g.px] * a.invK : 0.0f;
        float tau[T];
        uint32_t xbits;
        chunk_taus<T>(a, ck, tau, xbits);
        const float tc = chunk_centre<T>(tau, ck.n);
        uint64_t bgm[T];
        bool anybg = false;
        lds_sync();
        sh.gal[lane] = gal;
#pragma unroll
        for (int j = 0; j < T; ++j) {
            int vid = kVisOut;
            float P = 0.0f, om_lo = 1.0f;
            int nz = 0;
            if (j < ck.n) {
                const int k = ck.k0 + j;
                vid = a.vis_id[vis_index(a, g.tile, k, lane)];
                if (vid == -1) {
                    P = exp2f(a.pix[pix_index(a, g.tile, k, 0, lane)]);
                    nz = __float_as_int(a.pix[pix_index(a, g.tile, k, 1, lane)]);
                    om_lo = fminf(a.pix[pix_index(a, g.tile, k, 2, lane)], 0.5f);
                }
            }
            sh.P[j][lane] = nz == 0 ? P : (nz == 1 ? -P : -0.0f);
            // every term's weight prod_{m != j}(1 - A_m) A_j is at most
            // P / min(min(1 - A), 1/2): below kAdjWMin the pixel-sub-frame is
            // skipped; with two zero factors every weight is 0
            const bool live = nz == 1 || (nz == 0 && !(P < kAdjWMin * om_lo));
            const bool act = vid == -1 && gal != 0.0f && live;
            bgm[j] = __ballot(act);
            anybg = anybg || bgm[j] != 0ull;
            // squared reach of the pixel's terms: with no zero factor a term's
            // weight is P A / (1 - A) = P / (exp(d / delta) - 1), at least
            // kAdjWMin only for d <= delta ln(1 + P / kAdjWMin); with one zero
            // factor only that factor's own term (d = 0) has weight.  The
            // margin (1%, 1e-3 delta, 1e-8) is far above float rounding, so no
            // term the weight test keeps is cut off; the maximum over the tile
            // row grows the faces' boxes in staging
            float rr = -1.0f;
            if (act)
                rr = nz == 0 ? fminf(halo2, fmaf(log1pf(P * (1.0f / kAdjWMin)) / a.inv_delta, 1.01f, reach_pad))
                             : reach_pad;
            for (int o = 1; o < a.tw; o <<= 1) rr = fmaxf(rr, __shfl_xor(rr, o, 64));
            if ((lane & (a.tw - 1)) == 0) sh.reach[j][lane / a.tw] = rr;
        }
        if (!anybg) continue;
        const int64_t idx = (int64_t)a.NC * a.ntiles + ct;
        const int64_t beg = a.off[idx];
        const int n_e = a.cnt[idx];
        const int e0 = slice * a.SL, e1 = min(n_e, e0 + nsl * a.SL);
        int used = 0;
        Pref pf = prefetch(a, beg + e0, min(NB, e1 - e0));
        for (int base = e0; base < e1; base += NB) {
            const int nb = min(NB, e1 - base);
            const Pref cur = pf;
            if (base + NB < e1) pf = prefetch(a, beg + base + NB, min(NB, e1 - base - NB));
            if (used + 3 * nb > sh.vt.kLoad) {
                vt_flush(sh.vt, ck.s, a);
                used = 0;
            }
            int cnt, pre;
            const int total = stage_items<T>(a, sh.it, cur, nb, ck.s, g, tc, tau, kRecBg, a.halo, bgm, nullptr,
                                             sh.vslot, cnt, pre, sh.reach);
            used += vt_bind(sh.vt, sh.vslot, nb);
            float gK[12];
#pragma unroll
            for (int q = 0; q < 12; ++q) gK[q] = 0.0f;
            for_runs(
                a.seq_bg, total, pre, sh.it.pre, sh.it.U, [&](int e, int p) { bg_item_bwd<T, SOLVER>(a, sh, e, p, tau, xbits, tc, gK); },
                [&](int e) {
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const int slot = sh.vslot[e][q];
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            vt_add(sh.vt, slot, k, gK[q * 4 + k]);
                            gK[q * 4 + k] = 0.0f;
                        }
                    }
                });
        }
        if (used > 0) vt_flush(sh.vt, ck.s, a);
    }
    }
    }
}

// dL/dP0 = sum_s (d(x, y)_s / dP0)^T dL/d(x, y)_s through the projection and
// the keyframe transform (App. I); camera depth carries no gradient.
__global__ void k_kf_to_vertex(const Inst *__restrict__ tab, int n)
{
    const Inst a = tab[inst_of<&Inst::b_vtx>(tab, n, blockIdx.x)];
    const int v = (blockIdx.x - a.b_vtx) * blockDim.x + threadIdx.x;
    const int V = a.V, S = a.S;
    const float *__restrict__ verts = a.verts;
    const float *__restrict__ model = a.model;
    const float *__restrict__ gkf = a.gkf;
    float *__restrict__ grad_verts = a.grad_verts;
    const ViewArgs &vw = a.vw;
    if (v >= V) return;
    const double p0 = verts[3 * v], p1 = verts[3 * v + 1], p2 = verts[3 * v + 2];
    const double t = (double)vw.tanf;
    double g[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s <= S; ++s) {
        const float *m = model + (size_t)s * 12;
        double w[3], c[3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            w[r] = (double)m[4 * r] * p0 + (double)m[4 * r + 1] * p1 + (double)m[4 * r + 2] * p2 + (double)m[4 * r + 3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            c[r] = (double)vw.m[4 * r] * w[0] + (double)vw.m[4 * r + 1] * w[1] + (double)vw.m[4 * r + 2] * w[2] +
                   (double)vw.m[4 * r + 3];
        const double gx = gkf[((size_t)s * V + v) * 2], gy = gkf[((size_t)s * V + v) * 2 + 1];
        const double gc[3] = {gx / (c[2] * t), gy / (c[2] * t), -(gx * c[0] + gy * c[1]) / (c[2] * c[2] * t)};
        double gw[3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            gw[j] = (double)vw.m[j] * gc[0] + (double)vw.m[4 + j] * gc[1] + (double)vw.m[8 + j] * gc[2];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            g[j] += (double)m[j] * gw[0] + (double)m[4 + j] * gw[1] + (double)m[8 + j] * gw[2];
    }
    grad_verts[3 * v] = (float)g[0];
    grad_verts[3 * v + 1] = (float)g[1];
    grad_verts[3 * v + 2] = (float)g[2];
}

// ---------------------------------------------------------------- launches

// Waves a persistent kernel keeps resident on the current device: its
// occupancy (registers, LDS) times the compute units.
template <class K>
static unsigned resident_waves(K kernel)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWave, 0) != hipSuccess || per_cu <= 0)
        per_cu = 8;
    return (unsigned)(cus * per_cu);
}

static inline void mark(const PhaseEvents *pe, int i, hipStream_t st)
{
    if (pe && pe->ev[i]) (void)hipEventRecord(pe->ev[i], st);
}

static Inst make_inst(const Plan &p, const Io &io, char *base, const Grids &start)
{
    Inst a;
    std::memset(&a, 0, sizeof(a));
    a.verts = (decltype(a.verts))io.verts;
    a.faces = (decltype(a.faces))io.faces;
    a.attrs = (decltype(a.attrs))io.attrs;
    a.model = (decltype(a.model))io.model;
    a.image = (decltype(a.image))io.image;
    a.grad_image = (decltype(a.grad_image))io.grad_image;
    a.grad_verts = (decltype(a.grad_verts))io.grad_verts;
    a.grad_attrs = (decltype(a.grad_attrs))io.grad_attrs;
    a.hdr = (decltype(a.hdr))(base + p.o_hdr);
    a.kf = (decltype(a.kf))(base + p.o_kf);
    a.kfz = (decltype(a.kfz))(base + p.o_kfz);
    a.cnt = (decltype(a.cnt))(base + p.o_cnt);
    a.off = (decltype(a.off))(base + p.o_off);
    a.cur = (decltype(a.cur))(base + p.o_cur);
    a.bsum = (decltype(a.bsum))(base + p.o_bsum);
    a.list = (decltype(a.list))(base + p.o_list);
    a.vis_id = (decltype(a.vis_id))(base + p.o_vis_id);
    a.pix = (decltype(a.pix))(base + p.o_pix);
    a.tsl = (decltype(a.tsl))(base + p.o_tsl);
    a.toff = (decltype(a.toff))(base + p.o_toff);
    a.tbsum = (decltype(a.tbsum))(base + p.o_tbsum);
    a.tasks = (decltype(a.tasks))(base + p.o_tasks);
    a.gkf = (decltype(a.gkf))(base + p.o_gkf);
    a.fgw = (decltype(a.fgw))(base + p.o_fgw);
    a.gfx = p.det ? (decltype(a.gfx))(base + p.o_gfx) : nullptr;
    a.det = p.det ? 1 : 0;
    a.V = p.V;
    a.F = p.F;
    a.C = p.C;
    a.S = p.S;
    a.K = p.K;
    a.W = p.W;
    a.H = p.H;
    a.tiles_x = p.tiles_x;
    a.tw = p.tw;
    a.th = p.th;
    a.lw = __builtin_ctz((unsigned)p.tw);
    a.lh = __builtin_ctz((unsigned)p.th);
    a.rep = ~0ull / ((1ull << p.tw) - 1ull);
    a.tiles_y = p.tiles_y;
    a.ntiles = p.ntiles;
    a.CPS = p.CPS;
    a.NC = p.NC;
    a.SL = p.SL;
    a.seq_bg = p.seq_bg;
    a.fgg = p.fgg;
    a.bwd_merge = p.bwd_merge;
    a.NS = p.NS;
    a.nfb = p.nfb;
    a.ntct = (int)p.ntct;
    a.nblocks_scan = (int)p.nblocks_scan;
    a.nblocks_tscan = (int)p.nblocks_tscan;
    a.cap = p.cap;
    a.maxtasks = p.maxtasks;
    a.ncounts = p.ncounts;
    a.inv_w = (float)(1.0 / (double)p.W);
    a.inv_h = (float)(1.0 / (double)p.H);
    a.dmax = p.dmax;
    a.halo = p.halo;
    a.neg_log2e_over_delta = (float)(-1.4426950408889634 / (double)p.delta);
    a.inv_delta = (float)(1.0 / (double)p.delta);
    a.invK = 1.0f / (float)p.K;
    for (int i = 0; i < 12; ++i) a.vw.m[i] = p.view[i];
    a.vw.tanf = p.tanf;
    a.b_init = (int)start.init;
    a.b_proj = (int)start.proj;
    a.b_bin = (int)start.bin;
    a.b_scan1 = (int)start.scan1;
    a.b_scan3 = (int)start.scan3;
    a.b_tscan1 = (int)start.tscan1;
    a.b_tscan3 = (int)start.tscan3;
    a.b_fg = (int)start.fg;
    a.b_fgb = (int)start.fgb;
    a.b_res = (int)start.res;
    a.b_bwdinit = (int)start.bwdinit;
    a.b_vtx = (int)start.vtx;
    a.b_sort = (int)start.sort;
    a.b_detp = (int)start.detp;
    return a;
}

// Fill the device instance table (kernel arguments carry the values, so the
// call stays a pure launch sequence) and return it.
static const Inst *write_table(const Batch &bt, const std::vector<Io> &io, void *ws, hipStream_t st)
{
    char *w = (char *)ws;
    Inst *tab = (Inst *)(w + bt.o_table);
    Grids start{};
    TabChunk c;
    c.first = 0;
    c.count = 0;
    for (int i = 0; i < bt.n; ++i) {
        const Plan &p = bt.plans[i];
        c.v[c.count++] = make_inst(p, io[i], w + bt.base[i], start);
        const Grids q = plan_grids(p);
        start.init += q.init;
        start.proj += q.proj;
        start.bin += q.bin;
        start.scan1 += q.scan1;
        start.scan3 += q.scan3;
        start.tscan1 += q.tscan1;
        start.tscan3 += q.tscan3;
        start.fg += q.fg;
        start.fgb += q.fgb;
        start.res += q.res;
        start.bwdinit += q.bwdinit;
        start.vtx += q.vtx;
        start.sort += q.sort;
        start.detp += q.detp;
        if (c.count == kTabChunk || i == bt.n - 1) {
            hipLaunchKernelGGL(k_set_table, dim3(c.count), dim3(64), 0, st, c, tab);
            c.first = i + 1;
            c.count = 0;
        }
    }
    return tab;
}

template <int T, int SOLVER>
static void forward_T(const Batch &bt, const Inst *tab, void *ws, hipStream_t st, const PhaseEvents *pe)
{
    const int n = bt.n;
    const Grids &g = bt.g;
    int64_t *tprefix = (int64_t *)((char *)ws + bt.o_tprefix);
    const auto kbin = bt.tw == 16 ? k_bin<T, 16> : (bt.tw == 4 ? k_bin<T, 4> : k_bin<T, 8>);
    hipLaunchKernelGGL(kbin, dim3((unsigned)g.bin), dim3(kBinThreads), 0, st, tab, n, 0);
    hipLaunchKernelGGL(k_scan1, dim3((unsigned)g.scan1), dim3(kScanThreads), 0, st, tab, n, 0);
    hipLaunchKernelGGL(k_scan2, dim3((unsigned)n), dim3(kScanThreads), 0, st, tab, 0);
    hipLaunchKernelGGL(k_scan3, dim3((unsigned)g.scan3), dim3(256), 0, st, tab, n, 0);
    hipLaunchKernelGGL(kbin, dim3((unsigned)g.bin), dim3(kBinThreads), 0, st, tab, n, 1);
    if (bt.det) hipLaunchKernelGGL(k_sort_lists, dim3((unsigned)g.sort), dim3(kSortThreads), 0, st, tab, n);
    mark(pe, 2, st);
    if (bt.tw == 8)
        hipLaunchKernelGGL((k_fg<T, SOLVER, 8>), dim3((unsigned)g.fg), dim3(kWave), 0, st, tab, n);
    else
        hipLaunchKernelGGL((k_fg<T, SOLVER, 0>), dim3((unsigned)g.fg), dim3(kWave), 0, st, tab, n);
    hipLaunchKernelGGL(k_scan1, dim3((unsigned)g.tscan1), dim3(kScanThreads), 0, st, tab, n, 1);
    hipLaunchKernelGGL(k_scan2, dim3((unsigned)n), dim3(kScanThreads), 0, st, tab, 1);
    hipLaunchKernelGGL(k_scan3, dim3((unsigned)g.tscan3), dim3(256), 0, st, tab, n, 1);
    hipLaunchKernelGGL(k_tasks, dim3((unsigned)g.tscan3), dim3(256), 0, st, tab, n);
    hipLaunchKernelGGL(k_tprefix, dim3(1), dim3(64), 0, st, tab, n, tprefix);
    mark(pe, 3, st);
    // tasks are dealt to waves in a fixed stride of the grid size; a grid of
    // several times the resident waves lets waves that drew cheap tasks hand
    // their slots to fresh ones, which evens out the tail
    if (bt.wide) {
        static const unsigned nw = kBgFwdOversubWide * resident_waves(k_bg<T, SOLVER, true>);
        hipLaunchKernelGGL((k_bg<T, SOLVER, true>), dim3(nw), dim3(kWave), 0, st, tab, n, (const int64_t *)tprefix);
    } else {
        static const unsigned nw = kBgFwdOversubNarrow * resident_waves(k_bg<T, SOLVER, false>);
        hipLaunchKernelGGL((k_bg<T, SOLVER, false>), dim3(nw), dim3(kWave), 0, st, tab, n, (const int64_t *)tprefix);
    }
}

// Library-held workspace of rb_render_blur_fwd_static.  In host code the
// name `scratch` is only a host-side stand-in: its device address comes from
// hipGetSymbolAddress, once per device (each device holds its own copy, at
// its own address, until the process ends), and only that address is passed
// to kernels.
static __device__ __align__(256) unsigned char scratch[RB_STATIC_SCRATCH_BYTES];

hipError_t static_scratch(void **ptr)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_forward(const Batch &bt, const std::vector<Io> &io, void *ws, hipStream_t st, const PhaseEvents *pe)
{
    const int n = bt.n;
    const Grids &g = bt.g;
    mark(pe, 0, st);
    const Inst *tab = write_table(bt, io, ws, st);
    hipLaunchKernelGGL(k_init, dim3((unsigned)g.init), dim3(256), 0, st, tab, n);
    hipLaunchKernelGGL(k_project, dim3((unsigned)g.proj), dim3(256), 0, st, tab, n);
    mark(pe, 1, st);
    const bool fast = bt.solver == RB_SOLVER_FAST;
    switch (bt.T) {
    case 1: fast ? forward_T<1, RB_SOLVER_FAST>(bt, tab, ws, st, pe) : forward_T<1, RB_SOLVER_RECOMPUTE>(bt, tab, ws, st, pe); break;
    case 2: fast ? forward_T<2, RB_SOLVER_FAST>(bt, tab, ws, st, pe) : forward_T<2, RB_SOLVER_RECOMPUTE>(bt, tab, ws, st, pe); break;
    case 3: fast ? forward_T<3, RB_SOLVER_FAST>(bt, tab, ws, st, pe) : forward_T<3, RB_SOLVER_RECOMPUTE>(bt, tab, ws, st, pe); break;
    case 4: fast ? forward_T<4, RB_SOLVER_FAST>(bt, tab, ws, st, pe) : forward_T<4, RB_SOLVER_RECOMPUTE>(bt, tab, ws, st, pe); break;
    default: fast ? forward_T<8, RB_SOLVER_FAST>(bt, tab, ws, st, pe) : forward_T<8, RB_SOLVER_RECOMPUTE>(bt, tab, ws, st, pe); break;
    }
    mark(pe, 4, st);
    hipLaunchKernelGGL(k_resolve, dim3((unsigned)g.res), dim3(kWave * kResWaves), 0, st, tab, n);
    mark(pe, 5, st);
    return hipGetLastError();
}

template <int T, int SOLVER>
static void backward_T(const Batch &bt, const Inst *tab, void *ws, hipStream_t st, const PhaseEvents *pe)
{
    const int n = bt.n;
    hipLaunchKernelGGL((k_fg_bwd<T, SOLVER>), dim3((unsigned)bt.g.fgb), dim3(kWave), 0, st, tab, n);
    mark(pe, 1, st);
    // the tasks vary in cost: one wave per resident slot, each taking tasks
    // from a counter until none are left
    if (bt.wide) {
        static const unsigned nw = resident_waves(k_bg_bwd<T, SOLVER, 4>);
        hipLaunchKernelGGL((k_bg_bwd<T, SOLVER, 4>), dim3(nw), dim3(kWave), 0, st, tab, n);
    } else {
        static const unsigned nw = resident_waves(k_bg_bwd<T, SOLVER, 3>);
        hipLaunchKernelGGL((k_bg_bwd<T, SOLVER, 3>), dim3(nw), dim3(kWave), 0, st, tab, n);
    }
}

hipError_t launch_backward(const Batch &bt, const std::vector<Io> &io, void *ws, hipStream_t st, const PhaseEvents *pe)
{
    const int n = bt.n;
    mark(pe, 0, st);
    const Inst *tab = write_table(bt, io, ws, st);
    hipLaunchKernelGGL(k_bwd_init, dim3((unsigned)bt.g.bwdinit), dim3(256), 0, st, tab, n);
    if (bt.det) hipLaunchKernelGGL(k_det_prep, dim3((unsigned)bt.g.detp), dim3(256), 0, st, tab, n);
    const bool fast = bt.solver == RB_SOLVER_FAST;
    switch (bt.T) {
    case 1: fast ? backward_T<1, RB_SOLVER_FAST>(bt, tab, ws, st, pe) : backward_T<1, RB_SOLVER_RECOMPUTE>(bt, tab, ws, st, pe); break;
    case 2: fast ? backward_T<2, RB_SOLVER_FAST>(bt, tab, ws, st, pe) : backward_T<2, RB_SOLVER_RECOMPUTE>(bt, tab, ws, st, pe); break;
    case 3: fast ? backward_T<3, RB_SOLVER_FAST>(bt, tab, ws, st, pe) : backward_T<3, RB_SOLVER_RECOMPUTE>(bt, tab, ws, st, pe); break;
    case 4: fast ? backward_T<4, RB_SOLVER_FAST>(bt, tab, ws, st, pe) : backward_T<4, RB_SOLVER_RECOMPUTE>(bt, tab, ws, st, pe); break;
    default: fast ? backward_T<8, RB_SOLVER_FAST>(bt, tab, ws, st, pe) : backward_T<8, RB_SOLVER_RECOMPUTE>(bt, tab, ws, st, pe); break;
    }
    mark(pe, 2, st);
    if (bt.det) hipLaunchKernelGGL(k_det_finish, dim3((unsigned)bt.g.bwdinit), dim3(256), 0, st, tab, n);
    hipLaunchKernelGGL(k_kf_to_vertex, dim3((unsigned)bt.g.vtx), dim3(256), 0, st, tab, n);
    mark(pe, 3, st);
    return hipGetLastError();
}

}  // namespace rb
