// HIP kernels (gfx950) of the motion-blur differentiable rasterizer.
//
// Work decomposition
//   * keyframes: one thread per (keyframe, vertex) projects M_s P0 (App. I)
//     in double precision and keeps (x, y) in double, depth in float.  A face
//     seen almost edge-on has a tiny area, so its barycentrics move by
//     (position error)/(height); float32 keyframes alone would cost ~1e-5 of
//     the image there.  Each list entry turns the doubles into float32
//     coordinates relative to the tile anchor at the chunk's middle time,
//     where they are small and exact to ~1e-9.
//   * chunks: the sub-frames t_k = k/(K-1) (Sec. 3.2) of each linear segment
//     (Sec. 3.3) are cut into chunks of at most T consecutive sub-frames that
//     share one segment, hence one pair of keyframes and one set of
//     fast-solver coefficients (eq 8, "computed only once").
//   * binning: one thread per (face, chunk) computes the face's exact
//     screen bounding box at every sub-frame of the chunk and emits, for every
//     8x8 tile the chunk's boxes touch, one entry face << 8 | mask where bit j
//     says "touches this tile at sub-frame j".  Two lists per (chunk, tile):
//     foreground (exact box) and background (box grown by the influence
//     radius sqrt(d_max)).  Count, exclusive scan, fill.
//   * raster: one 64-lane wave per (8x8 tile, group of chunks); lane = pixel.
//     List entries are staged in LDS a batch at a time (one entry per lane);
//     foreground faces are tested by every lane (z-buffer in registers);
//     background (pixel, face) pairs are filtered by a distance lower bound
//     and compacted into an LDS queue so that all 64 lanes evaluate useful
//     pairs (details above k_raster_fwd).
//   * backward: same walks over the lists, reading the forward's per
//     (pixel, sub-frame) visibility; per-entry LDS gradient slots collect the
//     lanes' contributions and are added atomically to per-keyframe vertex
//     gradients; a last kernel maps those through the projection to
//     rest-vertex gradients.
#include <cfloat>
#include <climits>

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

__device__ __forceinline__ float wave_sum(float x)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t x)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x |= (uint32_t)__shfl_xor((int)x, m, 64);
    return x;
}

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

// ------------------------------------------------------------ small kernels

__global__ void k_init(DevHeader *hdr, int64_t cap, int32_t *cnt, int32_t *cur, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        hdr->error_bits = 0;
        hdr->reserved = 0;
        hdr->list_entries = 0;
        hdr->list_capacity = cap;
    }
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        cnt[i] = 0;
        cur[i] = 0;
    }
}

__global__ void k_zero(float *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

struct ViewArgs {
    float m[12];
    float tanf;
};

// Keyframe projection (App. I): X = view (M_s P0), x = X.x/(X.z tan), y = X.y/(X.z tan)
__global__ void k_project(const float *__restrict__ verts, const float *__restrict__ model,
                          const int32_t *__restrict__ faces, int V, int S, int F, ViewArgs vw,
                          double2 *__restrict__ kf, float *__restrict__ kfz, DevHeader *hdr)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nkf = (int64_t)(S + 1) * V;
    if (i < nkf) {
        int s = (int)(i / V), v = (int)(i - (int64_t)s * V);
        const float *m = model + (size_t)s * 12;
        double p0 = verts[3 * v], p1 = verts[3 * v + 1], p2 = verts[3 * v + 2];
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
        kf[i] = make_double2(x, y);
        kfz[i] = (float)c[2];
        if (!(c[2] > 1e-6)) atomicOr(&hdr->error_bits, kHdrBehind);
    } else if (i < nkf + F) {
        int f = (int)(i - nkf);
        int a = faces[3 * f], b = faces[3 * f + 1], c = faces[3 * f + 2];
        if (a < 0 || a >= V || b < 0 || b >= V || c < 0 || c >= V) atomicOr(&hdr->error_bits, kHdrFaceRange);
    }
}

struct BinArgs {
    const int32_t *faces;
    const double2 *kf;
    int32_t *cnt;
    const int64_t *off;
    int32_t *cur;
    uint32_t *list;
    int V, F, S, K, W, H, tiles_x, tiles_y, ntiles, CPS, NC;
    float halo;
    int64_t cap;
};

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
__device__ __forceinline__ void face_tiles(const float x[3], const float y[3], const BinArgs &a, float grow,
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
    tx0 = c0 / kTile;
    tx1 = c1 / kTile;
    ty0 = r0 / kTile;
    ty1 = r1 / kTile;
}

template <int T>
__global__ __launch_bounds__(256) void k_bin(BinArgs a, int pass)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)a.F * a.NC) return;
    int c = (int)(i / a.F), f = (int)(i - (int64_t)c * a.F);
    Chunk ch = chunk_info(c, a.K, a.S, a.CPS);
    if (ch.n <= 0) return;
    float ax[3], ay[3], bx[3], by[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        int v = clampi(a.faces[3 * f + q], 0, a.V - 1);
        double2 p = a.kf[(size_t)ch.s * a.V + v];
        double2 r = a.kf[(size_t)(ch.s + 1) * a.V + v];
        ax[q] = (float)p.x;
        ay[q] = (float)p.y;
        bx[q] = (float)(r.x - p.x);
        by[q] = (float)(r.y - p.y);
    }
    int ftx0[T], ftx1[T], fty0[T], fty1[T], btx0[T], btx1[T], bty0[T], bty1[T];
    int ux0 = INT_MAX, ux1 = INT_MIN, uy0 = INT_MAX, uy1 = INT_MIN;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        ftx0[j] = fty0[j] = btx0[j] = bty0[j] = 1;
        ftx1[j] = fty1[j] = btx1[j] = bty1[j] = 0;
        if (j < ch.n) {
            int rem = (ch.k0 + j) * a.S - ch.s * (a.K - 1);
            float tau = a.K > 1 ? (float)rem / (float)(a.K - 1) : 0.0f;
            float x[3], y[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                x[q] = fmaf(tau, bx[q], ax[q]);
                y[q] = fmaf(tau, by[q], ay[q]);
            }
            face_tiles(x, y, a, 0.0f, ftx0[j], ftx1[j], fty0[j], fty1[j]);
            face_tiles(x, y, a, a.halo, btx0[j], btx1[j], bty0[j], bty1[j]);
            if (btx0[j] <= btx1[j]) {
                ux0 = min(ux0, btx0[j]);
                ux1 = max(ux1, btx1[j]);
                uy0 = min(uy0, bty0[j]);
                uy1 = max(uy1, bty1[j]);
            }
        }
    }
    if (ux0 > ux1) return;
    for (int ty = uy0; ty <= uy1; ++ty) {
        for (int tx = ux0; tx <= ux1; ++tx) {
            uint32_t fm = 0, bm = 0;
#pragma unroll
            for (int j = 0; j < T; ++j) {
                if (tx >= ftx0[j] && tx <= ftx1[j] && ty >= fty0[j] && ty <= fty1[j]) fm |= 1u << j;
                if (tx >= btx0[j] && tx <= btx1[j] && ty >= bty0[j] && ty <= bty1[j]) bm |= 1u << j;
            }
            int tile = ty * a.tiles_x + tx;
#pragma unroll
            for (int L = 0; L < 2; ++L) {
                uint32_t m = L == 0 ? fm : bm;
                if (!m) continue;
                int64_t idx = ((int64_t)L * a.NC + c) * a.ntiles + tile;
                if (pass == 0) {
                    atomicAdd(&a.cnt[idx], 1);
                } else {
                    int64_t pos = a.off[idx] + atomicAdd(&a.cur[idx], 1);
                    if (pos < a.cap) a.list[pos] = ((uint32_t)f << 8) | m;
                }
            }
        }
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

__global__ __launch_bounds__(kScanThreads) void k_scan1(const int32_t *__restrict__ cnt, int64_t *__restrict__ off,
                                                        int64_t *__restrict__ bsum, int64_t n)
{
    __shared__ int64_t tot;
    int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
    int64_t v[kScanPer];
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        v[q] = base + q < n ? cnt[base + q] : 0;
        s += v[q];
    }
    int64_t ex = block_exclusive_scan(s, &tot);
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        if (base + q < n) off[base + q] = ex;
        ex += v[q];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan2(int64_t *__restrict__ bsum, int64_t nb, DevHeader *hdr,
                                                        int64_t cap)
{
    __shared__ int64_t tot;
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        int64_t i = b0 + threadIdx.x;
        int64_t x = i < nb ? bsum[i] : 0;
        int64_t ex = block_exclusive_scan(x, &tot);
        if (i < nb) bsum[i] = ex + carry;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        hdr->list_entries = carry;
        if (carry > cap) atomicOr(&hdr->error_bits, kHdrOverflow);
    }
}

__global__ void k_scan3(int64_t *__restrict__ off, const int64_t *__restrict__ bsum, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) off[i] += bsum[i / kScanBlock];
}

// ----------------------------------------------------------------- raster
//
// One 64-lane wave per (8x8 tile, group of chunks).  For each chunk the wave
// walks its foreground list, then its background list, NB entries at a time.
//
//  * staging: lane e gathers entry e's face indices and double keyframes and
//    forms a FaceRec of float32 coordinates relative to the tile anchor at the
//    chunk's middle time.  It also forms, per sub-frame of the chunk, the
//    64-bit mask of tile pixels the entry can reach (its box at that
//    sub-frame, grown by the influence radius for the background, restricted
//    to the pixels still in question) and their union U_e.
//  * items: a batch's work is the set of (entry, pixel) pairs with the pixel
//    in U_e.  An exclusive scan over the entries numbers them and they are
//    dealt out 64 at a time, one per lane, so a face that reaches 3 pixels of
//    the tile costs 3 lane-evaluations instead of 64.  An item carries the
//    sub-frames where its pixel is in the entry's mask; the fast solver's
//    coefficients are formed once per item and evaluated per sub-frame.
//  * foreground (eq 9): items update an LDS z-buffer by a 64-bit atomic min
//    of (depth bits, face index), which keeps the lowest face index on exact
//    depth ties.  Afterwards each (pixel, sub-frame) shades its winner from
//    the face's keyframes.
//  * background (eqs 10, 13-15): items on uncovered pixels accumulate
//    sum log2(1 - A) per (pixel, sub-frame) with LDS float atomics, zero
//    factors counted apart.
//  * backward: the same item walk over the background list.  The foreground
//    goes the other way round: each (pixel, sub-frame) knows its winning face
//    from the forward, finds it among the staged entries through a small LDS
//    hash table and is queued for that entry.  Per-entry LDS gradient slots
//    collect the items' contributions and are added to global memory with
//    one atomic per non-zero value and batch.

struct RasterArgs {
    const double2 *kf;
    const float *kfz;
    const int32_t *faces;
    const float *attrs;
    const int32_t *cnt;
    const int64_t *off;
    const uint32_t *list;
    int32_t *vis_id;
    float *vis_p;
    float *part;
    const DevHeader *hdr;
    int V, F, C, S, K, W, H, tiles_x, ntiles, CPS, NC, G, NG;
    float dmax, halo, neg_log2e_over_delta, inv_delta;
    int64_t cap;
};

constexpr int NCH = RB_MAX_CHANNELS;
constexpr int NB = 32;              // list entries staged per batch
constexpr int NGA = 12 + 3 * NCH;   // per-entry gradient slot: 3 vertices x 2 keyframes x (x, y), attributes
constexpr int kHash = 128;          // face -> staged entry table (NB keys at most)

enum { kRecFg = 0, kRecBg = 1, kRecGeom = 2 };

// One list entry staged in LDS.  Edge i runs from vertex (i+1)%3 to (i+2)%3.
struct __align__(16) FaceRec {
    float xc[3], yc[3];       // positions at the chunk's middle time tc, minus the tile anchor
    float dx[3], dy[3];       // segment displacement
    float e0x[3], e0y[3];     // edge i at the segment start
    float e1x[3], e1y[3];     // edge i at the segment end
    float aux0[3], aux1[3];   // foreground: camera depth at the start and its change;
                              // background: 1/|edge i|^2 at the start and the end (0 if degenerate)
    int f;
    uint32_t msk;             // sub-frames of the chunk this entry touches
};
static_assert(sizeof(FaceRec) == 128, "FaceRec layout");

__device__ __forceinline__ void lds_sync()
{
    // LDS operations of one wave execute in order; keep the compiler from
    // moving memory accesses across this point
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
}

__device__ __forceinline__ void stage_rec(const RasterArgs &a, int f, int s, double ua, double va, float tc, int kind,
                                          FaceRec &r, int vid[3])
{
    r.f = f;
    double X0[3], Y0[3], X1[3], Y1[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int v = clampi(a.faces[3 * f + q], 0, a.V - 1);
        vid[q] = v;
        const double2 p = a.kf[(size_t)s * a.V + v];
        const double2 e = a.kf[(size_t)(s + 1) * a.V + v];
        X0[q] = p.x;
        Y0[q] = p.y;
        X1[q] = e.x;
        Y1[q] = e.y;
        r.xc[q] = (float)(fma((double)tc, e.x - p.x, p.x) - ua);
        r.yc[q] = (float)(fma((double)tc, e.y - p.y, p.y) - va);
        r.dx[q] = (float)(e.x - p.x);
        r.dy[q] = (float)(e.y - p.y);
        if (kind == kRecFg) {
            const float z0 = a.kfz[(size_t)s * a.V + v], z1 = a.kfz[(size_t)(s + 1) * a.V + v];
            r.aux0[q] = z0;
            r.aux1[q] = z1 - z0;
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int j = (i + 1) % 3, k = (i + 2) % 3;
        const double ax = X0[k] - X0[j], ay = Y0[k] - Y0[j], bx = X1[k] - X1[j], by = Y1[k] - Y1[j];
        r.e0x[i] = (float)ax;
        r.e0y[i] = (float)ay;
        r.e1x[i] = (float)bx;
        r.e1y[i] = (float)by;
        if (kind == kRecBg) {
            const double ea = ax * ax + ay * ay, eb = bx * bx + by * by;
            r.aux0[i] = ea > 0.0 ? (float)(1.0 / ea) : 0.0f;
            r.aux1[i] = eb > 0.0 ? (float)(1.0 / eb) : 0.0f;
        }
    }
    if (kind == kRecGeom) {
#pragma unroll
        for (int i = 0; i < 3; ++i) r.aux0[i] = r.aux1[i] = 0.0f;
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
    __device__ __forceinline__ void setup(const FaceRec &r, float tc, float du, float dv)
    {
        if (SOLVER == RB_SOLVER_FAST) {
            float ax[3], ay[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                ax[q] = r.xc[q] - du;
                ay[q] = r.yc[q] - dv;
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int j = (i + 1) % 3;
                const float dex = r.e1x[i] - r.e0x[i], dey = r.e1y[i] - r.e0y[i];
                const float ecx = fmaf(tc, dex, r.e0x[i]), ecy = fmaf(tc, dey, r.e0y[i]);
                c1[i] = fmaf(r.dx[j], dey, -r.dy[j] * dex);
                c2[i] = fmaf(ax[j], dey, -ay[j] * dex) + fmaf(r.dx[j], ecy, -r.dy[j] * ecx);
                c3[i] = fmaf(ax[j], ecy, -ay[j] * ecx);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                c1[i] = r.xc[i] - du;
                c2[i] = r.yc[i] - dv;
                c3[i] = 0.0f;
            }
        }
    }
    __device__ __forceinline__ void eval(const FaceRec &r, float t, float N[3]) const
    {
        // t = tau - tc
        if (SOLVER == RB_SOLVER_FAST) {
#pragma unroll
            for (int i = 0; i < 3; ++i) N[i] = fmaf(fmaf(c1[i], t, c2[i]), t, c3[i]);
        } else {
            float xt[3], yt[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                xt[i] = fmaf(t, r.dx[i], c1[i]);
                yt[i] = fmaf(t, r.dy[i], c2[i]);
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
// the sub-frame (eq 14): d = |p - F(tau) w*|^2.  q itself is never formed:
// outside a nearly edge-on face |w| is large and q = sum w_i v_i would
// amplify position rounding; the edge search only needs q - v_e, which is
// w_{e+1} E_e - w_{e+2} E_{e+2} with the (double-derived) edge vectors
// E_e = v_{e+1} - v_e.
struct BgEval {
    float w[3];
    float rx, ry;             // q - v_be in F(X)
    float sr, sg;             // raw and clamped edge parameter
    float psx, psy, d;        // closest point at tau (anchor-local) and squared distance
    int be;                   // chosen edge: vertices be and (be+1)%3
};

// closest-point edge e of F(X) (from vertex e to e+1) is FaceRec edge (e+2)%3
__device__ __forceinline__ void kedges(const FaceRec &r, int X, float tc, float Ex[3], float Ey[3], float iee[3])
{
    const float tx = (X ? 1.0f : 0.0f) - tc;
    float kx[3], ky[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        kx[q] = fmaf(tx, r.dx[q], r.xc[q]);
        ky[q] = fmaf(tx, r.dy[q], r.yc[q]);
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int i = (e + 2) % 3, b = (e + 1) % 3;
        Ex[e] = kx[b] - kx[e];
        Ey[e] = ky[b] - ky[e];
        iee[e] = X ? r.aux1[i] : r.aux0[i];
    }
}

__device__ __forceinline__ void bg_eval(const FaceRec &r, float tc, float tau, int X, const float N[3], float invD,
                                        float du, float dv, BgEval &b)
{
#pragma unroll
    for (int i = 0; i < 3; ++i) b.w[i] = N[i] * invD;
    float Ex[3], Ey[3], iee[3];
    kedges(r, X, tc, Ex, Ey, iee);
    float best = FLT_MAX;
    b.be = 0;
    b.sr = 0.0f;
    b.sg = 0.0f;
    b.rx = 0.0f;
    b.ry = 0.0f;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int e1 = (e + 1) % 3, e2 = (e + 2) % 3;
        const float rx = fmaf(b.w[e1], Ex[e], -b.w[e2] * Ex[e2]);
        const float ry = fmaf(b.w[e1], Ey[e], -b.w[e2] * Ey[e2]);
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
        xt[q] = fmaf(t, r.dx[q], r.xc[q]);
        yt[q] = fmaf(t, r.dy[q], r.yc[q]);
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

struct TileGeom {
    int tile, grp, px, py;
    bool inimg;
    double ua, va;   // tile anchor (between the 4 centre pixels) in normalized coordinates
    float du, dv;    // this lane's pixel centre relative to the anchor (exact for W, H powers of 2)
};

__device__ __forceinline__ float lane_du(int lane, int W) { return (float)(2 * (lane & 7) - 7) / (float)W; }
__device__ __forceinline__ float lane_dv(int lane, int H) { return (float)(7 - 2 * (lane >> 3)) / (float)H; }

__device__ __forceinline__ bool tile_geom(const RasterArgs &a, TileGeom &g)
{
    const int lane = threadIdx.x & 63;
    int lb = xcd_remap(blockIdx.x, gridDim.x);
    int wave = lb * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (wave >= a.ntiles * a.NG) return false;
    g.tile = wave % a.ntiles;
    g.grp = wave / a.ntiles;
    int tx = g.tile % a.tiles_x, ty = g.tile / a.tiles_x;
    g.px = tx * kTile + (lane & 7);
    g.py = ty * kTile + (lane >> 3);
    g.inimg = g.px < a.W && g.py < a.H;
    g.ua = (double)(16 * tx + 8 - a.W) / (double)a.W;
    g.va = (double)(a.H - 16 * ty - 8) / (double)a.H;
    g.du = lane_du(lane, a.W);
    g.dv = lane_dv(lane, a.H);
    return true;
}

// local time of sub-frame j of a chunk and whether eq 13 takes the segment's
// end keyframe (tau > 1/2, decided in integers)
__device__ __forceinline__ float chunk_tau(const RasterArgs &a, const Chunk &ch, int j, int &X)
{
    const int rem = (ch.k0 + j) * a.S - ch.s * (a.K - 1);
    X = 2 * rem > a.K - 1 ? 1 : 0;
    return a.K > 1 ? (float)rem / (float)(a.K - 1) : 0.0f;
}

template <int T>
__device__ __forceinline__ void chunk_taus(const RasterArgs &a, const Chunk &ch, float tau[T], uint32_t &xbits)
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

// ------------------------------------------------------------ item machinery

// mask of the tile pixels whose centres lie in [x0 - g, x1 + g] x [y0 - g, y1 + g]
// (anchor-local; bit = 8 * row + column), with a margin of 0.05 pixel so that
// the box never cuts off a pixel the exact test below would accept
__device__ __forceinline__ uint64_t rect_mask(float x0, float x1, float y0, float y1, float g, float W, float H)
{
    // column c has centre du = (2c - 7)/W, row r has dv = (7 - 2r)/H
    const float ca = fmaf(x0 - g, W, 7.0f) * 0.5f - 0.05f, cb = fmaf(x1 + g, W, 7.0f) * 0.5f + 0.05f;
    const float ra = (7.0f - (y1 + g) * H) * 0.5f - 0.05f, rb = (7.0f - (y0 - g) * H) * 0.5f + 0.05f;
    const int c0 = max((int)ceilf(fmaxf(ca, -1.0f)), 0), c1 = min((int)floorf(fminf(cb, 8.0f)), 7);
    const int r0 = max((int)ceilf(fmaxf(ra, -1.0f)), 0), r1 = min((int)floorf(fminf(rb, 8.0f)), 7);
    if (c0 > c1 || r0 > r1) return 0ull;
    const uint64_t row = (uint64_t)((0xffu >> (7 - c1 + c0)) << c0);
    const uint64_t hi = r1 == 7 ? ~0ull : ((1ull << (8 * (r1 + 1))) - 1ull);
    const uint64_t lo = (1ull << (8 * r0)) - 1ull;
    return (row * 0x0101010101010101ull) & hi & ~lo;
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

// Item bookkeeping shared by the forward and backward walks.
template <int T>
struct ItemShared {
    FaceRec rec[NB];
    uint64_t m[NB][T];   // per entry and sub-frame: pixels to evaluate
    uint64_t U[NB];      // union over the sub-frames
    int pre[NB];         // number of the entry's first item
    int ne[NB];          // entries with at least one item, in order
    uint8_t flag[kWave];
};

// Stage entries [first, first + nb) of a list (one per lane) with their
// per-sub-frame pixel masks; allow[j] is the set of pixels in question at
// sub-frame j (0 for sub-frames outside the chunk).  Returns the number of
// items; cnt / pre are the lane's entry's item count and first item.
template <int T>
__device__ __forceinline__ int stage_items(const RasterArgs &a, ItemShared<T> &sh, int64_t first, int nb, int s,
                                           const TileGeom &g, float tc, const float tau[T], int kind, float grow,
                                           const uint64_t allow[T], float (*at)[3][NCH], int (*vids)[3], int &cnt,
                                           int &pre)
{
    const int lane = threadIdx.x & 63;
    lds_sync();
    cnt = 0;
    if (lane < nb) {
        const uint32_t ent = a.list[first + lane];
        FaceRec r;
        int vid[3];
        stage_rec(a, (int)(ent >> 8), s, g.ua, g.va, tc, kind, r, vid);
        uint32_t msk = 0;
        uint64_t U = 0;
#pragma unroll
        for (int j = 0; j < T; ++j) {
            uint64_t mj = 0;
            if (((ent >> j) & 1u) && allow[j]) {
                const float t = tau[j] - tc;
                float x0 = FLT_MAX, x1 = -FLT_MAX, y0 = FLT_MAX, y1 = -FLT_MAX;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const float xt = fmaf(t, r.dx[q], r.xc[q]), yt = fmaf(t, r.dy[q], r.yc[q]);
                    x0 = fminf(x0, xt);
                    x1 = fmaxf(x1, xt);
                    y0 = fminf(y0, yt);
                    y1 = fmaxf(y1, yt);
                }
                mj = rect_mask(x0, x1, y0, y1, grow, (float)a.W, (float)a.H) & allow[j];
            }
            sh.m[lane][j] = mj;
            if (mj) msk |= 1u << j;
            U |= mj;
        }
        r.msk = msk;
        sh.rec[lane] = r;
        sh.U[lane] = U;
        if (at) {
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int c = 0; c < NCH; ++c) at[lane][q][c] = c < a.C ? a.attrs[(size_t)vid[q] * a.C + c] : 0.0f;
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
    if (cnt > 0) {
        sh.pre[lane] = pre;
        sh.ne[lane_rank(bal)] = lane;
    }
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

// ------------------------------------------------------------------ forward

template <int T>
struct FwdShared {
    ItemShared<T> it;
    union {
        unsigned long long zb[T][kWave];   // foreground: depth bits << 32 | face
        struct {
            float lsum[T][kWave];          // sum of log2(1 - A) over non-zero factors
            int nz[T][kWave];              // number of zero factors (A == 1)
        } bg;
    } u;
};

// foreground item: coverage (eqs 1-3 / 8) and depth test (eq 9) per sub-frame
template <int T, int SOLVER>
__device__ __forceinline__ void fg_item(const RasterArgs &a, FwdShared<T> &sh, int e, int p, const float tau[T],
                                        float tc)
{
    const FaceRec &r = sh.it.rec[e];
    const float du = lane_du(p, a.W), dv = lane_dv(p, a.H);
    Bary<SOLVER> bc;
    bc.setup(r, tc, du, dv);
    const unsigned long long f = (uint32_t)r.f;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        if (!((sh.it.m[e][j] >> p) & 1ull)) continue;
        float N[3];
        bc.eval(r, tau[j] - tc, N);
        const float D = N[0] + N[1] + N[2];
        if (!(fabsf(D) > kTauDet)) continue;
        const bool cov = D > 0.0f ? fminf(N[0], fminf(N[1], N[2])) >= 0.0f : fmaxf(N[0], fmaxf(N[1], N[2])) <= 0.0f;
        if (!cov) continue;
        const float invD = 1.0f / D;
        float zt[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) zt[q] = fmaf(tau[j], r.aux1[q], r.aux0[q]);
        const float z = fmaf(N[0], zt[0], fmaf(N[1], zt[1], N[2] * zt[2])) * invD;
        // z > 0 (all vertices in front of the camera), so its bits order like its value
        atomicMin(&sh.u.zb[j][p], ((unsigned long long)__float_as_uint(z) << 32) | f);
    }
}

// background item: eqs 10, 13-15, accumulated as log2(1 - A)
template <int T, int SOLVER>
__device__ __forceinline__ void bg_item_fwd(const RasterArgs &a, FwdShared<T> &sh, int e, int p, const float tau[T],
                                            uint32_t xbits, float tc)
{
    const FaceRec &r = sh.it.rec[e];
    const float du = lane_du(p, a.W), dv = lane_dv(p, a.H);
    Bary<SOLVER> bc;
    bc.setup(r, tc, du, dv);
#pragma unroll
    for (int j = 0; j < T; ++j) {
        if (!((sh.it.m[e][j] >> p) & 1ull)) continue;
        float N[3];
        bc.eval(r, tau[j] - tc, N);
        const float D = N[0] + N[1] + N[2];
        if (!(fabsf(D) > kTauDet)) continue;
        BgEval b;
        bg_eval(r, tc, tau[j], (xbits >> j) & 1u, N, 1.0f / D, du, dv, b);
        if (!(b.d <= a.dmax)) continue;
        const float A = exp2f(b.d * a.neg_log2e_over_delta);
        const float om = one_minus_exp_neg(b.d * a.inv_delta, A);
        if (om > 0.0f)
            atomicAdd(&sh.u.bg.lsum[j][p], log2_one_minus(A, om));
        else
            atomicAdd(&sh.u.bg.nz[j][p], 1);
    }
}

// colour of the winning face at this lane's pixel: barycentric interpolation
// of the vertex attributes (eq 9), from the same float32 record the depth
// test used
template <int SOLVER>
__device__ __forceinline__ void shade_winner(const RasterArgs &a, int f, int s, const TileGeom &g, float tc, float tau,
                                             float rgb[NCH])
{
    FaceRec r;
    int vid[3];
    stage_rec(a, f, s, g.ua, g.va, tc, kRecGeom, r, vid);
    Bary<SOLVER> bc;
    bc.setup(r, tc, g.du, g.dv);
    float N[3];
    bc.eval(r, tau - tc, N);
    const float invD = 1.0f / (N[0] + N[1] + N[2]);
    const float w0 = N[0] * invD, w1 = N[1] * invD, w2 = N[2] * invD;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        float at[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) at[q] = ch < a.C ? a.attrs[(size_t)vid[q] * a.C + ch] : 0.0f;
        rgb[ch] = fmaf(w0, at[0], fmaf(w1, at[1], w2 * at[2]));
    }
}

template <int T, int SOLVER>
__global__ __launch_bounds__(256) void k_raster_fwd(RasterArgs a)
{
    __shared__ FwdShared<T> shm[4];
    TileGeom g;
    if (!tile_geom(a, g)) return;
    if (a.hdr->error_bits & kHdrOverflow) return;
    const int lane = threadIdx.x & 63;
    FwdShared<T> &sh = shm[threadIdx.x >> 6];
    const uint64_t inimg = __ballot(g.inimg);
    float acc[NCH + 1];
#pragma unroll
    for (int ch = 0; ch <= NCH; ++ch) acc[ch] = 0.0f;

    const int c_end = min((g.grp + 1) * a.G, a.NC);
    for (int c = g.grp * a.G; c < c_end; ++c) {
        const Chunk ck = chunk_info(c, a.K, a.S, a.CPS);
        if (ck.n <= 0) continue;
        float tau[T];
        uint32_t xbits;
        chunk_taus<T>(a, ck, tau, xbits);
        const float tc = chunk_centre<T>(tau, ck.n);
        uint64_t allow[T];
#pragma unroll
        for (int j = 0; j < T; ++j) allow[j] = j < ck.n ? inimg : 0ull;

        // ---- foreground: z-buffer over the tile's foreground list (eq 9)
        lds_sync();
#pragma unroll
        for (int j = 0; j < T; ++j) sh.u.zb[j][lane] = ~0ull;
        {
            const int64_t idx = (int64_t)c * a.ntiles + g.tile;
            const int64_t beg = a.off[idx];
            const int n_e = a.cnt[idx];
            for (int base = 0; base < n_e; base += NB) {
                const int nb = min(NB, n_e - base);
                int cnt, pre;
                const int total = stage_items<T>(a, sh.it, beg + base, nb, ck.s, g, tc, tau, kRecFg, 0.0f, allow,
                                                 nullptr, nullptr, cnt, pre);
                for_items<T>(sh.it, total, cnt, pre, [&](int e, int p) { fg_item<T, SOLVER>(a, sh, e, p, tau, tc); });
            }
        }
        lds_sync();
        int zid[T];
        uint64_t unc[T];
        bool anybg = false;
#pragma unroll
        for (int j = 0; j < T; ++j) {
            const unsigned long long key = sh.u.zb[j][lane];
            zid[j] = key == ~0ull ? -1 : (int)(uint32_t)key;
            unc[j] = __ballot(zid[j] < 0) & allow[j];
            anybg = anybg || unc[j] != 0ull;
        }
        lds_sync();
#pragma unroll
        for (int j = 0; j < T; ++j) {
            sh.u.bg.lsum[j][lane] = 0.0f;
            sh.u.bg.nz[j][lane] = 0;
        }

        // ---- background: soft aggregation (eqs 10, 13-15) where uncovered
        if (anybg) {
            const int64_t idx = ((int64_t)a.NC + c) * a.ntiles + g.tile;
            const int64_t beg = a.off[idx];
            const int n_e = a.cnt[idx];
            for (int base = 0; base < n_e; base += NB) {
                const int nb = min(NB, n_e - base);
                int cnt, pre;
                const int total = stage_items<T>(a, sh.it, beg + base, nb, ck.s, g, tc, tau, kRecBg, a.halo, unc,
                                                 nullptr, nullptr, cnt, pre);
                for_items<T>(sh.it, total, cnt, pre,
                             [&](int e, int p) { bg_item_fwd<T, SOLVER>(a, sh, e, p, tau, xbits, tc); });
            }
        }

        // ---- shade, store visibility, accumulate the sub-frame average
        lds_sync();
#pragma unroll
        for (int j = 0; j < T; ++j) {
            if (j >= ck.n) continue;
            const size_t vi = ((size_t)g.tile * a.K + (ck.k0 + j)) * kWave + lane;
            if (!g.inimg) {
                a.vis_id[vi] = -4;
                a.vis_p[vi] = 0.0f;
            } else if (zid[j] >= 0) {
                float rgb[NCH];
                shade_winner<SOLVER>(a, zid[j], ck.s, g, tc, tau[j], rgb);
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) acc[ch] += rgb[ch];
                acc[NCH] += 1.0f;
                a.vis_id[vi] = zid[j];
                a.vis_p[vi] = 0.0f;
            } else {
                const int nz = sh.u.bg.nz[j][lane];
                const float P = exp2f(sh.u.bg.lsum[j][lane]);
                acc[NCH] += nz > 0 ? 1.0f : 1.0f - P;
                a.vis_id[vi] = -1 - min(nz, 2);
                a.vis_p[vi] = P;
            }
        }
    }
    float *out = a.part + ((size_t)g.grp * a.ntiles + g.tile) * (a.C + 1) * kWave + lane;
    for (int ch = 0; ch < a.C; ++ch) out[(size_t)ch * kWave] = acc[ch];
    out[(size_t)a.C * kWave] = acc[NCH];
}

__global__ void k_reduce_image(const float *__restrict__ part, float *__restrict__ image, int C, int W, int H,
                               int tiles_x, int ntiles, int NG, float invK, const DevHeader *hdr)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = (int64_t)(C + 1) * W * H;
    if (i >= n) return;
    int ch = (int)(i / ((int64_t)W * H));
    int rem = (int)(i - (int64_t)ch * W * H);
    int y = rem / W, x = rem - y * W;
    int tile = (y / kTile) * tiles_x + x / kTile;
    int lane = (y % kTile) * kTile + (x % kTile);
    double s = 0.0;
    for (int gq = 0; gq < NG; ++gq) s += part[(((size_t)gq * ntiles + tile) * (C + 1) + ch) * kWave + lane];
    image[i] = (hdr->error_bits & kHdrOverflow) ? __builtin_nanf("") : (float)(s * (double)invK);
}

// ---------------------------------------------------------------- adjoint

struct GradArgs {
    const float *grad_image;
    float *gkf;
    float *gattr;
    float invK;
};

template <int T>
struct BwdShared {
    ItemShared<T> it;
    float at[NB][3][NCH];     // staged entries' vertex attributes (foreground)
    int vid[NB][3];           // staged entries' vertex indices
    float gacc[NB][NGA];      // per-entry gradient slots
    float P[T][kWave];        // forward product over non-zero factors
    int nz[T][kWave];
    float gI[NCH + 1][kWave]; // dL/d(colour, alpha) of each pixel, already divided by K
    int hkey[kHash];          // face -> staged entry (open addressing, -1 = empty)
    int hval[kHash];
    uint32_t q[T * kWave];    // foreground items: entry | pixel << 8 | sub-frame << 16
};

__device__ __forceinline__ int hash_face(int f) { return (int)(((uint32_t)f * 2654435761u) >> 25); }

// Add a lane's per-entry contribution to the entry's LDS slot.
__device__ __forceinline__ void slot_add(float *slot, int i, float v)
{
    if (v != 0.0f) atomicAdd(&slot[i], v);
}

// Flush the staged entries' gradient slots to global memory and clear them.
template <int T>
__device__ __forceinline__ void flush_slots(BwdShared<T> &sh, int nb, int s, const RasterArgs &a, const GradArgs &ga,
                                            bool with_attr)
{
    const int lane = threadIdx.x & 63;
    lds_sync();
    if (lane < nb) {
        float *slot = sh.gacc[lane];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int v = sh.vid[lane][q];
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
                float *p = ga.gkf + ((size_t)(s + sl) * a.V + v) * 2;
                const float gx = slot[q * 4 + sl * 2], gy = slot[q * 4 + sl * 2 + 1];
                if (gx != 0.0f) unsafeAtomicAdd(p, gx);
                if (gy != 0.0f) unsafeAtomicAdd(p + 1, gy);
            }
            if (with_attr)
                for (int c = 0; c < a.C; ++c) {
                    const float gv = slot[12 + q * NCH + c];
                    if (gv != 0.0f) unsafeAtomicAdd(ga.gattr + (size_t)v * a.C + c, gv);
                }
        }
#pragma unroll
        for (int i = 0; i < NGA; ++i) slot[i] = 0.0f;
    }
    lds_sync();
}

// Foreground adjoint of one (pixel, sub-frame) whose winner is staged entry e:
// colour = sum_i w_i c_i, dL/dw through the static solve (dw = -F^-1 dF w),
// dL/dc_i = w_i dL/dcolour.
template <int T, int SOLVER>
__device__ __forceinline__ void fg_item_bwd(const RasterArgs &a, BwdShared<T> &sh, int e, int p, float tau, float tc)
{
    const FaceRec &r = sh.it.rec[e];
    const float du = lane_du(p, a.W), dv = lane_dv(p, a.H);
    float gI[NCH], gw[3];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) gI[ch] = sh.gI[ch][p];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        gw[q] = 0.0f;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) gw[q] = fmaf(gI[ch], sh.at[e][q][ch], gw[q]);
    }
    Bary<SOLVER> bc;
    bc.setup(r, tc, du, dv);
    const float t = tau - tc;
    float N[3];
    bc.eval(r, t, N);
    const float invD = 1.0f / (N[0] + N[1] + N[2]);
    const float w[3] = {N[0] * invD, N[1] * invD, N[2] * invD};
    float xt[3], yt[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        xt[q] = fmaf(t, r.dx[q], r.xc[q]);
        yt[q] = fmaf(t, r.dy[q], r.yc[q]);
    }
    const float gxs = fmaf(gw[0], yt[1] - yt[2], fmaf(gw[1], yt[2] - yt[0], gw[2] * (yt[0] - yt[1]))) * invD;
    const float gys = fmaf(gw[0], xt[2] - xt[1], fmaf(gw[1], xt[0] - xt[2], gw[2] * (xt[1] - xt[0]))) * invD;
    const float t1 = tau, t0 = 1.0f - tau;
    float *slot = sh.gacc[e];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const float gx = -w[q] * gxs, gy = -w[q] * gys;
        slot_add(slot, q * 4 + 0, t0 * gx);
        slot_add(slot, q * 4 + 1, t0 * gy);
        slot_add(slot, q * 4 + 2, t1 * gx);
        slot_add(slot, q * 4 + 3, t1 * gy);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) slot_add(slot, 12 + q * NCH + ch, w[q] * gI[ch]);
    }
}

// Background adjoint of one item: dalpha/dA_j = prod_{m != j}(1 - A_m),
// dA/dd = -A/delta, then the chain through d = |p - p*|^2, the closest point
// (edge parameter where unclamped), q = F(X) w and w(tau) (dw = -F^-1 dF w).
template <int T, int SOLVER>
__device__ __forceinline__ void bg_item_bwd(const RasterArgs &a, BwdShared<T> &sh, int e, int p, const float tau[T],
                                            uint32_t xbits, float tc)
{
    const FaceRec &r = sh.it.rec[e];
    const float du = lane_du(p, a.W), dv = lane_dv(p, a.H);
    const float galpha = sh.gI[NCH][p];
    Bary<SOLVER> bc;
    bc.setup(r, tc, du, dv);
    float gK[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) gK[q] = 0.0f;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        if (!((sh.it.m[e][j] >> p) & 1ull)) continue;
        const float t = tau[j] - tc;
        float N[3];
        bc.eval(r, t, N);
        const float D = N[0] + N[1] + N[2];
        if (!(fabsf(D) > kTauDet)) continue;
        const float invD = 1.0f / D;
        const int X = (xbits >> j) & 1u;
        BgEval b;
        bg_eval(r, tc, tau[j], X, N, invD, du, dv, b);
        if (!(b.d <= a.dmax)) continue;
        const float A = exp2f(b.d * a.neg_log2e_over_delta);
        const float om = one_minus_exp_neg(b.d * a.inv_delta, A);
        const int nzc = sh.nz[j][p];
        const float P = sh.P[j][p];
        const float Pe = nzc == 0 ? P / om : (nzc == 1 ? (om > 0.0f ? 0.0f : P) : 0.0f);
        const float gd = -galpha * Pe * A * a.inv_delta;
        if (gd == 0.0f) continue;
        const float gpx = 2.0f * gd * (b.psx - du), gpy = 2.0f * gd * (b.psy - dv);
        float xt[3], yt[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            xt[q] = fmaf(t, r.dx[q], r.xc[q]);
            yt[q] = fmaf(t, r.dy[q], r.yc[q]);
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
            float Ex[3], Ey[3], iee3[3];
            kedges(r, X, tc, Ex, Ey, iee3);
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
    float *slot = sh.gacc[e];
#pragma unroll
    for (int q = 0; q < 12; ++q) slot_add(slot, q, gK[q]);
}

template <int T, int SOLVER>
__global__ __launch_bounds__(256) void k_raster_bwd(RasterArgs a, GradArgs ga)
{
    __shared__ BwdShared<T> shm[4];
    TileGeom g;
    if (!tile_geom(a, g)) return;
    if (a.hdr->error_bits & kHdrOverflow) return;
    const int lane = threadIdx.x & 63;
    BwdShared<T> &sh = shm[threadIdx.x >> 6];
    bool gcol = false;
    float gal = 0.0f;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        float v = 0.0f;
        if (g.inimg && ch < a.C) v = ga.grad_image[((size_t)ch * a.H + g.py) * a.W + g.px] * ga.invK;
        sh.gI[ch][lane] = v;
        gcol = gcol || v != 0.0f;
    }
    if (g.inimg) gal = ga.grad_image[((size_t)a.C * a.H + g.py) * a.W + g.px] * ga.invK;
    sh.gI[NCH][lane] = gal;
    if (lane < NB)
        for (int i = 0; i < NGA; ++i) sh.gacc[lane][i] = 0.0f;
    sh.hkey[lane] = -1;
    sh.hkey[lane + kWave] = -1;

    const int c_end = min((g.grp + 1) * a.G, a.NC);
    for (int c = g.grp * a.G; c < c_end; ++c) {
        const Chunk ck = chunk_info(c, a.K, a.S, a.CPS);
        if (ck.n <= 0) continue;
        float tau[T];
        uint32_t xbits;
        chunk_taus<T>(a, ck, tau, xbits);
        const float tc = chunk_centre<T>(tau, ck.n);
        int vid[T];
        lds_sync();
#pragma unroll
        for (int j = 0; j < T; ++j) {
            vid[j] = -4;
            float vp = 0.0f;
            if (j < ck.n) {
                const size_t vi = ((size_t)g.tile * a.K + (ck.k0 + j)) * kWave + lane;
                vid[j] = a.vis_id[vi];
                vp = a.vis_p[vi];
            }
            sh.P[j][lane] = vp;
            sh.nz[j][lane] = vid[j] <= -1 && vid[j] >= -3 ? -1 - vid[j] : 0;
        }

        // ---- foreground: each (pixel, sub-frame) finds its winner among the
        //      staged entries through the hash table
        bool anyfg = false;
#pragma unroll
        for (int j = 0; j < T; ++j) anyfg = anyfg || __ballot(gcol && vid[j] >= 0) != 0ull;
        if (anyfg) {
            const int64_t idx = (int64_t)c * a.ntiles + g.tile;
            const int64_t beg = a.off[idx];
            const int n_e = a.cnt[idx];
            for (int base = 0; base < n_e; base += NB) {
                const int nb = min(NB, n_e - base);
                lds_sync();
                int hb = -1;
                if (lane < nb) {
                    const uint32_t ent = a.list[beg + base + lane];
                    const int f = (int)(ent >> 8);
                    FaceRec r;
                    int vq[3];
                    stage_rec(a, f, ck.s, g.ua, g.va, tc, kRecGeom, r, vq);
                    r.msk = ent & 0xffu;
                    sh.it.rec[lane] = r;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        sh.vid[lane][q] = vq[q];
#pragma unroll
                        for (int ch = 0; ch < NCH; ++ch)
                            sh.at[lane][q][ch] = ch < a.C ? a.attrs[(size_t)vq[q] * a.C + ch] : 0.0f;
                    }
                    // faces are unique within a list and NB < kHash: an empty
                    // bucket is always found
                    int h = hash_face(f);
                    for (int probe = 0; probe < kHash; ++probe) {
                        if (atomicCAS(&sh.hkey[h], -1, f) == -1) {
                            hb = h;
                            break;
                        }
                        h = (h + 1) & (kHash - 1);
                    }
                    if (hb >= 0) sh.hval[hb] = lane;
                }
                lds_sync();
                int qn = 0;
#pragma unroll
                for (int j = 0; j < T; ++j) {
                    int sl = -1;
                    if (gcol && vid[j] >= 0) {
                        int h = hash_face(vid[j]);
                        for (int probe = 0; probe < kHash; ++probe) {
                            const int k = sh.hkey[h];
                            if (k == vid[j]) {
                                sl = sh.hval[h];
                                break;
                            }
                            if (k == -1) break;
                            h = (h + 1) & (kHash - 1);
                        }
                    }
                    const uint64_t bal = __ballot(sl >= 0);
                    if (sl >= 0) sh.q[qn + lane_rank(bal)] = (uint32_t)sl | ((uint32_t)lane << 8) | ((uint32_t)j << 16);
                    qn += __popcll(bal);
                }
                lds_sync();
                for (int rb = 0; rb < qn; rb += kWave) {
                    if (rb + lane < qn) {
                        const uint32_t item = sh.q[rb + lane];
                        const int jj = (int)(item >> 16);
                        int X;
                        const float tj = chunk_tau(a, ck, jj, X);
                        fg_item_bwd<T, SOLVER>(a, sh, (int)(item & 0xffu), (int)((item >> 8) & 0xffu), tj, tc);
                    }
                }
                lds_sync();
                if (hb >= 0) sh.hkey[hb] = -1;
                flush_slots<T>(sh, nb, ck.s, a, ga, true);
            }
        }

        // ---- background
        uint64_t bgm[T];
        bool anybg = false;
#pragma unroll
        for (int j = 0; j < T; ++j) {
            bgm[j] = __ballot(vid[j] <= -1 && vid[j] >= -3 && gal != 0.0f);
            anybg = anybg || bgm[j] != 0ull;
        }
        if (anybg) {
            const int64_t idx = ((int64_t)a.NC + c) * a.ntiles + g.tile;
            const int64_t beg = a.off[idx];
            const int n_e = a.cnt[idx];
            for (int base = 0; base < n_e; base += NB) {
                const int nb = min(NB, n_e - base);
                int cnt, pre;
                const int total = stage_items<T>(a, sh.it, beg + base, nb, ck.s, g, tc, tau, kRecBg, a.halo, bgm,
                                                 nullptr, sh.vid, cnt, pre);
                for_items<T>(sh.it, total, cnt, pre,
                             [&](int e, int p) { bg_item_bwd<T, SOLVER>(a, sh, e, p, tau, xbits, tc); });
                flush_slots<T>(sh, nb, ck.s, a, ga, false);
            }
        }
    }
}

// dL/dP0 = sum_s (d(x, y)_s / dP0)^T dL/d(x, y)_s through the projection and
// the keyframe transform (App. I); camera depth carries no gradient.
__global__ void k_kf_to_vertex(const float *__restrict__ verts, const float *__restrict__ model,
                               const float *__restrict__ gkf, int V, int S, ViewArgs vw, float *__restrict__ grad_verts)
{
    int v = blockIdx.x * blockDim.x + threadIdx.x;
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

static inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

static RasterArgs raster_args(const Plan &p, const Inputs &in, const Bufs &b)
{
    RasterArgs a;
    a.kf = b.kf;
    a.kfz = b.kfz;
    a.faces = in.faces;
    a.attrs = in.attrs;
    a.cnt = b.cnt;
    a.off = b.off;
    a.list = b.list;
    a.vis_id = b.vis_id;
    a.vis_p = b.vis_p;
    a.part = b.part;
    a.hdr = b.hdr;
    a.V = p.V;
    a.F = p.F;
    a.C = p.C;
    a.S = p.S;
    a.K = p.K;
    a.W = p.W;
    a.H = p.H;
    a.tiles_x = p.tiles_x;
    a.ntiles = p.ntiles;
    a.CPS = p.CPS;
    a.NC = p.NC;
    a.G = p.G;
    a.NG = p.NG;
    a.dmax = p.dmax;
    a.halo = p.halo;
    a.neg_log2e_over_delta = (float)(-1.4426950408889634 / (double)p.delta);
    a.inv_delta = (float)(1.0 / (double)p.delta);
    a.cap = p.cap;
    return a;
}

static inline void mark(const PhaseEvents *pe, int i, hipStream_t st)
{
    if (pe && pe->ev[i]) (void)hipEventRecord(pe->ev[i], st);
}

template <int T>
static hipError_t fwd_T(const Plan &p, const Inputs &in, const Bufs &b, hipStream_t st, const PhaseEvents *pe)
{
    BinArgs ba;
    ba.faces = in.faces;
    ba.kf = b.kf;
    ba.cnt = b.cnt;
    ba.off = b.off;
    ba.cur = b.cur;
    ba.list = b.list;
    ba.V = p.V;
    ba.F = p.F;
    ba.S = p.S;
    ba.K = p.K;
    ba.W = p.W;
    ba.H = p.H;
    ba.tiles_x = p.tiles_x;
    ba.tiles_y = p.tiles_y;
    ba.ntiles = p.ntiles;
    ba.CPS = p.CPS;
    ba.NC = p.NC;
    ba.halo = p.halo;
    ba.cap = p.cap;
    const int64_t nbin = (int64_t)p.F * p.NC;
    hipLaunchKernelGGL(k_bin<T>, dim3(grid_for(nbin, 256)), dim3(256), 0, st, ba, 0);
    hipLaunchKernelGGL(k_scan1, dim3((unsigned)p.nblocks_scan), dim3(kScanThreads), 0, st, b.cnt, b.off, b.bsum,
                       p.ncounts);
    hipLaunchKernelGGL(k_scan2, dim3(1), dim3(kScanThreads), 0, st, b.bsum, p.nblocks_scan, b.hdr, p.cap);
    hipLaunchKernelGGL(k_scan3, dim3(grid_for(p.ncounts, 256)), dim3(256), 0, st, b.off, b.bsum, p.ncounts);
    hipLaunchKernelGGL(k_bin<T>, dim3(grid_for(nbin, 256)), dim3(256), 0, st, ba, 1);
    mark(pe, 2, st);
    RasterArgs ra = raster_args(p, in, b);
    const int64_t waves = (int64_t)p.ntiles * p.NG;
    const unsigned blocks = grid_for(waves, 4);
    if (p.solver == RB_SOLVER_FAST)
        hipLaunchKernelGGL((k_raster_fwd<T, RB_SOLVER_FAST>), dim3(blocks), dim3(256), 0, st, ra);
    else
        hipLaunchKernelGGL((k_raster_fwd<T, RB_SOLVER_RECOMPUTE>), dim3(blocks), dim3(256), 0, st, ra);
    mark(pe, 3, st);
    return hipGetLastError();
}

hipError_t launch_forward(const Plan &p, const Inputs &in, const Bufs &b, float *image, hipStream_t st,
                          const PhaseEvents *pe)
{
    mark(pe, 0, st);
    hipLaunchKernelGGL(k_init, dim3(grid_for(p.ncounts, 256) > 4096 ? 4096 : grid_for(p.ncounts, 256) + 1), dim3(256), 0,
                       st, b.hdr, p.cap, b.cnt, b.cur, p.ncounts);
    ViewArgs vw;
    for (int i = 0; i < 12; ++i) vw.m[i] = p.view[i];
    vw.tanf = p.tanf;
    const int64_t nproj = (int64_t)(p.S + 1) * p.V + p.F;
    hipLaunchKernelGGL(k_project, dim3(grid_for(nproj, 256)), dim3(256), 0, st, in.verts, in.model, in.faces, p.V,
                       p.S, p.F, vw, b.kf, b.kfz, b.hdr);
    mark(pe, 1, st);
    hipError_t e;
    switch (p.T) {
    case 1: e = fwd_T<1>(p, in, b, st, pe); break;
    case 2: e = fwd_T<2>(p, in, b, st, pe); break;
    case 4: e = fwd_T<4>(p, in, b, st, pe); break;
    default: e = fwd_T<8>(p, in, b, st, pe); break;
    }
    if (e != hipSuccess) return e;
    const int64_t npix = (int64_t)(p.C + 1) * p.W * p.H;
    hipLaunchKernelGGL(k_reduce_image, dim3(grid_for(npix, 256)), dim3(256), 0, st, b.part, image, p.C, p.W, p.H,
                       p.tiles_x, p.ntiles, p.NG, 1.0f / (float)p.K, b.hdr);
    mark(pe, 4, st);
    return hipGetLastError();
}

template <int T>
static void bwd_T(const Plan &p, const Inputs &in, const Bufs &b, const GradArgs &ga, hipStream_t st)
{
    RasterArgs ra = raster_args(p, in, b);
    const int64_t waves = (int64_t)p.ntiles * p.NG;
    const unsigned blocks = grid_for(waves, 4);
    if (p.solver == RB_SOLVER_FAST)
        hipLaunchKernelGGL((k_raster_bwd<T, RB_SOLVER_FAST>), dim3(blocks), dim3(256), 0, st, ra, ga);
    else
        hipLaunchKernelGGL((k_raster_bwd<T, RB_SOLVER_RECOMPUTE>), dim3(blocks), dim3(256), 0, st, ra, ga);
}

hipError_t launch_backward(const Plan &p, const Inputs &in, const Bufs &b, const float *grad_image, float *grad_verts,
                           float *grad_attrs, hipStream_t st, const PhaseEvents *pe)
{
    mark(pe, 0, st);
    const int64_t ngkf = (int64_t)(p.S + 1) * p.V * 2;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(ngkf, 256) > 4096 ? 4096 : grid_for(ngkf, 256)), dim3(256), 0, st, b.gkf,
                       ngkf);
    const int64_t nga = (int64_t)p.V * p.C;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(nga, 256) > 4096 ? 4096 : grid_for(nga, 256)), dim3(256), 0, st,
                       grad_attrs, nga);
    GradArgs ga;
    ga.grad_image = grad_image;
    ga.gkf = b.gkf;
    ga.gattr = grad_attrs;
    ga.invK = 1.0f / (float)p.K;
    mark(pe, 1, st);
    switch (p.T) {
    case 1: bwd_T<1>(p, in, b, ga, st); break;
    case 2: bwd_T<2>(p, in, b, ga, st); break;
    case 4: bwd_T<4>(p, in, b, ga, st); break;
    default: bwd_T<8>(p, in, b, ga, st); break;
    }
    mark(pe, 2, st);
    ViewArgs vw;
    for (int i = 0; i < 12; ++i) vw.m[i] = p.view[i];
    vw.tanf = p.tanf;
    hipLaunchKernelGGL(k_kf_to_vertex, dim3(grid_for(p.V, 256)), dim3(256), 0, st, in.verts, in.model, b.gkf, p.V,
                       p.S, vw, grad_verts);
    mark(pe, 3, st);
    return hipGetLastError();
}

}  // namespace rb
