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
//     Per chunk the wave walks the foreground list (z-buffer per lane and
//     sub-frame in registers), then, only for sub-frames with uncovered lanes,
//     the background list (soft product per lane and sub-frame).  The
//     per-(pixel, face, segment) fast-solver coefficients are set up once per
//     list entry and evaluated by Horner's rule for each masked sub-frame.
//   * backward: same walk over the lists, reading the forward's per
//     (pixel, sub-frame) visibility; per-face adjoint contributions are summed
//     over the chunk's sub-frames in registers, then over the wave, then added
//     atomically to per-keyframe vertex gradients; a last kernel maps them
//     through the projection to rest-vertex gradients.
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
    float dmax, neg_log2e_over_delta, inv_delta;
    int64_t cap;
};

constexpr int NCH = RB_MAX_CHANNELS;

// One face of one list entry, seen from one tile, over one chunk: float32
// coordinates relative to the tile anchor, formed in double precision.
struct FaceData {
    int v[3];
    float xc[3], yc[3];     // positions at the chunk's middle time tc
    float dx[3], dy[3];     // segment displacement (position at tau = xc + (tau - tc) dx)
    float xk0[3], yk0[3];   // keyframe s (segment start)
    float xk1[3], yk1[3];   // keyframe s + 1 (segment end)
    float ecx[3], ecy[3];   // edge i = v[(i+2)%3] - v[(i+1)%3] at tc
    float dex[3], dey[3];   // change of edge i over the segment
    float z0[3], dz[3];     // camera depth at the segment start and its change
    float tc;
};

__device__ __forceinline__ void load_face(const RasterArgs &a, int f, int s, double ua, double va, float tc,
                                          FaceData &fd)
{
    double X0[3], Y0[3], X1[3], Y1[3], Xc[3], Yc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        int v = clampi(a.faces[3 * f + q], 0, a.V - 1);
        fd.v[q] = v;
        const double2 p = a.kf[(size_t)s * a.V + v];
        const double2 r = a.kf[(size_t)(s + 1) * a.V + v];
        X0[q] = p.x;
        Y0[q] = p.y;
        X1[q] = r.x;
        Y1[q] = r.y;
        Xc[q] = fma((double)tc, r.x - p.x, p.x);
        Yc[q] = fma((double)tc, r.y - p.y, p.y);
        fd.xc[q] = (float)(Xc[q] - ua);
        fd.yc[q] = (float)(Yc[q] - va);
        fd.dx[q] = (float)(r.x - p.x);
        fd.dy[q] = (float)(r.y - p.y);
        fd.xk0[q] = (float)(p.x - ua);
        fd.yk0[q] = (float)(p.y - va);
        fd.xk1[q] = (float)(r.x - ua);
        fd.yk1[q] = (float)(r.y - va);
        const float z0 = a.kfz[(size_t)s * a.V + v], z1 = a.kfz[(size_t)(s + 1) * a.V + v];
        fd.z0[q] = z0;
        fd.dz[q] = z1 - z0;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int j = (i + 1) % 3, k = (i + 2) % 3;
        fd.ecx[i] = (float)(Xc[k] - Xc[j]);
        fd.ecy[i] = (float)(Yc[k] - Yc[j]);
        fd.dex[i] = (float)((X1[k] - X1[j]) - (X0[k] - X0[j]));
        fd.dey[i] = (float)((Y1[k] - Y1[j]) - (Y0[k] - Y0[j]));
    }
    fd.tc = tc;
}

// anchor-local vertex positions at local time tau
__device__ __forceinline__ void pos_at(const FaceData &fd, float tau, float xt[3], float yt[3])
{
    const float t = tau - fd.tc;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        xt[q] = fmaf(t, fd.dx[q], fd.xc[q]);
        yt[q] = fmaf(t, fd.dy[q], fd.yc[q]);
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
    __device__ __forceinline__ void setup(const FaceData &fd, float du, float dv)
    {
        if (SOLVER == RB_SOLVER_FAST) {
            float ax[3], ay[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                ax[q] = fd.xc[q] - du;
                ay[q] = fd.yc[q] - dv;
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int j = (i + 1) % 3;
                c1[i] = fmaf(fd.dx[j], fd.dey[i], -fd.dy[j] * fd.dex[i]);
                c2[i] = fmaf(ax[j], fd.dey[i], -ay[j] * fd.dex[i]) + fmaf(fd.dx[j], fd.ecy[i], -fd.dy[j] * fd.ecx[i]);
                c3[i] = fmaf(ax[j], fd.ecy[i], -ay[j] * fd.ecx[i]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                c1[i] = fd.xc[i] - du;
                c2[i] = fd.yc[i] - dv;
                c3[i] = 0.0f;
            }
        }
    }
    __device__ __forceinline__ void eval(const FaceData &fd, float tau, float N[3]) const
    {
        const float t = tau - fd.tc;
        if (SOLVER == RB_SOLVER_FAST) {
#pragma unroll
            for (int i = 0; i < 3; ++i) N[i] = fmaf(fmaf(c1[i], t, c2[i]), t, c3[i]);
        } else {
            float xt[3], yt[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                xt[i] = fmaf(t, fd.dx[i], c1[i]);
                yt[i] = fmaf(t, fd.dy[i], c2[i]);
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int j = (i + 1) % 3, k = (i + 2) % 3;
                N[i] = fmaf(xt[j], yt[k], -xt[k] * yt[j]);
            }
        }
    }
};

// Closest point of the keyframe triangle F(X) to q = F(X) w (App. B edge
// projections, edges (0,1), (1,2), (2,0), first edge wins ties) and the
// eq 14 distance at the sub-frame.
struct EdgeSet {
    float ax[3], ay[3], ex[3], ey[3], inv_ee[3];
    __device__ __forceinline__ void setup(const FaceData &fd, int X)
    {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            ax[q] = X ? fd.xk1[q] : fd.xk0[q];
            ay[q] = X ? fd.yk1[q] : fd.yk0[q];
        }
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const int b = (e + 1) % 3;
            ex[e] = ax[b] - ax[e];
            ey[e] = ay[b] - ay[e];
            float ee = fmaf(ex[e], ex[e], ey[e] * ey[e]);
            inv_ee[e] = ee > 0.0f ? 1.0f / ee : 0.0f;
        }
    }
};

struct BgEval {
    float w[3];
    float qx, qy, sr, sg, psx, psy, d;
    int be;
};

__device__ __forceinline__ void bg_eval(const FaceData &fd, const EdgeSet &es, float tau, const float N[3],
                                        float invD, float du, float dv, BgEval &r)
{
#pragma unroll
    for (int i = 0; i < 3; ++i) r.w[i] = N[i] * invD;
    r.qx = fmaf(r.w[0], es.ax[0], fmaf(r.w[1], es.ax[1], r.w[2] * es.ax[2]));
    r.qy = fmaf(r.w[0], es.ay[0], fmaf(r.w[1], es.ay[1], r.w[2] * es.ay[2]));
    float best = FLT_MAX;
    r.be = 0;
    r.sr = 0.0f;
    r.sg = 0.0f;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        float rx = r.qx - es.ax[e], ry = r.qy - es.ay[e];
        float sr = fmaf(rx, es.ex[e], ry * es.ey[e]) * es.inv_ee[e];
        float sg = __builtin_amdgcn_fmed3f(sr, 0.0f, 1.0f);
        float hx = fmaf(-sg, es.ex[e], rx), hy = fmaf(-sg, es.ey[e], ry);
        float dist = fmaf(hx, hx, hy * hy);
        bool better = dist < best || e == 0;
        best = better ? dist : best;
        r.be = better ? e : r.be;
        r.sr = better ? sr : r.sr;
        r.sg = better ? sg : r.sg;
    }
    // sub-frame positions of the chosen edge's end points (anchor-local)
    float xt[3], yt[3];
    pos_at(fd, tau, xt, yt);
    float xa = r.be == 0 ? xt[0] : (r.be == 1 ? xt[1] : xt[2]);
    float ya = r.be == 0 ? yt[0] : (r.be == 1 ? yt[1] : yt[2]);
    float xb = r.be == 0 ? xt[1] : (r.be == 1 ? xt[2] : xt[0]);
    float yb = r.be == 0 ? yt[1] : (r.be == 1 ? yt[2] : yt[0]);
    r.psx = fmaf(r.sg, xb - xa, xa);
    r.psy = fmaf(r.sg, yb - ya, ya);
    float ddx = r.psx - du, ddy = r.psy - dv;
    r.d = fmaf(ddx, ddx, ddy * ddy);
}

struct TileGeom {
    int tile, grp, px, py;
    bool inimg;
    double ua, va;   // tile anchor (between the 4 centre pixels) in normalized coordinates
    float du, dv;    // this lane's pixel centre relative to the anchor (exact for W, H powers of 2)
};

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
    g.du = (float)(2 * (lane & 7) - 7) / (float)a.W;
    g.dv = (float)(7 - 2 * (lane >> 3)) / (float)a.H;
    return true;
}

template <int T>
__device__ __forceinline__ void chunk_taus(const RasterArgs &a, const Chunk &ch, float tau[T], uint32_t &xbits)
{
    xbits = 0;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        int rem = (ch.k0 + j) * a.S - ch.s * (a.K - 1);
        tau[j] = a.K > 1 ? (float)rem / (float)(a.K - 1) : 0.0f;
        if (j < ch.n && 2 * rem > a.K - 1) xbits |= 1u << j;
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

template <int T, int SOLVER>
__global__ __launch_bounds__(256) void k_raster_fwd(RasterArgs a)
{
    TileGeom g;
    if (!tile_geom(a, g)) return;
    if (a.hdr->error_bits & kHdrOverflow) return;
    const int lane = threadIdx.x & 63;
    float acc[NCH + 1];
#pragma unroll
    for (int ch = 0; ch <= NCH; ++ch) acc[ch] = 0.0f;

    const int c_end = min((g.grp + 1) * a.G, a.NC);
    for (int c = g.grp * a.G; c < c_end; ++c) {
        Chunk ck = chunk_info(c, a.K, a.S, a.CPS);
        if (ck.n <= 0) continue;
        const uint32_t live = (1u << ck.n) - 1u;
        float tau[T];
        uint32_t xbits;
        chunk_taus<T>(a, ck, tau, xbits);
        const float tcen = chunk_centre<T>(tau, ck.n);
        float zb[T], rgb[T][NCH], P[T];
        int zid[T], nz[T];
#pragma unroll
        for (int j = 0; j < T; ++j) {
            zb[j] = FLT_MAX;
            zid[j] = -1;
            P[j] = 1.0f;
            nz[j] = 0;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) rgb[j][ch] = 0.0f;
        }

        // ---- foreground: z-buffer over the tile's foreground list (eq 9)
        {
            const int64_t idx = (int64_t)c * a.ntiles + g.tile;
            const int64_t beg = a.off[idx];
            const int n_e = a.cnt[idx];
            for (int e = 0; e < n_e; ++e) {
                const uint32_t ent = __builtin_amdgcn_readfirstlane(a.list[beg + e]);
                const int f = (int)(ent >> 8);
                const uint32_t msk = ent & live;
                if (!msk) continue;
                FaceData fd;
                load_face(a, f, ck.s, g.ua, g.va, tcen, fd);
                float at[3][NCH];
#pragma unroll
                for (int q = 0; q < 3; ++q)
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch)
                        at[q][ch] = ch < a.C ? a.attrs[(size_t)fd.v[q] * a.C + ch] : 0.0f;
                Bary<SOLVER> bc;
                bc.setup(fd, g.du, g.dv);
#pragma unroll
                for (int j = 0; j < T; ++j) {
                    if (!((msk >> j) & 1u)) continue;
                    float N[3];
                    bc.eval(fd, tau[j], N);
                    const float D = N[0] + N[1] + N[2];
                    if (!(fabsf(D) > kTauDet)) continue;
                    const bool cov = D > 0.0f ? fminf(N[0], fminf(N[1], N[2])) >= 0.0f
                                              : fmaxf(N[0], fmaxf(N[1], N[2])) <= 0.0f;
                    if (!cov) continue;
                    const float invD = 1.0f / D;
                    float zt[3];
#pragma unroll
                    for (int q = 0; q < 3; ++q) zt[q] = fmaf(tau[j], fd.dz[q], fd.z0[q]);
                    const float z = fmaf(N[0], zt[0], fmaf(N[1], zt[1], N[2] * zt[2])) * invD;
                    if (z < zb[j] || (z == zb[j] && f < zid[j])) {
                        zb[j] = z;
                        zid[j] = f;
                        const float w0 = N[0] * invD, w1 = N[1] * invD, w2 = N[2] * invD;
#pragma unroll
                        for (int ch = 0; ch < NCH; ++ch)
                            rgb[j][ch] = fmaf(w0, at[0][ch], fmaf(w1, at[1][ch], w2 * at[2][ch]));
                    }
                }
            }
        }

        // ---- background: soft aggregation (eqs 10, 13-15) where uncovered
        uint32_t bgbits = 0;
#pragma unroll
        for (int j = 0; j < T; ++j)
            if (__ballot(g.inimg && zid[j] < 0)) bgbits |= 1u << j;
        bgbits &= live;
        if (bgbits) {
            const int64_t idx = ((int64_t)a.NC + c) * a.ntiles + g.tile;
            const int64_t beg = a.off[idx];
            const int n_e = a.cnt[idx];
            for (int e = 0; e < n_e; ++e) {
                const uint32_t ent = __builtin_amdgcn_readfirstlane(a.list[beg + e]);
                const int f = (int)(ent >> 8);
                const uint32_t msk = ent & bgbits;
                if (!msk) continue;
                FaceData fd;
                load_face(a, f, ck.s, g.ua, g.va, tcen, fd);
                EdgeSet es0, es1;
                if (msk & ~xbits) es0.setup(fd, 0);
                if (msk & xbits) es1.setup(fd, 1);
                Bary<SOLVER> bc;
                bc.setup(fd, g.du, g.dv);
#pragma unroll
                for (int j = 0; j < T; ++j) {
                    if (!((msk >> j) & 1u)) continue;
                    if (!(g.inimg && zid[j] < 0)) continue;
                    float N[3];
                    bc.eval(fd, tau[j], N);
                    const float D = N[0] + N[1] + N[2];
                    if (!(fabsf(D) > kTauDet)) continue;
                    BgEval be;
                    bg_eval(fd, ((xbits >> j) & 1u) ? es1 : es0, tau[j], N, 1.0f / D, g.du, g.dv, be);
                    if (!(be.d <= a.dmax)) continue;
                    const float A = exp2f(be.d * a.neg_log2e_over_delta);
                    const float om = one_minus_exp_neg(be.d * a.inv_delta, A);
                    if (om > 0.0f)
                        P[j] *= om;
                    else
                        nz[j] += 1;
                }
            }
        }

        // ---- shade, store visibility, accumulate the sub-frame average
#pragma unroll
        for (int j = 0; j < T; ++j) {
            if (j >= ck.n) continue;
            const size_t vi = ((size_t)g.tile * a.K + (ck.k0 + j)) * kWave + lane;
            if (!g.inimg) {
                a.vis_id[vi] = -4;
                a.vis_p[vi] = 0.0f;
            } else if (zid[j] >= 0) {
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) acc[ch] += rgb[j][ch];
                acc[NCH] += 1.0f;
                a.vis_id[vi] = zid[j];
                a.vis_p[vi] = 0.0f;
            } else {
                acc[NCH] += nz[j] > 0 ? 1.0f : 1.0f - P[j];
                a.vis_id[vi] = -1 - min(nz[j], 2);
                a.vis_p[vi] = P[j];
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

template <bool ATTR>
__device__ __forceinline__ void flush_face(bool hit, float (&gK)[12], float (&gA)[3][NCH], const FaceData &fd, int s,
                                           const RasterArgs &a, const GradArgs &ga)
{
    const uint64_t bal = __ballot(hit);
    if (!bal) return;
    const int lane = threadIdx.x & 63;
    if (__popcll(bal) <= 2) {
        if (hit) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
#pragma unroll
                for (int sl = 0; sl < 2; ++sl) {
                    float *p = ga.gkf + ((size_t)(s + sl) * a.V + fd.v[q]) * 2;
                    if (gK[q * 4 + sl * 2] != 0.0f) unsafeAtomicAdd(p, gK[q * 4 + sl * 2]);
                    if (gK[q * 4 + sl * 2 + 1] != 0.0f) unsafeAtomicAdd(p + 1, gK[q * 4 + sl * 2 + 1]);
                }
                if (ATTR)
                    for (int ch = 0; ch < a.C; ++ch)
                        if (gA[q][ch] != 0.0f) unsafeAtomicAdd(ga.gattr + (size_t)fd.v[q] * a.C + ch, gA[q][ch]);
            }
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
            float sx = wave_sum(hit ? gK[q * 4 + sl * 2] : 0.0f);
            float sy = wave_sum(hit ? gK[q * 4 + sl * 2 + 1] : 0.0f);
            if (lane == 0) {
                float *p = ga.gkf + ((size_t)(s + sl) * a.V + fd.v[q]) * 2;
                unsafeAtomicAdd(p, sx);
                unsafeAtomicAdd(p + 1, sy);
            }
        }
        if (ATTR)
            for (int ch = 0; ch < a.C; ++ch) {
                float sa = wave_sum(hit ? gA[q][ch] : 0.0f);
                if (lane == 0) unsafeAtomicAdd(ga.gattr + (size_t)fd.v[q] * a.C + ch, sa);
            }
    }
}

template <int T, int SOLVER>
__global__ __launch_bounds__(256) void k_raster_bwd(RasterArgs a, GradArgs ga)
{
    TileGeom g;
    if (!tile_geom(a, g)) return;
    if (a.hdr->error_bits & kHdrOverflow) return;
    const int lane = threadIdx.x & 63;
    float gI[NCH + 1];
#pragma unroll
    for (int ch = 0; ch <= NCH; ++ch) gI[ch] = 0.0f;
    if (g.inimg) {
        for (int ch = 0; ch < a.C; ++ch) gI[ch] = ga.grad_image[((size_t)ch * a.H + g.py) * a.W + g.px] * ga.invK;
        gI[NCH] = ga.grad_image[((size_t)a.C * a.H + g.py) * a.W + g.px] * ga.invK;
    }
    const float galpha = gI[NCH];

    const int c_end = min((g.grp + 1) * a.G, a.NC);
    for (int c = g.grp * a.G; c < c_end; ++c) {
        Chunk ck = chunk_info(c, a.K, a.S, a.CPS);
        if (ck.n <= 0) continue;
        const uint32_t live = (1u << ck.n) - 1u;
        float tau[T];
        uint32_t xbits;
        chunk_taus<T>(a, ck, tau, xbits);
        const float tcen = chunk_centre<T>(tau, ck.n);
        int vid[T];
        float vp[T];
#pragma unroll
        for (int j = 0; j < T; ++j) {
            vid[j] = -4;
            vp[j] = 0.0f;
            if (j < ck.n) {
                const size_t vi = ((size_t)g.tile * a.K + (ck.k0 + j)) * kWave + lane;
                vid[j] = a.vis_id[vi];
                vp[j] = a.vis_p[vi];
            }
        }

        // ---- foreground: dL/dw through the static solve (dw = -F^-1 dF w)
        uint32_t fgbits = 0;
#pragma unroll
        for (int j = 0; j < T; ++j)
            if (__ballot(vid[j] >= 0)) fgbits |= 1u << j;
        if (fgbits) {
            const int64_t idx = (int64_t)c * a.ntiles + g.tile;
            const int64_t beg = a.off[idx];
            const int n_e = a.cnt[idx];
            for (int e = 0; e < n_e; ++e) {
                const uint32_t ent = __builtin_amdgcn_readfirstlane(a.list[beg + e]);
                const int f = (int)(ent >> 8);
                uint32_t hits = 0;
#pragma unroll
                for (int j = 0; j < T; ++j)
                    if (vid[j] == f) hits |= 1u << j;
                const uint32_t msk = wave_or(hits) & ent & fgbits;
                if (!msk) continue;
                FaceData fd;
                load_face(a, f, ck.s, g.ua, g.va, tcen, fd);
                float at[3][NCH];
#pragma unroll
                for (int q = 0; q < 3; ++q)
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch)
                        at[q][ch] = ch < a.C ? a.attrs[(size_t)fd.v[q] * a.C + ch] : 0.0f;
                float gw[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    gw[q] = 0.0f;
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) gw[q] = fmaf(gI[ch], at[q][ch], gw[q]);
                }
                Bary<SOLVER> bc;
                bc.setup(fd, g.du, g.dv);
                float gK[12], gA[3][NCH];
#pragma unroll
                for (int q = 0; q < 12; ++q) gK[q] = 0.0f;
#pragma unroll
                for (int q = 0; q < 3; ++q)
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) gA[q][ch] = 0.0f;
                bool hit = false;
#pragma unroll
                for (int j = 0; j < T; ++j) {
                    if (!((msk >> j) & 1u)) continue;
                    if (vid[j] != f) continue;
                    float N[3];
                    bc.eval(fd, tau[j], N);
                    const float invD = 1.0f / (N[0] + N[1] + N[2]);
                    const float w[3] = {N[0] * invD, N[1] * invD, N[2] * invD};
                    float xt[3], yt[3];
                    pos_at(fd, tau[j], xt, yt);
                    const float gxs =
                        fmaf(gw[0], yt[1] - yt[2], fmaf(gw[1], yt[2] - yt[0], gw[2] * (yt[0] - yt[1]))) * invD;
                    const float gys =
                        fmaf(gw[0], xt[2] - xt[1], fmaf(gw[1], xt[0] - xt[2], gw[2] * (xt[1] - xt[0]))) * invD;
                    const float t1 = tau[j], t0 = 1.0f - tau[j];
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const float gx = -w[q] * gxs, gy = -w[q] * gys;
                        gK[q * 4 + 0] = fmaf(t0, gx, gK[q * 4 + 0]);
                        gK[q * 4 + 1] = fmaf(t0, gy, gK[q * 4 + 1]);
                        gK[q * 4 + 2] = fmaf(t1, gx, gK[q * 4 + 2]);
                        gK[q * 4 + 3] = fmaf(t1, gy, gK[q * 4 + 3]);
#pragma unroll
                        for (int ch = 0; ch < NCH; ++ch) gA[q][ch] = fmaf(w[q], gI[ch], gA[q][ch]);
                    }
                    hit = true;
                }
                flush_face<true>(hit, gK, gA, fd, ck.s, a, ga);
            }
        }

        // ---- background: dalpha/dA_j = prod_{m != j} (1 - A_m), chain
        //      through d, the closest point, q = F(X) w and w(tau)
        uint32_t bgbits = 0;
#pragma unroll
        for (int j = 0; j < T; ++j)
            if (__ballot(vid[j] <= -1 && vid[j] >= -3 && galpha != 0.0f)) bgbits |= 1u << j;
        bgbits &= live;
        if (bgbits) {
            const int64_t idx = ((int64_t)a.NC + c) * a.ntiles + g.tile;
            const int64_t beg = a.off[idx];
            const int n_e = a.cnt[idx];
            for (int e = 0; e < n_e; ++e) {
                const uint32_t ent = __builtin_amdgcn_readfirstlane(a.list[beg + e]);
                const int f = (int)(ent >> 8);
                const uint32_t msk = ent & bgbits;
                if (!msk) continue;
                FaceData fd;
                load_face(a, f, ck.s, g.ua, g.va, tcen, fd);
                EdgeSet es0, es1;
                if (msk & ~xbits) es0.setup(fd, 0);
                if (msk & xbits) es1.setup(fd, 1);
                Bary<SOLVER> bc;
                bc.setup(fd, g.du, g.dv);
                float gK[12];
                float gA[3][NCH];
#pragma unroll
                for (int q = 0; q < 12; ++q) gK[q] = 0.0f;
                bool hit = false;
#pragma unroll
                for (int j = 0; j < T; ++j) {
                    if (!((msk >> j) & 1u)) continue;
                    if (!(vid[j] <= -1 && vid[j] >= -3)) continue;
                    float N[3];
                    bc.eval(fd, tau[j], N);
                    const float D = N[0] + N[1] + N[2];
                    if (!(fabsf(D) > kTauDet)) continue;
                    const float invD = 1.0f / D;
                    const int X = (xbits >> j) & 1u;
                    const EdgeSet &es = X ? es1 : es0;
                    BgEval be;
                    bg_eval(fd, es, tau[j], N, invD, g.du, g.dv, be);
                    if (!(be.d <= a.dmax)) continue;
                    const float A = exp2f(be.d * a.neg_log2e_over_delta);
                    const float om = one_minus_exp_neg(be.d * a.inv_delta, A);
                    const int nzc = -1 - vid[j];
                    const float Pe = nzc == 0 ? vp[j] / om : (nzc == 1 ? (om > 0.0f ? 0.0f : vp[j]) : 0.0f);
                    const float gd = -galpha * Pe * A * a.inv_delta;
                    if (gd == 0.0f) continue;
                    hit = true;
                    // d = |p* - p|^2, p* = (1 - sg) v_a(tau) + sg v_b(tau)
                    const float gpx = 2.0f * gd * (be.psx - g.du), gpy = 2.0f * gd * (be.psy - g.dv);
                    float xt[3], yt[3];
                    pos_at(fd, tau[j], xt, yt);
                    // per-vertex gradient at tau (gt) and at keyframe X (gk)
                    float gtx[3], gty[3], gkx[3], gky[3];
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const float wq = be.be == q ? 1.0f - be.sg : (be.be == (q + 2) % 3 ? be.sg : 0.0f);
                        gtx[q] = wq * gpx;
                        gty[q] = wq * gpy;
                        gkx[q] = 0.0f;
                        gky[q] = 0.0f;
                    }
                    const bool interior = !(be.sr < 0.0f) && !(be.sr > 1.0f);
                    if (interior) {
                        const int ea = be.be;
                        const float exs = ea == 0 ? es.ex[0] : (ea == 1 ? es.ex[1] : es.ex[2]);
                        const float eys = ea == 0 ? es.ey[0] : (ea == 1 ? es.ey[1] : es.ey[2]);
                        const float iee = ea == 0 ? es.inv_ee[0] : (ea == 1 ? es.inv_ee[1] : es.inv_ee[2]);
                        const float axs = ea == 0 ? es.ax[0] : (ea == 1 ? es.ax[1] : es.ax[2]);
                        const float ays = ea == 0 ? es.ay[0] : (ea == 1 ? es.ay[1] : es.ay[2]);
                        const float xa = ea == 0 ? xt[0] : (ea == 1 ? xt[1] : xt[2]);
                        const float ya = ea == 0 ? yt[0] : (ea == 1 ? yt[1] : yt[2]);
                        const float xb = ea == 0 ? xt[1] : (ea == 1 ? xt[2] : xt[0]);
                        const float yb = ea == 0 ? yt[1] : (ea == 1 ? yt[2] : yt[0]);
                        const float gsig = fmaf(gpx, xb - xa, gpy * (yb - ya));
                        const float rx = be.qx - axs, ry = be.qy - ays;
                        const float grx = gsig * exs * iee, gry = gsig * eys * iee;
                        const float gex = gsig * fmaf(-2.0f * be.sr, exs, rx) * iee;
                        const float gey = gsig * fmaf(-2.0f * be.sr, eys, ry) * iee;
                        float gwq[3];
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            const bool isa = ea == q, isb = ea == (q + 2) % 3;
                            gkx[q] = fmaf(be.w[q], grx, isa ? -grx - gex : (isb ? gex : 0.0f));
                            gky[q] = fmaf(be.w[q], gry, isa ? -gry - gey : (isb ? gey : 0.0f));
                            gwq[q] = fmaf(grx, es.ax[q], gry * es.ay[q]);
                        }
                        const float gxs =
                            fmaf(gwq[0], yt[1] - yt[2], fmaf(gwq[1], yt[2] - yt[0], gwq[2] * (yt[0] - yt[1]))) * invD;
                        const float gys =
                            fmaf(gwq[0], xt[2] - xt[1], fmaf(gwq[1], xt[0] - xt[2], gwq[2] * (xt[1] - xt[0]))) * invD;
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            gtx[q] = fmaf(-be.w[q], gxs, gtx[q]);
                            gty[q] = fmaf(-be.w[q], gys, gty[q]);
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
                flush_face<false>(hit, gK, gA, fd, ck.s, a, ga);
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
