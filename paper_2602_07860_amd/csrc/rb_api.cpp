// Host entry points of the C ABI declared in motion_blur_raster.h:
// argument validation, the launch plan (tiles, sub-frame chunks, workspace
// layout) and the kernel sequence.  No allocation, no synchronization (except
// rb_read_header, documented as waiting).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "rb_internal.h"

namespace rb {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static rb_status make_plan(int32_t V, int32_t F, int32_t C, const rb_motion *motion, const rb_camera *cam,
                           const rb_options *opt, Plan &p)
{
    if (!motion || !cam || !opt) return RB_EINVAL;
    if (V <= 0 || F <= 0 || C <= 0) return RB_EINVAL;
    if (motion->num_segments <= 0 || opt->num_subframes <= 0) return RB_EINVAL;
    if (cam->width <= 0 || cam->height <= 0) return RB_EINVAL;
    if (!(cam->tan_half_fov > 0.0f) || !std::isfinite(cam->tan_half_fov)) return RB_EINVAL;
    if (!(opt->delta > 0.0f) || !std::isfinite(opt->delta)) return RB_EINVAL;
    if (!(opt->eps_cutoff > 0.0f && opt->eps_cutoff < 1.0f)) return RB_EINVAL;
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(cam->view[i])) return RB_EINVAL;
    if (opt->solver != RB_SOLVER_FAST && opt->solver != RB_SOLVER_RECOMPUTE) return RB_EINVAL;
    if (opt->chunk_len < 0 || opt->slice_len < 0 || opt->list_capacity < 0) return RB_EINVAL;
    if (opt->flags & ~RB_FLAG_DETERMINISTIC) return RB_EINVAL;
    if (opt->tile_w < 0 || opt->reserved != 0) return RB_EINVAL;
    if (opt->tile_w != 0 && opt->tile_w != 4 && opt->tile_w != 8 && opt->tile_w != 16) return RB_EUNSUPPORTED;
    if (C > RB_MAX_CHANNELS) return RB_EUNSUPPORTED;
    if (F >= RB_MAX_FACES) return RB_EUNSUPPORTED;
    const int T = opt->chunk_len == 0 ? 4 : opt->chunk_len;
    if (T != 1 && T != 2 && T != 4 && T != 8) return RB_EUNSUPPORTED;
    const int S = motion->num_segments, K = opt->num_subframes;
    // sub-frame index arithmetic k*S must stay in int range
    if ((long long)K * S >= (1LL << 31)) return RB_EUNSUPPORTED;

    p.V = V;
    p.F = F;
    p.C = C;
    p.S = S;
    p.K = K;
    p.W = cam->width;
    p.H = cam->height;
    p.tanf = cam->tan_half_fov;
    p.delta = opt->delta;
    const double dmax = (double)opt->delta * std::log(1.0 / (double)opt->eps_cutoff);
    p.dmax = (float)dmax;
    p.halo = (float)(std::sqrt(dmax) * (1.0 + 1e-6));
    std::memcpy(p.view, cam->view, sizeof(p.view));
    p.solver = opt->solver;
    p.tw = opt->tile_w ? opt->tile_w : kTileWDefault;
    p.th = kWave / p.tw;
    p.tiles_x = (p.W + p.tw - 1) / p.tw;
    p.tiles_y = (p.H + p.th - 1) / p.th;
    p.ntiles = p.tiles_x * p.tiles_y;
    int nmax = 0;
    for (int s = 0; s < S; ++s) {
        int lo = seg_first(s, K, S), hi = (s == S - 1) ? K : seg_first(s + 1, K, S);
        nmax = std::max(nmax, hi - lo);
    }
    p.CPS = std::max(1, (nmax + T - 1) / T);
    // chunk_len bounds the chunk; the kernels are built for the longest chunk
    // the balanced split makes (1, 2, 3, 4 or 8 sub-frames), which keeps the
    // per-lane sub-frame arrays (and register use) no larger than needed
    const int lmax = (nmax + p.CPS - 1) / p.CPS;
    p.T = lmax <= 4 ? std::max(1, lmax) : 8;
    p.NC = S * p.CPS;
    // 32-bit chunk and (chunk, tile) index arithmetic on the device
    if ((long long)p.CPS * K >= (1LL << 31) || (long long)p.NC * p.ntiles >= (1LL << 31)) return RB_EUNSUPPORTED;
    // background list entries per task: small enough that the longest lists
    // (silhouette tiles) spread over many waves, large enough to amortize a
    // task's set-up
    p.det = (opt->flags & RB_FLAG_DETERMINISTIC) != 0;
    p.SL = p.det ? kDetSliceLen : (opt->slice_len > 0 ? opt->slice_len : 64);
    // When the background halo spans many pixels, faces reach many pixels of
    // a tile: longer per-lane runs of items pay off in the background adjoint
    // (fewer LDS atomics per item), and the background forward groups its
    // items by pixel so that runs add up one pixel's factors (measured on
    // 256^2 with a 5.5-pixel halo and 1024^2 with a 22-pixel halo).
    const bool wide_halo = std::sqrt(dmax) * 0.5 * std::max(p.W, p.H) >= 12.0;
    p.seq_bg = wide_halo ? 8 : 4;
    // foreground adjoint: chunks of a segment grouped per wave on large
    // images (fewer flushes), one per wave otherwise (more waves in flight;
    // grouping measured slower on the mixed batch of small images)
    p.fgg = wide_halo ? 3 : 1;
    // background adjoint: units of two tasks where faces reach few pixels
    // (per-task steps weigh more there); single tasks on wide halos
    p.bwd_merge = wide_halo ? 1 : 2;
    p.wide = wide_halo;
    p.NS = std::max(C, 3);
    p.nfb = (F + 255) / 256;
    p.cap = opt->list_capacity > 0 ? opt->list_capacity
                                   : std::max<int64_t>(1 << 20, (int64_t)64 * F * std::min(p.NC, 64));
    p.ncounts = (int64_t)2 * p.NC * p.ntiles;
    p.nblocks_scan = std::max<int64_t>(1, (p.ncounts + 4095) / 4096);
    p.ntct = (int64_t)p.NC * p.ntiles;
    p.nblocks_tscan = std::max<int64_t>(1, (p.ntct + 4095) / 4096);
    // every (chunk, tile) contributes at most ceil(n_bg / SL) <= n_bg / SL + 1 tasks
    p.maxtasks = p.ntct + p.cap / p.SL + 1;

    size_t o = 0;
    p.o_hdr = o;
    o = align256(o + sizeof(DevHeader));
    p.o_kf = o;
    o = align256(o + (size_t)(S + 1) * V * sizeof(double2));
    p.o_kfz = o;
    o = align256(o + (size_t)(S + 1) * V * sizeof(float));
    p.o_cnt = o;
    o = align256(o + (size_t)p.ncounts * 4);
    p.o_off = o;
    o = align256(o + (size_t)p.ncounts * 8);
    p.o_cur = o;
    o = align256(o + (size_t)p.ncounts * 4);
    p.o_bsum = o;
    o = align256(o + (size_t)p.nblocks_scan * 8);
    p.o_list = o;
    o = align256(o + (size_t)p.cap * 4);
    p.o_vis_id = o;
    o = align256(o + (size_t)p.ntiles * K * kWave * 4);
    p.o_pix = o;
    o = align256(o + (size_t)p.ntiles * K * p.NS * kWave * 4);
    p.o_tsl = o;
    o = align256(o + (size_t)p.ntct * 4);
    p.o_toff = o;
    o = align256(o + (size_t)p.ntct * 8);
    p.o_tbsum = o;
    o = align256(o + (size_t)p.nblocks_tscan * 8);
    p.o_tasks = o;
    o = align256(o + (size_t)p.maxtasks * 8);
    p.o_gkf = o;
    o = align256(o + (size_t)(S + 1) * V * 2 * 4);
    p.o_fgw = o;
    o = align256(o + (size_t)p.ntct * 4);
    p.o_gfx = o;
    if (p.det) o = align256(o + ((size_t)(S + 1) * V * 2 + (size_t)V * C) * 8);
    p.total = o;
    return RB_OK;
}

// Plan a batch: instance workspaces one after another (256-byte aligned),
// then the device instance table and the batch's task numbering.
static rb_status make_batch(const std::vector<Plan> &plans, Batch &bt)
{
    bt.n = (int)plans.size();
    if (bt.n <= 0) return RB_EINVAL;
    // every instance's chunks hold at most its own p.T <= the batch template
    bt.T = 1;
    for (const Plan &p : plans) bt.T = std::max(bt.T, p.T);
    bt.solver = plans[0].solver;
    bt.wide = true;
    for (const Plan &p : plans) bt.wide = bt.wide && p.wide;
    bt.det = plans[0].det;
    bt.tw = plans[0].tw;
    bt.plans = plans;
    bt.base.resize(bt.n);
    Grids g{};
    size_t o = 0;
    for (int i = 0; i < bt.n; ++i) {
        const Plan &p = plans[i];
        bt.base[i] = o;
        o = align256(o + p.total);
        const Grids q = plan_grids(p);
        g.init += q.init;
        g.proj += q.proj;
        g.bin += q.bin;
        g.scan1 += q.scan1;
        g.scan3 += q.scan3;
        g.tscan1 += q.tscan1;
        g.tscan3 += q.tscan3;
        g.fg += q.fg;
        g.fgb += q.fgb;
        g.res += q.res;
        g.bwdinit += q.bwdinit;
        g.vtx += q.vtx;
        g.sort += q.sort;
        g.detp += q.detp;
    }
    // one launch covers every instance: block counts must fit the grid and
    // the 32-bit block starts of the table
    const int64_t lim = (1LL << 31) - 1;
    for (int64_t v : {g.init, g.proj, g.bin, g.scan1, g.scan3, g.tscan1, g.tscan3, g.fg, g.fgb, g.res, g.bwdinit, g.vtx,
                      g.sort, g.detp})
        if (v > lim) return RB_EUNSUPPORTED;
    bt.g = g;
    bt.o_table = o;
    o = align256(o + (size_t)bt.n * sizeof(Inst));
    bt.o_tprefix = o;
    o = align256(o + (size_t)(bt.n + 1) * sizeof(int64_t));
    bt.total = o;
    return RB_OK;
}

static rb_status single_batch(int32_t V, int32_t F, int32_t C, const rb_motion *motion, const rb_camera *camera,
                              const rb_options *options, Batch &bt)
{
    Plan p;
    rb_status st = make_plan(V, F, C, motion, camera, options, p);
    if (st != RB_OK) return st;
    return make_batch(std::vector<Plan>{p}, bt);
}

// per-instance options of a batch: the batch's, with the instance's K and capacity
static rb_status batch_plans(const rb_instance *inst, int32_t n, const rb_options *opt, std::vector<Plan> &plans)
{
    if (!inst || !opt || n <= 0) return RB_EINVAL;
    plans.resize(n);
    for (int i = 0; i < n; ++i) {
        rb_options o = *opt;
        o.num_subframes = inst[i].num_subframes;
        o.list_capacity = inst[i].list_capacity;
        rb_status st = make_plan(inst[i].V, inst[i].F, inst[i].C, &inst[i].motion, &inst[i].camera, &o, plans[i]);
        if (st != RB_OK) return st;
    }
    return RB_OK;
}

// ---- benchmark timing (rb_profile_*)
struct ProfRec {
    int kind;   // 0 forward, 1 backward
    PhaseEvents pe;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof;

static void prof_clear_locked()
{
    for (auto &r : g_prof)
        for (auto e : r.pe.ev)
            if (e) (void)hipEventDestroy(e);
    g_prof.clear();
}

// events for one call, or nullptr when timing is off
static const PhaseEvents *prof_begin(int kind, PhaseEvents &pe)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return nullptr;
    const int n = kind == 0 ? 6 : 4;
    for (int i = 0; i < 6; ++i) pe.ev[i] = nullptr;
    for (int i = 0; i < n; ++i)
        if (hipEventCreate(&pe.ev[i]) != hipSuccess) pe.ev[i] = nullptr;
    g_prof.push_back(ProfRec{kind, pe});
    return &pe;
}

}  // namespace rb

using namespace rb;

extern "C" {

rb_status rb_workspace_size(int32_t V, int32_t F, int32_t C, const rb_motion *motion, const rb_camera *camera,
                            const rb_options *options, size_t *bytes)
{
    if (!bytes) return RB_EINVAL;
    Batch bt;
    rb_status st = single_batch(V, F, C, motion, camera, options, bt);
    if (st != RB_OK) return st;
    *bytes = bt.total;
    return RB_OK;
}

rb_status rb_validate(int32_t V, int32_t F, int32_t C, const rb_motion *motion, const rb_camera *camera,
                      const rb_options *options, size_t workspace_bytes)
{
    Batch bt;
    rb_status st = single_batch(V, F, C, motion, camera, options, bt);
    if (st != RB_OK) return st;
    if (!motion->keyframe_model) return RB_EINVAL;
    if (workspace_bytes < bt.total) return RB_EWORKSPACE;
    return RB_OK;
}

rb_status rb_render_blur_fwd(const float *verts, int32_t V, const int32_t *faces, int32_t F, const float *attrs,
                             int32_t C, const rb_motion *motion, const rb_camera *camera, const rb_options *options,
                             float *image, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!verts || !faces || !attrs || !image || !workspace) return RB_EINVAL;
    rb_status st = rb_validate(V, F, C, motion, camera, options, workspace_bytes);
    if (st != RB_OK) return st;
    Batch bt;
    single_batch(V, F, C, motion, camera, options, bt);
    std::vector<Io> io{Io{verts, faces, attrs, motion->keyframe_model, image, nullptr, nullptr, nullptr}};
    PhaseEvents pe;
    const PhaseEvents *pp = prof_begin(0, pe);
    hipError_t e = launch_forward(bt, io, workspace, (hipStream_t)stream, pp);
    return e == hipSuccess ? RB_OK : RB_EDEVICE;
}

rb_status rb_render_blur_fwd_static(const float *verts, int32_t V, const int32_t *faces, int32_t F,
                                    const float *attrs, int32_t C, const rb_motion *motion, const rb_camera *camera,
                                    const rb_options *options, float *image, void *stream)
{
    if (!verts || !faces || !attrs || !image) return RB_EINVAL;
    Batch bt;
    rb_status st = single_batch(V, F, C, motion, camera, options, bt);
    if (st != RB_OK) return st;
    if (!motion->keyframe_model) return RB_EINVAL;
    if (bt.total > (size_t)RB_STATIC_SCRATCH_BYTES) return RB_EWORKSPACE;
    void *ws = nullptr;
    if (static_scratch(&ws) != hipSuccess) return RB_EDEVICE;
    std::vector<Io> io{Io{verts, faces, attrs, motion->keyframe_model, image, nullptr, nullptr, nullptr}};
    PhaseEvents pe;
    const PhaseEvents *pp = prof_begin(0, pe);
    hipError_t e = launch_forward(bt, io, ws, (hipStream_t)stream, pp);
    return e == hipSuccess ? RB_OK : RB_EDEVICE;
}

rb_status rb_render_blur_bwd(const float *verts, int32_t V, const int32_t *faces, int32_t F, const float *attrs,
                             int32_t C, const rb_motion *motion, const rb_camera *camera, const rb_options *options,
                             const float *grad_image, float *grad_verts, float *grad_attrs, void *workspace,
                             size_t workspace_bytes, void *stream)
{
    if (!verts || !faces || !attrs || !grad_image || !grad_verts || !grad_attrs || !workspace) return RB_EINVAL;
    rb_status st = rb_validate(V, F, C, motion, camera, options, workspace_bytes);
    if (st != RB_OK) return st;
    Batch bt;
    single_batch(V, F, C, motion, camera, options, bt);
    std::vector<Io> io{Io{verts, faces, attrs, motion->keyframe_model, nullptr, grad_image, grad_verts, grad_attrs}};
    PhaseEvents pe;
    const PhaseEvents *pp = prof_begin(1, pe);
    hipError_t e = launch_backward(bt, io, workspace, (hipStream_t)stream, pp);
    return e == hipSuccess ? RB_OK : RB_EDEVICE;
}

rb_status rb_batch_workspace_size(const rb_instance *instances, int32_t n, const rb_options *options, size_t *bytes)
{
    if (!bytes) return RB_EINVAL;
    std::vector<Plan> plans;
    rb_status st = batch_plans(instances, n, options, plans);
    if (st != RB_OK) return st;
    Batch bt;
    st = make_batch(plans, bt);
    if (st != RB_OK) return st;
    *bytes = bt.total;
    return RB_OK;
}

rb_status rb_render_blur_batched(const rb_instance *instances, int32_t n, const rb_options *options, int32_t mode,
                                 void *workspace, size_t workspace_bytes, void *stream)
{
    if (!workspace || (mode != RB_BATCH_FORWARD && mode != RB_BATCH_BACKWARD)) return RB_EINVAL;
    std::vector<Plan> plans;
    rb_status st = batch_plans(instances, n, options, plans);
    if (st != RB_OK) return st;
    Batch bt;
    st = make_batch(plans, bt);
    if (st != RB_OK) return st;
    if (workspace_bytes < bt.total) return RB_EWORKSPACE;
    std::vector<Io> io(n);
    for (int i = 0; i < n; ++i) {
        const rb_instance &x = instances[i];
        if (!x.verts || !x.faces || !x.attrs || !x.motion.keyframe_model) return RB_EINVAL;
        if (mode == RB_BATCH_FORWARD && !x.image) return RB_EINVAL;
        if (mode == RB_BATCH_BACKWARD && (!x.grad_image || !x.grad_verts || !x.grad_attrs)) return RB_EINVAL;
        io[i] = Io{x.verts, x.faces, x.attrs, x.motion.keyframe_model, x.image, x.grad_image, x.grad_verts,
                   x.grad_attrs};
    }
    PhaseEvents pe;
    const PhaseEvents *pp = prof_begin(mode == RB_BATCH_FORWARD ? 0 : 1, pe);
    hipError_t e = mode == RB_BATCH_FORWARD ? launch_forward(bt, io, workspace, (hipStream_t)stream, pp)
                                             : launch_backward(bt, io, workspace, (hipStream_t)stream, pp);
    return e == hipSuccess ? RB_OK : RB_EDEVICE;
}

rb_status rb_batch_read_headers(const rb_instance *instances, int32_t n, const rb_options *options,
                                const void *workspace, rb_header *out, void *stream)
{
    if (!workspace || !out) return RB_EINVAL;
    std::vector<Plan> plans;
    rb_status st = batch_plans(instances, n, options, plans);
    if (st != RB_OK) return st;
    Batch bt;
    st = make_batch(plans, bt);
    if (st != RB_OK) return st;
    for (int i = 0; i < n; ++i) {
        st = rb_read_header((const char *)workspace + bt.base[i], &out[i], stream);
        if (st != RB_OK) return st;
    }
    return RB_OK;
}

rb_status rb_read_header(const void *workspace, rb_header *out, void *stream)
{
    if (!workspace || !out) return RB_EINVAL;
    DevHeader h;
    hipStream_t st = (hipStream_t)stream;
    if (hipMemcpyAsync(&h, workspace, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return RB_EDEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return RB_EDEVICE;
    out->error_bits = h.error_bits;
    out->reserved = 0;
    out->list_entries = h.list_entries;
    out->list_capacity = h.list_capacity;
    return RB_OK;
}

rb_status rb_profile_enable(int32_t enable)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_clear_locked();
    g_prof_on = enable != 0;
    return RB_OK;
}

rb_status rb_profile_read(rb_profile_stats *out)
{
    if (!out) return RB_EINVAL;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    std::memset(out, 0, sizeof(*out));
    rb_status st = RB_OK;
    auto span = [&](hipEvent_t a, hipEvent_t b) -> double {
        float ms = 0.0f;
        if (!a || !b) return 0.0;
        if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) {
            st = RB_EDEVICE;
            return 0.0;
        }
        return (double)ms;
    };
    for (auto &r : g_prof) {
        const hipEvent_t *e = r.pe.ev;
        if (r.kind == 0) {
            out->project_ms += span(e[0], e[1]);
            out->bin_ms += span(e[1], e[2]);
            out->fg_ms += span(e[2], e[3]);
            out->bg_ms += span(e[3], e[4]);
            out->resolve_ms += span(e[4], e[5]);
            out->fwd_calls += 1;
        } else {
            out->fg_bwd_ms += span(e[0], e[1]);
            out->bg_bwd_ms += span(e[1], e[2]);
            out->vertex_grad_ms += span(e[2], e[3]);
            out->bwd_calls += 1;
        }
    }
    prof_clear_locked();
    return st;
}

const char *rb_status_string(rb_status s)
{
    switch (s) {
    case RB_OK: return "ok";
    case RB_EINVAL: return "invalid argument";
    case RB_ERANGE: return "face index out of range";
    case RB_EWORKSPACE: return "workspace too small";
    case RB_EBEHIND: return "vertex behind the camera";
    case RB_EOVERFLOW: return "bin list capacity exceeded";
    case RB_EDEVICE: return "HIP runtime error";
    case RB_EUNSUPPORTED: return "unsupported size or option";
    default: return "unknown status";
    }
}

}  // extern "C"
