/*
 * motion_blur_raster.h -- C ABI of the MI355X (gfx950) motion-blur
 * differentiable rasterizer.
 *
 * Method: arXiv 2602.07860, "Recovering 3D Shapes from Ultra-Fast
 * Motion-Blurred Images".  The problem is I, alpha = R(V, C) for a triangle
 * mesh with vertex positions V and per-vertex attributes C under a known
 * camera and a known blur motion (Sec. 5.1).  Each output pixel averages K
 * sub-frames at t_k = k/(K-1) (Sec. 3.2); the motion is cut into S segments
 * inside which every vertex moves linearly between two keyframes (Sec. 3.3,
 * eqs 4-6).  Barycentric weights of every (pixel, face, sub-frame) come from
 * the fast solver w(t) = (A1 t^2 + A2 t + A3)/(a1 t^2 + a2 t + a3) (eqs 7-8,
 * App. B), or, with RB_SOLVER_RECOMPUTE, from a fresh 3x3 solve per sub-frame
 * (eqs 1-3).  Covered pixels take the z-buffer winner's interpolated
 * attributes (eq 9); uncovered pixels take alpha = 1 - prod_j (1 - A_j) with
 * A_j = exp(-d_j/delta) (eqs 10, 15) and d_j the squared distance to face j
 * measured through the keyframe closest-point approximation (eqs 13-14,
 * App. B "Euclidean Distance Approximation").  The backward pass is the exact
 * derivative of that forward with every discrete decision held fixed
 * (Sec. 3.3 "Gradient Computation").
 *
 * Conventions (all entry points):
 *  - Every pointer argument is a DEVICE pointer unless stated otherwise.
 *  - The caller owns all memory (rb_render_blur_fwd_static excepted: it
 *    uses a library-held device array).  The library never allocates and
 *    never synchronizes; work is enqueued on the given stream (a hipStream_t
 *    passed as void*, NULL = the default stream).  rb_read_header,
 *    rb_batch_read_headers and rb_profile_read are the calls that wait, and
 *    say so.
 *  - Layouts are dense, row-major, float32 / int32.
 *  - Nothing throws across the ABI; failures are negative rb_status codes.
 *    Asynchronous device-side findings (face index out of range, vertex
 *    behind the camera, bin-list overflow) are written to the workspace
 *    header and read with rb_read_header.
 *  - Calls that share a workspace must not overlap in time.  Distinct
 *    workspaces may be used concurrently from several threads / streams.
 *  - Every call is a fixed sequence of kernel launches on the stream (no
 *    host-device copies, no allocation), so it can be captured in a hipGraph
 *    and replayed.
 */
#ifndef MOTION_BLUR_RASTER_H
#define MOTION_BLUR_RASTER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rb_status;
enum {
    RB_OK = 0,
    RB_EINVAL = -1,        /* null pointer, size <= 0, delta <= 0, eps outside (0,1), ... */
    RB_ERANGE = -2,        /* (header) a face index lies outside [0, V)                  */
    RB_EWORKSPACE = -3,    /* workspace smaller than rb_workspace_size reports           */
    RB_EBEHIND = -4,       /* (header) a keyframe vertex has camera depth <= 1e-6        */
    RB_EOVERFLOW = -5,     /* (header) bin lists exceeded list_capacity: enlarge, rerun  */
    RB_EDEVICE = -6,       /* a HIP runtime call failed                                  */
    RB_EUNSUPPORTED = -7   /* channel count, face count or option the library lacks     */
};

enum { RB_SOLVER_FAST = 0, RB_SOLVER_RECOMPUTE = 1 };

/* rb_options.flags.
 * RB_FLAG_DETERMINISTIC: image and gradients are bitwise the same on every
 * run with the same inputs, options and device, whatever order the GPU's
 * waves run in (the default mode adds partial sums with floating-point
 * atomics, whose order varies, so its results vary in the last bits).  The
 * library then (1) sorts every bin list into face order, (2) gives each
 * (chunk, tile) a single background task, so that one wave adds up each
 * (pixel, sub-frame)'s factors, and (3) adds the gradient partial sums as
 * 64-bit integers in units of 2^(e - 32), where 2^(e-1) <= max |dL/dI| < 2^e,
 * converting them to float at the end.  Slower; results agree with the
 * default mode to float rounding and the unit above.  A partial sum of
 * 2^30 max |dL/dI| or more (or a NaN) sets header bit 8 and fills that
 * instance's gradients with NaN. */
#define RB_FLAG_DETERMINISTIC 1

#define RB_MAX_CHANNELS 4          /* attributes per vertex (C)            */
#define RB_MAX_FACES (1 << 23)     /* faces per mesh                       */
#define RB_MAX_CHUNK 8             /* sub-frames per work chunk            */

/* Perspective camera (App. I, eqs A33-A34): a world point P maps to camera
 * coordinates X = view[:, :3] P + view[:, 3] (camera looks along +Z) and to
 * normalized image coordinates x = X.x / (X.z tan_half_fov),
 * y = X.y / (X.z tan_half_fov).  Pixel (row r, column c) has its centre at
 * ((2c + 1 - W) / W, (H - 2r - 1) / H): row 0 is the top row. */
typedef struct {
    float view[12];            /* HOST array, row-major 3x4 world -> camera  */
    float tan_half_fov;        /* > 0                                        */
    int32_t width, height;     /* W, H >= 1                                  */
} rb_camera;

/* Blur motion (Sec. 3.3): S linear segments between S+1 keyframes at
 * t_s = s/S.  keyframe_model[s] is the row-major 3x4 rigid transform taking a
 * rest vertex to its position at t_s; the vertex moves linearly in screen
 * space between consecutive keyframes (eq 5). */
typedef struct {
    int32_t num_segments;          /* S >= 1                                   */
    const float *keyframe_model;   /* DEVICE, [S+1][3][4]                      */
} rb_motion;

typedef struct {
    int32_t num_subframes;   /* K >= 1 (paper: >= 50 for translation)           */
    float delta;             /* softness of the background probability (1e-4)  */
    float eps_cutoff;        /* probabilities A < eps are dropped: 0 < eps < 1  */
    int32_t solver;          /* RB_SOLVER_FAST or RB_SOLVER_RECOMPUTE           */
    int32_t flags;           /* 0 or RB_FLAG_DETERMINISTIC                      */
    int32_t chunk_len;       /* max sub-frames per work chunk: 1, 2, 4 or 8; 0 = 4;
                                a segment is split into equal chunks         */
    int32_t slice_len;       /* background-list entries per task; 0 = auto (64) */
    int64_t list_capacity;   /* bin-list entries (foreground + background); 0 = auto */
    int32_t tile_w;          /* tile width in pixels: 4, 8 or 16 (height 64 / tile_w,
                                one 64-lane wave per tile); 0 = 8              */
    int32_t reserved;        /* 0                                               */
} rb_options;

/* Device-side findings of the last call on a workspace (rb_read_header). */
typedef struct {
    int32_t error_bits;      /* 1: face index out of range, 2: vertex behind camera, 4: overflow,
                                8: deterministic gradient sum out of range (RB_FLAG_DETERMINISTIC) */
    int32_t reserved;
    int64_t list_entries;    /* entries the last forward needed (fg + bg)        */
    int64_t list_capacity;   /* entries available                                */
} rb_header;

/* Bytes of device workspace for these sizes (HOST only; no device access).
 * The forward keeps in it what the backward reuses (keyframes, bin lists,
 * per pixel-sub-frame visibility), so one workspace serves a fwd/bwd pair.
 * Returns RB_OK, RB_EINVAL or RB_EUNSUPPORTED. */
rb_status rb_workspace_size(int32_t V, int32_t F, int32_t C, const rb_motion *motion,
                            const rb_camera *camera, const rb_options *options, size_t *bytes);

/* Argument checks of rb_render_blur_fwd/bwd without touching the device
 * (HOST only).  Returns the status those calls would return before launch. */
rb_status rb_validate(int32_t V, int32_t F, int32_t C, const rb_motion *motion,
                      const rb_camera *camera, const rb_options *options, size_t workspace_bytes);

/* Forward render.  verts [V][3] rest positions, faces [F][3] vertex indices,
 * attrs [V][C]; image [C+1][H][W] is overwritten with the K-sub-frame average
 * of (attributes, alpha) -- background pixels carry zero attributes.
 * If the bin lists overflow (header bit 4) the image is filled with NaN. */
rb_status rb_render_blur_fwd(const float *verts, int32_t V, const int32_t *faces, int32_t F,
                             const float *attrs, int32_t C, const rb_motion *motion,
                             const rb_camera *camera, const rb_options *options, float *image,
                             void *workspace, size_t workspace_bytes, void *stream);

/* Forward render without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments and output as
 * rb_render_blur_fwd; the workspace is a library-held device array of
 * RB_STATIC_SCRATCH_BYTES, one per device, kept until the process ends.
 * Returns RB_EWORKSPACE when rb_workspace_size reports more than that for
 * these sizes (lower options->list_capacity, or use rb_render_blur_fwd).
 * Calls no allocator.  Every call on a device reuses that device's array
 * (the forward initialises what it reads), so calls that overlap in time on
 * one device race; the array's state is not kept for a backward pass and
 * its header cannot be read (an overflow shows as a NaN image). */
#define RB_STATIC_SCRATCH_BYTES (64u << 20)
rb_status rb_render_blur_fwd_static(const float *verts, int32_t V, const int32_t *faces, int32_t F,
                                    const float *attrs, int32_t C, const rb_motion *motion,
                                    const rb_camera *camera, const rb_options *options, float *image,
                                    void *stream);

/* Backward (adjoint) pass.  Same inputs and the SAME workspace as the forward
 * it differentiates, untouched in between.  grad_image [C+1][H][W] is
 * dL/dimage; grad_verts [V][3] and grad_attrs [V][C] are OVERWRITTEN with
 * dL/dverts and dL/dattrs. */
rb_status rb_render_blur_bwd(const float *verts, int32_t V, const int32_t *faces, int32_t F,
                             const float *attrs, int32_t C, const rb_motion *motion,
                             const rb_camera *camera, const rb_options *options,
                             const float *grad_image, float *grad_verts, float *grad_attrs,
                             void *workspace, size_t workspace_bytes, void *stream);

/* Copies the workspace header to *out (HOST pointer).  SYNCHRONIZES the
 * stream.  Returns RB_OK, RB_EINVAL or RB_EDEVICE. */
rb_status rb_read_header(const void *workspace, rb_header *out, void *stream);

/* Batched rendering: n meshes of any sizes, sub-frame counts and image sizes
 * in one sequence of launches, every kernel covering all instances (the
 * background passes are persistent kernels over the tasks of all instances).
 * The rb_instance array is HOST memory holding DEVICE pointers.  options
 * supplies delta, eps_cutoff, solver, flags, chunk_len, slice_len and tile_w
 * for the whole batch; num_subframes and list_capacity of options are ignored
 * in favour of each instance's own.  mode RB_BATCH_FORWARD writes every instance's image;
 * RB_BATCH_BACKWARD reads grad_image and overwrites grad_verts / grad_attrs,
 * reusing the state the forward left in the same workspace. */
typedef struct {
    const float *verts;      /* [V][3]                                          */
    int32_t V;
    const int32_t *faces;    /* [F][3]                                          */
    int32_t F;
    const float *attrs;      /* [V][C]                                          */
    int32_t C;
    rb_motion motion;
    rb_camera camera;
    int32_t num_subframes;   /* K >= 1                                          */
    int64_t list_capacity;   /* bin-list entries; 0 = auto                      */
    float *image;            /* [C+1][H][W], forward output                     */
    const float *grad_image; /* [C+1][H][W], backward input                     */
    float *grad_verts;       /* [V][3], backward output                         */
    float *grad_attrs;       /* [V][C], backward output                         */
} rb_instance;

enum { RB_BATCH_FORWARD = 0, RB_BATCH_BACKWARD = 1 };

/* Workspace bytes for a batch (HOST only).  Returns RB_OK, RB_EINVAL or
 * RB_EUNSUPPORTED (n <= 0 or an instance's sizes). */
rb_status rb_batch_workspace_size(const rb_instance *instances, int32_t n, const rb_options *options,
                                  size_t *bytes);

/* Render a batch (see above).  Returns the first failing instance's status
 * for argument errors, RB_EWORKSPACE or RB_EDEVICE. */
rb_status rb_render_blur_batched(const rb_instance *instances, int32_t n, const rb_options *options,
                                 int32_t mode, void *workspace, size_t workspace_bytes, void *stream);

/* Headers of every instance of a batch into out[n] (HOST).  SYNCHRONIZES. */
rb_status rb_batch_read_headers(const rb_instance *instances, int32_t n, const rb_options *options,
                                const void *workspace, rb_header *out, void *stream);

/* Kernel timing for benchmarks.  While enabled, every call records HIP events
 * on its stream between its kernels.  Forward: projection (with workspace
 * initialisation), binning, foreground pass (with the background task list),
 * background pass, sub-frame average.  Backward: foreground adjoint (with
 * the gradient clear), background adjoint, vertex-gradient mapping.
 * rb_profile_read SYNCHRONIZES on those events, returns the accumulated
 * milliseconds and call counts, and clears them.  Enabling or disabling also
 * clears.  Thread-safe. */
typedef struct {
    double project_ms, bin_ms, fg_ms, bg_ms, resolve_ms;   /* forward phases  */
    double fg_bwd_ms, bg_bwd_ms, vertex_grad_ms;           /* backward phases */
    int64_t fwd_calls, bwd_calls;
} rb_profile_stats;

rb_status rb_profile_enable(int32_t enable);
rb_status rb_profile_read(rb_profile_stats *out);

/* Static description of a status code. */
const char *rb_status_string(rb_status status);

#ifdef __cplusplus
}
#endif
#endif /* MOTION_BLUR_RASTER_H */
