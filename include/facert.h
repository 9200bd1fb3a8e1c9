/*
 * facert: differentiable light-stage face rendering on AMD Instinct MI355X.
 *
 * The operations follow Dib et al., "Face Reflectance and Geometry Modeling
 * via Differentiable Ray Tracing" (CVMP 2019):
 *   - fr_blend: the morphable model of the Face Modeling paragraph, identity
 *     alpha (80), expression beta (90), albedo delta (80), geometry transform
 *     [R t] (6), and the vertex normals n_i(alpha, beta, R, t);
 *   - fr_render: p^T = F(f_r, l_j, alpha, beta, R, t) of the Optimization
 *     paragraph, the Monte-Carlo estimator of the lighting equation in a
 *     virtual light stage of N oriented area lights with colour intensities
 *     l_j, Cook-Torrance reflectance (Lambertian albedo + gray specular
 *     texture c_spec) and ray-traced self-shadows;
 *   - fr_backward: the gradient of a loss given its image gradient, e.g.
 *     E_data = sum ||p^T - p^R||^2 of Eq. 1, with respect to the light
 *     colours, specular texels, vertex positions and albedo and, through the
 *     model, alpha, beta, delta and the pose, including the edge-sampling
 *     terms of visibility discontinuities (Face Modeling paragraph: the
 *     differentiable ray tracer, then backpropagation).
 *
 * Conventions for every entry point:
 *   - status: 0 on success, negative fr_status on failure; nothing throws.
 *     On failure the context stays usable and fr_last_error() describes it.
 *   - memory: the context owns its own device buffers (model copies, BVH,
 *     edge tables, scratch).  Every array argument is owned by the caller.
 *     fr_create copies its host arrays.  The array arguments of the compute
 *     calls (fr_blend, fr_render, fr_backward, fr_loss_l2, fr_aov,
 *     fr_light_reg, fr_adam) are, except where a comment says "host":
 *       with FR_DEVICE_PTRS given to fr_create, DEVICE pointers (HIP global
 *       memory) read or written on the context's stream (the PyTorch path);
 *       without it, HOST pointers: the call copies its inputs to device
 *       buffers of the context, runs on the context's stream, copies its
 *       outputs back and waits for the stream before it returns.
 *     Comments below say "device" for the first mode.
 *   - streams: all work is enqueued on the stream set with fr_set_stream
 *     (default: the null stream; fr_render and fr_backward fork part of
 *     their work onto two more streams of the context's own and join them
 *     back) and the calls
 *     return without waiting, except fr_stats and fr_create, which
 *     synchronise.  One context must
 *     not be used from two host threads at once.
 *   - layouts: per-vertex arrays are structure-of-arrays [3][V] (x row, then
 *     y, then z; or r, g, b); bases are [K][3][V]; images are row-major
 *     [H][W][3] float; lights are [n][3] RGB.
 */
#ifndef FACERT_H
#define FACERT_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FR_OK = 0,
    FR_EINVAL = -1,   /* bad argument: size, null, non-finite, degenerate */
    FR_ENOMEM = -2,   /* device allocation failed                        */
    FR_EDEVICE = -3,  /* a HIP call failed; message in fr_last_error     */
    FR_ESTATE = -4    /* call out of order (backward before render)      */
} fr_status;

typedef struct fr_ctx fr_ctx;

/* Morphable face model (host arrays, copied by fr_create). */
typedef struct {
    int32_t n_vertices, n_faces;     /* V, F                                   */
    int32_t n_id, n_exp, n_alb;      /* basis sizes (80, 90, 80 in the paper)  */
    const int32_t *faces;            /* [F][3], counter-clockwise seen from
                                        the front; a manifold mesh (each edge
                                        in at most two faces)                  */
    const float *mean;               /* [3][V] mean shape                      */
    const float *b_id;               /* [n_id][3][V] identity basis            */
    const float *b_exp;              /* [n_exp][3][V] expression basis         */
    const float *alb_mean;           /* [3][V] mean RGB albedo                 */
    const float *b_alb;              /* [n_alb][3][V] albedo basis             */
    const float *uv;                 /* [2][V] specular-texture coordinates    */
} fr_model_desc;

/* Camera and light stage (host arrays, copied by fr_create). */
typedef struct {
    int32_t width, height;           /* image size in pixels                   */
    float cam[3];                    /* pinhole centre; the camera looks along
                                        -z, image y points down               */
    float pix_scale;                 /* size of one pixel on the plane at unit
                                        distance (tan(fov_y/2) / (H/2))        */
    int32_t n_lights;                /* N (20 in the paper), 1..64             */
    const float *light_geom;         /* [N][12]: centre, edge e1, edge e2, unit
                                        emitting normal (along e1 x e2); each
                                        light is the parallelogram
                                        centre + s e1 + t e2, |s|,|t| <= 1/2  */
    int32_t spec_res;                /* specular texture side (32)             */
} fr_scene_desc;

/* Parameters of one evaluation.  Arrays in the context's mode (device with
 * FR_DEVICE_PTRS, else host), except pose, which is always host. */
typedef struct {
    const float *alpha;              /* [n_id]                                 */
    const float *beta;               /* [n_exp]                                */
    const float *delta;              /* [n_alb]                                */
    const float *pose;               /* HOST [6]: rx, ry, rz (radians), t;
                                        R = Rz(rz) Ry(ry) Rx(rx), v = R v + t  */
    const float *lights;             /* [N][3] RGB intensities l_j             */
    const float *spec;               /* [spec_res^2] gray specular texels      */
} fr_params;

/* Gradient outputs (in the context's mode; each nullable; overwritten). */
typedef struct {
    float *d_lights;                 /* [N][3]                                 */
    float *d_spec;                   /* [spec_res^2]                           */
    float *d_vertices;               /* [3][V] w.r.t. posed vertex positions   */
    float *d_albedo;                 /* [3][V] w.r.t. per-vertex albedo        */
    float *d_alpha;                  /* [n_id]                                 */
    float *d_beta;                   /* [n_exp]                                */
    float *d_delta;                  /* [n_alb]                                */
    float *d_pose;                   /* [6]                                    */
} fr_grads;

typedef struct {
    /* rays traced by the last fr_render + fr_backward */
    uint64_t rays_camera, rays_shadow, rays_edge_primary, rays_edge_secondary;
    uint64_t traversal_overflow;     /* must be 0                              */
    uint64_t box_tests, tri_tests;   /* BVH node and ray/triangle tests (the
                                        camera step tests the triangles whose
                                        screen footprint holds the sample)     */
    /* per kernel: [0] camera rays, [1] shadow rays, [2] shading (forward),
       [3] interior adjoint (with any recomputation of hits and visibility),
       [4] camera-silhouette edges, [5] shadow-boundary edges */
    uint64_t kernel_rays[6], kernel_box_tests[6], kernel_tri_tests[6], kernel_shades[6];
    /* milliseconds of the last calls (when FR_TIMING was given)              */
    float ms_blend, ms_bvh, ms_edges, ms_render, ms_backward;
    float ms_kernel[6];              /* the kernels above alone (last chunk)   */
} fr_stats_t;

#define FR_TIMING 1u                 /* fr_create flag: time phases with events */
#define FR_DEVICE_PTRS 4u            /* fr_create flag: the compute calls take
                                        device pointers (see the conventions
                                        above); without it, host pointers     */
#define FR_REFIT  2u                 /* fr_create flag: build the BVH's shape
                                        once, over the model's mean shape, and
                                        only refit its boxes per evaluation,
                                        instead of rebuilding a Morton-code
                                        tree from the posed mesh every
                                        evaluation (the default); results are
                                        identical, only the work differs    */

/* Backward terms (fr_set_terms); all on by default. */
#define FR_TERM_INTERIOR  1u
#define FR_TERM_PRIMARY   2u         /* camera-silhouette edges                 */
#define FR_TERM_SECONDARY 4u         /* shadow-boundary edges                   */

/* Create a context: copies the model and scene to the device, builds the
 * topology (edges, vertex-to-face lists, and the BVH shape when FR_REFIT is
 * given).  flags: FR_TIMING, FR_REFIT, FR_DEVICE_PTRS.
 * Errors: FR_EINVAL (sizes <= 0, null arrays, unknown flags, non-manifold mesh, index out
 * of range, n_lights > 64, more than 2^21 edges), FR_ENOMEM, FR_EDEVICE.
 * *out is NULL on error. */
int fr_create(const fr_model_desc *model, const fr_scene_desc *scene,
              uint32_t flags, fr_ctx **out);

/* Enqueue all later work on this HIP stream (hipStream_t). */
int fr_set_stream(fr_ctx *ctx, void *hip_stream);

/* Select the backward terms (bit set of FR_TERM_*). */
int fr_set_terms(fr_ctx *ctx, uint32_t terms);

/* Camera samples per chunk (1 <= samples <= FR_CHUNK_MAX, default
 * FR_CHUNK_MAX).  fr_render keeps each camera sample's hit record (16 B) and
 * light-visibility mask (8 B) for fr_backward when the whole render fits in
 * one chunk; a larger render (high spp) keeps none and fr_backward
 * recomputes them chunk by chunk.  Takes effect at the next fr_render.
 * Errors: FR_EINVAL. */
#define FR_CHUNK_MAX (1 << 22)
int fr_set_chunk(fr_ctx *ctx, int32_t samples);

/* Morphable blend (Face Modeling paragraph): v_model = mean + B_id alpha +
 * B_exp beta, v = R v_model + t, A = alb_mean + B_alb delta, vertex normals.
 * Sums run over k in ascending order in double precision; positions and
 * albedo are then rounded to float.  out_vertices [3][V] and out_albedo
 * [3][V] (device, nullable) receive copies.  Errors: FR_EINVAL for null
 * alpha/beta/delta/pose or a non-finite pose. */
int fr_blend(fr_ctx *ctx, const float *alpha, const float *beta, const float *delta,
             const float *pose, float *out_vertices, float *out_albedo);

/* Monte-Carlo render (Optimization paragraph, estimator F): blend, BVH refit,
 * edge tables, then per pixel the mean over spp jittered camera samples of
 * the direct light from every light (one area sample and one shadow ray per
 * light per hit).  out_image [H][W][3] (device).  The realisation is fixed by
 * (params, seed, spp) and bitwise reproducible.  The BVH is built on the
 * context's second stream, beside the camera step, the shadow-ray
 * proposals and the edge tables, and joined before the first shadow ray.
 * Errors: FR_EINVAL (spp < 1 or > 4096, null pointers). */
int fr_render(fr_ctx *ctx, const fr_params *params, uint64_t seed, int32_t spp,
              float *out_image);

/* Adjoint of the last fr_render: given dL/dimage [H][W][3] (device), write
 * the requested gradients.  Uses the parameters, seed and spp of the last
 * render (the caller must keep its device arrays alive until this call is
 * enqueued).  Gradients are sums over samples with floating-point atomics:
 * reproducible up to summation order.  The camera-silhouette term runs on a
 * second stream and the shadow-boundary term on a third, both owned by the
 * context: each waits for an event recorded on the context's stream and the
 * context's stream waits for their ends, so the call is ordered with the
 * caller's stream like any other.  Errors: FR_ESTATE without a prior render, FR_EINVAL
 * for null dL/dimage. */
int fr_backward(fr_ctx *ctx, const float *dL_dimage, const fr_grads *grads);

/* Squared-L2 photo-consistency loss E_data (Eq. 1) and its image gradient:
 * dL_dimage = 2 (image - target), *loss_dev = sum (image - target)^2 (one
 * float, device).  Either output may be NULL.  n = H*W*3. */
int fr_loss_l2(fr_ctx *ctx, const float *image, const float *target,
               float *dL_dimage, float *loss_dev);

/* fr_loss_l2 for callers that cannot allocate device memory: code being
 * captured into a HIP graph, tight serving or fitting loops, harnesses that
 * forbid hipMalloc.  Needs no context: n elements (1 .. FR_LOSS_NOALLOC_MAX)
 * of image and target (device pointers always: the call has no context),
 * dL_dimage = 2 (image - target) and
 * *loss_dev = sum (image - target)^2 (either output may be NULL), enqueued
 * on hip_stream (a hipStream_t; NULL: the null stream) of the current
 * device.  The same kernels as fr_loss_l2, with their fp64 block partial
 * sums (one per 256 elements) in a fixed array that the library keeps on
 * each device it runs on (512 KiB, held until the process ends) instead of
 * a context's buffer: no call allocates.  Calls on one device share that
 * array, so two calls that overlap on one device (different streams, no
 * ordering between them) race and may return a wrong loss; order them.
 * Errors: FR_EINVAL (null image or target, n out of range; nothing is
 * enqueued), FR_EDEVICE; the message is fr_last_error(NULL). */
#define FR_LOSS_NOALLOC_MAX (1 << 24)
int fr_loss_l2_noalloc(void *hip_stream, const float *image, const float *target, int64_t n,
                       float *dL_dimage, float *loss_dev);

/* Auxiliary buffers of the last render, for the denoiser (fadenoise.h):
 * out [H][W][7] (device) = per pixel, the mean over its samples of the
 * first hit's albedo (RGB), unit shading normal turned toward the camera
 * (xyz) and distance from the camera; misses contribute zeros.  Needs the
 * last fr_render's hit records (a render of at most one chunk, see
 * fr_set_chunk).  Errors: FR_EINVAL (null out), FR_ESTATE (no render, or
 * its records were not kept). */
int fr_aov(fr_ctx *ctx, float *out);

/* Light regulariser of the objective, Eq. 1 (w2 E_light): E_light =
 * sum_j |l_j - m_j|^2 over the context's n lights, m_j the mean of light j's
 * three channels.  lights [n][3] (device).  grad_lights [n][3] (device,
 * may be NULL): 2 w2 (l_j - m_j) is ADDED to it, e.g. to fr_backward's
 * d_lights.  *loss_dev (device float, may be NULL) = w2 E_light.
 * Errors: FR_EINVAL (null lights, non-finite w2). */
int fr_light_reg(fr_ctx *ctx, const float *lights, float w2, float *grad_lights, float *loss_dev);

/* One Adam step (Kingma and Ba 2015) on n floats, in place, on the context's
 * stream; the paper leaves the optimiser of Eq. 1 open.  param, grad, m, v
 * [n] (device): m <- beta1 m + (1 - beta1) grad, v <- beta2 v + (1 - beta2)
 * grad^2, param <- param - lr (m / (1 - beta1^step)) / (sqrt(v / (1 -
 * beta2^step)) + eps).  m and v start at zero; step counts from 1.
 * Errors: FR_EINVAL (null array with n > 0, n < 0, step < 1, beta outside
 * [0, 1), eps <= 0, non-finite lr). */
int fr_adam(fr_ctx *ctx, float *param, const float *grad, float *m, float *v, int32_t n, int32_t step,
            float lr, float beta1, float beta2, float eps);

/* Counters and phase times of the last render/backward (synchronises). */
int fr_stats(const fr_ctx *ctx, fr_stats_t *out);

/* Message of the last error on this context ("" if none); valid until the
 * next call on the context.  With NULL: the message of this thread's last
 * failed context-free call (fr_loss_l2_noalloc), or a static string. */
const char *fr_last_error(const fr_ctx *ctx);

/* Release all device memory of the context (synchronises its stream). */
void fr_destroy(fr_ctx *ctx);

/* ---- batched evaluation ------------------------------------------------
 * Many faces at once: fr_render / fr_backward (the estimator F of the
 * Optimization paragraph and its adjoint) for several contexts together,
 * each with its own mesh, image size, light stage, parameters, seed and
 * spp, with one kernel launch per pipeline step for all of them (the
 * fitting of the paper evaluates one face per iteration; a batch serves a
 * set of subjects or the frames of a sequence).  Results equal those of
 * fr_render / fr_backward on each context: images bitwise, gradients up to
 * the summation order of their atomics.
 *
 * A batch borrows its contexts (they must outlive it and must not be used
 * on their own while a batched call is in flight); after fr_batch_render,
 * fr_backward and fr_aov on one of its contexts also follow that render.
 * All work runs on one stream: the contexts' common stream, or the one set
 * with fr_batch_set_stream (which sets it on every context too).
 *
 * Launch modes per kernel kind (kinds 0 .. fr_batch_num_kinds() - 1, named
 * by fr_batch_kind_name): FR_LAUNCH_FLAT, one block per tile, the tiles in
 * order; FR_LAUNCH_XCD, one block per tile, the tiles dealt to the eight
 * XCDs in contiguous eighths.  The shadow-boundary kind, whose blocks
 * each take a tile of samples and a group of five lights, also takes a tile
 * size (samples per block: 256 or 512).
 * fr_batch_tune picks them by measurement. */
typedef struct fr_batch fr_batch;

#define FR_LAUNCH_FLAT 0
#define FR_LAUNCH_XCD 1
typedef struct {
    int32_t mode;                    /* FR_LAUNCH_*                            */
    int32_t tile;                    /* edge_secondary, whose blocks each
                                        take a tile of samples (and five
                                        lights): 256 or 512; 0 for the
                                        others                                 */
} fr_launch;

/* n contexts (1..4096, distinct, created with FR_DEVICE_PTRS and without
 * FR_REFIT; batched calls take device pointers only).  flags:
 * FR_TIMING (per-kind times, needed by fr_batch_timing / fr_batch_tune).
 * Errors: FR_EINVAL, FR_ENOMEM.  *out is NULL on error. */
int fr_batch_create(int32_t n, fr_ctx *const *ctx, uint32_t flags, fr_batch **out);
int fr_batch_set_stream(fr_batch *batch, void *hip_stream);

/* Render every instance: params[n], seeds[n] (host), spp[n] (host, 1..4096),
 * out[n] image pointers (host array of device pointers, [H][W][3] each).
 * Instances with W*H*spp <= FR_CHUNK_MAX share one launch per kernel kind;
 * a larger one (high spp) runs its context's own fr_render after them, on
 * the same stream, and fr_batch_backward its fr_backward (chunked, records
 * recomputed), with the same results as those calls.  A new set of spp
 * values reallocates scratch and synchronises; the same set again does
 * not.  Errors: FR_EINVAL (null or out-of-range arguments, a context on
 * another stream), FR_ESTATE (new spp values during graph capture),
 * FR_ENOMEM.  A call after new spp values or a changed launch
 * (fr_batch_set_launch) first waits for the batch's enqueued work, which
 * reads the tables it rewrites. */
int fr_batch_render(fr_batch *batch, const fr_params *params, const uint64_t *seeds, const int32_t *spp,
                    float *const *out);

/* Adjoint of the last fr_batch_render: dL_dimage[n] (host array of device
 * pointers), grads[n] (as fr_backward's, each output nullable).  Errors:
 * FR_ESTATE (no batched render, or a context rendered on its own since),
 * FR_EINVAL (null arguments). */
int fr_batch_backward(fr_batch *batch, const float *const *dL_dimage, const fr_grads *grads);

int32_t fr_batch_num_kinds(void);
const char *fr_batch_kind_name(int32_t kind);   /* NULL out of range */
int fr_batch_get_launch(const fr_batch *batch, int32_t kind, fr_launch *out);
/* Errors: FR_EINVAL (kind, mode or tile out of range), FR_ESTATE (during
 * graph capture). */
int fr_batch_set_launch(fr_batch *batch, int32_t kind, const fr_launch *launch);

/* Autotuner: replays the last fr_batch_render + fr_batch_backward (same
 * inputs and outputs, which the caller keeps alive; the outputs are written
 * again with the same values up to atomics order; instances above one
 * chunk, which no batched launch holds, are left out) and picks the launches
 * by coordinate descent on the whole replay's time: each tunable kind in
 * turn tries its candidates ('trials' replays each, 1..16, median) with the
 * other kinds at their current choice and keeps the fastest.  ms_best
 * [fr_batch_num_kinds()] (host, nullable) gets each tuned kind's own time
 * in the final choice (0 for kinds not tuned).  Synchronises.  Errors:
 * FR_ESTATE (no FR_TIMING, no prior backward, during capture), FR_EINVAL. */
int fr_batch_tune(fr_batch *batch, int32_t trials, float *ms_best);

/* Times of the last batched calls (synchronises): ms_kind
 * [fr_batch_num_kinds()] (host, nullable) per kind from its first to its
 * last launch; whole render and backward.  Errors: FR_ESTATE without
 * FR_TIMING. */
int fr_batch_timing(fr_batch *batch, float *ms_kind, float *ms_render, float *ms_backward);

/* HIP graph of one iteration: between fr_batch_capture_begin and
 * fr_batch_capture_end, batched calls (and fr_loss_l2 / fr_adam /
 * fr_light_reg on the batch's contexts, which share its stream) are
 * recorded instead of run; capture_end instantiates the graph, or updates
 * the previous one in place when only arguments changed, and
 * fr_batch_graph_launch runs it.  A graph holds its calls' arguments
 * (seeds, poses, pointers) by value.  The batch must have run once with the
 * same spp values before a capture, on a stream other than the null
 * stream.  Errors: FR_ESTATE (order of calls), FR_EDEVICE. */
int fr_batch_capture_begin(fr_batch *batch);
int fr_batch_capture_end(fr_batch *batch);
int fr_batch_graph_launch(fr_batch *batch);

const char *fr_batch_last_error(const fr_batch *batch);
/* Release the batch (synchronises its stream); its contexts stay. */
void fr_batch_destroy(fr_batch *batch);

#ifdef __cplusplus
}
#endif
#endif
