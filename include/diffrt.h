/*
 * diffrt: differentiable Monte Carlo path tracer with edge sampling for
 * AMD Instinct MI355X (gfx950). C ABI.
 *
 * The operation (Li, "Differentiable Visual Computing", Ch. 5, Method): given
 * a triangle scene with continuous parameters Phi (vertex positions, per-
 * triangle albedo, camera pose), render an image by Monte Carlo path tracing
 * (eq. first, eq. gradient_monte_carlo, box pixel filter) and, given the
 * gradient of a scalar loss w.r.t. that image, return the loss gradient w.r.t.
 * Phi. The gradient is split by the product rule (eq. redner_product_rule)
 * into an interior term (reverse mode through each path sample with its
 * integration variables held fixed) and boundary terms sampled on silhouette
 * edges: on screen (eq. edge_equation, eq. mc) and from every path vertex in
 * direction space (Secondary visibility, eq. dirac_3d_edge), the latter drawn
 * from a per-view edge hierarchy (Importance Sampling the Edges).
 *
 * Conventions
 *  - Every array pointer is DEVICE memory owned by the caller, who keeps it
 *    alive until the work queued on `stream` has completed. The library owns
 *    the scene internals (BVH, edge tables, edge hierarchy, checkpoints) and
 *    frees them in drSceneDestroy.
 *  - Outputs are overwritten, not accumulated. A NULL gradient pointer skips
 *    that output.
 *  - All calls are asynchronous on `stream` unless stated; host-side argument
 *    checks fail fast with DR_ERROR_INVALID_VALUE before anything is queued.
 *    Device-side anomalies (traversal stack or tree-depth overflow) set a
 *    sticky flag read by drGetLastDeviceError.
 *  - A scene is not thread-safe; calls on one scene must be ordered.
 *  - drRenderBackward differentiates the estimator drawn by drRender with the
 *    same camera and options (seed, spp, depth): it reuses the forward pass's
 *    path checkpoints when they match and recomputes them otherwise.
 */
#ifndef DIFFRT_H
#define DIFFRT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DR_SUCCESS = 0,
    DR_ERROR_INVALID_VALUE = 1,   /* bad pointer, size, index or option */
    DR_ERROR_OUT_OF_MEMORY = 2,   /* device allocation failed */
    DR_ERROR_DEVICE = 3,          /* a HIP call failed, or a sticky device error is set */
    DR_ERROR_UNSUPPORTED = 4,     /* e.g. an edge shared by more than two triangles */
    DR_ERROR_DEGENERATE_GEOMETRY = 5  /* a triangle of zero area (no normal, never hit) */
} drStatus;

typedef struct drScene_t* drScene;

/* Scene description (thesis Ch. 5, Method: triangle meshes, no
 * interpenetration, area lights only). Arrays are device memory, read during
 * drSceneCreate only (the library copies what it needs). */
typedef struct {
    int32_t num_vertices;        /* V >= 3 */
    int32_t num_triangles;       /* 1 <= T <= 2^26 (larger: DR_ERROR_INVALID_VALUE) */
    const float*   vertices;     /* [V][3] world-space positions */
    const int32_t* indices;      /* [T][3] vertex indices, 0 <= i < V */
    const float*   normals;      /* [V][3] shading normals, or NULL for flat shading */
    const float*   albedo;       /* [T] Lambertian albedo (emitters: 0) */
    const float*   emission;     /* [T] radiance of emitters (> 0), 0 otherwise */
    int32_t emission_two_sided;  /* 0: emitters radiate along (v1-v0)x(v2-v0) only */
    float   background;          /* radiance of camera rays that hit nothing */
} drSceneDesc;

/* Pinhole look-at camera. Screen coordinates are pixels, y down; the ray
 * through screen point (x, y) has direction f + ndc_x*aspect*tan(fov/2)*r +
 * ndc_y*tan(fov/2)*u, so its parameter is camera-space depth. Geometry closer
 * than near_clip is invisible and edges are clipped there. `window` selects
 * the rendered pixels [x0,x1) x [y0,y1) of the full width x height image;
 * images passed to the calls below have the window's size. */
typedef struct {
    float position[3], look_at[3], up[3];
    float fov_y_deg;
    float near_clip;
    int32_t width, height;
    int32_t window[4];           /* x0, y0, x1, y1; all zero = full image */
} drCamera;

/* Terms of the gradient (all on by default; switches exist for tests). */
#define DR_TERM_INTERIOR  1u
#define DR_TERM_PRIMARY   2u
#define DR_TERM_SECONDARY 4u
#define DR_TERM_ALL       7u

typedef struct {
    int32_t  spp;                /* samples per pixel, >= 1 */
    int32_t  max_depth;          /* 0 = primary visibility (emission only); k = k path vertices with NEE; <= 6 */
    uint64_t seed;               /* Philox4x32-10 key */
    uint32_t view_id;            /* Philox counter word distinguishing views */
    uint32_t terms;              /* DR_TERM_* bits; 0 means DR_TERM_ALL */
    const uint8_t* unit_mask;    /* [M] device, or NULL. M = window pixels * spp; unit m
                                    = pixel sample m plus primary edge sample m; 0 = skip */
    /* Learned edge proposal (used by drRenderBackward only). edge_pdf[E]
     * (device) is a distribution over all edges, indexed by edge id: edges are
     * the unique undirected edges of the triangles, numbered in increasing
     * order of (smaller vertex index, larger vertex index). With edge_mix in
     * (0, 1) each edge sample of the terms in edge_mix_terms is drawn from
     * edge_pdf with probability edge_mix and from the plain sampler otherwise,
     * and weighted by the mixture pdf (importance sampling stays unbiased: the
     * mixture is positive wherever the plain pdf is). edge_mix = 0 or
     * edge_pdf = NULL: plain sampling. */
    const float* edge_pdf;
    float    edge_mix;
    uint32_t edge_mix_terms;     /* DR_TERM_PRIMARY | DR_TERM_SECONDARY; 0 means both */
    /* If not NULL, [E] device, overwritten: per edge, the sum over its boundary
     * samples (primary and secondary) of P * |c|^2, where P is the probability
     * with which the sample drew the edge and c its contribution to the edge's
     * two endpoints (6 numbers). Its expectation does not depend on the
     * sampler: the training target of the learned proposal. */
    float*   edge_stats;
    /* Geometry buffer in place of radiance (Ch. 5, Results: the method
     * differentiates G-buffers as well): 0 = radiance; 1, 2, 3 = world
     * position x, y, z of the camera ray's first hit; 4, 5, 6 = shading
     * normal x, y, z there, turned to face the camera ray; 7 = albedo of the
     * hit triangle; 8 = all seven at once, in which case drRender's image
     * and drRenderBackward's d_image are [7][Hw][Ww] (channel c at offset
     * (c-1)*Hw*Ww) and the gradient is that of the sum of the channels'
     * losses. A camera ray that hits nothing gives 0. The gradient is the
     * chain rule at the first hit (interior term) plus primary edge sampling
     * (boundary term); there is no secondary term and max_depth is not used.
     * Not combined with edge_pdf, edge_mix > 0 or edge_stats
     * (DR_ERROR_INVALID_VALUE); batches take 0 only. */
    int32_t  aov;
    /* Point on each secondary edge sample (drRenderBackward only; Ch. 5,
     * Importance sampling on an edge): 0 = uniform in the edge parameter t;
     * 1 = in proportion to the clamped cosine with the shading normal, in the
     * arc-length measure of the direction toward the point (closed-form
     * inverse; the Lambertian case of sampling the shading lobe along the
     * edge), weighted by its density. Other values: DR_ERROR_INVALID_VALUE. */
    int32_t  edge_t_mode;
    /* Edge chosen for each secondary edge sample (drRenderBackward only; Ch. 5,
     * Edge selection): 0 or 1 = one descent of the edge hierarchy, weighted
     * by its pdf; M in 2..16 = M samples distributed down the hierarchy, at
     * every node in proportion to the children's importance (the first child
     * receives floor(n p + xi) of the node's n samples), and one of the
     * leaves reached kept by weighted reservoir sampling with weight
     * n_e imp_e / pdf_e; the kept edge is weighted by W / (M imp) in place of
     * 1/pdf (W: total weight; unbiased because a leaf receives M pdf_e
     * samples in expectation). M > 1 needs max_depth <= 3, no proposal
     * mixture (edge_pdf with edge_mix > 0, either term), no edge_stats and no
     * geometry buffer, and is not taken by batches; otherwise, or M > 16:
     * DR_ERROR_INVALID_VALUE. */
    int32_t  edge_candidates;
    /* Next event estimation for edges (drRenderBackward only; Ch. 5, Next
     * event estimation for edges). edge_nee = alpha in [0, 1) (0: off): each
     * secondary edge sample comes with probability alpha from the strip
     * strategy and otherwise from the edge hierarchy. The strip strategy
     * draws a light point y as next-event estimation does, widens every edge
     * into a strip of width edge_nee_width that faces the shading point x,
     * and picks one of the strips the segment x -> y crosses in proportion to
     * its edge's importance; the crossing, projected onto the edge, is the
     * edge point. Every sample is weighted by the density of the mixture
     * (one-sample multiple importance sampling), so the estimate stays
     * unbiased for any alpha and width. Emitter edges and edges that are no
     * discontinuity from x are left to the hierarchy. edge_nee_width = 0:
     * the scene's default, the L2 norm over the coordinates of 2% of the
     * mean absolute deviation of the vertex positions (computed at
     * drSceneCreate / drSceneUpdateVertices; drSceneRefit keeps it).
     * alpha > 0 needs edge_t_mode 0, edge_candidates <= 1, no proposal
     * mixture (edge_pdf with edge_mix > 0, either term), no edge_stats and
     * no geometry buffer, and is not taken by batches; otherwise, alpha
     * outside [0, 1) or a negative or non-finite width:
     * DR_ERROR_INVALID_VALUE. */
    float    edge_nee;
    float    edge_nee_width;
} drRenderOptions;

/* Creates a scene: validates sizes and indices (host copy of the topology),
 * extracts unique edges (sorted by (min vertex, max vertex)), builds the
 * triangle BVH (binned-SAH topology on the host, boxes on the device; with
 * the environment variable DIFFRT_BVH=lbvh a Morton-code LBVH built on the
 * device). Non-finite vertex coordinates are rejected with
 * DR_ERROR_INVALID_VALUE, a triangle whose two edge vectors have an FP32
 * cross product of exactly zero with DR_ERROR_DEGENERATE_GEOMETRY.
 * Synchronises `stream`. */
drStatus drSceneCreate(drScene* out, const drSceneDesc* desc, hipStream_t stream);

/* Replaces all vertex positions ([V][3] device) and rebuilds the BVH as
 * drSceneCreate does (synchronises `stream`; for optimisation loops that must
 * not synchronise, drSceneRefit keeps the topology). On
 * DR_ERROR_INVALID_VALUE (non-finite coordinates) the scene may only be
 * updated again or destroyed. */
drStatus drSceneUpdateVertices(drScene scene, const float* vertices, hipStream_t stream);

/* Replaces all triangle albedos ([T] device, in [0, 1]) for material
 * fitting (Ch. 5, Results: inverse rendering of material parameters);
 * refreshes the edge kinds, which depend on the albedos of an edge's two
 * faces. Kernel launches only (no synchronisation). The values are not
 * checked. */
drStatus drSceneUpdateAlbedo(drScene scene, const float* albedo, hipStream_t stream);

/* Host query of the scene's sizes. */
drStatus drSceneGetInfo(drScene scene, int32_t* num_vertices, int32_t* num_triangles, int32_t* num_edges);

/* Forward pass: image[Hw][Ww] (window size), mean radiance per pixel. Stores
 * the path checkpoints drRenderBackward reuses. */
drStatus drRender(drScene scene, const drCamera* camera, const drRenderOptions* options,
                  float* image, hipStream_t stream);

/* Backward pass for the loss gradient d_image[Hw][Ww]: writes
 * d_vertices[V][3], d_albedo[T], d_camera[9] (position, look_at, up). */
drStatus drRenderBackward(drScene scene, const drCamera* camera, const drRenderOptions* options,
                          const float* d_image, float* d_vertices, float* d_albedo, float* d_camera,
                          hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batches of views and capturable optimisation steps. The thesis renders
 * several views of one scene inside an optimisation loop (Ch. 5, Results:
 * inverse rendering with Adam); a batch renders and differentiates many
 * views with their own image sizes and sample counts in one kernel launch
 * per pass, and its refit path (drSceneRefit + drBatchRefit) refreshes all
 * geometry-dependent data with kernel launches only (no host
 * synchronisation, no allocation), so update -> refit -> render -> loss ->
 * backward -> Adam can be captured once in a HIP graph and replayed.
 * ------------------------------------------------------------------------- */
typedef struct drBatch_t* drBatch;

/* Vertex update for optimisation loops: new positions ([V][3] device),
 * triangle records, edge kinds, light sampling tables and BVH bounds over the
 * existing BVH topology (the scene's scale constants, used for ray offsets,
 * keep their creation values). Kernel launches only: capturable. */
drStatus drSceneRefit(drScene scene, const float* vertices, hipStream_t stream);

/* Creates a batch of n views of `scene` (which must outlive it): cameras[n]
 * and options[n] (host arrays, copied; all views share max_depth; edge_pdf
 * and edge_stats must be NULL and edge_mix 0; a view's unit_mask, if given,
 * is read by every later pass and must stay alive with the batch), images[n] and
 * d_images[n] (host arrays of device pointers, each [H][W] of its view's
 * window, owned by the caller and used by every later call). Builds each
 * view's primary edge table and edge hierarchy; synchronises `stream`. */
drStatus drBatchCreate(drBatch* out, drScene scene, int32_t n, const drCamera* cameras,
                       const drRenderOptions* options, float* const* images, const float* const* d_images,
                       hipStream_t stream);

/* Per-view tables from the scene's current vertices (after drSceneRefit),
 * keeping each hierarchy's topology. Capturable. Which edges are
 * discontinuities, and which hierarchy holds them, can change when vertices
 * move (coplanar faces folding into a crease, a smooth edge becoming a
 * silhouette from the camera); the refit then raises a device flag of the
 * batch, which drBatchCheckHierarchy reads. */
drStatus drBatchRefit(drBatch batch, hipStream_t stream);

/* Reads the flag drBatchRefit raises (synchronises `stream`). If it is set,
 * rebuilds every view's primary edge table and edge hierarchies from the
 * scene's current vertices, clears the flag and sets *rebuilt = 1, else
 * *rebuilt = 0. Call it after drBatchRefit and before the next
 * drBatchBackward: a backward pass over a flagged batch misses boundary
 * terms. Not capturable; a HIP graph captured before a rebuild must be
 * captured again (its refit launches carry the old hierarchy sizes). Device
 * addresses held by the batch do not change. */
drStatus drBatchCheckHierarchy(drBatch batch, int32_t* rebuilt, hipStream_t stream);

/* Adds 1 to every view's Philox key (new random numbers for the next
 * forward/backward pair). Capturable. */
drStatus drBatchAdvanceSeed(drBatch batch, hipStream_t stream);

/* Renders every view into its image (one launch for all views). Capturable. */
drStatus drBatchForward(drBatch batch, hipStream_t stream);

/* Gradients of sum over views of <d_image_v, image_v>: d_vertices[V][3] and
 * d_albedo[T] (summed over views; NULL = not wanted), d_cameras[n][9] or
 * NULL. Reads each view's d_image buffer. Needs the forward pass of the same
 * seed. Capturable. */
drStatus drBatchBackward(drBatch batch, float* d_vertices, float* d_albedo, float* d_cameras, hipStream_t stream);

/* Launch shape (autotuning): ctas = 0 launches one workgroup per work item;
 * ctas > 0 launches at most ctas persistent workgroups that take work items
 * from an atomic counter. chunk = 64-unit blocks per work item (1..64). */
drStatus drBatchSetLaunch(drBatch batch, int32_t ctas, int32_t chunk);

drStatus drBatchDestroy(drBatch batch);

/* One Adam step (Kingma and Ba, with bias correction) on n FP32 parameters,
 * all device arrays of length n: x -= lr * mhat / (sqrt(vhat) + eps), with
 * m, v updated in place; `step` counts from 1. Used by inverse-rendering
 * loops (the thesis optimises with Adam, Ch. 5 Results). */
drStatus drAdamStep(float* x, const float* g, float* m, float* v, int64_t n, float lr, float beta1,
                    float beta2, float eps, int64_t step, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Learned edge proposal. The thesis samples edges by importance with a
 * hand-built pdf (Ch. 5, Importance Sampling the Edges) and names what such a
 * pdf should follow; these entry points train and evaluate a small network
 * that proposes a per-view distribution over edges from per-(edge, view)
 * features, for the mixture in drRenderOptions.
 *
 * Network: 32 inputs -> 64 (ReLU) -> 64 (ReLU) -> 1 logit. Parameters theta
 * are DR_MLP_PARAMS FP32 numbers (device), row-major:
 *   W1 [32][64] | b1 [64] | W2 [64][64] | b2 [64] | W3 [64] | b3 [1].
 * Inputs and weight matrices are rounded to BF16 for the matrix cores;
 * activations, gradients, biases and logits are FP32 (FP32 accumulation).
 * All arrays are device memory owned by the caller; errors: NULL pointers or
 * negative sizes give DR_ERROR_INVALID_VALUE; launch failures DR_ERROR_DEVICE.
 * ------------------------------------------------------------------------- */
#define DR_MLP_PARAMS 6337
#define DR_EDGE_FEATURES 32

/* features[E][32] of every edge seen from `camera`: endpoints and face
 * normals in the camera frame, endpoints in world space, albedo and emission
 * of both faces, boundary flag, cosine between the face normals, normalised
 * screen coordinates of the endpoints (depth clamped to the near plane,
 * clamped to +-8), edge length, zero padding. */
drStatus drEdgeFeatures(drScene scene, const drCamera* camera, float* features, hipStream_t stream);

/* logits[n] of the rows x[n][32]. */
drStatus drMlpForward(const float* theta, const float* x, int32_t n, float* logits, hipStream_t stream);

/* Per view v (rows offsets[v] .. offsets[v+1]-1; offsets[n_views+1] int32,
 * device): prob = softmax(logits) (if prob != NULL); if target != NULL, with
 * t = target / sum(target) over the view: view_loss[v] = -sum t log prob
 * (0 for views whose target sums to 0) and d_logits = (prob - t) / (number of
 * views whose target sum is positive), the gradient of the mean loss.
 * scratch: n_views floats. */
drStatus drMlpSoftmaxXent(const float* logits, const float* target, const int32_t* offsets, int32_t n_views,
                          float* prob, float* d_logits, float* view_loss, float* scratch, hipStream_t stream);

/* grad[DR_MLP_PARAMS] (overwritten) = gradient of sum_i d_logits[i] * logits[i]
 * w.r.t. theta (BF16 rounding passes gradients through unchanged). */
drStatus drMlpBackward(const float* theta, const float* x, int32_t n, const float* d_logits, float* grad,
                       hipStream_t stream);

/* drMlpSoftmaxXent without the caller's scratch argument and without any
 * device allocation, for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc). The per-view
 * target sums live in a fixed device array of DR_XENT_MAX_VIEWS floats
 * (256 KiB) that the library holds on each GPU it runs on until the process
 * ends; the stream must belong to the current device. Arguments and results
 * are those of drMlpSoftmaxXent. Errors: n_views > DR_XENT_MAX_VIEWS (or any
 * argument drMlpSoftmaxXent rejects) gives DR_ERROR_INVALID_VALUE; failing to
 * resolve the array's device address gives DR_ERROR_DEVICE. All calls on one
 * GPU share the array: calls whose work overlaps on that GPU (different
 * streams, no ordering) race and give undefined results. */
#define DR_XENT_MAX_VIEWS 65536
drStatus drMlpSoftmaxXentNoAlloc(const float* logits, const float* target, const int32_t* offsets, int32_t n_views,
                                 float* prob, float* d_logits, float* view_loss, hipStream_t stream);

/* drAdamStep with the step count in device memory (*step = steps taken so
 * far, int64, incremented by this call): for optimisation steps captured in a
 * HIP graph, whose launch arguments are fixed at capture. */
drStatus drAdamStepCounted(float* x, const float* g, float* m, float* v, int64_t n, float lr, float beta1,
                           float beta2, float eps, int64_t* step, hipStream_t stream);

/* Measurement support (not needed for rendering). With `events` on, every
 * forward, primary-edge and path-backward kernel launch is bracketed by HIP
 * events on the stream it runs on; with `counters` on, the kernels also count
 * their memory work (BVH node and triangle fetches, edge-tree node fetches,
 * gradient atomics, rays). Counting adds an atomic per lane and launch. */
typedef struct {
    double forward_ms, primary_ms, backward_ms;              /* summed kernel durations */
    int64_t forward_launches, primary_launches, backward_launches;
    /* per kernel (0 forward, 1 primary edges, 2 path backward): BVH node
     * fetches, triangle fetches, edge-tree node fetches, gradient atomics, rays */
    int64_t counts[3][5];
    /* internal nodes on the longest root-to-leaf path of the triangle BVH
     * (it bounds a traversal's stack) and of the current view's edge
     * hierarchy (-1 before the first backward pass) */
    int32_t bvh_depth, edge_tree_depth;
} drProfile;

drStatus drSetProfiling(drScene scene, int32_t events, int32_t counters);

/* Synchronises, returns the sums since the last reset, and optionally resets. */
drStatus drGetProfile(drScene scene, drProfile* out, int32_t reset);

/* Synchronises the scene's last stream and returns DR_ERROR_DEVICE if a
 * device-side anomaly was recorded (then clears it). */
drStatus drGetLastDeviceError(drScene scene);

drStatus drSceneDestroy(drScene scene);

const char* drGetErrorString(drStatus status);

#ifdef __cplusplus
}
#endif
#endif
