/*
 * handrt — differentiable Monte Carlo ray tracing of a skinned hand into many
 * calibrated views, for render-and-compare refinement (Karvounas et al.,
 * "Multiview Image-based Hand Geometry Refinement using Differentiable Monte
 * Carlo Ray Tracing", BMVC 2021).  C ABI over hand-written HIP kernels for
 * gfx950 (MI355X).
 *
 * The calls follow the paper's problem statement (Section 3): given calibrated
 * views {O_i, C_i} and hand parameters h, an iteration is
 *   hr_skin     h -> mesh vertices (the decoders G_v, G_J, Section 3.1)
 *   hr_render   vertices, colour map, cameras -> images R(G_v(h), V, C_i)
 *               (Monte Carlo pixel integrals, Section 3 "Method" and Eq. 3)
 *   hr_loss     E1 = sum_i mean |O_i - R_i| and dE1/dR (Eq. 3 and D_c of Eq. 4)
 *   hr_backward dE1/dh and dE1/d(colour map): derivative of the estimate at
 *               fixed samples plus the silhouette-edge (visibility) term
 *               sampled along edges (Section 4.2.2)
 *   hr_step     one Adam step (Section 3.3)
 *
 * Conventions shared by every call
 *  - Pointers named *_host are host memory; every other array pointer is
 *    device memory owned by the caller, contiguous, float32 unless stated.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls only enqueue
 *    work on `stream` and return; results are valid once the stream reaches
 *    them.  No call synchronises the stream or allocates device memory, except
 *    hr_scene_create (allocates the scene's buffers) and hr_scene_destroy.
 *  - A scene's internal buffers (normals, acceleration structure, edge tables,
 *    gradient accumulators) are shared by all calls on that scene: calls on
 *    one scene must be ordered (one stream, or explicit events).
 *  - Return value: HR_OK (0) or a negative HR_E* code; the message of the last
 *    error on the calling thread is in hr_last_error().  On error nothing has
 *    been enqueued unless the code is HR_EHIP (a HIP launch/runtime failure).
 *
 * Packed-view layout: views are numbered 0..n_views-1; view v has W_v x H_v
 * pixels stored row-major starting at pixel offset pix_off[v] = sum_{u<v} W_u H_u.
 * Images are [n_pixels, 3] float32 (RGB), masks [n_pixels] uint8.
 *
 * Parameter block of one hand (64 float32): [0:48] axis-angle rotations of the
 * 16 joints (joint 0 is the root), [48:58] shape coefficients, [58:61] global
 * rotation (axis-angle), [61:64] global translation (metres).
 */
#ifndef HANDRT_H
#define HANDRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HR_OK 0
#define HR_EINVAL (-1)       /* null pointer, bad count or option */
#define HR_ESHAPE (-2)       /* sizes inconsistent with the scene */
#define HR_EHIP (-4)         /* HIP runtime / launch failure */
#define HR_EUNSUPPORTED (-5) /* outside the supported range (see the call) */

/* backward flags */
#define HR_GRAD_INTERIOR 1u     /* derivative of the estimate at fixed samples */
#define HR_GRAD_EDGES 2u        /* silhouette-edge (visibility) term */
#define HR_GRAD_ALL 3u
#define HR_REUSE_GEOMETRY 4u    /* normals/BVH already prepared from `verts`
                                   by the previous hr_render on this scene */
#define HR_SKIP_PRIOR 8u        /* leave the joint prior's gradient out even when
                                   hr_set_joint_prior has set one (gradient of
                                   the data term alone) */

typedef struct hr_scene hr_scene;
typedef struct hr_graph hr_graph;

/* Hand model and mesh topology, HOST pointers, copied by hr_scene_create.
   Sizes: V vertices, F triangles, J joints (parents[j] < j, parents[0] = -1),
   K shape directions, E edges.  faces are wound counter-clockwise seen from
   outside; edges[e] = (a,b) appears as a->b in face edge_faces[e][0] and as
   b->a in edge_faces[e][1] (-1 for a boundary edge). */
typedef struct {
    int32_t n_verts, n_faces, n_joints, n_shape, n_edges;
    const float* v_template;   /* [V,3] rest-pose vertices (metres) */
    const float* shapedirs;    /* [V,3,K] shape displacement per coefficient */
    const float* j_regressor;  /* [J,V] joint = sum_v J[j,v] shaped vertex */
    const float* weights;      /* [V,J] skinning weights, rows sum to 1 */
    const int32_t* parents;    /* [J] */
    const int32_t* faces;      /* [F,3] */
    const float* uv;           /* [V,2] texture coordinates in [0,1] */
    const int32_t* edges;      /* [E,2] */
    const int32_t* edge_faces; /* [E,2] */
} hr_mesh_desc;

/* Pinhole camera: a world point x maps to camera coordinates R (x - o)
   (R row-major, rows = right, down, forward) and to pixel coordinates
   (fx X/Z + cx, fy Y/Z + cy); pixel (i,j) covers [j,j+1) x [i,i+1). */
typedef struct {
    float R[9];
    float o[3];
    float fx, fy, cx, cy;
    int32_t W, H;
    int32_t hand;   /* which hand of the batch this view observes */
} hr_camera;

/* Estimator configuration (fixed for a scene). */
typedef struct {
    float ka, kd;        /* colour = albedo(uv) * (ka + kd max(0, n.l)) */
    float light[3];      /* unit direction towards the light, world frame */
    int32_t spp;         /* camera samples per pixel, 1..256 */
    float edge_delta;    /* side-ray offset of an edge sample, pixels (> 0) */
    int32_t tex_h, tex_w;/* colour map size (texels) */
    uint64_t seed;       /* Philox key of all sample streams */
    uint32_t view_base;  /* sample-stream id of view 0; view v draws the streams
                            of id view_base + v, so a scene holding views
                            k..k+n-1 of a larger set (with view_base = k)
                            reproduces their samples exactly */
} hr_config;

/* Adam hyper-parameters.  Learning rates per parameter group; 0 freezes a
   group (its parameters and moments are left untouched). */
typedef struct {
    float lr_pose_root;  /* params [0:3]   */
    float lr_pose;       /* params [3:48]  */
    float lr_shape;      /* params [48:58] */
    float lr_rot;        /* params [58:61] */
    float lr_trans;      /* params [61:64] */
    float lr_albedo;     /* colour map; clamped to [0,1] after the step */
    float beta1, beta2, eps;
} hr_adam_config;

/* Create a scene for n_hands hands of the same model seen by n_views cameras
   (cams_host[v].hand in [0,n_hands)).  Allocates device buffers on the current
   HIP device; the scene may only be used on that device.
   HR_EUNSUPPORTED: V > 4096, F > 8192, J > 32, K > 16, a view larger than
   4096 x 4096, spp outside 1..256. */
int hr_scene_create(hr_scene** out, const hr_mesh_desc* mesh_host, int32_t n_hands,
                    const hr_camera* cams_host, int32_t n_views, const hr_config* cfg);
void hr_scene_destroy(hr_scene* scene);

/* Number of pixels over all views (length of packed image buffers). */
int64_t hr_num_pixels(const hr_scene* scene);

/* Skinning (Section 3.1 "Geometry"): shape blend, joint regression, Rodrigues
   rotations, forward kinematics along the joint tree, linear blend of joint
   transforms, global rotation and translation.
   params [n_hands,64] -> verts [n_hands,V,3], joints [n_hands,J,3] (nullable). */
int hr_skin(hr_scene* scene, const float* params, float* verts, float* joints, void* stream);

/* Rebuild the topology of each hand's bounding-volume hierarchy (binned
   surface-area heuristic) around the given vertices [n_hands,V,3].  Bounds
   are refit every iteration by hr_render; the topology only affects speed,
   never results.  Call it once the pose is roughly known (e.g. after the
   first hr_skin).  Synchronises `stream`; host-side work, not for use under
   graph capture.  The scene starts with a hierarchy of the rest pose. */
int hr_build_hierarchy(hr_scene* scene, const float* verts, void* stream);

/* Quality of each hand's hierarchy as last refit (by hr_render, hr_iterate
   or any call that prepares the geometry), so that a caller can decide when
   to call hr_build_hierarchy again: the sum over the internal nodes of their
   two child boxes' surface areas divided by the root box's surface area
   (the expected number of child-box tests of a ray crossing the root box, the
   measure the surface-area heuristic minimises).  It grows as the pose
   drifts from the one the topology was built around; 0 before the first
   refit.  cost_host [n_hands] float, host memory, written.  Synchronises the
   device; not for use under graph capture. */
int hr_hierarchy_cost(hr_scene* scene, float* cost_host);

/* Render all views: pixel = (1/spp) sum over samples of the colour of the
   first surface hit by the ray through a uniformly drawn point of the pixel,
   or the pixel's background colour (Section 3, Eq. 3).  Also prepares the
   scene's per-iteration geometry (vertex normals, acceleration structure,
   per-view screen bounds) from `verts`.
   verts [n_hands,V,3]; albedo [n_hands,tex_h,tex_w,3]; background [P,3];
   iter selects the sample streams; image [P,3] out;
   hit_face [P,spp] int32 out (nullable): first-hit triangle of every sample,
   -1 for a miss. */
int hr_render(hr_scene* scene, const float* verts, const float* albedo, const float* background,
              uint32_t iter, float* image, int32_t* hit_face, void* stream);

/* While enabled (default off), hr_render also traces the edge samples' side
   rays of its iteration (Section 4.2.2; they depend on the geometry only),
   in the same launch, and a following hr_backward with HR_REUSE_GEOMETRY at
   the same iter weighs them instead of tracing them again.  Worth it when
   the backward follows each render (a loop with its own loss, such as the
   full data term); hr_iterate does the same by itself. */
int hr_set_render_edges(hr_scene* scene, int32_t enable);

/* Photometric loss, per hand: E1 = sum over the hand's views of the mean of
   |image - target| over the view's masked pixels and the 3 channels
   (Eq. 3 with D_c of Eq. 4); dimage = dE1/dimage = sign(image - target) /
   (3 * masked pixel count of the view) on masked pixels, 0 elsewhere.
   mask [P] uint8 (nullable = all pixels); loss [n_hands] out; dimage [P,3] out. */
int hr_loss(hr_scene* scene, const float* image, const float* target, const uint8_t* mask,
            float* loss, float* dimage, void* stream);

/* hr_loss for callers that cannot allocate device memory (code under HIP
   graph capture, tight serving loops, harnesses that forbid hipMalloc): the
   same outputs as hr_loss (bit for bit), with its scratch (the chunk partial
   sums and the views' loss scales) in a fixed array of the library instead
   of the scene's buffers.  Allocates nothing and calls no allocating routine;
   the array (64 KiB, 16384 floats, one copy per device, held until the
   process ends) is looked up by hr_scene_create.  Limit: 2 * chunks + views
   <= 16384 floats, chunks = sum over views of ceil(W*H / 4096) (about 33 M
   pixels in total); larger scenes get HR_EUNSUPPORTED and nothing is
   enqueued.  Every call on a device shares that device's array, which keeps
   the last call's values: calls that overlap on one device (concurrent
   streams, other host threads) race and must be ordered by the caller.
   Arguments and errors as hr_loss. */
int hr_loss_noalloc(hr_scene* scene, const float* image, const float* target, const uint8_t* mask,
                    float* loss, float* dimage, void* stream);

/* Gradient of L = sum_p dimage[p] . image[p] (with the samples of hr_render
   at the same iter) with respect to the hand parameters and the colour map.
   flags: HR_GRAD_* terms to include, plus HR_REUSE_GEOMETRY and HR_SKIP_PRIOR.
   With a joint prior set (hr_set_joint_prior) and without HR_SKIP_PRIOR,
   grad_params also holds lambda dE2/dparams.
   grad_params [n_hands,64] out; grad_albedo [n_hands,tex_h,tex_w,3] out;
   grad_verts [n_hands,V,3] out (nullable): dL/dvertex before skinning
   backward, all terms; grad_normals [n_hands,V,3] out (nullable): dL/d(unit
   vertex normal) of the interior term.  Outputs are overwritten. */
int hr_backward(hr_scene* scene, const float* params, const float* verts, const float* albedo,
                const float* background, const float* dimage, uint32_t iter, uint32_t flags,
                float* grad_params, float* grad_albedo, float* grad_verts, float* grad_normals,
                void* stream);

/* Camera coverage (Section 4.2.3, camera coverage; Eq. 6).  hr_face_visibility:
   visible [n_views,F] int32 out (DEVICE): 1 where some camera sample of the
   view hit the face, from hit_face [pixels,spp] as hr_render writes it (the
   coverage of a view is the set of triangles its samples see), else 0.
   hr_camera_order: per hand, its views in greedy order, each next view the
   one adding the most faces not seen by those before it (ties: the earlier
   view of the hand in the camera list), so the coverage of the first i views
   never decreases with i.  order [n_views] int32 out (DEVICE): view indices
   in hand segments (hand 0's views first, then hand 1's, ...; position k of
   a segment is step k); covered [n_views] int32 out (DEVICE), same layout:
   faces seen by the hand's first k + 1 views.  HR_EINVAL: null argument;
   HR_EUNSUPPORTED: a face bitmap (ceil(F / 32) words) or, for the order, the
   bitmaps of one hand's views (views x ceil(F / 32) words + 2 per view)
   beyond 64 KiB. */
int hr_face_visibility(hr_scene* scene, const int32_t* hit_face, int32_t* visible, void* stream);
int hr_camera_order(hr_scene* scene, const int32_t* visible, int32_t* order, int32_t* covered, void* stream);

/* Joint prior of the objective E = E1 + lambda E2 (Section 3.2, Eq. 5): E2 sums,
   over the hands' joints and their three coordinates, the smooth L1
   distance f2(d) = d^2 / (2 gamma) for |d| < gamma, |d| - gamma / 2
   otherwise, between the posed joints (those hr_skin returns) and
   target_joints (DEVICE [n_hands,J,3] float32, caller-owned, read by every
   later backward until the next call, and by every launch of a graph
   captured meanwhile: it must stay valid that long).
   gamma is in the model's units (the paper's 5 mm is 0.005 for a model in
   metres).  From the next enqueued call on, hr_backward, hr_iterate and
   graphs created afterwards (a graph keeps the setting it was captured
   with) add lambda dE2/dparams to grad_params, and the
   loss that hr_iterate writes becomes E1 + lambda E2 per hand (hr_loss stays
   E1).  target_joints NULL or lambda 0 switches the prior off.
   HR_EINVAL: null scene, lambda < 0, gamma <= 0 or either not finite. */
int hr_set_joint_prior(hr_scene* scene, const float* target_joints, float lambda, float gamma);

/* One Adam step (t >= 1 counts steps) on params [n_hands,64] and albedo
   [n_hands,tex_h,tex_w,3] in place, with moments m_*, v_* (same shapes,
   caller-owned, zero before the first step). */
int hr_step(hr_scene* scene, float* params, float* albedo, const float* grad_params,
            const float* grad_albedo, float* m_params, float* v_params, float* m_albedo,
            float* v_albedo, int32_t t, const hr_adam_config* cfg, void* stream);

/* Buffers of a refinement loop, all DEVICE pointers owned by the caller
   (shapes as in the calls above; P = hr_num_pixels). */
typedef struct {
    float* params;            /* [n_hands,64] updated in place */
    float* albedo;            /* [n_hands,tex_h,tex_w,3] updated in place */
    float* m_params;          /* Adam moments, zero before the first step */
    float* v_params;
    float* m_albedo;
    float* v_albedo;
    const float* background;  /* [P,3] */
    const float* target;      /* [P,3] observed images */
    const uint8_t* mask;      /* [P] nullable = all pixels */
    float* verts;             /* [n_hands,V,3] out: vertices of the iteration */
    float* image;             /* [P,3] out: rendered images */
    float* dimage;            /* [P,3] out: dE1/dimage */
    float* loss;              /* [n_hands] out: the objective of the iteration (before its
                                 step): E1, or E1 + lambda E2 while a joint prior is set */
    float* grad_params;       /* [n_hands,64] out */
    float* grad_albedo;       /* [n_hands,tex_h,tex_w,3] out */
    int32_t* iter;            /* [1] int32 iteration index, read when the work
                                 runs and incremented by one at its end */
} hr_state;

/* One whole refinement iteration (Section 3.3): hr_skin, hr_render, hr_loss,
   hr_backward (terms in `flags`, HR_GRAD_*) and hr_step, with the iteration
   index i = *state->iter taken from device memory: samples of iteration i and
   Adam step count t = i + 1.  Equivalent to the five calls with iter = i,
   t = i + 1, followed by ++*state->iter.  Enqueues kernels only (no host
   synchronisation, no allocation), so it can be captured into a graph. */
int hr_iterate(hr_scene* scene, const hr_state* state, const hr_adam_config* cfg, uint32_t flags, void* stream);

/* A HIP graph of n_iters (1..1024) consecutive hr_iterate calls on `state`'s
   buffers (the pointers and cfg are fixed at creation; buffer contents are
   read when the graph runs).  hr_graph_launch enqueues it on `stream`; each
   launch advances *state->iter by n_iters.  The graph uses the scene's internal
   buffers: launches must be ordered with every other call on the scene.
   hr_graph_create captures on an internal stream and runs nothing. */
int hr_graph_create(hr_graph** out, hr_scene* scene, const hr_state* state, const hr_adam_config* cfg,
                    uint32_t flags, int32_t n_iters);
int hr_graph_launch(hr_graph* graph, void* stream);
void hr_graph_destroy(hr_graph* graph);

/* Launch tuning.  The render and interior-adjoint launches are persistent
   grids that walk the wave-tile list; their block counts change speed only:
   images are identical for any choice (each pixel sums its samples in a fixed
   order), gradients agree up to the order of floating-point atomic sums.
   Scenes whose views hold at most one wave tile per SIMD of the device (4
   per compute unit) render, with a grid of two blocks or more, with the
   four waves of a block sharing each tile (each walks a quarter of the
   tile's screen-bin list) and smaller edge-sample packets: the same images
   and hits, fewer idle SIMDs.  hr_set_grid sets them (0 keeps a value; values are capped at one block per
   four wave tiles of the views), hr_get_grid reads them.  hr_tune times
   candidates on `state`'s buffers (it runs skin, render, loss and the
   interior adjoint `reps` times per candidate, overwriting verts, image,
   dimage, loss and the gradient outputs, never params, albedo, moments or
   iter): first every wave-tile shape and screen-bin size (hr_set_tiles),
   then the render grid, then the adjoint grid; it keeps the fastest of each
   and writes (render blocks, adjoint blocks) to blocks_host (HOST,
   nullable).  Synchronises the device; not for use under graph capture.
   Graphs created before a change keep the grids they were captured with. */
int hr_set_grid(hr_scene* scene, int32_t render_blocks, int32_t adjoint_blocks);

/* Acceleration of the camera rays (speed only: hits and images are identical
   either way).  HR_ACCEL_AUTO (default): per-view screen bins (16 x 16
   pixels unless hr_set_tiles or hr_tune chose 8 or 32) list the triangles whose padded screen bounds touch them (camera
   rays all start at the camera centre), with the bounding-volume hierarchy
   for views where binning does not apply (a vertex within 1 mm of the camera
   plane, more than 8192 bins, more than 16 F entries) and for the edge
   samples' side rays; HR_ACCEL_HIERARCHY: the hierarchy for every ray.  Takes
   effect with the next preparation (hr_render, hr_backward without
   HR_REUSE_GEOMETRY, hr_iterate); graphs keep the mode they were captured
   with.  HR_EINVAL: unknown mode. */
#define HR_ACCEL_AUTO 0
#define HR_ACCEL_HIERARCHY 1
int hr_set_accel(hr_scene* scene, int32_t mode);
int hr_get_grid(const hr_scene* scene, int32_t* blocks_host);   /* (render, adjoint) */

/* Work layout of the camera samples (speed only: the samples, each pixel's
   sum and so the images are bit-identical for every choice).  A wave takes
   all samples of 2^spp_log2 lanes per pixel for a tile of 2^a x 2^b pixels,
   a + b = 6 - spp_log2 (spp_log2 = ceil(log2 spp), at most 6); screen bins
   are 2^bin_log2 pixels square, 3 <= bin_log2 <= 5, and a tile lies inside
   one bin (a, b <= bin_log2).  hr_set_tiles(scene, a, bin_log2) synchronises
   the device, rewrites the views' bin layout and drops the render's stored
   samples (a following hr_backward with HR_REUSE_GEOMETRY prepares and
   traces again);
   graphs captured before a change must be captured again.  hr_get_tiles
   writes (a, b, bin_log2) to out_host (HOST, 3 ints).  HR_EINVAL: a shape or
   bin size outside these rules. */
int hr_set_tiles(hr_scene* scene, int32_t tile_w_log2, int32_t bin_log2);

/* Renderer of the camera samples.  HR_RENDERER_RAY (default): the Monte Carlo
   ray tracer above.  HR_RENDERER_RASTER: hard rasterisation, the comparison
   renderer of Section 4.2.2 ("Ray tracing vs rasterization"): each pixel
   takes the colour of the nearest triangle covering its centre (edge
   functions of the projected vertices, either orientation, all >= 0 or all
   <= 0 with a non-zero sum; nearest = the largest perspective-correct 1/z
   rounded to float32, ties to the smaller triangle index; triangles with a
   vertex less than 1 mm in front of the camera are dropped; float64
   projection, edge functions and 1/z), or its background; the shading is
   the ray tracer's at the pixel centre.  Its gradient flows through the
   covering triangles' interpolation only: hr_backward and hr_iterate ignore
   HR_GRAD_EDGES (coverage is piecewise constant), and hr_backward without
   HR_REUSE_GEOMETRY renders the covering triangles first (into a scratch
   image of the scene).  hit_face of hr_render holds each pixel's covering
   triangle.  The raster mode needs a scene of spp = 1 (HR_EUNSUPPORTED
   otherwise); the first switch to it allocates the scratch image.
   Synchronises the device; graphs keep the renderer they were captured
   with.  HR_EINVAL: unknown mode. */
/* Edge-sample budget (Section 4.2.2): each view draws ceil(T / units)
   samples, T its total quantised silhouette length in 1/256 pixel; the
   default units = 256 draws one sample per pixel of silhouette.  Every
   budget gives an unbiased estimate (stratified samples, each weighted by
   its stratum); fewer samples, more variance.  Takes effect with the next
   preparation; graphs keep the budget they were captured with.  HR_EINVAL:
   units outside 1 .. 2^20. */
int hr_set_edge_budget(hr_scene* scene, int32_t units_per_sample);

#define HR_RENDERER_RAY 0
#define HR_RENDERER_RASTER 1
int hr_set_renderer(hr_scene* scene, int32_t mode);
int hr_get_tiles(const hr_scene* scene, int32_t* out_host);
int hr_tune(hr_scene* scene, const hr_state* state, int32_t reps, int32_t* blocks_host, void* stream);

/* ---- learned edge-sampling proposal (project addition) -----------------
   The silhouette term (Section 4.2.2) samples edges in proportion to their
   clipped screen length.  With a learned proposal, a network
   16 -> 64 -> 64 -> 1 (erf-GELU; bfloat16 operands on the matrix cores,
   float32 accumulation) maps features of each (view, silhouette edge) to a
   logit z_e, and the edge CDF uses the integer weights
     W_e = max(1, floor(w_e (1 + (1 - eps)(E_e / Ebar - 1))))
   with w_e the length weight, E_e = exp(z_e - max z), Ebar = sum w E / sum w:
   equal logits keep the length weights exactly, and every edge keeps at
   least eps of its length-proportional share.  The sample budget per view is
   unchanged and each sample is divided by its own probability, so the
   estimate stays unbiased for any network.  hr_backward draws with these
   weights and records, per (view, edge), the sum of |sample contribution| and
   of |c- - c+| per channel; hr_proposal_train (also run by hr_iterate) takes
   one Adam step on KL(target || q), target = the recorded |contribution|
   sums normalised per view, q_e = w_e exp(z_e) / sum_f w_f exp(z_f), updates
   the per-edge colour-jump averages (features 7-9) and clears the records.

   Features of a row (view v, edge e), in order: the clipped projected
   endpoints over (W, H) (4), the clipped length over the image diagonal, the
   larger and the smaller of n_f . vhat over the edge's faces (unit face
   normals; vhat the unit direction from the edge midpoint to the camera; 0
   for a missing face), the colour jump across the edge (3: the running
   average of measured |c- - c+|, or before any measurement |shade -
   background| at the edge midpoint), 6 zeros.

   Parameter vector (HR_MLP_PARAMS float32): W1 [16][64] (input-major), b1 [64],
   W2 [64][64], b2 [64], w3 [64], b3. */
#define HR_PROPOSAL_LENGTH 0
#define HR_PROPOSAL_LEARNED 1
#define HR_MLP_PARAMS 5313

typedef struct {
    int32_t kind;        /* HR_PROPOSAL_* */
    float eps;           /* floor share of the length-proportional weights, (0,1] */
    float ema;           /* decay of the colour-jump averages, [0,1) */
    float lr;            /* Adam learning rate of the network (0 = no training) */
    float beta1, beta2, adam_eps;
} hr_proposal_config;

/* Select the proposal.  Allocates the proposal's device state on the first
   call (HR_EUNSUPPORTED above 8192 edges); resets the optimiser, the records
   and the colour-jump averages; theta_host (HOST, HR_MLP_PARAMS, nullable =
   keep the current parameters, zero at first) sets the network.  Synchronises
   the device. */
int hr_proposal_set(hr_scene* scene, const hr_proposal_config* cfg, const float* theta_host);
/* Current network parameters to HOST memory (synchronises `stream`). */
int hr_proposal_get(hr_scene* scene, float* theta_host, void* stream);
/* Use the given logits z [n_views,E] (DEVICE, nullable = the network's)
   instead of the network's; training is skipped while set. */
int hr_proposal_override(hr_scene* scene, const float* z);
/* One training step on the records of the backward passes since the last
   call (see above). */
int hr_proposal_train(hr_scene* scene, void* stream);
/* Inputs the last backward pass gave the network, DEVICE [n_views,E,16]
   float32 (the bfloat16 values; zero rows for edges that were not sampled). */
int hr_proposal_features(hr_scene* scene, float* feats, void* stream);
/* Records of the last proposal pass, DEVICE outputs (each nullable):
   z [n_views,E] logits, wq [n_views,E] u32 sampling weights (= length weights
   under HR_PROPOSAL_LENGTH), a [n_views,E] sums of |sample contribution|,
   dc [n_views,E,4] sums of |c- - c+| per channel and sample counts. */
int hr_proposal_stats(hr_scene* scene, float* z, uint32_t* wq, float* a, float* dc, void* stream);
/* The network on caller rows: X [n,16] (DEVICE float32, rounded to bfloat16
   on input) -> z [n] (DEVICE). */
int hr_proposal_eval(hr_scene* scene, const float* X, int32_t n, float* z, void* stream);
/* Gradient of KL(a / sum a || q) over caller rows taken as one view: X [n,16],
   w [n] u32 length weights (0 = not a silhouette edge), a [n] float target
   weights, 1 <= n <= 16384 (all DEVICE); grad [HR_MLP_PARAMS] DEVICE out
   (nullable); apply != 0 also takes the Adam step with it. */
int hr_proposal_fit(hr_scene* scene, const float* X, const uint32_t* w, const float* a, int32_t n, float* grad,
                    int32_t apply, void* stream);

/* ---- the paper's full data term ---------------------------------------
   Eq. 3 compares each observed image O_i with T_i R_i, the rendering under a
   per-camera 3x3 colour transform T_i (Section 3.1, "Rendering"), through
   f1 = D_c + D_e of Eq. 4: the L1 colour difference and the L1 difference of
   edge maps B(Canny(.)), Canny edges blurred by an 11x11 Gaussian of sigma 5
   (Section 3.1, "Render-and-compare").  Per view:
     E1_i = mean over masked pixels and channels |O - T R|
          + w_edge mean over masked pixels |B(Canny(O)) - B(Canny(T R))|.
   Canny: luma 0.299 R + 0.587 G + 0.114 B, 5x5 Gaussian smoothing (sigma 1),
   Sobel filters / 8, magnitude sqrt(gx^2 + gy^2 + 1e-6), suppression of
   pixels below either neighbour along the gradient direction quantised to 0,
   45, 90, 135 degrees, thresholds low / high on the magnitude, one
   8-neighbour hysteresis step (a pixel above low is kept next to one above
   high); Canny(x) = the magnitude at the kept pixels.  Filters read
   clamped-to-edge pixels of their input.  Computed in float64; the kept set
   is held fixed in the derivative (it is piecewise constant), which flows
   through the magnitude.

   hr_data_term_set allocates the buffers on its first call (10 float64
   values per pixel; synchronises the device) and sets w_edge, low, high.
   HR_EINVAL: w_edge < 0, not 0 <= low <= high, not finite. */
typedef struct {
    float w_edge;        /* weight of D_e (the paper: 1) */
    float low, high;     /* Canny thresholds on the magnitude (0.1, 0.2) */
} hr_data_term;

int hr_data_term_set(hr_scene* scene, const hr_data_term* cfg);

/* B(Canny(T image)) of every view: image [P,3], T [n_views,9] row-major
   (nullable = identity), edge_map [P] out (all DEVICE).  Used once for the
   observed images.  HR_EINVAL: before hr_data_term_set. */
int hr_edge_map(hr_scene* scene, const float* image, const float* T, float* edge_map, void* stream);

/* The full data term of each hand (sum over its views of E1_i above) and
   its gradients: image = R [P,3] (what hr_render returns), T [n_views,9]
   (nullable = identity), target = O [P,3], target_edges = B(Canny(O)) [P]
   (from hr_edge_map), mask [P] (nullable = all pixels); loss [n_hands] out,
   dimage = dE1/dR [P,3] out (hand it to hr_backward), grad_T [n_views,9] out
   (nullable), edge_map = B(Canny(T R)) [P] out (nullable).  All DEVICE. */
int hr_loss_full(hr_scene* scene, const float* image, const float* T, const float* target,
                 const float* target_edges, const uint8_t* mask, float* loss, float* dimage, float* grad_T,
                 float* edge_map, void* stream);

/* Two-level colour map (Section 3.1, "Colour mapping"): albedo = high +
   low nearest-upsampled, low [n_hands,L,L,3], high and albedo
   [n_hands,tex_h,tex_w,3]; hr_albedo_low_grad sums dE/dalbedo over each low
   texel's block into grad_low [n_hands,L,L,3].  HR_ESHAPE: L does not divide
   tex_h and tex_w. */
int hr_compose_albedo(hr_scene* scene, const float* low, int32_t L, const float* high, float* albedo, void* stream);
int hr_albedo_low_grad(hr_scene* scene, const float* grad_albedo, int32_t L, float* grad_low, void* stream);

/* One Adam step on n float32 values x (gradient g, moments m, v; t >= 1
   counts steps) with learning rate lr and cfg's betas and epsilon, the
   result clamped to [lo, hi] (the colour transforms and the low colour map).
   HR_EINVAL: n < 0, t < 1, lo > hi. */
int hr_adam(hr_scene* scene, float* x, const float* g, float* m, float* v, int64_t n, int32_t t, float lr,
            float lo, float hi, const hr_adam_config* cfg, void* stream);

/* Diagnostics of the last backward call on this scene, copied to HOST memory
   after synchronising `stream`: per view the total quantised silhouette
   length (uint64, 1/256 px) and the number of edge samples drawn.
   total_host [n_views] u64 out, budget_host [n_views] i64 out. */
int hr_edge_stats(hr_scene* scene, uint64_t* total_host, int64_t* budget_host, void* stream);

/* Work counting (profiling aid).  While enabled, hr_render and hr_backward
   launch variants of their ray-tracing kernels that count their work.
   hr_read_counts synchronises `stream`, copies 18 uint64 to counts_host
   (HOST) and resets them: for the render, interior-adjoint and edge-sampling
   kernels in turn, six counts:
     rays traced; node visits of the rays' own traversals (nodes whose box the
     ray enters); ray/triangle tests of the rays' own traversals (triangles of
     leaves whose box the ray enters); rays that hit; node visits and
     triangle tests executed by the wave packets, counted once per active
     lane (the union of the wave's traversals: the own counts over these are
     the lane utilisation of the traversal). */
int hr_set_counting(hr_scene* scene, int32_t enable);
int hr_read_counts(hr_scene* scene, uint64_t* counts_host, void* stream);

/* Per-kernel timing (profiling aid).  While enabled, every kernel the scene
   launches is bracketed by HIP events on its stream.  hr_timing_read
   synchronises `stream`, returns per kernel name (names: n x 32 chars, HOST)
   the summed milliseconds and launch counts, and clears the record. */
int hr_timing_enable(hr_scene* scene, int32_t enable);
int hr_timing_read(hr_scene* scene, char* names, double* ms, int64_t* count, int32_t max_n, int32_t* n_out,
                   void* stream);

/* Message of the last error on the calling thread ("" if none). */
const char* hr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HANDRT_H */
