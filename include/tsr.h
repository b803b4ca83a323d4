/*
 * tsr.h -- C ABI of the MI355X (gfx950) differentiable triangle-soup rasterizer.
 *
 * The operation is the differentiable rasterisation of "Triangle Splatting SLAM":
 *   - vertices with world position, RGB colour and opacity; faces are vertex triplets
 *     (Sec. 3.1); the default layout is a soup, face m = vertices 3m, 3m+1, 3m+2;
 *   - projection v_I = pi(T_CW v_W) with a pinhole pi (eq. 1);
 *   - window I(p) = min(1, max(0, phi(p)/phi(s)))^sigma of the edge-distance field phi
 *     (eqs. 2-3), face opacity o_F = mean of the vertex opacities and barycentric vertex
 *     colour (Sec. 3.1);
 *   - front-to-back alpha compositing in depth order (eq. 4), of colour and of depth
 *     D = sum z_F alpha T (the rendered depth of eqs. 9 and 13);
 *   - the analytic backward pass to vertex positions, colours, opacities and the se(3)
 *     left perturbation of T_CW (eqs. 5-7);
 *   - the training energies around it: the L1 photometric and depth terms and the D-SSIM
 *     term (eqs. 8 and 10), the equilateral regulariser (eq. 14), and the per-face screen
 *     statistics that the map-management tests of Sec. 3.4 threshold.
 *
 * Conventions shared by every entry point
 *   - Pointers are DEVICE pointers unless marked (host).  Structs passed by pointer are host
 *     memory.  Float arrays are float32, integer arrays int32 / uint32 / uint64 as stated.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only enqueues work
 *     on `stream` and returns without synchronising, except tsr_check / tsr_count.
 *   - The caller owns every buffer, the workspace and scratch buffers included; the library
 *     never allocates or frees device memory.  A new workspace is initialised once with tsr_workspace_init.  The workspace carries the binning between tsr_bin_and_sort,
 *     tsr_render_forward and tsr_render_backward; reusing it for another scene, pose set or
 *     view set invalidates that state.
 *   - A pose is T_CW (world -> camera): 12 floats, R row-major then t.  Camera frame x right,
 *     y down, z forward; pixel (u, v) samples the image point (u, v) (integer pixel centres).
 *   - Several views may be rendered in one call (1 <= n_views <= TSR_MAX_VIEWS), each with
 *     its own pose and intrinsics.  Per-view images are packed view after view: view v
 *     starts at pixel offset P_v = sum_{v'<v} H_v' W_v'; colour is [3][H_v][W_v] at float
 *     offset 3 P_v, depth and transmittance [H_v][W_v] at offset P_v.
 *   - Outputs are overwritten.  Gradient outputs are sums over all views of the call.
 *     A NULL gradient output pointer skips that output.
 *   - Errors: functions never abort.  They return TSR_OK (0) or a negative code and set a
 *     thread-local message readable with tsr_last_error():
 *       TSR_EINVAL     null required pointer, n_views out of range, width/height outside
 *                      (0, 16384], sigma <= 0, t_min outside [0, 1), negative sizes,
 *                      n_views * n_faces >= 2^31;
 *       TSR_EWORKSPACE workspace smaller than tsr_workspace_size() for zero pairs;
 *       TSR_ECAPACITY  more (tile, face) pairs than the workspace holds.  Detected on the
 *                      device: tsr_bin_and_sort then leaves every tile list empty (all later
 *                      kernels do no work), and the condition is reported by tsr_check;
 *       TSR_EHIP       a HIP runtime call or launch failed (message has the HIP error);
 *       TSR_EINTERNAL  a device-side consistency check of the binning failed (a tile slot
 *                      outside its tile's range; the pair is dropped, never written out of
 *                      bounds); reported by tsr_check.
 *   - NaN or infinite inputs give unspecified image values but no fault.  Faces with a
 *     vertex closer than z_near, or with inradius below r_min pixels, are culled.
 *     Opacities are used as given (the caller applies any activation).
 *   - Thread safety: calls are safe from several host threads when each uses its own
 *     workspace and stream.
 */
#ifndef TSR_H
#define TSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define TSR_API __attribute__((visibility("default")))
#else
#define TSR_API
#endif

#define TSR_OK 0
#define TSR_EINVAL (-1)
#define TSR_EWORKSPACE (-2)
#define TSR_ECAPACITY (-3)
#define TSR_EHIP (-4)
#define TSR_EINTERNAL (-5)

#define TSR_MAX_VIEWS 32
#define TSR_TILE 16

/* Pinhole intrinsics of one view (host). */
typedef struct {
    int32_t width, height;   /* image size in pixels, each in (0, 16384] */
    float fx, fy, cx, cy;    /* u = fx x/z + cx, v = fy y/z + cy */
} tsr_intrinsics;

/* Rendering parameters (host). */
typedef struct {
    float sigma;    /* window exponent of eq. 3, > 0 (1: linear, 0.5: square root) */
    float t_min;    /* a pixel stops after the face that brings its transmittance below
                       t_min (0 disables the early stop) */
    float z_near;   /* near-plane cull distance in metres */
    float r_min;    /* cull faces whose projected inradius is below r_min pixels */
    float w_color;  /* L1 colour weight of the fused training loss (eq. 8, 1 - lambda) */
    float w_depth;  /* L1 depth weight of the fused training loss (eq. 10, lambda_dep) */
    int32_t opacity_min; /* 0: face opacity = mean of the vertex opacities (Sec. 3.1, the
                            paper's choice); 1: = their minimum (the Mesh Splatting variant the
                            paper's ablation compares with), the opacity gradient then going to
                            the lowest-opacity vertex (the lowest index on ties) */
    int32_t tight_tiles; /* 0: a face is listed in every tile of its pixel rectangle (conservative
                            bounding box); 1: only in the tiles whose box of pixel centres (clipped
                            to the rectangle) reaches below 0 in every edge function of eq. 2, i.e.
                            that can hold a pixel the face covers.  Images and gradients are the
                            same either way (the dropped pairs have alpha = 0 at every pixel of
                            their tile); the lists are shorter.  Decided in FP64. */
    int32_t perspective; /* 0: colour interpolated with the affine screen-space barycentrics of
                            the projected triangle and depth D = sum z_F alpha T (Sec. 3.1 and
                            eq. 4 as read); 1: perspective-correct barycentrics
                            mu_i = (lambda_i / z_i) / sum_j (lambda_j / z_j) for the colour and the
                            depth of the face's plane along the pixel's ray, 1 / sum_j (lambda_j /
                            z_j), in D (the variant); the depth order stays that of z_F.  Cannot be
                            combined with scene->face_sigma (TSR_EINVAL). */
} tsr_params;

/* Scene (host struct of device pointers). */
typedef struct {
    const float *pos;        /* [3][N] world positions, SoA */
    const float *col;        /* [3][N] RGB, SoA */
    const float *opa;        /* [N] opacities */
    const int32_t *faces;    /* [M][3] vertex indices, or NULL for a soup (N = 3M) */
    int64_t n_vertices;      /* N */
    int64_t n_faces;         /* M */
    const float *face_sigma; /* [M] each face's window exponent sigma_m of eq. 3, > 0 (the
                                Triangle Splatting variant that learns sigma per triangle,
                                Sec. 3.2), or NULL: every face uses params->sigma (the paper's
                                global constant).  Values <= 0 or NaN give unspecified images. */
    float *grad_face_sigma;  /* [M] output, or NULL: dL/dsigma_m summed over the call's views
                                (0 for faces no view blends), written by tsr_render_backward,
                                tsr_render_train_l1 and tsr_render_train_photometric when
                                face_sigma is set.  tsr_render_train_normal renders with the
                                per-face exponents but leaves this output alone. */
} tsr_scene;

/* Work schedule of the fused training kernel (host).  NULL selects the default
 * {persistent = 0, order = 0, grid = 0}.  Results do not depend on the schedule except for
 * the summation order of the floating-point gradient atomics. */
typedef struct {
    int32_t persistent;  /* 0: one workgroup per tile; 1: persistent workgroups pull tiles from a
                            device-side queue */
    int32_t order;       /* 0: tiles in id order (XCD-interleaved when not persistent);
                            1: longest tile lists first (computed on the device) */
    int32_t grid;        /* persistent workgroups; 0 = 2048 */
} tsr_schedule;

/* Read-only view of the binning held in a workspace (device pointers). */
typedef struct {
    const uint64_t *pairs;     /* [capacity] sorted pairs; pair i = (float32 bits of z_F << 32) | face,
                                  face = v * M + m; valid entries are those inside a tile range */
    const uint32_t *ranges;    /* [n_tiles][2] start, end of each tile's run in `pairs`;
                                  tile ids are view-major: tile_offset(v) + ty * tiles_x + tx */
    const int64_t *n_pairs;    /* device scalar: total pairs K emitted (also when it overflowed) */
    const uint32_t *overflow;  /* device scalar: nonzero when K exceeded the capacity */
    const uint32_t *tile_counts; /* [V * M] number of tiles each (view, face) overlaps, 0 = culled */
    const float *records;      /* [V * M][24] per-face setup records (visible faces only) */
    int64_t capacity;          /* pairs the workspace holds */
    int64_t n_tiles;           /* total tiles over all views */
    int64_t n_pixels;          /* total pixels over all views */
    const int32_t *last_face;  /* [n_pixels] position in `pairs` of each pixel's last blended face
                                  in the latest tsr_render_forward (-1: none), packed per view */
} tsr_binning;

/* Bytes of workspace needed for this scene size, view set and a capacity of `pair_capacity`
 * (tile, face) pairs.  Workspace size depends only on M, the intrinsics and the capacity. */
TSR_API int tsr_workspace_size(const tsr_scene *scene, const tsr_intrinsics *intr /* (host)[n_views] */,
                       int n_views, int64_t pair_capacity, size_t *bytes /* (host) out */);

/* Clears the workspace header (pair count, overflow flags, queue counter).  Call once on
 * every newly allocated workspace before its first use (enqueued on `stream`; a kernel, so
 * it may also be captured). */
TSR_API int tsr_workspace_init(void *ws, size_t ws_bytes, void *stream);

/* Projection, per-face setup, tile binning and per-tile depth sort (eqs. 1-3 and the depth
 * order of eq. 4): every visible face is listed in each 16x16 tile its pixel bounding box
 * overlaps; each tile's list is sorted by (float32 z_F, face).  z_F is the mean camera-space
 * depth of the face's vertices.  Poses: [n_views][12]. */
TSR_API int tsr_bin_and_sort(const tsr_scene *scene, const float *poses, const tsr_intrinsics *intr,
                     int n_views, const tsr_params *params, void *ws, size_t ws_bytes,
                     void *stream);

/* Exact pair count K for the given views without sorting; synchronises `stream`.
 * Uses the fixed part of `ws` only (any capacity, even 0, suffices) and invalidates any
 * binning held in `ws`. */
TSR_API int tsr_count(const tsr_scene *scene, const float *poses, const tsr_intrinsics *intr,
              int n_views, const tsr_params *params, void *ws, size_t ws_bytes, void *stream,
              int64_t *n_pairs /* (host) out */);

/* Device pointers into the binning state of `ws` (no device access, no synchronisation). */
TSR_API int tsr_binning_view(const tsr_scene *scene, const tsr_intrinsics *intr, int n_views,
                     const void *ws, size_t ws_bytes, tsr_binning *out /* (host) */);

/* Forward render (eq. 4) of the binned views: colour [3][H][W], depth, final transmittance
 * per view (packed as above).  Also stores in `ws` each pixel's last blended face and its
 * transmittance before that face, which the backward pass starts from.  Requires a
 * preceding tsr_bin_and_sort on the same workspace and inputs.  trans may be NULL. */
TSR_API int tsr_render_forward(const tsr_scene *scene, const float *poses, const tsr_intrinsics *intr,
                       int n_views, const tsr_params *params, void *ws, size_t ws_bytes,
                       float *color, float *depth, float *trans, void *stream);

/* Backward of tsr_render_forward (Sec. 3.3): given dL/dcolour, dL/ddepth and optionally
 * dL/dtrans (NULL = 0), packed like the outputs, writes dL/dpos [3][N], dL/dcol [3][N],
 * dL/dopa [N] and the pose gradient [n_views][6] = (dL/drho, dL/dtheta) of the left
 * perturbation Exp(tau) T_CW (eqs. 6-7).  Walks each tile back to front, recovering the
 * transmittance by division from the stored per-pixel state. */
TSR_API int tsr_render_backward(const tsr_scene *scene, const float *poses, const tsr_intrinsics *intr,
                        int n_views, const tsr_params *params, void *ws, size_t ws_bytes,
                        const float *grad_color, const float *grad_depth, const float *grad_trans,
                        float *grad_pos, float *grad_col, float *grad_opa, float *grad_pose,
                        void *stream);

/* Fused training step on binned views: forward render, the L1 loss of eqs. 8-10 without the
 * D-SSIM term, L = w_color mean|C - Cbar| + w_depth mean([Dbar > 0] |D - Dbar|) per view,
 * and its backward, with each tile's forward state kept on chip between the two passes.
 * Targets are packed like the outputs.  color/depth/trans/loss may be NULL (loss: [n_views]).
 * Gradients as in tsr_render_backward.  `schedule` (nullable) picks the tile schedule. */
TSR_API int tsr_render_train_l1(const tsr_scene *scene, const float *poses, const tsr_intrinsics *intr,
                        int n_views, const tsr_params *params, void *ws, size_t ws_bytes,
                        const float *target_color, const float *target_depth,
                        float *color, float *depth, float *trans, float *loss,
                        float *grad_pos, float *grad_col, float *grad_opa, float *grad_pose,
                        const tsr_schedule *schedule, void *stream);

/* Gradient-descent pose step on the device: T_CW <- Exp(-(lr_trans g_rho, lr_rot g_theta)) T_CW
 * for each view (the tracking update of Sec. 3.4); poses [n_views][12] updated in place. */
TSR_API int tsr_pose_step(float *poses, const float *grad_pose, int n_views, float lr_trans, float lr_rot,
                  void *stream);

/* Left perturbation of poses (eq. 6): out_poses[v] = Exp(tau_v) T_v for tau [n_views][6] =
 * (rho, theta), translation first, Exp of se(3) in closed form (Rodrigues rotation, SO(3) left
 * Jacobian on rho), evaluated in FP64 and stored as float32.  poses and out_poses [n_views][12]
 * may be the same buffer.  Errors: TSR_EINVAL for NULL pointers or n_views outside
 * [1, TSR_MAX_VIEWS].  Enqueued on `stream`. */
TSR_API int tsr_pose_compose(const float *tau, const float *poses, int n_views, float *out_poses, void *stream);

/* Gradient with respect to tau of a loss evaluated at the composed pose Exp(tau) T (eqs. 6-7):
 * given grad_pose [n_views][6], the left-perturbation gradient at Exp(tau) T that
 * tsr_render_backward returns for those poses, writes grad_tau [n_views][6] = J_l(tau)^T
 * grad_pose, J_l the left Jacobian of SE(3) (series of the se(3) adjoint, FP64).  At tau = 0
 * J_l = I.  grad_tau may alias grad_pose.  Errors as tsr_pose_compose. */
TSR_API int tsr_pose_tau_grad(const float *tau, const float *grad_pose, int n_views, float *grad_tau,
                              void *stream);

/* D-SSIM term of the photometric energy (Sec. 3.4, eq. 8).  Per view v,
 *   loss[v] = 1 - mean over its 3 channels and W H pixels of SSIM(p),
 *   SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),
 * x the rendered colour, y the target, mu / s^2 / s_xy the local means, variances and
 * covariance over an 11 x 11 Gaussian window (standard deviation 1.5, weights summing to 1;
 * pixels outside the image count as 0, the window is not renormalised), C1 = 0.01^2,
 * C2 = 0.03^2, s_x^2 = E[x^2] - mu_x^2.  The paper names the term without its parameters;
 * these are the usual ones.
 * color, target: device [sum_v 3 H_v W_v] packed like tsr_render_forward's colour output.
 * loss: device [n_views] or NULL.  grad_color: device, packed like color, or NULL; receives
 * weight * dloss[v]/dcolor (accumulate = 0) or has it added (accumulate != 0), so the L1
 * colour gradient of eq. 8 and this term can share one buffer for tsr_render_backward.
 * scratch: device, 256-byte aligned, at least tsr_dssim_scratch_size bytes (52 bytes per
 * pixel plus 16 per 32 x 32 tile and channel), owned by the caller; its contents need no
 * clearing.  Enqueued on `stream`; no allocation, no synchronisation (capturable).
 * Errors: TSR_EINVAL for NULL inputs, both outputs NULL, or a view size outside
 * (0, 16384]; TSR_EWORKSPACE for a short scratch. */
TSR_API int tsr_dssim_scratch_size(const tsr_intrinsics *intr /* (host)[n_views] */, int n_views,
                           size_t *bytes /* (host) out */);
TSR_API int tsr_dssim(const tsr_intrinsics *intr /* (host)[n_views] */, int n_views, const float *color,
              const float *target, float weight, int accumulate, float *loss, float *grad_color,
              void *scratch, size_t scratch_bytes, void *stream);

/* Full training step of the photometric and depth energies (eqs. 8 and 10) on binned views:
 * forward render into color / depth / trans, then per view
 *   loss[v] = w_color mean|C - Cbar| + w_ssim L_D-SSIM(C, Cbar) + w_depth mean([Dbar > 0] |D - Dbar|)
 * (w_color = 1 - lambda and w_depth = lambda_dep from params, w_ssim = lambda = 0.2 in the
 * paper; D-SSIM as in tsr_dssim), its per-pixel seeds, and their backward as in
 * tsr_render_backward.  Unlike tsr_render_train_l1 the forward and backward are separate
 * passes: the D-SSIM gradient at a pixel needs the rendered colour of its 11 x 11
 * neighbourhood.  color and depth must not be NULL; trans and loss may be.  scratch as for
 * tsr_dssim (the seeds live there).  Requires a preceding tsr_bin_and_sort. */
TSR_API int tsr_render_train_photometric(const tsr_scene *scene, const float *poses, const tsr_intrinsics *intr,
                                 int n_views, const tsr_params *params, void *ws, size_t ws_bytes,
                                 const float *target_color, const float *target_depth, float w_ssim,
                                 float *color, float *depth, float *trans, float *loss,
                                 float *grad_pos, float *grad_col, float *grad_opa, float *grad_pose,
                                 void *scratch, size_t scratch_bytes, void *stream);

/* Equilateral regulariser (Sec. 3.4, eq. 14):
 *   loss = (1/M) sum over faces (1/3) sum over corners (cos theta - 1/2)^2,
 * cos theta the dot product of the two unit edge vectors leaving the corner.  A face with a
 * zero-length edge contributes 0, gets no gradient and still counts in M (the paper leaves
 * it undefined).  Uses scene->pos and scene->faces only (a soup when faces is NULL).
 * loss: device [1] or NULL.  grad_pos: device [3][N] or NULL; receives weight * dloss/dpos
 * (accumulate = 0; vertices of no face get 0) or has it added (accumulate != 0).  Indexed
 * meshes add with float atomics, so their gradient sums in no fixed order.  Face indices
 * outside [0, N) skip their face.  scratch: device, 8-byte aligned, at least
 * tsr_equilateral_scratch_size bytes (8 per 256 faces).  Per-face arithmetic in FP64.
 * Enqueued on `stream`; no allocation, no synchronisation. */
TSR_API int tsr_equilateral_scratch_size(int64_t n_faces, size_t *bytes /* (host) out */);
TSR_API int tsr_equilateral(const tsr_scene *scene, float weight, int accumulate, float *loss, float *grad_pos,
                    void *scratch, size_t scratch_bytes, void *stream);

/* Allocation-free variant of tsr_equilateral, for callers that cannot allocate device memory
 * or hand over a scratch buffer (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Arguments, results and errors as tsr_equilateral without `scratch`:
 * the per-workgroup partial sums live in a static device array of the library (128 KiB on each
 * GPU it runs on, held until the process ends), so n_faces may be at most
 * TSR_EQUI_NOALLOC_MAX_FACES (TSR_EINVAL beyond).  `stream` must belong to the current device
 * (TSR_EINVAL otherwise).  The first call on a device looks up the array's address there.
 * Every call on one GPU shares its array: calls that overlap on one GPU (other streams or host
 * threads) race, and the caller must serialise them.  No device memory is allocated or freed. */
#define TSR_EQUI_NOALLOC_MAX_FACES 4194304
TSR_API int tsr_equilateral_noalloc(const tsr_scene *scene, float weight, int accumulate, float *loss,
                                    float *grad_pos, void *stream);

/* Per-(view, face) screen statistics behind the map-management tests of Sec. 3.4 (pruning by
 * projected area, densification by pixel coverage, keyframing by visibility), each [V * M]
 * indexed v * M + m, all device, each may be NULL:
 *   area:     projected image-space area in pixels^2 (FP64 setup as in the binning, stored as
 *             float) of faces that pass the near-plane and inradius culls and overlap the
 *             image; 0 for the others.  Needs no binning.
 *   coverage: number of pixels at which the face has the largest blending weight alpha T along
 *             the ray (the first in depth order on ties), with the forward pass's blending
 *             decisions and early stop;
 *   visible:  1 when the face is blended at one pixel or more, else 0.
 * coverage and visible need a preceding tsr_bin_and_sort with the same inputs; both are
 * overwritten.  The paper names the tests, not these definitions: coverage as the number of
 * pixels where the face dominates is the reading taken for its blur-split criterion. */
TSR_API int tsr_face_stats(const tsr_scene *scene, const float *poses, const tsr_intrinsics *intr, int n_views,
                   const tsr_params *params, void *ws, size_t ws_bytes, float *area, uint32_t *coverage,
                   uint32_t *visible, void *stream);

/* Sensor normals from depth (Sec. 3.4): for each pixel the back-projected points
 * p(u, v) = D(u, v) ((u - cx)/fx, (v - cy)/fy, 1) of its left/right and upper/lower
 * neighbours give central differences dx, dy and N_bar = (dx x dy) / |dx x dy| (camera frame;
 * a surface facing the camera gets a normal pointing away from it).  Border pixels, pixels
 * where the depth of the pixel or of a neighbour is <= 0, and zero cross products get
 * N_bar = (0, 0, 0), which marks them invalid for tsr_render_train_normal.  FP64 arithmetic.
 * depth: device [sum_v H_v W_v] packed like the rendered depth; normals: device, packed like
 * the rendered colour ([3][H][W] per view). */
TSR_API int tsr_sensor_normals(const float *depth, const tsr_intrinsics *intr /* (host)[n_views] */, int n_views,
                       float *normals, void *stream);

/* Normal loss of mapping (Sec. 3.4) on a soup, one step: per view
 *   loss[v] = w_norm * mean over valid pixels of (1 - N(p) . N_bar(p))   (0 without valid pixels),
 * N the rendered normal map (camera frame): each face's world unit normal
 * (v1 - v0) x (v2 - v0) / |.| (vertex order, no flip) composited front to back like a colour
 * constant over the face (eq. 4 weights), rotated by R_CW, not renormalised.  target_normals:
 * N_bar packed like colour; a zero vector marks an invalid pixel (as tsr_sensor_normals
 * writes).  Outputs (each may be NULL): normal_map (packed like colour), loss [n_views]
 * (overwritten), grad_pos [3][N], grad_opa [N], grad_pose [n_views][6]: the gradients of the
 * sum of loss[v], overwriting the outputs (accumulate = 0) or added to them (accumulate != 0,
 * so that the terms of the mapping energy can share one set of gradient buffers).  Runs its own binning, forward and backward with the face normals as vertex
 * colours: it needs no preceding tsr_bin_and_sort, and it leaves `ws` binned for that
 * normal-coloured scene, so bin again before rendering the scene's colours with `ws`.
 * scratch: device, 256-byte aligned, at least tsr_normal_scratch_size bytes (40 per vertex +
 * 32 per pixel + 2.1 KB).  Soups only (faces == NULL): TSR_EINVAL otherwise. */
TSR_API int tsr_normal_scratch_size(const tsr_scene *scene, const tsr_intrinsics *intr /* (host)[n_views] */,
                            int n_views, size_t *bytes /* (host) out */);
TSR_API int tsr_render_train_normal(const tsr_scene *scene, const float *poses, const tsr_intrinsics *intr,
                            int n_views, const tsr_params *params, void *ws, size_t ws_bytes,
                            const float *target_normals, float w_norm, float *normal_map, float *loss,
                            float *grad_pos, float *grad_opa, float *grad_pose, int accumulate, void *scratch,
                            size_t scratch_bytes, void *stream);

/* The mapping energy's rendering terms in one step (Sec. 3.4): the photometric and depth
 * terms of tsr_render_train_photometric and the normal term of tsr_render_train_normal on ONE
 * binning of the scene's colours.  The forward pass composites each face's world unit normal
 * as three more channels beside the colour (a normal is constant over its face, so it blends
 * like a flat colour, with the eq. 4 weights), and the backward pass takes the colour, depth
 * and normal seeds in one walk.  Per view:
 *   loss[v]      = as tsr_render_train_photometric (w_color, w_depth from params, w_ssim);
 *   loss_norm[v] = as tsr_render_train_normal's loss (w_norm).
 * grad_pos [3][N], grad_col [3][N], grad_opa [N], grad_pose [n_views][6] (each may be NULL)
 * receive the gradient of sum_v (loss[v] + loss_norm[v]), overwriting them; with per-face
 * exponents, scene->grad_face_sigma receives that of both terms.  With params->perspective the
 * colour and depth are interpolated perspective-correctly; a normal, constant over its face, is
 * the same either way.  color and depth must not be
 * NULL; trans, normal_map (N in the camera frame, packed like colour), loss and loss_norm may
 * be.  target_color, target_depth as for the photometric step, target_normals as for the
 * normal step (a zero vector marks an invalid pixel).  Requires a preceding tsr_bin_and_sort
 * of the same scene (its colours, not the normals: the normals ride in the walks).
 * scratch: device, 256-byte aligned, at least tsr_mapping_scratch_size bytes (the D-SSIM
 * scratch + 32 per face + 128 per 16 x 16 tile + 2.5 KB), owned by the caller, no clearing
 * needed.
 * Soups only (faces == NULL): TSR_EINVAL otherwise.  Enqueued on `stream`; no allocation. */
TSR_API int tsr_mapping_scratch_size(const tsr_scene *scene, const tsr_intrinsics *intr /* (host)[n_views] */,
                                     int n_views, size_t *bytes /* (host) out */);
TSR_API int tsr_render_train_mapping(const tsr_scene *scene, const float *poses, const tsr_intrinsics *intr,
                                     int n_views, const tsr_params *params, void *ws, size_t ws_bytes,
                                     const float *target_color, const float *target_depth,
                                     const float *target_normals, float w_ssim, float w_norm, float *color,
                                     float *depth, float *trans, float *normal_map, float *loss, float *loss_norm,
                                     float *grad_pos, float *grad_col, float *grad_opa, float *grad_pose,
                                     void *scratch, size_t scratch_bytes, void *stream);

/* Synchronise `stream` and report device-side conditions of `ws`: TSR_ECAPACITY when the
 * last binning, or any binning since the previous tsr_check (e.g. inside a replayed graph),
 * overflowed; that condition is then cleared.  Writes the last K to *n_pairs when non-NULL.
 * Never call it while `stream` is being captured. */
TSR_API int tsr_check(const void *ws, void *stream, int64_t *n_pairs /* (host) out, nullable */);

/* Kernel timing (diagnostics).  While enabled, every kernel the library launches is
 * bracketed by two HIP events recorded on its launch stream.  tsr_profile_read synchronises
 * on those events and writes a JSON object {"kernel name": [launches, total milliseconds], ...}
 * accumulated since the last reset into buf (host, len bytes).  Do not enable during HIP
 * graph capture.  Process-wide state, guarded by a mutex. */
TSR_API int tsr_profile_enable(int on);
TSR_API int tsr_profile_reset(void);
TSR_API int tsr_profile_read(char *buf, size_t len);

/* Message of the last failure on this thread ("" if none). */
TSR_API const char *tsr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TSR_H */
