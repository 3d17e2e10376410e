/*
 * orrb.h -- C ABI of the MI355X (gfx950) batched randomized renderer.
 *
 * The library renders many visually randomized robotics scenes at once into the four
 * channel kinds ORRB produces (arXiv:1906.11633, Sec. 4.4: RGB, segmentation, depth and
 * screen-space normal), for training-time batch rendering (Sec. 3).  Scenes follow the
 * paper's Single Scene Multiple States model (Sec. 3): meshes and the batch structure
 * ("layout") are uploaded once and stay resident; each call carries only the per-batch
 * state that randomizers change (Sec. 4.3.1: materials, lights, cameras, exposure).
 * Calls are asynchronous on a caller-supplied HIP stream, write into caller-allocated
 * destinations and never synchronize with the host (Sec. 4.4).
 *
 * Conventions (the paper prints no rendering rule; these are the library's definitions):
 *   - poses are 3x4 row-major [s*R | t], object -> world, rigid plus uniform scale;
 *   - views are 3x4 row-major world -> camera; the camera looks down -z, +y up;
 *   - intrinsics (fx, fy, cx, cy) in pixels, origin at the image's top-left corner,
 *     x right, y down, pixel (i, j) centred at (i + 1/2, j + 1/2);
 *   - meshes are counter-clockwise seen from outside; back faces are culled;
 *   - the vertex stage runs in FP64 with a fixed fma order, projected positions snap
 *     to 1/256 px (round half to even), triangles with a vertex nearer than the near
 *     plane or beyond +-65536 px are discarded, coverage uses exact integer edge
 *     functions with the top-left fill rule;
 *   - visibility: nearest fp32 eye depth wins, exact ties go to the lower scene-local
 *     triangle ID (objects in scene order, then triangles in mesh order);
 *   - depth = eye depth along -z in metres; normal = unit view-space normal
 *     interpolated perspective-correctly from vertex normals; seg = the object's id;
 *     rgb = exposure * sum over lights of A * max(0, n.l) * (albedo + k_s * s),
 *     s = max(0, n.h)^(2/r^2 - 2) (Blinn-Phong), A = I / max(|d|^2, 1e-4) for point
 *     lights and A = I for directional lights; background: rgb = depth = normal = 0,
 *     seg = -1, tri_id = -1.
 *
 * Output layout: frames are packed densely in layout order.  With P_f = W_f * H_f and
 * off_f = sum of P over earlier frames, frame f's depth / seg / tri_id / vis plane is
 * at [off_f, off_f + P_f) and its rgb / normal channel c plane at
 * [3 off_f + c P_f, 3 off_f + (c+1) P_f), row-major.  A uniform batch is [F,3,H,W].
 *
 * Errors: every entry point returns an orrb_status; nothing aborts and no C++
 * exception crosses the ABI.  Host-visible argument errors are reported before any
 * work is enqueued.  orrb_last_error() returns a thread-local message describing the
 * calling thread's most recent failure.
 *
 * Ownership: the caller owns every device buffer it passes (inputs, outputs,
 * workspace) and keeps it alive and unmodified until the stream work completes.  The
 * library owns the resident mesh pool (per context) and layout tables (per layout).
 *
 * Thread safety: a context may be used from several threads if calls on the same
 * layout are serialized by the caller; calls on different layouts and streams may
 * run concurrently.  orrb_layout_set_tuning and orrb_layout_destroy rewrite or free
 * device tables: no work that uses the layout may still be in flight.  The first
 * orrb_shade_backward call on a layout uploads its adjoint tables synchronously.
 */
#ifndef ORRB_H
#define ORRB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ORRB_OK = 0,
    ORRB_ERR_INVALID_ARGUMENT = 1,  /* a size, index, pointer or range is wrong */
    ORRB_ERR_OUT_OF_MEMORY = 2,     /* a library-owned device allocation failed */
    ORRB_ERR_WORKSPACE_TOO_SMALL = 3,
    ORRB_ERR_DEVICE = 4,            /* a HIP runtime call failed */
    ORRB_ERR_UNSUPPORTED = 5        /* the request exceeds a documented limit */
} orrb_status;

typedef struct orrb_context orrb_context;
typedef struct orrb_layout orrb_layout;

/* Documented limits. */
#define ORRB_MAX_LIGHTS_PER_SCENE 8
#define ORRB_MAX_SPOT_LIGHTS_PER_SCENE 4
#define ORRB_MAX_DIM 8192           /* frame width and height */
#define ORRB_MAX_SCENE_TRIANGLES 0x7fffff00  /* scene-local triangle IDs fit 31 bits */

/* --------------------------------------------------------------------------------- */
/* context and resident meshes (Sec. 3, Single Scene Multiple States)                 */
/* --------------------------------------------------------------------------------- */

/* Create a context on HIP device `hip_device`.  *out receives the handle.  The
 * environment is read here, once:
 *   ORRB_TILE=WxH, ORRB_BIN_CAP=N  the tuning new layouts of this context start from
 *                                  (otherwise tile 32x32, bin capacity 256); a pair that
 *                                  is no valid tuning is ORRB_ERR_INVALID_ARGUMENT;
 *   ORRB_DEBUG_VALIDATE (not "0")  every orrb_render_batch and orrb_render_batch_noalloc
 *                                  call with a stats destination first runs
 *                                  orrb_validate_batch into it;
 * and orrb_autotune reads ORRB_AUTOTUNE_CACHE when its cache_path is NULL. */
orrb_status orrb_create(int hip_device, orrb_context **out);

/* Destroy a context and free its mesh and texture pools.  If layouts of the context are
 * still alive, the context stays until the last of them is destroyed (then it is freed
 * with it); the handle must not be used after this call either way.  NULL is ignored. */
void orrb_destroy(orrb_context *ctx);

/* Message of the calling thread's last failure ("" if none); valid until that
 * thread's next orrb_* call. */
const char *orrb_last_error(void);

/* Add a mesh to the context's resident pool (host arrays, copied synchronously).
 *   pos   float [V,3] object-space positions (finite)
 *   nrm   float [V,3] object-space vertex normals (non-zero; normalized on use)
 *   idx   int32 [T,3] vertex indices in [0, V), counter-clockwise seen from outside
 * *mesh_id receives the new mesh's id (0, 1, 2, ... in call order).  Errors:
 * ORRB_ERR_INVALID_ARGUMENT for V or T < 1, V > 2^30, T > 2^26, an index out of range
 * or a non-finite value; ORRB_ERR_OUT_OF_MEMORY / ORRB_ERR_DEVICE from the upload. */
orrb_status orrb_add_mesh(orrb_context *ctx, const float *pos, const float *nrm, int32_t n_verts,
                          const int32_t *idx, int32_t n_tris, int32_t *mesh_id);

/* Texture coordinates of mesh `mesh_id`'s vertices (host [V,2], copied; meshes start
 * with all 0).  Errors: ORRB_ERR_INVALID_ARGUMENT for an unknown mesh or a non-finite
 * value. */
orrb_status orrb_set_mesh_uv(orrb_context *ctx, int32_t mesh_id, const float *uv);

/* Add a pattern texture to the context's resident pool (SSMS: textures are shared, Sec.
 * 3): host RGB texels [height, width, 3], row 0 first, copied.  *tex_id receives its id
 * (0, 1, 2, ... in call order).  Errors: ORRB_ERR_INVALID_ARGUMENT for a size outside
 * [1, ORRB_MAX_DIM] or a non-finite value. */
orrb_status orrb_add_texture(orrb_context *ctx, const float *rgb, int32_t width, int32_t height, int32_t *tex_id);

/* --------------------------------------------------------------------------------- */
/* layout: the structure of a batch (host arrays, validated and copied)               */
/* --------------------------------------------------------------------------------- */

typedef struct {
    int32_t n_scenes;
    const int32_t *scene_object_begin; /* [n_scenes+1], non-decreasing, starts at 0 */
    const int32_t *object_mesh;        /* [n_objects] mesh ids of this context */
    const int32_t *scene_light_begin;  /* [n_scenes+1], <= ORRB_MAX_LIGHTS_PER_SCENE each */
    const int32_t *light_type;         /* [n_lights] 0 = point, 1 = directional, 2 = spot light with a
                                          shadow map (<= ORRB_MAX_SPOT_LIGHTS_PER_SCENE per scene) */
    int32_t n_frames;
    const int32_t *frame_scene;        /* [n_frames] scene of each frame (camera image) */
    const int32_t *width;              /* [n_frames] in [1, ORRB_MAX_DIM] */
    const int32_t *height;             /* [n_frames] in [1, ORRB_MAX_DIM] */
    int32_t shadow_res;                /* shadow maps are shadow_res x shadow_res, in [8, 256]
                                          (ignored without spot lights) */
} orrb_layout_desc;

/* Launch choices.  They change speed only: the output bits are the same for every
 * valid tuning.  The frame kernel (one persistent launch, a workgroup renders whole
 * frames) takes frames of at most 256x256 pixels whose scene fits in LDS (<= 6976
 * vertices, <= 48 objects, < 65536 triangles) and, with path 2, also larger scenes
 * (<= 65536 vertices, <= 127 objects, < 65536 triangles) whose snapped vertices, bins
 * and survivors then live in workspace scratch; every triangle is set up once per
 * frame either way.  Other frames go through the tiled path (a vertex kernel, then one
 * workgroup per screen tile). */
typedef struct {
    int32_t tile_w, tile_h;  /* tiled path: tile size, each in {16, 32, 64} */
    int32_t bin_cap;         /* tiled path: triangles staged in LDS per flush, in {256, 512, 1024};
                                path 2: the frame kernel's global bins hold bin_cap / 128 entries
                                per triangle of the largest scratch-held scene (more: a frame falls
                                back to scanning every triangle per tile, same bits) */
    int32_t persistent;      /* tiled path: 1 = persistent grid pulling tiles from a device queue */
    int32_t path;            /* 0 = frame kernel where the scene fits in LDS, 1 = tiled path for
                                every frame, 2 = frame kernel for every frame it can take */
} orrb_tuning;

typedef struct {
    int64_t n_scenes, n_objects, n_lights, n_frames;
    int64_t total_pixels;       /* P: depth/seg hold P values, rgb/normal 3P */
    int64_t vertex_instances;   /* sum over frames of the frame's scene vertex count */
    int64_t triangle_instances; /* sum over frames of the frame's scene triangle count */
    int64_t tile_items;         /* tiled-path work items with the current tuning */
    int64_t frame_path_frames;  /* frames rendered by the frame kernel with the current tuning */
    size_t workspace_bytes;      /* workspace orrb_render_batch needs (current tuning) */
    size_t workspace_bytes_any;  /* workspace enough for every valid tuning */
    size_t grad_workspace_bytes; /* workspace orrb_shade_backward needs */
    size_t table_bytes;          /* device memory the layout itself holds (its tables) */
    orrb_tuning tuning;
    int64_t render_kernels;      /* kernel launches one orrb_render_batch makes (current tuning,
                                    shadow frames included): a captured graph's kernel nodes */
} orrb_layout_info;

/* Validate `desc` against the context's meshes and build a layout (device tables are
 * uploaded synchronously).  Errors: ORRB_ERR_INVALID_ARGUMENT for any malformed array
 * (negative counts, non-monotone offsets, unknown mesh id, bad light type, frame scene
 * out of range, size out of range), ORRB_ERR_UNSUPPORTED beyond a documented limit. */
orrb_status orrb_layout_create(orrb_context *ctx, const orrb_layout_desc *desc, orrb_layout **out);

/* Destroy a layout (waits for nothing: the caller must have synchronized the streams
 * that used it).  NULL is ignored. */
void orrb_layout_destroy(orrb_layout *layout);

orrb_status orrb_layout_info_get(const orrb_layout *layout, orrb_layout_info *info);

/* Set the layout's tuning (validated; ORRB_ERR_INVALID_ARGUMENT if out of range). */
orrb_status orrb_layout_set_tuning(orrb_layout *layout, const orrb_tuning *tuning);

/* --------------------------------------------------------------------------------- */
/* per-batch state (device pointers), the randomizers' outputs (Sec. 4.3.1)           */
/* --------------------------------------------------------------------------------- */

typedef struct {                  /* scenes: geometry state */
    const float *object_pose;     /* [O,3,4] object -> world, rigid + uniform scale */
    const int32_t *object_seg;    /* [O] segmentation id written for the object */
    const uint8_t *object_visible;/* [O] 0 hides the object (Hide component, Sec. 4.3.2) */
} orrb_scenes;

typedef struct {                  /* cameras, one per frame */
    const float *view;            /* [F,3,4] world -> camera */
    const float *intr;            /* [F,4] fx, fy, cx, cy (pixels) */
    const float *near_plane;      /* [F] > 0, metres */
} orrb_cameras;

typedef struct {                  /* sampled randomization parameters */
    const float *albedo;          /* [O,3] material tint */
    const float *roughness;       /* [O] in (0, 1] (1 - glossiness) */
    const float *specular;        /* [O] highlight weight (metallic level) */
    const float *light_vec;       /* [L,3] world position (point) or direction (directional) */
    const float *light_intensity; /* [L] */
    const float *exposure;        /* [F] linear post-processing gain */
    /* Post-processing of the 8-bit output (Sec. 4.3.1 PostprocessingRandomizer: colour
     * grading and grain; used only when orrb_outputs.rgb8 is set).  `post` [F,
     * ORRB_POST_WORDS] per frame, words ORRB_POST_*; NULL = identity grading, no grain.
     * `grain` [3, grain_h, grain_w] noise texture with values in [0, 1) (NULL = no
     * grain; at most 2^26 texels per plane, else ORRB_ERR_INVALID_ARGUMENT).  Per
     * channel c of pixel (i, j), from the linear rgb:
     *   1. white balance: c *= (1 + T/5, 1 - G/5, 1 - T/5)[c];
     *   2. clamp to [0, 1] and encode with the sRGB transfer function (IEC 61966-2-1);
     *   3. c = 1/2 + k (Y + s (c - Y) - 1/2), Y = Rec. 709 luma of the encoded pixel;
     *   4. rotate (r, g, b) by the hue angle h about the grey axis;
     *   5. grain: c += I ((1 - kappa) g0 + kappa g_c - 1/2), g at texel
     *      ((i div S + ox) mod grain_w, (j div S + oy) mod grain_h);
     *   6. code = floor(255 clamp(c, 0, 1) + 1/2), evaluated in fp32. */
    const float *post;
    const float *grain;
    int32_t grain_w, grain_h;
    /* Spot lights (type 2; the paper's benchmark scene has spot lights with soft
     * shadows, Sec. 5; the LightRandomizer draws spotlight angles, Sec. 4.3.1).  Needed
     * when the layout has spot lights (NULL otherwise).  A spot light sits at light_vec
     * and points along light_dir (world, any length); its light falls off like a point
     * light's, times smoothstep((c - cos_outer) / (cos_inner - cos_outer)) of the cosine
     * c between the axis and the direction from the light.  Each casts shadows through a
     * shadow map: the depth (along -z) of the scene seen from shadow_view / shadow_intr (a
     * camera at the light looking along its axis, over shadow_res x shadow_res pixels,
     * near plane 0.01 m), rendered with the same rules as the frames before them.  A
     * shaded point of eye depth w in the shadow camera sees the light by the fraction of
     * the 3 x 3 map texels around its texel with (1 - 0.02) w <= their depth (empty and
     * off-map texels count, a point not in front of the shadow camera is lit). */
    const float *light_dir;       /* [L,3] */
    const float *light_cone;      /* [L,2] cos(inner half-angle), cos(outer half-angle) */
    const float *shadow_view;     /* [L,3,4] world -> shadow camera (rigid) */
    const float *shadow_intr;     /* [L,4] fx, fy, cx, cy in shadow-map pixels */
    /* Materials (Sec. 4.3.1 MaterialRandomizer: pattern textures with randomized tiling
     * and offset; FixedHueMaterialRandomizer: emissive power).  Each may be NULL.  An
     * object with texture t >= 0 (a resident texture, orrb_add_texture) takes as albedo
     * its tint times the texture at (u su + ou, v sv + ov), where (u, v) is the
     * perspective-correct interpolation of the mesh's vertex UVs (orrb_set_mesh_uv) and
     * the sample is bilinear between texel centres ((i + 1/2)/W, (j + 1/2)/H), row 0
     * first, repeating; ids outside the pool mean no texture.  An emissive object adds
     * emission x albedo to the sum over lights (before exposure). */
    const int32_t *texture;       /* [O] texture id, -1 = none */
    const float *tex_xform;       /* [O,4] su, sv, ou, ov (needed with texture or normal_texture) */
    const float *emission;        /* [O] emissive power >= 0 */
    /* Normal (bump) textures (Sec. 4.3.1 MaterialRandomizer: random normal textures),
     * NULL = none: each object's normal texture id from the same pool (-1 = none),
     * sampled like `texture` at the same transformed UV.  The bilinear texel rgb encodes
     * a tangent-space direction t = normalize(2 rgb - 1); the tangent frame is the
     * triangle's (T, B from its object-space edges and UV differences, rotated with
     * the object, T orthogonalized against the interpolated normal n, B' = +-n x T' with
     * the UV mapping's handedness), and the lights see normalize(t_x T' + t_y B' +
     * t_z n).  The normal channel keeps n.  Degenerate UVs leave n unchanged. */
    const int32_t *normal_texture; /* [O] */
} orrb_params;

#define ORRB_POST_WORDS 12
#define ORRB_POST_TEMPERATURE 0  /* T, white balance warm (+) / cool (-) */
#define ORRB_POST_TINT 1         /* G, magenta (+) / green (-) */
#define ORRB_POST_HUE 2          /* h, radians */
#define ORRB_POST_SATURATION 3   /* s, 1 = unchanged */
#define ORRB_POST_CONTRAST 4     /* k, 1 = unchanged */
#define ORRB_POST_GRAIN 5        /* I, grain intensity */
#define ORRB_POST_GRAIN_COLOR 6  /* kappa in [0, 1]: 0 = the same noise on every channel */
#define ORRB_POST_GRAIN_SIZE 7   /* S >= 1, pixels per grain texel (integer-valued) */
#define ORRB_POST_GRAIN_X 8      /* ox, texel offset (integer-valued, >= 0) */
#define ORRB_POST_GRAIN_Y 9      /* oy, texel offset (integer-valued, >= 0) */

/* Tracker record (Sec. 4.3.2: screen-space coordinates and bounding boxes of the
 * tracked objects), one per (frame, object of the frame's scene): frame f's records
 * start at sum over earlier frames of their scene's object count, in scene order.
 * count, the box and the sums cover the pixels whose nearest fragment belongs to the
 * object (exact integers); the box is inclusive, (INT32_MAX, INT32_MAX, -1, -1) when
 * count is 0; the centroid is sum / count + 1/2.  (x, y) is the object frame's origin
 * projected with the frame's camera (pixels, y down) and w its eye depth along -z
 * (computed in FP64; x = y = NaN when w <= 0), hidden objects included. */
typedef struct {
    int32_t count;
    int32_t i_min, j_min, i_max, j_max;
    float x, y, w;
    uint64_t sum_i, sum_j;
} orrb_track;

/* Counters of one render call, written by its kernels into caller memory (the
 * `stats` destination of orrb_outputs).  The kernels ADD to the words, so a caller
 * zeroes the buffer before the call for per-call counts, or keeps adding across calls.
 * They are ordinary device memory: read them with a copy on the call's stream (no
 * device-wide synchronization).  Word meanings: */
#define ORRB_STAT_WAIT_TIMEOUTS     0  /* frame-kernel waits that reached their bound; the
                                          workgroup then stops, and the frames it had not
                                          finished hold unspecified pixels (0 in every test) */
#define ORRB_STAT_BIN_OVERFLOW      1  /* frame path: frames whose tile bins overflowed (each
                                          busy tile then scans every triangle; same bits) */
#define ORRB_STAT_SURVIVOR_RESETUP  2  /* frame path: frames whose survivor list overflowed
                                          (triangles set up a second time; same bits) */
#define ORRB_STAT_NEAR_VERTICES     3  /* vertex instances nearer than the near plane (their
                                          triangles are discarded) */
#define ORRB_STAT_GUARD_VERTICES    4  /* vertex instances beyond the +-65536 px guard band
                                          (their triangles are discarded) */
#define ORRB_STAT_TILED_EXTRA_FLUSH 5  /* tiled path: LDS bin flushes beyond one per tile */
#define ORRB_STAT_INVALID_STATE     6  /* objects, lights and frames whose state breaks a
                                          precondition, counted by orrb_validate_batch */
#define ORRB_STATS_WORDS 8             /* word 7 is reserved (written as 0 + 0) */

typedef struct {                  /* destinations; rgb, depth, normal, seg may each be NULL */
    float *rgb;                   /* [3P] */
    float *depth;                 /* [P] */
    float *normal;                /* [3P] */
    int32_t *seg;                 /* [P] */
    int32_t *tri_id;              /* [P] or NULL: scene-local winning triangle, -1 background */
    uint64_t *vis;                /* [P] or NULL: visibility key (fp32 depth bits << 32 | tri_id),
                                     ~0 for background; input of orrb_shade_backward */
    uint32_t *stats;              /* [ORRB_STATS_WORDS] or NULL: counters added to by the call */
    float *alpha;                 /* [P] or NULL: transparency channel (Sec. 4.4), 1 where a
                                     triangle covers the pixel centre, 0 for background */
    uint8_t *rgb8;                /* [3P] or NULL: post-processed 3 x 8-bit RGB, planar like
                                     rgb, encoded by the render kernels as they write each
                                     pixel; `rgb` may be NULL (the paper's 3 x 8-bit format) */
    orrb_track *track;            /* [sum over frames of the scene's objects] or NULL */
} orrb_outputs;

/* Render every frame of the layout.  `scenes`, `cameras`, `params`, `out` are host
 * structs holding device pointers; `workspace` is a device buffer of at least
 * orrb_layout_info.workspace_bytes (uninitialised is fine), `stream` a hipStream_t
 * (NULL: the null stream).  The kernels keep work counters in the workspace (and, on
 * the tiled path or for scratch-held scenes, vertex records, survivors and bins), so
 * calls that may overlap in time (other streams) need workspaces of their own.
 * Asynchronous: returns once the kernels are enqueued.  Preconditions the host cannot
 * check without a copy (values inside device arrays: rigid poses, near > 0, roughness
 * in (0, 1]) are the caller's; violating them gives unspecified pixels, never an
 * out-of-bounds access.  Errors: ORRB_ERR_INVALID_ARGUMENT (NULL handle or required
 * pointer), ORRB_ERR_WORKSPACE_TOO_SMALL, ORRB_ERR_DEVICE (launch failure). */
orrb_status orrb_render_batch(orrb_context *ctx, const orrb_layout *layout, const orrb_scenes *scenes,
                              const orrb_cameras *cameras, const orrb_params *params, const orrb_outputs *out,
                              void *workspace, size_t workspace_bytes, void *stream);

/* Check the per-call state of a render of `layout` against the preconditions the
 * render kernels assume without testing (they are device data: testing them on the
 * host would need a copy back).  Enqueues one kernel on `stream` that adds to
 * stats[ORRB_STAT_INVALID_STATE] (device, [ORRB_STATS_WORDS]) the number of
 *   objects: pose not a rotation times a uniform scale s > 0 (M^T M = s^2 I within 1e-3
 *            relative, det > 0), a non-finite value, albedo or specular < 0,
 *            roughness <= 0, emission < 0, a non-finite UV transform of a textured object;
 *   lights:  a non-finite value, intensity < 0, a zero directional vector; spot lights:
 *            a zero axis, cone cosines not 1 >= inner > outer >= -1, a shadow view that is
 *            not a rotation, shadow focal lengths <= 0;
 *   frames:  a view that is not a rotation (unit scale), focal lengths <= 0, near <= 0,
 *            exposure < 0, a non-finite value (post-processing words included);
 * each element counted once.  Renders nothing and reads no output.  Asynchronous like
 * orrb_render_batch; the count is read with a copy on the same stream.  Errors:
 * ORRB_ERR_INVALID_ARGUMENT for NULL arguments or missing arrays the layout needs. */
orrb_status orrb_validate_batch(orrb_context *ctx, const orrb_layout *layout, const orrb_scenes *scenes,
                                const orrb_cameras *cameras, const orrb_params *params, uint32_t *stats,
                                void *stream);

/* For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same as orrb_render_batch
 * (same kernels, same output bits) with the workspace taken from a fixed array in the
 * library's device image: ORRB_NOALLOC_SCRATCH_BYTES per device, resolved once by
 * orrb_create and held until the process ends.  The call allocates nothing (no
 * hipMalloc, no hipFree, no allocating library routine).  Every call on one device
 * shares that array and the kernels reuse it in place, so calls that overlap on one
 * device (other streams, other threads, other contexts) race and must be serialized
 * by the caller; consecutive calls on one stream are safe.  Errors: as
 * orrb_render_batch, plus ORRB_ERR_UNSUPPORTED (with nothing enqueued) when the
 * batch needs more workspace than the array holds (orrb_layout_info.workspace_bytes
 * > ORRB_NOALLOC_SCRATCH_BYTES; the frame path needs a few hundred bytes, the tiled
 * path 16 bytes per vertex instance plus 64 per object instance). */
#define ORRB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
orrb_status orrb_render_batch_noalloc(orrb_context *ctx, const orrb_layout *layout, const orrb_scenes *scenes,
                                      const orrb_cameras *cameras, const orrb_params *params,
                                      const orrb_outputs *out, void *stream);

/* --------------------------------------------------------------------------------- */
/* batched form: autotuning and graph replay                                          */
/* --------------------------------------------------------------------------------- */

/* Measure candidate tunings (frame/tiled path, tile size, bin capacity, persistent
 * grid) by rendering this batch on `stream` a few times each with HIP events, and set
 * the fastest on the layout (*chosen and *best_ms receive it; either may be NULL).
 * Every tuning gives bit-identical outputs, so tuning changes speed only.  The
 * workspace must hold orrb_layout_info.workspace_bytes_any.  `cache_path` (may be
 * NULL: ORRB_AUTOTUNE_CACHE if set, else none) names a JSON-lines file: an entry for
 * this device and batch structure is used without measuring; a new result is appended.  Synchronizes `stream`.  No work that
 * uses the layout may be in flight on other streams. */
orrb_status orrb_autotune(orrb_context *ctx, orrb_layout *layout, const orrb_scenes *scenes, const orrb_cameras *cameras,
                          const orrb_params *params, const orrb_outputs *out, void *workspace, size_t workspace_bytes,
                          void *stream, const char *cache_path, orrb_tuning *chosen, double *best_ms);

typedef struct orrb_graph orrb_graph;

/* Capture one orrb_render_batch with these exact buffers into a HIP graph and
 * instantiate it.  Replays (orrb_graph_launch) render whatever the buffers hold at
 * replay time, so a caller updates scene state, cameras and parameters in place and
 * replays.  The graph holds the layout's device tables and tuning as they were at
 * capture: once orrb_layout_set_tuning or orrb_autotune has changed the layout, or
 * orrb_add_mesh has grown the context's mesh pool (either may move device tables),
 * orrb_graph_launch refuses the graph with ORRB_ERR_INVALID_ARGUMENT and launches
 * nothing; capture a new graph then.  `stream` must not be the null stream (it is used
 * for capture only).  The layout, buffers and workspace must outlive the graph. */
orrb_status orrb_graph_create(orrb_context *ctx, const orrb_layout *layout, const orrb_scenes *scenes,
                              const orrb_cameras *cameras, const orrb_params *params, const orrb_outputs *out,
                              void *workspace, size_t workspace_bytes, void *stream, orrb_graph **graph);

/* Enqueue a replay of the captured render on `stream` (NULL: the null stream).
 * ORRB_ERR_INVALID_ARGUMENT, with nothing enqueued, if the layout or the mesh pool
 * changed since capture (see orrb_graph_create). */
orrb_status orrb_graph_launch(orrb_graph *graph, void *stream);

/* Destroy a graph (the caller must have synchronized its replays).  NULL is ignored. */
void orrb_graph_destroy(orrb_graph *graph);

/* --------------------------------------------------------------------------------- */
/* shading adjoint (gradients with respect to the randomization parameters)           */
/* --------------------------------------------------------------------------------- */

typedef struct {                  /* device destinations, overwritten (not accumulated) */
    float *albedo;                /* [O,3] */
    float *roughness;             /* [O] */
    float *specular;              /* [O] */
    float *light_vec;             /* [L,3] d/d light_vec: the world position of a point
                                     light, the world direction vector u of a directional
                                     light (l = -R_V u / |R_V u| toward the light) */
    float *light_intensity;       /* [L] */
    float *exposure;              /* [F] */
} orrb_grads;

/* Gradient of a scalar loss L through the shading, given dL/d(rgb) (`grad_rgb`, device
 * [3P], planar like the rgb output) and the visibility keys `vis` (device [P]) written
 * by an orrb_render_batch call with the same layout, scenes and cameras.  The
 * visibility is held fixed (no parameter here moves geometry).  The adjoint is the
 * analytic derivative of the shading function in include/orrb.h's conventions,
 * evaluated per pixel in FP64 and reduced in a fixed order, so repeated calls are
 * bit-identical.  Sub-gradient 0 is taken where a max(0, .) is inactive.  Scenes with
 * more than 1024 objects, layouts with spot lights and textured or emissive materials
 * return ORRB_ERR_UNSUPPORTED.  `workspace` needs
 * orrb_layout_info.grad_workspace_bytes.  Asynchronous on `stream`. */
orrb_status orrb_shade_backward(orrb_context *ctx, const orrb_layout *layout, const orrb_scenes *scenes,
                                const orrb_cameras *cameras, const orrb_params *params, const uint64_t *vis,
                                const float *grad_rgb, const orrb_grads *grads, void *workspace,
                                size_t workspace_bytes, void *stream);

/* --------------------------------------------------------------------------------- */
/* kernel timing (observability)                                                      */
/* --------------------------------------------------------------------------------- */

typedef struct {
    double vertex_ms;          /* summed device time of k_vertex launches (tiled path) */
    double raster_ms;          /* summed device time of k_raster_shade launches (tiled path) */
    double frame_ms;           /* summed device time of k_frame launches (frame path) */
    int64_t vertex_launches, raster_launches, frame_launches;
} orrb_kernel_times;

/* Enable or disable (0) per-kernel timing and reset the totals.  While enabled, every
 * timed orrb_render_batch call brackets each kernel with HIP events recorded on the
 * call's own stream (a few microseconds of overhead per timed call): with enable = 1
 * every call is timed, with enable = N > 1 every N-th (the first, then one in N), which
 * spreads that overhead over N calls.  Errors: ORRB_ERR_INVALID_ARGUMENT for a NULL
 * context or enable < 0. */
orrb_status orrb_profile_enable(orrb_context *ctx, int enable);

/* Wait for the recorded events and return the totals since the last enable. */
orrb_status orrb_profile_read(orrb_context *ctx, orrb_kernel_times *out);

/* Number of waits inside the frame kernel (compute-wave barrier, staging slot,
 * background publication, store-wave polling) that reached their bound on the
 * context's device since the library was loaded.  Each wait is bounded (about 0.3 s)
 * so that a stalled wave cannot hang the GPU; the workgroup whose wait reached the
 * bound stops at once and the frames it had not finished hold unspecified pixels.
 * Synchronizes with the device (reads a device counter, all streams); cumulative,
 * never reset.  Per-call counts without a device-wide synchronization: the stats
 * destination of orrb_outputs (ORRB_STAT_WAIT_TIMEOUTS).  Errors:
 * ORRB_ERR_INVALID_ARGUMENT for NULL arguments, ORRB_ERR_DEVICE if the read fails. */
orrb_status orrb_wait_timeouts(orrb_context *ctx, uint64_t *count_out);

#ifdef __cplusplus
}
#endif

#endif /* ORRB_H */
