// Device-side data structures shared by the HIP kernels and the host runtime of the
// batched renderer.  Nothing here is used by the CPU oracle.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/orrb.h"

namespace orrb {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // threads per raster / vertex workgroup
constexpr int kMaxLights = 8;
constexpr int kMaxSpots = 4;         // spot lights per scene
constexpr int kGuard = 1 << 24;      // snapped coordinates beyond this are discarded
constexpr int kSmallExtent = 1 << 14;// triangles up to 64 px wide use exact int32 edges
constexpr unsigned long long kEmptyKey = ~0ull;
constexpr int kFrameQueue = 8;       // word of the workspace counters the frame kernel claims from

// Per frame, built on the host from the layout.
struct FrameInfo {
    int64_t pixel_offset;  // first pixel of the frame's planes
    int64_t vbase;         // first transformed-vertex instance of the frame
    int32_t scene, width, height, tiles_x;
    int32_t obj_begin, n_obj;   // the scene's objects (global indices)
    int32_t oi_base;            // first (frame, object) instance
    int32_t light_begin, n_lights;
    int32_t track_base;         // first tracker record (frame, object) of the frame
    int32_t mode;               // frame kernel: 0 scene data in LDS, 1 in the global frame scratch
    int32_t pad0;
};

// Per object, built on the host from the layout and the mesh pool.
struct ObjInfo {
    int32_t mesh_vbegin, n_verts;  // vertex range in the mesh pool
    int32_t mesh_tbegin, n_tris;   // triangle range in the mesh pool
    int32_t scene_vbase;           // vertex offset inside its scene's block
    int32_t scene_tbase;           // scene-local triangle ID of its first triangle
};

struct RenderArgs {
    // layout tables
    const FrameInfo *frames;
    const ObjInfo *objs;
    const int2 *vitems;     // (frame, object-in-scene) work items of k_vertex
    const int2 *titems;     // (frame, tile) work items of k_raster_shade
    const int32_t *fitems;  // frames rendered by k_frame
    const int32_t *light_type;
    int32_t n_vitems, n_titems, n_fitems;
    int32_t f_grid;         // frame kernel grid: workgroup b starts with fitems[b]
    int32_t f_dynamic;      // 0: workgroup b then renders fitems[b + k f_grid]; 1: it claims
                            // fitems[f_grid + queue[kFrameQueue]++] after each frame
    int32_t tile_w, tile_h, bin_cap;
    int32_t persistent;
    // resident meshes
    const float4 *mesh_pos;  // xyz, 0
    const float4 *mesh_nrm;  // xyz, 0
    const int4 *mesh_tri;    // local vertex indices, 0
    // scenes
    const float *pose;
    const int32_t *seg;
    const uint8_t *visible;
    // cameras
    const float *view;
    const float *intr;
    const float *near_plane;
    // params
    const float *albedo, *roughness, *specular, *light_vec, *light_intensity, *exposure;
    // outputs
    float *out_rgb, *out_depth, *out_normal;
    int32_t *out_seg, *out_tri;
    unsigned long long *out_vis;
    float *out_alpha;
    uint8_t *out_rgb8;
    orrb_track *out_track;
    // spot lights (type 2) and their shadow maps (null without spot lights)
    const float *light_dir, *light_cone, *shadow_view, *shadow_intr;
    const int32_t *spot_slot;  // per light: shadow-map slot
    const float *shadow_maps;  // [slots, N, N] eye depths from the lights (0: empty)
    int32_t shadow_res;        // N
    int32_t shade_mode;        // frame kernel: bit 0 spot lights, bit 1 textures / emission; 4 depth only
    // materials: per-vertex UVs, resident textures, each object's texture, UV transform
    // and emission (null when unused)
    const float2 *mesh_uv;
    const float4 *tex_texels;
    const int4 *tex_info;      // first texel, width, height
    int32_t n_tex;
    const int32_t *obj_tex;
    const float *tex_xform;
    const float *emission;
    const int32_t *obj_ntex;  // each object's normal texture (-1 none) or null
    // post-processing of rgb8
    const float *post;   // [F, ORRB_POST_WORDS] or null
    const float *grain;  // [3, grain_h, grain_w] or null
    int32_t grain_w, grain_h;
    // workspace
    int4 *vtx_pos;     // per vertex instance: X, Y (1/256 px), bits of fp32 1/w, valid flag
    float4 *obj_rot;   // per (frame, object): rows of the fp32 view rotation (x, y, z, 0)
    int4 *obj_bbox;    // per (frame, object): covered pixel-centre range i0, j0, i1, j1
    unsigned int *queue;  // persistent work counters: [0] tiled path, [kFrameQueue] frame kernel
    // frame kernel, frames whose scene data live in global scratch (mode 1): one slice
    // of fscratch_stride bytes per workgroup holding fs_verts snapped vertices (X, Y,
    // 1/w), fs_surv survivor entries and fs_bins 16-bit bin entries; null if none
    char *fscratch;
    int64_t fscratch_stride;
    int64_t fs_verts;
    int32_t fs_surv, fs_bins;
    unsigned int *stats;  // caller's ORRB_STATS_WORDS counters of the call, or null
};

// Add v to counter `word` of the call's stats (no-op without a stats buffer).
__device__ __attribute__((always_inline)) inline void stat_add(const RenderArgs &a, int word, unsigned v) {
    if (a.stats && v) atomicAdd(a.stats + word, v);
}

// Shading adjoint over a fixed visibility buffer (orrb_adjoint.hip).
struct GradArgs {
    RenderArgs r;                    // every frame on the tiled-path tables (vertex stage)
    const unsigned long long *vis;   // forward visibility keys
    const float *grad_rgb;           // dL/d rgb, planar like the forward rgb
    const int2 *gitems;              // (frame, 32x32 tile) work items
    const int64_t *gitem_pbase;      // first partial (double) of each item
    int32_t n_gitems;
    double *partial;                 // per item: 5 per object, 4 per light, 1 exposure
    const int32_t *scene_frames, *scene_frame_begin;  // frames of each scene (CSR)
    const int32_t *frame_item_begin;                  // [F+1] item range of each frame
    const int32_t *obj_scene, *obj_local, *light_scene, *light_local;
    const int32_t *scene_obj_begin, *scene_light_begin;  // [S+1] each
    float *g_albedo, *g_rough, *g_spec, *g_lpos, *g_lint, *g_expo;
    int32_t n_objects, n_lights, n_frames;
    int32_t n_scenes, max_scene_params;  // parameters of a scene: 5 per object, 4 per light, 1 per frame
};

// launchers (defined in orrb_kernels.hip and orrb_adjoint.hip)
hipError_t launch_grad(const GradArgs &g, hipStream_t stream);
int grad_tile_size();
int grad_max_objects();

}  // namespace orrb

struct orrb_layout;
struct orrb_context;

namespace orrb {
// host-runtime internals used by the autotuner and graph code (orrb_tune.cpp)
orrb_status set_error(orrb_status st, const char *msg);
uint64_t layout_signature(const orrb_layout *L);
uint64_t layout_generation(const orrb_layout *L);    // bumped whenever its tables or tuning change
uint64_t context_generation(const orrb_context *ctx); // bumped whenever the mesh pool grows
int context_device(const orrb_context *ctx);
bool context_profiling(const orrb_context *ctx);
void context_set_profiling(orrb_context *ctx, bool on);
hipError_t launch_vertex(const RenderArgs &a, hipStream_t stream);
hipError_t launch_raster(const RenderArgs &a, hipStream_t stream, int n_cu);
hipError_t launch_frame(const RenderArgs &a, hipStream_t stream, int n_cu);
hipError_t launch_shadow_cams(const int32_t *spot_light, int n_spot, const float *shadow_view, const float *shadow_intr,
                              float *view, float *intr, float *nearp, hipStream_t stream);
hipError_t launch_validate(const RenderArgs &a, const float *post, int n_obj, int n_lights, int n_frames,
                           uint32_t *stats, hipStream_t stream);
hipError_t read_wait_timeouts(unsigned int *out);  // frame-kernel waits that hit their bound
bool frame_fits(int n_verts, int n_obj, int n_tris, int width, int height);
bool frame_fits_global(int64_t n_verts, int n_obj, int64_t n_tris, int width, int height);
size_t raster_lds_bytes(int tile_w, int tile_h, int bin_cap);
// render call shared by orrb_render_batch and orrb_render_batch_noalloc (orrb_host.cpp)
orrb_status debug_validate(orrb_context *ctx, const orrb_layout *L, const orrb_scenes *sc, const orrb_cameras *cam,
                           const orrb_params *par, const orrb_outputs *out, void *stream);
orrb_status render_impl(orrb_context *ctx, const orrb_layout *L, const orrb_scenes *sc, const orrb_cameras *cam,
                        const orrb_params *par, const orrb_outputs *out, void *workspace, size_t workspace_bytes,
                        void *stream, bool timing);
size_t render_workspace_bytes(const orrb_layout *L);  // workspace of one render call (current tuning)
hipError_t scratch_init(int device);  // resolve the device's copy of the fixed scratch (orrb_noalloc.cpp)

}  // namespace orrb
