// Host runtime of the batched renderer: the C ABI declared in include/orrb.h.
//
// A context owns the resident mesh pool (Single Scene Multiple States: geometry is
// uploaded once and shared by every scene instance).  A layout owns the device tables
// describing one batch structure (which meshes each scene uses, frame sizes, tile and
// vertex work items); building it validates every host-visible argument, so a render
// call only checks pointers and the workspace size before enqueueing two kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/orrb.h"
#include "orrb_device.h"

using namespace orrb;

// --------------------------------------------------------------------------------------
// errors
// --------------------------------------------------------------------------------------

static thread_local std::string g_last_error;

static orrb_status fail(orrb_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t _e = (expr);                                                                    \
        if (_e != hipSuccess)                                                                      \
            return fail(_e == hipErrorOutOfMemory ? ORRB_ERR_OUT_OF_MEMORY : ORRB_ERR_DEVICE,       \
                        "%s failed: %s", #expr, hipGetErrorString(_e));                            \
    } while (0)

// --------------------------------------------------------------------------------------
// device buffers
// --------------------------------------------------------------------------------------

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t upload(const void *src, size_t n) {
        if (n > bytes) {
            if (p) (void)hipFree(p);
            p = nullptr;
            bytes = 0;
            hipError_t e = hipMalloc(&p, n);
            if (e != hipSuccess) return e;
            bytes = n;
        }
        if (n == 0) return hipSuccess;
        return hipMemcpy(p, src, n, hipMemcpyHostToDevice);
    }
};

// Several host tables packed into one device allocation (one malloc, one copy).
struct Packed {
    std::vector<char> host;
    DevBuf dev;
    size_t add(const void *src, size_t n) {
        const size_t off = (host.size() + 255) & ~size_t(255);
        host.resize(off + n);
        if (n) memcpy(host.data() + off, src, n);
        return off;
    }
    template <class T>
    size_t add(const std::vector<T> &v) { return add(v.data(), sizeof(T) * v.size()); }
    hipError_t upload() { return dev.upload(host.data(), host.size()); }
    template <class T>
    const T *at(size_t off) const { return (const T *)((const char *)dev.p + off); }
    void clear() { host.clear(); }
};

struct ScopedDevice {
    int prev = -1;
    explicit ScopedDevice(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        // a failed switch must not leave its error for the caller's next HIP call
        if (prev != dev && hipSetDevice(dev) != hipSuccess) (void)hipGetLastError();
    }
    ~ScopedDevice() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Per-kernel timing with HIP events on the caller's stream (observability).
struct KernelTimer {
    bool enabled = false;
    int every = 1;      // time every `every`-th render call
    int64_t calls = 0;  // render calls since enabled
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[3];  // 0 vertex, 1 raster, 2 frame
    double total_ms[3] = {0, 0, 0};
    int64_t count[3] = {0, 0, 0};
    hipEvent_t get() {
        hipEvent_t e = nullptr;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }
    hipError_t drain() {
        for (int k = 0; k < 3; ++k) {
            for (auto &pr : pending[k]) {
                hipError_t e = hipEventSynchronize(pr.second);
                if (e != hipSuccess) return e;
                float ms = 0.f;
                e = hipEventElapsedTime(&ms, pr.first, pr.second);
                if (e != hipSuccess) return e;
                total_ms[k] += ms;
                count[k] += 1;
                pool.push_back(pr.first);
                pool.push_back(pr.second);
            }
            pending[k].clear();
        }
        return hipSuccess;
    }
    ~KernelTimer() {
        (void)drain();
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

struct orrb_context {
    int device = 0;
    int n_cu = 256;
    KernelTimer timer;
    // host copies of the pool
    std::vector<float4> pos, nrm;
    std::vector<int4> tri;
    std::vector<int32_t> mesh_vbegin{0}, mesh_tbegin{0};
    DevBuf d_pos, d_nrm, d_tri;
    // per-vertex texture coordinates of the pool (0 until orrb_set_mesh_uv) and the
    // resident pattern textures (RGB texels as float4, per texture: first texel, w, h)
    std::vector<float2> uv;
    std::vector<float4> texels;
    std::vector<int4> tex_info;
    DevBuf d_uv, d_texels, d_tex_info;
    int n_layouts = 0;
    bool destroy_pending = false;  // orrb_destroy called while layouts were alive: freed with the last one
    uint64_t generation = 0;  // bumped whenever the mesh pool grows (its buffers may move)
    // from the environment at orrb_create
    orrb_tuning default_tuning{32, 32, 256, 0, 0};  // new layouts start from it
    bool debug_validate = false;  // every render call first checks its preconditions
};

struct orrb_layout {
    orrb_context *ctx = nullptr;
    int64_t n_scenes = 0, n_objects = 0, n_lights = 0, n_frames = 0;
    int64_t total_pixels = 0, vertex_instances = 0, triangle_instances = 0;
    int64_t max_frame_pixels = 0;
    // tiled-path sizes with the current tuning, and with every frame on the tiled path
    int64_t tiled_vertex_instances = 0, tiled_object_instances = 0;
    int64_t all_vertex_instances = 0, all_object_instances = 0;
    std::vector<FrameInfo> frames;
    std::vector<ObjInfo> objs;
    std::vector<int64_t> scene_verts, scene_tris;
    std::vector<uint8_t> fits;  // per frame: 1 scene fits the frame kernel's LDS, 2 its global scratch, 0 neither
    // frames on the frame kernel with scene data in global scratch (tuning path 2)
    int64_t gframes = 0, gf_verts = 0, gf_tris = 0;
    std::vector<int2> vitems, titems;
    std::vector<int32_t> fitems;  // frame-kernel schedule (see schedule_frames)
    int64_t f_frames = 0;          // frames on the frame kernel
    int32_t f_grid = 0;            // its persistent grid
    int32_t f_dynamic = 0;         // 1: frames claimed from a counter (uneven batch)
    std::vector<int32_t> light_type;
    Packed tab;  // frames, objs, vitems, titems, fitems, light_type, spot tables
    size_t o_frames = 0, o_objs = 0, o_vitems = 0, o_titems = 0, o_fitems = 0, o_light_type = 0;
    // spot lights (type 2) with shadow maps: one N x N depth frame per spot light, from
    // its shadow camera, rendered by a sub-layout before the frames themselves
    int64_t n_spot = 0;
    int32_t shadow_res = 0;
    std::vector<int32_t> spot_slot;   // per light: its shadow-map slot, -1 for other lights
    std::vector<int32_t> spot_light;  // per slot: the light
    std::vector<int32_t> spot_scene;  // per slot: the light's scene
    size_t o_spot_slot = 0, o_spot_light = 0;
    orrb_layout *shadow = nullptr;
    orrb_tuning tuning{32, 32, 256, 0, 0};
    // shading adjoint: every frame on the tiled-path vertex tables, gradient tiles
    std::vector<FrameInfo> frames_all;
    std::vector<int2> vitems_all, gitems;
    std::vector<int64_t> gitem_pbase;
    std::vector<int32_t> frame_item_begin, scene_frame_begin, scene_frames, obj_scene, obj_local, light_scene,
        light_local, scene_obj_begin, scene_light_begin;
    int max_scene_params = 0;
    uint64_t signature = 0;  // hash of the batch structure (autotuner cache key)
    uint64_t generation = 0; // bumped whenever the tuning or the device tables change
    int64_t grad_partials = 0;
    int max_scene_objects = 0;
    bool grad_ready = false;  // tables uploaded on the first backward call
    Packed gtab;
    size_t g_frames_all = 0, g_vitems_all = 0, g_gitems = 0, g_gitem_pbase = 0, g_frame_item_begin = 0,
           g_scene_frame_begin = 0, g_scene_frames = 0, g_obj_scene = 0, g_obj_local = 0, g_light_scene = 0,
           g_light_local = 0, g_scene_obj_begin = 0, g_scene_light_begin = 0;
};

// --------------------------------------------------------------------------------------
// workspace
// --------------------------------------------------------------------------------------

static size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

struct WsLayout {
    size_t vtx_pos, obj_rot, obj_bbox, queue, fscratch, total;
    size_t fs_stride;
    int64_t fs_verts, fs_surv, fs_bins;
};

// Global scratch of the frame kernel for frames whose scene data do not fit in LDS:
// one slice per workgroup (grid = min(frames, CUs)) with the largest such scene's
// snapped vertices (16 B each: X, Y, 1/w and padding, one load), a survivor entry per
// triangle (4 B) and
// bin_cap / 128 16-bit bin entries per triangle (at least 4096).
struct FrameScratch {
    int64_t grid = 0, verts = 0, surv = 0, bins = 0;
    size_t stride = 0;
};
static FrameScratch frame_scratch(int64_t gframes, int64_t frame_kernel_frames, int64_t verts, int64_t tris, int bin_cap,
                                  int n_cu) {
    FrameScratch f;
    if (gframes <= 0) return f;
    f.grid = std::min<int64_t>(frame_kernel_frames, n_cu);  // the frame kernel's grid: any workgroup may take such a frame
    f.verts = verts;
    f.surv = tris;
    f.bins = std::max<int64_t>(4096, (bin_cap / 128) * tris);
    f.stride = al256(16 * (size_t)verts) + al256(4 * (size_t)f.surv) + al256(2 * (size_t)f.bins);
    return f;
}

static WsLayout ws_layout(int64_t vertex_instances, int64_t object_instances, const FrameScratch &fs = FrameScratch()) {
    WsLayout w;
    size_t off = 0;
    w.vtx_pos = off;
    off = al256(off + sizeof(int4) * (size_t)vertex_instances);
    w.obj_rot = off;
    off = al256(off + 3 * sizeof(float4) * (size_t)object_instances);
    w.obj_bbox = off;
    off = al256(off + sizeof(int4) * (size_t)object_instances);
    w.queue = off;
    off = al256(off + 64);
    w.fscratch = off;
    w.fs_stride = fs.stride;
    w.fs_verts = fs.verts;
    w.fs_surv = fs.surv;
    w.fs_bins = fs.bins;
    off += fs.stride * (size_t)fs.grid;
    w.total = off;
    return w;
}

static bool valid_tuning(const orrb_tuning &t) {
    auto ok_dim = [](int d) { return d == 16 || d == 32 || d == 64; };
    if (!ok_dim(t.tile_w) || !ok_dim(t.tile_h)) return false;
    if (t.tile_w * t.tile_h > 4096) return false;
    if (t.bin_cap != 256 && t.bin_cap != 512 && t.bin_cap != 1024) return false;
    if (t.persistent != 0 && t.persistent != 1) return false;
    if (t.path < 0 || t.path > 2) return false;
    return raster_lds_bytes(t.tile_w, t.tile_h, t.bin_cap) <= 160 * 1024;
}

// Schedule of the frame kernel's persistent grid (min(frames, CUs) workgroups).  A
// uniform batch keeps the plain frame order and a static assignment: workgroup b
// renders fitems[b], fitems[b + grid], ...  An uneven batch is sorted by estimated work,
// heaviest first, and handed out at run time: workgroup b starts with fitems[b] and each
// workgroup takes the next unclaimed frame from a counter as it finishes one, so the
// workgroups end within about one light frame of each other whatever the estimate's
// error.  Estimated work: triangles (half again when the scene data live in global
// scratch) plus a quarter per pixel.
static void schedule_frames(orrb_layout *L) {
    const int64_t n = (int64_t)L->fitems.size();
    L->f_frames = n;
    L->f_grid = (int32_t)std::min<int64_t>(n, L->ctx ? L->ctx->n_cu : 256);
    L->f_dynamic = 0;
    if (n == 0) return;
    std::vector<double> cost(n);
    bool uniform = true;
    for (int64_t k = 0; k < n; ++k) {
        const FrameInfo &fi = L->frames[L->fitems[k]];
        cost[k] = (double)L->scene_tris[fi.scene] * (fi.mode ? 1.5 : 1.0) + 0.25 * (double)fi.width * fi.height;
        uniform = uniform && cost[k] == cost[0];
    }
    if (uniform || n <= L->f_grid) return;
    std::vector<int64_t> order(n);
    for (int64_t k = 0; k < n; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return cost[x] > cost[y]; });
    std::vector<int32_t> sorted(n);
    for (int64_t k = 0; k < n; ++k) sorted[k] = L->fitems[order[k]];
    L->fitems.swap(sorted);
    L->f_dynamic = 1;
}

// Kernel launches of one render call: the shadow frames' (camera gather + their own),
// vertex + raster for the tiled path, the frame kernel (after a counter clear when its
// frames are claimed at run time).
static int64_t render_kernels(const orrb_layout *L) {
    if (L->n_frames == 0) return 0;
    int64_t n = L->shadow ? 1 + render_kernels(L->shadow) : 0;
    if (!L->titems.empty()) n += 2;
    if (!L->fitems.empty()) n += 1 + L->f_dynamic;
    return n;
}

static WsLayout ws_layout(const orrb_layout *L) {
    const FrameScratch fs =
        frame_scratch(L->gframes, L->f_frames, L->gf_verts, L->gf_tris, L->tuning.bin_cap,
                      L->ctx ? L->ctx->n_cu : 256);
    return ws_layout(L->tiled_vertex_instances, L->tiled_object_instances, fs);
}

// Workspace enough for every valid tuning: every frame on the tiled path, plus the
// frame scratch of path 2 at the largest bin capacity.
static size_t ws_bytes_any(const orrb_layout *L) {
    int64_t g = 0, v = 0, t = 0, nf = 0;
    for (int64_t f = 0; f < L->n_frames; ++f) {
        nf += L->fits[f] != 0;
        if (L->fits[f] == 2) {
            ++g;
            v = std::max<int64_t>(v, L->scene_verts[L->frames[f].scene]);
            t = std::max<int64_t>(t, L->scene_tris[L->frames[f].scene]);
        }
    }
    const FrameScratch fs = frame_scratch(g, nf, v, t, 1024, L->ctx ? L->ctx->n_cu : 256);
    return ws_layout(L->all_vertex_instances, L->all_object_instances).total + fs.stride * (size_t)fs.grid + 256;
}

// Workspace of one render call: the frames' own, then (with spot lights) the shadow
// frames' (rendered first, on the same stream), the shadow maps (N x N fp32 per spot
// light) and the gathered shadow cameras (view 12, intrinsics 4, near 1 floats each).
struct CallWs {
    WsLayout w;
    size_t shadow_ws = 0, shadow_ws_bytes = 0, maps = 0, cams = 0, total = 0;
};

static CallWs call_ws(const orrb_layout *L, size_t shadow_ws_bytes) {
    CallWs c;
    c.w = ws_layout(L);
    c.total = c.w.total;
    if (L->shadow) {
        c.shadow_ws = al256(c.total);
        c.shadow_ws_bytes = shadow_ws_bytes;
        c.maps = al256(c.shadow_ws + shadow_ws_bytes);
        c.cams = al256(c.maps + sizeof(float) * (size_t)L->n_spot * L->shadow_res * L->shadow_res);
        c.total = c.cams + sizeof(float) * 17 * (size_t)L->n_spot;
    }
    return c;
}
static CallWs call_ws(const orrb_layout *L) { return call_ws(L, L->shadow ? ws_layout(L->shadow).total : 0); }

// Split frames between the frame kernel and the tiled path and build the work items.
// Path 0: the frame kernel takes frames whose scene fits in LDS; path 1: every frame
// on the tiled path; path 2: the frame kernel also takes larger scenes (up to 65,536
// vertices, 127 objects, 65,535 triangles, 256 x 256 pixels) with their data in global
// scratch, so an uneven batch of such frames is one launch.
static void build_items(orrb_layout *L) {
    L->titems.clear();
    L->vitems.clear();
    L->fitems.clear();
    const int TW = L->tuning.tile_w, TH = L->tuning.tile_h;
    int64_t vi = 0, oi = 0;
    L->gframes = L->gf_verts = L->gf_tris = 0;
    for (int64_t f = 0; f < L->n_frames; ++f) {
        FrameInfo &fi = L->frames[f];
        fi.tiles_x = (fi.width + TW - 1) / TW;
        fi.mode = 0;
        const int path = L->tuning.path;
        if ((path == 0 || path == 2) && L->fits[f] == 1) {
            L->fitems.push_back((int32_t)f);
            fi.vbase = 0;
            fi.oi_base = 0;
            continue;
        }
        if (path == 2 && L->fits[f] == 2) {
            L->fitems.push_back((int32_t)f);
            fi.vbase = 0;
            fi.oi_base = 0;
            fi.mode = 1;
            L->gframes++;
            L->gf_verts = std::max<int64_t>(L->gf_verts, L->scene_verts[fi.scene]);
            L->gf_tris = std::max<int64_t>(L->gf_tris, L->scene_tris[fi.scene]);
            continue;
        }
        fi.vbase = vi;
        fi.oi_base = (int32_t)oi;
        for (int k = 0; k < fi.n_obj; ++k) L->vitems.push_back(make_int2((int)f, k));
        vi += L->scene_verts[fi.scene];
        oi += fi.n_obj;
        const int ty = (fi.height + TH - 1) / TH;
        for (int t = 0; t < fi.tiles_x * ty; ++t) L->titems.push_back(make_int2((int)f, t));
    }
    L->tiled_vertex_instances = vi;
    L->tiled_object_instances = oi;
    schedule_frames(L);
}

// Tables of the shading adjoint (independent of the tuning).
static void build_grad_tables(orrb_layout *L, const orrb_layout_desc *d) {
    const int S = (int)L->n_scenes, F = (int)L->n_frames;
    L->frames_all = L->frames;
    int64_t vi = 0, oi = 0;
    for (int f = 0; f < F; ++f) {
        FrameInfo &fi = L->frames_all[f];
        fi.vbase = vi;
        fi.oi_base = (int32_t)oi;
        for (int k = 0; k < fi.n_obj; ++k) L->vitems_all.push_back(make_int2(f, k));
        vi += L->scene_verts[fi.scene];
        oi += fi.n_obj;
    }
    const int G = grad_tile_size();
    int64_t pb = 0;
    L->frame_item_begin.assign(F + 1, 0);
    for (int f = 0; f < F; ++f) {
        const FrameInfo &fi = L->frames_all[f];
        const int nt = ((fi.width + G - 1) / G) * ((fi.height + G - 1) / G);
        L->frame_item_begin[f] = (int32_t)L->gitems.size();
        for (int t = 0; t < nt; ++t) {
            L->gitems.push_back(make_int2(f, t));
            L->gitem_pbase.push_back(pb);
            pb += 5 * (int64_t)fi.n_obj + 4 * (int64_t)fi.n_lights + 1;
        }
    }
    L->frame_item_begin[F] = (int32_t)L->gitems.size();
    L->grad_partials = pb;
    L->scene_frame_begin.assign(S + 1, 0);
    for (int f = 0; f < F; ++f) L->scene_frame_begin[d->frame_scene[f] + 1]++;
    for (int s = 0; s < S; ++s) L->scene_frame_begin[s + 1] += L->scene_frame_begin[s];
    L->scene_frames.assign(F, 0);
    std::vector<int32_t> cur(L->scene_frame_begin.begin(), L->scene_frame_begin.end() - 1);
    for (int f = 0; f < F; ++f) L->scene_frames[cur[d->frame_scene[f]]++] = f;
    L->obj_scene.resize(L->n_objects);
    L->obj_local.resize(L->n_objects);
    L->light_scene.resize(L->n_lights);
    L->light_local.resize(L->n_lights);
    for (int s = 0; s < S; ++s) {
        for (int o = d->scene_object_begin[s]; o < d->scene_object_begin[s + 1]; ++o) {
            L->obj_scene[o] = s;
            L->obj_local[o] = o - d->scene_object_begin[s];
        }
        for (int l = d->scene_light_begin[s]; l < d->scene_light_begin[s + 1]; ++l) {
            L->light_scene[l] = s;
            L->light_local[l] = l - d->scene_light_begin[s];
        }
        L->max_scene_objects = std::max(L->max_scene_objects, d->scene_object_begin[s + 1] - d->scene_object_begin[s]);
    }
    L->scene_obj_begin.assign(d->scene_object_begin, d->scene_object_begin + S + 1);
    L->scene_light_begin.assign(d->scene_light_begin, d->scene_light_begin + S + 1);
    for (int s = 0; s < S; ++s)
        L->max_scene_params = std::max(L->max_scene_params,
                                       5 * (d->scene_object_begin[s + 1] - d->scene_object_begin[s]) +
                                           4 * (d->scene_light_begin[s + 1] - d->scene_light_begin[s]) +
                                           (L->scene_frame_begin[s + 1] - L->scene_frame_begin[s]));
}

static orrb_status upload_grad_tables(orrb_layout *L) {
    ScopedDevice sd(L->ctx->device);
    Packed &P = L->gtab;
    P.clear();
    L->g_frames_all = P.add(L->frames_all);
    L->g_vitems_all = P.add(L->vitems_all);
    L->g_gitems = P.add(L->gitems);
    L->g_gitem_pbase = P.add(L->gitem_pbase);
    L->g_frame_item_begin = P.add(L->frame_item_begin);
    L->g_scene_frame_begin = P.add(L->scene_frame_begin);
    L->g_scene_frames = P.add(L->scene_frames);
    L->g_obj_scene = P.add(L->obj_scene);
    L->g_obj_local = P.add(L->obj_local);
    L->g_light_scene = P.add(L->light_scene);
    L->g_light_local = P.add(L->light_local);
    L->g_scene_obj_begin = P.add(L->scene_obj_begin);
    L->g_scene_light_begin = P.add(L->scene_light_begin);
    HIP_TRY(P.upload());
    L->grad_ready = true;
    return ORRB_OK;
}

static size_t grad_workspace(const orrb_layout *L) {
    return al256(ws_layout(L->all_vertex_instances, L->all_object_instances).total) +
           al256(sizeof(double) * (size_t)L->grad_partials);
}

static orrb_status upload_layout(orrb_layout *L) {
    ScopedDevice sd(L->ctx->device);
    Packed &P = L->tab;
    P.clear();
    L->o_frames = P.add(L->frames);
    L->o_objs = P.add(L->objs);
    L->o_vitems = P.add(L->vitems);
    L->o_titems = P.add(L->titems);
    L->o_fitems = P.add(L->fitems);
    L->o_light_type = P.add(L->light_type);
    if (L->n_spot > 0) {
        L->o_spot_slot = P.add(L->spot_slot);
        L->o_spot_light = P.add(L->spot_light);
    }
    HIP_TRY(P.upload());
    return ORRB_OK;
}

namespace orrb {
orrb_status set_error(orrb_status st, const char *msg) {
    g_last_error = msg;
    return st;
}
uint64_t layout_signature(const orrb_layout *L) { return L->signature; }
uint64_t layout_generation(const orrb_layout *L) { return L->generation; }
uint64_t context_generation(const orrb_context *ctx) { return ctx->generation; }
int context_device(const orrb_context *ctx) { return ctx->device; }
bool context_profiling(const orrb_context *ctx) { return ctx->timer.enabled; }
void context_set_profiling(orrb_context *ctx, bool on) { ctx->timer.enabled = on; }
}  // namespace orrb

// --------------------------------------------------------------------------------------
// C ABI
// --------------------------------------------------------------------------------------

static void fill_args(const orrb_context *ctx, const orrb_layout *L, const orrb_scenes *sc, const orrb_cameras *cam,
                      const orrb_params *par, RenderArgs *a) {
    memset(a, 0, sizeof(*a));
    a->objs = L->tab.at<ObjInfo>(L->o_objs);
    a->light_type = L->tab.at<int32_t>(L->o_light_type);
    a->mesh_pos = (const float4 *)ctx->d_pos.p;
    a->mesh_nrm = (const float4 *)ctx->d_nrm.p;
    a->mesh_tri = (const int4 *)ctx->d_tri.p;
    a->mesh_uv = (const float2 *)ctx->d_uv.p;
    a->tex_texels = (const float4 *)ctx->d_texels.p;
    a->tex_info = (const int4 *)ctx->d_tex_info.p;
    a->n_tex = (int32_t)ctx->tex_info.size();
    a->obj_tex = par->texture;
    a->tex_xform = par->tex_xform;
    a->emission = par->emission;
    a->obj_ntex = par->normal_texture;
    a->pose = sc->object_pose;
    a->seg = sc->object_seg;
    a->visible = sc->object_visible;
    a->view = cam->view;
    a->intr = cam->intr;
    a->near_plane = cam->near_plane;
    a->albedo = par->albedo;
    a->roughness = par->roughness;
    a->specular = par->specular;
    a->light_vec = par->light_vec;
    a->light_intensity = par->light_intensity;
    a->exposure = par->exposure;
}

static orrb_status check_inputs(const orrb_layout *L, const orrb_scenes *sc, const orrb_cameras *cam,
                                const orrb_params *par) {
    if (L->n_objects > 0 && (!sc->object_pose || !sc->object_seg || !sc->object_visible || !par->albedo ||
                             !par->roughness || !par->specular))
        return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL object array");
    if (L->n_lights > 0 && (!par->light_vec || !par->light_intensity))
        return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL light array");
    if (!cam->view || !cam->intr || !cam->near_plane || !par->exposure)
        return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL camera array");
    return ORRB_OK;
}

extern "C" {

const char *orrb_last_error(void) { return g_last_error.c_str(); }

orrb_status orrb_create(int hip_device, orrb_context **out) {
    g_last_error.clear();
    if (!out) return fail(ORRB_ERR_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (hip_device < 0 || hip_device >= n)
        return fail(ORRB_ERR_INVALID_ARGUMENT, "device %d out of range [0, %d)", hip_device, n);
    ScopedDevice sd(hip_device);
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, hip_device));
    auto *c = new (std::nothrow) orrb_context();
    if (!c) return fail(ORRB_ERR_OUT_OF_MEMORY, "host allocation failed");
    c->device = hip_device;
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if (const char *v = getenv("ORRB_TILE")) {
        int w = 0, h = 0;
        char x = 0;
        if (sscanf(v, "%d%c%d", &w, &x, &h) != 3 || (x != 'x' && x != 'X')) {
            delete c;
            return fail(ORRB_ERR_INVALID_ARGUMENT, "ORRB_TILE=%s: expected WxH", v);
        }
        c->default_tuning.tile_w = w;
        c->default_tuning.tile_h = h;
    }
    if (const char *v = getenv("ORRB_BIN_CAP")) {
        char *end = nullptr;
        const long n = strtol(v, &end, 10);
        if (end == v || *end != 0) {
            delete c;
            return fail(ORRB_ERR_INVALID_ARGUMENT, "ORRB_BIN_CAP=%s: expected an integer", v);
        }
        c->default_tuning.bin_cap = (int)n;
    }
    if (!valid_tuning(c->default_tuning)) {
        const orrb_tuning &t = c->default_tuning;
        delete c;
        return fail(ORRB_ERR_INVALID_ARGUMENT, "ORRB_TILE / ORRB_BIN_CAP give no valid tuning (tile %dx%d, cap %d)",
                    t.tile_w, t.tile_h, t.bin_cap);
    }
    if (const char *v = getenv("ORRB_DEBUG_VALIDATE")) c->debug_validate = *v && strcmp(v, "0") != 0;
    {
        // the device's copy of the fixed scratch array (orrb_render_batch_noalloc)
        const hipError_t e = scratch_init(hip_device);
        if (e != hipSuccess) {
            delete c;
            return fail(ORRB_ERR_DEVICE, "scratch set-up on device %d failed: %s", hip_device, hipGetErrorString(e));
        }
    }
    *out = c;
    return ORRB_OK;
}

void orrb_destroy(orrb_context *ctx) {
    if (!ctx) return;
    if (ctx->n_layouts > 0) {  // layouts still point into the pool: free it with the last of them
        ctx->destroy_pending = true;
        return;
    }
    ScopedDevice sd(ctx->device);
    delete ctx;
}

orrb_status orrb_add_mesh(orrb_context *ctx, const float *pos, const float *nrm, int32_t n_verts, const int32_t *idx,
                          int32_t n_tris, int32_t *mesh_id) {
    g_last_error.clear();
    if (!ctx || !pos || !nrm || !idx || !mesh_id) return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL argument");
    if (n_verts < 1 || n_verts > (1 << 30)) return fail(ORRB_ERR_INVALID_ARGUMENT, "n_verts %d out of range", n_verts);
    if (n_tris < 1 || n_tris > (1 << 26)) return fail(ORRB_ERR_INVALID_ARGUMENT, "n_tris %d out of range", n_tris);
    if ((int64_t)ctx->pos.size() + n_verts > 0x7fffffff || (int64_t)ctx->tri.size() + n_tris > 0x7fffffff)
        return fail(ORRB_ERR_UNSUPPORTED, "mesh pool would exceed 2^31 entries");
    for (int64_t k = 0; k < 3 * (int64_t)n_verts; ++k) {
        if (!std::isfinite(pos[k]) || !std::isfinite(nrm[k]))
            return fail(ORRB_ERR_INVALID_ARGUMENT, "non-finite position or normal at vertex %lld", (long long)(k / 3));
    }
    for (int64_t v = 0; v < n_verts; ++v) {
        const float *n = nrm + 3 * v;
        if (n[0] == 0.f && n[1] == 0.f && n[2] == 0.f)
            return fail(ORRB_ERR_INVALID_ARGUMENT, "zero normal at vertex %lld", (long long)v);
    }
    for (int64_t k = 0; k < 3 * (int64_t)n_tris; ++k) {
        if (idx[k] < 0 || idx[k] >= n_verts)
            return fail(ORRB_ERR_INVALID_ARGUMENT, "index %d of triangle %lld out of range", idx[k], (long long)(k / 3));
    }
    const size_t v0 = ctx->pos.size(), t0 = ctx->tri.size();
    for (int64_t v = 0; v < n_verts; ++v) {
        ctx->pos.push_back(make_float4(pos[3 * v], pos[3 * v + 1], pos[3 * v + 2], 0.f));
        // stored unit length: shading interpolates object-space normals, then rotates
        const double nx = nrm[3 * v], ny = nrm[3 * v + 1], nz = nrm[3 * v + 2];
        const double inv = 1.0 / std::sqrt(nx * nx + ny * ny + nz * nz);
        ctx->nrm.push_back(make_float4((float)(nx * inv), (float)(ny * inv), (float)(nz * inv), 0.f));
    }
    for (int64_t t = 0; t < n_tris; ++t) ctx->tri.push_back(make_int4(idx[3 * t], idx[3 * t + 1], idx[3 * t + 2], 0));
    ctx->uv.resize(ctx->pos.size(), make_float2(0.f, 0.f));
    ScopedDevice sd(ctx->device);
    hipError_t e = ctx->d_pos.upload(ctx->pos.data(), sizeof(float4) * ctx->pos.size());
    if (e == hipSuccess) e = ctx->d_nrm.upload(ctx->nrm.data(), sizeof(float4) * ctx->nrm.size());
    if (e == hipSuccess) e = ctx->d_tri.upload(ctx->tri.data(), sizeof(int4) * ctx->tri.size());
    if (e == hipSuccess) e = ctx->d_uv.upload(ctx->uv.data(), sizeof(float2) * ctx->uv.size());
    if (e != hipSuccess) {
        ctx->pos.resize(v0);
        ctx->nrm.resize(v0);
        ctx->tri.resize(t0);
        ctx->uv.resize(v0);
        return fail(e == hipErrorOutOfMemory ? ORRB_ERR_OUT_OF_MEMORY : ORRB_ERR_DEVICE, "mesh upload failed: %s",
                    hipGetErrorString(e));
    }
    ctx->generation++;
    ctx->mesh_vbegin.push_back((int32_t)ctx->pos.size());
    ctx->mesh_tbegin.push_back((int32_t)ctx->tri.size());
    *mesh_id = (int32_t)ctx->mesh_vbegin.size() - 2;
    return ORRB_OK;
}

orrb_status orrb_set_mesh_uv(orrb_context *ctx, int32_t mesh_id, const float *uv) {
    g_last_error.clear();
    if (!ctx || !uv) return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL argument");
    const int n_meshes = (int)ctx->mesh_vbegin.size() - 1;
    if (mesh_id < 0 || mesh_id >= n_meshes) return fail(ORRB_ERR_INVALID_ARGUMENT, "unknown mesh %d", mesh_id);
    const int32_t v0 = ctx->mesh_vbegin[mesh_id], nv = ctx->mesh_vbegin[mesh_id + 1] - v0;
    for (int64_t k = 0; k < 2 * (int64_t)nv; ++k)
        if (!std::isfinite(uv[k])) return fail(ORRB_ERR_INVALID_ARGUMENT, "non-finite uv at vertex %lld", (long long)(k / 2));
    std::vector<float2> old(ctx->uv.begin() + v0, ctx->uv.begin() + v0 + nv);
    for (int32_t v = 0; v < nv; ++v) ctx->uv[v0 + v] = make_float2(uv[2 * v], uv[2 * v + 1]);
    ScopedDevice sd(ctx->device);
    const hipError_t e = ctx->d_uv.upload(ctx->uv.data(), sizeof(float2) * ctx->uv.size());
    if (e != hipSuccess) {
        std::copy(old.begin(), old.end(), ctx->uv.begin() + v0);
        return fail(e == hipErrorOutOfMemory ? ORRB_ERR_OUT_OF_MEMORY : ORRB_ERR_DEVICE, "uv upload failed: %s",
                    hipGetErrorString(e));
    }
    ctx->generation++;
    return ORRB_OK;
}

orrb_status orrb_add_texture(orrb_context *ctx, const float *rgb, int32_t width, int32_t height, int32_t *tex_id) {
    g_last_error.clear();
    if (!ctx || !rgb || !tex_id) return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL argument");
    if (width < 1 || height < 1 || width > ORRB_MAX_DIM || height > ORRB_MAX_DIM)
        return fail(ORRB_ERR_INVALID_ARGUMENT, "texture size %dx%d out of range", width, height);
    const int64_t n = (int64_t)width * height;
    if ((int64_t)ctx->texels.size() + n > 0x7fffffff) return fail(ORRB_ERR_UNSUPPORTED, "texture pool would exceed 2^31 texels");
    for (int64_t k = 0; k < 3 * n; ++k)
        if (!std::isfinite(rgb[k])) return fail(ORRB_ERR_INVALID_ARGUMENT, "non-finite texel value at %lld", (long long)(k / 3));
    const size_t t0 = ctx->texels.size();
    for (int64_t k = 0; k < n; ++k) ctx->texels.push_back(make_float4(rgb[3 * k], rgb[3 * k + 1], rgb[3 * k + 2], 0.f));
    ctx->tex_info.push_back(make_int4((int)t0, width, height, 0));
    ScopedDevice sd(ctx->device);
    hipError_t e = ctx->d_texels.upload(ctx->texels.data(), sizeof(float4) * ctx->texels.size());
    if (e == hipSuccess) e = ctx->d_tex_info.upload(ctx->tex_info.data(), sizeof(int4) * ctx->tex_info.size());
    if (e != hipSuccess) {
        ctx->texels.resize(t0);
        ctx->tex_info.pop_back();
        return fail(e == hipErrorOutOfMemory ? ORRB_ERR_OUT_OF_MEMORY : ORRB_ERR_DEVICE, "texture upload failed: %s",
                    hipGetErrorString(e));
    }
    ctx->generation++;
    *tex_id = (int32_t)ctx->tex_info.size() - 1;
    return ORRB_OK;
}

orrb_status orrb_layout_create(orrb_context *ctx, const orrb_layout_desc *d, orrb_layout **out) {
    g_last_error.clear();
    if (!ctx || !d || !out) return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL argument");
    *out = nullptr;
    if (d->n_scenes < 0 || d->n_frames < 0) return fail(ORRB_ERR_INVALID_ARGUMENT, "negative scene or frame count");
    if (d->n_scenes > 0 && (!d->scene_object_begin || !d->scene_light_begin))
        return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL scene arrays");
    if (d->n_frames > 0 && (!d->frame_scene || !d->width || !d->height))
        return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL frame arrays");
    const int S = d->n_scenes;
    if (S > 0 && (d->scene_object_begin[0] != 0 || d->scene_light_begin[0] != 0))
        return fail(ORRB_ERR_INVALID_ARGUMENT, "scene offsets must start at 0");
    for (int s = 0; s < S; ++s) {
        if (d->scene_object_begin[s + 1] < d->scene_object_begin[s])
            return fail(ORRB_ERR_INVALID_ARGUMENT, "scene_object_begin decreases at scene %d", s);
        const int nl = d->scene_light_begin[s + 1] - d->scene_light_begin[s];
        if (nl < 0) return fail(ORRB_ERR_INVALID_ARGUMENT, "scene_light_begin decreases at scene %d", s);
        if (nl > ORRB_MAX_LIGHTS_PER_SCENE)
            return fail(ORRB_ERR_UNSUPPORTED, "scene %d has %d lights (max %d)", s, nl, ORRB_MAX_LIGHTS_PER_SCENE);
    }
    const int64_t O = S > 0 ? d->scene_object_begin[S] : 0, NL = S > 0 ? d->scene_light_begin[S] : 0;
    if (O > 0 && !d->object_mesh) return fail(ORRB_ERR_INVALID_ARGUMENT, "object_mesh is NULL");
    if (NL > 0 && !d->light_type) return fail(ORRB_ERR_INVALID_ARGUMENT, "light_type is NULL");
    const int n_meshes = (int)ctx->mesh_vbegin.size() - 1;
    for (int64_t o = 0; o < O; ++o)
        if (d->object_mesh[o] < 0 || d->object_mesh[o] >= n_meshes)
            return fail(ORRB_ERR_INVALID_ARGUMENT, "object %lld uses unknown mesh %d", (long long)o, d->object_mesh[o]);
    int64_t n_spot = 0;
    for (int64_t l = 0; l < NL; ++l) {
        if (d->light_type[l] < 0 || d->light_type[l] > 2)
            return fail(ORRB_ERR_INVALID_ARGUMENT, "light %lld has type %d (0 point, 1 directional, 2 spot)",
                        (long long)l, d->light_type[l]);
        n_spot += d->light_type[l] == 2;
    }
    if (n_spot > 0) {
        if (d->shadow_res < 8 || d->shadow_res > 256)
            return fail(ORRB_ERR_INVALID_ARGUMENT, "shadow_res %d out of [8, 256] with spot lights", d->shadow_res);
        for (int s = 0; s < S; ++s) {
            int k = 0;
            for (int l = d->scene_light_begin[s]; l < d->scene_light_begin[s + 1]; ++l) k += d->light_type[l] == 2;
            if (k > ORRB_MAX_SPOT_LIGHTS_PER_SCENE)
                return fail(ORRB_ERR_UNSUPPORTED, "scene %d has %d spot lights (max %d)", s, k,
                            ORRB_MAX_SPOT_LIGHTS_PER_SCENE);
        }
    }
    for (int f = 0; f < d->n_frames; ++f) {
        if (d->frame_scene[f] < 0 || d->frame_scene[f] >= S)
            return fail(ORRB_ERR_INVALID_ARGUMENT, "frame %d refers to scene %d of %d", f, d->frame_scene[f], S);
        if (d->width[f] < 1 || d->width[f] > ORRB_MAX_DIM || d->height[f] < 1 || d->height[f] > ORRB_MAX_DIM)
            return fail(ORRB_ERR_INVALID_ARGUMENT, "frame %d size %dx%d out of range", f, d->width[f], d->height[f]);
    }
    auto *L = new (std::nothrow) orrb_layout();
    if (!L) return fail(ORRB_ERR_OUT_OF_MEMORY, "host allocation failed");
    L->ctx = ctx;
    L->tuning = ctx->default_tuning;
    L->n_scenes = S;
    L->n_objects = O;
    L->n_lights = NL;
    L->n_frames = d->n_frames;
    // objects: mesh ranges and scene-local vertex / triangle bases
    L->scene_verts.assign(S, 0);
    L->scene_tris.assign(S, 0);
    L->objs.resize(O);
    for (int s = 0; s < S; ++s) {
        int64_t vb = 0, tb = 0;
        for (int o = d->scene_object_begin[s]; o < d->scene_object_begin[s + 1]; ++o) {
            const int m = d->object_mesh[o];
            ObjInfo &ob = L->objs[o];
            ob.mesh_vbegin = ctx->mesh_vbegin[m];
            ob.n_verts = ctx->mesh_vbegin[m + 1] - ctx->mesh_vbegin[m];
            ob.mesh_tbegin = ctx->mesh_tbegin[m];
            ob.n_tris = ctx->mesh_tbegin[m + 1] - ctx->mesh_tbegin[m];
            ob.scene_vbase = (int32_t)vb;
            ob.scene_tbase = (int32_t)tb;
            vb += ob.n_verts;
            tb += ob.n_tris;
            if (vb > 0x7fffffff || tb > ORRB_MAX_SCENE_TRIANGLES) {
                delete L;
                return fail(ORRB_ERR_UNSUPPORTED, "scene %d exceeds the vertex or triangle limit", s);
            }
        }
        L->scene_verts[s] = vb;
        L->scene_tris[s] = tb;
    }
    L->light_type.assign(d->light_type, d->light_type + NL);
    if (n_spot > 0) {
        L->n_spot = n_spot;
        L->shadow_res = d->shadow_res;
        L->spot_slot.assign(NL, -1);
        std::vector<int32_t> frame_scene;
        for (int s = 0; s < S; ++s)
            for (int l = d->scene_light_begin[s]; l < d->scene_light_begin[s + 1]; ++l)
                if (d->light_type[l] == 2) {
                    L->spot_slot[l] = (int32_t)L->spot_light.size();
                    L->spot_light.push_back(l);
                    frame_scene.push_back(s);
                }
        L->spot_scene.swap(frame_scene);
    }
    L->frames.resize(d->n_frames);
    L->fits.resize(d->n_frames);
    int64_t pix = 0, vi = 0, oi = 0, ti = 0;
    for (int f = 0; f < d->n_frames; ++f) {
        const int s = d->frame_scene[f];
        FrameInfo &fi = L->frames[f];
        fi.pixel_offset = pix;
        fi.vbase = 0;
        fi.scene = s;
        fi.width = d->width[f];
        fi.height = d->height[f];
        fi.tiles_x = 0;
        fi.obj_begin = d->scene_object_begin[s];
        fi.n_obj = d->scene_object_begin[s + 1] - d->scene_object_begin[s];
        fi.oi_base = 0;
        fi.light_begin = d->scene_light_begin[s];
        fi.n_lights = d->scene_light_begin[s + 1] - d->scene_light_begin[s];
        fi.track_base = (int32_t)oi;
        L->fits[f] = frame_fits((int)std::min<int64_t>(L->scene_verts[s], 0x7fffffff), fi.n_obj,
                                (int)std::min<int64_t>(L->scene_tris[s], 0x7fffffff), fi.width, fi.height)
                         ? 1
                     : frame_fits_global(L->scene_verts[s], fi.n_obj, L->scene_tris[s], fi.width, fi.height) ? 2
                                                                                                              : 0;
        fi.mode = 0;
        fi.pad0 = 0;
        pix += (int64_t)fi.width * fi.height;
        L->max_frame_pixels = std::max<int64_t>(L->max_frame_pixels, (int64_t)fi.width * fi.height);
        vi += L->scene_verts[s];
        ti += L->scene_tris[s];
        oi += fi.n_obj;
        if (oi > 0x7fffffff) {
            delete L;
            return fail(ORRB_ERR_UNSUPPORTED, "too many (frame, object) instances");
        }
    }
    L->total_pixels = pix;
    L->vertex_instances = vi;
    L->triangle_instances = ti;
    L->all_vertex_instances = vi;
    L->all_object_instances = oi;
    build_items(L);
    if ((int64_t)L->titems.size() > 0x7fffffff || (int64_t)L->vitems.size() > 0x7fffffff) {
        delete L;
        return fail(ORRB_ERR_UNSUPPORTED, "too many tiles");
    }
    build_grad_tables(L, d);
    {   // FNV-1a over the structure: frame sizes, scenes' mesh sizes and light counts
        uint64_t h = 1469598103934665603ull;
        auto mix = [&h](int64_t x) {
            for (int b = 0; b < 8; ++b) {
                h ^= (uint64_t)((x >> (8 * b)) & 0xff);
                h *= 1099511628211ull;
            }
        };
        mix(L->n_frames);
        for (const FrameInfo &fi : L->frames) {
            mix(fi.width);
            mix(fi.height);
            mix(fi.n_obj);
            mix(fi.n_lights);
            mix(L->scene_verts[fi.scene]);
            mix(L->scene_tris[fi.scene]);
        }
        L->signature = h;
    }
    orrb_status st = upload_layout(L);
    if (st != ORRB_OK) {
        delete L;
        return st;
    }
    if (L->n_spot > 0) {  // the shadow frames: the same scenes, no lights, one N x N frame per spot light
        std::vector<int32_t> no_lights(S + 1, 0), side(L->n_spot, d->shadow_res);
        orrb_layout_desc sd{};
        sd.n_scenes = S;
        sd.scene_object_begin = d->scene_object_begin;
        sd.object_mesh = d->object_mesh;
        sd.scene_light_begin = no_lights.data();
        sd.light_type = nullptr;
        sd.n_frames = (int32_t)L->n_spot;
        sd.frame_scene = L->spot_scene.data();
        sd.width = side.data();
        sd.height = side.data();
        sd.shadow_res = 0;
        st = orrb_layout_create(ctx, &sd, &L->shadow);
        if (st != ORRB_OK) {
            delete L;
            return st;
        }
    }
    ctx->n_layouts++;
    *out = L;
    return ORRB_OK;
}

void orrb_layout_destroy(orrb_layout *L) {
    if (!L) return;
    orrb_context *ctx = L->ctx;
    ScopedDevice sd(ctx->device);
    if (L->shadow) orrb_layout_destroy(L->shadow);
    ctx->n_layouts--;
    delete L;
    if (ctx->destroy_pending && ctx->n_layouts == 0) delete ctx;
}

orrb_status orrb_layout_info_get(const orrb_layout *L, orrb_layout_info *info) {
    g_last_error.clear();
    if (!L || !info) return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL argument");
    info->n_scenes = L->n_scenes;
    info->n_objects = L->n_objects;
    info->n_lights = L->n_lights;
    info->n_frames = L->n_frames;
    info->total_pixels = L->total_pixels;
    info->vertex_instances = L->vertex_instances;
    info->triangle_instances = L->triangle_instances;
    info->tile_items = (int64_t)L->titems.size();
    info->frame_path_frames = L->f_frames;
    info->workspace_bytes = call_ws(L).total;
    info->workspace_bytes_any = ws_bytes_any(L);
    if (L->shadow) info->workspace_bytes_any += call_ws(L, ws_bytes_any(L->shadow)).total - ws_layout(L).total + 256;
    info->grad_workspace_bytes = grad_workspace(L);
    info->table_bytes = L->tab.dev.bytes + L->gtab.dev.bytes;
    info->tuning = L->tuning;
    info->render_kernels = render_kernels(L);
    return ORRB_OK;
}

orrb_status orrb_layout_set_tuning(orrb_layout *L, const orrb_tuning *t) {
    g_last_error.clear();
    if (!L || !t) return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL argument");
    if (!valid_tuning(*t))
        return fail(ORRB_ERR_INVALID_ARGUMENT, "invalid tuning tile %dx%d cap %d persistent %d", t->tile_w, t->tile_h,
                    t->bin_cap, t->persistent);
    const bool rebuild = t->tile_w != L->tuning.tile_w || t->tile_h != L->tuning.tile_h || t->path != L->tuning.path;
    if (memcmp(t, &L->tuning, sizeof(*t)) != 0) L->generation++;  // captured graphs are now stale
    L->tuning = *t;
    if (L->shadow) {  // the shadow frames follow the same tuning
        const orrb_status st = orrb_layout_set_tuning(L->shadow, t);
        if (st != ORRB_OK) return st;
    }
    if (rebuild) {
        build_items(L);
        return upload_layout(L);
    }
    return ORRB_OK;
}

}  // extern "C"

size_t orrb::render_workspace_bytes(const orrb_layout *L) { return call_ws(L).total; }

// A render call: host checks, then the kernels on `stream`.  With `timing` false it
// records no kernel-timing events (and so creates none).
orrb_status orrb::render_impl(orrb_context *ctx, const orrb_layout *L, const orrb_scenes *sc, const orrb_cameras *cam,
                               const orrb_params *par, const orrb_outputs *out, void *workspace,
                               size_t workspace_bytes, void *stream, bool timing) {
    if (!ctx || !L || !sc || !cam || !par || !out) return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL handle or struct");
    if (L->ctx != ctx) return fail(ORRB_ERR_INVALID_ARGUMENT, "layout belongs to another context");
    if (L->n_frames == 0) return ORRB_OK;
    {
        const orrb_status st = check_inputs(L, sc, cam, par);
        if (st != ORRB_OK) return st;
    }
    const CallWs cw = call_ws(L);
    const WsLayout &w = cw.w;
    if (!workspace) return fail(ORRB_ERR_INVALID_ARGUMENT, "workspace is NULL");
    if (workspace_bytes < cw.total)
        return fail(ORRB_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu required", workspace_bytes, cw.total);
    if ((uintptr_t)workspace % 16 != 0) return fail(ORRB_ERR_INVALID_ARGUMENT, "workspace must be 16-byte aligned");
    if (L->shadow && (!par->light_dir || !par->light_cone || !par->shadow_view || !par->shadow_intr))
        return fail(ORRB_ERR_INVALID_ARGUMENT, "spot lights need light_dir, light_cone, shadow_view and shadow_intr");
    if (L->shadow) {
        // shadow frames first: gather each spot light's shadow camera, then render their
        // depth (no shading) into the shadow maps
        char *wsb = (char *)workspace;
        float *cview = (float *)(wsb + cw.cams), *cintr = cview + 12 * L->n_spot, *cnear = cintr + 4 * L->n_spot;
        ScopedDevice sd(ctx->device);
        hipError_t e = launch_shadow_cams(L->tab.at<int32_t>(L->o_spot_light), (int)L->n_spot, par->shadow_view,
                                          par->shadow_intr, cview, cintr, cnear, (hipStream_t)stream);
        if (e != hipSuccess) return fail(ORRB_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
        const orrb_cameras cs{cview, cintr, cnear};
        orrb_params ps = *par;
        ps.exposure = cnear;  // never read: depth only (any n_spot floats)
        ps.post = nullptr;
        ps.grain = nullptr;
        orrb_outputs os{};
        os.depth = (float *)(wsb + cw.maps);
        os.stats = out->stats;
        const orrb_status st = render_impl(ctx, L->shadow, sc, &cs, &ps, &os, wsb + cw.shadow_ws, cw.shadow_ws_bytes,
                                           stream, timing);
        if (st != ORRB_OK) return st;
    }
    RenderArgs a;
    fill_args(ctx, L, sc, cam, par, &a);
    a.frames = L->tab.at<FrameInfo>(L->o_frames);
    a.vitems = L->tab.at<int2>(L->o_vitems);
    a.titems = L->tab.at<int2>(L->o_titems);
    a.fitems = L->tab.at<int32_t>(L->o_fitems);
    a.n_fitems = (int32_t)L->fitems.size();
    a.f_grid = L->f_grid;
    a.f_dynamic = L->f_dynamic;
    a.n_vitems = (int32_t)L->vitems.size();
    a.n_titems = (int32_t)L->titems.size();
    a.tile_w = L->tuning.tile_w;
    a.tile_h = L->tuning.tile_h;
    a.bin_cap = L->tuning.bin_cap;
    a.persistent = L->tuning.persistent;
    a.out_rgb = out->rgb;
    a.out_depth = out->depth;
    a.out_normal = out->normal;
    a.out_seg = out->seg;
    a.out_tri = out->tri_id;
    a.out_vis = (unsigned long long *)out->vis;
    a.stats = out->stats;
    a.out_alpha = out->alpha;
    a.out_rgb8 = out->rgb8;
    a.out_track = out->track;
    a.post = par->post;
    a.grain = par->grain;
    a.grain_w = par->grain_w;
    a.grain_h = par->grain_h;
    // shading mode of the frame kernel: depth only when nothing shaded is written
    a.shade_mode = (!out->rgb && !out->normal && !out->rgb8) ? 4
                   : (L->shadow ? 1 : 0) | ((par->texture || par->emission || par->normal_texture) ? 2 : 0);
    if ((par->texture || par->normal_texture) && !par->tex_xform)
        return fail(ORRB_ERR_INVALID_ARGUMENT, "texture and normal_texture need tex_xform");
    if (L->shadow) {
        a.light_dir = par->light_dir;
        a.light_cone = par->light_cone;
        a.shadow_view = par->shadow_view;
        a.shadow_intr = par->shadow_intr;
        a.spot_slot = L->tab.at<int32_t>(L->o_spot_slot);
        a.shadow_maps = (const float *)((char *)workspace + cw.maps);
        a.shadow_res = L->shadow_res;
    }
    if (out->rgb8 && par->grain &&
        (par->grain_w < 1 || par->grain_h < 1 || (int64_t)par->grain_w * par->grain_h > (int64_t)1 << 26))
        return fail(ORRB_ERR_INVALID_ARGUMENT, "grain texture size %d x %d (1 .. 2^26 texels per plane)",
                    par->grain_w, par->grain_h);
    char *ws = (char *)workspace;
    a.vtx_pos = (int4 *)(ws + w.vtx_pos);
    a.obj_rot = (float4 *)(ws + w.obj_rot);
    a.obj_bbox = (int4 *)(ws + w.obj_bbox);
    a.queue = (unsigned int *)(ws + w.queue);
    if (L->gframes > 0) {
        a.fscratch = ws + w.fscratch;
        a.fscratch_stride = (int64_t)w.fs_stride;
        a.fs_verts = w.fs_verts;
        a.fs_surv = (int32_t)w.fs_surv;
        a.fs_bins = (int32_t)std::min<int64_t>(w.fs_bins, 0x7fffffff);
    }
    ScopedDevice sd(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    KernelTimer &T = ctx->timer;
    hipError_t e = hipSuccess;
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
        if (k < 2 && a.n_titems == 0) continue;  // no frame on the tiled path
        if (k == 2 && a.n_fitems == 0) continue;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (T.enabled && timing) {
            e0 = T.get();
            e1 = T.get();
            if (e0) e = hipEventRecord(e0, st);
        }
        if (e == hipSuccess)
            e = k == 0 ? launch_vertex(a, st) : k == 1 ? launch_raster(a, st, ctx->n_cu) : launch_frame(a, st, ctx->n_cu);
        if (T.enabled && timing && e0 && e1 && e == hipSuccess) {
            e = hipEventRecord(e1, st);
            T.pending[k].push_back({e0, e1});
        }
    }
    if (e != hipSuccess) return fail(ORRB_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return ORRB_OK;
}

// With ORRB_DEBUG_VALIDATE set when the context was created: the precondition check
// (orrb_validate_batch) into the call's stats destination, ahead of the render kernels.
orrb_status orrb::debug_validate(orrb_context *ctx, const orrb_layout *L, const orrb_scenes *sc,
                                 const orrb_cameras *cam, const orrb_params *par, const orrb_outputs *out,
                                 void *stream) {
    if (!ctx || !ctx->debug_validate || !out || !out->stats) return ORRB_OK;
    return orrb_validate_batch(ctx, L, sc, cam, par, out->stats, stream);
}

extern "C" {

orrb_status orrb_render_batch(orrb_context *ctx, const orrb_layout *L, const orrb_scenes *sc, const orrb_cameras *cam,
                              const orrb_params *par, const orrb_outputs *out, void *workspace, size_t workspace_bytes,
                              void *stream) {
    g_last_error.clear();
    const orrb_status st = debug_validate(ctx, L, sc, cam, par, out, stream);
    if (st != ORRB_OK) return st;
    bool timing = true;  // with profiling on: every `every`-th call is timed
    if (ctx && ctx->timer.enabled) timing = ctx->timer.calls++ % ctx->timer.every == 0;
    return render_impl(ctx, L, sc, cam, par, out, workspace, workspace_bytes, stream, timing);
}

orrb_status orrb_validate_batch(orrb_context *ctx, const orrb_layout *L, const orrb_scenes *sc, const orrb_cameras *cam,
                                const orrb_params *par, uint32_t *stats, void *stream) {
    g_last_error.clear();
    if (!ctx || !L || !sc || !cam || !par || !stats) return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL handle, struct or stats");
    if (L->ctx != ctx) return fail(ORRB_ERR_INVALID_ARGUMENT, "layout belongs to another context");
    if (L->n_frames == 0 && L->n_objects == 0 && L->n_lights == 0) return ORRB_OK;
    {
        const orrb_status st = check_inputs(L, sc, cam, par);
        if (st != ORRB_OK) return st;
    }
    if (L->n_spot > 0 && (!par->light_dir || !par->light_cone || !par->shadow_view || !par->shadow_intr))
        return fail(ORRB_ERR_INVALID_ARGUMENT, "spot lights need light_dir, light_cone, shadow_view and shadow_intr");
    RenderArgs a;
    fill_args(ctx, L, sc, cam, par, &a);
    a.light_dir = par->light_dir;
    a.light_cone = par->light_cone;
    a.shadow_view = par->shadow_view;
    a.shadow_intr = par->shadow_intr;
    ScopedDevice sd(ctx->device);
    const hipError_t e = launch_validate(a, par->post, (int)L->n_objects, (int)L->n_lights, (int)L->n_frames, stats,
                                         (hipStream_t)stream);
    if (e != hipSuccess) return fail(ORRB_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return ORRB_OK;
}

orrb_status orrb_shade_backward(orrb_context *ctx, const orrb_layout *L, const orrb_scenes *sc, const orrb_cameras *cam,
                                const orrb_params *par, const uint64_t *vis, const float *grad_rgb, const orrb_grads *gr,
                                void *workspace, size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    if (!ctx || !L || !sc || !cam || !par || !gr) return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL handle or struct");
    if (L->ctx != ctx) return fail(ORRB_ERR_INVALID_ARGUMENT, "layout belongs to another context");
    if (L->n_frames == 0 && L->n_objects == 0 && L->n_lights == 0) return ORRB_OK;
    {
        const orrb_status st = check_inputs(L, sc, cam, par);
        if (st != ORRB_OK) return st;
    }
    if (L->n_frames > 0 && (!vis || !grad_rgb)) return fail(ORRB_ERR_INVALID_ARGUMENT, "vis or grad_rgb is NULL");
    if ((L->n_objects > 0 && (!gr->albedo || !gr->roughness || !gr->specular)) ||
        (L->n_lights > 0 && (!gr->light_vec || !gr->light_intensity)) || (L->n_frames > 0 && !gr->exposure))
        return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL gradient destination");
    if (L->n_spot > 0) return fail(ORRB_ERR_UNSUPPORTED, "the shading adjoint does not cover spot lights");
    if (par->texture || par->emission || par->normal_texture)
        return fail(ORRB_ERR_UNSUPPORTED, "the shading adjoint does not cover textured or emissive materials");
    if (L->max_scene_objects > grad_max_objects())
        return fail(ORRB_ERR_UNSUPPORTED, "a scene has %d objects; the adjoint supports %d", L->max_scene_objects,
                    grad_max_objects());
    const size_t need = grad_workspace(L);
    if (!workspace) return fail(ORRB_ERR_INVALID_ARGUMENT, "workspace is NULL");
    if (workspace_bytes < need)
        return fail(ORRB_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu required", workspace_bytes, need);
    if ((uintptr_t)workspace % 16 != 0) return fail(ORRB_ERR_INVALID_ARGUMENT, "workspace must be 16-byte aligned");
    if (!L->grad_ready) {
        const orrb_status st = upload_grad_tables(const_cast<orrb_layout *>(L));
        if (st != ORRB_OK) return st;
    }
    GradArgs g;
    memset(&g, 0, sizeof(g));
    fill_args(ctx, L, sc, cam, par, &g.r);
    const WsLayout w = ws_layout(L->all_vertex_instances, L->all_object_instances);
    char *ws = (char *)workspace;
    g.r.frames = L->gtab.at<FrameInfo>(L->g_frames_all);
    g.r.vitems = L->gtab.at<int2>(L->g_vitems_all);
    g.r.n_vitems = (int32_t)L->vitems_all.size();
    g.r.vtx_pos = (int4 *)(ws + w.vtx_pos);
    g.r.obj_rot = (float4 *)(ws + w.obj_rot);
    g.r.obj_bbox = (int4 *)(ws + w.obj_bbox);
    g.r.queue = (unsigned int *)(ws + w.queue);
    g.vis = (const unsigned long long *)vis;
    g.grad_rgb = grad_rgb;
    g.gitems = L->gtab.at<int2>(L->g_gitems);
    g.gitem_pbase = L->gtab.at<int64_t>(L->g_gitem_pbase);
    g.n_gitems = (int32_t)L->gitems.size();
    g.partial = (double *)(ws + al256(w.total));
    g.scene_frames = L->gtab.at<int32_t>(L->g_scene_frames);
    g.scene_frame_begin = L->gtab.at<int32_t>(L->g_scene_frame_begin);
    g.frame_item_begin = L->gtab.at<int32_t>(L->g_frame_item_begin);
    g.obj_scene = L->gtab.at<int32_t>(L->g_obj_scene);
    g.obj_local = L->gtab.at<int32_t>(L->g_obj_local);
    g.light_scene = L->gtab.at<int32_t>(L->g_light_scene);
    g.light_local = L->gtab.at<int32_t>(L->g_light_local);
    g.g_albedo = gr->albedo;
    g.g_rough = gr->roughness;
    g.g_spec = gr->specular;
    g.g_lpos = gr->light_vec;
    g.g_lint = gr->light_intensity;
    g.g_expo = gr->exposure;
    g.n_objects = (int32_t)L->n_objects;
    g.n_lights = (int32_t)L->n_lights;
    g.n_frames = (int32_t)L->n_frames;
    g.scene_obj_begin = L->gtab.at<int32_t>(L->g_scene_obj_begin);
    g.scene_light_begin = L->gtab.at<int32_t>(L->g_scene_light_begin);
    g.n_scenes = (int32_t)L->n_scenes;
    g.max_scene_params = L->max_scene_params;
    ScopedDevice sd(ctx->device);
    const hipError_t e = launch_grad(g, (hipStream_t)stream);
    if (e != hipSuccess) return fail(ORRB_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return ORRB_OK;
}

orrb_status orrb_profile_enable(orrb_context *ctx, int enable) {
    g_last_error.clear();
    if (!ctx) return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL context");
    ScopedDevice sd(ctx->device);
    if (enable < 0) return fail(ORRB_ERR_INVALID_ARGUMENT, "negative sampling interval %d", enable);
    HIP_TRY(ctx->timer.drain());
    ctx->timer.enabled = enable != 0;
    ctx->timer.every = enable > 1 ? enable : 1;
    ctx->timer.calls = 0;
    for (int k = 0; k < 3; ++k) {
        ctx->timer.total_ms[k] = 0;
        ctx->timer.count[k] = 0;
    }
    return ORRB_OK;
}

orrb_status orrb_wait_timeouts(orrb_context *ctx, uint64_t *count_out) {
    g_last_error.clear();
    if (!ctx || !count_out) return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL argument");
    ScopedDevice sd(ctx->device);
    unsigned int n = 0;
    HIP_TRY(read_wait_timeouts(&n));
    *count_out = n;
    return ORRB_OK;
}

orrb_status orrb_profile_read(orrb_context *ctx, orrb_kernel_times *out) {
    g_last_error.clear();
    if (!ctx || !out) return fail(ORRB_ERR_INVALID_ARGUMENT, "NULL argument");
    ScopedDevice sd(ctx->device);
    HIP_TRY(ctx->timer.drain());
    out->vertex_ms = ctx->timer.total_ms[0];
    out->raster_ms = ctx->timer.total_ms[1];
    out->frame_ms = ctx->timer.total_ms[2];
    out->vertex_launches = ctx->timer.count[0];
    out->raster_launches = ctx->timer.count[1];
    out->frame_launches = ctx->timer.count[2];
    return ORRB_OK;
}

}  // extern "C"
