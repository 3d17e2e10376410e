// HIP kernels of the batched randomized renderer, written for CDNA4 (gfx950, wave64).
//
// Two paths render a batch; both produce bit-identical outputs because they share
// every arithmetic primitive below (vertex snapping, edge functions, fragment depth,
// shading), compiled with floating-point contraction off.
//
// Frame path (k_frame), for frames whose scene fits in LDS: a persistent kernel, one
// 1024-thread workgroup per CU rendering frames one after another with no intermediate
// data in global memory.  Twelve compute waves, per frame:
//   1. transform and snap every vertex of the scene (FP64) into LDS;
//   2. set up every triangle once (exact area, back-face and range cull) and count, per
//      64x4 screen tile, the triangles whose pixel-centre range touches it;
//   3. scan the counts, hand the tiles no triangle touches to the store waves, and
//      scatter 16-bit triangle IDs into per-tile LDS bins;
//   4. take tiles with entries from an LDS counter, rasterize each bin into a 256-key
//      LDS visibility tile (ds_min_u64), shade the covered pixels and put the finished
//      tile into an LDS staging slot.
// The other four waves issue the global stores: the background of handed-over tiles
// (while the compute waves go on with the next frame) and the staged tiles; in the
// auxiliary-output kernels a compute wave out of busy tiles also writes background.
//
// Tiled path (k_vertex + k_raster_shade), for any scene size:
//   k_vertex        one workgroup per (frame, object): FP64 transform and snap into a
//                   global workspace, the object's covered pixel-centre range and its
//                   view rotation;
//   k_raster_shade  one workgroup per (frame, screen tile): cull objects by their
//                   range, set up their triangles and stage survivors in an LDS bin,
//                   rasterize (triangle, pixel) pairs into an LDS tile of 64-bit keys,
//                   then shade and write the tile.
//
// A visibility key is (fp32 eye depth bits << 32 | scene-local triangle ID); the
// nearest fragment wins and exact depth ties go to the lower ID.  Being a 64-bit
// minimum, the result does not depend on the order in which lanes, bins, tiles or
// workgroups run: outputs are bit-identical for every tuning and batch composition.
// (Inside k_frame's LDS tile the ID field also carries the object slot above the 16-bit
// ID; slots never decrease with the ID, so the order is the same, and the slot bits are
// cleared before a key is written out.)
#include "orrb_post.h"

namespace orrb {

// Light k of frame f's scene (global light l = fi.light_begin + k) in view space, its
// type word and, for a spot light, its record in spot[] (the index counts the scene's
// spot lights before it).
ORRB_INLINE void frame_light(const RenderArgs &a, int f, const FrameInfo &fi, int k, float4 *light, int *ltype,
                             SpotLight *spot) {
    const int l = fi.light_begin + k;
    const float *V = a.view + 12 * (int64_t)f;
    const int t = a.light_type[l];
    light[k] = view_light(V, a.light_vec + 3 * (int64_t)l, t == 2 ? 0 : t, a.light_intensity[l]);
    if (t == 2) {
        int idx = 0;
        for (int j = 0; j < k; ++j) idx += a.light_type[fi.light_begin + j] == 2;
        spot[idx] = spot_setup(a, V, l);
        ltype[k] = 2 | (idx << 4);
    } else {
        ltype[k] = t;
    }
}

// ------------------------------------------------------------------------------------
// tiled path: k_vertex
// ------------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_vertex(RenderArgs a) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.queue = 0u;  // persistent raster counter
    if ((int)blockIdx.x >= a.n_vitems) return;
    __shared__ double M[12];
    __shared__ int red[4][kBlock / kWave];
    const int2 it = a.vitems[blockIdx.x];
    const int f = it.x;
    const FrameInfo fi = a.frames[f];
    const int o = fi.obj_begin + it.y;
    const int oi = fi.oi_base + it.y;
    if (threadIdx.x < 12) M[threadIdx.x] = compose_entry(a.view + 12 * (int64_t)f, a.pose + 12 * (int64_t)o, threadIdx.x);
    __syncthreads();
    const float *K = a.intr + 4 * (int64_t)f;
    const double fx = K[0], fy = K[1], cx = K[2], cy = K[3], nearp = a.near_plane[f];
    if (a.out_track && threadIdx.x == 0)  // hidden objects too: their origin is still reported
        track_init(a.out_track + fi.track_base + it.y, M[3], M[7], M[11], fx, fy, cx, cy);
    if (!a.visible[o]) {
        if (threadIdx.x == 0) a.obj_bbox[oi] = make_int4(1, 1, 0, 0);
        return;
    }
    const ObjInfo ob = a.objs[o];
    if (threadIdx.x < 3) {
        const int r = threadIdx.x;
        a.obj_rot[3 * (int64_t)oi + r] = make_float4((float)M[4 * r + 0], (float)M[4 * r + 1], (float)M[4 * r + 2], 0.f);
    }
    double Mr[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) Mr[k] = M[k];
    int xmin = 0x7fffffff, ymin = 0x7fffffff, xmax = -0x7fffffff, ymax = -0x7fffffff;
    const int64_t vb = fi.vbase + ob.scene_vbase;
    unsigned n_near = 0, n_guard = 0;
    for (int v = threadIdx.x; v < ob.n_verts; v += kBlock) {
        const Snapped s = snap_vertex(Mr, a.mesh_pos[ob.mesh_vbegin + v], fx, fy, cx, cy, nearp);
        a.vtx_pos[vb + v] = make_int4(s.X, s.Y, __float_as_int(s.iw), s.valid);
        n_near += s.cull == 1;
        n_guard += s.cull == 2;
        if (s.valid) {
            xmin = min(xmin, s.X);
            xmax = max(xmax, s.X);
            ymin = min(ymin, s.Y);
            ymax = max(ymax, s.Y);
        }
    }
    stat_add(a, ORRB_STAT_NEAR_VERTICES, n_near);  // rare: one atomic per thread that saw one
    stat_add(a, ORRB_STAT_GUARD_VERTICES, n_guard);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        xmin = min(xmin, __shfl_xor(xmin, off));
        ymin = min(ymin, __shfl_xor(ymin, off));
        xmax = max(xmax, __shfl_xor(xmax, off));
        ymax = max(ymax, __shfl_xor(ymax, off));
    }
    const int wave = threadIdx.x / kWave;
    if (lane_id() == 0) {
        red[0][wave] = xmin;
        red[1][wave] = ymin;
        red[2][wave] = xmax;
        red[3][wave] = ymax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / kWave; ++w) {
            xmin = min(xmin, red[0][w]);
            ymin = min(ymin, red[1][w]);
            xmax = max(xmax, red[2][w]);
            ymax = max(ymax, red[3][w]);
        }
        int4 bb = make_int4(1, 1, 0, 0);
        if (xmin <= xmax) {
            bb.x = max(ceil256(xmin - 128), 0);
            bb.y = max(ceil256(ymin - 128), 0);
            bb.z = min(floor256(xmax - 128), fi.width - 1);
            bb.w = min(floor256(ymax - 128), fi.height - 1);
        }
        a.obj_bbox[oi] = bb;
    }
}

// ------------------------------------------------------------------------------------
// tiled path: k_raster_shade
// ------------------------------------------------------------------------------------

// LDS of one raster workgroup: a compile-time layout per (tile pixels, bin capacity)
// instantiation, so every access is a constant LDS address.
template <int VIS, int CAP>
struct TileLds {
    unsigned long long vis[VIS];  // visibility keys of the tile
    int b_tri[CAP], b_x0[CAP], b_y0[CAP], b_x1[CAP], b_y1[CAP], b_x2[CAP], b_y2[CAP], b_rng[CAP], b_flags[CAP];
    int b_pre[CAP + 1];
    float b_iw0[CAP], b_iw1[CAP], b_iw2[CAP], b_area[CAP];
    // overlapping objects of the current chunk, in scene order
    int ol_obj[kBlock], ol_tbase[kBlock], ol_mtb[kBlock], ol_mvb[kBlock], ol_vb[kBlock], ol_cnt[kBlock];
    int ol_pre[kBlock + 1];
    float ol_R[kBlock][9];
    float4 light[kMaxLights];
    int light_type[kMaxLights];
    SpotLight spot[kMaxSpots];
    int misc[16];  // [0] bin count, [1] next item, [4..8) scan, [8..12) wave counts
};

// Inclusive sum over the 64 lanes of a wave with DPP: shifts by 1, 2, 4 and 8 inside
// each 16-lane row, then the last lane of row 0 into row 1 and of row 2 into row 3, then
// lane 31 into rows 2 and 3 (lanes without a source add 0).
ORRB_INLINE int wave_scan_add(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
    return v;
}

// Exclusive scan over n <= 4 * kBlock counts; writes pre[0..n].
template <class F>
ORRB_INLINE void block_scan(F cnt, int n, int *pre, int *wave_tot) {
    const int per = (n + kBlock - 1) / kBlock;
    const int t = threadIdx.x, lane = lane_id(), wave = t / kWave;
    const int start = t * per;
    int local = 0;
    for (int k = 0; k < per; ++k)
        if (start + k < n) local += cnt(start + k);
    const int incl = wave_scan_add(local);
    if (lane == kWave - 1) wave_tot[wave] = incl;
    __syncthreads();
    int wbase = 0;
    for (int w = 0; w < wave; ++w) wbase += wave_tot[w];
    int run = wbase + incl - local;
    for (int k = 0; k < per; ++k) {
        if (start + k < n) {
            pre[start + k] = run;
            run += cnt(start + k);
        }
    }
    if (t == kBlock - 1) pre[n] = wbase + incl;
    __syncthreads();
}

// Raster every staged triangle of the bin: one lane per (triangle, bounding-box pixel)
// pair, so lanes stay busy whatever the triangle sizes.
template <class LD>
ORRB_INLINE void flush_bin(LD &L, int n, int tx0, int ty0, int tile_w) {
    block_scan([&](int k) { const unsigned r = (unsigned)L.b_rng[k]; return (int)(((r >> 16) & 0xff) * (r >> 24)); },
               n, L.b_pre, L.misc + 4);
    const int total = L.b_pre[n];
    for (int w = threadIdx.x; w < total; w += kBlock) {
        const int k = find_slot(L.b_pre, n, w);
        const unsigned rng = (unsigned)L.b_rng[k];
        const int nx = (rng >> 16) & 0xff;
        const int r = w - L.b_pre[k];
        const int dj = (int)(((float)r + 0.5f) * __builtin_amdgcn_rcpf((float)nx));  // exact: r < 4096, nx <= 64
        const int di = r - dj * nx;
        const int li = (int)(rng & 0xff) + di, lj = (int)((rng >> 8) & 0xff) + dj;
        const Edges e = edge_eval(L.b_x0[k], L.b_y0[k], L.b_x1[k], L.b_y1[k], L.b_x2[k], L.b_y2[k],
                                  ((tx0 + li) << 8) + 128, ((ty0 + lj) << 8) + 128, L.b_flags[k]);
        if (!e.covered) continue;
        const float z = fragment_depth(e, L.b_iw0[k], L.b_iw1[k], L.b_iw2[k], L.b_area[k]);
        atomicMin(&L.vis[lj * tile_w + li], vis_key(z, L.b_tri[k]));
    }
    __syncthreads();
}

template <class LD>
ORRB_INLINE void raster_shade_tile(const RenderArgs &a, int item, LD &L) {
    const int2 it = a.titems[item];
    const int f = it.x;
    const FrameInfo fi = a.frames[f];
    const int TW = a.tile_w, TH = a.tile_h, cap = a.bin_cap;
    const int tx0 = (it.y % fi.tiles_x) * TW, ty0 = (it.y / fi.tiles_x) * TH;
    const int tw = min(TW, fi.width - tx0), th = min(TH, fi.height - ty0);
    const int tx1 = tx0 + tw - 1, ty1 = ty0 + th - 1;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;

    for (int p = tid; p < TW * TH; p += kBlock) L.vis[p] = kEmptyKey;
    if (tid == 0) L.misc[0] = 0;
    if (tid < fi.n_lights) frame_light(a, f, fi, tid, L.light, L.light_type, L.spot);
    __syncthreads();

    // ---- visibility: object cull, triangle set-up into the LDS bin, raster ----
    const int64_t vbase = fi.vbase;
    int n_ol = 0, n_flush = 0;
    for (int c0 = 0; c0 < fi.n_obj; c0 += kBlock) {
        const int s = c0 + tid;
        bool ov = false;
        if (s < fi.n_obj) {
            const int4 bb = a.obj_bbox[fi.oi_base + s];
            ov = bb.x <= bb.z && bb.y <= bb.w && bb.x <= tx1 && bb.z >= tx0 && bb.y <= ty1 && bb.w >= ty0;
        }
        {   // order-preserving compaction: the list stays sorted by scene triangle base
            const unsigned long long m = __ballot(ov);
            if (lane == 0) L.misc[8 + wave] = __popcll(m);
            __syncthreads();
            int base = 0;
            for (int w = 0; w < wave; ++w) base += L.misc[8 + w];
            n_ol = L.misc[8] + L.misc[9] + L.misc[10] + L.misc[11];
            if (ov) {
                const ObjInfo ob = a.objs[fi.obj_begin + s];
                const int slot = base + lanes_below(m);
                L.ol_obj[slot] = fi.obj_begin + s;
                L.ol_tbase[slot] = ob.scene_tbase;
                L.ol_mtb[slot] = ob.mesh_tbegin;
                L.ol_mvb[slot] = ob.mesh_vbegin;
                L.ol_vb[slot] = ob.scene_vbase;
                L.ol_cnt[slot] = ob.n_tris;
                const float4 *rot = a.obj_rot + 3 * (int64_t)(fi.oi_base + s);
                for (int r = 0; r < 3; ++r) {
                    const float4 q = rot[r];
                    L.ol_R[slot][3 * r + 0] = q.x;
                    L.ol_R[slot][3 * r + 1] = q.y;
                    L.ol_R[slot][3 * r + 2] = q.z;
                }
            }
        }
        __syncthreads();
        block_scan([&](int k) { return L.ol_cnt[k]; }, n_ol, L.ol_pre, L.misc + 4);
        const int n_cand = L.ol_pre[n_ol];
        for (int base = 0; base < n_cand; base += kBlock) {
            const int k = base + tid;
            bool keep = false;
            int xa = 0, ya = 0, xb = 0, yb = 0, xc = 0, yc = 0, rng = 0, flags = 0, tri_id = 0;
            float iwa = 0.f, iwb = 0.f, iwc = 0.f, area = 0.f;
            if (k < n_cand) {
                const int sl = find_slot(L.ol_pre, n_ol, k);
                const int t = k - L.ol_pre[sl];
                const int4 tri = a.mesh_tri[L.ol_mtb[sl] + t];
                const int64_t vb = vbase + L.ol_vb[sl];
                const int4 p0 = a.vtx_pos[vb + tri.x], p1 = a.vtx_pos[vb + tri.y], p2 = a.vtx_pos[vb + tri.z];
                const int xmin = min(p0.x, min(p1.x, p2.x)), xmax = max(p0.x, max(p1.x, p2.x));
                const int ymin = min(p0.y, min(p1.y, p2.y)), ymax = max(p0.y, max(p1.y, p2.y));
                const int i0 = max(ceil256(xmin - 128), tx0), i1 = min(floor256(xmax - 128), tx1);
                const int j0 = max(ceil256(ymin - 128), ty0), j1 = min(floor256(ymax - 128), ty1);
                if ((p0.w & p1.w & p2.w) && i0 <= i1 && j0 <= j1) {
                    const long long A = (long long)(p1.x - p0.x) * (p2.y - p0.y) - (long long)(p1.y - p0.y) * (p2.x - p0.x);
                    if (A < 0) {
                        // front face: a = v0, b = v2, c = v1 gives a positive area
                        keep = true;
                        xa = p0.x; ya = p0.y; xb = p2.x; yb = p2.y; xc = p1.x; yc = p1.y;
                        rng = (i0 - tx0) | ((j0 - ty0) << 8) | ((i1 - i0 + 1) << 16) | ((j1 - j0 + 1) << 24);
                        flags = tri_flags(xa, ya, xb, yb, xc, yc);
                        iwa = __int_as_float(p0.z);
                        iwb = __int_as_float(p2.z);
                        iwc = __int_as_float(p1.z);
                        area = (float)(-A);
                        tri_id = L.ol_tbase[sl] + t;
                    }
                }
            }
            const unsigned long long m = __ballot(keep);
            int wb = 0;
            if (lane == 0 && m) wb = atomicAdd(&L.misc[0], __popcll(m));
            wb = __builtin_amdgcn_readlane(wb, 0);
            if (keep) {
                const int slot = wb + lanes_below(m);
                L.b_tri[slot] = tri_id;
                L.b_x0[slot] = xa; L.b_y0[slot] = ya;
                L.b_x1[slot] = xb; L.b_y1[slot] = yb;
                L.b_x2[slot] = xc; L.b_y2[slot] = yc;
                L.b_rng[slot] = rng;
                L.b_flags[slot] = flags;
                L.b_iw0[slot] = iwa; L.b_iw1[slot] = iwb; L.b_iw2[slot] = iwc;
                L.b_area[slot] = area;
            }
            __syncthreads();
            const int nb = L.misc[0];
            if (nb > cap - kBlock) {
                ++n_flush;
                flush_bin(L, nb, tx0, ty0, TW);
                if (tid == 0) L.misc[0] = 0;
                __syncthreads();
            }
        }
    }
    {
        const int nb = L.misc[0];
        if (nb > 0) {
            ++n_flush;
            flush_bin(L, nb, tx0, ty0, TW);
        }
        if (tid == 0 && n_flush > 1) stat_add(a, ORRB_STAT_TILED_EXTRA_FLUSH, (unsigned)(n_flush - 1));
    }

    // ---- deferred shading of the tile ----
    const bool lds_objs = fi.n_obj <= kBlock;  // the (single) object list is still in LDS
    const CamF cam = frame_camera(a, f);
    const int64_t HW = (int64_t)fi.width * fi.height, po = fi.pixel_offset;
    const float inv_tw = __builtin_amdgcn_rcpf((float)tw);
    const bool fused = a.out_rgb8 != nullptr;  // 8-bit output encoded as the pixel is written
    PostFrame pq;
    if (fused) pq = post_frame(a, f);
    for (int p = tid; p < tw * th; p += kBlock) {
        const int lj = (int)(((float)p + 0.5f) * inv_tw);  // exact: p < 4096, tw <= 64
        const int li = p - lj * tw;
        const int i = tx0 + li, j = ty0 + lj;
        const int64_t pix = (int64_t)j * fi.width + i;
        const unsigned long long key = L.vis[lj * TW + li];
        PixelOut o = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float z = 0.f;
        int segv = -1, triv = -1;
        if (key != kEmptyKey) {
            const int tri = (int)(unsigned)(key & 0xffffffffu);
            z = __uint_as_float((unsigned)(key >> 32));
            int obj, tbase, mtb, mvb;
            int64_t vb;
            float R[9];
            if (lds_objs) {
                const int sl = find_slot(L.ol_tbase, n_ol, tri);
                obj = L.ol_obj[sl];
                tbase = L.ol_tbase[sl];
                mtb = L.ol_mtb[sl];
                mvb = L.ol_mvb[sl];
                vb = vbase + L.ol_vb[sl];
#pragma unroll
                for (int q = 0; q < 9; ++q) R[q] = L.ol_R[sl][q];
            } else {
                int lo = 0, hi = fi.n_obj;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (a.objs[fi.obj_begin + mid].scene_tbase <= tri) lo = mid; else hi = mid;
                }
                const ObjInfo ob = a.objs[fi.obj_begin + lo];
                obj = fi.obj_begin + lo;
                tbase = ob.scene_tbase;
                mtb = ob.mesh_tbegin;
                mvb = ob.mesh_vbegin;
                vb = vbase + ob.scene_vbase;
                const float4 *rot = a.obj_rot + 3 * (int64_t)(fi.oi_base + lo);
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const float4 q = rot[r];
                    R[3 * r + 0] = q.x;
                    R[3 * r + 1] = q.y;
                    R[3 * r + 2] = q.z;
                }
            }
            const int4 tv = a.mesh_tri[mtb + (tri - tbase)];
            // the winning triangle is front-facing: same vertex order as in set-up
            const int4 pa = a.vtx_pos[vb + tv.x], pb = a.vtx_pos[vb + tv.z], pc = a.vtx_pos[vb + tv.y];
            const MatTex mt = mat_inputs(a, obj, mvb, tv);
            o = shade_pixel<true, true>(pa.x, pa.y, pb.x, pb.y, pc.x, pc.y, __int_as_float(pa.z), __int_as_float(pb.z),
                            __int_as_float(pc.z), a.mesh_nrm[mvb + tv.x], a.mesh_nrm[mvb + tv.z], a.mesh_nrm[mvb + tv.y], R,
                            i, j, z, cam, L.light, L.light_type, fi.n_lights, object_material(a, obj), L.spot,
                            a.shadow_maps, a.shadow_res, &mt, a.tex_texels, a.tex_info);
            segv = a.seg[obj];
            triv = tri;
        }
        store_pixel(a, po, HW, pix, o, z, segv, triv, key);
        if (fused) {
            float n0 = 0.f, n1 = 0.f, n2 = 0.f;
            if (pq.gi != 0.f) {
                const unsigned t = grain_texel(a, pq, i, j);
                n0 = grain_at(pq.g0, t);
                n1 = grain_at(pq.g1, t);
                n2 = grain_at(pq.g2, t);
            }
            const uchar3 u = post_pixel(pq, o.r0, o.r1, o.r2, n0, n1, n2);
            uint8_t *d = a.out_rgb8 + 3 * po + pix;
            d[0] = u.x;
            d[HW] = u.y;
            d[2 * HW] = u.z;
        }
    }

    // ---- tracker: every lane of a wave takes part (the trip count is uniform) ----
    if (a.out_track) {
        for (int p0 = 0; p0 < tw * th; p0 += kBlock) {
            const int p = p0 + tid;
            int rec = -1, i = 0, j = 0;
            if (p < tw * th) {
                const int lj = (int)(((float)p + 0.5f) * inv_tw), li = p - lj * tw;
                const unsigned long long key = L.vis[lj * TW + li];
                if (key != kEmptyKey) {
                    const int tri = (int)(unsigned)(key & 0xffffffffu);
                    int local;
                    if (lds_objs) {
                        local = L.ol_obj[find_slot(L.ol_tbase, n_ol, tri)] - fi.obj_begin;
                    } else {
                        int lo = 0, hi = fi.n_obj;
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (a.objs[fi.obj_begin + mid].scene_tbase <= tri) lo = mid; else hi = mid;
                        }
                        local = lo;
                    }
                    rec = fi.track_base + local;
                    i = tx0 + li;
                    j = ty0 + lj;
                }
            }
            if (fi.width <= 1024 && fi.height <= 1024)
                track_wave<true>(a.out_track, rec, i, j);
            else
                track_wave<false>(a.out_track, rec, i, j);
        }
    }
}

// Work-item index of workgroup `bid` among `n`, grouping consecutive items on the same
// XCD (workgroups are dispatched to the 8 XCDs round-robin), so the tiles of one frame
// share that XCD's L2.
ORRB_INLINE int xcd_remap(int bid, int n) {
    const int q = n >> 3, r = n & 7, xcd = bid & 7, local = bid >> 3;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

template <int VIS, int CAP>
__global__ __launch_bounds__(kBlock) void k_raster_shade(RenderArgs a) {
    __shared__ TileLds<VIS, CAP> L;
    if (!a.persistent) {
        raster_shade_tile(a, xcd_remap(blockIdx.x, gridDim.x), L);
        return;
    }
    int item = blockIdx.x;
    while (item < a.n_titems) {
        raster_shade_tile(a, item, L);
        __syncthreads();
        if (threadIdx.x == 0) L.misc[1] = (int)gridDim.x + (int)atomicAdd(a.queue, 1u);
        __syncthreads();
        item = L.misc[1];
    }
}

// ------------------------------------------------------------------------------------
// frame path: k_frame
// ------------------------------------------------------------------------------------

constexpr int kFT = 1024;           // threads of a frame workgroup
constexpr int kFW = kFT / kWave;    // 16 waves
constexpr int kFVMax = 6976;        // scene vertices held in LDS
constexpr int kFOMax = 48;          // scene objects
constexpr int kFGOMax = 127;        // scene objects of a frame whose data live in global scratch
constexpr int kFGVMax = 65536;      // scene vertices of such a frame
constexpr int kFTileW = 64;         // wave tile: 64 x 4 pixels, so that a wave's store
constexpr int kFTileH = 4;          // instruction writes 256-byte row segments
constexpr int kFTilesMax = 256;     // frames up to 256 x 256 (4 x 64 tiles)
constexpr int kFBinMax = 7680;      // (tile, triangle) bin entries (hand scenes: < 7,000)
constexpr int kFSurvMax = 6144;     // survivors remembered between set-up and scatter (< 5,200)
constexpr int kFHint = 64;          // elements per object-lookup hint
constexpr int kFCW = 12;            // compute waves: geometry, raster, shading
constexpr int kFCT = kFCW * kWave;  // compute threads
constexpr int kFSlots = 4;          // frames whose background tiles may be pending at once
constexpr int kFStage = 3;          // staged busy tiles (compute -> store waves)
constexpr int kFPace = 60;          // store instructions in flight per store wave
constexpr bool kFStageWave = true;  // the last wave writes only staged tiles
constexpr int kFVN = 2;             // vertices per thread per pass
constexpr int kFTN = 3;             // triangles per thread per pass
constexpr unsigned kFSpinCap = 1u << 22;  // bound on every wait loop (about 0.3 s, far beyond
                                          // the slowest legitimate tile): reached only if a
                                          // peer wave stalls; the kernel then ends with
                                          // unspecified pixels rather than hanging
constexpr int kInvalidX = (int)0x80000000;

struct BgFrame {
    long long po;  // pixel offset of the frame
    int W, H, ntx, vec;
    int n;         // background tiles of the frame
    int f;         // the frame
};

struct StageInfo {
    long long po;  // pixel offset of the frame
    int W, H, x0, y0, vec, f;
};

// The 8-bit output, encoded by the frame kernel as it writes tiles out: the waves that
// write them keep the grading constants of the last frame they wrote.
struct PostCache {
    int f = -1;
    PostFrame q;
    float3 o_bg;  // post_grade of a background pixel (rgb 0)
};

ORRB_INLINE bool fused_rgb8(const RenderArgs &a) { return a.out_rgb8 != nullptr; }

// Codes of the lane's four pixels (i .. i + 3, j) of frame f from linear rgb v, stored
// to the 8-bit planes: one 4-byte store per plane when the group is whole and aligned.
// v == nullptr: four background pixels (rgb 0).
ORRB_INLINE void store_codes4(const RenderArgs &a, PostCache &pc, int f, int64_t po, int64_t HW, int64_t pix, int i,
                              int j, const float (*v)[4], bool vec, int n) {
    if (pc.f != f) {  // uniform: every lane writes the same frame
        pc.q = post_frame(a, f);
        pc.o_bg = post_grade(pc.q, 0.f, 0.f, 0.f);
        pc.f = f;
    }
    unsigned code[3];
    if (v)
        post_codes_row(a, pc.q, i, j, v, code);
    else
        post_codes_row_bg(a, pc.q, pc.o_bg, i, j, code);
    uint8_t *dst = a.out_rgb8 + 3 * po + pix;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (vec) {
            *reinterpret_cast<unsigned *>(dst + c * HW) = code[c];
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k < n) dst[c * HW + k] = (uint8_t)(code[c] >> (8 * k));
        }
    }
}

struct FrameLds {
    union {
        struct {  // scenes held in LDS: the snapped vertices
            int2 XY[kFVMax];
            float iw[kFVMax];
        } v;
        struct {  // larger scenes (vertices, bins, survivors in global scratch): object tables
            int o_tbase[kFGOMax], o_vbase[kFGOMax], o_mtb[kFGOMax], o_mvb[kFGOMax], o_nt[kFGOMax], o_seg[kFGOMax],
                o_vis[kFGOMax];
            float o_R[kFGOMax][9];
            Material o_mat[kFGOMax];
            unsigned char vtx_hint[kFGVMax / kFHint];
        } g;
    } m;
    union {
        double M[kFGOMax][12];                        // vertex phase
        unsigned int surv[kFSurvMax];                 // set-up -> scatter: (tri << 16) | tile range
        unsigned long long vis[kFCW][kFTileW * kFTileH];  // tile phase
    } u;
    unsigned short bin[kFBinMax];
    int cnt[kFTilesMax + 1], off[kFTilesMax + 1];
    unsigned char order[kFTilesMax];                 // tile order: tiles with bin entries first
    unsigned char cov[kFCW][kFTileW * kFTileH];      // per compute wave: covered pixels of its tile
    unsigned char tri_hint[65536 / kFHint];          // object of triangle 64 b
    unsigned char vtx_hint[(kFVMax + kFHint - 1) / kFHint];
    int o_tbase[kFOMax], o_vbase[kFOMax], o_mtb[kFOMax], o_mvb[kFOMax], o_nt[kFOMax], o_seg[kFOMax], o_vis[kFOMax];
    float o_R[kFOMax][9];
    Material o_mat[kFOMax];
    float4 light[kMaxLights];
    int light_type[kMaxLights];
    SpotLight spot[kMaxSpots];
    int misc[8];  // [0] next tile with entries, [1] bin overflow, [2] total entries, [3] survivors,
                  // [4] tiles with entries
    // Background tiles (no triangle touches them) handed from the compute waves to the
    // store waves, for the last kFSlots frames this workgroup published.
    unsigned char bg_tile[kFSlots][kFTilesMax];
    BgFrame bgf[kFSlots];
    int bg_next[kFSlots], bg_done[kFSlots];  // tiles taken / written, per slot
    int cons_seq[kFW];                       // frame each store wave takes tiles from
    int published, all_published;            // frames published; 1 once no more will be
    int cbar;                                // compute-wave barrier arrivals
    int next_item[2];                        // claimed work item after frame seq, in [seq & 1]
    int abort_flag;                          // 1 once a wait reached its bound: every wave stops
    // Busy tiles rendered by a compute wave and written out by a store wave: planes
    // r, g, b, nx, ny, nz, seg (as bits) and the visibility key per tile pixel.
    alignas(16) unsigned int stage_val[kFStage][7][kFTileW * kFTileH];
    alignas(16) unsigned long long stage_key[kFStage][kFTileW * kFTileH];
    StageInfo stage_info[kFStage];
    int stage_state[kFStage];  // 0 free, 2 being filled, 1 full, 3 being written
};
static_assert(sizeof(FrameLds) <= 160 * 1024, "frame LDS exceeds 160 KB");

bool frame_fits(int n_verts, int n_obj, int n_tris, int width, int height) {
    // <= 4 x 64 tiles: a tile range packs into 2-bit x and 6-bit y fields
    return n_verts <= kFVMax && n_obj <= kFOMax && n_tris < 65536 && width <= 4 * kFTileW && height <= 64 * kFTileH;
}

bool frame_fits_global(int64_t n_verts, int n_obj, int64_t n_tris, int width, int height) {
    return n_verts <= kFGVMax && n_obj <= kFGOMax && n_tris < 65536 && width <= 4 * kFTileW && height <= 64 * kFTileH;
}

// Where one frame's scene data live.  G = false: the scene fits in LDS (vertices,
// bins, survivors and object tables all in FrameLds).  G = true: a larger scene; its
// snapped vertices, tile bins and survivor list are in the workgroup's slice of the
// global frame scratch (a few hundred KB, mostly served by the L2) and its object
// tables in the LDS the vertices would otherwise take.  Every triangle is still set
// up once per frame.  Separate instantiations keep LDS accesses LDS instructions.
template <bool G>
struct FrameMem {
    int2 *xy;   // G = false: snapped (X, Y) per vertex (LDS)
    float *iw;  // G = false: 1 / w per vertex (LDS)
    int4 *v4;   // G = true: (X, Y, 1 / w as bits, 0) per vertex, one 16-byte load (scratch)
    unsigned short *bin;
    unsigned *surv;
    int bin_max, surv_max;
    int *o_tbase, *o_vbase, *o_mtb, *o_mvb, *o_nt, *o_seg, *o_vis;
    float (*o_R)[9];
    Material *o_mat;
    unsigned char *vtx_hint;

    ORRB_INLINE int2 vxy(int v) const {
        if constexpr (G) {
            const int4 q = v4[v];
            return make_int2(q.x, q.y);
        } else {
            return xy[v];
        }
    }
    // (X, Y, 1 / w as bits, 0)
    ORRB_INLINE int4 vall(int v) const {
        if constexpr (G) {
            return v4[v];
        } else {
            const int2 p = xy[v];
            return make_int4(p.x, p.y, __float_as_int(iw[v]), 0);
        }
    }
    ORRB_INLINE void vput(int v, int X, int Y, float w) const {
        if constexpr (G)
            v4[v] = make_int4(X, Y, __float_as_int(w), 0);
        else {
            xy[v] = make_int2(X, Y);
            iw[v] = w;
        }
    }
};

template <bool G>
ORRB_INLINE FrameMem<G> frame_mem(const RenderArgs &a, FrameLds &S) {
    FrameMem<G> F;
    if constexpr (G) {
        char *base = a.fscratch + (int64_t)blockIdx.x * a.fscratch_stride;
        const int64_t nv = a.fs_verts;
        F.xy = nullptr;
        F.iw = nullptr;
        F.v4 = reinterpret_cast<int4 *>(base);
        F.surv = reinterpret_cast<unsigned *>(F.v4 + nv);
        F.bin = reinterpret_cast<unsigned short *>(F.surv + a.fs_surv);
        F.bin_max = a.fs_bins;
        F.surv_max = a.fs_surv;
        F.o_tbase = S.m.g.o_tbase;
        F.o_vbase = S.m.g.o_vbase;
        F.o_mtb = S.m.g.o_mtb;
        F.o_mvb = S.m.g.o_mvb;
        F.o_nt = S.m.g.o_nt;
        F.o_seg = S.m.g.o_seg;
        F.o_vis = S.m.g.o_vis;
        F.o_R = S.m.g.o_R;
        F.o_mat = S.m.g.o_mat;
        F.vtx_hint = S.m.g.vtx_hint;
    } else {
        F.xy = S.m.v.XY;
        F.iw = S.m.v.iw;
        F.v4 = nullptr;
        F.surv = S.u.surv;
        F.bin = S.bin;
        F.bin_max = kFBinMax;
        F.surv_max = kFSurvMax;
        F.o_tbase = S.o_tbase;
        F.o_vbase = S.o_vbase;
        F.o_mtb = S.o_mtb;
        F.o_mvb = S.o_mvb;
        F.o_nt = S.o_nt;
        F.o_seg = S.o_seg;
        F.o_vis = S.o_vis;
        F.o_R = S.o_R;
        F.o_mat = S.o_mat;
        F.vtx_hint = S.vtx_hint;
    }
    return F;
}

// Object owning element x (a scene triangle or vertex): start from the hint of x's
// 64-element block and step forward over the objects that begin at or before x.
ORRB_INLINE int slot_hint(const int *base, int n, const unsigned char *hint, int x) {
    int k = hint[x / kFHint];
    if (k & 0x80) return k & 0x7f;  // the whole block lies in one object
    while (k + 1 < n && base[k + 1] <= x) ++k;
    return k;
}

// Hint of block b: the object holding element b * kFHint, bit 7 set when no other
// object starts inside the block.
ORRB_INLINE unsigned char object_hint(const int *base, int n, int b) {
    const int k = find_slot(base, n, b * kFHint);
    const bool one = k + 1 >= n || base[k + 1] > b * kFHint + kFHint - 1;
    return (unsigned char)(k | (one ? 0x80 : 0));
}

// Scene triangle t of object k and its mesh triangle (mesh-local vertex indices).
template <bool G>
ORRB_INLINE int4 frame_tri(const RenderArgs &a, const FrameMem<G> &F, int k, int t) {
    return a.mesh_tri[F.o_mtb[k] + (t - F.o_tbase[k])];
}

// Set-up of scene triangle t (object k, mesh triangle tri): front-facing, valid, with
// pixel centres in [cx0, cx1] x [cy0, cy1].  Vertices in positive-area order a, b, c.
struct TriSetup {
    int xa, ya, xb, yb, xc, yc;
    int i0, j0, i1, j1;  // pixel-centre range inside the clip box
    int va, vb, vc;      // vertex indices
    float iwa, iwb, iwc; // 1 / w of the vertices (tile set-up only)
    long long area;
};

// Set-up of a binned triangle (front-facing with valid vertices, as checked when it was
// binned) clipped to the tile [x0, x1] x [y0, y1]: false if its pixel-centre range
// misses the tile.  Also returns the edge flags and the area as a float, the area from
// 24-bit products when the triangle is small (the same integer as the 64-bit form).
template <bool G>
ORRB_INLINE bool tile_setup(const FrameMem<G> &F, int k, int4 tri, int x0, int y0, int x1, int y1, TriSetup &T,
                            int &flags, float &area) {
    const int vb = F.o_vbase[k];
    const int i0v = vb + tri.x, i1v = vb + tri.y, i2v = vb + tri.z;
    const int4 pa = F.vall(i0v), pb = F.vall(i2v), pc = F.vall(i1v);
    const int xa = pa.x, xb = pb.x, xc = pc.x;
    const int ya = pa.y, yb = pb.y, yc = pc.y;
    const int xmin = min(xa, min(xb, xc)), xmax = max(xa, max(xb, xc));
    const int ymin = min(ya, min(yb, yc)), ymax = max(ya, max(yb, yc));
    T.i0 = max(ceil256(xmin - 128), x0);
    T.i1 = min(floor256(xmax - 128), x1);
    T.j0 = max(ceil256(ymin - 128), y0);
    T.j1 = min(floor256(ymax - 128), y1);
    if (T.i0 > T.i1 || T.j0 > T.j1) return false;
    T.xa = xa; T.ya = ya; T.xb = xb; T.yb = yb; T.xc = xc; T.yc = yc;
    T.va = i0v; T.vb = i2v; T.vc = i1v;
    T.iwa = __int_as_float(pa.z); T.iwb = __int_as_float(pb.z); T.iwc = __int_as_float(pc.z);
    flags = top_left(xc - xb, yc - yb) | (top_left(xa - xc, ya - yc) << 1) | (top_left(xb - xa, yb - ya) << 2) |
            (max(xmax - xmin, ymax - ymin) > kSmallExtent ? 8 : 0);
    if (!(flags & 8))
        area = (float)(__mul24(xb - xa, yc - ya) - __mul24(yb - ya, xc - xa));
    else
        area = (float)((long long)(xb - xa) * (yc - ya) - (long long)(yb - ya) * (xc - xa));
    return true;
}

// (Hidden objects need no test: their vertices are all marked invalid.)
template <bool G>
ORRB_INLINE bool frame_setup(const FrameMem<G> &F, int k, int4 tri, int cx0, int cy0, int cx1, int cy1, TriSetup &T) {
    const int vb = F.o_vbase[k];
    const int i0v = vb + tri.x, i1v = vb + tri.y, i2v = vb + tri.z;
    const int2 p0 = F.vxy(i0v), p1 = F.vxy(i1v), p2 = F.vxy(i2v);
    const int x0 = p0.x, x1 = p1.x, x2 = p2.x;
    if (x0 == kInvalidX || x1 == kInvalidX || x2 == kInvalidX) return false;
    const int y0 = p0.y, y1 = p1.y, y2 = p2.y;
    const int xmin = min(x0, min(x1, x2)), xmax = max(x0, max(x1, x2));
    const int ymin = min(y0, min(y1, y2)), ymax = max(y0, max(y1, y2));
    T.i0 = max(ceil256(xmin - 128), cx0);
    T.i1 = min(floor256(xmax - 128), cx1);
    T.j0 = max(ceil256(ymin - 128), cy0);
    T.j1 = min(floor256(ymax - 128), cy1);
    if (T.i0 > T.i1 || T.j0 > T.j1) return false;
    // exact area: 24-bit products when the extent allows (|A| < 2^29), else 64-bit
    const long long A = max(xmax - xmin, ymax - ymin) <= kSmallExtent
                            ? (long long)(__mul24(x1 - x0, y2 - y0) - __mul24(y1 - y0, x2 - x0))
                            : (long long)(x1 - x0) * (y2 - y0) - (long long)(y1 - y0) * (x2 - x0);
    if (A >= 0) return false;
    T.xa = x0; T.ya = y0; T.xb = x2; T.yb = y2; T.xc = x1; T.yc = y1;
    T.va = i0v; T.vb = i2v; T.vc = i1v;
    T.area = -A;
    return true;
}

// Snap vertex v (object k, object-space position p) into the LDS vertex arrays.
// Returns the vertex's cull reason (Snapped::cull; 0 for hidden objects).
template <bool G>
ORRB_INLINE int frame_vertex(const FrameLds &S, const FrameMem<G> &F, int v, int k, float4 p, double fx, double fy,
                             double cx, double cy, double nearp) {
    int X = kInvalidX, Y = 0, cull = 0;
    float iw = 0.f;
    if (F.o_vis[k]) {
        double M[12];
#pragma unroll
        for (int q = 0; q < 12; ++q) M[q] = S.u.M[k][q];
        const Snapped s = snap_vertex(M, p, fx, fy, cx, cy, nearp);
        cull = s.cull;
        if (s.valid) {
            X = s.X;
            Y = s.Y;
            iw = s.iw;
        }
    }
    F.vput(v, X, Y, iw);
    return cull;
}

// Per-tile counts and the survivor entry of a set-up triangle.
ORRB_INLINE unsigned frame_count(FrameLds &S, int t, const TriSetup &T, int ntx) {
    // pixel ranges are clipped to the frame, so non-negative: plain shifts
    const int tx0 = (unsigned)T.i0 / kFTileW, tx1 = (unsigned)T.i1 / kFTileW;
    const int ty0 = (unsigned)T.j0 / kFTileH, ty1 = (unsigned)T.j1 / kFTileH;
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) atomicAdd(&S.cnt[ty * ntx + tx], 1);
    return ((unsigned)t << 16) | (unsigned)(tx0 | (tx1 << 2) | (ty0 << 4) | (ty1 << 10));
}

template <bool G>
ORRB_INLINE void frame_append(FrameLds &S, const FrameMem<G> &F, bool keep, unsigned entry, int lane) {
    const unsigned long long m = __ballot(keep);
    int wb = 0;
    if (lane == 0 && m) wb = atomicAdd(&S.misc[3], __popcll(m));
    wb = __builtin_amdgcn_readlane(wb, 0);
    if (keep) {
        const int slot = wb + lanes_below(m);
        if (slot < F.surv_max) F.surv[slot] = entry;
    }
}

// Four horizontally adjacent pixels of one plane: one 16-byte store when the group is
// whole and 16-byte aligned, else one store per pixel inside the frame.  Plain stores:
// the L2 merges a tile's 256-byte row segments with its neighbours' into whole lines,
// which non-temporal stores forgo.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

ORRB_INLINE void store4f(float *p, const float *v, bool vec, int n) {
    if (vec) {
        *reinterpret_cast<f32x4 *>(p) = f32x4{v[0], v[1], v[2], v[3]};
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q < n) p[q] = v[q];
    }
}

ORRB_INLINE void store4i(int *p, const int *v, bool vec, int n) {
    if (vec) {
        *reinterpret_cast<i32x4 *>(p) = i32x4{v[0], v[1], v[2], v[3]};
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q < n) p[q] = v[q];
    }
}

// Background (no fragment) for four adjacent pixels: rgb, depth, normal 0, seg and
// tri_id -1, vis the empty key.
template <bool AUX>
ORRB_INLINE void store_background4(const RenderArgs &a, int64_t po, int64_t HW, int64_t pix, bool vec, int n, int f,
                                   int i, int j, PostCache &pc) {
    // materialized at each use: hoisted out of the tile loops these constants get
    // spilled, and their reloads would wait for every earlier store of the wave
    float z;
    int m;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    asm volatile("v_mov_b32 %0, -1" : "=v"(m));
    const float zf[4] = {z, z, z, z};
    const int mi[4] = {m, m, m, m};
    if (a.out_rgb) {
        store4f(a.out_rgb + 3 * po + pix, zf, vec, n);
        store4f(a.out_rgb + 3 * po + HW + pix, zf, vec, n);
        store4f(a.out_rgb + 3 * po + 2 * HW + pix, zf, vec, n);
    }
    if (a.out_depth) store4f(a.out_depth + po + pix, zf, vec, n);
    if (a.out_normal) {
        store4f(a.out_normal + 3 * po + pix, zf, vec, n);
        store4f(a.out_normal + 3 * po + HW + pix, zf, vec, n);
        store4f(a.out_normal + 3 * po + 2 * HW + pix, zf, vec, n);
    }
    if (a.out_seg) store4i(a.out_seg + po + pix, mi, vec, n);
    if (a.out_tri) store4i(a.out_tri + po + pix, mi, vec, n);
    if (a.out_vis) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q < n) a.out_vis[po + pix + q] = kEmptyKey;
    }
    if (AUX && a.out_alpha) store4f(a.out_alpha + po + pix, zf, vec, n);
    if (AUX && fused_rgb8(a)) store_codes4(a, pc, f, po, HW, pix, i, j, nullptr, vec, n);
}

// ---- synchronization of the persistent frame workgroup ----
//
// The 12 compute waves render the workgroup's frames one after another and
// synchronize among themselves with an LDS counter (the 4 store waves never join, so
// the hardware barrier cannot be used).  After each frame's tile scan, wave 0 publishes
// the frame's background tiles into one of kFSlots slots; the store waves take them
// from per-slot counters and write them while the compute waves go on.  Every wait is
// bounded by kFSpinCap polls.  A wait that reaches the bound means a peer wave stopped
// making progress: the workgroup then stops (every wait ends at once and no wave starts
// new work), so the kernel ends promptly with the unfinished frames' pixels
// unspecified, and the event is counted for the call and for the device.

// Waits that reached kFSpinCap on this device since the library was loaded; read by
// orrb_wait_timeouts.
__device__ unsigned int g_wait_timeouts;

ORRB_INLINE int lds_load(const int *p) { return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP); }
ORRB_INLINE void lds_store(int *p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP); }

ORRB_INLINE bool frame_aborted(FrameLds &S) { return lds_load(&S.abort_flag) != 0; }

// A wait reached its bound: stop the workgroup (counted once per workgroup).
ORRB_INLINE void wait_bound_reached(const RenderArgs &a, FrameLds &S) {
    if (atomicExch(&S.abort_flag, 1) == 0) {
        atomicAdd(&g_wait_timeouts, 1u);
        stat_add(a, ORRB_STAT_WAIT_TIMEOUTS, 1u);
    }
}

// Barrier of the compute waves; true if the workgroup has stopped.  G: the frame also
// keeps data in global scratch, so the fences cover global memory too.
template <bool G = false>
ORRB_INLINE bool frame_barrier(const RenderArgs &a, FrameLds &S, int &gen) {
    gen += kFCW;
    if constexpr (G)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    else
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    int stop = 0;
    if (lane_id() == 0) {
        atomicAdd(&S.cbar, 1);
        unsigned spin = 0;
        for (; lds_load(&S.cbar) < gen && !frame_aborted(S) && spin < kFSpinCap; ++spin) __builtin_amdgcn_s_sleep(1);
        if (spin == kFSpinCap) wait_bound_reached(a, S);
        stop = frame_aborted(S);
    }
    stop = __builtin_amdgcn_readlane(stop, 0);
    __builtin_amdgcn_wave_barrier();
    if constexpr (G)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    else
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    return stop != 0;
}

// 16-byte stores possible for the frame: width and offset multiples of 4 pixels and
// every output 16-byte aligned.
ORRB_INLINE bool frame_vec(const RenderArgs &a, int W, int64_t po) {
    const uintptr_t align = (uintptr_t)a.out_rgb | (uintptr_t)a.out_depth | (uintptr_t)a.out_normal |
                            (uintptr_t)a.out_seg | (uintptr_t)a.out_tri | (uintptr_t)a.out_rgb8;
    return ((W | (int)(po & 3)) & 3) == 0 && (align & 15) == 0;
}

// Wave 0: hand frame seq's background tiles, order[n_busy .. n_tiles), to the store
// waves.  The slot is reused only after every store wave has moved past the frame that
// held it before (so none still takes from it) and all its tiles are written.
ORRB_INLINE void frame_publish(const RenderArgs &a, FrameLds &S, int seq, int f, int64_t po, int W, int H, int ntx, int n_busy,
                               int n_tiles, int lane) {
    const int slot = seq % kFSlots, n_empty = n_tiles - n_busy;
    int stop = 0;
    if (lane == 0 && seq >= kFSlots) {
        unsigned spin = 0;
        for (; spin < kFSpinCap && !frame_aborted(S); ++spin) {
            bool free = lds_load(&S.bg_done[slot]) >= S.bgf[slot].n;
            for (int w = kFCW; w < kFW; ++w) free = free && lds_load(&S.cons_seq[w]) > seq - kFSlots;
            if (free) break;
            __builtin_amdgcn_s_sleep(2);
        }
        if (spin == kFSpinCap) wait_bound_reached(a, S);
        stop = frame_aborted(S);
    }
    if (__builtin_amdgcn_readlane(stop, 0)) return;  // stopped: publish nothing
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    for (int i = lane; i < n_empty; i += kWave) S.bg_tile[slot][i] = S.order[n_busy + i];
    if (lane == 0) {
        BgFrame &b = S.bgf[slot];
        b.po = po;
        b.W = W;
        b.H = H;
        b.ntx = ntx;
        b.vec = frame_vec(a, W, po);
        b.n = n_empty;
        b.f = f;
        S.bg_next[slot] = 0;
        S.bg_done[slot] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) lds_store(&S.published, seq + 1);
}

// ---- staged busy tiles: a compute wave fills a slot, a store wave writes it out ----

// Claim a free staging slot and fill it with the background for the whole tile (each
// lane its 4-pixel group).  Waits while every slot is in use; -1 if the workgroup has
// stopped.
ORRB_INLINE int stage_begin(const RenderArgs &a, FrameLds &S, int lane, int lj, int li0) {
    int s = -1;
    if (lane == 0) {
        unsigned spin = 0;
        for (; spin < kFSpinCap && !frame_aborted(S); ++spin) {
            int k = 0;
            for (; k < kFStage; ++k)
                if (lds_load(&S.stage_state[k]) == 0 && atomicCAS(&S.stage_state[k], 0, 2) == 0) break;
            if (k < kFStage) {
                s = k;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (spin == kFSpinCap) wait_bound_reached(a, S);
    }
    s = __builtin_amdgcn_readlane(s, 0);
    if (s < 0) return -1;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    const int p = lj * kFTileW + li0;
    uint4 z4;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z4.x));
    z4.y = z4.z = z4.w = z4.x;
#pragma unroll
    for (int c = 0; c < 6; ++c) *reinterpret_cast<uint4 *>(&S.stage_val[s][c][p]) = z4;
    *reinterpret_cast<uint4 *>(&S.stage_val[s][6][p]) = make_uint4(~z4.x, ~z4.x, ~z4.x, ~z4.x);  // seg -1
    *reinterpret_cast<uint4 *>(&S.stage_key[s][p]) = make_uint4(~z4.x, ~z4.x, ~z4.x, ~z4.x);
    *reinterpret_cast<uint4 *>(&S.stage_key[s][p + 2]) = make_uint4(~z4.x, ~z4.x, ~z4.x, ~z4.x);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return s;
}

ORRB_INLINE void stage_pixel(FrameLds &S, int s, int p, const PixelOut &o, int seg, unsigned long long key) {
    S.stage_val[s][0][p] = __float_as_uint(o.r0);
    S.stage_val[s][1][p] = __float_as_uint(o.r1);
    S.stage_val[s][2][p] = __float_as_uint(o.r2);
    S.stage_val[s][3][p] = __float_as_uint(o.n0);
    S.stage_val[s][4][p] = __float_as_uint(o.n1);
    S.stage_val[s][5][p] = __float_as_uint(o.n2);
    S.stage_val[s][6][p] = (unsigned)seg;
    S.stage_key[s][p] = key;
}

// Hand the filled slot to the store waves, with where the tile goes.
ORRB_INLINE void stage_end(FrameLds &S, int s, int f, int64_t po, int W, int H, int x0, int y0, bool vec, int lane) {
    if (lane == 0) {
        StageInfo &in = S.stage_info[s];
        in.po = po;
        in.W = W;
        in.H = H;
        in.x0 = x0;
        in.y0 = y0;
        in.vec = vec;
        in.f = f;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) lds_store(&S.stage_state[s], 1);
}

// Touch the tables phase 0 of work item `item` reads (frame, objects, poses, materials,
// view, intrinsics, lights), so that the next frame's set-up finds them in the caches
// instead of waiting on memory behind the store traffic.  Called by the first compute
// wave that runs out of tiles, while the others finish theirs.
ORRB_INLINE void frame_warm(const RenderArgs &a, int item, int lane) {
    if (item >= a.n_fitems) return;
    const int f = a.fitems[item];
    const FrameInfo fi = a.frames[f];
    int acc = 0;
    if (lane < fi.n_obj) {
        const int o = fi.obj_begin + lane;
        const float *pose = a.pose + 12 * (int64_t)o;
        acc += a.objs[o].n_verts + a.seg[o] + a.visible[o] + __float_as_int(pose[0]) + __float_as_int(pose[11]) +
               __float_as_int(a.roughness[o]) + __float_as_int(a.specular[o]) + __float_as_int(a.albedo[3 * o]);
    }
    if (lane < fi.n_lights) {
        const int l = fi.light_begin + lane;
        acc += a.light_type[l] + __float_as_int(a.light_vec[3 * l]) + __float_as_int(a.light_intensity[l]);
    }
    if (lane == 0)
        acc += __float_as_int(a.view[12 * (int64_t)f]) + __float_as_int(a.view[12 * (int64_t)f + 11]) +
               __float_as_int(a.intr[4 * (int64_t)f]) + __float_as_int(a.near_plane[f]) + __float_as_int(a.exposure[f]);
    asm volatile("" ::"v"(acc));
}

// The workgroup's work item after frame `seq` (item `item`), found by the first compute
// wave that runs out of tiles: with the dynamic schedule it claims the next frame from
// the counter and leaves it in LDS for the other waves, read after the frame's last
// barrier.  The wave then touches that item's tables (frame_warm).
ORRB_INLINE void frame_next(const RenderArgs &a, FrameLds &S, int item, int seq, int lane) {
    int next = item + (int)gridDim.x;
    if (a.f_dynamic) {
        if (lane == 0) {
            next = a.f_grid + (int)atomicAdd(a.queue + kFrameQueue, 1u);
            S.next_item[seq & 1] = next;
        }
        next = __builtin_amdgcn_readlane(next, 0);
    }
    frame_warm(a, next, lane);
}

// Store wave: write staged tile s (every output plane) and free the slot.
template <bool AUX>
ORRB_INLINE void stage_write(const RenderArgs &a, FrameLds &S, int s, int lj, int li0, int lane, PostCache &pc) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    const StageInfo in = S.stage_info[s];
    const int p = lj * kFTileW + li0;
    const int x1 = min(in.x0 + kFTileW, in.W) - 1, y1 = min(in.y0 + kFTileH, in.H) - 1;
    const int j = in.y0 + lj, i0 = in.x0 + li0;
    const int n = j <= y1 ? max(0, min(4, x1 - i0 + 1)) : 0;
    float v[7][4];
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        const uint4 u = *reinterpret_cast<const uint4 *>(&S.stage_val[s][c][p]);
        v[c][0] = __uint_as_float(u.x);
        v[c][1] = __uint_as_float(u.y);
        v[c][2] = __uint_as_float(u.z);
        v[c][3] = __uint_as_float(u.w);
    }
    unsigned long long key[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) key[q] = S.stage_key[s][p + q];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");  // slot contents read
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) lds_store(&S.stage_state[s], 0);
    if (n == 0) return;
    const bool vec = in.vec && n == 4;
    const int64_t HW = (int64_t)in.W * in.H, po = in.po, pix = (int64_t)j * in.W + i0;
    float z[4];
    int seg[4], tri[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool e = key[q] == kEmptyKey;
        z[q] = e ? 0.f : __uint_as_float((unsigned)(key[q] >> 32));
        tri[q] = e ? -1 : (int)(unsigned)(key[q] & 0xffffffffu);
        seg[q] = __float_as_int(v[6][q]);
    }
    if (a.out_rgb) {
        store4f(a.out_rgb + 3 * po + pix, v[0], vec, n);
        store4f(a.out_rgb + 3 * po + HW + pix, v[1], vec, n);
        store4f(a.out_rgb + 3 * po + 2 * HW + pix, v[2], vec, n);
    }
    if (a.out_depth) store4f(a.out_depth + po + pix, z, vec, n);
    if (a.out_normal) {
        store4f(a.out_normal + 3 * po + pix, v[3], vec, n);
        store4f(a.out_normal + 3 * po + HW + pix, v[4], vec, n);
        store4f(a.out_normal + 3 * po + 2 * HW + pix, v[5], vec, n);
    }
    if (a.out_seg) store4i(a.out_seg + po + pix, seg, vec, n);
    if (a.out_tri) store4i(a.out_tri + po + pix, tri, vec, n);
    if (a.out_vis) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q < n) a.out_vis[po + pix + q] = key[q];
    }
    if (AUX && a.out_alpha) {
        float al[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) al[q] = key[q] == kEmptyKey ? 0.f : 1.f;
        store4f(a.out_alpha + po + pix, al, vec, n);
    }
    if (AUX && fused_rgb8(a)) {  // the staged rgb (background 0) encoded on its way out
        const float rv[3][4] = {{v[0][0], v[0][1], v[0][2], v[0][3]},
                                {v[1][0], v[1][1], v[1][2], v[1][3]},
                                {v[2][0], v[2][1], v[2][2], v[2][3]}};
        store_codes4(a, pc, in.f, po, HW, pix, i0, j, rv, vec, n);
    }
}

// Pace a store wave: at most kFPace store instructions in flight, so the CU's memory
// queue does not fill with stores ahead of the compute waves' loads.
ORRB_INLINE void store_pace() { asm volatile("s_waitcnt vmcnt(%0)" ::"n"(kFPace) : "memory"); }

// Take the next background tile of slot `slot` and write it (each lane its 4-pixel row
// group); false when the slot's tiles are all taken.
template <bool AUX>
ORRB_INLINE bool bg_write_next(const RenderArgs &a, FrameLds &S, int slot, int lj, int li0, int lane, PostCache &pc) {
    int i = 0;
    if (lane == 0) i = atomicAdd(&S.bg_next[slot], 1);
    i = __builtin_amdgcn_readlane(i, 0);
    const BgFrame b = S.bgf[slot];
    if (i >= b.n) return false;
    const int t = S.bg_tile[slot][i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");  // slot read
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) atomicAdd(&S.bg_done[slot], 1);
    const int tyi = t / b.ntx, txi = t - tyi * b.ntx;
    const int x0 = txi * kFTileW, y0 = tyi * kFTileH;
    const int x1 = min(x0 + kFTileW, b.W) - 1, y1 = min(y0 + kFTileH, b.H) - 1;
    const int j = y0 + lj, i0 = x0 + li0;
    const int n_in = j <= y1 ? max(0, min(4, x1 - i0 + 1)) : 0;
    if (n_in > 0)
        store_background4<AUX>(a, b.po, (int64_t)b.W * b.H, (int64_t)j * b.W + i0, b.vec && n_in == 4, n_in, b.f, i0,
                               j, pc);
    return true;
}

// Write the background of published tiles until every frame is published and taken.
// Store waves run this from the start; compute waves join after their last frame,
// starting at the oldest frame that may still have tiles.
template <bool AUX>
ORRB_INLINE void frame_drain(const RenderArgs &a, FrameLds &S, int wave, int lj, int li0, int lane) {
    const bool store_wave = wave >= kFCW;
    // a wave kept for staged tiles answers them without delay (no background tiles)
    const bool staged_only = kFStageWave && wave == kFW - 1;
    int my = store_wave ? 0 : max(0, lds_load(&S.published) - kFSlots);
    PostCache pc;  // grading constants of the last frame this wave encoded (fused rgb8)
    while (true) {
        // 1: staged tile st claimed, 2: frame my is published, 0: nothing more will come
        int action = 0, st = 0;
        if (lane == 0) {
            unsigned spin = 0;
            for (; spin < kFSpinCap && !frame_aborted(S); ++spin) {
                for (int k = 0; k < kFStage && !action; ++k)
                    if (lds_load(&S.stage_state[k]) == 1 && atomicCAS(&S.stage_state[k], 1, 3) == 1) {
                        action = 1;
                        st = k;
                    }
                if (action) break;
                const int fin = lds_load(&S.all_published);
                if (!staged_only && my < lds_load(&S.published)) {
                    action = 2;
                    break;
                }
                if (fin) {  // compute waves are done: only full slots may remain
                    bool pending = false;
                    for (int k = 0; k < kFStage; ++k) pending = pending || lds_load(&S.stage_state[k]) == 1;
                    if (!pending) break;
                    continue;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            if (spin == kFSpinCap) wait_bound_reached(a, S);
            if (frame_aborted(S)) action = 0;
        }
        action = __builtin_amdgcn_readlane(action, 0);
        if (!action) break;
        if (action == 1) {
            stage_write<AUX>(a, S, __builtin_amdgcn_readlane(st, 0), lj, li0, lane, pc);
            if (store_wave && !staged_only) store_pace();
            continue;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        if (!bg_write_next<AUX>(a, S, my % kFSlots, lj, li0, lane, pc)) {  // the frame's tiles are all taken
            ++my;
            if (store_wave && lane == 0) lds_store(&S.cons_seq[wave], my);
            continue;
        }
        if (store_wave) store_pace();
    }
}

// With the auxiliary outputs (8-bit encoding with grain, alpha) the store waves carry
// more per pixel than the compute waves produce, so a compute wave with no busy tile
// left writes background tiles of frame seq (taken from the same counter as the store
// waves) while the other compute waves finish.  The plain kernel leaves this out: its
// store waves keep up, so the same help only delays the end of each frame (measured
// 8 % slower).
template <bool AUX>
ORRB_INLINE void frame_bg_help(const RenderArgs &a, FrameLds &S, int seq, int lj, int li0, int lane) {
    PostCache pc;
    while (bg_write_next<AUX>(a, S, seq % kFSlots, lj, li0, lane, pc)) {
    }
}

// One frame rendered by the compute waves (phases 0-4 below); true if the workgroup has
// stopped.  G selects where the scene's data live (FrameMem).
template <bool AUX, bool G, int SHADE>
ORRB_INLINE bool frame_render(const RenderArgs &a, FrameLds &S, int item, int seq, int &gen) {
    const FrameMem<G> F = frame_mem<G>(a, S);
    // Thread indices made opaque per frame: address arithmetic derived from them is
    // recomputed inside the frame instead of being hoisted (and spilled) across frames.
    int tid = threadIdx.x, lane = tid & (kWave - 1);
    asm volatile("" : "+v"(tid), "+v"(lane));
    const int wave = __builtin_amdgcn_readfirstlane(tid) / kWave;
    const int lj = lane / (kFTileW / 4), li0 = (lane % (kFTileW / 4)) * 4;  // the lane's 4-pixel row group
    const int f = a.fitems[item];
    const FrameInfo fi = a.frames[f];
    const int n_obj = fi.n_obj, W = fi.width, H = fi.height;
    const int ntx = (W + kFTileW - 1) / kFTileW, nty = (H + kFTileH - 1) / kFTileH, n_tiles = ntx * nty;

    // ---- phase 0: per-object tables, matrices, lights ----
    if (tid < n_obj) {
        const int o = fi.obj_begin + tid;
        const ObjInfo ob = a.objs[o];
        F.o_tbase[tid] = ob.scene_tbase;
        F.o_vbase[tid] = ob.scene_vbase;
        F.o_mtb[tid] = ob.mesh_tbegin;
        F.o_mvb[tid] = ob.mesh_vbegin;
        F.o_nt[tid] = ob.n_tris;
        F.o_seg[tid] = a.seg[o];
        F.o_vis[tid] = a.visible[o];
        F.o_mat[tid] = object_material(a, o);
    }
    for (int e = tid; e < 12 * n_obj; e += kFCT) {
        const int k = e / 12, q = e - 12 * k;
        const double m = compose_entry(a.view + 12 * (int64_t)f, a.pose + 12 * (int64_t)(fi.obj_begin + k), q);
        S.u.M[k][q] = m;
        if ((q & 3) != 3) F.o_R[k][(q >> 2) * 3 + (q & 3)] = (float)m;
    }
    if (tid < fi.n_lights) {
        if constexpr (SHADE == 1 || SHADE == 3) {
            frame_light(a, f, fi, tid, S.light, S.light_type, S.spot);
        } else if constexpr (SHADE != 4) {
            const int l = fi.light_begin + tid;
            S.light[tid] = view_light(a.view + 12 * (int64_t)f, a.light_vec + 3 * (int64_t)l, a.light_type[l],
                                      a.light_intensity[l]);
            S.light_type[tid] = a.light_type[l];
        }
    }
    for (int t = tid; t <= n_tiles; t += kFCT) S.cnt[t] = 0;
    if (tid < 8) S.misc[tid] = 0;
    const int n_verts = n_obj > 0 ? a.objs[fi.obj_begin + n_obj - 1].scene_vbase + a.objs[fi.obj_begin + n_obj - 1].n_verts : 0;
    if (frame_barrier<G>(a, S, gen)) return true;
    const int n_tris = n_obj > 0 ? F.o_tbase[n_obj - 1] + F.o_nt[n_obj - 1] : 0;
    if (AUX && a.out_track && tid < n_obj) {
        const float *K = a.intr + 4 * (int64_t)f;
        track_init(a.out_track + fi.track_base + tid, S.u.M[tid][3], S.u.M[tid][7], S.u.M[tid][11], K[0], K[1], K[2],
                   K[3]);
        // the record must be in memory before any wave adds to it (after the barriers)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    for (int b = tid; b * kFHint < n_tris; b += kFCT) S.tri_hint[b] = object_hint(F.o_tbase, n_obj, b);
    for (int b = tid; b * kFHint < n_verts; b += kFCT) F.vtx_hint[b] = object_hint(F.o_vbase, n_obj, b);
    if (frame_barrier<G>(a, S, gen)) return true;

    // ---- phase 1: vertices, kFVN per thread per pass; the next pass's positions are
    // loaded before the current pass is transformed, hiding the load latency ----
    {
        const float *K = a.intr + 4 * (int64_t)f;
        const double fx = K[0], fy = K[1], cx = K[2], cy = K[3], nearp = a.near_plane[f];
        // vertex v (clamped to the last one) of object k: its mesh position
        auto vload = [&](int v, int &k) {
            const int u = min(v, n_verts - 1);
            k = slot_hint(F.o_vbase, n_obj, F.vtx_hint, u);
            return a.mesh_pos[F.o_mvb[k] + (u - F.o_vbase[k])];
        };
        int kn[kFVN];
        float4 pn[kFVN];
        unsigned n_near = 0, n_guard = 0;
#pragma unroll
        for (int r = 0; r < kFVN; ++r) {
            kn[r] = 0;
            pn[r] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (n_verts > 0) pn[r] = vload(tid + r * kFCT, kn[r]);
        }
        for (int base = 0; base < n_verts; base += kFVN * kFCT) {
            float4 p[kFVN];
            int k[kFVN];
#pragma unroll
            for (int r = 0; r < kFVN; ++r) {
                p[r] = pn[r];
                k[r] = kn[r];
            }
            if (base + kFVN * kFCT < n_verts) {
#pragma unroll
                for (int r = 0; r < kFVN; ++r) pn[r] = vload(base + (kFVN + r) * kFCT + tid, kn[r]);
            }
#pragma unroll
            for (int r = 0; r < kFVN; ++r) {
                const int v = base + r * kFCT + tid;
                if (v < n_verts) {
                    const int cull = frame_vertex(S, F, v, k[r], p[r], fx, fy, cx, cy, nearp);
                    n_near += cull == 1;
                    n_guard += cull == 2;
                }
            }
        }
        stat_add(a, ORRB_STAT_NEAR_VERTICES, n_near);  // rare: one atomic per thread that saw one
        stat_add(a, ORRB_STAT_GUARD_VERTICES, n_guard);
    }
    if (frame_barrier<G>(a, S, gen)) return true;

    // ---- phase 2: set-up, per-tile counts, survivor list; kFTN triangles per thread
    // per pass, the next pass's mesh triangles loaded ahead ----
    {
        auto tload = [&](int t, int &k) {
            const int u = min(t, n_tris - 1);  // out-of-range lanes load the last triangle
            k = slot_hint(F.o_tbase, n_obj, S.tri_hint, u);
            return frame_tri(a, F, k, u);
        };
        int kn[kFTN];
        int4 tn[kFTN];
#pragma unroll
        for (int r = 0; r < kFTN; ++r) {
            kn[r] = 0;
            tn[r] = make_int4(0, 0, 0, 0);
            if (n_tris > 0) tn[r] = tload(tid + r * kFCT, kn[r]);
        }
        for (int base = 0; base < n_tris; base += kFTN * kFCT) {
            int4 tr[kFTN];
            int k[kFTN];
#pragma unroll
            for (int r = 0; r < kFTN; ++r) {
                tr[r] = tn[r];
                k[r] = kn[r];
            }
            if (base + kFTN * kFCT < n_tris) {
#pragma unroll
                for (int r = 0; r < kFTN; ++r) tn[r] = tload(base + (kFTN + r) * kFCT + tid, kn[r]);
            }
#pragma unroll
            for (int r = 0; r < kFTN; ++r) {
                const int t = base + r * kFCT + tid;
                TriSetup T;
                const bool keep = t < n_tris && frame_setup(F, k[r], tr[r], 0, 0, W - 1, H - 1, T);
                const unsigned e = keep ? frame_count(S, t, T, ntx) : 0u;
                frame_append(S, F, keep, e, lane);
            }
        }
    }
    if (frame_barrier<G>(a, S, gen)) return true;
    if (wave == 0) {  // exclusive scan of n_tiles <= 256 counts (4 per lane) and the tile order
        int c[4], local = 0, ne = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int t = lane * 4 + q;
            c[q] = t < n_tiles ? S.cnt[t] : 0;
            local += c[q];
            ne += c[q] > 0;
        }
        const int incl = wave_scan_add(local), incl_ne = wave_scan_add(ne);
        const int total_ne = __builtin_amdgcn_readlane(incl_ne, kWave - 1);
        const bool overflow = __builtin_amdgcn_readlane(incl, kWave - 1) > F.bin_max;
        int run = incl - local, run_ne = incl_ne - ne;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int t = lane * 4 + q;
            if (t < n_tiles) {
                S.off[t] = run;
                S.cnt[t] = run;  // becomes the scatter cursor
                // without bins every tile is rasterized, in plain order; otherwise tiles
                // with entries first
                S.order[overflow ? t : (c[q] > 0 ? run_ne : total_ne + t - run_ne)] = (unsigned char)t;
            }
            run += c[q];
            run_ne += c[q] > 0;
        }
        if (lane == kWave - 1) {
            S.off[n_tiles] = incl;
            S.misc[2] = incl;
            S.misc[1] = overflow;
            S.misc[4] = overflow ? n_tiles : total_ne;
            stat_add(a, ORRB_STAT_BIN_OVERFLOW, overflow ? 1u : 0u);
        }
        // queue the tiles no triangle touches for the store waves
        const int n_busy = overflow ? n_tiles : total_ne;
        frame_publish(a, S, seq, f, fi.pixel_offset, W, H, ntx, n_busy, n_tiles, lane);
    }
    if (frame_barrier<G>(a, S, gen)) return true;
    const bool overflow = S.misc[1] != 0;

    // ---- phase 3: scatter triangle IDs into the tile bins ----
    const int n_surv = S.misc[3];
    if (!overflow && n_surv <= F.surv_max) {
        for (int k = tid; k < n_surv; k += kFCT) {
            const unsigned e = F.surv[k];
            const int tx0 = e & 3, tx1 = (e >> 2) & 3, ty0 = (e >> 4) & 63, ty1 = (e >> 10) & 63;
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) F.bin[atomicAdd(&S.cnt[ty * ntx + tx], 1)] = (unsigned short)(e >> 16);
        }
    } else if (!overflow) {  // too many survivors to remember: set them up again
        if (tid == 0) stat_add(a, ORRB_STAT_SURVIVOR_RESETUP, 1u);
        for (int t = tid; t < n_tris; t += kFCT) {
            const int k = slot_hint(F.o_tbase, n_obj, S.tri_hint, t);
            TriSetup T;
            if (!frame_setup(F, k, frame_tri(a, F, k, t), 0, 0, W - 1, H - 1, T)) continue;
            for (int ty = (unsigned)T.j0 / kFTileH; ty <= (int)((unsigned)T.j1 / kFTileH); ++ty)
                for (int tx = (unsigned)T.i0 / kFTileW; tx <= (int)((unsigned)T.i1 / kFTileW); ++tx)
                    F.bin[atomicAdd(&S.cnt[ty * ntx + tx], 1)] = (unsigned short)t;
        }
    }
    if (frame_barrier<G>(a, S, gen)) return true;

    // ---- phase 4: compute waves take the tiles with bin entries, rasterize, shade and
    // write them, issuing all loads of a tile before its stores; the store waves write
    // the rest meanwhile.
    const CamF cam = frame_camera(a, f);
    const int64_t HW = (int64_t)W * H, po = fi.pixel_offset;
    const int n_busy = S.misc[4];
    const bool vec_frame = frame_vec(a, W, po);
    unsigned long long *vis = S.u.vis[wave];
    bool stopped = false;
    while (!stopped) {
        int slot = 0;
        if (lane == 0) slot = atomicAdd(&S.misc[0], 1);
        slot = __builtin_amdgcn_readlane(slot, 0);
        if (slot >= n_busy) {
            if (slot == n_busy) frame_next(a, S, item, seq, lane);
            if constexpr (AUX) frame_bg_help<AUX>(a, S, seq, lj, li0, lane);
            break;
        }
        const int t = S.order[slot];
        const int tyi = t / ntx, txi = t - tyi * ntx;
        const int x0 = txi * kFTileW, y0 = tyi * kFTileH;
        const int x1 = min(x0 + kFTileW, W) - 1, y1 = min(y0 + kFTileH, H) - 1;
        const int j = y0 + lj, i0 = x0 + li0;
        const int n_in = j <= y1 ? max(0, min(4, x1 - i0 + 1)) : 0;
        const int64_t gpix = (int64_t)j * W + i0;
#pragma unroll
        for (int q = 0; q < 4; ++q) vis[lane + 64 * q] = kEmptyKey;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // Keys in the LDS tile carry the triangle's object slot in bits 16..23 above its
        // 16-bit ID: slots do not decrease with the ID, so the (depth, ID) order is
        // unchanged, shading needs no object lookup, and the bits are cleared before the
        // key leaves the tile.  Without bins (overflow) the wave scans every triangle.
        const int e0 = overflow ? 0 : S.off[t], e1 = overflow ? n_tris : S.off[t + 1];
        for (int e = e0 + lane; e < e1; e += kWave) {
            const int tri = overflow ? e : (int)F.bin[e];
            const int k = slot_hint(F.o_tbase, n_obj, S.tri_hint, tri);
            TriSetup T;
            int flags;
            float area;
            if (overflow) {  // unbinned: the full culling set-up
                if (!frame_setup(F, k, frame_tri(a, F, k, tri), x0, y0, x1, y1, T)) continue;
                flags = tri_flags(T.xa, T.ya, T.xb, T.yb, T.xc, T.yc);
                area = (float)T.area;
                T.iwa = __int_as_float(F.vall(T.va).z);
                T.iwb = __int_as_float(F.vall(T.vb).z);
                T.iwc = __int_as_float(F.vall(T.vc).z);
            } else if (!tile_setup(F, k, frame_tri(a, F, k, tri), x0, y0, x1, y1, T, flags, area)) {
                continue;
            }
            const float iwa = T.iwa, iwb = T.iwb, iwc = T.iwc;
            if (!(flags & 8)) {  // small triangle: step the integer edge functions
                const int b0 = (flags & 1) ? 0 : 1, b1 = (flags & 2) ? 0 : 1, b2 = (flags & 4) ? 0 : 1;
                EdgeStep es = edge_start(T.xa, T.ya, T.xb, T.yb, T.xc, T.yc, (T.i0 << 8) + 128, (T.j0 << 8) + 128);
                for (int jj = T.j0; jj <= T.j1; ++jj) {
                    int e0 = es.e0, e1 = es.e1, e2 = es.e2;
                    for (int ii = T.i0; ii <= T.i1; ++ii) {
                        if (((e0 - b0) | (e1 - b1) | (e2 - b2)) >= 0) {
                            Edges ed;
                            ed.e0 = (float)e0;
                            ed.e1 = (float)e1;
                            ed.e2 = (float)e2;
                            atomicMin(&vis[(jj - y0) * kFTileW + (ii - x0)], vis_key(fragment_depth(ed, iwa, iwb, iwc, area), tri | (k << 16)));
                        }
                        e0 += es.dx0;
                        e1 += es.dx1;
                        e2 += es.dx2;
                    }
                    es.e0 += es.dy0;
                    es.e1 += es.dy1;
                    es.e2 += es.dy2;
                }
            } else {
                for (int jj = T.j0; jj <= T.j1; ++jj) {
                    for (int ii = T.i0; ii <= T.i1; ++ii) {
                        const Edges ed = edge_eval(T.xa, T.ya, T.xb, T.yb, T.xc, T.yc, (ii << 8) + 128, (jj << 8) + 128, flags);
                        if (!ed.covered) continue;
                        atomicMin(&vis[(jj - y0) * kFTileW + (ii - x0)], vis_key(fragment_depth(ed, iwa, iwb, iwc, area), tri | (k << 16)));
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();

        // covered pixels of the lane's group, then the wave's list of covered pixels
        int covq = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q < n_in && vis[lj * kFTileW + li0 + q] != kEmptyKey) covq |= 1 << q;
        unsigned char *list = S.cov[wave];
        int n_cov = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool c = (covq >> q) & 1;
            const unsigned long long m = __ballot(c);
            if (c) list[n_cov + lanes_below(m)] = (unsigned char)(lj * kFTileW + li0 + q);
            n_cov += __popcll(m);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (AUX && a.out_track) {  // tracker: the object slot of each covered pixel's key
            int sl[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                sl[q] = (covq >> q) & 1 ? (int)((unsigned)vis[lj * kFTileW + li0 + q] >> 16) & 0xff : -1;
            track_tile(a.out_track + fi.track_base, sl, x0 + li0, y0 + lj);  // frames of at most 256 x 256
        }

        // shade the covered pixels, lane-compacted (lane takes list[lane + 64 r]), in
        // passes of (up to) two per lane and put them, over the tile's background, into a
        // staging slot that a store wave writes out
        int stg = -1;
        for (int r0 = 0; r0 * kWave < n_cov; r0 += 2) {
            PixelOut o[2];
            unsigned long long kk[2];
            int sg[2], pl[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                kk[h] = kEmptyKey;
                sg[h] = -1;
                pl[h] = 0;
                const int c = (r0 + h) * kWave + lane;
                if (c >= n_cov) continue;
                const int p = list[c];
                const int pi = x0 + (int)((unsigned)p % kFTileW), pj = y0 + (int)((unsigned)p / kFTileW);
                const unsigned long long key = vis[p];
                const int tri = (int)(unsigned)(key & 0xffffu), k = (int)(unsigned)((key >> 16) & 0xffu);
                const float z = __uint_as_float((unsigned)(key >> 32));
                const int4 tv = frame_tri(a, F, k, tri);
                const int vb = F.o_vbase[k], mvb = F.o_mvb[k];
                const int va = vb + tv.x, vbb = vb + tv.z, vc = vb + tv.y;  // positive-area order
                if constexpr (SHADE == 4) {  // depth only (shadow maps): no shading
                    o[h] = PixelOut{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                } else {
                    constexpr bool kSpot = (SHADE & 1) != 0, kMat = (SHADE & 2) != 0;
                    MatTex mt;
                    if constexpr (kMat) mt = mat_inputs(a, fi.obj_begin + k, mvb, tv);
                    const int4 A = F.vall(va), B = F.vall(vbb), C = F.vall(vc);
                    o[h] = shade_pixel<kSpot, kMat>(A.x, A.y, B.x, B.y, C.x, C.y, __int_as_float(A.z),
                                                    __int_as_float(B.z), __int_as_float(C.z), a.mesh_nrm[mvb + tv.x],
                                                    a.mesh_nrm[mvb + tv.z],
                                                    a.mesh_nrm[mvb + tv.y], F.o_R[k], pi, pj, z, cam, S.light,
                                                    S.light_type, fi.n_lights, F.o_mat[k], S.spot, a.shadow_maps,
                                                    a.shadow_res, &mt, a.tex_texels, a.tex_info);
                }
                kk[h] = key & ~0xffff0000ull;
                sg[h] = F.o_seg[k];
                pl[h] = p;
                __builtin_amdgcn_sched_barrier(0);  // shade the two pixels one after the other
            }
            if (stg < 0) stg = stage_begin(a, S, lane, lj, li0);
            if (stg < 0) break;  // the workgroup has stopped
#pragma unroll
            for (int h = 0; h < 2; ++h)
                if (kk[h] != kEmptyKey) stage_pixel(S, stg, pl[h], o[h], sg[h], kk[h]);
        }
        if (stg < 0) stg = stage_begin(a, S, lane, lj, li0);
        if (stg < 0) {
            stopped = true;
            break;
        }
        stage_end(S, stg, f, po, W, H, x0, y0, vec_frame, lane);
    }
    return frame_barrier<G>(a, S, gen);  // the frame's LDS is reused by the next frame
}

// AUX: the transparency channel and the Tracker records are written (a separate
// instantiation, so the plain four-channel kernel carries none of that code).  MIXED:
// some frames keep their scene data in global scratch (frame_mem).
template <bool AUX, bool MIXED, int SHADE>
__global__ __launch_bounds__(kFT) void k_frame(RenderArgs a) {
    __shared__ FrameLds S;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    if (tid == 0) {
        S.published = S.all_published = S.cbar = S.abort_flag = 0;
        for (int k = 0; k < kFSlots; ++k) S.bgf[k].n = S.bg_next[k] = S.bg_done[k] = 0;
        for (int k = 0; k < kFStage; ++k) S.stage_state[k] = 0;
        for (int w = 0; w < kFW; ++w) S.cons_seq[w] = kFStageWave && w == kFW - 1 ? 0x7fffffff : 0;
    }
    __syncthreads();  // the only barrier of all 16 waves; compute waves use frame_barrier
    if (wave < kFCW) {
        int gen = 0;  // compute-wave barrier generation
        for (int item = blockIdx.x, seq = 0; item < a.n_fitems; ++seq) {
            const int f = a.fitems[item];
            const bool stop = MIXED && a.frames[f].mode != 0 ? frame_render<AUX, true, SHADE>(a, S, item, seq, gen)
                                                             : frame_render<AUX, false, SHADE>(a, S, item, seq, gen);
            if (stop) break;
            item = a.f_dynamic ? S.next_item[seq & 1] : item + (int)gridDim.x;  // after the frame's last barrier
        }
        if (wave == 0 && lane == 0) __hip_atomic_store(&S.all_published, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    // store waves from the start, compute waves after their last frame
    frame_drain<AUX>(a, S, wave, lane / (kFTileW / 4), (lane % (kFTileW / 4)) * 4, lane);
}

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------

hipError_t read_wait_timeouts(unsigned int *out) {
    return hipMemcpyFromSymbol(out, HIP_SYMBOL(g_wait_timeouts), sizeof(unsigned int));
}

size_t raster_lds_bytes(int tile_w, int tile_h, int bin_cap) {
    const size_t vis = sizeof(unsigned long long) * (size_t)tile_w * tile_h;
    const size_t bin = sizeof(int) * (size_t)bin_cap * 14 + sizeof(int);
    const size_t rest = sizeof(int) * (7 * kBlock + 1) + sizeof(float) * 9 * kBlock + sizeof(float4) * kMaxLights +
                        sizeof(int) * (kMaxLights + 16);
    return vis + bin + rest;
}

// Shadow cameras of the spot lights gathered per shadow frame (slot k <- light
// spot_light[k]), with the shadow frames' near plane (0.01 m).
__global__ __launch_bounds__(kBlock) void k_shadow_cams(const int32_t *spot_light, int n, const float *sview,
                                                         const float *sintr, float *view, float *intr, float *nearp) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int64_t l = spot_light[k];
#pragma unroll
    for (int q = 0; q < 12; ++q) view[12 * (int64_t)k + q] = sview[12 * l + q];
#pragma unroll
    for (int q = 0; q < 4; ++q) intr[4 * (int64_t)k + q] = sintr[4 * l + q];
    nearp[k] = 0.01f;
}

hipError_t launch_shadow_cams(const int32_t *spot_light, int n_spot, const float *shadow_view, const float *shadow_intr,
                              float *view, float *intr, float *nearp, hipStream_t stream) {
    if (n_spot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_shadow_cams, dim3((n_spot + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, spot_light, n_spot,
                       shadow_view, shadow_intr, view, intr, nearp);
    return hipGetLastError();
}

hipError_t launch_vertex(const RenderArgs &a, hipStream_t stream) {
    hipLaunchKernelGGL(k_vertex, dim3(a.n_vitems > 0 ? a.n_vitems : 1), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

template <int VIS, int CAP>
static hipError_t launch_raster_t(const RenderArgs &a, hipStream_t stream, int n_cu) {
    int grid = a.n_titems;
    if (a.persistent) {
        const size_t lds = sizeof(TileLds<VIS, CAP>);
        int per_cu = (int)((160 * 1024) / (lds + 1024));
        per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
        grid = n_cu * per_cu;
        if (grid > a.n_titems) grid = a.n_titems;
    }
    hipLaunchKernelGGL((k_raster_shade<VIS, CAP>), dim3(grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

template <int VIS>
static hipError_t launch_raster_cap(const RenderArgs &a, hipStream_t stream, int n_cu) {
    switch (a.bin_cap) {
        case 256: return launch_raster_t<VIS, 256>(a, stream, n_cu);
        case 512: return launch_raster_t<VIS, 512>(a, stream, n_cu);
        case 1024: return launch_raster_t<VIS, 1024>(a, stream, n_cu);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_raster(const RenderArgs &a, hipStream_t stream, int n_cu) {
    if (a.n_titems <= 0) return hipSuccess;
    switch (a.tile_w * a.tile_h) {
        case 256: return launch_raster_cap<256>(a, stream, n_cu);
        case 512: return launch_raster_cap<512>(a, stream, n_cu);
        case 1024: return launch_raster_cap<1024>(a, stream, n_cu);
        case 2048: return launch_raster_cap<2048>(a, stream, n_cu);
        case 4096: return launch_raster_cap<4096>(a, stream, n_cu);
    }
    return hipErrorInvalidValue;
}

__global__ void k_frame_queue_reset(unsigned int *q) {
    if (threadIdx.x == 0) *q = 0u;
}

// Persistent: one workgroup per CU (the frame LDS allows no more), each rendering
// frames blockIdx.x, blockIdx.x + gridDim.x, ... or, with the dynamic schedule, frame
// blockIdx.x and then the frames it claims (counter cleared by a one-thread kernel first:
// the workspace arrives uninitialised).
hipError_t launch_frame(const RenderArgs &a, hipStream_t stream, int n_cu) {
    if (a.n_fitems <= 0 || a.f_grid <= 0) return hipSuccess;
    if (a.f_dynamic) hipLaunchKernelGGL(k_frame_queue_reset, dim3(1), dim3(kWave), 0, stream, a.queue + kFrameQueue);
    const int grid = a.f_grid;  // the schedule's grid (at most the CU count)
    const bool aux = a.out_alpha || a.out_track || a.out_rgb8, mixed = a.fscratch != nullptr;
    const dim3 g(grid), b(kFT);
#define ORRB_FRAME(AUX_, MIXED_, SHADE_) hipLaunchKernelGGL((k_frame<AUX_, MIXED_, SHADE_>), g, b, 0, stream, a)
    switch (a.shade_mode) {
        case 4:  // depth only (shadow maps); no auxiliary outputs
            if (mixed) ORRB_FRAME(false, true, 4); else ORRB_FRAME(false, false, 4);
            break;
        case 1:  // spot lights with shadow maps
            if (aux && mixed) ORRB_FRAME(true, true, 1);
            else if (aux) ORRB_FRAME(true, false, 1);
            else if (mixed) ORRB_FRAME(false, true, 1);
            else ORRB_FRAME(false, false, 1);
            break;
        case 2:  // textured / emissive materials
            if (aux && mixed) ORRB_FRAME(true, true, 2);
            else if (aux) ORRB_FRAME(true, false, 2);
            else if (mixed) ORRB_FRAME(false, true, 2);
            else ORRB_FRAME(false, false, 2);
            break;
        case 3:  // both
            if (aux && mixed) ORRB_FRAME(true, true, 3);
            else if (aux) ORRB_FRAME(true, false, 3);
            else if (mixed) ORRB_FRAME(false, true, 3);
            else ORRB_FRAME(false, false, 3);
            break;
        default:
            if (aux && mixed) ORRB_FRAME(true, true, 0);
            else if (aux) ORRB_FRAME(true, false, 0);
            else if (mixed) ORRB_FRAME(false, true, 0);
            else ORRB_FRAME(false, false, 0);
    }
#undef ORRB_FRAME
    return hipGetLastError();
}

}  // namespace orrb
