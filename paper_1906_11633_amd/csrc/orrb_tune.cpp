// Batched form helpers on top of the C ABI: the autotuner (measures candidate
// tunings with HIP events and keeps the fastest, with a JSON-lines cache keyed by
// device and batch structure) and HIP-graph capture / replay of a render call.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <string>
#include <vector>

#include "../../include/orrb.h"
#include "orrb_device.h"

using namespace orrb;

namespace {

std::string device_key(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string k = std::string(p.gcnArchName) + "/" + std::to_string(p.multiProcessorCount) + "cu";
    for (char &c : k)
        if (c == '"' || c == '\\') c = '_';
    return k;
}

bool cache_lookup(const char *path, const std::string &dev, const std::string &lay, orrb_tuning *t, double *ms) {
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {  // the last matching entry wins
        if (line.find("\"device\": \"" + dev + "\"") == std::string::npos) continue;
        if (line.find("\"layout\": \"" + lay + "\"") == std::string::npos) continue;
        const size_t p = line.find("\"tuning\": [");
        const size_t q = line.find("\"ms\": ");
        if (p == std::string::npos || q == std::string::npos) continue;
        orrb_tuning c;
        double m = 0;
        if (sscanf(line.c_str() + p, "\"tuning\": [%d, %d, %d, %d, %d]", &c.tile_w, &c.tile_h, &c.bin_cap, &c.persistent,
                   &c.path) == 5 &&
            sscanf(line.c_str() + q, "\"ms\": %lf", &m) == 1) {
            *t = c;
            *ms = m;
            found = true;
        }
    }
    return found;
}

void cache_store(const char *path, const std::string &dev, const std::string &lay, const orrb_tuning &t, double ms) {
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "{\"device\": \"%s\", \"layout\": \"%s\", \"tuning\": [%d, %d, %d, %d, %d], \"ms\": %.6f}\n", dev.c_str(),
            lay.c_str(), t.tile_w, t.tile_h, t.bin_cap, t.persistent, t.path, ms);
    fclose(f);
}

}  // namespace

extern "C" {

orrb_status orrb_autotune(orrb_context *ctx, orrb_layout *layout, const orrb_scenes *scenes, const orrb_cameras *cameras,
                          const orrb_params *params, const orrb_outputs *out, void *workspace, size_t workspace_bytes,
                          void *stream, const char *cache_path, orrb_tuning *chosen, double *best_ms) {
    if (!ctx || !layout) return set_error(ORRB_ERR_INVALID_ARGUMENT, "NULL handle");
    if (!cache_path) {
        const char *v = getenv("ORRB_AUTOTUNE_CACHE");
        if (v && *v) cache_path = v;
    }
    orrb_layout_info inf;
    orrb_status st = orrb_layout_info_get(layout, &inf);
    if (st != ORRB_OK) return st;
    if (workspace_bytes < inf.workspace_bytes_any)
        return set_error(ORRB_ERR_WORKSPACE_TOO_SMALL, "autotuning needs workspace_bytes_any");
    const std::string dev = device_key(context_device(ctx));
    char lay[32];
    snprintf(lay, sizeof(lay), "%016llx", (unsigned long long)layout_signature(layout));
    orrb_tuning best{};
    double bms = 0;
    if (cache_lookup(cache_path, dev, lay, &best, &bms)) {
        st = orrb_layout_set_tuning(layout, &best);
        if (st != ORRB_OK) return st;
        if (chosen) *chosen = best;
        if (best_ms) *best_ms = bms;
        return ORRB_OK;
    }
    // candidates: the frame kernel with scenes in LDS (tile choices matter only for the
    // frames it leaves to the tiled path), the frame kernel for every frame it can take
    // (path 2: its global bin capacity; tile choices again only for what remains), and
    // the tiled path over tile shapes, bin capacities and the persistent grid
    std::vector<orrb_tuning> cand;
    const int shapes[][2] = {{16, 16}, {32, 16}, {32, 32}, {64, 32}};
    const int caps[] = {256, 512};
    orrb_tuning probe{32, 32, 256, 0, 0}, probe2{32, 32, 256, 0, 2};
    orrb_layout_info pi, pi2;
    st = orrb_layout_set_tuning(layout, &probe2);
    if (st == ORRB_OK) st = orrb_layout_info_get(layout, &pi2);
    if (st == ORRB_OK) st = orrb_layout_set_tuning(layout, &probe);
    if (st == ORRB_OK) st = orrb_layout_info_get(layout, &pi);
    if (st != ORRB_OK) return st;
    const bool all_fit = pi.frame_path_frames == pi.n_frames;
    for (int path = 0; path <= 2; ++path) {
        if (path == 0 && all_fit) {
            cand.push_back(probe);
            continue;
        }
        if (path == 0 && pi.frame_path_frames == 0) continue;  // same as the tiled path
        if (path == 2) {
            if (pi2.frame_path_frames == pi.frame_path_frames) continue;  // same as path 0
            if (pi2.frame_path_frames == pi2.n_frames) {  // one launch: only the global bin capacity matters
                for (int cap : {256, 512, 1024}) cand.push_back(orrb_tuning{32, 32, cap, 0, 2});
                continue;
            }
        }
        for (auto &sh : shapes)
            for (int cap : caps)
                for (int pers = 0; pers <= 1; ++pers) cand.push_back(orrb_tuning{sh[0], sh[1], cap, pers, path});
    }
    const bool prof = context_profiling(ctx);
    context_set_profiling(ctx, false);
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        context_set_profiling(ctx, prof);
        return set_error(ORRB_ERR_DEVICE, "hipEventCreate failed");
    }
    const int reps = 3;
    bms = -1;
    for (const orrb_tuning &t : cand) {
        st = orrb_layout_set_tuning(layout, &t);
        if (st == ORRB_OK) st = orrb_render_batch(ctx, layout, scenes, cameras, params, out, workspace, workspace_bytes, stream);
        if (st == ORRB_OK && hipEventRecord(e0, s) != hipSuccess) st = ORRB_ERR_DEVICE;
        for (int r = 0; r < reps && st == ORRB_OK; ++r)
            st = orrb_render_batch(ctx, layout, scenes, cameras, params, out, workspace, workspace_bytes, stream);
        float ms = 0;
        if (st == ORRB_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = ORRB_ERR_DEVICE;
        if (st != ORRB_OK) break;
        const double m = ms / reps;
        if (bms < 0 || m < bms) {
            bms = m;
            best = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    context_set_profiling(ctx, prof);
    if (st != ORRB_OK) return st == ORRB_ERR_DEVICE ? set_error(st, "timing a candidate failed") : st;
    st = orrb_layout_set_tuning(layout, &best);
    if (st != ORRB_OK) return st;
    cache_store(cache_path, dev, lay, best, bms);
    if (chosen) *chosen = best;
    if (best_ms) *best_ms = bms;
    return ORRB_OK;
}

struct orrb_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
    // what the captured kernel arguments point into, and its state at capture
    const orrb_layout *layout = nullptr;
    const orrb_context *ctx = nullptr;
    uint64_t layout_gen = 0, ctx_gen = 0;
};

orrb_status orrb_graph_create(orrb_context *ctx, const orrb_layout *layout, const orrb_scenes *scenes,
                              const orrb_cameras *cameras, const orrb_params *params, const orrb_outputs *out,
                              void *workspace, size_t workspace_bytes, void *stream, orrb_graph **graph) {
    if (!ctx || !layout || !graph) return set_error(ORRB_ERR_INVALID_ARGUMENT, "NULL handle");
    *graph = nullptr;
    if (!stream) return set_error(ORRB_ERR_INVALID_ARGUMENT, "capture needs a non-null stream");
    hipStream_t s = (hipStream_t)stream;
    const bool prof = context_profiling(ctx);
    context_set_profiling(ctx, false);  // no timing events inside the graph
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        context_set_profiling(ctx, prof);
        return set_error(ORRB_ERR_DEVICE, "hipStreamBeginCapture failed");
    }
    orrb_status st = orrb_render_batch(ctx, layout, scenes, cameras, params, out, workspace, workspace_bytes, stream);
    const hipError_t ec = hipStreamEndCapture(s, &g);
    context_set_profiling(ctx, prof);
    if (st != ORRB_OK || ec != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return st != ORRB_OK ? st : set_error(ORRB_ERR_DEVICE, "hipStreamEndCapture failed");
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return set_error(ORRB_ERR_DEVICE, "hipGraphInstantiate failed");
    }
    auto *G = new (std::nothrow) orrb_graph();
    if (!G) {
        (void)hipGraphExecDestroy(ex);
        (void)hipGraphDestroy(g);
        return set_error(ORRB_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    G->graph = g;
    G->exec = ex;
    G->device = context_device(ctx);
    G->layout = layout;
    G->ctx = ctx;
    G->layout_gen = layout_generation(layout);
    G->ctx_gen = context_generation(ctx);
    *graph = G;
    return ORRB_OK;
}

orrb_status orrb_graph_launch(orrb_graph *graph, void *stream) {
    if (!graph) return set_error(ORRB_ERR_INVALID_ARGUMENT, "NULL graph");
    // the captured arguments hold the layout's table pointers, item counts and tuning
    // and the mesh pool's pointers: refuse the replay once either may have moved
    if (layout_generation(graph->layout) != graph->layout_gen)
        return set_error(ORRB_ERR_INVALID_ARGUMENT, "the layout's tuning or tables changed since the graph was captured");
    if (context_generation(graph->ctx) != graph->ctx_gen)
        return set_error(ORRB_ERR_INVALID_ARGUMENT, "the mesh pool grew since the graph was captured");
    const hipError_t e = hipGraphLaunch(graph->exec, (hipStream_t)stream);
    if (e != hipSuccess) return set_error(ORRB_ERR_DEVICE, hipGetErrorString(e));
    return ORRB_OK;
}

void orrb_graph_destroy(orrb_graph *graph) {
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

}  // extern "C"
