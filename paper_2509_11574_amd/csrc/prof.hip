// Optional per-kernel timing (see prof.h).  State is thread-local and owned by
// the calling thread; events are created lazily and reused.
#include <cstring>
#include <vector>

#include "gps_internal.h"
#include "prof.h"

namespace gps {

static const char* kNames[K_COUNT] = {"fuse", "brick_min", "raycast", "tilemax", "project", "scan", "count",
                                      "scan_tiles", "emit", "tile_sort", "tile_sort_large", "composite_fwd", "loss_reduce", "composite_bwd", "gauss_bwd",
                                      "pose_reduce", "adam", "step_incr", "ws_reset",
                                      "upload_views", "remove", "insert", "icp", "hash"};

const char* kernel_name(int id) { return (id >= 0 && id < K_COUNT) ? kNames[id] : "?"; }

struct ProfRec {
    int id;
    hipEvent_t a, b;
};

struct ProfState {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t next = 0;
    std::vector<ProfRec> recs;
    ~ProfState()
    {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

static thread_local ProfState g_prof;

bool prof_active() { return g_prof.on; }

static hipEvent_t take_event()
{
    if (g_prof.next == g_prof.pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_prof.pool.push_back(e);
    }
    return g_prof.pool[g_prof.next++];
}

void prof_record(int id, hipStream_t s, bool after)
{
    hipEvent_t e = take_event();
    if (!e) return;
    if (hipEventRecord(e, s) != hipSuccess) return;
    if (!after) {
        g_prof.recs.push_back({id, e, nullptr});
    } else if (!g_prof.recs.empty() && g_prof.recs.back().id == id && !g_prof.recs.back().b) {
        g_prof.recs.back().b = e;
    }
}

}  // namespace gps

using namespace gps;

extern "C" {

gps_status gps_profile_start(void)
{
    g_prof.recs.clear();
    g_prof.next = 0;
    g_prof.on = true;
    return GPS_OK;
}

gps_status gps_profile_stop(void)
{
    g_prof.on = false;
    return GPS_OK;
}

gps_status gps_profile_read(gps_kernel_time* out, int32_t max_kernels, int32_t* n_out)
{
    if (!out || !n_out || max_kernels < 1) return GPS_ERR_INVALID_ARG;
    double ms[K_COUNT] = {0};
    long long cnt[K_COUNT] = {0};
    for (const ProfRec& r : g_prof.recs) {
        if (!r.b) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return GPS_ERR_HIP;
        float t = 0.0f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return GPS_ERR_HIP;
        ms[r.id] += t;
        cnt[r.id] += 1;
    }
    int n = 0;
    for (int k = 0; k < K_COUNT && n < max_kernels; ++k) {
        if (!cnt[k]) continue;
        std::memset(out[n].name, 0, sizeof(out[n].name));
        std::strncpy(out[n].name, kNames[k], sizeof(out[n].name) - 1);
        out[n].launches = cnt[k];
        out[n].total_ms = ms[k];
        ++n;
    }
    *n_out = n;
    return GPS_OK;
}

}  // extern "C"
