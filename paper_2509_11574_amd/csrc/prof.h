// Optional per-kernel timing with HIP events (off unless gps_profile_start was
// called on the launching thread).  Each launch site is wrapped in a scope that
// records an event before and after the launch on the launch stream.
#pragma once

#include <hip/hip_runtime.h>

namespace gps {

enum KernelId {
    K_FUSE = 0,
    K_BRICK_MIN,
    K_RAYCAST,
    K_TILEMAX,
    K_PROJECT,
    K_SCAN,
    K_TILE_COUNT,
    K_SCAN_TILES,
    K_EMIT,
    K_TILE_SORT,
    K_TILE_SORT_LARGE,
    K_COMPOSITE_FWD,
    K_LOSS_REDUCE,
    K_COMPOSITE_BWD,
    K_GAUSS_BWD,
    K_POSE_REDUCE,
    K_ADAM,
    K_STEP_INCR,
    K_WS_RESET,
    K_UPLOAD,
    K_REMOVE,
    K_INSERT,
    K_ICP,
    K_HASH,
    K_COUNT
};

const char* kernel_name(int id);
bool prof_active();
void prof_record(int id, hipStream_t s, bool after);

struct ProfScope {
    int id;
    hipStream_t s;
    bool on;
    ProfScope(int id_, hipStream_t s_) : id(id_), s(s_), on(prof_active())
    {
        if (on) prof_record(id, s, false);
    }
    ~ProfScope()
    {
        if (on) prof_record(id, s, true);
    }
};

}  // namespace gps

#define GPS_LAUNCH(kid, stream, ...)                 \
    do {                                             \
        ::gps::ProfScope gps_prof_scope_(kid, stream); \
        hipLaunchKernelGGL(__VA_ARGS__);             \
    } while (0)
