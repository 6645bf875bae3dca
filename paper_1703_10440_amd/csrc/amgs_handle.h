// amgs_handle.h -- the opaque handle behind amgs_handle_t (host only).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/amgs.h"

struct amgs_handle {
    int device;
    int num_cu;
    amgs_stats_t stats;
    int profiling;
    struct Rec {
        int cat;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;        // recorded since the last read/reset
    std::vector<hipEvent_t> pool; // idle events
    double prof_ms[3];
    int64_t prof_n[3];
};
