// amgs_handle.h -- the opaque handle behind amgs_handle_t (host only).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/amgs.h"

// kernel categories of amgs_profile_read
constexpr int AMGS_PROF_NCAT = 4;

struct amgs_handle {
    int device;
    int num_cu;
    void *scratch;   // this device's static scratch array (amgs_qr_csr_static)
    amgs_stats_t stats;
    int profiling;
    struct Rec {
        int cat;
        hipEvent_t a, b;
        int cat2;   // a second category the launch also counts in (-1: none)
    };
    std::vector<Rec> recs;        // recorded since the last read/reset
    std::vector<hipEvent_t> pool; // idle events
    double prof_ms[AMGS_PROF_NCAT];
    int64_t prof_n[AMGS_PROF_NCAT];
};
