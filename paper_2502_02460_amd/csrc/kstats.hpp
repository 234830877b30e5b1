// Live per-kernel-family accounting: when a handle enables it, every launch
// of an instrumented family is bracketed by HIP events on its stream and
// tagged with the algorithmic flops it performs; totals accumulate until read.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/gevd.h"

namespace gevd {

struct KStats {
    struct Rec {
        int fam;
        double flops;
        int e0, e1;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Rec> recs;
    int used = 0;
    double tot_ms[GEVD_NKFAM] = {};
    double tot_flops[GEVD_NKFAM] = {};
    long long tot_n[GEVD_NKFAM] = {};

    int take() {
        if (used == (int)pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            pool.push_back(e);
        }
        return used++;
    }
    // resolve recorded launches into the totals (the stream must be idle)
    void settle() {
        for (const Rec& r : recs) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pool[r.e0], pool[r.e1]) == hipSuccess) {
                tot_ms[r.fam] += ms;
                tot_flops[r.fam] += r.flops;
                tot_n[r.fam] += 1;
            }
        }
        recs.clear();
        used = 0;
    }
    void reset() {
        recs.clear();
        used = 0;
        for (int i = 0; i < GEVD_NKFAM; ++i) tot_ms[i] = tot_flops[i] = 0.0, tot_n[i] = 0;
    }
};

// The accounting of the handle whose entry point is running on this thread
// (nullptr when disabled).
extern thread_local KStats* g_kstats;

struct KProbe {
    hipStream_t st;
    int fam, e0 = -1;
    double flops;
    KProbe(hipStream_t s, int f, double fl) : st(s), fam(f), flops(fl) {
        if (g_kstats && (e0 = g_kstats->take()) >= 0) (void)hipEventRecord(g_kstats->pool[e0], st);
    }
    ~KProbe() {
        if (!g_kstats || e0 < 0) return;
        const int e1 = g_kstats->take();
        if (e1 < 0) return;
        (void)hipEventRecord(g_kstats->pool[e1], st);
        g_kstats->recs.push_back({fam, flops, e0, e1});
    }
};

}  // namespace gevd
