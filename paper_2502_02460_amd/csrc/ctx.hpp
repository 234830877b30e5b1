// The handle behind gevd_handle (shared by the host pipeline files).
#pragma once
#include <hip/hip_runtime.h>

#include "kstats.hpp"
#include "small.hpp"

struct gevd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int band_opt = 0;
    int leaf_opt = 0;
    int timing = 0;
    int prec = 0;          // GEVD_OPT_PRECISION
    int refine_iters = 2;  // GEVD_OPT_REFINE
    int panel_persist = 1; // GEVD_OPT_PANEL
    int persist_now = 0;   // the current call holds the persistent panel route (PanelLease)
    int gemm_tile = -1;    // GEVD_OPT_GEMM_TILE
    int stages = 2;        // GEVD_OPT_STAGES
    char* ws = nullptr;  // workspace (device)
    size_t ws_bytes = 0;
    int* flags = nullptr;  // small device status area
    double* dstat = nullptr;  // device: {max, min} |U_ii| of the last Cholesky
    double* dhost = nullptr;  // pinned host copy of dstat
    int warn = 0;             // GEVD_W_* bits of the last solve
    double kappa_lb = 0.0;    // lower bound of cond(S) from the last Cholesky
    hipEvent_t ev[GEVD_NPHASE + 1] = {};
    bool ev_made = false;
    bool ev_valid = false;
    int kstats_on = 0;
    gevd::KStats ks;
    // resident overlap (SCF reuse): U^{-1} of the last gevd_set_overlap
    void* uinv = nullptr;
    size_t uinv_bytes = 0;
    int res_n = 0, res_dtype = -1;
    // batched small problems: launch shape per (dtype, order bucket);
    // 0 = not chosen yet (the default heuristic applies)
    int bthreads[2][gevd::SMALL_NBUCKET] = {};
    int bwgpcu[2][gevd::SMALL_NBUCKET] = {};
    int ncu = 0;
    // second stream and events for overlapped stages (created on first use)
    hipStream_t aux = nullptr;
    hipEvent_t aux_fork = nullptr, aux_join = nullptr;
    // host staging of gevd_solve_batched_noalloc (GEVD_NOALLOC_MAX_COUNT
    // entries each, allocated by gevd_create)
    gevd::SmallDesc* na_desc = nullptr;
    int* na_ord = nullptr;
};
