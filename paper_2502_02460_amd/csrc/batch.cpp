// Batched small problems (gevd.h, "Batched small problems"): grouping of a
// batch by scalar type and order bucket, the persistent fused launches,
// their capture into a HIP graph, and the launch-shape tuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "ctx.hpp"
#include "batch.hpp"
#include "kernels.hpp"
#include "small.hpp"

using namespace gevd;

namespace {

// One group per scalar type: a single queue over all its problems, largest
// order first (longest-processing-time order balances the persistent
// workgroups); LDS and Z slots are sized for the group's largest order.
struct Group {
    bool cx;
    int bucket, first, count, threads, grid;
    long zoff;
};

}  // namespace

namespace gevd {

double batch_problem_flops(const gevd_problem& p) {
    // Cholesky n^3/3, the two triangular solves 2n^3, Householder
    // tridiagonalisation 4n^3/3, back-transformation 2n^2 k + n^2 k (real
    // count; x4 complex).  QL rotations are not counted.
    const double n = p.n, k = p.nev;
    const double chol = (p.flags & GEVD_PROBLEM_FACTORED) ? 0.0 : n * n * n / 3.0;
    const double f = chol + 2.0 * n * n * n + 4.0 * n * n * n / 3.0 + 3.0 * n * n * k;
    return p.dtype == GEVD_COMPLEX ? 4.0 * f : f;
}

int batch_num_cu(gevd_ctx* h) {
    if (h->ncu <= 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || v < 1) v = 1;
        h->ncu = v;
    }
    return h->ncu;
}

// Default launch shape per bucket (n <= 64, 128, 256, 512): threads per
// workgroup and workgroups per CU, as gevd_tune_batched chose them on MI355X
// for 512 problems of a bucket (bounded by the occupancy the device reports).
// Real problems take 256 threads at two workgroups per CU up to n = 256
// and 1024 threads with one workgroup per CU above; complex ones 128 threads
// up to n = 128 and 512 threads with one workgroup per CU above.  (Measured
// on the serving mix, first SCF iteration: 1490 solves/s with one workgroup
// size per bucket at full occupancy, 2007 with the tuned shapes up to 512
// threads, 2330 with 1024 threads for real n > 256.)
static void default_shape(bool cx, int bucket, int* threads, int* wgpcu) {
    static const int t[2][SMALL_NBUCKET] = {{256, 256, 256, 1024}, {128, 128, 512, 512}};
    static const int w[2][SMALL_NBUCKET] = {{2, 2, 2, 1}, {2, 2, 1, 1}};
    *threads = t[cx ? 1 : 0][bucket];
    *wgpcu = std::max(1, std::min(w[cx ? 1 : 0][bucket], small_occupancy(cx, *threads, small_bucket_n(bucket))));
}

void batch_shape_of(gevd_ctx* h, bool cx, int bucket, int* threads, int* wgpcu) {
    const int dt = cx ? 1 : 0;
    if (h->bthreads[dt][bucket] > 0) {
        *threads = h->bthreads[dt][bucket];
        *wgpcu = h->bwgpcu[dt][bucket];
    } else {
        default_shape(cx, bucket, threads, wgpcu);
    }
}

int batch_check_problem(const gevd_problem& p) {
    if (p.dtype != GEVD_REAL && p.dtype != GEVD_COMPLEX) return 1;
    if (p.n < 1 || p.n > SMALL_MAX || p.nev < 1 || p.nev > p.n) return 1;
    if (!p.H || !p.S || !p.C || !p.eval) return 1;
    if (p.ldh < p.n || p.lds < p.n || p.ldc < p.n) return 1;
    if (p.flags & ~GEVD_PROBLEM_FACTORED) return 1;
    return 0;
}

void batch_order(int count, const gevd_problem* probs, int* ord) {
    for (int i = 0; i < count; ++i) ord[i] = i;
    auto key = [&](int i) { return probs[i].dtype == GEVD_COMPLEX ? 0 : 1; };
    std::sort(ord, ord + count, [&](int a, int c) {
        if (key(a) != key(c)) return key(a) < key(c);
        if (probs[a].n != probs[c].n) return probs[a].n > probs[c].n;
        return a < c;
    });
}

}  // namespace gevd


struct gevd_batch_s {
    gevd_ctx* h = nullptr;
    int count = 0;
    SmallDesc* desc = nullptr;  // device
    int* info = nullptr;        // device, count
    int* counters = nullptr;    // device, one per group
    double* zws = nullptr;      // device
    std::vector<Group> groups;
    double flops = 0.0;
    bool graphed = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipStream_t aux = nullptr;  // second stream: the two scalar types run concurrently
};

namespace {

void release(gevd_batch_s* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->desc) (void)hipFree(b->desc);
    if (b->info) (void)hipFree(b->info);
    if (b->counters) (void)hipFree(b->counters);
    if (b->zws) (void)hipFree(b->zws);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->aux) (void)hipStreamDestroy(b->aux);
    delete b;
}

int launch_group(gevd_batch_s* b, size_t g, hipStream_t st) {
    const Group& G = b->groups[g];
    return small_launch(st, G.cx, G.threads, G.grid, small_bucket_n(G.bucket), b->desc + G.first, G.count,
                        b->zws + G.zoff, b->counters + g);
}

// The first group on st; a second one on st2, forked from and joined back
// into st with events (also inside a graph capture, where this makes two
// parallel branches).
int enqueue(gevd_batch_s* b, hipStream_t st, hipStream_t st2) {
    int rc = 0;
    if (b->groups.size() > 1) {
        GEVD_HIP(hipEventRecord(b->fork, st));
        GEVD_HIP(hipStreamWaitEvent(st2, b->fork, 0));
        if ((rc = launch_group(b, 1, st2))) return rc;
        GEVD_HIP(hipEventRecord(b->join, st2));
    }
    if ((rc = launch_group(b, 0, st))) return rc;
    if (b->groups.size() > 1) GEVD_HIP(hipStreamWaitEvent(st, b->join, 0));
    return 0;
}

// Groups the batch, uploads descriptors, sizes the Z workspace.
int build(gevd_ctx* h, int count, const gevd_problem* probs, bool graphed, gevd_batch_s** out) {
    *out = nullptr;
    gevd_batch_s* b = new (std::nothrow) gevd_batch_s();
    if (!b) return GEVD_E_NOMEM;
    b->h = h;
    b->count = count;
    b->graphed = graphed;
    // queue order: complex first, largest order first inside a scalar type
    std::vector<int> ord(count);
    batch_order(count, probs, ord.data());
    auto key = [&](int i) { return probs[i].dtype == GEVD_COMPLEX ? 0 : 1; };
    int rc = 0;
    if (hipMalloc(&b->desc, sizeof(SmallDesc) * count) != hipSuccess ||
        hipMalloc(&b->info, sizeof(int) * count) != hipSuccess ||
        hipMalloc(&b->counters, sizeof(int) * 2) != hipSuccess) {
        (void)hipGetLastError();
        release(b);
        return GEVD_E_NOMEM;
    }
    std::vector<SmallDesc> hd(count);
    long zmax = 0;
    for (int s = 0; s < count;) {
        const int k = key(ord[s]);
        int e = s;
        while (e < count && key(ord[e]) == k) ++e;
        Group G;
        G.cx = k == 0;
        G.bucket = small_bucket(probs[ord[s]].n);  // largest order of the group
        G.first = s;
        G.count = e - s;
        int wg = 1;
        batch_shape_of(h, G.cx, G.bucket, &G.threads, &wg);
        G.grid = std::max(1, std::min(G.count, wg * batch_num_cu(h)));
        if ((rc = small_prepare(G.cx, G.threads, small_bucket_n(G.bucket)))) {
            release(b);
            return rc;
        }
        G.zoff = zmax;
        zmax += (long)G.grid * small_zslot(small_bucket_n(G.bucket));
        b->groups.push_back(G);
        s = e;
    }
    for (int s = 0; s < count; ++s) {
        const gevd_problem& p = probs[ord[s]];
        hd[s] = SmallDesc{p.H, p.S, p.C, p.eval, b->info + ord[s], (long)p.ldh, (long)p.lds, (long)p.ldc, p.n, p.nev,
                          (p.flags & GEVD_PROBLEM_FACTORED) ? 1 : 0};
        b->flops += batch_problem_flops(p);
    }
    if (hipMalloc(&b->zws, sizeof(double) * std::max(zmax, 1L)) != hipSuccess) {
        (void)hipGetLastError();
        release(b);
        return GEVD_E_NOMEM;
    }
    if (hipMemcpy(b->desc, hd.data(), sizeof(SmallDesc) * count, hipMemcpyHostToDevice) != hipSuccess ||
        hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess ||
        (!graphed && b->groups.size() > 1 && hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking) != hipSuccess)) {
        (void)hipGetLastError();
        release(b);
        return GEVD_E_HIP;
    }
    if (graphed) {
        hipStream_t cs = nullptr, cs2 = nullptr;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&cs2, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            if (cs) (void)hipStreamDestroy(cs);
            release(b);
            return GEVD_E_HIP;
        }
        bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) == hipSuccess;
        if (ok) {
            rc = enqueue(b, cs, cs2);
            ok = hipStreamEndCapture(cs, &b->graph) == hipSuccess && rc == 0;
        }
        if (ok) ok = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
        (void)hipStreamDestroy(cs2);
        (void)hipStreamDestroy(cs);
        if (!ok) {
            (void)hipGetLastError();
            release(b);
            return rc ? rc : GEVD_E_HIP;
        }
    }
    *out = b;
    return 0;
}

int run(gevd_batch_s* b, int* info, int* info_dev = nullptr) {
    gevd_ctx* h = b->h;
    GEVD_HIP(hipSetDevice(h->device));
    {
        g_kstats = h->kstats_on ? &h->ks : nullptr;
        KProbe kp(h->stream, GEVD_K_SMALL, b->flops);
        int rc = 0;
        if (b->graphed) {
            if (hipGraphLaunch(b->exec, h->stream) != hipSuccess) rc = GEVD_E_HIP;
        } else {
            rc = enqueue(b, h->stream, b->aux);
        }
        if (rc) {
            g_kstats = nullptr;
            return rc;
        }
    }
    g_kstats = nullptr;
    if (info_dev)
        GEVD_HIP(hipMemcpyAsync(info_dev, b->info, sizeof(int) * b->count, hipMemcpyDeviceToDevice, h->stream));
    if (info) {
        GEVD_HIP(hipMemcpyAsync(info, b->info, sizeof(int) * b->count, hipMemcpyDeviceToHost, h->stream));
        GEVD_HIP(hipStreamSynchronize(h->stream));
    }
    return 0;
}

}  // namespace

extern "C" {

int gevd_batch_create(gevd_handle h, int count, const gevd_problem* probs, gevd_batch* out) {
    if (!h) return -1;
    if (count < 1) return -2;
    if (!probs) return -3;
    if (!out) return -4;
    *out = nullptr;
    for (int i = 0; i < count; ++i)
        if (batch_check_problem(probs[i])) return -3;
    GEVD_HIP(hipSetDevice(h->device));
    return build(h, count, probs, true, out);
}

int gevd_batch_run(gevd_batch b, int* info) {
    if (!b) return -1;
    return run(b, info);
}

int gevd_batch_run_async(gevd_batch b, int* info_dev) {
    if (!b) return -1;
    if (!info_dev) return -2;
    return run(b, nullptr, info_dev);
}

int gevd_batch_destroy(gevd_batch b) {
    if (!b) return -1;
    (void)hipSetDevice(b->h->device);
    (void)hipStreamSynchronize(b->h->stream);
    release(b);
    return 0;
}

int gevd_solve_batched(gevd_handle h, int count, const gevd_problem* probs, int* info) {
    if (!h) return -1;
    if (count < 1) return -2;
    if (!probs) return -3;
    if (!info) return -4;
    for (int i = 0; i < count; ++i)
        if (batch_check_problem(probs[i])) return -3;
    GEVD_HIP(hipSetDevice(h->device));
    gevd_batch_s* b = nullptr;
    int rc = build(h, count, probs, false, &b);
    if (rc) return rc;
    rc = run(b, info);
    (void)hipStreamSynchronize(h->stream);
    release(b);
    return rc;
}

int gevd_set_batch_shape(gevd_handle h, int dtype, int n, int threads, int wg_per_cu) {
    if (!h) return -1;
    if (dtype != GEVD_REAL && dtype != GEVD_COMPLEX) return -2;
    if (n < 1 || n > SMALL_MAX) return -3;
    if (threads != 0 && threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024)
        return -4;
    if (threads != 0 && (wg_per_cu < 1 || wg_per_cu > 32)) return -5;
    const int bk = small_bucket(n);
    h->bthreads[dtype][bk] = threads;
    h->bwgpcu[dtype][bk] = threads ? wg_per_cu : 0;
    return 0;
}

int gevd_get_batch_shape(gevd_handle h, int dtype, int n, int* threads, int* wg_per_cu) {
    if (!h) return -1;
    if (dtype != GEVD_REAL && dtype != GEVD_COMPLEX) return -2;
    if (n < 1 || n > SMALL_MAX) return -3;
    if (!threads) return -4;
    if (!wg_per_cu) return -5;
    GEVD_HIP(hipSetDevice(h->device));
    batch_shape_of(h, dtype == GEVD_COMPLEX, small_bucket(n), threads, wg_per_cu);
    return 0;
}

int gevd_tune_batched(gevd_handle h, int dtype, int n, int count, int* threads, int* wg_per_cu) {
    if (!h) return -1;
    if (dtype != GEVD_REAL && dtype != GEVD_COMPLEX) return -2;
    if (n < 1 || n > SMALL_MAX) return -3;
    if (count < 1) return -4;
    GEVD_HIP(hipSetDevice(h->device));
    const bool cx = dtype == GEVD_COMPLEX;
    const int bk = small_bucket(n), nb = small_bucket_n(bk);
    const size_t es = cx ? 16 : 8;
    const long per = (long)nb * nb;
    char *H = nullptr, *S = nullptr, *C = nullptr;
    double* ev = nullptr;
    auto cleanup = [&]() {
        if (H) (void)hipFree(H);
        if (S) (void)hipFree(S);
        if (C) (void)hipFree(C);
        if (ev) (void)hipFree(ev);
    };
    if (hipMalloc(&H, es * per * count) != hipSuccess || hipMalloc(&S, es * per * count) != hipSuccess ||
        hipMalloc(&C, es * per * count) != hipSuccess || hipMalloc(&ev, sizeof(double) * nb * count) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return GEVD_E_NOMEM;
    }
    std::vector<gevd_problem> probs(count);
    const int nev = std::max(1, (3 * nb) / 10);
    for (int p = 0; p < count; ++p)
        probs[p] = gevd_problem{dtype, nb, nev, H + es * per * p, nb, S + es * per * p, nb, ev + (long)nb * p,
                                C + es * per * p, nb, 0};
    hipEvent_t e0, e1;
    GEVD_HIP(hipEventCreate(&e0));
    GEVD_HIP(hipEventCreate(&e1));
    const int saved_t = h->bthreads[dtype][bk], saved_w = h->bwgpcu[dtype][bk];
    float best = 3.0e38f;
    int bt = 0, bw = 0, rc = 0;
    const int cand_t[5] = {64, 128, 256, 512, 1024};
    for (int ti = 0; ti < 5 && !rc; ++ti) {
        const int t = cand_t[ti];
        const int occ = small_occupancy(cx, t, nb);
        int ws[3] = {1, std::max(1, occ / 2), occ};
        for (int wi = 0; wi < 3 && !rc; ++wi) {
            if (wi > 0 && ws[wi] == ws[wi - 1]) continue;
            h->bthreads[dtype][bk] = t;
            h->bwgpcu[dtype][bk] = ws[wi];
            gevd_batch_s* b = nullptr;
            if ((rc = build(h, count, probs.data(), false, &b))) break;
            float tbest = 3.0e38f;
            for (int rep = 0; rep < 2 && !rc; ++rep) {
                if ((rc = small_gen(h->stream, cx, nb, count, H, S, per, 1234 + rep))) break;
                if (hipEventRecord(e0, h->stream) != hipSuccess) rc = GEVD_E_HIP;
                if (!rc) rc = enqueue(b, h->stream, b->aux);
                if (!rc && hipEventRecord(e1, h->stream) != hipSuccess) rc = GEVD_E_HIP;
                if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = GEVD_E_HIP;
                float ms = 0.f;
                if (!rc && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) tbest = std::min(tbest, ms);
            }
            release(b);
            if (!rc && tbest < best) {
                best = tbest;
                bt = t;
                bw = ws[wi];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    cleanup();
    if (rc || bt == 0) {
        h->bthreads[dtype][bk] = saved_t;
        h->bwgpcu[dtype][bk] = saved_w;
        return rc ? rc : GEVD_E_HIP;
    }
    h->bthreads[dtype][bk] = bt;
    h->bwgpcu[dtype][bk] = bw;
    if (threads) *threads = bt;
    if (wg_per_cu) *wg_per_cu = bw;
    return 0;
}

}  // extern "C"
