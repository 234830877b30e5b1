// Batched small-problem solve that allocates nothing (gevd.h,
// gevd_solve_batched_noalloc), for callers that may not allocate device
// memory while they run.  Its device scratch (descriptors, per-problem
// status, queue counters and the per-workgroup Z slots of the fused kernel)
// lives in one fixed file-scope device array; host-side staging lives in the
// handle.  The kernels are those of gevd_solve_batched, which take the
// scratch addresses as arguments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "batch.hpp"
#include "kernels.hpp"
#include "small.hpp"

using namespace gevd;

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)GEVD_NOALLOC_SCRATCH_BYTES;
static_assert(SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

// One copy per device, held until the process ends.  Host code never uses
// this name as an address: it uses the per-device pointer resolved by
// noalloc_attach.
static __device__ __align__(256) char scratch[SCRATCH_BYTES];

constexpr int MAXDEV = 64;
std::mutex g_attach_mu;
void* g_scratch[MAXDEV] = {};
// Calls on one device are serialised: they share that device's scratch.
std::mutex g_call_mu[MAXDEV];

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

namespace gevd {

int noalloc_attach(int device) {
    if (device < 0 || device >= MAXDEV) return GEVD_E_HIP;
    std::lock_guard<std::mutex> lk(g_attach_mu);
    if (g_scratch[device]) return 0;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        fprintf(stderr, "gevd: hipGetSymbolAddress(scratch) failed on device %d: %s\n", device,
                hipGetErrorString(e));
        (void)hipGetLastError();
        return GEVD_E_HIP;
    }
    g_scratch[device] = p;
    return 0;
}

}  // namespace gevd

extern "C" int gevd_solve_batched_noalloc(gevd_handle h, int count, const gevd_problem* probs, int* info) {
    if (!h) return -1;
    if (count < 1) return -2;
    if (!probs) return -3;
    if (!info) return -4;
    if (count > GEVD_NOALLOC_MAX_COUNT) return GEVD_E_SCRATCH;
    for (int i = 0; i < count; ++i)
        if (batch_check_problem(probs[i])) return -3;
    if (h->device < 0 || h->device >= MAXDEV || !h->na_desc || !h->na_ord) return GEVD_E_STATE;
    char* base = static_cast<char*>(g_scratch[h->device]);
    if (!base) return GEVD_E_STATE;
    GEVD_HIP(hipSetDevice(h->device));
    std::lock_guard<std::mutex> lk(g_call_mu[h->device]);

    // scratch layout: descriptors | status | two queue counters | Z slots
    const size_t off_info = align256(sizeof(SmallDesc) * (size_t)count);
    const size_t off_ctr = off_info + align256(sizeof(int) * (size_t)count);
    const size_t off_z = off_ctr + 256;
    if (off_z >= SCRATCH_BYTES) return GEVD_E_SCRATCH;
    SmallDesc* desc = reinterpret_cast<SmallDesc*>(base);
    int* dinfo = reinterpret_cast<int*>(base + off_info);
    int* ctr = reinterpret_cast<int*>(base + off_ctr);
    double* zws = reinterpret_cast<double*>(base + off_z);
    const long zdoubles = (long)((SCRATCH_BYTES - off_z) / sizeof(double));

    int* ord = h->na_ord;
    batch_order(count, probs, ord);
    for (int s = 0; s < count; ++s) {
        const gevd_problem& p = probs[ord[s]];
        h->na_desc[s] = SmallDesc{p.H, p.S, p.C, p.eval, dinfo + ord[s], (long)p.ldh, (long)p.lds, (long)p.ldc,
                                  p.n, p.nev, (p.flags & GEVD_PROBLEM_FACTORED) ? 1 : 0};
    }
    GEVD_HIP(hipMemcpyAsync(desc, h->na_desc, sizeof(SmallDesc) * (size_t)count, hipMemcpyHostToDevice, h->stream));

    // One group per scalar type, run one after the other on the handle's
    // stream; each uses the whole Z region, so a group's grid is also
    // bounded by the Z slots that fit.
    int rc = 0;
    for (int s = 0, g = 0; s < count && !rc; ++g) {
        const bool cx = probs[ord[s]].dtype == GEVD_COMPLEX;
        int e = s;
        while (e < count && (probs[ord[e]].dtype == GEVD_COMPLEX) == cx) ++e;
        const int bucket = small_bucket(probs[ord[s]].n);  // largest order of the group
        const int nmax = small_bucket_n(bucket);
        int threads = 0, wg = 1;
        batch_shape_of(h, cx, bucket, &threads, &wg);
        // the wider workgroup shapes spill registers, and a kernel with spills
        // needs private scratch that the runtime provides at launch: keep to
        // shapes that fit in registers (results do not depend on the shape)
        const int tfit = cx ? 256 : 512;
        if (threads > tfit) {
            threads = tfit;
            wg = std::max(1, small_occupancy(cx, threads, nmax));
        }
        const long slots = zdoubles / small_zslot(nmax);
        if (slots < 1) {
            rc = GEVD_E_SCRATCH;
            break;
        }
        const int grid = (int)std::max(1L, std::min<long>({(long)(e - s), (long)wg * batch_num_cu(h), slots}));
        if ((rc = small_prepare(cx, threads, nmax))) break;
        rc = small_launch(h->stream, cx, threads, grid, nmax, desc + s, e - s, zws, ctr + g);
        s = e;
    }
    if (rc) {
        (void)hipStreamSynchronize(h->stream);
        return rc;
    }
    GEVD_HIP(hipMemcpyAsync(info, dinfo, sizeof(int) * (size_t)count, hipMemcpyDeviceToHost, h->stream));
    GEVD_HIP(hipStreamSynchronize(h->stream));
    return 0;
}
