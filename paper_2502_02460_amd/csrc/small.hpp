// Batched small-problem path: descriptors and launcher of the persistent
// fused kernel (internal; the C interface wraps it).
#pragma once
#include "common.hpp"

namespace gevd {

// Largest order the fused kernel takes, and the order buckets a batch is
// split into (one launch shape per bucket and scalar type).
constexpr int SMALL_MAX = 512;
constexpr int SMALL_NBUCKET = 4;
inline int small_bucket(int n) { return n <= 64 ? 0 : n <= 128 ? 1 : n <= 256 ? 2 : 3; }
inline int small_bucket_n(int b) { return 64 << b; }

// One problem of a batch: device pointers and sizes (column-major).
struct SmallDesc {
    void* H;       // n x n, upper triangle read; clobbered
    void* S;       // n x n, upper triangle read; receives U (upper) and U^H (strictly lower)
    void* C;       // n x nev eigenvectors
    double* eval;  // n eigenvalues, ascending
    int* info;     // 0, j > 0 (S not positive definite at minor j) or GEVD_E_*
    long ldh, lds, ldc;
    int n, nev;
    int factored;  // S already holds U / U^H from an earlier solve: skip the Cholesky
};

// Dynamic LDS bytes of one workgroup for orders up to nmax.
size_t small_lds_bytes(bool cx, int nmax);
// Z slot (doubles) one workgroup needs for orders up to nmax.
inline long small_zslot(int nmax) { return (long)nmax * nmax; }
// Set the kernel attributes a launch shape needs (call before any launch or
// graph capture that uses it).
int small_prepare(bool cx, int threads, int nmax);
// Workgroups of `threads` lanes that fit on one CU at once (registers, LDS).
int small_occupancy(bool cx, int threads, int nmax);

// Launch: zero the queue counter, then `grid` persistent workgroups of
// `threads` (64, 128, 256, 512 or 1024) lanes drain `count` problems of one dtype
// with n <= nmax.  zws holds grid * small_zslot(nmax) doubles.  Nothing here
// synchronises or allocates, so the sequence may be captured in a graph.
int small_launch(hipStream_t st, bool cx, int threads, int grid, int nmax, const SmallDesc* desc, int count,
                 double* zws, int* counter);

// Synthetic well-conditioned problems for launch-shape tuning: count pairs
// of order n at H + p*stride, S + p*stride (ld n): H entries uniform in
// [-1, 1], S = I + R/(2n) with R's entries uniform in [-1, 1] (diagonally
// dominant, so positive definite).  Counter-based, from seed.
int small_gen(hipStream_t st, bool cx, int n, int count, void* H, void* S, long stride, unsigned long long seed);
}  // namespace gevd
