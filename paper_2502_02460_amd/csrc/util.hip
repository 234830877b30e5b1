// Elementwise and data-movement kernels (bandwidth-bound; coalesced through
// 32 x 32 LDS tiles where a transpose is involved).
#include "kernels.hpp"

namespace gevd {
namespace {

constexpr int TT = 32;  // transpose tile

// For tiles on or below the diagonal: A[i, j] = conj(A[j, i]) for i > j,
// and Im A[i, i] = 0.  Reads the mirrored upper tile coalesced into LDS.
template <typename T>
__global__ __launch_bounds__(256) void fill_lower_kernel(int n, T* A, long lda) {
    __shared__ T tile[TT][TT + 1];
    const int bi = blockIdx.x, bj = blockIdx.y;  // destination tile (rows bi, cols bj), bi >= bj
    if (bi < bj) return;
    const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;  // 32 x 8
    // source: rows bj*TT.., cols bi*TT.. (upper part)
    for (int r = ty; r < TT; r += 8) {
        int si = bj * TT + tx, sj = bi * TT + r;
        if (si < n && sj < n) tile[r][tx] = A[IDX(si, sj, lda)];
    }
    __syncthreads();
    for (int r = ty; r < TT; r += 8) {
        int di = bi * TT + tx, dj = bj * TT + r;  // destination element (di, dj) = conj(src (dj, di))
        if (di < n && dj < n) {
            if (di > dj) A[IDX(di, dj, lda)] = conjg(tile[tx][r]);
            else if (di == dj) A[IDX(di, dj, lda)] = from_real<T>(realp(tile[tx][r]));
        }
    }
}

template <typename T>
__global__ void copy_kernel(int m, int n, const T* A, long lda, T* B, long ldb) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)m * n) return;
    int i = (int)(idx % m), j = (int)(idx / m);
    B[IDX(i, j, ldb)] = A[IDX(i, j, lda)];
}

template <typename T>
__global__ void zero_kernel(int m, int n, T* A, long lda) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)m * n) return;
    int i = (int)(idx % m), j = (int)(idx / m);
    A[IDX(i, j, lda)] = zero_of<T>();
}

template <typename T>
__global__ void real_to_scalar_kernel(int m, int n, const double* Z, long ldz, T* C, long ldc) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)m * n) return;
    int i = (int)(idx % m), j = (int)(idx / m);
    C[IDX(i, j, ldc)] = from_real<T>(Z[IDX(i, j, ldz)]);
}

// flag <- 1 if any entry of the upper triangle is NaN or Inf.
template <typename T>
__global__ void finite_kernel(int n, const T* A, long lda, int* flag) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * n) return;
    int i = (int)(idx % n), j = (int)(idx / n);
    if (i > j) return;
    T v = A[IDX(i, j, lda)];
    if (!isfinite(realp(v)) || !isfinite(imagp(v))) atomicOr(flag, 1);
}

inline unsigned nblk(long long tot, int bs) { return (unsigned)((tot + bs - 1) / bs); }

}  // namespace

template <typename T>
int fill_lower_from_upper(hipStream_t st, int n, T* A, long lda) {
    if (n <= 0) return 0;
    int nt = (n + TT - 1) / TT;
    hipLaunchKernelGGL(fill_lower_kernel<T>, dim3(nt, nt), dim3(256), 0, st, n, A, lda);
    GEVD_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int copy_matrix(hipStream_t st, int m, int n, const T* A, long lda, T* B, long ldb) {
    if (m <= 0 || n <= 0) return 0;
    hipLaunchKernelGGL(copy_kernel<T>, dim3(nblk((long long)m * n, 256)), dim3(256), 0, st, m, n, A, lda, B, ldb);
    GEVD_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int set_zero(hipStream_t st, int m, int n, T* A, long lda) {
    if (m <= 0 || n <= 0) return 0;
    hipLaunchKernelGGL(zero_kernel<T>, dim3(nblk((long long)m * n, 256)), dim3(256), 0, st, m, n, A, lda);
    GEVD_LAUNCH_CHECK();
    return 0;
}

int real_to_scalar_d(hipStream_t st, int m, int n, const double* Z, long ldz, double* C, long ldc) {
    if (m <= 0 || n <= 0) return 0;
    hipLaunchKernelGGL(real_to_scalar_kernel<double>, dim3(nblk((long long)m * n, 256)), dim3(256), 0, st, m, n,
                       Z, ldz, C, ldc);
    GEVD_LAUNCH_CHECK();
    return 0;
}

int real_to_scalar_z(hipStream_t st, int m, int n, const double* Z, long ldz, zdouble* C, long ldc) {
    if (m <= 0 || n <= 0) return 0;
    hipLaunchKernelGGL(real_to_scalar_kernel<zdouble>, dim3(nblk((long long)m * n, 256)), dim3(256), 0, st, m,
                       n, Z, ldz, C, ldc);
    GEVD_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int check_finite_upper(hipStream_t st, int n, const T* A, long lda, int* flag) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(finite_kernel<T>, dim3(nblk((long long)n * n, 256)), dim3(256), 0, st, n, A, lda, flag);
    GEVD_LAUNCH_CHECK();
    return 0;
}

#define INST(T)                                                                    \
    template int fill_lower_from_upper<T>(hipStream_t, int, T*, long);             \
    template int copy_matrix<T>(hipStream_t, int, int, const T*, long, T*, long);  \
    template int set_zero<T>(hipStream_t, int, int, T*, long);                     \
    template int check_finite_upper<T>(hipStream_t, int, const T*, long, int*);
INST(double)
INST(zdouble)
#undef INST

}  // namespace gevd
