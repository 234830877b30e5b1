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

// A <- -A (m x n).
template <typename T>
__global__ void negate_kernel(int m, int n, T* A, long lda) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)m * n) return;
    int i = (int)(idx % m), j = (int)(idx / m);
    A[IDX(i, j, lda)] = -A[IDX(i, j, lda)];
}

// X[:, j] *= 1/sqrt(-ev[j]) (ev[j] < 0: an eigenvalue of -S).
template <typename T>
__global__ void scale_cols_kernel(int m, int n, T* X, long ldx, const double* ev) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)m * n) return;
    int i = (int)(idx % m), j = (int)(idx / m);
    X[IDX(i, j, ldx)] = X[IDX(i, j, ldx)] * (1.0 / sqrt(-ev[j]));
}

// G[:, j] = conj(C[:, j]) * (f[j] * (e ? e[j] : 1)), and B = conj(C) if B is
// not null (m x n).
template <typename T>
__global__ void conj_scale_kernel(int m, int n, const T* C, long ldc, const double* f, const double* e, T* G,
                                  long ldg, T* B, long ldb) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)m * n) return;
    int i = (int)(idx % m), j = (int)(idx / m);
    const T c = conjg(C[IDX(i, j, ldc)]);
    const double w = e ? f[j] * e[j] : f[j];
    G[IDX(i, j, ldg)] = c * w;
    if (B) B[IDX(i, j, ldb)] = c;
}

template <typename T>
__global__ void scale_diag_kernel(int n, T* A, long lda, double s) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) A[IDX(i, i, lda)] = A[IDX(i, i, lda)] * s;
}

// Z <- Z + Z^H in place: the workgroup of tile pair (bi, bj), bi >= bj,
// reads both 32 x 32 tiles into LDS before writing either, so no other
// workgroup touches them; the diagonal of the result is real.
template <typename T>
__global__ __launch_bounds__(256) void herm_sum_kernel(int n, T* Z, long ldz) {
    __shared__ T lo[TT][TT + 1];  // tile (bi, bj): rows bi*TT.., cols bj*TT..
    __shared__ T up[TT][TT + 1];  // tile (bj, bi)
    const int bi = blockIdx.x, bj = blockIdx.y;
    if (bi < bj) return;
    const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;  // 32 x 8
    for (int r = ty; r < TT; r += 8) {
        const int i = bi * TT + tx, j = bj * TT + r;  // lo[r][tx] = Z(i, j)
        if (i < n && j < n) lo[r][tx] = Z[IDX(i, j, ldz)];
        const int i2 = bj * TT + tx, j2 = bi * TT + r;  // up[r][tx] = Z(i2, j2)
        if (i2 < n && j2 < n) up[r][tx] = Z[IDX(i2, j2, ldz)];
    }
    __syncthreads();
    for (int r = ty; r < TT; r += 8) {
        // element (i, j) of tile (bi, bj): Z(i, j) + conj(Z(j, i)); Z(j, i) is up[tx... ]
        const int i = bi * TT + tx, j = bj * TT + r;
        if (i < n && j < n) {
            // Z(j, i) sits in tile (bj, bi) at row j - bj*TT = r, column i - bi*TT = tx: up[tx][r]
            T v = lo[r][tx] + conjg(up[tx][r]);
            if (i == j) v = from_real<T>(realp(v));
            Z[IDX(i, j, ldz)] = v;
        }
        if (bi != bj) {
            const int i2 = bj * TT + tx, j2 = bi * TT + r;  // (i2, j2) = Z(i2, j2) + conj(Z(j2, i2))
            // Z(j2, i2) sits in tile (bi, bj) at row j2 - bi*TT = r, column i2 - bj*TT = tx: lo[tx][r]
            if (i2 < n && j2 < n) Z[IDX(i2, j2, ldz)] = up[r][tx] + conjg(lo[tx][r]);
        }
    }
}

// sigma[i] = -ev[n-1-i]: eigenvalues of S ascending from those of -S.
__global__ void negate_reverse_kernel(int n, const double* ev, double* sigma) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) sigma[i] = -ev[n - 1 - i];
}

// out[0] = max |Re U_ii|, out[1] = min |Re U_ii| over the diagonal of U
// (one workgroup, fixed-order reduction).
template <typename T>
__global__ __launch_bounds__(256) void diag_range_kernel(int n, const T* U, long ldu, double* out) {
    __shared__ double smax[256], smin[256];
    double mx = 0.0, mn = 1.0e308;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double d = fabs(realp(U[IDX(i, i, ldu)]));
        mx = fmax(mx, d);
        mn = fmin(mn, d);
    }
    smax[threadIdx.x] = mx;
    smin[threadIdx.x] = mn;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = smax[0];
        out[1] = smin[0];
    }
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

template <typename T>
int negate_matrix(hipStream_t st, int m, int n, T* A, long lda) {
    if (m <= 0 || n <= 0) return 0;
    hipLaunchKernelGGL(negate_kernel<T>, dim3(nblk((long long)m * n, 256)), dim3(256), 0, st, m, n, A, lda);
    GEVD_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int scale_cols_rsqrt_neg(hipStream_t st, int m, int n, T* X, long ldx, const double* ev) {
    if (m <= 0 || n <= 0) return 0;
    hipLaunchKernelGGL(scale_cols_kernel<T>, dim3(nblk((long long)m * n, 256)), dim3(256), 0, st, m, n, X, ldx,
                       ev);
    GEVD_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int scale_diag(hipStream_t st, int n, T* A, long lda, double s) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(scale_diag_kernel<T>, dim3(nblk(n, 256)), dim3(256), 0, st, n, A, lda, s);
    GEVD_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int herm_sum_inplace(hipStream_t st, int n, T* Z, long ldz) {
    if (n <= 0) return 0;
    const int nt = (n + TT - 1) / TT;
    hipLaunchKernelGGL(herm_sum_kernel<T>, dim3(nt, nt), dim3(256), 0, st, n, Z, ldz);
    GEVD_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int conj_scale_cols(hipStream_t st, int m, int n, const T* C, long ldc, const double* f, const double* e, T* G,
                    long ldg, T* B, long ldb) {
    if (m <= 0 || n <= 0) return 0;
    hipLaunchKernelGGL(conj_scale_kernel<T>, dim3(nblk((long long)m * n, 256)), dim3(256), 0, st, m, n, C, ldc, f,
                       e, G, ldg, B, ldb);
    GEVD_LAUNCH_CHECK();
    return 0;
}

int negate_reverse(hipStream_t st, int n, const double* ev, double* sigma) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(negate_reverse_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, n, ev, sigma);
    GEVD_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int diag_range(hipStream_t st, int n, const T* U, long ldu, double* out) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(diag_range_kernel<T>, dim3(1), dim3(256), 0, st, n, U, ldu, out);
    GEVD_LAUNCH_CHECK();
    return 0;
}

#define INST(T)                                                                    \
    template int negate_matrix<T>(hipStream_t, int, int, T*, long);                \
    template int scale_cols_rsqrt_neg<T>(hipStream_t, int, int, T*, long, const double*); \
    template int diag_range<T>(hipStream_t, int, const T*, long, double*);         \
    template int scale_diag<T>(hipStream_t, int, T*, long, double);                \
    template int herm_sum_inplace<T>(hipStream_t, int, T*, long);                  \
    template int conj_scale_cols<T>(hipStream_t, int, int, const T*, long, const double*, const double*, T*, long, T*, long); \
    template int fill_lower_from_upper<T>(hipStream_t, int, T*, long);             \
    template int copy_matrix<T>(hipStream_t, int, int, const T*, long, T*, long);  \
    template int set_zero<T>(hipStream_t, int, int, T*, long);                     \
    template int check_finite_upper<T>(hipStream_t, int, const T*, long, int*);
INST(double)
INST(zdouble)
#undef INST

}  // namespace gevd
