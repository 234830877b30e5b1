// FP64 refinement of the wanted eigenpairs computed by the reduced-precision
// form (full -> band and stage-1 back-transformation products on the FP32
// matrix cores).  The method is the iterative refinement of Ogita and
// Aishima for symmetric eigendecompositions (a Newton-type correction built
// from matrix products only), applied to the nev-dimensional subspace of the
// wanted vectors: with X (n x nev) the current vectors,
//     G = X^H X,  M = X^H A X,  R = I - G,  lambda_i = M_ii / G_ii,
//     E_ij = (M_ij + lambda_j R_ij) / (lambda_j - lambda_i)   if |lambda_j - lambda_i| > delta
//     E_ij = R_ij / 2                                          otherwise (and on the diagonal),
//     X <- X + X E,
// with the cluster threshold delta = 2 (||M - diag(lambda)||_F + ||A|| ||R||_F)
// (Frobenius norms bound the 2-norms; ||A|| is taken as max |lambda|).  The
// products run in FP64 on the original A.  The correction acts inside
// span(X): components of the true eigenvectors outside it are not restored,
// so the refined accuracy is limited by how well the reduced-precision
// stages captured the wanted invariant subspace.
#include <algorithm>

#include "stages.hpp"

namespace gevd {
namespace {

constexpr int RNT = 1024;

template <typename T>
__global__ __launch_bounds__(RNT) void oa_prep(int k, const T* G, const T* M, long ld, double* lam, double* delta) {
    __shared__ double red[RNT / WAVE];
    for (int i = threadIdx.x; i < k; i += RNT) lam[i] = realp(M[IDX(i, i, ld)]) / realp(G[IDX(i, i, ld)]);
    __syncthreads();
    double off = 0.0, rr = 0.0, amax = 0.0;
    for (long x = threadIdx.x; x < (long)k * k; x += RNT) {
        const int j = (int)(x / k), i = (int)(x - (long)j * k);
        const T g = G[IDX(i, j, ld)];
        const T r = (i == j ? from_real<T>(1.0) : zero_of<T>()) - g;
        rr += abs2(r);
        T mo = M[IDX(i, j, ld)];
        if (i == j) mo = mo - from_real<T>(lam[i]);
        off += abs2(mo);
    }
    for (int i = threadIdx.x; i < k; i += RNT) amax = fmax(amax, fabs(lam[i]));
    off = block_sum<RNT>(off, red);
    rr = block_sum<RNT>(rr, red);
    // block max
    for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, WAVE));
    __syncthreads();
    if (threadIdx.x % WAVE == 0) red[threadIdx.x / WAVE] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int w = 0; w < RNT / WAVE; ++w) a = fmax(a, red[w]);
        *delta = 2.0 * (sqrt(off) + a * sqrt(rr));
    }
}

template <typename T>
__global__ void oa_coeffs(int k, const T* G, const T* M, long ld, const double* lam, const double* delta, T* E) {
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (long)k * k) return;
    const int j = (int)(x / k), i = (int)(x - (long)j * k);
    const T r = (i == j ? from_real<T>(1.0) : zero_of<T>()) - G[IDX(i, j, ld)];
    T e = from_real<T>(0.5) * r;
    if (i != j) {
        const double gap = lam[j] - lam[i];
        if (fabs(gap) > *delta) e = div_r(M[IDX(i, j, ld)] + lam[j] * r, gap);
    }
    E[IDX(i, j, ld)] = e;
}

// Ascending order of the refined values: rank of each (ties by index),
// then the columns and values are gathered into place.
__global__ void rank_kernel(int k, const double* lam, int* dest) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    const double v = lam[i];
    int r = 0;
    for (int q = 0; q < k; ++q) {
        const double w = lam[q];
        r += (w < v) || (w == v && q < i);
    }
    dest[i] = r;
}

template <typename T>
__global__ void gather_cols(int n, int k, const T* X, long ldx, const int* dest, const double* lam, T* Y, long ldy,
                            double* eval) {
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (long)n * k) return;
    const int c = (int)(x / n), r = (int)(x - (long)c * n);
    const int d = min(max(dest[c], 0), k - 1);
    Y[IDX(r, d, ldy)] = X[IDX(r, c, ldx)];
    if (r == 0) eval[d] = lam[c];
}

}  // namespace

template <typename T>
size_t refine_ws_elems(int n, int k) {
    return 2 * (size_t)n * k + 3 * (size_t)k * k + 2 * (size_t)k + 64;
}

template <typename T>
int refine(const StageCtx& c, int n, int k, const T* A, long lda, T* X, long ldx, double* eval, T* work, int iters) {
    Fp32Gemm fp64(false);
    T* P = work;                       // n x k
    T* Xn = P + (size_t)n * k;         // n x k
    T* G = Xn + (size_t)n * k;         // k x k
    T* M = G + (size_t)k * k;
    T* E = M + (size_t)k * k;
    double* lam = reinterpret_cast<double*>(E + (size_t)k * k);
    double* delta = lam + k;
    int* dest = reinterpret_cast<int*>(delta + 8);
    const T one = from_real<T>(1.0), zero = zero_of<T>();
    int rc = 0;
    for (int it = 0; it < iters; ++it) {
        if ((rc = gemm<T>(c.st, OP_N, OP_N, n, k, n, one, A, lda, X, ldx, zero, P, n))) return rc;
        if ((rc = gemm<T>(c.st, OP_C, OP_N, k, k, n, one, X, ldx, X, ldx, zero, G, k))) return rc;
        if ((rc = gemm<T>(c.st, OP_C, OP_N, k, k, n, one, X, ldx, P, n, zero, M, k))) return rc;
        hipLaunchKernelGGL(oa_prep<T>, dim3(1), dim3(RNT), 0, c.st, k, G, M, (long)k, lam, delta);
        GEVD_LAUNCH_CHECK();
        const long kk = (long)k * k;
        hipLaunchKernelGGL(oa_coeffs<T>, dim3((unsigned)((kk + 255) / 256)), dim3(256), 0, c.st, k, G, M, (long)k,
                           lam, delta, E);
        GEVD_LAUNCH_CHECK();
        if ((rc = copy_matrix<T>(c.st, n, k, X, ldx, Xn, n))) return rc;
        if ((rc = gemm<T>(c.st, OP_N, OP_N, n, k, k, one, X, ldx, E, k, one, Xn, n))) return rc;
        if ((rc = copy_matrix<T>(c.st, n, k, Xn, n, X, ldx))) return rc;
    }
    // final Rayleigh quotients of the refined vectors, then ascending order
    if ((rc = gemm<T>(c.st, OP_N, OP_N, n, k, n, one, A, lda, X, ldx, zero, P, n))) return rc;
    if ((rc = gemm<T>(c.st, OP_C, OP_N, k, k, n, one, X, ldx, X, ldx, zero, G, k))) return rc;
    if ((rc = gemm<T>(c.st, OP_C, OP_N, k, k, n, one, X, ldx, P, n, zero, M, k))) return rc;
    hipLaunchKernelGGL(oa_prep<T>, dim3(1), dim3(RNT), 0, c.st, k, G, M, (long)k, lam, delta);
    GEVD_LAUNCH_CHECK();
    hipLaunchKernelGGL(rank_kernel, dim3((k + 255) / 256), dim3(256), 0, c.st, k, lam, dest);
    GEVD_LAUNCH_CHECK();
    const long nk = (long)n * k;
    hipLaunchKernelGGL(gather_cols<T>, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, c.st, n, k, X, ldx, dest,
                       lam, Xn, (long)n, eval);
    GEVD_LAUNCH_CHECK();
    return copy_matrix<T>(c.st, n, k, Xn, n, X, ldx);
}

template size_t refine_ws_elems<double>(int, int);
template size_t refine_ws_elems<zdouble>(int, int);
template int refine<double>(const StageCtx&, int, int, const double*, long, double*, long, double*, double*, int);
template int refine<zdouble>(const StageCtx&, int, int, const zdouble*, long, zdouble*, long, double*, zdouble*,
                             int);

}  // namespace gevd
