// Step 1 (Cholesky S = U^H U) and step 2 (U -> U^{-1}) of the reduction to
// standard form (paper, section "Solving the generalized eigenproblem").
//
// Cholesky runs over block rows of 256 rows (left-looking): each block row
// first receives the contributions of all finished rows as one MFMA product
// with a long inner dimension, then is factored right-looking in 64-column
// steps: a one-workgroup kernel factors the 64 x 64 diagonal block in LDS
// and also inverts it; the rest of its rows U12 = U11^{-H} S12 is one MFMA
// product with that inverse (no triangular solve on the critical path), and
// the block row's remaining rows take S22 -= U12^H U12 on upper tiles.
//
// The inverse is formed recursively: inv([A B; 0 D]) = [Ai, -Ai B Di; 0, Di],
// with all 64 x 64 diagonal blocks inverted by one batched launch and every
// off-diagonal block produced by two triangular MFMA products.
#include "kernels.hpp"

namespace gevd {
namespace {

constexpr int NB = 64;
constexpr int NTD = 256;

// Factor the jb x jb upper block at S (ld lds) in place; write its inverse to
// Winv (ld NB, zeros below the diagonal).  *info is set to the global
// 1-based minor (gofs + k + 1) of the first non-positive or non-finite pivot.
template <typename T>
__global__ __launch_bounds__(NTD) void potrf_diag_kernel(int jb, T* S, long lds, T* Winv, int* info, int gofs) {
    __shared__ T a[NB][NB + 1];  // a[r][c], upper triangle used
    __shared__ T x[NB][NB + 1];  // the inverse, by columns
    __shared__ int bad;
    if (*info != 0) return;  // an earlier panel already failed
    const int t = threadIdx.x;
    if (t == 0) bad = 0;
    for (int e = t; e < jb * jb; e += NTD) {
        int r = e % jb, c = e / jb;
        a[r][c] = (r <= c) ? S[IDX(r, c, lds)] : zero_of<T>();
    }
    __syncthreads();
    for (int k = 0; k < jb; ++k) {
        if (t == 0) {
            double d = realp(a[k][k]);
            if (!(d > 0.0) || !isfinite(d)) {
                bad = 1;
                atomicCAS(info, 0, gofs + k + 1);
            } else {
                a[k][k] = from_real<T>(sqrt(d));
            }
        }
        __syncthreads();
        if (bad) return;
        const double ukk = realp(a[k][k]);
        for (int c = k + 1 + t; c < jb; c += NTD) a[k][c] = div_r(a[k][c], ukk);
        __syncthreads();
        // trailing: a[r][c] -= conj(a[k][r]) a[k][c], k < r <= c (lane = row,
        // the four waves take every fourth column)
        {
            const int r = t % NB;
            if (r > k && r < jb) {
                const T akr = conjg(a[k][r]);
                for (int c = r + (t / NB + NB - r % 4) % 4; c < jb; c += 4) a[r][c] -= akr * a[k][c];
            }
        }
        __syncthreads();
    }
    // write U11 (upper triangle only)
    for (int e = t; e < jb * jb; e += NTD) {
        int r = e % jb, c = e / jb;
        if (r <= c) S[IDX(r, c, lds)] = a[r][c];
    }
    // inverse by columns: four lanes solve U x = e_c for column c, each
    // summing every fourth term; the partial sums are added in a fixed order
    {
        const int c = t / 4, q = t % 4;
        if (c < jb) {
            if (q == 0) {
                for (int i = c + 1; i < NB; ++i) x[i][c] = zero_of<T>();
                x[c][c] = from_real<T>(1.0 / realp(a[c][c]));
            }
        }
        for (int i = NB - 2; i >= 0; --i) {
            // rows run from the bottom for every column at once (rows i >= c
            // are fixed already), so the loop bound stays uniform
            T sum = zero_of<T>();
            if (c < jb && i < c)
                for (int l = i + 1 + q; l <= c; l += 4) sum += a[i][l] * x[l][c];
            sum += shfl_xor_s(sum, 1);
            sum += shfl_xor_s(sum, 2);
            if (c < jb && i < c && q == 0) x[i][c] = div_r(-sum, realp(a[i][i]));
        }
        if (c < jb && q == 0)
            for (int i = 0; i < jb; ++i) Winv[IDX(i, c, NB)] = x[i][c];
    }
}

// Batched inverse of the diagonal NB x NB blocks of upper triangular U:
// block b covers rows/cols [b*NB, min(n, (b+1)*NB)).  Writes the inverse
// into the same position of Uinv (zeros below the diagonal).
template <typename T>
__global__ __launch_bounds__(NTD) void diag_inv_kernel(int n, const T* U, long ldu, T* Uinv, long ldi) {
    __shared__ T a[NB][NB + 1];
    __shared__ T x[NB][NB + 1];
    const int o = blockIdx.x * NB;
    const int jb = min(NB, n - o);
    const int t = threadIdx.x;
    for (int e = t; e < jb * jb; e += NTD) {
        int r = e % jb, c = e / jb;
        a[r][c] = (r <= c) ? U[IDX(o + r, o + c, ldu)] : zero_of<T>();
    }
    __syncthreads();
    if (t < jb) {
        const int c = t;  // this thread owns column c of the inverse
        for (int i = c + 1; i < NB; ++i) x[i][c] = zero_of<T>();
        x[c][c] = from_real<T>(1.0 / realp(a[c][c]));
        for (int i = c - 1; i >= 0; --i) {
            T s = zero_of<T>();
            for (int l = i + 1; l <= c; ++l) s += a[i][l] * x[l][c];
            x[i][c] = div_r(-s, realp(a[i][i]));
        }
        for (int i = 0; i < jb; ++i) Uinv[IDX(o + i, o + c, ldi)] = x[i][c];
    }
}

template <typename T>
int trtri_rec(hipStream_t st, int o, int s, const T* U, long ldu, T* Uinv, long ldi, T* tmp) {
    if (s <= NB) return 0;  // leaves done by the batched kernel
    int s1 = ((s / 2 + NB - 1) / NB) * NB;
    int s2 = s - s1;
    int rc = trtri_rec(st, o, s1, U, ldu, Uinv, ldi, tmp);
    if (rc) return rc;
    rc = trtri_rec(st, o + s1, s2, U, ldu, Uinv, ldi, tmp);
    if (rc) return rc;
    const T one = from_real<T>(1.0), mone = from_real<T>(-1.0), zero = zero_of<T>();
    // tmp = U12 * Uinv22   (s1 x s2), Uinv22 upper triangular
    rc = gemm<T>(st, OP_N, OP_N, s1, s2, s2, one, U + IDX(o, o + s1, ldu), ldu, Uinv + IDX(o + s1, o + s1, ldi),
                 ldi, zero, tmp, s1, K_B_UPPER);
    if (rc) return rc;
    // Uinv12 = -Uinv11 * tmp, Uinv11 upper triangular
    return gemm<T>(st, OP_N, OP_N, s1, s2, s1, mone, Uinv + IDX(o, o, ldi), ldi, tmp, s1, zero,
                   Uinv + IDX(o, o + s1, ldi), ldi, K_A_UPPER);
}

// Rows per block row of the Cholesky, and the split of its long inner
// dimension: a block row is updated by one product with inner length j0
// (all finished rows above it), split so that the product has enough
// workgroups to fill the device.
constexpr int NBR = 256;

int chol_splitk(int jb, int width, int k) {
    const long tiles = (long)((jb + 63) / 64) * ((width + 127) / 128);
    int sk = 1;
    while (sk < 16 && tiles * sk < 512 && k / (2 * sk) >= 256) sk *= 2;
    return sk;
}

}  // namespace

template <typename T>
size_t potrf_work_elems(int n) {
    // the diagonal block's inverse, a 64-row strip for U12, then the
    // split-K partials of the block-row update (at most 16 splits of NBR x n)
    return (size_t)NB * NB + 256 + (size_t)NB * std::max(n, 1) + 256 + (size_t)16 * NBR * (size_t)std::max(n, 1);
}
template <typename T>
size_t trtri_work_elems(int n) {
    size_t h = (size_t)(n / 2 + NB);
    return h * h;
}

// Block-row (left-looking) Cholesky.  For each block row of NBR rows:
//  1. R -= U_above^H U_above_row: all finished rows enter through one MFMA
//     product whose inner length is the number of finished rows (the long
//     dimension of the factorisation, so the products run near the matrix
//     cores' rate instead of as rank-64 updates);
//  2. the block row is factored right-looking in 64-column steps: the
//     diagonal 64 x 64 block in LDS (factor and inverse), the rest of its
//     rows U12 = U11^{-H} R12 by one product with that inverse, and the
//     remaining rows of the block row updated by U12^H U12 (upper tiles).
template <typename T>
int potrf(hipStream_t st, int n, T* S, long lds, T* work, int* info_dev) {
    const T one = from_real<T>(1.0), mone = from_real<T>(-1.0), zero = zero_of<T>();
    T* winv = work;
    T* strip = work + (size_t)NB * NB + 256;
    T* skw = strip + (size_t)NB * std::max(n, 1) + 256;
    for (int j0 = 0; j0 < n; j0 += NBR) {
        const int jb = min(NBR, n - j0);
        const int width = n - j0;
        T* R = S + IDX(j0, j0, lds);
        if (j0 > 0) {
            const int sk = chol_splitk(jb, width, j0);
            int rc = gemm<T>(st, OP_C, OP_N, jb, width, j0, mone, S + IDX(0, j0, lds), lds, S + IDX(0, j0, lds), lds,
                             one, R, lds, K_FULL, T_ALL, Batch(), sk, skw);
            if (rc) return rc;
        }
        for (int s0 = 0; s0 < jb; s0 += NB) {
            const int sb = min(NB, jb - s0);
            {
                KProbe probe(st, GEVD_K_OTHER, 0.0);
                hipLaunchKernelGGL(potrf_diag_kernel<T>, dim3(1), dim3(NTD), 0, st, sb, R + IDX(s0, s0, lds), lds,
                                   winv, info_dev, j0 + s0);
                GEVD_LAUNCH_CHECK();
            }
            const int w2 = width - s0 - sb;  // columns right of the diagonal block
            if (w2 <= 0) break;
            T* R12 = R + IDX(s0, s0 + sb, lds);
            // U12 = inv(U11)^H R12 through a strip (whatever the tile height)
            int rc = gemm<T>(st, OP_C, OP_N, sb, w2, sb, one, winv, NB, R12, lds, zero, strip, NB, K_A_LOWER);
            if (rc) return rc;
            if ((rc = copy_matrix<T>(st, sb, w2, strip, NB, R12, lds))) return rc;
            const int r2 = jb - s0 - sb;  // rows of the block row below this step
            if (r2 <= 0) continue;
            // R22 -= U12[:, :r2]^H U12 on the upper tiles of the block row's rest
            rc = gemm<T>(st, OP_C, OP_N, r2, w2, sb, mone, R12, lds, R12, lds, one, R + IDX(s0 + sb, s0 + sb, lds),
                         lds, K_FULL, T_UPPER_TILES);
            if (rc) return rc;
        }
    }
    return 0;
}

template <typename T>
int trtri(hipStream_t st, int n, const T* U, long ldu, T* Uinv, long ldi, T* work) {
    int rc = set_zero<T>(st, n, n, Uinv, ldi);
    if (rc) return rc;
    hipLaunchKernelGGL(diag_inv_kernel<T>, dim3((n + NB - 1) / NB), dim3(NTD), 0, st, n, U, ldu, Uinv, ldi);
    GEVD_LAUNCH_CHECK();
    return trtri_rec<T>(st, 0, n, U, ldu, Uinv, ldi, work);
}

#define INST(T)                                                              \
    template size_t potrf_work_elems<T>(int);                                \
    template size_t trtri_work_elems<T>(int);                                \
    template int potrf<T>(hipStream_t, int, T*, long, T*, int*);             \
    template int trtri<T>(hipStream_t, int, const T*, long, T*, long, T*);
INST(double)
INST(zdouble)
#undef INST

}  // namespace gevd
