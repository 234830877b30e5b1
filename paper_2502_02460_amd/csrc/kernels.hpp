// Internal launchers shared by the host pipeline (not part of the C ABI).
#pragma once
#include "common.hpp"
#include "../../include/gevd.h"
#include "kstats.hpp"

namespace gevd {

enum Op { OP_N = 0, OP_T = 1, OP_C = 2 };

// Structural zeros the GEMM loaders impose (entries on the zero side are
// never read from memory, so that triangle may hold anything):
enum KMode {
    K_FULL = 0,
    K_B_UPPER = 1,  // op(B)[l, j] = 0 for l > j
    K_A_UPPER = 2,  // op(A)[i, l] = 0 for l < i
    K_A_LOWER = 3,  // op(A)[i, l] = 0 for l > i
    K_B_LOWER = 4,  // op(B)[l, j] = 0 for l < j
    K_A_HERM_LOWER = 5,  // op(A) = A (N) Hermitian, read from its lower triangle only
    K_AU_BU = 6,    // op(A) upper and op(B) upper: l in [i, j]
    K_AL_BU = 7,    // op(A) lower and op(B) upper: l <= min(i, j)
};
// Output tiles computed / elements stored.
enum TMode {
    T_ALL = 0,
    T_UPPER_TILES = 1,   // tiles with tile_row <= tile_col (whole tiles stored)
    T_LOWER_TILES = 2,   // tiles with tile_row >= tile_col
    T_UPPER_STRICT = 3,  // upper tiles, and only elements i <= j stored
    T_LOWER_STRICT = 4,  // lower tiles, and only elements i >= j stored
};

// Products issued on this thread while set run on the FP32 matrix cores
// (operands rounded to FP32, FP32 accumulation); see Fp32Gemm.
extern thread_local bool g_gemm_fp32;
// Tile forced on the products issued on this thread (-1: chosen per shape);
// set from the calling handle's GEVD_OPT_GEMM_TILE for each entry point.
extern thread_local int g_tile_force;
struct Fp32Gemm {
    bool prev;
    explicit Fp32Gemm(bool on) : prev(g_gemm_fp32) { g_gemm_fp32 = on; }
    ~Fp32Gemm() { g_gemm_fp32 = prev; }
};

struct Batch {
    int count = 1;
    long long sA = 0, sB = 0, sC = 0;  // element strides between batch members
};

// C = alpha op(A) op(B) + beta C, m x n, inner dimension k.  When beta is
// zero C is not read.  splitk > 1 splits the inner dimension over blockIdx.z
// into a workspace of splitk*m*n scalars (work) and reduces deterministically.
template <typename T>
int gemm(hipStream_t st, int opA, int opB, int m, int n, int k, T alpha, const T* A, long lda, const T* B,
         long ldb, T beta, T* C, long ldc, int kmode = K_FULL, int tmode = T_ALL, Batch batch = Batch(),
         int splitk = 1, T* work = nullptr, const int* amap = nullptr, const int* cmap = nullptr);

// Elementwise helpers.
template <typename T>
int fill_lower_from_upper(hipStream_t st, int n, T* A, long lda);  // A[i,j] = conj(A[j,i]) for i > j
template <typename T>
int copy_matrix(hipStream_t st, int m, int n, const T* A, long lda, T* B, long ldb);
template <typename T>
int set_zero(hipStream_t st, int m, int n, T* A, long lda);
int real_to_scalar_d(hipStream_t st, int m, int n, const double* Z, long ldz, double* C, long ldc);
int real_to_scalar_z(hipStream_t st, int m, int n, const double* Z, long ldz, zdouble* C, long ldc);
template <typename T>
int check_finite_upper(hipStream_t st, int n, const T* A, long lda, int* flag);
template <typename T>
int negate_matrix(hipStream_t st, int m, int n, T* A, long lda);                        // A <- -A
template <typename T>
int scale_diag(hipStream_t st, int n, T* A, long lda, double s);                         // A_ii <- s A_ii
template <typename T>
int herm_sum_inplace(hipStream_t st, int n, T* Z, long ldz);                            // Z <- Z + Z^H
template <typename T>
int scale_cols_rsqrt_neg(hipStream_t st, int m, int n, T* X, long ldx, const double* ev);  // X_j /= sqrt(-ev_j)
int negate_reverse(hipStream_t st, int n, const double* ev, double* sigma);             // sigma_i = -ev_{n-1-i}
// G[:, j] = conj(C[:, j]) f_j (times e_j if e), and B = conj(C) if B
template <typename T>
int conj_scale_cols(hipStream_t st, int m, int n, const T* C, long ldc, const double* f, const double* e, T* G,
                    long ldg, T* B, long ldb);
template <typename T>
int diag_range(hipStream_t st, int n, const T* U, long ldu, double* out);  // out = {max, min} |Re U_ii|

// Cholesky / triangular inversion.
template <typename T>
int potrf(hipStream_t st, int n, T* S, long lds, T* work, int* info_dev);
template <typename T>
int trtri(hipStream_t st, int n, const T* U, long ldu, T* Uinv, long ldi, T* work);
template <typename T>
size_t potrf_work_elems(int n);
template <typename T>
size_t trtri_work_elems(int n);

}  // namespace gevd
