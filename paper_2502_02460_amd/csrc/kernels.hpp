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
