// FP64 matrix products on the CDNA4 matrix cores (v_mfma_f64_16x16x4_f64).
//
// One kernel serves every dense contraction of the solver: the Cholesky
// trailing update, the triangular inversion, the two products that form
// A = U^-H H U^-1, the two-sided update of the full -> band reduction, the
// divide-and-conquer merge products and the back-transformations.
// Triangular operands are handled by masking in the tile loaders (the zero
// triangle is never read) and by clipping the inner-dimension range per
// output tile, so triangular products cost what their nonzeros cost.
//
// Tiling: a 256-thread workgroup (4 wave64s) owns a 64 x 64 output tile;
// each wave owns 32 x 32 as 2 x 2 MFMA blocks of 16 x 16.  The inner
// dimension advances in slabs of 16 staged through LDS (double-buffered,
// one barrier per slab).  The MFMA is issued as D = op(B)^T op(A)^T so that
// 16 lanes of a register hold 16 consecutive rows of one column of C: every
// store instruction writes 128-byte column segments of the column-major C.
// Complex products use four real MFMAs per complex k-step (re*re - im*im,
// re*im + im*re) on separately staged real/imaginary tiles.
#include "kernels.hpp"

namespace gevd {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;
constexpr int LDS_PAD = BM + 4;

template <typename T>
struct GemmP {
    int m, n, k;
    const T* A;
    long lda;
    const T* B;
    long ldb;
    T* C;
    long ldc;
    T alpha, beta;
    int kmode, tmode;
    int tiles_m;
    long long sA, sB, sC;
    int splitk;
    T* work;
    const int* amap;  // op(A) = A (N only): inner index l reads column amap[l]
    const int* cmap;  // output column j is stored to column cmap[j] (< 0: skipped)
};

template <typename T, int OPA>
__device__ inline T load_opA(const GemmP<T>& p, const T* A, int i, int l, int kend) {
    if (i >= p.m || l >= kend) return zero_of<T>();
    if (p.kmode == K_A_UPPER && l < i) return zero_of<T>();
    if (p.kmode == K_A_LOWER && l > i) return zero_of<T>();
    if (OPA == OP_N) return A[IDX(i, p.amap ? p.amap[l] : l, p.lda)];
    T v = A[IDX(l, i, p.lda)];
    return OPA == OP_C ? conjg(v) : v;
}

template <typename T, int OPB>
__device__ inline T load_opB(const GemmP<T>& p, const T* B, int l, int j, int kend) {
    if (j >= p.n || l >= kend) return zero_of<T>();
    if (p.kmode == K_B_UPPER && l > j) return zero_of<T>();
    if (p.kmode == K_B_LOWER && l < j) return zero_of<T>();
    if (OPB == OP_N) return B[IDX(l, j, p.ldb)];
    T v = B[IDX(j, l, p.ldb)];
    return OPB == OP_C ? conjg(v) : v;
}


template <typename T, int OPA, int OPB>
__global__ __launch_bounds__(NT) void gemm_kernel(GemmP<T> p) {
    constexpr bool CX = is_cplx<T>::value;
    constexpr int NC = CX ? 2 : 1;
    __shared__ double sA[NC][2][BK][LDS_PAD];
    __shared__ double sB[NC][2][BK][LDS_PAD];

    const int ti = blockIdx.x % p.tiles_m, tj = blockIdx.x / p.tiles_m;
    if ((p.tmode == T_UPPER_TILES || p.tmode == T_UPPER_STRICT) && ti > tj) return;
    if ((p.tmode == T_LOWER_TILES || p.tmode == T_LOWER_STRICT) && ti < tj) return;
    const T* A = p.A + (long long)blockIdx.y * p.sA;
    const T* B = p.B + (long long)blockIdx.y * p.sB;
    T* C = p.C + (long long)blockIdx.y * p.sC;
    const int i0 = ti * BM, j0 = tj * BN;

    int kbeg = 0, kend = p.k;
    if (p.kmode == K_B_UPPER) kend = min(kend, j0 + BN);
    if (p.kmode == K_A_LOWER) kend = min(kend, i0 + BM);
    if (p.kmode == K_A_UPPER) kbeg = i0;
    if (p.kmode == K_B_LOWER) kbeg = j0;
    if (p.splitk > 1) {
        int len = max(kend - kbeg, 0);
        int chunk = ((len + p.splitk - 1) / p.splitk + BK - 1) / BK * BK;
        int kb = kbeg + (int)blockIdx.z * chunk;
        kend = min(kend, kb + chunk);
        kbeg = kb;
    }

    const int t = threadIdx.x;
    const int lane = t % WAVE, w = t / WAVE;
    const int wm = w % 2, wn = w / 2;

    dbl4 accR[2][2], accI[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            accR[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
            accI[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
        }

    T ra[4], rb[4];
    auto gload = [&](int kt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int e = t + r * NT;
            int ii, ll;
            if (OPA == OP_N) { ii = e % BM; ll = e / BM; }
            else { ii = e / BK; ll = e % BK; }
            ra[r] = load_opA<T, OPA>(p, A, i0 + ii, kt + ll, kend);
            int jj;
            if (OPB == OP_N) { ll = e % BK; jj = e / BK; }
            else { jj = e % BN; ll = e / BN; }
            rb[r] = load_opB<T, OPB>(p, B, kt + ll, j0 + jj, kend);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int e = t + r * NT;
            int ii, ll, jj;
            if (OPA == OP_N) { ii = e % BM; ll = e / BM; }
            else { ii = e / BK; ll = e % BK; }
            sA[0][buf][ll][ii] = realp(ra[r]);
            if (CX) sA[NC - 1][buf][ll][ii] = imagp(ra[r]);
            if (OPB == OP_N) { ll = e % BK; jj = e / BK; }
            else { jj = e % BN; ll = e / BN; }
            sB[0][buf][ll][jj] = realp(rb[r]);
            if (CX) sB[NC - 1][buf][ll][jj] = imagp(rb[r]);
        }
    };

    if (kbeg < kend) {
        gload(kbeg);
        sstore(0);
        __syncthreads();
        int buf = 0;
        for (int kt = kbeg; kt < kend; kt += BK) {
            const bool more = kt + BK < kend;
            if (more) gload(kt + BK);
#pragma unroll
            for (int kk = 0; kk < BK / 4; ++kk) {
                const int kr = kk * 4 + lane / 16;
                double aR[2], bR[2], aI[2], bI[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    aR[q] = sA[0][buf][kr][wm * 32 + q * 16 + lane % 16];
                    bR[q] = sB[0][buf][kr][wn * 32 + q * 16 + lane % 16];
                    if (CX) {
                        aI[q] = sA[NC - 1][buf][kr][wm * 32 + q * 16 + lane % 16];
                        bI[q] = sB[NC - 1][buf][kr][wn * 32 + q * 16 + lane % 16];
                    }
                }
#pragma unroll
                for (int qa = 0; qa < 2; ++qa)
#pragma unroll
                    for (int qb = 0; qb < 2; ++qb) {
                        // D[j][i] += sum_k opB[k][j] opA[i][k]
                        accR[qa][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bR[qb], aR[qa], accR[qa][qb], 0, 0, 0);
                        if (CX) {
                            accR[qa][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-bI[qb], aI[qa], accR[qa][qb], 0, 0, 0);
                            accI[qa][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bI[qb], aR[qa], accI[qa][qb], 0, 0, 0);
                            accI[qa][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bR[qb], aI[qa], accI[qa][qb], 0, 0, 0);
                        }
                    }
            }
            if (more) sstore(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }

    // Epilogue.  The f64 16x16x4 MFMA leaves D[4r + lane/16][lane%16] in
    // register r of each lane (checked on gfx950); with D = op(B)^T op(A)^T
    // that is C row lane%16, C column 4r + lane/16 of the 16 x 16 block.
    const bool strict_up = p.tmode == T_UPPER_STRICT, strict_lo = p.tmode == T_LOWER_STRICT;
    const bool use_beta = !is_zero(p.beta);
#pragma unroll
    for (int qa = 0; qa < 2; ++qa)
#pragma unroll
        for (int qb = 0; qb < 2; ++qb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = i0 + wm * 32 + qa * 16 + lane % 16;
                int col = j0 + wn * 32 + qb * 16 + 4 * r + lane / 16;
                if (row >= p.m || col >= p.n) continue;
                if (strict_up && row > col) continue;
                if (strict_lo && row < col) continue;
                if (p.cmap) {
                    col = p.cmap[col];
                    if (col < 0) continue;
                }
                T v;
                if constexpr (CX) v = zdouble{accR[qa][qb][r], accI[qa][qb][r]};
                else v = accR[qa][qb][r];
                if (p.splitk > 1) {
                    p.work[(size_t)blockIdx.z * p.m * p.n + IDX(row, col, p.m)] = v;
                } else {
                    T out = p.alpha * v;
                    if (use_beta) out = fma_s(p.beta, C[IDX(row, col, p.ldc)], out);
                    C[IDX(row, col, p.ldc)] = out;
                }
            }
}

// Deterministic reduction of split-K partials: C = alpha sum_z W_z + beta C.
template <typename T>
__global__ void splitk_reduce(int m, int n, int splits, const T* work, T alpha, T beta, T* C, long ldc,
                              int tmode) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)m * n) return;
    int row = (int)(idx % m), col = (int)(idx / m);
    if ((tmode == T_UPPER_STRICT && row > col) || (tmode == T_LOWER_STRICT && row < col)) return;
    if ((tmode == T_UPPER_TILES) && row / BM > col / BN) return;
    if ((tmode == T_LOWER_TILES) && row / BM < col / BN) return;
    T s = zero_of<T>();
    for (int z = 0; z < splits; ++z) s += work[(size_t)z * m * n + idx];
    T out = alpha * s;
    if (!is_zero(beta)) out = fma_s(beta, C[IDX(row, col, ldc)], out);
    C[IDX(row, col, ldc)] = out;
}

template <typename T, int OPA, int OPB>
void launch_t(hipStream_t st, const GemmP<T>& p, dim3 grid) {
    hipLaunchKernelGGL((gemm_kernel<T, OPA, OPB>), grid, dim3(NT), 0, st, p);
}

template <typename T, int OPA>
void launch_b(hipStream_t st, int opB, const GemmP<T>& p, dim3 grid) {
    if (opB == OP_N) launch_t<T, OPA, OP_N>(st, p, grid);
    else if (opB == OP_T) launch_t<T, OPA, OP_T>(st, p, grid);
    else launch_t<T, OPA, OP_C>(st, p, grid);
}

}  // namespace

template <typename T>
int gemm(hipStream_t st, int opA, int opB, int m, int n, int k, T alpha, const T* A, long lda, const T* B,
         long ldb, T beta, T* C, long ldc, int kmode, int tmode, Batch batch, int splitk, T* work, const int* amap,
         const int* cmap) {
    if (m <= 0 || n <= 0 || batch.count <= 0) return 0;
    if (amap && opA != OP_N) return GEVD_E_STATE;
    if (!is_cplx<T>::value) {  // conjugation is the identity for real data
        if (opA == OP_C) opA = OP_T;
        if (opB == OP_C) opB = OP_T;
    }
    if (splitk > 1 && (work == nullptr || batch.count != 1 || cmap)) splitk = 1;
    GemmP<T> p;
    p.m = m; p.n = n; p.k = k;
    p.A = A; p.lda = lda; p.B = B; p.ldb = ldb; p.C = C; p.ldc = ldc;
    p.alpha = alpha; p.beta = beta;
    p.kmode = kmode; p.tmode = tmode;
    p.tiles_m = (m + BM - 1) / BM;
    const int tiles_n = (n + BN - 1) / BN;
    p.sA = batch.sA; p.sB = batch.sB; p.sC = batch.sC;
    p.splitk = splitk; p.work = work;
    p.amap = amap; p.cmap = cmap;
    dim3 grid(p.tiles_m * tiles_n, batch.count, splitk);
    if (opA == OP_N) launch_b<T, OP_N>(st, opB, p, grid);
    else if (opA == OP_T) launch_b<T, OP_T>(st, opB, p, grid);
    else launch_b<T, OP_C>(st, opB, p, grid);
    GEVD_LAUNCH_CHECK();
    if (splitk > 1) {
        long long tot = (long long)m * n;
        hipLaunchKernelGGL(splitk_reduce<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, m, n, splitk,
                           (const T*)work, alpha, beta, C, ldc, tmode);
        GEVD_LAUNCH_CHECK();
    }
    return 0;
}

template int gemm<double>(hipStream_t, int, int, int, int, int, double, const double*, long, const double*, long,
                          double, double*, long, int, int, Batch, int, double*, const int*, const int*);
template int gemm<zdouble>(hipStream_t, int, int, int, int, int, zdouble, const zdouble*, long, const zdouble*,
                           long, zdouble, zdouble*, long, int, int, Batch, int, zdouble*, const int*, const int*);

}  // namespace gevd
