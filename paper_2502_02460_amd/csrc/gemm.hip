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
// Tiling: a workgroup of 4 wave64s owns a 64 x 64 output tile, each wave
// 32 x 32 as 2 x 2 MFMA blocks of 16 x 16; large products use 8 waves on a
// 128 x 128 tile (each wave 64 x 32), which halves the operand traffic per
// flop, and products with one side of at most 64 use 8 waves on 128 x 64 or
// 64 x 128.  The inner dimension advances in slabs of 16 staged through LDS
// (double-buffered, one barrier per slab).  The MFMA is issued as D = op(B)^T op(A)^T so that
// 16 lanes of a register hold 16 consecutive rows of one column of C: every
// store instruction writes 128-byte column segments of the column-major C.
// Complex products run on separately staged real/imaginary tiles.  Tiles
// with wave blocks of at most 32 x 32 use three real MFMAs per complex
// k-step (Gauss: P1 = re*re, P2 = im*im, P3 = (re + im)(re + im); real part
// P1 - P2, imaginary part P3 - P1 - P2, formed once in the epilogue), 3/4
// of the four-product form's matrix-core work; larger wave blocks and the
// FP32 compute type use four (re*re - im*im, re*im + im*re).
//
// Reduced-precision form: inside a Fp32Gemm scope the operands are rounded
// to FP32 when staged into LDS and the products run on the FP32 matrix
// cores (v_mfma_f32_16x16x4_f32, FP32 accumulation, twice the FP64 rate);
// the result is widened and combined with alpha / beta in FP64.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "kernels.hpp"

namespace gevd {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

constexpr int BK = 16, NT = 256;

// Accumulator of a 16x16 MFMA block and the MFMA itself, by compute type.
template <typename CT> struct Acc;
template <> struct Acc<double> {
    typedef dbl4 type;
    __device__ static inline dbl4 mma(double b, double a, dbl4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c, 0, 0, 0);
    }
};
template <> struct Acc<float> {
    typedef flt4 type;
    __device__ static inline flt4 mma(float b, float a, flt4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(b, a, c, 0, 0, 0);
    }
};

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
    int rev;     // bit 0: tile rows in descending order, bit 1: tile columns descending
    int amask;   // structural zeros of op(A): 1 for l < i, 2 for l > i (from kmode)
    int bmask;   // structural zeros of op(B): 1 for l > j, 2 for l < j
    int bm, bn;  // workgroup tile (for tile-level triangle tests)
    long long sA, sB, sC;
    int splitk;
    T* work;
    const int* amap;  // op(A) = A (N only, no structural zeros): inner index l reads column amap[l]
    const int* cmap;  // output column j is stored to column cmap[j] (< 0: skipped)
};

// v or conj(v), chosen per element without a branch
__device__ inline double conj_if(double v, bool) { return v; }
__device__ inline zdouble conj_if(zdouble v, bool c) { return {v.x, c ? -v.y : v.y}; }

// Operand loads through a buffer resource based near the slab: a byte
// offset at or beyond the resource's size (OOB) returns zero and touches no
// memory, so masked elements need neither a branch nor a valid address, and
// the compiler cannot turn the load into a conditional one.  Offsets from
// the base stay below 2^31 bytes (checked on the host from the leading
// dimensions).
constexpr unsigned OOB = 0x80000000u;
__device__ inline __amdgpu_buffer_rsrc_t rsrc_of(const void* base) {
    // stride 0, size 2^31 - 1 bytes, 32-bit data format (raw dword access)
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, 0x7fffffff, 0x00020000);
}
__device__ inline double bload(double*, __amdgpu_buffer_rsrc_t r, unsigned off) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    const u2 u = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    double v;
    __builtin_memcpy(&v, &u, sizeof v);
    return v;
}
__device__ inline zdouble bload(zdouble*, __amdgpu_buffer_rsrc_t r, unsigned off) {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    const u4 u = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    zdouble v;
    __builtin_memcpy(&v, &u, sizeof v);
    return v;
}
// Every offset from a slab's base is below 161 leading dimensions (at most
// 128 + 16 columns of the slab, plus a row range of at most one leading
// dimension), so leading dimensions under 2^31 / 192 bytes keep all offsets
// below 2^31.
constexpr long MAX_LD_BYTES = (1L << 31) / 192;


// Output tile of a workgroup.  Workgroups are dispatched to the 8 XCDs
// round-robin (block b on XCD b % 8), each XCD with its own L2: blocks are
// renumbered so that every XCD gets a contiguous range of tiles, and inside
// it tiles go in groups of GM tile rows, so the workgroups resident on one
// XCD at a time cover a compact block of C and share their A and B panels.
// Products whose tiles differ in work (one triangle of tiles computed, or a
// triangular operand clipping the inner range) keep the plain column-major
// order: contiguous ranges would load some XCDs far more than others.  Their
// rows or columns run in descending order where that puts the tiles with
// the longest inner range first (workgroups are dispatched in index order,
// so the largest jobs start first and the short ones fill the tail).
constexpr int NXCD = 8, GM = 8;
__device__ inline void tile_of(int bid, int nblocks, int tiles_m, bool swizzle, int rev, int& ti, int& tj) {
    if (!swizzle) {
        ti = bid % tiles_m;
        tj = bid / tiles_m;
        if (rev & 1) ti = tiles_m - 1 - ti;
        if (rev & 2) tj = nblocks / tiles_m - 1 - tj;
        return;
    }
    const int per = nblocks / NXCD;
    int l = bid;
    if (bid < per * NXCD) l = (bid % NXCD) * per + bid / NXCD;
    const int tiles_n = nblocks / tiles_m;
    const int in_group = GM * tiles_n;
    const int first = (l / in_group) * GM;
    const int gm = min(tiles_m - first, GM);
    const int r = l % in_group;
    ti = first + r % gm;
    tj = r / gm;
}

// Workgroup tile BM x BN = (WGM WM) x (WGN WN): WGM x WGN waves, each wave
// owns WM x WN as (WM/16) x (WN/16) MFMA blocks.
template <typename T, typename CT, int OPA, int OPB, int WM, int WN, int WGM = 2, int WGN = 2>
__global__ __launch_bounds__(WAVE * WGM * WGN) __attribute__((amdgpu_waves_per_eu(2))) void gemm_kernel(GemmP<T> p) {
    typedef typename Acc<CT>::type AccT;
    constexpr bool CX = is_cplx<T>::value;
    constexpr int NC = CX ? 2 : 1;
    constexpr int NTK = WAVE * WGM * WGN;  // threads
    constexpr int BM = WGM * WM, BN = WGN * WN;
    constexpr int FA = WM / 16, FB = WN / 16;  // MFMA blocks per wave
    constexpr int LA = BM * BK / NTK, LB = BN * BK / NTK;  // elements loaded per thread
    // Row pitch BM + 1 / BN + 1 (odd): the transposed stagings (16 lanes
    // writing one column, 16 consecutive k) then fall on 16 distinct bank
    // pairs; a 16-lane read of one row is contiguous whatever the pitch.
    // (Measured on gfx950: pitch + 1 runs the large products 2-4 % faster
    // than + 4, and + 16 up to 40 % slower.)
    __shared__ CT sA[NC][2][BK][BM + 1];
    __shared__ CT sB[NC][2][BK][BN + 1];

    int ti, tj;
    tile_of(blockIdx.x, gridDim.x, p.tiles_m,
            p.tmode == T_ALL && (p.kmode == K_FULL || p.kmode == K_A_HERM_LOWER), p.rev, ti, tj);
    // triangle modes skip tiles whose every element lies on the other side
    if ((p.tmode == T_UPPER_TILES || p.tmode == T_UPPER_STRICT) && ti * BM > tj * BN + BN - 1) return;
    if ((p.tmode == T_LOWER_TILES || p.tmode == T_LOWER_STRICT) && ti * BM + BM - 1 < tj * BN) return;
    const T* A = p.A + (long long)blockIdx.y * p.sA;
    const T* B = p.B + (long long)blockIdx.y * p.sB;
    T* C = p.C + (long long)blockIdx.y * p.sC;
    const int i0 = ti * BM, j0 = tj * BN;

    int kbeg = 0, kend = p.k;
    if (p.kmode == K_B_UPPER || p.kmode == K_AU_BU || p.kmode == K_AL_BU) kend = min(kend, j0 + BN);
    if (p.kmode == K_A_LOWER || p.kmode == K_AL_BU) kend = min(kend, i0 + BM);
    if (p.kmode == K_A_UPPER || p.kmode == K_AU_BU) kbeg = i0 / BK * BK;
    if (p.kmode == K_B_LOWER) kbeg = j0 / BK * BK;
    if (p.splitk > 1) {
        int len = max(kend - kbeg, 0);
        int chunk = ((len + p.splitk - 1) / p.splitk + BK - 1) / BK * BK;
        int kb = kbeg + (int)blockIdx.z * chunk;
        kend = min(kend, kb + chunk);
        kbeg = kb;
    }

    const int t = threadIdx.x;
    const int lane = t % WAVE, w = t / WAVE;
    const int wm = w % WGM, wn = w / WGM;

    // three-product complex form for the FP64 compute type, on the tiles
    // whose wave blocks (at most 32 x 32) leave room for the third
    // accumulator set (larger ones would spill); two waves per SIMD
    // (amdgpu_waves_per_eu) keep the four-wave tiles at two workgroups per CU
    constexpr bool G3 = CX && std::is_same<CT, double>::value && FA * FB <= 4;
    AccT accR[FA][FB], accI[FA][FB], accX[FA][FB];
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b) {
            accR[a][b] = AccT{0, 0, 0, 0};
            accI[a][b] = AccT{0, 0, 0, 0};
            accX[a][b] = AccT{0, 0, 0, 0};
        }

    // The next operand slab is loaded into registers while the MFMAs read the
    // current LDS buffer, then stored to the other buffer: one barrier per
    // slab.  (A second register set for two slabs of lead costs occupancy
    // and measured slower on gfx950.)
    T ra[LA], rb[LB];
    bool ca[LA], cb[LB];  // conjugate when staged (applied at the LDS store, after the loads have landed)
    // Every thread issues its slab loads unconditionally in straight-line
    // code (buffer loads; masked elements read zero), so that they are all in
    // flight together and the first wait comes at the LDS store after the
    // slab's MFMAs.  (Branches around the loads made the compiler wait for
    // each group of loads before issuing the next.)
    const bool herm = p.kmode == K_A_HERM_LOWER;
    auto gload = [&](int kt) {
        // Hermitian A kept in its lower triangle: a slab wholly above the
        // diagonal is read conjugate-transposed with the row-contiguous
        // mapping; elsewhere element (i, l) with i < l is conj(A[l, i])
        const bool herm_up = herm && i0 + BM - 1 < kt;
        if (OPA == OP_N && p.amap) {
            // the merge products' column map: columns anywhere in A, flat loads
#pragma unroll
            for (int r = 0; r < LA; ++r) {
                const int e = t + r * NTK;
                const int i = i0 + e % BM, l = kt + e / BM;
                const bool ok = i < p.m && l < kend;
                const int c = p.amap[ok ? l : kbeg];
                const T v = A[ok ? IDX(i, c, p.lda) : 0];
                ra[r] = ok ? v : zero_of<T>();
                ca[r] = false;
            }
        } else {
            // based at the smallest stored row and column the slab reads
            const int rb0 = OPA == OP_N ? (herm ? min(i0, kt) : i0) : kt;
            const int cb0 = OPA == OP_N ? (herm ? min(i0, kt) : kt) : i0;
            const auto rs = rsrc_of(A + IDX(rb0, cb0, p.lda));
#pragma unroll
            for (int r = 0; r < LA; ++r) {
                const int e = t + r * NTK;
                int ii, ll;
                if (OPA == OP_N) {
                    ii = herm_up ? e / BK : e % BM;
                    ll = herm_up ? e % BK : e / BM;
                } else {
                    ii = e / BK;
                    ll = e % BK;
                }
                const int i = i0 + ii, l = kt + ll;
                const bool ok = i < p.m && l < kend && !(p.amask == 1 && l < i) && !(p.amask == 2 && l > i);
                int sr, sc;
                bool cj;
                if (OPA == OP_N) {
                    const bool up = herm && i < l;
                    sr = up ? l : i;
                    sc = up ? i : l;
                    cj = up;
                } else {
                    sr = l;
                    sc = i;
                    cj = OPA == OP_C;
                }
                const unsigned off =
                    ok ? (unsigned)(((size_t)(sr - rb0) + (size_t)(sc - cb0) * p.lda) * sizeof(T)) : OOB;
                ra[r] = bload((T*)nullptr, rs, off);
                ca[r] = cj && ok;
            }
        }
        const int rb0 = OPB == OP_N ? kt : j0, cb0 = OPB == OP_N ? j0 : kt;
        const auto rs = rsrc_of(B + IDX(rb0, cb0, p.ldb));
#pragma unroll
        for (int r = 0; r < LB; ++r) {
            const int e = t + r * NTK;
            int jj, ll;
            if (OPB == OP_N) { ll = e % BK; jj = e / BK; }
            else { jj = e % BN; ll = e / BN; }
            const int j = j0 + jj, l = kt + ll;
            const bool ok = j < p.n && l < kend && !(p.bmask == 1 && l > j) && !(p.bmask == 2 && l < j);
            const size_t el = OPB == OP_N ? IDX(ll, jj, p.ldb) : IDX(jj, ll, p.ldb);
            const unsigned off = ok ? (unsigned)(el * sizeof(T)) : OOB;
            rb[r] = bload((T*)nullptr, rs, off);
            cb[r] = OPB == OP_C && ok;
        }
    };
    auto sstore = [&](int buf, int kt) {
        const bool herm_up = p.kmode == K_A_HERM_LOWER && i0 + BM - 1 < kt;
#pragma unroll
        for (int r = 0; r < LA; ++r) {
            const int e = t + r * NTK;
            int ii, ll;
            if (OPA == OP_N && !herm_up) { ii = e % BM; ll = e / BM; }
            else { ii = e / BK; ll = e % BK; }
            const T v = conj_if(ra[r], ca[r]);
            sA[0][buf][ll][ii] = (CT)realp(v);
            if (CX) sA[NC - 1][buf][ll][ii] = (CT)imagp(v);
        }
#pragma unroll
        for (int r = 0; r < LB; ++r) {
            const int e = t + r * NTK;
            int jj, ll;
            if (OPB == OP_N) { ll = e % BK; jj = e / BK; }
            else { jj = e % BN; ll = e / BN; }
            const T v = conj_if(rb[r], cb[r]);
            sB[0][buf][ll][jj] = (CT)realp(v);
            if (CX) sB[NC - 1][buf][ll][jj] = (CT)imagp(v);
        }
    };
    auto compute = [&](int buf) {
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            const int kr = kk * 4 + lane / 16;
            CT aR[FA], bR[FB], aI[FA], bI[FB];
#pragma unroll
            for (int q = 0; q < FA; ++q) {
                aR[q] = sA[0][buf][kr][wm * WM + q * 16 + lane % 16];
                if (CX) aI[q] = sA[NC - 1][buf][kr][wm * WM + q * 16 + lane % 16];
            }
#pragma unroll
            for (int q = 0; q < FB; ++q) {
                bR[q] = sB[0][buf][kr][wn * WN + q * 16 + lane % 16];
                if (CX) bI[q] = sB[NC - 1][buf][kr][wn * WN + q * 16 + lane % 16];
            }
            // D[j][i] += sum_k opB[k][j] opA[i][k]; issued in phases so
            // that consecutive MFMAs update independent accumulators
#pragma unroll
            for (int qa = 0; qa < FA; ++qa)
#pragma unroll
                for (int qb = 0; qb < FB; ++qb)
                    accR[qa][qb] = Acc<CT>::mma(bR[qb], aR[qa], accR[qa][qb]);
            if constexpr (G3) {
                // accR = P1 (above), accI = P2, accX = P3
#pragma unroll
                for (int qa = 0; qa < FA; ++qa)
#pragma unroll
                    for (int qb = 0; qb < FB; ++qb)
                        accI[qa][qb] = Acc<CT>::mma(bI[qb], aI[qa], accI[qa][qb]);
                CT aS[FA], bS[FB];
#pragma unroll
                for (int q = 0; q < FA; ++q) aS[q] = aR[q] + aI[q];
#pragma unroll
                for (int q = 0; q < FB; ++q) bS[q] = bR[q] + bI[q];
#pragma unroll
                for (int qa = 0; qa < FA; ++qa)
#pragma unroll
                    for (int qb = 0; qb < FB; ++qb)
                        accX[qa][qb] = Acc<CT>::mma(bS[qb], aS[qa], accX[qa][qb]);
            } else if (CX) {
#pragma unroll
                for (int qa = 0; qa < FA; ++qa)
#pragma unroll
                    for (int qb = 0; qb < FB; ++qb)
                        accI[qa][qb] = Acc<CT>::mma(bI[qb], aR[qa], accI[qa][qb]);
#pragma unroll
                for (int qa = 0; qa < FA; ++qa)
#pragma unroll
                    for (int qb = 0; qb < FB; ++qb)
                        accR[qa][qb] = Acc<CT>::mma(-bI[qb], aI[qa], accR[qa][qb]);
#pragma unroll
                for (int qa = 0; qa < FA; ++qa)
#pragma unroll
                    for (int qb = 0; qb < FB; ++qb)
                        accI[qa][qb] = Acc<CT>::mma(bR[qb], aI[qa], accI[qa][qb]);
            }
        }
    };

    if (kbeg < kend) {
        gload(kbeg);
        sstore(0, kbeg);
        __syncthreads();
        int buf = 0;
        // the last slab is peeled off, so that the loop body loads and
        // stages unconditionally (no load can be in flight across the back
        // edge, and the compiler places no wait before the next slab's loads)
        int kt = kbeg;
        for (; kt + BK < kend; kt += BK) {
            gload(kt + BK);
            compute(buf);
            sstore(buf ^ 1, kt + BK);
            __syncthreads();
            buf ^= 1;
        }
        compute(buf);
    }

    // Epilogue.  The f64 16x16x4 MFMA leaves D[4r + lane/16][lane%16] in
    // register r of each lane (checked on gfx950); with D = op(B)^T op(A)^T
    // that is C row lane%16, C column 4r + lane/16 of the 16 x 16 block.
    const bool strict_up = p.tmode == T_UPPER_STRICT, strict_lo = p.tmode == T_LOWER_STRICT;
    const bool use_beta = !is_zero(p.beta) && p.splitk <= 1;
    // One 16-row block at a time: destinations first (with the merge
    // products' column map), then every old value of C the block needs, all
    // loads issued before any is used, then the stores.
#pragma unroll
    for (int qa = 0; qa < FA; ++qa) {
        const int row = i0 + wm * WM + qa * 16 + lane % 16;
        int col[FB][4];
        bool ok[FB][4];
#pragma unroll
        for (int qb = 0; qb < FB; ++qb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // f32 16x16x4 differs: register r of lane l holds D[4 (l/16) + r][l%16]
                const int c = j0 + wn * WN + qb * 16 + (std::is_same<CT, float>::value ? 4 * (lane / 16) + r
                                                                                      : 4 * r + lane / 16);
                ok[qb][r] = row < p.m && c < p.n && !(strict_up && row > c) && !(strict_lo && row < c);
                col[qb][r] = c;
            }
        if (p.cmap) {
#pragma unroll
            for (int qb = 0; qb < FB; ++qb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = p.cmap[ok[qb][r] ? col[qb][r] : 0];
                    ok[qb][r] = ok[qb][r] && c >= 0;
                    col[qb][r] = c;
                }
        }
        T old[FB][4];
        if (use_beta && p.cmap) {
#pragma unroll
            for (int qb = 0; qb < FB; ++qb)
#pragma unroll
                for (int r = 0; r < 4; ++r) old[qb][r] = C[ok[qb][r] ? IDX(row, col[qb][r], p.ldc) : 0];
        } else if (use_beta) {
            const int rb0 = i0 + wm * WM + qa * 16, cb0 = j0 + wn * WN;
            const auto rs = rsrc_of(C + IDX(rb0, cb0, p.ldc));
#pragma unroll
            for (int qb = 0; qb < FB; ++qb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const unsigned off =
                        ok[qb][r] ? (unsigned)(IDX(row - rb0, col[qb][r] - cb0, p.ldc) * sizeof(T)) : OOB;
                    old[qb][r] = bload((T*)nullptr, rs, off);
                }
        }
#pragma unroll
        for (int qb = 0; qb < FB; ++qb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (!ok[qb][r]) continue;
                T v;
                if constexpr (G3)
                    v = zdouble{accR[qa][qb][r] - accI[qa][qb][r],
                                accX[qa][qb][r] - accR[qa][qb][r] - accI[qa][qb][r]};
                else if constexpr (CX) v = zdouble{(double)accR[qa][qb][r], (double)accI[qa][qb][r]};
                else v = (double)accR[qa][qb][r];
                if (p.splitk > 1) {
                    p.work[(size_t)blockIdx.z * p.m * p.n + IDX(row, col[qb][r], p.m)] = v;
                } else {
                    T out = p.alpha * v;
                    if (use_beta) out = fma_s(p.beta, old[qb][r], out);
                    C[IDX(row, col[qb][r], p.ldc)] = out;
                }
            }
    }
}

// Deterministic reduction of split-K partials: C = alpha sum_z W_z + beta C.
template <typename T>
__global__ void splitk_reduce(int m, int n, int splits, const T* work, T alpha, T beta, T* C, long ldc,
                              int tmode, int bm, int bn) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)m * n) return;
    int row = (int)(idx % m), col = (int)(idx / m);
    if ((tmode == T_UPPER_STRICT && row > col) || (tmode == T_LOWER_STRICT && row < col)) return;
    if ((tmode == T_UPPER_TILES) && (row / bm) * bm > (col / bn) * bn + bn - 1) return;
    if ((tmode == T_LOWER_TILES) && (row / bm) * bm + bm - 1 < (col / bn) * bn) return;
    T s = zero_of<T>();
    for (int z = 0; z < splits; ++z) s += work[(size_t)z * m * n + idx];
    T out = alpha * s;
    if (!is_zero(beta)) out = fma_s(beta, C[IDX(row, col, ldc)], out);
    C[IDX(row, col, ldc)] = out;
}

template <typename T, typename CT, int OPA, int OPB>
void launch_c(hipStream_t st, const GemmP<T>& p, dim3 grid, int cfg) {
    switch (cfg) {
        case 1: hipLaunchKernelGGL((gemm_kernel<T, CT, OPA, OPB, 64, 32>), grid, dim3(NT), 0, st, p); break;
        case 2: hipLaunchKernelGGL((gemm_kernel<T, CT, OPA, OPB, 32, 64>), grid, dim3(NT), 0, st, p); break;
        case 3: hipLaunchKernelGGL((gemm_kernel<T, CT, OPA, OPB, 64, 64>), grid, dim3(NT), 0, st, p); break;
        case 4: hipLaunchKernelGGL((gemm_kernel<T, CT, OPA, OPB, 32, 16>), grid, dim3(NT), 0, st, p); break;
        case 5: hipLaunchKernelGGL((gemm_kernel<T, CT, OPA, OPB, 16, 32>), grid, dim3(NT), 0, st, p); break;
        case 6: hipLaunchKernelGGL((gemm_kernel<T, CT, OPA, OPB, 64, 32, 2, 4>), grid, dim3(8 * WAVE), 0, st, p); break;
        case 7: hipLaunchKernelGGL((gemm_kernel<T, CT, OPA, OPB, 32, 32, 4, 2>), grid, dim3(8 * WAVE), 0, st, p); break;
        case 8: hipLaunchKernelGGL((gemm_kernel<T, CT, OPA, OPB, 32, 32, 2, 4>), grid, dim3(8 * WAVE), 0, st, p); break;
        default: hipLaunchKernelGGL((gemm_kernel<T, CT, OPA, OPB, 32, 32>), grid, dim3(NT), 0, st, p); break;
    }
}

template <typename T, int OPA, int OPB>
void launch_t(hipStream_t st, const GemmP<T>& p, dim3 grid, int cfg) {
    if (g_gemm_fp32) launch_c<T, float, OPA, OPB>(st, p, grid, cfg);
    else launch_c<T, double, OPA, OPB>(st, p, grid, cfg);
}

template <typename T, int OPA>
void launch_b(hipStream_t st, int opB, const GemmP<T>& p, dim3 grid, int cfg) {
    if (opB == OP_N) launch_t<T, OPA, OP_N>(st, p, grid, cfg);
    else if (opB == OP_T) launch_t<T, OPA, OP_T>(st, p, grid, cfg);
    else launch_t<T, OPA, OP_C>(st, p, grid, cfg);
}

// Workgroup tile for a product: 0 = 64x64, 1 = 128x64, 2 = 64x128,
// 3 = 128x128 (four waves each), 4 = 64x32 (outputs at most 32 columns
// wide), 5 = 32x64 (at most 32 rows); eight waves: 6 = 128x128, 7 = 128x64,
// 8 = 64x128.  GEVD_GEMM_TILE forces one (for measurements).
constexpr int NTILE = 9;
constexpr int TILE_BM[NTILE] = {64, 128, 64, 128, 64, 32, 128, 128, 64};
constexpr int TILE_BN[NTILE] = {64, 64, 128, 128, 32, 64, 128, 64, 128};
int g_tile_override = -2;  // -2: not read yet, -1: none
}  // namespace
thread_local int g_tile_force = -1;  // the calling handle's GEVD_OPT_GEMM_TILE (-1: automatic)
namespace {
// Measured on gfx950 (FP64, n = 16384 class shapes, single launches).
// Complex: the eight-wave 64 x 128 tile runs square N/N and N/C products at
// 95 % of the FP64 peak on the method's flops (three-product form); the
// four-wave 64 x 64 tile, also three-product and two workgroups per CU,
// runs C/N products at 96-99 % and rank-128 updates at 68 % against 65 %
// (its second workgroup overlaps one tile's C traffic with another's
// products); 128 x 64 wins for outputs 64 wide.  Real: the eight-wave
// 128 x 128 tile runs square products about 20 % faster than 64 x 64.  The
// large tiles need enough of them to fill the 256 CUs, so medium products
// keep 64 x 64.
int pick_tile(int m, int n, int k, int opA, bool cx, int splitk, int batch, int tmode) {
    if (g_tile_override == -2) {
        const char* e = getenv("GEVD_GEMM_TILE");
        g_tile_override = e ? atoi(e) : -1;
    }
    if (g_tile_force >= 0 && g_tile_force < NTILE) return (cx && g_tile_force == 3) ? 1 : g_tile_force;
    if (g_tile_override >= 0 && g_tile_override < NTILE) return (cx && g_tile_override == 3) ? 1 : g_tile_override;
    if (n <= 32 && m > 32) return 4;
    if (m <= 32 && n > 32) return 5;
    const long long par = (long long)splitk * batch;
    const long long tm = (m + 127) / 128, tn = (n + 127) / 128;
    const bool tri = tmode != T_ALL;
    if (cx) {
        if (n <= 64 && m > 64) return tm * par >= 256 ? 7 : 0;
        if (m <= 64) return tn * par >= 256 ? 8 : 0;
        // C/N products and short inner dimensions: the 64 x 64 tile, when
        // there are enough tiles for two workgroups on every CU
        const long long t64 = (long long)((m + 63) / 64) * ((n + 63) / 64) * par / (tri ? 2 : 1);
        if ((opA == OP_C || k <= 256) && t64 >= 1024) return 0;
        return ((m + 63) / 64) * tn * par / (tri ? 2 : 1) >= 512 ? 8 : 0;
    }
    if (m > 64 && n > 64 && tm * tn * par / (tri ? 2 : 1) >= 512) return 6;
    if (m <= 64 && n > 64 && tn * par >= 256) return 8;
    if (n <= 64 && m > 64 && tm * par >= 256) return 7;
    return 0;
}

// Multiply-adds the product needs given its structural zeros and the
// stored output elements (2 flops each; a complex multiply-add counts 8).
double algorithmic_flops(int m, int n, int k, int kmode, int tmode, bool cx) {
    auto kfor = [&](int i, int j) -> double {
        switch (kmode) {
            case K_B_UPPER: return std::min(k, j + 1);
            case K_A_UPPER: return std::max(0, k - i);
            case K_A_LOWER: return std::min(k, i + 1);
            case K_B_LOWER: return std::max(0, k - j);
            case K_AU_BU: return std::max(0, std::min(k, j + 1) - i);
            case K_AL_BU: return std::min(k, std::min(i, j) + 1);
            default: return k;
        }
    };
    double macs = 0.0;
    const bool tiles_up = tmode == T_UPPER_TILES || tmode == T_UPPER_STRICT;
    const bool tiles_lo = tmode == T_LOWER_TILES || tmode == T_LOWER_STRICT;
    if (kmode == K_FULL && tmode == T_ALL) {
        macs = (double)m * n * k;
    } else if (kmode == K_AU_BU || kmode == K_AL_BU) {
        // the inner length depends on both i and j: sum over the stored
        // elements (upper when a triangle of tiles is kept)
        const bool up = tmode != T_ALL;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < (up ? std::min(m, j + 1) : m); ++i) macs += kfor(i, j);
    } else if (tmode == T_ALL) {
        if (kmode == K_B_UPPER || kmode == K_B_LOWER)
            for (int j = 0; j < n; ++j) macs += (double)m * kfor(0, j);
        else
            for (int i = 0; i < m; ++i) macs += (double)n * kfor(i, 0);
    } else {
        // stored elements: i <= j (upper) or i >= j (lower); the inner
        // length depends on i only for the modes used with a triangle
        for (int i = 0; i < m; ++i) {
            const double cnt = tiles_up ? std::max(0, n - i) : (tiles_lo ? std::min(n, i + 1) : n);
            macs += cnt * kfor(i, i);
        }
    }
    return 2.0 * macs * (cx ? 4.0 : 1.0);
}

}  // namespace

thread_local bool g_gemm_fp32 = false;

template <typename T>
int gemm(hipStream_t st, int opA, int opB, int m, int n, int k, T alpha, const T* A, long lda, const T* B,
         long ldb, T beta, T* C, long ldc, int kmode, int tmode, Batch batch, int splitk, T* work, const int* amap,
         const int* cmap) {
    if (m <= 0 || n <= 0 || batch.count <= 0) return 0;
    if (amap && (opA != OP_N || kmode != K_FULL)) return GEVD_E_STATE;
    if (!is_cplx<T>::value) {  // conjugation is the identity for real data
        if (opA == OP_C) opA = OP_T;
        if (opB == OP_C) opB = OP_T;
    }
    if (splitk > 1 && (work == nullptr || batch.count != 1 || cmap)) splitk = 1;
    if ((long)sizeof(T) * std::max(lda, std::max(ldb, ldc)) >= MAX_LD_BYTES) return GEVD_E_STATE;
    GemmP<T> p;
    p.m = m; p.n = n; p.k = k;
    p.A = A; p.lda = lda; p.B = B; p.ldb = ldb; p.C = C; p.ldc = ldc;
    p.alpha = alpha; p.beta = beta;
    p.kmode = kmode; p.tmode = tmode;
    // longest inner ranges first: the range grows with the tile row for
    // K_A_LOWER / K_AL_BU and with the tile column for K_B_UPPER / K_AU_BU /
    // K_AL_BU (K_A_UPPER and K_B_LOWER shrink along them: ascending already)
    p.rev = ((kmode == K_A_LOWER || kmode == K_AL_BU) ? 1 : 0) |
            ((kmode == K_B_UPPER || kmode == K_AU_BU || kmode == K_AL_BU) ? 2 : 0);
    p.amask = (kmode == K_A_UPPER || kmode == K_AU_BU) ? 1 : (kmode == K_A_LOWER || kmode == K_AL_BU) ? 2 : 0;
    p.bmask = (kmode == K_B_UPPER || kmode == K_AU_BU || kmode == K_AL_BU) ? 1 : kmode == K_B_LOWER ? 2 : 0;
    const int cfg = pick_tile(m, n, k, opA, is_cplx<T>::value, splitk, batch.count, tmode);
    const int bm = TILE_BM[cfg], bn = TILE_BN[cfg];
    p.bm = bm;
    p.bn = bn;
    p.tiles_m = (m + bm - 1) / bm;
    const int tiles_n = (n + bn - 1) / bn;
    p.sA = batch.sA; p.sB = batch.sB; p.sC = batch.sC;
    p.splitk = splitk; p.work = work;
    p.amap = amap; p.cmap = cmap;
    dim3 grid(p.tiles_m * tiles_n, batch.count, splitk);
    KProbe probe(st, g_gemm_fp32 ? GEVD_K_GEMM32 : GEVD_K_GEMM,
                 g_kstats ? batch.count * algorithmic_flops(m, n, k, kmode, tmode, is_cplx<T>::value) : 0.0);
    if (opA == OP_N) launch_b<T, OP_N>(st, opB, p, grid, cfg);
    else if (opA == OP_T) launch_b<T, OP_T>(st, opB, p, grid, cfg);
    else launch_b<T, OP_C>(st, opB, p, grid, cfg);
    GEVD_LAUNCH_CHECK();
    if (splitk > 1) {
        long long tot = (long long)m * n;
        hipLaunchKernelGGL(splitk_reduce<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, m, n, splitk,
                           (const T*)work, alpha, beta, C, ldc, tmode, bm, bn);
        GEVD_LAUNCH_CHECK();
    }
    return 0;
}

template int gemm<double>(hipStream_t, int, int, int, int, int, double, const double*, long, const double*, long,
                          double, double*, long, int, int, Batch, int, double*, const int*, const int*);
template int gemm<zdouble>(hipStream_t, int, int, int, int, int, zdouble, const zdouble*, long, const zdouble*,
                           long, zdouble, zdouble*, long, int, int, Batch, int, zdouble*, const int*, const int*);

}  // namespace gevd
