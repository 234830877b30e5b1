// First stage of the two-stage reduction (the route the paper recommends for
// subsets of eigenvectors, section "ELPA - Usability"): full Hermitian A ->
// Hermitian band B of half-bandwidth b, A = Q1 B Q1^H.
//
// For each panel of b columns starting at column c, the m x b block below
// the band (rows c+b .. n-1) is QR-factored by Householder reflectors
// H_s = I - tau_s v_s v_s^H (beta real), then the trailing m x m block is
// updated two-sidedly with the compact WY form Q = I - V T V^H:
//   X = A22 V T,  W = X - 1/2 V (T^H V^H X),  A22 <- A22 - W V^H - V W^H,
// all as MFMA products.  The panel QR is latency-bound: one persistent
// launch per panel with a grid barrier per column (very tall panels: one
// row-parallel launch per column whose reductions finish in the last
// workgroup to arrive); sums run in a fixed order, so results are
// deterministic.
#include <algorithm>

#include "stages.hpp"

namespace gevd {
namespace {

constexpr int PT = 256;    // threads per panel workgroup = rows per workgroup
constexpr int MAXB = 64;  // largest supported band

template <typename T>
struct PanelScratch {
    T tau[MAXB];
    T w[MAXB];
    T scale;
    double beta;
    unsigned counter;
    unsigned bar;        // grid barrier of the persistent panel kernel (monotonic)
    T prow[2][MAXB];     // pivot row of the current column (by column parity)
};

// Largest grid of the persistent panel kernel: all its workgroups (one CU
// each) must be resident together, also beside the persistent panels of a
// few concurrent solves on the same device; larger panels use one launch
// per column.
constexpr int PANEL_MAX_WG = 64;
constexpr unsigned long long PANEL_WAIT_TICKS = 120ull * 100000000ull;  // 120 s at 100 MHz

template <typename T>
__device__ inline void make_reflector(T alpha, double xn2, T* tau, T* scale, double* beta) {
    const double ar = realp(alpha), ai = imagp(alpha);
    if (xn2 == 0.0 && ai == 0.0) {
        *tau = zero_of<T>();
        *scale = zero_of<T>();
        *beta = ar;
        return;
    }
    const double nrm = sqrt(ar * ar + ai * ai + xn2);
    const double bt = ar >= 0.0 ? -nrm : nrm;
    *tau = div_r(from_real<T>(bt) - alpha, bt);
    *scale = div_s(from_real<T>(1.0), alpha - from_real<T>(bt));
    *beta = bt;
}

// The whole panel in one launch, column-parallel: lane j of every wave owns
// column j of RPW consecutive panel rows and keeps them in registers, so the
// panel is read and written once and the row sums of a column step are
// per-lane sums (no cross-lane reduction).  Per column s:
//  1. apply reflector s-1: a[i] -= x_i * (scale conj(tau) w_j), with x the
//     reflector's column broadcast from its lane (rows <= s-1 are zero there,
//     see 2);
//  2. the wave holding row s takes the pivot row out of its registers (kept
//     in pv and published for the other workgroups) and zeroes it, so every
//     lane's rows <= s are zero from now on;
//  3. y_j = sum_i conj(x_i) a_j[i] over the wave's rows (x = column s, so
//     y_s = ||x||^2), added over the waves in fixed order and written as the
//     workgroup's partial;
//  4. one grid barrier; every workgroup adds all partials in workgroup order
//     (the same values everywhere, deterministic) and forms reflector s and
//     w_j = v^H P[:, j] = conj(scale) y_j + P[s, j] itself;
//  5. the wave holding row s stores the finished row s of the panel (beta on
//     the diagonal, P[s, j] - conj(tau) w_j right of it, the x entries of the
//     finished columns left of it) and of V.
// The rows at and below nref are stored once at the end.  All workgroups
// are resident together (one per CU at most PANEL_MAX_WG), so every barrier
// is reached; a time bound turns a broken invariant into an error flag.
// bar_base: barrier count before this panel (the counter is zeroed once per
// reduction).
constexpr int RPW = 32;                  // panel rows per wave
constexpr int PNW = PT / RPW;            // waves per workgroup (PT rows)
constexpr int PCT = PNW * WAVE;          // threads per workgroup
template <typename T>
__global__ __launch_bounds__(PCT) void panel_cols(T* P, long lda, int m, int b, int nref, T* Vp,
                                                  PanelScratch<T>* ps, T* partial, unsigned bar_base, int* hang) {
    __shared__ T ysh[PNW][WAVE];
    __shared__ T ysum[PNW][WAVE];
    __shared__ int stop;
    const int tid = threadIdx.x, g = tid / WAVE, j = tid % WAVE;
    const int G = gridDim.x;
    const int rb = blockIdx.x * PT + g * RPW;  // first panel row of this wave
    const bool col = j < b;
    T a[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) a[i] = (col && rb + i < m) ? P[IDX(rb + i, j, lda)] : zero_of<T>();
    if (tid == 0) stop = 0;
    T tau = zero_of<T>(), scale = zero_of<T>(), wj = zero_of<T>(), myscale = zero_of<T>();
    for (int s = 0; s <= nref; ++s) {
        if (s > 0) {
            const int sp = s - 1;
            const T ck = scale * (conjg(tau) * wj);  // zero outside columns s .. b-1
#pragma unroll
            for (int i = 0; i < RPW; ++i) a[i] -= lane_bcast(a[i], sp) * ck;
        }
        if (s >= nref) break;
        const int par = s & 1;
        const bool top = rb <= s && s < rb + RPW;  // this wave holds pivot row s
        T pv = zero_of<T>();
        if (top) {
#pragma unroll
            for (int i = 0; i < RPW; ++i)
                if (rb + i == s) {
                    pv = a[i];
                    a[i] = zero_of<T>();
                }
            sys_store(&ps->prow[par][j], pv);
            __builtin_amdgcn_s_waitcnt(0);  // stored before this wave reaches the barrier below
        }
        // four interleaved partial sums, added in a fixed order
        T y0 = zero_of<T>(), y1 = zero_of<T>(), y2 = zero_of<T>(), y3 = zero_of<T>();
#pragma unroll
        for (int i = 0; i < RPW; i += 4) {
            y0 += conjg(lane_bcast(a[i], s)) * a[i];
            y1 += conjg(lane_bcast(a[i + 1], s)) * a[i + 1];
            y2 += conjg(lane_bcast(a[i + 2], s)) * a[i + 2];
            y3 += conjg(lane_bcast(a[i + 3], s)) * a[i + 3];
        }
        ysh[g][j] = (y0 + y1) + (y2 + y3);
        __syncthreads();
        if (g == 0) {
            T t = ysh[0][j];
#pragma unroll
            for (int q = 1; q < PNW; ++q) t += ysh[q][j];
            sys_store(&partial[((size_t)par * G + blockIdx.x) * WAVE + j], t);
            // grid barrier for column s; the partials and the pivot row are
            // stored at system scope and complete before the arrival
            __builtin_amdgcn_s_waitcnt(0);
            if (j == 0) {
                const unsigned target = bar_base + (unsigned)(s + 1) * (unsigned)G;
                __hip_atomic_fetch_add(&ps->bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                unsigned spins = 0;
                unsigned long long t0 = 0;
                while (__hip_atomic_load(&ps->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                    if ((++spins & 63u) == 0) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                        const unsigned long long now = wall_clock64();
                        if (t0 == 0) t0 = now;
                        if (now - t0 > PANEL_WAIT_TICKS ||
                            __hip_atomic_load(hang, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                            atomicOr(hang, 1);
                            stop = 1;
                            break;
                        }
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
        }
        __syncthreads();
        if (stop) return;
        // all partials of column s: wave g adds workgroups g, g + PNW, ...
        // (independent loads, four at a time), then the waves' sums in order
        const T prj = sys_load(&ps->prow[par][j]);
        T acc = zero_of<T>();
        for (int q0 = g; q0 < G; q0 += PNW * 4) {
            T v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * PNW;
                v[u] = q < G ? sys_load(&partial[((size_t)par * G + q) * WAVE + j]) : zero_of<T>();
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc += v[u];
        }
        ysum[g][j] = acc;
        __syncthreads();
        T tot = ysum[0][j];
#pragma unroll
        for (int q = 1; q < PNW; ++q) tot += ysum[q][j];
        double beta;
        make_reflector<T>(lane_bcast(prj, s), realp(lane_bcast(tot, s)), &tau, &scale, &beta);
        wj = (j > s && col) ? conjg(scale) * tot + prj : zero_of<T>();
        if (j == s) myscale = scale;
        if (top && col) {  // row s of the panel and of V is final
            T pr = pv, vr = zero_of<T>();
            if (j < s) {
                vr = pv * myscale;
            } else if (j == s) {
                pr = from_real<T>(beta);
                vr = from_real<T>(1.0);
            } else {
                pr = pv - conjg(tau) * wj;
            }
            P[IDX(s, j, lda)] = pr;
            Vp[IDX(s, j, m)] = vr;
        }
        if (blockIdx.x == 0 && tid == 0) {
            ps->tau[s] = tau;
            ps->scale = scale;
            ps->beta = beta;
        }
    }
    if (col) {
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = rb + i;
            if (r < m && r >= nref) {
                P[IDX(r, j, lda)] = a[i];
                Vp[IDX(r, j, m)] = j < nref ? a[i] * myscale : zero_of<T>();
            }
        }
    }
}

// One launch per panel column s (0 <= s <= nref), for panels whose
// persistent grid would be too large and for solves that share the device
// (no co-residency needed).  Same column-parallel layout as panel_cols (lane
// j of every wave holds column j of RPW rows):
//  1. if s > 0, apply reflector s-1 to columns j >= s: a -= x_i scale
//     conj(tau) w_j on the rows below s-1 (x = column s-1), a -= conj(tau)
//     w_j on row s-1 (v = 1 there); the lane of column s-1 stores V's column;
//  2. store the updated columns;
//  3. if s < nref, per-lane sums y_j = sum_{i > s} conj(x_i) a_j[i] (x =
//     column s, so y_s = ||x||^2), added over the waves; the last workgroup
//     to finish adds all partials in workgroup order, forms reflector s from
//     alpha = P[s, s] and y_s, stores tau, scale, beta and w_j = conj(scale)
//     y_j + P[s, j], and writes beta to P[s, s].
template <typename T>
__global__ __launch_bounds__(PCT) void panel_col_step(T* P, long lda, int m, int b, int s, int nref, T* Vp,
                                                      PanelScratch<T>* ps, T* partial) {
    __shared__ T ysh[PNW][WAVE];
    __shared__ int last;
    const int tid = threadIdx.x, g = tid / WAVE, j = tid % WAVE;
    const int G = gridDim.x;
    const int rb = blockIdx.x * PT + g * RPW;
    const bool col = j < b;
    T a[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) a[i] = (col && rb + i < m) ? P[IDX(rb + i, j, lda)] : zero_of<T>();
    if (s > 0) {
        const int sp = s - 1;
        const T scale = ps->scale;
        const T c1 = (j > sp && col) ? conjg(ps->tau[sp]) * ps->w[j] : zero_of<T>();
        const T ck = scale * c1;
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = rb + i;
            const T x = lane_bcast(a[i], sp);
            if (r > sp) a[i] -= x * ck;
            else if (r == sp) a[i] -= c1;
            if (j == sp && r < m)
                Vp[IDX(r, sp, m)] = r > sp ? x * scale : (r == sp ? from_real<T>(1.0) : zero_of<T>());
        }
#pragma unroll
        for (int i = 0; i < RPW; ++i)
            if (col && j >= s && rb + i < m) P[IDX(rb + i, j, lda)] = a[i];
    }
    if (s >= nref) return;
    T y0 = zero_of<T>(), y1 = zero_of<T>(), y2 = zero_of<T>(), y3 = zero_of<T>();
#pragma unroll
    for (int i = 0; i < RPW; i += 4) {
        y0 += conjg(rb + i > s ? lane_bcast(a[i], s) : zero_of<T>()) * a[i];
        y1 += conjg(rb + i + 1 > s ? lane_bcast(a[i + 1], s) : zero_of<T>()) * a[i + 1];
        y2 += conjg(rb + i + 2 > s ? lane_bcast(a[i + 2], s) : zero_of<T>()) * a[i + 2];
        y3 += conjg(rb + i + 3 > s ? lane_bcast(a[i + 3], s) : zero_of<T>()) * a[i + 3];
    }
    ysh[g][j] = (y0 + y1) + (y2 + y3);
    __syncthreads();
    if (g == 0) {
        T t = ysh[0][j];
#pragma unroll
        for (int q = 1; q < PNW; ++q) t += ysh[q][j];
        partial[(size_t)blockIdx.x * WAVE + j] = t;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // partials and the stored columns
    __syncthreads();
    if (tid == 0) last = (atomicAdd(&ps->counter, 1u) == (unsigned)G - 1);
    __syncthreads();
    if (!last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    T acc = zero_of<T>();
    for (int q = g; q < G; q += PNW) acc += partial[(size_t)q * WAVE + j];
    ysh[g][j] = acc;
    __syncthreads();
    T tot = ysh[0][j];
#pragma unroll
    for (int q = 1; q < PNW; ++q) tot += ysh[q][j];
    const T prj = col ? P[IDX(s, j, lda)] : zero_of<T>();
    T tau, scale;
    double beta;
    make_reflector<T>(lane_bcast(prj, s), realp(lane_bcast(tot, s)), &tau, &scale, &beta);
    if (g == 0) {
        if (j > s && col) ps->w[j] = conjg(scale) * tot + prj;
        if (j == 0) {
            ps->tau[s] = tau;
            ps->scale = scale;
            ps->beta = beta;
            ps->counter = 0;
            P[IDX(s, s, lda)] = from_real<T>(beta);
        }
    }
}

// T (b x b upper) of Q = H_0 ... H_{b-1} = I - V T V^H from the Gram matrix
// G = V^H V: T[s, s] = tau_s, T[0:s, s] = -tau_s T[0:s, 0:s] G[0:s, s].  G is
// staged in LDS; four lanes share each row's dot product (strided quarters
// of the inner range, added in a fixed order with two lane exchanges).
constexpr int TFT = 4 * MAXB;
template <typename T>
__global__ __launch_bounds__(TFT) void tfactor_kernel(int b, const T* G, const PanelScratch<T>* ps, T* Tf) {
    __shared__ T t[MAXB][MAXB + 1];
    __shared__ T g[MAXB][MAXB + 1];
    const int tid = threadIdx.x, i = tid / 4, q = tid % 4;
    for (int e = tid; e < b * b; e += TFT) g[e % b][e / b] = G[e];
    for (int e = tid; e < MAXB * MAXB; e += TFT) t[e / MAXB][e % MAXB] = zero_of<T>();
    __syncthreads();
    for (int s = 0; s < b; ++s) {
        T acc = zero_of<T>();
        if (i < s)
            for (int l = i + q; l < s; l += 4) acc += t[i][l] * g[l][s];
        acc += shfl_xor_s(acc, 1);
        acc += shfl_xor_s(acc, 2);
        if (q == 0) {
            if (i < s) t[i][s] = -(ps->tau[s] * acc);
            else if (i == s) t[i][s] = ps->tau[s];
        }
        __syncthreads();
    }
    for (int e = tid; e < b * b; e += TFT) Tf[e] = t[e % b][e / b];
}

// Band in lower band storage from the reduced A: columns of processed panels
// take the (final) diagonal block and the R factor, zero below R's diagonal.
template <typename T>
__global__ void extract_band(int n, int b, int np, const T* A, long lda, T* Bd, long ldb) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)ldb * n) return;
    const int rho = (int)(idx % ldb), j = (int)(idx / ldb);
    const int i = j + rho;
    T val = zero_of<T>();
    if (rho <= b && i < n) {
        const int p = j / b, cp = p * b;
        val = A[IDX(i, j, lda)];
        if (p < np && i >= cp + b && (i - cp - b) > (j - cp)) val = zero_of<T>();
        if (rho == 0) val = from_real<T>(realp(val));
    }
    Bd[IDX(rho, j, ldb)] = val;
}

struct Carve {
    char* p;
    size_t off = 0;
    template <typename U>
    U* take(size_t elems) {
        off = (off + 255) & ~size_t(255);
        U* r = reinterpret_cast<U*>(p ? p + off : nullptr);
        off += elems * sizeof(U);
        return r;
    }
};

// Split of the inner dimension (m) of Y = A22 V (m x b output): enough
// splits for about 512 output-tile workgroups of 128 rows, each split at
// least 512 rows long.
constexpr int SKY_MAX = 16;
int sk_y(int m) {
    const int tm = (m + 127) / 128;
    return std::max(1, std::min({SKY_MAX, (512 + tm - 1) / tm, m / 512}));
}
// The b x b products over the panel's m rows (V^H V, V^H W) are a single
// output tile: their inner dimension is split into chunks of about 128 rows
// so that they fill the device (partials added in a fixed order).
constexpr int SKS_MAX = 256;
int sk_small(int m) { return std::max(1, std::min(SKS_MAX, (m + 127) / 128)); }

int count_panels(int n, int b) {
    int np = 0;
    while (n - np * b - b >= 2) ++np;
    return np;
}

template <typename T>
struct He2hbWs {
    T *Y, *skY, *LR, *G, *M1, *M2, *skS, *partialT;
    double* partialD;
    PanelScratch<T>* ps;
};

template <typename T>
size_t carve_ws(char* base, int n, int b, He2hbWs<T>* w) {
    Carve c{base};
    const size_t nb = (size_t)n * b;
    He2hbWs<T> t;
    t.Y = c.take<T>(nb);
    t.skY = c.take<T>(SKY_MAX * nb);
    t.LR = c.take<T>(3 * nb);
    t.G = c.take<T>((size_t)b * b);
    t.M1 = c.take<T>((size_t)b * b);
    t.M2 = c.take<T>((size_t)b * b);
    t.skS = c.take<T>((size_t)SKS_MAX * b * b);
    const size_t nwg = (size_t)(n + PT - 1) / PT + 1;
    t.partialT = c.take<T>(2 * nwg * (MAXB + 1));
    t.partialD = c.take<double>(nwg);
    t.ps = c.take<PanelScratch<T>>(1);
    if (w) *w = t;
    return c.off;
}

}  // namespace

template <typename T>
size_t he2hb_ws_elems(int n, int b) {
    return (carve_ws<T>(nullptr, n, b, nullptr) + sizeof(T) - 1) / sizeof(T);
}

template <typename T>
int he2hb(const StageCtx& c, int n, T* A, long lda, BandRefl<T>& R, T* Bd, long ldb, T* work) {
    hipStream_t st = c.st;
    const int b = R.b;
    const int np = count_panels(n, b);
    R.n = n;
    R.np = np;
    He2hbWs<T> w;
    carve_ws<T>(reinterpret_cast<char*>(work), n, b, &w);
    const T one = from_real<T>(1.0), mone = from_real<T>(-1.0), zero = zero_of<T>();
    const T mhalf = from_real<T>(-0.5);
    int rc;
    const bool look = c.aux != nullptr && c.fork != nullptr && c.join != nullptr;
    bool pending = false;
    unsigned bar_base = 0;  // grid-barrier count of the persistent panel kernel
    // the panel scratch counter must start at zero
    if ((rc = set_zero<T>(st, (int)((sizeof(PanelScratch<T>) + sizeof(T) - 1) / sizeof(T)), 1, (T*)w.ps, 1)))
        return rc;
    for (int p = 0; p < np; ++p) {
        const int c0 = p * b;
        const int m = n - c0 - b;
        const int nref = min(b, m - 1);
        T* P = A + IDX(c0 + b, c0, lda);
        T* Vp = R.V + R.voff(p);
        T* Tp = R.Tf + (size_t)p * b * b;
        const int gall = (m + PT - 1) / PT;
        if (gall <= PANEL_MAX_WG && c.hang && c.panel_persist) {
            // one persistent launch for the panel (writes all m x b entries of Vp)
            double fl = 0.0;
            for (int s = 0; s <= nref; ++s) fl += (double)(m - (s > 0 ? s - 1 : 0)) * std::max(0, b - s);
            KProbe probe(st, GEVD_K_PANEL, (is_cplx<T>::value ? 16.0 : 4.0) * fl);
            hipLaunchKernelGGL(panel_cols<T>, dim3(gall), dim3(PCT), 0, st, P, lda, m, b, nref, Vp, w.ps,
                               w.partialT, bar_base, c.hang);
            GEVD_LAUNCH_CHECK();
            bar_base += (unsigned)nref * (unsigned)gall;
        } else {
            if ((rc = set_zero<T>(st, m, b, Vp, m))) return rc;
            for (int s = 0; s <= nref; ++s) {
                KProbe probe(st, GEVD_K_PANEL,
                             (is_cplx<T>::value ? 16.0 : 4.0) * (double)(m - (s > 0 ? s - 1 : 0)) *
                                 std::max(0, b - s));
                hipLaunchKernelGGL(panel_col_step<T>, dim3(gall), dim3(PCT), 0, st, P, lda, m, b, s, nref, Vp,
                                   w.ps, w.partialT);
                GEVD_LAUNCH_CHECK();
            }
        }
        // T factor from G = V^H V
        if ((rc = gemm<T>(st, OP_C, OP_N, b, b, m, one, Vp, m, Vp, m, zero, w.G, b, K_FULL, T_ALL, Batch(),
                          sk_small(m), w.skS)))
            return rc;
        {
            KProbe probe(st, GEVD_K_OTHER, 0.0);
            hipLaunchKernelGGL(tfactor_kernel<T>, dim3(1), dim3(TFT), 0, st, b, (const T*)w.G,
                               (const PanelScratch<T>*)w.ps, Tp);
        }
        GEVD_LAUNCH_CHECK();
        // two-sided update of A22 = A[c0+b:, c0+b:]
        T* A22 = A + IDX(c0 + b, c0 + b, lda);
        T* Wb = w.LR;                  // columns [0, b): W
        T* Vb = w.LR + (size_t)m * b;  // columns [b, 2b): V
        T* W2 = w.LR + (size_t)2 * m * b;  // columns [2b, 3b): W again
        if (pending) {  // the previous trailing update on the second stream
            GEVD_HIP(hipStreamWaitEvent(st, c.join, 0));
            pending = false;
        }
        // A22 is kept only in its lower triangle: Y = A22 V reads it as Hermitian
        if ((rc = gemm<T>(st, OP_N, OP_N, m, b, m, one, A22, lda, Vp, m, zero, w.Y, m, K_A_HERM_LOWER, T_ALL,
                          Batch(), sk_y(m), w.skY)))
            return rc;
        if ((rc = gemm<T>(st, OP_N, OP_N, m, b, b, one, w.Y, m, Tp, b, zero, Wb, m, K_B_UPPER))) return rc;  // X
        if ((rc = gemm<T>(st, OP_C, OP_N, b, b, m, one, Vp, m, Wb, m, zero, w.M1, b, K_FULL, T_ALL, Batch(),
                          sk_small(m), w.skS)))
            return rc;
        if ((rc = gemm<T>(st, OP_C, OP_N, b, b, b, one, Tp, b, w.M1, b, zero, w.M2, b, K_A_LOWER))) return rc;
        if ((rc = gemm<T>(st, OP_N, OP_N, m, b, b, mhalf, Vp, m, w.M2, b, one, Wb, m))) return rc;  // W
        if ((rc = copy_matrix<T>(st, m, b, Wb, m, W2, m))) return rc;
        if ((rc = copy_matrix<T>(st, m, b, Vp, m, Vb, m))) return rc;
        // lower tiles of A22 -= W V^H + V W^H (the upper triangle is never read
        // again).  With a second stream: the next panel's b columns first,
        // then the rest on the second stream while the next panel is
        // factored; the next product with A22 waits for it.
        if (!look || m <= b) {
            if ((rc = gemm<T>(st, OP_N, OP_C, m, m, 2 * b, mone, w.LR, m, Vb, m, one, A22, lda, K_FULL,
                              T_LOWER_TILES)))
                return rc;
        } else {
            if ((rc = gemm<T>(st, OP_N, OP_C, m, b, 2 * b, mone, w.LR, m, Vb, m, one, A22, lda))) return rc;
            GEVD_HIP(hipEventRecord(c.fork, st));
            GEVD_HIP(hipStreamWaitEvent(c.aux, c.fork, 0));
            if ((rc = gemm<T>(c.aux, OP_N, OP_C, m - b, m - b, 2 * b, mone, w.LR + b, m, Vb + b, m, one,
                              A22 + IDX(b, b, lda), lda, K_FULL, T_LOWER_TILES)))
                return rc;
            GEVD_HIP(hipEventRecord(c.join, c.aux));
            pending = true;
        }
    }
    if (pending) GEVD_HIP(hipStreamWaitEvent(st, c.join, 0));
    const long long tot = (long long)ldb * n;
    hipLaunchKernelGGL(extract_band<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, b, np, (const T*)A,
                       lda, Bd, ldb);
    GEVD_LAUNCH_CHECK();
    return 0;
}

#define INST(T)                                                                                  \
    template size_t he2hb_ws_elems<T>(int, int);                                                 \
    template int he2hb<T>(const StageCtx&, int, T*, long, BandRefl<T>&, T*, long, T*);
INST(double)
INST(zdouble)
#undef INST

}  // namespace gevd
