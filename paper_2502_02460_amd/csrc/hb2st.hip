// Second stage of the two-stage reduction: Hermitian band (half-bandwidth b)
// -> real symmetric tridiagonal T = Q2^H B Q2 by bulge chasing, and the
// back-transformation through Q2.
//
// Sweep s removes column s below its first subdiagonal with a length-b
// reflector and chases the resulting bulge down the band in blocks of b rows:
// task (s, 0) reflects column s and updates the diagonal block two-sidedly;
// task (s, t>0) applies the previous reflector from the right to the block
// below, reflects its first column, applies that reflector from the left to
// the rest of the block and two-sidedly to the next diagonal block.  Every
// reflector makes its leading entry real, so T is real without a separate
// phase step.  Task (s+1, t) may start once task (s, t+1) has finished;
// one persistent kernel runs the sweeps concurrently, each workgroup taking
// the next sweep in order and waiting on its predecessor's progress counter
// (the predecessor was taken earlier by a running workgroup, so every wait
// ends; a spin bound turns a broken invariant into an error flag instead of
// a hang).
//
// Band storage: lower band with ldw >= 2b rows, B[i, j] at Bw[(i-j) + j*ldw];
// the bulge reaches 2b-1 below the diagonal.
#include "stages.hpp"

namespace gevd {
namespace {

constexpr int HT = 256;
constexpr int MAXB = 64;
constexpr long long SPIN_LIMIT = 200000000LL;

__device__ inline int ntasks(int n, int b, int sw) { return (n - 1 - sw + b - 1) / b; }

template <typename T>
__device__ inline void dot_rows(const T (*M)[MAXB + 1], const T* x, T* y, T (*red)[MAXB], int L, int C) {
    // y[i] = sum_j M[i][j] x[j], i < L, j < C; 4 waves split the columns.
    const int tid = threadIdx.x, i = tid % MAXB, seg = tid / MAXB;
    T acc = zero_of<T>();
    if (i < L)
        for (int j = seg * 16; j < min(C, seg * 16 + 16); ++j) acc += M[i][j] * x[j];
    red[seg][i] = acc;
    __syncthreads();
    if (tid < L) y[tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    __syncthreads();
}

template <typename T>
__device__ inline void dot_cols(const T (*M)[MAXB + 1], const T* x, T* z, T (*red)[MAXB], int L, int C) {
    // z[j] = sum_i conj(x[i]) M[i][j], j < C, i < L.
    const int tid = threadIdx.x, j = tid % MAXB, seg = tid / MAXB;
    T acc = zero_of<T>();
    if (j < C)
        for (int i = seg * 16; i < min(L, seg * 16 + 16); ++i) acc += conjg(x[i]) * M[i][j];
    red[seg][j] = acc;
    __syncthreads();
    if (tid < C) z[tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    __syncthreads();
}

// Householder reflector for x[0..L-1] (in LDS, overwritten by v with
// v[0] = 1): H^H x = beta e1, beta real.  Wave 0 computes; the result is
// broadcast through sc[] = {tau, beta}.
template <typename T>
__device__ inline void reflect(T* x, int L, T* sc) {
    const int tid = threadIdx.x;
    if (tid < WAVE) {
        double a2 = (tid >= 1 && tid < L) ? abs2(x[tid]) : 0.0;
        a2 = wave_sum(a2);
        if (tid == 0) {
            const T alpha = x[0];
            const double ar = realp(alpha), ai = imagp(alpha);
            if (a2 == 0.0 && ai == 0.0) {
                sc[0] = zero_of<T>();
                sc[1] = from_real<T>(ar);
                sc[2] = zero_of<T>();
            } else {
                const double nrm = sqrt(ar * ar + ai * ai + a2);
                const double bt = ar >= 0.0 ? -nrm : nrm;
                sc[0] = div_r(from_real<T>(bt) - alpha, bt);
                sc[1] = from_real<T>(bt);
                sc[2] = div_s(from_real<T>(1.0), alpha - from_real<T>(bt));
            }
        }
    }
    __syncthreads();
    if (tid >= 1 && tid < L) x[tid] = x[tid] * sc[2];
    if (tid == 0) x[0] = from_real<T>(1.0);
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(HT) void hb2st_kernel(int n, int b, T* Bw, long ldw, T* V2, T* tau2, int nsw,
                                                   int* progress, int* counter, int* hang) {
    __shared__ T E[MAXB][MAXB + 1];
    __shared__ T D[MAXB][MAXB + 1];
    __shared__ T v[MAXB], vp[MAXB], y[MAXB], red[4][MAXB];
    __shared__ T sc[4];
    __shared__ T ptau;
    __shared__ int sw_s, stop;
    const int tid = threadIdx.x;

    for (;;) {
        if (tid == 0) {
            sw_s = atomicAdd(counter, 1);
            stop = 0;
        }
        __syncthreads();
        const int sw = sw_s;
        if (sw >= nsw) return;
        const int nt = ntasks(n, b, sw);
        for (int t = 0; t < nt; ++t) {
            if (sw > 0) {
                if (tid == 0) {
                    const int need = min(t + 2, ntasks(n, b, sw - 1));
                    long long spins = 0;
                    while (__hip_atomic_load(&progress[sw - 1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        if (++spins > SPIN_LIMIT ||
                            __hip_atomic_load(hang, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                            atomicOr(hang, 1);
                            stop = 1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
                __syncthreads();
                if (stop) return;
                __threadfence();  // acquire for every wave before reading the band
            }
            const int r0 = sw + 1 + t * b;
            const int L = min(b, n - r0);
            if (t == 0) {
                // column sw, rows r0 .. r0+L-1 (band rows 1 .. L)
                if (tid < L) v[tid] = Bw[IDX(1 + tid, sw, ldw)];
                __syncthreads();
                reflect<T>(v, L, sc);
                if (tid < L) Bw[IDX(1 + tid, sw, ldw)] = (tid == 0) ? sc[1] : zero_of<T>();
            } else {
                const int pr0 = r0 - b;  // previous block (always b rows)
                for (int e = tid; e < L * b; e += HT) {
                    const int i = e % L, j = e / L;
                    E[i][j] = Bw[IDX(b + i - j, pr0 + j, ldw)];
                }
                __syncthreads();
                // E <- E (I - ptau vp vp^H)
                dot_rows<T>(E, vp, y, red, L, b);
                const T pt = ptau;
                for (int e = tid; e < L * b; e += HT) {
                    const int i = e % L, j = e / L;
                    E[i][j] -= pt * y[i] * conjg(vp[j]);
                }
                __syncthreads();
                if (L >= 2) {
                    if (tid < L) v[tid] = E[tid][0];
                    __syncthreads();
                    reflect<T>(v, L, sc);
                    // E[:, 1:] <- (I - tau v v^H)^H E[:, 1:]
                    dot_cols<T>(E, v, y, red, L, b);
                    const T ctau = conjg(sc[0]);
                    for (int e = tid; e < L * b; e += HT) {
                        const int i = e % L, j = e / L;
                        if (j >= 1) E[i][j] -= ctau * v[i] * y[j];
                        else E[i][0] = (i == 0) ? sc[1] : zero_of<T>();
                    }
                    __syncthreads();
                } else {
                    if (tid == 0) {
                        v[0] = from_real<T>(1.0);
                        sc[0] = zero_of<T>();
                    }
                    __syncthreads();
                }
                for (int e = tid; e < L * b; e += HT) {
                    const int i = e % L, j = e / L;
                    Bw[IDX(b + i - j, pr0 + j, ldw)] = E[i][j];
                }
            }
            // two-sided update of the diagonal block rows/cols r0 .. r0+L-1
            const T tau = sc[0];
            for (int e = tid; e < L * L; e += HT) {
                const int i = e % L, j = e / L;
                if (i >= j) {
                    const T x = Bw[IDX(i - j, r0 + j, ldw)];
                    D[i][j] = x;
                    D[j][i] = conjg(x);
                }
            }
            __syncthreads();
            if (!is_zero(tau)) {
                dot_rows<T>(D, v, y, red, L, L);  // y = D v
                if (tid < WAVE) {
                    T yi = (tid < L) ? tau * y[tid] : zero_of<T>();
                    T s = (tid < L) ? conjg(yi) * v[tid] : zero_of<T>();
                    s = wave_sum(s);
                    const T coef = from_real<T>(-0.5) * tau * s;  // -1/2 tau (y^H v)
                    if (tid < L) y[tid] = yi + coef * v[tid];     // w
                }
                __syncthreads();
                for (int e = tid; e < L * L; e += HT) {
                    const int i = e % L, j = e / L;
                    if (i >= j) {
                        T x = D[i][j] - v[i] * conjg(y[j]) - y[i] * conjg(v[j]);
                        if (i == j) x = from_real<T>(realp(x));
                        Bw[IDX(i - j, r0 + j, ldw)] = x;
                    }
                }
            }
            // keep the reflector for the back-transformation and the next task
            const size_t slot = (size_t)t * nsw + sw;
            if (tid < b) V2[slot * b + tid] = (tid < L) ? v[tid] : zero_of<T>();
            if (tid == 0) tau2[slot] = tau;
            __syncthreads();
            if (tid < MAXB) vp[tid] = (tid < L) ? v[tid] : zero_of<T>();
            if (tid == 0) ptau = tau;
            __threadfence();  // every wave's band stores visible device-wide
            __syncthreads();
            if (tid == 0)
                __hip_atomic_store(&progress[sw], t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <typename T>
__global__ void extract_tridiag(int n, const T* Bw, long ldw, double* d, double* e) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    d[j] = realp(Bw[IDX(0, j, ldw)]);
    if (j + 1 < n) e[j] = realp(Bw[IDX(1, j, ldw)]);
}

// ---------------------------------------------------------------------------
// Back-transformation Z <- Q2 Z.  Q2 = prod over sweeps (ascending) of prod
// over blocks (ascending) of H(s, t).  Reflectors of one sweep touch disjoint
// rows; H(s', t-1) and H(s', t) with s' > s must precede H(s, t).  Sweeps are
// grouped in blocks of NBS <= b; blocks are applied last-first, within a
// block the groups G(S, t) in t order, inside a group the sweeps last-first.
// A workgroup owns CT columns of Z and keeps the rows of the current group
// in an LDS window indexed modulo 2b (a group spans at most 2b-1 rows and
// consecutive groups slide by b).  Each wave owns CT/4 columns, so a
// reflector costs only wave-level reductions, no workgroup barrier.
// ---------------------------------------------------------------------------
template <typename T, int CT>
__global__ __launch_bounds__(256) void back_chase_kernel(int n, int b, int nsw, int nbs, const T* V2, const T* tau2,
                                                         int nev, T* Z, long ldz) {
    __shared__ T win[2 * MAXB][CT];
    const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    const int c0 = blockIdx.x * CT;
    const int ncol = min(CT, nev - c0);
    const int W2 = 2 * b;
    constexpr int CPW = CT / 4;  // columns per wave
    const int nblk = (nsw + nbs - 1) / nbs;

    auto load_rows = [&](int ra, int rb) {  // rows [ra, rb) of Z into the window
        const int nr = rb - ra;
        for (int e = tid; e < nr * CT; e += 256) {
            const int r = ra + e % nr, c = e / nr;
            win[r % W2][c] = (c < ncol) ? Z[IDX(r, c0 + c, ldz)] : zero_of<T>();
        }
    };
    auto store_rows = [&](int ra, int rb) {
        const int nr = rb - ra;
        for (int e = tid; e < nr * CT; e += 256) {
            const int r = ra + e % nr, c = e / nr;
            if (c < ncol) Z[IDX(r, c0 + c, ldz)] = win[r % W2][c];
        }
    };

    for (int S = nblk - 1; S >= 0; --S) {
        const int s0 = S * nbs, s1 = min(nsw, s0 + nbs);
        int lo = -1, hi = -1;  // rows currently held in the window
        for (int t = 0;; ++t) {
            const int wr0 = s0 + 1 + t * b;
            if (wr0 >= n) break;
            const int wr1 = min(n, (s1 - 1) + 1 + t * b + b);
            // write back rows leaving the window, load rows entering it
            if (hi > lo) store_rows(lo, min(hi, wr0));
            const int la = (hi > wr0) ? hi : wr0;
            __syncthreads();
            if (wr1 > la) load_rows(la, wr1);
            lo = wr0;
            hi = wr1;
            __syncthreads();
            for (int s = s1 - 1; s >= s0; --s) {
                const int r0 = s + 1 + t * b;
                if (r0 >= n) continue;
                const int L = min(b, n - r0);
                const size_t slot = (size_t)t * nsw + s;
                const T tau = tau2[slot];
                if (is_zero(tau)) continue;
                const T vi = (lane < L) ? V2[slot * b + lane] : zero_of<T>();
                const T cvi = conjg(vi);
#pragma unroll
                for (int q = 0; q < CPW; ++q) {
                    const int c = wv * CPW + q;
                    T z = (lane < L) ? win[(r0 + lane) % W2][c] : zero_of<T>();
                    T dot = wave_sum(cvi * z);
                    if (lane < L) win[(r0 + lane) % W2][c] = z - tau * vi * dot;
                }
            }
            __syncthreads();
        }
        if (hi > lo) store_rows(lo, hi);
        __syncthreads();
    }
}

}  // namespace

template <typename T>
int hb2st(const StageCtx& c, int n, T* Bw, long ldw, ChaseRefl<T>& R, double* d, double* e, int* sync_area) {
    hipStream_t st = c.st;
    const int b = R.b;
    R.n = n;
    R.nsw = n - 1;
    R.tmax = n > 1 ? (n - 1 + b - 1) / b : 0;
    int rc;
    if (R.nsw > 0) {
        // progress[nsw] and the sweep counter start at zero
        if ((rc = set_zero<double>(st, (R.nsw + 2 + 1) / 2 + 1, 1, reinterpret_cast<double*>(sync_area), 1)))
            return rc;
        int* progress = sync_area;
        int* counter = sync_area + R.nsw + 1;
        const int grid = std::min(R.nsw, 240);
        hipLaunchKernelGGL(hb2st_kernel<T>, dim3(grid), dim3(HT), 0, st, n, b, Bw, ldw, R.V2, R.tau2, R.nsw, progress,
                           counter, c.hang);
        GEVD_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(extract_tridiag<T>, dim3((n + 255) / 256), dim3(256), 0, st, n, (const T*)Bw, ldw, d, e);
    GEVD_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int back_chase(const StageCtx& c, const ChaseRefl<T>& R, int nev, T* Z, long ldz) {
    if (R.nsw <= 0 || nev <= 0) return 0;
    constexpr int CT = is_cplx<T>::value ? 8 : 16;
    const int grid = (nev + CT - 1) / CT;
    const int nbs = R.b;  // sweeps per block (<= b keeps a group within 2b-1 rows)
    hipLaunchKernelGGL((back_chase_kernel<T, CT>), dim3(grid), dim3(256), 0, c.st, R.n, R.b, R.nsw, nbs,
                       (const T*)R.V2, (const T*)R.tau2, nev, Z, ldz);
    GEVD_LAUNCH_CHECK();
    return 0;
}

#define INST(T)                                                                              \
    template int hb2st<T>(const StageCtx&, int, T*, long, ChaseRefl<T>&, double*, double*, int*); \
    template int back_chase<T>(const StageCtx&, const ChaseRefl<T>&, int, T*, long);
INST(double)
INST(zdouble)
#undef INST

}  // namespace gevd
