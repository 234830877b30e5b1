// Many small independent generalized problems (n <= 512) in one persistent
// launch: the trivially parallel k-point / spin-channel problems of the
// paper's introduction and its usability section, when each one is far too
// small to fill the GPU.  Each workgroup takes the next problem from an
// atomic queue and runs the whole solve of the paper's section on the
// generalized eigenproblem (its Eq. (2), by Cholesky reduction) on it:
//   1. Cholesky S = U^H U (blocked left-looking, L = U^H kept too),
//   2. A = U^{-H} H U^{-1} by two row-wise triangular solves,
//   3. one-stage Householder tridiagonalisation (for small orders the
//      one-stage method is the cheaper one, as the paper notes),
//   4. all eigenvalues of the tridiagonal T by bisection and only the
//      wanted eigenvectors by twisted factorisations (implicit QL with every
//      eigenvector as the fallback when a vector fails its checks),
//   5. back-transformation of the wanted vectors through the reflectors and
//      U^{-1}.
// Work is split so that global accesses are coalesced and the workgroup
// rarely needs a barrier: triangular solves are one matrix row per lane;
// the tridiagonalisation fuses the rank-2 update of one step with the
// matrix-vector product of the next (one read+write pass per step); an
// eigenvalue's bisection and an eigenvector's recurrences run on one lane;
// QL rotations of a sweep are formed by one lane and applied by all; each
// wanted eigenvector is back-transformed by one wave with its rows in
// registers.
#include "kernels.hpp"
#include "small.hpp"

namespace gevd {
namespace {

// Phase hooks for an external profiling build; empty here.
#ifndef SMALL_MARK
#define SMALL_MARK_INIT() ((void)0)
#define SMALL_MARK(phase) ((void)0)
#endif

constexpr double SEPS = 2.220446049250313e-16;
constexpr int RB = 8;                    // register block of the Cholesky and substitutions
constexpr int QMAX = SMALL_MAX / WAVE;   // rows per lane when a wave owns a column
constexpr int ZC = 8;                    // entries per chunk of a row sweep (loads in flight)

template <typename T>
struct Lds {
    T *v, *w, *v2, *y2, *tau;
    double *d, *e, *rc, *rs;
    int* perm;
};

template <typename T>
__host__ __device__ inline size_t lds_layout(int nmax, Lds<T>* L, char* base) {
    size_t off = 0;
    T* t[5];
    for (int i = 0; i < 5; ++i) {
        t[i] = reinterpret_cast<T*>(base ? base + off : nullptr);
        off += (sizeof(T) * nmax + 15) & ~size_t(15);
    }
    double* d[4];
    for (int i = 0; i < 4; ++i) {
        d[i] = reinterpret_cast<double*>(base ? base + off : nullptr);
        off += (sizeof(double) * nmax + 15) & ~size_t(15);
    }
    int* p = reinterpret_cast<int*>(base ? base + off : nullptr);
    off += (sizeof(int) * nmax + 15) & ~size_t(15);
    if (L) *L = Lds<T>{t[0], t[1], t[2], t[3], t[4], d[0], d[1], d[2], d[3], p};
    return off;
}

__device__ inline double shfl_s(double v, int src) { return __shfl(v, src, WAVE); }
__device__ inline zdouble shfl_s(zdouble v, int src) { return {__shfl(v.x, src, WAVE), __shfl(v.y, src, WAVE)}; }

// Sum of x(i), 0 <= i < len, in an order that does not depend on the
// workgroup size: 64-element chunks reduced by the wave butterfly (the same
// tree in every lane), chunk sums added in chunk order.  A problem's result
// is then the same whatever launch shape runs it.  chunk holds
// SMALL_MAX / 64 entries.
template <int NT, typename U, typename F>
__device__ U chunked_sum(int len, F x, U* chunk) {
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    const int nch = (len + WAVE - 1) / WAVE;
    __syncthreads();
    for (int c = wv; c < nch; c += NT / WAVE) {
        const int i = c * WAVE + lane;
        U v = i < len ? x(i) : zero_of<U>();
        v = wave_sum(v);
        if (lane == 0) chunk[c] = v;
    }
    __syncthreads();
    U t = zero_of<U>();
    for (int c = 0; c < nch; ++c) t += chunk[c];
    return t;
}

// ---------------------------------------------------------------------------
// 1. Cholesky.  Reads the upper triangle of S; writes L = U^H into the lower
// triangle and U into the upper one (diagonal shared).  Column blocks of RB:
// the rows of a block's diagonal part are accumulated by RB lanes and
// factored by one lane in LDS; every row below is one lane, its RB entries in
// registers.  Returns 0 or the 1-based order of the first non-positive minor.
// ---------------------------------------------------------------------------
template <typename T, int NT>
__device__ int chol_small(T* S, long lds, int n, T (*dblk)[RB + 1], int* ctl) {
    const int tid = threadIdx.x;
    for (int J = 0; J < n; J += RB) {
        const int nb = min(RB, n - J);
        if (tid < nb) {
            const int i = J + tid;
            T acc[RB];
#pragma unroll
            for (int s = 0; s < RB; ++s) {
                const int c = J + s;
                acc[s] = s < nb ? (i <= c ? S[IDX(i, c, lds)] : conjg(S[IDX(c, i, lds)])) : zero_of<T>();
            }
            for (int l = 0; l < J; ++l) {
                const T a = S[IDX(i, l, lds)];
#pragma unroll
                for (int s = 0; s < RB; ++s)
                    if (s < nb) acc[s] -= a * conjg(S[IDX(J + s, l, lds)]);
            }
#pragma unroll
            for (int s = 0; s < RB; ++s) dblk[tid][s] = acc[s];
        }
        __syncthreads();
        if (tid == 0) {
            int bad = 0;
            for (int t = 0; t < nb; ++t) {
                double dt = realp(dblk[t][t]);
                for (int s = 0; s < t; ++s) dt -= abs2(dblk[t][s]);
                if (!(dt > 0.0) || !isfinite(dt)) {
                    bad = J + t + 1;
                    break;
                }
                const double lt = sqrt(dt);
                dblk[t][t] = from_real<T>(lt);
                for (int r = t + 1; r < nb; ++r) {
                    T x = dblk[r][t];
                    for (int s = 0; s < t; ++s) x -= dblk[r][s] * conjg(dblk[t][s]);
                    dblk[r][t] = div_r(x, lt);
                }
            }
            ctl[0] = bad;
        }
        __syncthreads();
        if (ctl[0]) return ctl[0];
        if (tid < nb * nb) {
            const int r = tid % nb, s = tid / nb;
            if (r >= s) {
                const T x = dblk[r][s];
                S[IDX(J + r, J + s, lds)] = x;
                S[IDX(J + s, J + r, lds)] = conjg(x);
            }
        }
        for (int i = J + nb + tid; i < n; i += NT) {
            T acc[RB];
#pragma unroll
            for (int s = 0; s < RB; ++s) acc[s] = s < nb ? conjg(S[IDX(J + s, i, lds)]) : zero_of<T>();
            for (int l = 0; l < J; ++l) {
                const T a = S[IDX(i, l, lds)];
#pragma unroll
                for (int s = 0; s < RB; ++s)
                    if (s < nb) acc[s] -= a * conjg(S[IDX(J + s, l, lds)]);
            }
#pragma unroll
            for (int s = 0; s < RB; ++s) {
                if (s < nb) {
                    T x = acc[s];
                    for (int q = 0; q < s; ++q) x -= acc[q] * conjg(dblk[s][q]);
                    acc[s] = div_r(x, realp(dblk[s][s]));
                }
            }
#pragma unroll
            for (int s = 0; s < RB; ++s) {
                if (s < nb) {
                    S[IDX(i, J + s, lds)] = acc[s];
                    S[IDX(J + s, i, lds)] = conjg(acc[s]);
                }
            }
        }
        __syncthreads();
    }
    return 0;
}

// Y U = B row by row, in place (B n x n); U upper from S, read through
// U[l, c] = conj(L[c, l]) so that the RB entries a block needs are adjacent.
template <typename T, int NT>
__device__ void row_solve(T* B, long ldb, const T* S, long lds, int n) {
    for (int r = threadIdx.x; r < n; r += NT) {
        for (int J = 0; J < n; J += RB) {
            const int nb = min(RB, n - J);
            T acc[RB];
#pragma unroll
            for (int s = 0; s < RB; ++s) acc[s] = s < nb ? B[IDX(r, J + s, ldb)] : zero_of<T>();
            for (int l = 0; l < J; ++l) {
                const T x = B[IDX(r, l, ldb)];
#pragma unroll
                for (int s = 0; s < RB; ++s)
                    if (s < nb) acc[s] -= x * conjg(S[IDX(J + s, l, lds)]);
            }
#pragma unroll
            for (int s = 0; s < RB; ++s) {
                if (s < nb) {
                    T x = acc[s];
                    for (int q = 0; q < s; ++q) x -= acc[q] * conjg(S[IDX(J + s, J + q, lds)]);
                    acc[s] = div_r(x, realp(S[IDX(J + s, J + s, lds)]));
                }
            }
#pragma unroll
            for (int s = 0; s < RB; ++s)
                if (s < nb) B[IDX(r, J + s, ldb)] = acc[s];
        }
    }
}

// ---------------------------------------------------------------------------
// 3. Lower Householder tridiagonalisation of the full Hermitian A.  Step j
// builds H_j = I - tau v v^H (v[0] = 1, rows j+1..) with H_j^H x = beta e_1
// for x = A[j+1:, j], beta real; the trailing block then becomes
// A - v w^H - w v^H with y = tau A v and w = y - (tau/2)(y^H v) v.  The
// update of step j is applied in the same pass over the trailing block that
// forms y for step j+1 (column j+1 is brought up to date first, since the
// next reflector is built from it).  v below its unit entry stays in column
// j of A; d, e (= beta) and tau stay in LDS.
// ---------------------------------------------------------------------------
template <typename T, int NT>
__device__ void tridiag_small(T* A, long lda, int n, Lds<T>& L, T* red, double* redd) {
    const int tid = threadIdx.x;
    T *v = L.v, *w = L.w, *v2 = L.v2, *y2 = L.y2;
    bool pending = false;
    for (int j = 0; j + 1 < n; ++j) {
        const int o = j + 1, len = n - o;
        if (pending) {  // previous reflector lives on rows j.., coordinate i - j
            const T vj = v[0], wj = w[0];
            for (int i = j + tid; i < n; i += NT) A[IDX(i, j, lda)] -= v[i - j] * conjg(wj) + w[i - j] * conjg(vj);
            __syncthreads();
        }
        const double part =
            chunked_sum<NT, double>(len, [&](int i) { return i > 0 ? abs2(A[IDX(o + i, j, lda)]) : 0.0; }, redd);
        if (tid == 0) {
            const T alpha = A[IDX(o, j, lda)];
            const double ar = realp(alpha), ai = imagp(alpha);
            T tau, scale;
            double beta;
            if (part == 0.0 && ai == 0.0) {
                tau = zero_of<T>();
                scale = zero_of<T>();
                beta = ar;
            } else {
                const double nrm = sqrt(ar * ar + ai * ai + part);
                beta = ar >= 0.0 ? -nrm : nrm;
                tau = div_r(from_real<T>(beta) - alpha, beta);
                scale = div_s(from_real<T>(1.0), alpha - from_real<T>(beta));
            }
            L.tau[j] = tau;
            L.e[j] = beta;
            L.d[j] = realp(A[IDX(j, j, lda)]);
            red[QMAX] = scale;
        }
        __syncthreads();
        const T tau = L.tau[j], scale = red[QMAX];
        for (int i = tid; i < len; i += NT) {
            if (i == 0) {
                v2[0] = from_real<T>(1.0);
            } else {
                const T x = A[IDX(o + i, j, lda)] * scale;
                v2[i] = x;
                A[IDX(o + i, j, lda)] = x;
            }
        }
        __syncthreads();
        const bool live = !is_zero(tau);
        // pending update of rows/cols >= o, and y2 = tau A22 v2
        for (int i = o + tid; i < n; i += NT) {
            T acc = zero_of<T>();
            const T vi = pending ? v[i - j] : zero_of<T>(), wi = pending ? w[i - j] : zero_of<T>();
            for (int c0 = o; c0 < n; c0 += ZC) {  // chunks: loads in flight together
                const int cnt = min(ZC, n - c0);
                T h[ZC];
#pragma unroll
                for (int q = 0; q < ZC; ++q) h[q] = q < cnt ? A[IDX(i, c0 + q, lda)] : zero_of<T>();
#pragma unroll
                for (int q = 0; q < ZC; ++q) {
                    if (q < cnt) {
                        const int c = c0 + q;
                        if (pending) h[q] -= vi * conjg(w[c - j]) + wi * conjg(v[c - j]);
                        if (live) acc += h[q] * v2[c - o];
                    }
                }
                if (pending) {
#pragma unroll
                    for (int q = 0; q < ZC; ++q)
                        if (q < cnt) A[IDX(i, c0 + q, lda)] = h[q];
                }
            }
            y2[i - o] = tau * acc;
        }
        const T yv = chunked_sum<NT, T>(len, [&](int i) { return conjg(y2[i]) * v2[i]; }, red);
        const T coef = from_real<T>(-0.5) * tau * yv;
        for (int i = tid; i < len; i += NT) y2[i] = y2[i] + coef * v2[i];
        __syncthreads();
        T* t = v;
        v = v2;
        v2 = t;
        t = w;
        w = y2;
        y2 = t;
        pending = live;
    }
    if (tid == 0) {
        T ann = A[IDX(n - 1, n - 1, lda)];
        if (pending) ann -= v[0] * conjg(w[0]) + w[0] * conjg(v[0]);
        L.d[n - 1] = realp(ann);
        L.e[n - 1] = 0.0;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// 4. Implicit QL with the shift from the leading 2x2 of the unreduced block
// (the classical tql2 iteration).  The first wave finds the end m of the
// unreduced block with one ballot per 64 entries; its lane 0 then forms the
// rotations of the sweep, a serial recurrence kept short: every d and e a
// step reads is a value the sweep has not yet overwritten, so it is loaded
// one step ahead, and each rotation takes one reciprocal.  All lanes apply
// the sweep to the rows of Z.  Returns false if an eigenvalue took more than
// 30 sweeps.
// ---------------------------------------------------------------------------
__device__ inline double pyth(double f, double g) {
    const double r2 = fma(f, f, g * g);
    return (r2 > 1e-290 && r2 < 1e290) ? sqrt(r2) : hypot(f, g);
}

template <int NT>
__device__ bool ql_small(int n, double* d, double* e, double* rc, double* rs, double* Z, int* ctl) {
    const int tid = threadIdx.x;
    for (long x = tid; x < (long)n * n; x += NT) {
        const int c = (int)(x / n), r = (int)(x - (long)c * n);
        Z[x] = r == c ? 1.0 : 0.0;
    }
    if (tid == 0) ctl[3] = 0;
    __syncthreads();
    for (int l = 0; l < n; ++l) {
        int iters = 0;
        for (;;) {
            if (tid < WAVE) {
                int m = n - 1;
                for (int base = l; base < n - 1; base += WAVE) {
                    const int i = base + tid;
                    const bool split = i >= n - 1 || !(fabs(e[i]) > SEPS * (fabs(d[i]) + fabs(d[i + 1])));
                    const unsigned long long bal = __ballot(split);
                    if (bal) {
                        m = base + __builtin_ctzll(bal);
                        break;
                    }
                }
                if (tid == 0) {
                    ctl[0] = l;
                    ctl[1] = -1;
                    if (m != l) {
                        if (++iters > 30) {
                            ctl[3] = 1;
                        } else {
                            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                            double r = pyth(g, 1.0);
                            g = d[m] - d[l] + e[l] / (g + copysign(r, g));
                            double s = 1.0, c = 1.0, p = 0.0;
                            int lo = l;
                            bool split = false;
                            double ei = e[m - 1], di = d[m - 1], di1 = d[m];
                            for (int i = m - 1; i >= l; --i) {
                                const double en = i > l ? e[i - 1] : 0.0, dn = i > l ? d[i - 1] : 0.0;
                                const double f = s * ei, b = c * ei;
                                r = pyth(f, g);
                                e[i + 1] = r;
                                if (r == 0.0) {
                                    d[i + 1] = di1 - p;
                                    e[m] = 0.0;
                                    lo = i + 1;
                                    split = true;
                                    break;
                                }
                                const double rinv = 1.0 / r;
                                s = f * rinv;
                                c = g * rinv;
                                g = di1 - p;
                                r = (di - g) * s + 2.0 * c * b;
                                p = s * r;
                                d[i + 1] = g + p;
                                g = c * r - b;
                                rc[i] = c;
                                rs[i] = s;
                                ei = en;
                                di1 = di;
                                di = dn;
                            }
                            if (!split) {
                                d[l] -= p;
                                e[l] = g;
                                e[m] = 0.0;
                            }
                            ctl[0] = lo;
                            ctl[1] = m;
                        }
                    }
                }
            }
            SMALL_MARK(8);
            __syncthreads();
            const int lo = ctl[0], m = ctl[1];
            if (m < 0) break;
            // rows of Z, ZC entries per chunk: all loads of a chunk are issued
            // before any of its stores, so they overlap in flight
            for (int k = tid; k < n; k += NT) {
                double carry = Z[IDX(k, m, n)];
                for (int i = m - 1; i >= lo; i -= ZC) {
                    const int cnt = min(ZC, i - lo + 1);
                    double a[ZC];
#pragma unroll
                    for (int q = 0; q < ZC; ++q) a[q] = q < cnt ? Z[IDX(k, i - q, n)] : 0.0;
#pragma unroll
                    for (int q = 0; q < ZC; ++q) {
                        if (q < cnt) {
                            const double c = rc[i - q], sn = rs[i - q];
                            const double up = sn * a[q] + c * carry;
                            carry = c * a[q] - sn * carry;
                            a[q] = up;  // new entry of column i - q + 1
                        }
                    }
#pragma unroll
                    for (int q = 0; q < ZC; ++q)
                        if (q < cnt) Z[IDX(k, i - q + 1, n)] = a[q];
                }
                Z[IDX(k, lo, n)] = carry;
            }
            __syncthreads();
            SMALL_MARK(9);
        }
        if (ctl[3]) return false;
    }
    return true;
}

// ---------------------------------------------------------------------------
// 4'. The faster route for the tridiagonal problem, tried first.  All n
// eigenvalues by bisection on Sturm counts (one eigenvalue per lane: the
// i-th smallest is where the count of eigenvalues below x passes i), then
// only the wanted eigenvectors, each from a twisted factorisation of
// T - lambda I (one vector per lane): the forward pivots D+ and backward
// pivots D- give gamma_r = D+_r + D-_r - (d_r - lambda) for every twist r,
// and at the r where |gamma_r| is least the vector with z_r = 1 follows
// from the two one-term recurrences z_i = -(e_i / D+_i) z_{i+1} above r and
// z_{i+1} = -(e_i / D-_{i+1}) z_i below it.  Vectors of eigenvalues closer
// than 1e-3 ||T|| to their neighbour (a cluster) are orthogonalised twice
// against the earlier members of their cluster; those of separated
// eigenvalues are orthogonal to working accuracy as computed.  Vectors are
// kept row-major in the Z slot (entry r of vector i at Z[r n + i]) so that
// the lanes' accesses coalesce; each one's pivots are stored in its own
// column and overwritten by the vector.  Returns false (the caller then
// takes the QL route) if a vector loses almost all of its norm to the
// orthogonalisation or its residual ||T z - lambda z|| exceeds 1e-10 ||T||
// (QL's vectors are orthogonal whatever the gaps, at O(n^3) cost).
// ---------------------------------------------------------------------------
__device__ inline int sturm_count(int n, const double* d, const double* e, double x, double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0;
    for (int i = 1; i < n; ++i) {
        q = d[i] - x - e[i - 1] * e[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
    }
    return cnt;
}

template <int NT>
__device__ bool bisect_twist_small(int n, int nev, const double* d, const double* e, double* w, double* dots,
                                   double* Z, double* redd, int* ctl) {
    const int tid = threadIdx.x;
    // Gershgorin interval and the pivot floor (every lane the same values)
    double glo = d[0], ghi = d[0], emax2 = 0.0;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
        glo = fmin(glo, d[i] - r);
        ghi = fmax(ghi, d[i] + r);
        if (i + 1 < n) emax2 = fmax(emax2, e[i] * e[i]);
    }
    const double tnorm = fmax(fabs(glo), fabs(ghi));
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
    glo -= 2.0 * SEPS * tnorm + 2.0 * pivmin;
    ghi += 2.0 * SEPS * tnorm + 2.0 * pivmin;
    for (int idx = tid; idx < n; idx += NT) {
        double lo = glo, hi = ghi;
        for (int it = 0; it < 256; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (!(mid > lo && mid < hi)) break;
            if (sturm_count(n, d, e, mid, pivmin) > idx) hi = mid;
            else lo = mid;
            if (hi - lo <= 2.0 * SEPS * fmax(fabs(lo), fabs(hi)) + pivmin) break;
        }
        w[idx] = 0.5 * (lo + hi);
    }
    __syncthreads();
    if (tid == 0) {  // ascending (bisections of nearly equal eigenvalues may end a rounding apart)
        for (int i = 1; i < n; ++i) w[i] = fmax(w[i], w[i - 1]);
        ctl[2] = 0;
    }
    __syncthreads();
    const double tiny = 1e-3 * SEPS * tnorm + pivmin;
    auto guard = [&](double x) { return fabs(x) < tiny ? (x < 0.0 ? -tiny : tiny) : x; };
    for (int i = tid; i < nev; i += NT) {
        const double lam = w[i];
        double* zc = Z + i;  // entry r at zc[r n]
        // forward pivots D+ into the vector's column
        double dp = d[0] - lam;
        for (int r = 0; r + 1 < n; ++r) {
            dp = guard(dp);
            zc[(size_t)r * n] = dp;
            dp = d[r + 1] - lam - (e[r] / dp) * e[r];
        }
        zc[(size_t)(n - 1) * n] = guard(dp);
        // backward pivots D-, and the twist with the least |gamma|
        double dm = d[n - 1] - lam;
        int tw = n - 1;
        double best = fabs(zc[(size_t)(n - 1) * n]);
        for (int r0 = n - 2; r0 >= 0; r0 -= ZC) {
            double dpr[ZC];
#pragma unroll
            for (int q = 0; q < ZC; ++q) dpr[q] = r0 - q >= 0 ? zc[(size_t)(r0 - q) * n] : 0.0;
#pragma unroll
            for (int q = 0; q < ZC; ++q) {
                const int r = r0 - q;
                if (r >= 0) {
                    dm = guard(dm);
                    dm = d[r] - lam - (e[r] / dm) * e[r];
                    const double g = fabs(dpr[q] + dm - (d[r] - lam));
                    if (g < best) {
                        best = g;
                        tw = r;
                    }
                }
            }
        }
        // the backward multipliers again, below the twist, into rows r + 1 > tw
        dm = d[n - 1] - lam;
        for (int r = n - 2; r >= tw; --r) {
            dm = guard(dm);
            const double u = e[r] / dm;
            zc[(size_t)(r + 1) * n] = u;
            dm = d[r] - lam - u * e[r];
        }
        // the vector, z_tw = 1
        double z = 1.0, nrm2 = 1.0;
        zc[(size_t)tw * n] = 1.0;
        for (int r = tw - 1; r >= 0; --r) {
            z = -(e[r] / zc[(size_t)r * n]) * z;
            zc[(size_t)r * n] = z;
            nrm2 += z * z;
        }
        z = 1.0;
        for (int r = tw; r + 1 < n; ++r) {
            z = -zc[(size_t)(r + 1) * n] * z;
            zc[(size_t)(r + 1) * n] = z;
            nrm2 += z * z;
        }
        const double sc = 1.0 / sqrt(nrm2);
        for (int r = 0; r < n; ++r) zc[(size_t)r * n] *= sc;
    }
    __syncthreads();
    // twice classical Gram-Schmidt inside clusters, one vector at a time
    const double gaptol = 1e-3 * tnorm;
    int c0 = 0;
    for (int i = 1; i < nev; ++i) {
        if (w[i] - w[i - 1] > gaptol) {
            c0 = i;
            continue;
        }
        const int m = i - c0;
        for (int pass = 0; pass < 2; ++pass) {
            for (int j = tid; j < m; j += NT) {
                double acc = 0.0;
                for (int r = 0; r < n; ++r) acc += Z[(size_t)r * n + c0 + j] * Z[(size_t)r * n + i];
                dots[j] = acc;
            }
            __syncthreads();
            for (int r = tid; r < n; r += NT) {
                double x = Z[(size_t)r * n + i];
                for (int j = 0; j < m; ++j) x -= dots[j] * Z[(size_t)r * n + c0 + j];
                Z[(size_t)r * n + i] = x;
            }
            __syncthreads();
        }
        const double nrm2 = chunked_sum<NT, double>(n, [&](int r) {
            const double x = Z[(size_t)r * n + i];
            return x * x;
        }, redd);
        if (!(nrm2 > 1e-4)) {  // (also catches NaN) the vector was almost in its cluster's span
            if (tid == 0) ctl[2] = 1;
        } else {
            const double sc = 1.0 / sqrt(nrm2);
            for (int r = tid; r < n; r += NT) Z[(size_t)r * n + i] *= sc;
        }
        __syncthreads();
    }
    // residual of every vector
    for (int i = tid; i < nev; i += NT) {
        const double lam = w[i];
        double res = 0.0, zm = 0.0, z0 = Z[i];
        for (int r = 0; r < n; ++r) {
            const double zp = r + 1 < n ? Z[(size_t)(r + 1) * n + i] : 0.0;
            const double t = (d[r] - lam) * z0 + (r > 0 ? e[r - 1] * zm : 0.0) + (r + 1 < n ? e[r] * zp : 0.0);
            res = fmax(res, fabs(t));
            zm = z0;
            z0 = zp;
        }
        if (!(res <= 1e-10 * tnorm + pivmin)) atomicOr(&ctl[2], 1);
    }
    __syncthreads();
    return ctl[2] == 0;
}

// ---------------------------------------------------------------------------
// 5. C[:, c] = U^{-1} Q Z[:, perm[c]]: one wave per column, rows in registers
// (row lane + 64 q).  Q = H_0 H_1 ... H_{n-2} is applied right to left; then
// U x = y by back substitution with columns of U (adjacent in memory).
// ---------------------------------------------------------------------------
template <typename T, int NT>
__device__ void back_small(const SmallDesc& D, const T* A, const T* S, const double* Z, const Lds<T>& L,
                           bool rowmajor) {
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    const int n = D.n;
    const long lda = D.ldh, lds = D.lds, ldc = D.ldc;
    T* C = reinterpret_cast<T*>(D.C);
    for (int c = wv; c < D.nev; c += NT / WAVE) {
        T y[QMAX];
        const int zc = min(max(L.perm[c], 0), n - 1);
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
            const int r = lane + q * WAVE;
            y[q] = r < n ? from_real<T>(Z[rowmajor ? (size_t)r * n + zc : IDX(r, zc, n)]) : zero_of<T>();
        }
        for (int j = n - 2; j >= 0; --j) {
            const T tau = L.tau[j];
            if (is_zero(tau)) continue;
            const int o = j + 1;
            T vq[QMAX];
            T dot = zero_of<T>();
#pragma unroll
            for (int q = 0; q < QMAX; ++q) {
                const int r = lane + q * WAVE;
                vq[q] = r == o ? from_real<T>(1.0) : (r > o && r < n ? A[IDX(r, j, lda)] : zero_of<T>());
                dot += conjg(vq[q]) * y[q];
            }
            const T wgt = tau * wave_sum(dot);
#pragma unroll
            for (int q = 0; q < QMAX; ++q) y[q] -= vq[q] * wgt;
        }
        for (int i = n - 1; i >= 0; --i) {
            const int qi = i / WAVE;
            T yi = zero_of<T>();
#pragma unroll
            for (int q = 0; q < QMAX; ++q)
                if (q == qi) yi = y[q];
            const T xi = div_r(shfl_s(yi, i % WAVE), realp(S[IDX(i, i, lds)]));
#pragma unroll
            for (int q = 0; q < QMAX; ++q) {
                const int r = lane + q * WAVE;
                if (r == i) y[q] = xi;
                else if (r < i) y[q] -= S[IDX(r, i, lds)] * xi;
            }
        }
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
            const int r = lane + q * WAVE;
            if (r < n) C[IDX(r, c, ldc)] = y[q];
        }
    }
}

template <typename T, int NT>
__device__ void solve_one(const SmallDesc& D, double* Z, Lds<T>& L, T (*dblk)[RB + 1], T* red, double* redd,
                          int* ctl) {
    const int tid = threadIdx.x;
    const int n = D.n;
    T* H = reinterpret_cast<T*>(D.H);
    T* S = reinterpret_cast<T*>(D.S);
    const long ldh = D.ldh, lds = D.lds;
    SMALL_MARK_INIT();
    const bool factor = !D.factored;
    int bad = 0;
    for (long x = tid; x < (long)n * n; x += NT) {
        const int j = (int)(x / n), i = (int)(x - (long)j * n);
        if (i <= j) {
            const T a = H[IDX(i, j, ldh)];
            if (!isfinite(realp(a)) || !isfinite(imagp(a))) bad = 1;
            if (factor) {
                const T b = S[IDX(i, j, lds)];
                if (!isfinite(realp(b)) || !isfinite(imagp(b))) bad = 1;
            }
        }
    }
    if (__syncthreads_or(bad)) {
        if (tid == 0) *D.info = GEVD_E_NONFINITE;
        return;
    }
    SMALL_MARK(0);
    if (factor) {  // otherwise S keeps U and U^H from an earlier solve (fixed overlap)
        const int minor = chol_small<T, NT>(S, lds, n, dblk, ctl);
        if (minor) {
            if (tid == 0) *D.info = minor;
            return;
        }
    }
    SMALL_MARK(1);
    // full Hermitian H from its upper triangle
    for (long x = tid; x < (long)n * n; x += NT) {
        const int j = (int)(x / n), i = (int)(x - (long)j * n);
        if (i > j) H[IDX(i, j, ldh)] = conjg(H[IDX(j, i, ldh)]);
        else if (i == j) H[IDX(i, i, ldh)] = from_real<T>(realp(H[IDX(i, i, ldh)]));
    }
    __syncthreads();
    row_solve<T, NT>(H, ldh, S, lds, n);  // X = H U^{-1}
    __syncthreads();
    SMALL_MARK(2);
    for (long x = tid; x < (long)n * n; x += NT) {  // X <- X^H
        const int j = (int)(x / n), i = (int)(x - (long)j * n);
        if (i < j) {
            const T a = H[IDX(i, j, ldh)], b = H[IDX(j, i, ldh)];
            H[IDX(i, j, ldh)] = conjg(b);
            H[IDX(j, i, ldh)] = conjg(a);
        } else if (i == j) {
            H[IDX(i, i, ldh)] = conjg(H[IDX(i, i, ldh)]);
        }
    }
    __syncthreads();
    row_solve<T, NT>(H, ldh, S, lds, n);  // X^H U^{-1} = U^{-H} H U^{-1}
    __syncthreads();
    for (long x = tid; x < (long)n * n; x += NT) {  // exact Hermitian part
        const int j = (int)(x / n), i = (int)(x - (long)j * n);
        if (i < j) {
            const T h = from_real<T>(0.5) * (H[IDX(i, j, ldh)] + conjg(H[IDX(j, i, ldh)]));
            H[IDX(i, j, ldh)] = h;
            H[IDX(j, i, ldh)] = conjg(h);
        } else if (i == j) {
            H[IDX(i, i, ldh)] = from_real<T>(realp(H[IDX(i, i, ldh)]));
        }
    }
    __syncthreads();
    SMALL_MARK(3);
    tridiag_small<T, NT>(H, ldh, n, L, red, redd);
    SMALL_MARK(4);
    for (int i = tid; i < n; i += NT) L.perm[i] = i;
    const bool fast = bisect_twist_small<NT>(n, D.nev, L.d, L.e, L.rc, L.rs, Z, redd, ctl);
    if (fast) {
        for (int i = tid; i < n; i += NT) D.eval[i] = L.rc[i];
    } else {
        // implicit QL with every vector (d and e are still T's)
        if (!ql_small<NT>(n, L.d, L.e, L.rc, L.rs, Z, ctl)) {
            if (tid == 0) *D.info = GEVD_E_NOCONV;
            return;
        }
        // ascending order by rank (ties broken by index)
        for (int i = tid; i < n; i += NT) {
            const double di = L.d[i];
            int rank = 0;
            for (int k = 0; k < n; ++k) {
                const double dk = L.d[k];
                rank += (dk < di) || (dk == di && k < i);
            }
            L.perm[rank] = i;
        }
        __syncthreads();
        for (int i = tid; i < n; i += NT) D.eval[i] = L.d[L.perm[i]];
    }
    SMALL_MARK(5);
    __syncthreads();
    SMALL_MARK(6);
    back_small<T, NT>(D, H, S, Z, L, fast);
    __syncthreads();
    SMALL_MARK(7);
    if (tid == 0) *D.info = 0;
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void small_solve_kernel(const SmallDesc* desc, int count, int nmax, double* zws,
                                                         long zslot, int* counter) {
    extern __shared__ __align__(16) char dyn[];
    __shared__ T dblk[RB][RB + 1];
    __shared__ T red[QMAX + 1];  // chunk sums, and the reflector scale in the last slot
    __shared__ double redd[QMAX];
    __shared__ int ctl[4];
    __shared__ int prob;
    Lds<T> L;
    lds_layout<T>(nmax, &L, dyn);
    double* Z = zws + (size_t)blockIdx.x * zslot;
    for (;;) {
        if (threadIdx.x == 0) prob = atomicAdd(counter, 1);
        __syncthreads();
        const int p = prob;
        __syncthreads();
        if (p >= count) return;
        solve_one<T, NT>(desc[p], Z, L, dblk, red, redd, ctl);
        __syncthreads();
    }
}

__global__ void zero_counter(int* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

__device__ inline double unit_hash(unsigned long long seed, unsigned long long idx) {
    unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (idx + 1);  // splitmix64 finaliser
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
}

template <typename T>
__global__ void gen_kernel(int n, int count, T* H, T* S, long stride, unsigned long long seed) {
    const long per = (long)n * n;
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= per * count) return;
    const long p = x / per, e = x - p * per;
    const int j = (int)(e / n), i = (int)(e - (long)j * n);
    const unsigned long long k = 4ull * (unsigned long long)x;
    T h, s;
    if constexpr (is_cplx<T>::value) {
        h = zmake(unit_hash(seed, k), i == j ? 0.0 : unit_hash(seed, k + 1));
        s = zmake(unit_hash(seed, k + 2), i == j ? 0.0 : unit_hash(seed, k + 3));
    } else {
        h = unit_hash(seed, k);
        s = unit_hash(seed, k + 2);
    }
    s = from_real<T>(0.5 / n) * s;
    if (i == j) s = from_real<T>(1.0 + realp(s));
    H[p * stride + e] = h;
    S[p * stride + e] = s;
}

template <typename T, int NT>
const void* kfun() {
    return reinterpret_cast<const void*>(&small_solve_kernel<T, NT>);
}

template <typename T>
const void* kfun_t(int threads) {
    switch (threads) {
        case 64: return kfun<T, 64>();
        case 128: return kfun<T, 128>();
        case 256: return kfun<T, 256>();
        case 512: return kfun<T, 512>();
        case 1024: return kfun<T, 1024>();
        default: return nullptr;
    }
}

template <typename T, int NT>
void go(hipStream_t st, int grid, int nmax, const SmallDesc* desc, int count, double* zws, int* counter) {
    hipLaunchKernelGGL((small_solve_kernel<T, NT>), dim3(grid), dim3(NT), lds_layout<T>(nmax, nullptr, nullptr),
                       st, desc, count, nmax, zws, small_zslot(nmax), counter);
}

template <typename T>
int go_t(hipStream_t st, int threads, int grid, int nmax, const SmallDesc* desc, int count, double* zws,
         int* counter) {
    switch (threads) {
        case 64: go<T, 64>(st, grid, nmax, desc, count, zws, counter); break;
        case 128: go<T, 128>(st, grid, nmax, desc, count, zws, counter); break;
        case 256: go<T, 256>(st, grid, nmax, desc, count, zws, counter); break;
        case 512: go<T, 512>(st, grid, nmax, desc, count, zws, counter); break;
        case 1024: go<T, 1024>(st, grid, nmax, desc, count, zws, counter); break;
        default: return GEVD_E_STATE;
    }
    GEVD_LAUNCH_CHECK();
    return 0;
}

}  // namespace

size_t small_lds_bytes(bool cx, int nmax) {
    return cx ? lds_layout<zdouble>(nmax, nullptr, nullptr) : lds_layout<double>(nmax, nullptr, nullptr);
}

int small_prepare(bool cx, int threads, int nmax) {
    const void* f = cx ? kfun_t<zdouble>(threads) : kfun_t<double>(threads);
    if (!f || nmax < 1 || nmax > SMALL_MAX) return GEVD_E_STATE;
    GEVD_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)small_lds_bytes(cx, nmax)));
    return 0;
}

int small_occupancy(bool cx, int threads, int nmax) {
    const void* f = cx ? kfun_t<zdouble>(threads) : kfun_t<double>(threads);
    if (!f) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, threads, small_lds_bytes(cx, nmax)) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return nb < 1 ? 1 : nb;
}

int small_launch(hipStream_t st, bool cx, int threads, int grid, int nmax, const SmallDesc* desc, int count,
                 double* zws, int* counter) {
    if (count <= 0) return 0;
    if (nmax < 1 || nmax > SMALL_MAX || grid < 1) return GEVD_E_STATE;
    hipLaunchKernelGGL(zero_counter, dim3(1), dim3(64), 0, st, counter);
    GEVD_LAUNCH_CHECK();
    return cx ? go_t<zdouble>(st, threads, grid, nmax, desc, count, zws, counter)
              : go_t<double>(st, threads, grid, nmax, desc, count, zws, counter);
}

int small_gen(hipStream_t st, bool cx, int n, int count, void* H, void* S, long stride, unsigned long long seed) {
    const long total = (long)n * n * count;
    if (total <= 0) return 0;
    const int nt = 256;
    const unsigned grid = (unsigned)((total + nt - 1) / nt);
    if (cx)
        hipLaunchKernelGGL(gen_kernel<zdouble>, dim3(grid), dim3(nt), 0, st, n, count, (zdouble*)H, (zdouble*)S,
                           stride, seed);
    else
        hipLaunchKernelGGL(gen_kernel<double>, dim3(grid), dim3(nt), 0, st, n, count, (double*)H, (double*)S, stride,
                           seed);
    GEVD_LAUNCH_CHECK();
    return 0;
}

}  // namespace gevd
