// One-stage Householder tridiagonalisation of a full Hermitian matrix and
// the back-transformation through its reflectors (the ELPA1-style route the
// paper benchmarks on GPUs for full spectra, section "ELPA - Usability").
//
// Blocked by panels of NB1 columns.  For column c of a panel: the column
// with the panel's pending updates applied (one workgroup) gives the
// reflector H_c = I - tau v v^H that zeroes it below the subdiagonal; the
// product y = A22 v with the stored trailing matrix runs over all CUs
// (memory-bound: this is where one-stage spends its time), the panel's
// pending updates are subtracted from y, and w = tau y - (tau/2)(y^H v) v.
// After the panel the trailing matrix takes A22 -= V W^H + W V^H as one MFMA
// product of inner length 2 NB1 ([V W] [W V]^H).  T = Q^H A Q is real
// tridiagonal: every reflector makes its subdiagonal entry real.
#include <algorithm>

#include "stages.hpp"

namespace gevd {
namespace {

constexpr int NB1 = 32;    // panel width
constexpr int NTC = 1024;  // threads of the column kernel
constexpr int HR = 256;    // rows per workgroup of the product y = A22 v
constexpr int HC = 128;    // columns per chunk of that product

// Column step of a panel (one workgroup).  Two phases, either may be off:
//  finish column qf: y (the reduced product A22 v) minus the pending panel
//    updates, times tau, then w = y - (tau/2)(y^H v) v into W[:, qf];
//  start column qn: a = A[:, c] minus the pending updates (rows >= c),
//    d[c] = Re a_c, the reflector of a[c+1:] into V[:, qn] (and its copy and
//    the kept reflector store Vall[:, c]), e[c] = beta, tau[c].
// Q holds [V | W | V] (three slots of pb columns, ld n); rows are absolute.
template <typename T>
__global__ __launch_bounds__(NTC) void s1_col_kernel(int n, const T* A, long lda, int c0, int pb, int qf, int qn,
                                                     T* Q, const T* y, T* Vall, double* d, double* e, T* tau) {
    __shared__ T red[NTC / WAVE];
    __shared__ T coef[2 * NB1];
    const int t = threadIdx.x;
    T* V = Q;
    T* W = Q + (size_t)pb * n;
    T* V2 = Q + (size_t)2 * pb * n;
    if (qf >= 0) {
        const int c = c0 + qf;
        const T* v = V + (size_t)qf * n;
        // p_j = W_j^H v, s_j = V_j^H v over rows c+1..n-1
        for (int j = 0; j < qf; ++j) {
            T ap = zero_of<T>(), as = zero_of<T>();
            for (int r = c + 1 + t; r < n; r += NTC) {
                ap += conjg(W[(size_t)j * n + r]) * v[r];
                as += conjg(V[(size_t)j * n + r]) * v[r];
            }
            ap = block_sum<NTC>(ap, red);
            as = block_sum<NTC>(as, red);
            if (t == 0) {
                coef[j] = ap;
                coef[NB1 + j] = as;
            }
        }
        __syncthreads();
        const T tc = tau[c];
        T dot = zero_of<T>();
        for (int r = c + 1 + t; r < n; r += NTC) {
            T yr = y[r - c - 1];
            for (int j = 0; j < qf; ++j) yr -= V[(size_t)j * n + r] * coef[j] + W[(size_t)j * n + r] * coef[NB1 + j];
            yr = tc * yr;
            W[(size_t)qf * n + r] = yr;  // y for now; w after the next sum
            dot += conjg(yr) * v[r];
        }
        dot = block_sum<NTC>(dot, red);
        const T al = from_real<T>(-0.5) * tc * dot;
        for (int r = c + 1 + t; r < n; r += NTC) W[(size_t)qf * n + r] += al * v[r];
        for (int r = t; r <= c; r += NTC) W[(size_t)qf * n + r] = zero_of<T>();
        __syncthreads();
    }
    if (qn >= 0) {
        const int c = c0 + qn;
        // a = A[c:, c] - sum_j (V_j conj(W[c, j]) + W_j conj(V[c, j])), held
        // back into V[:, qn] (rows c..n-1) until the reflector is known
        for (int j = t; j < qn; j += NTC) {
            coef[j] = conjg(W[(size_t)j * n + c]);
            coef[NB1 + j] = conjg(V[(size_t)j * n + c]);
        }
        __syncthreads();
        T* vq = V + (size_t)qn * n;
        double xn2 = 0.0;
        for (int r = c + t; r < n; r += NTC) {
            T a = A[IDX(r, c, lda)];
            for (int j = 0; j < qn; ++j) a -= V[(size_t)j * n + r] * coef[j] + W[(size_t)j * n + r] * coef[NB1 + j];
            vq[r] = a;
            if (r >= c + 2) xn2 += abs2(a);
        }
        xn2 = block_sum<NTC>(xn2, reinterpret_cast<double*>(red));
        __syncthreads();
        const T a0 = vq[c];
        const T alpha = c + 1 < n ? vq[c + 1] : zero_of<T>();
        const double ar = realp(alpha), ai = imagp(alpha);
        T tc;
        double beta;
        T scale;
        if (c + 1 >= n || (xn2 == 0.0 && ai == 0.0)) {
            tc = zero_of<T>();
            beta = ar;
            scale = zero_of<T>();
        } else {
            beta = -copysign(sqrt(ar * ar + ai * ai + xn2), ar);
            tc = div_r(from_real<T>(beta) - alpha, beta);
            scale = div_s(from_real<T>(1.0), alpha - from_real<T>(beta));
        }
        __syncthreads();  // every lane has read vq[c], vq[c+1]
        for (int r = t; r < n; r += NTC) {
            T v;
            if (r <= c) v = zero_of<T>();
            else if (r == c + 1) v = from_real<T>(1.0);
            else v = vq[r] * scale;
            vq[r] = v;
            V2[(size_t)qn * n + r] = v;
            Vall[IDX(r, c, n)] = v;
        }
        if (t == 0) {
            d[c] = realp(a0);
            if (c + 1 < n) e[c] = beta;
            tau[c] = tc;
        }
    }
}

// part[ch * m + i] = sum_{j in chunk ch} A22[i, j] v[j]: coalesced column
// reads, one pass over A22.
template <typename T>
__global__ __launch_bounds__(HR) void s1_hemv_kernel(int m, const T* A22, long lda, const T* v, T* part) {
    __shared__ T vs[HC];
    const int i = blockIdx.x * HR + threadIdx.x;
    const int j0 = blockIdx.y * HC;
    const int jn = min(HC, m - j0);
    for (int j = threadIdx.x; j < jn; j += HR) vs[j] = v[j0 + j];
    __syncthreads();
    if (i >= m) return;
    T acc = zero_of<T>();
    const T* col = A22 + IDX(i, j0, lda);
    for (int j = 0; j < jn; ++j) acc += col[(size_t)j * lda] * vs[j];
    part[(size_t)blockIdx.y * m + i] = acc;
}

template <typename T>
__global__ void s1_reduce_kernel(int m, int nch, const T* part, T* y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    T s = zero_of<T>();
    for (int c = 0; c < nch; ++c) s += part[(size_t)c * m + i];
    y[i] = s;
}

// last diagonal entry (untouched by any reflector)
template <typename T>
__global__ void s1_last_diag(int n, const T* A, long lda, double* d) {
    if (threadIdx.x == 0 && blockIdx.x == 0) d[n - 1] = realp(A[IDX(n - 1, n - 1, lda)]);
}

// T factor of a panel's compact WY form from G = V^H V and the tau's:
// T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j] (upper triangular).
template <typename T>
__global__ void s1_tfactor_kernel(int pb, const T* G, const T* tau, T* Tf) {
    const int i = threadIdx.x;
    if (i < pb)
        for (int j = 0; j < pb; ++j) Tf[IDX(i, j, pb)] = zero_of<T>();
    __syncthreads();
    for (int j = 0; j < pb; ++j) {
        if (i < j) {
            T s = zero_of<T>();
            for (int l = i; l < j; ++l) s += Tf[IDX(i, l, pb)] * G[IDX(l, j, pb)];
            Tf[IDX(i, j, pb)] = -tau[j] * s;
        }
        if (i == j) Tf[IDX(j, j, pb)] = tau[j];
        __syncthreads();
    }
}

inline int nchunks(int m) { return (m + HC - 1) / HC; }

}  // namespace

// Workspace of sytrd1 (elements of T): Q (3 NB1 n), y and the chunk
// partials, tau, the kept reflectors Vall (n x n).
template <typename T>
size_t sytrd1_ws_elems(int n) {
    return (size_t)3 * NB1 * n + 256 + (size_t)n + 256 + (size_t)nchunks(n) * n + 256 + (size_t)n + 256 +
           (size_t)n * n + 256;
}

template <typename T>
struct S1Ws {
    T *Q, *y, *part, *tau, *Vall;
};

template <typename T>
S1Ws<T> carve_s1(T* w, int n) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    S1Ws<T> s;
    size_t o = 0;
    s.Q = w + o; o = al(o + (size_t)3 * NB1 * n);
    s.y = w + o; o = al(o + n);
    s.part = w + o; o = al(o + (size_t)nchunks(n) * n);
    s.tau = w + o; o = al(o + n);
    s.Vall = w + o;
    return s;
}

// A (full Hermitian, both triangles read and clobbered) -> d, e (real
// tridiagonal); the reflectors stay in the workspace for sytrd1_back.
template <typename T>
int sytrd1(const StageCtx& c, int n, T* A, long lda, double* d, double* e, T* work) {
    S1Ws<T> w = carve_s1<T>(work, n);
    int rc = set_zero<T>(c.st, n, n, w.Vall, n);
    if (rc) return rc;
    const T one = from_real<T>(1.0), mone = from_real<T>(-1.0);
    for (int c0 = 0; c0 < n - 1; c0 += NB1) {
        const int pb = std::min(NB1, n - 1 - c0);
        for (int q = 0; q <= pb; ++q) {
            // finish column q-1 and start column q in one launch
            const int qf = q - 1, qn = q < pb ? q : -1;
            {
                KProbe probe(c.st, GEVD_K_PANEL, 0.0);
                hipLaunchKernelGGL(s1_col_kernel<T>, dim3(1), dim3(NTC), 0, c.st, n, (const T*)A, lda, c0, pb, qf, qn,
                                   w.Q, (const T*)w.y, w.Vall, d, e, w.tau);
                GEVD_LAUNCH_CHECK();
            }
            if (qn < 0) break;
            const int col = c0 + qn, m = n - col - 1;
            if (m <= 0) continue;
            // y = A22 v over the stored trailing matrix (rows/cols col+1..)
            const int nch = nchunks(m);
            {
                KProbe probe(c.st, GEVD_K_PANEL, (is_cplx<T>::value ? 8.0 : 2.0) * (double)m * m);
                hipLaunchKernelGGL(s1_hemv_kernel<T>, dim3((m + HR - 1) / HR, nch), dim3(HR), 0, c.st, m,
                                   (const T*)(A + IDX(col + 1, col + 1, lda)), lda,
                                   (const T*)(w.Q + (size_t)qn * n + col + 1), w.part);
                GEVD_LAUNCH_CHECK();
                hipLaunchKernelGGL(s1_reduce_kernel<T>, dim3((m + 255) / 256), dim3(256), 0, c.st, m, nch,
                                   (const T*)w.part, w.y);
                GEVD_LAUNCH_CHECK();
            }
        }
        // A22 -= [V W] [W V]^H on the trailing rows/columns
        const int r0 = c0 + pb, m2 = n - r0;
        if (m2 > 0) {
            rc = gemm<T>(c.st, OP_N, OP_C, m2, m2, 2 * pb, mone, w.Q + r0, n, w.Q + (size_t)pb * n + r0, n, one,
                         A + IDX(r0, r0, lda), lda);
            if (rc) return rc;
        }
    }
    hipLaunchKernelGGL(s1_last_diag<T>, dim3(1), dim3(64), 0, c.st, n, (const T*)A, lda, d);
    GEVD_LAUNCH_CHECK();
    return 0;
}

// Z (n x nev) <- Q Z with Q = H_0 H_1 ... H_{n-2}: panels last-first, each
// as (I - V T V^H) Z with V the panel's reflectors (zeros above the unit
// entries), G = V^H V, T from G and the tau's.
template <typename T>
size_t sytrd1_back_ws_elems(int n, int nev) {
    return (size_t)2 * NB1 * NB1 + 512 + (size_t)2 * NB1 * nev + 512;
}

template <typename T>
int sytrd1_back(const StageCtx& c, int n, int nev, const T* work1, T* Z, long ldz, T* work) {
    S1Ws<T> w = carve_s1<T>(const_cast<T*>(work1), n);
    T* G = work;
    T* Tf = G + NB1 * NB1 + 256;
    T* X = Tf + NB1 * NB1 + 256;
    T* Y = X + (size_t)NB1 * nev + 256;
    const T one = from_real<T>(1.0), mone = from_real<T>(-1.0), zero = zero_of<T>();
    const int np = n > 1 ? (n - 1 + NB1 - 1) / NB1 : 0;
    for (int p = np - 1; p >= 0; --p) {
        const int c0 = p * NB1, pb = std::min(NB1, n - 1 - c0), m = n - c0 - 1;
        const T* Vp = w.Vall + IDX(c0 + 1, c0, n);
        T* Zr = Z + (c0 + 1);
        int rc = gemm<T>(c.st, OP_C, OP_N, pb, pb, m, one, Vp, n, Vp, n, zero, G, pb);
        if (rc) return rc;
        {
            KProbe probe(c.st, GEVD_K_OTHER, 0.0);
            hipLaunchKernelGGL(s1_tfactor_kernel<T>, dim3(1), dim3(64), 0, c.st, pb, (const T*)G,
                               (const T*)(w.tau + c0), Tf);
            GEVD_LAUNCH_CHECK();
        }
        if ((rc = gemm<T>(c.st, OP_C, OP_N, pb, nev, m, one, Vp, n, Zr, ldz, zero, X, pb))) return rc;
        if ((rc = gemm<T>(c.st, OP_N, OP_N, pb, nev, pb, one, Tf, pb, X, pb, zero, Y, pb, K_A_UPPER))) return rc;
        if ((rc = gemm<T>(c.st, OP_N, OP_N, m, nev, pb, mone, Vp, n, Y, pb, one, Zr, ldz))) return rc;
    }
    return 0;
}

#define INST(T)                                                                              \
    template size_t sytrd1_ws_elems<T>(int);                                                 \
    template size_t sytrd1_back_ws_elems<T>(int, int);                                       \
    template int sytrd1<T>(const StageCtx&, int, T*, long, double*, double*, T*);            \
    template int sytrd1_back<T>(const StageCtx&, int, int, const T*, T*, long, T*);
INST(double)
INST(zdouble)
#undef INST

}  // namespace gevd
