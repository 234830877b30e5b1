// Orchestration of the standard Hermitian eigenproblem A z = eps z:
// full -> band (he2hb) -> tridiagonal (hb2st) -> divide-and-conquer (stedc)
// -> back-transformation through the bulge-chasing reflectors and then
// through the panel reflectors, for the wanted columns only.
#include <algorithm>
#include <vector>

#include "stages.hpp"

namespace gevd {
namespace {

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

int count_panels(int n, int b) {
    int np = 0;
    while (n - np * b - b >= 2) ++np;
    return np;
}

constexpr int SKB = 8;  // split of the long inner dimension in the stage-1 back-transform
constexpr int SKM = 128;  // largest split of the b x b product that joins two panels

template <typename T>
struct EighWs {
    BandRefl<T> R1;
    ChaseRefl<T> R2;
    T* Bw;
    long ldw;
    double *d, *e;
    int* sync_area;
    T* he_work;      // he2hb scratch
    T* bb_work;      // back_band scratch
    double* Zr;      // real eigenvectors from D&C (n x nev)
    char* dc_ws;     // D&C scratch
    T* acopy;        // reduced-precision form: FP64 copy of A for the refinement
    T* rf_work;      // refinement scratch
};

template <typename T>
size_t carve_eigh(char* base, int n, int nev, int b, int leaf, EighWs<T>* out, int prec = 0) {
    Carve c{base};
    EighWs<T> w;
    const int np = count_panels(n, b);
    w.R1.n = n;
    w.R1.b = b;
    w.R1.np = np;
    w.R1.V = c.take<T>(np > 0 ? w.R1.voff(np) : 1);
    w.R1.Tf = c.take<T>((size_t)std::max(np, 1) * b * b);
    w.ldw = 2 * b + 1;
    w.Bw = c.take<T>((size_t)w.ldw * n);
    const int nsw = n - 1;
    const int tmax = n > 1 ? (n - 1 + b - 1) / b : 0;
    w.R2.n = n;
    w.R2.b = b;
    w.R2.nsw = nsw;
    w.R2.tmax = tmax;
    w.R2.V2 = c.take<T>((size_t)std::max(tmax, 1) * std::max(nsw, 1) * b);
    w.R2.tau2 = c.take<T>((size_t)std::max(tmax, 1) * std::max(nsw, 1));
    w.R2.nbs = chase_group<T>();
    w.R2.nblk = (std::max(nsw, 1) + w.R2.nbs - 1) / w.R2.nbs;
    w.R2.Tg = c.take<T>((size_t)w.R2.nblk * std::max(tmax, 1) * w.R2.nbs * w.R2.nbs);
    w.d = c.take<double>(n);
    w.e = c.take<double>(n);
    w.sync_area = c.take<int>((size_t)n + 8);
    w.he_work = c.take<T>(he2hb_ws_elems<T>(n, b));
    w.bb_work = c.take<T>(back_band_ws_elems<T>(n, nev, b));
    w.Zr = c.take<double>((size_t)n * nev);
    w.dc_ws = c.take<char>(stedc_ws_bytes(n, nev, leaf));
    w.acopy = prec ? c.take<T>((size_t)n * n) : nullptr;
    w.rf_work = prec ? c.take<T>(refine_ws_elems<T>(n, nev)) : nullptr;
    if (out) *out = w;
    return c.off;
}

}  // namespace

// ---------------------------------------------------------------- stage 1 back
// Z <- Q1 Z with Q1 = prod_p (I - V_p T_p V_p^H): panels last-first, two at
// a time.  Panels q = p - 1 and p form one block reflector of width 2b,
// Q_q Q_p = I - [V_q V_p'] T_c [V_q V_p']^H with V_p' = V_p below b zero
// rows and T_c = [T_q, -T_q (V_q^H V_p') T_p; 0, T_p], applied as
// X = V^H Z_rows (split inner dimension), Y = T_c X, Z_rows -= V Y: one pass
// over the rows of Z per pair, with rank-2b updates.  An odd panel count
// applies the last panel alone.
template <typename T>
size_t back_band_ws_elems(int n, int nev, int b) {
    // X, Y (2b x nev), split-K partials (of X, or of the joining b x b
    // product), the pair's V (n x 2b), its T (2b x 2b), two b x b products
    const size_t part = std::max((size_t)SKB * 2 * b * nev, (size_t)SKM * b * b);
    return (size_t)2 * 2 * b * nev + part + (size_t)2 * b * n + (size_t)6 * b * b + 64;
}

template <typename T>
int back_band(const StageCtx& c, const BandRefl<T>& R, int nev, T* Z, long ldz, T* work) {
    const int b = R.b, n = R.n, b2 = 2 * b;
    T* X = work;
    T* Y = X + (size_t)b2 * nev;
    T* sk = Y + (size_t)b2 * nev;
    T* Vc = sk + std::max((size_t)SKB * b2 * nev, (size_t)SKM * b * b);
    T* Tc = Vc + (size_t)b2 * n;
    T* M = Tc + (size_t)b2 * b2;
    T* N1 = M + (size_t)b * b;
    const T one = from_real<T>(1.0), mone = from_real<T>(-1.0), zero = zero_of<T>();
    // apply the block reflector I - V Tm V^H (m x w, T upper w x w) to the rows of Z from r0
    auto apply = [&](const T* V, const T* Tm, int m, int w, int r0) -> int {
        T* Zr = Z + r0;
        int rc = gemm<T>(c.st, OP_C, OP_N, w, nev, m, one, V, m, Zr, ldz, zero, X, w, K_FULL, T_ALL, Batch(),
                         m >= 1024 ? SKB : 1, sk);
        if (rc) return rc;
        if ((rc = gemm<T>(c.st, OP_N, OP_N, w, nev, w, one, Tm, w, X, w, zero, Y, w, K_A_UPPER))) return rc;
        return gemm<T>(c.st, OP_N, OP_N, m, nev, w, mone, V, m, Y, w, one, Zr, ldz);
    };
    auto single = [&](int p) -> int {
        const int m = n - p * b - b;
        return apply(R.V + R.voff(p), R.Tf + (size_t)p * b * b, m, b, p * b + b);
    };
    int rc = 0;
    int p = R.np - 1;
    if (R.np % 2 == 1) {
        if ((rc = single(p))) return rc;
        --p;
    }
    for (; p >= 1; p -= 2) {
        const int q = p - 1;
        const int m = n - q * b - b, m2 = m - b;  // rows of V_q and of V_p
        if (m2 < 1) {
            if ((rc = single(p)) || (rc = single(q))) return rc;
            continue;
        }
        const T* Vq = R.V + R.voff(q);
        const T* Vp = R.V + R.voff(p);
        const T* Tq = R.Tf + (size_t)q * b * b;
        const T* Tp = R.Tf + (size_t)p * b * b;
        // V = [V_q, V_p'] (m x 2b)
        if ((rc = copy_matrix<T>(c.st, m, b, Vq, m, Vc, m))) return rc;
        if ((rc = set_zero<T>(c.st, b, b, Vc + (size_t)b * m, m))) return rc;
        if ((rc = copy_matrix<T>(c.st, m2, b, Vp, m2, Vc + (size_t)b * m + b, m))) return rc;
        // T_c: diagonal blocks T_q, T_p (only their upper triangles are read),
        // upper-right block -T_q (V_q^H V_p') T_p
        // one b x b output tile: the inner dimension in chunks of about 128
        // rows, so that the product spreads over the device
        const int skm = std::max(1, std::min(SKM, (m2 + 127) / 128));
        if ((rc = gemm<T>(c.st, OP_C, OP_N, b, b, m2, one, Vq + b, m, Vp, m2, zero, M, b, K_FULL, T_ALL, Batch(),
                          skm, sk)))
            return rc;
        if ((rc = gemm<T>(c.st, OP_N, OP_N, b, b, b, one, Tq, b, M, b, zero, N1, b, K_A_UPPER))) return rc;
        if ((rc = gemm<T>(c.st, OP_N, OP_N, b, b, b, mone, N1, b, Tp, b, zero, Tc + (size_t)b * b2, b2,
                          K_B_UPPER)))
            return rc;
        if ((rc = copy_matrix<T>(c.st, b, b, Tq, b, Tc, b2))) return rc;
        if ((rc = copy_matrix<T>(c.st, b, b, Tp, b, Tc + (size_t)b * b2 + b, b2))) return rc;
        if ((rc = apply(Vc, Tc, m, b2, q * b + b))) return rc;
    }
    if (p == 0 && (rc = single(0))) return rc;
    return 0;
}

template <typename T>
size_t band_ws_bytes(int n, int b) {
    return carve_eigh<T>(nullptr, n, 1, b, 0, nullptr) + 256;
}

// one-stage route: sytrd1's workspace (reflectors), its back-transformation
// scratch, d, e, the D&C eigenvectors and scratch
template <typename T>
size_t carve_eigh1(char* base, int n, int nev, int leaf, T** s1, T** bk, double** d, double** e, double** Zr,
                   char** dc) {
    Carve c{base};
    T* a = c.take<T>(sytrd1_ws_elems<T>(n));
    T* b = c.take<T>(sytrd1_back_ws_elems<T>(n, nev));
    double* dd = c.take<double>(n);
    double* ee = c.take<double>(n);
    double* zr = c.take<double>((size_t)n * nev);
    char* dw = c.take<char>(stedc_ws_bytes(n, nev, leaf));
    if (s1) *s1 = a;
    if (bk) *bk = b;
    if (d) *d = dd;
    if (e) *e = ee;
    if (Zr) *Zr = zr;
    if (dc) *dc = dw;
    return c.off;
}

template <typename T>
size_t eigh_ws_bytes(int n, int nev, int b, int leaf, int prec) {
    return std::max(carve_eigh<T>(nullptr, n, nev, b, leaf, nullptr, prec),
                    carve_eigh1<T>(nullptr, n, nev, leaf, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr)) +
           256;
}

template <typename T>
int band_run(const StageCtx& c, int n, T* A, long lda, T* Bd, long ldb, char* ws) {
    EighWs<T> w;
    carve_eigh<T>(ws, n, 1, c.b, 0, &w);
    // he2hb writes all ldb rows; rows beyond b are zero
    return he2hb<T>(c, n, A, lda, w.R1, Bd, ldb, w.he_work);
}

template <typename T>
int tridiag_run(const StageCtx& c, int n, T* A, long lda, double* d, double* e, char* ws) {
    if (c.stages == 1) {
        T* s1;
        double *dd, *ee;
        carve_eigh1<T>(ws, n, 1, c.leaf, &s1, nullptr, &dd, &ee, nullptr, nullptr);
        return sytrd1<T>(c, n, A, lda, d, e ? e : ee, s1);
    }
    EighWs<T> w;
    carve_eigh<T>(ws, n, 1, c.b, c.leaf, &w);
    int rc = he2hb<T>(c, n, A, lda, w.R1, w.Bw, w.ldw, w.he_work);
    if (rc) return rc;
    double* ee = e ? e : w.e;
    return hb2st<T>(c, n, w.Bw, w.ldw, w.R2, d, ee, w.sync_area);
}

// One-stage route (c.stages == 1): Householder tridiagonalisation,
// divide-and-conquer, one back-transformation.  FP64 throughout.
template <typename T>
int eigh1_run(const StageCtx& c, int n, int nev, T* A, long lda, double* eval, T* Z, long ldz, char* ws) {
    T *s1, *bk;
    double *d, *e, *Zr;
    char* dc;
    carve_eigh1<T>(ws, n, nev, c.leaf, &s1, &bk, &d, &e, &Zr, &dc);
    int rc = sytrd1<T>(c, n, A, lda, d, e, s1);
    if (rc) return rc;
    c.phase(GEVD_PH_TRIDIAG);
    c.phase(GEVD_PH_SOLVE);
    if ((rc = stedc_run(c, n, nev, d, e, eval, Zr, n, dc))) return rc;
    c.phase(GEVD_PH_BACK2);
    if (is_cplx<T>::value) rc = real_to_scalar_z(c.st, n, nev, Zr, n, reinterpret_cast<zdouble*>(Z), ldz);
    else rc = real_to_scalar_d(c.st, n, nev, Zr, n, reinterpret_cast<double*>(Z), ldz);
    if (rc) return rc;
    c.phase(GEVD_PH_BACK1);
    return sytrd1_back<T>(c, n, nev, s1, Z, ldz, bk);
}

template <typename T>
int eigh_run(const StageCtx& c, int n, int nev, T* A, long lda, double* eval, T* Z, long ldz, char* ws) {
    if (c.stages == 1) return eigh1_run<T>(c, n, nev, A, lda, eval, Z, ldz, ws);
    EighWs<T> w;
    carve_eigh<T>(ws, n, nev, c.b, c.leaf, &w, c.prec);
    int rc = 0;
    if (c.prec && (rc = copy_matrix<T>(c.st, n, n, A, lda, w.acopy, n))) return rc;
    {
        Fp32Gemm f32(c.prec != 0);
        if ((rc = he2hb<T>(c, n, A, lda, w.R1, w.Bw, w.ldw, w.he_work))) return rc;
    }
    c.phase(GEVD_PH_TRIDIAG);
    if ((rc = hb2st<T>(c, n, w.Bw, w.ldw, w.R2, w.d, w.e, w.sync_area))) return rc;
    // the stage-2 T factors on the second stream, beside the tridiagonal
    // solve (which leaves the device idle at its host synchronisations)
    const bool tf_aux = c.aux != nullptr && c.fork != nullptr && c.join != nullptr;
    if (tf_aux) {
        GEVD_HIP(hipEventRecord(c.fork, c.st));
        GEVD_HIP(hipStreamWaitEvent(c.aux, c.fork, 0));
        if ((rc = back_chase_tfactor<T>(w.R2, c.aux))) return rc;
        GEVD_HIP(hipEventRecord(c.join, c.aux));
    }
    c.phase(GEVD_PH_SOLVE);
    if ((rc = stedc_run(c, n, nev, w.d, w.e, eval, w.Zr, n, w.dc_ws))) return rc;
    c.phase(GEVD_PH_BACK2);
    if (is_cplx<T>::value) rc = real_to_scalar_z(c.st, n, nev, w.Zr, n, reinterpret_cast<zdouble*>(Z), ldz);
    else rc = real_to_scalar_d(c.st, n, nev, w.Zr, n, reinterpret_cast<double*>(Z), ldz);
    if (rc) return rc;
    if (tf_aux) GEVD_HIP(hipStreamWaitEvent(c.st, c.join, 0));
    if ((rc = back_chase<T>(c, w.R2, nev, Z, ldz, tf_aux))) return rc;
    c.phase(GEVD_PH_BACK1);
    {
        Fp32Gemm f32(c.prec != 0);
        if ((rc = back_band<T>(c, w.R1, nev, Z, ldz, w.bb_work))) return rc;
    }
    if (c.prec) rc = refine<T>(c, n, nev, w.acopy, n, Z, ldz, eval, w.rf_work, c.refine_iters);
    return rc;
}

// All eigenvalues of A, then the eigenvectors of those at or below thresh
// (the first m in ascending order): the count is taken on the host from the
// eigenvalues before any eigenvector is back-transformed.  Z needs room for
// n columns; ws is sized by eigh_ws_bytes(n, n, ...).
template <typename T>
int eigh_select_run(const StageCtx& c, int n, double thresh, T* A, long lda, double* eval, T* Z, long ldz,
                    char* ws, int* m_out) {
    EighWs<T> w;
    carve_eigh<T>(ws, n, n, c.b, c.leaf, &w, 0);
    *m_out = 0;
    int rc = he2hb<T>(c, n, A, lda, w.R1, w.Bw, w.ldw, w.he_work);
    if (rc) return rc;
    if ((rc = hb2st<T>(c, n, w.Bw, w.ldw, w.R2, w.d, w.e, w.sync_area))) return rc;
    if ((rc = stedc_run(c, n, n, w.d, w.e, eval, w.Zr, n, w.dc_ws))) return rc;
    std::vector<double> ev(n);
    GEVD_HIP(hipMemcpyAsync(ev.data(), eval, sizeof(double) * n, hipMemcpyDeviceToHost, c.st));
    GEVD_HIP(hipStreamSynchronize(c.st));
    const int m = (int)(std::upper_bound(ev.begin(), ev.end(), thresh) - ev.begin());
    *m_out = m;
    if (m == 0) return 0;
    if (is_cplx<T>::value) rc = real_to_scalar_z(c.st, n, m, w.Zr, n, reinterpret_cast<zdouble*>(Z), ldz);
    else rc = real_to_scalar_d(c.st, n, m, w.Zr, n, reinterpret_cast<double*>(Z), ldz);
    if (rc) return rc;
    if ((rc = back_chase<T>(c, w.R2, m, Z, ldz))) return rc;
    return back_band<T>(c, w.R1, m, Z, ldz, w.bb_work);
}

#define INST(T)                                                                              \
    template int eigh_select_run<T>(const StageCtx&, int, double, T*, long, double*, T*, long, char*, int*); \
    template size_t back_band_ws_elems<T>(int, int, int);                                    \
    template int back_band<T>(const StageCtx&, const BandRefl<T>&, int, T*, long, T*);       \
    template size_t band_ws_bytes<T>(int, int);                                              \
    template size_t eigh_ws_bytes<T>(int, int, int, int, int);                               \
    template int band_run<T>(const StageCtx&, int, T*, long, T*, long, char*);               \
    template int tridiag_run<T>(const StageCtx&, int, T*, long, double*, double*, char*);    \
    template int eigh_run<T>(const StageCtx&, int, int, T*, long, double*, T*, long, char*);
INST(double)
INST(zdouble)
#undef INST

}  // namespace gevd
