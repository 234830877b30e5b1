// Stages of the standard Hermitian eigenproblem (internal interface).
#pragma once
#include "kernels.hpp"

namespace gevd {

struct StageCtx {
    hipStream_t st;
    int* noconv;  // device flag: tridiagonal solver failed
    int* hang;    // device flag: a bounded device-side wait expired
    int b;        // half-bandwidth of the intermediate band
    int leaf;     // divide-and-conquer leaf size (0 = default)
    void (*mark)(void*, int) = nullptr;
    void* mark_arg = nullptr;
    // 1: reduced-precision form (full -> band and stage-1 back-transformation
    // products on the FP32 matrix cores, then FP64 refinement of the wanted
    // pairs against a copy of A)
    int prec = 0;
    int refine_iters = 2;
    // 1: one persistent launch per full -> band panel (needs its grid
    // resident at once); 0: one launch per panel column
    int panel_persist = 1;
    // 1: one-stage Householder tridiagonalisation (sytrd.hip) instead of
    // full -> band -> tridiagonal
    int stages = 2;
    // optional second stream and two events (owned by the handle): the
    // full -> band reduction runs each trailing update beside the next
    // panel's factorization
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    void phase(int p) const {
        if (mark) mark(mark_arg, p);
    }
};

// Reflectors of the full -> band stage, kept for the back-transformation.
template <typename T>
struct BandRefl {
    int n = 0, b = 0, np = 0;  // panels: panel p starts at column p*b, has m_p = n - p*b - b rows
    T* V = nullptr;            // panel p: m_p x b at V + voff(p), ld m_p
    T* Tf = nullptr;           // panel p: b x b at Tf + p*b*b
    size_t voff(int p) const {
        // sum_{q<p} (n - q b - b) b
        return (size_t)b * ((size_t)p * (n - b) - (size_t)b * p * (p - 1) / 2);
    }
};

// Reflectors of the band -> tridiagonal stage: reflector (sweep s, block t)
// acts on rows s+1+t*b .. s+t*b+b (clipped at n), v at V2 + (t*nsw + s)*b.
template <typename T>
struct ChaseRefl {
    int n = 0, b = 0, nsw = 0, tmax = 0;
    T* V2 = nullptr;
    T* tau2 = nullptr;
    // back-transformation groups: nbs consecutive sweeps at one block index t,
    // group (S, t) has compact-WY factor T at Tg + (t*nblk + S)*nbs*nbs
    int nbs = 0, nblk = 0;
    T* Tg = nullptr;
};
// sweeps per back-transformation group
template <typename T>
constexpr int chase_group() {
    return is_cplx<T>::value ? 32 : 64;
}

template <typename T>
size_t band_ws_bytes(int n, int b);
template <typename T>
size_t eigh_ws_bytes(int n, int nev, int b, int leaf, int prec = 0);
size_t stedc_ws_bytes(int n, int nev, int leaf);

// Full Hermitian A (clobbered) -> band in lower band storage (Bd, ldb).
template <typename T>
int band_run(const StageCtx& c, int n, T* A, long lda, T* Bd, long ldb, char* ws);
// Full Hermitian A -> tridiagonal (d, e).
template <typename T>
int tridiag_run(const StageCtx& c, int n, T* A, long lda, double* d, double* e, char* ws);
// Tridiagonal (d, e) -> eval (all n) and Z (n x nev, real).
int stedc_run(const StageCtx& c, int n, int nev, const double* d, const double* e, double* eval, double* Z,
              long ldz, char* ws);
// Whole standard eigenproblem.
template <typename T>
int eigh_run(const StageCtx& c, int n, int nev, T* A, long lda, double* eval, T* Z, long ldz, char* ws);
// All eigenvalues, and eigenvectors only of the m at or below thresh (m
// counted after the eigenvalues are known; synchronises the stream once).
template <typename T>
int eigh_select_run(const StageCtx& c, int n, double thresh, T* A, long lda, double* eval, T* Z, long ldz,
                    char* ws, int* m_out);

// ---- stage building blocks (he2hb.hip, hb2st.hip, backtr.hip)
template <typename T>
size_t he2hb_ws_elems(int n, int b);
template <typename T>
int he2hb(const StageCtx& c, int n, T* A, long lda, BandRefl<T>& R, T* Bd, long ldb, T* work);
template <typename T>
int hb2st(const StageCtx& c, int n, T* Bw, long ldw, ChaseRefl<T>& R, double* d, double* e, int* sync_area);
// The compact-WY T factors of all stage-2 reflector groups, on stream st
// (they depend only on the reflectors, so they may run beside the
// tridiagonal solve); back_chase forms them itself unless tfactored.
template <typename T>
int back_chase_tfactor(const ChaseRefl<T>& R, hipStream_t st);
template <typename T>
int back_chase(const StageCtx& c, const ChaseRefl<T>& R, int nev, T* Z, long ldz, bool tfactored = false);
template <typename T>
int back_band(const StageCtx& c, const BandRefl<T>& R, int nev, T* Z, long ldz, T* work);
template <typename T>
size_t back_band_ws_elems(int n, int nev, int b);
// One-stage tridiagonalisation and its back-transformation (sytrd.hip).
template <typename T>
size_t sytrd1_ws_elems(int n);
template <typename T>
size_t sytrd1_back_ws_elems(int n, int nev);
template <typename T>
int sytrd1(const StageCtx& c, int n, T* A, long lda, double* d, double* e, T* work);
template <typename T>
int sytrd1_back(const StageCtx& c, int n, int nev, const T* work1, T* Z, long ldz, T* work);
// FP64 refinement of k approximate eigenpairs (refine.hip).
template <typename T>
size_t refine_ws_elems(int n, int k);
template <typename T>
int refine(const StageCtx& c, int n, int k, const T* A, long lda, T* X, long ldx, double* eval, T* work, int iters);

}  // namespace gevd
