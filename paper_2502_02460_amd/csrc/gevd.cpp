// Host pipeline and C interface of the generalized eigensolver (gevd.h).
//
// Each entry point validates its arguments on the host, sizes the handle's
// workspace, and enqueues kernels on the handle's stream.  The only host
// waits are where a device-computed status must be returned (positive
// definiteness, convergence) and at the end of a whole solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "arbiter.hpp"
#include "batch.hpp"
#include "ctx.hpp"
#include "kernels.hpp"
#include "stages.hpp"

using namespace gevd;

namespace gevd {
thread_local KStats* g_kstats = nullptr;
}

namespace {

constexpr int NFLAGS = 16;
enum { F_INFO = 0, F_NONFINITE = 1, F_NOCONV = 2, F_HANG = 3 };

struct Bump {
    char* base;
    size_t off = 0;
    explicit Bump(char* b) : base(b) {}
    template <typename T>
    T* take(size_t elems) {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
        off += elems * sizeof(T);
        return p;
    }
};

int ensure_ws(gevd_ctx* h, size_t bytes) {
    if (bytes <= h->ws_bytes) return 0;
    GEVD_HIP(hipSetDevice(h->device));
    if (h->ws) {
        GEVD_HIP(hipStreamSynchronize(h->stream));
        GEVD_HIP(hipFree(h->ws));
        h->ws = nullptr;
        h->ws_bytes = 0;
    }
    size_t want = bytes + (bytes >> 4);
    if (hipMalloc(&h->ws, want) != hipSuccess) {
        (void)hipGetLastError();
        h->ws = nullptr;
        return GEVD_E_NOMEM;
    }
    h->ws_bytes = want;
    return 0;
}

int read_flags(gevd_ctx* h, int* host) {
    GEVD_HIP(hipMemcpyAsync(host, h->flags, NFLAGS * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    GEVD_HIP(hipStreamSynchronize(h->stream));
    return 0;
}

int clear_flags(gevd_ctx* h) {
    GEVD_HIP(hipMemsetAsync(h->flags, 0, NFLAGS * sizeof(int), h->stream));
    return 0;
}

// After a Cholesky S = U^H U: cond(S) = cond(U)^2 >= (max|U_ii| / min|U_ii|)^2
// (the diagonal of a triangular U holds its eigenvalues).  Enqueues the
// diagonal scan; settle_cond reads it once the stream has been synchronised.
template <typename T>
int scan_cond(gevd_ctx* h, int n, const T* U, int ldu) {
    int rc = diag_range<T>(h->stream, n, U, ldu, h->dstat);
    if (rc) return rc;
    GEVD_HIP(hipMemcpyAsync(h->dhost, h->dstat, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    return 0;
}

void settle_cond(gevd_ctx* h) {
    const double mx = h->dhost[0], mn = h->dhost[1];
    h->kappa_lb = mn > 0.0 ? (mx / mn) * (mx / mn) : INFINITY;
    if (h->kappa_lb > GEVD_ILLCOND_KAPPA) h->warn |= GEVD_W_ILLCOND;
}

void mark(gevd_ctx* h, int phase) {
    if (h->timing && h->ev_made) (void)hipEventRecord(h->ev[phase], h->stream);
}

// Points the launch probes of this thread at the handle's accounting for the
// duration of one entry point.
struct KScope {
    explicit KScope(gevd_ctx* h) {
        g_kstats = h->kstats_on ? &h->ks : nullptr;
        g_tile_force = h->gemm_tile;
    }
    ~KScope() {
        g_kstats = nullptr;
        g_tile_force = -1;
    }
};

// The persistent full -> band panel route for the duration of one entry
// point: taken when the handle asks for it (GEVD_OPT_PANEL) and no other
// handle of the process holds it on this device (arbiter.hpp); otherwise
// this call uses one launch per panel column.  An owner waits for its
// streams before giving the route back, so two persistent panel grids never
// run on the device at once.
struct PanelLease {
    gevd_ctx* h;
    bool owned = false;
    explicit PanelLease(gevd_ctx* hh) : h(hh) {
        owned = h->panel_persist && panel_arbiter().try_acquire(h->device, h);
        h->persist_now = owned ? 1 : 0;
    }
    ~PanelLease() {
        h->persist_now = 0;
        if (!owned) return;
        (void)hipStreamSynchronize(h->stream);
        if (h->aux) (void)hipStreamSynchronize(h->aux);
        panel_arbiter().release(h->device, h);
    }
};

// The second stream of overlapped stages (default priority, ordered against
// the handle's stream by events only); left null if it cannot be made.  It
// may use every CU: reserving the last 16 or 32 CUs for the latency-bound
// panel kernels running beside it made the full -> band stage 4 % slower
// on gfx950 (the trailing updates lost more than the panels gained).
void attach_aux(gevd_ctx* h, StageCtx& sc) {
    sc.panel_persist = h->persist_now;
    sc.stages = h->stages;
    if (!h->aux) {
        if (hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&h->aux_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&h->aux_join, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
    }
    sc.aux = h->aux;
    sc.fork = h->aux_fork;
    sc.join = h->aux_join;
}

// Default half-bandwidth: 64 for large orders (fewer, wider panels and
// bulge-reflector groups; the workgroup bulge-chasing kernel keeps the
// band -> tridiagonal stage in check), 32 below that.
int pick_band(const gevd_ctx* h, int n) {
    int b = h->band_opt > 0 ? h->band_opt : (n >= 4096 ? 64 : 32);
    if (n <= 2 * b) b = std::max(1, std::min(b, n / 2));
    return std::max(1, b);
}

// ------------------------------------------------------------- workspace plans
template <typename T>
size_t plan_cholesky(int n) {
    Bump b(nullptr);
    b.take<T>(potrf_work_elems<T>(n));
    return b.off;
}

template <typename T>
size_t plan_invert(int n) {
    Bump b(nullptr);
    b.take<T>(trtri_work_elems<T>(n));
    return b.off;
}

template <typename T>
size_t plan_reduce(int n) {
    Bump b(nullptr);
    b.take<T>((size_t)n * n);
    return b.off;
}

// ------------------------------------------------------------- steps
template <typename T>
int do_cholesky(gevd_ctx* h, int n, T* S, int lds, char* ws) {
    Bump b(ws);
    T* work = b.take<T>(potrf_work_elems<T>(n));
    return potrf<T>(h->stream, n, S, lds, work, h->flags + F_INFO);
}

template <typename T>
int do_invert(gevd_ctx* h, int n, const T* U, int ldu, T* Uinv, int ldi, char* ws) {
    Bump b(ws);
    T* work = b.take<T>(trtri_work_elems<T>(n));
    return trtri<T>(h->stream, n, U, ldu, Uinv, ldi, work);
}

// A = X^H H X with X = Uinv (upper triangular), in n^3 flops (real count;
// the explicit-inverse products H X then X^H (H X) take 4n^3/3): with
// H = M + M^H, M = triu(H) - diag(H)/2, the product Y = M X is upper
// triangular and costs n^3/3 (inner range [i, j] per element), Z = X^H Y
// costs 2n^3/3 (inner range up to min(i, j)), and A = Z + Z^H exactly
// Hermitian.  H's diagonal is halved in place (H is clobbered); Z is formed
// in A's storage (A may be H).
template <typename T>
int do_reduce(gevd_ctx* h, int n, T* H, int ldh, const T* Uinv, int ldi, T* A, int lda, char* ws) {
    Bump b(ws);
    T* Y = b.take<T>((size_t)n * n);
    const T one = from_real<T>(1.0), zero = zero_of<T>();
    int rc = scale_diag<T>(h->stream, n, H, ldh, 0.5);
    if (rc) return rc;
    rc = gemm<T>(h->stream, OP_N, OP_N, n, n, n, one, H, ldh, Uinv, ldi, zero, Y, n, K_AU_BU, T_UPPER_TILES);
    if (rc) return rc;
    rc = gemm<T>(h->stream, OP_C, OP_N, n, n, n, one, Uinv, ldi, Y, n, zero, A, lda, K_AL_BU);
    if (rc) return rc;
    return herm_sum_inplace<T>(h->stream, n, A, lda);
}

template <typename T>
int do_backtransform(gevd_ctx* h, int n, int nev, const T* Uinv, int ldi, const T* Ct, int ldct, T* C, int ldc) {
    const T one = from_real<T>(1.0), zero = zero_of<T>();
    return gemm<T>(h->stream, OP_N, OP_N, n, nev, n, one, Uinv, ldi, Ct, ldct, zero, C, ldc, K_A_UPPER);
}

template <typename T>
size_t plan_solve(const gevd_ctx* h, int n, int nev) {
    Bump b(nullptr);
    b.take<T>((size_t)n * n);  // Uinv
    size_t rest = std::max({plan_cholesky<T>(n), plan_invert<T>(n), plan_reduce<T>(n),
                            eigh_ws_bytes<T>(n, nev, pick_band(h, n), h->leaf_opt, h->prec)});
    return b.off + 256 + rest + (size_t)n * nev * sizeof(T) + 256;
}

template <typename T>
int do_eigh(gevd_ctx* h, int n, int nev, T* A, int lda, double* eval, T* Z, int ldz, char* ws, bool timed) {
    StageCtx sc{h->stream, h->flags + F_NOCONV, h->flags + F_HANG, pick_band(h, n), h->leaf_opt};
    attach_aux(h, sc);
    sc.prec = h->prec;
    sc.refine_iters = h->refine_iters;
    if (timed) {
        sc.mark = [](void* p, int ph) { mark((gevd_ctx*)p, ph); };
        sc.mark_arg = h;
    }
    return eigh_run<T>(sc, n, nev, A, lda, eval, Z, ldz, ws);
}

template <typename T>
int do_solve(gevd_ctx* h, int n, int nev, T* H, int ldh, T* S, int lds, double* eval, T* C, int ldc) {
    int rc = ensure_ws(h, plan_solve<T>(h, n, nev));
    if (rc) return rc;
    Bump b(h->ws);
    T* Uinv = b.take<T>((size_t)n * n);
    T* Ct = b.take<T>((size_t)n * nev);
    char* rest = reinterpret_cast<char*>(b.take<char>(0));
    if ((rc = clear_flags(h))) return rc;
    if ((rc = check_finite_upper<T>(h->stream, n, H, ldh, h->flags + F_NONFINITE))) return rc;
    if ((rc = check_finite_upper<T>(h->stream, n, S, lds, h->flags + F_NONFINITE))) return rc;
    h->ev_valid = false;
    mark(h, GEVD_PH_CHOLESKY);
    if ((rc = do_cholesky<T>(h, n, S, lds, rest))) return rc;
    if ((rc = scan_cond<T>(h, n, S, lds))) return rc;
    int fl[NFLAGS];
    if ((rc = read_flags(h, fl))) return rc;
    if (fl[F_NONFINITE]) return GEVD_E_NONFINITE;
    if (fl[F_INFO]) return fl[F_INFO];
    settle_cond(h);
    mark(h, GEVD_PH_INVERT);
    if ((rc = do_invert<T>(h, n, S, lds, Uinv, n, rest))) return rc;
    mark(h, GEVD_PH_MULTIPLY);
    if ((rc = do_reduce<T>(h, n, H, ldh, Uinv, n, H, ldh, rest))) return rc;
    mark(h, GEVD_PH_BAND);
    if ((rc = do_eigh<T>(h, n, nev, H, ldh, eval, Ct, n, rest, true))) return rc;
    mark(h, GEVD_PH_MULT);
    if ((rc = do_backtransform<T>(h, n, nev, Uinv, n, Ct, n, C, ldc))) return rc;
    mark(h, GEVD_NPHASE);
    if ((rc = read_flags(h, fl))) return rc;
    if (fl[F_HANG]) return GEVD_E_HANG;
    if (fl[F_NOCONV]) return GEVD_E_NOCONV;
    h->ev_valid = h->timing != 0;
    if (h->kstats_on) h->ks.settle();  // the stream is idle here
    return 0;
}

template <typename T>
int do_set_overlap(gevd_ctx* h, int n, const T* S, int lds) {
    const size_t need = (size_t)n * n * sizeof(T);
    if (h->uinv_bytes < need) {
        if (h->uinv) {
            GEVD_HIP(hipStreamSynchronize(h->stream));
            GEVD_HIP(hipFree(h->uinv));
            h->uinv = nullptr;
            h->uinv_bytes = 0;
        }
        if (hipMalloc(&h->uinv, need) != hipSuccess) {
            (void)hipGetLastError();
            return GEVD_E_NOMEM;
        }
        h->uinv_bytes = need;
    }
    h->res_n = 0;
    Bump plan(nullptr);
    plan.take<T>((size_t)n * n);
    const size_t ws = plan.off + 256 + std::max(plan_cholesky<T>(n), plan_invert<T>(n));
    int rc = ensure_ws(h, ws);
    if (rc) return rc;
    Bump b(h->ws);
    T* U = b.take<T>((size_t)n * n);
    char* rest = reinterpret_cast<char*>(b.take<char>(0));
    if ((rc = clear_flags(h))) return rc;
    if ((rc = check_finite_upper<T>(h->stream, n, S, lds, h->flags + F_NONFINITE))) return rc;
    if ((rc = copy_matrix<T>(h->stream, n, n, S, lds, U, n))) return rc;
    if ((rc = do_cholesky<T>(h, n, U, n, rest))) return rc;
    if ((rc = scan_cond<T>(h, n, U, n))) return rc;
    int fl[NFLAGS];
    if ((rc = read_flags(h, fl))) return rc;
    if (fl[F_NONFINITE]) return GEVD_E_NONFINITE;
    if (fl[F_INFO]) return fl[F_INFO];
    settle_cond(h);
    if ((rc = do_invert<T>(h, n, U, n, reinterpret_cast<T*>(h->uinv), n, rest))) return rc;
    if ((rc = read_flags(h, fl))) return rc;
    h->res_n = n;
    h->res_dtype = is_cplx<T>::value ? GEVD_COMPLEX : GEVD_REAL;
    return 0;
}

template <typename T>
int do_solve_resident(gevd_ctx* h, int nev, T* H, int ldh, double* eval, T* C, int ldc) {
    const int n = h->res_n;
    int rc = ensure_ws(h, plan_solve<T>(h, n, nev));
    if (rc) return rc;
    const T* Uinv = reinterpret_cast<const T*>(h->uinv);
    Bump b(h->ws);
    b.take<T>((size_t)n * n);  // (the Uinv slot of a full solve, unused here)
    T* Ct = b.take<T>((size_t)n * nev);
    char* rest = reinterpret_cast<char*>(b.take<char>(0));
    if ((rc = clear_flags(h))) return rc;
    if ((rc = check_finite_upper<T>(h->stream, n, H, ldh, h->flags + F_NONFINITE))) return rc;
    h->ev_valid = false;
    if ((rc = do_reduce<T>(h, n, H, ldh, Uinv, n, H, ldh, rest))) return rc;
    if ((rc = do_eigh<T>(h, n, nev, H, ldh, eval, Ct, n, rest, false))) return rc;
    if ((rc = do_backtransform<T>(h, n, nev, Uinv, n, Ct, n, C, ldc))) return rc;
    int fl[NFLAGS];
    if ((rc = read_flags(h, fl))) return rc;
    if (fl[F_NONFINITE]) return GEVD_E_NONFINITE;
    if (fl[F_HANG]) return GEVD_E_HANG;
    if (fl[F_NOCONV]) return GEVD_E_NOCONV;
    if (h->kstats_on) h->ks.settle();
    return 0;
}

// ------------------------------------------------ ill-conditioned overlap route
template <typename T>
size_t plan_reduced(const gevd_ctx* h, int n, int nev) {
    Bump b(nullptr);
    for (int i = 0; i < 4; ++i) b.take<T>((size_t)n * n);  // -S, X, H X, the reduced matrix
    b.take<T>((size_t)n * nev);                               // its eigenvectors
    b.take<double>(n);                                        // eigenvalues of -S
    size_t rest = eigh_ws_bytes<T>(n, n, pick_band(h, n), h->leaf_opt, 0);
    for (int bb : {8, 16, 32, 64}) rest = std::max(rest, eigh_ws_bytes<T>(n, nev, bb, h->leaf_opt, 0));
    return b.off + 256 + rest;
}

// The paper's route for an ill-conditioned S (end of its section on the
// reduction): diagonalise S, omit the eigenvectors with sigma_i < delta,
// solve the standard problem of X^H H X in the basis X = D_r sigma_r^(-1/2)
// of the m retained ones, and map back, C = X c~.  The eigenvectors of S
// come from the standard solver applied to -S, so that the largest sigma are
// the smallest eigenvalues and only the m retained vectors are formed.
template <typename T>
int do_solve_reduced(gevd_ctx* h, int n, int nev, double delta, T* H, int ldh, const T* S, int lds, double* eval,
                     T* C, int ldc, int* m_out, double* sigma_out) {
    int rc = ensure_ws(h, plan_reduced<T>(h, n, nev));
    if (rc) return rc;
    Bump b(h->ws);
    T* W = b.take<T>((size_t)n * n);
    T* X = b.take<T>((size_t)n * n);
    T* HX = b.take<T>((size_t)n * n);
    T* At = b.take<T>((size_t)n * n);
    T* Zt = b.take<T>((size_t)n * nev);
    double* evs = b.take<double>(n);
    char* rest = reinterpret_cast<char*>(b.take<char>(0));
    if ((rc = clear_flags(h))) return rc;
    if ((rc = check_finite_upper<T>(h->stream, n, H, ldh, h->flags + F_NONFINITE))) return rc;
    if ((rc = check_finite_upper<T>(h->stream, n, S, lds, h->flags + F_NONFINITE))) return rc;
    int fl[NFLAGS];
    if ((rc = read_flags(h, fl))) return rc;
    if (fl[F_NONFINITE]) return GEVD_E_NONFINITE;
    if ((rc = copy_matrix<T>(h->stream, n, n, S, lds, W, n))) return rc;
    if ((rc = fill_lower_from_upper<T>(h->stream, n, W, n))) return rc;
    if ((rc = negate_matrix<T>(h->stream, n, n, W, n))) return rc;
    StageCtx sc{h->stream, h->flags + F_NOCONV, h->flags + F_HANG, pick_band(h, n), h->leaf_opt};
    attach_aux(h, sc);
    int m = 0;
    if ((rc = eigh_select_run<T>(sc, n, -delta, W, n, evs, X, n, rest, &m))) return rc;
    if (sigma_out && (rc = negate_reverse(h->stream, n, evs, sigma_out))) return rc;
    if (m_out) *m_out = m;
    if (m < nev) {
        GEVD_HIP(hipStreamSynchronize(h->stream));
        return GEVD_E_RANK;
    }
    const T one = from_real<T>(1.0), zero = zero_of<T>();
    if ((rc = scale_cols_rsqrt_neg<T>(h->stream, n, m, X, n, evs))) return rc;
    if ((rc = fill_lower_from_upper<T>(h->stream, n, H, ldh))) return rc;
    if ((rc = gemm<T>(h->stream, OP_N, OP_N, n, m, n, one, H, ldh, X, n, zero, HX, n))) return rc;
    if ((rc = gemm<T>(h->stream, OP_C, OP_N, m, m, n, one, X, n, HX, n, zero, At, m, K_FULL, T_UPPER_TILES)))
        return rc;
    if ((rc = fill_lower_from_upper<T>(h->stream, m, At, m))) return rc;
    StageCtx sc2{h->stream, h->flags + F_NOCONV, h->flags + F_HANG, pick_band(h, m), h->leaf_opt};
    attach_aux(h, sc2);
    if ((rc = eigh_run<T>(sc2, m, nev, At, m, eval, Zt, m, rest))) return rc;
    if ((rc = gemm<T>(h->stream, OP_N, OP_N, n, nev, m, one, X, n, Zt, m, zero, C, ldc))) return rc;
    if ((rc = read_flags(h, fl))) return rc;
    if (fl[F_HANG]) return GEVD_E_HANG;
    if (fl[F_NOCONV]) return GEVD_E_NOCONV;
    if (h->kstats_on) h->ks.settle();
    return 0;
}

// ------------------------------------------------------------ density matrix
// P_ij = sum_l f_l conj(c_li) c_lj (the paper's density matrix, c_l the l-th
// eigenvector, i.e. column l of C): with B = conj(C) (n x k) and G = B F,
// P = G B^H.  Only the upper tiles are multiplied; the lower triangle is the
// Hermitian mirror.  Q (energy-weighted) uses f_l eps_l.
template <typename T>
int do_density(gevd_ctx* h, int n, int k, const T* C, int ldc, const double* f, const double* e, T* P, int ldp,
               T* Q, int ldq) {
    const bool cx = is_cplx<T>::value;
    Bump plan(nullptr);
    plan.take<T>((size_t)n * k);
    if (cx) plan.take<T>((size_t)n * k);
    int rc = ensure_ws(h, plan.off + 256);
    if (rc) return rc;
    Bump b(h->ws);
    T* G = b.take<T>((size_t)n * k);
    T* B = cx ? b.take<T>((size_t)n * k) : const_cast<T*>(C);
    const long ldb = cx ? n : ldc;
    const T one = from_real<T>(1.0), zero = zero_of<T>();
    for (int pass = 0; pass < (Q ? 2 : 1); ++pass) {
        T* out = pass == 0 ? P : Q;
        const int ldo = pass == 0 ? ldp : ldq;
        if ((rc = conj_scale_cols<T>(h->stream, n, k, C, ldc, f, pass == 0 ? nullptr : e, G, n,
                                     (cx && pass == 0) ? B : nullptr, ldb)))
            return rc;
        if ((rc = gemm<T>(h->stream, OP_N, OP_C, n, n, k, one, G, n, B, ldb, zero, out, ldo, K_FULL, T_UPPER_TILES)))
            return rc;
        if ((rc = fill_lower_from_upper<T>(h->stream, n, out, ldo))) return rc;
    }
    return 0;
}

bool bad_dtype(int t) { return t != GEVD_REAL && t != GEVD_COMPLEX; }

}  // namespace

// ============================================================== C interface
extern "C" {

int gevd_create(gevd_handle* out, int device) {
    if (!out) return -1;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return -2;
    gevd_ctx* h = new (std::nothrow) gevd_ctx();
    if (!h) return GEVD_E_NOMEM;
    h->device = device;
    if (hipSetDevice(device) != hipSuccess || hipMalloc(&h->flags, NFLAGS * sizeof(int)) != hipSuccess) {
        delete h;
        return GEVD_E_HIP;
    }
    (void)hipMemset(h->flags, 0, NFLAGS * sizeof(int));
    if (hipMalloc(&h->dstat, 4 * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void**)&h->dhost, 4 * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        gevd_destroy(h);
        return GEVD_E_HIP;
    }
    h->na_desc = new (std::nothrow) SmallDesc[GEVD_NOALLOC_MAX_COUNT];
    h->na_ord = new (std::nothrow) int[GEVD_NOALLOC_MAX_COUNT];
    if (!h->na_desc || !h->na_ord) {
        gevd_destroy(h);
        return GEVD_E_NOMEM;
    }
    const int rc = noalloc_attach(device);
    if (rc) {
        gevd_destroy(h);
        return rc;
    }
    *out = h;
    return 0;
}

int gevd_destroy(gevd_handle h) {
    if (!h) return -1;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    if (h->aux) (void)hipStreamSynchronize(h->aux);
    if (h->aux_fork) (void)hipEventDestroy(h->aux_fork);
    if (h->aux_join) (void)hipEventDestroy(h->aux_join);
    if (h->aux) (void)hipStreamDestroy(h->aux);
    if (h->ws) (void)hipFree(h->ws);
    if (h->uinv) (void)hipFree(h->uinv);
    if (h->flags) (void)hipFree(h->flags);
    if (h->dstat) (void)hipFree(h->dstat);
    if (h->dhost) (void)hipHostFree(h->dhost);
    if (h->ev_made)
        for (auto& e : h->ev) (void)hipEventDestroy(e);
    for (auto& e : h->ks.pool) (void)hipEventDestroy(e);
    delete[] h->na_desc;
    delete[] h->na_ord;
    delete h;
    return 0;
}

int gevd_set_stream(gevd_handle h, void* stream) {
    if (!h) return -1;
    h->stream = reinterpret_cast<hipStream_t>(stream);
    return 0;
}

int gevd_set_option(gevd_handle h, int option, int value) {
    if (!h) return -1;
    switch (option) {
        case GEVD_OPT_BAND:
            if (value != 0 && (value < 8 || value > 64)) return -3;
            h->band_opt = value;
            return 0;
        case GEVD_OPT_TIMING:
            h->timing = value ? 1 : 0;
            if (h->timing && !h->ev_made) {
                (void)hipSetDevice(h->device);
                for (auto& e : h->ev)
                    if (hipEventCreate(&e) != hipSuccess) return GEVD_E_HIP;
                h->ev_made = true;
            }
            return 0;
        case GEVD_OPT_LEAF:
            if (value != 0 && (value < 4 || value > 64)) return -3;
            h->leaf_opt = value;
            return 0;
        case GEVD_OPT_KSTATS:
            h->kstats_on = value ? 1 : 0;
            return 0;
        case GEVD_OPT_PRECISION:
            if (value != GEVD_PREC_FP64 && value != GEVD_PREC_FP32_REFINE) return -3;
            h->prec = value;
            return 0;
        case GEVD_OPT_REFINE:
            if (value < 0 || value > 10) return -3;
            h->refine_iters = value;
            return 0;
        case GEVD_OPT_PANEL:
            if (value != 0 && value != 1) return -3;
            h->panel_persist = value;
            return 0;
        case GEVD_OPT_STAGES:
            if (value != 0 && value != 1 && value != 2) return -3;
            h->stages = value == 1 ? 1 : 2;
            return 0;
        case GEVD_OPT_GEMM_TILE:
            if (value < -1 || value > 8) return -3;
            h->gemm_tile = value;
            return 0;
        default:
            return -2;
    }
}

const char* gevd_strerror(int code) {
    if (code == 0) return "success";
    if (code > 0) return "S is not positive definite (leading minor reported by the return value)";
    switch (code) {
        case GEVD_E_NONFINITE: return "non-finite value in H or S";
        case GEVD_E_NOCONV: return "tridiagonal eigensolver did not converge";
        case GEVD_E_NOMEM: return "out of device memory";
        case GEVD_E_HIP: return "HIP runtime error";
        case GEVD_E_STATE: return "invalid call order";
        case GEVD_E_HANG: return "device-side wait exceeded its bound";
        case GEVD_E_RANK: return "fewer overlap eigenvectors retained than eigenpairs requested";
        case GEVD_E_SCRATCH:
            return "request exceeds the fixed scratch of the no-allocation entry point (too many problems)";
        default: return "invalid argument (the negated return value is its 1-based position)";
    }
}

size_t gevd_workspace_bytes(int dtype, int n, int nev) {
    if (bad_dtype(dtype) || n < 1 || nev < 1 || nev > n) return 0;
    gevd_ctx tmp;
    return dtype == GEVD_REAL ? plan_solve<double>(&tmp, n, nev) : plan_solve<zdouble>(&tmp, n, nev);
}

size_t gevd_handle_workspace_bytes(gevd_handle h, int dtype, int n, int nev) {
    if (!h || bad_dtype(dtype) || n < 1 || nev < 1 || nev > n) return 0;
    return dtype == GEVD_REAL ? plan_solve<double>(h, n, nev) : plan_solve<zdouble>(h, n, nev);
}

int gevd_solve(gevd_handle h, int dtype, int n, int nev, void* H, int ldh, void* S, int lds, double* eval, void* C,
               int ldc) {
    if (!h) return -1;
    if (bad_dtype(dtype)) return -2;
    if (n < 1) return -3;
    if (nev < 1 || nev > n) return -4;
    if (!H) return -5;
    if (ldh < n) return -6;
    if (!S) return -7;
    if (lds < n) return -8;
    if (!eval) return -9;
    if (!C) return -10;
    if (ldc < n) return -11;
    if (hipSetDevice(h->device) != hipSuccess) return GEVD_E_HIP;
    KScope kscope(h);
    PanelLease lease(h);
    h->warn = 0;
    h->kappa_lb = 0.0;
    if (dtype == GEVD_REAL)
        return do_solve<double>(h, n, nev, (double*)H, ldh, (double*)S, lds, eval, (double*)C, ldc);
    return do_solve<zdouble>(h, n, nev, (zdouble*)H, ldh, (zdouble*)S, lds, eval, (zdouble*)C, ldc);
}

int gevd_set_overlap(gevd_handle h, int dtype, int n, const void* S, int lds) {
    if (!h) return -1;
    if (bad_dtype(dtype)) return -2;
    if (n < 1) return -3;
    if (!S) return -4;
    if (lds < n) return -5;
    if (hipSetDevice(h->device) != hipSuccess) return GEVD_E_HIP;
    KScope kscope(h);
    h->warn = 0;
    h->kappa_lb = 0.0;
    return dtype == GEVD_REAL ? do_set_overlap<double>(h, n, (const double*)S, lds)
                              : do_set_overlap<zdouble>(h, n, (const zdouble*)S, lds);
}

int gevd_solve_resident(gevd_handle h, int nev, void* H, int ldh, double* eval, void* C, int ldc) {
    if (!h) return -1;
    if (h->res_n < 1) return GEVD_E_STATE;
    const int n = h->res_n;
    if (nev < 1 || nev > n) return -2;
    if (!H) return -3;
    if (ldh < n) return -4;
    if (!eval) return -5;
    if (!C) return -6;
    if (ldc < n) return -7;
    if (hipSetDevice(h->device) != hipSuccess) return GEVD_E_HIP;
    KScope kscope(h);
    PanelLease lease(h);
    return h->res_dtype == GEVD_REAL
               ? do_solve_resident<double>(h, nev, (double*)H, ldh, eval, (double*)C, ldc)
               : do_solve_resident<zdouble>(h, nev, (zdouble*)H, ldh, eval, (zdouble*)C, ldc);
}

int gevd_solve_reduced(gevd_handle h, int dtype, int n, int nev, double delta, void* H, int ldh, const void* S,
                       int lds, double* eval, void* C, int ldc, int* m, double* sigma) {
    if (!h) return -1;
    if (bad_dtype(dtype)) return -2;
    if (n < 1) return -3;
    if (nev < 1 || nev > n) return -4;
    if (!(delta > 0.0) || !std::isfinite(delta)) return -5;
    if (!H) return -6;
    if (ldh < n) return -7;
    if (!S) return -8;
    if (lds < n) return -9;
    if (!eval) return -10;
    if (!C) return -11;
    if (ldc < n) return -12;
    if (hipSetDevice(h->device) != hipSuccess) return GEVD_E_HIP;
    KScope kscope(h);
    PanelLease lease(h);
    if (dtype == GEVD_REAL)
        return do_solve_reduced<double>(h, n, nev, delta, (double*)H, ldh, (const double*)S, lds, eval, (double*)C,
                                        ldc, m, sigma);
    return do_solve_reduced<zdouble>(h, n, nev, delta, (zdouble*)H, ldh, (const zdouble*)S, lds, eval, (zdouble*)C,
                                     ldc, m, sigma);
}

int gevd_density(gevd_handle h, int dtype, int n, int k, const void* C, int ldc, const double* f, const double* eval,
                 void* P, int ldp, void* Q, int ldq) {
    if (!h) return -1;
    if (bad_dtype(dtype)) return -2;
    if (n < 1) return -3;
    if (k < 1 || k > n) return -4;
    if (!C) return -5;
    if (ldc < n) return -6;
    if (!f) return -7;
    if (Q && !eval) return -8;
    if (!P) return -9;
    if (ldp < n) return -10;
    if (Q && ldq < n) return -12;
    if (hipSetDevice(h->device) != hipSuccess) return GEVD_E_HIP;
    KScope kscope(h);
    return dtype == GEVD_REAL
               ? do_density<double>(h, n, k, (const double*)C, ldc, f, eval, (double*)P, ldp, (double*)Q, ldq)
               : do_density<zdouble>(h, n, k, (const zdouble*)C, ldc, f, eval, (zdouble*)P, ldp, (zdouble*)Q, ldq);
}

int gevd_get_warnings(gevd_handle h, double* kappa_lower) {
    if (!h) return -1;
    if (kappa_lower) *kappa_lower = h->kappa_lb;
    return h->warn;
}

int gevd_cholesky(gevd_handle h, int dtype, int n, void* S, int lds) {
    if (!h) return -1;
    if (bad_dtype(dtype)) return -2;
    if (n < 1) return -3;
    if (!S) return -4;
    if (lds < n) return -5;
    if (hipSetDevice(h->device) != hipSuccess) return GEVD_E_HIP;
    KScope kscope(h);
    int rc = ensure_ws(h, dtype == GEVD_REAL ? plan_cholesky<double>(n) : plan_cholesky<zdouble>(n));
    if (rc) return rc;
    if ((rc = clear_flags(h))) return rc;
    rc = dtype == GEVD_REAL ? do_cholesky<double>(h, n, (double*)S, lds, h->ws)
                            : do_cholesky<zdouble>(h, n, (zdouble*)S, lds, h->ws);
    if (rc) return rc;
    int fl[NFLAGS];
    if ((rc = read_flags(h, fl))) return rc;
    return fl[F_INFO];
}

int gevd_invert_upper(gevd_handle h, int dtype, int n, const void* U, int ldu, void* Uinv, int ldi) {
    if (!h) return -1;
    if (bad_dtype(dtype)) return -2;
    if (n < 1) return -3;
    if (!U) return -4;
    if (ldu < n) return -5;
    if (!Uinv) return -6;
    if (ldi < n) return -7;
    if (hipSetDevice(h->device) != hipSuccess) return GEVD_E_HIP;
    KScope kscope(h);
    int rc = ensure_ws(h, dtype == GEVD_REAL ? plan_invert<double>(n) : plan_invert<zdouble>(n));
    if (rc) return rc;
    return dtype == GEVD_REAL ? do_invert<double>(h, n, (const double*)U, ldu, (double*)Uinv, ldi, h->ws)
                              : do_invert<zdouble>(h, n, (const zdouble*)U, ldu, (zdouble*)Uinv, ldi, h->ws);
}

int gevd_reduce(gevd_handle h, int dtype, int n, void* H, int ldh, const void* Uinv, int ldi, void* A, int lda) {
    if (!h) return -1;
    if (bad_dtype(dtype)) return -2;
    if (n < 1) return -3;
    if (!H) return -4;
    if (ldh < n) return -5;
    if (!Uinv) return -6;
    if (ldi < n) return -7;
    if (!A) return -8;
    if (lda < n) return -9;
    if (hipSetDevice(h->device) != hipSuccess) return GEVD_E_HIP;
    KScope kscope(h);
    int rc = ensure_ws(h, dtype == GEVD_REAL ? plan_reduce<double>(n) : plan_reduce<zdouble>(n));
    if (rc) return rc;
    return dtype == GEVD_REAL
               ? do_reduce<double>(h, n, (double*)H, ldh, (const double*)Uinv, ldi, (double*)A, lda, h->ws)
               : do_reduce<zdouble>(h, n, (zdouble*)H, ldh, (const zdouble*)Uinv, ldi, (zdouble*)A, lda, h->ws);
}

int gevd_backtransform(gevd_handle h, int dtype, int n, int nev, const void* Uinv, int ldi, const void* Ct, int ldct,
                       void* C, int ldc) {
    if (!h) return -1;
    if (bad_dtype(dtype)) return -2;
    if (n < 1) return -3;
    if (nev < 1 || nev > n) return -4;
    if (!Uinv) return -5;
    if (ldi < n) return -6;
    if (!Ct) return -7;
    if (ldct < n) return -8;
    if (!C) return -9;
    if (ldc < n) return -10;
    if (hipSetDevice(h->device) != hipSuccess) return GEVD_E_HIP;
    KScope kscope(h);
    return dtype == GEVD_REAL
               ? do_backtransform<double>(h, n, nev, (const double*)Uinv, ldi, (const double*)Ct, ldct, (double*)C, ldc)
               : do_backtransform<zdouble>(h, n, nev, (const zdouble*)Uinv, ldi, (const zdouble*)Ct, ldct,
                                           (zdouble*)C, ldc);
}

int gevd_eigh(gevd_handle h, int dtype, int n, int nev, void* A, int lda, double* eval, void* Z, int ldz) {
    if (!h) return -1;
    if (bad_dtype(dtype)) return -2;
    if (n < 1) return -3;
    if (nev < 1 || nev > n) return -4;
    if (!A) return -5;
    if (lda < n) return -6;
    if (!eval) return -7;
    if (!Z) return -8;
    if (ldz < n) return -9;
    if (hipSetDevice(h->device) != hipSuccess) return GEVD_E_HIP;
    KScope kscope(h);
    PanelLease lease(h);
    int b = pick_band(h, n);
    size_t need = dtype == GEVD_REAL ? eigh_ws_bytes<double>(n, nev, b, h->leaf_opt, h->prec)
                                     : eigh_ws_bytes<zdouble>(n, nev, b, h->leaf_opt, h->prec);
    int rc = ensure_ws(h, need);
    if (rc) return rc;
    if ((rc = clear_flags(h))) return rc;
    h->ev_valid = false;
    mark(h, GEVD_PH_BAND);
    rc = dtype == GEVD_REAL ? do_eigh<double>(h, n, nev, (double*)A, lda, eval, (double*)Z, ldz, h->ws, true)
                            : do_eigh<zdouble>(h, n, nev, (zdouble*)A, lda, eval, (zdouble*)Z, ldz, h->ws, true);
    if (rc) return rc;
    mark(h, GEVD_PH_MULT);
    mark(h, GEVD_NPHASE);
    int fl[NFLAGS];
    if ((rc = read_flags(h, fl))) return rc;
    if (fl[F_HANG]) return GEVD_E_HANG;
    if (fl[F_NOCONV]) return GEVD_E_NOCONV;
    return 0;
}

int gevd_get_band(gevd_handle h, int dtype, int n) {
    if (!h) return -1;
    if (bad_dtype(dtype)) return -2;
    if (n < 1) return -3;
    return pick_band(h, n);
}

int gevd_band(gevd_handle h, int dtype, int n, void* A, int lda, void* Bd, int ldb) {
    if (!h) return -1;
    if (bad_dtype(dtype)) return -2;
    if (n < 1) return -3;
    if (!A) return -4;
    if (lda < n) return -5;
    if (!Bd) return -6;
    int b = pick_band(h, n);
    if (ldb < b + 1) return -7;
    if (hipSetDevice(h->device) != hipSuccess) return GEVD_E_HIP;
    KScope kscope(h);
    PanelLease lease(h);
    size_t need = dtype == GEVD_REAL ? band_ws_bytes<double>(n, b) : band_ws_bytes<zdouble>(n, b);
    int rc = ensure_ws(h, need);
    if (rc) return rc;
    StageCtx sc{h->stream, h->flags + F_NOCONV, h->flags + F_HANG, b, h->leaf_opt};
    attach_aux(h, sc);
    return dtype == GEVD_REAL ? band_run<double>(sc, n, (double*)A, lda, (double*)Bd, ldb, h->ws)
                              : band_run<zdouble>(sc, n, (zdouble*)A, lda, (zdouble*)Bd, ldb, h->ws);
}

int gevd_tridiagonalize(gevd_handle h, int dtype, int n, void* A, int lda, double* d, double* e) {
    if (!h) return -1;
    if (bad_dtype(dtype)) return -2;
    if (n < 1) return -3;
    if (!A) return -4;
    if (lda < n) return -5;
    if (!d) return -6;
    if (!e && n > 1) return -7;
    if (hipSetDevice(h->device) != hipSuccess) return GEVD_E_HIP;
    KScope kscope(h);
    PanelLease lease(h);
    int b = pick_band(h, n);
    size_t need = dtype == GEVD_REAL ? eigh_ws_bytes<double>(n, 1, b, h->leaf_opt)
                                     : eigh_ws_bytes<zdouble>(n, 1, b, h->leaf_opt);
    int rc = ensure_ws(h, need);
    if (rc) return rc;
    if ((rc = clear_flags(h))) return rc;
    StageCtx sc{h->stream, h->flags + F_NOCONV, h->flags + F_HANG, b, h->leaf_opt};
    attach_aux(h, sc);
    rc = dtype == GEVD_REAL ? tridiag_run<double>(sc, n, (double*)A, lda, d, e, h->ws)
                            : tridiag_run<zdouble>(sc, n, (zdouble*)A, lda, d, e, h->ws);
    if (rc) return rc;
    int fl[NFLAGS];
    if ((rc = read_flags(h, fl))) return rc;
    if (fl[F_HANG]) return GEVD_E_HANG;
    return 0;
}

int gevd_stedc(gevd_handle h, int n, int nev, const double* d, const double* e, double* eval, double* Z, int ldz) {
    if (!h) return -1;
    if (n < 1) return -2;
    if (nev < 1 || nev > n) return -3;
    if (!d) return -4;
    if (!e && n > 1) return -5;
    if (!eval) return -6;
    if (!Z) return -7;
    if (ldz < n) return -8;
    if (hipSetDevice(h->device) != hipSuccess) return GEVD_E_HIP;
    KScope kscope(h);
    int rc = ensure_ws(h, stedc_ws_bytes(n, nev, h->leaf_opt));
    if (rc) return rc;
    if ((rc = clear_flags(h))) return rc;
    StageCtx sc{h->stream, h->flags + F_NOCONV, h->flags + F_HANG, 0, h->leaf_opt};
    attach_aux(h, sc);
    rc = stedc_run(sc, n, nev, d, e, eval, Z, ldz, h->ws);
    if (rc) return rc;
    int fl[NFLAGS];
    if ((rc = read_flags(h, fl))) return rc;
    if (fl[F_NOCONV]) return GEVD_E_NOCONV;
    return 0;
}

int gevd_get_kernel_stats(gevd_handle h, int family, long long* launches, double* ms, double* flops) {
    if (!h) return -1;
    if (family < 0 || family >= GEVD_NKFAM) return -2;
    GEVD_HIP(hipSetDevice(h->device));
    GEVD_HIP(hipStreamSynchronize(h->stream));
    h->ks.settle();
    if (launches) *launches = h->ks.tot_n[family];
    if (ms) *ms = h->ks.tot_ms[family];
    if (flops) *flops = h->ks.tot_flops[family];
    return 0;
}

int gevd_reset_kernel_stats(gevd_handle h) {
    if (!h) return -1;
    GEVD_HIP(hipSetDevice(h->device));
    GEVD_HIP(hipStreamSynchronize(h->stream));
    h->ks.settle();
    h->ks.reset();
    return 0;
}

int gevd_get_timings(gevd_handle h, double* ms, int nphase) {
    if (!h) return -1;
    if (!ms) return -2;
    if (nphase < 1) return -3;
    if (!h->ev_valid) return GEVD_E_STATE;
    GEVD_HIP(hipEventSynchronize(h->ev[GEVD_NPHASE]));
    for (int p = 0; p < nphase && p < GEVD_NPHASE; ++p) {
        float t = 0.f;
        GEVD_HIP(hipEventElapsedTime(&t, h->ev[p], h->ev[p + 1]));
        ms[p] = t;
    }
    return 0;
}

}  // extern "C"
