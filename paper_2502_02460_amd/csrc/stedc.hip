// Symmetric tridiagonal eigenproblem by divide-and-conquer (Cuppen 1981;
// deflation after Dongarra and Sorensen 1987; eigenvector orthogonality by
// recomputing z from the computed roots, Gu and Eisenstat 1995).  This is the
// "Solve" step of the standard eigenproblem in the paper's Table 1.
//
// T = diag(T1, T2) + |beta| u u^T with u = e_last(T1) + sign(beta) e_first(T2)
// and beta the coupling entry; the two halves are solved recursively, then
// the merge solves D + rho z z^T (D the children's eigenvalues, z the last
// row of Q1 and sign(beta) times the first row of Q2, rho = 2|beta| with z
// normalised).  Leaves (<= leaf size) run an implicit QL iteration in one
// workgroup.  Per merge: small |z_i| and near-equal d_i (after a Givens
// rotation) deflate; each remaining root of the secular equation
// 1 + rho sum z_i^2/(d_i - lam) = 0 is found by bisection on lam - d_origin,
// the origin being the nearer pole, so differences d_i - lam keep full
// relative accuracy; the merged eigenvectors are Q_children * U, one MFMA
// product whose input columns are gathered and output columns scattered to
// their sorted positions.  At the root only the wanted columns are formed.
//
// All merges of one tree level run in the same launches; the host reads the
// number of non-deflated values once per level to size the products.
#include <algorithm>
#include <cmath>
#include <vector>

#include "stages.hpp"

namespace gevd {
namespace {

constexpr int MAXLEAF = 64;
constexpr double DEPS = 2.220446049250313e-16;

struct MergeDesc {
    int off, n1, n2, pin;  // range [off, off+n1+n2), children results in Z buffer pin
    long long uoff;        // offset of U (knd x knd) in the U buffer
    int knd, pad;
};

struct LeafDesc {
    int off, size, parity, pad;
};

// ------------------------------------------------------------------ leaves
__global__ __launch_bounds__(64) void leaf_kernel(int n, const double* d, const double* e, double* w, double* Z0,
                                                  double* Z1, const LeafDesc* leaves, int* noconv) {
    __shared__ double dd[MAXLEAF], ee[MAXLEAF], rc[MAXLEAF], rs[MAXLEAF];
    __shared__ double z[MAXLEAF][MAXLEAF + 1];
    __shared__ int perm[MAXLEAF];
    __shared__ int ctl[3];  // l, m, status
    const LeafDesc L = leaves[blockIdx.x];
    const int s = L.size, off = L.off, k = threadIdx.x;
    double* Z = L.parity ? Z1 : Z0;
    if (k < s) {
        double dv = d[off + k];
        if (k == 0 && off > 0) dv -= fabs(e[off - 1]);
        if (k == s - 1 && off + s < n) dv -= fabs(e[off + s - 1]);
        dd[k] = dv;
        ee[k] = (k < s - 1) ? e[off + k] : 0.0;
        for (int j = 0; j < s; ++j) z[k][j] = (j == k) ? 1.0 : 0.0;
    }
    __syncthreads();
    // implicit QL: thread 0 runs the scalar recurrence of one sweep and
    // records its rotations; all threads then rotate their row of z.
    for (int l = 0; l < s; ++l) {
        int iters = 0;
        for (;;) {
            if (k == 0) {
                int m = l;
                while (m < s - 1) {
                    const double sc = fabs(dd[m]) + fabs(dd[m + 1]);
                    if (fabs(ee[m]) <= DEPS * sc) break;
                    ++m;
                }
                ctl[0] = l;
                ctl[1] = m;
                ctl[2] = 0;
                if (m != l) {
                    if (++iters > 30) {
                        atomicOr(noconv, 1);
                        ctl[1] = l;  // give up on this eigenvalue
                    } else {
                        double g = (dd[l + 1] - dd[l]) / (2.0 * ee[l]);
                        double r = hypot(g, 1.0);
                        const double mu = dd[l] - ee[l] / (g + copysign(r, g));
                        double sn = 1.0, cs = 1.0, p = 0.0;
                        g = dd[m] - mu;
                        int i = m - 1, lo = l;
                        for (; i >= l; --i) {
                            const double f = sn * ee[i], bb = cs * ee[i];
                            r = hypot(f, g);
                            ee[i + 1] = r;
                            if (r == 0.0) {
                                dd[i + 1] -= p;
                                ee[m] = 0.0;
                                lo = i + 1;  // rotations i+1 .. m-1 were recorded
                                ctl[2] = 1;
                                break;
                            }
                            sn = f / r;
                            cs = g / r;
                            g = dd[i + 1] - p;
                            r = (dd[i] - g) * sn + 2.0 * cs * bb;
                            p = sn * r;
                            dd[i + 1] = g + p;
                            g = cs * r - bb;
                            rc[i] = cs;
                            rs[i] = sn;
                        }
                        if (!ctl[2]) {
                            dd[l] -= p;
                            ee[l] = g;
                            ee[m] = 0.0;
                        }
                        ctl[0] = lo;  // rotations lo .. m-1 to apply, descending
                    }
                }
            }
            __syncthreads();
            const int lo = ctl[0], m = ctl[1];
            if (m == lo && !ctl[2]) break;  // converged (or gave up)
            if (k < s) {
                for (int i = m - 1; i >= lo; --i) {
                    const double a = z[k][i], b = z[k][i + 1];
                    z[k][i + 1] = rs[i] * a + rc[i] * b;
                    z[k][i] = rc[i] * a - rs[i] * b;
                }
            }
            __syncthreads();
        }
        __syncthreads();
    }
    // ascending order
    if (k == 0) {
        for (int i = 0; i < s; ++i) perm[i] = i;
        for (int i = 0; i < s - 1; ++i) {
            int kmin = i;
            for (int j = i + 1; j < s; ++j)
                if (dd[perm[j]] < dd[perm[kmin]]) kmin = j;
            const int t = perm[i];
            perm[i] = perm[kmin];
            perm[kmin] = t;
        }
    }
    __syncthreads();
    if (k < s) {
        w[off + k] = dd[perm[k]];
        for (int j = 0; j < s; ++j) Z[IDX(off + k, off + j, n)] = z[k][perm[j]];
    }
}

// --------------------------------------------------------------- merge steps
// Off-diagonal blocks of the children's block-diagonal eigenvector matrix.
__global__ void merge_zero_kernel(int n, double* Z0, double* Z1, const MergeDesc* md) {
    const MergeDesc M = md[blockIdx.y];
    double* Z = M.pin ? Z1 : Z0;
    const long long tot = 2LL * M.n1 * M.n2;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
         idx += (long long)gridDim.x * blockDim.x) {
        long long h = idx / 2;
        if ((idx & 1) == 0) {  // rows of child 1, columns of child 2
            const int r = (int)(h % M.n1), c = (int)(h / M.n1);
            Z[IDX(M.off + r, M.off + M.n1 + c, n)] = 0.0;
        } else {  // rows of child 2, columns of child 1
            const int r = (int)(h % M.n2), c = (int)(h / M.n2);
            Z[IDX(M.off + M.n1 + r, M.off + c, n)] = 0.0;
        }
    }
}

// Merge the children's sorted eigenvalue lists (ties: child 1 first) and
// gather z.  dsrt/zsrt/perm are indexed off + sorted position.
__global__ void merge_prep_kernel(int n, const double* e, const double* w, const double* Z0, const double* Z1,
                                  const MergeDesc* md, double* dsrt, double* zsrt, int* perm) {
    const MergeDesc M = md[blockIdx.y];
    const double* Z = M.pin ? Z1 : Z0;
    const int K = M.n1 + M.n2, off = M.off;
    const double sg = e[off + M.n1 - 1] >= 0.0 ? 1.0 : -1.0;
    const double is2 = 0.70710678118654752440;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < K; i += gridDim.x * blockDim.x) {
        double dv, zv;
        int pos;
        if (i < M.n1) {
            dv = w[off + i];
            zv = Z[IDX(off + M.n1 - 1, off + i, n)] * is2;
            int lo = 0, hi = M.n2;  // count of child-2 values < dv
            while (lo < hi) {
                const int mid = (lo + hi) / 2;
                if (w[off + M.n1 + mid] < dv) lo = mid + 1;
                else hi = mid;
            }
            pos = i + lo;
        } else {
            const int i2 = i - M.n1;
            dv = w[off + i];
            zv = sg * Z[IDX(off + M.n1, off + i, n)] * is2;
            int lo = 0, hi = M.n1;  // count of child-1 values <= dv
            while (lo < hi) {
                const int mid = (lo + hi) / 2;
                if (w[off + mid] <= dv) lo = mid + 1;
                else hi = mid;
            }
            pos = i2 + lo;
        }
        dsrt[off + pos] = dv;
        zsrt[off + pos] = zv;
        perm[off + pos] = i;
    }
}

// Deflation scan (one thread per merge): small rho|z_i| deflate directly;
// a value close to the previous kept one is rotated into it (Givens on
// (z_prev, z_q)) and deflates.  Produces the kept list (delta, zc, ndl),
// the deflated list (dval, dfl) and the rotations applied to the columns.
__global__ void merge_deflate_kernel(const double* e, const MergeDesc* md, int nm, double* dsrt, double* zsrt,
                                     int* flag, int* ndl, double* delta, double* zc, int* dfl, double* dval,
                                     int* rq1, int* rq2, double* rcs, double* rsn, int* counts) {
    const int mi = blockIdx.x * blockDim.x + threadIdx.x;
    if (mi >= nm) return;
    const MergeDesc M = md[mi];
    const int K = M.n1 + M.n2, off = M.off;
    const double rho = 2.0 * fabs(e[off + M.n1 - 1]);
    double* d = dsrt + off;
    double* z = zsrt + off;
    const double dmax = fmax(fabs(d[0]), fabs(d[K - 1]));
    const double tol = 8.0 * DEPS * fmax(dmax, rho);
    // The previous kept entry stays in registers (zp, dp); the next entry is
    // loaded one step ahead.  |t c s| <= tol is evaluated exactly (hypot and
    // divisions) only when the division-free |t zq zp| <= 2 tol (zp^2 + zq^2)
    // admits it: beyond that bound the exact test fails too, so the
    // decisions are those of the exact test alone.
    int prev = -1, nrot = 0;
    double zp = 0.0, dp = 0.0;
    double zn = K > 0 ? z[0] : 0.0, dn = K > 0 ? d[0] : 0.0;
    for (int q = 0; q < K; ++q) {
        double zq = zn, dq = dn;
        if (q + 1 < K) {
            zn = z[q + 1];
            dn = d[q + 1];
        }
        flag[off + q] = 0;
        if (rho * fabs(zq) <= tol) {
            flag[off + q] = 1;
            continue;
        }
        if (prev >= 0) {
            const double t = dq - dp;
            if (fabs(t * zq * zp) <= 2.0 * tol * (zp * zp + zq * zq)) {
                const double tau = hypot(zp, zq);
                const double c = zq / tau, s = zp / tau;
                if (fabs(t * c * s) <= tol) {
                    z[q] = tau;
                    z[prev] = 0.0;
                    const double dpn = c * c * dp + s * s * dq;
                    const double dqn = s * s * dp + c * c * dq;
                    d[prev] = dpn;
                    d[q] = dqn;
                    zq = tau;
                    dq = dqn;
                    rq1[off + nrot] = prev;
                    rq2[off + nrot] = q;
                    rcs[off + nrot] = c;
                    rsn[off + nrot] = s;
                    ++nrot;
                    flag[off + prev] = 1;
                }
            }
        }
        prev = q;
        zp = zq;
        dp = dq;
    }
    int kn = 0, kd = 0;
    for (int q = 0; q < K; ++q) {
        if (flag[off + q]) {
            dfl[off + kd] = q;
            dval[off + kd] = d[q];
            ++kd;
        } else {
            ndl[off + kn] = q;
            delta[off + kn] = d[q];
            zc[off + kn] = z[q];
            ++kn;
        }
    }
    counts[2 * mi] = kn;
    counts[2 * mi + 1] = nrot;
}

// Apply the recorded rotations to the children's eigenvector columns; each
// thread owns one row of the merge range.
__global__ void merge_rotate_kernel(int n, double* Z0, double* Z1, const MergeDesc* md, const int* perm,
                                    const int* rq1, const int* rq2, const double* rcs, const double* rsn,
                                    const int* counts) {
    const MergeDesc M = md[blockIdx.y];
    double* Z = M.pin ? Z1 : Z0;
    const int K = M.n1 + M.n2, off = M.off;
    const int nrot = counts[2 * blockIdx.y + 1];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= K || nrot == 0) return;
    for (int k = 0; k < nrot; ++k) {
        const int cp = off + perm[off + rq1[off + k]], cq = off + perm[off + rq2[off + k]];
        const double c = rcs[off + k], s = rsn[off + k];
        const double a = Z[IDX(off + r, cp, n)], b = Z[IDX(off + r, cq, n)];
        Z[IDX(off + r, cp, n)] = c * a - s * b;
        Z[IDX(off + r, cq, n)] = s * a + c * b;
    }
}

// Each root is found by SG consecutive lanes: lane q of the group takes the
// terms i = q, q + SG, ... of every sum over the poles, and the group adds
// its partial sums by exchanges (xor butterfly: every lane ends with the same
// bits, so the group follows one control path).
constexpr int SG = 8;
__device__ inline double group_sum(double v) {
#pragma unroll
    for (int m = 1; m < SG; m *= 2) v += __shfl_xor(v, m, WAVE);
    return v;
}

// f(origin + tau) for the secular equation, differences taken from the origin.
__device__ inline double secular(const double* delta, const double* zc, int kn, double rho, double dorg, double tau,
                                 int q) {
    double f = 0.0;
    for (int i = q; i < kn; i += SG) f += rho * zc[i] * zc[i] / ((delta[i] - dorg) - tau);
    return 1.0 + group_sum(f);
}

// Root j of 1 + rho sum_i z_i^2/(delta_i - lam), lam = delta[o] + tau with o
// the nearer pole.  Each iteration evaluates the poles left of the interval
// (psi) and right of it (phi) with their derivatives, replaces them by one
// pole each with matching value and slope (a two-pole rational model; for
// the last root one pole), and steps to the model's root in the interval.
// The sign of f keeps a bracket; a model step that leaves it is replaced by
// bisection, so convergence never depends on the model.
constexpr int SECT = 128;  // threads per workgroup (SECT / SG roots)
__global__ __launch_bounds__(SECT) void merge_secular_kernel(const double* e, const MergeDesc* md,
                                                             const double* delta_all, const double* zc_all, int* org,
                                                             double* tauv, double* lam) {
    const MergeDesc M = md[blockIdx.y];
    const int kn = M.knd, off = M.off;
    const int q = threadIdx.x % SG;
    const int j = (blockIdx.x * SECT + threadIdx.x) / SG;
    if (j >= kn) return;  // whole groups leave together
    const double rho = 2.0 * fabs(e[off + M.n1 - 1]);
    const double* delta = delta_all + off;
    const double* zc = zc_all + off;
    const bool last = j == kn - 1;
    int o;
    double lo, hi;
    if (!last) {
        const double gap = delta[j + 1] - delta[j];
        const double fm = secular(delta, zc, kn, rho, delta[j], 0.5 * gap, q);
        if (fm >= 0.0) {
            o = j;
            lo = 0.0;
            hi = 0.5 * gap;
        } else {
            o = j + 1;
            lo = -0.5 * gap;
            hi = 0.0;
        }
    } else {
        double zz = 0.0;
        for (int i = q; i < kn; i += SG) zz += zc[i] * zc[i];
        zz = group_sum(zz);
        o = j;
        lo = 0.0;
        hi = rho * zz;
        for (int g = 0; g < 64 && secular(delta, zc, kn, rho, delta[o], hi, q) < 0.0; ++g) hi *= 2.0;
    }
    const double dorg = delta[o];
    double tau = 0.5 * (lo + hi);
    for (int it = 0; it < 100; ++it) {
        double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
        for (int i = q; i <= j; i += SG) {
            const double r = zc[i] / ((delta[i] - dorg) - tau);
            psi += zc[i] * r;
            dpsi += r * r;
        }
        for (int i = j + 1 + q; i < kn; i += SG) {
            const double r = zc[i] / ((delta[i] - dorg) - tau);
            phi += zc[i] * r;
            dphi += r * r;
        }
        psi = rho * group_sum(psi);
        dpsi = rho * group_sum(dpsi);
        phi = rho * group_sum(phi);
        dphi = rho * group_sum(dphi);
        const double f = 1.0 + psi + phi;
        if (f == 0.0) break;
        // below this the sign of the computed f is not meaningful
        if (fabs(f) <= 8.0 * DEPS * (1.0 + fabs(psi) + fabs(phi))) break;
        if (f < 0.0) lo = tau;
        else hi = tau;
        if (hi - lo <= 4.0 * DEPS * fmax(fabs(lo), fabs(hi))) break;
        // model: c + s/(D1 - y) + S/(D2 - y) = 0 for the step y from tau
        const double D1 = (delta[j] - dorg) - tau;
        double y;
        bool ok = true;
        if (!last) {
            const double D2 = (delta[j + 1] - dorg) - tau;
            const double sl = dpsi * D1 * D1, sr = dphi * D2 * D2;
            const double c = f - dpsi * D1 - dphi * D2;
            const double bq = c * (D1 + D2) + sl + sr;
            const double cq = c * D1 * D2 + sl * D2 + sr * D1;
            if (c == 0.0) {
                y = cq / bq;
            } else {
                const double disc = bq * bq - 4.0 * c * cq;
                if (disc < 0.0) {
                    ok = false;
                    y = 0.0;
                } else {
                    const double qq = 0.5 * (bq + copysign(sqrt(disc), bq));
                    const double y1 = qq / c, y2 = (qq != 0.0) ? cq / qq : y1;
                    y = (y1 > D1 && y1 < D2) ? y1 : y2;
                }
            }
        } else {
            const double sl = dpsi * D1 * D1;
            const double c = f - dpsi * D1;
            ok = c > 0.0;
            y = ok ? D1 + sl / c : 0.0;
        }
        double tn = tau + y;
        if (!ok || !(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (fabs(tn - tau) <= 2.0 * DEPS * fabs(tn)) {
            tau = tn;
            break;
        }
        tau = tn;
    }
    if (q == 0) {
        org[off + j] = o;
        tauv[off + j] = tau;
        lam[off + j] = dorg + tau;
    }
}

// z recomputed from the roots (Gu-Eisenstat), products arranged as ratios
// of comparable size.
__global__ void merge_zhat_kernel(const double* e, const MergeDesc* md, const double* delta_all, const double* zc_all,
                                  const int* org_all, const double* tau_all, double* zhat) {
    const MergeDesc M = md[blockIdx.y];
    const int kn = M.knd, off = M.off;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kn) return;
    const double rho = 2.0 * fabs(e[off + M.n1 - 1]);
    const double* delta = delta_all + off;
    const int* org = org_all + off;
    const double* tau = tau_all + off;
    const double di = delta[i];
    auto lam_minus = [&](int j) { return (delta[org[j]] - di) + tau[j]; };
    double p = lam_minus(kn - 1) / rho;
    for (int j = 0; j < i; ++j) p *= lam_minus(j) / (delta[j] - di);
    for (int j = i; j < kn - 1; ++j) p *= lam_minus(j) / (delta[j + 1] - di);
    zhat[off + i] = copysign(sqrt(fmax(p, 0.0)), zc_all[off + i]);
}

// Final positions of all K merged values, eigenvalues written to w, and the
// column maps of the merge product.  Keys (value, kind, index) break ties.
__global__ void merge_pos_kernel(const MergeDesc* md, const double* lam_all, const double* dval_all,
                                 const int* dfl_all, const int* ndl_all, const int* perm_all, double* w, int* posL,
                                 int* posD, int* amap, int* cmap, int root, int nev) {
    const MergeDesc M = md[blockIdx.y];
    const int K = M.n1 + M.n2, kn = M.knd, off = M.off;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= K) return;
    const bool isl = x < kn;
    const int idx = isl ? x : x - kn;
    const double v = isl ? lam_all[off + idx] : dval_all[off + idx];
    int rank = 0;
    for (int j = 0; j < kn; ++j) {
        const double u = lam_all[off + j];
        rank += (u < v) || (u == v && (isl ? j < idx : true));
    }
    for (int c = 0; c < K - kn; ++c) {
        const double u = dval_all[off + c];
        rank += (u < v) || (u == v && (!isl && c < idx));
    }
    w[off + rank] = v;
    if (isl) {
        posL[off + idx] = rank;
        amap[off + idx] = off + perm_all[off + ndl_all[off + idx]];
        cmap[off + idx] = root ? (rank < nev ? rank : -1) : off + rank;
    } else {
        posD[off + idx] = rank;
    }
}

// Column j of U: zhat_i / (delta_i - lam_j), normalised.
__global__ __launch_bounds__(256) void merge_vec_kernel(const MergeDesc* md, const double* delta_all,
                                                        const int* org_all, const double* tau_all,
                                                        const double* zhat_all, double* Ubuf) {
    __shared__ double red[4];
    const MergeDesc M = md[blockIdx.y];
    const int kn = M.knd, off = M.off;
    const int j = blockIdx.x;
    if (j >= kn) return;
    const double* delta = delta_all + off;
    const double dorg = delta[org_all[off + j]], tj = tau_all[off + j];
    double* U = Ubuf + M.uoff + (size_t)j * kn;
    double ss = 0.0;
    for (int i = threadIdx.x; i < kn; i += 256) {
        const double u = zhat_all[off + i] / ((delta[i] - dorg) - tj);
        U[i] = u;
        ss += u * u;
    }
    ss = block_sum<256>(ss, red);
    const double inv = 1.0 / sqrt(ss);
    for (int i = threadIdx.x; i < kn; i += 256) U[i] *= inv;
}

// Deflated eigenvectors: copied (rotated) columns of the children's matrix.
__global__ void merge_defl_copy_kernel(int n, const double* Z0, const double* Z1, double* O0, double* O1,
                                       const MergeDesc* md, const int* perm_all, const int* dfl_all,
                                       const int* posD_all, int root, int nev, double* Zroot, long ldz) {
    const MergeDesc M = md[blockIdx.z];
    const int K = M.n1 + M.n2, kn = M.knd, off = M.off;
    const int c = blockIdx.y;
    if (c >= K - kn) return;
    const double* Zi = M.pin ? Z1 : Z0;
    double* Zo = M.pin ? O0 : O1;  // the other buffer
    const int pos = posD_all[off + c];
    if (root && pos >= nev) return;
    const int src = off + perm_all[off + dfl_all[off + c]];
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < K; r += gridDim.x * blockDim.x) {
        const double v = Zi[IDX(off + r, src, n)];
        if (root) Zroot[IDX(r, pos, ldz)] = v;
        else Zo[IDX(off + r, off + pos, n)] = v;
    }
}

__global__ void copy_cols_kernel(int n, int nev, const double* Zs, double* Z, long ldz) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * nev) return;
    const int r = (int)(idx % n), c = (int)(idx / n);
    Z[IDX(r, c, ldz)] = Zs[IDX(r, c, n)];
}

struct TreeNode {
    int off, size, depth;
    bool leaf;
};

void build_tree(int off, int size, int depth, int leaf, std::vector<TreeNode>& out) {
    if (size <= leaf) {
        out.push_back({off, size, depth, true});
        return;
    }
    out.push_back({off, size, depth, false});
    const int n1 = size / 2;
    build_tree(off, n1, depth + 1, leaf, out);
    build_tree(off + n1, size - n1, depth + 1, leaf, out);
}

int leaf_size(int leaf_opt) { return leaf_opt > 0 ? std::min(leaf_opt, MAXLEAF) : 32; }

struct DcWs {
    double *Z0, *Z1, *U, *dsrt, *zsrt, *delta, *zc, *dval, *rcs, *rsn, *tauv, *lam, *zhat;
    int *perm, *flag, *ndl, *dfl, *rq1, *rq2, *org, *posL, *posD, *amap, *cmap, *counts;
    MergeDesc* md;
    LeafDesc* ld;
};

size_t carve_dc(char* base, int n, int leaf, DcWs* w) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        off = (off + 255) & ~size_t(255);
        char* r = base ? base + off : nullptr;
        off += bytes;
        return r;
    };
    const size_t nn = (size_t)n * n, nd = (size_t)n * sizeof(double), ni = (size_t)n * sizeof(int);
    const int nleaf_max = n / 1 + 1;
    DcWs t;
    t.Z0 = (double*)take(nn * sizeof(double));
    t.Z1 = (double*)take(nn * sizeof(double));
    t.U = (double*)take(nn * sizeof(double));
    t.dsrt = (double*)take(nd);
    t.zsrt = (double*)take(nd);
    t.delta = (double*)take(nd);
    t.zc = (double*)take(nd);
    t.dval = (double*)take(nd);
    t.rcs = (double*)take(nd);
    t.rsn = (double*)take(nd);
    t.tauv = (double*)take(nd);
    t.lam = (double*)take(nd);
    t.zhat = (double*)take(nd);
    t.perm = (int*)take(ni);
    t.flag = (int*)take(ni);
    t.ndl = (int*)take(ni);
    t.dfl = (int*)take(ni);
    t.rq1 = (int*)take(ni);
    t.rq2 = (int*)take(ni);
    t.org = (int*)take(ni);
    t.posL = (int*)take(ni);
    t.posD = (int*)take(ni);
    t.amap = (int*)take(ni);
    t.cmap = (int*)take(ni);
    t.counts = (int*)take(2 * ni + 64);
    t.md = (MergeDesc*)take(sizeof(MergeDesc) * (size_t)(n + 1));
    t.ld = (LeafDesc*)take(sizeof(LeafDesc) * (size_t)nleaf_max);
    (void)leaf;
    if (w) *w = t;
    return off;
}

}  // namespace

size_t stedc_ws_bytes(int n, int nev, int leaf) {
    (void)nev;
    return carve_dc(nullptr, n, leaf_size(leaf), nullptr) + 256;
}

int stedc_run(const StageCtx& c, int n, int nev, const double* d, const double* e, double* eval, double* Z, long ldz,
              char* ws) {
    hipStream_t st = c.st;
    const int leaf = leaf_size(c.leaf);
    DcWs w;
    carve_dc(ws, n, leaf, &w);
    std::vector<TreeNode> nodes;
    build_tree(0, n, 0, leaf, nodes);
    int maxdepth = 0;
    std::vector<LeafDesc> leaves;
    for (auto& t : nodes) {
        maxdepth = std::max(maxdepth, t.depth);
        if (t.leaf) leaves.push_back({t.off, t.size, t.depth % 2, 0});
    }
    GEVD_HIP(hipMemcpyAsync(w.ld, leaves.data(), sizeof(LeafDesc) * leaves.size(), hipMemcpyHostToDevice, st));
    {
            KProbe kp_(st, GEVD_K_DC, 0.0);
            hipLaunchKernelGGL(leaf_kernel, dim3((unsigned)leaves.size()), dim3(64), 0, st, n, d, e, eval, w.Z0, w.Z1,
                       (const LeafDesc*)w.ld, c.noconv);
    GEVD_LAUNCH_CHECK();
        }
    if (nodes.size() == 1) {  // a single leaf: parity 0
        const long long tot = (long long)n * nev;
        {
            KProbe kp_(st, GEVD_K_DC, 0.0);
            hipLaunchKernelGGL(copy_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, nev,
                           (const double*)w.Z0, Z, ldz);
        GEVD_LAUNCH_CHECK();
        }
        return 0;
    }
    std::vector<MergeDesc> md;
    std::vector<int> counts;
    for (int dep = maxdepth - 1; dep >= 0; --dep) {
        md.clear();
        int maxK = 0, maxn12 = 0;
        for (auto& t : nodes)
            if (!t.leaf && t.depth == dep) {
                MergeDesc m{};
                m.off = t.off;
                m.n1 = t.size / 2;
                m.n2 = t.size - m.n1;
                m.pin = (dep + 1) % 2;
                md.push_back(m);
                maxK = std::max(maxK, t.size);
                maxn12 = std::max(maxn12, m.n1 * m.n2);
            }
        const int nm = (int)md.size();
        if (nm == 0) continue;
        const bool root = dep == 0;
        GEVD_HIP(hipMemcpyAsync(w.md, md.data(), sizeof(MergeDesc) * nm, hipMemcpyHostToDevice, st));
        {
            const long long tot = 2LL * maxn12;
            const unsigned gx = (unsigned)std::min<long long>((tot + 255) / 256, 4096);
            {
            KProbe kp_(st, GEVD_K_DC, 0.0);
            hipLaunchKernelGGL(merge_zero_kernel, dim3(gx, nm), dim3(256), 0, st, n, w.Z0, w.Z1,
                               (const MergeDesc*)w.md);
            GEVD_LAUNCH_CHECK();
        }
        }
        const unsigned gK = (unsigned)((maxK + 255) / 256);
        {
            KProbe kp_(st, GEVD_K_DC, 0.0);
            hipLaunchKernelGGL(merge_prep_kernel, dim3(gK, nm), dim3(256), 0, st, n, e, (const double*)eval,
                           (const double*)w.Z0, (const double*)w.Z1, (const MergeDesc*)w.md, w.dsrt, w.zsrt, w.perm);
        GEVD_LAUNCH_CHECK();
        }
        {
            KProbe kp_(st, GEVD_K_DC, 0.0);
            hipLaunchKernelGGL(merge_deflate_kernel, dim3((nm + 63) / 64), dim3(64), 0, st, e, (const MergeDesc*)w.md, nm,
                           w.dsrt, w.zsrt, w.flag, w.ndl, w.delta, w.zc, w.dfl, w.dval, w.rq1, w.rq2, w.rcs, w.rsn,
                           w.counts);
        GEVD_LAUNCH_CHECK();
        }
        {
            KProbe kp_(st, GEVD_K_DC, 0.0);
            hipLaunchKernelGGL(merge_rotate_kernel, dim3(gK, nm), dim3(256), 0, st, n, w.Z0, w.Z1,
                           (const MergeDesc*)w.md, (const int*)w.perm, (const int*)w.rq1, (const int*)w.rq2,
                           (const double*)w.rcs, (const double*)w.rsn, (const int*)w.counts);
        GEVD_LAUNCH_CHECK();
        }
        counts.resize(2 * nm);
        GEVD_HIP(hipMemcpyAsync(counts.data(), w.counts, sizeof(int) * 2 * nm, hipMemcpyDeviceToHost, st));
        GEVD_HIP(hipStreamSynchronize(st));
        long long uoff = 0;
        int maxkn = 0;
        for (int i = 0; i < nm; ++i) {
            md[i].knd = counts[2 * i];
            md[i].uoff = uoff;
            uoff += (long long)md[i].knd * md[i].knd;
            maxkn = std::max(maxkn, md[i].knd);
        }
        GEVD_HIP(hipMemcpyAsync(w.md, md.data(), sizeof(MergeDesc) * nm, hipMemcpyHostToDevice, st));
        if (maxkn > 0) {
            const unsigned gk = (unsigned)((maxkn + 127) / 128);
            {
            KProbe kp_(st, GEVD_K_DC, 0.0);
            const unsigned gs = (unsigned)(((long long)maxkn * SG + SECT - 1) / SECT);
            hipLaunchKernelGGL(merge_secular_kernel, dim3(gs, nm), dim3(SECT), 0, st, e, (const MergeDesc*)w.md,
                               (const double*)w.delta, (const double*)w.zc, w.org, w.tauv, w.lam);
            GEVD_LAUNCH_CHECK();
        }
            {
            KProbe kp_(st, GEVD_K_DC, 0.0);
            hipLaunchKernelGGL(merge_zhat_kernel, dim3(gk, nm), dim3(128), 0, st, e, (const MergeDesc*)w.md,
                               (const double*)w.delta, (const double*)w.zc, (const int*)w.org,
                               (const double*)w.tauv, w.zhat);
            GEVD_LAUNCH_CHECK();
        }
        }
        {
            KProbe kp_(st, GEVD_K_DC, 0.0);
            hipLaunchKernelGGL(merge_pos_kernel, dim3(gK, nm), dim3(256), 0, st, (const MergeDesc*)w.md,
                           (const double*)w.lam, (const double*)w.dval, (const int*)w.dfl, (const int*)w.ndl,
                           (const int*)w.perm, eval, w.posL, w.posD, w.amap, w.cmap, root ? 1 : 0, nev);
        GEVD_LAUNCH_CHECK();
        }
        if (maxkn > 0) {
            {
            KProbe kp_(st, GEVD_K_DC, 0.0);
            hipLaunchKernelGGL(merge_vec_kernel, dim3(maxkn, nm), dim3(256), 0, st, (const MergeDesc*)w.md,
                               (const double*)w.delta, (const int*)w.org, (const double*)w.tauv,
                               (const double*)w.zhat, w.U);
            GEVD_LAUNCH_CHECK();
        }
        }
        // number of wanted merge-product columns at the root
        std::vector<int> posL;
        if (root && md[0].knd > 0) {
            posL.resize(md[0].knd);
            GEVD_HIP(hipMemcpyAsync(posL.data(), w.posL, sizeof(int) * md[0].knd, hipMemcpyDeviceToHost, st));
            GEVD_HIP(hipStreamSynchronize(st));
        }
        for (int i = 0; i < nm; ++i) {
            const MergeDesc& M = md[i];
            const int K = M.n1 + M.n2;
            if (M.knd == 0) continue;
            const double* Zi = M.pin ? w.Z1 : w.Z0;
            int ncols = M.knd;
            double* Cout;
            long ldc;
            if (root) {
                ncols = 0;
                while (ncols < M.knd && posL[ncols] < nev) ++ncols;  // ascending roots: a prefix
                Cout = Z;
                ldc = ldz;
            } else {
                Cout = (M.pin ? w.Z0 : w.Z1) + M.off;
                ldc = n;
            }
            if (ncols == 0) continue;
            int rc = gemm<double>(st, OP_N, OP_N, K, ncols, M.knd, 1.0, Zi + M.off, n, w.U + M.uoff, M.knd, 0.0,
                                  Cout, ldc, K_FULL, T_ALL, Batch(), 1, nullptr, w.amap + M.off, w.cmap + M.off);
            if (rc) return rc;
        }
        {
            int maxdefl = 0;
            for (auto& M : md) maxdefl = std::max(maxdefl, M.n1 + M.n2 - M.knd);
            if (maxdefl > 0) {
                {
            KProbe kp_(st, GEVD_K_DC, 0.0);
            hipLaunchKernelGGL(merge_defl_copy_kernel, dim3((maxK + 255) / 256, maxdefl, nm), dim3(256), 0, st, n,
                                   (const double*)w.Z0, (const double*)w.Z1, w.Z0, w.Z1, (const MergeDesc*)w.md,
                                   (const int*)w.perm, (const int*)w.dfl, (const int*)w.posD, root ? 1 : 0, nev, Z,
                                   ldz);
                GEVD_LAUNCH_CHECK();
        }
            }
        }
    }
    return 0;
}

}  // namespace gevd
