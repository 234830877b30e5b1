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
// A wait gives up after this much device time (wall clock at 100 MHz):
// far beyond any legitimate wait, so only a broken invariant reaches it.
constexpr unsigned long long WAIT_LIMIT_TICKS = 120ull * 100000000ull;

// Band entries move between the workgroups of consecutive sweeps, which may
// sit on different XCDs whose L2 caches are not coherent with each other.
// They are therefore read and written at system scope (sys_load,
// sys_store): a task only has to wait for its own stores to complete before
// it publishes its progress counter, and a waiter reads fresh data without
// invalidating its L2 (which would also throw away every other workgroup's
// cached lines on that XCD).
__device__ inline int ntasks(int n, int b, int sw) { return (n - 1 - sw + b - 1) / b; }

// Band blocks of a task move through buffer resources at system scope
// (sc0 sc1, the same cache policy as sys_load / sys_store): one 64- or
// 128-bit access per element, and an element a lane does not own gets an
// out-of-range offset (loads return zero, stores are dropped), so the
// accesses need no branches.  Offsets stay far below 2^31 bytes (a task's
// blocks span 2b rows of at most 2b + 1 columns of the band storage).
constexpr unsigned BOOB = 0x80000000u;
constexpr int SYS_POLICY = 17;  // sc0 | sc1
__device__ inline __amdgpu_buffer_rsrc_t band_rsrc(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, 0x7fffffff, 0x00020000);
}
__device__ inline double band_load(double*, __amdgpu_buffer_rsrc_t r, unsigned off) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    const u2 u = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, SYS_POLICY);
    double v;
    __builtin_memcpy(&v, &u, sizeof v);
    return v;
}
__device__ inline zdouble band_load(zdouble*, __amdgpu_buffer_rsrc_t r, unsigned off) {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    const u4 u = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, SYS_POLICY);
    zdouble v;
    __builtin_memcpy(&v, &u, sizeof v);
    return v;
}
__device__ inline void band_store(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    u2 u;
    __builtin_memcpy(&u, &v, sizeof v);
    __builtin_amdgcn_raw_buffer_store_b64(u, r, off, 0, SYS_POLICY);
}
__device__ inline void band_store(zdouble v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    u4 u;
    __builtin_memcpy(&u, &v, sizeof v);
    __builtin_amdgcn_raw_buffer_store_b128(u, r, off, 0, SYS_POLICY);
}

// Reflector parameters for x = (alpha, x1..): H^H x = beta e1 with beta real,
// H = I - tau v v^H, v = (1, x1 * scale, ..); a2 = ||x1..||^2.
template <typename T>
__device__ inline void householder(T alpha, double a2, T* tau, double* beta, T* scale) {
    const double ar = realp(alpha), ai = imagp(alpha);
    if (a2 == 0.0 && ai == 0.0) {
        *tau = zero_of<T>();
        *beta = ar;
        *scale = zero_of<T>();
        return;
    }
    const double nrm = sqrt(ar * ar + ai * ai + a2);
    const double bt = ar >= 0.0 ? -nrm : nrm;
    *tau = div_r(from_real<T>(bt) - alpha, bt);
    *scale = div_s(from_real<T>(1.0), alpha - from_real<T>(bt));
    *beta = bt;
}

// Sum over the 64 lanes of each of C values per lane, C a power of two <= 16:
// exchanges that halve the values at each step (lane bit 2 log2(C)+1 .. 2
// picks the half), then plain exchanges over the remaining lane bits; on
// return v[0] of lane l holds the sum of value (l >> 2) % C.  Fixed order:
// the same bits on every run.
template <typename T, int C>
__device__ inline void lane_halve(T* v, int lane) {
    if constexpr (C > 1) {
        constexpr int H = C / 2;
        const bool up = (lane & (4 * H)) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const T keep = up ? v[i + H] : v[i];
            const T send = up ? v[i] : v[i + H];
            v[i] = keep + shfl_xor_s(send, 4 * H);
        }
        lane_halve<T, H>(v, lane);
    }
}
template <typename T, int C>
__device__ inline void lane_fold(T* v, int lane) {
    lane_halve<T, C>(v, lane);
    v[0] += shfl_xor_s(v[0], 1);
    v[0] += shfl_xor_s(v[0], 2);
#pragma unroll
    for (int m = 4 * C; m < WAVE; m *= 2) v[0] += shfl_xor_s(v[0], m);
}

// Householder reflector for x[0..L-1] (LDS, overwritten by v with v[0] = 1):
// H^H x = beta e1, beta real; sc[] receives {tau, beta, scale}.  One wave.
template <typename T>
__device__ inline void reflect1(T* x, int L, T* sc) {
    const int lane = threadIdx.x;
    double a2 = (lane >= 1 && lane < L) ? abs2(x[lane]) : 0.0;
    a2 = wave_sum(a2);
    if (lane == 0) {
        T tau, scale;
        double beta;
        householder<T>(x[0], a2, &tau, &beta, &scale);
        sc[0] = tau;
        sc[1] = from_real<T>(beta);
        sc[2] = scale;
    }
    __syncthreads();
    if (lane >= 1 && lane < L) x[lane] = x[lane] * sc[2];
    if (lane == 0) x[0] = from_real<T>(1.0);
    __syncthreads();
}

// One wave per workgroup; lane i owns row i of the b x b blocks, so the
// matrix-vector products and rank-1 updates need no cross-lane reduction
// and the only barriers are where a lane reads another lane's row.  E and D
// live in dynamic LDS, (b x (b+1)) each.
template <typename T>
__global__ __launch_bounds__(64) void hb2st_kernel(int n, int b, T* Bw, long ldw, T* V2, T* tau2, int nsw,
                                                  int* progress, int* counter, int* hang) {
    extern __shared__ char lds_raw[];
    T* Eb = reinterpret_cast<T*>(lds_raw);
    T* Db = Eb + (size_t)b * (b + 1);
    const int ldl = b + 1;
    __shared__ T v[MAXB], vp[MAXB], y[MAXB];
    __shared__ T sc[4];
    __shared__ T ptau;
    __shared__ int sw_s, stop;
    const int lane = threadIdx.x;
#define EL_(i, j) Eb[(i) * ldl + (j)]
#define DL_(i, j) Db[(i) * ldl + (j)]

    for (;;) {
        if (lane == 0) {
            sw_s = atomicAdd(counter, 1);
            stop = 0;
        }
        __syncthreads();
        const int sw = sw_s;
        if (sw >= nsw) return;
        const int nt = ntasks(n, b, sw);
        for (int t = 0; t < nt; ++t) {
            if (sw > 0) {
                if (lane == 0) {
                    const int need = min(t + 2, ntasks(n, b, sw - 1));
                    unsigned spins = 0;
                    unsigned long long t_start = 0;
                    // Relaxed polling, with an acquire every 64 polls: the L2
                    // of this XCD is not coherent with the writer's, and a
                    // relaxed load may keep hitting a stale line there until
                    // an acquire invalidates it.  The band itself is read
                    // past the caches (sys_load), so no fence follows.
                    while (__hip_atomic_load(&progress[sw - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        if ((++spins & 63u) == 0) {
                            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                            const unsigned long long now = wall_clock64();
                            if (t_start == 0) t_start = now;
                            if (now - t_start > WAIT_LIMIT_TICKS ||
                                __hip_atomic_load(hang, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                                atomicOr(hang, 1);
                                stop = 1;
                                break;
                            }
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                __syncthreads();
                if (stop) return;
            }
            const int r0 = sw + 1 + t * b;
            const int L = min(b, n - r0);
            const int pr0 = r0 - b;  // previous block (t > 0: always b rows)
            // Stage this task's blocks in LDS: E = B[r0.., pr0..] (t > 0) and
            // the lower triangle of D = B[r0.., r0..].  Lanes 0-31 and 32-63
            // take alternate columns of rows lane % 32 (b <= 32 here): all
            // loads are issued before the first one is used.
            // E's columns from pr0 (t > 0), D's from r0: single buffer
            // accesses at system scope, unowned elements masked by offset
            const auto rE = band_rsrc(Bw + IDX(0, max(pr0, 0), ldw));
            const auto rD = band_rsrc(Bw + IDX(0, r0, ldw));
            {
                constexpr int HB = 32;
                const int i = lane % HB, jh = lane / HB;
                T te[HB / 2], td[HB / 2];
#pragma unroll
                for (int k = 0; k < HB / 2; ++k) {
                    const int j = jh + 2 * k;
                    te[k] = band_load((T*)nullptr, rE,
                                      (t > 0 && i < L && j < b) ? (unsigned)(IDX(b + i - j, j, ldw) * sizeof(T)) : BOOB);
                    td[k] = band_load((T*)nullptr, rD,
                                      (i < L && j <= i) ? (unsigned)(IDX(i - j, j, ldw) * sizeof(T)) : BOOB);
                }
#pragma unroll
                for (int k = 0; k < HB / 2; ++k) {
                    const int j = jh + 2 * k;
                    if (t > 0 && i < L && j < b) EL_(i, j) = te[k];
                    if (i < L && j <= i) {
                        DL_(i, j) = td[k];
                        DL_(j, i) = conjg(td[k]);
                    }
                }
                if (t == 0 && lane < L) v[lane] = sys_load(&Bw[IDX(1 + lane, sw, ldw)]);
                __syncthreads();
            }
            if (t == 0) {
                reflect1<T>(v, L, sc);
                if (lane < L) sys_store(&Bw[IDX(1 + lane, sw, ldw)], (lane == 0) ? sc[1] : zero_of<T>());
            } else {
                const T pt = ptau;
                if (lane < L) {
                    const int i = lane;
                    T acc = zero_of<T>();
                    for (int j = 0; j < b; ++j) acc += EL_(i, j) * vp[j];
                    // row i of E (I - ptau vp vp^H)
                    const T pa = pt * acc;
                    for (int j = 0; j < b; ++j) EL_(i, j) -= pa * conjg(vp[j]);
                    v[i] = EL_(i, 0);
                }
                __syncthreads();
                if (L >= 2) {
                    reflect1<T>(v, L, sc);
                    // y_j = v^H E[:, j] (lane j), then E[:, 1:] -= conj(tau) v y^H
                    if (lane < b) {
                        T acc = zero_of<T>();
                        for (int i = 0; i < L; ++i) acc += conjg(v[i]) * EL_(i, lane);
                        y[lane] = acc;
                    }
                    __syncthreads();
                    const T ctau = conjg(sc[0]);
                    {
                        // every lane runs the same loop (rows >= L are masked
                        // by offset and read row 0 of the LDS block)
                        const int i = lane < L ? lane : 0;
                        const T cv = ctau * v[i];
                        for (int j = 0; j < b; ++j) {
                            const T x = (j == 0) ? ((lane == 0) ? sc[1] : zero_of<T>()) : EL_(i, j) - cv * y[j];
                            band_store(x, rE, lane < L ? (unsigned)(IDX(b + lane - j, j, ldw) * sizeof(T)) : BOOB);
                        }
                    }
                } else {
                    if (lane == 0) {
                        v[0] = from_real<T>(1.0);
                        sc[0] = zero_of<T>();
                    }
                    if (lane < L)
                        for (int j = 0; j < b; ++j) sys_store(&Bw[IDX(b + lane - j, pr0 + j, ldw)], EL_(lane, j));
                    __syncthreads();
                }
            }
            // two-sided update of the diagonal block rows/cols r0 .. r0+L-1
            const T tau = sc[0];
            if (!is_zero(tau)) {
                if (lane < L) {
                    T acc = zero_of<T>();
                    for (int j = 0; j < L; ++j) acc += DL_(lane, j) * v[j];
                    y[lane] = tau * acc;
                }
                T yv = (lane < L) ? conjg(y[lane]) * v[lane] : zero_of<T>();
                yv = wave_sum(yv);
                const T coef = from_real<T>(-0.5) * tau * yv;  // w = y - 1/2 tau (y^H v) v
                if (lane < L) y[lane] = y[lane] + coef * v[lane];
                __syncthreads();
                {
                    const int i = lane < L ? lane : 0;
                    for (int j = 0; j < b; ++j) {
                        T x = DL_(i, j) - v[i] * conjg(y[j]) - y[i] * conjg(v[j]);
                        if (i == j) x = from_real<T>(realp(x));
                        band_store(x, rD,
                                   (lane < L && j <= lane) ? (unsigned)(IDX(lane - j, j, ldw) * sizeof(T)) : BOOB);
                    }
                }
            }
            // keep the reflector for the back-transformation and the next task
            const size_t slot = (size_t)t * nsw + sw;
            if (lane < b) V2[slot * b + lane] = (lane < L) ? v[lane] : zero_of<T>();
            if (lane == 0) tau2[slot] = tau;
            __syncthreads();
            if (lane < MAXB) vp[lane] = (lane < L) ? v[lane] : zero_of<T>();
            if (lane == 0) ptau = tau;
            __builtin_amdgcn_s_waitcnt(0);  // this wave's band stores have reached memory
            __syncthreads();
            // The counter is stored at system scope too: written through,
            // not left in this XCD's L2 where a waiter on another XCD would
            // see it late.
            if (lane == 0) __hip_atomic_store(&progress[sw], t + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
#undef EL_
#undef DL_
}

// Workgroup variant (b > 8), where the single wave's row loops would
// dominate a task: row i of the blocks is handled by lane i of every
// wave, the CW waves split the inner index of each block product (wave w
// takes columns w, w + CW, ...) and add their partial sums in a fixed order
// (deterministic).  Sixteen waves (the largest workgroup) measured fastest:
// a task's arithmetic is short chains per lane, so more waves shorten it
// (complex n = 16384, b = 64: 340 ms with four waves, 282 with eight, 265 with
// sixteen; real n = 4096, b = 32: 106 ms with one wave, 46 with sixteen).
constexpr int CW = 16;  // waves per workgroup

template <typename T>
__global__ __launch_bounds__(64 * CW) void hb2st_kernel_wg(int n, int b, T* Bw, long ldw, T* V2, T* tau2, int nsw,
                                                          int* progress, int* counter, int* hang) {
    extern __shared__ char lds_raw[];
    T* Eb = reinterpret_cast<T*>(lds_raw);
    T* Db = Eb + (size_t)b * (b + 1);
    const int ldl = b + 1;
    __shared__ T v[MAXB], vp[MAXB], y[MAXB];
    __shared__ T part[CW][MAXB];
    __shared__ T rsum[MAXB];
    __shared__ T sc[4];
    __shared__ T ptau;
    __shared__ int sw_s, stop;
    const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    constexpr int NT = 64 * CW;
#define EL_(i, j) Eb[(i) * ldl + (j)]
#define DL_(i, j) Db[(i) * ldl + (j)]

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
                    unsigned spins = 0;
                    unsigned long long t_start = 0;
                    // polling as in the single-wave kernel
                    while (__hip_atomic_load(&progress[sw - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        if ((++spins & 63u) == 0) {
                            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                            const unsigned long long now = wall_clock64();
                            if (t_start == 0) t_start = now;
                            if (now - t_start > WAIT_LIMIT_TICKS ||
                                __hip_atomic_load(hang, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                                atomicOr(hang, 1);
                                stop = 1;
                                break;
                            }
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                __syncthreads();
                if (stop) return;
            }
            const int r0 = sw + 1 + t * b;
            const int L = min(b, n - r0);
            const int pr0 = r0 - b;
            // Stage this task's blocks: E = B[r0.., pr0..] (t > 0) and the lower
            // triangle of D = B[r0.., r0..].  Lane = row, wave = first column,
            // stepping by CW columns; all loads are issued before the first
            // one is used (one memory latency per task).  E stays in
            // registers; D also goes to LDS, mirrored, for its matrix-vector
            // product.
            constexpr int KW = MAXB / CW;  // columns per lane
            // E's columns from pr0 (t > 0), D's from r0
            const auto rE = band_rsrc(Bw + IDX(0, max(pr0, 0), ldw));
            const auto rD = band_rsrc(Bw + IDX(0, r0, ldw));
            T te[KW], td[KW];
#pragma unroll
            for (int k = 0; k < KW; ++k) {
                const int j = wv + CW * k;
                const unsigned oe =
                    (t > 0 && lane < L && j < b) ? (unsigned)(IDX(b + lane - j, j, ldw) * sizeof(T)) : BOOB;
                const unsigned od = (lane < L && j <= lane) ? (unsigned)(IDX(lane - j, j, ldw) * sizeof(T)) : BOOB;
                te[k] = band_load((T*)nullptr, rE, oe);
                td[k] = band_load((T*)nullptr, rD, od);
            }
#pragma unroll
            for (int k = 0; k < KW; ++k) {
                const int j = wv + CW * k;
                if (lane < L && j <= lane) {
                    DL_(lane, j) = td[k];
                    DL_(j, lane) = conjg(td[k]);
                }
            }
            if (t == 0 && tid < L) v[tid] = sys_load(&Bw[IDX(1 + tid, sw, ldw)]);
            __syncthreads();
            if (t == 0) {
                reflect1<T>(v, L, sc);
                if (tid < L) sys_store(&Bw[IDX(1 + tid, sw, ldw)], (tid == 0) ? sc[1] : zero_of<T>());
            } else {
                // E <- E (I - ptau vp vp^H), rows in registers; column 0 is the
                // next reflector's source
                {
                    T acc = zero_of<T>();
#pragma unroll
                    for (int k = 0; k < KW; ++k) acc += te[k] * vp[wv + CW * k];
                    part[wv][lane] = acc;
                }
                __syncthreads();
                // wave 0 adds the partial row sums, updates its columns and
                // forms the next reflector from column 0 (its first register
                // column: norm by a wave sum, alpha by a lane broadcast); the
                // other waves update their columns after the barrier
                if (wv == 0) {
                    T acc = part[0][lane];
#pragma unroll
                    for (int w = 1; w < CW; ++w) acc += part[w][lane];
                    const T pa = ptau * acc;
                    rsum[lane] = pa;
#pragma unroll
                    for (int k = 0; k < KW; ++k) te[k] -= pa * conjg(vp[CW * k]);
                    const T x = (lane < L) ? te[0] : zero_of<T>();
                    v[lane] = x;
                    if (L >= 2) {
                        const double a2 = wave_sum((lane >= 1 && lane < L) ? abs2(x) : 0.0);
                        T tau, scale;
                        double beta;
                        householder<T>(lane_bcast(x, 0), a2, &tau, &beta, &scale);
                        v[lane] = (lane == 0) ? from_real<T>(1.0) : (lane < L ? x * scale : zero_of<T>());
                        if (lane == 0) {
                            sc[0] = tau;
                            sc[1] = from_real<T>(beta);
                            sc[2] = scale;
                        }
                    }
                }
                __syncthreads();
                if (wv != 0) {
                    const T pa = rsum[lane];
#pragma unroll
                    for (int k = 0; k < KW; ++k) te[k] -= pa * conjg(vp[wv + CW * k]);
                }
                if (L >= 2) {
                    // y_j = v^H E[:, j] for this wave's columns, summed over the
                    // lanes (rows) by halving exchanges; lanes 4k .. 4k+3 end
                    // with y of column wv + CW k
                    const T vl = v[lane];
                    T yv[KW];
#pragma unroll
                    for (int k = 0; k < KW; ++k) yv[k] = conjg(vl) * te[k];
                    lane_fold<T, KW>(yv, lane);
                    const T ctau = conjg(sc[0]), beta = sc[1];
                    const T cv = ctau * vl;
#pragma unroll
                    for (int k = 0; k < KW; ++k) {
                        const int j = wv + CW * k;
                        const T yj = lane_bcast(yv[0], 4 * k);
                        const T x = (j == 0) ? ((lane == 0) ? beta : zero_of<T>()) : te[k] - cv * yj;
                        band_store(x, rE,
                                   (lane < L && j < b) ? (unsigned)(IDX(b + lane - j, j, ldw) * sizeof(T)) : BOOB);
                    }
                } else {
                    if (tid == 0) {
                        v[0] = from_real<T>(1.0);
                        sc[0] = zero_of<T>();
                    }
                    if (lane < L) {
#pragma unroll
                        for (int k = 0; k < KW; ++k) {
                            const int j = wv + CW * k;
                            if (j < b) sys_store(&Bw[IDX(b + lane - j, pr0 + j, ldw)], te[k]);
                        }
                    }
                    __syncthreads();
                }
            }
            // two-sided update of the diagonal block: y = tau D v,
            // w = y - 1/2 tau (y^H v) v, D <- D - v w^H - w v^H
            const T tau = sc[0];
            if (!is_zero(tau)) {
                if (lane < L) {
                    T acc = zero_of<T>();
#pragma unroll
                    for (int k = 0; k < KW; ++k) {
                        const int j = wv + CW * k;
                        if (j < L) acc += DL_(lane, j) * v[j];
                    }
                    part[wv][lane] = acc;
                }
                __syncthreads();
                if (tid < WAVE) {
                    T yl = zero_of<T>();
                    if (lane < L) {
                        T acc = part[0][lane];
#pragma unroll
                        for (int w = 1; w < CW; ++w) acc += part[w][lane];
                        yl = tau * acc;
                    }
                    T yv = (lane < L) ? conjg(yl) * v[lane] : zero_of<T>();
                    yv = wave_sum(yv);
                    const T coef = from_real<T>(-0.5) * tau * yv;
                    if (lane < L) y[lane] = yl + coef * v[lane];
                }
                __syncthreads();
                {
                    const T vi = v[lane], yi = y[lane];
#pragma unroll
                    for (int k = 0; k < KW; ++k) {
                        const int j = wv + CW * k;
                        T x = td[k] - vi * conjg(y[j]) - yi * conjg(v[j]);
                        if (lane == j) x = from_real<T>(realp(x));
                        band_store(x, rD, (lane < L && j <= lane) ? (unsigned)(IDX(lane - j, j, ldw) * sizeof(T)) : BOOB);
                    }
                }
            }
            if (tid < MAXB) vp[tid] = (tid < L) ? v[tid] : zero_of<T>();
            if (tid == 0) ptau = tau;
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (tid == 0) __hip_atomic_store(&progress[sw], t + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            // the reflector itself is read only after the kernel (back-transformation)
            const size_t slot = (size_t)t * nsw + sw;
            if (tid < b) V2[slot * b + tid] = (tid < L) ? v[tid] : zero_of<T>();
            if (tid == 0) tau2[slot] = tau;
        }
    }
#undef EL_
#undef DL_
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
// grouped in blocks of NBS; blocks are applied last-first and within a block
// the groups G(S, t) in t order.  A group's product H(s0,t)...H(s0+NBS-1,t)
// is I - V T V^H with V the NBS reflectors as a staircase (reflector j starts
// j rows below the group's first row, so the group spans NBS+b-1 rows), and
// is applied to the window of Z rows as three small products on the MFMA
// units: W = V^H Z, W <- T W, Z <- Z - V W.  The T factors of all groups are
// formed beforehand, in parallel (forward accumulation from the Gram matrix
// V^H V).  A workgroup (eight waves) owns 16 columns of Z and keeps the
// group's rows in an LDS ring of 128 rows (a group spans at most 127 rows;
// consecutive groups slide by b).  V is held dense in LDS (zeros outside the
// staircase, rows padded against bank conflicts), so every product is a
// fixed-length chain of MFMAs (three per complex k-step) whose operands
// are loaded into registers first: W's 16-row blocks with their inner range split over the waves
// (partials added in a fixed order), T W in two halves of its inner range,
// and one 16-row block of the window per wave for Z - V W.
// ---------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <typename T, int NBS>
__global__ __launch_bounds__(256) void chase_tfactor_kernel(int n, int b, int nsw, int nblk, const T* V2,
                                                            const T* tau2, T* Tg) {
    constexpr int NC = is_cplx<T>::value ? 2 : 1;
    __shared__ T vc[NBS][MAXB];
    __shared__ T G[NBS][NBS + 1];
    __shared__ T Tm[NBS][NBS + 1];
    __shared__ T tau[NBS];
    (void)NC;
    const int S = blockIdx.x, t = blockIdx.y, tid = threadIdx.x;
    const int s0 = S * NBS;
    for (int e = tid; e < NBS * b; e += 256) {
        const int j = e / b, q = e % b, s = s0 + j;
        const bool ok = s < nsw && s + 1 + t * b < n;
        vc[j][q] = ok ? V2[((size_t)t * nsw + s) * b + q] : zero_of<T>();
    }
    if (tid < NBS) {
        const int s = s0 + tid;
        const bool ok = s < nsw && s + 1 + t * b < n;
        tau[tid] = ok ? tau2[(size_t)t * nsw + s] : zero_of<T>();
    }
    __syncthreads();
    // Gram G[i][j] = v_i^H v_j over the overlap of their row ranges (i < j)
    for (int e = tid; e < NBS * NBS; e += 256) {
        const int i = e % NBS, j = e / NBS;
        T acc = zero_of<T>();
        if (i < j && j - i < b)
            for (int q = 0; q + (j - i) < b; ++q) acc += conjg(vc[i][q + (j - i)]) * vc[j][q];
        G[i][j] = acc;
    }
    __syncthreads();
    // T[j][j] = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j]
    for (int j = 0; j < NBS; ++j) {
        if (tid < j) {
            T acc = zero_of<T>();
            for (int l = tid; l < j; ++l) acc += Tm[tid][l] * G[l][j];
            Tm[tid][j] = -(tau[j] * acc);
        } else if (tid == j) {
            Tm[j][j] = tau[j];
        } else if (tid < NBS) {
            Tm[tid][j] = zero_of<T>();
        }
        __syncthreads();
    }
    T* out = Tg + ((size_t)t * nblk + S) * NBS * NBS;
    for (int e = tid; e < NBS * NBS; e += 256) out[e] = Tm[e / NBS][e % NBS];  // row-major
}

// 16 x 16 block accumulator on the FP64 matrix cores: one MFMA per k-step
// for real data; for complex data three (Gauss: ar br, ai bi and
// (ar + ai)(br + bi)), with the real and imaginary parts formed once at the
// end instead of four MFMAs per k-step.
template <typename T>
struct BlockAcc {
    dbl4 p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
    __device__ inline void mma(double ar, double ai, double br, double bi) {
        p1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, p1, 0, 0, 0);
        if constexpr (is_cplx<T>::value) {
            p2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, p2, 0, 0, 0);
            p3 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar + ai, br + bi, p3, 0, 0, 0);
        }
    }
    __device__ inline double re(int r) const { return is_cplx<T>::value ? p1[r] - p2[r] : p1[r]; }
    __device__ inline double im(int r) const { return p3[r] - p1[r] - p2[r]; }
};

template <typename T, int NBS>
__global__ __launch_bounds__(512) void back_chase_kernel(int n, int b, int nsw, int nblk, const T* V2, const T* Tg,
                                                   int nev, T* Z, long ldz) {
    constexpr int CX = is_cplx<T>::value ? 1 : 0;
    constexpr int NC = CX + 1;
    constexpr int NT = 512, NWV = NT / WAVE;
    constexpr int CT = 16, CTP = CT + 1, RING = 2 * MAXB;
    constexpr int NB1 = NBS / 16;                 // 16-row blocks of W = V^H Z
    constexpr int PA = NWV / NB1;                 // parts of W's inner dimension
    constexpr int KA = ((15 + MAXB + 3) / 4 + PA - 1) / PA;  // k-steps per part
    constexpr int VR = NBS + MAXB + 5;            // dense V row (r index), odd
    constexpr int TR = NBS + 5;                   // odd
    constexpr int KS = NBS / 4;                   // k-steps over the group's reflectors
    constexpr int KP = KS / 2;                    // k-steps per part of T W
    constexpr int NRB = (NBS + MAXB - 1 + 15) / 16;
    static_assert(NRB <= NWV && 2 * NB1 <= NWV, "wave split");
    // odd row pitches: the 16 lanes of an MFMA operand read (16 rows, one
    // column) fall on 16 distinct bank pairs
    static_assert(VR % 2 == 1 && TR % 2 == 1, "bank padding");
    static_assert(16 * (NB1 - 1) + 4 * PA * KA <= VR, "dense V rows");
    __shared__ double vd[NC][NBS][VR];
    __shared__ double tm[NC][NBS][TR];
    __shared__ double zr[NC][RING][CTP];
    __shared__ double wp[NC][PA][NBS][CTP];
    __shared__ double w1[NC][2][NBS][CTP];
    const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    const int c0 = blockIdx.x * CT;
    const int ncol = min(CT, nev - c0);
    const int li = lane % 16, lk = lane / 16;
    for (int e = tid; e < NC * NBS * VR; e += NT) (&vd[0][0][0])[e] = 0.0;
    for (int e = tid; e < NC * RING * CTP; e += NT) (&zr[0][0][0])[e] = 0.0;
    for (int e = tid; e < NC * 2 * NBS * CTP; e += NT) (&w1[0][0][0][0])[e] = 0.0;

    auto load_rows = [&](int ra, int rb) {
        const int nr = rb - ra;
        for (int e = tid; e < nr * CT; e += NT) {
            const int r = ra + e % nr, c = e / nr;
            const T v = (c < ncol) ? Z[IDX(r, c0 + c, ldz)] : zero_of<T>();
            zr[0][r & (RING - 1)][c] = realp(v);
            if (CX) zr[NC - 1][r & (RING - 1)][c] = imagp(v);
        }
    };
    auto store_rows = [&](int ra, int rb) {
        const int nr = rb - ra;
        for (int e = tid; e < nr * CT; e += NT) {
            const int r = ra + e % nr, c = e / nr;
            if (c < ncol) {
                T v;
                if constexpr (CX) v = zdouble{zr[0][r & (RING - 1)][c], zr[NC - 1][r & (RING - 1)][c]};
                else v = zr[0][r & (RING - 1)][c];
                Z[IDX(r, c0 + c, ldz)] = v;
            }
        }
    };
    constexpr int VPT = NBS * MAXB / NT, TPT = NBS * NBS / NT;
    T vreg[VPT], treg[TPT];
    auto fetch = [&](int S, int t) {
        const int s0 = S * NBS, s1 = min(nsw, s0 + NBS);
        const T* vsrc = V2 + ((size_t)t * nsw + s0) * b;
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int e = tid + NT * k;
            const int j = e / b, s = s0 + j;
            const bool ok = e < NBS * b && s < s1 && s + 1 + t * b < n;
            vreg[k] = ok ? vsrc[e] : zero_of<T>();
        }
        const T* tsrc = Tg + ((size_t)t * nblk + S) * NBS * NBS;
#pragma unroll
        for (int k = 0; k < TPT; ++k) treg[k] = tsrc[tid + NT * k];
    };
    auto next_group = [&](int& S, int& t) {
        if (S * NBS + 1 + (t + 1) * b < n) {
            ++t;
        } else {
            --S;
            t = 0;
        }
    };
    constexpr int ZPT = MAXB * CT / NT;
    T zpre[ZPT];
    int pre_a = -1, pre_b = -1;
    auto prefetch_rows = [&](int ra, int rb) {
        const int nr = rb - ra;
#pragma unroll
        for (int k = 0; k < ZPT; ++k) {
            const int e = tid + NT * k;
            zpre[k] = zero_of<T>();
            if (e < nr * CT) {
                const int r = ra + e % nr, c = e / nr;
                if (c < ncol) zpre[k] = Z[IDX(r, c0 + c, ldz)];
            }
        }
        pre_a = ra;
        pre_b = rb;
    };
    auto commit_rows = [&]() {
        const int nr = pre_b - pre_a;
#pragma unroll
        for (int k = 0; k < ZPT; ++k) {
            const int e = tid + NT * k;
            if (e < nr * CT) {
                const int r = pre_a + e % nr, c = e / nr;
                zr[0][r & (RING - 1)][c] = realp(zpre[k]);
                if (CX) zr[NC - 1][r & (RING - 1)][c] = imagp(zpre[k]);
            }
        }
    };
    if (nblk > 0) fetch(nblk - 1, 0);
    for (int S = nblk - 1; S >= 0; --S) {
        const int s0 = S * NBS, s1 = min(nsw, s0 + NBS);
        int lo = -1, hi = -1;
        pre_a = pre_b = -1;
        for (int t = 0;; ++t) {
            const int wr0 = s0 + 1 + t * b;
            if (wr0 >= n) break;
            const int wr1 = min(n, s1 + t * b + b);
            const int lg = wr1 - wr0;
            if (hi > lo) store_rows(lo, min(hi, wr0));
            const int la = (hi > wr0) ? hi : wr0;
            __syncthreads();
            if (wr1 > la) {
                if (pre_a == la && pre_b == wr1) commit_rows();
                else load_rows(la, wr1);
            }
            pre_a = pre_b = -1;
            lo = wr0;
            hi = wr1;
#pragma unroll
            for (int k = 0; k < VPT; ++k) {
                const int e = tid + NT * k;
                if (e < NBS * b) {
                    const int j = e / b, q = e % b;
                    const bool in = j + q < lg;  // rows past the matrix end hold no reflector entries
                    vd[0][j][j + q] = in ? realp(vreg[k]) : 0.0;
                    if (CX) vd[NC - 1][j][j + q] = in ? imagp(vreg[k]) : 0.0;
                }
            }
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
                const int e = tid + NT * k;
                tm[0][e / NBS][e % NBS] = realp(treg[k]);
                if (CX) tm[NC - 1][e / NBS][e % NBS] = imagp(treg[k]);
            }
            __syncthreads();
            {
                int Sn = S, tn = t;
                next_group(Sn, tn);
                if (Sn >= 0) fetch(Sn, tn);
                if (Sn == S) {
                    const int nw1 = min(n, s1 + (t + 1) * b + b);
                    if (nw1 > wr1 && nw1 - wr1 <= MAXB) prefetch_rows(wr1, nw1);
                }
            }
            const int base = wr0;
            // ---- W = V^H Z: block jb, inner rows split in PA parts of KA k-steps
            {
                const int jb = wv % NB1, part = wv / NB1;
                const int j = jb * 16 + li;
                const int rk = jb * 16 + part * KA * 4 + lk;
                double ar[KA], ai[KA], br[KA], bi[KA];
#pragma unroll
                for (int kk = 0; kk < KA; ++kk) {
                    const int r = rk + 4 * kk;
                    ar[kk] = vd[0][j][r];
                    ai[kk] = CX ? -vd[NC - 1][j][r] : 0.0;
                    br[kk] = zr[0][(base + r) & (RING - 1)][li];
                    bi[kk] = CX ? zr[NC - 1][(base + r) & (RING - 1)][li] : 0.0;
                }
                BlockAcc<T> acc;
#pragma unroll
                for (int kk = 0; kk < KA; ++kk) acc.mma(ar[kk], ai[kk], br[kk], bi[kk]);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    wp[0][part][jb * 16 + 4 * rr + lk][li] = acc.re(rr);
                    if (CX) wp[NC - 1][part][jb * 16 + 4 * rr + lk][li] = acc.im(rr);
                }
            }
            __syncthreads();
            // ---- W1 = T W (T upper triangular), in two parts of the inner range
            if (wv < 2 * NB1) {
                const int jb = wv % NB1, part = wv / NB1;
                double ar[KP], ai[KP], br[KP], bi[KP];
#pragma unroll
                for (int kk = 0; kk < KP; ++kk) {
                    const int ks = part * KP + kk;
                    const bool on = ks >= 4 * jb;  // T[i][k] = 0 for k < i
                    const int k = 4 * ks + lk;
                    ar[kk] = on ? tm[0][jb * 16 + li][k] : 0.0;
                    ai[kk] = (CX && on) ? tm[NC - 1][jb * 16 + li][k] : 0.0;
                    double sr = 0.0, si = 0.0;
#pragma unroll
                    for (int p = 0; p < PA; ++p) {
                        sr += wp[0][p][k][li];
                        if (CX) si += wp[NC - 1][p][k][li];
                    }
                    br[kk] = on ? sr : 0.0;
                    bi[kk] = on ? si : 0.0;
                }
                BlockAcc<T> acc;
#pragma unroll
                for (int kk = 0; kk < KP; ++kk) acc.mma(ar[kk], ai[kk], br[kk], bi[kk]);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    w1[0][part][jb * 16 + 4 * rr + lk][li] = acc.re(rr);
                    if (CX) w1[NC - 1][part][jb * 16 + 4 * rr + lk][li] = acc.im(rr);
                }
            }
            __syncthreads();
            // ---- Z <- Z - V W1: one 16-row block of the window per wave
            if (wv < NRB && wv * 16 < lg) {
                const int r = wv * 16 + li;
                double ar[KS], ai[KS], br[KS], bi[KS];
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const int j = 4 * ks + lk;
                    ar[ks] = vd[0][j][r];
                    ai[ks] = CX ? vd[NC - 1][j][r] : 0.0;
                    br[ks] = w1[0][0][j][li] + w1[0][1][j][li];
                    bi[ks] = CX ? w1[NC - 1][0][j][li] + w1[NC - 1][1][j][li] : 0.0;
                }
                BlockAcc<T> acc;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) acc.mma(ar[ks], ai[ks], br[ks], bi[ks]);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int rw = wv * 16 + 4 * rr + lk;
                    if (rw < lg) {
                        zr[0][(base + rw) & (RING - 1)][li] -= acc.re(rr);
                        if (CX) zr[NC - 1][(base + rw) & (RING - 1)][li] -= acc.im(rr);
                    }
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
        const int grid = std::min(R.nsw, 1024);
        const size_t lds = (size_t)2 * b * (b + 1) * sizeof(T);
        const bool wide = b > 8;  // a workgroup per sweep pays off except for the narrowest bands
        GEVD_HIP(hipFuncSetAttribute(wide ? reinterpret_cast<const void*>(&hb2st_kernel_wg<T>)
                                          : reinterpret_cast<const void*>(&hb2st_kernel<T>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        // algorithmic work: about 6 n^2 b real flops (x4 complex)
        KProbe probe(st, GEVD_K_CHASE, (is_cplx<T>::value ? 24.0 : 6.0) * (double)n * n * b);
        if (wide)
            hipLaunchKernelGGL(hb2st_kernel_wg<T>, dim3(grid), dim3(64 * CW), lds, st, n, b, Bw, ldw, R.V2, R.tau2,
                               R.nsw, progress, counter, c.hang);
        else
            hipLaunchKernelGGL(hb2st_kernel<T>, dim3(grid), dim3(64), lds, st, n, b, Bw, ldw, R.V2, R.tau2, R.nsw,
                               progress, counter, c.hang);
        GEVD_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(extract_tridiag<T>, dim3((n + 255) / 256), dim3(256), 0, st, n, (const T*)Bw, ldw, d, e);
    GEVD_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int back_chase_tfactor(const ChaseRefl<T>& R, hipStream_t st) {
    if (R.nsw <= 0) return 0;
    constexpr int NBS = chase_group<T>();
    if (R.nbs != NBS || R.Tg == nullptr || R.b > MAXB) return GEVD_E_STATE;
    KProbe probe(st, GEVD_K_OTHER, 0.0);
    hipLaunchKernelGGL((chase_tfactor_kernel<T, NBS>), dim3(R.nblk, R.tmax), dim3(256), 0, st, R.n, R.b, R.nsw,
                       R.nblk, (const T*)R.V2, (const T*)R.tau2, R.Tg);
    GEVD_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int back_chase(const StageCtx& c, const ChaseRefl<T>& R, int nev, T* Z, long ldz, bool tfactored) {
    if (R.nsw <= 0 || nev <= 0) return 0;
    constexpr int NBS = chase_group<T>();
    if (R.nbs != NBS || R.Tg == nullptr || R.b > MAXB) return GEVD_E_STATE;
    int rc;
    if (!tfactored && (rc = back_chase_tfactor<T>(R, c.st))) return rc;
    const int grid = (nev + 15) / 16;
    // algorithmic work: every reflector applied to every column, 4 L nev
    // real flops each (x4 complex): about 2 n^2 nev in total
    KProbe probe(c.st, GEVD_K_BACKCHASE, (is_cplx<T>::value ? 8.0 : 2.0) * (double)R.n * R.n * nev);
    hipLaunchKernelGGL((back_chase_kernel<T, NBS>), dim3(grid), dim3(512), 0, c.st, R.n, R.b, R.nsw, R.nblk,
                       (const T*)R.V2, (const T*)R.Tg, nev, Z, ldz);
    GEVD_LAUNCH_CHECK();
    return 0;
}

#define INST(T)                                                                              \
    template int hb2st<T>(const StageCtx&, int, T*, long, ChaseRefl<T>&, double*, double*, int*); \
    template int back_chase_tfactor<T>(const ChaseRefl<T>&, hipStream_t);                          \
    template int back_chase<T>(const StageCtx&, const ChaseRefl<T>&, int, T*, long, bool);
INST(double)
INST(zdouble)
#undef INST

}  // namespace gevd
