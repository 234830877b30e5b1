// Shared device/host helpers for the gfx950 generalized eigensolver.
// Scalars: double (real symmetric problems) and zdouble (complex Hermitian,
// interleaved re/im, layout-compatible with C99 double _Complex).
// All matrices are column-major: element (i, j) at p[i + j*ld].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

struct zdouble {
    double x, y;
};

__host__ __device__ inline zdouble zmake(double re, double im) { return zdouble{re, im}; }
__host__ __device__ inline zdouble operator+(zdouble a, zdouble b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ inline zdouble operator-(zdouble a, zdouble b) { return {a.x - b.x, a.y - b.y}; }
__host__ __device__ inline zdouble operator-(zdouble a) { return {-a.x, -a.y}; }
__host__ __device__ inline zdouble operator*(zdouble a, zdouble b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__host__ __device__ inline zdouble operator*(double s, zdouble a) { return {s * a.x, s * a.y}; }
__host__ __device__ inline zdouble operator*(zdouble a, double s) { return {s * a.x, s * a.y}; }
__host__ __device__ inline zdouble& operator+=(zdouble& a, zdouble b) { a.x += b.x; a.y += b.y; return a; }
__host__ __device__ inline zdouble& operator-=(zdouble& a, zdouble b) { a.x -= b.x; a.y -= b.y; return a; }

// Scalar traits: conj, real part, |x|^2, construction from a real.
__host__ __device__ inline double conjg(double a) { return a; }
__host__ __device__ inline zdouble conjg(zdouble a) { return {a.x, -a.y}; }
__host__ __device__ inline double realp(double a) { return a; }
__host__ __device__ inline double realp(zdouble a) { return a.x; }
__host__ __device__ inline double imagp(double) { return 0.0; }
__host__ __device__ inline double imagp(zdouble a) { return a.y; }
__host__ __device__ inline double abs2(double a) { return a * a; }
__host__ __device__ inline double abs2(zdouble a) { return a.x * a.x + a.y * a.y; }
template <typename T> __host__ __device__ inline T from_real(double r);
template <> __host__ __device__ inline double from_real<double>(double r) { return r; }
template <> __host__ __device__ inline zdouble from_real<zdouble>(double r) { return {r, 0.0}; }
template <typename T> __host__ __device__ inline T zero_of() { return from_real<T>(0.0); }
__host__ __device__ inline double fma_s(double a, double b, double c) { return fma(a, b, c); }
__host__ __device__ inline zdouble fma_s(zdouble a, zdouble b, zdouble c) {
    return {fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y))};
}
// a / b for b real
__host__ __device__ inline double div_r(double a, double b) { return a / b; }
__host__ __device__ inline zdouble div_r(zdouble a, double b) { return {a.x / b, a.y / b}; }
// complex division
__host__ __device__ inline double div_s(double a, double b) { return a / b; }
__host__ __device__ inline zdouble div_s(zdouble a, zdouble b) {
    double d = b.x * b.x + b.y * b.y;
    return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}
__host__ __device__ inline bool is_zero(double a) { return a == 0.0; }
__host__ __device__ inline bool is_zero(zdouble a) { return a.x == 0.0 && a.y == 0.0; }

template <typename T> struct is_cplx { static constexpr bool value = false; };
template <> struct is_cplx<zdouble> { static constexpr bool value = true; };

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

// ---------------------------------------------------------------------------
// Error handling inside the library: every HIP call is checked; the first
// failure is recorded and returned to the caller of the C interface.
// ---------------------------------------------------------------------------
#define GEVD_HIP(call)                                                          \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) {                                                 \
            fprintf(stderr, "gevd: %s failed: %s (%s:%d)\n", #call,             \
                    hipGetErrorString(e_), __FILE__, __LINE__);                 \
            return GEVD_E_HIP;                                                  \
        }                                                                       \
    } while (0)

#define GEVD_LAUNCH_CHECK() GEVD_HIP(hipGetLastError())

// Wave size on CDNA.
constexpr int WAVE = 64;

// Lane exchange (xor of the lane index) for the scalar types.
__device__ inline double shfl_xor_s(double v, int m) { return __shfl_xor(v, m, 64); }
__device__ inline zdouble shfl_xor_s(zdouble v, int m) { return {__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64)}; }

// Value of v in lane `lane` of the wavefront (lane uniform), as a scalar
// broadcast: two 32-bit lane reads per double.
__device__ inline double lane_bcast(double v, int lane) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)u, lane);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline zdouble lane_bcast(zdouble v, int lane) { return {lane_bcast(v.x, lane), lane_bcast(v.y, lane)}; }

// Sum over a 64-lane wavefront (all lanes receive the result).
__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ inline zdouble wave_sum(zdouble v) {
    return {wave_sum(v.x), wave_sum(v.y)};
}

// System-scope loads and stores of data shared between workgroups of one
// running kernel: loads bypass the (per-XCD, mutually non-coherent) caches,
// stores are written through to memory.  A writer that waits for its own
// stores (s_waitcnt) before it raises a flag needs no cache write-back, and
// a reader that sees the flag needs no cache invalidation.
__device__ inline double sys_load(const double* p) {
    return __longlong_as_double(
        __hip_atomic_load(reinterpret_cast<const long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
}
__device__ inline zdouble sys_load(const zdouble* p) { return {sys_load(&p->x), sys_load(&p->y)}; }
__device__ inline void sys_store(double* p, double v) {
    __hip_atomic_store(reinterpret_cast<long long*>(p), __double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ inline void sys_store(zdouble* p, zdouble v) {
    sys_store(&p->x, v.x);
    sys_store(&p->y, v.y);
}

// Block-wide sum for blockDim.x == NT (multiple of 64); all threads receive
// the result.  red must hold NT/64 entries of T.
template <int NT, typename T>
__device__ inline T block_sum(T v, T* red) {
    v = wave_sum(v);
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    T s = red[0];
#pragma unroll
    for (int i = 1; i < NT / WAVE; ++i) s += red[i];
    return s;
}
