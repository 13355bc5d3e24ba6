// bttb_cgls.hip -- vector kernels of the inversion driver (CGLS for the
// regularised least-squares problem min ||G m - d||^2 + lambda^2 ||m||^2, the
// inverse problem the transpose product serves: Sec. 1 and Sec. 7).
//
// All reductions accumulate in FP64 (one partial per block, then one block
// sums the partials in a fixed order: results are deterministic).  The step
// scalars live in device memory (CglsScalars), so an iteration needs no host
// synchronisation.
#include "kern_common.h"

namespace bttbk {

constexpr int RED_THREADS = 256;

// block sum of a per-thread FP64 value (wave64 shuffles, then LDS); the
// result is valid in thread 0
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double part[RED_THREADS / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    if (lane == 0) part[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < RED_THREADS / 64; ++i) s += part[i];
    return s;
}

// the partials of one reduction: sum over blocks in a fixed order
__device__ __forceinline__ double sum_partials(const double* p, int nb)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += RED_THREADS) v += p[i];
    return block_sum(v);
}

// four consecutive values with 16-byte accesses (the address must be
// 16-byte aligned)
template <typename T> struct V4 { T x[4]; };
template <typename T> __device__ __forceinline__ V4<T> ld4(const T* p)
{
    V4<T> v;
    if constexpr (sizeof(T) == 4) {
        const float4 f = *(const float4*)p;
        v.x[0] = f.x; v.x[1] = f.y; v.x[2] = f.z; v.x[3] = f.w;
    } else {
        const double2 a = *(const double2*)p, b = *(const double2*)(p + 2);
        v.x[0] = a.x; v.x[1] = a.y; v.x[2] = b.x; v.x[3] = b.y;
    }
    return v;
}
template <typename T> __device__ __forceinline__ void st4(T* p, const V4<T>& v)
{
    if constexpr (sizeof(T) == 4) {
        *(float4*)p = make_float4(v.x[0], v.x[1], v.x[2], v.x[3]);
    } else {
        *(double2*)p = make_double2(v.x[0], v.x[1]);
        *(double2*)(p + 2) = make_double2(v.x[2], v.x[3]);
    }
}
__device__ __forceinline__ bool al16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// The element-wise kernels visit [0, n) in 4-element chunks with a grid-stride
// loop when every array is 16-byte aligned (n4 = n / 4 chunks), then the
// remaining elements one by one.
#define BTTB_GRID_LOOPS(n, aligned, CHUNK, ONE)                                                      \
    {                                                                                               \
        const int64_t stride_ = (int64_t)gridDim.x * RED_THREADS;                                  \
        const int64_t n4_ = (aligned) ? (n) / 4 : 0;                                                \
        for (int64_t c = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; c < n4_; c += stride_) { \
            const int64_t i = 4 * c;                                                                \
            CHUNK                                                                                   \
        }                                                                                           \
        for (int64_t i = 4 * n4_ + (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < (n); i += stride_) { \
            ONE                                                                                     \
        }                                                                                           \
    }

// out[blockIdx.x] = partial of sum_i a_i b_i over a grid-stride range
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_dot(const T* __restrict__ a, const T* __restrict__ b, int64_t n,
                                                     double* __restrict__ out)
{
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * RED_THREADS)
        v += (double)a[i] * (double)b[i];
    const double s = block_sum(v);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// r = d - q; partials of ||r||^2
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_residual(const T* __restrict__ d, const T* __restrict__ q,
                                                          T* __restrict__ r, int64_t n, double* __restrict__ out)
{
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * RED_THREADS) {
        const T x = d[i] - q[i];
        r[i] = x;
        v += (double)x * (double)x;
    }
    const double s = block_sum(v);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// with step: m = m + alpha p (alpha from the scalars); then s = s - lambda^2 m;
// partials of ||s||^2 (out_s) and ||m||^2 (out_m).  The step of m is done
// here rather than beside r's (k_step): the transpose product between them
// reads r only, and one pass over m, p and s saves a pass over m.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_grad(T* __restrict__ s, T* __restrict__ m, const T* __restrict__ p,
                                                      const CglsScalars* __restrict__ sc, int step, double lam2,
                                                      int64_t n, double* __restrict__ out_s, double* __restrict__ out_m)
{
    const double alpha = step ? sc->alpha : 0.0;
    double vs = 0.0, vm = 0.0;
    BTTB_GRID_LOOPS(n, al16(s) && al16(m) && (!step || al16(p)), {
        V4<T> sv = ld4(s + i);
        V4<T> mv = ld4((const T*)m + i);
        if (step) {
            const V4<T> pv = ld4(p + i);
            for (int k = 0; k < 4; ++k) mv.x[k] = (T)((double)mv.x[k] + alpha * (double)pv.x[k]);
            st4(m + i, mv);
        }
        for (int k = 0; k < 4; ++k) {
            sv.x[k] = (T)((double)sv.x[k] - lam2 * (double)mv.x[k]);
            vs += (double)sv.x[k] * (double)sv.x[k];
            vm += (double)mv.x[k] * (double)mv.x[k];
        }
        st4(s + i, sv);
    }, {
        T mi = m[i];
        if (step) {
            mi = (T)((double)mi + alpha * (double)p[i]);
            m[i] = mi;
        }
        const T x = (T)((double)s[i] - lam2 * (double)mi);
        s[i] = x;
        vs += (double)x * (double)x;
        vm += (double)mi * (double)mi;
    })
    const double a = block_sum(vs);
    __syncthreads();
    const double b = block_sum(vm);
    if (threadIdx.x == 0) {
        out_s[blockIdx.x] = a;
        out_m[blockIdx.x] = b;
    }
}

// p = s + beta p (beta from the scalars; first: p = s, p not read); partials
// of ||p||^2
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_direction(const T* __restrict__ s, T* __restrict__ p, int64_t n,
                                                           const CglsScalars* __restrict__ sc, int first,
                                                           double* __restrict__ out)
{
    const double beta = first ? 0.0 : sc->beta;
    double v = 0.0;
    BTTB_GRID_LOOPS(n, al16(s) && al16(p), {
        V4<T> x = ld4(s + i);
        if (!first) {
            const V4<T> pv = ld4((const T*)p + i);
            for (int k = 0; k < 4; ++k) x.x[k] = (T)((double)x.x[k] + beta * (double)pv.x[k]);
        }
        for (int k = 0; k < 4; ++k) v += (double)x.x[k] * (double)x.x[k];
        st4(p + i, x);
    }, {
        const T x = first ? s[i] : (T)((double)s[i] + beta * (double)p[i]);
        p[i] = x;
        v += (double)x * (double)x;
    })
    const double a = block_sum(v);
    if (threadIdx.x == 0) out[blockIdx.x] = a;
}

// r = r - alpha q over [0, nd); partials of ||r||^2 after the update (the
// matching step of m is done by k_grad)
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_step(T* __restrict__ r, const T* __restrict__ q, int64_t nd,
                                                      const CglsScalars* __restrict__ sc, double* __restrict__ out)
{
    const double alpha = sc->alpha;
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < nd; i += (int64_t)gridDim.x * RED_THREADS) {
        const T x = (T)((double)r[i] - alpha * (double)q[i]);
        r[i] = x;
        v += (double)x * (double)x;
    }
    const double a = block_sum(v);
    if (threadIdx.x == 0) out[blockIdx.x] = a;
}

// alpha = gamma / (||q||^2 + lambda^2 ||p||^2); 0 when the denominator is 0
// or once the gradient has converged, gamma <= tol2 gamma0: from there on the
// steps leave m and r as they are
__global__ void __launch_bounds__(RED_THREADS) k_alpha(const double* __restrict__ pq, const double* __restrict__ pp,
                                                       int nb, double lam2, double tol2, CglsScalars* __restrict__ sc)
{
    const double qq = sum_partials(pq, nb);
    __syncthreads();
    const double ppv = sum_partials(pp, nb);
    if (threadIdx.x == 0) {
        const double den = qq + lam2 * ppv;
        const bool converged = sc->gamma <= tol2 * sc->gamma0;
        sc->alpha = den > 0.0 && !converged ? sc->gamma / den : 0.0;
    }
}

// gamma' = ||s||^2, beta = gamma' / gamma, gamma = gamma'; history entry k:
// (||r||^2, ||m||^2, ||s||^2)
__global__ void __launch_bounds__(RED_THREADS) k_beta(const double* __restrict__ ps, const double* __restrict__ pr,
                                                      const double* __restrict__ pm, int nb, CglsScalars* __restrict__ sc,
                                                      double* __restrict__ hist, int k, int first)
{
    const double ss = sum_partials(ps, nb);
    __syncthreads();
    const double rr = sum_partials(pr, nb);
    __syncthreads();
    const double mm = sum_partials(pm, nb);
    if (threadIdx.x == 0) {
        sc->beta = (!first && sc->gamma > 0.0) ? ss / sc->gamma : 0.0;
        sc->gamma = ss;
        if (first) sc->gamma0 = ss;
        if (hist) {
            hist[3 * k] = rr;
            hist[3 * k + 1] = mm;
            hist[3 * k + 2] = ss;
        }
    }
}

// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_cgls_dot(const T* a, const T* b, int64_t n, double* out, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot<T>, dim3(nb), dim3(RED_THREADS), 0, s, a, b, n, out);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_cgls_residual(const T* d, const T* q, T* r, int64_t n, double* out, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual<T>, dim3(nb), dim3(RED_THREADS), 0, s, d, q, r, n, out);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_cgls_grad(T* sv, T* m, const T* p, const CglsScalars* sc, int step, double lam2, int64_t n,
                            double* out_s, double* out_m, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_grad<T>, dim3(nb), dim3(RED_THREADS), 0, s, sv, m, p, sc, step, lam2, n, out_s, out_m);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_cgls_direction(const T* sv, T* p, int64_t n, const CglsScalars* sc, int first, double* out, int nb,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(k_direction<T>, dim3(nb), dim3(RED_THREADS), 0, s, sv, p, n, sc, first, out);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_cgls_step(T* r, const T* q, int64_t nd, const CglsScalars* sc, double* out, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_step<T>, dim3(nb), dim3(RED_THREADS), 0, s, r, q, nd, sc, out);
    return hipGetLastError();
}
hipError_t launch_cgls_alpha(const double* pq, const double* pp, int nb, double lam2, double tol2, CglsScalars* sc,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_alpha, dim3(1), dim3(RED_THREADS), 0, s, pq, pp, nb, lam2, tol2, sc);
    return hipGetLastError();
}
hipError_t launch_cgls_beta(const double* ps, const double* pr, const double* pm, int nb, CglsScalars* sc,
                            double* hist, int k, int first, hipStream_t s)
{
    hipLaunchKernelGGL(k_beta, dim3(1), dim3(RED_THREADS), 0, s, ps, pr, pm, nb, sc, hist, k, first);
    return hipGetLastError();
}

#define BTTB_CGLS_INST(T)                                                                                   \
    template hipError_t launch_cgls_dot<T>(const T*, const T*, int64_t, double*, int, hipStream_t);         \
    template hipError_t launch_cgls_residual<T>(const T*, const T*, T*, int64_t, double*, int, hipStream_t); \
    template hipError_t launch_cgls_grad<T>(T*, T*, const T*, const CglsScalars*, int, double, int64_t, double*, \
                                            double*, int, hipStream_t);                                     \
    template hipError_t launch_cgls_direction<T>(const T*, T*, int64_t, const CglsScalars*, int, double*, int, \
                                                 hipStream_t);                                              \
    template hipError_t launch_cgls_step<T>(T*, const T*, int64_t, const CglsScalars*, double*, int, hipStream_t);
BTTB_CGLS_INST(float)
BTTB_CGLS_INST(double)
#undef BTTB_CGLS_INST

}  // namespace bttbk
