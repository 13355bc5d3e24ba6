// bttb_kernels.hip -- gfx950 kernels of the fast BTTB products.
//
//   k_twiddles       FP64 twiddle tables exp(-2 pi i k / N), rounded to the
//                    working precision
//   k_generate       FP64 circulant generator T_r of each depth layer from
//                    the closed-form prism integrals (Sec. 3, eq. Tcircpadded /
//                    eq. Tcircpaddedgeneral; Sec. 4.1 / 4.2 entries)
//   k_rows_r2c       real rows -> half spectra along x, pairs of rows packed
//                    into one complex transform, written column-major
//                    ([kx][row]) through an LDS tile
//   k_cols_spec      FP64 column transforms of the generator -> stored spectra
//                    (scaled by 1 / (Nx Ny), rounded to the working precision)
//   k_cols_fwd_mac   forward product: per column kx, the depth loop
//                    A += T^_r * FFT_y(X_r) with an extended accumulator, then
//                    one inverse FFT_y (eq. GrviaT summed over layers)
//   k_cols_tr_mac    transpose product: R^ = FFT_y(R) once per column, then per
//                    layer IFFT_y(conj(T^_r) R^)
//   k_rows_c2r       half spectra ([kx][row]) -> real rows along x, two rows per
//                    complex transform, extraction of the leading columns
//
// All kernels take caller-owned device buffers; none allocates.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.h"
#include "bttb_internal.h"

namespace bttbk {

// ---------------------------------------------------------------------------
// twiddles
// ---------------------------------------------------------------------------
__global__ void k_twiddles(double2* __restrict__ t64, float2* __restrict__ t32, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double s, c;
    // exp(-2 pi i k / n) = cospi(2k/n) - i sinpi(2k/n); 2k/n is exact for
    // power-of-two n
    sincospi(2.0 * (double)k / (double)n, &s, &c);
    t64[k] = make_double2(c, -s);
    if (t32) t32[k] = make_float2((float)c, (float)-s);
}

// ---------------------------------------------------------------------------
// generator (FP64)
// ---------------------------------------------------------------------------
// ln(rho + x); for x < 0 the identity rho + x = (rho^2 - x^2) / (rho - x)
// avoids the cancellation (other2 = rho^2 - x^2 as a sum of squares)
__device__ __forceinline__ double ln_rho_plus(double rho, double x, double other2)
{
    return x >= 0.0 ? log(rho + x) : log(other2 / (rho - x));
}

// gravity corner term (Sec. 4.1): z atan(x y / (z rho)) - x ln(rho + y) - y ln(rho + x);
// the atan term's limit at z = 0 is 0
__device__ __forceinline__ double corner_gz(double x, double y, double z)
{
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double rho = sqrt(x2 + y2 + z2);
    double f = -x * ln_rho_plus(rho, y, x2 + z2) - y * ln_rho_plus(rho, x, y2 + z2);
    if (z != 0.0) f += z * atan((x * y) / (z * rho));
    return f;
}

// magnetic corner term (Sec. 4.2, eq. magnetickernel with ln F_i and F_i as
// signed corner sums): w0 ln(rho+x) + w1 ln(rho+y) + w2 ln(rho+z)
//   + w3 atan(x z / (y rho)) + w4 atan(y z / (x rho))
__device__ __forceinline__ double corner_tmi(double x, double y, double z, const MagWeights& w)
{
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double rho = sqrt(x2 + y2 + z2);
    double f = w.g[0] * ln_rho_plus(rho, x, y2 + z2) + w.g[1] * ln_rho_plus(rho, y, x2 + z2) +
               w.g[2] * ln_rho_plus(rho, z, x2 + y2);
    if (z != 0.0) f += w.g[3] * atan((x * z) / (y * rho)) + w.g[4] * atan((y * z) / (x * rho));
    return f;
}

// One thread per circulant position (X, Y) of layer r = r0 + blockIdx.y:
//   T_r[Y][X] = h_r(-ax - pxl, -ay - pyl) if ax in [-(nx-1), sx-1] and
//   ay in [-(ny-1), sy-1], with ax = X or X - Nx (and likewise ay), else 0.
// h_r(dx, dy) is the prism integral over x in [(dx-1/2), (dx+1/2)] Dx,
// y in [(dy-1/2), (dy+1/2)] Dy, z in [z_r + h, z_{r+1} + h]: the entry of
// G for a station and a prism offset by (dx, dy) cells (Sec. 2.1.1-2.1.2).
__global__ void k_generate(GenParams P, int r0, double* __restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)P.Nx * P.Ny;
    if (idx >= per) return;
    const int r = r0 + blockIdx.y;
    const int X = (int)(idx % P.Nx), Y = (int)(idx / P.Nx);
    int ax = X <= P.sx - 1 ? X : (X >= P.Nx - (P.nx - 1) ? X - P.Nx : INT32_MIN);
    int ay = Y <= P.sy - 1 ? Y : (Y >= P.Ny - (P.ny - 1) ? Y - P.Ny : INT32_MIN);
    double val = 0.0;
    if (ax != INT32_MIN && ay != INT32_MIN) {
        const int ox = -ax - P.pxl, oy = -ay - P.pyl;
        if (P.kind == KIND_PROBE) {
            val = (double)ox + 4096.0 * (double)oy + 16777216.0 * (double)r;
        } else {
            const double x1 = ((double)ox - 0.5) * P.dx, x2 = ((double)ox + 0.5) * P.dx;
            const double y1 = ((double)oy - 0.5) * P.dy, y2 = ((double)oy + 0.5) * P.dy;
            const double z1 = P.z[blockIdx.y] + P.h, z2 = P.z[blockIdx.y + 1] + P.h;
            const double xs[2] = {x1, x2}, ys[2] = {y1, y2}, zs[2] = {z1, z2};
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        const double f = P.kind == KIND_GRAVITY ? corner_gz(xs[i], ys[j], zs[k])
                                                                : corner_tmi(xs[i], ys[j], zs[k], P.w);
                        // (-1)^(i+j+k) with 1-based indices: + when the
                        // 0-based index sum is odd
                        s += ((i + j + k) & 1) ? f : -f;
                    }
            val = P.scale * s;
        }
    }
    out[(int64_t)blockIdx.y * per + idx] = val;
}

// ---------------------------------------------------------------------------
// row transforms
// ---------------------------------------------------------------------------
template <typename T, int N> struct RowCfg {
    static constexpr int TPL = N / 8;
    static constexpr int PAIRS = sizeof(T) == 4 ? (N <= 2048 ? (256 / TPL > 4 ? 256 / TPL : 4) : 2)
                                                : (N <= 1024 ? (256 / TPL > 4 ? 256 / TPL : 4)
                                                             : (N == 2048 ? 2 : 1));
    static constexpr int RT = 2 * PAIRS;            // rows per block
    static constexpr int THREADS = PAIRS * TPL;
    static constexpr int HALF = N / 2 + 1;          // columns of a half spectrum
    static constexpr int SROW = RT + 1;             // padded staging row
    static constexpr int STAGE = HALF * SROW;
    static constexpr int XCH = PAIRS * lds_line_elems(N);
    static constexpr int LDS = STAGE > XCH ? STAGE : XCH;
};

// in:  batch b, row y, column x at in[b * in_bs + y * in_ld + x], x < nvx valid
// out: out[b * out_bs + kx * out_ld + y] for kx <= N/2, y < nrows
template <typename TI, typename T, int N>
__global__ void __launch_bounds__((RowCfg<T, N>::THREADS))
k_rows_r2c(const TI* __restrict__ in, int64_t in_bs, int64_t in_ld, int nvx, int nrows,
           cT<T>* __restrict__ out, int64_t out_bs, int64_t out_ld, const cT<T>* __restrict__ tw,
           int blocks_per_batch)
{
    using C = RowCfg<T, N>;
    constexpr int TPL = C::TPL;
    __shared__ cT<T> lds[C::LDS];
    const int b = blockIdx.x / blocks_per_batch;
    const int row0 = (blockIdx.x % blocks_per_batch) * C::RT;
    const int pr = threadIdx.x / TPL, t = threadIdx.x % TPL;
    const int ra = row0 + 2 * pr, rb = ra + 1;
    const TI* src = in + (int64_t)b * in_bs;
    cT<T> v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int x = t + m * TPL;
        T a = 0, c = 0;
        if (x < nvx) {
            if (ra < nrows) a = (T)src[(int64_t)ra * in_ld + x];
            if (rb < nrows) c = (T)src[(int64_t)rb * in_ld + x];
        }
        v[m] = mk<T>(a, c);
    }
    LineTwiddles<T, N> twl;
    twl.load(tw, t);
    cT<T>* xl = lds + pr * lds_line_elems(N);
    if (nvx <= N / 2) fft_line<T, N, -1, true>(v, xl, twl, t);
    else fft_line<T, N, -1, false>(v, xl, twl, t);
    // split Z = FFT(a + i c) into A = FFT(a), C = FFT(c):
    // A[k] = (Z[k] + conj Z[N-k]) / 2, C[k] = (Z[k] - conj Z[N-k]) / (2 i)
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 8; ++m) xl[lpad(t + m * TPL)] = v[m];
    __syncthreads();
    cT<T> A[5], Cc[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        const int k = t + m * TPL;
        if (m < 4 || t == 0) {
            const cT<T> z = v[m];
            const cT<T> zr = xl[lpad((N - k) & (N - 1))];
            A[m] = mk<T>((T)0.5 * (z.x + zr.x), (T)0.5 * (z.y - zr.y));
            Cc[m] = mk<T>((T)0.5 * (z.y + zr.y), (T)0.5 * (zr.x - z.x));
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        const int k = t + m * TPL;
        if (m < 4 || t == 0) {
            lds[k * C::SROW + 2 * pr] = A[m];
            lds[k * C::SROW + 2 * pr + 1] = Cc[m];
        }
    }
    __syncthreads();
    cT<T>* dst = out + (int64_t)b * out_bs;
    for (int e = threadIdx.x; e < C::HALF * C::RT; e += C::THREADS) {
        const int kx = e / C::RT, rr = e % C::RT;
        if (row0 + rr < nrows) dst[(int64_t)kx * out_ld + row0 + rr] = lds[kx * C::SROW + rr];
    }
}

// in:  in[b * in_bs + kx * in_ld + y], kx <= N/2, y < nrows (half spectra)
// out: out[b * out_bs + y * out_ld + x] for x < nvx_out (real, unnormalised
//      inverse transform; the 1/(Nx Ny) factor lives in the spectra)
template <typename T, int N>
__global__ void __launch_bounds__((RowCfg<T, N>::THREADS))
k_rows_c2r(const cT<T>* __restrict__ in, int64_t in_bs, int64_t in_ld, int nrows,
           T* __restrict__ out, int64_t out_bs, int64_t out_ld, int nvx_out,
           const cT<T>* __restrict__ tw, int blocks_per_batch)
{
    using C = RowCfg<T, N>;
    constexpr int TPL = C::TPL;
    __shared__ cT<T> lds[C::LDS];
    const int b = blockIdx.x / blocks_per_batch;
    const int row0 = (blockIdx.x % blocks_per_batch) * C::RT;
    const int pr = threadIdx.x / TPL, t = threadIdx.x % TPL;
    const cT<T>* src = in + (int64_t)b * in_bs;
    for (int e = threadIdx.x; e < C::HALF * C::RT; e += C::THREADS) {
        const int kx = e / C::RT, rr = e % C::RT;
        lds[kx * C::SROW + rr] = (row0 + rr < nrows) ? src[(int64_t)kx * in_ld + row0 + rr] : mk<T>(0, 0);
    }
    __syncthreads();
    // Z[k] = A[k] + i C[k] over the full length, using Hermitian symmetry
    // above N/2; the imaginary parts at k = 0 and k = N/2 are dropped (real
    // transform convention)
    cT<T> v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int k = t + m * TPL;
        const int kk = k <= N / 2 ? k : N - k;
        cT<T> A = lds[kk * C::SROW + 2 * pr], Cc = lds[kk * C::SROW + 2 * pr + 1];
        if (k > N / 2) { A.y = -A.y; Cc.y = -Cc.y; }
        if (kk == 0 || kk == N / 2) { A.y = 0; Cc.y = 0; }
        v[m] = mk<T>(A.x - Cc.y, A.y + Cc.x);
    }
    LineTwiddles<T, N> twl;
    twl.load(tw, t);
    cT<T>* xl = lds + pr * lds_line_elems(N);
    fft_line<T, N, +1, false>(v, xl, twl, t);   // begins with a barrier
    const int ra = row0 + 2 * pr, rb = ra + 1;
    T* dst = out + (int64_t)b * out_bs;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int x = t + m * TPL;
        if (x < nvx_out) {
            if (ra < nrows) dst[(int64_t)ra * out_ld + x] = v[m].x;
            if (rb < nrows) dst[(int64_t)rb * out_ld + x] = v[m].y;
        }
    }
}

// ---------------------------------------------------------------------------
// column transforms
// ---------------------------------------------------------------------------
template <int N> struct ColCfg {
    static constexpr int TPL = N / 8;
    static constexpr int CPW = TPL >= 256 ? 1 : 256 / TPL;   // columns per block
    static constexpr int THREADS = CPW * TPL;
};

// spectra from the FP64 generator: in[(l * ncols + kx) * N + y] (l = layer in
// batch) -> spec[((r0 + l) * ncols + kx) * N + ky] = FFT_y(in) * scale
template <typename T, int N>
__global__ void __launch_bounds__(ColCfg<N>::THREADS)
k_cols_spec(const double2* __restrict__ in, int ncols, cT<T>* __restrict__ spec, int r0, double scale,
            const double2* __restrict__ tw)
{
    using C = ColCfg<N>;
    constexpr int TPL = C::TPL;
    __shared__ double2 lds[C::CPW * lds_line_elems(N)];
    const int cl = threadIdx.x / TPL, t = threadIdx.x % TPL;
    const int col = blockIdx.x * C::CPW + cl;
    const int l = blockIdx.y;
    const bool ok = col < ncols;
    double2 v[8];
    const double2* src = in + ((int64_t)l * ncols + col) * N;
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = ok ? src[t + m * TPL] : make_double2(0.0, 0.0);
    LineTwiddles<double, N> twl;
    twl.load(tw, t);
    fft_line<double, N, -1, false>(v, lds + cl * lds_line_elems(N), twl, t);
    if (!ok) return;
    cT<T>* dst = spec + ((int64_t)(r0 + l) * ncols + col) * N;
#pragma unroll
    for (int m = 0; m < 8; ++m) dst[t + m * TPL] = mk<T>((T)(v[m].x * scale), (T)(v[m].y * scale));
}

// depth accumulators ------------------------------------------------------
template <typename T, int ACC> struct Acc;
template <typename T> struct Acc<T, ACC_PLAIN> {
    cT<T> s;
    __device__ __forceinline__ void zero() { s = mk<T>(0, 0); }
    __device__ __forceinline__ void add(cT<T> p) { s.x += p.x; s.y += p.y; }
    __device__ __forceinline__ cT<T> get() const { return s; }
};
// compensated (TwoSum) accumulation in the working precision
template <typename T> struct Acc<T, ACC_TWOSUM> {
    cT<T> s, c;
    __device__ __forceinline__ void zero() { s = mk<T>(0, 0); c = mk<T>(0, 0); }
    __device__ __forceinline__ static void two_sum(T& s, T& c, T p) {
        const T n = s + p;
        const T bp = n - s;
        const T e = (s - (n - bp)) + (p - bp);
        s = n;
        c += e;
    }
    __device__ __forceinline__ void add(cT<T> p) { two_sum(s.x, c.x, p.x); two_sum(s.y, c.y, p.y); }
    __device__ __forceinline__ cT<T> get() const { return mk<T>(s.x + c.x, s.y + c.y); }
};
// FP64 accumulation of FP32 products
template <typename T> struct Acc<T, ACC_WIDE> {
    double sx, sy;
    __device__ __forceinline__ void zero() { sx = 0.0; sy = 0.0; }
    __device__ __forceinline__ void add(cT<T> p) { sx += (double)p.x; sy += (double)p.y; }
    __device__ __forceinline__ cT<T> get() const { return mk<T>((T)sx, (T)sy); }
};

// forward: X[((q * nz + r) * ncols + kx) * ldx + y], y < ny (row-pass output);
// Y[(q * ncols + kx) * ldy + y], y < sy
template <typename T, int N, int NR, int ACC>
__global__ void __launch_bounds__(ColCfg<N>::THREADS)
k_cols_fwd_mac(const cT<T>* __restrict__ X, int64_t ldx, int ny, int nz, int ncols,
               const cT<T>* __restrict__ spec, cT<T>* __restrict__ Y, int64_t ldy, int sy,
               int nrhs, const cT<T>* __restrict__ tw)
{
    using C = ColCfg<N>;
    constexpr int TPL = C::TPL;
    __shared__ cT<T> lds[C::CPW * lds_line_elems(N)];
    const int cl = threadIdx.x / TPL, t = threadIdx.x % TPL;
    const int col = blockIdx.x * C::CPW + cl;
    const int q0 = blockIdx.y * NR;
    const bool ok = col < ncols;
    cT<T>* xl = lds + cl * lds_line_elems(N);
    LineTwiddles<T, N> twl;
    twl.load(tw, t);
    Acc<T, ACC> acc[NR][8];
#pragma unroll
    for (int q = 0; q < NR; ++q)
#pragma unroll
        for (int m = 0; m < 8; ++m) acc[q][m].zero();
    const bool zhi = ny <= N / 2;
    for (int r = 0; r < nz; ++r) {
        cT<T> tv[8];
        const cT<T>* sp = spec + ((int64_t)r * ncols + (ok ? col : 0)) * N;
#pragma unroll
        for (int m = 0; m < 8; ++m) tv[m] = ok ? sp[t + m * TPL] : mk<T>(0, 0);
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int qq = q0 + q;
            cT<T> v[8];
            const cT<T>* xs = X + (((int64_t)(qq < nrhs ? qq : 0) * nz + r) * ncols + (ok ? col : 0)) * ldx;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int y = t + m * TPL;
                v[m] = (ok && qq < nrhs && y < ny) ? xs[y] : mk<T>(0, 0);
            }
            if (zhi) fft_line<T, N, -1, true>(v, xl, twl, t);
            else fft_line<T, N, -1, false>(v, xl, twl, t);
#pragma unroll
            for (int m = 0; m < 8; ++m) acc[q][m].add(cmul<T>(tv[m], v[m]));
        }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const int qq = q0 + q;
        cT<T> v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = acc[q][m].get();
        fft_line<T, N, +1, false>(v, xl, twl, t);
        if (ok && qq < nrhs) {
            cT<T>* ys = Y + ((int64_t)qq * ncols + col) * ldy;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int y = t + m * TPL;
                if (y < sy) ys[y] = v[m];
            }
        }
    }
}

// transpose: R[(q * ncols + kx) * ldr + y], y < sy (row-pass output of the
// data); Z[((q * nz + r) * ncols + kx) * ldz + y], y < ny
template <typename T, int N, int NR>
__global__ void __launch_bounds__(ColCfg<N>::THREADS)
k_cols_tr_mac(const cT<T>* __restrict__ R, int64_t ldr, int sy, int nz, int ncols,
              const cT<T>* __restrict__ spec, cT<T>* __restrict__ Z, int64_t ldz, int ny,
              int nrhs, const cT<T>* __restrict__ tw)
{
    using C = ColCfg<N>;
    constexpr int TPL = C::TPL;
    __shared__ cT<T> lds[C::CPW * lds_line_elems(N)];
    const int cl = threadIdx.x / TPL, t = threadIdx.x % TPL;
    const int col = blockIdx.x * C::CPW + cl;
    const int q0 = blockIdx.y * NR;
    const bool ok = col < ncols;
    cT<T>* xl = lds + cl * lds_line_elems(N);
    LineTwiddles<T, N> twl;
    twl.load(tw, t);
    cT<T> rh[NR][8];
    const bool zhi = sy <= N / 2;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const int qq = q0 + q;
        const cT<T>* rs = R + ((int64_t)(qq < nrhs ? qq : 0) * ncols + (ok ? col : 0)) * ldr;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int y = t + m * TPL;
            rh[q][m] = (ok && qq < nrhs && y < sy) ? rs[y] : mk<T>(0, 0);
        }
        if (zhi) fft_line<T, N, -1, true>(rh[q], xl, twl, t);
        else fft_line<T, N, -1, false>(rh[q], xl, twl, t);
    }
    for (int r = 0; r < nz; ++r) {
        cT<T> tv[8];
        const cT<T>* sp = spec + ((int64_t)r * ncols + (ok ? col : 0)) * N;
#pragma unroll
        for (int m = 0; m < 8; ++m) tv[m] = ok ? sp[t + m * TPL] : mk<T>(0, 0);
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int qq = q0 + q;
            cT<T> v[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) v[m] = cmulc<T>(rh[q][m], tv[m]);
            fft_line<T, N, +1, false>(v, xl, twl, t);
            if (ok && qq < nrhs) {
                cT<T>* zs = Z + (((int64_t)qq * nz + r) * ncols + col) * ldz;
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int y = t + m * TPL;
                    if (y < ny) zs[y] = v[m];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// launchers (dispatch on the transform lengths)
// ---------------------------------------------------------------------------
#define BTTB_LEN_SWITCH(n, MACRO) \
    switch (n) {                  \
    case 8: MACRO(8); break;      \
    case 16: MACRO(16); break;    \
    case 32: MACRO(32); break;    \
    case 64: MACRO(64); break;    \
    case 128: MACRO(128); break;  \
    case 256: MACRO(256); break;  \
    case 512: MACRO(512); break;  \
    case 1024: MACRO(1024); break;\
    case 2048: MACRO(2048); break;\
    case 4096: MACRO(4096); break;\
    default: return hipErrorInvalidValue; }

hipError_t launch_twiddles(double2* t64, float2* t32, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_twiddles, dim3((n + 255) / 256), dim3(256), 0, s, t64, t32, n);
    return hipGetLastError();
}

hipError_t launch_generate(const GenParams& P, int r0, int nl, double* out, hipStream_t s)
{
    const int64_t per = (int64_t)P.Nx * P.Ny;
    dim3 grid((unsigned)((per + 255) / 256), (unsigned)nl);
    hipLaunchKernelGGL(k_generate, grid, dim3(256), 0, s, P, r0, out);
    return hipGetLastError();
}

template <typename TI, typename T>
hipError_t launch_rows_r2c(int N, const TI* in, int64_t in_bs, int64_t in_ld, int nvx, int nrows,
                           int nbatch, cT<T>* out, int64_t out_bs, int64_t out_ld, const cT<T>* tw,
                           hipStream_t s)
{
#define L_R2C(NN)                                                                          \
    {                                                                                      \
        using C = RowCfg<T, NN>;                                                           \
        const int bpb = (nrows + C::RT - 1) / C::RT;                                       \
        hipLaunchKernelGGL((k_rows_r2c<TI, T, NN>), dim3(bpb * nbatch), dim3(C::THREADS), 0, s, \
                           in, in_bs, in_ld, nvx, nrows, out, out_bs, out_ld, tw, bpb);    \
    }
    BTTB_LEN_SWITCH(N, L_R2C)
#undef L_R2C
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rows_c2r(int N, const cT<T>* in, int64_t in_bs, int64_t in_ld, int nrows,
                           int nbatch, T* out, int64_t out_bs, int64_t out_ld, int nvx_out,
                           const cT<T>* tw, hipStream_t s)
{
#define L_C2R(NN)                                                                          \
    {                                                                                      \
        using C = RowCfg<T, NN>;                                                           \
        const int bpb = (nrows + C::RT - 1) / C::RT;                                       \
        hipLaunchKernelGGL((k_rows_c2r<T, NN>), dim3(bpb * nbatch), dim3(C::THREADS), 0, s, \
                           in, in_bs, in_ld, nrows, out, out_bs, out_ld, nvx_out, tw, bpb); \
    }
    BTTB_LEN_SWITCH(N, L_C2R)
#undef L_C2R
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cols_spec(int N, const double2* in, int ncols, int nl, cT<T>* spec, int r0,
                            double scale, const double2* tw, hipStream_t s)
{
#define L_SPEC(NN)                                                                         \
    {                                                                                      \
        using C = ColCfg<NN>;                                                              \
        dim3 grid((ncols + C::CPW - 1) / C::CPW, nl);                                      \
        hipLaunchKernelGGL((k_cols_spec<T, NN>), grid, dim3(C::THREADS), 0, s, in, ncols, spec, \
                           r0, scale, tw);                                                 \
    }
    BTTB_LEN_SWITCH(N, L_SPEC)
#undef L_SPEC
    return hipGetLastError();
}

template <typename T, int ACC>
hipError_t launch_cols_fwd(int N, const cT<T>* X, int64_t ldx, int ny, int nz, int ncols,
                           const cT<T>* spec, cT<T>* Y, int64_t ldy, int sy, int nrhs,
                           const cT<T>* tw, hipStream_t s)
{
    const int NR = 1;
#define L_FWD(NN)                                                                          \
    {                                                                                      \
        using C = ColCfg<NN>;                                                              \
        dim3 grid((ncols + C::CPW - 1) / C::CPW, (nrhs + NR - 1) / NR);                    \
        hipLaunchKernelGGL((k_cols_fwd_mac<T, NN, 1, ACC>), grid, dim3(C::THREADS), 0, s, X, ldx, \
                           ny, nz, ncols, spec, Y, ldy, sy, nrhs, tw);                     \
    }
    BTTB_LEN_SWITCH(N, L_FWD)
#undef L_FWD
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cols_tr(int N, const cT<T>* R, int64_t ldr, int sy, int nz, int ncols,
                          const cT<T>* spec, cT<T>* Z, int64_t ldz, int ny, int nrhs,
                          const cT<T>* tw, hipStream_t s)
{
    const int NR = 1;
#define L_TR(NN)                                                                           \
    {                                                                                      \
        using C = ColCfg<NN>;                                                              \
        dim3 grid((ncols + C::CPW - 1) / C::CPW, (nrhs + NR - 1) / NR);                    \
        hipLaunchKernelGGL((k_cols_tr_mac<T, NN, 1>), grid, dim3(C::THREADS), 0, s, R, ldr, sy, \
                           nz, ncols, spec, Z, ldz, ny, nrhs, tw);                         \
    }
    BTTB_LEN_SWITCH(N, L_TR)
#undef L_TR
    return hipGetLastError();
}

// explicit instantiations used by the host code
template hipError_t launch_rows_r2c<double, double>(int, const double*, int64_t, int64_t, int, int, int,
                                                    double2*, int64_t, int64_t, const double2*, hipStream_t);
template hipError_t launch_rows_r2c<float, float>(int, const float*, int64_t, int64_t, int, int, int,
                                                  float2*, int64_t, int64_t, const float2*, hipStream_t);
template hipError_t launch_rows_c2r<double>(int, const double2*, int64_t, int64_t, int, int, double*,
                                            int64_t, int64_t, int, const double2*, hipStream_t);
template hipError_t launch_rows_c2r<float>(int, const float2*, int64_t, int64_t, int, int, float*,
                                           int64_t, int64_t, int, const float2*, hipStream_t);
template hipError_t launch_cols_spec<double>(int, const double2*, int, int, double2*, int, double,
                                             const double2*, hipStream_t);
template hipError_t launch_cols_spec<float>(int, const double2*, int, int, float2*, int, double,
                                            const double2*, hipStream_t);
template hipError_t launch_cols_fwd<double, ACC_PLAIN>(int, const double2*, int64_t, int, int, int,
                                                       const double2*, double2*, int64_t, int, int,
                                                       const double2*, hipStream_t);
template hipError_t launch_cols_fwd<float, ACC_PLAIN>(int, const float2*, int64_t, int, int, int,
                                                      const float2*, float2*, int64_t, int, int,
                                                      const float2*, hipStream_t);
template hipError_t launch_cols_fwd<float, ACC_TWOSUM>(int, const float2*, int64_t, int, int, int,
                                                       const float2*, float2*, int64_t, int, int,
                                                       const float2*, hipStream_t);
template hipError_t launch_cols_fwd<float, ACC_WIDE>(int, const float2*, int64_t, int, int, int,
                                                     const float2*, float2*, int64_t, int, int,
                                                     const float2*, hipStream_t);
template hipError_t launch_cols_tr<double>(int, const double2*, int64_t, int, int, int, const double2*,
                                           double2*, int64_t, int, int, const double2*, hipStream_t);
template hipError_t launch_cols_tr<float>(int, const float2*, int64_t, int, int, int, const float2*,
                                          float2*, int64_t, int, int, const float2*, hipStream_t);

}  // namespace bttbk
