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

#include <algorithm>
#include <cstdio>
#include <cstdlib>

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
// half-spectrum format
// ---------------------------------------------------------------------------
// The x transform of a real row of even length N has N/2 + 1 distinct bins;
// bins 0 and N/2 are real.  Every half spectrum is stored "packed" as N/2
// complex values: slot 0 holds (X[0], X[N/2]) as (real, imaginary) and slot
// k in [1, N/2) holds X[k].  Along y, the packed slot-0 column is then the
// sum A + i B of two real sequences, whose transforms are Hermitian; the
// column kernels separate them with the mirror index -k when they need them
// individually (block 0 only).  The number of columns is exactly N/2.

// hardware block b -> logical block such that the blocks that the hardware
// places on one XCD (b mod 8) get consecutive logical indices
__device__ __forceinline__ int xcd_order(int b, int G)
{
    const int xcd = b & 7, k = b >> 3;
    const int per = G >> 3, rem = G & 7;
    return xcd < rem ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

// ---------------------------------------------------------------------------
// row transforms
// ---------------------------------------------------------------------------
// P0: pairs of rows per block for long rows (a tuning choice, 2 or 4)
template <typename T, int N, int P0 = 4> struct RowCfg {
    static constexpr int TPL = N / 8;
    static constexpr int PAIRS = sizeof(T) == 4 ? (N <= 2048 ? (256 / TPL > P0 ? 256 / TPL : P0) : 2)
                                                : (N <= 1024 ? (256 / TPL > P0 ? 256 / TPL : P0)
                                                             : (N == 2048 ? 2 : 1));
    static constexpr int RT = 2 * PAIRS;            // rows per block
    static constexpr int THREADS = PAIRS * TPL;
    static constexpr int HALF = N / 2;              // packed half-spectrum columns
    static constexpr int SROW = RT + 1;             // padded staging row
    static constexpr int STAGE = HALF * SROW;
    static constexpr int XCH = PAIRS * lds_line_elems(N);
    static constexpr int LDS = STAGE > XCH ? STAGE : XCH;
    static constexpr int TWO = LDS;                 // offset of the LDS twiddle table
};

// Row kernels are persistent: gridDim.x blocks (about the number that fit on
// the device at once) walk over the row groups g = lb, lb + G, lb + 2G, ...
// (lb = XCD-ordered block index, so neighbouring groups, which share 128-byte
// lines of the column-major half spectra, run on one XCD at the same time).
// The loads of the next group are issued before the current group is
// transformed, so memory latency overlaps the FFT.

// index of the job whose work range [begin, next begin) contains w
template <typename JT> __device__ __forceinline__ int find_job(const JT& js, int w)
{
    int k = 0;
    for (int i = 1; i < js.njobs; ++i)
        if (w >= js.j[i].begin) k = i;
    return k;
}

// Row transform, real -> packed half spectra, over every job of the table.
// Job input: batch b, row y, column x at in[b * in_bs + y * in_ld + x],
// x < nv valid (zero beyond, up to N); output: packed half spectra at
// out[b * out_bs + kx * out_ld + y], kx < N/2, y < nrows.
template <typename TI, typename T, int N, int P0>
__global__ void __launch_bounds__((RowCfg<T, N, P0>::THREADS))
k_rows_r2c(RowJobs jobs, const cT<T>* __restrict__ tw)
{
    using C = RowCfg<T, N, P0>;
    constexpr int TPL = C::TPL;
    __shared__ cT<T> lds[C::LDS + TableTwiddles<T, N>::size()];
    const int G = gridDim.x, total = jobs.total;
    const int pr = threadIdx.x / TPL, t = threadIdx.x % TPL;
    TableTwiddles<T, N>::build(lds + C::TWO, tw, threadIdx.x, C::THREADS);
    __syncthreads();
    const TableTwiddles<T, N> twl{lds + C::TWO};
    cT<T>* xl = lds + pr * lds_line_elems(N);
    auto load = [&](int g, cT<T> (&v)[8]) {
        const RowJob& J = jobs.j[find_job(jobs, g)];
        const int gl = g - J.begin;
        const int b = gl / J.bpb;
        const int ra = (gl % J.bpb) * C::RT + 2 * pr, rb = ra + 1;
        const TI* src = (const TI*)J.in + (int64_t)b * J.in_bs;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int x = t + m * TPL;
            T a = 0, c = 0;
            if (x < J.nv) {
                if (ra < J.nrows) a = (T)src[(int64_t)ra * J.in_ld + x];
                if (rb < J.nrows) c = (T)src[(int64_t)rb * J.in_ld + x];
            }
            v[m] = mk<T>(a, c);
        }
    };
    int g = xcd_order(blockIdx.x, G);
    cT<T> v[8];
    if (g < total) load(g, v);
    for (; g < total; g += G) {
        cT<T> vn[8];
        if (g + G < total) load(g + G, vn);
        const RowJob& J = jobs.j[find_job(jobs, g)];
        const int gl = g - J.begin;
        const int b = gl / J.bpb;
        const int row0 = (gl % J.bpb) * C::RT;
        if (J.nv <= N / 2) fft_line<T, N, -1, true>(v, xl, twl, t);
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
        if (t == 0) {   // pack the real bins 0 and N/2 into slot 0
            A[0] = mk<T>(A[0].x, A[4].x);
            Cc[0] = mk<T>(Cc[0].x, Cc[4].x);
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int k = t + m * TPL;
            lds[k * C::SROW + 2 * pr] = A[m];
            lds[k * C::SROW + 2 * pr + 1] = Cc[m];
        }
        __syncthreads();
        cT<T>* dst = (cT<T>*)J.out + (int64_t)b * J.out_bs;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = threadIdx.x + i * C::THREADS;   // HALF * RT = 8 * THREADS
            const int kx = e / C::RT, rr = e % C::RT;
            if (row0 + rr < J.nrows) dst[(int64_t)kx * J.out_ld + row0 + rr] = lds[kx * C::SROW + rr];
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = vn[m];
    }
}

// Row transform, packed half spectra -> real rows, over every job of the
// table.  Job input: in[b * in_bs + kx * in_ld + y], kx < N/2, y < nrows;
// output: out[b * out_bs + y * out_ld + x] for x < nv (real, unnormalised
// inverse transform; the 1/(Nx Ny) factor lives in the spectra).
template <typename T, int N, int P0>
__global__ void __launch_bounds__((RowCfg<T, N, P0>::THREADS))
k_rows_c2r(RowJobs jobs, const cT<T>* __restrict__ tw)
{
    using C = RowCfg<T, N, P0>;
    constexpr int TPL = C::TPL;
    __shared__ cT<T> lds[C::LDS + TableTwiddles<T, N>::size()];
    const int G = gridDim.x, total = jobs.total;
    const int pr = threadIdx.x / TPL, t = threadIdx.x % TPL;
    TableTwiddles<T, N>::build(lds + C::TWO, tw, threadIdx.x, C::THREADS);
    __syncthreads();
    const TableTwiddles<T, N> twl{lds + C::TWO};
    cT<T>* xl = lds + pr * lds_line_elems(N);
    // tile of the packed half spectra of RT rows: HALF * RT = 8 * THREADS
    // elements, element e = threadIdx.x + i THREADS at (kx, row) = (e / RT, e % RT)
    auto load = [&](int g, cT<T> (&tl)[8]) {
        const RowJob& J = jobs.j[find_job(jobs, g)];
        const int gl = g - J.begin;
        const int b = gl / J.bpb;
        const int row0 = (gl % J.bpb) * C::RT;
        const cT<T>* src = (const cT<T>*)J.in + (int64_t)b * J.in_bs;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = threadIdx.x + i * C::THREADS;
            const int kx = e / C::RT, rr = e % C::RT;
            tl[i] = (row0 + rr < J.nrows) ? src[(int64_t)kx * J.in_ld + row0 + rr] : mk<T>(0, 0);
        }
    };
    int g = xcd_order(blockIdx.x, G);
    cT<T> tl[8];
    if (g < total) load(g, tl);
    for (; g < total; g += G) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = threadIdx.x + i * C::THREADS;
            lds[(e / C::RT) * C::SROW + e % C::RT] = tl[i];
        }
        __syncthreads();
        if (g + G < total) load(g + G, tl);
        // Z[k] = A[k] + i C[k] over the full length: slot 0 unpacks the real
        // bins 0 and N/2, Hermitian symmetry gives k > N/2
        cT<T> v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int k = t + m * TPL;
            const int kk = k <= N / 2 ? k : N - k;
            cT<T> A, Cc;
            if (kk == 0 || kk == N / 2) {
                const cT<T> pa = lds[2 * pr], pc = lds[2 * pr + 1];
                A = mk<T>(kk == 0 ? pa.x : pa.y, 0);
                Cc = mk<T>(kk == 0 ? pc.x : pc.y, 0);
            } else {
                A = lds[kk * C::SROW + 2 * pr];
                Cc = lds[kk * C::SROW + 2 * pr + 1];
                if (k > N / 2) { A.y = -A.y; Cc.y = -Cc.y; }
            }
            v[m] = mk<T>(A.x - Cc.y, A.y + Cc.x);
        }
        fft_line<T, N, +1, false>(v, xl, twl, t);   // begins with a barrier
        const RowJob& J = jobs.j[find_job(jobs, g)];
        const int gl = g - J.begin;
        const int b = gl / J.bpb;
        const int ra = (gl % J.bpb) * C::RT + 2 * pr, rb = ra + 1;
        T* dst = (T*)J.out + (int64_t)b * J.out_bs;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int x = t + m * TPL;
            if (x < J.nv) {
                if (ra < J.nrows) dst[(int64_t)ra * J.out_ld + x] = v[m].x;
                if (rb < J.nrows) dst[(int64_t)rb * J.out_ld + x] = v[m].y;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// row transforms, tile-per-thread variant (row tile 8)
// ---------------------------------------------------------------------------
// A tile is 8 consecutive rows of one batch.  The TPL = N/8 threads of a
// tile each hold, for their 8 positions x = t + m TPL, the values of all 8
// rows; the 4 packed pairs of rows are transformed one after another through
// one LDS line buffer, and every thread writes (r2c) or reads (c2r) the 8
// rows of each of its half-spectrum columns as one contiguous 8-element
// segment of the column-major layout, straight from registers.  No staging
// tile is needed, so the LDS per block is one line buffer and the twiddle
// table, and several independent blocks share a CU.
template <int N> struct TileCfg {
    static constexpr int TPL = N / 8;
    static constexpr int LPB = TPL >= 256 ? 1 : 256 / TPL;   // tiles per block
    static constexpr int THREADS = LPB * TPL;
};

template <typename TI, typename T, int N>
__global__ void __launch_bounds__(TileCfg<N>::THREADS)
k_rows_r2c_t(RowJobs jobs, const cT<T>* __restrict__ tw)
{
    using C = TileCfg<N>;
    constexpr int TPL = C::TPL;
    constexpr int LL = lds_line_elems(N);
    __shared__ cT<T> lds[C::LPB * LL + TableTwiddles<T, N>::size()];
    TableTwiddles<T, N>::build(lds + C::LPB * LL, tw, threadIdx.x, C::THREADS);
    __syncthreads();
    const TableTwiddles<T, N> twl{lds + C::LPB * LL};
    const int tl = threadIdx.x / TPL, t = threadIdx.x % TPL;
    cT<T>* xl = lds + tl * LL;
    const int total = jobs.total;
    const int nb = (total + C::LPB - 1) / C::LPB;           // block-level iterations
    for (int gb = xcd_order(blockIdx.x, gridDim.x); gb < nb; gb += gridDim.x) {
        const int g = gb * C::LPB + tl;
        const bool live = g < total;
        const RowJob& J = jobs.j[find_job(jobs, live ? g : 0)];
        const int gl = (live ? g : 0) - J.begin;
        const int b = gl / J.bpb, row0 = (gl % J.bpb) * 8;
        const TI* src = (const TI*)J.in + (int64_t)b * J.in_bs;
        T a[8][8];
#pragma unroll
        for (int rr = 0; rr < 8; ++rr)
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int x = t + m * TPL;
                a[rr][m] = (live && x < J.nv && row0 + rr < J.nrows) ? (T)src[(int64_t)(row0 + rr) * J.in_ld + x] : (T)0;
            }
        cT<T> o[4][8];   // o[m][row]: half-spectrum value at k = t + m TPL
        cT<T> o0n[2];    // bin N/2 of the pair's two rows (thread 0)
        const bool zhi = J.nv <= N / 2;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            cT<T> v[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) v[m] = mk<T>(a[2 * p][m], a[2 * p + 1][m]);
            if (zhi) fft_line<T, N, -1, true>(v, xl, twl, t);
            else fft_line<T, N, -1, false>(v, xl, twl, t);
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 8; ++m) xl[lpad(t + m * TPL)] = v[m];
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                const int k = t + m * TPL;
                if (m < 4 || t == 0) {
                    const cT<T> z = v[m], zr = xl[lpad((N - k) & (N - 1))];
                    const cT<T> A = mk<T>((T)0.5 * (z.x + zr.x), (T)0.5 * (z.y - zr.y));
                    const cT<T> Cc = mk<T>((T)0.5 * (z.y + zr.y), (T)0.5 * (zr.x - z.x));
                    if (m < 4) {
                        o[m][2 * p] = A;
                        o[m][2 * p + 1] = Cc;
                    } else {
                        o0n[0] = A;
                        o0n[1] = Cc;
                    }
                }
            }
            if (t == 0) {   // pack the real bins 0 and N/2 into slot 0
                o[0][2 * p] = mk<T>(o[0][2 * p].x, o0n[0].x);
                o[0][2 * p + 1] = mk<T>(o[0][2 * p + 1].x, o0n[1].x);
            }
        }
        if (live) {
            cT<T>* dst = (cT<T>*)J.out + (int64_t)b * J.out_bs;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                cT<T>* col = dst + (int64_t)(t + m * TPL) * J.out_ld + row0;
#pragma unroll
                for (int rr = 0; rr < 8; ++rr)
                    if (row0 + rr < J.nrows) col[rr] = o[m][rr];
            }
        }
    }
}

template <typename T, int N>
__global__ void __launch_bounds__(TileCfg<N>::THREADS)
k_rows_c2r_t(RowJobs jobs, const cT<T>* __restrict__ tw)
{
    using C = TileCfg<N>;
    constexpr int TPL = C::TPL;
    constexpr int LL = lds_line_elems(N);
    __shared__ cT<T> lds[C::LPB * LL + TableTwiddles<T, N>::size()];
    TableTwiddles<T, N>::build(lds + C::LPB * LL, tw, threadIdx.x, C::THREADS);
    __syncthreads();
    const TableTwiddles<T, N> twl{lds + C::LPB * LL};
    const int tl = threadIdx.x / TPL, t = threadIdx.x % TPL;
    cT<T>* xl = lds + tl * LL;
    const int total = jobs.total;
    const int nb = (total + C::LPB - 1) / C::LPB;
    for (int gb = xcd_order(blockIdx.x, gridDim.x); gb < nb; gb += gridDim.x) {
        const int g = gb * C::LPB + tl;
        const bool live = g < total;
        const RowJob& J = jobs.j[find_job(jobs, live ? g : 0)];
        const int gl = (live ? g : 0) - J.begin;
        const int b = gl / J.bpb, row0 = (gl % J.bpb) * 8;
        const cT<T>* src = (const cT<T>*)J.in + (int64_t)b * J.in_bs;
        cT<T> c[4][8];   // c[m][row]: packed half spectrum at k = t + m TPL
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const cT<T>* col = src + (int64_t)(t + m * TPL) * J.in_ld + row0;
#pragma unroll
            for (int rr = 0; rr < 8; ++rr) c[m][rr] = (live && row0 + rr < J.nrows) ? col[rr] : mk<T>(0, 0);
        }
        T* dst = (T*)J.out + (int64_t)b * J.out_bs;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            // the pair's half spectra A (row 2p) and C (row 2p+1) at k < N/2
            // go through LDS so that each thread can read its mirror positions
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                xl[lpad(t + m * TPL)] = c[m][2 * p];
                xl[lpad(N / 2 + t + m * TPL)] = c[m][2 * p + 1];
            }
            __syncthreads();
            cT<T> v[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int k = t + m * TPL;
                cT<T> A, Cc;
                if (k == 0 || k == N / 2) {
                    const cT<T> pa = xl[lpad(0)], pc = xl[lpad(N / 2)];
                    A = mk<T>(k == 0 ? pa.x : pa.y, 0);
                    Cc = mk<T>(k == 0 ? pc.x : pc.y, 0);
                } else if (k < N / 2) {
                    A = c[m][2 * p];
                    Cc = c[m][2 * p + 1];
                } else {
                    A = xl[lpad(N - k)];
                    Cc = xl[lpad(N / 2 + N - k)];
                    A.y = -A.y;
                    Cc.y = -Cc.y;
                }
                v[m] = mk<T>(A.x - Cc.y, A.y + Cc.x);
            }
            fft_line<T, N, +1, false>(v, xl, twl, t);   // begins with a barrier
            const int ra = row0 + 2 * p, rb = ra + 1;
            if (live) {
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int x = t + m * TPL;
                    if (x < J.nv) {
                        if (ra < J.nrows) dst[(int64_t)ra * J.out_ld + x] = v[m].x;
                        if (rb < J.nrows) dst[(int64_t)rb * J.out_ld + x] = v[m].y;
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// column transforms
// ---------------------------------------------------------------------------
// minimum waves per SIMD requested for the column kernels (bounds the VGPRs
// the compiler may use: 512 / waves)
#ifndef BTTB_COL_WAVES
#define BTTB_COL_WAVES 2
#endif
// CM: multiplier of the columns per block (a tuning choice, 1 or 2)
template <int N, int CM = 1> struct ColCfg {
    static constexpr int TPL = N / 8;
    static constexpr int CPW = (TPL >= 256 ? 1 : 256 / TPL) * CM;   // columns per block
    static constexpr int THREADS = CPW * TPL;
};

// spectra from the FP64 generator: in[(l * ncols + kx) * N + y] (l = layer in
// batch, packed half spectra along x) -> spec[((r0 + l) * ncols + kx) * N + ky]
// = FFT_y(in) * scale (column 0 becomes T^[0] + i T^[N/2], the packed pair of
// Hermitian columns)
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
    const double2* src = in + ((int64_t)l * ncols + (ok ? col : 0)) * N;
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

// Column 0 of the packed format holds z = A + i B with A, B the transforms
// of two real sequences (Hermitian).  With zr = z at -k:
//   A = (z + conj zr) / 2,  B = (z - conj zr) / (2 i).
template <typename T> __device__ __forceinline__ cT<T> herm_a(cT<T> z, cT<T> zr) {
    return mk<T>((T)0.5 * (z.x + zr.x), (T)0.5 * (z.y - zr.y));
}
template <typename T> __device__ __forceinline__ cT<T> herm_b(cT<T> z, cT<T> zr) {
    return mk<T>((T)0.5 * (z.y + zr.y), (T)0.5 * (zr.x - z.x));
}

// Store two register lines (positions t + m TPL) into two LDS line buffers so
// that their values at the mirror positions -k can be read back one at a
// time.  Contains barriers: every thread of the block calls it; only
// `active` threads write.
template <typename T, int N>
__device__ __forceinline__ void stage_pair(const cT<T> (&u)[8], const cT<T> (&w)[8], cT<T>* bu, cT<T>* bw,
                                           int t, bool active)
{
    constexpr int TPL = N / 8;
    __syncthreads();
    if (active) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            bu[lpad(t + m * TPL)] = u[m];
            bw[lpad(t + m * TPL)] = w[m];
        }
    }
    __syncthreads();
}
template <int N> __device__ __forceinline__ int mirror_idx(int t, int m) {
    return lpad((N - t - m * (N / 8)) & (N - 1));
}

// Forward column pass over every job of the table (one block per CPW
// columns of one right-hand-side block of one job).  Job: a = X with
// X[((q * nz + r) * ncols + kx) * lda + y], y < na = ny (packed row-pass
// output), nl = nz layers; b = Y with Y[(q * ncols + kx) * ldb + y], y < nb = sy.
template <typename T, int N, int NR, int ACC, int CM>
__global__ void __launch_bounds__((ColCfg<N, CM>::THREADS), BTTB_COL_WAVES)
k_cols_fwd_mac(ColJobs jobs, const cT<T>* __restrict__ tw)
{
    using C = ColCfg<N, CM>;
    constexpr int TPL = C::TPL;
    constexpr int LL = lds_line_elems(N);
    __shared__ cT<T> lds[(C::CPW + 1) * LL];
    const ColJob& J = jobs.j[find_job(jobs, blockIdx.x)];
    const cT<T>* __restrict__ X = (const cT<T>*)J.a;
    const cT<T>* __restrict__ spec = (const cT<T>*)J.spec;
    cT<T>* __restrict__ Y = (cT<T>*)J.b;
    const int64_t ldx = J.lda, ldy = J.ldb;
    const int ny = J.na, sy = J.nb, nz = J.nl, ncols = J.ncols, nrhs = J.nrhs;
    const int lb = blockIdx.x - J.begin, cb = lb % J.nbx;
    const int cl = threadIdx.x / TPL, t = threadIdx.x % TPL;
    const int col = cb * C::CPW + cl;
    const int q0 = (lb / J.nbx) * NR;
    const bool ok = col < ncols;
    const bool packed_blk = cb == 0;              // block holding column 0
    const bool packed = packed_blk && cl == 0;
    cT<T>* xl = lds + cl * LL;
    cT<T>* xs2 = lds + C::CPW * LL;               // second buffer (column 0)
    LineTwiddles<T, N> twl;
    twl.load(tw, t);
    Acc<T, ACC> acc[NR][8];
#pragma unroll
    for (int q = 0; q < NR; ++q)
#pragma unroll
        for (int m = 0; m < 8; ++m) acc[q][m].zero();
    const bool zhi = ny <= N / 2;
    const int ccol = ok ? col : 0;
    // software pipeline: the next layer's spectra and input columns are
    // loaded while the current layer is transformed
    cT<T> tn[8], xn[NR][8];
    auto load_layer = [&](int r) {
        const cT<T>* sp = spec + ((int64_t)r * ncols + ccol) * N;
#pragma unroll
        for (int m = 0; m < 8; ++m) tn[m] = sp[t + m * TPL];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int qq = q0 + q;
            const cT<T>* xs = X + (((int64_t)(qq < nrhs ? qq : 0) * nz + r) * ncols + ccol) * ldx;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int y = t + m * TPL;
                xn[q][m] = (ok && qq < nrhs && y < ny) ? xs[y] : mk<T>(0, 0);
            }
        }
    };
    load_layer(0);
    for (int r = 0; r < nz; ++r) {
        cT<T> tv[8], v[NR][8];
#pragma unroll
        for (int m = 0; m < 8; ++m) tv[m] = tn[m];
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int m = 0; m < 8; ++m) v[q][m] = xn[q][m];
        if (r + 1 < nz) load_layer(r + 1);
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            if (zhi) fft_line<T, N, -1, true>(v[q], xl, twl, t);
            else fft_line<T, N, -1, false>(v[q], xl, twl, t);
            if (packed_blk) {
                stage_pair<T, N>(v[q], tv, xl, xs2, t, packed);
                if (packed) {
                    // column 0 carries bins 0 and N/2: accumulate
                    // T0 F0 + i T1 F1 of the separated Hermitian parts
#pragma unroll
                    for (int m = 0; m < 8; ++m) {
                        const int mi = mirror_idx<N>(t, m);
                        const cT<T> vr = xl[mi], tr = xs2[mi];
                        const cT<T> p0 = cmul<T>(herm_a<T>(tv[m], tr), herm_a<T>(v[q][m], vr));
                        const cT<T> p1 = cmul<T>(herm_b<T>(tv[m], tr), herm_b<T>(v[q][m], vr));
                        acc[q][m].add(mk<T>(p0.x - p1.y, p0.y + p1.x));
                    }
                    continue;
                }
            }
#pragma unroll
            for (int m = 0; m < 8; ++m) acc[q][m].add(cmul<T>(tv[m], v[q][m]));
        }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const int qq = q0 + q;
        cT<T> w[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) w[m] = acc[q][m].get();
        fft_line<T, N, +1, false>(w, xl, twl, t);
        if (ok && qq < nrhs) {
            cT<T>* ys = Y + ((int64_t)qq * ncols + col) * ldy;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int y = t + m * TPL;
                if (y < sy) ys[y] = w[m];
            }
        }
    }
}

// Transpose column pass over every job of the table, layers [r0, r0 + nl).
// Job: a = R with R[(q * ncols + kx) * lda + y], y < na = sy (packed row-pass
// output of the data); b = Z with Z[((q * nl + r - r0) * ncols + kx) * ldb + y],
// y < nb = ny.
// The kernel is persistent and balanced: the work of all jobs is the list of
// units (job, right-hand side q, column block cb, layer l), layer fastest,
// and block w processes the contiguous range [w U / G, (w + 1) U / G).  A
// block recomputes R^ = FFT_y(R) whenever its range enters a new column
// block (at most a few times), so every block gets the same number of layers
// whatever the number of resident blocks.
template <typename T, int N, int NR, int CM>
__global__ void __launch_bounds__((ColCfg<N, CM>::THREADS), BTTB_COL_WAVES)
k_cols_tr_mac(ColJobs jobs, const cT<T>* __restrict__ tw)
{
    using C = ColCfg<N, CM>;
    constexpr int TPL = C::TPL;
    constexpr int LL = lds_line_elems(N);
    __shared__ cT<T> lds[(C::CPW + 1) * LL];
    const int cl = threadIdx.x / TPL, t = threadIdx.x % TPL;
    cT<T>* xl = lds + cl * LL;
    cT<T>* xs2 = lds + C::CPW * LL;
    LineTwiddles<T, N> twl;
    twl.load(tw, t);
    const int64_t U = jobs.total, G = gridDim.x;
    const int u0 = (int)((int64_t)blockIdx.x * U / G), u1 = (int)((int64_t)(blockIdx.x + 1) * U / G);
    // unit u -> (job k, key = q * nbx + cb, layer l)
    auto decode = [&](int u, int& k, int& key, int& l) {
        k = find_job(jobs, u);
        const int lu = u - jobs.j[k].begin;
        l = lu % jobs.j[k].nl;
        key = lu / jobs.j[k].nl;
    };
    cT<T> tn[8];
    auto load_spec = [&](int u) {
        int k, key, l;
        decode(u, k, key, l);
        const ColJob& J = jobs.j[k];
        const int col = (key % J.nbx) * C::CPW + cl;
        const cT<T>* sp = (const cT<T>*)J.spec + ((int64_t)(J.r0 + l) * J.ncols + (col < J.ncols ? col : 0)) * N;
#pragma unroll
        for (int m = 0; m < 8; ++m) tn[m] = sp[t + m * TPL];
    };
    int cur_k = -1, cur_key = -1;
    cT<T> rh[8];
    if (u0 < u1) load_spec(u0);
    for (int u = u0; u < u1; ++u) {
        int k, key, l;
        decode(u, k, key, l);
        const ColJob& J = jobs.j[k];
        const int cb = key % J.nbx, q = key / J.nbx;
        const int col = cb * C::CPW + cl;
        const bool ok = col < J.ncols;
        const bool packed_blk = cb == 0;
        const bool packed = packed_blk && cl == 0;
        cT<T> tv[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) tv[m] = tn[m];
        if (u + 1 < u1) load_spec(u + 1);
        if (k != cur_k || key != cur_key) {
            // R^ of this column: FFT_y of the packed row-pass output of the data
            const cT<T>* rs = (const cT<T>*)J.a + ((int64_t)q * J.ncols + (ok ? col : 0)) * J.lda;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int y = t + m * TPL;
                rh[m] = (ok && y < J.na) ? rs[y] : mk<T>(0, 0);
            }
            if (J.na <= N / 2) fft_line<T, N, -1, true>(rh, xl, twl, t);
            else fft_line<T, N, -1, false>(rh, xl, twl, t);
            cur_k = k;
            cur_key = key;
        }
        cT<T> v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = cmulc<T>(rh[m], tv[m]);
        if (packed_blk) {
            stage_pair<T, N>(rh, tv, xl, xs2, t, packed);
            if (packed) {
                // column 0: conj(T0) R0 + i conj(T1) R1
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int mi = mirror_idx<N>(t, m);
                    const cT<T> rr = xl[mi], tr = xs2[mi];
                    const cT<T> p0 = cmulc<T>(herm_a<T>(rh[m], rr), herm_a<T>(tv[m], tr));
                    const cT<T> p1 = cmulc<T>(herm_b<T>(rh[m], rr), herm_b<T>(tv[m], tr));
                    v[m] = mk<T>(p0.x - p1.y, p0.y + p1.x);
                }
            }
        }
        fft_line<T, N, +1, false>(v, xl, twl, t);
        if (ok) {
            cT<T>* zs = (cT<T>*)J.b + (((int64_t)q * J.nl + l) * J.ncols + col) * J.ldb;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int y = t + m * TPL;
                if (y < J.nb) zs[y] = v[m];
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

// blocks of `kernel` that are resident on the whole current device at once
// (occupancy per CU times the number of CUs); at least 1
static int resident_blocks(const void* kernel, int threads)
{
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) { (void)hipGetLastError(); return 256; }
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        ncu = 256;
    }
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0);
    if (e != hipSuccess || per < 1) {
        // a failed query must not leave its error for the launch check
        (void)hipGetLastError();
        if (std::getenv("BTTB_DEBUG"))
            std::fprintf(stderr, "bttb: occupancy query failed (%s, per=%d, threads=%d)\n", hipGetErrorString(e),
                         per, threads);
        per = 1;
    }
    return std::max(1, ncu * per);
}

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

template <typename T> int row_group_rows(int N, int tile)
{
    if (tile == 8) return 8;
#define L_RT(NN) return tile == 1 ? RowCfg<T, NN, 1>::RT : tile == 2 ? RowCfg<T, NN, 2>::RT : RowCfg<T, NN, 4>::RT;
    switch (N) {
    case 8: L_RT(8) case 16: L_RT(16) case 32: L_RT(32) case 64: L_RT(64) case 128: L_RT(128)
    case 256: L_RT(256) case 512: L_RT(512) case 1024: L_RT(1024) case 2048: L_RT(2048)
    case 4096: L_RT(4096) default: return 1;
    }
#undef L_RT
}
template int row_group_rows<float>(int, int);
template int row_group_rows<double>(int, int);

// a column tile of 2 is used only where its LDS fits in 160 KB
template <typename T, int NN> constexpr bool col_tile2_fits()
{
    return (ColCfg<NN, 2>::CPW + 1) * lds_line_elems(NN) * (int)sizeof(cT<T>) <= 160 * 1024;
}

template <typename T> int col_block_lines(int N, int tile)
{
#define L_CB(NN) return (tile == 2 && col_tile2_fits<T, NN>()) ? ColCfg<NN, 2>::CPW : ColCfg<NN, 1>::CPW;
    switch (N) {
    case 8: L_CB(8) case 16: L_CB(16) case 32: L_CB(32) case 64: L_CB(64) case 128: L_CB(128)
    case 256: L_CB(256) case 512: L_CB(512) case 1024: L_CB(1024) case 2048: L_CB(2048)
    case 4096: L_CB(4096) default: return 1;
    }
#undef L_CB
}
template int col_block_lines<float>(int, int);
template int col_block_lines<double>(int, int);

template <typename TI, typename T, int NN, int P0>
static hipError_t launch_r2c_n(const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    using C = RowCfg<T, NN, P0>;
    static int resident = 0;
    if (!resident) resident = resident_blocks((const void*)k_rows_r2c<TI, T, NN, P0>, C::THREADS);
    hipLaunchKernelGGL((k_rows_r2c<TI, T, NN, P0>), dim3(std::min(jobs.total, resident)), dim3(C::THREADS), 0, s,
                       jobs, tw);
    return hipGetLastError();
}

template <typename T, int NN, int P0>
static hipError_t launch_c2r_n(const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    using C = RowCfg<T, NN, P0>;
    static int resident = 0;
    if (!resident) resident = resident_blocks((const void*)k_rows_c2r<T, NN, P0>, C::THREADS);
    hipLaunchKernelGGL((k_rows_c2r<T, NN, P0>), dim3(std::min(jobs.total, resident)), dim3(C::THREADS), 0, s,
                       jobs, tw);
    return hipGetLastError();
}

template <typename TI, typename T, int NN>
static hipError_t launch_r2c_t(const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    using C = TileCfg<NN>;
    static int resident = 0;
    if (!resident) resident = resident_blocks((const void*)k_rows_r2c_t<TI, T, NN>, C::THREADS);
    const int nb = (jobs.total + C::LPB - 1) / C::LPB;
    hipLaunchKernelGGL((k_rows_r2c_t<TI, T, NN>), dim3(std::min(nb, resident)), dim3(C::THREADS), 0, s, jobs, tw);
    return hipGetLastError();
}

template <typename T, int NN>
static hipError_t launch_c2r_t(const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    using C = TileCfg<NN>;
    static int resident = 0;
    if (!resident) resident = resident_blocks((const void*)k_rows_c2r_t<T, NN>, C::THREADS);
    const int nb = (jobs.total + C::LPB - 1) / C::LPB;
    hipLaunchKernelGGL((k_rows_c2r_t<T, NN>), dim3(std::min(nb, resident)), dim3(C::THREADS), 0, s, jobs, tw);
    return hipGetLastError();
}

template <typename TI, typename T>
hipError_t launch_rows_r2c(int N, int tile, const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    if (jobs.total <= 0) return hipSuccess;
#define L_R2C(NN) return tile == 8 ? launch_r2c_t<TI, T, NN>(jobs, tw, s) : tile == 1 ? launch_r2c_n<TI, T, NN, 1>(jobs, tw, s) : tile == 2 ? launch_r2c_n<TI, T, NN, 2>(jobs, tw, s) : launch_r2c_n<TI, T, NN, 4>(jobs, tw, s);
    BTTB_LEN_SWITCH(N, L_R2C)
#undef L_R2C
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_rows_c2r(int N, int tile, const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    if (jobs.total <= 0) return hipSuccess;
#define L_C2R(NN) return tile == 8 ? launch_c2r_t<T, NN>(jobs, tw, s) : tile == 1 ? launch_c2r_n<T, NN, 1>(jobs, tw, s) : tile == 2 ? launch_c2r_n<T, NN, 2>(jobs, tw, s) : launch_c2r_n<T, NN, 4>(jobs, tw, s);
    BTTB_LEN_SWITCH(N, L_C2R)
#undef L_C2R
    return hipErrorInvalidValue;
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
hipError_t launch_cols_fwd(int N, int tile, const ColJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    if (jobs.total <= 0) return hipSuccess;
#define L_FWD(NN)                                                                          \
    if constexpr (col_tile2_fits<T, NN>()) {                                               \
        if (tile == 2) {                                                                   \
            hipLaunchKernelGGL((k_cols_fwd_mac<T, NN, 1, ACC, 2>), dim3(jobs.total), dim3(ColCfg<NN, 2>::THREADS), \
                               0, s, jobs, tw);                                            \
            break;                                                                         \
        }                                                                                  \
    }                                                                                      \
    hipLaunchKernelGGL((k_cols_fwd_mac<T, NN, 1, ACC, 1>), dim3(jobs.total), dim3(ColCfg<NN, 1>::THREADS), 0, \
                       s, jobs, tw);
    BTTB_LEN_SWITCH(N, L_FWD)
#undef L_FWD
    return hipGetLastError();
}

// persistent: as many blocks as are resident at once (at most one per unit)
template <typename T, int NN, int CM>
static void launch_tr_n(const ColJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    static int resident = 0;
    if (!resident) resident = resident_blocks((const void*)k_cols_tr_mac<T, NN, 1, CM>, ColCfg<NN, CM>::THREADS);
    hipLaunchKernelGGL((k_cols_tr_mac<T, NN, 1, CM>), dim3(std::min(jobs.total, resident)),
                       dim3(ColCfg<NN, CM>::THREADS), 0, s, jobs, tw);
}

template <typename T>
hipError_t launch_cols_tr(int N, int tile, const ColJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    if (jobs.total <= 0) return hipSuccess;
#define L_TR(NN)                                                                           \
    if constexpr (col_tile2_fits<T, NN>()) {                                               \
        if (tile == 2) {                                                                   \
            launch_tr_n<T, NN, 2>(jobs, tw, s);                                            \
            break;                                                                         \
        }                                                                                  \
    }                                                                                      \
    launch_tr_n<T, NN, 1>(jobs, tw, s);
    BTTB_LEN_SWITCH(N, L_TR)
#undef L_TR
    return hipGetLastError();
}

// explicit instantiations used by the host code
template hipError_t launch_rows_r2c<double, double>(int, int, const RowJobs&, const double2*, hipStream_t);
template hipError_t launch_rows_r2c<float, float>(int, int, const RowJobs&, const float2*, hipStream_t);
template hipError_t launch_rows_c2r<double>(int, int, const RowJobs&, const double2*, hipStream_t);
template hipError_t launch_rows_c2r<float>(int, int, const RowJobs&, const float2*, hipStream_t);
template hipError_t launch_cols_spec<double>(int, const double2*, int, int, double2*, int, double,
                                             const double2*, hipStream_t);
template hipError_t launch_cols_spec<float>(int, const double2*, int, int, float2*, int, double,
                                            const double2*, hipStream_t);
template hipError_t launch_cols_fwd<double, ACC_PLAIN>(int, int, const ColJobs&, const double2*, hipStream_t);
template hipError_t launch_cols_fwd<float, ACC_PLAIN>(int, int, const ColJobs&, const float2*, hipStream_t);
template hipError_t launch_cols_fwd<float, ACC_TWOSUM>(int, int, const ColJobs&, const float2*, hipStream_t);
template hipError_t launch_cols_fwd<float, ACC_WIDE>(int, int, const ColJobs&, const float2*, hipStream_t);
template hipError_t launch_cols_tr<double>(int, int, const ColJobs&, const double2*, hipStream_t);
template hipError_t launch_cols_tr<float>(int, int, const ColJobs&, const float2*, hipStream_t);

}  // namespace bttbk
