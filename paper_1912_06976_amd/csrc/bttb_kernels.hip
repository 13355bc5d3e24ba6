// bttb_kernels.hip -- gfx950 kernels of the fast BTTB products.
//
//   k_twiddles       FP64 twiddle tables exp(-2 pi i k / N), rounded to the
//                    working precision
//   k_generate       FP64 circulant generator T_r of each depth layer from
//                    the closed-form prism integrals (Sec. 3, eq. Tcircpadded /
//                    eq. Tcircpaddedgeneral; Sec. 4.1 / 4.2 entries)
//   k_rows_r2c       real rows -> half spectra along x, pairs of rows packed
//                    into one complex transform, written in 8-row panels
//                    (bttb_internal.h) through an LDS tile
//   k_cols_spec      FP64 column transforms of the generator -> stored spectra
//                    (scaled by 1 / (Nx Ny), rounded to the working precision)
//   k_rows_c2r       half spectra (panels) -> real rows along x, two rows per
//                    complex transform, extraction of the leading columns
//
// The column kernels of the products are in bttb_cols.hip.  All kernels take
// caller-owned device buffers; none allocates.
#include "kern_common.h"

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

// Corner grid (the paper's gravity / magnetic algorithms evaluate the
// closed form once per corner of the grid of prism edges, Sec. 4.1 / 4.2):
// one thread per corner (ex, ey) of depth edge k = blockIdx.y of the batch,
// F[k][ey][ex] = f((oxmin + ex - 1/2) dx, (oymin + ey - 1/2) dy, z_k + h).
// Each value is shared by the four entries whose prisms meet at that corner
// and by the two layers on either side of the edge.
__global__ void k_corners(GenParams P, double* __restrict__ F)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)P.cx * P.cy;
    if (idx >= per) return;
    const int ex = (int)(idx % P.cx), ey = (int)(idx / P.cx);
    const double x = ((double)(P.oxmin + ex) - 0.5) * P.dx;
    const double y = ((double)(P.oymin + ey) - 0.5) * P.dy;
    const double z = P.z[blockIdx.y] + P.h;
    F[(int64_t)blockIdx.y * per + idx] = P.kind == KIND_GRAVITY ? corner_gz(x, y, z) : corner_tmi(x, y, z, P.w);
}

// One thread per circulant position (X, Y) of layer r = r0 + blockIdx.y:
//   T_r[Y][X] = h_r(-ax - pxl, -ay - pyl) if ax in [-(nx-1), sx-1] and
//   ay in [-(ny-1), sy-1], with ax = X or X - Nx (and likewise ay), else 0.
// h_r(dx, dy) is the prism integral over x in [(dx-1/2), (dx+1/2)] Dx,
// y in [(dy-1/2), (dy+1/2)] Dy, z in [z_r + h, z_{r+1} + h]: the entry of
// G for a station and a prism offset by (dx, dy) cells (Sec. 2.1.1-2.1.2).
// Centred placement (P.sym, for a kernel even in dx and dy): T_r[Y][X] =
// h_r(|ax|, |ay|) for |ax| <= bx, |ay| <= by with ax = X or X - Nx in
// (-Nx/2, Nx/2]; the product's generator is this one shifted by (pxl, pyl).
__global__ void k_generate(GenParams P, int r0, double* __restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)P.Nx * P.Ny;
    if (idx >= per) return;
    const int r = r0 + blockIdx.y;
    const int X = (int)(idx % P.Nx), Y = (int)(idx / P.Nx);
    bool inside;
    int ox, oy;
    if (P.sym) {
        ox = X <= P.Nx / 2 ? X : P.Nx - X;
        oy = Y <= P.Ny / 2 ? Y : P.Ny - Y;
        inside = ox <= P.bx && oy <= P.by;
    } else {
        const int ax = X <= P.sx - 1 ? X : (X >= P.Nx - (P.nx - 1) ? X - P.Nx : INT32_MIN);
        const int ay = Y <= P.sy - 1 ? Y : (Y >= P.Ny - (P.ny - 1) ? Y - P.Ny : INT32_MIN);
        inside = ax != INT32_MIN && ay != INT32_MIN;
        ox = inside ? -ax - P.pxl : 0;
        oy = inside ? -ay - P.pyl : 0;
    }
    double val = 0.0;
    if (inside) {
        if (P.kind == KIND_PROBE) {
            val = (double)ox + 4096.0 * (double)oy + 16777216.0 * (double)r;
        } else if (P.kind == KIND_TABLE) {
            // the caller's entry; the centred placement of an even kernel
            // reads the mirror of an offset the table has on one side only
            int tx = ox + P.offx, ty = oy + P.offy;
            if (tx >= P.wx) tx = P.offx - ox;
            if (ty >= P.wy) ty = P.offy - oy;
            val = P.scale * P.table[((int64_t)r * P.wy + ty) * P.wx + tx];
        } else {
            // signed sum of the 8 corner terms of the prism (corner grid of
            // the batch, edges blockIdx.y and blockIdx.y + 1)
            const int64_t per = (int64_t)P.cx * P.cy;
            const double* F = P.corners + (int64_t)blockIdx.y * per + (int64_t)(oy - P.oymin) * P.cx + (ox - P.oxmin);
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        const double f = F[k * per + j * P.cx + i];
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


// ---------------------------------------------------------------------------
// row transforms
// ---------------------------------------------------------------------------
// two adjacent complex values with one 16-byte (FP32) store; the address
// must be 16-byte aligned (FP64: two 16-byte stores)
template <typename T> __device__ __forceinline__ void store_pair(cT<T>* o, cT<T> a, cT<T> b)
{
    if constexpr (sizeof(T) == 4) *(float4*)o = make_float4(a.x, a.y, b.x, b.y);
    else { o[0] = a; o[1] = b; }
}
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
    // r2c: the complex transforms Z of the PAIRS row pairs staged by
    // frequency, [k][pair] with a padded row (bank spread of the writes)
    // (FP32 only; FP64 splits through the line buffers and stages the half
    // spectra [kx][row] like the c2r tile, which measured faster there)
    static constexpr int ZROW = PAIRS > 1 ? PAIRS + 1 : 1;
    static constexpr int ZSTAGE = N * ZROW;
    static constexpr int LDS_R2C = sizeof(T) == 4 ? (ZSTAGE > XCH ? ZSTAGE : XCH) : LDS;
};

// Row kernels are persistent: gridDim.x blocks (about the number that fit on
// the device at once) walk over the row groups g = lb, lb + G, lb + 2G, ...
// (lb = XCD-ordered block index, so neighbouring groups, which share 128-byte
// lines of the column-major half spectra, run on one XCD at the same time).
// The loads of the next group are issued before the current group is
// transformed, so memory latency overlaps the FFT.


// Row transform, real -> packed half spectra, over every job of the table.
// Job input: batch b, row y, column x at in[b * in_bs + y * in_ld + x],
// x < nv valid (zero beyond, up to N); output: packed half spectra in
// panels, out[b * out_bs + pidx(kx, y, N/2)], kx < N/2, y < nrows.
template <typename TI, typename T, int N, int P0>
__global__ void __launch_bounds__((RowCfg<T, N, P0>::THREADS))
k_rows_r2c(RowJobs jobs, const cT<T>* __restrict__ tw)
{
    using C = RowCfg<T, N, P0>;
    constexpr int TPL = C::TPL;
    __shared__ cT<T> lds[C::LDS_R2C + TableTwiddles<T, N>::size()];
    const int G = gridDim.x, total = jobs.total;
    const int pr = threadIdx.x / TPL, t = threadIdx.x % TPL;
    TableTwiddles<T, N>::build(lds + C::LDS_R2C, tw, threadIdx.x, C::THREADS);
    __syncthreads();
    const TableTwiddles<T, N> twl{lds + C::LDS_R2C};
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
        cT<T>* dst = (cT<T>*)J.out + (int64_t)b * J.out_bs;
        if constexpr (sizeof(T) == 4) {
            // stage Z = FFT(a + i c) of every pair by frequency, then split it
            // into the two rows' half spectra while the tile is stored:
            //   A[k] = (Z[k] + conj Z[N-k]) / 2,  C[k] = (Z[k] - conj Z[N-k]) / (2 i),
            // slot 0 packing the real bins 0 and N/2; element (kx, pair) stores
            // both rows (adjacent in the column) with one 16-byte store
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 8; ++m) lds[(t + m * TPL) * C::ZROW + pr] = v[m];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < (C::HALF * C::PAIRS) / C::THREADS; ++i) {
                const int e = threadIdx.x + i * C::THREADS;
                const int kx = e / C::PAIRS, q = e % C::PAIRS;
                const cT<T> z = lds[kx * C::ZROW + q];
                cT<T> A, Cc;
                if (kx == 0) {
                    const cT<T> zh = lds[(N / 2) * C::ZROW + q];
                    A = mk<T>(z.x, zh.x);
                    Cc = mk<T>(z.y, zh.y);
                } else {
                    const cT<T> zr = lds[(N - kx) * C::ZROW + q];
                    A = mk<T>((T)0.5 * (z.x + zr.x), (T)0.5 * (z.y - zr.y));
                    Cc = mk<T>((T)0.5 * (z.y + zr.y), (T)0.5 * (zr.x - z.x));
                }
                const int ra = row0 + 2 * q;
                cT<T>* o = dst + pidx(kx, ra, C::HALF);
                if (ra + 1 < J.nrows && ((uintptr_t)o & 15) == 0) {
                    store_pair<T>(o, A, Cc);
                } else {
                    if (ra < J.nrows) o[0] = A;
                    if (ra + 1 < J.nrows) o[1] = Cc;
                }
            }
        } else {
            // split through the line buffer (mirror reads), then stage the
            // half spectra [kx][row] and store the tile
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
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int e = threadIdx.x + i * C::THREADS;   // HALF * RT = 8 * THREADS
                const int kx = e / C::RT, rr = e % C::RT;
                if (row0 + rr < J.nrows) dst[pidx(kx, row0 + rr, C::HALF)] = lds[kx * C::SROW + rr];
            }
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = vn[m];
    }
}

// Row transform, packed half spectra -> real rows, over every job of the
// table.  Job input: in[b * in_bs + pidx(kx, y, N/2)], kx < N/2, y < nrows;
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
    // (8-byte loads: eight lanes per 64-byte column segment; 16-byte loads,
    // with twice the segments per instruction, measured slower)
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
            tl[i] = (row0 + rr < J.nrows) ? src[pidx(kx, row0 + rr, C::HALF)] : mk<T>(0, 0);
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
                cT<T>* col = dst + pidx(t + m * TPL, row0, N / 2);   // row0 % PANEL == 0
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
            const cT<T>* col = src + pidx(t + m * TPL, row0, N / 2);   // row0 % PANEL == 0
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
// spectra from the FP64 generator: in = packed half spectra along x of the
// nl layers, N rows each, in panels (block l at in + l * ncols * N) ->
// FFT_y(in) * scale, stored as
//   FORM_COMPLEX:   spec[((r0 + l) * ncols + kx) * N + ky] (column 0 becomes
//                   T^[0] + i T^[N/2], the packed pair of Hermitian columns)
//   FORM_REAL_EVEN: the real parts for ky in [0, N/2] at
//                   spec[((r0 + l) * (ncols + 1) + kx) * ldr + ky], with
//                   kx = Nx/2 (the imaginary part of column 0) in line ncols.
//                   For the centred even generator the transform is real up to
//                   rounding (its imaginary parts are dropped).
template <typename T, int N>
__global__ void __launch_bounds__(ColCfg<N>::THREADS)
k_cols_spec(const double2* __restrict__ in, int ncols, void* __restrict__ spec, int r0, double scale,
            const double2* __restrict__ tw, int form, int64_t ldr)
{
    using C = ColCfg<N>;
    constexpr int TPL = C::TPL;
    __shared__ double2 lds[C::CPW * lds_line_elems(N)];
    const int cl = threadIdx.x / TPL, t = threadIdx.x % TPL;
    const int col = blockIdx.x * C::CPW + cl;
    const int l = blockIdx.y;
    const bool ok = col < ncols;
    double2 v[8];
    const double2* src = in + (int64_t)l * ncols * N;
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = ok ? src[pidx(col, t + m * TPL, ncols)] : make_double2(0.0, 0.0);
    LineTwiddles<double, N> twl;
    twl.load(tw, t);
    fft_line<double, N, -1, false>(v, lds + cl * lds_line_elems(N), twl, t);
    if (!ok) return;
    if (form == FORM_COMPLEX) {
        cT<T>* dst = (cT<T>*)spec + ((int64_t)(r0 + l) * ncols + col) * N;
#pragma unroll
        for (int m = 0; m < 8; ++m) dst[t + m * TPL] = mk<T>((T)(v[m].x * scale), (T)(v[m].y * scale));
    } else {
        T* base = (T*)spec + (int64_t)(r0 + l) * (ncols + 1) * ldr;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int y = t + m * TPL;
            if (y > N / 2) continue;
            base[(int64_t)col * ldr + y] = (T)(v[m].x * scale);
            if (col == 0) base[(int64_t)ncols * ldr + y] = (T)(v[m].y * scale);
        }
    }
}

// ---------------------------------------------------------------------------
// launchers (dispatch on the transform lengths)
// ---------------------------------------------------------------------------

hipError_t launch_twiddles(double2* t64, float2* t32, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_twiddles, dim3((n + 255) / 256), dim3(256), 0, s, t64, t32, n);
    return hipGetLastError();
}

hipError_t launch_corners(const GenParams& P, int nl, double* corners, hipStream_t s)
{
    const int64_t per = (int64_t)P.cx * P.cy;
    dim3 grid((unsigned)((per + 255) / 256), (unsigned)(nl + 1));
    hipLaunchKernelGGL(k_corners, grid, dim3(256), 0, s, P, corners);
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
    // thread-safe one-time initialisation (function-local static)
    static const int resident = resident_blocks((const void*)k_rows_r2c<TI, T, NN, P0>, C::THREADS);
    hipLaunchKernelGGL((k_rows_r2c<TI, T, NN, P0>), dim3(std::min(jobs.total, resident)), dim3(C::THREADS), 0, s,
                       jobs, tw);
    return hipGetLastError();
}

template <typename T, int NN, int P0>
static hipError_t launch_c2r_n(const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    using C = RowCfg<T, NN, P0>;
    // thread-safe one-time initialisation (function-local static)
    static const int resident = resident_blocks((const void*)k_rows_c2r<T, NN, P0>, C::THREADS);
    hipLaunchKernelGGL((k_rows_c2r<T, NN, P0>), dim3(std::min(jobs.total, resident)), dim3(C::THREADS), 0, s,
                       jobs, tw);
    return hipGetLastError();
}

template <typename TI, typename T, int NN>
static hipError_t launch_r2c_t(const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    using C = TileCfg<NN>;
    // thread-safe one-time initialisation (function-local static)
    static const int resident = resident_blocks((const void*)k_rows_r2c_t<TI, T, NN>, C::THREADS);
    const int nb = (jobs.total + C::LPB - 1) / C::LPB;
    hipLaunchKernelGGL((k_rows_r2c_t<TI, T, NN>), dim3(std::min(nb, resident)), dim3(C::THREADS), 0, s, jobs, tw);
    return hipGetLastError();
}

template <typename T, int NN>
static hipError_t launch_c2r_t(const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    using C = TileCfg<NN>;
    // thread-safe one-time initialisation (function-local static)
    static const int resident = resident_blocks((const void*)k_rows_c2r_t<T, NN>, C::THREADS);
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
hipError_t launch_cols_spec(int N, const double2* in, int ncols, int nl, void* spec, int r0,
                            double scale, const double2* tw, int form, int64_t ldr, hipStream_t s)
{
#define L_SPEC(NN)                                                                         \
    {                                                                                      \
        using C = ColCfg<NN>;                                                              \
        dim3 grid((ncols + C::CPW - 1) / C::CPW, nl);                                      \
        hipLaunchKernelGGL((k_cols_spec<T, NN>), grid, dim3(C::THREADS), 0, s, in, ncols, spec, \
                           r0, scale, tw, form, ldr);                                      \
    }
    BTTB_LEN_SWITCH(N, L_SPEC)
#undef L_SPEC
    return hipGetLastError();
}

// explicit instantiations used by the host code
template hipError_t launch_rows_r2c<double, double>(int, int, const RowJobs&, const double2*, hipStream_t);
template hipError_t launch_rows_r2c<float, float>(int, int, const RowJobs&, const float2*, hipStream_t);
template hipError_t launch_rows_c2r<double>(int, int, const RowJobs&, const double2*, hipStream_t);
template hipError_t launch_rows_c2r<float>(int, int, const RowJobs&, const float2*, hipStream_t);
template hipError_t launch_cols_spec<double>(int, const double2*, int, int, void*, int, double,
                                             const double2*, int, int64_t, hipStream_t);
template hipError_t launch_cols_spec<float>(int, const double2*, int, int, void*, int, double,
                                            const double2*, int, int64_t, hipStream_t);

}  // namespace bttbk
