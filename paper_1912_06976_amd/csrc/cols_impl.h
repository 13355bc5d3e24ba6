// cols_impl.h -- gfx950 column kernels of the two products: the y
// transforms with the multiply-accumulate over depth layers in the Fourier
// domain (Sec. 3, eq. GrviaT summed over layers; Sec. 5, eq. Gslice).
//
//   k_cols_fwd_mac   forward product: per column kx, the depth loop
//                    A += T^_r * FFT_y(X_r) with an extended accumulator, then
//                    one inverse FFT_y (or, with the layers split into ranges,
//                    the range's FP64 sum)
//   k_cols_fwd_fin   adds the ranges' sums in order and finishes the column
//   k_cols_tr_mac    transpose product: R^ = FFT_y(R) once per column, then per
//                    layer IFFT_y(conj(T^_r) R^)
//
// Both kernels read the stored spectra in one of two forms (template
// parameter SF):
//   FORM_COMPLEX    T^_r as packed complex half spectra, [r][kx][ky], N
//                   complex values per column
//   FORM_REAL_EVEN  for a generator that is even in both offsets and placed
//                   centred on offset 0 (the symmetric gravity kernel), the
//                   transform is real and even in kx and ky: only
//                   R_r(kx, ky), kx in [0, Nx/2], ky in [0, Ny/2], is stored,
//                   [r][kx][ky] with line stride `lds` (line Nx/2 holds
//                   kx = Nx/2).  The product's generator is that one shifted
//                   by (pxl, pyl) cells, whose transform is
//                   T^(kx, ky) = P(kx, ky) R(kx, ky) with the phase
//                   P = exp(2 pi i (pxl kx / Nx + pyl ky / Ny)); P does not
//                   depend on the layer and is applied once per column:
//                   after the depth sum (forward) or to R^ (transpose).
// Included by the translation units that instantiate the kernels for groups
// of transform lengths (bttb_cols_*.hip); bttb_cols.hip dispatches on the
// length.
#pragma once
#include <type_traits>

#include "kern_common.h"

namespace bttbk {

// Twiddles of the column MAC kernels: registers for power-of-two lines;
// 12-point lines keep them in an LDS table (their registers would spill).
template <typename T, int N>
using ColTwiddles = std::conditional_t<FftShape<N>::POW2, LineTwiddles<T, N>, TableTwiddles<T, N>>;
template <typename T, int N> constexpr int col_tw_lds() { return FftShape<N>::POW2 ? 0 : TableTwiddles<T, N>::size(); }
template <typename T, int N>
__device__ __forceinline__ void init_twiddles(LineTwiddles<T, N>& w, const cT<T>* __restrict__ tw, cT<T>*, int t)
{
    w.load(tw, t);
}
// (contains a block barrier: every thread of the block calls it)
template <typename T, int N>
__device__ __forceinline__ void init_twiddles(TableTwiddles<T, N>& w, const cT<T>* __restrict__ tw, cT<T>* tab, int)
{
    TableTwiddles<T, N>::build(tab, tw, threadIdx.x, blockDim.x);
    lds_barrier();
    w.p = tab;
}

// depth accumulators ------------------------------------------------------
template <typename T, int ACC> struct Acc;
template <typename T> struct Acc<T, ACC_PLAIN> {
    cT<T> s;
    __device__ __forceinline__ void zero() { s = mk<T>(0, 0); }
    __device__ __forceinline__ void add(cT<T> p) { s.x += p.x; s.y += p.y; }
    __device__ __forceinline__ cT<T> get() const { return s; }
    __device__ __forceinline__ double2 wide() const { return make_double2(s.x, s.y); }
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
    __device__ __forceinline__ double2 wide() const {
        return make_double2((double)s.x + (double)c.x, (double)s.y + (double)c.y);
    }
};
// FP64 accumulation of FP32 products
template <typename T> struct Acc<T, ACC_WIDE> {
    double sx, sy;
    __device__ __forceinline__ void zero() { sx = 0.0; sy = 0.0; }
    __device__ __forceinline__ void add(cT<T> p) { sx += (double)p.x; sy += (double)p.y; }
    __device__ __forceinline__ cT<T> get() const { return mk<T>((T)sx, (T)sy); }
    __device__ __forceinline__ double2 wide() const { return make_double2(sx, sy); }
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

// Store register lines (positions t + m TPL) into LDS line buffers so that
// their values at the mirror positions -k can be read back one at a time.
// Contain barriers: every thread of the block calls them; only `active`
// threads write.
template <typename T, int N>
__device__ __forceinline__ void stage_line(const cT<T> (&u)[FftShape<N>::P], cT<T>* bu, int t, bool active)
{
    constexpr int TPL = FftShape<N>::TPL;
    lds_barrier();
    if (active) {
#pragma unroll
        for (int m = 0; m < FftShape<N>::P; ++m) bu[lpad(t + m * TPL)] = u[m];
    }
    lds_barrier();
}
template <typename T, int N>
__device__ __forceinline__ void stage_pair(const cT<T> (&u)[FftShape<N>::P], const cT<T> (&w)[FftShape<N>::P],
                                           cT<T>* bu, cT<T>* bw, int t, bool active)
{
    constexpr int TPL = FftShape<N>::TPL;
    lds_barrier();
    if (active) {
#pragma unroll
        for (int m = 0; m < FftShape<N>::P; ++m) {
            bu[lpad(t + m * TPL)] = u[m];
            bw[lpad(t + m * TPL)] = w[m];
        }
    }
    lds_barrier();
}
// LDS slot of the mirror -k (mod N) of position k = t + m TPL
template <int N> __device__ __forceinline__ int mirror_idx(int t, int m) {
    const int k = t + m * FftShape<N>::TPL;
    if constexpr (FftShape<N>::POW2) return lpad((N - k) & (N - 1));
    else return lpad(k == 0 ? 0 : N - k);
}
// (a b) mod M for 0 <= a, 0 <= b < M (32-bit products: M <= 4096)
__device__ __forceinline__ int mulmod(int a, int b, int M) { return ((a % M) * b) % M; }

// minimum waves per SIMD of the column kernels: FP64 keeps its twiddles (80
// VGPRs) and the prefetch buffers in registers only with the full 512 VGPRs;
// the FP32 transpose kernel fits three waves (168 VGPRs) without spills at
// N = 2048 with one column per block (other shapes would spill)
template <typename T> constexpr int col_waves() { return sizeof(T) == 8 ? 1 : BTTB_COL_WAVES; }
template <typename T, int N, int CM> constexpr int col_waves_tr()
{
    return sizeof(T) == 8 ? 1 : (N == 2048 && CM == 1 ? 3 : BTTB_COL_WAVES);
}

// Real even form: position k = t + m TPL of a line reads the stored value at
// min(k, N - k), i.e. t + m TPL for m < P/2 and (P - m) TPL - t for m >= P/2
// (m = P/2, t = 0 is the Nyquist bin N/2).  Consecutive threads read
// consecutive (or reversed consecutive) addresses.
template <int N> __device__ __forceinline__ int fold_idx(int t, int m) {
    constexpr int P = FftShape<N>::P, TPL = FftShape<N>::TPL;
    return m < P / 2 ? t + m * TPL : (P - m) * TPL - t;
}

// exp(2 pi i (a / Na + b / Nb)) for integers 0 <= a < Na, 0 <= b < Nb (for
// powers of two the argument is exact in FP64, else rounded once per term)
template <typename T> __device__ __forceinline__ cT<T> phase(int a, int Na, int b, int Nb) {
    double s, c;
    sincospi(2.0 * ((double)a / (double)Na + (double)b / (double)Nb), &s, &c);
    return mk<T>((T)c, (T)s);
}

// The real even form's stored values R(kx, ky) of layer r for one line of
// positions t + m TPL of column `col` (for the packed column, kx = 0).
template <typename T, int N>
__device__ __forceinline__ void load_real_even(T (&tn)[FftShape<N>::P], const ColJob& J, int r, int col, int t)
{
    constexpr int P = FftShape<N>::P;
    const T* sp = (const T*)J.spec + ((int64_t)r * (J.ncols + 1) + col) * J.lds;
#pragma unroll
    for (int m = 0; m < P; ++m) tn[m] = sp[fold_idx<N>(t, m)];
}
// The packed column's second part: (-1)^pxl R(Nx/2, ky), the x phase at
// Nx/2 folded in.
template <typename T, int N>
__device__ __forceinline__ void load_real_even_nyq(T (&th)[FftShape<N>::P], const ColJob& J, int r, int t)
{
    constexpr int P = FftShape<N>::P;
    const T sgn = (J.px & 1) ? (T)-1 : (T)1;
    const T* sq = (const T*)J.spec + ((int64_t)r * (J.ncols + 1) + J.ncols) * J.lds;
#pragma unroll
    for (int m = 0; m < P; ++m) th[m] = sgn * sq[fold_idx<N>(t, m)];
}

// Both parts in one complex value per position (.x = R(kx, ky); for the
// packed column .y = (-1)^pxl R(Nx/2, ky), else 0): the transpose kernel's
// form, whose register allocation is best with complex spectra.
template <typename T, int N>
__device__ __forceinline__ void load_real_even_c(cT<T> (&tn)[FftShape<N>::P], const ColJob& J, int r, int col,
                                                 bool packed, int t)
{
    constexpr int P = FftShape<N>::P;
    T re[P], im[P];
    load_real_even<T, N>(re, J, r, col, t);
    if (packed) {
        load_real_even_nyq<T, N>(im, J, r, t);
    } else {
#pragma unroll
        for (int m = 0; m < P; ++m) im[m] = (T)0;
    }
#pragma unroll
    for (int m = 0; m < P; ++m) tn[m] = mk<T>(re[m], im[m]);
}

// End of the forward column pass for one line: the depth sum w of column
// `col` (positions t + m TPL) times the phase of the real even form, the
// inverse y transform, and the store of rows y < nb into block q of Y
// (`store` false: transform only, every thread of the block takes part).
template <typename T, int N, int SF, typename TW>
__device__ __forceinline__ void fwd_finish(cT<T> (&w)[FftShape<N>::P], const ColJob& J, int col, bool packed, bool store,
                                           int q, cT<T>* xl, const TW& twl, int t)
{
    constexpr int P = FftShape<N>::P, TPL = FftShape<N>::TPL;
    if constexpr (SF == FORM_REAL_EVEN) {
        // T^ = P R: the phase of this column (kx = 0 for the packed one)
        const int ax = packed ? 0 : mulmod(J.px, col, 2 * J.ncols);
#pragma unroll
        for (int m = 0; m < P; ++m) w[m] = cmul<T>(w[m], phase<T>(ax, 2 * J.ncols, mulmod(J.py, t + m * TPL, N), N));
    }
    fft_line<T, N, +1, false, TW>(w, xl, twl, t);
    if (store) {
        cT<T>* ys = (cT<T>*)J.b + (int64_t)q * J.ncols * J.ldb;
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int y = t + m * TPL;
            if (y < J.nb) ys[pidx(col, y, J.ncols)] = w[m];
        }
    }
}

// Forward column pass over every job of the table (one block per CPW
// columns of one right-hand-side block and one layer range of one job).
// Job: a = X, the packed row-pass output in panels, block (q, r) at
// X + (q * nz + r) * ncols * lda, y < na = ny, nl = nz layers; b = Y, block
// q at Y + q * ncols * ldb, y < nb = sy.  With ns = 1 a block sums all
// layers and finishes the column; with ns > 1 the layers are split into ns
// ranges and a block writes its range's sum, in FP64, to the partial sums p
// (k_cols_fwd_fin adds them in range order and finishes).
template <typename T, int N, int NR, int ACC, int CM, int SF>
__global__ void __launch_bounds__((ColCfg<N, CM>::THREADS), (col_waves<T>()))
k_cols_fwd_mac(ColJobs jobs, const cT<T>* __restrict__ tw)
{
    using C = ColCfg<N, CM>;
    constexpr int TPL = C::TPL, P = FftShape<N>::P;
    constexpr int LL = lds_line_elems(N);
    __shared__ cT<T> lds[(C::CPW + 1) * LL + col_tw_lds<T, N>()];
    // XCD-ordered block index: neighbouring column blocks, whose panel
    // segments share 128-byte lines, run on one XCD and share its L2
    const int bid = xcd_order(blockIdx.x, gridDim.x);
    const ColJob& J = jobs.j[find_job(jobs, bid)];
    const cT<T>* __restrict__ X = (const cT<T>*)J.a;
    const cT<T>* __restrict__ spec = (const cT<T>*)J.spec;
    const int64_t ldx = J.lda;
    const int ny = J.na, nz = J.nl, ncols = J.ncols, nrhs = J.nrhs;
    // the right-hand-side blocks of one column block are consecutive blocks,
    // which run at the same time on one XCD and share that column's spectra
    // through its L2
    const int nqb = (J.nrhs + NR - 1) / NR, ns = J.ns;
    const int lb = bid - J.begin, rest = lb / nqb, split = rest % ns, cb = rest / ns;
    const int cl = threadIdx.x / TPL, t = threadIdx.x % TPL;
    const int col = cb * C::CPW + cl;
    const int q0 = (lb % nqb) * NR;
    const int rb = (int)((int64_t)split * nz / ns), re = (int)((int64_t)(split + 1) * nz / ns);
    const bool ok = col < ncols;
    const bool packed_blk = cb == 0;              // block holding column 0
    const bool packed = packed_blk && cl == 0;
    cT<T>* xl = lds + cl * LL;
    cT<T>* xs2 = lds + C::CPW * LL;               // second buffer (column 0)
    ColTwiddles<T, N> twl;
    init_twiddles(twl, tw, lds + (C::CPW + 1) * LL, t);
    Acc<T, ACC> acc[NR][P];
#pragma unroll
    for (int q = 0; q < NR; ++q)
#pragma unroll
        for (int m = 0; m < P; ++m) acc[q][m].zero();
    const bool zhi = ny <= N / 2;
    const int ccol = ok ? col : 0;
    // software pipeline: the next layer's spectra and input columns are
    // loaded while the current layer is transformed.  Real even spectra are
    // real except in the packed column, whose second part (the values at
    // kx = Nx/2) is loaded when it is used.
    using S = std::conditional_t<SF == FORM_REAL_EVEN, T, cT<T>>;
    S tn[P];
    cT<T> xn[NR][P];
    auto load_layer = [&](int r) {
        if constexpr (SF == FORM_COMPLEX) {
            const cT<T>* sp = spec + ((int64_t)r * ncols + ccol) * N;
#pragma unroll
            for (int m = 0; m < P; ++m) tn[m] = sp[t + m * TPL];
        } else {
            load_real_even<T, N>(tn, J, r, ccol, t);
        }
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int qq = q0 + q;
            const cT<T>* xs = X + ((int64_t)(qq < nrhs ? qq : 0) * nz + r) * ncols * ldx;
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const int y = t + m * TPL;
                xn[q][m] = (ok && qq < nrhs && y < ny) ? xs[pidx(ccol, y, ncols)] : mk<T>(0, 0);
            }
        }
    };
    // the 12-point lines have no registers left for the next layer's loads
    // (they would spill): they load each layer when they reach it
    constexpr bool PIPE = FftShape<N>::POW2;
    if (PIPE) load_layer(rb);
    for (int r = rb; r < re; ++r) {
        if (!PIPE) load_layer(r);
        S tv[P];
        cT<T> v[NR][P];
#pragma unroll
        for (int m = 0; m < P; ++m) tv[m] = tn[m];
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int m = 0; m < P; ++m) v[q][m] = xn[q][m];
        if (PIPE && r + 1 < re) load_layer(r + 1);
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            if (zhi) fft_line<T, N, -1, true, ColTwiddles<T, N>>(v[q], xl, twl, t);
            else fft_line<T, N, -1, false, ColTwiddles<T, N>>(v[q], xl, twl, t);
            if constexpr (SF == FORM_COMPLEX) {
                if (packed_blk) {
                    stage_pair<T, N>(v[q], tv, xl, xs2, t, packed);
                    if (packed) {
                        // column 0 carries bins 0 and N/2: accumulate
                        // T0 F0 + i T1 F1 of the separated Hermitian parts
#pragma unroll
                        for (int m = 0; m < P; ++m) {
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
                for (int m = 0; m < P; ++m) acc[q][m].add(cmul<T>(tv[m], v[q][m]));
            } else {
                if (packed_blk) {
                    stage_line<T, N>(v[q], xl, t, packed);
                    if (packed) {
                        // R(0) F0 + i (-1)^pxl R(Nx/2) F1 (R is even: no mirror)
                        T th[P];
                        load_real_even_nyq<T, N>(th, J, r, t);
#pragma unroll
                        for (int m = 0; m < P; ++m) {
                            const cT<T> vr = xl[mirror_idx<N>(t, m)];
                            const cT<T> a = herm_a<T>(v[q][m], vr), b = herm_b<T>(v[q][m], vr);
                            acc[q][m].add(mk<T>(tv[m] * a.x - th[m] * b.y, tv[m] * a.y + th[m] * b.x));
                        }
                        continue;
                    }
                }
#pragma unroll
                for (int m = 0; m < P; ++m) acc[q][m].add(mk<T>(tv[m] * v[q][m].x, tv[m] * v[q][m].y));
            }
        }
    }
    if (ns > 1) {
        // this layer range's sum, for k_cols_fwd_fin (ns is uniform in the
        // block: no thread is left at a barrier)
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int qq = q0 + q;
            if (ok && qq < nrhs) {
                double2* pp = (double2*)J.p + (((int64_t)qq * ns + split) * ncols + col) * N;
#pragma unroll
                for (int m = 0; m < P; ++m) pp[t + m * TPL] = acc[q][m].wide();
            }
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const int qq = q0 + q;
        cT<T> w[P];
#pragma unroll
        for (int m = 0; m < P; ++m) w[m] = acc[q][m].get();
        fwd_finish<T, N, SF>(w, J, ccol, packed, ok && qq < nrhs, qq, xl, twl, t);
    }
}

// Finishing kernel of the forward column pass for jobs with ns > 1: one
// block per CPW columns (FinCfg) of one right-hand side, which adds the ns
// partial depth sums in range order in FP64 and finishes the columns (phase,
// inverse y transform, store).
template <typename T, int N, int SF>
__global__ void __launch_bounds__((FinCfg<N>::THREADS)) k_cols_fwd_fin(ColJobs jobs, const cT<T>* __restrict__ tw)
{
    using C = FinCfg<N>;
    constexpr int TPL = C::TPL, P = FftShape<N>::P;
    constexpr int LL = lds_line_elems(N);
    __shared__ cT<T> lds[C::CPW * LL];
    const int bid = xcd_order(blockIdx.x, gridDim.x);
    const ColJob& J = jobs.j[find_job(jobs, bid)];
    const int lb = bid - J.begin, q = lb % J.nrhs, cb = lb / J.nrhs;
    const int cl = threadIdx.x / TPL, t = threadIdx.x % TPL;
    const int col = cb * C::CPW + cl, ns = J.ns;
    const bool ok = col < J.ncols;
    LineTwiddles<T, N> twl;
    twl.load(tw, t);
    double sx[P], sy[P];
#pragma unroll
    for (int m = 0; m < P; ++m) sx[m] = sy[m] = 0.0;
    if (ok) {
        const double2* pp = (const double2*)J.p + ((int64_t)q * ns * J.ncols + col) * N;
        const int64_t stride = (int64_t)J.ncols * N;
        // the loads of FB ranges are issued together (the kernel is bound by
        // their latency), then added in range order
        constexpr int FB = P == 8 ? 4 : 3;
        for (int s0 = 0; s0 < ns; s0 += FB) {
            double2 v[FB][P];
#pragma unroll
            for (int k = 0; k < FB; ++k)
#pragma unroll
                for (int m = 0; m < P; ++m)
                    v[k][m] = s0 + k < ns ? pp[(s0 + k) * stride + t + m * TPL] : make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < FB; ++k) {
                if (s0 + k < ns) {
#pragma unroll
                    for (int m = 0; m < P; ++m) {
                        sx[m] += v[k][m].x;
                        sy[m] += v[k][m].y;
                    }
                }
            }
        }
    }
    cT<T> w[P];
#pragma unroll
    for (int m = 0; m < P; ++m) w[m] = mk<T>((T)sx[m], (T)sy[m]);
    fwd_finish<T, N, SF>(w, J, ok ? col : 0, cb == 0 && cl == 0, ok, q, lds + cl * LL, twl, t);
}

// Transpose column pass over every job of the table, layers [r0, r0 + nl).
// Job: a = R, the packed row-pass output of the data in panels, block q at
// R + q * ncols * lda, y < na = sy; b = Z, block (q, r - r0) at
// Z + (q * nl + r - r0) * ncols * ldb, y < nb = ny.
// The kernel is persistent and balanced: the work of all jobs is the list of
// units (job, column block cb, right-hand side q, layer l), layer fastest,
// and block w processes the contiguous range [w U / G, (w + 1) U / G).  The
// right-hand sides of one column block thus fall to neighbouring blocks,
// which run at the same time on one XCD and share its spectra through L2.  A
// block recomputes R^ = FFT_y(R) whenever its range enters a new column
// block (at most a few times), so every block gets the same number of layers
// whatever the number of resident blocks.
template <typename T, int N, int NR, int CM, int SF>
__global__ void __launch_bounds__((ColCfg<N, CM>::THREADS), (col_waves_tr<T, N, CM>()))
k_cols_tr_mac(ColJobs jobs, const cT<T>* __restrict__ tw)
{
    using C = ColCfg<N, CM>;
    constexpr int TPL = C::TPL, P = FftShape<N>::P;
    constexpr int LL = lds_line_elems(N);
    __shared__ cT<T> lds[(C::CPW + 1) * LL + col_tw_lds<T, N>()];
    const int cl = threadIdx.x / TPL, t = threadIdx.x % TPL;
    cT<T>* xl = lds + cl * LL;
    cT<T>* xs2 = lds + C::CPW * LL;
    ColTwiddles<T, N> twl;
    init_twiddles(twl, tw, lds + (C::CPW + 1) * LL, t);
    const int64_t U = jobs.total, G = gridDim.x;
    // XCD-ordered: blocks with neighbouring unit ranges (the right-hand
    // sides of one column block, then neighbouring column blocks, whose
    // panel segments share 128-byte lines) run on one XCD
    const int w = xcd_order(blockIdx.x, (int)G);
    const int u0 = (int)((int64_t)w * U / G), u1 = (int)((int64_t)(w + 1) * U / G);
    // unit u -> (job k, column block cb, right-hand side q, layer l); a job's
    // units run layer-fastest, then right-hand side, then column block, so
    // the walk decodes its first unit and then advances the position (a full
    // decode again only where the next job begins)
    struct UPos { int k, cb, q, l; };
    auto decode = [&](int u) {
        UPos p;
        p.k = find_job(jobs, u);
        const ColJob& J = jobs.j[p.k];
        const int lu = u - J.begin;
        const int key = lu / J.nl;
        p.l = lu - key * J.nl;
        p.cb = key / J.nrhs;
        p.q = key - p.cb * J.nrhs;
        return p;
    };
    auto advance = [&](const UPos& p, int un) {   // position of un, the unit after p's
        if (p.k + 1 < jobs.njobs && un >= jobs.j[p.k + 1].begin) return decode(un);
        UPos n = p;
        if (++n.l == jobs.j[p.k].nl) {
            n.l = 0;
            if (++n.q == jobs.j[p.k].nrhs) {
                n.q = 0;
                ++n.cb;
            }
        }
        return n;
    };
    cT<T> tn[P];
    auto load_spec = [&](const UPos& p) {
        const ColJob& J = jobs.j[p.k];
        const int col = p.cb * C::CPW + cl;
        const int ccol = col < J.ncols ? col : 0;
        if constexpr (SF == FORM_COMPLEX) {
            const cT<T>* sp = (const cT<T>*)J.spec + ((int64_t)(J.r0 + p.l) * J.ncols + ccol) * N;
#pragma unroll
            for (int m = 0; m < P; ++m) tn[m] = sp[t + m * TPL];
        } else {
            load_real_even_c<T, N>(tn, J, J.r0 + p.l, ccol, p.cb == 0 && cl == 0, t);
        }
    };
    int cur_k = -1, cur_cb = -1, cur_q = -1;
    cT<T> rh[P];
    // the 12-point lines have no registers left for the next layer's loads
    // (they would spill): they load each layer when they reach it
    constexpr bool PIPE = FftShape<N>::POW2;
    UPos pn{0, 0, 0, 0};
    if (u0 < u1) pn = decode(u0);
    // tv: this unit's spectra (from tn, the prefetch registers)
    cT<T> tv[P];
    if (PIPE && u0 < u1) {
        load_spec(pn);
#pragma unroll
        for (int m = 0; m < P; ++m) tv[m] = tn[m];
    }
    for (int u = u0; u < u1; ++u) {
        const UPos pc = pn;
        if (u + 1 < u1) pn = advance(pc, u + 1);
        if (!PIPE) {
            load_spec(pc);
#pragma unroll
            for (int m = 0; m < P; ++m) tv[m] = tn[m];
        }
        const int k = pc.k, l = pc.l, cb = pc.cb, q = pc.q;
        const ColJob& J = jobs.j[k];
        const int col = cb * C::CPW + cl;
        const bool ok = col < J.ncols;
        const bool packed_blk = cb == 0;
        const bool packed = packed_blk && cl == 0;
        if (PIPE && u + 1 < u1) load_spec(pn);
        if (k != cur_k || cb != cur_cb || q != cur_q) {
            // R^ of this column: FFT_y of the packed row-pass output of the data
            const cT<T>* rs = (const cT<T>*)J.a + (int64_t)q * J.ncols * J.lda;
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const int y = t + m * TPL;
                rh[m] = (ok && y < J.na) ? rs[pidx(col, y, J.ncols)] : mk<T>(0, 0);
            }
            if (J.na <= N / 2) fft_line<T, N, -1, true, ColTwiddles<T, N>>(rh, xl, twl, t);
            else fft_line<T, N, -1, false, ColTwiddles<T, N>>(rh, xl, twl, t);
            if constexpr (SF == FORM_REAL_EVEN) {
                // conj(T^) R^ = R conj(P) R^: apply conj(P) once.  The packed
                // column keeps conj(P) A in rh and conj(P) B in its second LDS
                // buffer (read back by the same thread only).
                if (packed_blk) {
                    stage_line<T, N>(rh, xl, t, packed);
                    if (packed) {
#pragma unroll
                        for (int m = 0; m < P; ++m) {
                            const cT<T> rr = xl[mirror_idx<N>(t, m)];
                            const cT<T> ph = phase<T>(0, 2, mulmod(J.py, t + m * TPL, N), N);
                            const cT<T> a = cmulc<T>(herm_a<T>(rh[m], rr), ph);
                            xs2[lpad(t + m * TPL)] = cmulc<T>(herm_b<T>(rh[m], rr), ph);
                            rh[m] = a;
                        }
                    }
                }
                if (!packed) {
                    const int ax = mulmod(J.px, ok ? col : 0, 2 * J.ncols);
#pragma unroll
                    for (int m = 0; m < P; ++m)
                        rh[m] = cmulc<T>(rh[m], phase<T>(ax, 2 * J.ncols, mulmod(J.py, t + m * TPL, N), N));
                }
            }
            cur_k = k;
            cur_cb = cb;
            cur_q = q;
        }
        cT<T> v[P];
        if constexpr (SF == FORM_COMPLEX) {
#pragma unroll
            for (int m = 0; m < P; ++m) v[m] = cmulc<T>(rh[m], tv[m]);
            if (packed_blk) {
                stage_pair<T, N>(rh, tv, xl, xs2, t, packed);
                if (packed) {
                    // column 0: conj(T0) R0 + i conj(T1) R1
#pragma unroll
                    for (int m = 0; m < P; ++m) {
                        const int mi = mirror_idx<N>(t, m);
                        const cT<T> rr = xl[mi], tr = xs2[mi];
                        const cT<T> p0 = cmulc<T>(herm_a<T>(rh[m], rr), herm_a<T>(tv[m], tr));
                        const cT<T> p1 = cmulc<T>(herm_b<T>(rh[m], rr), herm_b<T>(tv[m], tr));
                        v[m] = mk<T>(p0.x - p1.y, p0.y + p1.x);
                    }
                }
            }
        } else {
            if (packed) {
                // R(0) A' + i (-1)^pxl R(Nx/2) B'
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    const cT<T> b = xs2[lpad(t + m * TPL)];
                    v[m] = mk<T>(tv[m].x * rh[m].x - tv[m].y * b.y, tv[m].x * rh[m].y + tv[m].y * b.x);
                }
            } else {
#pragma unroll
                for (int m = 0; m < P; ++m) v[m] = mk<T>(tv[m].x * rh[m].x, tv[m].x * rh[m].y);
            }
        }
        fft_line<T, N, +1, false, ColTwiddles<T, N>>(v, xl, twl, t);
        // the next unit's spectra, taken before this unit's stores so that
        // waiting for them does not wait for the stores
        if (PIPE) {
            wait_vmem();
#pragma unroll
            for (int m = 0; m < P; ++m) tv[m] = tn[m];
        }
        if (ok) {
            cT<T>* zs = (cT<T>*)J.b + ((int64_t)q * J.nl + l) * J.ncols * J.ldb;
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const int y = t + m * TPL;
                if (y < J.nb) zs[pidx(col, y, J.ncols)] = v[m];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// launchers of one transform length (instantiated per length group in
// bttb_cols_*.hip, dispatched on the length in bttb_cols.hip)
// ---------------------------------------------------------------------------
template <typename T, int ACC, int NN>
hipError_t cols_fwd_n(int tile, int form, const ColJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    if (form == FORM_REAL_EVEN) {
        if constexpr (col_tile2_fits<T, NN>()) {
            if (tile == 2) {
                hipLaunchKernelGGL((k_cols_fwd_mac<T, NN, 1, ACC, 2, FORM_REAL_EVEN>), dim3(jobs.total),
                                   dim3(ColCfg<NN, 2>::THREADS), 0, s, jobs, tw);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((k_cols_fwd_mac<T, NN, 1, ACC, 1, FORM_REAL_EVEN>), dim3(jobs.total),
                           dim3(ColCfg<NN, 1>::THREADS), 0, s, jobs, tw);
        return hipGetLastError();
    }
    if constexpr (col_tile2_fits<T, NN>()) {
        if (tile == 2) {
            hipLaunchKernelGGL((k_cols_fwd_mac<T, NN, 1, ACC, 2, FORM_COMPLEX>), dim3(jobs.total),
                               dim3(ColCfg<NN, 2>::THREADS), 0, s, jobs, tw);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_cols_fwd_mac<T, NN, 1, ACC, 1, FORM_COMPLEX>), dim3(jobs.total),
                       dim3(ColCfg<NN, 1>::THREADS), 0, s, jobs, tw);
    return hipGetLastError();
}

// (blocks of FinCfg<NN>::CPW columns, whatever the column tile)
template <typename T, int NN>
hipError_t cols_fin_n(int, int form, const ColJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    if (form == FORM_REAL_EVEN)
        hipLaunchKernelGGL((k_cols_fwd_fin<T, NN, FORM_REAL_EVEN>), dim3(jobs.total), dim3(FinCfg<NN>::THREADS), 0, s,
                           jobs, tw);
    else
        hipLaunchKernelGGL((k_cols_fwd_fin<T, NN, FORM_COMPLEX>), dim3(jobs.total), dim3(FinCfg<NN>::THREADS), 0, s,
                           jobs, tw);
    return hipGetLastError();
}

// persistent: as many blocks as are resident at once (at most one per unit)
template <typename T, int NN, int CM, int SF>
static void launch_tr_k(const ColJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    // thread-safe one-time initialisation (function-local static)
    static const int resident = resident_blocks((const void*)k_cols_tr_mac<T, NN, 1, CM, SF>, ColCfg<NN, CM>::THREADS);
    hipLaunchKernelGGL((k_cols_tr_mac<T, NN, 1, CM, SF>), dim3(persistent_grid(jobs.total, resident)),
                       dim3(ColCfg<NN, CM>::THREADS), 0, s, jobs, tw);
}
template <typename T, int NN>
hipError_t cols_tr_n(int tile, int form, const ColJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    if constexpr (col_tile2_fits<T, NN>()) {
        if (tile == 2) {
            if (form == FORM_REAL_EVEN) launch_tr_k<T, NN, 2, FORM_REAL_EVEN>(jobs, tw, s);
            else launch_tr_k<T, NN, 2, FORM_COMPLEX>(jobs, tw, s);
            return hipGetLastError();
        }
    }
    if (form == FORM_REAL_EVEN) launch_tr_k<T, NN, 1, FORM_REAL_EVEN>(jobs, tw, s);
    else launch_tr_k<T, NN, 1, FORM_COMPLEX>(jobs, tw, s);
    return hipGetLastError();
}

// every launcher of length NN
#define BTTB_COLS_INSTANTIATE(NN)                                                                              \
    template hipError_t cols_fwd_n<double, ACC_PLAIN, NN>(int, int, const ColJobs&, const double2*, hipStream_t); \
    template hipError_t cols_fwd_n<float, ACC_PLAIN, NN>(int, int, const ColJobs&, const float2*, hipStream_t);   \
    template hipError_t cols_fwd_n<float, ACC_TWOSUM, NN>(int, int, const ColJobs&, const float2*, hipStream_t);  \
    template hipError_t cols_fwd_n<float, ACC_WIDE, NN>(int, int, const ColJobs&, const float2*, hipStream_t);    \
    template hipError_t cols_fin_n<double, NN>(int, int, const ColJobs&, const double2*, hipStream_t);            \
    template hipError_t cols_fin_n<float, NN>(int, int, const ColJobs&, const float2*, hipStream_t);              \
    template hipError_t cols_tr_n<double, NN>(int, int, const ColJobs&, const double2*, hipStream_t);             \
    template hipError_t cols_tr_n<float, NN>(int, int, const ColJobs&, const float2*, hipStream_t);

}  // namespace bttbk
