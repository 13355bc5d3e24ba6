// rows_impl.h -- gfx950 row transforms of the products and the column
// transforms of the spectra (kernel templates and the launchers of one
// transform length).  Included by bttb_rows_*.hip, which instantiate them for
// groups of lengths; the block shapes are in rows_cfg.h.
#pragma once
#include "rows_cfg.h"

namespace bttbk {

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
// mirror position (N - k) mod N of k in [0, N]
template <int N> __device__ __forceinline__ int mirror_pos(int k)
{
    if constexpr (FftShape<N>::POW2) return (N - k) & (N - 1);
    else return k == 0 || k == N ? 0 : N - k;
}
// Twiddles of the R2C row kernels: 2048-point lines keep the radix-8
// stages' stored powers in registers and read the last stage from the LDS
// table (0.39 -> 0.35 ms for the rows of a 1024 x 1024 x 128 volume); other
// lengths read every stage from the table (in registers the 1024-point
// kernel would pass 128 registers, and with them the occupancy its blocks
// need; 4096 would spill).
template <typename T, int N>
using RowTwiddles = std::conditional_t<N == 2048, RegTableTwiddles<T, N>, TableTwiddles<T, N>>;
// The C2R kernels hold the first such stage only (both would take them past
// the 128 registers of a 16-wave block).
template <typename T, int N>
using RowTwiddlesC2R = std::conditional_t<N == 2048, RegTableTwiddles<T, N, 1>, TableTwiddles<T, N>>;
template <typename T, int N, int NREG>
__device__ __forceinline__ void row_twiddles(RegTableTwiddles<T, N, NREG>& w, const cT<T>* __restrict__ tw, cT<T>* tab,
                                             int t)
{
    w.load(tw, tab, t);
}
template <typename T, int N>
__device__ __forceinline__ void row_twiddles(TableTwiddles<T, N>& w, const cT<T>* __restrict__, cT<T>* tab, int)
{
    w.p = tab;
}

// Power-of-two row kernels load the next group's rows into registers while
// the current group is transformed. The 2^a 3^b kernels hold more registers
// per line (radix 12) and run faster loading each group when they reach it.
template <int N> constexpr bool row_pipe() { return FftShape<N>::POW2; }

// Position of row group g of a job table: job k, batch b, group rg of the
// batch.  A persistent block visits g, g + G, g + 2G, ...: it decodes its
// first group and then advances by the job's gq = G / bpb batches and
// gr = G % bpb groups (set at launch), decoding again only where the step
// enters another job.
struct RowPos { int k, b, rg; };
__device__ __forceinline__ RowPos row_pos(const RowJobs& js, int g)
{
    RowPos p;
    p.k = find_job(js, g);
    const RowJob& J = js.j[p.k];
    const int gl = g - J.begin;
    p.b = gl / J.bpb;
    p.rg = gl - p.b * J.bpb;
    return p;
}
__device__ __forceinline__ RowPos row_pos_next(const RowJobs& js, const RowPos& p, int gn)
{
    if (p.k + 1 < js.njobs && gn >= js.j[p.k + 1].begin) return row_pos(js, gn);
    const RowJob& J = js.j[p.k];
    RowPos n{p.k, p.b + J.gq, p.rg + J.gr};
    if (n.rg >= J.bpb) {
        n.rg -= J.bpb;
        ++n.b;
    }
    return n;
}
// The host side of it: the table as launched on a grid of G blocks.
static inline RowJobs rows_for_grid(const RowJobs& jobs, int G)
{
    RowJobs js = jobs;
    for (int i = 0; i < js.njobs; ++i) {
        const int bpb = js.j[i].bpb > 0 ? js.j[i].bpb : 1;   // a job has >= 1 row
        js.j[i].gq = G / bpb;
        js.j[i].gr = G % bpb;
    }
    return js;
}

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
    constexpr int TPL = C::TPL, P = C::P;
    __shared__ cT<T> lds[C::LDS_R2C + TableTwiddles<T, N>::size()];
    const int G = gridDim.x, total = jobs.total;
    const int pr = threadIdx.x / TPL, t = threadIdx.x % TPL;
    TableTwiddles<T, N>::build(lds + C::LDS_R2C, tw, threadIdx.x, C::THREADS);
    lds_barrier();
    RowTwiddles<T, N> twl;
    row_twiddles(twl, tw, lds + C::LDS_R2C, threadIdx.x % C::TPL);
    cT<T>* xl = lds + pr * lds_line_elems(N);
    auto load = [&](const RowPos& p, cT<T> (&v)[P]) {
        const RowJob& J = jobs.j[p.k];
        const int ra = p.rg * C::RT + 2 * pr, rb = ra + 1;
        const TI* src = (const TI*)J.in + (int64_t)p.b * J.in_bs;
#pragma unroll
        for (int m = 0; m < P; ++m) {
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
    cT<T> v[P];
    constexpr bool PIPE = row_pipe<N>();
    RowPos pn = row_pos(jobs, g < total ? g : 0);
    if (PIPE && g < total) load(pn, v);
    for (; g < total; g += G) {
        const RowPos pc = pn;
        if (g + G < total) pn = row_pos_next(jobs, pc, g + G);
        cT<T> vn[P];
        if (!PIPE) load(pc, v);
        if (PIPE && g + G < total) load(pn, vn);
        const RowJob& J = jobs.j[pc.k];
        const int b = pc.b;
        const int row0 = pc.rg * C::RT;
        if (J.nv <= N / 2) fft_line<T, N, -1, true>(v, xl, twl, t);
        else fft_line<T, N, -1, false>(v, xl, twl, t);
        cT<T>* dst = (cT<T>*)J.out + (int64_t)b * J.out_bs;
        if constexpr (sizeof(T) == 4) {
            // stage Z = FFT(a + i c) of every pair by frequency, then split it
            // into the two rows' half spectra while the tile is stored:
            //   A[k] = (Z[k] + conj Z[N-k]) / 2,  C[k] = (Z[k] - conj Z[N-k]) / (2 i),
            // slot 0 packing the real bins 0 and N/2; element (kx, pair) stores
            // both rows (adjacent in the column) with one 16-byte store
            lds_barrier();
#pragma unroll
            for (int m = 0; m < P; ++m) lds[pr * C::ZR + t + m * TPL] = v[m];
            // v is free: take the next group's rows now, before this group's
            // stores, so that waiting for them does not wait for the stores
            if (PIPE) {
                wait_vmem();
#pragma unroll
                for (int m = 0; m < P; ++m) v[m] = vn[m];
            }
            lds_barrier();
#pragma unroll
            for (int i = 0; i < (C::HALF * C::PAIRS) / C::THREADS; ++i) {
                const int e = threadIdx.x + i * C::THREADS;
                const int kx = e / C::PAIRS, q = e % C::PAIRS;
                const cT<T> z = lds[q * C::ZR + kx];
                cT<T> A, Cc;
                if (kx == 0) {
                    const cT<T> zh = lds[q * C::ZR + N / 2];
                    A = mk<T>(z.x, zh.x);
                    Cc = mk<T>(z.y, zh.y);
                } else {
                    const cT<T> zr = lds[q * C::ZR + N - kx];
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
            lds_barrier();
#pragma unroll
            for (int m = 0; m < P; ++m) xl[lpad(t + m * TPL)] = v[m];
            lds_barrier();
            cT<T> A[P / 2 + 1], Cc[P / 2 + 1];
#pragma unroll
            for (int m = 0; m < P / 2 + 1; ++m) {
                const int k = t + m * TPL;
                if (m < P / 2 || t == 0) {
                    const cT<T> z = v[m];
                    const cT<T> zr = xl[lpad(mirror_pos<N>(k))];
                    A[m] = mk<T>((T)0.5 * (z.x + zr.x), (T)0.5 * (z.y - zr.y));
                    Cc[m] = mk<T>((T)0.5 * (z.y + zr.y), (T)0.5 * (zr.x - z.x));
                }
            }
            if (t == 0) {   // pack the real bins 0 and N/2 into slot 0
                A[0] = mk<T>(A[0].x, A[P / 2].x);
                Cc[0] = mk<T>(Cc[0].x, Cc[P / 2].x);
            }
            // v is free: take the next group's rows before the stores (as
            // in the FP32 branch)
            if (PIPE) {
                wait_vmem();
#pragma unroll
                for (int m = 0; m < P; ++m) v[m] = vn[m];
            }
            lds_barrier();
#pragma unroll
            for (int m = 0; m < P / 2; ++m) {
                const int k = t + m * TPL;
                lds[k * C::SROW + 2 * pr] = A[m];
                lds[k * C::SROW + 2 * pr + 1] = Cc[m];
            }
            lds_barrier();
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const int e = threadIdx.x + i * C::THREADS;   // HALF * RT = P * THREADS
                const int kx = e / C::RT, rr = e % C::RT;
                if (row0 + rr < J.nrows) dst[pidx(kx, row0 + rr, C::HALF)] = lds[kx * C::SROW + rr];
            }
        }
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
    constexpr int TPL = C::TPL, P = C::P;
    __shared__ cT<T> lds[C::LDS + TableTwiddles<T, N>::size()];
    const int G = gridDim.x, total = jobs.total;
    const int pr = threadIdx.x / TPL, t = threadIdx.x % TPL;
    TableTwiddles<T, N>::build(lds + C::TWO, tw, threadIdx.x, C::THREADS);
    lds_barrier();
    RowTwiddlesC2R<T, N> twl;
    row_twiddles(twl, tw, lds + C::TWO, threadIdx.x % C::TPL);
    cT<T>* xl = lds + pr * lds_line_elems(N);
    // tile of the packed half spectra of RT rows: HALF * RT = P * THREADS
    // elements, element e = threadIdx.x + i THREADS at (kx, row) = (e / RT, e % RT)
    // (8-byte loads: eight lanes per 64-byte column segment; 16-byte loads,
    // with twice the segments per instruction, measured slower)
    auto load = [&](const RowPos& p, cT<T> (&tl)[P]) {
        const RowJob& J = jobs.j[p.k];
        const int row0 = p.rg * C::RT;
        const cT<T>* src = (const cT<T>*)J.in + (int64_t)p.b * J.in_bs;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int e = threadIdx.x + i * C::THREADS;
            const int kx = e / C::RT, rr = e % C::RT;
            tl[i] = (row0 + rr < J.nrows) ? src[pidx(kx, row0 + rr, C::HALF)] : mk<T>(0, 0);
        }
    };
    int g = xcd_order(blockIdx.x, G);
    cT<T> tl[P];
    constexpr bool PIPE = row_pipe<N>();
    RowPos pn = row_pos(jobs, g < total ? g : 0);
    if (PIPE && g < total) load(pn, tl);
    for (; g < total; g += G) {
        const RowPos pc = pn;
        if (g + G < total) pn = row_pos_next(jobs, pc, g + G);
        if (!PIPE) load(pc, tl);
        lds_barrier();
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int e = threadIdx.x + i * C::THREADS;
            lds[(e % C::RT) * C::CR + e / C::RT] = tl[i];
        }
        lds_barrier();
        if (PIPE && g + G < total) load(pn, tl);
        // Z[k] = A[k] + i C[k] over the full length: slot 0 unpacks the real
        // bins 0 and N/2, Hermitian symmetry gives k > N/2.  Every lane reads
        // whole elements (the two bins in slot 0 are selected afterwards), so
        // the reads stay 8-byte accesses of consecutive slots.
        cT<T> v[P];
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int k = t + m * TPL;
            const int kk = k <= N / 2 ? k : N - k;
            const int ks = kk == N / 2 ? 0 : kk;
            cT<T> A = lds[(2 * pr) * C::CR + ks], Cc = lds[(2 * pr + 1) * C::CR + ks];
            if (kk == 0) {
                A.y = 0;
                Cc.y = 0;
            } else if (kk == N / 2) {
                A = mk<T>(A.y, 0);
                Cc = mk<T>(Cc.y, 0);
            } else if (k > N / 2) {
                A.y = -A.y;
                Cc.y = -Cc.y;
            }
            v[m] = mk<T>(A.x - Cc.y, A.y + Cc.x);
        }
        fft_line<T, N, +1, false>(v, xl, twl, t);   // begins with a barrier
        const RowJob& J = jobs.j[pc.k];
        const int ra = pc.rg * C::RT + 2 * pr, rb = ra + 1;
        // buffer stores (no branches; the launcher checks the sizes)
        const auto rs = buf_rsrc((T*)J.out + (int64_t)pc.b * J.out_bs,
                                 (uint32_t)((int64_t)J.nrows * J.out_ld * (int64_t)sizeof(T)));
        const uint32_t ska = ra < J.nrows ? 0u : BUF_SKIP, skb = rb < J.nrows ? 0u : BUF_SKIP;
        const uint32_t oa0 = (uint32_t)((int64_t)ra * J.out_ld * (int64_t)sizeof(T));
        const uint32_t ld = (uint32_t)(J.out_ld * (int64_t)sizeof(T));
        // rows that end within the first half of the transform issue no
        // stores for the second half (a uniform branch: the stores of the
        // first half stay unconditional, so the wait stays countable)
        const bool half = J.nv <= N / 2;
#pragma unroll
        for (int m = 0; m < P; ++m) {
            if (m >= P / 2 && half) continue;
            const int x = t + m * TPL;
            const uint32_t oa = oa0 + (uint32_t)x * (uint32_t)sizeof(T), skx = x < J.nv ? 0u : BUF_SKIP;
            buf_store(v[m].x, rs, oa | ska | skx);
            buf_store(v[m].y, rs, (oa + ld) | skb | skx);
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
    static constexpr int TPL = FftShape<N>::TPL;
    static constexpr int LPB = lines_per_block(TPL);          // tiles per block
    static constexpr int THREADS = LPB * TPL;
};

template <typename TI, typename T, int N>
__global__ void __launch_bounds__(TileCfg<N>::THREADS)
k_rows_r2c_t(RowJobs jobs, const cT<T>* __restrict__ tw)
{
    using C = TileCfg<N>;
    constexpr int TPL = C::TPL, P = FftShape<N>::P;
    constexpr int LL = lds_line_elems(N);
    __shared__ cT<T> lds[C::LPB * LL + TableTwiddles<T, N>::size()];
    TableTwiddles<T, N>::build(lds + C::LPB * LL, tw, threadIdx.x, C::THREADS);
    lds_barrier();
    RowTwiddles<T, N> twl;
    row_twiddles(twl, tw, lds + C::LPB * LL, threadIdx.x % C::TPL);
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
        T a[8][P];
#pragma unroll
        for (int rr = 0; rr < 8; ++rr)
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const int x = t + m * TPL;
                a[rr][m] = (live && x < J.nv && row0 + rr < J.nrows) ? (T)src[(int64_t)(row0 + rr) * J.in_ld + x] : (T)0;
            }
        cT<T> o[P / 2][8];   // o[m][row]: half-spectrum value at k = t + m TPL
        cT<T> o0n[2];    // bin N/2 of the pair's two rows (thread 0)
        const bool zhi = J.nv <= N / 2;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            cT<T> v[P];
#pragma unroll
            for (int m = 0; m < P; ++m) v[m] = mk<T>(a[2 * p][m], a[2 * p + 1][m]);
            if (zhi) fft_line<T, N, -1, true>(v, xl, twl, t);
            else fft_line<T, N, -1, false>(v, xl, twl, t);
            lds_barrier();
#pragma unroll
            for (int m = 0; m < P; ++m) xl[lpad(t + m * TPL)] = v[m];
            lds_barrier();
#pragma unroll
            for (int m = 0; m < P / 2 + 1; ++m) {
                const int k = t + m * TPL;
                if (m < P / 2 || t == 0) {
                    const cT<T> z = v[m], zr = xl[lpad(mirror_pos<N>(k))];
                    const cT<T> A = mk<T>((T)0.5 * (z.x + zr.x), (T)0.5 * (z.y - zr.y));
                    const cT<T> Cc = mk<T>((T)0.5 * (z.y + zr.y), (T)0.5 * (zr.x - z.x));
                    if (m < P / 2) {
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
            for (int m = 0; m < P / 2; ++m) {
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
    constexpr int TPL = C::TPL, P = FftShape<N>::P;
    constexpr int LL = lds_line_elems(N);
    __shared__ cT<T> lds[C::LPB * LL + TableTwiddles<T, N>::size()];
    TableTwiddles<T, N>::build(lds + C::LPB * LL, tw, threadIdx.x, C::THREADS);
    lds_barrier();
    RowTwiddlesC2R<T, N> twl;
    row_twiddles(twl, tw, lds + C::LPB * LL, threadIdx.x % C::TPL);
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
        cT<T> c[P / 2][8];   // c[m][row]: packed half spectrum at k = t + m TPL
#pragma unroll
        for (int m = 0; m < P / 2; ++m) {
            const cT<T>* col = src + pidx(t + m * TPL, row0, N / 2);   // row0 % PANEL == 0
#pragma unroll
            for (int rr = 0; rr < 8; ++rr) c[m][rr] = (live && row0 + rr < J.nrows) ? col[rr] : mk<T>(0, 0);
        }
        T* dst = (T*)J.out + (int64_t)b * J.out_bs;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            // the pair's half spectra A (row 2p) and C (row 2p+1) at k < N/2
            // go through LDS so that each thread can read its mirror positions
            lds_barrier();
#pragma unroll
            for (int m = 0; m < P / 2; ++m) {
                xl[lpad(t + m * TPL)] = c[m][2 * p];
                xl[lpad(N / 2 + t + m * TPL)] = c[m][2 * p + 1];
            }
            lds_barrier();
            cT<T> v[P];
#pragma unroll
            for (int m = 0; m < P; ++m) {
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
                for (int m = 0; m < P; ++m) {
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
    constexpr int TPL = C::TPL, P = FftShape<N>::P;
    __shared__ double2 lds[C::CPW * lds_line_elems(N)];
    const int cl = threadIdx.x / TPL, t = threadIdx.x % TPL;
    const int col = blockIdx.x * C::CPW + cl;
    const int l = blockIdx.y;
    const bool ok = col < ncols;
    double2 v[P];
    const double2* src = in + (int64_t)l * ncols * N;
#pragma unroll
    for (int m = 0; m < P; ++m) v[m] = ok ? src[pidx(col, t + m * TPL, ncols)] : make_double2(0.0, 0.0);
    LineTwiddles<double, N> twl;
    twl.load(tw, t);
    fft_line<double, N, -1, false>(v, lds + cl * lds_line_elems(N), twl, t);
    if (!ok) return;
    if (form == FORM_COMPLEX) {
        cT<T>* dst = (cT<T>*)spec + ((int64_t)(r0 + l) * ncols + col) * N;
#pragma unroll
        for (int m = 0; m < P; ++m) dst[t + m * TPL] = mk<T>((T)(v[m].x * scale), (T)(v[m].y * scale));
    } else {
        T* base = (T*)spec + (int64_t)(r0 + l) * (ncols + 1) * ldr;
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int y = t + m * TPL;
            if (y > N / 2) continue;
            base[(int64_t)col * ldr + y] = (T)(v[m].x * scale);
            if (col == 0) base[(int64_t)ncols * ldr + y] = (T)(v[m].y * scale);
        }
    }
}

template <typename TI, typename T, int NN, int P0>
static hipError_t launch_r2c_n(const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    using C = RowCfg<T, NN, P0>;
    // thread-safe one-time initialisation (function-local static)
    static const int resident = resident_blocks((const void*)k_rows_r2c<TI, T, NN, P0>, C::THREADS);
    const int G = persistent_grid(jobs.total, resident);
    hipLaunchKernelGGL((k_rows_r2c<TI, T, NN, P0>), dim3(G), dim3(C::THREADS), 0, s, rows_for_grid(jobs, G), tw);
    return hipGetLastError();
}

template <typename T, int NN, int P0>
static hipError_t launch_c2r_n(const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    using C = RowCfg<T, NN, P0>;
    // thread-safe one-time initialisation (function-local static)
    static const int resident = resident_blocks((const void*)k_rows_c2r<T, NN, P0>, C::THREADS);
    // the kernel's buffer stores address a batch's rows (and the rows of a
    // partial last group) with 32-bit byte offsets below 2^31
    for (int i = 0; i < jobs.njobs; ++i)
        if ((int64_t)(jobs.j[i].nrows + C::RT) * jobs.j[i].out_ld * (int64_t)sizeof(T) >= BUF_MAX_BYTES)
            return hipErrorInvalidValue;
    const int G = persistent_grid(jobs.total, resident);
    hipLaunchKernelGGL((k_rows_c2r<T, NN, P0>), dim3(G), dim3(C::THREADS), 0, s, rows_for_grid(jobs, G), tw);
    return hipGetLastError();
}

template <typename TI, typename T, int NN>
static hipError_t launch_r2c_t(const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    using C = TileCfg<NN>;
    // thread-safe one-time initialisation (function-local static)
    static const int resident = resident_blocks((const void*)k_rows_r2c_t<TI, T, NN>, C::THREADS);
    const int nb = (jobs.total + C::LPB - 1) / C::LPB;
    hipLaunchKernelGGL((k_rows_r2c_t<TI, T, NN>), dim3(persistent_grid(nb, resident)), dim3(C::THREADS), 0, s, jobs, tw);
    return hipGetLastError();
}

template <typename T, int NN>
static hipError_t launch_c2r_t(const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    using C = TileCfg<NN>;
    // thread-safe one-time initialisation (function-local static)
    static const int resident = resident_blocks((const void*)k_rows_c2r_t<T, NN>, C::THREADS);
    const int nb = (jobs.total + C::LPB - 1) / C::LPB;
    hipLaunchKernelGGL((k_rows_c2r_t<T, NN>), dim3(persistent_grid(nb, resident)), dim3(C::THREADS), 0, s, jobs, tw);
    return hipGetLastError();
}

template <typename TI, typename T, int NN>
hipError_t rows_r2c_n(int tile, const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    return tile == 8 ? launch_r2c_t<TI, T, NN>(jobs, tw, s)
         : tile == 1 ? launch_r2c_n<TI, T, NN, 1>(jobs, tw, s)
         : tile == 2 ? launch_r2c_n<TI, T, NN, 2>(jobs, tw, s)
                     : launch_r2c_n<TI, T, NN, 4>(jobs, tw, s);
}

template <typename T, int NN>
hipError_t rows_c2r_n(int tile, const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    return tile == 8 ? launch_c2r_t<T, NN>(jobs, tw, s)
         : tile == 1 ? launch_c2r_n<T, NN, 1>(jobs, tw, s)
         : tile == 2 ? launch_c2r_n<T, NN, 2>(jobs, tw, s)
                     : launch_c2r_n<T, NN, 4>(jobs, tw, s);
}

template <typename T, int NN>
hipError_t cols_spec_n(const double2* in, int ncols, int nl, void* spec, int r0, double scale, const double2* tw,
                       int form, int64_t ldr, hipStream_t s)
{
    using C = ColCfg<NN>;
    dim3 grid((ncols + C::CPW - 1) / C::CPW, nl);
    hipLaunchKernelGGL((k_cols_spec<T, NN>), grid, dim3(C::THREADS), 0, s, in, ncols, spec, r0, scale, tw, form, ldr);
    return hipGetLastError();
}

// every launcher of length NN
#define BTTB_ROWS_INSTANTIATE(NN)                                                                               \
    template hipError_t rows_r2c_n<double, double, NN>(int, const RowJobs&, const double2*, hipStream_t);      \
    template hipError_t rows_r2c_n<float, float, NN>(int, const RowJobs&, const float2*, hipStream_t);         \
    template hipError_t rows_c2r_n<double, NN>(int, const RowJobs&, const double2*, hipStream_t);              \
    template hipError_t rows_c2r_n<float, NN>(int, const RowJobs&, const float2*, hipStream_t);                \
    template hipError_t cols_spec_n<double, NN>(const double2*, int, int, void*, int, double, const double2*,  \
                                                int, int64_t, hipStream_t);                                     \
    template hipError_t cols_spec_n<float, NN>(const double2*, int, int, void*, int, double, const double2*,   \
                                               int, int64_t, hipStream_t);

}  // namespace bttbk
