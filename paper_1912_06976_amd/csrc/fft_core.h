// fft_core.h -- register/LDS Stockham FFT building blocks for gfx950.
//
// One transform ("line") of length N is spread over TPL = N / P threads;
// thread t of the line holds the P elements at positions t + m * TPL
// (m = 0..P-1) in registers, both before and after the transform, in natural
// order.  Two families of lengths:
//   * powers of two, 8 <= N <= 4096: P = 8, radix-8 stages followed by at
//     most one radix-2 or radix-4 stage;
//   * N = 2^a 3^b with b in {1, 2}, 96 <= N <= 3072: P = 12, a radix-12
//     first stage, a second radix-12 stage when a factor 3 remains, then
//     radix-4 stages and at most one radix-2 stage.
// All stages are decimation in time, Stockham auto-sort: a stage of radix R
// with current sub-transform length L maps butterfly b (P / R of them per
// thread: b = t + u * TPL, u < P / R) with inputs at b + i N / R to outputs at
// (b / L) L R + (b mod L) + i L after multiplying input i by w^(i (b mod L)),
// w = exp(-+ 2 pi i / (L R)).  Between stages the elements are exchanged
// through a padded LDS buffer.  For the last stage L R = N, so its outputs
// land on the same register slots as the inputs: no final exchange.
//
// Twiddles are read from a table tw[k] = exp(-2 pi i k / N), k < N, computed
// in FP64 and rounded to the working precision.  A per-thread copy of the
// twiddles each stage needs is held in registers (struct LineTwiddles) so a
// kernel that transforms many lines of the same length loads them once; the
// alternative TableTwiddles reads a stage-major copy of them in LDS (for the
// radix-8 stages three powers per butterfly, the other four formed by
// products), and RegTableTwiddles keeps those three powers in registers.
// Every twiddle product is rounded the same way whatever the source.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "bttb_internal.h"

namespace bttbk {

template <typename T> __device__ __forceinline__ cT<T> mk(T x, T y) { cT<T> r; r.x = x; r.y = y; return r; }
template <typename T> __device__ __forceinline__ cT<T> cadd(cT<T> a, cT<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cT<T> csub(cT<T> a, cT<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cT<T> cmul(cT<T> a, cT<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T> __device__ __forceinline__ cT<T> cmulc(cT<T> a, cT<T> b) {
    return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T> __device__ __forceinline__ cT<T> cconj(cT<T> a) { return mk<T>(a.x, -a.y); }
// multiply by -i (DIR = -1) or +i (DIR = +1)
template <typename T, int DIR> __device__ __forceinline__ cT<T> mul_i(cT<T> a) {
    return DIR < 0 ? mk<T>(a.y, -a.x) : mk<T>(-a.y, a.x);
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n >> 1); }

// LDS index of position x of a line buffer: the low five bits XORed with
// bits 3..7, a permutation within each aligned block of 32 elements that
// spreads the strided Stockham writes and the contiguous reads of fft_line
// over the LDS banks (no conflicts for N >= 64 with 8- or 16-byte elements).
// Line buffers of one block are lds_line_elems(n) elements apart; the small
// offset spreads the lines that share a wave.
// A line buffer holds whole aligned blocks of 32 (the permutation stays
// inside its block): lengths that are neither a power of two (below 32 the
// permutation is the identity or stays below the length) nor a multiple of
// 32 are rounded up.
constexpr bool is_pow2c(int n) { return n > 0 && (n & (n - 1)) == 0; }
__device__ __forceinline__ int lpad(int x) { return x ^ ((x >> 3) & 31); }
constexpr int lds_line_elems(int n)
{
    return (is_pow2c(n) || n % 32 == 0 ? n : (n / 32 + 1) * 32) + (n >= 64 ? 8 : 4);
}

// Radix of stage s (0 = first) of a 12-points-per-thread transform of length
// N, 0 past the last stage: 12 while the remaining length has a factor 12,
// 6 or 3 for a last factor 3, then 4 while a factor 4 remains, then 2.
constexpr int mr_radix(int N, int s)
{
    int M = N;
    for (int k = 0; M > 1; ++k) {
        const int R = M % 3 == 0 ? (M % 12 == 0 ? 12 : (M % 6 == 0 ? 6 : 3)) : (M % 4 == 0 ? 4 : 2);
        if (k == s) return R;
        M /= R;
    }
    return 0;
}
// sub-transform length before stage s (product of the earlier radices)
constexpr int mr_span(int N, int s)
{
    int L = 1;
    for (int k = 0; k < s; ++k) L *= mr_radix(N, k);
    return L;
}
constexpr int mr_nstages(int N)
{
    int k = 0;
    while (mr_radix(N, k) != 0) ++k;
    return k;
}
// register twiddles of stages 1.. (P / R butterflies of R - 1 twiddles each)
constexpr int mr_ntw(int N)
{
    int n = 0;
    for (int s = 1; s < mr_nstages(N); ++s) n += (12 / mr_radix(N, s)) * (mr_radix(N, s) - 1);
    return n;
}
// stage-major table entries of stages 1.. ((R - 1) L each)
constexpr int mr_ntab(int N)
{
    int n = 0;
    for (int s = 1; s < mr_nstages(N); ++s) n += (mr_radix(N, s) - 1) * mr_span(N, s);
    return n;
}
constexpr bool mr_length_ok(int N)
{
    int M = N, b = 0;
    while (M % 3 == 0) { M /= 3; ++b; }
    return b >= 1 && b <= 2 && is_pow2c(M) && N >= 96 && N <= 3072;
}

template <int N> struct FftShape {
    static constexpr bool POW2 = is_pow2c(N);
    static constexpr int P = POW2 ? 8 : 12;        // points per thread
    static constexpr int TPL = N / P;              // threads per line
    static constexpr int LOG = ilog2(N);
    static constexpr int S8 = LOG / 3;             // radix-8 stages (powers of two)
    static constexpr int RL = 1 << (LOG % 3);      // last small radix (1: none)
    static constexpr int NTW = POW2 ? 7 * (S8 > 0 ? S8 - 1 : 0) + (RL > 1 ? (8 / RL) * (RL - 1) : 0) : mr_ntw(N);
    // a line lies within one wavefront (no line straddles two)
    static constexpr bool WAVE_LOCAL = 64 % TPL == 0;
    static_assert((POW2 && N >= 8 && N <= 4096) || (!POW2 && mr_length_ok(N)),
                  "length: a power of two in [8, 4096] or 2^a 3^b (b = 1, 2) in [96, 3072]");
};

// ---- small DFTs (in place on register arrays) ----
template <typename T, int DIR> __device__ __forceinline__ void dft2(cT<T>& a, cT<T>& b) {
    cT<T> s = cadd<T>(a, b), d = csub<T>(a, b);
    a = s; b = d;
}
template <typename T, int DIR>
__device__ __forceinline__ void dft4(cT<T>& a0, cT<T>& a1, cT<T>& a2, cT<T>& a3) {
    cT<T> s0 = cadd<T>(a0, a2), d0 = csub<T>(a0, a2);
    cT<T> s1 = cadd<T>(a1, a3), d1 = mul_i<T, DIR>(csub<T>(a1, a3));
    a0 = cadd<T>(s0, s1);
    a2 = csub<T>(s0, s1);
    a1 = cadd<T>(d0, d1);
    a3 = csub<T>(d0, d1);
}
// x * w8 and x * w8^3, w8 = exp(DIR 2 pi i / 8)
template <typename T, int DIR> __device__ __forceinline__ cT<T> mul_w8(cT<T> a) {
    const T r = (T)0.70710678118654752440084436210484903928;
    return DIR < 0 ? mk<T>((a.x + a.y) * r, (a.y - a.x) * r) : mk<T>((a.x - a.y) * r, (a.x + a.y) * r);
}
template <typename T, int DIR> __device__ __forceinline__ cT<T> mul_w83(cT<T> a) {
    const T r = (T)0.70710678118654752440084436210484903928;
    return DIR < 0 ? mk<T>((a.y - a.x) * r, -(a.x + a.y) * r) : mk<T>(-(a.x + a.y) * r, (a.x - a.y) * r);
}
// 8-point DFT of a[0..7] (natural order in, natural order out)
template <typename T, int DIR> __device__ __forceinline__ void dft8(cT<T>* a) {
    // even / odd 4-point halves
    cT<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
    cT<T> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
    dft4<T, DIR>(e0, e1, e2, e3);
    dft4<T, DIR>(o0, o1, o2, o3);
    o1 = mul_w8<T, DIR>(o1);
    o2 = mul_i<T, DIR>(o2);
    o3 = mul_w83<T, DIR>(o3);
    a[0] = cadd<T>(e0, o0); a[4] = csub<T>(e0, o0);
    a[1] = cadd<T>(e1, o1); a[5] = csub<T>(e1, o1);
    a[2] = cadd<T>(e2, o2); a[6] = csub<T>(e2, o2);
    a[3] = cadd<T>(e3, o3); a[7] = csub<T>(e3, o3);
}

// 3-point DFT in place, w3 = exp(DIR 2 pi i / 3): with s = b + c, d = b - c,
// X0 = a + s, X1 = a - s/2 + DIR i (sqrt 3 / 2) d, X2 = a - s/2 - DIR i (sqrt 3 / 2) d
template <typename T, int DIR> __device__ __forceinline__ void dft3(cT<T>& a, cT<T>& b, cT<T>& c) {
    const T h = (T)0.86602540378443864676372317075293618;   // sin(pi / 3)
    const cT<T> s = cadd<T>(b, c), d = csub<T>(b, c);
    const cT<T> x0 = cadd<T>(a, s);
    const cT<T> m = mk<T>(a.x - (T)0.5 * s.x, a.y - (T)0.5 * s.y);
    const cT<T> u = mul_i<T, DIR>(mk<T>(h * d.x, h * d.y));
    a = x0;
    b = cadd<T>(m, u);
    c = csub<T>(m, u);
}
// x * (c + i DIR s) for the constants (c, s) = (cos, sin) of an angle
template <typename T, int DIR> __device__ __forceinline__ cT<T> mul_cs(cT<T> a, T c, T s) {
    const T ds = DIR < 0 ? -s : s;
    return mk<T>(a.x * c - a.y * ds, a.x * ds + a.y * c);
}
// 12-point DFT of the slots a[u + i K], i < 12 (natural order in and out),
// as three 4-point DFTs over n = n1 + 3 n2, the twiddles w12^(n1 k2), and
// four 3-point DFTs giving X[k2 + 4 k1].  ZERO_HI: inputs 6..11 are zero
// (each 4-point DFT then has two zero inputs).
template <typename T, int DIR, bool ZERO_HI, int K>
__device__ __forceinline__ void dft12(cT<T>* a, int u)
{
    const T c30 = (T)0.86602540378443864676372317075293618, s30 = (T)0.5;
    cT<T> y[3][4];
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1) {
        if constexpr (ZERO_HI) {
            const cT<T> p = a[u + n1 * K], q = a[u + (n1 + 3) * K];
            const cT<T> iq = mul_i<T, DIR>(q);
            y[n1][0] = cadd<T>(p, q);
            y[n1][1] = cadd<T>(p, iq);
            y[n1][2] = csub<T>(p, q);
            y[n1][3] = csub<T>(p, iq);
        } else {
            y[n1][0] = a[u + n1 * K];
            y[n1][1] = a[u + (n1 + 3) * K];
            y[n1][2] = a[u + (n1 + 6) * K];
            y[n1][3] = a[u + (n1 + 9) * K];
            dft4<T, DIR>(y[n1][0], y[n1][1], y[n1][2], y[n1][3]);
        }
    }
    // w12^1 = (c30, s30), w12^2 = (s30, c30), w12^3 = DIR i, w12^4 = (-s30, c30), w12^6 = -1
    y[1][1] = mul_cs<T, DIR>(y[1][1], c30, s30);
    y[1][2] = mul_cs<T, DIR>(y[1][2], s30, c30);
    y[1][3] = mul_i<T, DIR>(y[1][3]);
    y[2][1] = mul_cs<T, DIR>(y[2][1], s30, c30);
    y[2][2] = mul_cs<T, DIR>(y[2][2], -s30, c30);
    y[2][3] = mk<T>(-y[2][3].x, -y[2][3].y);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
        dft3<T, DIR>(y[0][k2], y[1][k2], y[2][k2]);
        a[u + k2 * K] = y[0][k2];
        a[u + (k2 + 4) * K] = y[1][k2];
        a[u + (k2 + 8) * K] = y[2][k2];
    }
}
// 6-point DFT of the slots a[u + i K] (3 x 2: n = n1 + 3 n2, X[k2 + 2 k1])
template <typename T, int DIR, int K>
__device__ __forceinline__ void dft6(cT<T>* a, int u)
{
    const T c60 = (T)0.5, s60 = (T)0.86602540378443864676372317075293618;
    cT<T> y[3][2];
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1) {
        y[n1][0] = a[u + n1 * K];
        y[n1][1] = a[u + (n1 + 3) * K];
        dft2<T, DIR>(y[n1][0], y[n1][1]);
    }
    // w6^(n1 k2): w6^1 = (c60, s60), w6^2 = (-c60, s60)
    y[1][1] = mul_cs<T, DIR>(y[1][1], c60, s60);
    y[2][1] = mul_cs<T, DIR>(y[2][1], -c60, s60);
#pragma unroll
    for (int k2 = 0; k2 < 2; ++k2) {
        dft3<T, DIR>(y[0][k2], y[1][k2], y[2][k2]);
        a[u + k2 * K] = y[0][k2];
        a[u + (k2 + 2) * K] = y[1][k2];
        a[u + (k2 + 4) * K] = y[2][k2];
    }
}

// register twiddles of stages 1 .. s - 1 of a 12-points-per-thread transform
constexpr int mr_twc(int N, int s)
{
    int n = 0;
    for (int k = 1; k < s; ++k) n += (12 / mr_radix(N, k)) * (mr_radix(N, k) - 1);
    return n;
}

// compile-time loop: f(integral_constant<int, i>) for i in [B, E)
template <int B, int E, typename F> __device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Per-thread twiddles of one line of length N (forward sign; the inverse
// uses the conjugates).  tw points to the table of length N.
template <typename T, int N> struct LineTwiddles {
    using S = FftShape<N>;
    cT<T> w[S::NTW > 0 ? S::NTW : 1];
    __device__ __forceinline__ void load(const cT<T>* __restrict__ tw, int t) {
        if constexpr (S::POW2) {
            int c = 0;
            int L = 8;
#pragma unroll
            for (int s = 1; s < S::S8; ++s) {
                const int j = t % L;
                const int step = N / (8 * L);
#pragma unroll
                for (int i = 1; i < 8; ++i) w[c++] = tw[(i * j * step) & (N - 1)];
                L *= 8;
            }
            if constexpr (S::RL > 1) {
#pragma unroll
                for (int u = 0; u < 8 / S::RL; ++u) {
                    const int j = (t + u * S::TPL) % L;
#pragma unroll
                    for (int i = 1; i < S::RL; ++i) w[c++] = tw[(i * j) & (N - 1)];
                }
            }
        } else {
            // stage s >= 1 of radix R, span L: butterfly u's input i takes
            // w^(i j) = tw[i j N / (L R)], j = (t + u TPL) mod L
            static_for<1, mr_nstages(N)>([&](auto sI) {
                constexpr int s = decltype(sI)::value;
                constexpr int R = mr_radix(N, s), L = mr_span(N, s), NB = 12 / R, C0 = mr_twc(N, s);
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    const int j = (t + u * S::TPL) % L;
#pragma unroll
                    for (int i = 1; i < R; ++i) w[C0 + u * (R - 1) + i - 1] = tw[i * j * (N / (L * R))];
                }
            });
        }
    }
};

// Alternative twiddle source: a stage-major table (typically in LDS) that
// saves the registers of LineTwiddles.  Stage s >= 1 of radix R and span L
// holds w^(i j N/(L R)) at [off(s) + (i-1) L + j], 1 <= i < R, j < L; for
// powers of two the radix-8 stages (L = 8^s) hold only i = 1, 2, 4 at
// [off(s) + k L + j], i = 2^k (the other four are their products, formed at
// use by tw_stage8), and the final radix-RL stage sits at off(S8) in the
// full form.  A stage's reads by consecutive threads are consecutive (or
// broadcast) entries, so they do not conflict on the LDS banks.
template <typename T, int N> struct TableTwiddles {
    using S = FftShape<N>;
    const cT<T>* p;
    // entries before stage s
    static constexpr int off(int s) {
        int o = 0;
        if constexpr (S::POW2) {
            int L = 8;
            for (int k = 1; k < s; ++k) { o += 3 * L; L *= 8; }
        } else {
            for (int k = 1; k < s; ++k) o += (mr_radix(N, k) - 1) * mr_span(N, k);
        }
        return o;
    }
    static constexpr int size() {
        if constexpr (S::POW2) return off(S::S8) + (S::RL > 1 ? (S::RL - 1) * (N / S::RL) : 0);
        else return mr_ntab(N);
    }
    // fill dst[0 .. size()) from the natural table tw (all threads of the block)
    static __device__ void build(cT<T>* dst, const cT<T>* __restrict__ tw, int tid, int nthreads) {
        if constexpr (S::POW2) {
            for (int e = tid; e < size(); e += nthreads) {
                int idx;
                if (e < off(S::S8)) {
                    // radix-8 stage s: w^j, w^(2j), w^(4j) (w = the stage's
                    // root), component-major
                    int s = 1, L = 8;
                    while (e >= off(s + 1)) { ++s; L *= 8; }
                    const int r = e - off(s), i = 1 << (r / L), j = r % L;
                    idx = i * j * (N / (8 * L));
                } else {
                    const int L = N / S::RL, r = e - off(S::S8), i = r / L + 1, j = r % L;
                    idx = i * j;
                }
                dst[e] = tw[idx & (N - 1)];
            }
        } else {
            // stage by stage, with the stage's span, radix and offset known at
            // compile time (divisions by constants)
            static_for<1, mr_nstages(N)>([&](auto sI) {
                constexpr int s = decltype(sI)::value;
                constexpr int R = mr_radix(N, s), L = mr_span(N, s), O = off(s);
                for (int e = tid; e < (R - 1) * L; e += nthreads) {
                    const int i = e / L + 1, j = e % L;
                    dst[O + e] = tw[i * j * (N / (L * R))];
                }
            });
        }
    }
};

template <typename T, int N>
__device__ __forceinline__ cT<T> tw_get(const LineTwiddles<T, N>& tw, int c, int, int, int, int) { return tw.w[c]; }
template <typename T, int N>
__device__ __forceinline__ cT<T> tw_get(const TableTwiddles<T, N>& tw, int, int s, int L, int i, int j) {
    return tw.p[TableTwiddles<T, N>::off(s) + (i - 1) * L + j];
}
// product a b with the contraction written out (the table route forms four
// of a radix-8 butterfly's seven twiddles this way; every kernel that reads
// the table thus gets the same values)
template <typename T> __device__ __forceinline__ cT<T> cmul_fixed(cT<T> a, cT<T> b) {
    if constexpr (sizeof(T) == 4)
        return mk<T>(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
    else
        return mk<T>(__builtin_fma(a.x, b.x, -(a.y * b.y)), __builtin_fma(a.x, b.y, a.y * b.x));
}
// the seven twiddles w^(i j), i = 1..7, of radix-8 stage s (span L) for
// butterfly j: from registers, or from the table's w^j, w^(2j), w^(4j) and
// their products (three LDS reads instead of seven)
template <typename T, int N>
__device__ __forceinline__ void tw_stage8(const LineTwiddles<T, N>& tw, int c, int, int, int, cT<T> (&w)[7]) {
#pragma unroll
    for (int i = 0; i < 7; ++i) w[i] = tw.w[c + i];
}
template <typename T, int N>
__device__ __forceinline__ void tw_stage8(const TableTwiddles<T, N>& tw, int, int s, int L, int j, cT<T> (&w)[7]) {
    const cT<T>* q = tw.p + TableTwiddles<T, N>::off(s) + j;
    const cT<T> w1 = q[0], w2 = q[L], w4 = q[2 * L];
    const cT<T> w3 = cmul_fixed<T>(w1, w2);
    w[0] = w1;
    w[1] = w2;
    w[2] = w3;
    w[3] = w4;
    w[4] = cmul_fixed<T>(w1, w4);
    w[5] = cmul_fixed<T>(w2, w4);
    w[6] = cmul_fixed<T>(w3, w4);
}
// Twiddles of a kernel whose threads each keep one position t in every
// transform (the row kernels), powers of two: the three stored powers w^j,
// w^(2j), w^(4j) of each radix-8 stage in registers (j = t mod L is fixed
// per thread), the final radix-RL stage read from the table.  The values
// equal TableTwiddles' bit for bit (the same entries, the same products).
template <typename T, int N, int NREG = FftShape<N>::S8 - 1> struct RegTableTwiddles {
    using S = FftShape<N>;
    static_assert(S::POW2, "register-held radix-8 powers need a power-of-two length");
    static constexpr int NR = NREG < S::S8 - 1 ? NREG : S::S8 - 1;   // radix-8 stages held in registers
    cT<T> b[NR > 0 ? NR : 1][3];
    const cT<T>* p;            // the table (built by TableTwiddles::build)
    // tw: the natural table in global memory; tab: the LDS table
    __device__ __forceinline__ void load(const cT<T>* __restrict__ tw, const cT<T>* tab, int t) {
        p = tab;
        int L = 8;
#pragma unroll
        for (int s = 1; s <= NR; ++s) {
            const int j = t % L, step = N / (8 * L);
#pragma unroll
            for (int k = 0; k < 3; ++k) b[s - 1][k] = tw[((1 << k) * j * step) & (N - 1)];
            L *= 8;
        }
    }
};
template <typename T, int N, int NREG>
__device__ __forceinline__ void tw_stage8(const RegTableTwiddles<T, N, NREG>& tw, int c, int s, int L, int j,
                                          cT<T> (&w)[7]) {
    if (s > RegTableTwiddles<T, N, NREG>::NR) {
        tw_stage8<T, N>(TableTwiddles<T, N>{tw.p}, c, s, L, j, w);
        return;
    }
    const cT<T> w1 = tw.b[s - 1][0], w2 = tw.b[s - 1][1], w4 = tw.b[s - 1][2];
    const cT<T> w3 = cmul_fixed<T>(w1, w2);
    w[0] = w1;
    w[1] = w2;
    w[2] = w3;
    w[3] = w4;
    w[4] = cmul_fixed<T>(w1, w4);
    w[5] = cmul_fixed<T>(w2, w4);
    w[6] = cmul_fixed<T>(w3, w4);
}
template <typename T, int N, int NREG>
__device__ __forceinline__ cT<T> tw_get(const RegTableTwiddles<T, N, NREG>& tw, int, int s, int L, int i, int j) {
    return tw.p[TableTwiddles<T, N>::off(s) + (i - 1) * L + j];
}
// the same for stage S of a 12-point transform (the table offset a constant)
template <typename T, int N, int S>
__device__ __forceinline__ cT<T> tw_get_mr(const LineTwiddles<T, N>& tw, int c, int, int, int) { return tw.w[c]; }
template <typename T, int N, int S>
__device__ __forceinline__ cT<T> tw_get_mr(const TableTwiddles<T, N>& tw, int, int L, int i, int j) {
    constexpr int O = TableTwiddles<T, N>::off(S);
    return tw.p[O + (i - 1) * L + j];
}

// Block barrier for the LDS exchanges and staging buffers: the fences order
// the block's LDS accesses only (workgroup scope, local address space), so
// the barrier waits for this wavefront's LDS operations but not for its
// global loads in flight -- a prefetch of the next layer or row group keeps
// running across the exchanges of the current transform (__syncthreads()
// would wait for it at the first exchange).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Ordering of one wavefront's LDS writes and reads without a block barrier:
// the LDS executes a wavefront's operations in issue order, so a scheduling
// barrier between wavefront-scope fences suffices for lanes of one wavefront
// to read what other lanes of it wrote.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// a w (DIR < 0) or a conj(w) (DIR > 0), with the contraction into fused
// multiply-adds written out: every kernel rounds a twiddle product the same
// way, whatever its twiddles' source (registers or LDS)
template <typename T> __device__ __forceinline__ T fma_t(T a, T b, T c) {
    if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}
template <typename T, int DIR> __device__ __forceinline__ cT<T> twmul(cT<T> a, cT<T> w) {
    if constexpr (DIR < 0) return mk<T>(fma_t<T>(a.x, w.x, -(a.y * w.y)), fma_t<T>(a.x, w.y, a.y * w.x));
    else return mk<T>(fma_t<T>(a.x, w.x, a.y * w.y), fma_t<T>(a.y, w.x, -(a.x * w.y)));
}

// Power-of-two lengths (8 points per thread).
template <typename T, int N, int DIR, bool ZERO_HI, typename TW>
__device__ __forceinline__ void fft_line_p2(cT<T> (&v)[8], cT<T>* __restrict__ lds, const TW& tw, int t)
{
    using S = FftShape<N>;
    constexpr int TPL = S::TPL;
    int c = 0;
    int L = 1;
#pragma unroll
    for (int s = 0; s < S::S8; ++s) {
        // radix-8 butterfly b = t: inputs at t + i * TPL = v[i]
        if (s > 0) {
            const int j = t % L;
            cT<T> w[7];
            tw_stage8<T, N>(tw, c, s, L, j, w);
#pragma unroll
            for (int i = 1; i < 8; ++i) v[i] = twmul<T, DIR>(v[i], w[i - 1]);
            c += 7;
        }
        if (ZERO_HI && s == 0) {
            // inputs 4..7 are zero: X_k = E_k + w^k O_k with E = DFT4(a0, a2, 0, 0),
            // O = DFT4(a1, a3, 0, 0)
            cT<T> a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
            cT<T> e0 = cadd<T>(a0, a2), e2 = csub<T>(a0, a2);
            cT<T> e1 = cadd<T>(a0, mul_i<T, DIR>(a2)), e3 = csub<T>(a0, mul_i<T, DIR>(a2));
            cT<T> o0 = cadd<T>(a1, a3), o2 = csub<T>(a1, a3);
            cT<T> o1 = cadd<T>(a1, mul_i<T, DIR>(a3)), o3 = csub<T>(a1, mul_i<T, DIR>(a3));
            o1 = mul_w8<T, DIR>(o1);
            o2 = mul_i<T, DIR>(o2);
            o3 = mul_w83<T, DIR>(o3);
            v[0] = cadd<T>(e0, o0); v[4] = csub<T>(e0, o0);
            v[1] = cadd<T>(e1, o1); v[5] = csub<T>(e1, o1);
            v[2] = cadd<T>(e2, o2); v[6] = csub<T>(e2, o2);
            v[3] = cadd<T>(e3, o3); v[7] = csub<T>(e3, o3);
        } else {
            dft8<T, DIR>(v);
        }
        const bool last = (s == S::S8 - 1) && (S::RL == 1);
        if (!last) {
            constexpr bool WAVE_LOCAL = TPL <= 64;
            const int j = t % L;
            const int base = (t / L) * L * 8 + j;
            if (!WAVE_LOCAL || s == 0) lds_barrier();
            else wave_lds_sync();
#pragma unroll
            for (int i = 0; i < 8; ++i) lds[lpad(base + i * L)] = v[i];
            if (WAVE_LOCAL) wave_lds_sync();
            else lds_barrier();
#pragma unroll
            for (int m = 0; m < 8; ++m) v[m] = lds[lpad(t + m * TPL)];
        }
        L *= 8;
    }
    if constexpr (S::RL == 4) {
        // two radix-4 butterflies per thread: b = t + u TPL, inputs at
        // b + i N/4 = t + (u + 2 i) TPL -> slots u + 2 i
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int j = (t + u * TPL) % L;
#pragma unroll
            for (int i = 1; i < 4; ++i) v[u + 2 * i] = twmul<T, DIR>(v[u + 2 * i], tw_get<T, N>(tw, c++, S::S8, L, i, j));
            dft4<T, DIR>(v[u], v[u + 2], v[u + 4], v[u + 6]);
        }
    } else if constexpr (S::RL == 2) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = (t + u * TPL) % L;
            v[u + 4] = twmul<T, DIR>(v[u + 4], tw_get<T, N>(tw, c++, S::S8, L, 1, j));
            dft2<T, DIR>(v[u], v[u + 4]);
        }
    }
}

// Lengths 2^a 3^b (12 points per thread): the stages of mr_radix.  Stage 0
// is radix 12 (pruned for ZERO_HI); the others take their twiddles first.
template <typename T, int N, int DIR, bool ZERO_HI, typename TW>
__device__ __forceinline__ void fft_line_mr(cT<T> (&v)[12], cT<T>* __restrict__ lds, const TW& tw, int t)
{
    using S = FftShape<N>;
    constexpr int TPL = S::TPL, NS = mr_nstages(N);
    static_assert(mr_radix(N, 0) == 12, "the first stage is radix 12");
    static_for<0, NS>([&](auto sI) {
        constexpr int s = decltype(sI)::value;
        constexpr int R = mr_radix(N, s), L = mr_span(N, s), NB = 12 / R, C0 = mr_twc(N, s);
        // butterfly u of this thread: b = t + u TPL, inputs at b + i N / R,
        // i.e. slots u + i NB
        if constexpr (s > 0) {
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int j = (t + u * TPL) % L;
#pragma unroll
                for (int i = 1; i < R; ++i)
                    v[u + i * NB] = twmul<T, DIR>(v[u + i * NB], tw_get_mr<T, N, s>(tw, C0 + u * (R - 1) + i - 1, L, i, j));
            }
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            if constexpr (R == 12) dft12<T, DIR, ZERO_HI && s == 0, NB>(v, u);
            else if constexpr (R == 6) dft6<T, DIR, NB>(v, u);
            else if constexpr (R == 4) dft4<T, DIR>(v[u], v[u + NB], v[u + 2 * NB], v[u + 3 * NB]);
            else if constexpr (R == 3) dft3<T, DIR>(v[u], v[u + NB], v[u + 2 * NB]);
            else dft2<T, DIR>(v[u], v[u + NB]);
        }
        if constexpr (s + 1 < NS) {
            if (!S::WAVE_LOCAL || s == 0) lds_barrier();
            else wave_lds_sync();
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int b = t + u * TPL, j = b % L;
                const int base = (b / L) * L * R + j;
#pragma unroll
                for (int i = 0; i < R; ++i) lds[lpad(base + i * L)] = v[u + i * NB];
            }
            if (S::WAVE_LOCAL) wave_lds_sync();
            else lds_barrier();
#pragma unroll
            for (int m = 0; m < 12; ++m) v[m] = lds[lpad(t + m * TPL)];
        }
    });
}

// In-place transform of one line.  v[m] holds position t + m * TPL on entry
// and on exit.  lds points at this line's padded buffer of
// lds_line_elems(N) elements.  Every thread of the block calls it (all lines
// of the block run the same stages; a line is TPL consecutive threads).  The
// first exchange begins with a block barrier, so the buffer may overlap LDS
// that other wavefronts used before the call; the remaining exchanges of a
// line that lies within one wavefront (TPL divides 64) synchronise only
// that wavefront.  ZERO_HI: positions >= N / 2 are known to be zero on entry
// (pruned first stage).
template <typename T, int N, int DIR, bool ZERO_HI = false, typename TW = LineTwiddles<T, N>>
__device__ __forceinline__ void fft_line(cT<T> (&v)[FftShape<N>::P], cT<T>* __restrict__ lds, const TW& tw, int t)
{
    if constexpr (FftShape<N>::POW2) fft_line_p2<T, N, DIR, ZERO_HI, TW>(v, lds, tw, t);
    else fft_line_mr<T, N, DIR, ZERO_HI, TW>(v, lds, tw, t);
}

}  // namespace bttbk
