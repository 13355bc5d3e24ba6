// fft_core.h -- register/LDS Stockham FFT building blocks for gfx950.
//
// One transform ("line") of power-of-two length N is spread over TPL = N / 8
// threads; thread t of the line holds the 8 elements at positions
// t + m * TPL (m = 0..7) in registers, both before and after the transform,
// in natural order.  Stages are radix-8 (decimation in time, Stockham
// auto-sort) followed by at most one radix-2 or radix-4 stage; between stages
// the elements are exchanged through a padded LDS buffer.  A stage of radix R
// with current sub-transform length L maps butterfly b = t + u * TPL
// (u < 8 / R) with inputs at b + i N / R to outputs at
// (b / L) L R + (b mod L) + i L after multiplying input i by w^(i (b mod L))
// with w = exp(-+ 2 pi i / (L R)).  For the last stage L R = N, so its
// outputs land on the same register slots as the inputs: no final exchange.
//
// Twiddles are read from a table tw[k] = exp(-2 pi i k / N), k < N, computed
// in FP64 and rounded to the working precision.  A per-thread copy of the
// twiddles each stage needs is held in registers (struct LineTwiddles) so a
// kernel that transforms many lines of the same length loads them once.
#pragma once
#include <hip/hip_runtime.h>

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
__device__ __forceinline__ int lpad(int x) { return x ^ ((x >> 3) & 31); }
constexpr int lds_line_elems(int n) { return n + (n >= 64 ? 8 : 4); }

template <int N> struct FftShape {
    static constexpr int LOG = ilog2(N);
    static constexpr int S8 = LOG / 3;             // radix-8 stages
    static constexpr int RL = 1 << (LOG % 3);      // last small radix (1: none)
    static constexpr int TPL = N / 8;              // threads per line
    static constexpr int NTW = 7 * (S8 > 0 ? S8 - 1 : 0) + (RL > 1 ? (8 / RL) * (RL - 1) : 0);
    static_assert(N >= 8 && (N & (N - 1)) == 0, "power-of-two length >= 8");
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

// Per-thread twiddles of one line of length N (forward sign; the inverse
// uses the conjugates).  tw points to the table of length N.
template <typename T, int N> struct LineTwiddles {
    using S = FftShape<N>;
    cT<T> w[S::NTW > 0 ? S::NTW : 1];
    __device__ __forceinline__ void load(const cT<T>* __restrict__ tw, int t) {
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
    }
};

// Alternative twiddle source: a stage-major table (typically in LDS) that
// saves the registers of LineTwiddles.  For radix-8 stage s >= 1 (L = 8^s)
// it holds w^(i j N/(8L)) at [off_s + (i-1) L + j], j < L; for the final
// radix-RL stage (L = N/RL) w^(i j) at [off_f + (i-1) L + j].  A stage's
// reads by consecutive threads are consecutive (or broadcast) entries, so
// they do not conflict on the LDS banks.
template <typename T, int N> struct TableTwiddles {
    const cT<T>* p;
    // entries before stage s (1 <= s <= S8; s = S8 is the final small stage)
    static constexpr int off(int s) {
        int o = 0, L = 8;
        for (int k = 1; k < s; ++k) { o += 7 * L; L *= 8; }
        return o;
    }
    static constexpr int size() {
        using S = FftShape<N>;
        return off(S::S8) + (S::RL > 1 ? (S::RL - 1) * (N / S::RL) : 0);
    }
    // fill dst[0 .. size()) from the natural table tw (all threads of the block)
    static __device__ void build(cT<T>* dst, const cT<T>* __restrict__ tw, int tid, int nthreads) {
        using S = FftShape<N>;
        for (int e = tid; e < size(); e += nthreads) {
            int idx;
            if (e < off(S::S8)) {
                int s = 1, L = 8;
                while (e >= off(s + 1)) { ++s; L *= 8; }
                const int r = e - off(s), i = r / L + 1, j = r % L;
                idx = i * j * (N / (8 * L));
            } else {
                const int L = N / S::RL, r = e - off(S::S8), i = r / L + 1, j = r % L;
                idx = i * j;
            }
            dst[e] = tw[idx & (N - 1)];
        }
    }
};

template <typename T, int N>
__device__ __forceinline__ cT<T> tw_get(const LineTwiddles<T, N>& tw, int c, int, int, int, int) { return tw.w[c]; }
template <typename T, int N>
__device__ __forceinline__ cT<T> tw_get(const TableTwiddles<T, N>& tw, int, int s, int L, int i, int j) {
    return tw.p[TableTwiddles<T, N>::off(s) + (i - 1) * L + j];
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

template <typename T, int DIR> __device__ __forceinline__ cT<T> twmul(cT<T> a, cT<T> w) {
    return DIR < 0 ? cmul<T>(a, w) : cmulc<T>(a, w);
}

// In-place transform of one line.  v[m] holds position t + m * TPL on entry
// and on exit.  lds points at this line's padded buffer of
// lds_line_elems(N) elements.  Every thread of the block calls it (all lines
// of the block run the same stages; a line is TPL consecutive threads).  The
// first exchange begins with a block barrier, so the buffer may overlap LDS
// that other wavefronts used before the call; the remaining exchanges of a
// line that lies within one wavefront (TPL <= 64) synchronise only that
// wavefront.  ZERO_HI: positions >= N / 2 are known to be zero on entry
// (pruned first stage).
template <typename T, int N, int DIR, bool ZERO_HI = false, typename TW = LineTwiddles<T, N>>
__device__ __forceinline__ void fft_line(cT<T> (&v)[8], cT<T>* __restrict__ lds, const TW& tw, int t)
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
#pragma unroll
            for (int i = 1; i < 8; ++i) v[i] = twmul<T, DIR>(v[i], tw_get<T, N>(tw, c + i - 1, s, L, i, j));
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
            if (!WAVE_LOCAL || s == 0) __syncthreads();
            else wave_lds_sync();
#pragma unroll
            for (int i = 0; i < 8; ++i) lds[lpad(base + i * L)] = v[i];
            if (WAVE_LOCAL) wave_lds_sync();
            else __syncthreads();
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

}  // namespace bttbk
