// kern_common.h -- device helpers and launch utilities shared by the kernel
// translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "fft_core.h"
#include "bttb_internal.h"

namespace bttbk {

// hardware block b -> logical block such that the blocks that the hardware
// places on one XCD (b mod 8) get consecutive logical indices
__device__ __forceinline__ int xcd_order(int b, int G)
{
    const int xcd = b & 7, k = b >> 3;
    const int per = G >> 3, rem = G & 7;
    return xcd < rem ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

// index of the job whose work range [begin, next begin) contains w
template <typename JT> __device__ __forceinline__ int find_job(const JT& js, int w)
{
    int k = 0;
    for (int i = 1; i < js.njobs; ++i)
        if (w >= js.j[i].begin) k = i;
    return k;
}

// minimum waves per SIMD requested for the column kernels (bounds the VGPRs
// the compiler may use: 512 / waves)
#ifndef BTTB_COL_WAVES
#define BTTB_COL_WAVES 2
#endif
// CM: multiplier of the columns per block (a tuning choice, 1 or 2)
// Lines per block of 256 threads, or of 192 where a line's thread count
// divides 192 but not 256 (12-point lines of 12, 24, 48, 96 or 192 threads),
// so that a block is whole wavefronts.
constexpr int lines_per_block(int tpl)
{
    return tpl >= 256 ? 1 : (256 % tpl == 0 ? 256 / tpl : (192 % tpl == 0 ? 192 / tpl : 256 / tpl));
}
template <int N, int CM = 1> struct ColCfg {
    static constexpr int TPL = FftShape<N>::TPL;
    static constexpr int CPW = lines_per_block(TPL) * CM;   // columns per block
    static constexpr int THREADS = CPW * TPL;
};

// Lines per block of the forward's finishing kernel (which adds the depth
// ranges' partial sums): about one wavefront per block, since the kernel is
// bound by the latency of those loads and wants many small blocks.
#ifndef BTTB_FIN_WAVE
#define BTTB_FIN_WAVE 1
#endif
template <int N> struct FinCfg {
    static constexpr int TPL = FftShape<N>::TPL;
    static constexpr int CPW = BTTB_FIN_WAVE ? (TPL >= 64 ? 1 : 64 / TPL) : lines_per_block(TPL);
    static constexpr int THREADS = CPW * TPL;
};

// a column tile of 2 is used only where its LDS (line buffers and, for
// 12-point lines, the twiddle table) fits in 160 KB
template <typename T, int NN> constexpr bool col_tile2_fits()
{
    return ((ColCfg<NN, 2>::CPW + 1) * lds_line_elems(NN) + (FftShape<NN>::POW2 ? 0 : TableTwiddles<T, NN>::size())) *
               (int)sizeof(cT<T>) <= 160 * 1024;
}

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
    case 96: MACRO(96); break;    \
    case 144: MACRO(144); break;  \
    case 192: MACRO(192); break;  \
    case 288: MACRO(288); break;  \
    case 384: MACRO(384); break;  \
    case 576: MACRO(576); break;  \
    case 768: MACRO(768); break;  \
    case 1152: MACRO(1152); break;\
    case 1536: MACRO(1536); break;\
    case 2304: MACRO(2304); break;\
    case 3072: MACRO(3072); break;\
    default: return hipErrorInvalidValue; }

// Stores through a raw buffer resource over [base, base + bytes).  The
// hardware drops a buffer store whose byte offset lies at or past the
// resource's size, so a lane that must not store is given an offset with
// bit 31 set (every size stays below 2^31) and the store needs no branch.
// With no stores skipped by branches the compiler knows how many memory
// operations were issued after a prefetch, and waits for the prefetch alone
// instead of draining the stores with it.
constexpr uint32_t BUF_SKIP = 0x80000000u;
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(void* base, uint32_t bytes)
{
    // descriptor word 3 for raw (unformatted) access on gfx9-family targets
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, 0x00020000);
}
template <typename V> __device__ __forceinline__ void buf_store(const V& v, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    if constexpr (sizeof(V) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, 0);
    else if constexpr (sizeof(V) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, (int)off, 0, 0);
    else {
        static_assert(sizeof(V) == 16, "4, 8 or 16 bytes");
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), r, (int)off, 0, 0);
    }
}
constexpr int64_t BUF_MAX_BYTES = int64_t(1) << 31;

// Wait until every vector memory operation this wavefront has issued so far
// is complete (s_waitcnt vmcnt(0); the LDS and export counters are left
// alone).  Placed after a prefetch has had time to arrive and before a
// batch of stores, it keeps the later wait for the prefetched registers
// from also waiting for those stores.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// grid of a persistent launch over `total` work units (at most the blocks
// resident at once, and at most the test hook's cap when one is set)
static inline int persistent_grid(int total, int resident)
{
    const int cap = g_persistent_grid_cap.load(std::memory_order_relaxed);
    const int g = std::min(total, resident);
    return cap > 0 && cap < g ? cap : g;
}

// blocks of `kernel` that are resident on the whole current device at once
// (occupancy per CU times the number of CUs); at least 1
static inline int resident_blocks(const void* kernel, int threads)
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

}  // namespace bttbk
