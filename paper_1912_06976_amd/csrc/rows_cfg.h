// rows_cfg.h -- block shapes and LDS layouts of the row transforms (shared
// by the kernels in rows_impl.h and the host-side dispatch in
// bttb_kernels.hip, which must not see the kernel templates: including them
// there would instantiate every row kernel a second time).
#pragma once
#include "kern_common.h"

namespace bttbk {

// Row length of an LDS staging tile of k rows whose accesses by a
// wavefront touch k rows at a few consecutive columns: the smallest
// length >= n congruent to 32 / k modulo 32, so that those elements sit in
// distinct 8-byte bank pairs (for many rows or short ones: an odd length).
constexpr int spread_len(int n, int k)
{
    if (k >= 32 || n < 32) return n % 2 ? n : n + 1;
    const int r = 32 / k;
    return n + ((r - n) % 32 + 32) % 32;
}
// The same for a tile that a wavefront writes with 8-byte LDS stores as k
// rows at a few consecutive columns: such stores are conflict-free when each
// group of sixteen lanes covers sixteen distinct 8-byte slots modulo 16
// (measured: k = 8 rows at a stride of 2 modulo 16 is conflict-free, at 4
// modulo 32 half the stores conflict), so the length is congruent to 16 / k
// modulo 16 (odd for k >= 16).
constexpr int spread_len_st(int n, int k)
{
    if (k >= 16 || n < 16) return n % 2 ? n : n + 1;
    const int r = 16 / k;
    return n + ((r - n) % 16 + 16) % 16;
}
// P0: pairs of rows per block for long rows (a tuning choice, 2 or 4)
template <typename T, int N, int P0 = 4> struct RowCfg {
    static constexpr int TPL = FftShape<N>::TPL;
    static constexpr int P = FftShape<N>::P;     // points per thread
    static constexpr int LPB = lines_per_block(TPL);
    static constexpr int PAIRS = sizeof(T) == 4 ? (N <= 2048 ? (LPB > P0 ? LPB : P0) : 2)
                                                : (N <= 1024 ? (LPB > P0 ? LPB : P0) : (N <= 2048 ? 2 : 1));
    static constexpr int RT = 2 * PAIRS;            // rows per block
    static constexpr int THREADS = PAIRS * TPL;
    static constexpr int HALF = N / 2;              // packed half-spectrum columns
    static constexpr int XCH = PAIRS * lds_line_elems(N);
    // c2r: the tile of packed half spectra staged [row][kx], row length CR:
    // the tile's stores (RT rows of a few kx per wavefront) and the line
    // reads (consecutive kx of one row) fall on distinct banks
    static constexpr int CR = sizeof(T) == 4 ? spread_len_st(HALF, RT) : spread_len(HALF, RT);
    static constexpr int CSTAGE = RT * CR;
    static constexpr int LDS = CSTAGE > XCH ? CSTAGE : XCH;
    static constexpr int TWO = LDS;                 // offset of the LDS twiddle table
    // r2c (FP32): the complex transforms Z of the PAIRS row pairs staged
    // [pair][k], row length ZR (the writes of a line are consecutive, the
    // split's reads take PAIRS pairs of a few k)
    static constexpr int ZR = spread_len(N, PAIRS);
    static constexpr int ZSTAGE = PAIRS * ZR;
    // r2c (FP64): the half spectra of the RT rows staged [kx][row] (split
    // through the line buffers first, which measured faster there)
    static constexpr int SROW = RT + 1;
    static constexpr int STAGE = HALF * SROW;
    static constexpr int LDS_R2C = sizeof(T) == 4 ? (ZSTAGE > XCH ? ZSTAGE : XCH) : (STAGE > XCH ? STAGE : XCH);
};

}  // namespace bttbk
