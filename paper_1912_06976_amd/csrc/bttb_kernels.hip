// bttb_kernels.hip -- gfx950 kernels of the fast BTTB products.
//
//   k_twiddles       FP64 twiddle tables exp(-2 pi i k / N), rounded to the
//                    working precision
//   k_generate       FP64 circulant generator T_r of each depth layer from
//                    the closed-form prism integrals (Sec. 3, eq. Tcircpadded /
//                    eq. Tcircpaddedgeneral; Sec. 4.1 / 4.2 entries)
//
// and the dispatch on the transform length of the row transforms and the
// spectra's column transforms (rows_impl.h, instantiated per group of lengths
// in bttb_rows_*.hip):
//   k_rows_r2c       real rows -> half spectra along x, pairs of rows packed
//                    into one complex transform, written in 8-row panels
//                    (bttb_internal.h) through an LDS tile
//   k_cols_spec      FP64 column transforms of the generator -> stored spectra
//                    (scaled by 1 / (Nx Ny), rounded to the working precision)
//   k_rows_c2r       half spectra (panels) -> real rows along x, two rows per
//                    complex transform, extraction of the leading columns
//
// The row kernels are in rows_impl.h, the column kernels of the products in
// cols_impl.h.  All kernels take caller-owned device buffers; none allocates.
#include "rows_cfg.h"

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
    // power-of-two n and rounded once otherwise
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
// launchers (dispatch on the transform lengths)
// ---------------------------------------------------------------------------

// Seeded values uniform in [-0.5, 0.5): an integer hash of the index (the
// autotuner's synthetic inputs, so that timings see data of ordinary bit
// activity).  Grid-stride loop: every index below n, any grid.
template <typename T>
__global__ void k_fill_uniform(T* __restrict__ p, int64_t n, uint32_t seed)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)i * 0x9E3779B1u ^ seed ^ (uint32_t)(i >> 32);
        h ^= h >> 16;
        h *= 0x85EBCA6Bu;
        h ^= h >> 13;
        h *= 0xC2B2AE35u;
        h ^= h >> 16;
        p[i] = (T)((double)h * (1.0 / 4294967296.0) - 0.5);
    }
}

hipError_t launch_fill_uniform(void* p, int64_t n, bool fp64, uint32_t seed, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    if (fp64) hipLaunchKernelGGL(k_fill_uniform<double>, dim3(blocks), dim3(256), 0, s, (double*)p, n, seed);
    else hipLaunchKernelGGL(k_fill_uniform<float>, dim3(blocks), dim3(256), 0, s, (float*)p, n, seed);
    return hipGetLastError();
}

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
    case 4096: L_RT(4096) case 96: L_RT(96) case 144: L_RT(144) case 192: L_RT(192) case 288: L_RT(288)
    case 384: L_RT(384) case 576: L_RT(576) case 768: L_RT(768) case 1152: L_RT(1152) case 1536: L_RT(1536)
    case 2304: L_RT(2304) case 3072: L_RT(3072) default: return 1;
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
    case 4096: L_CB(4096) case 96: L_CB(96) case 144: L_CB(144) case 192: L_CB(192) case 288: L_CB(288)
    case 384: L_CB(384) case 576: L_CB(576) case 768: L_CB(768) case 1152: L_CB(1152) case 1536: L_CB(1536)
    case 2304: L_CB(2304) case 3072: L_CB(3072) default: return 1;
    }
#undef L_CB
}
template int col_block_lines<float>(int, int);
template int col_block_lines<double>(int, int);

int fin_block_lines(int N)
{
#define L_FB(NN) return FinCfg<NN>::CPW;
    switch (N) {
    case 8: L_FB(8) case 16: L_FB(16) case 32: L_FB(32) case 64: L_FB(64) case 128: L_FB(128)
    case 256: L_FB(256) case 512: L_FB(512) case 1024: L_FB(1024) case 2048: L_FB(2048)
    case 4096: L_FB(4096) case 96: L_FB(96) case 144: L_FB(144) case 192: L_FB(192) case 288: L_FB(288)
    case 384: L_FB(384) case 576: L_FB(576) case 768: L_FB(768) case 1152: L_FB(1152) case 1536: L_FB(1536)
    case 2304: L_FB(2304) case 3072: L_FB(3072) default: return 1;
    }
#undef L_FB
}

// defined in rows_impl.h, instantiated per length in bttb_rows_*.hip
template <typename TI, typename T, int NN>
hipError_t rows_r2c_n(int tile, const RowJobs& jobs, const cT<T>* tw, hipStream_t s);
template <typename T, int NN>
hipError_t rows_c2r_n(int tile, const RowJobs& jobs, const cT<T>* tw, hipStream_t s);
template <typename T, int NN>
hipError_t cols_spec_n(const double2* in, int ncols, int nl, void* spec, int r0, double scale, const double2* tw,
                       int form, int64_t ldr, hipStream_t s);

template <typename TI, typename T>
hipError_t launch_rows_r2c(int N, int tile, const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    if (jobs.total <= 0) return hipSuccess;
#define L_R2C(NN) return rows_r2c_n<TI, T, NN>(tile, jobs, tw, s)
    BTTB_LEN_SWITCH(N, L_R2C)
#undef L_R2C
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_rows_c2r(int N, int tile, const RowJobs& jobs, const cT<T>* tw, hipStream_t s)
{
    if (jobs.total <= 0) return hipSuccess;
#define L_C2R(NN) return rows_c2r_n<T, NN>(tile, jobs, tw, s)
    BTTB_LEN_SWITCH(N, L_C2R)
#undef L_C2R
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_cols_spec(int N, const double2* in, int ncols, int nl, void* spec, int r0,
                            double scale, const double2* tw, int form, int64_t ldr, hipStream_t s)
{
#define L_SPEC(NN) return cols_spec_n<T, NN>(in, ncols, nl, spec, r0, scale, tw, form, ldr, s)
    BTTB_LEN_SWITCH(N, L_SPEC)
#undef L_SPEC
    return hipErrorInvalidValue;
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
