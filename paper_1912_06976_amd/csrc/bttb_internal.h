// bttb_internal.h -- declarations shared by the host library and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bttbk {

enum { KIND_GRAVITY = 0, KIND_MAGNETIC = 1, KIND_PROBE = 99 };
enum { ACC_PLAIN = 0, ACC_TWOSUM = 1, ACC_WIDE = 2 };

// weights G_1..G_5 of the magnetic corner terms
struct MagWeights { double g[5]; };

constexpr int MAX_GEN_BATCH = 8;   // layers per generator launch

struct GenParams {
    int kind;
    int sx, sy, nx, ny, pxl, pyl;
    int Nx, Ny;
    double dx, dy, h, scale;
    double z[MAX_GEN_BATCH + 1];   // depth edges z_{r0} .. z_{r0 + nl} of the batch
    MagWeights w;
};

template <typename T> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };
template <typename T> using cT = typename cplx<T>::type;

hipError_t launch_twiddles(double2* t64, float2* t32, int n, hipStream_t s);
hipError_t launch_generate(const GenParams& P, int r0, int nl, double* out, hipStream_t s);
template <typename TI, typename T>
hipError_t launch_rows_r2c(int N, const TI* in, int64_t in_bs, int64_t in_ld, int nvx, int nrows,
                           int nbatch, cT<T>* out, int64_t out_bs, int64_t out_ld, const cT<T>* tw,
                           hipStream_t s);
template <typename T>
hipError_t launch_rows_c2r(int N, const cT<T>* in, int64_t in_bs, int64_t in_ld, int nrows,
                           int nbatch, T* out, int64_t out_bs, int64_t out_ld, int nvx_out,
                           const cT<T>* tw, hipStream_t s);
template <typename T>
hipError_t launch_cols_spec(int N, const double2* in, int ncols, int nl, cT<T>* spec, int r0,
                            double scale, const double2* tw, hipStream_t s);
template <typename T, int ACC>
hipError_t launch_cols_fwd(int N, const cT<T>* X, int64_t ldx, int ny, int nz, int ncols,
                           const cT<T>* spec, cT<T>* Y, int64_t ldy, int sy, int nrhs,
                           const cT<T>* tw, hipStream_t s);
template <typename T>
hipError_t launch_cols_tr(int N, const cT<T>* R, int64_t ldr, int sy, int r0, int nl, int ncols,
                          const cT<T>* spec, cT<T>* Z, int64_t ldz, int ny, int nrhs,
                          const cT<T>* tw, hipStream_t s);

}  // namespace bttbk
