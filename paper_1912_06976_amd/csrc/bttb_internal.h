// bttb_internal.h -- declarations shared by the host library and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

namespace bttbk {

enum { KIND_GRAVITY = 0, KIND_MAGNETIC = 1, KIND_TABLE = 2, KIND_PROBE = 99 };
enum { ACC_PLAIN = 0, ACC_TWOSUM = 1, ACC_WIDE = 2 };
// stored spectrum forms (see bttb_cols.hip)
enum { FORM_COMPLEX = 0, FORM_REAL_EVEN = 1 };

// weights G_1..G_5 of the magnetic corner terms
struct MagWeights { double g[5]; };

constexpr int MAX_GEN_BATCH = 8;   // layers per generator launch

// Test hook (bttb_debug_cap_grid): an upper bound on the grid of the
// persistent kernels, 0 for none.  A smaller grid makes every block walk more
// work units; the results do not depend on the grid.
inline std::atomic<int> g_persistent_grid_cap{0};

struct GenParams {
    int kind;
    int sx, sy, nx, ny, pxl, pyl;
    int Nx, Ny;
    double dx, dy, h, scale;
    double z[MAX_GEN_BATCH + 1];   // depth edges z_{r0} .. z_{r0 + nl} of the batch
    MagWeights w;
    // centred even placement (real even spectra): T[ay][ax] = h(|ax|, |ay|)
    // for |ax| <= bx, |ay| <= by
    int sym, bx, by;
    // KIND_TABLE: caller's entries [nz][wy][wx], offset (dx, dy) at
    // [dy + offy][dx + offx]
    const double* table;
    int wx, wy, offx, offy;
    // gravity / magnetic: the corner grid of the batch, cy x cx corner terms
    // per depth edge z_{r0} .. z_{r0 + nl}; corner (ex, ey) at
    // x = (oxmin + ex - 1/2) dx, y = (oymin + ey - 1/2) dy
    const double* corners;
    int oxmin, oymin, cx, cy;
};

// Half spectra along x (packed: N/2 columns) of a block of R rows are stored
// in panels of PANEL rows: element (kx, y) at
// ((y / PANEL) * ncols + kx) * PANEL + y % PANEL, and the block takes
// ncols * panel_rows(R) elements.  A row group of the row kernels then reads
// or writes contiguous memory, and a column is PANEL-row segments.
constexpr int PANEL = 8;
__host__ __device__ constexpr int64_t panel_rows(int64_t r) { return (r + PANEL - 1) / PANEL * PANEL; }
__host__ __device__ __forceinline__ int64_t pidx(int kx, int y, int ncols)
{
    return ((int64_t)(y / PANEL) * ncols + kx) * PANEL + (y % PANEL);
}

// Work tables.  A launch of a row or column kernel processes every job of
// its table (one job per problem instance / right-hand-side batch, all with
// the same transform length); the table is passed by value as a kernel
// argument, so no device memory holds it.
constexpr int MAX_JOBS = 32;

struct RowJob {
    const void* in;       // real rows (r2c) or packed half spectra in panels (c2r)
    void* out;            // packed half spectra in panels (r2c) or real rows (c2r)
    int64_t in_bs, in_ld; // batch stride and row stride of the input (elements;
                          // the row stride is unused for half spectra)
    int64_t out_bs, out_ld;
    int nv;               // r2c: valid input length of a row; c2r: output length
    int nrows;            // rows per batch
    int bpb;              // row groups per batch
    int begin;            // first global row-group index of this job
    int gq, gr;           // persistent kernels (set at launch): grid / bpb, grid % bpb
};
struct RowJobs {
    RowJob j[MAX_JOBS];
    int njobs, total;     // total = row groups of all jobs
};

struct ColJob {
    const void* a;        // input columns: X (forward) or R (transpose)
    const void* spec;     // spectra of the job's plan
    void* b;              // output columns: Y (forward) or Z (transpose)
    int64_t lda, ldb;     // padded rows (panel_rows) of a and b: a block of one
                          // layer / right-hand side is ncols * lda elements
    int na, nb;           // valid rows of a (ny or sy), rows written to b (sy or ny)
    int r0, nl;           // layers [r0, r0 + nl)
    int ncols, nrhs;
    int nbx;              // column blocks per right-hand-side block
    int begin;            // first global block index of this job
    int px, py;           // real even spectra: phase offsets (pxl, pyl)
    int64_t lds;          // real even spectra: line stride (elements)
    void* p;              // forward with ns > 1: FP64 partial depth sums,
                          // [nrhs][ns][ncols][N] complex
    int ns;               // forward: layer ranges (depth splits) per column block
};
struct ColJobs {
    ColJob j[MAX_JOBS];
    int njobs, total;     // total = blocks of all jobs
};

// device scalars of the CGLS iteration
struct CglsScalars { double gamma, alpha, beta, gamma0; };   // gamma0 = ||s_0||^2

template <typename T> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };
template <typename T> using cT = typename cplx<T>::type;

hipError_t launch_twiddles(double2* t64, float2* t32, int n, hipStream_t s);
hipError_t launch_fill_uniform(void* p, int64_t n, bool fp64, uint32_t seed, hipStream_t s);
// corner grid of the depth edges z_{r0} .. z_{r0 + nl} into P.corners
// (gravity / magnetic), then the generator of layers [r0, r0 + nl)
hipError_t launch_corners(const GenParams& P, int nl, double* corners, hipStream_t s);
hipError_t launch_generate(const GenParams& P, int r0, int nl, double* out, hipStream_t s);
// rows per row group (row tile 2 or 4 pairs) and columns per column block
// (column tile 1 or 2 times the default) of the kernels for length N
template <typename T> int row_group_rows(int N, int tile);
template <typename T> int col_block_lines(int N, int tile);
// columns per block of the forward's finishing kernel for length N
int fin_block_lines(int N);
template <typename TI, typename T>
hipError_t launch_rows_r2c(int N, int tile, const RowJobs& jobs, const cT<T>* tw, hipStream_t s);
template <typename T>
hipError_t launch_rows_c2r(int N, int tile, const RowJobs& jobs, const cT<T>* tw, hipStream_t s);
// spectra of nl generator layers (row-transformed, packed) into layers
// [r0, r0 + nl) of `spec` in the given form (ldr: line stride of the real
// even form)
template <typename T>
hipError_t launch_cols_spec(int N, const double2* in, int ncols, int nl, void* spec, int r0,
                            double scale, const double2* tw, int form, int64_t ldr, hipStream_t s);
template <typename T, int ACC>
hipError_t launch_cols_fwd(int N, int tile, int form, const ColJobs& jobs, const cT<T>* tw, hipStream_t s);
// sums the partial depth sums of jobs with ns > 1, then the forward's inverse
// y transform and store (one block per column block and right-hand side)
template <typename T>
hipError_t launch_cols_fwd_fin(int N, int tile, int form, const ColJobs& jobs, const cT<T>* tw, hipStream_t s);
template <typename T>
hipError_t launch_cols_tr(int N, int tile, int form, const ColJobs& jobs, const cT<T>* tw, hipStream_t s);

// CGLS vector kernels (nb blocks; each reduction writes nb FP64 partials)
template <typename T> hipError_t launch_cgls_dot(const T* a, const T* b, int64_t n, double* out, int nb, hipStream_t s);
template <typename T>
hipError_t launch_cgls_residual(const T* d, const T* q, T* r, int64_t n, double* out, int nb, hipStream_t s);
template <typename T>
hipError_t launch_cgls_grad(T* sv, T* m, const T* p, const CglsScalars* sc, int step, double lam2, int64_t n,
                            double* out_s, double* out_m, int nb, hipStream_t s);
template <typename T>
hipError_t launch_cgls_direction(const T* sv, T* p, int64_t n, const CglsScalars* sc, int first, double* out, int nb,
                                 hipStream_t s);
template <typename T>
hipError_t launch_cgls_step(T* r, const T* q, int64_t nd, const CglsScalars* sc, double* out, int nb, hipStream_t s);
hipError_t launch_cgls_alpha(const double* pq, const double* pp, int nb, double lam2, double tol2, CglsScalars* sc,
                             hipStream_t s);
hipError_t launch_cgls_beta(const double* ps, const double* pr, const double* pm, int nb, CglsScalars* sc,
                            double* hist, int k, int first, hipStream_t s);

}  // namespace bttbk
