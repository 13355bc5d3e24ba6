/*
 * bttb.h -- C ABI of the gfx950 fast BTTB product library (libbttb.so).
 *
 * Forward and transpose products with the 3-D gravity (g_z) and magnetic
 * total-field-anomaly sensitivity matrices of Hogue, Renaut & Vatankhah,
 * "A Tutorial and Open Source Software for the Efficient Evaluation of
 * Gravity and Magnetic Kernels" (arXiv 1912.06976):
 *
 *   d = G m = sum_r G^(r) m_r,     G^T r = [G^(1)^T r; ...; G^(nz)^T r]
 *   (Sec. 2, eq. Gslice; Sec. 5, the depth-layer split),
 *
 * where each depth-layer block G^(r) is block-Toeplitz with Toeplitz blocks
 * (symmetric for gravity without padding, non-symmetric for the magnetic
 * kernel; Sec. 2.2), embedded in a block-circulant matrix whose generator
 * T_r (Sec. 3, eq. Tcircpadded / eq. Tcircpaddedgeneral) is transformed once
 * with a 2-D FFT; the products are then pointwise multiplications in the
 * Fourier domain (Sec. 3, eq. GrviaT), accumulated over depth before one
 * inverse 2-D FFT for the forward product.
 *
 * Conventions (0-based; the paper's 1-based indices shifted by one):
 *   station (i, j), i < sx, j < sy, at ((i + 1/2) dx, (j + 1/2) dy, -h);
 *   prism (p, q, r), p < nx = sx + pxl + pxr, q < ny = sy + pyl + pyr,
 *   r < nz, spans [(p - pxl) dx, (p - pxl + 1) dx] x
 *   [(q - pyl) dy, (q - pyl + 1) dy] x [z_r, z_{r+1}], z pointing down
 *   (Sec. 2.1.2 and the coordinate table of the appendix);
 *   G[k][l] with k = j sx + i and l = r nx ny + q nx + p (Sec. 2, eq. htilde).
 *
 * Memory layouts (x fastest everywhere):
 *   model m, transpose output mt:   [nrhs][nz][ny][nx]
 *   data d, transpose input r:      [nrhs][sy][sx]
 *   all in the plan's precision (float for BTTB_FP32, double for BTTB_FP64).
 *
 * Ownership: the plan is a host object owned by the caller.  All device
 * memory (spectra, workspace, inputs, outputs) is allocated and owned by the
 * caller; the library never allocates device memory and never synchronises
 * the stream (except bttb_debug_generator, a test hook).  Device calls only
 * enqueue work on the given stream (a hipStream_t passed as void*, NULL =
 * the default stream) and return; asynchronous faults surface at the
 * caller's next synchronisation.  Invalid arguments are rejected before
 * anything is enqueued, with a status code and a thread-local message
 * (bttb_last_error).  No C++ exception crosses this interface.
 *
 * Thread safety: a plan is immutable after creation; concurrent calls on one
 * plan are safe if each uses its own workspace.
 */
#ifndef BTTB_H
#define BTTB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BTTB_OK = 0,
    BTTB_ERR_INVALID_VALUE = 1,      /* a descriptor field or argument is out of range  */
    BTTB_ERR_NULL_POINTER = 2,       /* a required pointer is NULL                      */
    BTTB_ERR_UNSUPPORTED = 3,        /* valid but not supported (e.g. FFT length > 4096) */
    BTTB_ERR_WORKSPACE_TOO_SMALL = 4,/* ws_bytes below what bttb_plan_query reports     */
    BTTB_ERR_HIP = 5,                /* a HIP launch or runtime call failed             */
    BTTB_ERR_INTERNAL = 6,
    BTTB_ERR_OUT_OF_MEMORY = 7       /* bttb_plan_memory_check: more than is available  */
} bttb_status;

typedef enum {
    BTTB_GRAVITY_GZ = 0,   /* vertical gravity, mGal per (g/cm^3) (Sec. 4.1)           */
    BTTB_MAGNETIC_TMI = 1, /* total-field anomaly of induced magnetisation, nT per SI
                              susceptibility (Sec. 4.2)                                */
    BTTB_USER_TABLE = 2,   /* any spatially invariant kernel: the caller supplies
                              the entries per layer and cell offset
                              (bttb_kernel_generate_table; Sec. 1 (vi))           */
    BTTB_HESSIAN = 3,      /* scale * sum_ab w_ab U_ab: any linear combination, with
                              the weights hessian[6], of the second derivatives
                              U_ab = d_a d_b (integral over the prism of 1/|P - r'|)
                              with respect to the station position P (x North,
                              y East, z down), evaluated on the device from the
                              closed forms of Sec. 4.2 (the user-chosen kernel of
                              Sec. 1 (vi)): gravity-gradient components
                              (scale 66.743 Eotvos per g/cm^3), the total-field
                              anomaly of a remanent or induced magnetisation
                              m (w = f m^T symmetrised; scale 100 nT per A/m, or
                              F / (4 pi) per SI susceptibility), field components   */
    BTTB_PROBE = 99        /* test hook: entry = dx + 4096 dy + 2^24 r for the cell
                              offsets dx = p - pxl - i, dy = q - pyl - j               */
} bttb_problem;

typedef enum { BTTB_FP32 = 0, BTTB_FP64 = 1 } bttb_precision;

/* Depth accumulation of the FP32 forward product (ignored for FP64):
 * BTTB_ACC_WIDE accumulates the per-layer products in FP64 (default),
 * BTTB_ACC_TWOSUM uses compensated FP32 (TwoSum) accumulation,
 * BTTB_ACC_PLAIN plain FP32 sums. */
typedef enum { BTTB_ACC_DEFAULT = 0, BTTB_ACC_PLAIN = 1, BTTB_ACC_TWOSUM = 2, BTTB_ACC_WIDE = 3 } bttb_accumulation;

/* Stored form of the layer spectra.
 * BTTB_SPECTRUM_COMPLEX: the transform of the circulant generator of
 *   Sec. 3 (eq. Tcircpadded), N_y x N_x / 2 complex values per layer.
 * BTTB_SPECTRUM_REAL_EVEN: for the symmetric gravity kernel (entries even in
 *   both cell offsets, Sec. 4.1: the symmetric BTTB case of sym_BTTBFFT), the
 *   generator placed centred on offset 0 is even, so its transform is real
 *   and even in both frequencies and a quarter of it, (N_x/2 + 1)(N_y/2 + 1)
 *   real values per layer, holds all of it; the paddings become a phase
 *   applied once per column.  Needs N_x >= 2 (s_x - 1 + max(pxl, pxr)) + 1
 *   and the same in y (always true for equal paddings on both sides).
 * BTTB_SPECTRUM_AUTO: REAL_EVEN where it applies (the gravity kernel, a
 *   BTTB_HESSIAN kernel with zero off-diagonal weights), else COMPLEX.  A BTTB_USER_TABLE plan uses REAL_EVEN only when asked for (the
 *   caller declares the table even).
 * The results of both forms agree to rounding. */
typedef enum { BTTB_SPECTRUM_AUTO = 0, BTTB_SPECTRUM_COMPLEX = 1, BTTB_SPECTRUM_REAL_EVEN = 2 } bttb_spectrum_form;

/*
 * Problem description: the parameter set of the paper's Table 2
 * (prob_params, gsx/gsy/gsz, z_blocks, I, D, F).
 */
typedef struct {
    int32_t problem;           /* bttb_problem                                         */
    int32_t precision;         /* bttb_precision of spectra, inputs and outputs        */
    int32_t nx, ny, nz;        /* prism grid; nx, ny must equal sx + pxl + pxr, sy + pyl + pyr
                                  (0: derived); nz >= 1                                */
    int32_t sx, sy;            /* station grid, >= 1                                   */
    int32_t pxl, pxr, pyl, pyr;/* padding prisms left/right in x and y, >= 0           */
    double dx, dy, dz;         /* cell sizes [m], > 0; dz unused if z_edges != NULL    */
    const double* z_edges;     /* optional host array of nz + 1 strictly increasing
                                  depths [m], z_edges[0] >= 0; copied at creation     */
    double station_height;     /* h >= 0: stations at z = -h (z down)                  */
    double inclination_deg;    /* magnetic field inclination I in [-90, 90]            */
    double declination_deg;    /* declination D from +x (North) towards +y (East)      */
    double field_nT;           /* field intensity F [nT], > 0 for BTTB_MAGNETIC_TMI    */
    double scale;              /* 0: default (6.6743e-3 mGal per (g/cm^3 m) for gravity,
                                  F / (4 pi) for the magnetic kernel, 1 for the probe,
                                  the user table and BTTB_HESSIAN)                     */
    int32_t nx_fft, ny_fft;    /* 0: the smallest supported length >= max(8, s + n - 1)
                                  (the real even form, that is the gravity kernel
                                  with spectrum_form AUTO or spectrum_form
                                  REAL_EVEN: the smallest that also admits it);
                                  else a supported length >= max(8, s + n - 1).
                                  Supported: powers of two in [8, 4096] and
                                  2^a 3^b with b = 1 or 2 in [96, 3072]
                                  (96, 144, 192, 288, 384, 576, 768, 1152, 1536,
                                  2304, 3072)                                          */
    int32_t accumulation;      /* bttb_accumulation                                    */
    int32_t layer_chunk;       /* tuning: layers per pass of the transpose product (0: all
                                  layers); smaller chunks keep the per-layer intermediate
                                  in the device's last-level cache and shrink the
                                  workspace.  Results do not depend on it.              */
    int32_t row_tile;          /* tuning: 0 (default) or 1 / 2 / 4 pairs of rows per
                                  block of the row transforms staged through LDS, or 8:
                                  tiles of 8 rows held per thread                     */
    int32_t col_tile;          /* tuning: 0 (default) or 1 / 2 times the default number of
                                  columns per block of the column transforms          */
    int32_t spectrum_form;     /* bttb_spectrum_form; REAL_EVEN where it does not apply
                                  is an UNSUPPORTED error                             */
    double hessian[6];         /* BTTB_HESSIAN: weights (w_xx, w_yy, w_zz, w_xy, w_xz,
                                  w_yz) of U_xx, U_yy, U_zz, U_xy, U_xz, U_yz (each
                                  off-diagonal component counted once), finite.  The
                                  entry is evaluated with U_zz = -U_xx - U_yy
                                  (Laplace's equation outside the prism): for a
                                  station on a prism's top face (h = 0) this is the
                                  limit from the air side.  With w_xy = w_xz = w_yz
                                  = 0 the kernel is even in both cell offsets and
                                  BTTB_SPECTRUM_AUTO uses the real even form.         */
} bttb_problem_desc;

typedef struct bttb_plan_s* bttb_plan_t;

/* Validate the descriptor and build a host-only plan (no device work).
 * Errors: NULL_POINTER, INVALID_VALUE, UNSUPPORTED. */
bttb_status bttb_plan_create(const bttb_problem_desc* desc, bttb_plan_t* out);

/* Release a plan (NULL is accepted). */
bttb_status bttb_plan_destroy(bttb_plan_t plan);

/* Sizes: spectra_bytes for the opaque spectra buffer; workspace_bytes that
 * suffices for bttb_kernel_generate and for bttb_forward / bttb_transpose
 * with up to nrhs right-hand sides; the chosen FFT lengths.  Any output
 * pointer may be NULL.  Errors: NULL_POINTER (plan), INVALID_VALUE (nrhs < 1). */
bttb_status bttb_plan_query(bttb_plan_t plan, int32_t nrhs, size_t* spectra_bytes,
                            size_t* workspace_bytes, int32_t* nx_fft, int32_t* ny_fft);

/* Memory guard, to call before allocating a plan's buffers (the paper's
 * software tests each problem size's memory use at set-up so that a problem
 * too large for the machine is not attempted; Sec. 6, software package).
 * need = spectra_bytes + workspace_bytes for nrhs + one product's input and
 * output for nrhs right-hand sides (m and d), each rounded up to 256 bytes.
 * available: a budget in bytes chosen by the caller, or 0 for the current
 * device's free memory (hipMemGetInfo).  *need_bytes and *available_bytes
 * (the figure compared against) are written when not NULL, also on
 * OUT_OF_MEMORY.  Allocates nothing.  Errors: NULL_POINTER (plan),
 * INVALID_VALUE (nrhs < 1), OUT_OF_MEMORY (need > available), HIP (the
 * device query failed). */
bttb_status bttb_plan_memory_check(bttb_plan_t plan, int32_t nrhs, size_t available, size_t* need_bytes,
                                   size_t* available_bytes);

/* The spectrum form the plan uses (BTTB_SPECTRUM_COMPLEX or
 * BTTB_SPECTRUM_REAL_EVEN).  Errors: NULL_POINTER. */
bttb_status bttb_plan_spectrum_form(bttb_plan_t plan, int32_t* form);

/* Fill the caller's spectra buffer (device, spectra_bytes, 256-byte aligned):
 * the generator T_r of every layer is evaluated in FP64 from the closed-form
 * prism integrals (Sec. 4.1 Algorithm gravity, Sec. 4.2 Algorithm magnetic),
 * placed in the circulant (Sec. 3, eq. Tcircpadded / Tcircpaddedgeneral),
 * transformed with an FP64 2-D FFT, scaled by 1 / (Nx Ny) and rounded to the
 * plan precision (the transform of the paper's sym_BTTBFFT / BTTBFFT), in
 * the plan's spectrum form (BTTB_SPECTRUM_REAL_EVEN: the centred generator,
 * the real parts of a quarter of its transform).  The transpose uses the
 * conjugate of the same spectra (for a real generator the transform of the
 * flipped generator of eq. Ttran is the conjugate).
 * workspace: device, >= workspace_bytes of bttb_plan_query(plan, 1, ...). */
bttb_status bttb_kernel_generate(bttb_plan_t plan, void* spectra, void* workspace,
                                 size_t ws_bytes, void* stream);

/* Fill the spectra of a BTTB_USER_TABLE plan from the caller's entries (the
 * paper's software takes the kernel's matrix entries from the user, Sec. 1
 * (vi); the entries depend on the cell offsets only, Sec. 2.1).
 * table: device, FP64, [nz][wy][wx] with wx = sx + nx - 1, wy = sy + ny - 1:
 * table[r][dy + sy - 1 + pyl][dx + sx - 1 + pxl] is the entry of G for a
 * station and a prism of layer r offset by dx = p - pxl - i in
 * [-(sx - 1 + pxl), nx - 1 - pxl] and dy = q - pyl - j likewise; the plan's
 * scale (default 1) multiplies it.  With spectrum_form
 * BTTB_SPECTRUM_REAL_EVEN the caller declares the kernel even,
 * h_r(dx, dy) = h_r(|dx|, |dy|) (the centred generator then reads, for an
 * offset outside the table on one side, its mirror).  Other arguments as for
 * bttb_kernel_generate.  Errors: NULL_POINTER, INVALID_VALUE (not a
 * BTTB_USER_TABLE plan; bttb_kernel_generate rejects those), WORKSPACE_TOO_SMALL,
 * HIP. */
bttb_status bttb_kernel_generate_table(bttb_plan_t plan, const double* table, void* spectra, void* workspace,
                                       size_t ws_bytes, void* stream);

/* d = G m for nrhs right-hand sides (the paper's mult_BTTB with t = 1).
 * m: device [nrhs][nz][ny][nx]; d: device [nrhs][sy][sx]; workspace >=
 * workspace_bytes of bttb_plan_query(plan, nrhs, ...).  m, d and the
 * spectra must not overlap the workspace, nor d the spectra (checked:
 * INVALID_VALUE).  Errors: NULL_POINTER, INVALID_VALUE (nrhs < 1, a
 * misaligned buffer or an overlap), WORKSPACE_TOO_SMALL, HIP.
 * Results are deterministic for a given plan and nrhs.  When a call has few
 * column blocks, the depth sum is split into layer ranges whose FP64 partial
 * sums are added in order.  The split depends on nrhs, and for a batch on
 * the other problems of its branch.  A different nrhs or a batch may
 * therefore round the FP32 result differently, within its accuracy. */
bttb_status bttb_forward(bttb_plan_t plan, const void* spectra, const void* m, void* d,
                         int32_t nrhs, void* workspace, size_t ws_bytes, void* stream);

/* mt = G^T r for nrhs right-hand sides (mult_BTTB with t = 2).
 * r: device [nrhs][sy][sx]; mt: device [nrhs][nz][ny][nx].  Workspace,
 * overlap rules and errors as for bttb_forward. */
bttb_status bttb_transpose(bttb_plan_t plan, const void* spectra, const void* r, void* mt,
                           int32_t nrhs, void* workspace, size_t ws_bytes, void* stream);

/* Bytes of the library's own device scratch array used by
 * bttb_forward_noalloc (64 MiB; one copy per GPU the library runs on, held
 * until the process ends). */
#define BTTB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* d = G m exactly as bttb_forward, without a workspace argument: for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The workspace bttb_forward
 * would take lives in a file-scope device array of BTTB_NOALLOC_SCRATCH_BYTES
 * inside the library; the call allocates nothing (no hipMalloc, no hipFree,
 * no allocating library routine).  Results equal bttb_forward's bit for bit
 * for the same plan, spectra, m and nrhs.
 * The stream (NULL = default stream) must belong to the current device; the
 * first call on a device looks up that device's copy of the array.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (other streams, other threads, other plans) race and must be
 * ordered by the caller.  The array keeps the last call's contents; nothing
 * in it needs to start at zero.
 * Errors: as bttb_forward, plus UNSUPPORTED when the workspace of the plan
 * for nrhs right-hand sides (bttb_plan_query) exceeds
 * BTTB_NOALLOC_SCRATCH_BYTES, INVALID_VALUE when the stream belongs to
 * another device, HIP when the array's address cannot be obtained. */
bttb_status bttb_forward_noalloc(bttb_plan_t plan, const void* spectra, const void* m, void* d,
                                 int32_t nrhs, void* stream);

/* ------------------------------------------------------------------------
 * Inversion driver: the regularised least-squares problem
 *     min_m ||G m - d||^2 + lambda^2 ||m||^2
 * that the transpose product exists for (Sec. 1: conjugate gradients with
 * FFT-based products; Sec. 7: use in the inverse problem), solved by CGLS,
 * conjugate gradients on the normal equations (G^T G + lambda^2 I) m = G^T d
 * without forming G^T G:
 *   r = d - G m,  s = G^T r - lambda^2 m,  p = s,  gamma = ||s||^2;  per step
 *   q = G p,  alpha = gamma / (||q||^2 + lambda^2 ||p||^2),
 *   m += alpha p,  r -= alpha q,  s = G^T r - lambda^2 m,
 *   beta = ||s||^2 / gamma,  p = s + beta p.
 * Once ||s_k|| <= tau ||s_0|| (tau = 1e-6 for FP32 plans, 1e-12 for FP64)
 * the remaining steps leave m unchanged (alpha = 0; the history repeats):
 * the products are each other's adjoint only to their rounding, and
 * conjugate gradients iterated far below that level can drift away from
 * the solution.
 * Every step runs on the device (the product kernels plus FP64-accumulating
 * vector kernels); scalars stay on the device, so the call does not
 * synchronise and can be captured in a graph.
 * ------------------------------------------------------------------------ */

/* Workspace bytes of bttb_cgls for this plan (one right-hand side).
 * Errors: NULL_POINTER. */
bttb_status bttb_cgls_query(bttb_plan_t plan, size_t* workspace_bytes);

/* Run `iterations` CGLS steps from the initial model in m.
 * d: device [sy][sx] (plan precision, not modified); m: device [nz][ny][nx],
 * the initial guess on entry and the result on exit; lambda >= 0;
 * history: optional device array of 3 (iterations + 1) doubles receiving,
 * after the start and after each step k, (||r_k||^2, ||m_k||^2, ||s_k||^2)
 * (||r||^2 + lambda^2 ||m||^2 does not increase); workspace: device,
 * >= bttb_cgls_query bytes, 16-byte aligned; spectra from
 * bttb_kernel_generate.  Errors: NULL_POINTER, INVALID_VALUE,
 * WORKSPACE_TOO_SMALL, HIP. */
bttb_status bttb_cgls(bttb_plan_t plan, const void* spectra, const void* d, void* m, double lambda,
                      int32_t iterations, double* history, void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batches: many problems (uneven sizes, gravity and magnetic mixed, one
 * precision) run together.  The problems are split into up to four
 * independent branches balanced by work (problems with the same transform
 * lengths share a branch); in a branch every stage of the products is
 * launched once per transform length with a work table covering all its
 * problems of that length.  The whole run is captured into one HIP graph
 * whose branches execute concurrently, so a run is a single graph launch.
 * The graph is rebuilt only when the pointers or right-hand-side counts of a
 * run differ from the previous run's.
 * ------------------------------------------------------------------------ */
typedef struct bttb_batch_s* bttb_batch_t;

/* Per-problem inputs of a batch run (all device pointers, caller-owned).
 * A NULL forward (m, d) or transpose (r, mt) pair skips that product for this
 * problem; layouts as for bttb_forward / bttb_transpose. */
typedef struct {
    const void* spectra;       /* generated spectra of the plan                 */
    const void* m;             /* [nrhs][nz][ny][nx]                            */
    void* d;                   /* [nrhs][sy][sx]                                */
    const void* r;             /* [nrhs][sy][sx]                                */
    void* mt;                  /* [nrhs][nz][ny][nx]                            */
    int32_t nrhs;              /* 1 .. max_nrhs                                 */
} bttb_batch_io;

/* Group nplans plans (not owned; they must outlive the batch) for runs with
 * at most max_nrhs right-hand sides per problem.  All plans must have the
 * same precision.  Creates five non-blocking streams (default priority) and
 * five events used for graph capture.  Errors: NULL_POINTER, INVALID_VALUE,
 * HIP. */
bttb_status bttb_batch_create(const bttb_plan_t* plans, int32_t nplans, int32_t max_nrhs,
                              bttb_batch_t* out);

/* Workspace bytes a run needs (device, 256-byte aligned). */
bttb_status bttb_batch_query(bttb_batch_t batch, size_t* workspace_bytes);

/* Enqueue the products of every problem on `stream` as one graph launch.
 * io: host array of nplans entries.  Errors: NULL_POINTER, INVALID_VALUE,
 * WORKSPACE_TOO_SMALL, HIP.  Calls on one batch must not overlap.  A call
 * with other pointers or counts than the previous one captures a new graph
 * and first waits for the previous launch to finish. */
bttb_status bttb_batch_run(bttb_batch_t batch, const bttb_batch_io* io, void* workspace,
                           size_t ws_bytes, void* stream);

/* Release the graph, the capture streams and events and the batch (NULL
 * accepted).  Waits for the batch's last launch to finish first, so a batch
 * may be destroyed right after bttb_batch_run returns. */
bttb_status bttb_batch_destroy(bttb_batch_t batch);

/* ------------------------------------------------------------------------
 * Autotuner (the analogue of FFTW's planner "wisdom" the paper's MATLAB
 * runs preload, Sec. 5): for one descriptor and right-hand-side count, time
 * the products on the device for every candidate configuration -- the FFT
 * lengths along each axis whose nx_fft / ny_fft is 0 (the plan's default,
 * the smallest supported length and the smallest power of two holding the
 * circulant; the spectra are generated for each), and for each length pair
 * row_tile in {2, 4, 8} (wavefronts per block of the row transforms),
 * col_tile in {1, 2} and layer_chunk in {0, 8, 16, 32} below nz -- and
 * return the descriptor with the fastest one filled in (nx_fft, ny_fft,
 * row_tile, col_tile, layer_chunk).  Each candidate runs one forward and one
 * transpose product on seeded uniform inputs, once untimed and then 5 timed
 * times, and counts its fastest time; the plan's default configuration is
 * timed first (after at least 200 ms of untimed products on it, while the
 * device's clocks come up) and another candidate replaces the best so far
 * only when it is at least 2 % faster.  A winner of the default lengths
 * other than the default configuration is then timed 5 more times
 * alternately with the default and kept only if it is again at least 2 %
 * faster.  The lengths change the products only by rounding.
 * Results are cached in a text file (path: environment variable
 * BTTB_TUNE_CACHE, default $HOME/.cache/bttb_autotune.txt), keyed by the
 * shape, precision, accumulation, nrhs and device; a cached key is returned
 * without timing.  Synchronises the stream.  scratch: device memory of at
 * least bttb_autotune_query bytes (spectra, workspace and test vectors).
 * ------------------------------------------------------------------------ */
bttb_status bttb_autotune_query(const bttb_problem_desc* desc, int32_t nrhs, size_t* scratch_bytes);
bttb_status bttb_autotune(const bttb_problem_desc* desc, int32_t nrhs, void* scratch, size_t scratch_bytes,
                          void* stream, bttb_problem_desc* tuned, float* best_ms);

/* Profiling hooks: the same work as bttb_forward / bttb_transpose, with HIP
 * events recorded on the stream around every launch of each of the three
 * stages (row transform; column transform with the depth multiply-accumulate
 * and, for a split depth sum, its finishing kernel; output row transform);
 * waits for the events and stores each stage's summed duration in
 * milliseconds in kernel_ms[0..2] (with layer chunks the transpose runs the
 * column and output row stages once per chunk).  Synchronises the stream. */
bttb_status bttb_forward_profiled(bttb_plan_t plan, const void* spectra, const void* m, void* d,
                                  int32_t nrhs, void* workspace, size_t ws_bytes, void* stream,
                                  float* kernel_ms);
bttb_status bttb_transpose_profiled(bttb_plan_t plan, const void* spectra, const void* r, void* mt,
                                    int32_t nrhs, void* workspace, size_t ws_bytes, void* stream,
                                    float* kernel_ms);

/* Test hook: evaluate the FP64 circulant generator T_r of one layer into the
 * workspace and copy it to host_out ([ny_fft][nx_fft] doubles, x fastest).
 * Synchronises the stream.  Errors: NULL_POINTER, INVALID_VALUE (layer out
 * of range, or a BTTB_USER_TABLE plan), WORKSPACE_TOO_SMALL, HIP. */
bttb_status bttb_debug_generator(bttb_plan_t plan, int32_t layer, double* host_out,
                                 void* workspace, size_t ws_bytes, void* stream);

/* Test hook: cap the grid of the persistent kernels (the row transforms and
 * the transpose multiply-accumulate, which size their grids to the blocks
 * resident at once and walk the work units) at max_blocks blocks, for every
 * launch this process makes afterwards (graphs already captured keep their
 * grids); 0 restores the default.  Each block then walks more units; the
 * results are the same bit for bit.  Not for use while other threads launch.
 * Errors: INVALID_VALUE (max_blocks < 0). */
bttb_status bttb_debug_cap_grid(int32_t max_blocks);

/* Static description of a status code. */
const char* bttb_status_string(bttb_status s);

/* Message of the last failing call on this thread ("" if none). */
const char* bttb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BTTB_H */
