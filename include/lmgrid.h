/*
 * lmgrid.h -- C ABI of the least-misfit gridding / degridding library (gfx950).
 *
 * Method: Ye, Gull, Tan & Nikolic, "Optimal gridding and degridding in radio
 * interferometry imaging", MNRAS 2019. Equation numbers refer to the paper's
 * main text.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every function returns an lmg_status; nothing prints, throws or exits.
 * - Pointers documented "device" must point to device memory of the current
 *   HIP device; "host" pointers to host memory. The library never allocates
 *   device memory: every device buffer, including workspaces, is owned by the
 *   caller (for example a torch tensor) and must outlive the work enqueued on
 *   it.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream). Calls
 *   that take a stream only enqueue work and return; argument errors are
 *   detected on the host before anything is enqueued.
 * - uv coordinates are in grid cells (Sec. 2.1: u' = u L), an (nvis, 2)
 *   float64 array with u in column 0 and v in column 1.
 * - Grids are N x N, complex, stored centred: element [m + N/2][n + N/2]
 *   holds G_{m,n} for m, n in [-N/2, N/2); rows follow v, columns follow u.
 *   Taps that fall outside the grid wrap modulo N.
 * - Images hold the pixels p, q in [-x0 N, x0 N) (x_p = p/N, y_q = q/N) as a
 *   (2 x0 N) x (2 x0 N) complex array, element [q + x0 N][p + x0 N].
 * - Complex data are interleaved (re, im): complex64 for LMG_F32 and
 *   LMG_F32_KAHAN, complex128 for LMG_F64. Weights are float32 in all modes.
 */
#ifndef LMGRID_H
#define LMGRID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LMG_OK = 0,
    LMG_EINVAL = -1,      /* invalid argument (checked on the host, nothing enqueued) */
    LMG_EWORKSPACE = -2,  /* workspace NULL or smaller than the size query returned */
    LMG_EHIP = -3,        /* a HIP runtime call failed */
    LMG_EDATA = -4,       /* non-finite uv coordinates were met (reported by lmg_plan_check) */
    LMG_ENOTSUP = -5,     /* a valid request the library does not support (e.g. an image call on a multi-channel plan) */
    LMG_ENOCONV = -6      /* the table optimiser did not reach its tolerance */
} lmg_status;

typedef enum {
    LMG_F32 = 0,        /* complex64 data, plain FP32 accumulation */
    LMG_F32_KAHAN = 1,  /* complex64 data, compensated FP32 tile sums: each piece (at most 32 visibilities of
                           one cell) summed in FP32, the tile sums kept as (hi, lo) pairs by TwoSum */
    LMG_F64 = 2         /* complex128 data, FP64 throughout */
} lmg_precision;

/* ------------------------------------------------------------------ tables
 * A table bundles the least-misfit correcting function h sampled at the
 * N_g + 1 = 33 points x_i = i x0 / 32 of [0, x0] (App. A), the tabulated
 * gridding function (App. E) and the interpolation degree (App. F).
 *
 * Offsets: a visibility at u spreads onto cells n_first .. n_first + W - 1
 * with n_first = ceil(u - W/2) (the set S_k, Eq. 6). Its offset is
 * delta = u - (n_first + ref), ref = (W-1)/2 for odd W and W/2 - 1 for even
 * W, so delta lies in (-1/2, 1/2] (odd W) or (0, 1] (even W); tap j sits at
 * distance t_j - delta with t_j = j - ref. The table holds, for each tap j,
 * nodes C(t_j - delta_i) at delta_i = delta_lo + i / Ms, i = 0 .. Ms + degree
 * (row-major W x (Ms + 1 + degree)); the `degree` nodes past the top of the
 * interval continue the same smooth branch so that forward Newton stencils
 * stay on it. Ms = table_size / W (a "300-entry" W = 3 table has 100 samples
 * per cell, Abstract and Sec. 7).
 * Interpolation: degree 0 takes the nearest node (ties to the upper one);
 * degree d >= 1 the polynomial through nodes k .. k+d with
 * delta_k <= delta < delta_{k+1} (App. F).
 */
typedef struct lmg_table lmg_table;

/* Optimise h by Levenberg-Marquardt (App. A; initial guess h = 1 for W <= 4,
 * h_{W-1}^2 / h_{W-2} otherwise, so W > 4 optimises the chain W = 3 .. W),
 * solve the normal equations A C = B (Eqs. 17-19) by Cholesky at every node,
 * and build the table. From W = 12, where A is too ill-conditioned for
 * Cholesky (cond(A) 7e7 at W = 12), the kernel is App. B's least-squares
 * solution by Householder QR instead, in the optimiser as well as for the
 * nodes and the correction. W in [1, 16]; x0 in (0, 0.5]; table_size >= W;
 * degree in [0, 3]. Host only; takes milliseconds to a few seconds.
 * On success *out owns a new table (free with lmg_table_destroy). */
lmg_status lmg_table_create(int W, double x0, int table_size, int degree, lmg_table** out);

/* Same, with h given (33 host doubles, h_coarse[0] is the scale and need not
 * be 1): no optimisation, only the normal-equation solve (Eqs. 18-19). */
lmg_status lmg_table_create_from_h(int W, double x0, int table_size, int degree,
                                   const double* h_coarse, lmg_table** out);

/* Same, with both h (33 host doubles) and the node values given
 * (W * (Ms + 1 + degree) host doubles, layout above): the table is taken as
 * data. Used to run the kernels on a table produced elsewhere. */
lmg_status lmg_table_create_from_nodes(int W, double x0, int table_size, int degree,
                                       const double* h_coarse, const double* nodes, lmg_table** out);

/* Direct calculation (the paper's Sec. 6 alternative to a look-up table):
 * a table object with the same W, x0 and h as `from` whose gridding and
 * degridding kernels evaluate the exact kernel C(t_j - delta) = [A^{-1}
 * B(delta)]_j (Eq. 18) at each visibility's offset instead of interpolating
 * nodes, so no table error enters. The solve is expanded once on the host
 * over the 33 h samples (App. A), c_j(delta) = sum_i P_ji cos(i theta) + Q_ji
 * sin(i theta) with theta = 2 pi delta x0 / 32, and the device evaluates
 * that sum in FP64 in every precision mode (about 1,300 FP64 operations per
 * visibility: an arithmetic-bound variant). The grid and visibilities keep
 * the plan's precision. `from` is not modified and may be destroyed first.
 * Plans take the table like any other; the FFT, correction and crop are
 * unchanged. Errors: LMG_EINVAL (NULL argument, singular normal matrix);
 * LMG_ENOTSUP for W >= 12 (the expansion multiplies by A^{-1}, whose
 * conditioning then costs FP64 accuracy). */
lmg_status lmg_table_create_direct(const lmg_table* from, lmg_table** out);

/* Tables larger than the kernels' LDS budget (LMG_LDS_TABLE_BYTES of
 * coefficients: Ms above 145 at W = 7 for FP64 with cubic interpolation, 290
 * for FP32; App. F's rates of 1e3 .. 1e6 samples per cell) are read by the
 * kernels from device memory, through the caches, instead of being staged in
 * LDS. Their coefficients (4 per interval and tap: float for LMG_F32 and
 * LMG_F32_KAHAN, double for LMG_F64) live in a caller-owned device buffer
 * attached to the table. lmg_table_device_bytes gives the buffer's size for a
 * precision: 0 when the kernels stage the table in LDS (or for a direct
 * table), and then nothing needs attaching. lmg_table_attach_device enqueues
 * the copy of the coefficients into `device` on `stream` and records the
 * buffer for that precision; plans created afterwards read it, so it must
 * outlive them and not be written while they run. A plan whose table needs a
 * device copy that was not attached returns LMG_ENOTSUP, and so does a plan
 * for a table of 2^24 or more intervals (Ms >= 16,777,216). Errors:
 * LMG_EWORKSPACE (NULL or short buffer), LMG_EHIP. */
#define LMG_LDS_TABLE_BYTES 32768
lmg_status lmg_table_device_bytes(const lmg_table* t, lmg_precision prec, size_t* bytes);
lmg_status lmg_table_attach_device(lmg_table* t, lmg_precision prec, void* device, size_t bytes, void* stream);

/* *direct = 1 for a table made by lmg_table_create_direct, else 0. */
lmg_status lmg_table_is_direct(const lmg_table* t, int* direct);

/* Parameters of a table. Any output pointer may be NULL. */
lmg_status lmg_table_info(const lmg_table* t, int* W, double* x0, int* Ms, int* degree,
                          double* integrated_misfit);

/* Copy out h (33 host doubles) and the nodes (W * (Ms + 1 + degree) host
 * doubles). Either pointer may be NULL. */
lmg_status lmg_table_export(const lmg_table* t, double* h_coarse, double* nodes);

/* The exact least-misfit kernel (Eq. 18 solved at each offset): out[k*W + j]
 * = C(t_j - delta[k]) for n host offsets (any real delta; the formula
 * continues smoothly past the ends of the interval). */
lmg_status lmg_table_kernel(const lmg_table* t, int n, const double* delta, double* out);

/* Optimal correcting function (Eq. 12, equivalently Eq. 15) with the exact
 * kernel at x_p = p / N, p = -N/2 .. N/2 - 1, into N host doubles. The nu
 * integrals use 64-point Gauss-Legendre quadrature over one offset interval. */
lmg_status lmg_correction(const lmg_table* t, int N, double* h_pix);

/* Map error l(x) (Eq. 11) with the optimal correction at n host points x:
 * ell_exact with the exact kernel, ell_table with the tabulated and
 * interpolated kernel (App. F). Either output may be NULL. */
lmg_status lmg_map_error(const lmg_table* t, int n, const double* x, double* ell_exact, double* ell_table);

void lmg_table_destroy(lmg_table* t);

/* ------------------------------------------------------------------- plans
 * A plan holds, in a caller-owned device workspace, everything the kernels
 * derive from the uv coordinates alone: the first tap cell and fractional
 * offsets of every visibility (computed in FP64) and a counting sort of the
 * visibilities by uv tile with per-tile work lists. Build one per uv set and
 * reuse it for every grid / degrid / image / prediction call on that set
 * (the paper notes that this per-visibility work need be done only once,
 * Sec. 6.2). The plan keeps pointers into `workspace` and a reference to
 * `table`: both must outlive it.
 *
 * N: power of two in [max(64, 2W), 8192]; x0 * N * 2 an integer (taken
 * from the table). nvis >= 0. uv: device (nvis, 2) float64.
 * lmg_plan_create only enqueues work on `stream`: the plan's counts (work
 * items, occupied band, dropped visibilities) come back asynchronously and
 * the host waits for them only where it needs them (lmg_plan_check,
 * lmg_plan_info, and the transforms of the image calls, after the gridding
 * kernels are queued). Planned calls on any stream wait on the device for
 * the plan's kernels. Visibilities with a NaN or infinite coordinate are
 * dropped from every later call and reported as LMG_EDATA by lmg_plan_check.
 * A plan may be used by several host threads; its calls must not overlap
 * with lmg_plan_destroy.
 */
typedef struct lmg_plan lmg_plan;

lmg_status lmg_plan_workspace_size(int N, int W, int64_t nvis, lmg_precision prec, size_t* bytes);
lmg_status lmg_plan_create(const lmg_table* table, int N, lmg_precision prec, int64_t nvis,
                           const double* uv, void* workspace, size_t ws_bytes, void* stream,
                           lmg_plan** out);
/* LMG_OK, or LMG_EDATA if non-finite coordinates were dropped. Host query
 * (waits for the plan's kernels). */
lmg_status lmg_plan_check(const lmg_plan* p);
/* Tile edge, number of work items and occupied tiles (any pointer may be
 * NULL). Waits for the plan's kernels. */
lmg_status lmg_plan_info(const lmg_plan* p, int* tile, int* n_items, int* n_busy_tiles, int64_t* n_valid);
void lmg_plan_destroy(lmg_plan* p);

/* Scratch a planned call needs beyond its inputs and outputs (device bytes),
 * sized for the most work items the plan can have (known without waiting). */
lmg_status lmg_plan_scratch_size(const lmg_plan* p, int op, size_t* bytes);
#define LMG_OP_GRID 0
#define LMG_OP_DEGRID 1
#define LMG_OP_DIRTY 2
#define LMG_OP_PREDICT 3

/* --------------------------------------------------------- planned calls */

/* Gridding (Eq. 5 in 2D): G[m][n] = sum_k w_k V_k C(m - v_k) C(n - u_k) over
 * the plan's visibilities. accumulate = 0 overwrites the N x N device grid
 * (every cell is written, zero where no footprint reaches); accumulate = 1
 * adds G to what the grid holds (grid += G), reading and writing only the uv
 * tiles that receive contributions, so that chunks of a visibility set (or
 * channels) can be summed into one grid: Eq. 5 is a sum over k. Any other
 * value: LMG_EINVAL. vis: device complex (nvis), w: device float32 (nvis) or
 * NULL for unit weights. The sum is computed in the plan's precision (FP32,
 * compensated FP32 tile sums with (hi, lo) pairs, or FP64) in an order fixed by the
 * plan, so repeated calls on the same plan and data give identical bits, and
 * so do plans built again from the same coordinates. */
lmg_status lmg_grid_planned(const lmg_plan* p, const void* vis, const float* w, void* grid, int accumulate,
                            void* scratch, size_t scratch_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * lmg_grid_planned with its scratch taken from a fixed device array of
 * LMG_STATIC_SCRATCH_BYTES (64 MiB) that the library holds on each device it
 * runs on until the process ends, instead of a caller workspace. Same
 * arguments and results as lmg_grid_planned (accumulate 0 or 1). It calls no
 * hipMalloc, hipFree or allocating library routine; the first call on a
 * device looks up the array's address there. LMG_ENOTSUP, with nothing
 * enqueued, when the plan's gridding scratch (lmg_plan_scratch_size with
 * LMG_OP_GRID) exceeds the array. Every call on a device shares that
 * device's array, which keeps the previous call's contents (the call
 * initialises what it reads): calls that overlap in time on one device
 * (different streams or host threads) race and give wrong grids, so
 * serialise them, for example on one stream. */
#define LMG_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
lmg_status lmg_grid_planned_noalloc(const lmg_plan* p, const void* vis, const float* w, void* grid, int accumulate,
                                    void* stream);

/* Degridding, the transpose of gridding (Sec. 1, Sec. 5):
 * vis_out[k] = sum_{m,n} C(m - v_k) C(n - u_k) grid[m][n]. Weights do not
 * apply. vis_out: device complex (nvis), overwritten. */
lmg_status lmg_degrid_planned(const lmg_plan* p, const void* grid, void* vis_out,
                              void* scratch, size_t scratch_bytes, void* stream);

/* ------------------------------------------------------ calls in plan order
 * A plan grids visibilities in its own order ("plan order": by uv tile, then
 * footprint cell), and the planned calls above reorder the caller's arrays on
 * the way in (lmg_grid_planned) and out (lmg_degrid_planned). Iterative
 * imaging (major cycles: predict, subtract, grid the residuals; gradient
 * steps) can keep its visibility data in plan order instead, reorder once, and
 * skip both passes in every call. A plan-ordered array holds
 * lmg_plan_order_length elements (nvis plus padding that the kernels may read
 * and never write), of the plan's complex type; visibilities dropped for
 * non-finite coordinates have no element. */
lmg_status lmg_plan_order_length(const lmg_plan* p, int64_t* n);
/* vis_plan = w V in plan order (w: device float32 (nvis) or NULL for unit
 * weights; vis: device complex (nvis), caller order). */
lmg_status lmg_to_plan_order(const lmg_plan* p, const void* vis, const float* w, void* vis_plan, void* stream);
/* vis = the caller-order copy of vis_plan (zero for dropped visibilities). */
lmg_status lmg_from_plan_order(const lmg_plan* p, const void* vis_plan, void* vis, void* stream);
/* lmg_grid_planned and lmg_degrid_planned on plan-ordered data (weights
 * already applied by lmg_to_plan_order); same grids and visibilities, bit for
 * bit, as the caller-order calls give after reordering. Scratch: the sizes
 * lmg_plan_scratch_size returns for LMG_OP_GRID and LMG_OP_DEGRID. */
lmg_status lmg_grid_planned_ordered(const lmg_plan* p, const void* vis_plan, void* grid, int accumulate,
                                    void* scratch, size_t scratch_bytes, void* stream);
lmg_status lmg_degrid_planned_ordered(const lmg_plan* p, const void* grid, void* vis_plan_out, void* scratch,
                                      size_t scratch_bytes, void* stream);

/* Dirty image (Eq. 4 in 2D): grid, inverse 2D FFT (exponent +i2pi), multiply
 * by h(x_p) h(y_q) and keep |x|, |y| <= x0. image: device complex
 * (2 x0 N)^2, overwritten. No normalisation by sum(w). The transforms are
 * pruned to the occupied band of the grid, which the plan's counts give: the
 * first image or prediction call on a plan waits on the host for the plan's
 * kernels (after its gridding kernels are queued); later calls do not. */
lmg_status lmg_make_dirty_image_planned(const lmg_plan* p, const void* vis, const float* w, void* image,
                                        void* scratch, size_t scratch_bytes, void* stream);

/* Prediction (Eq. 2 through the FFT, Sec. 5): multiply the image by
 * h(x_p) h(y_q), zero-pad to N x N, forward 2D FFT (exponent -i2pi) and
 * degrid. image: device complex (2 x0 N)^2; vis_out: device complex (nvis). */
lmg_status lmg_predict_visibilities_planned(const lmg_plan* p, const void* image, void* vis_out,
                                            void* scratch, size_t scratch_bytes, void* stream);

/* ------------------------------------------------ one-shot (unplanned) calls
 * Build a plan inside `workspace`, run the call, and release the plan. The
 * workspace size comes from lmg_workspace_size for the same (N, W, nvis,
 * prec, op). They return after the plan's kernels have finished (the plan is
 * released), so they may block the host. lmg_grid ACCUMULATES: grid += G
 * (the caller zeroes the grid first), so that a visibility set too large for
 * one call (nvis <= INT32_MAX per plan) is streamed into one grid in chunks.
 * The other three overwrite their outputs. */
lmg_status lmg_workspace_size(int N, int W, double x0, int64_t nvis, lmg_precision prec, int op, size_t* bytes);
lmg_status lmg_grid(const lmg_table* t, int N, lmg_precision prec, int64_t nvis, const double* uv,
                    const void* vis, const float* w, void* grid, void* workspace, size_t ws_bytes, void* stream);
lmg_status lmg_degrid(const lmg_table* t, int N, lmg_precision prec, int64_t nvis, const double* uv,
                      const void* grid, void* vis_out, void* workspace, size_t ws_bytes, void* stream);
lmg_status lmg_make_dirty_image(const lmg_table* t, int N, lmg_precision prec, int64_t nvis, const double* uv,
                                const void* vis, const float* w, void* image, void* workspace, size_t ws_bytes,
                                void* stream);
lmg_status lmg_predict_visibilities(const lmg_table* t, int N, lmg_precision prec, int64_t nvis, const double* uv,
                                    const void* image, void* vis_out, void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------- batched channels
 * Many independent problems (e.g. frequency channels) with uneven numbers of
 * visibilities, each gridded onto its own N x N grid, in one plan and one
 * launch per kernel (not part of the paper's method, which images one
 * channel; the per-channel arithmetic is that of lmg_grid / lmg_degrid).
 * Channel c owns the visibilities [offsets[c], offsets[c+1]) of uv / vis and
 * grid c of `grids` (nchan x N x N, device, channel-major). offsets: host,
 * nchan + 1 non-decreasing int64 with offsets[0] = 0. nchan in [1, 65536].
 * The plan is an lmg_plan: lmg_grid_planned and lmg_degrid_planned accept it
 * and then read / write nchan grids; lmg_make_dirty_image_planned and
 * lmg_predict_visibilities_planned return LMG_ENOTSUP for nchan > 1.
 * tile: edge of the uv tiles in cells, 0 for the library default, else a
 * power of two in [max(8, W), min(128, N)] with N / tile <= 128 (LMG_EINVAL
 * otherwise: a footprint of W cells must not reach two tiles away); the best
 * value depends on the density of the data, which is what an autotuner
 * measures. Workspace sizes are upper bounds for any tile.
 */
lmg_status lmg_batch_workspace_size(int N, int W, int nchan, int64_t nvis, lmg_precision prec, size_t* bytes);
lmg_status lmg_batch_plan_create(const lmg_table* table, int N, lmg_precision prec, int nchan, const int64_t* offsets,
                                 const double* uv, int tile, void* workspace, size_t ws_bytes, void* stream,
                                 lmg_plan** out);
/* Channels, tile edge and waves per gridding workgroup of a plan (any pointer may be NULL). */
lmg_status lmg_batch_info(const lmg_plan* p, int* nchan, int* tile, int* waves);

/* One-shot batched gridding (accumulates into all nchan grids: grids += G_c) and degridding; op is
 * LMG_OP_GRID or LMG_OP_DEGRID. They return after the plan's kernels have
 * finished (the plan is released), so they may block the host. */
lmg_status lmg_workspace_size_batched(int N, int W, int nchan, int64_t nvis, lmg_precision prec, int op,
                                      size_t* bytes);
lmg_status lmg_grid_batched(const lmg_table* t, int N, lmg_precision prec, int nchan, const int64_t* offsets,
                            const double* uv, const void* vis, const float* w, void* grids, void* ws,
                            size_t ws_bytes, void* stream);
lmg_status lmg_degrid_batched(const lmg_table* t, int N, lmg_precision prec, int nchan, const int64_t* offsets,
                              const double* uv, const void* grids, void* vis_out, void* ws, size_t ws_bytes,
                              void* stream);

/* ------------------------------------------------------- 2D FFT building block
 * Centred 2D transform F[q][p] = sum_{m,n} G[m][n] exp(sign i 2 pi (n p + m q) / N)
 * of an N x N device array in place of `data` (all indices centred in
 * [-N/2, N/2)); sign = +1 or -1. scratch: N*N complex device elements. */
lmg_status lmg_fft2_centred(int N, lmg_precision prec, int sign, void* data, void* scratch, void* stream);

/* ------------------------------------------------------------------ tracing
 * When enabled, every kernel the library launches is bracketed by a pair of
 * HIP events recorded on the launch stream. lmg_trace_report synchronizes
 * those events and writes one line per kernel name, "name count total_ms",
 * into `buf` (NUL-terminated, truncated to `len`), then clears the record.
 * Also enabled by the environment variable LMG_TRACE=1. Not thread-safe
 * with respect to concurrent launches from several host threads. */
lmg_status lmg_trace_enable(int on);
lmg_status lmg_trace_report(char* buf, size_t len);
/* Record only the kernel of this trace name ("grid_items", "plan_scatter",
 * ...); NULL or "" records every kernel again. The name is copied. */
lmg_status lmg_trace_only(const char* name);

/* Wait for all work enqueued on `stream` (a hipStream_t as void*, NULL = the
 * null stream), then report device-side data errors: LMG_EDATA if any plan
 * built on the current device since the last call met non-finite uv
 * coordinates (those visibilities were dropped), else LMG_OK; LMG_EHIP if a
 * HIP call failed. The device-wide flag is cleared by the call that reports
 * it. Host-blocking. */
lmg_status lmg_sync_status(void* stream);

const char* lmg_status_string(lmg_status s);

/* Text of the last HIP failure seen by this thread (the call and the HIP
 * error string), or "" if none. Owned by the library. */
const char* lmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LMGRID_H */
