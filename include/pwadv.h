/*
 * libpwadv -- Piacsek-Williams (PW) advection source terms on AMD MI355X (gfx950).
 *
 * The operation (paper, Sec. 2.2): from the three wind fields u, v, w on a
 * halo-padded 3-D grid, compute one advective "source term" per field and
 * interior cell -- su, sv, sw -- with a depth-one stencil that reaches the
 * neighbouring cells in all three dimensions.  Per field and cell the scheme
 * forms six face sums of advecting velocities, six products of a neighbouring
 * value with a face sum, and their signed reduction (Sec. 4, Fig. 2); the
 * three fields share that arithmetic and differ only in stencil locations.
 *
 * Reading of the scheme (the paper prints no equations): the energy-
 * conserving PW form on a staggered grid, u on east faces, v on north faces,
 * w on top faces, upstream face minus downstream face.  In padded coordinates
 * (k, j, i), x fastest, interior level index kk = k - halo:
 *
 *   su = tcx*( u[k,j,i-1]*(u[k,j,i]+u[k,j,i-1]) - u[k,j,i+1]*(u[k,j,i]+u[k,j,i+1]) )
 *      + tcy*( u[k,j-1,i]*(v[k,j-1,i]+v[k,j-1,i+1]) - u[k,j+1,i]*(v[k,j,i]+v[k,j,i+1]) )
 *      + tzc1[kk]*u[k-1,j,i]*(w[k-1,j,i]+w[k-1,j,i+1]) - tzc2[kk]*u[k+1,j,i]*(w[k,j,i]+w[k,j,i+1])
 *   sv = tcx*( v[k,j,i-1]*(u[k,j,i-1]+u[k,j+1,i-1]) - v[k,j,i+1]*(u[k,j,i]+u[k,j+1,i]) )
 *      + tcy*( v[k,j-1,i]*(v[k,j,i]+v[k,j-1,i]) - v[k,j+1,i]*(v[k,j,i]+v[k,j+1,i]) )
 *      + tzc1[kk]*v[k-1,j,i]*(w[k-1,j,i]+w[k-1,j+1,i]) - tzc2[kk]*v[k+1,j,i]*(w[k,j,i]+w[k,j+1,i])
 *   sw = tcx*( w[k,j,i-1]*(u[k,j,i-1]+u[k+1,j,i-1]) - w[k,j,i+1]*(u[k,j,i]+u[k+1,j,i]) )
 *      + tcy*( w[k,j-1,i]*(v[k,j-1,i]+v[k+1,j-1,i]) - w[k,j+1,i]*(v[k,j,i]+v[k+1,j,i]) )
 *      + tzd1[kk]*w[k-1,j,i]*(w[k,j,i]+w[k-1,j,i]) - tzd2[kk]*w[k+1,j,i]*(w[k,j,i]+w[k+1,j,i])
 *
 * Conventions shared by every call below
 * --------------------------------------
 * Memory:    every array argument is a caller-owned DEVICE buffer on the
 *            current HIP device.  The library never frees or keeps them.
 * Inputs:    u, v, w have the padded shape (nz+2h, ny+2h, nx+2h); element
 *            (k, j, i) lives at  base[k*in_sz + j*in_sy + i]  (x stride 1).
 * Outputs:   su, sv, sw are interior-shaped (nz, ny, nx); element (kk, jj, ii)
 *            at  base[kk*out_sz + jj*out_sy + ii].
 * Vertical:  tzc1, tzc2, tzd1, tzd2 are device arrays of nz entries indexed by
 *            the interior level.  Element type: float for PW_F32/PW_BF16/PW_F16,
 *            double for PW_F64.  tcx, tcy are passed as double and rounded
 *            (to nearest even) to float for the float-family dtypes.
 * Precision: PW_F32  -- float storage, float arithmetic, float outputs.
 *            PW_BF16 / PW_F16 -- 16-bit storage of u, v, w only; values are
 *            widened exactly to float in registers, float arithmetic and float
 *            outputs.  PW_F64 -- double throughout.
 * Streams:   work is enqueued on `hip_stream` (a hipStream_t; NULL = the
 *            default stream) and the call returns without synchronising.
 *            Faults inside a kernel surface at the caller's next
 *            synchronisation.
 * Errors:    every call returns a pw_status; nothing aborts or throws across
 *            the ABI.  On a non-OK status nothing was enqueued, and
 *            pw_last_error() holds a message (per thread).  Arguments are
 *            validated before any HIP call, so argument errors are reported
 *            the same way on a machine with no GPU; with valid arguments and no
 *            usable device the status is PW_ERR_NO_DEVICE.
 * Threads:   all calls are reentrant; distinct calls may run concurrently.
 */
#ifndef PWADV_H
#define PWADV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PW_OK = 0,
    PW_ERR_INVALID_ARG = 1,   /* null/misaligned pointer, bad size, stride or alias */
    PW_ERR_UNSUPPORTED = 2,   /* valid arguments, combination not implemented      */
    PW_ERR_NO_DEVICE = 3,     /* no usable HIP device                               */
    PW_ERR_HIP = 4,           /* a HIP runtime call failed (message in last_error)  */
    PW_ERR_ALLOC = 5          /* host or device allocation failed                   */
} pw_status;

typedef enum {
    PW_F32 = 0,
    PW_F64 = 1,
    PW_BF16 = 2,
    PW_F16 = 3
} pw_dtype;

/* Interior extent and halo width.  nx, ny, nz >= 1; halo >= 1 (the stencil
 * has depth one, Sec. 2.2; a wider halo is just padding).  nx*ny*nz < 2^40. */
typedef struct {
    int64_t nx, ny, nz;
    int32_t halo;
} pw_grid;

/* Element strides.  Input strides must be at least the dense padded ones
 * (in_sy >= nx+2h, in_sz >= in_sy*(ny+2h)), output strides at least the dense
 * interior ones (out_sy >= nx, out_sz >= out_sy*ny).  A NULL pw_layout* means
 * dense in both. */
typedef struct {
    int64_t in_sy, in_sz;
    int64_t out_sy, out_sz;
} pw_layout;

/* Coefficients: tcx, tcy scalars; tz* device pointers to nz elements. */
typedef struct {
    double tcx, tcy;
    const void *tzc1, *tzc2, *tzd1, *tzd2;
} pw_coeffs;

/* Forward operator (the equations above): writes su, sv, sw at every
 * interior cell.  Inputs of element type `in_dtype`; outputs float (double
 * for PW_F64).  Outputs must not overlap any input or coefficient array
 * (the kernels read the coefficients through the scalar cache).  Halo cells
 * of u, v, w are read, never written. */
pw_status pw_advect(const pw_grid *grid, const pw_layout *layout, pw_dtype in_dtype,
                    const void *u, const void *v, const void *w,
                    const pw_coeffs *coeffs,
                    void *su, void *sv, void *sw,
                    void *hip_stream);

/* Launch shape of the stencil kernels (a performance choice; results are
 * bit-identical across shapes).  A wavefront of 64 lanes owns a strip of
 * 64*cols_per_lane x rows_per_strip interior cells and marches through zlen
 * levels, with `prefetch` planes loaded ahead of the level it computes;
 * waves_per_group strips are stacked in y per workgroup.
 * Forward (pw_advect_ex):
 *   cols_per_lane 1 or 2: rows_per_strip in {1, 2, 4};
 *   cols_per_lane 4 (not PW_F64): rows_per_strip in {1, 2, 4};
 *   cols_per_lane 8 (16-bit storage): rows_per_strip in {1, 2};
 *   PW_F64: cols_per_lane in {1, 2}, rows_per_strip in {1, 2, 4};
 *   prefetch 1 or 2 (0 means 1).  A deeper prefetch keeps more bytes in
 *   flight per wavefront; it pays when few wavefronts run.
 * Adjoint (pw_advect_adjoint_ex): cols_per_lane 1 (strips of 62 padded
 *   columns), rows_per_strip in {1, 2, 4}, prefetch 0, 1 or 2.
 * Batched form: as the forward with cols_per_lane <= 4 (FP32), prefetch 0, 1 or 2;
 *   or cols_per_lane 0: per subdomain 2 where that leaves no more lanes idle
 *   than 1 (nx rounded up to 128 equals nx rounded up to 64), else 1, with
 *   rows_per_strip in {1, 2, 4}; share_rows 0.
 * Tangent: prefetch 0, 1 or 2.
 * Tangent (pw_advect_tangent_ex): cols_per_lane 1 or 2 (PW_F64: 1),
 *   rows_per_strip in {1, 2}.
 * share_rows (forward only; 0 everywhere else): 0 = the wavefronts of a
 *   workgroup are independent, each reading the row below and the row above
 *   its strip from memory (served by L2); 1 = the waves_per_group (2 or 4)
 *   wavefronts own consecutive strips in y and hand their edge rows to each
 *   other through LDS, so every row is read once per workgroup (the 2.5-D
 *   tile staged in LDS, paper Sec. 2.2 and Fig. 1: each value from memory
 *   once, neighbours on chip); 2 = as 1, and the rows that no other
 *   workgroup reads are loaded non-temporally.  Shared tiles take prefetch 1
 *   and: FP32 cols_per_lane 4 with rows_per_strip 1, 2 or 4; BF16 / FP16
 *   cols_per_lane 4 with rows 2 or 4, or 8 with rows 2; FP64 cols_per_lane 2
 *   with rows 2 or 4.  pw_advect_bc runs a shared tile as the same shape
 *   with share_rows 0.
 * Always zlen >= 1 and waves_per_group in 1..8.  Other values give
 * PW_ERR_INVALID_ARG.
 * The environment variable PWADV_TILE (an override for experiments) sets the
 * shape of the x-fastest forward calls that pass no tile (pw_advect,
 * pw_advect_ex, pw_advect_epilogue, pw_advect_bc) and what pw_launch_shape
 * reports for the forward: the pw_tile fields in order separated by 'x' or
 * ',', at least cols_per_lane, rows_per_strip and zlen (waves_per_group 4,
 * prefetch 1 and share_rows 0 when left out), e.g. PWADV_TILE=4x2x32x4x1x2.
 * It is read on every call and takes precedence over tuned and built-in
 * shapes; a value that does not parse, or is not a forward shape for the
 * call's storage type, makes those calls return PW_ERR_INVALID_ARG before
 * any device work.  Results do not depend on the shape. */
typedef struct {
    int32_t cols_per_lane;
    int32_t rows_per_strip;
    int32_t zlen;
    int32_t waves_per_group;
    int32_t prefetch;
    int32_t share_rows;
} pw_tile;

/* pw_advect with an explicit launch shape; tile == NULL means the library's
 * choice (the tuned shape for this grid class if pw_tune has run, else a
 * fixed default).  Same contract and results as pw_advect. */
pw_status pw_advect_ex(const pw_grid *grid, const pw_layout *layout, pw_dtype in_dtype,
                       const void *u, const void *v, const void *w,
                       const pw_coeffs *coeffs,
                       void *su, void *sv, void *sw,
                       const pw_tile *tile, void *hip_stream);

/* Forward operator with a fused epilogue:
 *   su = cu + alpha * F_u(u, v, w),  sv = cv + alpha * F_v,  sw = cw + alpha * F_w
 * in the compute type (float; double for PW_F64), one rounding per element
 * (fma).  cu/cv/cw are arrays in the output layout and compute type.  Two
 * uses: accumulation into the outputs (cu == su etc., alpha = 1: other
 * components of a model add to the same source terms), and a fused explicit
 * time step (cu = the interior of u, su = the interior of the next state,
 * alpha = dt; pass a layout whose output strides are the padded strides).
 * Each addend must be its own output or overlap no output at all; it may
 * overlap the inputs.  Same launch shapes and rules as pw_advect_ex; tile ==
 * NULL means the library's choice. */
typedef struct {
    double alpha;
    const void *cu, *cv, *cw;
} pw_epilogue;
pw_status pw_advect_epilogue(const pw_grid *grid, const pw_layout *layout, pw_dtype in_dtype,
                             const void *u, const void *v, const void *w,
                             const pw_coeffs *coeffs, const pw_epilogue *epilogue,
                             void *su, void *sv, void *sw,
                             const pw_tile *tile, void *hip_stream);

/* Adjoint (vector-Jacobian product) of the forward operator:
 *   (gu, gv, gw) = J(u, v, w)^T (gsu, gsv, gsw)
 * i.e. the gradient of <su, gsu> + <sv, gsv> + <sw, gsw> with respect to every
 * padded entry of u, v, w, halo included.  gsu/gsv/gsw are interior-shaped
 * (output layout); gu/gv/gw are padded-shaped (input layout) and fully
 * overwritten, halo cells included (entries no output reads get 0).  dtype
 * PW_F32 or PW_F64 (PW_ERR_UNSUPPORTED otherwise).  Gradients must not
 * overlap any other argument, coefficient arrays included. */
pw_status pw_advect_adjoint(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                            const void *u, const void *v, const void *w,
                            const pw_coeffs *coeffs,
                            const void *gsu, const void *gsv, const void *gsw,
                            void *gu, void *gv, void *gw,
                            void *hip_stream);

/* pw_advect_adjoint with an explicit launch shape (see pw_tile); tile ==
 * NULL as in pw_advect_adjoint.  Results are bit-identical across shapes. */
pw_status pw_advect_adjoint_ex(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                               const void *u, const void *v, const void *w,
                               const pw_coeffs *coeffs,
                               const void *gsu, const void *gsv, const void *gsw,
                               void *gu, void *gv, void *gw,
                               const pw_tile *tile, void *hip_stream);

/* Tangent-linear operator (Jacobian-vector product) of the forward operator:
 *   (tu, tv, tw) = J(u, v, w) (du, dv, dw)
 * the derivative of (su, sv, sw) in direction (du, dv, dw): every term
 * s*c*a*(b+d) of the equations above contributes s*c*(da*(b+d) + a*(db+dd)).
 * The operator is quadratic, so in exact arithmetic this equals
 * (F(x+d) - F(x-d)) / 2.  du/dv/dw are padded-shaped (input layout, halo
 * read); tu/tv/tw interior-shaped (output layout).  dtype PW_F32 or PW_F64
 * (PW_ERR_UNSUPPORTED otherwise); arithmetic in that type.  Outputs must not
 * overlap any input or coefficient array.  With pw_advect_adjoint it forms a
 * tangent-linear / adjoint pair: <J d, y> = <d, J^T y>. */
pw_status pw_advect_tangent(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                            const void *u, const void *v, const void *w,
                            const pw_coeffs *coeffs,
                            const void *du, const void *dv, const void *dw,
                            void *tu, void *tv, void *tw,
                            void *hip_stream);

/* pw_advect_tangent with an explicit launch shape (see pw_tile); tile ==
 * NULL means the library's choice.  Results are bit-identical across shapes. */
pw_status pw_advect_tangent_ex(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                               const void *u, const void *v, const void *w,
                               const pw_coeffs *coeffs,
                               const void *du, const void *dv, const void *dw,
                               void *tu, void *tv, void *tw,
                               const pw_tile *tile, void *hip_stream);

/* Gradients of L = <su, gsu> + <sv, gsv> + <sw, gsw> with respect to the
 * coefficients.  L is linear in each coefficient (every term of the equations
 * above is one coefficient times a coefficient-free product), so the
 * gradients do not depend on the coefficients' values and need none.
 * `grad` (device, 6*nz + 2 doubles) receives, in this order:
 *   dL/dtzc1[0..nz), dL/dtzc2[0..nz), dL/dtzd1[0..nz), dL/dtzd2[0..nz),
 *   each level's share of dL/dtcx [0..nz) and of dL/dtcy [0..nz),
 *   dL/dtcx, dL/dtcy.
 * Sums are accumulated in FP64 in a fixed order (the same result on every
 * run): per point and strip of the adjoint's march (strips of 62 padded
 * columns and a number of rows fixed by the grid's size), then over the
 * strips, then (tcx, tcy) over the levels.  u, v, w padded (input
 * layout), gsu/gsv/gsw interior (output layout); dtype PW_F32 or PW_F64.
 * `workspace` is device memory of at least pw_advect_coeff_grad_workspace()
 * bytes (6 nz ceil((nx+2h)/62) (ny+2h) doubles), owned by the caller; it and
 * grad must be 8-byte aligned and overlap nothing else.  No allocation. */
pw_status pw_advect_coeff_grad_workspace(const pw_grid *grid, pw_dtype dtype, int64_t *bytes);
pw_status pw_advect_coeff_grad(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                               const void *u, const void *v, const void *w,
                               const void *gsu, const void *gsv, const void *gsw,
                               double *grad, void *workspace, int64_t workspace_bytes,
                               void *hip_stream);

/* pw_advect_coeff_grad for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same result, bit for bit, with the
 * per-strip partials in the library's own static device scratch of 16 MiB
 * (PW_COEFF_GRAD_STATIC_MAX_BYTES) instead of a caller workspace.  Grids
 * whose partials need more (pw_advect_coeff_grad_workspace() bytes) are
 * rejected with PW_ERR_UNSUPPORTED before anything runs.  No allocation and
 * no memset: every partial is written before it is read.  Each GPU holds its
 * own copy of the scratch until the process ends; its address is looked up
 * on a device's first call (make that first call outside graph capture).
 * All calls on one GPU share that scratch, so calls that overlap in time on
 * one GPU (on different streams, or from different threads without ordering)
 * race and give wrong results. */
#define PW_COEFF_GRAD_STATIC_MAX_BYTES (16LL << 20)
pw_status pw_advect_coeff_grad_static(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                                      const void *u, const void *v, const void *w,
                                      const void *gsu, const void *gsv, const void *gsw,
                                      double *grad, void *hip_stream);

/* The whole backward of L = <su, gsu> + <sv, gsv> + <sw, gsw> in one pass
 * over u, v, w and the cotangents: the wind gradients of pw_advect_adjoint
 * (gu, gv, gw) and the coefficient gradients of pw_advect_coeff_grad (grad),
 * from the same adjoint march (Sec. 4's term structure: every term is one
 * coefficient times a coefficient-free product, whose factors the adjoint
 * already holds).  Both results equal, bit for bit, those of
 * pw_advect_adjoint and pw_advect_coeff_grad called separately: the wind
 * gradients do not depend on the launch shape, and the coefficient partials
 * are per strip of one shape that depends on the grid's size alone, whether
 * or not the wind gradients come with them.  Arguments, ownership and errors
 * as the two calls; grad and the workspace must also overlap none of gu, gv,
 * gw.  PW_F32 / PW_F64.  No allocation. */
pw_status pw_advect_adjoint_coeff_grad(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype,
                                       const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                                       const void *gsu, const void *gsv, const void *gsw,
                                       void *gu, void *gv, void *gw, double *grad, void *workspace,
                                       int64_t workspace_bytes, void *hip_stream);

/* Autotuner for single-grid launches.  Times candidate launch shapes of the
 * forward kernel (flags & PW_TUNE_FORWARD), the z-fastest forward kernel
 * (flags & PW_TUNE_ZFAST) and, for PW_F32 / PW_F64, of the adjoint
 * (flags & PW_TUNE_ADJOINT) and tangent (flags & PW_TUNE_TANGENT) kernels;
 * flags == 0 means forward, adjoint and tangent.  The candidates run on scratch grids
 * of this extent (allocated and freed here; seeded pseudo-random winds in
 * [-10, 10), which also serve as cotangents, directions in [-1, 1) and
 * coefficients in [0.0025, 0.0075), since kernel times depend on the data),
 * rotating over as many copies as span about 1 GiB so that repeats are not
 * served by the MALL.  Each candidate is timed over 12 launches; the eight
 * fastest are re-timed in three interleaved rounds of 40 and ranked by their
 * median.  The fastest shape per shape class -- kernel, dtype and the
 * power-of-two ceilings of nx, ny, nz -- goes into a process-wide table that
 * the kernels consult when called without a tile.  The z-cut is kept as a
 * number of chunks, so an entry serves every nz of its class.  If the
 * environment variable PWADV_TUNE_CACHE names a file, the table is read from
 * it on first use (unreadable or malformed lines are ignored) and the
 * measured entries are rewritten to it after each pw_tune.  Entries measured
 * on MI355X for common shape classes are built in and used when nothing else
 * is known.  fwd_best / adj_best (may be NULL) receive the chosen forward and
 * adjoint shapes (pw_launch_shape reports any kernel's).  Allocates device
 * memory; synchronises its own stream. */
#define PW_TUNE_FORWARD 1
#define PW_TUNE_ADJOINT 2
#define PW_TUNE_TANGENT 4
#define PW_TUNE_ZFAST 8
pw_status pw_tune(const pw_grid *grid, pw_dtype dtype, int32_t flags, pw_tile *fwd_best, pw_tile *adj_best);

/* The launch shape a kernel takes for this grid and dtype when called with
 * tile == NULL: the tuned entry of its shape class if there is one, else the
 * library's default.  No device work.  PW_ERR_UNSUPPORTED for an adjoint or
 * tangent of a 16-bit dtype. */
typedef enum { PW_KERNEL_FORWARD = 0, PW_KERNEL_ADJOINT = 1, PW_KERNEL_TANGENT = 2, PW_KERNEL_ZFAST = 3 } pw_kernel;
pw_status pw_launch_shape(pw_kernel kind, const pw_grid *grid, pw_dtype dtype, pw_tile *out);

/* Empties the process-wide tuning table, built-in entries included (the
 * cache file is left as is). */
pw_status pw_tune_reset(void);

/* ------------------------------------------------------------------------
 * Batched form: many independent subdomains of their own shapes processed by
 * one persistent launch (the paper's multi-compute-unit design decomposes the
 * grid into independent parts, one per compute unit, Sec. 5; here the parts
 * are MONC-rank-sized subdomains that share one launch on one GPU).
 *
 * A batch is created once for a fixed set of subdomains (pointers, shapes,
 * strides and coefficients are captured at creation; the arrays' contents
 * may change between runs).  Its work list holds one work item per
 * (subdomain, strip, z-chunk); wavefronts of the persistent grid pull items
 * from a device counter until the list is exhausted.
 * ------------------------------------------------------------------------ */
typedef struct {
    pw_grid grid;
    pw_layout layout;           /* element strides; all four zero = dense */
    const void *u, *v, *w;      /* padded inputs (device), dtype of the batch */
    pw_coeffs coeffs;           /* tz* device arrays of grid.nz elements */
    void *su, *sv, *sw;         /* interior outputs (device) */
} pw_batch_item;

typedef struct pw_batch pw_batch;   /* opaque handle */

/* Validates every item as pw_advect would (and that no output overlaps any
 * input or output of any item), builds the work list for `tile` (NULL: the
 * library's default shape) and uploads it.  dtype: PW_F32.  Allocates the
 * device work list and counter (freed by pw_batch_destroy).  *out receives
 * the handle; on error *out is NULL and nothing is allocated. */
pw_status pw_batch_create(const pw_batch_item *items, int32_t n, pw_dtype dtype, const pw_tile *tile,
                          pw_batch **out);

/* One pass over every subdomain: a counter-reset kernel and the persistent
 * kernel, enqueued on hip_stream.  Capturable into a graph. */
pw_status pw_batch_run(pw_batch *batch, void *hip_stream);

/* Captures pw_batch_run into a HIP graph (on hip_stream, which must not be
 * the NULL stream) and instantiates it; replaces a previous capture. */
pw_status pw_batch_capture(pw_batch *batch, void *hip_stream);

/* Launches the captured graph on hip_stream (PW_ERR_INVALID_ARG if the batch
 * has not been captured since its last re-tiling). */
pw_status pw_batch_replay(pw_batch *batch, void *hip_stream);

/* Autotuner: times candidate launch shapes on the batch's own buffers
 * (outputs are overwritten with valid results), keeps the fastest, rebuilds
 * the work list for it and drops any captured graph.  Synchronises
 * hip_stream.  If `chosen` is non-NULL it receives the shape. */
pw_status pw_batch_tune(pw_batch *batch, void *hip_stream, pw_tile *chosen);

/* Current launch shape and work-list size of a batch. */
pw_status pw_batch_info(const pw_batch *batch, pw_tile *tile, int64_t *work_items, int32_t *workgroups);

/* Frees the batch (device work list, counter, graph).  NULL is a no-op. */
pw_status pw_batch_destroy(pw_batch *batch);

/* ------------------------------------------------------- z-fastest layout
 * The forward operator (the same equations and, per point, the same
 * arithmetic as pw_advect, so the results are bit-identical) on arrays stored
 * with z contiguous -- column-major, the way a model keeps its columns
 * (Sec. 2.1 names the host model; its Fortran arrays are indexed (k, j, i)):
 *   input   (k, j, i), padded indices, at  i*in_si  + j*in_sj  + k
 *   output  (kk, jj, ii), interior indices, at  ii*out_si + jj*out_sj + kk
 * Strides in elements; layout NULL means dense (in_sj = nz+2h,
 * in_si = (ny+2h)*in_sj, out_sj = nz, out_si = ny*nz).  in_sj >= nz+2h,
 * in_si >= (ny+2h)*in_sj, out_sj >= nz, out_si >= ny*out_sj, and one x-plane
 * (in_si, out_si elements) below 2 GiB.  dtype, coefficients, ownership,
 * streams and errors as for pw_advect_ex.  The tile's fields mean: levels per
 * lane (1, 2, or 4 except PW_F64), y-rows per strip (1, 2; 4 with at most 2
 * levels per lane; 8 with 1), x-columns per work item (zlen),
 * waves_per_group 1..8, prefetch 1 or 2 x-planes.  tile NULL: the tuned
 * shape (PW_KERNEL_ZFAST) or the default. */
typedef struct {
    int64_t in_sj, in_si;
    int64_t out_sj, out_si;
} pw_layout_zfast;
pw_status pw_advect_zfast(const pw_grid *grid, const pw_layout_zfast *layout, pw_dtype in_dtype,
                          const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                          void *su, void *sv, void *sw, const pw_tile *tile, void *hip_stream);

/* The fused epilogue of pw_advect_epilogue (out = c + alpha * F, one fma per
 * element) on z-fastest arrays: cu/cv/cw in the output layout (out_sj,
 * out_si) and compute type, each either its own output (accumulation into a
 * model's source terms) or overlapping no output.  Results are bit-identical
 * to pw_advect_epilogue on the transposed arrays. */
pw_status pw_advect_zfast_epilogue(const pw_grid *grid, const pw_layout_zfast *layout, pw_dtype in_dtype,
                                   const void *u, const void *v, const void *w, const pw_coeffs *coeffs,
                                   const pw_epilogue *ep, void *su, void *sv, void *sw, const pw_tile *tile,
                                   void *hip_stream);

/* ------------------------------------------------------------- halo fill
 * The step before the stencil: fill the halo of padded arrays from their
 * interiors.  The stencil (Sec. 2.2) reads one layer of neighbours, which a
 * model provides by a periodic or neighbour exchange in the horizontal and a
 * boundary condition at the surface and lid (Sec. 2.1 places the scheme in
 * such a model; the paper fixes no rule, these are the library's).
 *
 * Per axis, with n interior cells and halo width h, halo cell p (padded
 * index, p < h or p >= n+h) becomes:
 *   PW_HALO_KEEP         untouched
 *   PW_HALO_PERIODIC     interior cell h + ((p - h) mod n)
 *   PW_HALO_COPY         nearest interior cell (zero normal gradient)
 *   PW_HALO_ZERO         0 (+0.0)
 *   PW_HALO_REFLECT      the mirror image across the boundary face,
 *                        2h-1-p below and 2(n+h)-1-p above; needs n >= h
 *   PW_HALO_REFLECT_NEG  minus that mirror image (exact sign flip), so the
 *                        field's linear interpolant vanishes on the face
 * The result equals filling x first (all rows and planes), then y (whole
 * rows, x-halo included), then z (whole planes), so edges and corners take
 * the value of a sequential exchange.  E.g. a free-slip rigid lid: u, v with
 * z = COPY and w with z = ZERO; a no-slip wall: u, v with z = REFLECT_NEG.
 *
 * fields[f] (f < nfields, 1 <= nfields <= 8) are distinct padded arrays of
 * `dtype` on the current device, in the input layout of `layout` (in_sy,
 * in_sz; out_* ignored; NULL = dense), updated in place on `hip_stream`;
 * modes[f] gives field f's x, y, z rules.  Interior cells are never written
 * and are the only cells read (on KEEP axes, the cell's own line), so the
 * fill is one kernel with no ordering between its writes.  The rules are
 * per axis, so arrays stored z-fastest (pw_advect_zfast's layout) are filled
 * by passing nx and nz exchanged in `grid` and the x and z rules exchanged
 * in `modes`, with in_sy = the column stride and in_sz = the x-plane stride.
 * Errors
 * (PW_ERR_INVALID_ARG): NULL or misaligned fields, overlapping fields, an
 * unknown mode, REFLECT with n < h, nfields out of range. */
typedef enum {
    PW_HALO_KEEP = 0,
    PW_HALO_PERIODIC = 1,
    PW_HALO_COPY = 2,
    PW_HALO_ZERO = 3,
    PW_HALO_REFLECT = 4,
    PW_HALO_REFLECT_NEG = 5
} pw_halo_mode;
typedef struct {
    int32_t x, y, z; /* pw_halo_mode per axis */
} pw_halo_modes;
pw_status pw_halo_fill(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype, void *const fields[],
                       const pw_halo_modes modes[], int32_t nfields, void *hip_stream);

/* The adjoint (transpose) of pw_halo_fill with the same rules, in place:
 * gradients with respect to filled arrays become gradients with respect to
 * the arrays before the fill.  The fill is x, then y, then z; the fold takes
 * the per-axis transposes in the order z, y, x: every halo cell of the axis
 * is added, times the sign of its rule (-1 for REFLECT_NEG), into the cell it
 * was copied from, in ascending order of its index, and then set to zero
 * (ZERO: only set to zero; KEEP: the axis is left alone).  On one GPU this
 * is the reverse of the halo exchange: halo gradients go back to their
 * owners.  PW_F32 / PW_F64 only (PW_ERR_UNSUPPORTED otherwise); other
 * arguments and errors as pw_halo_fill.  Three small launches on
 * hip_stream. */
pw_status pw_halo_fold(const pw_grid *grid, const pw_layout *layout, pw_dtype dtype, void *const fields[],
                       const pw_halo_modes modes[], int32_t nfields, void *hip_stream);

/* ------------------------------------------------ boundaries by addressing
 * The forward operator, optionally with the fused epilogue, with the halo's
 * boundary rules applied by addressing instead of a halo fill: the result is
 * bit for bit that of pw_halo_fill(u, v, w with rules bc[0], bc[1], bc[2])
 * followed by pw_advect_ex / pw_advect_epilogue, but the halo is neither
 * written nor (on axes whose rule is not KEEP) read.  bc[f] holds the x, y, z
 * rules of field f (u, v, w), any of the six pw_halo_mode rules.  The
 * stencil reads one layer of halo (Sec. 2.2), and for those cells the
 * mirror image of REFLECT / REFLECT_NEG is the nearest interior cell; so a
 * read of a halo cell goes to its periodic or nearest-interior source, and
 * ZERO and REFLECT_NEG then replace the value by +0 or flip its sign, per
 * field, in the fill's axis order (corner cells included).  A periodic
 * x-y domain with a free-slip lid (u, v: z = COPY, w: z = ZERO) or a
 * no-slip wall (REFLECT_NEG) then needs no fill step at all.  The read
 * remapping is shared by the three fields: on each axis they must all be
 * KEEP, all PERIODIC, or all nearest-cell rules (COPY, ZERO, REFLECT,
 * REFLECT_NEG), else PW_ERR_UNSUPPORTED.  REFLECT / REFLECT_NEG on an axis
 * with fewer interior cells than the halo width, or an unknown rule:
 * PW_ERR_INVALID_ARG (as pw_halo_fill).  ep == NULL: out = F; otherwise as
 * pw_advect_epilogue.  Same layouts, dtypes, tiles, ownership and errors as
 * pw_advect_ex. */
pw_status pw_advect_bc(const pw_grid *grid, const pw_layout *layout, pw_dtype in_dtype, const void *u,
                       const void *v, const void *w, const pw_coeffs *coeffs, const pw_halo_modes bc[3],
                       const pw_epilogue *ep, void *su, void *sv, void *sw, const pw_tile *tile, void *hip_stream);

/* Library version string (static storage). */
const char *pw_version(void);

/* Message for the last non-OK status returned on the calling thread
 * (static per-thread storage; "" if none).  With the environment variable
 * PWADV_LOG set (and not "0"), every launching call also prints one line on
 * stderr: the entry point, grid, storage type, launch shape and whether the
 * shape was given, came from PWADV_TILE, was tuned, the default or a fixed
 * rule. */
const char *pw_last_error(void);

/* Measurement helper: a plain vectorised device-to-device copy of `nbytes`
 * (a multiple of 16, both pointers 16-byte aligned) on `hip_stream`, with the
 * same launch shape policy as the stencil kernels.  Used to calibrate the
 * reachable HBM bandwidth and the memory counters. */
pw_status pw_stream_copy(const void *src, void *dst, int64_t nbytes, void *hip_stream);

/* Measurement helper: three such copies (src[i] -> dst[i], i = 0..2, each of
 * `nbytes`) in one kernel -- the stencil's traffic pattern of three arrays
 * read and three written, without the stencil.  Its bandwidth is the
 * reachable rate for that pattern.  Same argument rules as pw_stream_copy;
 * no two of the six ranges may overlap. */
pw_status pw_stream_copy3(const void *const src[3], void *const dst[3], int64_t nbytes, void *hip_stream);

/* Bandwidth probe (measurement only: the rate the HBM reaches for plain
 * streams, the ceiling the stencil kernels are compared with).
 *   mode 0: copy src -> dst; 1: read src only (dst is a sink of at least
 *   4096 bytes, written only if an XOR of all data read equals one fixed
 *   128-bit pattern); 2: write dst only (src unused, may be NULL).
 *   loads_per_lane in {1, 2, 4, 8}: independent 16-byte loads (or stores)
 *   per lane in flight before the matching stores.
 *   flags bit 0: non-temporal loads; bit 1: non-temporal stores.
 *   blocks: workgroups of 256 threads, 1 .. 1048576 (grid-stride loop).
 * nbytes > 0 and a multiple of 16; buffers 16-byte aligned device memory of
 * nbytes each (the read-only sink: 4096), not overlapping. */
pw_status pw_stream_probe(int32_t mode, int32_t loads_per_lane, int32_t flags, const void *src, void *dst,
                          int64_t nbytes, int32_t blocks, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PWADV_H */
