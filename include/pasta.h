/*
 * pasta.h - C ABI of the MI355X (gfx950) COO MTTKRP library (libpasta.so).
 *
 * The operation is the mode-n MTTKRP of a sparse tensor stored in COO form
 * (Section 4.6, eq. mttkrp-init; Section 5.2, Alg. 6 and its text):
 *
 *     out[i][r] = alpha * sum over nonzeros m with i_n(m) = i of
 *                 x(m) * prod_{k != n} U^(k)[i_k(m)][r],
 *
 * for every row i of mode n (rows without nonzeros are zero), plus the
 * sampled CP model and its residual-weighted MTTKRP gradient (CP
 * decomposition, Section 3.1.1), a CP-ALS sweep, the fiber-based sparse
 * TTM and TTV of Sections 4.3-4.4 (Algs. 4 and 5), and the element-wise
 * (TEW) and tensor-scalar (TS) operations of Sections 4.1-4.2 (Algs. 1-3).
 *
 * Conventions shared by every entry point
 *   - Coordinates are 0-based (the COO example of Section 5.1); indices are
 *     uint32 and values fp32 (the storage assumption of Table 2).
 *   - Factor U^(k) is row-major I_k x ldf, element type fp32 or bf16, only
 *     the first R columns are read (Alg. 6 addresses rows as i*R + r).
 *   - Outputs are fp32, row-major with leading dimension ldo; only columns
 *     0..R-1 are written.
 *   - Every pointer named d_* is HIP device memory owned by the caller; the
 *     library allocates no device memory. Host arrays are read during the
 *     call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     All work is enqueued on it and the call returns without waiting,
 *     except pasta_coo_create, which waits once for its index check, and
 *     pasta_fibers_create and pasta_tew, which wait once to read a count.
 *   - Argument errors are reported synchronously through the return value
 *     and nothing is enqueued; the library never aborts or throws.
 *   - Calls that share a handle may run concurrently only if they do not
 *     share a workspace or an output buffer.
 */
#ifndef PASTA_H
#define PASTA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PASTA_OK = 0,
    PASTA_EINVAL = 1,       /* a null pointer, a zero size, mode >= order, ld < rank, ... */
    PASTA_ERANGE = 2,       /* some coordinate is >= its dimension */
    PASTA_EUNSUPPORTED = 3, /* order, rank, dtype or alignment outside the supported set */
    PASTA_EWORKSPACE = 4,   /* workspace smaller than the queried size, or not 256-byte aligned */
    PASTA_EHIP = 5,         /* a HIP runtime call failed; see pasta_last_hip_error() */
    PASTA_EINTERNAL = 6     /* a kernel found the preprocessed tensor inconsistent (pasta_coo_check) */
} pasta_status;

typedef enum { PASTA_F32 = 0, PASTA_BF16 = 1 } pasta_dtype;

/* Element-wise / tensor-scalar operator (Sections 4.1-4.2). */
typedef enum { PASTA_ADD = 0, PASTA_SUB = 1, PASTA_MUL = 2, PASTA_DIV = 3 } pasta_ewop;

/* Opaque host-side handle of a preprocessed COO tensor. It points into the
 * caller's workspace and the caller's original index/value arrays, which
 * must stay alive and unchanged until pasta_coo_destroy. */
typedef struct pasta_coo pasta_coo;

/* Supported ranges. */
#define PASTA_MAX_ORDER 8
#define PASTA_MAX_RANK 256

/* Bytes of device workspace that pasta_coo_create needs for an order-N
 * tensor with these dimensions and nnz nonzeros (nnz < 2^32, 2 <= N <= 8,
 * 1 <= dims[k] <= 2^31). Holds, for every mode, the nonzeros sorted by
 * that mode's index (SoA), the sort permutation and the row offsets. */
pasta_status pasta_coo_workspace_bytes(uint32_t order, const uint64_t *dims, uint64_t nnz, size_t *bytes);

/* Preprocess a COO tensor (the sorting and fiber/row pointers the suite
 * builds before its kernels, Section 5.2): checks every coordinate against
 * its dimension, then for every mode n sorts the nonzeros by i_n and stores
 * the sorted copy, the permutation and the row offsets in the workspace.
 * Mode n's order is lexicographic in (i_n, i_{n-1}, ..., i_0), then i_{N-1}
 * (for n < N-1), then caller position: each mode's order is the stable sort
 * by i_n of the previous mode's order.
 *   d_inds  host array of `order` device pointers; d_inds[k][m] = i_k(m).
 *   d_vals  device array of nnz fp32 values.
 *   d_workspace  >= pasta_coo_workspace_bytes, 256-byte aligned.
 * Waits for the stream once. Returns PASTA_ERANGE (and no handle) if any
 * coordinate is out of range. On success *out owns only host memory. */
pasta_status pasta_coo_create(uint32_t order, const uint64_t *dims, uint64_t nnz, const uint32_t *const *d_inds,
                              const float *d_vals, void *d_workspace, size_t workspace_bytes, void *stream,
                              pasta_coo **out);

/* Waits for `stream`, then reports whether any MTTKRP-based kernel that ran on X
 * since pasta_coo_create found its mode-sorted stream out of order (PASTA_EINTERNAL;
 * their outputs are then undefined) or none did (PASTA_OK). The wave-run MTTKRP
 * kernel checks the row order it relies on and, instead of looping on a stream that
 * breaks it, sets a device flag in X's workspace and stops that row walk; the flag
 * stays set for the life of the handle. A preprocessed tensor is always in order,
 * so PASTA_EINTERNAL means its workspace was overwritten or a library defect. */
pasta_status pasta_coo_check(const pasta_coo *X, void *stream);

/* Free the host handle. Device memory stays the caller's. */
pasta_status pasta_coo_destroy(pasta_coo *X);

/* Order and nonzero count of a handle. */
pasta_status pasta_coo_info(const pasta_coo *X, uint32_t *order, uint64_t *nnz);

/* Device views of the mode-`mode` preprocessing (all read-only, valid
 * while the workspace lives). Any output pointer may be NULL.
 *   d_perm[p]    caller position of the p-th nonzero in mode order (nnz);
 *   d_rowptr[i]  first position of row i in mode order (dims[mode] + 1);
 *   d_sorted_inds  host array of `order` pointers, filled with the sorted
 *                  index arrays (nnz each);
 *   d_sorted_vals  the values in mode order (nnz). */
pasta_status pasta_coo_mode_view(const pasta_coo *X, uint32_t mode, const uint32_t **d_perm,
                                 const uint32_t **d_rowptr, const uint32_t **d_sorted_inds,
                                 const float **d_sorted_vals);

/* Bytes of scratch workspace pasta_mttkrp needs for this mode and rank
 * (partial rows of the chunks a row spans). */
pasta_status pasta_mttkrp_workspace_bytes(const pasta_coo *X, uint32_t mode, uint32_t rank, pasta_dtype dtype,
                                          size_t *bytes);

/* Mode-n MTTKRP (eq. mttkrp-init; Alg. 6 for order N and any mode):
 *   d_factors  host array of `order` device pointers; d_factors[mode] is
 *              not read and may be NULL.
 *   dtype      element type of every factor (fp32 or bf16; arithmetic and
 *              accumulation are fp32 either way).
 *   rank R     1..PASTA_MAX_RANK; ldf >= R (elements).
 *   d_vals_override  NULL to use the tensor's values, else nnz fp32 values
 *              in the caller's order used instead (the residual-weighted
 *              MTTKRP of a CP gradient).
 *   alpha      scale applied to the result.
 *   d_out      dims[mode] x ldo fp32, OVERWRITTEN (every row, empty rows
 *              get zeros); ldo >= R.
 *   d_work     >= pasta_mttkrp_workspace_bytes, 256-byte aligned.
 * The result is deterministic: the same inputs give the same bits. */
pasta_status pasta_mttkrp(const pasta_coo *X, uint32_t mode, const void *const *d_factors, pasta_dtype dtype,
                          uint32_t rank, uint32_t ldf, const float *d_vals_override, float alpha, float *d_out,
                          uint32_t ldo, void *d_work, size_t work_bytes, void *stream);

/* pasta_mttkrp for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the same
 * arguments and the same kernels and results, without d_work. Its scratch (the
 * partial rows of the chunks a row spans) is a fixed array of
 * PASTA_STATIC_SCRATCH_BYTES inside the library; each GPU it runs on holds its own
 * copy until the process ends. It allocates nothing (no hipMalloc, no library
 * allocation). Returns PASTA_EWORKSPACE, and launches nothing, if the call needs
 * more scratch than the array holds (pasta_mttkrp_workspace_bytes gives an upper
 * bound of the need: e.g. R = 64 fp32 at up to ~130M nonzeros fits). All calls on
 * one GPU share its array and it keeps the last call's contents (no call relies on
 * them: every slot a call reads, the same call wrote first), so calls that overlap
 * in time on one GPU race: serialise them (one stream, or events). */
#define PASTA_STATIC_SCRATCH_BYTES (64u << 20)
pasta_status pasta_mttkrp_static(const pasta_coo *X, uint32_t mode, const void *const *d_factors, pasta_dtype dtype,
                                 uint32_t rank, uint32_t ldf, const float *d_vals_override, float alpha, float *d_out,
                                 uint32_t ldo, void *stream);

/* The same product computed the way the suite's parallel CPU code does with
 * atomics (Section 5.3): nonzeros in caller order, one atomic row update
 * per nonzero, no sorting. Kept as a reference point for measurements;
 * not deterministic in the last bits. d_out is overwritten. */
pasta_status pasta_mttkrp_atomic(const pasta_coo *X, uint32_t mode, const void *const *d_factors, pasta_dtype dtype,
                                 uint32_t rank, uint32_t ldf, float *d_out, uint32_t ldo, void *stream);

/* Rank-R CP model sampled at the nonzeros (CP decomposition, Section
 * 3.1.1): d_mhat[m] = sum_r prod_k U^(k)[i_k(m)][r], in caller order.
 * Every factor is read, including all modes. */
pasta_status pasta_cp_sample(const pasta_coo *X, const void *const *d_factors, pasta_dtype dtype, uint32_t rank,
                             uint32_t ldf, float *d_mhat, void *stream);

/* Bytes of scratch for pasta_cp_residual_loss (fp64 loss partials). */
pasta_status pasta_cp_workspace_bytes(const pasta_coo *X, uint32_t rank, pasta_dtype dtype, size_t *bytes);

/* Residual and loss of the observed-entry least-squares CP fit:
 *   d_resid[m] = mhat(m) - x(m) (caller order, fp32; may be NULL),
 *   *d_loss    = 1/2 sum_m resid(m)^2, accumulated in fp64 (device scalar).
 * d_work >= pasta_cp_workspace_bytes. */
pasta_status pasta_cp_residual_loss(const pasta_coo *X, const void *const *d_factors, pasta_dtype dtype,
                                    uint32_t rank, uint32_t ldf, float *d_resid, double *d_loss, void *d_work,
                                    size_t work_bytes, void *stream);

/* Loss and gradient of the observed-entry least-squares CP fit in one pass
 * per mode: for every mode n,
 *   d_grads[n] = alpha * dL/dU^(n) = alpha * MTTKRP_n(values = mhat - x),
 * with the residual recomputed in mode-n order (never stored), and
 *   *d_loss = 1/2 sum_m (mhat(m) - x(m))^2 in fp64 (may be NULL).
 * d_grads: host array of `order` device pointers, each dims[n] x ldg fp32,
 * overwritten. d_work >= max over modes of pasta_mttkrp_workspace_bytes
 * plus pasta_cp_workspace_bytes (see pasta_cp_grad_workspace_bytes). */
pasta_status pasta_cp_grad_workspace_bytes(const pasta_coo *X, uint32_t rank, pasta_dtype dtype, size_t *bytes);
pasta_status pasta_cp_grad(const pasta_coo *X, const void *const *d_factors, pasta_dtype dtype, uint32_t rank,
                           uint32_t ldf, float alpha, float *const *d_grads, uint32_t ldg, double *d_loss,
                           void *d_work, size_t work_bytes, void *stream);

/* One sweep of CP-ALS (alternating least squares, one of the CPD methods of
 * Section 3.1.1, whose bottleneck is the MTTKRP): for every mode n in turn,
 *   M = MTTKRP_n(X; U),  V = Hadamard_{k != n} (U_k^T U_k),
 *   U_n <- M V^{-1} (V^{-1} by Gauss-Jordan elimination; V is symmetric
 *   positive definite, so no pivoting),  lambda_r = ||U_n[:, r]||_2,
 *   U_n[:, r] /= lambda_r (zero columns stay zero).
 *   d_factors  host array of `order` device pointers to fp32 I_k x ldf
 *              factors, updated in place; rank R <= 64.
 *   d_lambda   R fp32 column norms of the last mode after the sweep.
 *   d_fit      (NULL or device scalar) 1 - ||X - [[lambda; U]]|| / ||X||,
 *              with the norms in fp64 (||X||^2 = sum of squared values, so
 *              repeated coordinates are taken as separate entries).
 *   d_info     (NULL or device uint32) set to 1 if some V was not
 *              numerically positive definite, else 0.
 * d_work >= pasta_cp_als_workspace_bytes. */
pasta_status pasta_cp_als_workspace_bytes(const pasta_coo *X, uint32_t rank, size_t *bytes);
pasta_status pasta_cp_als_sweep(const pasta_coo *X, float *const *d_factors, uint32_t rank, uint32_t ldf,
                                float *d_lambda, double *d_fit, uint32_t *d_info, void *d_work, size_t work_bytes,
                                void *stream);

/* fp32 -> bf16 with round to nearest, ties to even (NaN stays NaN):
 * d_dst[i] = bf16(d_src[i]) for i < count, bf16 given as uint16 bits. */
pasta_status pasta_cast_f32_to_bf16(const float *d_src, uint16_t *d_dst, uint64_t count, void *stream);

/* Measurement hook: the next main kernel that this thread launches (from
 * pasta_mttkrp, the first mode of pasta_cp_grad, pasta_ttm or pasta_ttv)
 * records ev_start
 * (a hipEvent_t) on its stream right before the launch and ev_stop right
 * after it, so their elapsed time is that kernel alone. The pair is used
 * once and then disarmed; NULL disarms. Calls with nnz = 0 leave it armed. */
pasta_status pasta_arm_kernel_events(void *ev_start, void *ev_stop);

/* Which form of the MTTKRP kernel the MTTKRP-based calls run,
 * for every later call in the process: 0 = automatic (the default: the
 * wave-run form when rows average at least 48 nonzeros, else the run form),
 * 1 = the run form (each lane group walks its own run of nonzeros), 2 = the
 * wave-run form (a wave walks one run, its groups taking consecutive
 * nonzeros). Both give the same results to rounding; it applies to
 * pasta_mttkrp (with or without a value override), pasta_cp_grad and the
 * CP-ALS sweep; TTM and the strided shape always use the run form. For
 * tuning and tests; not thread-safe against concurrent calls. */
pasta_status pasta_set_mttkrp_form(int form);

/* *form = the form (1 = run, 2 = wave-run) of the main kernel that the most
 * recent MTTKRP-based call with nnz > 0 launched in this process, 0 if there
 * was none: which kernel a timing taken with pasta_arm_kernel_events measured.
 * Not thread-safe against concurrent calls. */
pasta_status pasta_last_mttkrp_form(int *form);

/* Measurement kernel: the gather rate of the vector memory pipeline, the
 * ceiling the MTTKRP kernels' factor-row gathers are compared with. Launches
 * `blocks` workgroups of 4 waves; each wave is 64 / lanes groups of `lanes`
 * lanes, and in each of `steps` steps every group reads one row of
 * lanes x 16 bytes from d_table (lane j reads bytes 16j .. 16j+15), the rows
 * starting at a hash of (wave, group / share) and advancing by an odd stride per
 * step: share = 1 gives every group its own row, share = 64 / lanes one row per
 * wave. Only groups 0 .. active-1
 * load (1 <= active <= 64 / lanes; the others' lanes are masked off). Eight
 * steps' loads are in flight at a time. Bytes delivered =
 * blocks * 256 * steps * 16 * active / (64 / lanes).
 *   d_table  rows * lanes * 16 bytes, 16-byte aligned; rows a power of two
 *            (the table's size picks the cache level that serves it).
 *   lanes    4, 8 or 16 (the group widths of the MTTKRP kernels' 16-byte
 *            slices); share a power of two <= 64 / lanes; steps a multiple
 *            of 8.
 *   d_out    blocks * 256 * 16 bytes, 16-byte aligned; receives a fold of
 *            the loaded words (kept so that no load is dropped).
 * Asynchronous on `stream`. */
pasta_status pasta_probe_gather(const void *d_table, uint32_t rows, uint32_t lanes, uint32_t share, uint32_t active,
                                uint32_t steps, uint32_t blocks, void *d_out, void *stream);

/* d_x[i] *= (float)*d_alpha for i < count: scales a gradient by an upstream
 * derivative held on the device (no host round trip). */
pasta_status pasta_scale_f32(float *d_x, uint64_t count, const double *d_alpha, void *stream);

/* One Adam step on fp32 parameters (the optimiser of a gradient-based CP fit,
 * a gradient-descent CPD method as listed in Section 3.1.1), in place:
 *   m = b1*m + (1-b1)*g;  v = b2*v + (1-b2)*g^2;
 *   p -= lr/(1-b1^t) * m / (sqrt(v)/sqrt(1-b2^t) + eps),  t = step >= 1;
 * if d_shadow_bf16 is not NULL the updated p is also written there as bf16
 * (round to nearest even), which is the factor copy a bf16 step reads.
 * All arrays hold `count` elements. */
pasta_status pasta_adam_step(float *d_param, const float *d_grad, float *d_m, float *d_v, uint16_t *d_shadow_bf16,
                             uint64_t count, float lr, float beta1, float beta2, float eps, uint32_t step,
                             void *stream);

/* ---- Mode-n fibers, sparse TTM and TTV ---------------------------------
 * A mode-n fiber fixes every index but i_n (Section 3). TTV (Section 4.3)
 * and TTM (Section 4.4, eq. ttm) contract mode n with a vector v (I_n) or a
 * matrix U (I_n x R, the paper's orientation: row i_n holds R entries), and
 * every fiber of X that holds nonzeros gives one output entry (TTV) or one
 * dense R-vector (TTM): the result keeps the other modes sparse (Algs. 4 and
 * 5, which size the output by the fiber count nfibs). */
typedef struct pasta_fibers pasta_fibers;

/* Bytes of device workspace for pasta_fibers_create on this mode. */
pasta_status pasta_fibers_workspace_bytes(const pasta_coo *X, uint32_t mode, size_t *bytes);

/* The pre-processing step of Algs. 4 and 5: reorder the nonzeros so that
 * each mode-`mode` fiber is one contiguous run, and find nfibs, the run
 * offsets (fptr) and each fiber's coordinates. The fiber order is
 * lexicographic in the other modes' indices (in mode order), then i_mode,
 * then caller position; fibers are numbered 0..nfibs-1 in that order.
 * Reads X's preprocessed arrays on the stream; the handle then depends only
 * on d_workspace (>= pasta_fibers_workspace_bytes, 256-byte aligned), not on
 * X. Waits for the stream once. */
pasta_status pasta_fibers_create(const pasta_coo *X, uint32_t mode, void *d_workspace, size_t workspace_bytes,
                                 void *stream, pasta_fibers **out);
pasta_status pasta_fibers_destroy(pasta_fibers *F);
/* Mode and number of fibers holding nonzeros. */
pasta_status pasta_fibers_info(const pasta_fibers *F, uint32_t *mode, uint64_t *nfibs);
/* Device views (read-only; any output may be NULL):
 *   d_fptr[f]      first position of fiber f in fiber order (nfibs + 1
 *                  entries, d_fptr[nfibs] = nnz);
 *   d_coords       host array of order - 1 pointers: the fixed indices of
 *                  each fiber (nfibs each), modes in order without `mode`;
 *   d_perm[p]      caller position of the p-th nonzero in fiber order;
 *   d_fid[p]       fiber of the p-th nonzero in fiber order. */
pasta_status pasta_fibers_view(const pasta_fibers *F, const uint32_t **d_fptr, const uint32_t **d_coords,
                               const uint32_t **d_perm, const uint32_t **d_fid);

/* Sparse TTM, Y = X x_mode U (Alg. 5): for every fiber f,
 *   d_out[f][r] = sum over the nonzeros m of fiber f of x(m) * U[i_mode(m)][r].
 *   d_U    I_mode x ldu, fp32 or bf16 (fp32 arithmetic); rank R <= 256.
 *   d_out  nfibs x ldo fp32, overwritten; ldo >= R.
 *   d_work >= pasta_ttm_workspace_bytes, 256-byte aligned.
 * Deterministic (same inputs, same bits). */
pasta_status pasta_ttm_workspace_bytes(const pasta_fibers *F, uint32_t rank, pasta_dtype dtype, size_t *bytes);
pasta_status pasta_ttm(const pasta_fibers *F, const void *d_U, pasta_dtype dtype, uint32_t rank, uint32_t ldu,
                       float *d_out, uint32_t ldo, void *d_work, size_t work_bytes, void *stream);

/* Sparse TTV, Y = X x_mode v (Alg. 4): for every fiber f,
 *   d_out[f] = sum over the nonzeros m of fiber f of x(m) * v[i_mode(m)].
 *   d_v    I_mode fp32;  d_out  nfibs fp32, overwritten.
 *   d_work >= pasta_ttv_workspace_bytes, 256-byte aligned.
 * Deterministic. */
pasta_status pasta_ttv_workspace_bytes(const pasta_fibers *F, size_t *bytes);
pasta_status pasta_ttv(const pasta_fibers *F, const float *d_v, float *d_out, void *d_work, size_t work_bytes,
                       void *stream);

/* ---- Element-wise and tensor-scalar operations ------------------------- */
/* Same-pattern element-wise operation (Section 4.1; Alg. 1 for addition):
 * X and Y hold the same coordinates in the same order, so only the values
 * are combined: d_z[m] = d_x[m] op d_y[m] for m < nnz (fp32, IEEE
 * semantics: correctly rounded, x / 0 gives inf or nan). Z's coordinates
 * are X's: the caller shares (or copies) the index arrays. d_z may alias
 * d_x or d_y. */
pasta_status pasta_tew_eq(pasta_ewop op, uint64_t nnz, const float *d_x, const float *d_y, float *d_z, void *stream);

/* Tensor-scalar operation on every nonzero (Section 4.2; Alg. 3 for
 * multiplication): d_y[m] = d_x[m] op s; the pattern is unchanged (implicit
 * zeros stay zero). d_y may alias d_x. */
pasta_status pasta_ts(pasta_ewop op, uint64_t nnz, const float *d_x, float s, float *d_y, void *stream);

/* General element-wise operation of two sparse tensors of the same order
 * with any patterns and shapes (Section 4.1; Alg. 2): the output shape is
 * the element-wise maximum of the two shapes; the output lists, in
 * lexicographic order (mode 0 most significant), every coordinate that
 *   PASTA_ADD: either input holds, with x + y (or the one present);
 *   PASTA_SUB: either input holds, with x - y (or x, or -y);
 *   PASTA_MUL: both inputs hold, with x * y;
 * PASTA_DIV is not offered (an implicit zero divisor). Repeated coordinates
 * inside one input count as their sum (in that input's order).
 *   d_inds_*  host arrays of `order` device pointers (1 <= order <= 8);
 *   dims_z    host array filled with the output shape;
 *   d_inds_z, d_vals_z  capacity nnz_x + nnz_y each; *nnz_z receives the
 *             output count (host).
 *   d_work    >= pasta_tew_workspace_bytes, 256-byte aligned.
 * Waits for the stream once. PASTA_ERANGE if a coordinate is outside its
 * input's shape (the output is then undefined). */
pasta_status pasta_tew_workspace_bytes(uint32_t order, uint64_t nnz_x, uint64_t nnz_y, size_t *bytes);
pasta_status pasta_tew(uint32_t order, pasta_ewop op, const uint64_t *dims_x, uint64_t nnz_x,
                       const uint32_t *const *d_inds_x, const float *d_vals_x, const uint64_t *dims_y, uint64_t nnz_y,
                       const uint32_t *const *d_inds_y, const float *d_vals_y, uint64_t *dims_z,
                       uint32_t *const *d_inds_z, float *d_vals_z, uint64_t *nnz_z, void *d_work, size_t work_bytes,
                       void *stream);

/* Text of a status code (static storage). */
const char *pasta_status_str(pasta_status s);

/* The hipError_t of the last HIP failure on the calling thread (0 if none). */
int pasta_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PASTA_H */
