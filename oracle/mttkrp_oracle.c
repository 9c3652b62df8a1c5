/*
 * FP64 CPU oracle for COO MTTKRP and the sampled CP model.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do. It shares no code, header or table with the HIP
 * library.
 *
 * Conventions (all functions):
 *   order N (1..16), dims[k] = I_k, nnz = M;
 *   inds: SoA, inds[k*M + m] is the 0-based mode-k index of nonzero m
 *         (0-based coordinates as in the COO example of Section 5.1);
 *   vals: M doubles (the fp32 inputs widened exactly);
 *   factors: N pointers, factors[k] is U^(k), row-major I_k x ldf doubles,
 *            only the first R columns are read; factors[mode] is never read
 *            by the MTTKRP functions;
 *   out: I_n x R doubles, row-major, OVERWRITTEN.
 * Return 0 on success, -1 on a bad argument, -2 if an index is out of range,
 * -3 if a buffer could not be allocated.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static int check_args(int N, const uint64_t *dims, uint64_t M, const uint32_t *inds, int R, int ldf, int mode)
{
    if (N < 1 || N > 16 || R < 1 || ldf < R || mode < 0 || mode >= N) return -1;
    if (M > 0 && !inds) return -1;
    for (int k = 0; k < N; ++k) {
        const uint32_t *ik = inds + (uint64_t)k * M;
        for (uint64_t m = 0; m < M; ++m)
            if ((uint64_t)ik[m] >= dims[k]) return -2;
    }
    return 0;
}

/*
 * Mode-n MTTKRP, sequential (Section 4.6, eq. mttkrp-init; Section 5.2,
 * Alg. 6, generalised from order 3 / mode 1 to order N and any mode n):
 *   out[i][r] = sum over nonzeros m with i_n(m) = i of
 *               val(m) * prod_{k != n} U^(k)[i_k(m)][r].
 * Nonzeros are visited in the order given; for each, the R-wide product of
 * the N-1 factor rows is formed in ascending k and added to the output row.
 */
int oracle_mttkrp_seq(int N, const uint64_t *dims, uint64_t M, const uint32_t *inds, const double *vals,
                      const double *const *factors, int R, int ldf, int mode, double *out)
{
    int rc = check_args(N, dims, M, inds, R, ldf, mode);
    if (rc) return rc;
    memset(out, 0, sizeof(double) * dims[mode] * (uint64_t)R);
    double *t = (double *)malloc(sizeof(double) * (size_t)R);
    if (!t) return -3;
    for (uint64_t m = 0; m < M; ++m) {
        for (int r = 0; r < R; ++r) t[r] = vals[m];
        for (int k = 0; k < N; ++k) {
            if (k == mode) continue;
            const double *row = factors[k] + (uint64_t)inds[(uint64_t)k * M + m] * (uint64_t)ldf;
            for (int r = 0; r < R; ++r) t[r] *= row[r];
        }
        double *o = out + (uint64_t)inds[(uint64_t)mode * M + m] * (uint64_t)R;
        for (int r = 0; r < R; ++r) o[r] += t[r];
    }
    free(t);
    return 0;
}

/*
 * Parallel MTTKRP with privatisation (Section 5.3): every thread accumulates
 * its share of the nonzeros into a private I_n x R buffer, then the buffers
 * are reduced into the output row by row.
 */
int oracle_mttkrp_priv(int N, const uint64_t *dims, uint64_t M, const uint32_t *inds, const double *vals,
                       const double *const *factors, int R, int ldf, int mode, double *out)
{
    int rc = check_args(N, dims, M, inds, R, ldf, mode);
    if (rc) return rc;
    const uint64_t In = dims[mode];
    const int T = omp_get_max_threads();
    double *priv = (double *)calloc((size_t)T * In * (uint64_t)R, sizeof(double));
    if (!priv) return -3;
#pragma omp parallel num_threads(T)
    {
        const int tid = omp_get_thread_num();
        double *mine = priv + (uint64_t)tid * In * (uint64_t)R;
        double t[512];
#pragma omp for schedule(static)
        for (uint64_t m = 0; m < M; ++m) {
            for (int r0 = 0; r0 < R; r0 += 512) {
                const int rn = (R - r0) < 512 ? (R - r0) : 512;
                for (int r = 0; r < rn; ++r) t[r] = vals[m];
                for (int k = 0; k < N; ++k) {
                    if (k == mode) continue;
                    const double *row = factors[k] + (uint64_t)inds[(uint64_t)k * M + m] * (uint64_t)ldf + r0;
                    for (int r = 0; r < rn; ++r) t[r] *= row[r];
                }
                double *o = mine + (uint64_t)inds[(uint64_t)mode * M + m] * (uint64_t)R + r0;
                for (int r = 0; r < rn; ++r) o[r] += t[r];
            }
        }
#pragma omp for schedule(static)
        for (uint64_t e = 0; e < In * (uint64_t)R; ++e) {
            double s = 0.0;
            for (int q = 0; q < T; ++q) s += priv[(uint64_t)q * In * (uint64_t)R + e];
            out[e] = s;
        }
    }
    free(priv);
    return 0;
}

/*
 * Parallel MTTKRP with atomics (Section 5.3): nonzeros are split across
 * threads and every output update is an atomic add.
 */
int oracle_mttkrp_atomic(int N, const uint64_t *dims, uint64_t M, const uint32_t *inds, const double *vals,
                         const double *const *factors, int R, int ldf, int mode, double *out)
{
    int rc = check_args(N, dims, M, inds, R, ldf, mode);
    if (rc) return rc;
    memset(out, 0, sizeof(double) * dims[mode] * (uint64_t)R);
#pragma omp parallel
    {
        double t[512];
#pragma omp for schedule(static)
        for (uint64_t m = 0; m < M; ++m) {
            for (int r0 = 0; r0 < R; r0 += 512) {
                const int rn = (R - r0) < 512 ? (R - r0) : 512;
                for (int r = 0; r < rn; ++r) t[r] = vals[m];
                for (int k = 0; k < N; ++k) {
                    if (k == mode) continue;
                    const double *row = factors[k] + (uint64_t)inds[(uint64_t)k * M + m] * (uint64_t)ldf + r0;
                    for (int r = 0; r < rn; ++r) t[r] *= row[r];
                }
                double *o = out + (uint64_t)inds[(uint64_t)mode * M + m] * (uint64_t)R + r0;
                for (int r = 0; r < rn; ++r) {
#pragma omp atomic
                    o[r] += t[r];
                }
            }
        }
    }
    return 0;
}

/*
 * Rank-R CP model sampled at the nonzeros (CP decomposition, Section 3.1.1):
 *   mhat(m) = sum_r prod_{k=0..N-1} U^(k)[i_k(m)][r].
 * Uses every factor, including the one of any mode.
 */
int oracle_cp_sample(int N, const uint64_t *dims, uint64_t M, const uint32_t *inds, const double *const *factors,
                     int R, int ldf, double *mhat)
{
    int rc = check_args(N, dims, M, inds, R, ldf, 0);
    if (rc) return rc;
#pragma omp parallel for schedule(static)
    for (uint64_t m = 0; m < M; ++m) {
        double s = 0.0;
        for (int r = 0; r < R; ++r) {
            double p = 1.0;
            for (int k = 0; k < N; ++k)
                p *= factors[k][(uint64_t)inds[(uint64_t)k * M + m] * (uint64_t)ldf + r];
            s += p;
        }
        mhat[m] = s;
    }
    return 0;
}

/*
 * Observed-entry least-squares loss of a CP model:
 *   resid(m) = mhat(m) - x(m),  loss = 1/2 sum_m resid(m)^2.
 * Its gradient with respect to U^(n) is the mode-n MTTKRP with the residuals
 * in place of the values (call oracle_mttkrp_* with vals = resid).
 */
int oracle_cp_loss(int N, const uint64_t *dims, uint64_t M, const uint32_t *inds, const double *vals,
                   const double *const *factors, int R, int ldf, double *resid, double *loss)
{
    int rc = oracle_cp_sample(N, dims, M, inds, factors, R, ldf, resid);
    if (rc) return rc;
    double acc = 0.0;
    for (uint64_t m = 0; m < M; ++m) {
        resid[m] -= vals[m];
        acc += resid[m] * resid[m];
    }
    *loss = 0.5 * acc;
    return 0;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

/*
 * General element-wise operation of two sparse tensors of the same order
 * (Section 5.2, Alg. 2 and its text): both inputs arrive sorted
 * lexicographically (mode 0 most significant); two cursors walk them and
 * every coordinate present in either input is appended once, in order:
 *   op 0 (add): x + y, x alone, y alone;
 *   op 1 (sub): x - y, x alone, -y alone;
 *   op 2 (mul): x * y only where both hold the coordinate.
 * Repeated coordinates inside one input are summed first (the tensor is the
 * sum of its entries). inds_*: SoA [k*M + m]; the output holds at most
 * Mx + My entries (SoA stride cap). Returns the output count, or -1.
 */
static int lex_cmp(int N, const uint32_t *a, uint64_t sa, uint64_t ia, const uint32_t *b, uint64_t sb, uint64_t ib)
{
    for (int k = 0; k < N; ++k) {
        const uint32_t x = a[k * sa + ia], y = b[k * sb + ib];
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}

int64_t oracle_tew_merge(int N, int op, uint64_t Mx, const uint32_t *ix, const double *vx, uint64_t My,
                         const uint32_t *iy, const double *vy, uint64_t cap, uint32_t *iz, double *vz)
{
    if (N < 1 || N > 16 || op < 0 || op > 2 || cap < Mx + My) return -1;
    uint64_t a = 0, b = 0, nz = 0;
    while (a < Mx || b < My) {
        int c;
        if (a >= Mx) c = 1;
        else if (b >= My) c = -1;
        else c = lex_cmp(N, ix, Mx, a, iy, My, b);
        const uint32_t *src = c <= 0 ? ix : iy;
        const uint64_t ss = c <= 0 ? Mx : My, is = c <= 0 ? a : b;
        double sx = 0.0, sy = 0.0;
        int hx = 0, hy = 0;
        if (c <= 0) {  /* the run of this coordinate in X */
            const uint64_t a0 = a;
            while (a < Mx && lex_cmp(N, ix, Mx, a, ix, Mx, a0) == 0) sx += vx[a++];
            hx = 1;
        }
        if (c >= 0) {  /* and in Y */
            const uint64_t b0 = b;
            while (b < My && lex_cmp(N, iy, My, b, iy, My, b0) == 0) sy += vy[b++];
            hy = 1;
        }
        double z;
        if (op == 0) z = sx + sy;
        else if (op == 1) z = sx - sy;
        else {
            if (!(hx && hy)) continue;
            z = sx * sy;
        }
        for (int k = 0; k < N; ++k) iz[k * cap + nz] = src[k * ss + is];
        vz[nz++] = z;
    }
    return (int64_t)nz;
}
