// CP-ALS around the MTTKRP (CP decomposition, Section 3.1.1: alternating least
// squares is one of the listed CPD methods, and MTTKRP is its bottleneck).
// For mode n, with M = MTTKRP_n(X; U) and V = Hadamard_{k != n} (U_k^T U_k):
//     U_n <- M V^{-1},  lambda_r = ||U_n[:, r]||_2,  U_n[:, r] /= lambda_r.
// The R x R work is tiny; these kernels are bandwidth-bound passes over the
// I_n x R matrices plus one small R x R inversion (Gauss-Jordan elimination)
// in a single workgroup.
// All sums run in a fixed order (deterministic).
#include "common.h"

namespace pasta {

constexpr int kAlsMaxRank = 64;
constexpr uint32_t kGramRows = 256;  // rows of U per partial Gram

// partial[b][r1][r2] = sum over rows i of block b of U[i, r1] * U[i, r2]
__global__ __launch_bounds__(256) void gram_partial_kernel(const float *__restrict__ U, uint64_t I, uint32_t ld,
                                                           uint32_t R, float *__restrict__ partial)
{
    __shared__ float tile[64][kAlsMaxRank + 1];
    const uint64_t r0 = (uint64_t)blockIdx.x * kGramRows;
    const uint64_t r1 = r0 + kGramRows < I ? r0 + kGramRows : I;
    const uint32_t RR = R * R;
    float acc[kAlsMaxRank * kAlsMaxRank / 256];
#pragma unroll
    for (int t = 0; t < kAlsMaxRank * kAlsMaxRank / 256; ++t) acc[t] = 0.0f;
    for (uint64_t base = r0; base < r1; base += 64) {
        const uint32_t rows = (uint32_t)(r1 - base < 64 ? r1 - base : 64);
        for (uint32_t e = threadIdx.x; e < 64 * R; e += 256) {
            const uint32_t i = e / R, c = e % R;
            tile[i][c] = i < rows ? U[(base + i) * ld + c] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < kAlsMaxRank * kAlsMaxRank / 256; ++t) {
            const uint32_t p = threadIdx.x + 256u * t;
            if (p < RR) {
                const uint32_t a = p / R, b = p % R;
                float s = 0.0f;
                for (uint32_t i = 0; i < rows; ++i) s += tile[i][a] * tile[i][b];
                acc[t] += s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < kAlsMaxRank * kAlsMaxRank / 256; ++t) {
        const uint32_t p = threadIdx.x + 256u * t;
        if (p < RR) partial[(uint64_t)blockIdx.x * RR + p] = acc[t];
    }
}

// G[p] = sum_b partial[b][p]
__global__ void gram_finish_kernel(const float *__restrict__ partial, uint32_t nb, uint32_t RR, float *__restrict__ G)
{
    // eight interleaved running sums over the blocks, so eight loads are in
    // flight; added in a fixed order (deterministic)
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < RR; p += gridDim.x * blockDim.x) {
        float acc[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] = 0.0f;
        for (uint32_t b = 0; b < nb; b += 8) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                acc[k] += b + k < nb ? partial[(uint64_t)(b + k) * RR + p] : 0.0f;
        }
        G[p] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    }
}

// One workgroup: V = Hadamard of the Grams of every mode but n, then
// Vinv = V^{-1} by Gauss-Jordan elimination on [V | I] without pivoting (V is
// symmetric positive definite: its pivots are the Schur-complement diagonals,
// the squared diagonal of its Cholesky factor). Thread t works on columns
// t % 64 (+ 64) and rows t / 64 (+ 4k) of the augmented matrix in LDS, so no
// index needs a division. flag |= 1 if a pivot is not positive (V not
// numerically positive definite).
__global__ __launch_bounds__(256) void als_solve_kernel(const float *__restrict__ grams, uint32_t order,
                                                        uint32_t mode, uint32_t R, float *__restrict__ Vinv,
                                                        uint32_t *__restrict__ flag)
{
    __shared__ float A[kAlsMaxRank][2 * kAlsMaxRank + 1];
    __shared__ float F[kAlsMaxRank];
    const uint32_t RR = R * R, W2 = 2 * R, cl = threadIdx.x & 63, rb = threadIdx.x >> 6;
    for (uint32_t i = rb; i < R; i += 4)
        for (uint32_t c = cl; c < R; c += 64) {
            float v = 1.0f;
            for (uint32_t k = 0; k < order; ++k)
                if (k != mode) v *= grams[(uint64_t)k * RR + i * R + c];
            A[i][c] = v;
            A[i][R + c] = i == c ? 1.0f : 0.0f;
        }
    __syncthreads();
    for (uint32_t j = 0; j < R; ++j) {
        const float piv = A[j][j];  // read by every thread before row j changes
        if (threadIdx.x == 0 && !(piv > 0.0f)) atomicOr(flag, 1u);
        const float inv = piv > 0.0f ? 1.0f / piv : 1.0f;
        for (uint32_t i = threadIdx.x; i < R; i += blockDim.x) F[i] = A[i][j];
        __syncthreads();
        for (uint32_t c = threadIdx.x; c < W2; c += blockDim.x) A[j][c] *= inv;
        __syncthreads();
        for (uint32_t c = cl; c < W2; c += 64) {
            const float rj = A[j][c];
            for (uint32_t i = rb; i < R; i += 4)
                if (i != j) A[i][c] -= F[i] * rj;
        }
        __syncthreads();
    }
    for (uint32_t i = rb; i < R; i += 4)
        for (uint32_t c = cl; c < R; c += 64) Vinv[i * R + c] = A[i][R + c];
}

// U[i, :] = M[i, :] Vinv (row by row; Vinv staged in LDS)
__global__ __launch_bounds__(256) void als_update_kernel(const float *__restrict__ M, uint32_t ldm,
                                                         const float *__restrict__ Vinv, uint32_t R, uint64_t I,
                                                         float *__restrict__ U, uint32_t ldu)
{
    __shared__ float S[kAlsMaxRank * kAlsMaxRank];
    for (uint32_t p = threadIdx.x; p < R * R; p += blockDim.x) S[p] = Vinv[p];
    __syncthreads();
    const uint64_t total = I * R;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = e / R;
        const uint32_t c = (uint32_t)(e % R);
        const float *m = M + i * ldm;
        float s = 0.0f;
        for (uint32_t k = 0; k < R; ++k) s += m[k] * S[k * R + c];
        U[i * ldu + c] = s;
    }
}

// From the Gram matrix of the updated (unnormalised) U_n: lambda_r = sqrt(G[r][r]),
// and the Gram of the normalised columns, G[a][b] / (lambda_a lambda_b).
__global__ void gram_normalize_kernel(float *__restrict__ G, uint32_t R, float *__restrict__ lambda)
{
    __shared__ float l[kAlsMaxRank];
    for (uint32_t c = threadIdx.x; c < R; c += blockDim.x) {
        const float d = G[c * R + c];
        l[c] = d > 0.0f ? sqrtf(d) : 0.0f;
        lambda[c] = l[c];
    }
    __syncthreads();
    for (uint32_t p = threadIdx.x; p < R * R; p += blockDim.x) {
        const float la = l[p / R], lb = l[p % R];
        G[p] = (la > 0.0f && lb > 0.0f) ? G[p] / (la * lb) : 0.0f;
    }
}

__global__ void scale_cols_kernel(float *__restrict__ U, uint64_t I, uint32_t ld, uint32_t R,
                                  const float *__restrict__ lambda)
{
    const uint64_t total = I * R;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = e / R;
        const uint32_t c = (uint32_t)(e % R);
        const float l = lambda[c];
        U[i * ld + c] = l > 0.0f ? U[i * ld + c] / l : 0.0f;
    }
}

// partial[b] = sum over rows of block b of sum_r M[i, r] U[i, r] lambda[r]  (fp64 out)
__global__ __launch_bounds__(256) void inner_partial_kernel(const float *__restrict__ M, uint32_t ldm,
                                                            const float *__restrict__ U, uint32_t ldu,
                                                            const float *__restrict__ lambda, uint64_t I, uint32_t R,
                                                            double *__restrict__ partial)
{
    __shared__ double lds[4];
    const uint64_t r0 = (uint64_t)blockIdx.x * kGramRows;
    const uint64_t r1 = r0 + kGramRows < I ? r0 + kGramRows : I;
    double s = 0.0;
    for (uint64_t e = r0 * R + threadIdx.x; e < r1 * R; e += blockDim.x) {
        const uint64_t i = e / R;
        const uint32_t c = (uint32_t)(e % R);
        s += (double)(M[i * ldm + c] * U[i * ldu + c] * lambda[c]);
    }
    s = wave_sum_f64(s);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// fit = 1 - sqrt(max(0, |X|^2 + |model|^2 - 2 <X, model>)) / |X|, where
// |model|^2 = lambda^T (Hadamard_k G_k) lambda and <X, model> = sum of the inner partials.
__global__ __launch_bounds__(256) void fit_kernel(const float *__restrict__ grams, uint32_t order, uint32_t R,
                                                  const float *__restrict__ lambda, const double *__restrict__ inner,
                                                  uint32_t ninner, const double *__restrict__ xnorm2,
                                                  double *__restrict__ fit)
{
    __shared__ double lds[4];
    const uint32_t RR = R * R;
    double s = 0.0;
    for (uint32_t p = threadIdx.x; p < RR; p += blockDim.x) {
        double v = (double)lambda[p / R] * (double)lambda[p % R];
        for (uint32_t k = 0; k < order; ++k) v *= (double)grams[(uint64_t)k * RR + p];
        s += v;
    }
    double in = 0.0;
    for (uint32_t b = threadIdx.x; b < ninner; b += blockDim.x) in += inner[b];
    s = wave_sum_f64(s);
    in = wave_sum_f64(in);
    __shared__ double lds2[4];
    if ((threadIdx.x & 63) == 0) {
        lds[threadIdx.x >> 6] = s;
        lds2[threadIdx.x >> 6] = in;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double mn = (lds[0] + lds[1]) + (lds[2] + lds[3]);
        const double ip = (lds2[0] + lds2[1]) + (lds2[2] + lds2[3]);
        const double x2 = *xnorm2;
        const double r2 = x2 + mn - 2.0 * ip;
        *fit = x2 > 0.0 ? 1.0 - sqrt(r2 > 0.0 ? r2 : 0.0) / sqrt(x2) : 0.0;
    }
}

// partial[b] = sum of squares of the values of block b (fp64), grid-stride blocks of 256
__global__ __launch_bounds__(256) void sumsq_partial_kernel(const float *__restrict__ x, uint64_t n,
                                                            double *__restrict__ partial)
{
    // 16-byte loads when the array allows them, four in flight per thread
    // (interleaved running sums, added in a fixed order); the scalar tail goes
    // to the first thread
    __shared__ double lds[4];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const bool vec = ((uintptr_t)x % 16) == 0;
    const uint64_t n4 = vec ? n / 4 : 0;
    const float4 *x4 = reinterpret_cast<const float4 *>(x);
    for (uint64_t i = t0; i < n4; i += 4 * stride) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t q = i + (uint64_t)k * stride;
            const float4 v = q < n4 ? x4[q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            acc[k] += ((double)v.x * v.x + (double)v.y * v.y) + ((double)v.z * v.z + (double)v.w * v.w);
        }
    }
    for (uint64_t i = 4 * n4 + t0; i < n; i += stride) acc[0] += (double)x[i] * (double)x[i];
    double s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    s = wave_sum_f64(s);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

uint32_t gram_blocks(uint64_t I) { return (uint32_t)((I + kGramRows - 1) / kGramRows); }

hipError_t launch_gram(const float *U, uint64_t I, uint32_t ld, uint32_t R, float *partial, float *G, hipStream_t st)
{
    const uint32_t nb = gram_blocks(I);
    gram_partial_kernel<<<nb, 256, 0, st>>>(U, I, ld, R, partial);
    gram_finish_kernel<<<(R * R + 255) / 256, 256, 0, st>>>(partial, nb, R * R, G);
    return hipGetLastError();
}

hipError_t launch_als_solve(const float *grams, uint32_t order, uint32_t mode, uint32_t R, float *Vinv,
                            uint32_t *flag, hipStream_t st)
{
    als_solve_kernel<<<1, 256, 0, st>>>(grams, order, mode, R, Vinv, flag);
    return hipGetLastError();
}

hipError_t launch_als_update(const float *M, uint32_t ldm, const float *Vinv, uint32_t R, uint64_t I, float *U,
                             uint32_t ldu, hipStream_t st)
{
    const uint64_t total = I * R;
    unsigned g = (unsigned)((total + 255) / 256);
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    als_update_kernel<<<g, 256, 0, st>>>(M, ldm, Vinv, R, I, U, ldu);
    return hipGetLastError();
}

hipError_t launch_normalize(float *U, uint64_t I, uint32_t ld, uint32_t R, float *partial, float *G, float *lambda,
                            hipStream_t st)
{
    hipError_t e = launch_gram(U, I, ld, R, partial, G, st);
    if (e != hipSuccess) return e;
    gram_normalize_kernel<<<1, 256, 0, st>>>(G, R, lambda);
    const uint64_t total = I * R;
    unsigned g = (unsigned)((total + 255) / 256);
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    scale_cols_kernel<<<g, 256, 0, st>>>(U, I, ld, R, lambda);
    return hipGetLastError();
}

hipError_t launch_fit(const float *M, uint32_t ldm, const float *U, uint32_t ldu, const float *lambda, uint64_t I,
                      uint32_t R, const float *grams, uint32_t order, double *inner_partial,
                      const double *xnorm2, double *fit, hipStream_t st)
{
    const uint32_t nb = gram_blocks(I);
    inner_partial_kernel<<<nb, 256, 0, st>>>(M, ldm, U, ldu, lambda, I, R, inner_partial);
    fit_kernel<<<1, 256, 0, st>>>(grams, order, R, lambda, inner_partial, nb, xnorm2, fit);
    return hipGetLastError();
}

hipError_t launch_sumsq(const float *x, uint64_t n, double *partial, uint32_t nparts, double *out, hipStream_t st)
{
    sumsq_partial_kernel<<<nparts, 256, 0, st>>>(x, n, partial);
    return launch_sum_f64(partial, nparts, out, st);
}

}  // namespace pasta
