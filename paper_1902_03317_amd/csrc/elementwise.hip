// Element-wise (TEW) and tensor-scalar (TS) kernels for gfx950.
//
// Same-pattern element-wise operations (Section 4.1, Alg. 1) and the
// tensor-scalar operations (Section 4.2, Alg. 3) are one pass over the value
// arrays: 16-byte loads and stores in a grid-stride loop, so they run at
// streaming bandwidth. The general element-wise operation (Alg. 2) works on
// the concatenation of the two inputs sorted lexicographically: runs of equal
// coordinates are reduced (each input's entries summed, then combined) and the
// surviving runs compacted into the output in order.
#include "elementwise.h"

namespace pasta {
namespace {

unsigned grid_of(uint64_t n, unsigned threads, unsigned cap = 16384)
{
    uint64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

template <int OP>
__device__ __forceinline__ float ew(float a, float b)
{
    if constexpr (OP == kEwAdd) return a + b;
    else if constexpr (OP == kEwSub) return a - b;
    else if constexpr (OP == kEwMul) return a * b;
    else return a / b;
}

// z = x op y (y == nullptr: z = x op s), vector body and scalar tail.
template <int OP>
__global__ __launch_bounds__(256) void ew_vec_kernel(const float *__restrict__ x, const float *__restrict__ y, float s,
                                                     float *__restrict__ z, uint64_t n)
{
    const uint64_t n4 = n / 4;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = t0; i < n4; i += stride) {
        const float4 a = reinterpret_cast<const float4 *>(x)[i];
        const float4 b = y ? reinterpret_cast<const float4 *>(y)[i] : make_float4(s, s, s, s);
        float4 c;
        c.x = ew<OP>(a.x, b.x);
        c.y = ew<OP>(a.y, b.y);
        c.z = ew<OP>(a.z, b.z);
        c.w = ew<OP>(a.w, b.w);
        reinterpret_cast<float4 *>(z)[i] = c;
    }
    for (uint64_t i = 4 * n4 + t0; i < n; i += stride) z[i] = ew<OP>(x[i], y ? y[i] : s);
}

template <int OP>
__global__ __launch_bounds__(256) void ew_scalar_kernel(const float *__restrict__ x, const float *__restrict__ y,
                                                        float s, float *__restrict__ z, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        z[i] = ew<OP>(x[i], y ? y[i] : s);
}

// One thread per run head of the sorted concatenation: sum the run's entries
// from X (perm < nx) and from Y, combine them, and record whether the run
// survives (multiplication keeps only coordinates both inputs hold).
__global__ __launch_bounds__(256) void tew_runs_kernel(const uint32_t *__restrict__ head,
                                                       const uint32_t *__restrict__ run_of,
                                                       const uint32_t *__restrict__ perm,
                                                       const float *__restrict__ vals, uint64_t n, uint64_t nx,
                                                       int op, float *__restrict__ run_val,
                                                       uint32_t *__restrict__ run_pos,
                                                       uint32_t *__restrict__ run_keep)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        if (!head[p]) continue;
        float sx = 0.0f, sy = 0.0f;
        bool hx = false, hy = false;
        uint64_t q = p;
        do {
            if (perm[q] < nx) {
                sx = hx ? sx + vals[q] : vals[q];
                hx = true;
            } else {
                sy = hy ? sy + vals[q] : vals[q];
                hy = true;
            }
            ++q;
        } while (q < n && !head[q]);
        float zv;
        bool keep = true;
        if (op == kEwMul) {
            keep = hx && hy;
            zv = sx * sy;
        } else if (hx && hy) {
            zv = op == kEwAdd ? sx + sy : sx - sy;
        } else {
            zv = hx ? sx : (op == kEwSub ? -sy : sy);
        }
        const uint32_t r = run_of[p] + head[p] - 1u;  // inclusive count of heads, minus one
        run_val[r] = zv;
        run_pos[r] = (uint32_t)p;
        run_keep[r] = keep ? 1u : 0u;
    }
}

// Surviving runs to the output, in order.
__global__ __launch_bounds__(256) void tew_emit_kernel(const TewInds sorted, uint32_t order,
                                                       const uint32_t *__restrict__ run_pos,
                                                       const float *__restrict__ run_val,
                                                       const uint32_t *__restrict__ run_keep,
                                                       const uint32_t *__restrict__ out_of, uint64_t nruns,
                                                       const TewOut out, float *__restrict__ vals_out,
                                                       uint32_t *__restrict__ count)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nruns; r += stride) {
        const uint32_t o = out_of[r];
        if (run_keep[r]) {
            const uint32_t p = run_pos[r];
            for (uint32_t k = 0; k < order; ++k) out.p[k][o] = sorted.p[k][p];
            vals_out[o] = run_val[r];
        }
        if (r == nruns - 1) *count = o + run_keep[r];
    }
}

template <int OP>
hipError_t launch_ew_op(const float *x, const float *y, float s, float *z, uint64_t n, hipStream_t st)
{
    const bool al = ((uintptr_t)x % 16 == 0) && ((uintptr_t)z % 16 == 0) && (!y || (uintptr_t)y % 16 == 0);
    if (al)
        ew_vec_kernel<OP><<<grid_of(n / 4 + 1, 256), 256, 0, st>>>(x, y, s, z, n);
    else
        ew_scalar_kernel<OP><<<grid_of(n, 256), 256, 0, st>>>(x, y, s, z, n);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ew(int op, const float *x, const float *y, float s, float *z, uint64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    switch (op) {
    case kEwAdd: return launch_ew_op<kEwAdd>(x, y, s, z, n, st);
    case kEwSub: return launch_ew_op<kEwSub>(x, y, s, z, n, st);
    case kEwMul: return launch_ew_op<kEwMul>(x, y, s, z, n, st);
    case kEwDiv: return launch_ew_op<kEwDiv>(x, y, s, z, n, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tew_runs(const uint32_t *head, const uint32_t *run_of, const uint32_t *perm, const float *vals,
                           uint64_t n, uint64_t nx, int op, float *run_val, uint32_t *run_pos, uint32_t *run_keep,
                           hipStream_t st)
{
    if (n == 0) return hipSuccess;
    tew_runs_kernel<<<grid_of(n, 256), 256, 0, st>>>(head, run_of, perm, vals, n, nx, op, run_val, run_pos,
                                                      run_keep);
    return hipGetLastError();
}

hipError_t launch_tew_emit(const TewInds &sorted, uint32_t order, const uint32_t *run_pos, const float *run_val,
                           const uint32_t *run_keep, const uint32_t *out_of, uint64_t nruns, const TewOut &out,
                           float *vals_out, uint32_t *count, hipStream_t st)
{
    if (nruns == 0) return hipSuccess;
    tew_emit_kernel<<<grid_of(nruns, 256), 256, 0, st>>>(sorted, order, run_pos, run_val, run_keep, out_of, nruns,
                                                         out, vals_out, count);
    return hipGetLastError();
}

}  // namespace pasta
