// Mode-n fibers and the TTV kernel for gfx950.
//
// A mode-n fiber fixes every index but i_n (Section 3). Algs. 4 (TTV) and 5
// (TTM) first find the fibers that hold nonzeros and where each begins (nfibs
// and fptr), then reduce over each fiber. Here the nonzeros are already sorted
// so that every fiber is one contiguous run; these kernels mark the run heads,
// number the fibers and record their coordinates, and compute TTV over the
// runs with a segmented reduction that needs no atomics.
#include "fibers.h"

namespace pasta {
namespace {

unsigned grid_of(uint64_t n, unsigned threads, unsigned cap = 16384)
{
    uint64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

__global__ __launch_bounds__(256) void fiber_heads_kernel(const FiberInds in, uint64_t nnz, uint32_t *__restrict__ head)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += stride) {
        uint32_t h = p == 0;
        if (!h)
            for (uint32_t q = 0; q < in.count; ++q) h |= in.p[q][p] != in.p[q][p - 1];
        head[p] = h;
    }
}

__global__ __launch_bounds__(256) void fiber_compact_kernel(const FiberInds in, uint64_t nnz,
                                                            const uint32_t *__restrict__ head,
                                                            const uint32_t *__restrict__ excl,
                                                            uint32_t *__restrict__ fid, uint32_t *__restrict__ fptr,
                                                            const FiberCoords coords, uint32_t *__restrict__ nfibs)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += stride) {
        const uint32_t h = head[p];
        const uint32_t f = excl[p] + h - 1u;  // inclusive count of heads, minus one
        fid[p] = f;
        if (h) {
            fptr[f] = (uint32_t)p;
            for (uint32_t q = 0; q < in.count; ++q) coords.p[q][f] = in.p[q][p];
        }
        if (p == nnz - 1) {
            fptr[f + 1] = (uint32_t)nnz;
            *nfibs = f + 1;
        }
    }
}

__global__ __launch_bounds__(256) void count_keys_kernel(const uint32_t *__restrict__ rowptr, uint32_t n,
                                                         uint64_t nnz, uint32_t *__restrict__ keys)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        keys[i] = (uint32_t)(nnz - (uint64_t)(rowptr[i + 1] - rowptr[i]));
}

__global__ __launch_bounds__(256) void invert_perm_kernel(const uint32_t *__restrict__ perm, uint32_t n,
                                                          uint32_t *__restrict__ inv)
{
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (uint64_t)gridDim.x * blockDim.x)
        inv[perm[j]] = (uint32_t)j;
}

template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(const T *__restrict__ table, const uint32_t *__restrict__ idx,
                                                     uint64_t n, T *__restrict__ out)
{
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (uint64_t)gridDim.x * blockDim.x)
        out[p] = table[idx[p]];
}

// ---------------------------------------------------------------------------
// TTV over the fiber-ordered stream. Lane l of the wave takes nonzeros
// 4l .. 4l+3 of a 256-nonzero tile (one 16-byte load per stream, so a tile is
// read with fully coalesced loads), multiplies each value by its gathered
// vector entry and sums runs of equal fiber id in registers. A fiber that
// starts and ends inside a lane's four entries is complete and stored there.
// The lanes' edge runs are joined by a segmented scan across the wave; the
// run still open at the end of the tile is carried into the next tile as a
// wave-uniform (fiber, sum) pair. At the chunk's two ends, a fiber that
// continues into a neighbouring chunk leaves its partial in a slot instead.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void ttv_seg_kernel(const uint32_t *__restrict__ fid,
                                                      const uint32_t *__restrict__ idx,
                                                      const float *__restrict__ vals, const float *__restrict__ v,
                                                      float *__restrict__ out, float *__restrict__ part, uint64_t nnz,
                                                      uint32_t nchunks)
{
    const int lane = threadIdx.x & 63;
    const uint32_t chunk = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (chunk >= nchunks) return;  // whole wave leaves together
    const uint64_t c0 = (uint64_t)chunk * kTtvChunk;
    const uint64_t c1 = c0 + kTtvChunk < nnz ? c0 + kTtvChunk : nnz;
    const uint32_t cfirst = fid[c0], clast = fid[c1 - 1];
    const bool before = c0 > 0 && fid[c0 - 1] == cfirst;
    const bool after = c1 < nnz && fid[c1] == clast;
    auto emit = [&](uint32_t r, float s) {
        if (r == cfirst && before)
            part[2 * (uint64_t)chunk] = s;
        else if (r == clast && after)
            part[2 * (uint64_t)chunk + 1] = s;
        else
            out[r] = s;
    };

    uint32_t carry_row = kNoRow;  // open fiber at the end of the previous tile (wave-uniform)
    float carry = 0.0f;
    struct Tile {
        uint32_t f[4], ix[4];
        float x[4];
        int nv;
    };
    auto load_tile = [&](uint64_t base, Tile &T) {
        const uint64_t q = base + 4u * (uint64_t)lane;
        T.nv = q < c1 ? (c1 - q < 4 ? (int)(c1 - q) : 4) : 0;
        if (T.nv == 4) {
            const uint4 tf = *reinterpret_cast<const uint4 *>(fid + q);
            const uint4 ti = *reinterpret_cast<const uint4 *>(idx + q);
            const float4 tx = *reinterpret_cast<const float4 *>(vals + q);
            T.f[0] = tf.x; T.f[1] = tf.y; T.f[2] = tf.z; T.f[3] = tf.w;
            T.ix[0] = ti.x; T.ix[1] = ti.y; T.ix[2] = ti.z; T.ix[3] = ti.w;
            T.x[0] = tx.x; T.x[1] = tx.y; T.x[2] = tx.z; T.x[3] = tx.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool on = e < T.nv;
                T.f[e] = on ? fid[q + e] : kNoRow;
                T.ix[e] = on ? idx[q + e] : 0u;
                T.x[e] = on ? vals[q + e] : 0.0f;
            }
        }
    };
    // One tile: the gathers for T go out first, then the next tile's loads
    // (so their latency overlaps this tile's work), then the reduction.
    auto tile = [&](uint64_t base, Tile &T, Tile &next) {
        float w[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = v[T.ix[e]];
        __builtin_amdgcn_sched_barrier(0);
        if (base + kTtvTile < c1) load_tile(base + kTtvTile, next);
        const int nv = T.nv;
        float p[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) p[e] = T.x[e] * w[e];

        // runs inside the lane
        uint32_t cur = kNoRow, hrow = kNoRow;
        float acc = 0.0f, head = 0.0f;
        bool multi = false;  // the lane has closed its first run
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (e < nv) {
                if (T.f[e] != cur) {
                    if (cur != kNoRow) {
                        if (!multi) {
                            head = acc;
                            hrow = cur;
                            multi = true;
                        } else {
                            emit(cur, acc);  // a whole fiber inside the lane
                        }
                    }
                    cur = T.f[e];
                    acc = 0.0f;
                }
                acc += p[e];
            }
        }

        // join the lanes' edge runs; lane 0 continues the tile carry
        const uint32_t first = multi ? hrow : cur;
        uint32_t prev_last = (uint32_t)__shfl_up((int)cur, 1);
        if (lane == 0) prev_last = carry_row;
        const bool cont = cur != kNoRow && first == prev_last;
        bool seg_start = !(cont && !multi);
        float c = acc;
        if (lane == 0 && cont && !multi) c += carry;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const bool ps = __shfl_up((int)seg_start, d) != 0;
            const float pv = __shfl_up(c, d);
            if (lane >= d && !seg_start) c += pv;
            if (lane >= d) seg_start = seg_start || ps;
        }
        float prev_c = __shfl_up(c, 1);
        if (lane == 0) prev_c = carry;
        const bool next_cont = __shfl_down((int)cont, 1) != 0;
        const int lastlane = (int)((c1 - base - 1) / 4 < 63 ? (c1 - base - 1) / 4 : 63);

        if (lane == 0 && carry_row != kNoRow && !cont) emit(carry_row, carry);  // it ended with the last tile
        if (multi) emit(hrow, cont ? head + prev_c : head);
        if (cur != kNoRow && lane < lastlane && !next_cont) emit(cur, c);
        carry_row = (uint32_t)__shfl((int)cur, lastlane);
        carry = __shfl(c, lastlane);
    };
    // tiles with the two buffers' roles alternating (no register copies of loads in flight)
    static_assert(kTtvTiles % 2 == 0, "tiles come in pairs");
    Tile ta, tb;
    load_tile(c0, ta);
#pragma unroll
    for (uint32_t t = 0; t < kTtvTiles; t += 2) {
        const uint64_t base = c0 + (uint64_t)t * kTtvTile;
        if (base >= c1) break;
        tile(base, ta, tb);
        if (base + kTtvTile >= c1) break;
        tile(base + kTtvTile, tb, ta);
    }
    if (lane == 0 && carry_row != kNoRow) emit(carry_row, carry);
}

}  // namespace

hipError_t launch_fiber_heads(const FiberInds &in, uint64_t nnz, uint32_t *head, hipStream_t st)
{
    if (nnz == 0) return hipSuccess;
    fiber_heads_kernel<<<grid_of(nnz, 256), 256, 0, st>>>(in, nnz, head);
    return hipGetLastError();
}

hipError_t launch_fiber_compact(const FiberInds &in, uint64_t nnz, const uint32_t *head, const uint32_t *excl,
                                uint32_t *fid, uint32_t *fptr, const FiberCoords &coords, uint32_t *nfibs,
                                hipStream_t st)
{
    if (nnz == 0) return hipSuccess;
    fiber_compact_kernel<<<grid_of(nnz, 256), 256, 0, st>>>(in, nnz, head, excl, fid, fptr, coords, nfibs);
    return hipGetLastError();
}

hipError_t launch_count_keys(const uint32_t *rowptr, uint32_t n, uint64_t nnz, uint32_t *keys, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    count_keys_kernel<<<grid_of(n, 256), 256, 0, st>>>(rowptr, n, nnz, keys);
    return hipGetLastError();
}

hipError_t launch_invert_perm(const uint32_t *perm, uint32_t n, uint32_t *inv, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    invert_perm_kernel<<<grid_of(n, 256), 256, 0, st>>>(perm, n, inv);
    return hipGetLastError();
}

hipError_t launch_gather_u32(const uint32_t *table, const uint32_t *idx, uint64_t n, uint32_t *out, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    gather_kernel<uint32_t><<<grid_of(n, 256), 256, 0, st>>>(table, idx, n, out);
    return hipGetLastError();
}

hipError_t launch_gather_f32(const float *table, const uint32_t *idx, uint64_t n, float *out, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    gather_kernel<float><<<grid_of(n, 256), 256, 0, st>>>(table, idx, n, out);
    return hipGetLastError();
}

hipError_t launch_ttv(const uint32_t *fid, const uint32_t *idx, const float *vals, const float *v, float *out,
                      float *part, uint64_t nnz, uint32_t nchunks, hipStream_t st)
{
    if (nnz == 0 || nchunks == 0) return hipSuccess;
    ttv_seg_kernel<<<(nchunks + 3) / 4, 256, 0, st>>>(fid, idx, vals, v, out, part, nnz, nchunks);
    return hipGetLastError();
}

}  // namespace pasta
