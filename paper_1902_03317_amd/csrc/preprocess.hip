// Preprocessing of a COO tensor for gfx950 and the order-independent kernels:
// index check, stable LSD radix sort by one mode, SoA permutation, row
// offsets, the split-row fixup of MTTKRP, fp64 reductions and the bf16 cast.
//
// The suite preprocesses its tensors before the TTV/TTM kernels (the fiber
// pointers of Algs. 4-5) and sorts them lexicographically for TEW (Section
// 5.2). Here every mode gets its own copy of the nonzeros sorted stably by
// that mode's index, so the MTTKRP of that mode reads a stream in which each
// output row is one contiguous run.
#include "common.h"

namespace pasta {

// ---------------------------------------------------------------------------
// Fill / identity / index check
// ---------------------------------------------------------------------------
__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static unsigned grid_for(uint64_t n, unsigned threads, unsigned cap = 8192)
{
    uint64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    fill_u32_kernel<<<grid_for(n, 256), 256, 0, st>>>(p, v, n);
    return hipGetLastError();
}

struct IndexPtrs {
    const uint32_t *p[kMaxOrder];
    uint64_t dim[kMaxOrder];
};

// flag |= 1 if any coordinate is outside its dimension. Each thread checks
// four positions of the grid-stride walk at a time, their loads issued together.
__global__ void validate_kernel(IndexPtrs ip, uint32_t order, uint64_t nnz, uint32_t *flag)
{
    uint32_t bad = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; m < nnz; m += 4 * stride) {
        for (uint32_t k = 0; k < order; ++k) {
            uint32_t v[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint64_t q = m + (uint64_t)t * stride;
                v[t] = q < nnz ? ip.p[k][q] : 0u;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) bad |= (uint64_t)v[t] >= ip.dim[k];
        }
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

hipError_t launch_validate(const uint32_t *const *inds, const uint64_t *dims, uint32_t order, uint64_t nnz,
                           uint32_t *flag, hipStream_t st)
{
    if (nnz == 0) return hipSuccess;
    IndexPtrs ip{};
    for (uint32_t k = 0; k < order; ++k) {
        ip.p[k] = inds[k];
        ip.dim[k] = dims[k];
    }
    validate_kernel<<<grid_for(nnz, 256), 256, 0, st>>>(ip, order, nnz, flag);
    return hipGetLastError();
}

__global__ void identity_sort_kernel(const uint32_t *keys, uint64_t n, uint32_t *keys_out, uint32_t *perm_out)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        keys_out[i] = keys[i];
        perm_out[i] = (uint32_t)i;
    }
}

hipError_t launch_identity_sort(const uint32_t *keys, uint64_t n, uint32_t *keys_out, uint32_t *perm_out,
                                hipStream_t st)
{
    if (n == 0) return hipSuccess;
    identity_sort_kernel<<<grid_for(n, 256), 256, 0, st>>>(keys, n, keys_out, perm_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exclusive scan of uint32 counts (three kernels: tile sums, one-block scan
// of the tile sums, tile scan plus offset).
// ---------------------------------------------------------------------------
constexpr uint32_t kScanThreads = 256;
constexpr uint32_t kScanItems = 16;
constexpr uint32_t kScanTile = kScanThreads * kScanItems;

uint64_t scan_partials_count(uint64_t n) { return (n + kScanTile - 1) / kScanTile; }

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(v, d);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread over a 256-thread block; returns the
// block total through *total.
__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t *lds4, uint32_t *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan_u32(v, lane);
    if (lane == 63) lds4[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t s = lds4[w];
        before += w < wave ? s : 0u;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

__global__ __launch_bounds__(256) void scan_reduce_kernel(const uint32_t *in, uint64_t n, uint32_t *partials)
{
    __shared__ uint32_t lds[4];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (uint32_t i = 0; i < kScanItems; ++i)
        if (base + i < n) s += in[base + i];
    uint32_t total;
    block_excl_scan_u32(s, lds, &total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void scan_partials_kernel(uint32_t *partials, uint64_t np)
{
    __shared__ uint32_t lds[4];
    uint32_t carry = 0;
    for (uint64_t base = 0; base < np; base += 256) {
        const uint64_t i = base + threadIdx.x;
        const uint32_t v = i < np ? partials[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_scan_u32(v, lds, &total);
        if (i < np) partials[i] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(256) void scan_apply_kernel(const uint32_t *in, uint32_t *out, uint64_t n,
                                                         const uint32_t *partials)
{
    __shared__ uint32_t lds[4];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (uint32_t i = 0; i < kScanItems; ++i) {
        v[i] = base + i < n ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t total;
    uint32_t run = partials[blockIdx.x] + block_excl_scan_u32(s, lds, &total);
#pragma unroll
    for (uint32_t i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *partials, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const uint64_t np = scan_partials_count(n);
    scan_reduce_kernel<<<(unsigned)np, kScanThreads, 0, st>>>(in, n, partials);
    scan_partials_kernel<<<1, 256, 0, st>>>(partials, np);
    scan_apply_kernel<<<(unsigned)np, kScanThreads, 0, st>>>(in, out, n, partials);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One pass of a stable LSD radix sort over 8-bit digits.
//   hist:    per tile, the count of every digit, stored digit-major
//            (hist[d * ntiles + t]) so that its exclusive scan is the first
//            output position of digit d from tile t;
//   scatter: tile t walks its keys in order, 256 at a time; a key's place is
//            the scanned offset of its digit plus the number of equal digits
//            before it in the tile (wave ballots + per-wave counts in LDS),
//            which keeps equal keys in input order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void radix_hist_kernel(const uint32_t *__restrict__ keys, uint64_t n, int shift,
                                                         uint32_t *__restrict__ hist, uint32_t ntiles)
{
    __shared__ uint32_t cnt[4][kRadix];
    const int wave = threadIdx.x >> 6;
    for (uint32_t d = threadIdx.x; d < 4 * kRadix; d += 256) (&cnt[0][0])[d] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    uint32_t key[kSortItems];  // every load goes out before the first count
#pragma unroll
    for (uint32_t i = 0; i < kSortItems; ++i) {
        const uint64_t idx = base + (uint64_t)i * kSortThreads + threadIdx.x;
        key[i] = idx < n ? keys[idx] : 0u;
    }
#pragma unroll
    for (uint32_t i = 0; i < kSortItems; ++i) {
        const uint64_t idx = base + (uint64_t)i * kSortThreads + threadIdx.x;
        if (idx < n) atomicAdd(&cnt[wave][(key[i] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < kRadix; d += 256)
        hist[(uint64_t)d * ntiles + blockIdx.x] = cnt[0][d] + cnt[1][d] + cnt[2][d] + cnt[3][d];
}

hipError_t launch_radix_hist(const uint32_t *keys, uint64_t n, int shift, uint32_t *hist, uint32_t ntiles,
                             hipStream_t st)
{
    radix_hist_kernel<<<ntiles, kSortThreads, 0, st>>>(keys, n, shift, hist, ntiles);
    return hipGetLastError();
}

// The scatter moves the key and every payload array (the permutation, the
// other modes' indices and the values) together, so the last pass writes the
// sorted SoA copy directly and nothing is gathered afterwards. Writes are
// staged in LDS: each key's place inside the tile (digit start within the
// tile + equal digits before it) is found first, the tile is laid out in LDS
// in that order, and then each digit's run is written to its global place as
// one contiguous range, so global writes are coalesced.
//
// Wave w of the block takes the contiguous quarter w of the tile and ranks its
// keys alone (ballots per 64 keys and a wave-private running count per digit),
// so ranking needs no block barrier; the waves' counts are then turned into
// per-wave digit offsets, which keeps equal digits in input order (stable).
// Payload arrays go through LDS one at a time, each one's loads issued while
// the previous one is being written.
__global__ __launch_bounds__(256) void radix_scatter_kernel(const uint32_t *__restrict__ keys_in, uint64_t n,
                                                            int shift, const uint32_t *__restrict__ offsets,
                                                            uint32_t ntiles, uint32_t *__restrict__ keys_out,
                                                            SortPayload pl)
{
    constexpr uint32_t kPer = kSortTile / kSortThreads;  // keys per lane (rounds of 64 per wave)
    constexpr uint32_t kQuarter = kSortTile / 4;         // keys per wave
    __shared__ uint32_t lstart[kRadix];                  // first slot of each digit inside the tile
    __shared__ uint32_t gstart[kRadix];                  // its first place in the output
    __shared__ uint32_t wc[4][kRadix];                   // per-wave digit counts, then per-wave offsets
    __shared__ uint32_t s_key[kSortTile];
    __shared__ uint32_t s_val[kSortTile];
    __shared__ uint32_t lds4[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // neighbouring tiles fill neighbouring pieces of each digit's output run:
    // on one XCD, their partial cache lines meet in the same L2
    const uint32_t tile = xcd_contiguous(blockIdx.x, ntiles);
    const uint64_t base = (uint64_t)tile * kSortTile;
    const uint32_t tile_n = (uint32_t)(n - base < kSortTile ? n - base : kSortTile);
    const uint32_t wbase = (uint32_t)wave * kQuarter + (uint32_t)lane;  // + 64 * r: this lane's r-th key

    // keys first, then the first payload array (loads return in order)
    uint32_t key[kPer], pv[kPer];
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
        const uint32_t li = wbase + 64u * r;
        key[r] = li < tile_n ? keys_in[base + li] : 0u;
    }
    const uint32_t *src0 = pl.count > 0 ? pl.in[0] : nullptr;
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
        const uint32_t li = wbase + 64u * r;
        pv[r] = li < tile_n ? (src0 ? src0[base + li] : (uint32_t)(base + li)) : 0u;
    }
    // this tile's digit counts from the scanned histogram (digit-major, exclusive)
    {
        const uint32_t d = threadIdx.x;
        const uint64_t j = (uint64_t)d * ntiles + tile;
        const uint64_t last = (uint64_t)kRadix * ntiles - 1;
        const uint32_t g0 = offsets[j];
        const uint32_t cnt = (j < last ? offsets[j + 1] : (uint32_t)n) - g0;
        gstart[d] = g0;
        uint32_t total;
        lstart[d] = block_excl_scan_u32(cnt, lds4, &total);
        wc[0][d] = wc[1][d] = wc[2][d] = wc[3][d] = 0;
    }
    __syncthreads();

    // rank inside the wave: equal digits before this key in the wave's quarter
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t rk[kPer];
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
        const bool on = wbase + 64u * r < tile_n;
        const uint32_t d = on ? ((key[r] >> shift) & (kRadix - 1)) : kRadix;  // idle lanes: digit kRadix
        uint64_t peers = ~0ull;
#pragma unroll
        for (int b = 0; b <= kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const uint32_t da = d & (kRadix - 1);                // an in-range address for idle lanes too
        const uint32_t before = on ? wc[wave][da] : 0u;      // read by every lane before the leader writes
        const uint32_t within = __popcll(peers & lt_mask);
        if (on && within == 0) wc[wave][da] = before + (uint32_t)__popcll(peers);
        rk[r] = before + within;
    }
    __syncthreads();
    // per-wave offsets of each digit (waves in tile order)
    {
        const uint32_t d = threadIdx.x;
        uint32_t a = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint32_t t = wc[w][d];
            wc[w][d] = a;
            a += t;
        }
    }
    __syncthreads();
    uint32_t lpos[kPer];
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
        lpos[r] = 0;
        if (wbase + 64u * r < tile_n) {
            const uint32_t d = (key[r] >> shift) & (kRadix - 1);
            lpos[r] = lstart[d] + wc[wave][d] + rk[r];
            s_key[lpos[r]] = key[r];
        }
    }
    __syncthreads();
    // keys, in tile order: slot i of digit d goes to gstart[d] + (i - lstart[d])
    for (uint32_t i = threadIdx.x; i < tile_n; i += kSortThreads) {
        const uint32_t k = s_key[i];
        const uint32_t d = (k >> shift) & (kRadix - 1);
        keys_out[gstart[d] + (i - lstart[d])] = k;
    }
    for (int k = 0; k < pl.count; ++k) {
        uint32_t nv[kPer];
        if (k + 1 < pl.count) {  // the next array's loads go out before this one is written
            const uint32_t *src = pl.in[k + 1];
#pragma unroll
            for (uint32_t r = 0; r < kPer; ++r) {
                const uint32_t li = wbase + 64u * r;
                nv[r] = li < tile_n ? src[base + li] : 0u;
            }
        }
#pragma unroll
        for (uint32_t r = 0; r < kPer; ++r)
            if (wbase + 64u * r < tile_n) s_val[lpos[r]] = pv[r];
        __syncthreads();
        uint32_t *dst = pl.out[k];
        for (uint32_t i = threadIdx.x; i < tile_n; i += kSortThreads) {
            const uint32_t d = (s_key[i] >> shift) & (kRadix - 1);
            dst[gstart[d] + (i - lstart[d])] = s_val[i];
        }
        __syncthreads();
        if (k + 1 < pl.count) {
#pragma unroll
            for (uint32_t r = 0; r < kPer; ++r) pv[r] = nv[r];
        }
    }
}

hipError_t launch_radix_scatter(const uint32_t *keys_in, uint64_t n, int shift, const uint32_t *offsets,
                                uint32_t ntiles, uint32_t *keys_out, const SortPayload &pl, hipStream_t st)
{
    radix_scatter_kernel<<<ntiles, kSortThreads, 0, st>>>(keys_in, n, shift, offsets, ntiles, keys_out, pl);
    return hipGetLastError();
}

// Copy a key array and its payload unchanged (the stable order of a mode of size 1).
__global__ void copy_payload_kernel(const uint32_t *__restrict__ keys_in, uint64_t n, uint32_t *__restrict__ keys_out,
                                    SortPayload pl)
{
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (uint64_t)gridDim.x * blockDim.x) {
        keys_out[p] = keys_in[p];
        pl.out[0][p] = pl.in[0] ? pl.in[0][p] : (uint32_t)p;
        for (int k = 1; k < pl.count; ++k) pl.out[k][p] = pl.in[k][p];
    }
}

hipError_t launch_copy_payload(const uint32_t *keys_in, uint64_t n, uint32_t *keys_out, const SortPayload &pl,
                               hipStream_t st)
{
    if (n == 0) return hipSuccess;
    copy_payload_kernel<<<grid_for(n, 256), 256, 0, st>>>(keys_in, n, keys_out, pl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gather every other mode's index and the value into mode order.
// ---------------------------------------------------------------------------
struct PermPtrs {
    const uint32_t *in[kMaxOrder];
    uint32_t *out[kMaxOrder];
};

__global__ void permute_kernel(PermPtrs pp, uint32_t order, uint32_t mode, uint64_t n,
                               const uint32_t *__restrict__ perm, const float *__restrict__ vals_in,
                               float *__restrict__ vals_out)
{
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t q = perm[p];
        for (uint32_t k = 0; k < order; ++k)
            if (k != mode) pp.out[k][p] = pp.in[k][q];
        vals_out[p] = vals_in[q];
    }
}

hipError_t launch_permute(uint32_t order, uint32_t mode, uint64_t n, const uint32_t *perm,
                          const uint32_t *const *inds_in, const float *vals_in, uint32_t *const *inds_out,
                          float *vals_out, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    PermPtrs pp{};
    for (uint32_t k = 0; k < order; ++k) {
        pp.in[k] = inds_in[k];
        pp.out[k] = inds_out[k];
    }
    permute_kernel<<<grid_for(n, 256, 16384), 256, 0, st>>>(pp, order, mode, n, perm, vals_in, vals_out);
    return hipGetLastError();
}

// rowptr[i] = first position p with sorted_rows[p] >= i (binary search), i = 0..nrows.
__global__ void rowptr_kernel(const uint32_t *__restrict__ rows, uint64_t n, uint32_t nrows,
                              uint32_t *__restrict__ rowptr)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= nrows;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t lo = 0, hi = n;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if ((uint64_t)rows[mid] < i)
                lo = mid + 1;
            else
                hi = mid;
        }
        rowptr[i] = (uint32_t)lo;
    }
}

hipError_t launch_rowptr(const uint32_t *sorted_rows, uint64_t n, uint32_t nrows, uint32_t *rowptr, hipStream_t st)
{
    rowptr_kernel<<<grid_for((uint64_t)nrows + 1, 256), 256, 0, st>>>(sorted_rows, n, nrows, rowptr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// MTTKRP fixup. The main kernel stores every row that lies inside one chunk
// of the mode-ordered stream. A row that crosses chunk boundaries left one
// partial per chunk: the first chunk c_a in its tail slot (2*c_a + 1), every
// later chunk c in its head slot (2*c). This kernel sums those partials in a
// fixed order (deterministic), scales by alpha and stores the row; rows with
// no nonzeros get zeros. Each wave takes 64 rows at a time and ballots the
// rows that need work: rows with few partials are summed one per lane group
// (G rows at once), rows with many partials by the whole wave, every group
// taking a strided share with several loads in flight.
// ---------------------------------------------------------------------------
constexpr uint32_t kFixupLight = 16;  // at most this many partials: one lane group per row
constexpr uint32_t kFixupBlock = 64;  // chunks per level-one block

// Level-one sums for rows that span very many chunks. A block of kFixupBlock
// consecutive chunks whose nonzeros all belong to the row that also holds the
// nonzero just before the block (two reads decide it, since the stream is
// sorted) has that row's whole-chunk partials in its head slots; their sum, in
// a fixed order, goes to blk[b]. The fixup then reads one value per such block
// instead of kFixupBlock.
template <int VEC, int L, bool STRIDED>
__global__ __launch_bounds__(256) void fixup_blocks_kernel(const uint32_t *__restrict__ row, uint64_t nnz,
                                                           const float *__restrict__ part, uint32_t ldp,
                                                           float *__restrict__ blk, uint64_t nblk, uint32_t rank,
                                                           uint64_t chunk)
{
    constexpr int G = kWave / L;
    using S = Slice<float, VEC, STRIDED>;
    const int lane = threadIdx.x & 63;
    const int g = lane / L, j = lane % L;
    const uint64_t b = (uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (b >= nblk) return;
    const uint64_t lo = b * kFixupBlock * chunk, hi = (b + 1) * kFixupBlock * chunk;
    if (lo == 0 || hi > nnz || row[lo - 1] != row[hi - 1]) return;  // not inside one row
    float acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = 0.0f;
    if (S::active(j, rank)) {
#pragma unroll 8
        for (uint32_t q = g; q < kFixupBlock; q += G) {
            float v[VEC];
            S::load_f(part + 2 * (b * kFixupBlock + q) * ldp, j, rank, v);
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[e] += v[e];
        }
    }
#pragma unroll
    for (int off = L; off < 64; off <<= 1)
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] += __shfl_xor(acc[e], off);
    if (g == 0 && S::active(j, rank)) store_slice<VEC, STRIDED>(blk + b * ldp, j, rank, acc, 1.0f);
}

//
// Chunk-driven form (for streams whose rows are never empty, such as fibers,
// where rows far outnumber chunks): candidate rows come from the chunk edges
// instead of from a scan over all rows. Chunk c proposes the row that holds
// its last nonzero when that row continues into chunk c + 1 and starts inside
// chunk c, so each split row is proposed exactly once.
template <int VEC, int L, bool STRIDED>
__global__ __launch_bounds__(256) void fixup_kernel(const uint32_t *__restrict__ rowptr, uint32_t nrows,
                                                    const float *__restrict__ part, uint32_t ldp,
                                                    const float *__restrict__ blk, float *__restrict__ out,
                                                    uint32_t ldo, uint32_t rank, uint64_t chunk, float alpha,
                                                    const uint32_t *__restrict__ row, uint64_t nnz, uint64_t nchunks,
                                                    bool by_chunk)
{
    constexpr int G = kWave / L;
    using S = Slice<float, VEC, STRIDED>;
    const int lane = threadIdx.x & 63;
    const int g = lane / L, j = lane % L;
    const bool lane_on = S::active(j, rank);
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    const uint64_t wid = (uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    auto slot_of = [&](uint64_t ca, uint64_t q) { return q == 0 ? 2 * ca + 1 : 2 * (ca + q); };
    const uint64_t items = by_chunk ? nchunks : nrows;
    for (uint64_t t = wid; t * 64 < items; t += waves) {
        uint64_t r = t * 64 + lane;
        uint32_t a = 0, b = 0;
        bool live = r < items;
        if (by_chunk && live) {
            const uint64_t c = r, c1 = (c + 1) * chunk;
            live = c1 < nnz && row[c1] == row[c1 - 1];
            r = live ? row[c1 - 1] : 0;
            if (live) live = rowptr[r] >= c * chunk;  // the row starts in this chunk
        }
        if (live) {
            a = rowptr[r];
            b = rowptr[r + 1];
        }
        const bool empty = live && a == b;
        const bool split = live && a < b && (a / chunk) != ((b - 1) / chunk);
        const uint64_t cnt = split ? (b - 1) / chunk - a / chunk + 1 : 0;
        if (empty) {  // each lane clears its own row
            float *o = out + r * (uint64_t)ldo;
            for (uint32_t c = 0; c < rank; ++c) o[c] = 0.0f;
        }
        // light rows: lane group g takes the g-th remaining one
        uint64_t light = __ballot(split && cnt <= kFixupLight);
        while (light) {
            uint64_t m = light;
            for (int i = 0; i < g && m; ++i) m &= m - 1;
            // The shuffles run with every lane active: a shuffle whose source lane is
            // inactive yields 0, and the row's lane may sit in a group without a row.
            const int src = m ? __ffsll((long long)m) - 1 : 0;
            const uint32_t aa = __shfl(a, src), bb = __shfl(b, src);
            const uint64_t rr = (uint32_t)__shfl((int)(uint32_t)r, src);
            if (m && bb > aa) {
                const uint64_t ca = aa / chunk, n = (bb - 1) / chunk - ca + 1;
                float acc[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[e] = 0.0f;
                if (lane_on) {
#pragma unroll 4
                    for (uint64_t q = 0; q < n; ++q) {
                        float v[VEC];
                        S::load_f(part + slot_of(ca, q) * ldp, j, rank, v);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) acc[e] += v[e];
                    }
                    store_slice<VEC, STRIDED>(out + rr * (uint64_t)ldo, j, rank, acc, alpha);
                }
            }
            for (int i = 0; i < G && light; ++i) light &= light - 1;
        }
        // heavy rows: the whole wave, G strided shares with 8 loads in flight per lane
        uint64_t heavy = __ballot(split && cnt > kFixupLight);
        while (heavy) {
            const int src = __ffsll((long long)heavy) - 1;
            heavy &= heavy - 1;
            const uint32_t aa = __shfl(a, src), bb = __shfl(b, src);
            const uint64_t rr = (uint32_t)__shfl((int)(uint32_t)r, src);
            const uint64_t ca = aa / chunk, cb = (bb - 1) / chunk;
            // items: the tail of chunk ca, the heads of chunks ca+1..cb, where the
            // level-one blocks lying wholly in ca+1..cb-1 (chunks of this row only)
            // stand for their kFixupBlock heads
            const uint64_t blo = (ca + 1 + kFixupBlock - 1) / kFixupBlock;
            const uint64_t bhi_end = cb / kFixupBlock;  // one past the last usable block
            const bool blocks = blo < bhi_end;
            const uint64_t n1 = blocks ? blo * kFixupBlock - (ca + 1) : cb - ca;
            const uint64_t nb = blocks ? bhi_end - blo : 0;
            const uint64_t n3 = blocks ? cb + 1 - bhi_end * kFixupBlock : 0;
            const uint64_t n = 1 + n1 + nb + n3;
            auto item = [&](uint64_t q) -> const float * {
                if (q == 0) return part + (2 * ca + 1) * ldp;
                if (q <= n1) return part + 2 * (ca + q) * ldp;
                if (q <= n1 + nb) return blk + (blo + (q - 1 - n1)) * ldp;
                return part + 2 * (bhi_end * kFixupBlock + (q - 1 - n1 - nb)) * ldp;
            };
            float acc[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[e] = 0.0f;
            if (lane_on) {
                uint64_t q = g;
                for (; q + 7 * G < n; q += 8 * G) {
                    float v[8][VEC];
#pragma unroll
                    for (int u = 0; u < 8; ++u) S::load_f(item(q + u * G), j, rank, v[u]);
#pragma unroll
                    for (int u = 0; u < 8; ++u)
#pragma unroll
                        for (int e = 0; e < VEC; ++e) acc[e] += v[u][e];
                }
                for (; q < n; q += G) {
                    float v[VEC];
                    S::load_f(item(q), j, rank, v);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) acc[e] += v[e];
                }
            }
#pragma unroll
            for (int off = L; off < 64; off <<= 1)
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[e] += __shfl_xor(acc[e], off);
            if (g == 0 && lane_on) store_slice<VEC, STRIDED>(out + rr * (uint64_t)ldo, j, rank, acc, alpha);
        }
    }
}

hipError_t launch_fixup(const uint32_t *rowptr, const uint32_t *row, uint64_t nnz, uint32_t nrows,
                        const float *part, uint32_t ldp, float *blk, uint64_t nchunks, float *out, uint32_t ldo,
                        uint32_t rank, uint64_t chunk, float alpha, KernelShape s, hipStream_t st, bool by_chunk)
{
    const uint64_t tiles = ((by_chunk ? nchunks : (uint64_t)nrows) + 63) / 64;
    const unsigned grid = grid_for(tiles, 4, 4096);
    const uint64_t nblk = (nchunks + kFixupBlock - 1) / kFixupBlock;
    const unsigned bgrid = (unsigned)((nblk + 3) / 4);
#define PASTA_FIXUP(V, LL, STR)                                                                                   \
    do {                                                                                                         \
        if (nblk > 0 && nnz > 0)                                                                                 \
            fixup_blocks_kernel<V, LL, STR><<<bgrid, 256, 0, st>>>(row, nnz, part, ldp, blk, nblk, rank, chunk);  \
        fixup_kernel<V, LL, STR><<<grid, 256, 0, st>>>(rowptr, nrows, part, ldp, blk, out, ldo, rank, chunk, alpha, \
                                                       row, nnz, nchunks, by_chunk);                                \
    } while (0)
    if (s.strided && rank == 1) {
        // one scalar row per lane, 64 rows per wave: a strided slice with one
        // lane and one element covers element 0, the whole row when R = 1
        PASTA_FIXUP(1, 1, true);
    } else if (s.strided) {
        PASTA_FIXUP(4, 64, true);
    } else {
        // partial rows are fp32: a bf16 shape (8 per lane) maps to 4 per lane on twice the lanes
        const int lanes = s.vec == 8 ? s.lanes * 2 : s.lanes;
        switch (lanes) {
        case 1: PASTA_FIXUP(4, 1, false); break;
        case 2: PASTA_FIXUP(4, 2, false); break;
        case 4: PASTA_FIXUP(4, 4, false); break;
        case 8: PASTA_FIXUP(4, 8, false); break;
        case 16: PASTA_FIXUP(4, 16, false); break;
        case 32: PASTA_FIXUP(4, 32, false); break;
        default: PASTA_FIXUP(4, 64, true); break;
        }
    }
#undef PASTA_FIXUP
    return hipGetLastError();
}

// Zero rows 0..nrows-1 (columns 0..rank-1); used when a mode has no nonzeros at all.
__global__ void zero_rows_kernel(float *out, uint32_t nrows, uint32_t ldo, uint32_t rank)
{
    const uint64_t total = (uint64_t)nrows * rank;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (uint64_t)gridDim.x * blockDim.x)
        out[(e / rank) * ldo + (e % rank)] = 0.0f;
}

hipError_t launch_zero_rows(float *out, uint32_t nrows, uint32_t ldo, uint32_t rank, hipStream_t st)
{
    if ((uint64_t)nrows * rank == 0) return hipSuccess;
    zero_rows_kernel<<<grid_for((uint64_t)nrows * rank, 256), 256, 0, st>>>(out, nrows, ldo, rank);
    return hipGetLastError();
}

// Deterministic sum of n fp64 partials by one block (fixed tree order).
__global__ __launch_bounds__(256) void sum_f64_kernel(const double *part, uint32_t n, double *out)
{
    // eight interleaved running sums per thread, so eight loads are in flight;
    // they are added in a fixed order, so the result stays deterministic
    __shared__ double lds[4];
    double acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.0;
    for (uint32_t i = threadIdx.x; i < n; i += 256 * 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t q = i + 256u * k;
            acc[k] += q < n ? part[q] : 0.0;
        }
    }
    double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    s = wave_sum_f64(s);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

hipError_t launch_sum_f64(const double *part, uint32_t n, double *out, hipStream_t st)
{
    sum_f64_kernel<<<1, 256, 0, st>>>(part, n, out);
    return hipGetLastError();
}

// fp32 -> bf16, round to nearest with ties to even; NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x0040u);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__global__ void cast_bf16_kernel(const float *__restrict__ src, uint16_t *__restrict__ dst, uint64_t n)
{
    const uint64_t n4 = n / 4;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (uint64_t)gridDim.x * blockDim.x) {
        const float4 v = reinterpret_cast<const float4 *>(src)[i];
        ushort4 o;
        o.x = f32_to_bf16_rne(v.x);
        o.y = f32_to_bf16_rne(v.y);
        o.z = f32_to_bf16_rne(v.z);
        o.w = f32_to_bf16_rne(v.w);
        reinterpret_cast<ushort4 *>(dst)[i] = o;
    }
    const uint64_t tail = n4 * 4 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tail < n) dst[tail] = f32_to_bf16_rne(src[tail]);
}

__global__ void cast_bf16_scalar_kernel(const float *__restrict__ src, uint16_t *__restrict__ dst, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = f32_to_bf16_rne(src[i]);
}

hipError_t launch_cast_bf16(const float *src, uint16_t *dst, uint64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    if (((uintptr_t)src % 16 == 0) && ((uintptr_t)dst % 8 == 0))
        cast_bf16_kernel<<<grid_for(n / 4 + 1, 256), 256, 0, st>>>(src, dst, n);
    else
        cast_bf16_scalar_kernel<<<grid_for(n, 256), 256, 0, st>>>(src, dst, n);
    return hipGetLastError();
}

// x[i] *= (float)(*alpha): scales a gradient by an upstream derivative that lives on the device.
__global__ void scale_kernel(float *__restrict__ x, uint64_t n, const double *__restrict__ alpha)
{
    const float a = (float)*alpha;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        x[i] *= a;
}

hipError_t launch_scale(float *x, uint64_t n, const double *alpha, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    scale_kernel<<<grid_for(n, 256), 256, 0, st>>>(x, n, alpha);
    return hipGetLastError();
}

// One Adam step (Kingma and Ba) on fp32 parameters, with the bias corrections
// folded into the step size, and an optional bf16 copy of the updated
// parameters written in the same pass (round to nearest even).
__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, uint16_t *__restrict__ shadow, uint64_t n, float lr, float b1,
                            float b2, float eps, float step_size, float inv_sqrt_bc2)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - step_size * mi / (sqrtf(vi) * inv_sqrt_bc2 + eps);
        p[i] = pi;
        if (shadow) shadow[i] = f32_to_bf16_rne(pi);
    }
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, uint16_t *shadow, uint64_t n, float lr,
                       float b1, float b2, float eps, uint32_t step, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const double bc1 = 1.0 - pow((double)b1, (double)step);
    const double bc2 = 1.0 - pow((double)b2, (double)step);
    adam_kernel<<<grid_for(n, 256), 256, 0, st>>>(p, g, m, v, shadow, n, lr, b1, b2, eps, (float)(lr / bc1),
                                                  (float)(1.0 / sqrt(bc2)));
    return hipGetLastError();
}

}  // namespace pasta
