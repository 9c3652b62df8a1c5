// Order-specialised gfx950 kernels: mode-n MTTKRP over the mode-sorted
// stream, the sampled CP model, and the atomic variant. This file is
// compiled once per order with PASTA_NM1 = order - 1 (the number of factor
// rows gathered per nonzero), so every loop over modes is unrolled.
//
// MTTKRP (Section 4.6, eq. mttkrp-init; Alg. 6 of Section 5.2, generalised
// to order N and any mode n): out[i,:] = alpha * sum_{m: i_n(m)=i} x_m *
// (U^(k1)[i_k1(m),:] * ... * U^(kN-1)[i_kN-1(m),:]) (Hadamard product).
//
// Work split. The nonzeros, sorted by i_n, are cut into chunks of
// C = G * sub consecutive nonzeros, one chunk per wave64. A wave is G lane
// groups of L lanes; lane j of a group owns elements j*VEC .. j*VEC+VEC-1 of
// the R-wide rows (16-byte gathers). Group g walks its own contiguous run of
// `sub` nonzeros and keeps the running row sum in registers while i_n does
// not change, so a row that starts and ends inside the run is finished
// there and stored once with a plain store. At the end of the chunk the
// first and last rows of the G runs are joined by a segmented scan across
// the groups (cross-lane shuffles); joined rows that stay inside the chunk
// are stored, and a row that crosses a chunk edge leaves a partial in a
// scratch slot for the fixup kernel. No atomics, and the summation order is
// fixed, so results are bitwise reproducible.
#include "common.h"

#ifndef PASTA_NM1
#error "compile with -DPASTA_NM1=<order-1>"
#endif

namespace pasta {
namespace {

constexpr int NM1 = PASTA_NM1;
// Nonzeros a group handles per step; their NM1 gathers are issued together.
constexpr int kStep = NM1 <= 2 ? 8 : (NM1 <= 4 ? 4 : 2);

struct MttkrpArgs {
    const uint32_t *row;
    const uint32_t *idx[NM1];
    const void *fac[NM1];
    const void *facn;
    const float *vals;
    const uint32_t *perm;
    float *out;
    float *part;
    double *loss_part;
    uint32_t *flag;
    uint64_t nnz;
    uint32_t ldf, ldo, ldp, rank, sub, nchunks;
    uint32_t row_bytes;  // ldf * element size (contiguous shapes: 32-bit row offsets)
    uint32_t keys;       // factors 0 .. keys-1 are the stream's sort keys after i_n, in key order (0..2)
    uint32_t lds_rows;   // rows of factor NM1-1, which is read from LDS (0: none)
    float alpha;
};

// Plain (temporal) loads for the index/value stream: non-temporal loads were
// measured 25-50% slower on gfx950 for this kernel.
template <typename T>
__device__ __forceinline__ T stream_load(const T *p)
{
    return *p;
}

// Chunk handled by a wave: each XCD takes one contiguous run of chunks, which
// keeps the factor rows a run touches in that XCD's own L2.
__device__ __forceinline__ uint32_t chunk_of_wave(uint32_t nblocks)
{
    return xcd_contiguous(blockIdx.x, nblocks) * 4 + (threadIdx.x >> 6);
}

// A factor small enough for LDS (the host sizes it; the last of the list): every
// workgroup copies its rows there once, with a row stride of L x 16 bytes (the
// slices the lanes read), so its gathers become LDS reads and leave the vector
// memory pipeline to the other factors. Every wave of the workgroup takes part,
// before any of them leaves.
template <typename FT, int L>
__device__ __forceinline__ void stage_lds_factor(const MttkrpArgs &a, uint4 *lds)
{
    const uint32_t slices = (a.rank * (uint32_t)sizeof(FT) + 15u) / 16u;  // active 16-byte slices per row
    const char *src = static_cast<const char *>(a.fac[NM1 - 1]);
    for (uint32_t e = threadIdx.x; e < a.lds_rows * (uint32_t)L; e += 256u) {
        const uint32_t r = e / (uint32_t)L, sl = e % (uint32_t)L;
        if (sl < slices) lds[e] = *reinterpret_cast<const uint4 *>(src + (uint64_t)r * a.row_bytes + sl * 16u);
    }
    __syncthreads();
}

// With LDSF (contiguous shapes) the last factor is read from LDS.
template <typename FT, int VEC, int L, bool STRIDED, bool FUSED, bool OVR, bool LDSF>
__global__ __launch_bounds__(256) void mttkrp_seg_kernel(const MttkrpArgs a)
{
    constexpr int G = kWave / L;
    constexpr int U = kStep;
    static_assert((U & (U - 1)) == 0, "steps are powers of two");
    constexpr int EPL = L >= U ? 1 : U / L;  // entries each lane loads per step
    using S = Slice<FT, VEC, STRIDED>;
    using Packed = typename S::Packed;
    // Row reuse pays with bf16 factors (measured: ~8% faster per mode on the
    // 50M-nonzero Zipf tensor) but costs ~20% with fp32 rows, so it is only
    // compiled in for bf16.
    constexpr bool kReuse = sizeof(FT) == 2;

    static_assert(!(LDSF && STRIDED), "LDS rows have the contiguous slice layout");
    const int lane = threadIdx.x & 63;
    extern __shared__ uint4 lds_fac[];
    if constexpr (LDSF) stage_lds_factor<FT, L>(a, lds_fac);
    const uint32_t chunk = chunk_of_wave(gridDim.x);
    if (chunk >= a.nchunks) return;  // whole wave leaves together
    const int g = lane / L, j = lane % L;
    const int gbase = lane & ~(L - 1);
    const uint64_t C = (uint64_t)a.sub * G;
    const uint64_t c0 = (uint64_t)chunk * C;
    const uint64_t c1 = c0 + C < a.nnz ? c0 + C : a.nnz;
    const uint64_t s0 = c0 + (uint64_t)g * a.sub < c1 ? c0 + (uint64_t)g * a.sub : c1;
    const uint64_t s1 = s0 + a.sub < c1 ? s0 + a.sub : c1;
    const bool lane_on = S::active(j, a.rank);

    float acc[VEC], head[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = head[e] = 0.0f;
    float rowfac[VEC];  // fused: U^(n) slice of the current row
#pragma unroll
    for (int e = 0; e < VEC; ++e) rowfac[e] = 0.0f;
    float loss_run = 0.0f;  // fused: this run's sum of squared residuals (<= 256 terms)
    // the factor rows of the previous nonzero (their indices in lastk), reused
    // without a memory request when the next nonzero names the same rows
    float rowk[NM1][VEC];
    uint32_t lastk[NM1];
#pragma unroll
    for (int k = 0; k < NM1; ++k) {
        lastk[k] = kNoRow;
#pragma unroll
        for (int e = 0; e < VEC; ++e) rowk[k][e] = 0.0f;
    }
    uint32_t cur = kNoRow, hrow = kNoRow;
    bool multi = false;  // this group has already closed its first row

    // Index stream, software-pipelined two steps ahead: the loads for step
    // i + 2 are issued after the gathers of step i. Loads return in order, so
    // waiting for the gathers of a step never waits for the prefetch, and a
    // step's gathers never wait for a fresh trip to memory for their indices.
    // The prefetch is branch-free (indices clamped into the stream) so the
    // compiler can count the loads in flight exactly. With a value override
    // the permutation is prefetched and the value itself gathered one step
    // ahead of its use.
    struct Entries {
        uint32_t r[EPL], i[EPL][NM1];
        float v[EPL];
    };
    const uint64_t last = a.nnz - 1;
    auto load_entries = [&](uint64_t p, Entries &E) {
#pragma unroll
        for (int t = 0; t < EPL; ++t) {
            const uint64_t q0 = p + (uint64_t)(j + L * t);
            const uint64_t q = q0 < last ? q0 : last;
            E.r[t] = stream_load(a.row + q);
#pragma unroll
            for (int k = 0; k < NM1; ++k) E.i[t][k] = stream_load(a.idx[k] + q);
            if constexpr (OVR)
                E.v[t] = __uint_as_float(stream_load(a.perm + q));
            else
                E.v[t] = stream_load(a.vals + q);
        }
    };
    auto resolve_values = [&](Entries &E) {
        if constexpr (OVR) {
#pragma unroll
            for (int t = 0; t < EPL; ++t) E.v[t] = a.vals[__float_as_uint(E.v[t])];
        }
    };
    // One step of U entries: gathers for E0, values of E1, prefetch into E2.
    // The loop below is unrolled three times with the buffers' roles rotated,
    // so no register holding a load in flight is ever copied (a copy would
    // have to wait for the load).
    // One 16-byte slice of factor row iu. Contiguous shapes add a 32-bit byte
    // offset (24-bit row index times the row bytes) to the factor's base, which
    // the host guarantees fits; the strided shape keeps 64-bit addressing.
    auto gather = [&](int k, uint32_t iu, int jj, Packed &pk) {
        if constexpr (STRIDED) {
            S::load(static_cast<const FT *>(a.fac[k]) + (uint64_t)iu * a.ldf, jj, a.rank, pk);
        } else {
            uint4 t;
            if (LDSF && k == NM1 - 1) {
                t = lds_fac[iu * (uint32_t)L + (uint32_t)jj];
            } else {
                const uint32_t off = __umul24(iu, a.row_bytes) + (uint32_t)jj * 16u;
                t = *reinterpret_cast<const uint4 *>(static_cast<const char *>(a.fac[k]) + off);
            }
            pk.w[0] = t.x;
            pk.w[1] = t.y;
            pk.w[2] = t.z;
            pk.w[3] = t.w;
        }
    };
    // FULL: every group's run is whole steps (a full chunk), so no step checks
    // how many of its entries exist.
    auto step = [&](Entries &E0, Entries &E1, Entries &E2, uint64_t p, auto full) {
        constexpr bool FULL = decltype(full)::value;
        const uint32_t navail = FULL ? (uint32_t)U : (uint32_t)(s1 - p < (uint64_t)U ? s1 - p : (uint64_t)U);
        // broadcast each entry's factor indices to the group and issue all its
        // gathers; its row and value are broadcast later, where they are used
        Packed gp[U][NM1];
        bool reuse[U][NM1];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int src = gbase | (u % L);
#pragma unroll
            for (int k = 0; k < NM1; ++k) {
                const uint32_t iu = (uint32_t)__shfl((int)E0.i[u / L][k], src);
                if constexpr (kReuse) {
                    // the same factor row as the previous nonzero: keep it, no request
                    reuse[u][k] = iu == lastk[k];
                    if (FULL || (uint32_t)u < navail) lastk[k] = iu;
                    if ((FULL || (uint32_t)u < navail) && lane_on && !reuse[u][k]) gather(k, iu, j, gp[u][k]);
                } else {
                    // branch-free: entries past the run read their (clamped, valid)
                    // row and idle lanes read slice 0; both results are discarded
                    gather(k, iu, lane_on ? j : 0, gp[u][k]);
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);  // the prefetch goes out after this step's gathers
        resolve_values(E1);
        load_entries(p + 2 * U, E2);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (!FULL) {
                if ((uint32_t)u >= navail) break;
            }
            const int src = gbase | (u % L);
            const uint32_t ru = (uint32_t)__shfl((int)E0.r[u / L], src);
            const float vu = __shfl(E0.v[u / L], src);
            float q[VEC];
            if constexpr (kReuse) {
#pragma unroll
                for (int k = 0; k < NM1; ++k)
                    if (!reuse[u][k]) S::unpack(gp[u][k], rowk[k]);
#pragma unroll
                for (int e = 0; e < VEC; ++e) q[e] = rowk[0][e];
#pragma unroll
                for (int k = 1; k < NM1; ++k)
#pragma unroll
                    for (int e = 0; e < VEC; ++e) q[e] *= rowk[k][e];
            } else {
                S::unpack(gp[u][0], q);
#pragma unroll
                for (int k = 1; k < NM1; ++k) {
                    float t[VEC];
                    S::unpack(gp[u][k], t);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) q[e] *= t[e];
                }
            }
            if (ru != cur) {
                if (cur != kNoRow) {
                    if (!multi) {  // the run's first row may continue in earlier runs: keep it
#pragma unroll
                        for (int e = 0; e < VEC; ++e) head[e] = acc[e];
                        hrow = cur;
                        multi = true;
                    } else if (lane_on) {  // a row inside the run: complete, store it
                        store_slice_nt<VEC, STRIDED>(a.out + (uint64_t)cur * a.ldo, j, a.rank, acc, a.alpha);
                    }
                }
                cur = ru;
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[e] = 0.0f;
                if constexpr (FUSED) {
                    if (lane_on) S::load_f(static_cast<const FT *>(a.facn) + (uint64_t)cur * a.ldf, j, a.rank, rowfac);
                }
            }
            float w = vu;
            if constexpr (FUSED) {  // residual of the CP model at this nonzero
                float d = 0.0f;
#pragma unroll
                for (int e = 0; e < VEC; ++e) d += rowfac[e] * q[e];
                d = group_sum<L>(lane_on ? d : 0.0f);
                w = d - vu;
                loss_run += w * w;
            }
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[e] += w * q[e];
        }
    };
    Entries e0, e1, e2;
    load_entries(s0, e0);
    __builtin_amdgcn_sched_barrier(0);  // keep e0's loads ahead of e1's (in-order waits)
    load_entries(s0 + U, e1);
    resolve_values(e0);
    static_assert(256 % U == 0, "runs of whole steps in full chunks");
    if (c1 - c0 == C && a.sub % U == 0) {  // wave-uniform
        for (uint64_t p = s0; p < s1; p += 3 * U) {
            step(e0, e1, e2, p, std::true_type{});
            if (p + U >= s1) break;
            step(e1, e2, e0, p + U, std::true_type{});
            if (p + 2 * U >= s1) break;
            step(e2, e0, e1, p + 2 * U, std::true_type{});
        }
    } else {
        for (uint64_t p = s0; p < s1; p += 3 * U) {
            step(e0, e1, e2, p, std::false_type{});
            if (p + U >= s1) break;
            step(e1, e2, e0, p + U, std::false_type{});
            if (p + 2 * U >= s1) break;
            step(e2, e0, e1, p + 2 * U, std::false_type{});
        }
    }

    // ---- join the runs' edge rows across the G groups of the wave ----
    const uint32_t first = multi ? hrow : cur;  // the run's first row (kNoRow if empty)
    uint32_t prev_last = (uint32_t)__shfl_up((int)cur, L);
    if (g == 0) prev_last = kNoRow;
    const bool cont = cur != kNoRow && first == prev_last;  // continues the previous run's last row
    // segmented inclusive scan of the last-row sums; only single-row runs pass a sum on
    bool seg_start = !(cont && !multi);
    float carry[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) carry[e] = acc[e];
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        const bool ps = __shfl_up((int)seg_start, d * L) != 0;
        float pv[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) pv[e] = __shfl_up(carry[e], d * L);
        if (g >= d && !seg_start) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) carry[e] += pv[e];
        }
        if (g >= d) seg_start = seg_start || ps;
    }
    float prev_carry[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) prev_carry[e] = __shfl_up(carry[e], L);
    int next_cont = __shfl_down((int)cont, L);
    if (g == G - 1) next_cont = 0;

    // chunk-edge classification
    const uint32_t cfirst = a.row[c0];
    const uint32_t clast = a.row[c1 - 1];
    const bool before = c0 > 0 && a.row[c0 - 1] == cfirst;
    const bool after = c1 < a.nnz && a.row[c1] == clast;
    auto emit = [&](uint32_t r, const float (&v)[VEC]) {
        if (!lane_on) return;
        if (r == cfirst && before)
            store_slice<VEC, STRIDED>(a.part + (uint64_t)(2 * (uint64_t)chunk) * a.ldp, j, a.rank, v, 1.0f);
        else if (r == clast && after)
            store_slice<VEC, STRIDED>(a.part + (uint64_t)(2 * (uint64_t)chunk + 1) * a.ldp, j, a.rank, v, 1.0f);
        else
            store_slice_nt<VEC, STRIDED>(a.out + (uint64_t)r * a.ldo, j, a.rank, v, a.alpha);
    };
    if (multi) {  // first row closed inside this run; add what earlier runs carried
        if (cont) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) head[e] += prev_carry[e];
        }
        emit(hrow, head);
    }
    if (cur != kNoRow && !next_cont) emit(cur, carry);

    if constexpr (FUSED) {
        if (a.loss_part) {  // every lane of a group holds its run's sum: count it once per group
            const double tot = wave_sum_f64(j == 0 ? 0.5 * (double)loss_run : 0.0);
            if (lane == 0) a.loss_part[chunk] = tot;
        }
    }
}

// Steps per gather group of the fused wave-run kernel. Its residual needs more
// registers than plain MTTKRP, and fewer gathers in flight buy back a wave per
// SIMD where that pays (measured at R = 32 and 64: bf16 at order 3 and every
// dtype at orders 5+ go from 3 to 4 or from 2 to 3 waves; the rest keep theirs).
constexpr int fused_group_steps(bool bf16)
{
    return NM1 <= 2 ? (bf16 ? 2 : 4) : (NM1 == 3 ? 4 : 2);
}

// ---------------------------------------------------------------------------
// Wave-run form, for streams whose rows are long. A wave owns one chunk of
// `sub` consecutive nonzeros and walks it G at a time: in each step, group g
// takes the g-th of G consecutive nonzeros. Nonzeros next to each other in the
// mode order often name the same factor row (the order's second key is the
// previous mode), so those gathers land in one instruction and share its
// cache-line request. The row being summed is the same for the whole wave;
// each group keeps its own share of it in registers, and the shares are added
// across groups (shuffles) only when the row ends. A tile of 64 entries is
// loaded with one coalesced load per stream and broadcast from the lane that
// holds each entry; `US` steps' gathers go out together, and the entries two
// tiles ahead are loaded behind them. Rows crossing the chunk's edges leave
// partials in the same slots as the run form, for the same fixup.
// ---------------------------------------------------------------------------
// With LDSF the last factor is read from LDS.
template <typename FT, int VEC, int L, bool FUSED, bool OVR, bool LDSF>
__global__ __launch_bounds__(256) void mttkrp_wave_kernel(const MttkrpArgs a)
{
    constexpr int G = kWave / L;                 // nonzeros per step
    // steps whose gathers go out together, and such groups per tile of 64 entries
    // With a factor in LDS, a step has one memory gather fewer; with fp32 rows the LDS form
    // then keeps 8 steps of the others in flight (measured at order 5: modes 1-3 6.3-6.7 ->
    // 5.9-6.1 ms, although the registers allow one wave per SIMD fewer; with bf16 rows, in
    // the other forms and in the fused kernel more steps were slower).
    constexpr int US_MAX = FUSED ? fused_group_steps(sizeof(FT) == 2) : (LDSF && sizeof(FT) == 4 ? 8 : kStep);
    constexpr int US = L < US_MAX ? L : US_MAX;
    constexpr int MS = L / US;
    using S = Slice<FT, VEC, false>;
    using Packed = typename S::Packed;
    const int lane = threadIdx.x & 63;
    extern __shared__ uint4 lds_fac[];
    if constexpr (LDSF) stage_lds_factor<FT, L>(a, lds_fac);
    const uint32_t chunk = chunk_of_wave(gridDim.x);
    if (chunk >= a.nchunks) return;  // whole wave leaves together
    const int g = lane / L, j = lane % L;
    const uint64_t C = a.sub;
    const uint64_t c0 = (uint64_t)chunk * C;
    const uint64_t c1 = c0 + C < a.nnz ? c0 + C : a.nnz;
    const bool lane_on = S::active(j, a.rank);
    const uint32_t cfirst = a.row[c0], clast = a.row[c1 - 1];
    const bool before = c0 > 0 && a.row[c0 - 1] == cfirst;
    const bool after = c1 < a.nnz && a.row[c1] == clast;
    uint32_t cur = cfirst;  // the row being summed (wave-uniform)
    float acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = 0.0f;
    // fused: the U^(n) slice of a row, and this group's sum of squared residuals
    // (one term per step: chunk / G terms in fp32, then fp64 across the groups)
    auto load_rowfac = [&](uint32_t r, float (&rf)[VEC]) __attribute__((always_inline)) {
        if (lane_on) {
            S::load_f(static_cast<const FT *>(a.facn) + (uint64_t)r * a.ldf, j, a.rank, rf);
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) rf[e] = 0.0f;
        }
    };
    float rowfac[VEC];
    if constexpr (FUSED) load_rowfac(cur, rowfac);
    float loss_run = 0.0f;
    // Factor 0 is the mode order's second key (the host lists it first). Where a
    // group of steps stays in the current row and its first and last nonzeros share
    // the second key's row, all of its nonzeros do (the stream is sorted by
    // (i_n, second key, ...)): that row is gathered once for the whole group of
    // steps, and not at all if it is the row already held.
    // From order 4 on, factor 1 is treated the same way where the group of steps also
    // shares its row and the stream is sorted by it next (it is the third key: every
    // mode but mode 0, whose order falls back to caller position after two keys).
    uint32_t held = kNoRow, held1 = kNoRow;  // wave-uniform: the rows whose slices hold / hold1 hold
    Packed hold, hold1;
#pragma unroll
    for (int w = 0; w < S::kWords; ++w) hold.w[w] = hold1.w[w] = 0u;

    // total of row `cur` over every group (plus `extra` from this step), stored by group 0
    auto close_row = [&](const float (&extra)[VEC]) __attribute__((always_inline)) {
        float t[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) t[e] = acc[e] + extra[e];
#pragma unroll
        for (int off = L; off < kWave; off <<= 1)
#pragma unroll
            for (int e = 0; e < VEC; ++e) t[e] += __shfl_xor(t[e], off);
        if (g == 0 && lane_on) {
            if (cur == cfirst && before)
                store_slice<VEC, false>(a.part + (uint64_t)(2 * (uint64_t)chunk) * a.ldp, j, a.rank, t, 1.0f);
            else if (cur == clast && after)
                store_slice<VEC, false>(a.part + (uint64_t)(2 * (uint64_t)chunk + 1) * a.ldp, j, a.rank, t, 1.0f);
            else
                store_slice<VEC, false>(a.out + (uint64_t)cur * a.ldo, j, a.rank, t, a.alpha);
        }
    };
    auto gather = [&](int k, uint32_t iu, Packed &pk) __attribute__((always_inline)) {
        uint4 t;
        if (LDSF && k == NM1 - 1) {
            t = lds_fac[iu * (uint32_t)L + (uint32_t)(lane_on ? j : 0)];
        } else {
            const uint32_t off = __umul24(iu, a.row_bytes) + (uint32_t)(lane_on ? j : 0) * 16u;
            t = *reinterpret_cast<const uint4 *>(static_cast<const char *>(a.fac[k]) + off);
        }
        pk.w[0] = t.x;
        pk.w[1] = t.y;
        pk.w[2] = t.z;
        pk.w[3] = t.w;
    };
    // the CP model's residual at a nonzero whose row slice of U^(n) is rf, and the
    // product q of its other rows: sum_r rf[r] q[r] - x (group reduction, fixed order)
    auto residual = [&](const float (&rf)[VEC], const float (&q)[VEC], float x) __attribute__((always_inline)) {
        float d = 0.0f;
#pragma unroll
        for (int e = 0; e < VEC; ++e) d += rf[e] * q[e];
        return group_sum<L>(lane_on ? d : 0.0f) - x;
    };
    struct Entries {
        uint32_t r, i[NM1];
        float v;  // with a value override: the position in caller order until resolved
    };
    const uint64_t last = a.nnz - 1;
    // entries past the chunk carry its last row (their contributions are masked off)
    auto load_tile = [&](uint64_t base, Entries &E) __attribute__((always_inline)) {
        const uint64_t q0 = base + (uint64_t)lane;
        const uint64_t q = q0 < last ? q0 : last;
        E.r = stream_load(a.row + q);
#pragma unroll
        for (int k = 0; k < NM1; ++k) E.i[k] = stream_load(a.idx[k] + q);
        if constexpr (OVR)
            E.v = __uint_as_float(stream_load(a.perm + q));
        else
            E.v = stream_load(a.vals + q);
        if (q0 >= c1) E.r = clast;
    };
    auto resolve = [&](Entries &E) __attribute__((always_inline)) {
        if constexpr (OVR) E.v = a.vals[__float_as_uint(E.v)];
    };
    // One tile: MS groups of US steps. After the first group's gathers go out, the
    // next tile's values are resolved and the tile after it is loaded.
    auto tile = [&](const Entries &E, Entries &follow, Entries &target, uint64_t base, auto full)
                    __attribute__((always_inline)) {
        constexpr bool FULLT = decltype(full)::value;
#pragma unroll
        for (int m = 0; m < MS; ++m) {
            // gathers of factors kfrom.. for every step of the group
            auto issue = [&](Packed (&gp)[US][NM1], int kfrom) __attribute__((always_inline)) {
#pragma unroll
                for (int u = 0; u < US; ++u) {
                    const int src = (m * US + u) * G + g;
#pragma unroll
                    for (int k = 0; k < NM1; ++k)
                        if (k >= kfrom) gather(k, (uint32_t)__shfl((int)E.i[k], src), gp[u][k]);
                }
                if (m == 0) {
                    __builtin_amdgcn_sched_barrier(0);  // the next loads go out after these gathers
                    resolve(follow);
                    load_tile(base + 2 * (uint64_t)kWave, target);
                }
            };
            // the Hadamard product of step u's rows, factor 0 from `f0`, factor 1 from `f1`
            // when `one` is set, the rest from gp
            auto product = [&](const Packed &f0, const Packed &f1, bool one, const Packed (&gp)[US][NM1], int u,
                               float (&q)[VEC]) __attribute__((always_inline)) {
                S::unpack(f0, q);
#pragma unroll
                for (int k = 1; k < NM1; ++k) {
                    float t[VEC];
                    S::unpack(k == 1 && one ? f1 : gp[u][k], t);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) q[e] *= t[e];
                }
            };
            // every entry of the group of steps is in the current row
            auto fast = [&](auto prod) __attribute__((always_inline)) {
#pragma unroll
                for (int u = 0; u < US; ++u) {
                    const int src = (m * US + u) * G + g;
                    const float vu = __shfl(E.v, src);
                    const bool on = FULLT || base + (uint64_t)src < c1;
                    float q[VEC];
                    prod(u, q);
                    float w = vu;
                    if constexpr (FUSED) {
                        w = residual(rowfac, q, vu);
                        loss_run += on ? w * w : 0.0f;
                    }
                    if constexpr (FULLT) {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) acc[e] += w * q[e];
                    } else {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) acc[e] = on ? acc[e] + w * q[e] : acc[e];
                    }
                }
            };
            // the row of the group of steps' last entry decides the path for all of them
            const int lfirst = m * US * G, llast = (m + 1) * US * G - 1;
            const uint32_t mlast = (uint32_t)__builtin_amdgcn_readlane((int)E.r, llast);
            const uint32_t k0f = (uint32_t)__builtin_amdgcn_readlane((int)E.i[0], lfirst);
            const uint32_t k0l = (uint32_t)__builtin_amdgcn_readlane((int)E.i[0], llast);
            if (a.keys >= 1 && mlast == cur && k0f == k0l) {  // one factor-0 row for the whole group of steps
                bool one = false;
                if constexpr (NM1 >= 3) {
                    one = a.keys >= 2 && __builtin_amdgcn_readlane((int)E.i[1], lfirst) ==
                                             __builtin_amdgcn_readlane((int)E.i[1], llast);
                }
                // the conditional gathers go out before the others, so the counted waits
                // for the later loads stay exact
                if (k0f != held) {
                    gather(0, k0f, hold);
                    held = k0f;
                }
                Packed gp[US][NM1];
                if (one) {  // and one factor-1 row
                    const uint32_t k1f = (uint32_t)__builtin_amdgcn_readlane((int)E.i[1], lfirst);
                    if (k1f != held1) {
                        gather(1, k1f, hold1);
                        held1 = k1f;
                    }
                    issue(gp, 2);
                    fast([&](int u, float (&q)[VEC]) __attribute__((always_inline)) {
                        product(hold, hold1, true, gp, u, q);
                    });
                } else {
                    issue(gp, 1);
                    fast([&](int u, float (&q)[VEC]) __attribute__((always_inline)) {
                        product(hold, hold1, false, gp, u, q);
                    });
                }
                continue;
            }
            Packed gp[US][NM1];
            issue(gp, 0);
            if (mlast == cur) {  // the common case: every entry is in the current row
                fast([&](int u, float (&q)[VEC]) __attribute__((always_inline)) {
                    product(gp[u][0], hold1, false, gp, u, q);
                });
            } else {  // rows end inside this group of steps
#pragma unroll
                for (int u = 0; u < US; ++u) {
                    const int src = (m * US + u) * G + g;
                    const uint32_t ru = (uint32_t)__shfl((int)E.r, src);
                    const float vu = __shfl(E.v, src);
                    const bool on = FULLT || base + (uint64_t)src < c1;
                    float q[VEC];
                    product(gp[u][0], hold1, false, gp, u, q);
                    float w = vu;
                    if constexpr (FUSED) {  // each group's own row slice of U^(n)
                        float rf[VEC];
                        load_rowfac(ru, rf);
                        w = residual(rf, q, vu);
                        loss_run += on ? w * w : 0.0f;
                    }
                    float contrib[VEC];
#pragma unroll
                    for (int e = 0; e < VEC; ++e) contrib[e] = on ? w * q[e] : 0.0f;
                    const uint32_t rl = (uint32_t)__builtin_amdgcn_readlane((int)E.r, (m * US + u) * G + G - 1);
                    const bool moved = cur != rl;
                    int closed = 0;
                    while (cur != rl) {  // wave-uniform: close every row that ends in this step
                        float extra[VEC];
#pragma unroll
                        for (int e = 0; e < VEC; ++e) extra[e] = ru == cur ? contrib[e] : 0.0f;
                        close_row(extra);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) acc[e] = 0.0f;
                        // the next row: that of the first group past the current one. Only the
                        // first lane of each group votes, so the lowest set bit is that lane.
                        const uint64_t ahead = __ballot(j == 0 && ru > cur);
                        if (ahead == 0 || ++closed > G) {
                            // In a stream sorted by row some group is past `cur` while cur != rl,
                            // and at most G rows end in one step. Otherwise the stream is out of
                            // order: flag it and leave the loop (the results are then undefined).
                            if (lane == 0 && a.flag) *a.flag = 2u;
                            cur = rl;
                            break;
                        }
                        const int first_lane = __ffsll((long long)ahead) - 1;
                        cur = (uint32_t)__builtin_amdgcn_readlane((int)ru, first_lane);
                    }
#pragma unroll
                    for (int e = 0; e < VEC; ++e) acc[e] += ru == cur ? contrib[e] : 0.0f;
                    if constexpr (FUSED) {
                        if (moved) load_rowfac(cur, rowfac);
                    }
                }
            }
        }
    };
    Entries e0, e1, e2;
    load_tile(c0, e0);
    __builtin_amdgcn_sched_barrier(0);  // keep e0's loads ahead of e1's (in-order waits)
    load_tile(c0 + kWave, e1);
    resolve(e0);
    const uint64_t ntiles = (c1 - c0 + kWave - 1) / kWave;
    auto walk = [&](auto full) __attribute__((always_inline)) {
        for (uint64_t t = 0; t < ntiles; t += 3) {
            tile(e0, e1, e2, c0 + t * kWave, full);
            if (t + 1 >= ntiles) break;
            tile(e1, e2, e0, c0 + (t + 1) * kWave, full);
            if (t + 2 >= ntiles) break;
            tile(e2, e0, e1, c0 + (t + 2) * kWave, full);
        }
    };
    if (c1 - c0 == C)  // wave-uniform
        walk(std::true_type{});
    else
        walk(std::false_type{});
    float zero[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) zero[e] = 0.0f;
    close_row(zero);  // the last row of the chunk
    if constexpr (FUSED) {
        if (a.loss_part) {  // every lane of a group holds its sum: count it once per group
            const double tot = wave_sum_f64(j == 0 ? 0.5 * (double)loss_run : 0.0);
            if (lane == 0) a.loss_part[chunk] = tot;
        }
    }
}

// ---------------------------------------------------------------------------
// Sampled CP model: mhat_m = sum_r prod_k U^(k)[i_k(m), r], caller order.
// A wave takes 64 consecutive nonzeros at a time (coalesced index loads, one
// per lane); group g handles the L of them held by its own lanes.
// ---------------------------------------------------------------------------
struct SampleArgs {
    const uint32_t *inds[NM1 + 1];
    const void *fac[NM1 + 1];
    const float *vals;
    float *out;
    double *loss_part;
    uint64_t nnz;
    uint32_t ldf, rank, tiles_per_wave;
};

template <typename FT, int VEC, int L, bool STRIDED>
__global__ __launch_bounds__(256) void cp_sample_kernel(const SampleArgs a)
{
    constexpr int N = NM1 + 1;
    constexpr int B = L < 8 ? L : 8;  // entries per batch
    using S = Slice<FT, VEC, STRIDED>;
    using Packed = typename S::Packed;
    __shared__ double lds[4];
    const int lane = threadIdx.x & 63;
    const int j = lane % L;
    const int gbase = lane & ~(L - 1);
    const bool lane_on = S::active(j, a.rank);
    const uint64_t wave_id = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    double loss = 0.0;
    for (uint32_t tt = 0; tt < a.tiles_per_wave; ++tt) {
        const uint64_t base = (wave_id * a.tiles_per_wave + tt) * 64;
        if (base >= a.nnz) break;
        const uint64_t m = base + lane;
        const bool on = m < a.nnz;
        uint32_t li[N];
#pragma unroll
        for (int k = 0; k < N; ++k) li[k] = on ? a.inds[k][m] : 0u;
        float mine = 0.0f;
#pragma unroll
        for (int b0 = 0; b0 < L; b0 += B) {
            Packed gp[B][N];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int src = gbase | (b0 + u);
                const bool src_on = base + (uint64_t)src < a.nnz;
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const uint32_t iu = (uint32_t)__shfl((int)li[k], src);
                    if (src_on && lane_on) {
                        S::load(static_cast<const FT *>(a.fac[k]) + (uint64_t)iu * a.ldf, j, a.rank, gp[u][k]);
                    } else {
#pragma unroll
                        for (int w = 0; w < S::kWords; ++w) gp[u][k].w[w] = 0u;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                float q[VEC];
                S::unpack(gp[u][0], q);
#pragma unroll
                for (int k = 1; k < N; ++k) {
                    float t[VEC];
                    S::unpack(gp[u][k], t);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) q[e] *= t[e];
                }
                float s = 0.0f;
#pragma unroll
                for (int e = 0; e < VEC; ++e) s += q[e];
                s = group_sum<L>(s);
                if (j == b0 + u) mine = s;
            }
        }
        if (on) {
            if (a.vals) {
                const float r = mine - a.vals[m];
                if (a.out) a.out[m] = r;
                loss += 0.5 * (double)r * (double)r;
            } else {
                a.out[m] = mine;
            }
        }
    }
    if (a.loss_part) {
        const double w = wave_sum_f64(loss);
        if (lane == 0) lds[threadIdx.x >> 6] = w;
        __syncthreads();
        if (threadIdx.x == 0) a.loss_part[blockIdx.x] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
    }
}

// ---------------------------------------------------------------------------
// The parallel-with-atomics form of Section 5.3 on the GPU: nonzeros in
// caller order, every lane group adds its nonzero's product row into the
// output with fp32 atomics (output zeroed first).
// ---------------------------------------------------------------------------
struct AtomicArgs {
    const uint32_t *row;
    const uint32_t *idx[NM1];
    const void *fac[NM1];
    const float *vals;
    float *out;
    uint64_t nnz;
    uint32_t ldf, ldo, rank;
};

template <typename FT, int VEC, int L, bool STRIDED>
__global__ __launch_bounds__(256) void mttkrp_atomic_kernel(const AtomicArgs a)
{
    constexpr int G = kWave / L;
    using S = Slice<FT, VEC, STRIDED>;
    const int lane = threadIdx.x & 63;
    const int g = lane / L, j = lane % L;
    if (!S::active(j, a.rank)) return;
    const uint64_t nwaves = (uint64_t)gridDim.x * 4;
    for (uint64_t m = ((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * G + g; m < a.nnz; m += nwaves * G) {
        float q[VEC];
        S::load_f(static_cast<const FT *>(a.fac[0]) + (uint64_t)a.idx[0][m] * a.ldf, j, a.rank, q);
#pragma unroll
        for (int k = 1; k < NM1; ++k) {
            float t[VEC];
            S::load_f(static_cast<const FT *>(a.fac[k]) + (uint64_t)a.idx[k][m] * a.ldf, j, a.rank, t);
#pragma unroll
            for (int e = 0; e < VEC; ++e) q[e] *= t[e];
        }
        const float x = a.vals[m];
        float *o = a.out + (uint64_t)a.row[m] * a.ldo;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const uint32_t c = STRIDED ? (uint32_t)j + 64u * e : (uint32_t)(j * VEC + e);
            if (c < a.rank) atomicAdd(o + c, x * q[e]);
        }
    }
}

unsigned clamp_grid(uint64_t g, uint64_t cap)
{
    if (g < 1) g = 1;
    return (unsigned)(g > cap ? cap : g);
}

template <typename FT, int VEC, int L, bool STRIDED>
hipError_t run_mttkrp(const MttkrpArgs &args, bool fused, bool wave, hipStream_t st)
{
    const unsigned grid = (unsigned)((args.nchunks + 3) / 4);
    if constexpr (!STRIDED && (L == 8 || L == 16) && NM1 >= 2 && NM1 <= 4) {
        if (args.lds_rows && !args.perm) {  // the host sized lds_rows to fit (kLdsFactorBytes)
            const size_t lds = (size_t)args.lds_rows * L * 16;
            if (wave) {
                if (fused)
                    mttkrp_wave_kernel<FT, VEC, L, true, false, true><<<grid, 256, lds, st>>>(args);
                else
                    mttkrp_wave_kernel<FT, VEC, L, false, false, true><<<grid, 256, lds, st>>>(args);
            } else {
                if (fused)
                    mttkrp_seg_kernel<FT, VEC, L, false, true, false, true><<<grid, 256, lds, st>>>(args);
                else
                    mttkrp_seg_kernel<FT, VEC, L, false, false, false, true><<<grid, 256, lds, st>>>(args);
            }
            return hipGetLastError();
        }
    }
    if constexpr (!STRIDED) {
        if (wave) {
            if (fused)
                mttkrp_wave_kernel<FT, VEC, L, true, false, false><<<grid, 256, 0, st>>>(args);
            else if (args.perm)
                mttkrp_wave_kernel<FT, VEC, L, false, true, false><<<grid, 256, 0, st>>>(args);
            else
                mttkrp_wave_kernel<FT, VEC, L, false, false, false><<<grid, 256, 0, st>>>(args);
            return hipGetLastError();
        }
    }
    if (fused)
        mttkrp_seg_kernel<FT, VEC, L, STRIDED, true, false, false><<<grid, 256, 0, st>>>(args);
    else if (args.perm)
        mttkrp_seg_kernel<FT, VEC, L, STRIDED, false, true, false><<<grid, 256, 0, st>>>(args);
    else
        mttkrp_seg_kernel<FT, VEC, L, STRIDED, false, false, false><<<grid, 256, 0, st>>>(args);
    return hipGetLastError();
}

template <typename FT, int VEC, int L, bool STRIDED>
hipError_t run_sample(const SampleArgs &args, hipStream_t st)
{
    const uint64_t tiles = (args.nnz + 63) / 64;
    const uint64_t waves = (tiles + args.tiles_per_wave - 1) / args.tiles_per_wave;
    cp_sample_kernel<FT, VEC, L, STRIDED><<<clamp_grid((waves + 3) / 4, 1u << 30), 256, 0, st>>>(args);
    return hipGetLastError();
}

template <typename FT, int VEC, int L, bool STRIDED>
hipError_t run_atomic(const AtomicArgs &args, hipStream_t st)
{
    constexpr int G = kWave / L;
    const uint64_t waves = (args.nnz + G - 1) / G;
    mttkrp_atomic_kernel<FT, VEC, L, STRIDED><<<clamp_grid((waves + 3) / 4, 16384), 256, 0, st>>>(args);
    return hipGetLastError();
}

// Dispatch on (dtype, shape): contiguous fp32 float4 / bf16 8-wide slices
// with L in {1,2,4,8,16}, or the strided generic path (L = 64, 4 per lane).
template <template <typename, int, int, bool> class F, typename Args, typename... X>
hipError_t dispatch(const Args &args, bool bf16, KernelShape s, hipStream_t st, X... extra)
{
    if (s.strided) {
        if (bf16) return F<uint16_t, 4, 64, true>::run(args, st, extra...);
        return F<float, 4, 64, true>::run(args, st, extra...);
    }
#define PASTA_CASE(LL)                                                                                           \
    case LL:                                                                                                     \
        if (bf16) return F<uint16_t, 8, LL, false>::run(args, st, extra...);                                   \
        return F<float, 4, LL, false>::run(args, st, extra...);
    switch (s.lanes) {
        PASTA_CASE(1)
        PASTA_CASE(2)
        PASTA_CASE(4)
        PASTA_CASE(8)
        PASTA_CASE(16)
    default:
        return hipErrorInvalidValue;
    }
#undef PASTA_CASE
}

template <typename FT, int VEC, int L, bool STRIDED>
struct MttkrpRun {
    static hipError_t run(const MttkrpArgs &a, hipStream_t st, bool fused, bool wave)
    {
        return run_mttkrp<FT, VEC, L, STRIDED>(a, fused, wave, st);
    }
};
template <typename FT, int VEC, int L, bool STRIDED>
struct SampleRun {
    static hipError_t run(const SampleArgs &a, hipStream_t st) { return run_sample<FT, VEC, L, STRIDED>(a, st); }
};
template <typename FT, int VEC, int L, bool STRIDED>
struct AtomicRun {
    static hipError_t run(const AtomicArgs &a, hipStream_t st) { return run_atomic<FT, VEC, L, STRIDED>(a, st); }
};

}  // namespace

#define PASTA_CAT2(a, b) a##b
#define PASTA_CAT(a, b) PASTA_CAT2(a, b)

hipError_t PASTA_CAT(launch_mttkrp_nm1_, PASTA_NM1)(const MttkrpLaunch &l, bool bf16, KernelShape s, bool fused,
                                                    hipStream_t st)
{
    if (l.nchunks == 0) return hipSuccess;
    MttkrpArgs a{};
    a.row = l.row;
    for (int k = 0; k < NM1; ++k) {
        a.idx[k] = l.idx[k];
        a.fac[k] = l.fac[k];
    }
    a.facn = l.facn;
    a.vals = l.vals;
    a.perm = l.perm;
    a.out = l.out;
    a.part = l.part;
    a.loss_part = l.loss_part;
    a.nnz = l.nnz;
    a.ldf = l.ldf;
    a.ldo = l.ldo;
    a.ldp = l.ldp;
    a.rank = l.rank;
    a.sub = l.sub;
    a.nchunks = l.nchunks;
    a.row_bytes = l.ldf * (bf16 ? 2u : 4u);
    a.keys = l.keys;
    a.lds_rows = l.lds_rows;
    a.flag = l.flag;
    a.alpha = l.alpha;
    return dispatch<MttkrpRun>(a, bf16, s, st, fused, l.wave);
}

hipError_t PASTA_CAT(launch_sample_nm1_, PASTA_NM1)(const SampleLaunch &l, bool bf16, KernelShape s, hipStream_t st)
{
    if (l.nnz == 0) return hipSuccess;
    SampleArgs a{};
    for (int k = 0; k <= NM1; ++k) {
        a.inds[k] = l.inds[k];
        a.fac[k] = l.fac[k];
    }
    a.vals = l.vals;
    a.out = l.out;
    a.loss_part = l.loss_part;
    a.nnz = l.nnz;
    a.ldf = l.ldf;
    a.rank = l.rank;
    a.tiles_per_wave = l.tiles_per_wave;
    return dispatch<SampleRun>(a, bf16, s, st);
}

hipError_t PASTA_CAT(launch_atomic_nm1_, PASTA_NM1)(const AtomicLaunch &l, bool bf16, KernelShape s, hipStream_t st)
{
    if (l.nnz == 0) return hipSuccess;
    AtomicArgs a{};
    a.row = l.row;
    for (int k = 0; k < NM1; ++k) {
        a.idx[k] = l.idx[k];
        a.fac[k] = l.fac[k];
    }
    a.vals = l.vals;
    a.out = l.out;
    a.nnz = l.nnz;
    a.ldf = l.ldf;
    a.ldo = l.ldo;
    a.rank = l.rank;
    return dispatch<AtomicRun>(a, bf16, s, st);
}

}  // namespace pasta
