// Device helpers and launch interfaces shared by the gfx950 kernels of libpasta.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace pasta {

constexpr int kMaxOrder = 8;
constexpr int kWave = 64;
constexpr uint32_t kNoRow = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// Cross-lane helpers (wave64). DPP patterns stay inside a row of 16 lanes.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

// Sum of v over aligned groups of L consecutive lanes; every lane of the
// group receives the total. The butterfly order is fixed, so the result is
// deterministic.
template <int L>
__device__ __forceinline__ float group_sum(float v)
{
    if constexpr (L >= 2) v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
    if constexpr (L >= 4) v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
    if constexpr (L >= 8) v += dpp_mov<0x141>(v);  // row_half_mirror
    if constexpr (L >= 16) v += dpp_mov<0x140>(v); // row_mirror
    if constexpr (L >= 32) v += __shfl_xor(v, 16);
    if constexpr (L >= 64) v += __shfl_xor(v, 32);
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// ---------------------------------------------------------------------------
// The R-wide slice of a factor or output row owned by one lane of a group.
//   contiguous (STRIDED = false): elements j*VEC .. j*VEC+VEC-1, one vector
//       load (float4 for fp32 VEC=4, 16 bytes of bf16 for VEC=8); R, ld and
//       the base pointer are multiples of VEC / 16-byte aligned;
//   strided (STRIDED = true, L = 64): elements j + 64*e, e < VEC, scalar
//       loads; any R <= 64*VEC, any ld, any alignment.
// ---------------------------------------------------------------------------
template <typename FT, int VEC, bool STRIDED>
struct Slice {
    static_assert(std::is_same<FT, float>::value || std::is_same<FT, uint16_t>::value, "fp32 or bf16 bits");
    // words of packed storage per lane
    static constexpr int kWords = STRIDED ? VEC : (VEC * (int)sizeof(FT) + 3) / 4;
    struct Packed {
        uint32_t w[kWords];
    };

    __device__ __forceinline__ static bool active(int j, uint32_t R)
    {
        return STRIDED ? (uint32_t)j < R : (uint32_t)(j * VEC) < R;
    }

    __device__ __forceinline__ static void load(const FT *__restrict__ row, int j, uint32_t R, Packed &p)
    {
        if constexpr (STRIDED) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const uint32_t c = (uint32_t)j + 64u * e;
                if constexpr (std::is_same<FT, float>::value)
                    p.w[e] = c < R ? __float_as_uint(row[c]) : 0u;
                else
                    p.w[e] = c < R ? ((uint32_t)row[c] << 16) : 0u;
            }
        } else if constexpr (std::is_same<FT, float>::value && VEC == 4) {
            const uint4 t = *reinterpret_cast<const uint4 *>(row + j * 4);
            p.w[0] = t.x; p.w[1] = t.y; p.w[2] = t.z; p.w[3] = t.w;
        } else if constexpr (std::is_same<FT, uint16_t>::value && VEC == 8) {
            const uint4 t = *reinterpret_cast<const uint4 *>(row + j * 8);
            p.w[0] = t.x; p.w[1] = t.y; p.w[2] = t.z; p.w[3] = t.w;
        } else {
            static_assert(STRIDED, "contiguous slices are float4 or 8 x bf16");
        }
    }

    __device__ __forceinline__ static void unpack(const Packed &p, float (&v)[VEC])
    {
        if constexpr (STRIDED || std::is_same<FT, float>::value) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[e] = __uint_as_float(p.w[e]);
        } else {
#pragma unroll
            for (int e = 0; e < VEC / 2; ++e) {
                v[2 * e] = __uint_as_float(p.w[e] << 16);
                v[2 * e + 1] = __uint_as_float(p.w[e] & 0xFFFF0000u);
            }
        }
    }

    __device__ __forceinline__ static void load_f(const FT *__restrict__ row, int j, uint32_t R, float (&v)[VEC])
    {
        Packed p;
        load(row, j, R, p);
        unpack(p, v);
    }
};

// Store VEC fp32 values of lane j into an output row (same lane mapping).
template <int VEC, bool STRIDED>
__device__ __forceinline__ void store_slice(float *__restrict__ row, int j, uint32_t R, const float (&v)[VEC],
                                            float alpha)
{
    if constexpr (STRIDED) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const uint32_t c = (uint32_t)j + 64u * e;
            if (c < R) row[c] = alpha * v[e];
        }
    } else {
        static_assert(VEC % 4 == 0, "contiguous stores are float4");
#pragma unroll
        for (int e = 0; e < VEC; e += 4) {
            float4 t;
            t.x = alpha * v[e];
            t.y = alpha * v[e + 1];
            t.z = alpha * v[e + 2];
            t.w = alpha * v[e + 3];
            *reinterpret_cast<float4 *>(row + j * VEC + e) = t;
        }
    }
}

// The same with non-temporal stores (contiguous slices), for outputs written
// once and too large to stay in cache: TTM's fiber rows, MTTKRP on many short rows.
template <int VEC, bool STRIDED>
__device__ __forceinline__ void store_slice_nt(float *__restrict__ row, int j, uint32_t R, const float (&v)[VEC],
                                               float alpha)
{
    if constexpr (STRIDED) {
        store_slice<VEC, STRIDED>(row, j, R, v, alpha);
    } else {
        typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int e = 0; e < VEC; e += 4) {
            const f4 t = {alpha * v[e], alpha * v[e + 1], alpha * v[e + 2], alpha * v[e + 3]};
            __builtin_nontemporal_store(t, reinterpret_cast<f4 *>(row + j * VEC + e));
        }
    }
}

// ---------------------------------------------------------------------------
// Launch interfaces (host side). Every pointer is device memory.
// ---------------------------------------------------------------------------
struct KernelShape {
    int vec;       // fp32 elements per lane (4 / 8 contiguous, or 4 strided)
    int lanes;     // L, lanes per group (power of two, <= 64)
    bool strided;  // generic path
};

struct MttkrpLaunch {
    const uint32_t *row;             // mode-n index in mode-n order
    const uint32_t *idx[kMaxOrder];  // other modes' indices in mode-n order (order-1 used)
    const void *fac[kMaxOrder];      // matching factors
    const void *facn;                // factor of mode n (fused CP gradient)
    const float *vals;               // values in mode-n order, or override in caller order
    const uint32_t *perm;            // non-null: value of position p is vals[perm[p]]
    float *out;
    float *part;                     // partial rows: 2 per chunk, stride ldp
    double *loss_part;               // fused: one fp64 partial per chunk (nullable)
    uint64_t nnz;
    uint32_t ldf, ldo, ldp, rank;
    uint32_t sub;                    // nonzeros per group per chunk (wave form: per chunk)
    uint32_t nchunks;
    uint32_t keys;                   // leading factors whose indices are sort keys of the stream
    uint32_t lds_rows;               // rows of the last factor, read from LDS (0: none)
    uint32_t *flag;                  // set to 2 if the stream is found out of order (nullable)
    float alpha;
    bool wave;                       // the wave-run form (contiguous shapes)
};

struct SampleLaunch {
    const uint32_t *inds[kMaxOrder];  // caller order
    const void *fac[kMaxOrder];
    const float *vals;                // caller-order values (residual mode)
    float *out;                       // mhat, or resid when vals != null (nullable in loss mode)
    double *loss_part;                // per-block partial of 1/2 sum resid^2 (nullable)
    uint64_t nnz;
    uint32_t ldf, rank;
    uint32_t tiles_per_wave;
};

struct AtomicLaunch {
    const uint32_t *row;
    const uint32_t *idx[kMaxOrder];
    const void *fac[kMaxOrder];
    const float *vals;
    float *out;
    uint64_t nnz;
    uint32_t ldf, ldo, rank;
};

// Per-order launchers (one translation unit per order; nm1 = order - 1).
#define PASTA_DECLARE_ORDER(NM1)                                                                                 \
    hipError_t launch_mttkrp_nm1_##NM1(const MttkrpLaunch &a, bool bf16, KernelShape s, bool fused,             \
                                       hipStream_t st);                                                         \
    hipError_t launch_sample_nm1_##NM1(const SampleLaunch &a, bool bf16, KernelShape s, hipStream_t st);         \
    hipError_t launch_atomic_nm1_##NM1(const AtomicLaunch &a, bool bf16, KernelShape s, hipStream_t st);
PASTA_DECLARE_ORDER(1)
PASTA_DECLARE_ORDER(2)
PASTA_DECLARE_ORDER(3)
PASTA_DECLARE_ORDER(4)
PASTA_DECLARE_ORDER(5)
PASTA_DECLARE_ORDER(6)
PASTA_DECLARE_ORDER(7)
#undef PASTA_DECLARE_ORDER

// Order-independent launchers (preprocess.hip).
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t st);
hipError_t launch_validate(const uint32_t *const *inds, const uint64_t *dims, uint32_t order, uint64_t nnz,
                           uint32_t *flag, hipStream_t st);
hipError_t launch_radix_hist(const uint32_t *keys, uint64_t n, int shift, uint32_t *hist, uint32_t ntiles,
                             hipStream_t st);
// Arrays that travel with the sort key: [0] the permutation (in[0] == NULL
// means the identity), then the other modes' indices and the values' bits.
struct SortPayload {
    const uint32_t *in[kMaxOrder + 1];
    uint32_t *out[kMaxOrder + 1];
    int count;
};
hipError_t launch_radix_scatter(const uint32_t *keys_in, uint64_t n, int shift, const uint32_t *offsets,
                                uint32_t ntiles, uint32_t *keys_out, const SortPayload &pl, hipStream_t st);
hipError_t launch_copy_payload(const uint32_t *keys_in, uint64_t n, uint32_t *keys_out, const SortPayload &pl,
                               hipStream_t st);
hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *partials,
                                 hipStream_t st);
uint64_t scan_partials_count(uint64_t n);
hipError_t launch_identity_sort(const uint32_t *keys, uint64_t n, uint32_t *keys_out, uint32_t *perm_out,
                                hipStream_t st);
hipError_t launch_permute(uint32_t order, uint32_t mode, uint64_t n, const uint32_t *perm,
                          const uint32_t *const *inds_in, const float *vals_in, uint32_t *const *inds_out,
                          float *vals_out, hipStream_t st);
hipError_t launch_rowptr(const uint32_t *sorted_rows, uint64_t n, uint32_t nrows, uint32_t *rowptr,
                         hipStream_t st);
// Rows crossing chunk edges (and empty rows) after the main MTTKRP kernel; blk
// holds ceil(nchunks / 64) level-one partial rows (stride ldp). by_chunk:
// find the split rows from the chunk edges (streams with no empty rows).
hipError_t launch_fixup(const uint32_t *rowptr, const uint32_t *row, uint64_t nnz, uint32_t nrows,
                        const float *part, uint32_t ldp, float *blk, uint64_t nchunks, float *out, uint32_t ldo,
                        uint32_t rank, uint64_t chunk, float alpha, KernelShape s, hipStream_t st,
                        bool by_chunk = false);
hipError_t launch_sum_f64(const double *part, uint32_t n, double *out, hipStream_t st);
hipError_t launch_cast_bf16(const float *src, uint16_t *dst, uint64_t n, hipStream_t st);
hipError_t launch_zero_rows(float *out, uint32_t nrows, uint32_t ldo, uint32_t rank, hipStream_t st);
hipError_t launch_scale(float *x, uint64_t n, const double *alpha, hipStream_t st);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, uint16_t *shadow, uint64_t n, float lr,
                       float b1, float b2, float eps, uint32_t step, hipStream_t st);

// CP-ALS (als.hip)
uint32_t gram_blocks(uint64_t I);
hipError_t launch_gram(const float *U, uint64_t I, uint32_t ld, uint32_t R, float *partial, float *G, hipStream_t st);
hipError_t launch_als_solve(const float *grams, uint32_t order, uint32_t mode, uint32_t R, float *Vinv,
                            uint32_t *flag, hipStream_t st);
hipError_t launch_als_update(const float *M, uint32_t ldm, const float *Vinv, uint32_t R, uint64_t I, float *U,
                             uint32_t ldu, hipStream_t st);
// G <- Gram of U; lambda <- its column norms; U and G <- their normalised forms
hipError_t launch_normalize(float *U, uint64_t I, uint32_t ld, uint32_t R, float *partial, float *G, float *lambda,
                            hipStream_t st);
hipError_t launch_fit(const float *M, uint32_t ldm, const float *U, uint32_t ldu, const float *lambda, uint64_t I,
                      uint32_t R, const float *grams, uint32_t order, double *inner_partial,
                      const double *xnorm2, double *fit, hipStream_t st);
hipError_t launch_sumsq(const float *x, uint64_t n, double *partial, uint32_t nparts, double *out, hipStream_t st);

// Measurement (calibrate.hip): `blocks` workgroups of row gathers, L x 16 bytes
// per row, rows hashed over a power-of-two table; see pasta_probe_gather.
hipError_t launch_gather_probe(const void *table, uint32_t rows, uint32_t lanes, uint32_t share, uint32_t active,
                               uint32_t steps, uint32_t blocks, void *out, hipStream_t st);

// Workgroups are dealt round-robin to the 8 XCDs (workgroup b runs on XCD
// b % 8). This renumbering gives each XCD one contiguous run of logical
// indices (a bijection on [0, nblocks)), so neighbouring pieces of work share
// that XCD's own L2.
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t nblocks)
{
    const uint32_t x = b % 8, i = b / 8;
    const uint32_t q = nblocks / 8, r = nblocks % 8;
    return x * q + (x < r ? x : r) + i;
}

constexpr uint32_t kSortThreads = 256;
constexpr uint32_t kSortItems = 16;
constexpr uint32_t kSortTile = kSortThreads * kSortItems;  // keys per sort tile
constexpr int kRadixBits = 8;
constexpr uint32_t kRadix = 1u << kRadixBits;

}  // namespace pasta
