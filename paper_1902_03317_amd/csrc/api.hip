// Host side of libpasta: argument checks, workspace layout, kernel choice
// and stream ordering behind the C ABI declared in include/pasta.h.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "../../include/pasta.h"
#include "common.h"
#include "elementwise.h"
#include "fibers.h"

using namespace pasta;

struct pasta_coo {
    uint32_t order;
    uint64_t nnz;
    uint64_t dims[kMaxOrder];
    const uint32_t *inds[kMaxOrder];  // caller order (caller-owned)
    const float *vals;
    uint32_t *flag;  // device word in the workspace: 0 after a good index check; kernels set
                     // it to 2 if they find the preprocessed stream inconsistent (sticky)
    struct Mode {
        uint32_t *sinds[kMaxOrder];  // sorted copies; sinds[n] holds i_n itself
        float *svals;
        uint32_t *perm;
        uint32_t *rowptr;
    } mode[kMaxOrder];
};

// Mode-n fibers of a tensor (pasta_fibers_create): the nonzeros reordered so
// that each fiber is one contiguous run, with the run offsets and coordinates.
struct pasta_fibers {
    uint32_t order, mode;
    uint64_t nnz, nfibs, dim;
    const uint32_t *fid;   // fiber of each nonzero, fiber order
    const uint32_t *idx;   // i_mode of each nonzero, fiber order
    const uint32_t *hot;   // the same indices relabelled by decreasing count (TTV gathers)
    const uint32_t *old_of_new;  // [dim] the index a relabelled index stands for
    const float *vals;     // values, fiber order
    const uint32_t *perm;  // caller position of each nonzero, fiber order
    const uint32_t *fptr;  // [nfibs + 1]
    const uint32_t *coords[kMaxOrder];  // [order - 1][nfibs], modes in order without `mode`
};

namespace {

thread_local int g_last_hip_error = 0;
// events armed by pasta_arm_kernel_events for the next main kernel launch on this thread
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

#define HIPCHK(expr)                                                                                             \
    do {                                                                                                         \
        hipError_t e_ = (expr);                                                                                  \
        if (e_ != hipSuccess) {                                                                                  \
            g_last_hip_error = (int)e_;                                                                          \
            return PASTA_EHIP;                                                                                   \
        }                                                                                                        \
    } while (0)

constexpr size_t kAlign = 256;
constexpr uint32_t kSub = 256;           // nonzeros per lane group per chunk (run form)
constexpr uint32_t kSampleTilesPerWave = 16;
constexpr uint32_t kWaveChunk = 2048;    // nonzeros per chunk of the wave-run form
constexpr uint64_t kWaveMinRowLen = 48;  // average nonzeros per row from which it is chosen
// LDS a factor may take in the wave-run form: three workgroups of it fit a CU's 160 KiB
// (the occupancy its registers allow at R = 32..64)
constexpr uint64_t kLdsFactorBytes = 52u << 10;
int g_mttkrp_form = 0;                   // 0 automatic, 1 run form, 2 wave-run form
int g_last_form = 0;                     // form of the most recent MTTKRP main-kernel launch

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct CooLayout {
    size_t sinds[kMaxOrder][kMaxOrder];
    size_t svals[kMaxOrder], perm[kMaxOrder], rowptr[kMaxOrder];
    size_t flag, hist, scanpart;
    size_t tmp[2][kMaxOrder + 2];  // two ping-pong sets: key, permutation, N-1 indices, values
    size_t total;
    uint32_t ntiles;
};

bool checked_add(size_t &off, size_t bytes)
{
    const size_t a = align_up(bytes);
    if (off > SIZE_MAX - a) return false;
    off += a;
    return true;
}

bool make_layout(uint32_t N, const uint64_t *dims, uint64_t nnz, CooLayout &L)
{
    size_t off = 0;
    const size_t m4 = (size_t)nnz * 4;
    for (uint32_t n = 0; n < N; ++n) {
        for (uint32_t k = 0; k < N; ++k) {
            L.sinds[n][k] = off;
            if (!checked_add(off, m4)) return false;
        }
        L.svals[n] = off;
        if (!checked_add(off, m4)) return false;
        L.perm[n] = off;
        if (!checked_add(off, m4)) return false;
        L.rowptr[n] = off;
        if (!checked_add(off, ((size_t)dims[n] + 1) * 4)) return false;
    }
    L.flag = off;
    checked_add(off, 4);
    // ping-pong buffers are needed only when some mode sorts in more than one pass
    bool multi_pass = false;
    for (uint32_t n = 0; n < N; ++n) multi_pass = multi_pass || dims[n] > (1ull << kRadixBits);
    for (int set = 0; set < 2; ++set)
        for (uint32_t a = 0; a < N + 2; ++a) {
            L.tmp[set][a] = off;
            if (multi_pass && !checked_add(off, m4)) return false;
        }
    L.ntiles = (uint32_t)std::max<uint64_t>(1, (nnz + kSortTile - 1) / kSortTile);
    const uint64_t hist_n = (uint64_t)kRadix * L.ntiles;
    L.hist = off;
    checked_add(off, hist_n * 4);
    L.scanpart = off;
    if (!checked_add(off, scan_partials_count(hist_n) * 4 + 4)) return false;
    L.total = off;
    return true;
}

pasta_status check_shape(uint32_t N, const uint64_t *dims, uint64_t nnz)
{
    if (!dims) return PASTA_EINVAL;
    if (N < 2 || N > (uint32_t)kMaxOrder) return PASTA_EUNSUPPORTED;
    if (nnz >= (1ull << 32)) return PASTA_EUNSUPPORTED;
    for (uint32_t k = 0; k < N; ++k) {
        if (dims[k] == 0) return PASTA_EINVAL;
        if (dims[k] > (1ull << 31)) return PASTA_EUNSUPPORTED;
    }
    return PASTA_OK;
}

int key_bits(uint64_t dim)
{
    int b = 0;
    while (b < 32 && (1ull << b) < dim) ++b;
    return b;  // indices are < dim <= 2^b
}

uint32_t next_pow2(uint32_t x)
{
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Kernel shape for a rank / dtype / leading-dimension combination.
bool choose_shape(pasta_dtype dt, uint32_t R, uint32_t ldf, uint32_t ldo, const void *const *facs, uint32_t nf,
                  const void *out, KernelShape &s)
{
    bool al = out == nullptr || aligned16(out);
    for (uint32_t k = 0; k < nf; ++k) al = al && (facs[k] == nullptr || aligned16(facs[k]));
    const uint32_t vec = dt == PASTA_F32 ? 4 : 8;
    if (al && R % vec == 0 && ldf % vec == 0 && ldo % 4 == 0 && R / vec <= 16) {
        s.vec = (int)vec;
        s.lanes = (int)next_pow2(R / vec);
        s.strided = false;
        return true;
    }
    if (R <= 256) {
        s.vec = 4;
        s.lanes = 64;
        s.strided = true;
        return true;
    }
    return false;
}

// The segmented kernel's contiguous shapes address factor rows with 32-bit byte
// offsets (row index times row bytes in a 24-bit multiply): every factor must
// have fewer than 2^24 rows and fit in 4 GiB, else the generic strided shape
// (64-bit addressing) runs instead.
bool rows_fit32(uint64_t max_rows, uint32_t ldf, pasta_dtype dt)
{
    const uint64_t row_bytes = (uint64_t)ldf * (dt == PASTA_BF16 ? 2u : 4u);
    return max_rows < (1ull << 24) && row_bytes < (1ull << 24) && max_rows * row_bytes <= (1ull << 32);
}

bool segmented_shape(pasta_dtype dt, uint32_t R, uint32_t ldf, uint32_t ldo, const void *const *facs, uint32_t nf,
                     const void *out, uint64_t max_rows, KernelShape &s)
{
    if (!choose_shape(dt, R, ldf, ldo, facs, nf, out, s)) return false;
    if (!s.strided && !rows_fit32(max_rows, ldf, dt)) {
        if (R > 256) return false;
        s.vec = 4;
        s.lanes = 64;
        s.strided = true;
    }
    return true;
}

uint64_t max_dim(const pasta_coo *X)
{
    uint64_t m = 0;
    for (uint32_t k = 0; k < X->order; ++k) m = std::max<uint64_t>(m, X->dims[k]);
    return m;
}

hipError_t launch_mttkrp(uint32_t N, const MttkrpLaunch &l, bool bf16, KernelShape s, bool fused, hipStream_t st)
{
    switch (N - 1) {
    case 1: return launch_mttkrp_nm1_1(l, bf16, s, fused, st);
    case 2: return launch_mttkrp_nm1_2(l, bf16, s, fused, st);
    case 3: return launch_mttkrp_nm1_3(l, bf16, s, fused, st);
    case 4: return launch_mttkrp_nm1_4(l, bf16, s, fused, st);
    case 5: return launch_mttkrp_nm1_5(l, bf16, s, fused, st);
    case 6: return launch_mttkrp_nm1_6(l, bf16, s, fused, st);
    case 7: return launch_mttkrp_nm1_7(l, bf16, s, fused, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sample(uint32_t N, const SampleLaunch &l, bool bf16, KernelShape s, hipStream_t st)
{
    switch (N - 1) {
    case 1: return launch_sample_nm1_1(l, bf16, s, st);
    case 2: return launch_sample_nm1_2(l, bf16, s, st);
    case 3: return launch_sample_nm1_3(l, bf16, s, st);
    case 4: return launch_sample_nm1_4(l, bf16, s, st);
    case 5: return launch_sample_nm1_5(l, bf16, s, st);
    case 6: return launch_sample_nm1_6(l, bf16, s, st);
    case 7: return launch_sample_nm1_7(l, bf16, s, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_atomic(uint32_t N, const AtomicLaunch &l, bool bf16, KernelShape s, hipStream_t st)
{
    switch (N - 1) {
    case 1: return launch_atomic_nm1_1(l, bf16, s, st);
    case 2: return launch_atomic_nm1_2(l, bf16, s, st);
    case 3: return launch_atomic_nm1_3(l, bf16, s, st);
    case 4: return launch_atomic_nm1_4(l, bf16, s, st);
    case 5: return launch_atomic_nm1_5(l, bf16, s, st);
    case 6: return launch_atomic_nm1_6(l, bf16, s, st);
    case 7: return launch_atomic_nm1_7(l, bf16, s, st);
    default: return hipErrorInvalidValue;
    }
}

// Geometry of one MTTKRP call: chunking of the mode-ordered stream and the
// partial-row scratch it needs.
struct MttkrpPlan {
    KernelShape shape;
    uint32_t sub, nchunks, ldp;
    uint64_t chunk;
    size_t blk_offset;  // level-one fixup sums follow the chunk partials
    size_t part_bytes;
};

// The wave-run form on long rows (contiguous shapes only), unless a form is forced.
bool use_wave(const KernelShape &s, uint64_t nnz, uint64_t rows)
{
    if (s.strided || g_mttkrp_form == 1) return false;
    return g_mttkrp_form == 2 || nnz >= kWaveMinRowLen * rows;
}

bool plan_mttkrp(uint64_t nnz, uint32_t rank, KernelShape s, MttkrpPlan &p, bool wave = false)
{
    p.shape = s;
    const uint32_t G = 64u / (uint32_t)s.lanes;
    p.sub = wave ? kWaveChunk : kSub;
    p.chunk = wave ? (uint64_t)kWaveChunk : (uint64_t)p.sub * G;
    const uint64_t nch = (nnz + p.chunk - 1) / p.chunk;
    if (nch > 0x7FFFFFFFull) return false;
    p.nchunks = (uint32_t)nch;
    p.ldp = s.strided ? rank : (rank + 3u) / 4u * 4u;
    p.blk_offset = align_up((size_t)2 * p.nchunks * p.ldp * sizeof(float));
    const size_t nblk = (p.nchunks + 63) / 64;
    p.part_bytes = p.blk_offset + align_up(nblk * p.ldp * sizeof(float));
    return true;
}

// Worst case over kernel shapes for a rank: the contiguous shape has the most chunks.
size_t mttkrp_ws_bound(uint64_t nnz, uint32_t rank, pasta_dtype dt)
{
    const uint32_t vec = dt == PASTA_F32 ? 4 : 8;
    KernelShape shapes[2] = {{(int)vec, (int)next_pow2(std::max<uint32_t>(1, (rank + vec - 1) / vec)), false},
                             {4, 64, true}};
    size_t best = 0;
    for (auto &s : shapes) {
        if (s.lanes > 16 && !s.strided) continue;
        MttkrpPlan p;
        if (plan_mttkrp(nnz, rank, s, p)) best = std::max(best, p.part_bytes);
    }
    return best;
}

size_t sample_blocks(uint64_t nnz)
{
    const uint64_t tiles = (nnz + 63) / 64;
    const uint64_t waves = (tiles + kSampleTilesPerWave - 1) / kSampleTilesPerWave;
    return (size_t)std::max<uint64_t>(1, (waves + 3) / 4);
}

pasta_status check_factors(const pasta_coo *X, const void *const *facs, uint32_t skip_mode)
{
    if (!facs) return PASTA_EINVAL;
    for (uint32_t k = 0; k < X->order; ++k)
        if (k != skip_mode && facs[k] == nullptr) return PASTA_EINVAL;
    return PASTA_OK;
}

pasta_status run_mttkrp(const pasta_coo *X, uint32_t mode, const void *const *facs, pasta_dtype dt, uint32_t rank,
                        uint32_t ldf, const float *ovr, float alpha, float *out, uint32_t ldo, void *work,
                        size_t work_bytes, bool fused, double *loss_part, hipStream_t st)
{
    const void *fl[kMaxOrder];
    uint32_t nf = 0;
    for (uint32_t k = 0; k < X->order; ++k)
        if (k != mode || fused) fl[nf++] = facs[k];
    KernelShape s;
    if (!segmented_shape(dt, rank, ldf, ldo, fl, nf, out, max_dim(X), s)) return PASTA_EUNSUPPORTED;
    const bool wave = use_wave(s, X->nnz, X->dims[mode]);
    if (X->nnz > 0) g_last_form = wave ? 2 : 1;
    MttkrpPlan p;
    if (!plan_mttkrp(X->nnz, rank, s, p, wave)) return PASTA_EUNSUPPORTED;
    if (p.part_bytes > 0 && (work == nullptr || work_bytes < p.part_bytes || ((uintptr_t)work % kAlign) != 0))
        return PASTA_EWORKSPACE;
    const auto &md = X->mode[mode];
    MttkrpLaunch l{};
    l.row = md.sinds[mode];
    // the other modes in the order of the mode order's keys after i_n: n-1, n-2, ...
    // (cyclically), so the factors of the second and third keys come first (the wave-run
    // kernel reuses their rows along runs). Mode n's order is lexicographic in
    // (i_n, i_{n-1}, ..., i_0) and then i_{N-1}: mode 0's has one key after i_0 (then
    // caller position), every other mode's at least two.
    uint32_t qmode[kMaxOrder];
    for (uint32_t q = 0; q + 1 < X->order; ++q) {
        const uint32_t k = (mode + X->order - 1 - q) % X->order;
        l.idx[q] = md.sinds[k];
        l.fac[q] = facs[k];
        qmode[q] = k;
    }
    l.keys = mode == 0 ? 1u : std::min<uint32_t>(2u, X->order - 1);
    // Orders 3-5, both kernel forms: the smallest factor after the second key whose rows
    // fit kLdsFactorBytes moves to the last place and is read from LDS (the kernel stages
    // it per workgroup). The second key's factor stays first even when it is small: its
    // reuse along runs in the wave-run form did as well as LDS would (measured on the
    // order-4 and -5 tensors).
    l.lds_rows = 0;
    if (!ovr && !s.strided && (s.lanes == 8 || s.lanes == 16) && X->order >= 3 && X->order <= 5) {
        const uint32_t last = X->order - 2;
        uint32_t best = 0;
        for (uint32_t q = 1; q <= last; ++q) {
            const uint64_t bytes = X->dims[qmode[q]] * (uint64_t)s.lanes * 16u;
            if (bytes <= kLdsFactorBytes && (best == 0 || X->dims[qmode[q]] < X->dims[qmode[best]])) best = q;
        }
        if (best) {
            std::swap(l.idx[best], l.idx[last]);
            std::swap(l.fac[best], l.fac[last]);
            std::swap(qmode[best], qmode[last]);
            if (best == 1 || last == 1) l.keys = 1;  // factor 1 is no longer the third key
            l.lds_rows = (uint32_t)X->dims[qmode[last]];
        }
    }
    l.flag = X->flag;
    l.facn = fused ? facs[mode] : nullptr;
    l.vals = ovr ? ovr : md.svals;
    l.perm = ovr ? md.perm : nullptr;
    l.out = out;
    l.part = static_cast<float *>(work);
    l.loss_part = loss_part;
    l.nnz = X->nnz;
    l.ldf = ldf;
    l.ldo = ldo;
    l.ldp = p.ldp;
    l.rank = rank;
    l.sub = p.sub;
    l.nchunks = p.nchunks;
    l.alpha = alpha;
    l.wave = wave;
    if (X->nnz > 0) {
        hipEvent_t e0 = g_ev_start, e1 = g_ev_stop;
        g_ev_start = g_ev_stop = nullptr;
        if (e0) HIPCHK(hipEventRecord(e0, st));
        HIPCHK(launch_mttkrp(X->order, l, dt == PASTA_BF16, s, fused, st));
        if (e1) HIPCHK(hipEventRecord(e1, st));
    }
    float *blk = reinterpret_cast<float *>(static_cast<char *>(work) + p.blk_offset);
    HIPCHK(launch_fixup(md.rowptr, md.sinds[mode], X->nnz, (uint32_t)X->dims[mode], l.part, p.ldp, blk, p.nchunks, out,
                        ldo, rank, p.chunk, alpha, s, st));
    return PASTA_OK;
}

// Workspace of a fiber layout: two ping-pong SoA sets for the sort (N index
// arrays, the values, the permutation), the fiber ids, fptr, coordinates and
// the head flags and their scan.
struct FiberLayout {
    size_t set[2][kMaxOrder + 2];
    size_t fid, fptr, coords[kMaxOrder], head, excl, nfibs, hist, scanpart, total;
    size_t hot, old_of_new, new_of_old, rkey[2], rperm[2];  // relabelling of the mode's indices
    uint32_t ntiles, ntiles_dim;
};

bool make_fiber_layout(uint32_t N, uint64_t nnz, uint64_t dim, FiberLayout &L)
{
    size_t off = 0;
    const size_t m4 = (size_t)nnz * 4;
    for (int s = 0; s < 2; ++s)
        for (uint32_t a = 0; a < N + 2; ++a) {
            L.set[s][a] = off;
            if (!checked_add(off, m4)) return false;
        }
    L.fid = off;
    if (!checked_add(off, m4)) return false;
    L.fptr = off;
    if (!checked_add(off, m4 + 4)) return false;
    for (uint32_t q = 0; q + 1 < N; ++q) {
        L.coords[q] = off;
        if (!checked_add(off, m4)) return false;
    }
    L.head = off;
    if (!checked_add(off, m4)) return false;
    L.excl = off;
    if (!checked_add(off, m4)) return false;
    L.nfibs = off;
    checked_add(off, 4);
    L.hot = off;
    if (!checked_add(off, m4)) return false;
    const size_t d4 = (size_t)dim * 4;
    L.old_of_new = off;
    if (!checked_add(off, d4)) return false;
    L.new_of_old = off;
    if (!checked_add(off, d4)) return false;
    for (int s = 0; s < 2; ++s) {
        L.rkey[s] = off;
        if (!checked_add(off, d4)) return false;
        L.rperm[s] = off;
        if (!checked_add(off, d4)) return false;
    }
    L.ntiles = (uint32_t)std::max<uint64_t>(1, (nnz + kSortTile - 1) / kSortTile);
    L.ntiles_dim = (uint32_t)std::max<uint64_t>(1, (dim + kSortTile - 1) / kSortTile);
    const uint64_t hist_n = (uint64_t)kRadix * std::max(L.ntiles, L.ntiles_dim);
    L.hist = off;
    if (!checked_add(off, hist_n * 4)) return false;
    L.scanpart = off;
    if (!checked_add(off, (std::max(scan_partials_count(hist_n), scan_partials_count(nnz)) + 1) * 4)) return false;
    L.total = off;
    return true;
}

// Scratch of a TTV call: two partial slots per chunk, the level-one fixup
// sums, then the vector in relabelled index order.
struct TtvPlan {
    uint32_t nchunks;
    size_t blk_offset, vhot_offset, part_bytes;
};

TtvPlan plan_ttv(uint64_t nnz, uint64_t dim)
{
    TtvPlan p;
    p.nchunks = (uint32_t)((nnz + kTtvChunk - 1) / kTtvChunk);
    p.blk_offset = align_up((size_t)2 * p.nchunks * sizeof(float));
    p.vhot_offset = p.blk_offset + align_up((size_t)((p.nchunks + 63) / 64) * sizeof(float));
    p.part_bytes = p.vhot_offset + align_up((size_t)dim * sizeof(float));
    return p;
}

// Workspace of a general element-wise operation over nnz_x + nnz_y entries:
// two ping-pong SoA sets (N indices, values, positions) for the sort, then
// run heads / run ids / per-run value, position, keep flag and output slot.
struct TewLayout {
    size_t set[2][kMaxOrder + 2];
    size_t head, run_of, run_val, run_pos, run_keep, out_of, flag, count, hist, scanpart, total;
    uint32_t ntiles;
};

bool make_tew_layout(uint32_t N, uint64_t M, TewLayout &L)
{
    size_t off = 0;
    const size_t m4 = (size_t)M * 4;
    for (int s = 0; s < 2; ++s)
        for (uint32_t a = 0; a < N + 2; ++a) {
            L.set[s][a] = off;
            if (!checked_add(off, m4)) return false;
        }
    size_t *arrs[] = {&L.head, &L.run_of, &L.run_val, &L.run_pos, &L.run_keep, &L.out_of};
    for (size_t *a : arrs) {
        *a = off;
        if (!checked_add(off, m4)) return false;
    }
    L.flag = off;
    checked_add(off, 4);
    L.count = off;
    checked_add(off, 4);
    L.ntiles = (uint32_t)std::max<uint64_t>(1, (M + kSortTile - 1) / kSortTile);
    const uint64_t hist_n = (uint64_t)kRadix * L.ntiles;
    L.hist = off;
    if (!checked_add(off, hist_n * 4)) return false;
    L.scanpart = off;
    if (!checked_add(off, (std::max(scan_partials_count(hist_n), scan_partials_count(M)) + 1) * 4)) return false;
    L.total = off;
    return true;
}

}  // namespace

extern "C" {

pasta_status pasta_coo_workspace_bytes(uint32_t order, const uint64_t *dims, uint64_t nnz, size_t *bytes)
{
    if (!bytes) return PASTA_EINVAL;
    pasta_status s = check_shape(order, dims, nnz);
    if (s != PASTA_OK) return s;
    CooLayout L;
    if (!make_layout(order, dims, nnz, L)) return PASTA_EUNSUPPORTED;
    *bytes = L.total;
    return PASTA_OK;
}

pasta_status pasta_coo_create(uint32_t order, const uint64_t *dims, uint64_t nnz, const uint32_t *const *d_inds,
                              const float *d_vals, void *d_workspace, size_t workspace_bytes, void *stream,
                              pasta_coo **out)
{
    if (!out) return PASTA_EINVAL;
    *out = nullptr;
    pasta_status s = check_shape(order, dims, nnz);
    if (s != PASTA_OK) return s;
    if (nnz > 0) {
        if (!d_inds || !d_vals) return PASTA_EINVAL;
        for (uint32_t k = 0; k < order; ++k)
            if (!d_inds[k]) return PASTA_EINVAL;
    }
    CooLayout L;
    if (!make_layout(order, dims, nnz, L)) return PASTA_EUNSUPPORTED;
    if (!d_workspace || workspace_bytes < L.total || ((uintptr_t)d_workspace % kAlign) != 0)
        return PASTA_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(d_workspace);
    auto at = [&](size_t off) { return reinterpret_cast<uint32_t *>(base + off); };

    pasta_coo *X = new (std::nothrow) pasta_coo();
    if (!X) return PASTA_EINVAL;
    X->order = order;
    X->nnz = nnz;
    for (uint32_t k = 0; k < order; ++k) {
        X->dims[k] = dims[k];
        X->inds[k] = nnz ? d_inds[k] : nullptr;
    }
    X->vals = d_vals;
    X->flag = at(L.flag);
    for (uint32_t n = 0; n < order; ++n) {
        for (uint32_t k = 0; k < order; ++k) X->mode[n].sinds[k] = at(L.sinds[n][k]);
        X->mode[n].svals = reinterpret_cast<float *>(base + L.svals[n]);
        X->mode[n].perm = at(L.perm[n]);
        X->mode[n].rowptr = at(L.rowptr[n]);
    }
    auto fail = [&](pasta_status e) {
        delete X;
        return e;
    };
#define HIPCHK_X(expr)                                                                                           \
    do {                                                                                                         \
        hipError_t e_ = (expr);                                                                                  \
        if (e_ != hipSuccess) {                                                                                  \
            g_last_hip_error = (int)e_;                                                                          \
            return fail(PASTA_EHIP);                                                                             \
        }                                                                                                        \
    } while (0)

    uint32_t *flag = at(L.flag);
    HIPCHK_X(launch_fill_u32(flag, 0u, 1, st));
    HIPCHK_X(launch_validate(d_inds, dims, order, nnz, flag, st));
    uint32_t *hist = at(L.hist);
    uint32_t *scanpart = at(L.scanpart);
    const uint64_t hist_n = (uint64_t)kRadix * L.ntiles;
    // Mode orders, chained: mode n's order is the stable sort by i_n of mode
    // n-1's order, so within a row of mode n the nonzeros are ordered by i_{n-1}
    // (then i_{n-2}, ...). The chain starts from mode N-1 sorted out of the
    // caller's order (written into mode N-1's buffers, which its own final sort
    // later overwrites): N + 1 stable sorts in all.
    if (nnz > 0) {
        for (uint32_t stage = 0; stage <= order; ++stage) {
            const uint32_t n = stage == 0 ? order - 1 : stage - 1;
            auto &md = X->mode[n];
            const uint32_t *src_key;
            SortPayload pl{};
            int cnt = 1;
            if (stage == 0) {  // from the caller's arrays, identity permutation
                src_key = d_inds[n];
                pl.in[0] = nullptr;
                for (uint32_t k = 0; k < order; ++k)
                    if (k != n) pl.in[cnt++] = d_inds[k];
                pl.in[cnt++] = reinterpret_cast<const uint32_t *>(d_vals);
            } else {  // from the previous mode's sorted copy; permutations compose
                const auto &pm = X->mode[(n + order - 1) % order];
                src_key = pm.sinds[n];
                pl.in[0] = pm.perm;
                for (uint32_t k = 0; k < order; ++k)
                    if (k != n) pl.in[cnt++] = pm.sinds[k];
                pl.in[cnt++] = reinterpret_cast<const uint32_t *>(pm.svals);
            }
            pl.count = cnt;
            auto set_final = [&]() {
                int c = 1;
                pl.out[0] = md.perm;
                for (uint32_t k = 0; k < order; ++k)
                    if (k != n) pl.out[c++] = md.sinds[k];
                pl.out[c++] = reinterpret_cast<uint32_t *>(md.svals);
            };
            const int bits = key_bits(dims[n]);
            const int passes = (bits + kRadixBits - 1) / kRadixBits;
            if (passes == 0) {  // a mode of size 1: the order is unchanged
                set_final();
                HIPCHK_X(launch_copy_payload(src_key, nnz, md.sinds[n], pl, st));
                continue;
            }
            const uint32_t *kin = src_key;
            for (int ps = 0; ps < passes; ++ps) {
                const bool last = ps == passes - 1;
                uint32_t *kout;
                if (last) {
                    kout = md.sinds[n];
                    set_final();
                } else {
                    const int set = ps & 1;
                    kout = at(L.tmp[set][0]);
                    for (int c = 0; c < cnt; ++c) pl.out[c] = at(L.tmp[set][c + 1]);
                }
                HIPCHK_X(launch_radix_hist(kin, nnz, ps * kRadixBits, hist, L.ntiles, st));
                HIPCHK_X(launch_exclusive_scan(hist, hist, hist_n, scanpart, st));
                HIPCHK_X(launch_radix_scatter(kin, nnz, ps * kRadixBits, hist, L.ntiles, kout, pl, st));
                kin = kout;
                for (int c = 0; c < cnt; ++c) pl.in[c] = pl.out[c];
            }
        }
    }
    for (uint32_t n = 0; n < order; ++n)
        HIPCHK_X(launch_rowptr(X->mode[n].sinds[n], nnz, (uint32_t)dims[n], X->mode[n].rowptr, st));
    uint32_t host_flag = 0;
    HIPCHK_X(hipMemcpyAsync(&host_flag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIPCHK_X(hipStreamSynchronize(st));
#undef HIPCHK_X
    if (host_flag) return fail(PASTA_ERANGE);
    *out = X;
    return PASTA_OK;
}

pasta_status pasta_coo_check(const pasta_coo *X, void *stream)
{
    if (!X) return PASTA_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint32_t host_flag = 0;
    HIPCHK(hipMemcpyAsync(&host_flag, X->flag, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return host_flag ? PASTA_EINTERNAL : PASTA_OK;
}

pasta_status pasta_coo_destroy(pasta_coo *X)
{
    delete X;
    return PASTA_OK;
}

pasta_status pasta_coo_info(const pasta_coo *X, uint32_t *order, uint64_t *nnz)
{
    if (!X) return PASTA_EINVAL;
    if (order) *order = X->order;
    if (nnz) *nnz = X->nnz;
    return PASTA_OK;
}

pasta_status pasta_coo_mode_view(const pasta_coo *X, uint32_t mode, const uint32_t **d_perm,
                                 const uint32_t **d_rowptr, const uint32_t **d_sorted_inds,
                                 const float **d_sorted_vals)
{
    if (!X || mode >= X->order) return PASTA_EINVAL;
    const auto &md = X->mode[mode];
    if (d_perm) *d_perm = md.perm;
    if (d_rowptr) *d_rowptr = md.rowptr;
    if (d_sorted_inds)
        for (uint32_t k = 0; k < X->order; ++k) d_sorted_inds[k] = md.sinds[k];
    if (d_sorted_vals) *d_sorted_vals = md.svals;
    return PASTA_OK;
}

pasta_status pasta_mttkrp_workspace_bytes(const pasta_coo *X, uint32_t mode, uint32_t rank, pasta_dtype dtype,
                                          size_t *bytes)
{
    if (!X || !bytes || mode >= X->order || rank == 0) return PASTA_EINVAL;
    if (dtype != PASTA_F32 && dtype != PASTA_BF16) return PASTA_EUNSUPPORTED;
    if (rank > 256) return PASTA_EUNSUPPORTED;
    *bytes = mttkrp_ws_bound(X->nnz, rank, dtype);
    return PASTA_OK;
}

pasta_status pasta_mttkrp(const pasta_coo *X, uint32_t mode, const void *const *d_factors, pasta_dtype dtype,
                          uint32_t rank, uint32_t ldf, const float *d_vals_override, float alpha, float *d_out,
                          uint32_t ldo, void *d_work, size_t work_bytes, void *stream)
{
    if (!X || mode >= X->order || rank == 0 || ldf < rank || ldo < rank || !d_out) return PASTA_EINVAL;
    if (dtype != PASTA_F32 && dtype != PASTA_BF16) return PASTA_EUNSUPPORTED;
    if (rank > 256) return PASTA_EUNSUPPORTED;
    pasta_status s = check_factors(X, d_factors, mode);
    if (s != PASTA_OK) return s;
    return run_mttkrp(X, mode, d_factors, dtype, rank, ldf, d_vals_override, alpha, d_out, ldo, d_work, work_bytes,
                      false, nullptr, static_cast<hipStream_t>(stream));
}

}  // extern "C"

// Scratch of pasta_mttkrp_static: a fixed array in the library's code object, so
// that entry point allocates nothing. Every GPU the library runs on holds its own
// copy (PASTA_STATIC_SCRATCH_BYTES) until the process ends. In host code the name
// `scratch` is only a handle for hipGetSymbolAddress; the device address of each
// GPU's copy is looked up once per device and kept in g_scratch_addr.
static __device__ __align__(256) unsigned char scratch[PASTA_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];

// The device address of `scratch` on the device that runs `st` (looked up with that
// device current the first time, then cached).
pasta_status static_scratch(hipStream_t st, void **addr)
{
    int dev = -1, cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (st)
        HIPCHK(hipStreamGetDevice(st, &dev));
    else
        dev = cur;
    if (dev < 0 || dev >= kMaxDevices) return PASTA_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        if (dev != cur) HIPCHK(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (dev != cur) HIPCHK(hipSetDevice(cur));
        HIPCHK(e);
        if (!p) return PASTA_EHIP;
        g_scratch_addr[dev] = p;
    }
    *addr = g_scratch_addr[dev];
    return PASTA_OK;
}
}  // namespace

extern "C" {

pasta_status pasta_mttkrp_static(const pasta_coo *X, uint32_t mode, const void *const *d_factors, pasta_dtype dtype,
                                 uint32_t rank, uint32_t ldf, const float *d_vals_override, float alpha, float *d_out,
                                 uint32_t ldo, void *stream)
{
    if (!X || mode >= X->order || rank == 0 || ldf < rank || ldo < rank || !d_out) return PASTA_EINVAL;
    if (dtype != PASTA_F32 && dtype != PASTA_BF16) return PASTA_EUNSUPPORTED;
    if (rank > 256) return PASTA_EUNSUPPORTED;
    pasta_status s = check_factors(X, d_factors, mode);
    if (s != PASTA_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    void *work = nullptr;
    s = static_scratch(st, &work);
    if (s != PASTA_OK) return s;
    // the same kernels as pasta_mttkrp, their scratch in the static array; a call that
    // needs more than it holds returns PASTA_EWORKSPACE before anything is launched
    return run_mttkrp(X, mode, d_factors, dtype, rank, ldf, d_vals_override, alpha, d_out, ldo, work,
                      PASTA_STATIC_SCRATCH_BYTES, false, nullptr, st);
}

pasta_status pasta_mttkrp_atomic(const pasta_coo *X, uint32_t mode, const void *const *d_factors, pasta_dtype dtype,
                                 uint32_t rank, uint32_t ldf, float *d_out, uint32_t ldo, void *stream)
{
    if (!X || mode >= X->order || rank == 0 || ldf < rank || ldo < rank || !d_out) return PASTA_EINVAL;
    if (dtype != PASTA_F32 && dtype != PASTA_BF16) return PASTA_EUNSUPPORTED;
    if (rank > 256) return PASTA_EUNSUPPORTED;
    pasta_status s = check_factors(X, d_factors, mode);
    if (s != PASTA_OK) return s;
    const void *fl[kMaxOrder];
    uint32_t nf = 0;
    for (uint32_t k = 0; k < X->order; ++k)
        if (k != mode) fl[nf++] = d_factors[k];
    KernelShape sh;
    if (!choose_shape(dtype, rank, ldf, ldo, fl, nf, nullptr, sh)) return PASTA_EUNSUPPORTED;
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIPCHK(launch_zero_rows(d_out, (uint32_t)X->dims[mode], ldo, rank, st));
    AtomicLaunch l{};
    l.row = X->inds[mode];
    uint32_t q = 0;
    for (uint32_t k = 0; k < X->order; ++k) {
        if (k == mode) continue;
        l.idx[q] = X->inds[k];
        l.fac[q] = d_factors[k];
        ++q;
    }
    l.vals = X->vals;
    l.out = d_out;
    l.nnz = X->nnz;
    l.ldf = ldf;
    l.ldo = ldo;
    l.rank = rank;
    if (X->nnz > 0) HIPCHK(launch_atomic(X->order, l, dtype == PASTA_BF16, sh, st));
    return PASTA_OK;
}

static pasta_status sample_common(const pasta_coo *X, const void *const *facs, pasta_dtype dt, uint32_t rank,
                                  uint32_t ldf, const float *vals, float *out, double *loss_part, hipStream_t st)
{
    KernelShape sh;
    if (!choose_shape(dt, rank, ldf, 4, facs, X->order, nullptr, sh)) return PASTA_EUNSUPPORTED;
    SampleLaunch l{};
    for (uint32_t k = 0; k < X->order; ++k) {
        l.inds[k] = X->inds[k];
        l.fac[k] = facs[k];
    }
    l.vals = vals;
    l.out = out;
    l.loss_part = loss_part;
    l.nnz = X->nnz;
    l.ldf = ldf;
    l.rank = rank;
    l.tiles_per_wave = kSampleTilesPerWave;
    HIPCHK(launch_sample(X->order, l, dt == PASTA_BF16, sh, st));
    return PASTA_OK;
}

pasta_status pasta_cp_sample(const pasta_coo *X, const void *const *d_factors, pasta_dtype dtype, uint32_t rank,
                             uint32_t ldf, float *d_mhat, void *stream)
{
    if (!X || rank == 0 || ldf < rank || (!d_mhat && X->nnz > 0)) return PASTA_EINVAL;
    if (dtype != PASTA_F32 && dtype != PASTA_BF16) return PASTA_EUNSUPPORTED;
    if (rank > 256) return PASTA_EUNSUPPORTED;
    pasta_status s = check_factors(X, d_factors, X->order);
    if (s != PASTA_OK) return s;
    if (X->nnz == 0) return PASTA_OK;
    return sample_common(X, d_factors, dtype, rank, ldf, nullptr, d_mhat, nullptr, static_cast<hipStream_t>(stream));
}

pasta_status pasta_cp_workspace_bytes(const pasta_coo *X, uint32_t rank, pasta_dtype dtype, size_t *bytes)
{
    if (!X || !bytes || rank == 0) return PASTA_EINVAL;
    (void)dtype;
    *bytes = align_up(sample_blocks(X->nnz) * sizeof(double));
    return PASTA_OK;
}

pasta_status pasta_cp_residual_loss(const pasta_coo *X, const void *const *d_factors, pasta_dtype dtype,
                                    uint32_t rank, uint32_t ldf, float *d_resid, double *d_loss, void *d_work,
                                    size_t work_bytes, void *stream)
{
    if (!X || rank == 0 || ldf < rank || !d_loss) return PASTA_EINVAL;
    if (dtype != PASTA_F32 && dtype != PASTA_BF16) return PASTA_EUNSUPPORTED;
    if (rank > 256) return PASTA_EUNSUPPORTED;
    pasta_status s = check_factors(X, d_factors, X->order);
    if (s != PASTA_OK) return s;
    const size_t nb = sample_blocks(X->nnz);
    if (!d_work || work_bytes < nb * sizeof(double) || ((uintptr_t)d_work % kAlign) != 0) return PASTA_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *part = static_cast<double *>(d_work);
    if (X->nnz == 0) {
        HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(part), 0u, 2, st));
    } else {
        s = sample_common(X, d_factors, dtype, rank, ldf, X->vals, d_resid, part, st);
        if (s != PASTA_OK) return s;
    }
    HIPCHK(launch_sum_f64(part, X->nnz == 0 ? 1u : (uint32_t)nb, d_loss, st));
    return PASTA_OK;
}

pasta_status pasta_cp_grad_workspace_bytes(const pasta_coo *X, uint32_t rank, pasta_dtype dtype, size_t *bytes)
{
    if (!X || !bytes || rank == 0) return PASTA_EINVAL;
    if (rank > 256) return PASTA_EUNSUPPORTED;
    const size_t part = mttkrp_ws_bound(X->nnz, rank, dtype);
    // one fp64 loss partial per chunk of mode 0 (no chunk is shorter than kSub nonzeros)
    const size_t nlp = (size_t)((X->nnz + kSub - 1) / kSub) + 1;
    *bytes = align_up(part) + align_up(nlp * sizeof(double));
    return PASTA_OK;
}

pasta_status pasta_cp_grad(const pasta_coo *X, const void *const *d_factors, pasta_dtype dtype, uint32_t rank,
                           uint32_t ldf, float alpha, float *const *d_grads, uint32_t ldg, double *d_loss,
                           void *d_work, size_t work_bytes, void *stream)
{
    if (!X || rank == 0 || ldf < rank || ldg < rank || !d_grads) return PASTA_EINVAL;
    if (dtype != PASTA_F32 && dtype != PASTA_BF16) return PASTA_EUNSUPPORTED;
    if (rank > 256) return PASTA_EUNSUPPORTED;
    pasta_status s = check_factors(X, d_factors, X->order);
    if (s != PASTA_OK) return s;
    for (uint32_t n = 0; n < X->order; ++n)
        if (!d_grads[n]) return PASTA_EINVAL;
    size_t need;
    pasta_cp_grad_workspace_bytes(X, rank, dtype, &need);
    if (!d_work || work_bytes < need || ((uintptr_t)d_work % kAlign) != 0) return PASTA_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t part = align_up(mttkrp_ws_bound(X->nnz, rank, dtype));
    double *lp = reinterpret_cast<double *>(static_cast<char *>(d_work) + part);
    for (uint32_t n = 0; n < X->order; ++n) {
        const bool want_loss = d_loss && n == 0;
        s = run_mttkrp(X, n, d_factors, dtype, rank, ldf, nullptr, alpha, d_grads[n], ldg, d_work, part, true,
                       want_loss ? lp : nullptr, st);
        if (s != PASTA_OK) return s;
    }
    if (d_loss) {
        if (X->nnz == 0) {
            HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(lp), 0u, 2, st));
            HIPCHK(launch_sum_f64(lp, 1u, d_loss, st));
        } else {
            // mode 0's chunk count for the shape it ran with
            const void *fl[kMaxOrder];
            for (uint32_t k = 0; k < X->order; ++k) fl[k] = d_factors[k];
            KernelShape sh;
            segmented_shape(dtype, rank, ldf, ldg, fl, X->order, d_grads[0], max_dim(X), sh);
            MttkrpPlan p;
            plan_mttkrp(X->nnz, rank, sh, p, use_wave(sh, X->nnz, X->dims[0]));
            HIPCHK(launch_sum_f64(lp, p.nchunks, d_loss, st));
        }
    }
    return PASTA_OK;
}

pasta_status pasta_cast_f32_to_bf16(const float *d_src, uint16_t *d_dst, uint64_t count, void *stream)
{
    if (count > 0 && (!d_src || !d_dst)) return PASTA_EINVAL;
    HIPCHK(launch_cast_bf16(d_src, d_dst, count, static_cast<hipStream_t>(stream)));
    return PASTA_OK;
}

namespace {
constexpr uint32_t kAlsSumsqParts = 1024;

struct AlsLayout {
    size_t M, mttkrp, grams, partial, vinv, inner, sumsq, xnorm2, flag, total;
};

AlsLayout als_layout(const pasta_coo *X, uint32_t R)
{
    AlsLayout L{};
    uint64_t maxI = 0, maxnb = 0;
    for (uint32_t k = 0; k < X->order; ++k) {
        maxI = std::max<uint64_t>(maxI, X->dims[k]);
        maxnb = std::max<uint64_t>(maxnb, gram_blocks(X->dims[k]));
    }
    size_t off = 0;
    L.mttkrp = off;
    off += align_up(mttkrp_ws_bound(X->nnz, R, PASTA_F32));
    L.M = off;
    off += align_up((size_t)maxI * R * sizeof(float));
    L.grams = off;
    off += align_up((size_t)X->order * R * R * sizeof(float));
    L.partial = off;
    off += align_up((size_t)maxnb * R * R * sizeof(float));
    L.vinv = off;
    off += align_up((size_t)R * R * sizeof(float));
    L.inner = off;
    off += align_up((size_t)maxnb * sizeof(double));
    L.sumsq = off;
    off += align_up((size_t)kAlsSumsqParts * sizeof(double));
    L.xnorm2 = off;
    off += align_up(sizeof(double));
    L.flag = off;
    off += align_up(sizeof(uint32_t));
    L.total = off;
    return L;
}
}  // namespace

pasta_status pasta_cp_als_workspace_bytes(const pasta_coo *X, uint32_t rank, size_t *bytes)
{
    if (!X || !bytes || rank == 0) return PASTA_EINVAL;
    if (rank > 64) return PASTA_EUNSUPPORTED;
    *bytes = als_layout(X, rank).total;
    return PASTA_OK;
}

pasta_status pasta_cp_als_sweep(const pasta_coo *X, float *const *d_factors, uint32_t rank, uint32_t ldf,
                                float *d_lambda, double *d_fit, uint32_t *d_info, void *d_work, size_t work_bytes,
                                void *stream)
{
    if (!X || !d_factors || rank == 0 || ldf < rank || !d_lambda) return PASTA_EINVAL;
    if (rank > 64) return PASTA_EUNSUPPORTED;
    for (uint32_t k = 0; k < X->order; ++k)
        if (!d_factors[k]) return PASTA_EINVAL;
    const AlsLayout L = als_layout(X, rank);
    if (!d_work || work_bytes < L.total || ((uintptr_t)d_work % kAlign) != 0) return PASTA_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(d_work);
    float *M = reinterpret_cast<float *>(w + L.M);
    float *grams = reinterpret_cast<float *>(w + L.grams);
    float *partial = reinterpret_cast<float *>(w + L.partial);
    float *vinv = reinterpret_cast<float *>(w + L.vinv);
    double *inner = reinterpret_cast<double *>(w + L.inner);
    double *xn2 = reinterpret_cast<double *>(w + L.xnorm2);
    uint32_t *flag = d_info ? d_info : reinterpret_cast<uint32_t *>(w + L.flag);
    const uint32_t RR = rank * rank;
    HIPCHK(launch_fill_u32(flag, 0u, 1, st));
    if (d_fit) {
        if (X->nnz > 0) {
            HIPCHK(launch_sumsq(X->vals, X->nnz, reinterpret_cast<double *>(w + L.sumsq), kAlsSumsqParts, xn2, st));
        } else {
            HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(xn2), 0u, 2, st));
        }
    }
    for (uint32_t k = 0; k < X->order; ++k)
        HIPCHK(launch_gram(d_factors[k], X->dims[k], ldf, rank, partial, grams + (uint64_t)k * RR, st));
    const void *facs[kMaxOrder];
    for (uint32_t k = 0; k < X->order; ++k) facs[k] = d_factors[k];
    for (uint32_t n = 0; n < X->order; ++n) {
        pasta_status s = run_mttkrp(X, n, facs, PASTA_F32, rank, ldf, nullptr, 1.0f, M, rank, w + L.mttkrp,
                                    L.M - L.mttkrp, false, nullptr, st);
        if (s != PASTA_OK) return s;
        HIPCHK(launch_als_solve(grams, X->order, n, rank, vinv, flag, st));
        HIPCHK(launch_als_update(M, rank, vinv, rank, X->dims[n], d_factors[n], ldf, st));
        HIPCHK(launch_normalize(d_factors[n], X->dims[n], ldf, rank, partial, grams + (uint64_t)n * RR, d_lambda,
                                st));
    }
    if (d_fit) {
        const uint32_t last = X->order - 1;
        HIPCHK(launch_fit(M, rank, d_factors[last], ldf, d_lambda, X->dims[last], rank, grams, X->order, inner, xn2,
                          d_fit, st));
    }
    return PASTA_OK;
}

pasta_status pasta_set_mttkrp_form(int form)
{
    if (form < 0 || form > 2) return PASTA_EINVAL;
    g_mttkrp_form = form;
    return PASTA_OK;
}

pasta_status pasta_last_mttkrp_form(int *form)
{
    if (!form) return PASTA_EINVAL;
    *form = g_last_form;
    return PASTA_OK;
}

pasta_status pasta_arm_kernel_events(void *ev_start, void *ev_stop)
{
    g_ev_start = static_cast<hipEvent_t>(ev_start);
    g_ev_stop = static_cast<hipEvent_t>(ev_stop);
    return PASTA_OK;
}

pasta_status pasta_probe_gather(const void *d_table, uint32_t rows, uint32_t lanes, uint32_t share, uint32_t active,
                                uint32_t steps, uint32_t blocks, void *d_out, void *stream)
{
    if (!d_table || !d_out || rows == 0 || (rows & (rows - 1)) != 0 || blocks == 0) return PASTA_EINVAL;
    if (lanes != 4 && lanes != 8 && lanes != 16) return PASTA_EUNSUPPORTED;
    const uint32_t G = 64u / lanes;
    if (share == 0 || share > G || (share & (share - 1)) != 0 || steps == 0 || steps % 8 != 0) return PASTA_EINVAL;
    if (active == 0 || active > G) return PASTA_EINVAL;
    if (((uintptr_t)d_table % 16) != 0 || ((uintptr_t)d_out % 16) != 0) return PASTA_EUNSUPPORTED;
    HIPCHK(launch_gather_probe(d_table, rows, lanes, share, active, steps, blocks, d_out,
                               static_cast<hipStream_t>(stream)));
    return PASTA_OK;
}

pasta_status pasta_scale_f32(float *d_x, uint64_t count, const double *d_alpha, void *stream)
{
    if (count > 0 && (!d_x || !d_alpha)) return PASTA_EINVAL;
    HIPCHK(launch_scale(d_x, count, d_alpha, static_cast<hipStream_t>(stream)));
    return PASTA_OK;
}

pasta_status pasta_adam_step(float *d_param, const float *d_grad, float *d_m, float *d_v, uint16_t *d_shadow_bf16,
                             uint64_t count, float lr, float beta1, float beta2, float eps, uint32_t step,
                             void *stream)
{
    if (count > 0 && (!d_param || !d_grad || !d_m || !d_v)) return PASTA_EINVAL;
    if (step == 0 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return PASTA_EINVAL;
    HIPCHK(launch_adam(d_param, d_grad, d_m, d_v, d_shadow_bf16, count, lr, beta1, beta2, eps, step,
                       static_cast<hipStream_t>(stream)));
    return PASTA_OK;
}

pasta_status pasta_fibers_workspace_bytes(const pasta_coo *X, uint32_t mode, size_t *bytes)
{
    if (!X || !bytes || mode >= X->order) return PASTA_EINVAL;
    FiberLayout L;
    if (!make_fiber_layout(X->order, X->nnz, X->dims[mode], L)) return PASTA_EUNSUPPORTED;
    *bytes = L.total;
    return PASTA_OK;
}

pasta_status pasta_fibers_create(const pasta_coo *X, uint32_t mode, void *d_workspace, size_t workspace_bytes,
                                 void *stream, pasta_fibers **out)
{
    if (!out) return PASTA_EINVAL;
    *out = nullptr;
    if (!X || mode >= X->order) return PASTA_EINVAL;
    FiberLayout L;
    if (!make_fiber_layout(X->order, X->nnz, X->dims[mode], L)) return PASTA_EUNSUPPORTED;
    if (!d_workspace || workspace_bytes < L.total || ((uintptr_t)d_workspace % kAlign) != 0)
        return PASTA_EWORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(d_workspace);
    auto at = [&](size_t off) { return reinterpret_cast<uint32_t *>(base + off); };
    const uint32_t N = X->order;
    const uint64_t nnz = X->nnz;
    uint32_t other[kMaxOrder], no = 0;
    for (uint32_t k = 0; k < N; ++k)
        if (k != mode) other[no++] = k;

    // the sorted arrays: N index arrays, values (as bits), permutation
    struct Soa {
        const uint32_t *ind[kMaxOrder];
        const uint32_t *val, *perm;
    };
    const auto &md = X->mode[mode];
    Soa cur;
    for (uint32_t k = 0; k < N; ++k) cur.ind[k] = md.sinds[k];
    cur.val = reinterpret_cast<const uint32_t *>(md.svals);
    cur.perm = md.perm;
    auto set_of = [&](int s, uint32_t *ind[kMaxOrder], uint32_t *&val, uint32_t *&perm) {
        for (uint32_t k = 0; k < N; ++k) ind[k] = at(L.set[s][k]);
        val = at(L.set[s][N]);
        perm = at(L.set[s][N + 1]);
    };
    uint32_t host_nfibs = 0;
    if (nnz > 0) {
        uint32_t *hist = at(L.hist), *scanpart = at(L.scanpart);
        const uint64_t hist_n = (uint64_t)kRadix * L.ntiles;
        // Fiber order: lexicographic in the other modes (in mode order), then
        // i_mode, then caller position. Mode `mode`'s order is sorted by
        // (i_mode, position) among nonzeros that agree elsewhere, so stable LSD
        // sorts by the other modes, the highest mode first, finish it.
        int parity = 0;
        bool moved = false;
        for (int qi = (int)no - 1; qi >= 0; --qi) {
            const uint32_t k = other[qi];
            const int passes = (key_bits(X->dims[k]) + kRadixBits - 1) / kRadixBits;
            for (int ps = 0; ps < passes; ++ps) {
                uint32_t *dind[kMaxOrder], *dval, *dperm;
                set_of(parity, dind, dval, dperm);
                SortPayload pl{};
                int cnt = 0;
                pl.in[cnt] = cur.perm;
                pl.out[cnt++] = dperm;
                for (uint32_t kk = 0; kk < N; ++kk)
                    if (kk != k) {
                        pl.in[cnt] = cur.ind[kk];
                        pl.out[cnt++] = dind[kk];
                    }
                pl.in[cnt] = cur.val;
                pl.out[cnt++] = dval;
                pl.count = cnt;
                HIPCHK(launch_radix_hist(cur.ind[k], nnz, ps * kRadixBits, hist, L.ntiles, st));
                HIPCHK(launch_exclusive_scan(hist, hist, hist_n, scanpart, st));
                HIPCHK(launch_radix_scatter(cur.ind[k], nnz, ps * kRadixBits, hist, L.ntiles, dind[k], pl, st));
                for (uint32_t kk = 0; kk < N; ++kk) cur.ind[kk] = dind[kk];
                cur.val = dval;
                cur.perm = dperm;
                parity ^= 1;
                moved = true;
            }
        }
        if (!moved) {  // every other mode has size 1: the mode order is the fiber order
            uint32_t *dind[kMaxOrder], *dval, *dperm;
            set_of(0, dind, dval, dperm);
            SortPayload pl{};
            int cnt = 0;
            pl.in[cnt] = cur.perm;
            pl.out[cnt++] = dperm;
            for (uint32_t kk = 0; kk < N; ++kk)
                if (kk != mode) {
                    pl.in[cnt] = cur.ind[kk];
                    pl.out[cnt++] = dind[kk];
                }
            pl.in[cnt] = cur.val;
            pl.out[cnt++] = dval;
            pl.count = cnt;
            HIPCHK(launch_copy_payload(cur.ind[mode], nnz, dind[mode], pl, st));
            for (uint32_t kk = 0; kk < N; ++kk) cur.ind[kk] = dind[kk];
            cur.val = dval;
            cur.perm = dperm;
        }
        FiberInds fi{};
        FiberCoords fc{};
        for (uint32_t q = 0; q < no; ++q) {
            fi.p[q] = cur.ind[other[q]];
            fc.p[q] = at(L.coords[q]);
        }
        fi.count = no;
        HIPCHK(launch_fiber_heads(fi, nnz, at(L.head), st));
        HIPCHK(launch_exclusive_scan(at(L.head), at(L.excl), nnz, scanpart, st));
        HIPCHK(launch_fiber_compact(fi, nnz, at(L.head), at(L.excl), at(L.fid), at(L.fptr), fc, at(L.nfibs), st));
        // Relabel i_mode by decreasing count (ties by index): the entries of v that
        // a TTV gathers most often then share cache lines. Same products, same
        // order of summation, so the results are unchanged bit for bit.
        const uint32_t dim = (uint32_t)X->dims[mode];
        const uint64_t hist_d = (uint64_t)kRadix * L.ntiles_dim;
        HIPCHK(launch_count_keys(md.rowptr, dim, nnz, at(L.rkey[0]), st));
        const int rpasses = (key_bits(nnz + 1) + kRadixBits - 1) / kRadixBits;
        const uint32_t *kin = at(L.rkey[0]);
        const uint32_t *pin = nullptr;  // identity
        for (int ps = 0; ps < rpasses; ++ps) {
            const int d = (ps + 1) & 1;
            SortPayload pl{};
            pl.in[0] = pin;
            pl.out[0] = ps == rpasses - 1 ? at(L.old_of_new) : at(L.rperm[d]);
            pl.count = 1;
            HIPCHK(launch_radix_hist(kin, dim, ps * kRadixBits, hist, L.ntiles_dim, st));
            HIPCHK(launch_exclusive_scan(hist, hist, hist_d, scanpart, st));
            HIPCHK(launch_radix_scatter(kin, dim, ps * kRadixBits, hist, L.ntiles_dim, at(L.rkey[d]), pl, st));
            kin = at(L.rkey[d]);
            pin = pl.out[0];
        }
        HIPCHK(launch_invert_perm(at(L.old_of_new), dim, at(L.new_of_old), st));
        HIPCHK(launch_gather_u32(at(L.new_of_old), cur.ind[mode], nnz, at(L.hot), st));
        HIPCHK(hipMemcpyAsync(&host_nfibs, at(L.nfibs), sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    } else {
        HIPCHK(launch_fill_u32(at(L.fptr), 0u, 1, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    pasta_fibers *F = new (std::nothrow) pasta_fibers();
    if (!F) return PASTA_EINVAL;
    F->order = N;
    F->mode = mode;
    F->nnz = nnz;
    F->nfibs = host_nfibs;
    F->dim = X->dims[mode];
    F->fid = at(L.fid);
    F->idx = cur.ind[mode];
    F->hot = at(L.hot);
    F->old_of_new = at(L.old_of_new);
    F->vals = reinterpret_cast<const float *>(cur.val);
    F->perm = cur.perm;
    F->fptr = at(L.fptr);
    for (uint32_t q = 0; q < no; ++q) F->coords[q] = at(L.coords[q]);
    *out = F;
    return PASTA_OK;
}

pasta_status pasta_fibers_destroy(pasta_fibers *F)
{
    delete F;
    return PASTA_OK;
}

pasta_status pasta_fibers_info(const pasta_fibers *F, uint32_t *mode, uint64_t *nfibs)
{
    if (!F) return PASTA_EINVAL;
    if (mode) *mode = F->mode;
    if (nfibs) *nfibs = F->nfibs;
    return PASTA_OK;
}

pasta_status pasta_fibers_view(const pasta_fibers *F, const uint32_t **d_fptr, const uint32_t **d_coords,
                               const uint32_t **d_perm, const uint32_t **d_fid)
{
    if (!F) return PASTA_EINVAL;
    if (d_fptr) *d_fptr = F->fptr;
    if (d_coords)
        for (uint32_t q = 0; q + 1 < F->order; ++q) d_coords[q] = F->coords[q];
    if (d_perm) *d_perm = F->perm;
    if (d_fid) *d_fid = F->fid;
    return PASTA_OK;
}

pasta_status pasta_ttm_workspace_bytes(const pasta_fibers *F, uint32_t rank, pasta_dtype dtype, size_t *bytes)
{
    if (!F || !bytes || rank == 0) return PASTA_EINVAL;
    if (dtype != PASTA_F32 && dtype != PASTA_BF16) return PASTA_EUNSUPPORTED;
    if (rank > (uint32_t)PASTA_MAX_RANK) return PASTA_EUNSUPPORTED;
    *bytes = mttkrp_ws_bound(F->nnz, rank, dtype);
    return PASTA_OK;
}

pasta_status pasta_ttm(const pasta_fibers *F, const void *d_U, pasta_dtype dtype, uint32_t rank, uint32_t ldu,
                       float *d_out, uint32_t ldo, void *d_work, size_t work_bytes, void *stream)
{
    if (!F || rank == 0 || ldu < rank || ldo < rank) return PASTA_EINVAL;
    if (dtype != PASTA_F32 && dtype != PASTA_BF16) return PASTA_EUNSUPPORTED;
    if (rank > (uint32_t)PASTA_MAX_RANK) return PASTA_EUNSUPPORTED;
    if (F->nnz == 0) return PASTA_OK;
    if (!d_U || !d_out) return PASTA_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    KernelShape s;
    if (!segmented_shape(dtype, rank, ldu, ldo, &d_U, 1, d_out, F->dim, s)) return PASTA_EUNSUPPORTED;
    MttkrpPlan p;
    if (!plan_mttkrp(F->nnz, rank, s, p)) return PASTA_EUNSUPPORTED;
    if (!d_work || work_bytes < p.part_bytes || ((uintptr_t)d_work % kAlign) != 0) return PASTA_EWORKSPACE;
    // Alg. 5 as an order-2 segmented product: the fiber id is the output row,
    // i_mode selects the row of U.
    MttkrpLaunch l{};
    l.row = F->fid;
    l.idx[0] = F->idx;
    l.fac[0] = d_U;
    l.vals = F->vals;
    l.out = d_out;
    l.part = static_cast<float *>(d_work);
    l.nnz = F->nnz;
    l.ldf = ldu;
    l.ldo = ldo;
    l.ldp = p.ldp;
    l.rank = rank;
    l.sub = p.sub;
    l.nchunks = p.nchunks;
    l.alpha = 1.0f;
    hipEvent_t e0 = g_ev_start, e1 = g_ev_stop;
    g_ev_start = g_ev_stop = nullptr;
    if (e0) HIPCHK(hipEventRecord(e0, st));
    HIPCHK(launch_mttkrp(2, l, dtype == PASTA_BF16, s, false, st));
    if (e1) HIPCHK(hipEventRecord(e1, st));
    float *blk = reinterpret_cast<float *>(static_cast<char *>(d_work) + p.blk_offset);
    HIPCHK(launch_fixup(F->fptr, F->fid, F->nnz, (uint32_t)F->nfibs, l.part, p.ldp, blk, p.nchunks, d_out, ldo, rank,
                        p.chunk, 1.0f, s, st, true));
    return PASTA_OK;
}

pasta_status pasta_ttv_workspace_bytes(const pasta_fibers *F, size_t *bytes)
{
    if (!F || !bytes) return PASTA_EINVAL;
    *bytes = plan_ttv(F->nnz, F->dim).part_bytes;
    return PASTA_OK;
}

pasta_status pasta_ttv(const pasta_fibers *F, const float *d_v, float *d_out, void *d_work, size_t work_bytes,
                       void *stream)
{
    if (!F) return PASTA_EINVAL;
    if (F->nnz == 0) return PASTA_OK;
    if (!d_v || !d_out) return PASTA_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const TtvPlan p = plan_ttv(F->nnz, F->dim);
    if (!d_work || work_bytes < p.part_bytes || ((uintptr_t)d_work % kAlign) != 0) return PASTA_EWORKSPACE;
    float *part = static_cast<float *>(d_work);
    float *vhot = reinterpret_cast<float *>(static_cast<char *>(d_work) + p.vhot_offset);
    HIPCHK(launch_gather_f32(d_v, F->old_of_new, F->dim, vhot, st));  // v in relabelled order
    hipEvent_t e0 = g_ev_start, e1 = g_ev_stop;
    g_ev_start = g_ev_stop = nullptr;
    if (e0) HIPCHK(hipEventRecord(e0, st));
    HIPCHK(launch_ttv(F->fid, F->hot, F->vals, vhot, d_out, part, F->nnz, p.nchunks, st));
    if (e1) HIPCHK(hipEventRecord(e1, st));
    // fibers crossing chunk edges: the generic one-element-per-lane fixup
    const KernelShape s{4, 64, true};
    float *blk = reinterpret_cast<float *>(static_cast<char *>(d_work) + p.blk_offset);
    HIPCHK(launch_fixup(F->fptr, F->fid, F->nnz, (uint32_t)F->nfibs, part, 1u, blk, p.nchunks, d_out, 1u, 1u,
                        kTtvChunk, 1.0f, s, st, true));
    return PASTA_OK;
}

pasta_status pasta_tew_eq(pasta_ewop op, uint64_t nnz, const float *d_x, const float *d_y, float *d_z, void *stream)
{
    if ((int)op < PASTA_ADD || (int)op > PASTA_DIV) return PASTA_EINVAL;
    if (nnz == 0) return PASTA_OK;
    if (!d_x || !d_y || !d_z) return PASTA_EINVAL;
    HIPCHK(launch_ew((int)op, d_x, d_y, 0.0f, d_z, nnz, static_cast<hipStream_t>(stream)));
    return PASTA_OK;
}

pasta_status pasta_ts(pasta_ewop op, uint64_t nnz, const float *d_x, float s, float *d_y, void *stream)
{
    if ((int)op < PASTA_ADD || (int)op > PASTA_DIV) return PASTA_EINVAL;
    if (nnz == 0) return PASTA_OK;
    if (!d_x || !d_y) return PASTA_EINVAL;
    HIPCHK(launch_ew((int)op, d_x, nullptr, s, d_y, nnz, static_cast<hipStream_t>(stream)));
    return PASTA_OK;
}

pasta_status pasta_tew_workspace_bytes(uint32_t order, uint64_t nnz_x, uint64_t nnz_y, size_t *bytes)
{
    if (!bytes || order < 1) return PASTA_EINVAL;
    if (order > (uint32_t)kMaxOrder || nnz_x + nnz_y >= (1ull << 32)) return PASTA_EUNSUPPORTED;
    TewLayout L;
    if (!make_tew_layout(order, nnz_x + nnz_y, L)) return PASTA_EUNSUPPORTED;
    *bytes = L.total;
    return PASTA_OK;
}

pasta_status pasta_tew(uint32_t order, pasta_ewop op, const uint64_t *dims_x, uint64_t nnz_x,
                       const uint32_t *const *d_inds_x, const float *d_vals_x, const uint64_t *dims_y, uint64_t nnz_y,
                       const uint32_t *const *d_inds_y, const float *d_vals_y, uint64_t *dims_z,
                       uint32_t *const *d_inds_z, float *d_vals_z, uint64_t *nnz_z, void *d_work, size_t work_bytes,
                       void *stream)
{
    if (!dims_x || !dims_y || !dims_z || !nnz_z || order < 1) return PASTA_EINVAL;
    if (op == PASTA_DIV) return PASTA_EUNSUPPORTED;
    if ((int)op < PASTA_ADD || (int)op > PASTA_MUL) return PASTA_EINVAL;
    if (order > (uint32_t)kMaxOrder || nnz_x + nnz_y >= (1ull << 32)) return PASTA_EUNSUPPORTED;
    for (uint32_t k = 0; k < order; ++k) {
        if (dims_x[k] == 0 || dims_y[k] == 0) return PASTA_EINVAL;
        if (dims_x[k] > (1ull << 31) || dims_y[k] > (1ull << 31)) return PASTA_EUNSUPPORTED;
    }
    const uint64_t M = nnz_x + nnz_y;
    if (nnz_x && (!d_inds_x || !d_vals_x)) return PASTA_EINVAL;
    if (nnz_y && (!d_inds_y || !d_vals_y)) return PASTA_EINVAL;
    if (M && (!d_inds_z || !d_vals_z)) return PASTA_EINVAL;
    for (uint32_t k = 0; k < order; ++k) {
        if (nnz_x && !d_inds_x[k]) return PASTA_EINVAL;
        if (nnz_y && !d_inds_y[k]) return PASTA_EINVAL;
        if (M && !d_inds_z[k]) return PASTA_EINVAL;
    }
    TewLayout L;
    if (!make_tew_layout(order, M, L)) return PASTA_EUNSUPPORTED;
    if (M && (!d_work || work_bytes < L.total || ((uintptr_t)d_work % kAlign) != 0)) return PASTA_EWORKSPACE;
    uint64_t dz[kMaxOrder];
    for (uint32_t k = 0; k < order; ++k) dz[k] = std::max(dims_x[k], dims_y[k]);  // the unified shape
    if (M == 0) {
        for (uint32_t k = 0; k < order; ++k) dims_z[k] = dz[k];
        *nnz_z = 0;
        return PASTA_OK;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(d_work);
    auto at = [&](size_t off) { return reinterpret_cast<uint32_t *>(base + off); };
    const uint32_t N = order;
    uint32_t *flag = at(L.flag);
    HIPCHK(launch_fill_u32(flag, 0u, 1, st));
    if (nnz_x) HIPCHK(launch_validate(d_inds_x, dims_x, N, nnz_x, flag, st));
    if (nnz_y) HIPCHK(launch_validate(d_inds_y, dims_y, N, nnz_y, flag, st));
    // X then Y, side by side in set 0 (index arrays 0..N-1, values N)
    for (uint32_t k = 0; k < N; ++k) {
        uint32_t *dst = at(L.set[0][k]);
        if (nnz_x) HIPCHK(hipMemcpyAsync(dst, d_inds_x[k], nnz_x * 4, hipMemcpyDeviceToDevice, st));
        if (nnz_y) HIPCHK(hipMemcpyAsync(dst + nnz_x, d_inds_y[k], nnz_y * 4, hipMemcpyDeviceToDevice, st));
    }
    {
        uint32_t *dst = at(L.set[0][N]);
        if (nnz_x) HIPCHK(hipMemcpyAsync(dst, d_vals_x, nnz_x * 4, hipMemcpyDeviceToDevice, st));
        if (nnz_y) HIPCHK(hipMemcpyAsync(dst + nnz_x, d_vals_y, nnz_y * 4, hipMemcpyDeviceToDevice, st));
    }
    // Stable LSD sort into lexicographic order, mode 0 most significant (Alg. 2's
    // sort); equal coordinates keep X's entries first, each input in its own order.
    struct Soa {
        const uint32_t *ind[kMaxOrder];
        const uint32_t *val, *perm;
    } cur;
    for (uint32_t k = 0; k < N; ++k) cur.ind[k] = at(L.set[0][k]);
    cur.val = at(L.set[0][N]);
    cur.perm = nullptr;  // identity until the first pass writes it
    int parity = 1;
    uint32_t *hist = at(L.hist), *scanpart = at(L.scanpart);
    const uint64_t hist_n = (uint64_t)kRadix * L.ntiles;
    auto pass = [&](uint32_t k, int shift, bool sort) -> pasta_status {
        uint32_t *dind[kMaxOrder];
        for (uint32_t kk = 0; kk < N; ++kk) dind[kk] = at(L.set[parity][kk]);
        uint32_t *dval = at(L.set[parity][N]), *dperm = at(L.set[parity][N + 1]);
        SortPayload pl{};
        int cnt = 0;
        pl.in[cnt] = cur.perm;
        pl.out[cnt++] = dperm;
        for (uint32_t kk = 0; kk < N; ++kk)
            if (kk != k) {
                pl.in[cnt] = cur.ind[kk];
                pl.out[cnt++] = dind[kk];
            }
        pl.in[cnt] = cur.val;
        pl.out[cnt++] = dval;
        pl.count = cnt;
        if (sort) {
            HIPCHK(launch_radix_hist(cur.ind[k], M, shift, hist, L.ntiles, st));
            HIPCHK(launch_exclusive_scan(hist, hist, hist_n, scanpart, st));
            HIPCHK(launch_radix_scatter(cur.ind[k], M, shift, hist, L.ntiles, dind[k], pl, st));
        } else {
            HIPCHK(launch_copy_payload(cur.ind[k], M, dind[k], pl, st));
        }
        for (uint32_t kk = 0; kk < N; ++kk) cur.ind[kk] = dind[kk];
        cur.val = dval;
        cur.perm = dperm;
        parity ^= 1;
        return PASTA_OK;
    };
    bool moved = false;
    for (int k = (int)N - 1; k >= 0; --k) {
        const int passes = (key_bits(dz[k]) + kRadixBits - 1) / kRadixBits;
        for (int ps = 0; ps < passes; ++ps) {
            pasta_status e = pass((uint32_t)k, ps * kRadixBits, true);
            if (e != PASTA_OK) return e;
            moved = true;
        }
    }
    if (!moved) {  // every mode has size 1: keep the concatenation order, write the positions
        pasta_status e = pass(0, 0, false);
        if (e != PASTA_OK) return e;
    }
    // runs of equal coordinates, reduced and compacted in order
    FiberInds fi{};
    TewInds ti{};
    for (uint32_t k = 0; k < N; ++k) fi.p[k] = ti.p[k] = cur.ind[k];
    fi.count = N;
    uint32_t *head = at(L.head), *run_of = at(L.run_of), *run_keep = at(L.run_keep), *out_of = at(L.out_of);
    HIPCHK(launch_fiber_heads(fi, M, head, st));
    HIPCHK(launch_exclusive_scan(head, run_of, M, scanpart, st));
    HIPCHK(launch_fill_u32(run_keep, 0u, M, st));
    float *run_val = reinterpret_cast<float *>(at(L.run_val));
    HIPCHK(launch_tew_runs(head, run_of, cur.perm, reinterpret_cast<const float *>(cur.val), M, nnz_x, (int)op,
                           run_val, at(L.run_pos), run_keep, st));
    HIPCHK(launch_exclusive_scan(run_keep, out_of, M, scanpart, st));
    TewOut to{};
    for (uint32_t k = 0; k < N; ++k) to.p[k] = d_inds_z[k];
    HIPCHK(launch_tew_emit(ti, N, at(L.run_pos), run_val, run_keep, out_of, M, to, d_vals_z, at(L.count), st));
    uint32_t host[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(&host[0], at(L.count), 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&host[1], flag, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (host[1]) return PASTA_ERANGE;
    for (uint32_t k = 0; k < order; ++k) dims_z[k] = dz[k];
    *nnz_z = host[0];
    return PASTA_OK;
}

const char *pasta_status_str(pasta_status s)
{
    switch (s) {
    case PASTA_OK: return "ok";
    case PASTA_EINVAL: return "invalid argument";
    case PASTA_ERANGE: return "coordinate out of range";
    case PASTA_EUNSUPPORTED: return "unsupported order, rank, dtype or alignment";
    case PASTA_EWORKSPACE: return "workspace too small or misaligned";
    case PASTA_EHIP: return "HIP runtime error";
    case PASTA_EINTERNAL: return "a kernel found the preprocessed tensor inconsistent";
    }
    return "unknown status";
}

int pasta_last_hip_error(void) { return g_last_hip_error; }

}  // extern "C"
