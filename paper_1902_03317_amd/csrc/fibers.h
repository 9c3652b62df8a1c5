// Launch interfaces of the fiber kernels (fibers.hip): the mode-n fiber
// pre-processing of Algs. 4 and 5 and the TTV kernel. Every pointer is device
// memory.
#pragma once

#include "common.h"

namespace pasta {

// The other modes' index arrays of a fiber-ordered stream (count = order - 1).
struct FiberInds {
    const uint32_t *p[kMaxOrder];
    uint32_t count;
};
struct FiberCoords {
    uint32_t *p[kMaxOrder];
};

// head[p] = 1 where nonzero p starts a fiber (p = 0, or some other-mode index
// differs from nonzero p - 1), else 0.
hipError_t launch_fiber_heads(const FiberInds &in, uint64_t nnz, uint32_t *head, hipStream_t st);
// From the heads and their exclusive scan: fid[p] (fiber of nonzero p),
// fptr[f] (first nonzero of fiber f; fptr[nfibs] = nnz), coords[q][f] (the
// fiber's fixed indices) and *nfibs.
hipError_t launch_fiber_compact(const FiberInds &in, uint64_t nnz, const uint32_t *head, const uint32_t *excl,
                                uint32_t *fid, uint32_t *fptr, const FiberCoords &coords, uint32_t *nfibs,
                                hipStream_t st);

// Frequency relabelling of a mode's index space (so that the entries of v a
// TTV gathers most often share cache lines): keys[i] = nnz - count[i] from a
// row-offset array, so an ascending stable sort lists indices by decreasing
// count; inv[perm[j]] = j; out[p] = table[idx[p]] (u32 and f32).
hipError_t launch_count_keys(const uint32_t *rowptr, uint32_t n, uint64_t nnz, uint32_t *keys, hipStream_t st);
hipError_t launch_invert_perm(const uint32_t *perm, uint32_t n, uint32_t *inv, hipStream_t st);
hipError_t launch_gather_u32(const uint32_t *table, const uint32_t *idx, uint64_t n, uint32_t *out, hipStream_t st);
hipError_t launch_gather_f32(const float *table, const uint32_t *idx, uint64_t n, float *out, hipStream_t st);

// TTV: out[f] = sum over the nonzeros p of fiber f of vals[p] * v[idx[p]].
// One wave per chunk of kTtvChunk nonzeros, walked in tiles of kTtvTile (four
// per lane); fibers crossing a chunk edge leave partials in part[2c] (the
// chunk's first fiber) and part[2c + 1] (its last) for launch_fixup.
constexpr uint32_t kTtvTile = 256;
constexpr uint32_t kTtvTiles = 4;
constexpr uint64_t kTtvChunk = (uint64_t)kTtvTile * kTtvTiles;
hipError_t launch_ttv(const uint32_t *fid, const uint32_t *idx, const float *vals, const float *v, float *out,
                      float *part, uint64_t nnz, uint32_t nchunks, hipStream_t st);

}  // namespace pasta
