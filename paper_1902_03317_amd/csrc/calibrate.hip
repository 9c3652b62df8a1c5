// Measurement kernel: the rate at which gfx950's vector memory pipeline serves
// 16-byte-per-lane row gathers, the access the MTTKRP kernels make for every
// factor row of every nonzero. It gives the gather ceiling the MTTKRP kernels
// are compared with (bytes delivered to lanes per second), beside the HBM peak.
//
// A wave is G = 64 / L lane groups of L lanes; in every step, group g reads
// one row of L x 16 bytes from a table (lane j reads bytes 16j .. 16j+15), the
// same shape as the MTTKRP gathers at that lane count. Rows start at an integer
// hash of (wave, group / share) and advance by an odd stride each step: with
// share = 1 every group of an instruction reads its own row, with share = G the
// whole wave reads one row. Groups g >= active skip their loads (the lanes are masked off), which
// shows whether an instruction's cost follows its active lanes. The table size
// sets which cache level serves the gathers. Eight steps'
// loads are issued before any is consumed (the MTTKRP kernels keep as many in
// flight), and every loaded word feeds the output, so none is dropped.
#include "common.h"

namespace pasta {
namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

template <int L, bool ALL>
__device__ __forceinline__ void probe_walk(const uint4 *__restrict__ table, uint32_t row_mask, uint32_t active,
                                           uint32_t steps, uint32_t g, uint32_t j, uint32_t row, uint4 &acc)
{
    constexpr int kInFlight = 8;
    constexpr uint32_t kRowShift = __builtin_ctz(16u * L);  // bytes per row, a power of two
    const char *base = reinterpret_cast<const char *>(table) + 16u * j;
    uint4 v[kInFlight];
#pragma unroll
    for (int u = 0; u < kInFlight; ++u) v[u] = make_uint4(0u, 0u, 0u, 0u);
    for (uint32_t s = 0; s < steps; s += kInFlight) {
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            row += 0x9E3779B1u;
            const uint32_t off = (row & row_mask) << kRowShift;  // 32-bit byte offset from the table base
            if (ALL || g < active) v[u] = *reinterpret_cast<const uint4 *>(base + off);
        }
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            acc.x ^= v[u].x ^ v[u].y;
            acc.y ^= v[u].z ^ v[u].w;
        }
    }
}

template <int L>
__global__ __launch_bounds__(256) void gather_probe_kernel(const uint4 *__restrict__ table, uint32_t row_mask,
                                                           uint32_t share, uint32_t active, uint32_t steps,
                                                           uint4 *__restrict__ out)
{
    constexpr uint32_t G = kWave / L;
    const int lane = threadIdx.x & 63;
    const uint32_t g = (uint32_t)(lane / L), j = (uint32_t)(lane % L);
    const uint32_t wave = blockIdx.x * 4u + (threadIdx.x >> 6);
    // a hashed start per (wave, group / share), then an odd additive stride per step:
    // a few integer operations per row, so the probe's own arithmetic stays far below
    // the rate of the loads it measures (masked-off groups keep their last values)
    const uint32_t row = mix32(mix32(wave * 0x9E3779B9u) ^ (g / share) * 0x85EBCA6Bu);
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    if (active >= G)
        probe_walk<L, true>(table, row_mask, active, steps, g, j, row, acc);
    else
        probe_walk<L, false>(table, row_mask, active, steps, g, j, row, acc);
    out[(uint64_t)blockIdx.x * 256u + threadIdx.x] = acc;
}

}  // namespace

hipError_t launch_gather_probe(const void *table, uint32_t rows, uint32_t lanes, uint32_t share, uint32_t active,
                               uint32_t steps, uint32_t blocks, void *out, hipStream_t st)
{
    const uint4 *t = static_cast<const uint4 *>(table);
    uint4 *o = static_cast<uint4 *>(out);
    switch (lanes) {
    case 4: gather_probe_kernel<4><<<blocks, 256, 0, st>>>(t, rows - 1, share, active, steps, o); break;
    case 8: gather_probe_kernel<8><<<blocks, 256, 0, st>>>(t, rows - 1, share, active, steps, o); break;
    case 16: gather_probe_kernel<16><<<blocks, 256, 0, st>>>(t, rows - 1, share, active, steps, o); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pasta
