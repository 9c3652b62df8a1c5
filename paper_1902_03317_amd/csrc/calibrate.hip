// Measurement kernel: the rate at which gfx950's vector memory pipeline serves
// 16-byte-per-lane row gathers, the access the MTTKRP kernels make for every
// factor row of every nonzero. It gives the gather ceiling the MTTKRP kernels
// are compared with (bytes delivered to lanes per second), beside the HBM peak.
//
// A wave is G = 64 / L lane groups of L lanes; in every step, group g reads
// one row of L x 16 bytes from a table (lane j reads bytes 16j .. 16j+15), the
// same shape as the MTTKRP gathers at that lane count. Rows are drawn by an
// integer hash of (wave, step, group / share): with share = 1 every group of
// an instruction reads its own row, with share = G the whole wave reads one
// row. The table size sets which cache level serves the gathers. Eight steps'
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

template <int L>
__global__ __launch_bounds__(256) void gather_probe_kernel(const uint4 *__restrict__ table, uint32_t row_mask,
                                                           uint32_t share, uint32_t steps, uint4 *__restrict__ out)
{
    constexpr int G = kWave / L;
    constexpr int kInFlight = 8;
    const int lane = threadIdx.x & 63;
    const uint32_t g = (uint32_t)(lane / L), j = (uint32_t)(lane % L);
    const uint32_t wave = blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t key = mix32(wave * 0x9E3779B9u) ^ (g / share) * 0x85EBCA6Bu;
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    for (uint32_t s = 0; s < steps; s += kInFlight) {
        uint4 v[kInFlight];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            const uint32_t row = mix32(key + (s + (uint32_t)u) * 0xC2B2AE35u) & row_mask;
            v[u] = table[(uint64_t)row * L + j];
        }
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            acc.x ^= v[u].x;
            acc.y += v[u].y;
            acc.z ^= v[u].z;
            acc.w += v[u].w;
        }
    }
    out[(uint64_t)blockIdx.x * 256u + threadIdx.x] = acc;
}

}  // namespace

hipError_t launch_gather_probe(const void *table, uint32_t rows, uint32_t lanes, uint32_t share, uint32_t steps,
                               uint32_t blocks, void *out, hipStream_t st)
{
    const uint4 *t = static_cast<const uint4 *>(table);
    uint4 *o = static_cast<uint4 *>(out);
    switch (lanes) {
    case 4: gather_probe_kernel<4><<<blocks, 256, 0, st>>>(t, rows - 1, share, steps, o); break;
    case 8: gather_probe_kernel<8><<<blocks, 256, 0, st>>>(t, rows - 1, share, steps, o); break;
    case 16: gather_probe_kernel<16><<<blocks, 256, 0, st>>>(t, rows - 1, share, steps, o); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pasta
