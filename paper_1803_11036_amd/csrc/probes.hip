// Memory ceiling probes (measurement only; no part of the detector): the
// rates the scan and the close are bound by, measured on the device itself.
//   - stream read: every 16-byte chunk of a buffer read once, coalesced;
//   - random byte scatter: n one-byte stores at counter-hashed positions,
//     either uniform over the whole buffer or XCD-local (workgroup g stores
//     only into a 2 MiB region of its own XCD, g mod 8, as the binned scan's
//     stores do);
//   - random 16-byte read-modify-write in bins: one 1024-thread workgroup
//     per bin, bins dealt to the XCDs as the counted stores deal theirs, each
//     workgroup loading, changing and storing hashed 16-byte chunks of its
//     bin, four per thread in flight (the memory side of the counted stores'
//     visit, without their offsets).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ssd_probe.h"

namespace {

__global__ __launch_bounds__(256) void k_probe_read(const uint4* buf, uint64_t n16, uint32_t* sink)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    uint32_t acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < n16; i += stride) {
        const uint4 v = buf[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    // one word per thread that the compiler cannot drop; the host never reads it
    if (acc == 0x9E3779B9u) sink[threadIdx.x] = acc;
}

// 64-bit mixer (the finaliser of SplitMix64) for store positions
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Grid-stride scatter: store i writes one byte at a hashed position.  XCD-
// local (region_shift > 0): workgroup g stores inside region ((g / 8) / per)
// * 8 + g mod 8 (mod n_regions) of 2^region_shift bytes, so that the
// workgroups resident on one XCD share a region its L2 holds.
__global__ __launch_bounds__(256) void k_probe_scatter(uint8_t* buf, uint64_t bytes, uint64_t n, uint64_t seed,
                                                       uint32_t region_shift, uint32_t per)
{
    const uint64_t total_threads = (uint64_t)gridDim.x * 256u;
    const uint64_t tid = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (region_shift) {
        const uint64_t n_regions = bytes >> region_shift;
        const uint64_t g = blockIdx.x;
        const uint64_t region = (((g >> 3) / per) * 8u + (g & 7u)) % n_regions;
        uint8_t* base = buf + (region << region_shift);
        const uint64_t mask = (1ull << region_shift) - 1u;
        for (uint64_t i = tid; i < n; i += total_threads) base[mix64(seed + i) & mask] = (uint8_t)(i | 1u);
    } else {
        // position = high half of hash * bytes: uniform over [0, bytes)
        for (uint64_t i = tid; i < n; i += total_threads) buf[__umul64hi(mix64(seed + i), bytes)] = (uint8_t)(i | 1u);
    }
}

// Workgroup g takes bin (g mod 8) * per_xcd + g / 8 of n_bins bins of
// 2^bin_shift bytes and makes ops read-modify-writes of hashed chunks in it.
__global__ __launch_bounds__(1024) void k_probe_rmw16(uint4* buf, uint64_t n_bins, uint32_t bin_shift, uint32_t ops,
                                                      uint64_t seed)
{
    const uint64_t per_xcd = (n_bins + 7u) >> 3;
    const uint64_t bin = (blockIdx.x & 7u) * per_xcd + (blockIdx.x >> 3);
    if (bin >= n_bins) return;
    uint4* base = buf + (bin << (bin_shift - 4u));
    const uint64_t mask = (1ull << (bin_shift - 4u)) - 1u;
    const uint64_t key = seed + bin * ops;
    for (uint32_t i0 = threadIdx.x; i0 < ops; i0 += 4u * 1024u) {
        uint4 v[4];
        uint64_t at[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const uint32_t i = i0 + (uint32_t)u * 1024u;
            at[u] = mix64(key + i) & mask;
            if (i < ops) v[u] = base[at[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            if (i0 + (uint32_t)u * 1024u >= ops) continue;
            v[u].x ^= 1u;
            base[at[u]] = v[u];
        }
    }
}

}  // namespace

extern "C" {

int ssd_probe_stream_read(const void* buf_dev, uint64_t bytes, void* sink_dev, void* stream)
{
    if (!buf_dev || !sink_dev || bytes < 16 || (bytes & 15u) || ((uintptr_t)buf_dev & 15u)) return -1;
    const uint64_t n16 = bytes / 16u;
    uint64_t blocks = (n16 + 255u) / 256u;
    if (blocks > 256u * 32u) blocks = 256u * 32u;
    k_probe_read<<<(uint32_t)blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<const uint4*>(buf_dev), n16, static_cast<uint32_t*>(sink_dev));
    return hipGetLastError() == hipSuccess ? 0 : -7;
}

int ssd_probe_scatter(void* buf_dev, uint64_t bytes, uint64_t n_stores, uint64_t seed, uint32_t xcd_local,
                      void* stream)
{
    if (!buf_dev || bytes < 4096 || n_stores == 0) return -1;
    const uint32_t region_shift = xcd_local ? 21u : 0u;      // 2 MiB regions
    if (region_shift && (bytes < (8ull << region_shift) || (bytes & ((1ull << region_shift) - 1u)))) return -1;
    // XCD-local: 128 workgroups of 256 threads of one XCD share a region (as
    // about 500 of the binned scan's 64-thread store workgroups share a bin),
    // and the grid covers every region once; uniform: 64 workgroups per
    // compute unit, grid-stride
    const uint32_t per = 128u;
    const uint64_t blocks = region_shift ? ((bytes >> region_shift) + 7u) / 8u * 8u * per : 256u * 64u;
    if (blocks > 0x7FFFFFFFull) return -1;
    k_probe_scatter<<<(uint32_t)blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<uint8_t*>(buf_dev), bytes, n_stores, seed, region_shift, per);
    return hipGetLastError() == hipSuccess ? 0 : -7;
}

int ssd_probe_rmw16(void* buf_dev, uint64_t bytes, uint64_t bin_bytes, uint32_t ops_per_bin, uint64_t seed,
                    void* stream)
{
    if (!buf_dev || ((uintptr_t)buf_dev & 15u) || bin_bytes < 4096 || bin_bytes > (1ull << 30) ||
        (bin_bytes & (bin_bytes - 1u)) || bytes < bin_bytes || (bytes & (bin_bytes - 1u)) || ops_per_bin == 0 ||
        ops_per_bin > (1u << 20))
        return -1;
    uint32_t shift = 0;
    while ((1ull << shift) < bin_bytes) shift++;
    const uint64_t n_bins = bytes >> shift;
    const uint64_t blocks = (n_bins + 7u) / 8u * 8u;
    if (blocks > 0x7FFFFFFFull) return -1;
    k_probe_rmw16<<<(uint32_t)blocks, 1024, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<uint4*>(buf_dev), n_bins, shift, ops_per_bin, seed);
    return hipGetLastError() == hipSuccess ? 0 : -7;
}

}  // extern "C"
