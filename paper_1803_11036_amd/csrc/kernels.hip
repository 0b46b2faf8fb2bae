// HIP kernels (gfx950, wave64) of the sliding super point detector.
//
// Cell encoding: a sliding-estimator cell is one byte.  0 = never hit; a hit
// in slot s stores the stamp 1 + (s mod 255).  At the close of slot t the
// cell's distance (Sec. 3.2 distance recorder) is (stamp(t) - stamp) mod 255,
// valid because every cell whose distance reaches k is cleared before it can
// reach 255 (rotating expiry, see k_hot_detect).  This replaces the paper's
// 16-bit recorder and its +1 sweep over all recorders every slot (Sec. 4.3)
// with one byte per cell and no per-slot write pass.
//
// Liveness test (distance < k) on four packed cells at once: the byte values
// are rebased so that live stamps map to [0, K') and tested in 16-bit slots
// (see LiveCfg); the rebasing constants are computed per slot from the clock.
//
// Windows longer than 254 slots (the paper's k up to 65534, Sec. 3.2) take
// 16-bit cells: stamp 1 + (s mod 65535), the same rules modulo 65535.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "internal.h"

namespace ssd {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ uint32_t tab_hash(const uint32_t* t, uint32_t x)
{
    // simple tabulation hashing: four byte-indexed tables XORed (Sec. 3.2, 3.3)
    return t[x & 255u] ^ t[256u + ((x >> 8) & 255u)] ^ t[512u + ((x >> 16) & 255u)] ^ t[768u + (x >> 24)];
}

__device__ __forceinline__ uint32_t shr32(uint32_t x, uint32_t s) { return s < 32u ? (x >> s) : 0u; }

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Reserve `cnt` consecutive slots of a device-wide list for this thread of a
// 256-thread block (every thread must call it): one atomic per block.
__device__ __forceinline__ unsigned long long block_append_256(uint32_t cnt, unsigned long long* counter)
{
    __shared__ uint32_t wtot[4];
    __shared__ unsigned long long bbase;
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    uint32_t incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t v = __shfl_up(incl, o, 64);
        if (lane >= (uint32_t)o) incl += v;
    }
    if (lane == 63) wtot[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t tot = wtot[0] + wtot[1] + wtot[2] + wtot[3];
        bbase = tot ? atomicAdd(counter, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    uint32_t woff = 0;
    for (uint32_t w = 0; w < wid; w++) woff += wtot[w];
    const unsigned long long base = bbase;
    __syncthreads();
    return base + woff + (incl - cnt);
}

// Live cells of a 32-bit word of four cells: bits 8, 24 (bytes 0, 2) and
// 9, 25 (bytes 1, 3) are set for live cells.
__device__ __forceinline__ uint32_t live_bits(uint32_t w, const LiveCfg& L)
{
    const uint32_t M = 0x00FF00FFu, H = 0x01000100u;
    const uint32_t e = w & M, o = (w >> 8) & M;
    const uint32_t be = ((e + L.c1) & M) + L.c2;   // bit 8 of a slot: rebased stamp >= K'
    const uint32_t bo = ((o + L.c1) & M) + L.c2;
    uint32_t live = (~be & H) | ((~bo & H) << 1);
    if (L.wrap) live &= ((e + M) & H) | (((o + M) & H) << 1);   // exclude empty cells
    return live;
}

// The live cells of a 16-byte chunk as a 16-bit mask (bit i = cell i).
__device__ __forceinline__ uint32_t live_mask16(const uint4& v, const LiveCfg& L)
{
    auto nib = [](uint32_t x) { return ((x >> 8) & 3u) | ((x >> 22) & 12u); };
    return nib(live_bits(v.x, L)) | (nib(live_bits(v.y, L)) << 4) | (nib(live_bits(v.z, L)) << 8) |
           (nib(live_bits(v.w, L)) << 12);
}

// The word with every dead non-empty cell cleared (distance >= k).
__device__ __forceinline__ uint32_t expire_word(uint32_t w, const LiveCfg& L)
{
    const uint32_t M = 0x00FF00FFu;
    const uint32_t e = w & M, o = (w >> 8) & M;
    const uint32_t be = ((e + L.c1) & M) + L.c2;
    const uint32_t bo = ((o + L.c1) & M) + L.c2;
    const uint32_t de = ((be >> 8) & 0x00010001u) * 0xFFu;
    const uint32_t dd = (((bo >> 8) & 0x00010001u) * 0xFFu) << 8;
    return w & ~(de | dd);
}

// 16-bit cells: c is live iff (c - lo) mod 2^16 < K' and, when the live
// stamps wrap past 65535, c is not empty (LiveCfg c1 = lo, c2 = K').
__device__ __forceinline__ uint32_t live_cell16(uint32_t c, const LiveCfg& L)
{
    return (((c - L.c1) & 0xFFFFu) < L.c2 && (!L.wrap || c != 0u)) ? 1u : 0u;
}

// The live cells of a 16-byte chunk of eight 16-bit cells (bit i = cell i).
__device__ __forceinline__ uint32_t live_mask8_c16(const uint4& v, const LiveCfg& L)
{
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < 4; i++)
        m |= (live_cell16(w[i] & 0xFFFFu, L) << (2 * i)) | (live_cell16(w[i] >> 16, L) << (2 * i + 1));
    return m;
}

// Two 16-bit cells with every dead non-empty one cleared (distance >= k).
__device__ __forceinline__ uint32_t expire_word16(uint32_t w, const LiveCfg& L)
{
    const uint32_t lo = w & 0xFFFFu, hi = w >> 16;
    return (live_cell16(lo, L) ? lo : 0u) | ((live_cell16(hi, L) ? hi : 0u) << 16);
}

// Index of the link owning flattened item g: the largest l with prefix[l] <= g
// (empty links have prefix[l] == prefix[l+1] and are skipped).
template <class U>
__device__ __forceinline__ uint32_t find_link(const U* prefix, uint32_t n_links, uint64_t g)
{
    uint32_t lo = 0, hi = n_links;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ void block_exclusive_scan_u64_1024(unsigned long long v, unsigned long long* lds /*[1024]*/,
                                                              unsigned long long* excl, unsigned long long* total)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t o = 1; o < 1024u; o <<= 1) {
        const unsigned long long t = threadIdx.x >= o ? lds[threadIdx.x - o] : 0ull;
        __syncthreads();
        lds[threadIdx.x] += t;
        __syncthreads();
    }
    *excl = lds[threadIdx.x] - v;
    *total = lds[1023];
    __syncthreads();
}

__device__ __forceinline__ uint32_t block_exclusive_scan_1024(uint32_t v, uint32_t* lds /*[16]*/, uint32_t* total)
{
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= (uint32_t)o) incl += t;
    }
    if (lane == 63) lds[wid] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (uint32_t w = 0; w < 16; w++) {
        uint32_t x = lds[w];
        off += w < wid ? x : 0u;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

// ---------------------------------------------------------------- fill / clock

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Per-slice constants of every link from its device clock (the open slice t).
// Per-slice constants of every link from its slot clock (grid: links x 16,
// thread 0 of block (l, 0)), and the hot bitmasks cleared for this close.
__global__ __launch_bounds__(256) void k_prepare(LinkDesc* links, uint32_t clear_hot)
{
    const uint32_t l = blockIdx.x;
    if (clear_hot) {
        const LinkDesc* D = links + l;
        uint32_t* p = reinterpret_cast<uint32_t*>(D->hotbits);     // hotT follows hotbits
        const uint64_t n = D->hot_words;
        for (uint64_t i = blockIdx.y * 256u + threadIdx.x; i < n; i += 256u * gridDim.y) p[i] = 0u;
    }
    if (blockIdx.y != 0 || threadIdx.x != 0) return;
    const unsigned long long t = links[l].clock->t;
    const uint32_t k = links[l].k;
    if (links[l].cell16) {
        // 16-bit cells: stamps 1 + t mod 65535, expiry period 65535 - k
        const uint32_t cur = 1u + (uint32_t)(t % 65535u);
        LiveCfg c;
        if (cur >= k) { c.c1 = cur - k + 1u; c.c2 = k; c.wrap = 0u; }
        else { c.c1 = cur + 65536u - k; c.c2 = k + 1u; c.wrap = 1u; }
        links[l].L = c;
        links[l].expire_period = 65535u - k;
        links[l].expire_phase = (uint32_t)(t % (65535u - k));
        return;
    }
    const uint32_t cur = 1u + (uint32_t)(t % 255u);
    uint32_t lo, kp, wrap;
    if (cur >= k) { lo = cur - k + 1u; kp = k; wrap = 0u; }
    else { lo = cur + 256u - k; kp = k + 1u; wrap = 1u; }
    LiveCfg c;
    c.c1 = (256u - lo) * 0x00010001u;
    c.c2 = (256u - kp) * 0x00010001u;
    c.wrap = wrap;
    links[l].L = c;
    links[l].expire_period = 255u - k;
    links[l].expire_phase = (uint32_t)(t % (255u - k));
}

__global__ void k_advance(const LinkDesc* links, uint32_t n_links)
{
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n_links) links[l].clock->t += 1ull;
}

// Copy every link's control block into one contiguous array (links whose
// blocks live in separate allocations).
__global__ void k_gather_ctl(const LinkDesc* links, uint32_t n_links, Ctl* dst)
{
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n_links) dst[l] = *links[l].ctl;
}

// Clear every link's hot bitmasks (grid: links x 16 blocks).

// ---------------------------------------------------------------- scan
// Alg. 2 for every pair: one byte store per row.  `se_lo..se_hi` restricts
// the stores to one estimator window so that a pass's random stores stay in
// the last-level cache.

template <class T>
__device__ __forceinline__ void scan_pair(const uint32_t* tab, uint2 pr, T* state, uint32_t q, uint32_t delta,
                                          uint32_t log2eta, uint32_t row_lo, uint32_t row_hi, uint64_t se_lo,
                                          uint64_t se_hi, T stamp)
{
    const uint32_t qmask = (1u << q) - 1u;
    const uint32_t d = tab_hash(tab + 1024, pr.y) & ((1u << log2eta) - 1u);   // H1(oip)
    const uint32_t h0 = tab_hash(tab, pr.x) & qmask;                          // RHFG[0](cip)
    for (uint32_t i = row_lo; i < row_hi; i++) {
        const uint32_t col = i == 0 ? h0 : ((shr32(pr.x, (i - 1) * delta) ^ h0) & qmask);
        const uint64_t se = ((uint64_t)i << q) | col;
        if (se >= se_lo && se < se_hi) state[(se << log2eta) | d] = stamp;
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_scan(ScanArgs a)
{
    __shared__ uint32_t tab[2048];
    for (uint32_t i = threadIdx.x; i < 2048u; i += 256u) tab[i] = a.tables[i];
    __syncthreads();
    const uint32_t row_lo = (uint32_t)(a.se_lo >> a.q);
    const uint32_t row_hi = (uint32_t)((a.se_hi - 1) >> a.q) + 1u;
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    for (uint64_t p = (uint64_t)blockIdx.x * 256u + threadIdx.x; p < a.n; p += stride)
        scan_pair<T>(tab, a.pairs[p], reinterpret_cast<T*>(a.state), a.q, a.delta, a.log2eta, row_lo, row_hi,
                     a.se_lo, a.se_hi, (T)a.stamp);
}

// Persistent scan over many links: workgroups pull tile numbers from a device
// counter; a tile is `tile` pairs of one link restricted to one estimator
// window, found by binary search over the windows' tile prefix.  Windows are
// ordered by state address and tiles are small, so the tiles in flight store
// into a cache-sized range of state; a workgroup reloads the tabulation
// tables only when its link changes.  Every workgroup leaves once the counter
// passes the last tile.
__global__ __launch_bounds__(256) void k_scan_tiles(TileScanArgs a)
{
    __shared__ uint32_t tab[2048];
    __shared__ unsigned long long next;
    uint32_t loaded = 0xFFFFFFFFu;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(a.counter, 1ull);
        __syncthreads();
        const unsigned long long t = next;
        __syncthreads();
        if (t >= a.n_tiles) break;
        uint32_t lo = 0, hi = a.n_wins;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.wins[mid].tile_base <= t) lo = mid;
            else hi = mid;
        }
        const ScanWindow W = a.wins[lo];
        const uint64_t first = W.start + (t - W.tile_base) * a.tile;
        const uint64_t last = min(first + a.tile, W.start + W.n);
        const LinkDesc* D = a.links + W.link;
        if (W.link != loaded) {
            for (uint32_t i = threadIdx.x; i < 2048u; i += 256u) tab[i] = D->tables[i];
            __syncthreads();
            loaded = W.link;
        }
        const uint32_t q = D->q, delta = D->delta, log2eta = D->log2eta;
        uint8_t* state = D->state;
        const uint32_t row_lo = (uint32_t)(W.se_lo >> q);
        const uint32_t row_hi = (uint32_t)((W.se_hi - 1) >> q) + 1u;
        for (uint64_t p = first + threadIdx.x; p < last; p += 256u)
            scan_pair<uint8_t>(tab, a.pairs[p], state, q, delta, log2eta, row_lo, row_hi, W.se_lo, W.se_hi,
                               (uint8_t)W.stamp);
    }
}

// ---------------------------------------------------------------- binned scan
// Alg. 2 in two steps, for states much larger than the caches.
// k_bin: each workgroup takes `pb` pairs, computes their r cell addresses and
// counting-sorts the bin-local offsets by state bin (bins of 2^bin_shift
// bytes) in LDS, then writes them as one coalesced segment; the start of every
// bin in the segment goes to a bin-major table.
// k_apply: the byte stores, bin by bin.  Workgroup g runs on XCD g mod 8 (the
// dispatcher deals workgroups to the XCDs in turn) and the bins of an XCD are
// visited in ascending order by all its workgroups together, so the stores of
// each XCD land in a range its own L2 holds.  Results do not depend on the
// placement: every store is independent.

__device__ __forceinline__ void pair_hashes(const uint32_t* tab, uint2 pr, uint32_t q, uint32_t log2eta,
                                            uint32_t* h0, uint32_t* d)
{
    *d = tab_hash(tab + 1024, pr.y) & ((1u << log2eta) - 1u);   // H1(oip)
    *h0 = tab_hash(tab, pr.x) & ((1u << q) - 1u);               // RHFG[0](cip)
}

__device__ __forceinline__ uint64_t cell_addr(uint2 pr, uint32_t i, uint32_t h0, uint32_t d, uint32_t q,
                                              uint32_t delta, uint32_t log2eta)
{
    const uint32_t col = i == 0 ? h0 : ((shr32(pr.x, (i - 1) * delta) ^ h0) & ((1u << q) - 1u));
    return ((((uint64_t)i << q) | col) << log2eta) | d;
}


// The segment (chunk of pairs) of this binning workgroup: workgroup g runs on
// XCD g mod 8, which takes a contiguous eighth of the segments, so that the
// bin table entries of neighbouring segments, which share sectors, are
// written through one L2 and leave it merged.  At least the segment count.
__device__ __forceinline__ uint32_t bin_segment(uint32_t g, uint32_t blocks)
{
    return (g & 7u) * ((blocks + 7u) >> 3) + (g >> 3);
}

// A workgroup's sorted offsets out to its segment, coalesced: 4 bytes each, or
// (bins of at most 2 MiB) three 21-bit offsets per 8-byte word.
__device__ __forceinline__ void write_segment(const BinArgs& a, uint32_t sg, const uint32_t* stage, uint32_t n)
{
    const uint64_t seg_items = (uint64_t)a.pb * a.r;
    if (a.pack) {
        uint64_t* seg = reinterpret_cast<uint64_t*>(a.items) + (uint64_t)sg * packed_seg_words(seg_items);
        for (uint32_t w = threadIdx.x; w * 3u < n; w += 1024u) {
            const uint32_t i = w * 3u;
            uint64_t v = stage[i];
            if (i + 1 < n) v |= (uint64_t)stage[i + 1] << 21;
            if (i + 2 < n) v |= (uint64_t)stage[i + 2] << 42;
            seg[w] = v;
        }
    } else {
        uint32_t* seg = a.items + (uint64_t)sg * seg_items;
        for (uint32_t i = threadIdx.x; i < n; i += 1024u) seg[i] = stage[i];
    }
}

// Item i of segment j as written by write_segment.
__device__ __forceinline__ uint32_t read_item(const ApplyArgs& a, uint32_t j, uint32_t i)
{
    if (a.pack) {
        const uint64_t w = reinterpret_cast<const uint64_t*>(a.items)[(uint64_t)j * packed_seg_words(a.seg) + i / 3u];
        return (uint32_t)(w >> (21u * (i % 3u))) & 0x1FFFFFu;
    }
    return a.items[(uint64_t)j * a.seg + i];
}

// Up to 160 KiB of LDS per workgroup: about 6000 pairs, so that the run of
// one bin in one segment is long (about 50 offsets at 2 MiB bins) and
// k_apply's reads of the runs are dense.  Pass 1 counts the bins' offsets,
// pass 2 hashes again and places each offset at its bin's next free slot.
// (workgroup g of this link's launch; lds: the dynamic LDS, wsum: 16 words)
__device__ __forceinline__ void bin_generic(const BinArgs& a, uint32_t g, uint32_t* lds, uint32_t* wsum)
{
    const uint32_t sg = bin_segment(g, a.blocks);
    if (sg >= a.blocks) return;
    uint32_t* tab = lds;
    uint32_t* hist = lds + 2048;
    uint32_t* stage = hist + a.n_bins + 1;
    for (uint32_t i = threadIdx.x; i < 2048u; i += 1024u) tab[i] = a.tables[i];
    for (uint32_t i = threadIdx.x; i <= a.n_bins; i += 1024u) hist[i] = 0u;
    __syncthreads();
    const uint64_t p0 = (uint64_t)sg * a.pb;
    const uint32_t np = (uint32_t)min((uint64_t)a.pb, a.n - p0);
    const uint32_t q = a.q, r = a.r, delta = a.delta, log2eta = a.log2eta, bs = a.bin_shift;
    const uint32_t bmask = (1u << bs) - 1u;
    for (uint32_t p = threadIdx.x; p < np; p += 1024u) {
        const uint2 pr = a.pairs[p0 + p];
        uint32_t h0, d;
        pair_hashes(tab, pr, q, log2eta, &h0, &d);
        for (uint32_t i = 0; i < r; i++) atomicAdd(&hist[(uint32_t)(cell_addr(pr, i, h0, d, q, delta, log2eta) >> bs)], 1u);
    }
    __syncthreads();
    const uint32_t per = (a.n_bins + 1023u) / 1024u;
    const uint32_t b0 = min(a.n_bins, threadIdx.x * per), b1 = min(a.n_bins, b0 + per);
    uint32_t sum = 0;
    for (uint32_t b = b0; b < b1; b++) sum += hist[b];
    uint32_t total;
    uint32_t start = block_exclusive_scan_1024(sum, wsum, &total);
    for (uint32_t b = b0; b < b1; b++) {
        const uint32_t c = hist[b];
        hist[b] = start;
        a.table[(uint64_t)b * a.blocks + sg] = start;
        start += c;
    }
    if (threadIdx.x == 0) a.table[(uint64_t)a.n_bins * a.blocks + sg] = np * r;
    __syncthreads();
    for (uint32_t p = threadIdx.x; p < np; p += 1024u) {
        const uint2 pr = a.pairs[p0 + p];
        uint32_t h0, d;
        pair_hashes(tab, pr, q, log2eta, &h0, &d);
        for (uint32_t i = 0; i < r; i++) {
            const uint64_t addr = cell_addr(pr, i, h0, d, q, delta, log2eta);
            stage[atomicAdd(&hist[(uint32_t)(addr >> bs)], 1u)] = (uint32_t)addr & bmask;
        }
    }
    __syncthreads();
    write_segment(a, sg, stage, np * r);
}

// The same sort for the common row counts with every item kept in registers
// between the two passes (R rows, up to PPT pairs per thread): the pairs are
// hashed once, and each offset's rank in its bin comes from the count pass.
template <int R, int PPT>
__device__ __forceinline__ void bin_reg(const BinArgs& a, uint32_t g, uint32_t* lds, uint32_t* wsum)
{
    const uint32_t sg = bin_segment(g, a.blocks);
    if (sg >= a.blocks) return;
    uint32_t* tab = lds;
    uint32_t* hist = lds + 2048;
    uint32_t* stage = hist + a.n_bins + 1;
    for (uint32_t i = threadIdx.x; i < 2048u; i += 1024u) tab[i] = a.tables[i];
    for (uint32_t i = threadIdx.x; i <= a.n_bins; i += 1024u) hist[i] = 0u;
    __syncthreads();
    const uint64_t p0 = (uint64_t)sg * a.pb;
    const uint32_t np = (uint32_t)min((uint64_t)a.pb, a.n - p0);
    const uint32_t q = a.q, delta = a.delta, log2eta = a.log2eta, bs = a.bin_shift;
    const uint32_t bmask = (1u << bs) - 1u;
    uint32_t off[PPT][R], key[PPT][R];
#pragma unroll
    for (int u = 0; u < PPT; u++) {
        const uint32_t p = threadIdx.x + u * 1024u;
        if (p >= np) continue;
        const uint2 pr = a.pairs[p0 + p];
        uint32_t h0, d;
        pair_hashes(tab, pr, q, log2eta, &h0, &d);
#pragma unroll
        for (int i = 0; i < R; i++) {
            const uint64_t addr = cell_addr(pr, i, h0, d, q, delta, log2eta);
            const uint32_t bin = (uint32_t)(addr >> bs);
            off[u][i] = (uint32_t)addr & bmask;
            key[u][i] = (bin << 16) | atomicAdd(&hist[bin], 1u);
        }
    }
    __syncthreads();
    const uint32_t per = (a.n_bins + 1023u) / 1024u;
    const uint32_t b0 = min(a.n_bins, threadIdx.x * per), b1 = min(a.n_bins, b0 + per);
    uint32_t sum = 0;
    for (uint32_t b = b0; b < b1; b++) sum += hist[b];
    uint32_t total;
    uint32_t start = block_exclusive_scan_1024(sum, wsum, &total);
    for (uint32_t b = b0; b < b1; b++) {
        const uint32_t c = hist[b];
        hist[b] = start;
        a.table[(uint64_t)b * a.blocks + sg] = start;
        start += c;
    }
    if (threadIdx.x == 0) a.table[(uint64_t)a.n_bins * a.blocks + sg] = np * R;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PPT; u++) {
        if (threadIdx.x + u * 1024u >= np) continue;
#pragma unroll
        for (int i = 0; i < R; i++) stage[hist[key[u][i] >> 16] + (key[u][i] & 0xFFFFu)] = off[u][i];
    }
    __syncthreads();
    write_segment(a, sg, stage, np * R);
}

// R = 0: the general binning; else the register binning of R rows.
template <int R, int PPT>
__global__ __launch_bounds__(1024) void k_bin(BinArgs a)
{
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t wsum[16];
    if constexpr (R == 0) bin_generic(a, blockIdx.x, lds, wsum);
    else bin_reg<R, PPT>(a, blockIdx.x, lds, wsum);
}

// Several links in one launch: workgroup g belongs to the link whose range
// of the workgroup prefix holds it.  Every link's range is a multiple of 8
// workgroups, so that the dealing of its segments to XCDs is the one of a
// launch of its own.  Each workgroup takes its link's binning variant (the
// register binning of five or six rows where the segment fits it, else the
// general one); the launch keeps the larger register count of the two.
__global__ __launch_bounds__(1024) void k_bin_multi_rows(MultiBinArgs m)
{
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t wsum[16];
    const uint32_t l = uniform(find_link(m.wg_prefix, m.n, blockIdx.x));
    const BinArgs a = m.args[l];
    const uint32_t g = blockIdx.x - m.wg_prefix[l];
    if (a.r == 6 && a.pb <= 6u * 1024u) bin_reg<6, 6>(a, g, lds, wsum);
    else if (a.r == 5 && a.pb <= 7u * 1024u) bin_reg<5, 7>(a, g, lds, wsum);
    else bin_generic(a, g, lds, wsum);
}

// One wave per workgroup.  Workgroup g: XCD g mod 8, the (g mod 8) + 8 * (w /
// parts)-th bin from the top with w = g / 8, segments [part * per_part, ...),
// 64 segments per round: lane j holds segment j's run of the bin, and the
// wave walks the concatenated runs 64 items at a time.
constexpr uint32_t APPLY_UNROLL = 2;      // items per lane in flight

template <bool PACK, class T>
__device__ __forceinline__ void apply_body(const ApplyArgs& a, uint32_t g)
{
    const uint64_t seg_words = PACK ? packed_seg_words(a.seg) : a.seg;   // item words per segment
    const uint32_t w = g >> 3;
    const uint32_t walk = (g & 7u) + 8u * (w / a.parts);
    if (walk >= a.n_bins) return;
    const uint32_t bin = a.n_bins - 1u - walk;     // highest bins first: the lowest stay cached for hot detection
    const uint32_t part = w % a.parts;
    const uint32_t lane = threadIdx.x;
    const uint32_t j0 = part * a.per_part;
    const uint32_t j1 = min(a.blocks, j0 + a.per_part);
    T* base = reinterpret_cast<T*>(a.state) + ((uint64_t)bin << a.bin_shift);    // bins count cells
    const T stamp = (T)a.stamp;
    const uint32_t* row = a.table + (uint64_t)bin * a.blocks;
    for (uint32_t jb = j0; jb < j1; jb += 64u) {
        const uint32_t j = jb + lane;
        uint32_t st = 0, c = 0;
        if (j < j1) {
            st = row[j];
            c = row[a.blocks + j] - st;
        }
        uint32_t incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(incl, o, 64);
            if (lane >= (uint32_t)o) incl += v;
        }
        const uint32_t excl = incl - c;
        const uint32_t total = __shfl(incl, 63, 64);
        for (uint32_t t0 = 0; t0 < total; t0 += 64u * APPLY_UNROLL) {
            // every lane loads (past the end: the first word of segment jb),
            // so that the loads issue back to back and are waited for once
            uint32_t it[APPLY_UNROLL], sg[APPLY_UNROLL];
            bool ok[APPLY_UNROLL];
#pragma unroll
            for (int u = 0; u < (int)APPLY_UNROLL; u++) {
                const uint32_t t = t0 + (uint32_t)u * 64u + lane;
                // the run holding item t: the largest lane whose run starts at or before t
                uint32_t lo = 0;
#pragma unroll
                for (uint32_t sft = 32; sft > 0; sft >>= 1) {
                    const uint32_t e = __shfl(excl, (int)(lo + sft), 64);
                    if (e <= t) lo += sft;
                }
                const uint32_t rs = __shfl(st, (int)lo, 64);
                const uint32_t re = __shfl(excl, (int)lo, 64);
                ok[u] = t < total;
                it[u] = ok[u] ? rs + (t - re) : 0u;
                sg[u] = ok[u] ? jb + lo : jb;
            }
            uint64_t raw[APPLY_UNROLL];
#pragma unroll
            for (int u = 0; u < (int)APPLY_UNROLL; u++) {
                const uint64_t w = (uint64_t)sg[u] * seg_words + (PACK ? it[u] / 3u : it[u]);
                raw[u] = PACK ? reinterpret_cast<const uint64_t*>(a.items)[w] : (uint64_t)a.items[w];
            }
            // offsets taken on every lane and pinned before the first store (an
            // empty asm reading them), so that no load sinks into a store's
            // branch and waits for the stores before it
            uint32_t off[APPLY_UNROLL];
#pragma unroll
            for (int u = 0; u < (int)APPLY_UNROLL; u++) {
                off[u] = PACK ? (uint32_t)(raw[u] >> (21u * (it[u] % 3u))) & 0x1FFFFFu : (uint32_t)raw[u];
                asm volatile("" : : "v"(off[u]));
            }
#pragma unroll
            for (int u = 0; u < (int)APPLY_UNROLL; u++)
                if (ok[u]) base[off[u]] = stamp;
        }
    }
}

template <bool PACK, class T>
__global__ __launch_bounds__(64) void k_apply(ApplyArgs a)
{
    apply_body<PACK, T>(a, blockIdx.x);
}

// Several links in one launch (8-bit cells), as k_bin_multi.
template <bool PACK>
__global__ __launch_bounds__(64) void k_apply_multi(MultiApplyArgs m)
{
    const uint32_t l = uniform(find_link(m.wg_prefix, m.n, blockIdx.x));
    const ApplyArgs a = m.args[l];
    apply_body<PACK, uint8_t>(a, blockIdx.x - m.wg_prefix[l]);
}

// Counted variant: one workgroup per bin.  The walk over the bin's items only
// marks their cells in an LDS bitmap (a bit per cell); then every marked cell
// is visited once, 16-byte chunk by chunk: a cell whose stamp is not the open
// slice's yet takes it and moves in its estimator's per-slot counters (+1 for
// the open slot, -1 for the slot of an old stamp still in the window).
// Stamps of earlier launches into the same slice are recognised by their
// value, so every cell is counted once per slice.  The workgroup owns its
// bin's cells and estimators: chunks are written back whole, and the
// counters, summed in LDS, are added to memory by atomics whose result is
// unused (so that nothing waits for a read of the old values).
constexpr uint32_t CAPPLY_WAVES = 16;
constexpr uint32_t CAPPLY_CHUNKS = 4;     // bitmap words per thread in flight in the visit
constexpr uint32_t CAPPLY_LIST = 4096;    // marked words listed for the visit (more: the whole bitmap is swept)

// Add d to 16-bit counter i of the LDS counters (two biased halves per word;
// the halves never carry into each other, so a 32-bit add does it).
__device__ __forceinline__ void cnt_add(uint32_t* cw, uint32_t i, int d)
{
    atomicAdd(&cw[i >> 1], (uint32_t)d << ((i & 1u) * 16u));
}

// The marked cells of one 4-byte word (mask m, a bit per byte): the new
// stamps, the count of cells restamped, and -1 on the slot of every old stamp
// still in the window (counters ce0 + slot of the LDS counters cw).  Byte
// masks are formed SWAR; only the restamped cells with an old stamp are
// visited one by one.
__device__ __forceinline__ uint32_t stamp_word(uint32_t x, uint32_t m, uint32_t stamp, uint32_t k, uint32_t slot,
                                               uint32_t* cw, uint32_t ce0, uint32_t& changed)
{
    const uint32_t lanes = ((m * 0x00204081u) & 0x01010101u) * 0xFFu;       // bit i of m -> byte i
    const uint32_t y = x ^ (stamp * 0x01010101u);
    const uint32_t ne = ((((y & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | y) & 0x80808080u) >> 7;   // byte != stamp
    const uint32_t nz = ((((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u) >> 7;   // byte != 0
    const uint32_t chg = lanes & (ne * 0xFFu);
    changed += (uint32_t)__popc(chg) >> 3;
    uint32_t old = (chg & (nz * 0xFFu)) & 0x01010101u;      // restamped cells with an old stamp
    while (old) {
        const uint32_t i = ((uint32_t)__ffs(old) - 1u) >> 3;
        old &= old - 1u;
        const uint32_t b = (x >> (8u * i)) & 0xFFu;
        const uint32_t d = (stamp + 255u - b) % 255u;      // slices since the old stamp
        if (d < k) cnt_add(cw, ce0 + (slot >= d ? slot - d : slot + k - d), -1);
    }
    return (x & ~chg) | ((stamp * 0x01010101u) & chg);
}

// Workgroup barrier that orders LDS only: global stores issued before it stay
// in flight (a plain __syncthreads waits for their completion).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The first half of the bitmap stores (bin `bin` of this launch): the LDS is
// cleared -- its first bm_words words, the bitmap of the bin's cells, to 0,
// the rest of its n_words to 0x80008000 (two biased 16-bit counters) -- and
// every cell that an offset of the bin names is marked in the bitmap; a
// word's first mark appends it to list (the marked words, in the order they
// were first marked; n_list counts them all, also past CAPPLY_LIST).
__device__ __forceinline__ void mark_runs(const ApplyArgs& a, uint32_t bin, uint32_t* lds, uint32_t bm_words,
                                          uint32_t n_words, uint16_t* list, uint32_t& n_list)
{
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t* row = a.table + (uint64_t)bin * a.blocks;
    // this lane's run (segment j) of the wave's first group, loaded before the
    // LDS is cleared so that the two overlap
    uint32_t j = wave * 64u + lane, st = 0, c = 0;
    if (j < a.blocks) {
        st = row[j];
        c = row[a.blocks + j] - st;
    }
    for (uint32_t i = threadIdx.x; i < n_words; i += blockDim.x) lds[i] = i < bm_words ? 0u : 0x80008000u;
    if (threadIdx.x == 0) n_list = 0u;
    __syncthreads();
    // walk: lane j reads run j itself, four aligned 16-byte loads (24 offsets)
    // at a time; words past the segment's end are read from its last pair and
    // fall outside the run
    const uint64_t seg_words = packed_seg_words(a.seg);
    const uint64_t* items = reinterpret_cast<const uint64_t*>(a.items);
    const uint32_t last_pair = (uint32_t)(seg_words / 2u) - 1u;
    for (uint32_t jb = wave * 64u; jb < a.blocks; jb += 64u * CAPPLY_WAVES) {
        if (jb != wave * 64u) {
            j = jb + lane;
            st = 0;
            c = 0;
            if (j < a.blocks) {
                st = row[j];
                c = row[a.blocks + j] - st;
            }
        }
        const uint32_t end = st + c;                                   // items [st, end)
        const uint32_t w_end = (end + 2u) / 3u;
        const uint4* seg = reinterpret_cast<const uint4*>(items + (uint64_t)min(j, a.blocks - 1u) * seg_words);
        for (uint32_t base = (st / 3u) & ~1u; c && base < w_end; base += 8u) {
            uint4 q[4];
#pragma unroll
            for (int i = 0; i < 4; i++) q[i] = seg[min(base / 2u + (uint32_t)i, last_pair)];
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const uint64_t wd = (i & 1) ? ((uint64_t)q[i / 2].w << 32 | q[i / 2].z)
                                            : ((uint64_t)q[i / 2].y << 32 | q[i / 2].x);
                const uint32_t i0 = 3u * (base + (uint32_t)i);
#pragma unroll
                for (uint32_t sft = 0; sft < 3; sft++) {
                    if (i0 + sft < st || i0 + sft >= end) continue;
                    const uint32_t off = (uint32_t)(wd >> (21u * sft)) & 0x1FFFFFu;
                    if (atomicOr(&lds[off >> 5], 1u << (off & 31u)) == 0u) {
                        const uint32_t at = atomicAdd(&n_list, 1u);
                        if (at < CAPPLY_LIST) list[at] = (uint16_t)(off >> 5);
                    }
                }
            }
        }
    }
    __syncthreads();
}

// (workgroup g of this link's launch; lds: the dynamic LDS; list / n_list:
// the workgroup's list of marked words)
__device__ __forceinline__ void apply_counted_body(const ApplyArgs& a, uint32_t g, uint32_t* lds, uint16_t* list,
                                                   uint32_t& n_list, uint32_t* wsum)
{
    // workgroup g runs on XCD g mod 8, which takes a contiguous eighth of the
    // bins in order: neighbouring bins, whose runs share cache lines in every
    // segment, are read through the same L2 at about the same time
    const uint32_t per_xcd = (a.n_bins + 7u) >> 3;
    const uint32_t bin = (g & 7u) * per_xcd + (g >> 3);
    if (bin >= a.n_bins) return;
    const uint32_t bm_words = 1u << (a.bin_shift - 5u);
    const uint32_t n_est = 1u << (a.bin_shift - a.log2eta);
    const uint32_t k = a.k, slot = a.slot;
    const uint32_t n_words = bm_words + (n_est * k + 1u) / 2u;
    uint32_t* bm = lds;
    uint32_t* cnt = lds + bm_words;                 // 16-bit counters [estimator][slot], biased by 0x8000
    mark_runs(a, bin, lds, bm_words, n_words, list, n_list);
    // visit: bitmap word w covers the 32 cells of 16-byte chunks 2w and 2w + 1;
    // unmarked halves load the bin's first chunk instead (one line, cached),
    // so that the loads issue back to back
    uint4* chunk = reinterpret_cast<uint4*>(a.state + ((uint64_t)bin << a.bin_shift));
    const uint32_t stamp = a.stamp;
    // the listed words when they all fit the list, else every word of the bitmap
    const bool listed = n_list <= CAPPLY_LIST;
    const uint32_t n_visit = listed ? n_list : bm_words;
    // new stamps and counter moves for every chunk of a pass first, then its
    // stores; the last pass (the only one when the list holds every marked
    // word) stores after the counters, at the kernel's end, so that no wait
    // of the workgroup covers a store
    uint4 v[2 * CAPPLY_CHUNKS];
    uint32_t wd[CAPPLY_CHUNKS];
    uint32_t dirty = 0;
    for (uint32_t w0 = threadIdx.x; w0 < n_visit; w0 += blockDim.x * CAPPLY_CHUNKS) {
#pragma unroll
        for (int u = 0; u < (int)(2 * CAPPLY_CHUNKS); u++)
            if (dirty & (1u << u)) chunk[2u * wd[u / 2] + (u & 1)] = v[u];
        dirty = 0;
        uint32_t m[CAPPLY_CHUNKS];
#pragma unroll
        for (int u = 0; u < (int)CAPPLY_CHUNKS; u++) {
            const uint32_t i = w0 + (uint32_t)u * blockDim.x;
            wd[u] = i < n_visit ? (listed ? (uint32_t)list[i] : i) : 0u;
            m[u] = i < n_visit ? bm[wd[u]] : 0u;
        }
#pragma unroll
        for (int u = 0; u < (int)CAPPLY_CHUNKS; u++) {
            const uint32_t w = wd[u];
            v[2 * u] = chunk[(m[u] & 0xFFFFu) ? 2u * w : 0u];
            v[2 * u + 1] = chunk[(m[u] >> 16) ? 2u * w + 1u : 0u];
        }
#pragma unroll
        for (int u = 0; u < (int)CAPPLY_CHUNKS; u++) {
            if (!m[u]) continue;
            const uint32_t ce0 = ((wd[u] << 5) >> a.log2eta) * k;
            uint32_t changed = 0;
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const uint32_t mh = (m[u] >> (16 * h)) & 0xFFFFu;
                if (!mh) continue;
                uint4& x = v[2 * u + h];
                const uint32_t before = changed;
                x.x = stamp_word(x.x, mh & 0xFu, stamp, k, slot, cnt, ce0, changed);
                x.y = stamp_word(x.y, (mh >> 4) & 0xFu, stamp, k, slot, cnt, ce0, changed);
                x.z = stamp_word(x.z, (mh >> 8) & 0xFu, stamp, k, slot, cnt, ce0, changed);
                x.w = stamp_word(x.w, (mh >> 12) & 0xFu, stamp, k, slot, cnt, ce0, changed);
                if (changed != before) dirty |= 1u << (2 * u + h);
            }
            if (changed) cnt_add(cnt, ce0 + slot, (int)changed);
        }
    }
    // every chunk load is waited for here, before any store or counter atomic
    // is in flight (a wait after them would count them too)
#pragma unroll
    for (int u = 0; u < (int)(2 * CAPPLY_CHUNKS); u++) asm volatile("" : : "v"(v[u].x), "v"(v[u].y), "v"(v[u].z), "v"(v[u].w));
    lds_barrier();
    // counters added without waiting for them (atomics whose result is unused)
    // (slot-major in memory: consecutive threads take consecutive estimators)
    uint32_t* dst = a.counts + ((uint64_t)bin << (a.bin_shift - a.log2eta));
    for (uint32_t i = threadIdx.x; i < n_est * (k + 1u); i += blockDim.x) {
        const uint32_t j = i / n_est, e = i - j * n_est;
        int c = 0;
        if (j < k) {
            const uint32_t c16 = e * k + j;
            c = (int)((cnt[c16 >> 1] >> ((c16 & 1u) * 16u)) & 0xFFFFu) - 0x8000;
        } else {
            // slot k: the estimator's live-cell total, moved by the sum of its
            // slots' moves (+1 for every cell that was not live before)
            for (uint32_t jj = 0; jj < k; jj++) {
                const uint32_t c16 = e * k + jj;
                c += (int)((cnt[c16 >> 1] >> ((c16 & 1u) * 16u)) & 0xFFFFu) - 0x8000;
            }
        }
        if (c) atomicAdd(&dst[(uint64_t)j * a.n_se + e], (uint32_t)c);
    }
#pragma unroll
    for (int u = 0; u < (int)(2 * CAPPLY_CHUNKS); u++)
        if (dirty & (1u << u)) chunk[2u * wd[u / 2] + (u & 1)] = v[u];
    // the stored values stay live to here: no register of a store in flight
    // is reused (which would wait for the store)
#pragma unroll
    for (int u = 0; u < (int)(2 * CAPPLY_CHUNKS); u++) asm volatile("" : : "v"(v[u].x), "v"(v[u].y), "v"(v[u].z), "v"(v[u].w));
}

__global__ __launch_bounds__(64 * CAPPLY_WAVES) void k_apply_counted(ApplyArgs a)
{
    extern __shared__ uint32_t lds[];
    // the marked words, in the order they were first marked
    __shared__ uint16_t list[CAPPLY_LIST];
    __shared__ uint32_t n_list;
    __shared__ uint32_t wsum[16];
    apply_counted_body(a, blockIdx.x, lds, list, n_list, wsum);
}

// Several links in one launch, as k_bin_multi (the dynamic LDS is sized for
// the largest of them).
__global__ __launch_bounds__(64 * CAPPLY_WAVES) void k_apply_counted_multi(MultiApplyArgs m)
{
    extern __shared__ uint32_t lds[];
    __shared__ uint16_t list[CAPPLY_LIST];
    __shared__ uint32_t n_list;
    __shared__ uint32_t wsum[16];
    const uint32_t l = uniform(find_link(m.wg_prefix, m.n, blockIdx.x));
    const ApplyArgs a = m.args[l];
    apply_counted_body(a, blockIdx.x - m.wg_prefix[l], lds, list, n_list, wsum);
}

// 16-bit cells (windows above 254 slots), which keep no counters: the bitmap
// stores without the counters, for calls whose offsets repeat cells.  After
// the walk a bitmap word covers 32 cells, four 16-byte chunks of eight
// cells; each chunk holding a marked cell is read once, its marked cells take
// the stamp, and it is written back if that changed it.  Unmarked chunks of a
// visited word load the bin's first chunk instead (one line, cached), so that
// the loads issue back to back.
constexpr uint32_t MARKED16_WORDS = 2;    // bitmap words per thread in flight in the visit

// Cells (two to a 32-bit word) whose bits are set in m2 take the doubled stamp s2.
__device__ __forceinline__ uint32_t restamp16(uint32_t x, uint32_t m2, uint32_t s2)
{
    const uint32_t lanes = ((m2 & 1u) ? 0x0000FFFFu : 0u) | ((m2 & 2u) ? 0xFFFF0000u : 0u);
    return (x & ~lanes) | (s2 & lanes);
}

__global__ __launch_bounds__(64 * CAPPLY_WAVES) void k_apply_marked16(ApplyArgs a)
{
    extern __shared__ uint32_t lds[];
    __shared__ uint16_t list[CAPPLY_LIST];
    __shared__ uint32_t n_list;
    const uint32_t g = blockIdx.x;
    const uint32_t per_xcd = (a.n_bins + 7u) >> 3;
    const uint32_t bin = (g & 7u) * per_xcd + (g >> 3);
    if (bin >= a.n_bins) return;
    const uint32_t bm_words = 1u << (a.bin_shift - 5u);
    mark_runs(a, bin, lds, bm_words, bm_words, list, n_list);
    uint4* chunk = reinterpret_cast<uint4*>(a.state + ((uint64_t)bin << (a.bin_shift + 1u)));    // 2 bytes a cell
    const uint32_t s2 = (a.stamp & 0xFFFFu) * 0x00010001u;
    const bool listed = n_list <= CAPPLY_LIST;
    const uint32_t n_visit = listed ? n_list : bm_words;
    for (uint32_t w0 = threadIdx.x; w0 < n_visit; w0 += blockDim.x * MARKED16_WORDS) {
        uint32_t wd[MARKED16_WORDS], m[MARKED16_WORDS];
#pragma unroll
        for (int u = 0; u < (int)MARKED16_WORDS; u++) {
            const uint32_t i = w0 + (uint32_t)u * blockDim.x;
            wd[u] = i < n_visit ? (listed ? (uint32_t)list[i] : i) : 0u;
            m[u] = i < n_visit ? lds[wd[u]] : 0u;
        }
        uint4 v[4 * MARKED16_WORDS];
#pragma unroll
        for (int u = 0; u < (int)MARKED16_WORDS; u++)
#pragma unroll
            for (int c = 0; c < 4; c++) v[4 * u + c] = chunk[((m[u] >> (8 * c)) & 0xFFu) ? 4u * wd[u] + c : 0u];
#pragma unroll
        for (int u = 0; u < (int)MARKED16_WORDS; u++) {
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const uint32_t mc = (m[u] >> (8 * c)) & 0xFFu;     // cells 8c .. 8c + 7 of the word
                if (!mc) continue;
                const uint4 x = v[4 * u + c];
                uint4 y;
                y.x = restamp16(x.x, mc & 3u, s2);
                y.y = restamp16(x.y, (mc >> 2) & 3u, s2);
                y.z = restamp16(x.z, (mc >> 4) & 3u, s2);
                y.w = restamp16(x.w, (mc >> 6) & 3u, s2);
                if (y.x != x.x || y.y != x.y || y.z != x.z || y.w != x.w) chunk[4u * wd[u] + c] = y;
            }
        }
    }
}

// ---------------------------------------------------------------- hot detection
// One wave per sliding estimator: R_k = live cells (Sec. 3.2); a hot estimator
// (Sec. 3.3) sets its bit in the row bitmask and in the key-transposed bitmask;
// estimators of this slot's expiry phase clear their dead cells.  Up to CH
// 1 KiB wave loads in flight per group.

constexpr uint32_t DETECT_WAVES = 4;   // waves (estimators) per workgroup (4, 8, 16 measured: 4 best)

// The end of one estimator's test: R_k, and if hot, its live-cell snapshot
// (for the final test, which then reads no state) and its bits in the row
// and key-transposed bitmasks.
// R_k of estimator s and, if it is hot, its bits in the row and
// key-transposed bitmasks (lane 0 writes).
__device__ __forceinline__ void hot_mark(const LinkDesc* D, uint64_t s, uint32_t live, uint32_t lane)
{
    if (lane == 0) {
        D->rk[s] = live;
        if (live >= D->T) {
            const uint32_t q = D->q;
            const uint32_t row = (uint32_t)(s >> q), c = (uint32_t)s & ((1u << q) - 1u);
            const uint32_t sh = q - D->delta;
            const uint32_t key = c & ((1u << sh) - 1u), j = c >> sh;
            const uint32_t rw = q >= 6 ? (1u << (q - 6)) : 1u;    // words per row bitmask
            atomicOr(reinterpret_cast<unsigned long long*>(D->hotbits) + (uint64_t)row * rw + (c >> 6),
                     1ull << (c & 63u));
            atomicOr(reinterpret_cast<unsigned long long*>(D->hotT) + ((uint64_t)row * (1ull << sh) + key) * D->nw +
                         (j >> 6),
                     1ull << (j & 63u));
        }
    }
}

template <bool SNAP>
__device__ __forceinline__ void hot_finish(const LinkDesc* D, uint64_t s, uint32_t live, const uint4* se, uint32_t lane)
{
    const uint32_t log2eta = D->log2eta;
    if (SNAP && live >= D->T) {
        const uint32_t chunks = 1u << (log2eta - 4);
        uint16_t* snap = D->live16 + s * chunks;
        for (uint32_t c = lane; c < chunks; c += 64u) snap[c] = (uint16_t)live_mask16(se[c], D->L);
    }
    hot_mark(D, s, live, lane);
}

// A wave covers 4 KiB of state at least: one estimator when eta >= 4096, else
// 4096 / eta consecutive estimators (load round c of the wave's four belongs
// to estimator c / (eta / 1024)), so that small estimators still give every
// wave four 1 KiB loads in flight.
template <int CH, bool SMALL>
__global__ __launch_bounds__(64 * DETECT_WAVES) void k_hot_detect(DetectArgs a)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t g = (uint64_t)blockIdx.x * DETECT_WAVES + (threadIdx.x >> 6);
    // batches of up to 256 links search the wave prefix in LDS (one coalesced
    // load per workgroup instead of a chain of dependent loads per wave)
    __shared__ unsigned long long pre_lds[SMALL ? 257 : 1];
    const bool lds_prefix = SMALL && a.n_links > 1 && a.n_links <= 256u && !a.expire_only;
    if (lds_prefix) {
        for (uint32_t i = threadIdx.x; i <= a.n_links; i += blockDim.x) pre_lds[i] = a.se_prefix[i];
        __syncthreads();
    }
    if (g >= a.total) return;
    uint32_t l;
    uint64_t s;                                         // first estimator of the wave
    if (a.expire_only) {
        l = 0;
        s = a.links[0].expire_phase + g * a.links[0].expire_period;
        if (s >= a.links[0].n_se) return;
    } else {
        const unsigned long long* pre = lds_prefix ? pre_lds : reinterpret_cast<const unsigned long long*>(a.se_prefix);
        l = uniform(find_link(pre, a.n_links, g));
        const uint32_t lg = a.links[l].log2eta;
        s = (g - pre[l]) << (lg < 12u ? 12u - lg : 0u);
    }
    const LinkDesc* D = a.links + l;
    const uint32_t log2eta = D->log2eta;
    const LiveCfg L = D->L;
    const bool count = !a.expire_only;
    if (SMALL && log2eta < 12u && count) {
        // several estimators per wave: four rounds of 1 KiB, one estimator per
        // 2^(log2eta-10) rounds; every estimator is whole in this wave
        const uint32_t rpe = 1u << (log2eta - 10);       // rounds per estimator (1 or 2)
        const uint32_t ne = 4u / rpe;                    // estimators of the wave
        uint4* base = reinterpret_cast<uint4*>(D->state + (s << log2eta));
        uint4 v[4];
#pragma unroll
        for (int c = 0; c < 4; c++) v[c] = base[c * 64u + lane];
        uint32_t cnt[4];
#pragma unroll
        for (int c = 0; c < 4; c++)
            cnt[c] = __popc(live_bits(v[c].x, L)) + __popc(live_bits(v[c].y, L)) + __popc(live_bits(v[c].z, L)) +
                     __popc(live_bits(v[c].w, L));
        for (uint32_t e = 0; e < ne; e++) {
            const uint64_t se_idx = s + e;
            const bool expire = (se_idx % D->expire_period) == D->expire_phase;
            uint32_t live = 0;
#pragma unroll
            for (int c = 0; c < 4; c++) {
                if ((uint32_t)c / rpe != e) continue;
                live += cnt[c];
                if (expire) {
                    uint4 n;
                    n.x = expire_word(v[c].x, L); n.y = expire_word(v[c].y, L);
                    n.z = expire_word(v[c].z, L); n.w = expire_word(v[c].w, L);
                    if (n.x != v[c].x || n.y != v[c].y || n.z != v[c].z || n.w != v[c].w) base[c * 64u + lane] = n;
                }
            }
            live = wave_sum(live);
            hot_finish<true>(D, se_idx, live, base + (uint64_t)e * rpe * 64u, lane);
        }
        return;
    }
    uint4* se = reinterpret_cast<uint4*>(D->state + (s << log2eta));
    const uint32_t per_lane = (1u << log2eta) >> 10;    // uint4 chunks per lane (eta >= 1024)
    const bool expire = (s % D->expire_period) == D->expire_phase;
    uint32_t live = 0;
    uint4 v[CH];                                        // the last group stays for the snapshot
    for (uint32_t g0 = 0; g0 < per_lane; g0 += CH) {
#pragma unroll
        for (int c = 0; c < CH; c++)
            v[c] = (g0 + c < per_lane) ? se[(g0 + c) * 64u + lane] : make_uint4(0u, 0u, 0u, 0u);
        if (count) {
#pragma unroll
            for (int c = 0; c < CH; c++)
                if (g0 + c < per_lane)
                    live += __popc(live_bits(v[c].x, L)) + __popc(live_bits(v[c].y, L)) +
                            __popc(live_bits(v[c].z, L)) + __popc(live_bits(v[c].w, L));
        }
        if (expire) {
#pragma unroll
            for (int c = 0; c < CH; c++) {
                if (g0 + c >= per_lane) continue;
                uint4 n;
                n.x = expire_word(v[c].x, L); n.y = expire_word(v[c].y, L);
                n.z = expire_word(v[c].z, L); n.w = expire_word(v[c].w, L);
                if (n.x != v[c].x || n.y != v[c].y || n.z != v[c].z || n.w != v[c].w)
                    se[(g0 + c) * 64u + lane] = n;
            }
        }
    }
    if (count) {
        live = wave_sum(live);
        if (per_lane <= (uint32_t)CH && live >= D->T) {
            // the whole estimator is still in registers: snapshot from there
            uint16_t* snap = D->live16 + s * (per_lane * 64u);
#pragma unroll
            for (int c = 0; c < CH; c++)
                if ((uint32_t)c < per_lane) snap[c * 64u + lane] = (uint16_t)live_mask16(v[c], L);
            hot_finish<false>(D, s, live, se, lane);
        } else {
            hot_finish<true>(D, s, live, se, lane);
        }
    }
}

// 16-bit cells (windows above 254 slots), one link: one wave per estimator;
// in round c lane j takes the 16 cells of snapshot word c * 64 + j (two
// 16-byte chunks, so a wave reads 2 KiB in one go).  Up to CH rounds stay in
// registers for the snapshot of a hot estimator; larger estimators are read
// again.  With expire_only, only the estimators of this slot's expiry phase
// are visited (and not counted).
template <int CH>
__global__ __launch_bounds__(64 * DETECT_WAVES) void k_hot_detect16(DetectArgs a)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t g = (uint64_t)blockIdx.x * DETECT_WAVES + (threadIdx.x >> 6);
    if (g >= a.total) return;
    const LinkDesc* D = a.links;
    uint64_t s = g;
    if (a.expire_only) {
        s = D->expire_phase + g * D->expire_period;
        if (s >= D->n_se) return;
    }
    const uint32_t log2eta = D->log2eta;
    const LiveCfg L = D->L;
    const uint32_t rounds = (1u << log2eta) >> 10;      // 1024 cells per wave round (eta >= 1024)
    uint4* se = reinterpret_cast<uint4*>(D->state + (s << (log2eta + 1)));
    const bool expire = (s % D->expire_period) == D->expire_phase;
    const bool count = !a.expire_only;
    uint32_t live = 0;
    uint32_t snap[CH];
    for (uint32_t g0 = 0; g0 < rounds; g0 += CH) {
        uint4 v[2 * CH];
#pragma unroll
        for (int c = 0; c < CH; c++) {
            const uint64_t w = 2ull * ((g0 + (uint32_t)c) * 64u + lane);
            if (g0 + (uint32_t)c < rounds) {
                v[2 * c] = se[w];
                v[2 * c + 1] = se[w + 1];
            }
        }
#pragma unroll
        for (int c = 0; c < CH; c++) {
            if (g0 + (uint32_t)c >= rounds) continue;
            const uint32_t m = live_mask8_c16(v[2 * c], L) | (live_mask8_c16(v[2 * c + 1], L) << 8);
            snap[c] = m;
            live += __popc(m);
            if (expire) {
                const uint64_t w = 2ull * ((g0 + (uint32_t)c) * 64u + lane);
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const uint4 x = v[2 * c + h];
                    uint4 n;
                    n.x = expire_word16(x.x, L); n.y = expire_word16(x.y, L);
                    n.z = expire_word16(x.z, L); n.w = expire_word16(x.w, L);
                    if (n.x != x.x || n.y != x.y || n.z != x.z || n.w != x.w) se[w + h] = n;
                }
            }
        }
    }
    if (!count) return;
    live = wave_sum(live);
    if (live >= D->T) {
        uint16_t* out = D->live16 + s * (1u << (log2eta - 4));
        if (rounds <= (uint32_t)CH) {
#pragma unroll
            for (int c = 0; c < CH; c++)
                if ((uint32_t)c < rounds) out[c * 64u + lane] = (uint16_t)snap[c];
        } else {
            // liveness is unchanged by the expiry writes above (dead cells only)
            for (uint32_t c = 0; c < rounds; c++) {
                const uint64_t w = 2ull * (c * 64u + lane);
                out[c * 64u + lane] = (uint16_t)(live_mask8_c16(se[w], L) | (live_mask8_c16(se[w + 1], L) << 8));
            }
        }
    }
    hot_mark(D, s, live, lane);
}

// ---------------------------------------------------------------- counted detection
// R_k of every estimator from its counters (one thread per estimator): slot
// k holds the live-cell total, which every store moves by the sum of its
// moves of the per-slice slots -- the same live-cell count as a scan of the
// state, since every live cell carries the stamp of exactly one slice of the
// window.  Only the estimators that need their cells are then visited, by
// the workgroup's four waves in turn: hot ones (snapshot and bitmask bits)
// and those of this slot's expiry phase (dead cells cleared).  The slot of
// the next slice leaves the total and is zeroed for its scans.
// (workgroup blk of this link's launch; todo / todo_live / n_todo: the
// workgroup's list of estimators to visit)
__device__ __forceinline__ void count_body(const LinkDesc* D, uint64_t n_se, uint32_t blk, uint32_t* todo,
                                           uint32_t* todo_live, uint32_t& n_todo)
{
    if (threadIdx.x == 0) n_todo = 0u;
    __syncthreads();
    const uint64_t s0 = (uint64_t)blk * 256u;
    const uint64_t s = s0 + threadIdx.x;
    const uint32_t k = D->k;
    const uint32_t next = (uint32_t)((D->clock->t + 1ull) % k);
    if (s < n_se) {
        // the live-cell total (slot k) is R_k; the slot of the next slice,
        // whose cells leave the window, leaves the total and is zeroed
        const uint32_t live = D->counts[(uint64_t)k * n_se + s];
        D->counts[(uint64_t)k * n_se + s] = live - D->counts[(uint64_t)next * n_se + s];
        D->counts[(uint64_t)next * n_se + s] = 0u;
        const bool hot = live >= D->T;
        const bool expire = (s % D->expire_period) == D->expire_phase;
        if (!hot) D->rk[s] = live;
        if (hot || expire) {
            const uint32_t at = atomicAdd(&n_todo, 1u);
            todo[at] = threadIdx.x | (hot ? 0x100u : 0u) | (expire ? 0x200u : 0u);
            todo_live[at] = live;
        }
    }
    __syncthreads();
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t log2eta = D->log2eta;
    const uint32_t chunks = 1u << (log2eta - 4);
    const LiveCfg L = D->L;
    for (uint32_t i = wave; i < n_todo; i += 4u) {
        const uint32_t e = todo[i];
        const uint64_t si = s0 + (e & 0xFFu);
        const bool hi = (e & 0x100u) != 0u, ei = (e & 0x200u) != 0u;
        uint4* se = reinterpret_cast<uint4*>(D->state + (si << log2eta));
        uint16_t* snap = D->live16 + si * chunks;
        for (uint32_t c = lane; c < chunks; c += 64u) {
            const uint4 v = se[c];
            if (hi) snap[c] = (uint16_t)live_mask16(v, L);
            if (ei) {
                uint4 n;
                n.x = expire_word(v.x, L); n.y = expire_word(v.y, L);
                n.z = expire_word(v.z, L); n.w = expire_word(v.w, L);
                if (n.x != v.x || n.y != v.y || n.z != v.z || n.w != v.w) se[c] = n;
            }
        }
        if (hi) hot_finish<false>(D, si, todo_live[i], se, lane);
    }
}

__global__ __launch_bounds__(256) void k_count(const LinkDesc* link, uint64_t n_se)
{
    __shared__ uint32_t todo[256];      // local estimator | 0x100 hot | 0x200 expiring
    __shared__ uint32_t todo_live[256];
    __shared__ uint32_t n_todo;
    count_body(link, n_se, blockIdx.x, todo, todo_live, n_todo);
}

// Several counted links of an engine in one launch: workgroup g works for
// link ids[l] with wg_prefix[l] <= g < wg_prefix[l + 1].
__global__ __launch_bounds__(256) void k_count_multi(CountMultiArgs m)
{
    __shared__ uint32_t todo[256];
    __shared__ uint32_t todo_live[256];
    __shared__ uint32_t n_todo;
    const uint32_t l = uniform(find_link(m.wg_prefix, m.n, blockIdx.x));
    const LinkDesc* D = m.links + m.ids[l];
    count_body(D, D->n_se, blockIdx.x - m.wg_prefix[l], todo, todo_live, n_todo);
}

// Bytes of a word equal to stamp s.
__device__ __forceinline__ uint32_t count_eq(uint32_t w, uint32_t s)
{
    const uint32_t x = w ^ (s * 0x01010101u);
    const uint32_t nz = (((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
    return 4u - __popc(nz);
}

// The per-slot counters rebuilt from the state (one wave per estimator): for
// every slice of the window, the cells holding its stamp.
__global__ __launch_bounds__(256) void k_recount(const LinkDesc* link, uint64_t n_se)
{
    const LinkDesc* D = link;
    const uint64_t s = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    if (s >= n_se) return;
    const uint32_t k = D->k;
    const unsigned long long t = D->clock->t;
    const uint32_t slot = (uint32_t)(t % k);
    const uint32_t chunks = 1u << (D->log2eta - 4);
    const uint4* se = reinterpret_cast<const uint4*>(D->state + (s << D->log2eta));
    uint32_t total = 0;
    for (uint32_t j = 0; j < k; j++) {
        const uint32_t d = slot >= j ? slot - j : slot + k - j;   // slices back from t
        uint32_t n = 0;
        if (d <= t) {
            const uint32_t st = 1u + (uint32_t)((t - d) % 255ull);
            for (uint32_t c = lane; c < chunks; c += 64u) {
                const uint4 v = se[c];
                n += count_eq(v.x, st) + count_eq(v.y, st) + count_eq(v.z, st) + count_eq(v.w, st);
            }
        }
        n = wave_sum(n);
        total += n;
        if (lane == 0) D->counts[(uint64_t)j * n_se + s] = n;
    }
    if (lane == 0) D->counts[(uint64_t)k * n_se + s] = total;      // the live-cell total
}

// ---------------------------------------------------------------- hot lists
// One 1024-thread block per (link, row): the ascending list of hot columns,
// from the row bitmask.  The row-0 block also clears the link's counters.

__global__ __launch_bounds__(1024) void k_hot_compact(const LinkDesc* links, const uint32_t* row_table)
{
    __shared__ uint32_t lds[16];
    const uint32_t rt = row_table[blockIdx.x];
    const LinkDesc* D = links + (rt >> 8);
    const uint32_t row = rt & 255u;
    const uint32_t q = D->q;
    const uint32_t words = q >= 6 ? (1u << (q - 6)) : 1u;
    const uint64_t* bits = D->hotbits + (uint64_t)row * words;
    if (row == 0 && threadIdx.x == 0) {
        for (int l = 0; l < (int)MAX_ROWS; l++) D->ctl->level_n[l] = 0;
        D->ctl->n_acc = 0;
        D->ctl->n_out = 0;
    }
    const uint32_t per = (words + 1023u) / 1024u;
    const uint32_t w0 = min(words, threadIdx.x * per), w1 = min(words, w0 + per);
    uint32_t cnt = 0;
    for (uint32_t w = w0; w < w1; w++) cnt += __popcll(bits[w]);
    uint32_t total;
    uint32_t off = block_exclusive_scan_1024(cnt, lds, &total);
    uint32_t* list = D->hot_list + ((uint64_t)row << q);
    for (uint32_t w = w0; w < w1; w++) {
        uint64_t b = bits[w];
        while (b) {
            const uint32_t i = (uint32_t)__ffsll((long long)b) - 1u;
            b &= b - 1;
            list[off++] = w * 64u + i;
        }
    }
    if (threadIdx.x == 0) D->ctl->hot_n[row] = total;
}

// ---------------------------------------------------------------- level work
// Work items of one level for every link, prefix-summed; expansion levels pad
// each link to whole 256-item blocks so that a block never spans two links.

// Work items of one link at a level: 0 = |HSE(0)| x |HSE(1)| pairs of rows
// 0, 1; L = the tuples of level L-1 (extended by row L+2); LEVEL_VERIFY = the
// full tuples.  Expansion items are padded to whole 256-item workgroups, so a
// workgroup never spans two links and appends with one atomic.
__device__ __forceinline__ unsigned long long level_items(const LinkDesc* D, uint32_t level)
{
    const Ctl* c = D->ctl;
    unsigned long long n = 0;
    if (level == 0) {
        n = (unsigned long long)c->hot_n[0] * c->hot_n[1];
    } else if (level == LEVEL_VERIFY) {
        const unsigned long long m = c->level_n[D->r - 3];
        return m < D->max_tuples ? m : D->max_tuples;
    } else if (level + 2 < D->r) {
        const unsigned long long m = c->level_n[level - 1];
        n = m < D->max_tuples ? m : D->max_tuples;
    }
    return (n + 255ull) & ~255ull;
}

// Every 256-thread workgroup of a level kernel computes the level's prefix of
// work items over the links into LDS (pre[0..n_links]) from the counters the
// previous kernel left: no separate launch between levels.
__device__ void level_prefix_lds(const LevelArgs& a, unsigned long long* pre)
{
    __shared__ unsigned long long part[256];
    if (a.n_links == 1) {
        if (threadIdx.x == 0) {
            pre[0] = 0;
            pre[1] = level_items(a.links, a.level);
        }
        __syncthreads();
        return;
    }
    const uint32_t per = (a.n_links + 255u) / 256u;
    const uint32_t l0 = min(a.n_links, threadIdx.x * per), l1 = min(a.n_links, l0 + per);
    unsigned long long sum = 0;
    for (uint32_t l = l0; l < l1; l++) {
        const unsigned long long n = level_items(a.links + l, a.level);
        pre[l] = n;
        sum += n;
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    for (uint32_t o = 1; o < 256u; o <<= 1) {
        const unsigned long long v = threadIdx.x >= o ? part[threadIdx.x - o] : 0ull;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    unsigned long long run = part[threadIdx.x] - sum;
    for (uint32_t l = l0; l < l1; l++) {
        const unsigned long long n = pre[l];
        pre[l] = run;
        run += n;
    }
    if (threadIdx.x == 255u) pre[a.n_links] = part[255];
    __syncthreads();
}

// ---------------------------------------------------------------- expansion
// Sec. 4.2, with the cross products of Alg. 6/7 replaced by a lookup: for a
// tuple with he_0 and he_{i-1}, the overlap test fixes the low q-delta bits of
// he_i, so the candidates are exactly the hot columns of row i under that key
// (one transposed bitmask word per 64 candidates).  A tuple is stored as
// (he_0, x) with x the host bits regained so far; he_i = (x >> (i-1)delta) mod
// 2^q XOR he_0.  Tuples are appended with one atomic per block; their order is
// not deterministic, the set is.

template <bool EMIT>
__device__ __forceinline__ uint32_t extend_one(const LinkDesc* D, uint32_t he0, uint64_t x, uint32_t row,
                                               uint64_t* out_x, uint32_t* out_h0, uint64_t slot, uint32_t valid)
{
    if (!valid) return 0;
    const uint32_t q = D->q, delta = D->delta, nw = D->nw, key_bits = D->key_bits;
    const uint32_t qmask = (1u << q) - 1u;
    const uint32_t sh = q - delta;
    const uint32_t kmask = (1u << sh) - 1u;
    const uint32_t bprev = (uint32_t)(x >> ((row - 2) * delta)) & qmask;       // B(row-1)
    const uint32_t key = ((bprev >> delta) ^ he0) & kmask;
    const uint64_t* w = D->hotT + ((uint64_t)row * (1ull << sh) + key) * nw;
    const uint32_t newpos = (row - 2) * delta + q;           // first host bit B(row) adds
    const uint32_t dmask = (1u << delta) - 1u;
    const uint32_t top0 = he0 >> sh;
    const uint64_t cap = D->max_tuples;
    uint32_t cnt = 0;
    for (uint32_t wi = 0; wi < nw; wi++) {
        uint64_t bits = w[wi];
        while (bits) {
            const uint32_t j = (uint32_t)__ffsll((long long)bits) - 1u + wi * 64u;
            bits &= bits - 1;
            const uint64_t v = (uint64_t)((top0 ^ j) & dmask);              // top delta bits of B(row)
            const uint64_t nx = x | (v << newpos);
            if ((nx >> key_bits) != 0) continue;                           // bits beyond the key width
            if (EMIT) {
                if (slot + cnt < cap) {
                    out_x[slot + cnt] = nx;
                    out_h0[slot + cnt] = he0;
                }
            }
            cnt++;
        }
    }
    return cnt;
}

// Level 0: every (he_0, he_1) from HSE(0) x HSE(1), extended over row 2.
__global__ __launch_bounds__(256) void k_expand0(LevelArgs a)
{
    extern __shared__ unsigned long long pre[];      // [n_links + 1], sized at launch
    level_prefix_lds(a, pre);
    const uint64_t total = pre[a.n_links];
    for (uint64_t base = (uint64_t)blockIdx.x * 256u; base < total; base += (uint64_t)gridDim.x * 256u) {
        const uint32_t l = uniform(find_link(pre, a.n_links, base));
        const LinkDesc* D = a.links + l;
        const uint64_t n0 = D->ctl->hot_n[0], n1 = D->ctl->hot_n[1];
        const uint64_t Q = n0 * n1;
        const uint64_t idx = base - pre[l] + threadIdx.x;
        const uint32_t qmask = (1u << D->q) - 1u;
        uint32_t ok = idx < Q;
        uint32_t he0 = 0;
        uint64_t x = 0;
        if (ok) {
            uint64_t ia, ib;
            if (Q <= 0xFFFFFFFFull) { ia = (uint32_t)idx / (uint32_t)n1; ib = (uint32_t)idx - (uint32_t)ia * (uint32_t)n1; }
            else { ia = idx / n1; ib = idx % n1; }
            he0 = D->hot_list[ia];
            const uint32_t he1 = D->hot_list[(1ull << D->q) + ib];
            x = (uint64_t)((he0 ^ he1) & qmask);                 // B(1): host bits 0..q-1
            if ((x >> D->key_bits) != 0) ok = 0;
        }
        uint64_t* ox = D->ctb_x[0];
        uint32_t* oh = D->ctb_h0[0];
        const uint32_t cnt = extend_one<false>(D, he0, x, 2, ox, oh, 0, ok);
        const unsigned long long slot = block_append_256(cnt, &D->ctl->level_n[0]);
        extend_one<true>(D, he0, x, 2, ox, oh, slot, ok);
    }
}

// Level L >= 1: extend the tuples of level L-1 over row L+2.
__global__ __launch_bounds__(256) void k_extend(LevelArgs a)
{
    extern __shared__ unsigned long long pre[];      // [n_links + 1], sized at launch
    level_prefix_lds(a, pre);
    const uint32_t level = a.level, row = level + 2;
    const uint64_t total = pre[a.n_links];
    for (uint64_t base = (uint64_t)blockIdx.x * 256u; base < total; base += (uint64_t)gridDim.x * 256u) {
        const uint32_t l = uniform(find_link(pre, a.n_links, base));
        const LinkDesc* D = a.links + l;
        const unsigned long long raw = D->ctl->level_n[level - 1];
        const uint64_t nin = raw < D->max_tuples ? raw : D->max_tuples;
        const uint64_t idx = base - pre[l] + threadIdx.x;
        const uint32_t valid = idx < nin;
        const uint64_t* ix = D->ctb_x[(level - 1) & 1];
        const uint32_t* ih = D->ctb_h0[(level - 1) & 1];
        const uint32_t he0 = valid ? ih[idx] : 0u;
        const uint64_t x = valid ? ix[idx] : 0ull;
        uint64_t* ox = D->ctb_x[level & 1];
        uint32_t* oh = D->ctb_h0[level & 1];
        const uint32_t cnt = extend_one<false>(D, he0, x, row, ox, oh, 0, valid);
        const unsigned long long slot = block_append_256(cnt, &D->ctl->level_n[level]);
        extend_one<true>(D, he0, x, row, ox, oh, slot, valid);
    }
}

// ---------------------------------------------------------------- depth-first expansion
// The same candidate tuples as the level-by-level kernels above, in one
// launch: each thread takes one (HSE(0), HSE(1)) pair and extends it row by
// row depth first; rows are template levels, so the loop state of every row
// lives in registers.  A count pass reserves the workgroup's slots in the
// full-tuple buffer, a second pass writes them.  Every level's tuple count
// still goes to level_n (capacity checks and diagnostics).

template <int RMAX>
struct DfsCtx {
    uint32_t lv[RMAX];            // tuples accepted per level, this thread
    uint32_t full;                // full tuples, this thread
    uint64_t slot;                // write pass: first slot of this thread
    uint64_t* out_x;
    uint32_t* out_h0;
};

// rows ROW..r-1 still to choose (r <= RMAX, a compile-time bound that keeps
// every row's loop state in registers)
template <int ROW, int RMAX, bool EMIT>
__device__ __forceinline__ void dfs_row(const LinkDesc* D, uint32_t he0, uint64_t x, DfsCtx<RMAX>& c)
{
    if (ROW == RMAX || (uint32_t)ROW >= D->r) {             // rows 0..r-1 all chosen: a full tuple
        if (EMIT) {
            const uint64_t i = c.slot + c.full;
            if (i < D->max_tuples) {
                c.out_x[i] = x;
                c.out_h0[i] = he0;
            }
        }
        c.full++;
        return;
    }
    if constexpr (ROW < RMAX) {
        const uint32_t q = D->q, delta = D->delta, nw = D->nw, key_bits = D->key_bits;
        const uint32_t qmask = (1u << q) - 1u;
        const uint32_t sh = q - delta;
        const uint32_t bprev = (uint32_t)(x >> ((ROW - 2) * delta)) & qmask;     // B(ROW-1)
        const uint32_t key = ((bprev >> delta) ^ he0) & ((1u << sh) - 1u);
        const uint64_t* w = D->hotT + ((uint64_t)ROW * (1ull << sh) + key) * nw;
        const uint32_t newpos = (ROW - 2) * delta + q;                           // first host bit B(ROW) adds
        const uint32_t top0 = he0 >> sh;
        for (uint32_t wi = 0; wi < nw; wi++) {
            uint64_t bits = w[wi];
            while (bits) {
                const uint32_t j = (uint32_t)__ffsll((long long)bits) - 1u + wi * 64u;
                bits &= bits - 1;
                const uint64_t nx = x | ((uint64_t)((top0 ^ j) & ((1u << delta) - 1u)) << newpos);
                if ((nx >> key_bits) != 0) continue;                              // bits beyond the key width
                c.lv[ROW - 2]++;
                dfs_row<ROW + 1, RMAX, EMIT>(D, he0, nx, c);
            }
        }
    }
}

// Level-0 pair idx of link D: (he0, B(1)); false if idx is padding or B(1)
// has bits beyond the key width.
__device__ __forceinline__ bool level0_pair(const LinkDesc* D, uint64_t idx, uint32_t* he0, uint64_t* x)
{
    const uint64_t n0 = D->ctl->hot_n[0], n1 = D->ctl->hot_n[1];
    const uint64_t Q = n0 * n1;
    if (idx >= Q) return false;
    uint64_t ia, ib;
    if (Q <= 0xFFFFFFFFull) { ia = (uint32_t)idx / (uint32_t)n1; ib = (uint32_t)idx - (uint32_t)ia * (uint32_t)n1; }
    else { ia = idx / n1; ib = idx % n1; }
    *he0 = D->hot_list[ia];
    const uint32_t he1 = D->hot_list[(1ull << D->q) + ib];
    *x = (uint64_t)((*he0 ^ he1) & ((1u << D->q) - 1u));                 // B(1): host bits 0..q-1
    return (*x >> D->key_bits) == 0;
}

// Grid-stride over every link's level-0 pairs.  Pass 1 counts (per level and
// full tuples) in registers; the workgroup then reserves its slots for each
// link once, with one atomic per link and level; pass 2 repeats the walk and
// writes.  A workgroup's 256-item chunks never span two links (padding), and
// a workgroup handles chunks of one link at a time, so per-link totals are
// flushed whenever the link changes.
template <int RMAX>
__global__ __launch_bounds__(256) void k_expand_dfs(LevelArgs a)
{
    extern __shared__ unsigned long long pre[];      // [n_links + 1], sized at launch
    __shared__ uint32_t wsum[4][RMAX];
    __shared__ unsigned long long base_slot;
    level_prefix_lds(a, pre);
    const uint64_t total = pre[a.n_links];
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    uint64_t chunk = blockIdx.x;
    const uint64_t n_chunks = total / 256u;
    while (chunk < n_chunks) {
        // the run of this workgroup's chunks that belong to one link
        const uint32_t l = uniform(find_link(pre, a.n_links, chunk * 256u));
        const LinkDesc* D = a.links + l;
        const uint64_t link_end = pre[l + 1] / 256u;
        const uint32_t lf = D->r - 3;
        DfsCtx<RMAX> c{};
        c.out_x = D->ctb_x[lf & 1];
        c.out_h0 = D->ctb_h0[lf & 1];
        uint64_t ch = chunk;
        for (; ch < link_end; ch += gridDim.x) {
            uint32_t he0;
            uint64_t x;
            if (level0_pair(D, ch * 256u - pre[l] + threadIdx.x, &he0, &x)) dfs_row<2, RMAX, false>(D, he0, x, c);
        }
        // workgroup totals per level; the last level is the full tuples
#pragma unroll
        for (uint32_t L = 0; L < (uint32_t)RMAX; L++) {
            const uint32_t v = wave_sum(L + 3 <= D->r ? (L + 3 == D->r ? c.full : c.lv[L]) : 0u);
            if (lane == 0) wsum[wid][L] = v;
        }
        __syncthreads();
        if (threadIdx.x < (uint32_t)RMAX && threadIdx.x + 3 <= D->r) {
            const uint32_t L = threadIdx.x;
            const unsigned long long v = (unsigned long long)wsum[0][L] + wsum[1][L] + wsum[2][L] + wsum[3][L];
            if (L + 3 == D->r) base_slot = v ? atomicAdd(&D->ctl->level_n[L], v) : 0ull;
            else if (v) atomicAdd(&D->ctl->level_n[L], v);
        }
        // this thread's first slot: the workgroup's base plus the full
        // tuples of the lanes and waves before it
        uint32_t incl = c.full;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(incl, o, 64);
            if (lane >= (uint32_t)o) incl += v;
        }
        __syncthreads();
        uint64_t before = 0;
        for (uint32_t w = 0; w < wid; w++) before += wsum[w][lf];
        if (c.full) {
            DfsCtx<RMAX> e{};
            e.out_x = c.out_x;
            e.out_h0 = c.out_h0;
            e.slot = base_slot + before + (incl - c.full);
            for (uint64_t cw = chunk; cw < link_end; cw += gridDim.x) {
                uint32_t he0;
                uint64_t x;
                if (level0_pair(D, cw * 256u - pre[l] + threadIdx.x, &he0, &x)) dfs_row<2, RMAX, true>(D, he0, x, e);
            }
        }
        __syncthreads();
        chunk = ch;
    }
}

// ---------------------------------------------------------------- verify
// Final test of every full tuple (end of Alg. 4, Sec. 4.2 last pass): optional
// re-hash check, then the UnionSE of Alg. 1 -- a cell counts only when it is
// live in all r estimators -- and R >= T.  One wave per tuple.

__global__ __launch_bounds__(256) void k_verify(LevelArgs a)
{
    extern __shared__ unsigned long long pre[];      // [n_links + 1], sized at launch
    level_prefix_lds(a, pre);
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves = (uint64_t)gridDim.x * 4u;
    const uint64_t total = pre[a.n_links];
    for (uint64_t t = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6); t < total; t += waves) {
        const uint32_t l = uniform(find_link(pre, a.n_links, t));
        const LinkDesc* D = a.links + l;
        const uint64_t idx = t - pre[l];
        const uint32_t lf = D->r - 3;
        const uint32_t he0 = D->ctb_h0[lf & 1][idx];
        const uint64_t x = D->ctb_x[lf & 1][idx];
        const uint32_t q = D->q, qmask = (1u << q) - 1u;
        if (D->rehash && (tab_hash(D->tables, (uint32_t)x) & qmask) != he0) continue;
        // UnionSE (Alg. 1): a cell counts when it is live in all r estimators,
        // from the live-cell snapshots hot detection took of these (hot) estimators
        const uint32_t words = D->eta >> 6;                  // 64 cells per word
        const uint64_t* snap = reinterpret_cast<const uint64_t*>(D->live16);
        uint32_t cnt = 0;
        for (uint32_t w = lane; w < words; w += 64u) {
            uint64_t m = ~0ull;
            for (uint32_t i = 0; i < D->r; i++) {
                const uint32_t col = i == 0 ? he0 : (((uint32_t)(x >> ((i - 1) * D->delta)) & qmask) ^ he0);
                m &= snap[((((uint64_t)i << q) | col) * words) + w];
            }
            cnt += __popcll(m);
        }
        const uint32_t R = wave_sum(cnt);
        if (lane == 0 && R >= D->T) {
            const unsigned long long i = atomicAdd(&D->ctl->n_acc, 1ull);
            if (i < D->max_results) D->acc[i] = (x << 32) | (uint64_t)(0xFFFFFFFFu - R);
        }
    }
}

// ---------------------------------------------------------------- sort + report
// Accepted keys are (ip << 32) | (2^32-1 - R): ascending order gives ascending
// ip with the largest R first, so the first key of every ip run is kept.

__device__ __forceinline__ double estimate(uint32_t eta, uint32_t R)
{
    // Eq. 1 with z0 = eta - R, at least 1
    double z0 = (double)eta - (double)R;
    if (z0 < 1.0) z0 = 1.0;
    return -(double)eta * log(z0 / (double)eta);
}

// Links whose host mailbox is mapped (single detectors) get the control
// block written into it by the close's last kernel, instead of a copy.
__device__ __forceinline__ void ctl_to_host(const LinkDesc* D, unsigned long long n_out)
{
    if (!D->host_ctl) return;
    __syncthreads();
    const uint32_t* src = reinterpret_cast<const uint32_t*>(D->ctl);
    uint32_t* dst = reinterpret_cast<uint32_t*>(D->host_ctl);
    constexpr uint32_t words = sizeof(Ctl) / 4;
    constexpr uint32_t nout_word = offsetof(Ctl, n_out) / 4;
    if (threadIdx.x < words) {
        uint32_t v = src[threadIdx.x];
        if (threadIdx.x == nout_word) v = (uint32_t)n_out;
        if (threadIdx.x == nout_word + 1) v = (uint32_t)(n_out >> 32);
        dst[threadIdx.x] = v;
    }
}

// One block per link: up to SORT_SMALL keys sorted in LDS (bitonic),
// de-duplicated by ip and written as the result list.  Lists above the link's
// limit are left to the multi-kernel sort.
__global__ __launch_bounds__(1024) void k_sort_small(const LinkDesc* links)
{
    __shared__ unsigned long long s[SORT_SMALL];
    __shared__ uint32_t lds[16];
    const LinkDesc* D = links + blockIdx.x;
    if (threadIdx.x == 0) D->clock->t += 1ull;       // the close's last kernel per link: the next slot opens
    const uint64_t nraw = D->ctl->n_acc;
    if (nraw > D->sort_limit || nraw > D->max_results) {
        ctl_to_host(D, D->ctl->n_out);               // the host finishes this list
        return;
    }
    const uint32_t n = (uint32_t)(nraw < SORT_SMALL ? nraw : SORT_SMALL);
    const unsigned long long* keys = D->acc;
    uint32_t N = 1;
    while (N < n) N <<= 1;
    for (uint32_t i = threadIdx.x; i < N; i += 1024u) s[i] = i < n ? keys[i] : ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= N; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < N; i += 1024u) {
                const uint32_t p = i ^ j;
                if (p > i) {
                    const unsigned long long u = s[i], v = s[p];
                    const bool up = (i & k) == 0;
                    if ((u > v) == up) { s[i] = v; s[p] = u; }
                }
            }
            __syncthreads();
        }
    }
    const uint32_t per = (N + 1023u) / 1024u;
    const uint32_t i0 = min(n, threadIdx.x * per), i1 = min(n, i0 + per);
    uint32_t cnt = 0;
    for (uint32_t i = i0; i < i1; i++) cnt += (i == 0 || (s[i] >> 32) != (s[i - 1] >> 32));
    uint32_t total;
    uint32_t off = block_exclusive_scan_1024(cnt, lds, &total);
    for (uint32_t i = i0; i < i1; i++) {
        if (i == 0 || (s[i] >> 32) != (s[i - 1] >> 32)) {
            const uint32_t R = 0xFFFFFFFFu - (uint32_t)s[i];
            SuperPointDev sp;
            sp.ip = (uint32_t)(s[i] >> 32); sp.rk = R; sp.est = estimate(D->eta, R);
            if (off < D->host_cap) D->host_out[off] = sp;     // straight into the host's pinned mailbox
            D->out[off++] = sp;
        }
    }
    if (threadIdx.x == 0) D->ctl->n_out = total;
    ctl_to_host(D, total);
}

// Global bitonic step over N (power of two) keys, for lists above SORT_SMALL.
__global__ __launch_bounds__(256) void k_bitonic_step(unsigned long long* keys, uint64_t N, uint64_t j, uint64_t k)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < N; i += stride) {
        const uint64_t p = i ^ j;
        if (p > i) {
            const unsigned long long u = keys[i], v = keys[p];
            const bool up = (i & k) == 0;
            if ((u > v) == up) { keys[i] = v; keys[p] = u; }
        }
    }
}

// Pad keys[n..N) with the largest key.
__global__ void k_pad_keys(unsigned long long* dst, const unsigned long long* src, uint64_t n, uint64_t N)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
        dst[i] = i < n ? src[i] : ~0ull;
}

// Single block: de-duplicate n sorted keys into the link's result list.
__global__ __launch_bounds__(1024) void k_dedup_sorted(const LinkDesc* D, const unsigned long long* sorted, uint64_t n)
{
    __shared__ uint32_t lds[16];
    uint64_t out_base = 0;
    const uint32_t CHUNK = 8192u;
    for (uint64_t c0 = 0; c0 < n; c0 += CHUNK) {
        const uint64_t c1 = c0 + CHUNK < n ? c0 + CHUNK : n;
        const uint64_t i0 = c0 + (uint64_t)threadIdx.x * 8u;
        const uint64_t i1 = i0 + 8u < c1 ? i0 + 8u : c1;
        uint32_t cnt = 0;
        for (uint64_t i = i0; i < i1; i++) cnt += (i == 0 || (sorted[i] >> 32) != (sorted[i - 1] >> 32));
        uint32_t total;
        uint32_t off = block_exclusive_scan_1024(cnt, lds, &total);
        uint64_t o = out_base + off;
        for (uint64_t i = i0; i < i1; i++) {
            if (i == 0 || (sorted[i] >> 32) != (sorted[i - 1] >> 32)) {
                const uint32_t R = 0xFFFFFFFFu - (uint32_t)sorted[i];
                SuperPointDev sp;
                sp.ip = (uint32_t)(sorted[i] >> 32); sp.rk = R; sp.est = estimate(D->eta, R);
                D->out[o++] = sp;
            }
        }
        out_base += total;
    }
    if (threadIdx.x == 0) D->ctl->n_out = out_base;
}

// One block per link: copy the link's list behind those of the links before it
// into one packed array (up to cap entries in total) and record the offsets.
__global__ __launch_bounds__(256) void k_pack(PackArgs a)
{
    const uint32_t l = blockIdx.x;
    unsigned long long off = 0;
    for (uint32_t j = 0; j < l; j++) off += a.links[j].ctl->n_out;
    const LinkDesc* D = a.links + l;
    const unsigned long long n = D->ctl->n_out;
    if (threadIdx.x == 0) {
        a.offsets[l] = off;
        if (l == a.n_links - 1) a.offsets[a.n_links] = off + n;
    }
    for (unsigned long long i = threadIdx.x; i < n; i += 256u)
        if (off + i < a.cap) a.packed[off + i] = D->out[i];
}

// ---------------------------------------------------------------- merge
// Alg. 5 with the per-cell most recent hit over the routers: for every cell the
// stamp with the smallest distance wins; cells not live anywhere become empty.

__global__ __launch_bounds__(256) void k_merge(MergeArgs a)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < a.n16; i += stride) {
        uint32_t best[16];
        uint32_t code[16];
#pragma unroll
        for (int b = 0; b < 16; b++) { best[b] = 255u; code[b] = 0u; }
        for (uint32_t j = 0; j < a.n_src; j++) {
            const uint4 v = reinterpret_cast<const uint4*>(a.src[j])[i];
            if ((v.x | v.y | v.z | v.w) == 0u) continue;
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int b = 0; b < 16; b++) {
                const uint32_t c = (w[b >> 2] >> ((b & 3) * 8)) & 255u;
                if (c) {
                    int age = (int)a.cur - (int)c;
                    if (age < 0) age += 255;
                    if ((uint32_t)age < best[b]) { best[b] = (uint32_t)age; code[b] = c; }
                }
            }
        }
        uint32_t o[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int b = 0; b < 16; b++)
            if (best[b] < a.k) o[b >> 2] |= code[b] << ((b & 3) * 8);
        reinterpret_cast<uint4*>(a.dst)[i] = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

// The same for 16-bit cells: eight per chunk, distances modulo 65535.
__global__ __launch_bounds__(256) void k_merge16(MergeArgs a)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < a.n16; i += stride) {
        uint32_t best[8];
        uint32_t code[8];
#pragma unroll
        for (int b = 0; b < 8; b++) { best[b] = 65535u; code[b] = 0u; }
        for (uint32_t j = 0; j < a.n_src; j++) {
            const uint4 v = reinterpret_cast<const uint4*>(a.src[j])[i];
            if ((v.x | v.y | v.z | v.w) == 0u) continue;
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int b = 0; b < 8; b++) {
                const uint32_t c = (w[b >> 1] >> ((b & 1) * 16)) & 0xFFFFu;
                if (c) {
                    int age = (int)a.cur - (int)c;
                    if (age < 0) age += 65535;
                    if ((uint32_t)age < best[b]) { best[b] = (uint32_t)age; code[b] = c; }
                }
            }
        }
        uint32_t o[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int b = 0; b < 8; b++)
            if (best[b] < a.k) o[b >> 1] |= code[b] << ((b & 1) * 16);
        reinterpret_cast<uint4*>(a.dst)[i] = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

// ---------------------------------------------------------------- canonical

// Distance of every cell (t - slot of its latest hit) where it is below k,
// else 0xFFFF; stamps modulo M = 255 (8-bit cells) or 65535 (16-bit).
template <class T, int M>
__global__ __launch_bounds__(256) void k_canonical(const uint8_t* state, uint16_t* out, uint64_t n, uint32_t cur, uint32_t k)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    const T* cells = reinterpret_cast<const T*>(state);
    for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < n; i += stride) {
        const uint32_t c = cells[i];
        uint32_t v = 0xFFFFu;
        if (c) {
            int age = (int)cur - (int)c;
            if (age < 0) age += M;
            if ((uint32_t)age < k) v = (uint32_t)age;
        }
        out[i] = (uint16_t)v;
    }
}

// ---------------------------------------------------------------- launchers

static dim3 grid_for(uint64_t n, uint32_t block, uint32_t max_blocks)
{
    uint64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > max_blocks) g = max_blocks;
    return dim3((uint32_t)g);
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s)
{
    k_fill_u32<<<grid_for(n, 256, 8192), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_prepare(const LinkDesc* links, uint32_t n_links, bool clear_hot, hipStream_t s)
{
    k_prepare<<<dim3(n_links, clear_hot ? 16 : 1), 256, 0, s>>>(const_cast<LinkDesc*>(links), clear_hot ? 1u : 0u);
    return hipGetLastError();
}

hipError_t launch_advance(const LinkDesc* links, uint32_t n_links, hipStream_t s)
{
    k_advance<<<grid_for(n_links, 256, 64), 256, 0, s>>>(links, n_links);
    return hipGetLastError();
}

hipError_t launch_gather_ctl(const LinkDesc* links, uint32_t n_links, Ctl* dst, hipStream_t s)
{
    k_gather_ctl<<<grid_for(n_links, 256, 64), 256, 0, s>>>(links, n_links, dst);
    return hipGetLastError();
}



hipError_t launch_scan(const ScanArgs& a, hipStream_t s)
{
    if (a.cell16) k_scan<uint16_t><<<grid_for(a.n, 256, 256 * 16), 256, 0, s>>>(a);
    else k_scan<uint8_t><<<grid_for(a.n, 256, 256 * 16), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_scan_tiles(const TileScanArgs& a, uint32_t blocks, hipStream_t s)
{
    k_scan_tiles<<<blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

// the dynamic LDS of the binning kernels, set once per kernel
static hipError_t bin_lds_attr()
{
    static bool attr = false;
    if (attr) return hipSuccess;
    for (const void* f : {reinterpret_cast<const void*>(&k_bin<0, 0>), reinterpret_cast<const void*>(&k_bin<6, 6>),
                          reinterpret_cast<const void*>(&k_bin<5, 7>),
                          reinterpret_cast<const void*>(&k_bin_multi_rows)}) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(BIN_LDS_WORDS * 4u));
        if (e != hipSuccess) return e;
    }
    attr = true;
    return hipSuccess;
}

uint32_t bin_variant(const BinArgs& a)
{
    if (a.r == 6 && a.pb <= 6u * 1024u) return 6;
    if (a.r == 5 && a.pb <= 7u * 1024u) return 5;
    return 0;
}

uint32_t bin_workgroups(const BinArgs& a) { return 8u * ((a.blocks + 7u) / 8u); }   // segments dealt to XCDs in eighths

hipError_t launch_bin(const BinArgs& a, hipStream_t s)
{
    const uint32_t words = bin_lds_words(a.n_bins, a.pb, a.r);
    if (a.blocks == 0 || words > BIN_LDS_WORDS) return hipErrorInvalidValue;
    hipError_t e = bin_lds_attr();
    if (e != hipSuccess) return e;
    const uint32_t grid = bin_workgroups(a);
    switch (bin_variant(a)) {
    case 6: k_bin<6, 6><<<grid, 1024, words * 4u, s>>>(a); break;
    case 5: k_bin<5, 7><<<grid, 1024, words * 4u, s>>>(a); break;
    default: k_bin<0, 0><<<grid, 1024, words * 4u, s>>>(a); break;
    }
    return hipGetLastError();
}

hipError_t launch_bin_multi(const MultiBinArgs& m, uint32_t total_wg, hipStream_t s)
{
    if (m.n == 0 || total_wg == 0) return hipErrorInvalidValue;
    hipError_t e = bin_lds_attr();
    if (e != hipSuccess) return e;
    k_bin_multi_rows<<<total_wg, 1024, BIN_LDS_WORDS * 4u, s>>>(m);    // every link's plan fits the LDS
    return hipGetLastError();
}

uint32_t apply_workgroups(const ApplyArgs& a) { return (uint32_t)(8ull * a.parts * ((a.n_bins + 7u) / 8u)); }
uint32_t apply_counted_workgroups(const ApplyArgs& a) { return 8u * ((a.n_bins + 7u) / 8u); }

hipError_t launch_apply_multi(const MultiApplyArgs& m, uint32_t total_wg, hipStream_t s)
{
    if (m.n == 0 || total_wg == 0) return hipErrorInvalidValue;
    k_apply_multi<true><<<total_wg, 64, 0, s>>>(m);
    return hipGetLastError();
}

hipError_t launch_apply(const ApplyArgs& a, hipStream_t s)
{
    if (a.parts == 0 || a.per_part == 0) return hipErrorInvalidValue;
    const uint32_t grid = apply_workgroups(a);
    if (a.cell16) {
        if (a.pack) k_apply<true, uint16_t><<<grid, 64, 0, s>>>(a);
        else k_apply<false, uint16_t><<<grid, 64, 0, s>>>(a);
    } else {
        if (a.pack) k_apply<true, uint8_t><<<grid, 64, 0, s>>>(a);
        else k_apply<false, uint8_t><<<grid, 64, 0, s>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_apply_marked16(const ApplyArgs& a, hipStream_t s)
{
    if (!a.cell16 || !a.pack || a.bin_shift < 10 || a.bin_shift > MARKED16_MAX_SHIFT) return hipErrorInvalidValue;
    const uint32_t lds = (1u << (a.bin_shift - 5u)) * 4u;      // the bitmap
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_apply_marked16),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)MARKED16_LDS_MAX);
        if (e != hipSuccess) return e;
        attr = true;
    }
    k_apply_marked16<<<apply_counted_workgroups(a), 64 * CAPPLY_WAVES, lds, s>>>(a);
    return hipGetLastError();
}

static hipError_t counted_lds_attr()
{
    static bool attr = false;
    if (attr) return hipSuccess;
    for (const void* f : {reinterpret_cast<const void*>(&k_apply_counted),
                          reinterpret_cast<const void*>(&k_apply_counted_multi)}) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)COUNTED_LDS_BYTES);
        if (e != hipSuccess) return e;
    }
    attr = true;
    return hipSuccess;
}

hipError_t launch_apply_counted(const ApplyArgs& a, hipStream_t s)
{
    const uint64_t bytes = counted_lds_bytes(a.bin_shift, a.log2eta, a.k);
    if (!a.counts || a.k == 0 || a.slot >= a.k || a.bin_shift < a.log2eta || a.bin_shift < 5 ||
        bytes > COUNTED_LDS_BYTES || a.n_bins == 0)
        return hipErrorInvalidValue;
    if (!a.pack || a.seg < 6u) return hipErrorInvalidValue;     // counted bins are at most 2 MiB: always packed
    if (a.cell16) return hipErrorInvalidValue;                   // counters are kept for 8-bit cells only
    hipError_t e = counted_lds_attr();
    if (e != hipSuccess) return e;
    k_apply_counted<<<apply_counted_workgroups(a), 64 * CAPPLY_WAVES, (uint32_t)bytes, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_apply_counted_multi(const MultiApplyArgs& m, uint32_t total_wg, uint32_t lds_bytes, hipStream_t s)
{
    if (m.n == 0 || total_wg == 0 || lds_bytes > COUNTED_LDS_BYTES) return hipErrorInvalidValue;
    hipError_t e = counted_lds_attr();
    if (e != hipSuccess) return e;
    k_apply_counted_multi<<<total_wg, 64 * CAPPLY_WAVES, lds_bytes, s>>>(m);
    return hipGetLastError();
}

hipError_t launch_count(const LinkDesc* link, uint64_t n_se, hipStream_t s)
{
    if (n_se == 0) return hipErrorInvalidValue;
    k_count<<<(uint32_t)((n_se + 255u) / 256u), 256, 0, s>>>(link, n_se);
    return hipGetLastError();
}

uint32_t count_workgroups(uint64_t n_se) { return (uint32_t)((n_se + 255u) / 256u); }

hipError_t launch_count_multi(const CountMultiArgs& m, uint32_t total_wg, hipStream_t s)
{
    if (m.n == 0 || total_wg == 0) return hipErrorInvalidValue;
    k_count_multi<<<total_wg, 256, 0, s>>>(m);
    return hipGetLastError();
}

hipError_t launch_recount(const LinkDesc* link, uint64_t n_se, hipStream_t s)
{
    if (n_se == 0) return hipErrorInvalidValue;
    k_recount<<<(uint32_t)((n_se + 3u) / 4u), 256, 0, s>>>(link, n_se);
    return hipGetLastError();
}

hipError_t launch_hot_detect(const DetectArgs& a, uint32_t max_chunks_per_lane, bool small, hipStream_t s)
{
    // SMALL: some link has eta < 4096 (several estimators per wave) or the
    // engine has several links (link prefix in LDS); the plain variant keeps
    // half the registers, so more waves stream the state
    const dim3 g((uint32_t)((a.total + DETECT_WAVES - 1) / DETECT_WAVES));
    const uint32_t bs = 64u * DETECT_WAVES;
    if (small) {
        if (max_chunks_per_lane >= 8) k_hot_detect<8, true><<<g, bs, 0, s>>>(a);
        else k_hot_detect<4, true><<<g, bs, 0, s>>>(a);
    } else {
        if (max_chunks_per_lane >= 8) k_hot_detect<8, false><<<g, bs, 0, s>>>(a);
        else if (max_chunks_per_lane >= 4) k_hot_detect<4, false><<<g, bs, 0, s>>>(a);
        else if (max_chunks_per_lane >= 2) k_hot_detect<2, false><<<g, bs, 0, s>>>(a);
        else k_hot_detect<1, false><<<g, bs, 0, s>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_hot_detect16(const DetectArgs& a, hipStream_t s)
{
    if (a.n_links != 1 || a.total == 0) return hipErrorInvalidValue;
    const dim3 g((uint32_t)((a.total + DETECT_WAVES - 1) / DETECT_WAVES));
    k_hot_detect16<4><<<g, 64u * DETECT_WAVES, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_hot_compact(const LinkDesc* links, const uint32_t* row_table, uint32_t rows, hipStream_t s)
{
    k_hot_compact<<<rows, 1024, 0, s>>>(links, row_table);
    return hipGetLastError();
}


// dynamic LDS of the level kernels: the work prefix over the links
static inline size_t prefix_lds(const LevelArgs& a) { return ((size_t)a.n_links + 1) * 8u; }

hipError_t launch_expand0(const LevelArgs& a, hipStream_t s)
{
    k_expand0<<<2048, 256, prefix_lds(a), s>>>(a);
    return hipGetLastError();
}

// workgroups of the depth-first expansion: each flushes its counts with one
// atomic per level, so fewer is better until the grid stops filling the chip
// (512 and 1024 measured equal, 2048 slower)
// Grids of the close's small kernels (fewer workgroups, which would leave
// more of the chip to the overlapping scan, made them slower than the scan:
// 128/256 and 256/512 workgroups measured worse than 512/2048)
constexpr uint32_t DFS_BLOCKS = 512;
constexpr uint32_t VERIFY_BLOCKS = 2048;
hipError_t launch_expand_dfs(const LevelArgs& a, uint32_t max_r, hipStream_t s)
{
    if (max_r <= 6) k_expand_dfs<6><<<DFS_BLOCKS, 256, prefix_lds(a), s>>>(a);
    else if (max_r <= 8) k_expand_dfs<8><<<DFS_BLOCKS, 256, prefix_lds(a), s>>>(a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_extend(const LevelArgs& a, hipStream_t s)
{
    k_extend<<<2048, 256, prefix_lds(a), s>>>(a);
    return hipGetLastError();
}

hipError_t launch_verify(const LevelArgs& a, hipStream_t s)
{
    k_verify<<<VERIFY_BLOCKS, 256, prefix_lds(a), s>>>(a);
    return hipGetLastError();
}

hipError_t launch_sort_small(const LinkDesc* links, uint32_t n_links, hipStream_t s)
{
    k_sort_small<<<n_links, 1024, 0, s>>>(links);
    return hipGetLastError();
}

hipError_t launch_sort_large(const LinkDesc* link, const LinkDesc& host_copy, unsigned long long* tmp, uint64_t n,
                             hipStream_t s)
{
    uint64_t N = 1;
    while (N < n) N <<= 1;
    k_pad_keys<<<grid_for(N, 256, 8192), 256, 0, s>>>(tmp, host_copy.acc, n, N);
    for (uint64_t k = 2; k <= N; k <<= 1)
        for (uint64_t j = k >> 1; j > 0; j >>= 1)
            k_bitonic_step<<<grid_for(N, 256, 8192), 256, 0, s>>>(tmp, N, j, k);
    k_dedup_sorted<<<1, 1024, 0, s>>>(link, tmp, n);
    return hipGetLastError();
}

hipError_t launch_pack(const PackArgs& a, hipStream_t s)
{
    k_pack<<<a.n_links, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t s)
{
    if (a.cell16) k_merge16<<<grid_for(a.n16, 256, 256 * 16), 256, 0, s>>>(a);
    else k_merge<<<grid_for(a.n16, 256, 256 * 16), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_canonical(const uint8_t* state, uint16_t* out, uint64_t n, uint32_t cur, uint32_t k, bool cell16,
                            hipStream_t s)
{
    if (cell16) k_canonical<uint16_t, 65535><<<grid_for(n, 256, 256 * 16), 256, 0, s>>>(state, out, n, cur, k);
    else k_canonical<uint8_t, 255><<<grid_for(n, 256, 256 * 16), 256, 0, s>>>(state, out, n, cur, k);
    return hipGetLastError();
}

}  // namespace ssd
