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
// (see LiveCfg); the rebasing constants are computed on the host per slot.
#include <hip/hip_runtime.h>
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

// Reserve `cnt` consecutive slots in a device-wide list for this lane; every
// lane of the wave must call it.  One atomic per wave.
__device__ __forceinline__ unsigned long long wave_append(uint32_t cnt, unsigned long long* counter)
{
    const int lane = threadIdx.x & 63;
    uint32_t incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    uint32_t total = __shfl(incl, 63, 64);
    unsigned long long base = 0;
    if (lane == 63 && total) base = atomicAdd(counter, (unsigned long long)total);
    base = __shfl(base, 63, 64);
    return base + (incl - cnt);
}

// Same for a 256-thread block (every thread must call it): one atomic per block.
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

// ---------------------------------------------------------------- fill

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------- scan
// Alg. 2 for every pair: one byte store per row.  The grid strides over the
// pairs; `se_lo..se_hi` restricts the stores to one pass window of the state
// so that a pass's random stores stay within the last-level cache.

__global__ __launch_bounds__(256) void k_scan(ScanArgs a)
{
    __shared__ uint32_t tab[2048];
    for (uint32_t i = threadIdx.x; i < 2048u; i += 256u) tab[i] = a.tables[i];
    __syncthreads();
    const uint32_t qmask = (1u << a.q) - 1u;
    const uint32_t emask = (1u << a.log2eta) - 1u;
    const uint8_t stamp = (uint8_t)a.stamp;
    const uint32_t row_lo = (uint32_t)(a.se_lo >> a.q);
    const uint32_t row_hi = (uint32_t)((a.se_hi - 1) >> a.q) + 1u;
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    for (uint64_t p = (uint64_t)blockIdx.x * 256u + threadIdx.x; p < a.n; p += stride) {
        const uint2 pr = a.pairs[p];                      // x = cip, y = oip
        const uint32_t d = tab_hash(tab + 1024, pr.y) & emask;   // H1(oip)
        const uint32_t h0 = tab_hash(tab, pr.x) & qmask;          // RHFG[0](cip)
        for (uint32_t i = row_lo; i < row_hi; i++) {
            const uint32_t col = i == 0 ? h0 : ((shr32(pr.x, (i - 1) * a.delta) ^ h0) & qmask);
            const uint64_t se = ((uint64_t)i << a.q) | col;
            if (se >= a.se_lo && se < a.se_hi) a.state[(se << a.log2eta) | d] = stamp;
        }
    }
}

// ---------------------------------------------------------------- hot detection
// One wave per sliding estimator: R_k = live cells (Sec. 3.2), plus the
// rotating expiry of estimators with index = phase (mod period).  CH uint4
// chunks per lane per group keep several 1 KiB wave loads in flight.

template <int CH>
__global__ __launch_bounds__(256) void k_hot_detect(DetectArgs a)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
    if (wave >= a.n_waves) return;
    const uint64_t s = a.se_base + wave * a.se_step;
    uint4* se = reinterpret_cast<uint4*>(a.state + (s << a.log2eta));
    const uint32_t groups = a.chunks / (CH * 64u);
    const bool expire = (s % a.expire_period) == a.expire_phase;
    uint32_t live = 0;
    for (uint32_t g = 0; g < groups; g++) {
        uint4 v[CH];
#pragma unroll
        for (int c = 0; c < CH; c++) v[c] = se[(g * CH + c) * 64u + lane];
        if (a.count) {
#pragma unroll
            for (int c = 0; c < CH; c++)
                live += __popc(live_bits(v[c].x, a.L)) + __popc(live_bits(v[c].y, a.L)) +
                        __popc(live_bits(v[c].z, a.L)) + __popc(live_bits(v[c].w, a.L));
        }
        if (expire) {
#pragma unroll
            for (int c = 0; c < CH; c++) {
                uint4 n;
                n.x = expire_word(v[c].x, a.L); n.y = expire_word(v[c].y, a.L);
                n.z = expire_word(v[c].z, a.L); n.w = expire_word(v[c].w, a.L);
                if (n.x != v[c].x || n.y != v[c].y || n.z != v[c].z || n.w != v[c].w)
                    se[(g * CH + c) * 64u + lane] = n;
            }
        }
    }
    if (a.count) {
        live = wave_sum(live);
        if (lane == 0) {
            a.rk[s] = live;
            if (live >= a.T) {
                // hot (Sec. 3.3): row bitmask and key-transposed bitmask
                const uint32_t row = (uint32_t)(s >> a.q), c = (uint32_t)s & ((1u << a.q) - 1u);
                const uint32_t sh = a.q - a.delta;
                const uint32_t key = c & ((1u << sh) - 1u), j = c >> sh;
                const uint32_t rw = a.q >= 6 ? (1u << (a.q - 6)) : 1u;    // words per row bitmask
                atomicOr(reinterpret_cast<unsigned long long*>(a.hotbits) + (uint64_t)row * rw + (c >> 6),
                         1ull << (c & 63u));
                atomicOr(reinterpret_cast<unsigned long long*>(a.hotT) +
                             ((uint64_t)row * (1ull << sh) + key) * a.nw + (j >> 6),
                         1ull << (j & 63u));
            }
        }
    }
}

// ---------------------------------------------------------------- hot lists
// One 1024-thread block per row: the ascending list of hot columns, read from
// the row bitmask that hot detection set.

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

__global__ __launch_bounds__(1024) void k_hot_compact(CompactArgs a)
{
    __shared__ uint32_t lds[16];
    const uint32_t row = blockIdx.x;
    const uint32_t words = a.q >= 6 ? (1u << (a.q - 6)) : 1u;
    const uint64_t* bits = a.hotbits + (uint64_t)row * words;
    if (row == 0 && threadIdx.x == 0) {
        for (int l = 0; l < 16; l++) a.ctl->level_n[l] = 0;
        a.ctl->n_acc = 0;
        a.ctl->n_out = 0;
    }
    const uint32_t per = (words + 1023u) / 1024u;
    const uint32_t w0 = min(words, threadIdx.x * per), w1 = min(words, w0 + per);
    uint32_t cnt = 0;
    for (uint32_t w = w0; w < w1; w++) cnt += __popcll(bits[w]);
    uint32_t total;
    uint32_t off = block_exclusive_scan_1024(cnt, lds, &total);
    uint32_t* list = a.hot_list + ((uint64_t)row << a.q);
    for (uint32_t w = w0; w < w1; w++) {
        uint64_t b = bits[w];
        while (b) {
            const uint32_t i = (uint32_t)__ffsll((long long)b) - 1u;
            b &= b - 1;
            list[off++] = w * 64u + i;
        }
    }
    if (threadIdx.x == 0) a.ctl->hot_n[row] = total;
}

// ---------------------------------------------------------------- expansion
// Sec. 4.2, with the cross products of Alg. 6/7 replaced by a lookup: for a
// tuple with he_0 and he_{i-1}, the overlap test fixes the low q-delta bits of
// he_i, so the candidates are exactly the hot columns of row i under that key
// (one transposed bitmask word per 64 candidates).  A tuple is stored as
// (he_0, x) with x the host bits regained so far; he_i = (x >> (i-1)delta) mod
// 2^q XOR he_0.  Tuples are appended with one atomic per wave; their order is
// not deterministic, the set is.

struct Cand {
    const uint64_t* words;   // candidate bitmask words of the key
    uint32_t nw;
};

// count (pass 0) or emit (pass 1) the extensions of (he0, x) into row `row`
template <bool EMIT>
__device__ __forceinline__ uint32_t extend_one(const ExpandArgs& a, uint32_t he0, uint64_t x, uint32_t row,
                                               uint64_t slot, uint32_t valid)
{
    if (!valid) return 0;
    const uint32_t qmask = (1u << a.q) - 1u;
    const uint32_t sh = a.q - a.delta;
    const uint32_t kmask = (1u << sh) - 1u;
    const uint32_t bprev = (uint32_t)(x >> ((row - 2) * a.delta)) & qmask;       // B(row-1)
    const uint32_t key = ((bprev >> a.delta) ^ he0) & kmask;
    const uint64_t* w = a.hotT + ((uint64_t)row * (1ull << sh) + key) * a.nw;
    const uint32_t newpos = (row - 2) * a.delta + a.q;       // first host bit B(row) adds
    const uint32_t dmask = (1u << a.delta) - 1u;
    const uint32_t top0 = he0 >> sh;
    uint32_t cnt = 0;
    for (uint32_t wi = 0; wi < a.nw; wi++) {
        uint64_t bits = w[wi];
        while (bits) {
            const uint32_t j = (uint32_t)__ffsll((long long)bits) - 1u + wi * 64u;
            bits &= bits - 1;
            const uint64_t v = (uint64_t)((top0 ^ j) & dmask);              // top delta bits of B(row)
            const uint64_t nx = x | (v << newpos);
            if (a.key_bits < 64 && (nx >> a.key_bits) != 0) continue;      // bits beyond the key width
            if (EMIT) {
                if (slot + cnt < a.cap) {
                    a.out_x[slot + cnt] = nx;
                    a.out_h0[slot + cnt] = he0;
                }
            }
            cnt++;
        }
    }
    return cnt;
}

// Level 0: every (he_0, he_1) from HSE(0) x HSE(1), extended over row 2.
__global__ __launch_bounds__(256) void k_expand0(ExpandArgs a)
{
    const uint64_t n0 = a.ctl->hot_n[0], n1 = a.ctl->hot_n[1];
    const uint64_t Q = n0 * n1;
    const uint32_t qmask = (1u << a.q) - 1u;
    const uint32_t* l0 = a.hot_list;
    const uint32_t* l1 = a.hot_list + (1ull << a.q);
    const bool small = Q <= 0xFFFFFFFFull;
    for (uint64_t base = (uint64_t)blockIdx.x * 256u; base < Q; base += (uint64_t)gridDim.x * 256u) {
        const uint64_t idx = base + threadIdx.x;
        const uint32_t valid = idx < Q;
        uint32_t he0 = 0;
        uint64_t x = 0;
        if (valid) {
            uint64_t ia, ib;
            if (small) { ia = (uint32_t)idx / (uint32_t)n1; ib = (uint32_t)idx - (uint32_t)ia * (uint32_t)n1; }
            else { ia = idx / n1; ib = idx % n1; }
            he0 = l0[ia];
            const uint32_t he1 = l1[ib];
            x = (uint64_t)((he0 ^ he1) & qmask);                // B(1): host bits 0..q-1
            if (a.key_bits < 64 && (x >> a.key_bits) != 0) x = ~0ull;
        }
        const uint32_t ok = valid && x != ~0ull;
        const uint32_t cnt = extend_one<false>(a, he0, x, 2, 0, ok);
        const unsigned long long slot = block_append_256(cnt, &a.ctl->level_n[0]);
        extend_one<true>(a, he0, x, 2, slot, ok);
    }
}

// Level L >= 1: extend the tuples of level L-1 over row L+2.
__global__ __launch_bounds__(256) void k_extend(ExpandArgs a)
{
    const uint32_t level = a.row - 2;
    const uint64_t nin_raw = a.ctl->level_n[level - 1];
    const uint64_t nin = nin_raw < a.cap ? nin_raw : a.cap;
    for (uint64_t base = (uint64_t)blockIdx.x * 256u; base < nin; base += (uint64_t)gridDim.x * 256u) {
        const uint64_t idx = base + threadIdx.x;
        const uint32_t valid = idx < nin;
        const uint32_t he0 = valid ? a.in_h0[idx] : 0u;
        const uint64_t x = valid ? a.in_x[idx] : 0ull;
        const uint32_t cnt = extend_one<false>(a, he0, x, a.row, 0, valid);
        const unsigned long long slot = block_append_256(cnt, &a.ctl->level_n[level]);
        extend_one<true>(a, he0, x, a.row, slot, valid);
    }
}

// ---------------------------------------------------------------- verify
// Final test of every full tuple (end of Alg. 4, Sec. 4.2 last pass): optional
// re-hash check, then the UnionSE of Alg. 1 -- a cell counts only when it is
// live in all r estimators -- and R >= T.  One wave per tuple.

__global__ __launch_bounds__(256) void k_verify(VerifyArgs a)
{
    const uint64_t nraw = a.ctl->level_n[a.level];
    const uint64_t n = nraw < a.cap ? nraw : a.cap;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves = (uint64_t)gridDim.x * 4u;
    const uint32_t qmask = (1u << a.q) - 1u;
    for (uint64_t t = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6); t < n; t += waves) {
        const uint32_t he0 = a.in_h0[t];
        const uint64_t x = a.in_x[t];
        if (a.rehash && (tab_hash(a.tables, (uint32_t)x) & qmask) != he0) continue;
        const uint4* se[16];
        for (uint32_t i = 0; i < a.r; i++) {
            const uint32_t col = i == 0 ? he0 : (((uint32_t)(x >> ((i - 1) * a.delta)) & qmask) ^ he0);
            se[i] = reinterpret_cast<const uint4*>(a.state + ((((uint64_t)i << a.q) | col) << a.log2eta));
        }
        uint32_t cnt = 0;
        for (uint32_t c = lane; c < a.chunks; c += 64u) {
            uint32_t m0 = ~0u, m1 = ~0u, m2 = ~0u, m3 = ~0u;
            for (uint32_t i = 0; i < a.r; i++) {
                const uint4 v = se[i][c];
                m0 &= live_bits(v.x, a.L); m1 &= live_bits(v.y, a.L);
                m2 &= live_bits(v.z, a.L); m3 &= live_bits(v.w, a.L);
            }
            cnt += __popc(m0) + __popc(m1) + __popc(m2) + __popc(m3);
        }
        const uint32_t R = wave_sum(cnt);
        if (lane == 0 && R >= a.T) {
            const unsigned long long idx = atomicAdd(&a.ctl->n_acc, 1ull);
            if (idx < a.max_results) a.acc[idx] = (x << 32) | (uint64_t)(0xFFFFFFFFu - R);
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

// Single block: up to SORT_SMALL keys sorted in LDS (bitonic), de-duplicated
// by ip and written as the result list.
__global__ __launch_bounds__(1024) void k_sort_small(ReportArgs a)
{
    __shared__ unsigned long long s[SORT_SMALL];
    __shared__ uint32_t lds[16];
    const uint64_t nraw = a.ctl->n_acc;
    if (nraw > a.limit) return;               // longer lists take the multi-kernel sort
    const uint32_t n = (uint32_t)(nraw < SORT_SMALL ? nraw : SORT_SMALL);
    uint32_t N = 1;
    while (N < n) N <<= 1;
    for (uint32_t i = threadIdx.x; i < N; i += 1024u) s[i] = i < n ? a.keys[i] : ~0ull;
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
    // keep the first key of every ip run
    const uint32_t per = (N + 1023u) / 1024u;
    const uint32_t i0 = min(n, threadIdx.x * per), i1 = min(n, i0 + per);
    uint32_t cnt = 0;
    for (uint32_t i = i0; i < i1; i++) cnt += (i == 0 || (s[i] >> 32) != (s[i - 1] >> 32));
    uint32_t total;
    uint32_t off = block_exclusive_scan_1024(cnt, lds, &total);
    for (uint32_t i = i0; i < i1; i++) {
        if (i == 0 || (s[i] >> 32) != (s[i - 1] >> 32)) {
            const uint32_t ip = (uint32_t)(s[i] >> 32);
            const uint32_t R = 0xFFFFFFFFu - (uint32_t)s[i];
            SuperPointDev sp;
            sp.ip = ip; sp.rk = R; sp.est = estimate(a.eta, R);
            a.out[off++] = sp;
        }
    }
    if (threadIdx.x == 0) a.ctl->n_out = total;
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

// Single block: de-duplicate n sorted keys into the result list, in chunks.
__global__ __launch_bounds__(1024) void k_dedup_sorted(ReportArgs a, const unsigned long long* sorted, uint64_t n)
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
                sp.ip = (uint32_t)(sorted[i] >> 32); sp.rk = R; sp.est = estimate(a.eta, R);
                a.out[o++] = sp;
            }
        }
        out_base += total;
    }
    if (threadIdx.x == 0) a.ctl->n_out = out_base;
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

// ---------------------------------------------------------------- canonical

__global__ __launch_bounds__(256) void k_canonical(const uint8_t* state, uint16_t* out, uint64_t n, uint32_t cur, uint32_t k)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < n; i += stride) {
        const uint32_t c = state[i];
        uint32_t v = 0xFFFFu;
        if (c) {
            int age = (int)cur - (int)c;
            if (age < 0) age += 255;
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

hipError_t launch_scan(const ScanArgs& a, hipStream_t s)
{
    k_scan<<<grid_for(a.n, 256, 256 * 16), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_hot_detect(const DetectArgs& a, hipStream_t s)
{
    const dim3 g((uint32_t)((a.n_waves + 3) / 4));
    const uint32_t per_lane = a.chunks / 64u;   // uint4 chunks per lane per estimator
    if (per_lane >= 8) k_hot_detect<8><<<g, 256, 0, s>>>(a);
    else if (per_lane >= 4) k_hot_detect<4><<<g, 256, 0, s>>>(a);
    else if (per_lane >= 2) k_hot_detect<2><<<g, 256, 0, s>>>(a);
    else k_hot_detect<1><<<g, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_hot_compact(const CompactArgs& a, uint32_t rows, hipStream_t s)
{
    k_hot_compact<<<rows, 1024, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_expand0(const ExpandArgs& a, hipStream_t s)
{
    k_expand0<<<2048, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_extend(const ExpandArgs& a, hipStream_t s)
{
    k_extend<<<2048, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_verify(const VerifyArgs& a, hipStream_t s)
{
    k_verify<<<2048, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_sort_small(const ReportArgs& a, hipStream_t s)
{
    k_sort_small<<<1, 1024, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_sort_large(const ReportArgs& a, unsigned long long* tmp, uint64_t n, hipStream_t s)
{
    uint64_t N = 1;
    while (N < n) N <<= 1;
    k_pad_keys<<<grid_for(N, 256, 8192), 256, 0, s>>>(tmp, a.keys, n, N);
    for (uint64_t k = 2; k <= N; k <<= 1)
        for (uint64_t j = k >> 1; j > 0; j >>= 1)
            k_bitonic_step<<<grid_for(N, 256, 8192), 256, 0, s>>>(tmp, N, j, k);
    k_dedup_sorted<<<1, 1024, 0, s>>>(a, tmp, n);
    return hipGetLastError();
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t s)
{
    k_merge<<<grid_for(a.n16, 256, 256 * 16), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_canonical(const uint8_t* state, uint16_t* out, uint64_t n, uint32_t cur, uint32_t k, hipStream_t s)
{
    k_canonical<<<grid_for(n, 256, 256 * 16), 256, 0, s>>>(state, out, n, cur, k);
    return hipGetLastError();
}

}  // namespace ssd
