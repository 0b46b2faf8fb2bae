// Internal structures shared by the HIP kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssd {

constexpr uint32_t MAX_ROWS = 16;
constexpr uint32_t MAX_MERGE_SOURCES = 64;
constexpr uint32_t SORT_SMALL = 8192;   // result lists up to this size sort in one block's LDS
constexpr uint32_t MAX_LINKS = 1024;    // detectors in one batch
constexpr uint32_t LEVEL_VERIFY = 0xFFFFu;

// Device control block of one detector: counters written by the kernels.
struct Ctl {
    uint32_t hot_n[MAX_ROWS];
    unsigned long long level_n[MAX_ROWS];
    unsigned long long n_acc;
    unsigned long long n_out;
};

struct SuperPointDev {
    uint32_t ip;
    uint32_t rk;
    double est;
};

// Liveness constants for the close of slot t.  8-bit cells (stamp(t) = 1 +
// t mod 255): a cell is live iff (cell - lo) mod 256 < K' and, when the live
// stamps wrap past 255, the cell is not empty; c1 = (256 - lo) and c2 = (256
// - K') are replicated into both 16-bit halves.  16-bit cells (stamp(t) = 1 +
// t mod 65535): live iff (cell - lo) mod 65536 < K' and, when the live stamps
// wrap past 65535, not empty; c1 = lo and c2 = K'.
struct LiveCfg {
    uint32_t c1, c2, wrap;
};

// One detector ("link") as every close kernel sees it.  Device resident; the
// per-slice fields are written by k_prepare from the device clock at the start
// of every close, so a captured close replays with fixed arguments.
struct Clock {
    unsigned long long t;         // open slice
};

struct LinkDesc {
    uint8_t* state;
    Clock* clock;                 // this link's slot clock (device)
    const uint32_t* tables;       // [2][4][256]
    uint32_t* rk;                 // [r][2^q]
    uint64_t* hotbits;            // [r][max(1, 2^q / 64)] row bitmasks of hot estimators
    uint64_t* hotT;               // [r][2^(q-delta)][nw] key-transposed hot bits
    Ctl* host_ctl;                // mapped pinned mailbox of a single detector (else null):
    SuperPointDev* host_out;      //   the control block and the first host_cap results
    uint64_t host_cap;            //   are written there by the close's last kernel
    uint32_t* hot_list;           // [r][2^q]
    uint16_t* live16;             // [r][2^q][eta / 16] live-cell bits of hot estimators (written at hot detection)
    uint32_t* counts;             // [k + 1][r][2^q] live cells per slot t mod k and estimator, then the
                                  // live-cell total (counted detectors, else null)
    uint64_t* ctb_x[2];           // candidate buffers: regained bits
    uint32_t* ctb_h0[2];          //                    and he_0
    unsigned long long* acc;      // accepted keys
    SuperPointDev* out;           // result list
    unsigned long long* sort_tmp; // scratch of the multi-kernel sort (may be shared)
    Ctl* ctl;
    uint64_t n_se, max_tuples, max_results, sort_limit;
    uint64_t hot_words;           // u32 words of hotbits + hotT (cleared before every close)
    uint32_t q, r, delta, eta, log2eta, k, T, nw, key_bits, rehash;
    uint32_t cell16, pad;         // 1: 16-bit cells (stamp 1 + t mod 65535), else 8-bit
    // per slice
    LiveCfg L;
    uint32_t expire_period, expire_phase;
};

// direct scan of one detector, one pass window
struct ScanArgs {
    const uint2* pairs;
    uint64_t n;
    uint8_t* state;
    const uint32_t* tables;
    uint32_t q, r, delta, log2eta;
    uint64_t se_lo, se_hi;        // estimator window of this pass
    uint32_t stamp;
    uint32_t cell16;              // 1: 16-bit cells
};

// persistent batched scan: one estimator window of one link and that link's
// pairs, cut into tiles of `tile` pairs; windows are ordered by state address
struct ScanWindow {
    uint32_t link, pad;
    uint64_t start, n;            // the link's pairs [start, start + n) of the batch buffer
    uint64_t se_lo, se_hi;        // estimator window of the link
    uint64_t tile_base;           // tiles before this window
    uint32_t stamp, pad2;         // the link's stamp for its open slice
};

struct TileScanArgs {
    const uint2* pairs;
    const LinkDesc* links;
    const ScanWindow* wins;
    unsigned long long* counter;  // next tile; zero before the launch
    uint32_t n_wins;
    uint64_t n_tiles, tile;
};

// binned scan, step 1: `pb` pairs per workgroup, their cell offsets sorted
// by state bin into the workgroup's own segment of `pb * r` items
struct BinArgs {
    const uint2* pairs;
    uint64_t n;                   // pairs of this chunk
    const uint32_t* tables;
    uint32_t* items;              // [blocks][pb * r] bin-local cell offsets
    uint32_t* table;              // [n_bins + 1][blocks] start of bin b in segment j; row n_bins = item count
    uint32_t q, r, delta, log2eta;
    uint32_t bin_shift, n_bins, pb, blocks;
    uint32_t pack, pad;           // 1: three 21-bit offsets per 8-byte word (bins of at most 2 MiB)
};

// binned scan, step 2: the stores of every bin
struct ApplyArgs {
    const uint32_t* items;
    const uint32_t* table;
    uint8_t* state;
    uint32_t n_bins, blocks, seg, bin_shift;
    uint32_t parts, per_part;     // workgroups per bin, segments per workgroup
    uint32_t stamp, pack;         // pack: as BinArgs::pack
    // counted apply only: the link's per-slot counters, its window, the open
    // slice's slot (t mod k) and the estimator size
    uint32_t* counts;
    uint32_t k, slot, log2eta;
    uint32_t cell16;              // 1: 16-bit cells (k_apply; bins and offsets count cells)
    uint64_t n_se;                // estimators of the link (the counters' slot stride)
};

// binned scans of several links in one launch: workgroup g works for the
// link l with wg_prefix[l] <= g < wg_prefix[l + 1] (ranges are multiples of 8)
struct MultiBinArgs {
    const BinArgs* args;          // [n]
    const uint32_t* wg_prefix;    // [n + 1]
    uint32_t n;
};
struct MultiApplyArgs {
    const ApplyArgs* args;        // [n]
    const uint32_t* wg_prefix;    // [n + 1]
    uint32_t n;
};

// counted hot detection of several links of an engine in one launch
struct CountMultiArgs {
    const LinkDesc* links;        // the engine's descriptors
    const uint32_t* ids;          // [n] links counted by this launch
    const uint32_t* wg_prefix;    // [n + 1] workgroups before each of them (256 estimators each)
    uint32_t n;
};

// 8-byte words of one packed binning segment of n items (three 21-bit
// offsets per word), rounded up to an even count so that every segment
// starts 16-byte aligned
__host__ __device__ inline uint64_t packed_seg_words(uint64_t n_items) { return ((n_items + 2) / 3 + 1) & ~1ull; }

// LDS of the counted apply: a bit per cell of the bin, then a 16-bit counter
// per estimator of the bin and slot, two to a word (each biased by 0x8000:
// a counter moves by at most eta <= 2^14 in one call, so a half never carries
// into the other)
inline uint64_t counted_lds_bytes(uint32_t bin_shift, uint32_t log2eta, uint32_t k)
{
    return (1ull << (bin_shift - 3)) + ((1ull << (bin_shift - log2eta)) * k + 1u) / 2u * 4ull;
}
constexpr uint32_t COUNTED_LDS_BYTES = 151u * 1024u;   // 160 KiB less the kernel's static list of marked words
// at most this much dynamic LDS lets two counted workgroups (the most their
// 16 waves allow) share a compute unit
constexpr uint32_t COUNTED_LDS_PAIR = 71u * 1024u;
constexpr uint32_t COUNTED_MAX_LOG2ETA = 14;          // counters in 16-bit halves: eta <= 2^14

struct DetectArgs {
    const LinkDesc* links;
    const uint64_t* se_prefix;    // [n_links + 1] waves before each link (a wave covers >= 4 KiB of state)
    uint32_t n_links;
    uint64_t total;               // waves launched
    uint32_t expire_only;         // link 0 only: visit the estimators of this slot's expiry phase
};

struct LevelArgs {
    const LinkDesc* links;
    uint32_t n_links;
    uint32_t level;               // 0 = rows 0..2, L = row L+2, LEVEL_VERIFY = final test
};

struct MergeArgs {
    const uint8_t* src[MAX_MERGE_SOURCES];
    uint32_t n_src;
    uint8_t* dst;
    uint64_t n16;                 // uint4 chunks per state
    uint32_t cur, k;
    uint32_t cell16;              // 1: 16-bit cells
};

struct PackArgs {
    const LinkDesc* links;
    uint32_t n_links;
    SuperPointDev* packed;        // all links' lists, link after link
    uint64_t cap;
    unsigned long long* offsets;  // [n_links + 1]
};

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_prepare(const LinkDesc* links, uint32_t n_links, bool clear_hot, hipStream_t s);
hipError_t launch_advance(const LinkDesc* links, uint32_t n_links, hipStream_t s);
hipError_t launch_gather_ctl(const LinkDesc* links, uint32_t n_links, Ctl* dst, hipStream_t s);
hipError_t launch_scan(const ScanArgs& a, hipStream_t s);
hipError_t launch_scan_tiles(const TileScanArgs& a, uint32_t blocks, hipStream_t s);
// LDS words k_bin needs, and the launches of the two binned scan steps
inline uint32_t bin_lds_words(uint32_t n_bins, uint32_t pb, uint32_t r) { return 2048u + n_bins + 1u + pb * r; }
// dynamic LDS of k_bin: 160 KiB per workgroup less its static words (128 and
// 144 KiB, which leave room for the overlapped close's workgroups, measured
// the same)
constexpr uint32_t BIN_LDS_WORDS = 40960u - 32u;
hipError_t launch_bin(const BinArgs& a, hipStream_t s);
hipError_t launch_apply(const ApplyArgs& a, hipStream_t s);
hipError_t launch_apply_counted(const ApplyArgs& a, hipStream_t s);
// Workgroups of one link in the multi-link launches (multiples of 8): its
// binning, its uncounted stores and its counted stores.  The variant of the
// binning kernel (0 general, else the register binning of that many rows).
uint32_t bin_workgroups(const BinArgs& a);
uint32_t apply_workgroups(const ApplyArgs& a);
uint32_t apply_counted_workgroups(const ApplyArgs& a);
uint32_t bin_variant(const BinArgs& a);
// one launch over several links: bin (all of one variant), apply (uncounted,
// packed offsets, 8-bit cells), counted apply (lds_bytes: the largest need)
hipError_t launch_bin_multi(const MultiBinArgs& m, uint32_t total_wg, hipStream_t s);
hipError_t launch_apply_multi(const MultiApplyArgs& m, uint32_t total_wg, hipStream_t s);
hipError_t launch_apply_counted_multi(const MultiApplyArgs& m, uint32_t total_wg, uint32_t lds_bytes, hipStream_t s);
// bitmap stores of 16-bit cells (no counters): bins of 2^10 .. 2^MARKED16_MAX_SHIFT
// cells, packed offsets; the bitmap (a bit per cell) is the workgroup's LDS
constexpr uint32_t MARKED16_MAX_SHIFT = 20;
constexpr uint32_t MARKED16_LDS_MAX = (1u << (MARKED16_MAX_SHIFT - 5)) * 4u;
hipError_t launch_apply_marked16(const ApplyArgs& a, hipStream_t s);
hipError_t launch_count(const LinkDesc* link, uint64_t n_se, hipStream_t s);
hipError_t launch_recount(const LinkDesc* link, uint64_t n_se, hipStream_t s);
uint32_t count_workgroups(uint64_t n_se);
hipError_t launch_count_multi(const CountMultiArgs& m, uint32_t total_wg, hipStream_t s);
hipError_t launch_hot_detect(const DetectArgs& a, uint32_t max_chunks_per_lane, bool small, hipStream_t s);
// hot detection (or, with expire_only, the rotating expiry) of one link of 16-bit cells
hipError_t launch_hot_detect16(const DetectArgs& a, hipStream_t s);
hipError_t launch_hot_compact(const LinkDesc* links, const uint32_t* row_table, uint32_t rows, hipStream_t s);
hipError_t launch_expand0(const LevelArgs& a, hipStream_t s);
hipError_t launch_expand_dfs(const LevelArgs& a, uint32_t max_r, hipStream_t s);
hipError_t launch_extend(const LevelArgs& a, hipStream_t s);
hipError_t launch_verify(const LevelArgs& a, hipStream_t s);
hipError_t launch_sort_small(const LinkDesc* links, uint32_t n_links, hipStream_t s);
hipError_t launch_sort_large(const LinkDesc* link, const LinkDesc& host_copy, unsigned long long* tmp, uint64_t n,
                             hipStream_t s);
hipError_t launch_pack(const PackArgs& a, hipStream_t s);
hipError_t launch_merge(const MergeArgs& a, hipStream_t s);
hipError_t launch_canonical(const uint8_t* state, uint16_t* out, uint64_t n, uint32_t cur, uint32_t k, bool cell16,
                            hipStream_t s);

// host-side copies of the per-slice rules (also used by the merge and the canonical reader)
inline uint32_t stamp_of(uint64_t t, bool cell16) { return 1u + (uint32_t)(t % (cell16 ? 65535u : 255u)); }

}  // namespace ssd
