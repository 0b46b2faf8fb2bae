// Internal structures shared by the HIP kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssd {

constexpr uint32_t MAX_ROWS = 16;
constexpr uint32_t MAX_MERGE_SOURCES = 64;
constexpr uint32_t SORT_SMALL = 8192;   // result lists up to this size sort in one block's LDS

// Device control block: counters written by the kernels, read back per close.
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

// Liveness constants for the close of slot t (stamp(t) = 1 + t mod 255):
// a cell is live iff (cell - lo) mod 256 < K' and, when the live stamps wrap
// past 255, the cell is not empty.  c1 = (256 - lo) and c2 = (256 - K') are
// replicated into both 16-bit halves.
struct LiveCfg {
    uint32_t c1, c2, wrap;
};

struct ScanArgs {
    const uint2* pairs;
    uint64_t n;
    uint8_t* state;
    const uint32_t* tables;   // [2][4][256]
    uint32_t q, r, delta, log2eta;
    uint64_t se_lo, se_hi;    // estimator window of this pass
    uint32_t stamp;
};

struct DetectArgs {
    uint8_t* state;
    uint32_t* rk;
    uint64_t* hotbits;        // [r][2^q / 64] row bitmasks of hot estimators
    uint64_t* hotT;           // [r][2^(q-delta)][nw] key-transposed hot bits
    uint32_t q, delta, nw, T;
    uint64_t n_waves;         // estimators visited
    uint64_t se_base, se_step;
    uint32_t log2eta, chunks; // chunks = eta / 16
    uint32_t count;           // compute R_k (0: expiry only)
    uint32_t expire_period, expire_phase;
    LiveCfg L;
};

struct CompactArgs {
    const uint64_t* hotbits;
    uint32_t* hot_list;
    Ctl* ctl;
    uint32_t q;
};

struct ExpandArgs {
    const uint32_t* hot_list;
    const uint64_t* hotT;
    Ctl* ctl;
    const uint64_t* in_x;
    const uint32_t* in_h0;
    uint64_t* out_x;
    uint32_t* out_h0;
    uint64_t cap;
    uint32_t q, delta, nw, key_bits, row;
};

struct VerifyArgs {
    const uint8_t* state;
    const uint32_t* tables;
    Ctl* ctl;
    const uint64_t* in_x;
    const uint32_t* in_h0;
    unsigned long long* acc;
    uint64_t cap, max_results;
    uint32_t q, r, delta, log2eta, chunks, T, level, rehash;
    LiveCfg L;
};

struct ReportArgs {
    const unsigned long long* keys;
    SuperPointDev* out;
    Ctl* ctl;
    uint32_t eta;
    uint64_t limit;           // single-block sort only when n_acc <= limit
};

struct MergeArgs {
    const uint8_t* src[MAX_MERGE_SOURCES];
    uint32_t n_src;
    uint8_t* dst;
    uint64_t n16;             // uint4 chunks per state
    uint32_t cur, k;
};

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_scan(const ScanArgs& a, hipStream_t s);
hipError_t launch_hot_detect(const DetectArgs& a, hipStream_t s);
hipError_t launch_hot_compact(const CompactArgs& a, uint32_t rows, hipStream_t s);
hipError_t launch_expand0(const ExpandArgs& a, hipStream_t s);
hipError_t launch_extend(const ExpandArgs& a, hipStream_t s);
hipError_t launch_verify(const VerifyArgs& a, hipStream_t s);
hipError_t launch_sort_small(const ReportArgs& a, hipStream_t s);
hipError_t launch_sort_large(const ReportArgs& a, unsigned long long* tmp, uint64_t n, hipStream_t s);
hipError_t launch_merge(const MergeArgs& a, hipStream_t s);
hipError_t launch_canonical(const uint8_t* state, uint16_t* out, uint64_t n, uint32_t cur, uint32_t k, hipStream_t s);

}  // namespace ssd
