// C ABI of the sliding super point detector: parameter validation, device
// layout, slot clock and launch sequencing.  Every step of the hot path runs
// in the kernels of kernels.hip; this file only validates, sequences and
// copies.
//
// An Engine is a set of detectors ("links") that share a slot clock, a stream
// and one caller-owned state and scratch buffer, and are closed together by
// one fixed launch sequence.  A single detector (ssd_detector) is an engine
// of one link closed eagerly; a batch (ssd_batch) is an engine of n links
// scanned by one persistent launch and closed by a replayed HIP graph.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "ssd.h"

using namespace ssd;

// Staging of ssd_scan_slice_noalloc: a static device array that every device
// the library runs on holds until the process ends.  Host code never uses
// its name as an address: the per-device address comes from
// hipGetSymbolAddress, taken once per device at ssd_init_detector.
static __device__ __align__(256) uint8_t scratch[SSD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
uint8_t* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Look up (once per device, with that device current) the address of this
// device's copy of the static array.
hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (err != hipSuccess) return err;
    g_noalloc_ptr[device] = static_cast<uint8_t*>(ptr);
    return hipSuccess;
}

uint8_t* noalloc_scratch(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    return g_noalloc_ptr[device];
}

}  // namespace

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

constexpr uint64_t ALIGN = 256;
uint64_t align_up(uint64_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }
bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }
uint32_t log2u(uint64_t x)
{
    uint32_t l = 0;
    while ((1ull << l) < x) l++;
    return l;
}

// 16-bit cells (windows above 254 slots) or 8-bit
bool cell16(const ssd_params& p) { return p.cell_bits == 16; }
uint64_t state_cells(const ssd_params& p) { return ((uint64_t)p.r << p.q) * p.eta; }
uint64_t state_bytes_of(const ssd_params& p) { return state_cells(p) << (cell16(p) ? 1 : 0); }

constexpr uint32_t PREFIX_MAX = SORT_SMALL;       // result entries staged in pinned memory per close
// Scan pass window: random byte stores confined to 128 MiB of state stay in
// the 256 MB Infinity Cache (measured best of 64..768 MiB on the core-link
// workload; one pass when the state is smaller).
constexpr uint64_t DEFAULT_PASS_BYTES = 128ull << 20;
constexpr uint64_t DEFAULT_TILE_PAIRS = 4096;
constexpr uint64_t MAX_WINDOWS = 65536;           // batched scan windows per call
constexpr uint64_t BATCH_STAGE = 16384;           // result entries staged by the batch graph
constexpr uint32_t N_PHASES = SSD_PHASES;

int validate(const ssd_params* p)
{
    if (!p) return fail(SSD_E_PARAM, "params is NULL");
    if (p->abi_version != SSD_ABI_VERSION) return fail(SSD_E_PARAM, "abi_version %u != %u", p->abi_version, SSD_ABI_VERSION);
    if (p->r < 3 || p->r > MAX_ROWS) return fail(SSD_E_PARAM, "r=%u outside 3..%u", p->r, MAX_ROWS);
    if (p->q < 4 || p->q > 20) return fail(SSD_E_PARAM, "q=%u outside 4..20", p->q);
    if (p->delta < 1 || p->delta >= p->q || p->delta > 12) return fail(SSD_E_PARAM, "delta=%u must satisfy 1 <= delta < q, delta <= 12", p->delta);
    if (!is_pow2(p->eta) || p->eta < 1024 || p->eta > 65536) return fail(SSD_E_PARAM, "eta=%u must be a power of two in 1024..65536", p->eta);
    if (p->cell_bits != 0 && p->cell_bits != 8 && p->cell_bits != 16)
        return fail(SSD_E_PARAM, "cell_bits=%u must be 8 or 16 (0 = 8)", p->cell_bits);
    const uint32_t kmax = p->cell_bits == 16 ? 65534u : 254u;
    if (p->k < 1 || p->k > kmax)
        return fail(SSD_E_PARAM, "k=%u outside 1..%u for %u-bit cells", p->k, kmax, p->cell_bits == 16 ? 16u : 8u);
    if (p->theta < 1) return fail(SSD_E_PARAM, "theta must be >= 1");
    if (p->key_bits < 8 || p->key_bits > 32) return fail(SSD_E_PARAM, "key_bits=%u outside 8..32", p->key_bits);
    const uint32_t cover = (p->r - 2) * p->delta + p->q;
    if (cover < p->key_bits) return fail(SSD_E_PARAM, "(r-2)*delta+q=%u does not cover key_bits=%u", cover, p->key_bits);
    if (cover > 64) return fail(SSD_E_PARAM, "(r-2)*delta+q=%u exceeds 64", cover);
    if (p->flags & ~SSD_VERIFY_REHASH) return fail(SSD_E_PARAM, "unknown flags 0x%x", p->flags);
    if (p->max_tuples < 1 || p->max_tuples > (1ull << 32)) return fail(SSD_E_PARAM, "max_tuples outside 1..2^32");
    if (p->max_results < 1 || p->max_results > (1ull << 28)) return fail(SSD_E_PARAM, "max_results outside 1..2^28");
    return SSD_OK;
}

uint32_t hot_threshold(uint32_t eta, uint32_t theta)
{
    // Sec. 3.3: R_k >= eta * (1 - e^(-theta/eta)), rounded up once
    return (uint32_t)ceil((double)eta * (1.0 - exp(-(double)theta / (double)eta)));
}

// Binned scan geometry for a bin size request: bins of 2^shift bytes (at
// least eta and 256 KiB, at most MAX_BINS of them), `pb` pairs per k_bin
// workgroup (as many as its LDS holds).
constexpr uint32_t MAX_BINS = 4096;
constexpr uint64_t MIN_BIN_BYTES = 256ull << 10;
constexpr uint64_t DEFAULT_BIN_BYTES = 2ull << 20;
// counted scans: 512 KiB bins let two workgroups share a compute unit (0.40 ms
// per 6M-pair call into the 1.5 GiB core-link state against 0.55 ms at 1 MiB)
constexpr uint64_t DEFAULT_COUNTED_BIN_BYTES = 512ull << 10;
// A counted scan costs a workgroup per bin whatever the call's size: calls
// with fewer offsets per bin on average store uncounted (and leave the
// counters stale); many small calls per slice then close with the
// full-state hot detection instead (the served streams' 64K-4M-pair calls:
// counting at 256 slowed their per-stream closes eightfold).
constexpr uint64_t DEFAULT_COUNTED_MIN_ITEMS = 2048;
// Batches scan every link once per slice, so that a link's counted stores
// cost their workgroups per bin once, against a read of its whole state at
// the close when uncounted: a lower bar (on the 64-link batch, 256 and 0 both
// count every link, 2048 leaves 4 large states of slow links to be read)
constexpr uint64_t BATCH_COUNTED_MIN_ITEMS = 256;
// Pairs binned per step, at most.  The stores of a bin are spread over the
// workgroups of one XCD, so the work in flight is about (bins in flight) x
// (items per bin): larger steps put more items in every bin (8M and 16M
// measured equal, 4M slower on 6M-pair calls).
constexpr uint64_t BIN_CHUNK_PAIRS = 8ull << 20;
// k_bin segments one k_apply workgroup walks: with 2 MiB bins and about 6000
// pairs per segment this puts about 500 workgroups on every bin of a 6M-pair
// step, so the workgroups resident on an XCD cover one or two bins (measured
// best of 1..64 on the core-link workload, 6M pairs per slice into 1.5 GiB)
constexpr uint32_t DEFAULT_APPLY_SEGMENTS = 2;
// binned scan for states above this size (measured: faster on the 1.5 GiB
// core-link state, slower on a 24 MiB state that the Infinity Cache holds)
constexpr uint64_t AUTO_BINNED_ABOVE = 256ull << 20;
constexpr uint32_t PHASE_SCAN_BIN = 8;
constexpr uint32_t PHASE_SCAN_TILES = 10;
// batch links scanned binned: at least this many pairs in the call (fewer
// go to the persistent tile scan, since the binned stores cost workgroups
// per bin whatever the call's size)
constexpr uint64_t BATCH_BINNED_MIN_PAIRS = 1ull << 16;
// group members scanned binned (in the multi-member launches): at least this
// many pairs in the call, whatever the state's size (a member whose scan mode
// is SSD_SCAN_PASSES keeps the tile scan)
constexpr uint64_t GROUP_BINNED_MIN_PAIRS = 1ull << 18;
// staging of a batch's binned scan: the binning segments of up to this many
// pairs (at 4 bytes per offset) for the links of one group of launches.  On
// the 64-link workload (152M pairs per slice) one group, 4.6 GB of staging,
// ran 5.91 ms per slice against 6.05 ms for three groups of up to 64M pairs
// (fewer launches, fewer partly filled last waves of workgroups)
constexpr uint64_t BATCH_BIN_PAIRS = 192ull << 20;
// Candidate expansion: depth first in one launch up to this many rows (its
// per-row loop state is held in registers), level by level above.
constexpr uint32_t DFS_MAX_ROWS = 8;
struct BinPlan {
    uint32_t shift = 0, n_bins = 0, pb = 0;
};
BinPlan bin_plan(const ssd_params& p, uint64_t bin_bytes)
{
    // bins and their offsets count cells (2 bytes each for 16-bit cells)
    const uint64_t state = state_cells(p);
    BinPlan b;
    b.shift = log2u(std::max<uint64_t>(std::max<uint64_t>(bin_bytes, MIN_BIN_BYTES) >> (cell16(p) ? 1 : 0), p.eta));
    while (((state + (1ull << b.shift) - 1) >> b.shift) > MAX_BINS) b.shift++;
    b.n_bins = (uint32_t)((state + (1ull << b.shift) - 1) >> b.shift);
    b.pb = (BIN_LDS_WORDS - 2048u - b.n_bins - 1u) / p.r;
    // rows 5 and 6 keep every pair's offsets in registers (k_bin_reg): at
    // most 7 and 6 pairs per thread
    if (p.r == 6) b.pb = std::min<uint32_t>(b.pb, 6u * 1024u);
    if (p.r == 5) b.pb = std::min<uint32_t>(b.pb, 7u * 1024u);
    return b;
}
// Bin size of the counted scan (k_apply_counted) for a bin size request: of
// 1 MiB, 512 KiB and 256 KiB, those whose cell bits and counters fit one
// workgroup's LDS and that give at most MAX_BINS bins; the largest of them
// not above the request whose LDS lets two workgroups share a compute unit,
// else the largest not above the request, else the smallest.  0 when none
// fits, when eta > 2^14 (16-bit LDS counters) or when the counters would
// exceed half the state (eta < 8 k: summing them at the close would read
// more than half of what reading the cells does): the link cannot count.
uint32_t counted_shift(const ssd_params& p, uint64_t want = 1ull << 20)
{
    if (8ull * p.k > p.eta || cell16(p)) return 0;      // 16-bit cells keep no counters
    const uint32_t le = log2u(p.eta);
    if (le > COUNTED_MAX_LOG2ETA) return 0;
    uint32_t pair = 0, best = 0, smallest = 0;
    for (uint32_t sh = 20; sh >= 18; sh--) {
        const uint64_t lds = counted_lds_bytes(sh, le, p.k);
        if (sh < le || lds > COUNTED_LDS_BYTES) continue;
        if (bin_plan(p, 1ull << sh).shift != sh) break;   // more bins than MAX_BINS, and more below
        smallest = sh;
        if ((1ull << sh) <= want) {
            if (!best) best = sh;
            if (!pair && lds <= COUNTED_LDS_PAIR) pair = sh;
        }
    }
    return pair ? pair : best ? best : smallest;
}
// Item and table words that every allowed bin size fits, for chunks of up to
// BIN_CHUNK_PAIRS pairs (fewer for small states).
void bin_capacity(const ssd_params& p, uint64_t* items_words, uint64_t* table_words)
{
    const uint64_t state = state_cells(p);
    const uint64_t chunk = std::min<uint64_t>(BIN_CHUNK_PAIRS, std::max<uint64_t>(1ull << 16, state >> 4));
    const BinPlan worst = bin_plan(p, 0);     // the most bins, the fewest pairs per workgroup
    const uint64_t blocks = (chunk + worst.pb - 1) / worst.pb;
    *items_words = blocks * worst.pb * p.r;
    *table_words = (uint64_t)(worst.n_bins + 1) * blocks;
}

uint32_t nw_of(const ssd_params& p) { return p.delta > 6 ? 1u << (p.delta - 6) : 1u; }

// Hot detection waves of a link: one per estimator from eta = 4096 up, one
// per 4 KiB of state below (k_hot_detect).
// (16-bit cells: one wave per estimator, k_hot_detect16).
uint64_t detect_waves(const LinkDesc& D)
{
    if (D.cell16) return D.n_se;
    return D.log2eta >= 12 ? D.n_se : D.n_se >> (12 - D.log2eta);
}
uint64_t row_words(const ssd_params& p) { return p.q >= 6 ? (1ull << (p.q - 6)) : 1ull; }

struct LinkLayout {
    uint64_t state_off, state_bytes;
    uint64_t tables, ctl, rk, hot_list, live16, hotbits, hotT, ctb_x[2], ctb_h0[2], acc, out;
    uint64_t counts;              // per-slot counters of a single detector that can count (else 0)
};

struct Layout {
    uint64_t links = 0, se_prefix = 0, row_table = 0, clock = 0, pack_offsets = 0, tiles = 0;
    uint64_t ctl = 0, hot_begin = 0, hot_end = 0, sort_tmp = 0, packed = 0, total = 0;
    uint64_t state_total = 0, pack_cap = 0, tile_cap = 0;
    uint64_t bin_items = 0, bin_table = 0, bin_items_words = 0, bin_table_words = 0;   // binned scan staging
    uint64_t multi_args = 0;      // batches: arguments of the multi-link binned launches
    uint64_t count_list = 0;      // the links counted at a close and their workgroup prefix (2n + 1 words)
    std::vector<LinkLayout> link;
};

// Arguments of a batch's multi-link binned launches for n links: per link
// one BinArgs and one ApplyArgs, and the workgroup prefixes of the launches
// (at most five per group of links -- three binning variants, counted and
// uncounted stores -- and at most n groups: 10 (n + 1) words).
uint64_t multi_args_bytes(uint32_t n)
{
    return align_up((uint64_t)n * sizeof(BinArgs)) + align_up((uint64_t)n * sizeof(ApplyArgs)) +
           align_up(10 * ((uint64_t)n + 1) * 4);
}

// Scratch layout of an engine: header (descriptors, prefix tables, clock,
// scan tiles), tables, control blocks, the hot-bit pool (cleared by one fill
// per close), then every link's own buffers; states are packed link after link.
Layout plan(const ssd_params* p, uint32_t n, uint64_t pack_cap, uint64_t tile_cap, bool bins = false)
{
    Layout L;
    L.link.resize(n);
    L.pack_cap = pack_cap;
    L.tile_cap = tile_cap;
    uint64_t rows = 0, maxres = 1;
    for (uint32_t l = 0; l < n; l++) {
        rows += p[l].r;
        maxres = std::max<uint64_t>(maxres, p[l].max_results);
    }
    uint64_t o = 0;
    L.links = o; o = align_up(o + n * sizeof(LinkDesc));
    L.se_prefix = o; o = align_up(o + (n + 1) * 8);
    L.row_table = o; o = align_up(o + rows * 4);
    L.clock = o; o = align_up(o + n * sizeof(Clock));       // one clock per link
    L.pack_offsets = o; o = align_up(o + (n + 1) * 8);
    L.tiles = o; o = align_up(o + 8 + tile_cap * sizeof(ScanWindow));
    L.count_list = o; o = align_up(o + (2ull * n + 1) * 4);
    for (uint32_t l = 0; l < n; l++) { L.link[l].tables = o; o += 2048 * 4; }
    o = align_up(o);
    L.ctl = o;
    for (uint32_t l = 0; l < n; l++) L.link[l].ctl = o + l * sizeof(Ctl);
    o = align_up(o + n * sizeof(Ctl));
    L.hot_begin = o;
    for (uint32_t l = 0; l < n; l++) {
        const ssd_params& q = p[l];
        L.link[l].hotbits = o; o += q.r * row_words(q) * 8;
        L.link[l].hotT = o; o += (uint64_t)q.r * (1ull << (q.q - q.delta)) * nw_of(q) * 8;
    }
    L.hot_end = o;
    o = align_up(o);
    for (uint32_t l = 0; l < n; l++) {
        const ssd_params& q = p[l];
        const uint64_t n_se = (uint64_t)q.r << q.q;
        LinkLayout& K = L.link[l];
        K.rk = o; o = align_up(o + n_se * 4);
        K.hot_list = o; o = align_up(o + n_se * 4);
        K.live16 = o; o = align_up(o + n_se * (q.eta / 16) * 2);
        for (int b = 0; b < 2; b++) { K.ctb_x[b] = o; o = align_up(o + q.max_tuples * 8); }
        for (int b = 0; b < 2; b++) { K.ctb_h0[b] = o; o = align_up(o + q.max_tuples * 4); }
        K.acc = o; o = align_up(o + q.max_results * 8);
        K.out = o; o = align_up(o + q.max_results * sizeof(SuperPointDev));
        // per-slot counters for the links whose scans are binned (single
        // detectors; batch links above the binned threshold) and can count
        // (k per-slice slots and the live-cell total)
        if (bins && counted_shift(q)) { K.counts = o; o = align_up(o + n_se * (q.k + 1ull) * 4); }
    }
    uint64_t pw = 1;
    while (pw < maxres) pw <<= 1;
    L.sort_tmp = o; o = align_up(o + pw * 8);
    L.packed = o; o = align_up(o + pack_cap * sizeof(SuperPointDev));
    if (bins && n == 1) {
        uint64_t iw = 0, tw = 0;
        bin_capacity(p[0], &iw, &tw);
        L.bin_items_words = iw;
        L.bin_table_words = tw;
    } else if (bins) {
        // a batch: the links binned in one group of launches share these
        // (a table word per bin and binning workgroup, whose segment holds
        // at least 8 times as many offsets); at least one link's largest
        // step, at most a quarter offset per cell of the batch's state
        uint64_t cells = 0;
        uint32_t rmax = 0;
        for (uint32_t l = 0; l < n; l++) {
            cells += state_cells(p[l]);
            rmax = std::max(rmax, p[l].r);
            uint64_t iw = 0, tw = 0;
            bin_capacity(p[l], &iw, &tw);
            L.bin_items_words = std::max(L.bin_items_words, iw);
            L.bin_table_words = std::max(L.bin_table_words, tw);
        }
        const uint64_t iw = std::min<uint64_t>(BATCH_BIN_PAIRS * rmax, cells / 4);
        L.bin_items_words = std::max(L.bin_items_words, iw);
        L.bin_table_words = std::max(L.bin_table_words, iw / 8 + MAX_BINS + 1);
        // the per-link arguments and workgroup prefixes of the multi-link launches
        L.multi_args = o;
        o = align_up(o + multi_args_bytes(n));
    }
    if (bins) {
        L.bin_items = o; o = align_up(o + L.bin_items_words * 4);
        L.bin_table = o; o = align_up(o + L.bin_table_words * 4);
    }
    L.total = o;
    uint64_t so = 0;
    for (uint32_t l = 0; l < n; l++) {
        L.link[l].state_off = so;
        L.link[l].state_bytes = state_bytes_of(p[l]);
        so += L.link[l].state_bytes;
    }
    L.state_total = so;
    return L;
}

}  // namespace

// ---------------------------------------------------------------- engine

struct Engine {
    uint32_t n = 0;
    std::vector<ssd_params> p;
    std::vector<uint32_t> T;
    Layout L;
    uint8_t* state = nullptr;
    uint8_t* scratch = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    uint64_t clock = 0;
    bool broken = false;
    uint64_t se_total = 0;
    uint32_t rows_total = 0, max_r = 0, max_chunks = 1;
    bool detect_small = false;          // a link with eta < 4096, or several links (k_hot_detect SMALL)
    // counted detection, per link: the counters are exact for the open
    // slice's scans so far (count_valid), or a binned scan of this slice ran
    // uncounted and the close rebuilds them (count_rebuild)
    std::vector<uint8_t> counting, count_valid, count_rebuild;
    std::vector<uint64_t> detect_prefix;   // the hot detection wave prefix on the device
    uint64_t counted_bin_bytes = DEFAULT_COUNTED_BIN_BYTES;   // bin size request of counted scans
    uint64_t counted_min_items = DEFAULT_COUNTED_MIN_ITEMS;   // offsets per bin a call needs to count
    std::vector<uint8_t> count_small;      // a call of this slice stored uncounted for being small
    std::vector<uint8_t> last_mode;        // hot detection of the last close: 0 state, 1 counters, 2 rebuilt
    std::vector<uint64_t> bin_req;         // per link: bin size request of its counted scans (0: counted_bin_bytes)
    std::vector<uint8_t> last_csh;         // per link: bin shift of its last counted binned call (0: none)
    uint32_t* cl_pinned = nullptr;         // staging of the counted-link list (2n + 1 words)
    hipEvent_t cl_done = nullptr;          // its last copy has run
    std::vector<LinkDesc> hl;          // host copies of the device descriptors
    std::vector<uint32_t> tables;      // n x 2048
    // pinned host mailbox: control blocks, staged result entries, pack offsets
    void* pinned = nullptr;
    Ctl* mb_ctl = nullptr;
    SuperPointDev* mb_stage = nullptr;
    unsigned long long* mb_offsets = nullptr;
    uint64_t stage_cap = 0;
    // phase timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<uint32_t> ev_free;
    struct Pending { uint32_t a, b, phase, launches; };
    std::vector<Pending> pending;
    double ph_ms[N_PHASES] = {};
    uint64_t ph_launches[N_PHASES] = {};
    bool gather_ctl = false;           // control blocks live with their links (groups)
    bool direct_mailbox = false;       // the sort kernel writes control block and list to pinned memory
    // graph replay of the close
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t capture_stream = nullptr;   // records the close graph (never runs work)
    uint64_t graph_prefix = 0;              // result entries the graph copies to pinned memory
    // results of the last close
    std::vector<std::vector<ssd_super_point>> results;
    std::vector<int> status;
    std::vector<Ctl> last;
    bool have_last = false;
    std::vector<SuperPointDev> staging;

    template <class X> X* at(uint64_t off) const { return reinterpret_cast<X*>(scratch + off); }
    LinkDesc* dev_links() const { return at<LinkDesc>(L.links); }
};

namespace {

int dev_fail(Engine* e, hipError_t err, const char* what)
{
    if (e) e->broken = true;
    return fail(SSD_E_DEVICE, "%s: %s", what, hipGetErrorString(err));
}

#define HIPCHK(e, call)                                            \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return dev_fail((e), e_, #call);     \
    } while (0)

int usable(Engine* e)
{
    if (e->broken) return fail(SSD_E_STATE, "detector unusable after an earlier device error");
    hipError_t err = hipSetDevice(e->device);
    if (err != hipSuccess) return dev_fail(e, err, "hipSetDevice");
    return SSD_OK;
}

// ---- phase timing: a start/stop event pair around each phase's launches
uint32_t ev_get(Engine* e)
{
    if (!e->ev_free.empty()) {
        uint32_t i = e->ev_free.back();
        e->ev_free.pop_back();
        return i;
    }
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return UINT32_MAX;
    e->ev_pool.push_back(ev);
    return (uint32_t)e->ev_pool.size() - 1;
}

struct PhaseMark {
    uint32_t a = UINT32_MAX;
};

PhaseMark phase_begin(Engine* e)
{
    PhaseMark m;
    if (!e->timing) return m;
    m.a = ev_get(e);
    if (m.a != UINT32_MAX && hipEventRecord(e->ev_pool[m.a], e->stream) != hipSuccess) {
        e->ev_free.push_back(m.a);
        m.a = UINT32_MAX;
    }
    return m;
}

void phase_end(Engine* e, PhaseMark m, uint32_t phase, uint32_t launches)
{
    if (!e->timing || m.a == UINT32_MAX) return;
    uint32_t b = ev_get(e);
    if (b == UINT32_MAX) { e->ev_free.push_back(m.a); return; }
    if (hipEventRecord(e->ev_pool[b], e->stream) != hipSuccess) {
        e->ev_free.push_back(m.a);
        e->ev_free.push_back(b);
        return;
    }
    e->pending.push_back({m.a, b, phase, launches});
}

// after the stream passed every pending stop event
void phase_collect(Engine* e)
{
    std::vector<Engine::Pending> later;
    for (const auto& pd : e->pending) {
        if (hipEventQuery(e->ev_pool[pd.b]) != hipSuccess) {   // work enqueued after the waited-for point
            (void)hipGetLastError();
            later.push_back(pd);
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e->ev_pool[pd.a], e->ev_pool[pd.b]) == hipSuccess) {
            e->ph_ms[pd.phase] += ms;
            e->ph_launches[pd.phase] += pd.launches;
        } else {
            (void)hipGetLastError();     // a missing sample is not an error of the next call
        }
        e->ev_free.push_back(pd.a);
        e->ev_free.push_back(pd.b);
    }
    e->pending.swap(later);
}

void graph_reset(Engine* e)
{
    if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    e->gexec = nullptr;
    e->graph = nullptr;
}

void engine_release(Engine* e)
{
    (void)hipSetDevice(e->device);
    if (!e->broken && e->scratch) (void)hipStreamSynchronize(e->stream);
    if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    if (e->capture_stream) (void)hipStreamDestroy(e->capture_stream);
    if (e->pinned) (void)hipHostFree(e->pinned);
    if (e->cl_pinned) (void)hipHostFree(e->cl_pinned);
    if (e->cl_done) (void)hipEventDestroy(e->cl_done);
    for (hipEvent_t ev : e->ev_pool) (void)hipEventDestroy(ev);
}

int engine_query(const ssd_params* p, uint32_t n, uint64_t pack_cap, uint64_t tile_cap, uint64_t* state_bytes,
                 uint64_t* scratch_bytes, bool bins = false)
{
    if (!p || n < 1 || n > MAX_LINKS) return fail(SSD_E_PARAM, "need 1..%u detectors", MAX_LINKS);
    for (uint32_t l = 0; l < n; l++) {
        int rc = validate(p + l);
        if (rc) return rc;
    }
    Layout L = plan(p, n, pack_cap, tile_cap, bins);
    if (state_bytes) *state_bytes = L.state_total;
    if (scratch_bytes) *scratch_bytes = L.total;
    return SSD_OK;
}

int engine_init(Engine* e, const ssd_params* p, uint32_t n, const uint32_t* tables, void* state_dev,
                uint64_t state_bytes, void* scratch_dev, uint64_t scratch_bytes, void* stream, uint64_t pack_cap,
                uint64_t tile_cap, uint64_t stage_cap, bool bins = false, bool single = false)
{
    int rc = engine_query(p, n, pack_cap, tile_cap, nullptr, nullptr, bins);
    if (rc) return rc;
    if (!tables) return fail(SSD_E_PARAM, "tables_host is NULL");
    e->n = n;
    e->p.assign(p, p + n);
    e->L = plan(p, n, pack_cap, tile_cap, bins);
    if (!state_dev || state_bytes < e->L.state_total || ((uintptr_t)state_dev & 15u))
        return fail(SSD_E_NOMEM, "state buffer needs %llu bytes, 16-byte aligned", (unsigned long long)e->L.state_total);
    if (!scratch_dev || scratch_bytes < e->L.total || ((uintptr_t)scratch_dev & (ALIGN - 1)))
        return fail(SSD_E_NOMEM, "scratch buffer needs %llu bytes, 256-byte aligned", (unsigned long long)e->L.total);
    e->state = static_cast<uint8_t*>(state_dev);
    e->scratch = static_cast<uint8_t*>(scratch_dev);
    e->stream = static_cast<hipStream_t>(stream);
    e->tables.assign(tables, tables + (uint64_t)n * 2048);
    e->T.resize(n);
    e->hl.resize(n);
    std::vector<uint64_t> se_prefix(n + 1, 0);
    std::vector<uint32_t> row_table;
    for (uint32_t l = 0; l < n; l++) {
        const ssd_params& q = p[l];
        const LinkLayout& K = e->L.link[l];
        LinkDesc& D = e->hl[l];
        memset(&D, 0, sizeof D);
        D.state = e->state + K.state_off;
        D.tables = e->at<uint32_t>(K.tables);
        D.rk = e->at<uint32_t>(K.rk);
        D.hotbits = e->at<uint64_t>(K.hotbits);
        D.hotT = e->at<uint64_t>(K.hotT);
        D.hot_list = e->at<uint32_t>(K.hot_list);
        D.live16 = e->at<uint16_t>(K.live16);
        D.counts = K.counts ? e->at<uint32_t>(K.counts) : nullptr;
        for (int b = 0; b < 2; b++) {
            D.ctb_x[b] = e->at<uint64_t>(K.ctb_x[b]);
            D.ctb_h0[b] = e->at<uint32_t>(K.ctb_h0[b]);
        }
        D.acc = e->at<unsigned long long>(K.acc);
        D.out = e->at<SuperPointDev>(K.out);
        D.sort_tmp = e->at<unsigned long long>(e->L.sort_tmp);
        D.ctl = e->at<Ctl>(K.ctl);
        D.clock = e->at<Clock>(e->L.clock) + l;
        D.hot_words = (K.hotT - K.hotbits + (uint64_t)q.r * (1ull << (q.q - q.delta)) * nw_of(q) * 8) / 4;
        D.n_se = (uint64_t)q.r << q.q;
        D.max_tuples = q.max_tuples;
        D.max_results = q.max_results;
        D.sort_limit = SORT_SMALL;
        D.q = q.q; D.r = q.r; D.delta = q.delta; D.eta = q.eta; D.log2eta = log2u(q.eta); D.k = q.k;
        D.cell16 = cell16(q) ? 1u : 0u;
        D.T = e->T[l] = hot_threshold(q.eta, q.theta);
        D.nw = nw_of(q);
        D.key_bits = q.key_bits;
        D.rehash = (q.flags & SSD_VERIFY_REHASH) ? 1u : 0u;
        se_prefix[l + 1] = se_prefix[l] + detect_waves(D);
        for (uint32_t i = 0; i < q.r; i++) row_table.push_back((l << 8) | i);
        e->max_r = std::max(e->max_r, q.r);
        e->max_chunks = std::max(e->max_chunks, q.eta >> 10);
        e->detect_small = e->detect_small || q.eta < 4096 || n > 1;
    }
    e->se_total = se_prefix[n];
    e->rows_total = (uint32_t)row_table.size();
    // the counters start zero with the state: exact from the first slice
    e->counting.assign(n, 0);
    e->count_valid.assign(n, 0);
    e->count_rebuild.assign(n, 0);
    e->count_small.assign(n, 0);
    e->last_mode.assign(n, 0);
    e->bin_req.assign(n, 0);
    e->last_csh.assign(n, 0);
    for (uint32_t l = 0; l < n; l++)
        if (e->hl[l].counts) e->counting[l] = e->count_valid[l] = 1;
    e->detect_prefix = se_prefix;
    hipError_t err = hipGetDevice(&e->device);
    if (err != hipSuccess) return dev_fail(e, err, "hipGetDevice");
    e->stage_cap = stage_cap;
    const uint64_t pinned_bytes = n * sizeof(Ctl) + stage_cap * sizeof(SuperPointDev) + (n + 1) * 8;
    err = hipHostMalloc(&e->pinned, pinned_bytes, hipHostMallocDefault);
    if (err != hipSuccess) return dev_fail(e, err, "hipHostMalloc");
    e->mb_ctl = static_cast<Ctl*>(e->pinned);
    e->mb_stage = reinterpret_cast<SuperPointDev*>(e->mb_ctl + n);
    e->mb_offsets = reinterpret_cast<unsigned long long*>(e->mb_stage + stage_cap);
    if (single) {
        // a single detector's close writes its control block and list into
        // the mailbox directly (no copies after the sort)
        void* dctl = nullptr;
        void* dout = nullptr;
        HIPCHK(e, hipHostGetDevicePointer(&dctl, e->mb_ctl, 0));
        HIPCHK(e, hipHostGetDevicePointer(&dout, e->mb_stage, 0));
        e->hl[0].host_ctl = static_cast<Ctl*>(dctl);
        e->hl[0].host_out = static_cast<SuperPointDev*>(dout);
        e->hl[0].host_cap = std::min<uint64_t>(stage_cap, p[0].max_results);
        e->direct_mailbox = true;
    }
    // every cell starts empty (Sec. 3.2: initialised once); scratch and clock zero
    HIPCHK(e, launch_fill_u32(reinterpret_cast<uint32_t*>(e->state), e->L.state_total / 4, 0u, e->stream));
    HIPCHK(e, launch_fill_u32(e->at<uint32_t>(0), e->L.total / 4, 0u, e->stream));
    HIPCHK(e, hipMemcpyAsync(e->dev_links(), e->hl.data(), n * sizeof(LinkDesc), hipMemcpyHostToDevice, e->stream));
    HIPCHK(e, hipMemcpyAsync(e->at<uint64_t>(e->L.se_prefix), se_prefix.data(), (n + 1) * 8, hipMemcpyHostToDevice, e->stream));
    HIPCHK(e, hipMemcpyAsync(e->at<uint32_t>(e->L.row_table), row_table.data(), row_table.size() * 4,
                             hipMemcpyHostToDevice, e->stream));
    for (uint32_t l = 0; l < n; l++)
        HIPCHK(e, hipMemcpyAsync(e->at<uint32_t>(e->L.link[l].tables), tables + (uint64_t)l * 2048, 2048 * 4,
                                 hipMemcpyHostToDevice, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    e->results.assign(n, {});
    e->status.assign(n, SSD_OK);
    e->last.assign(n, Ctl{});
    return SSD_OK;
}

// The binned scan of a call of n pairs of link l: whether it takes the
// counted stores (the link keeps per-slot counters and the call is large
// enough), whether its counters stay exact through it (they were before),
// and its bin geometry.  A link whose counters are stale still takes the
// counted stores for a large call: each touched 16-byte chunk is restamped
// once, which beats a byte store per offset when the pairs repeat, and the
// counters are rebuilt at the close (or, in a group, left untrusted).
// (16-bit cells keep no counters: a large call of theirs takes the bitmap
// stores without counters, `marked`, over bins of MARKED16_BIN_BYTES.)
constexpr uint64_t MARKED16_BIN_BYTES = 512ull << 10;
struct BinnedCall {
    bool large = false, counted = false, exact = false, marked = false;
    uint32_t csh = 0;        // counted bin shift (0: the link cannot count)
    BinPlan bp;
    uint64_t seg = 0;        // offsets per binning workgroup (pb * r)
};
BinnedCall binned_call(const Engine* e, uint32_t l, uint64_t n, uint64_t bin_bytes)
{
    BinnedCall c;
    c.csh = e->counting[l] ? counted_shift(e->p[l], e->bin_req[l] ? e->bin_req[l] : e->counted_bin_bytes) : 0;
    c.large = c.csh && n * e->p[l].r >= e->counted_min_items * bin_plan(e->p[l], 1ull << c.csh).n_bins;
    c.counted = e->counting[l] && c.large;
    c.exact = c.counted && e->count_valid[l];
    if (cell16(e->p[l])) {
        const BinPlan mp = bin_plan(e->p[l], MARKED16_BIN_BYTES);
        c.marked = mp.shift <= MARKED16_MAX_SHIFT && n * e->p[l].r >= e->counted_min_items * mp.n_bins;
    }
    c.bp = bin_plan(e->p[l], c.counted ? 1ull << c.csh : c.marked ? MARKED16_BIN_BYTES : bin_bytes);
    c.seg = (uint64_t)c.bp.pb * e->p[l].r;
    return c;
}

// Staging of the binned scan: the binning workgroups' offset segments (4 *
// seg bytes each at most) and the bin-major table (n_bins + 1 words each).
struct BinBufs {
    uint32_t* items = nullptr;
    uint32_t* table = nullptr;
    uint64_t items_words = 0, table_words = 0;
};
BinBufs engine_bins(const Engine* e)
{
    return {e->at<uint32_t>(e->L.bin_items), e->at<uint32_t>(e->L.bin_table), e->L.bin_items_words,
            e->L.bin_table_words};
}

// The counter bookkeeping of a binned call of link l: after stores that do
// not keep the counters exact, the counters are stale (rebuilt at the close
// after a large call).
void binned_count_state(Engine* e, uint32_t l, const BinnedCall& c)
{
    if (c.counted) e->last_csh[l] = (uint8_t)c.csh;
    else if (c.marked) e->last_csh[l] = (uint8_t)c.bp.shift;
    if (e->counting[l] && !c.exact) {
        e->count_valid[l] = 0;                 // the counters are not exact after these stores
        // the close rebuilds the counters from the state after large calls
        // only; with a small call in the slice it reads the state once
        if (!c.large) e->count_small[l] = 1;
        e->count_rebuild[l] = c.large && !e->count_small[l];
    }
}

// The arguments of both binned steps of link l for its plan c, staging at
// items / table, segments per store workgroup segs; pairs and sizes are set
// per step.
void binned_args(const Engine* e, uint32_t l, const BinnedCall& c, uint32_t* items, uint32_t* table, uint32_t segs,
                 BinArgs* ba_out, ApplyArgs* aa_out)
{
    const LinkDesc& D = e->hl[l];
    const BinPlan bp = c.bp;
    BinArgs ba{};
    ba.tables = D.tables;
    ba.items = items;
    ba.table = table;
    ba.q = D.q; ba.r = D.r; ba.delta = D.delta; ba.log2eta = D.log2eta;
    ba.bin_shift = bp.shift; ba.n_bins = bp.n_bins; ba.pb = bp.pb;
    ba.pack = bp.shift <= 21 ? 1u : 0u;
    ApplyArgs aa{};
    aa.pack = ba.pack;
    aa.items = ba.items;
    aa.table = ba.table;
    aa.state = D.state;
    aa.n_bins = bp.n_bins;
    aa.seg = (uint32_t)c.seg;
    aa.bin_shift = bp.shift;
    aa.per_part = segs;
    aa.stamp = stamp_of(e->clock, D.cell16);
    aa.cell16 = D.cell16;
    if (c.counted) {
        aa.counts = D.counts;
        aa.k = D.k;
        aa.slot = (uint32_t)(e->clock % D.k);
        aa.log2eta = D.log2eta;
        aa.n_se = D.n_se;
    }
    *ba_out = ba;
    *aa_out = aa;
}

// Binned scan (k_bin, then k_apply_counted or k_apply) of n pairs of link l,
// in steps that fit the staging buffers bb (the engine's own are shared by
// every binned link of a batch: the steps run one after another on the
// engine's stream).  The counted stores keep the link's per-slot counters
// exact when they were; otherwise the counters are left stale.
int enqueue_binned_scan(Engine* e, uint32_t l, const uint2* pairs, uint64_t n, uint64_t bin_bytes, uint32_t segs,
                        const BinBufs& bb)
{
    const BinnedCall c = binned_call(e, l, n, bin_bytes);
    const bool counted = c.counted;
    binned_count_state(e, l, c);
    const BinPlan bp = c.bp;
    if (counted && (!c.csh || bp.shift != c.csh)) return fail(SSD_E_STATE, "counted bin plan mismatch");
    const uint64_t seg = c.seg;
    const uint64_t max_blocks = std::min(bb.items_words / seg, bb.table_words / (bp.n_bins + 1));
    const uint64_t chunk = max_blocks * bp.pb;
    if (chunk == 0) return fail(SSD_E_STATE, "binned scan buffers too small");
    BinArgs ba{};
    ApplyArgs aa{};
    binned_args(e, l, c, bb.items, bb.table, segs, &ba, &aa);
    for (uint64_t done = 0; done < n; done += chunk) {
        const uint64_t m = std::min(chunk, n - done);
        ba.pairs = pairs + done;
        ba.n = m;
        ba.blocks = (uint32_t)((m + bp.pb - 1) / bp.pb);
        aa.blocks = ba.blocks;
        aa.parts = (ba.blocks + aa.per_part - 1) / aa.per_part;
        PhaseMark pm = phase_begin(e);
        HIPCHK(e, launch_bin(ba, e->stream));
        phase_end(e, pm, PHASE_SCAN_BIN, 1);
        pm = phase_begin(e);
        HIPCHK(e, counted    ? launch_apply_counted(aa, e->stream)
                  : c.marked ? launch_apply_marked16(aa, e->stream)
                             : launch_apply(aa, e->stream));
        phase_end(e, pm, 0, 1);
    }
    return SSD_OK;
}

// The close of every link: per-slice constants, hot bitmasks cleared, hot
// detection (this first part, eager and timed), then hot lists, the
// candidate levels, the final test, sorting, the control blocks (and, for
// batches, the packed lists) to pinned memory and the clock advance (the
// second part, recordable in a graph).  Hot detection takes R_k from the
// per-slot counters of the links where they are exact or rebuilt, and reads
// the state of the others.
int enqueue_close_head(Engine* e)
{
    const hipStream_t s = e->stream;
    LinkDesc* links = e->dev_links();
    HIPCHK(e, launch_prepare(links, e->n, true, s));
    // per link: R_k from the per-slot counters (1), from counters rebuilt
    // from the state first (2), or by reading the whole state (0)
    const uint32_t n = e->n;
    std::vector<uint8_t> mode(n, 0);
    std::vector<uint64_t> pre(n + 1, 0);
    for (uint32_t l = 0; l < n; l++) {
        if (e->counting[l] && (e->count_valid[l] || e->count_rebuild[l])) mode[l] = e->count_valid[l] ? 1 : 2;
        pre[l + 1] = pre[l] + (mode[l] ? 0 : detect_waves(e->hl[l]));      // counted links take no waves
    }
    if (pre != e->detect_prefix) {
        HIPCHK(e, hipMemcpyAsync(e->at<uint64_t>(e->L.se_prefix), pre.data(), (n + 1) * 8, hipMemcpyHostToDevice, s));
        e->detect_prefix = pre;
    }
    if (pre[n]) {
        DetectArgs da{};
        da.links = links;
        da.se_prefix = e->at<uint64_t>(e->L.se_prefix);
        da.n_links = n;
        da.total = pre[n];
        PhaseMark pm = phase_begin(e);
        // 16-bit cells only in single detectors (batches and groups take 8-bit links)
        HIPCHK(e, e->hl[0].cell16 ? launch_hot_detect16(da, s) : launch_hot_detect(da, e->max_chunks, e->detect_small, s));
        phase_end(e, pm, 1, 1);
    }
    // counted links: counters rebuilt from the state where needed, then R_k
    // from the counters (the next slot starts at zero) -- one launch for one
    // link, one launch over all of them for several
    std::vector<uint32_t> ids;
    for (uint32_t l = 0; l < n; l++)
        if (mode[l]) ids.push_back(l);
    if (!ids.empty()) {
        PhaseMark pm = phase_begin(e);
        uint32_t launches = 1;
        for (uint32_t l : ids)
            if (mode[l] == 2) {
                HIPCHK(e, launch_recount(links + l, e->hl[l].n_se, s));
                launches++;
            }
        if (ids.size() == 1) {
            HIPCHK(e, launch_count(links + ids[0], e->hl[ids[0]].n_se, s));
        } else {
            if (!e->cl_pinned) {
                HIPCHK(e, hipHostMalloc(reinterpret_cast<void**>(&e->cl_pinned), (2ull * n + 1) * 4, hipHostMallocDefault));
                HIPCHK(e, hipEventCreateWithFlags(&e->cl_done, hipEventDisableTiming));
            } else {
                HIPCHK(e, hipEventSynchronize(e->cl_done));     // the last copy out of the staging has run
            }
            const uint32_t m = (uint32_t)ids.size();
            uint32_t total = 0;
            for (uint32_t i = 0; i < m; i++) {
                e->cl_pinned[i] = ids[i];
                e->cl_pinned[m + i] = total;
                total += count_workgroups(e->hl[ids[i]].n_se);
            }
            e->cl_pinned[2 * m] = total;
            uint32_t* dev = e->at<uint32_t>(e->L.count_list);
            HIPCHK(e, hipMemcpyAsync(dev, e->cl_pinned, (2ull * m + 1) * 4, hipMemcpyHostToDevice, s));
            HIPCHK(e, hipEventRecord(e->cl_done, s));
            CountMultiArgs cm{links, dev, dev + m, m};
            HIPCHK(e, launch_count_multi(cm, total, s));
        }
        phase_end(e, pm, 9, launches);
    }
    for (uint32_t l = 0; l < n; l++) {
        e->last_mode[l] = mode[l];
        e->count_valid[l] = mode[l] != 0;
        e->count_rebuild[l] = 0;
        e->count_small[l] = 0;
    }
    return SSD_OK;
}

// The close, second part: hot lists, expansion levels, final test, sort, and
// the copies to pinned memory -- many small launches, replayed as a graph
// when the engine uses one (its phases are then timed as one).
int enqueue_close_tail(Engine* e, bool pack, uint64_t single_prefix, bool capturing)
{
    const hipStream_t s = e->stream;
    LinkDesc* links = e->dev_links();
    const bool t = e->timing && !capturing;
    auto begin = [&]() { return t ? phase_begin(e) : PhaseMark(); };
    auto end = [&](PhaseMark m, uint32_t ph, uint32_t nl) { if (t) phase_end(e, m, ph, nl); };
    PhaseMark pm = begin();
    HIPCHK(e, launch_hot_compact(links, e->at<uint32_t>(e->L.row_table), e->rows_total, s));
    end(pm, 2, 1);
    LevelArgs la{};
    la.links = links;
    la.n_links = e->n;
    la.level = 0;
    pm = begin();
    if (e->max_r <= DFS_MAX_ROWS) {
        // one depth-first launch for all levels
        HIPCHK(e, launch_expand_dfs(la, e->max_r, s));
        end(pm, 3, 1);
    } else {
        HIPCHK(e, launch_expand0(la, s));
        for (uint32_t lvl = 1; lvl + 3 <= e->max_r; lvl++) {
            la.level = lvl;
            HIPCHK(e, launch_extend(la, s));
        }
        end(pm, 3, e->max_r - 2);
    }
    la.level = LEVEL_VERIFY;
    pm = begin();
    HIPCHK(e, launch_verify(la, s));
    end(pm, 4, 1);
    pm = begin();
    HIPCHK(e, launch_sort_small(links, e->n, s));
    end(pm, 5, 1);
    if (e->direct_mailbox) return SSD_OK;   // k_sort_small wrote the mailbox and advanced the clock
    if (e->gather_ctl) HIPCHK(e, launch_gather_ctl(links, e->n, e->at<Ctl>(e->L.ctl), s));
    HIPCHK(e, hipMemcpyAsync(e->mb_ctl, e->at<Ctl>(e->L.ctl), e->n * sizeof(Ctl), hipMemcpyDeviceToHost, s));
    if (pack) {
        PackArgs pa{};
        pa.links = links;
        pa.n_links = e->n;
        pa.packed = e->at<SuperPointDev>(e->L.packed);
        pa.cap = e->L.pack_cap;
        pa.offsets = e->at<unsigned long long>(e->L.pack_offsets);
        HIPCHK(e, launch_pack(pa, s));
        HIPCHK(e, hipMemcpyAsync(e->mb_offsets, pa.offsets, (e->n + 1) * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(e, hipMemcpyAsync(e->mb_stage, pa.packed, e->stage_cap * sizeof(SuperPointDev),
                                 hipMemcpyDeviceToHost, s));
    } else if (single_prefix) {
        HIPCHK(e, hipMemcpyAsync(e->mb_stage, e->hl[0].out, single_prefix * sizeof(SuperPointDev),
                                 hipMemcpyDeviceToHost, s));
    }
    return SSD_OK;     // k_sort_small advanced every link's clock
}

int enqueue_close(Engine* e, bool pack, uint64_t single_prefix)
{
    int rc = enqueue_close_head(e);
    if (rc) return rc;
    return enqueue_close_tail(e, pack, single_prefix, false);
}

// The close with its second part as a HIP graph: captured once on a stream
// of our own (the caller's may be the legacy default stream, which cannot be
// captured) and replayed on the caller's stream after the eager first part.
// Recaptured when the result prefix it copies changes.
int close_graph_tail(Engine* e, bool pack, uint64_t prefix)
{
    int rc = SSD_OK;
    if (e->gexec && e->graph_prefix != prefix) graph_reset(e);
    if (!e->gexec) {
        if (!e->capture_stream) HIPCHK(e, hipStreamCreateWithFlags(&e->capture_stream, hipStreamNonBlocking));
        const hipStream_t caller = e->stream;
        e->stream = e->capture_stream;
        hipError_t err = hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal);
        if (err != hipSuccess) {
            e->stream = caller;
            return dev_fail(e, err, "hipStreamBeginCapture");
        }
        rc = enqueue_close_tail(e, pack, prefix, true);
        hipGraph_t g = nullptr;
        err = hipStreamEndCapture(e->stream, &g);
        e->stream = caller;
        e->graph = g;
        if (rc) { graph_reset(e); return rc; }
        if (err != hipSuccess) { graph_reset(e); return dev_fail(e, err, "hipStreamEndCapture"); }
        err = hipGraphInstantiate(&e->gexec, e->graph, nullptr, nullptr, 0);
        if (err != hipSuccess) { graph_reset(e); return dev_fail(e, err, "hipGraphInstantiate"); }
        e->graph_prefix = prefix;
    }
    PhaseMark pm = phase_begin(e);
    HIPCHK(e, hipGraphLaunch(e->gexec, e->stream));
    phase_end(e, pm, 7, 1);
    return SSD_OK;
}

int close_graph(Engine* e, bool pack, uint64_t prefix)
{
    int rc = enqueue_close_head(e);
    if (rc) return rc;
    return close_graph_tail(e, pack, prefix);
}

// After the close's synchronisation: check every link's capacities, finish
// links whose list needs the multi-kernel sort, and collect the lists.
int collect_results(Engine* e, bool packed, uint64_t single_prefix)
{
    const hipStream_t s = e->stream;
    e->have_last = true;
    for (uint32_t l = 0; l < e->n; l++) {
        const ssd_params& q = e->p[l];
        Ctl c = e->mb_ctl[l];
        e->last[l] = c;
        e->results[l].clear();
        e->status[l] = SSD_OK;
        bool over = c.n_acc > q.max_results;
        for (uint32_t lv = 0; lv + 3 <= q.r; lv++) over |= c.level_n[lv] > q.max_tuples;
        if (over) {
            e->status[l] = SSD_E_OVERFLOW;
            continue;
        }
        const SuperPointDev* src = nullptr;
        uint64_t m = c.n_out;
        if (c.n_acc > e->hl[l].sort_limit) {
            // long list: multi-kernel sort of this link, then its whole list
            PhaseMark pm = phase_begin(e);
            HIPCHK(e, launch_sort_large(e->dev_links() + l, e->hl[l], e->hl[l].sort_tmp, c.n_acc, s));
            phase_end(e, pm, 5, 1);
            e->staging.resize(c.n_acc);
            HIPCHK(e, hipMemcpyAsync(&e->mb_ctl[l], e->hl[l].ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
            HIPCHK(e, hipMemcpyAsync(e->staging.data(), e->hl[l].out, c.n_acc * sizeof(SuperPointDev),
                                     hipMemcpyDeviceToHost, s));
            HIPCHK(e, hipStreamSynchronize(s));
            phase_collect(e);
            m = e->mb_ctl[l].n_out;
            e->last[l].n_out = m;
            src = e->staging.data();
        } else if (packed && e->mb_offsets[l] + m <= e->stage_cap) {
            src = e->mb_stage + e->mb_offsets[l];
        } else if (!packed && m <= single_prefix) {
            src = e->mb_stage;
        } else {
            e->staging.resize(m);
            if (m) {
                HIPCHK(e, hipMemcpyAsync(e->staging.data(), e->hl[l].out, m * sizeof(SuperPointDev),
                                         hipMemcpyDeviceToHost, s));
                HIPCHK(e, hipStreamSynchronize(s));
            }
            src = e->staging.data();
        }
        e->results[l].resize(m);
        for (uint64_t i = 0; i < m; i++) {
            e->results[l][i].ip = src[i].ip;
            e->results[l][i].rk = src[i].rk;
            e->results[l][i].est = src[i].est;
        }
    }
    return SSD_OK;
}

// Rotating expiry only (a router that only advances): per-slice constants,
// the estimators of this slot's expiry phase, clock advance.
int enqueue_advance_only(Engine* e)
{
    const hipStream_t s = e->stream;
    e->count_valid[0] = 0;            // the next slot's counters are not zeroed
    e->count_rebuild[0] = 0;
    e->count_small[0] = 0;
    LinkDesc* links = e->dev_links();
    HIPCHK(e, launch_prepare(links, e->n, false, s));
    DetectArgs da{};
    da.links = links;
    da.se_prefix = e->at<uint64_t>(e->L.se_prefix);
    da.n_links = 1;
    da.expire_only = 1;
    const uint64_t period = (e->hl[0].cell16 ? 65535u : 255u) - e->p[0].k;
    da.total = (e->hl[0].n_se + period - 1) / period;
    HIPCHK(e, e->hl[0].cell16 ? launch_hot_detect16(da, s) : launch_hot_detect(da, e->max_chunks, e->detect_small, s));
    HIPCHK(e, launch_advance(links, e->n, s));
    return SSD_OK;
}

int read_timing(Engine* e, double* ms_out, uint64_t* launches_out, int reset)
{
    int rc = usable(e);
    if (rc) return rc;
    HIPCHK(e, hipStreamSynchronize(e->stream));
    phase_collect(e);
    for (uint32_t i = 0; i < N_PHASES; i++) {
        if (ms_out) ms_out[i] = e->ph_ms[i];
        if (launches_out) launches_out[i] = e->ph_launches[i];
        if (reset) { e->ph_ms[i] = 0; e->ph_launches[i] = 0; }
    }
    return SSD_OK;
}

// Facts about link l of an engine.
void engine_info(const Engine& e, uint32_t l, ssd_info* out)
{
    memset(out, 0, sizeof *out);
    out->open_slice = e.clock;
    out->hot_threshold = e.T[l];
    out->r = e.p[l].r;
    out->state_bytes = e.L.link.empty() ? state_bytes_of(e.p[l]) : e.L.link[l].state_bytes;
    if (e.have_last) {
        for (uint32_t i = 0; i < MAX_ROWS; i++) {
            out->level_counts[i] = e.last[l].level_n[i];
            out->hot_counts[i] = e.last[l].hot_n[i];
        }
        out->accepted = e.last[l].n_acc;
        out->reported = e.results[l].size();
        out->counted = e.last_mode[l];
    }
    if (l < e.last_csh.size() && e.last_csh[l]) out->counted_bin_kib = 1u << (e.last_csh[l] - 10);
}

// R_k of link l at the last close (host copy).
int engine_read_rk(Engine* e, uint32_t l, uint32_t* out_host, uint64_t n)
{
    int rc = usable(e);
    if (rc) return rc;
    if (!e->have_last) return fail(SSD_E_STATE, "no reconstructing close yet");
    const uint64_t n_se = e->hl[l].n_se;
    if (!out_host || n < n_se) return fail(SSD_E_NOMEM, "R_k needs %llu entries", (unsigned long long)n_se);
    HIPCHK(e, hipMemcpyAsync(out_host, e->hl[l].rk, n_se * 4, hipMemcpyDeviceToHost, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    return SSD_OK;
}

// Hot lists HSE(0..r-1) of link l at the last close: counts, then the lists
// packed row after row.
int engine_read_hot(Engine* e, uint32_t l, uint32_t* counts_host, uint32_t* lists_host, uint64_t cap)
{
    int rc = usable(e);
    if (rc) return rc;
    if (!e->have_last) return fail(SSD_E_STATE, "no reconstructing close yet");
    if (!counts_host) return fail(SSD_E_PARAM, "counts_host is NULL");
    const Ctl& c = e->last[l];
    const ssd_params& p = e->p[l];
    uint64_t total = 0;
    for (uint32_t i = 0; i < p.r; i++) { counts_host[i] = c.hot_n[i]; total += c.hot_n[i]; }
    if (total > cap || (total && !lists_host)) return fail(SSD_E_TRUNC, "hot lists need %llu entries", (unsigned long long)total);
    uint64_t o = 0;
    for (uint32_t i = 0; i < p.r; i++) {
        if (c.hot_n[i])
            HIPCHK(e, hipMemcpyAsync(lists_host + o, e->hl[l].hot_list + ((uint64_t)i << p.q),
                                     (uint64_t)c.hot_n[i] * 4, hipMemcpyDeviceToHost, e->stream));
        o += c.hot_n[i];
    }
    HIPCHK(e, hipStreamSynchronize(e->stream));
    return SSD_OK;
}

}  // namespace

// ---------------------------------------------------------------- single detector

std::atomic<uint64_t> g_next_detector_id{1};

struct ssd_detector {
    Engine e;
    uint64_t id = g_next_detector_id.fetch_add(1);   // unique for the process: host addresses get reused
    uint64_t pass_bytes = DEFAULT_PASS_BYTES;
    uint32_t scan_mode = SSD_SCAN_AUTO;
    uint64_t bin_bytes = DEFAULT_BIN_BYTES;
    uint32_t apply_segments = DEFAULT_APPLY_SEGMENTS;
    bool pending = false;               // a close begun and not yet ended
    bool group_pending = false;         // a group close of this member begun and not yet ended
    uint64_t pending_prefix = 0;
    hipStream_t close_stream = nullptr; // runs the close after hot detection
    hipEvent_t detect_done = nullptr;   // hot detection of the last close done
    hipEvent_t close_done = nullptr;    // the last close done
    const ssd_params& p() const { return e.p[0]; }
    const LinkDesc& D() const { return e.hl[0]; }
};

namespace {

// A close of the detector, its own or a group's, has begun and not ended.
bool close_pending(const ssd_detector* d) { return d->pending || d->group_pending; }

// The second stream of a single detector and its events (created on first use).
int detector_streams(ssd_detector* d)
{
    Engine* e = &d->e;
    if (!d->detect_done) HIPCHK(e, hipEventCreateWithFlags(&d->detect_done, hipEventDisableTiming));
    if (!d->close_done) HIPCHK(e, hipEventCreateWithFlags(&d->close_done, hipEventDisableTiming));
    if (!d->close_stream) HIPCHK(e, hipStreamCreateWithFlags(&d->close_stream, hipStreamNonBlocking));
    return SSD_OK;
}

// Argument and state checks shared by the scan calls.
int scan_checks(ssd_detector* d, const uint32_t* pairs_dev, uint64_t n, uint64_t slice_id)
{
    Engine* e = &d->e;
    int rc = usable(e);
    if (rc) return rc;
    if (slice_id != e->clock)
        return fail(SSD_E_ORDER, "scan of slice %llu while slice %llu is open", (unsigned long long)slice_id,
                    (unsigned long long)e->clock);
    if (n == 0) return SSD_OK;
    if (!pairs_dev || ((uintptr_t)pairs_dev & 7u)) return fail(SSD_E_PARAM, "pairs must be a non-NULL 8-byte aligned device pointer");
    return SSD_OK;
}

// The detector's scans are binned: SSD_SCAN_BINNED, or SSD_SCAN_AUTO with a
// state above AUTO_BINNED_ABOVE.
bool scans_binned(const ssd_detector* d)
{
    const LinkDesc& D = d->D();
    const uint64_t state_bytes = (D.n_se << D.log2eta) << D.cell16;
    return d->scan_mode == SSD_SCAN_BINNED || (d->scan_mode == SSD_SCAN_AUTO && state_bytes > AUTO_BINNED_ABOVE);
}

// Pass-window scan (k_scan): passes over estimator windows of about
// pass_bytes each, highest window first: the last pass leaves the lowest
// estimators cache-resident, and hot detection reads them first.
int enqueue_pass_scan(ssd_detector* d, const uint2* pairs, uint64_t n)
{
    Engine* e = &d->e;
    const LinkDesc& D = d->D();
    e->count_valid[0] = 0;            // pass scans store without counting
    ScanArgs a{};
    a.pairs = pairs;
    a.n = n;
    a.state = D.state;
    a.tables = D.tables;
    a.q = D.q; a.r = D.r; a.delta = D.delta; a.log2eta = D.log2eta;
    a.stamp = stamp_of(e->clock, D.cell16);
    a.cell16 = D.cell16;
    const uint64_t n_se = D.n_se;
    uint64_t per_pass = n_se;
    if (d->pass_bytes) per_pass = std::max<uint64_t>(1, d->pass_bytes / ((uint64_t)D.eta << D.cell16));
    const uint64_t n_pass = (n_se + per_pass - 1) / per_pass;
    PhaseMark pm = phase_begin(e);
    uint32_t launches = 0;
    for (uint64_t j = n_pass; j-- > 0;) {
        a.se_lo = j * per_pass;
        a.se_hi = std::min(a.se_lo + per_pass, n_se);
        HIPCHK(e, launch_scan(a, e->stream));
        launches++;
    }
    phase_end(e, pm, 0, launches);
    return SSD_OK;
}


}  // namespace

// ---------------------------------------------------------------- batch

struct ssd_batch {
    Engine e;
    uint32_t scan_mode = SSD_SCAN_AUTO;   // SSD_SCAN_PASSES: every link in the tile scan
    uint64_t pass_bytes = DEFAULT_PASS_BYTES;
    uint64_t tile_pairs = DEFAULT_TILE_PAIRS;
    // pinned double-buffered window lists for the persistent scan
    void* tile_pinned[2] = {nullptr, nullptr};
    hipEvent_t tile_done[2] = {nullptr, nullptr};
    bool tile_used[2] = {false, false};
    uint32_t tile_next = 0;
    uint32_t scan_blocks = 2048;
    // pinned double-buffered arguments of the multi-link binned launches
    void* mb_pinned[2] = {nullptr, nullptr};
    hipEvent_t mb_done[2] = {nullptr, nullptr};
    bool mb_used[2] = {false, false};
    uint32_t mb_next = 0;
    // autotuner: candidate (pass window, tile pairs), each scan timed with events
    struct Cand { uint64_t pass, tile; double ns_per_pair; };
    std::vector<Cand> cands;
    int tune_idx = -1;                 // next candidate to time, -1 = not tuning
    std::vector<std::pair<int, uint64_t>> tune_pending;   // (candidate, pairs) per timed scan
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tune_events;
    // autotuner, second dimension: the bin size request of the counted binned
    // stores, by class of binned links (same q and eta, pairs per call within
    // the same factor-4 band).  Every trial times the whole binned scan of a
    // tuning scan (the classes share its launches, so a class is only as fast
    // as the launches it shares): trials 0-2 give every class bin candidate
    // 0-2; then, for the TUNE_CLASSES classes with the most pairs in turn,
    // each other candidate, kept when it beats the best so far by 1%.
    struct BinTrial { uint64_t cls; int cand; };       // cls = NO_CLASS: every class
    std::vector<BinTrial> bt_trials;
    int bt_next = -1;                                  // next trial, -1 = none
    std::map<uint64_t, int> bt_choice;                 // classes whose candidate differs from bt_global
    int bt_global = 1;
    double bt_best = -1.0, bt_global_ns[3] = {-1.0, -1.0, -1.0};
    std::map<uint64_t, uint64_t> bt_class_pairs;       // pairs per class over the tuning scans
    struct BinTiming { int trial; uint64_t pairs; hipEvent_t a, b; };
    std::vector<BinTiming> bt_pending;
    // a close begun (ssd_batch_close_begin) and not yet ended
    bool pending = false;
    hipEvent_t done = nullptr;
    std::vector<uint64_t> link_class;                  // per link: its class in its last tuning scan
};

// Bin size candidates of the counted stores (a link takes the largest of
// its sizes that fit, not above the candidate, else its smallest).
constexpr uint64_t TUNE_BIN_BYTES[3] = {256ull << 10, 512ull << 10, 1ull << 20};
constexpr uint64_t NO_CLASS = ~0ull;
constexpr uint32_t TUNE_CLASSES = 4;

// Tuning class of a binned link with n pairs in the call.
static uint64_t tune_class(const ssd_params& p, uint64_t n)
{
    const uint64_t band = n ? (uint64_t)log2u(n) / 2u : 0u;
    return ((uint64_t)p.q << 16) | ((uint64_t)log2u(p.eta) << 8) | band;
}

namespace {

// After a close's synchronisation: credit the timed scans to their candidates;
// once every candidate has run, keep the fastest per pair.
void autotune_collect(ssd_batch* b)
{
    // samples of scans enqueued after the waited-for close (the next slice's,
    // with the close pipelined) stay for the next collection
    auto ran = [](hipEvent_t ev) {
        if (hipEventQuery(ev) == hipSuccess) return true;
        (void)hipGetLastError();
        return false;
    };
    std::vector<std::pair<int, uint64_t>> keep_p;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> keep_e;
    for (size_t i = 0; i < b->tune_pending.size(); i++) {
        const auto ev = b->tune_events[i];
        if (!ran(ev.second)) {
            keep_p.push_back(b->tune_pending[i]);
            keep_e.push_back(ev);
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess && b->tune_pending[i].second) {
            ssd_batch::Cand& c = b->cands[b->tune_pending[i].first];
            const double ns = ms * 1e6 / (double)b->tune_pending[i].second;
            if (c.ns_per_pair < 0 || ns < c.ns_per_pair) c.ns_per_pair = ns;
        }
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    b->tune_pending.swap(keep_p);
    b->tune_events.swap(keep_e);
    std::vector<ssd_batch::BinTiming> keep_b;
    for (const auto& c : b->bt_pending) {
        if (!ran(c.b)) {
            keep_b.push_back(c);
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c.a, c.b) == hipSuccess && c.pairs) {
            const double ns = ms * 1e6 / (double)c.pairs;
            const ssd_batch::BinTrial& tr = b->bt_trials[c.trial];
            if (tr.cls == NO_CLASS) {
                b->bt_global_ns[tr.cand] = ns;
            } else if (ns < 0.99 * b->bt_best) {
                b->bt_choice[tr.cls] = tr.cand;
                b->bt_best = ns;
            }
        }
        (void)hipEventDestroy(c.a);
        (void)hipEventDestroy(c.b);
        if (c.trial == 2) {
            // the global candidates timed: keep the fastest, then try the
            // others on the classes with the most pairs
            int g = 1;
            for (int i = 0; i < 3; i++)
                if (b->bt_global_ns[i] >= 0 && (b->bt_global_ns[g] < 0 || b->bt_global_ns[i] < b->bt_global_ns[g])) g = i;
            b->bt_global = g;
            b->bt_best = b->bt_global_ns[g];
            std::vector<std::pair<uint64_t, uint64_t>> by(b->bt_class_pairs.begin(), b->bt_class_pairs.end());
            std::sort(by.begin(), by.end(), [](const auto& x, const auto& y) { return x.second > y.second; });
            if (b->bt_best >= 0)
                for (size_t i = 0; i < by.size() && i < TUNE_CLASSES; i++)
                    for (int c2 = 0; c2 < 3; c2++)
                        if (c2 != g) b->bt_trials.push_back({by[i].first, c2});
        }
    }
    b->bt_pending.swap(keep_b);
    if (b->bt_next >= 0 && b->bt_next >= (int)b->bt_trials.size() && b->bt_pending.empty()) {
        // every trial done: each tuned link takes its class's candidate
        for (uint32_t l = 0; l < b->e.n; l++) {
            if (b->link_class[l] == NO_CLASS) continue;
            const auto it = b->bt_choice.find(b->link_class[l]);
            b->e.bin_req[l] = TUNE_BIN_BYTES[it == b->bt_choice.end() ? b->bt_global : it->second];
        }
        b->bt_next = -1;
    }
    if (b->tune_idx >= (int)b->cands.size() && b->tune_pending.empty()) {
        int best = 0;
        for (int i = 1; i < (int)b->cands.size(); i++)
            if (b->cands[i].ns_per_pair >= 0 &&
                (b->cands[best].ns_per_pair < 0 || b->cands[i].ns_per_pair < b->cands[best].ns_per_pair))
                best = i;
        b->pass_bytes = b->cands[best].pass;
        b->tile_pairs = b->cands[best].tile;
        b->tune_idx = -1;
    }
}

// The binned scan of the batch's links `links` (each with enough pairs in
// this call; offsets as in ssd_batch_scan).  The links are packed, in order,
// into groups whose staging fits the batch's bin buffers; a group takes one
// binning launch and one store launch per kind (counted, in two LDS classes;
// uncounted), every workgroup finding its link in the launch's workgroup
// prefix.  A link whose staging alone exceeds the buffers (or whose offsets
// are not packed) is scanned on its own, in steps.
int enqueue_batch_binned(ssd_batch* b, const uint2* pairs, const uint64_t* offsets, const std::vector<uint32_t>& links)
{
    Engine* e = &b->e;
    const uint32_t n = e->n;
    struct Plan {
        uint32_t l;
        BinnedCall c;
        uint64_t blocks, items, table;
    };
    std::vector<Plan> plans;
    std::vector<uint32_t> alone;
    for (uint32_t l : links) {
        const uint64_t np = offsets[l + 1] - offsets[l];
        Plan p{l, binned_call(e, l, np, DEFAULT_BIN_BYTES), 0, 0, 0};
        if (p.c.counted && (!p.c.csh || p.c.bp.shift != p.c.csh)) return fail(SSD_E_STATE, "counted bin plan mismatch");
        p.blocks = (np + p.c.bp.pb - 1) / p.c.bp.pb;
        p.items = p.blocks * p.c.seg;
        p.table = (uint64_t)(p.c.bp.n_bins + 1) * p.blocks;
        if (p.items > e->L.bin_items_words || p.table > e->L.bin_table_words || p.c.bp.shift > 21 || e->hl[l].cell16)
            alone.push_back(l);
        else
            plans.push_back(p);
    }
    // the arguments of every launch of this call, staged in pinned memory
    // and copied to the device once
    const uint64_t bin_region = 0;
    const uint64_t app_region = align_up((uint64_t)n * sizeof(BinArgs));
    const uint64_t pre_region = app_region + align_up((uint64_t)n * sizeof(ApplyArgs));
    const uint32_t buf = b->mb_next;
    b->mb_next ^= 1u;
    if (b->mb_used[buf]) HIPCHK(e, hipEventSynchronize(b->mb_done[buf]));      // its last copy has run
    uint8_t* host = static_cast<uint8_t*>(b->mb_pinned[buf]);
    uint8_t* dev = e->at<uint8_t>(e->L.multi_args);
    BinArgs* hb = reinterpret_cast<BinArgs*>(host + bin_region);
    ApplyArgs* ha = reinterpret_cast<ApplyArgs*>(host + app_region);
    uint32_t* hp = reinterpret_cast<uint32_t*>(host + pre_region);
    struct Launch {
        uint32_t kind;        // 1: binning (every variant); 10, 12 counted stores (LDS for two workgroups
                              // per compute unit, more); 11 uncounted stores
        uint32_t first, count, pre, total_wg, lds;
    };
    std::vector<Launch> launches;
    uint32_t nb = 0, na = 0, np_words = 0;
    uint32_t* items = e->at<uint32_t>(e->L.bin_items);
    uint32_t* table = e->at<uint32_t>(e->L.bin_table);
    for (size_t g0 = 0; g0 < plans.size();) {
        // the group [g0, g1): staging fits the buffers
        size_t g1 = g0;
        uint64_t iw = 0, tw = 0;
        while (g1 < plans.size() && iw + plans[g1].items <= e->L.bin_items_words &&
               tw + plans[g1].table <= e->L.bin_table_words) {
            iw += plans[g1].items;
            tw += plans[g1].table;
            g1++;
        }
        std::vector<BinArgs> ba(g1 - g0);
        std::vector<ApplyArgs> aa(g1 - g0);
        uint64_t io = 0, to = 0;
        for (size_t i = g0; i < g1; i++) {
            const Plan& p = plans[i];
            binned_count_state(e, p.l, p.c);
            BinArgs& x = ba[i - g0];
            ApplyArgs& y = aa[i - g0];
            binned_args(e, p.l, p.c, items + io, table + to, DEFAULT_APPLY_SEGMENTS, &x, &y);
            x.pairs = pairs + offsets[p.l];
            x.n = offsets[p.l + 1] - offsets[p.l];
            x.blocks = (uint32_t)p.blocks;
            y.blocks = x.blocks;
            y.parts = (y.blocks + y.per_part - 1) / y.per_part;
            io += p.items;
            to += p.table;
        }
        // binning: one launch, each workgroup in its link's variant
        {
            Launch L{1u, nb, 0, np_words, 0, 0};
            for (const BinArgs& x : ba) {
                hb[nb++] = x;
                hp[np_words + L.count] = L.total_wg;
                L.count++;
                L.total_wg += bin_workgroups(x);
            }
            hp[np_words + L.count] = L.total_wg;
            np_words += L.count + 1;
            launches.push_back(L);
        }
        // stores: counted (the links whose LDS lets two workgroups share a
        // compute unit, then the others: a launch's LDS is its largest
        // link's), then uncounted
        auto kind_of = [](const ApplyArgs& y) {
            if (!y.counts) return 11u;
            return counted_lds_bytes(y.bin_shift, y.log2eta, y.k) <= COUNTED_LDS_PAIR ? 10u : 12u;
        };
        for (uint32_t kind : {10u, 12u, 11u}) {
            Launch L{kind, na, 0, np_words, 0, 0};
            for (const ApplyArgs& y : aa) {
                if (kind_of(y) != kind) continue;
                ha[na++] = y;
                hp[np_words + L.count] = L.total_wg;
                L.count++;
                L.total_wg += kind == 11u ? apply_workgroups(y) : apply_counted_workgroups(y);
                if (kind != 11u)
                    L.lds = std::max<uint32_t>(L.lds, (uint32_t)counted_lds_bytes(y.bin_shift, y.log2eta, y.k));
            }
            if (!L.count) continue;
            hp[np_words + L.count] = L.total_wg;
            np_words += L.count + 1;
            launches.push_back(L);
        }
        g0 = g1;
    }
    if (!launches.empty()) {
        HIPCHK(e, hipMemcpyAsync(dev, host, multi_args_bytes(n), hipMemcpyHostToDevice, e->stream));
        HIPCHK(e, hipEventRecord(b->mb_done[buf], e->stream));
        b->mb_used[buf] = true;
        const BinArgs* db = reinterpret_cast<const BinArgs*>(dev + bin_region);
        const ApplyArgs* da = reinterpret_cast<const ApplyArgs*>(dev + app_region);
        const uint32_t* dp = reinterpret_cast<const uint32_t*>(dev + pre_region);
        for (const Launch& L : launches) {
            PhaseMark pm = phase_begin(e);
            if (L.kind >= 10u) {
                MultiApplyArgs m{da + L.first, dp + L.pre, L.count};
                HIPCHK(e, L.kind != 11u ? launch_apply_counted_multi(m, L.total_wg, L.lds, e->stream)
                                        : launch_apply_multi(m, L.total_wg, e->stream));
                phase_end(e, pm, 0, 1);
            } else {
                MultiBinArgs m{db + L.first, dp + L.pre, L.count};
                HIPCHK(e, launch_bin_multi(m, L.total_wg, e->stream));
                phase_end(e, pm, PHASE_SCAN_BIN, 1);
            }
        }
    }
    for (uint32_t l : alone) {
        int rc = enqueue_binned_scan(e, l, pairs + offsets[l], offsets[l + 1] - offsets[l], DEFAULT_BIN_BYTES,
                                     DEFAULT_APPLY_SEGMENTS, engine_bins(e));
        if (rc) return rc;
    }
    return SSD_OK;
}

}  // namespace

// ---------------------------------------------------------------- group

struct ssd_group {
    Engine e;                          // header-only engine over the bound members
    uint32_t max_members = 0;
    uint32_t scan_blocks = 2048;       // tile-scan workgroups: 8 per compute unit
    std::vector<uint64_t> bound;       // ids of the members whose descriptors are on the device
    // a close begun and not yet ended: its members and its completion
    bool pending = false;
    std::vector<ssd_detector*> pending_members;
    hipEvent_t done = nullptr;
    // arguments of the binned members' multi-link launches, staged in pinned
    // memory (two buffers, each reused once its last copy has run)
    void* mb_pinned[2] = {nullptr, nullptr};
    hipEvent_t mb_done[2] = {nullptr, nullptr};
    bool mb_used[2] = {false, false};
    uint32_t mb_next = 0;
    // the tile scan's zeroed counter and windows, staged the same way
    void* tile_pinned[2] = {nullptr, nullptr};
    hipEvent_t tile_done[2] = {nullptr, nullptr};
    bool tile_used[2] = {false, false};
    uint32_t tile_next = 0;
    // the bound members' descriptors, wave prefix and row table, staged the same way
    void* bind_pinned[2] = {nullptr, nullptr};
    hipEvent_t bind_done[2] = {nullptr, nullptr};
    bool bind_used[2] = {false, false};
    uint32_t bind_next = 0;
};

namespace {

// Host staging of a group's bound members: descriptors, wave prefix, row table.
uint64_t group_bind_bytes(uint32_t max_members)
{
    return align_up((uint64_t)max_members * sizeof(LinkDesc)) + align_up(((uint64_t)max_members + 1) * 8) +
           (uint64_t)max_members * MAX_ROWS * 4;
}

Layout plan_group(uint32_t max_members)
{
    Layout L;
    uint64_t o = 0;
    L.links = o; o = align_up(o + max_members * sizeof(LinkDesc));
    L.se_prefix = o; o = align_up(o + (max_members + 1) * 8);
    L.row_table = o; o = align_up(o + (uint64_t)max_members * MAX_ROWS * 4);
    L.pack_offsets = o; o = align_up(o + (max_members + 1) * 8);
    L.tiles = o; o = align_up(o + 8 + MAX_WINDOWS * sizeof(ScanWindow));
    L.count_list = o; o = align_up(o + (2ull * max_members + 1) * 4);
    L.ctl = o; o = align_up(o + max_members * sizeof(Ctl));    // unused: members' own blocks are read
    L.packed = o; o = align_up(o + BATCH_STAGE * sizeof(SuperPointDev));
    L.multi_args = o; o = align_up(o + multi_args_bytes(max_members));
    L.total = o;
    L.pack_cap = BATCH_STAGE;
    L.tile_cap = MAX_WINDOWS;
    return L;
}

// Point the group's descriptors at these members (uploads only on change).
int group_bind(ssd_group* g, ssd_detector* const* m, uint32_t n)
{
    Engine* e = &g->e;
    if (!m || n < 1 || n > g->max_members) return fail(SSD_E_PARAM, "need 1..%u members", g->max_members);
    bool same = g->bound.size() == n;
    for (uint32_t i = 0; i < n; i++) {
        if (!m[i]) return fail(SSD_E_PARAM, "member %u is NULL", i);
        if (m[i]->e.broken) return fail(SSD_E_STATE, "member %u is unusable", i);
        if (m[i]->e.device != e->device) return fail(SSD_E_INCOMPAT, "member %u is on another device", i);
        if (m[i]->e.stream != e->stream) return fail(SSD_E_INCOMPAT, "member %u uses another stream", i);
        if (m[i]->e.hl[0].cell16) return fail(SSD_E_PARAM, "member %u has 16-bit cells: groups take 8-bit members", i);
        for (uint32_t j = 0; j < i; j++)
            if (m[j] == m[i]) return fail(SSD_E_PARAM, "member %u appears twice", i);
        same = same && g->bound[i] == m[i]->id;
    }
    if (same) return SSD_OK;
    e->n = n;
    e->p.resize(n);
    e->T.resize(n);
    e->hl.resize(n);
    e->max_r = 0;
    e->max_chunks = 1;
    e->detect_small = n > 1;
    std::vector<uint64_t> se_prefix(n + 1, 0);
    std::vector<uint32_t> row_table;
    for (uint32_t i = 0; i < n; i++) {
        e->p[i] = m[i]->e.p[0];
        e->T[i] = m[i]->e.T[0];
        e->hl[i] = m[i]->e.hl[0];
        e->hl[i].host_ctl = nullptr;         // the group collects its members' lists itself
        e->hl[i].host_out = nullptr;
        e->hl[i].host_cap = 0;
        se_prefix[i + 1] = se_prefix[i] + detect_waves(e->hl[i]);
        for (uint32_t r = 0; r < e->p[i].r; r++) row_table.push_back((i << 8) | r);
        e->max_r = std::max(e->max_r, e->p[i].r);
        e->max_chunks = std::max(e->max_chunks, e->p[i].eta >> 10);
        e->detect_small = e->detect_small || e->p[i].eta < 4096;
    }
    e->se_total = se_prefix[n];
    e->rows_total = (uint32_t)row_table.size();
    e->counting.assign(n, 0);              // set from the members at every close
    e->count_valid.assign(n, 0);
    e->count_rebuild.assign(n, 0);
    e->count_small.assign(n, 0);
    e->last_mode.assign(n, 0);
    e->bin_req.assign(n, 0);
    e->last_csh.assign(n, 0);
    e->detect_prefix = se_prefix;
    // uploaded from pinned staging (a buffer is reused once its last copies have run)
    const uint32_t buf = g->bind_next;
    g->bind_next ^= 1u;
    if (g->bind_used[buf]) HIPCHK(e, hipEventSynchronize(g->bind_done[buf]));
    uint8_t* host = static_cast<uint8_t*>(g->bind_pinned[buf]);
    const uint64_t pre_at = align_up((uint64_t)g->max_members * sizeof(LinkDesc));
    const uint64_t row_at = pre_at + align_up(((uint64_t)g->max_members + 1) * 8);
    memcpy(host, e->hl.data(), n * sizeof(LinkDesc));
    memcpy(host + pre_at, se_prefix.data(), (n + 1) * 8);
    memcpy(host + row_at, row_table.data(), row_table.size() * 4);
    HIPCHK(e, hipMemcpyAsync(e->dev_links(), host, n * sizeof(LinkDesc), hipMemcpyHostToDevice, e->stream));
    HIPCHK(e, hipMemcpyAsync(e->at<uint64_t>(e->L.se_prefix), host + pre_at, (n + 1) * 8, hipMemcpyHostToDevice,
                             e->stream));
    HIPCHK(e, hipMemcpyAsync(e->at<uint32_t>(e->L.row_table), host + row_at, row_table.size() * 4,
                             hipMemcpyHostToDevice, e->stream));
    HIPCHK(e, hipEventRecord(g->bind_done[buf], e->stream));
    g->bind_used[buf] = true;
    g->bound.resize(n);
    for (uint32_t i = 0; i < n; i++) g->bound[i] = m[i]->id;
    e->results.assign(n, {});
    e->status.assign(n, SSD_OK);
    e->last.assign(n, Ctl{});
    return SSD_OK;
}

}  // namespace

extern "C" {

const char* ssd_strerror(int s)
{
    switch (s) {
    case SSD_OK: return "ok";
    case SSD_E_PARAM: return "invalid parameter";
    case SSD_E_NOMEM: return "buffer too small or misaligned";
    case SSD_E_ORDER: return "slice out of order";
    case SSD_E_OVERFLOW: return "candidate or result capacity exceeded";
    case SSD_E_INCOMPAT: return "incompatible detectors";
    case SSD_E_TRUNC: return "output array too small";
    case SSD_E_DEVICE: return "HIP device error";
    case SSD_E_STATE: return "detector unusable";
    default: return "unknown status";
    }
}

const char* ssd_last_error(void) { return g_last_error.c_str(); }

// ---- single detector

int ssd_query_sizes(const ssd_params* p, uint64_t* state_bytes, uint64_t* scratch_bytes)
{
    if (!p) return fail(SSD_E_PARAM, "params is NULL");
    return engine_query(p, 1, 0, 0, state_bytes, scratch_bytes, true);
}

int ssd_init_detector(const ssd_params* p, const uint32_t* tables_host, void* state_dev, uint64_t state_bytes,
                      void* scratch_dev, uint64_t scratch_bytes, void* stream, ssd_detector** out)
{
    if (!out) return fail(SSD_E_PARAM, "out is NULL");
    *out = nullptr;
    if (!p) return fail(SSD_E_PARAM, "params is NULL");
    int rc = validate(p);
    if (rc) return rc;
    ssd_detector* d = new (std::nothrow) ssd_detector();
    if (!d) return fail(SSD_E_NOMEM, "host allocation failed");
    rc = engine_init(&d->e, p, 1, tables_host, state_dev, state_bytes, scratch_dev, scratch_bytes, stream, 0, 0,
                     PREFIX_MAX, true, true);
    if (rc) {
        engine_release(&d->e);
        delete d;
        return rc;
    }
    // the address of this device's static scratch (ssd_scan_slice_noalloc)
    const hipError_t err = noalloc_setup(d->e.device);
    if (err != hipSuccess) {
        rc = dev_fail(&d->e, err, "hipGetSymbolAddress(scratch)");
        engine_release(&d->e);
        delete d;
        return rc;
    }
    d->e.use_graph = true;
    *out = d;
    return SSD_OK;
}

void ssd_destroy(ssd_detector* d)
{
    if (!d) return;
    (void)hipSetDevice(d->e.device);
    if (d->close_stream) {
        if (!d->e.broken) (void)hipStreamSynchronize(d->close_stream);
        (void)hipStreamDestroy(d->close_stream);
    }
    engine_release(&d->e);
    for (hipEvent_t ev : {d->detect_done, d->close_done})
        if (ev) (void)hipEventDestroy(ev);
    delete d;
}

int ssd_set_tuning(ssd_detector* d, uint32_t knob, uint64_t value)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    switch (knob) {
    case SSD_TUNE_SCAN_PASS_BYTES: d->pass_bytes = value; return SSD_OK;
    case SSD_TUNE_TIMING: d->e.timing = value != 0; return SSD_OK;
    case SSD_TUNE_GRAPH: d->e.use_graph = value != 0; return SSD_OK;
    case SSD_TUNE_SCAN_MODE:
        if (value != SSD_SCAN_PASSES && value != SSD_SCAN_BINNED && value != SSD_SCAN_AUTO)
            return fail(SSD_E_PARAM, "unknown scan mode %llu", (unsigned long long)value);
        d->scan_mode = (uint32_t)value;
        return SSD_OK;
    case SSD_TUNE_SCAN_BIN_BYTES:
        if (!is_pow2(value)) return fail(SSD_E_PARAM, "bin bytes must be a power of two");
        d->bin_bytes = value;
        d->e.counted_bin_bytes = value;
        return SSD_OK;
    case SSD_TUNE_SCAN_APPLY_SEGMENTS:
        if (value < 1 || value > 4096) return fail(SSD_E_PARAM, "apply segments outside 1..4096");
        d->apply_segments = (uint32_t)value;
        return SSD_OK;
    case SSD_TUNE_COUNTED_MIN_ITEMS:
        d->e.counted_min_items = value;
        return SSD_OK;
    case SSD_TUNE_COUNTED:
        if (value > 1) return fail(SSD_E_PARAM, "counted detection is 0 or 1");
        if (value && !d->e.hl[0].counts) return fail(SSD_E_PARAM, "this detector cannot count (eta < 8 k, counters beyond the LDS, or too many bins)");
        if (close_pending(d)) return fail(SSD_E_ORDER, "a close is pending (ssd_close_end first)");
        if (d->e.counting[0] != (value != 0)) {
            d->e.counting[0] = value != 0;
            d->e.count_valid[0] = 0;
            d->e.count_rebuild[0] = 0;
        }
        return SSD_OK;
    case SSD_TUNE_SORT_BLOCK_LIMIT: {
        if (value > SORT_SMALL) return fail(SSD_E_PARAM, "sort block limit above %u", SORT_SMALL);
        if (close_pending(d)) return fail(SSD_E_ORDER, "a close is pending (ssd_close_end first)");
        int rc = usable(&d->e);
        if (rc) return rc;
        d->e.hl[0].sort_limit = value;
        HIPCHK(&d->e, hipMemcpyAsync(&d->e.dev_links()[0].sort_limit, &d->e.hl[0].sort_limit, 8,
                                     hipMemcpyHostToDevice, d->e.stream));
        HIPCHK(&d->e, hipStreamSynchronize(d->e.stream));
        return SSD_OK;
    }
    default: return fail(SSD_E_PARAM, "unknown tuning knob %u", knob);
    }
}

int ssd_scan_slice(ssd_detector* d, const uint32_t* pairs_dev, uint64_t n, uint64_t slice_id)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    Engine* e = &d->e;
    int rc = scan_checks(d, pairs_dev, n, slice_id);
    if (rc || n == 0) return rc;
    if (scans_binned(d))
        return enqueue_binned_scan(e, 0, reinterpret_cast<const uint2*>(pairs_dev), n, d->bin_bytes, d->apply_segments,
                                   engine_bins(e));
    return enqueue_pass_scan(d, reinterpret_cast<const uint2*>(pairs_dev), n);
}

int ssd_scan_slice_noalloc(ssd_detector* d, const uint32_t* pairs_dev, uint64_t n, uint64_t slice_id)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    Engine* e = &d->e;
    int rc = scan_checks(d, pairs_dev, n, slice_id);
    if (rc || n == 0) return rc;
    // no phase timing: its events would be created on first use
    const bool timing = e->timing;
    e->timing = false;
    if (scans_binned(d)) {
        // the binning's staging in this device's static array, looked up at
        // ssd_init_detector; one step for the whole call
        uint8_t* base = noalloc_scratch(e->device);
        const BinnedCall c = binned_call(e, 0, n, d->bin_bytes);
        const uint64_t blocks = (n + c.bp.pb - 1) / c.bp.pb;
        const uint64_t items = align_up(blocks * c.seg * 4), table = (uint64_t)(c.bp.n_bins + 1) * blocks * 4;
        if (!base) rc = fail(SSD_E_STATE, "no static scratch for device %d", e->device);
        else if (items + table > SSD_NOALLOC_SCRATCH_BYTES)
            rc = fail(SSD_E_NOMEM, "a binned scan of %llu pairs needs %llu bytes of staging, the static scratch holds "
                      "%llu: split the slice over smaller calls", (unsigned long long)n,
                      (unsigned long long)(items + table), (unsigned long long)SSD_NOALLOC_SCRATCH_BYTES);
        else
            rc = enqueue_binned_scan(e, 0, reinterpret_cast<const uint2*>(pairs_dev), n, d->bin_bytes,
                                     d->apply_segments,
                                     {reinterpret_cast<uint32_t*>(base), reinterpret_cast<uint32_t*>(base + items),
                                      blocks * c.seg, (uint64_t)(c.bp.n_bins + 1) * blocks});
    } else {
        rc = enqueue_pass_scan(d, reinterpret_cast<const uint2*>(pairs_dev), n);     // no staging
    }
    e->timing = timing;
    return rc;
}

int ssd_close_begin(ssd_detector* d)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    Engine* e = &d->e;
    int rc = usable(e);
    if (rc) return rc;
    if (close_pending(d)) return fail(SSD_E_ORDER, "a close is already pending (ssd_close_end first)");
    rc = detector_streams(d);
    if (rc) return rc;
    // the sort kernel writes the first host_cap entries of the list into the
    // pinned mailbox; longer lists take a second copy when collected
    const uint64_t prefix = e->hl[0].host_cap;
    // hot detection on the caller's stream, after the slice's scans; it
    // reuses the hot bitmasks and snapshots of the previous close, whose
    // second part must have finished.  (Run on the second stream instead, hot
    // detection overlapped with the next slice's binning and both slowed:
    // 0.764 ms per core-link step against 0.714.)
    HIPCHK(e, hipStreamWaitEvent(e->stream, d->close_done, 0));
    rc = enqueue_close_head(e);
    if (rc) return rc;
    HIPCHK(e, hipEventRecord(d->detect_done, e->stream));
    // the rest of the close reads no state: it runs on the second stream
    // while the caller's stream goes on with the next slice's scans
    HIPCHK(e, hipStreamWaitEvent(d->close_stream, d->detect_done, 0));
    const hipStream_t caller = e->stream;
    e->stream = d->close_stream;
    rc = e->use_graph ? close_graph_tail(e, false, prefix) : enqueue_close_tail(e, false, prefix, false);
    if (rc == SSD_OK) {
        hipError_t err = hipEventRecord(d->close_done, e->stream);
        if (err != hipSuccess) rc = dev_fail(e, err, "hipEventRecord");
    }
    e->stream = caller;
    if (rc) return rc;
    d->pending = true;
    d->pending_prefix = prefix;
    e->clock++;
    return SSD_OK;
}

int ssd_close_end(ssd_detector* d, ssd_super_point* out_host, uint64_t cap, uint64_t* n_out)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    Engine* e = &d->e;
    int rc = usable(e);
    if (rc) return rc;
    if (n_out) *n_out = 0;
    if (!d->pending) return fail(SSD_E_ORDER, "no close is pending");
    d->pending = false;
    HIPCHK(e, hipEventSynchronize(d->close_done));
    phase_collect(e);
    rc = collect_results(e, false, d->pending_prefix);
    if (rc) return rc;
    const ssd_params& p = d->p();
    if (e->status[0] != SSD_OK) {
        const Ctl& c = e->last[0];
        if (c.n_acc > p.max_results)
            return fail(SSD_E_OVERFLOW, "%llu accepted hosts > max_results %llu", (unsigned long long)c.n_acc,
                        (unsigned long long)p.max_results);
        return fail(SSD_E_OVERFLOW, "a candidate level exceeded max_tuples %llu", (unsigned long long)p.max_tuples);
    }
    return ssd_get_results(d, out_host, cap, n_out);
}

int ssd_close_slice(ssd_detector* d, uint32_t flags, ssd_super_point* out_host, uint64_t cap, uint64_t* n_out)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    Engine* e = &d->e;
    int rc = usable(e);
    if (rc) return rc;
    if (flags & ~SSD_ADVANCE_ONLY) return fail(SSD_E_PARAM, "unknown close flags 0x%x", flags);
    if (n_out) *n_out = 0;
    if (close_pending(d)) return fail(SSD_E_ORDER, "a close is pending (ssd_close_end first)");
    if (flags & SSD_ADVANCE_ONLY) {
        rc = enqueue_advance_only(e);
        if (rc) return rc;
        e->clock++;
        e->results[0].clear();
        e->have_last = false;
        return SSD_OK;
    }
    // a synchronous close: both parts on the caller's stream (nothing is
    // enqueued between them, so the second stream would only add its event
    // hand-over)
    rc = detector_streams(d);
    if (rc) return rc;
    const uint64_t prefix = e->hl[0].host_cap;
    HIPCHK(e, hipStreamWaitEvent(e->stream, d->close_done, 0));     // a pipelined close before it
    rc = enqueue_close_head(e);
    if (rc) return rc;
    rc = e->use_graph ? close_graph_tail(e, false, prefix) : enqueue_close_tail(e, false, prefix, false);
    if (rc) return rc;
    HIPCHK(e, hipEventRecord(d->close_done, e->stream));
    d->pending = true;
    d->pending_prefix = prefix;
    e->clock++;
    return ssd_close_end(d, out_host, cap, n_out);
}

int ssd_get_results(ssd_detector* d, ssd_super_point* out_host, uint64_t cap, uint64_t* n_out)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    const auto& r = d->e.results[0];
    const uint64_t m = r.size();
    if (n_out) *n_out = m;
    if (m > cap) return fail(SSD_E_TRUNC, "result list holds %llu entries, cap is %llu", (unsigned long long)m,
                             (unsigned long long)cap);
    if (m && !out_host) return fail(SSD_E_PARAM, "out_host is NULL");
    if (m) memcpy(out_host, r.data(), m * sizeof(ssd_super_point));
    return SSD_OK;
}

int ssd_merge_router_state(ssd_detector* g, ssd_detector* const* routers, uint32_t n)
{
    if (!g) return fail(SSD_E_PARAM, "detector is NULL");
    int rc = usable(&g->e);
    if (rc) return rc;
    if (close_pending(g)) return fail(SSD_E_ORDER, "the global detector has a close pending");
    if (!routers || n < 1) return fail(SSD_E_PARAM, "need at least one router");
    const ssd_params& gp = g->p();
    for (uint32_t j = 0; j < n; j++) {
        const ssd_detector* r = routers[j];
        if (!r) return fail(SSD_E_PARAM, "router %u is NULL", j);
        if (r == g) return fail(SSD_E_PARAM, "router %u is the global detector", j);
        if (r->e.broken) return fail(SSD_E_STATE, "router %u is unusable", j);
        if (close_pending(r)) return fail(SSD_E_ORDER, "router %u has a close pending", j);
        const ssd_params& rp = r->p();
        if (rp.q != gp.q || rp.r != gp.r || rp.delta != gp.delta || rp.eta != gp.eta || rp.k != gp.k ||
            cell16(rp) != cell16(gp) ||
            rp.key_bits != gp.key_bits || r->e.tables != g->e.tables)
            return fail(SSD_E_INCOMPAT, "router %u differs in geometry or hash tables", j);
        if (r->e.clock != g->e.clock) return fail(SSD_E_INCOMPAT, "router %u is at slice %llu, global at %llu", j,
                                                  (unsigned long long)r->e.clock, (unsigned long long)g->e.clock);
        if (r->e.device != g->e.device) return fail(SSD_E_INCOMPAT, "router %u is on another device", j);
    }
    g->e.count_valid[0] = 0;          // merged cells are not counted
    g->e.count_rebuild[0] = 0;
    MergeArgs a{};
    a.dst = g->D().state;
    a.n16 = g->e.L.state_total / 16u;
    a.cur = stamp_of(g->e.clock, cell16(gp));
    a.k = gp.k;
    a.cell16 = cell16(gp) ? 1u : 0u;
    // associative merge in batches; later batches fold the partial result in
    uint32_t done = 0, launches = 0;
    PhaseMark pm = phase_begin(&g->e);
    while (done < n) {
        uint32_t m = 0;
        if (done > 0) a.src[m++] = g->D().state;
        while (m < MAX_MERGE_SOURCES && done < n) a.src[m++] = routers[done++]->D().state;
        a.n_src = m;
        HIPCHK(&g->e, launch_merge(a, g->e.stream));
        launches++;
    }
    phase_end(&g->e, pm, 6, launches);
    return SSD_OK;
}

int ssd_read_canonical_state(ssd_detector* d, uint16_t* out_dev, uint64_t n_cells)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    Engine* e = &d->e;
    int rc = usable(e);
    if (rc) return rc;
    const uint64_t n = state_cells(d->p());
    if (!out_dev || n_cells < n) return fail(SSD_E_NOMEM, "canonical state needs %llu cells", (unsigned long long)n);
    const bool c16 = cell16(d->p());
    HIPCHK(e, launch_canonical(d->D().state, out_dev, n, stamp_of(e->clock, c16), d->p().k, c16, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    return SSD_OK;
}

// ---- checkpoint: header, then the state bytes
namespace {
struct StateHeader {
    char magic[8];                 // "SSDSTATE"
    uint32_t version, header_bytes;
    uint32_t q, r, delta, eta, k, theta, key_bits, flags, cell_bits, pad;
    uint64_t tables_hash;          // FNV-1a 64 of the 2048 table words
    uint64_t clock;                // the open slice
    uint64_t state_bytes;
};
constexpr uint32_t STATE_VERSION = 1;
static_assert(sizeof(StateHeader) == 80, "the checkpoint header is 80 bytes");

uint64_t tables_hash(const uint32_t* t)
{
    uint64_t h = 0xCBF29CE484222325ull;
    for (uint32_t i = 0; i < 2048; i++)
        for (int b = 0; b < 4; b++) h = (h ^ ((t[i] >> (8 * b)) & 0xFFu)) * 0x100000001B3ull;
    return h;
}

StateHeader state_header(const ssd_detector* d)
{
    StateHeader h{};
    memcpy(h.magic, "SSDSTATE", 8);
    h.version = STATE_VERSION;
    h.header_bytes = sizeof(StateHeader);
    const ssd_params& p = d->p();
    h.q = p.q; h.r = p.r; h.delta = p.delta; h.eta = p.eta; h.k = p.k; h.theta = p.theta;
    h.key_bits = p.key_bits; h.flags = p.flags; h.cell_bits = cell16(p) ? 16u : 8u;
    h.tables_hash = tables_hash(d->e.tables.data());
    h.clock = d->e.clock;
    h.state_bytes = state_bytes_of(p);
    return h;
}
}  // namespace

int ssd_export_state(ssd_detector* d, void* out_host, uint64_t cap, uint64_t* n_out)
{
    if (!d || !n_out) return fail(SSD_E_PARAM, "NULL argument");
    Engine* e = &d->e;
    int rc = usable(e);
    if (rc) return rc;
    if (close_pending(d)) return fail(SSD_E_ORDER, "a close is pending (ssd_close_end first)");
    const StateHeader h = state_header(d);
    const uint64_t need = sizeof(StateHeader) + h.state_bytes;
    *n_out = need;
    if (!out_host || cap < need)
        return fail(SSD_E_TRUNC, "the state blob holds %llu bytes, cap is %llu", (unsigned long long)need,
                    (unsigned long long)cap);
    memcpy(out_host, &h, sizeof h);
    HIPCHK(e, hipMemcpyAsync(static_cast<uint8_t*>(out_host) + sizeof h, d->D().state, h.state_bytes,
                             hipMemcpyDeviceToHost, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    return SSD_OK;
}

int ssd_import_state(ssd_detector* d, const void* blob_host, uint64_t n)
{
    if (!d || !blob_host) return fail(SSD_E_PARAM, "NULL argument");
    Engine* e = &d->e;
    int rc = usable(e);
    if (rc) return rc;
    if (close_pending(d)) return fail(SSD_E_ORDER, "a close is pending (ssd_close_end first)");
    StateHeader h;
    if (n < sizeof h) return fail(SSD_E_PARAM, "a state blob holds at least a %zu-byte header", sizeof h);
    memcpy(&h, blob_host, sizeof h);
    if (memcmp(h.magic, "SSDSTATE", 8) != 0 || h.version != STATE_VERSION || h.header_bytes != sizeof h)
        return fail(SSD_E_PARAM, "not a state blob of this library (format %u)", h.version);
    const StateHeader mine = state_header(d);
    if (h.q != mine.q || h.r != mine.r || h.delta != mine.delta || h.eta != mine.eta || h.k != mine.k ||
        h.theta != mine.theta || h.key_bits != mine.key_bits || h.flags != mine.flags ||
        h.cell_bits != mine.cell_bits)
        return fail(SSD_E_INCOMPAT, "the blob's parameters differ from the detector's");
    if (h.tables_hash != mine.tables_hash) return fail(SSD_E_INCOMPAT, "the blob's hash tables differ from the detector's");
    if (h.state_bytes != mine.state_bytes || n != sizeof h + h.state_bytes)
        return fail(SSD_E_PARAM, "the blob holds %llu bytes, its header says %llu", (unsigned long long)n,
                    (unsigned long long)(sizeof h + h.state_bytes));
    HIPCHK(e, hipMemcpyAsync(d->D().state, static_cast<const uint8_t*>(blob_host) + sizeof h, h.state_bytes,
                             hipMemcpyHostToDevice, e->stream));
    const Clock c{h.clock};
    HIPCHK(e, hipMemcpyAsync(d->D().clock, &c, sizeof c, hipMemcpyHostToDevice, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    e->clock = h.clock;
    // the counters are not in the blob: stale, rebuilt from the state after
    // the next large binned call, else the next close reads the state
    e->count_valid[0] = 0;
    e->count_rebuild[0] = 0;
    e->count_small[0] = 0;
    e->have_last = false;
    e->results[0].clear();
    return SSD_OK;
}

int ssd_read_rk(ssd_detector* d, uint32_t* out_host, uint64_t n)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    if (close_pending(d)) return fail(SSD_E_ORDER, "a close is pending (ssd_close_end first)");
    return engine_read_rk(&d->e, 0, out_host, n);
}

int ssd_read_hot(ssd_detector* d, uint32_t* counts_host, uint32_t* lists_host, uint64_t cap)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    if (close_pending(d)) return fail(SSD_E_ORDER, "a close is pending (ssd_close_end first)");
    return engine_read_hot(&d->e, 0, counts_host, lists_host, cap);
}

int ssd_read_tuples(ssd_detector* d, uint32_t* out_host, uint64_t cap, uint64_t* n_out)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    Engine* e = &d->e;
    int rc = usable(e);
    if (rc) return rc;
    if (close_pending(d)) return fail(SSD_E_ORDER, "a close is pending (ssd_close_end first)");
    if (!e->have_last) return fail(SSD_E_STATE, "no reconstructing close yet");
    const ssd_params& p = d->p();
    const uint32_t lf = p.r - 3;
    const uint64_t n = e->last[0].level_n[lf];
    if (e->status[0] != SSD_OK) return fail(SSD_E_OVERFLOW, "the last close overflowed");
    if (n_out) *n_out = n;
    if (n > cap) return fail(SSD_E_TRUNC, "%llu tuples, cap %llu", (unsigned long long)n, (unsigned long long)cap);
    if (!n) return SSD_OK;
    if (!out_host) return fail(SSD_E_PARAM, "out_host is NULL");
    std::vector<uint64_t> x(n);
    std::vector<uint32_t> h0(n);
    HIPCHK(e, hipMemcpyAsync(x.data(), d->D().ctb_x[lf & 1], n * 8, hipMemcpyDeviceToHost, e->stream));
    HIPCHK(e, hipMemcpyAsync(h0.data(), d->D().ctb_h0[lf & 1], n * 4, hipMemcpyDeviceToHost, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    // inspection only: expand the stored (he_0, regained bits) form to one column per row
    const uint32_t qmask = (1u << p.q) - 1u;
    for (uint64_t t = 0; t < n; t++) {
        uint32_t* o = out_host + t * p.r;
        o[0] = h0[t];
        for (uint32_t i = 1; i < p.r; i++) o[i] = ((uint32_t)(x[t] >> ((i - 1) * p.delta)) & qmask) ^ h0[t];
    }
    return SSD_OK;
}

int ssd_read_timing(ssd_detector* d, double* ms_out, uint64_t* launches_out, int reset)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    if (d->close_stream && !d->e.broken) HIPCHK(&d->e, hipStreamSynchronize(d->close_stream));
    return read_timing(&d->e, ms_out, launches_out, reset);
}

int ssd_get_info(ssd_detector* d, ssd_info* out)
{
    if (!d || !out) return fail(SSD_E_PARAM, "NULL argument");
    engine_info(d->e, 0, out);
    return SSD_OK;
}

// ---- batch

// a batch keeps the staging of the binned scan (any link with enough pairs
// in a call is scanned binned)
static bool batch_bins(const ssd_params* p, uint32_t n) { return p && n >= 1; }

// batch links take 8-bit cells (the persistent tile scan and the batched hot
// detection are written for them)
static int batch_cells_ok(const ssd_params* p, uint32_t n)
{
    for (uint32_t l = 0; p && l < n && l < MAX_LINKS; l++)
        if (p[l].cell_bits == 16) return fail(SSD_E_PARAM, "link %u: batches take 8-bit cells (k <= 254)", l);
    return SSD_OK;
}

int ssd_batch_query_sizes(const ssd_params* p, uint32_t n, uint64_t* state_bytes, uint64_t* scratch_bytes)
{
    if (int rc = batch_cells_ok(p, n)) return rc;
    return engine_query(p, n, BATCH_STAGE, MAX_WINDOWS, state_bytes, scratch_bytes, batch_bins(p, n));
}

int ssd_batch_init(const ssd_params* p, uint32_t n, const uint32_t* tables_host, void* state_dev,
                   uint64_t state_bytes, void* scratch_dev, uint64_t scratch_bytes, void* stream, ssd_batch** out)
{
    if (!out) return fail(SSD_E_PARAM, "out is NULL");
    *out = nullptr;
    if (int rc = batch_cells_ok(p, n)) return rc;
    const bool bins = batch_bins(p, n);
    int rc = engine_query(p, n, BATCH_STAGE, MAX_WINDOWS, nullptr, nullptr, bins);
    if (rc) return rc;
    ssd_batch* b = new (std::nothrow) ssd_batch();
    if (!b) return fail(SSD_E_NOMEM, "host allocation failed");
    rc = engine_init(&b->e, p, n, tables_host, state_dev, state_bytes, scratch_dev, scratch_bytes, stream,
                     BATCH_STAGE, MAX_WINDOWS, BATCH_STAGE, bins);
    if (rc == SSD_OK) {
        b->e.use_graph = true;
        b->e.counted_min_items = BATCH_COUNTED_MIN_ITEMS;
        for (int i = 0; i < 2 && rc == SSD_OK; i++) {
            hipError_t err = hipHostMalloc(&b->tile_pinned[i], 8 + MAX_WINDOWS * sizeof(ScanWindow), hipHostMallocDefault);
            if (err == hipSuccess) err = hipEventCreateWithFlags(&b->tile_done[i], hipEventDisableTiming);
            if (err == hipSuccess) err = hipHostMalloc(&b->mb_pinned[i], multi_args_bytes(n), hipHostMallocDefault);
            if (err == hipSuccess) err = hipEventCreateWithFlags(&b->mb_done[i], hipEventDisableTiming);
            if (err != hipSuccess) rc = dev_fail(&b->e, err, "batch staging");
        }
        hipDeviceProp_t prop;
        if (rc == SSD_OK && hipGetDeviceProperties(&prop, b->e.device) == hipSuccess)
            b->scan_blocks = (uint32_t)prop.multiProcessorCount * 8u;
    }
    if (rc) {
        for (int i = 0; i < 2; i++) {
            if (b->tile_pinned[i]) (void)hipHostFree(b->tile_pinned[i]);
            if (b->tile_done[i]) (void)hipEventDestroy(b->tile_done[i]);
            if (b->mb_pinned[i]) (void)hipHostFree(b->mb_pinned[i]);
            if (b->mb_done[i]) (void)hipEventDestroy(b->mb_done[i]);
        }
        engine_release(&b->e);
        delete b;
        return rc;
    }
    *out = b;
    return SSD_OK;
}

void ssd_batch_destroy(ssd_batch* b)
{
    if (!b) return;
    engine_release(&b->e);
    if (b->done) (void)hipEventDestroy(b->done);
    for (auto& ev : b->tune_events) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    for (auto& c : b->bt_pending) {
        (void)hipEventDestroy(c.a);
        (void)hipEventDestroy(c.b);
    }
    for (int i = 0; i < 2; i++) {
        if (b->tile_pinned[i]) (void)hipHostFree(b->tile_pinned[i]);
        if (b->tile_done[i]) (void)hipEventDestroy(b->tile_done[i]);
        if (b->mb_pinned[i]) (void)hipHostFree(b->mb_pinned[i]);
        if (b->mb_done[i]) (void)hipEventDestroy(b->mb_done[i]);
    }
    delete b;
}

int ssd_batch_set_tuning(ssd_batch* b, uint32_t knob, uint64_t value)
{
    if (!b) return fail(SSD_E_PARAM, "batch is NULL");
    switch (knob) {
    case SSD_TUNE_SCAN_PASS_BYTES: b->pass_bytes = value; return SSD_OK;
    case SSD_TUNE_SCAN_TILE_PAIRS:
        if (value < 256) return fail(SSD_E_PARAM, "tile pairs below 256");
        b->tile_pairs = value;
        return SSD_OK;
    case SSD_TUNE_TIMING: b->e.timing = value != 0; return SSD_OK;
    case SSD_TUNE_GRAPH: b->e.use_graph = value != 0; return SSD_OK;
    case SSD_TUNE_SCAN_MODE:
        if (value != SSD_SCAN_PASSES && value != SSD_SCAN_AUTO)
            return fail(SSD_E_PARAM, "batches take SSD_SCAN_PASSES or SSD_SCAN_AUTO");
        b->scan_mode = (uint32_t)value;
        return SSD_OK;
    case SSD_TUNE_COUNTED_MIN_ITEMS:
        b->e.counted_min_items = value;
        return SSD_OK;
    case SSD_TUNE_COUNTED: {
        // every link whose scans are binned and that can count (others: no effect)
        if (value > 1) return fail(SSD_E_PARAM, "counted detection is 0 or 1");
        Engine& e = b->e;
        for (uint32_t l = 0; l < e.n; l++) {
            if (!e.hl[l].counts || e.counting[l] == (value != 0)) continue;
            e.counting[l] = value != 0;
            e.count_valid[l] = 0;
            e.count_rebuild[l] = 0;
        }
        return SSD_OK;
    }
    case SSD_TUNE_AUTOTUNE:
        if (!value) { b->tune_idx = -1; b->bt_next = -1; return SSD_OK; }
        b->cands.clear();
        for (uint64_t pass : {64ull << 20, 128ull << 20, 256ull << 20})
            for (uint64_t tile : {1024ull, 4096ull, 16384ull}) b->cands.push_back({pass, tile, -1.0});
        b->bt_trials = {{NO_CLASS, 0}, {NO_CLASS, 1}, {NO_CLASS, 2}};
        b->bt_next = 0;
        b->bt_choice.clear();
        b->bt_class_pairs.clear();
        b->bt_best = -1.0;
        for (double& x : b->bt_global_ns) x = -1.0;
        b->link_class.assign(b->e.n, NO_CLASS);
        b->tune_idx = 0;
        return SSD_OK;
    default: return fail(SSD_E_PARAM, "unknown tuning knob %u", knob);
    }
}

int ssd_batch_get_tuning(ssd_batch* b, uint32_t knob, uint64_t* value)
{
    if (!b || !value) return fail(SSD_E_PARAM, "NULL argument");
    switch (knob) {
    case SSD_TUNE_SCAN_PASS_BYTES: *value = b->pass_bytes; return SSD_OK;
    case SSD_TUNE_SCAN_TILE_PAIRS: *value = b->tile_pairs; return SSD_OK;
    case SSD_TUNE_TIMING: *value = b->e.timing; return SSD_OK;
    case SSD_TUNE_GRAPH: *value = b->e.use_graph; return SSD_OK;
    case SSD_TUNE_AUTOTUNE: *value = b->tune_idx >= 0 || b->bt_next >= 0; return SSD_OK;
    case SSD_TUNE_COUNTED:
        *value = 0;
        for (uint32_t l = 0; l < b->e.n; l++) *value |= b->e.counting[l];
        return SSD_OK;
    default: return fail(SSD_E_PARAM, "unknown tuning knob %u", knob);
    }
}

int ssd_batch_scan(ssd_batch* b, const uint32_t* pairs_dev, const uint64_t* offsets_host, uint64_t slice_id)
{
    if (!b) return fail(SSD_E_PARAM, "batch is NULL");
    Engine* e = &b->e;
    int rc = usable(e);
    if (rc) return rc;
    if (slice_id != e->clock)
        return fail(SSD_E_ORDER, "scan of slice %llu while slice %llu is open", (unsigned long long)slice_id,
                    (unsigned long long)e->clock);
    if (!offsets_host) return fail(SSD_E_PARAM, "offsets_host is NULL");
    for (uint32_t l = 0; l < e->n; l++)
        if (offsets_host[l + 1] < offsets_host[l]) return fail(SSD_E_PARAM, "offsets decrease at link %u", l);
    const uint64_t total_pairs = offsets_host[e->n] - offsets_host[0];
    if (total_pairs == 0) return SSD_OK;
    if (!pairs_dev || ((uintptr_t)pairs_dev & 7u)) return fail(SSD_E_PARAM, "pairs must be a non-NULL 8-byte aligned device pointer");
    uint64_t pass = b->pass_bytes, tile = b->tile_pairs;
    int cand = -1;
    if (b->tune_idx >= 0 && b->tune_idx < (int)b->cands.size()) {
        cand = b->tune_idx++;
        pass = b->cands[cand].pass;
        tile = b->cands[cand].tile;
    }
    // links with a large state and enough pairs take the binned scan (as a
    // separate detector would); the others share one persistent tile scan
    std::vector<uint32_t> binned;
    if (b->scan_mode != SSD_SCAN_PASSES && e->L.bin_items_words) {
        for (uint32_t l = 0; l < e->n; l++)
            if (offsets_host[l + 1] - offsets_host[l] >= BATCH_BINNED_MIN_PAIRS) binned.push_back(l);
    }
    auto is_binned = [&](uint32_t l) { return std::find(binned.begin(), binned.end(), l) != binned.end(); };
    // windows of every other link's state, ordered by address; tiles are implicit
    struct Win { uint64_t at; uint32_t link; uint64_t lo, hi; };
    std::vector<Win> wins;
    for (uint32_t l = 0; l < e->n; l++) {
        if (offsets_host[l + 1] == offsets_host[l] || is_binned(l)) continue;
        e->count_valid[l] = 0;             // the tile scan stores without counting
        const LinkDesc& D = e->hl[l];
        const uint64_t per = pass ? std::max<uint64_t>(1, pass / D.eta) : D.n_se;
        for (uint64_t lo = 0; lo < D.n_se; lo += per)
            wins.push_back({e->L.link[l].state_off + lo * D.eta, l, lo, std::min(lo + per, D.n_se)});
    }
    if (wins.size() > MAX_WINDOWS) return fail(SSD_E_PARAM, "scan pass window too small: %zu windows", wins.size());
    if (wins.empty()) cand = -1;
    std::sort(wins.begin(), wins.end(), [](const Win& a, const Win& c) { return a.at < c.at; });
    uint64_t tile_pairs_total = 0;
    for (uint32_t l = 0; l < e->n; l++)
        if (!is_binned(l)) tile_pairs_total += offsets_host[l + 1] - offsets_host[l];
    if (!wins.empty()) {
        const uint32_t buf = b->tile_next;
        b->tile_next ^= 1u;
        if (b->tile_used[buf]) HIPCHK(e, hipEventSynchronize(b->tile_done[buf]));   // its last copy has run
        unsigned long long* counter = static_cast<unsigned long long*>(b->tile_pinned[buf]);
        ScanWindow* ws = reinterpret_cast<ScanWindow*>(counter + 1);
        *counter = 0;
        uint64_t tiles = 0;
        for (size_t i = 0; i < wins.size(); i++) {
            const Win& w = wins[i];
            ScanWindow& W = ws[i];
            W.link = w.link;
            W.pad = 0;
            W.start = offsets_host[w.link];
            W.n = offsets_host[w.link + 1] - W.start;
            W.se_lo = w.lo;
            W.se_hi = w.hi;
            W.tile_base = tiles;
            W.stamp = stamp_of(e->clock, false);
            W.pad2 = 0;
            tiles += (W.n + tile - 1) / tile;
        }
        unsigned long long* dcounter = e->at<unsigned long long>(e->L.tiles);
        HIPCHK(e, hipMemcpyAsync(dcounter, counter, 8 + wins.size() * sizeof(ScanWindow), hipMemcpyHostToDevice,
                                 e->stream));
        HIPCHK(e, hipEventRecord(b->tile_done[buf], e->stream));
        b->tile_used[buf] = true;
        TileScanArgs a{};
        a.pairs = reinterpret_cast<const uint2*>(pairs_dev);
        a.links = e->dev_links();
        a.wins = reinterpret_cast<const ScanWindow*>(dcounter + 1);
        a.counter = dcounter;
        a.n_wins = (uint32_t)wins.size();
        a.n_tiles = tiles;
        a.tile = tile;
        hipEvent_t ta = nullptr, tb = nullptr;
        if (cand >= 0) {
            HIPCHK(e, hipEventCreate(&ta));
            HIPCHK(e, hipEventCreate(&tb));
            HIPCHK(e, hipEventRecord(ta, e->stream));
        }
        PhaseMark pm = phase_begin(e);
        HIPCHK(e, launch_scan_tiles(a, (uint32_t)std::min<uint64_t>(b->scan_blocks, tiles), e->stream));
        phase_end(e, pm, PHASE_SCAN_TILES, 1);
        if (cand >= 0) {
            HIPCHK(e, hipEventRecord(tb, e->stream));
            b->tune_pending.push_back({cand, tile_pairs_total});
            b->tune_events.push_back({ta, tb});
        }
    }
    if (binned.empty()) return SSD_OK;
    const uint2* pp = reinterpret_cast<const uint2*>(pairs_dev);
    if (b->bt_next < 0 || b->bt_next >= (int)b->bt_trials.size())
        return enqueue_batch_binned(b, pp, offsets_host, binned);
    // a bin-size trial: its candidate for its class (every class for the
    // global trials), the kept choices for the others; the whole binned scan
    // timed
    const int trial = b->bt_next++;
    const ssd_batch::BinTrial tr = b->bt_trials[trial];
    uint64_t pairs = 0;
    for (uint32_t l : binned) {
        const uint64_t n = offsets_host[l + 1] - offsets_host[l];
        const uint64_t key = tune_class(e->p[l], n);
        b->link_class[l] = key;
        b->bt_class_pairs[key] += n;
        pairs += n;
        int c = b->bt_global;
        const auto it = b->bt_choice.find(key);
        if (it != b->bt_choice.end()) c = it->second;
        if (tr.cls == NO_CLASS || tr.cls == key) c = tr.cand;
        e->bin_req[l] = TUNE_BIN_BYTES[c];
    }
    ssd_batch::BinTiming bt{trial, pairs, nullptr, nullptr};
    HIPCHK(e, hipEventCreate(&bt.a));
    if (hipEventCreate(&bt.b) != hipSuccess) {
        (void)hipEventDestroy(bt.a);
        return dev_fail(e, hipErrorOutOfMemory, "hipEventCreate");
    }
    b->bt_pending.push_back(bt);
    HIPCHK(e, hipEventRecord(bt.a, e->stream));
    rc = enqueue_batch_binned(b, pp, offsets_host, binned);
    if (rc) return rc;
    HIPCHK(e, hipEventRecord(bt.b, e->stream));
    return SSD_OK;
}

int ssd_batch_close_begin(ssd_batch* b)
{
    if (!b) return fail(SSD_E_PARAM, "batch is NULL");
    Engine* e = &b->e;
    int rc = usable(e);
    if (rc) return rc;
    if (b->pending) return fail(SSD_E_ORDER, "a batch close is already pending (ssd_batch_close_end first)");
    if (!b->done) HIPCHK(e, hipEventCreateWithFlags(&b->done, hipEventDisableTiming));
    rc = e->use_graph ? close_graph(e, true, 0) : enqueue_close(e, true, 0);
    if (rc) return rc;
    HIPCHK(e, hipEventRecord(b->done, e->stream));
    b->pending = true;
    e->clock++;          // the next slice opens now: its scans may be enqueued before the lists are collected
    return SSD_OK;
}

int ssd_batch_close_end(ssd_batch* b, ssd_super_point* out_host, uint64_t cap, uint64_t* counts_host,
                        int* status_host)
{
    if (!b) return fail(SSD_E_PARAM, "batch is NULL");
    Engine* e = &b->e;
    int rc = usable(e);
    if (rc) return rc;
    if (!b->pending) return fail(SSD_E_ORDER, "no batch close is pending");
    b->pending = false;
    HIPCHK(e, hipEventSynchronize(b->done));
    phase_collect(e);
    autotune_collect(b);
    rc = collect_results(e, true, 0);
    if (rc) return rc;
    return ssd_batch_get_results(b, out_host, cap, counts_host, status_host);
}

int ssd_batch_close(ssd_batch* b, ssd_super_point* out_host, uint64_t cap, uint64_t* counts_host, int* status_host)
{
    int rc = ssd_batch_close_begin(b);
    if (rc) return rc;
    return ssd_batch_close_end(b, out_host, cap, counts_host, status_host);
}

int ssd_batch_get_results(ssd_batch* b, ssd_super_point* out_host, uint64_t cap, uint64_t* counts_host,
                          int* status_host)
{
    if (!b) return fail(SSD_E_PARAM, "batch is NULL");
    if (b->pending) return fail(SSD_E_ORDER, "a batch close is pending (ssd_batch_close_end first)");
    const Engine& e = b->e;
    uint64_t total = 0;
    for (uint32_t l = 0; l < e.n; l++) {
        if (counts_host) counts_host[l] = e.results[l].size();
        if (status_host) status_host[l] = e.status[l];
        total += e.results[l].size();
    }
    if (total > cap) return fail(SSD_E_TRUNC, "result lists hold %llu entries, cap is %llu",
                                 (unsigned long long)total, (unsigned long long)cap);
    if (total && !out_host) return fail(SSD_E_PARAM, "out_host is NULL");
    uint64_t o = 0;
    for (uint32_t l = 0; l < e.n; l++) {
        if (!e.results[l].empty())
            memcpy(out_host + o, e.results[l].data(), e.results[l].size() * sizeof(ssd_super_point));
        o += e.results[l].size();
    }
    return SSD_OK;
}

int ssd_batch_read_timing(ssd_batch* b, double* ms_out, uint64_t* launches_out, int reset)
{
    if (!b) return fail(SSD_E_PARAM, "batch is NULL");
    return read_timing(&b->e, ms_out, launches_out, reset);
}

int ssd_batch_get_info(ssd_batch* b, uint32_t link, ssd_info* out)
{
    if (!b || !out) return fail(SSD_E_PARAM, "NULL argument");
    if (link >= b->e.n) return fail(SSD_E_PARAM, "link %u of %u", link, b->e.n);
    engine_info(b->e, link, out);
    return SSD_OK;
}

int ssd_batch_read_rk(ssd_batch* b, uint32_t link, uint32_t* out_host, uint64_t n)
{
    if (!b) return fail(SSD_E_PARAM, "batch is NULL");
    if (b->pending) return fail(SSD_E_ORDER, "a batch close is pending (ssd_batch_close_end first)");
    if (link >= b->e.n) return fail(SSD_E_PARAM, "link %u of %u", link, b->e.n);
    return engine_read_rk(&b->e, link, out_host, n);
}

int ssd_batch_read_hot(ssd_batch* b, uint32_t link, uint32_t* counts_host, uint32_t* lists_host, uint64_t cap)
{
    if (!b) return fail(SSD_E_PARAM, "batch is NULL");
    if (b->pending) return fail(SSD_E_ORDER, "a batch close is pending (ssd_batch_close_end first)");
    if (link >= b->e.n) return fail(SSD_E_PARAM, "link %u of %u", link, b->e.n);
    return engine_read_hot(&b->e, link, counts_host, lists_host, cap);
}

// ---- group

int ssd_group_query_sizes(uint32_t max_members, uint64_t* scratch_bytes)
{
    if (max_members < 1 || max_members > MAX_LINKS) return fail(SSD_E_PARAM, "max_members outside 1..%u", MAX_LINKS);
    if (scratch_bytes) *scratch_bytes = plan_group(max_members).total;
    return SSD_OK;
}

int ssd_group_init(uint32_t max_members, void* scratch_dev, uint64_t scratch_bytes, void* stream, ssd_group** out)
{
    if (!out) return fail(SSD_E_PARAM, "out is NULL");
    *out = nullptr;
    if (max_members < 1 || max_members > MAX_LINKS) return fail(SSD_E_PARAM, "max_members outside 1..%u", MAX_LINKS);
    const Layout L = plan_group(max_members);
    if (!scratch_dev || scratch_bytes < L.total || ((uintptr_t)scratch_dev & (ALIGN - 1)))
        return fail(SSD_E_NOMEM, "scratch buffer needs %llu bytes, 256-byte aligned", (unsigned long long)L.total);
    ssd_group* g = new (std::nothrow) ssd_group();
    if (!g) return fail(SSD_E_NOMEM, "host allocation failed");
    Engine* e = &g->e;
    g->max_members = max_members;
    e->gather_ctl = true;
    e->L = L;
    e->scratch = static_cast<uint8_t*>(scratch_dev);
    e->stream = static_cast<hipStream_t>(stream);
    e->stage_cap = BATCH_STAGE;
    hipError_t err = hipGetDevice(&e->device);
    if (err == hipSuccess)
        err = hipHostMalloc(&e->pinned, max_members * sizeof(Ctl) + BATCH_STAGE * sizeof(SuperPointDev) +
                                            (max_members + 1) * 8, hipHostMallocDefault);
    if (err != hipSuccess) {
        int rc = dev_fail(e, err, "group init");
        delete g;
        return rc;
    }
    e->mb_ctl = static_cast<Ctl*>(e->pinned);
    e->mb_stage = reinterpret_cast<SuperPointDev*>(e->mb_ctl + max_members);
    e->mb_offsets = reinterpret_cast<unsigned long long*>(e->mb_stage + BATCH_STAGE);
    for (int i = 0; i < 2 && err == hipSuccess; i++) {
        err = hipHostMalloc(&g->mb_pinned[i], multi_args_bytes(max_members), hipHostMallocDefault);
        if (err == hipSuccess) err = hipEventCreateWithFlags(&g->mb_done[i], hipEventDisableTiming);
        if (err == hipSuccess) err = hipHostMalloc(&g->tile_pinned[i], 8 + MAX_WINDOWS * sizeof(ScanWindow), hipHostMallocDefault);
        if (err == hipSuccess) err = hipEventCreateWithFlags(&g->tile_done[i], hipEventDisableTiming);
        if (err == hipSuccess) err = hipHostMalloc(&g->bind_pinned[i], group_bind_bytes(max_members), hipHostMallocDefault);
        if (err == hipSuccess) err = hipEventCreateWithFlags(&g->bind_done[i], hipEventDisableTiming);
    }
    if (err != hipSuccess) {
        int rc = dev_fail(e, err, "group staging");
        ssd_group_destroy(g);
        return rc;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, e->device) == hipSuccess) g->scan_blocks = (uint32_t)prop.multiProcessorCount * 8u;
    *out = g;
    return SSD_OK;
}

void ssd_group_destroy(ssd_group* g)
{
    if (!g) return;
    if (g->pending)     // members outlive a pending group close (see ssd_group_close_begin)
        for (ssd_detector* m : g->pending_members) m->group_pending = false;
    engine_release(&g->e);
    if (g->done) (void)hipEventDestroy(g->done);
    for (int i = 0; i < 2; i++) {
        if (g->mb_pinned[i]) (void)hipHostFree(g->mb_pinned[i]);
        if (g->mb_done[i]) (void)hipEventDestroy(g->mb_done[i]);
        if (g->tile_pinned[i]) (void)hipHostFree(g->tile_pinned[i]);
        if (g->tile_done[i]) (void)hipEventDestroy(g->tile_done[i]);
        if (g->bind_pinned[i]) (void)hipHostFree(g->bind_pinned[i]);
        if (g->bind_done[i]) (void)hipEventDestroy(g->bind_done[i]);
    }
    delete g;
}

int ssd_group_scan(ssd_group* g, ssd_detector* const* members, uint32_t n, const uint32_t* pairs_dev,
                   const uint64_t* offsets_host, const uint64_t* slice_ids_host)
{
    if (!g) return fail(SSD_E_PARAM, "group is NULL");
    Engine* e = &g->e;
    int rc = usable(e);
    if (rc) return rc;
    if (!offsets_host || !slice_ids_host) return fail(SSD_E_PARAM, "offsets or slice ids NULL");
    rc = group_bind(g, members, n);
    if (rc) return rc;
    for (uint32_t i = 0; i < n; i++) {
        if (offsets_host[i + 1] < offsets_host[i]) return fail(SSD_E_PARAM, "offsets decrease at member %u", i);
        if (slice_ids_host[i] != members[i]->e.clock)
            return fail(SSD_E_ORDER, "member %u: scan of slice %llu while slice %llu is open", i,
                        (unsigned long long)slice_ids_host[i], (unsigned long long)members[i]->e.clock);
    }
    if (offsets_host[n] == offsets_host[0]) return SSD_OK;
    if (!pairs_dev || ((uintptr_t)pairs_dev & 7u)) return fail(SSD_E_PARAM, "pairs must be a non-NULL 8-byte aligned device pointer");
    // members with at least GROUP_BINNED_MIN_PAIRS pairs in the call are
    // scanned binned, each into its own bin buffers, after the tile scan of
    // the others (as the links of a batch: XCD-local stores beat pass windows
    // for such calls whatever the state's size) -- when they were set up on
    // the group's stream, so that the group's close stays ordered after them
    auto binned = [&](uint32_t i) {
        const ssd_detector* m = members[i];
        if (m->e.stream != e->stream) return false;
        const uint64_t np = offsets_host[i + 1] - offsets_host[i];
        return m->scan_mode != SSD_SCAN_PASSES && np >= GROUP_BINNED_MIN_PAIRS;
    };
    // windows of every other member's state (its own pass window), in member order
    std::vector<ScanWindow> ws;
    uint64_t tiles = 0;
    const uint64_t tile = DEFAULT_TILE_PAIRS;
    ws.push_back({});   // slot for the counter (8 bytes) ahead of the windows
    for (uint32_t i = 0; i < n; i++) {
        const uint64_t np = offsets_host[i + 1] - offsets_host[i];
        if (!np || binned(i)) continue;
        const LinkDesc& D = e->hl[i];
        const uint64_t pass = members[i]->pass_bytes;
        const uint64_t per = pass ? std::max<uint64_t>(1, pass / D.eta) : D.n_se;
        for (uint64_t lo = 0; lo < D.n_se; lo += per) {
            ScanWindow W{};
            W.link = i;
            W.start = offsets_host[i];
            W.n = np;
            W.se_lo = lo;
            W.se_hi = std::min(lo + per, D.n_se);
            W.tile_base = tiles;
            W.stamp = stamp_of(members[i]->e.clock, false);
            tiles += (np + tile - 1) / tile;
            ws.push_back(W);
        }
    }
    const uint64_t n_wins = ws.size() - 1;
    if (n_wins > MAX_WINDOWS) return fail(SSD_E_PARAM, "too many scan windows (%llu)", (unsigned long long)n_wins);
    if (n_wins) {
        // the device block is [counter (8 bytes)][windows], copied from
        // pinned staging (the first vector entry is only a placeholder)
        const uint32_t buf = g->tile_next;
        g->tile_next ^= 1u;
        if (g->tile_used[buf]) HIPCHK(e, hipEventSynchronize(g->tile_done[buf]));   // its last copy has run
        unsigned long long* counter = static_cast<unsigned long long*>(g->tile_pinned[buf]);
        *counter = 0;
        memcpy(counter + 1, ws.data() + 1, n_wins * sizeof(ScanWindow));
        unsigned long long* dcounter = e->at<unsigned long long>(e->L.tiles);
        HIPCHK(e, hipMemcpyAsync(dcounter, counter, 8 + n_wins * sizeof(ScanWindow), hipMemcpyHostToDevice,
                                 e->stream));
        HIPCHK(e, hipEventRecord(g->tile_done[buf], e->stream));
        g->tile_used[buf] = true;
        TileScanArgs a{};
        a.pairs = reinterpret_cast<const uint2*>(pairs_dev);
        a.links = e->dev_links();
        a.wins = reinterpret_cast<const ScanWindow*>(dcounter + 1);
        a.counter = dcounter;
        a.n_wins = (uint32_t)n_wins;
        a.n_tiles = tiles;
        a.tile = tile;
        PhaseMark pm = phase_begin(e);
        HIPCHK(e, launch_scan_tiles(a, (uint32_t)std::min<uint64_t>(g->scan_blocks, tiles), e->stream));
        phase_end(e, pm, PHASE_SCAN_TILES, 1);
    }
    for (uint32_t i = 0; i < n; i++) members[i]->e.count_valid[0] = 0;   // group scans leave the counters stale
    // the binned members: rounds of one binning launch and one store launch
    // per kind over all of them, each member binning into its own staging (a
    // member whose pairs exceed its staging takes part in several rounds); a
    // member whose bins are too large for packed offsets is scanned alone.
    // A member that keeps per-slot counters takes the counted stores for a
    // large call (binned_call); its counters stay untrusted (the group's
    // close reads every member's state; the member's own close rebuilds them
    // before it counts again).
    struct Binned {
        ssd_detector* m;
        BinnedCall c;
        BinBufs bb;
        uint64_t begin, n, chunk, done;
    };
    std::vector<Binned> bm;
    for (uint32_t i = 0; i < n; i++) {
        if (!binned(i)) continue;
        ssd_detector* m = members[i];
        const uint64_t np = offsets_host[i + 1] - offsets_host[i];
        const BinnedCall c = binned_call(&m->e, 0, np, m->bin_bytes);
        if (c.bp.shift > 21) {
            rc = enqueue_binned_scan(&m->e, 0, reinterpret_cast<const uint2*>(pairs_dev) + offsets_host[i], np,
                                     m->bin_bytes, m->apply_segments, engine_bins(&m->e));
            if (rc) return rc;
            continue;
        }
        binned_count_state(&m->e, 0, c);
        const BinBufs bb = engine_bins(&m->e);
        const uint64_t max_blocks = std::min(bb.items_words / c.seg, bb.table_words / (c.bp.n_bins + 1));
        if (max_blocks == 0) return fail(SSD_E_STATE, "binned scan buffers too small");
        bm.push_back({m, c, bb, offsets_host[i], np, max_blocks * c.bp.pb, 0});
    }
    const uint64_t app_region = align_up((uint64_t)g->max_members * sizeof(BinArgs));
    const uint64_t pre_region = app_region + align_up((uint64_t)g->max_members * sizeof(ApplyArgs));
    uint8_t* dev = e->at<uint8_t>(e->L.multi_args);
    std::vector<uint32_t> round;
    std::vector<PhaseMark> pm;
    for (;;) {
        round.clear();
        for (uint32_t j = 0; j < (uint32_t)bm.size(); j++)
            if (bm[j].done < bm[j].n) round.push_back(j);
        if (round.empty()) break;
        const uint32_t cnt = (uint32_t)round.size();
        const uint32_t buf = g->mb_next;
        g->mb_next ^= 1u;
        if (g->mb_used[buf]) HIPCHK(e, hipEventSynchronize(g->mb_done[buf]));     // its last copy has run
        uint8_t* host = static_cast<uint8_t*>(g->mb_pinned[buf]);
        BinArgs* hb = reinterpret_cast<BinArgs*>(host);
        ApplyArgs* ha = reinterpret_cast<ApplyArgs*>(host + app_region);
        uint32_t* hp = reinterpret_cast<uint32_t*>(host + pre_region);    // [binning prefix][3 store prefixes]
        // the round's members by store kind: counted whose LDS lets two
        // workgroups share a compute unit (0), uncounted (1), counted needing
        // more LDS (2); a launch per kind, with its own workgroup prefix
        auto kind_of = [&](const Binned& b) -> uint32_t {
            if (!b.c.counted) return 1u;
            const LinkDesc& D = b.m->e.hl[0];
            return counted_lds_bytes(b.c.bp.shift, D.log2eta, D.k) <= COUNTED_LDS_PAIR ? 0u : 2u;
        };
        std::stable_sort(round.begin(), round.end(),
                         [&](uint32_t a, uint32_t c) { return kind_of(bm[a]) < kind_of(bm[c]); });
        uint32_t bin_wg = 0, app_wg[3] = {0, 0, 0}, kcount[3] = {0, 0, 0}, lds[3] = {0, 0, 0};
        for (uint32_t x = 0; x < cnt; x++) kcount[kind_of(bm[round[x]])]++;
        const uint32_t kfirst[3] = {0, kcount[0], kcount[0] + kcount[1]};
        for (uint32_t x = 0; x < cnt; x++) {
            Binned& b = bm[round[x]];
            const uint64_t np = std::min(b.chunk, b.n - b.done);
            BinArgs ba{};
            ApplyArgs aa{};
            binned_args(&b.m->e, 0, b.c, b.bb.items, b.bb.table, b.m->apply_segments, &ba, &aa);
            ba.pairs = reinterpret_cast<const uint2*>(pairs_dev) + b.begin + b.done;
            ba.n = np;
            ba.blocks = (uint32_t)((np + b.c.bp.pb - 1) / b.c.bp.pb);
            aa.blocks = ba.blocks;
            aa.parts = (aa.blocks + aa.per_part - 1) / aa.per_part;
            b.done += np;
            hb[x] = ba;
            ha[x] = aa;
            hp[x] = bin_wg;
            bin_wg += bin_workgroups(ba);
            const uint32_t kd = kind_of(b);
            hp[(kd + 1) * (cnt + 1) + (x - kfirst[kd])] = app_wg[kd];
            app_wg[kd] += kd == 1u ? apply_workgroups(aa) : apply_counted_workgroups(aa);
            if (kd != 1u) lds[kd] = std::max<uint32_t>(lds[kd], (uint32_t)counted_lds_bytes(aa.bin_shift, aa.log2eta, aa.k));
        }
        hp[cnt] = bin_wg;
        for (uint32_t kd = 0; kd < 3; kd++) hp[(kd + 1) * (cnt + 1) + kcount[kd]] = app_wg[kd];
        HIPCHK(e, hipMemcpyAsync(dev, host, multi_args_bytes(g->max_members), hipMemcpyHostToDevice, e->stream));
        HIPCHK(e, hipEventRecord(g->mb_done[buf], e->stream));
        g->mb_used[buf] = true;
        const uint32_t* dp = reinterpret_cast<const uint32_t*>(dev + pre_region);
        // each member's own phase timing counts the launches that scanned it
        pm.resize(cnt);
        for (uint32_t x = 0; x < cnt; x++) pm[x] = phase_begin(&bm[round[x]].m->e);
        HIPCHK(e, launch_bin_multi(MultiBinArgs{reinterpret_cast<const BinArgs*>(dev), dp, cnt}, bin_wg, e->stream));
        for (uint32_t x = 0; x < cnt; x++) phase_end(&bm[round[x]].m->e, pm[x], PHASE_SCAN_BIN, 1);
        for (uint32_t x = 0; x < cnt; x++) pm[x] = phase_begin(&bm[round[x]].m->e);
        for (uint32_t kd = 0; kd < 3; kd++) {
            if (!kcount[kd]) continue;
            const MultiApplyArgs ma{reinterpret_cast<const ApplyArgs*>(dev + app_region) + kfirst[kd],
                                    dp + (kd + 1) * (cnt + 1), kcount[kd]};
            if (kd == 1u) HIPCHK(e, launch_apply_multi(ma, app_wg[kd], e->stream));
            else HIPCHK(e, launch_apply_counted_multi(ma, app_wg[kd], lds[kd], e->stream));
        }
        for (uint32_t x = 0; x < cnt; x++) phase_end(&bm[round[x]].m->e, pm[x], 0, 1);
    }
    return SSD_OK;
}

int ssd_group_close_begin(ssd_group* g, ssd_detector* const* members, uint32_t n)
{
    if (!g) return fail(SSD_E_PARAM, "group is NULL");
    Engine* e = &g->e;
    int rc = usable(e);
    if (rc) return rc;
    if (g->pending) return fail(SSD_E_ORDER, "a group close is already pending (ssd_group_close_end first)");
    rc = group_bind(g, members, n);
    if (rc) return rc;
    for (uint32_t i = 0; i < n; i++)
        if (close_pending(members[i])) return fail(SSD_E_ORDER, "member %u has a close pending", i);
    if (!g->done) HIPCHK(e, hipEventCreateWithFlags(&g->done, hipEventDisableTiming));
    // a group's close reads every member's state (served streams' calls are
    // mostly too small to count; counted group closes measured slower) and
    // zeroes no member's next slot
    for (uint32_t i = 0; i < n; i++) {
        members[i]->e.count_valid[0] = 0;
        members[i]->e.count_rebuild[0] = 0;
    }
    rc = enqueue_close(e, true, 0);
    if (rc) return rc;
    HIPCHK(e, hipEventRecord(g->done, e->stream));
    // every member's next slice opens now: its scans may be enqueued before
    // the lists are collected
    g->pending = true;
    g->pending_members.assign(members, members + n);
    for (uint32_t i = 0; i < n; i++) {
        members[i]->group_pending = true;
        members[i]->e.clock++;
    }
    return SSD_OK;
}

int ssd_group_close_end(ssd_group* g, ssd_super_point* out_host, uint64_t cap, uint64_t* counts_host,
                        int* status_host)
{
    if (!g) return fail(SSD_E_PARAM, "group is NULL");
    Engine* e = &g->e;
    int rc = usable(e);
    if (rc) return rc;
    if (!g->pending) return fail(SSD_E_ORDER, "no group close is pending");
    g->pending = false;
    std::vector<ssd_detector*> members;
    members.swap(g->pending_members);
    const uint32_t n = (uint32_t)members.size();
    for (ssd_detector* m : members) m->group_pending = false;
    HIPCHK(e, hipEventSynchronize(g->done));
    phase_collect(e);
    // the group may have been bound to other members since the close began
    // (scans of the next slots): the close's lists are those of these members
    for (uint32_t i = 0; i < n; i++)
        if (members[i]->e.broken) return fail(SSD_E_STATE, "member %u is unusable", i);
    rc = group_bind(g, members.data(), n);
    if (rc) return rc;
    rc = collect_results(e, true, 0);
    if (rc) return rc;
    uint64_t total = 0;
    for (uint32_t i = 0; i < n; i++) {
        Engine& me = members[i]->e;
        me.results[0] = e->results[i];
        me.status[0] = e->status[i];
        me.last[0] = e->last[i];
        me.last_mode[0] = e->last_mode[i];
        me.have_last = true;
        if (counts_host) counts_host[i] = e->results[i].size();
        if (status_host) status_host[i] = e->status[i];
        total += e->results[i].size();
    }
    if (total > cap) return fail(SSD_E_TRUNC, "result lists hold %llu entries, cap is %llu",
                                 (unsigned long long)total, (unsigned long long)cap);
    if (total && !out_host) return fail(SSD_E_PARAM, "out_host is NULL");
    uint64_t o = 0;
    for (uint32_t i = 0; i < n; i++) {
        if (!e->results[i].empty())
            memcpy(out_host + o, e->results[i].data(), e->results[i].size() * sizeof(ssd_super_point));
        o += e->results[i].size();
    }
    return SSD_OK;
}

int ssd_group_close(ssd_group* g, ssd_detector* const* members, uint32_t n, ssd_super_point* out_host,
                    uint64_t cap, uint64_t* counts_host, int* status_host)
{
    int rc = ssd_group_close_begin(g, members, n);
    if (rc) return rc;
    return ssd_group_close_end(g, out_host, cap, counts_host, status_host);
}

}  // extern "C"
