// C ABI of the sliding super point detector: parameter validation, scratch
// layout, slot clock and launch sequencing.  Every step of the hot path runs
// in the kernels of kernels.hip; this file only validates, sequences and
// copies.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "ssd.h"

using namespace ssd;

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

struct Layout {
    uint64_t ctl, tables, rk, hot_list, hotbits, hotT, hot_end, ctb_x[2], ctb_h0[2], acc, sort_tmp, out, total;
    uint32_t nw;
};

constexpr uint32_t PREFIX_MAX = SORT_SMALL;   // result entries staged in pinned memory per close
// Scan pass window: random byte stores confined to 128 MiB of state stay in
// the 256 MB Infinity Cache (measured best of 64..768 MiB on the core-link
// workload; one pass when the state is smaller).
constexpr uint64_t DEFAULT_PASS_BYTES = 128ull << 20;

int validate(const ssd_params* p)
{
    if (!p) return fail(SSD_E_PARAM, "params is NULL");
    if (p->abi_version != SSD_ABI_VERSION) return fail(SSD_E_PARAM, "abi_version %u != %u", p->abi_version, SSD_ABI_VERSION);
    if (p->r < 3 || p->r > MAX_ROWS) return fail(SSD_E_PARAM, "r=%u outside 3..%u", p->r, MAX_ROWS);
    if (p->q < 4 || p->q > 20) return fail(SSD_E_PARAM, "q=%u outside 4..20", p->q);
    if (p->delta < 1 || p->delta >= p->q || p->delta > 12) return fail(SSD_E_PARAM, "delta=%u must satisfy 1 <= delta < q, delta <= 12", p->delta);
    if (!is_pow2(p->eta) || p->eta < 1024 || p->eta > 65536) return fail(SSD_E_PARAM, "eta=%u must be a power of two in 1024..65536", p->eta);
    if (p->k < 1 || p->k > 254) return fail(SSD_E_PARAM, "k=%u outside 1..254", p->k);
    if (p->theta < 1) return fail(SSD_E_PARAM, "theta must be >= 1");
    if (p->key_bits < 8 || p->key_bits > 32) return fail(SSD_E_PARAM, "key_bits=%u outside 8..32", p->key_bits);
    const uint32_t cover = (p->r - 2) * p->delta + p->q;
    if (cover < p->key_bits) return fail(SSD_E_PARAM, "(r-2)*delta+q=%u does not cover key_bits=%u", cover, p->key_bits);
    if (cover > 64) return fail(SSD_E_PARAM, "(r-2)*delta+q=%u exceeds 64", cover);
    if (p->flags & ~SSD_VERIFY_REHASH) return fail(SSD_E_PARAM, "unknown flags 0x%x", p->flags);
    if (p->reserved) return fail(SSD_E_PARAM, "reserved must be 0");
    if (p->max_tuples < 1 || p->max_tuples > (1ull << 32)) return fail(SSD_E_PARAM, "max_tuples outside 1..2^32");
    if (p->max_results < 1 || p->max_results > (1ull << 28)) return fail(SSD_E_PARAM, "max_results outside 1..2^28");
    return SSD_OK;
}

Layout layout(const ssd_params* p)
{
    Layout L{};
    const uint64_t n_se = (uint64_t)p->r << p->q;
    L.nw = p->delta > 6 ? 1u << (p->delta - 6) : 1u;
    uint64_t o = 0;
    L.ctl = o; o = align_up(o + sizeof(Ctl));
    L.tables = o; o = align_up(o + 2048 * 4);
    L.rk = o; o = align_up(o + n_se * 4);
    L.hot_list = o; o = align_up(o + n_se * 4);
    // hotbits and hotT are adjacent: one fill clears both before every close
    L.hotbits = o; o = o + (uint64_t)p->r * (p->q >= 6 ? (1ull << (p->q - 6)) : 1ull) * 8;
    L.hotT = o; o = o + (uint64_t)p->r * (1ull << (p->q - p->delta)) * L.nw * 8;
    L.hot_end = o; o = align_up(o);
    for (int b = 0; b < 2; b++) { L.ctb_x[b] = o; o = align_up(o + p->max_tuples * 8); }
    for (int b = 0; b < 2; b++) { L.ctb_h0[b] = o; o = align_up(o + p->max_tuples * 4); }
    L.acc = o; o = align_up(o + p->max_results * 8);
    uint64_t pw = 1;
    while (pw < p->max_results) pw <<= 1;
    L.sort_tmp = o; o = align_up(o + pw * 8);
    L.out = o; o = align_up(o + p->max_results * sizeof(SuperPointDev));
    L.total = o;
    return L;
}

uint32_t hot_threshold(uint32_t eta, uint32_t theta)
{
    // Sec. 3.3: R_k >= eta * (1 - e^(-theta/eta)), rounded up once
    return (uint32_t)ceil((double)eta * (1.0 - exp(-(double)theta / (double)eta)));
}

uint32_t stamp_of(uint64_t t) { return 1u + (uint32_t)(t % 255u); }

LiveCfg live_cfg(uint64_t t, uint32_t k)
{
    const uint32_t cur = stamp_of(t);
    uint32_t lo, kp, wrap;
    if (cur >= k) { lo = cur - k + 1; kp = k; wrap = 0; }
    else { lo = cur + 256 - k; kp = k + 1; wrap = 1; }
    LiveCfg c;
    c.c1 = (256u - lo) * 0x00010001u;
    c.c2 = (256u - kp) * 0x00010001u;
    c.wrap = wrap;
    return c;
}

}  // namespace

struct ssd_detector {
    ssd_params p;
    Layout L;
    uint32_t T, log2eta;
    uint64_t clock;
    uint8_t* state;
    uint8_t* scratch;
    hipStream_t stream;
    int device;
    bool broken;
    uint64_t pass_bytes;
    uint64_t sort_block_limit;
    uint32_t tables_host[2048];
    Ctl* mailbox;                       // pinned host copy of the control block
    std::vector<ssd_super_point> results;
    std::vector<SuperPointDev> staging;
    Ctl last;                           // control block of the last close
    bool have_last;
    uint64_t last_reported;             // list length of the last close (sizes the staged prefix)
    // phase timing with HIP events (opt-in)
    bool timing;
    std::vector<hipEvent_t> ev_pool;
    std::vector<uint32_t> ev_free;
    struct Pending { uint32_t a, b, phase, launches; };
    std::vector<Pending> pending;
    double ph_ms[SSD_PHASES];
    uint64_t ph_launches[SSD_PHASES];

    template <class T> T* at(uint64_t off) const { return reinterpret_cast<T*>(scratch + off); }
    uint64_t n_se() const { return (uint64_t)p.r << p.q; }
    uint64_t state_bytes() const { return n_se() << log2eta; }
    uint32_t expire_period() const { return 255u - p.k; }
};

namespace {

int dev_fail(ssd_detector* d, hipError_t e, const char* what)
{
    if (d) d->broken = true;
    return fail(SSD_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(d, call)                                          \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return dev_fail((d), e_, #call);   \
    } while (0)

// ---- phase timing: a start/stop event pair around each phase's launches
uint32_t ev_get(ssd_detector* d)
{
    if (!d->ev_free.empty()) {
        uint32_t i = d->ev_free.back();
        d->ev_free.pop_back();
        return i;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return UINT32_MAX;
    d->ev_pool.push_back(e);
    return (uint32_t)d->ev_pool.size() - 1;
}

struct PhaseMark {
    uint32_t a = UINT32_MAX;
};

PhaseMark phase_begin(ssd_detector* d)
{
    PhaseMark m;
    if (!d->timing) return m;
    m.a = ev_get(d);
    if (m.a != UINT32_MAX && hipEventRecord(d->ev_pool[m.a], d->stream) != hipSuccess) {
        d->ev_free.push_back(m.a);
        m.a = UINT32_MAX;
    }
    return m;
}

void phase_end(ssd_detector* d, PhaseMark m, uint32_t phase, uint32_t launches)
{
    if (!d->timing || m.a == UINT32_MAX) return;
    uint32_t b = ev_get(d);
    if (b == UINT32_MAX) { d->ev_free.push_back(m.a); return; }
    if (hipEventRecord(d->ev_pool[b], d->stream) != hipSuccess) {
        d->ev_free.push_back(m.a);
        d->ev_free.push_back(b);
        return;
    }
    d->pending.push_back({m.a, b, phase, launches});
}

// after the stream passed every pending stop event
void phase_collect(ssd_detector* d)
{
    for (const auto& p : d->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, d->ev_pool[p.a], d->ev_pool[p.b]) == hipSuccess) {
            d->ph_ms[p.phase] += ms;
            d->ph_launches[p.phase] += p.launches;
        }
        d->ev_free.push_back(p.a);
        d->ev_free.push_back(p.b);
    }
    d->pending.clear();
}

int usable(ssd_detector* d)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    if (d->broken) return fail(SSD_E_STATE, "detector unusable after an earlier device error");
    hipError_t e = hipSetDevice(d->device);
    if (e != hipSuccess) return dev_fail(d, e, "hipSetDevice");
    return SSD_OK;
}

// Rotating expiry: estimators with index = t (mod 255-k) clear their dead
// cells at this close, so a cell is cleared at most 254-k slots after it
// left the window and stamps never wrap onto a live value.
DetectArgs detect_args(const ssd_detector* d, bool count)
{
    DetectArgs a{};
    a.state = d->state;
    a.rk = d->at<uint32_t>(d->L.rk);
    a.hotbits = d->at<uint64_t>(d->L.hotbits);
    a.hotT = d->at<uint64_t>(d->L.hotT);
    a.q = d->p.q;
    a.delta = d->p.delta;
    a.nw = d->L.nw;
    a.T = d->T;
    a.log2eta = d->log2eta;
    a.chunks = d->p.eta / 16u;
    a.count = count ? 1u : 0u;
    a.expire_period = d->expire_period();
    a.expire_phase = (uint32_t)(d->clock % a.expire_period);
    a.L = live_cfg(d->clock, d->p.k);
    if (count) {
        a.n_waves = d->n_se();
        a.se_base = 0;
        a.se_step = 1;
    } else {
        const uint64_t n = d->n_se();
        a.se_base = a.expire_phase;
        a.se_step = a.expire_period;
        a.n_waves = a.se_base < n ? (n - a.se_base + a.se_step - 1) / a.se_step : 0;
    }
    return a;
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

int ssd_query_sizes(const ssd_params* p, uint64_t* state_bytes, uint64_t* scratch_bytes)
{
    int rc = validate(p);
    if (rc) return rc;
    if (state_bytes) *state_bytes = ((uint64_t)p->r << p->q) * p->eta;
    if (scratch_bytes) *scratch_bytes = layout(p).total;
    return SSD_OK;
}

int ssd_init_detector(const ssd_params* p, const uint32_t* tables_host, void* state_dev, uint64_t state_bytes,
                      void* scratch_dev, uint64_t scratch_bytes, void* stream, ssd_detector** out)
{
    if (!out) return fail(SSD_E_PARAM, "out is NULL");
    *out = nullptr;
    int rc = validate(p);
    if (rc) return rc;
    if (!tables_host) return fail(SSD_E_PARAM, "tables_host is NULL");
    const Layout L = layout(p);
    const uint64_t need_state = ((uint64_t)p->r << p->q) * p->eta;
    if (!state_dev || state_bytes < need_state || ((uintptr_t)state_dev & 15u))
        return fail(SSD_E_NOMEM, "state buffer needs %llu bytes, 16-byte aligned", (unsigned long long)need_state);
    if (!scratch_dev || scratch_bytes < L.total || ((uintptr_t)scratch_dev & (ALIGN - 1)))
        return fail(SSD_E_NOMEM, "scratch buffer needs %llu bytes, 256-byte aligned", (unsigned long long)L.total);
    ssd_detector* d = new (std::nothrow) ssd_detector();
    if (!d) return fail(SSD_E_NOMEM, "host allocation failed");
    d->p = *p;
    d->L = L;
    d->T = hot_threshold(p->eta, p->theta);
    d->log2eta = log2u(p->eta);
    d->clock = 0;
    d->state = static_cast<uint8_t*>(state_dev);
    d->scratch = static_cast<uint8_t*>(scratch_dev);
    d->stream = static_cast<hipStream_t>(stream);
    d->broken = false;
    d->pass_bytes = DEFAULT_PASS_BYTES;
    d->sort_block_limit = SORT_SMALL;
    d->have_last = false;
    d->last_reported = 0;
    d->timing = false;
    for (uint32_t i = 0; i < SSD_PHASES; i++) { d->ph_ms[i] = 0; d->ph_launches[i] = 0; }
    memcpy(d->tables_host, tables_host, sizeof d->tables_host);
    hipError_t e = hipGetDevice(&d->device);
    if (e != hipSuccess) { rc = dev_fail(d, e, "hipGetDevice"); delete d; return rc; }
    e = hipHostMalloc((void**)&d->mailbox, sizeof(Ctl) + PREFIX_MAX * sizeof(SuperPointDev), hipHostMallocDefault);
    if (e != hipSuccess) { rc = dev_fail(d, e, "hipHostMalloc"); delete d; return rc; }
    uint32_t* tab_stage = reinterpret_cast<uint32_t*>(d->mailbox + 1);   // 8 KiB fits the prefix area
    memcpy(tab_stage, tables_host, 2048 * 4);
    // every cell starts empty (Sec. 3.2: initialised once)
    e = launch_fill_u32(reinterpret_cast<uint32_t*>(d->state), need_state / 4, 0u, d->stream);
    if (e == hipSuccess) e = launch_fill_u32(d->at<uint32_t>(0), L.total / 4, 0u, d->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d->at<uint32_t>(L.tables), tab_stage, 2048 * 4, hipMemcpyHostToDevice, d->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(d->stream);
    if (e != hipSuccess) { rc = dev_fail(d, e, "init"); (void)hipHostFree(d->mailbox); delete d; return rc; }
    *out = d;
    return SSD_OK;
}

void ssd_destroy(ssd_detector* d)
{
    if (!d) return;
    (void)hipSetDevice(d->device);
    if (!d->broken) (void)hipStreamSynchronize(d->stream);
    if (d->mailbox) (void)hipHostFree(d->mailbox);
    for (hipEvent_t e : d->ev_pool) (void)hipEventDestroy(e);
    delete d;
}

int ssd_set_tuning(ssd_detector* d, uint32_t knob, uint64_t value)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    switch (knob) {
    case SSD_TUNE_SCAN_PASS_BYTES: d->pass_bytes = value; return SSD_OK;
    case SSD_TUNE_TIMING: d->timing = value != 0; return SSD_OK;
    case SSD_TUNE_SORT_BLOCK_LIMIT:
        if (value > SORT_SMALL) return fail(SSD_E_PARAM, "sort block limit above %u", SORT_SMALL);
        d->sort_block_limit = value;
        return SSD_OK;
    default: return fail(SSD_E_PARAM, "unknown tuning knob %u", knob);
    }
}

int ssd_scan_slice(ssd_detector* d, const uint32_t* pairs_dev, uint64_t n, uint64_t slice_id)
{
    int rc = usable(d);
    if (rc) return rc;
    if (slice_id != d->clock)
        return fail(SSD_E_ORDER, "scan of slice %llu while slice %llu is open", (unsigned long long)slice_id,
                    (unsigned long long)d->clock);
    if (n == 0) return SSD_OK;
    if (!pairs_dev || ((uintptr_t)pairs_dev & 7u)) return fail(SSD_E_PARAM, "pairs must be a non-NULL 8-byte aligned device pointer");
    ScanArgs a{};
    a.pairs = reinterpret_cast<const uint2*>(pairs_dev);
    a.n = n;
    a.state = d->state;
    a.tables = d->at<uint32_t>(d->L.tables);
    a.q = d->p.q;
    a.r = d->p.r;
    a.delta = d->p.delta;
    a.log2eta = d->log2eta;
    a.stamp = stamp_of(d->clock);
    // passes over estimator windows of about pass_bytes each
    const uint64_t n_se = d->n_se();
    const uint64_t se_bytes = d->p.eta;
    uint64_t per_pass = n_se;
    if (d->pass_bytes) {
        per_pass = d->pass_bytes / se_bytes;
        if (per_pass < 1) per_pass = 1;
    }
    PhaseMark pm = phase_begin(d);
    uint32_t launches = 0;
    for (uint64_t lo = 0; lo < n_se; lo += per_pass) {
        a.se_lo = lo;
        a.se_hi = lo + per_pass < n_se ? lo + per_pass : n_se;
        HIPCHK(d, launch_scan(a, d->stream));
        launches++;
    }
    phase_end(d, pm, 0, launches);
    return SSD_OK;
}

int ssd_close_slice(ssd_detector* d, uint32_t flags, ssd_super_point* out_host, uint64_t cap, uint64_t* n_out)
{
    int rc = usable(d);
    if (rc) return rc;
    if (flags & ~SSD_ADVANCE_ONLY) return fail(SSD_E_PARAM, "unknown close flags 0x%x", flags);
    if (n_out) *n_out = 0;
    const ssd_params& p = d->p;
    if (flags & SSD_ADVANCE_ONLY) {
        DetectArgs da = detect_args(d, false);
        if (da.n_waves) HIPCHK(d, launch_hot_detect(da, d->stream));
        d->clock++;
        d->results.clear();
        d->have_last = false;
        return SSD_OK;
    }
    const hipStream_t s = d->stream;
    Ctl* ctl = d->at<Ctl>(d->L.ctl);
    // 1. R_k of every estimator, hot bits, rotating expiry
    HIPCHK(d, launch_fill_u32(d->at<uint32_t>(d->L.hotbits), (d->L.hot_end - d->L.hotbits) / 4, 0u, s));
    DetectArgs da = detect_args(d, true);
    PhaseMark pm = phase_begin(d);
    HIPCHK(d, launch_hot_detect(da, s));
    phase_end(d, pm, 1, 1);
    // 2. ascending hot lists
    CompactArgs ca{};
    ca.hotbits = d->at<uint64_t>(d->L.hotbits);
    ca.hot_list = d->at<uint32_t>(d->L.hot_list);
    ca.ctl = ctl;
    ca.q = p.q;
    pm = phase_begin(d);
    HIPCHK(d, launch_hot_compact(ca, p.r, s));
    phase_end(d, pm, 2, 1);
    // 3. candidate levels: rows 0..2, then one row per level
    ExpandArgs ea{};
    ea.hot_list = ca.hot_list;
    ea.hotT = d->at<uint64_t>(d->L.hotT);
    ea.ctl = ctl;
    ea.cap = p.max_tuples;
    ea.q = p.q; ea.delta = p.delta; ea.nw = d->L.nw; ea.key_bits = p.key_bits;
    ea.row = 2;
    ea.out_x = d->at<uint64_t>(d->L.ctb_x[0]);
    ea.out_h0 = d->at<uint32_t>(d->L.ctb_h0[0]);
    pm = phase_begin(d);
    HIPCHK(d, launch_expand0(ea, s));
    for (uint32_t row = 3; row < p.r; row++) {
        const uint32_t lvl = row - 2;
        ea.row = row;
        ea.in_x = d->at<uint64_t>(d->L.ctb_x[(lvl - 1) & 1]);
        ea.in_h0 = d->at<uint32_t>(d->L.ctb_h0[(lvl - 1) & 1]);
        ea.out_x = d->at<uint64_t>(d->L.ctb_x[lvl & 1]);
        ea.out_h0 = d->at<uint32_t>(d->L.ctb_h0[lvl & 1]);
        HIPCHK(d, launch_extend(ea, s));
    }
    phase_end(d, pm, 3, p.r - 2);
    // 4. final test of every full tuple
    const uint32_t lf = p.r - 3;
    VerifyArgs va{};
    va.state = d->state;
    va.tables = d->at<uint32_t>(d->L.tables);
    va.ctl = ctl;
    va.in_x = d->at<uint64_t>(d->L.ctb_x[lf & 1]);
    va.in_h0 = d->at<uint32_t>(d->L.ctb_h0[lf & 1]);
    va.acc = d->at<unsigned long long>(d->L.acc);
    va.cap = p.max_tuples;
    va.max_results = p.max_results;
    va.q = p.q; va.r = p.r; va.delta = p.delta; va.log2eta = d->log2eta;
    va.chunks = p.eta / 16u; va.T = d->T; va.level = lf;
    va.rehash = (p.flags & SSD_VERIFY_REHASH) ? 1u : 0u;
    va.L = da.L;
    pm = phase_begin(d);
    HIPCHK(d, launch_verify(va, s));
    phase_end(d, pm, 4, 1);
    // 5. sort by ip, keep the largest R per ip, estimate (Eq. 1) -- in one
    // block when the list is short; the control block and a prefix of the
    // list come back with a single synchronisation
    ReportArgs ra{};
    ra.keys = d->at<unsigned long long>(d->L.acc);
    ra.out = d->at<SuperPointDev>(d->L.out);
    ra.ctl = ctl;
    ra.eta = p.eta;
    ra.limit = d->sort_block_limit < p.max_results ? d->sort_block_limit : p.max_results;
    pm = phase_begin(d);
    HIPCHK(d, launch_sort_small(ra, s));
    phase_end(d, pm, 5, 1);
    uint64_t prefix = 2 * d->last_reported + 64;
    if (prefix > PREFIX_MAX) prefix = PREFIX_MAX;
    if (prefix > p.max_results) prefix = p.max_results;
    SuperPointDev* stage = reinterpret_cast<SuperPointDev*>(d->mailbox + 1);
    HIPCHK(d, hipMemcpyAsync(d->mailbox, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIPCHK(d, hipMemcpyAsync(stage, ra.out, prefix * sizeof(SuperPointDev), hipMemcpyDeviceToHost, s));
    HIPCHK(d, hipStreamSynchronize(s));
    phase_collect(d);
    Ctl c = *d->mailbox;
    d->clock++;
    d->last = c;
    d->have_last = true;
    d->results.clear();
    for (uint32_t l = 0; l <= lf; l++)
        if (c.level_n[l] > p.max_tuples) {
            d->last_reported = 0;
            return fail(SSD_E_OVERFLOW, "candidate level %u holds %llu tuples > max_tuples %llu", l,
                        (unsigned long long)c.level_n[l], (unsigned long long)p.max_tuples);
        }
    if (c.n_acc > p.max_results) {
        d->last_reported = 0;
        return fail(SSD_E_OVERFLOW, "%llu accepted hosts > max_results %llu", (unsigned long long)c.n_acc,
                    (unsigned long long)p.max_results);
    }
    const SuperPointDev* src = stage;
    if (c.n_acc > ra.limit) {
        // long list: multi-kernel sort, then the whole list
        pm = phase_begin(d);
        HIPCHK(d, launch_sort_large(ra, d->at<unsigned long long>(d->L.sort_tmp), c.n_acc, s));
        phase_end(d, pm, 5, 1);
        d->staging.resize(c.n_acc);
        HIPCHK(d, hipMemcpyAsync(d->mailbox, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIPCHK(d, hipMemcpyAsync(d->staging.data(), ra.out, c.n_acc * sizeof(SuperPointDev), hipMemcpyDeviceToHost, s));
        HIPCHK(d, hipStreamSynchronize(s));
        phase_collect(d);
        c.n_out = d->mailbox->n_out;
        src = d->staging.data();
    } else if (c.n_out > prefix) {
        d->staging.resize(c.n_out);
        HIPCHK(d, hipMemcpyAsync(d->staging.data(), ra.out, c.n_out * sizeof(SuperPointDev), hipMemcpyDeviceToHost, s));
        HIPCHK(d, hipStreamSynchronize(s));
        src = d->staging.data();
    }
    const uint64_t m = c.n_out;
    d->last.n_out = m;
    d->last_reported = m;
    d->results.resize(m);
    for (uint64_t i = 0; i < m; i++) {
        d->results[i].ip = src[i].ip;
        d->results[i].rk = src[i].rk;
        d->results[i].est = src[i].est;
    }
    return ssd_get_results(d, out_host, cap, n_out);
}

int ssd_get_results(ssd_detector* d, ssd_super_point* out_host, uint64_t cap, uint64_t* n_out)
{
    if (!d) return fail(SSD_E_PARAM, "detector is NULL");
    const uint64_t m = d->results.size();
    if (n_out) *n_out = m;
    if (m > cap) return fail(SSD_E_TRUNC, "result list holds %llu entries, cap is %llu", (unsigned long long)m,
                             (unsigned long long)cap);
    if (m && !out_host) return fail(SSD_E_PARAM, "out_host is NULL");
    if (m) memcpy(out_host, d->results.data(), m * sizeof(ssd_super_point));
    return SSD_OK;
}

int ssd_merge_router_state(ssd_detector* g, ssd_detector* const* routers, uint32_t n)
{
    int rc = usable(g);
    if (rc) return rc;
    if (!routers || n < 1) return fail(SSD_E_PARAM, "need at least one router");
    for (uint32_t j = 0; j < n; j++) {
        const ssd_detector* r = routers[j];
        if (!r) return fail(SSD_E_PARAM, "router %u is NULL", j);
        if (r == g) return fail(SSD_E_PARAM, "router %u is the global detector", j);
        if (r->broken) return fail(SSD_E_STATE, "router %u is unusable", j);
        if (r->p.q != g->p.q || r->p.r != g->p.r || r->p.delta != g->p.delta || r->p.eta != g->p.eta ||
            r->p.k != g->p.k || r->p.key_bits != g->p.key_bits ||
            memcmp(r->tables_host, g->tables_host, sizeof g->tables_host) != 0)
            return fail(SSD_E_INCOMPAT, "router %u differs in geometry or hash tables", j);
        if (r->clock != g->clock) return fail(SSD_E_INCOMPAT, "router %u is at slice %llu, global at %llu", j,
                                              (unsigned long long)r->clock, (unsigned long long)g->clock);
        if (r->device != g->device) return fail(SSD_E_INCOMPAT, "router %u is on another device", j);
    }
    MergeArgs a{};
    a.dst = g->state;
    a.n16 = g->state_bytes() / 16u;
    a.cur = stamp_of(g->clock);
    a.k = g->p.k;
    // associative merge in batches; later batches fold the partial result in
    uint32_t done = 0, launches = 0;
    PhaseMark pm = phase_begin(g);
    while (done < n) {
        uint32_t m = 0;
        if (done > 0) a.src[m++] = g->state;
        while (m < MAX_MERGE_SOURCES && done < n) a.src[m++] = routers[done++]->state;
        a.n_src = m;
        HIPCHK(g, launch_merge(a, g->stream));
        launches++;
    }
    phase_end(g, pm, 6, launches);
    return SSD_OK;
}

int ssd_read_canonical_state(ssd_detector* d, uint16_t* out_dev, uint64_t n_cells)
{
    int rc = usable(d);
    if (rc) return rc;
    const uint64_t n = d->state_bytes();
    if (!out_dev || n_cells < n) return fail(SSD_E_NOMEM, "canonical state needs %llu cells", (unsigned long long)n);
    HIPCHK(d, launch_canonical(d->state, out_dev, n, stamp_of(d->clock), d->p.k, d->stream));
    HIPCHK(d, hipStreamSynchronize(d->stream));
    return SSD_OK;
}

int ssd_read_rk(ssd_detector* d, uint32_t* out_host, uint64_t n)
{
    int rc = usable(d);
    if (rc) return rc;
    if (!d->have_last) return fail(SSD_E_STATE, "no reconstructing close yet");
    if (!out_host || n < d->n_se()) return fail(SSD_E_NOMEM, "R_k needs %llu entries", (unsigned long long)d->n_se());
    HIPCHK(d, hipMemcpyAsync(out_host, d->at<uint32_t>(d->L.rk), d->n_se() * 4, hipMemcpyDeviceToHost, d->stream));
    HIPCHK(d, hipStreamSynchronize(d->stream));
    return SSD_OK;
}

int ssd_read_hot(ssd_detector* d, uint32_t* counts_host, uint32_t* lists_host, uint64_t cap)
{
    int rc = usable(d);
    if (rc) return rc;
    if (!d->have_last) return fail(SSD_E_STATE, "no reconstructing close yet");
    if (!counts_host) return fail(SSD_E_PARAM, "counts_host is NULL");
    uint64_t total = 0;
    for (uint32_t i = 0; i < d->p.r; i++) { counts_host[i] = d->last.hot_n[i]; total += d->last.hot_n[i]; }
    if (total > cap || (total && !lists_host)) return fail(SSD_E_TRUNC, "hot lists need %llu entries", (unsigned long long)total);
    uint64_t o = 0;
    for (uint32_t i = 0; i < d->p.r; i++) {
        if (d->last.hot_n[i])
            HIPCHK(d, hipMemcpyAsync(lists_host + o, d->at<uint32_t>(d->L.hot_list) + ((uint64_t)i << d->p.q),
                                     (uint64_t)d->last.hot_n[i] * 4, hipMemcpyDeviceToHost, d->stream));
        o += d->last.hot_n[i];
    }
    HIPCHK(d, hipStreamSynchronize(d->stream));
    return SSD_OK;
}

int ssd_read_tuples(ssd_detector* d, uint32_t* out_host, uint64_t cap, uint64_t* n_out)
{
    int rc = usable(d);
    if (rc) return rc;
    if (!d->have_last) return fail(SSD_E_STATE, "no reconstructing close yet");
    const uint32_t lf = d->p.r - 3;
    uint64_t n = d->last.level_n[lf];
    if (n > d->p.max_tuples) return fail(SSD_E_OVERFLOW, "the last close overflowed");
    if (n_out) *n_out = n;
    if (n > cap) return fail(SSD_E_TRUNC, "%llu tuples, cap %llu", (unsigned long long)n, (unsigned long long)cap);
    if (!n) return SSD_OK;
    if (!out_host) return fail(SSD_E_PARAM, "out_host is NULL");
    std::vector<uint64_t> x(n);
    std::vector<uint32_t> h0(n);
    HIPCHK(d, hipMemcpyAsync(x.data(), d->at<uint64_t>(d->L.ctb_x[lf & 1]), n * 8, hipMemcpyDeviceToHost, d->stream));
    HIPCHK(d, hipMemcpyAsync(h0.data(), d->at<uint32_t>(d->L.ctb_h0[lf & 1]), n * 4, hipMemcpyDeviceToHost, d->stream));
    HIPCHK(d, hipStreamSynchronize(d->stream));
    // inspection only: expand the stored (he_0, regained bits) form to one column per row
    const uint32_t qmask = (1u << d->p.q) - 1u;
    for (uint64_t t = 0; t < n; t++) {
        uint32_t* o = out_host + t * d->p.r;
        o[0] = h0[t];
        for (uint32_t i = 1; i < d->p.r; i++) o[i] = ((uint32_t)(x[t] >> ((i - 1) * d->p.delta)) & qmask) ^ h0[t];
    }
    return SSD_OK;
}

int ssd_read_timing(ssd_detector* d, double* ms_out, uint64_t* launches_out, int reset)
{
    int rc = usable(d);
    if (rc) return rc;
    HIPCHK(d, hipStreamSynchronize(d->stream));
    phase_collect(d);
    for (uint32_t i = 0; i < SSD_PHASES; i++) {
        if (ms_out) ms_out[i] = d->ph_ms[i];
        if (launches_out) launches_out[i] = d->ph_launches[i];
        if (reset) { d->ph_ms[i] = 0; d->ph_launches[i] = 0; }
    }
    return SSD_OK;
}

int ssd_get_info(ssd_detector* d, ssd_info* out)
{
    if (!d || !out) return fail(SSD_E_PARAM, "NULL argument");
    memset(out, 0, sizeof *out);
    out->open_slice = d->clock;
    out->hot_threshold = d->T;
    out->r = d->p.r;
    out->state_bytes = d->state_bytes();
    if (d->have_last) {
        for (uint32_t i = 0; i < MAX_ROWS; i++) {
            out->level_counts[i] = d->last.level_n[i];
            out->hot_counts[i] = d->last.hot_n[i];
        }
        out->accepted = d->last.n_acc;
        out->reported = d->last.n_out;
    }
    return SSD_OK;
}

}  // extern "C"
