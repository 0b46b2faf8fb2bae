/*
 * ssd.h -- C ABI of the MI355X sliding super point detector.
 *
 * The method is the one of "Regain Sliding super point from distributed edge
 * routers by GPU" (Jie Xu, 2018): a reversible sliding estimator array (RSEA,
 * Sec. 3.3) of r rows x 2^q sliding estimators (Sec. 3.2) of eta cells each,
 * updated by every (cip, oip) pair (Alg. 2) and inverted at the end of every
 * slot to regain the hosts whose opposite number over the last k slots is at
 * least theta (Def. 4, Alg. 3/4, parallel form Sec. 4.2), with per-router
 * arrays merged per slot in the distributed deployment (Alg. 5).
 *
 * Conventions shared by every call:
 *   - Every call returns an int status: SSD_OK (0) or a negative SSD_E_* code.
 *     No C++ exception crosses the ABI.  ssd_last_error() gives a message for
 *     the last failing call on the calling thread.
 *   - Device memory and the HIP stream belong to the caller.  The library owns
 *     only the opaque host object (and a small pinned host mailbox inside it).
 *     Device pointers must stay valid until ssd_destroy().
 *   - Work is enqueued on the caller's stream.  ssd_scan_slice() is
 *     asynchronous; ssd_close_slice() returns after the results reached host
 *     memory.  A detector is not thread-safe; separate detectors are
 *     independent.
 *   - IPv4 addresses are host-order uint32 (a.b.c.d = a<<24|b<<16|c<<8|d).
 *   - SSD_E_DEVICE means a HIP call failed; the detector then refuses further
 *     work (SSD_E_STATE) and must be destroyed.
 */
#ifndef SSD_H
#define SSD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSD_ABI_VERSION 1u

#define SSD_OK 0
#define SSD_E_PARAM (-1)    /* invalid parameter or argument                       */
#define SSD_E_NOMEM (-2)    /* a caller buffer is too small or misaligned          */
#define SSD_E_ORDER (-3)    /* slice_id is not the open slice                       */
#define SSD_E_OVERFLOW (-4) /* a candidate level exceeded max_tuples, or accepted
                               hosts exceeded max_results; no list is returned      */
#define SSD_E_INCOMPAT (-5) /* merged detectors differ in geometry, tables or clock */
#define SSD_E_TRUNC (-6)    /* the output array is too small; *n_out = needed size  */
#define SSD_E_DEVICE (-7)   /* a HIP call failed                                    */
#define SSD_E_STATE (-8)    /* the detector is unusable after an earlier failure    */

/* ssd_params.flags */
#define SSD_VERIFY_REHASH 0x1u /* drop a regained host x unless RHFG[0](x) equals the
                                  tuple's row-0 column (off = the paper's method)   */
/* ssd_close_slice() flags */
#define SSD_ADVANCE_ONLY 0x1u  /* only advance the slot clock (router detectors)    */

/*
 * Detector geometry and limits.
 *   q, r, delta: RSEA of r rows x 2^q columns; RHFG[i](cip) =
 *       ((cip >> ((i-1)*delta)) XOR RHFG[0](cip)) mod 2^q for i >= 1 (Eq. 2,
 *       read with a (i-1)*delta shift so that the hashes are invertible).
 *       3 <= r <= 16, 4 <= q <= 20, 1 <= delta < q, delta <= 12,
 *       key_bits <= (r-2)*delta + q <= 64.
 *   eta: cells per sliding estimator, a power of two, 1024..65536 (Sec. 3.2).
 *   k: window length in slots: 1..254 with 8-bit cells, 1..65534 with 16-bit
 *       cells (the paper's 16-bit distance recorders allow k < 65535,
 *       Sec. 3.2).
 *   cell_bits: 8 (or 0) or 16, the width of a cell's slot stamp.  8-bit
 *       cells halve the state; windows above 254 slots need 16-bit cells.
 *       Detectors with 16-bit cells scan with pass windows or binned stores
 *       and read the whole state at hot detection (no per-slot counters);
 *       batches and groups take 8-bit cells only (SSD_E_PARAM).
 *   theta: super point threshold on the opposite number (Def. 2), >= 1.  An
 *       estimator is hot when its in-window cell count reaches
 *       T = ceil(eta * (1 - exp(-theta/eta))) (Sec. 3.3).
 *   key_bits: host address width, 8..32 (32 for IPv4).  Regained values with
 *       a bit at or above key_bits are dropped.
 *   flags: SSD_VERIFY_REHASH or 0.
 *   max_tuples: capacity of each candidate-tuple level (Sec. 4.2 buffers).
 *   max_results: capacity for accepted hosts before de-duplication.
 */
typedef struct {
    uint32_t abi_version; /* = SSD_ABI_VERSION */
    uint32_t q, r, delta;
    uint32_t eta;
    uint32_t k;
    uint32_t theta;
    uint32_t key_bits;
    uint32_t flags;
    uint32_t cell_bits; /* 8 (0 = 8) or 16 */
    uint64_t max_tuples;
    uint64_t max_results;
} ssd_params;

/* One regained host: its address, the in-window cell count R of its union
 * estimator (Alg. 1 over its r estimators) and the estimate of Eq. 1,
 * -eta * ln(max(eta - R, 1) / eta), in double. */
typedef struct {
    uint32_t ip;
    uint32_t rk;
    double est;
} ssd_super_point;

typedef struct ssd_detector ssd_detector;

/* Read-only facts about a detector. */
typedef struct {
    uint64_t open_slice;     /* slice that scans currently write               */
    uint32_t hot_threshold;  /* T                                              */
    uint32_t r;
    uint64_t state_bytes;    /* r * 2^q * eta * cell_bits / 8                  */
    uint64_t level_counts[16]; /* tuples per candidate level at the last close
                                  (level 0 = rows 0..2, level L = row L+2)      */
    uint32_t hot_counts[16]; /* |HSE(i)| at the last close                     */
    uint64_t accepted;       /* accepted tuples at the last close              */
    uint64_t reported;       /* hosts in the last result list                  */
    uint32_t counted;        /* R_k of the last close: 0 read from the state,
                                1 from the per-slot counters, 2 from counters
                                rebuilt from the state first                  */
    uint32_t counted_bin_kib; /* bin size (KiB of cells) of the last scan call
                                that took the bitmap stores (the counted
                                ones, or those of 16-bit cells), 0 if none   */
} ssd_info;

/* Sizes the caller must allocate on the device for params p: the estimator
 * state (16-byte aligned) and the library's scratch (256-byte aligned).
 * Returns SSD_E_PARAM if p is invalid. */
int ssd_query_sizes(const ssd_params *p, uint64_t *state_bytes, uint64_t *scratch_bytes);

/* Create a detector (Sec. 3.2: every cell starts empty, once).
 *   tables_host: uint32[2][4][256] host array, the tabulation tables of
 *       RHFG[0] ([0]) and of the cell hash H1 ([1]) (simple tabulation
 *       hashing, cited in Sec. 3.2 and 3.3); copied, not retained.
 *   state_dev / scratch_dev: caller-owned device buffers of at least the
 *       sizes from ssd_query_sizes(); their contents are overwritten.
 *   stream: hipStream_t (NULL = default stream) on which all work runs; the
 *       device current at this call is the detector's device.
 *   out: receives the detector.  The open slice is 0. */
int ssd_init_detector(const ssd_params *p, const uint32_t *tables_host,
                      void *state_dev, uint64_t state_bytes,
                      void *scratch_dev, uint64_t scratch_bytes,
                      void *stream, ssd_detector **out);

/* Scan n (cip, oip) pairs into the open slice (Alg. 2; parallel form
 * Sec. 4.1).  pairs_dev: device array uint32[n][2], 8-byte aligned, with
 * [i][0] the monitored host cip and [i][1] its peer oip; borrowed until the
 * stream passes this call.  slice_id must equal the open slice
 * (SSD_E_ORDER otherwise).  Any number of calls per slice; the result does
 * not depend on how pairs are split over calls or ordered.  n = 0 is a no-op. */
int ssd_scan_slice(ssd_detector *d, const uint32_t *pairs_dev, uint64_t n, uint64_t slice_id);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * scan as ssd_scan_slice (same arguments, errors and resulting state; the
 * scan mode is chosen the same way), but the staging of the binned scan (the
 * binning's offset segments and bin-major table) is taken from a static
 * device array of SSD_NOALLOC_SCRATCH_BYTES (64 MiB) instead of the
 * detector's scratch.  The library holds one such array on every device it
 * runs on, until the process ends.  The call allocates nothing (no
 * hipMalloc, no host or pinned allocation, no event) and records no phase
 * timing.  A binned call whose staging exceeds the array fails with
 * SSD_E_NOMEM before any work is enqueued (about 2.8M pairs at r = 6 with
 * the default bins): split the slice over smaller calls.  Every call on one
 * device shares that device's array, which keeps the last call's contents
 * (nothing in it needs to start at zero: each call writes all the staging
 * it reads).  Calls that overlap on one device race: calls of detectors on
 * different streams must be ordered by the caller (events or
 * synchronisation). */
#define SSD_NOALLOC_SCRATCH_BYTES 67108864ull   /* 64 MiB */
int ssd_scan_slice_noalloc(ssd_detector *d, const uint32_t *pairs_dev, uint64_t n, uint64_t slice_id);

/* Close the open slice t.  Without flags: estimate every sliding estimator
 * over slots max(0, t-k+1)..t, regain the candidate hosts (Sec. 4.2) and
 * report SSP(max(0, t-k+1), k) sorted by ip, one entry per ip with its largest
 * R; write up to cap entries to out_host (host memory) and the count to
 * *n_out.  With SSD_ADVANCE_ONLY (router detectors in the distributed case):
 * only advance the clock; *n_out = 0.  The open slice becomes t+1 in every
 * case except SSD_E_DEVICE.  SSD_E_TRUNC: cap was too small (the list is kept
 * for ssd_get_results()).  SSD_E_OVERFLOW: a capacity was exceeded and no
 * list is returned; the window contents are unchanged. */
int ssd_close_slice(ssd_detector *d, uint32_t flags, ssd_super_point *out_host,
                    uint64_t cap, uint64_t *n_out);

/* The same close in two halves, so that the next slice's scans can be
 * enqueued while this close runs and its list is collected (pipelining).
 * ssd_close_begin enqueues the close of the open slice t on the detector's
 * stream and opens slice t+1 at once; it does not wait.  ssd_close_end waits
 * for that close only (not for work enqueued after it) and returns its list
 * exactly as ssd_close_slice would, with the same errors.  At most one close
 * may be pending: ssd_close_begin, ssd_close_slice, merges and group closes
 * of a detector with a pending close fail with SSD_E_ORDER, as does
 * ssd_close_end with none pending.  Scans of slice t+1 are allowed while the
 * close of t is pending. */
int ssd_close_begin(ssd_detector *d);
int ssd_close_end(ssd_detector *d, ssd_super_point *out_host, uint64_t cap, uint64_t *n_out);

/* The list of the last close again (host copy). */
int ssd_get_results(ssd_detector *d, ssd_super_point *out_host, uint64_t cap, uint64_t *n_out);

/* Distributed merge (Alg. 5): overwrite global's window contents, for every
 * cell, with the most recent hit over the routers' cells (per-cell maximum
 * slot stamp, i.e. minimum distance).  All detectors must share geometry,
 * tables, device and open slice (SSD_E_INCOMPAT otherwise) and run on one
 * device; the work runs on global's stream, after the routers' scans (the
 * caller orders the streams if they differ).  n >= 1; routers must not
 * include global. */
int ssd_merge_router_state(ssd_detector *global, ssd_detector *const *routers, uint32_t n);

/* Checkpoint and resume.  The paper's distance recorders are set up once and
 * then only stored to (Sec. 3.2), so a detector is its parameters, its hash
 * tables, its open slice and its state.  The blob: an 80-byte header (format, the
 * parameters' geometry, window, threshold, key width, flags and cell width,
 * a hash of the tables, the open slice), then the state bytes as they lie in
 * HBM (little-endian host).  The per-slot counters of a counting detector
 * are not in it: the importing detector takes them as stale (rebuilt from
 * the state after its next large binned call, else its next close reads the
 * state), which changes no result.
 * ssd_export_state: *n_out = the blob's size; the blob is written to
 * out_host (host) when cap is at least that, else SSD_E_TRUNC.  No close may
 * be pending (SSD_E_ORDER); waits for the detector's stream.
 * ssd_import_state: the blob of ssd_export_state (n bytes, host) into a
 * detector made with the same parameters and tables (SSD_E_INCOMPAT
 * otherwise; SSD_E_PARAM for a blob of another format or size); no close
 * pending.  The detector then continues from the blob's open slice exactly as
 * the exporting detector would: same states, same lists.  Synchronous. */
int ssd_export_state(ssd_detector *d, void *out_host, uint64_t cap, uint64_t *n_out);
int ssd_import_state(ssd_detector *d, const void *blob_host, uint64_t n);

/* Parity and inspection. */

/* Canonical window state of the open slice t, after its scans and before its
 * close (the same for 8- and 16-bit cells): out_dev[i] (device, uint16,
 * n_cells = r*2^q*eta entries in [row][column][cell] order) = t - (slot of
 * the cell's latest hit) when that is below k, else 0xFFFF.  Synchronous. */
int ssd_read_canonical_state(ssd_detector *d, uint16_t *out_dev, uint64_t n_cells);

/* R_k of every estimator at the last close, uint32[r][2^q] (host). */
int ssd_read_rk(ssd_detector *d, uint32_t *out_host, uint64_t n);

/* Hot estimator lists HSE(0..r-1) of the last close: counts_host[r] and the
 * ascending column lists packed row after row into lists_host (capacity
 * cap entries). */
int ssd_read_hot(ssd_detector *d, uint32_t *counts_host, uint32_t *lists_host, uint64_t cap);

/* Candidate tuples that reached the final test at the last close, one column
 * per row: out_host is uint32[cap][r]; *n_out = number of tuples (order is
 * not specified).  SSD_E_TRUNC if cap is too small. */
int ssd_read_tuples(ssd_detector *d, uint32_t *out_host, uint64_t cap, uint64_t *n_out);

int ssd_get_info(ssd_detector *d, ssd_info *out);

/* Tuning knobs; none changes results.
 *   SSD_TUNE_SCAN_PASS_BYTES: state bytes one scan pass covers (0 = one pass
 *       over the whole state; default 128 MiB).  Passes sized to the device's
 *       last-level cache keep a pass's random byte stores cache-resident.
 *   SSD_TUNE_SORT_BLOCK_LIMIT: result lists up to this many accepted hosts
 *       are sorted inside one workgroup (at most 8192, the default); longer
 *       lists use the multi-kernel sort. */
#define SSD_TUNE_SCAN_PASS_BYTES 1u
#define SSD_TUNE_SORT_BLOCK_LIMIT 2u
#define SSD_TUNE_TIMING 3u          /* 1: time every phase with HIP events */
#define SSD_TUNE_SCAN_TILE_PAIRS 4u /* batches: pairs per scan work tile (default 4096) */
#define SSD_TUNE_GRAPH 5u           /* 1 (default) = replay the close as a HIP graph (detectors, batches) */
#define SSD_TUNE_AUTOTUNE 6u        /* batches: 1 = tune on the next scans (reads 1 until
                                       done, 9 to 11 scans): the tile scan's (pass window,
                                       tile) pair, each of 9 timed on one scan; and the bin
                                       size of the counted stores by class of binned links
                                       (same q and eta, pairs per call in the same factor-4
                                       band), timed on the whole binned scan: 256 KiB,
                                       512 KiB and 1 MiB for every class, the fastest kept,
                                       then the two others for each of the 4 classes with
                                       the most pairs, kept when 1% faster */
/*   SSD_TUNE_SCAN_MODE: SSD_SCAN_PASSES = pass windows as above;
 *       SSD_SCAN_BINNED = each call's pairs are first sorted by state bin
 *       (SSD_TUNE_SCAN_BIN_BYTES, a power of two, default 2 MiB), then each
 *       bin's stores are made by workgroups of one XCD, inside its L2;
 *       SSD_SCAN_AUTO (default) = binned for states above 256 MiB, else passes
 *       (batches: every link with at least 2^16 pairs in the call is scanned
 *       binned, all such links together -- per group of links whose staging
 *       fits, one binning launch and one store launch per kind, 2 MiB bins
 *       uncounted -- the others in
 *       the tile scan; batches take SSD_SCAN_PASSES or SSD_SCAN_AUTO). */
#define SSD_TUNE_SCAN_MODE 7u
#define SSD_TUNE_SCAN_BIN_BYTES 8u
#define SSD_TUNE_SCAN_APPLY_SEGMENTS 9u   /* binned: binning segments per store workgroup (default 2) */
#define SSD_SCAN_PASSES 0u
#define SSD_SCAN_BINNED 1u
#define SSD_SCAN_AUTO 2u
/*   SSD_TUNE_COUNTED: 1 (default) = while a detector's scans are binned, it
 *       keeps for every estimator and every slice of the window the number of
 *       cells that hold that slice's stamp, updated by the scan's stores (bins
 *       of 1 MiB, 512 KiB or 256 KiB: the largest not above 512 KiB, or
 *       above SSD_TUNE_SCAN_BIN_BYTES once set, that fits; each stored by one
 *       workgroup that marks the cells it has visited).  Its close then takes R_k from these
 *       counters and reads only the cells of hot estimators and of the
 *       estimators whose expiry phase it is, instead of the whole state.
 *       Possible when eta >= 8 k (the counters take at most half the
 *       state), eta <= 2^14, the cell bits and 16-bit counters of one bin
 *       fit a workgroup's LDS (a bit per cell and 2 bytes per estimator and
 *       slice: at 256 KiB bins 32 KiB + 512 k bytes for eta = 1024; bins
 *       are chosen so that two workgroups share a compute unit where one
 *       size allows it) and the state fits 4096 bins; the counters (k
 *       per-slice slots and a live-cell total) take r * 2^q * (k + 1) * 4
 *       bytes of
 *       scratch (included in ssd_query_sizes).  A scan call with fewer cell
 *       offsets per bin on average than SSD_TUNE_COUNTED_MIN_ITEMS (default
 *       2048 for detectors, 256 for batches, which scan each link once per
 *       slice) stores uncounted (the counted stores cost a workgroup per
 *       bin); it, a router
 *       merge into the detector, an advance-only close, a pass scan or a
 *       group call leaves the counters stale: the close reads the state,
 *       or, when every binned call of the slice was large, rebuilds the
 *       counters from it.  Large calls take the counted stores also while
 *       the counters are stale (each touched 16-byte chunk is restamped
 *       once, faster than a byte store per offset when pairs repeat); the
 *       counters then stay stale until the rebuild.  Batches: the same for every link that can count
 *       (reading 1 if any link counts); a link scanned by the tile scan in a
 *       slice (fewer than 2^16 pairs in the call, or SSD_SCAN_PASSES) leaves
 *       its counters stale likewise. */
#define SSD_TUNE_COUNTED 10u
#define SSD_TUNE_COUNTED_MIN_ITEMS 11u   /* counted scans: offsets per bin a call needs (default 2048, batches 256);
                                           the same bar, over bins of 2^18 cells, lets a binned call of a
                                           detector of 16-bit cells (which keep no counters) take the bitmap
                                           stores: each touched 16-byte chunk restamped once */
int ssd_set_tuning(ssd_detector *d, uint32_t knob, uint64_t value);

/* Phase timing (with SSD_TUNE_TIMING on): device time in ms accumulated per
 * phase, measured with HIP events recorded on the detector's stream around
 * each phase's kernels, and the number of kernel launches per phase.
 * Phases: 0 scan stores, 1 hot detection, 2 hot lists, 3 candidate expansion,
 * 4 final test, 5 sort/report, 6 merge, 7 the close after hot detection
 * replayed as a graph (phases 2-5 are then timed as this one), 8 scan
 * binning (the sort step of the binned scan), 9 hot detection from the
 * per-slot counters (SSD_TUNE_COUNTED; two launches when the counters are
 * rebuilt from the state first), 10 the persistent tile scan of batches and
 * groups (phase 0 then holds their binned links' stores).  Synchronises the
 * stream; reset != 0 clears the totals after reading. */
#define SSD_PHASES 11u
int ssd_read_timing(ssd_detector *d, double *ms_out, uint64_t *launches_out, int reset);

void ssd_destroy(ssd_detector *d);
const char *ssd_strerror(int status);
const char *ssd_last_error(void);

/* ---- Batches: many monitored links closed together ------------------------
 *
 * n independent detectors ("links"), each with its own ssd_params and hash
 * tables, sharing one slot clock, one stream and one caller-owned state and
 * scratch buffer.  A scan covers every link's pairs of the open slice in one
 * persistent launch; a close reconstructs every link with one fixed launch
 * sequence, captured once as a HIP graph and replayed every slot.  Each
 * link's results are identical to those of a separate detector fed the same
 * pairs (same method as above: Alg. 2 scans, Sec. 4.2 reconstruction). */
typedef struct ssd_batch ssd_batch;

/* Device sizes for the n links described by p[0..n-1] (1 <= n <= 1024). */
int ssd_batch_query_sizes(const ssd_params *p, uint32_t n, uint64_t *state_bytes, uint64_t *scratch_bytes);

/* tables_host: uint32[n][2][4][256], each link's RHFG[0] and H1 tables
 * (copied).  state_dev (16-byte aligned) and scratch_dev (256-byte aligned)
 * are caller-owned device buffers of at least the queried sizes; stream is
 * a hipStream_t.  The open slice is 0. */
int ssd_batch_init(const ssd_params *p, uint32_t n, const uint32_t *tables_host,
                   void *state_dev, uint64_t state_bytes, void *scratch_dev, uint64_t scratch_bytes,
                   void *stream, ssd_batch **out);

/* Scan the open slice of every link: link l's pairs are
 * pairs_dev[offsets_host[l] .. offsets_host[l+1]) (uint32[.][2] on the device,
 * 8-byte aligned, cip first; offsets non-decreasing, host array of n+1).
 * Asynchronous; the pairs are borrowed until the stream passes this call.
 * slice_id must equal the open slice (SSD_E_ORDER). */
int ssd_batch_scan(ssd_batch *b, const uint32_t *pairs_dev, const uint64_t *offsets_host, uint64_t slice_id);

/* Close the open slice of every link (see ssd_close_slice).  Writes the
 * links' lists one after another into out_host (up to cap entries in total),
 * counts_host[l] = entries of link l and status_host[l] = SSD_OK or
 * SSD_E_OVERFLOW (that link's capacities were exceeded; it reports nothing).
 * Returns SSD_E_TRUNC when cap is too small (counts are set; fetch the lists
 * with ssd_batch_get_results).  The open slice advances in every case except
 * SSD_E_DEVICE. */
int ssd_batch_close(ssd_batch *b, ssd_super_point *out_host, uint64_t cap, uint64_t *counts_host,
                    int *status_host);

/* ssd_batch_close in two halves, so that the next slice's ssd_batch_scan can
 * be enqueued while the close runs (the pipelined close of a detector, for
 * a batch): _begin enqueues the close of every link and opens the next slice
 * at once; _end waits for it and returns the lists as ssd_batch_close.  One
 * close may be pending (SSD_E_ORDER otherwise); ssd_batch_get_results,
 * ssd_batch_read_rk and ssd_batch_read_hot are refused while it is
 * (SSD_E_ORDER).  Tuning samples of scans enqueued after the close are
 * credited at a later _end. */
int ssd_batch_close_begin(ssd_batch *b);
int ssd_batch_close_end(ssd_batch *b, ssd_super_point *out_host, uint64_t cap, uint64_t *counts_host,
                        int *status_host);
int ssd_batch_get_results(ssd_batch *b, ssd_super_point *out_host, uint64_t cap, uint64_t *counts_host,
                          int *status_host);

/* Tuning knobs SSD_TUNE_* (none changes results) and phase timing (as for
 * single detectors). */
int ssd_batch_set_tuning(ssd_batch *b, uint32_t knob, uint64_t value);
int ssd_batch_get_tuning(ssd_batch *b, uint32_t knob, uint64_t *value);
int ssd_batch_read_timing(ssd_batch *b, double *ms_out, uint64_t *launches_out, int reset);
/* Inspection of link `link` at the last close, as ssd_get_info, ssd_read_rk
 * and ssd_read_hot for a single detector (facts, R_k per estimator, hot
 * lists). */
int ssd_batch_get_info(ssd_batch *b, uint32_t link, ssd_info *out);
int ssd_batch_read_rk(ssd_batch *b, uint32_t link, uint32_t *out_host, uint64_t n);
int ssd_batch_read_hot(ssd_batch *b, uint32_t link, uint32_t *counts_host, uint32_t *lists_host, uint64_t cap);
void ssd_batch_destroy(ssd_batch *b);

/* ---- Groups: continuous batching over independent detectors ---------------
 *
 * A group runs one batched scan launch, or one batched close sequence, over
 * any set of single detectors (each with its own parameters, tables, memory
 * and slot clock), chosen afresh at every call.  A serving loop uses it to
 * scan every stream whose packets have arrived, and to close every stream
 * whose slot has ended, in one launch each while streams come and go.  Every
 * member's results equal those of its own ssd_scan_slice / ssd_close_slice.
 * Members must live on the group's device and use the group's stream; the
 * group's scratch (caller-owned device memory) holds the members'
 * descriptors and staging. */
typedef struct ssd_group ssd_group;

int ssd_group_query_sizes(uint32_t max_members, uint64_t *scratch_bytes);
int ssd_group_init(uint32_t max_members, void *scratch_dev, uint64_t scratch_bytes, void *stream, ssd_group **out);

/* Scan into the open slice of every member: member i's pairs are
 * pairs_dev[offsets_host[i] .. offsets_host[i+1]); slice_ids_host[i] must
 * equal member i's open slice (SSD_E_ORDER).  Asynchronous.  The members
 * that get at least 2^18 pairs (and whose scan mode is not SSD_SCAN_PASSES)
 * are scanned binned, each into its own bin buffers: per round one binning
 * launch and one store launch per store kind over all of them (a member
 * whose pairs exceed its buffers takes part in several rounds); all others
 * share one tile-scan launch.  A member that keeps per-slot counters takes
 * the counted stores for a large call (each touched chunk restamped once),
 * its counters then untrusted until its own close rebuilds them: group
 * closes read every member's state. */
int ssd_group_scan(ssd_group *g, ssd_detector *const *members, uint32_t n, const uint32_t *pairs_dev,
                   const uint64_t *offsets_host, const uint64_t *slice_ids_host);

/* Close the open slice of every member (each advances by one slot); lists
 * one after another in out_host, counts_host[i] / status_host[i] as for
 * ssd_batch_close.  A member's list is also kept as its own last result
 * (ssd_get_results). */
int ssd_group_close(ssd_group *g, ssd_detector *const *members, uint32_t n, ssd_super_point *out_host,
                    uint64_t cap, uint64_t *counts_host, int *status_host);

/* The same close in two halves (as ssd_close_begin / ssd_close_end), so that
 * a serving loop keeps admitting and scanning while a close runs:
 * ssd_group_close_begin enqueues the close of every member's open slice on
 * the group's stream and opens each member's next slice at once, without
 * waiting; ssd_group_close_end waits for that close only and returns the
 * lists exactly as ssd_group_close would.  At most one close per group may
 * be pending (SSD_E_ORDER).  While it is, its members may scan their next
 * slice (group or own scans) but not close, merge or be inspected
 * (SSD_E_ORDER), and must not be destroyed. */
int ssd_group_close_begin(ssd_group *g, ssd_detector *const *members, uint32_t n);
int ssd_group_close_end(ssd_group *g, ssd_super_point *out_host, uint64_t cap, uint64_t *counts_host,
                        int *status_host);
void ssd_group_destroy(ssd_group *g);

#ifdef __cplusplus
}
#endif

#endif /* SSD_H */
