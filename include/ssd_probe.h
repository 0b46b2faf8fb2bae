/*
 * ssd_probe.h -- memory ceiling probes of the MI355X detector library
 * (measurement only; the detector's calls are in ssd.h).
 *
 * The paper reports the scan's throughput only (Sec. 5); these probes give
 * the ceilings the hot path is measured against on the same device: the
 * stream read that bounds hot detection and the merge, and the random byte
 * scatter that bounds the scan's distance-recorder stores (Alg. 2 writes one
 * recorder per row at a hashed address).  Work is enqueued on `stream`
 * (hipStream_t, NULL = default) and not waited for; the caller times it.
 * Return 0, -1 for invalid arguments, -7 for a failed launch.
 */
#ifndef SSD_PROBE_H
#define SSD_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Read every 16-byte chunk of buf_dev (bytes, a multiple of 16, 16-byte
 * aligned) once, coalesced.  sink_dev: a device buffer of at least 1 KiB the
 * kernel may write (its contents are meaningless). */
int ssd_probe_stream_read(const void *buf_dev, uint64_t bytes, void *sink_dev, void *stream);

/* n_stores one-byte stores at positions hashed from (seed, store index) into
 * buf_dev (bytes, at least 4 KiB).  xcd_local = 0: uniform over the whole
 * buffer.  xcd_local = 1: workgroup g stores only inside one 2 MiB region,
 * chosen so that the workgroups of one XCD (g mod 8) share regions that its
 * L2 holds (the pattern of the binned scan's stores), every region in turn;
 * bytes must then be a multiple of 2 MiB and at least 16 MiB. */
int ssd_probe_scatter(void *buf_dev, uint64_t bytes, uint64_t n_stores, uint64_t seed, uint32_t xcd_local,
                      void *stream);

/* Random 16-byte read-modify-writes in bins: buf_dev (bytes, a multiple of
 * bin_bytes, 16-byte aligned) is cut into bins of bin_bytes (a power of two,
 * 4 KiB to 1 GiB); one workgroup per bin, the bins dealt to the XCDs in
 * contiguous eighths, loads ops_per_bin (at most 2^20) chunks of its bin at
 * positions hashed from (seed, bin, op), changes and stores them.  The
 * memory side of the counted stores' visit (one read and one write of
 * every touched 16-byte chunk), at the same density. */
int ssd_probe_rmw16(void *buf_dev, uint64_t bytes, uint64_t bin_bytes, uint32_t ops_per_bin, uint64_t seed,
                    void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SSD_PROBE_H */
