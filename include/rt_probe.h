/* rt_probe.h -- memory-system probes of the MI355X ray tracing library.
 *
 * Measurement helpers, not part of the ray tracing path: they give the
 * roofline of the traversal kernel its measured ceilings (streaming reads
 * from working sets that live in L2, in the Infinity Cache or in HBM) and a
 * copy of known size that calibrates the hardware byte counters.
 *
 * Same conventions as rt_mi355x.h: device pointers, work enqueued on the
 * given stream (no wait), RT_OK or a negative RT_E* code, error text from
 * rt_last_error().
 */
#ifndef RT_PROBE_H
#define RT_PROBE_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Streaming reads: each of `groups` work-groups (256 threads) reads `span`
 * bytes of the buffer, starting at byte (g * span) mod bytes for work-group g
 * and wrapping at the end, `passes` times over, with 16-byte loads (lanes on
 * consecutive addresses).  span = bytes makes every work-group read the whole
 * working set (so each XCD's L2 holds all of it when it fits); span = bytes /
 * groups gives disjoint slices.  Bytes moved = span * passes * groups.  One
 * 32-bit word per work-group is written to sink[0 .. groups - 1] so the loads
 * cannot be dropped.  buf and sink 16-byte aligned; bytes and span positive
 * multiples of 16, span <= bytes; passes >= 1; groups in 1..65536.
 * Errors: RT_EINVAL (null, misaligned, sizes), RT_EHIP. */
int rt_probe_read(const void* buf, int64_t bytes, int64_t span, int32_t passes, int32_t groups,
                  uint32_t* sink, hipStream_t s);

/* Plain copy of `bytes` bytes from src to dst with 16-byte loads and stores
 * (one kernel, named k_probe_copy, for counter calibration).  Both 16-byte
 * aligned, bytes a positive multiple of 16, the ranges must not overlap.
 * Errors: RT_EINVAL, RT_EHIP. */
int rt_probe_copy(const void* src, void* dst, int64_t bytes, hipStream_t s);

#ifdef __cplusplus
}
#endif

#endif /* RT_PROBE_H */
