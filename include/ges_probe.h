/* Device peak probes used by the measurement script (not part of the render
 * path).  They give the measured ceilings the per-stage rooflines are also
 * quoted against: the HBM bandwidth a plain copy reaches and the rate of
 * global 32-bit atomic adds on a counter array laid out like the tile
 * counters of the binning passes.
 *
 * Both allocate their own device buffers (hipMalloc), time `reps` launches
 * with HIP events on the null stream of `device`, free the buffers and return
 * the best rate.  They return 0 on success and a HIP error code otherwise;
 * *out is untouched on failure.  Not thread-safe with other work on the
 * device (they synchronise it).
 */
#ifndef GES_PROBE_H
#define GES_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Copies `bytes` (rounded down to a multiple of 16) from one buffer to
 * another with 16-byte vector loads and stores; *out_gbs = (bytes read +
 * bytes written) / time, in GB/s (1e9 bytes). */
int ges_probe_copy(int device, size_t bytes, int reps, double *out_gbs);

/* `atomics` lane-level atomicAdd(1) on uint32 counters, each lane picking one
 * of `counters` counters (each on its own 128-byte line) by a hash of its
 * index; *out_gops = atomics / time, in 1e9 atomics/s. */
int ges_probe_atomics(int device, int64_t atomics, int32_t counters, int reps, double *out_gops);

#ifdef __cplusplus
}
#endif
#endif
