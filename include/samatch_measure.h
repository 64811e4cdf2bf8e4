/*
 * samatch_measure.h -- measurement helpers of libsamatch.so that are not part
 * of the matching path: the benchmark uses them to put the search kernels'
 * figures beside what the device can do at best.  Same return codes and
 * error reporting as samatch.h.
 */
#ifndef SAMATCH_MEASURE_H
#define SAMATCH_MEASURE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The rate (loads per second, into *loads_per_s) at which the device serves
 * random 16-byte loads from a table of 2^log2_entries 16-byte entries
 * (8 <= log2_entries <= 28), the access pattern of the search kernels'
 * probes (Section IV: each binary-search step reads one suffix-array row at
 * a data-dependent position).  Every lane follows two independent chains of
 * 16 dependent loads at hashed positions, 16 waves per compute unit; the
 * best of five timed launches.  Allocates and frees the table; runs on the
 * null stream and waits for it.  SA_EINVAL (-1) for a size out of range,
 * SA_EDEVICE (-5) / SA_ENOMEM (-4) on device failures. */
int sa_random_read_rate(int device, int log2_entries, double *loads_per_s);

#ifdef __cplusplus
}
#endif

#endif /* SAMATCH_MEASURE_H */
