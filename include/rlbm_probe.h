/*
 * rlbm_probe.h -- measurement helper of the rlbm library: the memory
 * bandwidth this device reaches for simple access patterns, the practical
 * ceilings against which the step kernel's roofline fraction is read.  Not
 * part of the method; nothing else in the library calls it.
 */
#ifndef RLBM_PROBE_H
#define RLBM_PROBE_H

#include "rlbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RLBM_PROBE_READ = 0,   /* read the array once (16-byte loads, four per thread in flight) */
    RLBM_PROBE_COPY = 1,   /* copy it into a second array (16-byte loads and stores, four per thread) */
    RLBM_PROBE_PULL48 = 2, /* the step's pattern: at every site with x, y in [5, n - 5), 48 loads from the
                              planes of the population layout, each shifted by its population's hop, and 48
                              aligned stores, with trivial arithmetic between them */
    RLBM_PROBE_PULL48_PAIR = 3, /* the same with two adjacent sites (x even, x in [6, nx - 6)) per thread: each
                                  plane read as one two-element load from the hop-shifted address (aligned to
                                  one element only for odd hops) and written as one aligned two-element store;
                                  nx must be even */
    RLBM_PROBE_PULL12_TUPLE = 4, /* the step's pull in a direction-tuple layout: 12 arrays of nx ny tuples, a
                                   tuple holding the four energy shells of one direction at one site (they
                                   share the hop); per site with x, y in [5, n - 5), 12 hop-shifted tuple
                                   loads (4 elem_bytes each) and 12 aligned tuple stores */
    RLBM_PROBE_PULL24_TUPLE = 5, /* the same with tuples of two shells: 24 arrays, 24 loads and 24 stores of
                                    2 elem_bytes per site */
    RLBM_PROBE_PULL48_T64 = 6,        /* PULL48 by blocks of 64 x 4 sites (the other pull patterns use blocks of
                                         256 x 1 sites) */
    RLBM_PROBE_PULL24_TUPLE_T64 = 7,  /* PULL24_TUPLE by blocks of 64 x 4 sites */
    RLBM_PROBE_PULL12_TUPLE_T64 = 8   /* PULL12_TUPLE by blocks of 64 x 4 sites */
} rlbm_probe_pattern;

/* Time `pattern` on arrays the size of one population array of an nx x ny
 * lattice (48 nx ny elements of elem_bytes = 2, 4 or 8), allocated and freed
 * by the call on the current device: 3 untimed launches, then `reps` timed
 * with HIP events on hip_stream (NULL = the null stream); for PULL48 the two
 * arrays swap roles between launches.  nontemporal = 1 makes the stores of
 * COPY and PULL48 streaming (non-temporal) stores.  Writes the bytes moved
 * per launch over the average launch time in GB/s (READ: the array once;
 * COPY: twice; PULL48: 2 x 48 x elem_bytes per interior site) to *gbs and
 * that time in microseconds to *us (either may be NULL).  RLBM_EINVAL for
 * nx <= 12 or ny <= 10, ny > 65545, an odd nx for PULL48_PAIR, an array beyond 2^34 bytes, elem_bytes other
 * than 2, 4 or 8, reps < 1 or an unknown pattern; RLBM_ENOMEM if the arrays
 * do not fit; synchronises the stream. */
rlbm_status rlbm_bandwidth_probe(int pattern, int elem_bytes, int nx, int ny, int nontemporal, int reps,
                                 void *hip_stream, double *gbs, double *us);

#ifdef __cplusplus
}
#endif

#endif /* RLBM_PROBE_H */
