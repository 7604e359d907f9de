/*
 * goc_ceiling.h -- C-ABI of the bandwidth instruments (libgocceiling.so).
 *
 * Measurement aids for the roofline of the GOC-LBM time step, kept out of
 * the solver library: they allocate and free their own device buffers and
 * never touch a solver handle.  The step they mirror is the one-pass
 * collide-and-stream update of App. E (every slot pulled from its neighbour
 * node, the node's own slots, ghost rows and lagged force written back),
 * with the D2Q5 slots of the induction scheme of App. G.
 *
 * Conventions: sizes are plain integers; stream is a hipStream_t (NULL: the
 * default stream) of the current device; results go to a host double.
 * All return GOC_OK (0), GOC_EINVAL for a bad argument, GOC_ENOMEM when an
 * allocation fails or GOC_EDEVICE when a HIP call fails (the goc_status
 * codes of goc_lbm.h); they synchronise with the stream before returning.
 */
#ifndef GOC_CEILING_H
#define GOC_CEILING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The memory pattern of one tiled step without its arithmetic: a straight
   run of nx x ny nodes (nx, ny >= 3; periodic along xi1, walls on the xi2
   faces) in the solver's layout (rows of 9 slot planes, or with mhd != 0
   20: the 9 population planes, one unused and the 10 D2Q5 planes; each
   plane padded to an odd number of 64-node pieces; two ghost rows; two force
   planes) for storage_bytes = 4 (FP32) or 2 (16-bit), in tiles of
   tile_cols x tile_rows nodes (64 x 4, 8 or 16, or 128 x 4) with plain
   (nontemporal = 0) or non-temporal stores.  Each launch pulls every slot
   and lagged force of the tile and of the ring around it, writes one LDS
   value per pulled node, waits at a barrier and stores the node's slots,
   ghost rows and force.
   Runs `reps` launches (>= 1, after 4 untimed ones) alternating two state
   buffers and writes the mean microseconds per launch (HIP events on
   `stream`) to *us_per_launch. */
int goc_ceiling_pattern(int nx, int ny, int mhd, int storage_bytes, int tile_cols, int tile_rows, int nontemporal,
                        int reps, void* stream, double* us_per_launch);

/* A plain one-stream copy of `bytes` (a positive multiple of 16) between two
   device buffers, 16-byte vectors (four loads in flight per thread), 32
   work-groups of 256 threads per compute unit; mean microseconds per launch
   over `reps` launches after 4 untimed ones. */
int goc_ceiling_copy(int64_t bytes, int reps, void* stream, double* us_per_launch);

/* Plain streams in a chosen read / write mix: `reads` input buffers (0, 1 or
   2) and `writes` output buffers (0, 1 or 2, reads + writes >= 1) of `bytes`
   each (a positive multiple of 16), 16-byte vectors, element k of every
   output written from element k of every input (four in flight per
   thread), with plain (nontemporal = 0) or non-temporal stores, wg_per_cu
   (1 .. 64) work-groups of 256 threads per compute unit, swept grid-stride
   (chunked = 0: the whole grid moves through the buffers together) or in
   contiguous shares (chunked = 1: each work-group sweeps one share of them
   on its own); mean microseconds per launch over `reps` launches after 4
   untimed ones.  A launch moves (reads + writes) * bytes. */
int goc_ceiling_mix(int64_t bytes, int reads, int writes, int nontemporal, int chunked, int wg_per_cu, int reps,
                    void* stream, double* us_per_launch);

#ifdef __cplusplus
}
#endif

#endif /* GOC_CEILING_H */
