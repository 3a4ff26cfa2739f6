// md_kernels.h -- host-side launchers of the gfx950 kernels (md_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "md_device.h"

namespace md {

// Step (a) for clean replicas that have steps to go: kick, drift, binning.
void launch_kick(const Tables &T, int grid, hipStream_t s);
// Precisions present in an engine (bit mask): one step-kernel variant each.
enum { PREC_FP32 = 1, PREC_FP64 = 2 };

// One step (MODE_STEP, step index s of the replay) or an evaluation of the
// held clean state (MODE_FORCES / MODE_BUILD).  only >= 0: that replica only.
// accum: steps also add their properties to the block sums; mix: the
// replicas have several species.
void launch_step(const Tables &T, int grid, int step_in_replay, int mode, int force_build,
                 int only, int precisions, hipStream_t s, bool accum = false, bool mix = false);
// Traced replicas: the properties of the replay's K steps into their trace
// rings (before launch_replay_end).
void launch_trace(const Tables &T, int K, hipStream_t s);
// Advance the step counters after a replay of K steps.
void launch_replay_end(const Tables &T, int K, hipStream_t s);
// target = target; base = done (one replica).
void launch_set_target(const Tables &T, int slot, long long target, hipStream_t s);
// Reduce the property partials into the control blocks.
void launch_props(const Tables &T, int only, hipStream_t s);
// Step (f): scale the held clean velocities to temperature T (after
// launch_props, which reduces the kinetic energy it scales from).
void launch_adjust(const Tables &T, int grid, int only, double temperature, hipStream_t s);
// Bin the held state into its cell-layer set (optionally wrapping in place).
void launch_insert(const Tables &T, int grid, int wrap_store, int only, hipStream_t s);
// Counting sort by cell into the other buffer variant: in a step
// (MODE_STEP, step index s of the replay; only where the rebuild rule fires)
// or of the held clean state (any other mode; follow with launch_flip).
void launch_sort(const Tables &T, int cgrid, int step_in_replay, int mode, int only,
                 hipStream_t s);
// Cell index of every atom of replica `only` at its held position (storage
// order) into out[n].
void launch_cells(const Tables &T, int grid, int only, int32_t *out, hipStream_t s);
// After a sort of the held states: make the sorted variant current.
void launch_flip(const Tables &T, int only, hipStream_t s);
// Clear the held state's cell-layer set.
void launch_clear_set(const Tables &T, int cgrid, int only, hipStream_t s);

// Newton's-third-law A/B (md_ab.hip): a plain storage-index list, full or
// half, over the cell-sorted atoms, and its force loop (F: FP32 [3][npad];
// zero before a half launch).
void launch_ab_build(bool half, const double *x, const double *y, const double *z,
                     const int32_t *cell, const int32_t *cs, int n, int npad, int G, double L,
                     double rn2, int mcap, int32_t *W, int32_t *m, int32_t *overflow,
                     hipStream_t s);
// The cell-centric full list (one workgroup per cell, one thread per
// occupant): the same list as launch_ab_build(false, ...).
void launch_ab_build_cells(const double *x, const double *y, const double *z, const int32_t *cs,
                           int npad, int G, double L, double rn2, int mcap, int32_t *W,
                           int32_t *m, int32_t *overflow, hipStream_t s);
// Zero device memory with a kernel (bytes a multiple of 4).
void launch_ab_zero(void *p, size_t bytes, hipStream_t s);
// The A/B forces in the caller's order (out: n x 3 doubles) and the summed
// list lengths into *entries (zero before the launch).
void launch_ab_output(const float *F, const int32_t *id, const int32_t *m, int n, int npad,
                      double *out, unsigned long long *entries, hipStream_t s);
void launch_ab_forces(bool half, const double *x, const double *y, const double *z,
                      const int32_t *W, const int32_t *m, int n, int npad, double L, double rc2,
                      float *F, hipStream_t s);

}  // namespace md
