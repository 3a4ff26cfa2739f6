// md_device.h -- data layout shared by the gfx950 kernels and the host engine.
//
// Every system ("replica") owns its own device buffers; kernels find them
// through a per-replica descriptor (SlotDev) and keep per-replica mutable
// state in a control block (CtlDev).  A launch covers the tiles of all
// replicas of an engine (tile -> replica via a table), so one kernel launch
// advances many systems and a single system is an engine with one replica.
//
// Step numbering: step k (k >= 1) of a replica is the k-th leapfrog step
// after creation; "state k" is r(k), v(k).  Storage of the time levels:
//   r(k)      in P[k & 1]
//   v(k-1/2)  in V[k & 1]   (during a run)
//   v(k)      in V[(k+1) & 1] when the replica is clean at step k
// The cell-layer matrix comes in three sets; the rows of state k live in set
// k % 3, so one step can read its rows while the next step's rows are
// written and the set after that is cleared.
//
// Storage order: the atoms are stored in cell order as of the last rebuild.
// A rebuild step sorts r(k) by cell (stable counting sort from the rows of
// set k % 3) into the other descriptor variant, so the atoms of a cell are
// contiguous and cell_start gives their range.  CtlDev::var_ring[k % 3] is
// the variant that holds state k.
#pragma once

#include <stdint.h>

namespace md {

constexpr int TILE = 256;          // atoms per tile (one workgroup of 4 wave64)
constexpr int CTILE = 256;         // cells per sort tile (one per thread)
// Neighbour entry (32 bits): bits 0-24 an index, bit 25 (GFLAG) set when the
// index is a storage index and clear when it is a slot of the tile's LDS
// window, bits 26-31 the periodic image code (2 bits per dimension, x
// lowest: 0 none, 1 +L, 3 -L).
constexpr int J_BITS = 26;         // image code starts here
constexpr int IDX_BITS = 25;
constexpr uint32_t IDX_MASK = (1u << IDX_BITS) - 1;
constexpr uint32_t GFLAG = 1u << IDX_BITS;
// LDS window of a tile: the storage-index intervals holding every candidate
// neighbour of the tile's atoms at the last sort, staged into LDS each step.
constexpr int WCAP = 1640;         // atoms (FP64 x, y, z: 38.4 KB, four workgroups per CU)
constexpr int NROWS = 64;          // (source row, dz, dy) combinations a window describes
constexpr int NOSLOT = INT32_MIN;  // storage-index-to-slot offset of a piece not in LDS
constexpr int NWIN = 32;           // intervals
constexpr int WSTRIDE = 1 + 3 * NWIN;  // ints per tile: count, then (start, len, slot)
constexpr int NPART = 8;           // doubles per tile in the property partials
constexpr int NACC = 4;            // doubles per tile in the block accumulators
constexpr int MAX_GRID = 2048;     // persistent-style grid bound (256 CUs x 8)
constexpr int SORT_GRID = 512;     // sort workgroups of a single system (fewer, fuller
                                   // workgroups: idle launches cost less)
constexpr int OVF_CAP = 4096;      // per-set overflow list of cell-layer rows
constexpr int VSPREAD = 32;        // slots of each max-speed ring entry (one per 128-byte line)
constexpr int MAXSP = 4;           // species of a mixture
constexpr int MAX_REPLAY = 64;     // steps of the longest replay graph
constexpr int TRACE_RING = 65536;  // steps held by a replica's property trace
constexpr int TRACE_W = 5;         // doubles per trace row: step, KE, PE, virial, max v^2

// Pair parameters of a mixture, for species pair k = a * MAXSP + b: Eq. (1)
// in units of sigma_ab and epsilon_ab, r^2 < rc2 inside the pair's cutoff,
// energy shift added there.  Stored as products the force loop uses.
struct PairTab {
  double rc2[MAXSP * MAXSP];
  double sig2[MAXSP * MAXSP];   // sigma^2
  double eps48[MAXSP * MAXSP];  // 48 epsilon
  double eps4[MAXSP * MAXSP];   // 4 epsilon
  double shift[MAXSP * MAXSP];
};

// Latched error bits (CtlDev::err).
enum : int32_t {
  ERR_CELL = 2,       // a cell-layer set overflowed beyond its overflow list (repairable)
  ERR_ESCAPED = 4,    // a coordinate outside [-3L/2, 3L/2) when binned
  ERR_NONFINITE = 8,  // NaN / Inf coordinate
  ERR_UNBINNED = 16,  // the rule fired at a step whose positions were not binned
                      // ahead (repairable: the host bins them and resumes)
};

// Binning ahead (see bins_due): r(k) is binned during step k-1 when the
// displacement rule, accumulated with BIN_AHEAD times the maximum speed of
// step k-2, would fire at step k.
constexpr double BIN_AHEAD = 1.5;

// CtlDev::rb_ring values of a rebuilding step.
enum : int32_t { RB_NONE = 0, RB_REORDER = 1, RB_PERM = 2 };

// Modes of the step kernel (and of the sort kernel: MODE_STEP or not).
enum : int32_t {
  MODE_STEP = 0,    // forces (c) + (d) + (e) [+ (a) of the next step and its binning]
  MODE_FORCES = 1,  // force evaluation at a clean state: store F, u_i, w_i, partials
  MODE_BUILD = 2,   // neighbour matrix only, at a clean state
};

// Per-replica device descriptor, read-only while kernels run.  The two
// variants of a replica differ in the sorted arrays: variant 1 swaps the two
// time-level buffers of P and V, and id with id_alt, cell with cell_alt.  A
// sort gathers the current time level into the other variant's buffers,
// which hold a time level nobody reads any more.
struct SlotDev {
  double *P[2][3];                  // positions x, y, z; two time-level buffers
  double *V[2][3];                  // velocities; two time-level buffers
  int32_t *id, *id_alt;             // original atom index of each storage position
  int32_t *cell, *cell_alt;         // cell of each atom at its latest binning
  void *F;                          // forces, SoA [3][npad] of float or double
  void *UA;                         // per-atom u then w, [2][npad] of float or double
  int32_t *m;                       // neighbour-list length per atom
  int32_t *W;                       // neighbour matrix [mcap][npad]
  int32_t *cnt[3];                  // per set: occupancy of every cell
  int32_t *tcnt[3];                 // per set: occupancy of every cell tile (CTILE cells)
  int32_t *H[3];                    // per set: cell-layer rows [ncell][hcap]
  int32_t *ovf[3];                  // per set: (cell, atom) pairs beyond hcap
  int32_t *ovf_n;                   // [3] fill of the overflow lists
  int32_t *cs;                      // cell_start[ncell + 1] of the last sort
  int32_t *win;                     // per atom tile: LDS window [WSTRIDE] (count < 0: none)
  double *part;                     // per-tile partial properties [ntiles][NPART]
  double *acc;                      // per-tile sums over the steps of a block [ntiles][NACC]:
                                    // sum v^2, sum u_i, sum w_i, sum m_i
  unsigned long long *vring;        // max v^2 of step k: [k % 3][VSPREAD] slots, 16 words apart
  double *tpart;                    // traced replica: per-tile KE, PE, virial, max v^2 of
                                    // step s of the replay, [MAX_REPLAY][ntiles][4] (else null)
  double *trace;                    // traced replica: [TRACE_RING][TRACE_W], row k % TRACE_RING
  int32_t *perm;                    // MD_NO_REORDER: storage index of the atom at each
                                    // position of cell order at the last sort (else null)
  int32_t *sp, *sp_alt;             // mixture: species of each storage position (else null)
  const PairTab *tab;               // mixture: pair parameters (else null)
  double L, halfL, invW, rn2, rc2, dt, hdt, half_shell, ushift, pad0;
  int32_t n, G, ncell, hcap, mcap, npad;
  int32_t ntiles;    // atom tiles: ceil(n / TILE)
  int32_t nctiles;   // cell tiles: ceil((ncell + 1) / CTILE), so one holds cell_start[ncell]
  int32_t tile_off, ctile_off;
  int32_t cpt;       // cells cleared per atom tile: ceil(ncell / ntiles)
  int32_t fp64, cell_only;
  int32_t nsp;       // species of a mixture (0: one species, the r_c / ushift above)
  int32_t noreo;     // MD_NO_REORDER: a sort finds the cell order (perm, cs) and the
                     // cells, wraps in place and moves nothing
  int32_t nr;        // reorder interval N_R in steps (0: every rebuild reorders); a
                     // rebuild that does not reorder works like one under noreo
  int32_t nowin;     // MD_NO_WINDOW: no LDS window (every read from global memory)
};

// Per-replica mutable control block.  Written by the host between launches,
// by single-workgroup kernels, or by one designated thread of the step kernel
// (fields nobody else reads in that launch).
struct CtlDev {
  int64_t done;        // steps completed
  int64_t target;      // steps to reach
  int64_t base;        // `done` when the current graph replay started
  int64_t force_step;  // step whose binning is a rebuild regardless of the rule
  int64_t err_step;    // first step that could not be evaluated
  int64_t bins_step;   // step whose positions the host binned after ERR_UNBINNED (-1: none)
  int64_t reo_ring[3]; // step of the last reordering as of step k, slot k % 3
  int64_t n_rebuilds;  // rebuilds by the displacement rule
  uint64_t vmax_ring[3];  // max v(k)^2 of ring entry k % 3, gathered by k_props (host view)
  double disp_ring[3];    // accumulated displacement after step k, slot k % 3
  int32_t clean;       // 1: r(done), v(done), F(done) are held; 0: drifted to r(done+1)
  int32_t var_ring[3]; // descriptor variant holding state k, slot k % 3
  int32_t rb_ring[3];  // step k rebuilds (decided by k_sort of step k), slot k % 3:
                       // RB_REORDER into the other variant, RB_PERM in place
  int32_t ord_ring[3]; // 1 if the storage of state k is not the cell order of the last
                       // sort (it rebuilt without reordering since), slot k % 3
  int32_t bin_ring[3]; // 1 if step k bins r(k+1) (decided by k_sort of step k), slot k % 3
  int32_t err;         // latched ERR_* bits
  int32_t max_h;       // largest cell occupancy seen by a sort
  int32_t pad1;
  // properties reduced by k_props
  double ke, pe, vir, vmax2;
  int64_t sum_m;
  int32_t max_m, pad0;
  // block sums reduced by k_props from SlotDev::acc
  double acc_sum[NACC];
};

// Engine-wide header (device int32[8]).
enum { HDR_NTILES = 0, HDR_NCTILES = 1, HDR_SPLIT = 2, HDR_ORDER = 3 };
// SPLIT: workgroups per cell tile in k_sort; ORDER: tile order of the step
// kernel's workgroups (ORDER_PASSES or ORDER_SLABS, see TileWalk)
enum { ORDER_PASSES = 0, ORDER_SLABS = 1 };
constexpr size_t WALK_BYTES = 16 * 64 * 4;  // Tables::walk

// Each replica has two descriptors (see SlotDev); CtlDev::var_ring says
// which one holds a given state.
struct Tables {
  const SlotDev *slots;       // [2 * nslots]: descriptor variant v of replica r at 2 r + v
  CtlDev *ctl;
  const int32_t *tile_rep;    // atom tile -> replica
  const int32_t *ctile_rep;   // cell tile -> replica
  int32_t *hdr;
  // k_step's tile claims: walk[64 x] counts the tiles claimed by workgroup
  // group x (x = block & 7), walk[64 (8 + x)] its workgroups that finished;
  // zero between launches (the group's last workgroup resets both)
  int32_t *walk;
  int32_t nslots;
};

}  // namespace md
