/*
 * md.h -- C ABI of the MI355X (gfx950) soft-sphere molecular-dynamics hot path.
 *
 * Method: D. C. Rapaport, "Enhanced molecular dynamics performance with a
 * programmable graphics processor" (arXiv:0911.5631).  The library advances
 * atoms interacting through the soft-sphere potential -- Eq. (1), the
 * Lennard-Jones form, truncated at r_c = 2^(1/6) with the constant epsilon
 * added so that u(r_c) = 0 (Sec. 3.1) -- in a periodic cube centred at the
 * origin, in reduced units sigma = epsilon = m = 1.
 *
 * The path per time step (Sec. 3.1, loop steps (a)-(e)):
 *   (a) half-step velocity update and full-step position update (leapfrog);
 *   (b) when a rebuild is due: periodic wrap, cell binning (cell assignment
 *       and layer assignment, Secs. 3.2 and 3.4), reordering of the atoms
 *       into cell order (Sec. 3.5; done at every rebuild, as a stable
 *       counting sort) and the neighbour-matrix build over 27 cells without
 *       Newton's third law (Secs. 3.3-3.4);
 *   (c) forces and potential energy from the neighbour matrix (Sec. 3.4);
 *   (d) second half-step velocity update;
 *   (e) kinetic energy, maximum speed and the rebuild decision: the list is
 *       rebuilt when the accumulated sum of vmax*dt exceeds delta/2
 *       (Sec. 3.1);
 *   (f) during equilibration, the velocity adjustment (md_adjust_temp);
 *       properties averaged over blocks of steps (md_block_begin/end).
 * With shell == 0 the library runs the plain cell method instead (Sec. 3.1):
 * every step re-bins and evaluates forces straight from the 27 neighbouring
 * cells, with no stored list.
 *
 * Conventions shared by every entry point:
 *   - Host arrays of per-atom vectors are row-major double[n][3] in the
 *     caller's ORIGINAL atom order; the library keeps its own storage order
 *     (cell order) on the device and translates.
 *   - Ownership: the library copies host inputs and owns all device memory,
 *     which it obtains through the caller's md_allocator (NULL: hipMalloc /
 *     hipFree).  Host buffers passed in are never retained.
 *   - Streams: device work is ordered after everything already enqueued on
 *     the HIP stream given at creation (NULL: the null stream), and later
 *     work on that stream waits for it (also after a call that returns an
 *     error).  Calls marked "async" return before
 *     the device work completes; calls marked "sync" wait for it.
 *   - Errors found on the device (an escaped atom, a non-finite coordinate)
 *     are latched in the system, stop its device work at the step where
 *     they arose, and are returned by the next synchronising call.  A cell
 *     whose occupancy exceeds the layer capacity spills into an overflow
 *     list; when that fills too, the library enlarges the capacity and
 *     resumes the interrupted steps (error only if the allocation fails).
 *     An atom whose neighbour list exceeds nebr_cap is evaluated from the
 *     cells instead (same pairs, exact), and md_get_pairs reports
 *     MD_ERR_NEBR_OVERFLOW.  MD_ERR_HIP is sticky: after it only
 *     md_destroy / md_batch_destroy is valid.
 *   - Threading: one host thread at a time per md_system / md_batch.
 */
#ifndef PAPER_0911_5631_AMD_MD_H
#define PAPER_0911_5631_AMD_MD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct md_system md_system; /* one periodic system (opaque) */
typedef struct md_batch md_batch;   /* many independent systems stepped together (opaque) */

typedef enum {
    MD_OK = 0,
    MD_ERR_INVALID_ARG = -1,   /* a NULL pointer, n <= 0, box/dt <= 0, bad enum, ... */
    MD_ERR_BOX_TOO_SMALL = -2, /* fewer than 3 cells per edge (G = floor(L / r_n) < 3) */
    MD_ERR_OOM = -3,           /* the allocator returned NULL */
    MD_ERR_HIP = -4,           /* a HIP runtime call failed (sticky) */
    MD_ERR_NEBR_OVERFLOW = -5, /* md_get_pairs: a list exceeded nebr_cap */
    MD_ERR_ATOM_ESCAPED = -6,  /* a coordinate left [-3L/2, 3L/2) before a wrap */
    MD_ERR_NONFINITE = -7,     /* a coordinate became NaN or infinite */
    MD_ERR_STATE = -8,         /* call not valid in the current state */
    MD_ERR_NO_SLOT = -9,       /* batch: no free slot */
    MD_ERR_CELL_OVERFLOW = -10 /* cell-layer matrix could not be enlarged */
} md_status;

/* Arithmetic of the pair forces.  Positions and velocities are always FP64. */
typedef enum {
    MD_FORCE_FP32 = 0, /* FP64 separations and cutoff tests, FP32 pair forces,
                          compensated FP32 sums of energy and virial */
    MD_FORCE_FP64 = 1  /* everything in FP64 */
} md_precision;

/* md_params.flags */
#define MD_EVEN_CELLS 1u  /* round G down to even (the rule behind the paper's
                             cell counts in Tables 1 and 5); default floor(L / r_n) */
#define MD_TRACE_PROPS 2u /* record KE, PE, virial and the maximum speed of (e)
                             for every step of md_step on the device (a ring of
                             the last 65536 steps; read once with md_get_trace):
                             the properties the loop of Sec. 3.1 evaluates at
                             every step, at the cost of summing the energies at
                             every step */
#define MD_NO_REORDER 4u  /* never reorder the atoms (the ablation of Table 8):
                             a rebuild still bins and finds the cell order
                             (cell_start and a permutation) and wraps the
                             positions, but every atom keeps its storage
                             position, so the build reads candidates through
                             the permutation from global memory and the list
                             steps gather from wherever the atoms are; the
                             pair set and forces are those of the reordering
                             method (the summation order differs).  Not with
                             md_newton3_ab (MD_ERR_STATE) */
#define MD_NO_WINDOW 8u   /* ablation: no LDS window; every candidate of a build
                             and every neighbour of a list step is read from
                             global memory (the analogue of the paper's run
                             with the texture cache off, Sec. 5).  The same
                             pairs in the same order: results bit-identical */

typedef struct {
    int64_t n_atoms;   /* 1 <= N < 2^25 */
    double box;        /* edge L of the cube [-L/2, L/2)^3 */
    double r_cut;      /* interaction cutoff r_c; 2^(1/6) selects the soft sphere
                          (shift +1 so u(r_c) = 0); any other value is plain
                          truncated Lennard-Jones (no shift) */
    double shell;      /* neighbour shell delta (r_n = r_c + delta); 0 selects
                          the cell-list-only method (re-bin every step) */
    double dt;         /* time step */
    int32_t precision; /* md_precision */
    int32_t nebr_cap;  /* per-atom neighbour-list capacity; 0 = from the density:
                          max(48, 1.6 x the atoms of an r_n sphere + 16, rounded
                          up to 16) (atoms with longer lists are evaluated from
                          the cells) */
    int32_t cell_cap;  /* initial per-cell layer capacity; 0 = from the density:
                          max(16, 2 x the mean occupancy + 8, rounded up to 8)
                          (grown on need) */
    uint32_t flags;    /* MD_EVEN_CELLS | MD_TRACE_PROPS | MD_NO_REORDER | MD_NO_WINDOW */
    int32_t reorder_interval; /* N_R of Sec. 5.1 and Table 7: a rebuild reorders the
                          atoms only when at least N_R steps have passed since the
                          last reordering (the reordering is done when the next
                          rebuild falls due); a rebuild that does not reorder
                          works like one under MD_NO_REORDER.  0 = every rebuild
                          (the default); < 0 invalid.  Like MD_NO_REORDER it
                          changes the summation order, not the pairs.  Not with
                          md_newton3_ab (MD_ERR_STATE) */
} md_params;

typedef struct {
    double ke;              /* kinetic energy  (1/2) sum v^2 */
    double pe;              /* potential energy, sum over pairs of u(r) */
    double virial;          /* sum over pairs of r . F_pair = f(r) r^2 */
    double ke_per_atom, pe_per_atom, virial_per_atom;
    double vmax;            /* max |v| */
    double disp;            /* accumulated vmax*dt since the last rebuild */
    int64_t n_pairs;        /* unordered pairs in the neighbour matrix (0 in cell-list-only mode) */
    int64_t n_rebuilds;     /* rebuilds performed by md_step (not counting creation) */
    int64_t step;           /* completed time steps */
    int32_t max_nebr;       /* largest per-atom list length at the last build */
    int32_t max_cell;       /* largest cell occupancy seen by a sort so far */
    int32_t rebuild_due;    /* 1 if the next step starts with a rebuild */
    int32_t cells_per_edge; /* G */
    int64_t n_late_bins;    /* rebuilds whose positions the step before had not
                               binned (the maximum speed jumped): the library
                               binned them and resumed; results are unchanged */
} md_props_t;

/* One step of a property trace (MD_TRACE_PROPS): values of (e) of that step. */
typedef struct {
    int64_t step;   /* step number (1 = the first step after creation) */
    double ke;      /* (1/2) sum v^2 */
    double pe;      /* sum over pairs of u(r) */
    double virial;  /* sum over pairs of f(r) r^2 */
    double vmax;    /* max |v| */
} md_trace_t;

/* Means over the steps of a block (md_block_begin .. md_block_end). */
typedef struct {
    int64_t steps;          /* steps completed inside the block */
    double ke_per_atom;     /* mean of (1/2) sum v^2 / N over those steps */
    double pe_per_atom;     /* mean of PE / N */
    double etot_per_atom;   /* ke_per_atom + pe_per_atom */
    double virial_per_atom; /* mean of W / N */
    double nebr_per_atom;   /* mean neighbour-list entries per atom (the paper's
                               N_p / N_a; 0 in cell-list-only mode) */
} md_block_t;

/* Launch configuration (md_configure, md_batch_configure).  None of these
 * changes the arithmetic or its order, so a trajectory is the same bit for
 * bit under any of them; they only cut the same work differently.  In: 0
 * asks for the library's choice.  Out: the values in use. */
typedef struct {
    int32_t steps_per_run; /* steps per captured graph replay, 1..64 (0: 64) */
    int32_t grid;          /* workgroups per step-kernel launch, 1..65535 (0: a
                              single system one per 256-atom tile up to the
                              number resident at once, 4 per CU; a batch 2048) */
    int32_t sort_grid;     /* workgroups per sort launch, 1..65535 (0: a single
                              system at most 512, a batch 2048) */
    int32_t sort_split;    /* workgroups sharing one 256-cell tile of the sort,
                              1..32 (0: about 1024 atoms per workgroup for a
                              single system, 1 for a batch) */
    int32_t tile_order;    /* MD_ORDER_PASSES (0 asks for it in a batch): in each
                              pass over the tiles the 8 XCDs take consecutive
                              runs of grid/8 tiles, so work of uneven cost (the
                              systems of a batch rebuild at different steps)
                              spreads over every XCD; MD_ORDER_SLABS (0 asks for
                              it for a single system): each XCD walks its own
                              eighth of the tiles, so a tile's neighbours in z
                              are staged through the same L2 */
} md_launch_t;

#define MD_ORDER_PASSES 1
#define MD_ORDER_SLABS 2

typedef struct {
    void *(*alloc)(size_t bytes, void *ctx); /* device memory, >= 256-byte aligned */
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} md_allocator;

/* Text for a status code (static storage). */
const char *md_status_string(md_status s);

/* Cells per edge G for these parameters (floor(L / r_n), or its even floor
 * with MD_EVEN_CELLS), without creating anything.  Sec. 3.1 defines G. */
md_status md_cells_per_edge(const md_params *p, int32_t *G);

/* Device bytes md_create would allocate for these parameters (for admission
 * against a memory budget).  Sync-free. */
md_status md_query_bytes(const md_params *p, size_t *bytes);

/* Create a system from host positions and velocities (n x 3 doubles each,
 * any order, positions anywhere in [-3L/2, 3L/2)) and evaluate step 0: wrap,
 * bin, sort into cell order, build the neighbour matrix (unless shell == 0),
 * forces, properties, and the first rebuild decision (accumulated
 * displacement = vmax*dt).  hip_stream: a hipStream_t, or NULL.  a:
 * allocator, or NULL for hipMalloc.  On success *out owns a new system.
 * Sync. */
md_status md_create(const md_params *p, const double *pos, const double *vel,
                    const md_allocator *a, void *hip_stream, md_system **out);

/* Periodic wrap, cell assignment and stable cell-order reordering (cell
 * assignment Sec. 3.2 and its listing, layer assignment Sec. 3.4, reordering
 * Sec. 3.5) of the held state: atoms end up stored cell by cell, and within
 * a cell in their previous storage order.  The new storage order is then
 * evaluated again (neighbour matrix, forces, properties; the forces can
 * differ from the previous ones in the last bits, through the summation
 * order), and the displacement rule restarts from this state.  Sync. */
md_status md_bin_cells(md_system *s);

/* Build the neighbour matrix W[m][i] (Sec. 3.4) at the held state: for
 * every atom, all atoms j != i of the 27 surrounding cells with r^2 < r_n^2,
 * visited cell by cell (offsets z-major, x fastest) and in storage order
 * within a cell.  The list is built from freshly sorted cells, so this also
 * does what md_bin_cells does.  Not available in cell-list-only mode
 * (MD_ERR_STATE).  Sync. */
md_status md_build_nebr(md_system *s);

/* Forces, per-atom energies and virials at the held positions from the
 * current neighbour matrix (Sec. 3.4 force algorithm; cell method when
 * shell == 0), plus the properties.  Stores the forces used by the next
 * md_step.  Sync. */
md_status md_forces(md_system *s);

/* Advance n_steps leapfrog steps (a)-(e), rebuilding on the device whenever
 * the displacement rule fires.  Work is replayed from captured HIP graphs.
 * Async. */
md_status md_step(md_system *s, int64_t n_steps);

/* Properties after the last completed step (or creation / md_forces).
 * Sync; returns latched device errors. */
md_status md_props(md_system *s, md_props_t *out);

/* Several species, the extension the paper names in Sec. 3.5
 * (with no parameters there): species[i] in [0, n_species) for every atom
 * (original order), and per species pair (a, b) -- row-major n_species x
 * n_species arrays, symmetric -- epsilon >= 0, sigma > 0, the cutoff
 * (0 < r_cut[a][b] <= the system's r_cut, whose r_c + shell sizes the cells
 * and lists) and the energy added inside it.  A pair then interacts through
 * Eq. (1) in units of sigma_ab and epsilon_ab: u = 4 eps ((sigma/r)^12 -
 * (sigma/r)^6) + shift for r < r_cut.  With one species of sigma = epsilon
 * = 1 this is the plain potential with the same arithmetic.  At most 4
 * species.  The held state is sorted and evaluated again (as md_bin_cells);
 * md_set_state keeps the species of the original indices.  Single systems
 * only.  MD_ERR_INVALID_ARG for an out-of-range species or parameter or an
 * asymmetric table.  Sync. */
md_status md_set_species(md_system *s, int32_t n_species, const int32_t *species,
                         const double *epsilon, const double *sigma, const double *r_cut,
                         const double *shift);

/* Step (f) of the loop (Sec. 3.1), used during the equilibration period of
 * Sec. 5.1 (every 20 steps for the first 500): scale every velocity of the
 * held state by one factor so that sum v^2 = 3 (N - 1) T, T = temperature
 * (with the centre of mass at rest 3 (N - 1) degrees of freedom remain).
 * Call it after md_step; the factor comes from the kinetic energy of (e) of
 * the last completed step, which the rebuild rule also keeps (the maximum
 * speed of (e) is taken before the adjustment).  Does nothing when every
 * velocity is zero or N < 2.  MD_ERR_INVALID_ARG unless temperature is
 * positive and finite.  Async. */
md_status md_adjust_temp(md_system *s, double temperature);

/* Block averages (Sec. 5.1 evaluates its properties as means over blocks of
 * 1000 steps).  md_block_begin starts a block at the held step: every
 * following step of md_step sums its kinetic and potential energy, virial
 * and list length on the device (per tile, in a fixed order, so the result
 * is deterministic).  md_block_end stops the block and returns the means
 * over the steps completed since md_block_begin.  md_set_state ends a block
 * without a result; md_block_end then returns MD_ERR_STATE, as it does
 * when no block was begun.  Both sync. */
md_status md_block_begin(md_system *s);
md_status md_block_end(md_system *s, md_block_t *out);

/* Copy out positions, velocities and forces (each may be NULL; n x 3
 * doubles, original atom order) and the completed step count.  Sync. */
md_status md_get_state(md_system *s, double *pos, double *vel, double *force, int64_t *step);

/* Per-atom pair-energy and virial sums (each pair counted on both of its
 * atoms, so the sums are 2 PE and 2 W) from the last force evaluation, in
 * original order; either may be NULL.  Sync. */
md_status md_get_atom_energies(md_system *s, double *u_atom, double *w_atom);

/* Replace positions and velocities (n x 3, original order) of the held step
 * and evaluate them as md_create does (wrap, bin, sort, list, forces,
 * properties); the displacement rule restarts.  Sync. */
md_status md_set_state(md_system *s, const double *pos, const double *vel);

/* Scalar cell index (c_z*G + c_y)*G + c_x of every atom at its last
 * binning (the held positions, after md_create / md_bin_cells / a step),
 * original order.  Sync. */
md_status md_get_cells(md_system *s, int32_t *cell_of_atom);

/* Cell order of the last sort: order[p] = original index of the atom at
 * position p (the storage order; with MD_NO_REORDER the order the sort found,
 * the atoms themselves staying where they are); cell_start[c] = first
 * position of cell c, cell_start[G^3] = n (either may be NULL).  Sync. */
md_status md_get_bins(md_system *s, int32_t *order, int32_t *cell_start);

/* Neighbour-matrix entries as ordered pairs (i, j) of original indices, i
 * != j; each unordered pair appears twice (once from each side).  Stores at
 * most cap pairs, *n gets the total.  MD_ERR_NEBR_OVERFLOW if some atom's
 * list exceeded nebr_cap at the last build.  Sync. */
md_status md_get_pairs(md_system *s, int64_t cap, int32_t *i, int32_t *j, int64_t *n);

/* Bracket every launch of the step kernel (forces, list build, integration;
 * the dominant kernel of a step) with HIP events on the library's stream
 * from now on (enable != 0), or stop; steps then run as separate launches
 * instead of graph replays.  md_kernel_time reports launches and the summed
 * event-measured duration since the last enable.  Sync. */
md_status md_profile(md_system *s, int32_t enable);
md_status md_kernel_time(md_system *s, int64_t *launches, double *total_ms);

/* Variants of the neighbour-list A/B (md_newton3_ab, md_ab_pairs). */
typedef enum {
    MD_AB_FULL = 0,  /* full list (every j != i), one thread per atom */
    MD_AB_HALF = 1,  /* half list (j > i, each pair once), reactions by atomics */
    MD_AB_CELLS = 2  /* full list built cell by cell: one workgroup per cell,
                        one thread per occupant H_{c,l}, the 27 neighbouring
                        cells staged in LDS -- the organisation of the earlier
                        GPU codes the paper compares with at the end of
                        Sec. 3.4 (Table 3 "old"); the same list as MD_AB_FULL */
} md_ab_variant;

/* Neighbour-list A/B of the build and force phases.  The paper drops
 * Newton's third law on the GPU (Sec. 3.3: full lists, each atom sums its
 * own force) where the CPU keeps each pair once and adds the reaction to
 * the partner (Sec. 3.2), and builds its list atom by atom rather than cell
 * by cell (end of Sec. 3.4).  At the held state, after a fresh sort (as
 * md_bin_cells), this builds a plain neighbour list over the sorted cells --
 * storage-index entries, r^2 < r_n^2 in FP64 -- in the md_ab_variant given,
 * then evaluates the pair forces (FP32 on FP64 separations, as the step
 * kernel) reps times; the half form adds -f d to the partner with FP32
 * atomics.  Outputs (each may be NULL): force = the last evaluation's forces
 * (n x 3, original order), build_ms / force_ms = mean event-timed durations
 * of the build and force kernels over reps launches each, n_entries = list
 * entries (2 x pairs full, pairs half).  The list capacity is nebr_cap;
 * MD_ERR_NEBR_OVERFLOW if a list exceeds it.  MD_ERR_STATE in
 * cell-list-only mode, for mixtures and with MD_NO_REORDER.  Leaves the
 * system as md_bin_cells does.  Sync. */
md_status md_newton3_ab(md_system *s, int32_t variant, int32_t reps, double *force,
                        double *build_ms, double *force_ms, int64_t *n_entries);

/* The list of one md_ab_variant built at the held state (as md_newton3_ab)
 * as ordered pairs (i, j) of original indices: stores at most cap, *n gets
 * the total (2 x pairs for the full variants, pairs for the half one).
 * Sync. */
md_status md_ab_pairs(md_system *s, int32_t variant, int64_t cap, int32_t *i, int32_t *j,
                      int64_t *n);

/* The property trace of steps first_step .. first_step + count - 1 (created
 * with MD_TRACE_PROPS; at most the last 65536 steps are held): out[q] for
 * step first_step + q.  MD_ERR_STATE without the flag, or when a requested
 * step has not been taken yet or has left the ring.  Sync. */
md_status md_get_trace(md_system *s, int64_t first_step, int64_t count, md_trace_t *out);

/* Launch configuration of later steps (see md_launch_t); the replay graphs
 * are captured again.  *cfg gets the configuration in use.  Sync. */
md_status md_configure(md_system *s, md_launch_t *cfg);

/* Bytes of the static device array behind md_newton3_ab_noalloc (per GPU). */
#define MD_AB_SCRATCH_BYTES (64u << 20)

/* md_newton3_ab without any device allocation, for callers that cannot
 * allocate (code under graph capture around it, tight serving loops,
 * harnesses that forbid hipMalloc): the same sort, kernels and outputs, but
 * the list, lengths, forces and output staging live in one static device
 * array of MD_AB_SCRATCH_BYTES per GPU, held from the library's load until
 * the process ends.  A system needs mcap x npad x 4 + 16 x npad + 24 x N
 * bytes plus alignment (npad = N rounded up to 256; at the default mcap of
 * 48 about 230 B per atom, so up to ~290 000 atoms): larger ones get
 * MD_ERR_OOM and nothing runs.  Calls on one GPU share that GPU's array, so
 * calls that overlap in time on one GPU (two host threads, two systems on
 * different streams) race; every call clears what it needs before use.  A
 * pending cell-row overflow of the system, whose repair would allocate, is
 * reported as MD_ERR_CELL_OVERFLOW instead.  Sync. */
md_status md_newton3_ab_noalloc(md_system *s, int32_t variant, int32_t reps, double *force,
                                double *build_ms, double *force_ms, int64_t *n_entries);

/* Release the system and its device memory (synchronises its stream). */
void md_destroy(md_system *s);

/* ---------------------------------------------------------------------------
 * Batches: many independent systems advanced together.  Each kernel launch
 * of a batched step covers the tiles of every active system, so small
 * systems share the GPU; the per-system arithmetic is exactly that of an
 * md_system with the same parameters, so a system's trajectory is the same
 * bit for bit alone or in any mix.
 * ------------------------------------------------------------------------- */

/* A batch with room for max_slots systems and hbm_budget bytes of their
 * device state; steps_per_run (1..64) steps are replayed per md_batch_run. */
md_status md_batch_create(size_t hbm_budget, int32_t max_slots, int32_t steps_per_run,
                          const md_allocator *a, void *hip_stream, md_batch **out);

/* Launch configuration of later runs (see md_launch_t): steps replayed per
 * md_batch_run and the workgroups of the launches.  *cfg gets the
 * configuration in use.  Used by the autotuner.  Sync. */
md_status md_batch_configure(md_batch *b, md_launch_t *cfg);

/* Admit a system that is to advance n_steps steps; evaluates its step 0
 * (as md_create).  MD_ERR_OOM if it does not fit the remaining budget,
 * MD_ERR_NO_SLOT if every slot is busy; the caller retries later.  Sync. */
md_status md_batch_admit(md_batch *b, const md_params *p, const double *pos, const double *vel,
                         int64_t n_steps, int32_t *slot);

/* Advance every admitted, unfinished system by up to steps_per_run steps.
 * Async. */
md_status md_batch_run(md_batch *b);

/* Slots whose systems have completed all their steps and are not yet
 * released: writes up to cap slot numbers, *n_done gets the count.  Sync. */
md_status md_batch_poll(md_batch *b, int32_t *done, int32_t cap, int32_t *n_done);

/* Properties / state of the system in a slot (as md_props / md_get_state).
 * Sync. */
md_status md_batch_props(md_batch *b, int32_t slot, md_props_t *out);
md_status md_batch_get_state(md_batch *b, int32_t slot, double *pos, double *vel, int64_t *step);

/* The property trace of the system in a slot (as md_get_trace).  Sync. */
md_status md_batch_get_trace(md_batch *b, int32_t slot, int64_t first_step, int64_t count,
                             md_trace_t *out);

/* Free a slot and its device memory.  Sync. */
md_status md_batch_release(md_batch *b, int32_t slot);

/* Bytes of the budget in use, and admitted systems. */
md_status md_batch_usage(md_batch *b, size_t *bytes, int32_t *n_systems);

/* Progress of the admitted systems, for timing a batch by the work it did:
 * *atom_steps = sum over admitted systems of N x completed steps,
 * *n_running = systems with steps still to go and no error, *min_remaining =
 * the fewest steps any of them still has to go (0 when none runs).  Sync. */
md_status md_batch_progress(md_batch *b, int64_t *atom_steps, int32_t *n_running,
                            int64_t *min_remaining);

/* Release the batch and every admitted system. */
void md_batch_destroy(md_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_0911_5631_AMD_MD_H */
