// md_kernels.hip -- gfx950 kernels of the soft-sphere MD hot path.
//
// One time step k of every replica of an engine is two launches:
//   k_sort  (b) when the displacement rule fires (always with the plain cell
//           method): wrap, and a stable counting sort of the atoms by cell
//           (Secs. 3.4, 3.5) -- cell_start from the occupancy counts, ranks
//           from the cell-layer rows, scatter into the other buffer variant.
//           Replicas that do not rebuild leave at once.
//   k_step  (b) the neighbour matrix W from the contiguous cell ranges of
//           the sorted atoms when rebuilding; (c) forces from W (or from the
//           cells); (d), (e) second half kick, kinetic energy, maximum speed;
//           (a) of the next step: half kick and drift, and the binning of the
//           new positions into the next cell-layer set.
// Nothing waits for other workgroups inside a launch: the rebuild decision of
// step k is recomputed by every workgroup of k_sort from the maximum speed of
// step k-1 (one atomicMax per workgroup into a spread ring slot) and the
// displacement committed by step k-1, and committed for k_step by the
// workgroup of the replica's first cell tile, so no device-scope fence or
// "last block" finalisation is needed (on gfx950 a device-scope release writes
// back the whole L2).  Properties are reduced on demand (k_props) in a fixed
// order.
//
// Floating point: compiled with -ffp-contract=off, so every FP64 expression
// rounds as written (no fused multiply-add); cell indices and neighbour
// decisions are then the ones an FP64 CPU evaluation of the same expressions
// makes.
#include <hip/hip_runtime.h>

#include <limits.h>

#include <type_traits>

#include "md_device.h"
#include "md_kernels.h"

namespace md {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Global-address-space view of a pointer read from a descriptor: the loads
// and stores through it are global_* instructions instead of flat_* ones
// (which also count against the LDS wait counter).
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gp(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}
typedef const __attribute__((address_space(1))) double *gcdouble;
typedef const __attribute__((address_space(1))) int32_t *gcint;

// Replica descriptors are written by the host only, between launches: read
// through the constant address space their fields are scalar loads held in
// SGPRs (a wave-uniform descriptor) instead of vector loads into VGPRs.
typedef const __attribute__((address_space(4))) SlotDev SlotC;
__device__ __forceinline__ SlotC &slot(const Tables &T, int idx) {
  return *(SlotC *)(T.slots + idx);
}
// The same view of other host-written tables, and of control words that a
// kernel reads while no workgroup of the same launch writes them.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *cview(const T *p) {
  return (const __attribute__((address_space(4))) T *)p;
}

// Workgroups go to the 8 XCDs round-robin; renumber them so that each XCD
// walks a contiguous range of tiles and neighbouring atoms share an L2.
__device__ __forceinline__ int xcd_block(int b, int g) {
  if ((g & 7) == 0) return (b & 7) * (g >> 3) + (b >> 3);
  return b;
}

// The tiles workgroup b of g takes in a launch over n tiles (t = first;
// t < end; t += step).  ORDER_PASSES: in pass p the 8 XCDs take consecutive
// runs of g/8 tiles, XCD x the x-th run of the pass.  ORDER_SLABS: XCD x
// takes the x-th eighth of all tiles and its workgroups walk it together,
// g/8 tiles at a time, so the neighbour rows of a tile in z (the halo of its
// window) are staged by the same XCD shortly before or after it, while its
// L2 still holds them.  Both visit every tile exactly once.
struct TileWalk {
  int t, step, end;
  __device__ __forceinline__ TileWalk(int b, int g, int n, int order) {
    if ((g & 7) != 0) {
      t = b;
      step = g;
      end = n;
    } else if (order == ORDER_SLABS) {
      const int per = (n + 7) >> 3;
      t = (b & 7) * per + (b >> 3);
      step = g >> 3;
      end = min(n, ((b & 7) + 1) * per);
    } else {
      t = (b & 7) * (g >> 3) + (b >> 3);
      step = g;
      end = n;
    }
  }
};

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Maximum over the wave of a 64-bit unsigned value, in every lane: DPP row
// shifts within rows of 16 lanes, then row broadcasts (ALU only, no LDS
// round trips); lanes that have no source keep their own value.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_max_step(unsigned long long v) {
  const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
  const uint32_t slo = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
  const uint32_t shi = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
  const unsigned long long o = ((unsigned long long)shi << 32) | slo;
  return o > v ? o : v;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  v = dpp_max_step<0x111, 0xF>(v);  // row_shr:1
  v = dpp_max_step<0x112, 0xF>(v);  // row_shr:2
  v = dpp_max_step<0x114, 0xF>(v);  // row_shr:4
  v = dpp_max_step<0x118, 0xF>(v);  // row_shr:8: lane 15 of a row holds the row maximum
  v = dpp_max_step<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_max_step<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3: lane 63 holds all
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

// Compensated FP32 pair (value, error) and exact TwoSum combination.
struct F2 {
  float hi, lo;
};
__device__ __forceinline__ F2 f2_add(F2 a, F2 b) {
  float s = a.hi + b.hi;
  float bp = s - a.hi;
  float e = (a.hi - (s - bp)) + (b.hi - bp);
  return F2{s, (a.lo + b.lo) + e};
}
__device__ __forceinline__ F2 wave_sum_f2(F2 v) {
  for (int o = 32; o > 0; o >>= 1) {
    F2 w{__shfl_xor(v.hi, o, 64), __shfl_xor(v.lo, o, 64)};
    v = f2_add(v, w);
  }
  return v;
}

__device__ __forceinline__ int64_t mod3(int64_t k) { return ((k % 3) + 3) % 3; }

// Periodic wrap into [-L/2, L/2) (exact: Sterbenz) -- idempotent.
__device__ __forceinline__ double wrap1(double x, double L, double halfL) {
  if (x >= halfL) return x - L;
  if (x < -halfL) return x + L;
  return x;
}

// (int)((x + L/2) * invW) clamped to [0, G-1]; the clamp is applied before the
// conversion (same result for every finite x, no out-of-range conversion).
__device__ __forceinline__ int cell_coord(double x, double halfL, double invW, int G) {
  const double q = (x + halfL) * invW;
  return (int)fmin(fmax(q, 0.0), (double)(G - 1));
}

__device__ __forceinline__ int cell_of(SlotC &S, double x, double y, double z) {
  const int G = S.G;
  return (cell_coord(z, S.halfL, S.invW, G) * G + cell_coord(y, S.halfL, S.invW, G)) * G +
         cell_coord(x, S.halfL, S.invW, G);
}

// Descriptor of the state a replica holds between launches (r(done), or the
// drifted r(done+1), which lives in the same variant).
__device__ __forceinline__ SlotC &slot_held(const Tables &T, int r) {
  const CtlDev &C = T.ctl[r];
  return slot(T, 2 * r + C.var_ring[mod3(C.done)]);
}

// State index held by a replica between launches.
__device__ __forceinline__ int64_t cur_state(const CtlDev &C) {
  return C.clean ? C.done : C.done + 1;
}

__device__ __forceinline__ void latch_error(CtlDev &C, int bits, int64_t step) {
  atomicOr(&C.err, bits);
  atomicMin((unsigned long long *)&C.err_step, (unsigned long long)step);
}

// A new position of step `step`: latch an error for a non-finite coordinate
// or one outside [-3L/2, 3L/2) (the wrap at the next rebuild could not bring
// it back); returns false for a non-finite one.
__device__ __forceinline__ bool check_atom(SlotC &S, CtlDev &C, double x, double y, double z,
                                           int64_t step) {
  int bad = 0;
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
    bad = ERR_NONFINITE;
  } else if (fabs(x) >= 3.0 * S.halfL || fabs(y) >= 3.0 * S.halfL || fabs(z) >= 3.0 * S.halfL) {
    bad = ERR_ESCAPED;
  }
  if (bad) latch_error(C, bad, step);
  return bad != ERR_NONFINITE;
}

// Cell and layer assignment of one atom (Secs. 3.2, 3.4): the atom's cell
// from its wrapped coordinates, a layer slot from the cell's occupancy
// counter (atomic), the row entry, or the set's overflow list beyond hcap.
// The sort of a rebuild step reads the rows; the cell each atom lands in
// there is written by the sort itself.
__device__ __forceinline__ void bin_atom(SlotC &S, CtlDev &C, int set, int i, double x, double y,
                         double z, int64_t step) {
  // Called by a prefix of the lanes of a wave (the active atoms of a tile).
  if (!check_atom(S, C, x, y, z, step)) x = y = z = 0.0;
  const int c = cell_of(S, wrap1(x, S.L, S.halfL), wrap1(y, S.L, S.halfL), wrap1(z, S.L, S.halfL));
  // Consecutive lanes with the same cell take their layer slots with one
  // atomic: atoms are stored in cell order, so most of a cell's atoms are
  // neighbours in a wave.
  // (the empty asm keeps the lane masks below from being hoisted out of the
  // tile loop, where they would be held across it and spilled)
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
  const unsigned long long active = __ballot(1);
  const int na = __popcll(active);
  const int cp = __shfl_up(c, 1, 64);
  const bool leader = lane == 0 || cp != c;
  const unsigned long long lmask = __ballot(leader) & active;
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
  const int lead = 63 - __clzll(lmask & upto);
  const unsigned long long after = lmask & ~upto;
  const int next = after ? __ffsll((long long)after) - 1 : na;
  int base = 0;
  if (leader) base = atomicAdd(&S.cnt[set][c], next - lane);
  const int slot = __shfl(base, lead, 64) + (lane - lead);
  // the occupancy of the cell's tile, one atomic per run of lanes in one tile
  // (the shuffle runs on every active lane: a lane reading from an inactive
  // one gets 0)
  const int ct = c / CTILE;
  const int ctp = __shfl_up(ct, 1, 64);
  const bool tlead = lane == 0 || ctp != ct;
  const unsigned long long tmask = __ballot(tlead) & active;
  const unsigned long long tafter = tmask & ~upto;
  const int tnext = tafter ? __ffsll((long long)tafter) - 1 : na;
  if (tlead) atomicAdd(&S.tcnt[set][ct], tnext - lane);
  if (slot < S.hcap) {
    gp(S.H[set])[(size_t)c * S.hcap + slot] = i;
  } else {
    const int o = atomicAdd(&S.ovf_n[set], 1);
    if (o < OVF_CAP) {
      S.ovf[set][2 * o] = c;
      S.ovf[set][2 * o + 1] = i;
    } else {
      latch_error(C, ERR_CELL, step);
    }
  }
}

#define MD_CX(p, q)                             \
  {                                             \
    const int lo_ = min(p, q), hi_ = max(p, q); \
    p = lo_;                                    \
    q = hi_;                                    \
  }
// Compare-exchange network ordering eight values (Batcher odd-even merge).
__device__ __forceinline__ void sort8(int (&v)[8]) {
  MD_CX(v[0], v[1]) MD_CX(v[2], v[3]) MD_CX(v[4], v[5]) MD_CX(v[6], v[7])
  MD_CX(v[0], v[2]) MD_CX(v[1], v[3]) MD_CX(v[4], v[6]) MD_CX(v[5], v[7])
  MD_CX(v[1], v[2]) MD_CX(v[5], v[6])
  MD_CX(v[0], v[4]) MD_CX(v[1], v[5]) MD_CX(v[2], v[6]) MD_CX(v[3], v[7])
  MD_CX(v[2], v[4]) MD_CX(v[3], v[5])
  MD_CX(v[1], v[2]) MD_CX(v[3], v[4]) MD_CX(v[5], v[6])
}
#undef MD_CX

// Visit the atoms of cell c (occupancy cnt) of a set in ascending storage
// index, passing each one's rank (the order of the row entries themselves
// depends on atomic timing, so it is not used).  Up to eight atoms held in
// the row are ordered with a sorting network; larger or overflowing cells
// take repeated minimum searches over the row and the set's overflow list.
template <class Visit>
__device__ __forceinline__ void visit_cell(SlotC &S, int set, int c, int cnt,
                                           Visit &&visit) {
  const int32_t *__restrict__ row = S.H[set] + (size_t)c * S.hcap;
  const int inrow = min(cnt, S.hcap);
  if (cnt <= 8 && inrow == cnt) {
    int v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = e < cnt ? gp(row)[e] : INT_MAX;
    sort8(v);
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (e < cnt) visit(v[e], e);
    return;
  }
  int last = -1;
  for (int r = 0; r < cnt; ++r) {
    int best = INT_MAX;
    for (int e = 0; e < inrow; ++e) {
      const int v = gp(row)[e];
      best = (v > last && v < best) ? v : best;
    }
    if (cnt > inrow) {
      const int no = min(S.ovf_n[set], OVF_CAP);
      const int32_t *__restrict__ ov = S.ovf[set];
      for (int e = 0; e < no; ++e)
        if (ov[2 * e] == c) {
          const int v = ov[2 * e + 1];
          best = (v > last && v < best) ? v : best;
        }
    }
    if (best == INT_MAX) break;
    last = best;
    visit(best, r);
  }
}

// Maximum of the spread slots of ring entry e (each wave reads all slots;
// every lane loads, the upper half the same slots again, and those copies
// count as zero: no lane-dependent branch for the loads to wait behind).  A
// slot without a replica has no ring and reads as zero.
static_assert((VSPREAD & (VSPREAD - 1)) == 0 && VSPREAD <= 64, "VSPREAD: a power of two");
__device__ __forceinline__ double ring_max(SlotC &S, int64_t e) {
  const int l = threadIdx.x & 63;
  double v = 0.0;
  if (S.vring != nullptr)
    v = __longlong_as_double((long long)S.vring[(e * VSPREAD + (l & (VSPREAD - 1))) * 16]);
  return wave_max(l < VSPREAD ? v : 0.0);
}

// The same for all three ring entries at once: the loads do not wait for the
// step number that selects an entry.  A slot without a replica has no ring
// and reads as zero.
__device__ __forceinline__ void ring_max3(SlotC &S, double (&v)[3]) {
  const int l = threadIdx.x & 63;
  double a[3] = {0.0, 0.0, 0.0};
  if (l < VSPREAD && S.vring != nullptr)
    for (int e = 0; e < 3; ++e)
      a[e] = __longlong_as_double((long long)S.vring[(e * VSPREAD + l) * 16]);
  for (int e = 0; e < 3; ++e) v[e] = wave_max(a[e]);
}

// Entry e (0, 1 or 2) of three values held in registers.
template <class X>
__device__ __forceinline__ X pick3(X a0, X a1, X a2, int64_t e) {
  return e == 0 ? a0 : e == 1 ? a1 : a2;
}

// Whether r(k) is binned during step k-1, so that a sort at step k finds its
// rows (binning every step would cost a step's worth of atomics and row
// writes where a rebuild comes about one step in ten).  Always with the cell
// method and at a forced rebuild; otherwise when the displacement rule of
// rebuild_rule, accumulated with BIN_AHEAD times the maximum speed of step
// k-2 (that of step k-1 is not known while step k-1 runs), would fire at
// step k.  The sort of step k-1, which holds every input of the rule, takes
// this decision for the step kernel of step k-1 (CtlDev::bin_ring); the sort
// of step k evaluates the same expression from the same committed words, so
// it knows whether the rows exist; when the rule fires
// without them (the maximum speed grew by more than BIN_AHEAD in one step)
// it latches ERR_UNBINNED and the host bins r(k) and resumes, so the
// trajectory does not depend on the guess.  Called by whole waves.
// bins_rule takes the words already read: D2 the committed displacement
// after step k-2, V2 the maximum v^2 of step k-2.
__device__ __forceinline__ bool bins_rule(const SlotC &S, int64_t force_step, int64_t k,
                                          double D2, double V2) {
  if (S.cell_only || k == force_step) return true;
  const bool rb1 = (k - 1 == force_step) || D2 > S.half_shell;
  const double D1 = (rb1 ? 0.0 : D2) + BIN_AHEAD * sqrt(V2) * S.dt;
  return D1 > S.half_shell;
}
template <class Ctl>
__device__ __forceinline__ bool bins_due(SlotC &S, const Ctl &C, int64_t k) {
  const double D2 = C.disp_ring[mod3(k - 2)];
  const double V2 = ring_max(S, mod3(k - 2));
  return bins_rule(S, C.force_step, k, D2, V2);
}

// Rebuild decision for step k (Sec. 3.1): rebuilt when the accumulated sum
// of vmax*dt exceeds delta/2.  disp after step k-1 is recomputed from the
// committed disp after step k-2 (D2) and vmax^2 of step k-1 (V1); *disp1
// receives it.
__device__ __forceinline__ bool rebuild_rule(const SlotC &S, int64_t force_step, int64_t k,
                                             double D2, double V1, double *disp1) {
  const bool rb1 = (k - 1 == force_step) || D2 > S.half_shell;
  const double D1 = (rb1 ? 0.0 : D2) + sqrt(V1) * S.dt;
  *disp1 = D1;
  return (k == force_step) || D1 > S.half_shell;
}

// ---------------------------------------------------------------------------
// (a): first half kick and drift of a clean replica, and binning of r(k+1)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TILE) void k_kick(Tables T) {
  const int nt = T.hdr[HDR_NTILES];
  for (int t = xcd_block(blockIdx.x, gridDim.x); t < nt; t += gridDim.x) {
    const int r = T.tile_rep[t];
    if (slot(T, 2 * r).n <= 0) continue;
    SlotC &S = slot_held(T, r);
    CtlDev &C = T.ctl[r];
    // errors latched by this launch (err_step = done + 1) do not stop it
    if ((C.err != 0 && C.err_step <= C.done) || !C.clean || C.done >= C.target) continue;
    const int64_t k = C.done;
    const bool bin = bins_due(slot(T, 2 * r), C, k + 1);
    const int i = (t - S.tile_off) * TILE + threadIdx.x;
    if (i >= S.n) continue;
    const int pb = (int)(k & 1), vb = (int)((k + 1) & 1);
    double f[3];
    for (int a = 0; a < 3; ++a)
      f[a] = S.fp64 ? gp((const double *)S.F)[a * S.npad + i]
                    : (double)gp((const float *)S.F)[a * S.npad + i];
    double xn[3];
    for (int a = 0; a < 3; ++a) {
      const double v = gp(S.V[vb][a])[i] + S.hdt * f[a];
      gp(S.V[vb][a])[i] = v;
      xn[a] = gp(S.P[pb][a])[i] + S.dt * v;
      gp(S.P[pb ^ 1][a])[i] = xn[a];
    }
    if (bin)
      bin_atom(S, C, (int)mod3(k + 1), i, xn[0], xn[1], xn[2], k + 1);
    else
      check_atom(S, C, xn[0], xn[1], xn[2], k + 1);
  }
}

// After k_kick: the kicked replicas hold a drifted state (one thread per
// replica; same gate as the kick).
__global__ void k_kick_end(Tables T) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= T.nslots) return;
  CtlDev &C = T.ctl[r];
  if (slot(T, 2 * r).n <= 0) return;
  if ((C.err != 0 && C.err_step <= C.done) || !C.clean || C.done >= C.target) return;
  C.clean = 0;
}

// ---------------------------------------------------------------------------
// (b): the counting sort by cell
// ---------------------------------------------------------------------------
// Workgroup t of a replica takes cell tile t (CTILE cells, one per thread):
// cell_start of the tile's first cell is the sum of the occupancies of the
// earlier tiles (counted while binning), cell_start of its cells follows
// from a workgroup scan, and every atom goes to cell_start of its cell plus
// its rank among the cell's atoms by current storage index -- the sequential
// layer assignment of Sec. 3.4 read in cell order (Sec. 3.5), i.e. a stable
// counting sort.  Positions are wrapped on the way (Sec. 3.1, step (b)).
// Workgroups depend on nobody.
//   mode == MODE_STEP: step k = base + s + 1 of a run; replicas whose rule
//   does not fire leave; v(k-1/2) is carried.
//   otherwise: the held clean state (k = done); v(k) is carried; k_flip
//   switches the variant afterwards.
__global__ __launch_bounds__(TILE) void k_sort(Tables T, int s, int mode, int only) {
  __shared__ int s_red[4];
  __shared__ int s_wsum[4];
  __shared__ int s_bsum[4];
  __shared__ int s_bc[TILE], s_bb[TILE], s_bp[TILE];
  // the decision for a replica is launch-invariant: a workgroup works it out
  // once for a run of consecutive cell tiles of one replica
  int rc = -1, var = 0;
  int64_t k = 0;
  bool skip = true, rebuild = false, unbinned = false, reo = true;
  double d1 = 0.0;
  // the atoms in a replica's tiles before tile run_upto (see below)
  int run_rep = -1, run_upto = 0, run_pre = 0;
  // one replica: every unit is replica 0's
  const bool solo = T.nslots == 1;
  // last reordering before step k, and whether step k bins r(k+1) (MODE_STEP)
  int64_t reo1 = 0;
  bool bin1 = false;
  // works out the decision for replica r; leaves skip set when the launch
  // has nothing to do for it
  auto decide = [&](int r) {
    CtlDev &C = T.ctl[r];
    SlotC &S0 = slot(T, 2 * r);
    rc = r;
    skip = true;
    if (only >= 0 && r != only) return;
    if (mode == MODE_STEP) {
      // every word the rule reads is loaded before any is tested: an idle
      // launch is this evaluation, and tested one after another the words
      // were a chain of dependent loads
      const int64_t base = C.base, target = C.target, err_step = C.err_step;
      const int64_t force_step = C.force_step, bins_step = C.bins_step;
      const int32_t err = C.err;
      const int64_t ro0 = C.reo_ring[0], ro1 = C.reo_ring[1], ro2 = C.reo_ring[2];
      const double dp0 = C.disp_ring[0], dp1 = C.disp_ring[1], dp2 = C.disp_ring[2];
      const int32_t vr0 = C.var_ring[0], vr1 = C.var_ring[1], vr2 = C.var_ring[2];
      double vm[3];
      ring_max3(S0, vm);
      k = base + s + 1;
      const int64_t e1 = mod3(k - 1), e2 = mod3(k - 2);
      const double D2 = pick3(dp0, dp1, dp2, e2);
      var = pick3(vr0, vr1, vr2, e1);
      reo1 = pick3(ro0, ro1, ro2, e1);
      rebuild = true;
      d1 = 0.0;
      const double V1 = pick3(vm[0], vm[1], vm[2], e1);
      if (!S0.cell_only) rebuild = rebuild_rule(S0, force_step, k, D2, V1, &d1);
      unbinned = rebuild && !bins_rule(S0, force_step, k, D2, pick3(vm[0], vm[1], vm[2], e2)) &&
                 k != bins_step;
      // the step kernel's binning ahead for step k + 1 (see bins_due): the
      // rule of step k + 1 from the displacement after step k-1 (d1, which
      // this launch commits) and the maximum speed of step k-1
      bin1 = k != target && bins_rule(S0, force_step, k + 1, d1, V1);
      // reorder at this rebuild, or keep the storage order (Table 7: the
      // reordering is done at the first rebuild N_R steps after the last)
      reo = !S0.noreo && (S0.nr <= 0 || k - reo1 >= S0.nr);
      if (k > target || (err != 0 && err_step <= k)) return;
    } else {
      if (!C.clean) return;
      k = C.done;
      if (C.err != 0 && C.err_step <= k) return;
      var = C.var_ring[mod3(k)];
      rebuild = true;
      unbinned = false;
      reo = !S0.noreo;  // a sort of the held state reorders (k_flip records it)
    }
    skip = false;
  };
  if (solo) {
    // (needs no table read, so it overlaps the header's loads) with nothing
    // to sort in this launch only the workgroup of unit 0 has work: it
    // records the decision
    decide(0);
    if (skip || (mode == MODE_STEP && (!rebuild || unbinned) &&
                 xcd_block(blockIdx.x, gridDim.x) != 0))
      return;
  }
  const int nct = cview(T.hdr)[HDR_NCTILES];
  // a cell tile is shared by nsp workgroups (dense systems, whose cells hold
  // many atoms); unit u = (tile u / nsp, share u % nsp)
  const int nsp = max(cview(T.hdr)[HDR_SPLIT], 1);
  const int nunits = nct * nsp;
  for (int u = xcd_block(blockIdx.x, gridDim.x); u < nunits; u += gridDim.x) {
    const int t = u / nsp, sp = u - t * nsp;
    const int r = solo ? 0 : cview(T.ctile_rep)[t];
    CtlDev &C = T.ctl[r];
    SlotC &S0 = slot(T, 2 * r);
    if (r != rc) decide(r);
    // one replica: its units are all the launch has, so a workgroup with
    // nothing to do for it stops instead of visiting its other units (an
    // idle launch then costs one unit per workgroup)
    if (skip) {
      if (solo) break;
      continue;
    }
    if (mode == MODE_STEP) {
      if (t == S0.ctile_off && sp == 0 && threadIdx.x == 0) {
        // the one writer of these ring slots for step k (with one replica
        // that is unit 0, the first unit of its workgroup, so no workgroup
        // stops before it); a step whose rows are missing is stopped here
        // and done again once the host has binned it
        if (unbinned) {
          latch_error(C, ERR_UNBINNED, k);
        } else {
          C.rb_ring[mod3(k)] = rebuild ? (reo ? RB_REORDER : RB_PERM) : RB_NONE;
          C.bin_ring[mod3(k)] = bin1 ? 1 : 0;
          C.reo_ring[mod3(k)] = rebuild && reo ? k : reo1;
          if (!S0.cell_only) {
            C.disp_ring[mod3(k - 1)] = d1;
            if (rebuild && k != C.force_step) C.n_rebuilds += 1;
          }
        }
      }
      if (!rebuild || unbinned) {
        if (solo) break;
        continue;
      }
    }
    SlotC &S = slot(T, 2 * r + var);
    SlotC &D = slot(T, 2 * r + (var ^ 1));
    const int set = (int)mod3(k);
    const int pb = (int)(k & 1);
    const int vb = mode == MODE_STEP ? pb : pb ^ 1;
    const int lt = t - S.ctile_off;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;

    // atoms in the earlier tiles: a workgroup takes its units in increasing
    // order, so the sum kept from its previous unit of the same replica only
    // grows by the tiles in between (about the grid's size; O(tiles) loads
    // per workgroup instead of every earlier tile at every unit).  Eight
    // loads in flight per thread: integer sums, so the grouping does not
    // change the result.
    const auto TC = gp((const int32_t *)S.tcnt[set]);
    if (run_rep != r || run_upto > lt) {
      run_rep = r;
      run_upto = 0;
      run_pre = 0;
    }
    int pre = 0;
    {
      int q = run_upto + (int)threadIdx.x;
      for (; q + 7 * TILE < lt; q += 8 * TILE) {
        int p8[8];
#pragma unroll
        for (int u8 = 0; u8 < 8; ++u8) p8[u8] = TC[q + u8 * TILE];
#pragma unroll
        for (int u8 = 0; u8 < 8; ++u8) pre += p8[u8];
      }
      for (; q < lt; q += TILE) pre += TC[q];
    }
    for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o, 64);
    if (l == 0) s_red[w] = pre;

    // workgroup exclusive scan of one cell count per thread
    const int c = lt * CTILE + threadIdx.x;
    const int cnt = c < S.ncell ? gp(S.cnt[set])[c] : 0;
    int incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o, 64);
      if (l >= o) incl += y;
    }
    if (l == 63) s_wsum[w] = incl;
    const int wmax = wave_max_i(cnt);
    __syncthreads();
    run_pre += ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
    run_upto = lt;
    int before = run_pre;
    for (int q = 0; q < w; ++q) before += s_wsum[q];
    const int base = before + incl - cnt;
    if (sp == 0) {
      if (l == 0 && wmax > C.max_h) atomicMax(&C.max_h, wmax);
      if (c <= S.ncell) gp(S.cs)[c] = base;  // c == ncell: the total, n
    }

    // every atom goes to base of its cell + its rank by current index
    const int n = S.n;
    const double L = S.L, halfL = S.halfL;
    const bool mixsp = S.nsp > 0;  // a mixture: the species move with the atoms
    const bool noreo = !reo;
    auto move = [&](int a, int cc, int p) {
      if (p >= n || a < 0 || a >= n) return;  // inconsistent counts: never expected
      if (noreo) {
        // no reordering: position p of cell order refers to the atom where
        // it is; it is wrapped in place (read and written by this thread only)
        gp(S.perm)[p] = a;
        gp(S.cell)[a] = cc;
#pragma unroll
        for (int d = 0; d < 3; ++d) gp(S.P[pb][d])[a] = wrap1(gp(S.P[pb][d])[a], L, halfL);
        return;
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        gp(D.P[pb][d])[p] = wrap1(gp(S.P[pb][d])[a], L, halfL);
        gp(D.V[vb][d])[p] = gp(S.V[vb][d])[a];
      }
      gp(D.id)[p] = gp(S.id)[a];
      gp(D.cell)[p] = cc;
      if (mixsp) gp(D.sp)[p] = gp(S.sp)[a];
    };
    // cells of up to eight atoms (the usual ones) by the thread that holds
    // them: a sorting network, then moves four at a time with every load of
    // a batch issued before its stores; with shares, thread i of share i %
    // nsp
    const bool big = c < S.ncell && cnt > 8 && cnt <= min(S.hcap, 8191);
    if (c < S.ncell && cnt > 0 && !big && threadIdx.x % nsp == sp) {
      if (cnt <= 8 && cnt <= S.hcap && !noreo) {
        const int32_t *row = S.H[set] + (size_t)c * S.hcap;
        int v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = e < cnt ? gp(row)[e] : INT_MAX;
        sort8(v);
#pragma unroll
        for (int b = 0; b < 8; b += 4) {
          if (b < cnt) {
            double pv[4][6];
            int idv[4], spv[4];
#pragma unroll
            for (int u4 = 0; u4 < 4; ++u4) {
              const int a = min(max(b + u4 < cnt ? v[b + u4] : v[0], 0), n - 1);
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                pv[u4][d] = gp(S.P[pb][d])[a];
                pv[u4][3 + d] = gp(S.V[vb][d])[a];
              }
              idv[u4] = gp(S.id)[a];
              spv[u4] = mixsp ? gp(S.sp)[a] : 0;
            }
#pragma unroll
            for (int u4 = 0; u4 < 4; ++u4) {
              const int p = base + b + u4, a = v[b + u4];
              if (b + u4 >= cnt || p >= n || a < 0 || a >= n) continue;
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                gp(D.P[pb][d])[p] = wrap1(pv[u4][d], L, halfL);
                gp(D.V[vb][d])[p] = pv[u4][3 + d];
              }
              gp(D.id)[p] = idv[u4];
              gp(D.cell)[p] = c;
              if (mixsp) gp(D.sp)[p] = spv[u4];
            }
          }
        }
      } else {
        // a cell that spilled into the overflow list (repeated minimum
        // searches), and every cell without reordering
        visit_cell(S, set, c, cnt, [&](int a, int q) { move(a, c, base + q); });
      }
    }
    // larger cells whose members all sit in their rows, by the whole
    // workgroup: their atoms are listed (big cell j holds entries
    // s_bp[j] ... of the list), this share takes its slice, and each atom's
    // rank is the number of smaller indices in its row
    if (__syncthreads_or(big)) {
      const int bv = big ? ((1 << 21) | cnt) : 0;  // (cell count, atom count)
      int binc = bv;
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(binc, o, 64);
        if (l >= o) binc += y;
      }
      if (l == 63) s_bsum[w] = binc;
      __syncthreads();
      int bbefore = 0;
      for (int q = 0; q < w; ++q) bbefore += s_bsum[q];
      const int bex = bbefore + binc - bv;
      if (big) {
        const int j = bex >> 21;
        s_bc[j] = c;
        s_bb[j] = base;
        s_bp[j] = bex & ((1 << 21) - 1);
      }
      const int btot = ((s_bsum[0] + s_bsum[1]) + s_bsum[2]) + s_bsum[3];
      const int nb = btot >> 21, B = btot & ((1 << 21) - 1);
      __syncthreads();
      const int a0 = (int)((int64_t)B * sp / nsp), a1 = (int)((int64_t)B * (sp + 1) / nsp);
      for (int a = a0 + (int)threadIdx.x; a < a1; a += TILE) {
        int lo = 0, hi = nb - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_bp[mid] <= a) lo = mid;
          else hi = mid - 1;
        }
        const int cj = s_bc[lo];
        const int cntj = (lo + 1 < nb ? s_bp[lo + 1] : B) - s_bp[lo];
        const auto row = gp((const int32_t *)S.H[set]) + (size_t)cj * S.hcap;
        const int v = row[a - s_bp[lo]];
        int rank = 0;
        for (int f = 0; f < cntj; ++f) rank += row[f] < v ? 1 : 0;
        move(v, cj, s_bb[lo] + rank);
      }
    }
    __syncthreads();
  }
}

// After a sort of the held states (mode != MODE_STEP): switch the replicas
// that were sorted to their other variant (same gate as k_sort).
__global__ void k_flip(Tables T, int only) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= T.nslots || (only >= 0 && r != only)) return;
  if (slot(T, 2 * r).n <= 0) return;
  CtlDev &C = T.ctl[r];
  if (!C.clean || slot(T, 2 * r).noreo) return;  // no reordering: nothing moved
  const int64_t k = C.done;
  if (C.err != 0 && C.err_step <= k) return;
  C.var_ring[mod3(k)] ^= 1;
  C.ord_ring[mod3(k)] = 0;  // the held state is in cell order again
  C.reo_ring[mod3(k)] = k;
}

// ---------------------------------------------------------------------------
// (b)-(e) and the next (a): the step kernel
// ---------------------------------------------------------------------------
template <typename R>
struct Acc {
  R fx, fy, fz, u, w;
};

// FP32 1/s: the hardware reciprocal (within 1 ulp) refined by one Newton step
// (two explicit FMAs), which brings it to about half an ulp.  The refinement
// matters where every pair has the same separation (a lattice): a reciprocal
// 1 ulp off then shifts every pair's virial term by ~2e-6 relative through
// the cancellation in r^-6 - 1/2, and the shift does not average out.
__device__ __forceinline__ float recip(float s) {
  const float r = __builtin_amdgcn_rcpf(s);
  return __builtin_fmaf(r, __builtin_fmaf(-s, r, 1.0f), r);
}
__device__ __forceinline__ double recip(double s) { return 1.0 / s; }

// Pair force and energy of Eq. (1) with the soft-sphere shift: for r^2 = s,
// f = 48 r^-8 (r^-6 - 1/2) (force on i is f d), u = 4 r^-6 (r^-6 - 1) + shift.
// FP32 uses the refined hardware reciprocal above.
// The energy and virial terms are summed only when ENERGY is set (a
// wave-uniform flag: the steps whose per-atom sums somebody reads); the
// force arithmetic is the same either way.
template <typename R>
__device__ __forceinline__ void pair_accum(Acc<R> &a, double dx, double dy, double dz, double s,
                                           R ushift, bool energy) {
  const R sr = (R)s;
  const R rri = recip(sr);
  const R rri3 = rri * rri * rri;
  const R f = (R)48 * rri3 * (rri3 - (R)0.5) * rri;
  a.fx += f * (R)dx;
  a.fy += f * (R)dy;
  a.fz += f * (R)dz;
  if (energy) {
    a.u += (R)4 * rri3 * (rri3 - (R)1) + ushift;
    a.w += f * sr;
  }
}

// The same for species pair k of a mixture: Eq. (1) in units of sigma_ab and
// epsilon_ab, r^-2 scaled by sigma^2 (with sigma = epsilon = 1 every product
// is the one-species arithmetic above).
template <typename R>
__device__ __forceinline__ void pair_accum_mix(Acc<R> &a, double dx, double dy, double dz,
                                               double s, const PairTab *t, int k, bool energy) {
  const R sr = (R)s;
  const R rinv = recip(sr);
  const R rri = (R)t->sig2[k] * rinv;
  const R rri3 = rri * rri * rri;
  const R f = (R)t->eps48[k] * rri3 * (rri3 - (R)0.5) * rinv;
  a.fx += f * (R)dx;
  a.fy += f * (R)dy;
  a.fz += f * (R)dz;
  if (energy) {
    a.u += (R)t->eps4[k] * rri3 * (rri3 - (R)1) + (R)t->shift[k];
    a.w += f * sr;
  }
}

// Image shift code: 2 bits per dimension, a two's-complement multiple of L
// (0 -> 0, 1 -> +L, 3 -> -L).
__device__ __forceinline__ double img_shift(uint32_t code, double L) {
  return code == 0 ? 0.0 : (code == 1 ? L : -L);
}

// Cell coordinate c (one of the 27 offsets, so -1..G) wrapped into [0, G),
// and the image code of the atoms found there.
__device__ __forceinline__ int wrap_cell(int c, int G, uint32_t *code) {
  if (c >= G) {
    *code = 3;
    return c - G;
  }
  if (c < 0) {
    *code = 1;
    return c + G;
  }
  *code = 0;
  return c;
}

// ---------------------------------------------------------------------------
// LDS window of a tile
// ---------------------------------------------------------------------------
// Shared state of a tile's window while the tile is evaluated.
struct Window {
  int wt[WSTRIDE];       // staging intervals: count (-1: none), then (start, len, slot)
  int dl[NROWS * 3];     // per (source row, dz, dy): slot - storage index for the
                         // target row's main piece, its cell 0 and its cell G-1
  int rf;                // first source row (cz G + cy) of the tile
  int whole;             // 1: the window is the whole system, slot = storage index
};

// At a sort: the candidates of the tile's atoms (sorted, so the tile is a run
// of cells spanning source rows rf..rl) lie in the 9 target rows (dz, dy) of
// every source row, in the x-range of that source row widened by one cell
// (with the periodic wrap).  Wave 0 lists (target row, x-range) for every
// (source row, dz, dy), sorts the list by target row (bitonic, across the
// lanes), unites the x-ranges of equal rows, and turns each row into 1-3 cell
// pieces (cell 0 | main | cell G-1 when the x-range wraps, else one piece),
// i.e. storage-index intervals via cell_start.  Wave 0 then gives the pieces
// LDS slots in list order while they fit in WCAP (from the first that does
// not, pieces stay in global memory), merging storage-adjacent ones into
// staging intervals, with wave prefix sums.  The staging table also goes to
// S.win for the list steps until the next sort.
__device__ void make_window(SlotC &S, int lt, Window &w, int *scratch) {
  __shared__ int s_np;
  int *piece = scratch;              // [2 * 192] start, end
  int *pdelta = scratch + 2 * 192;   // [192] slot - storage index, or NOSLOT
  const int n = S.n;
  const int lane = threadIdx.x;
  int T = INT_MAX, xa = 0, xb = 0, ell = 0, pos = 0, np = 0;
  bool full = false, w0 = false, wg = false;
  if (threadIdx.x < 64) {
    const int G = S.G;
    const int i_f = lt * TILE, i_l = min(n, i_f + TILE) - 1;
    const auto CL = gp((const int32_t *)S.cell);
    const int c_f = CL[i_f], c_l = CL[i_l];
    const int rf = c_f / G, rl = c_l / G, ns = rl - rf + 1;
    const bool whole = n <= WCAP && !S.nowin;
    if (lane == 0) {
      w.rf = rf;
      w.whole = whole;
    }
    if (whole || ns * 9 > NROWS || S.nowin) {
      if (lane == 0) s_np = whole ? -2 : -1;  // whole system / no window
    } else {
      if (lane < ns * 9) {
        const int sr = lane / 9, q = lane % 9;
        const int rho = rf + sr, cz = rho / G, cy = rho % G;
        uint32_t im;
        const int tz = wrap_cell(cz + q / 3 - 1, G, &im);
        const int ty = wrap_cell(cy + q % 3 - 1, G, &im);
        T = tz * G + ty;
        xa = (sr == 0 ? c_f % G : 0) - 1;
        xb = (sr == ns - 1 ? c_l % G : G - 1) + 1;
        ell = lane;
      }
      {
        // sort the ns * 9 entries by row: each entry's rank is the number
        // of entries before it (smaller row, or the same row and a lower
        // lane), read lane by lane through scalar registers; the entries
        // then move to their ranks through LDS (lanes without an entry keep
        // theirs, past every rank)
        const int ne9 = ns * 9;
        int rank = lane;
        if (lane < ne9) {
          rank = 0;
          for (int j = 0; j < ne9; ++j) {
            const int Tj = __builtin_amdgcn_readlane(T, j);
            rank += (Tj < T || (Tj == T && j < lane)) ? 1 : 0;
          }
        }
        int *srt = scratch + 3 * 192;  // [4][64], after the pieces
        srt[rank] = T;
        srt[64 + rank] = xa;
        srt[128 + rank] = xb;
        srt[192 + rank] = ell;
        T = srt[lane];
        xa = srt[64 + lane];
        xb = srt[128 + lane];
        ell = srt[192 + lane];
      }
      const int Tp = __shfl_up(T, 1, 64);
      const bool lead = T != INT_MAX && (lane == 0 || Tp != T);
      int ua = xa, ub = xb;
      for (int d = 1; d < 64; ++d) {
        const int T2 = __shfl_down(T, d, 64), a2 = __shfl_down(xa, d, 64),
                  b2 = __shfl_down(xb, d, 64);
        const bool same = lane + d < 64 && T2 == T && T != INT_MAX;
        if (same) {
          ua = min(ua, a2);
          ub = max(ub, b2);
        }
        if (__ballot(same) == 0) break;
      }
      int c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0};
      if (lead) {
        const int rb = T * G;
        full = ub - ua + 1 >= G;
        if (full) {
          c0[0] = rb;
          c1[0] = rb + G;
          np = 1;
        } else {
          w0 = ub >= G;  // x = G is cell 0 of the row
          wg = ua < 0;   // x = -1 is cell G-1 of the row
          if (w0) {
            c0[np] = rb;
            c1[np] = rb + 1;
            ++np;
          }
          c0[np] = rb + max(ua, 0);
          c1[np] = rb + min(ub, G - 1) + 1;
          ++np;
          if (wg) {
            c0[np] = rb + G - 1;
            c1[np] = rb + G;
            ++np;
          }
        }
      }
      pos = np;
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(pos, o, 64);
        if (lane >= o) pos += y;
      }
      const int total = __shfl(pos, 63, 64);
      pos -= np;
      const auto CS = gp((const int32_t *)S.cs);
      for (int e = 0; e < np; ++e) {
        piece[2 * (pos + e)] = CS[c0[e]];
        piece[2 * (pos + e) + 1] = CS[c1[e]];
      }
      // every lane of a run takes its leader's pieces
      const unsigned long long lmask = __ballot(lead);
      const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
      const int ll = 63 - __clzll(lmask & upto);
      pos = __shfl(pos, ll, 64);
      np = __shfl(np, ll, 64);
      full = __shfl((int)full, ll, 64);
      w0 = __shfl((int)w0, ll, 64);
      wg = __shfl((int)wg, ll, 64);
      if (lane == 0) s_np = total;
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int npc = s_np;
    if (npc == -2) {
      if (lane == 0) {
        w.wt[0] = 1;
        w.wt[1] = 0;
        w.wt[2] = n;
        w.wt[3] = 0;
      }
    } else if (npc < 0) {
      if (lane == 0) w.wt[0] = -1;
    } else {
      // Pieces take slots in list order while they fit (from the first that
      // does not, the rest stay in global memory).  A non-empty piece that
      // continues the previous non-empty one in storage extends its staging
      // interval, else it opens one (at most NWIN).  Lane l holds pieces
      // 3l .. 3l+2; offsets and interval numbers are wave prefix sums.
      int ps[3], pe[3], ln[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const int p = 3 * lane + e;
        ps[e] = p < npc ? piece[2 * p] : 0;
        pe[e] = p < npc ? piece[2 * p + 1] : 0;
        ln[e] = p < npc ? max(pe[e] - ps[e], 0) : 0;
      }
      auto scan = [&](int v) {  // inclusive prefix sum over the wave
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(v, o, 64);
          if (lane >= o) v += y;
        }
        return v;
      };
      const int lsum = (ln[0] + ln[1]) + ln[2];
      int off[3];
      off[0] = scan(lsum) - lsum;
      off[1] = off[0] + ln[0];
      off[2] = off[1] + ln[1];
      const int pe_prev = __shfl_up(pe[2], 1, 64), ln_prev = __shfl_up(ln[2], 1, 64);
      bool fit[3], st[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const int p = 3 * lane + e;
        const int prev_end = e == 0 ? pe_prev : pe[e - 1];
        const bool prev_full = e == 0 ? (lane > 0 && ln_prev > 0) : ln[e - 1] > 0;
        fit[e] = p < npc && ln[e] > 0 && off[e] + ln[e] <= WCAP;
        st[e] = fit[e] && !(prev_full && ps[e] == prev_end);
      }
      const int nst = (int)st[0] + (int)st[1] + (int)st[2];
      const int kincl = scan(nst), nstarts = __shfl(kincl, 63, 64);
      int k[3];
      k[0] = kincl - nst + (int)st[0] - 1;
      k[1] = k[0] + (int)st[1];
      k[2] = k[1] + (int)st[2];
      bool ok[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) ok[e] = fit[e] && k[e] < NWIN;
      // the piece after e continues e's interval?
      const bool ok_next0 = __shfl_down((int)ok[0], 1, 64) != 0,
                 st_next0 = __shfl_down((int)st[0], 1, 64) != 0;
      const bool cont[3] = {ok[1] && !st[1], ok[2] && !st[2],
                            lane < 63 && ok_next0 && !st_next0};
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const int p = 3 * lane + e;
        if (p < npc) pdelta[p] = ln[e] == 0 ? 0 : (ok[e] ? off[e] - ps[e] : NOSLOT);
        if (ok[e] && st[e]) {
          w.wt[3 * k[e] + 1] = ps[e];
          w.wt[3 * k[e] + 3] = off[e];
        }
        if (ok[e] && !cont[e]) w.wt[3 * k[e] + 2] = off[e] + ln[e];  // end slot
      }
      // (same wave, later instructions: the end slots are written) length =
      // end - first slot
#pragma unroll
      for (int e = 0; e < 3; ++e)
        if (ok[e] && st[e]) w.wt[3 * k[e] + 2] -= off[e];
      if (lane == 0) w.wt[0] = min(nstarts, NWIN);
    }
  }
  __syncthreads();
  if (threadIdx.x < 64 && T != INT_MAX) {
    const int dm = pdelta[pos + (w0 ? 1 : 0)];
    w.dl[3 * ell] = dm;
    w.dl[3 * ell + 1] = full ? dm : (w0 ? pdelta[pos] : NOSLOT);
    w.dl[3 * ell + 2] = full ? dm : (wg ? pdelta[pos + np - 1] : NOSLOT);
  }
  // the staging table for the list steps until the next sort
  auto WG = gp(S.win) + (size_t)lt * WSTRIDE;
  const int nint = w.wt[0];
  if ((int)threadIdx.x < 1 + 3 * max(nint, 0)) WG[threadIdx.x] = w.wt[threadIdx.x];
  __syncthreads();
}

// Stage the window's atoms (positions of the current step) into LDS.
// MIX: the species of the window's atoms go to ssp beside the coordinates.
template <bool MIX>
__device__ __forceinline__ void stage_window(const int *wt, gcdouble X, gcdouble Y, gcdouble Z,
                                             double *sx, double *sy, double *sz, gcint SP,
                                             int8_t *ssp) {
  // The intervals fill slots 0 .. total-1 in order.  The coordinates go
  // straight from global memory into LDS (loads that write LDS, not
  // registers): wave w fills chunks of 32 slots c = w, w + 4, ..., lane l
  // the low (l even) or high (l odd) word of slot 32c + l/2, whose source it
  // finds by walking the interval table forward.  Nothing waits for the
  // data here, so all of a wave's loads are in flight together; the barrier
  // after the staging waits for them.
  const int nint = wt[0];
  if (nint <= 0) return;
  const int total = wt[3 * nint] + wt[3 * nint - 1];
  typedef __attribute__((address_space(1))) const char *gcchar;
  typedef __attribute__((address_space(3))) void *lvoid;
  const int l = threadIdx.x & 63;
  const int c0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nch = (total + 31) >> 5;
  int q = 0, end = wt[2];
  for (int c = c0; c < nch; c += TILE / 64) {
    const int sl = 32 * c + (l >> 1);
    if (sl < total) {
      while (sl >= end) {
        ++q;
        end = wt[3 * q + 3] + wt[3 * q + 2];
      }
      const size_t off = (size_t)(wt[3 * q + 1] + (sl - wt[3 * q + 3])) * 8 + 4 * (l & 1);
      __builtin_amdgcn_global_load_lds((gcchar)X + off, (lvoid)((char *)sx + 256 * c), 4, 0, 0);
      __builtin_amdgcn_global_load_lds((gcchar)Y + off, (lvoid)((char *)sy + 256 * c), 4, 0, 0);
      __builtin_amdgcn_global_load_lds((gcchar)Z + off, (lvoid)((char *)sz + 256 * c), 4, 0, 0);
    }
  }
  if constexpr (MIX) {
    // the species bytes through registers (after the coordinates' loads
    // have gone out)
    int qs = 0, es = wt[2];
    for (int sl = threadIdx.x; sl < total; sl += TILE) {
      while (sl >= es) {
        ++qs;
        es = wt[3 * qs + 3] + wt[3 * qs + 2];
      }
      ssp[sl] = (int8_t)SP[wt[3 * qs + 1] + (sl - wt[3 * qs + 3])];
    }
  }
}

// Storage bounds of neighbour row q (dz = q / 3 - 1, dy = q % 3 - 1) of an
// atom in cell (cx, cy, cz): the x-neighbours that do not wrap (one
// contiguous range, b[0] .. b[1]) and the one wrapped cell (b[2] .. b[3]).
template <class CSP>
__device__ __forceinline__ void row_bounds(CSP CS, int G, int cx, int cy, int cz, int q,
                                           int (&b)[4]) {
  const int xm0 = max(cx - 1, 0), xm1 = min(cx + 2, G);
  const int xe = cx == 0 ? G - 1 : 0;
  const int nz = cz + q / 3 - 1, ny = cy + q % 3 - 1;
  const int row = ((nz < 0 ? nz + G : nz >= G ? nz - G : nz) * G +
                   (ny < 0 ? ny + G : ny >= G ? ny - G : ny)) * G;
  b[0] = CS[row + xm0];
  b[1] = CS[row + xm1];
  b[2] = CS[row + xe];
  b[3] = CS[row + xe + 1];
}

// 27-cell traversal over the sorted atoms (offsets z-major, x fastest;
// ascending storage index within a cell, which is ascending index before the
// sort).  The three cells of an x-row are one contiguous range of storage
// indices unless the row wraps, where it is two.  Candidates are read from
// the LDS window (slot = storage index + the row piece's offset), or from
// global memory for a piece the window could not hold.  Accepts r^2 < r_n^2
// into W when building (window slot, or storage index with GFLAG), and
// accumulates the forces of pairs with r^2 < r_c^2.  Positions were wrapped
// by the sort, so they are read as stored.
// MIX: a mixture; the candidates' species come from ssp (LDS) or SP, atom
// i's is spi, and each pair takes its own cutoff and parameters from tab.
template <typename R, bool MIX>
__device__ __forceinline__ int traverse_sorted(SlotC &S, int i, int ci, gcdouble X,
                                               gcdouble Y, gcdouble Z, const Window &w,
                                               const double *sx, const double *sy,
                                               const double *sz, double xi, double yi,
                                               double zi, bool build, bool force, bool energy,
                                               Acc<R> &a, const int8_t *ssp, gcint SP, int spi,
                                               const PairTab *tab, bool unord,
                                               bool global_only = false,
                                               const int *pre0 = nullptr) {
  const int G = S.G;
  const double L = S.L, rn2 = S.rn2, rc2 = S.rc2;
  const R ushift = (R)S.ushift;
  const int mcap = S.mcap;
  // the next list entry's address: row min(m, mcap - 1) of W (an atom whose
  // list overflows keeps overwriting its last row; its list is not used)
  auto wp = gp(S.W) + i;
  const size_t np = (size_t)S.npad;
  const auto CS = cview((const int32_t *)S.cs);  // written by the sort, read-only here
  const int cx = ci % G, cy = (ci / G) % G, cz = ci / (G * G);
  // global_only: candidates from global memory (the window's row table is
  // not at hand)
  const bool whole = !global_only && w.whole, rows = !global_only && !whole && w.wt[0] >= 0;
  const int sr = rows ? ci / G - w.rf : 0;  // source row of the atom within the tile
  int m = 0;
  // candidates j of [lo, hi); FROM_LDS: every lane of the wave reads the
  // window (the usual case: one code path, the reads of four candidates in
  // flight together), else each lane reads where its piece lives
  // without reordering, position j of cell order is the atom stored at perm[j]
  const bool noreo = unord;
  const gcint PERM = gp((const int32_t *)S.perm);
  // SELF: the row holds atom i itself (the atom's own row, q = 4: the 27
  // cells are distinct for G >= 3, so no other row does)
  auto candidates = [&](auto from_lds, auto self, int lo, int hi, int delta, uint32_t code,
                        double bx, double by, double bz) {
    // ALL_LDS also means that no lane of the wave applies an image shift
    constexpr bool ALL_LDS = decltype(from_lds)::value, SELF = decltype(self)::value;
    const bool lds = ALL_LDS || delta != NOSLOT;
    for (int j0 = lo; j0 < hi; j0 += 4) {
      double xj[4], yj[4], zj[4];
      int sj[4], js[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        // from the window, a candidate past hi reads one of the (padded)
        // slots after the range's last, and is not taken
        const int j = ALL_LDS ? j0 + u : min(j0 + u, hi - 1);
        js[u] = j;
        if (ALL_LDS || lds) {
          xj[u] = sx[j + delta];
          yj[u] = sy[j + delta];
          zj[u] = sz[j + delta];
          if (MIX) sj[u] = ssp[j + delta];
        } else {
          if (noreo) js[u] = PERM[j];
          xj[u] = X[js[u]];
          yj[u] = Y[js[u]];
          zj[u] = Z[js[u]];
          if (MIX) sj[u] = SP[js[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j0 + u;
        if (j >= hi || (SELF && js[u] == i)) continue;
        double dx = xi - xj[u], dy = yi - yj[u], dz = zi - zj[u];
        if (!ALL_LDS) {
          dx = dx + bx;
          dy = dy + by;
          dz = dz + bz;
        }
        const double s = (dx * dx + dy * dy) + dz * dz;
        if (s < rn2) {
          if (build) {
            const uint32_t idx = lds ? (uint32_t)(j + delta) : ((uint32_t)js[u] | GFLAG);
            *wp = (int32_t)(idx | code);
            ++m;
            wp += m < mcap ? np : (size_t)0;
          }
          if (MIX) {
            const int kk = (spi * MAXSP + sj[u]) & (MAXSP * MAXSP - 1);
            if (force && s < tab->rc2[kk]) pair_accum_mix<R>(a, dx, dy, dz, s, tab, kk, energy);
          } else if (force && s < rc2) {
            pair_accum<R>(a, dx, dy, dz, s, ushift, energy);
          }
        }
      }
    }
  };
  auto range = [&](bool own, int lo, int hi, int delta, uint32_t code, double bx, double by,
                   double bz) {
    if (__ballot(lo < hi && (delta == NOSLOT || code != 0)) != 0)
      candidates(std::false_type{}, std::true_type{}, lo, hi, delta, code, bx, by, bz);
    else if (own)
      candidates(std::true_type{}, std::true_type{}, lo, hi, delta, code, bx, by, bz);
    else
      candidates(std::true_type{}, std::false_type{}, lo, hi, delta, code, bx, by, bz);
  };
  // storage bounds of row q: the x-neighbours that do not wrap (one
  // contiguous range) and the one wrapped cell, visited first when cx == 0
  // (cell G-1) and last when cx == G-1 (cell 0).  The bounds of the next row
  // are loaded before the current one is visited, so their latency is hidden
  // behind it.
  const int xm0 = max(cx - 1, 0), xm1 = min(cx + 2, G);
  const int xe = cx == 0 ? G - 1 : 0;
  const bool wlo = cx == 0, whi = cx == G - 1 && cx != 0;
  auto bounds = [&](int q, int (&b)[4]) { row_bounds(CS, G, cx, cy, cz, q, b); };
  // A wave with lanes at an x-edge of the box (cx = 0 or G-1) visits each
  // row as one loop over the lane's two ranges, the wrapped cell and the
  // row's own cells in x order (cell G-1 first when cx = 0, cell 0 last
  // when cx = G-1: the order of separate visits, so the same list and the
  // same sums), instead of three loops of which two run for a few lanes.
  // Every candidate then takes its own window offset and x image shift.
  const bool edge = wlo || whi;
  const bool anyedge = __ballot(edge) != 0;
  // ALL_LDS: every piece of the row is in the window for every lane; YZ:
  // some lane's row is a y or z image; SELF: the atom's own row
  auto merged_t = [&](auto all_lds, auto yz, auto self, int loM, int hiM, int dM, int loW,
                      int hiW, int dW, uint32_t cyz, double by, double bz) {
    constexpr bool ALL_LDS = decltype(all_lds)::value, YZ = decltype(yz)::value,
                   SELF = decltype(self)::value;
    const int loF = wlo ? loW : loM, hiF = wlo ? hiW : hiM;
    const int loS = wlo ? loM : loW, hiS = wlo ? hiM : hiW;
    const int lenF = hiF - loF, tot = lenF + (hiS - loS);
    const double bw = wlo ? L : -L;
    const uint32_t cw = cyz | ((wlo ? 1u : 3u) << J_BITS);
    for (int k0 = 0; k0 < tot; k0 += 4) {
      double xj[4], yj[4], zj[4];
      int sj[4], js[4], jj[4];
      bool isw[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = min(k0 + u, tot - 1);
        const bool inF = k < lenF;
        const int j = inF ? loF + k : loS + (k - lenF);
        isw[u] = edge && inF == wlo;
        const int d = isw[u] ? dW : dM;
        jj[u] = j;
        js[u] = j;
        if (ALL_LDS || d != NOSLOT) {
          xj[u] = sx[j + d];
          yj[u] = sy[j + d];
          zj[u] = sz[j + d];
          if (MIX) sj[u] = ssp[j + d];
        } else {
          if (noreo) js[u] = PERM[j];
          xj[u] = X[js[u]];
          yj[u] = Y[js[u]];
          zj[u] = Z[js[u]];
          if (MIX) sj[u] = SP[js[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (k0 + u >= tot || (SELF && js[u] == i)) continue;
        double dx = xi - xj[u], dy = yi - yj[u], dz = zi - zj[u];
        dx = dx + (isw[u] ? bw : 0.0);
        if (YZ) {
          dy = dy + by;
          dz = dz + bz;
        }
        const double s = (dx * dx + dy * dy) + dz * dz;
        if (s < rn2) {
          if (build) {
            const int d = isw[u] ? dW : dM;
            const uint32_t idx =
                ALL_LDS || d != NOSLOT ? (uint32_t)(jj[u] + d) : ((uint32_t)js[u] | GFLAG);
            *wp = (int32_t)(idx | (isw[u] ? cw : cyz));
            ++m;
            wp += m < mcap ? np : (size_t)0;
          }
          if (MIX) {
            const int kk = (spi * MAXSP + sj[u]) & (MAXSP * MAXSP - 1);
            if (force && s < tab->rc2[kk]) pair_accum_mix<R>(a, dx, dy, dz, s, tab, kk, energy);
          } else if (force && s < rc2) {
            pair_accum<R>(a, dx, dy, dz, s, ushift, energy);
          }
        }
      }
    }
  };
  // the usual row (interior, wholly in the window, not the atom's own) skips
  // the per-candidate choice of window or global memory, the y/z image
  // shifts (zero there: x + 0 == x) and the test for atom i itself
  auto merged = [&](bool own, int loM, int hiM, int dM, int loW, int hiW, int dW, uint32_t cyz,
                    double by, double bz) {
    if (!edge) loW = hiW = 0;
    const bool glob = (hiM > loM && dM == NOSLOT) || (hiW > loW && dW == NOSLOT);
    if (own || __ballot(glob || by != 0.0 || bz != 0.0) != 0)
      merged_t(std::false_type{}, std::true_type{}, std::true_type{}, loM, hiM, dM, loW, hiW, dW,
               cyz, by, bz);
    else
      merged_t(std::true_type{}, std::false_type{}, std::false_type{}, loM, hiM, dM, loW, hiW,
               dW, cyz, by, bz);
  };
  // (row 0's bounds may have been loaded by the caller, ahead of the window)
  int cur[4], nxt[4];
  if (pre0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) cur[u] = pre0[u];
  } else {
    bounds(0, cur);
  }
#pragma unroll 1
  for (int q = 0; q < 9; ++q) {
    if (q < 8) bounds(q + 1, nxt);
    uint32_t iz, iy;
    wrap_cell(cz + q / 3 - 1, G, &iz);
    wrap_cell(cy + q % 3 - 1, G, &iy);
    const double by = img_shift(iy, L), bz = img_shift(iz, L);
    const uint32_t cyz = ((iy << 2) | (iz << 4)) << J_BITS;
    int dm = NOSLOT, d0 = NOSLOT, dg = NOSLOT;
    if (whole) {
      dm = d0 = dg = 0;
    } else if (rows) {
      const int e = 3 * (sr * 9 + q);
      dm = w.dl[e];
      d0 = w.dl[e + 1];
      dg = w.dl[e + 2];
    }
    if (anyedge)
      merged(q == 4, cur[0], cur[1], dm, cur[2], cur[3], wlo ? dg : d0, cyz, by, bz);
    else
      range(q == 4, cur[0], cur[1], dm, cyz, 0.0, by, bz);
#pragma unroll
    for (int u = 0; u < 4; ++u) cur[u] = nxt[u];
  }
  return m;
}

// Coordinates of neighbour-list entry e: from the LDS window, or from
// global memory when the entry carries a storage index.
template <bool MIX>
__device__ __forceinline__ void entry_pos(uint32_t e, gcdouble X, gcdouble Y, gcdouble Z,
                                          const double *sx, const double *sy, const double *sz,
                                          double &xj, double &yj, double &zj, gcint SP,
                                          const int8_t *ssp, int &sj) {
  const uint32_t idx = e & IDX_MASK;
  if (e & GFLAG) {
    xj = X[idx];
    yj = Y[idx];
    zj = Z[idx];
    if (MIX) sj = SP[idx];
  } else {
    xj = sx[idx];
    yj = sy[idx];
    zj = sz[idx];
    if (MIX) sj = ssp[idx];
  }
}

// One neighbour-list entry e (index + image code) of atom i, counted when ok.
// SHIFT = false when no entry of the wave's current group carries an image
// code.
// MIX: kk = the species pair (masked into the table: a masked-off entry may
// carry any species byte).
template <typename R, bool SHIFT, bool MIX>
__device__ __forceinline__ void list_pair(Acc<R> &a, bool ok, uint32_t e, double xi, double yi,
                                          double zi, double xj, double yj, double zj, double L,
                                          double rc2, R ushift, bool energy, int kk,
                                          const PairTab *tab) {
  double dx = xi - xj, dy = yi - yj, dz = zi - zj;
  if (SHIFT) {
    // each 2-bit field sign-extended is the multiple of L (exact products)
    dx = dx + (double)((int32_t)(e << (32 - J_BITS - 2)) >> 30) * L;
    dy = dy + (double)((int32_t)(e << (32 - J_BITS - 4)) >> 30) * L;
    dz = dz + (double)((int32_t)e >> 30) * L;
  }
  const double s = (dx * dx + dy * dy) + dz * dz;
  if (MIX) {
    if (ok && s < tab->rc2[kk]) pair_accum_mix<R>(a, dx, dy, dz, s, tab, kk, energy);
  } else if (ok && s < rc2) {
    pair_accum<R>(a, dx, dy, dz, s, ushift, energy);
  }
}

// Whether the storage of the state that step k (or a host evaluation at
// the held state k) works on is not the cell order of the last sort: always
// without reordering, else after a rebuild that kept the storage order
// (CtlDev::rb_ring) and until the next reordering (CtlDev::ord_ring).  The
// words are read through the constant view (written by earlier launches), so
// the test can be made again wherever it is needed instead of held.
template <class Ctl>
__device__ __forceinline__ bool unordered(SlotC &S, const Ctl &C, int64_t k, int mode) {
  if (S.noreo) return true;
  if (mode != MODE_STEP) return C.ord_ring[mod3(k)] != 0;
  const int rb = C.rb_ring[mod3(k)];
  return rb != RB_NONE ? rb == RB_PERM : C.ord_ring[mod3(k - 1)] != 0;
}

// ACC: the steps of a block, which sum their properties and add them to the
// block sums.  MIX: a mixture (species staged with the window, pair
// parameters in LDS).
// pub: thread TILE - 64 stores pubv there before the tile's last barrier
// (the step kernel's next tile, published to the workgroup without a
// barrier of its own).
template <typename R, bool ACC, bool MIX>
__device__ __forceinline__ void step_tile(SlotC &S, CtlDev &C, int lt, int64_t k, int mode, bool cells,
                          bool build, bool last, bool bin_next, int *pub, int pubv) {
  const int i = lt * TILE + threadIdx.x;
  const bool act = i < S.n;
  const int pb = (int)(k & 1);
  const int vb = mode == MODE_STEP ? pb : pb ^ 1;  // v(k-1/2) during a run, v(k) when clean
  const gcdouble X = gp((const double *)S.P[pb][0]);
  const gcdouble Y = gp((const double *)S.P[pb][1]);
  const gcdouble Z = gp((const double *)S.P[pb][2]);
  const bool force = mode != MODE_BUILD;
  const double L = S.L;

  // loads that do not wait for the window: own position and velocity, list
  // length and the first NE list entries (or the own cell when sorted).
  // Velocities, list lengths and these entries are read once a step:
  // streaming (non-temporal) loads, so they do not displace the window data
  // that neighbouring tiles read again from the caches.  (Entries past the
  // first NE, the bulk of a long list such as LJ r_c = 3's, are read plainly:
  // such lists stay in the last-level cache from step to step.)
  constexpr int NE = sizeof(R) == 8 ? 8 : 12;
  const bool list = !cells && force;
  const auto Wc = gp((const int32_t *)S.W) + i;
  const size_t np = (size_t)S.npad;
  double xi = 0, yi = 0, zi = 0, v[3] = {0.0, 0.0, 0.0};
  int m = 0, ci = 0;
  uint32_t e[NE];
  // the window table first: the staging waits for it, not for the rest
  int wtv = 0;
  if (list && threadIdx.x < WSTRIDE) wtv = gp((const int32_t *)S.win)[lt * WSTRIDE + threadIdx.x];
  if (act) {
    xi = X[i];
    yi = Y[i];
    zi = Z[i];
    if (force)
      for (int q = 0; q < 3; ++q) v[q] = __builtin_nontemporal_load(&gp(S.V[vb][q])[i]);
    if (list) {
      m = __builtin_nontemporal_load(&gp(S.m)[i]);
#pragma unroll
      for (int u = 0; u < NE; ++u)
        e[u] = u < S.mcap ? (uint32_t)__builtin_nontemporal_load(&Wc[(size_t)u * np]) : 0u;
    } else if (cells) {
      ci = gp(S.cell)[i];
    }
  }

  // the tile's LDS window: made with the list at a sort, read back otherwise
  // (4 slots of padding: a traversal group may read up to 3 slots past the
  // window's last)
  __shared__ double sx[WCAP + 4], sy[WCAP + 4], sz[WCAP + 4];
  __shared__ Window win;
  // a mixture: the window's species and the pair table (the barriers below
  // publish them)
  __shared__ typename std::conditional<MIX, PairTab, char>::type stab;
  __shared__ int8_t ssp_store[MIX ? WCAP + 4 : 1];
  const PairTab *tab = nullptr;
  int8_t *ssp = nullptr;
  const gcint SP = gp((const int32_t *)S.sp);
  int spi = 0;
  if constexpr (MIX) {
    tab = &stab;
    ssp = ssp_store;
    constexpr int NT = (int)(sizeof(PairTab) / sizeof(double));
    if (threadIdx.x < NT)
      ((double *)&stab)[threadIdx.x] = gp((const double *)S.tab)[threadIdx.x];
    if (act) spi = SP[i];
  }
  // a cell step: the bounds of the first neighbour row of the traversal go
  // out before the window is built (wave 0 builds it; the others wait)
  int b0[4] = {0, 0, 0, 0};
  if (cells && act) {
    const int G = S.G;
    row_bounds(cview((const int32_t *)S.cs), G, ci % G, (ci / G) % G, ci / (G * G), 0, b0);
  }
  if (cells && unordered(S, *cview(&C), k, mode)) {
    // no reordering: the tile's atoms are not a run of cells, so there is no
    // window; candidates are read from global memory through perm, and the
    // list steps until the next sort stage nothing
    if (threadIdx.x == 0) {
      win.wt[0] = -1;
      win.whole = 0;
      win.rf = 0;
      gp(S.win)[(size_t)lt * WSTRIDE] = -1;
    }
    __syncthreads();
  } else if (cells) {
    make_window(S, lt, win, (int *)sx);
  } else if (list) {
    if (threadIdx.x < WSTRIDE) win.wt[threadIdx.x] = wtv;
    __syncthreads();
  }
  // The first NP entries that live outside the window: their coordinates
  // are gathered now, while the window is staged, instead of inside the
  // pair loop (by the waves that have such entries; only a group holding
  // one reads them).
  constexpr int NP = 8;  // (all NE = 12 of FP32 forces: more registers, spills)
  double gx[NP], gy[NP], gz[NP];
  int gs[NP];
  uint32_t gor = 0;
  if (list && act && m <= S.mcap)
    for (int u = 0; u < NP; ++u) gor |= u < m ? e[u] : 0u;
  if (__ballot((gor & GFLAG) != 0) != 0) {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      gx[u] = gy[u] = gz[u] = 0.0;
      gs[u] = 0;
      if (u < m && (e[u] & GFLAG) && m <= S.mcap && act) {
        const uint32_t idx = e[u] & IDX_MASK;
        gx[u] = X[idx];
        gy[u] = Y[idx];
        gz[u] = Z[idx];
        if (MIX) gs[u] = SP[idx];
      }
    }
  }
  if (cells || list) {
    stage_window<MIX>(win.wt, X, Y, Z, sx, sy, sz, SP, ssp);
    __syncthreads();
  }

  Acc<R> a{(R)0, (R)0, (R)0, (R)0, (R)0};
  if (act) {
    if (cells) {
      m = traverse_sorted<R, MIX>(S, i, ci, X, Y, Z, win, sx, sy, sz, xi, yi, zi, build, force,
                                  mode != MODE_STEP || last || ACC, a, ssp, SP, spi, tab,
                                  unordered(S, *cview(&C), k, mode), false, b0);
      if (build) gp(S.m)[i] = m;
    } else if (list) {
      if (m <= S.mcap) {
        const double rc2 = S.rc2;
        const R ushift = (R)S.ushift;
        const bool energy = mode != MODE_STEP || last || ACC;
        // entries in order, four at a time (their coordinate reads together),
        // for as long as any lane of the wave has some left: a lane past its
        // length takes the group with no effect, so the wave runs max(m)/4
        // groups whatever the spread of m.  A group without image codes
        // anywhere in the wave skips the shifts.
        // PRE: entries q0 .. q0+3 are among the first NP (their global
        // coordinates gathered above)
        auto group = [&](auto pre, int q0, uint32_t e0, uint32_t e1, uint32_t e2, uint32_t e3) {
          constexpr bool PRE = decltype(pre)::value;
          const bool ok[4] = {q0 < m, q0 + 1 < m, q0 + 2 < m, q0 + 3 < m};
          const uint32_t eg[4] = {ok[0] ? e0 : 0u, ok[1] ? e1 : 0u, ok[2] ? e2 : 0u,
                                  ok[3] ? e3 : 0u};
          const uint32_t any = (eg[0] | eg[1]) | (eg[2] | eg[3]);
          double xj[4], yj[4], zj[4];
          int sj[4] = {0, 0, 0, 0};
          if (__ballot((any & GFLAG) != 0) == 0) {
            // the usual case: every entry of the wave is a window slot
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const uint32_t sl = eg[u] & IDX_MASK;
              xj[u] = sx[sl];
              yj[u] = sy[sl];
              zj[u] = sz[sl];
              if (MIX) sj[u] = ssp[sl];
            }
          } else if constexpr (PRE) {
            // window slots from LDS (slot 0 for an entry outside it), the
            // others from the gathered coordinates
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const bool g = (eg[u] & GFLAG) != 0;
              const uint32_t sl = g ? 0u : eg[u] & IDX_MASK;
              const int qu = min(q0 + u, NP - 1);
              xj[u] = g ? gx[qu] : sx[sl];
              yj[u] = g ? gy[qu] : sy[sl];
              zj[u] = g ? gz[qu] : sz[sl];
              if (MIX) sj[u] = g ? gs[qu] : ssp[sl];
            }
          } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
              entry_pos<MIX>(eg[u], X, Y, Z, sx, sy, sz, xj[u], yj[u], zj[u], SP, ssp, sj[u]);
          }
          if (__ballot((any >> J_BITS) != 0) == 0) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
              list_pair<R, false, MIX>(a, ok[u], eg[u], xi, yi, zi, xj[u], yj[u], zj[u], L, rc2,
                                       ushift, energy, (spi * MAXSP + sj[u]) & (MAXSP * MAXSP - 1), tab);
          } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
              list_pair<R, true, MIX>(a, ok[u], eg[u], xi, yi, zi, xj[u], yj[u], zj[u], L, rc2,
                                      ushift, energy, (spi * MAXSP + sj[u]) & (MAXSP * MAXSP - 1), tab);
          }
        };
#pragma unroll
        for (int g = 0; g < NP / 4; ++g)
          if (__ballot(4 * g < m) != 0)
            group(std::true_type{}, 4 * g, e[4 * g], e[4 * g + 1], e[4 * g + 2], e[4 * g + 3]);
#pragma unroll
        for (int g = NP / 4; g < NE / 4; ++g)
          if (__ballot(4 * g < m) != 0)
            group(std::false_type{}, 4 * g, e[4 * g], e[4 * g + 1], e[4 * g + 2], e[4 * g + 3]);
        for (int q = NE; __ballot(q < m) != 0; q += 4) {
          uint32_t ew[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) ew[u] = q + u < m ? (uint32_t)Wc[(size_t)(q + u) * np] : 0u;
          group(std::false_type{}, q, ew[0], ew[1], ew[2], ew[3]);
        }
      } else {
        // the list overflowed its capacity at the last build: evaluate this
        // atom over the 27 cells of its cell at that sort, with the positions
        // of now (exact: an atom within r_c now was within r_n then, since
        // neither moved more than delta/2), reading them from global memory
        traverse_sorted<R, MIX>(S, i, gp(S.cell)[i], X, Y, Z, win, sx, sy, sz, xi, yi, zi,
                                false, true, mode != MODE_STEP || last || ACC, a, ssp, SP, spi,
                                tab, unordered(S, *cview(&C), k, mode), true);
      }
    }
  }

  // (d), (e) and the next (a)
  double vv = 0.0;
  if (act && force) {
    const double f[3] = {(double)a.fx, (double)a.fy, (double)a.fz};
    if (mode == MODE_STEP)
      for (int q = 0; q < 3; ++q) v[q] = v[q] + S.hdt * f[q];  // (d)
    vv = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];            // (e)
    if (mode == MODE_STEP) {
      if (!last) {
        double xn[3];
        const double xo[3] = {xi, yi, zi};
        for (int q = 0; q < 3; ++q) {
          v[q] = v[q] + S.hdt * f[q];  // (a) of step k+1
          xn[q] = xo[q] + S.dt * v[q];
          // streaming stores: the next step's kernels read these from
          // any XCD, so they are not kept in this XCD's L2 (less for its
          // write-back when the kernel ends)
          __builtin_nontemporal_store(xn[q], &gp(S.P[pb ^ 1][q])[i]);
        }
        if (bin_next)
          bin_atom(S, C, (int)mod3(k + 1), i, xn[0], xn[1], xn[2], k + 1);
        else
          check_atom(S, C, xn[0], xn[1], xn[2], k + 1);
      }
      for (int q = 0; q < 3; ++q) __builtin_nontemporal_store(v[q], &gp(S.V[pb ^ 1][q])[i]);
    }
    if (mode != MODE_STEP || last) {
      auto F = gp((R *)S.F);
      F[i] = a.fx;
      F[S.npad + i] = a.fy;
      F[2 * S.npad + i] = a.fz;
      auto U = gp((R *)S.UA);
      U[i] = a.u;
      U[S.npad + i] = a.w;
    }
  }

  // the set after next is cleared for the binning of step k+2
  if (mode == MODE_STEP) {
    const int zs = (int)mod3(k + 2);
    const int c0 = lt * S.cpt, c1 = min(c0 + S.cpt, S.ncell);
    for (int c = c0 + threadIdx.x; c < c1; c += TILE) gp(S.cnt[zs])[c] = 0;
    for (int q = lt * TILE + threadIdx.x; q < S.nctiles; q += S.ntiles * TILE)
      gp(S.tcnt[zs])[q] = 0;
    if (lt == 0 && threadIdx.x == 0) S.ovf_n[zs] = 0;
  }

  // the maximum speed of the step (the rebuild rule needs it every step):
  // v^2 >= 0, so its bit pattern orders like the value
  __shared__ unsigned long long sv[4];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const unsigned long long vbits = wave_max_u64((unsigned long long)__double_as_longlong(vv));
  if (l == 0) sv[w] = vbits;
  // the other properties only where somebody reads them: the last step of a
  // run, evaluations of a held state, and the steps of a block
  const bool full = mode != MODE_STEP || last || ACC;
  __shared__ double sh[4][8];
  if (full) {
    const int mm = act && !S.cell_only ? m : 0;
    const double ke = wave_sum(vv);
    const double sm = wave_sum((double)mm);
    const int mmax = wave_max_i(mm);
    double pe_hi, pe_lo, vr_hi, vr_lo;
    if (sizeof(R) == 8) {
      pe_hi = wave_sum((double)a.u);
      vr_hi = wave_sum((double)a.w);
      pe_lo = vr_lo = 0.0;
    } else {
      F2 pe = wave_sum_f2(F2{(float)a.u, 0.0f});
      F2 vr = wave_sum_f2(F2{(float)a.w, 0.0f});
      pe_hi = pe.hi;
      pe_lo = pe.lo;
      vr_hi = vr.hi;
      vr_lo = vr.lo;
    }
    if (l == 0) {
      sh[w][0] = ke;
      sh[w][2] = pe_hi;
      sh[w][3] = pe_lo;
      sh[w][4] = vr_hi;
      sh[w][5] = vr_lo;
      sh[w][6] = sm;
      sh[w][7] = (double)mmax;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long b01 = sv[0] > sv[1] ? sv[0] : sv[1];
    const unsigned long long b23 = sv[2] > sv[3] ? sv[2] : sv[3];
    const unsigned long long vmb = b01 > b23 ? b01 : b23;
    // one atomic per workgroup, spread over VSPREAD cache lines
    if (force) atomicMax(&S.vring[(mod3(k) * VSPREAD + (lt & (VSPREAD - 1))) * 16], vmb);
    if (full) {
      auto q = gp(S.part) + (size_t)lt * NPART;
      if (force) {
        q[0] = ((sh[0][0] + sh[1][0]) + sh[2][0]) + sh[3][0];
        q[1] = __longlong_as_double((long long)vmb);
        if (sizeof(R) == 8) {
          q[2] = ((sh[0][2] + sh[1][2]) + sh[2][2]) + sh[3][2];
          q[3] = 0.0;
          q[4] = ((sh[0][4] + sh[1][4]) + sh[2][4]) + sh[3][4];
          q[5] = 0.0;
        } else {
          F2 e{(float)sh[0][2], (float)sh[0][3]}, v2{(float)sh[0][4], (float)sh[0][5]};
          for (int k2 = 1; k2 < 4; ++k2) {
            e = f2_add(e, F2{(float)sh[k2][2], (float)sh[k2][3]});
            v2 = f2_add(v2, F2{(float)sh[k2][4], (float)sh[k2][5]});
          }
          q[2] = e.hi;
          q[3] = e.lo;
          q[4] = v2.hi;
          q[5] = v2.lo;
        }
      }
      q[6] = ((sh[0][6] + sh[1][6]) + sh[2][6]) + sh[3][6];
      q[7] = fmax(fmax(sh[0][7], sh[1][7]), fmax(sh[2][7], sh[3][7]));
      if (ACC && mode == MODE_STEP) {
        // this tile's part of the block sums (the tile's atoms change at a
        // sort, the total over tiles does not)
        auto A = gp(S.acc) + (size_t)lt * NACC;
        A[0] = A[0] + q[0];
        A[1] = A[1] + (q[2] + q[3]);
        A[2] = A[2] + (q[4] + q[5]);
        A[3] = A[3] + q[6];
        if (S.tpart) {
          // a traced replica: this step's tile partials, reduced by k_trace
          // at the end of the replay
          const int si = (int)(k - C.base - 1);
          auto Q = gp(S.tpart) + ((size_t)si * S.ntiles + lt) * 4;
          Q[0] = q[0];
          Q[1] = q[2] + q[3];
          Q[2] = q[4] + q[5];
          Q[3] = q[1];
        }
      }
    }
  }
  if (pub != nullptr && threadIdx.x == TILE - 64) *pub = pubv;
  __syncthreads();
}

// ACC: every step of this launch also adds its properties to the block sums
// (a separate instantiation, so steps outside a block run the plain kernel).
// MIX: the replicas are mixtures (more LDS: three workgroups per CU).
template <typename R, bool ACC, bool MIX>
__global__ __launch_bounds__(TILE, MIX ? 3 : 4) void k_step(Tables T, int s, int mode,
                                                          int force_build, int only) {
  // what a workgroup decides per replica is launch-invariant: it is worked
  // out once for a run of consecutive tiles of one replica (every tile, for
  // a single system).  The control words used here are written by earlier
  // launches only (this launch writes other ring slots, read alongside but
  // not used, and err_step > k).
  int rc = -1, var = 0;
  int64_t k = 0;
  bool skip = true, last = false, cells = false, build = false, bin_next = false;
  // the header's words, lane l holding word l % 8: a vector load that goes
  // out with the decision's loads and is waited for only where the tile
  // loop needs it
  const int hdr_l = cview(T.hdr)[threadIdx.x & 7];
  // works out the decision for replica r; leaves skip set when the launch
  // has nothing to do for it
  auto decide = [&](int r) {
    rc = r;
    skip = true;
    SlotC &S0 = slot(T, 2 * r);
    auto &C = *cview(T.ctl + r);
    if (only >= 0 && r != only) return;
    last = false;
    if (mode == MODE_STEP) {
      // every word is read before any is tested: one round of loads where
      // tests one after another made a chain of them
      const int64_t base = C.base, target = C.target, err_step = C.err_step;
      const int32_t err = C.err, fp64 = S0.fp64, cell_only = S0.cell_only;
      const int32_t vr0 = C.var_ring[0], vr1 = C.var_ring[1], vr2 = C.var_ring[2];
      const int32_t rb0 = C.rb_ring[0], rb1 = C.rb_ring[1], rb2 = C.rb_ring[2];
      const int32_t bn0 = C.bin_ring[0], bn1 = C.bin_ring[1], bn2 = C.bin_ring[2];
      // (the empty asm takes these words at one point: left to itself the
      // compiler issued the descriptor's loads only after waiting for the
      // control words)
      asm volatile("" ::"s"(base), "s"(fp64), "s"(cell_only));
      k = base + s + 1;
      const int64_t e0 = mod3(k), e1 = mod3(k - 1);
      last = k == target;
      var = pick3(vr0, vr1, vr2, e1);
      // k_sort of this step decided, and if so gathered r(k) into the other
      // variant (or, without reordering, found the cell order in place)
      const int rb = pick3(rb0, rb1, rb2, e0);
      cells = rb != RB_NONE;
      build = cells && !cell_only;
      if (rb == RB_REORDER) var ^= 1;
      // r(k+1) is binned here if a sort at step k+1 may need its rows (the
      // rule of bins_due, evaluated by k_sort of this step)
      bin_next = pick3(bn0, bn1, bn2, e0) != 0;
      // stop at an error of an earlier step; one latched by this launch
      // (while binning r(k+1), err_step = k + 1) must not stop the others
      skip = fp64 != (sizeof(R) == 8) || k > target || (err != 0 && err_step <= k);
    } else {
      if (S0.fp64 != (sizeof(R) == 8) || !C.clean) return;
      k = C.done;
      var = C.var_ring[mod3(k)];
      build = !S0.cell_only && (force_build || mode == MODE_BUILD);
      cells = build || S0.cell_only;
      skip = C.err != 0 && C.err_step <= k;
    }
  };
  const int x = blockIdx.x & 7, nwg = gridDim.x >> 3;
  constexpr int CLAIMER = TILE - 64;
  int32_t *cnt = T.walk + 64 * x, *fin = T.walk + 64 * (8 + x);
  // one replica: decided before the tile loop (the decision needs no tile
  // table, so its loads go out with the header's); a launch with nothing to
  // step for it ends here, counting every workgroup finished if it takes
  // its tiles on demand (below)
  const bool solo = T.nslots == 1;
  if (solo) {
    decide(0);
    if (skip) {
      const int nt = __builtin_amdgcn_readlane(hdr_l, HDR_NTILES);
      if ((gridDim.x & 7) == 0 && nt > (int)gridDim.x && threadIdx.x == CLAIMER &&
          atomicAdd(fin, 1) == nwg - 1) {
        atomicExch(cnt, 0);
        atomicExch(fin, 0);
      }
      return;
    }
  }
  const int nt = __builtin_amdgcn_readlane(hdr_l, HDR_NTILES);
  const int order = __builtin_amdgcn_readlane(hdr_l, HDR_ORDER);
  const TileWalk tw(blockIdx.x, gridDim.x, nt, order);
  // A launch with more tiles than workgroups takes them on demand; the
  // others walk them statically.  On demand: workgroup group x = block & 7
  // (the XCD the block is dispatched to) owns the tiles of the static
  // walk's share of x (TileWalk); a workgroup does the first tile of its
  // static walk, then claims the next ones from the group's counter, so one
  // whose tiles ran long does fewer of them.  The claim for the next tile
  // goes out from the last wave as a tile starts (that wave waits for the
  // window build anyway, so the claim's latency hides) and is published to
  // the workgroup before the tile's last barrier.  Every workgroup counts
  // itself finished once a claim finds no tile left; the last of the group
  // resets the group's counters for the next launch.
  const bool dyn = (gridDim.x & 7) == 0 && nt > (int)gridDim.x;
  const bool slabs = order == ORDER_SLABS;
  __shared__ int s_claim[2];
  // the tile after this one: the static walk's, or the claimed one (double-
  // buffered: a slot is written again only after the last barrier of the
  // next tile, which every thread passes after reading it)
  int it = 0, claim = 0;
  bool stepped = false;
  auto next = [&](int t) {
    if (!dyn) return t + tw.step;
    const int b = it & 1;
    ++it;
    if (!stepped) {
      if (threadIdx.x == CLAIMER) s_claim[b] = claim;
      __syncthreads();
    }
    const int q = nwg + s_claim[b];  // the q-th tile of group x in the walk's order
    const int u = slabs ? tw.t - (int)(blockIdx.x >> 3) + q
                        : x * nwg + q % nwg + (q / nwg) * (int)gridDim.x;
    return u < tw.end ? u : nt;
  };
  for (int t = tw.t; t < tw.end; t = next(t)) {
    stepped = false;
    if (dyn && threadIdx.x == CLAIMER) claim = atomicAdd(cnt, 1);
    const int r = solo ? 0 : cview(T.tile_rep)[t];
    if (r != rc) decide(r);
    if (skip) continue;
    CtlDev &C = T.ctl[r];
    SlotC &S = slot(T, 2 * r + var);
    const int lt = t - S.tile_off;
    if (mode == MODE_STEP && lt == 0 && threadIdx.x == 0) {
      // the one writer of these ring slots in this launch (nobody reads them
      // before the next launch)
      C.var_ring[mod3(k)] = var;
      C.ord_ring[mod3(k)] = unordered(S, *cview(&C), k, mode) ? 1 : 0;
    }
    step_tile<R, ACC, MIX>(S, C, lt, k, mode, cells, build, last, bin_next,
                           dyn ? &s_claim[it & 1] : nullptr, claim);
    stepped = true;
    if (mode == MODE_STEP && lt == 0 && threadIdx.x < VSPREAD)
      S.vring[(mod3(k + 1) * VSPREAD + threadIdx.x) * 16] = 0ull;
  }
  if (dyn && threadIdx.x == CLAIMER && atomicAdd(fin, 1) == nwg - 1) {
    atomicExch(cnt, 0);
    atomicExch(fin, 0);
  }
}

// End of a graph replay of K steps, before k_replay_end: for every traced
// replica (workgroup (s, r)) the properties of step base + s + 1, reduced
// from the tile partials in a fixed order (as k_props), into its trace ring.
__global__ __launch_bounds__(TILE) void k_trace(Tables T, int K) {
  const int s = blockIdx.x, r = blockIdx.y;
  if (s >= K || r >= T.nslots) return;
  SlotC &S = slot(T, 2 * r);
  if (S.n <= 0 || S.tpart == nullptr) return;
  const CtlDev &C = T.ctl[r];
  const int64_t k = C.base + s + 1;
  if (k > C.target || (C.err != 0 && C.err_step <= k)) return;
  __shared__ double sh[TILE][4];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int t = threadIdx.x; t < S.ntiles; t += TILE) {
    const double *q = S.tpart + ((size_t)s * S.ntiles + t) * 4;
    v[0] += q[0];
    v[1] += q[1];
    v[2] += q[2];
    v[3] = fmax(v[3], q[3]);
  }
  for (int j = 0; j < 4; ++j) sh[threadIdx.x][j] = v[j];
  __syncthreads();
  for (int h = TILE / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int j = 0; j < 4; ++j) {
        const double o = sh[threadIdx.x + h][j];
        sh[threadIdx.x][j] = j == 3 ? fmax(sh[threadIdx.x][j], o) : sh[threadIdx.x][j] + o;
      }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double *row = S.trace + (size_t)(k % TRACE_RING) * TRACE_W;
    row[0] = (double)k;
    row[1] = 0.5 * sh[0][0];
    row[2] = 0.5 * sh[0][1];
    row[3] = 0.5 * sh[0][2];
    row[4] = sh[0][3];
  }
}

// End of a graph replay of K steps: advance the step counters (one thread
// per replica; no other kernel of the replay reads what is written here).
__global__ void k_replay_end(Tables T, int K) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= T.nslots) return;
  CtlDev &C = T.ctl[r];
  if (slot(T, 2 * r).n <= 0) return;
  if (C.base >= C.target && C.done >= C.target) return;
  int64_t done = C.base + K < C.target ? C.base + K : C.target;
  if (C.err != 0) done = C.err_step - 1 < done ? C.err_step - 1 : done;
  if (done < C.done) done = C.done;
  C.done = done;
  C.base = done;
  // a replica that ran this replay holds a drifted state unless it finished
  C.clean = (done == C.target && C.err == 0) ? 1 : 0;
}

// Host-ordered update of a replica's target (single thread).
__global__ void k_set_target(Tables T, int slot, long long target) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    CtlDev &C = T.ctl[slot];
    C.target = target;
    C.base = C.done;
  }
}

// Fixed-order reduction of the per-tile partials of each replica (one
// workgroup per replica): thread t takes tiles t, t+256, ... in sequence, then
// a fixed tree.
__global__ __launch_bounds__(TILE) void k_props(Tables T, int only) {
  const int r = blockIdx.x;
  if (r >= T.nslots || (only >= 0 && r != only)) return;
  if (slot(T, 2 * r).n <= 0) return;
  SlotC &S = slot_held(T, r);
  CtlDev &C = T.ctl[r];
  constexpr int NV = 6 + NACC;
  __shared__ double sh[TILE][NV];
  double v[NV] = {};
  for (int t = threadIdx.x; t < S.ntiles; t += TILE) {
    const double *q = S.part + (size_t)t * NPART;
    v[0] += q[0];
    v[1] = fmax(v[1], q[1]);
    v[2] += q[2] + q[3];
    v[3] += q[4] + q[5];
    v[4] += q[6];
    v[5] = fmax(v[5], q[7]);
    const double *A = S.acc + (size_t)t * NACC;
    for (int j = 0; j < NACC; ++j) v[6 + j] += A[j];
  }
  for (int j = 0; j < NV; ++j) sh[threadIdx.x][j] = v[j];
  __syncthreads();
  for (int h = TILE / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      for (int j = 0; j < NV; ++j) {
        const double o = sh[threadIdx.x + h][j];
        sh[threadIdx.x][j] = (j == 1 || j == 5) ? fmax(sh[threadIdx.x][j], o)
                                                : sh[threadIdx.x][j] + o;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) {
    double vm = 0.0;
    for (int q = 0; q < VSPREAD; ++q)
      vm = fmax(vm, __longlong_as_double((long long)S.vring[(threadIdx.x * VSPREAD + q) * 16]));
    C.vmax_ring[threadIdx.x] = (uint64_t)__double_as_longlong(vm);
  }
  if (threadIdx.x == 0) {
    C.ke = 0.5 * sh[0][0];
    C.vmax2 = sh[0][1];
    C.pe = 0.5 * sh[0][2];
    C.vir = 0.5 * sh[0][3];
    C.sum_m = (int64_t)sh[0][4];
    C.max_m = (int)sh[0][5];
    for (int j = 0; j < NACC; ++j) C.acc_sum[j] = sh[0][6 + j];
  }
}

// Step (f) during equilibration (Secs. 3.1 and 5.1): scale the velocities of a
// held clean state by one factor so that sum v^2 = 3 (N - 1) T (the centre of
// mass is at rest, leaving 3 (N - 1) degrees of freedom), from the kinetic
// energy k_props reduced just before.  The tile's kinetic-energy and max-v^2
// partials are recomputed from the scaled velocities, in the step kernel's
// order; the rebuild rule keeps the maximum speed of (e), taken before (f).
__global__ __launch_bounds__(TILE) void k_adjust(Tables T, int only, double temperature) {
  __shared__ double sk[4];
  __shared__ unsigned long long sv[4];
  const int nt = cview(T.hdr)[HDR_NTILES];
  for (int t = xcd_block(blockIdx.x, gridDim.x); t < nt; t += gridDim.x) {
    const int r = cview(T.tile_rep)[t];
    if (only >= 0 && r != only) continue;
    if (slot(T, 2 * r).n <= 0) continue;
    SlotC &S = slot_held(T, r);
    const CtlDev &C = T.ctl[r];
    const double ke = C.ke;
    if (!C.clean || C.err != 0 || S.n < 2 || !(ke > 0.0)) continue;
    const double fac = sqrt((1.5 * (double)(S.n - 1) * temperature) / ke);
    const int lt = t - S.tile_off;
    const int i = lt * TILE + threadIdx.x;
    const int vb = (int)((C.done + 1) & 1);
    double vv = 0.0;
    if (i < S.n) {
      double v[3];
      for (int a = 0; a < 3; ++a) {
        v[a] = gp(S.V[vb][a])[i] * fac;
        gp(S.V[vb][a])[i] = v[a];
      }
      vv = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const double ks = wave_sum(vv);
    const unsigned long long vb2 = wave_max_u64((unsigned long long)__double_as_longlong(vv));
    if (l == 0) {
      sk[w] = ks;
      sv[w] = vb2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      auto q = gp(S.part) + (size_t)lt * NPART;
      q[0] = ((sk[0] + sk[1]) + sk[2]) + sk[3];
      const unsigned long long b01 = sv[0] > sv[1] ? sv[0] : sv[1];
      const unsigned long long b23 = sv[2] > sv[3] ? sv[2] : sv[3];
      q[1] = __longlong_as_double((long long)(b01 > b23 ? b01 : b23));
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// binning of the held state outside a step (creation, host-side sorts)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TILE) void k_insert(Tables T, int wrap_store, int only) {
  const int nt = T.hdr[HDR_NTILES];
  for (int t = xcd_block(blockIdx.x, gridDim.x); t < nt; t += gridDim.x) {
    const int r = T.tile_rep[t];
    if (only >= 0 && r != only) continue;
    if (slot(T, 2 * r).n <= 0) continue;
    SlotC &S = slot_held(T, r);
    CtlDev &C = T.ctl[r];
    const int i = (t - S.tile_off) * TILE + threadIdx.x;
    if (i >= S.n) continue;
    const int64_t k = cur_state(C);
    const int pb = (int)(k & 1);
    const double x = S.P[pb][0][i], y = S.P[pb][1][i], z = S.P[pb][2][i];
    bin_atom(S, C, (int)mod3(k), i, x, y, z, k);  // checks the unwrapped coordinates
    if (wrap_store && isfinite(x) && isfinite(y) && isfinite(z)) {
      S.P[pb][0][i] = wrap1(x, S.L, S.halfL);
      S.P[pb][1][i] = wrap1(y, S.L, S.halfL);
      S.P[pb][2][i] = wrap1(z, S.L, S.halfL);
    }
  }
}

// Cell index of the held position of every atom of replica `only`, storage
// order, into out (md_get_cells): the cell of bin_atom without binning.
__global__ __launch_bounds__(TILE) void k_cells(Tables T, int only, int32_t *out) {
  const int nt = T.hdr[HDR_NTILES];
  for (int t = xcd_block(blockIdx.x, gridDim.x); t < nt; t += gridDim.x) {
    const int r = T.tile_rep[t];
    if (r != only || slot(T, 2 * r).n <= 0) continue;
    SlotC &S = slot_held(T, r);
    const CtlDev &C = T.ctl[r];
    const int i = (t - S.tile_off) * TILE + threadIdx.x;
    if (i >= S.n) continue;
    const int pb = (int)(cur_state(C) & 1);
    double x = S.P[pb][0][i], y = S.P[pb][1][i], z = S.P[pb][2][i];
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) x = y = z = 0.0;
    out[i] = cell_of(S, wrap1(x, S.L, S.halfL), wrap1(y, S.L, S.halfL), wrap1(z, S.L, S.halfL));
  }
}

// Clear the cell-layer set of the held state (before re-binning it).
__global__ __launch_bounds__(TILE) void k_clear_set(Tables T, int only) {
  const int nct = T.hdr[HDR_NCTILES];
  for (int t = xcd_block(blockIdx.x, gridDim.x); t < nct; t += gridDim.x) {
    const int r = T.ctile_rep[t];
    if (only >= 0 && r != only) continue;
    SlotC &S = slot(T, 2 * r);
    const CtlDev &C = T.ctl[r];
    const int set = (int)mod3(cur_state(C));
    const int lt = t - S.ctile_off;
    const int c = lt * CTILE + threadIdx.x;
    if (c < S.ncell) S.cnt[set][c] = 0;
    if (threadIdx.x == 0) S.tcnt[set][lt] = 0;
    if (lt == 0 && threadIdx.x == 0) S.ovf_n[set] = 0;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_kick(const Tables &T, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_kick, dim3(grid), dim3(TILE), 0, s, T);
  hipLaunchKernelGGL(k_kick_end, dim3((T.nslots + TILE - 1) / TILE), dim3(TILE), 0, s, T);
}
void launch_sort(const Tables &T, int cgrid, int step_in_replay, int mode, int only,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_sort, dim3(cgrid), dim3(TILE), 0, s, T, step_in_replay, mode, only);
}
template <typename R, bool ACC, bool MIX>
static void launch_k_step(const Tables &T, int grid, int step_in_replay, int mode,
                          int force_build, int only, hipStream_t s) {
  hipLaunchKernelGGL((k_step<R, ACC, MIX>), dim3(grid), dim3(TILE), 0, s, T, step_in_replay, mode,
                     force_build, only);
}
template <typename R>
static void launch_k_step_r(const Tables &T, int grid, int step_in_replay, int mode,
                            int force_build, int only, hipStream_t s, bool accum, bool mix) {
  if (accum) {
    if (mix) launch_k_step<R, true, true>(T, grid, step_in_replay, mode, force_build, only, s);
    else launch_k_step<R, true, false>(T, grid, step_in_replay, mode, force_build, only, s);
  } else {
    if (mix) launch_k_step<R, false, true>(T, grid, step_in_replay, mode, force_build, only, s);
    else launch_k_step<R, false, false>(T, grid, step_in_replay, mode, force_build, only, s);
  }
}
void launch_step(const Tables &T, int grid, int step_in_replay, int mode, int force_build,
                 int only, int precisions, hipStream_t s, bool accum, bool mix) {
  if (precisions & PREC_FP32)
    launch_k_step_r<float>(T, grid, step_in_replay, mode, force_build, only, s, accum, mix);
  if (precisions & PREC_FP64)
    launch_k_step_r<double>(T, grid, step_in_replay, mode, force_build, only, s, accum, mix);
}
void launch_trace(const Tables &T, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_trace, dim3(K, T.nslots), dim3(TILE), 0, s, T, K);
}
void launch_replay_end(const Tables &T, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_replay_end, dim3((T.nslots + TILE - 1) / TILE), dim3(TILE), 0, s, T, K);
}
void launch_set_target(const Tables &T, int slot, long long target, hipStream_t s) {
  hipLaunchKernelGGL(k_set_target, dim3(1), dim3(64), 0, s, T, slot, target);
}
void launch_props(const Tables &T, int only, hipStream_t s) {
  hipLaunchKernelGGL(k_props, dim3(T.nslots), dim3(TILE), 0, s, T, only);
}
void launch_adjust(const Tables &T, int grid, int only, double temperature, hipStream_t s) {
  hipLaunchKernelGGL(k_adjust, dim3(grid), dim3(TILE), 0, s, T, only, temperature);
}
void launch_insert(const Tables &T, int grid, int wrap_store, int only, hipStream_t s) {
  hipLaunchKernelGGL(k_insert, dim3(grid), dim3(TILE), 0, s, T, wrap_store, only);
}
void launch_cells(const Tables &T, int grid, int only, int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_cells, dim3(grid), dim3(TILE), 0, s, T, only, out);
}
void launch_flip(const Tables &T, int only, hipStream_t s) {
  hipLaunchKernelGGL(k_flip, dim3((T.nslots + TILE - 1) / TILE), dim3(TILE), 0, s, T, only);
}
void launch_clear_set(const Tables &T, int cgrid, int only, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_set, dim3(cgrid), dim3(TILE), 0, s, T, only);
}

}  // namespace md
