// md_kernels.hip -- gfx950 kernels of the soft-sphere MD hot path.
//
// One time step of every replica of an engine is ONE launch of k_step:
//   (b) when the displacement rule fires (or always with the plain cell
//       method): wrap, and build the neighbour matrix W from the cell-layer
//       rows of the current positions;
//   (c) forces from W (or from the rows);
//   (d), (e) second half kick, kinetic energy, maximum speed;
//   (a) of the next step: half kick and drift, and the binning of the new
//       positions into the next cell-layer set (cell + layer assignment).
// Nothing in k_step waits for other workgroups: the rebuild decision of step
// k is recomputed by every workgroup from the maximum speed of step k-1
// (one atomicMax per wave into a ring slot) and the displacement committed
// by step k-1, so no device-scope fence or "last block" finalisation is
// needed (on gfx950 a device-scope release writes back the whole L2).
//
// Reordering into cell order (Sec. 2.5) is a relabeling done between graph
// replays: scan of the cell occupancy (k_scan), stable in-cell ranks
// (k_rank), and a gather of every per-atom array with the neighbour indices
// remapped (k_permute).  Properties are reduced on demand (k_props) in a
// fixed order.
//
// Floating point: compiled with -ffp-contract=off, so every FP64 expression
// rounds as written (no fused multiply-add); cell indices and neighbour
// decisions are then the ones an FP64 CPU evaluation of the same expressions
// makes.
#include <hip/hip_runtime.h>

#include <limits.h>

#include "md_device.h"
#include "md_kernels.h"

namespace md {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Workgroups go to the 8 XCDs round-robin; renumber them so that each XCD
// walks a contiguous range of tiles and neighbouring atoms share an L2.
__device__ __forceinline__ int xcd_block(int b, int g) {
  if ((g & 7) == 0) return (b & 7) * (g >> 3) + (b >> 3);
  return b;
}

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

__device__ __forceinline__ int cell_of(const SlotDev &S, double x, double y, double z) {
  const int G = S.G;
  return (cell_coord(z, S.halfL, S.invW, G) * G + cell_coord(y, S.halfL, S.invW, G)) * G +
         cell_coord(x, S.halfL, S.invW, G);
}

__device__ __forceinline__ const SlotDev &slot_of(const Tables &T, int r) {
  return T.slots[2 * r + T.ctl[r].variant];
}

// State index held by a replica between launches, and where v lives.
__device__ __forceinline__ int64_t cur_state(const CtlDev &C) {
  return C.clean ? C.done : C.done + 1;
}
__device__ __forceinline__ int vbuf_of(const CtlDev &C) {
  const int64_t k = cur_state(C);
  return (int)((C.clean ? k + 1 : k) & 1);
}

__device__ __forceinline__ void latch_error(CtlDev &C, int bits, int64_t step) {
  atomicOr(&C.err, bits);
  atomicMin((unsigned long long *)&C.err_step, (unsigned long long)step);
}

// Cell and layer assignment of one atom (Secs. 2.2, 2.4): the atom's cell
// from its wrapped coordinates, a layer slot from the cell's occupancy
// counter (atomic), the row entry, or the set's overflow list beyond hcap.
__device__ void bin_atom(const SlotDev &S, CtlDev &C, int set, int i, double x, double y,
                         double z, int64_t step) {
  // Called by a prefix of the lanes of a wave (the active atoms of a tile).
  int bad = 0;
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
    bad = ERR_NONFINITE;
    x = y = z = 0.0;
  } else if (fabs(x) >= 3.0 * S.halfL || fabs(y) >= 3.0 * S.halfL || fabs(z) >= 3.0 * S.halfL) {
    bad = ERR_ESCAPED;
  }
  if (bad) latch_error(C, bad, step);
  const int c = cell_of(S, wrap1(x, S.L, S.halfL), wrap1(y, S.L, S.halfL), wrap1(z, S.L, S.halfL));
  S.cell[i] = c;
  // Consecutive lanes with the same cell take their layer slots with one
  // atomic: atoms are stored in cell order, so most of a cell's atoms are
  // neighbours in a wave.
  const int lane = threadIdx.x & 63;
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
  if (slot < S.hcap) {
    S.H[set][(size_t)c * S.hcap + slot] = i;
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

// Visit the atoms of cell c of a set in ascending storage index (the order
// of the row entries themselves depends on atomic timing, so it is not used).
template <class Visit>
__device__ __forceinline__ void visit_cell(const SlotDev &S, int set, int c, Visit &&visit) {
  const int cnt = S.cnt[set][c];
  const int32_t *__restrict__ row = S.H[set] + (size_t)c * S.hcap;
  if (cnt <= 4 && S.hcap >= 4) {
    // load the (at most four) entries together and order them with a
    // sorting network; unused places hold INT_MAX
    int a0 = cnt > 0 ? row[0] : INT_MAX, a1 = cnt > 1 ? row[1] : INT_MAX;
    int a2 = cnt > 2 ? row[2] : INT_MAX, a3 = cnt > 3 ? row[3] : INT_MAX;
#define MD_CX(p, q) { const int lo = min(p, q), hi = max(p, q); p = lo; q = hi; }
    MD_CX(a0, a1) MD_CX(a2, a3) MD_CX(a0, a2) MD_CX(a1, a3) MD_CX(a1, a2)
#undef MD_CX
    if (cnt > 0) visit(a0);
    if (cnt > 1) visit(a1);
    if (cnt > 2) visit(a2);
    if (cnt > 3) visit(a3);
    return;
  }
  const int inrow = min(cnt, S.hcap);
  int last = -1;
  for (int r = 0; r < cnt; ++r) {
    int best = INT_MAX;
    for (int e = 0; e < inrow; ++e) {
      const int v = row[e];
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
    visit(best);
  }
}

// Rebuild decision for step k (Sec. 2.1): rebuilt when the accumulated sum
// of vmax*dt exceeds delta/2.  disp after step k-1 is recomputed from the
// committed disp after step k-2 and vmax of step k-1; *disp1 receives it.
// Maximum of the spread slots of ring entry e (each wave reads all slots).
__device__ __forceinline__ double ring_max(const SlotDev &S, int64_t e) {
  const int l = threadIdx.x & 63;
  double v = 0.0;
  if (l < VSPREAD) v = __longlong_as_double((long long)S.vring[(e * VSPREAD + l) * 16]);
  return wave_max(v);
}

__device__ __forceinline__ bool rebuild_at(const SlotDev &S, const CtlDev &C, int64_t k,
                                           double *disp1) {
  const double D2 = C.disp_ring[mod3(k - 2)];
  const double V1 = ring_max(S, mod3(k - 1));
  const bool rb1 = (k - 1 == C.force_step) || D2 > S.half_shell;
  const double D1 = (rb1 ? 0.0 : D2) + sqrt(V1) * S.dt;
  *disp1 = D1;
  return (k == C.force_step) || D1 > S.half_shell;
}

// ---------------------------------------------------------------------------
// (a): first half kick and drift of a clean replica, and binning of r(k+1)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TILE) void k_kick(Tables T) {
  const int nt = T.hdr[HDR_NTILES];
  for (int t = xcd_block(blockIdx.x, gridDim.x); t < nt; t += gridDim.x) {
    const int r = T.tile_rep[t];
    const SlotDev &S = slot_of(T, r);
    CtlDev &C = T.ctl[r];
    // errors latched by this launch (err_step = done + 1) do not stop it
    if ((C.err != 0 && C.err_step <= C.done) || !C.clean || C.done >= C.target) continue;
    const int64_t k = C.done;
    const int i = (t - S.tile_off) * TILE + threadIdx.x;
    if (i >= S.n) continue;
    const int pb = (int)(k & 1), vb = (int)((k + 1) & 1);
    double f[3];
    for (int a = 0; a < 3; ++a)
      f[a] = S.fp64 ? ((const double *)S.F)[a * S.npad + i]
                    : (double)((const float *)S.F)[a * S.npad + i];
    double xn[3];
    for (int a = 0; a < 3; ++a) {
      const double v = S.V[vb][a][i] + S.hdt * f[a];
      S.V[vb][a][i] = v;
      xn[a] = S.P[pb][a][i] + S.dt * v;
      S.P[pb ^ 1][a][i] = xn[a];
    }
    bin_atom(S, C, (int)mod3(k + 1), i, xn[0], xn[1], xn[2], k + 1);
  }
}

// After k_kick: the kicked replicas hold a drifted state (one thread per
// replica; same gate as the kick).
__global__ void k_kick_end(Tables T) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= T.nslots) return;
  CtlDev &C = T.ctl[r];
  if (slot_of(T, r).n <= 0) return;
  if ((C.err != 0 && C.err_step <= C.done) || !C.clean || C.done >= C.target) return;
  C.clean = 0;
}

// ---------------------------------------------------------------------------
// (b)-(e) and the next (a): the step kernel
// ---------------------------------------------------------------------------
template <typename R>
struct Acc {
  R fx, fy, fz, u, w;
};

// Pair force and energy of Eq. (1) with the soft-sphere shift: for r^2 = s,
// f = 48 r^-8 (r^-6 - 1/2) (force on i is f d), u = 4 r^-6 (r^-6 - 1) + shift.
template <typename R>
__device__ __forceinline__ void pair_accum(Acc<R> &a, double dx, double dy, double dz, double s,
                                           R ushift) {
  const R sr = (R)s;
  const R rri = (R)1 / sr;
  const R rri3 = rri * rri * rri;
  const R f = (R)48 * rri3 * (rri3 - (R)0.5) * rri;
  a.fx += f * (R)dx;
  a.fy += f * (R)dy;
  a.fz += f * (R)dz;
  a.u += (R)4 * rri3 * (rri3 - (R)1) + ushift;
  a.w += f * sr;
}

// Image shift code: 2 bits per dimension, 0 -> 0, 1 -> +L, 2 -> -L.
__device__ __forceinline__ double img_shift(uint32_t code, double L) {
  return code == 0 ? 0.0 : (code == 1 ? L : -L);
}

// Compare-exchange network ordering eight values (Batcher odd-even merge).
#define MD_CX(p, q)                        \
  {                                        \
    const int lo_ = min(p, q), hi_ = max(p, q); \
    p = lo_;                               \
    q = hi_;                               \
  }
__device__ __forceinline__ void sort8(int (&v)[8]) {
  MD_CX(v[0], v[1]) MD_CX(v[2], v[3]) MD_CX(v[4], v[5]) MD_CX(v[6], v[7])
  MD_CX(v[0], v[2]) MD_CX(v[1], v[3]) MD_CX(v[4], v[6]) MD_CX(v[5], v[7])
  MD_CX(v[1], v[2]) MD_CX(v[5], v[6])
  MD_CX(v[0], v[4]) MD_CX(v[1], v[5]) MD_CX(v[2], v[6]) MD_CX(v[3], v[7])
  MD_CX(v[2], v[4]) MD_CX(v[3], v[5])
  MD_CX(v[1], v[2]) MD_CX(v[3], v[4]) MD_CX(v[5], v[6])
}
#undef MD_CX

// Neighbour cell number q (0..26; offsets z-major, x fastest) of the cell
// (cx, cy, cz), with the periodic image code of its atoms and their shifts.
struct NCell {
  int c;
  uint32_t code;
  double bx, by, bz;
};
__device__ __forceinline__ NCell ncell(int q, int cx, int cy, int cz, int G, double L) {
  int n[3] = {cx + q % 3 - 1, cy + (q / 3) % 3 - 1, cz + q / 9 - 1};
  uint32_t im[3];
  for (int a = 0; a < 3; ++a) {
    im[a] = 0;
    if (n[a] >= G) {
      n[a] -= G;
      im[a] = 2;
    } else if (n[a] < 0) {
      n[a] += G;
      im[a] = 1;
    }
  }
  NCell r;
  r.c = (n[2] * G + n[1]) * G + n[0];
  r.code = (im[0] | (im[1] << 2) | (im[2] << 4)) << J_BITS;
  r.bx = img_shift(im[0], L);
  r.by = img_shift(im[1], L);
  r.bz = img_shift(im[2], L);
  return r;
}

// 27-cell traversal (offsets z-major, x fastest; ascending index within a
// cell) around the wrapped position of atom i.  Accepts r^2 < r_n^2 into W
// when building, and accumulates the forces of pairs with r^2 < r_c^2.
// The occupancy and the first four row entries of the next cell are loaded
// while the current cell is evaluated; a cell's atoms are ordered with a
// sorting network and their coordinates loaded four at a time.  Cells with
// more than eight atoms take the general path.
template <typename R>
__device__ __forceinline__ int traverse_cells(const SlotDev &S, int set, int i, int ci,
                                              const double *__restrict__ X,
                                              const double *__restrict__ Y,
                                              const double *__restrict__ Z, double xi, double yi,
                                              double zi, bool build, bool force, Acc<R> &a) {
  const int G = S.G;
  const double L = S.L, halfL = S.halfL, rn2 = S.rn2, rc2 = S.rc2;
  const R ushift = (R)S.ushift;
  const int mcap = S.mcap, hcap = S.hcap;
  int32_t *__restrict__ Wc = S.W + i;
  const size_t np = (size_t)S.npad;
  const int32_t *__restrict__ CNT = S.cnt[set];
  const int32_t *__restrict__ HS = S.H[set];
  const int cx = ci % G, cy = (ci / G) % G, cz = ci / (G * G);
  const bool fast = hcap >= 8;
  int m = 0;
  auto accept = [&](int j, const NCell &nc, double xj, double yj, double zj) {
    const double dx = (xi - wrap1(xj, L, halfL)) + nc.bx;
    const double dy = (yi - wrap1(yj, L, halfL)) + nc.by;
    const double dz = (zi - wrap1(zj, L, halfL)) + nc.bz;
    const double s = (dx * dx + dy * dy) + dz * dz;
    if (s < rn2) {
      if (build) {
        if (m < mcap) Wc[(size_t)m * np] = (int32_t)((uint32_t)j | nc.code);
        ++m;
      }
      if (force && s < rc2) pair_accum<R>(a, dx, dy, dz, s, ushift);
    }
  };
  // evaluate four ordered candidates (INT_MAX marks an empty place)
  auto four = [&](const NCell &nc, int v0, int v1, int v2, int v3) {
    const int vv[4] = {v0, v1, v2, v3};
    double xj[4], yj[4], zj[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = vv[e] != INT_MAX ? vv[e] : i;
      xj[e] = X[j];
      yj[e] = Y[j];
      zj[e] = Z[j];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (vv[e] != INT_MAX && vv[e] != i) accept(vv[e], nc, xj[e], yj[e], zj[e]);
  };
  NCell cur = ncell(0, cx, cy, cz, G, L);
  int ccnt = CNT[cur.c];
  int crow[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) crow[e] = fast ? HS[(size_t)cur.c * hcap + e] : 0;
  for (int q = 0; q < 27; ++q) {
    NCell nxt = cur;
    int ncnt = 0;
    int nrow[4] = {0, 0, 0, 0};
    if (q < 26) {
      nxt = ncell(q + 1, cx, cy, cz, G, L);
      ncnt = CNT[nxt.c];
#pragma unroll
      for (int e = 0; e < 4; ++e) nrow[e] = fast ? HS[(size_t)nxt.c * hcap + e] : 0;
    }
    if (fast && ccnt <= 8) {
      int v[8];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = e < ccnt ? crow[e] : INT_MAX;
#pragma unroll
      for (int e = 4; e < 8; ++e) v[e] = e < ccnt ? HS[(size_t)cur.c * hcap + e] : INT_MAX;
      sort8(v);
      four(cur, v[0], v[1], v[2], v[3]);
      if (ccnt > 4) four(cur, v[4], v[5], v[6], v[7]);
    } else {
      visit_cell(S, set, cur.c, [&](int j) {
        if (j != i) accept(j, cur, X[j], Y[j], Z[j]);
      });
    }
    cur = nxt;
    ccnt = ncnt;
#pragma unroll
    for (int e = 0; e < 4; ++e) crow[e] = nrow[e];
  }
  return m;
}

template <typename R>
__device__ void step_tile(const SlotDev &S, CtlDev &C, int lt, int64_t k, int mode, bool cells,
                          bool build, bool last) {
  const int i = lt * TILE + threadIdx.x;
  const bool act = i < S.n;
  const int pb = (int)(k & 1);
  const int vb = mode == MODE_STEP ? pb : pb ^ 1;  // v(k-1/2) during a run, v(k) when clean
  const int set = (int)mod3(k);
  const double *__restrict__ X = S.P[pb][0];
  const double *__restrict__ Y = S.P[pb][1];
  const double *__restrict__ Z = S.P[pb][2];
  const bool force = mode != MODE_BUILD;
  const double L = S.L, halfL = S.halfL;
  Acc<R> a{(R)0, (R)0, (R)0, (R)0, (R)0};
  int m = 0;
  double xi = 0, yi = 0, zi = 0;
  if (act) {
    xi = X[i];
    yi = Y[i];
    zi = Z[i];
    if (cells) {
      // (b): the periodic correction is applied to the stored coordinates;
      // readers of neighbours wrap what they read, so the order of these
      // in-place writes does not matter.
      xi = wrap1(xi, L, halfL);
      yi = wrap1(yi, L, halfL);
      zi = wrap1(zi, L, halfL);
      S.P[pb][0][i] = xi;
      S.P[pb][1][i] = yi;
      S.P[pb][2][i] = zi;
      m = traverse_cells<R>(S, set, i, S.cell[i], X, Y, Z, xi, yi, zi, build, force, a);
      if (build) S.m[i] = m;
    } else if (force) {
      m = S.m[i];
      if (m <= S.mcap) {
        const double rc2 = S.rc2;
        const R ushift = (R)S.ushift;
        const int32_t *__restrict__ Wc = S.W + i;
        const size_t np = (size_t)S.npad;
        // four entries at a time: their twelve coordinate loads are in
        // flight together (same summation order as one at a time)
        int q = 0;
        for (; q + 4 <= m; q += 4) {
          uint32_t e[4];
          double xj[4], yj[4], zj[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) e[u] = (uint32_t)Wc[(size_t)(q + u) * np];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int j = (int)(e[u] & (uint32_t)J_MASK);
            xj[u] = X[j];
            yj[u] = Y[j];
            zj[u] = Z[j];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t code = e[u] >> J_BITS;
            const double dx = (xi - xj[u]) + img_shift(code & 3u, L);
            const double dy = (yi - yj[u]) + img_shift((code >> 2) & 3u, L);
            const double dz = (zi - zj[u]) + img_shift((code >> 4) & 3u, L);
            const double s = (dx * dx + dy * dy) + dz * dz;
            if (s < rc2) pair_accum<R>(a, dx, dy, dz, s, ushift);
          }
        }
        for (; q < m; ++q) {
          const uint32_t e = (uint32_t)Wc[(size_t)q * np];
          const int j = (int)(e & (uint32_t)J_MASK);
          const uint32_t code = e >> J_BITS;
          const double dx = (xi - X[j]) + img_shift(code & 3u, L);
          const double dy = (yi - Y[j]) + img_shift((code >> 2) & 3u, L);
          const double dz = (zi - Z[j]) + img_shift((code >> 4) & 3u, L);
          const double s = (dx * dx + dy * dy) + dz * dz;
          if (s < rc2) pair_accum<R>(a, dx, dy, dz, s, ushift);
        }
      } else {
        // the list overflowed its capacity at the last build: evaluate this
        // atom from the cells of the current positions (still exact)
        traverse_cells<R>(S, set, i, S.cell[i], X, Y, Z, wrap1(xi, L, halfL),
                          wrap1(yi, L, halfL), wrap1(zi, L, halfL), false, true, a);
      }
    }
  }

  // (d), (e) and the next (a)
  double vv = 0.0;
  if (act && force) {
    double v[3] = {S.V[vb][0][i], S.V[vb][1][i], S.V[vb][2][i]};
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
          S.P[pb ^ 1][q][i] = xn[q];
        }
        bin_atom(S, C, (int)mod3(k + 1), i, xn[0], xn[1], xn[2], k + 1);
      }
      for (int q = 0; q < 3; ++q) S.V[pb ^ 1][q][i] = v[q];
    }
    if (mode != MODE_STEP || last) {
      R *F = (R *)S.F;
      F[i] = a.fx;
      F[S.npad + i] = a.fy;
      F[2 * S.npad + i] = a.fz;
      R *U = (R *)S.UA;
      U[i] = a.u;
      U[S.npad + i] = a.w;
    }
  }

  // the set after next is cleared for the binning of step k+2
  if (mode == MODE_STEP) {
    const int zs = (int)mod3(k + 2);
    const int c0 = lt * S.cpt, c1 = min(c0 + S.cpt, S.ncell);
    for (int c = c0 + threadIdx.x; c < c1; c += TILE) S.cnt[zs][c] = 0;
    if (lt == 0 && threadIdx.x == 0) S.ovf_n[zs] = 0;
  }

  // per-tile partials (fixed reduction order) and the wave maxima of v^2
  __shared__ double sh[4][8];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int mm = act && !S.cell_only ? m : 0;
  const double ke = wave_sum(vv);
  const double vmx = wave_max(vv);
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
    sh[w][1] = vmx;
    sh[w][2] = pe_hi;
    sh[w][3] = pe_lo;
    sh[w][4] = vr_hi;
    sh[w][5] = vr_lo;
    sh[w][6] = sm;
    sh[w][7] = (double)mmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double *q = S.part + (size_t)lt * NPART;
    if (force) {
      q[0] = ((sh[0][0] + sh[1][0]) + sh[2][0]) + sh[3][0];
      q[1] = fmax(fmax(sh[0][1], sh[1][1]), fmax(sh[2][1], sh[3][1]));
      // one atomic per workgroup, spread over VSPREAD cache lines
      atomicMax(&S.vring[(mod3(k) * VSPREAD + (lt & (VSPREAD - 1))) * 16],
                (unsigned long long)__double_as_longlong(q[1]));
      if (sizeof(R) == 8) {
        q[2] = ((sh[0][2] + sh[1][2]) + sh[2][2]) + sh[3][2];
        q[3] = 0.0;
        q[4] = ((sh[0][4] + sh[1][4]) + sh[2][4]) + sh[3][4];
        q[5] = 0.0;
      } else {
        F2 e{(float)sh[0][2], (float)sh[0][3]}, v{(float)sh[0][4], (float)sh[0][5]};
        for (int k2 = 1; k2 < 4; ++k2) {
          e = f2_add(e, F2{(float)sh[k2][2], (float)sh[k2][3]});
          v = f2_add(v, F2{(float)sh[k2][4], (float)sh[k2][5]});
        }
        q[2] = e.hi;
        q[3] = e.lo;
        q[4] = v.hi;
        q[5] = v.lo;
      }
    }
    q[6] = ((sh[0][6] + sh[1][6]) + sh[2][6]) + sh[3][6];
    q[7] = fmax(fmax(sh[0][7], sh[1][7]), fmax(sh[2][7], sh[3][7]));
  }
  __syncthreads();
}

template <typename R>
__global__ __launch_bounds__(TILE, 4) void k_step(Tables T, int s, int mode, int force_build,
                                               int only) {
  const int nt = T.hdr[HDR_NTILES];
  for (int t = xcd_block(blockIdx.x, gridDim.x); t < nt; t += gridDim.x) {
    const int r = T.tile_rep[t];
    if (only >= 0 && r != only) continue;
    const SlotDev &S = slot_of(T, r);
    if (S.fp64 != (sizeof(R) == 8)) continue;  // the other precision's kernel
    CtlDev &C = T.ctl[r];
    int64_t k;
    bool last = false, cells, build;
    double disp1 = 0.0;
    if (mode == MODE_STEP) {
      k = C.base + s + 1;
      if (k > C.target) continue;
      last = k == C.target;
      if (S.cell_only) {
        cells = true;
        build = false;
      } else {
        build = rebuild_at(S, C, k, &disp1);
        cells = build;
      }
    } else {
      if (!C.clean) continue;
      k = C.done;
      build = !S.cell_only && (force_build || mode == MODE_BUILD);
      cells = build || S.cell_only;
    }
    // stop at an error of an earlier step; one latched by this launch (while
    // binning r(k+1), err_step = k + 1) must not stop the other workgroups
    if (C.err != 0 && C.err_step <= k) continue;
    const int lt = t - S.tile_off;
    step_tile<R>(S, C, lt, k, mode, cells, build, last);
    if (mode == MODE_STEP && lt == 0 && threadIdx.x == 0) {
      // the one writer of these ring slots in this launch
      if (!S.cell_only) {
        C.disp_ring[mod3(k - 1)] = disp1;
        if (build && k != C.force_step) C.n_rebuilds += 1;
      }
    }
    if (mode == MODE_STEP && lt == 0 && threadIdx.x < VSPREAD)
      S.vring[(mod3(k + 1) * VSPREAD + threadIdx.x) * 16] = 0ull;
  }
}

// End of a graph replay of K steps: advance the step counters (one thread
// per replica; no other kernel of the replay reads what is written here).
__global__ void k_replay_end(Tables T, int K) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= T.nslots) return;
  CtlDev &C = T.ctl[r];
  if (slot_of(T, r).n <= 0) return;
  if (C.base >= C.target && C.done >= C.target) return;
  int64_t done = C.base + K < C.target ? C.base + K : C.target;
  if (C.err != 0) done = C.err_step - 1 < done ? C.err_step - 1 : done;
  if (done < C.done) done = C.done;
  C.done = done;
  C.base = done;
  // a replica that ran this replay holds a drifted state unless it finished
  C.clean = (done == C.target && C.err == 0) ? 1 : 0;
}

// Switch every replica (or one) to its other descriptor after k_permute.
__global__ void k_flip(Tables T, int only) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= T.nslots || (only >= 0 && r != only)) return;
  if (T.slots[2 * r].n <= 0) return;
  T.ctl[r].variant ^= 1;
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
  const SlotDev &S = slot_of(T, r);
  CtlDev &C = T.ctl[r];
  if (S.n <= 0) return;
  __shared__ double sh[TILE][6];
  double ke = 0, vm = 0, pe = 0, vir = 0, sm = 0, mm = 0;
  for (int t = threadIdx.x; t < S.ntiles; t += TILE) {
    const double *q = S.part + (size_t)t * NPART;
    ke += q[0];
    vm = fmax(vm, q[1]);
    pe += q[2] + q[3];
    vir += q[4] + q[5];
    sm += q[6];
    mm = fmax(mm, q[7]);
  }
  sh[threadIdx.x][0] = ke;
  sh[threadIdx.x][1] = vm;
  sh[threadIdx.x][2] = pe;
  sh[threadIdx.x][3] = vir;
  sh[threadIdx.x][4] = sm;
  sh[threadIdx.x][5] = mm;
  __syncthreads();
  for (int h = TILE / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      sh[threadIdx.x][0] += sh[threadIdx.x + h][0];
      sh[threadIdx.x][1] = fmax(sh[threadIdx.x][1], sh[threadIdx.x + h][1]);
      sh[threadIdx.x][2] += sh[threadIdx.x + h][2];
      sh[threadIdx.x][3] += sh[threadIdx.x + h][3];
      sh[threadIdx.x][4] += sh[threadIdx.x + h][4];
      sh[threadIdx.x][5] = fmax(sh[threadIdx.x][5], sh[threadIdx.x + h][5]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) {
    double v = 0.0;
    for (int q = 0; q < VSPREAD; ++q)
      v = fmax(v, __longlong_as_double((long long)S.vring[(threadIdx.x * VSPREAD + q) * 16]));
    C.vmax_ring[threadIdx.x] = (uint64_t)__double_as_longlong(v);
  }
  if (threadIdx.x == 0) {
    C.ke = 0.5 * sh[0][0];
    C.vmax2 = sh[0][1];
    C.pe = 0.5 * sh[0][2];
    C.vir = 0.5 * sh[0][3];
    C.sum_m = (int64_t)sh[0][4];
    C.max_m = (int)sh[0][5];
  }
}

// ---------------------------------------------------------------------------
// binning of the held state outside a step (creation, reordering)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TILE) void k_insert(Tables T, int wrap_store, int only) {
  const int nt = T.hdr[HDR_NTILES];
  for (int t = xcd_block(blockIdx.x, gridDim.x); t < nt; t += gridDim.x) {
    const int r = T.tile_rep[t];
    if (only >= 0 && r != only) continue;
    const SlotDev &S = slot_of(T, r);
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

// cell_start = exclusive scan of the occupancy of the held state's set, in a
// single pass: tiles take tickets in launch order and look back at earlier
// tiles of the same replica.  The status words carry the values themselves,
// so relaxed device-scope atomics suffice (no fences).
__device__ __forceinline__ unsigned long long st_pack(uint32_t epoch, int flag, uint32_t v) {
  return ((unsigned long long)(epoch & 0x3FFFFFFFu) << 34) | ((unsigned long long)flag << 32) | v;
}

__global__ __launch_bounds__(TILE) void k_scan(Tables T, unsigned epoch, int only) {
  __shared__ int s_ticket;
  __shared__ int s_wsum[4];
  __shared__ int s_excl;
  const int nct = T.hdr[HDR_NCTILES];
  for (;;) {
    if (threadIdx.x == 0) s_ticket = atomicAdd(&T.hdr[HDR_TICKET], 1);
    __syncthreads();
    const int t = s_ticket;
    __syncthreads();
    if (t >= nct) break;
    const int r = T.ctile_rep[t];
    if (only >= 0 && r != only) continue;
    const SlotDev &S = slot_of(T, r);
    CtlDev &C = T.ctl[r];
    const int set = (int)mod3(cur_state(C));
    const int lt = t - S.ctile_off;
    const int c0 = lt * CTILE + threadIdx.x * 8;
    int v[8];
    int run = 0, vmax = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int c = c0 + q;
      const int cnt = c < S.ncell ? S.cnt[set][c] : 0;
      v[q] = run;
      run += cnt;
      vmax = max(vmax, cnt);
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    int incl = run;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o, 64);
      if (l >= o) incl += y;
    }
    if (l == 63) s_wsum[w] = incl;
    vmax = wave_max_i(vmax);
    __syncthreads();
    int before = 0;
    for (int q = 0; q < w; ++q) before += s_wsum[q];
    const int excl_thread = before + incl - run;
    const int agg = s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
    if (l == 0) atomicMax(&C.max_h, vmax);
    if (threadIdx.x == 0) {
      unsigned long long *st = S.scan_st;
      int excl = 0;
      if (lt == 0) {
        __hip_atomic_store(&st[0], st_pack(epoch, 2, (uint32_t)agg), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      } else {
        __hip_atomic_store(&st[lt], st_pack(epoch, 1, (uint32_t)agg), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        int j = lt - 1;
        long spins = 0;
        while (j >= 0) {
          const unsigned long long sv =
              __hip_atomic_load(&st[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const int flag = (int)((sv >> 32) & 3ull);
          if ((uint32_t)(sv >> 34) != (epoch & 0x3FFFFFFFu) || flag == 0) {
            if (++spins > (1l << 24)) {
              atomicOr(&C.err, ERR_SCAN);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
          }
          excl += (int)(sv & 0xFFFFFFFFull);
          if (flag == 2) break;
          --j;
        }
        __hip_atomic_store(&st[lt], st_pack(epoch, 2, (uint32_t)(excl + agg)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
      s_excl = excl;
    }
    __syncthreads();
    const int base = s_excl + excl_thread;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int c = c0 + q;
      if (c < S.ncell) S.cs[c] = base + v[q];
    }
    if (c0 <= S.ncell && S.ncell < c0 + 8) S.cs[S.ncell] = base + run;
    __syncthreads();
  }
}

// New position of every atom: cell_start of its cell plus its rank among the
// cell's atoms by current storage index (the sequential layer assignment of
// Sec. 2.4 read in cell order, Sec. 2.5).
__global__ __launch_bounds__(TILE) void k_rank(Tables T, int only) {
  const int nct = T.hdr[HDR_NCTILES];
  for (int t = xcd_block(blockIdx.x, gridDim.x); t < nct; t += gridDim.x) {
    const int r = T.ctile_rep[t];
    if (only >= 0 && r != only) continue;
    const SlotDev &S = slot_of(T, r);
    const CtlDev &C = T.ctl[r];
    const int set = (int)mod3(cur_state(C));
    const int lt = t - S.ctile_off;
    for (int q = 0; q < CTILE / TILE; ++q) {
      const int c = lt * CTILE + q * TILE + threadIdx.x;
      if (c >= S.ncell) break;
      const int start = S.cs[c];
      const int stop = S.cs[c + 1];
      int rank = 0;
      visit_cell(S, set, c, [&](int a) {
        if (start + rank < stop && start + rank < S.n) {
          S.perm[start + rank] = a;
          S.inv[a] = start + rank;
        }
        ++rank;
      });
    }
  }
}

// Gather every per-atom array into cell order; neighbour indices are mapped
// to the new positions.  Writes the alternate buffers (the host swaps them).
__global__ __launch_bounds__(TILE) void k_permute(Tables T, int only) {
  if (blockIdx.x == 0 && threadIdx.x == 0) T.hdr[HDR_TICKET] = 0;  // for the next k_scan
  const int nt = T.hdr[HDR_NTILES];
  for (int t = xcd_block(blockIdx.x, gridDim.x); t < nt; t += gridDim.x) {
    const int r = T.tile_rep[t];
    if (only >= 0 && r != only) continue;
    const SlotDev &S = slot_of(T, r);
    const CtlDev &C = T.ctl[r];
    const int p = (t - S.tile_off) * TILE + threadIdx.x;
    if (p >= S.n) continue;
    const int64_t k = cur_state(C);
    const int pb = (int)(k & 1), vb = vbuf_of(C);
    // a replica with a latched error keeps its order (identity gather), so
    // the descriptor flip below stays consistent without reading its ranks
    const bool ident = C.err != 0;
    const int a = ident ? p : S.perm[p];
    for (int q = 0; q < 3; ++q) {
      S.P[pb ^ 1][q][p] = S.P[pb][q][a];
      S.V[vb ^ 1][q][p] = S.V[vb][q][a];
    }
    S.id_alt[p] = S.id[a];
    S.cell_alt[p] = S.cell[a];
    const int m = S.m[a];
    S.m_alt[p] = m;
    const int mq = min(m, S.mcap);
    const size_t np = (size_t)S.npad;
    for (int q = 0; q < mq; ++q) {
      const uint32_t e = (uint32_t)S.W[(size_t)q * np + a];
      const uint32_t j = e & (uint32_t)J_MASK;
      S.W_alt[(size_t)q * np + p] =
          (int32_t)((ident ? j : (uint32_t)S.inv[j]) | (e & ~(uint32_t)J_MASK));
    }
    if (S.fp64) {
      const double *F = (const double *)S.F, *U = (const double *)S.UA;
      double *Fo = (double *)S.F_alt, *Uo = (double *)S.UA_alt;
      for (int q = 0; q < 3; ++q) Fo[q * np + p] = F[q * np + a];
      Uo[p] = U[a];
      Uo[np + p] = U[np + a];
    } else {
      const float *F = (const float *)S.F, *U = (const float *)S.UA;
      float *Fo = (float *)S.F_alt, *Uo = (float *)S.UA_alt;
      for (int q = 0; q < 3; ++q) Fo[q * np + p] = F[q * np + a];
      Uo[p] = U[a];
      Uo[np + p] = U[np + a];
    }
  }
}

// Clear the cell-layer set of the held state (before re-binning it).
__global__ __launch_bounds__(TILE) void k_clear_set(Tables T, int only) {
  const int nct = T.hdr[HDR_NCTILES];
  for (int t = xcd_block(blockIdx.x, gridDim.x); t < nct; t += gridDim.x) {
    const int r = T.ctile_rep[t];
    if (only >= 0 && r != only) continue;
    const SlotDev &S = slot_of(T, r);
    const CtlDev &C = T.ctl[r];
    const int set = (int)mod3(cur_state(C));
    const int lt = t - S.ctile_off;
    for (int q = 0; q < CTILE / TILE; ++q) {
      const int c = lt * CTILE + q * TILE + threadIdx.x;
      if (c < S.ncell) S.cnt[set][c] = 0;
    }
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
void launch_step(const Tables &T, int grid, int step_in_replay, int mode, int force_build,
                 int only, int precisions, hipStream_t s) {
  if (precisions & PREC_FP32)
    hipLaunchKernelGGL(k_step<float>, dim3(grid), dim3(TILE), 0, s, T, step_in_replay, mode,
                       force_build, only);
  if (precisions & PREC_FP64)
    hipLaunchKernelGGL(k_step<double>, dim3(grid), dim3(TILE), 0, s, T, step_in_replay, mode,
                       force_build, only);
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
void launch_insert(const Tables &T, int grid, int wrap_store, int only, hipStream_t s) {
  hipLaunchKernelGGL(k_insert, dim3(grid), dim3(TILE), 0, s, T, wrap_store, only);
}
void launch_reorder(const Tables &T, int grid, int cgrid, unsigned epoch, int only,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(cgrid), dim3(TILE), 0, s, T, epoch, only);
  hipLaunchKernelGGL(k_rank, dim3(cgrid), dim3(TILE), 0, s, T, only);
  hipLaunchKernelGGL(k_permute, dim3(grid), dim3(TILE), 0, s, T, only);
}
void launch_flip(const Tables &T, int only, hipStream_t s) {
  hipLaunchKernelGGL(k_flip, dim3((T.nslots + TILE - 1) / TILE), dim3(TILE), 0, s, T, only);
}
void launch_clear_set(const Tables &T, int cgrid, int only, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_set, dim3(cgrid), dim3(TILE), 0, s, T, only);
}

}  // namespace md
