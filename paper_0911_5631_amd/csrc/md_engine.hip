// md_engine.hip -- host side of the C ABI declared in include/md.h.
//
// An Engine owns a HIP stream, the per-replica descriptors and control
// blocks, and the tile tables every kernel walks.  md_system is an engine
// with one replica; md_batch is an engine with many slots.
//
// Steps are replayed from captured HIP graphs of K steps (K a power of two up
// to 64): per step a launch of the sort kernel (which does work only where
// the rebuild rule fires) and one of the step kernel, then one counter
// update.  All kernel arguments are pointers to device tables, so graphs stay
// valid when slots are admitted or released -- except when the tile tables
// have to grow: then the graphs are dropped and captured again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "md.h"
#include "md_device.h"
#include "md_kernels.h"

using namespace md;

// Device memory of md_newton3_ab_noalloc, the A/B entry point for callers
// that cannot allocate: one array per GPU, held from the library's load to
// the end of the process.  Host code never passes this name to a kernel (on
// the host it is a stand-in, not a device address): scratch_ptr() looks up
// the array's address on the calling engine's device once and keeps it.
static __device__ __align__(256) unsigned char scratch[MD_AB_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES] = {};

}  // namespace

namespace {

constexpr int MIN_DEFAULT_MCAP = 48;
constexpr int MIN_DEFAULT_HCAP = 16;
constexpr int GRAPH_CHUNK = 64;      // steps per replay graph (largest)
constexpr int PROFILE_SETS = 2;      // ping-pong event sets when profiling

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Geometry {
  int64_t n;
  int G, ncell, ntiles, nctiles, npad, hcap, mcap, cpt;
  bool cell_only, fp64, trace, noreo, nowin;
  int nr;  // reorder interval in steps (0: every rebuild)
  double L, rc, shell, rn;
};

md_status geometry(const md_params *p, Geometry *g) {
  if (!p || !g) return MD_ERR_INVALID_ARG;
  if (p->n_atoms <= 0 || p->n_atoms > (int64_t)IDX_MASK) return MD_ERR_INVALID_ARG;
  if (!(p->box > 0) || !(p->dt > 0) || !(p->r_cut > 0) || !(p->shell >= 0))
    return MD_ERR_INVALID_ARG;
  if (!std::isfinite(p->box) || !std::isfinite(p->dt) || !std::isfinite(p->r_cut) ||
      !std::isfinite(p->shell))
    return MD_ERR_INVALID_ARG;
  if (p->precision != MD_FORCE_FP32 && p->precision != MD_FORCE_FP64) return MD_ERR_INVALID_ARG;
  if (p->nebr_cap < 0 || p->cell_cap < 0 || p->reorder_interval < 0 ||
      (p->flags & ~(MD_EVEN_CELLS | MD_TRACE_PROPS | MD_NO_REORDER | MD_NO_WINDOW)))
    return MD_ERR_INVALID_ARG;
  g->n = p->n_atoms;
  g->L = p->box;
  g->rc = p->r_cut;
  g->shell = p->shell;
  g->rn = p->r_cut + p->shell;
  g->cell_only = p->shell == 0.0;
  g->fp64 = p->precision == MD_FORCE_FP64;
  g->trace = (p->flags & MD_TRACE_PROPS) != 0;
  g->noreo = (p->flags & MD_NO_REORDER) != 0;
  g->nowin = (p->flags & MD_NO_WINDOW) != 0;
  g->nr = g->noreo ? 0 : p->reorder_interval;
  const double q = std::floor(g->L / g->rn);
  if (q < 3) return MD_ERR_BOX_TOO_SMALL;
  if (q > 1290) return MD_ERR_INVALID_ARG;  // G^3 must fit int32 cell indices
  int G = (int)q;
  if (p->flags & MD_EVEN_CELLS) G -= (G & 1);
  if (G < 3) return MD_ERR_BOX_TOO_SMALL;
  g->G = G;
  g->ncell = G * G * G;
  g->ntiles = (int)((g->n + TILE - 1) / TILE);
  g->nctiles = (g->ncell + 1 + CTILE - 1) / CTILE;
  g->npad = g->ntiles * TILE;
  g->cpt = (g->ncell + g->ntiles - 1) / g->ntiles;
  // default capacities from the mean density: a list holds the atoms of a
  // sphere of radius r_n, a cell N / N_c atoms on average; the margins cover
  // the fluctuations of a fluid (rarer excesses are handled exactly: a long
  // list by the cell path, a full cell by the overflow list and regrowth)
  const double rho = (double)g->n / (g->L * g->L * g->L);
  const double sphere = 4.0 / 3.0 * M_PI * g->rn * g->rn * g->rn * rho;
  const double occ = (double)g->n / (double)g->ncell;
  const int mdef = (int)round_up((size_t)std::ceil(1.6 * sphere + 16.0), 16);
  const int hdef = (int)round_up((size_t)std::ceil(2.0 * occ + 8.0), 8);
  g->hcap = p->cell_cap > 0 ? p->cell_cap : std::max(MIN_DEFAULT_HCAP, std::min(hdef, 4096));
  g->mcap = g->cell_only ? 0
                         : (p->nebr_cap > 0 ? p->nebr_cap
                                            : std::max(MIN_DEFAULT_MCAP, std::min(mdef, 4096)));
  return MD_OK;
}

// Layout of the per-replica state block (everything but H and W), in order.
struct Layout {
  size_t pv, ids, fu, cellm, cnt, tcnt, cs, win, ovf, part, acc, vring, tpart, trace, perm, total;
};
// Bytes of one set's cell counters (cnt) and tile counters (tcnt).
size_t cnt_set_bytes(const Geometry &g) { return round_up((size_t)g.nctiles * CTILE * 4, 256); }
size_t tcnt_set_bytes(const Geometry &g) { return round_up((size_t)g.nctiles * 4, 256); }
Layout layout(const Geometry &g) {
  const size_t R = g.fp64 ? 8 : 4, np = g.npad;
  const size_t cells = (size_t)g.nctiles * CTILE;
  Layout l{};
  size_t b = 0;
  l.pv = b;
  b += round_up(12 * np * 8, 256);          // P[2][3], V[2][3]
  l.ids = b;
  b += round_up(2 * np * 4, 256);           // id, id_alt
  l.fu = b;
  b += round_up(5 * np * R, 256);           // F[3], UA[2]
  l.cellm = b;
  b += round_up(3 * np * 4, 256);           // cell, cell_alt, m
  l.cnt = b;
  b += 3 * cnt_set_bytes(g);                // cnt[3]
  l.tcnt = b;
  b += 3 * tcnt_set_bytes(g);               // tcnt[3]
  l.cs = b;
  b += round_up(cells * 4, 256);            // cell_start
  l.win = b;
  b += round_up((size_t)g.ntiles * WSTRIDE * 4, 256);  // LDS windows of the tiles
  l.ovf = b;
  b += round_up(3 * 2 * OVF_CAP * 4 + 3 * 4, 256);  // ovf[3], ovf_n[3]
  l.part = b;
  b += round_up((size_t)g.ntiles * NPART * 8, 256);
  l.acc = b;
  b += round_up((size_t)g.ntiles * NACC * 8, 256);
  l.vring = b;
  b += round_up((size_t)3 * VSPREAD * 16 * 8, 256);
  l.tpart = l.trace = 0;
  if (g.trace) {  // MD_TRACE_PROPS: per-step tile partials and the trace ring
    l.tpart = b;
    b += round_up((size_t)MAX_REPLAY * g.ntiles * 4 * 8, 256);
    l.trace = b;
    b += round_up((size_t)TRACE_RING * TRACE_W * 8, 256);
  }
  l.perm = 0;
  if (g.noreo || g.nr > 0) {  // the cell-order permutation of a sort that does not reorder
    l.perm = b;
    b += round_up((size_t)g.npad * 4, 256);
  }
  l.total = b;
  return l;
}
size_t h_bytes(const Geometry &g, int hcap) {
  return 3 * round_up((size_t)g.ncell * hcap * 4, 256);
}
size_t w_bytes(const Geometry &g, int mcap) { return round_up((size_t)mcap * g.npad * 4, 256); }
size_t total_bytes(const Geometry &g) {
  return layout(g).total + h_bytes(g, g.hcap) + (g.mcap ? w_bytes(g, g.mcap) : 0);
}

struct Replica {
  md_params p{};
  Geometry g{};
  SlotDev dev[2]{};   // descriptor variants
  void *state = nullptr, *hmat = nullptr, *wmat = nullptr;
  size_t bytes = 0;
  // a mixture: species buffers (two variants) and pair table on the device,
  // the species in original order on the host
  void *mixbuf = nullptr;
  int nsp = 0;
  std::vector<int32_t> species;
  int64_t late_bins = 0;  // ERR_UNBINNED repairs
};

}  // namespace

struct Engine {
  hipStream_t user = nullptr;
  hipStream_t work = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipEvent_t ev_t[2] = {nullptr, nullptr};  // timing events of the A/B launches
  void *h_scalar = nullptr;                 // pinned: scalars read back from the device
  int device = 0;
  md_allocator alloc{};
  bool custom_alloc = false;
  int max_slots = 0;
  bool batch = false;
  std::vector<Replica *> rep;
  SlotDev *d_slots = nullptr;   // [2 * max_slots]
  CtlDev *d_ctl = nullptr;
  int32_t *d_tile_rep = nullptr, *d_ctile_rep = nullptr, *d_hdr = nullptr;
  int32_t *d_walk = nullptr;    // k_step's tile claims (Tables::walk)
  int tile_cap = 0, ctile_cap = 0;
  CtlDev *h_ctl = nullptr;      // pinned
  SlotDev *h_slots = nullptr;   // pinned [2 * max_slots]
  int32_t *h_tab = nullptr;     // pinned: hdr + tile tables
  size_t h_tab_cap = 0;
  int grid = 1, cgrid = 1;
  // launch configuration asked for by md_configure / md_batch_configure (0:
  // the library's choice from the sizes; see apply_launch)
  int grid_req = 0, cgrid_req = 0, split_req = 0, order_req = 0;
  int split = 1;                // workgroups per cell tile of the sort in use
  int resident = MAX_GRID / 2;  // step-kernel workgroups resident at once (4 per CU)
  std::map<int, hipGraphExec_t> graphs;
  bool sticky_hip = false;
  bool verbose = getenv("MD_VERBOSE") != nullptr;
  size_t budget = 0, used = 0;
  int steps_per_run = GRAPH_CHUNK;
  int64_t host_target = 0;      // single system: target of the last md_step
  bool accum = false;           // single system: a block is open (steps sum their properties)
  bool trace = false;           // some admitted replica records a property trace
  int64_t acc_from = 0;         // single system: step at which the open block began
  bool mix = false;             // single system: several species (the mixture kernels)
  int prec = 0;                 // PREC_* bits of the admitted replicas (step-kernel variants)
  // profiling of the step kernel (eager launches bracketed by events: events
  // recorded by graph nodes cannot be timed with hipEventElapsedTime)
  bool profiling = false;
  hipEvent_t prof_ev[PROFILE_SETS][GRAPH_CHUNK][2]{};
  int prof_pending[PROFILE_SETS] = {0, 0};
  int prof_next = 0;
  long long prof_launches = 0;
  double prof_ms = 0.0;

  Tables tables() const {
    Tables t;
    t.slots = d_slots;
    t.ctl = d_ctl;
    t.tile_rep = d_tile_rep;
    t.ctile_rep = d_ctile_rep;
    t.hdr = d_hdr;
    t.walk = d_walk;
    t.nslots = max_slots;
    return t;
  }

  void *dmalloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (custom_alloc) {
      p = alloc.alloc(bytes, alloc.ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
    }
    return p;
  }
  void dfree(void *p) {
    if (!p) return;
    if (custom_alloc)
      alloc.free(p, alloc.ctx);
    else
      (void)hipFree(p);
  }
  md_status fail(const char *where = nullptr, hipError_t err = hipSuccess) {
    sticky_hip = true;
    if (verbose)
      fprintf(stderr, "md: HIP failure%s%s%s%s\n", where ? " in " : "", where ? where : "",
              err != hipSuccess ? ": " : "", err != hipSuccess ? hipGetErrorString(err) : "");
    return MD_ERR_HIP;
  }
  md_status check(const char *where) {
    hipError_t err = hipGetLastError();
    return err == hipSuccess ? MD_OK : fail(where, err);
  }
  md_status enter() {
    if (sticky_hip) return MD_ERR_HIP;
    hipError_t err = hipEventRecord(ev_in, user);
    if (err == hipSuccess) err = hipStreamWaitEvent(work, ev_in, 0);
    return err == hipSuccess ? MD_OK : fail("enter", err);
  }
  md_status leave() {
    hipError_t err = hipEventRecord(ev_out, work);
    if (err == hipSuccess) err = hipStreamWaitEvent(user, ev_out, 0);
    return err == hipSuccess ? MD_OK : fail("leave", err);
  }
};

struct md_system {
  Engine *e;
};
struct md_batch {
  Engine *e;
};

namespace {

// One ABI call's stay on the library's stream.  enter() orders that stream
// after the caller's; leave() orders the caller's stream after the work the
// call enqueued and reports its status, and an early return (an error) leaves
// through the destructor, so the caller's stream is ordered on every exit.
class Visit {
 public:
  explicit Visit(Engine *e) : e_(e) {}
  Visit(const Visit &) = delete;
  Visit &operator=(const Visit &) = delete;
  ~Visit() {
    if (open_) (void)e_->leave();
  }
  md_status enter() {
    const md_status st = e_->enter();
    open_ = st == MD_OK;
    return st;
  }
  md_status leave() {
    open_ = false;
    return e_->leave();
  }

 private:
  Engine *e_;
  bool open_ = false;
};

md_status engine_init(Engine *e, int max_slots, const md_allocator *a, void *stream) {
  e->max_slots = max_slots;
  e->rep.assign(max_slots, nullptr);
  e->user = (hipStream_t)stream;
  if (a) {
    if (!a->alloc || !a->free) return MD_ERR_INVALID_ARG;
    e->alloc = *a;
    e->custom_alloc = true;
  }
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess) e->device = dev;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      cus > 0)
    e->resident = 4 * cus;
  hipError_t err = hipStreamCreateWithFlags(&e->work, hipStreamNonBlocking);
  if (err == hipSuccess) err = hipEventCreateWithFlags(&e->ev_in, hipEventDisableTiming);
  if (err == hipSuccess) err = hipEventCreateWithFlags(&e->ev_out, hipEventDisableTiming);
  if (err == hipSuccess) err = hipEventCreate(&e->ev_t[0]);
  if (err == hipSuccess) err = hipEventCreate(&e->ev_t[1]);
  if (err == hipSuccess) err = hipHostMalloc(&e->h_scalar, 256, hipHostMallocDefault);
  if (err != hipSuccess) return e->fail("engine init", err);
  e->d_slots = (SlotDev *)e->dmalloc(sizeof(SlotDev) * 2 * max_slots);
  e->d_ctl = (CtlDev *)e->dmalloc(sizeof(CtlDev) * max_slots);
  e->d_hdr = (int32_t *)e->dmalloc(256);
  e->d_walk = (int32_t *)e->dmalloc(WALK_BYTES);
  if (!e->d_slots || !e->d_ctl || !e->d_hdr || !e->d_walk) return MD_ERR_OOM;
  err = hipHostMalloc((void **)&e->h_ctl, sizeof(CtlDev) * max_slots, hipHostMallocDefault);
  if (err == hipSuccess)
    err = hipHostMalloc((void **)&e->h_slots, sizeof(SlotDev) * 2 * max_slots,
                        hipHostMallocDefault);
  if (err != hipSuccess) return e->fail("pinned host buffers", err);
  memset(e->h_ctl, 0, sizeof(CtlDev) * max_slots);
  memset(e->h_slots, 0, sizeof(SlotDev) * 2 * max_slots);
  err = hipMemsetAsync(e->d_ctl, 0, sizeof(CtlDev) * max_slots, e->work);
  if (err == hipSuccess) err = hipMemsetAsync(e->d_slots, 0, sizeof(SlotDev) * 2 * max_slots, e->work);
  if (err == hipSuccess) err = hipMemsetAsync(e->d_hdr, 0, 256, e->work);
  if (err == hipSuccess) err = hipMemsetAsync(e->d_walk, 0, WALK_BYTES, e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  return err == hipSuccess ? MD_OK : e->fail("engine init", err);
}

void engine_free(Engine *e) {
  if (!e) return;
  if (e->work) (void)hipStreamSynchronize(e->work);
  for (auto &kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
  for (int s = 0; s < PROFILE_SETS; ++s)
    for (int k = 0; k < GRAPH_CHUNK; ++k)
      for (int q = 0; q < 2; ++q)
        if (e->prof_ev[s][k][q]) (void)hipEventDestroy(e->prof_ev[s][k][q]);
  for (Replica *r : e->rep) {
    if (!r) continue;
    e->dfree(r->state);
    e->dfree(r->hmat);
    e->dfree(r->wmat);
    delete r;
  }
  e->dfree(e->d_slots);
  e->dfree(e->d_ctl);
  e->dfree(e->d_hdr);
  e->dfree(e->d_walk);
  e->dfree(e->d_tile_rep);
  e->dfree(e->d_ctile_rep);
  if (e->h_ctl) (void)hipHostFree(e->h_ctl);
  if (e->h_slots) (void)hipHostFree(e->h_slots);
  if (e->h_tab) (void)hipHostFree(e->h_tab);
  for (hipEvent_t x : e->ev_t)
    if (x) (void)hipEventDestroy(x);
  if (e->h_scalar) (void)hipHostFree(e->h_scalar);
  if (e->ev_in) (void)hipEventDestroy(e->ev_in);
  if (e->ev_out) (void)hipEventDestroy(e->ev_out);
  if (e->work) (void)hipStreamDestroy(e->work);
  delete e;
}

// Fill both descriptor variants of a replica from its allocations.  Variant 1
// swaps the time-level buffers of P and V, id with id_alt and cell with
// cell_alt.
void describe(Replica *r) {
  const Geometry &g = r->g;
  const Layout l = layout(g);
  const size_t np = g.npad, R = g.fp64 ? 8 : 4;
  char *b = (char *)r->state;
  SlotDev d{};
  double *pv = (double *)(b + l.pv);
  for (int buf = 0; buf < 2; ++buf)
    for (int a = 0; a < 3; ++a) {
      d.P[buf][a] = pv + (buf * 3 + a) * np;
      d.V[buf][a] = pv + (6 + buf * 3 + a) * np;
    }
  d.id = (int32_t *)(b + l.ids);
  d.id_alt = d.id + np;
  d.F = b + l.fu;
  d.UA = b + l.fu + 3 * np * R;
  d.cell = (int32_t *)(b + l.cellm);
  d.cell_alt = d.cell + np;
  d.m = d.cell + 2 * np;
  for (int s = 0; s < 3; ++s) {
    d.cnt[s] = (int32_t *)(b + l.cnt + s * cnt_set_bytes(g));
    d.tcnt[s] = (int32_t *)(b + l.tcnt + s * tcnt_set_bytes(g));
    d.H[s] = (int32_t *)((char *)r->hmat + s * round_up((size_t)g.ncell * g.hcap * 4, 256));
    d.ovf[s] = (int32_t *)(b + l.ovf) + s * 2 * OVF_CAP;
  }
  d.ovf_n = (int32_t *)(b + l.ovf) + 3 * 2 * OVF_CAP;
  d.cs = (int32_t *)(b + l.cs);
  d.win = (int32_t *)(b + l.win);
  d.part = (double *)(b + l.part);
  d.acc = (double *)(b + l.acc);
  d.vring = (unsigned long long *)(b + l.vring);
  d.tpart = g.trace ? (double *)(b + l.tpart) : nullptr;
  d.trace = g.trace ? (double *)(b + l.trace) : nullptr;
  d.perm = g.noreo || g.nr > 0 ? (int32_t *)(b + l.perm) : nullptr;
  d.noreo = g.noreo ? 1 : 0;
  d.nr = g.nr;
  d.nowin = g.nowin ? 1 : 0;
  d.W = (int32_t *)r->wmat;
  d.L = g.L;
  d.halfL = 0.5 * g.L;
  d.invW = (double)g.G / g.L;
  d.rn2 = g.rn * g.rn;
  d.rc2 = g.rc * g.rc;
  d.dt = r->p.dt;
  d.hdt = 0.5 * r->p.dt;
  d.half_shell = 0.5 * g.shell;
  d.ushift = (g.rc == std::pow(2.0, 1.0 / 6.0)) ? 1.0 : 0.0;
  d.n = (int32_t)g.n;
  d.G = g.G;
  d.ncell = g.ncell;
  d.hcap = g.hcap;
  d.mcap = g.mcap;
  d.npad = g.npad;
  d.ntiles = g.ntiles;
  d.nctiles = g.nctiles;
  d.cpt = g.cpt;
  d.fp64 = g.fp64 ? 1 : 0;
  d.cell_only = g.cell_only ? 1 : 0;
  if (r->mixbuf) {
    d.tab = (const PairTab *)r->mixbuf;
    d.sp = (int32_t *)((char *)r->mixbuf + round_up(sizeof(PairTab), 256));
    d.sp_alt = d.sp + np;
    d.nsp = r->nsp;
  }
  SlotDev e = d;
  for (int a = 0; a < 3; ++a) {
    std::swap(e.P[0][a], e.P[1][a]);
    std::swap(e.V[0][a], e.V[1][a]);
  }
  std::swap(e.id, e.id_alt);
  std::swap(e.cell, e.cell_alt);
  std::swap(e.sp, e.sp_alt);
  const int32_t to = r->dev[0].tile_off, co = r->dev[0].ctile_off;
  r->dev[0] = d;
  r->dev[1] = e;
  for (int v = 0; v < 2; ++v) {
    r->dev[v].tile_off = to;
    r->dev[v].ctile_off = co;
  }
}

// Rebuild the tile tables and upload the descriptors of every slot (sync).
// Tile order of the step kernel in use: the one asked for, else passes for
// a batch (its systems rebuild at different steps, so the cost of the tiles
// is uneven and is best spread over every XCD) and XCD slabs for a single
// system (z-neighbour rows staged through the same L2).
int tile_order(const Engine *e) {
  if (e->order_req == MD_ORDER_PASSES || e->order_req == MD_ORDER_SLABS) return e->order_req;
  return e->batch ? MD_ORDER_PASSES : MD_ORDER_SLABS;
}

md_status upload_tables(Engine *e) {
  hipError_t err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) return e->fail("upload tables", err);
  int nt = 0, nct = 0;
  e->trace = false;
  for (int s = 0; s < e->max_slots; ++s) {
    Replica *r = e->rep[s];
    if (!r) continue;
    e->trace = e->trace || r->g.trace;
    for (int v = 0; v < 2; ++v) {
      r->dev[v].tile_off = nt;
      r->dev[v].ctile_off = nct;
    }
    nt += r->g.ntiles;
    nct += r->g.nctiles;
  }
  if (nt > e->tile_cap || nct > e->ctile_cap) {
    // the captured graphs hold the table pointers in their kernel arguments:
    // drop them before the tables move (the stream is idle here)
    for (auto &kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
    e->graphs.clear();
    e->dfree(e->d_tile_rep);
    e->dfree(e->d_ctile_rep);
    e->tile_cap = std::max(nt, 2 * e->tile_cap);
    e->ctile_cap = std::max(nct, 2 * e->ctile_cap);
    e->d_tile_rep = (int32_t *)e->dmalloc((size_t)e->tile_cap * 4);
    e->d_ctile_rep = (int32_t *)e->dmalloc((size_t)e->ctile_cap * 4);
    if (!e->d_tile_rep || !e->d_ctile_rep) return MD_ERR_OOM;
  }
  const size_t need = 8 + (size_t)nt + (size_t)nct;
  if (need > e->h_tab_cap) {
    if (e->h_tab) (void)hipHostFree(e->h_tab);
    e->h_tab_cap = std::max(need, 2 * e->h_tab_cap);
    err = hipHostMalloc((void **)&e->h_tab, e->h_tab_cap * 4, hipHostMallocDefault);
    if (err != hipSuccess) return e->fail("pinned tables", err);
  }
  int32_t *hdr = e->h_tab, *tr = e->h_tab + 8, *ctr = tr + nt;
  memset(hdr, 0, 32);
  hdr[HDR_NTILES] = nt;
  hdr[HDR_NCTILES] = nct;
  // workgroups per cell tile in the sort: about 1024 atoms each (a single
  // dense system has few cell tiles; a batch keeps one per tile)
  int split = 1;
  if (!e->batch && e->rep[0]) {
    const Geometry &g = e->rep[0]->g;
    const double occ = (double)g.n / (double)g.ncell;
    split = std::max(1, std::min(32, (int)std::ceil(occ * CTILE / 1024.0)));
  }
  if (e->split_req > 0) split = e->split_req;
  hdr[HDR_SPLIT] = split;
  hdr[HDR_ORDER] = tile_order(e) == MD_ORDER_PASSES ? ORDER_PASSES : ORDER_SLABS;
  for (int s = 0; s < e->max_slots; ++s) {
    Replica *r = e->rep[s];
    if (!r) {
      memset(&e->h_slots[2 * s], 0, 2 * sizeof(SlotDev));
      continue;
    }
    for (int k = 0; k < r->g.ntiles; ++k) tr[r->dev[0].tile_off + k] = s;
    for (int k = 0; k < r->g.nctiles; ++k) ctr[r->dev[0].ctile_off + k] = s;
    e->h_slots[2 * s] = r->dev[0];
    e->h_slots[2 * s + 1] = r->dev[1];
  }
  err = hipMemcpyAsync(e->d_hdr, hdr, 32, hipMemcpyHostToDevice, e->work);
  if (err == hipSuccess && nt)
    err = hipMemcpyAsync(e->d_tile_rep, tr, (size_t)nt * 4, hipMemcpyHostToDevice, e->work);
  if (err == hipSuccess && nct)
    err = hipMemcpyAsync(e->d_ctile_rep, ctr, (size_t)nct * 4, hipMemcpyHostToDevice, e->work);
  if (err == hipSuccess)
    err = hipMemcpyAsync(e->d_slots, e->h_slots, sizeof(SlotDev) * 2 * e->max_slots,
                         hipMemcpyHostToDevice, e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) return e->fail("upload tables", err);
  // workgroups per launch: a single system one per tile up to MAX_GRID (the
  // sort at most SORT_GRID: its idle launches then cost less); a batch, whose
  // tiles change with every admission, MAX_GRID for both
  if (e->batch) {
    e->grid = MAX_GRID;
    e->cgrid = MAX_GRID;
  } else {
    // as many step-kernel workgroups as the chip holds at once (four per
    // CU), each walking its XCD's slab of tiles
    e->grid = std::max(1, std::min(nt, e->resident));
    // the sort: one unit per workgroup up to SORT_GRID, rounded up to a
    // multiple of 8 so that runs of consecutive units share an XCD (see
    // xcd_block; the few workgroups past the last unit find none)
    e->cgrid = std::max(1, std::min((nct * split + 7) / 8 * 8, SORT_GRID));
  }
  if (e->grid_req > 0) e->grid = e->grid_req;
  if (e->cgrid_req > 0) e->cgrid = e->cgrid_req;
  e->split = split;
  return MD_OK;
}

md_status read_ctl(Engine *e) {
  hipError_t err = hipStreamSynchronize(e->work);
  if (err == hipSuccess)
    err = hipMemcpyAsync(e->h_ctl, e->d_ctl, sizeof(CtlDev) * e->max_slots,
                         hipMemcpyDeviceToHost, e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  return err == hipSuccess ? MD_OK : e->fail("read control blocks", err);
}

md_status write_ctl(Engine *e, int s) {
  hipError_t err = hipMemcpyAsync(&e->d_ctl[s], &e->h_ctl[s], sizeof(CtlDev),
                                  hipMemcpyHostToDevice, e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  return err == hipSuccess ? MD_OK : e->fail("write control block", err);
}

md_status status_of(int err) {
  if (err & ERR_NONFINITE) return MD_ERR_NONFINITE;
  if (err & ERR_ESCAPED) return MD_ERR_ATOM_ESCAPED;
  if (err & ERR_CELL) return MD_ERR_CELL_OVERFLOW;
  if (err & ERR_UNBINNED) return MD_ERR_STATE;  // repaired by settle(); never expected here
  return MD_OK;
}

md_status first_error(Engine *e, int only = -1) {
  for (int s = 0; s < e->max_slots; ++s)
    if (e->rep[s] && (only < 0 || s == only) && e->h_ctl[s].err) return status_of(e->h_ctl[s].err);
  return MD_OK;
}

// Wrap, bin and sort the held clean state of the replicas (all, or `only`)
// into cell order.
md_status host_sort(Engine *e, int only) {
  Tables T = e->tables();
  launch_clear_set(T, e->cgrid, only, e->work);
  launch_insert(T, e->grid, 1, only, e->work);
  launch_sort(T, e->cgrid, 0, MODE_FORCES, only, e->work);
  launch_flip(T, only, e->work);
  return e->check("sort launches");
}

// Sort and evaluate the held clean state of the replicas (all or `only`):
// the creation-time evaluation (step 0's (b)-(e)), also used after
// md_set_state and by md_bin_cells / md_build_nebr.
md_status evaluate_clean(Engine *e, int only, int mode, int force_build) {
  Tables T = e->tables();
  md_status st = host_sort(e, only);
  if (st != MD_OK) return st;
  launch_step(T, e->grid, 0, mode, force_build, only, e->prec, e->work, false, e->mix);
  launch_props(T, only, e->work);
  if ((st = e->check("evaluate launches")) != MD_OK) return st;
  if ((st = read_ctl(e)) != MD_OK) return st;
  return first_error(e, only);
}

md_status alloc_replica(Engine *e, const md_params *p, Replica **out) {
  Geometry g;
  md_status st = geometry(p, &g);
  if (st != MD_OK) return st;
  Replica *r = new (std::nothrow) Replica();
  if (!r) return MD_ERR_OOM;
  r->p = *p;
  r->g = g;
  r->bytes = total_bytes(g);
  if (e->batch && e->used + r->bytes > e->budget) {
    delete r;
    return MD_ERR_OOM;
  }
  r->state = e->dmalloc(layout(g).total);
  r->hmat = e->dmalloc(h_bytes(g, g.hcap));
  r->wmat = g.mcap ? e->dmalloc(w_bytes(g, g.mcap)) : nullptr;
  if (!r->state || !r->hmat || (g.mcap && !r->wmat)) {
    e->dfree(r->state);
    e->dfree(r->hmat);
    e->dfree(r->wmat);
    delete r;
    return MD_ERR_OOM;
  }
  hipError_t err = hipMemsetAsync(r->state, 0, layout(g).total, e->work);
  if (err == hipSuccess) err = hipMemsetAsync(r->hmat, 0, h_bytes(g, g.hcap), e->work);
  if (err == hipSuccess && r->wmat) err = hipMemsetAsync(r->wmat, 0, w_bytes(g, g.mcap), e->work);
  if (err != hipSuccess) {
    e->dfree(r->state);
    e->dfree(r->hmat);
    e->dfree(r->wmat);
    delete r;
    return e->fail("clear replica", err);
  }
  describe(r);
  e->prec |= g.fp64 ? PREC_FP64 : PREC_FP32;
  *out = r;
  return MD_OK;
}

void free_replica(Engine *e, Replica *r) {
  (void)hipStreamSynchronize(e->work);
  e->dfree(r->state);
  e->dfree(r->hmat);
  e->dfree(r->wmat);
  e->dfree(r->mixbuf);
  delete r;
}

// Upload positions (n x 3) and velocities of a clean state `step` into the
// buffers of descriptor variant `variant`; ids are reset to 0..n-1.
md_status upload_state(Engine *e, Replica *r, int variant, int64_t step, const double *pos,
                       const double *vel) {
  const int64_t n = r->g.n;
  double *h = nullptr;
  hipError_t err =
      hipHostMalloc((void **)&h, (size_t)n * 6 * 8 + (size_t)n * 4, hipHostMallocDefault);
  if (err != hipSuccess) return e->fail("pinned staging", err);
  int32_t *hid = (int32_t *)(h + 6 * n);
  for (int64_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) {
      h[a * n + i] = pos[3 * i + a];
      h[(3 + a) * n + i] = vel[3 * i + a];
    }
    hid[i] = (int32_t)i;
  }
  const SlotDev &d = r->dev[variant];
  const int pb = (int)(step & 1), vb = (int)((step + 1) & 1);
  double *dst[6] = {d.P[pb][0], d.P[pb][1], d.P[pb][2], d.V[vb][0], d.V[vb][1], d.V[vb][2]};
  for (int a = 0; a < 6 && err == hipSuccess; ++a)
    err = hipMemcpyAsync(dst[a], h + a * n, (size_t)n * 8, hipMemcpyHostToDevice, e->work);
  if (err == hipSuccess)
    err = hipMemcpyAsync(d.id, hid, (size_t)n * 4, hipMemcpyHostToDevice, e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  (void)hipHostFree(h);
  return err == hipSuccess ? MD_OK : e->fail("upload state", err);
}

// Control block of a freshly (re)initialised clean state at `step`.
void reset_ctl(CtlDev &c, int64_t step, int variant, int64_t n_rebuilds, int max_h) {
  memset(&c, 0, sizeof(CtlDev));
  c.done = c.target = c.base = step;
  c.force_step = step;
  c.err_step = INT64_MAX;
  c.bins_step = -1;
  c.n_rebuilds = n_rebuilds;
  c.clean = 1;
  for (int q = 0; q < 3; ++q) {
    c.var_ring[q] = variant;
    c.reo_ring[q] = step;  // a clean state is (re)sorted by the host in cell order
  }
  c.max_h = max_h;
}

// Clear the three cell-layer sets of a replica (counters and overflow fill).
hipError_t clear_sets(Engine *e, Replica *r) {
  const Layout l = layout(r->g);
  hipError_t err = hipMemsetAsync((char *)r->state + l.cnt, 0, l.cs - l.cnt, e->work);
  if (err == hipSuccess) err = hipMemsetAsync(r->dev[0].ovf_n, 0, 3 * 4, e->work);
  return err;
}

int held_variant(const CtlDev &c) { return c.var_ring[((c.done % 3) + 3) % 3] & 1; }

// Enlarge the cell-layer matrix of slot s after ERR_CELL and bin its held
// state again (the state itself is intact: the overflowing binning was the
// last thing the replica did).
md_status repair_cells(Engine *e, int s) {
  Replica *r = e->rep[s];
  CtlDev &c = e->h_ctl[s];
  const int hcap = std::max(2 * r->g.hcap, r->g.hcap + 16);
  const size_t grow = h_bytes(r->g, hcap) - h_bytes(r->g, r->g.hcap);
  // a batch keeps its systems within the memory budget: a system whose rows
  // cannot grow inside it keeps its error (reported for that slot alone)
  if (e->batch && e->used + grow > e->budget) return MD_ERR_OOM;
  void *h = e->dmalloc(h_bytes(r->g, hcap));
  if (!h) return MD_ERR_CELL_OVERFLOW;
  hipError_t err = hipMemsetAsync(h, 0, h_bytes(r->g, hcap), e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) return e->fail("regrow", err);
  e->dfree(r->hmat);
  r->bytes += grow;
  e->used += grow;
  r->hmat = h;
  r->g.hcap = hcap;
  describe(r);
  // all three sets start empty again (the counters live in the state block)
  if ((err = clear_sets(e, r)) != hipSuccess) return e->fail("regrow", err);
  c.err &= ~ERR_CELL;
  c.err_step = INT64_MAX;
  md_status st = upload_tables(e);
  if (st == MD_OK) st = write_ctl(e, s);
  if (st != MD_OK) return st;
  launch_insert(e->tables(), e->grid, 0, s, e->work);
  return e->check("rebin");
}

// After ERR_UNBINNED in slot s: the displacement rule fired at step
// done + 1 although the step before did not bin r(done + 1) (the maximum
// speed grew faster than the binning-ahead guess allows).  The replica holds
// r(done + 1) unchanged: bin it now and let the sort of that step use the
// rows (bins_step), then the interrupted steps resume.
md_status repair_unbinned(Engine *e, int s) {
  Replica *r = e->rep[s];
  CtlDev &c = e->h_ctl[s];
  hipError_t err = clear_sets(e, r);
  if (err != hipSuccess) return e->fail("rebin", err);
  c.err &= ~ERR_UNBINNED;
  c.err_step = INT64_MAX;
  c.bins_step = c.done + 1;
  r->late_bins += 1;
  md_status st = write_ctl(e, s);
  if (st != MD_OK) return st;
  launch_insert(e->tables(), e->grid, 0, s, e->work);
  return e->check("rebin");
}

hipGraphExec_t step_graph(Engine *e, int k) {
  const int key =
      (((k * 4 + e->prec) * 2 + (e->accum ? 1 : 0)) * 2 + (e->mix ? 1 : 0)) * 2 + (e->trace ? 1 : 0);
  auto it = e->graphs.find(key);
  if (it != e->graphs.end()) return it->second;
  Tables T = e->tables();
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  hipError_t err = hipStreamBeginCapture(e->work, hipStreamCaptureModeThreadLocal);
  if (err != hipSuccess) {
    e->fail("begin capture", err);
    return nullptr;
  }
  // a trace (like a block) needs every step's energies: the summing kernels
  for (int s = 0; s < k; ++s) {
    launch_sort(T, e->cgrid, s, MODE_STEP, -1, e->work);
    launch_step(T, e->grid, s, MODE_STEP, 0, -1, e->prec, e->work, e->accum || e->trace,
                e->mix);
  }
  if (e->trace) launch_trace(T, k, e->work);
  launch_replay_end(T, k, e->work);
  err = hipStreamEndCapture(e->work, &g);
  if (err == hipSuccess) err = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  // the executable graph goes to the device now, not at its first launch
  if (err == hipSuccess) err = hipGraphUpload(x, e->work);
  if (err != hipSuccess) {
    e->fail("graph capture", err);
    return nullptr;
  }
  e->graphs[key] = x;
  return x;
}

md_status prof_collect(Engine *e, int set) {
  const int k = e->prof_pending[set];
  if (!k) return MD_OK;
  hipError_t err = hipEventSynchronize(e->prof_ev[set][k - 1][1]);
  for (int s = 0; s < k && err == hipSuccess; ++s) {
    float ms = 0.f;
    err = hipEventElapsedTime(&ms, e->prof_ev[set][s][0], e->prof_ev[set][s][1]);
    e->prof_ms += ms;
  }
  if (err != hipSuccess) return e->fail("profile events", err);
  e->prof_launches += k;
  e->prof_pending[set] = 0;
  return MD_OK;
}

// Capture every replay graph a run of a single system can use (K =
// steps_per_run and its repeated halvings, plain kernels), so that no
// md_step pays for a capture.
md_status prepare_graphs(Engine *e) {
  for (int k = e->steps_per_run; k >= 1; k >>= 1)
    if (!step_graph(e, k)) return MD_ERR_HIP;
  hipError_t err = hipStreamSynchronize(e->work);
  return err == hipSuccess ? MD_OK : e->fail("graph upload", err);
}

// K steps of every running replica, then the counter update.
md_status replay(Engine *e, int k) {
  if (e->profiling) {
    const int set = e->prof_next;
    e->prof_next = (set + 1) % PROFILE_SETS;
    md_status st = prof_collect(e, set);
    if (st != MD_OK) return st;
    Tables T = e->tables();
    for (int s = 0; s < k; ++s) {
      launch_sort(T, e->cgrid, s, MODE_STEP, -1, e->work);
      hipError_t err = hipEventRecord(e->prof_ev[set][s][0], e->work);
      launch_step(T, e->grid, s, MODE_STEP, 0, -1, e->prec, e->work, e->accum || e->trace,
                  e->mix);
      if (err == hipSuccess) err = hipEventRecord(e->prof_ev[set][s][1], e->work);
      if (err != hipSuccess) return e->fail("profile event record", err);
    }
    if (e->trace) launch_trace(T, k, e->work);
    launch_replay_end(T, k, e->work);
    e->prof_pending[set] = k;
    return e->check("profiled step launches");
  }
  hipGraphExec_t x = step_graph(e, k);
  if (!x) return MD_ERR_HIP;
  hipError_t err = hipGraphLaunch(x, e->work);
  return err == hipSuccess ? MD_OK : e->fail("graph launch", err);
}

// Advance a single system from absolute step `from` to `to` in replays of
// steps_per_run steps and a halving decomposition of the rest.
md_status run_steps(Engine *e, int64_t from, int64_t to) {
  int64_t pos = from;
  while (pos < to) {
    int k = e->steps_per_run;
    while (k > to - pos) k >>= 1;
    md_status st = replay(e, k);
    if (st != MD_OK) return st;
    pos += k;
  }
  return MD_OK;
}

// Synchronise and repair cell-layer overflows, resuming the remaining steps
// of a single system.  Returns the first hard error.  Without may_alloc a
// repair that needs device memory (larger cell-layer rows) is not made and
// reported as MD_ERR_CELL_OVERFLOW.
md_status settle(Engine *e, bool may_alloc = true) {
  for (int round = 0; round < 8; ++round) {
    md_status st = read_ctl(e);
    if (st != MD_OK) return st;
    bool repaired = false;
    for (int s = 0; s < e->max_slots; ++s) {
      if (!e->rep[s]) continue;
      const int err = e->h_ctl[s].err;
      if (err != ERR_CELL && err != ERR_UNBINNED) continue;
      if (err == ERR_CELL && !may_alloc) return MD_ERR_CELL_OVERFLOW;
      st = err == ERR_CELL ? repair_cells(e, s) : repair_unbinned(e, s);
      if (st == MD_ERR_OOM && e->batch) continue;  // over budget: the slot keeps its error
      if (st != MD_OK) return st;
      repaired = true;
      const CtlDev &c = e->h_ctl[s];
      if (!e->batch && c.target > c.done) {
        launch_set_target(e->tables(), s, c.target, e->work);
        if ((st = run_steps(e, c.done, c.target)) != MD_OK) return st;
      }
    }
    if (!repaired || e->batch) return MD_OK;
  }
  return MD_ERR_STATE;
}

// Copy the held state of a replica to the host in original order.
md_status fetch(Engine *e, int s, double *pos, double *vel, double *force, double *u_atom,
                double *w_atom, int32_t *cell_of_atom) {
  Replica *r = e->rep[s];
  const CtlDev &c = e->h_ctl[s];
  const SlotDev &d = r->dev[held_variant(c)];
  const int64_t n = r->g.n, np = r->g.npad;
  const size_t R = r->g.fp64 ? 8 : 4;
  const int64_t k = c.clean ? c.done : c.done + 1;
  const int pb = (int)(k & 1), vb = (int)((c.clean ? k + 1 : k) & 1);
  char *h = nullptr;
  const size_t bytes = (size_t)n * (6 * 8 + 5 * R + 8);
  hipError_t err = hipHostMalloc((void **)&h, bytes, hipHostMallocDefault);
  if (err != hipSuccess) return e->fail("pinned staging", err);
  double *hp = (double *)h;
  char *hf = h + (size_t)n * 48;
  int32_t *hid = (int32_t *)(hf + (size_t)n * 5 * R);
  int32_t *hcell = hid + n;
  const double *src[6] = {d.P[pb][0], d.P[pb][1], d.P[pb][2], d.V[vb][0], d.V[vb][1], d.V[vb][2]};
  for (int a = 0; a < 6 && err == hipSuccess; ++a)
    err = hipMemcpyAsync(hp + a * n, src[a], (size_t)n * 8, hipMemcpyDeviceToHost, e->work);
  for (int a = 0; a < 3 && err == hipSuccess; ++a)
    err = hipMemcpyAsync(hf + a * n * R, (char *)d.F + a * np * R, (size_t)n * R,
                         hipMemcpyDeviceToHost, e->work);
  for (int a = 0; a < 2 && err == hipSuccess; ++a)
    err = hipMemcpyAsync(hf + (3 + a) * n * R, (char *)d.UA + a * np * R, (size_t)n * R,
                         hipMemcpyDeviceToHost, e->work);
  if (err == hipSuccess)
    err = hipMemcpyAsync(hid, d.id, (size_t)n * 4, hipMemcpyDeviceToHost, e->work);
  if (err == hipSuccess)
    err = hipMemcpyAsync(hcell, d.cell, (size_t)n * 4, hipMemcpyDeviceToHost, e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) {
    (void)hipHostFree(h);
    return e->fail("fetch", err);
  }
  for (int64_t p = 0; p < n; ++p) {
    const int64_t i = hid[p];
    if (i < 0 || i >= n) continue;
    for (int a = 0; a < 3; ++a) {
      if (pos) pos[3 * i + a] = hp[a * n + p];
      if (vel) vel[3 * i + a] = hp[(3 + a) * n + p];
      if (force)
        force[3 * i + a] = R == 8 ? ((double *)hf)[a * n + p] : (double)((float *)hf)[a * n + p];
    }
    if (u_atom) u_atom[i] = R == 8 ? ((double *)hf)[3 * n + p] : (double)((float *)hf)[3 * n + p];
    if (w_atom) w_atom[i] = R == 8 ? ((double *)hf)[4 * n + p] : (double)((float *)hf)[4 * n + p];
    if (cell_of_atom) cell_of_atom[i] = hcell[p];
  }
  (void)hipHostFree(h);
  return MD_OK;
}

void fill_props(const Replica *r, const CtlDev &c, md_props_t *o) {
  memset(o, 0, sizeof(*o));
  const double n = (double)r->g.n;
  o->ke = c.ke;
  o->pe = c.pe;
  o->virial = c.vir;
  o->ke_per_atom = c.ke / n;
  o->pe_per_atom = c.pe / n;
  o->virial_per_atom = c.vir / n;
  o->vmax = std::sqrt(c.vmax2);
  o->n_pairs = r->g.cell_only ? 0 : c.sum_m / 2;
  o->n_rebuilds = c.n_rebuilds;
  o->step = c.done;
  o->max_nebr = c.max_m;
  o->max_cell = c.max_h;
  o->cells_per_edge = r->g.G;
  o->n_late_bins = r->late_bins;
  // displacement accumulated through the held step and the rule's decision
  // for the next one (the step kernel recomputes the same from the rings)
  if (!r->g.cell_only && c.clean) {
    const int64_t k = c.done + 1;
    const double D2 = c.disp_ring[((k - 2) % 3 + 3) % 3];
    double V1;
    const uint64_t b = c.vmax_ring[((k - 1) % 3 + 3) % 3];
    memcpy(&V1, &b, 8);
    const bool rb1 = (k - 1 == c.force_step) || D2 > 0.5 * r->g.shell;
    const double D1 = (rb1 ? 0.0 : D2) + std::sqrt(V1) * r->p.dt;
    o->disp = D1;
    o->rebuild_due = D1 > 0.5 * r->g.shell ? 1 : 0;
  }
}

md_status sys_ok(md_system *s) {
  if (!s || !s->e || !s->e->rep[0]) return MD_ERR_INVALID_ARG;
  return s->e->sticky_hip ? MD_ERR_HIP : MD_OK;
}

// Synchronise a single system: repair, reduce the properties, read back.
md_status sync_system(Engine *e, bool may_alloc = true) {
  md_status st = settle(e, may_alloc);
  if (st != MD_OK) return st;
  launch_props(e->tables(), -1, e->work);
  if ((st = e->check("props")) != MD_OK) return st;
  if ((st = read_ctl(e)) != MD_OK) return st;
  return first_error(e);
}

md_status require_clean(Engine *e, bool may_alloc = true) {
  md_status st = sync_system(e, may_alloc);
  if (st != MD_OK) return st;
  return e->h_ctl[0].clean ? MD_OK : MD_ERR_STATE;
}

md_status set_force_step(Engine *e, int s) {
  md_status st = read_ctl(e);
  if (st != MD_OK) return st;
  e->h_ctl[s].force_step = e->h_ctl[s].done;
  return write_ctl(e, s);
}

// Device buffers of one A/B evaluation: the list [mcap][npad], the lengths
// [npad] followed by the overflow counter, the forces [3][npad] (FP32), the
// forces in the caller's order (n x 3, FP64) and the summed list length.
struct AbBufs {
  int32_t *W = nullptr, *M = nullptr;
  float *F = nullptr;
  double *out = nullptr;
  unsigned long long *entries = nullptr;
};

// Byte offsets of the AbBufs of one system within one block of memory.
struct AbLayout {
  size_t W, M, F, out, entries, total;
};
AbLayout ab_layout(const Geometry &g) {
  AbLayout l{};
  size_t b = 0;
  l.W = b;
  b += round_up((size_t)g.mcap * g.npad * 4, 256);
  l.M = b;
  b += round_up((size_t)g.npad * 4 + 256, 256);
  l.F = b;
  b += round_up((size_t)3 * g.npad * 4, 256);
  l.out = b;
  b += round_up((size_t)3 * g.n * 8, 256);
  l.entries = b;
  b += 256;
  l.total = b;
  return l;
}
AbBufs ab_bufs(void *base, const AbLayout &l) {
  char *c = (char *)base;
  AbBufs x;
  x.W = (int32_t *)(c + l.W);
  x.M = (int32_t *)(c + l.M);
  x.F = (float *)(c + l.F);
  x.out = (double *)(c + l.out);
  x.entries = (unsigned long long *)(c + l.entries);
  return x;
}

// Mean event-timed duration (ms) of `reps` launches of `launch` (with `before`
// enqueued ahead of each, untimed), on the engine's timing events.
template <class Before, class Launch>
hipError_t time_launches(Engine *e, int reps, Before &&before, Launch &&launch,
                         double *mean_ms) {
  double total = 0.0;
  hipError_t err = hipSuccess;
  for (int k = 0; k < reps && err == hipSuccess; ++k) {
    float ms = 0.f;
    before();
    err = hipGetLastError();
    if (err == hipSuccess) err = hipEventRecord(e->ev_t[0], e->work);
    if (err == hipSuccess) {
      launch();
      err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e->ev_t[1], e->work);
    if (err == hipSuccess) err = hipEventSynchronize(e->ev_t[1]);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e->ev_t[0], e->ev_t[1]);
    total += ms;
  }
  *mean_ms = total / reps;
  return err;
}

// The Newton's-third-law A/B at the held state, into the buffers x (however
// they were obtained: md_newton3_ab allocates them, md_newton3_ab_noalloc
// takes them from its static array).  Allocates nothing itself.
// Entries of the A/B list as (i, j) original indices (md_ab_pairs).
struct AbPairsOut {
  int64_t cap = 0;
  int32_t *pi = nullptr, *pj = nullptr;
  int64_t *n = nullptr;
};

md_status newton3_ab(Engine *e, Replica *r, int variant, int reps, const AbBufs &x,
                     double *force, double *build_ms, double *force_ms, int64_t *n_entries,
                     const AbPairsOut *pairs = nullptr) {
  const bool half = variant == MD_AB_HALF;
  // a fresh sort of the held state (as md_bin_cells), so the cells hold the
  // current positions
  md_status st = evaluate_clean(e, -1, MODE_FORCES, 1);
  if (st == MD_OK) st = set_force_step(e, 0);
  if (st != MD_OK) return st;
  const Geometry &g = r->g;
  const CtlDev &c = e->h_ctl[0];
  const SlotDev &d = r->dev[held_variant(c)];
  const int pb = (int)(c.done & 1);
  const int n = (int)g.n, np = g.npad, mcap = g.mcap;
  int32_t *dovf = x.M + np;
  launch_ab_zero(dovf, 4, e->work);
  double tb = 0.0, tf = 0.0;
  hipError_t err = time_launches(
      e, reps, [] {},
      [&] {
        if (variant == MD_AB_CELLS)
          launch_ab_build_cells(d.P[pb][0], d.P[pb][1], d.P[pb][2], d.cs, np, g.G, g.L,
                                g.rn * g.rn, mcap, x.W, x.M, dovf, e->work);
        else
          launch_ab_build(half, d.P[pb][0], d.P[pb][1], d.P[pb][2], d.cell, d.cs, n, np, g.G,
                          g.L, g.rn * g.rn, mcap, x.W, x.M, dovf, e->work);
      },
      &tb);
  if (err == hipSuccess)
    err = hipMemcpyAsync(e->h_scalar, dovf, 4, hipMemcpyDeviceToHost, e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) return e->fail("newton3 a/b build", err);
  if (*(volatile int32_t *)e->h_scalar != 0) return MD_ERR_NEBR_OVERFLOW;
  if (pairs) {
    // the list as it stands, in original indices
    std::vector<int32_t> W((size_t)mcap * np), M(n), id(n);
    err = hipMemcpyAsync(W.data(), x.W, W.size() * 4, hipMemcpyDeviceToHost, e->work);
    if (err == hipSuccess)
      err = hipMemcpyAsync(M.data(), x.M, (size_t)n * 4, hipMemcpyDeviceToHost, e->work);
    if (err == hipSuccess)
      err = hipMemcpyAsync(id.data(), d.id, (size_t)n * 4, hipMemcpyDeviceToHost, e->work);
    if (err == hipSuccess) err = hipStreamSynchronize(e->work);
    if (err != hipSuccess) return e->fail("a/b pairs", err);
    int64_t k = 0;
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < M[p]; ++q) {
        const int j = (int)((uint32_t)W[(size_t)q * np + p] & IDX_MASK);
        if (k < pairs->cap) {
          pairs->pi[k] = id[p];
          pairs->pj[k] = j < n ? id[j] : -1;
        }
        ++k;
      }
    *pairs->n = k;
  }
  // the half form accumulates into F: zero it before every launch
  err = time_launches(
      e, reps, [&] { if (half) launch_ab_zero(x.F, (size_t)3 * np * 4, e->work); },
      [&] {
        launch_ab_forces(half, d.P[pb][0], d.P[pb][1], d.P[pb][2], x.W, x.M, n, np, g.L,
                         g.rc * g.rc, x.F, e->work);
      },
      &tf);
  if (err != hipSuccess) return e->fail("newton3 a/b forces", err);
  launch_ab_zero(x.entries, 8, e->work);
  launch_ab_output(x.F, d.id, x.M, n, np, x.out, x.entries, e->work);
  if ((err = hipGetLastError()) == hipSuccess && force)
    err = hipMemcpyAsync(force, x.out, (size_t)3 * n * 8, hipMemcpyDeviceToHost, e->work);
  if (err == hipSuccess)
    err = hipMemcpyAsync(e->h_scalar, x.entries, 8, hipMemcpyDeviceToHost, e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) return e->fail("newton3 a/b output", err);
  if (n_entries) *n_entries = (int64_t) * (volatile unsigned long long *)e->h_scalar;
  if (build_ms) *build_ms = tb;
  if (force_ms) *force_ms = tf;
  return MD_OK;
}

// Address of this engine's device's copy of `scratch` (looked up once per
// device, with that device current; nullptr if the lookup fails).
void *scratch_ptr(Engine *e) {
  if (e->device < 0 || e->device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[e->device]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != e->device && hipSetDevice(e->device) != hipSuccess) return nullptr;
    void *p = nullptr;
    const hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != e->device) (void)hipSetDevice(cur);
    if (err != hipSuccess) return nullptr;
    g_scratch[e->device] = p;
  }
  return g_scratch[e->device];
}

// One md_newton3_ab call's allocation, released however the call ends.
struct AbAlloc {
  Engine *e;
  void *p = nullptr;
  explicit AbAlloc(Engine *eng) : e(eng) {}
  ~AbAlloc() {
    (void)hipStreamSynchronize(e->work);
    e->dfree(p);
  }
};

// Upload the species (original order) into the storage order of descriptor
// variant v, whose id array maps storage positions to original indices.
md_status upload_species(Engine *e, Replica *r, int v) {
  const int64_t n = r->g.n;
  std::vector<int32_t> id(n), sp(n);
  hipError_t err = hipMemcpyAsync(id.data(), r->dev[v].id, (size_t)n * 4, hipMemcpyDeviceToHost,
                                  e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) return e->fail("species ids", err);
  for (int64_t p = 0; p < n; ++p) {
    const int32_t i = id[p];
    sp[p] = (i >= 0 && i < n) ? r->species[i] : 0;
  }
  err = hipMemcpyAsync(r->dev[v].sp, sp.data(), (size_t)n * 4, hipMemcpyHostToDevice, e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  return err == hipSuccess ? MD_OK : e->fail("upload species", err);
}

// Trace rows of steps first .. first + count - 1 of slot s (sync).
md_status read_trace(Engine *e, int s, int64_t first, int64_t count, md_trace_t *out) {
  Replica *r = e->rep[s];
  if (!r->g.trace) return MD_ERR_STATE;
  if (count < 0 || first < 1 || count > TRACE_RING) return MD_ERR_INVALID_ARG;
  if (count == 0) return MD_OK;
  if (!out) return MD_ERR_INVALID_ARG;
  const double *ring = r->dev[0].trace;
  std::vector<double> rows((size_t)count * TRACE_W);
  // at most two contiguous runs of the ring
  const int64_t a = first % TRACE_RING, n1 = std::min(count, TRACE_RING - a);
  hipError_t err = hipMemcpyAsync(rows.data(), ring + a * TRACE_W, (size_t)n1 * TRACE_W * 8,
                                  hipMemcpyDeviceToHost, e->work);
  if (err == hipSuccess && n1 < count)
    err = hipMemcpyAsync(rows.data() + n1 * TRACE_W, ring, (size_t)(count - n1) * TRACE_W * 8,
                         hipMemcpyDeviceToHost, e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) return e->fail("read trace", err);
  for (int64_t q = 0; q < count; ++q) {
    const double *w = &rows[(size_t)q * TRACE_W];
    if (w[0] != (double)(first + q)) return MD_ERR_STATE;  // not taken yet, or overwritten
    out[q].step = first + q;
    out[q].ke = w[1];
    out[q].pe = w[2];
    out[q].virial = w[3];
    out[q].vmax = std::sqrt(w[4]);
  }
  return MD_OK;
}

// Apply a launch configuration (md_configure / md_batch_configure): the
// knobs change no arithmetic and no order of it, only how the work is cut
// into workgroups and graph replays.  Fields are written back with the
// values in use.
md_status configure(Engine *e, md_launch_t *cfg) {
  if (!cfg) return MD_ERR_INVALID_ARG;
  if (cfg->steps_per_run < 0 || cfg->steps_per_run > GRAPH_CHUNK || cfg->grid < 0 ||
      cfg->grid > 65535 || cfg->sort_grid < 0 || cfg->sort_grid > 65535 ||
      cfg->sort_split < 0 || cfg->sort_split > 32 ||
      cfg->tile_order < 0 || cfg->tile_order > MD_ORDER_SLABS)
    return MD_ERR_INVALID_ARG;
  if (e->sticky_hip) return MD_ERR_HIP;
  hipError_t err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) return e->fail("configure", err);
  const int spr = cfg->steps_per_run > 0 ? cfg->steps_per_run : GRAPH_CHUNK;
  // captured graphs bake the grids and replay lengths in
  for (auto &kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
  e->graphs.clear();
  e->steps_per_run = spr;
  e->grid_req = cfg->grid;
  e->cgrid_req = cfg->sort_grid;
  e->split_req = cfg->sort_split;
  e->order_req = cfg->tile_order;
  md_status st = upload_tables(e);
  if (st == MD_OK && !e->batch) st = prepare_graphs(e);
  if (st != MD_OK) return st;
  cfg->steps_per_run = e->steps_per_run;
  cfg->grid = e->grid;
  cfg->sort_grid = e->cgrid;
  cfg->sort_split = e->split;
  cfg->tile_order = tile_order(e);
  return MD_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *md_status_string(md_status s) {
  switch (s) {
    case MD_OK: return "ok";
    case MD_ERR_INVALID_ARG: return "invalid argument";
    case MD_ERR_BOX_TOO_SMALL: return "box too small: fewer than 3 cells per edge";
    case MD_ERR_OOM: return "device memory allocation failed";
    case MD_ERR_HIP: return "HIP runtime error";
    case MD_ERR_NEBR_OVERFLOW: return "neighbour matrix capacity exceeded";
    case MD_ERR_ATOM_ESCAPED: return "atom escaped the periodic region";
    case MD_ERR_NONFINITE: return "non-finite coordinate";
    case MD_ERR_STATE: return "operation not valid in the current state";
    case MD_ERR_NO_SLOT: return "no free batch slot";
    case MD_ERR_CELL_OVERFLOW: return "cell-layer capacity exceeded";
  }
  return "unknown status";
}

md_status md_cells_per_edge(const md_params *p, int32_t *G) {
  if (!G) return MD_ERR_INVALID_ARG;
  Geometry g;
  md_status st = geometry(p, &g);
  if (st == MD_OK) *G = g.G;
  return st;
}

md_status md_query_bytes(const md_params *p, size_t *bytes) {
  if (!bytes) return MD_ERR_INVALID_ARG;
  Geometry g;
  md_status st = geometry(p, &g);
  if (st != MD_OK) return st;
  *bytes = total_bytes(g);
  return MD_OK;
}

md_status md_create(const md_params *p, const double *pos, const double *vel,
                    const md_allocator *a, void *hip_stream, md_system **out) {
  if (!p || !pos || !vel || !out) return MD_ERR_INVALID_ARG;
  *out = nullptr;
  Geometry g;
  md_status st = geometry(p, &g);
  if (st != MD_OK) return st;
  Engine *e = new (std::nothrow) Engine();
  if (!e) return MD_ERR_OOM;
  Replica *r = nullptr;
  st = engine_init(e, 1, a, hip_stream);
  if (st == MD_OK) st = e->enter();
  if (st == MD_OK) st = alloc_replica(e, p, &r);
  if (st == MD_OK) {
    e->rep[0] = r;
    e->used += r->bytes;
    st = upload_state(e, r, 0, 0, pos, vel);
  }
  if (st == MD_OK) {
    reset_ctl(e->h_ctl[0], 0, 0, 0, 0);
    st = write_ctl(e, 0);
  }
  if (st == MD_OK) st = upload_tables(e);
  for (int attempt = 0; st == MD_OK && attempt < 4; ++attempt) {
    st = evaluate_clean(e, -1, MODE_FORCES, 1);
    if (st == MD_ERR_CELL_OVERFLOW) {
      if ((st = repair_cells(e, 0)) != MD_OK) break;
      st = MD_OK;
      continue;
    }
    break;
  }
  if (st == MD_OK) st = prepare_graphs(e);
  if (st == MD_OK) st = e->leave();
  if (st != MD_OK) {
    engine_free(e);
    return st;
  }
  md_system *s = new (std::nothrow) md_system{e};
  if (!s) {
    engine_free(e);
    return MD_ERR_OOM;
  }
  *out = s;
  return MD_OK;
}

md_status md_bin_cells(md_system *s) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  Engine *e = s->e;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  if ((st = require_clean(e)) != MD_OK) return st;
  // wrap + bin + sort the held state; the new storage order invalidates the
  // list and the stored forces, so both are evaluated again
  if ((st = evaluate_clean(e, -1, MODE_FORCES, 1)) != MD_OK) return st;
  if ((st = set_force_step(e, 0)) != MD_OK) return st;
  return v.leave();
}

md_status md_build_nebr(md_system *s) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  Engine *e = s->e;
  if (e->rep[0]->g.cell_only) return MD_ERR_STATE;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  if ((st = require_clean(e)) != MD_OK) return st;
  // the list is built from the contiguous cell ranges of freshly sorted atoms
  if ((st = evaluate_clean(e, -1, MODE_FORCES, 1)) != MD_OK) return st;
  if ((st = set_force_step(e, 0)) != MD_OK) return st;
  return v.leave();
}

md_status md_forces(md_system *s) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  Engine *e = s->e;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  if ((st = require_clean(e)) != MD_OK) return st;
  launch_step(e->tables(), e->grid, 0, MODE_FORCES, 0, -1, e->prec, e->work, false, e->mix);
  if ((st = sync_system(e)) != MD_OK) return st;
  return v.leave();
}

md_status md_step(md_system *s, int64_t n_steps) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  if (n_steps < 0) return MD_ERR_INVALID_ARG;
  Engine *e = s->e;
  if (n_steps == 0) return MD_OK;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  const int64_t from = e->host_target;
  const int64_t to = from + n_steps;
  Tables T = e->tables();
  launch_set_target(T, 0, to, e->work);
  launch_kick(T, e->grid, e->work);
  if ((st = e->check("kick")) != MD_OK) return st;
  if ((st = run_steps(e, from, to)) != MD_OK) return st;
  e->host_target = to;
  return v.leave();
}

md_status md_props(md_system *s, md_props_t *out) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  if (!out) return MD_ERR_INVALID_ARG;
  Engine *e = s->e;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  st = sync_system(e);
  if (st == MD_OK || st == MD_ERR_NONFINITE || st == MD_ERR_ATOM_ESCAPED)
    fill_props(e->rep[0], e->h_ctl[0], out);
  md_status st2 = v.leave();
  return st != MD_OK ? st : st2;
}

md_status md_get_state(md_system *s, double *pos, double *vel, double *force, int64_t *step) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  Engine *e = s->e;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  if ((st = sync_system(e)) != MD_OK) return st;
  if ((st = fetch(e, 0, pos, vel, force, nullptr, nullptr, nullptr)) != MD_OK) return st;
  if (step) *step = e->h_ctl[0].done;
  return v.leave();
}

md_status md_get_atom_energies(md_system *s, double *u_atom, double *w_atom) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  Engine *e = s->e;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  if ((st = sync_system(e)) != MD_OK) return st;
  if ((st = fetch(e, 0, nullptr, nullptr, nullptr, u_atom, w_atom, nullptr)) != MD_OK) return st;
  return v.leave();
}

md_status md_set_state(md_system *s, const double *pos, const double *vel) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  if (!pos || !vel) return MD_ERR_INVALID_ARG;
  Engine *e = s->e;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  st = sync_system(e);
  if (st != MD_OK && st != MD_ERR_NONFINITE && st != MD_ERR_ATOM_ESCAPED) return st;
  Replica *r = e->rep[0];
  CtlDev &c = e->h_ctl[0];
  const int64_t step = c.clean ? c.done : c.done + 1;
  const int variant = held_variant(c);
  e->accum = false;  // an open block ends without a result
  if ((st = upload_state(e, r, variant, step, pos, vel)) != MD_OK) return st;
  if (r->mixbuf && (st = upload_species(e, r, variant)) != MD_OK) return st;
  reset_ctl(c, step, variant, c.n_rebuilds, c.max_h);
  if ((st = write_ctl(e, 0)) != MD_OK) return st;
  if (clear_sets(e, r) != hipSuccess) return e->fail("clear sets");
  if (hipMemsetAsync(r->dev[0].vring, 0, 3 * VSPREAD * 16 * 8, e->work) != hipSuccess)
    return e->fail("clear ring");
  e->host_target = step;
  if ((st = evaluate_clean(e, -1, MODE_FORCES, 1)) != MD_OK) return st;
  return v.leave();
}

md_status md_adjust_temp(md_system *s, double temperature) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  if (!(temperature > 0) || !std::isfinite(temperature)) return MD_ERR_INVALID_ARG;
  Engine *e = s->e;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  // the held state is clean after every md_step that met no error; the
  // kernels skip a replica that is not (its error is reported by the next
  // synchronising call)
  Tables T = e->tables();
  launch_props(T, -1, e->work);
  launch_adjust(T, e->grid, -1, temperature, e->work);
  if ((st = e->check("adjust launches")) != MD_OK) return st;
  return v.leave();
}

md_status md_block_begin(md_system *s) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  Engine *e = s->e;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  if ((st = sync_system(e)) != MD_OK) return st;
  Replica *r = e->rep[0];
  const Layout l = layout(r->g);
  if (hipMemsetAsync((char *)r->state + l.acc, 0, l.vring - l.acc, e->work) != hipSuccess)
    return e->fail("clear block sums");
  e->accum = true;
  e->acc_from = e->h_ctl[0].done;
  return v.leave();
}

md_status md_block_end(md_system *s, md_block_t *out) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  if (!out) return MD_ERR_INVALID_ARG;
  Engine *e = s->e;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  st = sync_system(e);
  if (st != MD_OK && st != MD_ERR_NONFINITE && st != MD_ERR_ATOM_ESCAPED) return st;
  Replica *r = e->rep[0];
  const CtlDev &c = e->h_ctl[0];
  if (!e->accum) return MD_ERR_STATE;
  memset(out, 0, sizeof(*out));
  const int64_t steps = c.done - e->acc_from;
  const double n = (double)r->g.n;
  out->steps = steps;
  if (steps > 0) {
    // per-atom sums over the full list count every pair twice
    out->ke_per_atom = 0.5 * c.acc_sum[0] / (double)steps / n;
    out->pe_per_atom = 0.5 * c.acc_sum[1] / (double)steps / n;
    out->virial_per_atom = 0.5 * c.acc_sum[2] / (double)steps / n;
    out->etot_per_atom = out->ke_per_atom + out->pe_per_atom;
    out->nebr_per_atom = r->g.cell_only ? 0.0 : c.acc_sum[3] / (double)steps / n;
  }
  e->accum = false;
  md_status st2 = v.leave();
  return st != MD_OK ? st : st2;
}

md_status md_set_species(md_system *s, int32_t n_species, const int32_t *species,
                         const double *epsilon, const double *sigma, const double *r_cut,
                         const double *shift) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  if (!species || !epsilon || !sigma || !r_cut || !shift) return MD_ERR_INVALID_ARG;
  if (n_species < 1 || n_species > MAXSP) return MD_ERR_INVALID_ARG;
  Engine *e = s->e;
  Replica *r = e->rep[0];
  const int ns = n_species;
  const int64_t n = r->g.n;
  PairTab t{};
  for (int a = 0; a < ns; ++a)
    for (int b = 0; b < ns; ++b) {
      const int q = a * ns + b, qt = b * ns + a, k = a * MAXSP + b;
      if (epsilon[q] != epsilon[qt] || sigma[q] != sigma[qt] || r_cut[q] != r_cut[qt] ||
          shift[q] != shift[qt])
        return MD_ERR_INVALID_ARG;
      if (!(sigma[q] > 0) || !std::isfinite(sigma[q]) || !(epsilon[q] >= 0) ||
          !std::isfinite(epsilon[q]) || !(r_cut[q] > 0) || r_cut[q] > r->g.rc ||
          !std::isfinite(shift[q]))
        return MD_ERR_INVALID_ARG;
      t.rc2[k] = r_cut[q] * r_cut[q];
      t.sig2[k] = sigma[q] * sigma[q];
      t.eps48[k] = 48.0 * epsilon[q];
      t.eps4[k] = 4.0 * epsilon[q];
      t.shift[k] = shift[q];
    }
  for (int64_t i = 0; i < n; ++i)
    if (species[i] < 0 || species[i] >= ns) return MD_ERR_INVALID_ARG;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  if ((st = require_clean(e)) != MD_OK) return st;
  if (!r->mixbuf) {
    const size_t bytes = round_up(sizeof(PairTab), 256) + (size_t)2 * r->g.npad * 4;
    r->mixbuf = e->dmalloc(bytes);
    if (!r->mixbuf) return MD_ERR_OOM;
    r->bytes += bytes;
    e->used += bytes;
  }
  r->nsp = ns;
  r->species.assign(species, species + n);
  describe(r);
  hipError_t err = hipMemcpyAsync(r->mixbuf, &t, sizeof(PairTab), hipMemcpyHostToDevice, e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) return e->fail("pair table", err);
  if ((st = upload_species(e, r, held_variant(e->h_ctl[0]))) != MD_OK) return st;
  if ((st = upload_tables(e)) != MD_OK) return st;
  e->mix = true;
  // the held state with its new forces (sorted again, as md_bin_cells)
  if ((st = evaluate_clean(e, -1, MODE_FORCES, 1)) != MD_OK) return st;
  if ((st = set_force_step(e, 0)) != MD_OK) return st;
  return v.leave();
}

md_status md_newton3_ab(md_system *s, int32_t variant, int32_t reps, double *force,
                        double *build_ms, double *force_ms, int64_t *n_entries) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  if (reps < 1 || reps > 100000 || variant < MD_AB_FULL || variant > MD_AB_CELLS)
    return MD_ERR_INVALID_ARG;
  Engine *e = s->e;
  Replica *r = e->rep[0];
  if (r->g.cell_only || r->nsp > 0 || r->g.noreo || r->g.nr > 0) return MD_ERR_STATE;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  if ((st = require_clean(e)) != MD_OK) return st;
  const AbLayout l = ab_layout(r->g);
  AbAlloc mem(e);
  mem.p = e->dmalloc(l.total);
  if (!mem.p) return MD_ERR_OOM;
  st = newton3_ab(e, r, variant, reps, ab_bufs(mem.p, l), force, build_ms, force_ms, n_entries);
  md_status st2 = v.leave();
  return st != MD_OK ? st : st2;
}

md_status md_ab_pairs(md_system *s, int32_t variant, int64_t cap, int32_t *pi, int32_t *pj,
                      int64_t *n_out) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  if (!n_out || cap < 0 || (cap > 0 && (!pi || !pj)) || variant < MD_AB_FULL ||
      variant > MD_AB_CELLS)
    return MD_ERR_INVALID_ARG;
  Engine *e = s->e;
  Replica *r = e->rep[0];
  if (r->g.cell_only || r->nsp > 0 || r->g.noreo || r->g.nr > 0) return MD_ERR_STATE;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  if ((st = require_clean(e)) != MD_OK) return st;
  const AbLayout l = ab_layout(r->g);
  AbAlloc mem(e);
  mem.p = e->dmalloc(l.total);
  if (!mem.p) return MD_ERR_OOM;
  AbPairsOut out;
  out.cap = cap;
  out.pi = pi;
  out.pj = pj;
  out.n = n_out;
  st = newton3_ab(e, r, variant, 1, ab_bufs(mem.p, l), nullptr, nullptr, nullptr, nullptr, &out);
  md_status st2 = v.leave();
  return st != MD_OK ? st : st2;
}

md_status md_newton3_ab_noalloc(md_system *s, int32_t variant, int32_t reps, double *force,
                                double *build_ms, double *force_ms, int64_t *n_entries) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  if (reps < 1 || reps > 100000 || variant < MD_AB_FULL || variant > MD_AB_CELLS)
    return MD_ERR_INVALID_ARG;
  Engine *e = s->e;
  Replica *r = e->rep[0];
  if (r->g.cell_only || r->nsp > 0 || r->g.noreo || r->g.nr > 0) return MD_ERR_STATE;
  const AbLayout l = ab_layout(r->g);
  if (l.total > (size_t)MD_AB_SCRATCH_BYTES) return MD_ERR_OOM;  // beyond the static array
  void *base = scratch_ptr(e);
  if (!base) return e->fail("scratch address");
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  if ((st = require_clean(e, false)) != MD_OK) return st;
  st = newton3_ab(e, r, variant, reps, ab_bufs(base, l), force, build_ms, force_ms, n_entries);
  md_status st2 = v.leave();
  return st != MD_OK ? st : st2;
}

md_status md_get_cells(md_system *s, int32_t *cell_of_atom) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  if (!cell_of_atom) return MD_ERR_INVALID_ARG;
  Engine *e = s->e;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  if ((st = sync_system(e)) != MD_OK) return st;
  // the cells of the held positions, computed on the device into the cell
  // array of the variant not in use (the next sort overwrites it anyway)
  Replica *r = e->rep[0];
  const int h = held_variant(e->h_ctl[0]);
  int32_t *scratch = r->dev[h ^ 1].cell;
  launch_cells(e->tables(), e->grid, 0, scratch, e->work);
  if ((st = e->check("cells")) != MD_OK) return st;
  const int64_t n = r->g.n;
  std::vector<int32_t> cell(n), id(n);
  hipError_t err = hipMemcpyAsync(cell.data(), scratch, (size_t)n * 4, hipMemcpyDeviceToHost,
                                  e->work);
  if (err == hipSuccess)
    err = hipMemcpyAsync(id.data(), r->dev[h].id, (size_t)n * 4, hipMemcpyDeviceToHost, e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) return e->fail("get cells", err);
  for (int64_t p = 0; p < n; ++p)
    if (id[p] >= 0 && id[p] < n) cell_of_atom[id[p]] = cell[p];
  return v.leave();
}

md_status md_get_bins(md_system *s, int32_t *order, int32_t *cell_start) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  Engine *e = s->e;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  if ((st = sync_system(e)) != MD_OK) return st;
  Replica *r = e->rep[0];
  const SlotDev &d = r->dev[held_variant(e->h_ctl[0])];
  hipError_t err = hipSuccess;
  const int64_t n = r->g.n;
  const CtlDev &hc = e->h_ctl[0];
  if (order && (r->g.noreo || hc.ord_ring[((hc.done % 3) + 3) % 3] != 0)) {
    // no reordering: cell order is perm over the (unmoved) storage
    std::vector<int32_t> perm(n), id(n);
    err = hipMemcpyAsync(perm.data(), d.perm, (size_t)n * 4, hipMemcpyDeviceToHost, e->work);
    if (err == hipSuccess)
      err = hipMemcpyAsync(id.data(), d.id, (size_t)n * 4, hipMemcpyDeviceToHost, e->work);
    if (err == hipSuccess) err = hipStreamSynchronize(e->work);
    if (err != hipSuccess) return e->fail("get bins", err);
    for (int64_t p = 0; p < n; ++p)
      order[p] = perm[p] >= 0 && perm[p] < n ? id[perm[p]] : -1;
  } else if (order) {
    err = hipMemcpyAsync(order, d.id, (size_t)n * 4, hipMemcpyDeviceToHost, e->work);
  }
  if (err == hipSuccess && cell_start)
    err = hipMemcpyAsync(cell_start, d.cs, (size_t)(r->g.ncell + 1) * 4, hipMemcpyDeviceToHost,
                         e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) return e->fail("get bins", err);
  return v.leave();
}

md_status md_get_pairs(md_system *s, int64_t cap, int32_t *pi, int32_t *pj, int64_t *n_out) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  if (!n_out || cap < 0 || (cap > 0 && (!pi || !pj))) return MD_ERR_INVALID_ARG;
  Engine *e = s->e;
  Replica *r = e->rep[0];
  if (r->g.cell_only) return MD_ERR_STATE;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  if ((st = sync_system(e)) != MD_OK) return st;
  const SlotDev &d = r->dev[held_variant(e->h_ctl[0])];
  const int64_t n = r->g.n;
  const size_t np = r->g.npad;
  std::vector<int32_t> W((size_t)r->g.mcap * np), m(n), id(n),
      win((size_t)r->g.ntiles * WSTRIDE);
  hipError_t err = hipMemcpyAsync(W.data(), d.W, W.size() * 4, hipMemcpyDeviceToHost, e->work);
  if (err == hipSuccess)
    err = hipMemcpyAsync(win.data(), d.win, win.size() * 4, hipMemcpyDeviceToHost, e->work);
  if (err == hipSuccess)
    err = hipMemcpyAsync(m.data(), d.m, (size_t)n * 4, hipMemcpyDeviceToHost, e->work);
  if (err == hipSuccess)
    err = hipMemcpyAsync(id.data(), d.id, (size_t)n * 4, hipMemcpyDeviceToHost, e->work);
  if (err == hipSuccess) err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) return e->fail("get pairs", err);
  // an entry is a storage index (GFLAG) or a slot of the tile's LDS window
  auto storage_index = [&](int64_t p, uint32_t e) -> int64_t {
    const int64_t idx = e & IDX_MASK;
    if (e & GFLAG) return idx;
    const int32_t *wt = &win[(size_t)(p / TILE) * WSTRIDE];
    for (int q = 0; q < wt[0]; ++q)
      if (idx >= wt[3 * q + 3] && idx < wt[3 * q + 3] + wt[3 * q + 2])
        return wt[3 * q + 1] + (idx - wt[3 * q + 3]);
    return -1;
  };
  int64_t k = 0;
  for (int64_t p = 0; p < n; ++p) {
    if (m[p] > r->g.mcap) return MD_ERR_NEBR_OVERFLOW;  // list incomplete for this atom
    for (int q = 0; q < m[p]; ++q) {
      const int64_t j = storage_index(p, (uint32_t)W[(size_t)q * np + p]);
      if (k < cap) {
        pi[k] = id[p];
        pj[k] = (j >= 0 && j < n) ? id[j] : -1;
      }
      ++k;
    }
  }
  *n_out = k;
  return v.leave();
}

md_status md_profile(md_system *s, int32_t enable) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  Engine *e = s->e;
  hipError_t err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) return e->fail("profile", err);
  if (enable) {
    for (int set = 0; set < PROFILE_SETS; ++set)
      for (int k = 0; k < GRAPH_CHUNK; ++k)
        for (int q = 0; q < 2; ++q)
          if (!e->prof_ev[set][k][q] &&
              (err = hipEventCreate(&e->prof_ev[set][k][q])) != hipSuccess)
            return e->fail("profile events", err);
    e->prof_launches = 0;
    e->prof_ms = 0.0;
    e->prof_pending[0] = e->prof_pending[1] = 0;
    e->profiling = true;
  } else {
    for (int set = 0; set < PROFILE_SETS; ++set)
      if ((st = prof_collect(e, set)) != MD_OK) return st;
    e->profiling = false;
  }
  return MD_OK;
}

md_status md_kernel_time(md_system *s, int64_t *launches, double *total_ms) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  if (!launches || !total_ms) return MD_ERR_INVALID_ARG;
  Engine *e = s->e;
  for (int set = 0; set < PROFILE_SETS; ++set)
    if ((st = prof_collect(e, set)) != MD_OK) return st;
  *launches = e->prof_launches;
  *total_ms = e->prof_ms;
  return MD_OK;
}

md_status md_get_trace(md_system *s, int64_t first_step, int64_t count, md_trace_t *out) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  Engine *e = s->e;
  Visit v(e);
  if ((st = v.enter()) != MD_OK) return st;
  if ((st = sync_system(e)) != MD_OK) return st;
  if ((st = read_trace(e, 0, first_step, count, out)) != MD_OK) return st;
  return v.leave();
}

md_status md_configure(md_system *s, md_launch_t *cfg) {
  md_status st = sys_ok(s);
  if (st != MD_OK) return st;
  return configure(s->e, cfg);
}

void md_destroy(md_system *s) {
  if (!s) return;
  engine_free(s->e);
  delete s;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
md_status md_batch_create(size_t hbm_budget, int32_t max_slots, int32_t steps_per_run,
                          const md_allocator *a, void *hip_stream, md_batch **out) {
  if (!out || max_slots <= 0 || steps_per_run <= 0) return MD_ERR_INVALID_ARG;
  if (steps_per_run > GRAPH_CHUNK) return MD_ERR_INVALID_ARG;
  *out = nullptr;
  Engine *e = new (std::nothrow) Engine();
  if (!e) return MD_ERR_OOM;
  e->batch = true;
  e->budget = hbm_budget;
  e->steps_per_run = steps_per_run;
  md_status st = engine_init(e, max_slots, a, hip_stream);
  if (st == MD_OK) st = upload_tables(e);
  if (st != MD_OK) {
    engine_free(e);
    return st;
  }
  md_batch *b = new (std::nothrow) md_batch{e};
  if (!b) {
    engine_free(e);
    return MD_ERR_OOM;
  }
  *out = b;
  return MD_OK;
}

md_status md_batch_configure(md_batch *b, md_launch_t *cfg) {
  if (!b || !b->e) return MD_ERR_INVALID_ARG;
  return configure(b->e, cfg);
}

md_status md_batch_admit(md_batch *b, const md_params *p, const double *pos, const double *vel,
                         int64_t n_steps, int32_t *slot) {
  if (!b || !b->e || !p || !pos || !vel || !slot || n_steps < 0) return MD_ERR_INVALID_ARG;
  Engine *e = b->e;
  if (e->sticky_hip) return MD_ERR_HIP;
  int s = -1;
  for (int k = 0; k < e->max_slots; ++k)
    if (!e->rep[k]) {
      s = k;
      break;
    }
  if (s < 0) return MD_ERR_NO_SLOT;
  Visit v(e);
  md_status st = v.enter();
  if (st != MD_OK) return st;
  Replica *r = nullptr;
  if ((st = alloc_replica(e, p, &r)) != MD_OK) return st;
  if ((st = upload_state(e, r, 0, 0, pos, vel)) != MD_OK) {
    free_replica(e, r);
    return st;
  }
  if ((st = read_ctl(e)) != MD_OK) {
    free_replica(e, r);
    return st;
  }
  e->rep[s] = r;
  e->used += r->bytes;
  reset_ctl(e->h_ctl[s], 0, 0, 0, 0);
  if ((st = write_ctl(e, s)) == MD_OK) st = upload_tables(e);
  for (int attempt = 0; st == MD_OK && attempt < 4; ++attempt) {
    st = evaluate_clean(e, s, MODE_FORCES, 1);
    if (st == MD_ERR_CELL_OVERFLOW) {
      if ((st = repair_cells(e, s)) != MD_OK) break;
      st = MD_OK;
      continue;
    }
    break;
  }
  if (st == MD_OK) {
    // the target is set only now, so the evaluation above saw a clean,
    // finished replica; the next run kicks it
    e->h_ctl[s].target = n_steps;
    st = write_ctl(e, s);
  }
  if (st != MD_OK) {
    e->used -= r->bytes;
    e->rep[s] = nullptr;
    free_replica(e, r);
    e->h_ctl[s] = CtlDev{};
    (void)write_ctl(e, s);
    (void)upload_tables(e);
    return st;
  }
  *slot = s;
  return v.leave();
}

md_status md_batch_run(md_batch *b) {
  if (!b || !b->e) return MD_ERR_INVALID_ARG;
  Engine *e = b->e;
  Visit v(e);
  md_status st = v.enter();
  if (st != MD_OK) return st;
  launch_kick(e->tables(), e->grid, e->work);
  if ((st = e->check("kick")) != MD_OK) return st;
  if ((st = replay(e, e->steps_per_run)) != MD_OK) return st;
  return v.leave();
}

md_status md_batch_poll(md_batch *b, int32_t *done, int32_t cap, int32_t *n_done) {
  if (!b || !b->e || !n_done || cap < 0 || (cap > 0 && !done)) return MD_ERR_INVALID_ARG;
  Engine *e = b->e;
  Visit v(e);
  md_status st = v.enter();
  if (st != MD_OK) return st;
  if ((st = settle(e)) != MD_OK) return st;
  int k = 0;
  for (int s = 0; s < e->max_slots; ++s) {
    if (!e->rep[s]) continue;
    const CtlDev &c = e->h_ctl[s];
    const bool finished = c.clean && c.done >= c.target;
    if (finished || c.err != 0) {
      if (k < cap) done[k] = s;
      ++k;
    }
  }
  *n_done = k;
  return v.leave();
}

md_status md_batch_props(md_batch *b, int32_t slot, md_props_t *out) {
  if (!b || !b->e || !out || slot < 0 || slot >= b->e->max_slots || !b->e->rep[slot])
    return MD_ERR_INVALID_ARG;
  Engine *e = b->e;
  launch_props(e->tables(), slot, e->work);
  md_status st = e->check("props");
  if (st == MD_OK) st = read_ctl(e);
  if (st != MD_OK) return st;
  fill_props(e->rep[slot], e->h_ctl[slot], out);
  return status_of(e->h_ctl[slot].err);
}

md_status md_batch_get_state(md_batch *b, int32_t slot, double *pos, double *vel, int64_t *step) {
  if (!b || !b->e || slot < 0 || slot >= b->e->max_slots || !b->e->rep[slot])
    return MD_ERR_INVALID_ARG;
  Engine *e = b->e;
  md_status st = read_ctl(e);
  if (st != MD_OK) return st;
  if ((st = fetch(e, slot, pos, vel, nullptr, nullptr, nullptr, nullptr)) != MD_OK) return st;
  if (step) *step = e->h_ctl[slot].done;
  return status_of(e->h_ctl[slot].err);
}

md_status md_batch_get_trace(md_batch *b, int32_t slot, int64_t first_step, int64_t count,
                             md_trace_t *out) {
  if (!b || !b->e || slot < 0 || slot >= b->e->max_slots || !b->e->rep[slot])
    return MD_ERR_INVALID_ARG;
  Engine *e = b->e;
  if (e->sticky_hip) return MD_ERR_HIP;
  hipError_t err = hipStreamSynchronize(e->work);
  if (err != hipSuccess) return e->fail("batch trace", err);
  return read_trace(e, slot, first_step, count, out);
}

md_status md_batch_release(md_batch *b, int32_t slot) {
  if (!b || !b->e || slot < 0 || slot >= b->e->max_slots || !b->e->rep[slot])
    return MD_ERR_INVALID_ARG;
  Engine *e = b->e;
  Replica *r = e->rep[slot];
  e->used -= r->bytes;
  e->rep[slot] = nullptr;
  free_replica(e, r);
  e->h_ctl[slot] = CtlDev{};
  md_status st = write_ctl(e, slot);
  if (st != MD_OK) return st;
  return upload_tables(e);
}

md_status md_batch_usage(md_batch *b, size_t *bytes, int32_t *n_systems) {
  if (!b || !b->e || !bytes || !n_systems) return MD_ERR_INVALID_ARG;
  int k = 0;
  for (Replica *r : b->e->rep) k += r != nullptr;
  *bytes = b->e->used;
  *n_systems = k;
  return MD_OK;
}

md_status md_batch_progress(md_batch *b, int64_t *atom_steps, int32_t *n_running,
                            int64_t *min_remaining) {
  if (!b || !b->e || !atom_steps || !n_running || !min_remaining) return MD_ERR_INVALID_ARG;
  Engine *e = b->e;
  if (e->sticky_hip) return MD_ERR_HIP;
  md_status st = read_ctl(e);
  if (st != MD_OK) return st;
  int64_t work = 0, rem = 0;
  int32_t running = 0;
  for (int s = 0; s < e->max_slots; ++s) {
    const Replica *r = e->rep[s];
    if (!r) continue;
    const CtlDev &c = e->h_ctl[s];
    work += r->g.n * c.done;
    if (c.err == 0 && c.done < c.target) {
      rem = running == 0 ? c.target - c.done : std::min(rem, c.target - c.done);
      ++running;
    }
  }
  *atom_steps = work;
  *n_running = running;
  *min_remaining = rem;
  return MD_OK;
}

void md_batch_destroy(md_batch *b) {
  if (!b) return;
  engine_free(b->e);
  delete b;
}

}  // extern "C"
