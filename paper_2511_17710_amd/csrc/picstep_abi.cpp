// picstep_abi.cpp -- the C ABI declared in include/picstep.h: host-side
// validation, metric set-up in FP64, buffer layout, and the step loop that
// enqueues the HIP kernels on the bound stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/picstep.h"
#include "internal.h"

using namespace picstep;

namespace {
constexpr double PI = 3.14159265358979323846;
constexpr uint64_t ALIGN = 256;
constexpr uint64_t NONE = ~0ull;

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }
int bits_for(int64_t values) {  // bits to represent 0..values-1
  int b = 0;
  while ((int64_t(1) << b) < values) ++b;
  return b;
}
}  // namespace

struct pic_ctx {
  pic_grid_desc d{};
  GridConst g{};
  size_t eb = 4;  // element bytes
  int nspec = 0;
  double q[MAXSP]{}, m[MAXSP]{};
  int pusher[MAXSP]{};                       // pic_pusher per species
  double gca_e_ovr[MAXSP]{}, gca_larmor[MAXSP]{};
  uint64_t cap[MAXSP]{}, off[MAXSP]{}, cnt[MAXSP]{};
  uint64_t capacity = 0;  // elements per particle array
  // particle set layout (byte offsets)
  uint64_t o_cell = 0, o_offs[3]{NONE, NONE, NONE}, o_u[3]{}, o_w = 0, o_phi = NONE, o_id = 0;
  uint64_t set_bytes = 0;
  uint64_t p_cell = 0, p_offs[3]{NONE, NONE, NONE}, prev_bytes = 0;
  // scratch layout
  uint64_t s_keys[2]{}, s_vals[2]{}, s_hist = 0, s_bsum = 0, s_perm = 0, s_stats = 0,
           scratch_bytes = 0;
  int64_t max_tiles = 0;
  int keybits = 0;
  uint64_t ckpt_bytes = 0;
  // bound buffers
  char *fields = nullptr, *current = nullptr, *pset[2]{nullptr, nullptr}, *prev = nullptr,
       *scratch = nullptr;
  bool bound = false, fields_ok = false, loaded = false;
  int active = 0;
  hipStream_t stream = nullptr;
  int64_t step = 0;
  double dx_min = 0;  // Sec. 2.4 CFL length
  int32_t ckpt_K = -1, ckpt_m = -1;  // last pic_forward_checkpointed
  double ckpt_dt = 0.0;
  int64_t ckpt_step0 = 0;
  std::vector<int32_t> ckpt_sorts;  // steps n of that run that began with a sort
  bool perm_pending = false;        // a sort's reorder left to the next step
  // brick-neighbour sort: brick starts of the last sort per species (two
  // arrays each, bsel the current one), whether they describe the present
  // order, and a bound on the cells any particle can have moved since
  uint64_t s_bstart = 0, s_bcnt = 0, s_btot = 0, s_bdpre = 0, s_err = 0;
  int nbricks = 0, brick_min = 0;
  int bsel[MAXSP]{};
  bool bricks_valid = false;
  int64_t brick_sorts = 0;  // sorts that took the brick-neighbour form
  double moved = 0.0;
  double max_inv_dx = 0.0;  // Cartesian: largest 1 / dx
  bool timing = false;
  bool debug_serial = false;  // the fused step kernel launched one block at a time
  struct Ev {
    hipEvent_t a, b;
    int kind;  // 0 push, 1 sort, 2 adjoint
  };
  std::vector<Ev> events;
  std::string err;
  ~pic_ctx() {
    for (auto &e : events) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
  }
};

namespace {

pic_status fail(const pic_ctx *c, pic_status s, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    const_cast<pic_ctx *>(c)->err = buf;
  }
  return s;
}

pic_status hipchk(const pic_ctx *c, hipError_t e, const char *what) {
  if (e == hipSuccess) return PIC_OK;
  return fail(c, PIC_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ---- host metric (Sec. 2.4), FP64 ----
double h_r(const GridConst &g, double x1) {
  return (g.geom == 1) ? g.rmin + x1 * g.dr : g.r0 + std::exp(g.Rmin + x1 * g.dR);
}
double h_theta(const GridConst &g, double x2) {
  if (g.geom == 1) return x2 * g.dth;
  const double T = x2 * g.dT;
  return T + 2.0 * g.vt * T * (1.0 - 2.0 * T / PI) * (1.0 - T / PI);
}
void h_sqrt_h(const GridConst &g, double x1, double x2, double h[3]) {
  if (g.geom == 0) {
    for (int a = 0; a < 3; ++a) h[a] = g.dx[a];
    return;
  }
  const double r = h_r(g, x1);
  if (g.geom == 1) {
    h[0] = g.dr;
    h[1] = r * g.dth;
  } else {
    const double T = x2 * g.dT;
    const double tp = T / PI;
    h[0] = g.dR * std::exp(g.Rmin + x1 * g.dR);
    h[1] = g.dT * (1.0 + 2.0 * g.vt + 12.0 * g.vt * tp * (tp - 1.0)) * r;
  }
  h[2] = r * std::sin(h_theta(g, x2));
}

// Yee offsets (App. A) of E1..B3
const double STAG[6][3] = {{0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 0.5},
                           {0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}};

template <class Real>
PSet<Real> pset_of(const pic_ctx *c, int which) {
  PSet<Real> p{};
  char *b = c->pset[which];
  p.cell = reinterpret_cast<int32_t *>(b + c->o_cell);
  for (int a = 0; a < 3; ++a) {
    p.offs[a] = c->o_offs[a] == NONE ? nullptr : reinterpret_cast<OffT<Real> *>(b + c->o_offs[a]);
    p.u[a] = reinterpret_cast<Real *>(b + c->o_u[a]);
  }
  p.w = reinterpret_cast<Real *>(b + c->o_w);
  p.phi = c->o_phi == NONE ? nullptr : reinterpret_cast<Real *>(b + c->o_phi);
  p.id = reinterpret_cast<int32_t *>(b + c->o_id);
  return p;
}

SpeciesTable species_table(const pic_ctx *c, double dt, int64_t per_block) {
  SpeciesTable t{};
  t.nspec = c->nspec;
  t.blk0[0] = 0;
  for (int s = 0; s < c->nspec; ++s) {
    t.off[s] = (int64_t)c->off[s];
    t.n[s] = (int64_t)c->cnt[s];
    t.blk0[s + 1] = t.blk0[s] + (t.n[s] + per_block - 1) / per_block;
    t.k[s] = c->q[s] * dt / (2.0 * c->m[s] * c->d.rho0);
    t.kf[s] = (float)t.k[s];
    t.qdt[s] = c->q[s] / dt;
    t.pusher[s] = c->pusher[s];
    t.gca_e_ovr[s] = c->gca_e_ovr[s];
    t.gca_larmor[s] = c->gca_larmor[s];
  }
  for (int s = c->nspec; s < MAXSP; ++s) t.blk0[s + 1] = t.blk0[c->nspec];
  return t;
}

// The fused step kernel's chunks: BLOCK threads of 1, 2 or 4 particles.  A
// chunk of the sorted order covers about chunk / ppc cells, which the LDS
// tiles must hold after the drift between sorts: 4 per thread (1024, half a
// brick at 16 per cell) down to 1 (256) for species below 3 particles per
// cell on average, where a 1024-chunk would stretch over several bricks.
SpeciesTable push_species_table(const pic_ctx *c, double dt) {
  SpeciesTable t = species_table(c, dt, BLOCK * PUSH_PPT);
  const double ncells = (double)c->g.n[0] * c->g.n[1] * c->g.n[2];
  const int most = c->eb == 4 ? 4 : 2;  // the dense instance's layout (FP64: 2)
  for (int s = 0; s < c->nspec; ++s) {
    const double ppc = (double)t.n[s] / ncells;
    t.ppt[s] = std::min(most, ppc >= 8.0 ? 4 : (ppc >= 3.0 ? 2 : 1));
    const int64_t chunk = (int64_t)BLOCK * t.ppt[s];
    t.blk0[s + 1] = t.blk0[s] + (t.n[s] + chunk - 1) / chunk;
  }
  for (int s = c->nspec; s < MAXSP; ++s) t.blk0[s + 1] = t.blk0[c->nspec];
  return t;
}

// records the start event of a timed region; returns its index or -1
int ev_begin(pic_ctx *c, int kind) {
  if (!c->timing) return -1;
  pic_ctx::Ev e{};
  if (hipEventCreate(&e.a) != hipSuccess) return -1;
  if (hipEventCreate(&e.b) != hipSuccess) {
    (void)hipEventDestroy(e.a);
    return -1;
  }
  e.kind = kind;
  (void)hipEventRecord(e.a, c->stream);
  c->events.push_back(e);
  return (int)c->events.size() - 1;
}
void ev_end(pic_ctx *c, int idx) {
  if (idx >= 0) (void)hipEventRecord(c->events[idx].b, c->stream);
}

int32_t *bstart_of(pic_ctx *c, int s, int which) {
  return reinterpret_cast<int32_t *>(c->scratch + c->s_bstart) +
         (int64_t)(2 * s + which) * (c->nbricks + 2);
}
int32_t *err_word(pic_ctx *c) { return reinterpret_cast<int32_t *>(c->scratch + c->s_err); }

// cells a particle can cross in one step of size dt and dimension: below
// dt / dx on a Cartesian grid (|v| < c = 1); at most one on any grid (the
// move clamps its cell step to -1 ... 1)
double step_cells(const pic_ctx *c, double dt) {
  if (c->g.geom == 0) return std::min(1.0, dt * c->max_inv_dx * (1.0 + 1e-6));
  return 1.0;
}

// The brick-neighbour form applies when the present order is that of the
// previous sort (with its brick starts kept) and no particle can have
// crossed more than one brick in any dimension since: a move of at most
// brick_min cells changes the brick index by at most one.  Periodic
// dimensions need at least 3 bricks (so that the neighbours are distinct).
bool brick_sort_ok(const pic_ctx *c) {
  if (!c->bricks_valid || c->perm_pending || c->moved > c->brick_min) return false;
  if (c->g.geom == 0)
    for (int a = 0; a < c->g.dim; ++a)
      if (c->g.nbrick[a] < 3) return false;
  return true;
}

// The stable per-cell sort: the brick-neighbour form when brick_sort_ok,
// else the radix sort.  materialize: reorder every array now (into the other
// set); else the permutation stays pending and the next step reads through
// it while it writes the sorted, advanced particles into the other set (one
// pass over the particle data instead of two).  Either way the brick starts
// of the new order are kept for the next sort.
// tmp: the radix sort's temporaries (keys, values, tile histograms, column
// sums) from elsewhere than the bound scratch buffer (no timing events then).
template <class Real>
pic_status do_sort(pic_ctx *c, bool materialize, const SortScratch *tmp = nullptr) {
  const int ev = tmp ? -1 : ev_begin(c, 1);
  SortScratch S{};
  if (tmp) {
    S = *tmp;
  } else {
    for (int a = 0; a < 2; ++a) {
      S.keys[a] = reinterpret_cast<uint32_t *>(c->scratch + c->s_keys[a]);
      S.vals[a] = reinterpret_cast<int32_t *>(c->scratch + c->s_vals[a]);
    }
    S.hist = reinterpret_cast<int32_t *>(c->scratch + c->s_hist);
    S.bsum = reinterpret_cast<int32_t *>(c->scratch + c->s_bsum);
    S.max_tiles = c->max_tiles;
  }
  int32_t *perm = reinterpret_cast<int32_t *>(c->scratch + c->s_perm);
  PSet<Real> src = pset_of<Real>(c, c->active), dst = pset_of<Real>(c, c->active ^ 1);
  const uint32_t deadkey = 1u << (c->keybits - 1);
  const int localbits = c->g.brick_shift[0] + c->g.brick_shift[1] + c->g.brick_shift[2];
  const bool fast = brick_sort_ok(c);
  for (int s = 0; s < c->nspec; ++s) {
    const int64_t n = (int64_t)c->cnt[s];
    const int64_t o = (int64_t)c->off[s];
    hipError_t e = hipSuccess;
    if (fast) {
      BrickSortArgs a{};
      a.g = c->g;
      a.nb = c->nbricks;
      a.localbits = localbits;
      a.deadkey = deadkey;
      a.n = n;
      a.cell = src.cell + o;
      a.bold = bstart_of(c, s, c->bsel[s]);
      a.bnew = bstart_of(c, s, c->bsel[s] ^ 1);
      a.cnt = reinterpret_cast<int32_t *>(c->scratch + c->s_bcnt);
      a.tot = reinterpret_cast<int32_t *>(c->scratch + c->s_btot);
      a.dpre = reinterpret_cast<int32_t *>(c->scratch + c->s_bdpre);
      a.tkey = S.keys[0];
      a.tval = S.vals[0];
      a.perm = perm + o;
      a.err = err_word(c);
      a.flag = a.err + 1;
      e = launch_brick_sort<Real>(a, src, dst, o, c->o_phi != NONE, materialize, c->stream);
      if (e != hipSuccess) return hipchk(c, e, "brick sort");
      if (n > 0) c->bsel[s] ^= 1;  // an empty species keeps its (empty) starts
      continue;
    }
    if (n > 0) {
      const uint32_t *keys = nullptr;
      e = launch_sort_species(c->g, src.cell + o, n, S, perm + o, c->keybits, c->stream, &keys);
      if (e != hipSuccess) return hipchk(c, e, "sort");
      e = launch_brick_bounds(keys, n, c->nbricks, localbits, deadkey, bstart_of(c, s, c->bsel[s]),
                              c->stream);
      if (e != hipSuccess) return hipchk(c, e, "brick bounds");
      if (materialize) {
        e = launch_gather<Real>(src, dst, c->g.dim, c->o_phi != NONE, o, n, perm + o, c->stream);
        if (e != hipSuccess) return hipchk(c, e, "gather");
      }
    } else {
      e = launch_brick_bounds(nullptr, 0, c->nbricks, localbits, deadkey,
                              bstart_of(c, s, c->bsel[s]), c->stream);
      if (e != hipSuccess) return hipchk(c, e, "brick bounds");
    }
  }
  // species with no particles keep nothing worth copying; flip the set
  if (materialize)
    c->active ^= 1;
  else
    c->perm_pending = true;
  c->bricks_valid = true;
  c->moved = 0.0;
  c->brick_sorts += fast ? 1 : 0;
  ev_end(c, ev);
  return PIC_OK;
}

// apply a pending sort's reorder (after a failed step; entry points that
// touch the particle sets call this first)
template <class Real>
pic_status settle(pic_ctx *c) {
  if (!c->perm_pending) return PIC_OK;
  const int32_t *perm = reinterpret_cast<const int32_t *>(c->scratch + c->s_perm);
  const PSet<Real> src = pset_of<Real>(c, c->active), dst = pset_of<Real>(c, c->active ^ 1);
  for (int s = 0; s < c->nspec; ++s) {
    const int64_t n = (int64_t)c->cnt[s], o = (int64_t)c->off[s];
    hipError_t e = launch_gather<Real>(src, dst, c->g.dim, c->o_phi != NONE, o, n, perm + o,
                                       c->stream);
    if (e != hipSuccess) return hipchk(c, e, "gather");
  }
  c->active ^= 1;
  c->perm_pending = false;
  return PIC_OK;
}

template <class Real>
pic_status do_step(pic_ctx *c, double dt, bool write_prev, bool dep = true) {
  StepArgs<Real> a{};
  a.g = c->g;
  a.sp = push_species_table(c, dt);
  a.p = pset_of<Real>(c, c->active);
  a.perm = nullptr;
  if (c->perm_pending) {  // read through the pending sort, write the other set
    a.perm = reinterpret_cast<const int32_t *>(c->scratch + c->s_perm);
    a.src = a.p;
    a.p = pset_of<Real>(c, c->active ^ 1);
  }
  a.prev_cell = reinterpret_cast<int32_t *>(c->prev + c->p_cell);
  for (int d = 0; d < 3; ++d)
    a.prev_offs[d] = c->p_offs[d] == NONE ? nullptr : reinterpret_cast<OffT<Real> *>(c->prev + c->p_offs[d]);
  a.EB = reinterpret_cast<const Real *>(c->fields);
  a.J = reinterpret_cast<Real *>(c->current);
  a.dt = dt;
  a.dtf = (float)dt;
  a.write_prev = write_prev ? 1 : 0;
  a.deposit = dep ? 1 : 0;
  a.stats = c->timing ? reinterpret_cast<int32_t *>(c->scratch + c->s_stats) : nullptr;
  a.err = err_word(c);
  c->moved += step_cells(c, dt);
  hipError_t e = hipSuccess;
  if (dep) e = launch_zero<Real>(a.J, 3 * c->g.npts, c->stream);
  if (e != hipSuccess) return hipchk(c, e, "zero J");
  const int ev = dep ? ev_begin(c, 0) : -1;
  e = launch_push_deposit<Real>(a, c->stream, c->debug_serial);
  ev_end(c, ev);
  if (e != hipSuccess) return hipchk(c, e, "push_deposit");
  if (a.perm) {
    c->active ^= 1;
    c->perm_pending = false;
  }
  if (dep) e = launch_fold_ghosts<Real>(c->g, a.J, 3, c->stream);
  if (e != hipSuccess) return hipchk(c, e, "fold J");
  return PIC_OK;
}

template <class Real>
pic_status run_steps(pic_ctx *c, double dt, int32_t n, bool allow_sort) {
  for (int32_t s = 0; s < n; ++s) {
    if (allow_sort && c->d.sort_every > 0 && c->step % c->d.sort_every == 0) {
      pic_status st = do_sort<Real>(c, false);
      if (st != PIC_OK) return st;
    }
    pic_status st = do_step<Real>(c, dt, s == n - 1);
    if (st != PIC_OK) return st;
    c->step += 1;
  }
  return PIC_OK;
}

bool isfin(double x) { return std::isfinite(x); }

// ---- adjoint workspace: checkpoints, one segment of stored states, the
// permutations of the sorts inside the run, adjoints and one spare array
struct AdjLayout {
  uint64_t slot, nck, seg, ckpt0, seg0, nperm, perm0, perm_bytes, lam_u, lam_d, tmp, lamJ, total;
};

AdjLayout adj_layout(const pic_ctx *c, int32_t K, int32_t m) {
  AdjLayout L{};
  const uint64_t ab = align_up(c->capacity * c->eb, ALIGN);
  const int32_t S = c->d.sort_every;
  L.slot = align_up(c->ckpt_bytes, ALIGN);
  L.nck = (uint64_t)((K + m - 1) / m);
  L.seg = (uint64_t)std::min(K, m);
  // K consecutive steps hold at most ceil(K / S) multiples of S
  L.nperm = S > 0 ? (uint64_t)((K + S - 1) / S) : 0;
  L.perm_bytes = align_up(c->capacity * 4, ALIGN);
  L.ckpt0 = 0;
  L.seg0 = L.nck * L.slot;
  L.perm0 = L.seg0 + L.seg * L.slot;
  L.lam_u = L.perm0 + L.nperm * L.perm_bytes;
  L.lam_d = L.lam_u + 3 * ab;
  L.tmp = L.lam_d + 3 * ab;
  L.lamJ = L.tmp + ab;
  L.total = L.lamJ + align_up(3ull * c->g.npts * c->eb, ALIGN);
  return L;
}

// a checkpoint slot holds cell, offsets, u (and phi) of the whole capacity
template <class Real>
PSet<Real> slot_pset(const pic_ctx *c, char *slot) {
  const uint64_t ai = align_up(c->capacity * 4, ALIGN), ab = align_up(c->capacity * c->eb, ALIGN);
  PSet<Real> p{};
  uint64_t o = 0;
  p.cell = reinterpret_cast<int32_t *>(slot + o);
  o += ai;
  for (int a = 0; a < 3; ++a) {
    p.offs[a] = nullptr;
    if (a < c->g.dim) {
      p.offs[a] = reinterpret_cast<OffT<Real> *>(slot + o);
      o += ab;
    }
  }
  for (int a = 0; a < 3; ++a) {
    p.u[a] = reinterpret_cast<Real *>(slot + o);
    o += ab;
  }
  p.w = reinterpret_cast<Real *>(slot + o);
  o += ab;
  p.phi = nullptr;
  if (c->g.geom != 0) {
    p.phi = reinterpret_cast<Real *>(slot + o);
    o += ab;
  }
  p.id = reinterpret_cast<int32_t *>(slot + o);
  return p;
}

template <class Real>
hipError_t copy_state(const pic_ctx *c, const PSet<Real> &dst, const PSet<Real> &src) {
  const uint64_t n = c->capacity;
  hipError_t e = hipMemcpyAsync(dst.cell, src.cell, n * 4, hipMemcpyDeviceToDevice, c->stream);
  for (int a = 0; a < c->g.dim && e == hipSuccess; ++a)
    e = hipMemcpyAsync(dst.offs[a], src.offs[a], n * sizeof(OffT<Real>), hipMemcpyDeviceToDevice, c->stream);
  for (int a = 0; a < 3 && e == hipSuccess; ++a)
    e = hipMemcpyAsync(dst.u[a], src.u[a], n * sizeof(Real), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst.w, src.w, n * sizeof(Real), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst.id, src.id, n * 4, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && c->g.geom != 0)
    e = hipMemcpyAsync(dst.phi, src.phi, n * sizeof(Real), hipMemcpyDeviceToDevice, c->stream);
  return e;
}

// The K steps exactly as pic_push_deposit runs them (sorts included); before
// the sort of a step that starts a segment, the state is saved, so that a
// segment's recompute replays the segment's sorts from the stored
// permutations.
template <class Real>
pic_status fwd_ckpt(pic_ctx *c, double dt, int32_t K, int32_t m, char *ws) {
  const AdjLayout L = adj_layout(c, K, m);
  c->ckpt_K = -1;
  c->ckpt_m = m;
  c->ckpt_dt = dt;
  c->ckpt_step0 = c->step;
  c->ckpt_sorts.clear();
  int32_t *perm = reinterpret_cast<int32_t *>(c->scratch + c->s_perm);
  for (int32_t n = 0; n < K; ++n) {
    if (n % m == 0) {
      hipError_t e = copy_state<Real>(c, slot_pset<Real>(c, ws + L.ckpt0 + (n / m) * L.slot),
                                      pset_of<Real>(c, c->active));
      if (e != hipSuccess) return hipchk(c, e, "checkpoint save");
    }
    if (c->d.sort_every > 0 && c->step % c->d.sort_every == 0) {
      if (c->ckpt_sorts.size() >= L.nperm) return fail(c, PIC_E_STATE, "sort count");
      pic_status st = do_sort<Real>(c, false);
      if (st != PIC_OK) return st;
      hipError_t e = hipMemcpyAsync(ws + L.perm0 + c->ckpt_sorts.size() * L.perm_bytes, perm,
                                    c->capacity * 4, hipMemcpyDeviceToDevice, c->stream);
      if (e != hipSuccess) return hipchk(c, e, "store permutation");
      c->ckpt_sorts.push_back(n);
    }
    pic_status st = do_step<Real>(c, dt, n == K - 1, true);
    if (st != PIC_OK) return st;
    c->step += 1;
  }
  c->ckpt_K = K;
  return PIC_OK;
}

// index of the stored permutation of the sort at step n of the run, or -1
int sort_slot(const pic_ctx *c, int32_t n) {
  for (size_t r = 0; r < c->ckpt_sorts.size(); ++r)
    if (c->ckpt_sorts[r] == n) return (int)r;
  return -1;
}

template <class Real>
pic_status bwd(pic_ctx *c, double dt, int32_t K, int32_t m, char *ws, const void *lamJ,
               const void *lam_u, void *dEB, void *du0) {
  const AdjLayout L = adj_layout(c, K, m);
  const GridConst &g = c->g;
  const uint64_t cap = c->capacity;
  const uint64_t ab = align_up(cap * c->eb, ALIGN);
  Real *lu[3], *ld[3];
  for (int a = 0; a < 3; ++a) {
    lu[a] = reinterpret_cast<Real *>(ws + L.lam_u + a * ab);
    ld[a] = reinterpret_cast<Real *>(ws + L.lam_d + a * ab);
  }
  Real *lJ = reinterpret_cast<Real *>(ws + L.lamJ);
  Real *tmp = reinterpret_cast<Real *>(ws + L.tmp);
  Real *dE = static_cast<Real *>(dEB);
  hipError_t e = launch_zero<Real>(dE, 6 * g.npts, c->stream);
  for (int a = 0; a < 3 && e == hipSuccess; ++a) {
    if (lam_u)
      e = hipMemcpyAsync(lu[a], static_cast<const Real *>(lam_u) + a * cap, cap * sizeof(Real),
                         hipMemcpyDeviceToDevice, c->stream);
    else
      e = launch_zero<Real>(lu[a], (int64_t)cap, c->stream);
    if (e == hipSuccess) e = launch_zero<Real>(ld[a], (int64_t)cap, c->stream);
  }
  if (e == hipSuccess && lamJ) {
    // a deposit into a periodic ghost ends up in its image: gather from there
    e = hipMemcpyAsync(lJ, lamJ, 3ull * g.npts * sizeof(Real), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = launch_fill_ghosts<Real>(g, lJ, 3, c->stream);
  }
  if (e != hipSuccess) return hipchk(c, e, "backward setup");
  AdjArgs<Real> A{};
  A.g = g;
  A.sp = species_table(c, dt, adj_chunk(c->eb));
  A.EB = reinterpret_cast<const Real *>(c->fields);
  A.dEB = dE;
  A.dt = dt;
  for (int a = 0; a < 3; ++a) {
    A.lam_u[a] = lu[a];
    A.lam_d[a] = ld[a];
  }
  // axisymmetric grids: the third row of the offset adjoints carries dL/dphi
  A.lam_phi = g.geom != 0 ? ld[2] : nullptr;
  const int64_t saved_step = c->step;
  const bool has_phi = c->o_phi != NONE;
  for (int64_t j = (int64_t)L.nck - 1; j >= 0; --j) {
    const int32_t s0 = (int32_t)(j * m), s1 = std::min(K, s0 + m);
    PSet<Real> cur = pset_of<Real>(c, c->active);
    e = copy_state<Real>(c, cur, slot_pset<Real>(c, ws + L.ckpt0 + j * L.slot));
    if (e != hipSuccess) return hipchk(c, e, "checkpoint load");
    for (int32_t n = s0; n < s1; ++n) {
      const int r = sort_slot(c, n);
      if (r >= 0) {  // replay the step's sort from its stored permutation
        const int32_t *pm = reinterpret_cast<const int32_t *>(ws + L.perm0 + r * L.perm_bytes);
        const PSet<Real> dst = pset_of<Real>(c, c->active ^ 1);
        for (int sp = 0; sp < c->nspec && e == hipSuccess; ++sp)
          e = launch_gather<Real>(cur, dst, g.dim, has_phi, (int64_t)c->off[sp],
                                  (int64_t)c->cnt[sp], pm + c->off[sp], c->stream);
        if (e != hipSuccess) return hipchk(c, e, "sort replay");
        c->active ^= 1;
        cur = dst;
      }
      e = copy_state<Real>(c, slot_pset<Real>(c, ws + L.seg0 + (n - s0) * L.slot), cur);
      if (e != hipSuccess) return hipchk(c, e, "segment store");
      if (n < s1 - 1) {
        pic_status st = do_step<Real>(c, dt, false, false);
        if (st != PIC_OK) return st;
      }
    }
    for (int32_t n = s1 - 1; n >= s0; --n) {
      A.p = slot_pset<Real>(c, ws + L.seg0 + (n - s0) * L.slot);
      A.lamJ = (n == K - 1 && lamJ) ? lJ : nullptr;
      const int ev = ev_begin(c, 2);
      e = launch_adjoint_step<Real>(A, c->stream);
      ev_end(c, ev);
      if (e != hipSuccess) return hipchk(c, e, "adjoint step");
      const int r = sort_slot(c, n);
      if (r >= 0) {  // the adjoints follow their particles back to the order before the sort
        const int32_t *pm = reinterpret_cast<const int32_t *>(ws + L.perm0 + r * L.perm_bytes);
        Real *arr[6] = {lu[0], lu[1], lu[2], ld[0], ld[1], ld[2]};
        const int nadj = g.geom != 0 ? 6 : 3 + g.dim;
        for (int k = 0; k < nadj && e == hipSuccess; ++k) {
          for (int sp = 0; sp < c->nspec && e == hipSuccess; ++sp)
            e = launch_scatter_back<Real>(arr[k], tmp, (int64_t)c->off[sp], (int64_t)c->cnt[sp],
                                          pm + c->off[sp], c->stream);
          if (e == hipSuccess)
            e = hipMemcpyAsync(arr[k], tmp, cap * sizeof(Real), hipMemcpyDeviceToDevice, c->stream);
        }
        if (e != hipSuccess) return hipchk(c, e, "adjoint permutation");
      }
    }
  }
  e = launch_fold_ghosts<Real>(g, dE, 6, c->stream);
  for (int a = 0; a < 3 && e == hipSuccess; ++a)
    e = hipMemcpyAsync(static_cast<Real *>(du0) + a * cap, lu[a], cap * sizeof(Real),
                       hipMemcpyDeviceToDevice, c->stream);
  // leave the particles as they were at step 0 of the checkpointed run
  if (e == hipSuccess)
    e = copy_state<Real>(c, pset_of<Real>(c, c->active), slot_pset<Real>(c, ws + L.ckpt0));
  if (e != hipSuccess) return hipchk(c, e, "backward finish");
  (void)saved_step;
  c->step = c->ckpt_step0;
  return PIC_OK;
}


uint32_t offset_to_fixed(double d) {
  const double r = std::nearbyint(d * 4294967296.0);
  if (r >= 4294967295.0) return 0xffffffffu;
  if (r <= 0.0) return 0u;
  return (uint32_t)r;
}

double cfl_length(const GridConst &g) {
  double best = INFINITY;
  const int nd = g.geom == 0 ? g.dim : 2;
  const int n2 = g.dim >= 2 ? g.n[1] : 1;
  const int n3 = g.dim >= 3 ? g.n[2] : 1;
  // Sec. 2.4: minimum over cell centres of (sum_i 1/h_ii)^(-1/2)
  for (int k = 0; k < n3; ++k)
    for (int j = 0; j < n2; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        double h[3];
        h_sqrt_h(g, i + 0.5, j + 0.5, h);
        double s = 0;
        for (int a = 0; a < nd; ++a) s += 1.0 / (h[a] * h[a]);
        best = std::min(best, 1.0 / std::sqrt(s));
        if (g.geom == 0) return best;  // uniform cells
      }
  return best;
}

}  // namespace


template <class Real>
pic_status adjoint_one(pic_ctx *c, double dt, const void *lamJ, const pic_adjoint_buffers *io) {
  const GridConst &g = c->g;
  const uint64_t cap = c->capacity;
  AdjArgs<Real> A{};
  A.g = g;
  A.sp = species_table(c, dt, adj_chunk(c->eb));
  A.p = pset_of<Real>(c, c->active);
  A.EB = reinterpret_cast<const Real *>(c->fields);
  A.dEB = static_cast<Real *>(io->dEB);
  A.dt = dt;
  for (int a = 0; a < 3; ++a) {
    A.lam_u[a] = static_cast<Real *>(io->lam_u) + a * cap;
    A.lam_d[a] = static_cast<Real *>(io->lam_offs) + a * cap;
  }
  A.lam_phi = g.geom != 0 ? A.lam_d[2] : nullptr;
  A.lamJ = nullptr;
  hipError_t e = hipSuccess;
  if (lamJ) {  // a deposit into a periodic ghost ends up in its image: gather from there
    Real *w = static_cast<Real *>(io->lamJ_work);
    e = hipMemcpyAsync(w, lamJ, 3ull * g.npts * sizeof(Real), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = launch_fill_ghosts<Real>(g, w, 3, c->stream);
    A.lamJ = w;
  }
  if (e == hipSuccess) {
    const int ev = ev_begin(c, 2);
    e = launch_adjoint_step<Real>(A, c->stream);
    ev_end(c, ev);
  }
  if (e == hipSuccess) e = launch_fold_ghosts<Real>(g, A.dEB, 6, c->stream);
  return hipchk(c, e, "adjoint_step");
}

extern "C" {

pic_status pic_grid_init(const pic_grid_desc *desc, pic_ctx **out) {
  if (!desc || !out) return PIC_E_ARG;
  const pic_grid_desc &d = *desc;
  if (d.geom < 0 || d.geom > 2) return PIC_E_ARG;
  if (d.geom == PIC_CART && d.dim != 2 && d.dim != 3) return PIC_E_ARG;
  if (d.geom != PIC_CART && d.dim != 2) return PIC_E_ARG;
  if (d.prec != PIC_F32 && d.prec != PIC_F64) return PIC_E_ARG;
  for (int a = 0; a < d.dim; ++a)
    if (d.n[a] < 1 || d.n[a] > (1 << 20)) return PIC_E_ARG;
  if (!(d.rho0 > 0) || !isfin(d.rho0)) return PIC_E_ARG;
  if (d.sort_every < 0 || d.fp64_axis_cells < 0) return PIC_E_ARG;
  if (d.max_particles == 0 || d.max_particles > (1ull << 31) - (1ull << 20)) return PIC_E_ARG;
  if (d.geom == PIC_CART) {
    for (int a = 0; a < d.dim; ++a) {
      if (!(d.hi[a] > d.lo[a]) || !isfin(d.hi[a]) || !isfin(d.lo[a])) return PIC_E_ARG;
      if (!d.periodic[a]) return PIC_E_UNSUPPORTED;
    }
  } else {
    if (!(d.lo[0] > 0) || !(d.hi[0] > d.lo[0]) || !isfin(d.hi[0])) return PIC_E_ARG;
    if (d.geom == PIC_QSPH) {
      if (!(d.vartheta > -0.5 && d.vartheta < 1.0)) return PIC_E_ARG;
      if (!(d.lo[0] - d.r0 > 0) || !isfin(d.r0)) return PIC_E_ARG;
    }
    if (d.n[1] < 2) return PIC_E_ARG;
  }
  pic_ctx *c = new pic_ctx();
  c->d = d;
  GridConst &g = c->g;
  g.geom = d.geom;
  g.dim = d.dim;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = a < d.dim ? d.n[a] : 1;
    g.np[a] = a < d.dim ? d.n[a] + 2 * NG : 1;
    g.dx[a] = (d.geom == PIC_CART && a < d.dim) ? (d.hi[a] - d.lo[a]) / d.n[a] : 1.0;
    g.inv_dx[a] = 1.0 / g.dx[a];
    g.dxf[a] = (float)g.dx[a];
    g.inv_dxf[a] = (float)g.inv_dx[a];
  }
  g.npts = (int64_t)g.np[0] * g.np[1] * g.np[2];
  if (6 * g.npts >= (int64_t(1) << 31)) {  // device index math is 32-bit
    delete c;
    return PIC_E_UNSUPPORTED;
  }
  g.rmin = d.lo[0];
  g.dr = (d.geom != PIC_CART) ? (d.hi[0] - d.lo[0]) / d.n[0] : 0.0;
  g.dth = (d.geom != PIC_CART) ? PI / d.n[1] : 0.0;
  if (d.geom == PIC_QSPH) {
    g.Rmin = std::log(d.lo[0] - d.r0);
    g.dR = (std::log(d.hi[0] - d.r0) - g.Rmin) / d.n[0];
    g.dT = PI / d.n[1];
    g.r0 = d.r0;
    g.vt = d.vartheta;
  }
  g.fp64_cells = d.fp64_axis_cells;
  // cell packing: (i1 + 1) needs values 0..N1+1, then i2, i3
  const int b1 = bits_for((int64_t)g.n[0] + 2);
  const int b2 = d.dim >= 2 ? bits_for(g.n[1]) : 0;
  const int b3 = d.dim >= 3 ? bits_for(g.n[2]) : 0;
  if (b1 + b2 + b3 > 30) {
    delete c;
    return PIC_E_UNSUPPORTED;
  }
  g.shift2 = b1;
  g.shift3 = b1 + b2;
  g.mask1 = (1 << b1) - 1;
  g.mask2 = (1 << b2) - 1;
  g.mask3 = (1 << b3) - 1;
  // sort order: 4x4x4 bricks in 3D, 8x8 in 2D
  for (int a = 0; a < 3; ++a) {
    g.brick[a] = a < d.dim ? (d.dim == 3 ? 4 : 8) : 1;
    g.brick_shift[a] = a < d.dim ? (d.dim == 3 ? 2 : 3) : 0;
    g.nbrick[a] = (g.n[a] + g.brick[a] - 1) / g.brick[a];
  }
  const int64_t nkeys = (int64_t)g.nbrick[0] * g.nbrick[1] * g.nbrick[2] *
                        g.brick[0] * g.brick[1] * g.brick[2];
  c->nbricks = g.nbrick[0] * g.nbrick[1] * g.nbrick[2];
  c->brick_min = g.brick[0];
  for (int a = 1; a < d.dim; ++a) c->brick_min = std::min(c->brick_min, g.brick[a]);
  for (int a = 0; a < d.dim; ++a) c->max_inv_dx = std::max(c->max_inv_dx, g.inv_dx[a]);
  if (bits_for(nkeys) > 30) {
    delete c;
    return PIC_E_UNSUPPORTED;
  }
  c->keybits = bits_for(nkeys) + 1;
  c->eb = d.prec == PIC_F64 ? 8 : 4;
  // capacity: room for per-species alignment to 64 elements
  c->capacity = align_up(d.max_particles, 64) + 64 * MAXSP;
  const uint64_t cap = c->capacity;
  const uint64_t ab = align_up(cap * c->eb, ALIGN), ai = align_up(cap * 4, ALIGN);
  uint64_t o = 0;
  c->o_cell = o;
  o += ai;
  for (int a = 0; a < d.dim; ++a) {
    c->o_offs[a] = o;
    o += ab;
  }
  for (int a = 0; a < 3; ++a) {
    c->o_u[a] = o;
    o += ab;
  }
  c->o_w = o;
  o += ab;
  if (d.geom != PIC_CART) {
    c->o_phi = o;
    o += ab;
  }
  c->o_id = o;
  o += ai;
  c->set_bytes = o;
  o = 0;
  c->p_cell = o;
  o += ai;
  for (int a = 0; a < d.dim; ++a) {
    c->p_offs[a] = o;
    o += ab;
  }
  c->prev_bytes = o;
  c->max_tiles = (int64_t)((cap + SORT_TILE - 1) / SORT_TILE);
  o = 0;
  for (int a = 0; a < 2; ++a) {
    c->s_keys[a] = o;
    o += ai;
    c->s_vals[a] = o;
    o += ai;
  }
  c->s_hist = o;
  o += align_up((uint64_t)256 * c->max_tiles * 4, ALIGN);
  c->s_bsum = o;
  o += align_up((uint64_t)SCAN_CHUNKS * 256 * 4, ALIGN);
  c->s_perm = o;
  o += ai;
  c->s_stats = o;
  o += ALIGN;
  // brick-neighbour sort: two brick-start arrays per species, the counts per
  // (old brick, destination), the new bricks' totals, the dead prefixes
  const uint64_t nbk = (uint64_t)c->nbricks;
  const uint64_t ndest = (d.dim == 3 ? 27 : 9) + 1;
  c->s_bstart = o;
  o += align_up(2ull * MAXSP * (nbk + 2) * 4, ALIGN);
  c->s_bcnt = o;
  o += align_up((nbk + 1) * ndest * 4, ALIGN);
  c->s_btot = o;
  o += align_up((nbk + 1) * 4, ALIGN);
  c->s_bdpre = o;
  o += align_up((nbk + 1) * 4, ALIGN);
  c->s_err = o;  // [0] device error word, [1] the brick sort's flag
  o += ALIGN;
  c->scratch_bytes = o;
  // checkpoint: cell, offsets, u, w, phi, id
  c->ckpt_bytes = 2 * ai + (uint64_t)d.dim * ab + 4 * ab + (d.geom != PIC_CART ? ab : 0);
  c->dx_min = cfl_length(g);
  *out = c;
  return PIC_OK;
}

void pic_grid_destroy(pic_ctx *ctx) { delete ctx; }

pic_status pic_query_sizes(const pic_ctx *c, pic_sizes *out) {
  if (!c || !out) return PIC_E_ARG;
  out->fields_bytes = 6ull * c->g.npts * c->eb;
  out->current_bytes = 3ull * c->g.npts * c->eb;
  out->particle_set_bytes = c->set_bytes;
  out->prev_bytes = c->prev_bytes;
  out->scratch_bytes = c->scratch_bytes;
  out->checkpoint_bytes = c->ckpt_bytes;
  out->field_points = (uint64_t)c->g.npts;
  for (int a = 0; a < 3; ++a) out->np[a] = c->g.np[a];
  out->elem_bytes = (int32_t)c->eb;
  return PIC_OK;
}

pic_status pic_bind_buffers(pic_ctx *c, const pic_buffers *b) {
  if (!c || !b) return PIC_E_ARG;
  if (!b->fields || !b->current || !b->particles[0] || !b->particles[1] || !b->prev ||
      !b->scratch)
    return fail(c, PIC_E_ARG, "bind: null buffer");
  for (const void *p : {b->fields, b->current, b->particles[0], b->particles[1], b->prev,
                        b->scratch})
    if (reinterpret_cast<uintptr_t>(p) % 256 != 0)
      return fail(c, PIC_E_ARG, "bind: buffers must be 256-byte aligned");
  c->fields = static_cast<char *>(b->fields);
  c->current = static_cast<char *>(b->current);
  c->pset[0] = static_cast<char *>(b->particles[0]);
  c->pset[1] = static_cast<char *>(b->particles[1]);
  c->prev = static_cast<char *>(b->prev);
  c->scratch = static_cast<char *>(b->scratch);
  c->bound = true;
  c->active = 0;
  hipError_t e = hipMemsetAsync(c->prev, 0, c->prev_bytes, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->current, 0, 3ull * c->g.npts * c->eb, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->scratch + c->s_perm, 0, c->capacity * 4, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->scratch + c->s_err, 0, ALIGN, c->stream);
  c->bricks_valid = false;
  return hipchk(c, e, "bind: clear");
}

pic_status pic_set_stream(pic_ctx *c, void *s) {
  if (!c) return PIC_E_ARG;
  c->stream = static_cast<hipStream_t>(s);
  return PIC_OK;
}

pic_status pic_timestep_from_cfl(const pic_ctx *c, double cfl, double *dt) {
  if (!c || !dt || !(cfl > 0) || !isfin(cfl)) return PIC_E_ARG;
  *dt = cfl * c->dx_min;
  return PIC_OK;
}


pic_status pic_species_add(pic_ctx *c, double charge, double mass, uint64_t capacity,
                           int32_t *species_id) {
  if (!c || !species_id) return PIC_E_ARG;
  if (c->loaded) return fail(c, PIC_E_STATE, "species_add after particles_load");
  if (c->nspec >= MAXSP) return fail(c, PIC_E_CAPACITY, "at most %d species", MAXSP);
  if (!isfin(charge) || !(mass > 0) || !isfin(mass))
    return fail(c, PIC_E_ARG, "species: bad charge/mass");
  const uint64_t start = c->nspec ? align_up(c->off[c->nspec - 1] + c->cap[c->nspec - 1], 64) : 0;
  uint64_t used = 0;
  for (int s = 0; s < c->nspec; ++s) used += c->cap[s];
  if (used + capacity > c->d.max_particles || start + capacity > c->capacity)
    return fail(c, PIC_E_CAPACITY, "species capacity exceeds max_particles");
  const int s = c->nspec++;
  c->q[s] = charge;
  c->m[s] = mass;
  c->cap[s] = capacity;
  c->off[s] = start;
  c->cnt[s] = 0;
  *species_id = s;
  return PIC_OK;
}

pic_status pic_species_set_pusher(pic_ctx *c, int32_t species, int32_t pusher, double e_ovr,
                                  double larmor_max) {
  if (!c) return PIC_E_ARG;
  if (species < 0 || species >= c->nspec) return fail(c, PIC_E_ARG, "no species %d", species);
  if (pusher < 0 || pusher > (PIC_PUSH_VAY | PIC_PUSH_GCA))
    return fail(c, PIC_E_ARG, "unknown pusher %d", pusher);
  if (pusher & PIC_PUSH_GCA) {
    if (!(e_ovr > 0.0 && e_ovr < 1.0))
      return fail(c, PIC_E_ARG, "guiding-centre hybrid: e_ovr %g outside (0, 1)", e_ovr);
    if (!(larmor_max > 0.0) || !isfin(larmor_max))
      return fail(c, PIC_E_ARG, "guiding-centre hybrid: bad critical gyroradius %g", larmor_max);
  }
  c->pusher[species] = pusher;
  c->gca_e_ovr[species] = (pusher & PIC_PUSH_GCA) ? e_ovr : 0.0;
  c->gca_larmor[species] = (pusher & PIC_PUSH_GCA) ? larmor_max : 0.0;
  return PIC_OK;
}

// the hand-written reverse step differentiates the Boris push
static pic_status adjoint_pushers_ok(pic_ctx *c) {
  for (int s = 0; s < c->nspec; ++s)
    if (c->pusher[s] != PIC_PUSH_BORIS)
      return fail(c, PIC_E_UNSUPPORTED, "adjoint: species %d does not use the Boris pusher", s);
  return PIC_OK;
}

pic_status pic_fields_set(pic_ctx *c, const double *EB, int32_t basis, int32_t includes_ghosts) {
  if (!c || !EB) return PIC_E_ARG;
  if (!c->bound) return fail(c, PIC_E_STATE, "fields_set before bind_buffers");
  if (basis != PIC_BASIS_CONTRAVARIANT && basis != PIC_BASIS_TETRAD)
    return fail(c, PIC_E_ARG, "bad basis");
  const GridConst &g = c->g;
  if (g.geom != 0 && !includes_ghosts)
    return fail(c, PIC_E_ARG, "curvilinear fields need the padded array (includes_ghosts=1)");
  std::vector<double> F(6 * g.npts, 0.0);
  const int k0 = g.dim == 3 ? -NG : 0, k1 = g.dim == 3 ? g.n[2] + NG : 1;
  const int64_t nact = (int64_t)g.n[0] * g.n[1] * g.n[2];
  for (int cc = 0; cc < 6; ++cc)
    for (int k = k0; k < k1; ++k)
      for (int j = -NG; j < g.n[1] + NG; ++j)
        for (int i = -NG; i < g.n[0] + NG; ++i) {
          const int64_t pi = (int64_t)cc * g.npts + (i + NG) +
                             (int64_t)g.np[0] * ((j + NG) + (int64_t)g.np[1] * (g.dim == 3 ? k + NG : 0));
          double v;
          if (includes_ghosts) {
            v = EB[pi];
          } else {
            const bool act = i >= 0 && i < g.n[0] && j >= 0 && j < g.n[1] &&
                             (g.dim < 3 || (k >= 0 && k < g.n[2]));
            if (!act) continue;
            v = EB[(int64_t)cc * nact + i + (int64_t)g.n[0] * (j + (int64_t)g.n[1] * (g.dim == 3 ? k : 0))];
          }
          if (!isfin(v)) return fail(c, PIC_E_RANGE, "non-finite field value");
          if (basis == PIC_BASIS_TETRAD) {
            const bool axis = g.geom != 0 && (cc == 2 || cc == 4) && (j == 0 || j == g.n[1]);
            if (axis) {
              v = 0.0;
            } else {
              double h[3];
              h_sqrt_h(g, i + STAG[cc][0], j + STAG[cc][1], h);
              v = v / h[cc % 3];
            }
          } else if (g.geom != 0 && (cc == 2 || cc == 4) && (j == 0 || j == g.n[1])) {
            v = 0.0;  // axis rule of Sec. 2.6
          }
          F[pi] = v;
        }
  hipError_t e;
  if (c->eb == 8) {
    e = hipMemcpyAsync(c->fields, F.data(), F.size() * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_fill_ghosts<double>(g, reinterpret_cast<double *>(c->fields), 6, c->stream);
  } else {
    std::vector<float> f(F.size());
    for (size_t q = 0; q < F.size(); ++q) f[q] = (float)F[q];
    e = hipMemcpyAsync(c->fields, f.data(), f.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_fill_ghosts<float>(g, reinterpret_cast<float *>(c->fields), 6, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hipchk(c, e, "fields_set");
  c->fields_ok = true;
  return PIC_OK;
}

pic_status pic_fields_fill_ghosts(pic_ctx *c) {
  if (!c) return PIC_E_ARG;
  if (!c->bound) return fail(c, PIC_E_STATE, "not bound");
  hipError_t e = c->eb == 8
                     ? launch_fill_ghosts<double>(c->g, reinterpret_cast<double *>(c->fields), 6, c->stream)
                     : launch_fill_ghosts<float>(c->g, reinterpret_cast<float *>(c->fields), 6, c->stream);
  c->fields_ok = true;
  return hipchk(c, e, "fill_ghosts");
}

pic_status pic_particles_load(pic_ctx *c, int32_t s, uint64_t n, const int32_t *cell,
                              const double *offs, const double *u, const double *w,
                              const double *phi) {
  if (!c) return PIC_E_ARG;
  if (!c->bound) return fail(c, PIC_E_STATE, "particles_load before bind_buffers");
  if (s < 0 || s >= c->nspec) return fail(c, PIC_E_ARG, "bad species %d", s);
  if (n > c->cap[s]) return fail(c, PIC_E_CAPACITY, "%llu particles exceed species capacity %llu",
                                 (unsigned long long)n, (unsigned long long)c->cap[s]);
  if (n > 0 && (!cell || !offs || !u || !w)) return fail(c, PIC_E_ARG, "null particle array");
  {
    const pic_status st = c->eb == 8 ? settle<double>(c) : settle<float>(c);
    if (st != PIC_OK) return st;
  }
  const GridConst &g = c->g;
  const bool axi = g.geom != 0;
  if (n > 0 && axi && !phi) return fail(c, PIC_E_ARG, "phi required on (quasi-)spherical grids");
  const int D = g.dim;
  std::vector<int32_t> hc(n);
  for (uint64_t p = 0; p < n; ++p) {
    int ii[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
      ii[a] = cell[p * D + a];
      if (ii[a] < 0 || ii[a] >= g.n[a])
        return fail(c, PIC_E_RANGE, "particle %llu: cell index %d out of range in dim %d",
                    (unsigned long long)p, ii[a], a);
      const double o = offs[p * D + a];
      if (!(o >= 0.0 && o < 1.0))
        return fail(c, PIC_E_RANGE, "particle %llu: offset %g outside [0,1)", (unsigned long long)p, o);
    }
    for (int a = 0; a < 3; ++a)
      if (!isfin(u[p * 3 + a])) return fail(c, PIC_E_RANGE, "particle %llu: non-finite u", (unsigned long long)p);
    if (!isfin(w[p])) return fail(c, PIC_E_RANGE, "particle %llu: non-finite weight", (unsigned long long)p);
    if (axi && !(phi[p] >= 0.0 && phi[p] < 2 * PI))
      return fail(c, PIC_E_RANGE, "particle %llu: phi outside [0, 2pi)", (unsigned long long)p);
    hc[p] = (ii[0] + 1) | (ii[1] << g.shift2) | (ii[2] << g.shift3);
  }
  char *base = c->pset[c->active];
  const uint64_t o = c->off[s];
  hipError_t e = hipMemcpyAsync(base + c->o_cell + o * 4, hc.data(), n * 4, hipMemcpyHostToDevice, c->stream);
  auto put = [&](uint64_t boff, const double *src, int stride, int comp) -> hipError_t {
    if (c->eb == 8) {
      std::vector<double> t(n);
      for (uint64_t p = 0; p < n; ++p) t[p] = src[p * stride + comp];
      hipError_t r = hipMemcpyAsync(base + boff + o * 8, t.data(), n * 8, hipMemcpyHostToDevice, c->stream);
      if (r == hipSuccess) r = hipStreamSynchronize(c->stream);
      return r;
    }
    std::vector<float> t(n);
    for (uint64_t p = 0; p < n; ++p) {
      float v = (float)src[p * stride + comp];
      t[p] = v;
    }
    hipError_t r = hipMemcpyAsync(base + boff + o * 4, t.data(), n * 4, hipMemcpyHostToDevice, c->stream);
    if (r == hipSuccess) r = hipStreamSynchronize(c->stream);
    return r;
  };
  if (n > 0) {
    for (int a = 0; a < D && e == hipSuccess; ++a) {
      if (c->eb == 8) {
        e = put(c->o_offs[a], offs, D, a);
      } else {
        // FP32 build: 32-bit fixed point, nearest multiple of 2^-32 below 1
        std::vector<uint32_t> t(n);
        for (uint64_t p = 0; p < n; ++p) t[p] = offset_to_fixed(offs[p * D + a]);
        e = hipMemcpyAsync(base + c->o_offs[a] + o * 4, t.data(), n * 4, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      }
    }
    for (int a = 0; a < 3 && e == hipSuccess; ++a) e = put(c->o_u[a], u, 3, a);
    if (e == hipSuccess) e = put(c->o_w, w, 1, 0);
    if (e == hipSuccess && axi) e = put(c->o_phi, phi, 1, 0);
    if (e == hipSuccess) {
      std::vector<int32_t> ids(n);
      for (uint64_t p = 0; p < n; ++p) ids[p] = (int32_t)p;
      e = hipMemcpyAsync(base + c->o_id + o * 4, ids.data(), n * 4, hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hipchk(c, e, "particles_load");
  c->cnt[s] = n;
  c->loaded = true;
  c->bricks_valid = false;
  return PIC_OK;
}

pic_status pic_sort(pic_ctx *c) {
  if (!c) return PIC_E_ARG;
  if (!c->bound) return fail(c, PIC_E_STATE, "sort before bind_buffers");
  pic_status st = c->eb == 8 ? settle<double>(c) : settle<float>(c);
  if (st != PIC_OK) return st;
  return c->eb == 8 ? do_sort<double>(c, true) : do_sort<float>(c, true);
}

// ---- the allocation-free sort: the radix temporaries live in a static
// device array (one per GPU, held until the process ends) instead of the
// caller's scratch buffer.
namespace {
constexpr int64_t STATIC_SORT_MAX = int64_t(1) << 22;  // particles per species
constexpr int64_t STATIC_SORT_TILES = STATIC_SORT_MAX / SORT_TILE;
constexpr uint64_t SS_ARRAY = (uint64_t)STATIC_SORT_MAX * 4;  // one key or value array
constexpr uint64_t SS_HIST = (uint64_t)STATIC_SORT_TILES * 256 * 4;
constexpr uint64_t SS_BSUM = (uint64_t)SCAN_CHUNKS * 256 * 4;
constexpr uint64_t SS_BYTES = 4 * SS_ARRAY + SS_HIST + SS_BSUM;
static_assert(SS_ARRAY % ALIGN == 0 && SS_HIST % ALIGN == 0, "static scratch alignment");
constexpr int SS_MAX_DEVICES = 64;
std::mutex ss_mutex;
char *ss_ptr[SS_MAX_DEVICES] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[SS_BYTES];

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (the array's host-side name is not a device
// address and is never passed to a kernel or copy).
static pic_status static_scratch(pic_ctx *c, char **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hipchk(c, e, "hipGetDevice");
  if (dev < 0 || dev >= SS_MAX_DEVICES) return fail(c, PIC_E_UNSUPPORTED, "device %d", dev);
  std::lock_guard<std::mutex> lock(ss_mutex);
  if (!ss_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hipchk(c, e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(c, PIC_E_HIP, "hipGetSymbolAddress(scratch) returned null");
    ss_ptr[dev] = static_cast<char *>(p);
  }
  *out = ss_ptr[dev];
  return PIC_OK;
}

pic_status pic_sort_static(pic_ctx *c) {
  if (!c) return PIC_E_ARG;
  if (!c->bound) return fail(c, PIC_E_STATE, "sort before bind_buffers");
  for (int s = 0; s < c->nspec; ++s)
    if ((int64_t)c->cnt[s] > STATIC_SORT_MAX)
      return fail(c, PIC_E_CAPACITY,
                  "species %d holds %llu particles; the allocation-free sort takes at most %lld "
                  "per species (use pic_sort)",
                  s, (unsigned long long)c->cnt[s], (long long)STATIC_SORT_MAX);
  char *base = nullptr;
  pic_status st = static_scratch(c, &base);
  if (st != PIC_OK) return st;
  SortScratch S{};
  S.keys[0] = reinterpret_cast<uint32_t *>(base);
  S.vals[0] = reinterpret_cast<int32_t *>(base + SS_ARRAY);
  S.keys[1] = reinterpret_cast<uint32_t *>(base + 2 * SS_ARRAY);
  S.vals[1] = reinterpret_cast<int32_t *>(base + 3 * SS_ARRAY);
  S.hist = reinterpret_cast<int32_t *>(base + 4 * SS_ARRAY);
  S.bsum = reinterpret_cast<int32_t *>(base + 4 * SS_ARRAY + SS_HIST);
  S.max_tiles = STATIC_SORT_TILES;
  st = c->eb == 8 ? settle<double>(c) : settle<float>(c);
  if (st != PIC_OK) return st;
  return c->eb == 8 ? do_sort<double>(c, true, &S) : do_sort<float>(c, true, &S);
}

pic_status pic_push_deposit(pic_ctx *c, double dt, int32_t n_steps) {
  if (!c) return PIC_E_ARG;
  if (!c->bound || !c->fields_ok) return fail(c, PIC_E_STATE, "push before bind/fields_set");
  if (!(dt > 0) || !isfin(dt) || n_steps < 0) return fail(c, PIC_E_ARG, "bad dt or n_steps");
  if (dt > c->dx_min)
    return fail(c, PIC_E_ARG, "dt %g exceeds the CFL limit %g (Courant number 1)", dt, c->dx_min);
  const pic_status st = c->eb == 8 ? settle<double>(c) : settle<float>(c);
  if (st != PIC_OK) return st;
  return c->eb == 8 ? run_steps<double>(c, dt, n_steps, true) : run_steps<float>(c, dt, n_steps, true);
}

}  // extern "C"

// ---- field solver and the full loop (Sec. 2.3 steps 2, 9-11; App. A; Sec. 2.5, 2.6)
namespace {
template <class Real>
pic_status advance_b(pic_ctx *c, double f) {
  return hipchk(c, launch_faraday<Real>(c->g, reinterpret_cast<Real *>(c->fields), f, c->stream),
                "faraday");
}
template <class Real>
pic_status advance_e(pic_ctx *c, double dt, double coupling) {
  return hipchk(c,
                launch_ampere<Real>(c->g, reinterpret_cast<Real *>(c->fields),
                                    reinterpret_cast<const Real *>(c->current), dt, coupling,
                                    c->stream),
                "ampere");
}
// passes of the filter, ping-ponging between the current and `work`; an odd
// count ends with a copy back
template <class Real>
pic_status filter_current(pic_ctx *c, int32_t passes, void *work) {
  Real *J = reinterpret_cast<Real *>(c->current), *W = static_cast<Real *>(work);
  hipError_t e = hipSuccess;
  for (int32_t p = 0; p < passes && e == hipSuccess; ++p) {
    e = launch_filter<Real>(c->g, J, W, c->stream);
    std::swap(J, W);
  }
  if (e == hipSuccess && (passes & 1))
    e = hipMemcpyAsync(c->current, J, 3ull * c->g.npts * sizeof(Real), hipMemcpyDeviceToDevice,
                       c->stream);
  return hipchk(c, e, "filter");
}
template <class Real>
pic_status full_steps(pic_ctx *c, double dt, int32_t n, int32_t passes, double coupling,
                      void *work) {
  for (int32_t s = 0; s < n; ++s) {
    pic_status st = advance_b<Real>(c, 0.5 * dt);
    if (st == PIC_OK) st = run_steps<Real>(c, dt, 1, true);
    if (st == PIC_OK && passes > 0) st = filter_current<Real>(c, passes, work);
    if (st == PIC_OK) st = advance_b<Real>(c, 0.5 * dt);
    if (st == PIC_OK) st = advance_e<Real>(c, dt, coupling);
    if (st != PIC_OK) return st;
  }
  return PIC_OK;
}
bool field_dt_ok(pic_ctx *c, double dt) {
  return dt > 0 && isfin(dt) && dt <= c->dx_min;
}
}  // namespace

extern "C" {

pic_status pic_fields_advance_b(pic_ctx *c, double f) {
  if (!c) return PIC_E_ARG;
  if (!c->bound || !c->fields_ok) return fail(c, PIC_E_STATE, "faraday before bind/fields_set");
  if (!isfin(f) || std::fabs(f) > c->dx_min) return fail(c, PIC_E_ARG, "bad faraday step %g", f);
  return c->eb == 8 ? advance_b<double>(c, f) : advance_b<float>(c, f);
}

pic_status pic_fields_advance_e(pic_ctx *c, double dt, double coupling) {
  if (!c) return PIC_E_ARG;
  if (!c->bound || !c->fields_ok) return fail(c, PIC_E_STATE, "ampere before bind/fields_set");
  if (!field_dt_ok(c, dt) || !isfin(coupling)) return fail(c, PIC_E_ARG, "bad dt or coupling");
  return c->eb == 8 ? advance_e<double>(c, dt, coupling) : advance_e<float>(c, dt, coupling);
}

pic_status pic_current_filter(pic_ctx *c, int32_t passes, void *work) {
  if (!c || passes < 0 || (passes > 0 && !work)) return PIC_E_ARG;
  if (!c->bound) return fail(c, PIC_E_STATE, "filter before bind_buffers");
  return c->eb == 8 ? filter_current<double>(c, passes, work)
                    : filter_current<float>(c, passes, work);
}

pic_status pic_step_full(pic_ctx *c, double dt, int32_t n_steps, int32_t filter_passes,
                         double coupling, void *work) {
  if (!c || n_steps < 0 || filter_passes < 0 || (filter_passes > 0 && !work)) return PIC_E_ARG;
  if (!c->bound || !c->fields_ok) return fail(c, PIC_E_STATE, "step before bind/fields_set");
  if (!field_dt_ok(c, dt) || !isfin(coupling)) return fail(c, PIC_E_ARG, "bad dt or coupling");
  const pic_status st = c->eb == 8 ? settle<double>(c) : settle<float>(c);
  if (st != PIC_OK) return st;
  return c->eb == 8 ? full_steps<double>(c, dt, n_steps, filter_passes, coupling, work)
                    : full_steps<float>(c, dt, n_steps, filter_passes, coupling, work);
}

pic_status pic_current_get(const pic_ctx *c, void *dst, int32_t dst_is_device) {
  if (!c || !dst) return PIC_E_ARG;
  if (!c->bound) return fail(c, PIC_E_STATE, "not bound");
  const size_t nb = 3ull * c->g.npts * c->eb;
  hipError_t e = hipMemcpyAsync(dst, c->current, nb, dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && !dst_is_device) e = hipStreamSynchronize(c->stream);
  return hipchk(c, e, "current_get");
}

pic_status pic_fields_get(const pic_ctx *c, void *dst, int32_t dst_is_device) {
  if (!c || !dst) return PIC_E_ARG;
  if (!c->bound) return fail(c, PIC_E_STATE, "not bound");
  const size_t nb = 6ull * c->g.npts * c->eb;
  hipError_t e = hipMemcpyAsync(dst, c->fields, nb, dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && !dst_is_device) e = hipStreamSynchronize(c->stream);
  return hipchk(c, e, "fields_get");
}

pic_status pic_particles_get(const pic_ctx *c, int32_t s, pic_particle_view *v) {
  if (!c || !v) return PIC_E_ARG;
  if (!c->bound) return fail(c, PIC_E_STATE, "not bound");
  if (s < 0 || s >= c->nspec) return fail(c, PIC_E_ARG, "bad species %d", s);
  if (c->perm_pending)
    return fail(c, PIC_E_STATE, "a failed step left a sort unapplied: call pic_sort or push again");
  const uint64_t n = c->cnt[s];
  if (v->n < n) return fail(c, PIC_E_CAPACITY, "view holds %llu < %llu particles",
                           (unsigned long long)v->n, (unsigned long long)n);
  v->n = n;
  if (n == 0) return PIC_OK;
  const GridConst &g = c->g;
  const int D = g.dim;
  const uint64_t o = c->off[s];
  const char *base = c->pset[c->active];
  std::vector<int32_t> ci(n);
  std::vector<char> tmp(n * 8);
  hipError_t e = hipMemcpyAsync(ci.data(), base + c->o_cell + o * 4, n * 4, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  auto unpack = [&](const std::vector<int32_t> &cc, int32_t *dst, int32_t *alive) {
    for (uint64_t p = 0; p < n; ++p) {
      const int32_t x = cc[p];
      if (dst) {
        dst[3 * p] = (x & g.mask1) - 1;
        dst[3 * p + 1] = D >= 2 ? (x >> g.shift2) & g.mask2 : 0;
        dst[3 * p + 2] = D >= 3 ? (x >> g.shift3) & g.mask3 : 0;
      }
      if (alive) alive[p] = (x & DEAD_BIT) ? 0 : 1;
    }
  };
  unpack(ci, v->cell, v->alive);
  auto getx = [&](const char *src, double *dst, int stride, int comp, bool is_offset) -> hipError_t {
    hipError_t r = hipMemcpyAsync(tmp.data(), src + o * c->eb, n * c->eb, hipMemcpyDeviceToHost, c->stream);
    if (r == hipSuccess) r = hipStreamSynchronize(c->stream);
    if (r != hipSuccess) return r;
    for (uint64_t p = 0; p < n; ++p) {
      double v;
      if (c->eb == 8)
        v = reinterpret_cast<const double *>(tmp.data())[p];
      else if (is_offset)
        v = (double)reinterpret_cast<const uint32_t *>(tmp.data())[p] * 0x1p-32;
      else
        v = (double)reinterpret_cast<const float *>(tmp.data())[p];
      dst[p * stride + comp] = v;
    }
    return hipSuccess;
  };
  auto get = [&](const char *src, double *dst, int stride, int comp) { return getx(src, dst, stride, comp, false); };
  if (v->offs && e == hipSuccess) {
    for (uint64_t p = 0; p < n; ++p) v->offs[3 * p] = v->offs[3 * p + 1] = v->offs[3 * p + 2] = 0.0;
    for (int a = 0; a < D && e == hipSuccess; ++a) e = getx(base + c->o_offs[a], v->offs, 3, a, true);
  }
  for (int a = 0; a < 3 && v->u && e == hipSuccess; ++a) e = get(base + c->o_u[a], v->u, 3, a);
  if (v->w && e == hipSuccess) e = get(base + c->o_w, v->w, 1, 0);
  if (v->phi && e == hipSuccess && c->o_phi != NONE) e = get(base + c->o_phi, v->phi, 1, 0);
  if (v->cell_prev && e == hipSuccess) {
    e = hipMemcpyAsync(ci.data(), c->prev + c->p_cell + o * 4, n * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    unpack(ci, v->cell_prev, nullptr);
  }
  if (v->offs_prev && e == hipSuccess) {
    for (uint64_t p = 0; p < n; ++p)
      v->offs_prev[3 * p] = v->offs_prev[3 * p + 1] = v->offs_prev[3 * p + 2] = 0.0;
    for (int a = 0; a < D && e == hipSuccess; ++a) e = getx(c->prev + c->p_offs[a], v->offs_prev, 3, a, true);
  }
  if (v->perm && e == hipSuccess) {
    e = hipMemcpyAsync(v->perm, c->scratch + c->s_perm + o * 4, n * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  if (v->id && e == hipSuccess) {
    e = hipMemcpyAsync(v->id, base + c->o_id + o * 4, n * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  return hipchk(c, e, "particles_get");
}

pic_status pic_particle_layout(const pic_ctx *c, pic_layout *L) {
  if (!c || !L) return PIC_E_ARG;
  std::memset(L, 0, sizeof *L);
  L->cell = c->o_cell;
  for (int a = 0; a < 3; ++a) {
    L->offs[a] = c->o_offs[a];
    L->u[a] = c->o_u[a];
    L->prev_offs[a] = c->p_offs[a];
  }
  L->w = c->o_w;
  L->phi = c->o_phi;
  L->id = c->o_id;
  L->capacity = c->capacity;
  for (int s = 0; s < MAXSP; ++s) {
    L->species_offset[s] = s < c->nspec ? c->off[s] : 0;
    L->species_capacity[s] = s < c->nspec ? c->cap[s] : 0;
    L->species_count[s] = s < c->nspec ? c->cnt[s] : 0;
  }
  L->nspecies = c->nspec;
  L->active_set = c->active;
  L->shift2 = c->g.shift2;
  L->shift3 = c->g.shift3;
  L->prev_cell = c->p_cell;
  return PIC_OK;
}

pic_status pic_step_count(const pic_ctx *c, int64_t *step) {
  if (!c || !step) return PIC_E_ARG;
  *step = c->step;
  return PIC_OK;
}

pic_status pic_timing_enable(pic_ctx *c, int32_t enable) {
  if (!c) return PIC_E_ARG;
  if (!c->bound) return fail(c, PIC_E_STATE, "timing before bind_buffers");
  c->timing = enable != 0;
  return hipchk(c, hipMemsetAsync(c->scratch + c->s_stats, 0, 16, c->stream), "timing_enable");
}

pic_status pic_timing_read(pic_ctx *c, pic_timing *out) {
  if (!c || !out) return PIC_E_ARG;
  std::memset(out, 0, sizeof *out);
  hipError_t err = hipSuccess;
  for (auto &e : c->events) {
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventSynchronize(e.b);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e.a, e.b);
    if (e.kind == 0) {
      out->push_launches += 1;
      out->push_ms += ms;
    } else if (e.kind == 1) {
      out->sort_calls += 1;
      out->sort_ms += ms;
    } else {
      out->adjoint_launches += 1;
      out->adjoint_ms += ms;
    }
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  c->events.clear();
  out->sort_brick_calls = c->brick_sorts;
  c->brick_sorts = 0;
  if (err == hipSuccess && c->bound) {
    int32_t st[4] = {0, 0, 0, 0};
    err = hipMemcpyAsync(st, c->scratch + c->s_stats, 16, hipMemcpyDeviceToHost, c->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(c->stream);
    out->push_blocks = st[0];
    out->push_global_particles = st[1];
    if (err == hipSuccess) err = hipMemsetAsync(c->scratch + c->s_stats, 0, 16, c->stream);
  }
  return hipchk(c, err, "timing_read");
}

pic_status pic_adjoint_workspace(const pic_ctx *c, int32_t K, int32_t m, uint64_t *bytes) {
  if (!c || !bytes || K < 1 || m < 1) return PIC_E_ARG;
  *bytes = adj_layout(c, K, m).total;
  return PIC_OK;
}

pic_status pic_forward_checkpointed(pic_ctx *c, double dt, int32_t K, int32_t m, void *ws) {
  if (!c || !ws || K < 1 || m < 1) return PIC_E_ARG;
  if (adjoint_pushers_ok(c) != PIC_OK) return PIC_E_UNSUPPORTED;
  if (!c->bound || !c->fields_ok) return fail(c, PIC_E_STATE, "forward before bind/fields_set");
  if (!(dt > 0) || dt > c->dx_min) return fail(c, PIC_E_ARG, "bad dt");
  const pic_status st = c->eb == 8 ? settle<double>(c) : settle<float>(c);
  if (st != PIC_OK) return st;
  return c->eb == 8 ? fwd_ckpt<double>(c, dt, K, m, static_cast<char *>(ws))
                    : fwd_ckpt<float>(c, dt, K, m, static_cast<char *>(ws));
}

pic_status pic_backward(pic_ctx *c, double dt, int32_t K, int32_t m, void *ws, const void *lamJ,
                        const void *lam_u, void *dEB, void *du0) {
  if (!c || !ws || !dEB || !du0 || K < 1 || m < 1) return PIC_E_ARG;
  if (adjoint_pushers_ok(c) != PIC_OK) return PIC_E_UNSUPPORTED;
  if (!c->bound || !c->fields_ok) return fail(c, PIC_E_STATE, "backward before bind/fields_set");
  if (c->ckpt_K != K || c->ckpt_m != m)
    return fail(c, PIC_E_STATE, "backward(K=%d, m=%d) without a matching forward_checkpointed", K, m);
  if (dt != c->ckpt_dt)
    return fail(c, PIC_E_STATE, "backward dt %.17g differs from the forward's %.17g", dt, c->ckpt_dt);
  const pic_status st = c->eb == 8 ? settle<double>(c) : settle<float>(c);
  if (st != PIC_OK) return st;
  c->bricks_valid = false;  // the sweep restores and replays states
  return c->eb == 8 ? bwd<double>(c, dt, K, m, static_cast<char *>(ws), lamJ, lam_u, dEB, du0)
                    : bwd<float>(c, dt, K, m, static_cast<char *>(ws), lamJ, lam_u, dEB, du0);
}

pic_status pic_checkpointed_order(const pic_ctx *c, const void *ws, int32_t *dst) {
  if (!c || !ws || !dst) return PIC_E_ARG;
  if (c->ckpt_K < 1) return fail(c, PIC_E_STATE, "checkpointed_order before forward_checkpointed");
  const AdjLayout L = adj_layout(c, c->ckpt_K, c->ckpt_m);
  const uint64_t n = c->capacity;
  std::vector<int32_t> order(n), perm(n), next(n);
  for (uint64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
  for (size_t r = 0; r < c->ckpt_sorts.size(); ++r) {
    hipError_t e = hipMemcpyAsync(perm.data(), static_cast<const char *>(ws) + L.perm0 + r * L.perm_bytes,
                                  n * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hipchk(c, e, "checkpointed_order");
    next = order;
    for (int s = 0; s < c->nspec; ++s)
      for (uint64_t i = 0; i < c->cnt[s]; ++i) {
        const int32_t pl = perm[c->off[s] + i];
        if (pl < 0 || (uint64_t)pl >= c->cnt[s])
          return fail(c, PIC_E_STATE, "corrupt stored permutation");
        next[c->off[s] + i] = order[c->off[s] + pl];
      }
    order.swap(next);
  }
  std::memcpy(dst, order.data(), n * 4);
  return PIC_OK;
}

pic_status pic_checkpoint_save(pic_ctx *c, void *slot) {
  if (!c || !slot) return PIC_E_ARG;
  if (!c->bound) return fail(c, PIC_E_STATE, "checkpoint_save before bind_buffers");
  const pic_status st = c->eb == 8 ? settle<double>(c) : settle<float>(c);
  if (st != PIC_OK) return st;
  hipError_t e = c->eb == 8
      ? copy_state<double>(c, slot_pset<double>(c, static_cast<char *>(slot)), pset_of<double>(c, c->active))
      : copy_state<float>(c, slot_pset<float>(c, static_cast<char *>(slot)), pset_of<float>(c, c->active));
  return hipchk(c, e, "checkpoint_save");
}

pic_status pic_checkpoint_load(pic_ctx *c, const void *slot) {
  if (!c || !slot) return PIC_E_ARG;
  if (!c->bound) return fail(c, PIC_E_STATE, "checkpoint_load before bind_buffers");
  c->perm_pending = false;  // the loaded state replaces the sets' contents
  char *sl = const_cast<char *>(static_cast<const char *>(slot));
  hipError_t e = c->eb == 8
      ? copy_state<double>(c, pset_of<double>(c, c->active), slot_pset<double>(c, sl))
      : copy_state<float>(c, pset_of<float>(c, c->active), slot_pset<float>(c, sl));
  c->bricks_valid = false;
  return hipchk(c, e, "checkpoint_load");
}

pic_status pic_adjoint_step(pic_ctx *c, double dt, const void *lamJ, const pic_adjoint_buffers *io) {
  if (!c || !io || !io->lam_u || !io->lam_offs || !io->dEB || (lamJ && !io->lamJ_work))
    return PIC_E_ARG;
  if (adjoint_pushers_ok(c) != PIC_OK) return PIC_E_UNSUPPORTED;
  if (!c->bound || !c->fields_ok) return fail(c, PIC_E_STATE, "adjoint_step before bind/fields_set");
  if (!(dt > 0) || dt > c->dx_min) return fail(c, PIC_E_ARG, "bad dt");
  const pic_status st = c->eb == 8 ? settle<double>(c) : settle<float>(c);
  if (st != PIC_OK) return st;
  return c->eb == 8 ? adjoint_one<double>(c, dt, lamJ, io) : adjoint_one<float>(c, dt, lamJ, io);
}

pic_status pic_device_errors(pic_ctx *c, int32_t *flags, int32_t clear) {
  if (!c || !flags) return PIC_E_ARG;
  if (!c->bound) return fail(c, PIC_E_STATE, "device_errors before bind_buffers");
  int32_t *dev = reinterpret_cast<int32_t *>(c->scratch + c->s_err);
  hipError_t e = hipMemcpyAsync(flags, dev, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess && clear) e = launch_zero<int32_t>(dev, 1, c->stream);
  return hipchk(c, e, "device_errors");
}

pic_status pic_debug_serial(pic_ctx *c, int32_t on) {
  if (!c) return PIC_E_ARG;
  c->debug_serial = on != 0;
  return PIC_OK;
}

pic_status pic_particles_modified(pic_ctx *c) {
  if (!c) return PIC_E_ARG;
  c->bricks_valid = false;
  return PIC_OK;
}

const char *pic_last_error(const pic_ctx *c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
