// C-ABI layer of the narrow-band semi-Lagrangian level-set solver
// (include/lsr.h): argument checks, workspace carving, job state and the
// order of kernel launches for Algorithm 1's loop (Preda & Semplice,
// arXiv:2410.22205).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "lsr_job.h"

using namespace lsr;

namespace lsr {

thread_local std::string g_last_error;

lsr_status fail(lsr_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

}  // namespace lsr

namespace {

int bits_for(int n) {  // bits to hold indices 0..n-1
  int b = 0;
  while ((1LL << b) < (long long)n) ++b;
  return b;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t node_count(const lsr_grid& g) {
  int64_t N = (int64_t)g.n[0] * g.n[1];
  return g.dim == 3 ? N * g.n[2] : N;
}

// Cloud bins of `width` nodes per side over the grid's box, grouped in
// super-bins (see SUP).
BinGeom bin_geom(const lsr_grid& g, int width) {
  BinGeom b;
  for (int a = 0; a < 3; ++a) {
    b.nb[a] = a < g.dim ? (g.n[a] - 1) / width + 1 : 1;
    b.ns[a] = a < g.dim ? (b.nb[a] + SUP - 1) / SUP : 1;
    b.lo[a] = g.lo[a];
    b.hi[a] = a < g.dim ? g.lo[a] + (g.n[a] - 1) * g.h : g.lo[a];
  }
  b.kz = g.dim == 3 ? SUP : 1;
  b.ksup = SUP * SUP * b.kz;
  b.bw = width * g.h;
  b.inv_bw = 1.0 / b.bw;
  return b;
}

Layout make_layout(const lsr_grid& g, int64_t max_points, bool fp64) {
  Layout L;
  const size_t N = (size_t)node_count(g);
  const size_t P = (size_t)(max_points > 0 ? max_points : 1);
  const size_t es = fp64 ? 8 : 4;
  const BinGeom fine = bin_geom(g, BIN_W_FINE);  // room for the bins of either width
  L.nbins = bin_ids(fine);
  const int64_t nsup = (int64_t)fine.ns[0] * fine.ns[1] * fine.ns[2];
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.phi0 = take(es * N);
  L.phi1 = take(es * N);
  L.dp = take(4 * es * N);
  L.d64 = take(8 * N);
  // band lists: whole chunks, and room for the slot lists of a grid scan
  const uint32_t slots = gbar_slots(g.dim, g.n[0], g.n[1], g.dim == 3 ? g.n[2] : 1);
  const size_t nch = (N + LCHUNK - 1) / LCHUNK;
  L.list_cap = (int64_t)std::max(nch * LCHUNK, (size_t)slots * GBAR_CHUNK);
  L.list0 = take(4 * (size_t)L.list_cap);
  L.list1 = take(4 * (size_t)L.list_cap);
  L.ccnt0 = take(4 * nch);
  L.ccnt1 = take(4 * nch);
  L.scnt = take(4 * (size_t)slots);
  L.soff = take(4 * ((size_t)slots + 1));
  L.smark = take((size_t)slots);
  L.listM = take(4 * N);
  L.mflags = take(N);
  {
    // bricks of the distance kernel, marked for the approximate distance
    L.dmark = take(dist_bricks(g.dim, g.n[0], g.n[1], g.dim == 3 ? g.n[2] : 1));
  }
  {
    const size_t rows = g.dim == 3 ? (size_t)g.n[0] * g.n[1] : (size_t)g.n[0];
    L.sgn = take(4 * rows * sign_row_words(g.dim == 3 ? g.n[2] : g.n[1]));
  }
  L.cnt = take(4 * 16);
  L.stats = take(8 * STAT_WORDS);
  L.pts_raw = take(8 * (size_t)g.dim * P);
  L.pts = take(8 * (size_t)g.dim * P);
  L.pt_bin = take(4 * P);
  L.bin_count = take(4 * (size_t)L.nbins);
  L.bin_start = take(4 * ((size_t)L.nbins + 1));
  L.bin_fill = take(4 * (size_t)L.nbins);
  L.occ = take(4 * (size_t)L.nbins);
  L.scan_tmp = take(4 * (2 * (size_t)SCAN_TILES + 1));
  // bin frames: at most one per point and one per bin
  L.max_occ = (int64_t)std::min((size_t)L.nbins, P);
  L.geo = take(8 * (size_t)GEO * (size_t)L.max_occ);
  L.max_sup = (int64_t)std::min((size_t)nsup, P);
  L.sup = take(8 * (size_t)L.max_sup);
  L.sgeo = take(8 * (size_t)GEO * (size_t)L.max_sup);
  L.energy = take(8 * ((size_t)ENERGY_BLOCKS + 1));
  L.nn = take(8 * (P + 1));  // nearest-neighbour distances of a sample, and their mean
  L.total = off;
  return L;
}

lsr_status check_grid(const lsr_grid* g) {
  if (!g) return fail(LSR_E_INVALID, "grid is NULL");
  if (g->dim != 2 && g->dim != 3) return fail(LSR_E_INVALID, "dim must be 2 or 3");
  for (int a = 0; a < g->dim; ++a) {
    if (g->n[a] < 4) return fail(LSR_E_INVALID, "every axis needs at least 4 nodes");
    if (!isfinite(g->lo[a])) return fail(LSR_E_INVALID, "lo must be finite");
  }
  if (!(g->h > 0.0) || !isfinite(g->h)) return fail(LSR_E_INVALID, "h must be finite and > 0");
  const int64_t N = node_count(*g);
  if (N >= (int64_t)1 << 32) return fail(LSR_E_UNSUPPORTED, "grids of 2^32 nodes or more");
  int bits = bits_for(g->n[0]) + bits_for(g->n[1]) + (g->dim == 3 ? bits_for(g->n[2]) : 0);
  if (bits > 32) return fail(LSR_E_UNSUPPORTED, "packed node coordinates need more than 32 bits");
  return LSR_OK;
}

lsr_status check_params(const lsr_grid* g, const lsr_params* p) {
  if (!p) return fail(LSR_E_INVALID, "params is NULL");
  if (!(p->p >= 1.0)) return fail(LSR_E_INVALID, "p must be >= 1");
  if (p->p != 1.0 && p->p != 2.0) return fail(LSR_E_UNSUPPORTED, "p must be 1 or 2");
  if (!(p->delta >= 0.0) || !isfinite(p->delta)) return fail(LSR_E_INVALID, "delta must be >= 0");
  if (!(p->beta > 0.0) || !(p->gamma > p->beta) || !isfinite(p->gamma))
    return fail(LSR_E_INVALID, "need 0 < beta < gamma");
  if (!(p->grad_C >= 0.0) || !isfinite(p->grad_C) || !isfinite(p->grad_alpha))
    return fail(LSR_E_INVALID, "bad fallback threshold");
  if (p->reinit_every < 0 || p->reinit_iters < 0)
    return fail(LSR_E_INVALID, "reinit_every and reinit_iters must be >= 0");
  if (!(p->reinit_dtau > 0.0) || p->reinit_dtau > g->h / sqrt((double)g->dim) * (1.0 + 1e-12))
    return fail(LSR_E_INVALID, "reinit_dtau must be in (0, h/sqrt(dim)]");
  if (!(p->interface_floor > 0.0)) return fail(LSR_E_INVALID, "interface_floor must be > 0");
  if (p->precision != LSR_FP32 && p->precision != LSR_FP64)
    return fail(LSR_E_INVALID, "precision must be LSR_FP32 or LSR_FP64");
  return LSR_OK;
}

}  // namespace

namespace lsr {

lsr_status grid_ok(const lsr_grid* g) { return check_grid(g); }

DevGrid make_devgrid(const lsr_grid& g) {
  DevGrid d;
  d.n0 = g.n[0];
  d.n1 = g.n[1];
  d.n2 = g.dim == 3 ? g.n[2] : 1;
  d.s1 = (uint32_t)d.n2;
  d.s0 = (uint32_t)d.n1 * (uint32_t)d.n2;
  d.N = (uint32_t)node_count(g);
  d.bits_k = g.dim == 3 ? bits_for(d.n2) : 0;
  d.bits_j = bits_for(d.n1);
  d.hd = g.h;
  d.lo0 = g.lo[0];
  d.lo1 = g.lo[1];
  d.lo2 = g.dim == 3 ? g.lo[2] : 0.0;
  return d;
}

template <typename T>
static hipError_t launch_reinit_plan(lsr_job* j, const ReinitPlan<T>& r) {
  hipStream_t s = j->stream;
  const int dim = j->grid.dim;
  hipError_t e = launch_grid_list<T>(dim, r.gb, j->list_blocks, s);
  if (e == hipSuccess) e = launch_reinit_fix<T>(dim, r.fix, j->list_blocks, s);
  for (int it = 0; it < r.iters && e == hipSuccess; ++it)
    e = launch_reinit_iter<T>(dim, r.iter[it % 2], j->list_blocks, s);
  if (e == hipSuccess) e = launch_reinit_final<T>(r.fin, j->list_blocks, s);
  return e;
}

template <typename T>
static lsr_status run_reinit_t(lsr_job* j) {
  ReinitPlan<T> r = plan_reinit<T>(j);
  LSR_HIP(launch_reinit_plan<T>(j, r));
  return LSR_OK;
}

// n steps of the node-list kernel, each followed by the reinitialisation
// when due, from the current plan state, which they advance.  With launch
// false nothing is launched (the state of a replayed graph).
// Algorithm 1, step 2, for p != 1: the partial sums of E_p(phi^n)^p,
// left on the device for the step kernel that follows, which adds them.
template <typename T>
static hipError_t launch_step_energy(lsr_job* j) {
  return energy_now<T>(j, j->prm.p, ENERGY_R, j->energy_buf, nullptr, j->stream);
}

template <typename T>
static hipError_t issue_steps(lsr_job* j, int32_t n, const StepConst<T>& c, int interp,
                              bool launch) {
  hipStream_t s = j->stream;
  hipError_t e = hipSuccess;
  for (int32_t q = 0; q < n && e == hipSuccess; ++q) {
    if (launch && j->prm.p != 1.0) e = launch_step_energy<T>(j);
    SLArgs<T> a = plan_step<T>(j, c);
    if (launch && e == hipSuccess)
      e = launch_sl_step<T>(j->grid.dim, interp, j->lanes, a, j->list_blocks, s);
    if (reinit_due(j)) {
      ReinitPlan<T> r = plan_reinit<T>(j);
      if (launch && e == hipSuccess) e = launch_reinit_plan<T>(j, r);
    }
  }
  return e;
}

struct PlanState {
  int cur, cur_list, ring;
  int64_t step_index, n_reinits, n_steps;
};

static PlanState save_plan(const lsr_job* j) {
  return {j->cur, j->cur_list, j->ring, j->step_index, j->n_reinits, j->n_steps};
}

static void restore_plan(lsr_job* j, const PlanState& p) {
  j->cur = p.cur;
  j->cur_list = p.cur_list;
  j->ring = p.ring;
  j->step_index = p.step_index;
  j->n_reinits = p.n_reinits;
  j->n_steps = p.n_steps;
}

// Steps between two graph keys: twice the reinitialisation period, after
// which buffers, lists and counter slots are back in their roles (a step
// swaps phi and the lists and moves the counter ring by one; a
// reinitialisation moves the ring by two and swaps phi when its iteration
// count is even).
static int32_t graph_chunk(const lsr_job* j) {
  return j->prm.reinit_every > 0 ? 2 * j->prm.reinit_every : 16;
}

template <typename T>
static std::vector<int64_t> graph_key(const lsr_job* j, int32_t n, double dt, int interp) {
  int64_t dtb;
  memcpy(&dtb, &dt, sizeof dtb);
  const int64_t K = j->prm.reinit_every;
  return {(int64_t)sizeof(T), j->cur, j->cur_list, j->ring,
          K > 0 ? j->step_index % K : 0, n, dtb, interp, j->lanes, (int64_t)j->list_blocks};
}

// Steps launched one by one; while kernel timing is on, each step kernel
// carries start and stop events tied to its dispatch.
template <typename T>
static lsr_status direct_steps(lsr_job* j, int32_t n_steps, const StepConst<T>& c, int interp) {
  hipStream_t s = j->stream;
  for (int32_t q = 0; q < n_steps; ++q) {
    if (j->prm.p != 1.0) LSR_HIP(launch_step_energy<T>(j));
    SLArgs<T> a = plan_step<T>(j, c);
    const bool rec = j->prof_on && 2 * (size_t)j->prof_used + 1 < j->prof_ev.size();
    hipEvent_t e0 = rec ? j->prof_ev[2 * j->prof_used] : nullptr;
    hipEvent_t e1 = rec ? j->prof_ev[2 * j->prof_used + 1] : nullptr;
    LSR_HIP(launch_sl_step<T>(j->grid.dim, interp, j->lanes, a, j->list_blocks, s, e0, e1));
    if (rec) j->prof_used += 1;
    if (reinit_due(j)) {
      lsr_status st = run_reinit_t<T>(j);
      if (st != LSR_OK) return st;
    }
  }
  return LSR_OK;
}

template <typename T>
static lsr_status run_steps_t(lsr_job* j, int32_t n_steps, double dt, int interp) {
  hipStream_t s = j->stream;
  const StepConst<T> c = step_const<T>(j, dt);
  // whole chunks through recorded graphs (not while kernel timing is on,
  // never on the null stream, which cannot be captured)
  const int32_t chunk = graph_chunk(j);
  GraphCache& G = j->graphs;
  while (!j->prof_on && G.enabled && s != nullptr && n_steps >= chunk) {
    const std::vector<int64_t> key = graph_key<T>(j, chunk, dt, interp);
    GraphCache::Entry* g = G.find(key);
    bool direct = false;
    if (g) {
      (void)issue_steps<T>(j, chunk, c, interp, false);
      LSR_HIP(G.replay(*g, s));
    } else if (G.seen_before(key)) {
      const PlanState p0 = save_plan(j);
      bool launched = false;
      hipError_t e = G.capture_and_launch(
          s, key, [&]() { return issue_steps<T>(j, chunk, c, interp, true); }, &launched);
      if (e != hipSuccess && launched) LSR_HIP(e);
      if (e != hipSuccess) {
        // nothing ran and the stream cannot be captured: this chunk and
        // all later ones launch directly
        (void)hipGetLastError();
        restore_plan(j, p0);
        G.enabled = false;
        (void)fail(LSR_OK, "step graph not recorded (" + G.failure + "); launching directly");
        direct = true;
      }
    } else {
      direct = true;  // first sight of this key
    }
    if (direct) {
      lsr_status st = direct_steps<T>(j, chunk, c, interp);
      if (st != LSR_OK) return st;
    }
    n_steps -= chunk;
  }
  return direct_steps<T>(j, n_steps, c, interp);
}

lsr_status run_steps(lsr_job* j, int32_t n_steps, double dt, int interp) {
  return j->fp64 ? run_steps_t<double>(j, n_steps, dt, interp)
                 : run_steps_t<float>(j, n_steps, dt, interp);
}

lsr_status run_reinit(lsr_job* j) {
  return j->fp64 ? run_reinit_t<double>(j) : run_reinit_t<float>(j);
}

// Persistent grid of the list kernels: blocks_per_cu blocks per CU, fewer
// for small grids, always a multiple of 8 (one share per XCD).
void set_list_blocks(lsr_job* j) {
  uint64_t want = ((uint64_t)j->dg.N + 255) / 256;
  uint64_t cap = (uint64_t)j->ncu * (uint64_t)j->blocks_per_cu;
  uint64_t lb = want < cap ? want : cap;
  lb = ((lb + 7) / 8) * 8;
  j->list_blocks = (unsigned)lb;
}

hipError_t dpack(lsr_job* j) {
  return j->fp64 ? launch_dpack<double>(j->grid.dim, j->dg, j->d64,
                                        (typename Vec<double>::pack*)j->dp, j->stream)
                 : launch_dpack<float>(j->grid.dim, j->dg, j->d64,
                                       (typename Vec<float>::pack*)j->dp, j->stream);
}

// Passes of an iteration to its fixed point: groups of four passes, each
// flagging a change in its own counter slot, until the last pass of a group
// changes nothing (one synchronisation per group); at most about eight
// passes per node along the grid's axes.
template <typename F>
lsr_status until_still(lsr_job* j, const char* what, F pass) {
  hipStream_t s = j->stream;
  int32_t* fl = j->cnt + 12;
  constexpr int G = 4;
  const int64_t max_passes = 8 * ((int64_t)j->dg.n0 + j->dg.n1 + j->dg.n2) + 64;
  for (int64_t done = 0; done < max_passes; done += G) {
    LSR_HIP(launch_fill_u32((uint32_t*)fl, 0u, G, s));
    for (int q = 0; q < G; ++q) LSR_HIP(pass(fl + q));
    int32_t last = 1;
    LSR_HIP(hipMemcpyAsync(&last, fl + G - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LSR_HIP(hipStreamSynchronize(s));
    if (!last) return LSR_OK;
  }
  return fail(LSR_E_DEVICE, std::string(what) + " did not reach its fixed point");
}

// Arguments of the grid scan that builds the first band (|phi| < gamma) of
// freshly initialised data into list 0, chunked; list 1 holds the slots.
template <typename T>
GbarArgs<T> first_band(lsr_job* j) {
  GbarArgs<T> a;
  a.g = j->dg;
  a.gamma = (T)j->prm.gamma;
  a.nbr = 0;
  a.smark = nullptr;
  a.L = nullptr;
  a.Lccnt = a.Lcnt = nullptr;
  a.P = phi_buf<T>(j, 0);
  a.S = j->list[1];
  a.scnt = j->scnt;
  a.soff = j->soff;
  a.M = j->list[0];
  a.cnt_out = j->cnt;  // ring slot 0
  a.ccnt = j->ccnt[0];
  return a;
}

// After new initial data: counters and statistics cleared, the first band
// built (in the order of a brick-by-brick scan of the grid), the step index
// set.
lsr_status start_loop(lsr_job* j, int64_t step0) {
  hipStream_t s = j->stream;
  LSR_HIP(launch_fill_u32((uint32_t*)j->cnt, 0u, 3, s));
  LSR_HIP(launch_fill_u32((uint32_t*)j->stats, 0u, 2 * STAT_WORDS, s));
  if (j->fp64) {
    LSR_HIP(launch_grid_list<double>(j->grid.dim, first_band<double>(j), j->list_blocks, s));
    LSR_HIP(launch_sign_build<double>(j->dg, phi_buf<double>(j, 0), j->sgn, s));
  } else {
    LSR_HIP(launch_grid_list<float>(j->grid.dim, first_band<float>(j), j->list_blocks, s));
    LSR_HIP(launch_sign_build<float>(j->dg, phi_buf<float>(j, 0), j->sgn, s));
  }
  j->cur = 0;
  j->cur_list = 0;
  j->ring = 0;
  j->step_index = step0;
  j->n_reinits = 0;
  j->n_steps = 0;
  j->has_phi = true;
  return LSR_OK;
}

// Initial data into both phi buffers, or (write = false) only the check of
// the caller's array.
hipError_t init_phi(lsr_job* j, int kind, const double* a, const void* src, bool write) {
  const int dim = j->grid.dim;
  if (j->fp64)
    return launch_init_phi<double>(dim, j->dg, kind, a, j->prm.gamma, (const double*)src,
                                   write ? phi_buf<double>(j, 0) : nullptr,
                                   write ? phi_buf<double>(j, 1) : nullptr, j->cnt + 3, j->stream);
  return launch_init_phi<float>(dim, j->dg, kind, a, (float)j->prm.gamma, (const float*)src,
                                write ? phi_buf<float>(j, 0) : nullptr,
                                write ? phi_buf<float>(j, 1) : nullptr, j->cnt + 3, j->stream);
}

}  // namespace lsr

extern "C" {

const char* lsr_last_error(void) { return g_last_error.c_str(); }

lsr_status lsr_params_default(int32_t dim, double h, lsr_params* out) {
  if (!out) return fail(LSR_E_INVALID, "out is NULL");
  if (dim != 2 && dim != 3) return fail(LSR_E_INVALID, "dim must be 2 or 3");
  if (!(h > 0.0) || !isfinite(h)) return fail(LSR_E_INVALID, "h must be > 0");
  lsr_params p;
  p.p = 1.0;
  p.delta = 1.0;
  p.gamma = (dim == 2 ? 4.0 : 6.0) * h;
  p.beta = (dim == 2 ? 2.0 : 3.0) * h;
  p.grad_C = 1e-3;
  p.grad_alpha = 1.0;
  p.reinit_every = dim == 2 ? 1 : 10;
  p.reinit_dtau = 0.5 * h;
  p.reinit_iters = (int32_t)ceil((p.gamma + h) / p.reinit_dtau - 1e-9);
  p.interface_floor = 1e-3;
  p.precision = LSR_FP32;
  *out = p;
  return LSR_OK;
}

lsr_status lsr_schedule_run(int32_t r, int32_t dim, const double* box_lo, const double* box_hi,
                            double h_s, double k_s, lsr_grid* grid, lsr_params* params,
                            double* dt) {
  if (!box_lo || !box_hi || !grid || !params || !dt) return fail(LSR_E_INVALID, "NULL argument");
  if (r < 1 || r > 30) return fail(LSR_E_INVALID, "runs are numbered 1 .. 30");
  if (dim != 2 && dim != 3) return fail(LSR_E_INVALID, "dim must be 2 or 3");
  if (!(h_s > 0.0) || !isfinite(h_s)) return fail(LSR_E_INVALID, "h_s must be finite and > 0");
  if (!(k_s >= 0.0) || !isfinite(k_s)) return fail(LSR_E_INVALID, "k_s must be finite and >= 0");
  for (int a = 0; a < dim; ++a)
    if (!isfinite(box_lo[a]) || !isfinite(box_hi[a]) || box_hi[a] < box_lo[a])
      return fail(LSR_E_INVALID, "the cloud's box must be finite with hi >= lo");
  // eq. (dxdt)
  const double dx = h_s / pow(2.0, (double)(r - 1));
  // margin: the band half width in cells plus 4, and gamma_S in the first run
  int m = (dim == 2 ? 4 : 6) + 4;
  if (r == 1) m += (int)ceil(k_s * h_s / dx - 1e-9);
  lsr_grid g;
  memset(&g, 0, sizeof g);
  g.dim = dim;
  g.h = dx;
  for (int a = 0; a < 3; ++a) {
    if (a < dim) {
      const double cells = ceil((box_hi[a] - box_lo[a]) / dx);
      if (cells + 1.0 + 2.0 * m > 2147483647.0) return fail(LSR_E_INVALID, "grid too large");
      g.n[a] = (int32_t)cells + 1 + 2 * m;
      g.lo[a] = box_lo[a] - m * dx;
    } else {
      g.n[a] = 1;
      g.lo[a] = 0.0;
    }
  }
  lsr_params p;
  lsr_status st = lsr_params_default(dim, dx, &p);
  if (st != LSR_OK) return st;
  // Table param
  p.p = r == 1 ? 1.0 : 2.0;
  p.delta = r <= 2 ? 0.0 : 1.0;
  *grid = g;
  *params = p;
  *dt = dx / 4.0;
  return LSR_OK;
}

lsr_status lsr_workspace_bytes(const lsr_grid* grid, const lsr_params* params, int64_t max_points,
                               size_t* bytes) {
  lsr_status st = check_grid(grid);
  if (st != LSR_OK) return st;
  if (!bytes) return fail(LSR_E_INVALID, "bytes is NULL");
  if (max_points < 0) return fail(LSR_E_INVALID, "max_points must be >= 0");
  const bool fp64 = params && params->precision == LSR_FP64;
  *bytes = make_layout(*grid, max_points, fp64).total;
  return LSR_OK;
}

lsr_status lsr_create(const lsr_grid* grid, const lsr_params* params, void* dev_workspace,
                      size_t ws_bytes, void* hip_stream, lsr_job** out) {
  lsr_status st = check_grid(grid);
  if (st != LSR_OK) return st;
  st = check_params(grid, params);
  if (st != LSR_OK) return st;
  if (!out) return fail(LSR_E_INVALID, "out is NULL");
  if (!dev_workspace) return fail(LSR_E_INVALID, "workspace is NULL");
  if (((uintptr_t)dev_workspace) & 255) return fail(LSR_E_INVALID, "workspace must be 256-byte aligned");
  // the largest cloud the workspace holds
  const bool fp64 = params->precision == LSR_FP64;
  Layout L0 = make_layout(*grid, 1, fp64);
  if (ws_bytes < L0.total) return fail(LSR_E_NOMEM, "workspace smaller than lsr_workspace_bytes");
  // largest cloud that fits: the layout grows monotonically with the cloud size
  int64_t lo = 1, hi = 2;
  while (make_layout(*grid, hi, fp64).total <= ws_bytes) {
    lo = hi;
    hi *= 2;
  }
  while (hi - lo > 1) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (make_layout(*grid, mid, fp64).total <= ws_bytes)
      lo = mid;
    else
      hi = mid;
  }
  const int64_t maxp = lo;
  Layout L = make_layout(*grid, maxp, fp64);
  if (L.total > ws_bytes) return fail(LSR_E_NOMEM, "workspace too small");

  int dev = 0, ncu = 0;
  LSR_HIP(hipGetDevice(&dev));
  LSR_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));

  lsr_job* j = new (std::nothrow) lsr_job();
  if (!j) return fail(LSR_E_NOMEM, "host allocation failed");
  j->grid = *grid;
  if (grid->dim == 2) {
    j->grid.n[2] = 1;
    j->grid.lo[2] = 0.0;
  }
  j->prm = *params;
  j->fp64 = fp64;
  j->in_batch = false;
  j->own_stream = (hipStream_t)hip_stream;
  j->stream = (hipStream_t)hip_stream;
  j->ws = (char*)dev_workspace;
  j->ws_bytes = ws_bytes;
  j->L = L;
  j->max_points = maxp;
  const lsr_grid& g = j->grid;
  j->dg = make_devgrid(g);
  j->bg = bin_geom(g, BIN_W);
  j->bg_fine = bin_geom(g, BIN_W_FINE);

  char* w = j->ws;
  j->phi[0] = (void*)(w + L.phi0);
  j->phi[1] = (void*)(w + L.phi1);
  j->dp = (void*)(w + L.dp);
  j->d64 = (double*)(w + L.d64);
  j->list[0] = (uint32_t*)(w + L.list0);
  j->list[1] = (uint32_t*)(w + L.list1);
  j->ccnt[0] = (int32_t*)(w + L.ccnt0);
  j->ccnt[1] = (int32_t*)(w + L.ccnt1);
  j->scnt = (int32_t*)(w + L.scnt);
  j->soff = (int32_t*)(w + L.soff);
  j->smark = (uint8_t*)(w + L.smark);
  j->listM = (uint32_t*)(w + L.listM);
  j->mflags = (uint8_t*)(w + L.mflags);
  j->dmark = (uint8_t*)(w + L.dmark);
  j->sgn = (uint32_t*)(w + L.sgn);
  j->cnt = (int32_t*)(w + L.cnt);
  j->stats = (unsigned long long*)(w + L.stats);
  j->pts_raw = (double*)(w + L.pts_raw);
  j->pts = (double*)(w + L.pts);
  j->pt_bin = (int32_t*)(w + L.pt_bin);
  j->bin_count = (int32_t*)(w + L.bin_count);
  j->bin_start = (int32_t*)(w + L.bin_start);
  j->bin_fill = (int32_t*)(w + L.bin_fill);
  j->occ = (uint32_t*)(w + L.occ);
  j->scan_tmp = (int32_t*)(w + L.scan_tmp);
  j->geo = (double*)(w + L.geo);
  j->max_occ = L.max_occ;
  j->sup = (int2*)(w + L.sup);
  j->sgeo = (double*)(w + L.sgeo);
  j->max_sup = L.max_sup;
  j->energy_buf = (double*)(w + L.energy);
  j->nn = (double*)(w + L.nn);
  j->n_cloud = 0;
  j->ncu = ncu > 0 ? ncu : 256;
  j->lanes = 1;
  j->blocks_per_cu = 8;
  set_list_blocks(j);
  j->cur = 0;
  j->cur_list = 0;
  j->ring = 0;
  j->step_index = 0;
  j->n_reinits = 0;
  j->n_steps = 0;
  j->has_d = false;
  j->has_phi = false;
  j->prof_on = false;
  j->prof_used = 0;

  hipStream_t s = j->stream;
  hipError_t e = launch_fill_u32((uint32_t*)j->cnt, 0u, 16, s);
  if (e == hipSuccess)
    e = launch_fill_u8(j->smark, 0,
                       gbar_slots(grid->dim, grid->n[0], grid->n[1], grid->dim == 3 ? grid->n[2] : 1),
                       s);
  if (e == hipSuccess) e = launch_fill_u32((uint32_t*)j->stats, 0u, 2 * STAT_WORDS, s);
  if (e != hipSuccess) {
    delete j;
    return fail(LSR_E_DEVICE, std::string("clearing the workspace: ") + hipGetErrorString(e));
  }
  *out = j;
  return LSR_OK;
}

}  // extern "C"

namespace lsr {

// The cloud into the workspace, binned and sorted, and the distance field:
// exact at every node, or (approx) the paper's approximation of Section 3.4.
static lsr_status load_cloud(lsr_job* j, const double* dev_xyz, int64_t n, bool approx) {
  if (!j) return fail(LSR_E_INVALID, "job is NULL");
  if (j->in_batch) return fail(LSR_E_STATE, "job belongs to a batch");
  if (!dev_xyz) return fail(LSR_E_INVALID, "points are NULL");
  if (n < 1) return fail(LSR_E_INVALID, "the cloud needs at least one point");
  if (n > j->max_points) return fail(LSR_E_NOMEM, "cloud larger than the workspace allows");
  hipStream_t s = j->stream;
  const int dim = j->grid.dim;
  {
    // check the points before touching the stored cloud
    int32_t bad = 0;
    LSR_HIP(launch_fill_u32((uint32_t*)(j->cnt + 3), 0u, 1, s));
    LSR_HIP(launch_check_points(dim, j->bg, dev_xyz, n, j->cnt + 3, s));
    LSR_HIP(hipMemcpyAsync(&bad, j->cnt + 3, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LSR_HIP(hipStreamSynchronize(s));
    if (bad) return fail(LSR_E_INVALID, "cloud has a non-finite point or one outside the grid box");
  }
  j->n_cloud = 0;  // set again once the new cloud is binned and sorted
  LSR_HIP(hipMemcpyAsync(j->pts_raw, dev_xyz, sizeof(double) * dim * (size_t)n,
                         hipMemcpyDeviceToDevice, s));
  // bin at the standard width; validate the points and count occupied bins
  auto bin = [&](const BinGeom& bg) -> hipError_t {
    hipError_t e = launch_fill_u32((uint32_t*)j->bin_count, 0u, (uint64_t)bin_ids(bg), s);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t*)(j->cnt + 3), 0u, 1, s);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t*)(j->cnt + 6), 0u, 1, s);
    if (e == hipSuccess)
      e = launch_bin_points(dim, bg, j->pts_raw, n, j->bin_count, j->pt_bin, j->cnt + 3,
                            j->cnt + 6, s);
    return e;
  };
  LSR_HIP(bin(j->bg));
  int32_t got[4] = {0, 0, 0, 0};  // flag, -, -, occupied bins
  LSR_HIP(hipMemcpyAsync(got, j->cnt + 3, sizeof(got), hipMemcpyDeviceToHost, s));
  LSR_HIP(hipStreamSynchronize(s));
  if (got[0]) return fail(LSR_E_INVALID, "cloud has a non-finite point or one outside the grid box");
  // a dense cloud (many points per occupied bin) gets the finer bins: the
  // nodes of a brick then scan fewer points per bin they cannot rule out
  const bool fine = got[3] > 0 && n > (int64_t)DENSE_BIN * got[3];
  const BinGeom& bg = fine ? j->bg_fine : j->bg;
  if (fine) LSR_HIP(bin(bg));
  const int32_t nbins = bin_ids(bg);
  const int64_t max_occ = std::min(j->max_occ, (int64_t)nbins);
  const int64_t max_sup =
      std::min(j->max_sup, (int64_t)bg.ns[0] * bg.ns[1] * bg.ns[2]);
  LSR_HIP(launch_fill_u32((uint32_t*)j->bin_fill, 0u, (uint64_t)nbins, s));
  LSR_HIP(launch_fill_u32((uint32_t*)(j->cnt + 5), 0u, 1, s));
  LSR_HIP(launch_fill_u32((uint32_t*)(j->cnt + 7), 0u, 1, s));
  LSR_HIP(launch_scan_bins(j->bin_count, nbins, j->bin_start, j->scan_tmp, s));
  LSR_HIP(launch_occupied(j->bin_start, nbins, j->occ, j->cnt + 5, s));
  LSR_HIP(launch_super_list(bg, j->occ, j->cnt + 5, j->sup, j->cnt + 7, max_occ, s));
  LSR_HIP(launch_scatter_points(dim, j->pts_raw, n, j->pt_bin, j->bin_start, j->bin_fill, j->pts, s));
  LSR_HIP(launch_bin_geo(dim, j->pts, j->bin_start, j->occ, j->cnt + 5, j->geo, max_occ, s));
  LSR_HIP(launch_super_geo(dim, j->pts, j->bin_start, j->occ, j->sup, j->cnt + 7, j->sgeo, max_sup,
                           s));
  DistArgs da;
  da.g = j->dg;
  da.bg = bg;
  da.pts = j->pts;
  da.start = j->bin_start;
  da.occ = j->occ;
  da.occ_cnt = j->cnt + 5;
  da.geo = j->geo;
  da.sgeo = j->sgeo;
  da.sup_cnt = j->cnt + 7;
  {
    // margins that cover the rounding of the frame bounds: every coordinate
    // lies in the grid's box
    double diag2 = 0.0;
    for (int ax = 0; ax < dim; ++ax) diag2 += (bg.hi[ax] - bg.lo[ax]) * (bg.hi[ax] - bg.lo[ax]);
    const double diag = std::max(std::sqrt(diag2), j->grid.h);
    da.mu = 1e-12 * diag;
    da.mu2 = 1e-12 * diag * diag;
  }
  da.d64 = j->d64;
  da.bmark = nullptr;
  j->bg_load = bg;
  j->n_cloud = n;
  const unsigned bricks = (unsigned)dist_bricks(dim, j->dg.n0, j->dg.n1, j->dg.n2);
  if (approx) {
    // exact values only on the bricks holding a point's 4^dim box, then the
    // fast-sweeping fixed point from the box nodes outwards
    LSR_HIP(launch_fill_u8(j->mflags, 0, j->dg.N, s));
    LSR_HIP(launch_fill_u8(j->dmark, 0, bricks, s));
    LSR_HIP(launch_box_mark(dim, j->dg, j->pts_raw, n, j->mflags, j->dmark, s));
    da.bmark = j->dmark;
  }
  LSR_HIP(launch_distance(dim, da, bricks, s));
  j->has_d = false;
  if (approx) {
    LSR_HIP(launch_eik_init(j->dg, j->d64, j->mflags, j->d64, s));
    lsr_status st = until_still(j, "the approximate distance", [&](int32_t* fl) {
      return launch_eik_pass(dim, j->dg, j->d64, j->mflags, fl, s);
    });
    if (st != LSR_OK) return st;
  }
  LSR_HIP(dpack(j));
  j->has_d = true;
  return LSR_OK;
}

}  // namespace lsr

extern "C" {

lsr_status lsr_load_cloud(lsr_job* j, const double* dev_xyz, int64_t n) {
  return load_cloud(j, dev_xyz, n, false);
}

lsr_status lsr_load_cloud_approx(lsr_job* j, const double* dev_xyz, int64_t n) {
  return load_cloud(j, dev_xyz, n, true);
}

lsr_status lsr_set_distance(lsr_job* j, const double* dev_d) {
  if (!j) return fail(LSR_E_INVALID, "job is NULL");
  if (j->in_batch) return fail(LSR_E_STATE, "job belongs to a batch");
  if (!dev_d) return fail(LSR_E_INVALID, "distance is NULL");
  LSR_HIP(hipMemcpyAsync(j->d64, dev_d, sizeof(double) * j->dg.N, hipMemcpyDeviceToDevice,
                         j->stream));
  j->n_cloud = 0;  // a given field, no cloud
  LSR_HIP(dpack(j));
  j->has_d = true;
  return LSR_OK;
}

lsr_status lsr_get_distance(lsr_job* j, double* dev_out) {
  if (!j || !dev_out) return fail(LSR_E_INVALID, "NULL argument");
  if (!j->has_d) return fail(LSR_E_STATE, "no distance field yet");
  LSR_HIP(hipMemcpyAsync(dev_out, j->d64, sizeof(double) * j->dg.N, hipMemcpyDeviceToDevice,
                         j->stream));
  return LSR_OK;
}

lsr_status lsr_init_phi(lsr_job* j, const void* dev_phi0, int32_t kind, const double* args,
                        int64_t step0) {
  if (!j) return fail(LSR_E_INVALID, "job is NULL");
  if (j->in_batch) return fail(LSR_E_STATE, "job belongs to a batch");
  if (kind < 0 || kind > 2) return fail(LSR_E_INVALID, "unknown kind");
  if (kind == LSR_PHI_ARRAY && !dev_phi0) return fail(LSR_E_INVALID, "phi0 is NULL");
  if (kind == LSR_PHI_TORUS && j->grid.dim != 3) return fail(LSR_E_INVALID, "torus needs 3D");
  if (kind != LSR_PHI_ARRAY && !args) return fail(LSR_E_INVALID, "args is NULL");
  if (step0 < 0) return fail(LSR_E_INVALID, "step0 must be >= 0");
  double a[5] = {0, 0, 0, 0, 0};
  if (kind != LSR_PHI_ARRAY) {
    const int na = kind == LSR_PHI_SPHERE ? 4 : 5;
    for (int q = 0; q < na; ++q) {
      if (!isfinite(args[q])) return fail(LSR_E_INVALID, "args must be finite");
      a[q] = args[q];
    }
    if (j->grid.dim == 2) a[2] = 0.0;
  }
  hipStream_t s = j->stream;
  if (kind == LSR_PHI_ARRAY) {
    // check the input before touching the state (no output buffers: check only)
    LSR_HIP(launch_fill_u32((uint32_t*)(j->cnt + 3), 0u, 1, s));
    LSR_HIP(init_phi(j, 0, a, dev_phi0, false));
    int32_t flag = 0;
    LSR_HIP(hipMemcpyAsync(&flag, j->cnt + 3, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LSR_HIP(hipStreamSynchronize(s));
    if (flag) return fail(LSR_E_INVALID, "phi0 has a non-finite value");
  }
  LSR_HIP(init_phi(j, kind, a, dev_phi0, true));
  return start_loop(j, step0);
}

lsr_status lsr_init_phi_cloud(lsr_job* j, double gamma_s, int64_t step0) {
  if (!j) return fail(LSR_E_INVALID, "job is NULL");
  if (j->in_batch) return fail(LSR_E_STATE, "job belongs to a batch");
  if (!(gamma_s > 0.0) || !isfinite(gamma_s)) return fail(LSR_E_INVALID, "gamma_s must be > 0");
  if (step0 < 0) return fail(LSR_E_INVALID, "step0 must be >= 0");
  if (!j->has_d) return fail(LSR_E_STATE, "no distance field: call lsr_load_cloud first");
  hipStream_t s = j->stream;
  const int dim = j->grid.dim;
  uint8_t* ext = j->mflags;
  double* u = (double*)j->dp;  // the packed gradient is rebuilt from d afterwards
  LSR_HIP(launch_mark_init(dim, j->dg, j->d64, gamma_s, ext, s));
  lsr_status st = until_still(j, "the external marking", [&](int32_t* fl) {
    return launch_mark_pass(dim, j->dg, j->d64, gamma_s, ext, fl, s);
  });
  if (st == LSR_OK) {
    LSR_HIP(launch_eik_init_ext(j->dg, j->d64, gamma_s, ext, u, s));
    st = until_still(j, "the fast sweeping", [&](int32_t* fl) {
      return launch_eik_pass(dim, j->dg, u, ext, fl, s);
    });
  }
  if (st == LSR_OK) {
    if (j->fp64)
      LSR_HIP(launch_phi0_cloud<double>(j->dg, j->d64, u, ext, gamma_s, j->prm.gamma,
                                        phi_buf<double>(j, 0), phi_buf<double>(j, 1), s));
    else
      LSR_HIP(launch_phi0_cloud<float>(j->dg, j->d64, u, ext, gamma_s, (float)j->prm.gamma,
                                       phi_buf<float>(j, 0), phi_buf<float>(j, 1), s));
  }
  LSR_HIP(dpack(j));
  if (st != LSR_OK) return st;
  return start_loop(j, step0);
}

lsr_status lsr_init_phi_resample(lsr_job* j, const lsr_job* coarse, lsr_interp interp,
                                 int64_t step0) {
  if (!j || !coarse) return fail(LSR_E_INVALID, "job is NULL");
  if (j == coarse) return fail(LSR_E_INVALID, "the coarser job must be another job");
  if (j->in_batch) return fail(LSR_E_STATE, "job belongs to a batch");
  if (interp != LSR_Q1 && interp != LSR_WENO) return fail(LSR_E_INVALID, "unknown interpolator");
  if (step0 < 0) return fail(LSR_E_INVALID, "step0 must be >= 0");
  if (coarse->grid.dim != j->grid.dim || coarse->fp64 != j->fp64)
    return fail(LSR_E_INVALID, "both jobs need the same dimension and precision");
  if (!coarse->has_phi) return fail(LSR_E_STATE, "the coarser job has no phi");
  hipStream_t s = j->stream;
  LSR_HIP(order_after(s, coarse->stream));
  const double hc = coarse->grid.h;
  if (j->fp64)
    LSR_HIP(launch_resample<double>(j->grid.dim, (int)interp, j->dg, coarse->dg,
                                    (const double*)coarse->phi[coarse->cur], j->prm.gamma,
                                    hc * hc * hc * hc, phi_buf<double>(j, 0),
                                    phi_buf<double>(j, 1), s));
  else
    LSR_HIP(launch_resample<float>(j->grid.dim, (int)interp, j->dg, coarse->dg,
                                   (const float*)coarse->phi[coarse->cur], (float)j->prm.gamma,
                                   (float)(hc * hc * hc * hc), phi_buf<float>(j, 0),
                                   phi_buf<float>(j, 1), s));
  // the coarser job's stream waits for the read before it may change phi
  LSR_HIP(order_after(coarse->stream, s));
  return start_loop(j, step0);
}

lsr_status lsr_step(lsr_job* j, int32_t n_steps, double dt, lsr_interp interp) {
  if (!j) return fail(LSR_E_INVALID, "job is NULL");
  if (n_steps < 0) return fail(LSR_E_INVALID, "n_steps must be >= 0");
  if (!(dt > 0.0) || !isfinite(dt)) return fail(LSR_E_INVALID, "dt must be > 0");
  if (interp != LSR_Q1 && interp != LSR_WENO) return fail(LSR_E_INVALID, "unknown interpolator");
  if (!j->has_d) return fail(LSR_E_STATE, "no distance field: call lsr_load_cloud first");
  if (!j->has_phi) return fail(LSR_E_STATE, "no phi: call lsr_init_phi first");
  if (j->in_batch) return fail(LSR_E_STATE, "job belongs to a batch");
  return run_steps(j, n_steps, dt, (int)interp);
}

lsr_status lsr_reinit(lsr_job* j) {
  if (!j) return fail(LSR_E_INVALID, "job is NULL");
  if (!j->has_phi) return fail(LSR_E_STATE, "no phi: call lsr_init_phi first");
  if (j->in_batch) return fail(LSR_E_STATE, "job belongs to a batch");
  return run_reinit(j);
}

lsr_status lsr_energy(lsr_job* j, double p, int32_t R, double* out) {
  if (!j || !out) return fail(LSR_E_INVALID, "NULL argument");
  if (j->in_batch) return fail(LSR_E_STATE, "job belongs to a batch");
  if (!(p > 0.0) || !isfinite(p)) return fail(LSR_E_INVALID, "p must be finite and > 0");
  if (R < 1 || R > 64) return fail(LSR_E_INVALID, "R must be in 1..64");
  if (!j->has_phi) return fail(LSR_E_STATE, "no phi: call lsr_init_phi first");
  if (!j->has_d) return fail(LSR_E_STATE, "no distance field yet");
  hipStream_t s = j->stream;
  double* part = j->energy_buf;
  double* dout = part + ENERGY_BLOCKS;
  if (j->fp64)
    LSR_HIP(energy_now<double>(j, p, R, part, dout, s));
  else
    LSR_HIP(energy_now<float>(j, p, R, part, dout, s));
  double v = 0.0;
  LSR_HIP(hipMemcpyAsync(&v, dout, sizeof(double), hipMemcpyDeviceToHost, s));
  LSR_HIP(hipStreamSynchronize(s));
  *out = v;
  return LSR_OK;
}

lsr_status lsr_cloud_spacing(lsr_job* j, const int64_t* dev_sample, int64_t n_sample,
                             double* out) {
  if (!j || !dev_sample || !out) return fail(LSR_E_INVALID, "NULL argument");
  if (j->in_batch) return fail(LSR_E_STATE, "job belongs to a batch");
  if (j->n_cloud < 2) return fail(LSR_E_STATE, "needs a cloud of two or more points (lsr_load_cloud)");
  if (n_sample < 1 || n_sample > j->max_points)
    return fail(LSR_E_INVALID, "n_sample must be in 1..max_points");
  hipStream_t s = j->stream;
  int32_t* flag = j->cnt + 11;
  LSR_HIP(launch_fill_u32((uint32_t*)flag, 0u, 1, s));
  LSR_HIP(launch_cloud_spacing(j->grid.dim, j->bg_load, j->pts, j->bin_start, j->pts_raw,
                               j->n_cloud, dev_sample, n_sample, j->nn, flag,
                               j->nn + j->max_points, s));
  double v = 0.0;
  int32_t bad = 0;
  LSR_HIP(hipMemcpyAsync(&v, j->nn + j->max_points, sizeof(double), hipMemcpyDeviceToHost, s));
  LSR_HIP(hipMemcpyAsync(&bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  LSR_HIP(hipStreamSynchronize(s));
  if (bad) return fail(LSR_E_INVALID, "a sample index lies outside the cloud");
  *out = v;
  return LSR_OK;
}

int32_t lsr_energy_stop(const double* e, int32_t n, int32_t min_steps, int32_t max_steps,
                        double tol) {
  if (!e || n < 0) return -1;
  if (n >= max_steps) return 1;
  if (n < min_steps || n < 1) return 0;
  const int32_t k = n < LSR_ENERGY_WINDOW ? n : LSR_ENERGY_WINDOW;
  double cur = 0.0, prev = 0.0;
  for (int32_t i = n - k + 1; i <= n; ++i) cur += e[i];
  for (int32_t i = n - k; i <= n - 1; ++i) prev += e[i];
  cur /= k;
  prev /= k;
  if (!(cur > 0.0)) return 1;
  return fabs(prev - cur) / cur < tol ? 1 : 0;
}

lsr_status lsr_run_to_steady(lsr_job* j, double dt, lsr_interp interp, int32_t min_steps,
                             int32_t max_steps, double tol, double* energies, int32_t* n_done) {
  if (!j || !n_done) return fail(LSR_E_INVALID, "NULL argument");
  if (min_steps < 0 || max_steps < 1 || min_steps > max_steps)
    return fail(LSR_E_INVALID, "need 0 <= min_steps <= max_steps and max_steps >= 1");
  if (!(tol >= 0.0) || !isfinite(tol)) return fail(LSR_E_INVALID, "tol must be finite and >= 0");
  std::vector<double> e((size_t)max_steps + 1, 0.0);
  lsr_status st = lsr_energy(j, 2.0, ENERGY_R, &e[0]);
  int32_t n = 0;
  while (st == LSR_OK && lsr_energy_stop(e.data(), n, min_steps, max_steps, tol) == 0) {
    st = lsr_step(j, 1, dt, interp);
    if (st != LSR_OK) break;
    n += 1;
    st = lsr_energy(j, 2.0, ENERGY_R, &e[(size_t)n]);
  }
  *n_done = n;
  if (energies) memcpy(energies, e.data(), sizeof(double) * ((size_t)n + 1));
  return st;
}

lsr_status lsr_extract(lsr_job* j, void* dev_phi, uint8_t* dev_band, int64_t* n_band,
                       int64_t* step_index) {
  if (!j) return fail(LSR_E_INVALID, "job is NULL");
  if (!j->has_phi) return fail(LSR_E_STATE, "no phi: call lsr_init_phi first");
  hipStream_t s = j->stream;
  if (dev_phi)
    LSR_HIP(hipMemcpyAsync(dev_phi, j->phi[j->cur], (j->fp64 ? 8 : 4) * (size_t)j->dg.N,
                           hipMemcpyDeviceToDevice, s));
  if (dev_band || n_band) {
    if (dev_band) LSR_HIP(launch_fill_u8(dev_band, 0, j->dg.N, s));
    LSR_HIP(launch_fill_u32((uint32_t*)(j->cnt + 4), 0u, 1, s));
    if (j->fp64)
      LSR_HIP(launch_band_mask<double>(j->dg, j->prm.gamma, phi_buf<double>(j, j->cur),
                                       j->list[j->cur_list], j->ccnt[j->cur_list], ring_slot(j, 0),
                                       dev_band, j->cnt + 4, j->list_blocks, s));
    else
      LSR_HIP(launch_band_mask<float>(j->dg, (float)j->prm.gamma, phi_buf<float>(j, j->cur),
                                      j->list[j->cur_list], j->ccnt[j->cur_list], ring_slot(j, 0),
                                      dev_band, j->cnt + 4, j->list_blocks, s));
  }
  if (n_band) {
    int32_t c = 0;
    LSR_HIP(hipMemcpyAsync(&c, j->cnt + 4, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LSR_HIP(hipStreamSynchronize(s));
    *n_band = c;
  }
  if (step_index) *step_index = j->step_index;
  return LSR_OK;
}

lsr_status lsr_counters(lsr_job* j, int64_t* out, int32_t n) {
  if (!j || !out) return fail(LSR_E_INVALID, "NULL argument");
  if (n < 0) return fail(LSR_E_INVALID, "n must be >= 0");
  std::vector<unsigned long long> raw(STAT_WORDS);
  LSR_HIP(hipMemcpyAsync(raw.data(), j->stats, sizeof(unsigned long long) * STAT_WORDS,
                         hipMemcpyDeviceToHost, j->stream));
  LSR_HIP(hipStreamSynchronize(j->stream));
  unsigned long long dev[STAT_COUNTERS] = {};
  for (int c = 0; c < STAT_COUNTERS; ++c)
    for (int q = 0; q < STAT_SLOTS; ++q) dev[c] += raw[stat_index(c, q)];
  int64_t all[LSR_CNT_COUNT];
  all[LSR_CNT_NODE_UPDATES] = (int64_t)dev[0];
  all[LSR_CNT_FALLBACKS] = (int64_t)dev[1];
  all[LSR_CNT_FRAME0] = (int64_t)dev[2];
  all[LSR_CNT_REINITS] = j->n_reinits;
  all[LSR_CNT_GBAR] = (int64_t)dev[4];
  all[LSR_CNT_INTERFACE] = (int64_t)dev[5];
  all[LSR_CNT_STEPS] = j->n_steps;
  for (int32_t q = 0; q < n && q < LSR_CNT_COUNT; ++q) out[q] = all[q];
  return LSR_OK;
}

lsr_status lsr_set_launch(lsr_job* j, int32_t lanes, int32_t blocks_per_cu) {
  if (!j) return fail(LSR_E_INVALID, "job is NULL");
  if (j->in_batch) return fail(LSR_E_STATE, "job belongs to a batch");
  const int fp = j->grid.dim == 3 ? 4 : 2;
  if (lanes != 1 && lanes != fp)
    return fail(LSR_E_INVALID, "lanes must be 1 or the foot points per node");
  if (blocks_per_cu < 1 || blocks_per_cu > 64) return fail(LSR_E_INVALID, "blocks_per_cu must be in 1..64");
  j->lanes = lanes;
  j->blocks_per_cu = blocks_per_cu;
  set_list_blocks(j);
  return LSR_OK;
}

lsr_status lsr_set_graphs(lsr_job* j, int32_t enable) {
  if (!j) return fail(LSR_E_INVALID, "job is NULL");
  LSR_HIP(hipStreamSynchronize(j->stream));
  j->graphs.clear();
  j->graphs.enabled = enable != 0;
  return LSR_OK;
}

lsr_status lsr_profile_enable(lsr_job* j, int32_t enable, int32_t max_launches) {
  if (!j) return fail(LSR_E_INVALID, "job is NULL");
  if (enable && max_launches < 1) return fail(LSR_E_INVALID, "max_launches must be >= 1");
  LSR_HIP(hipStreamSynchronize(j->stream));
  for (hipEvent_t e : j->prof_ev) LSR_HIP(hipEventDestroy(e));
  j->prof_ev.clear();
  j->prof_used = 0;
  j->prof_on = false;
  if (!enable) return LSR_OK;
  j->prof_ev.resize(2 * (size_t)max_launches, nullptr);
  for (auto& e : j->prof_ev) LSR_HIP(hipEventCreate(&e));
  j->prof_on = true;
  return LSR_OK;
}

lsr_status lsr_profile_read(lsr_job* j, double* total_ms, int64_t* launches) {
  if (!j || !total_ms || !launches) return fail(LSR_E_INVALID, "NULL argument");
  LSR_HIP(hipStreamSynchronize(j->stream));
  double tot = 0.0;
  for (int q = 0; q < j->prof_used; ++q) {
    float ms = 0.0f;
    LSR_HIP(hipEventElapsedTime(&ms, j->prof_ev[2 * q], j->prof_ev[2 * q + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *launches = j->prof_used;
  return LSR_OK;
}

lsr_status lsr_destroy(lsr_job* j) {
  if (!j) return LSR_OK;
  if (j->in_batch) return fail(LSR_E_STATE, "remove the job from its batch first");
  hipError_t e = hipStreamSynchronize(j->stream);
  for (hipEvent_t ev : j->prof_ev) (void)hipEventDestroy(ev);
  j->graphs.clear();
  delete j;
  if (e != hipSuccess) return fail(LSR_E_DEVICE, hipGetErrorString(e));
  return LSR_OK;
}

}  // extern "C"

// Batched execution: filled in by lsr_batch.hip.
