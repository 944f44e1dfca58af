// Host-side job state shared by the single-job entry points (lsr_api.hip) and
// the batched ones (lsr_batch.hip).  The plan_* functions fill the kernel
// arguments of the next launch from the job state and advance that state
// without launching anything, so a single job and a batch of jobs drive the
// same kernels through the same sequence of buffers and counters.
#pragma once

#include <math.h>

#include <string>
#include <vector>

#include "../../include/lsr.h"
#include "lsr_graph.h"
#include "lsr_internal.h"

namespace lsr {

lsr_status fail(lsr_status st, const std::string& msg);

#define LSR_HIP(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return ::lsr::fail(LSR_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

struct Layout {
  size_t phi0, phi1, dp, d64, list0, list1, listM, mflags, cnt, stats;
  size_t ccnt0, ccnt1;  // entries per chunk of the two band lists
  size_t scnt, soff;    // members per grid slot and their prefix (list builds)
  size_t smark;         // grid slots marked for the Gbar scan
  size_t dmark;         // distance-kernel bricks marked for the approximate distance
  size_t sgn;           // sign words of phi
  int64_t list_cap;     // entries of a band-list buffer: chunks and grid slots
  size_t pts_raw, pts, pt_bin, bin_count, bin_start, bin_fill, occ, scan_tmp, geo, sup, sgeo;
  size_t energy;  // energy partial sums and result
  size_t nn;      // nearest-neighbour distances of a cloud sample
  int64_t max_occ, max_sup;
  size_t total;
  int64_t nbins;  // bin ids at the finer width, super-bin padding included
};

}  // namespace lsr

struct lsr_job {
  lsr_grid grid;
  lsr_params prm;
  bool fp64;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  lsr::Layout L;
  int64_t max_points;
  lsr::DevGrid dg;
  lsr::BinGeom bg, bg_fine;  // cloud bins of the standard and the finer width
  void* phi[2];
  void* dp;
  double* d64;
  uint32_t* list[2];     // band lists, chunked (LCHUNK entries per chunk)
  int32_t* ccnt[2];      // their entries per chunk
  int32_t* scnt;         // members per grid slot of a list build
  int32_t* soff;         // and their exclusive prefix
  uint8_t* smark;        // slots a Gbar build scans (clear between builds)
  uint32_t* listM;
  uint8_t* mflags;  // reinitialisation flags; scratch of the initial-data passes
  uint8_t* dmark;
  uint32_t* sgn;    // sign words of the current phi (lsr_device.h)
  int32_t* cnt;  // [0..2] list-count ring (chunks of a band list, entries of Gbar),
                 // [3] flag, [4] extract count, [5] occupied bins, [6] bins a
                 // cloud's points occupy (density check), [7] occupied
                 // super-bins, [11]
                 // sample-index flag of lsr_cloud_spacing, [12..15] change
                 // flags of the convergence passes
  unsigned long long* stats;
  double* pts_raw;
  double* pts;
  int32_t* pt_bin;
  int32_t* bin_count;
  int32_t* bin_start;
  int32_t* bin_fill;
  uint32_t* occ;
  int32_t* scan_tmp;
  double* geo;      // bin frames, GEO doubles per occupied bin
  int64_t max_occ;  // room for bin frames
  int2* sup;        // occupied super-bins: their runs in the occupied list
  double* sgeo;     // super-bin frames
  int64_t max_sup;  // room for super-bins
  double* energy_buf;  // ENERGY_BLOCKS partial sums, then E_p (lsr_energy)
  double* nn;          // max_points nearest-neighbour distances, then their mean
  int64_t n_cloud;     // points of the loaded cloud (0: none, or a given d)
  lsr::BinGeom bg_load;  // the bins the loaded cloud is sorted by
  unsigned list_blocks;
  int lanes;         // step kernel: 1 one lane per node, or one per foot point
  int blocks_per_cu; // persistent grid of the list kernels: blocks_per_cu x CUs (multiple of 8)
  int ncu;
  int cur;       // phi buffer holding the current phi
  int cur_list;  // list buffer holding the current band list
  int ring;      // counter slot holding the current list length
  int64_t step_index;
  int64_t n_reinits, n_steps;
  bool has_d, has_phi;
  bool in_batch;            // while in a batch, stream is the batch's stream
  hipStream_t own_stream;   // the job's stream, saved while it is in a batch
  // measurement hook
  bool prof_on;
  int prof_used;
  std::vector<hipEvent_t> prof_ev;
  lsr::GraphCache graphs;  // recorded step sequences (lsr_step)
};

namespace lsr {

template <typename T>
StepConst<T> step_const(const lsr_job* j, double dt) {
  StepConst<T> c;
  const double h = j->grid.h;
  const lsr_params& p = j->prm;
  c.gamma = (T)p.gamma;
  c.beta = (T)p.beta;
  const double gb = p.gamma - p.beta;
  c.inv_gb3 = (T)(1.0 / (gb * gb * gb));
  c.drift = (T)(dt / h);
  c.diff2 = (T)(p.delta * dt / (p.p * h * h));
  c.grad_thr = (T)(p.grad_C * pow(dt, p.grad_alpha));
  c.weno_e = (T)(h * h * h * h);
  c.half_inv_h = (T)(0.5 / h);
  c.inv_h = (T)(1.0 / h);
  c.pm1 = (T)(p.p - 1.0);
  c.inv_E = T(0);
  return c;
}

inline int32_t* ring_slot(lsr_job* j, int k) { return j->cnt + ((j->ring + k) % 3); }

template <typename T>
inline T* phi_buf(lsr_job* j, int b) {
  return (T*)j->phi[b];
}

// E_p of the current phi (Section 3.5) from the sign words, into the
// partial sums and out.
template <typename T>
hipError_t energy_now(lsr_job* j, double p, int R, double* partial, double* out, hipStream_t s) {
  return launch_energy_front<T>(j->grid.dim, j->dg, phi_buf<T>(j, j->cur), j->d64, p, R, j->sgn,
                                partial, out, s);
}

inline bool reinit_due(const lsr_job* j) {
  return j->prm.reinit_every > 0 && j->step_index % j->prm.reinit_every == 0;
}

// Arguments of the next step kernel; advances buffers, list, ring, step index.
template <typename T>
SLArgs<T> plan_step(lsr_job* j, const StepConst<T>& c) {
  SLArgs<T> a;
  a.g = j->dg;
  a.c = c;
  a.dp = (const typename Vec<T>::pack*)j->dp;
  a.stats = j->stats;
  a.Epart = j->prm.p != 1.0 ? j->energy_buf : nullptr;
  a.sgn = j->sgn;
  a.A = phi_buf<T>(j, j->cur);
  a.B = phi_buf<T>(j, 1 - j->cur);
  a.Lin = j->list[j->cur_list];
  a.Lout = j->list[1 - j->cur_list];
  a.ccnt_in = j->ccnt[j->cur_list];
  a.ccnt_out = j->ccnt[1 - j->cur_list];
  a.cnt_in = ring_slot(j, 0);
  a.cnt_out = ring_slot(j, 1);
  j->cur = 1 - j->cur;
  j->cur_list = 1 - j->cur_list;
  j->ring = (j->ring + 1) % 3;
  j->step_index += 1;
  j->n_steps += 1;
  return a;
}

// Arguments of one reinitialisation: Gbar scan, interface fix, iterations
// (iter[it % 2] is the it-th), final cut and compaction.
template <typename T>
struct ReinitPlan {
  GbarArgs<T> gb;
  RArgs<T> fix;
  RArgs<T> iter[2];
  FinArgs<T> fin;
  int iters;
};

template <typename T>
ReinitPlan<T> plan_reinit(lsr_job* j) {
  ReinitPlan<T> r;
  r.gb.g = j->dg;
  r.gb.gamma = (T)j->prm.gamma;
  r.gb.nbr = 1;
  r.gb.smark = j->smark;                // slots of the band list of the step
  r.gb.L = j->list[j->cur_list];
  r.gb.Lccnt = j->ccnt[j->cur_list];
  r.gb.Lcnt = ring_slot(j, 0);
  r.gb.P = phi_buf<T>(j, 1 - j->cur);  // phi^n: the step just taken read it
  r.gb.S = j->list[1 - j->cur_list];   // the step's input list, no longer needed
  r.gb.scnt = j->scnt;
  r.gb.soff = j->soff;
  r.gb.M = j->listM;
  r.gb.cnt_out = ring_slot(j, 1);
  r.gb.ccnt = nullptr;
  j->ring = (j->ring + 1) % 3;

  RArgs<T> ra;
  ra.g = j->dg;
  ra.c = step_const<T>(j, j->grid.h);
  ra.M = j->listM;
  ra.cnt = ring_slot(j, 0);
  ra.flags = j->mflags;
  ra.dtau = (T)j->prm.reinit_dtau;
  ra.floor_ = (T)j->prm.interface_floor;
  ra.stats = j->stats;
  ra.src = phi_buf<T>(j, j->cur);
  ra.dst = phi_buf<T>(j, 1 - j->cur);
  r.fix = ra;
  int w = 1 - j->cur;
  for (int q = 0; q < 2; ++q) {
    r.iter[q] = ra;
    r.iter[q].src = phi_buf<T>(j, w);
    r.iter[q].dst = phi_buf<T>(j, 1 - w);
    w = 1 - w;
  }
  r.iters = j->prm.reinit_iters;
  const int wf = (r.iters % 2 == 0) ? 1 - j->cur : j->cur;
  r.fin.g = j->dg;
  r.fin.gamma = (T)j->prm.gamma;
  r.fin.M = j->listM;
  r.fin.cnt_in = ring_slot(j, 0);
  r.fin.cur = phi_buf<T>(j, wf);
  r.fin.other = phi_buf<T>(j, 1 - wf);
  r.fin.Lout = j->list[j->cur_list];
  r.fin.ccnt_out = j->ccnt[j->cur_list];
  r.fin.cnt_out = ring_slot(j, 1);
  r.fin.sgn = j->sgn;
  j->ring = (j->ring + 1) % 3;
  j->cur = wf;
  j->n_reinits += 1;
  return r;
}

lsr_status run_steps(lsr_job* j, int32_t n_steps, double dt, int interp);
lsr_status start_loop(lsr_job* j, int64_t step0);
// Checks of a grid as lsr_create makes them, and the kernels' view of it.
lsr_status grid_ok(const lsr_grid* g);
DevGrid make_devgrid(const lsr_grid& g);

}  // namespace lsr

// Make `waiter` wait for the work queued on `signaller` so far (no host sync).
hipError_t order_after(hipStream_t waiter, hipStream_t signaller);

namespace lsr {
lsr_status run_reinit(lsr_job* j);

}  // namespace lsr
