// Batched execution of independent jobs (include/lsr.h, lsr_batch_*) and the
// launch-shape autotuner.
//
// A batch step launches each kernel of the step once for all jobs: the
// per-job arguments come from packed tables that the host fills with the
// same plan_* functions the single-job path uses (lsr_job.h), so every job
// goes through the same buffers, counters and per-node arithmetic as it would
// alone.  Tables for a group of steps are written to pinned host memory and
// copied to the caller's device workspace with one transfer per group.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "lsr_job.h"

using namespace lsr;

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Launch {
  int kind;  // 0 step, 1 Gbar scan, 2 fix, 3 iteration, 4 final, 5 energy of one p = 2 job
  size_t off;
  int n;
  int interp;    // kind 0 only
  int group;     // cache group (see cache_groups)
  lsr_job* job = nullptr;  // kind 5: the job, and the phi buffer its next step reads
  int phi = 0;
};

}  // namespace

struct lsr_batch {
  std::vector<lsr_job*> jobs;
  std::vector<double> dt;
  std::vector<int32_t> interp;
  int max_jobs, max_iters;
  hipStream_t stream;
  int dim;                           // 0 until the first job joins
  bool fp64;
  char* ws;
  size_t ws_bytes;
  int32_t* scratch_cnt;              // 2 ints per job for dry runs
  unsigned long long* scratch_stats;
  size_t table_off, table_bytes;
  int group_steps;
  char* host;
  size_t host_bytes;
  hipEvent_t copy_done;
  bool copy_pending;
  int lanes, bpc, ncu;
  unsigned blocks;
  lsr::GraphCache graphs;  // recorded group launch sequences
  // streams of the cache groups besides the batch's own (group g runs on
  // stream g % n_streams, 0 the batch's), forked and joined back per call
  static constexpr int kMaxStreams = 2;
  hipStream_t side[kMaxStreams - 1];
  hipEvent_t fork_ev, join_ev[kMaxStreams - 1];
  int n_streams;
};

namespace {

// Upper bound of the tables of one group: per step and cache group two step
// tables (one per interpolator) and at most one reinitialisation per job
// (Gbar scan, fix, max_iters iteration tables, final), each table 256-byte
// aligned; the double-precision argument structs bound the single-precision
// ones.  There are at most as many cache groups (see cache_groups) as jobs,
// so the alignment padding is counted per job.
size_t group_table_bytes(int n_jobs, int group_steps, int max_iters) {
  const size_t n = (size_t)n_jobs, a = 255;
  const size_t per_step = n * (sizeof(SLArgs<double>) + sizeof(GbarArgs<double>) +
                               (size_t)(max_iters + 1) * sizeof(RArgs<double>) +
                               sizeof(FinArgs<double>)) +
                          n * (size_t)(2 + 3 + max_iters) * a;
  return per_step * (size_t)group_steps + a;
}

// Jobs whose state is stepped together in one launch should fit the device's
// last-level cache (256 MB Infinity Cache on MI355X) with room to spare: a
// step then finds the group's phi and (grad d, d) where the previous step left
// them.  Larger launches lose that reuse and run up to 1.5x slower per node.
constexpr size_t kCacheGroupBytes = (size_t)192 << 20;

size_t step_footprint(const lsr_job* j) {
  return (size_t)j->dg.N * 6u * (j->fp64 ? 8u : 4u);  // phi A, B and (grad d, d)
}

// Consecutive members packed greedily into groups of at most
// kCacheGroupBytes (a larger job forms a group of its own).
std::vector<std::pair<int, int>> cache_groups(const lsr_batch* b);

unsigned batch_blocks(int ncu, int bpc) {
  unsigned b = (unsigned)(ncu * bpc);
  return (b + 7) / 8 * 8;
}

template <typename T>
struct Builder {
  lsr_batch* b;
  size_t off = 0;
  int group = 0;
  std::vector<Launch> launches;
  template <typename A>
  A* take(int n) {
    off = align256(off);
    A* p = (A*)(b->host + off);
    off += sizeof(A) * (size_t)n;
    return p;
  }
};

// Tables and launches of `steps` steps of the members q0 .. q1-1.
template <typename T>
lsr_status build_group(lsr_batch* b, int q0, int q1, int steps, Builder<T>& B) {
  for (int s = 0; s < steps; ++s) {
    // p = 2 members: E_2 of the phi this step reads, left on the device for
    // the step kernel (Algorithm 1, step 2)
    for (int q = q0; q < q1; ++q) {
      lsr_job* j = b->jobs[q];
      if (j->prm.p != 1.0) {
        Launch L{5, 0, 1, 0, B.group};
        L.job = j;
        L.phi = j->cur;
        B.launches.push_back(L);
      }
    }
    // one step table and launch per interpolator
    for (int itp = 0; itp < 2; ++itp) {
      int m = 0;
      for (int q = q0; q < q1; ++q) m += b->interp[q] == itp;
      if (!m) continue;
      size_t o = align256(B.off);
      SLArgs<T>* tab = B.template take<SLArgs<T>>(m);
      m = 0;
      for (int q = q0; q < q1; ++q) {
        if (b->interp[q] != itp) continue;
        lsr_job* j = b->jobs[q];
        tab[m++] = plan_step<T>(j, step_const<T>(j, b->dt[q]));
      }
      B.launches.push_back({0, o, m, itp, B.group});
    }
    std::vector<int> due;
    for (int q = q0; q < q1; ++q)
      if (reinit_due(b->jobs[q])) due.push_back(q);
    if (due.empty()) continue;
    const int nd = (int)due.size();
    std::vector<ReinitPlan<T>> plans;
    int max_it = 0;
    for (int q : due) {
      lsr_job* j = b->jobs[q];
      plans.push_back(plan_reinit<T>(j));
      max_it = std::max(max_it, plans.back().iters);
    }
    size_t od = align256(B.off);
    GbarArgs<T>* gb = B.template take<GbarArgs<T>>(nd);
    for (int q = 0; q < nd; ++q) gb[q] = plans[q].gb;
    B.launches.push_back({1, od, nd, 0, B.group});
    size_t of = align256(B.off);
    RArgs<T>* fix = B.template take<RArgs<T>>(nd);
    for (int q = 0; q < nd; ++q) fix[q] = plans[q].fix;
    B.launches.push_back({2, of, nd, 0, B.group});
    for (int it = 0; it < max_it; ++it) {
      size_t oi = align256(B.off);
      RArgs<T>* itab = B.template take<RArgs<T>>(nd);
      int m = 0;
      for (int q = 0; q < nd; ++q)
        if (it < plans[q].iters) itab[m++] = plans[q].iter[it % 2];
      B.launches.push_back({3, oi, m, 0, B.group});
    }
    size_t on = align256(B.off);
    FinArgs<T>* fin = B.template take<FinArgs<T>>(nd);
    for (int q = 0; q < nd; ++q) fin[q] = plans[q].fin;
    B.launches.push_back({4, on, nd, 0, B.group});
  }
  if (B.off > b->table_bytes) return fail(LSR_E_NOMEM, "batch table workspace too small");
  return LSR_OK;
}

// The cache groups hold different jobs, so their launches are independent:
// group g runs on stream g % n (stream 0 the batch's own, the others forked
// from it and joined back into it), so that one group's kernels fill the
// gaps between another's.
template <typename T>
hipError_t issue(lsr_batch* b, const Builder<T>& B) {
  char* dev = b->ws + b->table_off;
  hipError_t e = hipSuccess;
  const int ns = std::min(b->n_streams, B.group);
  // side[] and join_ev[] hold kMaxStreams - 1 entries; every index below is
  // q - 1 or sq - 1 with q, sq < ns
  if (ns > lsr_batch::kMaxStreams) return hipErrorInvalidValue;
  if (ns > 1) e = hipEventRecord(b->fork_ev, b->stream);
  for (int q = 1; q < ns && e == hipSuccess; ++q) e = hipStreamWaitEvent(b->side[q - 1], b->fork_ev, 0);
  for (const Launch& L : B.launches) {
    if (e != hipSuccess) break;
    if (L.group < 0) return hipErrorInvalidValue;
    const int sq = ns > 1 ? L.group % ns : 0;
    hipStream_t s = sq ? b->side[sq - 1] : b->stream;
    switch (L.kind) {
      case 0:
        e = launch_sl_step_batch<T>(b->dim, L.interp, b->lanes, (const SLArgs<T>*)(dev + L.off), L.n,
                                    b->blocks, s);
        break;
      case 1:
        e = launch_grid_list_batch<T>(b->dim, (const GbarArgs<T>*)(dev + L.off), L.n, b->blocks, s,
                                      true);
        break;
      case 2:
        e = launch_reinit_fix_batch<T>(b->dim, (const RArgs<T>*)(dev + L.off), L.n, b->blocks, s);
        break;
      case 3:
        if (L.n > 0)
          e = launch_reinit_iter_batch<T>(b->dim, (const RArgs<T>*)(dev + L.off), L.n, b->blocks, s);
        break;
      case 4:
        e = launch_reinit_final_batch<T>((const FinArgs<T>*)(dev + L.off), L.n, b->blocks, s);
        break;
      case 5: {
        lsr_job* j = L.job;
        e = launch_energy_front<T>(b->dim, j->dg, (const T*)j->phi[L.phi], j->d64, j->prm.p,
                                   ENERGY_R, j->sgn, j->energy_buf, nullptr, s);
        break;
      }
    }
  }
  for (int q = 1; q < ns; ++q) {
    hipError_t r = hipEventRecord(b->join_ev[q - 1], b->side[q - 1]);
    if (r == hipSuccess) r = hipStreamWaitEvent(b->stream, b->join_ev[q - 1], 0);
    if (e == hipSuccess) e = r;
  }
  return e;
}

// A group's launches read their arguments from the tables at fixed offsets
// of the workspace, so the launch sequence is fixed by the kinds, offsets and
// job counts of its launches and the launch shape: groups with the same
// sequence replay one recorded graph after their tables are copied.
template <typename T>
std::vector<int64_t> group_key(const lsr_batch* b, const Builder<T>& B) {
  std::vector<int64_t> k = {(int64_t)sizeof(T), b->dim, b->lanes, (int64_t)b->blocks,
                            b->n_streams};
  k.reserve(5 + 5 * B.launches.size());
  for (const Launch& L : B.launches) {
    k.push_back(L.kind);
    k.push_back((int64_t)L.off);
    k.push_back(L.n);
    k.push_back(L.interp);
    k.push_back(L.group);
    if (L.kind == 5) {
      // the energy launch bakes in the job's buffers and sizes, not the job
      // object (a job created where a destroyed one lived may reuse its
      // address with another workspace)
      const lsr_job* j = L.job;
      int64_t pb;
      memcpy(&pb, &j->prm.p, sizeof pb);
      k.push_back((int64_t)(intptr_t)j->phi[L.phi]);
      k.push_back((int64_t)(intptr_t)j->d64);
      k.push_back((int64_t)(intptr_t)j->energy_buf);
      k.push_back((int64_t)(intptr_t)j->sgn);
      k.push_back((int64_t)j->dg.N);
      k.push_back((int64_t)j->dg.n0 << 40 | (int64_t)j->dg.n1 << 20 | (int64_t)j->dg.n2);
      k.push_back(pb);
    }
  }
  return k;
}

template <typename T>
lsr_status launch_group(lsr_batch* b, const Builder<T>& B) {
  hipStream_t s = b->stream;
  if (b->graphs.enabled && s != nullptr) {
    const std::vector<int64_t> key = group_key<T>(b, B);
    GraphCache::Entry* g = b->graphs.find(key);
    if (g) {
      LSR_HIP(b->graphs.replay(*g, s));
      return LSR_OK;
    }
    if (b->graphs.seen_before(key)) {
      bool launched = false;
      hipError_t e =
          b->graphs.capture_and_launch(s, key, [&]() { return issue<T>(b, B); }, &launched);
      if (e == hipSuccess) return LSR_OK;
      if (launched) LSR_HIP(e);
      (void)hipGetLastError();
      (void)fail(LSR_OK, "batch graph not recorded (" + b->graphs.failure + "); launching directly");
      b->graphs.enabled = false;  // the stream cannot be captured: launch directly
    }
  }
  LSR_HIP(issue<T>(b, B));
  return LSR_OK;
}

std::vector<std::pair<int, int>> cache_groups(const lsr_batch* b) {
  std::vector<std::pair<int, int>> out;
  const int nj = (int)b->jobs.size();
  int q0 = 0;
  size_t bytes = 0;
  for (int q = 0; q < nj; ++q) {
    const size_t f = step_footprint(b->jobs[q]);
    if (q > q0 && bytes + f > kCacheGroupBytes) {
      out.push_back({q0, q});
      q0 = q;
      bytes = 0;
    }
    bytes += f;
  }
  if (nj > q0) out.push_back({q0, nj});
  return out;
}

// Tables must be in place before the launches: wait until the previous
// group's copy has left the pinned buffer, fill it, copy, launch.
template <typename T>
lsr_status run_group(lsr_batch* b, int steps) {
  if (b->jobs.empty()) return LSR_OK;
  if (b->copy_pending) {
    LSR_HIP(hipEventSynchronize(b->copy_done));
    b->copy_pending = false;
  }
  Builder<T> B;
  B.b = b;
  for (const auto& g : cache_groups(b)) {
    lsr_status st = build_group<T>(b, g.first, g.second, steps, B);
    if (st != LSR_OK) return st;
    B.group += 1;
  }
  LSR_HIP(hipMemcpyAsync(b->ws + b->table_off, b->host, B.off, hipMemcpyHostToDevice, b->stream));
  LSR_HIP(hipEventRecord(b->copy_done, b->stream));
  b->copy_pending = true;
  return launch_group<T>(b, B);
}

struct SavedState {
  int cur, cur_list, ring;
  int64_t step_index, n_steps;
};

SavedState save(const lsr_job* j) {
  return {j->cur, j->cur_list, j->ring, j->step_index, j->n_steps};
}

void restore(lsr_job* j, const SavedState& s) {
  j->cur = s.cur;
  j->cur_list = s.cur_list;
  j->ring = s.ring;
  j->step_index = s.step_index;
  j->n_steps = s.n_steps;
}

// Time the next step kernel under each candidate launch shape without
// changing the jobs: a dry step writes where the real one will (B, the next
// list), its list counters and statistics go to scratch.
template <typename T>
lsr_status tune(lsr_batch* b, int* best_lanes, int* best_bpc, double* best_ms) {
  const int nj = (int)b->jobs.size();
  if (b->copy_pending) {
    LSR_HIP(hipEventSynchronize(b->copy_done));
    b->copy_pending = false;
  }
  // the next step's tables, one per cache group and interpolator (as the
  // step launches them), with list counters and statistics redirected to
  // scratch
  struct Tab {
    size_t off;
    int n, interp;
  };
  std::vector<Tab> tabs;
  size_t top = 0;
  for (const auto& g : cache_groups(b)) {
    for (int itp = 0; itp < 2; ++itp) {
      top = align256(top);
      SLArgs<T>* tab = (SLArgs<T>*)(b->host + top);
      int m = 0;
      for (int q = g.first; q < g.second; ++q) {
        if (b->interp[q] != itp) continue;
        lsr_job* j = b->jobs[q];
        SavedState sv = save(j);
        SLArgs<T> a = plan_step<T>(j, step_const<T>(j, b->dt[q]));
        restore(j, sv);
        a.cnt_out = b->scratch_cnt + 2 * q;
        a.stats = b->scratch_stats;
        a.sgn = nullptr;  // a trial: the sign words stay those of phi^n
        tab[m++] = a;
      }
      if (m) tabs.push_back({top, m, itp});
      top += sizeof(SLArgs<T>) * (size_t)m;
    }
  }
  hipStream_t s = b->stream;
  char* dev = b->ws + b->table_off;
  LSR_HIP(hipMemcpyAsync(dev, b->host, top, hipMemcpyHostToDevice, s));
  // p = 2 members: the energy their next step will read
  for (lsr_job* j : b->jobs)
    if (j->prm.p != 1.0)
      LSR_HIP(energy_now<T>(j, j->prm.p, ENERGY_R, j->energy_buf, nullptr, s));
  hipEvent_t e0, e1;
  LSR_HIP(hipEventCreate(&e0));
  LSR_HIP(hipEventCreate(&e1));
  const int fp = b->dim == 3 ? 4 : 2;
  const int lanes_c[2] = {1, fp};
  const int bpc_c[3] = {2, 4, 8};  // 8 and more: every block resident
  double best = 1e30;
  for (int li = 0; li < 2; ++li) {
    for (int bi = 0; bi < 3; ++bi) {
      const unsigned blocks = batch_blocks(b->ncu, bpc_c[bi]);
      float tmin = 1e30f;
      for (int rep = 0; rep < 4; ++rep) {
        LSR_HIP(launch_fill_u32((uint32_t*)b->scratch_cnt, 0u, 2 * (uint64_t)nj, s));
        LSR_HIP(hipEventRecord(e0, s));
        for (const Tab& t : tabs)
          LSR_HIP(launch_sl_step_batch<T>(b->dim, t.interp, lanes_c[li],
                                          (const SLArgs<T>*)(dev + t.off), t.n, blocks, s));
        LSR_HIP(hipEventRecord(e1, s));
        LSR_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        LSR_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) tmin = std::min(tmin, ms);  // first run warms up
      }
      if (tmin < best) {
        best = tmin;
        *best_lanes = lanes_c[li];
        *best_bpc = bpc_c[bi];
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *best_ms = best;
  return LSR_OK;
}

// Tuned launch shapes, kept for the process: a batch whose signature (dimension,
// precision, jobs per interpolator, total grid nodes to the next power of
// two) was tuned before reuses the shape without timing again.
struct TuneEntry {
  int64_t key[5];
  int lanes, bpc;
  double ms;
};

std::mutex g_tune_mutex;
std::vector<TuneEntry> g_tune_cache;
std::string g_tune_path;  // file that keeps the choices across processes ("" = none)

// One line per choice: the five key fields, lanes, blocks per CU, time in ms.
bool parse_tune_line(const char* line, TuneEntry* e) {
  long long k[5];
  int lanes, bpc;
  double ms;
  if (sscanf(line, "%lld %lld %lld %lld %lld %d %d %lf", &k[0], &k[1], &k[2], &k[3], &k[4],
             &lanes, &bpc, &ms) != 8)
    return false;
  if (lanes < 1 || bpc < 1 || bpc > 64 || !(ms >= 0.0)) return false;
  for (int q = 0; q < 5; ++q) e->key[q] = k[q];
  e->lanes = lanes;
  e->bpc = bpc;
  e->ms = ms;
  return true;
}

void tune_key(const lsr_batch* b, int64_t key[5]) {
  int64_t nq = 0, nw = 0, nodes = 0;
  for (size_t q = 0; q < b->jobs.size(); ++q) {
    (b->interp[q] == LSR_Q1 ? nq : nw) += 1;
    nodes += (int64_t)b->jobs[q]->dg.N;
  }
  int64_t p2 = 1;
  while (p2 < nodes) p2 <<= 1;
  key[0] = b->dim;
  key[1] = b->fp64 ? 1 : 0;
  key[2] = nq;
  key[3] = nw;
  key[4] = p2;
}

}  // namespace

// Make `waiter` wait for the work queued on `signaller` so far (no host sync).
hipError_t order_after(hipStream_t waiter, hipStream_t signaller) {
  if (waiter == signaller) return hipSuccess;
  hipEvent_t ev;
  hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e != hipSuccess) return e;
  e = hipEventRecord(ev, signaller);
  if (e == hipSuccess) e = hipStreamWaitEvent(waiter, ev, 0);
  hipError_t e2 = hipEventDestroy(ev);
  return e != hipSuccess ? e : e2;
}

extern "C" {

lsr_status lsr_batch_workspace_bytes(int32_t max_jobs, int32_t group_steps, int32_t max_reinit_iters,
                                     size_t* bytes) {
  if (max_jobs < 1 || group_steps < 1 || max_reinit_iters < 0 || !bytes)
    return fail(LSR_E_INVALID, "need max_jobs >= 1, group_steps >= 1, max_reinit_iters >= 0");
  size_t tot = align256(8 * (size_t)max_jobs) + align256(8 * STAT_WORDS);
  tot += group_table_bytes(max_jobs, group_steps, max_reinit_iters);
  *bytes = tot;
  return LSR_OK;
}

lsr_status lsr_batch_create(int32_t max_jobs, int32_t group_steps, int32_t max_reinit_iters,
                            void* dev_workspace, size_t ws_bytes, void* hip_stream,
                            lsr_batch** out) {
  if (!out || !dev_workspace) return fail(LSR_E_INVALID, "NULL argument");
  if (((uintptr_t)dev_workspace) & 255) return fail(LSR_E_INVALID, "workspace must be 256-byte aligned");
  size_t need = 0;
  lsr_status st = lsr_batch_workspace_bytes(max_jobs, group_steps, max_reinit_iters, &need);
  if (st != LSR_OK) return st;
  if (ws_bytes < need) return fail(LSR_E_NOMEM, "batch workspace too small");
  int dev = 0, ncu = 0;
  LSR_HIP(hipGetDevice(&dev));
  LSR_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  lsr_batch* b = new (std::nothrow) lsr_batch();
  if (!b) return fail(LSR_E_NOMEM, "host allocation failed");
  b->max_jobs = max_jobs;
  b->max_iters = max_reinit_iters;
  b->stream = (hipStream_t)hip_stream;
  b->dim = 0;
  b->fp64 = false;
  b->ws = (char*)dev_workspace;
  b->ws_bytes = ws_bytes;
  size_t off = 0;
  b->scratch_cnt = (int32_t*)(b->ws + off);
  off = align256(off + 8 * (size_t)max_jobs);
  b->scratch_stats = (unsigned long long*)(b->ws + off);
  off = align256(off + 8 * STAT_WORDS);
  b->table_off = off;
  b->table_bytes = ws_bytes - off;
  b->group_steps = group_steps;
  b->host_bytes = group_table_bytes(max_jobs, group_steps, max_reinit_iters);
  b->copy_pending = false;
  b->ncu = ncu > 0 ? ncu : 256;
  b->lanes = 0;
  b->bpc = 8;
  b->blocks = batch_blocks(b->ncu, b->bpc);
  hipError_t e = hipHostMalloc((void**)&b->host, b->host_bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    delete b;
    return fail(LSR_E_DEVICE, std::string("hipHostMalloc: ") + hipGetErrorString(e));
  }
  b->fork_ev = b->copy_done = nullptr;
  for (int q = 0; q < lsr_batch::kMaxStreams - 1; ++q) {
    b->side[q] = nullptr;
    b->join_ev[q] = nullptr;
  }
  b->n_streams = 2;
  e = hipEventCreateWithFlags(&b->copy_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming);
  for (int q = 0; q < lsr_batch::kMaxStreams - 1 && e == hipSuccess; ++q) {
    e = hipEventCreateWithFlags(&b->join_ev[q], hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->side[q], hipStreamNonBlocking);
  }
  if (e != hipSuccess) {
    for (int q = 0; q < lsr_batch::kMaxStreams - 1; ++q) {
      if (b->side[q]) (void)hipStreamDestroy(b->side[q]);
      if (b->join_ev[q]) (void)hipEventDestroy(b->join_ev[q]);
    }
    for (hipEvent_t ev : {b->copy_done, b->fork_ev})
      if (ev) (void)hipEventDestroy(ev);
    (void)hipHostFree(b->host);
    delete b;
    return fail(LSR_E_DEVICE, hipGetErrorString(e));
  }
  *out = b;
  return LSR_OK;
}

lsr_status lsr_batch_add(lsr_batch* b, lsr_job* j, double dt, lsr_interp interp) {
  if (!b || !j) return fail(LSR_E_INVALID, "NULL argument");
  if (!j->has_d || !j->has_phi) return fail(LSR_E_STATE, "the job needs a distance field and phi");
  if (j->in_batch) return fail(LSR_E_STATE, "the job is already in a batch");
  if ((int)b->jobs.size() >= b->max_jobs) return fail(LSR_E_NOMEM, "the batch is full");
  if (j->prm.reinit_iters > b->max_iters) return fail(LSR_E_NOMEM, "reinit_iters above the batch's maximum");
  if (b->dim && (j->grid.dim != b->dim || j->fp64 != b->fp64))
    return fail(LSR_E_UNSUPPORTED, "a batch needs one dimension and one precision");
  if (!(dt > 0.0) || !isfinite(dt)) return fail(LSR_E_INVALID, "dt must be > 0");
  if (interp != LSR_Q1 && interp != LSR_WENO) return fail(LSR_E_INVALID, "unknown interpolator");
  LSR_HIP(order_after(b->stream, j->stream));
  if (!b->dim) {
    b->dim = j->grid.dim;
    b->fp64 = j->fp64;
    if (!b->lanes) b->lanes = j->lanes;
  }
  j->in_batch = true;
  j->own_stream = j->stream;
  j->stream = b->stream;
  b->jobs.push_back(j);
  b->dt.push_back(dt);
  b->interp.push_back((int32_t)interp);
  return LSR_OK;
}

lsr_status lsr_batch_remove(lsr_batch* b, lsr_job* j) {
  if (!b || !j) return fail(LSR_E_INVALID, "NULL argument");
  auto it = std::find(b->jobs.begin(), b->jobs.end(), j);
  if (it == b->jobs.end()) return fail(LSR_E_INVALID, "the job is not in this batch");
  const size_t q = (size_t)(it - b->jobs.begin());
  LSR_HIP(order_after(j->own_stream, b->stream));
  j->stream = j->own_stream;
  j->in_batch = false;
  b->jobs.erase(b->jobs.begin() + q);
  b->dt.erase(b->dt.begin() + q);
  b->interp.erase(b->interp.begin() + q);
  return LSR_OK;
}

lsr_status lsr_batch_step(lsr_batch* b, int32_t n_steps) {
  if (!b) return fail(LSR_E_INVALID, "batch is NULL");
  if (n_steps < 0) return fail(LSR_E_INVALID, "n_steps must be >= 0");
  while (n_steps > 0) {
    const int g = std::min<int>(n_steps, b->group_steps);
    lsr_status st = b->fp64 ? run_group<double>(b, g) : run_group<float>(b, g);
    if (st != LSR_OK) return st;
    n_steps -= g;
  }
  return LSR_OK;
}

lsr_status lsr_batch_set_launch(lsr_batch* b, int32_t lanes, int32_t blocks_per_cu) {
  if (!b) return fail(LSR_E_INVALID, "batch is NULL");
  if (!b->dim) return fail(LSR_E_STATE, "the batch has no job yet");
  const int fp = b->dim == 3 ? 4 : 2;
  if (lanes != 1 && lanes != fp) return fail(LSR_E_INVALID, "lanes must be 1 or the foot points per node");
  if (blocks_per_cu < 1 || blocks_per_cu > 64) return fail(LSR_E_INVALID, "blocks_per_cu must be in 1..64");
  b->lanes = lanes;
  b->bpc = blocks_per_cu;
  b->blocks = batch_blocks(b->ncu, b->bpc);
  return LSR_OK;
}

lsr_status lsr_batch_set_streams(lsr_batch* b, int32_t n_streams) {
  if (!b) return fail(LSR_E_INVALID, "batch is NULL");
  if (n_streams < 1 || n_streams > lsr_batch::kMaxStreams)
    return fail(LSR_E_INVALID, "n_streams must be 1 or 2");
  LSR_HIP(hipStreamSynchronize(b->stream));
  b->n_streams = n_streams;
  return LSR_OK;
}

lsr_status lsr_batch_set_graphs(lsr_batch* b, int32_t enable) {
  if (!b) return fail(LSR_E_INVALID, "batch is NULL");
  LSR_HIP(hipStreamSynchronize(b->stream));
  b->graphs.clear();
  b->graphs.enabled = enable != 0;
  return LSR_OK;
}

lsr_status lsr_graph_counts(lsr_job* j, lsr_batch* b, int64_t* captured, int64_t* replayed) {
  if ((j == nullptr) == (b == nullptr)) return fail(LSR_E_INVALID, "pass exactly one of job, batch");
  if (!captured || !replayed) return fail(LSR_E_INVALID, "NULL argument");
  const GraphCache& g = j ? j->graphs : b->graphs;
  *captured = g.n_captured;
  *replayed = g.n_replayed;
  return LSR_OK;
}

lsr_status lsr_batch_tune(lsr_batch* b, int32_t* lanes, int32_t* blocks_per_cu, double* ms) {
  if (!b) return fail(LSR_E_INVALID, "batch is NULL");
  if (b->jobs.empty()) return fail(LSR_E_STATE, "the batch has no job");
  int bl = b->lanes, bb = b->bpc;
  double t = 0.0;
  int64_t key[5];
  tune_key(b, key);
  bool cached = false;
  {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    for (const TuneEntry& e : g_tune_cache)
      if (std::equal(key, key + 5, e.key)) {
        bl = e.lanes;
        bb = e.bpc;
        t = e.ms;
        cached = true;
        break;
      }
  }
  if (!cached) {
    lsr_status st = b->fp64 ? tune<double>(b, &bl, &bb, &t) : tune<float>(b, &bl, &bb, &t);
    if (st != LSR_OK) return st;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    TuneEntry e;
    std::copy(key, key + 5, e.key);
    e.lanes = bl;
    e.bpc = bb;
    e.ms = t;
    g_tune_cache.push_back(e);
    if (!g_tune_path.empty()) {
      FILE* f = fopen(g_tune_path.c_str(), "a");
      if (f) {
        fprintf(f, "%lld %lld %lld %lld %lld %d %d %.17g\n", (long long)key[0], (long long)key[1],
                (long long)key[2], (long long)key[3], (long long)key[4], bl, bb, t);
        fclose(f);
      }
    }
  }
  lsr_status st = lsr_batch_set_launch(b, bl, bb);
  if (st != LSR_OK) return st;
  if (lanes) *lanes = bl;
  if (blocks_per_cu) *blocks_per_cu = bb;
  if (ms) *ms = t;
  return LSR_OK;
}

lsr_status lsr_set_tune_cache(const char* path) {
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  if (!path || !*path) {
    g_tune_path.clear();
    return LSR_OK;
  }
  std::vector<TuneEntry> got;
  if (FILE* f = fopen(path, "r")) {
    char line[512];
    int no = 0;
    bool bad = false;
    while (fgets(line, sizeof line, f)) {
      ++no;
      if (line[0] == '#' || line[0] == '\n') continue;
      TuneEntry e;
      if (!parse_tune_line(line, &e)) {
        bad = true;
        break;
      }
      got.push_back(e);
    }
    fclose(f);
    if (bad) return fail(LSR_E_INVALID, std::string(path) + ": malformed line " + std::to_string(no));
  }
  // entries already known in this process keep their values
  for (const TuneEntry& e : got) {
    bool known = false;
    for (const TuneEntry& c : g_tune_cache) known = known || std::equal(e.key, e.key + 5, c.key);
    if (!known) g_tune_cache.push_back(e);
  }
  g_tune_path = path;
  return LSR_OK;
}

lsr_status lsr_batch_destroy(lsr_batch* b) {
  if (!b) return LSR_OK;
  while (!b->jobs.empty()) {
    lsr_status st = lsr_batch_remove(b, b->jobs.back());
    if (st != LSR_OK) return st;
  }
  hipError_t e = hipStreamSynchronize(b->stream);
  b->graphs.clear();
  for (int q = 0; q < lsr_batch::kMaxStreams - 1; ++q) {
    (void)hipStreamDestroy(b->side[q]);
    (void)hipEventDestroy(b->join_ev[q]);
  }
  (void)hipEventDestroy(b->fork_ev);
  (void)hipEventDestroy(b->copy_done);
  (void)hipHostFree(b->host);
  delete b;
  if (e != hipSuccess) return fail(LSR_E_DEVICE, hipGetErrorString(e));
  return LSR_OK;
}

}  // extern "C"
