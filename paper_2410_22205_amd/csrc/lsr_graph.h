// Recorded launch sequences (HIP graphs) for the step loops of a job and of a
// batch.
//
// A sequence of launches is identified by a key that fixes every kernel
// argument of the sequence (buffer roles, counter slots, table offsets,
// launch shapes, step constants).  The first time a key is seen its launches
// go straight to the stream; the second time they are captured into a graph,
// which is instantiated and launched, and later sequences with the same key
// replay that graph.  The host side then only advances its plan state (the
// same plan_* calls, without launching) so that it stays where direct
// launches would have left it.  Replays run exactly the kernels, arguments
// and order of the direct launches, so results do not depend on whether a
// graph was used.
//
// Kernel timing: launches that a caller wants timed are bracketed by events.
// In a captured sequence these are external event-record nodes on events
// owned by the graph; their times are collected before the graph is launched
// again and when the caller reads the totals.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

namespace lsr {

struct GraphCache {
  struct Entry {
    std::vector<int64_t> key;
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> ev;  // start/stop pairs of the timed launches
    bool pending = false;        // ev hold times not yet collected
    hipEvent_t done = nullptr;   // recorded after each launch of exec
    uint64_t last = 0;
  };
  static constexpr int kCapacity = 6;
  static constexpr int kSeen = 16;
  std::vector<Entry> entries;
  std::vector<std::vector<int64_t>> seen;
  uint64_t clock = 0;
  bool enabled = true;
  // How timed launches are bracketed inside a capture: 2 event-record nodes
  // added to the capture graph by hand, 1 through the external-record flag,
  // 0 not at all (timed step loops then launch directly).  Lowered when a
  // capture with timing fails.
  int event_mode = 2;
  std::string failure;  // the last capture that failed, and why
  double timed_ms = 0.0;  // collected from replays
  int64_t timed_n = 0;
  int64_t n_captured = 0, n_replayed = 0;

  Entry* find(const std::vector<int64_t>& key) {
    for (Entry& e : entries)
      if (e.key == key) {
        e.last = ++clock;
        return &e;
      }
    return nullptr;
  }

  // True if the key was seen before (and is not yet a graph); records it.
  bool seen_before(const std::vector<int64_t>& key) {
    if (std::find(seen.begin(), seen.end(), key) != seen.end()) return true;
    if ((int)seen.size() >= kSeen) seen.erase(seen.begin());
    seen.push_back(key);
    return false;
  }

  hipError_t collect(Entry& e) {
    if (!e.pending) return hipSuccess;
    hipError_t r = hipEventSynchronize(e.ev.back());
    if (r != hipSuccess) return r;
    for (size_t q = 0; q + 1 < e.ev.size(); q += 2) {
      float ms = 0.0f;
      r = hipEventElapsedTime(&ms, e.ev[q], e.ev[q + 1]);
      if (r != hipSuccess) return r;
      timed_ms += ms;
      timed_n += 1;
    }
    e.pending = false;
    return hipSuccess;
  }

  hipError_t collect_all() {
    for (Entry& e : entries) {
      hipError_t r = collect(e);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  }

  // The graph's last launch must have finished (see evict, clear).
  static void destroy(Entry& e) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    for (hipEvent_t ev : e.ev) (void)hipEventDestroy(ev);
    if (e.done) (void)hipEventDestroy(e.done);
    e.exec = nullptr;
    e.done = nullptr;
    e.ev.clear();
  }

  // Drops every graph (the stream must be idle: callers synchronise first).
  void clear() {
    for (Entry& e : entries) destroy(e);
    entries.clear();
    seen.clear();
  }

  // Forgets the collected times and those not yet collected (the stream
  // must be idle); the graphs stay.
  void reset_timed() {
    for (Entry& e : entries) e.pending = false;
    timed_ms = 0.0;
    timed_n = 0;
  }

  // Captures the launches that `issue(events)` puts on stream s into a new
  // graph under `key` (n_timed launches bracketed by the returned events),
  // then launches it.  issue returns hipSuccess or the first error.  On
  // failure *launched tells whether the graph had been launched (then the
  // error is the caller's to report) or nothing ran (the caller may issue
  // the launches directly instead).
  template <typename F>
  hipError_t capture_and_launch(hipStream_t s, const std::vector<int64_t>& key, int n_timed,
                                F&& issue, bool* launched) {
    *launched = false;
    if ((int)entries.size() >= kCapacity) {
      // evict the least recently used graph once its last launch is done
      size_t lru = 0;
      for (size_t q = 1; q < entries.size(); ++q)
        if (entries[q].last < entries[lru].last) lru = q;
      hipError_t r = hipEventSynchronize(entries[lru].done);
      if (r == hipSuccess) r = collect(entries[lru]);
      if (r != hipSuccess) return r;
      destroy(entries[lru]);
      entries.erase(entries.begin() + (long)lru);
    }
    Entry e;
    e.key = key;
    e.ev.resize(2 * (size_t)n_timed, nullptr);
    hipError_t r = hipEventCreateWithFlags(&e.done, hipEventDisableTiming);
    for (hipEvent_t& ev : e.ev)
      if (r == hipSuccess) r = hipEventCreate(&ev);
    if (r != hipSuccess) {
      destroy(e);
      return r;
    }
    r = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (r != hipSuccess) {
      destroy(e);
      return note(r, "hipStreamBeginCapture");
    }
    hipError_t ri = issue(e.ev);
    const char* stage = "launches under capture";
    hipGraph_t g = nullptr;
    hipError_t rc = hipStreamEndCapture(s, &g);
    if (ri == hipSuccess && rc != hipSuccess) {
      ri = rc;
      stage = "hipStreamEndCapture";
    }
    if (ri == hipSuccess) {
      ri = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
      stage = "hipGraphInstantiate";
    }
    if (g) (void)hipGraphDestroy(g);
    if (ri == hipSuccess) {
      ri = hipGraphLaunch(e.exec, s);
      stage = "hipGraphLaunch";
    }
    if (ri != hipSuccess) {
      destroy(e);
      return note(ri, stage);
    }
    *launched = true;
    ri = hipEventRecord(e.done, s);
    if (ri != hipSuccess) {
      (void)hipStreamSynchronize(s);
      destroy(e);
      return ri;
    }
    e.pending = n_timed > 0;
    e.last = ++clock;
    n_captured += 1;
    seen.erase(std::remove(seen.begin(), seen.end(), key), seen.end());
    entries.push_back(std::move(e));
    return hipSuccess;
  }

  hipError_t note(hipError_t r, const char* stage) {
    failure = std::string(stage) + ": " + hipGetErrorString(r);
    return r;
  }

  hipError_t replay(Entry& e, hipStream_t s) {
    hipError_t r = collect(e);
    if (r != hipSuccess) return r;
    r = hipGraphLaunch(e.exec, s);
    if (r == hipSuccess) r = hipEventRecord(e.done, s);
    if (r == hipSuccess) e.pending = !e.ev.empty();
    if (r == hipSuccess) n_replayed += 1;
    return r;
  }
};

// Bracket for a timed launch.  mode 0: an ordinary record; inside a capture,
// mode 2 adds an event-record node after the captured work by hand and makes
// it the capture's dependency, mode 1 asks the runtime for that node through
// the external-record flag.
inline hipError_t record_timed(hipEvent_t ev, hipStream_t s, int mode) {
  if (mode == 0) return hipEventRecord(ev, s);
  if (mode == 1) return hipEventRecordWithFlags(ev, s, hipEventRecordExternal);
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  unsigned long long id = 0;
  hipGraph_t g = nullptr;
  const hipGraphNode_t* deps = nullptr;
  size_t nd = 0;
  hipError_t r = hipStreamGetCaptureInfo_v2(s, &st, &id, &g, &deps, &nd);
  if (r != hipSuccess) return r;
  if (st != hipStreamCaptureStatusActive || !g) return hipErrorStreamCaptureInvalidated;
  hipGraphNode_t node = nullptr;
  r = hipGraphAddEventRecordNode(&node, g, deps, nd, ev);
  if (r != hipSuccess) return r;
  return hipStreamUpdateCaptureDependencies(s, &node, 1, hipStreamSetCaptureDependencies);
}

}  // namespace lsr
