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
    hipEvent_t done = nullptr;  // recorded after each launch of exec
    uint64_t last = 0;
  };
  static constexpr int kCapacity = 6;
  static constexpr int kSeen = 16;
  std::vector<Entry> entries;
  std::vector<std::vector<int64_t>> seen;
  uint64_t clock = 0;
  bool enabled = true;
  std::string failure;  // the last capture that failed, and why
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

  // The graph's last launch must have finished (see capture_and_launch,
  // clear).
  static void destroy(Entry& e) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.done) (void)hipEventDestroy(e.done);
    e.exec = nullptr;
    e.done = nullptr;
  }

  // Drops every graph (the stream must be idle: callers synchronise first).
  void clear() {
    for (Entry& e : entries) destroy(e);
    entries.clear();
    seen.clear();
  }

  hipError_t note(hipError_t r, const char* stage) {
    failure = std::string(stage) + ": " + hipGetErrorString(r);
    return r;
  }

  // Captures the launches that `issue()` puts on stream s into a new graph
  // under `key`, then launches it.  issue returns hipSuccess or the first
  // error.  On failure *launched tells whether the graph had been launched
  // (then the error is the caller's to report) or nothing ran (the caller
  // may issue the launches directly instead).
  template <typename F>
  hipError_t capture_and_launch(hipStream_t s, const std::vector<int64_t>& key, F&& issue,
                                bool* launched) {
    *launched = false;
    if ((int)entries.size() >= kCapacity) {
      // evict the least recently used graph once its last launch is done
      size_t lru = 0;
      for (size_t q = 1; q < entries.size(); ++q)
        if (entries[q].last < entries[lru].last) lru = q;
      hipError_t r = hipEventSynchronize(entries[lru].done);
      if (r != hipSuccess) return note(r, "hipEventSynchronize");
      destroy(entries[lru]);
      entries.erase(entries.begin() + (long)lru);
    }
    Entry e;
    e.key = key;
    hipError_t r = hipEventCreateWithFlags(&e.done, hipEventDisableTiming);
    if (r != hipSuccess) return note(r, "hipEventCreateWithFlags");
    r = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (r != hipSuccess) {
      destroy(e);
      return note(r, "hipStreamBeginCapture");
    }
    hipError_t ri = issue();
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
      return note(ri, "hipEventRecord");
    }
    e.last = ++clock;
    n_captured += 1;
    seen.erase(std::remove(seen.begin(), seen.end(), key), seen.end());
    entries.push_back(std::move(e));
    return hipSuccess;
  }

  hipError_t replay(Entry& e, hipStream_t s) {
    hipError_t r = hipGraphLaunch(e.exec, s);
    if (r == hipSuccess) r = hipEventRecord(e.done, s);
    if (r == hipSuccess) n_replayed += 1;
    return r;
  }
};

}  // namespace lsr
