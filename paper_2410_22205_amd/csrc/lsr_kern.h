// Device helpers and launch helpers shared by the kernel files of the
// narrow-band semi-Lagrangian level-set solver (lsr_kernels.hip,
// lsr_step.hip): wave and block primitives, the XCD-aware sharing of list
// chunks, per-job argument tables of the batched kernels, and persistent
// launches.
#pragma once
#include <hip/hip_ext.h>

#include <algorithm>
#include <mutex>
#include <unordered_map>

#include "lsr_internal.h"

namespace lsr {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t wave_count(bool pred) { return (uint32_t)__popcll(__ballot(pred)); }

// Block-wide append (256 threads, called by all of them): the values of the
// lanes with pred set go to out[] in lane order within the block, behind one
// atomic on the list counter per block.  lds holds at least 5 ints.
template <int K>
__device__ __forceinline__ void block_append(const bool (&pred)[K], const uint32_t (&val)[K],
                                             gwptr<uint32_t> out, int32_t* counter, int* lds) {
  uint64_t m[K];
  int tot = 0;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    m[q] = __ballot(pred[q]);
    tot += (int)__popcll(m[q]);
  }
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) lds[w] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int q = 0; q < 4; ++q) {
      const int cq = lds[q];
      lds[q] = run;
      run += cq;
    }
    lds[4] = run ? atomicAdd(counter, run) : 0;
  }
  __syncthreads();
  int off = lds[4] + lds[w];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    if (pred[q]) out[off + (int)lanes_below(m[q])] = val[q];
    off += (int)__popcll(m[q]);
  }
  __syncthreads();
}

__device__ __forceinline__ void block_append1(bool pred, uint32_t val, gwptr<uint32_t> out,
                                              int32_t* counter, int* lds) {
  const bool p[1] = {pred};
  const uint32_t v[1] = {val};
  block_append<1>(p, v, out, counter, lds);
}

// Block-wide sum of up to three wave-uniform counts added to work counters
// ca, cb, cc (-1: none) of the statistics array, one atomic per nonzero total,
// in this block's slot.  lds holds at least 12 uints.
__device__ __forceinline__ void block_add3(uint32_t a, uint32_t b, uint32_t c,
                                           unsigned long long* stats, int ca, int cb, int cc,
                                           uint32_t* lds) {
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (lane_id() == 0) {
    lds[3 * w] = a;
    lds[3 * w + 1] = b;
    lds[3 * w + 2] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t[3] = {0, 0, 0};
    for (int q = 0; q < 4; ++q)
      for (int r = 0; r < 3; ++r) t[r] += lds[3 * q + r];
    const int slot = (int)(blockIdx.x % STAT_SLOTS);
    const int cs[3] = {ca, cb, cc};
    for (int r = 0; r < 3; ++r)
      if (t[r] && cs[r] >= 0) atomicAdd(&stats[stat_index(cs[r], slot)], (unsigned long long)t[r]);
  }
}


// Items [0, n) shared out in contiguous stretches, one per XCD: the blocks
// of XCD x (the dispatcher places workgroup b on XCD b mod 8) take the items
// [x * per, min(x * per + per, n)), per = ceil(n / 8), in increasing order,
// so that an XCD works through one stretch of a list at a time and its L2
// holds that stretch's neighbourhood.  Sets the block's first item and the
// stretch's end and returns the stride between the block's items.  The grid
// is a multiple of 8 blocks.
__device__ __forceinline__ uint32_t xcd_share(uint32_t n, uint32_t& first, uint32_t& end) {
  const uint32_t per = (n + 7u) / 8u, beg = (blockIdx.x % 8u) * per;
  end = min(beg + per, n);
  first = beg + blockIdx.x / 8u;
  return gridDim.x / 8u;
}

// Block-wide ordered compaction (256 threads, called by all of them): the
// values of the lanes with pred set go to out[0 ..) ordered by (q, wave,
// lane), q the index of the value in the thread; returns their number.  No
// atomics: the order is the order of the block's nodes.  lds holds at least
// 4 K + 1 ints.
template <int K>
__device__ __forceinline__ int block_compact(const bool (&pred)[K], const uint32_t (&val)[K],
                                             gwptr<uint32_t> out, int* lds) {
  uint64_t m[K];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    m[q] = __ballot(pred[q]);
    if (lane_id() == 0) lds[q * 4 + w] = (int)__popcll(m[q]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int e = 0; e < 4 * K; ++e) {
      const int c = lds[e];
      lds[e] = run;
      run += c;
    }
    lds[4 * K] = run;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < K; ++q)
    if (pred[q]) out[lds[q * 4 + w] + (int)lanes_below(m[q])] = val[q];
  const int tot = lds[4 * K];
  __syncthreads();
  return tot;
}

// A table entry read with scalar loads into scalar registers, as kernel
// arguments are: the table is read through the constant address space (the
// host writes it before the launch and nothing writes it during one) at a
// wave-uniform index, so the per-job arguments neither cost vector memory
// instructions nor occupy vector registers.
template <typename A>
__device__ __forceinline__ A uniform_load(const A* tab, int index) {
  static_assert(sizeof(A) % 4 == 0, "table entries are whole words");
  typedef const __attribute__((address_space(4))) uint32_t cword;
  const int q = __builtin_amdgcn_readfirstlane(index);
  cword* src = (cword*)(tab + q);
  A out;
  uint32_t* dst = (uint32_t*)&out;
#pragma unroll
  for (unsigned w = 0; w < sizeof(A) / 4; ++w) dst[w] = src[w];
  return out;
}

// A value that every lane of the wave holds alike, moved into scalar
// registers (lane 0's copy), so that keeping it costs no vector register.
template <typename V>
__device__ __forceinline__ V uniform_value(V x) {
  static_assert(sizeof(V) % 4 == 0, "whole words");
  uint32_t w[sizeof(V) / 4];
  __builtin_memcpy(w, &x, sizeof(V));
#pragma unroll
  for (unsigned q = 0; q < sizeof(V) / 4; ++q) w[q] = __builtin_amdgcn_readfirstlane(w[q]);
  __builtin_memcpy(&x, w, sizeof(V));
  return x;
}

// One field (at byte offset off) of table entry `index`, read the same way.
template <typename F, typename A>
__device__ __forceinline__ F uniform_field(const A* tab, int index, size_t off) {
  static_assert(sizeof(F) % 4 == 0, "fields are whole words");
  typedef const __attribute__((address_space(4))) uint32_t cword;
  const int q = __builtin_amdgcn_readfirstlane(index);
  cword* src = (cword*)((const char*)(tab + q) + off);
  F out;
  uint32_t* dst = (uint32_t*)&out;
#pragma unroll
  for (unsigned w = 0; w < sizeof(F) / 4; ++w) dst[w] = src[w];
  return out;
}
#define LSR_FIELD(tab, jb, Type, field) \
  uniform_field<decltype(Type::field)>(tab, jb, offsetof(Type, field))

// Chunks of one job in a launch: band-list chunks (step), grid slots (list
// builds), LCHUNK-entry chunks of Gbar (reinitialisation).
template <typename T>
__device__ __forceinline__ uint32_t job_chunks(const SLArgs<T>* tab, int jb) {
  return (uint32_t)*LSR_FIELD(tab, jb, SLArgs<T>, cnt_in);
}
template <typename T>
__device__ __forceinline__ uint32_t job_chunks(const GbarArgs<T>* tab, int jb) {
  return gbar_slots(LSR_FIELD(tab, jb, GbarArgs<T>, g));
}
template <typename T>
__device__ __forceinline__ uint32_t job_chunks(const RArgs<T>* tab, int jb) {
  return ((uint32_t)*LSR_FIELD(tab, jb, RArgs<T>, cnt) + LCHUNK - 1) / LCHUNK;
}
template <typename T>
__device__ __forceinline__ uint32_t job_chunks(const FinArgs<T>* tab, int jb) {
  return ((uint32_t)*LSR_FIELD(tab, jb, FinArgs<T>, cnt_in) + LCHUNK - 1) / LCHUNK;
}

template <typename A>
__device__ __forceinline__ uint32_t total_chunks(const A* tab, int n) {
  uint32_t t = 0;
  for (int jb = 0; jb < n; ++jb) t += job_chunks(tab, jb);
  return t;
}

// Cursor of a block over the jobs of a batched launch, whose chunks are
// numbered one job after the other: job jb holds the global chunks
// [beg, end).  advance() moves to the job holding chunk gch (gch never
// decreases) and returns false once gch lies past the last job; on every job
// change it calls leave(jb) for the job being left (uniform across the
// block).
struct JobCursor {
  int n, jb = -1;
  uint32_t beg = 0, end = 0;
  template <typename A, typename Leave>
  __device__ __forceinline__ bool advance(const A* tab, uint32_t gch, Leave leave) {
    while (gch >= end) {
      if (jb >= 0) leave(jb);
      if (++jb >= n) return false;
      beg = end;
      end = beg + job_chunks(tab, jb);
    }
    return true;
  }
};

// Blocks of a persistent launch: `blocks` (a multiple of 8) is an upper
// bound, and the launch takes no more blocks than fit on the device at once
// (this kernel's occupancy at 256 threads times the CU count), rounded down
// to a multiple of 8.  The chunks of a list are striped over the blocks up
// front, so a block that had to wait for a second round would finish its
// share late and hold up the whole launch.  Computed once per kernel (one
// device type per process).
static unsigned resident_blocks(const void* kern) {
  static std::mutex m;
  static std::unordered_map<const void*, unsigned> cache;
  std::lock_guard<std::mutex> lock(m);
  auto it = cache.find(kern);
  if (it != cache.end()) return it->second;
  int dev = 0, ncu = 0, nb = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, 256, 0) != hipSuccess)
    return 1u << 30;  // unknown: no clamp
  unsigned r = (unsigned)(ncu * (nb > 0 ? nb : 1)) / 8u * 8u;
  if (r < 8) r = 8;
  cache[kern] = r;
  return r;
}

template <typename... P, typename... A>
static hipError_t persistent_launch(void (*kern)(P...), unsigned blocks, hipStream_t s, A... args) {
  if (blocks == 0 || blocks % 8) return hipErrorInvalidConfiguration;
  const unsigned b = std::min(blocks, resident_blocks((const void*)kern));
  hipLaunchKernelGGL(kern, dim3(b), dim3(256), 0, s, args...);
  return hipGetLastError();
}

// The same launch with start and stop events tied to the dispatch itself, so
// that their elapsed time is the kernel's execution time.
template <typename... P, typename... A>
static hipError_t persistent_launch_timed(void (*kern)(P...), unsigned blocks, hipStream_t s,
                                          hipEvent_t start, hipEvent_t stop, A... args) {
  if (blocks == 0 || blocks % 8) return hipErrorInvalidConfiguration;
  const unsigned b = std::min(blocks, resident_blocks((const void*)kern));
  hipExtLaunchKernelGGL(kern, dim3(b), dim3(256), 0, s, start, stop, 0, args...);
  return hipGetLastError();
}

}  // namespace lsr
