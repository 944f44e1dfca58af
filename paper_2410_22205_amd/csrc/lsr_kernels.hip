// HIP kernels of the narrow-band semi-Lagrangian level-set solver for gfx950
// (Preda & Semplice, arXiv:2410.22205) and their launchers.
//
// Every list kernel is a grid-stride loop over a device-resident list whose
// length it reads from device memory, so launches have a fixed shape and need
// no host round trip.  Each of the 8 XCDs walks a contiguous stretch of the
// list (xcd_share), so its own L2 sees neighbouring nodes.  Lists are built
// in the order of a brick-by-brick scan of the grid and compacted per block
// in that order (block_compact), without atomics.
#include <hip/hip_ext.h>

#include <mutex>
#include <unordered_map>

#include "lsr_kern.h"

namespace lsr {

// ------------------------------------------------------------------ fills

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < n;
       e += (uint64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

__global__ void k_fill_u8(uint8_t* p, uint8_t v, uint64_t n) {
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < n;
       e += (uint64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

// ------------------------------------------------------------- init / band

// Closed-form signed distance (computed in double, stored in float) or a
// copy of the caller's array, cut to [-gamma, gamma]; written to both phi
// buffers (A == NULL: only check the array).  flag[0] |= 1 for a non-finite
// input value.
template <int DIM, typename T>
__global__ void k_init_phi(DevGrid g, int kind, double a0, double a1, double a2, double a3,
                           double a4, T gamma, const T* __restrict__ src, T* __restrict__ A,
                           T* __restrict__ B, int32_t* flag) {
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.N;
       idx += gridDim.x * blockDim.x) {
    T v;
    if (kind == 0) {
      v = src[idx];
      if (!isfinite(v)) atomicOr(flag, 1);
    } else {
      // no FMA contraction: nodes placed symmetrically about the centre get
      // bitwise symmetric values (the 3D tangent frame of the update switches
      // on an exact zero of two gradient components)
#pragma clang fp contract(off)
      uint32_t r = idx;
      int k = 0;
      if (DIM == 3) {
        k = (int)(r % (uint32_t)g.n2);
        r /= (uint32_t)g.n2;
      }
      int j = (int)(r % (uint32_t)g.n1);
      int i = (int)(r / (uint32_t)g.n1);
      double x = g.lo0 + i * g.hd - a0, y = g.lo1 + j * g.hd - a1;
      double z = DIM == 3 ? g.lo2 + k * g.hd - a2 : 0.0;
      double s;
      if (kind == 1) {
        s = sqrt(x * x + y * y + z * z) - a3;
      } else {
        double rho = sqrt(x * x + y * y) - a3;
        s = sqrt(rho * rho + z * z) - a4;
      }
      v = (T)s;
    }
    if (!A) continue;  // check-only pass over the caller's array
    v = fmin(fmax(v, -gamma), gamma);
    A[idx] = v;
    B[idx] = v;
  }
}

// Grid nodes of one slot of a grid scan (GBAR_CHUNK nodes; see GbarArgs):
// thread t's node of sub-slot u (in 3D brick u of the slot's 2 x 2 x 2, the
// brick's nodes in C order over the block's threads).  False past the grid.
template <int DIM>
__device__ __forceinline__ bool slot_node(const DevGrid& g, uint32_t slot, uint32_t u, int& i,
                                          int& j, int& k) {
  if (DIM == 3) {
    const uint32_t nsj = slots_along((uint32_t)g.n1, SB1), nsk = slots_along((uint32_t)g.n2, SB2);
    const uint32_t bi = 2 * (slot / (nsj * nsk)) + (u >> 2);
    const uint32_t bj = 2 * ((slot / nsk) % nsj) + ((u >> 1) & 1);
    const uint32_t bk = 2 * (slot % nsk) + (u & 1);
    i = (int)(bi * SB0 + threadIdx.x / (SB1 * SB2));
    j = (int)(bj * SB1 + (threadIdx.x / SB2) % SB1);
    k = (int)(bk * SB2 + threadIdx.x % SB2);
    return i < g.n0 && j < g.n1 && k < g.n2;
  }
  const uint32_t idx = slot * GBAR_CHUNK + u * 256u + threadIdx.x;
  k = 0;
  i = (int)(idx / (uint32_t)g.n1);
  j = (int)(idx % (uint32_t)g.n1);
  return idx < g.N;
}

// Members of one slot, in node order, to S at slot * GBAR_CHUNK; their
// number to scnt[slot].
template <int DIM, typename T>
__device__ __forceinline__ void grid_slot(const GbarArgs<T>& a, uint32_t slot, int* lds) {
  const gptr<T> P = (gptr<T>)a.P;
  bool in[GBAR_SUB];
  uint32_t code[GBAR_SUB];
#pragma unroll
  for (uint32_t u = 0; u < GBAR_SUB; ++u) {
    int i, j, k;
    in[u] = false;
    code[u] = 0;
    if (slot_node<DIM>(a.g, slot, u, i, j, k)) {
      const uint32_t idx = lin(a.g, i, j, k);
      T m = fabs(P[idx]);
      if (a.nbr) {
        // the six neighbours (a neighbour off the grid reads the node itself)
        const T xm = P[i > 0 ? idx - a.g.s0 : idx], xp = P[i < a.g.n0 - 1 ? idx + a.g.s0 : idx];
        const T ym = P[j > 0 ? idx - a.g.s1 : idx], yp = P[j < a.g.n1 - 1 ? idx + a.g.s1 : idx];
        m = fmin(fmin(m, fmin(fabs(xm), fabs(xp))), fmin(fabs(ym), fabs(yp)));
        if (DIM == 3) {
          const T zm = P[k > 0 ? idx - 1 : idx], zp = P[k < a.g.n2 - 1 ? idx + 1 : idx];
          m = fmin(m, fmin(fabs(zm), fabs(zp)));
        }
      }
      in[u] = m < a.gamma;
      code[u] = encode(a.g, i, j, k);
    }
  }
  const int tot = block_compact<GBAR_SUB>(in, code, (gwptr<uint32_t>)a.S + slot * GBAR_CHUNK, lds);
  if (threadIdx.x == 0) a.scnt[slot] = tot;
}

// Slot of grid node (i, j, k) in the scan order of slot_node.
template <int DIM>
__device__ __forceinline__ uint32_t slot_of(const DevGrid& g, int i, int j, int k) {
  if (DIM == 3) {
    const uint32_t nsj = slots_along((uint32_t)g.n1, SB1), nsk = slots_along((uint32_t)g.n2, SB2);
    return ((uint32_t)i / SB0 / 2 * nsj + (uint32_t)j / SB1 / 2) * nsk + (uint32_t)k / SB2 / 2;
  }
  return ((uint32_t)i * (uint32_t)g.n1 + (uint32_t)j) / GBAR_CHUNK;
}

// Marks of the slots that can hold a member of Gbar: those of every band
// node and of its face neighbours.
template <int DIM, typename T>
__device__ __forceinline__ void mark_chunk(const GbarArgs<T>& a, uint32_t c) {
  if ((int)threadIdx.x >= a.Lccnt[c]) return;
  int i, j, k;
  decode(a.g, a.L[c * LCHUNK + threadIdx.x], i, j, k);
  const DevGrid& g = a.g;
  a.smark[slot_of<DIM>(g, i, j, k)] = 1;
  if (i > 0) a.smark[slot_of<DIM>(g, i - 1, j, k)] = 1;
  if (i < g.n0 - 1) a.smark[slot_of<DIM>(g, i + 1, j, k)] = 1;
  if (j > 0) a.smark[slot_of<DIM>(g, i, j - 1, k)] = 1;
  if (j < g.n1 - 1) a.smark[slot_of<DIM>(g, i, j + 1, k)] = 1;
  if (DIM == 3) {
    if (k > 0) a.smark[slot_of<DIM>(g, i, j, k - 1)] = 1;
    if (k < g.n2 - 1) a.smark[slot_of<DIM>(g, i, j, k + 1)] = 1;
  }
}

template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_mark_slots(GbarArgs<T> a) {
  uint32_t c, end;
  const uint32_t step = xcd_share((uint32_t)*a.Lcnt, c, end);
  for (; c < end; c += step) mark_chunk<DIM, T>(a, c);
}

template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_mark_slots_batch(const GbarArgs<T>* __restrict__ tab,
                                                          int n) {
  // chunks of the band lists, numbered one job after the other
  uint32_t tot = 0;
  for (int jb = 0; jb < n; ++jb) tot += (uint32_t)*LSR_FIELD(tab, jb, GbarArgs<T>, Lcnt);
  uint32_t c, end;
  const uint32_t step = xcd_share(tot, c, end);
  int jb = -1;
  uint32_t beg = 0, stop = 0;
  for (; c < end; c += step) {
    while (c >= stop) {
      ++jb;
      beg = stop;
      stop = beg + (uint32_t)*LSR_FIELD(tab, jb, GbarArgs<T>, Lcnt);
    }
    mark_chunk<DIM, T>(uniform_load(tab, jb), c - beg);
  }
}

template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_grid_scan(GbarArgs<T> a) {
  __shared__ int lds[4 * GBAR_SUB + 1];
  uint32_t c, end;
  const uint32_t step = xcd_share(gbar_slots(a.g), c, end);
  for (; c < end; c += step) {
    if (a.smark) {
      // the mark is read and cleared here (one block per slot), so the
      // marks are all clear again for the next build
      const bool marked = a.smark[c] != 0;
      __syncthreads();
      if (threadIdx.x == 0) {
        a.smark[c] = 0;
        if (!marked) a.scnt[c] = 0;
      }
      if (!marked) continue;
    }
    grid_slot<DIM, T>(a, c, lds);
  }
}

template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_grid_scan_batch(const GbarArgs<T>* __restrict__ tab,
                                                         int n) {
  __shared__ int lds[4 * GBAR_SUB + 1];
  JobCursor cur{n};
  auto leave = [](int) {};
  uint32_t c, end;
  const uint32_t step = xcd_share(total_chunks(tab, n), c, end);
  for (; c < end; c += step) {
    if (!cur.advance(tab, c, leave)) break;
    const GbarArgs<T> a = uniform_load(tab, cur.jb);
    const uint32_t s = c - cur.beg;
    if (a.smark) {
      const bool marked = a.smark[s] != 0;
      __syncthreads();
      if (threadIdx.x == 0) {
        a.smark[s] = 0;
        if (!marked) a.scnt[s] = 0;
      }
      if (!marked) continue;
    }
    grid_slot<DIM, T>(a, s, lds);
  }
}

// Exclusive prefix of the slot counts (one block of 1024 threads per job):
// thread t sums a run of consecutive slots, the block scans the 1024 sums.
template <typename T>
__device__ __forceinline__ void slot_prefix(const GbarArgs<T>& a, int* lds) {
  const uint32_t G = gbar_slots(a.g);
  const uint32_t per = (G + 1023u) / 1024u;
  const uint32_t t = threadIdx.x, b0 = min(t * per, G), b1 = min(b0 + per, G);
  int s = 0;
  for (uint32_t u = b0; u < b1; ++u) s += a.scnt[u];
  // inclusive scan within the wave, then over the 16 wave totals
  const int lane = (int)lane_id(), w = (int)(t >> 6);
  int x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) lds[w] = x;
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int q = 0; q < 16; ++q) {
      const int c = lds[q];
      lds[q] = run;
      run += c;
    }
    lds[16] = run;
  }
  __syncthreads();
  int run = lds[w] + x - s;
  for (uint32_t u = b0; u < b1; ++u) {
    a.soff[u] = run;
    run += a.scnt[u];
  }
  const int total = lds[16];
  if (t == 0) {
    a.soff[G] = total;
    *a.cnt_out = a.ccnt ? (int)((total + (int)LCHUNK - 1) / (int)LCHUNK) : total;
  }
  if (a.ccnt) {
    const int nc = (total + (int)LCHUNK - 1) / (int)LCHUNK;
    for (int c = (int)t; c < nc; c += 1024) a.ccnt[c] = min((int)LCHUNK, total - c * (int)LCHUNK);
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_slot_prefix(GbarArgs<T> a) {
  __shared__ int lds[17];
  slot_prefix<T>(a, lds);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_slot_prefix_batch(const GbarArgs<T>* __restrict__ tab) {
  __shared__ int lds[17];
  slot_prefix<T>(uniform_load(tab, (int)blockIdx.x), lds);
}

// Every slot's members to their place in M.
template <typename T>
__device__ __forceinline__ void slot_pack(const GbarArgs<T>& a, uint32_t slot) {
  const int n = a.scnt[slot], o = a.soff[slot];
  const gptr<uint32_t> S = (gptr<uint32_t>)a.S + slot * GBAR_CHUNK;
  const gwptr<uint32_t> M = (gwptr<uint32_t>)a.M + o;
  for (int r = (int)threadIdx.x; r < n; r += 256) M[r] = S[r];
}

template <typename T>
__global__ __launch_bounds__(256) void k_slot_pack(GbarArgs<T> a) {
  uint32_t c, end;
  const uint32_t step = xcd_share(gbar_slots(a.g), c, end);
  for (; c < end; c += step) slot_pack<T>(a, c);
}

template <typename T>
__global__ __launch_bounds__(256) void k_slot_pack_batch(const GbarArgs<T>* __restrict__ tab,
                                                         int n) {
  JobCursor cur{n};
  auto leave = [](int) {};
  uint32_t c, end;
  const uint32_t step = xcd_share(total_chunks(tab, n), c, end);
  for (; c < end; c += step) {
    if (!cur.advance(tab, c, leave)) break;
    slot_pack<T>(uniform_load(tab, cur.jb), c - cur.beg);
  }
}

// Band mask of the current list: mask[idx] = 1 iff |phi| < gamma.
template <typename T>
__global__ __launch_bounds__(256) void k_band_mask(DevGrid g, T gamma, const T* __restrict__ A,
                                                   const uint32_t* __restrict__ L,
                                                   const int32_t* __restrict__ ccnt,
                                                   const int32_t* cnt, uint8_t* __restrict__ mask,
                                                   int32_t* count) {
  __shared__ uint32_t lds[12];
  uint32_t tot = 0;
  uint32_t c, end;
  const uint32_t step = xcd_share((uint32_t)*cnt, c, end);
  for (; c < end; c += step) {
    bool in = false;
    if ((int)threadIdx.x < ccnt[c]) {
      int i, j, k;
      decode(g, L[c * LCHUNK + threadIdx.x], i, j, k);
      const uint32_t idx = lin(g, i, j, k);
      in = fabs(A[idx]) < gamma;
      if (in && mask) mask[idx] = 1;
    }
    tot += wave_count(in);
  }
  __syncthreads();
  if (lane_id() == 0) lds[threadIdx.x >> 6] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t t = lds[0] + lds[1] + lds[2] + lds[3];
    if (t) atomicAdd(count, (int)t);
  }
}

// ------------------------------------------------------- reinitialisation

// Interface set and one-step fix on Gbar.  Reads phi~ from src, writes the
// working copy dst: dst = phi~ / max(|grad_c phi~|, floor) on interface nodes
// (a face neighbour of opposite or zero sign), dst = phi~ elsewhere on Gbar.
// flags: bit 7 interface, bits 0-1 sign of phi~ (1 positive, 2 negative).
template <int DIM, typename T>
__device__ __forceinline__ void fix_chunk(const RArgs<T>& a, uint32_t base, int n, uint32_t& ng,
                                          uint32_t& nif) {
  const gptr<T> src = (gptr<T>)a.src;
  const gwptr<T> dst = (gwptr<T>)a.dst;
  const gptr<uint32_t> M = (gptr<uint32_t>)a.M;
  const gwptr<uint8_t> flags = (gwptr<uint8_t>)a.flags;
  const uint32_t e = base + threadIdx.x;
  bool itf = false;
  const bool valid = e < (uint32_t)n;
  if (valid) {
    int i, j, k;
    decode(a.g, M[e], i, j, k);
    const uint32_t idx = lin(a.g, i, j, k);
    // neighbours off the grid read the node itself
    const T t = src[idx];
    const T xm = src[i > 0 ? idx - a.g.s0 : idx], xp = src[i < a.g.n0 - 1 ? idx + a.g.s0 : idx];
    const T ym = src[j > 0 ? idx - a.g.s1 : idx], yp = src[j < a.g.n1 - 1 ? idx + a.g.s1 : idx];
    T zm = t, zp = t;
    if (DIM == 3) {
      zm = src[k > 0 ? idx - 1 : idx];
      zp = src[k < a.g.n2 - 1 ? idx + 1 : idx];
    }
    const T z0 = T(0);
    itf = (i > 0 && t * xm <= z0) || (i < a.g.n0 - 1 && t * xp <= z0) ||
          (j > 0 && t * ym <= z0) || (j < a.g.n1 - 1 && t * yp <= z0);
    if (DIM == 3) itf = itf || (k > 0 && t * zm <= z0) || (k < a.g.n2 - 1 && t * zp <= z0);
    T w = t;
    if (itf) {
      const T gx = cdiff(xm, t, xp, i, a.g.n0, a.c);
      const T gy = cdiff(ym, t, yp, j, a.g.n1, a.c);
      const T gz = DIM == 3 ? cdiff(zm, t, zp, k, a.g.n2, a.c) : z0;
      const T nr = fmax(sqrt(gx * gx + gy * gy + gz * gz), a.floor_);
      w = t / nr;
    }
    dst[idx] = w;
    flags[e] = (uint8_t)((itf ? 0x80 : 0) | (t > z0 ? 1 : (t < z0 ? 2 : 0)));
  }
  nif += wave_count(itf);
  ng += wave_count(valid);
}

template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_reinit_fix(RArgs<T> a) {
  __shared__ uint32_t lds_st[12];
  const int n = *a.cnt;
  uint32_t nif = 0, ng = 0;
  uint32_t c, end;
  const uint32_t step = xcd_share(((uint32_t)n + LCHUNK - 1) / LCHUNK, c, end);
  for (; c < end; c += step) fix_chunk<DIM, T>(a, c * LCHUNK, n, ng, nif);
  block_add3(ng, nif, 0, a.stats, 4, 5, -1, lds_st);
}

template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_reinit_fix_batch(const RArgs<T>* __restrict__ tab, int n) {
  __shared__ uint32_t lds_st[12];
  uint32_t nif = 0, ng = 0;
  JobCursor cur{n};
  auto leave = [&](int jb) {
    block_add3(ng, nif, 0, LSR_FIELD(tab, jb, RArgs<T>, stats), 4, 5, -1, lds_st);
    ng = nif = 0;
  };
  uint32_t c, end;
  const uint32_t step = xcd_share(total_chunks(tab, n), c, end);
  for (; c < end; c += step) {
    if (!cur.advance(tab, c, leave)) break;
    const RArgs<T> a = uniform_load(tab, cur.jb);
    fix_chunk<DIM, T>(a, (c - cur.beg) * LCHUNK, *a.cnt, ng, nif);
  }
  if (cur.jb >= 0 && cur.jb < n) leave(cur.jb);
}

// One forward-Euler pseudo-time step of phi_tau + S (|grad phi| - 1) = 0 on
// Gbar minus the interface set, first-order upwind (Godunov) gradient; a
// neighbour off the grid contributes no difference.  src -> dst on Gbar.
template <int DIM, typename T>
__device__ __forceinline__ void iter_chunk(const RArgs<T>& a, uint32_t base, int n) {
  const gptr<T> src = (gptr<T>)a.src;
  const gwptr<T> dst = (gwptr<T>)a.dst;
  const gptr<uint32_t> M = (gptr<uint32_t>)a.M;
  const gptr<uint8_t> flags = (gptr<uint8_t>)a.flags;
  const uint32_t e = base + threadIdx.x;
  if (e >= (uint32_t)n) return;
  int i, j, k;
  decode(a.g, M[e], i, j, k);
  const uint32_t idx = lin(a.g, i, j, k);
  const uint8_t f = flags[e];
  T v = src[idx];
  if (!(f & 0x80) && (f & 3)) {
    const bool pos = f & 1;
    const T z0 = T(0);
    T G2 = z0;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
      const int ci = ax == 0 ? i : (ax == 1 ? j : k);
      const int nn = ax == 0 ? a.g.n0 : (ax == 1 ? a.g.n1 : a.g.n2);
      const uint32_t s = ax == 0 ? a.g.s0 : (ax == 1 ? a.g.s1 : 1u);
      // a neighbour off the grid reads the node: zero difference
      const T vm = src[ci > 0 ? idx - s : idx], vp = src[ci < nn - 1 ? idx + s : idx];
      const T Dm = (v - vm) * a.c.inv_h;
      const T Dp = (vp - v) * a.c.inv_h;
      T t1, t2;
      if (pos) {
        t1 = Dm > z0 ? Dm * Dm : z0;
        t2 = Dp < z0 ? Dp * Dp : z0;
      } else {
        t1 = Dm < z0 ? Dm * Dm : z0;
        t2 = Dp > z0 ? Dp * Dp : z0;
      }
      G2 += fmax(t1, t2);
    }
    const T S = pos ? T(1) : T(-1);
    v = v - a.dtau * S * (sqrt(G2) - T(1));
  }
  dst[idx] = v;
}

template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_reinit_iter(RArgs<T> a) {
  const int n = *a.cnt;
  uint32_t c, end;
  const uint32_t step = xcd_share(((uint32_t)n + LCHUNK - 1) / LCHUNK, c, end);
  for (; c < end; c += step) iter_chunk<DIM, T>(a, c * LCHUNK, n);
}

template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_reinit_iter_batch(const RArgs<T>* __restrict__ tab, int n) {
  JobCursor cur{n};
  auto leave = [](int) {};
  uint32_t c, end;
  const uint32_t step = xcd_share(total_chunks(tab, n), c, end);
  for (; c < end; c += step) {
    if (!cur.advance(tab, c, leave)) break;
    const RArgs<T> a = uniform_load(tab, cur.jb);
    iter_chunk<DIM, T>(a, (c - cur.beg) * LCHUNK, *a.cnt);
  }
}

// Cut of eq. (cut) on Gbar, both buffers made equal there, the sign words
// moved to the cut phi, and the new band list: Gbar's chunk c compacted into
// chunk c of Lout.
template <typename T>
__device__ __forceinline__ void final_chunk(const FinArgs<T>& a, uint32_t c, int n, int* lds) {
  const gptr<uint32_t> M = (gptr<uint32_t>)a.M;
  const gwptr<T> cur = (gwptr<T>)a.cur;
  const gwptr<T> other = (gwptr<T>)a.other;
  const uint32_t e = c * LCHUNK + threadIdx.x;
  bool in[1] = {false};
  uint32_t code[1] = {0};
  if (e < (uint32_t)n) {
    code[0] = M[e];
    int i, j, k;
    decode(a.g, code[0], i, j, k);
    const uint32_t idx = lin(a.g, i, j, k);
    const T v = fmin(fmax(cur[idx], -a.gamma), a.gamma);
    cur[idx] = v;
    other[idx] = v;
    in[0] = fabs(v) < a.gamma;
    // this node's bit is written by this thread alone (other bits of the
    // word may change meanwhile)
    uint32_t w, bit;
    sign_word_of(a.g, i, j, k, w, bit);
    const bool neg = v < T(0);
    if (((a.sgn[w] & bit) != 0) != neg) sign_set(a.sgn, w, bit, neg);
  }
  const int kept = block_compact<1>(in, code, (gwptr<uint32_t>)a.Lout + c * LCHUNK, lds);
  if (threadIdx.x == 0) a.ccnt_out[c] = kept;
}

template <typename T>
__global__ __launch_bounds__(256) void k_reinit_final(FinArgs<T> a) {
  __shared__ int lds[5];
  const int n = *a.cnt_in;
  const uint32_t nch = ((uint32_t)n + LCHUNK - 1) / LCHUNK;
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.cnt_out = (int32_t)nch;
  uint32_t c, end;
  const uint32_t step = xcd_share(nch, c, end);
  for (; c < end; c += step) final_chunk<T>(a, c, n, lds);
}

template <typename T>
__global__ __launch_bounds__(256) void k_reinit_final_batch(const FinArgs<T>* __restrict__ tab,
                                                            int n) {
  __shared__ int lds[5];
  if (blockIdx.x == 0)
    for (int t = (int)threadIdx.x; t < n; t += (int)blockDim.x)
      *tab[t].cnt_out = (int32_t)(((uint32_t)*tab[t].cnt_in + LCHUNK - 1) / LCHUNK);
  JobCursor cur{n};
  auto leave = [](int) {};
  uint32_t c, end;
  const uint32_t step = xcd_share(total_chunks(tab, n), c, end);
  for (; c < end; c += step) {
    if (!cur.advance(tab, c, leave)) break;
    const FinArgs<T> a = uniform_load(tab, cur.jb);
    final_chunk<T>(a, c - cur.beg, *a.cnt_in, lds);
  }
}


// ------------------------------------------------------------ distance

// Points of a candidate bin read per trip through the scalar unit (all of a
// trip's loads are in flight before the first is used).
#ifndef LSR_DIST_PTS
#define LSR_DIST_PTS 8
#endif

// Validate and bin the cloud (bin ids grouped by super-bin, see SUP); flag
// |= 1 for a non-finite point or one outside the grid's box.
template <int DIM>
__global__ void k_bin_points(BinGeom bg, const double* __restrict__ pts, int64_t n,
                             int32_t* __restrict__ bin_count, int32_t* __restrict__ pt_bin,
                             int32_t* flag, int32_t* occupied) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    bool ok = true;
    int b[3] = {0, 0, 0};
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
      const double x = pts[p * DIM + ax];
      const double lo = bg.lo[ax], hi = bg.hi[ax];
      if (!(x >= lo && x <= hi)) ok = false;  // also false for NaN
      int q = ok ? (int)floor((x - lo) * bg.inv_bw) : 0;
      b[ax] = q < 0 ? 0 : (q > bg.nb[ax] - 1 ? bg.nb[ax] - 1 : q);
    }
    if (!ok) {
      atomicOr(flag, 1);
      pt_bin[p] = -1;
      continue;
    }
    const int id = bin_id(bg, b);
    if (atomicAdd(&bin_count[id], 1) == 0) atomicAdd(occupied, 1);  // the bin's first point
    pt_bin[p] = id;
  }
}

// Exclusive scan of the bin counts (one block, 1024 threads, contiguous
// segments per thread).  start has nbins + 1 entries.
__global__ __launch_bounds__(1024) void k_scan_bins(const int32_t* __restrict__ count,
                                                    int32_t nbins, int32_t* __restrict__ start) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  const int seg = (nbins + 1023) / 1024;
  const int b0 = t * seg, b1 = min(b0 + seg, nbins);
  int32_t s = 0;
  for (int b = b0; b < b1; ++b) s += count[b];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int32_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = part[t] - s;
  for (int b = b0; b < b1; ++b) {
    start[b] = run;
    run += count[b];
  }
  if (t == 1023) start[nbins] = part[1023];
}

// The same exclusive scan for many bins, coalesced, in three launches:
// k_scan_tiles sums tiles of `tile` counts, k_scan_bins scans the tile sums,
// k_scan_apply scans each tile in passes of 256 from its tile's offset.
__global__ __launch_bounds__(256) void k_scan_tiles(const int32_t* __restrict__ count,
                                                    int32_t nbins, int32_t tile,
                                                    int32_t* __restrict__ sums) {
  __shared__ int32_t ws[4];
  const int64_t b0 = (int64_t)blockIdx.x * tile, b1 = min(b0 + (int64_t)tile, (int64_t)nbins);
  int32_t v = 0;
  for (int64_t q = b0 + threadIdx.x; q < b1; q += 256) v += count[q];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (lane_id() == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) sums[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(256) void k_scan_apply(const int32_t* __restrict__ count,
                                                    int32_t nbins, int32_t tile,
                                                    const int32_t* __restrict__ offs,
                                                    int32_t* __restrict__ start) {
  __shared__ int32_t ws[4];
  const int64_t b0 = (int64_t)blockIdx.x * tile, b1 = min(b0 + (int64_t)tile, (int64_t)nbins);
  const int w = (int)(threadIdx.x >> 6), l = (int)lane_id();
  int32_t run = offs[blockIdx.x];
  for (int64_t base = b0; base < b1; base += 256) {
    const int64_t q = base + threadIdx.x;
    const int32_t v = q < b1 ? count[q] : 0;
    int32_t x = v;  // inclusive scan within the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t y = __shfl_up(x, off);
      if (l >= off) x += y;
    }
    if (l == 63) ws[w] = x;
    __syncthreads();
    int32_t wo = 0;
    for (int q2 = 0; q2 < w; ++q2) wo += ws[q2];
    const int32_t total = ws[0] + ws[1] + ws[2] + ws[3];
    if (q < b1) start[q] = run + wo + x - v;
    __syncthreads();
    run += total;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) start[nbins] = run;
}

__global__ __launch_bounds__(256) void k_occupied(const int32_t* __restrict__ start, int32_t nbins,
                                                  uint32_t* __restrict__ occ, int32_t* cnt) {
  __shared__ int lds[8];
  for (uint32_t base = blockIdx.x * 256u; base < (uint32_t)nbins; base += gridDim.x * 256u) {
    const uint32_t b = base + threadIdx.x;
    const bool nz = b < (uint32_t)nbins && start[b + 1] > start[b];
    block_append1(nz, b, (gwptr<uint32_t>)occ, cnt, lds);
  }
}

template <int DIM>
__global__ void k_scatter_points(const double* __restrict__ pts, int64_t n,
                                 const int32_t* __restrict__ pt_bin,
                                 const int32_t* __restrict__ start, int32_t* __restrict__ fill,
                                 double* __restrict__ sorted) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int b = pt_bin[p];
    if (b < 0) continue;
    const int slot = start[b] + atomicAdd(&fill[b], 1);
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) sorted[(int64_t)slot * DIM + ax] = pts[p * DIM + ax];
  }
}

__device__ __forceinline__ double block_min(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (lane_id() == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
  for (int q = 1; q < (int)(blockDim.x >> 6); ++q) r = fmin(r, red[q]);
  return r;
}

// One bin's frame as a whole (see GEO).
struct Frame {
  double w[GEO];
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// A unit vector along which points with (unnormalised) covariance C spread
// least: the eigenvector of the smallest eigenvalue, found from the closed
// form of the eigenvalues of a symmetric 2 x 2 or 3 x 3 matrix.  Degenerate
// spreads (a single point, a line, an isotropic cloud) fall back to the axis
// of least variance; the bounds that use it hold for any unit vector.
template <int DIM>
__device__ void least_spread(const double C[3][3], double nv[3]) {
  double v[3] = {0.0, 0.0, 0.0};
  if (DIM == 2) {
    const double a = C[0][0], b = C[0][1], c = C[1][1];
    const double lam = 0.5 * (a + c) - sqrt(0.25 * (a - c) * (a - c) + b * b);
    const double n1 = b * b + (lam - a) * (lam - a), n2 = (lam - c) * (lam - c) + b * b;
    if (n1 >= n2) {
      v[0] = b;
      v[1] = lam - a;
    } else {
      v[0] = lam - c;
      v[1] = b;
    }
  } else {
    const double p1 = C[0][1] * C[0][1] + C[0][2] * C[0][2] + C[1][2] * C[1][2];
    const double q = (C[0][0] + C[1][1] + C[2][2]) / 3.0;
    const double b0 = C[0][0] - q, b1 = C[1][1] - q, b2 = C[2][2] - q;
    const double p2 = b0 * b0 + b1 * b1 + b2 * b2 + 2.0 * p1;
    double lam = q;
    if (p2 > 0.0) {
      const double pp = sqrt(p2 / 6.0);
      const double det = b0 * (b1 * b2 - C[1][2] * C[1][2]) -
                         C[0][1] * (C[0][1] * b2 - C[1][2] * C[0][2]) +
                         C[0][2] * (C[0][1] * C[1][2] - b1 * C[0][2]);
      const double r = fmin(fmax(det / (2.0 * pp * pp * pp), -1.0), 1.0);
      lam = q + 2.0 * pp * cos(acos(r) / 3.0 + 2.0943951023931957);  // + 2 pi / 3
    }
    const double M[3][3] = {{C[0][0] - lam, C[0][1], C[0][2]},
                            {C[0][1], C[1][1] - lam, C[1][2]},
                            {C[0][2], C[1][2], C[2][2] - lam}};
    double best = -1.0;
#pragma unroll
    for (int q0 = 0; q0 < 3; ++q0) {
      const int ra = q0 == 2 ? 1 : 0, rb = q0 == 0 ? 1 : 2;
      const double x[3] = {M[ra][1] * M[rb][2] - M[ra][2] * M[rb][1],
                           M[ra][2] * M[rb][0] - M[ra][0] * M[rb][2],
                           M[ra][0] * M[rb][1] - M[ra][1] * M[rb][0]};
      const double n2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
      if (n2 > best) {
        best = n2;
        v[0] = x[0];
        v[1] = x[1];
        v[2] = x[2];
      }
    }
  }
  double n2 = 0.0;
#pragma unroll
  for (int ax = 0; ax < DIM; ++ax) n2 += v[ax] * v[ax];
  if (!(n2 > 0.0) || !isfinite(n2)) {
    int k = 0;
#pragma unroll
    for (int ax = 1; ax < DIM; ++ax)
      if (C[ax][ax] < C[k][k]) k = ax;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) v[ax] = ax == k ? 1.0 : 0.0;
    n2 = 1.0;
  }
  const double inv = 1.0 / sqrt(n2);
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) nv[ax] = ax < DIM ? v[ax] * inv : 0.0;
}

// Bounding frame (see GEO, slots 0 to 13) of the points p0 .. p1 - 1, by one
// wave; lane 0 writes it to G.
template <int DIM>
__device__ void wave_frame(const double* __restrict__ pts, int p0, int p1, double* G) {
  const int l = (int)lane_id();
  double m[3] = {0.0, 0.0, 0.0};
  for (int p = p0 + l; p < p1; p += 64)
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) m[ax] += pts[(int64_t)p * DIM + ax];
#pragma unroll
  for (int ax = 0; ax < DIM; ++ax) m[ax] = wave_sum(m[ax]) / (double)(p1 - p0);
  double C[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  for (int p = p0 + l; p < p1; p += 64) {
    double v[3];
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) v[ax] = pts[(int64_t)p * DIM + ax] - m[ax];
#pragma unroll
    for (int r = 0; r < DIM; ++r)
#pragma unroll
      for (int c = r; c < DIM; ++c) C[r][c] += v[r] * v[c];
  }
#pragma unroll
  for (int r = 0; r < DIM; ++r)
#pragma unroll
    for (int c = r; c < DIM; ++c) {
      C[r][c] = wave_sum(C[r][c]);
      C[c][r] = C[r][c];
    }
  double nv[3];
  least_spread<DIM>(C, nv);
  double tmin = INFINITY, tmax = -INFINITY, rt2 = 0.0, rf2 = 0.0, E[3] = {0.0, 0.0, 0.0};
  for (int p = p0 + l; p < p1; p += 64) {
    double v[3], a = 0.0, r2 = 0.0;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
      v[ax] = pts[(int64_t)p * DIM + ax] - m[ax];
      a += nv[ax] * v[ax];
      r2 += v[ax] * v[ax];
      E[ax] = fmax(E[ax], fabs(v[ax]));
    }
    double w2 = 0.0;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
      const double w = v[ax] - a * nv[ax];
      w2 += w * w;
    }
    tmin = fmin(tmin, a);
    tmax = fmax(tmax, a);
    rt2 = fmax(rt2, w2);
    rf2 = fmax(rf2, r2);
  }
  tmin = wave_min(tmin);
  tmax = wave_max(tmax);
  rt2 = wave_max(rt2);
  rf2 = wave_max(rf2);
#pragma unroll
  for (int ax = 0; ax < DIM; ++ax) E[ax] = wave_max(E[ax]);
  if (l == 0) {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      G[ax] = ax < DIM ? m[ax] : 0.0;
      G[3 + ax] = nv[ax];
      G[6 + ax] = ax < DIM ? E[ax] : 0.0;
    }
    G[9] = tmin;
    G[10] = tmax;
    G[11] = sqrt(rt2);
    G[12] = sqrt(rf2);
    int32_t* r = (int32_t*)(G + 13);
    r[0] = p0;
    r[1] = p1;
  }
}

// Frames of the occupied bins, one wave per bin.
template <int DIM>
__global__ __launch_bounds__(256) void k_bin_geo(const double* __restrict__ pts,
                                                 const int32_t* __restrict__ start,
                                                 const uint32_t* __restrict__ occ,
                                                 const int32_t* __restrict__ occ_cnt,
                                                 double* __restrict__ geo) {
  const int nocc = *occ_cnt;
  const int nw = (int)(gridDim.x * (blockDim.x >> 6));
  for (int t = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)); t < nocc; t += nw) {
    const uint32_t id = occ[t];
    wave_frame<DIM>(pts, start[id], start[id + 1], geo + (size_t)t * GEO);
  }
}

// Occupied super-bins.  The occupied list holds a super-bin's bins as one
// run (ids of a super-bin are consecutive and k_occupied keeps the order of
// ids within each aligned chunk of 256, a multiple of ksup); the thread at
// the head of a run appends (head, end).
__global__ __launch_bounds__(256) void k_super_list(int ksup, const uint32_t* __restrict__ occ,
                                                    const int32_t* __restrict__ occ_cnt,
                                                    int2* __restrict__ sup, int32_t* sup_cnt) {
  const int nocc = *occ_cnt;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nocc; t += gridDim.x * blockDim.x) {
    const uint32_t S = occ[t] / (uint32_t)ksup;
    if (t > 0 && occ[t - 1] / (uint32_t)ksup == S) continue;
    int t1 = t + 1;
    while (t1 < nocc && occ[t1] / (uint32_t)ksup == S) ++t1;
    sup[atomicAdd(sup_cnt, 1)] = make_int2(t, t1);
  }
}

// Frames of the occupied super-bins, one wave per super-bin: its points are
// those of its bins, which are contiguous in the sorted cloud.
template <int DIM>
__global__ __launch_bounds__(256) void k_super_geo(const double* __restrict__ pts,
                                                   const int32_t* __restrict__ start,
                                                   const uint32_t* __restrict__ occ,
                                                   const int2* __restrict__ sup,
                                                   const int32_t* __restrict__ sup_cnt,
                                                   double* __restrict__ sgeo) {
  const int nsup = *sup_cnt;
  const int nw = (int)(gridDim.x * (blockDim.x >> 6));
  for (int u = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)); u < nsup; u += nw) {
    const int2 r = sup[u];
    double* G = sgeo + (size_t)u * GEO;
    wave_frame<DIM>(pts, start[occ[r.x]], start[occ[r.y - 1] + 1], G);
    if (lane_id() == 0) *(int2*)(G + 14) = r;
  }
}

// Lower bound of |x - p|^2 over the points p of a bin with frame G (see
// GEO), each of its two parts lowered by mu, which covers the rounding of
// the frame and of this evaluation.
template <int DIM>
__device__ __forceinline__ double frame_lb2(const double* G, const double x[3], double mu) {
  double v[3], a = 0.0;
#pragma unroll
  for (int ax = 0; ax < DIM; ++ax) {
    v[ax] = x[ax] - G[ax];
    a += G[3 + ax] * v[ax];
  }
  double w2 = 0.0;
#pragma unroll
  for (int ax = 0; ax < DIM; ++ax) {
    const double w = v[ax] - a * G[3 + ax];
    w2 += w * w;
  }
  const double gn = fmax(fmax(G[9] - a, a - G[10]), 0.0) - mu;
  const double gt = sqrt(w2) - G[11] - mu;
  const double un = fmax(gn, 0.0), ut = fmax(gt, 0.0);
  return un * un + ut * ut;
}

// Node (li, lj, lk) of the brick that thread threadIdx.x takes as its u-th
// node.  3D: 512 nodes, two per thread, a wave's 128 nodes forming a
// 4 x 4 x 8 box (nodes that are close together agree on the bins they can
// skip); 2D: 16^2 nodes, one per thread.
template <int DIM>
__device__ __forceinline__ void dist_node(int u, int& li, int& lj, int& lk) {
  if (DIM == 3) {
    const int w = (int)(threadIdx.x >> 6), l = (int)(threadIdx.x & 63);
    li = 4 * (w >> 1) + 2 * u + (l >> 5);
    lj = 4 * (w & 1) + ((l >> 3) & 3);
    lk = l & 7;
  } else {
    li = (int)threadIdx.x >> 4;
    lj = (int)threadIdx.x & 15;
    lk = 0;
  }
}

// Exact distance to the cloud at the nodes of one brick (8^3 nodes in 3D,
// 16^2 in 2D) per workgroup.  With c the brick centre, e its half extents
// and rho its half diagonal:
//  1. d(c) and a point p* that attains it are found exactly: the points of
//     the bin whose frame comes closest to c, within the super-bin whose
//     frame does, give an upper bound; then the points of every bin whose
//     frame bound does not exceed it, within a super-bin whose frame bound
//     does not either, are scanned;
//  2. a bin can hold a point y closer to a node x of the brick than p* only
//     if its frame meets the ball (c, d(c) + 2 rho), and only if
//     |c - y|^2 - |c - p*|^2 <= 2 sum_k e_k |y_k - p*_k| (|x - y|^2 -
//     |x - p*|^2 is linear in x, so its least value over the brick's box is
//     attained at a corner).  Super-bins are tested first and the bins of
//     those that pass next; the bins that pass, the candidates, are ordered
//     by their frame's distance from c in NSH shells (counting sort), so
//     that nodes meet close points first;
//  3. every node starts from |x - p*|, and a wave scans a candidate's points
//     only if one of its nodes could still find a closer point there by the
//     frame bound.
// The minimum is taken over all pairs that can attain it, so the result
// does not depend on the order.  All distance arithmetic in double.
template <int DIM>
// Registers held to 7 waves per SIMD (71 VGPRs, a few scalar values kept in
// vector lanes), the occupancy the LDS allows: the kernel is latency-bound.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) void k_distance(
    DistArgs a) {
  // no FMA contraction: node coordinates lo + i h and the sums of squares are
  // rounded exactly as the plain definition states them
#pragma clang fp contract(off)
  constexpr int NPT = DIM == 3 ? 2 : 1;
  // LDS: CAP + SCAP ints and a few words, about 21 KB (7 blocks of 4 waves
  // per CU)
  constexpr int CAP = 4608, SCAP = 512, NSH = 32;
  __shared__ double red[4];
  __shared__ uint32_t cand[CAP];
  __shared__ int slist[SCAP];
  __shared__ int ncand, nsl, ndc, pstar, ubest;
  __shared__ int shell_n[NSH], shell_at[NSH];
  const DevGrid& g = a.g;
  if (a.bmark && !a.bmark[blockIdx.x]) return;  // a brick the caller left out
  const int nbx = dist_bricks_along(DIM, 0, g.n0), nby = dist_bricks_along(DIM, 1, g.n1);
  const int nbz = dist_bricks_along(DIM, 2, g.n2);
  int b = blockIdx.x;
  const int bz = b % nbz;
  b /= nbz;
  const int by = b % nby, bx = b / nby;
  if (bx >= nbx) return;
  const int f[3] = {bx * dist_brick_extent(DIM, 0), by * dist_brick_extent(DIM, 1),
                    DIM == 3 ? bz * dist_brick_extent(DIM, 2) : 0};
  const int l[3] = {min(f[0] + dist_brick_extent(DIM, 0), g.n0) - 1,
                    min(f[1] + dist_brick_extent(DIM, 1), g.n1) - 1,
                    DIM == 3 ? min(f[2] + dist_brick_extent(DIM, 2), g.n2) - 1 : 0};
  const double glo[3] = {g.lo0, g.lo1, g.lo2};
  double c[3], e[3], rho2 = 0.0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    c[ax] = ax < DIM ? glo[ax] + g.hd * 0.5 * (f[ax] + l[ax]) : 0.0;
    e[ax] = 0.5 * g.hd * (l[ax] - f[ax]);
    rho2 += e[ax] * e[ax];
  }
  const double rho = sqrt(rho2);
  const int nocc = *a.occ_cnt, nsup = *a.sup_cnt;
  const double slack = 1.0 + 1e-12;
  const double mu = a.mu;
  const int tid = (int)threadIdx.x, wv = tid >> 6, ln = (int)lane_id();

  // 1. the super-bin whose frame bound from c is least (smallest index on
  // ties) ...
  double lmin = INFINITY;
  int umin = INT_MAX;
  for (int u = tid; u < nsup; u += blockDim.x) {
    const double v = frame_lb2<DIM>(a.sgeo + (size_t)u * GEO, c, mu);
    if (v < lmin) {
      lmin = v;
      umin = u;
    }
  }
  if (tid == 0) {
    ubest = INT_MAX;
    pstar = INT_MAX;
    nsl = 0;
    ndc = 0;
  }
  const double lbest = block_min(lmin, red);  // synchronises the block
  if (umin != INT_MAX && lmin == lbest) atomicMin(&ubest, umin);
  __syncthreads();
  // ... and its bin whose frame bound is least, whose points bound d(c)
  // from above (a lane per bin of the super-bin: ksup <= 64)
  double best = INFINITY;
  int bidx = -1;
  auto scan_c = [&](int p0, int p1, int first, int step) {
    for (int q = p0 + first; q < p1; q += step) {
      double s2 = 0.0;
#pragma unroll
      for (int ax = 0; ax < DIM; ++ax) {
        const double t2 = a.pts[(int64_t)q * DIM + ax] - c[ax];
        s2 += t2 * t2;
      }
      if (s2 < best) {
        best = s2;
        bidx = q;
      }
    }
  };
  if (ubest != INT_MAX && wv == 0) {
    const int2 r = *(const int2*)(a.sgeo + (size_t)ubest * GEO + 14);
    const int t = r.x + ln;
    double v = INFINITY;
    if (t < r.y) v = frame_lb2<DIM>(a.geo + (size_t)t * GEO, c, mu);
    const double vmin = wave_min(v);
    const uint64_t m = __ballot(t < r.y && v == vmin);
    const int tb = r.x + (m ? (int)__builtin_ctzll(m) : 0);
    const int2 rb = *(const int2*)(a.geo + (size_t)tb * GEO + 13);
    scan_c(rb.x, rb.y, ln, 64);
  }
  const double ub2 = block_min(best, red) * slack;
  // every other super-bin whose frame bound does not exceed that ...
  for (int u = tid; u < nsup; u += blockDim.x) {
    if (frame_lb2<DIM>(a.sgeo + (size_t)u * GEO, c, mu) > ub2) continue;
    const int pos = atomicAdd(&nsl, 1);
    if (pos < SCAP) slist[pos] = u;
  }
  __syncthreads();
  const int ns_dc = nsl;
  if (ns_dc <= SCAP) {
    // ... and of those, the bins whose frame bound does not (a wave per
    // super-bin, a lane per bin of it: ksup <= 64)
    for (int q = wv; q < ns_dc; q += (int)(blockDim.x >> 6)) {
      const int2 r = *(const int2*)(a.sgeo + (size_t)slist[q] * GEO + 14);
      const int t = r.x + ln;
      if (t >= r.y || frame_lb2<DIM>(a.geo + (size_t)t * GEO, c, mu) > ub2) continue;
      const int pos = atomicAdd(&ndc, 1);
      if (pos < CAP) cand[pos] = (uint32_t)t;
    }
    __syncthreads();
  }
  const int nd = ndc;
  if (ns_dc <= SCAP && nd <= CAP) {
    // a wave per listed bin, its lanes over the bin's points
    for (int q = wv; q < nd; q += (int)(blockDim.x >> 6)) {
      const int2 r = *(const int2*)(a.geo + (size_t)cand[q] * GEO + 13);
      scan_c(r.x, r.y, ln, 64);
    }
  } else if (ns_dc <= SCAP) {
    // too many bins to list: every point of the listed super-bins
    for (int q = 0; q < ns_dc; ++q) {
      const int2 r = *(const int2*)(a.sgeo + (size_t)slist[q] * GEO + 13);
      scan_c(r.x, r.y, tid, blockDim.x);
    }
  } else {
    for (int u = tid; u < nsup; u += blockDim.x) {
      if (frame_lb2<DIM>(a.sgeo + (size_t)u * GEO, c, mu) > ub2) continue;
      const int2 r = *(const int2*)(a.sgeo + (size_t)u * GEO + 13);
      scan_c(r.x, r.y, 0, 1);
    }
  }
  const double bmin = block_min(best, red);  // synchronises the block
  if (bidx >= 0 && best == bmin) atomicMin(&pstar, bidx);
  // the values of the whole block from here on sit in scalar registers
  best = uniform_value(bmin);
  const double R = sqrt(best) + 2.0 * rho;
  const double R2 = R * R * slack;
  if (tid < NSH) shell_n[tid] = 0;
  if (tid == 0) {
    ncand = 0;
    nsl = 0;
  }
  __syncthreads();

  // 2. candidates
  const int ps = uniform_value(pstar);
  const bool havep = ps != INT_MAX;
  double P[3] = {0.0, 0.0, 0.0};
  if (havep)
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) P[ax] = uniform_value(a.pts[(int64_t)ps * DIM + ax]);
  // every candidate frame lies at least d(c) - (bin diagonal) from c
  const double s0 = fmax(sqrt(best) - a.bg.bw * sqrt((double)DIM), 0.0);
  const double shell_scale = NSH / fmax(R - s0, 1e-300);
  // the test of step 2 for a frame G; *lbc = its bound from c
  auto passes = [&](const double* G, double* lbc) -> bool {
    const double lb2 = frame_lb2<DIM>(G, c, mu);
    *lbc = lb2;
    if (lb2 > R2) return false;
    if (!havep) return true;
    // sum_k e_k max_y |y_k - p*_k| over the frame's points y
    double w = 0.0;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) w += e[ax] * (fabs(G[ax] - P[ax]) + G[6 + ax] + mu);
    return !(lb2 - best - 2.0 * w > a.mu2);
  };
  auto shell_of = [&](double lb2) {
    const int k = (int)((sqrt(lb2) - s0) * shell_scale);
    return k < 0 ? 0 : (k > NSH - 1 ? NSH - 1 : k);
  };
  for (int u = tid; u < nsup; u += blockDim.x) {
    double lb2;
    if (!passes(a.sgeo + (size_t)u * GEO, &lb2)) continue;
    const int pos = atomicAdd(&nsl, 1);
    if (pos < SCAP) slist[pos] = u;
  }
  __syncthreads();
  const int ns_pass = nsl;
  if (ns_pass <= SCAP) {
    // a wave per passing super-bin, a lane per bin of it (ksup <= 64)
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = wv; q < ns_pass; q += (int)(blockDim.x >> 6)) {
        const int2 r = *(const int2*)(a.sgeo + (size_t)slist[q] * GEO + 14);
        const int t = r.x + ln;
        double lb2;
        if (t >= r.y || !passes(a.geo + (size_t)t * GEO, &lb2)) continue;
        const int sh = shell_of(lb2);
        if (pass == 0) {
          atomicAdd(&shell_n[sh], 1);
          atomicAdd(&ncand, 1);
        } else {
          const int pos = atomicAdd(&shell_at[sh], 1);
          if (pos < CAP) cand[pos] = (uint32_t)t;
        }
      }
      __syncthreads();
      if (pass == 0 && tid == 0) {
        int run = 0;
        for (int q = 0; q < NSH; ++q) {
          shell_at[q] = run;
          run += shell_n[q];
        }
      }
      __syncthreads();
    }
  } else if (tid == 0) {
    ncand = CAP + 1;  // too many super-bins to list: step 3 walks every bin
  }
  __syncthreads();
  const int nc = ncand;

  double x[NPT][3], bn[NPT];
  bool valid[NPT];
#pragma unroll
  for (int u = 0; u < NPT; ++u) {
    int li, lj, lk;
    dist_node<DIM>(u, li, lj, lk);
    const int node[3] = {f[0] + li, f[1] + lj, f[2] + lk};
    valid[u] = node[0] <= l[0] && node[1] <= l[1] && node[2] <= l[2];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) x[u][ax] = ax < DIM ? glo[ax] + node[ax] * g.hd : 0.0;
    // start from the distance to the centre's nearest point, one of the
    // pairs the minimum runs over
    bn[u] = INFINITY;
    if (havep) {
      double s2 = 0.0;
#pragma unroll
      for (int ax = 0; ax < DIM; ++ax) {
        const double t2 = x[u][ax] - P[ax];
        s2 += t2 * t2;
      }
      bn[u] = s2;
    }
  }
  // 3. A wave passes over a candidate when none of its nodes can find a
  // closer point in it by the frame bound.
  typedef const __attribute__((address_space(4))) double cdouble;
  cdouble* pts4 = (cdouble*)a.pts;
  auto visit = [&](const Frame& F) {
    bool need = false;
#pragma unroll
    for (int u = 0; u < NPT; ++u)
      need = need || (valid[u] && frame_lb2<DIM>(F.w, x[u], mu) <= bn[u] * slack);
    if (!__any(need)) return;
    const int2 rng = *(const int2*)(F.w + 13);
    // the same point for the whole block, read through the scalar unit,
    // LSR_DIST_PTS points per trip
    auto fold = [&](const double* Q) {
#pragma unroll
      for (int u = 0; u < NPT; ++u) {
        double s2 = 0.0;
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
          const double t2 = x[u][ax] - Q[ax];
          s2 += t2 * t2;
        }
        bn[u] = fmin(bn[u], s2);
      }
    };
    constexpr int PT = LSR_DIST_PTS;  // points per trip
    int p = rng.x;
    for (; p + PT - 1 < rng.y; p += PT) {
      double Q[PT][3];
#pragma unroll
      for (int r = 0; r < PT; ++r)
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) Q[r][ax] = pts4[(int64_t)(p + r) * DIM + ax];
#pragma unroll
      for (int r = 0; r < PT; ++r) fold(Q[r]);
    }
    for (; p < rng.y; ++p) {
      double Q0[3];
#pragma unroll
      for (int ax = 0; ax < DIM; ++ax) Q0[ax] = pts4[(int64_t)p * DIM + ax];
      fold(Q0);
    }
  };
  const Frame* frames = (const Frame*)a.geo;
  if (nc <= CAP) {
    // the sorted candidates; each frame is the same for the whole block and
    // read through the scalar unit, the next one while this one is used
    if (nc > 0) {
      Frame F = uniform_load(frames, (int)__builtin_amdgcn_readfirstlane(cand[0]));
      for (int q = 0; q < nc; ++q) {
        Frame Fn;
        if (q + 1 < nc) Fn = uniform_load(frames, (int)__builtin_amdgcn_readfirstlane(cand[q + 1]));
        visit(F);
        F = Fn;
      }
    }
  } else if (ns_pass <= SCAP) {
    // too many candidates to list: the bins of the super-bins that passed,
    // with the test of step 2, unsorted
    for (int q = 0; q < ns_pass; ++q) {
      const int2 r = *(const int2*)(a.sgeo + (size_t)slist[q] * GEO + 14);
      for (int t = r.x; t < r.y; ++t) {
        double lb2;
        if (passes(a.geo + (size_t)t * GEO, &lb2)) visit(uniform_load(frames, t));
      }
    }
  } else {
    // too many super-bins as well: every occupied bin, with the same test
    for (int t = 0; t < nocc; ++t) {
      double lb2;
      if (passes(a.geo + (size_t)t * GEO, &lb2)) visit(uniform_load(frames, t));
    }
  }
#pragma unroll
  for (int u = 0; u < NPT; ++u) {
    if (!valid[u]) continue;
    int li, lj, lk;
    dist_node<DIM>(u, li, lj, lk);
    a.d64[lin(g, f[0] + li, f[1] + lj, f[2] + lk)] = sqrt(bn[u]);
  }
}

// ------------------------------------------------------------ energy

// Energy functional of Section 3.5 over the front cells, the cells whose
// vertices do not all lie on one side of the front (inside: phi < 0):
//  2D (eq. energyApprox): the trapezoidal rule on the segment between the
//     zeros of the linear interpolants of phi on the crossed edges, with d
//     interpolated linearly along the edge there; a cell crossed on all four
//     edges gets two segments, which leave the centre (phi = mean of the
//     corners) on the side of corner (i, j) when the two agree;
//  3D (eq. energyApproxFiner): R^3 subcells of side h' = h / R per front
//     cell; a subcell whose trilinear phi at its centre is below
//     (sqrt 3 / 2) h' in magnitude adds |d|^p h'^2, d trilinear as well.
// All in double, without FMA contraction.
__device__ __forceinline__ double lerp_d(double a, double b, double t) { return a + t * (b - a); }

// |x|^p, with the common exponents exact to rounding and without pow
__device__ __forceinline__ double pow_abs(double x, double p) {
  const double a = fabs(x);
  return p == 2.0 ? a * a : (p == 1.0 ? a : pow(a, p));
}

// Corners of a 2D cell in edge order: (i,j), (i+1,j), (i+1,j+1), (i,j+1).
__device__ double energy_cell_2d(const DevGrid& g, const double f[4], const double e[4], int i,
                                 int j, double p) {
#pragma clang fp contract(off)
  const int ci[4] = {i, i + 1, i + 1, i}, cj[4] = {j, j, j + 1, j + 1};
  bool in[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) in[q] = f[q] < 0.0;
  double px[4], py[4], pd[4];
  bool has[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = (q + 1) & 3;
    has[q] = in[q] != in[r];
    px[q] = py[q] = pd[q] = 0.0;
    if (!has[q]) continue;
    const double t = f[q] / (f[q] - f[r]);
    px[q] = g.lo0 + g.hd * lerp_d((double)ci[q], (double)ci[r], t);
    py[q] = g.lo1 + g.hd * lerp_d((double)cj[q], (double)cj[r], t);
    pd[q] = lerp_d(e[q], e[r], t);
  }
  int a0 = -1, b0 = -1, a1 = -1, b1 = -1;
  if (has[0] && has[1] && has[2] && has[3]) {
    const double centre = 0.25 * (f[0] + f[1] + f[2] + f[3]);
    if ((centre < 0.0) == in[0]) {
      a0 = 0; b0 = 1; a1 = 2; b1 = 3;  // segments cut off corners 1 and 3
    } else {
      a0 = 3; b0 = 0; a1 = 1; b1 = 2;  // segments cut off corners 0 and 2
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (has[q]) {
        if (a0 < 0) a0 = q; else b0 = q;
      }
  }
  auto seg = [&](int a, int b) {
    const double L = hypot(px[a] - px[b], py[a] - py[b]);
    return L * 0.5 * (pow_abs(pd[a], p) + pow_abs(pd[b], p));
  };
  double s = seg(a0, b0);
  if (a1 >= 0) s += seg(a1, b1);
  return s;
}

// Sum over the subcells (3D) or segments (2D) of the cells whose vertex
// values are staged in F, E (and lower corners in IJ), n of them, one thread
// per (cell, subcell row u) in 3D, per cell in 2D; tt: the R subcell centres
// (w + 1/2) / R.  Added to s in a fixed order; in 3D the |d|^p of each line
// of R subcells are summed first and scaled by h'^2 once.
template <int DIM, int NV, int CAP>
__device__ __forceinline__ void energy_staged(const DevGrid& g, const double (&F)[CAP][NV],
                                              const double (&E)[CAP][NV], const int (&IJ)[CAP][2],
                                              int n, const double* tt, double p, int R, double& s) {
#pragma clang fp contract(off)
  const double hs = g.hd / R;
  const double lim = 0.5 * sqrt(3.0) * hs;
  const double hs2 = hs * hs;  // each subcell adds |d|^p h'^2
  if (DIM == 3) {
    for (int it = (int)threadIdx.x; it < n * R; it += 256) {
      const int cell = it / R, u = it - cell * R;
      const double* f = F[cell];
      const double* e = E[cell];
      // trilinear: along x, then y, then z; vertex (a, b, c') at 4a + 2b + c'
      const double tx = tt[u];
      const double f0 = lerp_d(f[0], f[4], tx), f2 = lerp_d(f[2], f[6], tx);
      const double f1 = lerp_d(f[1], f[5], tx), f3 = lerp_d(f[3], f[7], tx);
      const double e0 = lerp_d(e[0], e[4], tx), e2 = lerp_d(e[2], e[6], tx);
      const double e1 = lerp_d(e[1], e[5], tx), e3 = lerp_d(e[3], e[7], tx);
      for (int v = 0; v < R; ++v) {
        const double ty = tt[v];
        const double fz0 = lerp_d(f0, f2, ty), fz1 = lerp_d(f1, f3, ty);
        const double ez0 = lerp_d(e0, e2, ty), ez1 = lerp_d(e1, e3, ty);
        // lerp_d(a, b, t) = a + t (b - a), with b - a taken once per line
        const double fd = fz1 - fz0, ed = ez1 - ez0;
        double line = 0.0;
        for (int w = 0; w < R; ++w) {
          const double tz = tt[w];
          if (fabs(fz0 + tz * fd) < lim) line += pow_abs(ez0 + tz * ed, p);
        }
        s += line * hs2;
      }
    }
  } else {
    for (int it = (int)threadIdx.x; it < n; it += 256)
      s += energy_cell_2d(g, F[it], E[it], IJ[it][0], IJ[it][1], p);
  }
}

// Offset of vertex q of the cell with lower corner at node idx: 3D vertex
// (i+a, j+b, k+c') at q = 4a + 2b + c'; 2D edge order.
template <int DIM>
__device__ __forceinline__ uint32_t vertex_offset(const DevGrid& g, int q) {
  return DIM == 3 ? (uint32_t)(q >> 2) * g.s0 + (uint32_t)((q >> 1) & 1) * g.s1 + (uint32_t)(q & 1)
                  : (uint32_t)(q == 1 || q == 2) * g.s0 + (uint32_t)(q >= 2) * g.s1;
}

// Block b of nb (256 threads, called by all of them) sums the front cells of
// the whole grid: chunks of CAP cells, one lower-corner node per thread, with
// a stride of nb chunks; the front cells of a chunk are compacted into the
// caller's LDS arrays in lane order with their vertex values.  Returns the
// block's sum (in every thread), in a fixed order.
template <int DIM, typename T, int CAP>
__device__ double energy_grid_block(const DevGrid& g, const T* __restrict__ phi,
                                    const double* __restrict__ d, double p, int R, uint32_t b,
                                    uint32_t nb, double (&fv)[CAP][DIM == 3 ? 8 : 4],
                                    double (&ev)[CAP][DIM == 3 ? 8 : 4], int (&cij)[CAP][2],
                                    double* tt, int* wcnt, double* red) {
  constexpr int NV = DIM == 3 ? 8 : 4;
  const int tid = (int)threadIdx.x, wv = tid >> 6;
  if (tid < R) tt[tid] = (tid + 0.5) / R;
  const uint32_t m0 = (uint32_t)g.n0 - 1u, m1 = (uint32_t)g.n1 - 1u;
  const uint32_t m2 = DIM == 3 ? (uint32_t)g.n2 - 1u : 1u;
  const uint64_t ncell = (uint64_t)m0 * m1 * m2;
  double s = 0.0;
  for (uint64_t base = (uint64_t)b * CAP; base < ncell; base += (uint64_t)nb * CAP) {
    const uint64_t c = base + (uint64_t)tid;
    bool front = false;
    int i = 0, j = 0;
    uint32_t node = 0;
    T f[NV];
    if (tid < CAP && c < ncell) {
      const int k = (int)(c % m2);
      const uint64_t r = c / m2;
      j = (int)(r % m1);
      i = (int)(r / m1);
      node = (uint32_t)i * g.s0 + (uint32_t)j * g.s1 + (uint32_t)k;
      int n_in = 0;
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        f[q] = phi[node + vertex_offset<DIM>(g, q)];
        n_in += (double)f[q] < 0.0 ? 1 : 0;
      }
      front = n_in != 0 && n_in != NV;
    }
    const uint64_t m = __ballot(front);
    if (lane_id() == 0) wcnt[wv] = (int)__popcll(m);
    __syncthreads();
    int off = 0;
    for (int q = 0; q < wv; ++q) off += wcnt[q];
    const int nfront = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    if (front) {
      const int pos = off + (int)lanes_below(m);
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        fv[pos][q] = (double)f[q];
        ev[pos][q] = d[node + vertex_offset<DIM>(g, q)];
      }
      cij[pos][0] = i;
      cij[pos][1] = j;
    }
    __syncthreads();
    energy_staged<DIM, NV, CAP>(g, fv, ev, cij, nfront, tt, p, R, s);
    __syncthreads();
  }
  s = wave_sum(s);
  if (lane_id() == 0) red[wv] = s;
  __syncthreads();
  const double t = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  return t;
}

// Energy functional over the whole grid: block b's sum to partial[b].
template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_energy(DevGrid g, const T* __restrict__ phi,
                                                const double* __restrict__ d, double p, int R,
                                                double* __restrict__ partial) {
  constexpr int NV = DIM == 3 ? 8 : 4;
  __shared__ double fv[256][NV], ev[256][NV];
  __shared__ int cij[256][2];
  __shared__ double tt[64];
  __shared__ int wcnt[4];
  __shared__ double red[4];
  const double t = energy_grid_block<DIM, T, 256>(g, phi, d, p, R, blockIdx.x, gridDim.x, fv, ev,
                                                  cij, tt, wcnt, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Front cells of one word of a row of lower corners (see the sign words in
// lsr_device.h): unit = row * W + w, rows (i, j) with i < n0 - 1, j < n1 - 1
// in 3D (cells at k = 32 w + t), rows i < n0 - 1 in 2D (cells at j = 32 w +
// t).  Bit t is set where the cell's vertex bits are neither all 1 nor all 0;
// (i, j) and the first k (2D: j) of the word are returned.
template <int DIM>
__device__ __forceinline__ uint32_t front_word(const DevGrid& g, const uint32_t* __restrict__ sgn,
                                               uint32_t unit, int& i, int& j, int& kb) {
  const int nl = DIM == 3 ? g.n2 : g.n1;  // nodes along the rows
  const uint32_t W = sign_row_words(nl);
  const uint32_t row = unit / W, w = unit - row * W;
  uint32_t r[4];  // the words of the rows of the cells' vertices
  if (DIM == 3) {
    j = (int)(row % (uint32_t)(g.n1 - 1));
    i = (int)(row / (uint32_t)(g.n1 - 1));
    r[0] = ((uint32_t)i * (uint32_t)g.n1 + (uint32_t)j) * W + w;
    r[1] = r[0] + W;                       // (i, j + 1)
    r[2] = r[0] + (uint32_t)g.n1 * W;      // (i + 1, j)
    r[3] = r[2] + W;                       // (i + 1, j + 1)
  } else {
    i = (int)row;
    j = 0;
    r[0] = row * W + w;
    r[1] = r[0] + W;  // row i + 1
  }
  kb = (int)(32u * w);
  uint32_t all = ~0u, any = 0u;
#pragma unroll
  for (int q = 0; q < (DIM == 3 ? 4 : 2); ++q) {
    const uint32_t x = sgn[r[q]];
    const uint32_t nx = w + 1u < W ? sgn[r[q] + 1] : 0u;
    const uint32_t x1 = (x >> 1) | (nx << 31);  // bit t: the node one further along
    all &= x & x1;
    any |= x | x1;
  }
  const int nc = nl - 1 - kb;  // cells left in the row from kb on
  const uint32_t valid = nc >= 32 ? ~0u : (1u << nc) - 1u;
  return any & ~all & valid;
}

// The energy functional over every front cell of the grid, found from the
// sign words.  Word units are dealt out in groups of 8 consecutive units
// (thread t of block b takes unit r0 + ((t / 8) gridDim.x + b) 8 + t mod 8
// in round r0), so that neighbouring threads read neighbouring words and
// every block gets a share of every part of the front; per round the
// block's front cells are numbered in (thread, bit) order, listed in LDS
// and staged with their vertex values STAGE at a time, and summed.  The
// block's sum goes to partial[b] in a fixed order.
template <int DIM, typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_energy_front(DevGrid g, const T* __restrict__ phi,
                                                      const double* __restrict__ d, double p, int R,
                                                      const uint32_t* __restrict__ sgn,
                                                      double* __restrict__ partial) {
  constexpr int NV = DIM == 3 ? 8 : 4;
  constexpr int STAGE = 256;
  __shared__ double fv[STAGE][NV], ev[STAGE][NV];
  __shared__ int cij[STAGE][2];
  __shared__ uint32_t lst[STAGE];
  __shared__ double tt[64];
  __shared__ int wsum[4];
  __shared__ double red[4];
  const int tid = (int)threadIdx.x, wv = tid >> 6, lane = (int)lane_id();
  if (tid < R) tt[tid] = (tid + 0.5) / R;
  const uint32_t W = sign_row_words(DIM == 3 ? g.n2 : g.n1);
  const uint64_t units =
      (uint64_t)(DIM == 3 ? (uint32_t)(g.n0 - 1) * (uint32_t)(g.n1 - 1) : (uint32_t)(g.n0 - 1)) * W;
  const uint64_t G = gridDim.x;
  double s = 0.0;
  for (uint64_t r0 = 0; r0 < units; r0 += 256u * G) {
    const uint64_t u = r0 + ((uint64_t)(tid >> 3) * G + blockIdx.x) * 8u + (uint64_t)(tid & 7);
    uint32_t f = 0;
    int i = 0, j = 0, kb = 0;
    if (u < units) f = front_word<DIM>(g, sgn, (uint32_t)u, i, j, kb);
    // exclusive prefix of the counts over the block
    const int c = __popc(f);
    int x = c;
#pragma unroll
    for (int dd = 1; dd < 64; dd <<= 1) {
      const int y = __shfl_up(x, dd, 64);
      if (lane >= dd) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int off = x - c, total = 0;
    for (int q = 0; q < 4; ++q) {
      off += q < wv ? wsum[q] : 0;
      total += wsum[q];
    }
    for (int base = 0; base < total; base += STAGE) {
      // this thread's cells with numbers in [base, base + STAGE) to the list
      if (c && off < base + STAGE && off + c > base) {
        uint32_t bits = f;
        for (int pos = off - base; bits; ++pos) {
          const int t = __ffs(bits) - 1;
          bits &= bits - 1u;
          if (pos >= 0 && pos < STAGE)
            lst[pos] = DIM == 3 ? encode(g, i, j, kb + t) : encode(g, i, kb + t, 0);
        }
      }
      __syncthreads();
      const int nr = min(STAGE, total - base);
      if (tid < nr) {
        int ci, cj, ck;
        decode(g, lst[tid], ci, cj, ck);
        const uint32_t idx = lin(g, ci, cj, ck);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          const uint32_t o = vertex_offset<DIM>(g, q);
          fv[tid][q] = (double)phi[idx + o];
          ev[tid][q] = d[idx + o];
        }
        cij[tid][0] = ci;
        cij[tid][1] = cj;
      }
      __syncthreads();
      energy_staged<DIM, NV, STAGE>(g, fv, ev, cij, nr, tt, p, R, s);
      __syncthreads();
    }
  }
  s = wave_sum(s);
  if (lane == 0) red[wv] = s;
  __syncthreads();
  if (tid == 0) partial[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Sign words from scratch: one wave per 64 nodes of a row (two words), the
// bits from a ballot.
template <typename T>
__global__ __launch_bounds__(256) void k_sign_build(DevGrid g, const T* __restrict__ phi,
                                                    uint32_t* __restrict__ sgn) {
  const bool d3 = g.n2 > 1;
  const int nl = d3 ? g.n2 : g.n1;
  const uint32_t W = sign_row_words(nl);
  const uint32_t segs = ((uint32_t)nl + 63u) / 64u;
  const uint32_t rows = d3 ? (uint32_t)g.n0 * (uint32_t)g.n1 : (uint32_t)g.n0;
  const uint64_t total = (uint64_t)rows * segs;
  const uint32_t lane = lane_id();
  for (uint64_t q = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6); q < total;
       q += (uint64_t)gridDim.x * 4u) {
    const uint32_t row = (uint32_t)(q / segs), m = (uint32_t)(q - (uint64_t)row * segs);
    const uint32_t t = 64u * m + lane;  // position along the row
    // rows are contiguous in memory
    const bool neg = t < (uint32_t)nl && phi[row * (uint32_t)nl + t] < T(0);
    const uint64_t bits = __ballot(neg);
    const uint32_t w = 2u * m + lane;
    if (lane < 2 && w < W) sgn[(uint64_t)row * W + w] = (uint32_t)(bits >> (32u * lane));
  }
}

// Sum of the n partial sums in a fixed order, and its p-th root: out[0] = E_p.
__global__ __launch_bounds__(256) void k_energy_final(const double* __restrict__ partial, int n,
                                                      double p, double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int q = threadIdx.x; q < n; q += blockDim.x) s += partial[q];
  s = wave_sum(s);
  if (lane_id() == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = ((red[0] + red[1]) + red[2]) + red[3];
    out[0] = pow(t, 1.0 / p);
  }
}

// Centred gradient of d (one-sided on the boundary), in double, packed with
// d itself: dp = (d_x, d_y, d_z, d) in the state's precision (d_z = 0 in 2D).
template <int DIM, typename P>
__global__ void k_dpack(DevGrid g, const double* __restrict__ d, P* __restrict__ dp) {
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.N;
       idx += gridDim.x * blockDim.x) {
    uint32_t r = idx;
    int k = 0;
    if (DIM == 3) {
      k = (int)(r % (uint32_t)g.n2);
      r /= (uint32_t)g.n2;
    }
    const int j = (int)(r % (uint32_t)g.n1), i = (int)(r / (uint32_t)g.n1);
    const int ci[3] = {i, j, k};
    const int nn[3] = {g.n0, g.n1, g.n2};
    const uint32_t st[3] = {g.s0, g.s1, 1u};
    const double v = d[idx];
    double gr[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
      const bool hm = ci[ax] > 0, hp = ci[ax] < nn[ax] - 1;
      if (hm && hp)
        gr[ax] = (d[idx + st[ax]] - d[idx - st[ax]]) / (2.0 * g.hd);
      else if (hp)
        gr[ax] = (d[idx + st[ax]] - v) / g.hd;
      else
        gr[ax] = (v - d[idx - st[ax]]) / g.hd;
    }
    typedef decltype(dp->x) E;
    P out;
    out.x = (E)gr[0];
    out.y = (E)gr[1];
    out.z = (E)gr[2];
    out.w = (E)v;
    dp[idx] = out;
  }
}

// ------------------------------------------------------------ launchers

static inline unsigned grid_for(uint64_t n, unsigned block, unsigned cap) {
  uint64_t b = (n + block - 1) / block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, uint8_t v, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_init_phi(int dim, const DevGrid& g, int kind, const double* args, T gamma,
                           const T* src, T* A, T* B, int32_t* flag, hipStream_t s) {
  dim3 gr(grid_for(g.N, 256, 8192)), bl(256);
  if (dim == 3)
    hipLaunchKernelGGL((k_init_phi<3, T>), gr, bl, 0, s, g, kind, args[0], args[1], args[2],
                       args[3], args[4], gamma, src, A, B, flag);
  else
    hipLaunchKernelGGL((k_init_phi<2, T>), gr, bl, 0, s, g, kind, args[0], args[1], args[2],
                       args[3], args[4], gamma, src, A, B, flag);
  return hipGetLastError();
}

// The three launches of a list from a grid scan (see GbarArgs).
template <typename T>
hipError_t launch_grid_list(int dim, const GbarArgs<T>& a, unsigned blocks, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (a.smark) {
    e = persistent_launch(dim == 3 ? k_mark_slots<3, T> : k_mark_slots<2, T>, blocks, s, a);
    if (e != hipSuccess) return e;
  }
  e = persistent_launch(dim == 3 ? k_grid_scan<3, T> : k_grid_scan<2, T>, blocks, s, a);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_slot_prefix<T>, dim3(1), dim3(1024), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return persistent_launch(k_slot_pack<T>, blocks, s, a);
}

template <typename T>
hipError_t launch_band_mask(const DevGrid& g, T gamma, const T* A, const uint32_t* L,
                            const int32_t* ccnt, const int32_t* cnt, uint8_t* mask,
                            int32_t* count, unsigned blocks, hipStream_t s) {
  return persistent_launch(k_band_mask<T>, blocks, s, g, gamma, A, L, ccnt, cnt, mask, count);
}

template <typename T>
hipError_t launch_reinit_fix(int dim, const RArgs<T>& a, unsigned blocks, hipStream_t s) {
  return persistent_launch(dim == 3 ? k_reinit_fix<3, T> : k_reinit_fix<2, T>, blocks, s, a);
}

template <typename T>
hipError_t launch_reinit_iter(int dim, const RArgs<T>& a, unsigned blocks, hipStream_t s) {
  return persistent_launch(dim == 3 ? k_reinit_iter<3, T> : k_reinit_iter<2, T>, blocks, s, a);
}

template <typename T>
hipError_t launch_reinit_final(const FinArgs<T>& a, unsigned blocks, hipStream_t s) {
  return persistent_launch(k_reinit_final<T>, blocks, s, a);
}

hipError_t launch_bin_points(int dim, const BinGeom& bg, const double* pts, int64_t n,
                             int32_t* bin_count, int32_t* pt_bin, int32_t* flag,
                             int32_t* occupied, hipStream_t s) {
  dim3 gr(grid_for((uint64_t)n, 256, 4096)), bl(256);
  if (dim == 3)
    hipLaunchKernelGGL(k_bin_points<3>, gr, bl, 0, s, bg, pts, n, bin_count, pt_bin, flag,
                       occupied);
  else
    hipLaunchKernelGGL(k_bin_points<2>, gr, bl, 0, s, bg, pts, n, bin_count, pt_bin, flag,
                       occupied);
  return hipGetLastError();
}

hipError_t launch_scan_bins(const int32_t* count, int32_t nbins, int32_t* start, int32_t* tmp,
                            hipStream_t s) {
  if (nbins <= SCAN_ONE_BLOCK) {
    hipLaunchKernelGGL(k_scan_bins, dim3(1), dim3(1024), 0, s, count, nbins, start);
    return hipGetLastError();
  }
  // at most SCAN_TILES tiles of a multiple of 256 counts, at least 1024
  const int64_t per = ((int64_t)nbins + SCAN_TILES - 1) / SCAN_TILES;
  const int32_t tile = (int32_t)std::max<int64_t>(1024, (per + 255) / 256 * 256);
  const int32_t ntiles = (int32_t)(((int64_t)nbins + tile - 1) / tile);
  int32_t* sums = tmp;
  int32_t* offs = tmp + SCAN_TILES;
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(256), 0, s, count, nbins, tile, sums);
  hipLaunchKernelGGL(k_scan_bins, dim3(1), dim3(1024), 0, s, sums, ntiles, offs);
  hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(256), 0, s, count, nbins, tile, offs, start);
  return hipGetLastError();
}

hipError_t launch_occupied(const int32_t* start, int32_t nbins, uint32_t* occ, int32_t* cnt,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_occupied, dim3(grid_for((uint64_t)nbins, 256, 4096)), dim3(256), 0, s,
                     start, nbins, occ, cnt);
  return hipGetLastError();
}

hipError_t launch_scatter_points(int dim, const double* pts, int64_t n, const int32_t* pt_bin,
                                 const int32_t* start, int32_t* fill, double* sorted,
                                 hipStream_t s) {
  dim3 gr(grid_for((uint64_t)n, 256, 4096)), bl(256);
  if (dim == 3)
    hipLaunchKernelGGL(k_scatter_points<3>, gr, bl, 0, s, pts, n, pt_bin, start, fill, sorted);
  else
    hipLaunchKernelGGL(k_scatter_points<2>, gr, bl, 0, s, pts, n, pt_bin, start, fill, sorted);
  return hipGetLastError();
}

hipError_t launch_bin_geo(int dim, const double* pts, const int32_t* start, const uint32_t* occ,
                          const int32_t* occ_cnt, double* geo, int64_t max_occ, hipStream_t s) {
  // one wave per bin, four per block, the grid walking the list if longer
  dim3 gr(grid_for((uint64_t)max_occ, 4, 4096)), bl(256);
  if (dim == 3)
    hipLaunchKernelGGL(k_bin_geo<3>, gr, bl, 0, s, pts, start, occ, occ_cnt, geo);
  else
    hipLaunchKernelGGL(k_bin_geo<2>, gr, bl, 0, s, pts, start, occ, occ_cnt, geo);
  return hipGetLastError();
}

hipError_t launch_super_list(const BinGeom& bg, const uint32_t* occ, const int32_t* occ_cnt,
                             int2* sup, int32_t* sup_cnt, int64_t max_occ, hipStream_t s) {
  hipLaunchKernelGGL(k_super_list, dim3(grid_for((uint64_t)max_occ, 256, 4096)), dim3(256), 0, s,
                     bg.ksup, occ, occ_cnt, sup, sup_cnt);
  return hipGetLastError();
}

hipError_t launch_super_geo(int dim, const double* pts, const int32_t* start,
                            const uint32_t* occ, const int2* sup, const int32_t* sup_cnt,
                            double* sgeo, int64_t max_sup, hipStream_t s) {
  dim3 gr(grid_for((uint64_t)max_sup, 4, 4096)), bl(256);
  if (dim == 3)
    hipLaunchKernelGGL(k_super_geo<3>, gr, bl, 0, s, pts, start, occ, sup, sup_cnt, sgeo);
  else
    hipLaunchKernelGGL(k_super_geo<2>, gr, bl, 0, s, pts, start, occ, sup, sup_cnt, sgeo);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_energy_front(int dim, const DevGrid& g, const T* phi, const double* d, double p,
                               int R, const uint32_t* sgn, double* partial, double* out,
                               hipStream_t s) {
  dim3 gr(ENERGY_BLOCKS), bl(256);
  if (dim == 3)
    hipLaunchKernelGGL((k_energy_front<3, T>), gr, bl, 0, s, g, phi, d, p, R, sgn, partial);
  else
    hipLaunchKernelGGL((k_energy_front<2, T>), gr, bl, 0, s, g, phi, d, p, R, sgn, partial);
  if (out)
    hipLaunchKernelGGL(k_energy_final, dim3(1), bl, 0, s, (const double*)partial,
                       (int)ENERGY_BLOCKS, p, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sign_build(const DevGrid& g, const T* phi, uint32_t* sgn, hipStream_t s) {
  const bool d3 = g.n2 > 1;
  const int nl = d3 ? g.n2 : g.n1;
  const uint64_t waves = (uint64_t)(d3 ? (uint64_t)g.n0 * g.n1 : (uint64_t)g.n0) * ((nl + 63) / 64);
  const unsigned blocks = (unsigned)std::min<uint64_t>((waves + 3) / 4, 16384);
  hipLaunchKernelGGL((k_sign_build<T>), dim3(blocks), dim3(256), 0, s, g, phi, sgn);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_energy(int dim, const DevGrid& g, const T* phi, const double* d, double p, int R,
                         double* partial, double* out, hipStream_t s) {
  dim3 gr(ENERGY_BLOCKS), bl(256);
  if (dim == 3)
    hipLaunchKernelGGL((k_energy<3, T>), gr, bl, 0, s, g, phi, d, p, R, partial);
  else
    hipLaunchKernelGGL((k_energy<2, T>), gr, bl, 0, s, g, phi, d, p, R, partial);
  hipLaunchKernelGGL(k_energy_final, dim3(1), bl, 0, s, (const double*)partial, (int)ENERGY_BLOCKS,
                     p, out);
  return hipGetLastError();
}

hipError_t launch_distance(int dim, const DistArgs& a, unsigned bricks, hipStream_t s) {
  if (dim == 3)
    hipLaunchKernelGGL(k_distance<3>, dim3(bricks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_distance<2>, dim3(bricks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dpack(int dim, const DevGrid& g, const double* d, typename Vec<T>::pack* dp,
                        hipStream_t s) {
  typedef typename Vec<T>::pack P;
  dim3 gr(grid_for(g.N, 256, 8192)), bl(256);
  if (dim == 3)
    hipLaunchKernelGGL((k_dpack<3, P>), gr, bl, 0, s, g, d, dp);
  else
    hipLaunchKernelGGL((k_dpack<2, P>), gr, bl, 0, s, g, d, dp);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_grid_list_batch(int dim, const GbarArgs<T>* tab, int n, unsigned blocks,
                                  hipStream_t s, bool marked) {
  hipError_t e = hipSuccess;
  if (marked) {
    e = persistent_launch(dim == 3 ? k_mark_slots_batch<3, T> : k_mark_slots_batch<2, T>, blocks,
                          s, tab, n);
    if (e != hipSuccess) return e;
  }
  e = persistent_launch(dim == 3 ? k_grid_scan_batch<3, T> : k_grid_scan_batch<2, T>, blocks, s,
                        tab, n);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_slot_prefix_batch<T>, dim3(n), dim3(1024), 0, s, tab);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return persistent_launch(k_slot_pack_batch<T>, blocks, s, tab, n);
}

template <typename T>
hipError_t launch_reinit_fix_batch(int dim, const RArgs<T>* tab, int n, unsigned blocks,
                                   hipStream_t s) {
  return persistent_launch(dim == 3 ? k_reinit_fix_batch<3, T> : k_reinit_fix_batch<2, T>, blocks, s,
                           tab, n);
}

template <typename T>
hipError_t launch_reinit_iter_batch(int dim, const RArgs<T>* tab, int n, unsigned blocks,
                                    hipStream_t s) {
  return persistent_launch(dim == 3 ? k_reinit_iter_batch<3, T> : k_reinit_iter_batch<2, T>, blocks,
                           s, tab, n);
}

template <typename T>
hipError_t launch_reinit_final_batch(const FinArgs<T>* tab, int n, unsigned blocks, hipStream_t s) {
  return persistent_launch(k_reinit_final_batch<T>, blocks, s, tab, n);
}

#define LSR_INSTANTIATE(T)                                                                        \
  template hipError_t launch_init_phi<T>(int, const DevGrid&, int, const double*, T, const T*, T*, \
                                         T*, int32_t*, hipStream_t);                              \
  template hipError_t launch_grid_list<T>(int, const GbarArgs<T>&, unsigned, hipStream_t);        \
  template hipError_t launch_band_mask<T>(const DevGrid&, T, const T*, const uint32_t*,           \
                                          const int32_t*, const int32_t*, uint8_t*, int32_t*,     \
                                          unsigned, hipStream_t);                                 \
  template hipError_t launch_reinit_fix<T>(int, const RArgs<T>&, unsigned, hipStream_t);          \
  template hipError_t launch_reinit_iter<T>(int, const RArgs<T>&, unsigned, hipStream_t);         \
  template hipError_t launch_reinit_final<T>(const FinArgs<T>&, unsigned, hipStream_t);           \
  template hipError_t launch_dpack<T>(int, const DevGrid&, const double*, typename Vec<T>::pack*, \
                                      hipStream_t);                                               \
  template hipError_t launch_grid_list_batch<T>(int, const GbarArgs<T>*, int, unsigned,           \
                                                hipStream_t, bool);                               \
  template hipError_t launch_reinit_fix_batch<T>(int, const RArgs<T>*, int, unsigned, hipStream_t);\
  template hipError_t launch_reinit_iter_batch<T>(int, const RArgs<T>*, int, unsigned,             \
                                                  hipStream_t);                                   \
  template hipError_t launch_reinit_final_batch<T>(const FinArgs<T>*, int, unsigned, hipStream_t);\
  template hipError_t launch_energy_front<T>(int, const DevGrid&, const T*, const double*, double,  \
                                             int, const uint32_t*, double*, double*, hipStream_t); \
  template hipError_t launch_sign_build<T>(const DevGrid&, const T*, uint32_t*, hipStream_t);      \
  template hipError_t launch_energy<T>(int, const DevGrid&, const T*, const double*, double, int,  \
                                       double*, double*, hipStream_t);

LSR_INSTANTIATE(float)
LSR_INSTANTIATE(double)

}  // namespace lsr
