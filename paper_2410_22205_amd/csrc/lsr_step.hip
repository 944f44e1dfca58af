// The semi-Lagrangian step kernels of the narrow-band level-set solver for
// gfx950 (Preda & Semplice, arXiv:2410.22205, Section 3.1-3.2, eqs. (SL2d),
// (SL3d)) and their launchers: one job's band list, or the band lists of a
// batch of jobs.  The per-node update itself is sl_update (lsr_device.h).
#include "lsr_kern.h"

namespace lsr {

// ---------------------------------------------------------- the SL step

// One time step over the current band list: entries with |phi^n| < gamma get
// the update of eqs. (SL2d)/(SL3d) written to B; entries that left the band
// in the previous step get their value copied, so that A and B agree off
// the new list.  The new list is the set of entries updated here (the band
// of this step), chunk c of Lin compacted into chunk c of Lout.  LANES lanes
// share one entry (see sl_update).
//
// Each kernel below is a per-chunk body (one block, one chunk) driven either
// over one job's list or, in the batched kernels, over the chunks of all
// jobs of the table numbered one after the other; in both the chunks are
// shared out in contiguous stretches, one per XCD (xcd_share).

// 1 / E_2(phi^n) of a p = 2 step (the only p != 1 a step takes): every
// block adds the energy kernel's partial sums of E_2^2 in the same fixed
// order (so that every block, in the single-job and the batched kernels
// alike, takes the same value) and takes the square root; E_2 = 0 (no
// front) stops the motion (C = 0).  Called by all threads of the block with
// the field Epart of the step's arguments (null: p = 1, inv_E unused); red:
// 4 doubles of LDS.
template <typename T>
__device__ __forceinline__ T step_inv_energy(const double* Epart, double* red) {
  if (!Epart) return T(0);
  double s = 0.0;
  for (int q = (int)threadIdx.x; q < (int)ENERGY_BLOCKS; q += 256) s += Epart[q];
  // butterfly: the two lanes of every pair add the same two values
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  __syncthreads();  // red may still be read from the previous call
  if ((threadIdx.x & 63u) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double E = sqrt(((red[0] + red[1]) + red[2]) + red[3]);
  return uniform_value(E > 0.0 ? (T)(1.0 / E) : T(0));
}

template <int DIM, int INTERP, typename T, int LANES>
__device__ __forceinline__ void sl_chunk(const SLArgs<T>& a, T inv_E, uint32_t c, int* lds,
                                         uint32_t& nupd, uint32_t& nfb, uint32_t& nfr) {
  constexpr int CH = (int)LCHUNK / LANES;  // entries per round of the block
  StepConst<T> sc = a.c;
  sc.inv_E = inv_E;
  const gptr<T> A = (gptr<T>)a.A;
  const gwptr<T> B = (gwptr<T>)a.B;
  const gptr<typename Vec<T>::p4> DP = (gptr<typename Vec<T>::p4>)a.dp;
  const gptr<uint32_t> Lin = (gptr<uint32_t>)a.Lin + c * LCHUNK;
  const gwptr<uint32_t> Lout = (gwptr<uint32_t>)a.Lout + c * LCHUNK;
  const int nc = a.ccnt_in[c];
  const int sub = (int)(threadIdx.x % LANES);
  int kept = 0;
  for (int r = 0; r < LANES && r * CH < nc; ++r) {
    const int le = r * CH + (int)(threadIdx.x / LANES);
    bool act = false;
    int fl = 0;
    uint32_t code = 0;
    if (le < nc) {
      code = Lin[le];
      int i, j, k;
      decode(a.g, code, i, j, k);
      const uint32_t idx = lin(a.g, i, j, k);
      const T v = A[idx];
      T nv = v;
      if (fabs(v) < a.c.gamma) {
        act = true;
        nv = sl_update<DIM, INTERP, T, LANES>(A, a.g, sc, i, j, k, idx, v, DP[idx], sub, fl);
        if (sub == 0 && a.sgn && (nv < T(0)) != (v < T(0))) {
          uint32_t w, bit;
          sign_word_of(a.g, i, j, k, w, bit);
          sign_set(a.sgn, w, bit, nv < T(0));
        }
      }
      if (sub == 0) B[idx] = nv;
    }
    const bool lead = act && sub == 0;
    const bool p1[1] = {lead};
    const uint32_t v1[1] = {code};
    kept += block_compact<1>(p1, v1, Lout + kept, lds);
    nupd += wave_count(lead);
    nfb += wave_count(sub == 0 && (fl & UPD_FALLBACK));
    nfr += wave_count(sub == 0 && (fl & UPD_FRAME0));
  }
  if (threadIdx.x == 0) a.ccnt_out[c] = kept;
}

template <int DIM, int INTERP, typename T, int LANES>
__global__ __launch_bounds__(256) void k_sl_step(SLArgs<T> a) {
  __shared__ int lds[5];
  __shared__ uint32_t lds_st[12];
  __shared__ double red[4];
  const T inv_E = step_inv_energy<T>(a.Epart, red);
  const uint32_t nch = (uint32_t)*a.cnt_in;
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.cnt_out = (int32_t)nch;
  uint32_t nupd = 0, nfb = 0, nfr = 0;
  uint32_t c, end;
  const uint32_t step = xcd_share(nch, c, end);
  for (; c < end; c += step) sl_chunk<DIM, INTERP, T, LANES>(a, inv_E, c, lds, nupd, nfb, nfr);
  block_add3(nupd, nfb, nfr, a.stats, 0, 1, 2, lds_st);
}

// Batched step for the jobs of one interpolator (one launch per interpolator,
// so that each kernel keeps its own register count and resident grid).
template <int DIM, int INTERP, typename T, int LANES>
__global__ __launch_bounds__(256) void k_sl_step_batch(const SLArgs<T>* __restrict__ tab, int n) {
  __shared__ int lds[5];
  __shared__ uint32_t lds_st[12];
  __shared__ double red[4];
  if (blockIdx.x == 0)
    for (int t = (int)threadIdx.x; t < n; t += (int)blockDim.x) *tab[t].cnt_out = *tab[t].cnt_in;
  uint32_t nupd = 0, nfb = 0, nfr = 0;
  JobCursor cur{n};
  int cjob = -1;  // the job whose 1 / E_p inv_E holds
  T inv_E = T(0);
  auto leave = [&](int jb) {
    block_add3(nupd, nfb, nfr, LSR_FIELD(tab, jb, SLArgs<T>, stats), 0, 1, 2, lds_st);
    nupd = nfb = nfr = 0;
  };
  uint32_t c, end;
  const uint32_t step = xcd_share(total_chunks(tab, n), c, end);
  for (; c < end; c += step) {
    if (!cur.advance(tab, c, leave)) break;
    if (cur.jb != cjob) {
      inv_E = step_inv_energy<T>(LSR_FIELD(tab, cur.jb, SLArgs<T>, Epart), red);
      cjob = cur.jb;
    }
    sl_chunk<DIM, INTERP, T, LANES>(uniform_load(tab, cur.jb), inv_E, c - cur.beg, lds, nupd, nfb,
                                    nfr);
  }
  if (cur.jb >= 0 && cur.jb < n) leave(cur.jb);
}

template <typename T>
hipError_t launch_sl_step(int dim, int interp, int lanes, const SLArgs<T>& a, unsigned blocks,
                          hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  void (*k)(SLArgs<T>);
  if (dim == 3)
    k = lanes == 1 ? (interp == 0 ? k_sl_step<3, 0, T, 1> : k_sl_step<3, 1, T, 1>)
                   : (interp == 0 ? k_sl_step<3, 0, T, 4> : k_sl_step<3, 1, T, 4>);
  else
    k = lanes == 1 ? (interp == 0 ? k_sl_step<2, 0, T, 1> : k_sl_step<2, 1, T, 1>)
                   : (interp == 0 ? k_sl_step<2, 0, T, 2> : k_sl_step<2, 1, T, 2>);
  if (start) return persistent_launch_timed(k, blocks, s, start, stop, a);
  return persistent_launch(k, blocks, s, a);
}

template <typename T>
hipError_t launch_sl_step_batch(int dim, int interp, int lanes, const SLArgs<T>* tab, int n,
                                unsigned blocks, hipStream_t s) {
  void (*k)(const SLArgs<T>*, int);
  if (dim == 3)
    k = lanes == 1 ? (interp == 0 ? k_sl_step_batch<3, 0, T, 1> : k_sl_step_batch<3, 1, T, 1>)
                   : (interp == 0 ? k_sl_step_batch<3, 0, T, 4> : k_sl_step_batch<3, 1, T, 4>);
  else
    k = lanes == 1 ? (interp == 0 ? k_sl_step_batch<2, 0, T, 1> : k_sl_step_batch<2, 1, T, 1>)
                   : (interp == 0 ? k_sl_step_batch<2, 0, T, 2> : k_sl_step_batch<2, 1, T, 2>);
  return persistent_launch(k, blocks, s, tab, n);
}

#define LSR_INSTANTIATE_STEP(T)                                                                   \
  template hipError_t launch_sl_step<T>(int, int, int, const SLArgs<T>&, unsigned, hipStream_t,    \
                                        hipEvent_t, hipEvent_t);                                  \
  template hipError_t launch_sl_step_batch<T>(int, int, int, const SLArgs<T>*, int,               \
                                              unsigned, hipStream_t);

LSR_INSTANTIATE_STEP(float)
LSR_INSTANTIATE_STEP(double)

}  // namespace lsr
