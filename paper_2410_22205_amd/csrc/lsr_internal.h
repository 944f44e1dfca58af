// Internal interface between the C-ABI layer (lsr_api.hip, lsr_batch.hip)
// and the kernels (lsr_kernels.hip).  Not installed; the public interface is
// include/lsr.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lsr_device.h"

namespace lsr {

// Work statistics: each counter is spread over STAT_SLOTS slots a cache line
// apart (a block adds to slot blockIdx % STAT_SLOTS), so that the blocks of a
// launch do not all meet at one address; readers sum the slots.
constexpr int STAT_COUNTERS = 8, STAT_SLOTS = 64, STAT_STRIDE = 16;  // stride in 8-byte words
constexpr size_t STAT_WORDS = (size_t)STAT_COUNTERS * STAT_SLOTS * STAT_STRIDE;
__host__ __device__ inline size_t stat_index(int counter, int slot) {
  return ((size_t)counter * STAT_SLOTS + (size_t)slot) * STAT_STRIDE;
}

// Cloud bins: cubes of BIN_W nodes per side, or of BIN_W_FINE nodes for
// dense clouds (more than DENSE_BIN points per occupied BIN_W bin); the
// workspace holds the bins of the finer width.
constexpr int BIN_W = 4, BIN_W_FINE = 2, DENSE_BIN = 40;
// Bin-count scans: one block up to SCAN_ONE_BLOCK bins, else at most
// SCAN_TILES tiles (scratch of 2 * SCAN_TILES + 1 ints).
constexpr int32_t SCAN_ONE_BLOCK = 4096, SCAN_TILES = 1024;

// Bins are grouped in super-bins of SUP bins per axis (SUP^3 in 3D, SUP^2 in
// 2D), numbered so that the bins of one super-bin have consecutive ids:
// id = S * ksup + local, with S the super-bin's row-major index over ns[] and
// local the bin's row-major index inside it.  Sorting the points by bin id
// then also groups them by super-bin.
constexpr int SUP = 4;

struct BinGeom {
  int nb[3];        // bins per axis (nb[2] = 1 in 2D)
  int ns[3];        // super-bins per axis, ceil(nb / SUP) (ns[2] = 1 in 2D)
  int kz;           // SUP in 3D, 1 in 2D
  int ksup;         // bins per super-bin: SUP * SUP * kz
  double lo[3];     // grid box
  double hi[3];
  double bw, inv_bw;
};

// Bin id of bin coordinates b (see SUP).
__host__ __device__ inline int bin_id(const BinGeom& bg, const int b[3]) {
  const int S = ((b[0] / SUP) * bg.ns[1] + b[1] / SUP) * bg.ns[2] + b[2] / SUP;
  const int l = ((b[0] % SUP) * SUP + b[1] % SUP) * bg.kz + b[2] % SUP;
  return S * bg.ksup + l;
}
// Number of bin ids, super-bin padding included.
inline int32_t bin_ids(const BinGeom& bg) { return bg.ns[0] * bg.ns[1] * bg.ns[2] * bg.ksup; }

// Band lists are chunked: chunk c of a list holds its entries at
// [c * LCHUNK, c * LCHUNK + ccnt[c]) of the list buffer, and the list's
// counter slot holds its number of chunks.  A list is built in the order of
// a scan of the grid brick by brick (ordered compaction, no atomics); each
// step keeps the chunks of its input list and compacts every chunk in place
// into the output list, so the order, and with it the locality of the nodes
// a block or an XCD works on, lasts from one reinitialisation to the next.
constexpr uint32_t LCHUNK = 256;

template <typename T>
struct SLArgs {
  DevGrid g;
  StepConst<T> c;
  const T* A;                       // phi^n (read only)
  T* B;                             // phi^{n+1} (written on the list)
  const typename Vec<T>::pack* dp;  // (grad d, d)
  const uint32_t* Lin;              // band list of this step (chunked)
  uint32_t* Lout;                   // the entries updated here, chunk by chunk
  const int32_t* ccnt_in;           // entries per chunk of Lin
  int32_t* ccnt_out;                // entries per chunk of Lout
  const int32_t* cnt_in;            // chunks of Lin
  int32_t* cnt_out;                 // chunks of Lout (the same number)
  unsigned long long* stats;
  // when p = 2, the ENERGY_BLOCKS partial sums of E_2(phi^n)^2 that the
  // energy kernel leaves on the device before the step; p = 1: null
  const double* Epart;
  // sign words of phi (lsr_device.h), moved to phi^{n+1} where a node
  // changes side; null: left alone (a trial step)
  uint32_t* sgn;
};

// Grid scans in slots of GBAR_CHUNK nodes: in 3D a slot is 2 x 2 x 2 =
// GBAR_SUB bricks of SB0 x SB1 x SB2 = 256 nodes, slots numbered in C order
// of their coordinates, bricks in C order inside a slot and nodes in C
// order inside a brick; in 2D GBAR_CHUNK consecutive nodes.  Every band
// list follows this order, so a wave's 64 consecutive list entries are
// neighbours in the grid.
constexpr uint32_t GBAR_SUB = 8, GBAR_CHUNK = 256 * GBAR_SUB;
#ifndef LSR_SCAN_BRICK
#define LSR_SCAN_BRICK 2, 4, 32
#endif
constexpr uint32_t SCAN_BRICK[3] = {LSR_SCAN_BRICK};
constexpr uint32_t SB0 = SCAN_BRICK[0], SB1 = SCAN_BRICK[1], SB2 = SCAN_BRICK[2];
static_assert(SB0 * SB1 * SB2 == 256, "a scan brick is one workgroup's 256 nodes");

// Slots along an axis of n nodes with bricks b nodes long (3D).
__host__ __device__ inline uint32_t slots_along(uint32_t n, uint32_t b) {
  return ((n + b - 1) / b + 1) / 2;
}

__host__ __device__ inline uint32_t gbar_slots(int dim, int n0, int n1, int n2) {
  if (dim == 3)
    return slots_along((uint32_t)n0, SB0) * slots_along((uint32_t)n1, SB1) *
           slots_along((uint32_t)n2, SB2);
  return ((uint32_t)n0 * (uint32_t)n1 + GBAR_CHUNK - 1) / GBAR_CHUNK;
}
__host__ __device__ inline uint32_t gbar_slots(const DevGrid& g) {
  return gbar_slots(g.n2 > 1 ? 3 : 2, g.n0, g.n1, g.n2);
}

// A list from a scan of the grid: node x belongs to it iff |P| < gamma at x
// (nbr = 0: the band) or at x or a face neighbour (nbr = 1: Gbar, the band
// of the step and its face neighbours, with P = phi^n, the field whose band
// the step updated).  Three launches: each slot's members in node order into
// S at s * GBAR_CHUNK with their number in scnt[s]; the exclusive prefix of
// the counts into soff[0 .. slots] (one block per job); every slot's members
// copied to M at soff[s].  *cnt_out receives the length of M, or, when ccnt
// is given, M's number of LCHUNK chunks with their entries in ccnt.
// With smark, only the slots marked 1 are scanned (the others hold no
// member), and the scan clears every mark it reads (all marks are clear
// between builds); for Gbar the slots are marked from the band list L of the
// step: every node with |P| < gamma is on L, and a member of Gbar is such a
// node or its face neighbour.
template <typename T>
struct GbarArgs {
  DevGrid g;
  T gamma;
  int nbr;
  uint8_t* smark;        // null: every slot
  const uint32_t* L;     // with smark: the band list (chunked), its entries
  const int32_t* Lccnt;  // per chunk and its number of chunks
  const int32_t* Lcnt;
  const T* P;
  uint32_t* S;
  int32_t* scnt;
  int32_t* soff;
  uint32_t* M;
  int32_t* cnt_out;
  int32_t* ccnt;
};

template <typename T>
struct RArgs {
  DevGrid g;
  StepConst<T> c;
  const uint32_t* M;
  const int32_t* cnt;
  const T* src;
  T* dst;
  uint8_t* flags;
  T dtau;
  T floor_;
  unsigned long long* stats;
};

// Cut on Gbar (a compacted list of *cnt_in entries) and the new band list,
// chunked: Gbar's LCHUNK-entry chunk c gives chunk c of Lout.
template <typename T>
struct FinArgs {
  DevGrid g;
  T gamma;
  const uint32_t* M;
  const int32_t* cnt_in;
  T* cur;
  T* other;
  uint32_t* Lout;
  int32_t* ccnt_out;
  int32_t* cnt_out;
  uint32_t* sgn;  // sign words of phi, moved to the cut phi on Gbar
};

// Bounding frame of the points of one occupied bin, GEO doubles per bin at
// the bin's place t in the occupied list:
//   [0..2]  m, the mean of the points
//   [3..5]  nv, a unit vector along which the points spread least (any unit
//           vector keeps the bounds valid; this one makes them tight)
//   [6..8]  E, the largest |p_k - m_k| per axis
//   [9, 10] tmin, tmax, the range of nv . (p - m)
//   [11]    rt, the largest distance of p - m from the line along nv
//   [12]    rf, the largest |p - m|
//   [13]    the bin's point range, two int32 (begin, end)
//   [14]    super-bins only: the range of their bins in the occupied list,
//           two int32 (begin, end)
// For any x, with a = nv . (x - m) and tau the distance of x - m from that
// line, every point p of the bin has
//   |x - p|^2 >= gap(a, [tmin, tmax])^2 + max(tau - rt, 0)^2.
constexpr int GEO = 16;

// Bricks of the distance kernel, one workgroup each: 8^3 nodes in 3D (four
// waves, each a 4 x 4 x 8 box of two nodes per lane), 16 x 16 in 2D (one
// node per thread).  Bricks are numbered in C order.
__host__ __device__ constexpr int dist_brick_extent(int dim, int ax) {
  return dim == 3 ? 8 : (ax < 2 ? 16 : 1);
}
// Number of bricks per axis and in all.
__host__ __device__ constexpr int dist_bricks_along(int dim, int ax, int n) {
  const int b = dist_brick_extent(dim, ax);
  return ax < dim ? (n + b - 1) / b : 1;
}
inline size_t dist_bricks(int dim, int n0, int n1, int n2) {
  return (size_t)dist_bricks_along(dim, 0, n0) * dist_bricks_along(dim, 1, n1) *
         dist_bricks_along(dim, 2, n2);
}

struct DistArgs {
  DevGrid g;
  BinGeom bg;
  const double* pts;      // sorted by bin, dim doubles per point
  const int32_t* start;   // bin start offsets, nbins + 1
  const uint32_t* occ;    // occupied bin ids
  const int32_t* occ_cnt;
  const double* geo;      // GEO doubles per occupied bin
  const double* sgeo;     // GEO doubles per occupied super-bin
  const int32_t* sup_cnt; // occupied super-bins
  double mu;              // distance margin that covers rounding (1e-12 x box diagonal)
  double mu2;             // the same for squared distances (1e-12 x diagonal^2)
  double* d64;
  const uint8_t* bmark;   // null: every brick; else only the bricks marked 1
};

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, uint64_t n, hipStream_t s);
template <typename T>
hipError_t launch_init_phi(int dim, const DevGrid& g, int kind, const double* args, T gamma,
                           const T* src, T* A, T* B, int32_t* flag, hipStream_t s);
// The first band of a job (a.nbr = 0) or Gbar (a.nbr = 1), see GbarArgs.
template <typename T>
hipError_t launch_grid_list(int dim, const GbarArgs<T>& a, unsigned blocks, hipStream_t s);
// mask[idx] = 1 on the nodes of the chunked list L with |A| < gamma, *count
// += their number (mask may be null).
template <typename T>
hipError_t launch_band_mask(const DevGrid& g, T gamma, const T* A, const uint32_t* L,
                            const int32_t* ccnt, const int32_t* cnt, uint8_t* mask,
                            int32_t* count, unsigned blocks, hipStream_t s);
// lanes: 1, or the number of foot points per node (2 in 2D, 4 in 3D).
template <typename T>
hipError_t launch_sl_step(int dim, int interp, int lanes, const SLArgs<T>& a, unsigned blocks,
                          hipStream_t s, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
template <typename T>
hipError_t launch_reinit_fix(int dim, const RArgs<T>& a, unsigned blocks, hipStream_t s);
template <typename T>
hipError_t launch_reinit_iter(int dim, const RArgs<T>& a, unsigned blocks, hipStream_t s);
template <typename T>
hipError_t launch_reinit_final(const FinArgs<T>& a, unsigned blocks, hipStream_t s);
// bin_count[] counts the points per bin, *occupied the bins it makes
// non-empty; *flag |= 1 for a non-finite point or one outside the box.
hipError_t launch_bin_points(int dim, const BinGeom& bg, const double* pts, int64_t n,
                             int32_t* bin_count, int32_t* pt_bin, int32_t* flag,
                             int32_t* occupied, hipStream_t s);
// Exclusive scan of nbins counts into start[0 .. nbins] (tmp: scratch of
// 2 * SCAN_TILES + 1 ints).
hipError_t launch_scan_bins(const int32_t* count, int32_t nbins, int32_t* start, int32_t* tmp,
                            hipStream_t s);
hipError_t launch_occupied(const int32_t* start, int32_t nbins, uint32_t* occ, int32_t* cnt,
                           hipStream_t s);
hipError_t launch_scatter_points(int dim, const double* pts, int64_t n, const int32_t* pt_bin,
                                 const int32_t* start, int32_t* fill, double* sorted,
                                 hipStream_t s);
// Occupied super-bins: the runs of one super-bin's bins in the occupied
// list, appended to sup[] as (begin, end) with *sup_cnt counting them.
hipError_t launch_super_list(const BinGeom& bg, const uint32_t* occ, const int32_t* occ_cnt,
                             int2* sup, int32_t* sup_cnt, int64_t max_occ, hipStream_t s);
// Bounding frames (GEO doubles each) of the occupied bins, at most max_occ,
// and of the occupied super-bins, at most max_sup.
hipError_t launch_bin_geo(int dim, const double* pts, const int32_t* start, const uint32_t* occ,
                          const int32_t* occ_cnt, double* geo, int64_t max_occ, hipStream_t s);
hipError_t launch_super_geo(int dim, const double* pts, const int32_t* start,
                            const uint32_t* occ, const int2* sup, const int32_t* sup_cnt,
                            double* sgeo, int64_t max_sup, hipStream_t s);
hipError_t launch_distance(int dim, const DistArgs& a, unsigned bricks, hipStream_t s);
// Cloud resolution h_S: nearest-neighbour distances of the ns sampled points
// (indices into raw, the cloud in its given order) into nn[0 .. ns-1], their
// mean into out[0]; *flag |= 1 for an index outside [0, n_pts).  sorted and
// start: the cloud sorted by the bins of bg (lsr_cloud.hip).
hipError_t launch_cloud_spacing(int dim, const BinGeom& bg, const double* sorted,
                                const int32_t* start, const double* raw, int64_t n_pts,
                                const int64_t* sample, int64_t ns, double* nn, int32_t* flag,
                                double* out, hipStream_t s);
// Energy functional E_p of Section 3.5 (R subcells per axis in 3D) of the
// nodal phi and d: per-block sums into partial[ENERGY_BLOCKS], then
// out[0] = E_p.
constexpr unsigned ENERGY_BLOCKS = 1024;
// Subcells per axis of the energy that a p = 2 step computes (the paper's R)
constexpr int ENERGY_R = 5;
template <typename T>
hipError_t launch_energy(int dim, const DevGrid& g, const T* phi, const double* d, double p, int R,
                         double* partial, double* out, hipStream_t s);
// The same E_p from the sign words of phi (sgn, see lsr_device.h), which
// show every front cell of the grid 32 at a time; the front cells are
// shared out over ENERGY_BLOCKS blocks word by word.  Deterministic.  With
// out null only the partial sums are left (the p = 2 step reduces them).
template <typename T>
hipError_t launch_energy_front(int dim, const DevGrid& g, const T* phi, const double* d, double p,
                               int R, const uint32_t* sgn, double* partial, double* out,
                               hipStream_t s);
// The sign words of phi, built from scratch (fresh initial data).
template <typename T>
hipError_t launch_sign_build(const DevGrid& g, const T* phi, uint32_t* sgn, hipStream_t s);
template <typename T>
hipError_t launch_dpack(int dim, const DevGrid& g, const double* d, typename Vec<T>::pack* dp,
                        hipStream_t s);

// Initial data from the cloud (Section 3.6) and the approximate distance
// (Section 3.4), lsr_init.hip.  Passes set *changed = 1 when they change a
// node; a pass that changes nothing has reached the fixed point.
hipError_t launch_check_points(int dim, const BinGeom& bg, const double* pts, int64_t n,
                               int32_t* flag, hipStream_t s);
hipError_t launch_mark_init(int dim, const DevGrid& g, const double* d, double gs, uint8_t* ext,
                            hipStream_t s);
hipError_t launch_mark_pass(int dim, const DevGrid& g, const double* d, double gs, uint8_t* ext,
                            int32_t* changed, hipStream_t s);
hipError_t launch_eik_init(const DevGrid& g, const double* v, const uint8_t* fixed, double* u,
                           hipStream_t s);
hipError_t launch_eik_init_ext(const DevGrid& g, const double* d, double gs, const uint8_t* ext,
                               double* u, hipStream_t s);
hipError_t launch_eik_pass(int dim, const DevGrid& g, double* u, const uint8_t* fixed,
                           int32_t* changed, hipStream_t s);
template <typename T>
hipError_t launch_phi0_cloud(const DevGrid& g, const double* d, const double* u, const uint8_t* ext,
                             double gs, T gamma, T* A, T* B, hipStream_t s);
hipError_t launch_box_mark(int dim, const DevGrid& g, const double* pts, int64_t n, uint8_t* fixed,
                           uint8_t* bmark, hipStream_t s);
// Warm start (Section 4): src (phi on the coarser grid gc) interpolated at
// the nodes of g (interp 0: Q1, 1: WENO), cut to [-gamma, gamma], into A, B.
template <typename T>
hipError_t launch_resample(int dim, int interp, const DevGrid& g, const DevGrid& gc, const T* src,
                           T gamma, T weno_e, T* A, T* B, hipStream_t s);

// Batched forms: one launch over a packed table of per-job arguments.
template <typename T>
hipError_t launch_sl_step_batch(int dim, int interp, int lanes, const SLArgs<T>* tab, int n,
                                unsigned blocks, hipStream_t s);
// marked: the table's entries carry slot marks (all of them, or none).
template <typename T>
hipError_t launch_grid_list_batch(int dim, const GbarArgs<T>* tab, int n, unsigned blocks,
                                  hipStream_t s, bool marked);
template <typename T>
hipError_t launch_reinit_fix_batch(int dim, const RArgs<T>* tab, int n, unsigned blocks,
                                   hipStream_t s);
template <typename T>
hipError_t launch_reinit_iter_batch(int dim, const RArgs<T>* tab, int n, unsigned blocks,
                                    hipStream_t s);
template <typename T>
hipError_t launch_reinit_final_batch(const FinArgs<T>* tab, int n, unsigned blocks, hipStream_t s);

}  // namespace lsr
