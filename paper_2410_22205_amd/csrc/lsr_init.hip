// Initial data from the cloud (Section 3.6) and the paper's approximate
// distance field (Section 3.4) for gfx950 (Preda & Semplice,
// arXiv:2410.22205).
//
// Both need the first-order Godunov discretisation of |grad u| = 1 that
// Zhao's fast sweeping solves, with some nodes held fixed.  Its solution is
// the fixed point that every monotone iteration from above reaches, so here
// it is reached by tiled passes instead of sweeps in alternating orders:
// each block takes a tile of 4 x 8 x 8 nodes (16 x 16 in 2D) with a one-node
// halo in LDS and lowers the tile's values by Jacobi updates until they stop
// changing; passes repeat until one changes nothing.  The external marking of
// Section 3.6 (a flood from the boundary through nodes with d >= gamma_S) runs
// the same way on bytes.
#include "lsr_internal.h"

namespace lsr {

template <int DIM>
struct Tile;
template <>
struct Tile<3> {
  static constexpr int TI = 4, TJ = 8, TK = 8, HI = 6, HJ = 10, HK = 10;
};
template <>
struct Tile<2> {
  static constexpr int TI = 16, TJ = 16, TK = 1, HI = 18, HJ = 18, HK = 1;
};
constexpr int TILE_MAXIT = 64;  // Jacobi rounds per tile and pass

template <int DIM>
__device__ __forceinline__ uint32_t tile_count(const DevGrid& g) {
  typedef Tile<DIM> Q;
  return (uint32_t)((g.n0 + Q::TI - 1) / Q::TI) * (uint32_t)((g.n1 + Q::TJ - 1) / Q::TJ) *
         (uint32_t)((g.n2 + Q::TK - 1) / Q::TK);
}

// First node of tile t (tiles in C order of their coordinates).
template <int DIM>
__device__ __forceinline__ void tile_origin(const DevGrid& g, uint32_t t, int& i0, int& j0,
                                            int& k0) {
  typedef Tile<DIM> Q;
  const uint32_t nk = (uint32_t)((g.n2 + Q::TK - 1) / Q::TK), nj = (uint32_t)((g.n1 + Q::TJ - 1) / Q::TJ);
  k0 = (int)(t % nk) * Q::TK;
  t /= nk;
  j0 = (int)(t % nj) * Q::TJ;
  i0 = (int)(t / nj) * Q::TI;
}

// Halo entry e (0 .. HI*HJ*HK-1) as grid coordinates; false off the grid.
template <int DIM>
__device__ __forceinline__ bool halo_node(const DevGrid& g, int i0, int j0, int k0, int e, int& i,
                                          int& j, int& k) {
  typedef Tile<DIM> Q;
  const int lk = e % Q::HK, lj = (e / Q::HK) % Q::HJ, li = e / (Q::HK * Q::HJ);
  i = i0 + li - 1;
  j = j0 + lj - 1;
  k = DIM == 3 ? k0 + lk - 1 : 0;
  return i >= 0 && i < g.n0 && j >= 0 && j < g.n1 && k >= 0 && k < g.n2;
}

// The thread's node: its place in the halo array and grid coordinates.
template <int DIM>
__device__ __forceinline__ int tile_node(int i0, int j0, int k0, int& i, int& j, int& k) {
  typedef Tile<DIM> Q;
  const int t = (int)threadIdx.x;
  const int li = t / (Q::TJ * Q::TK), lj = (t / Q::TK) % Q::TJ, lk = t % Q::TK;
  i = i0 + li;
  j = j0 + lj;
  k = k0 + lk;
  return ((li + 1) * Q::HJ + lj + 1) * Q::HK + (DIM == 3 ? lk + 1 : 0);
}

// Section 3.6, external marking: ext = 1 on boundary nodes with d >= gamma_S,
// 0 elsewhere.
template <int DIM>
__global__ void k_mark_init(DevGrid g, const double* __restrict__ d, double gs,
                            uint8_t* __restrict__ ext) {
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.N;
       idx += gridDim.x * blockDim.x) {
    uint32_t r = idx;
    int k = 0;
    if (DIM == 3) {
      k = (int)(r % (uint32_t)g.n2);
      r /= (uint32_t)g.n2;
    }
    const int j = (int)(r % (uint32_t)g.n1), i = (int)(r / (uint32_t)g.n1);
    bool b = i == 0 || i == g.n0 - 1 || j == 0 || j == g.n1 - 1;
    if (DIM == 3) b = b || k == 0 || k == g.n2 - 1;
    ext[idx] = (b && d[idx] >= gs) ? 1 : 0;
  }
}

// One pass of the marking: inside each tile, nodes with d >= gamma_S that
// have an external face neighbour become external, until nothing changes.
template <int DIM>
__global__ __launch_bounds__(256) void k_mark_pass(DevGrid g, const double* __restrict__ d,
                                                   double gs, uint8_t* __restrict__ ext,
                                                   int32_t* changed) {
  typedef Tile<DIM> Q;
  constexpr int H = Q::HI * Q::HJ * Q::HK, SI = Q::HJ * Q::HK, SJ = Q::HK;
  __shared__ uint8_t e[H];
  const uint32_t nt = tile_count<DIM>(g);
  for (uint32_t t = blockIdx.x; t < nt; t += gridDim.x) {
    int i0, j0, k0;
    tile_origin<DIM>(g, t, i0, j0, k0);
    for (int q = (int)threadIdx.x; q < H; q += 256) {
      int i, j, k;
      e[q] = halo_node<DIM>(g, i0, j0, k0, q, i, j, k) ? ext[lin(g, i, j, k)] : 0;
    }
    int i, j, k;
    const int c = tile_node<DIM>(i0, j0, k0, i, j, k);
    const bool valid = i < g.n0 && j < g.n1 && k < g.n2;
    const uint32_t idx = valid ? lin(g, i, j, k) : 0;
    const bool open = valid && d[idx] >= gs;
    __syncthreads();
    bool mine = false;
    for (int it = 0; it < TILE_MAXIT; ++it) {
      bool nb = e[c - SI] | e[c + SI] | e[c - SJ] | e[c + SJ];
      if (DIM == 3) nb = nb | e[c - 1] | e[c + 1];
      const bool nw = open && !e[c] && nb;
      __syncthreads();
      if (nw) {
        e[c] = 1;
        mine = true;
      }
      if (!__syncthreads_or(nw)) break;
    }
    if (mine) ext[idx] = 1;
    if (__syncthreads_or(mine) && threadIdx.x == 0) *changed = 1;
  }
}

// Zhao's first-order Godunov update of |grad u| = 1 at a node from the
// smaller neighbour value along each axis (off the grid: +inf, no
// contribution), in the order and rounding of its plain statement: the
// one-dimensional solution, then the two- and three-dimensional ones when the
// previous exceeds the next smallest neighbour value.
__device__ __forceinline__ double eik_update(double a0, double a1, double a2, int dims, double h) {
#pragma clang fp contract(off)
  double m[3] = {a0, a1, a2};
  int n = 0;
  double s[3];
  for (int q = 0; q < dims; ++q)
    if (m[q] < INFINITY) s[n++] = m[q];
  for (int p = 0; p < n; ++p)
    for (int q = p + 1; q < n; ++q)
      if (s[q] < s[p]) {
        const double t = s[p];
        s[p] = s[q];
        s[q] = t;
      }
  if (n == 0) return INFINITY;
  double x = s[0] + h;
  if (n >= 2 && x > s[1]) {
    x = 0.5 * (s[0] + s[1] + sqrt(2.0 * h * h - (s[0] - s[1]) * (s[0] - s[1])));
    if (n >= 3 && x > s[2]) {
      const double sum = s[0] + s[1] + s[2];
      const double q = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
      x = (sum + sqrt(sum * sum - 3.0 * (q - h * h))) / 3.0;
    }
  }
  return x;
}

// u = v on fixed nodes, 1e30 (not yet reached) elsewhere; v = u allowed.
__global__ void k_eik_init(uint32_t N, const double* v, const uint8_t* __restrict__ fixed,
                           double* u) {
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N;
       idx += gridDim.x * blockDim.x)
    u[idx] = fixed[idx] ? v[idx] : 1e30;
}

// External marking to fixed values: u = d - gamma_S on external nodes.
__global__ void k_eik_init_ext(uint32_t N, const double* __restrict__ d, double gs,
                               const uint8_t* __restrict__ ext, double* __restrict__ u) {
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N;
       idx += gridDim.x * blockDim.x)
    u[idx] = ext[idx] ? d[idx] - gs : 1e30;
}

// One pass of the eikonal solve: every free node of a tile takes
// min(u, update of its neighbours), Jacobi rounds until the tile is still.
template <int DIM>
__global__ __launch_bounds__(256) void k_eik_pass(DevGrid g, double* __restrict__ u,
                                                  const uint8_t* __restrict__ fixed,
                                                  int32_t* changed) {
  typedef Tile<DIM> Q;
  constexpr int H = Q::HI * Q::HJ * Q::HK, SI = Q::HJ * Q::HK, SJ = Q::HK;
  __shared__ double v[H];
  const uint32_t nt = tile_count<DIM>(g);
  for (uint32_t t = blockIdx.x; t < nt; t += gridDim.x) {
    int i0, j0, k0;
    tile_origin<DIM>(g, t, i0, j0, k0);
    for (int q = (int)threadIdx.x; q < H; q += 256) {
      int i, j, k;
      v[q] = halo_node<DIM>(g, i0, j0, k0, q, i, j, k) ? u[lin(g, i, j, k)] : INFINITY;
    }
    int i, j, k;
    const int c = tile_node<DIM>(i0, j0, k0, i, j, k);
    const bool valid = i < g.n0 && j < g.n1 && k < g.n2;
    const uint32_t idx = valid ? lin(g, i, j, k) : 0;
    const bool free_ = valid && !fixed[idx];
    __syncthreads();
    bool mine = false;
    for (int it = 0; it < TILE_MAXIT; ++it) {
      bool nw = false;
      double x = 0.0;
      if (free_) {
        const double ax = fmin(v[c - SI], v[c + SI]), ay = fmin(v[c - SJ], v[c + SJ]);
        const double az = DIM == 3 ? fmin(v[c - 1], v[c + 1]) : INFINITY;
        x = eik_update(ax, ay, az, DIM, g.hd);
        nw = x < v[c];
      }
      __syncthreads();
      if (nw) {
        v[c] = x;
        mine = true;
      }
      if (!__syncthreads_or(nw)) break;
    }
    if (mine) u[idx] = v[c];
    if (__syncthreads_or(mine) && threadIdx.x == 0) *changed = 1;
  }
}

// phi0 of Section 3.6: d - gamma_S on external nodes, -u inside, cut to
// [-gamma, gamma], into both phi buffers.
template <typename T>
__global__ void k_phi0_cloud(uint32_t N, const double* __restrict__ d, const double* __restrict__ u,
                             const uint8_t* __restrict__ ext, double gs, T gamma,
                             T* __restrict__ A, T* __restrict__ B) {
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N;
       idx += gridDim.x * blockDim.x) {
    const double v = ext[idx] ? d[idx] - gs : -u[idx];
    const T w = fmin(fmax((T)v, -gamma), gamma);
    A[idx] = w;
    B[idx] = w;
  }
}

// Section 3.4: fixed = 1 at the nodes of the box of 4 nodes per axis around
// each point (the two nodes on either side of the cell holding it, clamped
// to the grid); bmark = 1 on the distance kernel's bricks that hold such
// nodes.
template <int DIM>
__global__ void k_box_mark(DevGrid g, const double* __restrict__ pts, int64_t n,
                           uint8_t* __restrict__ fixed, uint8_t* __restrict__ bmark) {
#pragma clang fp contract(off)
  const int B0 = dist_brick_extent(DIM, 0), B1 = dist_brick_extent(DIM, 1),
            B2 = dist_brick_extent(DIM, 2);
  const int nby = dist_bricks_along(DIM, 1, g.n1), nbz = dist_bricks_along(DIM, 2, g.n2);
  const int nn[3] = {g.n0, g.n1, g.n2};
  const double lo[3] = {g.lo0, g.lo1, g.lo2};
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    int a0[3] = {0, 0, 0}, a1[3] = {0, 0, 0};
    for (int ax = 0; ax < DIM; ++ax) {
      const int c = (int)floor((pts[q * DIM + ax] - lo[ax]) / g.hd);
      a0[ax] = c - 1 < 0 ? 0 : c - 1;
      a1[ax] = c + 2 > nn[ax] - 1 ? nn[ax] - 1 : c + 2;
    }
    for (int i = a0[0]; i <= a1[0]; ++i)
      for (int j = a0[1]; j <= a1[1]; ++j)
        for (int k = a0[2]; k <= a1[2]; ++k) fixed[lin(g, i, j, k)] = 1;
    for (int bi = a0[0] / B0; bi <= a1[0] / B0; ++bi)
      for (int bj = a0[1] / B1; bj <= a1[1] / B1; ++bj)
        for (int bk = a0[2] / B2; bk <= a1[2] / B2; ++bk) bmark[(bi * nby + bj) * nbz + bk] = 1;
  }
}

static inline unsigned blocks_for(uint64_t n, unsigned cap) {
  uint64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

static inline uint32_t host_tiles(int dim, const DevGrid& g) {
  if (dim == 3)
    return (uint32_t)((g.n0 + 3) / 4) * (uint32_t)((g.n1 + 7) / 8) * (uint32_t)((g.n2 + 7) / 8);
  return (uint32_t)((g.n0 + 15) / 16) * (uint32_t)((g.n1 + 15) / 16);
}

hipError_t launch_mark_init(int dim, const DevGrid& g, const double* d, double gs, uint8_t* ext,
                            hipStream_t s) {
  dim3 gr(blocks_for(g.N, 8192)), bl(256);
  if (dim == 3)
    hipLaunchKernelGGL(k_mark_init<3>, gr, bl, 0, s, g, d, gs, ext);
  else
    hipLaunchKernelGGL(k_mark_init<2>, gr, bl, 0, s, g, d, gs, ext);
  return hipGetLastError();
}

hipError_t launch_mark_pass(int dim, const DevGrid& g, const double* d, double gs, uint8_t* ext,
                            int32_t* changed, hipStream_t s) {
  dim3 gr(std::min<uint32_t>(host_tiles(dim, g), 4096u)), bl(256);
  if (dim == 3)
    hipLaunchKernelGGL(k_mark_pass<3>, gr, bl, 0, s, g, d, gs, ext, changed);
  else
    hipLaunchKernelGGL(k_mark_pass<2>, gr, bl, 0, s, g, d, gs, ext, changed);
  return hipGetLastError();
}

hipError_t launch_eik_init(const DevGrid& g, const double* v, const uint8_t* fixed, double* u,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_eik_init, dim3(blocks_for(g.N, 8192)), dim3(256), 0, s, g.N, v, fixed, u);
  return hipGetLastError();
}

hipError_t launch_eik_init_ext(const DevGrid& g, const double* d, double gs, const uint8_t* ext,
                               double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_eik_init_ext, dim3(blocks_for(g.N, 8192)), dim3(256), 0, s, g.N, d, gs, ext,
                     u);
  return hipGetLastError();
}

hipError_t launch_eik_pass(int dim, const DevGrid& g, double* u, const uint8_t* fixed,
                           int32_t* changed, hipStream_t s) {
  dim3 gr(std::min<uint32_t>(host_tiles(dim, g), 4096u)), bl(256);
  if (dim == 3)
    hipLaunchKernelGGL(k_eik_pass<3>, gr, bl, 0, s, g, u, fixed, changed);
  else
    hipLaunchKernelGGL(k_eik_pass<2>, gr, bl, 0, s, g, u, fixed, changed);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_phi0_cloud(const DevGrid& g, const double* d, const double* u, const uint8_t* ext,
                             double gs, T gamma, T* A, T* B, hipStream_t s) {
  hipLaunchKernelGGL(k_phi0_cloud<T>, dim3(blocks_for(g.N, 8192)), dim3(256), 0, s, g.N, d, u, ext,
                     gs, gamma, A, B);
  return hipGetLastError();
}

hipError_t launch_box_mark(int dim, const DevGrid& g, const double* pts, int64_t n, uint8_t* fixed,
                           uint8_t* bmark, hipStream_t s) {
  dim3 gr(blocks_for((uint64_t)n, 4096)), bl(256);
  if (dim == 3)
    hipLaunchKernelGGL(k_box_mark<3>, gr, bl, 0, s, g, pts, n, fixed, bmark);
  else
    hipLaunchKernelGGL(k_box_mark<2>, gr, bl, 0, s, g, pts, n, fixed, bmark);
  return hipGetLastError();
}

template hipError_t launch_phi0_cloud<float>(const DevGrid&, const double*, const double*,
                                             const uint8_t*, double, float, float*, float*,
                                             hipStream_t);
template hipError_t launch_phi0_cloud<double>(const DevGrid&, const double*, const double*,
                                              const uint8_t*, double, double, double*, double*,
                                              hipStream_t);

}  // namespace lsr

namespace lsr {

// Section 4, after eq. (dxdt): a finer run starts from the previous run's
// steady state interpolated onto its grid with the run's interpolator
// (Section 3.2); the node's position on the coarser grid is computed in
// double, as the node coordinate and then the cell coordinate, and moved
// onto that grid if it lies outside.
template <typename T>
__device__ __forceinline__ Loc<T> coarse_loc(double x, double lo, double h, int n) {
#pragma clang fp contract(off)
  double u = (x - lo) / h;
  const double umax = (double)(n - 1);
  u = u < 0.0 ? 0.0 : (u > umax ? umax : u);
  int i = (int)floor(u);
  if (i > n - 2) i = n - 2;
  Loc<T> r;
  r.i0 = i;
  r.t = (T)(u - (double)i);
  return r;
}

__device__ __forceinline__ double node_x(double lo, int i, double h) {
#pragma clang fp contract(off)
  return lo + i * h;
}

template <int DIM, int INTERP, typename T>
__global__ void k_resample(DevGrid g, DevGrid gc, const T* __restrict__ src, T gamma, T weno_e,
                           T* __restrict__ A, T* __restrict__ B) {
  const gptr<T> S = (gptr<T>)src;
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.N;
       idx += gridDim.x * blockDim.x) {
    uint32_t r = idx;
    int k = 0;
    if (DIM == 3) {
      k = (int)(r % (uint32_t)g.n2);
      r /= (uint32_t)g.n2;
    }
    const int j = (int)(r % (uint32_t)g.n1), i = (int)(r / (uint32_t)g.n1);
    const Loc<T> lx = coarse_loc<T>(node_x(g.lo0, i, g.hd), gc.lo0, gc.hd, gc.n0);
    const Loc<T> ly = coarse_loc<T>(node_x(g.lo1, j, g.hd), gc.lo1, gc.hd, gc.n1);
    T v;
    if (DIM == 3) {
      const Loc<T> lz = coarse_loc<T>(node_x(g.lo2, k, g.hd), gc.lo2, gc.hd, gc.n2);
      const GlobalRows<T> rows{S, gc.n0, gc.n1, gc.n2, gc.s0, gc.s1};
      v = INTERP == 0 ? interp_q1_3(rows, lx, ly, lz) : interp_weno3(rows, lx, ly, lz, weno_e);
    } else {
      v = INTERP == 0 ? interp_q1_2(S, gc, lx, ly) : interp_weno2(S, gc, lx, ly, weno_e);
    }
    v = fmin(fmax(v, -gamma), gamma);
    A[idx] = v;
    B[idx] = v;
  }
}

template <typename T>
hipError_t launch_resample(int dim, int interp, const DevGrid& g, const DevGrid& gc, const T* src,
                           T gamma, T weno_e, T* A, T* B, hipStream_t s) {
  dim3 gr(blocks_for(g.N, 8192)), bl(256);
  if (dim == 3) {
    if (interp == 0)
      hipLaunchKernelGGL((k_resample<3, 0, T>), gr, bl, 0, s, g, gc, src, gamma, weno_e, A, B);
    else
      hipLaunchKernelGGL((k_resample<3, 1, T>), gr, bl, 0, s, g, gc, src, gamma, weno_e, A, B);
  } else {
    if (interp == 0)
      hipLaunchKernelGGL((k_resample<2, 0, T>), gr, bl, 0, s, g, gc, src, gamma, weno_e, A, B);
    else
      hipLaunchKernelGGL((k_resample<2, 1, T>), gr, bl, 0, s, g, gc, src, gamma, weno_e, A, B);
  }
  return hipGetLastError();
}

template hipError_t launch_resample<float>(int, int, const DevGrid&, const DevGrid&, const float*,
                                           float, float, float*, float*, hipStream_t);
template hipError_t launch_resample<double>(int, int, const DevGrid&, const DevGrid&,
                                            const double*, double, double, double*, double*,
                                            hipStream_t);

// flag |= 1 for a point that is not finite or lies outside the grid's box
// (Algorithm 1, step 1: the grid encompasses the cloud).
template <int DIM>
__global__ void k_check_points(BinGeom bg, const double* __restrict__ pts, int64_t n,
                               int32_t* flag) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    bool bad = false;
    for (int ax = 0; ax < DIM; ++ax) {
      const double x = pts[q * DIM + ax];
      bad = bad || !isfinite(x) || x < bg.lo[ax] || x > bg.hi[ax];
    }
    if (bad) *flag = 1;
  }
}

hipError_t launch_check_points(int dim, const BinGeom& bg, const double* pts, int64_t n,
                               int32_t* flag, hipStream_t s) {
  dim3 gr(blocks_for((uint64_t)n, 4096)), bl(256);
  if (dim == 3)
    hipLaunchKernelGGL(k_check_points<3>, gr, bl, 0, s, bg, pts, n, flag);
  else
    hipLaunchKernelGGL(k_check_points<2>, gr, bl, 0, s, bg, pts, n, flag);
  return hipGetLastError();
}

}  // namespace lsr
