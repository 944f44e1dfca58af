// Preprocessing of the cloud: its resolution h_S (Section 4, the text after
// eq. dxdt), the mean distance from sampled points to their nearest
// neighbour in the cloud.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lsr_internal.h"

namespace lsr {

// Nearest-neighbour distance of every sampled point: the second smallest
// distance to the cloud, the point itself giving the smallest (an exact
// duplicate is a neighbour at distance 0).  Bins are visited in rings of
// Chebyshev bin distance r around the point's own bin; every point of ring
// r lies at least (r - 1) bw away, so the search stops once that bound
// exceeds the second best.  Distances in double without contraction.
template <int DIM>
__global__ __launch_bounds__(256) void k_nn_dist(BinGeom bg, const double* __restrict__ sorted,
                                                 const int32_t* __restrict__ start,
                                                 const double* __restrict__ raw, int64_t n_pts,
                                                 const int64_t* __restrict__ sample, int64_t ns,
                                                 double* __restrict__ nn, int32_t* flag) {
#pragma clang fp contract(off)
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < ns;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int64_t idx = sample[s];
    if (idx < 0 || idx >= n_pts) {
      atomicOr(flag, 1);
      nn[s] = 0.0;
      continue;
    }
    double q[3] = {0.0, 0.0, 0.0};
    int b[3] = {0, 0, 0};
    for (int ax = 0; ax < DIM; ++ax) {
      q[ax] = raw[idx * DIM + ax];
      const int c = (int)floor((q[ax] - bg.lo[ax]) * bg.inv_bw);
      b[ax] = c < 0 ? 0 : (c > bg.nb[ax] - 1 ? bg.nb[ax] - 1 : c);
    }
    double d1 = INFINITY, d2 = INFINITY;  // the two smallest squared distances
    auto scan = [&](int i, int j, int k) {
      const int bb[3] = {i, j, k};
      const int id = bin_id(bg, bb);
      for (int p = start[id]; p < start[id + 1]; ++p) {
        double d = 0.0;
        for (int ax = 0; ax < DIM; ++ax) {
          const double t = q[ax] - sorted[(int64_t)p * DIM + ax];
          d += t * t;
        }
        if (d < d1) {
          d2 = d1;
          d1 = d;
        } else if (d < d2) {
          d2 = d;
        }
      }
    };
    const int rmax = std::max(bg.nb[0], std::max(bg.nb[1], bg.nb[2]));
    for (int r = 0; r <= rmax; ++r) {
      if (r >= 1) {
        const double lb = (r - 1) * bg.bw;
        if (lb * lb > d2) break;
      }
      const int i0 = std::max(b[0] - r, 0), i1 = std::min(b[0] + r, bg.nb[0] - 1);
      const int j0 = std::max(b[1] - r, 0), j1 = std::min(b[1] + r, bg.nb[1] - 1);
      for (int i = i0; i <= i1; ++i)
        for (int j = j0; j <= j1; ++j) {
          const bool edge = abs(i - b[0]) == r || abs(j - b[1]) == r;
          if (DIM == 2) {
            if (edge) scan(i, j, 0);
            continue;
          }
          if (edge) {
            const int k0 = std::max(b[2] - r, 0), k1 = std::min(b[2] + r, bg.nb[2] - 1);
            for (int k = k0; k <= k1; ++k) scan(i, j, k);
          } else {
            if (b[2] - r >= 0) scan(i, j, b[2] - r);
            if (r > 0 && b[2] + r <= bg.nb[2] - 1) scan(i, j, b[2] + r);
          }
        }
    }
    nn[s] = sqrt(d2);
  }
}

// out[0] = mean of v[0 .. n-1], summed in a fixed order by one block.
__global__ __launch_bounds__(256) void k_mean(const double* __restrict__ v, int64_t n,
                                              double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < n; q += blockDim.x) s += v[q];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63u) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (((red[0] + red[1]) + red[2]) + red[3]) / (double)n;
}

hipError_t launch_cloud_spacing(int dim, const BinGeom& bg, const double* sorted,
                                const int32_t* start, const double* raw, int64_t n_pts,
                                const int64_t* sample, int64_t ns, double* nn, int32_t* flag,
                                double* out, hipStream_t s) {
  uint64_t blocks = ((uint64_t)ns + 255) / 256;
  dim3 gr((unsigned)std::min<uint64_t>(std::max<uint64_t>(blocks, 1), 4096)), bl(256);
  if (dim == 3)
    hipLaunchKernelGGL(k_nn_dist<3>, gr, bl, 0, s, bg, sorted, start, raw, n_pts, sample, ns, nn,
                       flag);
  else
    hipLaunchKernelGGL(k_nn_dist<2>, gr, bl, 0, s, bg, sorted, start, raw, n_pts, sample, ns, nn,
                       flag);
  hipLaunchKernelGGL(k_mean, dim3(1), bl, 0, s, nn, ns, out);
  return hipGetLastError();
}

}  // namespace lsr
