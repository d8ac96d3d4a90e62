// Plan-time binning of a displacement field on the device: the voxel lists
// per warp-spread tile that the image-space spread (Eq. 7-8) walks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace isg {

__global__ void fill_i32_kernel(int* __restrict__ p, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// bits of the field check
constexpr int kFieldNotFinite = 1;
constexpr int kFieldTooLarge = 2;

// The binning key of every voxel r: the warp-spread tile holding the first
// tap of its gather coordinate 2 (r + d(r)) along every axis (tile extents
// 2^lg[i] of the oversampled grid, nt[i] tiles per axis, row-major tile
// index), and r itself as the value.  The tap base is computed exactly as the
// spread kernel computes it: floor of the float coordinate 2 d, plus 2 r - 1,
// wrapped onto the periodic grid.  A displacement that is not finite or
// exceeds 1e6 voxels sets a bit of *bad and bins to tile 0.
template <int NDIM>
__global__ void motion_key_kernel(const float* __restrict__ d, int64_t N, int n0, int n1, int n2, int G0, int G1,
                                  int G2, int nt0, int nt1, int nt2, int lg0, int lg1, int lg2, int* __restrict__ key,
                                  int* __restrict__ val, int* __restrict__ bad) {
  const int n[3] = {n0, n1, n2}, G[3] = {G0, G1, G2}, nt[3] = {nt0, nt1, nt2}, lg[3] = {lg0, lg1, lg2};
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x) {
    int ri[3] = {0, 0, 0};
    int64_t t = r;
#pragma unroll
    for (int i = NDIM - 1; i >= 0; --i) {
      ri[i] = (int)(t % n[i]);
      t /= n[i];
    }
    int flags = 0, tile = 0;
#pragma unroll
    for (int i = 0; i < NDIM; ++i) {
      const float v = d[(int64_t)i * N + r];
      if (!isfinite(v)) {
        flags |= kFieldNotFinite;
      } else if (fabsf(v) > 1.0e6f) {
        flags |= kFieldTooLarge;
      } else {
        const float y = 2.0f * v;
        int64_t b = (2 * (int64_t)ri[i] + (int64_t)floorf(y) - 1) % G[i];
        if (b < 0) b += G[i];
        tile = tile * nt[i] + (int)(b >> lg[i]);
      }
    }
    if (flags) {
      atomicOr(bad, flags);
      tile = 0;
    }
    key[r] = tile;
    val[r] = (int)r;
  }
}

// First entry of every tile in the keys sorted ascending: tiles t with
// skey[i-1] < t <= skey[i] start at entry i (tile_off[ntiles] = N), so every
// one of the ntiles + 1 offsets is written exactly once.
__global__ void tile_offsets_kernel(const int* __restrict__ skey, int64_t N, int ntiles, int* __restrict__ tile_off) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= N; i += (int64_t)gridDim.x * blockDim.x) {
    const int lo = i == 0 ? 0 : skey[i - 1] + 1;
    const int hi = i == N ? ntiles : skey[i];
    for (int t = lo; t <= hi; ++t) tile_off[t] = (int)i;
  }
}

}  // namespace isg
