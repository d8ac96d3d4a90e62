// Backprojection Core (gather) and Projection Core (spread) kernels, in
// image space (the warp, Eq. 7-9) and in k-space (Eq. 1-3).
//
// Tap rule: a coordinate y in oversampled-grid units has taps
// g = floor(y) - 1 + m, m = 0..3, with weight c(y - g); indices wrap
// periodically.  In image space y = 2 (r + d(r)); 2 d is exact in FP32 and
// so are floor(2 d) and 2 d - floor(2 d), so the tap set and fractional
// offsets equal those of an FP64 evaluation bit for bit.
//
// Spreads are owner-computes: the oversampled grid is cut into tiles, a
// workgroup owns one tile, accumulates every contribution that lands in it
// in LDS, then writes the tile once.  The point lists per tile come from the
// plan-time binning, so no HBM atomics are used and every grid value is
// written exactly once per spread.
#pragma once

#include "common.h"

namespace isg {

constexpr int kGridThreads = 256;
constexpr int kMaxPhasesPerLaunch = 16;

struct Dims {
  int ndim;
  int n[3];       // image shape (n[2] = 1 in 2D)
  int G[3];       // oversampled shape (G[2] = 1 in 2D)
  int64_t N;      // voxels
};

__device__ __forceinline__ int wrap(int g, int G) {
  g %= G;
  return g < 0 ? g + G : g;
}

// ---------------------------------------------------------------------------
// image-space gather: out[r] = sum_taps prod_i c(y_i - g_i) u[g], y = 2(r+d(r))
// ---------------------------------------------------------------------------
template <int NDIM>
__global__ __launch_bounds__(kGridThreads) void warp_gather_kernel(const float2* __restrict__ u,
                                                                   const float* __restrict__ d,
                                                                   float2* __restrict__ out, Dims dm,
                                                                   KbPoly kb) {
  const int64_t r = (int64_t)blockIdx.x * kGridThreads + threadIdx.x;
  if (r >= dm.N) return;
  int ri[3];
  {
    int64_t t = r;
    for (int i = NDIM - 1; i >= 0; --i) {
      ri[i] = (int)(t % dm.n[i]);
      t /= dm.n[i];
    }
  }
  int base[NDIM];
  float w[NDIM][4];
#pragma unroll
  for (int i = 0; i < NDIM; ++i) {
    const float y = 2.0f * d[(int64_t)i * dm.N + r];
    const float fl = floorf(y);
    kb_weights(kb, y - fl, w[i]);
    base[i] = wrap(2 * ri[i] + (int)fl - 1, dm.G[i]);
  }
  float2 acc = make_float2(0.f, 0.f);
  if constexpr (NDIM == 3) {
    int g2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) g2[t] = base[2] + t >= dm.G[2] ? base[2] + t - dm.G[2] : base[2] + t;
#pragma unroll
    for (int t0 = 0; t0 < 4; ++t0) {
      int g0 = base[0] + t0;
      if (g0 >= dm.G[0]) g0 -= dm.G[0];
#pragma unroll
      for (int t1 = 0; t1 < 4; ++t1) {
        int g1 = base[1] + t1;
        if (g1 >= dm.G[1]) g1 -= dm.G[1];
        const float2* row = u + ((int64_t)g0 * dm.G[1] + g1) * dm.G[2];
        float2 s = make_float2(0.f, 0.f);
#pragma unroll
        for (int t2 = 0; t2 < 4; ++t2) {
          const float2 v = row[g2[t2]];
          s.x = fmaf(w[2][t2], v.x, s.x);
          s.y = fmaf(w[2][t2], v.y, s.y);
        }
        const float w01 = w[0][t0] * w[1][t1];
        acc.x = fmaf(w01, s.x, acc.x);
        acc.y = fmaf(w01, s.y, acc.y);
      }
    }
  } else {
#pragma unroll
    for (int t0 = 0; t0 < 4; ++t0) {
      int g0 = base[0] + t0;
      if (g0 >= dm.G[0]) g0 -= dm.G[0];
      const float2* row = u + (int64_t)g0 * dm.G[1];
      float2 s = make_float2(0.f, 0.f);
#pragma unroll
      for (int t1 = 0; t1 < 4; ++t1) {
        int g1 = base[1] + t1;
        if (g1 >= dm.G[1]) g1 -= dm.G[1];
        const float2 v = row[g1];
        s.x = fmaf(w[1][t1], v.x, s.x);
        s.y = fmaf(w[1][t1], v.y, s.y);
      }
      acc.x = fmaf(w[0][t0], s.x, acc.x);
      acc.y = fmaf(w[0][t0], s.y, acc.y);
    }
  }
  out[r] = acc;
}

// ---------------------------------------------------------------------------
// derivative of the warp with respect to d, contracted with a cotangent v:
// grad[i][r] = Re(conj(v[r]) * 2 * sum_taps c'(y_i - g_i) prod_{j!=i} c(y_j - g_j) u[g])
// ---------------------------------------------------------------------------
template <int NDIM>
__global__ __launch_bounds__(kGridThreads) void warp_grad_kernel(const float2* __restrict__ u,
                                                                 const float* __restrict__ d,
                                                                 const float2* __restrict__ v,
                                                                 float* __restrict__ grad, Dims dm,
                                                                 KbPoly kb) {
  const int64_t r = (int64_t)blockIdx.x * kGridThreads + threadIdx.x;
  if (r >= dm.N) return;
  int ri[3];
  {
    int64_t t = r;
    for (int i = NDIM - 1; i >= 0; --i) {
      ri[i] = (int)(t % dm.n[i]);
      t /= dm.n[i];
    }
  }
  int base[NDIM];
  float w[NDIM][4], dw[NDIM][4];
#pragma unroll
  for (int i = 0; i < NDIM; ++i) {
    const float y = 2.0f * d[(int64_t)i * dm.N + r];
    const float fl = floorf(y);
    kb_weights_deriv(kb, y - fl, w[i], dw[i]);
    base[i] = wrap(2 * ri[i] + (int)fl - 1, dm.G[i]);
  }
  float2 J[NDIM];
#pragma unroll
  for (int i = 0; i < NDIM; ++i) J[i] = make_float2(0.f, 0.f);
  if constexpr (NDIM == 3) {
#pragma unroll
    for (int t0 = 0; t0 < 4; ++t0) {
      int g0 = base[0] + t0;
      if (g0 >= dm.G[0]) g0 -= dm.G[0];
#pragma unroll
      for (int t1 = 0; t1 < 4; ++t1) {
        int g1 = base[1] + t1;
        if (g1 >= dm.G[1]) g1 -= dm.G[1];
        const float2* row = u + ((int64_t)g0 * dm.G[1] + g1) * dm.G[2];
        float2 s = make_float2(0.f, 0.f), sd = make_float2(0.f, 0.f);
#pragma unroll
        for (int t2 = 0; t2 < 4; ++t2) {
          int g2 = base[2] + t2;
          if (g2 >= dm.G[2]) g2 -= dm.G[2];
          const float2 val = row[g2];
          s.x = fmaf(w[2][t2], val.x, s.x);
          s.y = fmaf(w[2][t2], val.y, s.y);
          sd.x = fmaf(dw[2][t2], val.x, sd.x);
          sd.y = fmaf(dw[2][t2], val.y, sd.y);
        }
        const float a0 = dw[0][t0] * w[1][t1], a1 = w[0][t0] * dw[1][t1], a2 = w[0][t0] * w[1][t1];
        J[0] = make_float2(fmaf(a0, s.x, J[0].x), fmaf(a0, s.y, J[0].y));
        J[1] = make_float2(fmaf(a1, s.x, J[1].x), fmaf(a1, s.y, J[1].y));
        J[NDIM - 1] = make_float2(fmaf(a2, sd.x, J[NDIM - 1].x), fmaf(a2, sd.y, J[NDIM - 1].y));
      }
    }
  } else {
#pragma unroll
    for (int t0 = 0; t0 < 4; ++t0) {
      int g0 = base[0] + t0;
      if (g0 >= dm.G[0]) g0 -= dm.G[0];
      const float2* row = u + (int64_t)g0 * dm.G[1];
      float2 s = make_float2(0.f, 0.f), sd = make_float2(0.f, 0.f);
#pragma unroll
      for (int t1 = 0; t1 < 4; ++t1) {
        int g1 = base[1] + t1;
        if (g1 >= dm.G[1]) g1 -= dm.G[1];
        const float2 val = row[g1];
        s.x = fmaf(w[1][t1], val.x, s.x);
        s.y = fmaf(w[1][t1], val.y, s.y);
        sd.x = fmaf(dw[1][t1], val.x, sd.x);
        sd.y = fmaf(dw[1][t1], val.y, sd.y);
      }
      J[0] = make_float2(fmaf(dw[0][t0], s.x, J[0].x), fmaf(dw[0][t0], s.y, J[0].y));
      J[NDIM - 1] = make_float2(fmaf(w[0][t0], sd.x, J[NDIM - 1].x), fmaf(w[0][t0], sd.y, J[NDIM - 1].y));
    }
  }
  const float2 vv = v[r];
#pragma unroll
  for (int i = 0; i < NDIM; ++i) grad[(int64_t)i * dm.N + r] = 2.0f * (vv.x * J[i].x + vv.y * J[i].y);
}

// ---------------------------------------------------------------------------
// image-space spread, all states into one grid (Eq. 8: P_d, summed over the
// states of the adjoint stacked operator).
// ---------------------------------------------------------------------------
struct WarpSpreadPhases {
  int P;
  const int* tile_off[kMaxPhasesPerLaunch];  // [ntiles + 1]
  const int* vox[kMaxPhasesPerLaunch];       // voxel indices, grouped by tile
  const float* d[kMaxPhasesPerLaunch];       // [ndim][N]
  const float2* w[kMaxPhasesPerLaunch];      // values to spread, [N]
};

struct TileDims {
  int TS[3];      // tile extent per axis
  int nt[3];      // tiles per axis
};

template <int NDIM>
__global__ __launch_bounds__(kGridThreads) void warp_spread_kernel(WarpSpreadPhases ph, float2* __restrict__ U,
                                                                   int accumulate, Dims dm, TileDims td,
                                                                   KbPoly kb) {
  extern __shared__ float2 acc[];
  const int tile = blockIdx.x;
  int tc[3] = {0, 0, 0};
  {
    int t = tile;
    for (int i = NDIM - 1; i >= 0; --i) {
      tc[i] = t % td.nt[i];
      t /= td.nt[i];
    }
  }
  int lo[3], ext[3];
  int vol = 1;
#pragma unroll
  for (int i = 0; i < NDIM; ++i) {
    lo[i] = tc[i] * td.TS[i];
    ext[i] = min(td.TS[i], dm.G[i] - lo[i]);
    vol *= td.TS[i];
  }
  for (int e = threadIdx.x; e < vol; e += kGridThreads) acc[e] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int p = 0; p < ph.P; ++p) {
    const int beg = ph.tile_off[p][tile], end = ph.tile_off[p][tile + 1];
    const int* vox = ph.vox[p];
    const float* d = ph.d[p];
    const float2* w = ph.w[p];
    for (int e = beg + threadIdx.x; e < end; e += kGridThreads) {
      const int64_t r = vox[e];
      int ri[3];
      {
        int64_t t = r;
        for (int i = NDIM - 1; i >= 0; --i) {
          ri[i] = (int)(t % dm.n[i]);
          t /= dm.n[i];
        }
      }
      const float2 val = w[r];
      int loc[NDIM][4];
      float wt[NDIM][4];
#pragma unroll
      for (int i = 0; i < NDIM; ++i) {
        const float y = 2.0f * d[(int64_t)i * dm.N + r];
        const float fl = floorf(y);
        kb_weights(kb, y - fl, wt[i]);
        const int b = wrap(2 * ri[i] + (int)fl - 1, dm.G[i]);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          int g = b + t;
          if (g >= dm.G[i]) g -= dm.G[i];
          const int l = g - lo[i];
          loc[i][t] = (l >= 0 && l < ext[i]) ? l : -1;
        }
      }
      if constexpr (NDIM == 3) {
#pragma unroll
        for (int t0 = 0; t0 < 4; ++t0) {
          if (loc[0][t0] < 0) continue;
#pragma unroll
          for (int t1 = 0; t1 < 4; ++t1) {
            if (loc[1][t1] < 0) continue;
            const float w01 = wt[0][t0] * wt[1][t1];
            const int rowi = (loc[0][t0] * td.TS[1] + loc[1][t1]) * td.TS[2];
#pragma unroll
            for (int t2 = 0; t2 < 4; ++t2) {
              if (loc[2][t2] < 0) continue;
              const float ww = w01 * wt[2][t2];
              float2* a = acc + rowi + loc[2][t2];
              atomicAdd(&a->x, ww * val.x);
              atomicAdd(&a->y, ww * val.y);
            }
          }
        }
      } else {
#pragma unroll
        for (int t0 = 0; t0 < 4; ++t0) {
          if (loc[0][t0] < 0) continue;
#pragma unroll
          for (int t1 = 0; t1 < 4; ++t1) {
            if (loc[1][t1] < 0) continue;
            const float ww = wt[0][t0] * wt[1][t1];
            float2* a = acc + loc[0][t0] * td.TS[1] + loc[1][t1];
            atomicAdd(&a->x, ww * val.x);
            atomicAdd(&a->y, ww * val.y);
          }
        }
      }
    }
  }
  __syncthreads();
  // write the tile: rows along the last axis are contiguous in U
  const int last = NDIM - 1;
  for (int e = threadIdx.x; e < vol; e += kGridThreads) {
    int l[3] = {0, 0, 0};
    int t = e;
    for (int i = NDIM - 1; i >= 0; --i) {
      l[i] = t % td.TS[i];
      t /= td.TS[i];
    }
    bool ok = true;
    for (int i = 0; i < NDIM; ++i) ok = ok && l[i] < ext[i];
    if (!ok) continue;
    int64_t gi = 0;
    for (int i = 0; i < NDIM; ++i) gi = gi * dm.G[i] + lo[i] + l[i];
    (void)last;
    float2 v = acc[e];
    if (accumulate) v = cadd(v, U[gi]);
    U[gi] = v;
  }
}

// ---------------------------------------------------------------------------
// k-space taps, prepared at plan time: fractional offsets and the wrapped
// base index (10 bits per axis) of every sample.
// ---------------------------------------------------------------------------
struct KTap {
  float f[3];
  uint32_t base;  // b0 | b1 << 10 | b2 << 20
};

// y[j][c] = sum_taps prod_i c(kappa_ji - q_i) grid[q][c], grid [G...][C]
template <int NDIM, int S>
__global__ __launch_bounds__(kGridThreads) void kgather_kernel(const typename Elem<S>::T* __restrict__ grid,
                                                               const KTap* __restrict__ taps, int64_t M,
                                                               float2* __restrict__ y, int C, Dims dm,
                                                               KbPoly kb) {
  const int64_t j = (int64_t)blockIdx.x * kGridThreads + threadIdx.x;
  if (j >= M) return;
  const KTap tp = taps[j];
  float w[NDIM][4];
  int g[NDIM][4];
#pragma unroll
  for (int i = 0; i < NDIM; ++i) {
    kb_weights(kb, tp.f[i], w[i]);
    const int b = (tp.base >> (10 * i)) & 1023;
#pragma unroll
    for (int t = 0; t < 4; ++t) g[i][t] = b + t >= dm.G[i] ? b + t - dm.G[i] : b + t;
  }
  constexpr int CC = 4;
  for (int c0 = 0; c0 < C; c0 += CC) {
    float2 acc[CC];
#pragma unroll
    for (int c = 0; c < CC; ++c) acc[c] = make_float2(0.f, 0.f);
    if constexpr (NDIM == 3) {
#pragma unroll
      for (int t0 = 0; t0 < 4; ++t0) {
#pragma unroll
        for (int t1 = 0; t1 < 4; ++t1) {
          const float w01 = w[0][t0] * w[1][t1];
          const int64_t row = ((int64_t)g[0][t0] * dm.G[1] + g[1][t1]) * dm.G[2];
#pragma unroll
          for (int t2 = 0; t2 < 4; ++t2) {
            const float ww = w01 * w[2][t2];
            const typename Elem<S>::T* p = grid + (row + g[2][t2]) * C + c0;
#pragma unroll
            for (int c = 0; c < CC; ++c) {
              if (c0 + c < C) {
                const float2 v = Elem<S>::load(p + c);
                acc[c].x = fmaf(ww, v.x, acc[c].x);
                acc[c].y = fmaf(ww, v.y, acc[c].y);
              }
            }
          }
        }
      }
    } else {
#pragma unroll
      for (int t0 = 0; t0 < 4; ++t0) {
#pragma unroll
        for (int t1 = 0; t1 < 4; ++t1) {
          const float ww = w[0][t0] * w[1][t1];
          const typename Elem<S>::T* p = grid + ((int64_t)g[0][t0] * dm.G[1] + g[1][t1]) * C + c0;
#pragma unroll
          for (int c = 0; c < CC; ++c) {
            if (c0 + c < C) {
              const float2 v = Elem<S>::load(p + c);
              acc[c].x = fmaf(ww, v.x, acc[c].x);
              acc[c].y = fmaf(ww, v.y, acc[c].y);
            }
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CC; ++c)
      if (c0 + c < C) y[j * C + c0 + c] = acc[c];
  }
}

// k-space spread work unit: `count` samples of tile `tile` starting at
// `start` in the tile-sorted sample list.  slot < 0: the unit is the whole
// tile and writes the grid; slot >= 0: the unit writes a partial tile into
// scratch slot `slot`, and a reduce step sums the slots of the tile.
struct KUnit {
  int tile, start, count, slot;
};

struct KTile {
  int TS[3];
  int nt[3];
  int vol;        // points per tile
};

__device__ __forceinline__ void ktile_origin(int tile, const KTile& kt, int ndim, int lo[3]) {
  int t = tile;
  for (int i = ndim - 1; i >= 0; --i) {
    lo[i] = (t % kt.nt[i]) * kt.TS[i];
    t /= kt.nt[i];
  }
}

// one wavefront per sample and one lane per tap; C coil values per lane
template <int NDIM, int S>
__global__ __launch_bounds__(kGridThreads) void kspread_kernel(const KUnit* __restrict__ units,
                                                               const int* __restrict__ order,
                                                               const KTap* __restrict__ taps,
                                                               const float2* __restrict__ y, int C,
                                                               typename Elem<S>::T* __restrict__ grid,
                                                               float2* __restrict__ partial, Dims dm,
                                                               KTile kt, KbPoly kb) {
  extern __shared__ float2 acc[];  // [vol][C]
  const KUnit un = units[blockIdx.x];
  int lo[3] = {0, 0, 0};
  ktile_origin(un.tile, kt, NDIM, lo);
  const int volC = kt.vol * C;
  for (int e = threadIdx.x; e < volC; e += kGridThreads) acc[e] = make_float2(0.f, 0.f);
  __syncthreads();
  constexpr int TAPS = NDIM == 3 ? 64 : 16;
  constexpr int SPW = 64 / TAPS;  // samples per wavefront
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int sub = lane / TAPS;
  const int tap = lane - sub * TAPS;
  int tt[3];
  tt[NDIM - 1] = tap & 3;
  tt[NDIM >= 2 ? NDIM - 2 : 0] = (tap >> 2) & 3;
  if constexpr (NDIM == 3) tt[0] = tap >> 4;
  for (int s = wave * SPW + sub; s < un.count; s += (kGridThreads / 64) * SPW) {
    const int j = order[un.start + s];
    const KTap tp = taps[j];
    bool inside = true;
    float ww = 1.0f;
    int li = 0;
#pragma unroll
    for (int i = 0; i < NDIM; ++i) {
      const float f = tp.f[i];
      const int m = tt[i];
      // t_m = ((1 + m) - f)((3 - m) + f)/4, the same float operations as
      // kb_weights; the m = 3 tap is 0 when f == 0
      const float t = ((float)(1 + m) - f) * ((float)(3 - m) + f) * 0.25f;
      const float wi = (m == 3 && !(f > 0.0f)) ? 0.0f : kb_poly(kb, t);
      ww *= wi;
      int g = (int)((tp.base >> (10 * i)) & 1023) + m;
      if (g >= dm.G[i]) g -= dm.G[i];
      const int l = g - lo[i];
      inside = inside && l >= 0 && l < kt.TS[i] && g < dm.G[i];
      li = li * kt.TS[i] + l;
    }
    if (!inside) continue;
    const float2* yj = y + (int64_t)j * C;
    float2* a = acc + (int64_t)li * C;
    for (int c = 0; c < C; ++c) {
      const float2 v = yj[c];
      atomicAdd(&a[c].x, ww * v.x);
      atomicAdd(&a[c].y, ww * v.y);
    }
  }
  __syncthreads();
  // write out: rows along the last axis are TS*C contiguous values
  for (int e = threadIdx.x; e < volC; e += kGridThreads) {
    const int pt = e / C;
    const int c = e - pt * C;
    if (un.slot >= 0) {
      partial[(int64_t)un.slot * volC + e] = acc[e];
      continue;
    }
    int l[3] = {0, 0, 0};
    int t = pt;
    bool ok = true;
    int64_t gi = 0;
    for (int i = NDIM - 1; i >= 0; --i) {
      l[i] = t % kt.TS[i];
      t /= kt.TS[i];
    }
    for (int i = 0; i < NDIM; ++i) {
      const int g = lo[i] + l[i];
      ok = ok && g < dm.G[i];
      gi = gi * dm.G[i] + g;
    }
    if (ok) Elem<S>::store(grid + gi * C + c, acc[e]);
  }
}

// sum the partial tiles of every split tile (fixed slot order) and write them
struct KSplit {
  int tile, first_slot, nslots;
};

template <int NDIM, int S>
__global__ __launch_bounds__(kGridThreads) void kspread_reduce_kernel(const KSplit* __restrict__ splits,
                                                                      const float2* __restrict__ partial,
                                                                      int C, typename Elem<S>::T* __restrict__ grid,
                                                                      Dims dm, KTile kt) {
  const KSplit sp = splits[blockIdx.x];
  int lo[3] = {0, 0, 0};
  ktile_origin(sp.tile, kt, NDIM, lo);
  const int volC = kt.vol * C;
  for (int e = threadIdx.x; e < volC; e += kGridThreads) {
    float2 s = make_float2(0.f, 0.f);
    for (int k = 0; k < sp.nslots; ++k) s = cadd(s, partial[(int64_t)(sp.first_slot + k) * volC + e]);
    const int pt = e / C;
    const int c = e - pt * C;
    int l[3] = {0, 0, 0};
    int t = pt;
    for (int i = NDIM - 1; i >= 0; --i) {
      l[i] = t % kt.TS[i];
      t /= kt.TS[i];
    }
    bool ok = true;
    int64_t gi = 0;
    for (int i = 0; i < NDIM; ++i) {
      const int g = lo[i] + l[i];
      ok = ok && g < dm.G[i];
      gi = gi * dm.G[i] + g;
    }
    if (ok) Elem<S>::store(grid + gi * C + c, s);
  }
}

}  // namespace isg
