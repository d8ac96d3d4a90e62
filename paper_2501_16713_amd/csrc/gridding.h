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
  FastDiv nfd[3]; // division by n[i]
  float invG[3];  // 1 / G[i]
};

// g mod G in [0, G) for |g| < 2^24: a float quotient, then one correction
// either way
__device__ __forceinline__ int wrap(int g, int G, float invG) {
  g -= G * (int)floorf((float)g * invG);
  if (g >= G) g -= G;
  if (g < 0) g += G;
  return g;
}

// integer coordinates of voxel r (r < 2^31) of the image [n0][n1](/[n2])
template <int NDIM>
__device__ __forceinline__ void voxel_coords(int64_t r, const Dims& dm, int ri[3]) {
  const uint32_t rr = (uint32_t)r;
  if constexpr (NDIM == 3) {
    const uint32_t q = dm.nfd[2].div(rr);
    ri[2] = (int)(rr - q * (uint32_t)dm.n[2]);
    ri[0] = (int)dm.nfd[1].div(q);
    ri[1] = (int)(q - (uint32_t)ri[0] * (uint32_t)dm.n[1]);
  } else {
    ri[0] = (int)dm.nfd[1].div(rr);
    ri[1] = (int)(rr - (uint32_t)ri[0] * (uint32_t)dm.n[1]);
    ri[2] = 0;
  }
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
  voxel_coords<NDIM>(r, dm, ri);
  int base[NDIM];
  float w[NDIM][4];
#pragma unroll
  for (int i = 0; i < NDIM; ++i) {
    const float y = 2.0f * d[(int64_t)i * dm.N + r];
    const float fl = floorf(y);
    kb_weights(kb, y - fl, w[i]);
    base[i] = wrap(2 * ri[i] + (int)fl - 1, dm.G[i], dm.invG[i]);
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
  voxel_coords<NDIM>(r, dm, ri);
  int base[NDIM];
  float w[NDIM][4], dw[NDIM][4];
#pragma unroll
  for (int i = 0; i < NDIM; ++i) {
    const float y = 2.0f * d[(int64_t)i * dm.N + r];
    const float fl = floorf(y);
    kb_weights_deriv(kb, y - fl, w[i], dw[i]);
    base[i] = wrap(2 * ri[i] + (int)fl - 1, dm.G[i], dm.invG[i]);
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

// Image-space spread tiles and their regions.  Every (state, voxel) entry
// belongs to the one tile that holds its first tap along every axis (the tap
// run b .. b+3 starts in [lo, lo + ext)), so all 4^NDIM of its taps fall in
// that tile's region: the tile extended by a halo of three cells past its
// upper faces (wrapping periodically), ext + 3 cells per axis.  The regions
// of neighbouring tiles overlap in the halos; a second pass sums them.
// Tile extents are powers of two (at most G/2), and every G is a multiple
// of 4, so a ragged last tile is at least 4 wide and a cell gets
// contributions from its own tile and, within three cells above a tile
// boundary, from the tile below it: at most two tiles per axis.
struct TileDims {
  int TS[3];   // tile extent per axis (power of two)
  int lg[3];   // log2 TS
  int nt[3];   // tiles per axis
  int E[3];    // region extent per axis, TS + 3 (1 on a missing axis)
  int R0, R1;  // LDS strides of a region copy along axes 0 and 1 (last axis contiguous, rows padded to an
               // even length so that the 16 taps of one step hit 32 distinct banks)
  int P;       // LDS region copy size (float2, even)
  int RV;      // region cells in global memory (E0 E1 E2, compact)
};

// Wavefronts per workgroup and entries a wavefront stages per round.  Each
// wavefront accumulates into a region copy of its own.
constexpr int kWarpWaves = 4;
constexpr int kWarpStage = 64;
// entries a wavefront applies per step: in 3D its 64 lanes are the 64 taps
// of one entry, in 2D four entries of 16 taps (one region copy each)
template <int NDIM> struct WarpLanes {
  static constexpr int kEntries = NDIM == 3 ? 1 : 4;
};

__host__ __device__ inline size_t warp_spread_lds_bytes(const TileDims& td, int ndim) {
  const int q = ndim == 3 ? WarpLanes<3>::kEntries : WarpLanes<2>::kEntries;
  return sizeof(float2) * (size_t)kWarpWaves * q * td.P;
}

// Workgroup index -> tile such that the workgroups of one XCD (consecutive
// indices go to the 8 XCDs in turn) take one contiguous range of tiles, whose
// neighbouring tiles share source voxels in that XCD's L2.  Launch
// 8 * ceil(n / 8) workgroups; indices past the last tile return n or more.
__device__ __forceinline__ int xcd_contiguous(int b, int n) {
  const int per = (n + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

// Pass 1 of the image-space spread, without atomics: the entries of one
// tile over all states (voxel lists from the plan-time binning) are
// accumulated in LDS copies of the tile's region and the region is written
// to reg[tile][E0][E1][E2].  Entries are cut into batches of kWarpStage;
// wave w takes batches w, w + kWarpWaves, ...: its lanes stage one entry
// each (region offset of the first tap, the per-axis weights, the value),
// then the wave walks the staged entries, its lanes covering the taps of an
// entry (distinct cells, so plain read-modify-write is race free).  The
// copies are summed in a fixed order (deterministic).  The global reads of
// the staging are software-pipelined: a lane's voxel index is read two
// rounds ahead and its displacement and value one round ahead.
template <int NDIM>
__global__ __launch_bounds__(64 * kWarpWaves) void warp_spread_kernel(WarpSpreadPhases ph, float2* __restrict__ reg,
                                                                   int ntiles, Dims dm, TileDims td, KbPoly kb) {
  constexpr int Q = WarpLanes<NDIM>::kEntries;
  extern __shared__ float2 accw[];  // [kWarpWaves][Q][P]
  __shared__ int st_off[kWarpWaves][kWarpStage];
  __shared__ float st_w[kWarpWaves][kWarpStage * 12];  // entry s: weights of axis i at 12 s + 4 i + t
  __shared__ float2 st_v[kWarpWaves][kWarpStage];
  __shared__ int s_beg[kMaxPhasesPerLaunch];      // first entry of state p in its voxel list
  __shared__ int s_pfx[kMaxPhasesPerLaunch + 1];  // entries of the tile over states < p
  // per-state pointers in LDS: indexing the kernel arguments by a runtime
  // state would read them from memory in line with the staging loads, and
  // waiting for such a read waits for every load issued before it
  // (held as global-address-space pointers, so the loads through them are
  // global loads and not flat ones, which the LDS waits would also wait for)
  typedef const __attribute__((address_space(1))) int* GInt;
  typedef const __attribute__((address_space(1))) float* GFloat;
  __shared__ GInt s_vox[kMaxPhasesPerLaunch];
  __shared__ GFloat s_d[kMaxPhasesPerLaunch];
  __shared__ GFloat s_w[kMaxPhasesPerLaunch];  // complex values as (re, im) pairs
  const int tile = xcd_contiguous(blockIdx.x, ntiles);
  if (tile >= ntiles) return;
  int lo[3] = {0, 0, 0};
  {
    int t = tile;
    for (int i = NDIM - 1; i >= 0; --i) {
      lo[i] = (t % td.nt[i]) * td.TS[i];
      t /= td.nt[i];
    }
  }
  {
    float4* a4 = (float4*)accw;
    const int n4 = (kWarpWaves * Q * td.P) >> 1;  // P is even
    for (int e = threadIdx.x; e < n4; e += 64 * kWarpWaves) a4[e] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  // entries of this tile over all states, concatenated
  if ((int)threadIdx.x < ph.P) {
    const int b = ph.tile_off[threadIdx.x][tile];
    s_beg[threadIdx.x] = b;
    s_pfx[threadIdx.x + 1] = ph.tile_off[threadIdx.x][tile + 1] - b;
    s_vox[threadIdx.x] = (GInt)ph.vox[threadIdx.x];
    s_d[threadIdx.x] = (GFloat)ph.d[threadIdx.x];
    s_w[threadIdx.x] = (GFloat)ph.w[threadIdx.x];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s_pfx[0] = 0;
    for (int p = 0; p < ph.P; ++p) s_pfx[p + 1] += s_pfx[p];
  }
  __syncthreads();
  const int E = s_pfx[ph.P];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // lane roles: the entry slot of a step and the tap along each axis
  int q, ta0, ta1, ta2;
  if constexpr (NDIM == 3) {
    q = 0;
    ta0 = lane >> 4;
    ta1 = (lane >> 2) & 3;
    ta2 = lane & 3;
  } else {
    q = lane >> 4;
    ta0 = (lane >> 2) & 3;
    ta1 = lane & 3;
    ta2 = 0;
  }
  float2* copy = accw + (size_t)(wave * Q + q) * td.P;
  const int tapoff = NDIM == 3 ? __mul24(ta0, td.R0) + __mul24(ta1, td.R1) + ta2 : __mul24(ta0, td.R0) + ta1;
  const int nbatch = (E + kWarpStage - 1) / kWarpStage;
  const int rounds = (nbatch + kWarpWaves - 1) / kWarpWaves;
  // the entry this lane stages in round rd: its state and voxel (-1: none)
  auto voxel_of = [&](int rd, int& p) -> int {
    const int e = (rd * kWarpWaves + wave) * kWarpStage + lane;
    p = 0;
    if (rd >= rounds || lane >= kWarpStage || e >= E) return -1;
    while (e >= s_pfx[p + 1]) ++p;
    return s_vox[p][s_beg[p] + (e - s_pfx[p])];
  };
  float dn[NDIM];  // next round's displacement and value
  float2 vn = make_float2(0.f, 0.f);
  auto data_of = [&](int r, int p) {
    if (r < 0) return;
    const GFloat dp = s_d[p];
#pragma unroll
    for (int i = 0; i < NDIM; ++i) dn[i] = dp[(int64_t)i * dm.N + r];
    const GFloat wp = s_w[p] + 2 * (int64_t)r;
    vn = make_float2(wp[0], wp[1]);
  };
#pragma unroll
  for (int i = 0; i < NDIM; ++i) dn[i] = 0.f;
  int pn, p2;
  int rn = voxel_of(0, pn);  // staging round 0
  data_of(rn, pn);
  int r2 = voxel_of(1, p2);  // staging round 1
  for (int rd = 0; rd < rounds; ++rd) {
    const int b = rd * kWarpWaves + wave;
    const int e0 = b * kWarpStage;
    const int ne = max(0, min(kWarpStage, E - e0));
    const int r = rn;
    float dc[NDIM];
#pragma unroll
    for (int i = 0; i < NDIM; ++i) dc[i] = dn[i];
    const float2 vc = vn;
    __syncthreads();  // accumulators zeroed / this wave's previous batch consumed
    if (lane < ne) {  // stage entry e0 + lane
      int ri[3];
      voxel_coords<NDIM>(r, dm, ri);
      int off = 0;
#pragma unroll
      for (int i = 0; i < NDIM; ++i) {
        const float yv = 2.0f * dc[i];
        const float fl = floorf(yv);
        float w[4];
        kb_weights(kb, yv - fl, w);
#pragma unroll
        for (int t = 0; t < 4; ++t) st_w[wave][12 * lane + 4 * i + t] = w[t];
        // the binning put the first tap in this tile: 0 <= o < ext
        const int o = wrap(2 * ri[i] + (int)fl - 1, dm.G[i], dm.invG[i]) - lo[i];
        off += __mul24(o, i == 0 ? td.R0 : (i == NDIM - 1 ? 1 : td.R1));
      }
      st_off[wave][lane] = off;
      st_v[wave][lane] = vc;
    }
    __syncthreads();
    // reads for the next rounds, in flight during this round's accumulation
    rn = r2;
    pn = p2;
    data_of(rn, pn);
    r2 = voxel_of(rd + 2, p2);
    for (int s = 0; s < ne; s += Q) {
      const int sq = s + q;
      const bool has = sq < ne;  // 2D: a slot past the last entry adds zero
      const int sc = has ? sq : s;
      const int wi = __mul24(sc, 12);
      float wt = st_w[wave][wi + ta0] * st_w[wave][wi + 4 + ta1];
      if constexpr (NDIM == 3) wt *= st_w[wave][wi + 8 + ta2];
      const float2 v = has ? st_v[wave][sc] : make_float2(0.f, 0.f);
      float2* pt = copy + st_off[wave][sc] + tapoff;
      const float2 a = *pt;
      *pt = make_float2(fmaf(wt, v.x, a.x), fmaf(wt, v.y, a.y));
    }
  }
  __syncthreads();
  // sum the copies and write the region, [E0][E1][E2] compact
  const int e12 = td.E[1] * td.E[2];
  for (int e = threadIdx.x; e < td.RV; e += 64 * kWarpWaves) {
    const int l0 = e / e12;
    const int rem = e - l0 * e12;
    const int l1 = rem / td.E[2];
    const int l2 = rem - l1 * td.E[2];
    const int pi = NDIM == 3 ? l0 * td.R0 + l1 * td.R1 + l2 : l0 * td.R0 + l1;
    float2 v = make_float2(0.f, 0.f);
#pragma unroll
    for (int w = 0; w < kWarpWaves * Q; ++w) v = cadd(v, accw[(size_t)w * td.P + pi]);
    reg[(int64_t)tile * td.RV + e] = v;
  }
}

// Pass 2 of the image-space spread: U[g] (+)= the sum of every region that
// covers g, in a fixed order.  Along axis i, g lies at l = g - lo in its own
// tile t, and, when l < 3, also at l + ext(t') in the region of the tile
// below, t' = t - 1 (periodically: the last tile below tile 0).  One
// workgroup per row of U along the last axis (G_last <= 1024 threads).
template <int NDIM>
__global__ __launch_bounds__(1024) void warp_spread_sum_kernel(const float2* __restrict__ reg, float2* __restrict__ U,
                                                               int accumulate, Dims dm, TileDims td) {
  const int gl = threadIdx.x;  // along the last axis
  if (gl >= dm.G[NDIM - 1]) return;
  int g[3] = {0, 0, 0};
  if constexpr (NDIM == 3) {
    g[0] = blockIdx.x / dm.G[1];
    g[1] = blockIdx.x - g[0] * dm.G[1];
    g[2] = gl;
  } else {
    g[0] = blockIdx.x;
    g[1] = gl;
  }
  int tt[3][2], ll[3][2], nc[3] = {1, 1, 1};
#pragma unroll
  for (int i = 0; i < NDIM; ++i) {
    const int t = g[i] >> td.lg[i];
    const int l = g[i] - (t << td.lg[i]);
    tt[i][0] = t;
    ll[i][0] = l;
    if (l < 3) {
      const int tp = t == 0 ? td.nt[i] - 1 : t - 1;
      const int ext = tp == td.nt[i] - 1 ? dm.G[i] - (tp << td.lg[i]) : td.TS[i];
      tt[i][1] = tp;
      ll[i][1] = l + ext;
      nc[i] = 2;
    }
  }
  float2 v = make_float2(0.f, 0.f);
  if constexpr (NDIM == 3) {
    for (int a = 0; a < nc[0]; ++a)
      for (int b = 0; b < nc[1]; ++b)
        for (int c = 0; c < nc[2]; ++c) {
          const int tile = (tt[0][a] * td.nt[1] + tt[1][b]) * td.nt[2] + tt[2][c];
          v = cadd(v, reg[(int64_t)tile * td.RV + (ll[0][a] * td.E[1] + ll[1][b]) * td.E[2] + ll[2][c]]);
        }
  } else {
    for (int a = 0; a < nc[0]; ++a)
      for (int b = 0; b < nc[1]; ++b) {
        const int tile = tt[0][a] * td.nt[1] + tt[1][b];
        v = cadd(v, reg[(int64_t)tile * td.RV + ll[0][a] * td.E[1] + ll[1][b]]);
      }
  }
  const int64_t gi = (int64_t)blockIdx.x * dm.G[NDIM - 1] + gl;
  if (accumulate) v = cadd(U[gi], v);
  U[gi] = v;
}

// ---------------------------------------------------------------------------
// k-space taps, prepared at plan time: fractional offsets and the wrapped
// base index (10 bits per axis) of every sample.
// ---------------------------------------------------------------------------
// k-space spread work unit: `count` samples of tile `tile` starting at
// `start` in the tile-sorted sample list.  slot < 0: the unit is the whole
// tile and writes the grid; slot >= 0: the unit writes a partial tile into
// scratch slot `slot`, and a reduce step sums the slots of the tile.
struct KUnit {
  int tile, start, count, slot;
  int gslot;  // tile-major grids: the tile's slot among the touched tiles
  // 8 x 4 x 8 register spread: the unit's visits are ordered by the rows
  // their axis-0 taps reach, rows 0-3 only in [0, lo), rows 4-7 only in
  // [lo, lohi), both halves in [lohi, count) (0, 0 when not ordered)
  int lo, lohi;
};
// a tile whose samples were cut into several units: partial slots
// first_slot .. first_slot + nslots - 1
struct KSplit {
  int tile, first_slot, nslots;
  int gslot;  // as in KUnit
};
struct KTap {
  float f[3];
  uint32_t base;  // b0 | b1 << 10 | b2 << 20
};
// a tap record in one 16-byte load (field by field, the loads of later
// fields can be sunk past the branches of the weight evaluation and are then
// waited for one at a time)
__device__ __forceinline__ KTap ktap_load(const KTap* p) {
  const uint4 q = *reinterpret_cast<const uint4*>(p);
  KTap t;
  t.f[0] = __uint_as_float(q.x);
  t.f[1] = __uint_as_float(q.y);
  t.f[2] = __uint_as_float(q.z);
  t.base = q.w;
  return t;
}

// k-space interpolation work of up to kMaxPhasesPerLaunch states in one
// launch (each state has its own trajectory and its own grid): blocks
// first[p] .. first[p + 1] - 1 belong to state p.  Uneven per-state sample
// counts become one launch whose blocks are handed out across states.
template <class T>
struct KBatch {
  int n;
  int first[kMaxPhasesPerLaunch + 1];
  const KTap* taps[kMaxPhasesPerLaunch];   // gather: taps per sample; spread: taps per visit
  int64_t count[kMaxPhasesPerLaunch];      // gather: samples of the state
  const int* gorder[kMaxPhasesPerLaunch];  // gather: samples in processing order (null: index order)
  const KUnit* units[kMaxPhasesPerLaunch]; // spread: work units
  const KSplit* splits[kMaxPhasesPerLaunch];
  const int* vis_off[kMaxPhasesPerLaunch]; // gather into visit order: [M + 1] (null: sample order)
  const int* vis[kMaxPhasesPerLaunch];
  const float2* yin[kMaxPhasesPerLaunch];  // spread input, [visits][C]
  float2* yout[kMaxPhasesPerLaunch];       // gather output
  T* grid[kMaxPhasesPerLaunch];
  float2* partial[kMaxPhasesPerLaunch];
  Blk blk;  // row-blocked layout of every grid of the batch
  const float* oscale;  // gather: results multiplied by oscale[0] (device), unless null
  const float2* phase[kMaxPhasesPerLaunch];  // gather into sample order: times phase[j] (bulk translation), unless null
  // half-precision grids, else null: the gather into visit order takes the
  // largest |re|, |im| of member i into ymax[i kYmaxSlots ...] (zeroed
  // beforehand); the spread stores member i times 2^spread_exp(those, dens[i])
  unsigned* ymax;
  float dens[kMaxPhasesPerLaunch];
  // spread output tile-major instead: the touched tiles one after another,
  // each [TS0][TS1][TS2][C] contiguous at gslot * vol * C (spread and reduce);
  // the spread then stores only the runs fmask marks (the adjoint axis-0
  // pass reads no others)
  int tiled;
  const uint64_t* fmask[kMaxPhasesPerLaunch];  // touched runs per grid column (i1, i2)
};

// the state a block belongs to
__device__ __forceinline__ int batch_member(const int* first, int n, int b) {
  int p = 0;
  while (p + 1 < n && b >= first[p + 1]) ++p;
  return p;
}

// one interpolated value: sum over the 4^NDIM taps of tp of the weights
// times coil c of the grid (times oscale[0] unless null)
template <int NDIM, int S>
__device__ __forceinline__ float2 gather_one(const typename Elem<S>::T* __restrict__ grid, const KTap& tp,
                                             const Blk& blk, int c, int C, const Dims& dm, const KbPoly& kb,
                                             const float* oscale) {
  float w[NDIM][4];
  int g[NDIM][4];
#pragma unroll
  for (int i = 0; i < NDIM; ++i) {
    kb_weights(kb, tp.f[i], w[i]);
    const int b = (tp.base >> (10 * i)) & 1023;
#pragma unroll
    for (int t = 0; t < 4; ++t) g[i][t] = b + t >= dm.G[i] ? b + t - dm.G[i] : b + t;
  }
  float2 acc = make_float2(0.f, 0.f);
  if constexpr (NDIM == 3) {
#pragma unroll
    for (int t0 = 0; t0 < 4; ++t0) {
#pragma unroll
      for (int t1 = 0; t1 < 4; ++t1) {
        const float w01 = w[0][t0] * w[1][t1];
        const typename Elem<S>::T* row = grid + blk.off(g[0][t0], g[1][t1], c);
        float2 s = make_float2(0.f, 0.f);
#pragma unroll
        for (int t2 = 0; t2 < 4; ++t2) {
          const float2 v = Elem<S>::load(row + (int64_t)g[2][t2] * C);
          s.x = fmaf(w[2][t2], v.x, s.x);
          s.y = fmaf(w[2][t2], v.y, s.y);
        }
        acc.x = fmaf(w01, s.x, acc.x);
        acc.y = fmaf(w01, s.y, acc.y);
      }
    }
  } else {
#pragma unroll
    for (int t0 = 0; t0 < 4; ++t0) {
      const typename Elem<S>::T* row = grid + (int64_t)g[0][t0] * blk.rs + c;
      float2 s = make_float2(0.f, 0.f);
#pragma unroll
      for (int t1 = 0; t1 < 4; ++t1) {
        const float2 v = Elem<S>::load(row + (int64_t)g[1][t1] * C);
        s.x = fmaf(w[1][t1], v.x, s.x);
        s.y = fmaf(w[1][t1], v.y, s.y);
      }
      acc.x = fmaf(w[0][t0], s.x, acc.x);
      acc.y = fmaf(w[0][t0], s.y, acc.y);
    }
  }
  return oscale ? cscale(acc, oscale[0]) : acc;
}

// y[j][c] = sum_taps prod_i c(kappa_ji - q_i) grid[q][c], grid [G...][C].
// Lane mapping: each wavefront holds spw = 64 / C samples and lane (s, c)
// interpolates coil c of sample s, so the C coil values of every tap are one
// contiguous run per sample and the output row y[j][*] is one coalesced store.
// With vis_off != null the result of sample j is written to every spread
// visit of the sample (y_visit[v][c] for v in vis[vis_off[j] .. vis_off[j+1]))
// instead of y[j][c], which lets the spread read its inputs contiguously.
// Samples are taken in gorder (grouped by spread tile), so the waves working
// at one time read the same few grid tiles and the grid is fetched from HBM
// about once instead of once per spoke through it; each result is computed
// exactly as in index order.
template <int NDIM, int S>
__global__ __launch_bounds__(kGridThreads) void kgather_kernel(KBatch<typename Elem<S>::T> bt, int C, Dims dm,
                                                               KbPoly kb) {
  const int p = batch_member(bt.first, bt.n, blockIdx.x);
  const typename Elem<S>::T* __restrict__ grid = bt.grid[p];
  const int64_t M = bt.count[p];
  float2* __restrict__ y = bt.yout[p];
  const int* __restrict__ vis_off = bt.vis_off[p];
  const int* __restrict__ vis = bt.vis[p];
  const int lane = threadIdx.x & 63;
  const int spw = 64 / C;
  const int sub = lane / C;
  const int c = lane - sub * C;
  const int64_t wave = (int64_t)(blockIdx.x - bt.first[p]) * (kGridThreads / 64) + (threadIdx.x >> 6);
  const int64_t jo = wave * spw + sub;
  if (wave * spw >= M) return;  // wavefront-uniform
  const bool ok = sub < spw && jo < M;
  const int* __restrict__ gorder = bt.gorder[p];
  const int64_t j = ok && gorder ? (int64_t)gorder[jo] : jo;
  float m = 0.f;
  if (ok) {
    const float2 acc = gather_one<NDIM, S>(grid, ktap_load(bt.taps[p] + j), bt.blk, c, C, dm, kb, bt.oscale);
    m = fmaxf(fabsf(acc.x), fabsf(acc.y));
    if (vis_off) {
      const int v1 = vis_off[j + 1];
      for (int v = vis_off[j]; v < v1; ++v) y[(int64_t)vis[v] * C + c] = acc;
    } else {
      const float2* ph = bt.phase[p];
      y[j * C + c] = ph ? cmul(acc, ph[j]) : acc;
    }
  }
  // every lane of the wavefront is active again here
  if (bt.ymax && vis_off) wave_max_to(bt.ymax + p * kYmaxSlots, m);
}

// y_visit[v][c] = y[order[v]][c]: data in sample order to spread-visit order
// (half-precision grids: also the largest |re|, |im| into the kYmaxSlots
// words at ymax unless null)
// With phase != null the values are multiplied by conj(phase[j]) (the
// adjoint of a bulk translation's linear phase), with w != null by w[j]
// (density compensation).
__global__ __launch_bounds__(kGridThreads) void visit_permute_kernel(const float2* __restrict__ y,
                                                                     const int* __restrict__ order, int64_t nvis,
                                                                     int C, float2* __restrict__ yv,
                                                                     unsigned* __restrict__ ymax,
                                                                     const float2* __restrict__ phase,
                                                                     const float* __restrict__ w) {
  const int64_t e = (int64_t)blockIdx.x * kGridThreads + threadIdx.x;
  float m = 0.f;
  if (e < nvis * C) {
    const int64_t v = e / C;
    const int64_t j = order[v];
    float2 val = y[j * C + (e - v * C)];
    if (phase) val = cmulc(phase[j], val);
    if (w) val = cscale(val, w[j]);
    yv[e] = val;
    m = fmaxf(fabsf(val.x), fabsf(val.y));
  }
  if (ymax) wave_max_to(ymax, m);
}

// Tile of the k-space spread.  The LDS accumulator holds one plane of P
// complex values per coil; inside a plane the point (l0, l1, l2) sits at
// l0 * S0 + l1 * S1 + l2.  P = 4 (mod 16) puts the four coils of a wave on
// distinct banks (2P = 8 mod 32 banks of 4 bytes), and within a coil the
// lanes of one row step along l2, so a 16-lane group touches 32 distinct
// banks.
struct KTile {
  int TS[3];
  int nt[3];
  int vol;        // points per tile
  int S0, S1;     // plane strides (complex values)
  int P;          // plane size (complex values)
  FastDiv rowdiv; // divides by TS_last * C (one tile row of the [G...][C] grid)
};

__device__ __forceinline__ void ktile_origin(int tile, const KTile& kt, int ndim, int lo[3]) {
  int t = tile;
  for (int i = ndim - 1; i >= 0; --i) {
    lo[i] = (t % kt.nt[i]) * kt.TS[i];
    t /= kt.nt[i];
  }
}

// Staged sample of a k-space spread batch: offsets of tap 0 relative to the
// tile origin (tap t of axis i lands on tile row off[i] + t), and the tap
// weights of every axis.
constexpr int kSpreadBatch = 64;
// garbage slots that out-of-tile taps update instead of branching: 4 per lane
constexpr int kSpreadDump = 4 * 64;

// LDS bytes of one k-space spread workgroup for C coils (dynamic part)
__host__ __device__ inline size_t kspread_lds_bytes(const KTile& kt, int C) {
  return sizeof(float2) * ((size_t)C * kt.P + kSpreadDump + (size_t)kSpreadBatch * C);
}

// Touched columns of a tile for the tile-major write-out: s_touch[l1 TS2 +
// l2] = 1 when grid column (lo1 + l1, lo2 + l2) marks the tile's run along
// axis 0 (3D; the tile is one run).  Loaded at the start of a unit so the
// mask reads are done before the write-out needs them.
__device__ __forceinline__ void kspread_touch(const uint64_t* fm, const int lo[3], const KTile& kt, const Dims& dm,
                                              unsigned char* s_touch) {
  const int ncol = kt.TS[1] * kt.TS[2];
  const int run = lo[0] / kt.TS[0];
  for (int e = threadIdx.x; e < ncol; e += blockDim.x) {
    const int l1 = e / kt.TS[2], l2 = e - l1 * kt.TS[2];
    const int g1 = lo[1] + l1, g2 = lo[2] + l2;
    s_touch[e] = (g1 < dm.G[1] && g2 < dm.G[2]) ? (unsigned char)((fm[(int64_t)g1 * dm.G[2] + g2] >> run) & 1ull) : 0;
  }
}

// Write-out of a k-space spread unit from the LDS accumulator (one plane of
// P complex values per coil), row by row: a tile row (fixed l0, l1) is
// TS_last * C contiguous values of the [G...][C] grid.  Thread t takes
// element t mod rowlen of rows t / rowlen, + rpi, + 2 rpi, ... (rpi >= 1
// rows per round, since blockDim >= TS_last C).  Whole tiles of a
// tile-major output store only their touched columns (s_touch); partial
// tiles keep the point-major layout e = point * C + coil.
template <int NDIM, int S>
__device__ __forceinline__ void kspread_write_out(const KBatch<typename Elem<S>::T>& bt, int bp, const KUnit& un,
                                                  const float2* acc, int C, const Dims& dm, const KTile& kt,
                                                  FastDiv cdiv, const int lo[3], const unsigned char* s_touch) {
  typename Elem<S>::T* __restrict__ grid = bt.grid[bp];
  float2* __restrict__ partial = bt.partial[bp];
  const int nthr = blockDim.x;
  const int volC = kt.vol * C;
  const int rowlen = kt.TS[NDIM - 1] * C;
  const int rpi = nthr / rowlen;
  const float hs = bt.ymax ? ldexpf(1.f, spread_exp(bt.ymax + bp * kYmaxSlots, bt.dens[bp])) : 1.f;
  const int r0 = threadIdx.x / rowlen;
  if (r0 >= rpi) return;
  const int within = threadIdx.x - r0 * rowlen;
  const int l2 = (int)cdiv.div((uint32_t)within);  // point along the last axis
  const int cc = within - l2 * C;
  const float2* src = acc + (size_t)cc * kt.P + l2;
  const int gl = lo[NDIM - 1] + l2;
  const bool okl = gl < dm.G[NDIM - 1];
  const int nrows = kt.vol / kt.TS[NDIM - 1];
  if constexpr (NDIM == 3) {
    if (bt.tiled && un.slot < 0) {  // tile-major: one contiguous tile, touched columns only
      typename Elem<S>::T* dst = grid + (int64_t)un.gslot * volC + within;
      for (int row = r0; row < nrows; row += rpi) {
        const int l1 = row % kt.TS[1];
        const int pi = (row / kt.TS[1]) * kt.S0 + l1 * kt.S1;
        if (s_touch[l1 * kt.TS[2] + l2]) Elem<S>::store(dst + row * rowlen, store_scaled<S>(src[pi], hs));
      }
      return;
    }
  }
  for (int row = r0; row < nrows; row += rpi) {
    int l0, l1 = 0, pi;
    if constexpr (NDIM == 3) {
      l0 = row / kt.TS[1];
      l1 = row - l0 * kt.TS[1];
      pi = l0 * kt.S0 + l1 * kt.S1;
    } else {
      l0 = row;
      pi = row * kt.S0;
    }
    const float2 v = src[pi];
    if (un.slot >= 0) {
      partial[(int64_t)un.slot * volC + row * rowlen + within] = v;
      continue;
    }
    const int gl0 = lo[0] + l0;
    bool ok = okl && gl0 < dm.G[0];
    int64_t gi;
    if constexpr (NDIM == 3) {
      const int gl1 = lo[1] + l1;
      ok = ok && gl1 < dm.G[1];
      gi = bt.blk.off(gl0, gl1, (int64_t)gl * C + cc);
    } else {
      gi = bt.blk.off(gl0, gl, cc);
    }
    if (ok) Elem<S>::store(grid + gi, store_scaled<S>(v, hs));
  }
}

// most tile columns of a tiled k-space spread (TS1 TS2 <= 16 x 8)
constexpr int kMaxTileCols = 128;

// k-space spread of one work unit, without atomics.  The unit's samples are
// staged in LDS in batches of kSpreadBatch (tap offsets relative to the tile,
// tap weights, the C coil values); thread s stages sample s, and the loads
// of the next batch are in flight while the current one is accumulated.
// Wave w owns coils 4w .. 4w+3 (their planes
// are its alone); in 3D its 64 lanes are (coil, t2, t1) and each lane
// applies the sample's four t0 taps, in 2D the lanes are (coil, t1, t0).
// Within a wave every lane updates distinct points, so plain LDS
// read-modify-write is race free, and the summation order is fixed (the
// spread is deterministic).  Taps outside the tile, and lanes without a
// coil, update a private garbage slot instead of branching.  The workgroup
// has ceil(C/4) waves.  taps_v and yv are in visit order: the unit's
// samples are taps_v[start .. start + count) and yv[(start ..)][C].
template <int NDIM, int S>
__global__ __launch_bounds__(512) void kspread_kernel(KBatch<typename Elem<S>::T> bt, int C, Dims dm, KTile kt,
                                                      KbPoly kb, FastDiv cdiv) {
  const int bp = batch_member(bt.first, bt.n, blockIdx.x);
  const KTap* __restrict__ taps_v = bt.taps[bp];
  const float2* __restrict__ yv = bt.yin[bp];
  extern __shared__ float2 acc[];  // [C][P] accumulator, [4][64] garbage, [kSpreadBatch][C] coil values
  __shared__ int4 st_off[kSpreadBatch];
  __shared__ float4 st_w[kSpreadBatch][3];
  float2* dump = acc + (size_t)C * kt.P;
  float2* st_y = dump + kSpreadDump;
  const int nthr = blockDim.x;
  const KUnit un = bt.units[bp][blockIdx.x - bt.first[bp]];
  int lo[3] = {0, 0, 0};
  ktile_origin(un.tile, kt, NDIM, lo);
  __shared__ unsigned char s_touch[kMaxTileCols];
  if (NDIM == 3 && bt.tiled && un.slot < 0) kspread_touch(bt.fmask[bp], lo, kt, dm, s_touch);
  {
    float4* a4 = (float4*)acc;
    const int n4 = (C * kt.P) >> 1;  // P is even
    for (int e = threadIdx.x; e < n4; e += nthr) a4[e] = make_float4(0.f, 0.f, 0.f, 0.f);
  }

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int c = 4 * wave + (lane & 3);
  const int ta = (lane >> 2) & 3;  // 3D: t2; 2D: t1
  const int tb = lane >> 4;        // 3D: t1; 2D: t0
  const bool active = c < C;
  const int cr = active ? c : 0;
  float2* plane = acc + (size_t)cr * kt.P;
  float2* mydump = dump + lane;  // slot t at mydump[64 t]

  // The staging is software-pipelined: the coil values and tap records of
  // the next batch are loaded into registers while the current one is
  // accumulated.  nthr = 64 ceil(C/4) >= 16 C, so a batch holds at most
  // kSpreadBatch C / nthr <= 4 coil values per thread.  Addresses are clamped
  // into the batch (always valid), so the loads need no branch.
  constexpr int kYRegs = kSpreadBatch / 16;
  float2 yr[kYRegs];
  KTap tr;
  auto fetch = [&](int b0) {
    const int nb = min(kSpreadBatch, un.count - b0);
    const float2* src = yv + (int64_t)(un.start + b0) * C;
    const int ny = nb * C;
#pragma unroll
    for (int k = 0; k < kYRegs; ++k) yr[k] = src[min((int)threadIdx.x + k * nthr, ny - 1)];
    tr = ktap_load(taps_v + un.start + b0 + min((int)threadIdx.x, nb - 1));
  };
  fetch(0);
  for (int b0 = 0; b0 < un.count; b0 += kSpreadBatch) {
    const int nb = min(kSpreadBatch, un.count - b0);
    __syncthreads();  // previous batch consumed (and the accumulator zeroed)
#pragma unroll
    for (int k = 0; k < kYRegs; ++k) {
      const int e = (int)threadIdx.x + k * nthr;
      if (e < nb * C) st_y[e] = yr[k];
    }
    if ((int)threadIdx.x < nb) {  // thread s stages sample s: per-axis weights and tap-0 offsets
      int off[3] = {0, 0, 0};
#pragma unroll
      for (int i = 0; i < NDIM; ++i) {
        float w[4];
        kb_weights(kb, tr.f[i], w);
        st_w[threadIdx.x][i] = make_float4(w[0], w[1], w[2], w[3]);
        int o = (int)((tr.base >> (10 * i)) & 1023) - lo[i];  // periodic: the image next to the tile
        if (o > dm.G[i] / 2) o -= dm.G[i];
        if (o < -dm.G[i] / 2) o += dm.G[i];
        off[i] = o;
      }
      st_off[threadIdx.x] = make_int4(off[0], off[1], off[2], 0);
    }
    __syncthreads();
    // the next batch (the last one again at the end: valid addresses, unused)
    fetch(b0 + kSpreadBatch < un.count ? b0 + kSpreadBatch : b0);
    // the parameters of sample s + 1 are read before the accumulator update
    // of sample s, so each sample costs one LDS round trip
    int4 of = st_off[0];
    float2 y = st_y[cr];
    float wa = ((const float*)&st_w[0][NDIM - 2])[tb];
    float wb = ((const float*)&st_w[0][NDIM - 1])[ta];
    float4 w0 = st_w[0][0];
    for (int s = 0; s < nb; ++s) {
      const int4 cof = of;
      const float2 cy = y;
      const float cwa = wa, cwb = wb;
      const float4 cw0 = w0;
      {
        const int sn = min(s + 1, nb - 1);  // the last sample re-reads itself
        of = st_off[sn];
        y = st_y[sn * C + cr];
        wa = ((const float*)&st_w[sn][NDIM - 2])[tb];
        wb = ((const float*)&st_w[sn][NDIM - 1])[ta];
        if constexpr (NDIM == 3) w0 = st_w[sn][0];
      }
      if constexpr (NDIM == 3) {
        const int l1 = cof.y + tb, l2 = cof.z + ta;
        const bool lane_ok = active && (unsigned)l1 < (unsigned)kt.TS[1] && (unsigned)l2 < (unsigned)kt.TS[2];
        const float w12 = cwa * cwb;
        const float wt[4] = {cw0.x * w12, cw0.y * w12, cw0.z * w12, cw0.w * w12};
        const int base = cof.x * kt.S0 + l1 * kt.S1 + l2;
        float2* ptr[4];
        float2 v[4];
#pragma unroll
        for (int t0 = 0; t0 < 4; ++t0) {  // read all four, then write all four
          const bool ok = lane_ok && (unsigned)(cof.x + t0) < (unsigned)kt.TS[0];
          ptr[t0] = ok ? plane + (base + t0 * kt.S0) : mydump + 64 * t0;
          v[t0] = *ptr[t0];
        }
#pragma unroll
        for (int t0 = 0; t0 < 4; ++t0)
          *ptr[t0] = make_float2(fmaf(wt[t0], cy.x, v[t0].x), fmaf(wt[t0], cy.y, v[t0].y));
      } else {
        const int l1 = cof.y + ta, l0 = cof.x + tb;
        const bool ok = active && (unsigned)l1 < (unsigned)kt.TS[1] && (unsigned)l0 < (unsigned)kt.TS[0];
        const float ww = cwa * cwb;
        float2* pt = ok ? plane + (l0 * kt.S0 + l1) : mydump;
        const float2 v = *pt;
        *pt = make_float2(fmaf(ww, cy.x, v.x), fmaf(ww, cy.y, v.y));
      }
    }
  }
  __syncthreads();
  kspread_write_out<NDIM, S>(bt, bp, un, acc, C, dm, kt, cdiv, lo, s_touch);
}

// 3D k-space spread of one work unit with register accumulators, for tiles
// of 8 x 4 x 8 and an even number of coils: lane (coil pair, tile column)
// of wave w, coils 4w + 2h and 4w + 2h + 1 (h = lane / 32), holds the 8
// cells of its column (l1, l2) along axis 0 for both coils in registers.
// The staging thread of a sample expands its tap weights over the tile:
// W0[l0] (8 values), W1[l1] (4) and W2[l2] (8) hold the weight of the tap
// that lands on row l of the tile along that axis, zero where none does.
// Every lane then adds W0[l0] W1[l1] W2[l2] y_c to its cells (lanes outside
// the sample's footprint add zero): no cell is shared between lanes, no LDS
// read-modify-write and no branch per sample.  The unit's visits come
// ordered by the rows their four axis-0 taps reach (rows 0-3 only, rows 4-7
// only, both halves; see KUnit), so a batch runs as three branch-free loops
// of which the first two add into four rows only.  The summation order per
// cell is the unit's visit order (deterministic).  Staging as in
// kspread_kernel; the accumulators are stored from registers.
constexpr int kRegW = 20;  // expanded weights per staged sample: W0[8], W1[4], W2[8]

// samples s0 .. s1-1 of the staged batch into rows R0 .. R1-1 of the lane's
// register column (the other rows carry no weight for these samples);
// sample s + 1's parameters are read while sample s is applied
template <int R0, int R1>
__device__ __forceinline__ void kspread_reg_run(int s0, int s1, const float4 (*st_W)[kRegW / 4], const float* stw,
                                                const float2* st_y, int C, int l1, int l2, int cr, int cr1,
                                                float2 (&a0)[8], float2 (&a1)[8]) {
  if (s0 >= s1) return;
  float4 wa = st_W[s0][0], wb = st_W[s0][1];
  float w1 = stw[s0 * kRegW + 8 + l1], w2 = stw[s0 * kRegW + 12 + l2];
  float2 y0 = st_y[s0 * C + cr], y1 = st_y[s0 * C + cr1];
  for (int s = s0; s < s1; ++s) {
    const float4 cwa = wa, cwb = wb;
    const float cw12 = w1 * w2;
    const float2 cy0 = y0, cy1 = y1;
    {
      const int sn = min(s + 1, s1 - 1);
      wa = st_W[sn][0];
      wb = st_W[sn][1];
      w1 = stw[sn * kRegW + 8 + l1];
      w2 = stw[sn * kRegW + 12 + l2];
      y0 = st_y[sn * C + cr];
      y1 = st_y[sn * C + cr1];
    }
    const float2 v0 = make_float2(cw12 * cy0.x, cw12 * cy0.y);
    const float2 v1 = make_float2(cw12 * cy1.x, cw12 * cy1.y);
    const float W0[8] = {cwa.x, cwa.y, cwa.z, cwa.w, cwb.x, cwb.y, cwb.z, cwb.w};
#pragma unroll
    for (int j = R0; j < R1; ++j) {
      a0[j].x = fmaf(W0[j], v0.x, a0[j].x);
      a0[j].y = fmaf(W0[j], v0.y, a0[j].y);
      a1[j].x = fmaf(W0[j], v1.x, a1[j].x);
      a1[j].y = fmaf(W0[j], v1.y, a1[j].y);
    }
  }
}

template <int S>
__global__ __launch_bounds__(512) void kspread_reg_kernel(KBatch<typename Elem<S>::T> bt, int C, Dims dm, KTile kt,
                                                          KbPoly kb, FastDiv cdiv) {
  const int bp = batch_member(bt.first, bt.n, blockIdx.x);
  const KTap* __restrict__ taps_v = bt.taps[bp];
  const float2* __restrict__ yv = bt.yin[bp];
  extern __shared__ float2 st_y[];  // [kSpreadBatch][C] coil values
  __shared__ float4 st_W[kSpreadBatch][kRegW / 4];
  __shared__ unsigned char s_touch[kMaxTileCols];
  const int nthr = blockDim.x;
  const KUnit un = bt.units[bp][blockIdx.x - bt.first[bp]];
  int lo[3] = {0, 0, 0};
  ktile_origin(un.tile, kt, 3, lo);
  if (bt.tiled && un.slot < 0) kspread_touch(bt.fmask[bp], lo, kt, dm, s_touch);
  __syncthreads();  // s_touch visible to every wave (also for a unit without samples)

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 31;
  const int l1 = col >> 3, l2 = col & 7;
  const int c0 = 4 * wave + 2 * (lane >> 5);  // coils c0, c0 + 1
  const bool active = c0 < C;
  const int cr = active ? c0 : 0;
  const int cr1 = active && c0 + 1 < C ? c0 + 1 : cr;  // an odd C's last lane pair reads its coil twice
  float2 a0[8], a1[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a0[j] = a1[j] = make_float2(0.f, 0.f);

  // staging as in kspread_kernel (nthr = 64 ceil(C/4) >= 16 C)
  constexpr int kYRegs = kSpreadBatch / 16;
  float2 yr[kYRegs];
  KTap tr;
  auto fetch = [&](int b0) {
    const int nb = min(kSpreadBatch, un.count - b0);
    const float2* src = yv + (int64_t)(un.start + b0) * C;
    const int ny = nb * C;
#pragma unroll
    for (int k = 0; k < kYRegs; ++k) yr[k] = src[min((int)threadIdx.x + k * nthr, ny - 1)];
    tr = ktap_load(taps_v + un.start + b0 + min((int)threadIdx.x, nb - 1));
  };
  fetch(0);
  const float* stw = (const float*)st_W;
  for (int b0 = 0; b0 < un.count; b0 += kSpreadBatch) {
    const int nb = min(kSpreadBatch, un.count - b0);
    __syncthreads();  // previous batch consumed
#pragma unroll
    for (int k = 0; k < kYRegs; ++k) {
      const int e = (int)threadIdx.x + k * nthr;
      if (e < nb * C) st_y[e] = yr[k];
    }
    if ((int)threadIdx.x < nb) {  // thread s stages sample s: its weights expanded over the tile
      float W[kRegW];
      constexpr int wbase[3] = {0, 8, 12}, wlen[3] = {8, 4, 8};
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        float w[4];
        kb_weights(kb, tr.f[i], w);
        int o = (int)((tr.base >> (10 * i)) & 1023) - lo[i];  // periodic: the image next to the tile
        if (o > dm.G[i] / 2) o -= dm.G[i];
        if (o < -dm.G[i] / 2) o += dm.G[i];
#pragma unroll
        for (int l = 0; l < wlen[i]; ++l) {
          const int t = l - o;
          W[wbase[i] + l] = t == 0 ? w[0] : t == 1 ? w[1] : t == 2 ? w[2] : t == 3 ? w[3] : 0.f;
        }
      }
#pragma unroll
      for (int q = 0; q < kRegW / 4; ++q)
        st_W[threadIdx.x][q] = make_float4(W[4 * q], W[4 * q + 1], W[4 * q + 2], W[4 * q + 3]);
    }
    __syncthreads();
    fetch(b0 + kSpreadBatch < un.count ? b0 + kSpreadBatch : b0);
    // the batch's samples in the unit's row classes (uniform bounds)
    const int e0 = min(max(un.lo - b0, 0), nb), e1 = min(max(un.lohi - b0, 0), nb);
    kspread_reg_run<0, 4>(0, e0, st_W, stw, st_y, C, l1, l2, cr, cr1, a0, a1);
    kspread_reg_run<4, 8>(e0, e1, st_W, stw, st_y, C, l1, l2, cr, cr1, a0, a1);
    kspread_reg_run<0, 8>(e1, nb, st_W, stw, st_y, C, l1, l2, cr, cr1, a0, a1);
  }
  // registers straight to memory (each wave writes a strided third of every
  // tile row; the L2 merges the rows before they reach HBM)
  if (!active) return;
  const bool has1 = c0 + 1 < C;
  const float hs = bt.ymax ? ldexpf(1.f, spread_exp(bt.ymax + bp * kYmaxSlots, bt.dens[bp])) : 1.f;
  const int64_t volC = (int64_t)kt.vol * C;
  const int64_t in_tile = (int64_t)(l1 * kt.TS[2] + l2) * C + c0;  // + l0 TS1 TS2 C
  const int64_t rowC = (int64_t)kt.TS[1] * kt.TS[2] * C;
  if (un.slot >= 0) {  // partial tile, point-major
    float2* dst = bt.partial[bp] + (int64_t)un.slot * volC + in_tile;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      dst[j * rowC] = a0[j];
      if (has1) dst[j * rowC + 1] = a1[j];
    }
    return;
  }
  typename Elem<S>::T* __restrict__ grid = bt.grid[bp];
  if (bt.tiled) {  // tile-major, touched columns only
    if (!s_touch[col]) return;
    typename Elem<S>::T* dst = grid + (int64_t)un.gslot * volC + in_tile;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      Elem<S>::store(dst + j * rowC, store_scaled<S>(a0[j], hs));
      if (has1) Elem<S>::store(dst + j * rowC + 1, store_scaled<S>(a1[j], hs));
    }
    return;
  }
  const int g1 = lo[1] + l1, g2 = lo[2] + l2;  // row-blocked grid
  if (g1 >= dm.G[1] || g2 >= dm.G[2]) return;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (lo[0] + j >= dm.G[0]) break;
    const int64_t gi = bt.blk.off(lo[0] + j, g1, (int64_t)g2 * C + c0);
    Elem<S>::store(grid + gi, store_scaled<S>(a0[j], hs));
    if (has1) Elem<S>::store(grid + gi + 1, store_scaled<S>(a1[j], hs));
  }
}

// sum the partial tiles of every split tile (fixed slot order) and write them

template <int NDIM, int S>
__global__ __launch_bounds__(kGridThreads) void kspread_reduce_kernel(KBatch<typename Elem<S>::T> bt, int C,
                                                                      Dims dm, KTile kt) {
  const int bp = batch_member(bt.first, bt.n, blockIdx.x);
  const float2* __restrict__ partial = bt.partial[bp];
  typename Elem<S>::T* __restrict__ grid = bt.grid[bp];
  const KSplit sp = bt.splits[bp][blockIdx.x - bt.first[bp]];
  int lo[3] = {0, 0, 0};
  ktile_origin(sp.tile, kt, NDIM, lo);
  const int volC = kt.vol * C;
  const float hs = bt.ymax ? ldexpf(1.f, spread_exp(bt.ymax + bp * kYmaxSlots, bt.dens[bp])) : 1.f;
  for (int e = threadIdx.x; e < volC; e += kGridThreads) {
    float2 acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = make_float2(0.f, 0.f);
    int k = 0;
    for (; k + 8 <= sp.nslots; k += 8) {
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = cadd(acc[q], partial[(int64_t)(sp.first_slot + k + q) * volC + e]);
    }
    for (; k < sp.nslots; ++k) acc[0] = cadd(acc[0], partial[(int64_t)(sp.first_slot + k) * volC + e]);
    float2 s = acc[0];
#pragma unroll
    for (int q = 1; q < 8; ++q) s = cadd(s, acc[q]);
    if (bt.tiled) {  // tile-major: the point-major partial layout is the tile's
      Elem<S>::store(grid + (int64_t)sp.gslot * volC + e, store_scaled<S>(s, hs));
      continue;
    }
    const int pt = e / C;
    const int c = e - pt * C;
    int l[3] = {0, 0, 0};
    int t = pt;
    for (int i = NDIM - 1; i >= 0; --i) {
      l[i] = t % kt.TS[i];
      t /= kt.TS[i];
    }
    bool ok = true;
    int g[3] = {0, 0, 0};
    for (int i = 0; i < NDIM; ++i) {
      g[i] = lo[i] + l[i];
      ok = ok && g[i] < dm.G[i];
    }
    const int64_t gi = NDIM == 3 ? bt.blk.off(g[0], g[1], (int64_t)g[2] * C + c) : bt.blk.off(g[0], g[1], c);
    if (ok) Elem<S>::store(grid + gi, store_scaled<S>(s, hs));
  }
}

}  // namespace isg
