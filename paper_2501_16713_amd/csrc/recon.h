// Kernels of the reconstruction layer around the operators: the orthonormal
// Haar wavelet and soft threshold of wavelet-FISTA (Eq. 11, Eq. 13), the
// FISTA and power-iteration vector updates, the gradient-descent
// registration of displacement fields, the linear phase of a bulk
// translation and the density compensation of direct gridding.
#pragma once

#include "common.h"
#include "gridding.h"
#include "solver.h"

namespace isg {

constexpr float kInvSqrt2 = 0.70710678118654752440f;

// Extents of an image box and the strides of the array it lives in
// (2D: n2 = 1).
struct Box {
  int b[3];      // box extents (even on every wavelet axis)
  int64_t s[3];  // strides of the array (s2 = 1)
};

// One level of the orthonormal Haar transform on the box [0, b0) x [0, b1)
// x [0, b2): along every axis the pair (2j, 2j + 1) maps to the low-pass
// value (x_2j + x_2j+1)/sqrt2 at j and the high-pass value
// (x_2j - x_2j+1)/sqrt2 at j + b/2.  Thread per 2 x 2 (x 2) block; src and
// dst are different arrays.  INV = 1 runs the inverse map.
template <int NDIM, int INV>
__global__ __launch_bounds__(256) void haar_level_kernel(const float2* __restrict__ src, Box sb,
                                                         float2* __restrict__ dst, Box db) {
  const int h0 = sb.b[0] >> 1, h1 = sb.b[1] >> 1, h2 = NDIM == 3 ? sb.b[2] >> 1 : 1;
  const int64_t nblk = (int64_t)h0 * h1 * h2;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= nblk) return;
  const int k = (int)(t % h2);
  const int j = (int)((t / h2) % h1);
  const int i = (int)(t / ((int64_t)h1 * h2));
  constexpr int Q = NDIM == 3 ? 8 : 4;
  float2 v[Q];
  // element e = (a, b, c) bits: a along axis 0 (value 4 in 3D, 2 in 2D), ...
  auto pos_block = [&](int e, const Box& bx) {  // (2i + a, 2j + b, 2k + c)
    const int a = NDIM == 3 ? (e >> 2) & 1 : (e >> 1) & 1, bb = NDIM == 3 ? (e >> 1) & 1 : e & 1, c = e & 1;
    return (2 * i + a) * bx.s[0] + (int64_t)(2 * j + bb) * bx.s[1] + (NDIM == 3 ? 2 * k + c : 0);
  };
  auto pos_band = [&](int e, const Box& bx) {  // (i + a h0, j + b h1, k + c h2)
    const int a = NDIM == 3 ? (e >> 2) & 1 : (e >> 1) & 1, bb = NDIM == 3 ? (e >> 1) & 1 : e & 1, c = e & 1;
    return (i + a * h0) * bx.s[0] + (int64_t)(j + bb * h1) * bx.s[1] + (NDIM == 3 ? k + c * h2 : 0);
  };
#pragma unroll
  for (int e = 0; e < Q; ++e) v[e] = INV ? src[pos_band(e, sb)] : src[pos_block(e, sb)];
  // the 1D map along each axis: pairs differing in that axis's bit
#pragma unroll
  for (int ax = 0; ax < NDIM; ++ax) {
    const int bit = 1 << (NDIM - 1 - ax);
#pragma unroll
    for (int e = 0; e < Q; ++e) {
      if (e & bit) continue;
      const float2 p = v[e], q = v[e | bit];
      v[e] = make_float2((p.x + q.x) * kInvSqrt2, (p.y + q.y) * kInvSqrt2);
      v[e | bit] = make_float2((p.x - q.x) * kInvSqrt2, (p.y - q.y) * kInvSqrt2);
    }
  }
#pragma unroll
  for (int e = 0; e < Q; ++e) {
    if (INV)
      dst[pos_block(e, db)] = v[e];
    else
      dst[pos_band(e, db)] = v[e];
  }
}

// dst box <- src box (box extents equal, strides may differ)
__global__ __launch_bounds__(256) void box_copy_kernel(const float2* __restrict__ src, Box sb,
                                                       float2* __restrict__ dst, Box db, int ndim) {
  const int64_t n = (int64_t)sb.b[0] * sb.b[1] * (ndim == 3 ? sb.b[2] : 1);
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const int b2 = ndim == 3 ? sb.b[2] : 1;
  const int k = (int)(t % b2);
  const int j = (int)((t / b2) % sb.b[1]);
  const int i = (int)(t / ((int64_t)b2 * sb.b[1]));
  dst[i * db.s[0] + (int64_t)j * db.s[1] + k] = src[i * sb.s[0] + (int64_t)j * sb.s[1] + k];
}

// Soft threshold of every detail coefficient (outside the approximation
// box [0, a0) x [0, a1) x [0, a2)): c max(0, 1 - tau/|c|).
__global__ __launch_bounds__(256) void soft_threshold_kernel(float2* __restrict__ w, int64_t n, int n1, int n2,
                                                             int a0, int a1, int a2, float tau) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const int k = (int)(t % n2);
  const int j = (int)((t / n2) % n1);
  const int i = (int)(t / ((int64_t)n2 * n1));
  if (i < a0 && j < a1 && k < a2) return;
  const float2 c = w[t];
  const float m = sqrtf(c.x * c.x + c.y * c.y);
  const float s = m > tau ? 1.f - tau / m : 0.f;
  w[t] = make_float2(c.x * s, c.y * s);
}

// FISTA gradient step: v = z - c (q - b), q = A^H A z, b = A^H y, c = 2 / L
__global__ __launch_bounds__(kVecThreads) void fista_step_kernel(float2* __restrict__ v, const float2* __restrict__ z,
                                                                 const float2* __restrict__ q,
                                                                 const float2* __restrict__ b, float c, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads) {
    const float2 zz = z[i], qq = q[i], bb = b[i];
    v[i] = make_float2(zz.x - c * (qq.x - bb.x), zz.y - c * (qq.y - bb.y));
  }
}

// FISTA momentum: z = x_new + beta (x_new - x), then x = x_new; with a
// non-null `part`, the partial sums of ||x_new - x||^2 per block (FP64)
__global__ __launch_bounds__(kVecThreads) void fista_momentum_kernel(float2* __restrict__ z, float2* __restrict__ x,
                                                                     const float2* __restrict__ xn, float beta,
                                                                     int64_t n, double* __restrict__ part) {
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads) {
    const float2 a = xn[i], o = x[i];
    const float dx = a.x - o.x, dy = a.y - o.y;
    z[i] = make_float2(a.x + beta * dx, a.y + beta * dy);
    x[i] = a;
    s += (double)dx * dx + (double)dy * dy;
  }
  if (part) {
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
  }
}

// hist[k] = sqrt(sum(part)) (a norm from partial sums of squares)
__global__ __launch_bounds__(kVecThreads) void norm_to_kernel(const double* __restrict__ part, int np,
                                                              double* __restrict__ out) {
  const double s = sum_partials(part, np);
  if (threadIdx.x == 0) out[0] = sqrt(s);
}

// v = w / nrm[0] (power iteration; nrm on the device)
__global__ __launch_bounds__(kVecThreads) void scale_by_inverse_kernel(float2* __restrict__ v,
                                                                       const float2* __restrict__ w,
                                                                       const double* __restrict__ nrm, int64_t n) {
  const float f = (float)(1.0 / nrm[0]);
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads)
    v[i] = cscale(w[i], f);
}

// ---------------------------------------------------------------------------
// registration: E(d) = ||T_d m_ref - m_mov||^2 + mu sum_i sum_a ||D_a d_i||^2
// ---------------------------------------------------------------------------
// r = m - mov, and the partial sums of ||r||^2 per block
__global__ __launch_bounds__(kVecThreads) void residual_kernel(float2* __restrict__ r, const float2* __restrict__ m,
                                                               const float2* __restrict__ mov, int64_t n,
                                                               double* __restrict__ part) {
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads) {
    const float2 a = m[i], b = mov[i];
    const float2 d = make_float2(a.x - b.x, a.y - b.y);
    r[i] = d;
    s += (double)d.x * d.x + (double)d.y * d.y;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// periodic neighbour offsets of voxel r along every axis
template <int NDIM>
__device__ __forceinline__ void neighbours(int64_t r, const Dims& dm, int64_t up[3], int64_t dn[3]) {
  int ri[3];
  voxel_coords<NDIM>(r, dm, ri);
  int64_t stride = 1;
#pragma unroll
  for (int a = NDIM - 1; a >= 0; --a) {
    up[a] = r + (ri[a] + 1 < dm.n[a] ? stride : -(int64_t)(dm.n[a] - 1) * stride);
    dn[a] = r + (ri[a] > 0 ? -stride : (int64_t)(dm.n[a] - 1) * stride);
    stride *= dm.n[a];
  }
}

// partial sums (per block) of sum_i sum_a (d_i[r + e_a] - d_i[r])^2
template <int NDIM>
__global__ __launch_bounds__(kVecThreads) void smoothness_kernel(const float* __restrict__ d, Dims dm,
                                                                 double* __restrict__ part) {
  double s = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; r < dm.N; r += (int64_t)gridDim.x * kVecThreads) {
    int64_t up[3], dn[3];
    neighbours<NDIM>(r, dm, up, dn);
#pragma unroll
    for (int i = 0; i < NDIM; ++i) {
      const float* di = d + (int64_t)i * dm.N;
      const double c = di[r];
#pragma unroll
      for (int a = 0; a < NDIM; ++a) {
        const double e = (double)di[up[a]] - c;
        s += e * e;
      }
    }
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// hist[k] = sum(pdata) + mu sum(psmooth)
__global__ __launch_bounds__(kVecThreads) void energy_kernel(const double* __restrict__ pdata,
                                                             const double* __restrict__ psmooth, int np, double mu,
                                                             double* __restrict__ out) {
  const double a = sum_partials(pdata, np);
  __syncthreads();
  const double b = sum_partials(psmooth, np);
  if (threadIdx.x == 0) out[0] = a + mu * b;
}

// d_new = d - step (2 g + 2 mu (-Lap d)), g = Re(conj(r) dT/dd) per
// component (periodic Laplacian); d_new != d
template <int NDIM>
__global__ __launch_bounds__(kVecThreads) void register_update_kernel(float* __restrict__ dnew,
                                                                      const float* __restrict__ d,
                                                                      const float* __restrict__ g, Dims dm, float mu,
                                                                      float step) {
  for (int64_t r = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; r < dm.N; r += (int64_t)gridDim.x * kVecThreads) {
    int64_t up[3], dn[3];
    neighbours<NDIM>(r, dm, up, dn);
#pragma unroll
    for (int i = 0; i < NDIM; ++i) {
      const float* di = d + (int64_t)i * dm.N;
      const float c = di[r];
      float lap = 0.f;  // -Lap
#pragma unroll
      for (int a = 0; a < NDIM; ++a) lap += 2.f * c - di[up[a]] - di[dn[a]];
      const float grad = 2.f * g[(int64_t)i * dm.N + r] + 2.f * mu * lap;
      dnew[(int64_t)i * dm.N + r] = c - step * grad;
    }
  }
}

// ---------------------------------------------------------------------------
// bulk translation: ph_j = exp(-2 pi i k_j . t_j) (FP64 argument)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void shift_phase_kernel(const float* __restrict__ k, const float* __restrict__ t,
                                                          int ndim, int64_t M, float2* __restrict__ ph) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= M) return;
  double a = 0.0;
  for (int i = 0; i < ndim; ++i) a += (double)k[j * ndim + i] * (double)t[j * ndim + i];
  a -= rint(a);  // the phase is periodic in a; keep the argument small
  double s, c;
  sincospi(2.0 * a, &s, &c);
  ph[j] = make_float2((float)c, (float)-s);
}

// ---------------------------------------------------------------------------
// density compensation (Pipe and Menon): w <- w / (P w), P = gather o spread
// of real weights on the oversampled grid
// ---------------------------------------------------------------------------
// grid[q] += w_j prod_i c(kappa_ji - q_i) over the 4^ndim taps (atomic adds:
// the summation order varies from run to run, in the last bits only)
template <int NDIM>
__global__ __launch_bounds__(256) void dcf_spread_kernel(const KTap* __restrict__ taps, const float* __restrict__ w,
                                                         int64_t M, float* __restrict__ grid, Dims dm, KbPoly kb) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= M) return;
  const KTap tp = ktap_load(taps + j);
  float wt[NDIM][4];
  int g[NDIM][4];
#pragma unroll
  for (int i = 0; i < NDIM; ++i) {
    kb_weights(kb, tp.f[i], wt[i]);
    const int b = (tp.base >> (10 * i)) & 1023;
#pragma unroll
    for (int t = 0; t < 4; ++t) g[i][t] = b + t >= dm.G[i] ? b + t - dm.G[i] : b + t;
  }
  const float v = w[j];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if constexpr (NDIM == 3) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
          atomicAdd(grid + ((int64_t)g[0][a] * dm.G[1] + g[1][b]) * dm.G[2] + g[2][c],
                    v * wt[0][a] * wt[1][b] * wt[2][c]);
      } else {
        atomicAdd(grid + (int64_t)g[0][a] * dm.G[1] + g[1][b], v * wt[0][a] * wt[1][b]);
      }
    }
}

// w_j <- w_j / sum_taps prod_i c(kappa_ji - q_i) grid[q] (the kernel
// scaled to unit integral per axis, as the plan's kernel tables are)
template <int NDIM>
__global__ __launch_bounds__(256) void dcf_update_kernel(const KTap* __restrict__ taps, float* __restrict__ w,
                                                         int64_t M, const float* __restrict__ grid, Dims dm,
                                                         KbPoly kb) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= M) return;
  const KTap tp = ktap_load(taps + j);
  float wt[NDIM][4];
  int g[NDIM][4];
#pragma unroll
  for (int i = 0; i < NDIM; ++i) {
    kb_weights(kb, tp.f[i], wt[i]);
    const int b = (tp.base >> (10 * i)) & 1023;
#pragma unroll
    for (int t = 0; t < 4; ++t) g[i][t] = b + t >= dm.G[i] ? b + t - dm.G[i] : b + t;
  }
  float acc = 0.f;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if constexpr (NDIM == 3) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc = fmaf(wt[0][a] * wt[1][b] * wt[2][c], grid[((int64_t)g[0][a] * dm.G[1] + g[1][b]) * dm.G[2] + g[2][c]], acc);
      } else {
        acc = fmaf(wt[0][a] * wt[1][b], grid[(int64_t)g[0][a] * dm.G[1] + g[1][b]], acc);
      }
    }
  w[j] = w[j] / acc;
}

__global__ void fill_f32_kernel(float* __restrict__ p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

}  // namespace isg
