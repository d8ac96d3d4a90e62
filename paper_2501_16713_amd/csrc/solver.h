// Conjugate-gradient vector kernels with FP64 inner products and FP64
// scalars kept in device memory, so that a whole iteration can be captured
// in a HIP graph and replayed without any host round trip.
#pragma once

#include "common.h"

namespace isg {

constexpr int kVecThreads = 256;
constexpr int kDotBlocks = 1024;

struct CgScalars {
  double rho;      // <r, r>
  double pq;       // Re <p, N p>
  double alpha;
  double beta;
  int breakdown;   // set once Re<p, N p> <= 0 or not finite
  int iter;        // iterations completed
};

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kVecThreads / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kVecThreads / 64; ++i) s += red[i];
  return s;  // valid in thread 0
}

// partial[b] = sum over block b's grid-stride share of Re(conj(a) b)
__global__ __launch_bounds__(kVecThreads) void dot_partial_kernel(const float2* __restrict__ a,
                                                                  const float2* __restrict__ b, int64_t n,
                                                                  double* __restrict__ partial) {
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads) {
    const float2 x = a[i], y = b[i];
    s += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__device__ __forceinline__ double sum_partials(const double* partial, int np) {
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += kVecThreads) s += partial[i];
  return block_sum(s);
}

// Input scale of a half-precision operator application: sc[0] = 2^-e and
// sc[1] = 2^e with rms(v) = f 2^e, f in [0.5, 1) (1 and 1 for a zero or
// non-finite rms), from sum(partial) = ||v||^2 over n complex values.  The
// coil grids then hold the operator applied to an input of rms in
// [0.5, 1), inside FP16 range whatever the caller's scale, and powers of two
// scale exactly.
__global__ __launch_bounds__(kVecThreads) void half_scale_kernel(const double* __restrict__ partial, int np,
                                                                 int64_t n, float* __restrict__ sc) {
  const double s = sum_partials(partial, np);
  if (threadIdx.x == 0) {
    const double rms = sqrt(s / (double)(n > 0 ? n : 1));
    int e = 0;
    if (rms > 1e-30 && rms < 1e30) (void)frexp(rms, &e);
    sc[0] = ldexpf(1.f, -e);
    sc[1] = ldexpf(1.f, e);
  }
}

// out[0] = sum(partial)
__global__ __launch_bounds__(kVecThreads) void sum_partials_kernel(const double* __restrict__ partial, int np,
                                                                   double* __restrict__ out) {
  const double s = sum_partials(partial, np);
  if (threadIdx.x == 0) out[0] = s;
}

// p[0 .. n) = 0 (a kernel, not a memset node, so graph replays clear it too)
__global__ void zero_u32_kernel(unsigned* __restrict__ p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// rho = sum(partial); hist[0] = sqrt(rho); iter = 0; breakdown = 0
__global__ __launch_bounds__(kVecThreads) void cg_init_kernel(const double* __restrict__ partial, int np,
                                                              CgScalars* sc, double* hist) {
  const double s = sum_partials(partial, np);
  if (threadIdx.x == 0) {
    sc->rho = s;
    sc->iter = 0;
    sc->breakdown = 0;
    sc->alpha = 0.0;
    sc->beta = 0.0;
    hist[0] = sqrt(s);
  }
}

// pq = sum(partial); alpha = rho / pq, or 0 with the breakdown flag set
__global__ __launch_bounds__(kVecThreads) void cg_alpha_kernel(const double* __restrict__ partial, int np,
                                                               CgScalars* sc) {
  const double s = sum_partials(partial, np);
  if (threadIdx.x == 0) {
    sc->pq = s;
    const bool bad = !(s > 0.0) || !isfinite(s) || sc->breakdown;
    if (bad) sc->breakdown = 1;
    sc->alpha = bad ? 0.0 : sc->rho / s;
  }
}

// x += alpha p; r -= alpha q; partial sums of |r|^2
__global__ __launch_bounds__(kVecThreads) void cg_update_xr_kernel(float2* __restrict__ x, float2* __restrict__ r,
                                                                   const float2* __restrict__ p,
                                                                   const float2* __restrict__ q, int64_t n,
                                                                   const CgScalars* __restrict__ sc,
                                                                   double* __restrict__ partial) {
  const float a = (float)sc->alpha;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads) {
    const float2 pi = p[i], qi = q[i];
    float2 xi = x[i], ri = r[i];
    xi.x = fmaf(a, pi.x, xi.x);
    xi.y = fmaf(a, pi.y, xi.y);
    ri.x = fmaf(-a, qi.x, ri.x);
    ri.y = fmaf(-a, qi.y, ri.y);
    x[i] = xi;
    r[i] = ri;
    s += (double)ri.x * ri.x + (double)ri.y * ri.y;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// rho' = sum(partial); beta = rho'/rho; rho = rho'; hist[iter+1] = sqrt(rho')
__global__ __launch_bounds__(kVecThreads) void cg_beta_kernel(const double* __restrict__ partial, int np,
                                                              CgScalars* sc, double* hist) {
  const double s = sum_partials(partial, np);
  if (threadIdx.x == 0) {
    const bool bad = sc->breakdown != 0;
    const double rho_new = bad ? sc->rho : s;
    sc->beta = (bad || sc->rho == 0.0) ? 0.0 : rho_new / sc->rho;
    sc->rho = rho_new;
    sc->iter += 1;
    hist[sc->iter] = sqrt(rho_new);
  }
}

// p = r + beta p
__global__ __launch_bounds__(kVecThreads) void cg_update_p_kernel(float2* __restrict__ p, const float2* __restrict__ r,
                                                                  int64_t n, const CgScalars* __restrict__ sc) {
  if (sc->breakdown) return;
  const float b = (float)sc->beta;
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads) {
    const float2 ri = r[i], pi = p[i];
    p[i] = make_float2(fmaf(b, pi.x, ri.x), fmaf(b, pi.y, ri.y));
  }
}

// out = a - b
__global__ __launch_bounds__(kVecThreads) void sub_kernel(float2* __restrict__ out, const float2* __restrict__ a,
                                                          const float2* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads)
    out[i] = csub(a[i], b[i]);
}

// out += lam * x
__global__ __launch_bounds__(kVecThreads) void axpy_kernel(float2* __restrict__ out, const float2* __restrict__ x,
                                                           float lam, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads) {
    const float2 xi = x[i];
    float2 o = out[i];
    o.x = fmaf(lam, xi.x, o.x);
    o.y = fmaf(lam, xi.y, o.y);
    out[i] = o;
  }
}

__global__ __launch_bounds__(kVecThreads) void copy_kernel(float2* __restrict__ out, const float2* __restrict__ a,
                                                           int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads)
    out[i] = a[i];
}

}  // namespace isg
