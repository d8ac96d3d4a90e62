// Shared device helpers: complex arithmetic on float2 and the Kaiser-Bessel
// interpolation kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace isg {

constexpr int kWidth = 4;   // kernel width in oversampled-grid cells
constexpr int kAlpha = 2;   // oversampling factor
constexpr int kPolyDeg = 17;

// q = n / d for 0 <= n < 2^31 via a multiply-high (Granlund-Montgomery).
struct FastDiv {
  uint32_t d, m, s;
  __device__ __forceinline__ uint32_t div(uint32_t n) const { return (__umulhi(n, m) + n) >> s; }
  __device__ __forceinline__ uint32_t mod(uint32_t n) const { return n - div(n) * d; }
};

// Row-blocked layout of a coil-expanded array [R][G1][G2][C] (2D: [R][G1][C],
// with G2 C read as C): blocks of T = 2^tlog consecutive i1 keep their R rows
// together, so consecutive i0 are T G2 C elements apart instead of
// G1 G2 C.  Element (i0, i1, rest), rest = i2 C + c, sits at
//   (i1 >> tlog) bs + i0 rs + (i1 & (T - 1)) g2c + rest.
// tlog = 30 is the plain row-major layout (rs = G1 G2 C).
struct Blk {
  int tlog;
  int64_t rs;   // i0 stride
  int64_t bs;   // stride of a block of T values of i1
  int64_t g2c;  // i1 stride inside a block (G2 C)
  FastDiv g2cdiv;
  __device__ __forceinline__ int64_t off(int64_t i0, int i1, int64_t rest) const {
    return (int64_t)(i1 >> tlog) * bs + i0 * rs + (int64_t)(i1 & ((1 << tlog) - 1)) * g2c + rest;
  }
  // offset of column b = i1 G2 C + rest at i0 = 0 (b < 2^31)
  __device__ __forceinline__ int64_t col(int64_t b) const {
    const uint32_t i1 = g2cdiv.div((uint32_t)b);
    return off(0, (int)i1, b - (int64_t)i1 * g2c);
  }
};

// ---------------------------------------------------------------------------
// complex64 helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by s*i (s = +-1): (s i)(x + i y) = s(-y + i x)
__device__ __forceinline__ float2 cmul_si(float2 a, float s) { return make_float2(-s * a.y, s * a.x); }

// ---------------------------------------------------------------------------
// Kaiser-Bessel kernel c(u) = I0(beta sqrt(1 - (2u/W)^2)), |u| < W/2.
//
// With t = 1 - (u/2)^2 (W = 4), I0(beta sqrt(t)) = sum_k a_k t^k with
// a_k = (beta^2/4)^k / (k!)^2 (the power series of I0).  All a_k are
// positive and t is in [0, 1], so Horner's rule is well conditioned.  The
// host fills the coefficients in FP64 (degree 17: truncation < 1e-9
// relative) and passes them by value.
// ---------------------------------------------------------------------------
struct KbPoly {
  float a[kPolyDeg + 1];   // c as a polynomial in t
  float da[kPolyDeg];      // dc/dt
};

__device__ __forceinline__ float kb_poly(const KbPoly& k, float t) {
  float s = k.a[kPolyDeg];
#pragma unroll
  for (int i = kPolyDeg - 1; i >= 0; --i) s = fmaf(s, t, k.a[i]);
  return s;
}

__device__ __forceinline__ float kb_dpoly(const KbPoly& k, float t) {
  float s = k.da[kPolyDeg - 1];
#pragma unroll
  for (int i = kPolyDeg - 2; i >= 0; --i) s = fmaf(s, t, k.da[i]);
  return s;
}

// Weights of the four taps g = floor(y) - 1 + m, m = 0..3, for a coordinate
// with fractional part f = y - floor(y) in [0, 1).  The tap offset is
// u_m = f + 1 - m and t_m = 1 - u_m^2/4 = (1 - f + m)(3 + f - m)/4, written
// as a product so that no cancellation happens near the support edge.  The
// last tap sits at u = -2 when f == 0, where the open-support kernel is 0.
__device__ __forceinline__ void kb_weights(const KbPoly& k, float f, float w[4]) {
  w[0] = kb_poly(k, (1.0f - f) * (3.0f + f) * 0.25f);
  w[1] = kb_poly(k, (2.0f - f) * (2.0f + f) * 0.25f);
  w[2] = kb_poly(k, (3.0f - f) * (1.0f + f) * 0.25f);
  w[3] = (f > 0.0f) ? kb_poly(k, (4.0f - f) * f * 0.25f) : 0.0f;
}

// Weights and their derivatives with respect to the coordinate y:
// dc/du = dc/dt * dt/du with dt/du = -u/2.
__device__ __forceinline__ void kb_weights_deriv(const KbPoly& k, float f, float w[4], float dw[4]) {
  float t0 = (1.0f - f) * (3.0f + f) * 0.25f;
  float t1 = (2.0f - f) * (2.0f + f) * 0.25f;
  float t2 = (3.0f - f) * (1.0f + f) * 0.25f;
  float t3 = (4.0f - f) * f * 0.25f;
  w[0] = kb_poly(k, t0);
  w[1] = kb_poly(k, t1);
  w[2] = kb_poly(k, t2);
  w[3] = (f > 0.0f) ? kb_poly(k, t3) : 0.0f;
  dw[0] = kb_dpoly(k, t0) * (-(f + 1.0f) * 0.5f);
  dw[1] = kb_dpoly(k, t1) * (-f * 0.5f);
  dw[2] = kb_dpoly(k, t2) * (-(f - 1.0f) * 0.5f);
  dw[3] = (f > 0.0f) ? kb_dpoly(k, t3) * (-(f - 2.0f) * 0.5f) : 0.0f;
}

// ---------------------------------------------------------------------------
// grid element storage: complex64, or a pair of bf16 / fp16 halves
// ---------------------------------------------------------------------------
enum Storage { kFP32 = 0, kBF16 = 1, kFP16 = 2 };

template <int S> struct Elem;
template <> struct Elem<kFP32> {
  using T = float2;
  __device__ static __forceinline__ float2 load(const T* p) { return *p; }
  __device__ static __forceinline__ void store(T* p, float2 v) { *p = v; }
};
template <> struct Elem<kBF16> {
  using T = __hip_bfloat162;
  __device__ static __forceinline__ float2 load(const T* p) { return __bfloat1622float2(*p); }
  __device__ static __forceinline__ void store(T* p, float2 v) { *p = __float22bfloat162_rn(v); }
};
template <> struct Elem<kFP16> {
  using T = __half2;
  __device__ static __forceinline__ float2 load(const T* p) { return __half22float2(*p); }
  __device__ static __forceinline__ void store(T* p, float2 v) { *p = __float22half2_rn(v); }
};

// Half-precision grids are stored with a per-pass scale that keeps every
// intermediate on the scale of the k-space data; FP32 grids take the whole
// |N|^{-1/2} at the first load and store unscaled.
template <int S>
__device__ __forceinline__ float2 store_scaled(float2 v, float s) {
  if constexpr (S == kFP32) {
    return v;
  } else {
    return make_float2(v.x * s, v.y * s);
  }
}

// Half-precision spread output.  Radial sampling piles thousands of samples
// onto the cells near the k-space centre, so an unscaled spread of data of
// any magnitude overflows FP16.  Each state's spread output is stored times
// 2^e with e the largest exponent keeping dens * 2 * ymax * 2^e below
// kHalfSpreadTarget: dens bounds how many samples reach one cell (every
// kernel weight is at most 1), ymax is the largest |re| or |im| of the data
// (|z| <= sqrt 2 max(|re|, |im|)), so no stored cell can exceed the target.
// The target leaves headroom for the next pass (a line of 2n values summed
// and scaled by n^{-1/2}).  Powers of two scale exactly; zero or non-finite
// data takes e = 0.
// ymax of one state is kept over kYmaxSlots words (wavefronts pick one by
// index, readers take the largest), so the atomics of a launch do not all
// meet at one address.
constexpr float kHalfSpreadTarget = 1024.f;
constexpr int kYmaxSlots = 64;
__device__ __forceinline__ int spread_exp(const unsigned* ymax, float dens) {
  unsigned b = 0u;
  const uint4* y4 = reinterpret_cast<const uint4*>(ymax);
#pragma unroll
  for (int i = 0; i < kYmaxSlots / 4; ++i) {
    const uint4 v = y4[i];
    b = max(b, max(max(v.x, v.y), max(v.z, v.w)));
  }
  const float m = __uint_as_float(b);
  if (!(m > 0.f) || !(m < __builtin_inff())) return 0;
  const float v = kHalfSpreadTarget / (2.f * dens * m);
  if (!(v < __builtin_inff())) return 120;
  int e;
  (void)frexpf(v, &e);  // v = f 2^e with f in [0.5, 1)
  return max(-120, min(120, e - 1));
}

// ymax[slot] = max(ymax[slot], m) over the 64 lanes of the calling
// wavefront, slot chosen by the wavefront's index (m >= 0; every lane must be
// active; one atomic per wavefront; non-negative floats order as their bit
// patterns)
__device__ __forceinline__ void wave_max_to(unsigned* ymax, float m) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  const unsigned w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 0) atomicMax(ymax + (w & (kYmaxSlots - 1)), __float_as_uint(m));
}

// What the coil reduction multiplies by to undo the half-precision scales:
// dsc[0] (the inverse of the input scale of a normal-operator call) unless
// null, times 2^-e of the state's spread output unless ymax is null.
struct HalfUndo {
  const float* dsc = nullptr;
  const unsigned* ymax = nullptr;
  float dens = 1.f;
  __device__ __forceinline__ float factor() const {
    float f = dsc ? dsc[0] : 1.f;
    if (ymax) f *= ldexpf(1.f, -spread_exp(ymax, dens));
    return f;
  }
};

}  // namespace isg
