// Batched 1D FFT passes for gfx950, staged in LDS.
//
// A pass transforms a tile of lines along one array axis.  The array is seen
// as [A][L][B] (A outer indices, the transformed axis, B inner indices,
// inner contiguous), and a workgroup owns a tile of na x nb lines: na outer
// indices times nb consecutive inner indices.  Loads and stores walk the
// tile with the inner index fastest, so every wavefront touches runs of nb
// contiguous elements (or whole contiguous lines when B == 1).
//
// Each line is transformed with a Stockham autosort FFT in LDS: for a stage
// of radix R after Ns points have been combined, butterfly i (0 <= i < L/R)
// reads x[i + m L/R], multiplies input m by w^(m k) (k = i mod Ns,
// w = exp(sign 2 pi i / (Ns R))), does an R-point DFT and writes output m to
// (i div Ns) Ns R + k + m Ns.  The output comes out in natural order.
//
// Zero-padding and cropping (the Z and Z^H of Eq. 2, 3, 8, 9) cost no HBM
// traffic: a padded line loads only its n stored values and zero-fills the
// rest in LDS; a cropped line stores only the n kept values.  Pointwise
// factors (deapodization, coil sensitivities, scale) are applied by the load
// and store functors, so they cost no extra pass either.
#pragma once

#include "common.h"

namespace isg {

constexpr int kFftThreads = 256;
constexpr int kMaxPerThread = 32;   // L / threads-per-line must not exceed this
constexpr int kMaxStages = 10;


struct LinePlan {
  int L;                    // transform length
  int nst;                  // number of stages
  int R[kMaxStages];        // radix of each stage
  int step[kMaxStages];     // L / (Ns R): twiddle table stride of each stage
  FastDiv ns[kMaxStages];   // divide by Ns (points already combined)
  const float2* tw;         // device table exp(-2 pi i q / L), q < L
};

// Index maps between a stored axis of length n and a transform of length L.
enum AxisMap {
  kDense = 0,     // n == L
  kSpectral = 1,  // DFT bin order: bin j < n/2 -> j, j >= n/2 -> j + L - n
  kCentred = 2    // centred position x = j - n/2 placed at x mod L
};

__device__ __forceinline__ int map_index(int map, int j, int n, int L) {
  if (map == kSpectral) return j < n / 2 ? j : j + L - n;
  if (map == kCentred) return j < n / 2 ? j + L - n / 2 : j - n / 2;
  return j;
}

// R-point DFT in registers with exponent sign s (-1 forward, +1 inverse).
template <int R> __device__ __forceinline__ void dft(float2* v, float s);

template <> __device__ __forceinline__ void dft<2>(float2* v, float) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <> __device__ __forceinline__ void dft<3>(float2* v, float s) {
  const float h = 0.86602540378443864676f;  // sin(2 pi / 3)
  float2 t = cadd(v[1], v[2]);
  float2 d = cmul_si(csub(v[1], v[2]), s * h);
  float2 m = make_float2(v[0].x - 0.5f * t.x, v[0].y - 0.5f * t.y);
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, d);
  v[2] = csub(m, d);
}

template <> __device__ __forceinline__ void dft<4>(float2* v, float s) {
  float2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  float2 c = cadd(v[1], v[3]), d = cmul_si(csub(v[1], v[3]), s);
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, d);
  v[3] = csub(b, d);
}

template <> __device__ __forceinline__ void dft<5>(float2* v, float s) {
  const float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
  const float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
  const float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
  const float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
  float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  float2 a0 = v[0];
  float2 m1 = make_float2(a0.x + c1 * t1.x + c2 * t2.x, a0.y + c1 * t1.y + c2 * t2.y);
  float2 m2 = make_float2(a0.x + c2 * t1.x + c1 * t2.x, a0.y + c2 * t1.y + c1 * t2.y);
  float2 n1 = cmul_si(make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y), s);
  float2 n2 = cmul_si(make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y), s);
  v[0] = cadd(a0, cadd(t1, t2));
  v[1] = cadd(m1, n1);
  v[4] = csub(m1, n1);
  v[2] = cadd(m2, n2);
  v[3] = csub(m2, n2);
}

// 7 points: pairs t_m = v_m + v_{7-m}, d_m = v_m - v_{7-m} (m = 1..3), so
// X_k = v_0 + sum_m cos(2 pi mk/7) t_m + s i sum_m sin(2 pi mk/7) d_m and
// X_{7-k} the same with the sine sum negated.
template <> __device__ __forceinline__ void dft<7>(float2* v, float s) {
  const float c1 = 0.62348980185873353f;   // cos(2 pi / 7)
  const float c2 = -0.22252093395631440f;  // cos(4 pi / 7)
  const float c3 = -0.90096886790241913f;  // cos(6 pi / 7)
  const float s1 = 0.78183148246802981f;   // sin(2 pi / 7)
  const float s2 = 0.97492791218182361f;   // sin(4 pi / 7)
  const float s3 = 0.43388373911755812f;   // sin(6 pi / 7)
  const float2 a0 = v[0];
  const float2 t1 = cadd(v[1], v[6]), t2 = cadd(v[2], v[5]), t3 = cadd(v[3], v[4]);
  const float2 d1 = csub(v[1], v[6]), d2 = csub(v[2], v[5]), d3 = csub(v[3], v[4]);
  auto re = [&](float a, float b, float c) {
    return make_float2(a0.x + a * t1.x + b * t2.x + c * t3.x, a0.y + a * t1.y + b * t2.y + c * t3.y);
  };
  auto im = [&](float a, float b, float c) {
    return cmul_si(make_float2(a * d1.x + b * d2.x + c * d3.x, a * d1.y + b * d2.y + c * d3.y), s);
  };
  const float2 m1 = re(c1, c2, c3), n1 = im(s1, s2, s3);
  const float2 m2 = re(c2, c3, c1), n2 = im(s2, -s3, -s1);
  const float2 m3 = re(c3, c1, c2), n3 = im(s3, -s1, s2);
  v[0] = cadd(a0, cadd(t1, cadd(t2, t3)));
  v[1] = cadd(m1, n1);
  v[6] = csub(m1, n1);
  v[2] = cadd(m2, n2);
  v[5] = csub(m2, n2);
  v[3] = cadd(m3, n3);
  v[4] = csub(m3, n3);
}

template <> __device__ __forceinline__ void dft<8>(float2* v, float s) {
  // radix-2 split into even/odd radix-4 DFTs, then twiddles exp(s 2 pi i m / 8)
  const float r = 0.70710678118654752440f;
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft<4>(e, s);
  dft<4>(o, s);
  // o[1] *= r (1 + s i); o[2] *= s i; o[3] *= r (-1 + s i)
  float2 o1 = make_float2(r * (o[1].x - s * o[1].y), r * (o[1].y + s * o[1].x));
  float2 o2 = cmul_si(o[2], s);
  float2 o3 = make_float2(r * (-o[3].x - s * o[3].y), r * (-o[3].y + s * o[3].x));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

// One Stockham stage on one line held in LDS.  Every thread of the
// workgroup must call it (it contains barriers); inactive threads pass
// active = false.
template <int R>
__device__ __forceinline__ void fft_stage(float2* line, const LinePlan& lp, int st, int tl, int tpl,
                                          float s, const float2* tw, bool active) {
  constexpr int MAXB = (kMaxPerThread + R - 1) / R;
  const int L = lp.L;
  const int nbf = L / R;
  const int stride = nbf;
  const int step = lp.step[st];
  const FastDiv nsd = lp.ns[st];
  const int Ns = (int)nsd.d;
  float2 v[MAXB][R];
  int obase[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int bf = tl + i * tpl;
    if (active && bf < nbf) {
      const int q = (int)nsd.div((uint32_t)bf);
      const int k = bf - q * Ns;
#pragma unroll
      for (int m = 0; m < R; ++m) v[i][m] = line[bf + m * stride];
      if (Ns > 1) {
#pragma unroll
        for (int m = 1; m < R; ++m) {
          // table holds exp(-2 pi i q/L); for s = +1 take its conjugate, so
          // w = exp(s 2 pi i m k / (Ns R))
          float2 w = tw[m * k * step];
          w.y *= -s;
          v[i][m] = cmul(v[i][m], w);
        }
      }
      dft<R>(v[i], s);
      obase[i] = q * Ns * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int bf = tl + i * tpl;
    if (active && bf < nbf) {
#pragma unroll
      for (int m = 0; m < R; ++m) line[obase[i] + m * Ns] = v[i][m];
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void fft_line(float2* line, const LinePlan& lp, int tl, int tpl, float s,
                                         const float2* tw, bool active) {
  for (int st = 0; st < lp.nst; ++st) {
    switch (lp.R[st]) {
      case 2: fft_stage<2>(line, lp, st, tl, tpl, s, tw, active); break;
      case 3: fft_stage<3>(line, lp, st, tl, tpl, s, tw, active); break;
      case 4: fft_stage<4>(line, lp, st, tl, tpl, s, tw, active); break;
      case 5: fft_stage<5>(line, lp, st, tl, tpl, s, tw, active); break;
      case 7: fft_stage<7>(line, lp, st, tl, tpl, s, tw, active); break;
      default: fft_stage<8>(line, lp, st, tl, tpl, s, tw, active); break;
    }
  }
}

// Tile geometry shared by loads and stores.
struct TileGeom {
  int64_t A, B;     // outer count, inner extent
  int na, nb;       // lines per tile: na outer x nb inner
  int64_t tiles_b;  // ceil(B / nb)
  int LS;           // LDS line stride in float2
};

struct PassDesc {
  TileGeom g;
  LinePlan l1;      // first transform
  LinePlan l2;      // second transform (two-transform passes only)
  float s1, s2;     // exponent signs
  int two;          // 1 if a second transform follows the first
};

// The pass kernel.  Ld fills the tile's lines in LDS (including zero-fill of
// padded entries); Mid (two-transform passes) maps the result of the first
// transform onto the input of the second; St writes the tile back.
template <class Ld, class Mid, class St>
__global__ __launch_bounds__(kFftThreads) void fft_pass_kernel(Ld ld, Mid mid, St st, PassDesc pd) {
  extern __shared__ float2 smem[];
  const int tid = threadIdx.x;
  float2* tw1 = smem;
  float2* tw2 = smem + pd.l1.L;
  float2* lines = tw2 + (pd.two ? pd.l2.L : 0);
  for (int i = tid; i < pd.l1.L; i += kFftThreads) tw1[i] = pd.l1.tw[i];
  if (pd.two)
    for (int i = tid; i < pd.l2.L; i += kFftThreads) tw2[i] = pd.l2.tw[i];

  const int64_t tile = (int64_t)blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
  const int64_t ta = tile / pd.g.tiles_b;
  const int64_t a0 = ta * pd.g.na;
  const int64_t b0 = (tile - ta * pd.g.tiles_b) * pd.g.nb;
  if (a0 >= pd.g.A) return;  // whole workgroup exits together

  ld(lines, pd.g, a0, b0);
  __syncthreads();

  const int nl = pd.g.na * pd.g.nb;
  const int tpl = kFftThreads / nl;
  const int li = tid / tpl;
  const int tl = tid - li * tpl;
  const bool active = li < nl;
  float2* line = lines + (active ? li : 0) * pd.g.LS;
  fft_line(line, pd.l1, tl, tpl, pd.s1, tw1, active);
  if (pd.two) {
    mid(line, li, tl, tpl, active, pd.g, a0, b0);
    fft_line(line, pd.l2, tl, tpl, pd.s2, tw2, active);
  }
  st(lines, pd.g, a0, b0);
}

struct NoMid {
  __device__ void operator()(float2*, int, int, int, bool, const TileGeom&, int64_t, int64_t) const {}
};

// ---------------------------------------------------------------------------
// Generic strided load / store.
// element (al, j, bl) of the tile lives at p[(a0+al)*sa + j*sj + (b0+bl)].
// ---------------------------------------------------------------------------
template <int S>
struct LdStrided {
  const typename Elem<S>::T* p;
  int64_t sa, sj;
  int n;        // stored length along the axis
  int L;        // transform length
  int map;      // AxisMap
  FastDiv nbd, nd;
  __device__ void operator()(float2* lines, const TileGeom& g, int64_t a0, int64_t b0) const {
    const int nl = g.na * g.nb;
    if (n < L) {  // zero the entries the stored values do not cover
      const int gap = L - n;
      const int lo = (map == kCentred) ? (n - n / 2) : n / 2;  // first gap slot
      for (int e = threadIdx.x; e < nl * gap; e += kFftThreads) {
        const int l = e / gap;
        lines[l * g.LS + lo + (e - l * gap)] = make_float2(0.f, 0.f);
      }
    }
    // U elements per thread and round, all loads issued before the LDS
    // stores (unconditional loads from p itself for out-of-range elements)
    constexpr int U = 4;
    const int total = nl * n;
    for (int e0 = threadIdx.x; e0 < total; e0 += U * kFftThreads) {
      float2 v[U];
      int dst[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * kFftThreads;
        const bool in = e < total;
        const int ee = in ? e : 0;
        const int r = (int)nbd.div((uint32_t)ee);
        const int bl = ee - r * g.nb;
        const int al = (int)nd.div((uint32_t)r);
        const int j = r - al * n;
        const int64_t a = a0 + al, b = b0 + bl;
        const bool ok = in && a < g.A && b < g.B;
        const float2 x = Elem<S>::load(ok ? p + a * sa + (int64_t)j * sj + b : p);
        v[u] = ok ? x : make_float2(0.f, 0.f);
        dst[u] = in ? (al * g.nb + bl) * g.LS + map_index(map, j, n, L) : -1;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (dst[u] >= 0) lines[dst[u]] = v[u];
    }
  }
};

template <int S>
struct StStrided {
  typename Elem<S>::T* p;
  int64_t sa, sj;
  int n;        // stored length along the axis (n <= L: crop)
  int L;
  int map;
  float scale;  // applied to half-precision stores only
  FastDiv nbd, nd;
  __device__ void operator()(const float2* lines, const TileGeom& g, int64_t a0, int64_t b0) const {
    const int nl = g.na * g.nb;
    const int total = nl * n;
    for (int e = threadIdx.x; e < total; e += kFftThreads) {
      const int r = (int)nbd.div((uint32_t)e);
      const int bl = e - r * g.nb;
      const int al = (int)nd.div((uint32_t)r);
      const int j = r - al * n;
      const int64_t a = a0 + al, b = b0 + bl;
      if (a < g.A && b < g.B)
        Elem<S>::store(p + a * sa + (int64_t)j * sj + b,
                       store_scaled<S>(lines[(al * g.nb + bl) * g.LS + map_index(map, j, n, L)], scale));
    }
  }
};

}  // namespace isg
