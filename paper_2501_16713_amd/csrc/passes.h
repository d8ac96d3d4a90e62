// Load / mid / store functors of the FFT passes that make up the operators.
//
//  image-space gridding, forward front end (Eq. 9: F -> 1/C* -> Z -> F^H):
//    the axis-0 pass runs F along axis 0, divides by C(k/G) on all axes (and
//    by |N|), zero-pads the spectrum and runs F^H of the oversampled length
//    (UpMid), so that pair costs one trip through HBM.
//  image-space gridding, adjoint back end (Eq. 8: F -> Z^H -> 1/C -> F^H):
//    the mirror image (UpHMid).
//  inverse k-space gridding front end (Eq. 3: 1/c* -> Z -> F), per coil:
//    the first pass loads S_c . m, divides by c(x/G), scales by |N|^{-1/2}
//    and zero-pads the centred image (LdCoilExpand).
//  k-space gridding back end (Eq. 2: F^H -> Z^H -> 1/c), followed by the
//    conjugate coil multiply and coil sum of the adjoint SENSE operator
//    (Fig. 3b): the last pass crops, deapodizes, multiplies by conj(S_c) and
//    sums the coils of a line in LDS (StCoilReduce).
#pragma once

#include "fft.h"

namespace isg {

// Separable per-axis factor tables (length n_i each); tab[1] / tab[2] may be
// null for missing axes.
struct AxisTabs {
  const float* t[3];
};

// mid step of the forward upsampling pass along axis 0:
// bin j of the n-point spectrum -> times 1/C(k_j/G) * line factor -> bin
// position of the G-point spectrum (spectral zero-pad).
struct UpMid {
  AxisTabs tab;       // 1/C(k/G) per axis in DFT bin order
  float scale;        // 1/|N|
  int n, G;           // axis-0 lengths
  int n_inner;        // extent of the last axis (3D) or 1 (2D)
  int three_d;
  __device__ void operator()(float2* line, int li, int tl, int tpl, bool active, const TileGeom& g,
                             int64_t a0, int64_t b0) const {
    constexpr int MAXE = kMaxPerThread;
    float2 v[MAXE];
    // table reads are unconditional (index 0 for inactive threads) so the
    // compiler can issue them together instead of one per branch
    float f = scale;
    {
      const int64_t b = active ? b0 + li : 0;  // na == 1 for axis-0 passes
      if (three_d) {
        const int i1 = (int)(b / n_inner), i2 = (int)(b - (int64_t)i1 * n_inner);
        f *= tab.t[1][i1] * tab.t[2][i2];
      } else {
        f *= tab.t[1][b];
      }
    }
#pragma unroll
    for (int i = 0; i < MAXE; ++i) {
      const int j = tl + i * tpl;
      const int jj = active && j < n ? j : 0;
      v[i] = cscale(line[jj], f * tab.t[0][jj]);  // used only when active && j < n
    }
    __syncthreads();
    if (active) {
      for (int j = n / 2 + tl; j < G - n / 2; j += tpl) line[j] = make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < MAXE; ++i) {
      const int j = tl + i * tpl;
      if (active && j < n) line[j < n / 2 ? j : j + G - n] = v[i];
    }
    __syncthreads();
  }
};

// mid step of the adjoint upsampling pass along axis 0: crop the G-point
// spectrum to the n central bins, times 1/C(k_j/G) * line factor.
struct UpHMid {
  AxisTabs tab;
  float scale;
  int n, G;
  int n_inner;
  int three_d;
  __device__ void operator()(float2* line, int li, int tl, int tpl, bool active, const TileGeom& g,
                             int64_t a0, int64_t b0) const {
    constexpr int MAXE = kMaxPerThread;
    float2 v[MAXE];
    // table reads are unconditional (index 0 for inactive threads) so the
    // compiler can issue them together instead of one per branch
    float f = scale;
    {
      const int64_t b = active ? b0 + li : 0;
      if (three_d) {
        const int i1 = (int)(b / n_inner), i2 = (int)(b - (int64_t)i1 * n_inner);
        f *= tab.t[1][i1] * tab.t[2][i2];
      } else {
        f *= tab.t[1][b];
      }
    }
#pragma unroll
    for (int i = 0; i < MAXE; ++i) {
      const int j = tl + i * tpl;
      const int jj = active && j < n ? j : 0;
      v[i] = cscale(line[jj < n / 2 ? jj : jj + G - n], f * tab.t[0][jj]);  // used only when active && j < n
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXE; ++i) {
      const int j = tl + i * tpl;
      if (active && j < n) line[j] = v[i];
    }
    __syncthreads();
  }
};

// First pass of inverse k-space gridding over all coils of a line.
// Lines are (a, c): a indexes the outer image axes (i0 i1 in 3D, i0 in 2D),
// c the coil; the tile holds na outer indices x C coils.  Element j of the
// last axis: S_c[a, j] * m[a, j] * dx_last[j] * dx_outer(a) * scale, placed at
// the centred position of the zero-padded line.
struct LdCoilExpand {
  const float2* m;      // image [A][n]
  const float2* S;      // coils [C][A][n]
  AxisTabs dx;          // 1/C(x/G) per axis over centred positions
  float scale;          // |N|^{-1/2}
  const float* dsc;     // half-precision grids: per-call input scale dsc[0] (device), else null
  int64_t N;            // voxels per coil
  int n, L, C;
  int n1;               // extent of axis 1 (3D) for splitting a; 0 in 2D
  FastDiv nd, cd;
  __device__ void operator()(float2* lines, const TileGeom& g, int64_t a0, int64_t) const {
    const int nl = g.na * C;
    const int gap = L - n;
    for (int e = threadIdx.x; e < nl * gap; e += kFftThreads) {
      const int l = e / gap;
      lines[l * g.LS + n / 2 + (e - l * gap)] = make_float2(0.f, 0.f);
    }
    const int total = nl * n;
    for (int e = threadIdx.x; e < total; e += kFftThreads) {
      const int r = (int)nd.div((uint32_t)e);
      const int j = e - r * n;
      const int al = (int)cd.div((uint32_t)r);
      const int c = r - al * C;
      const int64_t a = a0 + al;
      float2 v = make_float2(0.f, 0.f);
      if (a < g.A) {
        float f = (dsc ? scale * dsc[0] : scale) * dx.t[n1 ? 2 : 1][j];
        if (n1) {
          const int i0 = (int)(a / n1), i1 = (int)(a - (int64_t)i0 * n1);
          f *= dx.t[0][i0] * dx.t[1][i1];
        } else {
          f *= dx.t[0][a];
        }
        const int64_t off = a * n + j;
        v = cscale(cmul(S[(int64_t)c * N + off], m[off]), f);
      }
      lines[(al * C + c) * g.LS + (j < n / 2 ? j + L - n / 2 : j - n / 2)] = v;
    }
  }
};

// Coil-interleaved strided load with element type S (for [..][G][C] grids).
// (LdStrided<S> covers this.)

// Last pass of k-space gridding plus the conjugate coil multiply and coil
// sum: out[a, j] = sum_c conj(S_c[a, j]) * line(a, c)[centred j] * factor.
struct StCoilReduce {
  float2* out;          // image [A][n]
  const float2* S;      // coils [C][A][n]
  AxisTabs dx;
  float scale;
  HalfUndo undo;         // half-precision grids: scales to undo (none for FP32)
  int64_t N;
  int n, L, C;
  int n1;
  FastDiv nd;
  __device__ void operator()(const float2* lines, const TileGeom& g, int64_t a0, int64_t) const {
    const int total = g.na * n;
    const float hs = scale * undo.factor();
    for (int e = threadIdx.x; e < total; e += kFftThreads) {
      const int al = (int)nd.div((uint32_t)e);
      const int j = e - al * n;
      const int64_t a = a0 + al;
      if (a >= g.A) continue;
      float f = hs * dx.t[n1 ? 2 : 1][j];
      if (n1) {
        const int i0 = (int)(a / n1), i1 = (int)(a - (int64_t)i0 * n1);
        f *= dx.t[0][i0] * dx.t[1][i1];
      } else {
        f *= dx.t[0][a];
      }
      const int64_t off = a * n + j;
      const int pos = j < n / 2 ? j + L - n / 2 : j - n / 2;
      float2 acc = make_float2(0.f, 0.f);
      for (int c = 0; c < C; ++c)
        acc = cadd(acc, cmulc(S[(int64_t)c * N + off], lines[(al * C + c) * g.LS + pos]));
      out[off] = cscale(acc, f);
    }
  }
};

}  // namespace isg
