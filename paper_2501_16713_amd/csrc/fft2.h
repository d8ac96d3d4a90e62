// Two-step register FFT for lines of compile-time length L = L1 * L2.
//
// With n = L2 n1 + n2 and k = k1 + L1 k2 (Cooley-Tukey, decimation in time):
//   X[k1 + L1 k2] = sum_n2 w_L^(n2 k1) w_L2^(n2 k2) sum_n1 x[L2 n1 + n2] w_L1^(n1 k1),
// w_M = exp(s 2 pi i / M).  Step 1: every thread owns one (line, n2), loads
// its L1 inputs straight from global memory into registers, does the L1-point
// DFT in registers and applies the twiddle w_L^(n2 k1).  The tile is exchanged
// once through LDS.  Step 2: every thread owns one (line, k1), does the
// L2-point DFT in registers and stores straight to global memory.  Each
// element crosses LDS once (one write, one read) and the stage structure is
// fully unrolled at compile time.
//
// The in-register DFTs are mixed-radix (4, 2, 5, 3) decimation-in-time
// recursions whose twiddles are compile-time constants, computed below from
// the Taylor series of sin and cos in double precision.
#pragma once

#include <type_traits>

#include "passes.h"

namespace isg {

// ---------------------------------------------------------------------------
// compile-time cos / sin of 2 pi j / M
// ---------------------------------------------------------------------------
constexpr double kCePi = 3.14159265358979323846264338327950288;

constexpr double ce_sin_series(double x) {  // |x| <= pi/4
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}

constexpr double ce_cos_series(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

// returns cos (which = 0) or sin (which = 1) of 2 pi j / M, reducing the
// angle to [0, pi/4] with exact integer comparisons on j / M
constexpr double ce_trig(long j, long M, int which) {
  j %= M;
  if (j < 0) j += M;
  double sgn_s = 1.0, sgn_c = 1.0;
  if (2 * j > M) {  // theta in (pi, 2 pi): use 2 pi - theta
    j = M - j;
    sgn_s = -1.0;
  }
  bool swap = false;
  long num = j, den = M;  // theta = 2 pi num / den in [0, pi]
  if (4 * num > den) {    // theta in (pi/2, pi]: use pi - theta
    num = den - 2 * num;  // theta' = pi - theta = 2 pi (den/2 - num)/den = pi (den - 2 num)/den
    den = 2 * den;        // keep theta' = 2 pi num / den
    sgn_c = -1.0;
  }
  if (8 * num > den) {  // theta in (pi/4, pi/2]: use pi/2 - theta
    num = den - 4 * num;
    den = 4 * den;
    swap = true;
  }
  const double x = 2.0 * kCePi * (double)num / (double)den;
  double c = ce_cos_series(x), s = ce_sin_series(x);
  if (swap) {
    const double t = c;
    c = s;
    s = t;
  }
  return which == 0 ? sgn_c * c : sgn_s * s;
}

template <int M>
struct TwTable {
  float c[M];
  float s[M];
  constexpr TwTable() : c(), s() {
    for (int j = 0; j < M; ++j) {
      c[j] = (float)ce_trig(j, M, 0);
      s[j] = (float)ce_trig(j, M, 1);
    }
  }
};

template <int M>
__device__ __forceinline__ float2 twiddle_ce(int jk, float sgn) {
  constexpr TwTable<M> t{};
  const int j = jk % M;
  return make_float2(t.c[j], sgn * t.s[j]);
}

constexpr int first_radix(int M) {
  return M % 4 == 0 ? 4 : M % 2 == 0 ? 2 : M % 5 == 0 ? 5 : M % 3 == 0 ? 3 : M;
}

// in-register DFT of compile-time length M with exponent sign S (-1 / +1)
template <int M, int S>
__device__ __forceinline__ void reg_dft(float2* v) {
  if constexpr (M == 1) {
    return;
  } else if constexpr (M == 2 || M == 3 || M == 4 || M == 5) {
    dft<M>(v, (float)S);
  } else {
    constexpr int R = first_radix(M);
    constexpr int Q = M / R;
    float2 sub[R][Q];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int q = 0; q < Q; ++q) sub[r][q] = v[R * q + r];
#pragma unroll
    for (int r = 0; r < R; ++r) reg_dft<Q, S>(sub[r]);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      float2 t[R];
      t[0] = sub[0][k];
#pragma unroll
      for (int r = 1; r < R; ++r) t[r] = cmul(sub[r][k], twiddle_ce<M>(r * k, (float)S));
      dft<R>(t, (float)S);
#pragma unroll
      for (int m = 0; m < R; ++m) v[k + Q * m] = t[m];
    }
  }
}

// ---------------------------------------------------------------------------
// tile geometry and thread mappings
// ---------------------------------------------------------------------------
enum Map2 { kBFast = 0, kJFast = 1 };  // which index varies fastest across lanes

struct Tile2 {
  int64_t A, B;     // outer count, inner extent
  int na, nb;       // lines per tile: na outer x nb inner
  int64_t tiles_b;  // ceil(B / nb)
  int LS;           // LDS line stride (floats)
  int64_t tiles;    // > 0: total tiles, launched as 8 ceil(tiles / 8) workgroups in XCD-contiguous
                    // order; 0: plain order (host: < 0 requests XCD order)
};

template <int MAP>
__device__ __forceinline__ void decode(int t, int nb, int span, int& bl, int& idx, int& al) {
  // span = L2 (step 1) or L1 (step 2)
  if (MAP == kBFast) {
    bl = t % nb;
    const int r = t / nb;
    idx = r % span;
    al = r / span;
  } else {
    idx = t % span;
    const int r = t / span;
    bl = r % nb;
    al = r / nb;
  }
}

// LDS slot of element (k1, n2) of a line: rows of L2 + 1 to spread banks
template <int L1, int L2>
__device__ __forceinline__ int slot(int k1, int n2) {
  return k1 * (L2 + 1) + n2;
}

// The kernel.  Ld / St: per-thread line setup, then the element loads
// (stores) of the thread.  Step 1 thread (al, bl, n2) of the tile at (a0, b0)
// loads positions L2 n1 + n2, n1 = 0..L1-1; step 2 thread (al, bl, k1) stores
// positions k1 + L1 k2, k2 = 0..L2-1.  Loaders and stores see the tile origin
// and the thread's place in it separately, so that the part of an address
// shared by the tile (and by an element index) can stay in scalar registers.
// St may request an LDS epilogue (coil reduction) through St::kEpilogue: it
// then sees the lines in natural order twice, real parts, then imaginary
// parts (epilogue_part, accumulating up to St::kMaxPerThread outputs per
// thread), and stores (epilogue_store); Ld
// may fill a table in LDS before any load through Ld::kPrologue (its size:
// lds_extra(ld) on the host).
// GAP bit 0: the loads zero-pad L/2 stored values, so positions [L/4, 3L/4)
// are zero; bit 1: the stores crop to L/2 values, so those positions are not
// stored.  With L1 (L2) a multiple of 4 the gap is the same step-1 inputs
// n1 in [L1/4, 3L1/4) (step-2 outputs k2 in [L2/4, 3L2/4)) for every thread:
// those loads are not issued, and the outputs that are never stored are not
// computed (dead code).
// Loaders and stores of the axis-0 passes know which tiles no sample reaches
// (T::kTileSkip, T::tile_active(b0, g)); other types take every tile.
template <class T, class = void>
struct tile_skip : std::false_type {};
template <class T>
struct tile_skip<T, std::void_t<decltype(T::kTileSkip)>> : std::bool_constant<T::kTileSkip> {};
// A store may read per-line data before the loads (T::Early, T::early(),
// then T::setup(early, ...)), so that its latency overlaps theirs.
struct NoEarly {};
template <class T, class = void>
struct EarlyOf {
  using type = NoEarly;
  static constexpr bool value = false;
};
template <class T>
struct EarlyOf<T, std::void_t<typename T::Early>> {
  using type = typename T::Early;
  static constexpr bool value = true;
};

template <int L1, int L2, int S, int MAP1, int MAP2, class Ld, class St, int GAP = 0>
__global__ __launch_bounds__(1024) void fft2_kernel(Ld ld, St st, Tile2 g) {
  constexpr int L = L1 * L2;
  constexpr bool kGapIn = (GAP & 1) && L1 % 4 == 0;
  constexpr bool kGapOut = (GAP & 2) && L2 % 4 == 0;
  // The lines go through LDS as real parts, then imaginary parts, in one
  // float buffer (as does the epilogue's input): half the LDS per line, so
  // twice the workgroups fit a CU, for two more barriers per tile.
  extern __shared__ float2 smem[];
  float2* tw = smem;  // exp(-2 pi i q / L)
  float* linesf = reinterpret_cast<float*>(smem + L);
  const int tid = threadIdx.x;
  const int nthreads = blockDim.x;

  int64_t tile = (int64_t)blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
  if (g.tiles > 0) {
    // consecutive workgroup indices go to the 8 XCDs in turn; give each XCD
    // one contiguous range of tiles so that its L2 and translation caches
    // see neighbouring columns of the same rows
    const int64_t per = (g.tiles + 7) >> 3;
    tile = (tile & 7) * per + (tile >> 3);
    if (tile >= g.tiles) return;
  }
  const int64_t ta = tile / g.tiles_b;
  const int64_t a0 = ta * g.na;
  const int64_t b0 = (tile - ta * g.tiles_b) * g.nb;
  if (a0 >= g.A) return;
  const int nl = g.na * g.nb;
  if constexpr (tile_skip<Ld>::value || tile_skip<St>::value) {
    // a tile of lines whose grid columns no sample reaches: the forward pass
    // stores nothing there; the adjoint pass reads only zeros and stores zeros
    bool active = true;
    if constexpr (tile_skip<Ld>::value) active = ld.tile_active(b0, g);
    if constexpr (tile_skip<St>::value) active = active && st.tile_active(b0, g);
    if (!active) {
      if constexpr (!tile_skip<St>::value && !St::kEpilogue) {
        if (st.zfill && tid < nl * L1) {  // zfill false: the next pass reads these columns as zero
          int bz, kz, az;
          decode<MAP2>(tid, g.nb, L1, bz, kz, az);
          auto line = st.setup(a0, b0, az, bz, kz, a0 + az < g.A && b0 + bz < g.B);
#pragma unroll
          for (int k2 = 0; k2 < L2; ++k2)
            if (!(kGapOut && k2 >= L2 / 4 && k2 < 3 * L2 / 4))
              st.template put<L1, L2>(line, k2, make_float2(0.f, 0.f));
        }
      }
      return;
    }
  }
  uint32_t* table = reinterpret_cast<uint32_t*>(linesf + (size_t)nl * g.LS);
  if constexpr (Ld::kPrologue) ld.prologue(table, a0, b0, g);
  for (int i = tid; i < L; i += nthreads) tw[i] = ld.tw[i];
  if constexpr (Ld::kPrologue) __syncthreads();  // the loader's table

  // ---- step 1: loads and the L1-point DFTs overlap the twiddle copy ----
  const bool act1 = tid < nl * L2;
  [[maybe_unused]] typename EarlyOf<St>::type pre{};
  if constexpr (EarlyOf<St>::value) {
    if (tid < nl * L1) {
      int be, ke, ae;
      decode<MAP2>(tid, g.nb, L1, be, ke, ae);
      pre = st.early(a0, b0, ae, be, ke, a0 + ae < g.A && b0 + be < g.B);
    }
  }
  int bl = 0, n2 = 0, al = 0;
  float2 v[L1];
  if (act1) {
    decode<MAP1>(tid, g.nb, L2, bl, n2, al);
    const bool valid = a0 + al < g.A && b0 + bl < g.B;
    auto line = ld.setup(a0, b0, al, bl, n2, valid, table);
#pragma unroll
    for (int n1 = 0; n1 < L1; ++n1)
      v[n1] = (kGapIn && n1 >= L1 / 4 && n1 < 3 * L1 / 4) ? make_float2(0.f, 0.f)
                                                          : ld.template get<L1, L2>(line, n1);
    reg_dft<L1, S>(v);
  }
  __syncthreads();  // twiddle table in LDS
  const bool act2 = tid < nl * L1;
  int bl2 = 0, k1 = 0, al2 = 0;
  float2 u[L2];
  if (act2) decode<MAP2>(tid, g.nb, L1, bl2, k1, al2);
  if (act1) {
#pragma unroll
    for (int j = 1; j < L1; ++j) {
      float2 w = tw[n2 * j];  // n2 j <= (L2 - 1)(L1 - 1) < L
      w.y *= -(float)S;       // conjugate the table entry for the inverse sign
      v[j] = cmul(v[j], w);
    }
    float* dst = linesf + (al * g.nb + bl) * g.LS;
#pragma unroll
    for (int j = 0; j < L1; ++j) dst[slot<L1, L2>(j, n2)] = v[j].x;
  }
  __syncthreads();
  const float* src = linesf + (al2 * g.nb + bl2) * g.LS;
  if (act2) {
#pragma unroll
    for (int m = 0; m < L2; ++m) u[m].x = src[slot<L1, L2>(k1, m)];
  }
  __syncthreads();
  if (act1) {
    float* dst = linesf + (al * g.nb + bl) * g.LS;
#pragma unroll
    for (int j = 0; j < L1; ++j) dst[slot<L1, L2>(j, n2)] = v[j].y;
  }
  __syncthreads();
  if (act2) {
#pragma unroll
    for (int m = 0; m < L2; ++m) u[m].y = src[slot<L1, L2>(k1, m)];
    reg_dft<L2, S>(u);
  }

  if constexpr (St::kEpilogue) {
    // results go back to LDS in natural order for a cross-line epilogue,
    // real parts, then imaginary parts
    float2 acc[St::kMaxPerThread];
#pragma unroll
    for (int i = 0; i < St::kMaxPerThread; ++i) acc[i] = make_float2(0.f, 0.f);
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      __syncthreads();  // the previous reads of the buffer are done
      if (act2) {
        float* dstl = linesf + (al2 * g.nb + bl2) * g.LS;
#pragma unroll
        for (int k2 = 0; k2 < L2; ++k2)
          if (!(kGapOut && k2 >= L2 / 4 && k2 < 3 * L2 / 4)) dstl[k1 + L1 * k2] = part ? u[k2].y : u[k2].x;
      }
      __syncthreads();
      st.epilogue_part(linesf, g, a0, part, acc);
    }
    st.epilogue_store(g, a0, acc);
  } else {
    if (act2) {
      const bool valid = a0 + al2 < g.A && b0 + bl2 < g.B;
      auto line = [&] {
        if constexpr (EarlyOf<St>::value)
          return st.setup(pre, a0, b0, al2, bl2, k1, valid);
        else
          return st.setup(a0, b0, al2, bl2, k1, valid);
      }();
#pragma unroll
      for (int k2 = 0; k2 < L2; ++k2)
        if (!(kGapOut && k2 >= L2 / 4 && k2 < 3 * L2 / 4)) st.template put<L1, L2>(line, k2, u[k2]);
    }
  }
}

// ---------------------------------------------------------------------------
// element maps of a line of length L holding n = L/2 stored values
// ---------------------------------------------------------------------------
// stored index of position p, or -1 in the zero gap
template <int L>
__device__ __forceinline__ int pad_src(int map, int p) {
  constexpr int n = L / 2;
  if (map == kCentred) return p < n / 2 ? p + n / 2 : (p >= L - n / 2 ? p - (L - n / 2) : -1);
  if (map == kSpectral) return p < n / 2 ? p : (p >= L - n / 2 ? p - (L - n) : -1);
  return p;
}

// Outside the gap the stored index is the position plus a constant of the
// range: +L/4 (centred) or 0 (spectral) below the gap, -3L/4 (centred) or
// -L/2 (spectral) above it, 0 for the dense map.
template <int L>
__device__ __forceinline__ int gap_shift(int map, bool upper) {
  if (map == kCentred) return upper ? -(3 * L / 4) : L / 4;
  if (map == kSpectral) return upper ? -(L / 2) : 0;
  return 0;
}

// Load of one element that reads as zero when `on` is false.  The load is
// issued either way (from `dummy`, any valid address, when off) and the
// result selected afterwards: a skipped load would sit in a branch of its
// own, and the compiler then waits for every earlier load at each branch
// join, so the loads of a line would be issued one at a time.
template <int S>
__device__ __forceinline__ float2 masked_load(const typename Elem<S>::T* addr, bool on, const float2* dummy) {
  const float2 v = Elem<S>::load(on ? addr : reinterpret_cast<const typename Elem<S>::T*>(dummy));
  return on ? v : make_float2(0.f, 0.f);
}

// ---------------------------------------------------------------------------
// buffer-addressed access.  A raw buffer resource (stride 0) over 2^31 bytes
// from a base held in scalar registers; the lane supplies a 32-bit byte
// offset.  Offsets at or above 2^31 are out of range: such a load returns
// zero and such a store is dropped, which is how untouched or invalid
// elements are masked without a branch or a select of the data.
// ---------------------------------------------------------------------------
constexpr uint32_t kOOB = 0x80000000u;
typedef int isg_v2i __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base) {
  // dword 3 of a gfx9 raw buffer: 32-bit data format, no swizzle
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)kOOB, 0x00020000);
}

template <int S>
__device__ __forceinline__ float2 buf_load(const void* base, uint32_t off) {
  if constexpr (S == kFP32) {
    const isg_v2i r = __builtin_amdgcn_raw_buffer_load_b64(buf_rsrc(base), off, 0, 0);
    return __builtin_bit_cast(float2, r);
  } else {
    const int r = __builtin_amdgcn_raw_buffer_load_b32(buf_rsrc(base), off, 0, 0);
    typename Elem<S>::T h;
    __builtin_memcpy(&h, &r, sizeof(r));
    return Elem<S>::load(&h);
  }
}

template <int S>
__device__ __forceinline__ void buf_store(void* base, uint32_t off, float2 v) {
  if constexpr (S == kFP32) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(isg_v2i, v), buf_rsrc(base), off, 0, 0);
  } else {
    typename Elem<S>::T h;
    Elem<S>::store(&h, v);
    int r;
    __builtin_memcpy(&r, &h, sizeof(r));
    __builtin_amdgcn_raw_buffer_store_b32(r, buf_rsrc(base), off, 0, 0);
  }
}

// ---------------------------------------------------------------------------
// general loaders and stores: every address computed per lane and element
// (any length, map and layout)
// ---------------------------------------------------------------------------
// strided load of element p of line (a, b): p[a*sa + j*sj + b]; map: dense,
// or zero-pad of L/2 stored values (centred or spectral)
template <int S>
struct Ld2Strided {
  static constexpr bool kPrologue = false;
  const typename Elem<S>::T* p;
  int64_t sa, sj;
  int tlog;     // stored position j sits at (j >> tlog) bs + (j & (2^tlog - 1)) sj
  int64_t bs;   // (tlog = 30: j sj, the plain stride)
  int map;
  const float2* tw;
  struct Line {
    const typename Elem<S>::T* base;
    int n2;
    bool valid;
  };
  __device__ Line setup(int64_t a0, int64_t b0, int al, int bl, int n2, bool valid, const uint32_t*) const {
    return Line{p + (a0 + al) * sa + b0 + bl, n2, valid};
  }
  template <int L1, int L2>
  __device__ float2 get(const Line& ln, int n1) const {
    const int j = pad_src<L1 * L2>(map, L2 * n1 + ln.n2);
    return masked_load<S>(ln.base + (int64_t)(j >> tlog) * bs + (int64_t)(j & ((1 << tlog) - 1)) * sj,
                          ln.valid && j >= 0, tw);
  }
};

// load along axis 0 of a row-blocked array: column b, stored rows j
template <int S>
struct Ld2Rows {
  static constexpr bool kPrologue = false;
  const typename Elem<S>::T* p;
  Blk blk;
  int map;
  const float2* tw;
  struct Line {
    const typename Elem<S>::T* base;
    int n2;
    bool valid;
  };
  __device__ Line setup(int64_t, int64_t b0, int, int bl, int n2, bool valid, const uint32_t*) const {
    return Line{valid ? p + blk.col(b0 + bl) : p, n2, valid};
  }
  template <int L1, int L2>
  __device__ float2 get(const Line& ln, int n1) const {
    const int j = pad_src<L1 * L2>(map, L2 * n1 + ln.n2);
    return masked_load<S>(ln.base + (int64_t)j * blk.rs, ln.valid && j >= 0, tw);
  }
};

template <int S>
struct St2Strided {
  static constexpr bool kEpilogue = false;
  bool zfill = true;  // a skipped (untouched) tile of the adjoint axis-0 pass stores zeros
  typename Elem<S>::T* p;
  int64_t sa, sj;
  int tlog;     // as in Ld2Strided
  int64_t bs;
  int map;      // dense, or crop to L/2 values (centred or spectral)
  float scale;  // applied to half-precision stores only
  struct Line {
    typename Elem<S>::T* base;
    int k1;
    bool valid;
  };
  __device__ Line setup(int64_t a0, int64_t b0, int al, int bl, int k1, bool valid) const {
    return Line{p + (a0 + al) * sa + b0 + bl, k1, valid};
  }
  template <int L1, int L2>
  __device__ void put(const Line& ln, int k2, float2 v) const {
    const int j = pad_src<L1 * L2>(map, ln.k1 + L1 * k2);
    if (ln.valid && j >= 0)
      Elem<S>::store(ln.base + (int64_t)(j >> tlog) * bs + (int64_t)(j & ((1 << tlog) - 1)) * sj,
                     store_scaled<S>(v, scale));
  }
};

// store along axis 0 of a row-blocked array (crop maps as St2Strided)
template <int S>
struct St2Rows {
  static constexpr bool kEpilogue = false;
  bool zfill = true;  // a skipped (untouched) tile of the adjoint axis-0 pass stores zeros
  typename Elem<S>::T* p;
  Blk blk;
  int map;
  float scale;  // applied to half-precision stores only
  struct Line {
    typename Elem<S>::T* base;
    int k1;
    bool valid;
  };
  __device__ Line setup(int64_t, int64_t b0, int, int bl, int k1, bool valid) const {
    return Line{valid ? p + blk.col(b0 + bl) : p, k1, valid};
  }
  template <int L1, int L2>
  __device__ void put(const Line& ln, int k2, float2 v) const {
    const int j = pad_src<L1 * L2>(map, ln.k1 + L1 * k2);
    if (ln.valid && j >= 0) Elem<S>::store(ln.base + (int64_t)j * blk.rs, store_scaled<S>(v, scale));
  }
};

// Whether a loader zero-pads (a store crops) L/2 stored values of every line,
// i.e. positions [L/4, 3L/4) are zero (not stored): checked on the host
// before a kernel is launched with the corresponding GAP bit.
template <class T>
inline bool half_gap(const T&, int) { return false; }
template <int S>
inline bool half_gap(const Ld2Strided<S>& x, int) { return x.map == kCentred || x.map == kSpectral; }
template <int S>
inline bool half_gap(const Ld2Rows<S>& x, int) { return x.map == kCentred || x.map == kSpectral; }
template <int S>
inline bool half_gap(const St2Strided<S>& x, int) { return x.map == kCentred || x.map == kSpectral; }
template <int S>
inline bool half_gap(const St2Rows<S>& x, int) { return x.map == kCentred || x.map == kSpectral; }

// The strided load and store of the single-image upsampling passes: the same
// code as Ld2Strided / St2Strided under types of their own, so that kernel
// names (and profiles) tell those passes from the coil passes of equal length.
template <int S>
struct Ld2Image : Ld2Strided<S> {};
template <int S>
struct St2Image : St2Strided<S> {};
template <int S>
inline bool half_gap(const Ld2Image<S>& x, int L) { return half_gap(static_cast<const Ld2Strided<S>&>(x), L); }
template <int S>
inline bool half_gap(const St2Image<S>& x, int L) { return half_gap(static_cast<const St2Strided<S>&>(x), L); }

// Touched-cell masks of a trajectory, read by the axis-0 passes.  Along
// axis 0 the grid is cut into runs of 2^ts0_log2 cells (the k-space spread
// tile extent along axis 0).  fmask[(i1, i2)] (i1 alone in 2D) has bit t set
// when some sample's taps reach a cell of run t of that column: the gather
// reads no other cell and the spread leaves every other cell zero, so the
// forward axis-0 pass stores only the marked runs and the adjoint one reads
// only those.  (A coarser per-tile-column mask, colmask, locates the tiles
// of the tile-major spread output.)
struct TileMask {
  const uint64_t* fmask;  // null: every run is touched
  int C, G2, three_d, ts0_log2;
  __device__ __forceinline__ uint64_t column(int64_t b) const {
    if (!fmask) return ~0ull;
    const uint32_t q = (uint32_t)b / (uint32_t)C;  // i1 G2 + i2 in 3D, i1 in 2D (< 2^31)
    return fmask[q];
  }
  // some sample reaches a grid column of the tile's columns b0 .. b0+nb-1
  __device__ __forceinline__ bool tile_active(int64_t b0, const Tile2& g) const {
    if (!fmask) return true;
    const int64_t b1 = (b0 + g.nb < g.B ? b0 + g.nb : g.B) - 1;
    uint64_t any = 0;
    for (uint32_t q = (uint32_t)b0 / (uint32_t)C; q <= (uint32_t)b1 / (uint32_t)C; ++q) any |= fmask[q];
    return any != 0ull;
  }
};

// axis-0 load that reads untouched tiles as zero (dense map)
template <int S>
struct Ld2Masked {
  static constexpr bool kPrologue = false;
  static constexpr bool kTileSkip = true;
  __device__ bool tile_active(int64_t b0, const Tile2& g) const { return tm.tile_active(b0, g); }
  const typename Elem<S>::T* p;
  Blk blk;  // the grid's row-blocked layout
  TileMask tm;
  const float2* tw;
  struct Line {
    const typename Elem<S>::T* base;
    uint64_t mask;
    int n2;
    bool valid;
  };
  __device__ Line setup(int64_t, int64_t b0, int, int bl, int n2, bool valid, const uint32_t*) const {
    const int64_t b = b0 + bl;
    return Line{valid ? p + blk.col(b) : p, valid ? tm.column(b) : 0ull, n2, valid};
  }
  template <int L1, int L2>
  __device__ float2 get(const Line& ln, int n1) const {
    const int pos = L2 * n1 + ln.n2;
    const bool on = ln.valid && ((ln.mask >> (pos >> tm.ts0_log2)) & 1ull);
    return masked_load<S>(ln.base + (int64_t)pos * blk.rs, on, tw);
  }
};

// axis-0 store that skips untouched tiles (dense map)
template <int S>
struct St2Masked {
  static constexpr bool kEpilogue = false;
  static constexpr bool kTileSkip = true;
  __device__ bool tile_active(int64_t b0, const Tile2& g) const { return tm.tile_active(b0, g); }
  typename Elem<S>::T* p;
  Blk blk;  // the grid's row-blocked layout
  TileMask tm;
  float scale;  // applied to half-precision stores only
  struct Line {
    typename Elem<S>::T* base;
    uint64_t mask;
    int k1;
    bool valid;
  };
  __device__ Line setup(int64_t, int64_t b0, int, int bl, int k1, bool valid) const {
    const int64_t b = b0 + bl;
    return Line{valid ? p + blk.col(b) : p, valid ? tm.column(b) : 0ull, k1, valid};
  }
  template <int L1, int L2>
  __device__ void put(const Line& ln, int k2, float2 v) const {
    const int pos = ln.k1 + L1 * k2;
    if (ln.valid && ((ln.mask >> (pos >> tm.ts0_log2)) & 1ull))
      Elem<S>::store(ln.base + (int64_t)pos * blk.rs, store_scaled<S>(v, scale));
  }
};

// axis-0 load of a tile-major spread output (3D): the touched tiles of each
// tile column are stored one after another from colbase[col]; the k-th
// touched tile of the column (k = touched tiles below it) holds rows t0 of
// that column.  Untouched tiles read as zero.
template <int S>
struct Ld2Tiles {
  static constexpr bool kPrologue = false;
  static constexpr bool kTileSkip = true;
  const typename Elem<S>::T* p;
  const uint64_t* colmask;  // per tile column: touched tiles (their slots)
  const uint64_t* fmask;    // per grid column (i1, i2): touched runs along axis 0
  const int* colbase;
  int C, G2, ts0_log2, ts1, ts2, nt2;
  int64_t volC;   // elements per tile
  int64_t rowC;   // elements per tile row of axis 0 (TS1 TS2 C)
  FastDiv cdiv, g2div;
  const float2* tw;
  __device__ bool tile_active(int64_t b0, const Tile2& g) const {
    const TileMask tm{fmask, C, G2, 1, ts0_log2};
    return tm.tile_active(b0, g);
  }
  struct Line {
    const typename Elem<S>::T* base;
    uint64_t mask;  // touched tiles of the tile column
    uint64_t fine;  // touched runs of the grid column
    int n2;
    bool valid;
  };
  __device__ Line setup(int64_t, int64_t b0, int, int bl, int n2, bool valid, const uint32_t*) const {
    if (!valid) return Line{p, 0ull, 0ull, n2, false};
    const int64_t b = b0 + bl;
    const uint32_t q = cdiv.div((uint32_t)b);
    const int c = (int)(b - (int64_t)q * C);
    const uint32_t i1 = g2div.div(q);
    const int i2 = (int)(q - i1 * (uint32_t)G2);
    const int col = (int)(i1 / (uint32_t)ts1) * nt2 + i2 / ts2;
    const int l1 = (int)(i1 % (uint32_t)ts1), l2 = i2 % ts2;
    return Line{p + (int64_t)colbase[col] * volC + (int64_t)(l1 * ts2 + l2) * C + c, colmask[col], fmask[q], n2,
                true};
  }
  template <int L1, int L2>
  __device__ float2 get(const Line& ln, int n1) const {
    const int pos = L2 * n1 + ln.n2;
    const int t0 = pos >> ts0_log2;
    const bool on = ln.valid && ((ln.fine >> t0) & 1ull);
    const int k = __popcll(ln.mask & ((1ull << t0) - 1ull));
    return masked_load<S>(ln.base + (int64_t)k * volC + (int64_t)(pos & ((1 << ts0_log2) - 1)) * rowC, on, tw);
  }
};

// ---------------------------------------------------------------------------
// buffer-addressed loaders and stores of the coil and upsampling passes.
// The tile origin's part of every address is a scalar base, each element
// index adds a scalar offset, and the lane keeps one 32-bit byte offset for
// the whole line, so an element costs no vector address arithmetic.  Valid
// only where the host has checked: both lengths L1, L2 multiples of 4 (the
// gap ranges of the maps are then whole element indices), a row-blocked
// stride's block T dividing the element-index step (L2 for loads, L1 for
// stores) and L/4, and every lane offset below 2^31 bytes.
// ---------------------------------------------------------------------------
template <int S>
struct Ld2StridedF {
  static constexpr bool kPrologue = false;
  const typename Elem<S>::T* p;
  int64_t sa, sj;
  int tlog;  // as in Ld2Strided (30: plain stride)
  int64_t bs;
  int map;
  const float2* tw;
  struct Line {
    const typename Elem<S>::T* base;
    uint32_t off;
  };
  __device__ Line setup(int64_t a0, int64_t b0, int al, int bl, int n2, bool valid, const uint32_t*) const {
    const int64_t row = tlog >= 30 ? (int64_t)n2 * sj
                                   : (int64_t)(n2 >> tlog) * bs + (int64_t)(n2 & ((1 << tlog) - 1)) * sj;
    const int64_t e = (int64_t)al * sa + bl + row;
    return Line{p + a0 * sa + b0, valid ? (uint32_t)(e * (int64_t)sizeof(typename Elem<S>::T)) : kOOB};
  }
  template <int L1, int L2>
  __device__ float2 get(const Line& ln, int n1) const {
    const int j = L2 * n1 + gap_shift<L1 * L2>(map, n1 >= 3 * L1 / 4);  // element index's stored row
    const int64_t r = tlog >= 30 ? (int64_t)j * sj : (int64_t)(j >> tlog) * bs;
    return buf_load<S>(ln.base + r, ln.off);
  }
};

template <int S>
struct St2StridedF {
  static constexpr bool kEpilogue = false;
  bool zfill = true;  // a skipped (untouched) tile of the adjoint axis-0 pass stores zeros
  typename Elem<S>::T* p;
  int64_t sa, sj;
  int tlog;
  int64_t bs;
  int map;
  float scale;  // applied to half-precision stores only
  struct Line {
    typename Elem<S>::T* base;
    uint32_t off;
  };
  __device__ Line setup(int64_t a0, int64_t b0, int al, int bl, int k1, bool valid) const {
    const int64_t row = tlog >= 30 ? (int64_t)k1 * sj
                                   : (int64_t)(k1 >> tlog) * bs + (int64_t)(k1 & ((1 << tlog) - 1)) * sj;
    const int64_t e = (int64_t)al * sa + bl + row;
    return Line{p + a0 * sa + b0, valid ? (uint32_t)(e * (int64_t)sizeof(typename Elem<S>::T)) : kOOB};
  }
  template <int L1, int L2>
  __device__ void put(const Line& ln, int k2, float2 v) const {
    const int j = L1 * k2 + gap_shift<L1 * L2>(map, k2 >= 3 * L2 / 4);
    const int64_t r = tlog >= 30 ? (int64_t)j * sj : (int64_t)(j >> tlog) * bs;
    buf_store<S>(ln.base + r, ln.off, store_scaled<S>(v, scale));
  }
};

// axis 0 of a row-blocked array; the tile's nb columns must be contiguous
template <int S>
struct Ld2RowsF {
  static constexpr bool kPrologue = false;
  const typename Elem<S>::T* p;
  Blk blk;
  int map;
  const float2* tw;
  struct Line {
    const typename Elem<S>::T* base;
    uint32_t off;
  };
  __device__ Line setup(int64_t, int64_t b0, int, int bl, int n2, bool valid, const uint32_t*) const {
    const int64_t e = bl + (int64_t)n2 * blk.rs;
    return Line{p + blk.col(b0), valid ? (uint32_t)(e * (int64_t)sizeof(typename Elem<S>::T)) : kOOB};
  }
  template <int L1, int L2>
  __device__ float2 get(const Line& ln, int n1) const {
    const int j = L2 * n1 + gap_shift<L1 * L2>(map, n1 >= 3 * L1 / 4);
    return buf_load<S>(ln.base + (int64_t)j * blk.rs, ln.off);
  }
};

template <int S>
struct St2RowsF {
  static constexpr bool kEpilogue = false;
  bool zfill = true;  // a skipped (untouched) tile of the adjoint axis-0 pass stores zeros
  typename Elem<S>::T* p;
  Blk blk;
  int map;
  float scale;
  struct Line {
    typename Elem<S>::T* base;
    uint32_t off;
  };
  __device__ Line setup(int64_t, int64_t b0, int, int bl, int k1, bool valid) const {
    const int64_t e = bl + (int64_t)k1 * blk.rs;
    return Line{p + blk.col(b0), valid ? (uint32_t)(e * (int64_t)sizeof(typename Elem<S>::T)) : kOOB};
  }
  template <int L1, int L2>
  __device__ void put(const Line& ln, int k2, float2 v) const {
    const int j = L1 * k2 + gap_shift<L1 * L2>(map, k2 >= 3 * L2 / 4);
    buf_store<S>(ln.base + (int64_t)j * blk.rs, ln.off, store_scaled<S>(v, scale));
  }
};

// axis-0 store of the touched runs only (dense map), runs of 8 cells and L1 a
// multiple of 8: position k1 + L1 k2 lies in run (k1 >> 3) + (L1 / 8) k2, so
// the lane shifts its column's run mask once by k1 >> 3 and each element
// tests a bit known at compile time
template <int S>
struct St2MaskedF {
  static constexpr bool kEpilogue = false;
  static constexpr bool kTileSkip = true;
  __device__ bool tile_active(int64_t b0, const Tile2& g) const { return tm.tile_active(b0, g); }
  typename Elem<S>::T* p;
  Blk blk;
  TileMask tm;
  float scale;
  struct Line {
    typename Elem<S>::T* base;
    uint32_t off;
    uint64_t mask;
  };
  __device__ Line setup(int64_t, int64_t b0, int, int bl, int k1, bool valid) const {
    const int64_t e = bl + (int64_t)k1 * blk.rs;
    const uint64_t m = valid ? tm.column(b0 + bl) >> (k1 >> 3) : 0ull;
    return Line{p + blk.col(b0), (uint32_t)(e * (int64_t)sizeof(typename Elem<S>::T)), m};
  }
  template <int L1, int L2>
  __device__ void put(const Line& ln, int k2, float2 v) const {
    const bool on = (ln.mask >> ((L1 / 8) * k2)) & 1ull;
    buf_store<S>(ln.base + (int64_t)(L1 * k2) * blk.rs, on ? ln.off : kOOB, store_scaled<S>(v, scale));
  }
};

// Axis-0 load of the tile-major spread output through a table in LDS.  The
// tile's nb columns b0 .. b0+nb-1 belong to at most ngp consecutive grid
// columns q = b / C.  Before any load the workgroup writes, for each of those
// grid columns and each run t0 of 8 cells along axis 0, the byte offset of
// the run's first cell (coil 0), or kOOB for a run no sample reaches (and for
// grid columns past the end).  Offsets are taken from the first touched tile
// of the first tile column in the tile row of q0 = b0 / C: the tile columns
// are numbered row by row and their slots follow that order, so every grid
// column of the tile (in that tile row or the next) lies at or after it.  An
// element at position pos of a lane's line then costs one LDS read (entry
// (q - q0, pos >> 3)) and one add (the lane's coil and the cell within the
// run).  Offsets stay below 2^31 bytes (checked on the host).
template <int S>
struct Ld2TilesF {
  static constexpr bool kPrologue = true;
  static constexpr bool kTileSkip = true;
  const typename Elem<S>::T* p;
  const uint64_t* colmask;
  const uint64_t* fmask;
  const int* colbase;
  int C, G2, ts1, ts2, nt2;
  int nruns;   // runs along axis 0 (G0 / 8)
  int ngp;     // table rows per tile
  int64_t Q;   // grid columns (G1 G2)
  int64_t volC, rowC;
  const float2* tw;
  __device__ bool tile_active(int64_t b0, const Tile2& g) const {
    const TileMask tm{fmask, C, G2, 1, 3};
    return tm.tile_active(b0, g);
  }
  struct Line {
    const typename Elem<S>::T* base;
    const uint32_t* row;  // the lane's table row
    int n2;
    uint32_t coff;        // the lane's coil, bytes
  };
  // grid columns and tile columns are below 2^31 (checked on the host)
  // (uniform: read into a scalar register, so that the buffer descriptor
  // built from it stays scalar and each load is a single instruction)
  __device__ int64_t row_base(uint32_t q0) const {  // first tile slot of q0's tile row, elements
    const uint32_t i1 = q0 / (uint32_t)G2;
    return (int64_t)__builtin_amdgcn_readfirstlane(colbase[(i1 / (uint32_t)ts1) * nt2]) * volC;
  }
  __device__ void prologue(uint32_t* table, int64_t, int64_t b0, const Tile2&) const {
    const uint32_t q0 = (uint32_t)b0 / (uint32_t)C;
    const int64_t base = row_base(q0);
    for (int e = threadIdx.x; e < ngp * nruns; e += blockDim.x) {
      const int gp = e / nruns, t0 = e - gp * nruns;
      const uint32_t q = q0 + gp;
      uint32_t v = kOOB;
      if (q < (uint32_t)Q && ((fmask[q] >> t0) & 1ull)) {
        const uint32_t i1 = q / (uint32_t)G2, i2 = q - i1 * (uint32_t)G2;
        const uint32_t col = (i1 / (uint32_t)ts1) * nt2 + i2 / (uint32_t)ts2;
        const int k = __popcll(colmask[col] & ((1ull << t0) - 1ull));
        const int64_t el = (int64_t)(colbase[col] + k) * volC +
                           (int64_t)((i1 % (uint32_t)ts1) * ts2 + i2 % (uint32_t)ts2) * C - base;
        v = (uint32_t)(el * (int64_t)sizeof(typename Elem<S>::T));
      }
      table[e] = v;
    }
  }
  __device__ Line setup(int64_t, int64_t b0, int, int bl, int n2, bool, const uint32_t* table) const {
    const uint32_t q0 = (uint32_t)b0 / (uint32_t)C;
    const uint32_t b = (uint32_t)b0 + bl;
    const uint32_t q = b / (uint32_t)C;
    return Line{p + row_base(q0), table + (q - q0) * nruns, n2,
                (b - q * (uint32_t)C) * (uint32_t)sizeof(typename Elem<S>::T)};
  }
  template <int L1, int L2>
  __device__ float2 get(const Line& ln, int n1) const {
    const int lo = (L2 * n1) & 7, hi = (L2 * n1) >> 3;  // known at compile time
    const int s = lo + ln.n2;
    const uint32_t e = ln.row[hi + (s >> 3)];
    const uint32_t cell = (uint32_t)((s & 7) * rowC * (int64_t)sizeof(typename Elem<S>::T));
    return buf_load<S>(ln.base, e + cell + ln.coff);
  }
};

// The adjoint axis-1 pass of the coil-expanded arrays along a trajectory's
// touched grid columns: line (i0, b = i2 C + c) runs over i1, and grid column
// (i1, i2) holds data only if some sample reaches it (its run mask is not
// zero).  cm[i2][w] holds bit i1 of those columns (W = ceil(G1 / 64) words,
// G1 <= 512).  The lane shifts its column's bits right by its own part of the
// position (n2), so an element index tests one bit known at compile time; an
// untouched column reads as zero, so the adjoint axis-0 pass need not write
// the tiles no sample reaches.
constexpr int kColWords = 8;
template <int S>
struct Ld2StridedM : Ld2StridedF<S> {
  const uint64_t* cm;
  int cmC, cmW;
  struct Line {
    typename Ld2StridedF<S>::Line f;
    uint64_t m[kColWords];
  };
  __device__ Line setup(int64_t a0, int64_t b0, int al, int bl, int n2, bool valid, const uint32_t* t) const {
    Line ln;
    ln.f = Ld2StridedF<S>::setup(a0, b0, al, bl, n2, valid, t);
    const uint64_t* c = cm + (int64_t)((uint32_t)(b0 + bl) / (uint32_t)cmC) * cmW;
#pragma unroll
    for (int w = 0; w < kColWords; ++w) {
      const uint64_t lo = w < cmW && valid ? c[w] : 0ull;
      const uint64_t hi = w + 1 < cmW && valid ? c[w + 1] : 0ull;
      ln.m[w] = n2 == 0 ? lo : (lo >> n2) | (hi << (64 - n2));  // n2 < 64
    }
    return ln;
  }
  template <int L1, int L2>
  __device__ float2 get(const Line& ln, int n1) const {
    const int bit = L2 * n1;  // position L2 n1 + n2 after the lane's shift
    const bool on = (ln.m[bit >> 6] >> (bit & 63)) & 1ull;
    typename Ld2StridedF<S>::Line f = ln.f;
    f.off = on ? f.off : kOOB;
    return Ld2StridedF<S>::template get<L1, L2>(f, n1);
  }
};

// axis-1 store of the forward pass restricted to a trajectory's touched grid
// columns (cm as in Ld2StridedM): the axis-0 pass after it transforms only
// tiles of lines holding a touched column and stores only touched runs, so
// the other columns are never read into a result.  The column words are
// read before the loads (Early).
template <int S>
struct St2StridedMF : St2StridedF<S> {
  const uint64_t* cm;
  int cmC, cmW;
  struct Early {
    uint64_t m[kColWords];
  };
  struct Line {
    typename St2StridedF<S>::Line f;
    uint64_t m[kColWords];
  };
  __device__ Early early(int64_t, int64_t b0, int, int bl, int, bool valid) const {
    Early e;
    const uint64_t* c = cm + (int64_t)((uint32_t)(b0 + bl) / (uint32_t)cmC) * cmW;
#pragma unroll
    for (int w = 0; w < kColWords; ++w) e.m[w] = w < cmW && valid ? c[w] : 0ull;
    return e;
  }
  __device__ Line setup(const Early& e, int64_t a0, int64_t b0, int al, int bl, int k1, bool valid) const {
    Line ln;
    ln.f = St2StridedF<S>::setup(a0, b0, al, bl, k1, valid);
#pragma unroll
    for (int w = 0; w < kColWords; ++w) {
      const uint64_t lo = e.m[w], hi = w + 1 < kColWords ? e.m[w + 1] : 0ull;
      ln.m[w] = k1 == 0 ? lo : (lo >> k1) | (hi << (64 - k1));  // k1 < 64
    }
    return ln;
  }
  template <int L1, int L2>
  __device__ void put(const Line& ln, int k2, float2 v) const {
    const int bit = L1 * k2;  // position k1 + L1 k2 after the lane's shift (dense map)
    const bool on = (ln.m[bit >> 6] >> (bit & 63)) & 1ull;
    typename St2StridedF<S>::Line f = ln.f;
    f.off = on ? f.off : kOOB;
    St2StridedF<S>::template put<L1, L2>(f, k2, v);
  }
};

template <int S>
struct Ld2ImageF : Ld2StridedF<S> {};
template <int S>
struct St2ImageF : St2StridedF<S> {};

template <int S>
inline bool half_gap(const Ld2StridedF<S>& x, int) { return x.map == kCentred || x.map == kSpectral; }
template <int S>
inline bool half_gap(const St2StridedF<S>& x, int) { return x.map == kCentred || x.map == kSpectral; }
template <int S>
inline bool half_gap(const Ld2ImageF<S>& x, int L) { return half_gap(static_cast<const Ld2StridedF<S>&>(x), L); }
template <int S>
inline bool half_gap(const St2ImageF<S>& x, int L) { return half_gap(static_cast<const St2StridedF<S>&>(x), L); }
template <int S>
inline bool half_gap(const Ld2RowsF<S>& x, int) { return x.map == kCentred || x.map == kSpectral; }
template <int S>
inline bool half_gap(const Ld2StridedM<S>& x, int L) { return half_gap(static_cast<const Ld2StridedF<S>&>(x), L); }
template <int S>
inline bool half_gap(const St2RowsF<S>& x, int) { return x.map == kCentred || x.map == kSpectral; }

// LDS bytes a loader's prologue needs beyond the tile
template <class T>
inline size_t lds_extra(const T&) { return 0; }
template <int S>
inline size_t lds_extra(const Ld2TilesF<S>& x) { return sizeof(uint32_t) * (size_t)x.ngp * x.nruns; }

// first pass of inverse k-space gridding: S_c . m / c(x/G) |N|^{-1/2},
// zero-padded (centred) along the last axis; lines are (a, c)
struct Ld2CoilExpand {
  static constexpr bool kPrologue = false;
  const float2* m;
  const float2* S;
  AxisTabs dx;
  float scale;
  const float* dsc;  // half-precision grids: per-call input scale dsc[0] (device), else null
  int64_t N;
  int n;    // stored length (L/2)
  int n1;   // axis-1 extent in 3D, 0 in 2D
  const float2* tw;
  struct Line {
    const float2* mrow;
    const float2* srow;
    float f;
    int n2;
    bool valid;
  };
  __device__ Line setup(int64_t a0, int64_t b0, int al, int bl, int n2, bool valid, const uint32_t*) const {
    const int64_t a = a0 + al, c = b0 + bl;
    Line ln{m, S, 0.f, n2, valid};
    if (!valid) return ln;
    float f = dsc ? scale * dsc[0] : scale;
    if (n1) {
      const int i0 = (int)(a / n1), i1 = (int)(a - (int64_t)i0 * n1);
      f *= dx.t[0][i0] * dx.t[1][i1];
    } else {
      f *= dx.t[0][a];
    }
    ln.mrow = m + a * n;
    ln.srow = S + c * N + a * n;
    ln.f = f;
    return ln;
  }
  template <int L1, int L2>
  __device__ float2 get(const Line& ln, int e1) const {  // e1: the element index (n1 is the axis-1 extent)
    const int j = pad_src<L1 * L2>(kCentred, L2 * e1 + ln.n2);
    const bool on = ln.valid && j >= 0;
    const int jj = on ? j : 0;  // every line's element 0 exists: unconditional loads, no branch
    const float* dl = dx.t[n1 ? 2 : 1];
    const float2 v = cscale(cmul(ln.srow[jj], ln.mrow[jj]), ln.f * dl[jj]);
    return on ? v : make_float2(0.f, 0.f);
  }
};

// last pass of k-space gridding: crop (centred) along the last axis, times
// 1/c(x/G) |N|^{-1/2}, times conj(S_c), summed over the coils of the tile
struct St2CoilReduce {
  static constexpr bool kEpilogue = true;
  float2* out;
  const float2* S;
  AxisTabs dx;
  float scale;
  HalfUndo undo;         // half-precision grids: scales to undo (none for FP32)
  int64_t N;
  int n, L, C;
  int n1;
  struct Line {};
  // output elements per thread: total = na n = na L / 2 and the workgroup
  // has at least na C L2 threads, so at most L1 / (2 C) <= 8 (L1 <= 16)
  static constexpr int kMaxPerThread = 8;
  // part 0: lines hold the real parts u.x of the transformed lines, part 1
  // the imaginary parts u.y; conj(S) u = (S.x u.x + S.y u.y) + i (S.x u.y - S.y u.x)
  __device__ void epilogue_part(const float* lines, const Tile2& g, int64_t a0, int part,
                                float2 (&acc)[kMaxPerThread]) const {
    const int total = g.na * n;
#pragma unroll
    for (int i = 0; i < kMaxPerThread; ++i) {
      const int e = (int)threadIdx.x + i * (int)blockDim.x;
      if (e >= total) break;
      const int al = e / n;
      const int j = e - al * n;
      if (a0 + al >= g.A) continue;
      const int64_t off = (a0 + al) * n + j;
      const int pos = j < n / 2 ? j + L - n / 2 : j - n / 2;
      float2 a = acc[i];
      for (int c = 0; c < C; ++c) {
        const float2 sv = S[(int64_t)c * N + off];
        const float v = lines[(al * C + c) * g.LS + pos];
        if (part == 0) {
          a.x = fmaf(sv.x, v, a.x);
          a.y = fmaf(-sv.y, v, a.y);
        } else {
          a.x = fmaf(sv.y, v, a.x);
          a.y = fmaf(sv.x, v, a.y);
        }
      }
      acc[i] = a;
    }
  }
  __device__ void epilogue_store(const Tile2& g, int64_t a0, const float2 (&acc)[kMaxPerThread]) const {
    const int total = g.na * n;
    const float hs = scale * undo.factor();
#pragma unroll
    for (int i = 0; i < kMaxPerThread; ++i) {
      const int e = (int)threadIdx.x + i * (int)blockDim.x;
      if (e >= total) break;
      const int al = e / n;
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
      out[a * n + j] = cscale(acc[i], f);
    }
  }
};

// the coil expansion always zero-pads (centred), the coil reduction crops
inline bool half_gap(const Ld2CoilExpand& x, int L) { return 2 * x.n == L; }
inline bool half_gap(const St2CoilReduce& x, int L) { return 2 * x.n == L; }

}  // namespace isg
