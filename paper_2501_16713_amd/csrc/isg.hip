// C ABI of the image-space gridding / nonrigid SENSE library (see isg.h):
// plans, plan-time preparation of displacement fields and trajectories, and
// the sequencing of the HIP kernels that make up each operator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <new>
#include <string>
#include <vector>

#include "../../include/isg.h"
#include "common.h"
#include "fft.h"
#include "fft2.h"
#include "gridding.h"
#include "passes.h"
#include "solver.h"
#include "recon.h"
#include "binning.h"

#include <hipcub/device/device_radix_sort.hpp>

using namespace isg;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static isg_status fail(isg_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

struct HipError {
  hipError_t e;
  std::string where;
};

#define HIP_OK(expr)                                                                   \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess) throw HipError{_e, std::string(#expr) + " @" + std::to_string(__LINE__)}; \
  } while (0)

#define LAUNCH_OK() HIP_OK(hipGetLastError())

// ---------------------------------------------------------------------------
// host-side helpers
// ---------------------------------------------------------------------------
static FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  f.s = s;
  f.m = (uint32_t)((((1ull << 32) * ((1ull << s) - d)) / d) + 1);
  return f;
}

// radices of the Stockham stages of a line of length L (factors 2, 3, 5, 7)
static bool factor_radices(int L, std::vector<int>& R) {
  R.clear();
  int m = L;
  while (m % 8 == 0 && m > 4) { R.push_back(8); m /= 8; }
  while (m % 4 == 0) { R.push_back(4); m /= 4; }
  while (m % 2 == 0) { R.push_back(2); m /= 2; }
  while (m % 5 == 0) { R.push_back(5); m /= 5; }
  while (m % 3 == 0) { R.push_back(3); m /= 3; }
  while (m % 7 == 0) { R.push_back(7); m /= 7; }
  return m == 1 && (int)R.size() <= kMaxStages;
}

// continuous Fourier transform of the Kaiser-Bessel kernel:
// W sinh(z)/z with z = sqrt(beta^2 - (pi W f)^2) (sin branch past the root)
static double kb_transform(double f, double beta) {
  const double W = kWidth;
  const double z2 = beta * beta - (M_PI * W * f) * (M_PI * W * f);
  if (z2 > 0) {
    const double z = std::sqrt(z2);
    return W * std::sinh(z) / z;
  }
  if (z2 < 0) {
    const double z = std::sqrt(-z2);
    return W * std::sin(z) / z;
  }
  return W;
}

static double kb_beta() {
  const double W = kWidth, a = kAlpha;
  return M_PI * std::sqrt((W / a) * (W / a) * (a - 0.5) * (a - 0.5) - 0.8);
}

// I0(beta sqrt(t)) / c(0) = sum_k (beta^2/4)^k t^k / (k!)^2 / c(0).  The
// kernel is divided by the zero frequency of its transform, c(0) (its
// integral), so that the taps of one axis sum to about 1 and k-space grids
// hold values on the scale of the data; the deapodization tables carry the
// matching factor c(0) per axis, which leaves every operator unchanged.
static KbPoly make_kbpoly(double beta) {
  KbPoly p;
  const double q = beta * beta / 4.0;
  const double norm = 1.0 / kb_transform(0.0, beta);
  double a = 1.0;
  double coef[kPolyDeg + 1];
  for (int k = 0; k <= kPolyDeg; ++k) {
    if (k) a *= q / ((double)k * k);
    coef[k] = a * norm;
    p.a[k] = (float)coef[k];
  }
  for (int k = 1; k <= kPolyDeg; ++k) p.da[k - 1] = (float)(coef[k] * k);
  return p;
}

// ---------------------------------------------------------------------------
// plan objects
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct isg_plan {
  int ndim = 0;
  int n[3] = {1, 1, 1};
  int G[3] = {1, 1, 1};
  int64_t N = 0, NG = 0;
  int C = 1, P = 1;
  int storage = 0;
  // options (isg_plan_set_option)
  int opt_spread_chunk = 512;  // samples per k-space spread work unit
  int opt_phase_batch = 1;     // states per k-space gather / spread launch
  int opt_graph = 0;           // isg_normal replays a captured graph
  int opt_fft_addr = 1;        // buffer-addressed FFT passes where allowed
  int opt_ktile_t1 = 8;        // k-space spread tile extent along axis 1
  float* hsc = nullptr;        // half-precision grids: per-call scale [s, 1/s] (device)
  double* hs_part = nullptr;   // partial sums for hsc
  unsigned* ymax = nullptr;    // half-precision grids: largest |re|, |im| of each batch slot's spread data
                               // ([kMaxPhasesPerLaunch][kYmaxSlots])
  int opt_blk_tlog = 3;        // log2 of the i1 block of the row-blocked k-space arrays
  Blk blk_grid, blk_k2;        // layouts of the coil-expanded grid and of k2buf
  hipStream_t stream = nullptr;
  int device = 0;
  int ncu = 256;  // compute units of the device
  bool failed = false;
  double beta = 0;
  KbPoly kb;
  Dims dims;
  TileDims wtile;   // image-space spread tiles
  KTile ktile;      // k-space spread tiles
  // tables
  float* dk[3] = {nullptr, nullptr, nullptr};  // c(0)/c(k/G), DFT bin order
  float* dx[3] = {nullptr, nullptr, nullptr};  // c(0)/c(x/G), centred positions
  std::map<int, LinePlan> lines;
  std::vector<void*> owned;
  std::map<void*, size_t> sizes;  // bytes of every device allocation the plan counts
  // live prepared handles; destroying the plan detaches them (their later
  // destroy then frees only their own memory)
  std::set<isg_motion*> motions;
  std::set<isg_traj*> trajs;
  // scratch
  float2* ugrid = nullptr;  // [NG]
  float2* bufA = nullptr;   // [N]
  float2* bufB = nullptr;   // [G0][n1][n2]
  float2* bufC = nullptr;   // [G0][G1][n2]
  float2* mbuf = nullptr;   // [N]
  float2* wbuf = nullptr;   // [P][N]
  DevBuf kgrid;             // [batch][NG][C]
  DevBuf kgrid_adj;         // [batch][touched tiles][tile][C], tile-major spread output
  void* k1buf = nullptr;
  void* k2buf = nullptr;
  DevBuf ybuf;              // normal-operator data, grown on demand
  DevBuf wreg;              // image-space spread regions, [tiles][E0][E1][E2]
  DevBuf partial;           // spread partial tiles, grown on demand
  // CG
  float2 *cg_r = nullptr, *cg_p = nullptr, *cg_q = nullptr;
  double* cg_part = nullptr;
  CgScalars* cg_sc = nullptr;
  DevBuf cg_hist;
  DevBuf tune_out;  // autotuner output image
  DevBuf sol;       // FISTA / power iteration / registration vectors, grown on demand
  DevBuf sol_part;  // their FP64 partial sums and histories
  DevBuf bin;       // motion binning: keys, sorted keys, values, sort scratch, check flags
  hipStream_t own_stream = nullptr;  // CG capture stream when the caller's is the null stream
  int64_t bytes = 0;
  // bumped whenever device memory a captured graph may reference is freed or
  // moved (buffer growth, unit rebuilds, handle destruction, option changes)
  uint64_t generation = 0;
  struct NormalGraph {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<const void*> key;
    double lam = 0;
  } ngraph;
  // per-kernel event timing (off unless enabled)
  struct Pending {
    std::string tag;
    hipEvent_t a, b;
  };
  bool timing = false;
  bool capturing = false;
  std::string timing_filter;  // only tags starting with this prefix ("" = all)
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<int64_t, double>> timed;  // tag -> (launches, total ms)
};

static hipEvent_t pool_event(isg_plan* pl) {
  if (!pl->pool.empty()) {
    hipEvent_t e = pl->pool.back();
    pl->pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIP_OK(hipEventCreate(&e));
  return e;
}

// brackets one launch with events on the plan's stream when timing is on
struct Tick {
  isg_plan* pl;
  bool on;
  hipEvent_t a = nullptr;
  const char* tag;
  Tick(isg_plan* p, const char* t) : pl(p), tag(t) {
    on = pl->timing && !pl->capturing &&
         (pl->timing_filter.empty() || std::string(t).rfind(pl->timing_filter, 0) == 0);
    if (on) {
      a = pool_event(pl);
      HIP_OK(hipEventRecord(a, pl->stream));
    }
  }
  ~Tick() noexcept(false) {
    if (!on) return;
    hipEvent_t b = pool_event(pl);
    HIP_OK(hipEventRecord(b, pl->stream));
    pl->pending.push_back({tag, a, b});
  }
};

static void collect_timing(isg_plan* pl) {
  for (auto& p : pl->pending) {
    HIP_OK(hipEventSynchronize(p.b));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, p.a, p.b));
    auto& t = pl->timed[p.tag];
    t.first += 1;
    t.second += ms;
    pl->pool.push_back(p.a);
    pl->pool.push_back(p.b);
  }
  pl->pending.clear();
}

struct isg_motion {
  isg_plan* plan = nullptr;
  float* d = nullptr;       // [ndim][N]
  int* tile_off = nullptr;  // [ntiles + 1]
  int* vox = nullptr;
  int64_t nentries = 0;
};

struct isg_traj {
  isg_plan* plan = nullptr;
  int64_t M = 0;
  uint64_t* colmask = nullptr;  // touched-tile masks (null: all tiles written)
  uint64_t* fmask = nullptr;    // touched-run masks per grid column (i1, i2) (null with colmask)
  uint64_t* cact = nullptr;     // 3D: bit i1 of word [i2][i1 / 64] set where fmask[(i1, i2)] != 0 (G1 <= 512)
  int cact_w = 0;               // words per i2
  int64_t fine_cells = 0;       // grid cells in the touched runs
  int64_t active_cols = 0;      // grid columns (i1, i2) holding a touched run
  int* colbase = nullptr;       // tile-major spread output: first slot of each tile column
  std::vector<uint64_t> colmask_h;
  std::vector<int> colbase_h;
  int64_t nvis = 0;             // spread visits (sample, tile) in tile order
  int64_t ntouched = 0;         // spread tiles any sample touches
  KTap* taps_v = nullptr;       // tap record of every visit
  int* vis_off = nullptr;       // [M + 1]: visits of sample j ...
  int* vis = nullptr;           // ... are vis[vis_off[j] .. vis_off[j + 1])
  KTap* taps = nullptr;
  int* order = nullptr;
  int* gorder = nullptr;          // [M]: gather processing order, samples grouped by their first spread tile
  KUnit* units = nullptr;
  int nunits = 0;
  KSplit* splits = nullptr;
  int nsplits = 0;
  int nslots = 0;
  int chunk = 0;                  // spread chunk the units were built for
  int ts[3] = {0, 0, 0};          // k-space tile shape the bins were built for
  float dens = 1.f;               // bound on the samples whose kernel reaches one grid cell
  float* k = nullptr;             // [M][ndim] the trajectory (cycles/voxel), for the translation phases
  float2* phase = nullptr;        // [M] exp(-2 pi i k_j . t_j) of a bulk translation, or null
  std::vector<int> tile_first;    // host: tile-sorted visits of tile t are tile_first[t] .. tile_first[t+1]
  std::vector<KTap> taps_h;        // host copy of taps (re-binning for another tile shape)
  std::vector<int> tile_rows;      // per tile: visits reaching rows 0-3 only, rows 4-7 only (register spread)
};

static bool tiled_adjoint(const isg_plan* pl);

static void* dmalloc(isg_plan* pl, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw std::bad_alloc();
  }
  pl->bytes += (int64_t)bytes;
  pl->sizes[p] = bytes;
  return p;
}

// free memory from dmalloc (it leaves the plan's count); pl may be null for
// a handle whose plan was destroyed first
static hipError_t dfree(isg_plan* pl, void* p) {
  if (!p) return hipSuccess;
  if (pl) {
    auto it = pl->sizes.find(p);
    if (it != pl->sizes.end()) {
      pl->bytes -= (int64_t)it->second;
      pl->sizes.erase(it);
    }
  }
  return hipFree(p);
}

static void* plan_alloc(isg_plan* pl, size_t bytes) {
  void* p = dmalloc(pl, bytes);
  pl->owned.push_back(p);
  return p;
}

static void grow(isg_plan* pl, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes) return;
  pl->generation++;
  if (b.p) {
    HIP_OK(hipStreamSynchronize(pl->stream));
    HIP_OK(dfree(pl, b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  b.p = dmalloc(pl, bytes);
  b.bytes = bytes;
}

static const LinePlan& line_plan(isg_plan* pl, int L) {
  auto it = pl->lines.find(L);
  if (it != pl->lines.end()) return it->second;
  std::vector<int> R;
  factor_radices(L, R);
  LinePlan lp;
  memset(&lp, 0, sizeof(lp));
  lp.L = L;
  lp.nst = (int)R.size();
  int Ns = 1;
  for (int s = 0; s < lp.nst; ++s) {
    lp.R[s] = R[s];
    lp.step[s] = L / (Ns * R[s]);
    lp.ns[s] = make_fastdiv((uint32_t)Ns);
    Ns *= R[s];
  }
  std::vector<float2> tw(L);
  for (int q = 0; q < L; ++q) {
    const double th = 2.0 * M_PI * (double)q / (double)L;
    tw[q] = make_float2((float)std::cos(th), (float)-std::sin(th));
  }
  float2* dtw = (float2*)plan_alloc(pl, sizeof(float2) * L);
  HIP_OK(hipMemcpy(dtw, tw.data(), sizeof(float2) * L, hipMemcpyHostToDevice));
  lp.tw = dtw;
  return pl->lines.emplace(L, lp).first->second;
}

// ---------------------------------------------------------------------------
// FFT pass launcher
// ---------------------------------------------------------------------------
static TileGeom make_geom(int64_t A, int64_t B, int Lmax, int nb_fixed) {
  TileGeom g;
  const int max_lines = std::max(1, std::min(64, std::min((kFftThreads * kMaxPerThread) / Lmax, 8192 / (Lmax + 1))));
  if (nb_fixed > 0) {
    g.nb = nb_fixed;
    g.na = (int)std::max<int64_t>(1, std::min<int64_t>(A, max_lines / nb_fixed));
  } else if (B == 1) {
    g.nb = 1;
    g.na = (int)std::min<int64_t>(A, std::min(16, max_lines));
  } else {
    g.nb = (int)std::min<int64_t>(B, std::min(16, max_lines));
    g.na = 1;
  }
  g.A = A;
  g.B = B;
  g.tiles_b = (B + g.nb - 1) / g.nb;
  g.LS = Lmax + 1;
  return g;
}

template <class K>
static void allow_lds(K kernel, size_t bytes) {
  static std::map<const void*, size_t> done;  // largest size already allowed per kernel
  if (bytes <= 65536) return;
  size_t& have = done[(const void*)kernel];
  if (have >= bytes) return;
  HIP_OK(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  have = bytes;
}

template <class Ld, class Mid, class St>
static void run_pass(isg_plan* pl, const char* tag, const Ld& ld, const Mid& mid, const St& st, const TileGeom& g,
                     const LinePlan& l1, float s1, const LinePlan* l2, float s2) {
  PassDesc pd;
  memset(&pd, 0, sizeof(pd));
  pd.g = g;
  pd.l1 = l1;
  pd.s1 = s1;
  pd.two = l2 ? 1 : 0;
  if (l2) pd.l2 = *l2;
  pd.s2 = s2;
  const int nl = g.na * g.nb;
  {  // every butterfly and every mid-step element must fit the per-thread arrays
    const int tpl = kFftThreads / nl;
    auto fits = [&](const LinePlan& lp) {
      for (int s = 0; s < lp.nst; ++s) {
        const int R = lp.R[s];
        const int per = (lp.L / R + tpl - 1) / tpl;
        if (per > (kMaxPerThread + R - 1) / R) return false;
      }
      return (lp.L + tpl - 1) / tpl <= kMaxPerThread && lp.L < g.LS;
    };
    if (nl < 1 || nl > kFftThreads || !fits(l1) || (l2 && !fits(*l2)))
      throw HipError{hipErrorInvalidConfiguration, "FFT pass tiling does not fit the per-thread arrays"};
  }
  const size_t lds = sizeof(float2) * ((size_t)l1.L + (l2 ? l2->L : 0) + (size_t)nl * g.LS);
  const int64_t tiles = ((g.A + g.na - 1) / g.na) * g.tiles_b;
  auto kern = fft_pass_kernel<Ld, Mid, St>;
  allow_lds(kern, lds);
  const int64_t gx = std::min<int64_t>(tiles, 1 << 30);
  const int64_t gy = (tiles + gx - 1) / gx;
  Tick tick(pl, tag);
  hipLaunchKernelGGL(kern, dim3((unsigned)gx, (unsigned)gy), dim3(kFftThreads), lds, pl->stream, ld, mid, st, pd);
  LAUNCH_OK();
}

// ---------------------------------------------------------------------------
// two-step register FFT passes (compile-time lengths)
// ---------------------------------------------------------------------------
static bool fft2_supported(int L) {
  switch (L) {
    case 32: case 40: case 48: case 64: case 80: case 96: case 128:
    case 160: case 192: case 256: case 320: case 512: return true;
    default: return false;
  }
}

// the same tile with XCD-contiguous workgroup order (measured faster for the
// adjoint axis-1 pass, whose lines are 30 KB apart; slower for the axis-0
// passes, the last-axis passes and the 32-line forward axis-1 pass)
static Tile2 xcd_order(Tile2 g) {
  g.tiles = -1;
  return g;
}

// nb_fixed > 0: nb_fixed lines along the inner extent per tile (several
// rows of tiles when they fit `budget` threads); < 0: up to -nb_fixed inner lines
// (at most 1024 threads), one row; 0: 16 inner lines, one row
static Tile2 make_tile2(int64_t A, int64_t B, int L, int nb_fixed, int budget = 512) {
  int L1 = 4, L2 = 8;
  switch (L) {
    case 32: L1 = 4; L2 = 8; break;
    case 40: L1 = 5; L2 = 8; break;
    case 48: L1 = 6; L2 = 8; break;
    case 64: L1 = 8; L2 = 8; break;
    case 80: L1 = 8; L2 = 10; break;
    case 96: L1 = 8; L2 = 12; break;
    case 128: L1 = 8; L2 = 16; break;
    case 160: L1 = 10; L2 = 16; break;
    case 192: L1 = 12; L2 = 16; break;
    case 256: L1 = 16; L2 = 16; break;
    case 320: L1 = 16; L2 = 20; break;
    case 512: L1 = 16; L2 = 32; break;
  }
  Tile2 g;
  g.A = A;
  g.B = B;
  if (nb_fixed > 0) {
    g.nb = nb_fixed;
    g.na = (int)std::max<int64_t>(1, std::min<int64_t>(A, budget / (nb_fixed * L2)));
  } else if (nb_fixed < 0) {
    g.nb = (int)std::min<int64_t>(B, std::min(-nb_fixed, 1024 / L2));
    g.na = 1;
  } else {
    g.nb = (int)std::min<int64_t>(B, 16);
    g.na = 1;
  }
  g.tiles_b = (B + g.nb - 1) / g.nb;
  // line stride in the float exchange buffer: with up to 16 lines along the
  // inner extent, 2 mod 4 keeps the step-1 stores and step-2 loads of a
  // wavefront on distinct LDS banks within each half-wavefront for every
  // factorization above; with 32 or more, an odd stride does (a bank model
  // of 32 four-byte banks per half-wavefront, and measured)
  int LS = L1 * (L2 + 1);
  if (g.nb >= 32) {
    if (!(LS & 1)) ++LS;
  } else {
    while (LS % 4 != 2) ++LS;
  }
  g.LS = LS;
  g.tiles = 0;
  return g;
}

template <int L1, int L2, int SG, int M1, int M2, int GAP, class Ld, class St>
static void launch_fft2(isg_plan* pl, const char* tag, const Ld& ld, const St& st, const Tile2& g) {
  constexpr int L = L1 * L2;
  const int nl = g.na * g.nb;
  const int threads = ((nl * L2 + 63) / 64) * 64;
  if (threads > 1024 || nl * L1 > threads)
    throw HipError{hipErrorInvalidConfiguration, "fft2 tile does not fit one workgroup"};
  if constexpr (St::kEpilogue) {
    if ((int64_t)g.na * st.n > (int64_t)St::kMaxPerThread * threads)
      throw HipError{hipErrorInvalidConfiguration, "fft2 epilogue outputs exceed the per-thread accumulators"};
  }
  // lines exchanged as float parts (see fft2_kernel)
  const size_t lds = sizeof(float2) * (size_t)L + sizeof(float) * (size_t)nl * g.LS + lds_extra(ld);
  if (((GAP & 1) && !half_gap(ld, L)) || ((GAP & 2) && !half_gap(st, L)))
    throw HipError{hipErrorInvalidConfiguration, "fft2 gap flags do not match the line maps"};
  auto kern = fft2_kernel<L1, L2, SG, M1, M2, Ld, St, GAP>;
  allow_lds(kern, lds);
  const int64_t tiles = ((g.A + g.na - 1) / g.na) * g.tiles_b;
  Tile2 gl = g;
  int64_t gx, gy;
  if (g.tiles < 0 && tiles <= (1 << 30)) {  // XCD-contiguous order requested (see fft2_kernel)
    gl.tiles = tiles;
    gx = 8 * ((tiles + 7) / 8);
    gy = 1;
  } else {
    gl.tiles = 0;
    gx = std::min<int64_t>(tiles, 1 << 30);
    gy = (tiles + gx - 1) / gx;
  }
  Tick tick(pl, tag);
  hipLaunchKernelGGL(kern, dim3((unsigned)gx, (unsigned)gy), dim3(threads), lds, pl->stream, ld, st, gl);
  LAUNCH_OK();
}

template <int SG, int M1, int M2, int GAP = 0, class Ld, class St>
static void run_fft2(isg_plan* pl, const char* tag, int L, const Ld& ld, const St& st, const Tile2& g) {
  switch (L) {
    case 32: launch_fft2<4, 8, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 40: launch_fft2<5, 8, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 48: launch_fft2<6, 8, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 64: launch_fft2<8, 8, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 80: launch_fft2<8, 10, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 96: launch_fft2<8, 12, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 128: launch_fft2<8, 16, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 160: launch_fft2<10, 16, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 192: launch_fft2<12, 16, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 256: launch_fft2<16, 16, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 320: launch_fft2<16, 20, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 512: launch_fft2<16, 32, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    default: throw HipError{hipErrorInvalidValue, "fft2: unsupported length"};
  }
}

// ---- buffer-addressed forms (see the F loaders in fft2.h) -------------------
// lengths whose two factors are both multiples of 4
static bool fft2_fast_length(int L) {
  switch (L) {
    case 32: case 64: case 96: case 128: case 192: case 256: case 320: case 512: return true;
    default: return false;
  }
}

static void fft2_factors(int L, int& L1, int& L2) {
  switch (L) {
    case 32: L1 = 4; L2 = 8; break;
    case 64: L1 = 8; L2 = 8; break;
    case 96: L1 = 8; L2 = 12; break;
    case 128: L1 = 8; L2 = 16; break;
    case 192: L1 = 12; L2 = 16; break;
    case 256: L1 = 16; L2 = 16; break;
    case 320: L1 = 16; L2 = 20; break;
    case 512: L1 = 16; L2 = 32; break;
    default: L1 = L2 = 0; break;
  }
}

constexpr int64_t kLaneSpan = (int64_t)1 << 31;  // lane byte offsets stay below this

// largest lane offset (elements) of a strided access: the tile's lines and
// the per-lane part of the row, `step` the element-index step (rows L2 for
// loads, L1 for stores), `cnt` the lane's part (n2 < L2 or k1 < L1)
static int64_t strided_lane_span(int64_t sa, int64_t sj, int tlog, int64_t bs, const Tile2& g, int cnt) {
  const int64_t row = tlog >= 30 ? (int64_t)(cnt - 1) * sj
                                 : (int64_t)((cnt - 1) >> tlog) * bs + (int64_t)((1 << tlog) - 1) * sj;
  return (int64_t)(g.na - 1) * sa + g.nb + row;
}

template <class T>
static bool strided_fast_ok(const T& x, int L, const Tile2& g, bool load, size_t es) {
  int L1, L2;
  fft2_factors(L, L1, L2);
  const int step = load ? L2 : L1, cnt = load ? L2 : L1;
  if (x.tlog < 30) {
    const int blk = 1 << x.tlog;
    if (step % blk) return false;
    if (x.map != kDense && (L / 4) % blk) return false;
  }
  return strided_lane_span(x.sa, x.sj, x.tlog, x.bs, g, cnt) * (int64_t)es < kLaneSpan;
}

// the nb columns of every tile of an axis-0 pass are contiguous in the
// row-blocked layout, and the lane offsets fit
static bool rows_fast_ok(const Blk& blk, int L, const Tile2& g, size_t es) {
  if (g.na != 1) return false;
  if (blk.tlog < 30 && (((int64_t)1 << blk.tlog) * blk.g2c) % g.nb) return false;
  return ((int64_t)g.nb + (int64_t)L * blk.rs) * (int64_t)es < kLaneSpan;
}

template <class T>
static bool fast_ok(const T&, int, const Tile2&) { return true; }  // no buffer form: used as is
template <int S>
static bool fast_ok(const Ld2Strided<S>& x, int L, const Tile2& g) {
  return strided_fast_ok(x, L, g, true, sizeof(typename Elem<S>::T));
}
template <int S>
static bool fast_ok(const St2Strided<S>& x, int L, const Tile2& g) {
  return strided_fast_ok(x, L, g, false, sizeof(typename Elem<S>::T));
}
template <int S>
static bool fast_ok(const Ld2Image<S>& x, int L, const Tile2& g) {
  return strided_fast_ok(x, L, g, true, sizeof(typename Elem<S>::T));
}
template <int S>
static bool fast_ok(const St2Image<S>& x, int L, const Tile2& g) {
  return strided_fast_ok(x, L, g, false, sizeof(typename Elem<S>::T));
}
template <int S>
static bool fast_ok(const Ld2Rows<S>& x, int L, const Tile2& g) {
  return rows_fast_ok(x.blk, L, g, sizeof(typename Elem<S>::T));
}
template <int S>
static bool fast_ok(const St2Rows<S>& x, int L, const Tile2& g) {
  return rows_fast_ok(x.blk, L, g, sizeof(typename Elem<S>::T));
}
template <int S>
static bool fast_ok(const St2Masked<S>& x, int L, const Tile2& g) {
  int L1, L2;
  fft2_factors(L, L1, L2);
  return x.tm.ts0_log2 == 3 && L1 % 8 == 0 && rows_fast_ok(x.blk, L, g, sizeof(typename Elem<S>::T));
}
template <int S>
static bool fast_ok(const Ld2Tiles<S>& x, int L, const Tile2& g) {
  // runs of 8 cells; one tile row of tile columns (or two) within 2^31 bytes
  const int64_t span = 2 * (int64_t)x.nt2 * (L / 8 + 1) * x.volC * (int64_t)sizeof(typename Elem<S>::T);
  return x.ts0_log2 == 3 && g.na == 1 && span < kLaneSpan && L / 8 <= 64 && g.B + g.nb < kLaneSpan;
}

template <int S>
static bool fast_ok(const Ld2StridedM<S>& x, int L, const Tile2& g) {
  return strided_fast_ok(x, L, g, true, sizeof(typename Elem<S>::T));
}

template <class T>
static const T& to_fast(const T& x, int, const Tile2&) { return x; }
template <int S>
static Ld2StridedF<S> to_fast(const Ld2Strided<S>& x, int, const Tile2&) {
  Ld2StridedF<S> f;
  f.p = x.p; f.sa = x.sa; f.sj = x.sj; f.tlog = x.tlog; f.bs = x.bs; f.map = x.map; f.tw = x.tw;
  return f;
}
template <int S>
static St2StridedF<S> to_fast(const St2Strided<S>& x, int, const Tile2&) {
  St2StridedF<S> f;
  f.p = x.p; f.sa = x.sa; f.sj = x.sj; f.tlog = x.tlog; f.bs = x.bs; f.map = x.map; f.scale = x.scale;
  f.zfill = x.zfill;
  return f;
}
template <int S>
static Ld2ImageF<S> to_fast(const Ld2Image<S>& x, int L, const Tile2& g) {
  Ld2ImageF<S> f;
  static_cast<Ld2StridedF<S>&>(f) = to_fast(static_cast<const Ld2Strided<S>&>(x), L, g);
  return f;
}
template <int S>
static St2ImageF<S> to_fast(const St2Image<S>& x, int L, const Tile2& g) {
  St2ImageF<S> f;
  static_cast<St2StridedF<S>&>(f) = to_fast(static_cast<const St2Strided<S>&>(x), L, g);
  return f;
}
template <int S>
static Ld2RowsF<S> to_fast(const Ld2Rows<S>& x, int, const Tile2&) {
  Ld2RowsF<S> f;
  f.p = x.p; f.blk = x.blk; f.map = x.map; f.tw = x.tw;
  return f;
}
template <int S>
static St2RowsF<S> to_fast(const St2Rows<S>& x, int, const Tile2&) {
  St2RowsF<S> f;
  f.p = x.p; f.blk = x.blk; f.map = x.map; f.scale = x.scale; f.zfill = x.zfill;
  return f;
}
template <int S>
static St2MaskedF<S> to_fast(const St2Masked<S>& x, int, const Tile2&) {
  St2MaskedF<S> f;
  f.p = x.p; f.blk = x.blk; f.tm = x.tm; f.scale = x.scale;
  return f;
}
template <int S>
static Ld2TilesF<S> to_fast(const Ld2Tiles<S>& x, int L, const Tile2& g) {
  Ld2TilesF<S> f;
  f.p = x.p; f.colmask = x.colmask; f.fmask = x.fmask; f.colbase = x.colbase;
  f.C = x.C; f.G2 = x.G2; f.ts1 = x.ts1; f.ts2 = x.ts2; f.nt2 = x.nt2;
  f.nruns = L / 8;
  f.ngp = (g.nb - 1) / x.C + 2;
  f.Q = g.B / x.C;
  f.volC = x.volC; f.rowC = x.rowC; f.tw = x.tw;
  return f;
}

template <int SG, int M1, int M2, int GAP, class Ld, class St>
static void run_fft2_fast(isg_plan* pl, const char* tag, int L, const Ld& ld, const St& st, const Tile2& g) {
  switch (L) {
    case 32: launch_fft2<4, 8, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 64: launch_fft2<8, 8, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 96: launch_fft2<8, 12, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 128: launch_fft2<8, 16, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 192: launch_fft2<12, 16, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 256: launch_fft2<16, 16, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 320: launch_fft2<16, 20, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    case 512: launch_fft2<16, 32, SG, M1, M2, GAP>(pl, tag, ld, st, g); break;
    default: throw HipError{hipErrorInvalidValue, "fft2: no buffer-addressed form for this length"};
  }
}

// one register-FFT pass: the buffer-addressed form where the plan allows it
// and both sides qualify, else the general form
template <int SG, int M1, int M2, int GAP = 0, class Ld, class St>
static void fft2_pass(isg_plan* pl, const char* tag, int L, const Ld& ld, const St& st, const Tile2& g) {
  // the tile geometry the launch will use (XCD order does not change it)
  if (pl->opt_fft_addr && fft2_fast_length(L) && fast_ok(ld, L, g) && fast_ok(st, L, g))
    run_fft2_fast<SG, M1, M2, GAP>(pl, tag, L, to_fast(ld, L, g), to_fast(st, L, g), g);
  else
    run_fft2<SG, M1, M2, GAP>(pl, tag, L, ld, st, g);
}

// a pass that must take the buffer-addressed form (its loader or store has
// no general one)
template <int SG, int M1, int M2, int GAP = 0, class Ld, class St>
static void fft2_pass_fast(isg_plan* pl, const char* tag, int L, const Ld& ld, const St& st, const Tile2& g) {
  if (!(fft2_fast_length(L) && fast_ok(ld, L, g) && fast_ok(st, L, g)))
    throw HipError{hipErrorInvalidConfiguration, "fft2: a masked pass needs the buffer-addressed form"};
  run_fft2_fast<SG, M1, M2, GAP>(pl, tag, L, to_fast(ld, L, g), to_fast(st, L, g), g);
}

template <int S>
static Ld2Strided<S> ld2(const isg_plan* pl, const void* p, int64_t sa, int64_t sj, int map, int L) {
  Ld2Strided<S> l;
  l.p = (const typename Elem<S>::T*)p;
  l.sa = sa;
  l.sj = sj;
  l.tlog = 30;
  l.bs = 0;
  l.map = map;
  l.tw = pl->lines.at(L).tw;
  return l;
}

template <int S>
static St2Strided<S> st2(void* p, int64_t sa, int64_t sj, int map, float scale = 1.f) {
  St2Strided<S> s;
  s.p = (typename Elem<S>::T*)p;
  s.sa = sa;
  s.sj = sj;
  s.tlog = 30;
  s.bs = 0;
  s.map = map;
  s.scale = scale;
  return s;
}

// the same for the single-image upsampling passes (types of their own)
static Ld2Image<kFP32> ld2_img(const isg_plan* pl, const float2* p, int64_t sa, int64_t sj, int map, int L) {
  Ld2Image<kFP32> l;
  static_cast<Ld2Strided<kFP32>&>(l) = ld2<kFP32>(pl, p, sa, sj, map, L);
  return l;
}
static St2Image<kFP32> st2_img(float2* p, int64_t sa, int64_t sj, int map) {
  St2Image<kFP32> s;
  static_cast<St2Strided<kFP32>&>(s) = st2<kFP32>(p, sa, sj, map);
  return s;
}

// lines along axis 1 of a row-blocked array: a = i0, b = i2 C + c, j = i1
template <int S>
static Ld2Strided<S> ld2_axis1(const isg_plan* pl, const void* p, const Blk& blk, int map, int L) {
  Ld2Strided<S> l = ld2<S>(pl, p, blk.rs, blk.g2c, map, L);
  l.tlog = blk.tlog;
  l.bs = blk.bs;
  return l;
}

template <int S>
static St2Strided<S> st2_axis1(void* p, const Blk& blk, int map, float scale) {
  St2Strided<S> s = st2<S>(p, blk.rs, blk.g2c, map, scale);
  s.tlog = blk.tlog;
  s.bs = blk.bs;
  return s;
}

// The adjoint axis-1 pass restricted to a trajectory's touched grid columns
// (see Ld2StridedM): only where its buffer-addressed form runs, so that the
// adjoint axis-0 pass may leave untouched columns unwritten.
static bool ax1_masked(const isg_plan* pl, const isg_traj* tr) {
  if (!tr || !tr->cact || !pl->opt_fft_addr || pl->ndim != 3 || !fft2_fast_length(pl->G[1])) return false;
  const Tile2 g = make_tile2(pl->n[0], (int64_t)pl->G[2] * pl->C, pl->G[1], 0);
  Ld2Strided<kFP32> l;
  l.sa = pl->blk_k2.rs;
  l.sj = pl->blk_k2.g2c;
  l.tlog = pl->blk_k2.tlog;
  l.bs = pl->blk_k2.bs;
  l.map = kDense;
  return strided_fast_ok(l, pl->G[1], g, true, sizeof(float2));
}

// the forward axis-1 store restricted to the trajectory's touched grid
// columns, where the buffer-addressed form runs (else null: plain store)
static bool fwd_ax1_masked(const isg_plan* pl, const isg_traj* tr, const Tile2& g) {
  if (!ax1_masked(pl, tr)) return false;
  St2Strided<kFP32> s;
  s.sa = pl->blk_k2.rs;
  s.sj = pl->blk_k2.g2c;
  s.tlog = pl->blk_k2.tlog;
  s.bs = pl->blk_k2.bs;
  s.map = kDense;
  Ld2Strided<kFP32> l;
  l.sa = (int64_t)pl->n[1] * pl->G[2] * pl->C;
  l.sj = (int64_t)pl->G[2] * pl->C;
  l.tlog = 30;
  l.bs = 0;
  l.map = kCentred;
  return strided_fast_ok(s, pl->G[1], g, false, sizeof(float2)) && strided_fast_ok(l, pl->G[1], g, true, sizeof(float2));
}

static St2StridedMF<kFP32> st2_axis1_masked(const isg_plan* pl, void* p, const Blk& blk, const isg_traj* tr, int L) {
  St2StridedMF<kFP32> s;
  static_cast<St2StridedF<kFP32>&>(s) = to_fast(st2_axis1<kFP32>(p, blk, kDense, 1.f), L, Tile2{});
  s.cm = tr->cact;
  s.cmC = pl->C;
  s.cmW = tr->cact_w;
  return s;
}

static Ld2StridedM<kFP32> ld2_axis1_masked(const isg_plan* pl, const void* p, const Blk& blk, const isg_traj* tr,
                                           int L) {
  Ld2StridedM<kFP32> l;
  static_cast<Ld2StridedF<kFP32>&>(l) = to_fast(ld2_axis1<kFP32>(pl, p, blk, kDense, L), L, Tile2{});
  l.cm = tr->cact;
  l.cmC = pl->C;
  l.cmW = tr->cact_w;
  return l;
}

// lines along axis 0 of a row-blocked array: b = column, j = i0
template <int S>
static Ld2Rows<S> ld2_rows(const isg_plan* pl, const void* p, const Blk& blk, int map, int L) {
  Ld2Rows<S> l;
  l.p = (const typename Elem<S>::T*)p;
  l.blk = blk;
  l.map = map;
  l.tw = pl->lines.at(L).tw;
  return l;
}

template <int S>
static St2Rows<S> st2_rows(void* p, const Blk& blk, int map, float scale) {
  St2Rows<S> s;
  s.p = (typename Elem<S>::T*)p;
  s.blk = blk;
  s.map = map;
  s.scale = scale;
  return s;
}

template <int S>
static LdStrided<S> ld_strided(const void* p, int64_t sa, int64_t sj, int n, int L, int map, const TileGeom& g) {
  LdStrided<S> l;
  l.p = (const typename Elem<S>::T*)p;
  l.sa = sa;
  l.sj = sj;
  l.n = n;
  l.L = L;
  l.map = map;
  l.nbd = make_fastdiv(g.nb);
  l.nd = make_fastdiv(n);
  return l;
}

template <int S>
static StStrided<S> st_strided(void* p, int64_t sa, int64_t sj, int n, int L, int map, const TileGeom& g,
                                float scale = 1.f) {
  StStrided<S> s;
  s.p = (typename Elem<S>::T*)p;
  s.sa = sa;
  s.sj = sj;
  s.n = n;
  s.L = L;
  s.map = map;
  s.scale = scale;
  s.nbd = make_fastdiv(g.nb);
  s.nd = make_fastdiv(n);
  return s;
}

static AxisTabs tabs(float* const t[3]) {
  AxisTabs a;
  for (int i = 0; i < 3; ++i) a.t[i] = t[i];
  return a;
}

// ---------------------------------------------------------------------------
// image-space gridding front end (Eq. 9 up to the gather):
// u = F^H_G Z (1/C*) F_N x / |N|  on the oversampled grid
// ---------------------------------------------------------------------------
static void upsample(isg_plan* pl, const float2* x, float2* u) {
  const int n0 = pl->n[0], n1 = pl->n[1], n2 = pl->n[2];
  const int G0 = pl->G[0], G1 = pl->G[1], G2 = pl->G[2];
  UpMid mid;
  mid.tab = tabs(pl->dk);
  mid.scale = (float)(1.0 / (double)pl->N);
  mid.n = n0;
  mid.G = G0;
  if (pl->ndim == 3) {
    mid.n_inner = n2;
    mid.three_d = 1;
    // the passes along axes 1 and 2 take the register FFT where the length
    // allows it (an in-place pass is safe there: a workgroup loads all its
    // lines before any store, and no line is shared between workgroups)
    if (fft2_supported(n2)) {  // F along axis 2
      fft2_pass<-1, kJFast, kJFast>(pl, "fft_up_ax2", n2, ld2_img(pl, x, n2, 1, kDense, n2),
                                   st2_img(pl->bufA, n2, 1, kDense), make_tile2((int64_t)n0 * n1, 1, n2, 1));
    } else {
      TileGeom g = make_geom((int64_t)n0 * n1, 1, n2, 0);
      run_pass(pl, "fft_up_ax2", ld_strided<kFP32>(x, n2, 1, n2, n2, kDense, g), NoMid(),
               st_strided<kFP32>(pl->bufA, n2, 1, n2, n2, kDense, g), g, line_plan(pl, n2), -1.f, nullptr, 0.f);
    }
    if (fft2_supported(n1)) {  // F along axis 1, in place
      fft2_pass<-1, kBFast, kBFast>(pl, "fft_up_ax1", n1, ld2_img(pl, pl->bufA, (int64_t)n1 * n2, n2, kDense, n1),
                                   st2_img(pl->bufA, (int64_t)n1 * n2, n2, kDense), make_tile2(n0, n2, n1, 0));
    } else {
      TileGeom g = make_geom(n0, n2, n1, 0);
      run_pass(pl, "fft_up_ax1", ld_strided<kFP32>(pl->bufA, (int64_t)n1 * n2, n2, n1, n1, kDense, g), NoMid(),
               st_strided<kFP32>(pl->bufA, (int64_t)n1 * n2, n2, n1, n1, kDense, g), g, line_plan(pl, n1), -1.f,
               nullptr, 0.f);
    }
    {  // F along axis 0, deapodize, pad, F^H of length G0
      TileGeom g = make_geom(1, (int64_t)n1 * n2, G0, 0);
      run_pass(pl, "fft_up_ax0", ld_strided<kFP32>(pl->bufA, 0, (int64_t)n1 * n2, n0, n0, kDense, g), mid,
               st_strided<kFP32>(pl->bufB, 0, (int64_t)n1 * n2, G0, G0, kDense, g), g, line_plan(pl, n0), -1.f,
               &line_plan(pl, G0), +1.f);
    }
    if (fft2_supported(G1)) {  // F^H along axis 1 with the spectral pad
      fft2_pass<+1, kBFast, kBFast, 1>(pl, "fft_up_G1", G1,
                                      ld2_img(pl, pl->bufB, (int64_t)n1 * n2, n2, kSpectral, G1),
                                      st2_img(pl->bufC, (int64_t)G1 * n2, n2, kDense), make_tile2(G0, n2, G1, 0));
    } else {
      TileGeom g = make_geom(G0, n2, G1, 0);
      run_pass(pl, "fft_up_G1", ld_strided<kFP32>(pl->bufB, (int64_t)n1 * n2, n2, n1, G1, kSpectral, g), NoMid(),
               st_strided<kFP32>(pl->bufC, (int64_t)G1 * n2, n2, G1, G1, kDense, g), g, line_plan(pl, G1), +1.f,
               nullptr, 0.f);
    }
    if (fft2_supported(G2)) {  // F^H along axis 2 with the spectral pad
      fft2_pass<+1, kJFast, kJFast, 1>(pl, "fft_up_G2", G2, ld2_img(pl, pl->bufC, n2, 1, kSpectral, G2),
                                      st2_img(u, G2, 1, kDense), make_tile2((int64_t)G0 * G1, 1, G2, 1));
    } else {
      TileGeom g = make_geom((int64_t)G0 * G1, 1, G2, 0);
      run_pass(pl, "fft_up_G2", ld_strided<kFP32>(pl->bufC, n2, 1, n2, G2, kSpectral, g), NoMid(),
               st_strided<kFP32>(u, G2, 1, G2, G2, kDense, g), g, line_plan(pl, G2), +1.f, nullptr, 0.f);
    }
  } else {
    mid.n_inner = 1;
    mid.three_d = 0;
    if (fft2_supported(n1)) {
      fft2_pass<-1, kJFast, kJFast>(pl, "fft_up_ax1", n1, ld2_img(pl, x, n1, 1, kDense, n1),
                                   st2_img(pl->bufA, n1, 1, kDense), make_tile2(n0, 1, n1, 1));
    } else {
      TileGeom g = make_geom(n0, 1, n1, 0);
      run_pass(pl, "fft_up_ax1", ld_strided<kFP32>(x, n1, 1, n1, n1, kDense, g), NoMid(),
               st_strided<kFP32>(pl->bufA, n1, 1, n1, n1, kDense, g), g, line_plan(pl, n1), -1.f, nullptr, 0.f);
    }
    {
      TileGeom g = make_geom(1, n1, G0, 0);
      run_pass(pl, "fft_up_ax0", ld_strided<kFP32>(pl->bufA, 0, n1, n0, n0, kDense, g), mid,
               st_strided<kFP32>(pl->bufB, 0, n1, G0, G0, kDense, g), g, line_plan(pl, n0), -1.f, &line_plan(pl, G0),
               +1.f);
    }
    if (fft2_supported(G1)) {
      fft2_pass<+1, kJFast, kJFast, 1>(pl, "fft_up_G1", G1, ld2_img(pl, pl->bufB, n1, 1, kSpectral, G1),
                                      st2_img(u, G1, 1, kDense), make_tile2(G0, 1, G1, 1));
    } else {
      TileGeom g = make_geom(G0, 1, G1, 0);
      run_pass(pl, "fft_up_G1", ld_strided<kFP32>(pl->bufB, n1, 1, n1, G1, kSpectral, g), NoMid(),
               st_strided<kFP32>(u, G1, 1, G1, G1, kDense, g), g, line_plan(pl, G1), +1.f, nullptr, 0.f);
    }
  }
}

// adjoint of upsample (Eq. 8 after the spread): x = F^H_N (1/C) Z^H F_G U / |N|
// Intermediate images of the adjoint upsampling passes: A [n0][n1][n2],
// B [G0][n1][n2], C [G0][G1][n2] (C unused in 2D).
struct UpBufs {
  float2 *A, *B, *C;
};

static UpBufs plan_up_bufs(const isg_plan* pl);

static void upsample_adjoint(isg_plan* pl, const float2* U, float2* out, const UpBufs& ub) {
  const int n0 = pl->n[0], n1 = pl->n[1], n2 = pl->n[2];
  const int G0 = pl->G[0], G1 = pl->G[1], G2 = pl->G[2];
  UpHMid mid;
  mid.tab = tabs(pl->dk);
  mid.scale = (float)(1.0 / (double)pl->N);
  mid.n = n0;
  mid.G = G0;
  if (pl->ndim == 3) {
    mid.n_inner = n2;
    mid.three_d = 1;
    // register FFTs along axes 2 and 1 where the length allows (as in upsample)
    if (fft2_supported(G2)) {  // F along axis 2, crop
      fft2_pass<-1, kJFast, kJFast, 2>(pl, "fft_uph_G2", G2, ld2_img(pl, U, G2, 1, kDense, G2),
                                      st2_img(ub.C, n2, 1, kSpectral), make_tile2((int64_t)G0 * G1, 1, G2, 1));
    } else {
      TileGeom g = make_geom((int64_t)G0 * G1, 1, G2, 0);
      run_pass(pl, "fft_uph_G2", ld_strided<kFP32>(U, G2, 1, G2, G2, kDense, g), NoMid(),
               st_strided<kFP32>(ub.C, n2, 1, n2, G2, kSpectral, g), g, line_plan(pl, G2), -1.f, nullptr, 0.f);
    }
    if (fft2_supported(G1)) {  // F along axis 1, crop
      fft2_pass<-1, kBFast, kBFast, 2>(pl, "fft_uph_G1", G1,
                                      ld2_img(pl, ub.C, (int64_t)G1 * n2, n2, kDense, G1),
                                      st2_img(ub.B, (int64_t)n1 * n2, n2, kSpectral), make_tile2(G0, n2, G1, 0));
    } else {
      TileGeom g = make_geom(G0, n2, G1, 0);
      run_pass(pl, "fft_uph_G1", ld_strided<kFP32>(ub.C, (int64_t)G1 * n2, n2, G1, G1, kDense, g), NoMid(),
               st_strided<kFP32>(ub.B, (int64_t)n1 * n2, n2, n1, G1, kSpectral, g), g, line_plan(pl, G1), -1.f,
               nullptr, 0.f);
    }
    {  // F along axis 0, crop, deapodize, F^H of length n0
      TileGeom g = make_geom(1, (int64_t)n1 * n2, G0, 0);
      run_pass(pl, "fft_uph_ax0", ld_strided<kFP32>(ub.B, 0, (int64_t)n1 * n2, G0, G0, kDense, g), mid,
               st_strided<kFP32>(ub.A, 0, (int64_t)n1 * n2, n0, n0, kDense, g), g, line_plan(pl, G0), -1.f,
               &line_plan(pl, n0), +1.f);
    }
    if (fft2_supported(n1)) {  // F^H along axis 1, in place
      fft2_pass<+1, kBFast, kBFast>(pl, "fft_uph_ax1", n1, ld2_img(pl, ub.A, (int64_t)n1 * n2, n2, kDense, n1),
                                   st2_img(ub.A, (int64_t)n1 * n2, n2, kDense), make_tile2(n0, n2, n1, 0));
    } else {
      TileGeom g = make_geom(n0, n2, n1, 0);
      run_pass(pl, "fft_uph_ax1", ld_strided<kFP32>(ub.A, (int64_t)n1 * n2, n2, n1, n1, kDense, g), NoMid(),
               st_strided<kFP32>(ub.A, (int64_t)n1 * n2, n2, n1, n1, kDense, g), g, line_plan(pl, n1), +1.f,
               nullptr, 0.f);
    }
    if (fft2_supported(n2)) {  // F^H along axis 2
      fft2_pass<+1, kJFast, kJFast>(pl, "fft_uph_ax2", n2, ld2_img(pl, ub.A, n2, 1, kDense, n2),
                                   st2_img(out, n2, 1, kDense), make_tile2((int64_t)n0 * n1, 1, n2, 1));
    } else {
      TileGeom g = make_geom((int64_t)n0 * n1, 1, n2, 0);
      run_pass(pl, "fft_uph_ax2", ld_strided<kFP32>(ub.A, n2, 1, n2, n2, kDense, g), NoMid(),
               st_strided<kFP32>(out, n2, 1, n2, n2, kDense, g), g, line_plan(pl, n2), +1.f, nullptr, 0.f);
    }
  } else {
    mid.n_inner = 1;
    mid.three_d = 0;
    if (fft2_supported(G1)) {
      fft2_pass<-1, kJFast, kJFast, 2>(pl, "fft_uph_G1", G1, ld2_img(pl, U, G1, 1, kDense, G1),
                                      st2_img(ub.B, n1, 1, kSpectral), make_tile2(G0, 1, G1, 1));
    } else {
      TileGeom g = make_geom(G0, 1, G1, 0);
      run_pass(pl, "fft_uph_G1", ld_strided<kFP32>(U, G1, 1, G1, G1, kDense, g), NoMid(),
               st_strided<kFP32>(ub.B, n1, 1, n1, G1, kSpectral, g), g, line_plan(pl, G1), -1.f, nullptr, 0.f);
    }
    {
      TileGeom g = make_geom(1, n1, G0, 0);
      run_pass(pl, "fft_uph_ax0", ld_strided<kFP32>(ub.B, 0, n1, G0, G0, kDense, g), mid,
               st_strided<kFP32>(ub.A, 0, n1, n0, n0, kDense, g), g, line_plan(pl, G0), -1.f, &line_plan(pl, n0),
               +1.f);
    }
    if (fft2_supported(n1)) {
      fft2_pass<+1, kJFast, kJFast>(pl, "fft_uph_ax1", n1, ld2_img(pl, ub.A, n1, 1, kDense, n1),
                                   st2_img(out, n1, 1, kDense), make_tile2(n0, 1, n1, 1));
    } else {
      TileGeom g = make_geom(n0, 1, n1, 0);
      run_pass(pl, "fft_uph_ax1", ld_strided<kFP32>(ub.A, n1, 1, n1, n1, kDense, g), NoMid(),
               st_strided<kFP32>(out, n1, 1, n1, n1, kDense, g), g, line_plan(pl, n1), +1.f, nullptr, 0.f);
    }
  }
}

static UpBufs plan_up_bufs(const isg_plan* pl) { return UpBufs{pl->bufA, pl->bufB, pl->bufC}; }

static void upsample_adjoint(isg_plan* pl, const float2* U, float2* out) {
  upsample_adjoint(pl, U, out, plan_up_bufs(pl));
}

// ---------------------------------------------------------------------------
// image-space gather / spread
// ---------------------------------------------------------------------------
static unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

static void warp_gather(isg_plan* pl, const float2* u, const isg_motion* mo, float2* out) {
  Tick tick(pl, "warp_gather");
  if (pl->ndim == 3)
    hipLaunchKernelGGL(warp_gather_kernel<3>, dim3(blocks_for(pl->N, kGridThreads)), dim3(kGridThreads), 0,
                       pl->stream, u, mo->d, out, pl->dims, pl->kb);
  else
    hipLaunchKernelGGL(warp_gather_kernel<2>, dim3(blocks_for(pl->N, kGridThreads)), dim3(kGridThreads), 0,
                       pl->stream, u, mo->d, out, pl->dims, pl->kb);
  LAUNCH_OK();
}

static int warp_ntiles(const isg_plan* pl) {
  int t = 1;
  for (int i = 0; i < pl->ndim; ++i) t *= pl->wtile.nt[i];
  return t;
}

// bytes of the image-space spread regions
static size_t warp_region_bytes(const isg_plan* pl) {
  return sizeof(float2) * (size_t)warp_ntiles(pl) * pl->wtile.RV;
}

// U = sum_p P_{d_p} w_p over the given states: pass 1 accumulates each
// tile's entries into its region (reg, warp_region_bytes), pass 2 sums the
// overlapping regions into U, both once per kMaxPhasesPerLaunch states
static void warp_spread(isg_plan* pl, int P, const isg_motion* const* mo, const float2* const* w, float2* U,
                        float2* reg) {
  const size_t lds = warp_spread_lds_bytes(pl->wtile, pl->ndim);
  const int nt = warp_ntiles(pl);
  const int Gl = pl->G[pl->ndim - 1];
  const int rows = (int)(pl->NG / Gl);
  const int sthreads = ((Gl + 63) / 64) * 64;
  if (sthreads > 1024) throw HipError{hipErrorInvalidConfiguration, "spread rows longer than a workgroup"};
  for (int p0 = 0; p0 < P; p0 += kMaxPhasesPerLaunch) {
    WarpSpreadPhases ph;
    memset(&ph, 0, sizeof(ph));
    ph.P = std::min(kMaxPhasesPerLaunch, P - p0);
    for (int i = 0; i < ph.P; ++i) {
      ph.tile_off[i] = mo[p0 + i]->tile_off;
      ph.vox[i] = mo[p0 + i]->vox;
      ph.d[i] = mo[p0 + i]->d;
      ph.w[i] = w[p0 + i];
    }
    const int acc = p0 > 0 ? 1 : 0;
    const unsigned nblk = 8u * (unsigned)((nt + 7) / 8);  // one workgroup per tile, XCD-contiguous order
    if (pl->ndim == 3)
      allow_lds(warp_spread_kernel<3>, lds);
    else
      allow_lds(warp_spread_kernel<2>, lds);
    {
      Tick tick(pl, "warp_spread");
      if (pl->ndim == 3)
        hipLaunchKernelGGL(warp_spread_kernel<3>, dim3(nblk), dim3(64 * kWarpWaves), lds, pl->stream, ph, reg, nt,
                           pl->dims, pl->wtile, pl->kb);
      else
        hipLaunchKernelGGL(warp_spread_kernel<2>, dim3(nblk), dim3(64 * kWarpWaves), lds, pl->stream, ph, reg, nt,
                           pl->dims, pl->wtile, pl->kb);
      LAUNCH_OK();
    }
    {
      Tick tick(pl, "warp_spread_sum");
      if (pl->ndim == 3)
        hipLaunchKernelGGL(warp_spread_sum_kernel<3>, dim3(rows), dim3(sthreads), 0, pl->stream, reg, U, acc, pl->dims,
                           pl->wtile);
      else
        hipLaunchKernelGGL(warp_spread_sum_kernel<2>, dim3(rows), dim3(sthreads), 0, pl->stream, reg, U, acc, pl->dims,
                           pl->wtile);
      LAUNCH_OK();
    }
  }
}

// the same with the plan's region buffer (grown on first use)
static void warp_spread(isg_plan* pl, int P, const isg_motion* const* mo, const float2* const* w, float2* U) {
  grow(pl, pl->wreg, warp_region_bytes(pl));
  warp_spread(pl, P, mo, w, U, (float2*)pl->wreg.p);
}

// ---------------------------------------------------------------------------
// coil-expanded k-space front end and back end
// ---------------------------------------------------------------------------
// |N|^{-1/2} of the coil passes, taken whole at the image end (first load
// of the forward, last store of the adjoint).  The pruned intermediates
// between the passes ([n0][n1][G2][C] and [n0][G1][G2][C]) are FP32 in every
// precision form; only the coil-expanded grid itself (the forward axis-0
// pass's output, the spread's output) takes the plan's storage, so a
// half-precision form rounds once per direction.  With the normalised kernel
// and the input scale, the grid holds values on the scale of the data (at
// most about |N|^{1/2} at the k-space centre: inside FP16 range).
static float image_end_scale(const isg_plan* pl) { return (float)(1.0 / std::sqrt((double)pl->N)); }

static Ld2CoilExpand ld2_expand(isg_plan* pl, const float2* m, const float2* Sm, int n, int n1, int L) {
  Ld2CoilExpand ld;
  ld.m = m;
  ld.S = Sm;
  ld.dx = tabs(pl->dx);
  ld.scale = image_end_scale(pl);
  ld.dsc = pl->hsc;
  ld.N = pl->N;
  ld.n = n;
  ld.n1 = n1;
  ld.tw = line_plan(pl, L).tw;
  return ld;
}

static St2CoilReduce st2_reduce(isg_plan* pl, float2* w, const float2* Sm, int n, int n1, int L,
                                const HalfUndo& undo) {
  St2CoilReduce st;
  st.out = w;
  st.S = Sm;
  st.dx = tabs(pl->dx);
  st.scale = image_end_scale(pl);
  st.undo = undo;
  st.N = pl->N;
  st.n = n;
  st.L = L;
  st.C = pl->C;
  st.n1 = n1;
  return st;
}

static TileMask tile_mask(const isg_plan* pl, const isg_traj* tr) {
  TileMask tm;
  tm.fmask = tr ? tr->fmask : nullptr;
  tm.C = pl->C;
  tm.G2 = pl->G[2];
  int lg = 0;
  while ((1 << lg) < pl->ktile.TS[0]) ++lg;
  tm.ts0_log2 = lg;
  tm.three_d = pl->ndim == 3;
  return tm;
}

template <int S>
static St2Masked<S> st2_masked(void* p, const Blk& blk, const TileMask& tm, float scale) {
  St2Masked<S> st;
  st.p = (typename Elem<S>::T*)p;
  st.blk = blk;
  st.tm = tm;
  st.scale = scale;
  return st;
}

template <int S>
static Ld2Tiles<S> ld2_tiles(isg_plan* pl, const void* p, const isg_traj* tr, int L) {
  Ld2Tiles<S> ld;
  ld.p = (const typename Elem<S>::T*)p;
  ld.colmask = tr->colmask;
  ld.fmask = tr->fmask;
  ld.colbase = tr->colbase;
  ld.C = pl->C;
  ld.G2 = pl->G[2];
  int lg = 0;
  while ((1 << lg) < pl->ktile.TS[0]) ++lg;
  ld.ts0_log2 = lg;
  ld.ts1 = pl->ktile.TS[1];
  ld.ts2 = pl->ktile.TS[2];
  ld.nt2 = pl->ktile.nt[2];
  ld.volC = (int64_t)pl->ktile.vol * pl->C;
  ld.rowC = (int64_t)pl->ktile.TS[1] * pl->ktile.TS[2] * pl->C;
  ld.cdiv = make_fastdiv((uint32_t)pl->C);
  ld.g2div = make_fastdiv((uint32_t)pl->G[2]);
  ld.tw = line_plan(pl, L).tw;
  return ld;
}

template <int S>
static Ld2Masked<S> ld2_masked(isg_plan* pl, const void* p, const Blk& blk, const TileMask& tm, int L) {
  Ld2Masked<S> ld;
  ld.p = (const typename Elem<S>::T*)p;
  ld.blk = blk;
  ld.tm = tm;
  ld.tw = line_plan(pl, L).tw;
  return ld;
}

// grid = F_G Z (S_c m / c(x/G)) |N|^{-1/2} for every coil; tiles of `tr`
// that no sample touches are not written (tr may be null)
template <int S>
static void coil_forward_t(isg_plan* pl, const float2* m, const float2* Sm, void* grid, const isg_traj* tr) {
  const int n0 = pl->n[0], n1 = pl->n[1], n2 = pl->n[2];
  const int G0 = pl->G[0], G1 = pl->G[1], G2 = pl->G[2];
  const int C = pl->C;
  const float scale = image_end_scale(pl);
  if (pl->ndim == 3 && fft2_supported(G0) && fft2_supported(G1) && fft2_supported(G2)) {
    // S_c m / c(x/G) |N|^{-1/2}, centred pad, F along axis 2
    fft2_pass<-1, kJFast, kBFast, 1>(pl, "fft_coil_fwd_last", G2, ld2_expand(pl, m, Sm, n2, n1, G2),
                                 st2<kFP32>(pl->k1buf, (int64_t)G2 * C, C, kDense),
                                 make_tile2((int64_t)n0 * n1, C, G2, C));
    // centred pad, F along axis 1 (into the row-blocked k2buf), storing only
    // the trajectory's touched grid columns where the buffer form runs (their
    // column words are read before the loads; read on the store path they
    // cost more than the stores they save)
    const Tile2 g1 = make_tile2(n0, (int64_t)G2 * C, G1, -32);  // 32 lines, plain order: measured faster
    if (tr && fwd_ax1_masked(pl, tr, g1))
      fft2_pass_fast<-1, kBFast, kBFast, 1>(pl, "fft_coil_fwd_ax1", G1,
                                            ld2<kFP32>(pl, pl->k1buf, (int64_t)n1 * G2 * C, (int64_t)G2 * C, kCentred, G1),
                                            st2_axis1_masked(pl, pl->k2buf, pl->blk_k2, tr, G1), g1);
    else
      fft2_pass<-1, kBFast, kBFast, 1>(pl, "fft_coil_fwd_ax1", G1,
                                       ld2<kFP32>(pl, pl->k1buf, (int64_t)n1 * G2 * C, (int64_t)G2 * C, kCentred, G1),
                                       st2_axis1<kFP32>(pl->k2buf, pl->blk_k2, kDense, 1.f), g1);
    // centred pad, F along axis 0
    fft2_pass<-1, kBFast, kBFast, 1>(pl, "fft_coil_fwd_ax0", G0, ld2_rows<kFP32>(pl, pl->k2buf, pl->blk_k2, kCentred, G0),
                                 st2_masked<S>(grid, pl->blk_grid, tile_mask(pl, tr), 1.f),
                                 make_tile2(1, (int64_t)G1 * G2 * C, G0, pl->blk_k2.tlog < 30 ? -32 : -48));
    // (lines per workgroup measured at 160^3: 32 with the row-blocked k2
    // layout, 48 with the plain one)
  } else if (pl->ndim == 2 && fft2_supported(G0) && fft2_supported(G1)) {
    fft2_pass<-1, kJFast, kBFast, 1>(pl, "fft_coil_fwd_last", G1, ld2_expand(pl, m, Sm, n1, 0, G1),
                                 st2<kFP32>(pl->k1buf, (int64_t)G1 * C, C, kDense), make_tile2(n0, C, G1, C));
    fft2_pass<-1, kBFast, kBFast, 1>(pl, "fft_coil_fwd_ax0", G0, ld2<kFP32>(pl, pl->k1buf, 0, (int64_t)G1 * C, kCentred, G0),
                                 st2_masked<S>(grid, pl->blk_grid, tile_mask(pl, tr), 1.f),
                                 make_tile2(1, (int64_t)G1 * C, G0, 0));
  } else if (pl->ndim == 3) {
    {  // S_c m / c(x/G) |N|^{-1/2}, centred pad, F along axis 2
      TileGeom g = make_geom((int64_t)n0 * n1, C, G2, C);
      LdCoilExpand ld;
      ld.m = m;
      ld.S = Sm;
      ld.dx = tabs(pl->dx);
      ld.scale = scale;
      ld.dsc = pl->hsc;
      ld.N = pl->N;
      ld.n = n2;
      ld.L = G2;
      ld.C = C;
      ld.n1 = n1;
      ld.nd = make_fastdiv(n2);
      ld.cd = make_fastdiv(C);
      run_pass(pl, "fft_coil_fwd_last", ld, NoMid(), st_strided<kFP32>(pl->k1buf, (int64_t)G2 * C, C, G2, G2, kDense, g), g,
               line_plan(pl, G2), -1.f, nullptr, 0.f);
    }
    {  // centred pad, F along axis 1
      TileGeom g = make_geom(n0, (int64_t)G2 * C, G1, 0);
      run_pass(pl, "fft_coil_fwd_ax1", ld_strided<kFP32>(pl->k1buf, (int64_t)n1 * G2 * C, (int64_t)G2 * C, n1, G1, kCentred, g), NoMid(),
               st_strided<kFP32>(pl->k2buf, (int64_t)G1 * G2 * C, (int64_t)G2 * C, G1, G1, kDense, g), g,
               line_plan(pl, G1), -1.f, nullptr, 0.f);
    }
    {  // centred pad, F along axis 0
      TileGeom g = make_geom(1, (int64_t)G1 * G2 * C, G0, 0);
      run_pass(pl, "fft_coil_fwd_ax0", ld_strided<kFP32>(pl->k2buf, 0, (int64_t)G1 * G2 * C, n0, G0, kCentred, g), NoMid(),
               st_strided<S>(grid, 0, (int64_t)G1 * G2 * C, G0, G0, kDense, g), g,
               line_plan(pl, G0), -1.f, nullptr, 0.f);
    }
  } else {
    {
      TileGeom g = make_geom(n0, C, G1, C);
      LdCoilExpand ld;
      ld.m = m;
      ld.S = Sm;
      ld.dx = tabs(pl->dx);
      ld.scale = scale;
      ld.dsc = pl->hsc;
      ld.N = pl->N;
      ld.n = n1;
      ld.L = G1;
      ld.C = C;
      ld.n1 = 0;
      ld.nd = make_fastdiv(n1);
      ld.cd = make_fastdiv(C);
      run_pass(pl, "fft_coil_fwd_last", ld, NoMid(), st_strided<kFP32>(pl->k1buf, (int64_t)G1 * C, C, G1, G1, kDense, g), g,
               line_plan(pl, G1), -1.f, nullptr, 0.f);
    }
    {
      TileGeom g = make_geom(1, (int64_t)G1 * C, G0, 0);
      run_pass(pl, "fft_coil_fwd_ax0", ld_strided<kFP32>(pl->k1buf, 0, (int64_t)G1 * C, n0, G0, kCentred, g), NoMid(),
               st_strided<S>(grid, 0, (int64_t)G1 * C, G0, G0, kDense, g), g,
               line_plan(pl, G0), -1.f, nullptr, 0.f);
    }
  }
}

// w = sum_c conj(S_c) crop(F_G^H grid) / c(x/G) |N|^{-1/2}; tiles of `tr`
// that no sample touches are read as zero (tr may be null)
template <int S>
static void coil_adjoint_t(isg_plan* pl, const void* grid, const float2* Sm, float2* w, const isg_traj* tr,
                           const HalfUndo& undo) {
  const int n0 = pl->n[0], n1 = pl->n[1], n2 = pl->n[2];
  const int G0 = pl->G[0], G1 = pl->G[1], G2 = pl->G[2];
  const int C = pl->C;
  const float scale = image_end_scale(pl);
  if (pl->ndim == 3 && fft2_supported(G0) && fft2_supported(G1) && fft2_supported(G2)) {
    // with the masked axis-1 pass, tiles no sample reaches are not written
    // (the axis-1 pass reads their columns as zero); else they store zeros
    const bool masked = ax1_masked(pl, tr);
    St2Rows<kFP32> k2st = st2_rows<kFP32>(pl->k2buf, pl->blk_k2, kCentred, 1.f);
    k2st.zfill = !masked;
    if (tr && tiled_adjoint(pl))  // spread output tile-major (touched tiles only)
      fft2_pass<+1, kBFast, kBFast, 2>(pl, "fft_coil_adj_ax0", G0, ld2_tiles<S>(pl, grid, tr, G0), k2st,
                                       make_tile2(1, (int64_t)G1 * G2 * C, G0, 0));
    else
      fft2_pass<+1, kBFast, kBFast, 2>(pl, "fft_coil_adj_ax0", G0,
                                       ld2_masked<S>(pl, grid, pl->blk_grid, tile_mask(pl, tr), G0), k2st,
                                       make_tile2(1, (int64_t)G1 * G2 * C, G0, 0));
    if (masked)
      fft2_pass_fast<+1, kBFast, kBFast, 2>(pl, "fft_coil_adj_ax1", G1,
                                            ld2_axis1_masked(pl, pl->k2buf, pl->blk_k2, tr, G1),
                                            st2<kFP32>(pl->k1buf, (int64_t)n1 * G2 * C, (int64_t)G2 * C, kCentred, 1.f),
                                            xcd_order(make_tile2(n0, (int64_t)G2 * C, G1, 0)));
    else
      fft2_pass<+1, kBFast, kBFast, 2>(pl, "fft_coil_adj_ax1", G1,
                                       ld2_axis1<kFP32>(pl, pl->k2buf, pl->blk_k2, kDense, G1),
                                       st2<kFP32>(pl->k1buf, (int64_t)n1 * G2 * C, (int64_t)G2 * C, kCentred, 1.f),
                                       xcd_order(make_tile2(n0, (int64_t)G2 * C, G1, 0)));
    fft2_pass<+1, kBFast, kBFast, 2>(pl, "fft_coil_adj_last", G2, ld2<kFP32>(pl, pl->k1buf, (int64_t)G2 * C, C, kDense, G2),
                                 st2_reduce(pl, w, Sm, n2, n1, G2, undo), make_tile2((int64_t)n0 * n1, C, G2, C, 256));  // one row of coils per workgroup: measured faster
  } else if (pl->ndim == 2 && fft2_supported(G0) && fft2_supported(G1)) {
    fft2_pass<+1, kBFast, kBFast, 2>(pl, "fft_coil_adj_ax0", G0, ld2_masked<S>(pl, grid, pl->blk_grid, tile_mask(pl, tr), G0),
                                 st2<kFP32>(pl->k1buf, 0, (int64_t)G1 * C, kCentred, 1.f),
                                 make_tile2(1, (int64_t)G1 * C, G0, 0));
    fft2_pass<+1, kBFast, kBFast, 2>(pl, "fft_coil_adj_last", G1, ld2<kFP32>(pl, pl->k1buf, (int64_t)G1 * C, C, kDense, G1),
                                 st2_reduce(pl, w, Sm, n1, 0, G1, undo), make_tile2(n0, C, G1, C));
  } else if (pl->ndim == 3) {
    {  // F^H along axis 0, centred crop
      TileGeom g = make_geom(1, (int64_t)G1 * G2 * C, G0, 0);
      run_pass(pl, "fft_coil_adj_ax0", ld_strided<S>(grid, 0, (int64_t)G1 * G2 * C, G0, G0, kDense, g), NoMid(),
               st_strided<kFP32>(pl->k2buf, 0, (int64_t)G1 * G2 * C, n0, G0, kCentred, g), g,
               line_plan(pl, G0), +1.f,
               nullptr, 0.f);
    }
    {  // F^H along axis 1, centred crop
      TileGeom g = make_geom(n0, (int64_t)G2 * C, G1, 0);
      run_pass(pl, "fft_coil_adj_ax1", ld_strided<kFP32>(pl->k2buf, (int64_t)G1 * G2 * C, (int64_t)G2 * C, G1, G1, kDense, g), NoMid(),
               st_strided<kFP32>(pl->k1buf, (int64_t)n1 * G2 * C, (int64_t)G2 * C, n1, G1, kCentred, g), g,
               line_plan(pl, G1), +1.f, nullptr, 0.f);
    }
    {  // F^H along axis 2, centred crop, 1/c(x/G) |N|^{-1/2}, conj(S_c), coil sum
      TileGeom g = make_geom((int64_t)n0 * n1, C, G2, C);
      StCoilReduce st;
      st.out = w;
      st.S = Sm;
      st.dx = tabs(pl->dx);
      st.scale = scale;
      st.undo = undo;
      st.N = pl->N;
      st.n = n2;
      st.L = G2;
      st.C = C;
      st.n1 = n1;
      st.nd = make_fastdiv(n2);
      run_pass(pl, "fft_coil_adj_last", ld_strided<kFP32>(pl->k1buf, (int64_t)G2 * C, C, G2, G2, kDense, g), NoMid(), st, g,
               line_plan(pl, G2), +1.f, nullptr, 0.f);
    }
  } else {
    {
      TileGeom g = make_geom(1, (int64_t)G1 * C, G0, 0);
      run_pass(pl, "fft_coil_adj_ax0", ld_strided<S>(grid, 0, (int64_t)G1 * C, G0, G0, kDense, g), NoMid(),
               st_strided<kFP32>(pl->k1buf, 0, (int64_t)G1 * C, n0, G0, kCentred, g), g,
               line_plan(pl, G0), +1.f,
               nullptr, 0.f);
    }
    {
      TileGeom g = make_geom(n0, C, G1, C);
      StCoilReduce st;
      st.out = w;
      st.S = Sm;
      st.dx = tabs(pl->dx);
      st.scale = scale;
      st.undo = undo;
      st.N = pl->N;
      st.n = n1;
      st.L = G1;
      st.C = C;
      st.n1 = 0;
      st.nd = make_fastdiv(n1);
      run_pass(pl, "fft_coil_adj_last", ld_strided<kFP32>(pl->k1buf, (int64_t)G1 * C, C, G1, G1, kDense, g), NoMid(), st, g,
               line_plan(pl, G1), +1.f, nullptr, 0.f);
    }
  }
}

// y[j][c] in sample order, or (to_visits) y[v][c] for every spread visit v
// One state's share of a batched k-space interpolation: its trajectory, its
// coil-expanded grid and its data.
struct KJob {
  const isg_traj* tr;
  void* grid;         // gather input (and spread output unless sgrid is set)
  const float2* yin;  // spread input, visit order [nvis][C]
  float2* yout;       // gather output ([M][C], or [nvis][C] in visit order)
  void* sgrid;        // spread output when it differs from grid (tile-major)
};

// the ymax words of n batch slots = 0 before the gather or permutes that fill them
static void zero_ymax(isg_plan* pl, unsigned* ymax, int n) {
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(256), 0, pl->stream, ymax, n * kYmaxSlots);
  LAUNCH_OK();
}

// y = G_p grid_p for every job, kMaxPhasesPerLaunch states per launch
template <int S>
static void kgather_t(isg_plan* pl, const KJob* jobs, int n, bool to_visits, const float* oscale = nullptr) {
  using T = typename Elem<S>::T;
  if (pl->ymax && n > kMaxPhasesPerLaunch)  // one spread-scale slot per state of a batch
    throw HipError{hipErrorInvalidValue, "k-space batch larger than the spread-scale slots"};
  const int spw = 64 / pl->C;  // samples per wavefront
  for (int j0 = 0; j0 < n; j0 += kMaxPhasesPerLaunch) {
    KBatch<T> bt{};
    memset(&bt, 0, sizeof(bt));
    bt.n = std::min(kMaxPhasesPerLaunch, n - j0);
    int64_t blocks = 0;
    for (int i = 0; i < bt.n; ++i) {
      const KJob& jb = jobs[j0 + i];
      bt.first[i] = (int)blocks;
      bt.taps[i] = jb.tr->taps;
      bt.count[i] = jb.tr->M;
      bt.gorder[i] = jb.tr->gorder;
      bt.phase[i] = to_visits ? nullptr : jb.tr->phase;  // into visit order (normal operator): the phases cancel
      bt.vis_off[i] = to_visits ? jb.tr->vis_off : nullptr;
      bt.vis[i] = to_visits ? jb.tr->vis : nullptr;
      bt.yout[i] = jb.yout;
      bt.grid[i] = (T*)jb.grid;
      const int64_t waves = (jb.tr->M + spw - 1) / spw;
      blocks += (waves + kGridThreads / 64 - 1) / (kGridThreads / 64);
    }
    bt.first[bt.n] = (int)blocks;
    bt.blk = pl->blk_grid;
    bt.oscale = oscale;
    bt.ymax = to_visits && pl->ymax ? pl->ymax + (size_t)j0 * kYmaxSlots : nullptr;
    if (bt.ymax) zero_ymax(pl, bt.ymax, bt.n);
    Tick tick(pl, "kgather");
    if (pl->ndim == 3)
      hipLaunchKernelGGL((kgather_kernel<3, S>), dim3((unsigned)blocks), dim3(kGridThreads), 0, pl->stream, bt,
                         pl->C, pl->dims, pl->kb);
    else
      hipLaunchKernelGGL((kgather_kernel<2, S>), dim3((unsigned)blocks), dim3(kGridThreads), 0, pl->stream, bt,
                         pl->C, pl->dims, pl->kb);
    LAUNCH_OK();
  }
}

// grid_p = G_p^H y_p for every job (visit-ordered inputs), kMaxPhasesPerLaunch
// states per launch; the "kspread" tag times the spread kernel alone,
// "kspread_reduce" the fixed-order reduction of split tiles
template <int NDIM, int S>
static void kspread_nd(isg_plan* pl, const KJob* jobs, int n) {
  using T = typename Elem<S>::T;
  const size_t lds = kspread_lds_bytes(pl->ktile, pl->C);
  const size_t volC = (size_t)pl->ktile.vol * pl->C;
  // 3D tiles of 8 x 4 x 8 take the register-accumulating spread, others the
  // LDS read-modify-write one (both one wave per 4 coils)
  const bool regk = NDIM == 3 && pl->ktile.TS[0] == 8 && pl->ktile.TS[1] == 4 && pl->ktile.TS[2] == 8;
  const int kthreads = 64 * ((pl->C + 3) / 4);
  const size_t lds_used = regk ? sizeof(float2) * (size_t)kSpreadBatch * pl->C : lds;
  if (pl->ktile.TS[NDIM - 1] * pl->C > kthreads)  // the write-out takes at least one tile row per round
    throw HipError{hipErrorInvalidConfiguration, "k-space tile row longer than the spread workgroup"};
  auto k = regk ? kspread_reg_kernel<S> : kspread_kernel<NDIM, S>;
  allow_lds(k, lds);
  if (pl->ymax && n > kMaxPhasesPerLaunch)  // one spread-scale slot per state of a batch
    throw HipError{hipErrorInvalidValue, "k-space batch larger than the spread-scale slots"};
  for (int j0 = 0; j0 < n; j0 += kMaxPhasesPerLaunch) {
    const int nb = std::min(kMaxPhasesPerLaunch, n - j0);
    int64_t slots = 0;
    for (int i = 0; i < nb; ++i) slots += jobs[j0 + i].tr->nslots;
    if (slots) grow(pl, pl->partial, sizeof(float2) * volC * slots);
    KBatch<T> bt{};
    memset(&bt, 0, sizeof(bt));
    bt.n = nb;
    int64_t units = 0, splits = 0, slot0 = 0;
    for (int i = 0; i < nb; ++i) {
      const KJob& jb = jobs[j0 + i];
      bt.first[i] = (int)units;
      bt.units[i] = jb.tr->units;
      bt.taps[i] = jb.tr->taps_v;
      bt.yin[i] = jb.yin;
      bt.grid[i] = (T*)(jb.sgrid ? jb.sgrid : jb.grid);
      bt.partial[i] = (float2*)pl->partial.p + slot0 * volC;
      bt.dens[i] = jb.tr->dens;
      bt.fmask[i] = jb.tr->fmask;
      units += jb.tr->nunits;
      splits += jb.tr->nsplits;
      slot0 += jb.tr->nslots;
    }
    bt.first[nb] = (int)units;
    bt.blk = pl->blk_grid;
    bt.ymax = pl->ymax ? pl->ymax + (size_t)j0 * kYmaxSlots : nullptr;
    bt.tiled = NDIM == 3 && tiled_adjoint(pl);
    {
      Tick tick(pl, "kspread");
      hipLaunchKernelGGL(k, dim3((unsigned)units), dim3(kthreads), lds_used, pl->stream, bt, pl->C, pl->dims, pl->ktile,
                         pl->kb, make_fastdiv(pl->C));
      LAUNCH_OK();
    }
    if (splits) {
      int64_t s0 = 0;
      for (int i = 0; i < nb; ++i) {
        bt.first[i] = (int)s0;
        bt.splits[i] = jobs[j0 + i].tr->splits;
        s0 += jobs[j0 + i].tr->nsplits;
      }
      bt.first[nb] = (int)s0;
      Tick tick(pl, "kspread_reduce");
      hipLaunchKernelGGL((kspread_reduce_kernel<NDIM, S>), dim3((unsigned)splits), dim3(kGridThreads), 0, pl->stream,
                         bt, pl->C, pl->dims, pl->ktile);
      LAUNCH_OK();
    }
  }
}

template <int S>
static void kspread_t(isg_plan* pl, const KJob* jobs, int n) {
  if (pl->ndim == 3)
    kspread_nd<3, S>(pl, jobs, n);
  else
    kspread_nd<2, S>(pl, jobs, n);
}

#define STORAGE_DISPATCH(pl, fn, ...)                                  \
  do {                                                                 \
    switch ((pl)->storage) {                                           \
      case kBF16: fn<kBF16>(__VA_ARGS__); break;                       \
      case kFP16: fn<kFP16>(__VA_ARGS__); break;                       \
      default: fn<kFP32>(__VA_ARGS__); break;                          \
    }                                                                  \
  } while (0)

// data of one state in sample order -> spread-visit order (into yv); with
// half-precision grids also the largest |re|, |im| into batch slot `slot`
// (zeroed beforehand)
static float2* to_visit_order(isg_plan* pl, const isg_traj* tr, const float2* y, float2* yv, int slot,
                              const float* w = nullptr) {
  const int64_t n = tr->nvis * pl->C;
  if (n > 0) {
    Tick tick(pl, "visit_permute");
    hipLaunchKernelGGL(visit_permute_kernel, dim3(blocks_for(n, kGridThreads)), dim3(kGridThreads), 0, pl->stream, y,
                       tr->order, tr->nvis, pl->C, yv, pl->ymax ? pl->ymax + (size_t)slot * kYmaxSlots : nullptr,
                       tr->phase, w);
    LAUNCH_OK();
  }
  return yv;
}

// the scales the coil reduction of batch slot `slot` undoes (nothing for
// FP32 grids): the input scale of a normal-operator call when
// `input_scaled`, and the slot's spread-output scale
static HalfUndo half_undo(const isg_plan* pl, int slot, const isg_traj* tr, bool input_scaled) {
  HalfUndo u;
  if (!pl->ymax) return u;
  u.dsc = input_scaled ? pl->hsc + 1 : nullptr;
  u.ymax = pl->ymax + (size_t)slot * kYmaxSlots;
  u.dens = tr->dens;
  return u;
}

// Half-precision grids: sc = [1/rms(v), rms(v)] on the device, taken by the
// coil expansion (or the spread input) and undone by the coil reduction (or
// the gather output).  No-op for FP32 grids.
static void set_half_scale(isg_plan* pl, const float2* v, int64_t n) {
  if (!pl->hsc) return;
  const unsigned vb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, blocks_for(n, kVecThreads)));
  Tick tick(pl, "half_scale");
  hipLaunchKernelGGL(dot_partial_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, v, v, n, pl->hs_part);
  hipLaunchKernelGGL(half_scale_kernel, dim3(1), dim3(kVecThreads), 0, pl->stream, pl->hs_part, (int)vb, n, pl->hsc);
  LAUNCH_OK();
}

// scratch of the k-space stages for `nb` states processed together: their
// grids (kgrid, [nb][NG][C]) and their visit-ordered data (ybuf)
static void ensure_kspace(isg_plan* pl, int nb = 1, int64_t visits = 0, int64_t adj_tiles = 0) {
  const size_t es = pl->storage == kFP32 ? 8 : 4;  // grid elements
  const size_t ei = sizeof(float2);                  // intermediates: FP32 in every form
  const int64_t C = pl->C;
  if (!pl->k1buf) {
    if (pl->ndim == 3) {
      pl->k1buf = plan_alloc(pl, ei * (size_t)pl->n[0] * pl->n[1] * pl->G[2] * C);
      pl->k2buf = plan_alloc(pl, ei * (size_t)pl->n[0] * pl->G[1] * pl->G[2] * C);
    } else {
      pl->k1buf = plan_alloc(pl, ei * (size_t)pl->n[0] * pl->G[1] * C);
    }
    pl->wbuf = (float2*)plan_alloc(pl, sizeof(float2) * (size_t)pl->N * pl->P);
  }
  grow(pl, pl->kgrid, es * (size_t)pl->NG * C * (size_t)std::max(1, nb));
  grow(pl, pl->ybuf, sizeof(float2) * (size_t)std::max<int64_t>(1, visits) * C);
  if (adj_tiles > 0)
    grow(pl, pl->kgrid_adj, es * (size_t)adj_tiles * pl->ktile.vol * C * (size_t)std::max(1, nb));
}

static void* grid_of(const isg_plan* pl, int i) {
  const size_t es = pl->storage == kFP32 ? 8 : 4;
  return (char*)pl->kgrid.p + es * (size_t)pl->NG * pl->C * (size_t)i;
}

// tile-major spread output of batch member i (tiles: the largest touched-tile
// count of the call's states), or the member's grid when not tile-major
static void* sgrid_of(const isg_plan* pl, int i, int64_t tiles) {
  if (!tiled_adjoint(pl)) return grid_of(pl, i);
  const size_t es = pl->storage == kFP32 ? 8 : 4;
  return (char*)pl->kgrid_adj.p + es * (size_t)tiles * pl->ktile.vol * pl->C * (size_t)i;
}

static int64_t max_touched(const isg_traj* const* k, int P) {
  int64_t t = 1;
  for (int p = 0; p < P; ++p) t = std::max(t, k[p]->ntouched);
  return t;
}

// states per batch of the k-space stages
static int phase_batch(const isg_plan* pl, int P) { return std::max(1, std::min(P, pl->opt_phase_batch)); }

static int64_t group_visits(const isg_traj* const* k, int p0, int nb) {
  int64_t v = 0;
  for (int i = 0; i < nb; ++i) v += k[p0 + i]->nvis;
  return v;
}

// ---------------------------------------------------------------------------
// operator sequences.  States go in groups of phase_batch(); within a group
// the coil FFT passes run per state and the k-space gather and spread run
// as one launch over the group.
// ---------------------------------------------------------------------------
static void op_sense_forward(isg_plan* pl, int P, const float2* x, const isg_motion* const* d, const float2* S,
                             const isg_traj* const* k, float2* y) {
  const int B = phase_batch(pl, P);
  ensure_kspace(pl, B);
  set_half_scale(pl, x, pl->N);
  upsample(pl, x, pl->ugrid);
  int64_t off = 0;
  std::vector<KJob> jobs(B);
  for (int p0 = 0; p0 < P; p0 += B) {
    const int nb = std::min(B, P - p0);
    for (int i = 0; i < nb; ++i) {
      const int p = p0 + i;
      warp_gather(pl, pl->ugrid, d[p], pl->mbuf);
      STORAGE_DISPATCH(pl, coil_forward_t, pl, pl->mbuf, S, grid_of(pl, i), k[p]);
      jobs[i] = KJob{k[p], grid_of(pl, i), nullptr, y + off, nullptr};
      off += k[p]->M * pl->C;
    }
    STORAGE_DISPATCH(pl, kgather_t, pl, jobs.data(), nb, false, pl->hsc ? pl->hsc + 1 : nullptr);
  }
}

static void op_sense_adjoint(isg_plan* pl, int P, const float2* y, const isg_motion* const* d, const float2* S,
                             const isg_traj* const* k, float2* x) {
  const int B = phase_batch(pl, P);
  int64_t vmax = 1;
  for (int p0 = 0; p0 < P; p0 += B) vmax = std::max(vmax, group_visits(k, p0, std::min(B, P - p0)));
  const int64_t tiles = max_touched(k, P);
  ensure_kspace(pl, B, vmax, tiled_adjoint(pl) ? tiles : 0);
  std::vector<const float2*> w(P);
  std::vector<KJob> jobs(B);
  int64_t off = 0;
  for (int p0 = 0; p0 < P; p0 += B) {
    const int nb = std::min(B, P - p0);
    float2* yv = (float2*)pl->ybuf.p;
    if (pl->ymax) zero_ymax(pl, pl->ymax, nb);
    for (int i = 0; i < nb; ++i) {
      const int p = p0 + i;
      to_visit_order(pl, k[p], y + off, yv, i);
      jobs[i] = KJob{k[p], grid_of(pl, i), yv, nullptr, sgrid_of(pl, i, tiles)};
      yv += k[p]->nvis * pl->C;
      off += k[p]->M * pl->C;
    }
    STORAGE_DISPATCH(pl, kspread_t, pl, jobs.data(), nb);
    for (int i = 0; i < nb; ++i) {
      const int p = p0 + i;
      STORAGE_DISPATCH(pl, coil_adjoint_t, pl, sgrid_of(pl, i, tiles), S, pl->wbuf + (int64_t)p * pl->N, k[p],
                       half_undo(pl, i, k[p], false));
      w[p] = pl->wbuf + (int64_t)p * pl->N;
    }
  }
  warp_spread(pl, P, d, w.data(), pl->ugrid);
  upsample_adjoint(pl, pl->ugrid, x);
}

static void op_normal(isg_plan* pl, int P, const float2* x, double lam, const isg_motion* const* d, const float2* S,
                      const isg_traj* const* k, float2* out) {
  const int B = phase_batch(pl, P);
  int64_t vmax = 1;
  for (int p0 = 0; p0 < P; p0 += B) vmax = std::max(vmax, group_visits(k, p0, std::min(B, P - p0)));
  const int64_t tiles = max_touched(k, P);
  ensure_kspace(pl, B, vmax, tiled_adjoint(pl) ? tiles : 0);
  set_half_scale(pl, x, pl->N);
  upsample(pl, x, pl->ugrid);
  std::vector<const float2*> w(P);
  std::vector<KJob> jobs(B);
  for (int p0 = 0; p0 < P; p0 += B) {
    const int nb = std::min(B, P - p0);
    float2* yv = (float2*)pl->ybuf.p;
    for (int i = 0; i < nb; ++i) {
      const int p = p0 + i;
      warp_gather(pl, pl->ugrid, d[p], pl->mbuf);
      STORAGE_DISPATCH(pl, coil_forward_t, pl, pl->mbuf, S, grid_of(pl, i), k[p]);
      // gathered straight into visit order, spread from there
      jobs[i] = KJob{k[p], grid_of(pl, i), yv, yv, sgrid_of(pl, i, tiles)};
      yv += k[p]->nvis * pl->C;
    }
    STORAGE_DISPATCH(pl, kgather_t, pl, jobs.data(), nb, true);
    STORAGE_DISPATCH(pl, kspread_t, pl, jobs.data(), nb);
    for (int i = 0; i < nb; ++i) {
      const int p = p0 + i;
      STORAGE_DISPATCH(pl, coil_adjoint_t, pl, sgrid_of(pl, i, tiles), S, pl->wbuf + (int64_t)p * pl->N, k[p],
                       half_undo(pl, i, k[p], true));
      w[p] = pl->wbuf + (int64_t)p * pl->N;
    }
  }
  warp_spread(pl, P, d, w.data(), pl->ugrid);
  upsample_adjoint(pl, pl->ugrid, out);
  if (lam != 0.0) {
    Tick tick(pl, "axpy");
    hipLaunchKernelGGL(axpy_kernel, dim3(std::min<int64_t>(blocks_for(pl->N, kVecThreads), 4096)), dim3(kVecThreads),
                       0, pl->stream, out, x, (float)lam, pl->N);
    LAUNCH_OK();
  }
}

// ---------------------------------------------------------------------------
// plan-time preparation
// ---------------------------------------------------------------------------
static int iwrap(int64_t g, int G) {
  int64_t r = g % G;
  return (int)(r < 0 ? r + G : r);
}

// tiles (along one axis) touched by taps b..b+3 (mod G) with tile size TS;
// TS >= kWidth (or TS = G), so the taps reach at most two tiles
static int axis_tiles(int b, int G, int TS, int out[2]) {
  const int t0 = b / TS;
  const int e = b + kWidth - 1;
  const int t1 = (e >= G ? e - G : e) / TS;
  out[0] = t0;
  if (t1 != t0) {
    out[1] = t1;
    return 2;
  }
  return 1;
}

// Extent of a spread tile along an axis of G cells: the requested extent,
// capped at the largest power of two not above G/2.  Both spreads place a
// tap run relative to the tile origin at its nearest periodic image, the
// offset folded into (-G/2, G/2]; a run of W = 4 taps meets a tile of
// extent at most G/2 in one periodic image only, so the fold finds every
// in-tile tap.  A wider tile (e.g. 16 on an axis of 16, 20 or 24 cells)
// would lose the taps of runs that start past G/2 from its origin.
static int spread_extent(int want, int G) {
  int cap = 1;
  while (2 * cap <= G / 2) cap *= 2;
  return std::min(want, cap);
}

// Every voxel joins the one warp-spread tile that holds its first tap along
// every axis (the spread kernel recomputes the same tap base from d).  On the
// device, on the plan's stream: the key of every voxel and a check of the
// field, a stable radix sort of (tile, voxel) pairs (voxels stay in index
// order within a tile, so the spread sums in the same order on every call),
// and the tile offsets from the sorted keys.  Only the 4-byte check result
// comes back to the host.
static isg_status prepare_motion(isg_plan* pl, const float* d_dev, isg_motion* mo) {
  const int nd = pl->ndim;
  const int64_t N = pl->N;
  if (N >= ((int64_t)1 << 31)) return fail(ISG_ERR_UNSUPPORTED_SHAPE, "more than 2^31 voxels");
  const int ntiles = warp_ntiles(pl);
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) < ntiles) ++bits;
  size_t sort_bytes = 0;
  HIP_OK(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (int*)nullptr, (int*)nullptr, (int*)nullptr,
                                            (int*)nullptr, (int)N, 0, bits, pl->stream));
  const size_t ints = (size_t)std::max<int64_t>(N, 1);
  const size_t off_keys = 0, off_skeys = ints, off_vals = 2 * ints, off_bad = 3 * ints;
  const size_t tmp_at = ((off_bad + 1) * sizeof(int) + 255) & ~(size_t)255;
  grow(pl, pl->bin, tmp_at + sort_bytes + 256);
  int* base = (int*)pl->bin.p;
  int *keys = base + off_keys, *skeys = base + off_skeys, *vals = base + off_vals, *bad = base + off_bad;
  void* tmp = (char*)pl->bin.p + tmp_at;
  mo->d = (float*)dmalloc(pl, sizeof(float) * (size_t)nd * N);
  mo->tile_off = (int*)dmalloc(pl, sizeof(int) * ((size_t)ntiles + 1));
  mo->vox = (int*)dmalloc(pl, sizeof(int) * ints);
  mo->nentries = N;
  HIP_OK(hipMemcpyAsync(mo->d, d_dev, sizeof(float) * (size_t)nd * N, hipMemcpyDeviceToDevice, pl->stream));
  hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, pl->stream, bad, (int64_t)1, 0);
  const unsigned kb = (unsigned)std::min<int64_t>(blocks_for(N, 256), 8192);
  const int* nt = pl->wtile.nt;
  const int* lg = pl->wtile.lg;
  if (nd == 3)
    hipLaunchKernelGGL(motion_key_kernel<3>, dim3(kb), dim3(256), 0, pl->stream, mo->d, N, pl->n[0], pl->n[1],
                       pl->n[2], pl->G[0], pl->G[1], pl->G[2], nt[0], nt[1], nt[2], lg[0], lg[1], lg[2], keys, vals,
                       bad);
  else
    hipLaunchKernelGGL(motion_key_kernel<2>, dim3(kb), dim3(256), 0, pl->stream, mo->d, N, pl->n[0], pl->n[1], 1,
                       pl->G[0], pl->G[1], 1, nt[0], nt[1], 1, lg[0], lg[1], 0, keys, vals, bad);
  LAUNCH_OK();
  HIP_OK(hipcub::DeviceRadixSort::SortPairs(tmp, sort_bytes, keys, skeys, vals, mo->vox, (int)N, 0, bits,
                                            pl->stream));
  hipLaunchKernelGGL(tile_offsets_kernel, dim3((unsigned)std::min<int64_t>(blocks_for(N + 1, 256), 8192)), dim3(256),
                     0, pl->stream, skeys, N, ntiles, mo->tile_off);
  LAUNCH_OK();
  int flags = 0;
  HIP_OK(hipMemcpyAsync(&flags, bad, sizeof(int), hipMemcpyDeviceToHost, pl->stream));
  HIP_OK(hipStreamSynchronize(pl->stream));
  if (flags & kFieldNotFinite) return fail(ISG_ERR_NOT_FINITE, "displacement field holds NaN or Inf");
  if (flags & kFieldTooLarge) return fail(ISG_ERR_INVALID_ARG, "displacement magnitude exceeds 1e6 voxels");
  return ISG_OK;
}

static bool fft2_supported(int L);
// untouched-tile skipping needs the two-step FFT on axis 0 and at most 64
// tiles along it (one 64-bit mask per tile column)
// k-space spread tiles with extent t1 along axis 1 (3D: 8 along axes 0 and 2,
// 4 along axis 0 for more than 16 coils to bound the LDS accumulator; 2D:
// 16 along axis 0)
static void set_ktile(isg_plan* pl, int t1) {
  for (int i = 0; i < 3; ++i) {
    pl->ktile.TS[i] = 1;
    pl->ktile.nt[i] = 1;
  }
  if (pl->ndim == 3) {
    const int ts[3] = {pl->C > 16 ? 4 : 8, t1, 8};
    for (int i = 0; i < 3; ++i) pl->ktile.TS[i] = spread_extent(ts[i], pl->G[i]);
  } else {
    const int ts[2] = {16, t1};
    for (int i = 0; i < 2; ++i) pl->ktile.TS[i] = spread_extent(ts[i], pl->G[i]);
  }
  for (int i = 0; i < pl->ndim; ++i)  // tap runs reach at most two tiles per axis (axis_tiles)
    if (pl->ktile.TS[i] < kWidth && pl->ktile.TS[i] < pl->G[i])
      throw HipError{hipErrorInvalidConfiguration, "k-space tiles narrower than the kernel"};
  pl->ktile.vol = 1;
  for (int i = 0; i < pl->ndim; ++i) {
    pl->ktile.nt[i] = (pl->G[i] + pl->ktile.TS[i] - 1) / pl->ktile.TS[i];
    pl->ktile.vol *= pl->ktile.TS[i];
  }
  // dense planes of complex values; plane size = 4 (mod 16) puts the four
  // coils of a spread wave on distinct banks
  if (pl->ndim == 3) {
    pl->ktile.S1 = pl->ktile.TS[2];
    pl->ktile.S0 = pl->ktile.TS[1] * pl->ktile.TS[2];
  } else {
    pl->ktile.S1 = 1;
    pl->ktile.S0 = pl->ktile.TS[1];
  }
  int P = pl->ktile.TS[0] * pl->ktile.S0;
  while (P % 16 != 4) ++P;
  pl->ktile.P = P;
  pl->ktile.rowdiv = make_fastdiv((uint32_t)(pl->ktile.TS[pl->ndim - 1] * pl->C));
  pl->opt_ktile_t1 = t1;
}

// Layouts of the coil-expanded grid [G0][G1][G2][C] and of k2buf
// [n0][G1][G2][C]: row-blocked in blocks of 2^opt_blk_tlog values of i1 on the
// 3D register-FFT path (the axis-0 passes then step T G2 C elements instead
// of G1 G2 C and touch far fewer translation pages), plain row-major
// elsewhere or when the block does not divide G1.
static void set_layouts(isg_plan* pl) {
  auto make = [&](int64_t rows, int tlog, int64_t g2c) {
    Blk b;
    b.g2c = g2c;
    b.g2cdiv = make_fastdiv((uint32_t)g2c);
    if (tlog < 30) {
      b.tlog = tlog;
      b.rs = ((int64_t)1 << tlog) * g2c;
      b.bs = rows * b.rs;
    } else {
      b.tlog = 30;
      b.rs = (int64_t)pl->G[1] * g2c;
      b.bs = 0;
    }
    return b;
  };
  const bool fast3 = pl->ndim == 3 && fft2_supported(pl->G[0]) && fft2_supported(pl->G[1]) && fft2_supported(pl->G[2]);
  int tlog = 30;
  if (fast3 && pl->opt_blk_tlog < 30 && pl->G[1] % (1 << pl->opt_blk_tlog) == 0) tlog = pl->opt_blk_tlog;
  const int64_t g2c = (int64_t)(pl->ndim == 3 ? pl->G[2] : 1) * pl->C;
  pl->blk_grid = make(pl->G[0], tlog, g2c);
  pl->blk_k2 = make(pl->n[0], tlog, g2c);
}

static bool traj_masked(const isg_plan* pl) {
  const char* e = getenv("ISG_NO_TILE_MASK");
  if (e && atoi(e)) return false;
  int ts = pl->ktile.TS[0], lg = 0;
  while ((1 << lg) < ts) ++lg;
  return fft2_supported(pl->G[0]) && pl->ktile.nt[0] <= 64 && (1 << lg) == ts &&
         (pl->ndim == 2 || (fft2_supported(pl->G[1]) && fft2_supported(pl->G[2]))) &&
         (pl->ndim == 3 || fft2_supported(pl->G[1]));
}


// Spread work units of a prepared trajectory for the plan's chunk size:
// one unit per touched tile, or (tiles with more than `chunk` visits) one
// unit per chunk writing a partial tile, summed afterwards in slot order.
// Untouched tiles get no unit when the axis-0 passes skip them, else a unit
// that writes zeros.  Units are ordered longest first.
// The spread output is stored tile-major (touched tiles only, each tile
// contiguous, columns in order) on the 3D register-FFT path with masks; the
// adjoint axis-0 pass then reads each column's rows from consecutive tiles.
static bool tiled_adjoint(const isg_plan* pl) { return pl->ndim == 3 && traj_masked(pl); }

// slot of tile t in the tile-major spread output of trajectory tr
static int tile_gslot(const isg_plan* pl, const isg_traj* tr, int t) {
  if (!tiled_adjoint(pl)) return -1;
  const int ncols = pl->ktile.nt[1] * pl->ktile.nt[2];
  const int t0 = t / ncols, col = t - t0 * ncols;
  const uint64_t below = tr->colmask_h[col] & ((1ull << t0) - 1ull);
  return tr->colbase_h[col] + __builtin_popcountll(below);
}

static void build_units(isg_plan* pl, isg_traj* tr) {
  const int chunk = pl->opt_spread_chunk;
  const bool masked = traj_masked(pl);
  const std::vector<int>& cnt = tr->tile_first;
  const int ntiles = (int)cnt.size() - 1;
  std::vector<KUnit> units;
  std::vector<KSplit> splits;
  int slots = 0;
  const bool rows = tr->tile_rows.size() == 2 * (size_t)ntiles;
  // a unit covering visits [off, off + n) of its tile: its row-class bounds
  auto unit = [&](int t, int off, int n, int slot, int gs) {
    KUnit u{t, cnt[t] + off, n, slot, gs, 0, 0};
    if (rows) {
      const int lo = tr->tile_rows[2 * t], hi = tr->tile_rows[2 * t + 1];
      u.lo = std::min(std::max(lo - off, 0), n);
      u.lohi = std::min(std::max(lo + hi - off, 0), n);
    }
    return u;
  };
  for (int t = 0; t < ntiles; ++t) {
    const int c = cnt[t + 1] - cnt[t];
    if (c == 0 && masked) continue;
    const int gs = c > 0 ? tile_gslot(pl, tr, t) : -1;
    if (c <= chunk) {
      units.push_back(unit(t, 0, c, -1, gs));
    } else {
      const int nch = (c + chunk - 1) / chunk;
      splits.push_back(KSplit{t, slots, nch, gs});
      for (int q = 0; q < nch; ++q) units.push_back(unit(t, q * chunk, std::min(chunk, c - q * chunk), slots + q, gs));
      slots += nch;
    }
  }
  std::stable_sort(units.begin(), units.end(), [](const KUnit& a, const KUnit& b) { return a.count > b.count; });
  if (units.empty()) units.push_back(KUnit{0, 0, 0, -1, -1, 0, 0});  // keep the launch non-empty
  HIP_OK(hipStreamSynchronize(pl->stream));
  pl->generation++;
  HIP_OK(dfree(pl, tr->units));
  HIP_OK(dfree(pl, tr->splits));
  tr->units = nullptr;
  tr->splits = nullptr;
  tr->units = (KUnit*)dmalloc(pl, sizeof(KUnit) * units.size());
  tr->nunits = (int)units.size();
  tr->splits = (KSplit*)dmalloc(pl, sizeof(KSplit) * std::max<size_t>(1, splits.size()));
  tr->nsplits = (int)splits.size();
  tr->nslots = slots;
  tr->chunk = chunk;
  HIP_OK(hipMemcpy(tr->units, units.data(), sizeof(KUnit) * units.size(), hipMemcpyHostToDevice));
  if (!splits.empty())
    HIP_OK(hipMemcpy(tr->splits, splits.data(), sizeof(KSplit) * splits.size(), hipMemcpyHostToDevice));
}

// free a device array of a trajectory (its memory leaves the plan's count)
static void traj_free(isg_plan* pl, void*& p) {
  if (p) {
    HIP_OK(dfree(pl, p));
    p = nullptr;
  }
}

// Tile bookkeeping of a trajectory for the plan's current k-space tile
// shape: the tile-sorted visit order, touched-tile masks, visit-ordered taps,
// each sample's visit list and the spread work units.
static void bin_traj(isg_plan* pl, isg_traj* tr) {
  const int nd = pl->ndim;
  const int64_t M = tr->M;
  const std::vector<KTap>& taps = tr->taps_h;
  HIP_OK(hipStreamSynchronize(pl->stream));
  pl->generation++;
  for (void** q : {(void**)&tr->order, (void**)&tr->gorder, (void**)&tr->colmask, (void**)&tr->fmask,
                   (void**)&tr->cact, (void**)&tr->colbase, (void**)&tr->taps_v, (void**)&tr->vis_off,
                   (void**)&tr->vis})
    traj_free(pl, *q);
  tr->cact_w = 0;
  tr->fine_cells = 0;
  tr->active_cols = 0;
  tr->colmask_h.clear();
  tr->colbase_h.clear();
  int ntiles = 1;
  for (int i = 0; i < nd; ++i) ntiles *= pl->ktile.nt[i];
  std::vector<int> cnt(ntiles + 1, 0);
  auto visit = [&](int64_t j, auto&& fn) {
    int ts[3][2], nts[3] = {1, 1, 1};
    for (int i = 0; i < nd; ++i) {
      const int b = (int)((taps[j].base >> (10 * i)) & 1023);
      nts[i] = axis_tiles(b, pl->G[i], pl->ktile.TS[i], ts[i]);
    }
    if (nd == 3) {
      for (int a = 0; a < nts[0]; ++a)
        for (int b = 0; b < nts[1]; ++b)
          for (int c = 0; c < nts[2]; ++c)
            fn((ts[0][a] * pl->ktile.nt[1] + ts[1][b]) * pl->ktile.nt[2] + ts[2][c]);
    } else {
      for (int a = 0; a < nts[0]; ++a)
        for (int b = 0; b < nts[1]; ++b) fn(ts[0][a] * pl->ktile.nt[1] + ts[1][b]);
    }
  };
  for (int64_t j = 0; j < M; ++j) visit(j, [&](int t) { cnt[t + 1]++; });
  for (int t = 0; t < ntiles; ++t) cnt[t + 1] += cnt[t];
  std::vector<int> pos(cnt.begin(), cnt.end() - 1);
  std::vector<int> order(std::max(1, cnt[ntiles]));
  for (int64_t j = 0; j < M; ++j) visit(j, [&](int t) { order[pos[t]++] = (int)j; });
  // for the register spread (8 x 4 x 8 tiles): each tile's visits by the
  // rows of the tile their axis-0 taps reach (0-3 only, 4-7 only, both),
  // sample order within a class; the row of the first tap is formed as the
  // spread forms it (periodic offset from the tile origin)
  tr->tile_rows.clear();
  if (nd == 3 && pl->ktile.TS[0] == 8 && pl->ktile.TS[1] == 4 && pl->ktile.TS[2] == 8) {
    tr->tile_rows.assign(2 * (size_t)ntiles, 0);
    const int plane = pl->ktile.nt[1] * pl->ktile.nt[2], G0 = pl->G[0];
    std::vector<int> part;
    for (int t = 0; t < ntiles; ++t) {
      const int beg = cnt[t], n = cnt[t + 1] - cnt[t];
      if (n == 0) continue;
      part.assign(order.begin() + beg, order.begin() + beg + n);
      auto cls = [&](int j) {
        int o = (int)(taps[j].base & 1023) - (t / plane) * 8;
        if (o > G0 / 2) o -= G0;
        if (o < -G0 / 2) o += G0;
        return o <= 0 ? 0 : (o >= 4 ? 1 : 2);
      };
      int w = beg;
      for (int c = 0; c < 3; ++c) {
        const int w0 = w;
        for (int j : part)
          if (cls(j) == c) order[w++] = j;
        if (c < 2) tr->tile_rows[2 * (size_t)t + c] = w - w0;
      }
    }
  }
  tr->ntouched = 0;
  for (int t = 0; t < ntiles; ++t)
    if (cnt[t + 1] > cnt[t]) tr->ntouched++;
  if (traj_masked(pl)) {
    const int ncols = nd == 3 ? pl->ktile.nt[1] * pl->ktile.nt[2] : pl->ktile.nt[1];
    std::vector<uint64_t> cm(ncols, 0ull);
    for (int t = 0; t < ntiles; ++t) {
      if (cnt[t + 1] == cnt[t]) continue;
      const int t0 = t / ncols, col = t - t0 * ncols;
      cm[col] |= 1ull << t0;
    }
    tr->colmask = (uint64_t*)dmalloc(pl, sizeof(uint64_t) * ncols);
    HIP_OK(hipMemcpy(tr->colmask, cm.data(), sizeof(uint64_t) * ncols, hipMemcpyHostToDevice));
    tr->colmask_h = cm;
    tr->colbase_h.assign(ncols, 0);
    int base = 0;
    for (int col = 0; col < ncols; ++col) {
      tr->colbase_h[col] = base;
      base += __builtin_popcountll(cm[col]);
    }
    tr->colbase = (int*)dmalloc(pl, sizeof(int) * ncols);
    HIP_OK(hipMemcpy(tr->colbase, tr->colbase_h.data(), sizeof(int) * ncols, hipMemcpyHostToDevice));
    // touched runs of 2^lg cells along axis 0, per grid column (i1, i2)
    int lg = 0;
    while ((1 << lg) < pl->ktile.TS[0]) ++lg;
    const int G0 = pl->G[0], G1 = pl->G[1], G2 = nd == 3 ? pl->G[2] : 1;
    std::vector<uint64_t> fm((size_t)G1 * G2, 0ull);
    for (int64_t j = 0; j < M; ++j) {
      const int b0 = (int)(taps[j].base & 1023), b1 = (int)((taps[j].base >> 10) & 1023);
      const int b2 = nd == 3 ? (int)((taps[j].base >> 20) & 1023) : 0;
      const int e0 = b0 + kWidth - 1;
      const uint64_t bits = (1ull << (b0 >> lg)) | (1ull << ((e0 >= G0 ? e0 - G0 : e0) >> lg));
      for (int t1 = 0; t1 < kWidth; ++t1) {
        const int i1 = b1 + t1 >= G1 ? b1 + t1 - G1 : b1 + t1;
        if (nd == 3) {
          for (int t2 = 0; t2 < kWidth; ++t2) {
            const int i2 = b2 + t2 >= G2 ? b2 + t2 - G2 : b2 + t2;
            fm[(size_t)i1 * G2 + i2] |= bits;
          }
        } else {
          fm[(size_t)i1] |= bits;
        }
      }
    }
    int64_t runs = 0;
    for (uint64_t m : fm) {
      runs += __builtin_popcountll(m);
      tr->active_cols += m != 0;
    }
    tr->fine_cells = runs * (1 << lg);  // ragged last runs counted whole
    tr->fmask = (uint64_t*)dmalloc(pl, sizeof(uint64_t) * fm.size());
    HIP_OK(hipMemcpy(tr->fmask, fm.data(), sizeof(uint64_t) * fm.size(), hipMemcpyHostToDevice));
    if (nd == 3 && G1 <= 64 * kColWords) {  // the touched grid columns, transposed for the axis-1 passes
      const int W = (G1 + 63) / 64;
      std::vector<uint64_t> ca((size_t)G2 * W, 0ull);
      for (int i1 = 0; i1 < G1; ++i1)
        for (int i2 = 0; i2 < G2; ++i2)
          if (fm[(size_t)i1 * G2 + i2]) ca[(size_t)i2 * W + (i1 >> 6)] |= 1ull << (i1 & 63);
      tr->cact = (uint64_t*)dmalloc(pl, sizeof(uint64_t) * ca.size());
      tr->cact_w = W;
      HIP_OK(hipMemcpy(tr->cact, ca.data(), sizeof(uint64_t) * ca.size(), hipMemcpyHostToDevice));
    }
  }
  tr->order = (int*)dmalloc(pl, sizeof(int) * order.size());
  HIP_OK(hipMemcpy(tr->order, order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice));
  {  // gather order: samples by the first tile they visit, index order within a tile
    std::vector<int> gcnt(ntiles + 1, 0), first(std::max<int64_t>(1, M));
    for (int64_t j = 0; j < M; ++j) {
      bool seen = false;
      visit(j, [&](int t) {
        if (!seen) first[j] = t;
        seen = true;
      });
      gcnt[first[j] + 1]++;
    }
    for (int t = 0; t < ntiles; ++t) gcnt[t + 1] += gcnt[t];
    std::vector<int> go(std::max<int64_t>(1, M));
    for (int64_t j = 0; j < M; ++j) go[gcnt[first[j]]++] = (int)j;
    tr->gorder = (int*)dmalloc(pl, sizeof(int) * go.size());
    HIP_OK(hipMemcpy(tr->gorder, go.data(), sizeof(int) * go.size(), hipMemcpyHostToDevice));
  }
  {  // visit-ordered taps and, per sample, the list of its visits
    const int64_t nvis = cnt[ntiles];
    std::vector<KTap> tv(std::max<int64_t>(1, nvis));
    std::vector<int> voff(M + 1, 0), vlist(std::max<int64_t>(1, nvis));
    for (int64_t v = 0; v < nvis; ++v) {
      tv[v] = taps[order[v]];
      voff[order[v] + 1]++;
    }
    for (int64_t j = 0; j < M; ++j) voff[j + 1] += voff[j];
    std::vector<int> vp(voff.begin(), voff.end() - 1);
    for (int64_t v = 0; v < nvis; ++v) vlist[vp[order[v]]++] = (int)v;
    tr->nvis = nvis;
    tr->taps_v = (KTap*)dmalloc(pl, sizeof(KTap) * tv.size());
    tr->vis_off = (int*)dmalloc(pl, sizeof(int) * voff.size());
    tr->vis = (int*)dmalloc(pl, sizeof(int) * vlist.size());
    HIP_OK(hipMemcpy(tr->taps_v, tv.data(), sizeof(KTap) * tv.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(tr->vis_off, voff.data(), sizeof(int) * voff.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(tr->vis, vlist.data(), sizeof(int) * vlist.size(), hipMemcpyHostToDevice));
  }
  tr->tile_first = cnt;
  for (int i = 0; i < 3; ++i) tr->ts[i] = pl->ktile.TS[i];
  build_units(pl, tr);
}

static isg_status prepare_traj(isg_plan* pl, const float* k_dev, int64_t M, isg_traj* tr) {
  const int nd = pl->ndim;
  std::vector<float> k((size_t)M * nd);
  HIP_OK(hipMemcpy(k.data(), k_dev, sizeof(float) * k.size(), hipMemcpyDeviceToHost));
  for (float v : k) {
    if (!std::isfinite(v)) return fail(ISG_ERR_NOT_FINITE, "trajectory holds NaN or Inf");
    if (std::fabs(v) > 1.0e6f) return fail(ISG_ERR_INVALID_ARG, "trajectory magnitude exceeds 1e6 cycles/voxel");
  }
  std::vector<KTap>& taps = tr->taps_h;
  taps.resize(M);
  for (int64_t j = 0; j < M; ++j) {
    KTap t;
    t.f[0] = t.f[1] = t.f[2] = 0.f;
    uint32_t packed = 0;
    for (int i = 0; i < nd; ++i) {
      const double kap = (double)pl->G[i] * (double)k[(size_t)j * nd + i];  // exact in FP64
      const double fl = std::floor(kap);
      float f = (float)(kap - fl);
      // a fraction just below 1 can round up to 1 in FP32.  The taps stay
      // those of the FP64 cell and the fraction is clamped below 1: moving
      // to the next cell instead would drop the first tap, whose weight is
      // the kernel's non-zero edge value just inside its open support.
      if (f >= 1.0f) f = 0.99999994f;
      t.f[i] = f;
      packed |= (uint32_t)iwrap((int64_t)fl - 1, pl->G[i]) << (10 * i);
    }
    t.base = packed;
    taps[j] = t;
  }
  // dens: a bound on the samples whose kernel support reaches one grid cell,
  // the largest number reaching one block of 8 cells per axis (scales the
  // half-precision spread output; independent of the spread tile shape)
  {
    int nbk[3] = {1, 1, 1};
    int64_t nblocks = 1;
    for (int i = 0; i < nd; ++i) {
      nbk[i] = (pl->G[i] + 7) / 8;
      nblocks *= nbk[i];
    }
    std::vector<int> cnt((size_t)nblocks, 0);
    int best = 0;
    for (int64_t j = 0; j < M; ++j) {
      int bs[3][2] = {{0, 0}, {0, 0}, {0, 0}}, nbs[3] = {1, 1, 1};
      for (int i = 0; i < nd; ++i) nbs[i] = axis_tiles((int)((taps[j].base >> (10 * i)) & 1023), pl->G[i], 8, bs[i]);
      for (int a = 0; a < nbs[0]; ++a)
        for (int b = 0; b < nbs[1]; ++b)
          for (int c = 0; c < nbs[2]; ++c)
            best = std::max(best, ++cnt[((size_t)bs[0][a] * nbk[1] + bs[1][b]) * nbk[2] + bs[2][c]]);
    }
    tr->dens = (float)std::max(1, best);
  }
  tr->M = M;
  tr->taps = (KTap*)dmalloc(pl, sizeof(KTap) * taps.size());
  HIP_OK(hipMemcpy(tr->taps, taps.data(), sizeof(KTap) * taps.size(), hipMemcpyHostToDevice));
  tr->k = (float*)dmalloc(pl, sizeof(float) * k.size());
  HIP_OK(hipMemcpy(tr->k, k.data(), sizeof(float) * k.size(), hipMemcpyHostToDevice));
  bin_traj(pl, tr);
  return ISG_OK;
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
static bool good_length(int64_t n) {
  if (n < 8 || n > 512 || (n & 1)) return false;
  std::vector<int> R;
  return factor_radices((int)n, R) && factor_radices((int)(2 * n), R);
}

static isg_status check_plan(const isg_plan* pl) {
  if (!pl) return fail(ISG_ERR_INVALID_ARG, "plan is NULL");
  if (pl->failed) return fail(ISG_ERR_STATE, "plan hit a device error earlier; destroy it");
  return ISG_OK;
}

static isg_status check_phases(const isg_plan* pl, int P, const isg_motion* const* d, const isg_traj* const* k) {
  if (P < 1 || P > pl->P) return fail(ISG_ERR_INVALID_ARG, "nphases must be in 1..plan nphases");
  if (!d || !k) return fail(ISG_ERR_INVALID_ARG, "motion / trajectory arrays must not be NULL");
  for (int p = 0; p < P; ++p) {
    if (!d[p] || !k[p]) return fail(ISG_ERR_INVALID_ARG, "NULL motion or trajectory handle");
    if (d[p]->plan != pl || k[p]->plan != pl) return fail(ISG_ERR_INVALID_ARG, "handle belongs to another plan");
    for (int i = 0; i < 3; ++i)
      if (k[p]->ts[i] != pl->ktile.TS[i])
        return fail(ISG_ERR_STATE, "trajectory was prepared for another k-space tile shape: re-create it or run "
                                   "isg_plan_tune with it");
  }
  return ISG_OK;
}

static isg_status device_error(isg_plan* pl, const HipError& e) {
  if (pl) pl->failed = true;
  return fail(ISG_ERR_DEVICE, std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.where);
}

template <class F>
static isg_status guarded(isg_plan* pl, F&& f) {
  try {
    return f();
  } catch (const HipError& e) {
    return device_error(pl, e);
  } catch (const std::bad_alloc&) {
    return fail(ISG_ERR_OUT_OF_MEMORY, "device or host allocation failed");
  }
}

// ---------------------------------------------------------------------------
// graph replay of the normal operator and the autotuner
// ---------------------------------------------------------------------------
static void drop_normal_graph(isg_plan* pl) {
  if (pl->ngraph.exec) (void)hipGraphExecDestroy(pl->ngraph.exec);
  if (pl->ngraph.graph) (void)hipGraphDestroy(pl->ngraph.graph);
  pl->ngraph = isg_plan::NormalGraph{};
}

// op_normal, replayed from a captured graph when ISG_OPT_GRAPH is set and the
// arguments, the stream and every buffer the graph references are unchanged
// since the capture.  A call with new arguments runs eagerly (growing any
// buffer it needs) and then captures the sequence for the next call.
static void normal_maybe_graph(isg_plan* pl, int P, const float2* x, double lam, const isg_motion* const* d,
                               const float2* S, const isg_traj* const* k, float2* out) {
  if (!pl->opt_graph || pl->stream == nullptr || pl->timing) {
    op_normal(pl, P, x, lam, d, S, k, out);
    return;
  }
  std::vector<const void*> key = {(const void*)pl->stream, x, S, out, (const void*)(uintptr_t)P};
  for (int p = 0; p < P; ++p) {
    key.push_back(d[p]);
    key.push_back(k[p]);
  }
  key.push_back((const void*)(uintptr_t)pl->generation);
  if (pl->ngraph.exec && pl->ngraph.key == key && pl->ngraph.lam == lam) {
    HIP_OK(hipGraphLaunch(pl->ngraph.exec, pl->stream));
    return;
  }
  drop_normal_graph(pl);
  op_normal(pl, P, x, lam, d, S, k, out);
  const uint64_t gen = pl->generation;
  hipGraph_t graph = nullptr;
  HIP_OK(hipStreamBeginCapture(pl->stream, hipStreamCaptureModeThreadLocal));
  pl->capturing = true;
  try {
    op_normal(pl, P, x, lam, d, S, k, out);
  } catch (...) {
    pl->capturing = false;
    hipGraph_t g2 = nullptr;
    (void)hipStreamEndCapture(pl->stream, &g2);
    if (g2) (void)hipGraphDestroy(g2);
    throw;
  }
  pl->capturing = false;
  HIP_OK(hipStreamEndCapture(pl->stream, &graph));
  if (pl->generation != gen) {  // a buffer moved while capturing: do not keep the graph
    (void)hipGraphDestroy(graph);
    return;
  }
  hipGraphExec_t exec = nullptr;
  HIP_OK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  pl->ngraph.graph = graph;
  pl->ngraph.exec = exec;
  pl->ngraph.key = key;
  pl->ngraph.lam = lam;
}

// best of `reps` timed normal-operator applications (ms), after one warm-up
static double time_normal(isg_plan* pl, int P, const float2* x, double lam, const isg_motion* const* d,
                          const float2* S, const isg_traj* const* k, float2* out, int reps) {
  normal_maybe_graph(pl, P, x, lam, d, S, k, out);  // warm-up (and capture)
  hipEvent_t a, b;
  HIP_OK(hipEventCreate(&a));
  HIP_OK(hipEventCreate(&b));
  double best = 1e30;
  for (int r = 0; r < reps; ++r) {
    HIP_OK(hipEventRecord(a, pl->stream));
    normal_maybe_graph(pl, P, x, lam, d, S, k, out);
    HIP_OK(hipEventRecord(b, pl->stream));
    HIP_OK(hipEventSynchronize(b));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, a, b));
    best = std::min(best, (double)ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

static isg_status tune(isg_plan* pl, int P, const float2* x, const isg_motion* const* d, const float2* S,
                       isg_traj* const* k, double lam, int reps, char* report, int64_t len) {
  if (pl->timing) return fail(ISG_ERR_INVALID_ARG, "disable timing before tuning");
  grow(pl, pl->tune_out, sizeof(float2) * (size_t)pl->N);
  float2* out = (float2*)pl->tune_out.p;
  const isg_traj* const* kc = (const isg_traj* const*)k;
  struct Cand {
    int kb, t1, chunk, batch, graph;
    double ms;
  };
  std::vector<Cand> tried;
  auto apply = [&](int kb, int t1, int chunk, int batch, int graph) {
    const bool retile = t1 != pl->opt_ktile_t1;
    HIP_OK(hipStreamSynchronize(pl->stream));
    if (retile) set_ktile(pl, t1);
    pl->opt_blk_tlog = kb == 0 ? 30 : kb;
    set_layouts(pl);
    pl->opt_spread_chunk = chunk;
    pl->opt_phase_batch = batch;
    pl->opt_graph = graph;
    pl->generation++;
    for (int p = 0; p < P; ++p) {
      if (retile || k[p]->ts[1] != pl->ktile.TS[1])
        bin_traj(pl, k[p]);
      else if (k[p]->chunk != chunk)
        build_units(pl, k[p]);
    }
  };
  auto measure = [&](int kb, int t1, int chunk, int batch, int graph) -> double {
    apply(kb, t1, chunk, batch, graph);
    double ms = 1e30;
    try {
      ms = time_normal(pl, P, x, lam, d, S, kc, out, reps);
    } catch (const std::bad_alloc&) {
      ms = 1e30;  // does not fit: skipped
    }
    tried.push_back(Cand{kb, t1, chunk, batch, graph, ms});
    return ms;
  };
  // coordinate search: k-space array blocking, tile extent, chunk (batch 1,
  // no graph), batch, graph
  const std::vector<int> t1s = pl->ndim == 3 ? std::vector<int>{8, 4} : std::vector<int>{16, 8};
  int best_kb = 0, best_t1 = t1s[0], best_chunk = 512, best_batch = 1, best_graph = 0;
  double best = 1e30;
  const std::vector<int> kbs = pl->ndim == 3 ? std::vector<int>{3, 2, 1, 4, 0} : std::vector<int>{0};
  for (int kb : kbs) {
    const double ms = measure(kb, t1s[0], 512, 1, 0);
    if (ms < best) {
      best = ms;
      best_kb = kb;
    }
  }
  for (int t1 : t1s) {
    if (t1 == t1s[0]) continue;
    const double ms = measure(best_kb, t1, 512, 1, 0);
    if (ms < best) {
      best = ms;
      best_t1 = t1;
    }
  }
  for (int c : {256, 1024, 2048}) {
    const double ms = measure(best_kb, best_t1, c, 1, 0);
    if (ms < best) {
      best = ms;
      best_chunk = c;
    }
  }
  std::vector<int> batches;
  for (int b : {2, 3, 4, 6, 8, 16})
    if (b <= std::min(P, kMaxPhasesPerLaunch)) batches.push_back(b);
  if (P > 1 && P <= kMaxPhasesPerLaunch && std::find(batches.begin(), batches.end(), P) == batches.end())
    batches.push_back(P);
  for (int b : batches) {
    const double ms = measure(best_kb, best_t1, best_chunk, b, 0);
    if (ms < best) {
      best = ms;
      best_batch = b;
    }
  }
  if (pl->stream != nullptr) {
    const double ms = measure(best_kb, best_t1, best_chunk, best_batch, 1);
    if (ms < best) {
      best = ms;
      best_graph = 1;
    }
  }
  // the blockings next to the chosen one again, with the other options
  // chosen (the first comparison ran with the defaults)
  if (pl->ndim == 3 && best_kb > 0) {
    const int kb0 = best_kb;
    for (int kb : {kb0 - 1, kb0 + 1}) {
      if (kb < 1 || kb > 4) continue;
      const double ms = measure(kb, best_t1, best_chunk, best_batch, best_graph);
      if (ms < best) {
        best = ms;
        best_kb = kb;
      }
    }
  }
  apply(best_kb, best_t1, best_chunk, best_batch, best_graph);
  drop_normal_graph(pl);
  HIP_OK(hipStreamSynchronize(pl->stream));
  if (report && len > 0) {
    std::string js = "{\"candidates\": [";
    char buf[160];
    for (size_t i = 0; i < tried.size(); ++i) {
      const Cand& c = tried[i];
      if (c.ms >= 1e29)
        snprintf(buf, sizeof(buf),
                 "%s{\"kblock\": %d, \"ktile_t1\": %d, \"chunk\": %d, \"batch\": %d, \"graph\": %d, \"ms\": null}",
                 i ? ", " : "", c.kb, c.t1, c.chunk, c.batch, c.graph);
      else
        snprintf(buf, sizeof(buf),
                 "%s{\"kblock\": %d, \"ktile_t1\": %d, \"chunk\": %d, \"batch\": %d, \"graph\": %d, \"ms\": %.4f}",
                 i ? ", " : "", c.kb, c.t1, c.chunk, c.batch, c.graph, c.ms);
      js += buf;
    }
    snprintf(buf, sizeof(buf),
             "], \"chosen\": {\"kblock\": %d, \"ktile_t1\": %d, \"chunk\": %d, \"batch\": %d, \"graph\": %d, "
             "\"ms\": %.4f}}",
             best_kb, best_t1, best_chunk, best_batch, best_graph, best);
    js += buf;
    const size_t n = std::min<size_t>(js.size(), (size_t)len - 1);
    memcpy(report, js.data(), n);
    report[n] = 0;
  }
  return ISG_OK;
}

// ---------------------------------------------------------------------------
// solvers
// ---------------------------------------------------------------------------
// Conjugate gradients on N x = b: apply(in, out) enqueues out = N in, rhs(out)
// enqueues out = b; x holds x0 on entry and x_iters on return; resnorm
// (host, may be null) receives ||r_0|| .. ||r_iters||.  Synchronizes.
template <class Apply, class Rhs>
static isg_status cg_core(isg_plan* pl, Apply&& apply, Rhs&& rhs, int iters, float2* xv, double* resnorm) {
    const int64_t N = pl->N;
    if (!pl->cg_r) {
      pl->cg_r = (float2*)plan_alloc(pl, sizeof(float2) * N);
      pl->cg_p = (float2*)plan_alloc(pl, sizeof(float2) * N);
      pl->cg_q = (float2*)plan_alloc(pl, sizeof(float2) * N);
      pl->cg_part = (double*)plan_alloc(pl, sizeof(double) * kDotBlocks);
      pl->cg_sc = (CgScalars*)plan_alloc(pl, sizeof(CgScalars));
    }
    grow(pl, pl->cg_hist, sizeof(double) * (iters + 1));
    double* hist = (double*)pl->cg_hist.p;
    const unsigned vb = (unsigned)std::min<int64_t>(kDotBlocks, blocks_for(N, kVecThreads));
    // r = b - N x0 with b = sum_p A_p^H y_p; p = r; rho = <r, r>.  For
    // x0 = 0 (the usual start) N x0 is exactly zero, so r = b without an
    // application of N: ||x0||^2, read back once, decides.
    hipLaunchKernelGGL(dot_partial_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, xv, xv, N, pl->cg_part);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kVecThreads), 0, pl->stream, pl->cg_part, (int)vb, hist);
    LAUNCH_OK();
    double x0_sq = -1.0;
    HIP_OK(hipMemcpyAsync(&x0_sq, hist, sizeof(double), hipMemcpyDeviceToHost, pl->stream));
    HIP_OK(hipStreamSynchronize(pl->stream));
    rhs(pl->cg_p);
    if (x0_sq == 0.0) {
      hipLaunchKernelGGL(copy_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, pl->cg_r, pl->cg_p, N);
    } else {
      apply(xv, pl->cg_q);
      hipLaunchKernelGGL(sub_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, pl->cg_r, pl->cg_p, pl->cg_q, N);
      hipLaunchKernelGGL(copy_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, pl->cg_p, pl->cg_r, N);
    }
    hipLaunchKernelGGL(dot_partial_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, pl->cg_r, pl->cg_r, N,
                       pl->cg_part);
    hipLaunchKernelGGL(cg_init_kernel, dim3(1), dim3(kVecThreads), 0, pl->stream, pl->cg_part, (int)vb, pl->cg_sc,
                       hist);
    LAUNCH_OK();
    auto iteration = [&]() {
      apply(pl->cg_p, pl->cg_q);
      Tick tick(pl, "cg_vector");
      hipLaunchKernelGGL(dot_partial_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, pl->cg_p, pl->cg_q, N,
                         pl->cg_part);
      hipLaunchKernelGGL(cg_alpha_kernel, dim3(1), dim3(kVecThreads), 0, pl->stream, pl->cg_part, (int)vb,
                         pl->cg_sc);
      hipLaunchKernelGGL(cg_update_xr_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, xv, pl->cg_r, pl->cg_p,
                         pl->cg_q, N, pl->cg_sc, pl->cg_part);
      hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(kVecThreads), 0, pl->stream, pl->cg_part, (int)vb, pl->cg_sc,
                         hist);
      hipLaunchKernelGGL(cg_update_p_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, pl->cg_p, pl->cg_r, N,
                         pl->cg_sc);
      LAUNCH_OK();
    };
    const char* ng = getenv("ISG_NO_GRAPH");
    const bool use_graph = iters > 1 && !(ng && atoi(ng));
    // a graph cannot be captured on the null stream: run the solve on a
    // plan-owned stream, ordered after the caller's work
    hipStream_t caller = pl->stream;
    if (use_graph && caller == nullptr) {
      if (!pl->own_stream) HIP_OK(hipStreamCreateWithFlags(&pl->own_stream, hipStreamNonBlocking));
      HIP_OK(hipStreamSynchronize(nullptr));
      pl->stream = pl->own_stream;
    }
    struct Restore {
      isg_plan* p;
      hipStream_t s;
      ~Restore() { p->stream = s; }
    } restore{pl, caller};
    if (use_graph) {
      // make sure every lazily grown buffer exists before capture
      iteration();
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      HIP_OK(hipStreamBeginCapture(pl->stream, hipStreamCaptureModeThreadLocal));
      pl->capturing = true;
      try {
        iteration();
      } catch (...) {
        pl->capturing = false;
        hipGraph_t g2 = nullptr;
        (void)hipStreamEndCapture(pl->stream, &g2);
        if (g2) (void)hipGraphDestroy(g2);
        throw;
      }
      pl->capturing = false;
      HIP_OK(hipStreamEndCapture(pl->stream, &graph));
      HIP_OK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      for (int it = 1; it < iters; ++it) HIP_OK(hipGraphLaunch(exec, pl->stream));
      HIP_OK(hipStreamSynchronize(pl->stream));
      (void)hipGraphExecDestroy(exec);
      (void)hipGraphDestroy(graph);
    } else {
      for (int it = 0; it < iters; ++it) iteration();
    }
    CgScalars sc;
    HIP_OK(hipMemcpyAsync(&sc, pl->cg_sc, sizeof(sc), hipMemcpyDeviceToHost, pl->stream));
    HIP_OK(hipStreamSynchronize(pl->stream));
    if (resnorm) HIP_OK(hipMemcpy(resnorm, hist, sizeof(double) * (iters + 1), hipMemcpyDeviceToHost));
    if (sc.breakdown) return fail(ISG_ERR_CG_BREAKDOWN, "CG breakdown: Re<p, N p> <= 0 or not finite");
    return ISG_OK;
}

// the warp's normal operator (T^H T + lambda I) z (Eq. 13, l2 form)
static void op_warp_normal(isg_plan* pl, const isg_motion* mo, const float2* z, double lam, float2* out) {
  upsample(pl, z, pl->ugrid);
  warp_gather(pl, pl->ugrid, mo, pl->mbuf);
  const float2* w = pl->mbuf;
  warp_spread(pl, 1, &mo, &w, pl->ugrid);
  upsample_adjoint(pl, pl->ugrid, out);
  if (lam != 0.0) {
    hipLaunchKernelGGL(axpy_kernel, dim3(std::min<int64_t>(blocks_for(pl->N, kVecThreads), 4096)), dim3(kVecThreads),
                       0, pl->stream, out, z, (float)lam, pl->N);
    LAUNCH_OK();
  }
}

// ---- orthonormal Haar wavelet (Mallat layout), `levels` levels ---------------
static bool wavelet_levels_ok(const isg_plan* pl, int levels) {
  if (levels < 1 || levels > 9) return false;
  for (int i = 0; i < pl->ndim; ++i)
    if (pl->n[i] % (1 << levels)) return false;
  return true;
}

static Box full_box(const isg_plan* pl, int level) {  // box of `level` in the full image array
  Box b;
  b.b[0] = pl->n[0] >> level;
  b.b[1] = pl->n[1] >> level;
  b.b[2] = pl->ndim == 3 ? pl->n[2] >> level : 1;
  b.s[0] = (int64_t)pl->n[1] * (pl->ndim == 3 ? pl->n[2] : 1);
  b.s[1] = pl->ndim == 3 ? pl->n[2] : 1;
  b.s[2] = 1;
  return b;
}

static Box compact_box(const Box& f) {  // the same extents, stored compactly
  Box b = f;
  b.s[2] = 1;
  b.s[1] = f.b[2];
  b.s[0] = (int64_t)f.b[1] * f.b[2];
  return b;
}

static void haar_launch(isg_plan* pl, bool inv, const float2* src, const Box& sb, float2* dst, const Box& db) {
  const int64_t blocks = (int64_t)(sb.b[0] / 2) * (sb.b[1] / 2) * (pl->ndim == 3 ? sb.b[2] / 2 : 1);
  const dim3 g((unsigned)((blocks + 255) / 256));
  if (pl->ndim == 3) {
    if (inv)
      hipLaunchKernelGGL((haar_level_kernel<3, 1>), g, dim3(256), 0, pl->stream, src, sb, dst, db);
    else
      hipLaunchKernelGGL((haar_level_kernel<3, 0>), g, dim3(256), 0, pl->stream, src, sb, dst, db);
  } else {
    if (inv)
      hipLaunchKernelGGL((haar_level_kernel<2, 1>), g, dim3(256), 0, pl->stream, src, sb, dst, db);
    else
      hipLaunchKernelGGL((haar_level_kernel<2, 0>), g, dim3(256), 0, pl->stream, src, sb, dst, db);
  }
  LAUNCH_OK();
}

static void box_copy(isg_plan* pl, const float2* src, const Box& sb, float2* dst, const Box& db) {
  const int64_t n = (int64_t)sb.b[0] * sb.b[1] * sb.b[2];
  hipLaunchKernelGGL(box_copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, pl->stream, src, sb, dst, db,
                     pl->ndim);
  LAUNCH_OK();
}

// w = W x; tmp: scratch image (N); x != w
static void wavelet_forward(isg_plan* pl, int levels, const float2* x, float2* w, float2* tmp) {
  Tick tick(pl, "wavelet");
  for (int l = 0; l < levels; ++l) {
    const Box fb = full_box(pl, l);
    if (l == 0) {
      haar_launch(pl, false, x, fb, w, fb);
    } else {  // the low-pass box of w, through tmp
      const Box cb = compact_box(fb);
      box_copy(pl, w, fb, tmp, cb);
      haar_launch(pl, false, tmp, cb, w, fb);
    }
  }
}

// x = W^H w; tmp: scratch image (N); x != w; w is left unchanged.  x is the
// working array: the coefficients are copied into it, then every level from
// the coarsest on is inverted in place through tmp.
static void wavelet_inverse(isg_plan* pl, int levels, const float2* w, float2* x, float2* tmp) {
  Tick tick(pl, "wavelet");
  HIP_OK(hipMemcpyAsync(x, w, sizeof(float2) * pl->N, hipMemcpyDeviceToDevice, pl->stream));
  for (int l = levels - 1; l >= 0; --l) {
    const Box fb = full_box(pl, l);
    const Box cb = compact_box(fb);
    box_copy(pl, x, fb, tmp, cb);
    haar_launch(pl, true, tmp, cb, x, fb);
  }
}

static void soft_threshold(isg_plan* pl, float2* w, int levels, float tau) {
  const int n1 = pl->n[1], n2 = pl->ndim == 3 ? pl->n[2] : 1;
  const int a0 = pl->n[0] >> levels, a1 = pl->n[1] >> levels, a2 = pl->ndim == 3 ? pl->n[2] >> levels : 1;
  Tick tick(pl, "soft_threshold");
  hipLaunchKernelGGL(soft_threshold_kernel, dim3(blocks_for(pl->N, 256)), dim3(256), 0, pl->stream, w, pl->N, n1, n2,
                     a0, a1, a2, tau);
  LAUNCH_OK();
}

// solver vectors: `count` images of N complex values, and `parts` doubles
static float2* sol_vectors(isg_plan* pl, int count, double** part, int parts) {
  grow(pl, pl->sol, sizeof(float2) * (size_t)pl->N * count);
  grow(pl, pl->sol_part, sizeof(double) * (size_t)std::max(parts, 1));
  if (part) *part = (double*)pl->sol_part.p;
  return (float2*)pl->sol.p;
}

// ---- FISTA: x_k = W^H S_{lam/L} W (z_k - (2/L)(A^H A z_k - A^H y)) ----------
template <class Apply, class Rhs>
static isg_status fista_core(isg_plan* pl, Apply&& apply_AhA, Rhs&& rhs, double lam, double L, int levels, int iters,
                             float2* x, double* change) {
  const int64_t N = pl->N;
  const unsigned vb = (unsigned)std::min<int64_t>(kDotBlocks, blocks_for(N, kVecThreads));
  double* part = nullptr;
  float2* V = sol_vectors(pl, 6, &part, kDotBlocks + iters + 1);
  float2 *Z = V, *Q = V + N, *B = V + 2 * N, *Wc = V + 3 * N, *T = V + 4 * N, *Xn = V + 5 * N;
  double* hist = part + kDotBlocks;
  rhs(B);  // A^H y
  HIP_OK(hipMemcpyAsync(Z, x, sizeof(float2) * N, hipMemcpyDeviceToDevice, pl->stream));  // z_1 = x_0
  double t = 1.0;
  for (int it = 0; it < iters; ++it) {
    apply_AhA(Z, Q);
    hipLaunchKernelGGL(fista_step_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, Xn, Z, Q, B, (float)(2.0 / L), N);
    LAUNCH_OK();
    wavelet_forward(pl, levels, Xn, Wc, T);
    soft_threshold(pl, Wc, levels, (float)(lam / L));
    wavelet_inverse(pl, levels, Wc, Xn, T);
    const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    hipLaunchKernelGGL(fista_momentum_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, Z, x, Xn,
                       (float)((t - 1.0) / tn), N, change ? part : nullptr);
    if (change)
      hipLaunchKernelGGL(norm_to_kernel, dim3(1), dim3(kVecThreads), 0, pl->stream, part, (int)vb, hist + it);
    LAUNCH_OK();
    t = tn;
  }
  HIP_OK(hipStreamSynchronize(pl->stream));
  if (change && iters > 0) HIP_OK(hipMemcpy(change, hist, sizeof(double) * iters, hipMemcpyDeviceToHost));
  return ISG_OK;
}

// ---- power iteration: v <- N v / ||N v|| --------------------------------------
template <class Apply>
static isg_status power_core(isg_plan* pl, Apply&& apply, int iters, float2* v, double* lmax) {
  const int64_t N = pl->N;
  const unsigned vb = (unsigned)std::min<int64_t>(kDotBlocks, blocks_for(N, kVecThreads));
  double* part = nullptr;
  float2* W = sol_vectors(pl, 1, &part, kDotBlocks + 1);
  double* nrm = part + kDotBlocks;
  // v_0 = x0 / ||x0||
  hipLaunchKernelGGL(dot_partial_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, v, v, N, part);
  hipLaunchKernelGGL(norm_to_kernel, dim3(1), dim3(kVecThreads), 0, pl->stream, part, (int)vb, nrm);
  hipLaunchKernelGGL(scale_by_inverse_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, v, v, nrm, N);
  LAUNCH_OK();
  for (int it = 0; it < iters; ++it) {
    apply(v, W);
    hipLaunchKernelGGL(dot_partial_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, W, W, N, part);
    hipLaunchKernelGGL(norm_to_kernel, dim3(1), dim3(kVecThreads), 0, pl->stream, part, (int)vb, nrm);
    hipLaunchKernelGGL(scale_by_inverse_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, v, W, nrm, N);
    LAUNCH_OK();
  }
  double h = 0.0;
  HIP_OK(hipMemcpyAsync(&h, nrm, sizeof(double), hipMemcpyDeviceToHost, pl->stream));
  HIP_OK(hipStreamSynchronize(pl->stream));
  if (!std::isfinite(h) || h <= 0.0) return fail(ISG_ERR_NOT_FINITE, "power iteration: ||N v|| is zero or not finite");
  *lmax = iters > 0 ? h : 0.0;
  return ISG_OK;
}

// ---- registration: gradient descent on E(d) = ||T_d ref - mov||^2 + mu ||grad d||^2
static isg_status register_core(isg_plan* pl, const float2* ref, const float2* mov, double mu, double step, int iters,
                                float* d, double* energy) {
  const int64_t N = pl->N;
  const int nd = pl->ndim;
  const unsigned vb = (unsigned)std::min<int64_t>(kDotBlocks, blocks_for(N, kVecThreads));
  double* part = nullptr;
  // vectors: residual r (N complex), then two fields of nd N floats (= nd N / 2 complex each)
  float2* V = sol_vectors(pl, 1 + nd, &part, 2 * kDotBlocks + iters + 1);
  float2* r = V;
  float* dB = (float*)(V + N);
  float* g = dB + (size_t)nd * N;
  double *p1 = part, *p2 = part + kDotBlocks, *hist = part + 2 * kDotBlocks;
  upsample(pl, ref, pl->ugrid);  // u: the reference on the oversampled grid, for every step
  float* cur = d;
  float* nxt = dB;
  auto energy_at = [&](const float* dc, int k) {
    if (nd == 3)
      hipLaunchKernelGGL(warp_gather_kernel<3>, dim3(blocks_for(N, kGridThreads)), dim3(kGridThreads), 0, pl->stream,
                         pl->ugrid, dc, pl->mbuf, pl->dims, pl->kb);
    else
      hipLaunchKernelGGL(warp_gather_kernel<2>, dim3(blocks_for(N, kGridThreads)), dim3(kGridThreads), 0, pl->stream,
                         pl->ugrid, dc, pl->mbuf, pl->dims, pl->kb);
    hipLaunchKernelGGL(residual_kernel, dim3(vb), dim3(kVecThreads), 0, pl->stream, r, pl->mbuf, mov, N, p1);
    if (nd == 3)
      hipLaunchKernelGGL(smoothness_kernel<3>, dim3(vb), dim3(kVecThreads), 0, pl->stream, dc, pl->dims, p2);
    else
      hipLaunchKernelGGL(smoothness_kernel<2>, dim3(vb), dim3(kVecThreads), 0, pl->stream, dc, pl->dims, p2);
    hipLaunchKernelGGL(energy_kernel, dim3(1), dim3(kVecThreads), 0, pl->stream, p1, p2, (int)vb, mu, hist + k);
    LAUNCH_OK();
  };
  for (int it = 0; it < iters; ++it) {
    energy_at(cur, it);
    Tick tick(pl, "register_step");
    if (nd == 3) {
      hipLaunchKernelGGL(warp_grad_kernel<3>, dim3(blocks_for(N, kGridThreads)), dim3(kGridThreads), 0, pl->stream,
                         pl->ugrid, cur, r, g, pl->dims, pl->kb);
      hipLaunchKernelGGL(register_update_kernel<3>, dim3(vb), dim3(kVecThreads), 0, pl->stream, nxt, cur, g, pl->dims,
                         (float)mu, (float)step);
    } else {
      hipLaunchKernelGGL(warp_grad_kernel<2>, dim3(blocks_for(N, kGridThreads)), dim3(kGridThreads), 0, pl->stream,
                         pl->ugrid, cur, r, g, pl->dims, pl->kb);
      hipLaunchKernelGGL(register_update_kernel<2>, dim3(vb), dim3(kVecThreads), 0, pl->stream, nxt, cur, g, pl->dims,
                         (float)mu, (float)step);
    }
    LAUNCH_OK();
    std::swap(cur, nxt);
  }
  energy_at(cur, iters);
  if (cur != d) HIP_OK(hipMemcpyAsync(d, cur, sizeof(float) * nd * N, hipMemcpyDeviceToDevice, pl->stream));
  HIP_OK(hipStreamSynchronize(pl->stream));
  if (energy) HIP_OK(hipMemcpy(energy, hist, sizeof(double) * (iters + 1), hipMemcpyDeviceToHost));
  return ISG_OK;
}

// ---- direct gridding: x = sum_c conj(S_c) G^H(w conj(ph) y_c) ---------------------
static void op_grid_recon(isg_plan* pl, const isg_traj* tr, const float2* y, const float* w, const float2* S,
                          float2* x) {
  const int64_t tiles = std::max<int64_t>(1, tr->ntouched);
  ensure_kspace(pl, 1, std::max<int64_t>(1, tr->nvis), tiled_adjoint(pl) ? tiles : 0);
  if (pl->ymax) zero_ymax(pl, pl->ymax, 1);
  float2* yv = to_visit_order(pl, tr, y, (float2*)pl->ybuf.p, 0, w);
  const KJob job{tr, grid_of(pl, 0), yv, nullptr, sgrid_of(pl, 0, tiles)};
  STORAGE_DISPATCH(pl, kspread_t, pl, &job, 1);
  STORAGE_DISPATCH(pl, coil_adjoint_t, pl, sgrid_of(pl, 0, tiles), S, x, tr, half_undo(pl, 0, tr, false));
}

// ---- Pipe-Menon density compensation -----------------------------------------
static isg_status dcf_core(isg_plan* pl, const isg_traj* tr, int iters, float* w) {
  const int64_t M = tr->M;
  grow(pl, pl->sol, sizeof(float) * (size_t)pl->NG);
  float* grid = (float*)pl->sol.p;
  const unsigned mb = blocks_for(M, 256);
  hipLaunchKernelGGL(fill_f32_kernel, dim3(std::min<unsigned>(mb, 4096)), dim3(256), 0, pl->stream, w, M, 1.f);
  LAUNCH_OK();
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(fill_f32_kernel, dim3(4096), dim3(256), 0, pl->stream, grid, pl->NG, 0.f);
    if (pl->ndim == 3) {
      hipLaunchKernelGGL(dcf_spread_kernel<3>, dim3(mb), dim3(256), 0, pl->stream, tr->taps, w, M, grid, pl->dims, pl->kb);
      hipLaunchKernelGGL(dcf_update_kernel<3>, dim3(mb), dim3(256), 0, pl->stream, tr->taps, w, M, grid, pl->dims, pl->kb);
    } else {
      hipLaunchKernelGGL(dcf_spread_kernel<2>, dim3(mb), dim3(256), 0, pl->stream, tr->taps, w, M, grid, pl->dims, pl->kb);
      hipLaunchKernelGGL(dcf_update_kernel<2>, dim3(mb), dim3(256), 0, pl->stream, tr->taps, w, M, grid, pl->dims, pl->kb);
    }
    LAUNCH_OK();
  }
  HIP_OK(hipStreamSynchronize(pl->stream));
  return ISG_OK;
}

// ---------------------------------------------------------------------------
// allocation-free variant of the warp adjoint: its oversampled grid and FFT
// intermediates live in a fixed device array instead of plan memory
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
// Never pass `scratch` itself to a kernel or a copy: in host code the name is
// a host-side stand-in.  static_scratch() returns the device address.
static __device__ __align__(256) char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;  // device ordinal -> address of that device's copy

// device address of the current device's copy of `scratch`, looked up once
// per device (each GPU holds its own copy at its own address)
static void* static_scratch() {
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) throw HipError{hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch) returned NULL"};
  g_scratch_ptr[dev] = ptr;
  return ptr;
}

// byte offsets of the warp-adjoint buffers inside the static scratch: U
// [G...], the spread regions, then C, B, A of the adjoint upsampling
// passes, each 256-aligned
struct StaticLayout {
  size_t u, reg, a, b, c, total;
};
static StaticLayout static_layout(const isg_plan* pl) {
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t e = sizeof(float2);
  StaticLayout L;
  L.u = 0;
  L.reg = up(L.u + e * (size_t)pl->NG);
  L.c = up(L.reg + warp_region_bytes(pl));
  const size_t cb = pl->ndim == 3 ? e * (size_t)pl->G[0] * pl->G[1] * pl->n[2] : 0;
  L.b = up(L.c + cb);
  L.a = up(L.b + e * (size_t)pl->G[0] * pl->n[1] * pl->n[2]);
  L.total = up(L.a + e * (size_t)pl->N);
  return L;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* isg_version(void) { return "isg 0.1 gfx950"; }

const char* isg_last_error(void) { return g_last_error.c_str(); }

isg_status isg_device_count(int* count) {
  if (!count) return fail(ISG_ERR_INVALID_ARG, "count is NULL");
  int c = 0;
  if (hipGetDeviceCount(&c) != hipSuccess) {
    (void)hipGetLastError();
    c = 0;
  }
  *count = c;
  return ISG_OK;
}

isg_status isg_plan_create(const isg_plan_desc* desc, isg_plan** out) {
  if (!desc || !out) return fail(ISG_ERR_INVALID_ARG, "desc and plan must not be NULL");
  *out = nullptr;
  if (desc->ndim != 2 && desc->ndim != 3) return fail(ISG_ERR_INVALID_ARG, "ndim must be 2 or 3");
  if (desc->ncoils < 1 || desc->ncoils > 32) return fail(ISG_ERR_INVALID_ARG, "ncoils must be in 1..32");
  if (desc->nphases < 1 || desc->nphases > 1024) return fail(ISG_ERR_INVALID_ARG, "nphases must be in 1..1024");
  if (desc->storage < ISG_STORE_FP32 || desc->storage > ISG_STORE_FP16)
    return fail(ISG_ERR_INVALID_ARG, "unknown storage type");
  if (desc->alpha != kAlpha) return fail(ISG_ERR_UNSUPPORTED_SHAPE, "alpha (oversampling) must be 2");
  if (desc->width != kWidth) return fail(ISG_ERR_UNSUPPORTED_SHAPE, "width (kernel taps per axis) must be 4");
  if (!(desc->beta <= 0.0) && !(std::fabs(desc->beta - kb_beta()) <= 1e-9 * kb_beta()))
    return fail(ISG_ERR_UNSUPPORTED_SHAPE, "beta must be <= 0 (the default Kaiser-Bessel shape) or equal to it");
  for (int i = 0; i < desc->ndim; ++i)
    if (!good_length(desc->n[i]))
      return fail(ISG_ERR_UNSUPPORTED_SHAPE,
                  "each n_i must be even, in 8..512, with prime factors 2, 3, 5, 7 only (got " +
                      std::to_string((long long)desc->n[i]) + ")");
  {  // the coil passes hold all C coils of a line: C * 2 n_last <= 8192
    const int64_t Gl = 2 * desc->n[desc->ndim - 1];
    if ((int64_t)desc->ncoils * Gl > kFftThreads * kMaxPerThread)
      return fail(ISG_ERR_UNSUPPORTED_SHAPE, "ncoils * 2 * n_last must not exceed 8192");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(ISG_ERR_DEVICE, "no HIP device available");
  }
  isg_plan* pl = new (std::nothrow) isg_plan();
  if (!pl) return fail(ISG_ERR_OUT_OF_MEMORY, "host allocation failed");
  pl->ndim = desc->ndim;
  pl->N = 1;
  pl->NG = 1;
  for (int i = 0; i < pl->ndim; ++i) {
    pl->n[i] = (int)desc->n[i];
    pl->G[i] = kAlpha * pl->n[i];
    pl->N *= pl->n[i];
    pl->NG *= pl->G[i];
  }
  pl->C = desc->ncoils;
  pl->P = desc->nphases;
  pl->storage = desc->storage;
  pl->stream = (hipStream_t)desc->stream;
  pl->beta = kb_beta();
  pl->kb = make_kbpoly(pl->beta);
  pl->dims.ndim = pl->ndim;
  for (int i = 0; i < 3; ++i) {
    pl->dims.n[i] = pl->n[i];
    pl->dims.G[i] = pl->G[i];
  }
  pl->dims.N = pl->N;
  for (int i = 0; i < 3; ++i) {
    pl->dims.nfd[i] = make_fastdiv((uint32_t)pl->n[i]);
    pl->dims.invG[i] = (float)(1.0 / pl->G[i]);
  }
  // spread tiles
  for (int i = 0; i < 3; ++i) {
    pl->wtile.TS[i] = 1;
    pl->wtile.nt[i] = 1;
    pl->ktile.TS[i] = 1;
    pl->ktile.nt[i] = 1;
  }
  // image-space spread tiles (powers of two, at most G/2) and their regions
  // (tile + 3 halo cells per axis; LDS rows padded to an even length)
  const int wts = pl->ndim == 3 ? 8 : 16;
  for (int i = 0; i < 3; ++i) {
    pl->wtile.TS[i] = 1;
    pl->wtile.lg[i] = 0;
    pl->wtile.nt[i] = 1;
    pl->wtile.E[i] = 1;
  }
  for (int i = 0; i < pl->ndim; ++i) {
    pl->wtile.TS[i] = spread_extent(wts, pl->G[i]);
    while ((1 << pl->wtile.lg[i]) < pl->wtile.TS[i]) pl->wtile.lg[i]++;
    pl->wtile.nt[i] = (pl->G[i] + pl->wtile.TS[i] - 1) / pl->wtile.TS[i];
    pl->wtile.E[i] = pl->wtile.TS[i] + kWidth - 1;
  }
  {
    const int last = pl->ndim - 1;
    const int row = pl->wtile.E[last] + (pl->wtile.E[last] & 1);
    if (pl->ndim == 3) {
      pl->wtile.R1 = row;
      pl->wtile.R0 = pl->wtile.E[1] * row;
    } else {
      pl->wtile.R1 = 1;
      pl->wtile.R0 = row;
    }
    pl->wtile.P = pl->wtile.E[0] * pl->wtile.R0;
    pl->wtile.RV = pl->wtile.E[0] * pl->wtile.E[1] * pl->wtile.E[2];
  }
  isg_status st = guarded(pl, [&]() -> isg_status {
    set_ktile(pl, pl->ndim == 3 ? 8 : 16);
    set_layouts(pl);
    HIP_OK(hipGetDevice(&pl->device));
    HIP_OK(hipDeviceGetAttribute(&pl->ncu, hipDeviceAttributeMultiprocessorCount, pl->device));
    // deapodization tables
    for (int i = 0; i < pl->ndim; ++i) {
      const int n = pl->n[i], G = pl->G[i];
      std::vector<float> k(n), x(n);
      for (int j = 0; j < n; ++j) {
        const int kk = j < n - n / 2 ? j : j - n;  // signed DFT bin
        k[j] = (float)(kb_transform(0.0, pl->beta) / kb_transform((double)kk / G, pl->beta));
        x[j] = (float)(kb_transform(0.0, pl->beta) / kb_transform((double)(j - n / 2) / G, pl->beta));
      }
      pl->dk[i] = (float*)plan_alloc(pl, sizeof(float) * n);
      pl->dx[i] = (float*)plan_alloc(pl, sizeof(float) * n);
      HIP_OK(hipMemcpy(pl->dk[i], k.data(), sizeof(float) * n, hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(pl->dx[i], x.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    }
    for (int i = 0; i < pl->ndim; ++i) {
      line_plan(pl, pl->n[i]);
      line_plan(pl, pl->G[i]);
    }
    const int n0 = pl->n[0], n1 = pl->n[1], n2 = pl->n[2];
    pl->ugrid = (float2*)plan_alloc(pl, sizeof(float2) * (size_t)pl->NG);
    pl->bufA = (float2*)plan_alloc(pl, sizeof(float2) * (size_t)pl->N);
    pl->mbuf = (float2*)plan_alloc(pl, sizeof(float2) * (size_t)pl->N);
    pl->bufB = (float2*)plan_alloc(pl, sizeof(float2) * (size_t)pl->G[0] * n1 * n2);
    if (pl->ndim == 3) pl->bufC = (float2*)plan_alloc(pl, sizeof(float2) * (size_t)pl->G[0] * pl->G[1] * n2);
    if (pl->storage != kFP32) {
      pl->hsc = (float*)plan_alloc(pl, 2 * sizeof(float));
      pl->hs_part = (double*)plan_alloc(pl, sizeof(double) * kDotBlocks);
      pl->ymax = (unsigned*)plan_alloc(pl, sizeof(unsigned) * kMaxPhasesPerLaunch * kYmaxSlots);
    }
    (void)n0;
    return ISG_OK;
  });
  if (st != ISG_OK) {
    isg_plan_destroy(pl);
    return st;
  }
  *out = pl;
  return ISG_OK;
}

isg_status isg_plan_destroy(isg_plan* pl) {
  if (!pl) return ISG_OK;
  (void)hipStreamSynchronize(pl->stream);
  // motions and trajectories that outlive the plan keep their own device
  // memory until their destroy call, which then touches no plan state
  for (isg_motion* mo : pl->motions) mo->plan = nullptr;
  for (isg_traj* tr : pl->trajs) tr->plan = nullptr;
  for (void* p : pl->owned) (void)hipFree(p);
  if (pl->ngraph.exec) (void)hipGraphExecDestroy(pl->ngraph.exec);
  if (pl->ngraph.graph) (void)hipGraphDestroy(pl->ngraph.graph);
  if (pl->kgrid.p) (void)hipFree(pl->kgrid.p);
  if (pl->wreg.p) (void)hipFree(pl->wreg.p);
  if (pl->kgrid_adj.p) (void)hipFree(pl->kgrid_adj.p);
  if (pl->ybuf.p) (void)hipFree(pl->ybuf.p);
  if (pl->partial.p) (void)hipFree(pl->partial.p);
  if (pl->cg_hist.p) (void)hipFree(pl->cg_hist.p);
  if (pl->tune_out.p) (void)hipFree(pl->tune_out.p);
  if (pl->sol.p) (void)hipFree(pl->sol.p);
  if (pl->sol_part.p) (void)hipFree(pl->sol_part.p);
  if (pl->bin.p) (void)hipFree(pl->bin.p);
  if (pl->own_stream) (void)hipStreamDestroy(pl->own_stream);
  for (auto& p : pl->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : pl->pool) (void)hipEventDestroy(e);
  (void)hipGetLastError();
  delete pl;
  return ISG_OK;
}

isg_status isg_plan_set_stream(isg_plan* pl, void* stream) {
  if (!pl) return fail(ISG_ERR_INVALID_ARG, "plan is NULL");
  pl->stream = (hipStream_t)stream;
  return ISG_OK;
}

isg_status isg_plan_device_bytes(const isg_plan* pl, int64_t* bytes) {
  if (!pl || !bytes) return fail(ISG_ERR_INVALID_ARG, "plan and bytes must not be NULL");
  *bytes = pl->bytes;
  return ISG_OK;
}

isg_status isg_plan_set_timing(isg_plan* pl, int enable, const char* prefix) {
  if (!pl) return fail(ISG_ERR_INVALID_ARG, "plan is NULL");
  return guarded(pl, [&]() {
    collect_timing(pl);
    pl->timed.clear();
    pl->timing = enable != 0;
    pl->timing_filter = prefix ? prefix : "";
    return ISG_OK;
  });
}

isg_status isg_plan_read_timing(isg_plan* pl, char* buf, int64_t len) {
  if (!pl || !buf || len < 3) return fail(ISG_ERR_INVALID_ARG, "plan / buffer invalid");
  return guarded(pl, [&]() -> isg_status {
    collect_timing(pl);
    std::string js = "{";
    bool first = true;
    for (auto& kv : pl->timed) {
      char tmp[256];
      snprintf(tmp, sizeof(tmp), "%s\"%s\": [%lld, %.6f]", first ? "" : ", ", kv.first.c_str(),
               (long long)kv.second.first, kv.second.second);
      js += tmp;
      first = false;
    }
    js += "}";
    if ((int64_t)js.size() + 1 > len) return fail(ISG_ERR_INVALID_ARG, "timing buffer too small");
    memcpy(buf, js.c_str(), js.size() + 1);
    return ISG_OK;
  });
}

isg_status isg_motion_create(isg_plan* pl, const float* d, isg_motion** out) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!d || !out) return fail(ISG_ERR_INVALID_ARG, "d and motion must not be NULL");
  *out = nullptr;
  isg_motion* mo = new (std::nothrow) isg_motion();
  if (!mo) return fail(ISG_ERR_OUT_OF_MEMORY, "host allocation failed");
  mo->plan = pl;
  pl->motions.insert(mo);
  st = guarded(pl, [&]() { return prepare_motion(pl, d, mo); });
  if (st != ISG_OK) {
    isg_motion_destroy(mo);
    return st;
  }
  *out = mo;
  return ISG_OK;
}

isg_status isg_motion_destroy(isg_motion* mo) {
  if (!mo) return ISG_OK;
  isg_plan* pl = mo->plan;
  if (pl) {
    (void)hipStreamSynchronize(pl->stream);
    pl->generation++;
    pl->motions.erase(mo);
  }
  for (void* p : {(void*)mo->d, (void*)mo->tile_off, (void*)mo->vox}) (void)dfree(pl, p);
  delete mo;
  return ISG_OK;
}

isg_status isg_traj_create(isg_plan* pl, const float* k, int64_t M, isg_traj** out) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!k || !out) return fail(ISG_ERR_INVALID_ARG, "k and traj must not be NULL");
  if (M < 1 || M > (int64_t)1 << 30) return fail(ISG_ERR_INVALID_ARG, "M must be in 1..2^30");
  *out = nullptr;
  isg_traj* tr = new (std::nothrow) isg_traj();
  if (!tr) return fail(ISG_ERR_OUT_OF_MEMORY, "host allocation failed");
  tr->plan = pl;
  pl->trajs.insert(tr);
  st = guarded(pl, [&]() { return prepare_traj(pl, k, M, tr); });
  if (st != ISG_OK) {
    isg_traj_destroy(tr);
    return st;
  }
  *out = tr;
  return ISG_OK;
}

isg_status isg_traj_destroy(isg_traj* tr) {
  if (!tr) return ISG_OK;
  isg_plan* pl = tr->plan;
  if (pl) {
    (void)hipStreamSynchronize(pl->stream);
    pl->generation++;
    pl->trajs.erase(tr);
  }
  for (void* p : {(void*)tr->taps, (void*)tr->order, (void*)tr->gorder, (void*)tr->units, (void*)tr->splits,
                  (void*)tr->colmask, (void*)tr->fmask, (void*)tr->cact, (void*)tr->colbase, (void*)tr->taps_v,
                  (void*)tr->vis_off, (void*)tr->vis, (void*)tr->k, (void*)tr->phase})
    (void)dfree(pl, p);
  delete tr;
  return ISG_OK;
}

isg_status isg_traj_info(const isg_traj* tr, int64_t* nvisits, int64_t* ntiles, int64_t* tile_points) {
  if (!tr || !nvisits || !ntiles || !tile_points) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  *nvisits = tr->nvis;
  *ntiles = tr->ntouched;
  *tile_points = (int64_t)tr->ts[0] * tr->ts[1] * tr->ts[2];  // no plan access: the plan may be gone
  return ISG_OK;
}

isg_status isg_traj_touched_cells(const isg_traj* tr, int64_t* cells) {
  if (!tr || !cells) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  *cells = tr->fine_cells;
  return ISG_OK;
}

isg_status isg_traj_active_columns(const isg_traj* tr, int64_t* cols) {
  if (!tr || !cols) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  *cols = tr->active_cols;
  return ISG_OK;
}

isg_status isg_traj_count(const isg_traj* tr, int64_t* M) {
  if (!tr || !M) return fail(ISG_ERR_INVALID_ARG, "traj and M must not be NULL");
  *M = tr->M;
  return ISG_OK;
}

isg_status isg_warp(isg_plan* pl, const isg_motion* d, const void* x, void* y) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!d || !x || !y) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (d->plan != pl) return fail(ISG_ERR_INVALID_ARG, "motion belongs to another plan");
  if (x == y) return fail(ISG_ERR_INVALID_ARG, "warp is out-of-place: x must differ from y");
  return guarded(pl, [&]() {
    upsample(pl, (const float2*)x, pl->ugrid);
    warp_gather(pl, pl->ugrid, d, (float2*)y);
    return ISG_OK;
  });
}

isg_status isg_warp_adjoint(isg_plan* pl, const isg_motion* d, const void* y, void* x) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!d || !x || !y) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (d->plan != pl) return fail(ISG_ERR_INVALID_ARG, "motion belongs to another plan");
  if (x == y) return fail(ISG_ERR_INVALID_ARG, "warp_adjoint is out-of-place: x must differ from y");
  return guarded(pl, [&]() {
    const float2* w = (const float2*)y;
    warp_spread(pl, 1, &d, &w, pl->ugrid);
    upsample_adjoint(pl, pl->ugrid, (float2*)x);
    return ISG_OK;
  });
}

isg_status isg_warp_adjoint_noalloc(isg_plan* pl, const isg_motion* d, const void* y, void* x) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!d || !x || !y) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (d->plan != pl) return fail(ISG_ERR_INVALID_ARG, "motion belongs to another plan");
  if (x == y) return fail(ISG_ERR_INVALID_ARG, "warp_adjoint is out-of-place: x must differ from y");
  const StaticLayout L = static_layout(pl);
  if (L.total > kStaticScratchBytes)
    return fail(ISG_ERR_INVALID_ARG, "isg_warp_adjoint_noalloc: the shape needs " + std::to_string(L.total >> 20) +
                                         " MiB of scratch, more than the fixed 64 MiB (use isg_warp_adjoint)");
  return guarded(pl, [&]() -> isg_status {
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev != pl->device) return fail(ISG_ERR_INVALID_ARG, "the plan's device must be current");
    char* base = (char*)static_scratch();
    float2* U = (float2*)(base + L.u);
    const UpBufs ub{(float2*)(base + L.a), (float2*)(base + L.b), pl->ndim == 3 ? (float2*)(base + L.c) : nullptr};
    const float2* w = (const float2*)y;
    // the spread writes every region cell and every cell of U (no
    // accumulation into old contents)
    warp_spread(pl, 1, &d, &w, U, (float2*)(base + L.reg));
    upsample_adjoint(pl, U, (float2*)x, ub);
    return ISG_OK;
  });
}

isg_status isg_warp_grad_d(isg_plan* pl, const isg_motion* d, const void* x, const void* v, float* grad) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!d || !x || !v || !grad) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (d->plan != pl) return fail(ISG_ERR_INVALID_ARG, "motion belongs to another plan");
  return guarded(pl, [&]() {
    upsample(pl, (const float2*)x, pl->ugrid);
    Tick tick(pl, "warp_grad");
    if (pl->ndim == 3)
      hipLaunchKernelGGL(warp_grad_kernel<3>, dim3(blocks_for(pl->N, kGridThreads)), dim3(kGridThreads), 0,
                         pl->stream, pl->ugrid, d->d, (const float2*)v, grad, pl->dims, pl->kb);
    else
      hipLaunchKernelGGL(warp_grad_kernel<2>, dim3(blocks_for(pl->N, kGridThreads)), dim3(kGridThreads), 0,
                         pl->stream, pl->ugrid, d->d, (const float2*)v, grad, pl->dims, pl->kb);
    LAUNCH_OK();
    return ISG_OK;
  });
}

isg_status isg_sense_forward(isg_plan* pl, int P, const void* x, const isg_motion* const* d, const void* S,
                             const isg_traj* const* k, void* y) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!x || !S || !y) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  st = check_phases(pl, P, d, k);
  if (st) return st;
  return guarded(pl, [&]() {
    op_sense_forward(pl, P, (const float2*)x, d, (const float2*)S, k, (float2*)y);
    return ISG_OK;
  });
}

isg_status isg_sense_adjoint(isg_plan* pl, int P, const void* y, const isg_motion* const* d, const void* S,
                             const isg_traj* const* k, void* x) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!x || !S || !y) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  st = check_phases(pl, P, d, k);
  if (st) return st;
  return guarded(pl, [&]() {
    op_sense_adjoint(pl, P, (const float2*)y, d, (const float2*)S, k, (float2*)x);
    return ISG_OK;
  });
}

isg_status isg_normal(isg_plan* pl, int P, const void* x, double lambda, const isg_motion* const* d, const void* S,
                      const isg_traj* const* k, void* out) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!x || !S || !out) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (x == out) return fail(ISG_ERR_INVALID_ARG, "normal is out-of-place: x must differ from out");
  if (!std::isfinite(lambda)) return fail(ISG_ERR_INVALID_ARG, "lambda must be finite");
  st = check_phases(pl, P, d, k);
  if (st) return st;
  return guarded(pl, [&]() {
    normal_maybe_graph(pl, P, (const float2*)x, lambda, d, (const float2*)S, k, (float2*)out);
    return ISG_OK;
  });
}

isg_status isg_plan_set_option(isg_plan* pl, isg_option option, int64_t value) {
  isg_status st = check_plan(pl);
  if (st) return st;
  switch (option) {
    case ISG_OPT_SPREAD_CHUNK:
      if (value < 32 || value > 65536) return fail(ISG_ERR_INVALID_ARG, "spread chunk must be in 32..65536");
      pl->opt_spread_chunk = (int)value;
      break;
    case ISG_OPT_PHASE_BATCH:
      if (value < 1 || value > kMaxPhasesPerLaunch) return fail(ISG_ERR_INVALID_ARG, "phase batch must be in 1..16");
      pl->opt_phase_batch = (int)value;
      break;
    case ISG_OPT_GRAPH:
      if (value != 0 && value != 1) return fail(ISG_ERR_INVALID_ARG, "graph option must be 0 or 1");
      pl->opt_graph = (int)value;
      break;
    case ISG_OPT_FFT_ADDR:
      if (value != 0 && value != 1) return fail(ISG_ERR_INVALID_ARG, "FFT addressing option must be 0 or 1");
      pl->opt_fft_addr = (int)value;
      break;
    case ISG_OPT_KBLOCK:
      if (value != 0 && (value < 1 || value > 6)) return fail(ISG_ERR_INVALID_ARG, "k-space block must be 0 or 1..6");
      {
        const isg_status s2 = guarded(pl, [&]() -> isg_status {
          HIP_OK(hipStreamSynchronize(pl->stream));
          pl->opt_blk_tlog = value == 0 ? 30 : (int)value;
          set_layouts(pl);
          return ISG_OK;
        });
        if (s2 != ISG_OK) return s2;
      }
      break;
    case ISG_OPT_KTILE_T1:
      if (value != 4 && value != 8 && value != 16) return fail(ISG_ERR_INVALID_ARG, "k-space tile extent must be 4, 8 or 16");
      {
        const isg_status s2 = guarded(pl, [&]() -> isg_status {
          HIP_OK(hipStreamSynchronize(pl->stream));
          set_ktile(pl, (int)value);
          return ISG_OK;
        });
        if (s2 != ISG_OK) return s2;
      }
      break;
    default:
      return fail(ISG_ERR_INVALID_ARG, "unknown option");
  }
  pl->generation++;
  return ISG_OK;
}

isg_status isg_plan_get_option(const isg_plan* pl, isg_option option, int64_t* value) {
  if (!pl || !value) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  switch (option) {
    case ISG_OPT_SPREAD_CHUNK: *value = pl->opt_spread_chunk; break;
    case ISG_OPT_PHASE_BATCH: *value = pl->opt_phase_batch; break;
    case ISG_OPT_GRAPH: *value = pl->opt_graph; break;
    case ISG_OPT_FFT_ADDR: *value = pl->opt_fft_addr; break;
    case ISG_OPT_KTILE_T1: *value = pl->opt_ktile_t1; break;
    case ISG_OPT_KBLOCK: *value = pl->opt_blk_tlog >= 30 ? 0 : pl->opt_blk_tlog; break;
    default: return fail(ISG_ERR_INVALID_ARG, "unknown option");
  }
  return ISG_OK;
}

isg_status isg_plan_tune(isg_plan* pl, int P, const void* x, const isg_motion* const* d, const void* S,
                         isg_traj* const* k, double lambda, int reps, char* report, int64_t len) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!x || !S) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (reps < 1 || reps > 1000) return fail(ISG_ERR_INVALID_ARG, "reps must be in 1..1000");
  if (!std::isfinite(lambda)) return fail(ISG_ERR_INVALID_ARG, "lambda must be finite");
  st = check_phases(pl, P, d, (const isg_traj* const*)k);
  if (st) return st;
  return guarded(pl, [&]() -> isg_status { return tune(pl, P, (const float2*)x, d, (const float2*)S, k, lambda,
                                                       reps, report, len); });
}

isg_status isg_sense_grad(isg_plan* pl, int P, const void* x, const isg_motion* const* d, const void* S,
                          const isg_traj* const* k, const void* r, void* grad_x, float* grad_d) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!x || !S || !r || (!grad_x && !grad_d)) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (grad_x == x) return fail(ISG_ERR_INVALID_ARG, "grad_x must differ from x");
  st = check_phases(pl, P, d, k);
  if (st) return st;
  return guarded(pl, [&]() {
    int64_t vmax = 1;
    for (int p = 0; p < P; ++p) vmax = std::max(vmax, k[p]->nvis);
    const int64_t tiles = max_touched(k, P);
    ensure_kspace(pl, 1, vmax, tiled_adjoint(pl) ? tiles : 0);
    const float2* Sm = (const float2*)S;
    // u = the upsampled x, needed by every d-gradient (before the spread reuses ugrid)
    if (grad_d) upsample(pl, (const float2*)x, pl->ugrid);
    std::vector<const float2*> w(P);
    int64_t off = 0;
    for (int p = 0; p < P; ++p) {
      // v_p = sum_c conj(S_c) G_p^H r_{p,c}
      if (pl->ymax) zero_ymax(pl, pl->ymax, 1);
      float2* yv = to_visit_order(pl, k[p], (const float2*)r + off, (float2*)pl->ybuf.p, 0);
      const KJob job{k[p], grid_of(pl, 0), yv, nullptr, sgrid_of(pl, 0, tiles)};
      STORAGE_DISPATCH(pl, kspread_t, pl, &job, 1);
      float2* v = pl->wbuf + (int64_t)p * pl->N;
      STORAGE_DISPATCH(pl, coil_adjoint_t, pl, sgrid_of(pl, 0, tiles), Sm, v, k[p], half_undo(pl, 0, k[p], false));
      w[p] = v;
      if (grad_d) {
        Tick tick(pl, "warp_grad");
        float* gd = grad_d + (int64_t)p * pl->ndim * pl->N;
        if (pl->ndim == 3)
          hipLaunchKernelGGL(warp_grad_kernel<3>, dim3(blocks_for(pl->N, kGridThreads)), dim3(kGridThreads), 0,
                             pl->stream, pl->ugrid, d[p]->d, v, gd, pl->dims, pl->kb);
        else
          hipLaunchKernelGGL(warp_grad_kernel<2>, dim3(blocks_for(pl->N, kGridThreads)), dim3(kGridThreads), 0,
                             pl->stream, pl->ugrid, d[p]->d, v, gd, pl->dims, pl->kb);
        LAUNCH_OK();
      }
      off += k[p]->M * pl->C;
    }
    if (grad_x) {
      warp_spread(pl, P, d, w.data(), pl->ugrid);
      upsample_adjoint(pl, pl->ugrid, (float2*)grad_x);
    }
    return ISG_OK;
  });
}

isg_status isg_cg_solve(isg_plan* pl, int P, const void* y, const isg_motion* const* d, const void* S,
                        const isg_traj* const* k, double lambda, int iters, void* x, double* resnorm) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!x || !S || !y) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (iters < 0 || iters > 100000) return fail(ISG_ERR_INVALID_ARG, "iters must be in 0..100000");
  if (!std::isfinite(lambda)) return fail(ISG_ERR_INVALID_ARG, "lambda must be finite");
  st = check_phases(pl, P, d, k);
  if (st) return st;
  return guarded(pl, [&]() -> isg_status {
    return cg_core(
        pl, [&](const float2* in, float2* out) { op_normal(pl, P, in, lambda, d, (const float2*)S, k, out); },
        [&](float2* out) { op_sense_adjoint(pl, P, (const float2*)y, d, (const float2*)S, k, out); }, iters,
        (float2*)x, resnorm);
  });
}

isg_status isg_warp_cg_solve(isg_plan* pl, const isg_motion* d, const void* q, double lambda, int iters, void* p,
                             double* resnorm) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!d || !q || !p) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (d->plan != pl) return fail(ISG_ERR_INVALID_ARG, "motion belongs to another plan");
  if (q == p) return fail(ISG_ERR_INVALID_ARG, "q and p must differ");
  if (iters < 0 || iters > 100000) return fail(ISG_ERR_INVALID_ARG, "iters must be in 0..100000");
  if (!std::isfinite(lambda)) return fail(ISG_ERR_INVALID_ARG, "lambda must be finite");
  return guarded(pl, [&]() -> isg_status {
    return cg_core(
        pl, [&](const float2* in, float2* out) { op_warp_normal(pl, d, in, lambda, out); },
        [&](float2* out) {  // T^H q
          const float2* w = (const float2*)q;
          warp_spread(pl, 1, &d, &w, pl->ugrid);
          upsample_adjoint(pl, pl->ugrid, out);
        },
        iters, (float2*)p, resnorm);
  });
}

isg_status isg_wavelet_forward(isg_plan* pl, int levels, const void* x, void* w) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!x || !w) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (x == w) return fail(ISG_ERR_INVALID_ARG, "the wavelet transform is out-of-place: x must differ from w");
  if (!wavelet_levels_ok(pl, levels))
    return fail(ISG_ERR_INVALID_ARG, "levels must be in 1..9 with every n_i divisible by 2^levels");
  return guarded(pl, [&]() -> isg_status {
    float2* T = sol_vectors(pl, 1, nullptr, 1);
    wavelet_forward(pl, levels, (const float2*)x, (float2*)w, T);
    return ISG_OK;
  });
}

isg_status isg_wavelet_inverse(isg_plan* pl, int levels, const void* w, void* x) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!x || !w) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (x == w) return fail(ISG_ERR_INVALID_ARG, "the wavelet transform is out-of-place: x must differ from w");
  if (!wavelet_levels_ok(pl, levels))
    return fail(ISG_ERR_INVALID_ARG, "levels must be in 1..9 with every n_i divisible by 2^levels");
  return guarded(pl, [&]() -> isg_status {
    float2* T = sol_vectors(pl, 1, nullptr, 1);
    wavelet_inverse(pl, levels, (const float2*)w, (float2*)x, T);
    return ISG_OK;
  });
}

isg_status isg_power_iteration(isg_plan* pl, int P, const isg_motion* const* d, const void* S,
                               const isg_traj* const* k, int iters, void* v, double* lmax) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!S || !v || !lmax) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (iters < 1 || iters > 100000) return fail(ISG_ERR_INVALID_ARG, "iters must be in 1..100000");
  st = check_phases(pl, P, d, k);
  if (st) return st;
  return guarded(pl, [&]() -> isg_status {
    return power_core(
        pl, [&](const float2* in, float2* out) { normal_maybe_graph(pl, P, in, 0.0, d, (const float2*)S, k, out); },
        iters, (float2*)v, lmax);
  });
}

isg_status isg_warp_power_iteration(isg_plan* pl, const isg_motion* d, int iters, void* v, double* lmax) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!d || !v || !lmax) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (d->plan != pl) return fail(ISG_ERR_INVALID_ARG, "motion belongs to another plan");
  if (iters < 1 || iters > 100000) return fail(ISG_ERR_INVALID_ARG, "iters must be in 1..100000");
  return guarded(pl, [&]() -> isg_status {
    return power_core(pl, [&](const float2* in, float2* out) { op_warp_normal(pl, d, in, 0.0, out); }, iters,
                      (float2*)v, lmax);
  });
}

static isg_status fista_args(isg_plan* pl, double lambda, double lipschitz, int levels, int iters) {
  if (!std::isfinite(lambda) || lambda < 0.0) return fail(ISG_ERR_INVALID_ARG, "lambda must be finite and >= 0");
  if (!std::isfinite(lipschitz) || lipschitz <= 0.0) return fail(ISG_ERR_INVALID_ARG, "lipschitz must be finite and > 0");
  if (iters < 0 || iters > 100000) return fail(ISG_ERR_INVALID_ARG, "iters must be in 0..100000");
  if (!wavelet_levels_ok(pl, levels))
    return fail(ISG_ERR_INVALID_ARG, "levels must be in 1..9 with every n_i divisible by 2^levels");
  return ISG_OK;
}

isg_status isg_fista_solve(isg_plan* pl, int P, const void* y, const isg_motion* const* d, const void* S,
                           const isg_traj* const* k, double lambda, double lipschitz, int levels, int iters, void* x,
                           double* change) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!y || !S || !x) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  st = fista_args(pl, lambda, lipschitz, levels, iters);
  if (st) return st;
  st = check_phases(pl, P, d, k);
  if (st) return st;
  return guarded(pl, [&]() -> isg_status {
    return fista_core(
        pl, [&](const float2* in, float2* out) { normal_maybe_graph(pl, P, in, 0.0, d, (const float2*)S, k, out); },
        [&](float2* out) { op_sense_adjoint(pl, P, (const float2*)y, d, (const float2*)S, k, out); }, lambda,
        lipschitz, levels, iters, (float2*)x, change);
  });
}

isg_status isg_warp_fista_solve(isg_plan* pl, const isg_motion* d, const void* q, double lambda, double lipschitz,
                                int levels, int iters, void* p, double* change) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!d || !q || !p) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (d->plan != pl) return fail(ISG_ERR_INVALID_ARG, "motion belongs to another plan");
  if (q == p) return fail(ISG_ERR_INVALID_ARG, "q and p must differ");
  st = fista_args(pl, lambda, lipschitz, levels, iters);
  if (st) return st;
  return guarded(pl, [&]() -> isg_status {
    return fista_core(
        pl, [&](const float2* in, float2* out) { op_warp_normal(pl, d, in, 0.0, out); },
        [&](float2* out) {
          const float2* w = (const float2*)q;
          warp_spread(pl, 1, &d, &w, pl->ugrid);
          upsample_adjoint(pl, pl->ugrid, out);
        },
        lambda, lipschitz, levels, iters, (float2*)p, change);
  });
}

isg_status isg_register(isg_plan* pl, const void* ref, const void* mov, double mu, double step, int iters, float* d,
                        double* energy) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!ref || !mov || !d) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (!std::isfinite(mu) || mu < 0.0) return fail(ISG_ERR_INVALID_ARG, "mu must be finite and >= 0");
  if (!std::isfinite(step) || step <= 0.0) return fail(ISG_ERR_INVALID_ARG, "step must be finite and > 0");
  if (iters < 0 || iters > 100000) return fail(ISG_ERR_INVALID_ARG, "iters must be in 0..100000");
  return guarded(pl, [&]() -> isg_status {
    return register_core(pl, (const float2*)ref, (const float2*)mov, mu, step, iters, d, energy);
  });
}

isg_status isg_traj_set_shift(isg_traj* tr, const float* t) {
  if (!tr) return fail(ISG_ERR_INVALID_ARG, "traj is NULL");
  isg_plan* pl = tr->plan;
  if (!pl) return fail(ISG_ERR_INVALID_ARG, "the trajectory's plan was destroyed");
  isg_status st = check_plan(pl);
  if (st) return st;
  return guarded(pl, [&]() -> isg_status {
    HIP_OK(hipStreamSynchronize(pl->stream));
    pl->generation++;
    if (!t) {  // back to no translation
      if (tr->phase) HIP_OK(dfree(pl, tr->phase));
      tr->phase = nullptr;
      return ISG_OK;
    }
    if (!tr->phase) tr->phase = (float2*)dmalloc(pl, sizeof(float2) * (size_t)tr->M);
    hipLaunchKernelGGL(shift_phase_kernel, dim3(blocks_for(tr->M, 256)), dim3(256), 0, pl->stream, tr->k, t,
                       pl->ndim, tr->M, tr->phase);
    LAUNCH_OK();
    HIP_OK(hipStreamSynchronize(pl->stream));
    return ISG_OK;
  });
}

isg_status isg_traj_dcf(isg_plan* pl, const isg_traj* tr, int iters, float* w) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!tr || !w) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (tr->plan != pl) return fail(ISG_ERR_INVALID_ARG, "trajectory belongs to another plan");
  if (iters < 0 || iters > 10000) return fail(ISG_ERR_INVALID_ARG, "iters must be in 0..10000");
  return guarded(pl, [&]() -> isg_status { return dcf_core(pl, tr, iters, w); });
}

isg_status isg_grid_recon(isg_plan* pl, const isg_traj* tr, const void* y, const float* w, const void* S, void* x) {
  isg_status st = check_plan(pl);
  if (st) return st;
  if (!tr || !y || !S || !x) return fail(ISG_ERR_INVALID_ARG, "NULL argument");
  if (tr->plan != pl) return fail(ISG_ERR_INVALID_ARG, "trajectory belongs to another plan");
  for (int i = 0; i < 3; ++i)
    if (tr->ts[i] != pl->ktile.TS[i])
      return fail(ISG_ERR_STATE, "trajectory was prepared for another k-space tile shape: re-create it");
  return guarded(pl, [&]() -> isg_status {
    op_grid_recon(pl, tr, (const float2*)y, w, (const float2*)S, (float2*)x);
    return ISG_OK;
  });
}

}  // extern "C"
