// bq_lib.hip -- host side of libbq (C ABI in include/bq.h) plus the set-up,
// state-transfer and diagnostic kernels.  The per-step kernels live in
// bq_kernels.hpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <algorithm>
#include <atomic>
#include <mutex>
#include <type_traits>
#include <vector>

#include "bq.h"
#include "bq_kernels.hpp"

using namespace bqk;

// ---------------------------------------------------------------------------
// tile shapes per precision
// ---------------------------------------------------------------------------
// A tile is 64 cells wide and TY tall (TY = the y-chunk length of the line
// solves); x-lines are cut into chunks of MX cells (a divisor of 64).  The
// shape is a runtime choice of a domain (and of a batch, whose members share
// it), among the candidates below, the first being the default; the
// workspace is laid out for all of them (fields padded for the tallest tile,
// chunk and tile tables for the shortest chunks), so a domain changes shape
// between steps without moving its state.
struct Shape {
  int ty, mx;
};
template <typename T> struct Cfg;
template <> struct Cfg<float> {
  static constexpr int NS = 4, TYMAX = 16, TYMIN = 8, MXMIN = 16;
  static constexpr Shape shape(int k) {
    return k == 0 ? Shape{16, 16} : k == 1 ? Shape{16, 32} : k == 2 ? Shape{8, 16} : Shape{8, 32};
  }
};
template <> struct Cfg<double> {
  static constexpr int NS = 3, TYMAX = 8, TYMIN = 4, MXMIN = 16;
  static constexpr Shape shape(int k) { return k == 0 ? Shape{8, 16} : k == 1 ? Shape{8, 32} : Shape{4, 16}; }
};
template <typename T>
static bool shape_ok(int ty, int mx) {
  for (int k = 0; k < Cfg<T>::NS; ++k)
    if (Cfg<T>::shape(k).ty == ty && Cfg<T>::shape(k).mx == mx) return true;
  return false;
}
template <int V>
using IC = std::integral_constant<int, V>;
// f(IC<TY>, IC<MX>) for the shape (ty, mx), which shape_ok<T> has accepted
template <typename T, typename F>
static void shape_dispatch(int ty, int mx, F&& f) {
  if constexpr (sizeof(T) == 4) {
    if (ty == 16 && mx == 16) f(IC<16>{}, IC<16>{});
    else if (ty == 16) f(IC<16>{}, IC<32>{});
    else if (mx == 16) f(IC<8>{}, IC<16>{});
    else f(IC<8>{}, IC<32>{});
  } else {
    if (ty == 8 && mx == 16) f(IC<8>{}, IC<16>{});
    else if (ty == 8) f(IC<8>{}, IC<32>{});
    else f(IC<4>{}, IC<16>{});
  }
}

static thread_local char g_err[512] = "";

static int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) return fail(BQ_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

static size_t rup(size_t v, size_t a) { return (v + a - 1) / a * a; }
static int cdiv(int a, int b) { return (a + b - 1) / b; }

// Streams, events and graph executables the library creates, counted while
// alive (bq_live_handles), so a test can check that freeing a batch or a
// domain releases everything it made.
static std::atomic<int> g_live[3];   // streams, events, graph execs
static hipError_t stream_new(hipStream_t* s) {
  const hipError_t e = hipStreamCreateWithFlags(s, hipStreamNonBlocking);
  if (e == hipSuccess) ++g_live[0];
  return e;
}
static void stream_del(hipStream_t& s) {
  if (s && hipStreamDestroy(s) == hipSuccess) --g_live[0];
  s = nullptr;
}
static hipError_t event_new(hipEvent_t* ev, bool timing) {
  const hipError_t e = timing ? hipEventCreate(ev) : hipEventCreateWithFlags(ev, hipEventDisableTiming);
  if (e == hipSuccess) ++g_live[1];
  return e;
}
static void event_del(hipEvent_t& ev) {
  if (ev && hipEventDestroy(ev) == hipSuccess) --g_live[1];
  ev = nullptr;
}
static hipError_t graph_new(hipGraphExec_t* x, hipGraph_t g) {
  const hipError_t e = hipGraphInstantiate(x, g, nullptr, nullptr, 0);
  if (e == hipSuccess) ++g_live[2];
  return e;
}
static void graph_del(hipGraphExec_t& x) {
  if (x && hipGraphExecDestroy(x) == hipSuccess) --g_live[2];
  x = nullptr;
}

// ---------------------------------------------------------------------------
// set-up kernels
// ---------------------------------------------------------------------------

// corner still-water depth with two mirrored ghost layers, from io (FP64
// (ny+1) x (nx+1) host copy)
template <typename T>
__global__ void k_setup_corners(const DomDev<T>* Dp) {
  const DomDev<T>& D = *Dp;
  const int w = D.nx + 5, h = D.ny + 5;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= w * h) return;
  const int ic = e % w - 2, jc = e / w - 2;
  const int mi = ic < 0 ? -ic : (ic > D.nx ? 2 * D.nx - ic : ic);
  const int mj = jc < 0 ? -jc : (jc > D.ny ? 2 * D.ny - jc : jc);
  D.Dc[(size_t)(jc + 2) * D.cpitch + ic + 2] = (T)D.io[(size_t)mj * (D.nx + 1) + mi];
}

template <typename T>
__device__ __forceinline__ T corner(const DomDev<T>& D, int ic, int jc) {
  return D.Dc[(size_t)(jc + 2) * D.cpitch + ic + 2];
}

template <typename T>
__device__ __forceinline__ T cellD(const DomDev<T>& D, int i, int j) {
  return dbar4(corner(D, i, j), corner(D, i + 1, j), corner(D, i, j + 1), corner(D, i + 1, j + 1));
}

template <typename T>
__global__ void k_setup_cells(const DomDev<T>* Dp) {
  const DomDev<T>& D = *Dp;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D.nx * D.ny) return;
  const int i = e % D.nx, j = e / D.nx;
  D.Dbar[(size_t)j * D.ipitch + i] = cellD(D, i, j);
}

// spikes of the chunk-local systems: responses to a unit value of the
// neighbour just left (v) and right (w) of the chunk; only their end values
// are kept, in rs[0..3] (v_first, v_last, w_first, w_last)
template <typename T, int M>
__global__ void k_setup_spikes(const DomDev<T>* Dp, int dir) {
  const DomDev<T>& D = *Dp;
  const int L = dir == 0 ? D.ny : D.nx;           // lines
  const int C = dir == 0 ? D.cx : D.cy;           // chunks per line
  const int n = dir == 0 ? D.nx : D.ny;           // unknowns per line
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= L * C) return;
  const int line = e % L, c = e / L;
  const int s = c * M, m = min(M, n - s);
  const T* tc = dir == 0 ? D.tcx : D.tcy;
  T Dl[M + 2], r[M];
  for (int k = 0; k < m + 2; ++k) {
    const int q = s - 1 + k;
    Dl[k] = dir == 0 ? cellD(D, q, line) : cellD(D, line, q);
  }
  const bool wave_w = dir == 0 && west_driven(D.bc[0]);
  const bool fold_lo = s == 0 && !wave_w, fold_hi = s + m == n;
  T a0, b0, c0, am, bm, cm;
  tri_coef(dpos(Dl[0]), dpos(Dl[1]), dpos(Dl[2]), tc, a0, b0, c0);
  tri_coef(dpos(Dl[m - 1]), dpos(Dl[m]), dpos(Dl[m + 1]), tc, am, bm, cm);
  T* rs = dir == 0 ? D.rsx : D.rsy;
  const size_t CL = (size_t)C * L, o = (size_t)c * L + line;
  // left spike
  for (int k = 0; k < m; ++k) r[k] = T(0);
  if (c > 0) {
    r[0] = -a0;
    chunk_solve_db<T, M>(Dl, 1, m, tc, fold_lo, fold_hi, r, 1);
  }
  rs[o] = r[0];
  rs[CL + o] = r[m - 1];
  // right spike
  for (int k = 0; k < m; ++k) r[k] = T(0);
  if (c < C - 1) {
    r[m - 1] = -cm;
    chunk_solve_db<T, M>(Dl, 1, m, tc, fold_lo, fold_hi, r, 1);
  }
  rs[2 * CL + o] = r[0];
  rs[3 * CL + o] = r[m - 1];
}

// static coefficients of the interface recurrence (see reduce_line)
template <typename T>
__global__ void k_setup_reduced(const DomDev<T>* Dp, int dir) {
  const DomDev<T>& D = *Dp;
  const int L = dir == 0 ? D.ny : D.nx;
  const int C = dir == 0 ? D.cx : D.cy;
  const int line = blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= L) return;
  T* rs = dir == 0 ? D.rsx : D.rsy;
  const size_t CL = (size_t)C * L;
  T gprev = T(0);
  for (int c = 0; c < C; ++c) {
    const size_t o = (size_t)c * L + line;
    const T vs = rs[o], ve = rs[CL + o], ws = rs[2 * CL + o], we = rs[3 * CL + o];
    const T kap = T(1) / (T(1) - vs * gprev);
    const T tau = kap * ws;
    const T gam = ve * gprev * tau + we;
    rs[o] = kap;
    rs[CL + o] = kap * vs;
    rs[2 * CL + o] = ve;
    rs[3 * CL + o] = ve * gprev;
    rs[4 * CL + o] = tau;
    rs[5 * CL + o] = gam;
    gprev = gam;
  }
}

// wave numbers of the wavemaker components: the linear dispersion relation of
// Eq. (1)-(3) on a flat bed is a quadratic in k^2,
//   g B d^3 K^2 + (g d - w^2 (B + 1/3) d^2) K - w^2 = 0,  K = k^2,
// with exactly one positive root; d = mean still-water depth of column 0.
template <typename T>
__global__ void k_setup_waves(const DomDev<T>* Dp, double B) {
  const DomDev<T>& D = *Dp;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double dsum = 0.0;
  for (int j = 0; j < D.ny; ++j) dsum += (double)dpos(D.Dbar[(size_t)j * D.ipitch]);
  const double d = dsum / D.ny;
  const int nw = D.n_waves;
  for (int m = 0; m < nw; ++m) {
    const double om = D.wave[nw + m];
    double k = 0.0;
    if (d > 0.0 && om > 0.0) {
      const double a = D.g_d * B * d * d * d;
      const double b = D.g_d * d - om * om * (B + 1.0 / 3.0) * d * d;
      const double disc = sqrt(b * b + 4.0 * a * om * om);
      const double K = b >= 0.0 ? 2.0 * om * om / (b + disc) : (disc - b) / (2.0 * a);
      k = sqrt(K);
    }
    D.wave[3 * nw + m] = k;
  }
}

// ---------------------------------------------------------------------------
// state transfer, ghosts and diagnostics
// ---------------------------------------------------------------------------

// scatter io (FP64 interior) into level 0: which 0 = eta -> w, 1 = P, 2 = Q
template <typename T>
__global__ void k_scatter(const DomDev<T>* Dp, int which, int* bad) {
  const DomDev<T>& D = *Dp;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D.nx * D.ny) return;
  const int i = e % D.nx, j = e / D.nx;
  const double v = D.io[e];
  const size_t g = (size_t)(j + 2) * D.pitch + D.xoff + i;
  if (which == 0) {
    const double Db = (double)D.Dbar[(size_t)j * D.ipitch + i];
    const double d = Db > 0.0 ? Db : 0.0;
    if (!(v + d >= 0.0)) atomicOr(bad, 1);
    // w = h + b with h = eta + d, b = -Dbar
    D.w[0][g] = (T)(v + d - Db);
  } else if (which == 1) {
    D.P[0][g] = (T)v;
  } else {
    D.Q[0][g] = (T)v;
  }
}

// ghosts of level 0 at t = 0 and the CFL maximum of the initial state
template <typename T>
__global__ void __launch_bounds__(256) k_init_ghosts(const DomDev<T>* Dp) {
  const DomDev<T>& D = *Dp;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  double sm = 0.0;
  if (e < D.nx * D.ny) {
    const int i = e % D.nx, j = e / D.nx;
    const size_t g = (size_t)(j + 2) * D.pitch + D.xoff + i;
    const T wv = D.w[0][g], p = D.P[0][g], qv = D.Q[0][g];
    ghost_cell(D, D.w[0], D.P[0], D.Q[0], i, j, wv, p, qv, D.st->gw, D.st->gP);
    const T h = fmax(wv + D.Dbar[(size_t)j * D.ipitch + i], T(0));
    if (D.runup) D.wmax[(size_t)j * D.ipitch + i] = h > D.runup_delta ? wv : (T)__builtin_nan("");
    const T u = desing(p, h, D.eps), v = desing(qv, h, D.eps);
    const T c = sqrt(D.g * h);
    const T sx = (fabs(u) + c) / D.dx, sy = (fabs(v) + c) / D.dy;
    sm = (sx != sx || sy != sy) ? __longlong_as_double(0x7ff0000000000000ll) : (double)fmax(sx, sy);
  }
  for (int o = 32; o > 0; o >>= 1) sm = fmax(sm, __shfl_xor(sm, o, 64));
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sm;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    atomicMax(&D.st->smax_bits, (unsigned long long)__double_as_longlong(m));
  }
}

// wavemaker ghost values at t = 0 (one block)
template <typename T>
__global__ void __launch_bounds__(64) k_init_waves(const DomDev<T>* Dp) {
  const DomDev<T>& D = *Dp;
  double gw[2], gP[2];
  west_ghosts(D, D.st->t, gw, gP);
  if (threadIdx.x == 0) {
    D.st->gw[0] = gw[0]; D.st->gw[1] = gw[1]; D.st->gP[0] = gP[0]; D.st->gP[1] = gP[1];
  }
}

// gather the current level into io: which 0 eta, 1 P, 2 Q, 3 w, 4 run-up
// record, 5 local CFL number with the last step's Delta t
template <typename T>
__global__ void k_gather(const DomDev<T>* Dp, int which, int wslot, int pslot) {
  const DomDev<T>& D = *Dp;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D.nx * D.ny) return;
  const int i = e % D.nx, j = e / D.nx;
  const size_t g = (size_t)(j + 2) * D.pitch + D.xoff + i;
  double v;
  if (which == 0 || which == 3) {
    const double wv = (double)D.w[wslot][g];
    const double Db = (double)D.Dbar[(size_t)j * D.ipitch + i];
    v = which == 3 ? wv : (wv + Db) - (Db > 0.0 ? Db : 0.0);
  } else if (which == 4) {
    v = (double)D.wmax[(size_t)j * D.ipitch + i];
  } else if (which == 5) {
    // Eq. (22) in the field precision, as the step's CFL maximum
    const T wv = D.w[wslot][g], p = D.P[pslot][g], qv = D.Q[pslot][g];
    const T h = fmax(wv + D.Dbar[(size_t)j * D.ipitch + i], T(0));
    const T u = desing(p, h, D.eps), vv = desing(qv, h, D.eps);
    const T c = sqrt(D.g * h);
    v = D.st->dt1 * (double)fmax((fabs(u) + c) / D.dx, (fabs(vv) + c) / D.dy);
  } else {
    v = (double)(which == 1 ? D.P[pslot][g] : D.Q[pslot][g]);
  }
  D.io[e] = v;
}

__device__ __forceinline__ int cdiv_d(int a, int b) { return (a + b - 1) / b; }

// FP64 mass and energy: fixed partition (block b takes a contiguous run of
// rows) and fixed-order trees, so the sums are reproducible
template <typename T>
__global__ void __launch_bounds__(256) k_diag_part(const DomDev<T>* Dp, int wslot, int pslot) {
  const DomDev<T>& D = *Dp;
  const int R = cdiv_d(D.ny, NDIAG), j0 = blockIdx.x * R, j1 = min(D.ny, j0 + R);
  double m = 0.0, en = 0.0;
  for (int j = j0; j < j1; ++j)
    for (int i = threadIdx.x; i < D.nx; i += 256) {
      const size_t g = (size_t)(j + 2) * D.pitch + D.xoff + i;
      const double Db = (double)D.Dbar[(size_t)j * D.ipitch + i];
      const double h = (double)D.w[wslot][g] + Db;
      const double d = Db > 0.0 ? Db : 0.0;
      m += h;
      double ec = 0.0;
      if (d > 0.0) ec += 0.5 * D.g_d * (h - d) * (h - d);
      if (h > 1e-6) {
        const double p = (double)D.P[pslot][g], q = (double)D.Q[pslot][g];
        ec += 0.5 * (p * p + q * q) / h;
      }
      en += ec;
    }
  __shared__ double sm[256], se[256];
  sm[threadIdx.x] = m;
  se[threadIdx.x] = en;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sm[threadIdx.x] += sm[threadIdx.x + s];
      se[threadIdx.x] += se[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    D.diag_part[blockIdx.x] = sm[0];
    D.diag_part[NDIAG + blockIdx.x] = se[0];
  }
}

// sum of the partials (fixed tree); the per-tile CFL maxima are folded into
// the state's maximum for reporting (idempotent for the next Delta t)
template <typename T>
__global__ void __launch_bounds__(NDIAG) k_diag_final(const DomDev<T>* Dp) {
  const DomDev<T>& D = *Dp;
  __shared__ double sm[NDIAG], se[NDIAG], sx[NDIAG];
  sm[threadIdx.x] = D.diag_part[threadIdx.x];
  se[threadIdx.x] = D.diag_part[NDIAG + threadIdx.x];
  double mx = 0.0;
  const int ntiles = D.tiles_x * D.tiles_y;
  for (int k = threadIdx.x; k < ntiles; k += NDIAG) mx = fmax(mx, D.smax_tile[k]);
  sx[threadIdx.x] = mx;
  __syncthreads();
  for (int s = NDIAG / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sm[threadIdx.x] += sm[threadIdx.x + s];
      se[threadIdx.x] += se[threadIdx.x + s];
      sx[threadIdx.x] = fmax(sx[threadIdx.x], sx[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    D.st->mass = sm[0] * D.dx_d * D.dy_d;
    D.st->energy = se[0] * D.dx_d * D.dy_d;
    const double s0 = __longlong_as_double((long long)D.st->smax_bits);
    D.st->smax_bits = (unsigned long long)__double_as_longlong(fmax(s0, sx[0]));
  }
}

// Plain device copy, one 16-byte vector per lane: the HBM bandwidth
// reference the step's kernels are measured against (bq_stream_copy).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_stream_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Before a change of tile shape: fold the per-tile CFL maxima of the old
// tiling (written by the finalize kernel for the next step's Delta t) into
// the state's maximum, then clear every slot, so the next Delta t sees the
// same maximum under the new tiling.
template <typename T>
__global__ void __launch_bounds__(256) k_fold_tiles(const DomDev<T>* Dp, int ntiles_old, int ntiles_max) {
  const DomDev<T>& D = *Dp;
  double m = 0.0;
  for (int k = threadIdx.x; k < ntiles_old; k += 256) m = fmax(m, D.smax_tile[k]);
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double mm = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const double s0 = __longlong_as_double((long long)D.st->smax_bits);
    D.st->smax_bits = (unsigned long long)__double_as_longlong(fmax(s0, mm));
  }
  for (int k = threadIdx.x; k < ntiles_max; k += 256) D.smax_tile[k] = 0.0;
}

// ---------------------------------------------------------------------------
// host objects
// ---------------------------------------------------------------------------

struct Launch {
  // device tables of one launch group (a domain or a batch)
  void* table = nullptr;        // DomDev<T>[nd]
  int* tile_map = nullptr;      // per tile: domain << MAP_SHIFT | tile (batches; NULL for one domain)
  int* line_map = nullptr;      // per line: domain << MAP_SHIFT | line
  void* status = nullptr;       // StatusRec[nd]: staging of bq_batch_status (batches)
  int nd = 0, tiles = 0, lines = 0;
  int ty = 0, mx = 0;           // tile shape shared by the members
  int any_pc = 0;               // some member runs the corrector pass
  // schedule (tuned per batch): threads per block of the line-coupling
  // kernel, XCD-aware tile order of the stencil kernel
  int rblock = 256;
  int swizzle = 1;
  int segs = 1;                 // 1: one thread per line; 4 or 8: segmented sweeps
  hipGraphExec_t graph = nullptr;
  int graph_steps = 0;          // steps per replay (0 = none)
  int graph_built = 0;          // steps captured in `graph`
};

struct bq_domain {
  bq_params p;
  std::vector<double> wamp, womg, wph;
  std::vector<double> ts;       // time-series samples: eta then P
  int precision = BQ_FP64;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int nx = 0, ny = 0;
  DomDev<float> df;
  DomDev<double> dd;
  void* ddev = nullptr;         // device DomDev<T>
  DevState* st = nullptr;
  Launch L;                     // tables in the workspace
  int graph_steps = 16;
};

constexpr int MAX_LANES = 4;     // launch lanes of a batch (hardware queues per process)

struct bq_batch {
  std::vector<bq_domain*> doms;
  int precision = BQ_FP64;
  hipStream_t stream = nullptr;
  void* mem = nullptr;          // tables of L and of the lane groups G[]
  size_t mem_bytes = 0;
  Launch L;                     // all members, one lane
  // Several lanes: the members split into groups of about equal cell
  // count, each advanced on a stream of its own, so one group's stencil
  // kernel (arithmetic-bound) runs beside another group's line-coupling and
  // finalize kernels (bandwidth- and latency-bound).  The batch creates the
  // lane streams itself, one right after the other, so the runtime puts them
  // on different hardware queues (two streams sharing a queue run one after
  // the other, and their lanes would not overlap).
  Launch G[MAX_LANES];
  int lanes_req = 2;            // requested lanes (1 .. MAX_LANES)
  int lanes = 1;                // lanes in use (at most the member count)
  hipStream_t lane[MAX_LANES] = {};
  hipEvent_t ev_fork = nullptr, ev_join[MAX_LANES] = {};
  int graph_steps = 16;
  int rblock = 256, swizzle = 1, segs = 1;  // schedule copied into the launches
  int static_dev = -1;          // >= 0: tables in that device's static array (bq_batch_set_static)
  int ty = 0, mx = 0;           // tile shape of the members (0: the first member's)
};

// ---------------------------------------------------------------------------
// static table memory (bq_batch_set_static)
// ---------------------------------------------------------------------------
// One fixed array per GPU holds the device tables of the batch that last
// called bq_batch_set_static on it, so that call allocates no device memory.
// In host code `scratch` only names the symbol: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) unsigned char scratch[BQ_STATIC_TABLE_BYTES];
constexpr int MAX_DEVICES = 64;
static std::mutex g_static_mu;
static char* g_static_ptr[MAX_DEVICES];        // device address of `scratch` per device
static bq_batch* g_static_owner[MAX_DEVICES];  // batch whose tables it holds

// address of the current device's array (looked up on the first use there)
static int static_tables(int* dev_out, char** ptr_out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(BQ_EDEVICE, "device %d out of range for static tables", dev);
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(BQ_EDEVICE, "hipGetSymbolAddress returned NULL");
    g_static_ptr[dev] = (char*)p;
  }
  *dev_out = dev;
  *ptr_out = g_static_ptr[dev];
  return BQ_OK;
}

// a batch on static tables may run only while it still owns them
static int static_owner_ok(const bq_batch* b) {
  if (b->static_dev < 0) return BQ_OK;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (g_static_owner[b->static_dev] != b)
    return fail(BQ_ESTATE, "another batch has taken this device's static tables; call bq_batch_set_static again");
  return BQ_OK;
}

// layout of a domain in its workspace
struct Layout {
  size_t off_state, off_desc;
  size_t off_w, off_P, off_Q, off_E, off_F, off_G, off_part, off_wmax;
  size_t off_Dc, off_Dbar, off_xhP, off_xhQ;
  size_t off_chx, off_chy, off_rsx, off_rsy, off_ifx, off_ify, off_wave, off_io;
  size_t ghosted, interior, corners, total;
  // sizes for every tile shape: chunks per line (shortest chunks), tiles
  // (shortest tiles)
  int pitch, xoff, ipitch, cpitch, cx, cy, tiles_x, tiles_max;
};

template <typename T>
static Layout layout_for(const bq_params* p) {
  Layout L{};
  const int nx = p->nx, ny = p->ny;
  const int A = 256 / (int)sizeof(T);
  L.cx = cdiv(nx, Cfg<T>::MXMIN);
  L.cy = cdiv(ny, Cfg<T>::TYMIN);
  L.tiles_x = cdiv(nx, TX);
  L.tiles_max = L.tiles_x * cdiv(ny, Cfg<T>::TYMIN);
  // fields are padded to whole tiles of the tallest shape plus the stencil
  // halo, so the stencil kernel reads every tile of every shape without
  // clamping its indices
  const int NX = L.tiles_x * TX, NY = cdiv(ny, Cfg<T>::TYMAX) * Cfg<T>::TYMAX;
  L.xoff = A;
  L.pitch = (int)rup((size_t)A + NX + 2, (size_t)A);
  L.ipitch = NX;
  L.cpitch = (int)rup((size_t)NX + 5, 64);
  L.ghosted = (size_t)(NY + 4) * L.pitch * sizeof(T);
  L.interior = (size_t)NY * L.ipitch * sizeof(T);
  L.corners = (size_t)(NY + 5) * L.cpitch * sizeof(T);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = rup(o + bytes, 256);
    return at;
  };
  L.off_state = take(sizeof(DevState));
  L.off_desc = take(sizeof(DomDev<T>));
  L.off_w = take((p->corrector ? 3 : 2) * L.ghosted);   // + the predicted surface
  L.off_P = take(3 * L.ghosted);
  L.off_Q = take(3 * L.ghosted);
  L.off_E = take(3 * L.interior);
  L.off_F = take(3 * L.interior);
  L.off_G = take(3 * L.interior);
  // per-tile CFL maxima and diagnostic partial sums (zeroed by set_state,
  // part of the checkpoint)
  L.off_part = take(sizeof(double) * ((size_t)L.tiles_max + 2 * NDIAG));
  L.off_wmax = take(p->runup_delta > 0.0 ? L.interior : 0);   // run-up record (checkpointed)
  L.off_Dc = take(L.corners);
  L.off_Dbar = take(L.interior);
  L.off_xhP = take(L.interior);
  L.off_xhQ = take(L.interior);
  L.off_chx = take(2 * (size_t)L.cx * ny * sizeof(T));
  L.off_chy = take(2 * (size_t)L.cy * nx * sizeof(T));
  L.off_rsx = take(6 * (size_t)L.cx * ny * sizeof(T));
  L.off_rsy = take(6 * (size_t)L.cy * nx * sizeof(T));
  L.off_ifx = take(2 * (size_t)L.cx * ny * sizeof(T));
  L.off_ify = take(2 * (size_t)L.cy * nx * sizeof(T));
  const size_t nwave = 4 * (size_t)(p->n_waves > 0 ? p->n_waves : 1);
  const size_t nser = p->bc[0] == BQ_TIMESERIES ? 2 * (size_t)p->ts_n : 0;
  L.off_wave = take((nwave > nser ? nwave : nser) * sizeof(double));
  L.off_io = take((size_t)(nx + 1) * (ny + 1) * sizeof(double));
  L.total = o;
  return L;
}

// elements of the largest padded field of a domain
template <typename T>
static size_t max_field_elements(const bq_params* p) {
  const Layout L = layout_for<T>(p);
  const size_t b = std::max(L.ghosted, std::max(L.interior, L.corners));
  return b / sizeof(T);
}

static int check_params(const bq_params* p) {
  if (!p) return fail(BQ_EINVAL, "params is NULL");
  if (p->nx < 4 || p->ny < 4) return fail(BQ_EINVAL, "nx, ny must be >= 4 (got %d, %d)", p->nx, p->ny);
  if ((double)p->nx * p->ny > 2.0e9) return fail(BQ_EINVAL, "domain too large");
  if (!(p->dx > 0) || !(p->dy > 0)) return fail(BQ_EINVAL, "dx, dy must be > 0");
  if (!(p->g > 0)) return fail(BQ_EINVAL, "g must be > 0");
  if (!(p->cfl > 0) || !(p->dt_max > 0) || !(p->dt_min >= 0)) return fail(BQ_EINVAL, "bad cfl / dt_max / dt_min");
  if (!(p->ema_alpha > 0 && p->ema_alpha <= 1)) return fail(BQ_EINVAL, "ema_alpha must be in (0, 1]");
  if (p->fixed_dt && !(p->dt_init > 0)) return fail(BQ_EINVAL, "fixed_dt needs dt_init > 0");
  if (!(p->theta == 0.0 || (p->theta >= 1.0 && p->theta <= 2.0))) return fail(BQ_EINVAL, "theta must be 0 or in [1, 2]");
  for (int s = 0; s < 4; ++s) {
    if (p->bc[s] < 0 || p->bc[s] > 4) return fail(BQ_EINVAL, "bad boundary type on side %d", s);
    if (s > 0 && west_driven(p->bc[s]))
      return fail(BQ_EINVAL, "wavemakers and time series are supported on the west side only");
  }
  if (p->bc[0] == BQ_TIMESERIES &&
      (p->ts_n < 1 || p->ts_n > (1 << 26) || !(p->ts_dt > 0) || !p->ts_eta || !p->ts_P))
    return fail(BQ_EINVAL, "a time-series boundary needs 1 <= ts_n <= 2^26 samples, ts_dt > 0 and both arrays");
  if (!(p->friction_f >= 0) || !(p->manning_n >= 0)) return fail(BQ_EINVAL, "friction coefficients must be >= 0");
  if (!(p->runup_delta >= 0)) return fail(BQ_EINVAL, "runup_delta must be >= 0");
  if (p->corrector != 0 && p->corrector != 1) return fail(BQ_EINVAL, "corrector must be 0 or 1");
  const bool wave = p->bc[0] == BQ_SINE || p->bc[0] == BQ_IRREGULAR;
  if (p->n_waves < 0 || p->n_waves > BQ_MAX_WAVES) return fail(BQ_EINVAL, "n_waves out of range");
  if (wave && (p->n_waves < 1 || !p->wave_amp || !p->wave_omega))
    return fail(BQ_EINVAL, "a wavemaker needs n_waves >= 1 with amplitudes and frequencies");
  if (p->fstar_order < 0 || p->fstar_order > 2) return fail(BQ_EINVAL, "fstar_order must be 0, 1 or 2");
  if (p->precision != BQ_FP64 && p->precision != BQ_FP32) return fail(BQ_EINVAL, "bad precision");
  {
    // the kernels index a field by 32-bit element offsets (row times pitch
    // plus column, in int arithmetic): every padded field, with its halo
    // and its padding to whole tiles, must stay below 2^31 elements
    const size_t el = p->precision == BQ_FP32 ? max_field_elements<float>(p) : max_field_elements<double>(p);
    if (el >= ((size_t)1 << 31))
      return fail(BQ_EINVAL, "domain too large: a padded field of %zu elements exceeds 32-bit offsets", el);
  }
  // the forcing must be finite (the kernels take it as given)
  if (p->bc[0] == BQ_TIMESERIES)
    for (int k = 0; k < p->ts_n; ++k)
      if (!std::isfinite(p->ts_eta[k]) || !std::isfinite(p->ts_P[k]))
        return fail(BQ_EINVAL, "time-series sample %d is not finite", k);
  if (wave)
    for (int m = 0; m < p->n_waves; ++m)
      if (!std::isfinite(p->wave_amp[m]) || !std::isfinite(p->wave_omega[m]) ||
          (p->wave_phase && !std::isfinite(p->wave_phase[m])))
        return fail(BQ_EINVAL, "wave component %d is not finite", m);
  return BQ_OK;
}

template <typename T>
static DomDev<T>& desc(bq_domain* d);
template <>
DomDev<float>& desc<float>(bq_domain* d) { return d->df; }
template <>
DomDev<double>& desc<double>(bq_domain* d) { return d->dd; }

// static data of the chunked line solves for the domain's current shape:
// the chunk spikes' end values, then the interface-recurrence coefficients
template <typename T>
static void setup_chunks(const DomDev<T>& D, const DomDev<T>* Dd, hipStream_t s) {
  shape_dispatch<T>(D.my, D.mx, [&](auto tyc, auto mxc) {
    constexpr int TY = decltype(tyc)::value, MX = decltype(mxc)::value;
    k_setup_spikes<T, MX><<<cdiv(D.ny * D.cx, 64), 64, 0, s>>>(Dd, 0);
    k_setup_spikes<T, TY><<<cdiv(D.nx * D.cy, 64), 64, 0, s>>>(Dd, 1);
  });
  k_setup_reduced<T><<<cdiv(D.ny, 64), 64, 0, s>>>(Dd, 0);
  k_setup_reduced<T><<<cdiv(D.nx, 64), 64, 0, s>>>(Dd, 1);
}

template <typename T>
static int create_t(bq_domain* d, const double* depth_c) {
  const bq_params* p = &d->p;
  const Layout Ly = layout_for<T>(p);
  if (d->ws_bytes < Ly.total) return fail(BQ_ENOMEM, "workspace of %zu bytes, need %zu", d->ws_bytes, Ly.total);
  char* b = d->ws;
  DomDev<T>& D = desc<T>(d);
  memset(&D, 0, sizeof(D));
  D.nx = p->nx;
  D.ny = p->ny;
  D.pitch = Ly.pitch;
  D.xoff = Ly.xoff;
  D.ipitch = Ly.ipitch;
  D.cpitch = Ly.cpitch;
  const Shape sh0 = Cfg<T>::shape(0);
  D.cx = cdiv(p->nx, sh0.mx);
  D.cy = cdiv(p->ny, sh0.ty);
  D.mx = sh0.mx;
  D.my = sh0.ty;
  D.tiles_x = Ly.tiles_x;
  D.tiles_y = cdiv(p->ny, sh0.ty);
  for (int s = 0; s < 4; ++s) {
    D.bc[s] = p->bc[s];
    D.sponge_w[s] = (T)p->sponge_width[s];
    if (p->bc[s] == BQ_SPONGE && p->sponge_width[s] > 0.0 && p->sponge_sigma > 0.0) D.any_sponge = 1;
  }
  D.fstar_order = p->fstar_order == 1 ? 1 : 2;
  D.fixed_dt = p->fixed_dt;
  const bool wave = p->bc[0] == BQ_SINE || p->bc[0] == BQ_IRREGULAR;
  D.n_waves = wave ? p->n_waves : 0;
  D.dx = (T)p->dx;
  D.dy = (T)p->dy;
  D.g = (T)p->g;
  D.B = (T)p->B;
  D.Bc = (T)(p->B + 1.0 / 3.0);
  D.gn2 = (T)(p->g * p->manning_n * p->manning_n);
  D.cf = (T)p->friction_f;
  D.ts_n = p->bc[0] == BQ_TIMESERIES ? p->ts_n : 0;
  D.ts_dt = p->ts_dt;
  D.runup = p->runup_delta > 0.0 ? 1 : 0;
  D.corrector = p->corrector ? 1 : 0;
  D.runup_delta = (T)p->runup_delta;
  {
    const double dx = p->dx, dy = p->dy, bc = p->B + 1.0 / 3.0;
    D.idx = (T)(1.0 / dx);
    D.idy = (T)(1.0 / dy);
    D.i2dx = (T)(1.0 / (2.0 * dx));
    D.i2dy = (T)(1.0 / (2.0 * dy));
    D.idx2 = (T)(1.0 / (dx * dx));
    D.idy2 = (T)(1.0 / (dy * dy));
    D.i4dxdy = (T)(1.0 / (4.0 * dx * dy));
    D.i2dx3 = (T)(1.0 / (2.0 * dx * dx * dx));
    D.i2dy3 = (T)(1.0 / (2.0 * dy * dy * dy));
    D.i2dxdy2 = (T)(1.0 / (2.0 * dx * dy * dy));
    D.i2dx2dy = (T)(1.0 / (2.0 * dx * dx * dy));
    D.tcx[0] = (T)(1.0 / (2.0 * dx));
    D.tcx[1] = (T)(bc / (dx * dx));
    D.tcx[2] = (T)(1.0 / (6.0 * dx));
    D.tcy[0] = (T)(1.0 / (2.0 * dy));
    D.tcy[1] = (T)(bc / (dy * dy));
    D.tcy[2] = (T)(1.0 / (6.0 * dy));
  }
  D.theta = (T)p->theta;
  const double eps = p->eps_desing > 0 ? p->eps_desing : fmax(pow(p->dx, 4), pow(p->dy, 4));
  D.eps = (T)eps;
  D.sponge_sigma = (T)p->sponge_sigma;
  D.dx_d = p->dx;
  D.dy_d = p->dy;
  D.g_d = p->g;
  D.cfl = p->cfl;
  D.ema_alpha = p->ema_alpha;
  D.dt_init = p->dt_init;
  D.dt_max = p->dt_max;
  D.dt_min = p->dt_min;
  D.wave_ramp = p->wave_ramp;
  D.t_end = p->t_end;
  for (int k = 0; k < 3; ++k) D.w[k] = k < 2 || D.corrector ? (T*)(b + Ly.off_w + k * Ly.ghosted) : nullptr;
  for (int k = 0; k < 3; ++k) {
    D.P[k] = (T*)(b + Ly.off_P + k * Ly.ghosted);
    D.Q[k] = (T*)(b + Ly.off_Q + k * Ly.ghosted);
    D.E[k] = (T*)(b + Ly.off_E + k * Ly.interior);
    D.F[k] = (T*)(b + Ly.off_F + k * Ly.interior);
    D.G[k] = (T*)(b + Ly.off_G + k * Ly.interior);
  }
  D.Dc = (T*)(b + Ly.off_Dc);
  D.Dbar = (T*)(b + Ly.off_Dbar);
  D.xhP = (T*)(b + Ly.off_xhP);
  D.xhQ = (T*)(b + Ly.off_xhQ);
  D.chx = (T*)(b + Ly.off_chx);
  D.chy = (T*)(b + Ly.off_chy);
  D.rsx = (T*)(b + Ly.off_rsx);
  D.rsy = (T*)(b + Ly.off_rsy);
  D.ifx = (T*)(b + Ly.off_ifx);
  D.ify = (T*)(b + Ly.off_ify);
  D.smax_tile = (double*)(b + Ly.off_part);
  D.diag_part = D.smax_tile + (size_t)Ly.tiles_max;
  D.wave = (double*)(b + Ly.off_wave);
  D.wmax = D.runup ? (T*)(b + Ly.off_wmax) : nullptr;
  D.io = (double*)(b + Ly.off_io);
  D.st = (DevState*)(b + Ly.off_state);
  d->st = D.st;
  d->ddev = b + Ly.off_desc;
  hipStream_t s = d->stream;
  HIPCHK(hipMemsetAsync(d->ws, 0, Ly.total, s));
  HIPCHK(hipMemcpyAsync(d->ddev, &D, sizeof(D), hipMemcpyHostToDevice, s));
  // tables of the single-domain launch group
  d->L.table = d->ddev;
  d->L.tile_map = d->L.line_map = nullptr;
  d->L.nd = 1;
  d->L.any_pc = D.corrector;
  d->L.tiles = D.tiles_x * D.tiles_y;
  d->L.lines = p->nx + p->ny;
  d->L.ty = sh0.ty;
  d->L.mx = sh0.mx;
  if (D.n_waves > 0) {
    std::vector<double> wv(4 * (size_t)D.n_waves, 0.0);
    for (int m = 0; m < D.n_waves; ++m) {
      wv[m] = d->wamp[m];
      wv[D.n_waves + m] = d->womg[m];
      wv[2 * D.n_waves + m] = d->wph[m];
    }
    HIPCHK(hipMemcpyAsync(D.wave, wv.data(), wv.size() * sizeof(double), hipMemcpyHostToDevice, s));
  }
  if (D.ts_n > 0)
    HIPCHK(hipMemcpyAsync(D.wave, d->ts.data(), d->ts.size() * sizeof(double), hipMemcpyHostToDevice, s));
  const size_t nc = (size_t)(p->nx + 1) * (p->ny + 1);
  HIPCHK(hipMemcpyAsync(D.io, depth_c, nc * sizeof(double), hipMemcpyHostToDevice, s));
  const DomDev<T>* Dd = (const DomDev<T>*)d->ddev;
  const int ncorn = (p->nx + 5) * (p->ny + 5);
  k_setup_corners<T><<<cdiv(ncorn, 256), 256, 0, s>>>(Dd);
  k_setup_cells<T><<<cdiv(p->nx * p->ny, 256), 256, 0, s>>>(Dd);
  setup_chunks<T>(D, Dd, s);
  if (D.n_waves > 0) k_setup_waves<T><<<1, 64, 0, s>>>(Dd, p->B);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return BQ_OK;
}

template <typename T>
static int set_state_t(bq_domain* d, const double* eta, const double* P, const double* Q) {
  DomDev<T>& D = desc<T>(d);
  const DomDev<T>* Dd = (const DomDev<T>*)d->ddev;
  hipStream_t s = d->stream;
  const size_t n = (size_t)d->nx * d->ny;
  const Layout Ly = layout_for<T>(&d->p);
  // clear all levels and histories
  HIPCHK(hipMemsetAsync(d->ws + Ly.off_w, 0, Ly.off_Dc - Ly.off_w, s));
  int* flag = (int*)((char*)D.io + n * sizeof(double));
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), s));
  const double* src[3] = {eta, P, Q};
  for (int k = 0; k < 3; ++k) {
    HIPCHK(hipMemcpyAsync(D.io, src[k], n * sizeof(double), hipMemcpyHostToDevice, s));
    k_scatter<T><<<cdiv((int)n, 256), 256, 0, s>>>(Dd, k, flag);
  }
  DevState h;
  memset(&h, 0, sizeof(h));
  HIPCHK(hipMemcpyAsync(d->st, &h, sizeof(h), hipMemcpyHostToDevice, s));
  if (west_driven(D.bc[0])) k_init_waves<T><<<1, 64, 0, s>>>(Dd);
  k_init_ghosts<T><<<cdiv((int)n, 256), 256, 0, s>>>(Dd);
  HIPCHK(hipGetLastError());
  int hflag = 0;
  HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hflag) {
    // leave a consistent lake-at-rest-free state: mark as failed
    h.status = BQ_EINVAL;
    HIPCHK(hipMemcpy(d->st, &h, sizeof(h), hipMemcpyHostToDevice));
    return fail(BQ_EINVAL, "eta < -d (negative depth) in the initial state");
  }
  return BQ_OK;
}

// Change a domain's tile shape between steps (the domain must be idle): the
// state stays where it is; the descriptor, the chunk tables and the per-tile
// maxima follow the new tiling.  Results continue up to the rounding of the
// line solves' different chunking.
template <typename T>
static int set_shape_t(bq_domain* d, int ty, int mx) {
  DomDev<T>& D = desc<T>(d);
  if (D.my == ty && D.mx == mx) return BQ_OK;
  if (!shape_ok<T>(ty, mx)) return fail(BQ_EINVAL, "tile shape %d x %d is not a candidate for this precision", ty, mx);
  const Layout Ly = layout_for<T>(&d->p);
  hipStream_t s = d->stream;
  const DomDev<T>* Dd = (const DomDev<T>*)d->ddev;
  k_fold_tiles<T><<<1, 256, 0, s>>>(Dd, D.tiles_x * D.tiles_y, Ly.tiles_max);
  D.mx = mx;
  D.my = ty;
  D.cx = cdiv(D.nx, mx);
  D.cy = cdiv(D.ny, ty);
  D.tiles_y = cdiv(D.ny, ty);
  HIPCHK(hipMemcpyAsync(d->ddev, &D, sizeof(D), hipMemcpyHostToDevice, s));
  setup_chunks<T>(D, Dd, s);
  HIPCHK(hipGetLastError());
  graph_del(d->L.graph);
  d->L.graph_built = 0;
  d->L.tiles = D.tiles_x * D.tiles_y;
  d->L.ty = ty;
  d->L.mx = mx;
  HIPCHK(hipStreamSynchronize(s));
  return BQ_OK;
}

// ---------------------------------------------------------------------------
// stepping
// ---------------------------------------------------------------------------

template <typename T>
static void launch_reduced(const Launch& L, hipStream_t s, int pass) {
  const DomDev<T>* tab = (const DomDev<T>*)L.table;
  if (L.segs == 8)
    k_reduced_seg<T, 8><<<cdiv(L.lines, 64), 64 * 8, 0, s>>>(tab, L.line_map, L.nd, L.lines, pass);
  else if (L.segs == 4)
    k_reduced_seg<T, 4><<<cdiv(L.lines, 64), 64 * 4, 0, s>>>(tab, L.line_map, L.nd, L.lines, pass);
  else
    k_reduced<T><<<cdiv(L.lines, L.rblock), L.rblock, 0, s>>>(tab, L.line_map, L.nd, L.lines, pass);
}

// the stencil/update kernel (pass 0: AB3 step, 1: corrector) and the
// finalize kernel (mode as in k_final) in the launch's tile shape
template <typename T>
static void launch_rhs(const Launch& L, hipStream_t s, int pass) {
  shape_dispatch<T>(L.ty, L.mx, [&](auto tyc, auto mxc) {
    constexpr int TY = decltype(tyc)::value, MX = decltype(mxc)::value;
    const DomDev<T>* tab = (const DomDev<T>*)L.table;
    if (pass == 0) k_rhs<T, TY, MX, false><<<L.tiles, NT, 0, s>>>(tab, L.tile_map, L.nd, L.swizzle);
    else k_rhs<T, TY, MX, true><<<L.tiles, NT, 0, s>>>(tab, L.tile_map, L.nd, L.swizzle);
  });
}

template <typename T>
static void launch_final(const Launch& L, hipStream_t s, int mode) {
  shape_dispatch<T>(L.ty, L.mx, [&](auto tyc, auto mxc) {
    constexpr int TY = decltype(tyc)::value, MX = decltype(mxc)::value;
    const DomDev<T>* tab = (const DomDev<T>*)L.table;
    if (mode == 0) k_final<T, TY, MX, 0><<<L.tiles, NT, 0, s>>>(tab, L.tile_map, L.nd, L.swizzle);
    else if (mode == 1) k_final<T, TY, MX, 1><<<L.tiles, NT, 0, s>>>(tab, L.tile_map, L.nd, L.swizzle);
    else k_final<T, TY, MX, 2><<<L.tiles, NT, 0, s>>>(tab, L.tile_map, L.nd, L.swizzle);
  });
}

template <typename T>
static void enqueue_step(const Launch& L, hipStream_t s, double dt_prescribed) {
  const DomDev<T>* tab = (const DomDev<T>*)L.table;
  k_dt<T><<<L.nd, DT_THREADS, 0, s>>>(tab, dt_prescribed);
  launch_rhs<T>(L, s, 0);
  launch_reduced<T>(L, s, 0);
  if (!L.any_pc) {
    launch_final<T>(L, s, 0);
  } else {
    launch_final<T>(L, s, 1);
    // corrector pass of the domains that run it (the others return at once)
    launch_rhs<T>(L, s, 1);
    launch_reduced<T>(L, s, 1);
    launch_final<T>(L, s, 2);
  }
}

template <typename T>
static void enqueue_commit(const Launch& L, hipStream_t s) {
  k_commit<T><<<cdiv(L.nd, 64), 64, 0, s>>>((const DomDev<T>*)L.table, L.nd);
}

template <typename T>
static int run_steps(Launch& L, hipStream_t s, int n_steps, int graph_steps) {
  if (n_steps <= 0) return BQ_OK;
  int left = n_steps;
  // graphs cannot be captured on the legacy null stream
  if (graph_steps > 0 && s != nullptr && n_steps >= graph_steps) {
    if (L.graph && L.graph_built != graph_steps) graph_del(L.graph);
    if (!L.graph) {
      hipGraph_t g;
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < graph_steps; ++k) enqueue_step<T>(L, s, 0.0);
      HIPCHK(hipStreamEndCapture(s, &g));
      const hipError_t ie = graph_new(&L.graph, g);
      (void)hipGraphDestroy(g);
      HIPCHK(ie);
      L.graph_built = graph_steps;
    }
    while (left >= graph_steps) {
      HIPCHK(hipGraphLaunch(L.graph, s));
      left -= graph_steps;
    }
  }
  for (int k = 0; k < left; ++k) enqueue_step<T>(L, s, 0.0);
  enqueue_commit<T>(L, s);
  HIPCHK(hipGetLastError());
  return BQ_OK;
}

template <typename T>
static int profile_t(Launch& L, hipStream_t s, int n_steps, double* ms_out) {
  const DomDev<T>* tab = (const DomDev<T>*)L.table;
  hipEvent_t ev[8] = {};
  for (int k = 0; k < 8; ++k)
    if (event_new(&ev[k], true) != hipSuccess) {
      for (hipEvent_t& e : ev) event_del(e);
      return fail(BQ_EDEVICE, "hipEventCreate");
    }
  double acc[4] = {0, 0, 0, 0};
  int rc = BQ_OK;
  const int last = L.any_pc ? 7 : 4;
  for (int it = 0; it < n_steps && rc == BQ_OK; ++it) {
    if (hipEventRecord(ev[0], s) != hipSuccess) { rc = fail(BQ_EDEVICE, "hipEventRecord"); break; }
    k_dt<T><<<L.nd, DT_THREADS, 0, s>>>(tab, 0.0);
    (void)hipEventRecord(ev[1], s);
    launch_rhs<T>(L, s, 0);
    (void)hipEventRecord(ev[2], s);
    launch_reduced<T>(L, s, 0);
    (void)hipEventRecord(ev[3], s);
    launch_final<T>(L, s, L.any_pc ? 1 : 0);
    (void)hipEventRecord(ev[4], s);
    if (L.any_pc) {
      launch_rhs<T>(L, s, 1);
      (void)hipEventRecord(ev[5], s);
      launch_reduced<T>(L, s, 1);
      (void)hipEventRecord(ev[6], s);
      launch_final<T>(L, s, 2);
      (void)hipEventRecord(ev[7], s);
    }
    if (hipEventSynchronize(ev[last]) != hipSuccess) { rc = fail(BQ_EDEVICE, "hipEventSynchronize"); break; }
    for (int k = 0; k < last; ++k) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      acc[k < 4 ? k : k - 3] += ms;     // the corrector pass adds to its kernels' entries
    }
  }
  enqueue_commit<T>(L, s);
  for (hipEvent_t& e : ev) event_del(e);
  if (rc) return rc;
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  for (int k = 0; k < 4; ++k) ms_out[k] = n_steps > 0 ? acc[k] / n_steps : 0.0;
  return BQ_OK;
}

template <typename T>
static int step_dt_t(bq_domain* d, double dt) {
  enqueue_step<T>(d->L, d->stream, dt);
  enqueue_commit<T>(d->L, d->stream);
  HIPCHK(hipGetLastError());
  return BQ_OK;
}

template <typename T>
static int sync_t(bq_domain* d, bq_info* out) {
  DevState h;
  HIPCHK(hipMemcpyAsync(&h, d->st, sizeof(h), hipMemcpyDeviceToHost, d->stream));
  HIPCHK(hipStreamSynchronize(d->stream));
  if (out) {
    k_diag_part<T><<<NDIAG, 256, 0, d->stream>>>((const DomDev<T>*)d->ddev, (int)(h.n & 1), (int)(h.n % 3));
    k_diag_final<T><<<1, NDIAG, 0, d->stream>>>((const DomDev<T>*)d->ddev);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&h, d->st, sizeof(h), hipMemcpyDeviceToHost, d->stream));
    HIPCHK(hipStreamSynchronize(d->stream));
    out->t = h.t;
    out->n = h.n;
    out->dt_last = h.dt1;
    out->dt_prev1 = h.dt2;
    out->dt_prev2 = h.dt3;
    out->smax = __builtin_bit_cast(double, h.smax_bits);
    out->mass = h.mass;
    out->energy = h.energy;
    out->status = h.status;
  }
  return h.status;
}

template <typename T>
static int read_t(bq_domain* d, int which, double* out) {
  DevState h;
  HIPCHK(hipMemcpyAsync(&h, d->st, sizeof(h), hipMemcpyDeviceToHost, d->stream));
  HIPCHK(hipStreamSynchronize(d->stream));
  const int n = d->nx * d->ny;
  k_gather<T><<<cdiv(n, 256), 256, 0, d->stream>>>((const DomDev<T>*)d->ddev, which, (int)(h.n & 1),
                                                  (int)(h.n % 3));
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(out, desc<T>(d).io, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, d->stream));
  HIPCHK(hipStreamSynchronize(d->stream));
  return BQ_OK;
}

// checkpoint: header + DevState + w, P, Q, E, F, G regions (the dynamic state)
struct CkptHeader {
  uint64_t magic;
  int32_t nx, ny, precision, version;
  uint64_t state_bytes, field_bytes;
};
static const uint64_t CKPT_MAGIC = 0x42515354'45503031ull;

template <typename T>
static size_t ckpt_bytes(const bq_domain* d) {
  const Layout Ly = layout_for<T>(&d->p);
  return sizeof(CkptHeader) + sizeof(DevState) + (Ly.off_Dc - Ly.off_w);
}

template <typename T>
static int save_t(bq_domain* d, void* host, size_t* bytes) {
  const size_t need = ckpt_bytes<T>(d);
  if (!host) {
    *bytes = need;
    return BQ_OK;
  }
  if (*bytes < need) return fail(BQ_EINVAL, "checkpoint buffer of %zu bytes, need %zu", *bytes, need);
  const Layout Ly = layout_for<T>(&d->p);
  CkptHeader hd{CKPT_MAGIC, d->nx, d->ny, d->precision, 1, sizeof(DevState), Ly.off_Dc - Ly.off_w};
  char* o = (char*)host;
  memcpy(o, &hd, sizeof(hd));
  HIPCHK(hipMemcpyAsync(o + sizeof(hd), d->st, sizeof(DevState), hipMemcpyDeviceToHost, d->stream));
  HIPCHK(hipMemcpyAsync(o + sizeof(hd) + sizeof(DevState), d->ws + Ly.off_w, hd.field_bytes, hipMemcpyDeviceToHost,
                        d->stream));
  HIPCHK(hipStreamSynchronize(d->stream));
  *bytes = need;
  return BQ_OK;
}

template <typename T>
static int load_t(bq_domain* d, const void* host, size_t bytes) {
  const Layout Ly = layout_for<T>(&d->p);
  CkptHeader hd;
  if (bytes < sizeof(hd)) return fail(BQ_EINVAL, "checkpoint too small");
  memcpy(&hd, host, sizeof(hd));
  if (hd.magic != CKPT_MAGIC || hd.nx != d->nx || hd.ny != d->ny || hd.precision != d->precision ||
      hd.state_bytes != sizeof(DevState) || hd.field_bytes != Ly.off_Dc - Ly.off_w ||
      bytes < ckpt_bytes<T>(d))
    return fail(BQ_EINVAL, "checkpoint does not match this domain");
  const char* o = (const char*)host;
  HIPCHK(hipMemcpyAsync(d->st, o + sizeof(hd), sizeof(DevState), hipMemcpyHostToDevice, d->stream));
  HIPCHK(hipMemcpyAsync(d->ws + Ly.off_w, o + sizeof(hd) + sizeof(DevState), hd.field_bytes, hipMemcpyHostToDevice,
                        d->stream));
  // the per-tile CFL maxima were written under the saving domain's tiling:
  // fold every slot into the state's maximum (the same value for the next
  // Delta t under any tiling)
  k_fold_tiles<T><<<1, 256, 0, d->stream>>>((const DomDev<T>*)d->ddev, Ly.tiles_max, Ly.tiles_max);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(d->stream));
  return BQ_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------

template <typename T>
static void drop_graph(Launch& L) {
  graph_del(L.graph);
  L.graph_built = 0;
}

// one member's committed time, step count and latched status, as gathered
// by bq_batch_status
struct StatusRec {
  double t;
  long long n;
  int status, pad;
};

template <typename T>
__global__ void k_batch_status(const DomDev<T>* __restrict__ doms, int nd, StatusRec* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nd) return;
  const DevState* st = doms[k].st;
  out[k] = StatusRec{st->t, st->n, st->status, 0};
}

// bytes of the device tables of one member list: DomDev<T>[nd], tile map,
// line map, status staging
template <typename T>
static size_t launch_bytes(const std::vector<bq_domain*>& doms) {
  size_t tiles = 0, lines = 0;
  for (const bq_domain* d : doms) {
    const DomDev<T>& D = desc<T>(const_cast<bq_domain*>(d));
    tiles += (size_t)D.tiles_x * D.tiles_y;
    lines += (size_t)D.nx + D.ny;
  }
  return rup(sizeof(DomDev<T>) * doms.size(), 256) + rup(sizeof(int) * tiles, 256) + rup(sizeof(int) * lines, 256) +
         rup(sizeof(StatusRec) * doms.size(), 256);
}

// defer_graph: leave a stale graph executable to the next step (which
// destroys and re-captures it) instead of destroying it here
template <typename T>
static int fill_launch(Launch& L, char* m, const std::vector<bq_domain*>& doms, hipStream_t s,
                       bool defer_graph = false) {
  const int nd = (int)doms.size();
  std::vector<DomDev<T>> tab(nd);
  std::vector<int> tmap, lmap;
  for (int k = 0; k < nd; ++k) {
    tab[k] = desc<T>(doms[k]);
    const int nt = tab[k].tiles_x * tab[k].tiles_y, nl = tab[k].nx + tab[k].ny;
    for (int t = 0; t < nt; ++t) tmap.push_back((k << MAP_SHIFT) | t);
    for (int l = 0; l < nl; ++l) lmap.push_back((k << MAP_SHIFT) | l);
  }
  const size_t tb = rup(sizeof(DomDev<T>) * nd, 256), mb = rup(sizeof(int) * tmap.size(), 256),
               lb = rup(sizeof(int) * lmap.size(), 256);
  HIPCHK(hipMemcpyAsync(m, tab.data(), sizeof(DomDev<T>) * nd, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(m + tb, tmap.data(), sizeof(int) * tmap.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(m + tb + mb, lmap.data(), sizeof(int) * lmap.size(), hipMemcpyHostToDevice, s));
  if (defer_graph) L.graph_built = 0;
  else drop_graph<T>(L);
  L.table = m;
  L.tile_map = (int*)(m + tb);
  L.line_map = (int*)(m + tb + mb);
  L.status = m + tb + mb + lb;
  L.nd = nd;
  L.tiles = (int)tmap.size();
  L.lines = (int)lmap.size();
  L.any_pc = 0;
  for (int k = 0; k < nd; ++k) L.any_pc |= tab[k].corrector;
  L.ty = tab[0].my;
  L.mx = tab[0].mx;
  return BQ_OK;
}

template <typename T>
static int batch_build_t(bq_batch* b) {
  const int nd = (int)b->doms.size();
  if (nd >= (1 << (31 - MAP_SHIFT))) return fail(BQ_EINVAL, "too many domains in one batch");
  for (bq_domain* d : b->doms) {
    const DomDev<T>& D = desc<T>(d);
    if ((long long)D.tiles_x * D.tiles_y >= (1 << MAP_SHIFT) || D.nx + D.ny >= (1 << MAP_SHIFT))
      return fail(BQ_EINVAL, "a batch member is too large for the work map");
  }
  // the previous tables may still be read by queued work
  HIPCHK(hipStreamSynchronize(b->stream));
  for (hipStream_t ls : b->lane)
    if (ls) HIPCHK(hipStreamSynchronize(ls));
  // every member takes the batch's tile shape (the first member's until a
  // schedule sets one)
  if (b->ty == 0) {
    b->ty = desc<T>(b->doms[0]).my;
    b->mx = desc<T>(b->doms[0]).mx;
  }
  for (bq_domain* d : b->doms) {
    const int rc = set_shape_t<T>(d, b->ty, b->mx);
    if (rc) return rc;
  }
  b->lanes = b->lanes_req < nd ? b->lanes_req : nd;
  const int nl = b->lanes;
  std::vector<bq_domain*> part[MAX_LANES];
  if (nl > 1) {
    // greedy split by cell count, largest first, each to the lightest
    // group; members keep their order within a group
    std::vector<int> ord(nd);
    for (int k = 0; k < nd; ++k) ord[k] = k;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
      return (long long)b->doms[x]->nx * b->doms[x]->ny > (long long)b->doms[y]->nx * b->doms[y]->ny;
    });
    std::vector<int> grp(nd, 0);
    long long cells[MAX_LANES] = {};
    for (int k : ord) {
      int gsel = 0;
      for (int g = 1; g < nl; ++g)
        if (cells[g] < cells[gsel]) gsel = g;
      grp[k] = gsel;
      cells[gsel] += (long long)b->doms[k]->nx * b->doms[k]->ny;
    }
    for (int k = 0; k < nd; ++k) part[grp[k]].push_back(b->doms[k]);
  }
  const size_t s0 = launch_bytes<T>(b->doms);
  size_t sg[MAX_LANES] = {}, need = s0;
  for (int g = 0; g < nl && nl > 1; ++g) need += (sg[g] = launch_bytes<T>(part[g]));
  // tables in the device's static array (no allocation; its owner was set
  // by bq_batch_set_static) or in the batch's own device memory
  const bool stat = b->static_dev >= 0;
  char* m = nullptr;
  if (stat) {
    if (need > (size_t)BQ_STATIC_TABLE_BYTES)
      return fail(BQ_EINVAL, "the batch's tables need %zu bytes, more than the %zu of the static array", need,
                  (size_t)BQ_STATIC_TABLE_BYTES);
    m = g_static_ptr[b->static_dev];
  } else {
    if (need > b->mem_bytes) {
      if (b->mem) HIPCHK(hipFree(b->mem));
      b->mem = nullptr;
      HIPCHK(hipMalloc(&b->mem, need));
      b->mem_bytes = need;
    }
    m = (char*)b->mem;
  }
  int rc = fill_launch<T>(b->L, m, b->doms, b->stream, stat);
  if (rc) return rc;
  b->L.rblock = b->rblock;
  b->L.swizzle = b->swizzle;
  b->L.segs = b->segs;
  for (int g = 0; g < MAX_LANES; ++g) {
    if (stat) b->G[g].graph_built = 0;
    else drop_graph<T>(b->G[g]);
  }
  if (nl > 1) {
    size_t off = s0;
    for (int g = 0; g < nl && !rc; ++g) {
      rc = fill_launch<T>(b->G[g], m + off, part[g], b->stream, stat);
      off += sg[g];
      b->G[g].rblock = b->rblock;
      b->G[g].swizzle = b->swizzle;
      b->G[g].segs = b->segs;
    }
    if (rc) return rc;
  }
  HIPCHK(hipStreamSynchronize(b->stream));
  return BQ_OK;
}

// the lane streams and their events, created together, one after the other,
// when the batch is created (later member changes create nothing)
static int make_lanes(bq_batch* b) {
  for (int l = 0; l < MAX_LANES; ++l)
    if (!b->lane[l]) HIPCHK(stream_new(&b->lane[l]));
  if (!b->ev_fork) HIPCHK(event_new(&b->ev_fork, false));
  for (int l = 0; l < MAX_LANES; ++l)
    if (!b->ev_join[l]) HIPCHK(event_new(&b->ev_join[l], false));
  return BQ_OK;
}

// the lanes start after the work queued so far on the batch's stream, and
// the batch's stream continues only after every lane's work
static int fork_lanes(bq_batch* b) {
  HIPCHK(hipEventRecord(b->ev_fork, b->stream));
  for (int l = 0; l < b->lanes; ++l) HIPCHK(hipStreamWaitEvent(b->lane[l], b->ev_fork, 0));
  return BQ_OK;
}

static int join_lanes(bq_batch* b) {
  for (int l = 0; l < b->lanes; ++l) {
    HIPCHK(hipEventRecord(b->ev_join[l], b->lane[l]));
    HIPCHK(hipStreamWaitEvent(b->stream, b->ev_join[l], 0));
  }
  return BQ_OK;
}

template <typename T>
static int batch_run_t(bq_batch* b, int n_steps) {
  if (b->lanes == 1) return run_steps<T>(b->L, b->stream, n_steps, b->graph_steps);
  if (n_steps <= 0) return BQ_OK;
  int rc = fork_lanes(b);
  for (int l = 0; l < b->lanes && !rc; ++l) rc = run_steps<T>(b->G[l], b->lane[l], n_steps, b->graph_steps);
  const int rj = join_lanes(b);
  return rc ? rc : rj;
}

// Kernel timing with all lanes running: hipEvents around every kernel on
// its own lane's stream; ms_out[k] is the mean duration of one launch of
// kernel k (a launch covers one group).
template <typename T>
static int batch_profile_t(bq_batch* b, int n_steps, double* ms_out) {
  if (b->lanes == 1) return profile_t<T>(b->L, b->stream, n_steps, ms_out);
  const int nl = b->lanes;
  hipStream_t* ss = b->lane;
  hipEvent_t ev[MAX_LANES][8] = {};
  for (int l = 0; l < nl; ++l)
    for (int k = 0; k < 8; ++k)
      if (event_new(&ev[l][k], true) != hipSuccess) {
        for (auto& row : ev)
          for (hipEvent_t& e : row) event_del(e);
        return fail(BQ_EDEVICE, "hipEventCreate");
      }
  double acc[4] = {0, 0, 0, 0};
  bool pc = false;
  for (int l = 0; l < nl; ++l) pc |= b->G[l].any_pc != 0;
  const int last = pc ? 7 : 4;
  int rc = fork_lanes(b);
  for (int it = 0; it < n_steps && rc == BQ_OK; ++it) {
    for (int l = 0; l < nl; ++l) (void)hipEventRecord(ev[l][0], ss[l]);
    for (int l = 0; l < nl; ++l) {
      const Launch& L = b->G[l];
      k_dt<T><<<L.nd, DT_THREADS, 0, ss[l]>>>((const DomDev<T>*)L.table, 0.0);
      (void)hipEventRecord(ev[l][1], ss[l]);
    }
    for (int pass = 0; pass < (last == 7 ? 2 : 1); ++pass) {
      const int e0 = pass == 0 ? 1 : 4;
      for (int l = 0; l < nl; ++l) {
        launch_rhs<T>(b->G[l], ss[l], pass);
        (void)hipEventRecord(ev[l][e0 + 1], ss[l]);
      }
      for (int l = 0; l < nl; ++l) {
        const Launch& L = b->G[l];
        launch_reduced<T>(L, ss[l], pass);
        (void)hipEventRecord(ev[l][e0 + 2], ss[l]);
      }
      for (int l = 0; l < nl; ++l) {
        const Launch& L = b->G[l];
        launch_final<T>(L, ss[l], pass == 1 ? 2 : (L.any_pc ? 1 : 0));
        (void)hipEventRecord(ev[l][e0 + 3], ss[l]);
      }
    }
    for (int l = 0; l < nl && rc == BQ_OK; ++l)
      if (hipEventSynchronize(ev[l][last]) != hipSuccess) rc = fail(BQ_EDEVICE, "hipEventSynchronize");
    for (int l = 0; l < nl && rc == BQ_OK; ++l)
      for (int k = 0; k < last; ++k) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[l][k], ev[l][k + 1]);
        acc[k < 4 ? k : k - 3] += ms / nl;
      }
  }
  for (int l = 0; l < nl; ++l) enqueue_commit<T>(b->G[l], ss[l]);
  const int rj = join_lanes(b);
  for (auto& row : ev)
    for (hipEvent_t& e : row) event_del(e);
  if (rc) return rc;
  if (rj) return rj;
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(b->stream));
  for (int k = 0; k < 4; ++k) ms_out[k] = n_steps > 0 ? acc[k] / n_steps : 0.0;
  return BQ_OK;
}

template <typename T>
static int batch_status_t(bq_batch* b, int32_t* status, int64_t* steps, double* t) {
  const int nd = b->L.nd;
  k_batch_status<T><<<cdiv(nd, 64), 64, 0, b->stream>>>((const DomDev<T>*)b->L.table, nd, (StatusRec*)b->L.status);
  HIPCHK(hipGetLastError());
  std::vector<StatusRec> h(nd);
  HIPCHK(hipMemcpyAsync(h.data(), b->L.status, sizeof(StatusRec) * nd, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  for (int k = 0; k < nd; ++k) {
    status[k] = h[k].status;
    if (steps) steps[k] = h[k].n;
    if (t) t[k] = h[k].t;
  }
  return BQ_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

#define DISPATCH(prec, fn, ...) ((prec) == BQ_FP32 ? fn<float>(__VA_ARGS__) : fn<double>(__VA_ARGS__))

// ---------------------------------------------------------------------------
// schedule autotuner
// ---------------------------------------------------------------------------

static void apply_schedule(bq_batch* b, int rblock, int swizzle, int segs) {
  b->rblock = rblock;
  b->swizzle = swizzle;
  b->segs = segs;
  Launch* ls[1 + MAX_LANES] = {&b->L};
  for (int g = 0; g < MAX_LANES; ++g) ls[1 + g] = &b->G[g];
  for (Launch* L : ls) {
    L->rblock = rblock;
    L->swizzle = swizzle;
    L->segs = segs;
    // graphs hold the launch parameters they were captured with
    graph_del(L->graph);
  }
}

static int set_tune(bq_batch* b, const bq_tune* t) {
  if (t->lanes < 1 || t->lanes > MAX_LANES) return fail(BQ_EINVAL, "lanes must be 1 .. %d", MAX_LANES);
  if (t->graph_steps < 0) return fail(BQ_EINVAL, "graph_steps must be >= 0");
  if (t->reduce_block != 64 && t->reduce_block != 128 && t->reduce_block != 256)
    return fail(BQ_EINVAL, "reduce_block must be 64, 128 or 256");
  if (t->swizzle != 0 && t->swizzle != 1) return fail(BQ_EINVAL, "swizzle must be 0 or 1");
  if (t->reduce_segments != 1 && t->reduce_segments != 4 && t->reduce_segments != 8)
    return fail(BQ_EINVAL, "reduce_segments must be 1, 4 or 8");
  const bool shape = (t->tile_y || t->chunk_x) && (t->tile_y != b->ty || t->chunk_x != b->mx);
  if (shape && !(b->precision == BQ_FP32 ? shape_ok<float>(t->tile_y, t->chunk_x)
                                         : shape_ok<double>(t->tile_y, t->chunk_x)))
    return fail(BQ_EINVAL, "tile shape %d x %d is not a candidate for this precision", t->tile_y, t->chunk_x);
  if (t->lanes != b->lanes_req || shape) {
    b->lanes_req = t->lanes;
    if (shape) {
      b->ty = t->tile_y;
      b->mx = t->chunk_x;
    }
    const int rc = DISPATCH(b->precision, batch_build_t, b);
    if (rc) return rc;
  }
  b->graph_steps = t->graph_steps;
  apply_schedule(b, t->reduce_block, t->swizzle, t->reduce_segments);
  return BQ_OK;
}

// Each candidate runs real steps of the method (every schedule gives the
// same results, bit for bit without segments and up to rounding with them),
// so tuning costs no simulation work: warm-up (which also captures the
// graph), then steps_per_trial timed steps.
template <typename T>
static int batch_autotune_t(bq_batch* b, int steps, bq_tune* out) {
  std::vector<bq_tune> cands;
  const int max_lanes = (int)b->doms.size() < MAX_LANES ? (int)b->doms.size() : MAX_LANES;
  // The XCD-aware tile order is not searched: it cuts the stencil kernel's
  // HBM traffic by a third (measured) while its effect on a whole step is
  // below the trials' timing noise, so a search would pick it by chance.
  const int ty0 = b->ty, mx0 = b->mx;
  for (int lanes = 1; lanes <= max_lanes; ++lanes)
    for (int graph : {4, 16}) {
      for (int rb : {64, 256}) cands.push_back(bq_tune{lanes, graph, rb, 1, 1, ty0, mx0, 0.0});
      for (int ns : {4, 8}) cands.push_back(bq_tune{lanes, graph, 256, 1, ns, ty0, mx0, 0.0});
    }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (event_new(&e0, true) != hipSuccess || event_new(&e1, true) != hipSuccess) {
    event_del(e0);
    return fail(BQ_EDEVICE, "hipEventCreate");
  }
  int rc = BQ_OK;
  auto trial = [&](bq_tune& c) -> int {
    int r = set_tune(b, &c);
    const int warm = c.graph_steps > steps / 4 ? c.graph_steps : steps / 4;
    if (!r) r = batch_run_t<T>(b, warm);
    if (r) return r;
    if (hipEventRecord(e0, b->stream) != hipSuccess) return fail(BQ_EDEVICE, "hipEventRecord");
    r = batch_run_t<T>(b, steps);
    if (r) return r;
    if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return fail(BQ_EDEVICE, "hipEvent");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    c.ms_per_step += 0.5 * ms / steps;
    return BQ_OK;
  };
  // every candidate twice, in forward then reverse order, scored by the mean:
  // a drift of the clocks over the tuning run (boost after idle, then
  // settling) cancels instead of favouring the first candidates
  auto search = [&](std::vector<bq_tune>& cs, int& best) -> int {
    int r = BQ_OK;
    for (size_t k = 0; k < cs.size() && r == BQ_OK; ++k) r = trial(cs[k]);
    for (size_t k = cs.size(); k-- > 0 && r == BQ_OK;) r = trial(cs[k]);
    if (r) return r;
    if (getenv("BQ_TUNE_LOG"))
      for (const bq_tune& c : cs)
        fprintf(stderr, "bq tune: lanes %d graph %d reduce_block %d segments %d swizzle %d tile %dx64 chunk %d: "
                "%.4f ms/step\n", c.lanes, c.graph_steps, c.reduce_block, c.reduce_segments, c.swizzle, c.tile_y,
                c.chunk_x, c.ms_per_step);
    best = 0;
    for (size_t k = 1; k < cs.size(); ++k)
      if (cs[k].ms_per_step < cs[best].ms_per_step) best = (int)k;
    // candidates within half a percent of the fastest are ties at the
    // trials' resolution: take the one with the longest graph replays among
    // them (fewest host launches over a long run)
    const double tie = 1.005 * cs[best].ms_per_step;
    for (size_t k = 0; k < cs.size(); ++k)
      if (cs[k].ms_per_step <= tie && cs[k].graph_steps > cs[best].graph_steps) best = (int)k;
    return BQ_OK;
  };
  // stage 1: the schedule in the current tile shape; stage 2: the tile
  // shapes under the best schedule (the shape changes the layout of the
  // line solves, the schedule only the launches)
  int best = 0;
  rc = search(cands, best);
  bq_tune pick = cands[best];
  if (!rc) {
    std::vector<bq_tune> shapes;
    for (int k = 0; k < Cfg<T>::NS; ++k) {
      bq_tune c = pick;
      c.tile_y = Cfg<T>::shape(k).ty;
      c.chunk_x = Cfg<T>::shape(k).mx;
      c.ms_per_step = 0.0;
      shapes.push_back(c);
    }
    rc = search(shapes, best);
    pick = shapes[best];
  }
  event_del(e0);
  event_del(e1);
  if (rc) return rc;
  rc = set_tune(b, &pick);
  if (rc) return rc;
  *out = pick;
  return BQ_OK;
}

extern "C" {

int bq_abi_version(void) { return BQ_ABI_VERSION; }

int bq_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (!dst || !src) return fail(BQ_EINVAL, "NULL argument");
  if (bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0)
    return fail(BQ_EINVAL, "bq_stream_copy needs 16-byte aligned buffers and a multiple of 16 bytes");
  const size_t n = bytes / 16;
  if (n == 0) return BQ_OK;
  if (n / 256 >= (size_t)INT32_MAX) return fail(BQ_EINVAL, "copy too large");
  k_stream_copy<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)hip_stream>>>((const u32x4*)src, (u32x4*)dst, n);
  HIPCHK(hipGetLastError());
  return BQ_OK;
}

int bq_live_handles(int32_t* counts) {
  if (!counts) return fail(BQ_EINVAL, "NULL argument");
  for (int k = 0; k < 3; ++k) counts[k] = g_live[k].load();
  return BQ_OK;
}

const char* bq_last_error(void) { return g_err; }

void bq_params_default(bq_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->g = 9.81;
  p->B = 1.0 / 15.0;
  p->cfl = 0.2;
  p->ema_alpha = 0.1;
  p->dt_max = 1.0;
  p->dt_min = 1e-9;
  p->theta = 1.3;
  p->fstar_order = 2;
  p->precision = BQ_FP64;
}

int bq_workspace_bytes(const bq_params* p, size_t* bytes) {
  const int rc = check_params(p);
  if (rc) return rc;
  if (!bytes) return fail(BQ_EINVAL, "bytes is NULL");
  *bytes = p->precision == BQ_FP32 ? layout_for<float>(p).total : layout_for<double>(p).total;
  return BQ_OK;
}

int bq_domain_create(const bq_params* p, const double* depth_c, void* dev_workspace, size_t bytes, void* hip_stream,
                     bq_domain** out) {
  int rc = check_params(p);
  if (rc) return rc;
  if (!depth_c || !dev_workspace || !out) return fail(BQ_EINVAL, "NULL argument");
  if (((uintptr_t)dev_workspace) % 256 != 0) return fail(BQ_EINVAL, "workspace must be 256-byte aligned");
  // still-water depths must be finite (the kernels take max(D, 0) and
  // min(D, 0) of finite values); checked before anything reaches the device
  for (size_t k = 0, nc = (size_t)(p->nx + 1) * (p->ny + 1); k < nc; ++k)
    if (!std::isfinite(depth_c[k])) return fail(BQ_EINVAL, "depth_c[%zu] is not finite", k);
  bq_domain* d = new (std::nothrow) bq_domain();
  if (!d) return fail(BQ_EINVAL, "out of host memory");
  d->p = *p;
  const bool wave = p->bc[0] == BQ_SINE || p->bc[0] == BQ_IRREGULAR;
  if (wave) {
    d->wamp.assign(p->wave_amp, p->wave_amp + p->n_waves);
    d->womg.assign(p->wave_omega, p->wave_omega + p->n_waves);
    d->wph.assign(p->n_waves, 0.0);
    if (p->wave_phase) d->wph.assign(p->wave_phase, p->wave_phase + p->n_waves);
  }
  if (p->bc[0] == BQ_TIMESERIES) {
    d->ts.assign(p->ts_eta, p->ts_eta + p->ts_n);
    d->ts.insert(d->ts.end(), p->ts_P, p->ts_P + p->ts_n);
  }
  d->p.wave_amp = d->p.wave_omega = d->p.wave_phase = nullptr;
  d->p.ts_eta = d->p.ts_P = nullptr;
  d->precision = p->precision;
  d->stream = (hipStream_t)hip_stream;
  d->ws = (char*)dev_workspace;
  d->ws_bytes = bytes;
  d->nx = p->nx;
  d->ny = p->ny;
  rc = DISPATCH(d->precision, create_t, d, depth_c);
  if (rc) {
    delete d;
    return rc;
  }
  // lake at rest
  std::vector<double> z((size_t)p->nx * p->ny, 0.0);
  rc = bq_set_state(d, z.data(), z.data(), z.data());
  if (rc) {
    delete d;
    return rc;
  }
  *out = d;
  return BQ_OK;
}

int bq_domain_free(bq_domain* d) {
  if (!d) return fail(BQ_EINVAL, "NULL domain");
  graph_del(d->L.graph);
  delete d;
  return BQ_OK;
}

int bq_set_state(bq_domain* d, const double* eta, const double* P, const double* Q) {
  if (!d || !eta || !P || !Q) return fail(BQ_EINVAL, "NULL argument");
  return DISPATCH(d->precision, set_state_t, d, eta, P, Q);
}

int bq_step(bq_domain* d, int32_t n_steps) {
  if (!d) return fail(BQ_EINVAL, "NULL domain");
  if (n_steps < 0) return fail(BQ_EINVAL, "n_steps < 0");
  return DISPATCH(d->precision, run_steps, d->L, d->stream, n_steps, d->graph_steps);
}

int bq_step_dt(bq_domain* d, double dt) {
  if (!d) return fail(BQ_EINVAL, "NULL domain");
  if (!(dt > 0.0)) return fail(BQ_EINVAL, "dt must be > 0");
  return DISPATCH(d->precision, step_dt_t, d, dt);
}

int bq_sync(bq_domain* d, bq_info* out) {
  if (!d) return fail(BQ_EINVAL, "NULL domain");
  return DISPATCH(d->precision, sync_t, d, out);
}

int bq_read(bq_domain* d, int32_t which, double* host_out) {
  if (!d || !host_out) return fail(BQ_EINVAL, "NULL argument");
  if (which < 0 || which > 5) return fail(BQ_EINVAL, "which must be 0..5");
  if (which == 4 && !(d->p.runup_delta > 0.0)) return fail(BQ_EINVAL, "the run-up record is not kept (runup_delta = 0)");
  return DISPATCH(d->precision, read_t, d, which, host_out);
}

int bq_save(bq_domain* d, void* host, size_t* bytes) {
  if (!d || !bytes) return fail(BQ_EINVAL, "NULL argument");
  return DISPATCH(d->precision, save_t, d, host, bytes);
}

int bq_load(bq_domain* d, const void* host, size_t bytes) {
  if (!d || !host) return fail(BQ_EINVAL, "NULL argument");
  return DISPATCH(d->precision, load_t, d, host, bytes);
}

int bq_profile_steps(bq_domain* d, int32_t n_steps, double* ms_out) {
  if (!d || !ms_out || n_steps < 0) return fail(BQ_EINVAL, "bad argument");
  return DISPATCH(d->precision, profile_t, d->L, d->stream, n_steps, ms_out);
}

int bq_batch_profile_steps(bq_batch* b, int32_t n_steps, double* ms_out) {
  if (!b || !ms_out || n_steps < 0) return fail(BQ_EINVAL, "bad argument");
  const int rc = static_owner_ok(b);
  if (rc) return rc;
  return DISPATCH(b->precision, batch_profile_t, b, n_steps, ms_out);
}

int bq_set_graph_steps(bq_domain* d, int32_t steps) {
  if (!d || steps < 0) return fail(BQ_EINVAL, "bad argument");
  d->graph_steps = steps;
  return BQ_OK;
}

int bq_batch_create(bq_domain* const* doms, int32_t n, void* hip_stream, bq_batch** out) {
  if (!out) return fail(BQ_EINVAL, "NULL argument");
  bq_batch* b = new (std::nothrow) bq_batch();
  if (!b) return fail(BQ_EINVAL, "out of host memory");
  b->stream = (hipStream_t)hip_stream;
  int rc = make_lanes(b);
  if (!rc) rc = bq_batch_set(b, doms, n);
  if (rc) {
    bq_batch_free(b);
    return rc;
  }
  *out = b;
  return BQ_OK;
}

static int check_members(bq_domain* const* doms, int32_t n) {
  if (n < 1 || !doms) return fail(BQ_EINVAL, "a batch needs at least one domain");
  if (!doms[0]) return fail(BQ_EINVAL, "NULL domain in batch");
  const int prec = doms[0]->precision;
  for (int k = 0; k < n; ++k) {
    if (!doms[k]) return fail(BQ_EINVAL, "NULL domain in batch");
    if (doms[k]->precision != prec) return fail(BQ_EINVAL, "batch members must share one precision");
  }
  return BQ_OK;
}

// give up the static tables (if this batch holds them)
static void release_static(bq_batch* b) {
  if (b->static_dev < 0) return;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (g_static_owner[b->static_dev] == b) g_static_owner[b->static_dev] = nullptr;
  b->static_dev = -1;
}

int bq_batch_set(bq_batch* b, bq_domain* const* doms, int32_t n) {
  if (!b) return fail(BQ_EINVAL, "NULL batch");
  const int rc = check_members(doms, n);
  if (rc) return rc;
  if (b->static_dev >= 0) {
    // queued steps may still read the static tables
    HIPCHK(hipStreamSynchronize(b->stream));
    release_static(b);
  }
  b->doms.assign(doms, doms + n);
  b->precision = doms[0]->precision;
  return DISPATCH(b->precision, batch_build_t, b);
}

int bq_batch_set_static(bq_batch* b, bq_domain* const* doms, int32_t n) {
  if (!b) return fail(BQ_EINVAL, "NULL batch");
  int rc = check_members(doms, n);
  if (rc) return rc;
  // the one-lane tables plus those of the lane groups (a partition of the
  // same members: at most as many bytes again, plus the groups' rounding of
  // their four regions)
  const std::vector<bq_domain*> dv(doms, doms + n);
  const size_t one = doms[0]->precision == BQ_FP32 ? launch_bytes<float>(dv) : launch_bytes<double>(dv);
  const size_t bound = 2 * one + (size_t)MAX_LANES * 4 * 256;
  if (bound > (size_t)BQ_STATIC_TABLE_BYTES)
    return fail(BQ_EINVAL, "%d domains need up to %zu bytes of tables, more than the %zu of the static array", n, bound,
                (size_t)BQ_STATIC_TABLE_BYTES);
  int dev = -1;
  char* ptr = nullptr;
  rc = static_tables(&dev, &ptr);
  if (rc) return rc;
  (void)ptr;
  {
    // the batch that held the array last must have finished reading it;
    // from here on its steps are refused until it sets its members again
    std::lock_guard<std::mutex> lk(g_static_mu);
    bq_batch* prev = g_static_owner[dev];
    if (prev && prev != b) {
      HIPCHK(hipStreamSynchronize(prev->stream));
      for (hipStream_t ls : prev->lane)
        if (ls) HIPCHK(hipStreamSynchronize(ls));
    }
    g_static_owner[dev] = b;
  }
  b->static_dev = dev;
  b->doms.assign(doms, doms + n);
  b->precision = doms[0]->precision;
  rc = DISPATCH(b->precision, batch_build_t, b);
  if (rc) release_static(b);
  return rc;
}

int bq_batch_step(bq_batch* b, int32_t n_steps) {
  if (!b) return fail(BQ_EINVAL, "NULL batch");
  if (n_steps < 0) return fail(BQ_EINVAL, "n_steps < 0");
  const int rc = static_owner_ok(b);
  if (rc) return rc;
  return DISPATCH(b->precision, batch_run_t, b, n_steps);
}

int bq_batch_status(bq_batch* b, int32_t* status, int64_t* steps, double* t) {
  if (!b || !status) return fail(BQ_EINVAL, "NULL argument");
  const int rc = static_owner_ok(b);
  if (rc) return rc;
  return DISPATCH(b->precision, batch_status_t, b, status, steps, t);
}

int bq_batch_sync(bq_batch* b) {
  if (!b) return fail(BQ_EINVAL, "NULL batch");
  HIPCHK(hipStreamSynchronize(b->stream));
  for (hipStream_t ls : b->lane)
    if (ls) HIPCHK(hipStreamSynchronize(ls));
  return BQ_OK;
}

int bq_batch_set_lanes(bq_batch* b, int32_t lanes) {
  if (!b || lanes < 1 || lanes > MAX_LANES) return fail(BQ_EINVAL, "lanes must be 1 .. %d", MAX_LANES);
  if (lanes == b->lanes_req) return BQ_OK;
  const int rc = static_owner_ok(b);
  if (rc) return rc;
  b->lanes_req = lanes;
  return DISPATCH(b->precision, batch_build_t, b);
}

int bq_batch_lanes(const bq_batch* b) { return b ? b->lanes : fail(BQ_EINVAL, "NULL batch"); }

int bq_batch_set_graph_steps(bq_batch* b, int32_t steps) {
  if (!b || steps < 0) return fail(BQ_EINVAL, "bad argument");
  b->graph_steps = steps;
  return BQ_OK;
}

int bq_batch_autotune(bq_batch* b, int32_t steps_per_trial, bq_tune* out) {
  if (!b || !out || steps_per_trial < 1) return fail(BQ_EINVAL, "bad argument");
  const int rc = static_owner_ok(b);
  if (rc) return rc;
  return DISPATCH(b->precision, batch_autotune_t, b, steps_per_trial, out);
}

int bq_batch_set_tune(bq_batch* b, const bq_tune* t) {
  if (!b || !t) return fail(BQ_EINVAL, "NULL argument");
  const int rc = static_owner_ok(b);
  if (rc) return rc;
  return set_tune(b, t);
}

int bq_batch_get_tune(const bq_batch* b, bq_tune* out) {
  if (!b || !out) return fail(BQ_EINVAL, "NULL argument");
  *out = bq_tune{b->lanes, b->graph_steps, b->rblock, b->swizzle, b->segs, b->ty, b->mx, 0.0};
  return BQ_OK;
}

int bq_batch_free(bq_batch* b) {
  if (!b) return fail(BQ_EINVAL, "NULL batch");
  (void)hipStreamSynchronize(b->stream);
  for (hipStream_t ls : b->lane)
    if (ls) (void)hipStreamSynchronize(ls);
  graph_del(b->L.graph);
  event_del(b->ev_fork);
  for (int l = 0; l < MAX_LANES; ++l) {
    graph_del(b->G[l].graph);
    event_del(b->ev_join[l]);
    stream_del(b->lane[l]);
  }
  release_static(b);
  if (b->mem) (void)hipFree(b->mem);
  delete b;
  return BQ_OK;
}

}  // extern "C"
