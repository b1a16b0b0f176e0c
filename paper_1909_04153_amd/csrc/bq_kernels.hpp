// bq_kernels.hpp -- gfx950 kernels of one adaptive-AB3 extended-Boussinesq
// time step (arXiv 1909.04153, Sec. 2-3).
//
// Data layout (per domain, all in the caller's workspace):
//   * state fields with two ghost layers (Sec. 3.3), row-major, row pitch a
//     multiple of 256 B and interior column 0 256-B aligned:
//       w[2] (double-buffered), P[3], Q[3] (rings: slot n % 3 = level n);
//   * interior-only fields: E, F, G rings (slot n % 3), local solutions
//     xhP, xhQ of the chunked line solves, cell still-water depth;
//   * corner still-water depth Dc with two mirrored ghost corner layers;
//   * per-chunk boundary/interface values of the line solves, [chunk][line];
//   * one FP64 DevState: time, Delta t history, weights, status.
//
// Per step (one launch each, over all domains of a batch):
//   k_dt      Delta t from the CFL maximum (Eq. 22) and Eq. (47), AB3 weights
//             (Eq. 42) and F*/G* weights (Eq. 43-46) in FP64, wavemaker
//             ghost values at t_{n+1};
//   k_rhs     LDS tile (64 x TY + halo 2): KP07 fluxes, bed source,
//             dispersion, friction, F*/G* of the weighted P/Q history, AB3
//             update of w and of U*, V* (as increments); then the chunk-local
//             tridiagonal solves of Eq. (19)-(20) for the P, Q increments;
//   k_reduced per line: the chunk-interface recurrence that couples the
//             chunk-local solutions into the exact line solution;
//   k_final   P, Q = local solution + the chunk systems' response to the
//             neighbour-chunk values, sponge, ghost cells of the new state,
//             CFL maximum of the new state.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bqk {

enum { WALL = 0, SINE = 1, SPONGE = 2, IRREGULAR = 3, TIMESERIES = 4 };
// west sides whose ghost cells are prescribed (wavemakers, time series)
__host__ __device__ inline bool west_driven(int bc) { return bc == SINE || bc == IRREGULAR || bc == TIMESERIES; }
enum { ST_OK = 0, ST_ENONFINITE = -4, ST_EDTMIN = -5, ST_EDONE = -7 };

constexpr int TX = 64;      // tile width (cells)
constexpr int NT = 256;     // threads per tile block
constexpr int NDIAG = 256;  // blocks of the diagnostic sums

struct alignas(64) DevState {
  // committed state
  double t;                 // time of the current state
  double dt1, dt2, dt3;     // Delta t of the last three steps (dt1 most recent)
  long long n;              // steps taken
  int status;
  int pending;              // a step was scheduled by k_dt and is not yet committed
  // the step being taken
  double dt;
  double alpha[3];
  double beta[3];
  double gamma[4];          // corrector weights of X^{n+1*}, X^n, X^{n-1}, X^{n-2}
  double t_next;
  double gw[2], gP[2];      // wavemaker ghost values (cells -1, -2) at t_next
  double smax_used;         // CFL maximum the step's Delta t was taken from
  int halt;                 // 1 = kernels of this step leave the domain untouched
  int slot;                 // n % 3 of the step being taken
  unsigned long long smax_bits;  // running max of the speeds of the new state
  double mass, energy;      // diagnostics (filled on demand)
  double pad[2];
};

template <typename T>
struct DomDev {
  int nx, ny;
  int pitch, xoff;          // ghosted fields: (i, j) at (j + 2) * pitch + xoff + i
  int ipitch;               // interior fields: (i, j) at j * ipitch + i
  int cpitch;               // corners: (ic, jc) at (jc + 2) * cpitch + ic + 2
  int cx, cy;               // chunks per x-line / y-line
  int mx, my;               // chunk lengths
  int tiles_x, tiles_y;
  int bc[4];
  int fstar_order, fixed_dt, n_waves, any_sponge;
  int ts_n;                 // time-series samples (BC TIMESERIES on the west side)
  int runup;                // 1 = keep the run-up record wmax
  int corrector;            // 1 = AB3 predictor + Adams-Moulton corrector
  T dx, dy, g, B, Bc, gn2, cf, theta, eps;
  T runup_delta;
  // reciprocals of the grid spacing combinations used by the stencils
  T idx, idy, i2dx, i2dy, idx2, idy2, i4dxdy, i2dx3, i2dy3, i2dxdy2, i2dx2dy;
  // constants of the Eq. (21) coefficients per direction: 1/(2h), (B+1/3)/h^2, 1/(6h)
  T tcx[3], tcy[3];
  T sponge_w[4];
  T sponge_sigma;
  double dx_d, dy_d, g_d, cfl, ema_alpha, dt_init, dt_max, dt_min, wave_ramp, t_end, ts_dt;
  T* w[3];                  // surface double buffer; w[2] holds the predicted surface
                            // of a predictor-corrector step
  T* P[3];
  T* Q[3];
  T* E[3];
  T* F[3];
  T* G[3];
  T* Dc;
  T* Dbar;
  T* xhP;
  T* xhQ;
  T* chx;                   // [2][cx][ny]: local solution at chunk first / last
  T* chy;                   // [2][cy][nx]
  T* rsx;                   // [6][cx][ny]: static interface-recurrence coefficients
  T* rsy;                   // [6][cy][nx]
  T* ifx;                   // [2][cx][ny]: neighbour values left / right of a chunk
  T* ify;                   // [2][cy][nx]
  double* smax_tile;        // per tile: CFL maximum of the new state (written by the finalize kernel)
  double* diag_part;        // [2][NDIAG]: per-block mass / energy partial sums
  double* wave;             // [4][n_waves]: amplitude, omega, phase, wave number;
                            // time series: [2][ts_n]: eta, P samples
  T* wmax;                  // run-up record (interior layout), if kept
  double* io;               // nx * ny doubles of staging for host transfers
  DevState* st;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Field pointers live in the per-domain descriptor in device memory, so the
// compiler cannot tell they address global memory and would emit flat
// accesses (which also wait on the LDS counter); name the address space.
template <typename T>
using gp = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gp<T> gbl(T* p) {
  return (gp<T>)p;
}

// A pointer read from device memory that is the same in every lane: pin it
// to scalar registers, so that loads through it take the scalar-base form.
template <typename P>
__device__ __forceinline__ P* uni(P* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
  return (P*)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
// materialise a value in a register at this point (the compiler may not sink
// its computation to a later use)
template <typename T>
__device__ __forceinline__ void pin(T& v) {
  __asm__ volatile("" : "+v"(v));
}

// Element `off` of a field whose base address is the same for the whole
// block: a scalar base plus a 32-bit per-lane byte offset (the workspace
// keeps every field below 4 GiB).
template <typename T>
__device__ __forceinline__ T ldu(const T* base, unsigned off) {
  const gp<const char> b = (gp<const char>)(const char*)base;
  return *(gp<const T>)(b + (unsigned)(off * (unsigned)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void stu(T* base, unsigned off, T v) {
  const gp<char> b = (gp<char>)(char*)base;
  *(gp<T>)(b + (unsigned)(off * (unsigned)sizeof(T))) = v;
}

// Square root, reciprocal and cube root.  FP64 uses the correctly rounded
// operations (parity with the FP64 oracle at 1e-12); FP32 uses the hardware
// transcendental instructions (about 1 ulp), whose error is far below the
// FP32 path's own rounding of the state.
template <typename T> __device__ __forceinline__ T fsqrt(T x);
template <typename T> __device__ __forceinline__ T frcp(T x);
template <typename T> __device__ __forceinline__ T frcbrt(T x);   // x^(-1/3), x > 0
template <> __device__ __forceinline__ double fsqrt<double>(double x) { return sqrt(x); }
template <> __device__ __forceinline__ double frcp<double>(double x) { return 1.0 / x; }
template <> __device__ __forceinline__ double frcbrt<double>(double x) { return 1.0 / cbrt(x); }
template <> __device__ __forceinline__ float fsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ float frcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
// a / b: correctly rounded in FP64, reciprocal-multiply in FP32
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
// The hardware log takes a subnormal input as 0 (giving +inf here, and a
// NaN once multiplied by the zero velocity of a film that thin): depths are
// raised to the smallest normal value first, which leaves h^(-1/3) finite
// (< 5e12) for every h > 0.
template <> __device__ __forceinline__ float frcbrt<float>(float x) {
  return __builtin_amdgcn_exp2f(-0.33333333f * __builtin_amdgcn_logf(__builtin_fmaxf(x, 1.17549435e-38f)));
}

// generalised minmod of three values: the one nearest zero when all three
// share a sign, else zero
template <typename T>
__device__ __forceinline__ T gmm(T a, T b, T c) {
  const T lo = fmin(a, fmin(b, c));
  const T hi = fmax(a, fmax(b, c));
  return lo > T(0) ? lo : (hi < T(0) ? hi : T(0));
}
// FP32: med3(a, c, 0) is minmod(a, c), and minmod(minmod(a, c), b) is the
// same value as above, in two median-of-three instructions
template <>
__device__ __forceinline__ float gmm<float>(float a, float b, float c) {
  return __builtin_amdgcn_fmed3f(__builtin_amdgcn_fmed3f(a, c, 0.0f), b, 0.0f);
}

// half the limited slope (times the cell size) of q at a cell from its two
// neighbours, ht = theta / 2: minmod(ht (q0 - qm), (qp - qm) / 4, ht (qp - q0));
// theta = 0 (LIM false; the caller takes that choice once per tile) selects
// the unlimited central slope.  Halving is exact, so the face values
// q0 -/+ hslope equal q0 -/+ slope / 2.
template <bool LIM, typename T>
__device__ __forceinline__ T hslope(T qm, T q0, T qp, T ht) {
  const T c = T(0.25) * (qp - qm);
  return LIM ? gmm(ht * (q0 - qm), c, ht * (qp - q0)) : c;
}

// Velocity factor of the KP07 desingularisation, u = q * vfac(h):
//   sqrt(2) h / sqrt(h^4 + max(h^4, eps)),
// which is exactly 1/h when h^4 >= eps (taken directly there).
template <typename T>
__device__ __forceinline__ T vfac(T h, T eps) {
  const T h2 = h * h;
  const T h4 = h2 * h2;
  if (h4 >= eps) return frcp(h);
  return T(1.4142135623730951) * h * frcp(fsqrt(h4 + eps));
}

template <typename T>
__device__ __forceinline__ T desing(T q, T h, T eps) {
  return q * vfac(h, eps);
}

// cell-average still-water depth from its four corners
template <typename T>
__device__ __forceinline__ T dbar4(T a, T b, T c, T d) {
  return T(0.25) * (a + b + c + d);
}

// max(D, 0) and min(D, 0) of a still-water depth (always finite).  FP32 takes
// one median-of-three: a plain fmax of a value read from memory costs a
// second instruction that quiets a possible signalling NaN first.
template <typename T>
__device__ __forceinline__ T dpos(T D) {
  return fmax(D, T(0));
}
template <>
__device__ __forceinline__ float dpos<float>(float D) {
  return __builtin_amdgcn_fmed3f(D, 0.0f, 3.402823466e38f);
}
template <typename T>
__device__ __forceinline__ T dneg(T D) {
  return fmin(D, T(0));
}
template <>
__device__ __forceinline__ float dneg<float>(float D) {
  return __builtin_amdgcn_fmed3f(D, 0.0f, -3.402823466e38f);
}

// max(a, b) of finite values; FP32 again without the quieting instruction
template <typename T>
__device__ __forceinline__ T dmax_nq(T a, T b) {
  return fmax(a, b);
}
template <>
__device__ __forceinline__ float dmax_nq<float>(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, 3.402823466e38f);
}

// Piecewise-linear w at a cell's low/high faces with the KP07 positivity
// correction; Dlo/Dhi are the still-water depths at the faces (bed = -D).
template <bool LIM, typename T>
__device__ __forceinline__ void recon_w(T wm, T w0, T wp, T ht, T Dlo, T Dhi, T& wlo, T& whi) {
  const T s = hslope<LIM>(wm, w0, wp, ht);
  wlo = w0 - s;
  whi = w0 + s;
  if (whi + Dhi < T(0)) {
    whi = -Dhi;
    wlo = T(2) * w0 + Dhi;
  } else if (wlo + Dlo < T(0)) {
    wlo = -Dlo;
    whi = T(2) * w0 + Dlo;
  }
}

// One side of a face.  The hydrostatic pressure g h^2 / 2 is carried as its
// departure from the still-water value g D+^2 / 2 at the face, D+ = max(D, 0):
//   pp = g (h - D+)(h + D+) / 2,
//   h - D+ = w (wet face below the still-water line), -D (dry there), h (land).
// The still-water parts of the flux differences and of the well-balanced bed
// source cancel exactly except in cells whose two faces straddle the
// still-water line (see add_shore); keeping them would leave FP32 with a
// difference of large numbers in deep water.
template <typename T>
struct Side {
  T w, h, un, ut, qn, qt, dev, pp;
};

template <typename T>
__device__ __forceinline__ Side<T> make_side(T w, T qn, T qt, T Dface, T eps, T g) {
  Side<T> s;
  s.w = w;
  s.h = fmax(w + Dface, T(0));
  const T h2 = s.h * s.h;
  const T h4 = h2 * h2;
  // FP32: for h^4 >= eps, u = q / h and the recomputed discharge h u is q
  // itself (exact identities); FP64 evaluates the general expression, so
  // that at wet/dry fronts it rounds like the FP64 reference
  if (sizeof(T) == 4 && h4 >= eps) {
    const T vf = frcp(s.h);
    s.un = qn * vf;
    s.ut = qt * vf;
    s.qn = qn;
    s.qt = qt;
  } else {
    // u = sqrt(2) h q / sqrt(h^4 + max(h^4, eps)), recomputed discharge h u
    const T den = fsqrt(h4 + fmax(h4, eps));
    const T sh = T(1.4142135623730951) * s.h;
    s.un = fdiv(sh * qn, den);
    s.ut = fdiv(sh * qt, den);
    s.qn = s.h * s.un;
    s.qt = s.h * s.ut;
  }
  const T Dp = dpos(Dface);
  // (h > 0 exactly when w > -D, so below the still-water line dev is max(w, -D))
  s.dev = Dface > T(0) ? dmax_nq(w, -Dface) : s.h;
  s.pp = T(0.5) * g * s.dev * (s.h + Dp);
  return s;
}

// central-upwind flux normal to a face, components (mass, normal momentum,
// tangential momentum); the normal momentum flux excludes g D^2 / 2
template <typename T>
__device__ __forceinline__ void cu_flux(const Side<T>& L, const Side<T>& R, T g, T Dface, T& f0, T& fn, T& ft) {
  const T cL = fsqrt(g * L.h), cR = fsqrt(g * R.h);
  const T ap = fmax(fmax(L.un + cL, R.un + cR), T(0));
  const T am = fmin(fmin(L.un - cL, R.un - cR), T(0));
  const T den = ap - am;
  if (den == T(0)) {
    // both sides dry and at rest: the full flux is zero
    const T Dp = dpos(Dface);
    f0 = ft = T(0);
    fn = -T(0.5) * g * Dp * Dp;
    return;
  }
  const T inv = frcp(den);
  const T dis = ap * am * inv;
  const T pL = L.qn * L.un + L.pp;
  const T pR = R.qn * R.un + R.pp;
  f0 = (ap * L.qn - am * R.qn) * inv + dis * (R.w - L.w);
  fn = (ap * pL - am * pR) * inv + dis * (R.qn - L.qn);
  ft = (ap * L.qn * L.ut - am * R.qn * R.ut) * inv + dis * (R.qt - L.qt);
}

// still-water remainder of (bed source - pressure flux difference) in a cell
// whose low/high faces have still-water depths Dl, Dh: zero unless exactly
// one of them is below the still-water line
template <typename T>
__device__ __forceinline__ void add_shore(T& bed, T Dl, T Dh, T g) {
  // a branch, not a select: shore faces are rare, so most waves skip it
  if (__builtin_expect((Dl > T(0)) != (Dh > T(0)), 0)) {
    const T pl = dpos(Dl), ph = dpos(Dh);
    bed += T(0.5) * g * ((Dh - Dl) * (ph + pl) - (ph * ph - pl * pl));
  }
}

// Coefficients of Eq. (21) at a cell from the still-water depths of the cell
// and its two neighbours along the line; tc = (1/(2h), (B+1/3)/h^2, 1/(6h)).
template <typename T>
__device__ __forceinline__ void tri_coef(T dm, T d0, T dp, const T* tc, T& a, T& b, T& c) {
  const T dd = (dp - dm) * tc[0];
  const T k = tc[1] * d0 * d0;
  const T s = d0 * dd * tc[2];
  a = s - k;
  b = T(1) + T(2) * k;
  c = -s - k;
}

// Chunk-local tridiagonal solve (zero coupling to the neighbouring chunks)
// of the m (<= M) unknowns of one chunk.  Dl[k * ds], k = 0..m+1, are the
// cell-average still-water depths of the chunk's cells with one neighbour on
// each side (d = max(D, 0)); tc are the Eq. (21) constants of the direction.
// fold_lo / fold_hi fold the odd mirror of a wall into the first / last
// diagonal.  rhs (stride rs) is overwritten with the solution; the forward
// sweep leaves y_k / u_k in rhs and keeps c_k / u_k in registers, so the
// backward sweep is one multiply-add per row (the loops are unrolled over M).
template <typename T, int M, bool FULL>
__device__ __forceinline__ void chunk_solve_db_(const T* Dl, int ds, int m, const T* tc, bool fold_lo, bool fold_hi,
                                                T* rhs, int rs) {
  if (FULL) m = M;
  T cu[M];                                     // c_k / u_k; rhs holds y_k / u_k
  T y_prev = T(0), iu_prev = T(1), c_prev = T(0);
#pragma unroll
  for (int k = 0; k < M; ++k) {
    if (FULL || k < m) {
      T a, b, c;
      tri_coef(dpos(Dl[k * ds]), dpos(Dl[(k + 1) * ds]), dpos(Dl[(k + 2) * ds]), tc, a, b, c);
      if (k == 0 && fold_lo) b -= a;
      if (k == m - 1 && fold_hi) b -= c;
      const T r = rhs[k * rs];
      T u, y;
      if (k == 0) {
        u = b;
        y = r;
      } else {
        const T l = a * iu_prev;
        u = b - l * c_prev;
        y = r - l * y_prev;
      }
      const T iu = frcp(u);
      cu[k] = c * iu;
      rhs[k * rs] = y * iu;
      y_prev = y;
      iu_prev = iu;
      c_prev = c;
    }
  }
  T x_next = T(0);
#pragma unroll
  for (int k = M - 1; k >= 0; --k) {
    if (FULL || k < m) {
      const T y = rhs[k * rs];
      const T x = (k == m - 1) ? y : y - cu[k] * x_next;
      rhs[k * rs] = x;
      x_next = x;
    }
  }
}
// full chunks (the common case) take a branch-free unrolled path, so the
// LDS reads can be issued ahead of the dependent arithmetic
template <typename T, int M>
__device__ __forceinline__ void chunk_solve_db(const T* Dl, int ds, int m, const T* tc, bool fold_lo, bool fold_hi,
                                               T* rhs, int rs) {
  if (m == M) chunk_solve_db_<T, M, true>(Dl, ds, m, tc, fold_lo, fold_hi, rhs, rs);
  else chunk_solve_db_<T, M, false>(Dl, ds, m, tc, fold_lo, fold_hi, rhs, rs);
}

// Work-groups of a launch are dealt round-robin to the 8 XCDs (each with its
// own L2): block b runs on XCD b % 8.  Renumber so that every XCD walks a
// contiguous run of tiles; a tile's halo rows and columns are then mostly
// the neighbour tiles' interiors, fetched from HBM once into the same L2.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int xcd = b % NXCD, local = b / NXCD;
  const int per = nb / NXCD, rem = nb % NXCD;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// Response of a chunk system to a right-hand side that is zero except r0 in
// the first row and r1 in the last (the coupling to the neighbour chunks'
// end values), for a kernel that must stay light on registers.  The forward
// sweep keeps y_k / u_k and c_k / u_k in LDS (out, cu; stride rs), so the
// backward sweep is one multiply-add per row: x_k = y_k/u_k - (c_k/u_k) x_{k+1}.
// Each iteration issues the next row's LDS read before its own dependent
// arithmetic, so the read latency overlaps the pivot recurrence.
template <typename T>
__device__ __forceinline__ void chunk_edge_solve(const T* Dl, int ds, int m, const T* tc, bool fold_lo, bool fold_hi,
                                                 T r0, T r1, T* out, T* cu, int rs) {
  T d0 = dpos(Dl[0]), d1 = dpos(Dl[ds]), d2 = dpos(Dl[2 * ds]);
  T r = m == 1 ? r0 + r1 : r0;
  T y_prev = T(0), iu_prev = T(1), c_prev = T(0);
  for (int k = 0; k < m; ++k) {
    const T d3 = dpos(Dl[(k + 3 <= m + 1 ? k + 3 : m + 1) * ds]);
    T a, b, c;
    tri_coef(d0, d1, d2, tc, a, b, c);
    if (k == 0 && fold_lo) b -= a;
    if (k == m - 1 && fold_hi) b -= c;
    T u, y;
    if (k == 0) {
      u = b;
      y = r;
    } else {
      const T l = a * iu_prev;
      u = b - l * c_prev;
      y = r - l * y_prev;
    }
    const T iu = frcp(u);
    out[k * rs] = y * iu;
    cu[k * rs] = c * iu;
    y_prev = y;
    iu_prev = iu;
    c_prev = c;
    d0 = d1;
    d1 = d2;
    d2 = d3;
    r = k + 2 == m ? r1 : T(0);
  }
  T x_next = out[(m - 1) * rs];
  if (m < 2) return;
  T yk = out[(m - 2) * rs], ck = cu[(m - 2) * rs];
  for (int k = m - 2; k >= 0; --k) {
    const int kn = k > 0 ? k - 1 : 0;
    const T yn = out[kn * rs], cn = cu[kn * rs];
    const T x = yk - ck * x_next;
    out[k * rs] = x;
    x_next = x;
    yk = yn;
    ck = cn;
  }
}

// Work item (tile or line) of a launch -> (domain, index within it).  A
// batch carries a packed map, one word per item: domain << MAP_SHIFT | index
// (a single dependent load, no search); a single domain is the identity.
constexpr int MAP_SHIFT = 18;
__device__ __forceinline__ void locate(const int* map, int nd, int idx, int& dom, int& loc) {
  if (nd == 1) {
    dom = 0;
    loc = idx;
    return;
  }
  const int v = map[idx];
  dom = v >> MAP_SHIFT;
  loc = v & ((1 << MAP_SHIFT) - 1);
}

// ---------------------------------------------------------------------------
// k_dt: Delta t and weights of the step (one block per domain)
// ---------------------------------------------------------------------------

// whole-state copies through the global address space: one batch of loads
// or stores (a generic pointer would make them flat accesses, which also
// wait on the LDS counter)
__device__ __forceinline__ DevState load_state(const DevState* st) {
  constexpr int NW = (int)(sizeof(DevState) / 8);
  static_assert(sizeof(DevState) % 8 == 0, "state is whole 8-byte words");
  const gp<const unsigned long long> src = gbl((const unsigned long long*)st);
  unsigned long long w[NW];
#pragma unroll
  for (int k = 0; k < NW; ++k) w[k] = src[k];
  DevState S;
  __builtin_memcpy(&S, w, sizeof S);
  return S;
}
__device__ __forceinline__ void store_state(DevState* st, const DevState& S) {
  constexpr int NW = (int)(sizeof(DevState) / 8);
  unsigned long long w[NW];
  __builtin_memcpy(w, &S, sizeof S);
  const gp<unsigned long long> dst = gbl((unsigned long long*)st);
#pragma unroll
  for (int k = 0; k < NW; ++k) dst[k] = w[k];
}

__device__ __forceinline__ void commit(DevState& st) {
  if (st.pending) {
    st.t = st.t_next;
    st.dt3 = st.dt2;
    st.dt2 = st.dt1;
    st.dt1 = st.dt;
    st.n += 1;
    st.pending = 0;
  }
}

template <typename T>
__device__ void west_ghosts(const DomDev<T>& D, double t, double* gw, double* gP) {
  // surface and flux prescribed at the centres of west ghost cells -1 and -2
  // (x = -dx/2, -3dx/2) at time t; only thread 0's result is used
  const int tid = threadIdx.x;
  const double r = D.wave_ramp > 0.0 ? 1.0 - exp(-(t / D.wave_ramp) * (t / D.wave_ramp)) : 1.0;
  if (D.bc[0] == TIMESERIES) {
    // samples interpolated linearly in time, held outside their span; the
    // same values in both ghost columns
    if (tid == 0) {
      const int n = D.ts_n;
      const double* se = D.wave;
      const double* sp = D.wave + n;
      const double s = t / D.ts_dt;
      double e, p;
      if (!(s > 0.0)) {
        e = se[0];
        p = sp[0];
      } else if (s >= (double)(n - 1)) {
        e = se[n - 1];
        p = sp[n - 1];
      } else {
        const int k = (int)s;
        const double f = s - (double)k;
        e = se[k] + f * (se[k + 1] - se[k]);
        p = sp[k] + f * (sp[k + 1] - sp[k]);
      }
      gw[0] = gw[1] = r * e;
      gP[0] = gP[1] = r * p;
    }
    return;
  }
  // incident wave train: sum of the components
  __shared__ double red[4][64];
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  const int nw = D.n_waves;
  for (int m = tid; tid < 64 && m < nw; m += 64) {
    const double amp = D.wave[m], om = D.wave[nw + m], ph = D.wave[2 * nw + m], k = D.wave[3 * nw + m];
    const double s1 = r * amp * sin(om * t + 0.5 * k * D.dx_d + ph);
    const double s2 = r * amp * sin(om * t + 1.5 * k * D.dx_d + ph);
    a0 += s1;
    a1 += om / k * s1;
    a2 += s2;
    a3 += om / k * s2;
  }
  if (tid < 64) {
    red[0][tid] = a0; red[1][tid] = a1; red[2][tid] = a2; red[3][tid] = a3;
  }
  __syncthreads();
  if (tid == 0) {
    // lanes past the component count hold zeros: summing them would change
    // nothing but the time
    double s[4] = {0, 0, 0, 0};
    const int nq = nw < 64 ? nw : 64;
    for (int q = 0; q < nq; ++q)
      for (int c = 0; c < 4; ++c) s[c] += red[c][q];
    gw[0] = s[0]; gP[0] = s[1]; gw[1] = s[2]; gP[1] = s[3];
  }
  __syncthreads();
}

// one block of DT_THREADS per domain
constexpr int DT_THREADS = 256;

template <typename T>
__global__ void __launch_bounds__(DT_THREADS) k_dt(const DomDev<T>* __restrict__ doms, double dt_prescribed) {
  const DomDev<T>& D = doms[blockIdx.x];
  DevState* st = D.st;
  __shared__ int go;
  __shared__ double tn;
  // The state and the step controls are loaded first, in one batch, so their
  // latency overlaps the reduction below (the barrier in it keeps the state's
  // loads here); the decision further down is then register arithmetic.
  DevState S = load_state(st);
  const double t_end = D.t_end, cfl = D.cfl, ema = D.ema_alpha, dt_init = D.dt_init, dt_max = D.dt_max,
               dt_min = D.dt_min;
  const int fixed_dt = D.fixed_dt, fstar_order = D.fstar_order;
  __asm__ volatile("" ::"s"(t_end), "s"(cfl), "s"(ema), "s"(dt_init), "s"(dt_max), "s"(dt_min), "s"(fixed_dt),
                   "s"(fstar_order));
  // CFL maximum of the current state: the finalize kernel's per-tile maxima
  // (a NaN there is already +inf) and the initial state's value
  double tmax = 0.0;
  {
    // eight independent loads in flight per lane (a large domain has
    // thousands of tiles; one dependent load at a time would serialise them)
    const int ntiles = D.tiles_x * D.tiles_y;
    const gp<const double> sp = gbl((const double*)D.smax_tile);
    double tm[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) tm[u] = 0.0;
    for (int k0 = threadIdx.x; k0 < ntiles; k0 += 8 * DT_THREADS) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = k0 + DT_THREADS * u;
        tm[u] = fmax(tm[u], k < ntiles ? sp[k] : 0.0);
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) tmax = fmax(tmax, tm[u]);
    for (int o = 32; o > 0; o >>= 1) tmax = fmax(tmax, __shfl_xor(tmax, o, 64));
    __shared__ double wmax[DT_THREADS / 64];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = tmax;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < DT_THREADS / 64; ++w) tmax = fmax(tmax, wmax[w]);
  }
  if (threadIdx.x == 0) {
    // one thread decides the step on the register copy of the state and
    // stores it back in one batch
    commit(S);
    go = 0;
    S.halt = 1;
    if (S.status == ST_OK) {
      if (t_end > 0.0 && S.t >= t_end) {
        S.status = ST_EDONE;
      } else {
        const double s = fmax(__longlong_as_double((long long)S.smax_bits), tmax);
        if (!(s <= 1.79e308)) {
          S.status = ST_ENONFINITE;
        } else {
          const long long n = S.n;
          double dt;
          bool ok = true;
          if (dt_prescribed > 0.0) {
            dt = dt_prescribed;
          } else if (fixed_dt) {
            dt = dt_init;
          } else {
            const double cand = s > 0.0 ? cfl / s : dt_max;
            if (n == 0) dt = dt_init > 0.0 ? dt_init : cand;
            else dt = cand <= S.dt1 ? cand : ema * cand + (1.0 - ema) * S.dt1;
            dt = fmin(dt, dt_max);
            if (dt < dt_min) {
              S.status = ST_EDTMIN;
              ok = false;
            }
          }
          if (ok) {
            const double h0 = dt, h1 = S.dt1, h2 = S.dt2;
            double a0 = h0, a1 = 0.0, a2 = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0;
            if (n == 1) {
              b0 = h0 / h1;
              b1 = -b0;
            } else if (n >= 2) {
              // Eq. (42): integral over [t_n, t_n + h0] of the quadratic
              // through the three last nodes
              const double r1 = h0 / h1, s12 = h1 + h2;
              a0 = h0 / 6.0 * (r1 * (2.0 * h0 + 6.0 * h1 + 3.0 * h2) / s12 + 6.0);
              a1 = -h0 / 6.0 * (r1 * (2.0 * h0 + 3.0 * h1 + 3.0 * h2) / h2);
              a2 = h0 / 6.0 * ((h0 / h2) * (2.0 * h0 + 3.0 * h1) / s12);
              if (fstar_order == 1) {
                b0 = r1;
                b1 = -r1;
              } else {
                // Eq. (43) with (44)-(46) sum to the increment of the quadratic
                // through (t_{n-k}, F*^{n-k}) from t_n to t_n + h0
                b0 = (h0 + h1) * (h0 + s12) / (h1 * s12) - 1.0;
                b1 = -h0 * (h0 + s12) / (h1 * h2);
                b2 = h0 * (h0 + h1) / (h2 * s12);
              }
            }
            // Adams-Moulton corrector: integral over [t_n, t_n + h0] of the
            // Lagrange basis through t_{n+1}, t_n, t_{n-1}, t_{n-2} (closed
            // forms with a = h1, b = h1 + h2), the cubic from n = 2 on, the
            // quadratic at n = 1, the trapezoidal rule at n = 0
            double g0 = 0.5 * h0, g1 = 0.5 * h0, g2 = 0.0, g3 = 0.0;
            if (n == 1) {
              const double a = h1;
              g0 = h0 * (2.0 * h0 + 3.0 * a) / (6.0 * (h0 + a));
              g1 = h0 * (h0 + 3.0 * a) / (6.0 * a);
              g2 = -h0 * h0 * h0 / (6.0 * a * (a + h0));
            } else if (n >= 2) {
              const double a = h1, b = h1 + h2, hh = h0 * h0 * h0;
              g0 = h0 * (3.0 * h0 * h0 + 4.0 * (a + b) * h0 + 6.0 * a * b) / (12.0 * (h0 + a) * (h0 + b));
              g1 = h0 * (h0 * h0 + 2.0 * (a + b) * h0 + 6.0 * a * b) / (12.0 * a * b);
              g2 = -hh * (h0 + 2.0 * b) / (12.0 * a * (a + h0) * h2);
              g3 = hh * (h0 + 2.0 * a) / (12.0 * b * (b + h0) * h2);
            }
            S.dt = dt;
            S.alpha[0] = a0; S.alpha[1] = a1; S.alpha[2] = a2;
            S.gamma[0] = g0; S.gamma[1] = g1; S.gamma[2] = g2; S.gamma[3] = g3;
            S.beta[0] = b0; S.beta[1] = b1; S.beta[2] = b2;
            S.t_next = S.t + dt;
            S.smax_used = s;
            S.slot = (int)(n % 3);
            S.smax_bits = 0ull;
            S.pending = 1;
            S.halt = 0;
            go = 1;
            tn = S.t_next;
          }
        }
      }
    }
    store_state(st, S);
  }
  __syncthreads();
  if (go && west_driven(D.bc[0])) {
    double gw[2], gP[2];
    west_ghosts(D, tn, gw, gP);
    if (threadIdx.x == 0) {
      st->gw[0] = gw[0]; st->gw[1] = gw[1]; st->gP[0] = gP[0]; st->gP[1] = gP[1];
    }
  }
}

template <typename T>
__global__ void k_commit(const DomDev<T>* __restrict__ doms, int nd) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d < nd) commit(*doms[d].st);
}

// ---------------------------------------------------------------------------
// k_rhs: fused spatial operator, AB3 update and chunk-local line solves
// ---------------------------------------------------------------------------

template <typename T, int TY, int MX>
struct alignas(16) RhsSmem {
  static constexpr int WX = TX + 4, WY = TY + 4;      // radius-2 tiles
  static constexpr int BX = TX + 2, BY = TY + 2;      // radius-1 tiles
  static constexpr int CXN = TX + 5, CYN = TY + 5;    // corners
  static constexpr int TXP = TX + 1;                  // padded row of the solve buffers
  // LDS row pitch of the radius-2 tiles: 5 mod 64 words, so the x-segment
  // threads (stride 4 within a row, 4 rows per wave) hit 64 distinct banks
  static constexpr int LW = WX + 1;
  static constexpr int AXP = TX + 1;                  // row pitch of ax (same reason)
  T w[WY * LW];
  T p[WY * LW];
  T q[WY * LW];
  T db[WY * LW];                                      // cell still-water depth
  union {
    struct {
      T pt[BY * BX];                                  // sum_k beta_k P^{n-k} (until the F* terms are formed)
      T qt[BY * BX];
    } h;
    T ax[3][TY * AXP];                                // x-direction parts of E, F, G per cell
    struct {
      T u[TY * TXP];
      T v[TY * TXP];
    } s;
  } x;
  T dc[CYN * CXN];
};

// CORR = false: the AB3 step of Eq. (42)-(43) from level n (the predictor
// when the domain runs the corrector, which then writes the surface to w[2]).
// CORR = true: the Adams-Moulton corrector from the same base w^n, U*^n, V*^n
// with the spatial operator of the predicted level (slot of level n+1, w[2])
// and the F*, G* terms as their change F*(P*) - F*(P^n); domains without the
// corrector are skipped.
template <typename T, int TY, int MX, bool CORR>
__global__ void __launch_bounds__(NT) k_rhs(const DomDev<T>* __restrict__ doms, const int* __restrict__ tile_map,
                                           int nd, int swizzle) {
  using S = RhsSmem<T, TY, MX>;
  constexpr int WX = S::WX, LW = S::LW, AXP = S::AXP, BX = S::BX, CXN = S::CXN, TXP = S::TXP;
  constexpr int CPT = (TX * TY) / NT;                 // cells per thread
  static_assert((TX * TY) % NT == 0, "tile must be a multiple of the block");
  __shared__ S sm;
  int dom, tile;
  // swizzle = 1: XCD-aware tile order (each XCD walks a contiguous run)
  locate(tile_map, nd, swizzle ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x, dom, tile);
  const DomDev<T>& D = doms[dom];
  const DevState* st = D.st;
  if (st->halt) return;
  if (CORR && !D.corrector) return;
  const int i0 = (tile % D.tiles_x) * TX, j0 = (tile / D.tiles_x) * TY;
  const int nx = D.nx, ny = D.ny, tid = threadIdx.x;
  const int slot = uni(st->slot), par = uni((int)(st->n & 1));
  const int s1 = slot == 0 ? 2 : slot - 1, s2 = slot == 2 ? 0 : slot + 1;
  const T beta0 = CORR ? T(1) : (T)st->beta[0];
  const T beta1 = CORR ? T(-1) : (T)st->beta[1];
  const T beta2 = CORR ? T(0) : (T)st->beta[2];
  const bool hist = CORR || st->beta[0] != 0.0 || st->beta[1] != 0.0 || st->beta[2] != 0.0;
  const int pitch = uni(D.pitch), xoff = uni(D.xoff), ipitch = uni(D.ipitch), cpitch = uni(D.cpitch);
  // Cells of a thread in the per-cell phases: column cY, rows rY0 .. rY0+CPT-1
  // (consecutive rows, so the vertical stencils of a thread's cells overlap).
  const int cY = tid % TX, rY0 = (tid / TX) * CPT;
  static_assert((NT / TX) * CPT == TY, "per-cell mapping covers the tile");
  const unsigned oI = (unsigned)((j0 + rY0) * ipitch + i0 + cY);          // interior fields
  const unsigned oG = (unsigned)((j0 + rY0 + 2) * pitch + xoff + i0 + cY);  // ghosted fields

  // ---- phase 0: issue every load of the tile before the first LDS store ----
  // Each LDS tile of width Wd is read RG = NT / Wd rows per round: thread
  // (r0, c) = (tid / Wd, tid % Wd) loads rows r0 + RG k, so the LDS index is
  // a per-thread base plus a constant.  The threads beyond RG whole rows and
  // the rows past the tile in the last round repeat a row of the tile (same
  // values to the same LDS words), so every round is branch-free.  The
  // workspace pads every field to whole tiles plus the halo, so no index is
  // clamped to the domain: values outside it only reach cells outside it.
  constexpr int RGW = NT / WX, KW = (S::WY + RGW - 1) / RGW;
  constexpr int RGC = NT / CXN, KC = (S::CYN + RGC - 1) / RGC;
  constexpr int RGB = NT / BX, KB = (S::BY + RGB - 1) / RGB;
  const int rW = min(tid / WX, RGW - 1), cW = tid - (tid / WX) * WX;
  const int rC = min(tid / CXN, RGC - 1), cC = tid - (tid / CXN) * CXN;
  const int rB = min(tid / BX, RGB - 1), cB = tid - (tid / BX) * BX;
  auto rowW = [&](int k) { return k < KW - 1 ? rW + RGW * k : min(rW + RGW * k, S::WY - 1); };
  auto rowC = [&](int k) { return k < KC - 1 ? rC + RGC * k : min(rC + RGC * k, S::CYN - 1); };
  auto rowB = [&](int k) { return k < KB - 1 ? rB + RGB * k : min(rB + RGB * k, S::BY - 1); };
  // E, F, G history of this thread's cells (consumed in phase 2)
  // combined as the AB3 history terms alpha_1 X^{n-1} + alpha_2 X^{n-2}
  // (Eq. 42) right away, so three values per cell stay live, not six; the
  // corrector's terms are gamma_1 X^n + gamma_2 X^{n-1} + gamma_3 X^{n-2}
  const T a1 = (T)(CORR ? st->gamma[1] : st->alpha[1]), a2 = (T)(CORR ? st->gamma[2] : st->alpha[2]);
  T hE[CPT], hF[CPT], hG[CPT];
  {
    const int l1 = CORR ? slot : s1, l2 = CORR ? s1 : s2;
    const T* E1 = uni((const T*)D.E[l1]);
    const T* E2 = uni((const T*)D.E[l2]);
    const T* F1 = uni((const T*)D.F[l1]);
    const T* F2 = uni((const T*)D.F[l2]);
    const T* G1 = uni((const T*)D.G[l1]);
    const T* G2 = uni((const T*)D.G[l2]);
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const unsigned o = oI + (unsigned)(q * ipitch);
      hE[q] = a1 * ldu(E1, o) + a2 * ldu(E2, o);
      hF[q] = a1 * ldu(F1, o) + a2 * ldu(F2, o);
      hG[q] = a1 * ldu(G1, o) + a2 * ldu(G2, o);
    }
    if (CORR) {
      const T a3 = (T)st->gamma[3];
      const T* E3 = uni((const T*)D.E[s2]);
      const T* F3 = uni((const T*)D.F[s2]);
      const T* G3 = uni((const T*)D.G[s2]);
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        const unsigned o = oI + (unsigned)(q * ipitch);
        hE[q] += a3 * ldu(E3, o);
        hF[q] += a3 * ldu(F3, o);
        hG[q] += a3 * ldu(G3, o);
      }
    }
  }
  T rw[KW], rp[KW], rq[KW], rc[KC], h1p[KB], h2p[KB], h1q[KB], h2q[KB];
  {
    // the state the spatial operator is taken of: level n, or the predicted level
    const T* w = uni((const T*)(CORR ? D.w[2] : D.w[par]));
    const T* Pn = uni((const T*)D.P[CORR ? s2 : slot]);
    const T* Qn = uni((const T*)D.Q[CORR ? s2 : slot]);
    const unsigned oW = (unsigned)(j0 * pitch + xoff + i0 - 2 + cW);       // radius-2 tile
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      const unsigned o = oW + (unsigned)(rowW(k) * pitch);
      rw[k] = ldu(w, o);
      rp[k] = ldu(Pn, o);
      rq[k] = ldu(Qn, o);
    }
    const T* Dc = uni((const T*)D.Dc);
    const unsigned oC = (unsigned)(j0 * cpitch + i0 + cC);                 // corners
#pragma unroll
    for (int k = 0; k < KC; ++k) rc[k] = ldu(Dc, oC + (unsigned)(rowC(k) * cpitch));
    const unsigned oB = (unsigned)((j0 + 1) * pitch + xoff + i0 - 1 + cB);   // radius-1 tile
    if (CORR) {
      // level n, for the change of the F*, G* terms
      const T* P1 = uni((const T*)D.P[slot]);
      const T* Q1 = uni((const T*)D.Q[slot]);
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const unsigned o = oB + (unsigned)(rowB(k) * pitch);
        h1p[k] = ldu(P1, o);
        h1q[k] = ldu(Q1, o);
        h2p[k] = h2q[k] = T(0);
      }
    } else if (hist) {
      const T* P1 = uni((const T*)D.P[s1]);
      const T* P2 = uni((const T*)D.P[s2]);
      const T* Q1 = uni((const T*)D.Q[s1]);
      const T* Q2 = uni((const T*)D.Q[s2]);
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const unsigned o = oB + (unsigned)(rowB(k) * pitch);
        h1p[k] = ldu(P1, o);
        h2p[k] = ldu(P2, o);
        h1q[k] = ldu(Q1, o);
        h2q[k] = ldu(Q2, o);
      }
    } else {
#pragma unroll
      for (int k = 0; k < KB; ++k) h1p[k] = h2p[k] = h1q[k] = h2q[k] = T(0);
    }
  }
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const int e = rowW(k) * LW + cW;
    sm.w[e] = rw[k];
    sm.p[e] = rp[k];
    sm.q[e] = rq[k];
  }
#pragma unroll
  for (int k = 0; k < KC; ++k) sm.dc[rowC(k) * CXN + cC] = rc[k];
  __syncthreads();
  // weighted P/Q history (level n from the staged tile) and cell depths
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int r = rowB(k);
    const int t2 = (r + 1) * LW + cB + 1;             // same cell in the radius-2 tile
    sm.x.h.pt[r * BX + cB] = hist ? beta0 * sm.p[t2] + beta1 * h1p[k] + beta2 * h2p[k] : T(0);
    sm.x.h.qt[r * BX + cB] = hist ? beta0 * sm.q[t2] + beta1 * h1q[k] + beta2 * h2q[k] : T(0);
  }
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const int c0 = rowW(k) * CXN + cW;
    sm.db[rowW(k) * LW + cW] = dbar4(sm.dc[c0], sm.dc[c0 + 1], sm.dc[c0 + CXN], sm.dc[c0 + CXN + 1]);
  }

  __syncthreads();
  // F*, G* terms of this thread's cells (Eq. 14-15 are linear, so
  // sum_k beta_k F*^{n-k} = F*(sum_k beta_k Q^{n-k})), folded into the AB3
  // history terms of U*, V* (Eq. 43); after them the history tiles' LDS
  // holds the x-parts of the face pass
  {
    const T i2dx = D.i2dx, i2dy = D.i2dy, i4dxdy = D.i4dxdy, Bc = D.Bc;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int r = rY0 + q, c = cY;
      const int C0 = (r + 2) * LW + c + 2;
      const T d0 = dpos(sm.db[C0]);
      const T ddx = (dpos(sm.db[C0 + 1]) - dpos(sm.db[C0 - 1])) * i2dx;
      const T ddy = (dpos(sm.db[C0 + LW]) - dpos(sm.db[C0 - LW])) * i2dy;
      const int B0 = (r + 1) * BX + c + 1;
      const T qy = (sm.x.h.qt[B0 + BX] - sm.x.h.qt[B0 - BX]) * i2dy;
      const T qx = (sm.x.h.qt[B0 + 1] - sm.x.h.qt[B0 - 1]) * i2dx;
      const T qxy = ((sm.x.h.qt[B0 + BX + 1] - sm.x.h.qt[B0 - BX + 1]) -
                     (sm.x.h.qt[B0 + BX - 1] - sm.x.h.qt[B0 - BX - 1])) * i4dxdy;
      const T py = (sm.x.h.pt[B0 + BX] - sm.x.h.pt[B0 - BX]) * i2dy;
      const T px = (sm.x.h.pt[B0 + 1] - sm.x.h.pt[B0 - 1]) * i2dx;
      const T pxy = ((sm.x.h.pt[B0 + BX + 1] - sm.x.h.pt[B0 - BX + 1]) -
                     (sm.x.h.pt[B0 + BX - 1] - sm.x.h.pt[B0 - BX - 1])) * i4dxdy;
      hF[q] += d0 * ddx * qy * T(1.0 / 6.0) + d0 * ddy * qx * T(1.0 / 6.0) + Bc * d0 * d0 * qxy;
      hG[q] += d0 * ddx * py * T(1.0 / 6.0) + d0 * ddy * px * T(1.0 / 6.0) + Bc * d0 * d0 * pxy;
      pin(hE[q]);
      pin(hF[q]);
      pin(hG[q]);
    }
  }
  __syncthreads();
  const T g = D.g, eps = D.eps, ht = T(0.5) * D.theta;
  const T idx = D.idx, idy = D.idy;
  // ---- phase 1x: x-faces by row segments ----------------------------------
  // Thread (row rx, cells cx0 .. cx0+CPT-1) reconstructs cells cx0-1 ..
  // cx0+CPT once, takes the CPT+1 faces between them (the last one is also
  // its right neighbour's first) and writes the x-parts of its cells' E, F, G
  // (flux differences plus the x bed-slope source) to LDS.
  constexpr int SPR = TX / CPT;
  static_assert(SPR * TY == NT, "one x-segment per thread");
  {
    const int rx = tid / SPR, cx0 = (tid - rx * SPR) * CPT;
    const T* wr = sm.w + (rx + 2) * LW + cx0;         // tile column cx0 = cell cx0 - 2
    const T* pr = sm.p + (rx + 2) * LW + cx0;
    const T* qr = sm.q + (rx + 2) * LW + cx0;
    const T* c0 = sm.dc + (rx + 2) * CXN + cx0 + 1;   // corners of face cx0 - 1
    T Dfx[CPT + 3];                                   // still-water depth of face cx0 - 1 + k
#pragma unroll
    for (int k = 0; k < CPT + 3; ++k) Dfx[k] = T(0.5) * (c0[k] + c0[k + CXN]);
    // cell cx0 - 1 + k at its low (l) and high (h) faces
    T wl[CPT + 2], wh[CPT + 2], pl[CPT + 2], ph[CPT + 2], ql[CPT + 2], qh[CPT + 2];
    // limited (theta > 0) or central slopes: one uniform branch per tile
    auto recon = [&](auto lim) {
      constexpr bool LIM = decltype(lim)::value;
#pragma unroll
      for (int k = 0; k < CPT + 2; ++k) {
        recon_w<LIM>(wr[k], wr[k + 1], wr[k + 2], ht, Dfx[k], Dfx[k + 1], wl[k], wh[k]);
        const T sp = hslope<LIM>(pr[k], pr[k + 1], pr[k + 2], ht);
        const T sq = hslope<LIM>(qr[k], qr[k + 1], qr[k + 2], ht);
        pl[k] = pr[k + 1] - sp;
        ph[k] = pr[k + 1] + sp;
        ql[k] = qr[k + 1] - sq;
        qh[k] = qr[k + 1] + sq;
      }
    };
    if (ht > T(0)) recon(std::true_type{});
    else recon(std::false_type{});
    T f0w = T(0), fnw = T(0), ftw = T(0), dvw = T(0);  // west face of the cell being closed
#pragma unroll
    for (int m = 0; m <= CPT; ++m) {
      // face cx0 + m between cells cx0 + m - 1 (k = m) and cx0 + m (k = m + 1)
      const T Df = Dfx[m + 1];
      const Side<T> L = make_side(wh[m], ph[m], qh[m], Df, eps, g);
      const Side<T> R = make_side(wl[m + 1], pl[m + 1], ql[m + 1], Df, eps, g);
      T f0, fn, ft;
      cu_flux(L, R, g, Df, f0, fn, ft);
      if (m > 0) {
        // cell cx0 + m - 1: well-balanced bed source -g h b_x with h the mean
        // of its own face depths; with the still-water parts of the pressure
        // fluxes taken out only the face-depth departures remain
        const T Dw = Dfx[m], De = Dfx[m + 1];
        T bed = g * (De - Dw) * (T(0.5) * (L.dev + dvw));
        add_shore(bed, Dw, De, g);
        const int o = rx * AXP + cx0 + m - 1;
        sm.x.ax[0][o] = -(f0 - f0w) * idx;
        sm.x.ax[1][o] = (bed - (fn - fnw)) * idx;
        sm.x.ax[2][o] = -(ft - ftw) * idx;
      }
      f0w = f0;
      fnw = fn;
      ftw = ft;
      dvw = R.dev;
    }
  }
  // ---- phase 1y: y-faces by column segments, kept in registers ---------------
  // normal = Q, tangential = P; thread cells (rY0 + q, cY)
  T acc_e[CPT], acc_f[CPT], acc_g[CPT];
  {
    const T* wc = sm.w + rY0 * LW + cY + 2;           // tile row rY0 = row rY0 - 2
    const T* pc = sm.p + rY0 * LW + cY + 2;
    const T* qc = sm.q + rY0 * LW + cY + 2;
    const T* c0 = sm.dc + (rY0 + 1) * CXN + cY + 2;   // corners of face rY0 - 1
    T Dfy[CPT + 3];
#pragma unroll
    for (int k = 0; k < CPT + 3; ++k) Dfy[k] = T(0.5) * (c0[k * CXN] + c0[k * CXN + 1]);
    T wl[CPT + 2], wh[CPT + 2], pl[CPT + 2], ph[CPT + 2], ql[CPT + 2], qh[CPT + 2];
    auto recon = [&](auto lim) {
      constexpr bool LIM = decltype(lim)::value;
#pragma unroll
      for (int k = 0; k < CPT + 2; ++k) {
        recon_w<LIM>(wc[k * LW], wc[(k + 1) * LW], wc[(k + 2) * LW], ht, Dfy[k], Dfy[k + 1], wl[k], wh[k]);
        const T sp = hslope<LIM>(pc[k * LW], pc[(k + 1) * LW], pc[(k + 2) * LW], ht);
        const T sq = hslope<LIM>(qc[k * LW], qc[(k + 1) * LW], qc[(k + 2) * LW], ht);
        pl[k] = pc[(k + 1) * LW] - sp;
        ph[k] = pc[(k + 1) * LW] + sp;
        ql[k] = qc[(k + 1) * LW] - sq;
        qh[k] = qc[(k + 1) * LW] + sq;
      }
    };
    if (ht > T(0)) recon(std::true_type{});
    else recon(std::false_type{});
    T f0s = T(0), fns = T(0), fts = T(0), dvs = T(0);
#pragma unroll
    for (int m = 0; m <= CPT; ++m) {
      const T Df = Dfy[m + 1];
      const Side<T> Sd = make_side(wh[m], qh[m], ph[m], Df, eps, g);
      const Side<T> Nd = make_side(wl[m + 1], ql[m + 1], pl[m + 1], Df, eps, g);
      T f0, fn, ft;
      cu_flux(Sd, Nd, g, Df, f0, fn, ft);
      if (m > 0) {
        const T Ds = Dfy[m], Dn = Dfy[m + 1];
        T bed = g * (Dn - Ds) * (T(0.5) * (Sd.dev + dvs));
        add_shore(bed, Ds, Dn, g);
        acc_e[m - 1] = -(f0 - f0s) * idy;
        acc_f[m - 1] = -(ft - fts) * idy;              // x-momentum through y-faces
        acc_g[m - 1] = (bed - (fn - fns)) * idy;       // y-momentum
      }
      f0s = f0;
      fns = fn;
      fts = ft;
      dvs = Nd.dev;
    }
  }
  __syncthreads();

  // ---- phase 2: per-cell right-hand sides and AB3 update -------------------
  const T B = D.B, gn2 = D.gn2, cf = D.cf;
  const T a0 = (T)(CORR ? st->gamma[0] : st->alpha[0]);
  T* const wn = uni(CORR ? D.w[par ^ 1] : (D.corrector ? D.w[2] : D.w[par ^ 1]));
  const T* const wbase = uni((const T*)D.w[par]);   // w^n (the corrector's base)
  T* const E0 = uni(D.E[slot]);
  T* const F0 = uni(D.F[slot]);
  T* const G0 = uni(D.G[slot]);
  // The thread's cells are consecutive rows of one column, and the body is
  // branch-free, so the stencil reads and the eta / depth values they share
  // are formed once for all of them (cells outside the domain compute
  // harmless values and store nothing).
  const T i2dx = D.i2dx, i2dy = D.i2dy, idx2 = D.idx2, idy2 = D.idy2, i4dxdy = D.i4dxdy;
  const T i2dx3 = D.i2dx3, i2dy3 = D.i2dy3, i2dxdy2 = D.i2dxdy2, i2dx2dy = D.i2dx2dy;
  const T Bg = B * g;
  static_assert(S::AXP == TXP, "U*, V* alias the x-parts cell by cell");
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int r = rY0 + q, c = cY;
    const bool in = (i0 + c < nx) & (j0 + r < ny);
    const int C0 = (r + 2) * LW + c + 2;   // radius-2 tile index of the cell
    const int o = r * AXP + c;
    T e_ = sm.x.ax[0][o] + acc_e[q];
    T f_ = sm.x.ax[1][o] + acc_f[q];
    T g_ = sm.x.ax[2][o] + acc_g[q];
    const T Db = sm.db[C0];
    const T d0 = dpos(Db);
    const T dxm = dpos(sm.db[C0 - 1]), dxp = dpos(sm.db[C0 + 1]);
    const T dym = dpos(sm.db[C0 - LW]), dyp = dpos(sm.db[C0 + LW]);
    const T ddx = (dxp - dxm) * i2dx, ddy = (dyp - dym) * i2dy;
    // dispersive terms of Eq. (12)-(13): eta = h - d = w + min(D, 0); they
    // vanish with d0 on land
    {
#define ETA(o) (sm.w[C0 + (o)] + dneg(sm.db[C0 + (o)]))
      const T e00 = ETA(0);
      const T exm = ETA(-1), exp_ = ETA(1), eym = ETA(-LW), eyp = ETA(LW);
      const T emm = ETA(-LW - 1), epm = ETA(-LW + 1), emp = ETA(LW - 1), epp = ETA(LW + 1);
      const T exm2 = ETA(-2), exp2 = ETA(2), eym2 = ETA(-2 * LW), eyp2 = ETA(2 * LW);
#undef ETA
      const T exx = (exp_ - T(2) * e00 + exm) * idx2;
      const T eyy = (eyp - T(2) * e00 + eym) * idy2;
      const T exy = ((epp - epm) - (emp - emm)) * i4dxdy;
      const T exxx = ((exp2 - exm2) - T(2) * (exp_ - exm)) * i2dx3;
      const T eyyy = ((eyp2 - eym2) - T(2) * (eyp - eym)) * i2dy3;
      const T exyy = ((epp - T(2) * exp_ + epm) - (emp - T(2) * exm + emm)) * i2dxdy2;
      const T exxy = ((epp - T(2) * eyp + emp) - (epm - T(2) * eym + emm)) * i2dx2dy;
      const T bg = Bg * d0 * d0;
      f_ += bg * d0 * (exxx + exyy) + bg * (ddx * (T(2) * exx + eyy) + ddy * exy);
      g_ += bg * d0 * (eyyy + exxy) + bg * (ddy * (T(2) * eyy + exx) + ddx * exy);
    }
    // bottom friction f1, f2 at the cell centre: Manning g n^2 u |U| / h^(1/3)
    // plus the quadratic law f u |U|
    const T Pc = sm.p[C0], Qc = sm.q[C0];
    if (gn2 > T(0) || cf > T(0)) {
      const T h = fmax(sm.w[C0] + Db, T(0));
      const T vf = vfac(h, eps);
      const T u = Pc * vf, v = Qc * vf;
      const T k = h > T(0) ? (gn2 * frcbrt(h) + cf) * fsqrt(u * u + v * v) : T(0);
      f_ -= k * u;
      g_ -= k * v;
    }
    // Eq. (42)-(43)
    if (in) {
      const unsigned ii = oI + (unsigned)(q * ipitch);
      const unsigned og = oG + (unsigned)(q * pitch);
      if (!CORR) {
        stu(E0, ii, e_);
        stu(F0, ii, f_);
        stu(G0, ii, g_);
      }
      stu(wn, og, (CORR ? ldu(wbase, og) : sm.w[C0]) + (a0 * e_ + hE[q]));
    }
    // increments U*^{n+1} - U*^n, V*^{n+1} - V*^n (Eq. 43); the line solves
    // below act on them: P^{n+1} = P^n + T^-1 (U*^{n+1} - U*^n) since
    // U*^n = T P^n with the same matrix.  They overwrite this cell's own
    // x-parts (same word of the union), which no other thread reads, so no
    // barrier is needed between the two.
    sm.x.s.u[o] = in ? a0 * f_ + hF[q] : T(0);
    sm.x.s.v[o] = in ? a0 * g_ + hG[q] : T(0);
  }
  __syncthreads();

  // ---- phase 3: chunk-local solves of Eq. (19) (x) and Eq. (20) (y) -------
  constexpr int NCX = TX / MX;                  // x-chunks per tile row
  static_assert(TX % MX == 0, "chunks must tile the tile width");
  static_assert(TY * NCX <= 64, "x-chunk solvers must fit one wave");
  const bool wave_w = west_driven(D.bc[0]);
  if (tid < TY * NCX) {
    const int r = tid / NCX, qc = tid - r * NCX;
    const int j = j0 + r, is = i0 + qc * MX;
    if (j < ny && is < nx) {
      const int m = min(MX, nx - is);
      // depths of cells is-1 .. is+m (tile columns qc*MX+1 ..)
      const T* dlx = sm.db + (r + 2) * LW + qc * MX + 1;
      T* rhs = sm.x.s.u + r * TXP + qc * MX;
      if (is == 0 && wave_w) {
        // Dirichlet ghost: the increment of P_{-1} from t_n to t_{n+1}
        T a, b, c;
        tri_coef(dpos(dlx[0]), dpos(dlx[1]), dpos(dlx[2]), D.tcx, a, b, c);
        const T pg = CORR ? D.P[slot][(size_t)(j + 2) * pitch + xoff - 1] : sm.p[(r + 2) * LW + 1];
        rhs[0] -= a * ((T)st->gP[0] - pg);
      }
      chunk_solve_db<T, MX>(dlx, 1, m, D.tcx, is == 0 && !wave_w, is + m == nx, rhs, 1);
      const int cgl = is / MX;
      const gp<T> chx = gbl(D.chx);
      chx[(size_t)cgl * ny + j] = rhs[0];
      chx[((size_t)D.cx + cgl) * ny + j] = rhs[m - 1];
    }
  } else if (tid >= 64 && tid < 64 + TX) {
    const int c = tid - 64;
    const int i = i0 + c;
    if (i < nx && j0 < ny) {
      const int m = min(TY, ny - j0);
      const T* dly = sm.db + LW + c + 2;        // depths of rows j0-1 .. j0+m
      T* rhs = sm.x.s.v + c;
      chunk_solve_db<T, TY>(dly, LW, m, D.tcy, j0 == 0, j0 + m == ny, rhs, TXP);
      const int cgl = j0 / TY;
      const gp<T> chy = gbl(D.chy);
      chy[(size_t)cgl * nx + i] = rhs[0];
      chy[((size_t)D.cy + cgl) * nx + i] = rhs[(m - 1) * TXP];
    }
  }
  __syncthreads();
  // local solutions (cells outside the domain land in the fields' padding),
  // on the base P^n, Q^n
  T* const xhP = uni(D.xhP);
  T* const xhQ = uni(D.xhQ);
  const T* const Pb = uni((const T*)D.P[slot]);
  const T* const Qb = uni((const T*)D.Q[slot]);
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int r = rY0 + q;
    const int C0 = (r + 2) * LW + cY + 2;
    const unsigned ii = oI + (unsigned)(q * ipitch);
    const unsigned og = oG + (unsigned)(q * pitch);
    stu(xhP, ii, (CORR ? ldu(Pb, og) : sm.p[C0]) + sm.x.s.u[r * TXP + cY]);
    stu(xhQ, ii, (CORR ? ldu(Qb, og) : sm.q[C0]) + sm.x.s.v[r * TXP + cY]);
  }
}

// ---------------------------------------------------------------------------
// k_reduced: per line, couple the chunk-local solutions (one thread per line)
// ---------------------------------------------------------------------------
//
// For chunk c with local solution xh, left spike v and right spike w, the
// exact solution is x = xh + v * X_{e}(c-1) + w * X_{s}(c+1).  With
// sigma_c = x_first(c) and alpha_c = x_last(c) written as affine functions
// of x_first(c+1), a forward sweep gives
//   sigma_c = k1 xh_s + k2 alpha_{c-1},  alpha_c = xh_e + m1 alpha_{c-1} + m2 sigma_c
// and a backward sweep X_s(c) = sigma_c + tau_c X_s(c+1),
// X_e(c) = alpha_c + gamma_c X_s(c+1).  (k1, k2, m1, m2, tau, gamma) are
// static and precomputed.

template <typename T>
__device__ __forceinline__ void reduce_line(int C, int L, int line, const gp<const T> ch, const gp<const T> rs,
                                            const gp<T> itf) {
  // The recurrences are serial in c, their inputs are not: the inputs of
  // RB chunks are loaded together ahead of the RB dependent steps.
  constexpr int RB = 8;
  const size_t CL = (size_t)C * L;
  T al = T(0);
  for (int c0 = 0; c0 < C; c0 += RB) {
    T xs[RB], xe[RB], r0[RB], r1[RB], r2[RB], r3[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const size_t o = (size_t)min(c0 + k, C - 1) * L + line;
      xs[k] = ch[o];
      xe[k] = ch[CL + o];
      r0[k] = rs[o];
      r1[k] = rs[CL + o];
      r2[k] = rs[2 * CL + o];
      r3[k] = rs[3 * CL + o];
    }
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      if (c0 + k < C) {
        const size_t o = (size_t)(c0 + k) * L + line;
        const T sg = r0[k] * xs[k] + r1[k] * al;
        al = xe[k] + r2[k] * al + r3[k] * sg;
        itf[o] = sg;          // temporarily sigma_c, alpha_c
        itf[CL + o] = al;
      }
    }
  }
  T xs_next = T(0);
  for (int c1 = C - 1; c1 >= 0; c1 -= RB) {
    T sg[RB], a[RB], r4[RB], r5[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const size_t o = (size_t)max(c1 - k, 0) * L + line;
      sg[k] = itf[o];
      a[k] = itf[CL + o];
      r4[k] = rs[4 * CL + o];
      r5[k] = rs[5 * CL + o];
    }
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const int c = c1 - k;
      if (c >= 0) {
        const size_t o = (size_t)c * L + line;
        const T Xs = sg[k] + r4[k] * xs_next;
        const T Xe = a[k] + r5[k] * xs_next;
        itf[CL + o] = xs_next;                    // right neighbour of chunk c
        if (c + 1 < C) itf[o + L] = Xe;          // left neighbour of chunk c + 1
        xs_next = Xs;
      }
    }
  }
  itf[line] = T(0);                           // chunk 0 has no left neighbour
}

template <typename T>
__global__ void __launch_bounds__(256) k_reduced(const DomDev<T>* __restrict__ doms, const int* __restrict__ line_map,
                                                int nd, int lines, int pass) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= lines) return;
  int dom, l;
  locate(line_map, nd, gid, dom, l);
  const DomDev<T>& D = doms[dom];
  if (D.st->halt) return;
  if (pass == 1 && !D.corrector) return;      // the corrector pass
  if (l < D.ny) reduce_line<T>(D.cx, D.ny, l, gbl((const T*)D.chx), gbl((const T*)D.rsx), gbl(D.ifx));
  else reduce_line<T>(D.cy, D.nx, l - D.ny, gbl((const T*)D.chy), gbl((const T*)D.rsy), gbl(D.ify));
}

// The same recurrences with each line's chunks cut into NS segments (4 or 8),
// one wave per segment (a block holds 64 lines x NS segments).  Both sweeps are
// affine recurrences (alpha_c = A_c alpha_{c-1} + B_c forward, with
// A_c = m1 + m2 k2 and B_c = xh_e + m2 k1 xh_s; X_s(c) = tau_c X_s(c+1) +
// sigma_c backward), so each segment first composes its maps, the segments
// exchange them through LDS, and each then runs its part with the right
// incoming value: twice the arithmetic, 1/NS of the serial length.  The
// results equal the serial sweep's up to rounding (the composition
// reassociates the products).
template <typename T, int NS>
__device__ __forceinline__ void reduce_line_seg(int C, int L, int line, int seg, bool active, const gp<const T> ch,
                                                const gp<const T> rs, const gp<T> itf, T (*xa)[64], T (*xb)[64],
                                                int lane) {
  // the loads of RB chunks are issued together ahead of their serial steps
  constexpr int RB = 8;
  const size_t CL = (size_t)C * L;
  const int c0 = (int)(((long long)seg * C) / NS), c1 = (int)(((long long)(seg + 1) * C) / NS);
  const int n = active ? c1 - c0 : 0;
  // forward, pass 1: the segment's composite map alpha_out = A alpha_in + B
  T A = T(1), B = T(0);
  for (int b0 = 0; b0 < n; b0 += RB) {
    T k1[RB], k2[RB], m1[RB], m2[RB], xs[RB], xe[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const size_t o = (size_t)(c0 + min(b0 + k, n - 1)) * L + line;
      k1[k] = rs[o];
      k2[k] = rs[CL + o];
      m1[k] = rs[2 * CL + o];
      m2[k] = rs[3 * CL + o];
      xs[k] = ch[o];
      xe[k] = ch[CL + o];
    }
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (b0 + k < n) {
        const T Ac = m1[k] + m2[k] * k2[k], Bc = xe[k] + m2[k] * k1[k] * xs[k];
        A = Ac * A;
        B = Ac * B + Bc;
      }
  }
  xa[seg][lane] = A;
  xb[seg][lane] = B;
  __syncthreads();
  T al = T(0);
  for (int k = 0; k < seg; ++k) al = xa[k][lane] * al + xb[k][lane];
  __syncthreads();
  // forward, pass 2: sigma_c, alpha_c of the segment's chunks
  for (int b0 = 0; b0 < n; b0 += RB) {
    T r0[RB], r1[RB], r2[RB], r3[RB], xs[RB], xe[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const size_t o = (size_t)(c0 + min(b0 + k, n - 1)) * L + line;
      r0[k] = rs[o];
      r1[k] = rs[CL + o];
      r2[k] = rs[2 * CL + o];
      r3[k] = rs[3 * CL + o];
      xs[k] = ch[o];
      xe[k] = ch[CL + o];
    }
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (b0 + k < n) {
        const size_t o = (size_t)(c0 + b0 + k) * L + line;
        const T sg = r0[k] * xs[k] + r1[k] * al;
        al = xe[k] + r2[k] * al + r3[k] * sg;
        itf[o] = sg;
        itf[CL + o] = al;
      }
  }
  // backward, pass 1: X_s(c0) = R X_s(c1) + S over the segment
  T R = T(1), Sv = T(0);
  for (int b1 = 0; b1 < n; b1 += RB) {
    T tau[RB], sg[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const size_t o = (size_t)(c1 - 1 - min(b1 + k, n - 1)) * L + line;
      tau[k] = rs[4 * CL + o];
      sg[k] = itf[o];
    }
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (b1 + k < n) {
        R = tau[k] * R;
        Sv = tau[k] * Sv + sg[k];
      }
  }
  xa[seg][lane] = R;
  xb[seg][lane] = Sv;
  __syncthreads();
  T xs_next = T(0);
  for (int k = NS - 1; k > seg; --k) xs_next = xa[k][lane] * xs_next + xb[k][lane];
  // backward, pass 2; the left-neighbour value of the next segment's first
  // chunk is written after the barrier (that segment reads the slot first)
  T held = T(0);
  bool hold = false;
  for (int b1 = 0; b1 < n; b1 += RB) {
    T sg[RB], a[RB], r4[RB], r5[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const size_t o = (size_t)(c1 - 1 - min(b1 + k, n - 1)) * L + line;
      sg[k] = itf[o];
      a[k] = itf[CL + o];
      r4[k] = rs[4 * CL + o];
      r5[k] = rs[5 * CL + o];
    }
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (b1 + k < n) {
        const int c = c1 - 1 - (b1 + k);
        const size_t o = (size_t)c * L + line;
        const T Xs = sg[k] + r4[k] * xs_next;
        const T Xe = a[k] + r5[k] * xs_next;
        itf[CL + o] = xs_next;                    // right neighbour of chunk c
        if (c + 1 < C) {
          if (c == c1 - 1) {
            held = Xe;
            hold = true;
          } else {
            itf[o + L] = Xe;                      // left neighbour of chunk c + 1
          }
        }
        xs_next = Xs;
      }
  }
  __syncthreads();
  if (hold) itf[(size_t)c1 * L + line] = held;
  if (active && seg == 0) itf[line] = T(0);       // chunk 0 has no left neighbour
}

template <typename T, int NS>
__global__ void __launch_bounds__(64 * NS) k_reduced_seg(const DomDev<T>* __restrict__ doms,
                                                        const int* __restrict__ line_map, int nd, int lines,
                                                        int pass) {
  __shared__ T xa[NS][64], xb[NS][64];
  const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6;
  const int gid = blockIdx.x * 64 + lane;
  // every thread reaches the barriers; inactive ones carry identity maps
  bool active = gid < lines;
  int dom = 0, l = 0;
  if (active) {
    locate(line_map, nd, gid, dom, l);
    const DomDev<T>& D = doms[dom];
    active = !D.st->halt && !(pass == 1 && !D.corrector);
  }
  // one call site: the barriers inside must be met by every wave once, and
  // the lanes of a wave may hold x-lines and y-lines
  const DomDev<T>& D = doms[dom];
  const bool xl = l < D.ny;
  reduce_line_seg<T, NS>(xl ? D.cx : D.cy, xl ? D.ny : D.nx, xl ? l : l - D.ny, seg, active,
                     gbl((const T*)(xl ? D.chx : D.chy)), gbl((const T*)(xl ? D.rsx : D.rsy)),
                     gbl(xl ? D.ifx : D.ify), xa, xb, lane);
}

// ---------------------------------------------------------------------------
// k_final: spike corrections, sponge, ghost cells, CFL maximum
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void put3(const DomDev<T>& D, T* w, T* P, T* Q, int i, int j, T vw, T vp, T vq) {
  const size_t g = (size_t)(j + 2) * D.pitch + D.xoff + i;
  gbl(w)[g] = vw;
  gbl(P)[g] = vp;
  gbl(Q)[g] = vq;
}

// ghost cells written by interior cell (i, j) of the new state: x sides for
// interior rows (wall mirror or wavemaker values), then y sides for all
// columns (the corners mirror the x ghosts)
template <typename T>
__device__ void ghost_cell(const DomDev<T>& D, T* w, T* P, T* Q, int i, int j, T wv, T p, T qv, const double* gw,
                           const double* gP) {
  const int nx = D.nx, ny = D.ny;
  const bool yg = j < 2 || j >= ny - 2;
  T gwv = wv, gpv = p, gqv = qv;
  int gi = 0;
  bool have_x = false;
  if (i < 2) {
    gi = -1 - i;
    have_x = true;
    if (west_driven(D.bc[0])) {
      gwv = (T)gw[i];
      gpv = (T)gP[i];
      gqv = T(0);
    } else {
      gpv = -p;
    }
    put3(D, w, P, Q, gi, j, gwv, gpv, gqv);
  } else if (i >= nx - 2) {
    gi = 2 * nx - 1 - i;
    have_x = true;
    gpv = -p;
    put3(D, w, P, Q, gi, j, gwv, gpv, gqv);
  }
  if (yg) {
    const int gj = j < 2 ? -1 - j : 2 * ny - 1 - j;
    put3(D, w, P, Q, i, gj, wv, p, -qv);
    if (have_x) put3(D, w, P, Q, gi, gj, gwv, gpv, -gqv);
  }
}

template <typename T, int TY, int MX>
struct alignas(16) FinSmem {
  static constexpr int CXN = TX + 3, CYN = TY + 3;    // corners of cells i0-1 .. i0+TX, j0-1 .. j0+TY
  static constexpr int BX = TX + 2, BY = TY + 2;      // cells with one neighbour on each side
  static constexpr int TXP = TX + 1;
  T db[BY * BX];                                      // cell still-water depth
  union {
    T dc[CYN * CXN];                                  // corners (until db is formed)
    struct {
      T cx[TY * TXP];                                 // x-line correction of P
      T cy[TY * TXP];                                 // y-line correction of Q
      T ux[TY * TXP];                                 // c_k / u_k of the x solves
      T uy[TY * TXP];                                 // and of the y solves
    } s;
  } u;
};

// MODE 0: finalizes the AB3 step in a launch where no domain runs the
// corrector.  MODE 1: the same where some do; for those it finalizes the
// predicted level (surface in w[2], no sponge, no run-up record).  MODE 2:
// finalizes the corrector of the domains that run it.
template <typename T, int TY, int MX, int MODE>
__global__ void __launch_bounds__(NT) k_final(const DomDev<T>* __restrict__ doms, const int* __restrict__ tile_map,
                                             int nd, int swizzle) {
  using S = FinSmem<T, TY, MX>;
  constexpr int CXN = S::CXN, BX = S::BX, TXP = S::TXP;
  constexpr int CPT = (TX * TY) / NT;
  __shared__ S sm;
  int dom, tile;
  // swizzle = 1: XCD-aware tile order, as in the stencil kernel (the corner
  // halo of a tile is then mostly in its XCD's L2)
  locate(tile_map, nd, swizzle ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x, dom, tile);
  const DomDev<T>& D = doms[dom];
  DevState* st = D.st;
  if (st->halt) return;
  if (MODE == 2 && !D.corrector) return;
  const bool pred = MODE == 1 && D.corrector;          // the predictor's level
  const int i0 = (tile % D.tiles_x) * TX, j0 = (tile / D.tiles_x) * TY;
  const int nx = D.nx, ny = D.ny, tid = threadIdx.x;
  const int ns = uni(st->slot == 2 ? 0 : st->slot + 1);   // slot of level n + 1
  const int par = uni((int)((st->n + 1) & 1));
  T* const w = uni(pred ? D.w[2] : D.w[par]);
  T* const P = uni(D.P[ns]);
  T* const Q = uni(D.Q[ns]);
  const int pitch = uni(D.pitch), xoff = uni(D.xoff), ipitch = uni(D.ipitch), cpitch = uni(D.cpitch);
  const T g = D.g, eps = D.eps, idx = D.idx, idy = D.idy;
  // cells of a thread: column cY, rows rY0 .. rY0+CPT-1 (as in the stencil kernel)
  const int cY = tid % TX, rY0 = (tid / TX) * CPT;
  const unsigned oI = (unsigned)((j0 + rY0) * ipitch + i0 + cY);
  const unsigned oG = (unsigned)((j0 + rY0 + 2) * pitch + xoff + i0 + cY);
  // all loads first: the neighbour-chunk end values of this thread's line
  // solve (if it has one), the corners of the tile's cells and their
  // neighbours (rows read in groups, no clamping: the fields are padded to
  // whole tiles), the local solutions and the new surface
  constexpr int NCX = TX / MX;
  T xl = T(0), xr = T(0);
  if (tid < TY * NCX) {
    const int r = tid / NCX, qc = tid - r * NCX;
    const int j = min(j0 + r, ny - 1), is = min(i0 + qc * MX, nx - 1);
    const size_t o = (size_t)(is / MX) * ny + j;
    xl = D.ifx[o];
    xr = D.ifx[(size_t)D.cx * ny + o];
  } else if (tid >= 64 && tid < 64 + TX) {
    const int i = min(i0 + tid - 64, nx - 1);
    const size_t o = (size_t)(j0 / TY) * nx + i;
    xl = D.ify[o];
    xr = D.ify[(size_t)D.cy * nx + o];
  }
  constexpr int RGC = NT / CXN, KC = (S::CYN + RGC - 1) / RGC;
  const int rC = min(tid / CXN, RGC - 1), cC = tid - (tid / CXN) * CXN;
  auto rowC = [&](int k) { return k < KC - 1 ? rC + RGC * k : min(rC + RGC * k, S::CYN - 1); };
  T rc[KC];
  {
    const T* Dc = uni((const T*)D.Dc);
    const unsigned oC = (unsigned)((j0 + 1) * cpitch + i0 + 1 + cC);   // corner (i0-1+cC, j0-1)
#pragma unroll
    for (int k = 0; k < KC; ++k) rc[k] = ldu(Dc, oC + (unsigned)(rowC(k) * cpitch));
  }
  T lp[CPT], lq[CPT], lw[CPT];
  {
    const T* xhP = uni((const T*)D.xhP);
    const T* xhQ = uni((const T*)D.xhQ);
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      lp[q] = ldu(xhP, oI + (unsigned)(q * ipitch));
      lq[q] = ldu(xhQ, oI + (unsigned)(q * ipitch));
      lw[q] = ldu((const T*)w, oG + (unsigned)(q * pitch));
    }
  }
#pragma unroll
  for (int k = 0; k < KC; ++k) sm.u.dc[rowC(k) * CXN + cC] = rc[k];
  __syncthreads();
  for (int e = tid; e < S::BY * BX; e += NT) {
    const int r = e / BX, c = e - r * BX;
    sm.db[e] = dbar4(sm.u.dc[r * CXN + c], sm.u.dc[r * CXN + c + 1], sm.u.dc[(r + 1) * CXN + c],
                     sm.u.dc[(r + 1) * CXN + c + 1]);
  }
  __syncthreads();
  // Exact line solution = local solution + the response of the chunk system
  // to its coupling with the neighbour chunks' end values (from the
  // line-coupling kernel): a right-hand side that is zero except -a x_left
  // in the first row and -c x_right in the last.  The response is solved
  // here from the static matrix instead of read as stored spikes.
  const bool wave_w = west_driven(D.bc[0]);
  if (tid < TY * NCX) {
    const int r = tid / NCX, qc = tid - r * NCX;
    const int j = j0 + r, is = i0 + qc * MX;
    if (j < ny && is < nx) {
      const int m = min(MX, nx - is);
      const T* dlx = sm.db + (r + 1) * BX + qc * MX;   // cells is-1 .. is+m
      T a, b, c0, cm;
      tri_coef(dpos(dlx[0]), dpos(dlx[1]), dpos(dlx[2]), D.tcx, a, b, c0);
      const T r0 = -a * xl;
      tri_coef(dpos(dlx[m - 1]), dpos(dlx[m]), dpos(dlx[m + 1]), D.tcx, a, b, cm);
      chunk_edge_solve<T>(dlx, 1, m, D.tcx, is == 0 && !wave_w, is + m == nx, r0, -cm * xr,
                          sm.u.s.cx + r * TXP + qc * MX, sm.u.s.ux + r * TXP + qc * MX, 1);
    }
  } else if (tid >= 64 && tid < 64 + TX) {
    const int c = tid - 64;
    const int i = i0 + c;
    if (i < nx && j0 < ny) {
      const int m = min(TY, ny - j0);
      const T* dly = sm.db + c + 1;                    // rows j0-1 .. j0+m
      T a, b, c0, cm;
      tri_coef(dpos(dly[0]), dpos(dly[BX]), dpos(dly[2 * BX]), D.tcy, a, b, c0);
      const T r0 = -a * xl;
      tri_coef(dpos(dly[(m - 1) * BX]), dpos(dly[m * BX]), dpos(dly[(m + 1) * BX]), D.tcy, a, b, cm);
      chunk_edge_solve<T>(dly, BX, m, D.tcy, j0 == 0, j0 + m == ny, r0, -cm * xr, sm.u.s.cy + c, sm.u.s.uy + c,
                          TXP);
    }
  }
  __syncthreads();
  // new state, sponge, CFL speeds (Eq. 22) and ghost cells
  const double dt = st->dt;
  T smax = T(0);
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int r = rY0 + q, i = i0 + cY, j = j0 + r;
    T p = lp[q] + sm.u.s.cx[r * TXP + cY];
    T qv = lq[q] + sm.u.s.cy[r * TXP + cY];
    T wv = lw[q];
    const T Db = sm.db[(r + 1) * BX + cY + 1];
    if (i >= nx || j >= ny) continue;
    const unsigned og = oG + (unsigned)(q * pitch);
    if (D.any_sponge && !pred && Db > T(0)) {
      const T dist[4] = {(T(i) + T(0.5)) * D.dx, (T(nx - i) - T(0.5)) * D.dx, (T(j) + T(0.5)) * D.dy,
                         (T(ny - j) - T(0.5)) * D.dy};
      T sig = T(0);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const T Ls = D.sponge_w[s];
        if (D.bc[s] == SPONGE && Ls > T(0) && dist[s] < Ls) {
          const T z = (Ls - dist[s]) / Ls;
          sig += D.sponge_sigma * z * z;
        }
      }
      if (sig > T(0)) {
        const T fac = exp(-sig * (T)dt);
        wv *= fac;
        p *= fac;
        qv *= fac;
        stu(w, og, wv);
      }
    }
    stu(P, og, p);
    stu(Q, og, qv);
    const T h = fmax(wv + Db, T(0));
    if (D.runup && !pred && h > D.runup_delta) {
      // run-up record: highest surface over the inundated states (NaN until
      // the first one)
      const gp<T> wm = gbl(D.wmax);
      const unsigned oi = oI + (unsigned)(q * ipitch);
      if (!(wm[oi] >= wv)) wm[oi] = wv;
    }
    const T vf = vfac(h, eps);
    const T u = p * vf, v = qv * vf;
    const T cel = fsqrt(g * h);
    const T sx = (fabs(u) + cel) * idx, sy = (fabs(v) + cel) * idy;
    // a NaN in either direction must reach the maximum as +inf
    const T sd = (sx != sx || sy != sy) ? T(INFINITY) : fmax(sx, sy);
    smax = fmax(smax, sd);
    if (i < 2 || i >= nx - 2 || j < 2 || j >= ny - 2) ghost_cell(D, w, P, Q, i, j, wv, p, qv, st->gw, st->gP);
  }
  // block max -> one word per tile (max commutes with the widening to FP64,
  // so the FP32 maximum converts to the same value); no atomics, so a large
  // domain's blocks do not serialise on one address
  __shared__ T red[NT / 64];
  for (int o = 32; o > 0; o >>= 1) smax = fmax(smax, __shfl_xor(smax, o, 64));
  if ((tid & 63) == 0) red[tid >> 6] = smax;
  __syncthreads();
  if (tid == 0) {
    T m = red[0];
    for (int k = 1; k < NT / 64; ++k) m = fmax(m, red[k]);
    gbl(D.smax_tile)[tile] = (double)m;               // reduced by the next step's k_dt
  }
}

}  // namespace bqk
