/*
 * bqo.h -- CPU oracle for the adaptive-AB3 extended-Boussinesq time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This header and bqo.c form a plain, slow,
 * single-threaded FP64 reference of the method of Tavakkol, Son & Lynett,
 * "Adaptive third order Adams-Bashforth time stepping for extended Boussinesq
 * equations" (arXiv 1909.04153).  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library under paper_1909_04153_amd/.
 *
 * Conventions (paper Sec. 2): b = bottom elevation, w_s = 0 still-water level,
 * d = max(w_s - b, 0) still-water depth, w = h + b water-surface elevation,
 * eta = h - d, (P, Q) depth-integrated fluxes.  Grid: nx x ny cells of size
 * dx x dy, cell (i, j) centred at ((i + 1/2) dx, (j + 1/2) dy); two ghost
 * layers per side (Sec. 3.3).  Bathymetry is given as still-water depth at
 * the (nx + 1) x (ny + 1) cell corners, row-major (j * (nx + 1) + i), so
 * b_corner = -depth_c.
 *
 * Parity status of each part is listed in the header comment of bqo.c.
 */
#ifndef BQO_H
#define BQO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { BQO_WALL = 0, BQO_SINE = 1, BQO_SPONGE = 2, BQO_IRREGULAR = 3, BQO_TIMESERIES = 4 };
enum { BQO_W = 0, BQO_E = 1, BQO_S = 2, BQO_N = 3 };
enum {
  BQO_OK = 0,
  BQO_EINVAL = -1,
  BQO_ENONFINITE = -4,
  BQO_EDTMIN = -5,
  BQO_EDONE = -7
};

typedef struct {
  int32_t nx, ny;
  double dx, dy;
  double g;          /* gravitational acceleration */
  double B;          /* dispersion calibration coefficient (Sec. 2: 1/15) */
  double manning_n;  /* Manning coefficient of the friction terms f1, f2 */
  double cfl;        /* target CFL number of Eq. (22) */
  double ema_alpha;  /* coefficient of the lazy moving average, Eq. (47) */
  double dt_init;    /* first step; 0 = from the CFL number */
  double dt_max, dt_min;
  int32_t fixed_dt;  /* 1 = every step uses dt_init */
  double theta;      /* generalised minmod parameter of the KP07 reconstruction
                        (1..2); 0 = unlimited central slopes */
  double eps_desing; /* desingularisation epsilon; 0 = max(dx^4, dy^4) */
  int32_t bc[4];     /* W, E, S, N */
  double sponge_width[4];
  double sponge_sigma;
  int32_t n_waves;   /* wavemaker components (SINE: 1) */
  const double* wave_amp;
  const double* wave_omega;
  const double* wave_phase;
  double wave_ramp;  /* tau of the start-up ramp 1 - exp(-(t/tau)^2); 0 = none */
  double t_end;      /* stop (status BQO_EDONE) once t >= t_end; 0 = never */
  int32_t fstar_order; /* time extrapolation of F*, G*: 2 = quadratic (Eq. 43-46),
                          1 = linear (two-point backward difference for every
                          derivative estimate); 0 selects 2 */
  double friction_f; /* quadratic friction factor: f1 = f u |U|, f2 = f v |U|
                        (Sec. 5.3-5.4 use 0.0025); adds to the Manning term */
  int32_t ts_n;      /* time-series boundary (BQO_TIMESERIES, west side):
                        samples of eta and P at t = k ts_dt, k = 0 .. ts_n-1 */
  double ts_dt;
  const double* ts_eta;
  const double* ts_P;
  double runup_delta; /* > 0: keep the run-up record, the highest w of every
                         cell over the states whose depth exceeded it (Sec. 5.1
                         uses s dx / 3) */
  int32_t corrector; /* 1 = each AB3 step (the predictor) is followed by an
                        Adams-Moulton corrector (Celeris' optional corrector,
                        Sec. 1), in variable-step form */
} bqo_params;

typedef struct bqo_domain bqo_domain;

typedef struct {
  double t;
  int64_t n;
  double dt_last;    /* dt of the step that produced the current state */
  double dt_prev1;   /* the one before */
  double dt_prev2;
  double smax;       /* max characteristic speed / cell size of the current state */
  double mass;
  double energy;
  int32_t status;
} bqo_info;

bqo_domain* bqo_create(const bqo_params* p, const double* depth_c);
void bqo_free(bqo_domain* d);
int bqo_set_state(bqo_domain* d, const double* eta, const double* P, const double* Q);
int bqo_step(bqo_domain* d, int32_t n_steps);
int bqo_step_dt(bqo_domain* d, double dt);
int bqo_info_get(bqo_domain* d, bqo_info* out);
/* which: 0 eta, 1 P, 2 Q, 3 w, 4 run-up record (NaN where the depth never
 * exceeded runup_delta; EINVAL unless it is kept), 5 local CFL number of
 * Eq. (22), dt_last * max((|u|+c)/dx, (|v|+c)/dy); interior nx*ny, row-major */
int bqo_read(bqo_domain* d, int32_t which, double* out);
/* spatial operator at the current state: E, F, G (Eq. 11-13), interior */
int bqo_rhs(bqo_domain* d, double* E, double* F, double* G);
/* operators of the current state, interior: which 0 U*^n (Eq. 9 as the row
 * of Eq. 19 with the coefficients of Eq. 21), 1 V*^n (Eq. 10 / 20),
 * 2 F*(Q^n) (Eq. 14), 3 G*(P^n) (Eq. 15) */
int bqo_operator(bqo_domain* d, int32_t which, double* out);
/* PLANTED MISTAKE for the pin tests only: multiply the depth gradient
 * d_x, d_y wherever it enters (Eq. 12-15 and the dd/(6 dalpha) terms of
 * Eq. 21) by `scale`; 1 restores the method */
int bqo_plant_depth_gradient_scale(bqo_domain* d, double scale);
/* west ghost values at time t (wavemaker or time series): out = eta and P
 * of ghost cell -1, then of ghost cell -2 */
int bqo_west_ghosts(bqo_domain* d, double t, double out[4]);
/* wave-number of the wavemaker components (Madsen-Sorensen relation) */
int bqo_wave_numbers(bqo_domain* d, double* k_out);

/* building blocks exposed for the pin tests */
void bqo_ab3_alpha(double h0, double h1, double h2, double alpha[3]);
/* corrector weights of (E, F, G) at t_{n+1}, t_n, t_{n-1}, t_{n-2}: fourth
 * order for n >= 2, third at n = 1, trapezoidal at n = 0 (unused ones 0) */
void bqo_am_weights(int64_t n, double h0, double h1, double h2, double gamma[4]);
void bqo_fd_weights(double h1, double h2, double D[9]);
void bqo_step_weights(int64_t n, int32_t fstar_order, double h0, double h1, double h2, double alpha[3], double D[9]);
double bqo_lazy_ema(double cand, double prev, double a);
void bqo_thomas(int32_t n, const double* a, const double* b, const double* c, const double* r, double* x);
/* Line solve of Eq. (19)-(21) used by the step: Thomas plus one step of
 * iterative refinement with the residual in extended precision. */
void bqo_solve_line(int32_t n, const double* a, const double* b, const double* c, const double* r, double* x);
double bqo_minmod(double a, double b, double c);
double bqo_ms_wavenumber(double omega, double depth, double g, double B);
/* single x-face KP07 flux between a left cell (wL, PL, QL) and a right cell
 * with piecewise-constant states and face bed bf: H[3] */
void bqo_face_flux_const(double g, double eps, double bf,
                         double wL, double PL, double QL,
                         double wR, double PR, double QR, double H[3]);

#ifdef __cplusplus
}
#endif
#endif
