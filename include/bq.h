/*
 * bq.h -- C ABI of libbq, an MI355X (gfx950) HIP implementation of one time
 * step of the extended Boussinesq solver of Tavakkol, Son & Lynett,
 * "Adaptive third order Adams-Bashforth time stepping for extended
 * Boussinesq equations" (arXiv 1909.04153).
 *
 * The step (all of it runs in HIP kernels, enqueued on the caller's stream):
 *   - ghost cells, two layers per side (Sec. 3.3): solid wall, sine
 *     wavemaker, sponge layer, irregular wavemaker, time series;
 *   - KP07 central-upwind finite volumes for the NLSW subset with a
 *     well-balanced bed source, central differences for the dispersive terms
 *     and bottom friction (Manning, and the quadratic law of the paper's
 *     experiments, Sec. 5.3-5.4): E, F, G of Eq. (11)-(13) (Sec. 3.1);
 *   - Delta t from the CFL number of Eq. (22) on the current state, passed
 *     through the lazy moving average of Eq. (47) (Sec. 3.2.2, 3.2.2.4);
 *   - the variable-step AB3 update of w, U*, V*: Eq. (42)-(43) with the
 *     variable-step finite differences of Eq. (44)-(46) for the time
 *     derivatives of F*, G* (Eq. 14-15), forward Euler for the first two
 *     steps (Sec. 3.2.1);
 *   - the tridiagonal systems of Eq. (19)-(21) for P and Q;
 *   - optionally (bq_params.corrector) an Adams-Moulton corrector after each
 *     AB3 step, the corrector Celeris offered (Sec. 1), in variable-step form:
 *     E, F, G of the predicted level enter the integral over [t_n, t_{n+1}]
 *     of the cubic through t_{n+1}, t_n, t_{n-1}, t_{n-2} (built like
 *     Eq. 30), and F*, G* their change from level n to the predicted level.
 *
 * Conventions.  Grid nx x ny cells of dx x dy; cell (i, j) is centred at
 * ((i + 1/2) dx, (j + 1/2) dy); host arrays are row-major with index
 * j * nx + i.  Bathymetry is the still-water depth at the (nx+1) x (ny+1)
 * cell corners (positive under water, negative on land), so the bottom
 * elevation is b = -depth and the still-water level is 0 (Sec. 2:
 * d = max(-b, 0), w = h + b, eta = h - d).
 *
 * Ownership.  The caller owns the device workspace passed to
 * bq_domain_create (for instance a torch uint8 tensor on the GPU) and must
 * keep it alive until bq_domain_free.  The library allocates nothing on the
 * device for a domain beyond that workspace; a batch allocates its own small
 * descriptor tables (bq_batch_set_static takes a static array instead) and
 * creates the streams and events of its lanes.  Host
 * pointers passed in are only read during the call.
 *
 * Errors.  Every call returns 0 (BQ_OK) or a negative bq_status; nothing
 * throws across the ABI.  bq_last_error() returns a message for the calling
 * thread's last failure.  Numerical failures inside a step (non-finite
 * state, Delta t below dt_min) are latched on the device per domain and
 * reported by bq_sync; a latched domain stops advancing.  A domain (or a
 * batch) must be driven by one host thread at a time.
 */
#ifndef BQ_H
#define BQ_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BQ_ABI_VERSION 6
#define BQ_MAX_WAVES 256
/* Size of the per-GPU static array that holds the device tables of a batch
 * set up by bq_batch_set_static (8 MiB: the tables take 4 bytes per tile of
 * 64 x 16 (FP32) or 64 x 8 (FP64) cells and per grid line, plus about 1 KB
 * per member, twice over with lanes). */
#define BQ_STATIC_TABLE_BYTES (8u << 20)

/* BQ_TIMESERIES: both west ghost columns take eta and P interpolated
 * linearly in time from the samples ts_eta, ts_P (held at the first / last
 * sample outside their span), times the start-up ramp; Q = 0 there. */
typedef enum { BQ_WALL = 0, BQ_SINE = 1, BQ_SPONGE = 2, BQ_IRREGULAR = 3, BQ_TIMESERIES = 4 } bq_bc;
typedef enum { BQ_SIDE_W = 0, BQ_SIDE_E = 1, BQ_SIDE_S = 2, BQ_SIDE_N = 3 } bq_side;
typedef enum { BQ_FP64 = 0, BQ_FP32 = 1 } bq_precision;
typedef enum {
  BQ_OK = 0,
  BQ_EINVAL = -1,      /* bad argument */
  BQ_ENOMEM = -2,      /* workspace smaller than bq_workspace_bytes */
  BQ_EDEVICE = -3,     /* HIP runtime error */
  BQ_ENONFINITE = -4,  /* NaN/Inf met by the CFL reduction (latched) */
  BQ_EDTMIN = -5,      /* adaptive Delta t fell below dt_min (latched) */
  BQ_ESTATE = -6,      /* call not valid in the current state */
  BQ_EDONE = -7        /* t reached t_end; the domain no longer advances */
} bq_status;

/* Parameters of one domain.  Field order is part of the ABI. */
typedef struct bq_params {
  int32_t nx, ny;          /* interior cells, each >= 4 */
  double dx, dy;           /* cell size [m] */
  double g;                /* gravitational acceleration [m/s^2] */
  double B;                /* dispersion coefficient of Eq. (2)-(3), 1/15 */
  double manning_n;        /* Manning coefficient of f1, f2 [s/m^(1/3)] */
  double cfl;              /* target CFL number of Eq. (22) */
  double ema_alpha;        /* alpha of the lazy moving average, Eq. (47) */
  double dt_init;          /* first Delta t; 0 = from the CFL number */
  double dt_max, dt_min;   /* clamp / failure threshold of the adaptive step */
  int32_t fixed_dt;        /* 1 = every step uses dt_init (uniform AB3, Eq. 16-18) */
  double theta;            /* generalised-minmod parameter in [1, 2]; 0 = central slopes */
  double eps_desing;       /* velocity desingularisation epsilon; 0 = max(dx^4, dy^4) */
  int32_t bc[4];           /* bq_bc per side W, E, S, N; wavemakers and time
                              series on W only */
  double sponge_width[4];  /* sponge band width per side [m] (BQ_SPONGE sides) */
  double sponge_sigma;     /* peak damping rate of the sponge [1/s] */
  int32_t n_waves;         /* wavemaker components (<= BQ_MAX_WAVES) */
  const double* wave_amp;  /* host arrays of n_waves: amplitude [m], */
  const double* wave_omega;/*   angular frequency [rad/s], */
  const double* wave_phase;/*   phase [rad] (may be NULL = 0) */
  double wave_ramp;        /* tau of the start-up ramp 1 - exp(-(t/tau)^2); 0 = none */
  double t_end;            /* stop once t >= t_end (status BQ_EDONE); 0 = never */
  int32_t fstar_order;     /* extrapolation of F*, G* in time: 2 = quadratic
                              (Eq. 43-46), 1 = linear (stable reading for 2D
                              dispersive cases); 0 selects 2 */
  int32_t precision;       /* bq_precision of the field arithmetic; Delta t,
                              the AB3/FD weights, time and mass/energy sums are
                              FP64 in both */
  /* fields added in ABI version 2 */
  double friction_f;       /* quadratic friction factor: f1 = f u |U|,
                              f2 = f v |U| (Sec. 5.3-5.4: 0.0025); added to
                              the Manning term; 0 = none */
  int32_t ts_n;            /* BQ_TIMESERIES: samples at t = k ts_dt, k < ts_n */
  double ts_dt;            /*   sample spacing [s] */
  const double* ts_eta;    /*   host arrays of ts_n: surface elevation [m] */
  const double* ts_P;      /*   and x-flux [m^2/s] at the west boundary */
  double runup_delta;      /* > 0: keep the run-up record (bq_read which 4):
                              per cell the highest w over the states whose
                              depth exceeded runup_delta (Sec. 5.1: s dx / 3);
                              0 = not kept */
  /* field added in ABI version 3 */
  int32_t corrector;       /* 1 = AB3 predictor + Adams-Moulton corrector
                              (two passes of the spatial operator and the
                              line solves per step; fourth order in time
                              where F* = G* = 0); 0 = AB3 only */
} bq_params;

typedef struct bq_info {
  double t;                /* simulated time of the current state */
  int64_t n;               /* steps taken since bq_set_state */
  double dt_last;          /* Delta t of the last step */
  double dt_prev1, dt_prev2;
  double smax;             /* max((|u|+c)/dx, (|v|+c)/dy) of the current state */
  double mass;             /* sum of h dx dy (FP64) */
  double energy;           /* sum of (g eta^2 / 2 [d > 0] + (P^2 + Q^2) / 2h [h > 1e-6]) dx dy */
  int32_t status;          /* latched bq_status of the domain */
} bq_info;

typedef struct bq_domain bq_domain;
typedef struct bq_batch bq_batch;

int bq_abi_version(void);
const char* bq_last_error(void);

/* A plain device-to-device copy of `bytes` (a multiple of 16, both buffers
 * 16-byte aligned), one 16-byte vector per lane, enqueued on hip_stream: the
 * achievable HBM bandwidth that the step's kernels are measured against
 * (read + write bytes over its duration). */
int bq_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

/* Streams, events and graph executables the library has created and not yet
 * destroyed, in counts[0..2] (all domains and batches of the process).  For
 * tests that freeing a batch or a domain releases what it made. */
int bq_live_handles(int32_t* counts);

/* Defaults: g 9.81, B 1/15, cfl 0.2, ema_alpha 0.1, dt_max 1, dt_min 1e-9,
 * theta 1.3, walls, fstar_order 2, FP64. */
void bq_params_default(bq_params* p);

/* Device bytes a domain with these parameters needs (pure host function).
 * BQ_EINVAL for a domain of more than 2e9 cells, or one whose largest field,
 * padded to whole tiles with its halo, reaches 2^31 elements (the kernels
 * index fields by 32-bit offsets; this bounds very elongated domains). */
int bq_workspace_bytes(const bq_params* p, size_t* bytes);

/* Create a domain in the caller's device workspace; hip_stream is a
 * hipStream_t (NULL = the null stream).  depth_c is the host corner
 * still-water depth, (ny+1) x (nx+1) row-major; a non-finite value is
 * rejected with BQ_EINVAL before anything reaches the device (so are
 * non-finite wave components and time-series samples, here and in
 * bq_workspace_bytes).  Precomputes the static fields and the factorisation
 * data of Eq. (19)-(21).  State: lake at rest. */
int bq_domain_create(const bq_params* p, const double* depth_c, void* dev_workspace, size_t bytes,
                     void* hip_stream, bq_domain** out);
int bq_domain_free(bq_domain* d);

/* Host FP64 interior arrays (nx*ny each): eta (Sec. 2: eta = h - d), P, Q.
 * Rejects eta < -d (negative depth) with BQ_EINVAL.  Clears the AB3 history,
 * so the next two steps are forward Euler.  Synchronous. */
int bq_set_state(bq_domain* d, const double* eta, const double* P, const double* Q);

/* Enqueue n_steps adaptive steps (asynchronous; returns launch errors only). */
int bq_step(bq_domain* d, int32_t n_steps);
/* Enqueue one step with a prescribed Delta t (bypasses Eq. 22 and 47). */
int bq_step_dt(bq_domain* d, double dt);

/* Wait for the domain's stream; fill *out (may be NULL) and return the
 * latched status. */
int bq_sync(bq_domain* d, bq_info* out);

/* Synchronous read of the interior, FP64: which = 0 eta, 1 P, 2 Q, 3 w,
 * 4 the run-up record (NaN where the depth never exceeded runup_delta;
 * BQ_EINVAL unless runup_delta > 0), 5 the local CFL number of Eq. (22) of
 * the current state with the Delta t of the last step,
 * dt_last * max((|u|+c)/dx, (|v|+c)/dy) (Sec. 5.2). */
int bq_read(bq_domain* d, int32_t which, double* host_out);

/* Checkpoint of the full state including the AB3 history, so a resumed run
 * continues bit-for-bit.  bq_save with host == NULL returns the size. */
int bq_save(bq_domain* d, void* host, size_t* bytes);
int bq_load(bq_domain* d, const void* host, size_t bytes);

/* Batches: domains of one precision advanced together, one launch per phase
 * over a flattened tile work-list.  Domains keep their own Delta t, time and
 * status; a halted domain is skipped.  bq_batch_set replaces the member list
 * (attach/detach between steps).  All members must have been created on the
 * batch's stream or be idle. */
int bq_batch_create(bq_domain* const* doms, int32_t n, void* hip_stream, bq_batch** out);
int bq_batch_set(bq_batch* b, bq_domain* const* doms, int32_t n);

/* For callers that cannot allocate device memory (code under stream capture,
 * a serving loop that admits and retires members between steps, hosts that
 * forbid hipMalloc): bq_batch_set without any device allocation or release.
 * The batch's tables (member descriptors, tile and line work maps) go into a
 * static array of BQ_STATIC_TABLE_BYTES on the current device instead of
 * memory the batch allocates; a member list needing more returns BQ_EINVAL
 * and leaves the batch as it was.  Call it with the batch's device current.
 * There is one such array per device, shared by every batch on it: the
 * call waits for the work queued by the batch that used the array before,
 * and from then on that batch's steps, profiles and schedule changes return
 * BQ_ESTATE until it sets its members again (either call).  Calls for two
 * batches of one device that overlap in time (from two host threads) race.
 * The batch's lane streams exist from bq_batch_create on; the step graphs
 * are re-captured by the next bq_batch_step.  Results are those of
 * bq_batch_set with the same members, bit for bit. */
int bq_batch_set_static(bq_batch* b, bq_domain* const* doms, int32_t n);
int bq_batch_step(bq_batch* b, int32_t n_steps);
int bq_batch_sync(bq_batch* b);

/* Latched status of every member after the work queued so far, for a loop
 * that polls many members (serving): one small kernel and one copy for the
 * whole batch instead of a bq_sync per member.  status[k] is member k's
 * bq_status (BQ_EDONE once its time reached t_end), steps[k] its step count
 * and t[k] its time (Sec. 3.2.2: the sum of its own Delta t); steps and t
 * may be NULL; arrays hold the member count.  Waits for the batch's stream. */
int bq_batch_status(bq_batch* b, int32_t* status, int64_t* steps, double* t);
int bq_batch_free(bq_batch* b);

/* Launch lanes of a batch (1 to 4; default 2, at most the member count).
 * With several lanes the members are split into groups of about equal cell
 * count and each group is advanced on its own stream; the batch creates the
 * streams itself, one after the other, so the runtime gives them different
 * hardware queues.  The lanes start after the work queued on the batch's
 * stream and the batch's stream waits for all of them (events at the start
 * and end of every bq_batch_step), so the caller sees one stream.  One
 * group's stencil/update kernel (arithmetic bound) then runs beside another
 * group's line-coupling and finalize kernels (latency and bandwidth bound).
 * Each domain's arithmetic is the same for any lane count, so results are
 * bitwise identical.  Changing the lane count waits for the batch's queued
 * work.  bq_batch_lanes returns the lanes in use. */
int bq_batch_set_lanes(bq_batch* b, int32_t lanes);
int bq_batch_lanes(const bq_batch* b);

/* Timing of the step's four kernels (Delta t, stencil + AB3 + local solves,
 * line coupling, finalize): runs n_steps plain launches with hipEvents around
 * every kernel on the launch stream and returns the mean duration of one
 * launch of each in ms_out[4].  A two-lane batch runs both lanes at once, as
 * bq_batch_step does, each launch covering one group.  With the corrector
 * each entry is the sum over the step's two passes of that kernel.  The
 * steps advance the state like bq_step / bq_batch_step. */
int bq_profile_steps(bq_domain* d, int32_t n_steps, double* ms_out);
int bq_batch_profile_steps(bq_batch* b, int32_t n_steps, double* ms_out);

/* Schedule of a batch: launch lanes, steps per hipGraph replay, threads per
 * block of the line-coupling kernel (64, 128 or 256), the XCD-aware tile
 * order of the stencil kernel (1 on, 0 off), the line-coupling variant
 * (reduce_segments 1 = one thread per line running over its chunks, 4 or 8 =
 * the chunks of a line cut into that many segments swept by as many waves
 * that exchange their composed maps; reduce_block is then ignored, give
 * 256), and the tile shape shared by the members (the chunking of the
 * tridiagonal solves of Eq. 19-20; the workspace is laid out for every
 * candidate, so members change shape between steps in place).  With
 * reduce_segments 1 every schedule of one tile shape gives bitwise the same
 * results; the segmented variant reassociates the line-coupling products,
 * and another tile shape chunks the line solves differently: both differ
 * at rounding level. */
typedef struct bq_tune {
  int32_t lanes;
  int32_t graph_steps;
  int32_t reduce_block;
  int32_t swizzle;
  int32_t reduce_segments;
  int32_t tile_y;          /* tile height = y-chunk length of the line solves */
  int32_t chunk_x;         /* x-chunk length of the line solves (tiles are 64
                              cells wide); FP32 takes 16 x 16, 16 x 32, 8 x 16,
                              8 x 32, FP64 8 x 16, 8 x 32, 4 x 16 (tile_y x
                              chunk_x; both 0 in bq_batch_set_tune: keep) */
  double ms_per_step;      /* bq_batch_autotune: measured time of one step */
} bq_tune;

/* Autotuner: times steps_per_trial steps of the batch under each candidate
 * schedule (lanes 1-4 x graph replays of 4 or 16 steps x line coupling by
 * one thread per line in blocks of 64 or 256, or segmented; XCD-aware tile
 * order on; the current tile shape) twice, in forward then reverse order,
 * keeps the one of the lowest mean time (among those within 0.5 % of it,
 * the one with the longest graph replays), then times every tile shape
 * under that schedule the same way and returns the fastest.  The
 * trial steps are real steps (the domains advance by them).  bq_batch_set_tune applies a schedule, for
 * instance one cached from an earlier autotune of a batch of the same shape;
 * bq_batch_get_tune reports the current one (ms_per_step 0). */
int bq_batch_autotune(bq_batch* b, int32_t steps_per_trial, bq_tune* out);
int bq_batch_set_tune(bq_batch* b, const bq_tune* t);
int bq_batch_get_tune(const bq_batch* b, bq_tune* out);

/* Number of steps captured per hipGraph replay (0 = plain launches). */
int bq_set_graph_steps(bq_domain* d, int32_t steps);
int bq_batch_set_graph_steps(bq_batch* b, int32_t steps);

#ifdef __cplusplus
}
#endif
#endif
