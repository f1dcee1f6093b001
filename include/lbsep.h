/*
 * lbsep -- binary-gas-mixture lattice Boltzmann channel solver for MI355X (gfx950).
 *
 * C ABI of the hot path of Wang, Xu & Guo, "Lattice Boltzmann simulation of
 * separation phenomenon in a binary gaseous flow through a microchannel"
 * (arXiv:1603.08221):
 *   - Sec. 2: an L x H channel between two reservoirs, pressure ratio theta,
 *     light-species mole fraction C_l (Eq. (C)), outlet Knudsen number Kn_out;
 *     separation degree CL (Eq. (CL)) and mean separation C~_l (Eq. (Clline)).
 *   - Sec. 3.1: two coupled D2Q9 populations (Eq. (MRT)), MRT collision
 *     (Eqs. (MR), (m), (S)) towards the species equilibrium built on the mixture
 *     velocity (Eq. (feq)), effective relaxation times with the mean-free-path
 *     wall function (Eqs. (EQFrb), (taos), (EQFrsp)).
 *   - Sec. 3.2: diffuse-bounce-back walls (Eqs. (bot), (bot2), (taoq), (A12))
 *     and the extrapolation-correction pressure inlet/outlet (Eqs. (rho1), (rho2)).
 *
 * Entry points: one channel (lbsep_init ... lbsep_destroy), batches of
 * channels advanced by one launch per step (lbsep_batch_*), and the discrete
 * adjoint of the step for gradients of CL (lbsep_adjoint_*).
 *
 * Lattice units: delta_x = delta_t = 1, c_s^2 = 1/3, H = ny. Outlet pressure
 * P_out = 1/3 (so that n_out * m_min = 1); P_in = theta * P_out.
 *
 * Conventions for every call:
 *   - Return 0 on success, a negative LBSEP_E* code on failure; the message of
 *     the last failure on the calling thread is in lbsep_last_error().
 *   - No C++ exception crosses this boundary. The library never allocates
 *     device memory: the caller owns the workspace and every host buffer; the
 *     library owns only the small host-side handle (and, for
 *     lbsep_adjoint_step_noalloc only, one fixed scratch array per GPU that
 *     is part of its code object).
 *   - Work is enqueued on the HIP stream given to lbsep_init, in order. Calls
 *     marked "synchronises" wait for that stream before returning.
 *   - A handle is not thread-safe; use one handle per thread or serialise.
 *
 * Population layout (lbsep_get_populations / lbsep_set_populations, and the
 * raw state of lbsep_get_state / lbsep_set_state): dense, element
 * ((s * 9 + i) * ny + j) * nx + x, s = 0 light species (a), 1 heavy (b); i in
 * the D2Q9 order c_0..c_8 = (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1)
 * (-1,-1) (1,-1); j = row across the channel (node centre y = j + 1/2, walls
 * at y = 0 and y = ny); x = column along the flow (column 0 = inlet node,
 * nx-1 = outlet node). Populations are the pre-collision state f_si(x, y, t).
 *
 * Storage types (lbsep_params.dtype):
 *   LBSEP_F64: f stored and collided in double. The raw state is f (double).
 *   LBSEP_F32, LBSEP_F16: the deviation d = f - f0 from the rest equilibrium
 *     f0_si(x) = w_i alpha_si rho0_s(x) (Eq. (feq) at u = 0), with rho0_s linear
 *     in x from rho_s,in at x = 0 to rho_s,out at x = nx-1 (constant rho_s,in
 *     with LBSEP_PERIODIC_X), is stored as float / IEEE binary16 and collided in
 *     float. The raw state is d in the storage type (4 / 2 bytes).
 * Column sums, CL and C~_l are always reduced in double.
 */
#ifndef LBSEP_H
#define LBSEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define LBSEP_OK 0
#define LBSEP_EINVAL (-1)     /* an argument outside its documented range           */
#define LBSEP_ESIZE (-2)      /* workspace smaller than lbsep_workspace_bytes()      */
#define LBSEP_EDEVICE (-3)    /* a HIP runtime call failed                           */
#define LBSEP_ENONFINITE (-4) /* the diagnostics saw NaN/Inf or a non-positive density */
#define LBSEP_ERANGE (-5)     /* a requested history record is no longer kept       */

/* ---- flags (lbsep_params.flags) -------------------------------------- */
#define LBSEP_PERIODIC_X 0x1u /* no inlet/outlet: columns wrap (test mode)                   */
#define LBSEP_PERIODIC_Y 0x2u /* no walls: rows wrap (test mode; requires LBSEP_MFP_OFF)      */
#define LBSEP_MFP_OFF 0x4u    /* wall function Psi == 1 (unbounded mean free path)            */
#define LBSEP_BGK_TEST 0x8u   /* every relaxation time = tau_bgk (BGK limit after Eq. (S))    */

/* ---- storage / arithmetic type (lbsep_params.dtype) ------------------ */
#define LBSEP_F64 0 /* populations stored and collided in double                              */
#define LBSEP_F32 1 /* deviations from the rest equilibrium stored and collided in float     */
#define LBSEP_F16 2 /* deviations stored as IEEE binary16, collided in float                 */
/* In FP64 the wall function (Sec. 3.1) is evaluated from piecewise polynomials
 * on channels of more than 2^17 nodes (fewest operations: the channels that
 * fill the GPU) and from its series and exponential form on smaller ones
 * (registers only: their steps are latency-bound when they run alone). The
 * two agree to about 1e-16; a channel uses one of them in every kernel that
 * steps it, alone, in a batch or in the adjoint. */

/* ---- tile shape of the sweep (lbsep_params.tile_mode) ----------------- */
#define LBSEP_TILE_AUTO 0  /* chosen from the channel size                                */
#define LBSEP_TILE_SPLIT 1 /* two lanes per node, one per species (latency-bound channels) */
#define LBSEP_TILE_NODE 2  /* one lane per node (channels that fill the GPU many times)   */

/* Problem statement (Sec. 2) plus the DBB inputs of Sec. 3.2. */
typedef struct lbsep_params {
  int32_t nx;       /* columns along the flow (channel length L): >= 6, or >= 1 with PERIODIC_X */
  int32_t ny;       /* rows across the channel (H = ny lattice units, the N of Eq. (taoq)): 2..2048 */
  double m_a;       /* molecular mass of the light species, > 0                                   */
  double m_b;       /* molecular mass of the heavy species, >= m_a (only ratios matter)          */
  double cl_in;     /* light-species mole fraction at the inlet, in (0, 1)                        */
  double cl_out;    /* light-species mole fraction at the outlet, in (0, 1)                       */
  double theta;     /* pressure ratio P_in / P_out, > 0                                          */
  double kn_out;    /* Kn_out = lambda_out / H, > 0                                              */
  double dbb_r;     /* DBB equilibrium fraction r of Eqs. (bot), (bot2), in [0, 2); both species */
  double accom;     /* accommodation coefficient alpha of Eq. (A12), in (0, 1]                   */
  double tau_bgk;   /* relaxation time for LBSEP_BGK_TEST, > 0.5; ignored otherwise             */
  uint32_t flags;   /* LBSEP_PERIODIC_X | LBSEP_PERIODIC_Y | LBSEP_MFP_OFF | LBSEP_BGK_TEST      */
  int32_t dtype;    /* LBSEP_F64, LBSEP_F32 or LBSEP_F16                                         */
  int32_t hist_cap; /* per-step diagnostic records kept on the device (ring), >= 1               */
  int32_t tile_mode; /* LBSEP_TILE_AUTO / _SPLIT / _NODE: how nodes map to lanes (same results)  */
  int32_t tile_rows; /* rows each wavefront of a tile walks (a tile is 8 wavefronts for
                        LBSEP_F32, 4 otherwise, each on 64 columns, or 32 with lane pairs):
                        0 = chosen from the size (4 if that leaves >= 2048 tiles, except for
                        LBSEP_F32; 2 if >= 512; else 1), else 1, 2 or 4. The states are the
                        same whatever the value; the column sums behind CL and the profiles are
                        associated per tile, so those may differ in the last bits. A channel in
                        a batch that fills the GPU can be faster with 2 or 4 (fewer row-tile
                        partial sums). */
  int32_t fused_steps; /* time levels per sweep launch: 0 = chosen by the library (currently 1),
                        1, or 2 (needs ny <= 128 for LBSEP_F32 and LBSEP_F16, ny <= 64 for
                        LBSEP_F64, and an inlet, an outlet and walls: no periodic flag; else
                        LBSEP_EINVAL). With 2, a launch advances two levels, keeping the first
                        in LDS (about half the HBM traffic per level); the states are bitwise
                        those of single-level launches, CL and the column sums agree to
                        rounding. A third state buffer is allocated; readouts right after a
                        two-level launch recompute the level before (one launch). Such a
                        channel joins only a batch whose members all use 2. Measured per level
                        on 64-row channels: faster in FP32 at every length (64x1280 5.3 vs
                        7.4 us, 64x81920 120 vs 150 us); in FP64 only on short ones (64x1280
                        11.6 vs 13.6 us; from 2560 columns on slower, 64x20480 137 vs 89 us). */
} lbsep_params;

typedef struct lbsep_channel lbsep_channel;

/* Device workspace needed for these parameters (bytes, 256-byte aligned start
 * required). Returns 0 if the parameters are invalid (see lbsep_last_error). */
size_t lbsep_workspace_bytes(const lbsep_params* params);

/* Bytes of one raw state (2 * 9 * ny * nx elements of the storage type). */
size_t lbsep_state_bytes(const lbsep_params* params);

/* Create a channel in the caller's device workspace and set the initial state:
 * local equilibrium at rest with pressure and C_l linear in x between the
 * inlet and outlet values. The diagnostics of t = 0 are recorded.
 *   params      : copied; validated (LBSEP_EINVAL).
 *   dev_ws      : device pointer, 256-byte aligned, ws_bytes >= lbsep_workspace_bytes.
 *   hip_stream  : hipStream_t the channel enqueues on (NULL = default stream).
 *   out         : receives the handle; *out is NULL on failure.
 * Enqueues work; does not synchronise. */
int lbsep_init(const lbsep_params* params, void* dev_ws, size_t ws_bytes, void* hip_stream,
               lbsep_channel** out);

/* Advance nsteps >= 0 time steps. Each step is one fused sweep: pull-streaming
 * of both species (Eq. (MRT)), DBB at the walls (Eqs. (bot), (bot2)), the
 * inlet/outlet correction (Eqs. (rho1), (rho2)), moments (Eq. (rhou)),
 * relaxation times (Eqs. (taos), (EQFrsp), (taoq)), MRT collision
 * (Eq. (MR)), and the reduction of the new state to C_l(x), CL and C~_l
 * (Eqs. (C), (CL), (Clline)) recorded for that step. Enqueues only. */
int lbsep_step(lbsep_channel* ch, int64_t nsteps);

/* One step as lbsep_step (same state, same record) that also writes, in
 * double and the dense layout of lbsep_get_populations (2 * 9 * ny * nx
 * doubles each, caller-owned device memory), the new level's pre-collision
 * populations f(t+1) to dev_pre and its post-collision populations
 * C(f(t+1)) to dev_post: what lbsep_get_populations and
 * lbsep_get_post_collision would return after the step, from the sweep
 * itself. For the recomputation of the adjoint's segments. Needs an FP64
 * channel with one level per launch (fused_steps 0 or 1): LBSEP_EINVAL
 * otherwise, or when a pointer is NULL. Enqueues only. */
int lbsep_step_record(lbsep_channel* ch, double* dev_pre, double* dev_post);

/* Current time level t (number of steps since the initial/loaded state plus its t). */
int64_t lbsep_time(const lbsep_channel* ch);

/* Diagnostics of the current state: CL (Eq. (CL)), C~_l (Eq. (Clline)), the
 * column of the smallest C_l (first on ties), and optionally the profile
 * C_l(x) (nx doubles) of Eq. (C) over each cross-section. Any pointer may be
 * NULL. Synchronises. LBSEP_ENONFINITE if any step since init saw NaN/Inf or a
 * non-positive column density. */
int lbsep_read_cl(lbsep_channel* ch, double* cl, double* cl_tilde, int32_t* x_min, double* cl_profile);

/* Column sums of the current state, host [4][nx]: sum_j n_a, sum_j n_b,
 * sum_j rho_a u_ax, sum_j rho_b u_bx (species velocity of Eq. (rhou)).
 * The density sums are those behind the CL record; one-level steps carry no
 * momentum sums, so for a channel last advanced by one-level launches these
 * come from an extra evaluation sweep of the current state (no store).
 * Synchronises. */
int lbsep_read_column_sums(lbsep_channel* ch, double* host);

/* Per-step records for time levels t0 .. t0+count-1, host [count][4]:
 * (t, CL, C~_l, x_min). LBSEP_ERANGE if a level is older than the last
 * hist_cap steps or newer than the current time. Synchronises. */
int lbsep_read_history(lbsep_channel* ch, int64_t t0, int64_t count, double* host);

/* Moments of the current state, host [6][ny][nx] doubles: rho_a, rho_b,
 * u_ax, u_ay, u_bx, u_by (species velocities of Eq. (rhou)). Uses the
 * workspace; synchronises. */
int lbsep_read_moments(lbsep_channel* ch, double* host);

/* Volume flow of the mixture through every cross-section (the Q_v of Sec. 4,
 * whose formula is not printed; reading: Q_v(x) = sum_j u_x(x, j) delta_y with
 * the mixture velocity u of Eq. (rhou), lattice units), host [nx] doubles.
 * Uses the workspace; synchronises. */
int lbsep_read_volume_flow(lbsep_channel* ch, double* host);

/* Write the current raw state (storage representation, layout above) to
 * device memory dev_dst (lbsep_state_bytes bytes): a bitwise checkpoint.
 * Enqueues only. */
int lbsep_get_state(lbsep_channel* ch, void* dev_dst);

/* Replace the state by a raw state dev_src (device, as written by
 * lbsep_get_state) at time level t >= 0 and record its diagnostics; stepping
 * on from it reproduces the original run bitwise. Enqueues only. */
int lbsep_set_state(lbsep_channel* ch, const void* dev_src, int64_t t);

/* Write the current pre-collision populations f in double (2 * 9 * ny * nx
 * doubles, layout above) to device memory dev_dst, whatever the storage type.
 * Enqueues only. */
int lbsep_get_populations(lbsep_channel* ch, double* dev_dst);

/* Write the current post-collision populations f'(t) = C(f(t)) in double
 * (2 * 9 * ny * nx doubles, layout above) to device memory dev_dst: the state
 * the next step streams, as the last sweep (or set / init) computed it. For
 * deviation storage the stored value plus f0 of the node's column. Sec. 3.1,
 * Eq. (MRT): the collision's output before streaming. Enqueues only. */
int lbsep_get_post_collision(lbsep_channel* ch, double* dev_dst);

/* Replace the state by the populations f given in double (device, layout
 * above), converted to the storage type, at time level t >= 0, and record
 * its diagnostics. Enqueues only. */
int lbsep_set_populations(lbsep_channel* ch, const double* dev_src, int64_t t);

/* DBB coefficient from a velocity slip coefficient c_m, Eq. (R) first form:
 * r = 2 - 2 / (1 + (c_m / 3) sqrt(pi m_x / (2 k_B T))), k_B T = m_min c_s^2,
 * m_x = cl m_a + (1 - cl) m_b. Returns NaN on invalid input. */
double lbsep_dbb_r_from_cm(double c_m, double m_a, double m_b, double cl);

/* The device wall function of Sec. 3.1, element-wise on n arguments:
 * psi(alpha) = 1 + (alpha - 1) e^-alpha - alpha^2 E1(alpha) and
 * h(alpha) = psi'(alpha) / 2 = e^-alpha - alpha E1(alpha), evaluated exactly as
 * the sweep kernel does in the arithmetic of dtype (double for LBSEP_F64, float
 * otherwise). table (0 or 1; LBSEP_F64 only, ignored otherwise): 1 evaluates as
 * FP64 channels of more than 2^17 nodes do (piecewise polynomials), 0 as
 * smaller FP64 channels do (power series, exponential and octave Chebyshev
 * series); the two agree to about 1e-16. dev_alpha, dev_psi, dev_h: device
 * arrays of n doubles (dev_h may be NULL). Enqueues on hip_stream (NULL =
 * default stream). LBSEP_EINVAL for n < 0, missing arrays, a bad dtype or
 * table. */
int lbsep_wall_function(const double* dev_alpha, double* dev_psi, double* dev_h, int64_t n, int32_t dtype,
                        int32_t table, void* hip_stream);

/* Release the host handle (the workspace stays the caller's). NULL is a no-op. */
void lbsep_destroy(lbsep_channel* ch);

/* Message of the last failure on this thread ("" if none). */
const char* lbsep_last_error(void);

/* ---- batches: the parametric sweeps of Table 1 / Sec. 4 as one launch ------
 * A batch advances several independent channels (uneven sizes, any parameters
 * of Table 1's kind) by one sweep kernel per step: every channel keeps its own
 * workspace, reductions and CL history, and its results are bitwise those of
 * stepping it alone. The member channels stay usable through the channel API
 * (read_cl, read_moments, get_state ...) between batch steps; stepping or
 * resetting a member on its own invalidates the batch (its next step fails
 * with LBSEP_EINVAL). Members must outlive the batch. The members share one
 * fused_steps value: with 2, each launch advances every member by two levels
 * (an odd remainder by one), as stepping each alone would. */
typedef struct lbsep_batch lbsep_batch;

/* Device workspace bytes for a batch of the n channels chans[0..n-1] (one
 * dtype, one stream, one fused_steps, no channel twice); 0 on invalid input. */
size_t lbsep_batch_workspace_bytes(lbsep_channel* const* chans, int32_t n);

/* Build the batch's instance table in dev_ws (caller-owned, 256-byte aligned,
 * >= lbsep_batch_workspace_bytes) from the members' current states.
 * Synchronises the stream once. */
int lbsep_batch_create(lbsep_channel* const* chans, int32_t n, void* dev_ws, size_t ws_bytes, lbsep_batch** out);

/* Advance every member by nsteps levels: replays of the captured step graph
 * while at least its length remains, single launches for the rest. Enqueues
 * only. */
int lbsep_batch_step(lbsep_batch* b, int64_t nsteps);

/* Capture `steps` batch steps (1 .. 100000) into a HIP graph replayed by
 * lbsep_batch_step; 0 drops the graph. Needs a non-default stream. The
 * executable graph's upload to the device is enqueued on that stream. */
int lbsep_batch_capture(lbsep_batch* b, int64_t steps);

/* Number of member channels; -1 for NULL. */
int32_t lbsep_batch_size(const lbsep_batch* b);

/* Release the batch's host handle and graph (members and workspace stay the
 * caller's). NULL is a no-op. */
void lbsep_batch_destroy(lbsep_batch* b);

/* ---- discrete adjoint (reverse mode) of the step --------------------------
 * The step of Sec. 3 as a map of the pre-collision populations,
 * f(t+1) = E(P(C(f(t)))): C the collision of Sec. 3.1 with the relaxation
 * times of Eqs. (taos), (EQFrsp), (taoq) recomputed from the node's densities,
 * P the streaming of Eq. (MRT) with the DBB walls of Eqs. (bot), (bot2), E the
 * inlet/outlet of Eqs. (rho1), (rho2). The parameters differentiated are
 * (theta, C_in, r): theta and C_in through the inlet densities of Eq. (rho2)
 * and the initial state of R18, r through the DBB walls; C_out, Kn_out and the
 * masses are held. All arithmetic is FP64 on populations and adjoints in the
 * dense layout [2][9][ny][nx] of lbsep_get_populations (whatever the channel's
 * storage type); the channel supplies the parameters and the stream. adj_ws:
 * caller-owned device workspace, 256-byte aligned, of
 * lbsep_adjoint_workspace_bytes. dparams: device double[3] (theta, C_in, r),
 * accumulated (+=). All calls enqueue only. */
size_t lbsep_adjoint_workspace_bytes(const lbsep_params* p);

/* lam_out = (d f(t+1) / d f(t))^T lam_next at the pre-collision state f_t;
 * dparams += lam_next . d f(t+1) / d(theta, C_in, r) at fixed f_t.
 *   f_post : C(f_t), the post-collision populations of the same level as
 *            written by lbsep_get_post_collision, or NULL: the library then
 *            recomputes C(f_t) in the adjoint workspace (one more launch).
 * lam_out must not alias f_t, f_post or lam_next. */
int lbsep_adjoint_step(lbsep_channel* ch, const double* f_t, const double* f_post, const double* lam_next,
                       double* lam_out, double* dparams, void* adj_ws, size_t adj_ws_bytes);

/* Size of the fixed device scratch of lbsep_adjoint_step_noalloc: 8 MiB per GPU. */
#define LBSEP_FIXED_SCRATCH_BYTES (8u << 20)

/* lbsep_adjoint_step without a workspace, for callers that cannot allocate
 * device memory at the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc). Same reverse step, same kernels,
 * same results as lbsep_adjoint_step; its scratch (the closure's adjoints on
 * the end columns, the per-block r partials and, when f_post is NULL, the
 * recomputed C(f_t)) lives in a fixed array of LBSEP_FIXED_SCRATCH_BYTES
 * inside the library, one per GPU, set up on the first call on that GPU and
 * held until the process ends. Allocates nothing, and calls no allocating
 * routine.
 *   Sizes: needs 864 ny + 8 ceil(nx ny / 256) bytes plus a few KB, and
 *   144 nx ny bytes more when f_post is NULL (at most about 57,000 nodes);
 *   LBSEP_ESIZE when that exceeds LBSEP_FIXED_SCRATCH_BYTES (nothing is
 *   enqueued then).
 *   Sharing: every call on one GPU uses that GPU's one array, and each call
 *   overwrites everything of it that the call reads. Calls that overlap in
 *   time on one GPU (several streams, several host threads) race on it and
 *   must be serialised by the caller; stream-ordered calls on one stream are
 *   safe. Other arguments, errors and aliasing rules as lbsep_adjoint_step.
 * Enqueues only. */
int lbsep_adjoint_step_noalloc(lbsep_channel* ch, const double* f_t, const double* f_post, const double* lam_next,
                               double* lam_out, double* dparams);

/* Seed of J = CL (Eq. (CL)) at the pre-collision state f_T: lam_out = dCL/df_T
 * (nonzero on the column of the smallest C_l only, R16) and dparams[1] +=
 * the explicit dCL/dC_in = C_l,min / C_in^2. */
int lbsep_adjoint_seed_cl(lbsep_channel* ch, const double* f_T, double* lam_out, double* dparams, void* adj_ws,
                          size_t adj_ws_bytes);

/* dparams[0..1] += lam0 . d f(0) / d(theta, C_in) for the initial state of R18
 * (local equilibrium at rest, pressure and C_l linear in x). Needs inlet and
 * outlet (not LBSEP_PERIODIC_X). */
int lbsep_adjoint_initial(lbsep_channel* ch, const double* lam0, double* dparams, void* adj_ws, size_t adj_ws_bytes);

#ifdef __cplusplus
}
#endif

#endif /* LBSEP_H */
