/*
 * sgtp.h -- C ABI of the MI355X SGTP planner (Sampling-based Game-Theoretic
 * Planning for multi-vehicle racing).
 *
 * One planning step is Alg. 1 of the paper: initial trajectories without the
 * game-aware cost, L_IBR Jacobi sweeps in which every vehicle computes a sampled
 * best response against the previous sweep's trajectories of its opponents,
 * then one extra best response of the ego vehicle.  A best response (Sec. III)
 * perturbs the nominal control sequence K times with Gaussian noise, clips the
 * controls to the admissible box, rolls every sequence out through the vehicle
 * model, scores it with the tracking cost (eq. ctrack) plus the game-aware cost
 * (eqs. game_cost, c_contest, c_long, c_block, c_safety; total eq. allc), checks
 * track boundary (eq. selection-boundary) and collision (eqs. Dmin,
 * selection-vehicle), and selects the lowest-cost feasible sample (eq.
 * selection), or the least-violation sample when none is feasible.
 *
 * Conventions for every call below
 *   - Arrays are contiguous, row-major.  Pointers inside sgtp_race and the
 *     output arrays are DEVICE pointers owned by the caller; the sgtp_params,
 *     sgtp_race structs themselves and the node table of sgtp_track_upload are
 *     HOST memory, read during the call only.
 *   - `stream` is a hipStream_t (NULL = default stream).  Calls only enqueue
 *     work and return; outputs are valid once the stream reaches that point.
 *   - Return value: SGTP_OK (0) or a negative error code.  Argument errors are
 *     detected before anything is enqueued, so outputs are untouched;
 *     sgtp_last_error() returns a text for the last failing call on a context.
 *   - A context is bound to the device current at creation and must be used
 *     from one host thread at a time.  Calls on one context must be issued on
 *     one stream (the context owns workspace that successive calls reuse).
 *   - The three planning calls allocate nothing.  They do not synchronise the host
 *     except in one case: the descriptor images of each call pass through a ring of
 *     8 pinned staging buffers, each guarded by an event, and a call that comes
 *     round to a buffer whose previous copy has not completed waits for that event
 *     (hipEventSynchronize) before it reuses the buffer.
 *
 * Frames and units: world frame in metres and radians; states are
 * (x, y, psi, v_x, v_y, omega) at the centre of gravity (the kinematic model
 * uses (x, y, psi, v) in the first four entries); controls (a [m/s^2], delta [rad]).
 */
#ifndef SGTP_H
#define SGTP_H

#ifdef __cplusplus
extern "C" {
#endif

#define SGTP_OK 0
#define SGTP_EINVAL (-1)  /* null pointer, bad enum or value out of range */
#define SGTP_ESHAPE (-2)  /* size beyond what the context was created for */
#define SGTP_ETRACK (-3)  /* unknown track id, or track does not fit the kernels */
#define SGTP_EDEVICE (-4) /* HIP runtime or launch error */
#define SGTP_ENOMEM (-5)  /* device allocation failed (calls that allocate: context, plans, autotune) */

/* Bits of the context status word (sgtp_ctx_status). */
#define SGTP_STATUS_WAIT_GAVE_UP 1   /* a sample's bounded LDS wait gave up: that sample was scored non-finite */
#define SGTP_STATUS_REROLL_GAVE_UP 2 /* a winner re-roll's bounded LDS wait gave up: its outputs are unreliable */

#define SGTP_MAX_AGENTS 16 /* vehicles per race */
#define SGTP_MAX_N 64      /* horizon steps */
#define SGTP_MAX_K (1 << 24)
#define SGTP_TRAJ_STRIDE 8 /* trajectory row: x, y, psi, vx, vy, omega, s, d */

typedef struct sgtp_ctx sgtp_ctx;

/* Planner parameters (Sec. IV-B lists the paper's values). */
typedef struct {
    int model;                 /* 0 = dynamic single-track, 1 = kinematic bicycle */
    float dt;                  /* control interval [s] */
    float a_min, a_max;        /* admissible box of Pi_U */
    float d_min, d_max;
    float sigma_a, sigma_d;    /* perturbation std devs, Sigma_u = diag(sigma_a^2, sigma_d^2) */
    float Q[4];                /* tracking weights on (x, y, psi, v) */
    float R[2];                /* control weights */
    float S[2];                /* control-rate weights */
    float w_game, w_contest, w_long, w_block, w_safety;
    float s_contest, s_role, eps_alpha;
    float g_safe;              /* safety distance of eq. (c_safety) */
    float m_bd;                /* boundary margin of eq. (selection-boundary) */
    float d_col;               /* collision threshold of eq. (selection-vehicle) */
    int n_disc;                /* footprint discs along the heading: 1 or 3 */
    float disc_off[4];         /* disc offsets from the centre of gravity [m] */
    float m, Iz, lf, lr;       /* vehicle mass, yaw inertia, CoG-axle distances */
    float B, C, mu, g;         /* tyre F_y = mu F_z sin(C atan(B alpha)); gravity */
    float v_eps;               /* speed floor inside the slip angles [m/s] */
    int max_moves;             /* segment-search limit of the Frenet projection */
    /* Best-response update.  0: feasibility selection (Sec. III-B).  1: path-integral
     * update of the GA-IBR-MPPI ablation (Sec. IV-A): every sample with a finite score
     * S = c + mppi_w_viol * nu is weighted by exp(-(S - S_min) / mppi_lambda) and the
     * nominal becomes the weighted mean of the sampled sequences (no feasibility
     * selection; needs sgtp_ctx_enable_path_integral; no learned proposal). */
    int update;
    float mppi_lambda;         /* temperature (> 0) */
    float mppi_w_viol;         /* weight of the violation nu in the score (>= 0) */
    /* Perturbation of the opponents' predicted positions (robustness experiment, Sec.
     * IV-F, Table II): each predicted position tau = 1..N of opponent j, as staged for
     * vehicle i in a phase, moves by pred_sig_lon z0 along and pred_sig_lat z1 across the
     * predicted heading, (z0, z1) the Box-Muller pair of Philox(counter = (2^31 | j, tau,
     * i | phase << 16, plan_step), key = seed).  0, 0 = off. */
    float pred_sig_lon, pred_sig_lat;
} sgtp_params;

/* One race (one game) at one planning instant. */
typedef struct {
    int n_agents;              /* 1..SGTP_MAX_AGENTS */
    int ego;                   /* index of the ego vehicle e */
    int track_id;              /* track uploaded with sgtp_track_upload */
    int N;                     /* horizon H, 1..SGTP_MAX_N */
    int n_tail;                /* |T_tail|, 1..N (final steps averaged by eq. c_block) */
    int K;                     /* samples per best response, 1..SGTP_MAX_K */
    unsigned long long seed;   /* Philox key of the race */
    unsigned int plan_step;    /* Philox counter word of this planning step */
    double *x;                 /* [n][6] current states (read; sgtp_advance updates them) */
    double *s_abs;             /* [n] unwrapped progress: in = previous value or NaN, out = current */
    const float *v_scale;      /* [n] reference-speed scale of each vehicle (opponents 0.9, Sec. IV-B) */
    float *u_nom;              /* [n][N][2] nominal sequences U-bar (in/out: warm start) */
    double *traj;              /* [n][N+1][8] out: planned trajectories, or NULL */
    float *prop;               /* [n][N][4] learned proposal (mu_a, mu_d, sigma_a, sigma_d), or NULL */
    int K_prop;                /* samples k < K_prop are drawn about the proposal, the rest about u_nom */
} sgtp_race;

/* Result of one best response. */
typedef struct {
    int k;                     /* selected sample k* */
    int fallback;              /* 1 when no sample was feasible (least-violation choice) */
    int n_feasible;            /* number of feasible samples */
    float cost;                /* c of k* (eq. allc) */
    float viol;                /* total violation nu of k* (0 when feasible) */
} sgtp_choice;

/* ---- context and tracks ---------------------------------------------------- */

/* Create a context on the current device with workspace for up to
 * max_agents_total vehicles over all races of one call, horizons up to max_N,
 * max_races races per call, track tables of up to max_track_nodes nodes and up to
 * max_K samples per best response (checkpoint slots: 576 bytes per 64 samples).
 * Allocates device memory (with sgtp_track_upload, plans and the autotuner). */
int sgtp_ctx_create(sgtp_ctx **out, int max_agents_total, int max_N, int max_races, int max_track_nodes,
                    int max_K);
int sgtp_ctx_destroy(sgtp_ctx *ctx);
const char *sgtp_last_error(const sgtp_ctx *ctx);
/* The two-wave sweep variant (and the winner re-roll) pass states and controls between
 * waves of a workgroup through LDS and wait for each other with bounded polls.  Both
 * waits always end by construction; should one give up all the same, the kernel scores
 * that sample non-finite (so it is never selected) and raises a bit of the context's
 * status word (SGTP_STATUS_*).  sgtp_ctx_status waits for `stream`, copies the word to
 * *flags, clears it when `clear` != 0 and, when it is not zero, sets the text of
 * sgtp_last_error. */
int sgtp_ctx_status(sgtp_ctx *ctx, int *flags, int clear, void *stream);
/* Polls of those bounded waits before they give up (default 2^22, each about 256 cycles
 * apart); takes effect for calls and plans made afterwards.  For tests of the give-up
 * path: a limit of a few polls makes the waits give up while every kernel still ends. */
int sgtp_ctx_set_poll_limit(sgtp_ctx *ctx, int polls);
/* Allocate the per-tile partial sums of the path-integral update (params.update = 1):
 * (2 max_N + 2) floats per 256 samples of the context's capacity.  Synchronous; calls
 * with update = 1 fail with SGTP_EINVAL before it.  A choice record of that update
 * holds the lowest-score sample k, S_min as cost, viol = 0, and fallback = 1 when no
 * score was finite (the nominal is then kept). */
int sgtp_ctx_enable_path_integral(sgtp_ctx *ctx);

/* Upload the raceline G (Sec. II) as a HOST table nodes[n_nodes][8] of
 * (x, y, psi, kappa, w_L, w_R, v_ref, s) at increasing arc length s, psi
 * unwrapped.  closed != 0 joins node n-1 to node 0; one lap adds `length` to s
 * and `psi_lap` to psi.  Synchronous; replaces a track with the same id. */
int sgtp_track_upload(sgtp_ctx *ctx, int track_id, const double *nodes, int n_nodes, int closed, double length,
                      double psi_lap);

/* ---- planning ------------------------------------------------------------- */

/* One best response of vehicle `agent` in `phase` (0 = initialisation without
 * the game-aware cost, 1..L = sweeps, any larger value = a sweep with the
 * game-aware cost), with every other vehicle predicted by the noise-free rollout
 * of its nominal sequence.  Per-sample DEVICE outputs (each may be NULL):
 *   cost[K]   c of eq. (allc)              flags[K]  bit0 b, bit1 o, bit2 h = b*o,
 *   viol[K]   total violation nu                      bit3 search limit, bit4 non-finite
 *   x_final[K][6] world state after N steps  noise[K][N][2] the drawn perturbations
 * `out` (DEVICE, 1 entry) receives the selection.  u_nom is not modified.
 * Also writes race->s_abs. */
int sgtp_rollout_cost(sgtp_ctx *ctx, const sgtp_params *p, const sgtp_race *race, int agent, int phase,
                      float *cost, unsigned char *flags, float *viol, double *x_final, float *noise,
                      sgtp_choice *out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): sgtp_rollout_cost with the same
 * arguments, outputs and bits, whose kernels keep every scratch buffer (vehicle records,
 * raceline windows, reference states, predictions, selection keys and counters,
 * checkpoint slots, the call's descriptors) in one static device array of about 1.5 MB
 * per GPU instead of the context's workspace.  It calls no hipMalloc, hipFree or other
 * device-allocating routine, uses no host staging buffer (descriptors are kernel
 * arguments) and never synchronises; the context supplies the uploaded tracks, the
 * parameters' checks, the status word and the error text.  Limits: K <= SGTP_NOALLOC_MAX_K,
 * the library's vehicle and horizon limits (not the context's), update = 0 (feasibility
 * selection).  Larger inputs fail with SGTP_ESHAPE, other limits with SGTP_EINVAL, before
 * anything is enqueued.  The array is shared by every call on a GPU and keeps the last
 * call's contents (each call rewrites what it reads): calls that overlap on one GPU, on
 * any stream or context, race and must not be issued. */
#define SGTP_NOALLOC_MAX_K 65536
int sgtp_rollout_cost_noalloc(sgtp_ctx *ctx, const sgtp_params *p, const sgtp_race *race, int agent, int phase,
                              float *cost, unsigned char *flags, float *viol, double *x_final, float *noise,
                              sgtp_choice *out, void *stream);

/* One Jacobi sweep (phase 0..L) over all vehicles of all races, or the extra ego
 * response (phase = L+1, pass ego_only = 1): every participating vehicle answers
 * the noise-free rollouts of its opponents' current nominals, then adopts its
 * selected controls as its new nominal (u_nom) and writes traj.
 * out: DEVICE [sum n_agents] selections (entries of non-participating vehicles
 * are left untouched). */
int sgtp_ibr_sweep(sgtp_ctx *ctx, const sgtp_params *p, const sgtp_race *races, int n_races, int phase,
                   int ego_only, sgtp_choice *out, void *stream);

/* Alg. 1 for every race: initialisation, L_ibr sweeps, extra ego response.
 * Writes traj (final predictions), s_abs, u_apply (DEVICE [sum n][2], the first
 * control of each vehicle's final plan), trace (DEVICE [(L_ibr+2)][sum n]
 * selections, or NULL; non-participants untouched) and replaces u_nom by the
 * warm start of the next step (final plan shifted by one, last control repeated). */
int sgtp_plan_step(sgtp_ctx *ctx, const sgtp_params *p, const sgtp_race *races, int n_races, int L_ibr,
                   float *u_apply, sgtp_choice *trace, void *stream);

/* Closed loop: apply u (DEVICE [sum n][2]) to every vehicle for one interval
 * dt through the same vehicle model (float64 RK4), updating race->x. */
int sgtp_advance(sgtp_ctx *ctx, const sgtp_params *p, const sgtp_race *races, int n_races, const float *u,
                 void *stream);

/* ---- batched planning: plans, persistent sweeps, graphs, autotuning -------- */

/* A plan fixes a set of races (any mix of vehicle counts, K and N), L_ibr and the
 * output arrays, uploads their descriptors once and runs Alg. 1 for all races per
 * call: one setup launch, then one sweep launch per phase covering every vehicle
 * of every race.  Tiles of BLOCK = 256 samples (x samples_per_lane) are the unit
 * of work; small plans (at most 65536 samples over all vehicles, at most 3
 * opponents, one sample per lane) run 128-sample tiles with each sample on two waves
 * (dynamics on one; perturbation, projection and scoring on the other), or, where
 * those LDS rings do not fit, with each sample on a pair of lanes (dynamic model,
 * feasibility selection, at most 32768 samples); these plans run one workgroup per
 * tile (persistent is ignored).  Every variant gives the same per-sample bits.  A
 * persistent sweep keeps a fixed grid of workgroups that pull chunks of
 * tiles from 8 queues (vehicles assigned longest-first; a workgroup serves its own
 * queue first, then steals), re-staging LDS only when the vehicle changes.  With
 * use_graph the whole planning step is captured once into a hipGraph and replayed
 * by sgtp_plan_run.  Each run advances the races' plan_step (Philox counter word)
 * on the device; the race structs passed at creation are not read again (their
 * device arrays are: x, s_abs, v_scale, u_nom, traj). */
typedef struct sgtp_plan sgtp_plan;

typedef struct {
    int persistent;       /* 1 = persistent sweep with tile queues, 0 = one workgroup per tile */
    int blocks_per_cu;    /* persistent grid per CU (0 = occupancy limit) */
    int tiles_per_fetch;  /* tiles taken per queue fetch (persistent) */
    int samples_per_lane; /* samples evaluated in turn by each lane of a tile */
    int use_graph;        /* capture the planning step into a hipGraph */
    int include_advance;  /* append sgtp_advance with u_apply (closed loop inside the graph) */
} sgtp_plan_options;

/* u_apply: DEVICE [sum n][2]; trace: DEVICE [(L_ibr+2)][sum n] or NULL; opt NULL = defaults
 * (persistent, 1 tile per fetch, graph).  Allocates the plan's descriptor memory and,
 * with use_graph, captures on an internal stream (`stream` orders nothing here). */
int sgtp_plan_create(sgtp_ctx *ctx, const sgtp_params *p, const sgtp_race *races, int n_races, int L_ibr,
                     float *u_apply, sgtp_choice *trace, const sgtp_plan_options *opt, sgtp_plan **out,
                     void *stream);
/* One planning step of every race of the plan (graph replay or eager launches). */
int sgtp_plan_run(sgtp_plan *plan, void *stream);
/* Set every race's planning-step counter (synchronises the device). */
int sgtp_plan_set_step(sgtp_plan *plan, unsigned int plan_step);
/* Launch shape of the plan's all-vehicle sweeps; any pointer may be NULL. */
int sgtp_plan_info(const sgtp_plan *plan, int *grid_sweep, int *tiles_sweep, int *lds_bytes);
int sgtp_plan_destroy(sgtp_plan *plan);

/* Time candidate schedules (one workgroup per tile with 1 or 2 samples per lane;
 * persistent with 1, 2, 4 tiles per fetch at full or 2-per-CU occupancy) on real
 * planning steps of these races and return the fastest in *best (use_graph set) and
 * its median step time in *best_ms (may be NULL).  The races' u_nom and s_abs are saved
 * and restored; allocates temporary memory.  The result is kept in the context, keyed
 * by model, footprint discs, opponent-count bucket (1, 3, 9, 15), longest horizon,
 * floor(log2) of the total samples and of the race count, update rule and L_ibr; a later
 * call with the same key returns it at once (no timing, no allocation, nothing
 * enqueued). */
int sgtp_autotune(sgtp_ctx *ctx, const sgtp_params *p, const sgtp_race *races, int n_races, int L_ibr,
                  float *u_apply, sgtp_plan_options *best, double *best_ms, void *stream);
/* Drop every schedule sgtp_autotune has kept in this context. */
int sgtp_autotune_forget(sgtp_ctx *ctx);

/* ---- learned proposal (project extension; network in sgtp_mlp_*) ------------ */

#define SGTP_FEAT_DIM 50
#define SGTP_MLP_OUT 200 /* 4 values per step for a horizon of 50 */

/* Features of every vehicle of every race, DEVICE X[sum n][50] in slot order (race
 * by race): ego (d / half width, heading error to the raceline, v_x / 30, v_y / 5,
 * omega, (v_x - v_ref) / 10); the 4 opponents nearest in progress (s_j - s_i) / 20,
 * (d_j - d_i) / half width, heading difference, (v_x,j - v_x,i) / 10, v_y,j / 5, 1 -
 * zeros when absent; curvature x 20 at 5, 10, ..., 100 m ahead.  Runs the setup of
 * the races (writes s_abs). */
int sgtp_features(sgtp_ctx *ctx, const sgtp_params *p, const sgtp_race *races, int n_races, float *X,
                  void *stream);
/* Proposal tables from DEVICE network outputs out[sum n][ld_out] (per step: o0..o3):
 * mu_a = 4 o0, mu_d = 0.2 o1 (residual != 0: plus the vehicle's nominal control
 * u_nom at that step), sigma_a = sigma_a,plain exp(clamp(o2, -4, 1)),
 * sigma_d = sigma_d,plain exp(clamp(o3, -4, 1)); written to races[r].prop (races
 * with prop == NULL are skipped; 4 N <= ld_out is required). */
int sgtp_proposal_from_outputs(sgtp_ctx *ctx, const sgtp_params *p, const sgtp_race *races, int n_races,
                               const float *out, int ld_out, int residual, void *stream);

/* Proposal network: 50 -> 256 -> 256 -> 200, tanh-form GELU after the two hidden
 * layers.  Parameters are float32 packed as W1[50][256] b1[256] W2[256][256] b2[256]
 * W3[256][200] b3[200] (W stored [fan_in][fan_out]), sgtp_mlp_num_params() values.
 * Every product runs on BF16 matrix cores with float32 accumulation; master weights
 * and Adam moments stay float32.  A network owns workspaces for batches up to B_max
 * rows; calls on one network are ordered by the caller's stream and must not overlap. */
typedef struct sgtp_mlp sgtp_mlp;
int sgtp_mlp_create(int B_max, sgtp_mlp **out);
int sgtp_mlp_destroy(sgtp_mlp *m);
const char *sgtp_mlp_last_error(const sgtp_mlp *m);
int sgtp_mlp_num_params(void);
int sgtp_mlp_batch_max(const sgtp_mlp *m);
/* HOST params in; resets the Adam moments and step count.  Synchronous. */
int sgtp_mlp_set_params(sgtp_mlp *m, const float *host_params);
/* HOST params out (current master weights).  Synchronous. */
int sgtp_mlp_get_params(sgtp_mlp *m, float *host_params);
/* DEVICE X[B][50] -> DEVICE out[B][ld_out] (ld_out >= 200), float32. */
int sgtp_mlp_forward(sgtp_mlp *m, const float *X, int B, float *out, int ld_out, void *stream);
/* Mean over the B rows of the Gaussian negative log-likelihood of the DEVICE targets
 * U[B][N][2] (N <= 50 steps; the constant 0.5 log 2 pi per value is dropped) under the
 * proposal of DEVICE features X[B][50] (means 4 o0 and 0.2 o1, log scales
 * log sigma_plain + clamp(o, -4, 1)), and its gradient w.r.t. every parameter, kept
 * for sgtp_mlp_adam.  loss (DEVICE, 1 value) and grads (DEVICE, num_params values)
 * receive copies when not NULL. */
int sgtp_mlp_grad(sgtp_mlp *m, const float *X, const float *U, int B, int N, float sig_a, float sig_d, float *loss,
                  float *grads, void *stream);
/* The BF16 operands and float32 outputs of the last sgtp_mlp_grad call, B rows each,
 * copied into DEVICE dst (stream-ordered): SGTP_MLP_WS_H1 / _H2 the hidden activations
 * GELU(z) as BF16 [B][256]; _OUT the outputs float32 [B][256] (columns 200..255 zero);
 * _D3 the output gradient as BF16 [B][256] (columns of steps >= N and 200..255 zero);
 * _D2 / _D1 the gradients w.r.t. the pre-activations of layers 2 and 1 as BF16
 * [B][256]; _IDX the data-set rows the last sgtp_mlp_grad_sampled drew, int32 [B]
 * (SGTP_EINVAL after a plain sgtp_mlp_grad).  They stay until the next gradient call.
 * SGTP_EINVAL before the first gradient call or for an unknown tensor. */
#define SGTP_MLP_WS_H1 0
#define SGTP_MLP_WS_H2 1
#define SGTP_MLP_WS_OUT 2
#define SGTP_MLP_WS_D3 3
#define SGTP_MLP_WS_D2 4
#define SGTP_MLP_WS_D1 5
#define SGTP_MLP_WS_IDX 6
int sgtp_mlp_workspace(sgtp_mlp *m, int which, void *dst, void *stream);
/* sgtp_mlp_grad on B rows drawn on the device from a data set of M rows (a training
 * minibatch with no host step, so a captured training step draws new rows on every
 * replay): row b is data row floor(r M / 2^32), r the first word of Philox4x32-10 at
 * counter (b, t, 0, 0) with key (seed & 0xffffffff, seed >> 32), t the number of Adam
 * steps the network has taken.  X_all float32 [M][50] and U_all float32 [M][N][2]
 * (DEVICE, row-major); the rows are gathered inside (features straight to BF16) and the
 * gradient is that of sgtp_mlp_grad on them, bit for bit.  SGTP_ESHAPE for M outside
 * [1, 2^31 - 1], otherwise the errors of sgtp_mlp_grad. */
int sgtp_mlp_grad_sampled(sgtp_mlp *m, const float *X_all, const float *U_all, long long M, int B, int N,
                          unsigned long long seed, float sig_a, float sig_d, float *loss, float *grads, void *stream);
/* One Adam step with the last gradients (bias-corrected moments). */
int sgtp_mlp_adam(sgtp_mlp *m, float lr, float beta1, float beta2, float eps, void *stream);
/* One training step: sgtp_mlp_grad_sampled (loss, DEVICE, 1 value, when not NULL) followed
 * by sgtp_mlp_adam, with the same results bit for bit, but each parameter takes its Adam
 * step as soon as its gradient is summed, and up to 8192 rows the step count advances
 * inside the gradient's own launches (two launches fewer, the gradient not read back).
 * The gradient is still left for sgtp_mlp_workspace and a later sgtp_mlp_adam.  Errors as
 * sgtp_mlp_grad_sampled. */
int sgtp_mlp_train_step_sampled(sgtp_mlp *m, const float *X_all, const float *U_all, long long M, int B, int N,
                                unsigned long long seed, float sig_a, float sig_d, float lr, float beta1, float beta2,
                                float eps, float *loss, void *stream);
/* Make every planning step of `plan` compute the proposal tables itself: after the
 * setup, the features of every vehicle, the network's forward pass and the tables of
 * the races created with prop != NULL (their K_prop samples come from the proposal).
 * m == NULL detaches.  The network must hold batches of the plan's vehicle count and
 * every race with a table must have N <= 50; it must outlive the plan (or be
 * detached), and parameter updates take effect at the next run.  A graph plan is
 * captured again.  Allocates the feature and output buffers; synchronises. */
int sgtp_plan_set_proposal(sgtp_plan *plan, sgtp_mlp *m, int residual);
/* The network's matrix product on its own: C[m][n] = sum_k A(m, k) B(k, n) over DEVICE
 * BF16 operands with element strides (A(m, k) = A[m a_m + k a_k], B(k, n) =
 * B[k b_k + n b_n]), plus bias[n] when not NULL, into DEVICE float32 C[M][ldc]. */
int sgtp_gemm_bf16(const void *A, long long a_m, long long a_k, const void *B, long long b_k, long long b_n, int M,
                   int N, int K, const float *bias, float *C, long long ldc, void *stream);

/* ---- instrumentation ------------------------------------------------------ */

/* Time every sweep-kernel launch with HIP events on its stream (on != 0). */
int sgtp_set_timing(sgtp_ctx *ctx, int on);
/* Sum of measured sweep-kernel durations [ms] and launch count since the last
 * reset; synchronises the events.  reset != 0 clears the counters afterwards. */
int sgtp_sweep_stats(sgtp_ctx *ctx, double *total_ms, long long *launches, long long *sample_steps, int reset);

/* The Gaussian transform of the sampler on given Philox words: out[2 i], out[2 i + 1] =
 * the pair (z_a, z_delta) of (r_even[i], r_odd[i]) (all DEVICE, n pairs) -- u1 = (2 (r_even
 * >> 9) + 1) 2^-24, u2 = (r_odd >> 8) 2^-24, z = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2),
 * the float32 operation sequence of the samplers (Sec. III draws i.i.d. Gaussian
 * perturbations; the sequence is fixed so that they are reproducible bit for bit). */
int sgtp_gauss_pairs(const unsigned int *r_even, const unsigned int *r_odd, float *out, int n, void *stream);

/* A kernel with a known FP32 instruction mix, for checking hardware-counter formulas:
 * n_waves workgroups of one 64-lane wave; every lane runs `iters` iterations of exactly one
 * v_add_f32, v_mul_f32, v_fma_f32 and v_exp_f32 (scalar loop control), then three
 * v_add_f32 and one store to out[64 n_waves] (DEVICE).  Per wave: ADD_F32 = iters + 3,
 * MUL_F32 = FMA_F32 = TRANS_F32 = iters wave-instructions. */
int sgtp_counter_probe_fp32(float *out, int n_waves, int iters, void *stream);

/* Issue-class probe: n_blocks workgroups of 256 lanes (four waves); every lane runs `iters`
 * iterations of eight independent instructions of one kind, then seven v_add_f32 and one
 * store to out[256 n_blocks] (DEVICE).  kind 0: v_fma_f32 with vector operands, 1: v_fma_f32
 * with one scalar operand, 2: v_min_f32, 3: v_sin_f32, 4: v_mul_f32 with a literal, 5:
 * v_xor_b32, 6: v_cndmask_b32 on a scalar mask, 7: v_med3_f32, 8: v_mad_u64_u32.  Per wave:
 * SQ_INSTS_VALU = 8 iters + 7 (+ the store's address arithmetic).  Timed alone and read with SQ_ACTIVE_INST_VALU2 (the issue cycles in which a
 * SIMD issued two VALU instructions), it shows which instruction forms are paired across
 * waves.  Returns SGTP_EINVAL for a kind outside 0..8. */
int sgtp_issue_probe(float *out, int kind, int n_blocks, int iters, void *stream);

int sgtp_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SGTP_H */
