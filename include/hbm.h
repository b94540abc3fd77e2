/*
 * hbm.h -- C ABI of the MI355X (gfx950) Metropolis-within-Gibbs sampler for
 * single-plate hierarchical Bayesian models.
 *
 * Method (Szalai-Gindl, Loredo, Kelly, Csabai, Budavari, Dobos -- CUDAHM):
 * alternate (Sec. 2.1, eqs 2.4/2.5)
 *   (a) a robust adaptive Metropolis (RAM) update of every object's latent
 *       vector chi_i given the population parameters theta (Sec. 2.2,
 *       eq 2.6), the objects being conditionally independent, and
 *   (b) a Metropolis-Hastings step on theta that consumes the N-term
 *       population log-likelihood sum_i log f(chi_i; theta) (Sec. 2.2), less
 *       N ln Z(theta) for flux-selected catalogs (eqs 4.3/4.4, 5.10).
 *
 * Every step runs in the library's HIP kernels.  The caller owns the latent
 * state and the data (device buffers it allocates, e.g. torch tensors); the
 * library owns only its scratch (per-object derived constants, reduction
 * partials, quadrature tables, the theta states and their traces), allocated
 * when a context is created and freed by destroy_chains.
 *
 * Pools.  A context is a pool of n_slots slots over packed buffers of
 * `capacity` object positions.  A loaded slot holds one dataset (one
 * catalog with its own seed, theta chain and configuration) whose objects
 * occupy positions [obj_start, obj_start + N) of every buffer, obj_start a
 * multiple of 256.  Every launch advances all active slots together,
 * covering slots and 256-object tiles up to the last loaded slot and the
 * last occupied tile (so placing datasets low keeps launches small); a
 * slot's chain is bit-identical to the same dataset run alone, wherever it
 * sits.  init_chains makes a one-slot pool (capacity N, obj_start 0), and the
 * functions below then behave as for a single dataset.  init_batch packs
 * datasets back to back; create_pool / load_datasets / unload_dataset let a
 * scheduler admit and retire datasets between launches.
 *
 * Conventions for every function below.
 *   - Return value: HBM_OK (0) or a negative hbm_status.  No exception or
 *     abort crosses the ABI.  last_error() gives a message for the last
 *     failure on a context.
 *   - A validation failure (HBM_EINVAL, HBM_ENOSPACE) leaves the context
 *     unchanged.  A HIP failure (HBM_EHIP) poisons the context: every later
 *     call except last_error and destroy_chains returns HBM_ESTATE.
 *   - Work is enqueued on the hip stream given when the context was
 *     created (init_chains, init_batch, create_pool).  Calls that
 *     return host values synchronise that stream; the others are
 *     asynchronous.  A context is not thread-safe; distinct contexts on
 *     distinct streams may run concurrently.
 *   - Layouts are structure-of-arrays: component j of object position i
 *     sits at [j * C + i], C = the pool's capacity (N for init_chains).
 *     Real arrays hold float for HBM_FP32 and double for HBM_FP64 (the
 *     per-object precision).  Per-slot host arrays are indexed by slot.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key = the
 *     dataset's seed and counter = (object index within the dataset, sweep,
 *     tag, block); tag 0 = latent RAM step, 1 = theta proposal, 2 = theta
 *     accept.  A chain is a pure function of (data, configuration, seed),
 *     independent of launch shape and of its slot and position in a pool.
 */
#ifndef HBM_H
#define HBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define HBM_API __attribute__((visibility("default")))
#else
#define HBM_API
#endif

typedef struct hbm_ctx hbm_ctx;
typedef int32_t hbm_status;

#define HBM_OK        0
#define HBM_EINVAL   -1  /* bad argument, shape or NULL pointer */
#define HBM_ENOMEM   -2  /* device allocation failed */
#define HBM_EHIP     -3  /* HIP runtime error; the context is poisoned */
#define HBM_EDOMAIN  -4  /* non-finite log density, or theta outside the prior support */
#define HBM_ESTATE   -5  /* poisoned context, or calls in the wrong order */
#define HBM_ENOSPACE -6  /* sample store full */

/* Models.  Latent coordinates, data columns and theta:
 *  HBM_NORMAL_NORMAL_1D (Sec. 3 with one heteroscedastic component):
 *      chi = latent value; data (y_i, sigma_i); theta = (mu, ln tau);
 *      prior flat in mu, uniform in tau > 0.  Per-object precision FP64.
 *  HBM_GAMMA_LF_1D (Sec. 4-5, gamma = BB1 with l -> 0, Appendix B):
 *      chi = ln L; data (Fhat_i, k_i = ln 4 pi r_i^2); theta = (beta, ln L*),
 *      L ~ Gamma(beta + 1, L*); prior 1/(1+beta^2) on -1 < beta < 0, flat
 *      in ln L*; selection by Fhat > F_th with noise sigma_F.  FP32.
 *  HBM_GAMMA_LF_COLOR_3D: chi = (ln L, ln r, c); data (Fhat_i, rhat_i, chat_i);
 *      theta = (beta, ln L*, a, b, s); c ~ N(a + b ln L, s^2), r with density
 *      3 r^2 / rmax^3 on (0, rmax]; rhat ~ N(r, (f_r rhat)^2),
 *      chat ~ N(c, sigma_c^2); prior as 1-D plus flat a, b and uniform s > 0.  FP32.
 *  HBM_NORMAL_NORMAL_3D (the paper's Sec. 3 instance): chi in R^3,
 *      chi ~ MVN(mu, C_pop), y_ij ~ N(chi_ij, sigma_j^2), C_pop and sigma
 *      known; theta = mu, flat prior.  FP64.
 *  HBM_BB1_LF (the paper's Sec. 5 case study, Appendix C): chi = ln L;
 *      data (Fhat_i, k_i = ln r_i^2) with L in units of a reference scale,
 *      r in units of rmax and F = L / r^2; theta = (beta, ln l, ln u),
 *      f(L) = C / u (1 - e^{-L/l}) (L/u)^beta e^{-L/u} (break-by-one PDF);
 *      Fhat ~ N(F, sigma0^2 + (alpha F)^2) with its normaliser; selection
 *      by Fhat > F_th; prior l / (1 + beta^2) in (beta, ln l, ln u) on
 *      -2 < beta < 0, l < u (eq 5.5).  FP32.
 * model_consts: LF models [0] F_th, [1] sigma_F, [2] rmax, [3] centre ln L0
 * of the ln L quadrature interval [ln L0 - 30, ln L0 + ln 40], [4] f_r,
 * [5] sigma_c.  NN3D: [0..5] lower triangle of C_pop (row-major),
 * [6..8] sigma_j.  NN1D: unused.  BB1: [0] F_th, [1] sigma0, [2] alpha,
 * [3] ln l and [4] ln u of a reference PDF (the selection quadrature runs
 * over ln L in [ln l - 80, ln u + ln 40]). */
#define HBM_NORMAL_NORMAL_1D  1
#define HBM_GAMMA_LF_1D       2
#define HBM_GAMMA_LF_COLOR_3D 3
#define HBM_NORMAL_NORMAL_3D  4
#define HBM_BB1_LF            5

#define HBM_FP64 1
#define HBM_FP32 2

/* How run_cycles issues fused cycles (set_cycle_mode). */
#define HBM_CYCLES_AUTO  0  /* one persistent launch where possible, else graphs */
#define HBM_CYCLES_GRAPH 1  /* always graphs (or plain launches) */
#define HBM_CYCLES_FUSED 2  /* graphs of fused cycles (one launch per cycle) where possible */

typedef struct hbm_config {
    int32_t model;               /* HBM_* model id */
    int32_t precision;           /* HBM_FP64 or HBM_FP32; must match the model */
    int64_t n_objects;           /* N >= 1 */
    uint64_t seed;               /* Philox key */
    double target_accept;        /* alpha* of the latent RAM (paper default 0.4) */
    double eta_exponent;         /* gamma in eta_n = n^-gamma, 0.5 < gamma <= 1 (paper 2/3) */
    double s0;                   /* initial latent factor S_1 = s0 I (paper: I) */
    double theta_target_accept;  /* alpha* of the theta random walk's RAM */
    int32_t adapt_theta;         /* 1: RAM-adapt the theta proposal factor; 0: keep it */
    int32_t n_quad;              /* Gauss-Legendre nodes of the selection normaliser (LF: 16..4096) */
    int32_t thin_chi;            /* latent snapshot after every sweep k with k % thin_chi == 0; 0: none */
    int32_t tiles_per_group;     /* launch shape: 256-object tiles per sweep workgroup, 1, 2 or 4 (0 = 1);
                                    init_chains / init_batch take it from (the first) config */
    int32_t theta_substeps;      /* 0: one theta step per cycle from the N-term sums of the proposal
                                    (any model); K in 1..64: K Metropolis steps on theta per cycle
                                    from the sweep's sufficient statistics (exponential-family
                                    populations: both normal-normal and both gamma-LF models), sub-step
                                    j of cycle k drawing Philox blocks (j, k, 1, b) and (j, k, 2, 0);
                                    K = 1 makes the same chain as 0 up to rounding of the log ratio.
                                    Every dataset of a context uses 0, or every one K >= 1. */
    int32_t snap_rows;           /* init_chains / init_batch: rows of chi_samples for this dataset
                                    (0: max_cycles / thin_chi, every snapshot of the run; fewer rows
                                    make a ring for run_cycles_streamed) */
    int64_t max_cycles;          /* capacity of the theta trace (and bound on snapshots) */
    double theta_chol0[25];      /* initial theta proposal factor, p x p lower, row-major */
    double model_consts[16];
} hbm_config;

typedef struct hbm_buffers {
    const void *data;   /* [m][C] model data (device), read only */
    void *chi;          /* [d][C] latents (device), read/write */
    void *chol;         /* [d(d+1)/2][C] packed lower RAM factors, row-major (0,0),(1,0),(1,1),... */
    uint32_t *acc;      /* [C] per-object accepted-move counters (device) */
    void *chi_samples;  /* [snap_rows][d][C] latent snapshots (device), or NULL */
} hbm_buffers;

typedef struct hbm_pool_config {
    int32_t model;               /* HBM_* model id shared by every slot */
    int32_t precision;           /* must match the model */
    int32_t n_slots;             /* datasets resident at once, 1..65535 */
    int32_t n_quad;              /* LF: Gauss-Legendre nodes of every slot (16..4096) */
    int64_t capacity;            /* C: object positions, the stride of every buffer (<= 2^31 - 257) */
    int64_t max_cycles;          /* theta trace rows per slot */
    int64_t snap_rows;           /* rows of chi_samples (0 when NULL) */
    int32_t tiles_per_group;     /* launch shape: tiles per sweep workgroup, 1, 2 or 4 (0 = 1) */
    int32_t stats_theta;         /* 1: every dataset takes its theta steps from sufficient statistics
                                    (its theta_substeps >= 1); 0: from the N-term sums (theta_substeps 0) */
} hbm_pool_config;

/* Create a sampler (Sec. 2.2: "X_1 with pi(X_1) > 0, S_1 = I").
 * chi0_host: [d][N] starting latents (copied into buffers->chi), or NULL to
 * keep what buffers->chi already holds.  theta0: [p] starting theta (host).
 * Sets chol = s0 I and acc = 0, builds the selection tables, evaluates
 * Z(theta0), and checks that every log pi_i(chi0_i) is finite
 * (HBM_EDOMAIN otherwise, first bad index in last_error) and theta0 is in
 * the prior support (HBM_EDOMAIN).  hip_stream: a hipStream_t or NULL for
 * the default stream.  On success *out owns library scratch. */
HBM_API hbm_status init_chains(const hbm_config *config, const hbm_buffers *buffers, const double *chi0_host,
                       const double *theta0, void *hip_stream, hbm_ctx **out);

/* A batch of n_datasets catalogs of one model, advanced together (one
 * launch per sweep for all of them).  Dataset j occupies positions
 * [o_j, o_j + N_j) with o_0 = 0 and o_{j+1} = o_j + 256 ceil(N_j / 256); the
 * capacity C is o_last + N_last.  The caller fills data and chi at those
 * positions before the call.  configs[j] carries N_j, its seed and every
 * other setting; model, precision and n_quad must agree.  theta0:
 * [n_datasets][p].  Datasets sit in slots 0..n_datasets-1.  Fails as
 * init_chains does, naming the first bad dataset. */
HBM_API hbm_status init_batch(int32_t n_datasets, const hbm_config *configs, const hbm_buffers *buffers,
                              const double *theta0, void *hip_stream, hbm_ctx **out);

/* An empty pool (every slot free) over the caller's packed buffers. */
HBM_API hbm_status create_pool(const hbm_pool_config *pool, const hbm_buffers *buffers, void *hip_stream,
                               hbm_ctx **out);

/* Load count datasets into free slots: dataset q goes to slots[q] at
 * positions [obj_start[q], obj_start[q] + N_q), obj_start[q] a multiple of
 * 256, inside the capacity and disjoint from every loaded dataset.  The
 * caller has written its data and starting latents there.  theta0:
 * [count][p].  budgets (nullable): theta steps after which the dataset
 * stops (0 = no limit, at most its max_cycles); a stopped dataset keeps its
 * samples until unloaded.  Initialises each dataset as init_chains does;
 * on failure no slot is loaded.  Synchronous. */
HBM_API hbm_status load_datasets(hbm_ctx *ctx, int32_t count, const int32_t *slots, const int64_t *obj_start,
                                 const hbm_config *configs, const double *theta0, const int64_t *budgets);

/* Free a slot and its object range (its samples are no longer readable).
 * Synchronous. */
HBM_API hbm_status unload_dataset(hbm_ctx *ctx, int32_t slot);

/* Host-side state of a slot, without touching the device: out[0] loaded,
 * out[1] active (loaded, budget not spent), out[2] sweeps done, out[3]
 * theta steps done, out[4] obj_start, out[5] N. */
HBM_API hbm_status slot_info(hbm_ctx *ctx, int32_t slot, int64_t out[6]);

/* n_sweeps RAM sweeps of all latents of every active slot at its current
 * theta (eq 2.4, eq 2.6).
 * Sweep k (1-based, counted over the context's life) draws block
 * (i, k, 0, 0) for object i, proposes Y = X + S U with U ~ N(0, I_d),
 * accepts when ln u < log pi(Y) - log pi(X), and adapts S with
 * eta = (k+1)^-gamma.  Each sweep also reduces, in FP64 and in a fixed
 * order, sum_i log f(chi_i; theta) and sum_i [log f(chi_i; theta') -
 * log f(chi_i; theta)] for the pending proposal theta', plus Z(theta'),
 * for the next theta_step.  out_accept_rate (nullable): [n_slots] mean
 * acceptance of the last sweep (NaN for inactive slots); non-NULL makes the
 * call synchronous. */
HBM_API hbm_status ram_sweep(hbm_ctx *ctx, int32_t n_sweeps, double *out_accept_rate);

/* sum_i log f(chi_i; theta) - N ln Z(theta) at the current latents, FP64
 * accumulation (the N-term sum a theta MH step consumes), for every loaded
 * slot.  theta: [n_slots][p] host; out: [n_slots] (NaN for free slots).
 * Synchronous. */
HBM_API hbm_status pop_loglik(hbm_ctx *ctx, const double *theta, double *out);

/* Marginal log-likelihood of theta with every object's latent integrated
 * out by quadrature instead of sampled (Sec. 6 proposes this for objects
 * with low-dimensional latents; conditional independence makes the N
 * integrals independent):
 *   out[j] = sum_i ln int l_i(chi) f(chi; theta_j) dchi - N ln Z(theta_j),
 * with f the model's population density in chi and ln l_i the member
 * log-likelihood as the sampler uses it: -z^2/2 for the normal-normal and
 * gamma LF models (z the datum's residual in its standard errors), and
 * -z^2/2 - ln sigma(F) for BB1; Z is the selection normaliser of
 * flux-limited catalogs (1 otherwise).  Models with a 1-D
 * latent only (normal-normal 1-D, gamma LF 1-D, BB1).  FP64 throughout.
 * slot: a loaded slot; its data are read from the context's data buffer.
 * theta: [n_theta][p] host, 1 <= n_theta <= 65535; out: [n_theta] host.
 * terms (nullable): DEVICE buffer of n_theta * N doubles receiving the
 * per-object log integrals, row j for theta_j.  Does not touch the chains.
 * HBM_EDOMAIN when some theta_j lies where the population density does not
 * exist (gamma LF: beta <= -1; BB1: beta <= -2); HBM_EINVAL for models with
 * latents of higher dimension.  Grows a device scratch area on first use
 * and when n_theta * N grows.  Synchronous. */
HBM_API hbm_status marginal_loglik(hbm_ctx *ctx, int32_t slot, int32_t n_theta, const double *theta, double *out,
                                   double *terms);

/* Bytes of the static device array behind marginal_loglik_noalloc. */
#define HBM_NOALLOC_SCRATCH_BYTES (8u << 20)

/* marginal_loglik for callers that cannot allocate device memory (serving
 * loops that must not allocate per request, harnesses that forbid
 * hipMalloc): the same arguments, checks, kernels and results, bit for bit,
 * but no device allocation in the call -- its scratch is a static device
 * array of HBM_NOALLOC_SCRATCH_BYTES (8 MiB), which each device holds from
 * the first context created on it until the process ends.  The array keeps
 * the node rule (8,448 bytes, written once per device when that first
 * context is created) and then one call's working set of
 *   8 * n_theta * (p + 9 + ceil(N / 32))  bytes
 * (N the slot's object count): theta rows, results, workgroup partial sums
 * and per-row scalars, every word written by the call before it is read.
 * HBM_EINVAL, with the sizes in last_error, when that exceeds the array
 * (e.g. n_theta <= 111 at N = 300,000 and p = 2); HBM_ENOMEM when the array
 * could not be set up on the context's device.  Every call on one device
 * shares the array, which keeps the last call's contents: calls that
 * overlap on a device (contexts on different streams or threads) race, so
 * the caller must serialise them.  Kernel timing (kernel_timing) records
 * nothing for these calls.  Synchronous. */
HBM_API hbm_status marginal_loglik_noalloc(hbm_ctx *ctx, int32_t slot, int32_t n_theta, const double *theta,
                                           double *out, double *terms);


/* One Metropolis-Hastings step on theta of every active slot, for the
 * sweep just done: the
 * pending proposal theta' = theta + S_theta z (z from block (0, k, 1, b)) is
 * accepted when ln u < Delta (u from block (0, k, 2, 0)),
 * Delta = sum_i [log f(chi_i; theta') - log f(chi_i; theta)]
 *         - N [ln Z(theta') - ln Z(theta)] + ln p(theta') - ln p(theta),
 * Delta = -inf outside the prior support; then S_theta is RAM-adapted and
 * theta is appended to the trace.  Runs on the device.  Requires a
 * ram_sweep since the last theta_step (HBM_ESTATE otherwise); HBM_ENOSPACE
 * when the trace is full.  out_accepted (nullable): [n_slots], 1 if
 * accepted, 0 if not, -1 for slots that took no step.  Synchronous. */
HBM_API hbm_status theta_step(hbm_ctx *ctx, int32_t *out_accepted);

/* n_cycles full cycles (sweep then theta step) of every active slot, with
 * no host round trip between cycles.  Four ways to issue them, all giving
 * bit-identical chains (and the chain of alternating ram_sweep(1) and
 * theta_step):
 *   - use_graph == 0: per cycle, the sweep kernel and an epilogue kernel
 *     that reduces the tile partials and takes the theta step on the device;
 *   - use_graph != 0, a one-dataset context (init_chains) in mode
 *     HBM_CYCLES_AUTO, on a device that holds the grid: one persistent
 *     cooperative launch of 256 (or 128, 64) workgroups that stay resident
 *     for all n cycles, each sweeping a fixed set of tiles and taking the
 *     theta step itself after an exchange of the per-lane partial sums
 *     (no kernel boundary between cycles);
 *   - otherwise with use_graph != 0: replays of captured hipGraphs,
 *     floor(n / 32) of a 32-cycle graph and one of a graph of the remaining
 *     n mod 32 cycles (captured on first need, again when the remainder
 *     changes; prepare_cycles captures ahead); in mode HBM_CYCLES_FUSED the
 *     graphs hold fused cycles (set_cycle_mode).
 * A slot whose budget is reached stops at that cycle.  Asynchronous. */
HBM_API hbm_status run_cycles(hbm_ctx *ctx, int64_t n_cycles, int32_t use_graph);

/* Captures the graphs run_cycles(ctx, n_cycles, 1) would replay when it
 * uses graphs, without running any cycle, so that a later run_cycles of
 * that length spends no time on capture.  Synchronous. */
HBM_API hbm_status prepare_cycles(hbm_ctx *ctx, int64_t n_cycles);

/* mode: HBM_CYCLES_AUTO (default) lets run_cycles use the persistent
 * launch where it can; HBM_CYCLES_GRAPH restricts it to graphs of the
 * two-kernel cycle; HBM_CYCLES_FUSED makes the graphs hold fused cycles:
 * after the first sweep kernel, one launch per cycle in which every
 * workgroup takes the previous sweep's theta step itself (from that sweep's
 * tile partials, in the epilogue's fixed order) and then sweeps its tiles,
 * buffers alternating between cycles, and one epilogue at the end -- the
 * same chains, bit for bit.  In a context with several slots each tile's
 * workgroup takes its own dataset's theta step (one tile per workgroup,
 * whatever set_launch chose).  Changing to or from HBM_CYCLES_FUSED drops
 * the captured graphs.  Synchronous. */
HBM_API hbm_status set_cycle_mode(hbm_ctx *ctx, int32_t mode);

/* How run_cycles has issued cycles since the context was created:
 * out[0] graph replays, out[1] cycles inside those replays, out[2] cycles
 * issued as plain kernel launches, out[3] graphs captured, out[4]
 * persistent launches, out[5] cycles inside those. */
HBM_API hbm_status launch_counts(hbm_ctx *ctx, int64_t out[6]);

/* Receives streamed latent snapshots of one slot: its snapshots number
 * first .. first + count - 1 (snapshot r is the state after sweep
 * (r + 1) * thin_chi), as count x d x N values of the context's precision
 * (FP32 or FP64), row-major, bytes in all, in host memory valid only during
 * the call.  Return 0 to go on; any other value stops the run after the
 * chunk in flight (run_cycles_streamed then returns HBM_ESTATE). */
typedef int32_t (*hbm_snapshot_sink)(void *user, int32_t slot, int64_t first, int64_t count, const void *rows,
                                     int64_t bytes);

/* A ready sink: appends each batch of rows, as raw bytes, to the open file
 * descriptor held in user (cast from intptr_t).  Returns nonzero (stopping
 * the run) when the write fails. */
HBM_API int32_t fd_sink(void *user, int32_t slot, int64_t first, int64_t count, const void *rows, int64_t bytes);

/* run_cycles with every latent snapshot streamed to the host as it is taken
 * (the paper's compact-memory sampler, Appendix A, keeps samples off the
 * device the same way): chi_samples serves each slot as a ring of its
 * snap_cap rows, so a run of any length needs only
 * 2 * ceil(chunk_cycles / thin_chi) rows of device memory per slot instead
 * of max_cycles / thin_chi.  Cycles go in chunks of chunk_cycles (graph
 * replays, as run_cycles with use_graph); the copy of chunk c's rows into
 * pinned host memory runs on a second stream while chunk c + 1 computes, and
 * sink is called with chunk c's rows, on the calling thread, while chunk
 * c + 1 computes.  Chunk c + 2 waits (on the device) for chunk c's copy
 * before it overwrites those rows.  Slots with thin_chi = 0 stream nothing.
 * Same chain, bit for bit, as run_cycles.  HBM_EINVAL when a streaming
 * slot's ring is smaller than 2 * ceil(chunk_cycles / thin_chi) rows or
 * sink is NULL.  Allocates its pinned staging (2 chunks of rows) on each
 * call.  Synchronous: returns after the last rows were delivered. */
HBM_API hbm_status run_cycles_streamed(hbm_ctx *ctx, int64_t n_cycles, int32_t chunk_cycles, hbm_snapshot_sink sink,
                                       void *user);

/* Copy a slot's recorded samples to host.  theta_out: [count][p] rows
 * first..first+count-1 of its theta trace (or NULL).  chi_out: [count][d][N]
 * latent snapshots first..first+count-1 of its N objects, in the per-object
 * precision (or NULL).  With both NULL *n_written receives the number of
 * theta rows recorded.  Synchronous. */
HBM_API hbm_status get_samples(hbm_ctx *ctx, int32_t slot, int64_t first, int64_t count, double *theta_out,
                       void *chi_out, int64_t *n_written);

/* A slot's current theta [p], theta factor [p][p] (either nullable) and
 * sweeps done. */
HBM_API hbm_status get_theta(hbm_ctx *ctx, int32_t slot, double *theta, double *chol_theta, int64_t *k);

/* Overwrite a slot's theta, its factor and its sweep counter k (lockstep
 * replay and resume).  The caller's latent buffers are taken as they are.
 * Recomputes Z(theta) and the pending proposal for sweep k + 1.
 * HBM_EDOMAIN when theta is outside the prior support. */
HBM_API hbm_status set_theta(hbm_ctx *ctx, int32_t slot, const double *theta, const double *chol_theta, int64_t k);

/* One sweep like ram_sweep that also writes, per object, in the per-object
 * precision: trace[0][i] = log pi_i(X), trace[1][i] = log pi_i(Y) (member
 * log likelihood plus log population density, with the constants of the
 * densities documented above), trace[2][i] = 1 if accepted else 0, and
 * trace[3 + j][i] = component j of the proposal Y; trace is a device buffer
 * [3 + d][C].  Synchronous. */
HBM_API hbm_status ram_sweep_trace(hbm_ctx *ctx, void *trace);

/* Checkpoint and resume of the library-held state: every slot's theta
 * chain (theta, S_theta, the pending proposal and its constants, the sweep
 * and theta-step counters, budgets) and its theta trace.  The latent
 * buffers are the caller's: save and restore them alongside.  get_state
 * with blob NULL returns the size in *size; a *size that is too small gives
 * HBM_ENOSPACE with the size needed; not allowed while a ram_sweep waits for
 * its theta_step (HBM_ESTATE).  set_state needs a context of the same shape
 * (model, slots, capacity, max_cycles) holding datasets at the same
 * positions (e.g. created by the same init_chains / init_batch / loads);
 * the datasets' data and configuration are not part of the blob.  A chain
 * resumed this way continues exactly as the saved one would have.
 * Synchronous. */
HBM_API hbm_status get_state(hbm_ctx *ctx, void *blob, size_t *size);
HBM_API hbm_status set_state(hbm_ctx *ctx, const void *blob, size_t size);

/* Statistics of a slot's last sweep and theta step: out[0] sum log f(chi; theta),
 * out[1] sum of per-object log f differences at theta', out[2] ln Z(theta),
 * out[3] ln Z(theta'), out[4] Delta of the last theta step, out[5] its
 * acceptance probability, out[6] accepted latent moves of the last sweep,
 * out[7] theta accepted (0/1).  Synchronous. */
HBM_API hbm_status get_stats(hbm_ctx *ctx, int32_t slot, double out[8]);

/* Launch shape of the sweep kernel: 256-object tiles per workgroup (1, 2 or
 * 4).  Every tile is still reduced on its own in a fixed order, so results
 * do not depend on the shape.  The sweep kernel of the two-kernel cycle
 * steps a workgroup's tiles with 256 threads, one object of each tile per
 * thread; the fused cycle (HBM_CYCLES_FUSED) with 2 or 4 tiles runs
 * 512- or 1024-thread workgroups, one object per thread (256 threads with
 * theta sub-steps).  Drops the captured graph.  Synchronous. */
HBM_API hbm_status set_launch(hbm_ctx *ctx, int32_t tiles_per_group);

/* Occupancy of the sweep kernel: at most groups_per_cu of its 256-thread
 * workgroups resident per compute unit (so at most groups_per_cu waves per
 * SIMD), enforced by dynamic LDS the kernel does not use; 0 removes the cap
 * (as many as registers and LDS allow: 8 per SIMD for the sweep kernels).
 * Results do not depend on it.  Drops the captured graphs.  Synchronous. */
HBM_API hbm_status set_occupancy(hbm_ctx *ctx, int32_t groups_per_cu);

/* Autotuner of how cycles run.  HBM_TUNE_CANDIDATES candidates, in this
 * order: the two-kernel cycle replayed from graphs with tiles per workgroup
 * 1, 2, 4 under no occupancy cap (candidates 0-2), a cap of 4 (3-5) and a
 * cap of 2 workgroups per compute unit (6-8); then the persistent launch
 * (9; one-dataset contexts in mode HBM_CYCLES_AUTO, else not timed); then
 * graphs of fused cycles with tiles per workgroup 1, 2, 4 and no cap
 * (10-12; contexts with several slots time candidate 10 only).  Each
 * runs 8 warm-up cycles then trial_cycles cycles timed by hipEvents on the
 * context's stream; the fastest is kept: its shape and cap, and the cycle
 * mode (HBM_CYCLES_AUTO when the persistent launch won, HBM_CYCLES_FUSED when
 * fused cycles did, else HBM_CYCLES_GRAPH).  The cycles are real cycles of every active slot
 * (HBM_TUNE_CANDIDATES (8 + trial_cycles) of them, counted against
 * max_cycles); results do not depend on the choice, so tuning during burn-in
 * changes no chain.  out_choice (nullable): [3] tiles per workgroup,
 * workgroups-per-CU cap (0: none), how cycles run (0: two-kernel graphs, 1:
 * persistent launch, 2: fused graphs); out_us (nullable):
 * [HBM_TUNE_CANDIDATES] microseconds per cycle (NaN: not timed).
 * Synchronous. */
#define HBM_TUNE_CANDIDATES 13
HBM_API hbm_status autotune(hbm_ctx *ctx, int32_t trial_cycles, int32_t out_choice[3],
                            double out_us[HBM_TUNE_CANDIDATES]);

/* Per-launch duration of the sweep, fused-cycle, persistent-cycle and
 * marginal kernels: when enabled, every launch of the sweep, fused or
 * marginal kernel carries a start and a stop hipEvent that the runtime
 * records from the dispatch itself (hipExtLaunchKernel), every persistent
 * launch is bracketed by events recorded on the stream, and run_cycles
 * issues plain launches where it would replay graphs (in mode
 * HBM_CYCLES_FUSED, the fused sequence, timing its fused kernels only).
 * read returns the launches timed and their mean duration in ms and resets
 * the counters.  Synchronous read. */
HBM_API hbm_status kernel_timing(hbm_ctx *ctx, int32_t enable);
HBM_API hbm_status read_kernel_timing(hbm_ctx *ctx, int64_t *n_launches, double *mean_ms);

/* Message of the last failure on ctx (or of the last failed init when ctx
 * is NULL); library-owned, valid until the next call on the context. */
HBM_API const char *last_error(const hbm_ctx *ctx);

/* Release the library's scratch; the caller's buffers are untouched. */
HBM_API void destroy_chains(hbm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* HBM_H */
