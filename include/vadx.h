/*
 * vadx.h -- C ABI of the MI355X TVB-AdEx sweep engine.
 *
 * The engine integrates many independent whole-brain networks at once, one
 * parameter combination per network ("instance"), as in the parameter sweeps
 * of van der Vlag et al., "Vast TVB parameter space exploration"
 * (arXiv:2311.13337), Section 2.3: each instance is a connectome of regions,
 * each region steps the second-order AdEx mean field of Section 2.1
 * (eq. 1-3: rates E, I, covariances C_ee, C_ei, C_ii, adaptation W_e, W_i)
 * plus Ornstein-Uhlenbeck noise (eq. 4), driven through the transfer function
 * of Section 2.2 (template + Table 1 threshold polynomial) by the delayed,
 * weighted excitatory rates of the other regions (eq. 5). After the run the
 * Pearson functional connectivity of the time-averaged rates (Section 2.4,
 * eq. 6) and summary statistics are formed per instance.
 *
 * Conventions
 *  - Every call returns a vadx_status; nothing throws across this boundary and
 *    nothing aborts. vadx_last_error() describes the last failure on a context.
 *  - Host arrays passed in are copied before the call returns (caller keeps
 *    ownership). Device pointers (workspace, outputs with where=VADX_DEVICE)
 *    are borrowed: the caller owns them and keeps them alive until the work
 *    that uses them has completed (vadx_sync).
 *  - Work is enqueued on the stream given to vadx_create (stream-ordered);
 *    reads with where=VADX_HOST synchronise that stream.
 *  - A context belongs to one device and one stream and is not thread-safe.
 *  - Results are a pure function of (model, connectome, parameters, run, seed,
 *    instance index): they do not depend on launch shapes or batch order.
 *  - Units: time in ms, rates in kHz inside the model (statistics report Hz),
 *    voltages in mV, conductances in nS, currents in pA, capacitance in pF,
 *    tract lengths in mm, conduction speeds in m/s (= mm/ms).
 */
#ifndef VADX_H
#define VADX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vadx_status;
enum {
    VADX_OK = 0,
    VADX_E_ARG = -1,         /* invalid argument (sizes, NaN/negative parameters, bad connectome) */
    VADX_E_OOM = -2,         /* workspace too small or a device allocation failed */
    VADX_E_HIP = -3,         /* a HIP runtime call failed */
    VADX_E_STATE = -4,       /* call out of order (e.g. integrate before set_batch) */
    VADX_E_NUMERIC = -5,     /* reserved */
    VADX_E_UNSUPPORTED = -6  /* request outside what the build supports (e.g. too many regions) */
};
enum { VADX_HOST = 0, VADX_DEVICE = 1 };
enum { VADX_PRESET_LITERATURE_B = 0, VADX_PRESET_PAPER_T1 = 1 };
enum { VADX_HEUN = 0, VADX_EULER = 1 };
/* per-instance flag bits in vadx_stats.flags */
enum { VADX_FLAG_NONFINITE = 1u, VADX_FLAG_CLAMP = 2u, VADX_FLAG_ZERO_VAR = 4u };

typedef struct vadx_ctx vadx_ctx;

/* Model constants shared by all instances (Section 2.1-2.2). P_e / P_i are
 * the ten threshold-polynomial coefficients of Table 1 (mV) in the table's
 * column order for the excitatory (RS) and inhibitory (FS) cell.
 * K_e, K_i: number of excitatory / inhibitory synapses per neuron (the
 * weights of the excitatory and inhibitory input rates). N_e, N_i: population
 * sizes in the finite-size term of eq. (2). cF_mn: constant drive to the
 * n-input of population m's transfer function (eq. 5). sigma_OU, w_noise: the
 * OU amplitude of eq. (4) and its weight on the excitatory input. x_floor:
 * minimum input rate of the transfer function. rate_max: upper clamp of E, I. */
typedef struct vadx_model {
    double C_m, g_L, E_e, E_i, Q_e, Q_i, tau_e, tau_i, K_e, K_i, N_e, N_i, T;
    double E_L_e, E_L_i, tau_w_e, tau_w_i, b_i, a_i;
    double cF_ee, cF_ei, cF_ie, cF_ii;
    double tau_OU, sigma_OU, w_noise;
    double muV0, dmuV0, sV0, dsV0, tN0, dtN0;
    double rate_max, E_init, I_init, x_floor;
    double P_e[10], P_i[10];
} vadx_model;

/* One run over the current batch. Samples are means of tavg_steps steps; the
 * first transient_steps are left out of the FC and statistics. seed keys the
 * Philox noise together with the instance index. n_trace_steps > 0 records the
 * full state after each of the first n_trace_steps steps for the instances
 * chosen with vadx_set_trace. noise_off = 1 runs the noise-free system. */
typedef struct vadx_run {
    double dt_ms;
    int64_t n_steps, transient_steps, tavg_steps, n_trace_steps;
    uint32_t seed;
    int32_t integrator;   /* VADX_HEUN (default) or VADX_EULER */
    int32_t noise_off;
    int32_t chunk_steps;  /* steps per kernel launch; 0 = library default (the whole
                             run with the persistent queue, 10000 otherwise) */
    double fc_min_std;    /* kHz; a region whose rate std over the samples is
                             below it is silent: zero variance and covariances,
                             FC row 0 (diagonal 1), VADX_FLAG_ZERO_VAR set */
} vadx_run;

/* Summary statistics of one instance (definitions in vadx_read_stats). */
typedef struct vadx_stats {
    float fc_mean, fc_std, fc_sc_corr, rate_mean_hz, rate_std_hz, sync_index;
    uint32_t flags;
    float fc_fit;         /* Pearson correlation of FC_kl with the connectome's reference FC
                             over k < l (vadx_set_reference_fc); 0 without a reference */
} vadx_stats;

/* Creates a context on HIP device `device` enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the null stream). The stream is borrowed. */
vadx_status vadx_create(int device, void *hip_stream, vadx_ctx **out);
void vadx_destroy(vadx_ctx *ctx);
/* Text of the last error on ctx (valid until the next call on ctx); never NULL. */
const char *vadx_last_error(const vadx_ctx *ctx);

/* Fills *out with a preset: VADX_PRESET_PAPER_T1 uses Table 1 as printed;
 * VADX_PRESET_LITERATURE_B reads three entries of Table 1 as misprints
 * (RS P0 = -49.8, FS P_muV = 4.0, both P_sigmaVtauN with opposite sign). */
vadx_status vadx_model_defaults(int preset, vadx_model *out);
/* Sets the model for subsequent runs (copied). */
vadx_status vadx_set_model(vadx_ctx *ctx, const vadx_model *model);

/* Registers a connectome of n regions (Section 2.4, "-cf"): raw weights w
 * [n*n] row-major (non-negative, zero diagonal) and tract lengths [n*n] in mm
 * (positive where w > 0). Weights are row-normalised on the device
 * (W_kj = w_kj / sum_j w_kj; all-zero rows stay zero); the raw w is the
 * structural connectivity used for the FC-SC correlation. 2 <= n <= 512 (one
 * lane per region, an instance within one workgroup); larger n gives
 * VADX_E_UNSUPPORTED.
 * *conn_id receives the index used by vadx_set_batch. */
vadx_status vadx_add_connectome(vadx_ctx *ctx, int32_t n, const double *weights,
                                const double *tract_mm, int32_t *conn_id);

/* Sets the batch: one parameter combination per instance (Section 2.3) --
 * global coupling S >= 0, spike-frequency adaptation b_e (pA), subthreshold
 * adaptation a_e (nS), conduction speed v > 0 (m/s) -- and the connectome of
 * each instance (NULL = all 0). Host arrays of n_inst entries, copied. */
vadx_status vadx_set_batch(vadx_ctx *ctx, int64_t n_inst, const float *S, const float *b_e,
                           const float *a_e, const float *v_mps, const int32_t *conn_id);

/* Sets the Philox key word of each instance of the current batch (n must equal
 * the batch size; host array, copied). The noise of eq. (4) for instance i is
 * drawn from the stream keyed by (run seed, keys[i]); set_batch resets the
 * keys to the batch indices 0..n-1. Giving a sub-batch the indices its points
 * have in a larger sweep reproduces exactly the runs of that sweep. */
vadx_status vadx_set_noise_keys(vadx_ctx *ctx, int64_t n, const uint32_t *keys);

/* Further sweep axes of the paper's vast exploration (Table 4) as
 * per-instance values of model parameters: the noise weight w_noise (>= 0),
 * the excitatory adaptation time constant tau_w_e (ms, > 0) and the external
 * drives cF_ee, cF_ei, cF_ie, cF_ii (kHz, >= 0). values: host array of n =
 * batch-size doubles (copied), or NULL to use the model's value for every
 * instance; vadx_set_batch resets all of them to the model's. Instances whose
 * populations see different drives (cF_ee != cF_ie or cF_ei != cF_ii) run the
 * general transfer-function path; results of the others do not change.
 * Takes effect at the next vadx_plan. */
enum { VADX_P_W_NOISE = 0, VADX_P_TAU_W_E = 1, VADX_P_CF_EE = 2, VADX_P_CF_EI = 3,
       VADX_P_CF_IE = 4, VADX_P_CF_II = 5 };
vadx_status vadx_set_instance_param(vadx_ctx *ctx, int32_t param, int64_t n, const double *values);

/* Chooses up to 1024 instances whose first run->n_trace_steps states are
 * recorded (trace slot i = inst[i]). n = 0 clears the selection. */
vadx_status vadx_set_trace(vadx_ctx *ctx, int64_t n, const int64_t *inst);

/* Bytes of device workspace vadx_integrate needs for `run` on the current
 * batch: state, delay rings, rate samples, traces, FC and statistics. */
vadx_status vadx_plan(vadx_ctx *ctx, const vadx_run *run, size_t *workspace_bytes);

/* Integrates every instance of the batch for run->n_steps steps of
 * stochastic Heun (or Euler), then forms the FC and the statistics.
 * workspace: device memory of at least the planned size, 256-byte aligned,
 * owned by the caller; results live there until the next integrate. */
vadx_status vadx_integrate(vadx_ctx *ctx, const vadx_run *run, void *workspace,
                           size_t workspace_bytes);

/* Waits for all work of ctx. After a run, reports VADX_E_HIP if one of the
 * integration's bounded waits timed out (the run's results are then void):
 * a workgroup's wait for the previous chunk of its group, or a wave's wait
 * for the previous block of the waves sharing its instances. */
vadx_status vadx_sync(vadx_ctx *ctx);

/* Reads results of the last vadx_integrate. `out` is host (VADX_HOST) or
 * device (VADX_DEVICE) memory owned by the caller.
 *  vadx_read_stats: `count` vadx_stats from instance `first`. fc_mean/fc_std:
 *    mean and population std of FC_kl over k<l; fc_sc_corr: Pearson
 *    correlation of FC_kl with the raw weights w_kl over k<l; rate_mean_hz:
 *    mean of E over regions and samples; rate_std_hz: mean over regions of
 *    the temporal std of E; sync_index: sqrt(var_t(mean_k E_k) /
 *    mean_k var_t(E_k)). flags: VADX_FLAG_* bits.
 *  vadx_read_fc: the n x n FC matrix (float) of instance `inst`.
 *  vadx_read_samples: the [n_samples][n] rate samples (kHz) of `inst`.
 *  vadx_read_state: the final [8][n] state of `inst` (E, I, C_ee, C_ei, C_ii,
 *    W_e, W_i, OU) as doubles: the drift is evaluated in single precision and
 *    the state accumulated in double precision.
 *  vadx_read_trace: [n_trace_steps][8][n] states of trace slot `slot`. */
vadx_status vadx_read_stats(vadx_ctx *ctx, int64_t first, int64_t count, vadx_stats *out,
                            int32_t where);
vadx_status vadx_read_fc(vadx_ctx *ctx, int64_t inst, float *out, int32_t where);
vadx_status vadx_read_samples(vadx_ctx *ctx, int64_t inst, float *out, int32_t where);
vadx_status vadx_read_state(vadx_ctx *ctx, int64_t inst, double *out, int32_t where);
vadx_status vadx_read_trace(vadx_ctx *ctx, int64_t slot, float *out, int32_t where);

/* Reference FC of connectome conn_id (Section 2.4, "-ff"): host array fc
 * [n*n] (row-major, copied; finite), or NULL to remove it. Each instance on
 * that connectome then reports vadx_stats.fc_fit, the Pearson correlation of
 * its FC with the reference over the pairs k < l (0 when either has no
 * variance) -- the fitness a grid search ranks (vadx_top_k). */
vadx_status vadx_set_reference_fc(vadx_ctx *ctx, int32_t conn_id, const float *fc);

/* Ranking of a sweep (the grid search's sort of fitness, Section 2.5, "-gs"):
 * of n device scores (FP32, not NaN), the k largest in decreasing order, ties
 * by increasing index. idx (device, k entries) receives the indices, val
 * (device, nullable) the scores. 0 <= k <= min(n, 1024). Synchronises the
 * context's stream. */
vadx_status vadx_top_k(vadx_ctx *ctx, const float *score, int64_t n, int32_t k, int64_t *idx,
                       float *val);

/* vadx_top_k for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * arguments and results, with its scratch (selection histogram, per-tile
 * counts and bases, the k candidate indices; 89 KB) in a fixed device array
 * that each GPU holds from vadx_create until the process ends. It calls no
 * allocator. At most 2^24 scores (VADX_E_UNSUPPORTED above). Calls that
 * overlap on one GPU share that array and race; every call clears what it
 * needs. Synchronises the context's stream. */
vadx_status vadx_top_k_noalloc(vadx_ctx *ctx, const float *score, int64_t n, int32_t k,
                               int64_t *idx, float *val);

/* Region count and number of post-transient samples of instance `inst` for
 * the last plan (sizes of the read_* outputs). */
vadx_status vadx_instance_shape(vadx_ctx *ctx, int64_t inst, int32_t *n_regions,
                                int64_t *n_samples);

/* Launch shape of the integration (takes effect at the next vadx_plan).
 * mode 0 (default): one persistent launch whose workgroups pull (group of
 * instances, chunk of item_steps steps) items from a queue, chunks of one
 * group in order, over the groups of every block length at once, so uneven
 * batches and grids larger than the GPU stay balanced and the run has a
 * single tail; mode 1: one workgroup per group, one launch per block length.
 * wg_instances caps the instances per workgroup (0 = as many as fit the lane
 * budget of their region count, vadx_class_lanes); item_steps 0 = 1000.
 * Results do not depend on the shape. */
vadx_status vadx_set_launch(vadx_ctx *ctx, int32_t mode, int32_t wg_instances, int32_t item_steps);

/* Lane budget of the workgroups holding instances of n_regions regions: each
 * packs floor(lanes / n_regions) instances (at least one) on consecutive
 * lanes. lanes in [64, 512] sets it, 0 returns it to the default (256), -1
 * leaves it; *current (nullable) receives the budget in effect. Takes effect
 * at the next vadx_plan; results do not depend on it. */
vadx_status vadx_class_lanes(vadx_ctx *ctx, int32_t n_regions, int32_t lanes, int32_t *current);

/* Register budget of the persistent integration kernel in waves per SIMD: 2
 * (one 512-lane or two 256-lane workgroups per CU; the default) or 3 (three
 * 256-lane workgroups per CU; registers spill inside the step loop, measured
 * about half as fast on 68-region sweeps). Takes effect at the next
 * vadx_plan; results do not depend on it. */
vadx_status vadx_set_waves_per_simd(vadx_ctx *ctx, int32_t waves);

/* Wave slack of the integration. The waves that hold an instance's regions
 * exchange delayed rates through its history ring once per block of steps.
 * 0 (the default): blocks of up to d_min + 1 steps (d_min: the instance's
 * shortest delay in steps), each reading what the other waves published by
 * the end of the previous block. 1: where half that bound still allows a
 * block of at least 12 steps, blocks of at most (d_min + 1) / 2 steps that
 * read only what was published two blocks back, so a wave may run one block
 * further ahead of the waves it shares instances with (the ring grows by one
 * block); other instances keep slack 0. slack in {0, 1} sets it, -1 leaves it;
 * *current (nullable) receives the setting in effect. Takes effect at the next
 * vadx_plan; results do not depend on it (the same sums in the same order). */
vadx_status vadx_wave_slack(vadx_ctx *ctx, int32_t slack, int32_t *current);

/* Autotuner of the launch shape for the current batch: times trial runs of
 * trial_steps steps (0 = 2000; no samples) of `run` in `ws` (device, at least
 * the size vadx_plan gave for `run`; its contents are overwritten) of the
 * persistent launch. Starting from 256-lane budgets with 2 waves per SIMD
 * and items of an eighth of the trial run (500..3000 steps), for wave slack 0
 * and 1 it tries each region-count
 * class's lane budgets in turn (64..512 lanes, one per distinct instance count
 * per workgroup; the other classes at their best so far), keeps the faster
 * slack, tries 3 waves per SIMD at the chosen budgets, then items of
 * 500..8000 steps over trial runs as long as `run` (at most
 * max(trial_steps, 60000) steps, so that the queue's tail weighs as in the
 * run), and keeps the fastest. With a cache_path (nullable) the
 * choice is read from / added to that JSON file, keyed by device, longest
 * block length (without slack) and the region-count mix; a cached choice is
 * applied without trials. *lanes (the widest class budget), *item_steps,
 * *waves (nullable) receive the choice; vadx_class_lanes and vadx_wave_slack
 * read the class budgets and the slack. Call vadx_plan again before
 * vadx_integrate. */
vadx_status vadx_autotune(vadx_ctx *ctx, const vadx_run *run, void *ws, size_t ws_bytes,
                          const char *cache_path, int32_t trial_steps, int32_t *lanes,
                          int32_t *item_steps, int32_t *waves);

/* Launch shape of the current plan: groups of instances, threads per
 * workgroup, workgroups launched (the persistent grid, or the most groups of
 * one launch) and the longest block of steps between two synchronisations of
 * an instance's waves. Each pointer nullable. */
vadx_status vadx_launch_info(vadx_ctx *ctx, int32_t *groups, int32_t *block_threads,
                             int32_t *grid, int32_t *steps_per_block);

/* Graph replay: with on = 1, vadx_integrate records the whole run (flag
 * clears, integration launches, FC) once into a HIP graph and replays it on
 * later calls with the same plan and workspace; the first call after
 * vadx_plan, a new workspace or vadx_set_graph re-records. Results are those
 * of the eager launches. Runs with timing enabled stay eager. Waits for the
 * context's stream. */
vadx_status vadx_set_graph(vadx_ctx *ctx, int32_t on);

/* Kernel timing: when enabled, HIP events on the context's stream bracket every
 * launch of the integration kernel; vadx_kernel_time reports their count and
 * summed duration (ms) since the last reset, and the duration of the FC
 * kernel launches. */
vadx_status vadx_enable_timing(vadx_ctx *ctx, int32_t on);
vadx_status vadx_kernel_time(vadx_ctx *ctx, int64_t *n_integrate_launches, double *integrate_ms,
                             int64_t *n_fc_launches, double *fc_ms);

/* ---------------------------------------------------------------------------
 * Surrogate network: a 4 -> 128 -> 128 -> 6 MLP with GELU (exact erf form)
 * mapping a sweep point (S, b_e, a_e, v) to the six statistics of
 * vadx_read_stats, trained on the GPU by this library's kernels so a dense grid
 * can be screened before simulating (the learning-guided exploration the
 * paper's discussion proposes; the plain simulation stays the reference).
 * Inputs are min-max scaled to [-1, 1] with cfg.x_lo / x_hi; targets are
 * z-scored with the network's target normalisation. Matrix products use
 * bfloat16 operands with FP32 accumulation (MFMA for the 128 x 128 products);
 * Adam (Kingma & Ba) in FP32. Parameter vector (17926 floats): W1 [128][4],
 * b1 [128], W2 [128][128], b2 [128], W3 [6][128], b3 [6], row-major,
 * concatenated. Data pointers X [n][4] and Y [n][6] are device arrays (FP32);
 * calls are ordered on cfg.hip_stream. */
typedef struct vadx_mlp vadx_mlp;
typedef struct vadx_mlp_cfg {
    float x_lo[4], x_hi[4];
    float lr, beta1, beta2, eps;
    void *hip_stream;
} vadx_mlp_cfg;

/* init_params: host array of 17926 floats (copied). */
vadx_status vadx_mlp_create(vadx_ctx *ctx, const vadx_mlp_cfg *cfg, const float *init_params,
                            vadx_mlp **out);
void vadx_mlp_destroy(vadx_mlp *mlp);
const char *vadx_mlp_last_error(const vadx_mlp *mlp);
/* Target normalisation: fit = mean and population std of each column of the
 * device array Y [n][6] (computed on the device); get/set use host arrays. */
vadx_status vadx_mlp_fit_target_norm(vadx_mlp *mlp, const float *Y, int64_t n);
vadx_status vadx_mlp_get_target_norm(vadx_mlp *mlp, float *mean, float *std_);
vadx_status vadx_mlp_set_target_norm(vadx_mlp *mlp, const float *mean, const float *std_);
/* Host copies of the 17926 parameters. */
vadx_status vadx_mlp_get_params(vadx_mlp *mlp, float *out);
vadx_status vadx_mlp_set_params(vadx_mlp *mlp, const float *params);
/* Mean squared error over the n samples and the 6 normalised outputs, and its
 * gradient (host, 17926 floats), without updating the parameters. */
vadx_status vadx_mlp_grad(vadx_mlp *mlp, const float *X, const float *Y, int64_t n, float *grad,
                          float *loss);
/* epochs passes over the n samples in order, in minibatches of `batch`, one
 * Adam step per minibatch; loss_hist (host, `epochs` floats) receives each
 * epoch's mean training loss. */
vadx_status vadx_mlp_train(vadx_mlp *mlp, const float *X, const float *Y, int64_t n,
                           int32_t epochs, int32_t batch, float *loss_hist);
/* Forward pass over n points: Y [n][6] in target units; J (nullable) [n][6][4]
 * = d(normalised output)/d(normalised input); score (nullable) [n] =
 * Euclidean norm of the input gradients of outputs score_out0 and score_out1
 * (the transition score used to pick points to simulate). Device arrays. */
vadx_status vadx_mlp_predict(vadx_mlp *mlp, const float *X, int64_t n, float *Y, float *J,
                             float *score, int32_t score_out0, int32_t score_out1);

/* Selection after screening a grid: of the n scores (device FP32), the k
 * largest (ties go to the lower index) plus an audit sample of the rest, each
 * remaining point taken independently with probability audit_frac by a
 * Philox4x32-10 draw keyed (seed, point index). sel (device, capacity
 * entries) receives the selected indices in ascending order; is_audit
 * (device, nullable) marks the audit picks with 1. *n_sel (host) receives the
 * count; VADX_E_OOM (with *n_sel set) when it exceeds capacity. Synchronises
 * the network's stream. */
vadx_status vadx_mlp_select(vadx_mlp *mlp, const float *score, int64_t n, int64_t k,
                            float audit_frac, uint32_t seed, int64_t *sel, uint8_t *is_audit,
                            int64_t capacity, int64_t *n_sel);

/* ---------------------------------------------------------------------------
 * Analysis metrics of Section 2.6 (Table 2) over stored excitatory rate
 * samples, one result per instance (mean_FC is vadx_stats.fc_mean):
 *  - window: the last `window` samples (a power of two, at most 16384; 0 = the
 *    largest power of two not above the sample count); every metric uses it.
 *  - psd: Welch's average of modified periodograms per region (segments of
 *    `segment` samples, a power of two in [16, min(window, 8192)], 0 =
 *    min(1024, window); hop segment/2; each segment's mean removed; periodic
 *    Hann window), one-sided density in Hz^2/Hz of the rate in Hz; the
 *    instance spectrum is the mean over regions. psd_peak_bin / psd_fmax_hz /
 *    psd_ampmax: its largest value among bins 1..segment/2 (lowest bin on
 *    ties). psd_slope_a, psd_log10_b: least-squares fit of
 *    log10 P = log10 b - a log10 f over the bins with fit_lo_hz <= f <=
 *    fit_hi_hz and P > 0 (psd_fit_bins of them; a = log10 b = 0 when fewer
 *    than 2) -- the paper's fit of log(PSD) to log(b / f^a).
 *  - mean_pli: mean over region pairs k < l of the phase lag index
 *    |mean_t sign(Im(z_k(t) conj z_l(t)))| (Stam et al. 2007), z the discrete
 *    analytic signal of the region's window with its mean removed (DFT, bin 0
 *    zeroed, bins 1..window/2-1 doubled, negative bins zeroed, inverse DFT);
 *    0 for one region.
 *  - Up/Down states per region on the stored single-precision rates (kHz):
 *    r = max - min over the window, centre = min + r/2, half-band
 *    h = ud_band r (single precision); a sample above centre + h enters Up,
 *    below centre - h enters Down; regions with r < ud_min_range_khz have no
 *    states; a state lasts from the sample that entered it to the one that
 *    left it, and the states cut by the window's ends are not counted.
 *    ud_up_ms / ud_down_ms: mean durations over every counted state of every
 *    region (0 without states); ud_*_count and ud_*_samples: their number and
 *    summed length in samples. */
typedef struct vadx_analysis_cfg {
    int32_t window, segment;
    double fit_lo_hz, fit_hi_hz;
    float ud_band, ud_min_range_khz;
} vadx_analysis_cfg;

typedef struct vadx_analysis {
    float psd_fmax_hz, psd_ampmax, psd_slope_a, psd_log10_b;
    float mean_pli, ud_up_ms, ud_down_ms, reserved;
    int32_t psd_peak_bin, psd_fit_bins, ud_up_count, ud_down_count;
    int64_t ud_up_samples, ud_down_samples;
} vadx_analysis;

/* Defaults: window 0, segment 0, fit band 1-100 Hz, ud_band 0.1,
 * ud_min_range_khz 1e-3 (1 Hz). */
vadx_status vadx_analysis_defaults(vadx_analysis_cfg *out);

/* Bytes of device workspace the analysis needs to take regions_per_pass
 * regions per pass (instances are processed in passes of whole instances;
 * more workspace, fewer passes), for series of n_samples samples and
 * instances of at most n_max regions. About 12 * window bytes per region
 * (the window and its analytic signal). */
vadx_status vadx_analysis_ws_bytes(int64_t n_samples, int32_t n_max, int64_t regions_per_pass,
                                   const vadx_analysis_cfg *cfg, size_t *bytes);

/* Analysis of n_inst series given as device arrays samples [n_inst][n_samples][n]
 * (FP32, kHz; the layout vadx_read_samples returns), sampled every
 * sample_period_ms. ws: device workspace (256-byte aligned, caller-owned,
 * contents overwritten) of at least the size vadx_analysis_ws_bytes gives for
 * one instance (VADX_E_OOM otherwise). out: device array of n_inst results.
 * psd_out (device, nullable): [n_inst][n][segment/2 + 1] region spectra;
 * pli_out (device, nullable): [n_inst][n][n] PLI matrices (diagonal 0). 1 <= n
 * <= 512. Stream-ordered on ctx's stream; no host synchronisation. */
vadx_status vadx_analyze_series(vadx_ctx *ctx, const float *samples, int64_t n_inst, int32_t n,
                                int64_t n_samples, double sample_period_ms,
                                const vadx_analysis_cfg *cfg, void *ws, size_t ws_bytes,
                                vadx_analysis *out, float *psd_out, float *pli_out);

/* The same analysis over the samples of the last vadx_integrate (any mix of
 * region counts; sample period tavg_steps * dt_ms) held in its workspace,
 * which must still be alive. out: device array, one result per instance of
 * the batch. */
vadx_status vadx_analyze(vadx_ctx *ctx, const vadx_analysis_cfg *cfg, void *ws, size_t ws_bytes,
                         vadx_analysis *out);

/* Analysis kernel timing: with vadx_enable_timing on, HIP events bracket each
 * analysis launch; launches[6] and ms[6] (host) receive, per kernel -- window
 * transpose, Welch spectra, analytic signals, phase lag index, Up/Down
 * durations, per-instance reduction -- the launch count and summed duration
 * since the last call (which resets them). Waits for the recorded events. */
vadx_status vadx_analysis_kernel_time(vadx_ctx *ctx, int64_t *launches, double *ms);

/* BOLD signal (Section 2.4's Balloon-Windkessel kernel; haemodynamics after
 * Stephan et al. 2007, classical output coefficients): per region, with the
 * neural input z = the excitatory rate sample (kHz) held over each sample
 * interval, from rest (s = 0, f = v = q = 1):
 *   ds/dt = z - kappa s - gamma (f - 1),  df/dt = s,
 *   tau0 dv/dt = f - v^(1/alpha),
 *   tau0 dq/dt = f (1 - (1 - E0)^(1/f)) / E0 - v^(1/alpha) q / v,
 *   BOLD = V0 (k1 (1 - q) + k2 (1 - q/v) + k3 (1 - v)),
 * integrated by classical Runge-Kutta with the sample period as the step
 * (time in s), sampled every tr_ms: sample m after round((m+1) tr / period)
 * samples, n_tr = floor(n_samples period / tr_ms) samples per region.
 * Defaults: kappa 0.65, gamma 0.41, tau0 0.98, alpha 0.32, E0 0.34, V0 0.02,
 * k1 = 7 E0, k2 = 2, k3 = 2 E0 - 0.2, tr_ms 2000. */
typedef struct vadx_bold_cfg {
    double kappa, gamma, tau0, alpha, E0, V0, k1, k2, k3, tr_ms;
} vadx_bold_cfg;
vadx_status vadx_bold_defaults(vadx_bold_cfg *out);
/* BOLD of device series samples [n_inst][n_samples][n] (kHz) into out
 * (device, [n_inst][n_tr][n]); *n_tr (host) receives the sample count per
 * region. Stream-ordered. */
vadx_status vadx_bold_series(vadx_ctx *ctx, const float *samples, int64_t n_inst, int32_t n,
                             int64_t n_samples, double sample_period_ms, const vadx_bold_cfg *cfg,
                             float *out, int32_t *n_tr);
/* BOLD of the samples of the last vadx_integrate (any mix of region counts):
 * out (device) holds each instance's [n_tr][n] block in instance order. */
vadx_status vadx_bold(vadx_ctx *ctx, const vadx_bold_cfg *cfg, float *out, int32_t *n_tr);

/* Arithmetic of one region-step in this library's formulation, counted by
 * running the kernel's own model code with an operation-counting scalar:
 * single- and double-precision FLOPs (add, mul = 1, fma = 2, transcendental =
 * 1) and the number of transcendentals among them. The delayed-coupling sum
 * adds 2 FLOPs per connectome edge and step on top (not included). For
 * roofline accounting. */
vadx_status vadx_region_step_ops(int32_t integrator, double *flop32, double *flop64,
                                 double *transcendental);

#ifdef __cplusplus
}
#endif
#endif /* VADX_H */
