/*
 * sim.h - C-ABI of the MI355X differentiable agent-based traffic simulator.
 *
 * One step phi = g(f(x)) of the paper (Results, "Differentiable agent-based
 * traffic simulation"): departures from origin queues, Newell car-following
 * on every link with the trajectory-grafted link cap (Methods eq.
 * newell_model; SI-A), Gumbel-softmax link choice with straight-through
 * estimator, merge choice and FIFO transfer with trajectory grafting (SI-B,
 * SI-C), and differentiable midpoint counting (SI-D); plus its reverse-mode
 * adjoint with checkpointed replay (Methods, "Optimization").
 *
 * Conventions for every entry point:
 *  - return value: SIM_OK (0) or a negative SIM_E* code; no C++ exception
 *    crosses this boundary.  sim_last_error() then holds a message.
 *  - inputs are copied (host or device memory as stated); the caller keeps
 *    ownership of everything it passes in.
 *  - outputs go into caller buffers; `on_device` = 1 means the pointer is
 *    device memory on the handle's device (e.g. a torch tensor's data_ptr),
 *    written in order on the handle's stream; 0 means host memory, and the
 *    call synchronises the stream before returning.
 *  - a handle is not thread-safe; calls on one handle are serialised by the
 *    caller.  All device work of a handle is ordered on its stream.
 *  - scenario batching: S scenarios share the network and agent pool; each
 *    has its own parameters (scenario-major [S x n]) and Philox key.
 */
#ifndef SIM_H
#define SIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SIM_OK = 0,
    SIM_EINVAL = -1,        /* argument out of range or inconsistent */
    SIM_ENOMEM = -2,        /* device or host allocation failed (nothing leaked) */
    SIM_EDEVICE = -3,       /* a HIP call failed */
    SIM_ESTATE = -4,        /* call not valid in the current state */
    SIM_EUNSUPPORTED = -5   /* valid input the kernels do not handle */
};

/* Parameter groups (sim_set_params / sim_backward).  Per link: [S x n_links];
 * rates: [S x n_origins x n_rate_bins]. */
enum sim_param {
    SIM_P_U = 0,          /* free-flow speed u (m/s), Methods eq. newell_model */
    SIM_P_KAPPA = 1,      /* jam density kappa per lane (veh/m), same */
    SIM_P_BETA = 2,       /* route-choice weight beta, SI-B link utility */
    SIM_P_ALPHA = 3,      /* merge priority alpha, SI-B merge choice */
    SIM_P_COST = 4,       /* link cost c, SI-B link utility */
    SIM_P_THETA_DEST = 5, /* destination-time coefficient theta of the link utility (gradient only: [S],
                             one value per scenario; the value itself is sim_config.dest_logit_coef) */
    SIM_P_RATES = 6,      /* departure rate per (origin, time bin), veh/s */
    SIM_P_CAP_MULT = 7,   /* outflow capacity multiplier per link */
    SIM_P_COUNT = 8
};

/* Counters per scenario (sim_get_state): */
enum {
    SIM_C_RELEASED = 0, SIM_C_DEPARTED = 1, SIM_C_ON_NET = 2, SIM_C_EXITED = 3,
    SIM_C_TRANSFERS = 4, SIM_C_TIES = 5, SIM_C_STUCK = 6, SIM_C_ORDER_VIOL = 7,
    SIM_C_COUNT = 8
};

/* Agent status codes (sim_get_state). */
enum { SIM_WAIT = 0, SIM_QUEUED = 1, SIM_ON = 2, SIM_EXITED = 3 };

/* Road network.  Host pointers; copied by sim_create.
 * tail/head: node ids in [0, n_nodes); lanes in [1, 8]; length, free_speed,
 * jam_density > 0; capacity >= 0 (veh/s/lane); beta/alpha/cost may be NULL
 * (defaults 0, 1, 1), cost > 0.  An agent stands for sim_config.platoon
 * vehicles, so a link passes at most capacity * lanes / platoon agents per
 * second.  Origins are nodes with a FIFO departure
 * queue (the paper's virtual inflow links).  Detectors count crossings of
 * position detector_pos (0 < pos <= length - 0.01) on detector_link (SI-D). */
typedef struct {
    int32_t n_nodes, n_links;
    const int32_t *tail, *head, *lanes;
    const float *length, *free_speed, *jam_density, *capacity;
    const float *beta, *alpha, *cost;
    int32_t n_origins;
    const int32_t *origin_node;
    int32_t n_detectors;
    const int32_t *detector_link;
    const float *detector_pos;
} sim_network;

/* Agent pool and demand.  Host pointers; copied by sim_create.
 * agent_origin: index into origin_node; agent_dest: node id, reachable
 * from the origin.  Either ready_time (fixed departure times, seconds) or
 * rates [n_origins x n_rate_bins] (departure-rate mode; rate_bin_s must be a
 * whole number of steps; rates count agents, i.e. platoons, per second).  In
 * rate mode agents of an origin are released in
 * agent-index order when the integrated rate crosses their queue index + 1. */
typedef struct {
    int32_t n_agents;
    const int32_t *agent_origin, *agent_dest;
    const float *ready_time;
    int32_t n_rate_bins;
    double rate_bin_s;
    const float *rates;
} sim_demand;

typedef struct {
    double dt;                /* step length (s); the paper ties dt = tau * platoon, tau = 1 */
    int32_t platoon;          /* platoon size dn (vehicles per agent) */
    double gumbel_tau;        /* Gumbel-softmax temperature (gradient only) */
    double dest_logit_coef;   /* theta: utility -= theta * (free-flow time to destination) */
    double big_m;             /* M of SI-A/SI-B (enters straight-through gradients only) */
    uint64_t seed;            /* Philox key of scenario 0 */
    const uint64_t *scenario_seed; /* NULL -> scenario s uses seed + s */
    int32_t n_scenarios;      /* S >= 1 */
    int32_t ckpt_every;       /* checkpoint interval of the recorded rollout (steps) */
    int32_t count_bin_steps;  /* detector sampling interval (steps) */
    int32_t n_count_bins;     /* number of samples kept per detector */
    int32_t max_steps;        /* longest recorded rollout (sizes the checkpoints) */
    int32_t allow_uturn;      /* 1: a head may take the reverse of its link */
    int32_t record_for_backward; /* 1: sim_rollout keeps checkpoints for sim_backward */
    size_t mem_budget_bytes;  /* 0 = no limit; sim_create fails with SIM_ENOMEM beyond it */
    int32_t tape_windows;     /* recording handles: windows of replay tape kept on the device.  The
                                 recording forward writes the tape of its last tape_windows windows
                                 as it goes; sim_backward replays only the windows before them (from
                                 their checkpoints).  0: as many as fit in 32 GiB, between 4 and 16;
                                 otherwise at least 4.  Never more than the recorded windows. */
} sim_config;

typedef struct sim_t sim_t;

/* Validate, copy the inputs, compute shortest free-flow times to every
 * destination (route-choice term), allocate device state on `hip_device`.
 * `hip_stream` (hipStream_t, may be NULL for the null stream) orders all
 * later device work.  On error *out is NULL and nothing is leaked.
 * SIM_EUNSUPPORTED for more than 4 detectors on one link or 2^24 or more
 * detectors in all. */
int sim_create(const sim_network *net, const sim_demand *dem, const sim_config *cfg,
               int hip_device, void *hip_stream, sim_t **out);

/* Free everything the handle owns.  NULL is accepted. */
int sim_destroy(sim_t *h);

/* Message for the last failing call on this handle (or the last failing
 * sim_create if h is NULL).  Valid until the next call on the handle. */
const char *sim_last_error(const sim_t *h);

/* Set one parameter group for all scenarios: values [S x n] scenario-major,
 * n = n_links (per-link groups) or n_origins*n_rate_bins (rates).  Takes
 * effect from the next step; SIM_P_KAPPA must keep dn/kappa >= the jam
 * spacing the link rings were sized for (SIM_EINVAL otherwise).  After
 * t = 0 it ends a recording: the rollout so far was made under other
 * parameters, so sim_backward needs a new one from t = 0 (SIM_ESTATE). */
int sim_set_params(sim_t *h, int which, const float *values, int64_t n, int on_device);

/* Current values of one parameter group, same layout and numbering as
 * sim_set_params: values [S x n], host or device (on_device). */
int sim_get_params(sim_t *h, int which, float *values, int64_t n, int on_device);

/* Back to t = 0: empty network, all agents waiting, counters, buckets and
 * observables cleared.  Parameters are kept.  The origin queues are rebuilt
 * on the host and uploaded only when a placement (sim_place, or a restored
 * state with placed agents) has changed them since the last reset; otherwise
 * the reset clears device state only and waits for the stream. */
int sim_reset(sim_t *h);

/* At t = 0 only: put agents on links at given positions (every scenario),
 * in the given order per link (which fixes their entry sequence), and drop
 * them from their origin queues.  Host arrays of length n. */
int sim_place(sim_t *h, int32_t n, const int32_t *agent, const int32_t *link, const float *pos);

/* Advance one step / T steps.  With record_for_backward, sim_rollout from
 * t = 0 stores a checkpoint every ckpt_every steps. */
int sim_step(sim_t *h);
int sim_rollout(sim_t *h, int32_t T);

/* Five-minute style counts: counts [S x n_detectors x n_count_bins] (float,
 * vehicles crossing each detector in each sampling interval; SI-D value
 * part) and total travel time ttt [S] (double, seconds agents spent queued
 * or on the network). */
int sim_get_observables(sim_t *h, float *counts, double *ttt, int on_device);

/* Reverse-mode adjoint of the recorded rollout (record_for_backward, rollout
 * from t = 0): the exact derivative of the step with every discrete decision
 * held fixed and every stop_gradient a constant, i.e. the gradient of the
 * paper's straight-through / trajectory-grafting construction (SI-A..SI-D).
 * Cotangents (each may be NULL): dL_dcounts [S x det x bins] float,
 * dL_dttt [S] double, dL_dpos [S x n_agents] float (final positions of
 * agents on the network).  grads[k] (for each bit k set in param_mask,
 * every group below SIM_P_COUNT) receives dL/d(group k), overwritten, float,
 * same layout as sim_set_params (SIM_P_THETA_DEST: [S]).  Rates reach the loss
 * through departure-time grafting and capacity multipliers through
 * admission-time grafting: a vehicle released, or let through a link's
 * outflow token bucket, carries the time at which its release count or
 * token was reached into its entry position, in the manner of the
 * trajectory grafting of SI-C.  beta, cost, alpha and theta reach it
 * through the straight-through estimator of SI-B: the relaxed route-choice
 * and merge weights (softmax at temperature gumbel_tau of the same scores
 * plus the same Gumbel noise) enter the transfer update with value zero and
 * the softmax's gradient, scaled by big_m; a merge with k winners is k
 * sequential softmax stages over the candidates not yet picked.  Unknown
 * bits: SIM_EINVAL; straight-through groups with gumbel_tau <= 0:
 * SIM_EINVAL. */
int sim_backward(sim_t *h, const float *dL_dcounts, const double *dL_dttt, const float *dL_dpos,
                 uint32_t param_mask, float *const *grads, int on_device);

/* ------------------------------------------------------------------------
 * Gradient-based calibration and control (Methods, "Optimization"): each
 * iteration runs the forward rollout from t = 0, evaluates the loss on the
 * detector counts, runs the adjoint, and updates the chosen parameter groups
 * with AdamW (Loshchilov and Hutter: decoupled weight decay; the paper uses
 * learning rate 0.1, weight decay 1e-5 and otherwise default
 * hyperparameters).  The loop stops when the loss has not improved for
 * `patience` iterations (the paper: 20) or after max_iters, and leaves the
 * handle on the parameters of the lowest loss seen.  Every step runs on the
 * device; the host reads one loss value per iteration.
 *
 * Losses: SIM_LOSS_COUNTS_MSE, mean over detectors and count bins of the
 * squared difference to `observed` [det x bins] (calibration, Methods
 * "Optimization"; the paper averages squared count errors over observed
 * links); SIM_LOSS_CUMULATIVE, (sum over the bins of detector
 * target_detector - target)^2 (control: the paper steers the cumulative
 * count of one target link to half its uncontrolled value through the link
 * costs; Results, "Gradient-guided traffic control").
 *
 * After each update a group is clipped to [lower[k], upper[k]] (k = its
 * sim_param; NULL arrays take wide defaults: u [0.5, 60], kappa [1e-3, the
 * jam density the rings were sized for], beta and alpha unbounded, cost
 * [0.01, 1e4], rates and capacity multipliers [0, 1e4]); kappa never exceeds
 * the value sim_create sized the link rings for.  Requirements: a recording
 * handle (record_for_backward) with one scenario, steps <= max_steps;
 * SIM_P_THETA_DEST cannot be optimised.  loss_history [max_iters] (host, may
 * be NULL) receives the loss of every iteration.
 * ------------------------------------------------------------------------ */
enum { SIM_LOSS_COUNTS_MSE = 0, SIM_LOSS_CUMULATIVE = 1 };
typedef struct {
    uint32_t groups;          /* bit k set: optimise sim_param k */
    int32_t steps;            /* rollout length of every iteration */
    int32_t max_iters;        /* at most this many loss evaluations */
    int32_t patience;         /* stop after this many iterations without a lower loss */
    double lr, weight_decay, beta1, beta2, eps;   /* AdamW */
    int32_t loss;             /* SIM_LOSS_COUNTS_MSE or SIM_LOSS_CUMULATIVE */
    int32_t target_detector;  /* SIM_LOSS_CUMULATIVE */
    double target;            /* SIM_LOSS_CUMULATIVE */
    const float *lower, *upper;   /* [SIM_P_COUNT] box per group, or NULL */
    int32_t normalized;       /* 1: AdamW works on x = (p - lower) / (upper - lower) of each optimised group
                                 (finite boxes required), so one learning rate moves groups of very
                                 different scales by the same fraction of their range; 0: on p */
    float *const *first_grad; /* NULL, or per sim_param k a host buffer [n_k] (NULL entries skipped)
                                 that receives dLoss/d(group k) at the starting parameters
                                 (written when max_iters >= 2) */
} sim_opt_config;
typedef struct {
    int32_t iterations;       /* loss evaluations made */
    int32_t best_iter;        /* iteration of the lowest loss (0 = the starting parameters) */
    double first_loss, best_loss;
    double seconds;           /* wall time of the loop */
} sim_opt_result;
int sim_optimize(sim_t *h, const sim_opt_config *oc, const float *observed, double *loss_history,
                 sim_opt_result *res);

/* Agent state, host arrays [S x n_agents] (any may be NULL): status
 * (SIM_WAIT..SIM_EXITED), link (-1 when not on a link), pos, seq (entry
 * sequence on its link); counters [S x SIM_C_COUNT]. */
int sim_get_state(sim_t *h, int32_t *status, int32_t *link, float *pos, int32_t *seq,
                  int64_t *counters);

/* Vehicle-steps per scenario [S] (host): the sum over completed steps of
 * the number of agents on the network after the step. */
int sim_get_stats(sim_t *h, int64_t *vehicle_steps);

/* Whole simulation state as an opaque host blob (agent rings, per-link and
 * per-origin state, per-agent times, counters, detector samples, placed
 * agents, step counter), for resuming a run or restarting it elsewhere.
 * sim_get_full_state: with blob NULL writes the size to *n; otherwise blob
 * must hold cap >= that many bytes (SIM_EINVAL if not).  sim_set_full_state
 * loads a blob taken from a handle created with the same network, agent
 * pool and configuration (SIM_EINVAL otherwise) and sets the step counter;
 * a handle restored to t > 0 cannot run sim_backward until sim_reset
 * (its checkpoints do not cover the restored past). */
int sim_get_full_state(sim_t *h, void *blob, size_t cap, size_t *n);
int sim_set_full_state(sim_t *h, const void *blob, size_t n);

/* Near-tie log of the forward steps since the last sim_reset (or
 * sim_set_full_state): decisions whose margin lies within rounding distance
 * of the other outcome, where an implementation with another rounding of the
 * same arithmetic (the double-precision Gumbel transform goes through the
 * platform's log) could decide otherwise.  Records are int32[6] (scenario,
 * step t, class, agent, link, decision), sorted; links in the caller's
 * numbering.  Classes: SIM_TIE_CHOICE, a route choice whose best and second
 * score differ by less than 1e-12 (1 + |best|): link = decision = the chosen
 * link (SI-B eq. gumbel); SIM_TIE_MERGE, a merge candidate whose key exceeds
 * another candidate's for the same target by less than 1e-12 (1 + |key|):
 * agent = the candidate ranked first, link = the target, decision 1.
 * Replays of the backward pass and autotuner probes append nothing.  *n
 * receives the number of records logged; min(*n, cap, SIM_TIE_LOG_MAX) are
 * copied to buf (host, may be NULL when cap = 0).  The device keeps the first
 * SIM_TIE_LOG_MAX records only. */
enum { SIM_TIE_CHOICE = 0, SIM_TIE_MERGE = 1 };
#define SIM_TIE_LOG_MAX (1 << 16)
int sim_get_tie_log(sim_t *h, int32_t *buf, int64_t cap, int64_t *n);

/* Per (scenario, link) state, host arrays [S x n_links] (any may be NULL):
 * token bucket B, cumulative outflow E, next entry sequence number. */
int sim_get_link_state(sim_t *h, double *B, int64_t *E, int32_t *next_seq);

/* Shortest free-flow time (s) from every node to every destination node,
 * host [n_dest x n_nodes] in increasing destination-node order; *n_dest
 * receives the count.  Pass out = NULL to query n_dest only. */
int sim_get_dist(sim_t *h, double *out, int32_t *n_dest);

/* Current step index. */
int sim_time(const sim_t *h, int32_t *t);

/* Philox4x32-10 (Salmon et al., SC'11) evaluated on the device: n counters
 * ctr [n x 4] with keys key [n x 2], host arrays; out [n x 4] host. */
int sim_philox(sim_t *h, int32_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out);

/* The single-precision Gumbel(0,1) transform the kernels take their fast
 * route-choice and merge decisions on, evaluated on the device: for each of n
 * host words w, g = -log(-log U) with U = ((w >> 8) + 1/2) 2^-24 (the same U
 * as the double-precision draw).  out [n] host floats.  A decision is
 * taken on these values only when it wins by a margin of 1e-4, five times
 * the largest error of a difference of two of them (2e-5); otherwise it is
 * recomputed in double precision.  SIM_EINVAL for
 * n < 0 or NULL arrays. */
int sim_gumbel_fast(sim_t *h, int32_t n, const uint32_t *words, float *out);

/* Segmented sort of n keys (segment id, position, sequence) into segment
 * order, position descending, sequence ascending; writes the permutation
 * perm [n] and segment offsets seg_off [n_segments + 1].  Device pointers,
 * ordered on the handle's stream.  Used to build the per-link layout from an
 * arbitrary agent list; exposed for testing. */
int sim_segsort(sim_t *h, int32_t n, int32_t n_segments, const int32_t *seg, const float *pos,
                const int32_t *seq, int32_t *perm, int32_t *seg_off);

/* Allocation-free variant of sim_segsort, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, order and results as sim_segsort;
 * it calls no allocating routine.  Its per-segment counters live in one fixed
 * device array of the library per GPU (8 MiB, held until the process ends),
 * so n_segments may be at most SIM_SEGSORT_NOALLOC_MAX_SEGMENTS (SIM_EINVAL
 * beyond); segments hold at most 2048 keys, as in sim_segsort.  The array is
 * cleared at the start of every call.  status: NULL -> the call waits for the
 * handle's stream and returns SIM_EUNSUPPORTED if a segment is too long;
 * otherwise a device int32 that receives 0, or 1 for that overflow, in
 * stream order, and the call returns without waiting.  All calls on one GPU
 * share the array: calls that may overlap on one GPU (other streams or
 * handles not ordered with this one) race and must be serialised by the
 * caller. */
#define SIM_SEGSORT_NOALLOC_MAX_SEGMENTS (1 << 20)
int sim_segsort_noalloc(sim_t *h, int32_t n, int32_t n_segments, const int32_t *seg, const float *pos,
                        const int32_t *seq, int32_t *perm, int32_t *seg_off, int32_t *status);

/* Launch schedule: lanes G per work item of the link-phase and reverse
 * kernels for rings of at most 128 slots (8, 16, 32 or 64; rings of at most
 * 256 slots run on max(G, 16) lanes, at most 512 on max(G, 32), larger on a
 * whole wavefront), and the floor of the node-phase lane group (8, 16, 32 or
 * 64: each node runs on the smallest group, not below the floor, that holds
 * its merge candidates and out-links).  Results do not depend on it. */
int sim_set_schedule(sim_t *h, int g_link, int g_node, int g_rev);
int sim_get_schedule(sim_t *h, int *g_link, int *g_node, int *g_rev);

/* Device time (ms) and launch count of each kernel kind accumulated since
 * the last call with reset = 1, while timing is enabled (sim_set_timing).
 * Kinds 0 link phase, 1 node phase, 2 reverse: each launch's execution
 * interval, first wave start to last wave end, which the kernels record
 * themselves; kind 3 tape/checkpoint copies: HIP events around the copy;
 * kinds 4, 5, 6: the link, node and reverse launches again, timed with HIP
 * events recorded on the launch's stream right before and after it (each
 * interval also holds the dispatch of the launch after the preceding work on
 * the stream ended).  n_kinds <= 7.
 * While timing is enabled the backward pass runs its windows one after
 * another instead of overlapping replays with the reverse sweep, so each
 * kernel's time is its own.  Within one sim_rollout or sim_backward call at
 * most 16384 launches are timed (their records take up to 1.5 GB of device
 * memory, allocated on first use); later launches of the call run untimed. */
int sim_set_timing(sim_t *h, int enable);
int sim_get_timing(sim_t *h, double *ms, int64_t *launches, int n_kinds, int reset);

/* Autotuner.  Picks the schedule of sim_set_schedule (lanes per work item of
 * the link and reverse kernels, lane-group floor of the node kernel) for
 * this handle's shape: each candidate runs
 * probe_steps steps from the current state (and, for a recording handle,
 * the reverse sweep over a window recorded from it), timed with HIP events
 * on the handle's stream, one dimension at a time.  The state is restored
 * afterwards, so call it on a representative state (e.g. mid-rollout);
 * results never depend on the schedule, only speed does.  The choice is
 * cached in the process and, if cache_path is not NULL, appended to that
 * text file ("key g_link g_node g_rev ms" per line) under a key of the
 * device architecture and log2-bucketed shape (scenarios, links, agents,
 * ring slots per link, node candidates, recording); a cached entry is used
 * without probing unless flags bit 0 is set.  Writes the chosen sizes to
 * g_link, g_node, g_rev (each may be NULL) and applies them. */
int sim_autotune(sim_t *h, int32_t probe_steps, const char *cache_path, int32_t flags, int32_t *g_link,
                 int32_t *g_node, int32_t *g_rev);

/* Device bytes sim_create would allocate for these inputs (host-only work:
 * validation, numbering, shortest times).  SIM_EINVAL for invalid inputs. */
int sim_footprint(const sim_network *net, const sim_demand *dem, const sim_config *cfg, size_t *bytes);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of forward rollout requests.
 *
 * A server owns a loop thread and host preparation workers.  srv_submit
 * copies the request (network, demand, config, T steps) and returns at once.
 * Requests are admitted in arrival order (a later one may pass one that does
 * not fit) when a slot is free and the request's device footprint
 * (sim_footprint) fits the remaining budget; each admitted request gets its
 * own device state and stream, and all running requests advance chunk by
 * chunk so their kernels overlap.  Results do not depend on the mix.  A
 * request that fails validation or exceeds the budget on its own ends
 * SRV_FAILED without disturbing the others.  hip_device = -1 runs a
 * host-only executor (admission logic only, zero observables) for tests.
 * ------------------------------------------------------------------------ */
typedef struct srv_t srv_t;
enum { SRV_QUEUED = 0, SRV_RUNNING = 1, SRV_DONE = 2, SRV_FAILED = 3, SRV_CANCELLED = 4 };

int srv_create(int hip_device, size_t mem_budget_bytes, int32_t max_slots, int32_t chunk_steps, srv_t **out);
int srv_submit(srv_t *s, const sim_network *net, const sim_demand *dem, const sim_config *cfg, int32_t T,
               int64_t *ticket);
int srv_poll(srv_t *s, int64_t ticket, int *state);
/* Block until the request is done, failed or cancelled, or timeout_s passes. */
int srv_wait(srv_t *s, int64_t ticket, double timeout_s, int *state);
/* Results of a SRV_DONE request into host buffers (each may be NULL): counts
 * [S x det x bins], total travel time [S], vehicle-steps [S] (S = the
 * request's n_scenarios), latency from submission to completion in seconds.
 * SIM_ESTATE before completion; the request's failure code after failure. */
int srv_result(srv_t *s, int64_t ticket, float *counts, double *ttt, int64_t *vehicle_steps, double *latency_s);
const char *srv_error(srv_t *s, int64_t ticket);
int srv_cancel(srv_t *s, int64_t ticket);
/* Latency percentiles of completed requests, vehicle-steps per second from
 * the first arrival to the last completion, completions, and the largest
 * number of requests that ran at once. */
int srv_stats(srv_t *s, double *p50_s, double *p99_s, double *vehicle_steps_per_s, int64_t *completed,
              int64_t *max_running);
int srv_destroy(srv_t *s);

#ifdef __cplusplus
}
#endif

#endif /* SIM_H */
