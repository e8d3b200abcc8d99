// Internal layout of the simulator's device state (library-private).
//
// Layout (scenario s, link j, node v, agent i; S scenarios, L links, N agents):
//  - every (s, j) "segment" seg = s*L + j owns a ring of cap[j] slots at
//    ring_base[j] + s*ring_total holding (agent id, position) of the agents on
//    the link in entry order; rhead/rtail are monotone counters, the agent in
//    counter q sits in slot q % cap[j] and its entry sequence number is q.
//    Entry order equals the order by (position desc, sequence asc): the
//    update rule is monotone in the leader's and the agent's own position,
//    so it never reorders a link (checked every step).
//  - per-agent arrays are [S*N]; per-origin [S*O]; per-segment [S*L].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sim.h"

namespace sim {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kMaxLanes = 8;     // lanes per link accepted by sim_create
constexpr int kSmallRing = 128;  // ring classes by slots: <= kSmallRing, <= kMidRing, <= kLongRing, larger
constexpr int kMidRing = 256;
constexpr int kLongRing = 512;
constexpr int kRingClasses = 4;
constexpr int kMaxDetPerLink = 4;
constexpr int kCtrSlots = 64;      // counters are spread over this many slots per scenario
enum : int32_t { CH_STUCK = -1, CH_EXIT = -2, CH_NONE = -3 };
enum : uint8_t { AG_WAIT = 0, AG_QUEUED = 1, AG_ON = 2, AG_EXITED = 3 };
enum { CTR_RELEASED = 0, CTR_DEPARTED, CTR_ON_NET, CTR_EXITED, CTR_TRANSFERS, CTR_TIES, CTR_STUCK,
       CTR_ORDER_VIOL, CTR_N };
enum { ERR_RING_OVERFLOW = 0, ERR_CAND_OVERFLOW = 1, ERR_N = 4 };
// near-tie log: classes of sim_get_tie_log, device capacity in records
enum { TIE_CHOICE = SIM_TIE_CHOICE, TIE_MERGE = SIM_TIE_MERGE };
constexpr int kTieLogMax = SIM_TIE_LOG_MAX;

// Per (scenario, link) state the link and node phases exchange, one 32-byte record, so that a
// phase touches one cache line per link instead of one per field.  Writers: the link phase (B,
// slots, nheads of its segment), the node phase at the link's head node (B, E, rhead) and at its
// tail node (rtail); different fields of one record are never written by two items of a launch.
struct __align__(32) LinkSt {
    double B;          // token bucket (before this step's idle cap)
    int64_t E;         // cumulative outflow
    int32_t rhead, rtail;    // ring counters (rtail is the next entry sequence number)
    int32_t slots, nheads;   // entry slots and heads found by this step's link phase
};
// Per (scenario, link) constants of the node phase, derived when parameters change (one record
// per out-link or in-link lane instead of six scattered arrays).
struct __align__(32) LinkNd {
    double util;       // beta / cost
    float alpha;       // merge priority
    int32_t head, tail, ring_base, cap, lanes;
};

// Per (scenario, link) constants of the link and reverse phases, derived when parameters change
// (one record per segment instead of nine arrays).
struct __align__(32) LinkCf {
    float vf, sp, L, thr;        // u * dt, jam spacing dn / kappa, length, arrival threshold L - 0.01
    int32_t cap, lanes, ring_base;
    int32_t det;                 // first detector (bits 0-23) | detectors on the link << 24
};

// Per (scenario, link) factors of the reverse sweep, derived when parameters change: dn / kappa^2
// (congested-branch gradient in kappa) and 1 / u in double, u in float.
struct __align__(16) RevCf {
    double dkap, inv_u;
    float u;
    int32_t pad;
};

struct Dev {
    // sizes
    int32_t S, L, Nn, O, N, D, nb, cbs, n_dest, maxl, n_rate_bins, fixed_mode, allow_uturn, platoon;
    int32_t rate_bin_steps;          // steps per departure-rate bin (rate bins are whole numbers of steps)
    int32_t g_link, g_node, g_rev;   // lanes per small segment / node floor / small reverse segment (8-64)
    int32_t lc_n[kRingClasses];      // links per ring class, contiguous ids: <= kSmallRing slots, <= kMidRing, ...
    int32_t nd_begin[4], nd_n[4];    // node id ranges of the node kernel's 8-, 16-, 32- and 64-lane roles
    int64_t ring_total;
    double dt, theta, rate_bin_s;
    double big_m, tau;               // M and the Gumbel-softmax temperature (straight-through gradients only)

    // network (shared by scenarios)
    const int32_t *tail, *head, *lanes, *cap, *ring_base;
    const float *length, *thr;
    const int32_t *out_off, *out_lnk, *in_off, *in_lnk, *org_off, *org_list;
    const int32_t *det_off, *det_list;
    const float *det_pos;
    const double *tff;      // route-choice free-flow time per link
    const double *route;    // per node and destination, per out-link m: t_ff(m) + shortest time from head(m)
    const int64_t *route_base;  // [Nn] first entry of the node's block (n_dest x out-degree)
    const int32_t *agent_didx, *agent_dest, *agent_origin;
    const int32_t *q_off, *q_list;   // origin queues (agent ids in release order)
    const int32_t *q_dest, *q_didx;  // destination node / table row of each queue entry
    const int32_t *node_cnt;         // per node: in-degree | out-degree << 8 | origins << 16
    const int32_t *in_pad, *out_pad; // [Nn x max_in], [Nn x max_out] link ids in CSR order
    const int32_t *in_loff;          // [Nn x max_in] first head lane of each in-link (prefix sum of lanes)
    const int2 *cand;                // [Nn x max_cand] candidate lane -> head lane: (in-link, in-link index |
                                     // rank << 8); then origin lane: (origin, first queue entry)
    int32_t max_cand;
    const int32_t *cbase;            // [Nn] first candidate record of each node (candidate lanes in order)
    int32_t n_cand;                  // candidate records per scenario and step (sum over nodes)
    int32_t max_in, max_out, max_org;
    const int64_t *q_rstep;          // fixed mode: release step of each queue entry
    const uint64_t *seed;            // [S]

    // parameters [S x L] / [S x O x B]
    const float *u, *kappa, *alpha, *rates;
    const float *beta, *cost;        // [S*L] route-choice weight and link cost
    const float *vfree, *spacing;    // derived: u*dt, platoon/kappa
    const double *util;              // beta / cost
    const double *acc;               // cap_mult * capacity * lanes * dt
    const float *capm;               // [S*L] capacity multipliers
    const float *capacity;           // [L] outflow capacity per lane

    // state
    float *ring_pos;
    int32_t *ring_agent;
    int2 *ring_aux;                  // [S * ring_total] (destination node, table row) of each slot's agent
    LinkSt *ls;                      // [S*L] bucket, outflow, ring counters, entry slots, heads
    const LinkNd *lnd;               // [S*L] node-phase constants
    const LinkCf *lcf;               // [S*L] link- and reverse-phase constants
    const RevCf *rcf;                // [S*L] reverse-sweep factors
    double *dB;                      // [S*L] dB/d cap_mult (recording handles only, else null)
    int4 *head_rec;                  // [S*L*maxl] (agent, destination, table row, -) of each head
    uint8_t *status;                 // [S*N]
    double *tstar;                   // [S*N] release time (rate mode)
    int32_t *rel_t, *dep_t, *exit_t; // [S*N]
    double *Dacc;                    // [S*O] integrated departures
    int32_t *rel_ptr, *dep_ptr;      // [S*O]
    int64_t *ctr;                    // [S*kCtrSlots*CTR_N], summed on read
    int32_t *cum;                    // [S*D*nb] cumulative detector counts
    int32_t *err;                    // [ERR_N]
    int32_t *tie_log;                // [tie_cap x 6] near-tie records of the forward (null in replays)
    int32_t *tie_n;                  // [1] records appended (may exceed tie_cap; the rest are dropped)
    int32_t tie_cap;

    // tape (replay window) and adjoint
    float *tape_pos;                 // [(W+1) * S * ring_total]
    int32_t *tape_agent;             // same
    int4 *tape_seg;                  // [(W+1) * S * L] per segment and state: (head counter, tail counter,
                                     // ring slot of the head, departure mask: bit e set when the link's
                                     // entrant of entry order e in this step left an origin; entrants per
                                     // step <= lanes <= 8)
    int32_t *tape_dst;               // [(W+1) * S * L * maxl] entry slot of each leaving head (-1: exit)
    float *tape_dstg;                // same shape as tape_dst: admission-graft factor -u_to dt_tok/dm
    int4 *tape_ste;                  // [(W+1) * S * n_cand] per node candidate: (agent, chosen out-link index |
                                     // slots << 8 | moved << 16, in-link or -1, ring slot of its adjoint or -1)
    float *adj_ring;                 // [S * ring_total] adjoint of the position of each ring slot's agent
    float *depg;                     // [S*N] adjoint reaching a departure graft, times u of the first link
    double *gu, *gk, *gm;            // [S*L] accumulated parameter gradients (u, kappa, cap_mult)
    double *gbeta, *gcost, *galpha;  // [S*L] straight-through gradients (beta, cost, alpha)
    double *gth;                     // [S*Nn] per-node part of the theta gradient
    const float *gQ;                 // [S*D*nb] dL/dcounts (device copy)
    const double *gT;                // [S]
    const float *gx;                 // [S*N]
    unsigned long long *kstamp;      // kernel timing: this launch's record, (start, end) per wave; or null
};

}  // namespace sim


#include "sim.h"
#include <string>

namespace sim {

// serving hooks (sim_runtime.cpp)
sim_t *host_prepare(const sim_network *net, const sim_demand *dem, const sim_config *cfg, int device, int *code,
                    std::string *err);
size_t footprint_of(const sim_t *h);
// allocate and upload a prepared handle's device state on `stream`, carving it from
// [arena, arena + arena_bytes) when arena is not null (hipMalloc for what does not fit)
int device_attach(sim_t *h, hipStream_t stream, void *arena, size_t arena_bytes, std::string *err);
void release_handle(sim_t *h);
int64_t arena_fallbacks(const sim_t *h);
int rollout_enqueue(sim_t *h, int T, std::string *err);
int results_enqueue(sim_t *h, float *counts, double *ttt, int64_t *vsteps, std::string *err);
int device_errors(sim_t *h, std::string *err);
int counts_size(const sim_t *h);
int scenarios_of(const sim_t *h);
void destroy_handle(sim_t *h);

// kernel launchers (sim_kernels.hip)
void launch_link(const Dev &d, int t, int sample_b, int tape_k, hipStream_t st);
void launch_node(const Dev &d, int t, int tape_k, hipStream_t st);
void launch_tape_snapshot(const Dev &d, int tape_k, hipStream_t st);
void launch_reverse(const Dev &d, int t, int tape_k, int init, hipStream_t st);
void launch_ste(const Dev &d, int t, int tape_k, hipStream_t st);
void launch_theta_sum(const Dev &d, float *out, hipStream_t st);
int link_blocks(const Dev &d);
int node_blocks(const Dev &d);
int reverse_blocks(const Dev &d);
void launch_stamp_reduce(const int64_t *off, const int32_t *waves, int n, const unsigned long long *st,
                         unsigned long long *out, hipStream_t s);
void launch_rate_grad(const Dev &d, float *g_rates, hipStream_t st);
void launch_philox(int n, const uint32_t *ctr, const uint32_t *key, uint32_t *out, hipStream_t st);
void launch_gumbel_fast(int n, const uint32_t *w, float *out, hipStream_t st);
int launch_segsort(int n, int n_seg, const int32_t *seg, const float *pos, const int32_t *seq,
                   int32_t *perm, int32_t *seg_off, int32_t *scratch, hipStream_t st);
// allocation-free variant: counters in a fixed per-device array (at most
// kNoAllocMaxSegments segments); status: device flag written in stream order
// (nothing waited for), or NULL to wait and return 1 on a segment overflow.
// Returns -2 for too many segments, -1 on a HIP failure or a device whose
// array address was not taken (segsort_scratch_init, with it current).
constexpr int kNoAllocMaxSegments = 1 << 20;
constexpr int kMaxDevices = 64;
int segsort_scratch_init(int device);
int launch_segsort_noalloc(int device, int n, int n_seg, const int32_t *seg, const float *pos, const int32_t *seq,
                           int32_t *perm, int32_t *seg_off, int32_t *status, hipStream_t st);
// Several device-to-device copies in one launch (16-byte aligned arrays; any byte count).
constexpr int kMaxCopyJobs = 12;
struct CopyJob { const void *src; void *dst; uint64_t bytes; };
struct CopyJobs { CopyJob job[kMaxCopyJobs]; int32_t n; };
void launch_copy_multi(const CopyJobs &jobs, hipStream_t st);
void launch_derive(const Dev &d, const float *cap_mult_scen, const float *capacity, const float *beta,
                   const float *cost, double *util, double *acc, float *vfree, float *spacing, LinkNd *lnd,
                   LinkCf *lcf, RevCf *rcf, hipStream_t st);
void launch_ttt(const Dev &d, int T, double *out, int64_t *vsteps, unsigned long long *acc, hipStream_t st);
void launch_counts(const Dev &d, float *out, hipStream_t st);
void launch_d2f(const double *src, float *dst, int64_t n, hipStream_t st);
void launch_gather_links(const double *src, const int32_t *linv, float *dst, int S, int L, hipStream_t st);
void launch_count_loss(int n, int nb, const float *q, const float *y, int kind, int det, double target,
                       double *loss, float *gq, hipStream_t st);
void launch_adamw(int64_t n, float *p, const float *g, float *m, float *v, int t, double lr, double b1, double b2,
                  double eps, double wd, double x0, double sc, double lo, double hi, const float *hi_vec,
                  hipStream_t st);

// handle facts for the optimisation loop (sim_optimize.cpp)
hipStream_t stream_of(const sim_t *h);
int device_of(const sim_t *h);
int detectors_of(const sim_t *h);
int count_bins_of(const sim_t *h);
int max_steps_of(const sim_t *h);
bool is_recording(const sim_t *h);
bool rate_mode(const sim_t *h);
int64_t group_size(const sim_t *h, int which);     // values per scenario of a parameter group (-1: none)
void kappa_ceiling(const sim_t *h, float *out);     // [L], caller order: the jam density the rings were sized for
int set_error(sim_t *h, int code, const std::string &msg);

}  // namespace sim
