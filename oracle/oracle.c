/*
 * Reference oracle for the differentiable agent-based traffic step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU path.
 *
 * Plain, slow, sequential C.  Every phase follows the paper in the order it
 * is described:
 *   release (departure-rate reading, see below)
 *   -> per-link ordering by position and leader lookup (SI-A, sort-based
 *      headway)
 *   -> Newell car-following with the trajectory-grafted link cap
 *      (Methods eq. newell_model; SI-A eqs. for dx_free, dx_cong and x_limit)
 *   -> node model: link choice by Gumbel-softmax with straight-through
 *      estimator, validity masks, merge choice by merge priority alpha
 *      (SI-B eqs. softmax, gumbel, straigththrough; merge choice)
 *   -> vehicle transfer with trajectory grafting (SI-B eq. transfer; SI-C)
 *   -> differentiable midpoint counting (SI-D).
 *
 * Precision.  Positions are carried in the precision that decides the
 * integer state on the GPU (float by default; build with -DORC_POS_F64 for
 * an all-double variant).  Every other floating-point quantity (utilities,
 * Gumbel noise, departure accumulators, token buckets, shortest paths, the
 * whole adjoint) is double.
 *
 * Readings where the paper is silent (each is also listed in the design
 * notes of the repository):
 *  - order inside a step: phi = g(f(x)): the link model f, then the node model g (Results);
 *  - lanes: the leader of rank r is rank r - lanes; jam spacing dn/kappa per
 *    lane; a link has lanes - #(x <= dn/kappa) free entry slots (the paper's
 *    vacancy mask X_min > dn/kappa is the one-lane case);
 *  - link outflow capacity: token bucket, accrue m*q*lanes*dt per step, a
 *    transfer takes one token, idle cap min(B, 1) at the end of each step;
 *  - route utility beta/c - theta*(t_ff(m) + shortest time from head(m) to
 *    the destination) (the paper allows origin/destination terms in V);
 *  - Gumbel-max: argmax(V + g) equals argmax of the tempered softmax for any
 *    tau, so the hard choice does not depend on tau;
 *  - merge: top-k by alpha_from + g' with k = free entry slots (k = 1 is the
 *    paper's single entrant);
 *  - FIFO: heads of a link leave in rank order, the first that fails blocks
 *    the ones behind it;
 *  - trip end: a head whose link ends at its destination leaves the network;
 *  - departures: origin FIFO queues play the paper's virtual inflow links;
 *    in departure-rate mode agents are released when the integrated rate
 *    crosses their queue index + 1; the gradient reaches the rates through a
 *    departure-time graft on the entry position;
 *  - straight-through node model: the relaxed route and merge weights enter
 *    the transfer update with value zero and the softmax's gradient; a merge
 *    with k winners is k sequential softmax stages over the candidates not
 *    yet picked; the merge score is alpha_from times the chooser's relaxed
 *    weight of the target link, plus its Gumbel noise.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORC_POS_F64
typedef double pos_t;
#else
typedef float pos_t;
#endif

enum { ST_WAIT = 0, ST_QUEUED = 1, ST_ON = 2, ST_EXITED = 3 };
enum { BR_FREE = 0, BR_CONG = 1, BR_STOP = 2 };
enum { MV_TRANSFER = 0, MV_EXIT = 1, MV_DEPART = 2 };
enum { CH_EXIT = -2, CH_STUCK = -1 };

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,       */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).                   */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1) from the top 24 bits: an odd multiple of 2^-25, exact in double. */
static double u01(uint32_t w) { return ((double)(w >> 8) + 0.5) * (1.0 / 16777216.0); }

/* One Gumbel(0,1) draw for (agent, step, purpose, word) under key `seed`.
 * purpose 0 = link choice (word = candidate index), 1 = merge (word 0). */
double orc_gumbel(uint64_t seed, int32_t agent, int32_t step, int32_t purpose, int32_t word)
{
    uint32_t ctr[4] = { (uint32_t)agent, (uint32_t)step,
                        (uint32_t)(purpose + 2 * (word >> 2)), 0u };
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    double U = u01(o[word & 3]);
    return -log(-log(U));
}

double orc_uniform(uint64_t seed, int32_t agent, int32_t step, int32_t purpose, int32_t word)
{
    uint32_t ctr[4] = { (uint32_t)agent, (uint32_t)step,
                        (uint32_t)(purpose + 2 * (word >> 2)), 0u };
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    return u01(o[word & 3]);
}

/* ------------------------------------------------------------------------ */
/* Inputs                                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_nodes, n_links;
    const int32_t *tail, *head, *lanes;
    const float *length, *free_speed, *jam_density, *capacity, *beta, *alpha, *cost, *cap_mult;
    const float *route_speed; /* speeds behind the route-choice travel times (fixed) */
    int32_t n_origins;
    const int32_t *origin_node;
    int32_t n_detectors;
    const int32_t *detector_link;
    const float *detector_pos;
    int32_t n_agents;
    const int32_t *agent_origin, *agent_dest;
    const float *ready_time;  /* NULL -> departure-rate mode */
    int32_t n_rate_bins;
    double rate_bin_s;
    const float *rates;       /* [n_origins x n_rate_bins] */
    double dt;
    int32_t platoon;
    double gumbel_tau, dest_logit_coef, big_m;
    uint64_t seed;
    int32_t count_bin_steps, n_count_bins, allow_uturn;
} orc_inputs;

/* growable arrays for the decision log */
typedef struct { int32_t agent, link, leader, branch, capped; double x0, x1; } cf_rec;
typedef struct { int32_t agent, kind, from, to, tok_k; double tstar, bacc; int32_t rate_bin, qidx; int64_t cfi; int32_t rel_t; double dbacc; } mv_rec;
typedef struct { int32_t det, agent; double x; } smp_rec;
typedef struct { int32_t t, n_cf, n_mv, n_smp; int64_t cf0, mv0, smp0; int32_t sample_k; int64_t ch0, mg0; int32_t n_ch, n_mg; } step_rec;
/* route choice of one head or origin front: its valid candidate links [c0, c0 + n) */
typedef struct { int32_t agent, from, chosen, n; int64_t c0; double xh; } ch_rec;
/* merge of one target link with free entry slots: candidates [c0, c0 + n) in key order, k winners */
typedef struct { int32_t link, n, k; int64_t c0; } mg_rec;

#define VEC(T) struct { T *p; int64_t n, cap; }
#define VPUSH(v, val) do { if ((v).n == (v).cap) { (v).cap = (v).cap ? 2 * (v).cap : 1024; \
    (v).p = realloc((v).p, (size_t)(v).cap * sizeof(*(v).p)); } (v).p[(v).n++] = (val); } while (0)

typedef struct orc {
    orc_inputs in;
    /* owned copies */
    int32_t *tail, *head, *lanes, *origin_node, *det_link, *agent_origin, *agent_dest;
    float *length, *u, *kappa, *cap, *beta, *alpha, *cost, *cap_mult, *det_pos, *ready, *rates, *rspeed;
    /* derived per link (position precision) */
    pos_t *vfree, *spacing, *thr;
    /* graph */
    int32_t *out_off, *out_lnk;  /* node -> outgoing links (CSR, link order) */
    int32_t *in_off, *in_lnk;    /* node -> incoming links */
    int32_t *org_off, *org_list; /* node -> origins */
    /* destinations */
    int32_t n_dest, *dest_index /* per node, -1 if not a destination */, *agent_didx;
    double *dist; /* [n_dest x n_nodes] shortest free-flow time to destination */
    /* origin queues */
    int32_t *q_off, *q_list, *rel_ptr, *dep_ptr;
    int64_t *rstep; /* fixed-time mode release step per agent */
    double *D;      /* per origin, integrated departures */
    /* agent state */
    int32_t *status, *link, *seq;
    pos_t *pos;
    double *tstar; int32_t *tstar_bin, *qidx, *rel_t;
    /* link state */
    double *B;
    double *dB;     /* d B / d cap_mult of the same link (frozen decisions: B is affine in it) */
    int64_t *E;
    int32_t *next_seq;
    /* observation */
    int64_t *cprev;
    double *counts; /* [n_det x n_count_bins] */
    double ttt;
    int64_t ctr[8]; /* released, departed, on_net, exited, transfers, ties, stuck, order_viol */
    int32_t t;
    int log_on;
    VEC(cf_rec) cf;
    VEC(mv_rec) mv;
    VEC(smp_rec) smp;
    VEC(step_rec) steps;
    /* straight-through log: choosers (candidate links, route term t_ff + D, Gumbel noise) and merge
     * groups (chooser record, merge noise, moved flag of each candidate) */
    VEC(ch_rec) chs;
    VEC(int32_t) chl;
    VEC(double) chr, chg;
    VEC(mg_rec) mgs;
    VEC(int32_t) mgc, mgmv;
    VEC(double) mgg;
    int64_t *chidx;     /* per agent: its chooser record this step */
    double *base_pi;    /* per chooser record: pi at the chosen link (base) */
    double *base_pim;   /* per merge group, stage and remaining candidate: pi' (base) */
    VEC(uint8_t) capf;  /* per logged step and link: 1 if the idle cap clipped the bucket */
    /* scratch */
    int32_t *bucket_off, *bucket, *rank, *leader_of, *branch, *capped, *choice, *won, *head_cnt, *slots, *cfidx;
    pos_t *xhat;
    double *mkey, *bacc;
    /* frozen surrogate base values */
    /* near-tie log: (t, class, id, aux, decision) per event; see orc_tie_log */
    pos_t *tietol;      /* per link: margin below which a position threshold is a near tie */
    VEC(int32_t) ties;
    const int32_t *adopt; int64_t adopt_n;   /* another run's log, sorted, whose decisions are taken */
    int64_t n_adopted, n_unmatched, n_flipped;
    double tie_rel;     /* relative margin of a route-choice or merge near tie (1e-12) */
    int restored;       /* state imported at t > 0: no log of the past, no reverse sweep */
    int have_base;
    double *base_x1;    /* per cf record: x' (before cap) in the base surrogate */
    double *base_xhat;  /* per cf record */
    double *base_psi;   /* per move record */
    double *base_sig;   /* per sample record: sigmoid at base */
} orc_t;

static void *dupa(const void *src, size_t n) {
    if (!src || n == 0) return NULL;
    void *p = malloc(n);
    memcpy(p, src, n);
    return p;
}

/* ------------------------------------------------------------------------ */
/* Shortest free-flow time to each destination (Dijkstra on the reversed    */
/* graph, link weight length/free_speed, double).                           */
/* ------------------------------------------------------------------------ */
typedef struct { double d; int32_t v; } hitem;
static void hpush(hitem *h, int64_t *n, hitem x) {
    int64_t i = (*n)++;
    h[i] = x;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].d <= h[i].d) break;
        hitem t = h[p]; h[p] = h[i]; h[i] = t; i = p;
    }
}
static hitem hpop(hitem *h, int64_t *n) {
    hitem top = h[0];
    h[0] = h[--(*n)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *n && h[l].d < h[m].d) m = l;
        if (r < *n && h[r].d < h[m].d) m = r;
        if (m == i) break;
        hitem t = h[m]; h[m] = h[i]; h[i] = t; i = m;
    }
    return top;
}

static void shortest_times(orc_t *o)
{
    int32_t N = o->in.n_nodes, L = o->in.n_links;
    hitem *h = malloc(sizeof(hitem) * (size_t)(L + N + 1));
    char *done = malloc((size_t)N);
    for (int32_t di = 0; di < o->n_dest; ++di) {
        int32_t dnode = -1;
        for (int32_t v = 0; v < N; ++v) if (o->dest_index[v] == di) { dnode = v; break; }
        double *dist = o->dist + (int64_t)di * N;
        for (int32_t v = 0; v < N; ++v) { dist[v] = INFINITY; done[v] = 0; }
        int64_t hn = 0;
        dist[dnode] = 0.0;
        hpush(h, &hn, (hitem){0.0, dnode});
        while (hn > 0) {
            hitem it = hpop(h, &hn);
            if (done[it.v]) continue;
            done[it.v] = 1;
            /* relax links entering it.v: tail -> it.v */
            for (int32_t k = o->in_off[it.v]; k < o->in_off[it.v + 1]; ++k) {
                int32_t m = o->in_lnk[k];
                double w = (double)o->length[m] / (double)o->rspeed[m];
                double cand = w + dist[it.v];
                int32_t x = o->tail[m];
                if (cand < dist[x]) { dist[x] = cand; hpush(h, &hn, (hitem){cand, x}); }
            }
        }
    }
    free(h); free(done);
}

/* ------------------------------------------------------------------------ */
/* create / destroy                                                         */
/* ------------------------------------------------------------------------ */
static int cmp_i64pair(const void *a, const void *b) {
    const int64_t *x = a, *y = b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    return x[1] < y[1] ? -1 : (x[1] > y[1]);
}

static void build_queues(orc_t *o)
{
    int32_t O = o->in.n_origins, N = o->in.n_agents;
    free(o->q_off); free(o->q_list);
    o->q_off = calloc((size_t)O + 1, sizeof(int32_t));
    int32_t *cnt = calloc((size_t)O + 1, sizeof(int32_t));
    for (int32_t i = 0; i < N; ++i) if (o->status[i] == ST_WAIT) cnt[o->agent_origin[i]]++;
    for (int32_t k = 0; k < O; ++k) o->q_off[k + 1] = o->q_off[k] + cnt[k];
    o->q_list = malloc(sizeof(int32_t) * (size_t)(o->q_off[O] + 1));
    /* queue order: fixed-time mode by (release step, agent id); rate mode by agent id */
    int64_t *key = malloc(sizeof(int64_t) * 2 * (size_t)(o->q_off[O] + 1));
    memset(cnt, 0, sizeof(int32_t) * (size_t)O);
    for (int32_t i = 0; i < N; ++i) {
        if (o->status[i] != ST_WAIT) continue;
        int32_t k = o->agent_origin[i];
        int64_t at = (int64_t)o->q_off[k] + cnt[k]++;
        key[2 * at] = o->ready ? o->rstep[i] : 0;
        key[2 * at + 1] = i;
    }
    for (int32_t k = 0; k < O; ++k) {
        int32_t n = o->q_off[k + 1] - o->q_off[k];
        int64_t *kk = key + 2 * (int64_t)o->q_off[k];
        qsort(kk, (size_t)n, 2 * sizeof(int64_t), cmp_i64pair);
        for (int32_t a = 0; a < n; ++a) {
            o->q_list[o->q_off[k] + a] = (int32_t)kk[2 * a + 1];
            o->qidx[kk[2 * a + 1]] = a;
        }
        o->rel_ptr[k] = 0;
        o->dep_ptr[k] = 0;
    }
    free(key); free(cnt);
}

orc_t *orc_create(const orc_inputs *in)
{
    orc_t *o = calloc(1, sizeof(orc_t));
    o->in = *in;
    int32_t L = in->n_links, Nn = in->n_nodes, O = in->n_origins, N = in->n_agents, Dd = in->n_detectors;
    o->tail = dupa(in->tail, 4 * (size_t)L);
    o->head = dupa(in->head, 4 * (size_t)L);
    o->lanes = dupa(in->lanes, 4 * (size_t)L);
    o->length = dupa(in->length, 4 * (size_t)L);
    o->u = dupa(in->free_speed, 4 * (size_t)L);
    o->rspeed = dupa(in->route_speed ? in->route_speed : in->free_speed, 4 * (size_t)L);
    o->kappa = dupa(in->jam_density, 4 * (size_t)L);
    o->cap = dupa(in->capacity, 4 * (size_t)L);
    /* an agent is a platoon of dn vehicles (Methods, Newell's model): a link
     * passes capacity * lanes / dn agents per second */
    for (int32_t j = 0; j < L; ++j) o->cap[j] = o->cap[j] / (float)in->platoon;
    o->beta = dupa(in->beta, 4 * (size_t)L);
    o->alpha = dupa(in->alpha, 4 * (size_t)L);
    o->cost = dupa(in->cost, 4 * (size_t)L);
    o->cap_mult = malloc(4 * (size_t)L);
    for (int32_t j = 0; j < L; ++j) o->cap_mult[j] = in->cap_mult ? in->cap_mult[j] : 1.0f;
    o->origin_node = dupa(in->origin_node, 4 * (size_t)O);
    o->det_link = dupa(in->detector_link, 4 * (size_t)Dd);
    o->det_pos = dupa(in->detector_pos, 4 * (size_t)Dd);
    o->agent_origin = dupa(in->agent_origin, 4 * (size_t)N);
    o->agent_dest = dupa(in->agent_dest, 4 * (size_t)N);
    o->ready = in->ready_time ? dupa(in->ready_time, 4 * (size_t)N) : NULL;
    o->rates = in->rates ? dupa(in->rates, 4 * (size_t)O * (size_t)in->n_rate_bins) : NULL;

    o->vfree = malloc(sizeof(pos_t) * (size_t)L);
    o->spacing = malloc(sizeof(pos_t) * (size_t)L);
    o->thr = malloc(sizeof(pos_t) * (size_t)L);
    for (int32_t j = 0; j < L; ++j) {
        o->vfree[j] = (pos_t)o->u[j] * (pos_t)in->dt;
        o->spacing[j] = (pos_t)in->platoon / (pos_t)o->kappa[j];
        o->thr[j] = (pos_t)o->length[j] - (pos_t)0.01;
    }
    o->tie_rel = 1e-12;
    o->tietol = malloc(sizeof(pos_t) * (size_t)(L + 1));
    for (int32_t j = 0; j < L; ++j) o->tietol[j] = (pos_t)(o->length[j] * 1e-5f);

    /* CSR adjacency, link order within each node */
    o->out_off = calloc((size_t)Nn + 1, 4); o->in_off = calloc((size_t)Nn + 1, 4);
    for (int32_t j = 0; j < L; ++j) { o->out_off[o->tail[j] + 1]++; o->in_off[o->head[j] + 1]++; }
    for (int32_t v = 0; v < Nn; ++v) { o->out_off[v + 1] += o->out_off[v]; o->in_off[v + 1] += o->in_off[v]; }
    o->out_lnk = malloc(4 * (size_t)(L + 1)); o->in_lnk = malloc(4 * (size_t)(L + 1));
    {
        int32_t *fo = calloc((size_t)Nn, 4), *fi = calloc((size_t)Nn, 4);
        for (int32_t j = 0; j < L; ++j) {
            o->out_lnk[o->out_off[o->tail[j]] + fo[o->tail[j]]++] = j;
            o->in_lnk[o->in_off[o->head[j]] + fi[o->head[j]]++] = j;
        }
        free(fo); free(fi);
    }
    o->org_off = calloc((size_t)Nn + 1, 4);
    for (int32_t k = 0; k < O; ++k) o->org_off[o->origin_node[k] + 1]++;
    for (int32_t v = 0; v < Nn; ++v) o->org_off[v + 1] += o->org_off[v];
    o->org_list = malloc(4 * (size_t)(O + 1));
    {
        int32_t *f = calloc((size_t)Nn, 4);
        for (int32_t k = 0; k < O; ++k) o->org_list[o->org_off[o->origin_node[k]] + f[o->origin_node[k]]++] = k;
        free(f);
    }

    /* destinations and shortest times */
    o->dest_index = malloc(4 * (size_t)Nn);
    for (int32_t v = 0; v < Nn; ++v) o->dest_index[v] = -1;
    o->n_dest = 0;
    for (int32_t i = 0; i < N; ++i) {
        int32_t d = o->agent_dest[i];
        if (o->dest_index[d] < 0) o->dest_index[d] = o->n_dest++;
    }
    /* number destinations in node order so the table layout is canonical */
    o->n_dest = 0;
    for (int32_t v = 0; v < Nn; ++v) if (o->dest_index[v] >= 0) o->dest_index[v] = o->n_dest++;
    o->agent_didx = malloc(4 * (size_t)N);
    for (int32_t i = 0; i < N; ++i) o->agent_didx[i] = o->dest_index[o->agent_dest[i]];
    o->dist = malloc(sizeof(double) * (size_t)o->n_dest * (size_t)Nn);
    shortest_times(o);

    /* agents */
    o->status = calloc((size_t)N, 4); o->link = malloc(4 * (size_t)N); o->seq = calloc((size_t)N, 4);
    o->pos = calloc((size_t)N, sizeof(pos_t));
    o->tstar = calloc((size_t)N, 8); o->tstar_bin = calloc((size_t)N, 4); o->qidx = calloc((size_t)N, 4);
    o->rel_t = calloc((size_t)N, 4);
    for (int32_t i = 0; i < N; ++i) o->link[i] = -1;
    o->rstep = malloc(8 * (size_t)N);
    for (int32_t i = 0; i < N; ++i) {
        if (o->ready) {
            double r = floor((double)o->ready[i] / in->dt);
            if (r < 0) r = 0;
            if (r > 4e18) r = 4e18;
            o->rstep[i] = (int64_t)r;
        } else {
            o->rstep[i] = 0;
        }
    }
    o->rel_ptr = calloc((size_t)O, 4); o->dep_ptr = calloc((size_t)O, 4);
    o->D = calloc((size_t)O, 8);
    build_queues(o);

    o->B = calloc((size_t)L, 8); o->dB = calloc((size_t)L, 8); o->E = calloc((size_t)L, 8); o->next_seq = calloc((size_t)L, 4);
    o->cprev = calloc((size_t)Dd + 1, 8);
    o->counts = calloc((size_t)Dd * (size_t)(in->n_count_bins > 0 ? in->n_count_bins : 1) + 1, 8);

    o->bucket_off = malloc(4 * (size_t)(L + 1)); o->bucket = malloc(4 * (size_t)(N + 1));
    o->rank = malloc(4 * (size_t)(N + 1)); o->leader_of = malloc(4 * (size_t)(N + 1));
    o->branch = malloc(4 * (size_t)(N + 1)); o->capped = malloc(4 * (size_t)(N + 1));
    o->choice = malloc(4 * (size_t)(N + 1)); o->won = malloc(4 * (size_t)(N + 1));
    o->head_cnt = malloc(4 * (size_t)(L + 1)); o->slots = malloc(4 * (size_t)(L + 1));
    o->cfidx = malloc(4 * (size_t)(N + 1));
    o->xhat = malloc(sizeof(pos_t) * (size_t)(N + 1));
    o->mkey = malloc(8 * (size_t)(N + 1)); o->bacc = malloc(8 * (size_t)(L + 1));
    o->chidx = malloc(8 * (size_t)(N + 1));
    return o;
}

void orc_destroy(orc_t *o)
{
    if (!o) return;
    void *ptrs[] = { o->tail, o->head, o->lanes, o->origin_node, o->det_link, o->agent_origin,
        o->agent_dest, o->length, o->u, o->rspeed, o->kappa, o->cap, o->beta, o->alpha, o->cost, o->cap_mult,
        o->det_pos, o->ready, o->rates, o->vfree, o->spacing, o->thr, o->out_off, o->out_lnk,
        o->in_off, o->in_lnk, o->org_off, o->org_list, o->dest_index, o->agent_didx, o->dist,
        o->q_off, o->q_list, o->rel_ptr, o->dep_ptr, o->rstep, o->D, o->status, o->link, o->seq,
        o->pos, o->tstar, o->tstar_bin, o->qidx, o->rel_t, o->B, o->dB, o->E, o->next_seq, o->cprev, o->counts,
        o->bucket_off, o->bucket, o->rank, o->leader_of, o->branch, o->capped, o->choice, o->won,
        o->head_cnt, o->slots, o->cfidx, o->xhat, o->mkey, o->bacc, o->cf.p, o->mv.p, o->smp.p, o->steps.p, o->capf.p,
        o->chs.p, o->chl.p, o->chr.p, o->chg.p, o->mgs.p, o->mgc.p, o->mgmv.p, o->mgg.p, o->chidx, o->base_pi, o->base_pim,
        o->base_x1, o->base_xhat, o->base_psi, o->base_sig, o->tietol, o->ties.p, (void *)o->adopt };
    for (size_t k = 0; k < sizeof(ptrs) / sizeof(ptrs[0]); ++k) free(ptrs[k]);
    free(o);
}

void orc_set_logging(orc_t *o, int on) { o->log_on = on; }

/* Place agents on links at t = 0 (for set-ups such as the grafting toy).
 * Seq numbers follow the given order per link.  Queues are rebuilt without
 * the placed agents. */
int orc_place(orc_t *o, int32_t n, const int32_t *agent, const int32_t *lnk, const float *p)
{
    if (o->t != 0) return -1;
    for (int32_t k = 0; k < n; ++k) {
        int32_t i = agent[k];
        o->status[i] = ST_ON;
        o->link[i] = lnk[k];
        o->pos[i] = (pos_t)p[k];
        o->seq[i] = o->next_seq[lnk[k]]++;
        o->ctr[0]++; o->ctr[1]++;
    }
    build_queues(o);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* forward step                                                             */
/* ------------------------------------------------------------------------ */
static orc_t *g_sort_ctx;
static int cmp_rank(const void *a, const void *b)
{
    /* position descending, then entry sequence ascending (FIFO tie-break) */
    int32_t i = *(const int32_t *)a, k = *(const int32_t *)b;
    pos_t xi = g_sort_ctx->pos[i], xk = g_sort_ctx->pos[k];
    if (xi > xk) return -1;
    if (xi < xk) return 1;
    return (g_sort_ctx->seq[i] < g_sort_ctx->seq[k]) ? -1 : (g_sort_ctx->seq[i] > g_sort_ctx->seq[k]);
}

typedef struct { double key; int32_t agent; } mcand;
static int cmp_mcand(const void *a, const void *b)
{
    const mcand *x = a, *y = b;
    if (x->key > y->key) return -1;
    if (x->key < y->key) return 1;
    return x->agent < y->agent ? -1 : (x->agent > y->agent);
}

static double rate_overlap(double b0, double b1, double t0, double t1)
{
    double lo = b0 > t0 ? b0 : t0, hi = b1 < t1 ? b1 : t1;
    return hi > lo ? hi - lo : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Near ties.  Decisions taken on values that lie closer together than the  */
/* rounding of another precision could move them are logged as             */
/* (t, class, id, aux, decision):                                           */
/*   TIE_CHOICE  route choice whose best and second score differ by less    */
/*               than 1e-12 (1 + |best|): id agent, aux chosen link;        */
/*   TIE_MERGE   merge keys of one target link adjacent in key order that   */
/*               differ by less than 1e-12 (1 + |key|): id the agent ranked */
/*               first of the pair, aux the target link;                    */
/*   TIE_ARRIVE  |x_hat - (L - 0.01)| < 1e-5 L for an agent not at the cap  */
/*               L: id agent, aux link, decision arrived;                   */
/*   TIE_VACANT  |x_hat - dn/kappa| < 1e-5 L: id agent, aux link, decision  */
/*               occupies an entry slot;                                    */
/*   TIE_DETECT  at a sampling step, |x - o| < 1e-5 L for an agent on the   */
/*               detector's link below L - 0.01: id detector, aux agent,    */
/*               decision counted.                                          */
/* With another run's log attached (orc_adopt_ties), a position threshold   */
/* whose own margin is below half the tolerance takes the decision that log */
/* holds for the same (t, class, id, aux); a near-tie route choice takes   */
/* the link that log chose for the same (t, agent) if it is a candidate;   */
/* a near-tie merge pair is swapped when that log ranked its second agent  */
/* first.  None found counts as unmatched.  Such a log may come from a run */
/* with other rounding of the same step (double positions, or a Gumbel    */
/* transform through another log implementation).                          */
/* ------------------------------------------------------------------------ */
enum { TIE_CHOICE = 0, TIE_MERGE = 1, TIE_ARRIVE = 2, TIE_VACANT = 3, TIE_DETECT = 4 };

static int cmp_tie(const void *a, const void *b)
{
    const int32_t *x = a, *y = b;
    for (int k = 0; k < 4; ++k) if (x[k] != y[k]) return x[k] < y[k] ? -1 : 1;
    return 0;
}

static void tie_push(orc_t *o, int32_t cls, int32_t id, int32_t aux, int32_t dec)
{
    VPUSH(o->ties, o->t); VPUSH(o->ties, cls); VPUSH(o->ties, id); VPUSH(o->ties, aux); VPUSH(o->ties, dec);
}

/* decision `own` of a position threshold at margin m (tolerance tol) */
static int tie_threshold(orc_t *o, int32_t cls, int32_t id, int32_t aux, int own, pos_t m, pos_t tol)
{
    pos_t am = m < 0 ? -m : m;
    if (!(am < tol)) return own;
    int dec = own;
    if (o->adopt_n > 0 && am < tol / 2) {
        int32_t key[4] = { o->t, cls, id, aux };
        const int32_t *f = bsearch(key, o->adopt, (size_t)o->adopt_n, 5 * sizeof(int32_t), cmp_tie);
        if (f) { dec = f[4]; o->n_adopted++; o->n_flipped += dec != own; }
        else o->n_unmatched++;
    }
    tie_push(o, cls, id, aux, dec);
    return dec;
}

/* the adopted log's record for (t, class, id), any aux, or NULL */
static int cmp_tie3(const void *a, const void *b)
{
    const int32_t *x = a, *y = b;
    for (int k = 0; k < 3; ++k) if (x[k] != y[k]) return x[k] < y[k] ? -1 : 1;
    return 0;
}

static const int32_t *adopted3(const orc_t *o, int32_t cls, int32_t id)
{
    if (o->adopt_n <= 0) return NULL;
    int32_t key[3] = { o->t, cls, id };
    return bsearch(key, o->adopt, (size_t)o->adopt_n, 5 * sizeof(int32_t), cmp_tie3);
}

static const int32_t *adopted4(const orc_t *o, int32_t cls, int32_t id, int32_t aux)
{
    if (o->adopt_n <= 0) return NULL;
    int32_t key[4] = { o->t, cls, id, aux };
    return bsearch(key, o->adopt, (size_t)o->adopt_n, 5 * sizeof(int32_t), cmp_tie);
}

int64_t orc_tie_count(const orc_t *o) { return o->ties.n / 5; }
void orc_tie_log(const orc_t *o, int32_t *out) { if (o->ties.n) memcpy(out, o->ties.p, 4 * (size_t)o->ties.n); }
void orc_tie_stats(const orc_t *o, int64_t *adopted, int64_t *unmatched, int64_t *flipped)
{
    *adopted = o->n_adopted;
    *unmatched = o->n_unmatched;
    *flipped = o->n_flipped;
}
/* Relative margin below which a route choice or merge pair counts as a near
 * tie (default 1e-12).  Tests widen it to exercise adoption on ordinary
 * decisions. */
void orc_set_tie_tolerance(orc_t *o, double rel) { o->tie_rel = rel; }
/* Take the decisions of another run's near-tie log (n records of 5 int32). */
void orc_adopt_ties(orc_t *o, const int32_t *log, int64_t n)
{
    free((void *)o->adopt);
    int32_t *c = malloc(sizeof(int32_t) * 5 * (size_t)(n > 0 ? n : 1));
    if (n > 0) memcpy(c, log, sizeof(int32_t) * 5 * (size_t)n);
    qsort(c, (size_t)n, 5 * sizeof(int32_t), cmp_tie);
    o->adopt = c;
    o->adopt_n = n;
}

/* Route choice of one agent standing at node v, coming from link `from`
 * (-1 for an origin queue).  Returns the chosen link, or CH_STUCK. */
static int32_t choose(orc_t *o, int32_t a, int32_t v, int32_t from)
{
    int32_t d = o->agent_didx[a];
    const double *dist = o->dist + (int64_t)d * o->in.n_nodes;
    double best = -INFINITY, second = -INFINITY;
    int32_t arg = CH_STUCK;
    ch_rec cr = { a, from, CH_STUCK, 0, o->chl.n, from >= 0 ? (double)o->xhat[a] : 0.0 };
    for (int32_t k = o->out_off[v]; k < o->out_off[v + 1]; ++k) {
        int32_t m = o->out_lnk[k], c = k - o->out_off[v];
        if (!o->in.allow_uturn && from >= 0 && o->head[m] == o->tail[from]) continue;
        double dm = dist[o->head[m]];
        if (!(dm < INFINITY)) continue;
        double tff = (double)o->length[m] / (double)o->rspeed[m];
        double V = (double)o->beta[m] / (double)o->cost[m] - o->in.dest_logit_coef * (tff + dm);
        double g = orc_gumbel(o->in.seed, a, o->t, 0, c);
        double s = V + g;
        if (s > best) { second = best; best = s; arg = m; }
        else if (s > second) second = s;
        if (o->log_on) { VPUSH(o->chl, m); VPUSH(o->chr, tff + dm); VPUSH(o->chg, g); cr.n++; }
    }
    if (arg >= 0 && second > -INFINITY && best - second < o->tie_rel * (1.0 + fabs(best))) {
        o->ctr[5]++;
        /* another run's decision at this near tie, if it is a candidate here */
        const int32_t *f = adopted3(o, TIE_CHOICE, a);
        if (f) {
            int ok = 0;
            for (int32_t k = o->out_off[v]; k < o->out_off[v + 1]; ++k) {
                int32_t m = o->out_lnk[k];
                if (m != f[4] || !(dist[o->head[m]] < INFINITY)) continue;
                if (!o->in.allow_uturn && from >= 0 && o->head[m] == o->tail[from]) continue;
                ok = 1;
            }
            if (ok) {
                o->n_adopted++;
                if (f[4] != arg) { o->n_flipped++; arg = f[4]; }
            } else {
                o->n_unmatched++;
            }
        } else if (o->adopt_n > 0) {
            o->n_unmatched++;
        }
        tie_push(o, TIE_CHOICE, a, arg, arg);
    }
    if (o->log_on) { cr.chosen = arg; o->chidx[a] = o->chs.n; VPUSH(o->chs, cr); }
    return arg;
}

int orc_step(orc_t *o)
{
    const orc_inputs *in = &o->in;
    int32_t L = in->n_links, N = in->n_agents, O = in->n_origins, Nn = in->n_nodes;
    int32_t t = o->t;
    double dt = in->dt;
    step_rec sr = { t, 0, 0, 0, o->cf.n, o->mv.n, o->smp.n, 0, o->chs.n, o->mgs.n, 0, 0 };

    /* ---- release ---- */
    for (int32_t k = 0; k < O; ++k) {
        int32_t qn = o->q_off[k + 1] - o->q_off[k];
        const int32_t *q = o->q_list + o->q_off[k];
        if (o->ready) {
            while (o->rel_ptr[k] < qn && o->rstep[q[o->rel_ptr[k]]] <= t) {
                o->status[q[o->rel_ptr[k]]] = ST_QUEUED;
                o->rel_ptr[k]++; o->ctr[0]++;
            }
        } else {
            double inc = 0.0, t0 = t * dt, t1 = (t + 1) * dt;
            int32_t bcur = -1;
            for (int32_t b = 0; b < in->n_rate_bins; ++b) {
                double ov = rate_overlap(b * in->rate_bin_s, (b + 1) * in->rate_bin_s, t0, t1);
                if (ov > 0) { inc += (double)o->rates[(int64_t)k * in->n_rate_bins + b] * ov; bcur = b; }
            }
            o->D[k] += inc;
            while (o->rel_ptr[k] < qn && (double)(o->rel_ptr[k] + 1) <= o->D[k]) {
                int32_t a = q[o->rel_ptr[k]];
                double r = inc / dt;
                o->status[a] = ST_QUEUED;
                o->tstar[a] = t1 - (o->D[k] - (double)(o->rel_ptr[k] + 1)) / r;
                o->tstar_bin[a] = bcur;
                o->rel_t[a] = t;
                o->rel_ptr[k]++; o->ctr[0]++;
            }
        }
    }

    /* ---- order: bucket ON agents by link, sort each bucket ---- */
    for (int32_t j = 0; j <= L; ++j) o->bucket_off[j] = 0;
    for (int32_t i = 0; i < N; ++i) if (o->status[i] == ST_ON) o->bucket_off[o->link[i] + 1]++;
    for (int32_t j = 0; j < L; ++j) o->bucket_off[j + 1] += o->bucket_off[j];
    for (int32_t j = 0; j < L; ++j) o->head_cnt[j] = 0;
    for (int32_t i = 0; i < N; ++i)
        if (o->status[i] == ST_ON) o->bucket[o->bucket_off[o->link[i]] + o->head_cnt[o->link[i]]++] = i;
    g_sort_ctx = o;
    for (int32_t j = 0; j < L; ++j)
        qsort(o->bucket + o->bucket_off[j], (size_t)(o->bucket_off[j + 1] - o->bucket_off[j]),
              sizeof(int32_t), cmp_rank);

    /* ---- car-following (all inputs at time t) ---- */
    for (int32_t j = 0; j < L; ++j) {
        int32_t b0 = o->bucket_off[j], n = o->bucket_off[j + 1] - b0, ln = o->lanes[j];
        for (int32_t r = 0; r < n; ++r) {
            int32_t a = o->bucket[b0 + r];
            pos_t x = o->pos[a];
            pos_t xf = x + o->vfree[j];
            pos_t xn;
            int32_t br, lead = -1;
            if (r >= ln) {
                lead = o->bucket[b0 + r - ln];
                pos_t xc = o->pos[lead] - o->spacing[j];
                /* max(x, x_lead - s): ties go to the leader term */
                pos_t c = (x > xc) ? x : xc;
                int32_t cb = (x > xc) ? BR_STOP : BR_CONG;
                /* min(free, c): ties go to the free term */
                if (xf <= c) { xn = xf; br = BR_FREE; } else { xn = c; br = cb; }
            } else {
                xn = xf; br = BR_FREE;
            }
            pos_t Lj = (pos_t)o->length[j];
            int32_t cp = xn > Lj;
            o->xhat[a] = cp ? Lj : xn;
            o->rank[a] = r;
            o->leader_of[a] = lead;
            o->branch[a] = br;
            o->capped[a] = cp;
            if (o->log_on) {
                cf_rec c = { a, j, lead, br, cp, (double)x, (double)xn };
                o->cfidx[a] = (int32_t)(o->cf.n - sr.cf0);
                VPUSH(o->cf, c);
            }
        }
    }

    /* ---- per-link aggregates ---- */
    for (int32_t j = 0; j < L; ++j) {
        int32_t b0 = o->bucket_off[j], n = o->bucket_off[j + 1] - b0;
        int32_t h = 0, occ = 0;
        for (int32_t r = 0; r < n; ++r) {
            int32_t a = o->bucket[b0 + r];
            if (r > 0) {  /* order check on the updated positions */
                int32_t p = o->bucket[b0 + r - 1];
                if (o->xhat[p] < o->xhat[a]) o->ctr[7]++;
            }
            int capped_now = o->xhat[a] == (pos_t)o->length[j];   /* exact at the cap: no tie */
            int arrived = o->xhat[a] >= o->thr[j];
            if (!capped_now)
                arrived = tie_threshold(o, TIE_ARRIVE, a, j, arrived, o->xhat[a] - o->thr[j], o->tietol[j]);
            int occupies = tie_threshold(o, TIE_VACANT, a, j, o->xhat[a] <= o->spacing[j],
                                         o->xhat[a] - o->spacing[j], o->tietol[j]);
            if (arrived && h == r) h++;
            if (occupies) occ++;
        }
        o->head_cnt[j] = h;
        o->slots[j] = o->lanes[j] - occ > 0 ? o->lanes[j] - occ : 0;   /* free entry slots */
        o->B[j] += (double)o->cap_mult[j] * (double)o->cap[j] * (double)o->lanes[j] * dt;
        o->dB[j] += (double)o->cap[j] * (double)o->lanes[j] * dt;
        o->bacc[j] = o->B[j];
    }

    /* ---- link choice for heads and origin-queue fronts ---- */
    for (int32_t i = 0; i < N; ++i) { o->choice[i] = CH_STUCK; o->won[i] = 0; }
    for (int32_t j = 0; j < L; ++j) {
        int32_t b0 = o->bucket_off[j], v = o->head[j];
        for (int32_t r = 0; r < o->head_cnt[j]; ++r) {
            int32_t a = o->bucket[b0 + r];
            if (o->agent_dest[a] == v) o->choice[a] = CH_EXIT;
            else o->choice[a] = choose(o, a, v, j);
            o->mkey[a] = (double)o->alpha[j] + orc_gumbel(in->seed, a, t, 1, 0);
        }
    }
    int32_t *front = malloc(4 * (size_t)(O + 1));
    for (int32_t k = 0; k < O; ++k) {
        front[k] = -1;
        int32_t qn = o->rel_ptr[k];
        const int32_t *q = o->q_list + o->q_off[k];
        while (o->dep_ptr[k] < qn && o->status[q[o->dep_ptr[k]]] != ST_QUEUED) o->dep_ptr[k]++;
        if (o->dep_ptr[k] < qn) {
            int32_t a = q[o->dep_ptr[k]];
            front[k] = a;
            o->choice[a] = choose(o, a, o->origin_node[k], -1);
            o->mkey[a] = 1.0 + orc_gumbel(in->seed, a, t, 1, 0);
        }
    }

    /* ---- merge: per downstream link, top-k by merge key among its choosers ---- */
    mcand *cand = malloc(sizeof(mcand) * 256);
    int32_t ccap = 256;
    int32_t *w_beg = malloc(4 * (size_t)(L + 1)), *w_end = malloc(4 * (size_t)(L + 1));
    int32_t *winners = malloc(4 * (size_t)(N + 1));
    int32_t wn = 0;
    for (int32_t v = 0; v < Nn; ++v) {
        for (int32_t kk = o->out_off[v]; kk < o->out_off[v + 1]; ++kk) {
            int32_t m = o->out_lnk[kk], nc = 0;
            /* candidates: heads of links entering v, fronts of origins at v */
            for (int32_t q = o->in_off[v]; q < o->in_off[v + 1]; ++q) {
                int32_t j = o->in_lnk[q];
                for (int32_t r = 0; r < o->head_cnt[j]; ++r) {
                    int32_t a = o->bucket[o->bucket_off[j] + r];
                    if (o->choice[a] != m) continue;
                    if (nc == ccap) { ccap *= 2; cand = realloc(cand, sizeof(mcand) * (size_t)ccap); }
                    cand[nc++] = (mcand){ o->mkey[a], a };
                }
            }
            for (int32_t q = o->org_off[v]; q < o->org_off[v + 1]; ++q) {
                int32_t a = front[o->org_list[q]];
                if (a < 0 || o->choice[a] != m) continue;
                if (nc == ccap) { ccap *= 2; cand = realloc(cand, sizeof(mcand) * (size_t)ccap); }
                cand[nc++] = (mcand){ o->mkey[a], a };
            }
            qsort(cand, (size_t)nc, sizeof(mcand), cmp_mcand);
            for (int32_t c = 0; c + 1 < nc; ++c)
                if (cand[c].key - cand[c + 1].key < o->tie_rel * (1.0 + fabs(cand[c].key))) {
                    o->ctr[5]++;
                    /* another run that ranked the second of the pair first: take its order */
                    if (o->adopt_n > 0) {
                        int second_first = adopted4(o, TIE_MERGE, cand[c + 1].agent, m) != NULL;
                        int first_first = adopted4(o, TIE_MERGE, cand[c].agent, m) != NULL;
                        if (second_first && !first_first) {
                            mcand tmp = cand[c]; cand[c] = cand[c + 1]; cand[c + 1] = tmp;
                            o->n_adopted++; o->n_flipped++;
                        } else if (first_first) {
                            o->n_adopted++;
                        } else {
                            o->n_unmatched++;
                        }
                    }
                    tie_push(o, TIE_MERGE, cand[c].agent, m, 1);
                }
            int32_t kwin = nc < o->slots[m] ? nc : o->slots[m];
            if (o->log_on && kwin > 0) {
                mg_rec g = { m, nc, kwin, o->mgc.n };
                for (int32_t c = 0; c < nc; ++c) {
                    VPUSH(o->mgc, (int32_t)o->chidx[cand[c].agent]);
                    VPUSH(o->mgg, orc_gumbel(in->seed, cand[c].agent, t, 1, 0));
                    VPUSH(o->mgmv, 0);
                }
                VPUSH(o->mgs, g);
            }
            w_beg[m] = wn;
            for (int32_t c = 0; c < kwin; ++c) { o->won[cand[c].agent] = 1; winners[wn++] = cand[c].agent; }
            w_end[m] = wn;
        }
    }

    /* ---- resolve: FIFO over each link's heads, tokens for transfers ---- */
    int32_t *passed = calloc((size_t)N + 1, 4);
    int32_t *tokk = calloc((size_t)N + 1, 4);
    for (int32_t j = 0; j < L; ++j) {
        int32_t b0 = o->bucket_off[j], ntok = 0;
        for (int32_t r = 0; r < o->head_cnt[j]; ++r) {
            int32_t a = o->bucket[b0 + r];
            int32_t ch = o->choice[a];
            if (ch == CH_EXIT) { passed[a] = 1; continue; }
            if (ch >= 0 && o->won[a] && o->B[j] >= 1.0) {
                o->B[j] -= 1.0;
                passed[a] = 1;
                tokk[a] = ntok++;
                continue;
            }
            if (ch == CH_STUCK) o->ctr[6]++;
            break;
        }
    }
    for (int32_t k = 0; k < O; ++k) if (front[k] >= 0 && o->choice[front[k]] >= 0 && o->won[front[k]]) passed[front[k]] = 1;
    if (o->log_on)   /* which merge candidates of this step actually moved */
        for (int64_t gi = sr.mg0; gi < o->mgs.n; ++gi)
            for (int32_t c = 0; c < o->mgs.p[gi].n; ++c) {
                int64_t q = o->mgs.p[gi].c0 + c;
                o->mgmv.p[q] = passed[o->chs.p[o->mgc.p[q]].agent];
            }

    /* ---- apply: stayers take the capped position, movers change link ---- */
    for (int32_t j = 0; j < L; ++j) {
        int32_t b0 = o->bucket_off[j], n = o->bucket_off[j + 1] - b0;
        for (int32_t r = 0; r < n; ++r) {
            int32_t a = o->bucket[b0 + r];
            if (passed[a]) continue;
            o->pos[a] = o->xhat[a];
        }
        for (int32_t r = 0; r < o->head_cnt[j]; ++r) {
            int32_t a = o->bucket[b0 + r];
            if (!passed[a]) break;
            o->E[j]++;
            if (o->choice[a] == CH_EXIT) {
                o->status[a] = ST_EXITED;
                o->link[a] = -1;
                o->ctr[3]++;
                if (o->log_on) { mv_rec m = { a, MV_EXIT, j, -1, 0, 0.0, 0.0, -1, 0, sr.cf0 + o->cfidx[a], 0, 0.0 }; VPUSH(o->mv, m); }
            }
        }
    }
    /* entrants of each link in merge-key order get consecutive sequence numbers */
    for (int32_t m = 0; m < L; ++m) {
        for (int32_t q = w_beg[m]; q < w_end[m]; ++q) {
            int32_t a = winners[q];
            if (!passed[a]) continue;
            int32_t from = (o->status[a] == ST_ON) ? o->link[a] : -1;
            if (o->log_on) {
                mv_rec mr;
                if (from >= 0) mr = (mv_rec){ a, MV_TRANSFER, from, m, tokk[a], 0.0, o->bacc[from], -1, 0, sr.cf0 + o->cfidx[a], t, o->dB[from] };
                else mr = (mv_rec){ a, MV_DEPART, o->agent_origin[a], m, 0, o->tstar[a], 0.0, o->tstar_bin[a], o->qidx[a], -1, o->rel_t[a], 0.0 };
                VPUSH(o->mv, mr);
            }
            if (from >= 0) o->ctr[4]++;
            else { o->ctr[1]++; o->dep_ptr[o->agent_origin[a]]++; }
            o->status[a] = ST_ON;
            o->link[a] = m;
            o->pos[a] = (pos_t)0;
            o->seq[a] = o->next_seq[m]++;
        }
    }
    /* idle cap; the clipped level no longer depends on the multiplier */
    for (int32_t j = 0; j < L; ++j) {
        int clip = o->B[j] > 1.0;
        if (clip) { o->B[j] = 1.0; o->dB[j] = 0.0; }
        if (o->log_on) VPUSH(o->capf, (uint8_t)clip);
    }

    /* ---- observe ---- */
    int64_t active = 0, onnet = 0;
    for (int32_t i = 0; i < N; ++i) {
        if (o->status[i] == ST_ON) { active++; onnet++; }
        else if (o->status[i] == ST_QUEUED) active++;
    }
    o->ctr[2] = onnet;
    o->ttt += dt * (double)active;
    if (in->count_bin_steps > 0 && (t + 1) % in->count_bin_steps == 0) {
        int32_t kb = (t + 1) / in->count_bin_steps - 1;
        if (kb < in->n_count_bins) {
            sr.sample_k = kb + 1;
            /* agents by link after the step */
            for (int32_t j = 0; j <= L; ++j) o->bucket_off[j] = 0;
            for (int32_t i = 0; i < N; ++i) if (o->status[i] == ST_ON) o->bucket_off[o->link[i] + 1]++;
            for (int32_t j = 0; j < L; ++j) o->bucket_off[j + 1] += o->bucket_off[j];
            for (int32_t j = 0; j < L; ++j) o->head_cnt[j] = 0;
            for (int32_t i = 0; i < N; ++i)
                if (o->status[i] == ST_ON) o->bucket[o->bucket_off[o->link[i]] + o->head_cnt[o->link[i]]++] = i;
            for (int32_t d = 0; d < in->n_detectors; ++d) {
                int32_t j = o->det_link[d];
                int64_t c = o->E[j];
                for (int32_t q = o->bucket_off[j]; q < o->bucket_off[j + 1]; ++q) {
                    int32_t i = o->bucket[q];
                    int counted = o->pos[i] >= (pos_t)o->det_pos[d];
                    if (o->pos[i] < o->thr[j])
                        counted = tie_threshold(o, TIE_DETECT, d, i, counted, o->pos[i] - (pos_t)o->det_pos[d],
                                                o->tietol[j]);
                    if (counted) c++;
                    if (o->log_on) { smp_rec sm = { d, i, (double)o->pos[i] }; VPUSH(o->smp, sm); }
                }
                o->counts[(int64_t)d * in->n_count_bins + kb] = (double)(c - o->cprev[d]);
                o->cprev[d] = c;
            }
        }
    }
    if (o->log_on) {
        sr.n_cf = (int32_t)(o->cf.n - sr.cf0);
        sr.n_mv = (int32_t)(o->mv.n - sr.mv0);
        sr.n_smp = (int32_t)(o->smp.n - sr.smp0);
        sr.n_ch = (int32_t)(o->chs.n - sr.ch0);
        sr.n_mg = (int32_t)(o->mgs.n - sr.mg0);
        VPUSH(o->steps, sr);
    }
    free(front); free(cand); free(winners); free(w_beg); free(w_end);
    free(passed); free(tokk);
    o->t++;
    return 0;
}

int orc_rollout(orc_t *o, int32_t T)
{
    for (int32_t k = 0; k < T; ++k) orc_step(o);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* accessors                                                                */
/* ------------------------------------------------------------------------ */
void orc_get_state(const orc_t *o, int32_t *status, int32_t *link, double *pos, int32_t *seq)
{
    for (int32_t i = 0; i < o->in.n_agents; ++i) {
        if (status) status[i] = o->status[i];
        if (link) link[i] = o->link[i];
        if (pos) pos[i] = (double)o->pos[i];
        if (seq) seq[i] = o->seq[i];
    }
}
void orc_get_link_state(const orc_t *o, double *B, int64_t *E, int32_t *next_seq)
{
    for (int32_t j = 0; j < o->in.n_links; ++j) {
        if (B) B[j] = o->B[j];
        if (E) E[j] = o->E[j];
        if (next_seq) next_seq[j] = o->next_seq[j];
    }
}
void orc_get_counters(const orc_t *o, int64_t *c) { for (int k = 0; k < 8; ++k) c[k] = o->ctr[k]; }
void orc_get_counts(const orc_t *o, double *counts, double *ttt)
{
    int64_t n = (int64_t)o->in.n_detectors * o->in.n_count_bins;
    for (int64_t k = 0; k < n; ++k) counts[k] = o->counts[k];
    if (ttt) *ttt = o->ttt;
}
int32_t orc_n_dest(const orc_t *o) { return o->n_dest; }
void orc_get_dist(const orc_t *o, double *out)
{
    memcpy(out, o->dist, sizeof(double) * (size_t)o->n_dest * (size_t)o->in.n_nodes);
}
void orc_get_origin_state(const orc_t *o, double *D, int32_t *rel, int32_t *dep)
{
    for (int32_t k = 0; k < o->in.n_origins; ++k) {
        if (D) D[k] = o->D[k];
        if (rel) rel[k] = o->rel_ptr[k];
        if (dep) dep[k] = o->dep_ptr[k];
    }
}
int32_t orc_time(const orc_t *o) { return o->t; }

/* ------------------------------------------------------------------------ */
/* State hand-off (the paper's nowcast starts from a state X(T); Methods,   */
/* "Optimization", and the nowcasting results): the whole forward state as  */
/* one flat blob, and its import into an oracle created from the same       */
/* inputs (and the same placed agents).  The blob holds, in order: t, N, L, */
/* O, detectors, bins (int32); per agent status, link, seq, release step,   */
/* release-time bin (int32), position (pos_t), release time (double); per   */
/* origin release and departure pointers (int32), accumulator (double); per */
/* link next sequence (int32), B, dB (double), E (int64); per detector the  */
/* last sample (int64) and its counts (double), travel time (double) and    */
/* the eight counters (int64).  An imported oracle keeps no decision log of */
/* the past, so it cannot run the reverse sweep (orc_backward fails).       */
/* ------------------------------------------------------------------------ */
typedef struct { char *p; size_t n; int wr; } blob_t;
static void bput(blob_t *b, void *x, size_t n)
{
    if (b->p) { if (b->wr) memcpy(b->p + b->n, x, n); else memcpy(x, b->p + b->n, n); }
    b->n += n;
}
static size_t state_io(orc_t *o, char *p, int wr)
{
    const orc_inputs *in = &o->in;
    int32_t N = in->n_agents, L = in->n_links, O = in->n_origins, Dd = in->n_detectors, nb = in->n_count_bins;
    blob_t b = { p, 0, wr };
    int32_t hdr[6] = { o->t, N, L, O, Dd, nb };
    bput(&b, hdr, sizeof hdr);
    if (p && !wr) o->t = hdr[0];
    bput(&b, o->status, 4 * (size_t)N); bput(&b, o->link, 4 * (size_t)N); bput(&b, o->seq, 4 * (size_t)N);
    bput(&b, o->rel_t, 4 * (size_t)N); bput(&b, o->tstar_bin, 4 * (size_t)N);
    bput(&b, o->pos, sizeof(pos_t) * (size_t)N); bput(&b, o->tstar, 8 * (size_t)N);
    bput(&b, o->rel_ptr, 4 * (size_t)O); bput(&b, o->dep_ptr, 4 * (size_t)O); bput(&b, o->D, 8 * (size_t)O);
    bput(&b, o->next_seq, 4 * (size_t)L); bput(&b, o->B, 8 * (size_t)L); bput(&b, o->dB, 8 * (size_t)L);
    bput(&b, o->E, 8 * (size_t)L);
    bput(&b, o->cprev, 8 * (size_t)Dd); bput(&b, o->counts, 8 * (size_t)Dd * (size_t)nb);
    bput(&b, &o->ttt, 8); bput(&b, o->ctr, sizeof o->ctr);
    return b.n;
}
int64_t orc_state_size(orc_t *o) { return (int64_t)state_io(o, NULL, 1); }
void orc_export_state(orc_t *o, void *blob) { state_io(o, blob, 1); }
/* 0 on success, -1 if the blob's sizes do not match this oracle's inputs */
int orc_import_state(orc_t *o, const void *blob, int64_t n)
{
    const orc_inputs *in = &o->in;
    int32_t hdr[6];
    if (n < (int64_t)sizeof hdr || n != orc_state_size(o)) return -1;
    memcpy(hdr, blob, sizeof hdr);
    if (hdr[1] != in->n_agents || hdr[2] != in->n_links || hdr[3] != in->n_origins ||
        hdr[4] != in->n_detectors || hdr[5] != in->n_count_bins) return -1;
    state_io(o, (char *)blob, 0);
    o->cf.n = o->mv.n = o->smp.n = o->steps.n = o->capf.n = 0;
    o->chs.n = o->chl.n = o->chr.n = o->chg.n = o->mgs.n = o->mgc.n = o->mgmv.n = o->mgg.n = 0;
    o->ties.n = 0;
    o->have_base = 0;
    o->restored = 1;
    return 0;
}
int64_t orc_log_sizes(const orc_t *o, int64_t *out)
{
    out[0] = o->cf.n; out[1] = o->mv.n; out[2] = o->smp.n; out[3] = o->steps.n;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Frozen surrogate: the forward with every discrete decision taken from    */
/* the recorded log and every stop_gradient replaced by its value at the   */
/* base parameters.  All arithmetic in double.  Its exact derivative is the */
/* gradient the adjoint computes; central differences of it pin the adjoint.*/
/*                                                                          */
/* Parameters (NULL -> the values given at create): u[L], kappa[L],        */
/* rates[O x B], cap_mult[L].                                               */
/* Outputs: soft counts [det x bins], surrogate total travel                */
/* time, positions of agents on the network at the end (0 elsewhere).       */
/* First call with record_base = 1 at the base parameters.                  */
/* ------------------------------------------------------------------------ */
static double sigm(double z) { return 1.0 / (1.0 + exp(-z)); }

/* Straight-through terms of the node model (SI-B).  Link choice: pi = softmax((V + g)/tau) over
 * the chooser's valid candidate links, V = beta/c - theta (t_ff + D); the sample is
 * onehot(pi) + pi - sg(pi).  Merge of a target link: V' = alpha_from * l (l the chooser's link-
 * choice entry for the target), pi' = softmax((V' + g')/tau) over the candidates; with k winners,
 * k stages, stage s over the candidates not picked before it (s = 0 alone is the paper's case).
 * pi at the chosen link of chooser record r, with parameters (beta, cost, theta); all n in p. */
static double choice_pi(const orc_t *o, int64_t r, const double *beta, const double *cost, double theta, double *p)
{
    const ch_rec *c = &o->chs.p[r];
    double tau = o->in.gumbel_tau, mx = -INFINITY, sum = 0.0, at = 0.0;
    for (int32_t k = 0; k < c->n; ++k) {
        int32_t m = o->chl.p[c->c0 + k];
        double y = (beta[m] / cost[m] - theta * o->chr.p[c->c0 + k] + o->chg.p[c->c0 + k]) / tau;
        p[k] = y;
        if (y > mx) mx = y;
    }
    for (int32_t k = 0; k < c->n; ++k) { p[k] = exp(p[k] - mx); sum += p[k]; }
    for (int32_t k = 0; k < c->n; ++k) { p[k] /= sum; if (o->chl.p[c->c0 + k] == c->chosen) at = p[k]; }
    return at;
}

/* softmax of y/tau over entries [s, n) (a merge stage) into q[s..n) */
static void stage_softmax(const double *y, int32_t s, int32_t n, double tau, double *q)
{
    double mx = -INFINITY, sum = 0.0;
    for (int32_t c = s; c < n; ++c) if (y[c] / tau > mx) mx = y[c] / tau;
    for (int32_t c = s; c < n; ++c) { q[c] = exp(y[c] / tau - mx); sum += q[c]; }
    for (int32_t c = s; c < n; ++c) q[c] /= sum;
}

int orc_frozen_eval(orc_t *o, const double *u_in, const double *kappa_in, const double *rates_in,
                    const double *capm_in, const double *beta_in, const double *cost_in, const double *alpha_in,
                    const double *theta_in, int record_base, double *out_counts, double *out_ttt, double *out_pos)
{
    const orc_inputs *in = &o->in;
    int32_t L = in->n_links, N = in->n_agents, O = in->n_origins, Bn = in->n_rate_bins;
    int32_t Dd = in->n_detectors, nb = in->n_count_bins;
    if (!o->log_on || o->steps.n == 0) return -1;
    if (!record_base && !o->have_base) return -2;
    if (record_base) {
        free(o->base_x1); free(o->base_xhat); free(o->base_psi); free(o->base_sig);
        o->base_x1 = malloc(8 * (size_t)(o->cf.n + 1));
        o->base_xhat = malloc(8 * (size_t)(o->cf.n + 1));
        o->base_psi = malloc(8 * (size_t)(o->mv.n + 1));
        o->base_sig = malloc(8 * (size_t)(o->smp.n + 1));
    }
    double *u = malloc(8 * (size_t)L), *kap = malloc(8 * (size_t)L), *capm = malloc(8 * (size_t)L);
    for (int32_t j = 0; j < L; ++j) {
        u[j] = u_in ? u_in[j] : (double)o->u[j];
        kap[j] = kappa_in ? kappa_in[j] : (double)o->kappa[j];
        capm[j] = capm_in ? capm_in[j] : (double)o->cap_mult[j];
    }
    /* token buckets replayed with the logged consumption and idle-cap clips */
    double *Bf = calloc((size_t)L + 1, 8), *Bacc = calloc((size_t)L + 1, 8);
    /* straight-through parameters and per-agent merge perturbation of this step */
    double *bet = malloc(8 * (size_t)L), *cst = malloc(8 * (size_t)L), *alp = malloc(8 * (size_t)L);
    for (int32_t j = 0; j < L; ++j) {
        bet[j] = beta_in ? beta_in[j] : (double)o->beta[j];
        cst[j] = cost_in ? cost_in[j] : (double)o->cost[j];
        alp[j] = alpha_in ? alpha_in[j] : (double)o->alpha[j];
    }
    const double theta = theta_in ? *theta_in : in->dest_logit_coef, bigm = in->big_m, tau = in->gumbel_tau;
    double *dA = calloc((size_t)N + 1, 8), *pw = malloc(8 * 256), *yv = NULL, *qv = NULL;
    int64_t ycap = 0, pim_k = 0;
    if (record_base) {
        free(o->base_pi); free(o->base_pim);
        int64_t npim = 0;
        for (int64_t gi = 0; gi < o->mgs.n; ++gi)
            for (int32_t st = 0; st < o->mgs.p[gi].k; ++st) npim += o->mgs.p[gi].n - st;
        o->base_pi = malloc(8 * (size_t)(o->chs.n + 1));
        o->base_pim = malloc(8 * (size_t)(npim + 1));
        for (int64_t r = 0; r < o->chs.n; ++r) {
            const ch_rec *c = &o->chs.p[r];
            double *pp = malloc(8 * (size_t)(c->n + 1));
            o->base_pi[r] = choice_pi(o, r, bet, cst, theta, pp);
            free(pp);
        }
    }
    double *x = calloc((size_t)N, 8), *xn = calloc((size_t)N, 8);
    int32_t *on = calloc((size_t)N, 4);
    /* agents placed at t = 0 */
    double *cint = calloc((size_t)Dd * (size_t)(nb > 0 ? nb : 1) + 1, 8);
    double *csoft = calloc((size_t)Dd * (size_t)(nb > 0 ? nb : 1) + 1, 8);
    /* the integer part of the cumulative counts comes straight from the forward's counts */
    for (int32_t d = 0; d < Dd; ++d) {
        double acc = 0.0;
        for (int32_t k = 0; k < nb; ++k) { acc += o->counts[(int64_t)d * nb + k]; cint[(int64_t)d * nb + k] = acc; }
    }
    double ttt_soft = 0.0;
    /* initial positions: agents that were ON before the first logged step */
    {
        const step_rec *s0 = &o->steps.p[0];
        for (int64_t c = s0->cf0; c < s0->cf0 + s0->n_cf; ++c) { x[o->cf.p[c].agent] = o->cf.p[c].x0; on[o->cf.p[c].agent] = 1; }
    }
    for (int64_t si = 0; si < o->steps.n; ++si) {
        const step_rec *s = &o->steps.p[si];
        for (int32_t j = 0; j < L; ++j) {
            Bf[j] += capm[j] * (double)o->cap[j] * (double)o->lanes[j] * in->dt;
            Bacc[j] = Bf[j];
        }
        for (int64_t c = s->cf0; c < s->cf0 + s->n_cf; ++c) {
            const cf_rec *r = &o->cf.p[c];
            int32_t j = r->link;
            double xp;
            if (r->branch == BR_FREE) xp = x[r->agent] + u[j] * in->dt;
            else if (r->branch == BR_CONG) xp = x[r->leader] - (double)in->platoon / kap[j];
            else xp = x[r->agent];
            if (record_base) o->base_x1[c] = xp;
            double xh = r->capped ? (double)o->length[j] + xp - o->base_x1[c] : xp;
            if (record_base) o->base_xhat[c] = xh;
            xn[r->agent] = xh;
        }
        for (int64_t c = s->cf0; c < s->cf0 + s->n_cf; ++c) x[o->cf.p[c].agent] = xn[o->cf.p[c].agent];
        /* straight-through merge perturbations: da = sum over stages of pi' - sg(pi') */
        for (int64_t gi = s->mg0; gi < s->mg0 + s->n_mg; ++gi) {
            const mg_rec *g = &o->mgs.p[gi];
            if (g->n > ycap) { ycap = 2 * g->n; yv = realloc(yv, 8 * (size_t)ycap); qv = realloc(qv, 8 * (size_t)ycap); }
            for (int32_t c = 0; c < g->n; ++c) {
                int64_t r = o->mgc.p[g->c0 + c];
                const ch_rec *cr = &o->chs.p[r];
                double *pp = cr->n <= 256 ? pw : malloc(8 * (size_t)cr->n);
                double pi = choice_pi(o, r, bet, cst, theta, pp);
                if (pp != pw) free(pp);
                double l = 1.0 + pi - o->base_pi[r];
                double al = cr->from >= 0 ? alp[cr->from] : 1.0;
                yv[c] = al * l + o->mgg.p[g->c0 + c];
                dA[cr->agent] = 0.0;
            }
            for (int32_t st = 0; st < g->k; ++st) {
                stage_softmax(yv, st, g->n, tau, qv);
                for (int32_t c = st; c < g->n; ++c) {
                    if (record_base) o->base_pim[pim_k] = qv[c];
                    dA[o->chs.p[o->mgc.p[g->c0 + c]].agent] += qv[c] - o->base_pim[pim_k];
                    ++pim_k;
                }
            }
            /* candidates that stayed on their link: the X - (M + x) I_remove term of the SI-B transfer update */
            for (int32_t c = 0; c < g->n; ++c) {
                const ch_rec *cr = &o->chs.p[o->mgc.p[g->c0 + c]];
                if (!o->mgmv.p[g->c0 + c] && cr->from >= 0) x[cr->agent] -= (bigm + x[cr->agent]) * dA[cr->agent];
            }
        }
        for (int64_t c = s->mv0; c < s->mv0 + s->n_mv; ++c) {
            const mv_rec *m = &o->mv.p[c];
            if (m->kind == MV_TRANSFER) {
                /* admission-time graft: the head's token became available at
                 * t_tok = (t+1)dt - (B_pre - 1)/(m q n), B_pre the level before its
                 * token; psi = -u_to * t_tok with u_to frozen */
                int32_t j = m->from;
                double mqn = capm[j] * (double)o->cap[j] * (double)o->lanes[j];
                double bpre = Bacc[j] - (double)m->tok_k;
                double ttok = (double)(s->t + 1) * in->dt - (bpre - 1.0) / mqn;
                double psi = -(double)o->u[m->to] * ttok;
                if (record_base) o->base_psi[c] = psi;
                Bf[j] -= 1.0;
                /* grafted entry: value 0, history of the capped position and of the token time;
                 * straight-through add: (M + x - sg x) (1 + da) at the new link */
                double tg = x[m->agent] - o->base_xhat[m->cfi];
                x[m->agent] = 0.0 + tg + (psi - o->base_psi[c]) + tg * dA[m->agent] + bigm * dA[m->agent];
            } else if (m->kind == MV_EXIT) {
                /* exit earlier by (xhat - sg xhat)/u of the last link */
                ttt_soft -= (x[m->agent] - o->base_xhat[m->cfi]) / (double)o->u[m->from];
                on[m->agent] = 0;
            } else {
                /* departure-time graft: psi = -u_m * t*(rates), u_m frozen */
                double tst = m->tstar;
                if (Bn > 0) {
                    int32_t k = m->from, b = m->rate_bin;
                    const double *rr = NULL;
                    double *tmp = NULL;
                    if (rates_in) rr = rates_in + (int64_t)k * Bn;
                    else {
                        tmp = malloc(8 * (size_t)Bn);
                        for (int32_t q = 0; q < Bn; ++q) tmp[q] = (double)o->rates[(int64_t)k * Bn + q];
                        rr = tmp;
                    }
                    double tstep = (double)m->rel_t * in->dt;   /* the release step */
                    double Dt0 = 0.0;
                    for (int32_t q = 0; q < Bn; ++q) Dt0 += rr[q] * rate_overlap(q * in->rate_bin_s, (q + 1) * in->rate_bin_s, 0.0, tstep);
                    tst = tstep + ((double)(m->qidx + 1) - Dt0) / rr[b];
                    free(tmp);
                }
                double psi = -(double)o->u[m->to] * tst;
                if (record_base) o->base_psi[c] = psi;
                x[m->agent] = 0.0 + (psi - o->base_psi[c]) + bigm * dA[m->agent];
                on[m->agent] = 1;
            }
        }
        for (int32_t j = 0; j < L; ++j) if (o->capf.p[si * L + j]) Bf[j] = 1.0;
        if (s->sample_k > 0) {
            int32_t kb = s->sample_k - 1;
            for (int64_t c = s->smp0; c < s->smp0 + s->n_smp; ++c) {
                const smp_rec *r = &o->smp.p[c];
                int32_t d = r->det, j = o->det_link[d];
                double sc = 5.0 / (double)o->length[j];
                double sg = sigm(sc * (x[r->agent] - (double)o->det_pos[d]));
                if (record_base) o->base_sig[c] = sg;
                csoft[(int64_t)d * nb + kb] += sg - o->base_sig[c];
            }
        }
    }
    if (out_counts) {
        for (int32_t d = 0; d < Dd; ++d)
            for (int32_t k = 0; k < nb; ++k) {
                double c1 = cint[(int64_t)d * nb + k] + csoft[(int64_t)d * nb + k];
                double c0 = k > 0 ? cint[(int64_t)d * nb + k - 1] + csoft[(int64_t)d * nb + k - 1] : 0.0;
                out_counts[(int64_t)d * nb + k] = c1 - c0;
            }
    }
    if (out_ttt) *out_ttt = o->ttt + ttt_soft;
    if (out_pos) for (int32_t i = 0; i < N; ++i) out_pos[i] = (o->status[i] == ST_ON) ? x[i] : 0.0;
    if (record_base) o->have_base = 1;
    free(u); free(kap); free(capm); free(Bf); free(Bacc); free(x); free(xn); free(on); free(cint); free(csoft);
    free(bet); free(cst); free(alp); free(dA); free(pw); free(yv); free(qv);
    (void)O;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reverse sweep over the log: the exact derivative of the frozen surrogate */
/* at the base parameters (the straight-through and grafting conventions    */
/* of SI-A/SI-B/SI-C/SI-D).  Cotangents: dL/dcounts [det x bins], dL/dTTT,  */
/* dL/d(final positions) [N].  Gradients (accumulated, caller zeroes):      */
/* g_u[L], g_kappa[L], g_rates[O x B], g_capm[L], and through the         */
/* straight-through node model g_beta[L], g_cost[L], g_alpha[L], g_theta[1] */
/* (each may be NULL).  flags bit 0: no transfer graft.                     */
/* ------------------------------------------------------------------------ */
int orc_backward(orc_t *o, const double *gQ, double gT, const double *gx,
                 double *g_u, double *g_kappa, double *g_rates, double *g_capm,
                 double *g_beta, double *g_cost, double *g_alpha, double *g_theta, int flags)
{
    const orc_inputs *in = &o->in;
    int32_t N = in->n_agents, Bn = in->n_rate_bins, nb = in->n_count_bins;
    if (!o->log_on || o->restored) return -1;
    double *adj = calloc((size_t)N, 8), *nadj = calloc((size_t)N, 8);
    const int ste = g_beta || g_cost || g_alpha || g_theta;
    double *bb = malloc(8 * (size_t)(in->n_links + 1)), *cc = malloc(8 * (size_t)(in->n_links + 1));
    for (int32_t j = 0; j < in->n_links; ++j) { bb[j] = (double)o->beta[j]; cc[j] = (double)o->cost[j]; }
    if (gx) for (int32_t i = 0; i < N; ++i) if (o->status[i] == ST_ON) adj[i] = gx[i];
    for (int64_t si = o->steps.n - 1; si >= 0; --si) {
        const step_rec *s = &o->steps.p[si];
        /* counts sampled at the end of this step */
        if (s->sample_k > 0 && gQ) {
            int32_t kb = s->sample_k - 1;
            for (int64_t c = s->smp0; c < s->smp0 + s->n_smp; ++c) {
                const smp_rec *r = &o->smp.p[c];
                int32_t d = r->det, j = o->det_link[d];
                double gC = gQ[(int64_t)d * nb + kb] - (kb + 1 < nb ? gQ[(int64_t)d * nb + kb + 1] : 0.0);
                double sc = 5.0 / (double)o->length[j];
                double sg = sigm(sc * (r->x - (double)o->det_pos[d]));
                adj[r->agent] += gC * sc * sg * (1.0 - sg);
            }
        }
        /* straight-through node model (SI-B), adjoints of the positions after the step:
         * a merge candidate's share of the transfer update is G = M adj(new) if it moved, and
         * -(M + x_hat) adj(stay) if it stayed on its link (an origin front that stayed has none) */
        if (ste) {
            const double bigm = in->big_m, tau = in->gumbel_tau, theta = in->dest_logit_coef;
            for (int64_t gi = s->mg0; gi < s->mg0 + s->n_mg; ++gi) {
                const mg_rec *g = &o->mgs.p[gi];
                double *y = malloc(8 * (size_t)g->n), *G = malloc(8 * (size_t)g->n);
                double *q = malloc(8 * (size_t)g->n), *dVp = calloc((size_t)g->n, 8);
                for (int32_t c = 0; c < g->n; ++c) {
                    const ch_rec *cr = &o->chs.p[o->mgc.p[g->c0 + c]];
                    double al = cr->from >= 0 ? (double)o->alpha[cr->from] : 1.0;
                    y[c] = al + o->mgg.p[g->c0 + c];
                    if (o->mgmv.p[g->c0 + c]) G[c] = bigm * adj[cr->agent];
                    else G[c] = cr->from >= 0 ? -(bigm + cr->xh) * adj[cr->agent] : 0.0;
                }
                for (int32_t st = 0; st < g->k; ++st) {
                    stage_softmax(y, st, g->n, tau, q);
                    double sg = 0.0;
                    for (int32_t c = st; c < g->n; ++c) sg += q[c] * G[c];
                    for (int32_t c = st; c < g->n; ++c) dVp[c] += q[c] / tau * (G[c] - sg);
                }
                for (int32_t c = 0; c < g->n; ++c) {
                    int64_t r = o->mgc.p[g->c0 + c];
                    const ch_rec *cr = &o->chs.p[r];
                    double al = cr->from >= 0 ? (double)o->alpha[cr->from] : 1.0;
                    if (g_alpha && cr->from >= 0) g_alpha[cr->from] += dVp[c];   /* dV'/d alpha = l = 1 */
                    double gam = al * dVp[c];                                      /* dL/d l at the target */
                    double *p = malloc(8 * (size_t)(cr->n + 1));
                    double ps = choice_pi(o, r, bb, cc, theta, p);
                    for (int32_t k = 0; k < cr->n; ++k) {
                        int32_t m2 = o->chl.p[cr->c0 + k];
                        double dV = gam / tau * ps * ((m2 == cr->chosen ? 1.0 : 0.0) - p[k]);
                        if (g_beta) g_beta[m2] += dV / (double)o->cost[m2];
                        if (g_cost) g_cost[m2] -= (double)o->beta[m2] / ((double)o->cost[m2] * (double)o->cost[m2]) * dV;
                        if (g_theta) g_theta[0] -= o->chr.p[cr->c0 + k] * dV;
                    }
                    free(p);
                }
                free(y); free(G); free(q); free(dVp);
            }
        }
        /* moves */
        for (int64_t c = s->mv0; c < s->mv0 + s->n_mv; ++c) {
            const mv_rec *m = &o->mv.p[c];
            if (m->kind == MV_EXIT) {
                adj[m->agent] = -gT / (double)o->u[m->from];
            } else if (m->kind == MV_DEPART) {
                if (Bn > 0 && g_rates) {
                    int32_t k = m->from;
                    double r = (double)o->rates[(int64_t)k * Bn + m->rate_bin];
                    for (int32_t b = 0; b < Bn; ++b) {
                        double ov = rate_overlap(b * in->rate_bin_s, (b + 1) * in->rate_bin_s, 0.0, m->tstar);
                        g_rates[(int64_t)k * Bn + b] += adj[m->agent] * (double)o->u[m->to] * ov / r;
                    }
                }
                adj[m->agent] = 0.0;
            }
            else {
                /* MV_TRANSFER.  Admission graft: d psi / d m = -u_to d t_tok / d m with
                 * d t_tok / d m = -(dB_pre/dm)/(m q n) + (B_pre - 1)/(m^2 q n). */
                if (g_capm) {
                    int32_t j = m->from;
                    double mm = (double)o->cap_mult[j], qn = (double)o->cap[j] * (double)o->lanes[j];
                    double bpre = m->bacc - (double)m->tok_k;
                    double dtdm = -m->dbacc / (mm * qn) + (bpre - 1.0) / (mm * mm * qn);
                    g_capm[j] += adj[m->agent] * (-(double)o->u[m->to]) * dtdm;
                }
                /* the entry position carries the capped position's history;
                 * flags bit 0 drops that graft (the paper's "without TG" comparison, SI-C) */
                if (flags & 1) adj[m->agent] = 0.0;
            }
        }
        /* car-following, branches frozen; the cap passes the adjoint unchanged */
        for (int64_t c = s->cf0; c < s->cf0 + s->n_cf; ++c) nadj[o->cf.p[c].agent] = 0.0;
        for (int64_t c = s->cf0; c < s->cf0 + s->n_cf; ++c) {
            const cf_rec *r = &o->cf.p[c];
            double a = adj[r->agent];
            int32_t j = r->link;
            if (r->branch == BR_FREE) { nadj[r->agent] += a; if (g_u) g_u[j] += in->dt * a; }
            else if (r->branch == BR_STOP) nadj[r->agent] += a;
            else {
                nadj[r->leader] += a;
                if (g_kappa) g_kappa[j] += (double)in->platoon / ((double)o->kappa[j] * (double)o->kappa[j]) * a;
            }
        }
        for (int64_t c = s->cf0; c < s->cf0 + s->n_cf; ++c) adj[o->cf.p[c].agent] = nadj[o->cf.p[c].agent];
    }
    free(adj); free(nadj); free(bb); free(cc);
    return 0;
}
