// Host runtime behind the C-ABI of include/sim.h: input validation, network
// preprocessing (CSR adjacency, per-link rings, origin queues, shortest
// free-flow times), device memory, the step loop, checkpoints and the
// checkpointed replay that feeds the adjoint kernels.
#include "sim.h"
#include "sim_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <limits>
#include <new>
#include <queue>
#include <string>
#include <thread>
#include <vector>

using sim::Dev;

namespace {

thread_local std::string g_create_error;
constexpr int kTimingKinds = 7;   // link, node, reverse (self-timed), copies, link, node, reverse (HIP events)

struct HipError {
    std::string msg;
};

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw HipError{std::string(#expr) + ": " + hipGetErrorString(e_)};             \
    } while (0)

struct InvalidArg {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &m) { throw InvalidArg{code, m}; }

// checkpoint of everything the replay reads
struct Ckpt {
    float *ring_pos = nullptr;
    int32_t *ring_agent = nullptr;
    int2 *ring_aux = nullptr;
    sim::LinkSt *ls = nullptr;
    double *dB = nullptr;
    double *Dacc = nullptr;
    int32_t *rel_ptr = nullptr, *dep_ptr = nullptr;
    int64_t *ctr = nullptr;
    uint8_t *status = nullptr;
    int t = -1;
};

}  // namespace

struct sim_t {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // copies of the inputs
    int32_t S = 1, L = 0, Nn = 0, O = 0, N = 0, D = 0, nb = 0, cbs = 0, B = 0, maxl = 1;
    bool fixed_mode = true;
    double dt = 1.0, rate_bin_s = 0.0;
    int32_t platoon = 1, ckpt_every = 60, max_steps = 0, record = 0;
    int32_t g_link = 16, g_node = 64, g_rev = 16;   // lanes per work item
    int32_t n_ring_cls[sim::kRingClasses] = {0, 0, 0, 0};   // internal links by ring class
    int32_t nd_off[5] = {0, 0, 0, 0, 0};  // internal nodes by lane-group class (8, 16, 32, 64 lanes), contiguous
    std::vector<int32_t> tail, head, lanes, origin_node, det_link, agent_origin, agent_dest;
    std::vector<float> length, free_speed, jam_density, capacity, beta, alpha, cost, det_pos, ready, rates;
    std::vector<uint64_t> seeds;

    // derived host structures
    std::vector<int32_t> cap, ring_base, out_off, out_lnk, in_off, in_lnk, org_off, org_list, det_off, det_list;
    std::vector<int32_t> nperm, ninv, lperm, linv;   // internal <-> caller numbering of nodes and links
    int32_t *linv_dev = nullptr;
    std::vector<int32_t> dest_nodes, agent_didx;
    std::vector<double> dist, tff;
    std::vector<double> route;        // [node][destination][out-link] t_ff(m) + shortest time from head(m)
    std::vector<int64_t> route_base;  // per node: first entry of its block (n_dest * out_off)
    std::vector<int32_t> q_off, q_list;  // full queues (as built at create)
    std::vector<int32_t> q_dest, q_didx;
    std::vector<int64_t> q_rstep;
    std::vector<float> min_spacing;      // jam spacing the rings were sized for
    int64_t ring_total = 0;

    Dev d{};
    std::vector<void *> allocs;
    // serving: device memory carved from a range of the server's pool (bump allocation, never
    // freed one by one); allocations that do not fit fall back to hipMalloc
    char *arena = nullptr;
    size_t arena_cap = 0, arena_off = 0;
    int64_t arena_fallbacks = 0;
    // mutable parameter buffers
    float *p_u = nullptr, *p_kappa = nullptr, *p_beta = nullptr, *p_alpha = nullptr, *p_cost = nullptr,
          *p_rates = nullptr, *p_capm = nullptr, *capacity_dev = nullptr;
    // tape sets: the reverse sweep of one window reads one while replays of earlier windows write
    // others, on their own streams; the recording forward fills the sets of the last windows
    struct TapeSet {
        float *pos = nullptr, *dstg = nullptr;
        int32_t *agent = nullptr, *dst = nullptr;
        int4 *seg = nullptr;   // (head, tail, head slot, departure mask) per segment
        int4 *ste = nullptr;   // node candidates' choices and outcomes (straight-through gradients)
    };
    std::vector<TapeSet> tapes;              // n_tape_sets sets
    // the recording forward writes window w's tape into set w % tapes.size(); tape_win[set] is the
    // window a set holds from the forward (-1: none) and tape_steps[set] how many of its steps
    std::vector<int> tape_win, tape_steps;
    // concurrent replays of the backward pass: each has its own copy of the mutable state and
    // its own stream, so windows are replayed side by side while the main stream sweeps
    int n_replay = 3;
    int n_tape_sets = 4;                     // tape sets (windows of tape kept on the device), >= n_replay + 1
    std::vector<Dev> rp_dev;
    std::vector<hipStream_t> rp_stream;
    std::vector<hipEvent_t> bw_events;       // replay-done and reverse-done events per window
    float *tape_dstg_buf = nullptr;   // admission-graft tape, attached only for cap_mult gradients
    double *gm_buf = nullptr;
    double *gbeta_buf = nullptr, *gcost_buf = nullptr, *galpha_buf = nullptr, *gth_buf = nullptr;
    // autotuner snapshot of the live state (allocated on first use)
    bool tune_alloc = false;
    Ckpt tune_ck;
    double *tune_tstar = nullptr;
    int32_t *tune_rel = nullptr, *tune_dep = nullptr, *tune_exit = nullptr, *tune_cum = nullptr;
    int32_t *tune_tie_n = nullptr;
    float *vfree = nullptr, *spacing = nullptr;
    double *util = nullptr, *acc = nullptr;
    sim::LinkNd *lnd_dev = nullptr;
    sim::LinkCf *lcf_dev = nullptr;
    sim::RevCf *rcf_dev = nullptr;
    // mutable queue buffers
    int32_t *q_off_dev = nullptr, *q_list_dev = nullptr, *q_dest_dev = nullptr, *q_didx_dev = nullptr;
    int64_t *q_rstep_dev = nullptr;
    int2 *cand_dev = nullptr;
    std::vector<int32_t> node_cnt, in_pad, out_pad;
    int32_t max_in = 1, max_out = 1, max_org = 1, max_cand = 1;
    std::vector<int32_t> in_loff;
    std::vector<int2> cand;
    std::vector<int32_t> cbase;   // first straight-through record of each node
    int32_t n_cand = 0;
    // adjoint buffers
    float *gQ_dev = nullptr, *gx_dev = nullptr;
    double *gT_dev = nullptr, *ttt_dev = nullptr;
    unsigned long long *ttt_acc = nullptr;   // [2 x S] integer sums behind the travel time
    float *counts_dev = nullptr, *grad_tmp = nullptr;
    int64_t *vsteps_dev = nullptr;
    int64_t *dalloc_scratch_i64(size_t n) {
        if (!vsteps_dev) vsteps_dev = dalloc<int64_t>(n);
        return vsteps_dev;
    }

    size_t footprint = 0;     // device bytes this handle allocates
    double theta_cfg = 0.0;   // config kept for deferred allocation (serving)
    int32_t uturn_cfg = 1;
    int n_ck = 0;
    int t = 0;
    std::vector<Ckpt> ckpts;  // [n_ckpt] + final
    int W = 0;                // tape window (= ckpt_every)
    bool rec_valid = false;
    std::vector<uint8_t> placed;  // agents put on links by sim_place (not in the origin queues)
    // the host and device origin queues hold every agent (no placement): a reset then has nothing
    // to rebuild, since the queues depend only on the demand fixed at create and the placed mask
    bool queues_unplaced = false;

    // timing
    bool timing = false;
    struct Ev { hipEvent_t a, b; int kind; };
    std::vector<Ev> evs;
    std::vector<hipEvent_t> ev_pool;
    double ms_acc[kTimingKinds] = {};
    int64_t n_acc[kTimingKinds] = {};

    template <class T>
    T *dalloc(size_t n) {
        if (n == 0) n = 1;
        if (arena) {
            const size_t off = (arena_off + 255) & ~(size_t)255;
            if (off + n * sizeof(T) <= arena_cap) {
                arena_off = off + n * sizeof(T);
                return reinterpret_cast<T *>(arena + off);
            }
            ++arena_fallbacks;
        }
        void *p = nullptr;
        if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            fail(SIM_ENOMEM, "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
        }
        allocs.push_back(p);
        return static_cast<T *>(p);
    }
    template <class T>
    T *upload(const std::vector<T> &v) {
        T *p = dalloc<T>(v.size());
        if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, stream));
        return p;
    }
    ~sim_t() {
        if (device >= 0) (void)hipSetDevice(device);
        if (stream) (void)hipStreamSynchronize(stream);
        for (auto &e : evs) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
        for (auto e : ev_pool) (void)hipEventDestroy(e);
        for (auto x : rp_stream) { (void)hipStreamSynchronize(x); (void)hipStreamDestroy(x); }
        for (auto e : bw_events) (void)hipEventDestroy(e);
        for (void *p : allocs) (void)hipFree(p);
    }

    hipEvent_t get_event() {
        if (!ev_pool.empty()) { hipEvent_t e = ev_pool.back(); ev_pool.pop_back(); return e; }
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        return e;
    }
    void time_begin(int kind, hipEvent_t *a, hipStream_t on = nullptr) {
        (void)kind;
        if (!timing) return;
        *a = get_event();
        HIPCHK(hipEventRecord(*a, on ? on : stream));
    }
    void time_end(int kind, hipEvent_t a, hipStream_t on = nullptr) {
        if (!timing) return;
        hipEvent_t b = get_event();
        HIPCHK(hipEventRecord(b, on ? on : stream));
        evs.push_back({a, b, kind});
    }
    // kernels time themselves: each launch gets a record of (start, end) per wave in a buffer
    // allocated on the first timed launch; records are folded at resolve time
    static constexpr int64_t kStampEntries = (int64_t)192 << 20;   // u64 entries (1.5 GB)
    unsigned long long *stamps = nullptr, *stamp_out = nullptr;
    int64_t *stamp_off_dev = nullptr;
    int32_t *stamp_waves_dev = nullptr;
    static constexpr int kStampRecords = 16384;
    std::vector<int> stamp_kind;
    std::vector<int64_t> stamp_off;
    std::vector<int32_t> stamp_waves;
    int64_t stamp_used = 0;
    double wall_khz = 100000.0;
    // the launch's Dev, with a timing record when timing is on (kind: 0 link, 1 node, 2 reverse)
    Dev stamped(const Dev &dv, int kind, int blocks) {
        Dev r = dv;
        r.kstamp = nullptr;
        if (!timing) return r;
        if (!stamps) {
            stamps = dalloc<unsigned long long>((size_t)kStampEntries);
            stamp_out = dalloc<unsigned long long>(2 * (size_t)kStampRecords);
            stamp_off_dev = dalloc<int64_t>(kStampRecords);
            stamp_waves_dev = dalloc<int32_t>(kStampRecords);
            int khz = 0;
            if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
                wall_khz = khz;
        }
        const int64_t waves = (int64_t)blocks * sim::kWavesPerBlock;
        if ((int)stamp_kind.size() == kStampRecords || stamp_used + 2 * waves > kStampEntries) return r;
        r.kstamp = stamps + stamp_used;
        stamp_kind.push_back(kind);
        stamp_off.push_back(stamp_used / 2);
        stamp_waves.push_back((int32_t)waves);
        stamp_used += 2 * waves;
        return r;
    }
    void sync_all() {
        HIPCHK(hipStreamSynchronize(stream));
        for (auto x : rp_stream) HIPCHK(hipStreamSynchronize(x));
    }
    void resolve_timing() {
        if (!stamp_kind.empty()) {
            sync_all();
            const int n = (int)stamp_kind.size();
            HIPCHK(hipMemcpy(stamp_off_dev, stamp_off.data(), (size_t)n * 8, hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(stamp_waves_dev, stamp_waves.data(), (size_t)n * 4, hipMemcpyHostToDevice));
            sim::launch_stamp_reduce(stamp_off_dev, stamp_waves_dev, n, stamps, stamp_out, stream);
            std::vector<unsigned long long> v(2 * (size_t)n);
            HIPCHK(hipMemcpyAsync(v.data(), stamp_out, v.size() * 8, hipMemcpyDeviceToHost, stream));
            HIPCHK(hipStreamSynchronize(stream));
            for (int k = 0; k < n; ++k) {
                if (v[2 * k + 1] < v[2 * k]) continue;
                ms_acc[stamp_kind[k]] += (double)(v[2 * k + 1] - v[2 * k]) / wall_khz;
                n_acc[stamp_kind[k]] += 1;
            }
            stamp_kind.clear();
            stamp_off.clear();
            stamp_waves.clear();
            stamp_used = 0;
        }
        if (evs.empty()) return;
        for (auto &e : evs) {   // events may sit on several streams
            HIPCHK(hipEventSynchronize(e.b));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
            ms_acc[e.kind] += ms;
            n_acc[e.kind] += 1;
            ev_pool.push_back(e.a);
            ev_pool.push_back(e.b);
        }
        evs.clear();
    }
};

namespace {

// ---------------------------------------------------------------------------
// shortest free-flow time to each destination: Dijkstra on the reversed
// graph, weights length / free speed in double, one destination per task.
// ---------------------------------------------------------------------------
void shortest_times(sim_t *h)
{
    const int Nn = h->Nn;
    const int nd = (int)h->dest_nodes.size();
    h->dist.assign((size_t)nd * Nn, std::numeric_limits<double>::infinity());
    std::vector<double> w(h->L);
    for (int m = 0; m < h->L; ++m) w[m] = (double)h->length[m] / (double)h->free_speed[m];
    std::atomic<int> next{0};
    auto worker = [&]() {
        std::vector<char> done(Nn);
        using QE = std::pair<double, int>;
        for (;;) {
            const int k = next.fetch_add(1);
            if (k >= nd) break;
            double *dist = h->dist.data() + (size_t)k * Nn;
            std::fill(done.begin(), done.end(), 0);
            std::priority_queue<QE, std::vector<QE>, std::greater<QE>> pq;
            dist[h->dest_nodes[k]] = 0.0;
            pq.push({0.0, h->dest_nodes[k]});
            while (!pq.empty()) {
                const int x = pq.top().second;
                pq.pop();
                if (done[x]) continue;
                done[x] = 1;
                for (int e = h->in_off[x]; e < h->in_off[x + 1]; ++e) {
                    const int m = h->in_lnk[e];
                    const double cand = w[m] + dist[x];
                    const int y = h->tail[m];
                    if (cand < dist[y]) { dist[y] = cand; pq.push({cand, y}); }
                }
            }
        }
    };
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned i = 0; i + 1 < nt && (int)i < nd; ++i) th.emplace_back(worker);
    worker();
    for (auto &x : th) x.join();
}

void build_csr(int n, const std::vector<int32_t> &key, std::vector<int32_t> &off, std::vector<int32_t> &lst)
{
    off.assign(n + 1, 0);
    for (int32_t k : key) off[k + 1]++;
    for (int i = 0; i < n; ++i) off[i + 1] += off[i];
    lst.assign(key.size(), 0);
    std::vector<int32_t> fill(n, 0);
    for (size_t i = 0; i < key.size(); ++i) lst[off[key[i]] + fill[key[i]]++] = (int32_t)i;
}

// origin queues, excluding agents not waiting (placed agents)
void build_queues(sim_t *h, const std::vector<uint8_t> *skip)
{
    const int O = h->O, N = h->N;
    std::vector<int32_t> cnt(O, 0);
    for (int i = 0; i < N; ++i)
        if (!skip || !(*skip)[i]) cnt[h->agent_origin[i]]++;
    h->q_off.assign(O + 1, 0);
    for (int k = 0; k < O; ++k) h->q_off[k + 1] = h->q_off[k] + cnt[k];
    h->q_list.assign(h->q_off[O], 0);
    h->q_rstep.assign(h->q_off[O], 0);
    std::vector<std::vector<std::pair<int64_t, int32_t>>> per(O);
    for (int i = 0; i < N; ++i) {
        if (skip && (*skip)[i]) continue;
        int64_t rs = 0;
        if (h->fixed_mode) {
            double r = std::floor((double)h->ready[i] / h->dt);
            if (r < 0) r = 0;
            if (r > 4e18) r = 4e18;
            rs = (int64_t)r;
        }
        per[h->agent_origin[i]].push_back({rs, i});
    }
    h->q_dest.assign(h->q_off[O], 0);
    h->q_didx.assign(h->q_off[O], 0);
    for (int k = 0; k < O; ++k) {
        std::sort(per[k].begin(), per[k].end());
        for (size_t a = 0; a < per[k].size(); ++a) {
            const int32_t i = per[k][a].second;
            h->q_list[h->q_off[k] + a] = i;
            h->q_rstep[h->q_off[k] + a] = per[k][a].first;
            h->q_dest[h->q_off[k] + a] = h->agent_dest[i];
            h->q_didx[h->q_off[k] + a] = h->agent_didx.empty() ? 0 : h->agent_didx[i];
        }
    }
}

void zero_state(sim_t *h)
{
    Dev &d = h->d;
    const hipStream_t st = h->stream;
    const size_t SL = (size_t)h->S * h->L, SN = (size_t)h->S * h->N, SO = (size_t)h->S * h->O;
    HIPCHK(hipMemsetAsync(d.ls, 0, SL * sizeof(sim::LinkSt), st));
    if (d.dB) HIPCHK(hipMemsetAsync(d.dB, 0, SL * 8, st));
    HIPCHK(hipMemsetAsync(d.status, 0, SN, st));
    HIPCHK(hipMemsetAsync(d.tstar, 0, SN * 8, st));
    HIPCHK(hipMemsetAsync(d.rel_t, 0xff, SN * 4, st));
    HIPCHK(hipMemsetAsync(d.dep_t, 0xff, SN * 4, st));
    HIPCHK(hipMemsetAsync(d.exit_t, 0xff, SN * 4, st));
    HIPCHK(hipMemsetAsync(d.Dacc, 0, SO * 8, st));
    HIPCHK(hipMemsetAsync(d.rel_ptr, 0, SO * 4, st));
    HIPCHK(hipMemsetAsync(d.dep_ptr, 0, SO * 4, st));
    HIPCHK(hipMemsetAsync(d.ctr, 0, (size_t)h->S * sim::kCtrSlots * sim::CTR_N * 8, st));
    if (h->D * h->nb) HIPCHK(hipMemsetAsync(d.cum, 0, (size_t)h->S * h->D * h->nb * 4, st));
    HIPCHK(hipMemsetAsync(d.err, 0, sim::ERR_N * 4, st));
    HIPCHK(hipMemsetAsync(d.tie_n, 0, 4, st));
    h->t = 0;
    h->rec_valid = h->record != 0;
    h->tape_win.assign(h->tapes.size(), -1);
    h->tape_steps.assign(h->tapes.size(), 0);
}

void upload_queues(sim_t *h)
{
    // queue buffers are sized for the full pool at create; copy the current lists
    HIPCHK(hipMemcpyAsync(h->q_off_dev, h->q_off.data(), h->q_off.size() * 4, hipMemcpyHostToDevice, h->stream));
    if (!h->q_list.empty()) {
        HIPCHK(hipMemcpyAsync(h->q_list_dev, h->q_list.data(), h->q_list.size() * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->q_dest_dev, h->q_dest.data(), h->q_dest.size() * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->q_didx_dev, h->q_didx.data(), h->q_didx.size() * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->q_rstep_dev, h->q_rstep.data(), h->q_rstep.size() * 8, hipMemcpyHostToDevice, h->stream));
    }
    // candidate lanes past a node's head lanes hold its origins as (origin, first queue entry), which
    // follow the queue offsets
    for (int v = 0; v < h->Nn; ++v) {
        const int nl = (h->node_cnt[v] >> 24) & 0xff;
        for (int k = h->org_off[v]; k < h->org_off[v + 1]; ++k) {
            const int o = h->org_list[k];
            h->cand[(size_t)v * h->max_cand + nl + (k - h->org_off[v])] = make_int2(o, h->q_off[o]);
        }
    }
    HIPCHK(hipMemcpyAsync(h->cand_dev, h->cand.data(), h->cand.size() * sizeof(int2), hipMemcpyHostToDevice,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
}

// Locality-preserving internal numbering: nodes in reverse Cuthill-McKee
// order of the undirected node graph (neighbours get nearby ids), links by
// (new tail node, original id), so a node's out-links stay in original-id
// order.  Callers always see the original numbering; the runtime translates
// at the boundary.
// ring slots of a link: a lane chain holds at most floor(L / spacing) + 2 agents under float
// rounding; one more row per lane keeps `lanes` slots free for the step's leavers
double ring_slots(float length, int lanes, float jam_density, int platoon)
{
    const float sp = (float)platoon / jam_density;
    return (std::floor((double)length / (double)sp) + 4.0) * lanes;
}

// lane-group class of a node from its merge candidates and out-links: 0 (8), 1 (16), 2 (32), 3 (64 lanes)
int node_class(int need) { return need <= 8 ? 0 : (need <= 16 ? 1 : (need <= 32 ? 2 : 3)); }

// Internal numbering.  Nodes: reverse Cuthill-McKee for locality, then grouped by lane-group class
// (stable), so each class of the node kernel is a contiguous id range.  Links: by ring class (at most
// kSmallRing slots, kMidRing, kLongRing, larger), then by new tail node and original id, so each class of
// the link and reverse kernels is a contiguous id range and a node's out-links lie together.
void renumber(sim_t *h)
{
    const int Nn = h->Nn, L = h->L;
    std::vector<std::vector<int>> adj(Nn);
    for (int j = 0; j < L; ++j) {
        adj[h->tail[j]].push_back(h->head[j]);
        adj[h->head[j]].push_back(h->tail[j]);
    }
    for (auto &a : adj) {
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
    }
    auto deg_less = [&](int a, int b) { return adj[a].size() != adj[b].size() ? adj[a].size() < adj[b].size() : a < b; };
    std::vector<int> start(Nn);
    for (int v = 0; v < Nn; ++v) start[v] = v;
    std::sort(start.begin(), start.end(), deg_less);
    std::vector<int> order;
    order.reserve(Nn);
    std::vector<char> seen(Nn, 0);
    for (int st : start) {
        if (seen[st]) continue;
        size_t qh = order.size();
        order.push_back(st);
        seen[st] = 1;
        while (qh < order.size()) {
            const int x = order[qh++];
            std::vector<int> nb;
            for (int y : adj[x]) if (!seen[y]) nb.push_back(y);
            std::sort(nb.begin(), nb.end(), deg_less);
            for (int y : nb) { seen[y] = 1; order.push_back(y); }
        }
    }
    std::reverse(order.begin(), order.end());
    {
        std::vector<int> din(Nn, 0), dout(Nn, 0), norg(Nn, 0), cls(Nn, 0);
        // candidates of a node: a head lane per lane of each in-link, plus its origin queues
        for (int j = 0; j < L; ++j) { din[h->head[j]] += h->lanes[j]; dout[h->tail[j]]++; }
        for (int o = 0; o < h->O; ++o) norg[h->origin_node[o]]++;
        for (int v = 0; v < Nn; ++v) cls[v] = node_class(std::max(din[v] + norg[v], dout[v]));
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cls[a] < cls[b]; });
        h->nd_off[0] = 0;
        for (int c = 0; c < 4; ++c) {
            int n = 0;
            for (int v = 0; v < Nn; ++v) n += cls[v] == c;
            h->nd_off[c + 1] = h->nd_off[c] + n;
        }
    }
    h->nperm = order;
    h->ninv.assign(Nn, 0);
    for (int k = 0; k < Nn; ++k) h->ninv[order[k]] = k;
    std::vector<char> cls(L);
    for (int c = 0; c < sim::kRingClasses; ++c) h->n_ring_cls[c] = 0;
    for (int j = 0; j < L; ++j) {
        const double slots = ring_slots(h->length[j], h->lanes[j], h->jam_density[j], h->platoon);
        cls[j] = slots <= sim::kSmallRing ? 0 : (slots <= sim::kMidRing ? 1 : (slots <= sim::kLongRing ? 2 : 3));
        h->n_ring_cls[(int)cls[j]]++;
    }
    h->lperm.resize(L);
    for (int j = 0; j < L; ++j) h->lperm[j] = j;
    std::sort(h->lperm.begin(), h->lperm.end(), [&](int a, int b) {
        if (cls[a] != cls[b]) return cls[a] < cls[b];
        const int ta = h->ninv[h->tail[a]], tb = h->ninv[h->tail[b]];
        return ta != tb ? ta < tb : a < b;
    });
    h->linv.assign(L, 0);
    for (int k = 0; k < L; ++k) h->linv[h->lperm[k]] = k;
    auto perm_f = [&](std::vector<float> &v) { std::vector<float> o(L); for (int k = 0; k < L; ++k) o[k] = v[h->lperm[k]]; v.swap(o); };
    auto perm_i = [&](std::vector<int32_t> &v) { std::vector<int32_t> o(L); for (int k = 0; k < L; ++k) o[k] = v[h->lperm[k]]; v.swap(o); };
    perm_i(h->tail); perm_i(h->head); perm_i(h->lanes);
    for (auto &x : h->tail) x = h->ninv[x];
    for (auto &x : h->head) x = h->ninv[x];
    perm_f(h->length); perm_f(h->free_speed); perm_f(h->jam_density); perm_f(h->capacity);
    perm_f(h->beta); perm_f(h->alpha); perm_f(h->cost);
    for (auto &x : h->origin_node) x = h->ninv[x];
    for (auto &x : h->det_link) x = h->linv[x];
    for (auto &x : h->agent_dest) x = h->ninv[x];
}

// per-link values [S x L]: caller order -> internal order
std::vector<float> links_in(const sim_t *h, const float *v)
{
    std::vector<float> o((size_t)h->S * h->L);
    for (int s = 0; s < h->S; ++s)
        for (int k = 0; k < h->L; ++k) o[(size_t)s * h->L + k] = v[(size_t)s * h->L + h->lperm[k]];
    return o;
}

// work-item ranges of the link, node and reverse kernels (contiguous id ranges, see renumber)
void build_classes(sim_t *h)
{
    Dev &d = h->d;
    for (int c = 0; c < sim::kRingClasses; ++c) d.lc_n[c] = h->n_ring_cls[c];
    // node roles of 8, 16, 32 and 64 lanes; the schedule's floor moves smaller classes up
    const int r1 = h->g_node <= 8 ? h->nd_off[1] : 0;
    const int r2 = h->g_node <= 16 ? h->nd_off[2] : 0;
    const int r3 = h->g_node <= 32 ? h->nd_off[3] : 0;
    d.nd_begin[0] = 0;  d.nd_n[0] = r1;
    d.nd_begin[1] = r1; d.nd_n[1] = r2 - r1;
    d.nd_begin[2] = r2; d.nd_n[2] = r3 - r2;
    d.nd_begin[3] = r3; d.nd_n[3] = h->Nn - r3;
}

void derive(sim_t *h)
{
    sim::launch_derive(h->d, h->p_capm, h->capacity_dev, h->p_beta, h->p_cost, h->util, h->acc, h->vfree, h->spacing,
                       h->lnd_dev, h->lcf_dev, h->rcf_dev, h->stream);
    HIPCHK(hipGetLastError());
}

void check_device_errors(sim_t *h)
{
    // under stream capture nothing may wait: the flags are read by the next call outside capture
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (h->stream && hipStreamIsCapturing(h->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return;
    int32_t e[sim::ERR_N];
    HIPCHK(hipMemcpyAsync(e, h->d.err, sizeof(e), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (e[sim::ERR_RING_OVERFLOW]) fail(SIM_ESTATE, "a link ring overflowed (agents closer than the jam spacing)");
    if (e[sim::ERR_CAND_OVERFLOW]) fail(SIM_EUNSUPPORTED, "more than 64 merge candidates at a node");
}

// --- checkpoints ---
void ckpt_alloc(sim_t *h, Ckpt &c)
{
    const size_t SR = (size_t)h->S * h->ring_total, SL = (size_t)h->S * h->L, SO = (size_t)h->S * h->O;
    c.ring_pos = h->dalloc<float>(SR);
    c.ring_agent = h->dalloc<int32_t>(SR);
    c.ring_aux = h->dalloc<int2>(SR);
    c.ls = h->dalloc<sim::LinkSt>(SL);
    c.dB = h->dalloc<double>(SL);
    c.Dacc = h->dalloc<double>(SO);
    c.rel_ptr = h->dalloc<int32_t>(SO);
    c.dep_ptr = h->dalloc<int32_t>(SO);
    c.ctr = h->dalloc<int64_t>((size_t)h->S * sim::kCtrSlots * sim::CTR_N);
    c.status = h->dalloc<uint8_t>((size_t)h->S * h->N);
}

void ckpt_copy(sim_t *h, Ckpt &c, bool save, Dev *target = nullptr, hipStream_t on = nullptr)
{
    Dev &d = target ? *target : h->d;
    const size_t SR = (size_t)h->S * h->ring_total, SL = (size_t)h->S * h->L, SO = (size_t)h->S * h->O;
    const hipStream_t st = on ? on : h->stream;
    // every array of the checkpoint in one copy launch (ten separate copies cost a launch each)
    sim::CopyJobs jobs{};
    auto cp = [&](void *ck, void *live, size_t bytes) {
        if (bytes == 0) return;
        jobs.job[jobs.n++] = save ? sim::CopyJob{live, ck, bytes} : sim::CopyJob{ck, live, bytes};
    };
    cp(c.ring_pos, d.ring_pos, SR * 4);
    cp(c.ring_agent, d.ring_agent, SR * 4);
    cp(c.ring_aux, d.ring_aux, SR * 8);
    cp(c.ls, d.ls, SL * sizeof(sim::LinkSt));
    if (d.dB) cp(c.dB, d.dB, SL * 8);
    cp(c.Dacc, d.Dacc, SO * 8);
    cp(c.rel_ptr, d.rel_ptr, SO * 4);
    cp(c.dep_ptr, d.dep_ptr, SO * 4);
    cp(c.ctr, d.ctr, (size_t)h->S * sim::kCtrSlots * sim::CTR_N * 8);
    cp(c.status, d.status, (size_t)h->S * h->N);
    sim::launch_copy_multi(jobs, st);
    HIPCHK(hipGetLastError());
}

// the mutable state arrays of `src`, put into `dst` (parameters, tables, tape stay dst's)
void with_state(Dev &dst, const Dev &src)
{
    dst.ring_pos = src.ring_pos; dst.ring_agent = src.ring_agent; dst.ring_aux = src.ring_aux;
    dst.ls = src.ls; dst.dB = src.dB; dst.head_rec = src.head_rec;
    dst.status = src.status; dst.tstar = src.tstar; dst.rel_t = src.rel_t; dst.dep_t = src.dep_t;
    dst.exit_t = src.exit_t; dst.Dacc = src.Dacc; dst.rel_ptr = src.rel_ptr; dst.dep_ptr = src.dep_ptr;
    dst.ctr = src.ctr; dst.cum = src.cum;
}

// one step of state set `dv` at step t on stream `on`
void step_on(sim_t *h, const Dev &dv, hipStream_t on, int t, int tape_k)
{
    int sb = -1;
    if (h->cbs > 0 && (t + 1) % h->cbs == 0 && (t + 1) / h->cbs <= h->nb) sb = (t + 1) / h->cbs - 1;
    hipEvent_t ea = nullptr, eb = nullptr;
    h->time_begin(4, &ea, on);
    sim::launch_link(h->stamped(dv, 0, sim::link_blocks(dv)), t, sb, tape_k, on);
    h->time_end(4, ea, on);
    h->time_begin(5, &eb, on);
    sim::launch_node(h->stamped(dv, 1, sim::node_blocks(dv)), t, tape_k, on);
    h->time_end(5, eb, on);
    HIPCHK(hipGetLastError());
}

void do_step(sim_t *h, int tape_k)
{
    step_on(h, h->d, h->stream, h->t, tape_k);
    h->t += 1;
}

int record_error(sim_t *h, int code, const std::string &msg)
{
    if (h) h->err = msg;
    else g_create_error = msg;
    return code;
}

template <class F>
int guarded(sim_t *h, F &&f)
{
    if (!h) return record_error(nullptr, SIM_EINVAL, "null handle");
    try {
        HIPCHK(hipSetDevice(h->device));
        f();
        return SIM_OK;
    } catch (const InvalidArg &e) {
        return record_error(h, e.code, e.msg);
    } catch (const HipError &e) {
        return record_error(h, SIM_EDEVICE, e.msg);
    } catch (const std::bad_alloc &) {
        return record_error(h, SIM_ENOMEM, "host allocation failed");
    } catch (...) {
        return record_error(h, SIM_EDEVICE, "unexpected failure");
    }
}

void copy_out(sim_t *h, void *dst, const void *src_dev, size_t bytes, int on_device)
{
    if (bytes == 0) return;
    HIPCHK(hipMemcpyAsync(dst, src_dev, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
}

// Host-side preparation of a handle: validation, renumbering, adjacency,
// rings, shortest times, queues and the device footprint.  No device calls.
void prepare_host(sim_t *h, const sim_network *net, const sim_demand *dem, const sim_config *cfg)
{
        // ---------------- validate and copy ----------------
    const int L = net->n_links, Nn = net->n_nodes;
    if (L <= 0 || Nn <= 0) fail(SIM_EINVAL, "network needs nodes and links");
    if (!net->tail || !net->head || !net->lanes || !net->length || !net->free_speed || !net->jam_density ||
        !net->capacity)
        fail(SIM_EINVAL, "missing link array");
    h->L = L; h->Nn = Nn;
    h->tail.assign(net->tail, net->tail + L);
    h->head.assign(net->head, net->head + L);
    h->lanes.assign(net->lanes, net->lanes + L);
    h->length.assign(net->length, net->length + L);
    h->free_speed.assign(net->free_speed, net->free_speed + L);
    h->jam_density.assign(net->jam_density, net->jam_density + L);
    h->capacity.assign(net->capacity, net->capacity + L);
    h->beta = net->beta ? std::vector<float>(net->beta, net->beta + L) : std::vector<float>(L, 0.f);
    h->alpha = net->alpha ? std::vector<float>(net->alpha, net->alpha + L) : std::vector<float>(L, 1.f);
    h->cost = net->cost ? std::vector<float>(net->cost, net->cost + L) : std::vector<float>(L, 1.f);
    int maxl = 1;
    for (int j = 0; j < L; ++j) {
        if (h->tail[j] < 0 || h->tail[j] >= Nn || h->head[j] < 0 || h->head[j] >= Nn)
            fail(SIM_EINVAL, "link " + std::to_string(j) + ": node index out of range");
        if (h->lanes[j] < 1 || h->lanes[j] > sim::kMaxLanes) fail(SIM_EINVAL, "lanes must be in [1, 8]");
        if (!(h->length[j] > 0.02f) || !(h->free_speed[j] > 0.f) || !(h->jam_density[j] > 0.f) ||
            !(h->capacity[j] >= 0.f) || !(h->cost[j] > 0.f) || !std::isfinite(h->length[j]) ||
            !std::isfinite(h->free_speed[j]) || !std::isfinite(h->capacity[j]))
            fail(SIM_EINVAL, "link " + std::to_string(j) + ": non-positive or non-finite length/speed/density/cost");
        maxl = std::max(maxl, h->lanes[j]);
    }
    h->maxl = maxl;
    h->O = net->n_origins;
    if (h->O < 0 || (h->O > 0 && !net->origin_node)) fail(SIM_EINVAL, "bad origins");
    h->origin_node.assign(net->origin_node, net->origin_node + h->O);
    for (int k = 0; k < h->O; ++k)
        if (h->origin_node[k] < 0 || h->origin_node[k] >= Nn) fail(SIM_EINVAL, "origin node out of range");
    h->D = net->n_detectors;
    if (h->D < 0 || (h->D > 0 && (!net->detector_link || !net->detector_pos))) fail(SIM_EINVAL, "bad detectors");
    if (h->D >= (1 << 24)) fail(SIM_EUNSUPPORTED, "at most 2^24 - 1 detectors");
    h->det_link.assign(net->detector_link, net->detector_link + h->D);
    h->det_pos.assign(net->detector_pos, net->detector_pos + h->D);
    for (int k = 0; k < h->D; ++k) {
        const int j = h->det_link[k];
        if (j < 0 || j >= L) fail(SIM_EINVAL, "detector link out of range");
        if (!(h->det_pos[k] > 0.f) || !(h->det_pos[k] <= h->length[j] - 0.01f))
            fail(SIM_EINVAL, "detector position must lie in (0, length - 0.01]");
    }
    h->N = dem->n_agents;
    if (h->N < 0 || (h->N > 0 && (!dem->agent_origin || !dem->agent_dest))) fail(SIM_EINVAL, "bad agents");
    h->agent_origin.assign(dem->agent_origin, dem->agent_origin + h->N);
    h->agent_dest.assign(dem->agent_dest, dem->agent_dest + h->N);
    h->fixed_mode = dem->ready_time != nullptr;
    if (h->fixed_mode) h->ready.assign(dem->ready_time, dem->ready_time + h->N);
    else {
        h->B = dem->n_rate_bins;
        h->rate_bin_s = dem->rate_bin_s;
        if (h->B <= 0 || !dem->rates || !(dem->rate_bin_s > 0)) fail(SIM_EINVAL, "rate mode needs rates and bins");
        h->rates.assign(dem->rates, dem->rates + (size_t)h->O * h->B);
        for (float r : h->rates)
            if (!(r >= 0.f) || !std::isfinite(r)) fail(SIM_EINVAL, "rates must be finite and >= 0");
    }
    for (int i = 0; i < h->N; ++i) {
        if (h->agent_origin[i] < 0 || h->agent_origin[i] >= h->O) fail(SIM_EINVAL, "agent origin out of range");
        if (h->agent_dest[i] < 0 || h->agent_dest[i] >= Nn) fail(SIM_EINVAL, "agent destination out of range");
        if (h->agent_dest[i] == h->origin_node[h->agent_origin[i]])
            fail(SIM_EINVAL, "agent destination equals its origin node");
    }
    h->dt = cfg->dt;
    h->platoon = cfg->platoon;
    if (!(cfg->dt > 0) || cfg->platoon < 1) fail(SIM_EINVAL, "dt > 0 and platoon >= 1 required");
    // an agent stands for `platoon` vehicles: the outflow bucket counts agents, capacity * lanes / platoon per second
    for (float &q : h->capacity) q = q / (float)h->platoon;
    if (!h->fixed_mode) {
        const double k = h->rate_bin_s / h->dt;
        if (std::fabs(k - std::round(k)) > 1e-9) fail(SIM_EINVAL, "rate bins must be a whole number of steps");
    }
    h->S = cfg->n_scenarios;
    if (h->S < 1) fail(SIM_EINVAL, "n_scenarios >= 1");
    h->cbs = cfg->count_bin_steps;
    h->nb = cfg->n_count_bins;
    if (h->nb < 0 || (h->nb > 0 && h->cbs < 1)) fail(SIM_EINVAL, "count bins need count_bin_steps >= 1");
    h->ckpt_every = cfg->ckpt_every > 0 ? cfg->ckpt_every : 60;
    h->max_steps = cfg->max_steps;
    h->record = cfg->record_for_backward;
    if (h->record && h->max_steps <= 0) fail(SIM_EINVAL, "record_for_backward needs max_steps > 0");
    h->seeds.resize(h->S);
    for (int s = 0; s < h->S; ++s) h->seeds[s] = cfg->scenario_seed ? cfg->scenario_seed[s] : cfg->seed + (uint64_t)s;

    // ---------------- graph ----------------
    renumber(h);
    build_csr(Nn, h->tail, h->out_off, h->out_lnk);
    build_csr(Nn, h->head, h->in_off, h->in_lnk);
    build_csr(Nn, h->origin_node, h->org_off, h->org_list);
    build_csr(L, h->det_link, h->det_off, h->det_list);
    // a node's out-links in original id order: the route-choice candidate index (which picks the
    // Gumbel draw) is the caller's CSR position
    for (int v = 0; v < Nn; ++v) {
        std::sort(h->out_lnk.begin() + h->out_off[v], h->out_lnk.begin() + h->out_off[v + 1],
                  [&](int a, int b) { return h->lperm[a] < h->lperm[b]; });
        std::sort(h->in_lnk.begin() + h->in_off[v], h->in_lnk.begin() + h->in_off[v + 1],
                  [&](int a, int b) { return h->lperm[a] < h->lperm[b]; });
    }
    for (int v = 0; v < Nn; ++v) {
        int nc = h->org_off[v + 1] - h->org_off[v];
        for (int k = h->in_off[v]; k < h->in_off[v + 1]; ++k) nc += h->lanes[h->in_lnk[k]];
        if (nc > sim::kWave) fail(SIM_EUNSUPPORTED, "node " + std::to_string(v) + ": more than 64 merge candidates");
        if (h->out_off[v + 1] - h->out_off[v] > sim::kWave) fail(SIM_EUNSUPPORTED, "node out-degree above 64");
    }
    for (int j = 0; j < L; ++j)
        if (h->det_off[j + 1] - h->det_off[j] > sim::kMaxDetPerLink) fail(SIM_EUNSUPPORTED, "more than 4 detectors on a link");
    // lanes per node: a floor; each node gets the smallest group (8, 16, 32, 64) above it that holds
    // its candidates and out-links
    h->g_node = 8;
    (void)maxl;
    for (int v = 0; v < Nn; ++v) {
        h->max_in = std::max(h->max_in, h->in_off[v + 1] - h->in_off[v]);
        h->max_out = std::max(h->max_out, h->out_off[v + 1] - h->out_off[v]);
        h->max_org = std::max(h->max_org, h->org_off[v + 1] - h->org_off[v]);
    }
    if (h->max_in > 255 || h->max_out > 255 || h->max_org > 255) fail(SIM_EUNSUPPORTED, "node degree above 255");
    for (int v = 0; v < Nn; ++v) {   // candidate lanes: the in-links' head lanes, then the origins
        int nl = h->org_off[v + 1] - h->org_off[v];
        for (int k = h->in_off[v]; k < h->in_off[v + 1]; ++k) nl += h->lanes[h->in_lnk[k]];
        h->max_cand = std::max(h->max_cand, nl);
    }
    h->node_cnt.resize(Nn);
    h->in_pad.assign((size_t)Nn * h->max_in, -1);
    h->in_loff.assign((size_t)Nn * h->max_in, 0);
    h->out_pad.assign((size_t)Nn * h->max_out, -1);
    h->cand.assign((size_t)Nn * h->max_cand, make_int2(0, 0));
    h->cbase.assign(Nn, 0);
    h->n_cand = 0;
    for (int v = 0; v < Nn; ++v) {
        const int di = h->in_off[v + 1] - h->in_off[v], dout = h->out_off[v + 1] - h->out_off[v];
        const int no = h->org_off[v + 1] - h->org_off[v];
        int nl = 0;
        for (int k = 0; k < di; ++k) {
            const int j = h->in_lnk[h->in_off[v] + k];
            h->in_pad[(size_t)v * h->max_in + k] = j;
            h->in_loff[(size_t)v * h->max_in + k] = nl;
            for (int r = 0; r < h->lanes[j]; ++r) h->cand[(size_t)v * h->max_cand + nl + r] = make_int2(j, k | (r << 8));
            nl += h->lanes[j];
        }
        h->node_cnt[v] = di | (dout << 8) | (no << 16) | (nl << 24);
        h->cbase[v] = h->n_cand;
        h->n_cand += nl + no;
        for (int k = 0; k < dout; ++k) h->out_pad[(size_t)v * h->max_out + k] = h->out_lnk[h->out_off[v] + k];
    }
    // rings: a link holds at most lanes * (floor(L / spacing) + 1) agents; two extra rows of slack
    h->cap.resize(L);
    h->ring_base.resize(L);
    h->min_spacing.resize(L);
    int64_t tot = 0;
    for (int j = 0; j < L; ++j) {
        h->min_spacing[j] = (float)h->platoon / h->jam_density[j];
        const double c = ring_slots(h->length[j], h->lanes[j], h->jam_density[j], h->platoon);
        if (c > 1e8) fail(SIM_EUNSUPPORTED, "link too long for its jam spacing");
        h->cap[j] = (int32_t)c;
        h->ring_base[j] = (int32_t)tot;
        tot += h->cap[j];
        if (tot > (int64_t)1 << 30) fail(SIM_EUNSUPPORTED, "ring storage above 2^30 slots");
    }
    h->ring_total = tot;
    if ((int64_t)h->S * tot >= ((int64_t)1 << 31)) fail(SIM_EUNSUPPORTED, "scenarios x ring slots above 2^31");
    // destinations, numbered in node order
    std::vector<int32_t> didx(Nn, -1);
    for (int i = 0; i < h->N; ++i) didx[h->agent_dest[i]] = 0;
    for (int v = 0; v < Nn; ++v)
        if (didx[v] == 0) { didx[v] = (int32_t)h->dest_nodes.size(); h->dest_nodes.push_back(v); }
    h->agent_didx.resize(h->N);
    for (int i = 0; i < h->N; ++i) h->agent_didx[i] = didx[h->agent_dest[i]];
    shortest_times(h);
    for (int i = 0; i < h->N; ++i) {
        const double dd = h->dist[(size_t)h->agent_didx[i] * Nn + h->origin_node[h->agent_origin[i]]];
        if (!(dd < std::numeric_limits<double>::infinity()))
            fail(SIM_EINVAL, "agent " + std::to_string(i) + ": destination unreachable from its origin");
    }
    h->tff.resize(L);
    for (int m = 0; m < L; ++m) h->tff[m] = (double)h->length[m] / (double)h->free_speed[m];
    // route table: the free-flow time of every (node, destination, out-link) choice, one contiguous
    // row per (node, destination), so a head's route choice reads one row instead of one shortest-
    // time entry per out-link; each entry is the same double sum the choice would form
    {
        const size_t nd = h->dest_nodes.size();
        h->route.assign(nd * (size_t)L, std::numeric_limits<double>::infinity());
        h->route_base.resize(Nn);
        for (int v = 0; v < Nn; ++v) {
            const int64_t base = (int64_t)nd * h->out_off[v];
            const int dg = h->out_off[v + 1] - h->out_off[v];
            h->route_base[v] = base;
            for (size_t dd = 0; dd < nd; ++dd)
                for (int k = 0; k < dg; ++k) {
                    const int m = h->out_lnk[h->out_off[v] + k];
                    h->route[base + dd * dg + k] = h->tff[m] + h->dist[dd * Nn + h->head[m]];
                }
        }
    }
    build_queues(h, nullptr);

    // ---------------- memory budget ----------------
    const size_t SL = (size_t)h->S * L, SN = (size_t)h->S * h->N, SO = (size_t)h->S * h->O;
    const size_t SR = (size_t)h->S * h->ring_total;
    // an upper bound of what allocate_device takes: every array below, each rounded up to 256 bytes
    // (the serving pool carves a request's state with that alignment)
    const size_t nQ = (size_t)h->S * h->D * std::max(h->nb, 1);
    size_t bytes = SR * 16                                   // ring positions, agents, (destination, row)
                   + SL * (24 + 8 + 16 + 32 + 96 + maxl * 16)   // parameters, derived, state, link records, heads
                   + SN * (1 + 8 + 12) + SO * 16             // per agent and per origin state
                   + (size_t)h->S * h->O * std::max(h->B, 1) * 4
                   + (size_t)L * 56 + (size_t)Nn * 32        // link constants, node offsets and words
                   + (h->in_pad.size() + h->in_loff.size() + h->out_pad.size()) * 4 + h->cand.size() * 8 +
                   (size_t)h->N * 44 + h->route.size() * 8 +
                   (size_t)h->D * 12 + (size_t)h->S * 8 +
                   (size_t)h->S * sim::kCtrSlots * sim::CTR_N * 8 + nQ * 8 + (size_t)6 * sim::kTieLogMax * 4 +
                   (size_t)h->S * 24 + 128 * 256;
    int n_ck = 0;
    if (h->record) {
        n_ck = (h->max_steps + h->ckpt_every - 1) / h->ckpt_every + 1;
        h->W = h->ckpt_every;
        bytes += (size_t)n_ck * (SR * 16 + SL * 40 + SO * 16 + SN);
        // one tape set: positions and agents per slot, head/tail/head slot/departure mask per segment,
        // entry slot and graft factor
        // per leaving head, and a straight-through record per node candidate, for W + 1 states
        const size_t per_set = (size_t)(h->W + 1) *
                               (SR * 8 + SL * 16 + SL * maxl * 8 + (size_t)h->S * std::max(h->n_cand, 1) * 16);
        const int min_sets = h->n_replay + 1, windows = std::max(n_ck - 1, 1);
        int sets = cfg->tape_windows > 0 ? std::max(min_sets, (int)cfg->tape_windows)
                                         : (int)std::min<size_t>(16, ((size_t)32 << 30) / std::max<size_t>(per_set, 1));
        sets = std::max(min_sets, std::min(sets, std::max(windows, min_sets)));
        h->n_tape_sets = sets;
        bytes += (size_t)sets * per_set + SR * 4 + SN * 4 + SL * 24 + SL * 8 * 4 + (size_t)h->S * Nn * 8;
        bytes += (size_t)h->n_replay * (SR * 16 + SL * (48 + maxl * 16) + SN * 21 + SO * 16 +
                                        (size_t)h->S * h->D * std::max(h->nb, 1) * 4);
    }
    h->footprint = bytes;
    h->n_ck = n_ck;
    if (cfg->mem_budget_bytes && bytes > cfg->mem_budget_bytes)
        fail(SIM_ENOMEM, "footprint " + std::to_string(bytes) + " B exceeds the memory budget");

}

// Device allocation and upload of a prepared handle.
void allocate_device(sim_t *h, const sim_config *cfg)
{
    const int L = h->L, Nn = h->Nn, maxl = h->maxl, n_ck = h->n_ck;
    const size_t SL = (size_t)h->S * L, SN = (size_t)h->S * h->N, SO = (size_t)h->S * h->O;
    const size_t SR = (size_t)h->S * h->ring_total;
        Dev &d = h->d;
    d.S = h->S; d.L = L; d.Nn = Nn; d.O = h->O; d.N = h->N; d.D = h->D; d.nb = h->nb; d.cbs = h->cbs;
    d.n_dest = (int)h->dest_nodes.size(); d.maxl = maxl; d.n_rate_bins = h->B;
    d.fixed_mode = h->fixed_mode; d.allow_uturn = cfg->allow_uturn; d.platoon = h->platoon;
    d.g_link = h->g_link; d.g_node = h->g_node; d.g_rev = h->g_rev;
    d.ring_total = h->ring_total; d.dt = h->dt; d.theta = cfg->dest_logit_coef; d.rate_bin_s = h->rate_bin_s;
    d.big_m = cfg->big_m; d.tau = cfg->gumbel_tau;
    d.rate_bin_steps = h->fixed_mode ? 1 : std::max(1, (int)std::lround(h->rate_bin_s / h->dt));
    d.tail = h->upload(h->tail); d.head = h->upload(h->head); d.lanes = h->upload(h->lanes);
    h->linv_dev = h->upload(h->linv);
    d.cap = h->upload(h->cap); d.ring_base = h->upload(h->ring_base);
    d.length = h->upload(h->length);
    std::vector<float> thr(L);
    for (int j = 0; j < L; ++j) thr[j] = h->length[j] - 0.01f;
    d.thr = h->upload(thr);
    d.out_off = h->upload(h->out_off); d.out_lnk = h->upload(h->out_lnk);
    d.in_off = h->upload(h->in_off); d.in_lnk = h->upload(h->in_lnk);
    d.org_off = h->upload(h->org_off); d.org_list = h->upload(h->org_list);
    d.det_off = h->upload(h->det_off); d.det_list = h->upload(h->det_list);
    d.det_pos = h->upload(h->det_pos);
    d.tff = h->upload(h->tff);
    d.route = h->upload(h->route); d.route_base = h->upload(h->route_base);
    d.agent_didx = h->upload(h->agent_didx); d.agent_dest = h->upload(h->agent_dest);
    d.agent_origin = h->upload(h->agent_origin);
    h->q_off_dev = h->upload(h->q_off);
    h->q_list_dev = h->dalloc<int32_t>(h->q_list.size());
    h->q_dest_dev = h->dalloc<int32_t>(h->q_list.size());
    h->q_didx_dev = h->dalloc<int32_t>(h->q_list.size());
    h->q_rstep_dev = h->dalloc<int64_t>(h->q_rstep.size());
    h->cand_dev = h->dalloc<int2>(h->cand.size());
    upload_queues(h);
    h->queues_unplaced = h->placed.empty();   // the queues of create: every agent waits at its origin
    d.q_off = h->q_off_dev; d.q_list = h->q_list_dev; d.q_rstep = h->q_rstep_dev;
    d.q_dest = h->q_dest_dev; d.q_didx = h->q_didx_dev;
    d.node_cnt = h->upload(h->node_cnt); d.in_pad = h->upload(h->in_pad); d.out_pad = h->upload(h->out_pad);
    d.in_loff = h->upload(h->in_loff); d.cand = h->cand_dev; d.max_cand = h->max_cand;
    d.cbase = h->upload(h->cbase); d.n_cand = h->n_cand;
    d.max_in = h->max_in; d.max_out = h->max_out; d.max_org = h->max_org;
    d.seed = h->upload(h->seeds);
    // parameters, scenario-major
    auto rep = [&](const std::vector<float> &v) {
        std::vector<float> r((size_t)h->S * v.size());
        for (int s = 0; s < h->S; ++s) std::copy(v.begin(), v.end(), r.begin() + (size_t)s * v.size());
        return r;
    };
    h->p_u = h->upload(rep(h->free_speed)); h->p_kappa = h->upload(rep(h->jam_density));
    h->p_beta = h->upload(rep(h->beta)); h->p_alpha = h->upload(rep(h->alpha)); h->p_cost = h->upload(rep(h->cost));
    h->p_capm = h->upload(rep(std::vector<float>(L, 1.f)));
    h->p_rates = h->fixed_mode ? h->dalloc<float>(1) : h->upload(rep(h->rates));
    h->capacity_dev = h->upload(h->capacity);
    d.capm = h->p_capm; d.capacity = h->capacity_dev;
    d.u = h->p_u; d.kappa = h->p_kappa; d.alpha = h->p_alpha; d.rates = h->p_rates;
    d.beta = h->p_beta; d.cost = h->p_cost;
    h->vfree = h->dalloc<float>(SL); h->spacing = h->dalloc<float>(SL);
    h->util = h->dalloc<double>(SL); h->acc = h->dalloc<double>(SL);
    d.vfree = h->vfree; d.spacing = h->spacing; d.util = h->util; d.acc = h->acc;
    // state
    d.ring_pos = h->dalloc<float>(SR); d.ring_agent = h->dalloc<int32_t>(SR); d.ring_aux = h->dalloc<int2>(SR);
    d.ls = h->dalloc<sim::LinkSt>(SL);
    h->lnd_dev = h->dalloc<sim::LinkNd>(SL);
    d.lnd = h->lnd_dev;
    h->lcf_dev = h->dalloc<sim::LinkCf>(SL);
    d.lcf = h->lcf_dev;
    h->rcf_dev = h->dalloc<sim::RevCf>(SL);
    d.rcf = h->rcf_dev;
    d.head_rec = h->dalloc<int4>(SL * maxl);
    d.status = h->dalloc<uint8_t>(SN); d.tstar = h->dalloc<double>(SN);
    d.rel_t = h->dalloc<int32_t>(SN); d.dep_t = h->dalloc<int32_t>(SN); d.exit_t = h->dalloc<int32_t>(SN);
    d.Dacc = h->dalloc<double>(SO); d.rel_ptr = h->dalloc<int32_t>(SO); d.dep_ptr = h->dalloc<int32_t>(SO);
    d.ctr = h->dalloc<int64_t>((size_t)h->S * sim::kCtrSlots * sim::CTR_N);
    d.cum = h->dalloc<int32_t>((size_t)h->S * h->D * std::max(h->nb, 1));
    d.err = h->dalloc<int32_t>(sim::ERR_N);
    d.tie_log = h->dalloc<int32_t>((size_t)6 * sim::kTieLogMax);
    d.tie_n = h->dalloc<int32_t>(1);
    d.tie_cap = sim::kTieLogMax;
    h->ttt_dev = h->dalloc<double>(h->S);
    h->ttt_acc = h->dalloc<unsigned long long>(2 * (size_t)h->S);
    h->counts_dev = h->dalloc<float>((size_t)h->S * h->D * std::max(h->nb, 1));
    if (h->record) {
        h->ckpts.resize(n_ck + 1);
        for (auto &c : h->ckpts) ckpt_alloc(h, c);
        h->tapes.resize((size_t)h->n_tape_sets);
        for (auto &ts : h->tapes) {
            ts.pos = h->dalloc<float>((size_t)(h->W + 1) * SR);
            ts.agent = h->dalloc<int32_t>((size_t)(h->W + 1) * SR);
            ts.seg = h->dalloc<int4>((size_t)(h->W + 1) * SL);
            ts.dst = h->dalloc<int32_t>((size_t)(h->W + 1) * SL * maxl);
            ts.dstg = h->dalloc<float>((size_t)(h->W + 1) * SL * maxl);
            ts.ste = h->dalloc<int4>((size_t)(h->W + 1) * h->S * std::max(h->n_cand, 1));
        }
        d.tape_pos = h->tapes[0].pos; d.tape_agent = h->tapes[0].agent;
        d.tape_seg = h->tapes[0].seg;
        h->rp_dev.assign((size_t)h->n_replay, d);
        h->rp_stream.assign((size_t)h->n_replay, nullptr);
        for (int k = 0; k < h->n_replay; ++k) {
            Dev &r = h->rp_dev[k];   // mutable state of replay slot k (errors go to the shared flags)
            r.tie_log = nullptr;     // a replay repeats decisions already logged by the forward
            r.tie_n = nullptr;
            r.ring_pos = h->dalloc<float>(SR); r.ring_agent = h->dalloc<int32_t>(SR); r.ring_aux = h->dalloc<int2>(SR);
            r.ls = h->dalloc<sim::LinkSt>(SL);
            r.dB = h->dalloc<double>(SL); r.head_rec = h->dalloc<int4>(SL * maxl);
            r.status = h->dalloc<uint8_t>(SN); r.tstar = h->dalloc<double>(SN);
            r.rel_t = h->dalloc<int32_t>(SN); r.dep_t = h->dalloc<int32_t>(SN); r.exit_t = h->dalloc<int32_t>(SN);
            r.Dacc = h->dalloc<double>(SO); r.rel_ptr = h->dalloc<int32_t>(SO); r.dep_ptr = h->dalloc<int32_t>(SO);
            r.ctr = h->dalloc<int64_t>((size_t)h->S * sim::kCtrSlots * sim::CTR_N);
            r.cum = h->dalloc<int32_t>((size_t)h->S * h->D * std::max(h->nb, 1));
            HIPCHK(hipStreamCreateWithFlags(&h->rp_stream[k], hipStreamNonBlocking));
        }
        h->bw_events.resize(2 * (size_t)n_ck + 2, nullptr);
        for (auto &e : h->bw_events) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        d.adj_ring = h->dalloc<float>(SR); d.depg = h->dalloc<float>(SN);
        d.tape_dst = h->tapes[0].dst;
        d.gu = h->dalloc<double>(SL); d.gk = h->dalloc<double>(SL);
        d.dB = h->dalloc<double>(SL);
        h->tape_dstg_buf = h->tapes[0].dstg;
        h->gm_buf = h->dalloc<double>(SL);
        d.tape_dstg = nullptr; d.gm = nullptr;
        h->gbeta_buf = h->dalloc<double>(SL); h->gcost_buf = h->dalloc<double>(SL);
        h->galpha_buf = h->dalloc<double>(SL); h->gth_buf = h->dalloc<double>((size_t)h->S * Nn);
        d.tape_ste = nullptr; d.gbeta = d.gcost = d.galpha = d.gth = nullptr;
        h->gQ_dev = h->dalloc<float>((size_t)h->S * h->D * std::max(h->nb, 1));
        h->gx_dev = h->dalloc<float>(SN);
        h->gT_dev = h->dalloc<double>(h->S);
        h->grad_tmp = h->dalloc<float>(std::max(SL, (size_t)h->S * h->O * std::max(h->B, 1)));
    }
    build_classes(h);
    derive(h);
    zero_state(h);
    HIPCHK(hipStreamSynchronize(h->stream));
}

}  // namespace

// ===========================================================================
// internal hooks for the serving loop (sim_serve.cpp)
// ===========================================================================
namespace sim {

sim_t *host_prepare(const sim_network *net, const sim_demand *dem, const sim_config *cfg, int device,
                    int *code, std::string *err)
{
    sim_t *h = nullptr;
    try {
        h = new sim_t();
        h->device = device;
        sim_config c = *cfg;
        c.mem_budget_bytes = 0;
        prepare_host(h, net, dem, &c);
        h->theta_cfg = cfg->dest_logit_coef;
        h->uturn_cfg = cfg->allow_uturn;
        *code = SIM_OK;
        return h;
    } catch (const InvalidArg &e) {
        delete h;
        *code = e.code;
        *err = e.msg;
    } catch (const std::bad_alloc &) {
        delete h;
        *code = SIM_ENOMEM;
        *err = "host allocation failed";
    }
    return nullptr;
}

size_t footprint_of(const sim_t *h) { return h->footprint; }

int device_attach(sim_t *h, hipStream_t stream, void *arena, size_t arena_bytes, std::string *err)
{
    try {
        h->stream = stream;
        h->arena = static_cast<char *>(arena);
        h->arena_cap = arena ? arena_bytes : 0;
        h->arena_off = 0;
        HIPCHK(hipSetDevice(h->device));
        sim_config c{};
        c.dest_logit_coef = h->theta_cfg;
        c.allow_uturn = h->uturn_cfg;
        allocate_device(h, &c);
        return SIM_OK;
    } catch (const InvalidArg &e) {
        *err = e.msg;
        return e.code;
    } catch (const HipError &e) {
        *err = e.msg;
        return SIM_EDEVICE;
    } catch (const std::bad_alloc &) {
        *err = "host allocation failed";
        return SIM_ENOMEM;
    }
}

// enqueue T steps on the handle's stream without waiting
int rollout_enqueue(sim_t *h, int T, std::string *err)
{
    try {
        HIPCHK(hipSetDevice(h->device));
        for (int k = 0; k < T; ++k) do_step(h, -1);
        return SIM_OK;
    } catch (const HipError &e) {
        *err = e.msg;
        return SIM_EDEVICE;
    }
}

// enqueue the observables into caller buffers (host memory, pinned for asynchrony)
int results_enqueue(sim_t *h, float *counts, double *ttt, int64_t *vsteps, std::string *err)
{
    try {
        HIPCHK(hipSetDevice(h->device));
        if (counts && h->D * h->nb > 0) {
            sim::launch_counts(h->d, h->counts_dev, h->stream);
            HIPCHK(hipMemcpyAsync(counts, h->counts_dev, (size_t)h->S * h->D * h->nb * 4, hipMemcpyDeviceToHost, h->stream));
        }
        int64_t *dv = h->dalloc_scratch_i64(h->S);
        sim::launch_ttt(h->d, h->t, h->ttt_dev, dv, h->ttt_acc, h->stream);
        if (ttt) HIPCHK(hipMemcpyAsync(ttt, h->ttt_dev, (size_t)h->S * 8, hipMemcpyDeviceToHost, h->stream));
        if (vsteps) HIPCHK(hipMemcpyAsync(vsteps, dv, (size_t)h->S * 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipGetLastError());
        return SIM_OK;
    } catch (const HipError &e) {
        *err = e.msg;
        return SIM_EDEVICE;
    } catch (const InvalidArg &e) {
        *err = e.msg;
        return e.code;
    }
}

int device_errors(sim_t *h, std::string *err)
{
    try {
        check_device_errors(h);
        return SIM_OK;
    } catch (const InvalidArg &e) {
        *err = e.msg;
        return e.code;
    } catch (const HipError &e) {
        *err = e.msg;
        return SIM_EDEVICE;
    }
}

hipStream_t stream_of(const sim_t *h) { return h->stream; }
int device_of(const sim_t *h) { return h->device; }
int detectors_of(const sim_t *h) { return h->D; }
int count_bins_of(const sim_t *h) { return h->nb; }
int max_steps_of(const sim_t *h) { return h->max_steps; }
bool is_recording(const sim_t *h) { return h->record != 0; }
bool rate_mode(const sim_t *h) { return !h->fixed_mode; }
int64_t group_size(const sim_t *h, int which)
{
    switch (which) {
    case SIM_P_U: case SIM_P_KAPPA: case SIM_P_BETA: case SIM_P_ALPHA: case SIM_P_COST: case SIM_P_CAP_MULT:
        return h->L;
    case SIM_P_RATES: return h->fixed_mode ? -1 : (int64_t)h->O * h->B;
    case SIM_P_THETA_DEST: return 1;
    default: return -1;
    }
}
void kappa_ceiling(const sim_t *h, float *out)
{
    for (int j = 0; j < h->L; ++j) out[j] = h->jam_density[h->linv[j]];
}
int set_error(sim_t *h, int code, const std::string &msg) { return record_error(h, code, msg); }
int counts_size(const sim_t *h) { return h->S * h->D * h->nb; }
int scenarios_of(const sim_t *h) { return h->S; }
void destroy_handle(sim_t *h) { delete h; }
// the handle's stream has no work left (its last event completed): free host state without waiting
void release_handle(sim_t *h)
{
    if (!h) return;
    h->stream = nullptr;
    delete h;
}
int64_t arena_fallbacks(const sim_t *h) { return h->arena_fallbacks; }

}  // namespace sim

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

const char *sim_last_error(const sim_t *h) { return h ? h->err.c_str() : g_create_error.c_str(); }

int sim_create(const sim_network *net, const sim_demand *dem, const sim_config *cfg, int hip_device,
               void *hip_stream, sim_t **out)
{
    if (!out) return record_error(nullptr, SIM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!net || !dem || !cfg) return record_error(nullptr, SIM_EINVAL, "null input struct");
    sim_t *h = nullptr;
    try {
        h = new sim_t();
        h->device = hip_device;
        h->stream = (hipStream_t)hip_stream;
        int ndev = 0;
        HIPCHK(hipGetDeviceCount(&ndev));
        if (hip_device < 0 || hip_device >= ndev) fail(SIM_EINVAL, "bad device index");
        HIPCHK(hipSetDevice(hip_device));
        // device address of the allocation-free sort's fixed scratch array, once per device
        if (hip_device < sim::kMaxDevices && sim::segsort_scratch_init(hip_device) != 0)
            fail(SIM_EDEVICE, "hipGetSymbolAddress of the sort scratch array failed");
        prepare_host(h, net, dem, cfg);
        allocate_device(h, cfg);
        *out = h;
        return SIM_OK;
    } catch (const InvalidArg &e) {
        delete h;
        return record_error(nullptr, e.code, e.msg);
    } catch (const HipError &e) {
        delete h;
        return record_error(nullptr, SIM_EDEVICE, e.msg);
    } catch (const std::bad_alloc &) {
        delete h;
        return record_error(nullptr, SIM_ENOMEM, "host allocation failed");
    }
}

int sim_footprint(const sim_network *net, const sim_demand *dem, const sim_config *cfg, size_t *bytes)
{
    if (!net || !dem || !cfg || !bytes) return record_error(nullptr, SIM_EINVAL, "null argument");
    sim_t *h = nullptr;
    try {
        h = new sim_t();
        h->device = -1;
        sim_config c = *cfg;
        c.mem_budget_bytes = 0;
        prepare_host(h, net, dem, &c);
        *bytes = h->footprint;
        delete h;
        return SIM_OK;
    } catch (const InvalidArg &e) {
        delete h;
        return record_error(nullptr, e.code, e.msg);
    } catch (const std::bad_alloc &) {
        delete h;
        return record_error(nullptr, SIM_ENOMEM, "host allocation failed");
    }
}

int sim_destroy(sim_t *h)
{
    delete h;
    return SIM_OK;
}

int sim_set_params(sim_t *h, int which, const float *values, int64_t n, int on_device)
{
    return guarded(h, [&] {
        if (!values) fail(SIM_EINVAL, "values is NULL");
        // a rollout recorded under other parameters can no longer be replayed
        if (h->t > 0) h->rec_valid = false;
        float *dst = nullptr;
        int64_t per = h->L;
        switch (which) {
        case SIM_P_U: dst = h->p_u; break;
        case SIM_P_KAPPA: dst = h->p_kappa; break;
        case SIM_P_BETA: dst = h->p_beta; break;
        case SIM_P_ALPHA: dst = h->p_alpha; break;
        case SIM_P_COST: dst = h->p_cost; break;
        case SIM_P_CAP_MULT: dst = h->p_capm; break;
        case SIM_P_RATES:
            if (h->fixed_mode) fail(SIM_EINVAL, "rates need departure-rate mode");
            dst = h->p_rates; per = (int64_t)h->O * h->B; break;
        default: fail(SIM_EINVAL, "unknown parameter group");
        }
        if (n != per * h->S) fail(SIM_EINVAL, "expected " + std::to_string(per * h->S) + " values");
        std::vector<float> host(n);
        HIPCHK(hipMemcpyAsync(host.data(), values, n * 4, on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        if (which != SIM_P_RATES) host = links_in(h, host.data());   // to the internal link order
        for (int64_t i = 0; i < n; ++i) {
            const float v = host[i];
            if (!std::isfinite(v)) fail(SIM_EINVAL, "non-finite parameter");
            if ((which == SIM_P_U || which == SIM_P_KAPPA || which == SIM_P_COST) && !(v > 0.f))
                fail(SIM_EINVAL, "u, kappa and cost must be > 0");
            if (which == SIM_P_RATES && !(v >= 0.f)) fail(SIM_EINVAL, "rates must be >= 0");
            if (which == SIM_P_CAP_MULT && !(v >= 0.f)) fail(SIM_EINVAL, "capacity multipliers must be >= 0");
            if (which == SIM_P_KAPPA) {
                const int j = (int)(i % h->L);
                if ((float)h->platoon / v < h->min_spacing[j])
                    fail(SIM_EINVAL, "kappa above the value the link rings were sized for");
            }
        }
        HIPCHK(hipMemcpyAsync(dst, host.data(), n * 4, hipMemcpyHostToDevice, h->stream));
        derive(h);
        HIPCHK(hipStreamSynchronize(h->stream));
    });
}

int sim_get_params(sim_t *h, int which, float *values, int64_t n, int on_device)
{
    return guarded(h, [&] {
        if (!values) fail(SIM_EINVAL, "values is NULL");
        const float *src = nullptr;
        int64_t per = h->L;
        switch (which) {
        case SIM_P_U: src = h->p_u; break;
        case SIM_P_KAPPA: src = h->p_kappa; break;
        case SIM_P_BETA: src = h->p_beta; break;
        case SIM_P_ALPHA: src = h->p_alpha; break;
        case SIM_P_COST: src = h->p_cost; break;
        case SIM_P_CAP_MULT: src = h->p_capm; break;
        case SIM_P_RATES:
            if (h->fixed_mode) fail(SIM_EINVAL, "rates need departure-rate mode");
            src = h->p_rates; per = (int64_t)h->O * h->B; break;
        default: fail(SIM_EINVAL, "unknown parameter group");
        }
        if (n != per * h->S) fail(SIM_EINVAL, "expected " + std::to_string(per * h->S) + " values");
        std::vector<float> host((size_t)n), out((size_t)n);
        HIPCHK(hipMemcpyAsync(host.data(), src, n * 4, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        if (which == SIM_P_RATES) out = host;
        else
            for (int s = 0; s < h->S; ++s)
                for (int k = 0; k < h->L; ++k) out[(size_t)s * h->L + h->lperm[k]] = host[(size_t)s * h->L + k];
        HIPCHK(hipMemcpyAsync(values, out.data(), n * 4, on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost,
                              h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    });
}

int sim_reset(sim_t *h)
{
    return guarded(h, [&] {
        h->placed.clear();
        if (!h->queues_unplaced) {
            build_queues(h, nullptr);
            upload_queues(h);
            h->queues_unplaced = true;
        }
        zero_state(h);
        HIPCHK(hipStreamSynchronize(h->stream));
    });
}

int sim_place(sim_t *h, int32_t n, const int32_t *agent, const int32_t *link, const float *pos)
{
    return guarded(h, [&] {
        if (h->t != 0) fail(SIM_ESTATE, "sim_place is only allowed at t = 0");
        if (n < 0 || (n > 0 && (!agent || !link || !pos))) fail(SIM_EINVAL, "bad placement arrays");
        std::vector<uint8_t> placed = h->placed;
        if (placed.empty()) placed.assign(h->N, 0);
        std::vector<int32_t> cnt(h->L, 0), lk(n > 0 ? n : 1);
        for (int k = 0; k < n; ++k) {
            if (agent[k] < 0 || agent[k] >= h->N || placed[agent[k]]) fail(SIM_EINVAL, "bad or repeated agent");
            if (link[k] < 0 || link[k] >= h->L) fail(SIM_EINVAL, "bad link");
            lk[k] = h->linv[link[k]];
            if (!(pos[k] >= 0.f) || !(pos[k] <= h->length[lk[k]])) fail(SIM_EINVAL, "position outside the link");
            placed[agent[k]] = 1;
            if (++cnt[lk[k]] > h->cap[lk[k]]) fail(SIM_EINVAL, "too many agents placed on a link");
        }
        // current (empty, t = 0) rings and per-agent arrays
        const size_t SR = (size_t)h->S * h->ring_total, SL = (size_t)h->S * h->L, SN = (size_t)h->S * h->N;
        std::vector<float> rp(SR, 0.f);
        std::vector<int32_t> ra(SR, 0);
        std::vector<sim::LinkSt> ls(SL);
        std::vector<int2> rx(SR);
        HIPCHK(hipMemcpyAsync(rx.data(), h->d.ring_aux, SR * 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(ls.data(), h->d.ls, SL * sizeof(sim::LinkSt), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(rp.data(), h->d.ring_pos, SR * 4, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(ra.data(), h->d.ring_agent, SR * 4, hipMemcpyDeviceToHost, h->stream));
        std::vector<uint8_t> st(SN);
        std::vector<int32_t> relt(SN), dept(SN);
        HIPCHK(hipMemcpyAsync(st.data(), h->d.status, SN, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(relt.data(), h->d.rel_t, SN * 4, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(dept.data(), h->d.dep_t, SN * 4, hipMemcpyDeviceToHost, h->stream));
        std::vector<int64_t> ctr((size_t)h->S * sim::kCtrSlots * sim::CTR_N);
        HIPCHK(hipMemcpyAsync(ctr.data(), h->d.ctr, ctr.size() * 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (int s = 0; s < h->S; ++s) {
            for (int k = 0; k < n; ++k) {
                const int j = lk[k];
                const size_t seg = (size_t)s * h->L + j;
                const size_t slot = (size_t)s * h->ring_total + h->ring_base[j] + (ls[seg].rtail % h->cap[j]);
                ra[slot] = agent[k];
                rx[slot] = make_int2(h->agent_dest[agent[k]], h->agent_didx[agent[k]]);
                rp[slot] = pos[k];
                ls[seg].rtail += 1;
                const size_t ga = (size_t)s * h->N + agent[k];
                st[ga] = sim::AG_ON;
                relt[ga] = 0;
                dept[ga] = -2;   // placed, not departed: no departure graft
            }
            ctr[(size_t)s * sim::kCtrSlots * sim::CTR_N + sim::CTR_RELEASED] += n;
            ctr[(size_t)s * sim::kCtrSlots * sim::CTR_N + sim::CTR_DEPARTED] += n;
        }
        HIPCHK(hipMemcpyAsync(h->d.ls, ls.data(), SL * sizeof(sim::LinkSt), hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->d.ring_pos, rp.data(), SR * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->d.ring_agent, ra.data(), SR * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->d.ring_aux, rx.data(), SR * 8, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->d.status, st.data(), SN, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->d.rel_t, relt.data(), SN * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->d.dep_t, dept.data(), SN * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->d.ctr, ctr.data(), ctr.size() * 8, hipMemcpyHostToDevice, h->stream));
        h->placed = placed;
        h->queues_unplaced = false;
        build_queues(h, &h->placed);
        upload_queues(h);
        HIPCHK(hipStreamSynchronize(h->stream));
    });
}

int sim_step(sim_t *h)
{
    return sim_rollout(h, 1);
}

int sim_rollout(sim_t *h, int32_t T)
{
    return guarded(h, [&] {
        if (T < 0) fail(SIM_EINVAL, "T < 0");
        // only the windows that end up as the last tapes.size() of this call are taped as the
        // forward goes (taping costs a load and a store per agent and step)
        const int64_t t_end = (int64_t)h->t + T;
        const int64_t first_taped = t_end > 0 ? (t_end - 1) / h->ckpt_every - (int64_t)h->tapes.size() + 1 : 0;
        for (int k = 0; k < T; ++k) {
            if (h->record && h->rec_valid) {
                if (h->t >= h->max_steps) h->rec_valid = false;
                else if (h->t % h->ckpt_every == 0) {
                    Ckpt &c = h->ckpts[h->t / h->ckpt_every];
                    hipEvent_t e = nullptr;
                    h->time_begin(3, &e);
                    ckpt_copy(h, c, true);
                    h->time_end(3, e);
                    c.t = h->t;
                }
            }
            if (h->record && h->rec_valid && h->t / h->ckpt_every < first_taped) {
                const int w = h->t / h->ckpt_every, set = w % (int)h->tapes.size();
                if (h->tape_win[set] == w) h->tape_win[set] = -1;
                do_step(h, -1);
            } else if (h->record && h->rec_valid) {
                // the window's tape, written as the forward goes: the last windows then need no replay
                const int w = h->t / h->ckpt_every, kw = h->t % h->ckpt_every;
                const int set = w % (int)h->tapes.size();
                if (kw == 0) { h->tape_win[set] = w; h->tape_steps[set] = 0; }
                const bool contiguous = h->tape_win[set] == w && h->tape_steps[set] == kw;
                Dev dt = h->d;
                const auto &ts = h->tapes[set];
                dt.tape_pos = ts.pos; dt.tape_agent = ts.agent; dt.tape_seg = ts.seg;
                dt.tape_dst = ts.dst; dt.tape_dstg = nullptr; dt.tape_ste = nullptr;
                step_on(h, dt, h->stream, h->t, contiguous ? kw : -1);
                h->t += 1;
                if (contiguous) {
                    h->tape_steps[set] = kw + 1;
                    if (kw + 1 == h->ckpt_every) sim::launch_tape_snapshot(dt, h->ckpt_every, h->stream);
                } else {
                    h->tape_win[set] = -1;
                }
            } else {
                do_step(h, -1);
            }
        }
        if (h->timing) h->resolve_timing();
        check_device_errors(h);
    });
}

int sim_get_observables(sim_t *h, float *counts, double *ttt, int on_device)
{
    return guarded(h, [&] {
        if (counts && h->D * h->nb > 0) {
            sim::launch_counts(h->d, h->counts_dev, h->stream);
            copy_out(h, counts, h->counts_dev, (size_t)h->S * h->D * h->nb * 4, on_device);
        }
        if (ttt) {
            sim::launch_ttt(h->d, h->t, h->ttt_dev, nullptr, h->ttt_acc, h->stream);
            copy_out(h, ttt, h->ttt_dev, (size_t)h->S * 8, on_device);
        }
        HIPCHK(hipGetLastError());
        if (!on_device) HIPCHK(hipStreamSynchronize(h->stream));
    });
}

int sim_backward(sim_t *h, const float *dL_dcounts, const double *dL_dttt, const float *dL_dpos,
                 uint32_t param_mask, float *const *grads, int on_device)
{
    return guarded(h, [&] {
        if (!h->record) fail(SIM_ESTATE, "handle was created without record_for_backward");
        if (!h->rec_valid || h->t == 0 || h->ckpts[0].t != 0)
            fail(SIM_ESTATE, "sim_backward needs a recorded rollout from t = 0 (at most max_steps)");
        if (param_mask >> SIM_P_COUNT) fail(SIM_EINVAL, "unknown gradient group in param_mask");
        const bool want_m = (param_mask & (1u << SIM_P_CAP_MULT)) != 0;
        const uint32_t ste_mask = (1u << SIM_P_BETA) | (1u << SIM_P_COST) | (1u << SIM_P_ALPHA) | (1u << SIM_P_THETA_DEST);
        const bool want_ste = (param_mask & ste_mask) != 0;
        if (want_ste && !(h->d.tau > 0.0)) fail(SIM_EINVAL, "straight-through gradients need gumbel_tau > 0");
        h->d.tape_dstg = want_m ? h->tape_dstg_buf : nullptr;
        h->d.gm = want_m ? h->gm_buf : nullptr;
        h->d.gbeta = want_ste ? h->gbeta_buf : nullptr;
        h->d.gcost = want_ste ? h->gcost_buf : nullptr;
        h->d.galpha = want_ste ? h->galpha_buf : nullptr;
        h->d.gth = want_ste ? h->gth_buf : nullptr;
        if ((param_mask & (1u << SIM_P_RATES)) && h->fixed_mode) fail(SIM_EINVAL, "rates need departure-rate mode");
        if (param_mask && !grads) fail(SIM_EINVAL, "grads is NULL");
        Dev d = h->d;
        const hipStream_t st = h->stream;
        const size_t SL = (size_t)h->S * h->L, SN = (size_t)h->S * h->N;
        const size_t nQ = (size_t)h->S * h->D * h->nb;
        const hipMemcpyKind kin = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        d.gQ = nullptr; d.gT = nullptr; d.gx = nullptr;
        if (dL_dcounts && nQ) { HIPCHK(hipMemcpyAsync(h->gQ_dev, dL_dcounts, nQ * 4, kin, st)); d.gQ = h->gQ_dev; }
        if (dL_dttt) { HIPCHK(hipMemcpyAsync(h->gT_dev, dL_dttt, h->S * 8, kin, st)); d.gT = h->gT_dev; }
        if (dL_dpos) { HIPCHK(hipMemcpyAsync(h->gx_dev, dL_dpos, SN * 4, kin, st)); d.gx = h->gx_dev; }
        HIPCHK(hipMemsetAsync(d.adj_ring, 0, (size_t)h->S * h->ring_total * 4, st));
        HIPCHK(hipMemsetAsync(d.depg, 0, SN * 4, st));
        HIPCHK(hipMemsetAsync(d.gu, 0, SL * 8, st));
        HIPCHK(hipMemsetAsync(d.gk, 0, SL * 8, st));
        if (want_m) HIPCHK(hipMemsetAsync(d.gm, 0, SL * 8, st));
        if (want_ste) {
            HIPCHK(hipMemsetAsync(d.gbeta, 0, SL * 8, st));
            HIPCHK(hipMemsetAsync(d.gcost, 0, SL * 8, st));
            HIPCHK(hipMemsetAsync(d.galpha, 0, SL * 8, st));
            HIPCHK(hipMemsetAsync(d.gth, 0, (size_t)h->S * h->Nn * 8, st));
        }
        const int T = h->t;
        const int nw = (T + h->ckpt_every - 1) / h->ckpt_every;
        // in timing mode the windows run one after another (one replay slot, each replay after the
        // previous sweep), so that per-kernel times are not stretched by concurrent kernels
        const int K = h->timing ? 1 : h->n_replay, NT = (int)h->tapes.size();
        // Window w is replayed from its checkpoint by slot w % K (its own copy of the mutable state,
        // on its own stream) into tape set w % NT, then swept in reverse on the main stream.
        // Up to K replays run at once beside the sweep; the live state is never touched.  A replay
        // waits for the sweep that last read its tape set; a sweep waits for its window's replay.
        hipEvent_t *rp_done = h->bw_events.data(), *rv_done = h->bw_events.data() + nw;
        hipEvent_t start = h->bw_events[2 * (size_t)nw];
        auto use_tapes = [&](Dev &dv, int set) {
            const auto &ts = h->tapes[set];
            dv.tape_pos = ts.pos; dv.tape_agent = ts.agent; dv.tape_seg = ts.seg;
            dv.tape_dst = ts.dst;
            dv.tape_dstg = want_m ? ts.dstg : nullptr;
            dv.tape_ste = want_ste ? ts.ste : nullptr;
        };
        // windows whose whole tape the forward wrote (the last NT windows) are swept without a
        // replay, unless the requested groups need tapes the forward does not write
        auto fwd_taped = [&](int w) {
            if (want_m || want_ste) return false;
            const int t0 = w * h->ckpt_every, Ww = std::min(h->ckpt_every, T - t0);
            return h->tape_win[w % NT] == w && h->tape_steps[w % NT] == Ww;
        };
        if (fwd_taped(nw - 1) && T - (nw - 1) * h->ckpt_every < h->ckpt_every) {
            Dev dl = h->d;   // the final partial window ends at the live state
            use_tapes(dl, (nw - 1) % NT);
            sim::launch_tape_snapshot(dl, T - (nw - 1) * h->ckpt_every, st);
        }
        HIPCHK(hipEventRecord(start, st));
        std::vector<char> slot_used((size_t)K, 0);
        auto replay = [&](int w) {
            if (fwd_taped(w)) return;
            const int t0 = w * h->ckpt_every, Ww = std::min(h->ckpt_every, T - t0);
            const int slot = w % K;
            const hipStream_t rs = h->rp_stream[slot];
            if (!slot_used[slot]) HIPCHK(hipStreamWaitEvent(rs, start, 0));   // first use of the slot in this call
            slot_used[slot] = 1;
            if (w + NT <= nw - 1) HIPCHK(hipStreamWaitEvent(rs, rv_done[w + NT], 0));
            if (h->timing && w + 1 <= nw - 1) HIPCHK(hipStreamWaitEvent(rs, rv_done[w + 1], 0));
            Dev r = h->d;
            with_state(r, h->rp_dev[slot]);
            use_tapes(r, w % NT);
            hipEvent_t e = nullptr;
            h->time_begin(3, &e, rs);
            ckpt_copy(h, h->ckpts[w], false, &r, rs);
            h->time_end(3, e, rs);
            for (int k = 0; k < Ww; ++k) step_on(h, r, rs, t0 + k, k);
            sim::launch_tape_snapshot(r, Ww, rs);
            HIPCHK(hipEventRecord(rp_done[w], rs));
        };
        for (int w = nw - 1; w >= std::max(0, nw - K); --w) replay(w);
        for (int w = nw - 1; w >= 0; --w) {
            const int t0 = w * h->ckpt_every, Ww = std::min(h->ckpt_every, T - t0);
            if (!fwd_taped(w)) HIPCHK(hipStreamWaitEvent(st, rp_done[w], 0));
            use_tapes(d, w % NT);
            if (w == nw - 1) sim::launch_reverse(d, T, Ww, 1, st);
            for (int k = Ww - 1; k >= 0; --k) {
                if (want_ste) sim::launch_ste(d, t0 + k, k, st);   // reads dL/dx(t+1) before the reverse replaces it
                hipEvent_t er = nullptr;
                h->time_begin(6, &er, st);
                sim::launch_reverse(h->stamped(d, 2, sim::reverse_blocks(d)), t0 + k, k, 0, st);
                h->time_end(6, er, st);
            }
            HIPCHK(hipEventRecord(rv_done[w], st));
            if (w - K >= 0) replay(w - K);
            HIPCHK(hipGetLastError());
        }
        // the main stream has waited for every replay (each sweep waits for its own); replays have
        // reused the tape sets
        h->tape_win.assign(h->tapes.size(), -1);
        h->d.gQ = nullptr; h->d.gT = nullptr; h->d.gx = nullptr;
        h->d.tape_dstg = nullptr; h->d.gm = nullptr;
        h->d.gbeta = h->d.gcost = h->d.galpha = h->d.gth = nullptr;
        const hipMemcpyKind kout = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        if (param_mask & (1u << SIM_P_U)) {
            sim::launch_gather_links(d.gu, h->linv_dev, h->grad_tmp, h->S, h->L, st);
            HIPCHK(hipMemcpyAsync(grads[SIM_P_U], h->grad_tmp, SL * 4, kout, st));
        }
        if (param_mask & (1u << SIM_P_KAPPA)) {
            sim::launch_gather_links(d.gk, h->linv_dev, h->grad_tmp, h->S, h->L, st);
            HIPCHK(hipMemcpyAsync(grads[SIM_P_KAPPA], h->grad_tmp, SL * 4, kout, st));
        }
        if (want_m) {
            sim::launch_gather_links(d.gm, h->linv_dev, h->grad_tmp, h->S, h->L, st);
            HIPCHK(hipMemcpyAsync(grads[SIM_P_CAP_MULT], h->grad_tmp, SL * 4, kout, st));
        }
        const std::pair<int, double *> ste_links[3] = {
            {SIM_P_BETA, d.gbeta}, {SIM_P_COST, d.gcost}, {SIM_P_ALPHA, d.galpha}};
        for (const auto &pg : ste_links) {
            if (!(param_mask & (1u << pg.first))) continue;
            sim::launch_gather_links(pg.second, h->linv_dev, h->grad_tmp, h->S, h->L, st);
            HIPCHK(hipMemcpyAsync(grads[pg.first], h->grad_tmp, SL * 4, kout, st));
        }
        if (param_mask & (1u << SIM_P_THETA_DEST)) {
            sim::launch_theta_sum(d, h->grad_tmp, st);
            HIPCHK(hipMemcpyAsync(grads[SIM_P_THETA_DEST], h->grad_tmp, (size_t)h->S * 4, kout, st));
        }
        if (param_mask & (1u << SIM_P_RATES)) {
            const size_t nr = (size_t)h->S * h->O * h->B;
            sim::launch_rate_grad(d, h->grad_tmp, st);
            HIPCHK(hipMemcpyAsync(grads[SIM_P_RATES], h->grad_tmp, nr * 4, kout, st));
        }
        HIPCHK(hipGetLastError());
        if (h->timing) h->resolve_timing();
        check_device_errors(h);
    });
}

int sim_get_state(sim_t *h, int32_t *status, int32_t *link, float *pos, int32_t *seq, int64_t *counters)
{
    return guarded(h, [&] {
        const size_t SR = (size_t)h->S * h->ring_total, SL = (size_t)h->S * h->L, SN = (size_t)h->S * h->N;
        std::vector<float> rp(SR);
        std::vector<int32_t> ra(SR);
        std::vector<sim::LinkSt> ls(SL);
        std::vector<uint8_t> st(SN);
        HIPCHK(hipMemcpyAsync(rp.data(), h->d.ring_pos, SR * 4, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(ra.data(), h->d.ring_agent, SR * 4, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(ls.data(), h->d.ls, SL * sizeof(sim::LinkSt), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(st.data(), h->d.status, SN, hipMemcpyDeviceToHost, h->stream));
        std::vector<int64_t> ctr((size_t)h->S * sim::kCtrSlots * sim::CTR_N);
        HIPCHK(hipMemcpyAsync(ctr.data(), h->d.ctr, ctr.size() * 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        if (status) for (size_t i = 0; i < SN; ++i) status[i] = st[i];
        if (link) std::fill(link, link + SN, -1);
        if (pos) std::fill(pos, pos + SN, 0.f);
        if (seq) std::fill(seq, seq + SN, 0);
        for (int s = 0; s < h->S; ++s)
            for (int j = 0; j < h->L; ++j) {
                const size_t seg = (size_t)s * h->L + j;
                for (int q = ls[seg].rhead; q < ls[seg].rtail; ++q) {
                    const size_t slot = (size_t)s * h->ring_total + h->ring_base[j] + (q % h->cap[j]);
                    const size_t ga = (size_t)s * h->N + ra[slot];
                    if (link) link[ga] = h->lperm[j];
                    if (pos) pos[ga] = rp[slot];
                    if (seq) seq[ga] = q;
                }
            }
        if (counters) {
            for (int s = 0; s < h->S; ++s) {
                int64_t *c = counters + (size_t)s * SIM_C_COUNT;
                int64_t g[sim::CTR_N] = {0};
                for (int q = 0; q < sim::kCtrSlots; ++q)
                    for (int k = 0; k < sim::CTR_N; ++k) g[k] += ctr[((size_t)s * sim::kCtrSlots + q) * sim::CTR_N + k];
                for (int k = 0; k < SIM_C_COUNT; ++k) c[k] = g[k];
                c[SIM_C_ON_NET] = g[sim::CTR_DEPARTED] - g[sim::CTR_EXITED];
            }
        }
    });
}

int sim_get_stats(sim_t *h, int64_t *vehicle_steps)
{
    return guarded(h, [&] {
        if (!vehicle_steps) fail(SIM_EINVAL, "null output");
        int64_t *dv = h->dalloc_scratch_i64(h->S);
        sim::launch_ttt(h->d, h->t, h->ttt_dev, dv, h->ttt_acc, h->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(vehicle_steps, dv, (size_t)h->S * 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    });
}

}  // extern "C"

namespace {

struct StateHeader {
    uint64_t magic;
    int32_t version, S, L, N, O, D, nb, t, has_dB, has_placed, pad;
    int64_t ring_total;
};
constexpr uint64_t kStateMagic = 0x31544154534d4953ull;   // "SIMSTAT1"

// (device pointer, bytes) of every array of the mutable simulation state
std::vector<std::pair<void *, size_t>> state_arrays(sim_t *h)
{
    Dev &d = h->d;
    const size_t SR = (size_t)h->S * h->ring_total, SL = (size_t)h->S * h->L, SO = (size_t)h->S * h->O;
    const size_t SN = (size_t)h->S * h->N, nc = (size_t)h->S * h->D * std::max(h->nb, 1);
    std::vector<std::pair<void *, size_t>> a = {
        {d.ring_pos, SR * 4}, {d.ring_agent, SR * 4}, {d.ring_aux, SR * 8}, {d.ls, SL * sizeof(sim::LinkSt)},
        {d.Dacc, SO * 8}, {d.rel_ptr, SO * 4}, {d.dep_ptr, SO * 4},
        {d.ctr, (size_t)h->S * sim::kCtrSlots * sim::CTR_N * 8}, {d.status, SN}, {d.tstar, SN * 8},
        {d.rel_t, SN * 4}, {d.dep_t, SN * 4}, {d.exit_t, SN * 4}, {d.cum, nc * 4}};
    if (d.dB) a.push_back({d.dB, SL * 8});
    return a;
}

size_t state_bytes(sim_t *h)
{
    size_t n = sizeof(StateHeader) + (size_t)h->N;
    for (auto &x : state_arrays(h)) n += x.second;
    return n;
}

}  // namespace

extern "C" {

int sim_get_full_state(sim_t *h, void *blob, size_t cap, size_t *n)
{
    return guarded(h, [&] {
        const size_t need = state_bytes(h);
        if (n) *n = need;
        if (!blob) return;
        if (cap < need) fail(SIM_EINVAL, "state buffer too small: need " + std::to_string(need) + " bytes");
        StateHeader hd{kStateMagic, 1, h->S, h->L, h->N, h->O, h->D, h->nb, h->t, h->d.dB ? 1 : 0,
                       h->placed.empty() ? 0 : 1, 0, h->ring_total};
        char *p = static_cast<char *>(blob);
        std::memcpy(p, &hd, sizeof hd);
        p += sizeof hd;
        for (auto &x : state_arrays(h)) {
            HIPCHK(hipMemcpyAsync(p, x.first, x.second, hipMemcpyDeviceToHost, h->stream));
            p += x.second;
        }
        if (h->placed.empty()) std::memset(p, 0, (size_t)h->N);
        else std::memcpy(p, h->placed.data(), (size_t)h->N);
        HIPCHK(hipStreamSynchronize(h->stream));
    });
}

int sim_set_full_state(sim_t *h, const void *blob, size_t n)
{
    return guarded(h, [&] {
        if (!blob || n < sizeof(StateHeader)) fail(SIM_EINVAL, "state blob too small");
        StateHeader hd;
        std::memcpy(&hd, blob, sizeof hd);
        if (hd.magic != kStateMagic || hd.version != 1) fail(SIM_EINVAL, "not a state blob of this library");
        if (hd.S != h->S || hd.L != h->L || hd.N != h->N || hd.O != h->O || hd.D != h->D || hd.nb != h->nb ||
            hd.ring_total != h->ring_total)
            fail(SIM_EINVAL, "state blob of a different network, agent pool or configuration");
        if (hd.t < 0) fail(SIM_EINVAL, "bad step counter in state blob");
        // the blob's layout: header, the arrays (dB only when its source recorded), placed mask
        size_t need = sizeof hd + (size_t)h->N;
        auto arr = state_arrays(h);
        const bool mine_dB = h->d.dB != nullptr;
        for (size_t k = 0; k < arr.size(); ++k)
            if (!(mine_dB && k + 1 == arr.size())) need += arr[k].second;
        if (hd.has_dB) need += (size_t)h->S * h->L * 8;
        if (n != need) fail(SIM_EINVAL, "state blob size does not match its header");
        const char *p = static_cast<const char *>(blob) + sizeof hd;
        const size_t base_n = mine_dB ? arr.size() - 1 : arr.size();
        for (size_t k = 0; k < base_n; ++k) {
            HIPCHK(hipMemcpyAsync(arr[k].first, p, arr[k].second, hipMemcpyHostToDevice, h->stream));
            p += arr[k].second;
        }
        const size_t SL8 = (size_t)h->S * h->L * 8;
        if (hd.has_dB) {
            if (mine_dB) HIPCHK(hipMemcpyAsync(h->d.dB, p, SL8, hipMemcpyHostToDevice, h->stream));
            p += SL8;
        } else if (mine_dB) {
            HIPCHK(hipMemsetAsync(h->d.dB, 0, SL8, h->stream));
        }
        const uint8_t *pl = reinterpret_cast<const uint8_t *>(p);
        bool any = false;
        for (int i = 0; i < h->N; ++i) any |= pl[i] != 0;
        if (any) h->placed.assign(pl, pl + h->N);
        else h->placed.clear();
        h->queues_unplaced = false;
        build_queues(h, any ? &h->placed : nullptr);
        upload_queues(h);
        h->queues_unplaced = !any;
        HIPCHK(hipMemsetAsync(h->d.tie_n, 0, 4, h->stream));   // the log restarts with the restored run
        h->t = hd.t;
        h->rec_valid = h->record && hd.t == 0;
        h->tape_win.assign(h->tapes.size(), -1);
        HIPCHK(hipStreamSynchronize(h->stream));
    });
}

int sim_get_tie_log(sim_t *h, int32_t *buf, int64_t cap, int64_t *n)
{
    return guarded(h, [&] {
        if (!n || cap < 0 || (cap > 0 && !buf)) fail(SIM_EINVAL, "bad tie-log arguments");
        int32_t total = 0;
        HIPCHK(hipMemcpyAsync(&total, h->d.tie_n, 4, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        *n = total;
        const int64_t k = std::min<int64_t>({(int64_t)total, (int64_t)sim::kTieLogMax, buf ? cap : 0});
        if (k <= 0) return;
        std::vector<int32_t> r((size_t)6 * k);
        HIPCHK(hipMemcpyAsync(r.data(), h->d.tie_log, r.size() * 4, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (int64_t q = 0; q < k; ++q) {   // links back to the caller's numbering
            int32_t *x = &r[(size_t)6 * q];
            x[4] = h->lperm[x[4]];
            if (x[2] == sim::TIE_CHOICE) x[5] = h->lperm[x[5]];
        }
        std::vector<int64_t> ord((size_t)k);
        for (int64_t q = 0; q < k; ++q) ord[(size_t)q] = q;
        std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
            return std::lexicographical_compare(&r[6 * a], &r[6 * a + 6], &r[6 * b], &r[6 * b + 6]);
        });
        for (int64_t q = 0; q < k; ++q) std::copy(&r[6 * ord[q]], &r[6 * ord[q] + 6], buf + 6 * q);
    });
}

int sim_get_link_state(sim_t *h, double *B, int64_t *E, int32_t *next_seq)
{
    return guarded(h, [&] {
        const size_t SL = (size_t)h->S * h->L;
        std::vector<sim::LinkSt> ls(SL);
        HIPCHK(hipMemcpyAsync(ls.data(), h->d.ls, SL * sizeof(sim::LinkSt), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (int s = 0; s < h->S; ++s)
            for (int jo = 0; jo < h->L; ++jo) {
                const size_t o = (size_t)s * h->L + jo, i = (size_t)s * h->L + h->linv[jo];
                // the device keeps the bucket before the end-of-step idle cap min(B, 1)
                if (B) B[o] = ls[i].B > 1.0 ? 1.0 : ls[i].B;
                if (E) E[o] = ls[i].E;
                if (next_seq) next_seq[o] = ls[i].rtail;
            }
    });
}

int sim_get_dist(sim_t *h, double *out, int32_t *n_dest)
{
    return guarded(h, [&] {
        const int nd = (int)h->dest_nodes.size();
        if (n_dest) *n_dest = nd;
        if (out) {
            // rows in increasing caller node id of the destination, columns caller node ids
            std::vector<std::pair<int, int>> rows(nd);
            for (int k = 0; k < nd; ++k) rows[k] = {h->nperm[h->dest_nodes[k]], k};
            std::sort(rows.begin(), rows.end());
            for (int r = 0; r < nd; ++r)
                for (int vo = 0; vo < h->Nn; ++vo)
                    out[(size_t)r * h->Nn + vo] = h->dist[(size_t)rows[r].second * h->Nn + h->ninv[vo]];
        }
    });
}

int sim_time(const sim_t *h, int32_t *t)
{
    if (!h || !t) return SIM_EINVAL;
    *t = h->t;
    return SIM_OK;
}

int sim_philox(sim_t *h, int32_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    return guarded(h, [&] {
        if (n < 0 || (n > 0 && (!ctr || !key || !out))) fail(SIM_EINVAL, "bad philox arrays");
        if (n == 0) return;
        uint32_t *dc = nullptr, *dk = nullptr, *dout = nullptr;
        HIPCHK(hipMalloc(&dc, (size_t)n * 16));
        HIPCHK(hipMalloc(&dk, (size_t)n * 8));
        HIPCHK(hipMalloc(&dout, (size_t)n * 16));
        HIPCHK(hipMemcpyAsync(dc, ctr, (size_t)n * 16, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(dk, key, (size_t)n * 8, hipMemcpyHostToDevice, h->stream));
        sim::launch_philox(n, dc, dk, dout, h->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(out, dout, (size_t)n * 16, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        (void)hipFree(dc); (void)hipFree(dk); (void)hipFree(dout);
    });
}

int sim_gumbel_fast(sim_t *h, int32_t n, const uint32_t *words, float *out)
{
    return guarded(h, [&] {
        if (n < 0 || (n > 0 && (!words || !out))) fail(SIM_EINVAL, "bad gumbel arrays");
        if (n == 0) return;
        uint32_t *dw = nullptr;
        float *dout = nullptr;
        HIPCHK(hipMalloc(&dw, (size_t)n * 4));
        HIPCHK(hipMalloc(&dout, (size_t)n * 4));
        HIPCHK(hipMemcpyAsync(dw, words, (size_t)n * 4, hipMemcpyHostToDevice, h->stream));
        sim::launch_gumbel_fast(n, dw, dout, h->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(out, dout, (size_t)n * 4, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        (void)hipFree(dw); (void)hipFree(dout);
    });
}

int sim_segsort(sim_t *h, int32_t n, int32_t n_segments, const int32_t *seg, const float *pos, const int32_t *seq,
                int32_t *perm, int32_t *seg_off)
{
    return guarded(h, [&] {
        if (n < 0 || n_segments < 1) fail(SIM_EINVAL, "bad sizes");
        if (n > 0 && (!seg || !pos || !seq || !perm || !seg_off)) fail(SIM_EINVAL, "null array");
        int32_t *scratch = nullptr;
        HIPCHK(hipMalloc(&scratch, ((size_t)n_segments + 1) * 4 * 2 + 64));
        const int rc = sim::launch_segsort(n, n_segments, seg, pos, seq, perm, seg_off, scratch, h->stream);
        HIPCHK(hipStreamSynchronize(h->stream));
        (void)hipFree(scratch);
        if (rc != 0) fail(SIM_EUNSUPPORTED, "a segment exceeds the LDS sort capacity");
    });
}

int sim_segsort_noalloc(sim_t *h, int32_t n, int32_t n_segments, const int32_t *seg, const float *pos,
                        const int32_t *seq, int32_t *perm, int32_t *seg_off, int32_t *status)
{
    return guarded(h, [&] {
        if (n < 0 || n_segments < 1) fail(SIM_EINVAL, "bad sizes");
        if (n_segments > SIM_SEGSORT_NOALLOC_MAX_SEGMENTS)
            fail(SIM_EINVAL, "n_segments above SIM_SEGSORT_NOALLOC_MAX_SEGMENTS");
        if (n > 0 && (!seg || !pos || !seq || !perm || !seg_off)) fail(SIM_EINVAL, "null array");
        const int rc = sim::launch_segsort_noalloc(h->device, n, n_segments, seg, pos, seq, perm, seg_off, status,
                                                   h->stream);
        if (rc < 0) fail(SIM_EDEVICE, "sort launch failed, or no scratch array address for this device");
        if (rc > 0) fail(SIM_EUNSUPPORTED, "a segment exceeds the LDS sort capacity");
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// autotuner: lane-group sizes of the link, node and reverse kernels, timed on
// the live state and cached per shape bucket
// ---------------------------------------------------------------------------
namespace {

std::mutex g_tune_mu;
std::map<std::string, std::array<int, 3>> g_tune_mem;

int node_group_need(const sim_t *h)
{
    int need = 1;
    for (int v = 0; v < h->Nn; ++v) need = std::max(need, (h->node_cnt[v] >> 24) + ((h->node_cnt[v] >> 16) & 0xff));
    return std::max(need, h->max_out);
}

std::string shape_key(const sim_t *h)
{
    hipDeviceProp_t p;
    HIPCHK(hipGetDeviceProperties(&p, h->device));
    auto lg = [](double x) { return (int)std::lround(std::log2(std::max(1.0, x))); };
    std::string arch = p.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    return arch + "/S" + std::to_string(h->S) + "/L" + std::to_string(lg(h->L)) + "/N" + std::to_string(lg(h->N)) +
           "/R" + std::to_string(lg((double)h->ring_total / std::max(1, h->L))) + "/in" +
           std::to_string(node_group_need(h)) + "/rec" + std::to_string(h->record ? 1 : 0);
}

bool cache_lookup(const std::string &path, const std::string &key, std::array<int, 3> &out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    bool hit = false;
    auto it = g_tune_mem.find(key);
    if (it != g_tune_mem.end()) { out = it->second; hit = true; }
    if (!path.empty()) {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line)) {   // "key g_link g_node g_rev"; the last entry of a key wins
            const size_t sp = line.find(' ');
            if (sp == std::string::npos || line.compare(0, sp, key) != 0 || sp != key.size()) continue;
            int a = 0, b = 0, c = 0;
            if (std::sscanf(line.c_str() + sp, "%d %d %d", &a, &b, &c) == 3) { out = {a, b, c}; hit = true; }
        }
    }
    return hit;
}

void cache_store(const std::string &path, const std::string &key, const std::array<int, 3> &v, double ms)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_mem[key] = v;
    if (path.empty()) return;
    std::ofstream f(path, std::ios::app);
    if (f) f << key << ' ' << v[0] << ' ' << v[1] << ' ' << v[2] << ' ' << ms << '\n';
}

void tune_snapshot(sim_t *h, bool save)
{
    Dev &d = h->d;
    const size_t SN = (size_t)h->S * h->N, nc = (size_t)h->S * h->D * std::max(h->nb, 1);
    if (!h->tune_alloc) {
        ckpt_alloc(h, h->tune_ck);
        h->tune_tstar = h->dalloc<double>(SN);
        h->tune_rel = h->dalloc<int32_t>(SN);
        h->tune_dep = h->dalloc<int32_t>(SN);
        h->tune_exit = h->dalloc<int32_t>(SN);
        h->tune_cum = h->dalloc<int32_t>(nc);
        h->tune_tie_n = h->dalloc<int32_t>(1);
        h->tune_alloc = true;
    }
    ckpt_copy(h, h->tune_ck, save);
    auto cp = [&](void *snap, void *live, size_t bytes) {
        if (save) HIPCHK(hipMemcpyAsync(snap, live, bytes, hipMemcpyDeviceToDevice, h->stream));
        else HIPCHK(hipMemcpyAsync(live, snap, bytes, hipMemcpyDeviceToDevice, h->stream));
    };
    cp(h->tune_tstar, d.tstar, SN * 8);
    cp(h->tune_rel, d.rel_t, SN * 4);
    cp(h->tune_dep, d.dep_t, SN * 4);
    cp(h->tune_exit, d.exit_t, SN * 4);
    cp(h->tune_cum, d.cum, nc * 4);
    cp(h->tune_tie_n, d.tie_n, 4);   // probe steps append no near-tie records
}

void set_groups(sim_t *h, int gl, int gn, int gr)
{
    h->g_link = h->d.g_link = gl;
    h->g_node = h->d.g_node = gn;
    h->g_rev = h->d.g_rev = gr;
    build_classes(h);
}

}  // namespace

extern "C" {

int sim_autotune(sim_t *h, int32_t probe_steps, const char *cache_path, int32_t flags, int32_t *g_link,
                 int32_t *g_node, int32_t *g_rev)
{
    return guarded(h, [&] {
        if (probe_steps < 1) fail(SIM_EINVAL, "probe_steps must be >= 1");
        h->tape_win.assign(h->tapes.size(), -1);   // probes record into the tape sets
        const std::string key = shape_key(h), path = cache_path ? cache_path : "";
        std::array<int, 3> best = {h->g_link, h->g_node, h->g_rev};
        auto valid = [&](const std::array<int, 3> &v) {
            auto ok = [](int g) { return g == 16 || g == 32 || g == 64; };
            return (ok(v[0]) || v[0] == 8) && (ok(v[1]) || v[1] == 8) && (ok(v[2]) || v[2] == 8);
        };
        std::array<int, 3> cached;
        if (!(flags & 1) && cache_lookup(path, key, cached) && valid(cached)) {
            set_groups(h, cached[0], cached[1], cached[2]);
            best = cached;
        } else {
            const hipStream_t st = h->stream;
            const int t0 = h->t;
            hipEvent_t ea, eb;
            HIPCHK(hipEventCreate(&ea));
            HIPCHK(hipEventCreate(&eb));
            const bool timing = h->timing;
            h->timing = false;
            tune_snapshot(h, true);
            auto elapsed = [&]() {
                HIPCHK(hipEventSynchronize(eb));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, ea, eb));
                return (double)ms;
            };
            // forward: steps from the snapshot (one untimed warm-up step per candidate)
            auto time_forward = [&](const std::array<int, 3> &v) {
                set_groups(h, v[0], v[1], v[2]);
                tune_snapshot(h, false);
                h->t = t0;
                do_step(h, -1);
                HIPCHK(hipEventRecord(ea, st));
                for (int k = 0; k < probe_steps; ++k) do_step(h, -1);
                HIPCHK(hipEventRecord(eb, st));
                return elapsed();
            };
            double best_ms = 0.0;
            for (int dim = 0; dim < 2; ++dim) {
                double bms = 1e300;
                std::array<int, 3> bv = best;
                for (int g : {8, 16, 32, 64}) {
                    std::array<int, 3> v = best;
                    v[dim] = g;
                    if (!valid(v)) continue;
                    const double ms = time_forward(v);
                    if (ms < bms) { bms = ms; bv = v; }
                }
                best = bv;
                best_ms = bms;
            }
            // reverse: record a window from the snapshot, then time the reverse sweep over it
            if (h->record) {
                set_groups(h, best[0], best[1], best[2]);
                tune_snapshot(h, false);
                h->t = t0;
                const int Ww = std::min(probe_steps, h->W);
                Dev d = h->d;
                d.gQ = nullptr; d.gT = nullptr; d.gx = nullptr; d.gm = nullptr;
                for (int k = 0; k < Ww; ++k) do_step(h, k);
                sim::launch_tape_snapshot(d, Ww, st);
                double bms = 1e300;
                int bg = best[2];
                for (int g : {8, 16, 32, 64}) {
                    h->g_rev = h->d.g_rev = g;
                    build_classes(h);
                    d.g_rev = g;
                    for (int rep = 0; rep < 2; ++rep) {   // first sweep warms up
                        HIPCHK(hipMemsetAsync(d.adj_ring, 0, (size_t)h->S * h->ring_total * 4, st));
                        HIPCHK(hipEventRecord(ea, st));
                        for (int k = Ww - 1; k >= 0; --k) sim::launch_reverse(d, t0 + k, k, 0, st);
                        HIPCHK(hipEventRecord(eb, st));
                        const double ms = elapsed();
                        if (rep == 1 && ms < bms) { bms = ms; bg = g; }
                    }
                }
                best[2] = bg;
                HIPCHK(hipMemsetAsync(d.gu, 0, (size_t)h->S * h->L * 8, st));
                HIPCHK(hipMemsetAsync(d.gk, 0, (size_t)h->S * h->L * 8, st));
                HIPCHK(hipMemsetAsync(d.depg, 0, (size_t)h->S * h->N * 4, st));
            }
            set_groups(h, best[0], best[1], best[2]);
            tune_snapshot(h, false);
            h->t = t0;
            HIPCHK(hipStreamSynchronize(st));
            HIPCHK(hipEventDestroy(ea));
            HIPCHK(hipEventDestroy(eb));
            h->timing = timing;
            cache_store(path, key, best, best_ms);
        }
        if (g_link) *g_link = best[0];
        if (g_node) *g_node = best[1];
        if (g_rev) *g_rev = best[2];
    });
}

int sim_set_schedule(sim_t *h, int g_link, int g_node, int g_rev)
{
    return guarded(h, [&] {
        auto ok = [](int g) { return g == 16 || g == 32 || g == 64; };
        if (!(ok(g_link) || g_link == 8) || !(ok(g_node) || g_node == 8) || !(ok(g_rev) || g_rev == 8))
            fail(SIM_EINVAL, "lanes per item must be 8, 16, 32 or 64");
        h->g_link = h->d.g_link = g_link;
        h->g_node = h->d.g_node = g_node;
        h->g_rev = h->d.g_rev = g_rev;
        build_classes(h);
    });
}

int sim_get_schedule(sim_t *h, int *g_link, int *g_node, int *g_rev)
{
    return guarded(h, [&] {
        if (g_link) *g_link = h->g_link;
        if (g_node) *g_node = h->g_node;
        if (g_rev) *g_rev = h->g_rev;
    });
}

int sim_set_timing(sim_t *h, int enable)
{
    return guarded(h, [&] { h->timing = enable != 0; });
}

int sim_get_timing(sim_t *h, double *ms, int64_t *launches, int n_kinds, int reset)
{
    return guarded(h, [&] {
        h->resolve_timing();
        for (int k = 0; k < n_kinds && k < kTimingKinds; ++k) {
            if (ms) ms[k] = h->ms_acc[k];
            if (launches) launches[k] = h->n_acc[k];
        }
        if (reset) for (int k = 0; k < kTimingKinds; ++k) { h->ms_acc[k] = 0; h->n_acc[k] = 0; }
    });
}

}  // extern "C"
