// Continuous-batching server of forward rollout requests (srv_* in sim.h).
//
// A request carries its own network, agent pool and configuration.  Worker
// threads prepare queued requests on the host (validation, renumbering,
// shortest-time tables, device footprint); the loop thread admits prepared
// requests in arrival order (later ones may go ahead when an earlier one does
// not fit) whenever a slot is free and the footprint fits the memory budget,
// gives each admitted request its own device state and HIP stream, and
// advances all running requests chunk by chunk, so their kernels overlap on
// the device.  A finished request's observables are copied to pinned host
// memory and its slot and memory range are reused.  Results do not depend on
// what else runs: every request owns its state.
//
// Nothing on the serving path allocates or frees device memory: the server
// takes one device pool of the whole budget at creation and carves each
// admitted request's state from a contiguous range of it (first fit,
// neighbouring free ranges merged on release), and every slot owns its
// stream, event and pinned result buffers.  hipFree would wait for the whole
// device, i.e. for every other request's work in flight.  Device state is
// uploaded by the worker threads outside the server lock, so admission,
// submission and polling never wait for a copy.
//
// hip_device = -1 selects a host-only executor (no GPU): requests are
// prepared, admitted and retired exactly as above, but a chunk "runs" for a
// fixed host time and produces zero observables.  It exists to test the
// admission and failure logic without a device.
#include "sim.h"
#include "sim_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

using clk = std::chrono::steady_clock;

struct Request {
    int64_t id = 0;
    std::vector<int32_t> tail, head, lanes, origin_node, det_link, agent_origin, agent_dest;
    std::vector<float> length, free_speed, jam_density, capacity, beta, alpha, cost, det_pos, ready, rates;
    std::vector<uint64_t> seeds;
    sim_network net{};
    sim_demand dem{};
    sim_config cfg{};
    int32_t T = 0;
    int state = SRV_QUEUED;
    int code = SIM_OK;
    std::string err;
    clk::time_point arrival, done_time;
    sim_t *h = nullptr;
    bool prepared = false, preparing = false, cancel = false, finishing = false, attaching = false;
    size_t footprint = 0;
    size_t range_off = 0, range_len = 0;   // the request's part of the device pool
    int slot = -1;
    int steps_done = 0;
    hipEvent_t ev = nullptr;               // the slot's event, stream and pinned buffers
    clk::time_point fake_ready;
    float *counts = nullptr;
    double *ttt = nullptr;
    int64_t *vsteps = nullptr;
    std::vector<float> counts_out;
    std::vector<double> ttt_out;
    std::vector<int64_t> vs_out;
    double latency = 0.0;
};

template <class T>
std::vector<T> copy_arr(const T *p, size_t n)
{
    return p ? std::vector<T>(p, p + n) : std::vector<T>();
}

template <class T>
const T *ptr_or_null(const std::vector<T> &v)
{
    return v.empty() ? nullptr : v.data();
}

bool terminal(int st) { return st == SRV_DONE || st == SRV_FAILED || st == SRV_CANCELLED; }

}  // namespace

struct srv_t {
    int device = -1;
    size_t budget = 0;
    int max_slots = 1, chunk = 60;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::map<int64_t, std::shared_ptr<Request>> reqs;
    std::deque<std::shared_ptr<Request>> queue;
    std::vector<std::shared_ptr<Request>> running;
    std::vector<hipStream_t> streams;
    std::vector<char> slot_used;
    // per slot: completion event and pinned result buffers (grown when a larger request arrives)
    std::vector<hipEvent_t> slot_ev;
    std::vector<float *> slot_counts;
    std::vector<double *> slot_ttt;
    std::vector<int64_t *> slot_vsteps;
    std::vector<size_t> slot_nc, slot_ns;
    // device pool of `budget` bytes and its free ranges (offset -> length); with no device the same
    // bookkeeping runs on offsets alone
    void *pool = nullptr;
    std::map<size_t, size_t> free_ranges;
    std::deque<std::shared_ptr<Request>> attach_q;   // admitted, waiting for a worker to upload them
    std::vector<sim_t *> graveyard;                  // handles of retired requests, freed outside the lock
    int attaching = 0;
    size_t used = 0;
    int64_t next_id = 1;
    bool stop = false;
    std::thread loop;
    std::vector<std::thread> preps;
    std::vector<double> latencies;
    int64_t vsteps_done = 0, completed = 0, max_running = 0;
    clk::time_point first_arrival, last_done;
    bool any_arrival = false;
    std::string create_error;

    // first fit of `need` bytes (multiple of 256) in the pool; false when no free range holds it
    bool range_alloc(size_t need, size_t *off)
    {
        for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
            if (it->second < need) continue;
            *off = it->first;
            const size_t rest = it->second - need, at = it->first + need;
            free_ranges.erase(it);
            if (rest) free_ranges[at] = rest;
            return true;
        }
        return false;
    }
    void range_free(size_t off, size_t len)
    {
        auto it = free_ranges.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free_ranges.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_ranges.erase(nx);
        }
        if (it != free_ranges.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_ranges.erase(it);
            }
        }
    }

    // called with mu held; the request's stream has no work left
    void retire(const std::shared_ptr<Request> &r, int state)
    {
        if (r->h) { graveyard.push_back(r->h); r->h = nullptr; }
        if (r->slot >= 0) {
            slot_used[r->slot] = 0;
            range_free(r->range_off, r->range_len);
            used -= r->range_len;
            r->slot = -1;
        }
        r->ev = nullptr;
        r->counts = nullptr;
        r->ttt = nullptr;
        r->vsteps = nullptr;
        r->state = state;
        r->done_time = clk::now();
        done_cv.notify_all();
    }

    // host state of retired requests, freed with mu released
    void bury(std::unique_lock<std::mutex> &lk)
    {
        if (graveyard.empty()) return;
        std::vector<sim_t *> g;
        g.swap(graveyard);
        lk.unlock();
        for (sim_t *h : g) sim::release_handle(h);
        lk.lock();
    }

    bool chunk_done(const std::shared_ptr<Request> &r)
    {
        if (device < 0) return clk::now() >= r->fake_ready;
        return hipEventQuery(r->ev) == hipSuccess;
    }

    // enqueue the next chunk (or the result copies) of a running request
    int advance(const std::shared_ptr<Request> &r)
    {
        const int n = std::min(chunk, r->T - r->steps_done);
        if (n > 0) {
            if (device >= 0) {
                const int rc = sim::rollout_enqueue(r->h, n, &r->err);
                if (rc != SIM_OK) return rc;
            }
            r->steps_done += n;
        } else {
            if (device >= 0) {
                const int rc = sim::results_enqueue(r->h, r->counts, r->ttt, r->vsteps, &r->err);
                if (rc != SIM_OK) return rc;
            }
            r->finishing = true;
        }
        if (device >= 0) {
            if (hipEventRecord(r->ev, streams[r->slot]) != hipSuccess) { r->err = "event record failed"; return SIM_EDEVICE; }
        } else {
            r->fake_ready = clk::now() + std::chrono::microseconds(200);
        }
        return SIM_OK;
    }

    void run()
    {
        if (device >= 0) (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (!stop) {
            bool progress = false;
            // ---- admission: arrival order, later requests may pass one that does not fit ----
            for (auto it = queue.begin(); it != queue.end();) {
                auto r = *it;
                if (r->cancel) { retire(r, SRV_CANCELLED); it = queue.erase(it); progress = true; continue; }
                if (r->state == SRV_FAILED) { it = queue.erase(it); progress = true; continue; }
                if (!r->prepared) { ++it; continue; }
                if ((int)running.size() + attaching >= max_slots) { ++it; continue; }
                const size_t need = (r->footprint + 255) & ~(size_t)255;
                size_t off = 0;
                if (!range_alloc(need, &off)) { ++it; continue; }
                int slot = 0;
                while (slot_used[slot]) ++slot;
                slot_used[slot] = 1;
                r->slot = slot;
                r->range_off = off;
                r->range_len = need;
                used += need;
                it = queue.erase(it);
                progress = true;
                int rc = SIM_OK;
                if (device >= 0) {
                    // the slot's pinned result buffers, grown if this request needs more
                    const size_t nc = (size_t)std::max(1, sim::counts_size(r->h));
                    const size_t ns = (size_t)std::max(1, sim::scenarios_of(r->h));
                    if (nc > slot_nc[slot]) {
                        if (slot_counts[slot]) (void)hipHostFree(slot_counts[slot]);
                        slot_counts[slot] = nullptr;
                        slot_nc[slot] = 0;
                        if (hipHostMalloc((void **)&slot_counts[slot], nc * 4) == hipSuccess) slot_nc[slot] = nc;
                    }
                    if (ns > slot_ns[slot]) {
                        if (slot_ttt[slot]) (void)hipHostFree(slot_ttt[slot]);
                        if (slot_vsteps[slot]) (void)hipHostFree(slot_vsteps[slot]);
                        slot_ttt[slot] = nullptr;
                        slot_vsteps[slot] = nullptr;
                        slot_ns[slot] = 0;
                        if (hipHostMalloc((void **)&slot_ttt[slot], ns * 8) == hipSuccess &&
                            hipHostMalloc((void **)&slot_vsteps[slot], ns * 8) == hipSuccess)
                            slot_ns[slot] = ns;
                    }
                    if (slot_nc[slot] < nc || slot_ns[slot] < ns) {
                        rc = SIM_ENOMEM;
                        r->err = "could not allocate the slot's pinned result buffers";
                    }
                    r->ev = slot_ev[slot];
                    r->counts = slot_counts[slot];
                    r->ttt = slot_ttt[slot];
                    r->vsteps = slot_vsteps[slot];
                }
                if (rc != SIM_OK) { r->code = rc; retire(r, SRV_FAILED); continue; }
                // device state is uploaded by a worker thread, outside the lock
                r->attaching = true;
                ++attaching;
                attach_q.push_back(r);
            }
            max_running = std::max<int64_t>(max_running, (int64_t)running.size());
            // ---- progress of running requests ----
            for (size_t k = 0; k < running.size();) {
                auto r = running[k];
                bool remove = false;
                if (r->cancel) {
                    if (device >= 0) (void)hipStreamSynchronize(streams[r->slot]);
                    retire(r, SRV_CANCELLED);
                    remove = true;
                } else if (chunk_done(r)) {
                    progress = true;
                    if (r->finishing) {
                        int rc = SIM_OK;
                        if (device >= 0) rc = sim::device_errors(r->h, &r->err);
                        if (rc == SIM_OK) {
                            const int nc = sim::counts_size(r->h), ns = sim::scenarios_of(r->h);
                            if (device >= 0) {
                                r->counts_out.assign(r->counts, r->counts + nc);
                                r->ttt_out.assign(r->ttt, r->ttt + ns);
                                r->vs_out.assign(r->vsteps, r->vsteps + ns);
                            } else {
                                r->counts_out.assign(nc, 0.0f);
                                r->ttt_out.assign(ns, 0.0);
                                r->vs_out.assign(ns, 0);
                            }
                            r->latency = std::chrono::duration<double>(clk::now() - r->arrival).count();
                            latencies.push_back(r->latency);
                            for (int64_t v : r->vs_out) vsteps_done += v;
                            ++completed;
                            last_done = clk::now();
                            retire(r, SRV_DONE);
                        } else {
                            r->code = rc;
                            retire(r, SRV_FAILED);
                        }
                        remove = true;
                    } else {
                        const int rc = advance(r);
                        if (rc != SIM_OK) { r->code = rc; retire(r, SRV_FAILED); remove = true; }
                    }
                }
                if (remove) running.erase(running.begin() + k);
                else ++k;
            }
            bury(lk);
            if (progress) cv.notify_all();
            else cv.wait_for(lk, std::chrono::microseconds(100));
        }
    }

    // worker side of an admission: device state and the first chunk, then the running set
    void attach(std::unique_lock<std::mutex> &lk, const std::shared_ptr<Request> &r)
    {
        lk.unlock();
        int rc = SIM_OK;
        std::string err;
        if (device >= 0) {
            (void)hipSetDevice(device);
            rc = sim::device_attach(r->h, streams[r->slot], static_cast<char *>(pool) + r->range_off, r->range_len,
                                    &err);
        }
        if (rc == SIM_OK) rc = advance(r);
        const bool cancelled_meanwhile = r->cancel;
        if (cancelled_meanwhile && device >= 0) (void)hipStreamSynchronize(streams[r->slot]);
        lk.lock();
        r->attaching = false;
        --attaching;
        if (rc != SIM_OK) {
            r->code = rc;
            if (r->err.empty()) r->err = err;
            retire(r, SRV_FAILED);
        } else if (r->cancel) {
            if (!cancelled_meanwhile && device >= 0) {
                lk.unlock();
                (void)hipStreamSynchronize(streams[r->slot]);
                lk.lock();
            }
            retire(r, SRV_CANCELLED);
        } else {
            r->state = SRV_RUNNING;
            running.push_back(r);
        }
        cv.notify_all();
    }

    void prepare_worker()
    {
        std::unique_lock<std::mutex> lk(mu);
        while (!stop) {
            if (!attach_q.empty()) {
                auto a = attach_q.front();
                attach_q.pop_front();
                attach(lk, a);
                continue;
            }
            std::shared_ptr<Request> r;
            for (auto &q : queue)
                if (!q->prepared && !q->preparing && !q->cancel && q->state == SRV_QUEUED) { r = q; break; }
            if (!r) { cv.wait_for(lk, std::chrono::milliseconds(1)); continue; }
            r->preparing = true;
            lk.unlock();
            int code = SIM_OK;
            std::string err;
            sim_t *h = sim::host_prepare(&r->net, &r->dem, &r->cfg, device, &code, &err);
            lk.lock();
            r->preparing = false;
            if (r->cancel || terminal(r->state) || stop) {
                // cancelled (or shutting down) while being prepared
                if (h) sim::destroy_handle(h);
                if (!terminal(r->state)) retire(r, SRV_CANCELLED);
            } else if (!h) {
                r->code = code;
                r->err = err;
                retire(r, SRV_FAILED);
            } else {
                r->h = h;
                r->footprint = sim::footprint_of(h);
                r->prepared = true;
                if (((r->footprint + 255) & ~(size_t)255) > (budget & ~(size_t)255)) {
                    r->code = SIM_ENOMEM;
                    r->err = "request footprint " + std::to_string(r->footprint) + " B exceeds the server budget";
                    retire(r, SRV_FAILED);
                }
            }
            cv.notify_all();
        }
    }
};

extern "C" {

int srv_create(int hip_device, size_t mem_budget_bytes, int32_t max_slots, int32_t chunk_steps, srv_t **out)
{
    if (!out || max_slots < 1 || chunk_steps < 1 || mem_budget_bytes == 0) return SIM_EINVAL;
    *out = nullptr;
    srv_t *s = new (std::nothrow) srv_t();
    if (!s) return SIM_ENOMEM;
    s->device = hip_device;
    s->budget = mem_budget_bytes;
    s->max_slots = max_slots;
    s->chunk = chunk_steps;
    s->slot_used.assign(max_slots, 0);
    if (hip_device >= 0) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device >= ndev || hipSetDevice(hip_device) != hipSuccess) {
            delete s;
            return SIM_EDEVICE;
        }
        s->streams.resize(max_slots, nullptr);
        s->slot_ev.resize(max_slots, nullptr);
        bool ok = true;
        for (int k = 0; k < max_slots && ok; ++k)
            ok = hipStreamCreateWithFlags(&s->streams[k], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&s->slot_ev[k], hipEventDisableTiming) == hipSuccess;
        int code = SIM_EDEVICE;
        if (ok && hipMalloc(&s->pool, mem_budget_bytes) != hipSuccess) {
            (void)hipGetLastError();
            s->pool = nullptr;
            ok = false;
            code = SIM_ENOMEM;
        }
        if (!ok) {
            for (auto x : s->streams) if (x) (void)hipStreamDestroy(x);
            for (auto e : s->slot_ev) if (e) (void)hipEventDestroy(e);
            delete s;
            return code;
        }
    }
    s->slot_counts.assign(max_slots, nullptr);
    s->slot_ttt.assign(max_slots, nullptr);
    s->slot_vsteps.assign(max_slots, nullptr);
    s->slot_nc.assign(max_slots, 0);
    s->slot_ns.assign(max_slots, 0);
    s->free_ranges[0] = mem_budget_bytes & ~(size_t)255;
    s->loop = std::thread([s] { s->run(); });
    const unsigned np = std::max(1u, std::min(4u, std::thread::hardware_concurrency()));
    for (unsigned k = 0; k < np; ++k) s->preps.emplace_back([s] { s->prepare_worker(); });
    *out = s;
    return SIM_OK;
}

int srv_submit(srv_t *s, const sim_network *net, const sim_demand *dem, const sim_config *cfg, int32_t T,
               int64_t *ticket)
{
    if (!s || !net || !dem || !cfg || !ticket || T < 0) return SIM_EINVAL;
    auto r = std::make_shared<Request>();
    try {
        const size_t L = net->n_links > 0 ? net->n_links : 0, O = net->n_origins > 0 ? net->n_origins : 0;
        const size_t D = net->n_detectors > 0 ? net->n_detectors : 0, N = dem->n_agents > 0 ? dem->n_agents : 0;
        r->tail = copy_arr(net->tail, L); r->head = copy_arr(net->head, L); r->lanes = copy_arr(net->lanes, L);
        r->length = copy_arr(net->length, L); r->free_speed = copy_arr(net->free_speed, L);
        r->jam_density = copy_arr(net->jam_density, L); r->capacity = copy_arr(net->capacity, L);
        r->beta = copy_arr(net->beta, L); r->alpha = copy_arr(net->alpha, L); r->cost = copy_arr(net->cost, L);
        r->origin_node = copy_arr(net->origin_node, O);
        r->det_link = copy_arr(net->detector_link, D); r->det_pos = copy_arr(net->detector_pos, D);
        r->agent_origin = copy_arr(dem->agent_origin, N); r->agent_dest = copy_arr(dem->agent_dest, N);
        r->ready = copy_arr(dem->ready_time, N);
        const size_t nr = dem->n_rate_bins > 0 ? O * (size_t)dem->n_rate_bins : 0;
        r->rates = copy_arr(dem->rates, nr);
        const int S = cfg->n_scenarios > 0 ? cfg->n_scenarios : 0;
        r->seeds = copy_arr(cfg->scenario_seed, (size_t)S);
    } catch (const std::bad_alloc &) {
        return SIM_ENOMEM;
    }
    r->net = *net;
    r->net.tail = ptr_or_null(r->tail); r->net.head = ptr_or_null(r->head); r->net.lanes = ptr_or_null(r->lanes);
    r->net.length = ptr_or_null(r->length); r->net.free_speed = ptr_or_null(r->free_speed);
    r->net.jam_density = ptr_or_null(r->jam_density); r->net.capacity = ptr_or_null(r->capacity);
    r->net.beta = ptr_or_null(r->beta); r->net.alpha = ptr_or_null(r->alpha); r->net.cost = ptr_or_null(r->cost);
    r->net.origin_node = ptr_or_null(r->origin_node);
    r->net.detector_link = ptr_or_null(r->det_link); r->net.detector_pos = ptr_or_null(r->det_pos);
    r->dem = *dem;
    r->dem.agent_origin = ptr_or_null(r->agent_origin); r->dem.agent_dest = ptr_or_null(r->agent_dest);
    r->dem.ready_time = ptr_or_null(r->ready); r->dem.rates = ptr_or_null(r->rates);
    r->cfg = *cfg;
    r->cfg.scenario_seed = ptr_or_null(r->seeds);
    r->cfg.record_for_backward = 0;
    r->cfg.mem_budget_bytes = 0;
    r->T = T;
    r->arrival = clk::now();
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    if (!s->any_arrival) { s->first_arrival = r->arrival; s->any_arrival = true; }
    s->reqs[r->id] = r;
    s->queue.push_back(r);
    *ticket = r->id;
    s->cv.notify_all();
    return SIM_OK;
}

int srv_poll(srv_t *s, int64_t ticket, int *state)
{
    if (!s || !state) return SIM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return SIM_EINVAL;
    *state = it->second->state;
    return SIM_OK;
}

int srv_wait(srv_t *s, int64_t ticket, double timeout_s, int *state)
{
    if (!s || !state) return SIM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return SIM_EINVAL;
    auto r = it->second;
    s->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return terminal(r->state); });
    *state = r->state;
    return SIM_OK;
}

int srv_result(srv_t *s, int64_t ticket, float *counts, double *ttt, int64_t *vehicle_steps, double *latency_s)
{
    if (!s) return SIM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return SIM_EINVAL;
    auto &r = it->second;
    if (r->state == SRV_FAILED) return r->code != SIM_OK ? r->code : SIM_EDEVICE;
    if (r->state != SRV_DONE) return SIM_ESTATE;
    if (counts) std::copy(r->counts_out.begin(), r->counts_out.end(), counts);
    if (ttt) std::copy(r->ttt_out.begin(), r->ttt_out.end(), ttt);
    if (vehicle_steps) std::copy(r->vs_out.begin(), r->vs_out.end(), vehicle_steps);
    if (latency_s) *latency_s = r->latency;
    return SIM_OK;
}

const char *srv_error(srv_t *s, int64_t ticket)
{
    if (!s) return "null server";
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return "unknown ticket";
    return it->second->err.c_str();
}

int srv_cancel(srv_t *s, int64_t ticket)
{
    if (!s) return SIM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return SIM_EINVAL;
    if (!terminal(it->second->state)) it->second->cancel = true;
    s->cv.notify_all();
    return SIM_OK;
}

int srv_stats(srv_t *s, double *p50_s, double *p99_s, double *vehicle_steps_per_s, int64_t *completed,
              int64_t *max_running)
{
    if (!s) return SIM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> l = s->latencies;
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {
        if (l.empty()) return 0.0;
        const size_t k = (size_t)std::min<double>((double)l.size() - 1, std::ceil(p * (double)l.size()) - 1);
        return l[k];
    };
    if (p50_s) *p50_s = pct(0.50);
    if (p99_s) *p99_s = pct(0.99);
    if (vehicle_steps_per_s) {
        const double w = s->completed ? std::chrono::duration<double>(s->last_done - s->first_arrival).count() : 0.0;
        *vehicle_steps_per_s = w > 0 ? (double)s->vsteps_done / w : 0.0;
    }
    if (completed) *completed = s->completed;
    if (max_running) *max_running = s->max_running;
    return SIM_OK;
}

int srv_destroy(srv_t *s)
{
    if (!s) return SIM_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->loop.joinable()) s->loop.join();
    for (auto &t : s->preps) if (t.joinable()) t.join();
    if (s->device >= 0) {
        (void)hipSetDevice(s->device);
        for (auto st : s->streams) (void)hipStreamSynchronize(st);
    }
    for (auto &kv : s->reqs) {
        auto &r = kv.second;
        if (r->h) { sim::release_handle(r->h); r->h = nullptr; }
    }
    for (sim_t *h : s->graveyard) sim::release_handle(h);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    for (auto e : s->slot_ev) (void)hipEventDestroy(e);
    for (auto p : s->slot_counts) if (p) (void)hipHostFree(p);
    for (auto p : s->slot_ttt) if (p) (void)hipHostFree(p);
    for (auto p : s->slot_vsteps) if (p) (void)hipHostFree(p);
    if (s->pool) (void)hipFree(s->pool);
    delete s;
    return SIM_OK;
}

}  // extern "C"
