// Gradient-based calibration and control loop (sim_optimize in sim.h).
//
// The paper's optimisation (Methods, "Optimization") repeats forward
// simulation, loss, gradient and parameter update until the loss has not
// improved for 20 iterations, with AdamW (learning rate 0.1, weight decay
// 1e-5), and keeps the parameters of the lowest loss.  Here every iteration
// is: sim_reset, sim_rollout, counts into a device buffer, the loss kernel
// (value and cotangent on the device), sim_backward into device gradient
// buffers, one AdamW kernel per optimised group, and sim_set_params from the
// updated device values.  The only host traffic is one double per iteration
// (the loss, for the stopping rule) and the parameter validation of
// sim_set_params.
#include "sim.h"
#include "sim_internal.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

namespace {

struct DevBuf {
    void *p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p) { o.p = nullptr; }
    ~DevBuf() { if (p) (void)hipFree(p); }
    template <class T>
    T *get() { return static_cast<T *>(p); }
};

int alloc(DevBuf &b, size_t bytes)
{
    if (hipMalloc(&b.p, bytes ? bytes : 1) != hipSuccess) { (void)hipGetLastError(); b.p = nullptr; return SIM_ENOMEM; }
    return SIM_OK;
}

struct Group {
    int which = 0;
    int64_t n = 0;
    double lo = 0, hi = 0, x0 = 0, sc = 1;
    DevBuf p, g, m, v, best, hi_vec;
};

void default_box(int which, double *lo, double *hi)
{
    const double inf = std::numeric_limits<double>::infinity();
    switch (which) {
    case SIM_P_U: *lo = 0.5; *hi = 60.0; break;
    case SIM_P_KAPPA: *lo = 1e-3; *hi = inf; break;
    case SIM_P_COST: *lo = 0.01; *hi = 1e4; break;
    case SIM_P_RATES: case SIM_P_CAP_MULT: *lo = 0.0; *hi = 1e4; break;
    default: *lo = -inf; *hi = inf; break;
    }
}

}  // namespace

extern "C" int sim_optimize(sim_t *h, const sim_opt_config *oc, const float *observed, double *loss_history,
                            sim_opt_result *res)
{
    using sim::set_error;
    if (!h) return SIM_EINVAL;
    if (!oc || !res) return set_error(h, SIM_EINVAL, "null config or result");
    if (!sim::is_recording(h)) return set_error(h, SIM_ESTATE, "sim_optimize needs a recording handle");
    if (sim::scenarios_of(h) != 1) return set_error(h, SIM_EUNSUPPORTED, "sim_optimize takes one scenario");
    if (oc->steps < 1 || oc->steps > sim::max_steps_of(h))
        return set_error(h, SIM_EINVAL, "steps must lie in [1, max_steps]");
    if (oc->max_iters < 1 || oc->patience < 1) return set_error(h, SIM_EINVAL, "max_iters and patience must be >= 1");
    if (!(oc->lr > 0) || !(oc->beta1 >= 0 && oc->beta1 < 1) || !(oc->beta2 >= 0 && oc->beta2 < 1) ||
        !(oc->eps > 0) || !(oc->weight_decay >= 0))
        return set_error(h, SIM_EINVAL, "bad AdamW hyperparameters");
    if (oc->groups == 0 || (oc->groups >> SIM_P_COUNT) || (oc->groups & (1u << SIM_P_THETA_DEST)))
        return set_error(h, SIM_EINVAL, "groups must name optimisable parameter groups");
    const int D = sim::detectors_of(h), nb = sim::count_bins_of(h), nq = D * nb;
    if (nq == 0) return set_error(h, SIM_EINVAL, "the loss needs detectors and count bins");
    if (oc->loss == SIM_LOSS_COUNTS_MSE) {
        if (!observed) return set_error(h, SIM_EINVAL, "observed counts are NULL");
    } else if (oc->loss == SIM_LOSS_CUMULATIVE) {
        if (oc->target_detector < 0 || oc->target_detector >= D) return set_error(h, SIM_EINVAL, "bad target detector");
        if (nb > 1024) return set_error(h, SIM_EUNSUPPORTED, "at most 1024 count bins");
    } else {
        return set_error(h, SIM_EINVAL, "unknown loss");
    }
    const hipStream_t st = sim::stream_of(h);
    if (hipSetDevice(sim::device_of(h)) != hipSuccess) return set_error(h, SIM_EDEVICE, "hipSetDevice failed");

    std::vector<Group> gs;
    gs.reserve(SIM_P_COUNT);
    for (int k = 0; k < SIM_P_COUNT; ++k) {
        if (!(oc->groups & (1u << k))) continue;
        const int64_t n = sim::group_size(h, k);
        if (n < 0) return set_error(h, SIM_EINVAL, "parameter group not available on this handle");
        gs.emplace_back();
        Group &g = gs.back();
        g.which = k;
        g.n = n;
        default_box(k, &g.lo, &g.hi);
        if (oc->lower) g.lo = oc->lower[k];
        if (oc->upper) g.hi = oc->upper[k];
        if (!(g.lo <= g.hi)) return set_error(h, SIM_EINVAL, "empty parameter box");
        if (oc->normalized) {
            if (!std::isfinite(g.lo) || !std::isfinite(g.hi) || !(g.hi > g.lo))
                return set_error(h, SIM_EINVAL, "normalized optimisation needs finite boxes of positive width");
            g.x0 = g.lo;
            g.sc = g.hi - g.lo;
        }
        const size_t b = (size_t)n * 4;
        if (alloc(g.p, b) || alloc(g.g, b) || alloc(g.m, b) || alloc(g.v, b) || alloc(g.best, b))
            return set_error(h, SIM_ENOMEM, "device allocation for the optimiser failed");
        int rc = sim_get_params(h, k, g.p.get<float>(), n, 1);
        if (rc != SIM_OK) return rc;
        if (hipMemsetAsync(g.m.p, 0, b, st) != hipSuccess || hipMemsetAsync(g.v.p, 0, b, st) != hipSuccess ||
            hipMemcpyAsync(g.best.p, g.p.p, b, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return set_error(h, SIM_EDEVICE, "optimiser state initialisation failed");
        if (k == SIM_P_KAPPA) {
            std::vector<float> top((size_t)n);
            sim::kappa_ceiling(h, top.data());
            if (alloc(g.hi_vec, b)) return set_error(h, SIM_ENOMEM, "device allocation for the optimiser failed");
            if (hipMemcpy(g.hi_vec.p, top.data(), b, hipMemcpyHostToDevice) != hipSuccess)
                return set_error(h, SIM_EDEVICE, "copy failed");
        }
    }
    DevBuf q, y, gq, loss;
    if (alloc(q, (size_t)nq * 4) || alloc(y, (size_t)nq * 4) || alloc(gq, (size_t)nq * 4) || alloc(loss, 8))
        return set_error(h, SIM_ENOMEM, "device allocation for the optimiser failed");
    if (oc->loss == SIM_LOSS_COUNTS_MSE &&
        hipMemcpy(y.p, observed, (size_t)nq * 4, hipMemcpyHostToDevice) != hipSuccess)
        return set_error(h, SIM_EDEVICE, "copy of the observed counts failed");
    std::vector<float *> grads(SIM_P_COUNT, nullptr);
    for (auto &g : gs) grads[g.which] = g.g.get<float>();

    const auto t0 = std::chrono::steady_clock::now();
    double best = std::numeric_limits<double>::infinity();
    int best_it = 0, since = 0, it = 0, rc = SIM_OK;
    res->first_loss = 0.0;
    for (; it < oc->max_iters; ++it) {
        if ((rc = sim_reset(h)) != SIM_OK) break;
        if ((rc = sim_rollout(h, oc->steps)) != SIM_OK) break;
        if ((rc = sim_get_observables(h, q.get<float>(), nullptr, 1)) != SIM_OK) break;
        sim::launch_count_loss(nq, nb, q.get<float>(), y.get<float>(), oc->loss, oc->target_detector, oc->target,
                               loss.get<double>(), gq.get<float>(), st);
        double lv = 0.0;
        if (hipMemcpyAsync(&lv, loss.p, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) { rc = set_error(h, SIM_EDEVICE, "loss read-back failed"); break; }
        if (loss_history) loss_history[it] = lv;
        if (it == 0) res->first_loss = lv;
        if (lv < best) {
            best = lv;
            best_it = it;
            since = 0;
            for (auto &g : gs)
                if (hipMemcpyAsync(g.best.p, g.p.p, (size_t)g.n * 4, hipMemcpyDeviceToDevice, st) != hipSuccess) {
                    rc = set_error(h, SIM_EDEVICE, "copy failed");
                    break;
                }
            if (rc != SIM_OK) break;
        } else if (++since >= oc->patience) {
            ++it;
            break;
        }
        if (it + 1 == oc->max_iters) { ++it; break; }   // no update after the last evaluation
        if ((rc = sim_backward(h, gq.get<float>(), nullptr, nullptr, oc->groups, grads.data(), 1)) != SIM_OK) break;
        if (it == 0 && oc->first_grad)
            for (auto &g : gs)
                if (oc->first_grad[g.which] &&
                    hipMemcpy(oc->first_grad[g.which], g.g.p, (size_t)g.n * 4, hipMemcpyDeviceToHost) != hipSuccess) {
                    rc = set_error(h, SIM_EDEVICE, "copy of the first gradient failed");
                    break;
                }
        if (rc != SIM_OK) break;
        for (auto &g : gs) {
            sim::launch_adamw(g.n, g.p.get<float>(), g.g.get<float>(), g.m.get<float>(), g.v.get<float>(), it + 1,
                              oc->lr, oc->beta1, oc->beta2, oc->eps, oc->weight_decay, g.x0, g.sc, g.lo, g.hi,
                              g.hi_vec.p ? g.hi_vec.get<float>() : nullptr, st);
            if ((rc = sim_set_params(h, g.which, g.p.get<float>(), g.n, 1)) != SIM_OK) break;
        }
        if (rc != SIM_OK) break;
    }
    // leave the handle on the best parameters seen
    for (auto &g : gs) {
        const int r2 = sim_set_params(h, g.which, g.best.get<float>(), g.n, 1);
        if (rc == SIM_OK) rc = r2;
    }
    if (rc == SIM_OK) rc = sim_reset(h);
    res->iterations = it;
    res->best_iter = best_it;
    res->best_loss = best;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}
