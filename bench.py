#!/usr/bin/env python3
"""Benchmark of the differentiable agent-based traffic step on one MI355X.

One benchmark step = one pass of the whole hot path over the synthetic
1M-agent metro workload (12k nodes, ~35k links, 1,800 simulated steps of
1 s): departures, per-link ordering and car-following, route choice, merge
and FIFO transfer, detector counts, a checkpoint every 60 steps, then the
reverse-mode adjoint with checkpointed replay.  `value` is vehicle-steps per
second of that forward+adjoint pass over K passes (vehicle-steps = sum over
simulated steps of agents on the network; the replay is not counted again);
the median, minimum and maximum pass time and N_pool * T per second are
reported beside it, and the same for the forward alone.

`roofline` is the node kernel (the largest share of device time): the
hot path's algorithmic bytes per launch over its average launch duration,
taken from the committed rocprofv3 kernel trace of this workload when that
was recorded on the current kernel sources, with the live HIP-event and
wave-stamp durations beside it.  Whole-pass fractions follow the hot path's
per-agent byte model (forward 28 B per agent-step; forward+adjoint 92 B).

Further legs: batched control (16 scenarios in one launch per step), the
calibration and cost-control loops, continuous-batching serving of a Poisson
stream of nowcast requests against the plain path, and the oracle timed on
the host as the CPU baseline.  Inputs are generated and uploaded before each
timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def byte_model(kind: str, S: int, L: int, Nn: int, O: int, T: int, vs: int, moves: int, launches: int,
               R: int = None, vs_r: int = None, moves_r: int = None) -> float:
    """Algorithmic (compulsory) bytes per launch of each kernel kind, from the
    structure-of-arrays layout; each array counted once per launch.
      link: per segment 72 B (ring counters, link constants, bucket r/w,
            entry slots, head count), per agent on the network 8 B (position
            read + write), per head 140 B (agent, destination, candidate links
            with shortest-time entries, merge key, head record); in the
            recorded replay also 8 B per agent and 8 B per segment of tape.
      node: per node 24 B (CSR offsets), per link 64 B (in-link head count,
            bucket, outflow, ring head; out-link ring tail and entry slots),
            per head candidate 16 B, per mover 12 B, per origin 40 B.
      reverse: per segment 40 B, per agent 24 B (tape position and agent id,
            adjoint read + write, departure step).
    `vs` = vehicle-steps of the forward, `moves` = transfers + exits + departures; R steps
    are replayed (the first R of the horizon) with `vs_r` vehicle-steps and `moves_r` moves
    (default: every step replayed once).  Every step is taped once, by the forward or by its
    replay."""
    if R is None:
        R, vs_r, moves_r = T, vs, moves
    if kind == "link":
        total = (T + R) * 72.0 * S * L + 8.0 * (vs + vs_r) + 140.0 * (moves + moves_r) + 8.0 * vs + 8.0 * S * L * T
    elif kind == "node":
        total = (T + R) * (24.0 * S * Nn + 64.0 * S * L + 40.0 * S * O) + (16.0 + 12.0) * (moves + moves_r)
    elif kind == "reverse":
        total = T * 40.0 * S * L + 24.0 * vs
    else:
        raise ValueError(kind)
    return total / max(launches, 1)


def _code_only(src: str) -> str:
    """C++ source without comments, trailing blanks and empty lines (what a counter depends on)."""
    import re
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(line.rstrip() for line in src.splitlines() if line.strip())


def kernel_source_digest(read=None) -> str:
    """Digest of the kernel sources' code (comments ignored); a counter summary names the digest
    it was taken on.  `read(name)` returns a source's text (default: the working tree's)."""
    import hashlib
    if read is None:
        def read(name):
            with open(os.path.join(ROOT, "paper_2603_25068_amd", "csrc", name)) as fh:
                return fh.read()
    h = hashlib.sha256()
    for f in ("sim_kernels.hip", "sim_internal.h"):
        h.update(_code_only(read(f)).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the factor a plain copy of known
    size gives), or None when there is none for this workload or the kernels
    have changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_digest") != kernel_source_digest():
        return None
    try:
        return int(float(vals["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def make_workload(name: str, sim_steps=None):
    from paper_2603_25068_amd import workloads as W
    if name == "metro":
        w = W.metro()
    elif name == "grid":
        w = W.grid_rates()
    elif name == "small":
        w = W.random_small(3, nx=6, ny=6, n_agents=3000, rates=True, steps=600)
    else:
        raise ValueError(name)
    if sim_steps:
        w.cfg.steps = int(sim_steps)
    return w


def host_info() -> dict:
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def _oracle_pass(w, n_steps=None, budget_s=None):
    """The oracle as it stands: logged forward over the first n_steps (all if None, or until
    budget_s passes), then its reverse sweep.  Returns (vehicle-steps, steps run, seconds)."""
    import numpy as np
    import oracle
    T = w.cfg.steps if n_steps is None else n_steps
    o = oracle.Oracle(w, log=True, steps=T)
    vs, done = 0, 0
    t0 = time.perf_counter()
    for _ in range(T):
        o.step()
        vs += o.counters()["on_net"]
        done += 1
        if budget_s is not None and time.perf_counter() - t0 > budget_s:
            break
    cnt, _ = o.counts()
    o.backward(gQ=np.ones(cnt.shape) if cnt.size else None, gT=1.0)
    return vs, done, time.perf_counter() - t0


def cpu_baseline(w, n_steps: int, budget_s: float, full=True):
    """The oracle (plain sequential C, one thread) on a bounded sample of the benchmark workload,
    and in full on the 4x4 and 32x32 lattices, forward with decision log + reverse sweep."""
    from paper_2603_25068_amd import workloads as W
    vs, done, el = _oracle_pass(w, n_steps, budget_s)
    out = {"value": round(vs / el, 1), "unit": "vehicle-steps/s", "cores": 1, "kind": "oracle",
           "sample": f"first {done} of {w.cfg.steps} steps of {w.name}, forward with decision log + "
                     f"reverse sweep, single thread, {vs} vehicle-steps in {el:.1f} s",
           "host": host_info()}
    if full:
        runs = {}
        for label, ww in (("grid4x4_1k_fixed", W.small_grid_fixed()), ("grid32x32_50k_rates", W.grid_rates())):
            v, d, e = _oracle_pass(ww)
            runs[label] = {"steps": d, "vehicle_steps": v, "seconds": round(e, 2),
                           "vehicle_steps_per_s": round(v / e, 1)}
        out["full_runs_fwd_adj"] = runs
    return out


def _pct(x, p):
    import numpy as np
    x = np.sort(np.asarray(x, np.float64))
    return float(x[min(len(x) - 1, max(0, int(np.ceil(p * len(x))) - 1))])


def _make_metro(spec):
    from paper_2603_25068_amd import workloads as W
    return W.metro(**spec)


def serving_leg(n_requests: int, rate: float, steps: int, max_slots: int, budget: int, seed: int = 41,
                saturate_factor: float = 16.0):
    """Poisson stream of nowcast rollouts on seeded metro networks of log-uniform size through the
    continuous-batching server, against the plain path (one request at a time, each through its
    own simulator handle).  Requests are generated before the clock starts (client side); latency
    is arrival to result on the host, host preparation included.

    - at the stated arrival rate: server in real time; plain path run back to back, each request's
      service time measured, and its FIFO latencies computed from the arrival times (a single
      server queue: finish_i = max(arrival_i, finish_(i-1)) + service_i);
    - saturated: the same requests arriving saturate_factor times faster, so arrivals outpace
      service; server in real time, plain path as the sum of the service times."""
    import numpy as np
    import torch
    from concurrent.futures import ProcessPoolExecutor
    from paper_2603_25068_amd import workloads as W
    from paper_2603_25068_amd.sim import Server, Simulator, SRV_DONE

    reqs = W.serving_requests(n_requests, rate_per_s=rate, steps=steps, seed=seed)
    arrivals = np.asarray([a for a, _ in reqs]) - reqs[0][0]
    t_gen = time.perf_counter()
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        ws = list(ex.map(_make_metro, [spec for _, spec in reqs], chunksize=4))
    gen_s = time.perf_counter() - t_gen

    def served(arr):
        srv = Server(device=0, mem_budget_bytes=budget, max_slots=max_slots, chunk_steps=60)
        t0 = time.perf_counter()
        tickets = []
        for a, w in zip(arr, ws):
            d = t0 + a - time.perf_counter()
            if d > 0:
                time.sleep(d)
            tickets.append(srv.submit(w, steps=steps))
        res = []
        for t in tickets:
            st = srv.wait(t, 1800.0)
            if st != SRV_DONE:
                raise RuntimeError(f"request {t} ended in state {st}: {srv.error(t)}")
            res.append(srv.result(t))
        sb = srv.stats()
        srv.close()
        return res, sb

    batched, sb = served(arrivals)
    # plain path, back to back: service time of each request
    torch.cuda.synchronize()
    service, same, vs_all = [], True, 0
    for i, w in enumerate(ws):
        t1 = time.perf_counter()
        sim = Simulator(w, steps=steps, max_steps=steps)
        sim.rollout(steps)
        c, T = sim.observables()
        v = sim.vehicle_steps()
        service.append(time.perf_counter() - t1)
        sim.close()
        vs_all += int(v.sum())
        same &= bool(np.array_equal(c, batched[i][0]) and np.array_equal(T, batched[i][1])
                     and np.array_equal(v, batched[i][2]))
    service = np.asarray(service)

    def fifo(arr):
        fin, lat, prev = np.zeros(len(arr)), np.zeros(len(arr)), 0.0
        for i, (a, sv) in enumerate(zip(arr, service)):
            prev = max(a, prev) + sv
            fin[i], lat[i] = prev, prev - a
        return lat, fin[-1] - arr[0]

    lat, span = fifo(arrivals)
    sat = arrivals / saturate_factor
    batched_sat, ss = served(sat)
    same &= all(np.array_equal(batched_sat[i][0], batched[i][0]) for i in range(len(ws)))
    lat_sat, span_sat = fifo(sat)
    agents = [int(w.dem.n_agents) for w in ws]
    links = [int(w.net.n_links) for w in ws]
    return {
        "workload": f"Poisson {rate:g} req/s, {n_requests} requests of {steps} steps on seeded metro networks, "
                    f"links {min(links)}-{max(links)}, agents {min(agents)}-{max(agents)} (log-uniform); "
                    f"client-side generation {gen_s:.1f} s, not timed",
        "batched": {"p50_s": round(sb["p50_s"], 4), "p99_s": round(sb["p99_s"], 4),
                    "vehicle_steps_per_s": round(sb["vehicle_steps_per_s"], 1),
                    "max_running": sb["max_running"], "max_slots": max_slots, "mem_budget_bytes": budget},
        "plain_fifo": {"p50_s": round(_pct(lat, 0.5), 4), "p99_s": round(_pct(lat, 0.99), 4),
                       "vehicle_steps_per_s": round(vs_all / span, 1),
                       "note": "back-to-back service times, FIFO latencies from the arrival times"},
        "saturated": {"arrival_rate_per_s": rate * saturate_factor,
                      "batched": {"p50_s": round(ss["p50_s"], 4), "p99_s": round(ss["p99_s"], 4),
                                  "vehicle_steps_per_s": round(ss["vehicle_steps_per_s"], 1),
                                  "max_running": ss["max_running"]},
                      "plain_fifo": {"p50_s": round(_pct(lat_sat, 0.5), 4), "p99_s": round(_pct(lat_sat, 0.99), 4),
                                     "vehicle_steps_per_s": round(vs_all / span_sat, 1)}},
        "service_s": {"sum": round(float(service.sum()), 2), "median": round(float(np.median(service)), 4),
                      "max": round(float(service.max()), 4)},
        "results_identical": bool(same),
    }


def control_leg(repeats: int = 2):
    """Batched control: 16 candidate scenarios of capacity multipliers on the 32x32 lattice, 3,600
    steps, one launch per step for all scenarios, then the adjoint of each scenario's total travel
    time in its multipliers.  Reports vehicle-steps/s of that forward+adjoint pass over all scenarios
    and the same for one scenario alone (scenario 0) for comparison."""
    import torch
    from paper_2603_25068_amd import workloads as W
    from paper_2603_25068_amd.sim import Simulator
    w = W.batched_control()
    S, T = int(w.extra["n_scenarios"]), w.cfg.steps
    m = w.extra["cap_mult"]
    dev = torch.device("cuda", 0)
    out = {}
    for label, n_s, mult in (("batched", S, m), ("single", 1, m[:1])):
        sim = Simulator(w, n_scenarios=n_s, record=True, max_steps=T, params={"cap_mult": mult})
        gT = torch.ones(n_s, dtype=torch.float64, device=dev)

        def one():
            sim.reset()
            sim.step(T)
            return sim.backward_device(gT=gT, groups=("cap_mult",))

        one()
        sim.autotune(probe_steps=20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(repeats):
            g = one()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / repeats
        vs = int(sim.vehicle_steps().sum())
        out[label] = {"scenarios": n_s, "ms_per_pass": round(1000.0 * el, 2),
                      "vehicle_steps_per_s": round(vs / el, 1),
                      "grad_norm": float(torch.linalg.vector_norm(g["cap_mult"].double()).item())}
        sim.close()
    out["workload"] = (f"{w.name}: {S} scenarios x {w.dem.n_agents} agents, {w.net.n_links} links, {T} steps, "
                       f"TTT gradient in {len(w.extra['controlled_links'])} controlled capacity multipliers")
    return out


def calibration_leg():
    """The optimisation loop of the paper (forward, loss, adjoint, AdamW, stop after 20 iterations
    without improvement, keep the best) on the device:
    - departure rates of the 32x32 lattice (768 parameters) against counts from ground-truth rates;
    - speed, jam density and route weight per link of the Sioux-Falls-sized synthetic network
      against counts from its ground truth, at platoon sizes 1, 2 and 4 (the paper's SI-E sweep;
      the vehicle demand is held, so agents = 20,000 / dn; losses in vehicle units);
    - control: link costs steering the busiest road link's cumulative count to half its value."""
    import numpy as np
    from paper_2603_25068_amd import workloads as W
    from paper_2603_25068_amd.sim import Simulator
    out = {}
    w = W.grid_rates()
    t = Simulator(w, params={"rates": w.extra["theta_true"]})
    t.rollout(w.cfg.steps)
    obs = t.observables()[0][0]
    t.close()
    s = Simulator(w, record=True, max_steps=w.cfg.steps)
    r = s.optimize(("rates",), observed=obs, lr=0.01, weight_decay=1e-5, max_iters=300, patience=20,
                   bounds={"rates": (0.0, 0.25)}, normalized=True)
    s.close()
    out["rates_grid32x32"] = {"parameters": int(w.dem.rates.size), "iterations": r["iterations"],
                              "seconds": round(r["seconds"], 3),
                              "seconds_per_iteration": round(r["seconds"] / max(r["iterations"], 1), 4),
                              "first_loss": round(r["first_loss"], 4), "best_loss": round(r["best_loss"], 4),
                              "best_iter": r["best_iter"]}
    sweep = {}
    groups = ("free_speed", "jam_density", "beta")
    for dn in (1, 2, 4):
        base = W.sioux_like(n_agents=20_000 // dn)
        w = W.with_platoon(W.calibration_start(base), dn)
        t = Simulator(w, params=base.extra["truth"])
        t.rollout(w.cfg.steps)
        obs = t.observables()[0][0]
        t.close()
        s = Simulator(w, record=True, max_steps=w.cfg.steps)
        s.set_params("jam_density", w.extra["start"]["jam_density"])
        r = s.optimize(groups, observed=obs, lr=0.01, weight_decay=1e-5, max_iters=300, patience=20,
                       bounds={g: W.PAPER_RANGES[g] for g in groups}, normalized=True)
        s.close()
        sweep[f"dn{dn}"] = {"agents": int(w.dem.n_agents), "steps": int(w.cfg.steps), "dt": w.cfg.dt,
                            "iterations": r["iterations"], "seconds": round(r["seconds"], 3),
                            "first_loss_veh": round(r["first_loss"] * dn * dn, 2),
                            "best_loss_veh": round(r["best_loss"] * dn * dn, 2), "best_iter": r["best_iter"]}
    out["per_link_sioux_like_platoon_sweep"] = sweep
    w = W.sioux_like()
    t = Simulator(w)
    t.rollout(w.cfg.steps)
    base = t.observables()[0][0]
    t.close()
    tot = base.sum(1)
    roads = int(w.net.n_links - w.net.n_nodes // 2)
    det = int(np.argmax(tot[:roads]))
    s = Simulator(w, record=True, max_steps=w.cfg.steps)
    r = s.optimize(("cost",), loss="cumulative", target_detector=det, target=0.5 * float(tot[det]), lr=0.1,
                   weight_decay=1e-5, max_iters=300, patience=20, bounds={"cost": (0.05, 20.0)})
    s.rollout(w.cfg.steps)
    after = float(s.observables()[0][0][det].sum())
    s.close()
    out["control_by_cost_sioux_like"] = {"target_link_count": float(tot[det]), "target": 0.5 * float(tot[det]),
                                         "count_at_best": after, "iterations": r["iterations"],
                                         "seconds": round(r["seconds"], 3)}
    return out


def profile_pass(args):
    """One forward+adjoint pass of the workload and nothing else (for counter
    runs), or a plain device copy of known size (the counters' calibration)."""
    import torch
    from paper_2603_25068_amd.sim import Simulator
    dev = torch.device("cuda", 0)
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 3}))
        return
    w = make_workload(args.workload, args.sim_steps)
    T = w.cfg.steps
    sim = Simulator(w, record=True, max_steps=T, tape_windows=(T + w.cfg.ckpt_every - 1) // w.cfg.ckpt_every)
    gQ = torch.ones((1, w.net.n_detectors, sim.n_count_bins), dtype=torch.float32, device=dev)
    gT = torch.ones(1, dtype=torch.float64, device=dev)
    if args.schedule:
        sim.set_schedule(*[int(x) for x in args.schedule.split(",")])
    sim.reset()
    sim.step(T)
    sim.backward_device(gQ=gQ, gT=gT)
    torch.cuda.synchronize()
    print(json.dumps({"profile_pass": w.name, "sim_steps": T, "vehicle_steps": int(sim.vehicle_steps()[0])}))


def rocprof_avg_us(kernel: str, workload: str):
    """Average duration (us) of `kernel` in a committed rocprofv3 kernel-trace summary of this
    workload (profiles/*_<workload>_kernel_trace.txt, one table of every step kernel), when the
    summary's kernel-source digest is the current one; else None."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(f"_{workload}_kernel_trace.txt"):
            continue
        text = open(os.path.join(pdir, name)).read()
        dig = None
        for line in text.splitlines():
            if line.startswith("kernel_source_digest:"):
                dig = line.split(":", 1)[1].strip()
        if dig != kernel_source_digest():
            continue
        for line in text.splitlines():
            parts = line.split()
            if (f"sim::{kernel}(" in line or f"sim::{kernel}<" in line) and len(parts) >= 7:
                try:
                    return float(parts[-4])    # ... calls, total ms, avg us, %, min us, max us
                except ValueError:
                    continue
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed forward+adjoint passes")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="metro", choices=["metro", "grid", "small"])
    ap.add_argument("--sim-steps", type=int, default=None, help="override simulated steps per pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=900)
    ap.add_argument("--cpu-budget-s", type=float, default=20.0)
    ap.add_argument("--serve-requests", type=int, default=256, help="requests in the serving leg (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=4.0)
    ap.add_argument("--serve-steps", type=int, default=3600)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--profile-pass", action="store_true", help="one forward+adjoint pass only")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tape-windows", type=int, default=-1,
                    help="windows of replay tape kept on the device (the forward tapes the last ones); "
                         "-1: every window of the rollout, so the backward replays none")
    ap.add_argument("--no-control", action="store_true", help="skip the batched-control leg")
    ap.add_argument("--no-calibration", action="store_true", help="skip the calibration and cost-control legs")
    ap.add_argument("--schedule", default="", help="g_link,g_node,g_rev instead of the autotuner's choice")
    ap.add_argument("--fwd-adj-only", action="store_true",
                    help="skip the forward-only timing (profiled runs: every pass then has the same kernel mix)")
    ap.add_argument("--copy-probe-mib", type=int, default=0, help="with --profile-pass: time a plain copy")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the simulator runs every scenario on a single device; "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.profile_pass:
        profile_pass(args)
        return

    import numpy as np
    import torch
    from paper_2603_25068_amd.sim import Simulator

    t_gen = time.perf_counter()
    w = make_workload(args.workload, args.sim_steps)
    T = w.cfg.steps
    gen_s = time.perf_counter() - t_gen
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.tape_windows < 0:   # 288 GB of HBM hold every window's tape (about 2 GB each at 1M agents)
        args.tape_windows = (T + w.cfg.ckpt_every - 1) // w.cfg.ckpt_every
    sim = Simulator(w, record=True, max_steps=T, tape_windows=args.tape_windows)
    fwd = Simulator(w, record=False)
    S, L, Nn, O = 1, w.net.n_links, w.net.n_nodes, w.net.n_origins
    nb = sim.n_count_bins
    gQ = torch.ones((S, w.net.n_detectors, nb), dtype=torch.float32, device=dev)
    gT = torch.ones(S, dtype=torch.float64, device=dev)

    def fwd_adj(s):
        s.reset()
        s.step(T)
        s.backward_device(gQ=gQ, gT=gT)

    def fwd_only(s):
        s.reset()
        s.step(T)

    for _ in range(args.warmup):
        fwd_adj(sim)
        if not args.fwd_adj_only:
            fwd_only(fwd)
    schedule = None
    if args.schedule:
        gs = [int(x) for x in args.schedule.split(",")]
        sim.set_schedule(*gs)
        fwd.set_schedule(*gs)
        schedule = {"fwd+adj": list(gs), "fwd": list(gs)}
    elif not args.no_autotune:
        # tune on the loaded end-of-rollout state (restored afterwards; results do not change)
        schedule = {"fwd+adj": sim.autotune(probe_steps=30), "fwd": fwd.autotune(probe_steps=30)}

    def timed(fn, s):
        """K passes between synchronisations; HIP events on the library's stream split the passes."""
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs[0].record(s.stream)
        for k in range(args.steps):
            fn(s)
            evs[k + 1].record(s.stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        per = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
        return el, {"median": round(float(np.median(per)), 3), "min": round(float(np.min(per)), 3),
                    "max": round(float(np.max(per)), 3)}

    el, pass_ms = timed(fwd_adj, sim)
    vs = int(sim.vehicle_steps()[0])
    st = sim.state()["counters"][0]
    el_f, fwd_ms, vs_f = None, None, None
    if not args.fwd_adj_only:
        el_f, fwd_ms = timed(fwd_only, fwd)
        vs_f = int(fwd.vehicle_steps()[0])
        assert vs_f == vs

    ms_per_step = 1000.0 * el / args.steps
    value = vs * args.steps / el
    fwd_value = vs_f * args.steps / el_f if el_f else None
    n_pool_T = int(w.dem.n_agents) * T

    # per-kernel device time, one extra pass: each launch's own wave stamps and HIP events around it
    sim.set_timing(True)
    sim.timing(reset=True)
    fwd_adj(sim)
    tm = sim.timing(reset=True)
    sim.set_timing(False)
    moves = st["transfers"] + st["exited"] + st["departed"]
    kinds = {k: v for k, v in tm.items() if k in ("link", "node", "reverse") and v[1] > 0}
    # the kernel with the largest share of device time: HIP events around each launch on its stream
    # (the ordering rocprofv3's trace totals give too); the waves' own stamps, which leave out each
    # launch's dispatch and drain, only when no events were taken
    def device_ms(k):
        ev = tm.get(k + "_ev", (0.0, 0))
        return ev[0] if ev[1] else kinds[k][0]
    dom = max(kinds, key=device_ms)
    ms_tot, launches = kinds[dom]
    self_us = 1000.0 * ms_tot / launches
    ev_ms, ev_n = tm.get(dom + "_ev", (0.0, 0))
    ev_us = 1000.0 * ev_ms / ev_n if ev_n else None
    rp_us = rocprof_avg_us(f"k_{dom}", w.name)
    # the replayed steps of the pass (the windows before the taped ones), measured on a forward run
    R = max(0, tm.get("node", (0.0, T))[1] - T)
    fwd.reset()
    fwd.step(R)
    vs_r = int(fwd.vehicle_steps()[0])
    cr = fwd.state()["counters"][0]
    moves_r = cr["transfers"] + cr["exited"] + cr["departed"]
    # hot-path byte model (28 B per agent-step forward, 68 B per head that moves, 48 B per link or
    # origin and step; 92 B per agent-step for forward+adjoint with every step replayed)
    def alg_of(kind, n_launch):
        if kind == "node":
            return (48.0 * (L + O) * (T + R) + 68.0 * (moves + moves_r)) / n_launch
        if kind == "link":
            return (28.0 * (vs + vs_r) + 48.0 * L * (T + R)) / n_launch
        return (24.0 * vs) / n_launch   # reverse: tape read 12 + adjoint read/write 8 + follower gather 4
    alg = alg_of(dom, launches)
    # every step kernel against its own hot-path byte model, with the trace's duration when the
    # committed summary is current, else the live HIP-event figure
    by_kernel = {}
    for kind, (k_ms, k_n) in kinds.items():
        k_ev = tm.get(kind + "_ev", (0.0, 0))
        k_us = rocprof_avg_us(f"k_{kind}", w.name)
        k_src = "rocprofv3 kernel trace (profiles/)"
        if k_us is None:
            k_us = 1000.0 * k_ev[0] / k_ev[1] if k_ev[1] else 1000.0 * k_ms / k_n
            k_src = "HIP events (live)" if k_ev[1] else "wave stamps (live)"
        k_alg = alg_of(kind, k_n)
        by_kernel[f"k_{kind}"] = {"alg_bytes_per_launch": int(k_alg), "avg_launch_us": round(k_us, 3),
                                  "source": k_src, "frac": round(k_alg / (k_us * 1e-6) / 1e9 / PEAK_HBM_GBS, 5),
                                  "traffic": measured_traffic(f"k_{kind}", w.name)}
    alg_kernel_model = byte_model(dom, S, L, Nn, O, T, vs, moves, launches, R, vs_r, moves_r)
    dur_us, src = (rp_us, "rocprofv3 kernel trace (profiles/)") if rp_us else (ev_us, "HIP events (live)")
    if dur_us is None:
        dur_us, src = self_us, "wave stamps (live)"
    achieved = alg / (dur_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 5), "traffic": measured_traffic(f"k_{dom}", w.name),
                "kernel": f"k_{dom}", "avg_launch_us": round(dur_us, 3), "avg_launch_source": src,
                "launch_us": {"hip_events_live": round(ev_us, 3) if ev_us else None,
                              "wave_stamps_live": round(self_us, 3),
                              "rocprof_kernel_trace": rp_us},
                "alg_bytes_per_launch": int(alg),
                "alg_model": {"node": "node phase: 48 B per link or origin and step + 68 B per moving head "
                                      "(transfer, exit, departure), forward and replayed steps",
                              "link": "link phase: 28 B per agent-step + 48 B per link and step, forward and "
                                      "replayed steps",
                              "reverse": "reverse sweep: 24 B per agent-step (tape read 12, adjoint read and "
                                         "write 8, follower-adjoint gather 4)"}[dom],
                "by_kernel": by_kernel,
                "alg_bytes_per_launch_kernel_model": int(alg_kernel_model),
                "kernel_ms": {k: [round(v[0], 3), v[1]] for k, v in tm.items()}}
    # whole passes
    fwd_bytes = 28.0 * vs + 68.0 * moves + 48.0 * (L + O) * T
    pass_survey = 92.0 * vs + 68.0 * 2 * moves + 48.0 * (L + O) * 2 * T
    pass_as_run = 64.0 * vs + 28.0 * vs_r + 68.0 * (moves + moves_r) + 48.0 * (L + O) * (T + R)
    sec = ms_per_step * 1e-3
    roofline["pass"] = {
        "survey_model": {"bytes": int(pass_survey), "frac": round(pass_survey / sec / 1e9 / PEAK_HBM_GBS, 5),
                         "model": "92 B/agent-step + 68 B/move + 48 B/(link|origin)-step, forward and a full replay"},
        "as_run_model": {"bytes": int(pass_as_run), "frac": round(pass_as_run / sec / 1e9 / PEAK_HBM_GBS, 5),
                         "model": "64 B/agent-step + 28 B per replayed agent-step + 68 B/move + 48 B/(link|origin)-step, "
                                  "%d of %d steps replayed" % (R, T)}}
    if el_f:
        secf = el_f / args.steps
        roofline["forward"] = {"bytes": int(fwd_bytes), "frac": round(fwd_bytes / secf / 1e9 / PEAK_HBM_GBS, 5),
                               "model": "28 B/agent-step + 68 B/move + 48 B/(link|origin)-step"}

    def leg(name, fn):
        t0 = time.perf_counter()
        r = fn()
        print(f"[bench] {name} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        return r

    control = None if args.no_control else leg("batched control", control_leg)
    calib = None if args.no_calibration else leg("calibration", calibration_leg)
    serving = None
    if args.serve_requests > 0:
        serving = leg("serving", lambda: serving_leg(args.serve_requests, args.serve_rate, args.serve_steps,
                                                     args.serve_slots, int(args.serve_budget_gib * (1 << 30))))
    cpu = None
    if not args.no_cpu_baseline:
        cpu = leg("cpu baseline", lambda: cpu_baseline(make_workload(args.workload, args.sim_steps), args.cpu_steps,
                                                       args.cpu_budget_s))

    line = {
        "metric": "vehicle-steps/s fwd & fwd+adjoint at 1M agents; nowcast p50/p99 latency",
        "value": round(value, 1), "unit": "vehicle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "agents": w.dem.n_agents, "links": L, "nodes": Nn, "origins": O,
                   "sim_steps": T, "ckpt_every": w.cfg.ckpt_every, "tape_windows": args.tape_windows,
                   "pass": "forward+adjoint", "vehicle_steps_per_pass": vs,
                   "pass_ms": pass_ms, "n_pool_T": n_pool_T, "n_pool_T_per_s": round(n_pool_T * args.steps / el, 1),
                   "forward_only_vehicle_steps_per_s": round(fwd_value, 1) if fwd_value else None,
                   "forward_only_ms": fwd_ms,
                   "counters": st, "generate_s": round(gen_s, 2),
                   "schedule_g_link_g_node_g_rev": schedule},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
        "batched_control": control,
        "calibration": calib,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
