#!/usr/bin/env python3
"""Benchmark of the differentiable agent-based traffic step on one MI355X.

One benchmark step = one pass of the whole hot path over the synthetic
1M-agent metro workload (12k nodes, ~35k links, 1,800 simulated steps of
1 s): departures, per-link ordering and car-following, route choice, merge
and FIFO transfer, detector counts, a checkpoint every 60 steps, then the
reverse-mode adjoint with checkpointed replay.  `value` is vehicle-steps per
second of that forward+adjoint pass (vehicle-steps = sum over simulated
steps of agents on the network; the replay is not counted again).  The
forward-only rate is reported beside it.

Inputs are generated and uploaded before the timed region.  The oracle (a
plain single-threaded C implementation) is timed on a bounded sample of the
same workload as the CPU baseline.
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


def cpu_baseline(w, n_steps: int, budget_s: float):
    """The oracle as it stands on the first n_steps of the workload: logged
    forward then the reverse sweep, single thread."""
    import numpy as np
    import oracle
    o = oracle.Oracle(w, log=True, steps=n_steps)
    vs = 0
    t0 = time.perf_counter()
    done = 0
    for k in range(n_steps):
        o.step()
        vs += o.counters()["on_net"]
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    cnt, _ = o.counts()
    o.backward(gQ=np.ones(cnt.shape) if cnt.size else None, gT=1.0)
    el = time.perf_counter() - t0
    return {"value": vs / el, "unit": "vehicle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} of {w.cfg.steps} steps of {w.name}, forward with decision log + "
                      f"reverse sweep, single thread, {vs} vehicle-steps in {el:.1f} s"}


def serving_leg(n_requests: int, rate: float, steps: int, max_slots: int, budget: int, seed: int = 41):
    """Poisson stream of nowcast rollouts on seeded metro networks of log-uniform
    size: the continuous-batching server against the plain path (one request
    at a time, in arrival order, each through its own simulator handle).
    Requests are generated before the clock starts (client side); latency is
    arrival to result on the host, including host preparation."""
    import numpy as np
    import torch
    from paper_2603_25068_amd import workloads as W
    from paper_2603_25068_amd.sim import Server, Simulator, SRV_DONE

    reqs = W.serving_requests(n_requests, rate_per_s=rate, steps=steps, seed=seed)
    arrivals = [a for a, _ in reqs]
    ws = [W.metro(**spec) for _, spec in reqs]

    # continuous batching
    srv = Server(device=0, mem_budget_bytes=budget, max_slots=max_slots, chunk_steps=60)
    t0 = time.perf_counter()
    tickets = []
    for a, w in zip(arrivals, ws):
        d = t0 + a - time.perf_counter()
        if d > 0:
            time.sleep(d)
        tickets.append(srv.submit(w, steps=steps))
    batched = []
    for t in tickets:
        st = srv.wait(t, 1200.0)
        if st != SRV_DONE:
            raise RuntimeError(f"request {t} ended in state {st}: {srv.error(t)}")
        batched.append(srv.result(t))
    sb = srv.stats()
    srv.close()

    # plain path: one request at a time, FIFO
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat, vs_total, plain_same = [], 0, True
    for i, (a, w) in enumerate(zip(arrivals, ws)):
        d = t0 + a - time.perf_counter()
        if d > 0:
            time.sleep(d)
        sim = Simulator(w, steps=steps, max_steps=steps)
        sim.rollout(steps)
        c, T = sim.observables()
        v = sim.vehicle_steps()
        done = time.perf_counter()
        lat.append(done - (t0 + a))
        vs_total += int(v.sum())
        plain_same &= bool(np.array_equal(c, batched[i][0]) and np.array_equal(T, batched[i][1])
                           and np.array_equal(v, batched[i][2]))
        sim.close()
    wall = time.perf_counter() - (t0 + arrivals[0])
    lat = np.sort(np.asarray(lat))

    def pct(x, p):
        return float(x[min(len(x) - 1, int(np.ceil(p * len(x))) - 1)])

    agents = [int(w.dem.n_agents) for w in ws]
    links = [int(w.net.n_links) for w in ws]
    return {
        "workload": f"Poisson {rate:g} req/s, {n_requests} requests of {steps} steps on seeded metro networks, "
                    f"links {min(links)}-{max(links)}, agents {min(agents)}-{max(agents)} (log-uniform)",
        "batched": {"p50_s": round(sb["p50_s"], 4), "p99_s": round(sb["p99_s"], 4),
                    "vehicle_steps_per_s": round(sb["vehicle_steps_per_s"], 1),
                    "max_running": sb["max_running"], "max_slots": max_slots, "mem_budget_bytes": budget},
        "plain_fifo": {"p50_s": round(pct(lat, 0.5), 4), "p99_s": round(pct(lat, 0.99), 4),
                       "vehicle_steps_per_s": round(vs_total / wall, 1)},
        "results_identical": plain_same,
    }


def control_leg(repeats: int = 2):
    """Batched control: 16 candidate scenarios of capacity multipliers on the 32x32 lattice, 3,600
    steps, one launch per step for all scenarios, then the adjoint of each scenario's total travel
    time in its multipliers.  Reports vehicle-steps/s of that forward+adjoint pass over all scenarios
    and the same for one scenario alone (scenario 0) for comparison."""
    import numpy as np
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
    sim = Simulator(w, record=True, max_steps=T)
    gQ = torch.ones((1, w.net.n_detectors, sim.n_count_bins), dtype=torch.float32, device=dev)
    gT = torch.ones(1, dtype=torch.float64, device=dev)
    if args.schedule:
        sim.set_schedule(*[int(x) for x in args.schedule.split(",")])
    sim.reset()
    sim.step(T)
    sim.backward_device(gQ=gQ, gT=gT)
    torch.cuda.synchronize()
    print(json.dumps({"profile_pass": w.name, "sim_steps": T, "vehicle_steps": int(sim.vehicle_steps()[0])}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed forward+adjoint passes")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="metro", choices=["metro", "grid", "small"])
    ap.add_argument("--sim-steps", type=int, default=None, help="override simulated steps per pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=900)
    ap.add_argument("--cpu-budget-s", type=float, default=25.0)
    ap.add_argument("--serve-requests", type=int, default=32, help="requests in the serving leg (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=4.0)
    ap.add_argument("--serve-steps", type=int, default=3600)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--profile-pass", action="store_true", help="one forward+adjoint pass only")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tape-windows", type=int, default=16,
                    help="windows of replay tape kept on the device (the forward tapes the last ones)")
    ap.add_argument("--no-control", action="store_true", help="skip the batched-control leg")
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
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fwd_adj(sim)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    vs = int(sim.vehicle_steps()[0])
    st = sim.state()["counters"][0]
    el_f, vs_f = None, None
    if not args.fwd_adj_only:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            fwd_only(fwd)
        torch.cuda.synchronize()
        el_f = time.perf_counter() - t1
        vs_f = int(fwd.vehicle_steps()[0])
        assert vs_f == vs

    ms_per_step = 1000.0 * el / args.steps
    value = vs * args.steps / el
    fwd_value = vs_f * args.steps / el_f if el_f else None

    # per-kernel device time with HIP events on the library's stream (one extra pass)
    sim.set_timing(True)
    sim.timing(reset=True)
    fwd_adj(sim)
    tm = sim.timing(reset=True)
    sim.set_timing(False)
    moves = st["transfers"] + st["exited"] + st["departed"]
    kinds = {k: v for k, v in tm.items() if k in ("link", "node", "reverse") and v[1] > 0}
    dom = max(kinds, key=lambda k: kinds[k][0])
    ms_tot, launches = kinds[dom]
    avg_ms = ms_tot / launches
    # the replayed steps of the pass (the windows before the taped ones), measured on a forward run
    R = max(0, tm.get("node", (0.0, T))[1] - T)
    fwd.reset()
    fwd.step(R)
    vs_r = int(fwd.vehicle_steps()[0])
    cr = fwd.state()["counters"][0]
    moves_r = cr["transfers"] + cr["exited"] + cr["departed"]
    bytes_launch = byte_model(dom, S, L, Nn, O, T, vs, moves, launches, R, vs_r, moves_r)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 5), "traffic": None, "kernel": f"k_{dom}",
                "avg_launch_us": round(1000.0 * avg_ms, 3), "alg_bytes_per_launch": int(bytes_launch),
                "kernel_ms": {k: [round(v[0], 3), v[1]] for k, v in tm.items()}}

    roofline["traffic"] = measured_traffic(f"k_{dom}", w.name)
    # whole-pass figure with the per-unit model of the hot path: per agent-step on the network 28 B
    # forward, 12 B tape (written once, by the forward or by the replay), 24 B reverse, and 28 B for
    # each replayed agent-step; 68 B per head that moves and 48 B per link or origin and step in each
    # forward sweep (the forward and the replayed steps)
    pass_bytes = 64.0 * vs + 28.0 * vs_r + 68.0 * (moves + moves_r) + 48.0 * (L + O) * (T + R)
    roofline["pass"] = {"model": "64 B/agent-step + 28 B/replayed agent-step + 68 B/move + 48 B/(link|origin)-step, "
                                 "forward and %d replayed steps" % R,
                        "bytes": int(pass_bytes), "achieved": round(pass_bytes / (ms_per_step * 1e-3) / 1e9, 2),
                        "frac": round(pass_bytes / (ms_per_step * 1e-3) / 1e9 / PEAK_HBM_GBS, 5)}

    control = None
    if not args.no_control:
        control = control_leg()

    serving = None
    if args.serve_requests > 0:
        serving = serving_leg(args.serve_requests, args.serve_rate, args.serve_steps, args.serve_slots,
                              int(args.serve_budget_gib * (1 << 30)))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(make_workload(args.workload, args.sim_steps), args.cpu_steps, args.cpu_budget_s)

    line = {
        "metric": "vehicle-steps/s fwd & fwd+adjoint at 1M agents; nowcast p50/p99 latency",
        "value": round(value, 1), "unit": "vehicle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "agents": w.dem.n_agents, "links": L, "nodes": Nn, "origins": O,
                   "sim_steps": T, "ckpt_every": w.cfg.ckpt_every, "tape_windows": args.tape_windows,
                   "pass": "forward+adjoint",
                   "vehicle_steps_per_pass": vs,
                   "forward_only_vehicle_steps_per_s": round(fwd_value, 1) if fwd_value else None,
                   "forward_only_ms": round(1000.0 * el_f / args.steps, 3) if el_f else None,
                   "counters": st, "generate_s": round(gen_s, 2),
                   "schedule_g_link_g_node_g_rev": schedule},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
        "batched_control": control,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
