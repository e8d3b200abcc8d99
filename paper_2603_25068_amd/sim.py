"""Python binding of the HIP simulator library (include/sim.h).

Argument marshalling only: every step of the simulation and of its adjoint
runs in the HIP kernels of libsim.so.  PyTorch supplies the stream (and
device tensors for on-device outputs).  There is no CPU fallback: without the
built library every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsim.so")

SIM_OK, SIM_EINVAL, SIM_ENOMEM, SIM_EDEVICE, SIM_ESTATE, SIM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PARAMS = {"free_speed": 0, "jam_density": 1, "beta": 2, "alpha": 3, "cost": 4, "theta": 5, "rates": 6,
          "cap_mult": 7}   # theta: gradient only (its value is the config's dest_logit_coef)
N_GROUPS = 8
PARAM_NAMES = {v: k for k, v in PARAMS.items()}
COUNTER_NAMES = ("released", "departed", "on_net", "exited", "transfers", "ties", "stuck", "order_viol")
WAIT, QUEUED, ON, EXITED = 0, 1, 2, 3


class SimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class _Network(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_links", C.c_int32),
                ("tail", C.c_void_p), ("head", C.c_void_p), ("lanes", C.c_void_p),
                ("length", C.c_void_p), ("free_speed", C.c_void_p), ("jam_density", C.c_void_p),
                ("capacity", C.c_void_p), ("beta", C.c_void_p), ("alpha", C.c_void_p), ("cost", C.c_void_p),
                ("n_origins", C.c_int32), ("origin_node", C.c_void_p),
                ("n_detectors", C.c_int32), ("detector_link", C.c_void_p), ("detector_pos", C.c_void_p)]


class _Demand(C.Structure):
    _fields_ = [("n_agents", C.c_int32), ("agent_origin", C.c_void_p), ("agent_dest", C.c_void_p),
                ("ready_time", C.c_void_p), ("n_rate_bins", C.c_int32), ("rate_bin_s", C.c_double),
                ("rates", C.c_void_p)]


class _OptConfig(C.Structure):
    _fields_ = [("groups", C.c_uint32), ("steps", C.c_int32), ("max_iters", C.c_int32), ("patience", C.c_int32),
                ("lr", C.c_double), ("weight_decay", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("loss", C.c_int32), ("target_detector", C.c_int32), ("target", C.c_double),
                ("lower", C.c_void_p), ("upper", C.c_void_p), ("normalized", C.c_int32), ("first_grad", C.c_void_p)]


class _OptResult(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("best_iter", C.c_int32), ("first_loss", C.c_double),
                ("best_loss", C.c_double), ("seconds", C.c_double)]


SIM_LOSS_COUNTS_MSE, SIM_LOSS_CUMULATIVE = 0, 1


class _Config(C.Structure):
    _fields_ = [("dt", C.c_double), ("platoon", C.c_int32), ("gumbel_tau", C.c_double),
                ("dest_logit_coef", C.c_double), ("big_m", C.c_double), ("seed", C.c_uint64),
                ("scenario_seed", C.c_void_p), ("n_scenarios", C.c_int32), ("ckpt_every", C.c_int32),
                ("count_bin_steps", C.c_int32), ("n_count_bins", C.c_int32), ("max_steps", C.c_int32),
                ("allow_uturn", C.c_int32), ("record_for_backward", C.c_int32), ("mem_budget_bytes", C.c_size_t),
                ("tape_windows", C.c_int32)]


_LIB = None


def lib():
    """The loaded libsim.so; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
    # torch first, so that the library binds to the HIP runtime torch already loaded (one runtime per
    # process: device memory and streams from torch are then valid in the library)
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "sim_create": ([vp, vp, vp, C.c_int, vp, vp], C.c_int),
        "sim_destroy": ([vp], C.c_int),
        "sim_last_error": ([vp], C.c_char_p),
        "sim_set_params": ([vp, C.c_int, vp, i64, C.c_int], C.c_int),
        "sim_reset": ([vp], C.c_int),
        "sim_place": ([vp, i32, vp, vp, vp], C.c_int),
        "sim_step": ([vp], C.c_int),
        "sim_rollout": ([vp, i32], C.c_int),
        "sim_get_observables": ([vp, vp, vp, C.c_int], C.c_int),
        "sim_backward": ([vp, vp, vp, vp, C.c_uint32, vp, C.c_int], C.c_int),
        "sim_get_state": ([vp, vp, vp, vp, vp, vp], C.c_int),
        "sim_get_link_state": ([vp, vp, vp, vp], C.c_int),
        "sim_get_stats": ([vp, vp], C.c_int),
        "sim_get_dist": ([vp, vp, vp], C.c_int),
        "sim_time": ([vp, vp], C.c_int),
        "sim_philox": ([vp, i32, vp, vp, vp], C.c_int),
        "sim_gumbel_fast": ([vp, i32, vp, vp], C.c_int),
        "sim_segsort": ([vp, i32, i32, vp, vp, vp, vp, vp], C.c_int),
        "sim_segsort_noalloc": ([vp, i32, i32, vp, vp, vp, vp, vp, vp], C.c_int),
        "sim_get_tie_log": ([vp, vp, i64, vp], C.c_int),
        "sim_get_params": ([vp, C.c_int, vp, i64, C.c_int], C.c_int),
        "sim_optimize": ([vp, vp, vp, vp, vp], C.c_int),
        "sim_set_schedule": ([vp, C.c_int, C.c_int, C.c_int], C.c_int),
        "sim_get_schedule": ([vp, vp, vp, vp], C.c_int),
        "sim_set_timing": ([vp, C.c_int], C.c_int),
        "sim_get_timing": ([vp, vp, vp, C.c_int, C.c_int], C.c_int),
        "sim_footprint": ([vp, vp, vp, vp], C.c_int),
        "sim_autotune": ([vp, i32, C.c_char_p, i32, vp, vp, vp], C.c_int),
        "sim_get_full_state": ([vp, vp, C.c_size_t, vp], C.c_int),
        "sim_set_full_state": ([vp, vp, C.c_size_t], C.c_int),
        "srv_create": ([C.c_int, C.c_size_t, i32, i32, vp], C.c_int),
        "srv_submit": ([vp, vp, vp, vp, i32, vp], C.c_int),
        "srv_poll": ([vp, i64, vp], C.c_int),
        "srv_wait": ([vp, i64, C.c_double, vp], C.c_int),
        "srv_result": ([vp, i64, vp, vp, vp, vp], C.c_int),
        "srv_error": ([vp, i64], C.c_char_p),
        "srv_cancel": ([vp, i64], C.c_int),
        "srv_stats": ([vp, vp, vp, vp, vp, vp], C.c_int),
        "srv_destroy": ([vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _LIB = L
    return L


def exported_symbols() -> list:
    return ["sim_create", "sim_destroy", "sim_last_error", "sim_set_params", "sim_reset", "sim_place",
            "sim_step", "sim_rollout", "sim_get_observables", "sim_backward", "sim_get_state",
            "sim_get_link_state", "sim_get_stats", "sim_get_dist", "sim_time", "sim_philox", "sim_gumbel_fast", "sim_segsort",
            "sim_segsort_noalloc", "sim_get_tie_log", "sim_get_params", "sim_optimize", "sim_set_schedule", "sim_get_schedule", "sim_set_timing", "sim_get_timing", "sim_footprint", "sim_autotune", "sim_get_full_state",
            "sim_set_full_state",
            "srv_create", "srv_submit", "srv_poll", "srv_wait", "srv_result", "srv_error", "srv_cancel",
            "srv_stats", "srv_destroy"]


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _f32(a):
    return np.ascontiguousarray(a, np.float32)


def _i32(a):
    return np.ascontiguousarray(a, np.int32)


def _marshal(w, S: int, seeds, steps: int, ckpt_every, max_steps, record: bool, mem_budget_bytes: int,
             tape_windows: int = 0):
    """The C structures of a workload (and the arrays they point into, which
    the caller keeps alive while the structures are in use)."""
    net, dem, cfg = w.net, w.dem, w.cfg
    cbs = int(cfg.count_bin_steps)
    n_count_bins = steps // cbs if cbs > 0 else 0
    K = {
        "tail": _i32(net.tail), "head": _i32(net.head), "lanes": _i32(net.lanes),
        "length": _f32(net.length), "free_speed": _f32(net.free_speed), "jam_density": _f32(net.jam_density),
        "capacity": _f32(net.capacity), "beta": _f32(net.beta), "alpha": _f32(net.alpha), "cost": _f32(net.cost),
        "origin_node": _i32(net.origin_node), "detector_link": _i32(net.detector_link),
        "detector_pos": _f32(net.detector_pos), "agent_origin": _i32(dem.agent_origin),
        "agent_dest": _i32(dem.agent_dest),
    }
    if dem.ready_time is not None:
        K["ready_time"] = _f32(dem.ready_time)
    else:
        K["rates"] = _f32(dem.rates)
    if seeds is not None:
        K["seeds"] = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    n = _Network(net.n_nodes, net.n_links, _p(K["tail"]), _p(K["head"]), _p(K["lanes"]), _p(K["length"]),
                 _p(K["free_speed"]), _p(K["jam_density"]), _p(K["capacity"]), _p(K["beta"]), _p(K["alpha"]),
                 _p(K["cost"]), net.n_origins, _p(K["origin_node"]), net.n_detectors, _p(K["detector_link"]),
                 _p(K["detector_pos"]))
    d = _Demand(dem.n_agents, _p(K["agent_origin"]), _p(K["agent_dest"]), _p(K.get("ready_time")),
                dem.n_rate_bins, float(dem.rate_bin_s), _p(K.get("rates")))
    c = _Config(float(cfg.dt), int(cfg.platoon), float(cfg.gumbel_tau), float(cfg.dest_logit_coef),
                float(cfg.big_m), int(cfg.seed) & (2 ** 64 - 1), _p(K.get("seeds")), int(S),
                int(ckpt_every or cfg.ckpt_every), cbs, n_count_bins,
                int(max_steps if max_steps is not None else steps), int(cfg.allow_uturn), int(record),
                int(mem_budget_bytes), int(tape_windows))
    return n, d, c, K


class Simulator:
    """A handle on the HIP simulator for one workload, batched over scenarios.

    `params`: optional {group: array [S x n] or [n]} overrides (free_speed,
    jam_density, beta, alpha, cost, cap_mult per link; rates per origin x bin).
    `seeds`: optional per-scenario Philox keys (default cfg.seed + s)."""

    def __init__(self, w, n_scenarios: int = 1, params: Optional[dict] = None, seeds: Optional[Sequence[int]] = None,
                 record: bool = False, max_steps: Optional[int] = None, steps: Optional[int] = None,
                 device: int = 0, stream=None, mem_budget_bytes: int = 0, ckpt_every: Optional[int] = None,
                 tape_windows: int = 0):
        import torch
        self._L = lib()
        self.w = w
        self.S = int(n_scenarios)
        net, dem, cfg = w.net, w.dem, w.cfg
        self.steps = int(steps if steps is not None else cfg.steps)
        cbs = int(cfg.count_bin_steps)
        self.n_count_bins = self.steps // cbs if cbs > 0 else 0
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        n, d, c, self._keep = _marshal(w, self.S, seeds, self.steps, ckpt_every, max_steps, record,
                                       mem_budget_bytes, tape_windows)
        h = C.c_void_p()
        rc = self._L.sim_create(C.byref(n), C.byref(d), C.byref(c), device, C.c_void_p(stream.cuda_stream),
                                C.byref(h))
        if rc != SIM_OK:
            raise SimError(rc, self._L.sim_last_error(None).decode())
        self._h = h
        for k, v in (params or {}).items():
            self.set_params(k, v)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.sim_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != SIM_OK:
            raise SimError(rc, self._L.sim_last_error(self._h).decode())

    # -- sizes -----------------------------------------------------------
    def n_per(self, group: str) -> int:
        if group == "rates":
            return self.w.net.n_origins * self.w.dem.n_rate_bins
        if group == "theta":
            return 1
        return self.w.net.n_links

    # -- control ----------------------------------------------------------
    def set_params(self, group: str, values):
        import torch
        n = self.n_per(group)
        if isinstance(values, torch.Tensor) and values.is_cuda:
            v = values.detach().to(torch.float32).reshape(-1).contiguous()
            if v.numel() == n:
                v = v.repeat(self.S)
            self._chk(self._L.sim_set_params(self._h, PARAMS[group], C.c_void_p(v.data_ptr()), v.numel(), 1))
            return
        v = np.asarray(values, np.float32).reshape(-1)
        if v.size == n:
            v = np.tile(v, self.S)
        v = np.ascontiguousarray(v)
        self._chk(self._L.sim_set_params(self._h, PARAMS[group], _p(v), v.size, 0))

    def get_params(self, group: str) -> np.ndarray:
        """Current values of a parameter group, [S x n] (sim_get_params)."""
        out = np.zeros((self.S, self.n_per(group)), np.float32)
        self._chk(self._L.sim_get_params(self._h, PARAMS[group], _p(out), out.size, 0))
        return out

    def optimize(self, groups, steps: Optional[int] = None, observed=None, loss: str = "counts",
                 target_detector: int = 0, target: float = 0.0, lr: float = 0.1, weight_decay: float = 1e-5,
                 betas=(0.9, 0.999), eps: float = 1e-8, max_iters: int = 200, patience: int = 20,
                 bounds: Optional[dict] = None, normalized: bool = False) -> dict:
        """Gradient-based calibration ("counts": mean squared count error against `observed`
        [det x bins]) or control ("cumulative": squared error of detector `target_detector`'s
        whole-horizon count against `target`) with AdamW, early stopping after `patience`
        iterations without improvement; the handle keeps the best parameters (sim_optimize).
        `bounds` maps group names to (lower, upper); `normalized` runs AdamW on each group's position in
        its box.  The result holds the gradient at the starting parameters ("first_grad")."""
        mask = 0
        for g in groups:
            mask |= 1 << PARAMS[g]
        lo = np.full(N_GROUPS, -np.inf, np.float32)
        hi = np.full(N_GROUPS, np.inf, np.float32)
        have = bool(bounds)
        defaults = {"free_speed": (0.5, 60.0), "jam_density": (1e-3, np.inf), "cost": (0.01, 1e4),
                    "rates": (0.0, 1e4), "cap_mult": (0.0, 1e4)}
        for g, (a, b) in defaults.items():
            lo[PARAMS[g]], hi[PARAMS[g]] = a, b
        for g, (a, b) in (bounds or {}).items():
            lo[PARAMS[g]], hi[PARAMS[g]] = a, b
        obs = None
        if loss == "counts":
            if observed is None:
                raise ValueError("calibration needs observed counts")
            obs = _f32(np.asarray(observed, np.float32).reshape(self.w.net.n_detectors, self.n_count_bins))
        elif loss != "cumulative":
            raise ValueError(loss)
        g0 = {g: np.zeros(self.n_per(g), np.float32) for g in groups}
        g0_arr = (C.c_void_p * N_GROUPS)()
        for g, a in g0.items():
            g0_arr[PARAMS[g]] = a.ctypes.data
        cfg = _OptConfig(mask, int(self.steps if steps is None else steps), int(max_iters), int(patience),
                         float(lr), float(weight_decay), float(betas[0]), float(betas[1]), float(eps),
                         SIM_LOSS_COUNTS_MSE if loss == "counts" else SIM_LOSS_CUMULATIVE, int(target_detector),
                         float(target), _p(lo) if have else None, _p(hi) if have else None, int(bool(normalized)),
                         C.cast(g0_arr, C.c_void_p))
        hist = np.full(int(max_iters), np.nan)
        res = _OptResult()
        self._chk(self._L.sim_optimize(self._h, C.byref(cfg), _p(obs), _p(hist), C.byref(res)))
        return {"iterations": res.iterations, "best_iter": res.best_iter, "first_loss": res.first_loss,
                "best_loss": res.best_loss, "seconds": res.seconds, "history": hist[:res.iterations],
                "first_grad": g0}

    def reset(self):
        self._chk(self._L.sim_reset(self._h))

    def place(self, agents, links, pos):
        a, l, p = _i32(agents), _i32(links), _f32(pos)
        self._chk(self._L.sim_place(self._h, len(a), _p(a), _p(l), _p(p)))

    def step(self, n: int = 1):
        self._chk(self._L.sim_rollout(self._h, int(n)))

    def rollout(self, T: Optional[int] = None):
        self.step(self.steps if T is None else T)
        return self

    @property
    def t(self) -> int:
        t = C.c_int32(0)
        self._chk(self._L.sim_time(self._h, C.byref(t)))
        return t.value

    # -- outputs ------------------------------------------------------------
    def observables(self):
        Dd, nb = self.w.net.n_detectors, self.n_count_bins
        cnt = np.zeros((self.S, Dd, nb), np.float32)
        ttt = np.zeros(self.S, np.float64)
        self._chk(self._L.sim_get_observables(self._h, _p(cnt), _p(ttt), 0))
        return cnt, ttt

    def observables_device(self):
        import torch
        Dd, nb = self.w.net.n_detectors, self.n_count_bins
        dev = torch.device("cuda", self.device)
        cnt = torch.zeros((self.S, Dd, nb), dtype=torch.float32, device=dev)
        ttt = torch.zeros(self.S, dtype=torch.float64, device=dev)
        self._chk(self._L.sim_get_observables(self._h, C.c_void_p(cnt.data_ptr()), C.c_void_p(ttt.data_ptr()), 1))
        return cnt, ttt

    def backward(self, gQ=None, gT=None, gx=None, groups=("free_speed", "jam_density", "rates")):
        S, net = self.S, self.w.net
        gQ = None if gQ is None else _f32(np.broadcast_to(np.asarray(gQ, np.float32),
                                                          (S, net.n_detectors, self.n_count_bins)))
        gT = None if gT is None else np.ascontiguousarray(np.broadcast_to(np.asarray(gT, np.float64), (S,)))
        gx = None if gx is None else _f32(np.asarray(gx, np.float32).reshape(S, -1))
        mask = 0
        bufs = {}
        arr = (C.c_void_p * N_GROUPS)()
        for g in groups:
            k = PARAMS[g]
            mask |= 1 << k
            bufs[g] = np.zeros((S, self.n_per(g)), np.float32)
            arr[k] = bufs[g].ctypes.data
        self._chk(self._L.sim_backward(self._h, _p(gQ), _p(gT), _p(gx), mask, arr, 0))
        return bufs

    def backward_device(self, gQ=None, gT=None, gx=None, groups=("free_speed", "jam_density", "rates")):
        import torch
        dev = torch.device("cuda", self.device)
        mask = 0
        out = {}
        arr = (C.c_void_p * N_GROUPS)()
        for g in groups:
            k = PARAMS[g]
            mask |= 1 << k
            out[g] = torch.zeros((self.S, self.n_per(g)), dtype=torch.float32, device=dev)
            arr[k] = out[g].data_ptr()
        ptr = lambda x: None if x is None else C.c_void_p(x.contiguous().data_ptr())
        self._chk(self._L.sim_backward(self._h, ptr(gQ), ptr(gT), ptr(gx), mask, arr, 1))
        return out

    def state(self):
        S, N = self.S, self.w.dem.n_agents
        st, lk, sq = (np.zeros((S, N), np.int32) for _ in range(3))
        ps = np.zeros((S, N), np.float32)
        ctr = np.zeros((S, 8), np.int64)
        self._chk(self._L.sim_get_state(self._h, _p(st), _p(lk), _p(ps), _p(sq), _p(ctr)))
        return {"status": st, "link": lk, "pos": ps, "seq": sq,
                "counters": [dict(zip(COUNTER_NAMES, c.tolist())) for c in ctr]}

    def vehicle_steps(self) -> np.ndarray:
        out = np.zeros(self.S, np.int64)
        self._chk(self._L.sim_get_stats(self._h, _p(out)))
        return out

    def link_state(self):
        S, L = self.S, self.w.net.n_links
        B = np.zeros((S, L), np.float64)
        E = np.zeros((S, L), np.int64)
        ns = np.zeros((S, L), np.int32)
        self._chk(self._L.sim_get_link_state(self._h, _p(B), _p(E), _p(ns)))
        return {"B": B, "E": E, "next_seq": ns}

    def dist_table(self):
        nd = C.c_int32(0)
        self._chk(self._L.sim_get_dist(self._h, None, C.byref(nd)))
        out = np.zeros((nd.value, self.w.net.n_nodes), np.float64)
        self._chk(self._L.sim_get_dist(self._h, _p(out), None))
        return out

    def philox(self, ctr, key):
        c = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
        k = np.ascontiguousarray(key, np.uint32).reshape(-1, 2)
        out = np.zeros_like(c)
        self._chk(self._L.sim_philox(self._h, c.shape[0], _p(c), _p(k), _p(out)))
        return out

    def gumbel_fast(self, words):
        w = np.ascontiguousarray(words, np.uint32).reshape(-1)
        out = np.zeros(w.shape, np.float32)
        self._chk(self._L.sim_gumbel_fast(self._h, w.size, _p(w), _p(out)))
        return out

    def segsort(self, seg, pos, seq, n_segments: int):
        """seg/pos/seq: torch device tensors; returns (perm, seg_off) device tensors."""
        import torch
        n = seg.numel()
        perm = torch.zeros(n, dtype=torch.int32, device=seg.device)
        off = torch.zeros(n_segments + 1, dtype=torch.int32, device=seg.device)
        self._chk(self._L.sim_segsort(self._h, n, n_segments, C.c_void_p(seg.data_ptr()), C.c_void_p(pos.data_ptr()),
                                      C.c_void_p(seq.data_ptr()), C.c_void_p(perm.data_ptr()),
                                      C.c_void_p(off.data_ptr())))
        return perm, off

    def segsort_noalloc(self, seg, pos, seq, n_segments: int, perm, seg_off, status=None):
        """Allocation-free sort into caller tensors perm [n] and seg_off [n_segments + 1] (int32, on the
        handle's device); status: optional int32 device tensor [1] that receives the overflow flag
        without waiting (sim_segsort_noalloc)."""
        n = seg.numel()
        st = None if status is None else C.c_void_p(status.data_ptr())
        self._chk(self._L.sim_segsort_noalloc(self._h, n, n_segments, C.c_void_p(seg.data_ptr()),
                                              C.c_void_p(pos.data_ptr()), C.c_void_p(seq.data_ptr()),
                                              C.c_void_p(perm.data_ptr()), C.c_void_p(seg_off.data_ptr()), st))

    def tie_log(self) -> np.ndarray:
        """Near-tie records of the forward since the last reset (sim_get_tie_log), int32 [n x 6]:
        (scenario, step, class, agent, link, decision); classes 0 route choice, 1 merge."""
        n = C.c_int64(0)
        self._chk(self._L.sim_get_tie_log(self._h, None, 0, C.byref(n)))
        k = min(n.value, 1 << 16)
        out = np.zeros((k, 6), np.int32)
        if k:
            self._chk(self._L.sim_get_tie_log(self._h, _p(out), k, C.byref(n)))
        return out

    def set_schedule(self, g_link: int, g_node: int, g_rev: int):
        self._chk(self._L.sim_set_schedule(self._h, g_link, g_node, g_rev))

    def schedule(self):
        a, b, c = C.c_int(0), C.c_int(0), C.c_int(0)
        self._chk(self._L.sim_get_schedule(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def full_state(self) -> bytes:
        """The whole simulation state as an opaque blob (sim_get_full_state)."""
        n = C.c_size_t()
        self._chk(self._L.sim_get_full_state(self._h, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._chk(self._L.sim_get_full_state(self._h, buf, n.value, C.byref(n)))
        return buf.raw

    def set_full_state(self, blob: bytes):
        self._chk(self._L.sim_set_full_state(self._h, blob, len(blob)))

    def autotune(self, probe_steps: int = 20, cache_path: Optional[str] = None, force: bool = False):
        """Pick and apply the fastest lane-group schedule for this shape from the
        current state (restored afterwards); returns (g_link, g_node, g_rev)."""
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        self._chk(self._L.sim_autotune(self._h, int(probe_steps), cache_path.encode() if cache_path else None,
                                       1 if force else 0, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def set_timing(self, on: bool = True):
        self._chk(self._L.sim_set_timing(self._h, int(on)))

    def timing(self, reset: bool = True):
        """(ms, launches) per kind: link, node, reverse (each launch's own wave stamps), copy, and
        link_ev, node_ev, reverse_ev (the same launches between HIP events on their stream)."""
        ms = np.zeros(7, np.float64)
        n = np.zeros(7, np.int64)
        self._chk(self._L.sim_get_timing(self._h, _p(ms), _p(n), 7, int(reset)))
        names = ("link", "node", "reverse", "copy", "link_ev", "node_ev", "reverse_ev")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(names)}


SRV_QUEUED, SRV_RUNNING, SRV_DONE, SRV_FAILED, SRV_CANCELLED = 0, 1, 2, 3, 4


def footprint(w, n_scenarios: int = 1, steps: Optional[int] = None, record: bool = False) -> int:
    """Device bytes sim_create would allocate for this workload (host-only)."""
    L = lib()
    T = int(steps if steps is not None else w.cfg.steps)
    n, d, c, keep = _marshal(w, n_scenarios, None, T, None, None, record, 0)
    out = C.c_size_t()
    rc = L.sim_footprint(C.byref(n), C.byref(d), C.byref(c), C.byref(out))
    if rc != SIM_OK:
        raise SimError(rc, "sim_footprint rejected the workload")
    return int(out.value)


class Server:
    """Continuous-batching server of forward rollouts (srv_* in sim.h).

    device = -1 selects the host-only executor (admission and failure logic
    without a GPU; observables are zero)."""

    def __init__(self, device: int = 0, mem_budget_bytes: int = 8 << 30, max_slots: int = 8, chunk_steps: int = 60):
        self._L = lib()
        h = C.c_void_p()
        rc = self._L.srv_create(int(device), int(mem_budget_bytes), int(max_slots), int(chunk_steps), C.byref(h))
        if rc != SIM_OK:
            raise SimError(rc, "srv_create failed")
        self._h = h
        self._meta = {}

    def submit(self, w, steps: Optional[int] = None, n_scenarios: int = 1, seeds: Optional[Sequence[int]] = None) -> int:
        T = int(steps if steps is not None else w.cfg.steps)
        n, d, c, keep = _marshal(w, n_scenarios, seeds, T, None, T, False, 0)
        t = C.c_int64()
        rc = self._L.srv_submit(self._h, C.byref(n), C.byref(d), C.byref(c), T, C.byref(t))
        if rc != SIM_OK:
            raise SimError(rc, "srv_submit failed")
        nb = T // int(w.cfg.count_bin_steps) if int(w.cfg.count_bin_steps) > 0 else 0
        self._meta[t.value] = (int(n_scenarios), int(w.net.n_detectors), nb)
        return t.value

    def poll(self, ticket: int) -> int:
        st = C.c_int()
        rc = self._L.srv_poll(self._h, ticket, C.byref(st))
        if rc != SIM_OK:
            raise SimError(rc, "unknown ticket")
        return st.value

    def wait(self, ticket: int, timeout_s: float = 600.0) -> int:
        st = C.c_int()
        rc = self._L.srv_wait(self._h, ticket, float(timeout_s), C.byref(st))
        if rc != SIM_OK:
            raise SimError(rc, "unknown ticket")
        return st.value

    def result(self, ticket: int):
        """(counts [S x det x bins], total travel time [S], vehicle-steps [S], latency s)."""
        S, D, nb = self._meta[ticket]
        counts = np.zeros((S, D, nb), np.float32)
        ttt = np.zeros(S, np.float64)
        vs = np.zeros(S, np.int64)
        lat = C.c_double()
        rc = self._L.srv_result(self._h, ticket, _p(counts), _p(ttt), _p(vs), C.byref(lat))
        if rc != SIM_OK:
            raise SimError(rc, self.error(ticket))
        return counts, ttt, vs, lat.value

    def error(self, ticket: int) -> str:
        return self._L.srv_error(self._h, ticket).decode()

    def cancel(self, ticket: int):
        self._L.srv_cancel(self._h, ticket)

    def stats(self) -> dict:
        p50, p99, vps = C.c_double(), C.c_double(), C.c_double()
        done, mr = C.c_int64(), C.c_int64()
        self._L.srv_stats(self._h, C.byref(p50), C.byref(p99), C.byref(vps), C.byref(done), C.byref(mr))
        return {"p50_s": p50.value, "p99_s": p99.value, "vehicle_steps_per_s": vps.value,
                "completed": done.value, "max_running": mr.value}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.srv_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def make_rollout_function():
    """torch.autograd.Function around one recorded rollout: forward sets the
    parameters and runs T steps, returning detector counts and total travel
    time; backward runs the checkpointed adjoint.  `rates`, `cap_mult`,
    `beta`, `cost` and `alpha` may be None (left as they are, no gradient);
    the last three take their gradient through the straight-through node
    model."""
    import torch

    optional = ("rates", "cap_mult", "beta", "cost", "alpha")

    class SimRollout(torch.autograd.Function):
        @staticmethod
        def forward(ctx, sim: Simulator, T: int, free_speed, jam_density, rates=None, cap_mult=None,
                    beta=None, cost=None, alpha=None):
            sim.set_params("free_speed", free_speed)
            sim.set_params("jam_density", jam_density)
            given = {"rates": rates, "cap_mult": cap_mult, "beta": beta, "cost": cost, "alpha": alpha}
            ctx.groups = ("free_speed", "jam_density")
            ctx.shapes = {"free_speed": free_speed.shape, "jam_density": jam_density.shape}
            for name in optional:
                v = given[name]
                if v is not None and v.numel() > 0:
                    sim.set_params(name, v)
                    ctx.groups += (name,)
                    ctx.shapes[name] = v.shape
            sim.reset()
            sim.step(T)
            counts, ttt = sim.observables_device()
            ctx.sim = sim
            return counts, ttt

        @staticmethod
        def backward(ctx, g_counts, g_ttt):
            g = ctx.sim.backward_device(gQ=g_counts.float() if g_counts is not None else None,
                                        gT=g_ttt.double() if g_ttt is not None else None, groups=ctx.groups)

            def shaped(name):   # [S, n] -> the input's shape; one set shared by all scenarios sums them
                if name not in g:
                    return None
                x, shp = g[name], ctx.shapes[name]
                return (x if x.numel() == shp.numel() else x.sum(0)).reshape(shp)
            return (None, None, shaped("free_speed"), shaped("jam_density")) + tuple(shaped(n) for n in optional)

    return SimRollout
