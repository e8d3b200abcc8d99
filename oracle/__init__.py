"""Python handle on the plain-C reference oracle.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the simulator itself never does.

`build()` compiles `oracle.c` twice with gcc: `liboracle_f32.so` carries
agent positions in float (the precision that decides the integer state on the
GPU) and `liboracle_f64.so` carries them in double.  Everything else in both
is double.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
ST_WAIT, ST_QUEUED, ST_ON, ST_EXITED = 0, 1, 2, 3
TIE_CHOICE, TIE_MERGE, TIE_ARRIVE, TIE_VACANT, TIE_DETECT = 0, 1, 2, 3, 4
COUNTER_NAMES = ("released", "departed", "on_net", "exited", "transfers", "ties", "stuck", "order_viol")


def lib_path(variant: str = "f32") -> str:
    return os.path.join(_HERE, f"liboracle_{variant}.so")


def build(force: bool = True) -> None:
    for variant, flags in (("f32", []), ("f64", ["-DORC_POS_F64"])):
        out = lib_path(variant)
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
            continue
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", *flags, "-o", out + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


class _Inputs(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int32), ("n_links", C.c_int32),
        ("tail", C.c_void_p), ("head", C.c_void_p), ("lanes", C.c_void_p),
        ("length", C.c_void_p), ("free_speed", C.c_void_p), ("jam_density", C.c_void_p),
        ("capacity", C.c_void_p), ("beta", C.c_void_p), ("alpha", C.c_void_p), ("cost", C.c_void_p),
        ("cap_mult", C.c_void_p), ("route_speed", C.c_void_p),
        ("n_origins", C.c_int32), ("origin_node", C.c_void_p),
        ("n_detectors", C.c_int32), ("detector_link", C.c_void_p), ("detector_pos", C.c_void_p),
        ("n_agents", C.c_int32), ("agent_origin", C.c_void_p), ("agent_dest", C.c_void_p),
        ("ready_time", C.c_void_p),
        ("n_rate_bins", C.c_int32), ("rate_bin_s", C.c_double), ("rates", C.c_void_p),
        ("dt", C.c_double), ("platoon", C.c_int32),
        ("gumbel_tau", C.c_double), ("dest_logit_coef", C.c_double), ("big_m", C.c_double),
        ("seed", C.c_uint64),
        ("count_bin_steps", C.c_int32), ("n_count_bins", C.c_int32), ("allow_uturn", C.c_int32),
    ]


_LIBS = {}


def _lib(variant: str):
    if variant in _LIBS:
        return _LIBS[variant]
    p = lib_path(variant)
    if not os.path.exists(p) or os.path.getmtime(p) < os.path.getmtime(_SRC):
        build(force=True)
    L = C.CDLL(p)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.orc_create.restype = vp
    L.orc_create.argtypes = [C.POINTER(_Inputs)]
    L.orc_destroy.argtypes = [vp]
    L.orc_set_logging.argtypes = [vp, C.c_int]
    L.orc_place.argtypes = [vp, i32, vp, vp, vp]
    L.orc_step.argtypes = [vp]
    L.orc_rollout.argtypes = [vp, i32]
    L.orc_get_state.argtypes = [vp, vp, vp, vp, vp]
    L.orc_get_link_state.argtypes = [vp, vp, vp, vp]
    L.orc_get_counters.argtypes = [vp, vp]
    L.orc_get_counts.argtypes = [vp, vp, vp]
    L.orc_n_dest.argtypes = [vp]
    L.orc_n_dest.restype = i32
    L.orc_get_dist.argtypes = [vp, vp]
    L.orc_get_origin_state.argtypes = [vp, vp, vp, vp]
    L.orc_time.argtypes = [vp]
    L.orc_time.restype = i32
    L.orc_frozen_eval.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int, vp, vp, vp]
    L.orc_frozen_eval.restype = C.c_int
    L.orc_backward.argtypes = [vp, vp, dbl, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int]
    L.orc_backward.restype = C.c_int
    L.orc_philox4x32_10.argtypes = [vp, vp, vp]
    L.orc_gumbel.argtypes = [C.c_uint64, i32, i32, i32, i32]
    L.orc_gumbel.restype = dbl
    L.orc_uniform.argtypes = [C.c_uint64, i32, i32, i32, i32]
    L.orc_uniform.restype = dbl
    L.orc_tie_count.argtypes = [vp]
    L.orc_tie_count.restype = i64
    L.orc_tie_log.argtypes = [vp, vp]
    L.orc_tie_stats.argtypes = [vp, vp, vp, vp]
    L.orc_adopt_ties.argtypes = [vp, vp, i64]
    L.orc_set_tie_tolerance.argtypes = [vp, C.c_double]
    L.orc_state_size.argtypes = [vp]
    L.orc_state_size.restype = i64
    L.orc_export_state.argtypes = [vp, vp]
    L.orc_import_state.argtypes = [vp, vp, i64]
    L.orc_import_state.restype = C.c_int
    _LIBS[variant] = L
    return L


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def philox(ctr, key, variant: str = "f32") -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    _lib(variant).orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def gumbel(seed: int, agent: int, step: int, purpose: int, word: int) -> float:
    return _lib("f32").orc_gumbel(seed, agent, step, purpose, word)


def uniform(seed: int, agent: int, step: int, purpose: int, word: int) -> float:
    return _lib("f32").orc_uniform(seed, agent, step, purpose, word)


class Oracle:
    """One simulation instance of the oracle (a single scenario).

    Parameters default to the workload's values; `params` may override
    free_speed, jam_density, capacity, beta, alpha, cost, cap_mult (per link)
    and rates (per origin x bin), and `seed` the Philox key."""

    def __init__(self, w, params: Optional[dict] = None, seed: Optional[int] = None,
                 variant: str = "f32", log: bool = False, steps: Optional[int] = None,
                 adopt: Optional[np.ndarray] = None, tie_tolerance: Optional[float] = None):
        self.w = w
        self._L = _lib(variant)
        net, dem, cfg = w.net, w.dem, w.cfg
        p = dict(params or {})
        f32 = lambda a: np.ascontiguousarray(a, np.float32)
        i32 = lambda a: np.ascontiguousarray(a, np.int32)
        self._keep = {
            "tail": i32(net.tail), "head": i32(net.head), "lanes": i32(net.lanes),
            "length": f32(net.length), "free_speed": f32(p.get("free_speed", net.free_speed)),
            "jam_density": f32(p.get("jam_density", net.jam_density)),
            "capacity": f32(p.get("capacity", net.capacity)),
            "beta": f32(p.get("beta", net.beta)), "alpha": f32(p.get("alpha", net.alpha)),
            "cost": f32(p.get("cost", net.cost)),
            "cap_mult": f32(p.get("cap_mult", np.ones(net.n_links))),
            "route_speed": f32(net.free_speed),
            "origin_node": i32(net.origin_node), "detector_link": i32(net.detector_link),
            "detector_pos": f32(net.detector_pos),
            "agent_origin": i32(dem.agent_origin), "agent_dest": i32(dem.agent_dest),
        }
        if dem.ready_time is not None:
            self._keep["ready_time"] = f32(dem.ready_time)
            rates = None
        else:
            rates = f32(p.get("rates", dem.rates))
            self._keep["rates"] = rates
        self.steps = int(steps if steps is not None else cfg.steps)
        cbs = int(cfg.count_bin_steps)
        self.n_count_bins = self.steps // cbs if cbs > 0 else 0
        if rates is not None:
            k = dem.rate_bin_s / cfg.dt
            if abs(k - round(k)) > 1e-9:
                raise ValueError("rate bins must be a whole number of steps")
        K = self._keep
        ins = _Inputs(
            n_nodes=net.n_nodes, n_links=net.n_links,
            tail=_ptr(K["tail"]), head=_ptr(K["head"]), lanes=_ptr(K["lanes"]),
            length=_ptr(K["length"]), free_speed=_ptr(K["free_speed"]),
            jam_density=_ptr(K["jam_density"]), capacity=_ptr(K["capacity"]),
            beta=_ptr(K["beta"]), alpha=_ptr(K["alpha"]), cost=_ptr(K["cost"]),
            cap_mult=_ptr(K["cap_mult"]), route_speed=_ptr(K["route_speed"]),
            n_origins=net.n_origins, origin_node=_ptr(K["origin_node"]),
            n_detectors=net.n_detectors, detector_link=_ptr(K["detector_link"]),
            detector_pos=_ptr(K["detector_pos"]),
            n_agents=dem.n_agents, agent_origin=_ptr(K["agent_origin"]), agent_dest=_ptr(K["agent_dest"]),
            ready_time=_ptr(K.get("ready_time")),
            n_rate_bins=dem.n_rate_bins, rate_bin_s=float(dem.rate_bin_s), rates=_ptr(K.get("rates")),
            dt=float(cfg.dt), platoon=int(cfg.platoon), gumbel_tau=float(cfg.gumbel_tau),
            dest_logit_coef=float(cfg.dest_logit_coef), big_m=float(cfg.big_m),
            seed=int(cfg.seed if seed is None else seed) & (2**64 - 1),
            count_bin_steps=cbs, n_count_bins=self.n_count_bins, allow_uturn=int(cfg.allow_uturn))
        self._ins = ins
        self._h = self._L.orc_create(C.byref(ins))
        if log:
            self._L.orc_set_logging(self._h, 1)
        if tie_tolerance is not None:
            self._L.orc_set_tie_tolerance(self._h, float(tie_tolerance))
        if adopt is not None:
            a = np.ascontiguousarray(adopt, np.int32).reshape(-1, 5)
            self._L.orc_adopt_ties(self._h, _ptr(a), len(a))

    @staticmethod
    def tie_log_from_library(records: np.ndarray, scenario: int = 0) -> np.ndarray:
        """A library near-tie log (rows scenario, step, class, agent, link, decision) as this
        oracle's adoptable log (rows step, class, id, aux, decision) for one scenario."""
        r = np.asarray(records, np.int32).reshape(-1, 6)
        return np.ascontiguousarray(r[r[:, 0] == scenario][:, 1:])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.orc_destroy(h)
            self._h = None

    # -- forward -----------------------------------------------------------
    def place(self, agents, links, pos):
        a = np.ascontiguousarray(agents, np.int32)
        l = np.ascontiguousarray(links, np.int32)
        p = np.ascontiguousarray(pos, np.float32)
        if self._L.orc_place(self._h, len(a), _ptr(a), _ptr(l), _ptr(p)) != 0:
            raise RuntimeError("place is only allowed at t = 0")

    def step(self, n: int = 1):
        self._L.orc_rollout(self._h, int(n))

    def run(self, T: Optional[int] = None):
        self.step(self.steps if T is None else T)
        return self

    @property
    def t(self) -> int:
        return int(self._L.orc_time(self._h))

    def state(self):
        n = self.w.dem.n_agents
        st, lk, sq = (np.zeros(n, np.int32) for _ in range(3))
        ps = np.zeros(n, np.float64)
        self._L.orc_get_state(self._h, _ptr(st), _ptr(lk), _ptr(ps), _ptr(sq))
        return {"status": st, "link": lk, "pos": ps, "seq": sq}

    def link_state(self):
        L = self.w.net.n_links
        B = np.zeros(L, np.float64)
        E = np.zeros(L, np.int64)
        ns = np.zeros(L, np.int32)
        self._L.orc_get_link_state(self._h, _ptr(B), _ptr(E), _ptr(ns))
        return {"B": B, "E": E, "next_seq": ns}

    def origin_state(self):
        O = self.w.net.n_origins
        D = np.zeros(O, np.float64)
        rel = np.zeros(O, np.int32)
        dep = np.zeros(O, np.int32)
        self._L.orc_get_origin_state(self._h, _ptr(D), _ptr(rel), _ptr(dep))
        return {"D": D, "released": rel, "departed": dep}

    def counters(self) -> dict:
        c = np.zeros(8, np.int64)
        self._L.orc_get_counters(self._h, _ptr(c))
        return dict(zip(COUNTER_NAMES, c.tolist()))

    def counts(self):
        Dd = self.w.net.n_detectors
        out = np.zeros((Dd, max(self.n_count_bins, 0)), np.float64)
        ttt = C.c_double(0.0)
        self._L.orc_get_counts(self._h, _ptr(out), C.byref(ttt))
        return out, float(ttt.value)

    def tie_log(self) -> np.ndarray:
        """Near-tie events so far, [n x 5] int32 rows (t, class, id, aux, decision); classes
        TIE_CHOICE, TIE_MERGE, TIE_ARRIVE, TIE_VACANT, TIE_DETECT."""
        n = int(self._L.orc_tie_count(self._h))
        out = np.zeros((n, 5), np.int32)
        if n:
            self._L.orc_tie_log(self._h, _ptr(out))
        return out

    def export_state(self) -> bytes:
        """The whole forward state as this oracle's own blob (orc_export_state)."""
        n = int(self._L.orc_state_size(self._h))
        buf = C.create_string_buffer(n)
        self._L.orc_export_state(self._h, buf)
        return buf.raw

    def import_state(self, blob: bytes):
        """Continue from another oracle's exported state (same inputs and placed agents)."""
        buf = C.create_string_buffer(bytes(blob), len(blob))
        if self._L.orc_import_state(self._h, buf, len(blob)) != 0:
            raise ValueError("state blob does not match this oracle's inputs")
        return self

    def tie_stats(self) -> dict:
        """Decisions taken from the adopted log, near ties it did not hold, and adopted
        decisions that differ from this run's own."""
        a, u, f = C.c_int64(0), C.c_int64(0), C.c_int64(0)
        self._L.orc_tie_stats(self._h, C.byref(a), C.byref(u), C.byref(f))
        return {"adopted": int(a.value), "unmatched": int(u.value), "flipped": int(f.value)}

    def dist_table(self):
        nd = self._L.orc_n_dest(self._h)
        out = np.zeros((nd, self.w.net.n_nodes), np.float64)
        self._L.orc_get_dist(self._h, _ptr(out))
        return out

    # -- frozen surrogate and adjoint -------------------------------------
    def frozen(self, u=None, kappa=None, rates=None, cap_mult=None, beta=None, cost=None, alpha=None, theta=None,
               record_base: bool = False):
        f64 = lambda a: None if a is None else np.ascontiguousarray(a, np.float64)
        u, kappa, rates, cap_mult = f64(u), f64(kappa), f64(rates), f64(cap_mult)
        beta, cost, alpha = f64(beta), f64(cost), f64(alpha)
        theta = None if theta is None else np.ascontiguousarray(np.reshape(theta, (1,)), np.float64)
        Dd = self.w.net.n_detectors
        cnt = np.zeros((Dd, self.n_count_bins), np.float64)
        ttt = C.c_double(0.0)
        pos = np.zeros(self.w.dem.n_agents, np.float64)
        rc = self._L.orc_frozen_eval(self._h, _ptr(u), _ptr(kappa), _ptr(rates), _ptr(cap_mult), _ptr(beta),
                                     _ptr(cost), _ptr(alpha), _ptr(theta), int(record_base),
                                     _ptr(cnt), C.byref(ttt), _ptr(pos))
        if rc != 0:
            raise RuntimeError(f"frozen_eval failed ({rc}); run with log=True first")
        return cnt, float(ttt.value), pos

    def backward(self, gQ=None, gT: float = 0.0, gx=None, transfer_graft: bool = True):
        net = self.w.net
        gQ = None if gQ is None else np.ascontiguousarray(gQ, np.float64)
        gx = None if gx is None else np.ascontiguousarray(gx, np.float64)
        g_u = np.zeros(net.n_links)
        g_k = np.zeros(net.n_links)
        nb = self.w.dem.n_rate_bins
        g_r = np.zeros((net.n_origins, max(nb, 1)))
        g_m = np.zeros(net.n_links)
        g_b, g_c, g_a, g_t = np.zeros(net.n_links), np.zeros(net.n_links), np.zeros(net.n_links), np.zeros(1)
        rc = self._L.orc_backward(self._h, _ptr(gQ), float(gT), _ptr(gx), _ptr(g_u), _ptr(g_k), _ptr(g_r),
                                   _ptr(g_m), _ptr(g_b), _ptr(g_c), _ptr(g_a), _ptr(g_t), 0 if transfer_graft else 1)
        if rc != 0:
            raise RuntimeError("backward needs a logged rollout")
        return {"free_speed": g_u, "jam_density": g_k, "rates": g_r[:, :nb] if nb else g_r[:, :0],
                "cap_mult": g_m, "beta": g_b, "cost": g_c, "alpha": g_a, "theta": g_t}
