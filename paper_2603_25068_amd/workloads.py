"""Seeded synthetic inputs: road networks, agent pools, demand and detectors.

This module only draws and arranges input data.  It holds none of the
simulator's arithmetic (no car-following, no choice, no shortest paths), so
both the FP64 oracle and the HIP path can consume what it produces without
sharing any of the method.

The paper calibrates on TNTP networks (Sioux Falls, Chicago Sketch; Methods,
"Experimental setting") that are not available here.  Every workload below is
a synthetic stand-in of the same kind: a directed road network with per-link
free speed u, jam density kappa, merge priority alpha, route-choice weight
beta and cost c (Methods, "Experimental setting"; SI-A/SI-B), an agent pool
that departs from origin queues (the paper's virtual inflow links), and
midpoint count detectors (SI-D).

Data contract (all numpy, C-contiguous):
  network: n_nodes, tail/head/lanes int32[L], length/free_speed/jam_density/
           capacity/beta/alpha/cost float32[L], origin_node int32[O],
           detector_link int32[D], detector_pos float32[D]
  demand:  agent_origin int32[N] (origin index), agent_dest int32[N] (node),
           either ready_time float32[N] (fixed departure times) or
           rates float32[O, B] + rate_bin_s (departure-rate mode)
  config:  dt, platoon, gumbel_tau, dest_logit_coef, big_m, seed,
           ckpt_every, count_bin_steps, allow_uturn, steps
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

# Link defaults shared by the grid and metro generators.
JAM_DENSITY_PER_LANE = 0.2      # veh/m/lane -> jam spacing 5 m (paper range 0.18-0.22)
CAPACITY_PER_LANE = 0.5         # veh/s/lane
SPEED_CHOICES = (11.1, 13.9, 16.7)


@dataclass
class Network:
    n_nodes: int
    tail: np.ndarray
    head: np.ndarray
    lanes: np.ndarray
    length: np.ndarray
    free_speed: np.ndarray
    jam_density: np.ndarray
    capacity: np.ndarray
    beta: np.ndarray
    alpha: np.ndarray
    cost: np.ndarray
    origin_node: np.ndarray
    detector_link: np.ndarray
    detector_pos: np.ndarray
    node_xy: Optional[np.ndarray] = None

    @property
    def n_links(self) -> int:
        return int(self.tail.shape[0])

    @property
    def n_origins(self) -> int:
        return int(self.origin_node.shape[0])

    @property
    def n_detectors(self) -> int:
        return int(self.detector_link.shape[0])


@dataclass
class Demand:
    agent_origin: np.ndarray
    agent_dest: np.ndarray
    ready_time: Optional[np.ndarray] = None
    rates: Optional[np.ndarray] = None
    rate_bin_s: float = 300.0

    @property
    def n_agents(self) -> int:
        return int(self.agent_origin.shape[0])

    @property
    def n_rate_bins(self) -> int:
        return 0 if self.rates is None else int(self.rates.shape[1])


@dataclass
class Config:
    dt: float = 1.0
    platoon: int = 1
    gumbel_tau: float = 0.5
    dest_logit_coef: float = 0.1
    big_m: float = 99999.0
    seed: int = 0
    ckpt_every: int = 60
    count_bin_steps: int = 300
    allow_uturn: int = 1
    steps: int = 900


@dataclass
class Workload:
    name: str
    net: Network
    dem: Demand
    cfg: Config
    extra: dict = field(default_factory=dict)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _links_from_roads(roads: np.ndarray):
    """Each undirected road (a, b) becomes the two directed links a->b, b->a
    (road k -> links 2k and 2k+1), so both directions share the road's draws."""
    tail = np.empty(2 * len(roads), np.int64)
    head = np.empty(2 * len(roads), np.int64)
    tail[0::2], head[0::2] = roads[:, 0], roads[:, 1]
    tail[1::2], head[1::2] = roads[:, 1], roads[:, 0]
    return tail, head


def make_network(n_nodes, roads, length, lanes, speed, *, origin_node, n_detectors,
                 rng, node_xy=None, beta=None, alpha=None, cost=None) -> Network:
    """Assemble a Network from per-road draws (duplicated to both directions)."""
    tail, head = _links_from_roads(np.asarray(roads))
    L = len(tail)
    rep = lambda v: np.repeat(np.asarray(v), 2)
    length = rep(length)
    lanes = rep(lanes)
    speed = rep(speed)
    if n_detectors > 0:
        det = np.sort(rng.choice(L, size=min(n_detectors, L), replace=False))
    else:
        det = np.zeros(0, np.int64)
    return Network(
        n_nodes=int(n_nodes), tail=_i32(tail), head=_i32(head), lanes=_i32(lanes),
        length=_f32(length), free_speed=_f32(speed),
        jam_density=_f32(np.full(L, JAM_DENSITY_PER_LANE)),
        capacity=_f32(np.full(L, CAPACITY_PER_LANE)),
        beta=_f32(np.zeros(L) if beta is None else beta),
        alpha=_f32(np.ones(L) if alpha is None else alpha),
        cost=_f32(np.ones(L) if cost is None else cost),
        origin_node=_i32(origin_node), detector_link=_i32(det),
        detector_pos=_f32(length[det] * np.float32(0.5)),
        node_xy=node_xy)


def grid_roads(nx: int, ny: int) -> np.ndarray:
    """Undirected roads of an nx-by-ny lattice; node id = r*nx + c."""
    roads = []
    for r in range(ny):
        for c in range(nx):
            v = r * nx + c
            if c + 1 < nx:
                roads.append((v, v + 1))
            if r + 1 < ny:
                roads.append((v, v + nx))
    return np.asarray(roads, np.int64)


def boundary_nodes(nx: int, ny: int) -> list[int]:
    """Boundary nodes of the lattice, each listed once, clockwise from (0,0)."""
    out = []
    out += [c for c in range(nx)]
    out += [r * nx + nx - 1 for r in range(1, ny)]
    out += [(ny - 1) * nx + c for c in range(nx - 2, -1, -1)]
    out += [r * nx for r in range(ny - 2, 0, -1)]
    return out


def _side_of(v: int, nx: int, ny: int) -> set:
    r, c = divmod(v, nx)
    s = set()
    if r == 0:
        s.add("S")
    if r == ny - 1:
        s.add("N")
    if c == 0:
        s.add("W")
    if c == nx - 1:
        s.add("E")
    return s


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

def small_grid_fixed(seed: int = 0) -> Workload:
    """Plain forward, FP64-oracle sized: 4x4 lattice, 48 directed links of
    200 m, 2 lanes, 13.9 m/s, 0.5 veh/s/lane; 1,000 agents over 12 boundary
    origin/destination pairs (point reflection), departures U[0, 600) s;
    Gumbel tau 0.5, destination logit -0.1 x free-flow time; dt 1 s, 900 steps."""
    rng = np.random.default_rng(10 * 0 + 2)
    nx = ny = 4
    roads = grid_roads(nx, ny)
    R = len(roads)
    bnd = boundary_nodes(nx, ny)
    net = make_network(nx * ny, roads, np.full(R, 200.0), np.full(R, 2), np.full(R, 13.9),
                       origin_node=bnd, n_detectors=0, rng=rng)
    # detectors on every link so counts are observed everywhere
    net.detector_link = _i32(np.arange(net.n_links))
    net.detector_pos = _f32(net.length * np.float32(0.5))
    n = 1000
    o = np.arange(n) % len(bnd)
    dest = []
    for k in o:
        r, c = divmod(bnd[k], nx)
        dest.append((ny - 1 - r) * nx + (nx - 1 - c))
    ready = rng.uniform(0.0, 600.0, size=n)
    dem = Demand(agent_origin=_i32(o), agent_dest=_i32(dest), ready_time=_f32(ready))
    cfg = Config(dt=1.0, gumbel_tau=0.5, dest_logit_coef=0.1, seed=seed, steps=900,
                 count_bin_steps=300)
    return Workload("grid4x4_1k_fixed", net, dem, cfg)


def grid_rates(nx: int = 32, ny: int = 32, n_agents: int = 50_000, n_detectors: int = 400,
               bins: int = 6, bin_s: float = 300.0, steps: int = 1800, seed: int = 2,
               rate_mode: str = "eval", lanes_max: int = 3) -> Workload:
    """Forward+adjoint workload: 32x32 lattice (3,968 links), lengths
    U[100, 500] m, 1-3 lanes, speeds in {11.1, 13.9, 16.7} m/s; 128 origin
    queues (boundary nodes, corners twice); 50k agents round-robin over the
    origins; departure rates per (origin, 5-min bin), ground truth
    lognormal(-3, 0.5) veh/s, evaluated at the mean exp(-2.875); 400 midpoint
    detectors; 1,800 steps of 1 s."""
    k = seed
    rng_net = np.random.default_rng(10 * k + 1)
    rng_dem = np.random.default_rng(10 * k + 2)
    rng_true = np.random.default_rng(10 * k + 3)
    rng_det = np.random.default_rng(10 * k + 4)
    roads = grid_roads(nx, ny)
    R = len(roads)
    length = rng_net.uniform(100.0, 500.0, R)
    lanes = rng_net.integers(1, lanes_max + 1, R)
    speed = rng_net.choice(np.asarray(SPEED_CHOICES), R)
    bnd = boundary_nodes(nx, ny)
    corners = [0, nx - 1, nx * ny - 1, (ny - 1) * nx]
    origin_nodes = bnd + corners
    net = make_network(nx * ny, roads, length, lanes, speed, origin_node=origin_nodes,
                       n_detectors=n_detectors, rng=rng_det)
    O = len(origin_nodes)
    o = np.arange(n_agents) % O
    # destination: a boundary node on a side the origin is not on
    sides = [_side_of(v, nx, ny) for v in bnd]
    dest = np.empty(n_agents, np.int64)
    for i in range(n_agents):
        ov = origin_nodes[o[i]]
        s0 = _side_of(ov, nx, ny)
        while True:
            d = bnd[rng_dem.integers(len(bnd))]
            if not (_side_of(d, nx, ny) & s0) and d != ov:
                break
        dest[i] = d
    theta_true = rng_true.lognormal(-3.0, 0.5, size=(O, bins))
    rates = np.full((O, bins), np.exp(-2.875)) if rate_mode == "eval" else theta_true
    dem = Demand(agent_origin=_i32(o), agent_dest=_i32(dest), rates=_f32(rates), rate_bin_s=bin_s)
    cfg = Config(dt=1.0, gumbel_tau=0.5, dest_logit_coef=0.1, seed=k, steps=steps,
                 count_bin_steps=300, ckpt_every=60)
    return Workload(f"grid{nx}x{ny}_{n_agents//1000}k_rates", net, dem, cfg,
                    extra={"theta_true": _f32(theta_true), "observed_seed": 1000 + k})


def metro_roads(n_nodes: int, n_roads: int, rng):
    """Planar metro-like road graph: Delaunay triangulation of uniform points,
    its Euclidean minimum spanning tree, then the shortest remaining Delaunay
    edges until n_roads roads exist."""
    from scipy.spatial import Delaunay
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree

    xy = rng.uniform(0.0, 1.0, size=(n_nodes, 2))
    tri = Delaunay(xy)
    s = tri.simplices
    e = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [2, 0]]])
    e = np.sort(e, axis=1)
    e = np.unique(e, axis=0)
    w = np.linalg.norm(xy[e[:, 0]] - xy[e[:, 1]], axis=1)
    g = coo_matrix((w, (e[:, 0], e[:, 1])), shape=(n_nodes, n_nodes)).tocsr()
    mst = minimum_spanning_tree(g).tocoo()
    in_mst = set(zip(np.minimum(mst.row, mst.col).tolist(), np.maximum(mst.row, mst.col).tolist()))
    chosen = [(a, b) for a, b in in_mst]
    order = np.argsort(w, kind="stable")
    need = n_roads - len(chosen)
    for idx in order:
        if need <= 0:
            break
        a, b = int(e[idx, 0]), int(e[idx, 1])
        if (a, b) in in_mst:
            continue
        chosen.append((a, b))
        need -= 1
    roads = np.asarray(sorted(chosen), np.int64)
    return xy, roads


def metro(n_nodes: int = 12_000, n_roads: int = 17_500, n_agents: int = 1_000_000,
          zones_side: int = 32, bins: int = 10, bin_s: float = 180.0,
          n_detectors: int = 2000, steps: int = 1800, seed: int = 3,
          rate_mode: str = "eval", mean_rate: Optional[float] = None) -> Workload:
    """Synthetic metro: Delaunay-based planar network (12k nodes, ~35k directed
    links), lengths lognormal with mean 250 m, 1-3 lanes, speeds as the grid;
    zones = cells of a zones_side^2 raster, each zone's origin and destination
    node is the node nearest the cell centre; departure rates per
    (zone, 3-min bin) lognormal(sigma 0.5) with mean chosen so that the
    expected departures equal the pool; pool split over zones in proportion to
    the ground-truth expected demand; destination zone uniform over the other
    zones; 2,000 midpoint detectors."""
    k = seed
    rng_net = np.random.default_rng(10 * k + 1)
    rng_dem = np.random.default_rng(10 * k + 2)
    rng_true = np.random.default_rng(10 * k + 3)
    rng_det = np.random.default_rng(10 * k + 4)
    xy, roads = metro_roads(n_nodes, n_roads, rng_net)
    R = len(roads)
    sigma = 0.5
    length = rng_net.lognormal(np.log(250.0) - sigma * sigma / 2, sigma, R)
    length = np.maximum(length, 20.0)
    lanes = rng_net.integers(1, 4, R)
    speed = rng_net.choice(np.asarray(SPEED_CHOICES), R)
    Z = zones_side * zones_side
    centres = (np.stack(np.meshgrid(np.arange(zones_side), np.arange(zones_side), indexing="ij"),
                        -1).reshape(-1, 2) + 0.5) / zones_side
    used = set()
    zone_node = []
    for c in centres:
        d = np.linalg.norm(xy - c, axis=1)
        for v in np.argsort(d):
            if int(v) not in used:
                used.add(int(v))
                zone_node.append(int(v))
                break
    net = make_network(n_nodes, roads, length, lanes, speed, origin_node=zone_node,
                       n_detectors=n_detectors, rng=rng_det, node_xy=xy.astype(np.float32))
    horizon = bins * bin_s
    if mean_rate is None:
        mean_rate = n_agents / (Z * horizon)
    mu = np.log(mean_rate) - sigma * sigma / 2
    theta_true = rng_true.lognormal(mu, sigma, size=(Z, bins))
    expect = theta_true.sum(1)
    pool = np.floor(n_agents * expect / expect.sum()).astype(np.int64)
    pool[: n_agents - pool.sum()] += 1
    o = np.repeat(np.arange(Z), pool)
    dz = rng_dem.integers(0, Z - 1, size=n_agents)
    dz = dz + (dz >= o)          # uniform over the other zones
    dest = np.asarray(zone_node)[dz]
    rates = np.full((Z, bins), mean_rate) if rate_mode == "eval" else theta_true
    dem = Demand(agent_origin=_i32(o), agent_dest=_i32(dest), rates=_f32(rates), rate_bin_s=bin_s)
    cfg = Config(dt=1.0, gumbel_tau=0.5, dest_logit_coef=0.1, seed=k, steps=steps,
                 count_bin_steps=300, ckpt_every=60)
    return Workload(f"metro{n_nodes//1000}k_{n_agents//1000}k", net, dem, cfg,
                    extra={"theta_true": _f32(theta_true), "zone_node": _i32(zone_node)})


# Ranges the paper samples its ground-truth per-link parameters from (Methods, "Experimental setting").
PAPER_RANGES = {"free_speed": (13.9, 22.2), "jam_density": (0.18, 0.22), "beta": (0.0, 5.0), "alpha": (0.01, 5.0)}


def sioux_like(seed: int = 7, n_agents: int = 20_000, steps: int = 1800, n_inter: int = 24, n_roads: int = 38,
               side_m: float = 8000.0) -> Workload:
    """A stand-in of the paper's per-link calibration network (Methods,
    "Experimental setting": a TNTP network of 24 intersections whose nodes
    each keep either a virtual inflow or a virtual outflow link, 48 nodes and
    100 links in all, 20,000 vehicles spread evenly over the inflow links).
    Here: 24 uniform points on an 8 km square, the Delaunay MST plus the
    shortest remaining edges up to 38 two-way roads (76 links, length = the
    distance), and one 200 m virtual link per intersection, half of them
    inflow (an origin queue at its outer node) and half outflow (a
    destination); agents spread evenly over the origins, all ready at t = 0,
    each bound to a uniformly drawn destination; ground-truth u, kappa, beta,
    alpha per link drawn uniformly from the paper's ranges, cost 1; a midpoint
    detector on every link, 5-min counts."""
    k = seed
    rng_net = np.random.default_rng(10 * k + 1)
    rng_dem = np.random.default_rng(10 * k + 2)
    rng_true = np.random.default_rng(10 * k + 3)
    xy, roads = metro_roads(n_inter, n_roads, rng_net)
    tail, head = _links_from_roads(roads)
    length = np.linalg.norm(xy[tail] - xy[head], axis=1) * side_m
    kind = rng_net.permutation(np.arange(n_inter) % 2)          # 0: inflow, 1: outflow
    virt = np.arange(n_inter) + n_inter                           # outer node of each intersection
    vt = np.where(kind == 0, virt, np.arange(n_inter))
    vh = np.where(kind == 0, np.arange(n_inter), virt)
    tail = np.concatenate([tail, vt])
    head = np.concatenate([head, vh])
    length = np.concatenate([np.maximum(length, 50.0), np.full(n_inter, 200.0)])
    L = len(tail)
    lanes = np.concatenate([rng_net.integers(1, 3, len(roads)).repeat(2), np.full(n_inter, 2)])
    truth = {g: rng_true.uniform(lo, hi, L) for g, (lo, hi) in PAPER_RANGES.items()}
    origins = virt[kind == 0]
    dests = virt[kind == 1]
    net = Network(
        n_nodes=2 * n_inter, tail=_i32(tail), head=_i32(head), lanes=_i32(lanes), length=_f32(length),
        free_speed=_f32(truth["free_speed"]), jam_density=_f32(truth["jam_density"]),
        capacity=_f32(np.full(L, CAPACITY_PER_LANE)), beta=_f32(truth["beta"]), alpha=_f32(truth["alpha"]),
        cost=_f32(np.ones(L)), origin_node=_i32(origins), detector_link=_i32(np.arange(L)),
        detector_pos=_f32(_f32(length) * np.float32(0.5)), node_xy=None)
    O = len(origins)
    o = np.arange(n_agents) % O
    dest = dests[rng_dem.integers(0, len(dests), n_agents)]
    dem = Demand(agent_origin=_i32(o), agent_dest=_i32(dest), ready_time=_f32(np.zeros(n_agents)))
    cfg = Config(dt=1.0, gumbel_tau=0.5, dest_logit_coef=0.1, seed=k, steps=steps, count_bin_steps=300,
                 ckpt_every=60, allow_uturn=1)
    return Workload(f"sioux_like_{L}links_{n_agents // 1000}k", net, dem, cfg,
                    extra={"truth": {g: _f32(v) for g, v in truth.items()}})


def calibration_start(w: Workload) -> Workload:
    """The same workload with every calibrated per-link parameter at the middle of the paper's range
    (the paper starts its calibration there) and the jam density of the network at the top of its
    range, so that link rings are sized for any value the calibration may reach; the starting
    values are in extra["start"]."""
    from copy import deepcopy
    v = deepcopy(w)
    v.extra["start"] = {g: _f32(np.full(w.net.n_links, 0.5 * (lo + hi))) for g, (lo, hi) in PAPER_RANGES.items()}
    v.net.jam_density = _f32(np.full(w.net.n_links, PAPER_RANGES["jam_density"][1]))
    for g in ("free_speed", "beta", "alpha"):
        setattr(v.net, g, v.extra["start"][g].copy())
    v.name = w.name + "_start"
    return v


def control_multipliers(n_links: int, n_controlled: int, n_scenarios: int, seed0: int = 500):
    """Capacity multipliers in [0.5, 1] on n_controlled links sampled
    uniformly; one independent draw per candidate scenario; 1 elsewhere."""
    rng = np.random.default_rng(seed0 - 1)
    ctrl = np.sort(rng.choice(n_links, size=min(n_controlled, n_links), replace=False))
    m = np.ones((n_scenarios, n_links), np.float32)
    for s in range(n_scenarios):
        r = np.random.default_rng(seed0 + s)
        m[s, ctrl] = r.uniform(0.5, 1.0, size=len(ctrl))
    return _i32(ctrl), _f32(m)


def batched_control(n_scenarios: int = 16, steps: int = 3600, n_controlled: int = 2000,
                    seed: int = 5) -> Workload:
    """Batched control: the 32x32 lattice workload with its ground-truth
    demand profile repeated to 3,600 s, 16 candidate scenarios of capacity
    multipliers U[0.5, 1] on 2,000 controlled links, loss = total travel time."""
    w = grid_rates(steps=steps, rate_mode="true", seed=2)
    rates = np.tile(w.dem.rates, (1, int(np.ceil(steps / (w.dem.rates.shape[1] * w.dem.rate_bin_s)))))
    w.dem.rates = _f32(rates)
    ctrl, m = control_multipliers(w.net.n_links, n_controlled, n_scenarios)
    w.cfg = replace(w.cfg, steps=steps, seed=seed)
    w.name = f"control{n_scenarios}x_grid32_{steps}s"
    w.extra.update({"controlled_links": ctrl, "cap_mult": m, "n_scenarios": n_scenarios})
    return w


def serving_requests(n_requests: int = 256, rate_per_s: float = 4.0, steps: int = 3600,
                     links_range=(1_000, 35_000), agents_range=(10_000, 1_000_000), seed: int = 41,
                     scale: float = 1.0):
    """Poisson stream of nowcast rollout requests on seeded metro networks of
    log-uniform size.  Returns (arrival_s, spec) pairs; spec holds the
    generator arguments so a request is materialised only when admitted.
    `scale` shrinks link and agent counts uniformly (for small tests)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, size=n_requests))
    out = []
    for i in range(n_requests):
        L = float(np.exp(rng.uniform(np.log(links_range[0]), np.log(links_range[1])))) * scale
        N = float(np.exp(rng.uniform(np.log(agents_range[0]), np.log(agents_range[1])))) * scale
        roads = max(8, int(L / 2))
        nodes = max(6, int(L / 2.92))
        zs = max(2, int(round(np.sqrt(1024 * L / 35_000))))
        out.append((float(t[i]), dict(n_nodes=nodes, n_roads=roads, n_agents=max(10, int(N)),
                                      zones_side=zs, bins=20, bin_s=180.0,
                                      n_detectors=min(200, roads), steps=steps,
                                      seed=1000 + i)))
    return out


def tg_toy(u1: float = 2.0, u2: float = 1.0) -> Workload:
    """The trajectory-grafting toy (SI-C): one agent, two 15 m links in
    series, free speeds u1 then u2, 10 s horizon; the agent starts at x = 0 on
    link 1 (placed by setting the state, not by a departure)."""
    roads = np.asarray([(0, 1), (1, 2)], np.int64)
    net = Network(
        n_nodes=3, tail=_i32([0, 1]), head=_i32([1, 2]), lanes=_i32([1, 1]),
        length=_f32([15.0, 15.0]), free_speed=_f32([u1, u2]),
        jam_density=_f32([JAM_DENSITY_PER_LANE] * 2), capacity=_f32([10.0, 10.0]),
        beta=_f32([0, 0]), alpha=_f32([1, 1]), cost=_f32([1, 1]),
        origin_node=_i32([0]), detector_link=_i32([1]), detector_pos=_f32([7.5]))
    del roads
    dem = Demand(agent_origin=_i32([0]), agent_dest=_i32([2]), ready_time=_f32([1e9]))
    cfg = Config(dt=1.0, steps=10, count_bin_steps=10, ckpt_every=60)
    return Workload("tg_toy", net, dem, cfg)


def merge_toy(alpha=(1.0, 1.0), length: float = 100.0, speed: float = 10.0, seed: int = 0,
              tau: float = 0.5) -> Workload:
    """Two one-lane links 0->2 and 1->2 merging into 2->3; one agent placed at
    the end of each in-link at t = 0, both bound for node 3, so in the first
    step both heads want the single entry slot of 2->3 and the merge decides."""
    net = Network(
        n_nodes=4, tail=_i32([0, 1, 2]), head=_i32([2, 2, 3]), lanes=_i32([1, 1, 1]),
        length=_f32([length] * 3), free_speed=_f32([speed] * 3),
        jam_density=_f32([JAM_DENSITY_PER_LANE] * 3), capacity=_f32([10.0] * 3),
        beta=_f32([0, 0, 0]), alpha=_f32(list(alpha) + [1.0]), cost=_f32([1, 1, 1]),
        origin_node=_i32([0]), detector_link=_i32([2]), detector_pos=_f32([length / 2]))
    dem = Demand(agent_origin=_i32([0, 0]), agent_dest=_i32([3, 3]), ready_time=_f32([1e9, 1e9]))
    cfg = Config(dt=1.0, steps=1, count_bin_steps=1, ckpt_every=60, seed=seed, gumbel_tau=tau)
    return Workload("merge_toy", net, dem, cfg)


def route_merge_toy(seed: int = 0, alpha=(1.0, 1.0), tau: float = 0.5) -> Workload:
    """A route choice whose chosen link is contested.  Links 0: 0->2 and
    1: 1->2 (one lane, 100 m) end at node 2, whose out-links 2: 2->3 and
    3: 2->4 lead on to node 5 through 4: 3->5 and 5: 4->5.  Agent 0 is placed
    at the end of link 0 and bound for node 5, so it chooses between links 2
    and 3 (distinct beta, cost and times to node 5); agent 1 is placed at the
    end of link 1 and bound for node 3, which only link 2 reaches.  When agent
    0 picks link 2, the two heads compete for its single entry slot."""
    net = Network(
        n_nodes=6, tail=_i32([0, 1, 2, 2, 3, 4]), head=_i32([2, 2, 3, 4, 5, 5]), lanes=_i32([1] * 6),
        length=_f32([100.0, 100.0, 120.0, 90.0, 200.0, 260.0]),
        free_speed=_f32([10.0, 10.0, 10.0, 12.0, 10.0, 13.0]),
        jam_density=_f32([JAM_DENSITY_PER_LANE] * 6), capacity=_f32([10.0] * 6),
        beta=_f32([0.0, 0.0, 1.2, 0.7, 0.0, 0.0]), alpha=_f32(list(alpha) + [1.0] * 4),
        cost=_f32([1.0, 1.0, 1.5, 0.8, 1.0, 1.0]),
        origin_node=_i32([0]), detector_link=_i32([2]), detector_pos=_f32([60.0]))
    dem = Demand(agent_origin=_i32([0, 0]), agent_dest=_i32([5, 3]), ready_time=_f32([1e9, 1e9]))
    cfg = Config(dt=1.0, steps=1, count_bin_steps=1, ckpt_every=60, seed=seed, gumbel_tau=tau)
    return Workload("route_merge_toy", net, dem, cfg)


def hub(n_spokes: int = 8, lanes: int = 8, long_len: float = 1500.0, short_len: float = 60.0,
        n_agents: int = 8000, steps: int = 600, capacity: float = 0.05, seed: int = 3) -> Workload:
    """The kernels' largest cases in one network.  A hub node 0 with n_spokes
    two-way roads of `lanes` lanes, so its in-links offer n_spokes * lanes
    merge candidates (64: one full wavefront).  Even roads are long (rings of
    lanes * (L / jam spacing + 4) slots, far above 128), odd roads short.  Low
    outflow capacity makes queues fill every lane at the hub.  Spoke 1 has
    four origin queues (one front each per step) releasing fast, so the long
    link 1 -> 0 holds many hundreds of agents (several staging pieces); it also
    carries four detectors, the per-link maximum.  One origin on every other
    spoke; each agent is bound for another spoke through the hub; departure
    rates per (origin, 4 bins)."""
    rng = np.random.default_rng(seed)
    roads = np.asarray([(0, k + 1) for k in range(n_spokes)], np.int64)
    length = np.where(np.arange(n_spokes) % 2 == 0, long_len, short_len)
    speed = rng.choice(np.asarray(SPEED_CHOICES), n_spokes)
    origin_node = np.asarray([1, 1, 1, 1] + list(range(2, n_spokes + 1)))
    net = make_network(n_spokes + 1, roads, length, np.full(n_spokes, lanes), speed,
                       origin_node=origin_node, n_detectors=0, rng=rng,
                       beta=np.repeat(rng.uniform(0.5, 2, n_spokes), 2),
                       alpha=np.repeat(rng.uniform(0.5, 2, n_spokes), 2),
                       cost=np.repeat(rng.uniform(0.5, 2, n_spokes), 2))
    net.capacity = _f32(np.full(net.n_links, capacity))
    # link 2k+1 is spoke k+1 -> hub: four detectors on link 1, one mid-link on every other in-link
    det = [1, 1, 1, 1] + [2 * k + 1 for k in range(1, n_spokes)]
    frac = [0.2, 0.4, 0.6, 0.8] + [0.5] * (n_spokes - 1)
    net.detector_link = _i32(det)
    net.detector_pos = _f32([net.length[j] * np.float32(f) for j, f in zip(det, frac)])
    O = len(origin_node)
    o = np.concatenate([np.arange(n_agents // 2) % 4, rng.integers(4, O, n_agents - n_agents // 2)])
    dest = np.empty(n_agents, np.int64)
    for i in range(n_agents):
        home = origin_node[o[i]]
        dest[i] = 1 + (home + rng.integers(n_spokes - 1)) % n_spokes   # any spoke but home
    bins = 4
    rates = rng.uniform(0.5, 1.0, (O, bins))
    rates[:4, :2] = 1.5
    dem = Demand(agent_origin=_i32(o), agent_dest=_i32(dest), rates=_f32(rates), rate_bin_s=steps / bins)
    cfg = Config(dt=1.0, steps=steps, count_bin_steps=steps // 4, gumbel_tau=0.5, seed=seed, ckpt_every=60)
    return Workload("hub64", net, dem, cfg)


def diamond(n_agents: int = 200, lanes: int = 1, seed: int = 7, length: float = 100.0,
            horizon_s: float = 300.0, capacity: float = 0.5) -> Workload:
    """Four-node diamond A(0)->B(1)->D(3), A->C(2)->D with reverse links;
    origins at A and D, destinations the opposite node."""
    rng = np.random.default_rng(seed)
    roads = np.asarray([(0, 1), (0, 2), (1, 3), (2, 3)], np.int64)
    net = make_network(4, roads, np.full(4, length), np.full(4, lanes), np.full(4, 13.9),
                       origin_node=[0, 3], n_detectors=0, rng=rng)
    net.capacity = _f32(np.full(net.n_links, capacity))
    net.detector_link = _i32(np.arange(net.n_links))
    net.detector_pos = _f32(net.length * np.float32(0.5))
    o = np.arange(n_agents) % 2
    dest = np.where(o == 0, 3, 0)
    ready = rng.uniform(0.0, horizon_s * 0.5, n_agents)
    dem = Demand(agent_origin=_i32(o), agent_dest=_i32(dest), ready_time=_f32(ready))
    cfg = Config(dt=1.0, steps=int(horizon_s), count_bin_steps=60, gumbel_tau=0.5, seed=seed)
    return Workload(f"diamond_{n_agents}", net, dem, cfg)


def line(n_links: int = 3, length: float = 200.0, speed: float = 13.9, lanes: int = 1,
         capacity: float = 0.5, n_agents: int = 1, ready=None, jam_density=JAM_DENSITY_PER_LANE,
         steps: int = 200) -> Workload:
    """A one-way corridor 0->1->...->n_links; origin at node 0, every agent's
    destination the last node.  Used for closed forms (free-flow travel time,
    throughput at capacity, spacing at jam)."""
    tail = np.arange(n_links)
    head = tail + 1
    net = Network(
        n_nodes=n_links + 1, tail=_i32(tail), head=_i32(head), lanes=_i32(np.full(n_links, lanes)),
        length=_f32(np.full(n_links, length)), free_speed=_f32(np.full(n_links, speed)),
        jam_density=_f32(np.full(n_links, jam_density)),
        capacity=_f32(np.full(n_links, capacity)),
        beta=_f32(np.zeros(n_links)), alpha=_f32(np.ones(n_links)), cost=_f32(np.ones(n_links)),
        origin_node=_i32([0]), detector_link=_i32(np.arange(n_links)),
        detector_pos=_f32(np.full(n_links, length) * np.float32(0.5)))
    if ready is None:
        ready = np.zeros(n_agents)
    dem = Demand(agent_origin=_i32(np.zeros(n_agents)), agent_dest=_i32(np.full(n_agents, n_links)),
                 ready_time=_f32(ready))
    cfg = Config(dt=1.0, steps=steps, count_bin_steps=max(1, steps // 4) if steps % 4 == 0 else steps)
    return Workload(f"line{n_links}", net, dem, cfg)


def with_platoon(w: Workload, dn: int, tau: float = 1.0) -> Workload:
    """The same network, agent pool and horizon with platoons of dn vehicles
    per agent and the step the paper ties to it, dt = tau * dn (Methods,
    Newell's model; SI-E): steps, sampling and checkpoint intervals shrink by
    dn, departure rates given in vehicles/s become agents/s (divided by dn).
    Capacities stay in vehicles/s/lane (the library divides by dn)."""
    from copy import deepcopy
    v = deepcopy(w)
    dt = float(tau) * dn
    for name, val in (("steps", w.cfg.steps), ("count_bin_steps", w.cfg.count_bin_steps)):
        if val % dn:
            raise ValueError(f"{name} = {val} is not a multiple of the platoon size {dn}")
    v.cfg.platoon = int(dn)
    v.cfg.dt = dt
    v.cfg.steps = w.cfg.steps // dn
    v.cfg.count_bin_steps = w.cfg.count_bin_steps // dn
    v.cfg.ckpt_every = max(1, w.cfg.ckpt_every // dn)
    if v.dem.rates is not None:
        if abs(v.dem.rate_bin_s / dt - round(v.dem.rate_bin_s / dt)) > 1e-9:
            raise ValueError("rate bins must be a whole number of platoon steps")
        v.dem.rates = _f32(v.dem.rates / np.float32(dn))
    v.name = f"{w.name}_dn{dn}"
    return v


def random_small(seed: int, nx: int = 3, ny: int = 3, n_agents: int = 60, rates: bool = False,
                 steps: int = 240, lanes_max: int = 2) -> Workload:
    """Small random lattice with random lengths/lanes/speeds/params, used for
    randomized oracle checks and parity cases that span several tiles."""
    rng = np.random.default_rng(seed)
    roads = grid_roads(nx, ny)
    R = len(roads)
    length = rng.uniform(40.0, 160.0, R)
    lanes = rng.integers(1, lanes_max + 1, R)
    speed = rng.choice(np.asarray(SPEED_CHOICES), R)
    bnd = boundary_nodes(nx, ny)
    net = make_network(nx * ny, roads, length, lanes, speed, origin_node=bnd,
                       n_detectors=max(1, R), rng=rng,
                       beta=np.repeat(rng.uniform(0, 2, R), 2),
                       alpha=np.repeat(rng.uniform(0.5, 2, R), 2),
                       cost=np.repeat(rng.uniform(0.5, 2, R), 2))
    net.capacity = _f32(rng.uniform(0.3, 1.0, net.n_links))
    O = len(bnd)
    o = rng.integers(0, O, n_agents)
    dest = np.empty(n_agents, np.int64)
    for i in range(n_agents):
        while True:
            d = bnd[rng.integers(O)]
            if d != bnd[o[i]]:
                break
        dest[i] = d
    if rates:
        bins = 4
        dem = Demand(agent_origin=_i32(o), agent_dest=_i32(dest),
                     rates=_f32(rng.uniform(0.02, 0.15, (O, bins))), rate_bin_s=steps / bins)
    else:
        dem = Demand(agent_origin=_i32(o), agent_dest=_i32(dest),
                     ready_time=_f32(rng.uniform(0, steps * 0.6, n_agents)))
    cfg = Config(dt=1.0, steps=steps, count_bin_steps=steps // 4, gumbel_tau=0.5, seed=seed,
                 ckpt_every=max(1, steps // 8))
    return Workload(f"rand{seed}", net, dem, cfg)
