"""Seeded synthetic unit-commitment grids.

This module only draws inputs: topology, branch impedances and ratings,
generator data, load profiles and contingency lists.  It holds none of the
solver's arithmetic (no power flow, no sensitivities, no objective), so both
the HIP library and the independent CPU checker can take their inputs from it.

The recipe stands in for the GO3 C3E3.1 division-1 cases the paper measures
on (Section IV, Table 1; Fig. 1 uses a 617-bus, 18-period case with 562 line
contingencies).  Those files are not available, so every grid here is drawn
from a seeded generator with the same shape:

* topology: a random tree plus uniformly drawn extra edges (no duplicates, no
  self loops); per-unit series impedance x ~ U[0.02, 0.2], r = x * U[0.1, 0.3],
  no line charging, tap ratio 1 and phase shift 0;
* generators at distinct buses, three equal cost blocks with increasing
  marginal cost (the convex block bids of Example 3, eq. (costs));
* bus loads lognormal(0, 0.3) times a sinusoidal daily profile, scaled so the
  peak total load is a fixed share of total capacity; a spinning-reserve
  requirement of 10 % of load per period;
* contingencies: single-branch outages that do not island the network
  (Section II-E), either all of them or a seeded subset of a given size.

Branch ratings come from a purely combinatorial estimate: the flow a
proportional dispatch would push through each tree edge if the extra edges
were absent (the sum of net injections below the edge), relieved by a fixed
meshing factor.  No network equations are solved here.

All quantities are per unit on a 100 MVA base; prices are $ per pu-hour.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = ["GridCase", "make_case", "CONFIGS", "config_case", "batch_cases", "load_draw",
           "with_loads",
           "flat_start",
           "random_point"]


@dataclasses.dataclass
class GridCase:
    """Plain container of host arrays describing one problem instance."""

    n_bus: int
    n_branch: int
    n_gen: int
    n_period: int
    n_seg: int
    br_from: np.ndarray      # int32 [L]
    br_to: np.ndarray        # int32 [L]
    br_r: np.ndarray         # [L]
    br_x: np.ndarray         # [L]
    br_bch: np.ndarray       # [L]
    br_smax: np.ndarray      # [L]
    br_smax_ctg: np.ndarray  # [L]
    gen_bus: np.ndarray      # int32 [G]
    gen_pmin: np.ndarray
    gen_pmax: np.ndarray
    gen_qmin: np.ndarray
    gen_qmax: np.ndarray
    gen_rmax: np.ndarray
    gen_ru: np.ndarray
    gen_rd: np.ndarray
    gen_ru_su: np.ndarray
    gen_rd_sd: np.ndarray
    gen_p0: np.ndarray
    gen_u0: np.ndarray
    gen_c_on: np.ndarray
    gen_c_su: np.ndarray
    gen_c_sd: np.ndarray
    gen_c_r: np.ndarray
    gen_seg_cost: np.ndarray  # [G, M]
    gen_seg_size: np.ndarray  # [G, M]
    load_p: np.ndarray        # [T, N]
    load_q: np.ndarray        # [T, N]
    reserve_req: np.ndarray   # [T]
    dt: np.ndarray            # [T] hours
    v_min: np.ndarray         # [N]
    v_max: np.ndarray         # [N]
    c_p: float
    c_q: float
    c_s: float
    c_ang: float
    ang_max: float
    c_rsv: float
    rho: float
    load_value: float
    ctg_list: np.ndarray      # int32 [K] outaged branch per contingency
    ref_bus: int = 0
    name: str = ""

    @property
    def n_ctg(self) -> int:
        return int(self.ctg_list.shape[0])

    @property
    def n_x(self) -> int:
        return 2 * self.n_period * self.n_bus + 4 * self.n_period * self.n_gen

    def block_slices(self):
        """Offsets of the six variable blocks V, TH, P, Q, R, U in x."""
        T, N, G = self.n_period, self.n_bus, self.n_gen
        lens = [T * N, T * N, T * G, T * G, T * G, T * G]
        offs = np.concatenate([[0], np.cumsum(lens)[:-1]])
        return [slice(int(o), int(o + n)) for o, n in zip(offs, lens)]


# --------------------------------------------------------------------------
# topology
# --------------------------------------------------------------------------

def _random_tree(rng: np.random.Generator, n: int, kind: str):
    """Return parent[] of a random tree rooted at 0 (parent[0] = -1)."""
    parent = np.full(n, -1, dtype=np.int64)
    if n == 1:
        return parent
    if kind == "recursive":
        for i in range(1, n):
            parent[i] = rng.integers(0, i)
        return parent
    if kind != "prufer":
        raise ValueError(kind)
    # Uniform labelled tree from a random Pruefer sequence, then rooted at 0.
    if n == 2:
        adj = [[1], [0]]
    else:
        seq = rng.integers(0, n, size=n - 2)
        degree = np.ones(n, dtype=np.int64)
        for s in seq:
            degree[s] += 1
        adj = [[] for _ in range(n)]
        import heapq
        leaves = [i for i in range(n) if degree[i] == 1]
        heapq.heapify(leaves)
        for s in seq:
            leaf = heapq.heappop(leaves)
            adj[leaf].append(int(s))
            adj[int(s)].append(leaf)
            degree[s] -= 1
            if degree[s] == 1:
                heapq.heappush(leaves, int(s))
        u = heapq.heappop(leaves)
        w = heapq.heappop(leaves)
        adj[u].append(w)
        adj[w].append(u)
    # root at 0 with an explicit stack
    seen = np.zeros(n, dtype=bool)
    seen[0] = True
    stack = [0]
    while stack:
        a = stack.pop()
        for b in adj[a]:
            if not seen[b]:
                seen[b] = True
                parent[b] = a
                stack.append(b)
    return parent


def _depths(parent):
    n = parent.shape[0]
    depth = np.full(n, -1, dtype=np.int64)
    depth[0] = 0
    for i in range(n):
        # walk up until a known depth, then fill the path
        path = []
        a = i
        while depth[a] < 0:
            path.append(a)
            a = parent[a]
        d = depth[a]
        for b in reversed(path):
            d += 1
            depth[b] = d
    return depth


def _cycle_edges(parent, depth, extra_pairs):
    """Tree edges (named by their child node) covered by a fundamental cycle.

    A tree edge lies on a cycle, and so is not a bridge, exactly when some
    extra edge's tree path passes over it.
    """
    covered = np.zeros(parent.shape[0], dtype=bool)
    for a, b in extra_pairs:
        a, b = int(a), int(b)
        while a != b:
            if depth[a] >= depth[b]:
                covered[a] = True
                a = int(parent[a])
            else:
                covered[b] = True
                b = int(parent[b])
    return covered


# --------------------------------------------------------------------------
# main generator
# --------------------------------------------------------------------------

def make_case(seed: int, n_bus: int, n_branch: int, n_gen: int, n_period: int,
              n_ctg: Optional[int] = None, tree: str = "recursive",
              load_share: float = 0.7, mesh: float = 0.55, name: str = "") -> GridCase:
    """Draw one seeded grid.

    n_ctg=None keeps every non-islanding single-branch outage; otherwise a
    seeded subset of exactly n_ctg of them (all of them if fewer exist).
    mesh scales the tree-flow estimate of the ratings (smaller: more
    congestion).
    """
    if n_branch < n_bus - 1:
        raise ValueError("need at least a spanning tree")
    if n_gen > n_bus:
        raise ValueError("generators sit at distinct buses")
    rng = np.random.default_rng(seed)
    N, L, G, T, M = n_bus, n_branch, n_gen, n_period, 3

    # --- topology: tree + uniform extra edges
    parent = _random_tree(rng, N, tree)
    depth = _depths(parent)
    edges = [(int(parent[i]), i) for i in range(1, N)]
    present = {(min(a, b), max(a, b)) for a, b in edges}
    extra = []
    n_extra = L - (N - 1)
    if n_extra > N * (N - 1) // 2 - (N - 1):
        raise ValueError("too many branches for a simple graph")
    while len(extra) < n_extra:
        a, b = (int(v) for v in rng.integers(0, N, size=2))
        if a == b:
            continue
        key = (min(a, b), max(a, b))
        if key in present:
            continue
        present.add(key)
        extra.append((a, b))
    all_edges = edges + extra
    # shuffle branch order and orientation so that nothing downstream can
    # rely on tree edges coming first
    perm = rng.permutation(L)
    flip = rng.random(L) < 0.5
    br_from = np.empty(L, dtype=np.int32)
    br_to = np.empty(L, dtype=np.int32)
    is_tree = np.zeros(L, dtype=bool)
    tree_child = np.full(L, -1, dtype=np.int64)
    for new_idx, old_idx in enumerate(perm):
        a, b = all_edges[old_idx]
        if old_idx < N - 1:
            is_tree[new_idx] = True
            tree_child[new_idx] = b  # edges[i] = (parent[b], b)
        if flip[new_idx]:
            a, b = b, a
        br_from[new_idx] = a
        br_to[new_idx] = b

    covered = _cycle_edges(parent, depth, extra)
    nonbridge = np.ones(L, dtype=bool)
    nonbridge[is_tree] = covered[tree_child[is_tree]]

    br_x = rng.uniform(0.02, 0.2, size=L)
    br_r = br_x * rng.uniform(0.1, 0.3, size=L)
    br_bch = np.zeros(L)

    # --- generators
    gen_bus = np.sort(rng.choice(N, size=G, replace=False)).astype(np.int32)
    pmax = rng.uniform(0.5, 3.0, size=G)
    pmin = rng.uniform(0.1, 0.4, size=G) * pmax
    qmin = -0.3 * pmax
    qmax = 0.5 * pmax
    seg_size = np.repeat((pmax / M)[:, None], M, axis=1)
    c1 = rng.uniform(1000.0, 4000.0, size=G)            # $/pu-h
    inc = rng.uniform(200.0, 1000.0, size=(G, M - 1))
    seg_cost = np.concatenate([c1[:, None], c1[:, None] + np.cumsum(inc, axis=1)],
                              axis=1)
    c_on = rng.uniform(0.0, 500.0, size=G) * pmax       # $/h when committed
    c_su = rng.uniform(50.0, 500.0, size=G) * 10.0      # $ per start-up
    c_sd = 0.1 * c_su
    c_r = rng.uniform(100.0, 500.0, size=G)             # $/pu-h of reserve
    ru = rng.uniform(0.3, 1.0, size=G) * pmax           # pu per hour
    rd = ru.copy()
    ru_su = pmin + 0.5 * ru
    rd_sd = ru_su.copy()
    rmax = ru / 6.0
    u0 = np.ones(G)

    # --- loads
    dt = np.full(T, 24.0 / T)
    hours = np.arange(T) * dt[0]
    profile = 1.0 + 0.2 * np.sin(2.0 * math.pi * (hours - 9.0) / 24.0)
    mu = rng.lognormal(0.0, 0.3, size=N)
    raw = profile[:, None] * mu[None, :]
    scale = load_share * pmax.sum() / raw.sum(axis=1).max()
    load_p = raw * scale
    pf = rng.uniform(0.92, 0.98, size=N)
    load_q = load_p * np.tan(np.arccos(pf))[None, :]
    reserve_req = 0.1 * load_p.sum(axis=1)

    # --- proportional dispatch (for p0 and the rating estimate only)
    def proportional(total):
        frac = np.clip(total / pmax.sum(), 0.0, 1.0)
        return frac * pmax

    p0 = proportional(load_p[0].sum())
    # tree-flow rating estimate at the peak period
    tpk = int(np.argmax(load_p.sum(axis=1)))
    inj = -load_p[tpk].copy()
    np.add.at(inj, gen_bus, proportional(load_p[tpk].sum()))
    inj -= inj.mean()
    order = np.argsort(-depth)        # children before parents
    sub = inj.copy()
    for i in order:
        if parent[i] >= 0:
            sub[parent[i]] += sub[i]
    est = np.zeros(L)
    est[is_tree] = np.abs(sub[tree_child[is_tree]])
    floor = 0.25
    base = np.where(is_tree, mesh * est, 0.0)
    tree_med = float(np.median(base[is_tree])) if is_tree.any() else floor
    base = np.where(is_tree, base, tree_med)
    smax = rng.uniform(0.8, 1.5, size=L) * np.maximum(base, floor)
    smax_ctg = 1.2 * smax

    # --- contingencies
    nb = np.flatnonzero(nonbridge).astype(np.int32)
    if n_ctg is None or n_ctg >= nb.shape[0]:
        ctg = nb
    else:
        ctg = np.sort(rng.choice(nb, size=n_ctg, replace=False)).astype(np.int32)

    max_block = float(seg_cost.max())
    return GridCase(
        n_bus=N, n_branch=L, n_gen=G, n_period=T, n_seg=M,
        br_from=br_from, br_to=br_to, br_r=br_r, br_x=br_x, br_bch=br_bch,
        br_smax=smax, br_smax_ctg=smax_ctg,
        gen_bus=gen_bus, gen_pmin=pmin, gen_pmax=pmax, gen_qmin=qmin,
        gen_qmax=qmax, gen_rmax=rmax, gen_ru=ru, gen_rd=rd, gen_ru_su=ru_su,
        gen_rd_sd=rd_sd, gen_p0=p0, gen_u0=u0, gen_c_on=c_on, gen_c_su=c_su,
        gen_c_sd=c_sd, gen_c_r=c_r, gen_seg_cost=seg_cost,
        gen_seg_size=seg_size, load_p=load_p, load_q=load_q,
        reserve_req=reserve_req, dt=dt, v_min=np.full(N, 0.9),
        v_max=np.full(N, 1.1), c_p=1.0e5, c_q=1.0e5, c_s=1.0e4, c_ang=1.0e4,
        ang_max=72.0 * math.pi / 180.0, c_rsv=5.0e3, rho=1.0e5,
        load_value=2.0 * max_block, ctg_list=ctg, ref_bus=0, name=name)


# Sizes of the workloads: a 14-bus toy case, a case at the paper's Fig. 1 scale
# (617 buses, 18 periods, about 560 contingencies) and a 2000-bus, 48-period
# case.
# Ratings use mesh = 3.0: with it the plain solve on the 617-bus case closes
# to within about 4 % of the copper-plate bound (a network that binds but can
# carry the economic dispatch); mesh = 0.55 leaves the penalties larger than
# the surplus.
CONFIGS = {
    "c1": dict(seed=1, n_bus=14, n_branch=20, n_gen=5, n_period=4, n_ctg=None,
               tree="recursive", mesh=3.0),
    "c2": dict(seed=2, n_bus=617, n_branch=850, n_gen=100, n_period=18,
               n_ctg=560, tree="recursive", mesh=3.0),
    "c3": dict(seed=3, n_bus=2000, n_branch=2800, n_gen=300, n_period=48,
               n_ctg=2500, tree="prufer", mesh=3.0),
}


def batch_cases(n: int = 64, seed0: int = 4000, n_bus=(100, 2000), n_period=(12, 48)):
    """Independent scenarios of uneven size for batched solves: bus counts and
    period counts drawn uniformly from the given ranges, 1.4 branches and 0.15
    generators per bus, every non-islanding outage, ratings as the configs."""
    rng = np.random.default_rng(seed0)
    out = []
    for i in range(n):
        N = int(rng.integers(n_bus[0], n_bus[1] + 1))
        T = int(rng.integers(n_period[0], n_period[1] + 1))
        out.append(make_case(seed=seed0 + 1 + i, n_bus=N, n_branch=int(round(1.4 * N)),
                             n_gen=max(2, int(round(0.15 * N))), n_period=T, n_ctg=None,
                             tree="prufer", mesh=3.0, name=f"batch-{i}"))
    return out


def config_case(name: str, **overrides) -> GridCase:
    kw = dict(CONFIGS[name])
    kw.update(overrides)
    return make_case(name=name, **kw)


def load_draw(case: GridCase, seed: int, phase_hours: float = 2.0,
              level: tuple = (0.85, 1.0)):
    """Loads of one operating day on the same grid: bus weights lognormal(0,
    0.3) drawn afresh, the daily profile shifted by U[-phase_hours,
    +phase_hours] hours, and the peak total scaled to U[level] times the
    grid's own peak.  Power factors as in the grid.  Returns (load_p, load_q,
    reserve_req) shaped [T, N], [T, N], [T]."""
    rng = np.random.default_rng(seed)
    T, N = case.n_period, case.n_bus
    dt = case.dt[0]
    shift = rng.uniform(-phase_hours, phase_hours)
    hours = np.arange(T) * dt
    profile = 1.0 + 0.2 * np.sin(2.0 * math.pi * (hours - 9.0 - shift) / 24.0)
    mu = rng.lognormal(0.0, 0.3, size=N)
    raw = profile[:, None] * mu[None, :]
    peak = case.load_p.sum(axis=1).max() * rng.uniform(*level)
    load_p = raw * (peak / raw.sum(axis=1).max())
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(case.load_p > 0, case.load_q / case.load_p, 0.0)
    load_q = load_p * ratio[0][None, :]
    reserve_req = 0.1 * load_p.sum(axis=1)
    return load_p, load_q, reserve_req


def with_loads(case: GridCase, draw) -> GridCase:
    """The same grid with the loads of a draw (see load_draw)."""
    load_p, load_q, reserve_req = draw
    return dataclasses.replace(case, load_p=np.asarray(load_p, dtype=np.float64),
                               load_q=np.asarray(load_q, dtype=np.float64),
                               reserve_req=np.asarray(reserve_req, dtype=np.float64))


def flat_start(case: GridCase, dispatch: Optional[np.ndarray] = None) -> np.ndarray:
    """x with v = 1, theta = 0, u = 1, r = 0, q = 0 and p = dispatch [T, G]
    (proportional-to-capacity if not given)."""
    T, N, G = case.n_period, case.n_bus, case.n_gen
    sl = case.block_slices()
    x = np.zeros(case.n_x)
    x[sl[0]] = 1.0
    if dispatch is None:
        tot = case.load_p.sum(axis=1)
        frac = np.clip(tot / case.gen_pmax.sum(), 0.0, 1.0)
        dispatch = frac[:, None] * case.gen_pmax[None, :]
    x[sl[2]] = np.asarray(dispatch, dtype=np.float64).reshape(-1)
    x[sl[5]] = 1.0
    return x


def random_point(case: GridCase, seed: int, spread: float = 1.0) -> np.ndarray:
    """A seeded interior point of the box (for derivative and parity checks).

    Angles are drawn around a smooth profile so that branch angle differences
    stay moderate; p, q, r, u are uniform inside their boxes.
    """
    rng = np.random.default_rng(seed)
    T, N, G = case.n_period, case.n_bus, case.n_gen
    sl = case.block_slices()
    x = np.empty(case.n_x)
    x[sl[0]] = rng.uniform(0.92, 1.08, size=T * N)
    x[sl[1]] = spread * rng.normal(0.0, 0.15, size=T * N)
    x[sl[2]] = (rng.uniform(0.05, 0.95, size=(T, G)) * case.gen_pmax).reshape(-1)
    x[sl[3]] = (case.gen_qmin + rng.uniform(0.05, 0.95, size=(T, G))
                * (case.gen_qmax - case.gen_qmin)).reshape(-1)
    x[sl[4]] = (rng.uniform(0.05, 0.95, size=(T, G)) * case.gen_rmax).reshape(-1)
    x[sl[5]] = rng.uniform(0.05, 0.95, size=T * G)
    return x
