"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the component-matrix method, of the hash
fusion or of the learned combiner: it only draws random temporal networks,
the random coefficients the hash family draws (passed to both sides as
inputs), random MLP initial weights and minibatch orders.  Every generator
uses numpy's counter-based Philox bit generator keyed by an explicit seed, so
the same call returns the same arrays on every machine with this numpy.

Event arrays are structure-of-arrays: ``src`` and ``dst`` are ``uint32`` node
ids in ``[0, n)``, ``t`` is ``int64`` integer time steps (the paper's temporal
network has events at discrete time steps, Sec. 2.1), and every generator
returns the events in chronological order (stable sort on ``t``), which is the
time-ordered list Algorithm 1 takes as input.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng", "sort_events", "uniform_pairs", "activity_driven", "er_poisson",
    "activities", "hash_coefficients", "MERSENNE61", "mlp_init", "MLP_SIZES",
    "mlp_param_count", "NetSpec", "batched_suite", "WORKLOADS", "make_workload",
    "static_graph_rounds", "chronological_path", "random_tiny", "hll_node_hashes",
    "star_steps",
]

MERSENNE61 = (1 << 61) - 1


def rng(seed: int) -> np.random.Generator:
    """A Philox (counter-based) generator keyed by ``seed``."""
    return np.random.Generator(np.random.Philox(key=int(seed) & ((1 << 64) - 1)))


def sort_events(src, dst, t):
    """Stable chronological order (ties keep their draw order)."""
    order = np.argsort(t, kind="stable")
    return (np.ascontiguousarray(src[order], dtype=np.uint32),
            np.ascontiguousarray(dst[order], dtype=np.uint32),
            np.ascontiguousarray(t[order], dtype=np.int64))


def _partner(g: np.random.Generator, n: int, first: np.ndarray) -> np.ndarray:
    """Uniform partner in [n] \\ {first}."""
    other = g.integers(0, n - 1, size=first.shape[0], dtype=np.int64)
    other += (other >= first)
    return other


def uniform_pairs(n: int, m: int, T: int, seed: int):
    """``m`` undirected events between uniformly drawn distinct endpoints.

    ``u`` uniform in [n], ``v`` uniform in [n] minus {u}, ``t`` uniform integer
    in [0, T).  Repeated pairs across events are allowed.
    """
    if n < 2 and m > 0:
        raise ValueError("need n >= 2 for distinct endpoints")
    g = rng(seed)
    u = g.integers(0, n, size=m, dtype=np.int64)
    v = _partner(g, n, u)
    t = g.integers(0, T, size=m, dtype=np.int64)
    return sort_events(u.astype(np.uint32), v.astype(np.uint32), t)


def two_block_pairs(n: int, m: int, T: int, seed: int):
    """``m`` undirected events inside two blocks, the even and the odd nodes:
    ``u`` uniform in [n], ``v`` uniform over the nodes of ``u``'s parity
    minus ``u``, ``t`` uniform integer in [0, T).  No path ever joins the
    blocks, so the component matrix keeps zero where a row's and a column's
    parities differ, however many events there are.
    """
    if n < 4 and m > 0:
        raise ValueError("need n >= 4 for two blocks of two nodes")
    g = rng(seed)
    u = g.integers(0, n, size=m, dtype=np.int64)
    p = u % 2
    size = (n - p + 1) // 2  # nodes of u's parity
    j = (g.random(m) * (size - 1)).astype(np.int64)
    j = np.minimum(j, size - 2)
    j += j >= u // 2  # skip u itself
    v = 2 * j + p
    t = g.integers(0, T, size=m, dtype=np.int64)
    return sort_events(u.astype(np.uint32), v.astype(np.uint32), t)


def activities(n: int, seed: int, gamma: float = 2.1, eps: float = 1e-3):
    """Node activities with density proportional to a^-gamma on [eps, 1] (inverse CDF)."""
    g = rng(seed ^ 0x5A5A5A5A)
    U = g.random(n)
    e = 1.0 - gamma
    lo = eps ** e
    return (lo + U * (1.0 - lo)) ** (1.0 / e)


def activity_driven(n: int, m: int, T: int, seed: int, gamma: float = 2.1,
                    eps: float = 1e-3, progress=None):
    """Activity-driven temporal network with ``m`` undirected events.

    Each node fires as an independent Poisson process of rate proportional to
    its activity; conditioned on ``m`` events in [0, T) this is: initiator
    drawn with probability a_i / sum(a), partner uniform among the other
    nodes, time uniform, then discretised to integer ticks.
    """
    a = activities(n, seed, gamma, eps)
    cdf = np.cumsum(a)
    cdf /= cdf[-1]
    g = rng(seed)
    out_u = np.empty(m, dtype=np.uint32)
    out_v = np.empty(m, dtype=np.uint32)
    out_t = np.empty(m, dtype=np.int64)
    chunk = 1 << 24
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        k = hi - lo
        u = np.searchsorted(cdf, g.random(k), side="right").astype(np.int64)
        np.minimum(u, n - 1, out=u)
        v = _partner(g, n, u)
        out_u[lo:hi] = u
        out_v[lo:hi] = v
        out_t[lo:hi] = g.integers(0, T, size=k, dtype=np.int64)
        if progress:
            progress(f"{hi} of {m} events drawn")
    return sort_events(out_u, out_v, out_t)


def er_poisson(n: int, m: int, T: int, seed: int, p: float | None = None):
    """Erdos-Renyi G(n, p=2/n) static graph with a Poisson process on each link.

    The link processes have equal rates, so conditioned on ``m`` events each
    event picks a link uniformly and a uniform time in [0, T) (Sec. 3.5's
    experimental setting).
    """
    g = rng(seed)
    if p is None:
        p = 2.0 / n
    # sample the static graph: number of links ~ Binomial(n(n-1)/2, p),
    # then distinct unordered pairs by rejection
    npairs = n * (n - 1) // 2
    E = int(g.binomial(npairs, p))
    E = max(E, 1)
    seen = set()
    links = []
    while len(links) < E:
        a = int(g.integers(0, n))
        b = int(g.integers(0, n - 1))
        b += b >= a
        key = (min(a, b), max(a, b))
        if key not in seen:
            seen.add(key)
            links.append(key)
    links = np.asarray(links, dtype=np.int64)
    pick = g.integers(0, E, size=m, dtype=np.int64)
    u = links[pick, 0].astype(np.uint32)
    v = links[pick, 1].astype(np.uint32)
    t = g.integers(0, T, size=m, dtype=np.int64)
    return sort_events(u, v, t)


def random_tiny(n: int, m: int, T: int, seed: int, allow_self: bool = False):
    """Tiny tie-heavy networks for brute-force checks (endpoints may repeat)."""
    g = rng(seed)
    u = g.integers(0, n, size=m, dtype=np.int64)
    if allow_self:
        v = g.integers(0, n, size=m, dtype=np.int64)
    else:
        v = _partner(g, n, u)
    t = g.integers(0, T, size=m, dtype=np.int64)
    return sort_events(u.astype(np.uint32), v.astype(np.uint32), t)


def static_graph_rounds(n: int, n_links: int, rounds: int, seed: int):
    """A random static graph replayed ``rounds`` times, one time step per round."""
    g = rng(seed)
    a = g.integers(0, n, size=n_links, dtype=np.int64)
    b = _partner(g, n, a)
    src = np.tile(a, rounds).astype(np.uint32)
    dst = np.tile(b, rounds).astype(np.uint32)
    t = np.repeat(np.arange(rounds, dtype=np.int64), n_links)
    return (a.astype(np.uint32), b.astype(np.uint32)), sort_events(src, dst, t)


def star_steps(n: int, steps: int, max_k: int, seed: int):
    """One star per time step: a random hub with 1..max_k distinct random
    partners (a partner equal to the hub makes a self-loop event), so time
    steps touch hubs with every number of partners up to max_k."""
    g = rng(seed)
    src, dst, t = [], [], []
    for step in range(steps):
        hub = int(g.integers(0, n))
        k = int(g.integers(1, max_k + 1))
        partners = g.choice(n, size=min(k, n), replace=False)
        for p in partners:
            if g.random() < 0.5:
                src.append(hub); dst.append(int(p))
            else:
                src.append(int(p)); dst.append(hub)
            t.append(step)
    return sort_events(np.asarray(src, dtype=np.uint32), np.asarray(dst, dtype=np.uint32),
                       np.asarray(t, dtype=np.int64))


def chronological_path(k: int):
    """Events (i, i+1) at time i for i < k on k+1 nodes."""
    src = np.arange(k, dtype=np.uint32)
    return src, src + np.uint32(1), np.arange(k, dtype=np.int64)


def hll_node_hashes(n: int, seed: int) -> np.ndarray:
    """One uniform 64-bit hash value per node, the element hashes of the
    HyperLogLog structures (drawn here, passed to both sides)."""
    g = rng(seed)
    hi = g.integers(0, 2**32, size=n, dtype=np.uint64)
    lo = g.integers(0, 2**32, size=n, dtype=np.uint64)
    return (hi << np.uint64(32)) | lo


def hash_coefficients(H: int, seed: int, order: int = 4) -> np.ndarray:
    """Random coefficients of ``H`` independent hash functions.

    Shape ``(H, 3, order)``, ``uint64``: entry (j, i, l) is
    ``((r1 << 32) + r2) mod (2^61 - 1)`` with r1, r2 uniform integers in
    [0, 2^31 - 2], the draw the hash family of Sec. 4.1 makes for its table A.
    """
    g = rng(seed)
    r = g.integers(0, (1 << 31) - 1, size=(H, 3, order, 2), dtype=np.uint64)
    A = ((r[..., 0] << np.uint64(32)) + r[..., 1]) % np.uint64(MERSENNE61)
    return np.ascontiguousarray(A, dtype=np.uint64)


MLP_SIZES = (16, 64, 64, 1)


def mlp_param_count(sizes=MLP_SIZES) -> int:
    return sum(sizes[i] * sizes[i + 1] + sizes[i + 1] for i in range(len(sizes) - 1))


def mlp_init(seed: int, sizes=MLP_SIZES) -> np.ndarray:
    """He-uniform initial weights, packed layer by layer as [W (out x in, row-major), b]."""
    g = rng(seed)
    parts = []
    for i in range(len(sizes) - 1):
        fan_in, fan_out = sizes[i], sizes[i + 1]
        bound = math.sqrt(6.0 / fan_in)
        parts.append(g.uniform(-bound, bound, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


@dataclass(frozen=True)
class NetSpec:
    """One network of the uneven batch."""
    n: int
    m: int
    T: int
    kind: str  # "uniform" or "activity"
    seed: int

    def generate(self):
        if self.kind == "uniform":
            return uniform_pairs(self.n, self.m, self.T, self.seed)
        return activity_driven(self.n, self.m, self.T, self.seed)


def batched_suite(B: int = 256, seed: int = 4000, n_range=(500, 20000),
                  m_range=(10_000, 1_000_000)) -> list[NetSpec]:
    """``B`` uneven networks: n and m log-uniform, even index uniform pairs,
    odd index activity-driven."""
    g = rng(seed)
    ln = g.uniform(math.log(n_range[0]), math.log(n_range[1]), size=B)
    lm = g.uniform(math.log(m_range[0]), math.log(m_range[1]), size=B)
    specs = []
    for b in range(B):
        n = int(round(math.exp(ln[b])))
        m = int(round(math.exp(lm[b])))
        if b % 2 == 0:
            specs.append(NetSpec(n, m, max(1, -(-m // 2)), "uniform", seed + b))
        else:
            specs.append(NetSpec(n, m, max(1, -(-m // 10)), "activity", seed + b))
    return specs


# Named workloads (sizes follow the paper's setting and the project's
# benchmark table; see the design doc for the recipe).
WORKLOADS = {
    "uniform_n1000_m20000": dict(kind="uniform", n=1000, m=20_000, T=10_000, seed=1),
    "activity_n100000_m10M": dict(kind="activity", n=100_000, m=10_000_000, T=1_000_000, seed=2),
    "activity_n1M_m100M": dict(kind="activity", n=1_000_000, m=100_000_000, T=10_000_000, seed=3),
    "activity_n20000_m1M": dict(kind="activity", n=20_000, m=1_000_000, T=100_000, seed=5000),
}


def make_workload(name: str, progress=None, **override):
    w = dict(WORKLOADS[name])
    w.update(override)
    if w["kind"] == "uniform":
        return uniform_pairs(w["n"], w["m"], w["T"], w["seed"])
    if w["kind"] == "activity":
        return activity_driven(w["n"], w["m"], w["T"], w["seed"], progress=progress)
    raise ValueError(w["kind"])
