"""Contact-layer generators (households, workplaces, Chung-Lu community).

The paper runs its simulator on multi-layer contact networks built from
census and mobility data (Section 3.1 "interaction networks as adjacency
matrices"; Section 4 and Appendix E describe the data).  Those data are not
available, so these generators stand in for them with the structure the
workload descriptions ask for:

* households: cliques of size uniform 1..6 over consecutive agent ids (a
  synthetic census enumerates people household by household);
* workplaces: cliques of size uniform 5..50 over a seeded random subset
  covering a given fraction of agents;
* community: a Chung-Lu graph whose expected degrees follow a power law
  with exponent gamma, scaled to a target mean, optionally capped.

Every generator returns undirected pairs ``(a, b)`` with ``a != b``;
:func:`to_symmetric_coo` turns a list of layers into the directed COO with
both directions that the simulator consumes.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Population:
    """Static agent attributes: age group per agent and population offsets."""

    n_agents: int
    age: np.ndarray  # uint8 [n_agents]
    pop_offsets: np.ndarray  # int32 [n_pops + 1]

    @property
    def n_pops(self) -> int:
        return len(self.pop_offsets) - 1


def _clique_pairs(members_by_group: list[np.ndarray]) -> tuple[np.ndarray, np.ndarray]:
    """All unordered pairs inside each group; groups of equal size are
    expanded together so the work stays vectorised."""
    a_parts, b_parts = [], []
    by_size: dict[int, list[np.ndarray]] = {}
    for g in members_by_group:
        if len(g) >= 2:
            by_size.setdefault(len(g), []).append(g)
    for s, groups in sorted(by_size.items()):
        mat = np.stack(groups)  # [n_groups, s]
        iu, ju = np.triu_indices(s, 1)
        a_parts.append(mat[:, iu].reshape(-1))
        b_parts.append(mat[:, ju].reshape(-1))
    if not a_parts:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(a_parts), np.concatenate(b_parts)


def _split_sizes(n: int, rng: np.random.Generator, lo: int, hi: int) -> np.ndarray:
    """Consecutive group sizes uniform on {lo..hi} that exactly cover n
    (the last group takes the remainder)."""
    est = max(1, int(2 * n / (lo + hi)) + 16)
    sizes = rng.integers(lo, hi + 1, size=est)
    while sizes.sum() < n:
        sizes = np.concatenate([sizes, rng.integers(lo, hi + 1, size=est)])
    c = np.cumsum(sizes)
    k = int(np.searchsorted(c, n))  # first index where cumsum >= n
    sizes = sizes[: k + 1].copy()
    sizes[-1] -= int(c[k] - n)
    return sizes[sizes > 0]


def households(n: int, rng: np.random.Generator, lo: int = 1, hi: int = 6):
    """Households: fully connected groups of size uniform lo..hi over
    consecutive agent ids 0..n-1."""
    sizes = _split_sizes(n, rng, lo, hi)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    # the pairs _clique_pairs would list for the groups arange(start, start + size)
    a_parts, b_parts = [], []
    for s in np.unique(sizes):
        if s < 2:
            continue
        mat = starts[sizes == s][:, None] + np.arange(s)  # [n_groups, s]
        iu, ju = np.triu_indices(s, 1)
        a_parts.append(mat[:, iu].reshape(-1))
        b_parts.append(mat[:, ju].reshape(-1))
    if not a_parts:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(a_parts), np.concatenate(b_parts)


def workplaces(n: int, rng: np.random.Generator, coverage: float = 0.6, lo: int = 5, hi: int = 50):
    """Workplaces: cliques of size uniform lo..hi over a random subset of
    round(coverage * n) agents."""
    n_cov = int(round(coverage * n))
    members = rng.permutation(n)[:n_cov]
    sizes = _split_sizes(n_cov, rng, lo, hi)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    groups = [members[s0 : s0 + s] for s0, s in zip(starts, sizes)]
    return _clique_pairs(groups)


def _searchsorted_right(cdf: np.ndarray, r: np.ndarray) -> np.ndarray:
    """``np.searchsorted(cdf, r, side="right")`` for queries in [0, 1), via a
    table of the answers at the 2^bits grid points: the answer for r in
    [k/L, (k+1)/L) lies between the table entries k and k+1, and the few
    cdf values in between are stepped over one at a time.  The grid points
    and r * L are exact, so the result is identical; random queries into a
    large cdf no longer miss the cache at every bisection step."""
    L = 1 << min(26, max(16, len(cdf).bit_length() + 1))  # about two grid points per cdf value
    tab = np.searchsorted(cdf, np.arange(L + 1, dtype=np.float64) / L, side="right")
    k = (r * L).astype(np.int64)
    pos = tab[k]
    end = tab[k + 1]
    act = np.nonzero(pos < end)[0]
    while len(act):
        step = cdf[pos[act]] <= r[act]
        act = act[step]
        pos[act] += 1
        act = act[pos[act] < end[act]]
    return pos


def chung_lu(n: int, rng: np.random.Generator, gamma: float, mean_deg: float, cap: float | None = None):
    """Chung-Lu community layer.

    Expected degrees w_i follow a Pareto tail with density exponent gamma,
    are scaled to ``mean_deg`` and capped at ``cap`` (rescaled after
    capping).  round(n * mean_deg / 2) endpoint pairs are drawn with
    probability proportional to w; self-loops are dropped and duplicate
    pairs merged, so the realised mean degree is slightly below target.
    """
    u = rng.random(n)
    w = (1.0 - u) ** (-1.0 / (gamma - 1.0))
    w *= mean_deg / w.mean()
    if cap is not None:
        for _ in range(20):
            w = np.minimum(w, cap)
            w *= mean_deg / w.mean()
        w = np.minimum(w, cap)
    m = int(round(n * mean_deg / 2))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    a = _searchsorted_right(cdf, rng.random(m))
    b = _searchsorted_right(cdf, rng.random(m))
    a = np.minimum(a, n - 1)
    b = np.minimum(b, n - 1)
    keep = a != b
    a, b = a[keep], b[keep]
    lo_, hi_ = np.minimum(a, b).astype(np.int64), np.maximum(a, b).astype(np.int64)
    key = np.unique(lo_ * n + hi_)
    return key // n, key % n


def complete_pairs(n: int):
    """Complete graph on n agents."""
    iu, ju = np.triu_indices(n, 1)
    return iu.astype(np.int64), ju.astype(np.int64)


def quantized_unit_weights(rng: np.random.Generator, m: int) -> np.ndarray:
    """Weights uniform on (0, 1] restricted to the grid k * 2^-24,
    k in 1..2^24.  Every value is an exact float32, and sums of them are
    exact in float64, so a weighted neighbour sum does not depend on the
    order in which it is formed."""
    k = rng.integers(1, (1 << 24) + 1, size=m, dtype=np.int64)
    return (k.astype(np.float64) * 2.0**-24).astype(np.float32)


def to_symmetric_coo(layers, offset: int = 0):
    """Directed COO with both directions of every undirected pair.

    ``layers`` is a list of ``(a, b, w)`` where ``w`` is either a scalar
    weight for the whole layer or a float32 array with one weight per pair.
    Returns ``(src, dst, w)`` as int32, int32, float32 arrays; the pair
    (a, b, w) is emitted as a->b followed, after all forward edges of the
    layer, by b->a.
    """
    srcs, dsts, ws = [], [], []
    for a, b, w in layers:
        a = np.asarray(a, np.int64) + offset
        b = np.asarray(b, np.int64) + offset
        if np.isscalar(w):
            wa = np.full(len(a), np.float32(w), np.float32)
        else:
            wa = np.asarray(w, np.float32)
        srcs += [a, b]
        dsts += [b, a]
        ws += [wa, wa]
    if not srcs:
        z = np.zeros(0, np.int32)
        return z, z.copy(), np.zeros(0, np.float32)
    return (
        np.concatenate(srcs).astype(np.int32),
        np.concatenate(dsts).astype(np.int32),
        np.concatenate(ws).astype(np.float32),
    )


def location_visits(pop: Population, rng: np.random.Generator, *, school=(100, 400), work=(5, 60),
                    work_share: float = 0.7, leisure=(10, 80), leisure_share: float = 0.5, kmax: int = 16):
    """One day of agent-location visits shaped like the JUNE model's venues
    (the agent-location bipartite graph of the paper's GradABM-JUNE
    discussion; no census data here, so sizes are drawn):

    * schools: every agent of age groups 0-1, in venues of size uniform on
      ``school``;
    * workplaces: a ``work_share`` subset of age groups 2-5, venues of size
      uniform on ``work``;
    * leisure: a ``leisure_share`` subset of everyone, venues of size
      uniform on ``leisure``.

    Venues never span populations; an agent visits at most one venue of each
    kind, so never one location twice.  Weights are k/64 with k uniform on
    1..kmax (exact products and sums in float64).  Returns
    ``(agent int32[V], location int32[V], weight float32[V], n_locations)``.
    """
    ag, lo = [], []
    n_loc = 0
    for p in range(pop.n_pops):
        a0, a1 = int(pop.pop_offsets[p]), int(pop.pop_offsets[p + 1])
        ids = np.arange(a0, a1, dtype=np.int64)
        age = pop.age[a0:a1]
        kinds = ((ids[age <= 1], 1.0, school), (ids[(age >= 2) & (age <= 5)], work_share, work),
                 (ids, leisure_share, leisure))
        for cand, share, (s_lo, s_hi) in kinds:
            members = rng.permutation(cand)[: int(round(share * len(cand)))]
            if len(members) == 0:
                continue
            sizes = _split_sizes(len(members), rng, s_lo, s_hi)
            ag.append(members)
            lo.append(n_loc + np.repeat(np.arange(len(sizes)), sizes))
            n_loc += len(sizes)
    agent = np.concatenate(ag).astype(np.int32) if ag else np.zeros(0, np.int32)
    loc = np.concatenate(lo).astype(np.int32) if lo else np.zeros(0, np.int32)
    w = (rng.integers(1, kmax + 1, size=len(agent)) / 64.0).astype(np.float32)
    return agent, loc, w, n_loc


def location_degree(n_agents: int, visits) -> np.ndarray:
    """Per-agent weighted degree the visits stand for: for agent i, the sum
    over its locations l of w_il times the other visitors' weights at l
    (the contact weight of i with j being the sum of w_il * w_jl)."""
    agent, loc, w = visits[0], visits[1], np.asarray(visits[2], np.float64)
    n_loc = int(loc.max()) + 1 if len(loc) else 0
    tot = np.bincount(loc, weights=w, minlength=n_loc)
    return np.bincount(agent, weights=w * (tot[loc] - w), minlength=n_agents)
