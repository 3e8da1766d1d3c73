"""Seeded synthetic graph layouts.

This module only draws inputs: node coordinates (integer-valued float32) and
undirected edge lists (int32 ``src``/``dst``).  It contains none of the metric
arithmetic, so both the CPU oracle and the HIP path can be fed from it.

Every generator takes a ``seed`` and uses one ``numpy.random.Generator``
(PCG64).  The workloads follow the paper's setting -- random layouts of sparse
social / citation graphs (Section 4, Table 1) -- at the sizes of the five
evaluation workloads:

* ``uniform_layout``      |V|=1,000, |E|=2,000 uniform random edges, coords in
                          [0,4096)^2, diameter 8;
* ``ba_cluster_layout``   |V|=50,000 preferential attachment (m=3, seed K4),
                          64 Gaussian clusters (sigma 2% of 2^20), diameter 64;
* ``batch_layouts``       512 layouts, |V| log-uniform in [200, 20000],
                          |E| = U[1.5,4] |V|, coords in [0,2^16)^2;
* ``geometric_layout``    |V|=20,000 random geometric graph, mean degree ~6,
                          coords in [0,2^16)^2;
* ``powerlaw_layout``     |V|=1,000,000, |E|=3,000,000 Chung-Lu power law
                          (gamma 2.3, expected degree capped at 10,000),
                          hub-heavy Gaussian clusters in [0,2^20)^2.

Hand-made layouts (convex K4, star, grid, K_n in convex position, two-row
complete bipartite, hubs beside a hatch) are here too, for the closed-form
checks.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

COORD_LIMIT = 1 << 20          # coordinates are integers with |c| <= 2^20
IDEAL_ANGLE = 70.0 * math.pi / 180.0


@dataclass
class Layout:
    """One graph layout: float32 integer-valued coords, int32 edge ends."""
    x: np.ndarray
    y: np.ndarray
    src: np.ndarray
    dst: np.ndarray
    diameter: float = 8.0
    ideal_angle: float = IDEAL_ANGLE
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.src.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.x, self.y, self.src, self.dst):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(repr((self.diameter, self.ideal_angle)).encode())
        return h.hexdigest()[:16]


def _finish(x, y, src, dst, **kw) -> Layout:
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float32))
    src = np.ascontiguousarray(np.asarray(src, dtype=np.int32))
    dst = np.ascontiguousarray(np.asarray(dst, dtype=np.int32))
    return Layout(x, y, src, dst, **kw)


def distinct_random_edges(rng: np.random.Generator, n_nodes: int, n_edges: int,
                          weights: np.ndarray | None = None):
    """Draw ``n_edges`` distinct unordered pairs without self-loops.

    Endpoints are uniform (or proportional to ``weights``); draws that repeat
    an earlier pair or are loops are rejected, keeping the order of first
    appearance so the result depends only on the seed.
    """
    if n_edges > n_nodes * (n_nodes - 1) // 2:
        raise ValueError("more edges than node pairs")
    if n_edges == 0:
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64)
    p = None
    if weights is not None:
        p = np.asarray(weights, dtype=np.float64)
        p = p / p.sum()
    keys_seen = np.empty(0, dtype=np.int64)
    src_out, dst_out = [], []
    have = 0
    while have < n_edges:
        batch = int((n_edges - have) * 1.3) + 64
        if p is None:
            u = rng.integers(0, n_nodes, size=batch, dtype=np.int64)
            v = rng.integers(0, n_nodes, size=batch, dtype=np.int64)
        else:
            u = rng.choice(n_nodes, size=batch, p=p)
            v = rng.choice(n_nodes, size=batch, p=p)
        keep = u != v
        u, v = u[keep], v[keep]
        key = np.minimum(u, v) * n_nodes + np.maximum(u, v)
        _, first = np.unique(key, return_index=True)
        first.sort()
        u, v, key = u[first], v[first], key[first]
        fresh = ~np.isin(key, keys_seen)
        u, v, key = u[fresh], v[fresh], key[fresh]
        take = min(n_edges - have, u.shape[0])
        src_out.append(u[:take])
        dst_out.append(v[:take])
        keys_seen = np.concatenate([keys_seen, key[:take]])
        have += take
    return np.concatenate(src_out), np.concatenate(dst_out)


def uniform_layout(n_nodes: int = 1000, n_edges: int = 2000, extent: int = 4096,
                   diameter: float = 8.0, seed: int = 0) -> Layout:
    """Uniform random edges; node coordinates uniform integers in [0,extent)^2."""
    rng = np.random.default_rng(seed)
    x = rng.integers(0, extent, size=n_nodes)
    y = rng.integers(0, extent, size=n_nodes)
    s, d = distinct_random_edges(rng, n_nodes, n_edges)
    return _finish(x, y, s, d, diameter=diameter,
                   name=f"uniform_V{n_nodes}_E{n_edges}",
                   meta=dict(seed=seed, extent=extent))


def _reflect(v: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """Fold values into [lo, hi] by mirror reflection at both ends."""
    span = hi - lo
    w = np.mod(v - lo, 2 * span)
    return lo + np.where(w > span, 2 * span - w, w)


def cluster_coords(rng: np.random.Generator, n_nodes: int, n_clusters: int = 64,
                   extent: int = COORD_LIMIT, sigma_frac: float = 0.02,
                   node_weight: np.ndarray | None = None):
    """Gaussian-cluster coordinates, rounded to integers and reflected into
    [0, extent-1].  With ``node_weight`` the offset of node i shrinks as
    sigma / sqrt(1 + w_i / mean(w)), so heavy nodes (hubs) sit densely at
    the cluster centres."""
    cx = rng.uniform(0, extent, size=n_clusters)
    cy = rng.uniform(0, extent, size=n_clusters)
    c = rng.integers(0, n_clusters, size=n_nodes)
    sigma = np.full(n_nodes, sigma_frac * extent)
    if node_weight is not None:
        w = np.asarray(node_weight, dtype=np.float64)
        sigma = sigma / np.sqrt(1.0 + w / w.mean())
    x = np.rint(cx[c] + rng.normal(0.0, 1.0, size=n_nodes) * sigma)
    y = np.rint(cy[c] + rng.normal(0.0, 1.0, size=n_nodes) * sigma)
    return _reflect(x, 0, extent - 1), _reflect(y, 0, extent - 1)


def preferential_attachment_edges(rng: np.random.Generator, n_nodes: int, m: int = 3):
    """Barabasi-Albert graph grown from a K_{m+1} seed; each new node links to
    m distinct earlier nodes chosen proportionally to degree (uniform draws
    from the list of all edge endpoints so far)."""
    k = m + 1
    src, dst = [], []
    for i in range(k):
        for j in range(i + 1, k):
            src.append(i)
            dst.append(j)
    ends = np.empty(2 * (len(src) + m * (n_nodes - k)), dtype=np.int64)
    n_ends = 0
    for a, b in zip(src, dst):
        ends[n_ends] = a
        ends[n_ends + 1] = b
        n_ends += 2
    # pre-drawn uniforms keep the loop cheap; redraw on collisions
    pool = rng.random(size=4 * m * n_nodes + 1024)
    pi = 0
    for v in range(k, n_nodes):
        chosen: list[int] = []
        while len(chosen) < m:
            if pi >= pool.shape[0]:
                pool = rng.random(size=pool.shape[0])
                pi = 0
            t = int(ends[int(pool[pi] * n_ends)])
            pi += 1
            if t not in chosen:
                chosen.append(t)
        for t in chosen:
            src.append(v)
            dst.append(t)
            ends[n_ends] = v
            ends[n_ends + 1] = t
            n_ends += 2
    return np.asarray(src, dtype=np.int64), np.asarray(dst, dtype=np.int64)


def ba_cluster_layout(n_nodes: int = 50_000, m: int = 3, n_clusters: int = 64,
                      extent: int = COORD_LIMIT, diameter: float = 64.0,
                      seed: int = 0) -> Layout:
    """Preferential-attachment graph on Gaussian-cluster coordinates."""
    rng = np.random.default_rng(seed)
    s, d = preferential_attachment_edges(rng, n_nodes, m)
    x, y = cluster_coords(rng, n_nodes, n_clusters, extent)
    return _finish(x, y, s, d, diameter=diameter,
                   name=f"ba{m}_cluster{n_clusters}_V{n_nodes}",
                   meta=dict(seed=seed, extent=extent))


def batch_layouts(n_layouts: int = 512, v_min: int = 200, v_max: int = 20_000,
                  extent: int = 1 << 16, diameter: float = 8.0,
                  seed: int = 0) -> list[Layout]:
    """Many layouts of uneven size: |V| log-uniform, |E| = U[1.5,4] |V|."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n_layouts):
        v = int(round(math.exp(rng.uniform(math.log(v_min), math.log(v_max)))))
        e = int(round(rng.uniform(1.5, 4.0) * v))
        x = rng.integers(0, extent, size=v)
        y = rng.integers(0, extent, size=v)
        s, d = distinct_random_edges(rng, v, e)
        out.append(_finish(x, y, s, d, diameter=diameter,
                           name=f"batch{b}_V{v}_E{e}", meta=dict(seed=seed, index=b)))
    return out


def concat_layouts(layouts: list[Layout]):
    """Concatenate layouts into one node/edge array set with offsets
    (edge ends stay local to their own layout)."""
    node_off = np.zeros(len(layouts) + 1, dtype=np.int64)
    edge_off = np.zeros(len(layouts) + 1, dtype=np.int64)
    for i, L in enumerate(layouts):
        node_off[i + 1] = node_off[i] + L.n_nodes
        edge_off[i + 1] = edge_off[i] + L.n_edges
    x = np.concatenate([L.x for L in layouts]).astype(np.float32)
    y = np.concatenate([L.y for L in layouts]).astype(np.float32)
    src = np.concatenate([L.src for L in layouts]).astype(np.int32)
    dst = np.concatenate([L.dst for L in layouts]).astype(np.int32)
    return x, y, src, dst, node_off, edge_off


def geometric_layout(n_nodes: int = 20_000, target_edges: int = 60_000,
                     extent: int = 1 << 16, seed: int = 0) -> Layout:
    """Random geometric graph: uniform integer points joined when their
    distance is at most r, with r bisected so |E| is closest to the target."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    x = rng.integers(0, extent, size=n_nodes).astype(np.float64)
    y = rng.integers(0, extent, size=n_nodes).astype(np.float64)
    tree = cKDTree(np.stack([x, y], axis=1))
    lo, hi = 0.0, 4.0 * math.sqrt(target_edges * 2 / n_nodes * extent * extent / (math.pi * n_nodes))
    best = None
    for _ in range(40):
        r = 0.5 * (lo + hi)
        cnt = tree.count_neighbors(tree, r) - n_nodes
        cnt //= 2
        if best is None or abs(cnt - target_edges) < abs(best[1] - target_edges):
            best = (r, cnt)
        if cnt < target_edges:
            lo = r
        else:
            hi = r
    r = best[0]
    pairs = tree.query_pairs(r, output_type="ndarray")
    pairs = pairs[np.lexsort((pairs[:, 1], pairs[:, 0]))]
    return _finish(x, y, pairs[:, 0], pairs[:, 1], diameter=8.0,
                   name=f"rgg_V{n_nodes}_E{pairs.shape[0]}",
                   meta=dict(seed=seed, radius=r, extent=extent))


def powerlaw_layout(n_nodes: int = 1_000_000, n_edges: int = 3_000_000,
                    gamma: float = 2.3, max_degree: float = 10_000.0,
                    n_clusters: int = 64, extent: int = COORD_LIMIT,
                    diameter: float = 16.0, seed: int = 0) -> Layout:
    """Chung-Lu graph: expected degree w_i ~ i^(-1/(gamma-1)) capped at
    ``max_degree`` and scaled to sum 2|E|; distinct non-loop edges drawn with
    endpoint probability proportional to w.  Coordinates are hub-heavy
    Gaussian clusters (see ``cluster_coords``)."""
    rng = np.random.default_rng(seed)
    i = np.arange(1, n_nodes + 1, dtype=np.float64)
    w = i ** (-1.0 / (gamma - 1.0))
    w *= 2.0 * n_edges / w.sum()
    for _ in range(50):                      # cap, then rescale the rest
        capped = w > max_degree
        if not capped.any():
            break
        w[capped] = max_degree
        free = ~capped
        w[free] *= (2.0 * n_edges - w[capped].sum()) / w[free].sum()
    perm = rng.permutation(n_nodes)          # hubs get random ids
    w = w[perm]
    s, d = distinct_random_edges(rng, n_nodes, n_edges, weights=w)
    x, y = cluster_coords(rng, n_nodes, n_clusters, extent, node_weight=w)
    return _finish(x, y, s, d, diameter=diameter,
                   name=f"powerlaw{gamma}_V{n_nodes}_E{n_edges}",
                   meta=dict(seed=seed, extent=extent))


def force_directed_coords(rng: np.random.Generator, n_nodes: int, src: np.ndarray,
                          dst: np.ndarray, iterations: int = 60, extent: int = 1 << 16,
                          block: int = 1024) -> tuple[np.ndarray, np.ndarray]:
    """Fruchterman-Reingold spring embedding (the layout algorithm of the
    paper's force-directed experiment): on a unit square, all node pairs
    repel with k^2/d and edges attract with d^2/k, k = sqrt(1/|V|); each
    iteration moves every node along its net force by at most a temperature
    that cools linearly from 0.1 to 0.  The result is scaled into
    [0, extent)^2 and rounded to integers.  Elementwise numpy only (the
    repulsion in row blocks), so the output is the same on every x86 host."""
    pos = rng.random((n_nodes, 2))
    k = math.sqrt(1.0 / max(n_nodes, 1))
    s = np.asarray(src, dtype=np.int64)
    d = np.asarray(dst, dtype=np.int64)
    for it in range(iterations):
        t = 0.1 * (1.0 - it / iterations)
        disp = np.zeros_like(pos)
        for b0 in range(0, n_nodes, block):
            p = pos[b0:b0 + block]
            dx = p[:, None, 0] - pos[None, :, 0]
            dy = p[:, None, 1] - pos[None, :, 1]
            d2 = dx * dx + dy * dy
            d2[d2 < 1e-12] = 1e-12                   # self and coincident pairs
            f = (k * k) / d2                         # k^2/d along the unit vector d/|d|
            f[np.arange(p.shape[0]), np.arange(b0, b0 + p.shape[0])] = 0.0
            disp[b0:b0 + block, 0] += (dx * f).sum(axis=1)
            disp[b0:b0 + block, 1] += (dy * f).sum(axis=1)
        ex = pos[s, 0] - pos[d, 0]
        ey = pos[s, 1] - pos[d, 1]
        el = np.sqrt(ex * ex + ey * ey)
        fa = el / k                                  # d^2/k along the unit vector
        np.subtract.at(disp[:, 0], s, ex * fa)
        np.subtract.at(disp[:, 1], s, ey * fa)
        np.add.at(disp[:, 0], d, ex * fa)
        np.add.at(disp[:, 1], d, ey * fa)
        dl = np.sqrt((disp * disp).sum(axis=1))
        step = np.minimum(dl, t) / np.maximum(dl, 1e-300)
        pos += disp * step[:, None]
        pos = np.clip(pos, 0.0, 1.0)
    lo, hi = pos.min(axis=0), pos.max(axis=0)
    scale = (extent - 1) / np.maximum(hi - lo, 1e-300)
    xy = np.rint((pos - lo) * scale).astype(np.int64)
    return xy[:, 0], xy[:, 1]


def community_edges(rng: np.random.Generator, n_nodes: int, n_groups: int, intra: int,
                    inter: int) -> tuple[np.ndarray, np.ndarray]:
    """Planted-partition graph: nodes split into n_groups equal groups,
    `intra` distinct edges drawn uniformly inside each group and `inter`
    distinct edges between different groups."""
    group = np.arange(n_nodes) % n_groups
    src, dst = [], []
    for g in range(n_groups):
        members = np.flatnonzero(group == g)
        a, b = distinct_random_edges(rng, members.shape[0], intra)
        src.append(members[a])
        dst.append(members[b])
    seen = set()
    while len(seen) < inter:
        a, b = (int(v) for v in rng.integers(0, n_nodes, size=2))
        if group[a] == group[b] or (min(a, b), max(a, b)) in seen:
            continue
        seen.add((min(a, b), max(a, b)))
    e = np.array(sorted(seen), dtype=np.int64).reshape(-1, 2)
    src.append(e[:, 0])
    dst.append(e[:, 1])
    return np.concatenate(src), np.concatenate(dst)


def force_directed_layout(n_nodes: int = 4000, n_groups: int = 16, intra: int = 5000,
                          inter: int = 5000, iterations: int = 60, extent: int = 1 << 16,
                          diameter: float = 64.0, seed: int = 0) -> Layout:
    """A community-structured graph of the size of the paper's smallest
    dataset (4,000 nodes, 16 groups, 85,000 edges by default) drawn by
    Fruchterman-Reingold: groups become clusters, most edges are short, as in
    layouts meant for reading."""
    rng = np.random.default_rng(seed)
    s, d = community_edges(rng, n_nodes, n_groups, intra, inter)
    x, y = force_directed_coords(rng, n_nodes, s, d, iterations, extent)
    return _finish(x, y, s, d, diameter=diameter,
                   name=f"fr_groups{n_groups}_V{n_nodes}_E{s.shape[0]}",
                   meta=dict(seed=seed, extent=extent, iterations=iterations))


# ---------------------------------------------------------------- hand cases

def convex_k4() -> Layout:
    """K4 on the corners of a square: exactly the two diagonals cross."""
    x = [0, 4, 4, 0]
    y = [0, 0, 4, 4]
    s, d = zip(*[(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)])
    return _finish(x, y, s, d, name="convex_k4")


def star(n_leaves: int = 8, seed: int = 0) -> Layout:
    """A centre joined to ``n_leaves`` leaves on distinct directions."""
    rng = np.random.default_rng(seed)
    ang = np.sort(rng.permutation(360)[:n_leaves]) * (2 * math.pi / 360)
    x = np.concatenate([[1000], np.rint(1000 + 500 * np.cos(ang))])
    y = np.concatenate([[1000], np.rint(1000 + 500 * np.sin(ang))])
    s = np.zeros(n_leaves, dtype=np.int64)
    d = np.arange(1, n_leaves + 1)
    return _finish(x, y, s, d, name=f"star{n_leaves}")


def grid(rows: int = 5, cols: int = 6, spacing: int = 10) -> Layout:
    """Straight-line drawing of the rows x cols grid graph."""
    idx = np.arange(rows * cols).reshape(rows, cols)
    x = (np.tile(np.arange(cols), rows) * spacing)
    y = (np.repeat(np.arange(rows), cols) * spacing)
    s, d = [], []
    for r in range(rows):
        for c in range(cols):
            if c + 1 < cols:
                s.append(idx[r, c]); d.append(idx[r, c + 1])
            if r + 1 < rows:
                s.append(idx[r, c]); d.append(idx[r + 1, c])
    return _finish(x, y, s, d, name=f"grid{rows}x{cols}")


def complete_convex(n: int) -> Layout:
    """K_n on the points (i, i^2): convex position, so C(n,4) crossings."""
    x = np.arange(n)
    y = np.arange(n) ** 2
    s, d = zip(*[(i, j) for i in range(n) for j in range(i + 1, n)])
    return _finish(x, y, s, d, name=f"K{n}_parabola")


def two_row_bipartite(m: int, n: int) -> Layout:
    """K_{m,n} with one side on y=0 and the other on y=1: C(m,2) C(n,2)
    crossings."""
    x = np.concatenate([np.arange(m), np.arange(n)])
    y = np.concatenate([np.zeros(m), np.ones(n)])
    s, d = zip(*[(i, m + j) for i in range(m) for j in range(n)])
    return _finish(x, y, s, d, name=f"K{m},{n}_two_rows")


def hatch_and_stars(n_lines: int, n_stars: int, q: int, r: int, seed: int = 0) -> Layout:
    """Hubs next to a hatch, with node ids and edge order shuffled.

    Hatch: n_lines horizontal segments (y = 2i + 1, x in [0, 2 n_lines]) and
    n_lines vertical ones (x = 2j + 1, y in [0, 2 n_lines]); every
    horizontal crosses every vertical at an interior point, at 90 degrees.
    Star k, to the right of the hatch: a centre (cx, cy) joined to leaves
    (cx - r, cy + t) and (cx + r, cy + t) for even t in [-2q, 2q], and a bar
    y = cy + 1 over x in [cx - r - 1, cx + r + 1].  The bar crosses, at an
    interior point of both, exactly the spokes with t >= 2 (2q per star, at
    the angle atan(t / r)); the spokes share the centre, and nothing else
    meets.  So there are n_lines^2 + 2 q n_stars crossings, and
    4 n_lines + n_stars (4q + 3) nodes and 2 n_lines + n_stars (4q + 3)
    edges, the centres of degree 4q + 2.
    """
    n = n_lines
    xs, ys, es = [], [], []
    m = 0

    def seg(x0, y0, x1, y1):
        nonlocal m
        xs.extend((x0, x1)); ys.extend((y0, y1)); es.append((m, m + 1)); m += 2

    for i in range(n):
        seg(0, 2 * i + 1, 2 * n, 2 * i + 1)
        seg(2 * i + 1, 0, 2 * i + 1, 2 * n)
    cx = 2 * n + r + 8
    for k in range(n_stars):
        cy = 2 * q + 4 + k * (4 * q + 8)
        c = m
        xs.append(cx); ys.append(cy); m += 1
        for t in range(-2 * q, 2 * q + 1, 2):
            for side in (-r, r):
                xs.append(cx + side); ys.append(cy + t); es.append((c, m)); m += 1
        seg(cx - r - 1, cy + 1, cx + r + 1, cy + 1)
    assert max(max(xs), max(ys)) < COORD_LIMIT
    rng = np.random.default_rng(seed)
    perm = rng.permutation(m)                 # node i gets id perm[i]
    x = np.empty(m); y = np.empty(m)
    x[perm] = xs; y[perm] = ys
    e = perm[np.asarray(es, dtype=np.int64)]
    e = e[rng.permutation(len(es))]
    flip = rng.random(len(es)) < 0.5
    s = np.where(flip, e[:, 1], e[:, 0]); d = np.where(flip, e[:, 0], e[:, 1])
    return _finish(x, y, s, d, name=f"hatch{n}_stars{n_stars}x{4 * q + 2}_s{seed}")


def square_lattice(k: int, spacing: int, diameter: float) -> Layout:
    """k x k lattice of nodes (no edges) for the occlusion closed form."""
    x = np.tile(np.arange(k), k) * spacing
    y = np.repeat(np.arange(k), k) * spacing
    e = np.zeros(0, dtype=np.int64)
    return _finish(x, y, e, e, diameter=diameter, name=f"lattice{k}_s{spacing}")


WORKLOADS = {
    "uniform_V1000_E2000": lambda seed=0: uniform_layout(seed=seed),
    "ba_cluster_V50000_E149994": lambda seed=0: ba_cluster_layout(seed=seed),
    "rgg_V20000_E60000": lambda seed=0: geometric_layout(seed=seed),
    "powerlaw_V1000000_E3000000": lambda seed=0: powerlaw_layout(seed=seed),
}
