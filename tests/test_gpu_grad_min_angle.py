"""Minimum-angle term w_m (1 - M_a) of rb_loss_grad / rb_loss_grad_pruned
against the oracle.

* loss and gradient of the term alone (w_angle = w_length = 0) and of the
  full loss, plain and pruned, against the oracle's analytic gradient on
  uniform layouts, a power-law layout and stars whose hub degree takes each
  of the three vertex paths (thread per vertex up to degree 16, a block
  sorting in LDS up to 2048, a block sorting in place above);
* the kinks: a lattice where every smallest gap is attained several times,
  coincident directions (a zero smallest gap), zero-length edges;
* FP64 central finite differences (step 0.1) of the oracle's term on 64
  sampled vertices.
Tolerance (floating point): |g - g_ref| <= 1e-5 max(|g_ref|, 1e-3 max|g_ref|).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2411_09809_amd import gen

pytestmark = pytest.mark.gpu
IDEAL = gen.IDEAL_ANGLE


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


def close(g, ref):
    cap = 1e-3 * np.abs(ref).max() if ref.size else 0.0
    return np.abs(g - ref) <= 1e-5 * np.maximum(np.abs(ref), cap)


def run(L, w, pruned=False):
    from paper_2411_09809_amd import metrics, optim
    D = metrics.DeviceLayout.from_host(L)
    loss, gx, gy, cnt = optim.loss_grad(D.x, D.y, D.src, D.dst, IDEAL, w[0], w[1],
                                        pruned=pruned, w_min_angle=w[2])
    return float(loss), gx.cpu().numpy(), gy.cpu().numpy(), int(cnt)


def check(L, w, pruned=False, tag=""):
    S = oracle.crossing_pairs(L.x, L.y, L.src, L.dst)
    f_ref, gx_ref, gy_ref = oracle.loss_grad(L.x, L.y, L.src, L.dst, S, IDEAL, *w)
    f, gx, gy, cnt = run(L, w, pruned)
    say(f"[ma-grad] {tag} V={L.n_nodes} E={L.n_edges} w={w} pruned={pruned} "
        f"loss={f:.15f} ref={f_ref:.15f}")
    assert cnt == S.shape[0]
    assert f == pytest.approx(f_ref, rel=1e-12, abs=1e-15)
    okx, oky = close(gx, gx_ref), close(gy, gy_ref)
    assert okx.all() and oky.all(), (np.abs(gx - gx_ref).max(), np.abs(gy - gy_ref).max(),
                                     np.abs(gx_ref).max())
    return gx_ref, gy_ref


def star(n_leaves, seed, extent=1 << 16, extra=(400, 900)):
    """A hub with n_leaves leaves at distinct random points, plus a random
    sparse graph on other nodes."""
    rng = np.random.default_rng(seed)
    V = 1 + n_leaves + extra[0]
    pts = rng.integers(0, extent * extent, size=2 * V)
    _, first = np.unique(pts, return_index=True)
    pts = pts[np.sort(first)][:V]                  # distinct points, in draw order
    assert pts.size == V
    x, y = pts % extent, pts // extent
    src = np.zeros(n_leaves, dtype=np.int64)
    dst = np.arange(1, n_leaves + 1)
    base = 1 + n_leaves
    a = rng.integers(0, extra[0], 3 * extra[1]) + base
    b = rng.integers(0, extra[0], 3 * extra[1]) + base
    keep = a != b
    pairs = np.unique(np.sort(np.stack([a[keep], b[keep]], 1), axis=1), axis=0)[:extra[1]]
    src = np.concatenate([src, pairs[:, 0]])
    dst = np.concatenate([dst, pairs[:, 1]])
    return gen._finish(x, y, src, dst, diameter=1.0, name=f"star{n_leaves}")


@pytest.mark.parametrize("pruned", [False, True])
@pytest.mark.parametrize("V,E,extent,seed", [(300, 700, 64, 1), (2000, 5000, 4096, 2),
                                             (1500, 3500, 1 << 16, 3)])
def test_term_alone_uniform(torch_mod, V, E, extent, seed, pruned):
    L = gen.uniform_layout(V, E, extent=extent, seed=seed)
    check(L, (0.0, 0.0, 1.0), pruned, "uniform")


@pytest.mark.parametrize("pruned", [False, True])
@pytest.mark.parametrize("leaves", [5, 40, 1000, 3000])
def test_term_alone_stars(torch_mod, leaves, pruned):
    """Hub degree 5 (thread path), 40 and 1000 (LDS sort), 3000 (in-place sort)."""
    check(star(leaves, seed=leaves), (0.0, 0.0, 2.0), pruned, f"star{leaves}")


def test_full_loss_with_term(torch_mod):
    L = gen.uniform_layout(2000, 5000, extent=4096, seed=4)
    for pruned in (False, True):
        check(L, (0.8, 1.3, 0.6), pruned, "full")


def test_power_law_layout(torch_mod):
    L = gen.WORKLOADS["ba_cluster_V50000_E149994"](seed=0)
    # the term alone: the oracle's crossing set is not needed
    from paper_2411_09809_amd import metrics, optim
    D = metrics.DeviceLayout.from_host(L)
    t_ref, gx_ref, gy_ref = oracle.min_angle_term(L.x, L.y, L.src, L.dst, 1.5, grad=True)
    for pruned in (False, True):
        loss, gx, gy, _ = optim.loss_grad(D.x, D.y, D.src, D.dst, IDEAL, 0.0, 0.0,
                                          pruned=pruned, w_min_angle=1.5)
        gx, gy = gx.cpu().numpy(), gy.cpu().numpy()
        say(f"[ma-grad] ba_cluster pruned={pruned} term={float(loss):.15f} ref={t_ref:.15f} "
            f"max deg={np.bincount(np.concatenate([L.src, L.dst])).max()}")
        assert float(loss) == pytest.approx(t_ref, rel=1e-12)
        assert close(gx, gx_ref).all() and close(gy, gy_ref).all()


def test_kinks_contribute_zero(torch_mod):
    # a square lattice: every interior smallest gap (pi/2) is attained 4 times,
    # borders 2 or 3 times, corners once (the gap pi/2 against 3 pi/2)
    k = 9
    ix, iy = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    x, y = (ix.ravel() * 10).astype(np.float64), (iy.ravel() * 10).astype(np.float64)
    idx = np.arange(k * k).reshape(k, k)
    src = np.concatenate([idx[:-1, :].ravel(), idx[:, :-1].ravel()])
    dst = np.concatenate([idx[1:, :].ravel(), idx[:, 1:].ravel()])
    L = gen._finish(x, y, src, dst, diameter=1.0, name="lattice")
    gx_ref, gy_ref = check(L, (0.0, 0.0, 1.0), False, "lattice")
    corners = [idx[0, 0], idx[0, -1], idx[-1, 0], idx[-1, -1]]
    mask = np.ones(k * k, dtype=bool)
    # only corners and their two lattice neighbours can move the term
    for c in corners:
        mask[c] = False
        cx, cy = divmod(int(c), k)
        for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            if 0 <= cx + dx < k and 0 <= cy + dy < k:
                mask[idx[cx + dx, cy + dy]] = False
    assert (gx_ref[mask] == 0).all() and (gy_ref[mask] == 0).all()
    # coincident directions at vertex 0 (a zero smallest gap), and a zero-length
    # edge bounding the smallest gap at vertex 4; every other vertex has
    # degree 1, so the whole gradient is zero while the term is not
    x = np.array([0, 10, 20, 0, 7, 7, 30], dtype=np.float64)
    y = np.array([0, 10, 20, 9, -3, -3, -5], dtype=np.float64)
    L = gen._finish(x, y, np.array([0, 0, 0, 4, 4]), np.array([1, 2, 3, 5, 6]), diameter=1.0,
                    name="kinks")
    for pruned in (False, True):
        gx_ref, gy_ref = check(L, (0.0, 0.0, 1.0), pruned, "kinks")
        f, gx, gy, _ = run(L, (0.0, 0.0, 1.0), pruned)
        assert f > 0
        assert (gx_ref == 0).all() and (gy_ref == 0).all()
        assert (gx == 0).all() and (gy == 0).all()


def _mirror_star(hub, pair, ring, radius, a0, a1):
    """A hub with neighbours in directions pair[0], (1,1), pair[1] (mirror
    images across the diagonal, so the two gaps between them are equal as
    real numbers) and `ring` more on a circle between angles a0 and a1."""
    dirs = [pair[0], (1, 1), pair[1]]
    for t in np.linspace(a0, a1, ring):
        dirs.append((int(round(radius * np.cos(t))), int(round(radius * np.sin(t)))))
    x = np.array([hub[0]] + [hub[0] + dx for dx, _ in dirs], dtype=np.float64)
    y = np.array([hub[1]] + [hub[1] + dy for _, dy in dirs], dtype=np.float64)
    k = len(dirs)
    return x, y, np.zeros(k, np.int64), np.arange(1, k + 1)


@pytest.mark.parametrize("shape", [
    ("thread", (0, 0), ((2, 1), (1, 2)), 0, 1, 0.0, 0.0),
    ("thread", (50, 60), ((7, 3), (3, 7)), 5, 30, 1.8, 6.0),
    ("lds", (1 << 12, 1 << 12), ((20, 19), (19, 20)), 40, 1000, 1.0, 2 * np.pi - 0.2),
    ("in-place", (1 << 19, 1 << 19), ((1000, 999), (999, 1000)), 2100, 500000, 1.0,
     2 * np.pi - 0.2),
])
def test_exact_ties_off_the_axes(torch_mod, shape):
    """A smallest gap attained twice contributes nothing, on each vertex
    path, also when the two gaps are equal only as real numbers; moving one
    neighbour of the pair by one unit breaks the tie and the gradient
    returns, as in the oracle."""
    path, hub, pair, ring, radius, a0, a1 = shape
    x, y, src, dst = _mirror_star(hub, pair, ring, radius, a0, a1)
    L = gen._finish(x, y, src, dst, diameter=1.0, name=f"tie-{path}")
    for pruned in (False, True):
        gx_ref, gy_ref = check(L, (0.0, 0.0, 1.0), pruned, f"tie {path}")
        assert (gx_ref == 0).all() and (gy_ref == 0).all()
        _, gx, gy, _ = run(L, (0.0, 0.0, 1.0), pruned)
        assert (gx == 0).all() and (gy == 0).all()
    y2 = y.copy()
    y2[3] += 1.0
    L = gen._finish(x, y2, src, dst, diameter=1.0, name=f"no-tie-{path}")
    gx_ref, gy_ref = check(L, (0.0, 0.0, 1.0), False, f"broken tie {path}")
    assert np.abs(gx_ref).max() > 0


def _unique_gap_margin(x, y, nbrs, v):
    """(second smallest gap - smallest gap, smallest gap, shortest edge) at v."""
    d = np.array([np.arctan2(y[u] - y[v], x[u] - x[v]) for u in nbrs[v]])
    a = np.sort(np.where(d < 0, d + 2 * np.pi, d))
    g = np.sort(np.diff(np.concatenate([a, [a[0] + 2 * np.pi]])))
    ln = min(np.hypot(x[u] - x[v], y[u] - y[v]) for u in nbrs[v])
    return (g[1] - g[0]) if g.size > 1 else np.inf, g[0], ln


def test_term_matches_finite_differences(torch_mod):
    L = gen.uniform_layout(2000, 4000, extent=1 << 14, seed=11)
    t, gx, gy, _ = run(L, (0.0, 0.0, 1.0))
    x, y = L.x.astype(np.float64), L.y.astype(np.float64)
    nbrs = [[] for _ in range(L.n_nodes)]
    for s, d in zip(L.src, L.dst):
        nbrs[s].append(d)
        nbrs[d].append(s)
    # the term's gradients are ~1e-9 here (a 1/(2 pi N) factor over edges
    # thousands of units long), so a step of 1e-3 leaves the quotient at the
    # rounding noise of the O(1) term; 0.1 units keeps the truncation error
    # (relative ~ (h / l)^2) and the noise both below 1e-6
    h = 0.1
    # a vertex is differenced only if no gap decision near it can flip
    # within the step: at v and at each neighbour the smallest gap stays
    # unique and positive by more than 4 h / (shortest edge there)
    cand = []
    for v in range(L.n_nodes):
        if len(nbrs[v]) < 1:
            continue
        ok = True
        for w in [v] + nbrs[v]:
            if len(nbrs[w]) < 2:
                continue
            sep, g0, ln = _unique_gap_margin(x, y, nbrs, w)
            if not (sep > 4 * h / ln and g0 > 4 * h / ln):
                ok = False
                break
        if ok:
            cand.append(v)
    rng = np.random.default_rng(1)
    nodes = rng.choice(np.array(cand), size=64, replace=False)
    fd = np.zeros((64, 2))
    for i, v in enumerate(nodes):
        for k, arr in enumerate((x, y)):
            old = arr[v]
            vals = []
            for step in (h, -h):
                arr[v] = old + step
                vals.append(oracle.min_angle_term(x, y, L.src, L.dst, 1.0))
            arr[v] = old
            fd[i, k] = (vals[0] - vals[1]) / (2 * h)
    got = np.stack([gx[nodes], gy[nodes]], axis=1)
    rel = np.abs(got - fd) / np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())
    say(f"[ma-grad-fd] {len(cand)} candidates, max relative error {rel.max():.3e}")
    assert rel.max() <= 1e-5


def test_nonfinite_weight_is_an_error(torch_mod):
    from paper_2411_09809_amd import _lib, metrics
    L = gen.uniform_layout(50, 80, extent=256, seed=2)
    D = metrics.DeviceLayout.from_host(L)
    torch = torch_mod
    lib = _lib.lib()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.zeros(2, 50, dtype=torch.float64, device="cuda")
    ws = metrics.workspace(50, L.n_edges, D.x.device)
    w, wb = metrics._ws_args(ws)
    rc = lib.rb_loss_grad(D.x.data_ptr(), D.y.data_ptr(), 50, D.src.data_ptr(), D.dst.data_ptr(),
                          L.n_edges, IDEAL, 1.0, 1.0, float("nan"), loss.data_ptr(),
                          g[0].data_ptr(), g[1].data_ptr(), None, w, wb,
                          metrics._stream(D.x.device))
    assert rc == 1                                   # RB_EINVAL
    assert b"finite" in lib.rb_last_error()
