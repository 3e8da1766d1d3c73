"""Write the stored oracle values of the full-size synthetic workloads.

Calls only the CPU oracle (``oracle/``) and the seeded generators.  The GPU
parity tests compare librb against these stored values where recomputing
them would take too long inside a test.  Every entry carries the input
digest of its layout, and the tests check it before comparing.

    python tests/golden/make_golden.py [name ...]

* ``uniform_V1000_E2000_s0``, ``ba_cluster_V50000_s0``, ``rgg_V20000_s0``:
  all five metrics in one oracle run each -> ``workloads.json``.
* ``batch512_s0``: the five metrics of each of the 512 layouts of the
  batched workload -> ``batch512_s0.json`` (one list per metric, in layout
  order, plus the digests).
* ``powerlaw_V1000000_s0``: the 1,000,000-node / 3,000,000-edge layout.  Its
  4.5e12 edge pairs take hours on a few cores, so Algorithms 4 and 5 (and
  Algorithm 1 over the 5e11 node pairs) run as row slices of about equal
  pair counts (``oracle.crossing_angle_rows`` / ``node_occlusion_rows``).
  Each finished slice is appended to ``powerlaw_V1000000_s0_rows.jsonl``;
  a rerun skips the slices recorded there for the same digest, so the job
  can be stopped and resumed.  When every slice is present, the sums go to
  ``workloads.json``: counts are exact integer sums, the deviation sum adds
  the per-slice sums exactly rounded (math.fsum), and
  E_ca = 1 - sum / E_c as the oracle forms it (reading R7 for no crossing).
"""
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2411_09809_amd import gen  # noqa: E402

OUT = os.path.join(HERE, "workloads.json")

BUILDERS = {
    "uniform_V1000_E2000_s0": lambda: gen.uniform_layout(seed=0),
    "ba_cluster_V50000_s0": lambda: gen.ba_cluster_layout(seed=0),
    "rgg_V20000_s0": lambda: gen.geometric_layout(seed=0),
}
BATCH = "batch512_s0"
POWERLAW = "powerlaw_V1000000_s0"
CROSS_SLICES = 480          # about 9.4e9 edge pairs each
OCCL_SLICES = 40            # about 1.25e10 node pairs each


def _load(path):
    if os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def _store(path, data):
    with open(path + ".tmp", "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(path + ".tmp", path)


def equal_pair_cuts(n, k):
    """Row boundaries 0 = r_0 < ... < r_k = n such that the rows of each
    slice hold about C(n,2)/k of the pairs (i, j), i < j."""
    total = n * (n - 1) // 2
    cuts = [0]
    for q in range(1, k):
        target = total * q // k
        lo, hi = cuts[-1], n          # smallest r with pairs_before(r) >= target
        while lo < hi:
            mid = (lo + hi) // 2
            before = mid * (n - 1) - mid * (mid - 1) // 2
            if before >= target:
                hi = mid
            else:
                lo = mid + 1
        if lo > cuts[-1]:
            cuts.append(lo)
    cuts.append(n)
    return cuts


def metrics_entry(L):
    vals = oracle.all_metrics(L)
    vals.update(n_nodes=L.n_nodes, n_edges=L.n_edges, diameter=L.diameter,
                ideal_angle=L.ideal_angle, digest=L.digest())
    return vals


def make_batch():
    layouts = gen.batch_layouts(seed=0)
    keys = ("node_occlusion", "edge_crossing", "proper_crossing", "crossing_angle",
            "crossing_dev_sum", "min_angle", "min_angle_sum_dv", "min_angle_n_used",
            "edge_length_variation")
    out = {k: [] for k in keys}
    out.update(digest=[], n_nodes=[], n_edges=[])
    t0 = time.time()
    for b, L in enumerate(layouts):
        c, p, dev = oracle.crossing_angle_rows(L.x, L.y, L.src, L.dst, L.ideal_angle, 0,
                                               L.n_edges, proper=True)
        ma, sdv, used = oracle.min_angle(L.x, L.y, L.src, L.dst)
        ml, _ = oracle.edge_length_variation(L.x, L.y, L.src, L.dst)
        vals = dict(node_occlusion=oracle.node_occlusion(L.x, L.y, L.diameter),
                    edge_crossing=c, proper_crossing=p,
                    crossing_angle=1.0 - dev / c if c else 1.0, crossing_dev_sum=dev,
                    min_angle=ma, min_angle_sum_dv=sdv, min_angle_n_used=used,
                    edge_length_variation=ml)
        for k in keys:
            out[k].append(vals[k])
        out["digest"].append(L.digest())
        out["n_nodes"].append(L.n_nodes)
        out["n_edges"].append(L.n_edges)
        if b % 32 == 31:
            print(f"{BATCH}: {b + 1} layouts, {time.time() - t0:.0f}s", flush=True)
    out["ideal_angle"] = layouts[0].ideal_angle
    out["diameter"] = layouts[0].diameter
    _store(os.path.join(HERE, BATCH + ".json"), out)


def make_powerlaw(data):
    L = gen.powerlaw_layout(seed=0)
    digest = L.digest()
    rows_path = os.path.join(HERE, POWERLAW + "_rows.jsonl")
    done = {}
    if os.path.exists(rows_path):
        with open(rows_path) as fh:
            for line in fh:
                r = json.loads(line)
                if r["digest"] == digest:
                    done[(r["kind"], r["r0"], r["r1"])] = r
    occl_cuts = equal_pair_cuts(L.n_nodes, OCCL_SLICES)
    cross_cuts = equal_pair_cuts(L.n_edges, CROSS_SLICES)
    work = [("occlusion", a, b) for a, b in zip(occl_cuts, occl_cuts[1:])]
    work += [("crossing", a, b) for a, b in zip(cross_cuts, cross_cuts[1:])]
    t0 = time.time()
    for i, (kind, a, b) in enumerate(work):
        if (kind, a, b) in done:
            continue
        t = time.time()
        if kind == "crossing":
            c, p, dev = oracle.crossing_angle_rows(L.x, L.y, L.src, L.dst, L.ideal_angle, a, b,
                                                   proper=True)
            r = dict(kind=kind, r0=a, r1=b, count=c, proper=p, dev_sum=dev, digest=digest)
        else:
            r = dict(kind=kind, r0=a, r1=b,
                     count=oracle.node_occlusion_rows(L.x, L.y, L.diameter, a, b),
                     digest=digest)
        r["seconds"] = round(time.time() - t, 1)
        with open(rows_path, "a") as fh:
            fh.write(json.dumps(r, sort_keys=True) + "\n")
        done[(kind, a, b)] = r
        print(f"{POWERLAW}: slice {i + 1}/{len(work)} {kind} [{a}, {b}) {r['seconds']}s "
              f"(total {time.time() - t0:.0f}s)", flush=True)
    cross = [done[w] for w in work if w[0] == "crossing"]
    occl = [done[w] for w in work if w[0] == "occlusion"]
    count = sum(r["count"] for r in cross)
    dev = math.fsum(r["dev_sum"] for r in cross)
    ma, sdv, used = oracle.min_angle(L.x, L.y, L.src, L.dst)
    ml, mu = oracle.edge_length_variation(L.x, L.y, L.src, L.dst)
    data[POWERLAW] = dict(
        node_occlusion=sum(r["count"] for r in occl), edge_crossing=count,
        proper_crossing=sum(r["proper"] for r in cross), crossing_dev_sum=dev,
        crossing_angle=1.0 - dev / count if count else 1.0, min_angle=ma,
        min_angle_sum_dv=sdv, min_angle_n_used=used, edge_length_variation=ml,
        mean_edge_length=mu, n_nodes=L.n_nodes, n_edges=L.n_edges, diameter=L.diameter,
        ideal_angle=L.ideal_angle, digest=digest,
        slices=dict(crossing=len(cross), occlusion=len(occl)))


def main(names):
    names = names or list(BUILDERS)
    for name in names:
        t0 = time.time()
        if name == BATCH:
            make_batch()
        else:
            data = _load(OUT)
            if name == POWERLAW:
                make_powerlaw(data)
            else:
                data[name] = metrics_entry(BUILDERS[name]())
            data = {**_load(OUT), name: data[name]}   # keep entries written meanwhile
            _store(OUT, data)
        print(f"{name}: {time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
