"""Write ``tests/golden/workloads.json``: oracle values of the full-size
synthetic workloads, keyed by workload name and input digest.

Calls only the CPU oracle (``oracle/``) and the seeded generators.  The GPU
parity tests compare librb against these stored values when recomputing them
would take too long inside a test.

    python tests/golden/make_golden.py [name ...]
"""
import json
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


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    for name in names or list(BUILDERS):
        t0 = time.time()
        L = BUILDERS[name]()
        vals = oracle.all_metrics(L)
        vals.update(n_nodes=L.n_nodes, n_edges=L.n_edges, diameter=L.diameter,
                    ideal_angle=L.ideal_angle, digest=L.digest())
        data[name] = vals
        print(f"{name}: {time.time() - t0:.1f}s {vals}", flush=True)
    with open(OUT, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
