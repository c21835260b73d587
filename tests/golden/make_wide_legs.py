"""Oracle matvec at the heaviest full node of a wide-leg workload (calls only
problems/ and oracle/).

From the seeded initial state the oracle moves the isometry centre to the
full node with the largest matvec flop count (QR moves across links as wide
as the bond dimension, gauge diag(R) >= 0) and applies H_eff there to a seeded
input.  The file records, for a GPU test to compare against:

* the node, its dims and the oracle's flop count;
* 4096 entries of y = H_eff x at seeded positions, and the whole slice
  y[:, :, p0] (one spectator index of the parent leg);
* 4096 seeded entries of the isometry left at the first node the centre moved
  through (its QR was taken across a link of the full width), and, after a
  further move from the heaviest node to its left child, of the isometry
  left at the heaviest node (QR of an (m m) x m matricisation).

x = default_rng(7).standard_normal(dims); positions from default_rng(8).

Usage: python tests/golden/make_wide_legs.py heis16_m96
Writes tests/golden/<config>_wide_matvec.json.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from problems import config_problem  # noqa: E402
from oracle.ttn import OracleTTN  # noqa: E402

P0 = 5
N_SAMPLES = 4096


def main():
    key = sys.argv[1] if len(sys.argv) > 1 else "heis16_m96"
    p = config_problem(key)
    t0 = time.time()
    o = OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u, p.raw_tensors)
    print(f"set-up {time.time() - t0:.0f} s", flush=True)
    full = [n for n in range(o.tree.n_nodes) if o.tree.dims[n] == (p.m, p.m, p.m)]
    node = max(full, key=o.flops)
    flops = o.flops(node)
    path = o.tree.path(o.center, node)
    t1 = time.time()
    o.move_center(node)
    print(f"centre moved along {path} in {time.time() - t1:.0f} s", flush=True)
    dims = o.tree.dims[node]
    x = np.random.default_rng(7).standard_normal(dims)
    t2 = time.time()
    y = o.matvec(node, x)
    print(f"matvec {flops / 1e9:.1f} GFLOP in {time.time() - t2:.0f} s", flush=True)
    M = int(np.prod(dims))
    g = np.random.default_rng(8)
    idx = np.sort(g.choice(M, N_SAMPLES, replace=False))
    isos = []

    def record_iso(qn):
        Q = o.T[qn]
        qidx = np.sort(g.choice(Q.size, min(N_SAMPLES, Q.size), replace=False))
        isos.append({"node": int(qn), "dims": list(Q.shape), "idx": qidx.tolist(),
                     "vals": Q.reshape(-1)[qidx].tolist()})

    record_iso(path[0])
    child = o.tree.children[node][0]
    assert child[0] == 'n'
    o.move_center(child[1])
    record_iso(node)
    rec = {
        "config": key, "node": int(node), "dims": list(dims), "flops": int(flops),
        "path": [int(v) for v in path], "x_seed": 7, "sample_seed": 8,
        "idx": idx.tolist(), "y": y.reshape(-1)[idx].tolist(),
        "p0": P0, "slice": y[:, :, P0].reshape(-1).tolist(),
        "y_norm": float(np.linalg.norm(y)),
        "child": int(child[1]), "isometries": isos,
        "source": "FP64 CPU oracle (oracle/ttn.py), seeded instance of problems.CONFIGS",
    }
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{key}_wide_matvec.json")
    with open(out, "w") as f:
        json.dump(rec, f)
    print(f"wrote {out} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
