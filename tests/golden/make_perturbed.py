"""Rounding sensitivity of the FP64 CPU oracle's sweep (calls only problems/
and oracle/).

Runs the oracle's sweeps on a seeded instance with every raw initial tensor
entry multiplied by (1 + eps g), g ~ N(0, 1) from default_rng(4242), and
records theta at every node visit and the energy after every sweep.  With
eps = 0 it is the plain oracle run (node by node).  Two such runs, eps = 0 and
eps = 1e-15 (a relative change at the level of one rounding of the input),
show how far two FP64 trajectories from the same start separate through the
single-tensor sweep alone: the separation that any other correct FP64
implementation, with its own rounding order, is expected to show as well.

Usage: python tests/golden/make_perturbed.py ising16_m64 3 1e-15
Writes tests/golden/<config>_oracle_eps<eps>.json.
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


def main():
    key = sys.argv[1] if len(sys.argv) > 1 else "ising16_m64"
    sweeps = int(sys.argv[2]) if len(sys.argv) > 2 else 3
    eps = float(sys.argv[3]) if len(sys.argv) > 3 else 1e-15
    p = config_problem(key)
    g = np.random.default_rng(4242)
    raw = [r * (1.0 + eps * g.standard_normal(r.shape)) for r in p.raw_tensors]
    o = OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u, raw)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                       f"{key}_oracle_eps{eps:g}.json")
    rec = {"config": key, "n_sites": p.n_sites, "m": p.m, "eps": eps,
           "perturbation": "raw *= 1 + eps * N(0,1) draws of default_rng(4242), per entry",
           "energies": [], "node_theta": [], "seconds": [],
           "source": "FP64 CPU oracle (oracle/ttn.py), seeded instance of problems.CONFIGS"}
    for s in range(sweeps):
        t0 = time.time()
        thetas = []
        for n in o.tree.post_order():
            o.move_center(n)
            thetas.append(o.eigsolve(n))
        rec["energies"].append(thetas[-1])
        rec["node_theta"].append(thetas)
        rec["seconds"].append(time.time() - t0)
        print(f"sweep {s}: E = {thetas[-1]:.12f}  ({time.time() - t0:.0f} s)", flush=True)
        with open(out, "w") as f:
            json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main()
