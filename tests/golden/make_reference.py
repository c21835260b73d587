"""Writes tests/golden/<config>_oracle.json: per-sweep energies of the FP64 CPU
oracle on the seeded instance (calls only problems/ and oracle/).

Usage: python tests/golden/make_reference.py ising16_m64 3
       python tests/golden/make_reference.py ising8_m32 40 1e-10
With a third argument the run stops early once two consecutive sweep
energies differ by less than that much per site (the run is then converged
to that level; the record says which stop was taken).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from problems import config_problem  # noqa: E402
from oracle.ttn import OracleTTN  # noqa: E402


def main():
    key = sys.argv[1] if len(sys.argv) > 1 else "ising16_m64"
    sweeps = int(sys.argv[2]) if len(sys.argv) > 2 else 3
    until = float(sys.argv[3]) if len(sys.argv) > 3 else None
    p = config_problem(key)
    o = OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u, p.raw_tensors)
    suffix = "_converged" if until is not None else ""
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{key}_oracle{suffix}.json")
    rec = {"config": key, "n_sites": p.n_sites, "m": p.m, "energies": [], "seconds": [],
           "source": "FP64 CPU oracle (oracle/ttn.py), seeded instance of problems.CONFIGS"}
    for s in range(sweeps):
        t0 = time.time()
        e = o.sweep()
        rec["energies"].append(e)
        rec["seconds"].append(time.time() - t0)
        print(f"sweep {s}: E = {e:.12f}  ({time.time() - t0:.0f} s)", flush=True)
        done = (until is not None and s > 0 and
                abs(rec["energies"][-1] - rec["energies"][-2]) / p.n_sites < until)
        if until is not None:
            rec["stop"] = (f"consecutive |dE|/N < {until:g} at sweep {s}" if done
                           else f"not converged to {until:g} after {s + 1} sweeps")
        with open(out, "w") as f:
            json.dump(rec, f, indent=1)
        if done:
            break


if __name__ == "__main__":
    main()
