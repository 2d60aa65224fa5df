"""Write the stored expected values under tests/golden/ from the CPU oracle only.

Run from the repository root:  python tests/golden/make_golden.py
The index-set sizes are also fixed by brute-force enumeration in the tests;
this file records them (and the fibre lengths) so GPU tests can check the
library's tables without re-running the oracle.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import lifted  # noqa: E402
from paper_2103_14897_amd import workloads as wl  # noqa: E402


def summary(spec, full=True):
    mn = lifted.index_set(spec.A1, spec.A2, spec.Ec, spec.cutoff)
    out = {"Ec": spec.Ec, "cutoff": spec.cutoff, "N": int(len(mn))}
    for layer in (1, 2):
        lens = [int(len(r)) for _, r in lifted.fibres(mn, layer)]
        out[f"nfibres_{layer}"] = len(lens)
        out[f"sum_L2_{layer}"] = int(sum(x * x for x in lens))
        out[f"minmax_L_{layer}"] = [min(lens), max(lens)]
        if full:
            out[f"fibre_lengths_{layer}"] = lens
    return out


if __name__ == "__main__":
    gold = {
        "tiny_chain": summary(wl.chain_system(200.0)),
        "chain": summary(wl.chain_system(2.0e4)),
        "twisted": summary(wl.twisted_system(6500.0), full=False),
    }
    with open(os.path.join(HERE, "index_sets.json"), "w") as f:
        json.dump(gold, f, indent=1)
    print({k: v["N"] for k, v in gold.items()})
