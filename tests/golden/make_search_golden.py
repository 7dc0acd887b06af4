"""Writes search_20x10.json: optima and critical-tree sizes of the 20 x 10
search workload (seeds 1..8, p ~ U[1,99]) computed by the CPU oracle only.

    python tests/golden/make_search_golden.py

For each seed: the NEH makespan, the optimum proven by the oracle's
depth-first search from NEH + 1 with LB1 and with full LB2 (they must agree),
and, with the incumbent fixed at the optimum, the number of decomposed nodes
and bounded children of the critical tree for each bound (Section 2.5: the
nodes whose bound is below the optimum; order-independent under MinMin).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2012_09511_amd import inputs  # noqa: E402


def main():
    out = {"source": "oracle/oracle.c or_neh and or_search; inputs.instance(20, 10, seed)",
           "n": 20, "m": 10, "cases": []}
    for seed in range(1, 9):
        p = inputs.instance(20, 10, seed)
        neh, _ = oracle.neh(p)
        case = {"seed": seed, "neh": neh}
        for name, kind in (("lb1", oracle.LB1), ("lb2", oracle.LB2_FULL)):
            r = oracle.search(p, neh + 1, kind)
            assert r["proven"] and r["found"]
            assert oracle.makespan(p, r["perm"]) == r["best"]
            case.setdefault("opt", r["best"])
            assert case["opt"] == r["best"]
            crit = oracle.search(p, r["best"], kind)
            assert crit["proven"] and not crit["found"]
            case[f"critical_nodes_{name}"] = crit["nodes"]
            case[f"critical_children_{name}"] = crit["children"]
        out["cases"].append(case)
        print(case, flush=True)
    with open(os.path.join(HERE, "search_20x10.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
