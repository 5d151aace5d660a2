"""Write the searched array codes of the workloads as JSON fixtures.

Calls only ``oracle/`` (plus the workload parameters, which are plain
numbers).  Run from the repository root:
    python tests/golden/make_search_fixtures.py
The library's ARRAY_SEARCH build must reproduce each file bit for bit.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import codes  # noqa: E402
from paper_1904_11563_amd.inputs import CODE_642, CODE_1282, CODE_1284  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main(which):
    for name, spec in (("642", CODE_642), ("1282", CODE_1282), ("1284", CODE_1284)):
        if which and name not in which:
            continue
        t = time.time()
        c = codes.array_search(spec.n, spec.k, spec.b, spec.sigma, spec.seed,
                               spec.restarts, spec.iters, walk=spec.walk)
        col_ptr, sym_ptr, sym_data = c.csr()
        out = {"n": spec.n, "k": spec.k, "b": spec.b, "sigma_max": spec.sigma,
               "seed": spec.seed, "restarts": spec.restarts, "iters": spec.iters,
               "walk": spec.walk,
               "columns": [[list(s) for s in col] for col in c.columns],
               "col_ptr": col_ptr, "sym_ptr": sym_ptr, "sym_data": sym_data}
        path = os.path.join(HERE, f"search_{name}.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(f"{path}: {time.time() - t:.1f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
