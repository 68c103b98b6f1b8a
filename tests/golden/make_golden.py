"""Write the oracle's full-size reference values (calls only oracle/ and workloads/).

    python tests/golden/make_golden.py maxcut3reg_n28_p8
    python tests/golden/make_golden.py bisection_g16_k8_p6 2
    python tests/golden/make_golden.py xorders_maxcut3reg_n24_p4
    python tests/golden/make_golden.py multiangle_maxcut3reg_n24_p4

Each output file records the workload, its graph and angles (so a reader can check the
inputs are the seeded ones), and the FP64 oracle's <C> (E / Nrm) and adjoint gradient
(divided by Nrm, the convention of the library).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402


def make(name: str, n_sets: int = 1, extra_sets=None):
    W = workloads.workload(name)
    g = W.graphs[0]
    t0 = time.time()
    table = oracle.graph_table(g, W.hamming_k)
    rows = []
    angle_rows = [W.angles[i] for i in range(min(n_sets, W.angles.shape[0]))]
    if extra_sets:
        angle_rows += [np.asarray(a, dtype=np.float64) for a in extra_sets]
    for a in angle_rows:
        if W.mixer == "x_orders":
            from oracle import xmixers
            E, N, gr = xmixers.grad(g.n, table, a, d=xmixers.diag_orders(g.n, W.extra["orders"]))
        elif W.mixer == "x_multiangle":
            from oracle import xmixers
            E, N, gr = xmixers.grad(g.n, table, a, multiangle=True)
        else:
            E, N, gr = oracle.grad(g.n, table, a, W.hamming_k)
        rows.append({"angles": a.tolist(), "expect": E / N, "norm": N, "grad": (gr / N).tolist()})
        print(name, "set done", time.time() - t0, flush=True)
    out = {
        "workload": name,
        "source": ("FP64 CPU oracle (oracle/xmixers.py), adjoint gradient" if W.mixer in ("x_orders", "x_multiangle")
                   else "FP64 CPU oracle (oracle/qaoa_oracle.c), adjoint gradient"),
        "n": g.n, "p": W.p, "hamming_k": W.hamming_k,
        "edges": [g.u.tolist(), g.v.tolist(), g.w.tolist()],
        "table_sum": int(table.sum()), "table_max": int(table.max()),
        "sets": rows,
        "oracle_threads": oracle.num_threads(),
        "seconds": time.time() - t0,
    }
    path = os.path.join(HERE, name + ".json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    make(sys.argv[1], n_sets=int(sys.argv[2]) if len(sys.argv) > 2 else 1)
