"""Write stored expected values for the large parity cases.

Every number written here comes from the CPU oracle (``oracle/``) run on the
seeded workloads of ``paper_2607_02749_amd.synth``; nothing comes from the GPU
path.  Usage:

    python tests/golden/make_golden.py n22     # ~1 min on 8 cores
    python tests/golden/make_golden.py n28     # ~2 h on 8 cores
    python tests/golden/make_golden.py batch   # a few minutes

Each file stores the workload name, seed, energy (re, im), the full gradient
and a handful of diagonal entries at seeded indices.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2607_02749_amd import synth  # noqa: E402


def solve(inst, with_mask=False):
    t0 = time.time()
    d = oracle.diag(inst.n, inst.x, inst.z, inst.c)
    t1 = time.time()
    mask = oracle.param_mask(inst.n, inst.layers, inst.cluster_mask) if with_mask else None
    e, g = oracle.energy_grad(inst.n, inst.layers, inst.ent, inst.theta, inst.x, inst.z,
                              inst.c, d=d, mask=mask)
    t2 = time.time()
    idx = np.random.default_rng(1234).integers(0, 1 << inst.n, size=16)
    return {
        "energy": [e.real, e.imag],
        "grad": g.tolist(),
        "diag_index": [int(i) for i in idx],
        "diag_value": [float(d[i]) for i in idx],
        "seconds_diag": t1 - t0,
        "seconds_energy_grad": t2 - t1,
    }


def write(name, payload):
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(payload, f, indent=1)
    print("wrote", path)


def main(which):
    if which == "n22":
        inst = synth.workload_n22()
        write("oracle_n22", {"workload": "workload_n22", "seed": 0, **solve(inst)})
    elif which == "n28":
        inst = synth.workload_n28()
        write("oracle_n28", {"workload": "workload_n28", "seed": 0, **solve(inst)})
    elif which == "batch":
        insts = synth.workload_batch()
        out = []
        for i, inst in enumerate(insts):
            r = solve(inst, with_mask=True)
            out.append({"index": i, "n": inst.n, "layers": inst.layers,
                        "energy": r["energy"], "grad": r["grad"]})
            print(i, inst.n, inst.layers, r["seconds_energy_grad"], flush=True)
        write("oracle_batch", {"workload": "workload_batch", "seed": 0, "count": len(insts),
                               "instances": out})
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "")
