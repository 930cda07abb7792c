"""Writes the stored oracle results used by the full-size GPU parity test.

Runs the CPU oracle (Alg. 4 with the readings of the oracle package) on the
n = 4096 multistage workload (randsvd, kappa_2 = 1e6, geometric singular
values; factors fp16 with column scaling, working precision fp32, residual
fp64, GMRES tolerance 1e-4, restart 50, k_max = 0.1 n) and stores the stage
history, the error figures and a fixed sample of the solution.  Only the
oracle and the seeded input generator are called.  About 20-40 minutes on 8
CPU cores.

    python tests/golden/make_golden.py [config_id]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import msir as OM  # noqa: E402
from paper_2107_06200_amd import workloads as WL  # noqa: E402

SAMPLE_STRIDE = 64


def main(cid=2):
    cfg = WL.CONFIGS[cid]
    A, x, b = WL.config_system(cid)
    t = time.perf_counter()
    ref = OM.msir(A, b, OM.Params(**cfg["params"]), x_true=x)
    dt = time.perf_counter() - t
    out = {
        "workload": cfg["name"], "n": cfg["n"], "kappa": cfg["kappa"], "mode": cfg["mode"],
        "params": cfg["params"],
        "source": "oracle.msir.msir (Alg. 4), oracle run of %.0f s" % dt,
        "history": [[s.level, s.stage, int(s.counted), int(s.k)] for s in ref.history],
        "render": OM.render(ref.history),
        "cged": bool(ref.cged), "nbe": float(ref.nbe), "ferr": float(ref.ferr),
        "sample_stride": SAMPLE_STRIDE,
        "x_sample": [float(v) for v in ref.x[::SAMPLE_STRIDE]],
    }
    path = os.path.join(HERE, "%s_oracle.json" % cfg["name"])
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["render"], out["nbe"], "%.0f s" % dt)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2)
