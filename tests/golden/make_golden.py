"""Writes the stored oracle results used by the full-size GPU parity tests.

Runs the CPU oracle (Alg. 4 with the readings of the oracle package) on a configured
workload at its full order and stores the stage history (level, variant, counted,
GMRES iterations), the event bits, the error figures and a fixed sample of the
solution.  Only the oracle and the seeded input generator are called.

    python tests/golden/make_golden.py 2            # n = 4096 multistage workload
    python tests/golden/make_golden.py 3 fp16       # n = 8192 double-double workload,
    python tests/golden/make_golden.py 3 bf16       #   with fp16 or bf16 factors
    python tests/golden/make_golden.py 3 fp16 --alt-threads 1
                                    # adds the history the oracle takes with its BLAS
                                    # library on 1 thread to the stored file

The oracle's float64 matrix-vector products and inner products go through the BLAS
library, whose summation order depends on its thread count; where a decision of the
method sits on a rounding boundary (a GMRES call stagnating near tau) the oracle's own
history then changes with that count.  --alt-threads records such histories beside the
stored one ("alt_histories"), so that the tests can tell a rounding-boundary spread
from a real difference.

Config 2: randsvd kappa_2 = 1e6, geometric singular values; fp16 factors with column
scaling, working precision fp32, residual fp64, GMRES tolerance 1e-4, restart 50,
k_max = 0.1 n.  Config 3: randsvd kappa_2 = 1e10, one small singular value; fp16 or
bf16 factors (fp16 with the automatic scaling retry), working precision fp64,
double-double residual, GMRES tolerance 1e-10, k_max = 0.1 n.  The LU runs as the
oracle's C loops when they are built (python -m oracle.native.build).  Each step is
printed as it completes.
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


def golden_name(cid, uf=None):
    cfg = WL.CONFIGS[cid]
    if uf is None or uf == cfg["params"]["uf"] and cid == 2:
        return "%s_oracle.json" % cfg["name"]
    return "%s_%s_oracle.json" % (cfg["name"], uf)


def run_alt(cid, uf, threads):
    """Run the oracle with its BLAS library on `threads` threads and add the history to
    the stored file under alt_histories[str(threads)]."""
    from threadpoolctl import threadpool_limits
    cfg = WL.CONFIGS[cid]
    params = dict(cfg["params"])
    if uf is not None:
        params["uf"] = uf
    A, x, b = WL.config_system(cid)
    t = time.perf_counter()
    with threadpool_limits(limits=threads, user_api="blas"):
        ref = OM.msir(A, b, OM.Params(**params), x_true=x)
    path = os.path.join(HERE, golden_name(cid, uf))
    with open(path) as f:
        out = json.load(f)
    alt = out.setdefault("alt_histories", {})
    alt[str(threads)] = {"history": [[s.level, s.stage, int(s.counted), int(s.k)] for s in ref.history],
                         "render": OM.render(ref.history), "nbe": float(ref.nbe),
                         "source": "BLAS on %d thread(s), oracle run of %.0f s" % (threads, time.perf_counter() - t)}
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, threads, OM.render(ref.history), flush=True)


def main(cid=2, uf=None):
    cfg = WL.CONFIGS[cid]
    params = dict(cfg["params"])
    if uf is not None:
        params["uf"] = uf
    t = time.perf_counter()
    A, x, b = WL.config_system(cid)
    print("input built in %.0f s" % (time.perf_counter() - t), flush=True)
    t = time.perf_counter()

    def log(step):
        print("%7.0f s  level %d uf %s stage %d iter %d k %d z %.3e nbe %.3e events %d" % (
            time.perf_counter() - t, step.level, step.uf, step.stage, step.iter, step.k, step.z, step.nbe,
            step.events), flush=True)

    ref = OM.msir(A, b, OM.Params(**params), x_true=x, log=log)
    dt = time.perf_counter() - t
    out = {
        "workload": cfg["name"], "n": cfg["n"], "kappa": cfg["kappa"], "mode": cfg["mode"],
        "params": params,
        "source": "oracle.msir.msir (Alg. 4), oracle run of %.0f s" % dt,
        "history": [[s.level, s.stage, int(s.counted), int(s.k)] for s in ref.history],
        "events": [int(s.events) for s in ref.history],
        "uf": [s.uf for s in ref.history],
        "render": OM.render(ref.history),
        "cged": bool(ref.cged), "nbe": float(ref.nbe), "ferr": float(ref.ferr), "n_lu": int(ref.n_lu),
        "sample_stride": SAMPLE_STRIDE,
        "x_sample": [float(v) for v in ref.x[::SAMPLE_STRIDE]],
    }
    path = os.path.join(HERE, golden_name(cid, uf))
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["render"], out["nbe"], "%.0f s" % dt, flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    if "--alt-threads" in args:
        i = args.index("--alt-threads")
        threads = int(args[i + 1])
        del args[i:i + 2]
        run_alt(int(args[0]), args[1] if len(args) > 1 else None, threads)
    else:
        main(int(args[0]) if args else 2, args[1] if len(args) > 1 else None)
