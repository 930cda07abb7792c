"""Throughput benchmark: multistage mixed precision iterative refinement on one MI355X.

Workload (the configuration the headline metric is quoted on): one dense system
of order n = 4096, randsvd with geometrically distributed singular values
(mode 3), kappa_2 = 1e6, float64 storage, x_true ~ N(0,1), b = A x_true; factor
precision fp16 with column scaling, working precision fp32, residual fp64,
GMRES tolerance 1e-4, restart 50, k_max = 0.1 n, i_max = 10; stopping when the
normwise backward error of x (double-double residual) is <= 1e-15.

One step = one complete solve from A and b already resident in HBM (scaling,
factorization(s), every refinement step, result) through the C ABI.

Printed: one JSON line with solves/s, the dominant kernel's roofline figures
(device time of every launch of that kernel class, measured with HIP events on
the library's stream during the timed solves), the FP64 getrf+getrs comparator
on the same GPU (torch.linalg.lu_factor + lu_solve), and the CPU oracle timed on
this host on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP16_MFMA_PEAK_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=None, help="override the order (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--lu-update", choices=["mfma", "fma"], default="mfma",
                    help="trailing update of the fp16/bf16 LU: matrix cores or fp32 FMA chains")
    ap.add_argument("--copy-only", type=int, default=0, metavar="MB",
                    help="only copy MB megabytes device to device once (calibrates HBM byte counters)")
    ap.add_argument("--workload", choices=["c1", "c2", "c3", "c4", "c5"], default="c2",
                    help="c2 (default): the n = 4096 multistage system the headline metric is quoted on; "
                         "c1: n = 100, kappa 1e2 (SIR); c3: n = 8192, kappa 1e10 mode 2 with a double-double "
                         "residual; "
                         "c4: the uneven batch of 512 systems (n log-uniform in [64, 1024]) solved by one "
                         "msir_solve_batched call per step; c5: served requests with Poisson arrivals")
    ap.add_argument("--requests", type=int, default=120, help="c5: number of requests (first 10%% warm-up)")
    ap.add_argument("--slots", type=int, default=8, help="c5: service slots")
    ap.add_argument("--load", type=float, default=0.75, help="c5: arrival rate as a fraction of saturation")
    ap.add_argument("--sparse", action="store_true",
                    help="time the CSR solve on the synthetic sparse workload instead (n=4096, 16 nonzeros "
                         "per row, magnitude spread 300; the multistage workload's solver parameters)")
    return ap.parse_args()


def copy_only(mb):
    """One device-to-device copy of a known size: the reference for FETCH_SIZE/WRITE_SIZE."""
    import torch
    n = mb * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 4 * n, "read_bytes": 4 * n, "written_bytes": 4 * n}))


# Bytes one launch of each memory-bound class must move at minimum: the matrix operand
# once, plus its input and output vectors (float64).  A launch of the GEMV classes is one
# partial-sum kernel (the ordered fold of the partials into the output is timed as the
# class "fold", or is done by the next product while it stages its input).
def algorithmic_bytes(cls, n):
    tri = n * (n + 1) // 2
    return {"matvec32": 4 * n * n + 16 * n,       # fp32 copy of A, v in, A v out
            "matvec64": 8 * n * n + 16 * n,       # float64 A
            "trgemv32": 4 * tri + 16 * n,         # one fp32 inverse triangle
            "trgemv64": 8 * tri + 16 * n,         # one fp64 inverse triangle
            "resid": 8 * n * n + 40 * n,          # A, x, b in; r, r_hat out
            }.get(cls)


def arnoldi_bytes(hist, n, restart, basis_bytes):
    """Algorithmic bytes of the Arnoldi launches of a solve: iteration t of a GMRES
    correction (j = t mod restart) reads w (float64) and the j + 1 basis vectors in the
    working format, and writes v_{j+1} (float64 and its working-format copy)."""
    tot = 0
    for s in hist:
        k = max(0, int(s.k_gmres))
        for t in range(k):
            j = t % restart if restart > 0 else t
            tot += n * (8 + basis_bytes * (j + 1) + 8 + basis_bytes)
    return tot


# Kernel sources the GEMV classes are built from; HBM traffic figures taken with the
# byte counters are used only while these are unchanged.
GEMV_SOURCES = ["paper_2107_06200_amd/csrc/gemv.hip", "paper_2107_06200_amd/csrc/inverse.hip",
                "paper_2107_06200_amd/csrc/common.hpp", "paper_2107_06200_amd/csrc/msir_internal.hpp"]
TRAFFIC_FILE = "profiles/msir_n4096_gemv_hbm_counters.md"


ARNOLDI_SOURCES = ["paper_2107_06200_amd/csrc/gmres.hip", "paper_2107_06200_amd/csrc/gmres.hpp",
                   "paper_2107_06200_amd/csrc/common.hpp", "paper_2107_06200_amd/csrc/msir_internal.hpp"]
ARNOLDI_TRAFFIC_FILE = "profiles/msir_n4096_arnoldi_hbm_counters.md"


def measured_traffic(cls, n, path=TRAFFIC_FILE, sources=GEMV_SOURCES):
    """HBM bytes per launch of class `cls` from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE runs calibrated on a copy of known size), or None when there is no figure for
    this class and order or the kernel sources have changed since the counters were taken."""
    import hashlib
    import re
    try:
        txt = open(os.path.join(ROOT, path)).read()
        h = hashlib.sha256(b"".join(open(os.path.join(ROOT, p), "rb").read() for p in sources)).hexdigest()[:16]
    except OSError:
        return None
    if n != 4096:
        return None
    m = re.search(r"traffic_bytes_per_launch\[%s\] = (\d+) \(kernel sources sha256 ([0-9a-f]+)\)" % re.escape(cls), txt)
    if not m or m.group(2) != h:
        return None
    return int(m.group(1))


def _compose(A, b, hs, reps=4):
    """The oracle's time per solve composed from its pieces, each timed here on (A, b):
    the LU (in full up to n = 1024; above, on the leading 1024 x 1024 block and
    scaled by (n/1024)^3, its flop count's growth), one u_f substitution pair, preconditioned-operator
    applications (matrix-vector product plus two substitutions), and a float64 plus a
    double-double residual; combined with the counts of a solve's history hs.  The
    substitution's cost does not depend on the values, so the converted matrix stands in
    for the factors.  Returns (seconds per solve, seconds spent timing)."""
    import numpy as np
    from oracle import fmt as F, lu as OLU, scaling as OSC, solve as OSV, gmres as OGM, ops as OOPS
    n = A.shape[0]
    t0 = time.perf_counter()
    scal = OSC.compute(A, "fp16", rows=False)
    Af = F.round_to(OSC.apply(A, *scal), "fp16")
    q = min(n, 1024)
    t = time.perf_counter()
    OLU.getrf(Af[:q, :q].copy(), "fp16", OLU.nb_auto(n, "fp16"))
    t_lu = (time.perf_counter() - t) * (n / q) ** 3
    Wlike = np.asfortranarray(Af)
    ident = np.arange(n)
    t = time.perf_counter()
    OSV.lu_solve(Wlike, ident, b, "fp16", scal)
    t_solve = time.perf_counter() - t
    Au = F.round_to(A, "fp32")
    t = time.perf_counter()
    for _ in range(reps):
        OGM.precond_apply(A, Wlike, ident, scal, b, "fp32", "fp32", A_u=Au)
    t_iter = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    OOPS.residual(A, b, b, "fp64")
    t_res = time.perf_counter() - t
    t = time.perf_counter()
    OOPS.residual(A, b, b, "dd")
    t_res_dd = time.perf_counter() - t
    t_total = (hs["n_lu"] * t_lu + hs["gmres_iters"] * t_iter + hs["sir_steps"] * t_solve
               + hs["steps"] * (t_res + t_res_dd))
    return t_total, time.perf_counter() - t0


def cpu_baseline(A, b, hs):
    """The CPU oracle timed on this host on a bounded sample of the same workload.

    Measured: one complete oracle solve of the workload at n = 1024 (the same recipe and
    parameters), wall time and the threads it actually kept busy (process CPU time over
    wall time).  Composed: the per-piece model of _compose at n = 1024 (checked against
    that measurement) and at the benchmark's order with the GPU solve's history; the
    reported value is the composed n = 4096 time corrected by the measured/composed
    ratio at n = 1024."""
    from oracle import msir as OM
    from paper_2107_06200_amd import workloads as WL
    prm = dict(WL.CONFIGS[2]["params"])
    A1, x1, b1 = WL.config_system(2, n=1024)
    c0, t = os.times(), time.perf_counter()
    ref = OM.msir(A1, b1, OM.Params(**prm))
    wall = time.perf_counter() - t
    c1 = os.times()
    busy = ((c1.user - c0.user) + (c1.system - c0.system)) / wall
    hs1 = {"n_lu": ref.n_lu, "gmres_iters": int(sum(max(0, s.k) for s in ref.history)),
           "sir_steps": sum(1 for s in ref.history if s.stage == 0), "steps": len(ref.history)}
    comp1, s1 = _compose(A1, b1, hs1)
    ratio = wall / comp1
    comp, s2 = _compose(A, b, hs)
    est = comp * ratio
    return {"value": 1.0 / est, "unit": "solves/s", "cores": round(busy, 2), "kind": "oracle",
            "measured_n1024_s": round(wall, 3), "composed_n1024_s": round(comp1, 3),
            "measured_over_composed": round(ratio, 3), "composed_n%d_s" % A.shape[0]: round(comp, 3),
            "sample": ("one full oracle solve at n=1024 (%s, %.1f s wall, %.2f threads busy on average) and the "
                       "oracle's pieces timed at n=1024 and n=%d (%.1f s of work); the per-solve time at n=%d is "
                       "the composed %.0f s (history: %d LU, %d GMRES iterations, %d SIR steps) times the "
                       "measured/composed ratio %.2f at n=1024"
                       % (OM.render(ref.history), wall, busy, A.shape[0], s1 + s2, A.shape[0], comp, hs["n_lu"],
                          hs["gmres_iters"], hs["sir_steps"], ratio))}


def cpu_baseline_full(A, b, prm):
    """The CPU oracle timed on one complete solve of the workload itself (small orders)."""
    from oracle import msir as OM
    c0, t = os.times(), time.perf_counter()
    reps = 0
    while True:
        ref = OM.msir(A, b, OM.Params(**prm))
        reps += 1
        wall = time.perf_counter() - t
        if wall >= 5.0:
            break
    c1 = os.times()
    busy = ((c1.user - c0.user) + (c1.system - c0.system)) / wall
    return {"value": reps / wall, "unit": "solves/s", "cores": round(busy, 2), "kind": "oracle",
            "sample": "%d complete oracle solves of the workload (%s), %.1f s wall" % (reps, OM.render(ref.history), wall)}


def sparse_bench(args):
    """Solves/s of Alg. 4 with a sparse A in CSR form (residual and GMRES A v on the CSR
    arrays); inputs resident in HBM before the timed region."""
    import numpy as np
    import torch
    from paper_2107_06200_amd import msir as M
    from paper_2107_06200_amd import workloads as WL
    n = args.n or 4096
    per_row, scale = 16, 300.0
    rp, ci, v, A, x_true, b = WL.sparse_system(n, per_row, scale, WL.rng_for(61, n))
    dev = torch.device("cuda:0")
    M.lib()
    h = M.Handle(0)
    t_rp, t_ci, t_v = (torch.from_numpy(a).to(dev) for a in (rp, ci, v))
    bt = torch.from_numpy(b).to(dev)
    prm = dict(WL.CONFIGS[2]["params"])
    P = M.params(lu_update=args.lu_update, **prm)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        x, res, hist, rc = M.solve_csr(h, t_rp, t_ci, t_v, bt, P=P, x=x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, res, hist, rc = M.solve_csr(h, t_rp, t_ci, t_v, bt, P=P, x=x)
        if rc != 0 or res.nbe > 1e-15:
            print("sparse solve did not reach nbe <= 1e-15: rc=%d nbe=%.3e" % (rc, res.nbe), file=sys.stderr)
            sys.exit(1)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    print(json.dumps({"metric": "solves/s to FP64 backward err 1e-15, sparse A (CSR)", "value": round(args.steps / el, 4),
                      "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": round(1000.0 * el / args.steps, 3), "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "fp16-factor/fp32-working/fp64-residual (mixed)",
                      "data": "synthetic sparse (seeded), float64",
                      "config": {"workload": "msir_csr_n%d_nnz%d_per_row" % (n, per_row), "n": n, "nnz": int(len(v)),
                                 "spread": scale},
                      "history": M.render(hist), "nbe": res.nbe}))
    h.close()


def batched_bench(args):
    """Solves/s of the uneven batch (512 independent randsvd systems, n log-uniform in
    [64, 1024], log10 kappa uniform in [1, 8], modes 2 and 3; fp16 factors, fp32
    working precision, fp64 residual): one step = one msir_solve_batched call over all
    512 systems, inputs resident in HBM; every system must reach nbe <= 1e-15.  The
    FP64 comparator is torch.linalg.lu_factor + lu_solve per system on the same GPU."""
    import numpy as np
    import torch
    from paper_2107_06200_amd import msir as M
    from paper_2107_06200_amd import workloads as WL
    dev = torch.device("cuda:0")
    M.lib()
    h = M.Handle(0)
    metas = WL.batched_meta()
    systems = [WL.batched_system(m) for m in metas]
    As = [M.colmajor(torch.from_numpy(np.asfortranarray(A)).to(dev)) for A, _, _ in systems]
    bs = [torch.from_numpy(b).to(dev) for _, _, b in systems]
    xs = [torch.empty(A.shape[0], dtype=torch.float64, device=dev) for A in As]
    P = M.params(lu_update=args.lu_update, **WL.BATCHED_PARAMS)
    for _ in range(args.warmup):
        M.solve_batched(h, As, bs, P=P, xs=xs, hist_cap=1)
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        xs, outs, hists, rc = M.solve_batched(h, As, bs, P=P, xs=xs, hist_cap=1)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        bad = [i for i, o in enumerate(outs) if not (o.status == 0 and o.nbe <= 1e-15)]
        if rc != 0 or bad:
            print("batched solve: %d systems did not reach nbe <= 1e-15" % len(bad), file=sys.stderr)
            sys.exit(1)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    count = len(systems)
    # FP64 getrf + getrs per system on the same GPU (black-box comparator)
    comp = []
    for rep in range(3):
        torch.cuda.synchronize()
        tc = time.perf_counter()
        for A, b in zip(As, bs):
            LU, piv = torch.linalg.lu_factor(A)
            torch.linalg.lu_solve(LU, piv, b.unsqueeze(1))
        torch.cuda.synchronize()
        if rep:
            comp.append(time.perf_counter() - tc)
    comp_s = min(comp)
    hist_lu = sum(o.n_lu for o in outs)
    print(json.dumps({
        "metric": "solves/s to FP64 backward err 1e-15, uneven batch", "value": round(args.steps * count / el, 2),
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000.0 * el / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp16-factor/fp32-working/fp64-residual (mixed)",
        "data": "synthetic randsvd (seeded), float64",
        "config": {"workload": "batched512_n64to1024", "systems": count,
                   "n_total": int(sum(m["n"] for m in metas)), "lu_update": args.lu_update},
        "latency_ms": {"p50": round(1000 * sorted(times)[len(times) // 2], 3), "max": round(1000 * max(times), 3)},
        "factorizations": hist_lu, "gmres_iters": int(sum(o.gmres_iters for o in outs)),
        "system_refine_ms": {"max": round(max(o.t_refine_ms for o in outs), 3),
                             "p50": round(sorted(o.t_refine_ms for o in outs)[count // 2], 3),
                             "sum": round(sum(o.t_refine_ms for o in outs), 3),
                             "slowest_n": int(metas[max(range(count), key=lambda i: outs[i].t_refine_ms)]["n"])},
        "fp64_getrf_getrs_per_system": {"ms_all": round(1000 * comp_s, 3),
                                        "solves_per_s": round(count / comp_s, 2),
                                        "impl": "torch.linalg.lu_factor+lu_solve float64, one call per system"},
        "speedup_vs_fp64_direct": round((args.steps * count / el) / (count / comp_s), 4)}))
    h.close()


def device_randsvd(n, kappa, mode, nrhs, gen, dev):
    """randsvd on the device (torch, float64): A = U diag(sigma) V^T with U, V Haar
    orthogonal (QR of N(0,1), signs of R moved into Q), sigma of mode 2 or 3, X ~ N(0,1),
    B = A X; the recipe of workloads.randsvd, drawn from a torch generator."""
    import torch
    def haar():
        G = torch.randn((n, n), generator=gen, dtype=torch.float64, device=dev)
        Q, R = torch.linalg.qr(G)
        return Q * torch.sign(torch.diagonal(R))[None, :]
    U, V = haar(), haar()
    if mode == 2:
        sig = torch.ones(n, dtype=torch.float64, device=dev)
        sig[-1] = 1.0 / kappa
    else:
        sig = kappa ** (-torch.arange(n, dtype=torch.float64, device=dev) / max(1.0, n - 1.0))
    A = (U * sig[None, :]) @ V.t().contiguous()
    X = torch.randn((n, nrhs), generator=gen, dtype=torch.float64, device=dev)
    B = A @ X
    return A.t().contiguous().t(), X, B.t().contiguous().t()


def serving_bench(args):
    """Served requests (msir_server): Poisson arrivals of solve requests with n uniform
    over {256, 512, 1024, 2048, 4096}, kappa log-uniform in [1e2, 1e8], modes 2 and 3
    alternating, 1-16 right-hand sides; fp16 factors, fp32 working precision, fp64
    residual, tau 1e-6, k_max 0.1 n.  Matrices are generated on the device before the
    timed region.  The saturation throughput is measured first (every request of the
    warm-up share submitted at once), then the requests arrive at args.load times that
    rate; latency = completion - arrival (host clock), solves = right-hand sides."""
    import numpy as np
    import torch
    from paper_2107_06200_amd import msir as M
    from paper_2107_06200_amd import workloads as WL
    dev = torch.device("cuda:0")
    M.lib()
    reqs = WL.serving_requests(count=args.requests, rate=1.0)
    gen = torch.Generator(device=dev).manual_seed(5)
    data = []
    for r in reqs:
        A, X, B = device_randsvd(r["n"], r["kappa"], r["mode"], r["nrhs"], gen, dev)
        Xo = torch.empty_like(B).t().contiguous().t()
        data.append((A, B, Xo))
    torch.cuda.synchronize()
    P = M.params(**WL.BATCHED_PARAMS)
    warm = max(1, args.requests // 10)
    srv = M.Server(0, slots=args.slots, budget=64 << 30, P=P)

    def run(ids, arrivals):
        t0 = time.perf_counter()
        comps = []
        k = 0
        while len(comps) < len(ids):
            now = time.perf_counter() - t0
            while k < len(ids) and arrivals[k] <= now:
                A, B, X = data[ids[k]]
                srv.submit(ids[k], A, B, X)
                k += 1
            wait = 0 if k < len(ids) else 1000
            if k < len(ids):
                wait = max(0, int(1000 * (arrivals[k] - (time.perf_counter() - t0))))
            c, _ = srv.poll(wait_ms=min(wait, 50) if k < len(ids) else 1000)
            comps += c
        return comps, time.perf_counter() - t0

    # warm-up and saturation: the warm-up share submitted at once
    ids_w = list(range(warm))
    comps, el = run(ids_w, [0.0] * warm)
    sat = warm / el
    comps, el = run(ids_w, [0.0] * warm)
    sat = max(sat, warm / el)
    # open loop at args.load x saturation
    rate = args.load * sat
    rng = np.random.default_rng(55)
    ids = list(range(warm, len(reqs)))
    arrivals = list(np.cumsum(rng.exponential(1.0 / rate, len(ids))))
    comps, el = run(ids, arrivals)
    srv.close()
    bad = [c.id for c in comps if not (c.status == 0 and c.nbe_max <= 1e-15)]
    if bad:
        print("served requests did not reach nbe <= 1e-15: %s" % bad[:10], file=sys.stderr)
        sys.exit(1)
    lat = sorted(c.t_end_ms - c.t_submit_ms for c in comps)
    rhs = sum(c.nrhs for c in comps)
    p99 = lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)]
    # FP64 getrf + getrs on the same GPU, requests one after another
    torch.cuda.synchronize()
    tc = time.perf_counter()
    for i in ids:
        A, B, _ = data[i]
        LU, piv = torch.linalg.lu_factor(A)
        torch.linalg.lu_solve(LU, piv, B)
    torch.cuda.synchronize()
    tcomp = time.perf_counter() - tc
    print(json.dumps({
        "metric": "solves/s to FP64 backward err 1e-15 vs FP64 getrf+getrs; p50/p99 latency",
        "value": round(rhs / el, 3), "unit": "solves/s", "n_gpus": 1, "steps": len(ids), "warmup": warm,
        "ms_per_step": round(1000.0 * el / len(ids), 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp16-factor/fp32-working/fp64-residual (mixed)",
        "data": "synthetic randsvd (seeded, generated on the device), float64",
        "config": {"workload": "serving_poisson_n256to4096_nrhs1to16", "requests": len(ids),
                   "slots": args.slots, "arrival_rate_per_s": round(rate, 3),
                   "saturation_requests_per_s": round(sat, 3), "load": args.load},
        "requests_per_s": round(len(ids) / el, 3),
        "latency_ms": {"p50": round(lat[len(lat) // 2], 3), "p99": round(p99, 3), "max": round(lat[-1], 3)},
        "fp64_getrf_getrs_sequential": {"solves_per_s": round(rhs / tcomp, 3), "s_total": round(tcomp, 3),
                                        "impl": "torch.linalg.lu_factor+lu_solve float64, request by request"}}))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the solver is a single-device library; "
              "--gpus %d is not supported (see the design notes for how it would shard)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.copy_only:
        copy_only(args.copy_only)
        return
    if args.sparse:
        sparse_bench(args)
        return
    if args.workload == "c4":
        batched_bench(args)
        return
    if args.workload == "c5":
        serving_bench(args)
        return
    import numpy as np
    import torch
    from paper_2107_06200_amd import msir as M
    from paper_2107_06200_amd import workloads as WL

    cid = {"c1": 1, "c2": 2, "c3": 3}[args.workload]
    cfg = WL.CONFIGS[cid]
    prm = cfg["params"]
    n = args.n or cfg["n"]
    A, x_true, b = WL.config_system(cid, n=n)
    dev = torch.device("cuda:0")
    M.lib()
    h = M.Handle(0)
    At = M.colmajor(torch.from_numpy(np.asfortranarray(A)).to(dev))
    bt = torch.from_numpy(b).to(dev)
    P = M.params(lu_update=args.lu_update, **prm)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    res = hist = None
    for _ in range(args.warmup):
        x, res, hist, rc = M.solve(h, At, bt, P=P, x=x)
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        x, res, hist, rc = M.solve(h, At, bt, P=P, x=x)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        if rc != 0 or res.nbe > 1e-15:
            print("solve did not reach nbe <= 1e-15: rc=%d nbe=%.3e" % (rc, res.nbe), file=sys.stderr)
            sys.exit(1)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    solves_per_s = args.steps / elapsed
    ms_per_step = 1000.0 * elapsed / args.steps

    # per kernel class device time: one more solve, outside the timed region, with every
    # launch of the instrumented classes bracketed by HIP events on the library's stream
    M.timing(h, True)
    M.solve(h, At, bt, P=P, x=x)
    torch.cuda.synchronize()
    tm = M.timing_get(h)
    M.timing(h, False)
    tsteps = 1

    # ferr of the last solve against the manufactured solution
    xe = x.cpu().numpy()
    ferr = float(np.abs(xe - x_true).max() / np.abs(x_true).max())

    per_step = {k: (v[0] / tsteps, v[1] / tsteps) for k, v in tm.items()}
    # the dominant kernel class by device time.  When it is the Arnoldi step (one
    # workgroup, j + 1 dependent inner products per launch: bound by the latency of its
    # reductions, not by a throughput), its algorithmic bytes are the basis vectors it
    # reads, summed over the launches of the solve's GMRES iterations
    dom_all = max(tm.items(), key=lambda kv: kv[1][1])[0]
    hbm = {k: v for k, v in tm.items() if algorithmic_bytes(k, n) is not None and v[0] > 0}
    dom = max(hbm.items(), key=lambda kv: kv[1][1])[0]
    launches, tot_ms = tm[dom]
    avg_ms = tot_ms / max(1, launches)
    byt = algorithmic_bytes(dom, n)
    ach = byt / (avg_ms * 1e-3) / 1e9
    roof_products = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom, n),
                     "bytes_per_launch": byt, "avg_launch_ms": round(avg_ms, 5), "launches": launches}
    roof = dict(roof_products)
    if dom_all == "arnoldi":
        a_launches, a_ms = tm["arnoldi"]
        a_bytes = arnoldi_bytes(hist, n, prm["restart"], 4 if prm["u"] == "fp32" else 8)
        a_ach = a_bytes / (a_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": "arnoldi", "achieved": round(a_ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(a_ach / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic("arnoldi", n, ARNOLDI_TRAFFIC_FILE, ARNOLDI_SOURCES),
                "bytes_per_launch": round(a_bytes / max(1, a_launches)), "avg_launch_ms": round(a_ms / max(1, a_launches), 5),
                "launches": a_launches,
                "note": "latency-bound: one workgroup runs the j+1 dependent Gram-Schmidt reductions of a step"}
    if dom_all in ("panel", "swap", "gemm"):
        # the LU dominates (n = 8192): (2/3) n^3 per factorization over the LU classes' device
        # time, against the dense matrix-core peak of the first factor format
        lu_ms = sum(tm[k][1] for k in ("panel", "swap", "gemm") if k in tm)
        flops = res.n_lu * 2.0 / 3.0 * n ** 3
        peak = {"fp16": FP16_MFMA_PEAK_TFLOPS, "bf16": FP16_MFMA_PEAK_TFLOPS, "fp32": 157.3, "fp64": 78.6}[prm["uf"]]
        ach = flops / (lu_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": "lu (panel + interchanges + trailing update)", "achieved": round(ach, 2),
                "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 5), "traffic": None,
                "flops_per_solve": flops, "lu_ms_per_solve": round(lu_ms, 3),
                "note": "set by the panel's pivot chain in one workgroup; the trailing update hides beside it"}
    roof["largest_class"] = dom_all

    # FP64 getrf + getrs on the same GPU (black-box comparator)
    comp = []
    for i in range(6):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        LU, piv = torch.linalg.lu_factor(At)
        xs = torch.linalg.lu_solve(LU, piv, bt.unsqueeze(1))
        e1.record()
        torch.cuda.synchronize()
        if i >= 1:
            comp.append(e0.elapsed_time(e1))
    comp_ms = sorted(comp)[len(comp) // 2]
    nbe_fp64, _ = M.backward_error(h, At, xs[:, 0].contiguous(), bt)

    hsum = {"n_lu": res.n_lu, "gmres_iters": res.gmres_iters,
            "sir_steps": sum(1 for s in hist if s.stage == 0), "steps": len(hist)}
    cpu = None
    if not args.no_cpu_baseline:
        try:
            if cid == 2:
                cpu = cpu_baseline(A, b, hsum)
            elif cid == 1:
                cpu = cpu_baseline_full(A, b, prm)
            else:
                cpu = {"value": None, "note": "the oracle's n = 8192 double-double solve takes hours; its stored "
                                              "run (tests/golden) is the reference for this workload"}
        except Exception as e:  # the baseline must not hide the measurement
            cpu = {"value": None, "error": repr(e)}
    nominal = 2.0 / 3.0 * n ** 3 + 2.0 * n ** 2

    out = {
        "metric": "solves/s to FP64 backward err 1e-15 vs FP64 getrf+getrs; p50/p99 latency",
        "value": round(solves_per_s, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "%s-factor/%s-working/%s-residual (mixed)" % (prm["uf"], prm["u"], prm["ur"]),
        "data": "synthetic randsvd (seeded), float64",
        "config": {"workload": cfg["name"], "n": n, "kappa2": cfg["kappa"], "mode": cfg["mode"],
                   "uf": prm["uf"], "u": prm["u"], "ur": prm["ur"], "ux": prm["ux"], "scaling": prm["scaling"],
                   "tau": prm["tau"], "restart": prm["restart"],
                   "k_max": prm["k_max"] if prm["k_max"] is not None else 0.1 * n, "i_max": prm["i_max"],
                   "stop": "nbe<=1e-15 (dd residual)"},
        "gflops_nominal": round(nominal * solves_per_s / 1e9, 2),
        "history": M.render(hist),
        "nbe": res.nbe,
        "ferr": ferr,
        "latency_ms": {"p50": round(1000 * sorted(times)[len(times) // 2], 3),
                       "p99": round(1000 * sorted(times)[min(len(times) - 1, int(math.ceil(0.99 * len(times))) - 1)], 3)},
        "fp64_getrf_getrs": {"ms": round(comp_ms, 3), "solves_per_s": round(1000.0 / comp_ms, 3),
                             "nbe": nbe_fp64, "impl": "torch.linalg.lu_factor+lu_solve float64"},
        "speedup_vs_fp64_direct": round(solves_per_s / (1000.0 / comp_ms), 4),
        "kernel_ms_per_solve": {k: round(v[1], 3) for k, v in per_step.items()},
        "kernel_launches_per_solve": {k: v[0] for k, v in per_step.items()},
        "roofline": roof,
        "roofline_products": roof_products,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    h.close()


if __name__ == "__main__":
    main()
