#!/usr/bin/env python3
"""Benchmark of the product-to-sum element-matrix fill on one MI355X.

One step = one full fill (geometry + coupling factors, moments, contraction)
of the whole batch, inputs resident in HBM.  Prints ONE JSON line.

Default workload (the headline): vector curl-curl + mass, N=6 (540 dofs),
4096 curved triquadratic hexahedra, 12^3 Gauss points, rotated anisotropic
permittivity.  The CPU baseline is the FP64 oracle (direct quadrature) on a
bounded sample of the same elements, run on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "element matrices/s at N=6 (rel. Frobenius err ≤1e-10); % of HBM/MFMA peak"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

WORKLOADS = {
    "vector_n6": "vector curl-curl+mass, N=6 (540 dofs), 4096 curved triquadratic hexahedra, "
                 "12^3 Gauss points, node noise 0.15, eps = R^T diag(1+0.5 sin(k.x+2 pi a/3)) R",
    "scalar_n4": "scalar diffusion+mass, N=4 (64 dofs), 64 elements, 8^3 points, node noise 0.1",
    "scalar_mixed": "scalar diffusion+mass, N~U{2..8}, Q=2N, 20000 elements, node noise 0.1",
    "vector_n8": "vector curl-curl+mass, N=8 (1344 dofs), 8192 elements, 16^3 points",
    "scalar_planewave": "scalar diffusion+mass, N=6 (216 dofs), 50000 elements, eps = 1 + 0.8 sin(k.x+phase), "
                        "|k| log-uniform in [0.5,16] pi, node noise U[0,0.3]; Gauss rule per axis chosen by the "
                        "learned order (full rule 24^3, tail check with fallback)",
}
CPU_SAMPLE = {"vector_n6": 24, "scalar_n4": 64, "scalar_mixed": 40, "vector_n8": 4, "scalar_planewave": 6}


def contract_bytes_per_element(problem: int, N: int, moment_bytes: int = 8) -> int:
    """Algorithmic HBM bytes of the contraction kernel per element: the
    dense FP64 output block written once plus the moment tensors read once
    (FP64, or FP32 in the split form)."""
    nd = N ** 3 if problem == 0 else 3 * (N - 1) * N * N
    F = 7 if problem == 0 else 12
    K = 2 * N - 1
    return 8 * nd * nd + moment_bytes * F * K ** 3


TRAFFIC_PROFILES = {("vector_n6", "fp64"): "profiles/k_contract_vector_n6.md"}


def measured_traffic(workload: str, precision: str):
    """HBM bytes per contraction stage from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-probe factors), or
    None when there is none or the contraction sources changed since."""
    import hashlib
    name = TRAFFIC_PROFILES.get((workload, precision))
    if name is None or not os.path.exists(os.path.join(ROOT, name)):
        return None
    fields = {}
    for line in open(os.path.join(ROOT, name)):
        if ":" in line and line.split(":", 1)[0] in ("traffic_bytes_per_step", "sources_sha256", "sources"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    try:
        h = hashlib.sha256()
        for f in fields["sources"].split():
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != fields["sources_sha256"]:
            return None
        return float(fields["traffic_bytes_per_step"])
    except (KeyError, OSError, ValueError):
        return None


def cpu_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="vector_n6", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--direct-elements", type=int, default=64,
                    help="elements of the same workload filled by the GPU direct-quadrature baseline "
                         "(0 = skip)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "split_fp32"],
                    help="arithmetic of the moment and contraction stages; split_fp32 also times the FP64 "
                         "path on the same inputs and reports the split error against it")
    ap.add_argument("--copy-probe", action="store_true",
                    help="before the fill, run a plain 1 GiB device copy three times (a known-size "
                         "reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the fill is element-parallel and is measured on a "
              "single MI355X; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1703_09619_amd as p2s
    from paper_1703_09619_amd import workloads as W

    w = W.make(args.workload)
    dev = torch.device("cuda", 0)
    ctx = p2s.Context(0)
    split = args.precision == "split_fp32"
    plan = ctx.plan(w.problem, w.material, w.orders, w.quad, precision=p2s.SPLIT_FP32 if split else p2s.FP64)
    learned = None
    if args.workload == "scalar_planewave":
        from paper_1703_09619_amd import learned_k
        meta = json.load(open(os.path.splitext(learned_k.DEFAULT_MODEL)[0] + ".json"))
        ctx.mlp_init(0, 1)
        ctx.mlp_load(learned_k.DEFAULT_MODEL)
        plan.set_learned(True, meta["p_cover"], meta["theta"], meta.get("k_direct", p2s.KMAX + 1))
        learned = meta
    nodes = torch.from_numpy(w.nodes).to(dev)
    mat = torch.from_numpy(w.mat).to(dev)
    out = torch.empty(int(plan.offsets[-1]), dtype=torch.float64, device=dev)
    status = torch.empty(w.E, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    schedule = None
    if len(set(w.orders.tolist())) > 1 and not split:
        # mixed orders: the schedule autotuner picks per-order-class launches
        # or the persistent launch (outside the timed region)
        plan.autotune(nodes, mat, out, status)
        mode, wpc = plan.schedule()
        schedule = {"mode": "per_order_class" if mode == 0 else "persistent", "wgs_per_cu": wpc,
                    "chosen_by": "p2s_plan_autotune"}

    for _ in range(args.warmup):
        plan.execute(nodes, mat, out, status)
    torch.cuda.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.execute(nodes, mat, out, status)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = plan.profile_read()
    plan.profile(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = w.E / (ms_per_step * 1e-3)
    st = status.cpu().numpy()

    # dominant kernel: the contraction stage (HIP events on the launch stream
    # around the stage's launches: one kernel per component block, per order
    # class for mixed orders, or one persistent kernel)
    c_ms, c_segments = stages["contraction"]
    if w.problem == 0 and len(set(w.orders.tolist())) > 1:
        alg_bytes = sum(contract_bytes_per_element(0, int(n)) for n in w.orders)
    else:
        alg_bytes = w.E * contract_bytes_per_element(w.problem, int(w.orders[0]), 4 if split else 8)
    stage_ms = c_ms / args.steps
    achieved = alg_bytes / (stage_ms * 1e-3) / 1e9
    n_uniform = len(set(w.orders.tolist())) == 1
    if split:
        kname, per_chunk = "k_contract_split<%d,I,J> (blocks J >= I)" % w.problem, 6 if w.problem else 1
    elif not n_uniform and schedule["mode"] == "persistent":
        kname, per_chunk = "k_contract_persistent_scalar", 1
    elif not n_uniform:
        kname, per_chunk = "k_contract<0,N,0,0> (one launch per order N)", len(set(w.orders.tolist()))
    else:
        kname = "k_contract<%d,%d,I,J> (blocks J >= I)" % (w.problem, int(w.orders[0]))
        per_chunk = 6 if w.problem else 1
    traffic = measured_traffic(args.workload, args.precision)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic),
                "kernel": kname, "unit_of_work": "one contraction stage over the batch",
                "algorithmic_bytes": alg_bytes, "stage_ms": round(stage_ms, 4),
                "launches_per_step": (c_segments // args.steps) * per_chunk}

    if learned is not None:
        # the same plan without the network (full rule on every axis)
        ref = torch.empty_like(out)
        rst = torch.empty_like(status)
        stn = st
        rules = plan.rules()
        plan.set_learned(False)
        plan.execute(nodes, mat, ref, rst)
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        for _ in range(args.steps):
            plan.execute(nodes, mat, ref, rst)
        torch.cuda.synchronize()
        f1 = time.perf_counter()
        err = ctx.rel_error(out, ref, offsets=torch.from_numpy(plan.offsets).to(dev)).cpu().numpy()
        learned.update(full_rule_elements_per_s=round(w.E / ((f1 - f0) / args.steps), 1),
                       speedup=round(((f1 - f0) / args.steps) / (ms_per_step * 1e-3), 3),
                       max_rel_err_vs_full_rule=float(err.max()),
                       fallback_rate=float(((stn & 4) != 0).mean()), mean_points=float(np.prod(rules, 1).mean()))
        del ref

    precision = None
    if split:
        # the same elements through the FP64 path: error on the first 64
        # elements, then the FP64 rate on the whole batch (into the same buffer,
        # after the split result has been checked)
        n64 = min(64, w.E)
        sub64 = W.subset(w, np.arange(n64))
        p64 = ctx.plan(sub64.problem, sub64.material, sub64.orders, sub64.quad)
        o64, _ = p64.execute(torch.from_numpy(sub64.nodes).to(dev), torch.from_numpy(sub64.mat).to(dev))
        e64 = ctx.rel_error(out[:int(p64.offsets[-1])], o64,
                            offsets=torch.from_numpy(p64.offsets).to(dev)).cpu().numpy()
        del o64
        precision = {"form": "split_fp32", "elements_compared": n64,
                     "max_rel_err_vs_fp64_gpu": float(e64.max()), "mean_rel_err_vs_fp64_gpu": float(e64.mean())}

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "element matrices/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (hi/lo split operands) + f64" if split else "f64",
        "data": "synthetic (seeded curved triquadratic hexahedra and analytic materials)",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "elements": w.E,
                   "orders": sorted(set(int(n) for n in w.orders)), "gauss_points": w.quad[0].tolist(),
                   **({"schedule": schedule} if schedule else {})},
        "roofline": roofline,
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items()},
        "status_nonzero": int((st != 0).sum()),
    }
    if learned is not None:
        result["learned_order"] = learned

    if args.direct_elements > 0 and len(set(w.orders.tolist())) == 1:
        # the method the paper compares against, on the GPU: direct quadrature
        # of every entry (same inputs, first elements of the batch)
        sub = W.subset(w, np.arange(min(args.direct_elements, w.E)))
        dplan = ctx.plan(sub.problem, sub.material, sub.orders, sub.quad, method=p2s.METHOD_DIRECT)
        dn = torch.from_numpy(sub.nodes).to(dev)
        dm = torch.from_numpy(sub.mat).to(dev)
        dout = torch.empty(int(dplan.offsets[-1]), dtype=torch.float64, device=dev)
        dst = torch.empty(sub.E, dtype=torch.int32, device=dev)
        dplan.execute(dn, dm, dout, dst)
        torch.cuda.synchronize()
        d0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            dplan.execute(dn, dm, dout, dst)
        torch.cuda.synchronize()
        d1 = time.perf_counter()
        ref = out[:int(dplan.offsets[-1])]
        derr = float(((dout - ref).norm() / ref.norm()).item())
        result["gpu_direct_quadrature"] = {
            "value": round(sub.E * reps / (d1 - d0), 1), "unit": "element matrices/s", "elements": sub.E,
            "rel_frobenius_diff_vs_p2s": derr}
        del dout

    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        n = min(CPU_SAMPLE[args.workload], w.E)
        idx = np.random.default_rng(7).choice(w.E, size=n, replace=False)
        idx.sort()
        sub = W.subset(w, idx)
        cores = cpu_threads()
        c0 = time.perf_counter()
        ref, roff, _ = oracle.fill(sub.problem, sub.material, sub.nodes, sub.mat, sub.orders, sub.quad,
                                   nthreads=cores)
        c1 = time.perf_counter()
        errs = []
        off = plan.offsets
        for i, e in enumerate(idx):
            g = out[int(off[e]):int(off[e + 1])].cpu().numpy()
            r = ref[roff[i]:roff[i + 1]]
            errs.append(float(np.linalg.norm(g - r) / np.linalg.norm(r)))
        result["cpu_baseline"] = {"value": round(n / (c1 - c0), 3), "unit": "element matrices/s",
                                  "cores": cores, "kind": "oracle",
                                  "sample": "%d seeded elements of the same workload, direct quadrature, "
                                            "FP64, OpenMP over elements" % n}
        result["max_rel_err_vs_oracle"] = max(errs)
    if precision is not None:
        del plan
        p64 = ctx.plan(w.problem, w.material, w.orders, w.quad)
        p64.execute(nodes, mat, out, status)
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        for _ in range(args.steps):
            p64.execute(nodes, mat, out, status)
        torch.cuda.synchronize()
        f1 = time.perf_counter()
        precision["fp64_elements_per_s"] = round(w.E * args.steps / (f1 - f0), 1)
        precision["split_speedup_vs_fp64"] = round((f1 - f0) / args.steps / (ms_per_step * 1e-3), 3)
        result["precision"] = precision
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
