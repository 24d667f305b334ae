#!/usr/bin/env python3
"""Benchmark of the product-to-sum element-matrix fill on one MI355X.

One step = one full fill (geometry + coupling factors, moments, contraction)
of the whole batch, inputs resident in HBM.  Prints ONE JSON line.

Default workload (the headline): vector curl-curl + mass, N=6 (540 dofs),
4096 curved triquadratic hexahedra, 12^3 Gauss points, rotated anisotropic
permittivity.  The default run also measures the other workloads (scalar
N=4, mixed orders, vector N=8 in FP64 and split-FP32, learned order) as
compact entries under "configs", each with its rate, the roofline fraction
of its contraction stage and its error against the oracle on a sample.  The
CPU baseline is the FP64 oracle (direct quadrature), built for the host CPU,
on a bounded sample of the headline elements.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
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
# CPU baseline: elements of the headline sample on all allotted threads,
# and on one thread
CPU_SAMPLE = {"vector_n6": 32, "scalar_n4": 64, "scalar_mixed": 40, "vector_n8": 4, "scalar_planewave": 6}
CPU_SAMPLE_1T = {"vector_n6": 6, "scalar_n4": 16, "scalar_mixed": 10, "vector_n8": 1, "scalar_planewave": 2}


def num_dofs(problem: int, N: int) -> int:
    return N ** 3 if problem == 0 else 3 * (N - 1) * N * N


def contract_bytes_per_element(problem: int, N: int, moment_bytes: int = 8) -> int:
    """Algorithmic HBM bytes of the contraction kernel per element: the
    dense FP64 output block written once plus the moment tensors read once
    (FP64, or FP32 in the split form)."""
    nd = num_dofs(problem, N)
    F = 7 if problem == 0 else 12
    K = 2 * N - 1
    return 8 * nd * nd + moment_bytes * F * K ** 3


def direct_flops_per_element(problem: int, N: int, Q) -> int:
    """Algorithmic FP64 flops of direct quadrature of eq. (2) per element:
    the upper triangle of the (symmetric) matrix, each entry a sum over the
    Qu*Qv*Qw points of the coupling-term products (scalar: 9 stiffness + 1
    mass; vector: 4 curl + 1 mass per entry), one multiply-add (2 flops)
    each."""
    nd = num_dofs(problem, N)
    terms = 10 if problem == 0 else 5
    return 2 * (nd * (nd + 1) // 2) * int(np.prod(Q)) * terms


def direct_sf_flops_per_element(problem: int, N: int, Q: int) -> int:
    """Algorithmic FP64 flops of sum-factorized direct quadrature per
    element (rule Q per axis), in the order the kernels take the axes:
    per coupling term of a block (I, J >= I), stage A contracts u
    (nm_I nm_J Q^3 multiply-adds), stage B v (nm_I nm_J nn_I nn_J Q^2),
    stage C w (nm_I nm_J nn_I nn_J np_I np_J Q); in a diagonal block only
    m2 >= m1.  Scalar: one block of 10 terms; vector: six blocks of 5."""
    def dims(g):
        return [N - 1 if (problem == 1 and ax == g) else N for ax in range(3)]
    blocks = [(0, 0)] if problem == 0 else [(i, j) for i in range(3) for j in range(i, 3)]
    terms = 10 if problem == 0 else 5
    macs = 0
    for i, j in blocks:
        di, dj = dims(i), dims(j)
        pairs = sum(dj[0] - (m1 if i == j else 0) for m1 in range(di[0]))
        macs += terms * pairs * (Q ** 3 + di[1] * dj[1] * Q ** 2 + di[1] * dj[1] * di[2] * dj[2] * Q)
    return 2 * macs


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
    """Threads the CPU baseline may use: the CPUs this process may run on,
    capped by OMP_NUM_THREADS when the host sets it (the share of the host
    allotted to one GPU's job)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def contraction_kernel_name(w, split, schedule):
    uniform = len(set(w.orders.tolist())) == 1
    if split:
        return "k_contract_split<%d,I,J,I8> (blocks J >= I)" % w.problem, 6 if w.problem else 1
    if not uniform and schedule and schedule["mode"] == "persistent":
        return "k_contract_persistent_scalar", 1
    if not uniform:
        return "k_contract<0,N,0,0> (one launch per order N)", len(set(w.orders.tolist()))
    N = int(w.orders[0])
    if w.problem == 1 and N <= 6:
        return "k_contract_vector<%d> (the six blocks J >= I in one launch)" % N, 1
    return "k_contract<%d,%d,I,J> (blocks J >= I)" % (w.problem, N), 6 if w.problem else 1


def timed_fill(torch, p2s, ctx, w, steps, warmup, split=False, learned=None, out=None, int8=False):
    """Plan + warm-up + `steps` timed executions of workload w.  Returns
    (info, plan, out, status): info holds ms per step, the stage times (HIP
    events on the launch stream) and the contraction stage's roofline."""
    dev = torch.device("cuda", 0)
    prec = (p2s.SPLIT_INT8 if int8 else p2s.SPLIT_FP32) if split else p2s.FP64
    plan = ctx.plan(w.problem, w.material, w.orders, w.quad, precision=prec)
    if learned is not None:
        plan.set_learned(True, learned["p_cover"], learned["theta"], learned.get("k_direct", p2s.KMAX + 1))
    nodes = torch.from_numpy(w.nodes).to(dev)
    mat = torch.from_numpy(w.mat).to(dev)
    if out is None:
        out = torch.empty(int(plan.offsets[-1]), dtype=torch.float64, device=dev)
    status = torch.empty(w.E, dtype=torch.int32, device=dev)
    schedule = None
    if len(set(w.orders.tolist())) > 1 and not split:
        # mixed orders: the schedule autotuner picks per-order-class launches
        # or the persistent launch (outside the timed region)
        plan.autotune(nodes, mat, out, status)
        mode, wpc = plan.schedule()
        schedule = {"mode": "per_order_class" if mode == 0 else "persistent", "wgs_per_cu": wpc,
                    "chosen_by": "p2s_plan_autotune"}
    for _ in range(warmup):
        plan.execute(nodes, mat, out, status)
    torch.cuda.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.execute(nodes, mat, out, status)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = plan.profile_read()
    plan.profile(False)
    ms_per_step = (t1 - t0) * 1e3 / steps
    c_ms, c_segments = stages["contraction"]
    if len(set(w.orders.tolist())) > 1:
        alg_bytes = sum(contract_bytes_per_element(w.problem, int(n)) for n in w.orders)
    else:
        alg_bytes = w.E * contract_bytes_per_element(w.problem, int(w.orders[0]), 4 if split else 8)
    stage_ms = c_ms / steps
    achieved = alg_bytes / (stage_ms * 1e-3) / 1e9
    kname, per_chunk = contraction_kernel_name(w, split, schedule)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": kname, "unit_of_work": "one contraction stage over the batch",
                "algorithmic_bytes": alg_bytes, "stage_ms": round(stage_ms, 4),
                "launches_per_step": (c_segments // steps) * per_chunk}
    info = {"ms_per_step": ms_per_step, "value": w.E / (ms_per_step * 1e-3), "roofline": roofline,
            "stages_ms_per_step": {k: round(v[0] / steps, 4) for k, v in stages.items()},
            "schedule": schedule, "nodes": nodes, "mat": mat}
    return info, plan, out, status


def oracle_errors(oracle, W, w, out, offsets, idx, nthreads=0, native=False):
    """Per-element relative Frobenius error of the GPU blocks of elements
    idx against the oracle's direct quadrature."""
    sub = W.subset(w, np.asarray(idx))
    ref, roff, _ = oracle.fill(sub.problem, sub.material, sub.nodes, sub.mat, sub.orders, sub.quad,
                               nthreads=nthreads, native=native)
    errs = []
    for i, e in enumerate(idx):
        g = out[int(offsets[e]):int(offsets[e + 1])].cpu().numpy()
        r = ref[roff[i]:roff[i + 1]]
        errs.append(float(np.linalg.norm(g - r) / np.linalg.norm(r)))
    return errs


def compact_configs(torch, p2s, ctx, W, oracle, steps, warmup, log):
    """The other workloads, each as a compact entry measured in this run.
    With `oracle` (the CPU-baseline leg of the run) each entry also holds
    the error of sampled elements against the oracle; without it (the
    --no-cpu-baseline runs) those fields are None."""
    res = {}
    oerr = oracle_errors if oracle is not None else (lambda *a, **k: [])
    top = lambda v: max(v) if v else None
    # scalar N=4, 64 elements (launch-bound), every element against the oracle
    w = W.make("scalar_n4")
    info, plan, out, st = timed_fill(torch, p2s, ctx, w, steps, warmup)
    errs = oerr(oracle, W, w, out, plan.offsets, list(range(w.E)))
    res["scalar_n4"] = {"elements": w.E, "value": round(info["value"], 1), "unit": "element matrices/s",
                        "ms_per_step": round(info["ms_per_step"], 4),
                        "roofline_frac": info["roofline"]["frac"], "bound": "hbm (launch-bound at 64 elements)",
                        "max_rel_err_vs_oracle": top(errs), "oracle_elements": len(errs),
                        "status_nonzero": int((st.cpu().numpy() != 0).sum())}
    log("scalar_n4 done")
    del plan, out
    # mixed orders, autotuned schedule; one sampled element per order class
    w = W.make("scalar_mixed")
    info, plan, out, st = timed_fill(torch, p2s, ctx, w, steps, warmup)
    rng = np.random.default_rng(7)
    pick = sorted(int(rng.choice(np.nonzero(w.orders == n)[0])) for n in range(2, 9))
    errs = oerr(oracle, W, w, out, plan.offsets, pick)
    res["scalar_mixed"] = {"elements": w.E, "value": round(info["value"], 1), "unit": "element matrices/s",
                           "ms_per_step": round(info["ms_per_step"], 4), "roofline_frac": info["roofline"]["frac"],
                           "bound": "hbm", "schedule": info["schedule"],
                           "stages_ms_per_step": info["stages_ms_per_step"],
                           "max_rel_err_vs_oracle": top(errs), "oracle_elements": len(errs),
                           "status_nonzero": int((st.cpu().numpy() != 0).sum())}
    log("scalar_mixed done")
    del plan, out
    torch.cuda.empty_cache()
    # vector N=8, FP64 and split-FP32 (one output buffer for both)
    w = W.make("vector_n8")
    info, plan, out, st = timed_fill(torch, p2s, ctx, w, max(3, steps // 2), 1)
    pick = [0]
    sub = W.subset(w, pick)
    if oracle is not None:
        ref, roff, _ = oracle.fill(sub.problem, sub.material, sub.nodes, sub.mat, sub.orders, sub.quad)
    rel0 = lambda o: (float(np.linalg.norm(o[:int(roff[1])].cpu().numpy() - ref) / np.linalg.norm(ref))
                      if oracle is not None else None)
    e64 = rel0(out)
    n64 = 64
    off64 = torch.from_numpy(plan.offsets[:n64 + 1]).cuda()
    keep64 = out[:int(plan.offsets[n64])].clone()
    res["vector_n8_fp64"] = {"elements": w.E, "value": round(info["value"], 1), "unit": "element matrices/s",
                             "ms_per_step": round(info["ms_per_step"], 4), "roofline_frac": info["roofline"]["frac"],
                             "bound": "hbm", "stages_ms_per_step": info["stages_ms_per_step"],
                             "max_rel_err_vs_oracle": e64, "oracle_elements": int(oracle is not None),
                             "status_nonzero": int((st.cpu().numpy() != 0).sum())}
    del plan
    log("vector_n8 fp64 done")
    info, plan, out, st = timed_fill(torch, p2s, ctx, w, max(3, steps // 2), 1, split=True, out=out)
    es = rel0(out)
    e_vs64 = ctx.rel_error(out[:int(plan.offsets[n64])], keep64, offsets=off64).cpu().numpy()
    res["vector_n8_split_fp32"] = {
        "elements": w.E, "value": round(info["value"], 1), "unit": "element matrices/s",
        "ms_per_step": round(info["ms_per_step"], 4), "roofline_frac": info["roofline"]["frac"], "bound": "hbm",
        "stages_ms_per_step": info["stages_ms_per_step"], "max_rel_err_vs_oracle": es, "oracle_elements": int(oracle is not None),
        "max_rel_err_vs_fp64_gpu": float(e_vs64.max()), "fp64_gpu_elements": n64,
        "speedup_vs_fp64": round(res["vector_n8_fp64"]["ms_per_step"] / info["ms_per_step"], 3)}
    del plan
    log("vector_n8 split done")
    info, plan, out, st = timed_fill(torch, p2s, ctx, w, max(3, steps // 2), 1, split=True, out=out, int8=True)
    ei = rel0(out)
    e_vs64 = ctx.rel_error(out[:int(plan.offsets[n64])], keep64, offsets=off64).cpu().numpy()
    res["vector_n8_split_int8"] = {
        "elements": w.E, "value": round(info["value"], 1), "unit": "element matrices/s",
        "ms_per_step": round(info["ms_per_step"], 4), "roofline_frac": info["roofline"]["frac"], "bound": "hbm",
        "stages_ms_per_step": info["stages_ms_per_step"], "max_rel_err_vs_oracle": ei, "oracle_elements": int(oracle is not None),
        "max_rel_err_vs_fp64_gpu": float(e_vs64.max()), "fp64_gpu_elements": n64,
        "speedup_vs_fp64": round(res["vector_n8_fp64"]["ms_per_step"] / info["ms_per_step"], 3)}
    del plan, out, keep64
    torch.cuda.empty_cache()
    log("vector_n8 split int8 done")
    # learned order against the full rule on the same 50000 elements
    from paper_1703_09619_amd import learned_k
    meta = json.load(open(os.path.splitext(learned_k.DEFAULT_MODEL)[0] + ".json"))
    ctx.mlp_init(0, 1)
    ctx.mlp_load(learned_k.DEFAULT_MODEL)
    w = W.make("scalar_planewave")
    info, plan, out, st = timed_fill(torch, p2s, ctx, w, steps, warmup, learned=meta)
    rules = plan.rules()
    stn = st.cpu().numpy()
    finfo, fplan, ref, _ = timed_fill(torch, p2s, ctx, w, steps, warmup)
    off = torch.from_numpy(plan.offsets).cuda()
    err = ctx.rel_error(out, ref, offsets=off).cpu().numpy()
    pick = [0, w.E - 1]
    eo = oerr(oracle, W, w, out, plan.offsets, pick)
    res["scalar_planewave_learned"] = {
        "elements": w.E, "value": round(info["value"], 1), "unit": "element matrices/s",
        "ms_per_step": round(info["ms_per_step"], 4), "roofline_frac": info["roofline"]["frac"], "bound": "hbm",
        "stages_ms_per_step": info["stages_ms_per_step"],
        "full_rule_value": round(finfo["value"], 1), "speedup_vs_full_rule": round(finfo["ms_per_step"] /
                                                                                  info["ms_per_step"], 3),
        "max_rel_err_vs_full_rule": float(err.max()), "elements_over_1e-8": int((err > 1e-8).sum()),
        "max_rel_err_vs_oracle_24": top(eo), "oracle_elements": len(eo),
        "fallback_rate": float(((stn & 4) != 0).mean()), "mean_points": float(np.prod(rules, 1).mean()),
        "model": {k: meta[k] for k in ("p_cover", "k_direct", "theta", "tol") if k in meta}}
    log("scalar_planewave done")
    del plan, fplan, out, ref
    torch.cuda.empty_cache()
    return res


TABLE1_ORDERS = (3, 4, 6, 8, 10, 12, 14, 16, 18)
# the paper's Table I: fill times (s) of the product-to-sum and the direct
# method for its 16-element mesh, per order M = N (Core2Duo 2.5 GHz; context)
PAPER_TABLE1 = {3: (0.104, 0.100), 4: (0.121, 0.148), 6: (0.170, 0.428), 8: (0.229, 1.103),
                10: (0.328, 2.375), 12: (0.461, 4.65), 14: (0.634, 8.21), 16: (0.934, 14.0), 18: (1.29, 22.14)}


def cheb2d_table1(torch, p2s, ctx, W, log, copies=256, reps=5, oracle=None):
    """The paper's 2-D example (Section III, Table I) on its stand-in mesh:
    per order M = N, the fill of the 16 elements by the product-to-sum form
    and by direct quadrature on the GPU (one call each, the paper's batch),
    the same 16 elements repeated `copies` times (throughput), the largest
    difference between the two forms and against the oracle, and the
    measured and predicted (D/15, D = MN, Section IV) reduction factors."""
    ocheb = oracle.cheb2d if oracle is not None else None
    rows = []
    mesh = W.cheb2d_mesh()
    big = W.cheb2d_replicated(copies)
    dev = torch.device("cuda", 0)
    for M in TABLE1_ORDERS:
        Q = min(32, M + 6)
        row = {"M": M, "Q": Q, "dofs": 2 * M * (M + 1)}
        for name, w in (("mesh16", mesh), ("replicated", big)):
            c = ctx.cheb2d(w.E, M, Q)
            nodes = torch.from_numpy(w.nodes).to(dev)
            mat = torch.from_numpy(w.mat).to(dev)
            out = torch.empty(w.E * c.ndof * c.ndof, dtype=torch.float64, device=dev)
            st = torch.empty(w.E, dtype=torch.int32, device=dev)
            res = {}
            for meth, key in ((p2s.METHOD_P2S, "p2s"), (p2s.METHOD_DIRECT, "direct")):
                c.execute(nodes, mat, meth, out=out, status=st)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    c.execute(nodes, mat, meth, out=out, status=st)
                torch.cuda.synchronize()
                res[key + "_ms"] = (time.perf_counter() - t0) * 1e3 / reps
                if name == "mesh16":
                    res[key + "_out"] = out.view(w.E, -1).cpu().numpy().copy()
            if name == "mesh16":
                d = res["p2s_out"] - res["direct_out"]
                row["max_rel_diff_p2s_vs_direct"] = float(
                    (np.linalg.norm(d, axis=1) / np.linalg.norm(res["direct_out"], axis=1)).max())
                if ocheb is not None:
                    ref, _ = ocheb.fill(w.nodes, w.mat, M, Q)
                    nrm = np.linalg.norm(ref, axis=1)
                    row["max_rel_err_p2s_vs_oracle"] = float(
                        (np.linalg.norm(res["p2s_out"] - ref, axis=1) / nrm).max())
                    row["max_rel_err_direct_vs_oracle"] = float(
                        (np.linalg.norm(res["direct_out"] - ref, axis=1) / nrm).max())
                row["mesh16_p2s_ms"] = round(res["p2s_ms"], 4)
                row["mesh16_direct_ms"] = round(res["direct_ms"], 4)
            else:
                c.profile(True)
                c.execute(nodes, mat, p2s.METHOD_P2S, out=out, status=st)
                ms = c.profile(False)
                nd = c.ndof
                gbs = w.E * (8 * nd * nd + 8 * 4 * (2 * M + 1) ** 2) / (ms[2] * 1e-3) / 1e9
                row["replicated_elements"] = w.E
                row["replicated_p2s_elements_per_s"] = round(w.E / (res["p2s_ms"] * 1e-3), 1)
                row["replicated_direct_elements_per_s"] = round(w.E / (res["direct_ms"] * 1e-3), 1)
                row["p2s_gather_roofline_frac"] = round(gbs / HBM_PEAK_GBS, 4)
            del out, c
        row["measured_reduction_mesh16"] = round(row["mesh16_direct_ms"] / row["mesh16_p2s_ms"], 3)
        row["measured_reduction_replicated"] = round(row["replicated_p2s_elements_per_s"] /
                                                     row["replicated_direct_elements_per_s"], 3)
        row["predicted_reduction_D_over_15"] = round(M * M / 15.0, 3)
        row["paper_reduction"] = round(PAPER_TABLE1[M][1] / PAPER_TABLE1[M][0], 3)
        rows.append(row)
        log("cheb2d M=%d done" % M)
    torch.cuda.empty_cache()
    return {"description": "paper's 2-D example (curl-curl + mass, Chebyshev basis of eq. (6), eps_r = "
                           "2 exp(x+y+2)) on a 16-element stand-in mesh of the Fig. 1 domain; Q = min(32, M+6)",
            "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="vector_n6", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--configs", default="auto", choices=["auto", "all", "none"],
                    help="measure the other workloads as compact entries (auto: with the default headline)")
    ap.add_argument("--direct-elements", type=int, default=64,
                    help="elements of the same workload filled by the GPU direct-quadrature baseline "
                         "(0 = skip)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "split_fp32", "split_int8"],
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

    def log(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    import torch
    import paper_1703_09619_amd as p2s
    from paper_1703_09619_amd import workloads as W

    w = W.make(args.workload)
    dev = torch.device("cuda", 0)
    ctx = p2s.Context(0)
    split = args.precision in ("split_fp32", "split_int8")
    int8 = args.precision == "split_int8"
    learned = None
    if args.workload == "scalar_planewave":
        from paper_1703_09619_amd import learned_k
        learned = json.load(open(os.path.splitext(learned_k.DEFAULT_MODEL)[0] + ".json"))
        ctx.mlp_init(0, 1)
        ctx.mlp_load(learned_k.DEFAULT_MODEL)
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    info, plan, out, status = timed_fill(torch, p2s, ctx, w, args.steps, args.warmup, split=split, learned=learned,
                                         int8=int8)
    nodes, mat = info["nodes"], info["mat"]
    ms_per_step = info["ms_per_step"]
    value = info["value"]
    st = status.cpu().numpy()
    roofline = info["roofline"]
    traffic = measured_traffic(args.workload, args.precision)
    roofline["traffic"] = None if traffic is None else round(traffic)
    log("headline %s: %.1f element matrices/s" % (args.workload, value))

    learned_info = None
    if learned is not None:
        # the same plan without the network (full rule on every axis)
        ref = torch.empty_like(out)
        rst = torch.empty_like(status)
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
        learned_info = dict(learned)
        learned_info.update(full_rule_elements_per_s=round(w.E / ((f1 - f0) / args.steps), 1),
                            speedup=round(((f1 - f0) / args.steps) / (ms_per_step * 1e-3), 3),
                            max_rel_err_vs_full_rule=float(err.max()),
                            fallback_rate=float(((st & 4) != 0).mean()), mean_points=float(np.prod(rules, 1).mean()))
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
        precision = {"form": args.precision, "elements_compared": n64,
                     "max_rel_err_vs_fp64_gpu": float(e64.max()), "mean_rel_err_vs_fp64_gpu": float(e64.mean())}

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "element matrices/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ("i8 MFMA on exact 7-bit operand slices + f64" if int8 else
                  "f32 MFMA on exact 10-bit operand slices + f64") if split else "f64",
        "data": "synthetic (seeded curved triquadratic hexahedra and analytic materials)",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "elements": w.E,
                   "orders": sorted(set(int(n) for n in w.orders)), "gauss_points": w.quad[0].tolist(),
                   **({"schedule": info["schedule"]} if info["schedule"] else {})},
        "roofline": roofline,
        "stages_ms_per_step": info["stages_ms_per_step"],
        "status_nonzero": int((st != 0).sum()),
    }
    if learned_info is not None:
        result["learned_order"] = learned_info

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
        reps = 3
        dplan.profile(True)
        d0 = time.perf_counter()
        for _ in range(reps):
            dplan.execute(dn, dm, dout, dst)
        torch.cuda.synchronize()
        d1 = time.perf_counter()
        dst_ms = dplan.profile_read()["other"][0] / reps
        ref = out[:int(dplan.offsets[-1])]
        derr = float(((dout - ref).norm() / ref.norm()).item())
        flops = sub.E * direct_flops_per_element(w.problem, int(w.orders[0]), w.quad[0])
        tf = flops / (dst_ms * 1e-3) / 1e12
        result["gpu_direct_quadrature"] = {
            "value": round(sub.E * reps / (d1 - d0), 1), "unit": "element matrices/s", "elements": sub.E,
            "rel_frobenius_diff_vs_p2s": derr,
            "roofline": {"bound": "fp64", "kernel": "k_direct<%d>" % w.problem, "achieved": round(tf, 2),
                         "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(tf / FP64_PEAK_TFLOPS, 4),
                         "algorithmic_flops": flops, "kernel_ms": round(dst_ms, 4)}}
        del dout
        log("direct baseline done")
    Nh = int(w.orders[0])
    if len(set(w.orders.tolist())) == 1 and (w.quad == 2 * Nh).all() and not split and learned is None:
        # sum-factorized direct quadrature of every entry on the whole batch
        # (the strong baseline: same discrete matrix, dense tables at the
        # 2N Gauss points instead of moments and linearization tables)
        splan = ctx.plan(w.problem, w.material, w.orders, w.quad, method=p2s.METHOD_DIRECT_SF)
        sout = torch.empty_like(out)
        sst = torch.empty_like(status)
        splan.execute(nodes, mat, sout, sst)
        torch.cuda.synchronize()
        splan.profile(True)
        d0 = time.perf_counter()
        for _ in range(args.steps):
            splan.execute(nodes, mat, sout, sst)
        torch.cuda.synchronize()
        d1 = time.perf_counter()
        sst_ms = splan.profile_read()["contraction"][0] / args.steps
        serr = ctx.rel_error(sout, out, offsets=torch.from_numpy(plan.offsets).to(dev)).cpu().numpy()
        flops = w.E * direct_sf_flops_per_element(w.problem, Nh, int(w.quad[0, 0]))
        tf = flops / (sst_ms * 1e-3) / 1e12
        sms = (d1 - d0) * 1e3 / args.steps
        result["gpu_direct_sum_factorized"] = {
            "value": round(w.E / (sms * 1e-3), 1), "unit": "element matrices/s", "elements": w.E,
            "ms_per_step": round(sms, 4), "p2s_speedup": round(sms / ms_per_step, 3),
            "max_rel_frobenius_diff_vs_p2s": float(serr.max()),
            "roofline": {"bound": "fp64", "kernel": ("k_contract_vector<%d,true> (the six blocks in one launch)" % Nh if w.problem == 1 and Nh <= 6
                                    else "k_contract<%d,%d,I,J,true> (blocks J >= I)" % (w.problem, Nh)),
                         "achieved": round(tf, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tf / FP64_PEAK_TFLOPS, 4), "algorithmic_flops": flops,
                         "stage_ms": round(sst_ms, 4)}}
        del sout, splan
        log("sum-factorized direct baseline done")

    if not split and learned is None and args.configs != "none":
        # the same fill writing each matrix's upper triangle only (packed
        # symmetric output: half the bytes of the dense blocks)
        pplan = ctx.plan(w.problem, w.material, w.orders, w.quad, output=p2s.OUTPUT_PACKED_UPPER)
        pout = torch.empty(int(pplan.offsets[-1]), dtype=torch.float64, device=dev)
        pst = torch.empty_like(status)
        pplan.execute(nodes, mat, pout, pst)
        torch.cuda.synchronize()
        pplan.profile(True)
        d0 = time.perf_counter()
        for _ in range(args.steps):
            pplan.execute(nodes, mat, pout, pst)
        torch.cuda.synchronize()
        d1 = time.perf_counter()
        pst_ms = pplan.profile_read()["contraction"][0] / args.steps
        nd = num_dofs(w.problem, int(w.orders[0]))
        F = 7 if w.problem == 0 else 12
        pbytes = w.E * (8 * nd * (nd + 1) // 2 + 8 * F * (2 * int(w.orders[0]) - 1) ** 3)
        pach = pbytes / (pst_ms * 1e-3) / 1e9
        pms = (d1 - d0) * 1e3 / args.steps
        result["packed_upper_output"] = {
            "value": round(w.E / (pms * 1e-3), 1), "unit": "element matrices/s", "ms_per_step": round(pms, 4),
            "layout": "upper triangle of each symmetric element matrix, row by row",
            "roofline": {"bound": "hbm", "achieved": round(pach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(pach / HBM_PEAK_GBS, 4), "algorithmic_bytes": pbytes,
                         "stage_ms": round(pst_ms, 4)}}
        del pout, pplan
        log("packed output done")

    if not args.no_cpu_baseline:
        import oracle
        tmpd = tempfile.mkdtemp(prefix="p2s_oracle_")
        oracle.use_native(tmpd)
        n = min(CPU_SAMPLE[args.workload], w.E)
        idx = np.random.default_rng(7).choice(w.E, size=n, replace=False)
        idx.sort()
        cores = cpu_threads()
        c0 = time.perf_counter()
        errs = oracle_errors(oracle, W, w, out, plan.offsets, idx, nthreads=cores, native=True)
        c1 = time.perf_counter()
        n1 = min(CPU_SAMPLE_1T[args.workload], n)
        sub1 = W.subset(w, idx[:n1])
        s0 = time.perf_counter()
        oracle.fill(sub1.problem, sub1.material, sub1.nodes, sub1.mat, sub1.orders, sub1.quad, nthreads=1,
                    native=True)
        s1 = time.perf_counter()
        result["cpu_baseline"] = {
            "value": round(n / (c1 - c0), 3), "unit": "element matrices/s", "cores": cores, "kind": "oracle",
            "sample": "%d seeded elements of the same workload (GPU blocks compared with them), direct "
                      "quadrature, FP64, gcc -O3 -march=native, OpenMP over elements" % n,
            "single_core_value": round(n1 / (s1 - s0), 3), "single_core_sample": "%d of those elements" % n1,
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
        result["max_rel_err_vs_oracle"] = max(errs)
        log("cpu baseline done")
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

    run_configs = args.configs == "all" or (args.configs == "auto" and args.workload == "vector_n6" and not split)
    if run_configs:
        # the oracle comparisons of the compact entries belong to the
        # CPU-baseline leg: skipped with --no-cpu-baseline
        oracle = None
        if not args.no_cpu_baseline:
            import oracle
            import oracle.cheb2d  # noqa: F401
        del out, status
        plan = None
        torch.cuda.empty_cache()
        result["configs"] = compact_configs(torch, p2s, ctx, W, oracle, args.steps, args.warmup, log)
        result["configs"]["cheb2d_table1"] = cheb2d_table1(torch, p2s, ctx, W, log, oracle=oracle)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
