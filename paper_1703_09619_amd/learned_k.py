"""Training and calibration of the learned quadrature order.

The network predicts, per element and axis, how many Gauss points K in
{6..24} the coupling factor needs before the moment stage.  Everything here
drives the C ABI: labels come from the method's own GPU fills, training uses
the library's forward/backward/Adam kernels, and the final check is the
plain method's full-rule fill.

Labels (per element e and axis x): the smallest K such that the moment
tensors sampled with K points along x (the full rule on the other axes)
differ from the full-rule moments by at most `tol_moment` in relative
Frobenius norm, for that K and every larger one.  The matrix is a fixed
linear image of the moments, so `tol_moment` is set from the measured ratio
of matrix error to moment error on a sample, with a safety factor.

    python -m paper_1703_09619_amd.learned_k --train 200000 --out model.p2sk
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import workloads as W

KMIN, KMAX = 6, 24
NCLS = KMAX - KMIN + 1
MODEL_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "models")
DEFAULT_MODEL = os.path.join(MODEL_DIR, "kmodel_scalar_n6.p2sk")


def _dev(w, torch):
    return torch.from_numpy(w.nodes).cuda(), torch.from_numpy(w.mat).cuda()


def moment_errors(ctx, w, batch=8192, log=print):
    """errs[e, x, c]: relative moment error with K = KMIN + c points on axis x."""
    import torch
    E = w.E
    errs = np.zeros((E, 3, NCLS))
    for s in range(0, E, batch):
        sub = W.subset(w, np.arange(s, min(E, s + batch)))
        nodes, mat = _dev(sub, torch)
        full = np.full((sub.E, 3), KMAX, np.int32)
        p = ctx.plan(sub.problem, sub.material, sub.orders, full)
        ref = p.moments(nodes, mat).reshape(sub.E, -1)
        p.close()
        block = ref.shape[1]
        for x in range(3):
            for c in range(NCLS - 1):
                q = full.copy()
                q[:, x] = KMIN + c
                p = ctx.plan(sub.problem, sub.material, sub.orders, q)
                m = p.moments(nodes, mat).reshape(sub.E, -1)
                errs[s:s + sub.E, x, c] = ctx.rel_error(m, ref, block=block).cpu().numpy()
                p.close()
                del m
        torch.cuda.synchronize()
        log("moment errors: %d/%d elements" % (min(E, s + batch), E))
    return errs


def labels_from_errors(errs, tol):
    """Smallest class c with errs[..., c'] <= tol for every c' >= c."""
    ok = errs <= tol
    ok[..., -1] = True
    # suffix-all: ok_from[c] = all(ok[c:])
    suffix = np.flip(np.cumprod(np.flip(ok, -1), -1), -1).astype(bool)
    return np.argmax(suffix, axis=-1).astype(np.int32)


def matrix_vs_moment_ratio(ctx, w, n=256):
    """max over a sample of (matrix error) / (moment error) for single-axis
    reductions, used to translate the matrix tolerance to moments."""
    import torch
    sub = W.subset(w, np.arange(min(n, w.E)))
    nodes, mat = _dev(sub, torch)
    full = np.full((sub.E, 3), KMAX, np.int32)
    pf = ctx.plan(sub.problem, sub.material, sub.orders, full)
    mref = pf.moments(nodes, mat).reshape(sub.E, -1)
    Mref, _ = pf.execute(nodes, mat)
    off = torch.from_numpy(pf.offsets).cuda()
    ratios = []
    for x in range(3):
        for K in (8, 11, 14, 17, 20):
            q = full.copy()
            q[:, x] = K
            p = ctx.plan(sub.problem, sub.material, sub.orders, q)
            m = p.moments(nodes, mat).reshape(sub.E, -1)
            M, _ = p.execute(nodes, mat)
            em = ctx.rel_error(m, mref, block=m.shape[1]).cpu().numpy()
            eM = ctx.rel_error(M, Mref, offsets=off).cpu().numpy()
            good = em > 1e-13
            ratios.append((eM[good] / em[good]).max() if good.any() else 0.0)
            p.close()
    pf.close()
    return float(max(ratios))


def train(ctx, X, Y, epochs=20, batch=1024, lr=1e-3, seed=0, log=print):
    """Minibatch Adam on the library's kernels; X [n][85] float32 (device),
    Y [n][3] int32 (device).  Returns the per-epoch mean loss."""
    import torch
    n = X.shape[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=g)
        tot = 0.0
        steps = 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            xb = X.index_select(0, idx).contiguous()
            yb = Y.index_select(0, idx).contiguous()
            ctx.mlp_train_step(xb, yb, lr, loss)
            tot += float(loss.item()) / batch
            steps += 1
        hist.append(tot / max(steps, 1))
        log("epoch %d loss %.4f" % (ep, hist[-1]))
    return hist


def learned_fill(ctx, w, p_cover, theta, k_direct=KMAX + 1):
    """(plan, out, status) of the learned fill of workload w (rules 24^3)."""
    import torch
    nodes, mat = _dev(w, torch)
    full = np.full((w.E, 3), KMAX, np.int32)
    plan = ctx.plan(w.problem, w.material, w.orders, full)
    plan.set_learned(True, p_cover, theta, k_direct)
    out, st = plan.execute(nodes, mat)
    return plan, out, st


def full_fill(ctx, w):
    """(plan, out, offsets) of the plain full-rule fill of workload w."""
    import torch
    nodes, mat = _dev(w, torch)
    pf = ctx.plan(w.problem, w.material, w.orders, np.full((w.E, 3), KMAX, np.int32))
    ref, _ = pf.execute(nodes, mat)
    return pf, ref, torch.from_numpy(pf.offsets).cuda()


def calibrate_theta(ctx, w, tol, p_cover, k_direct, ref, off, safety=0.5):
    """Largest theta (times `safety`) with no accepted element above tol on
    this held-out set: run the learned fill with no fallback, compare every
    element with the full-rule fill `ref`, and put theta below the smallest
    tail value of an element that misses the tolerance.  Also returns the
    expected cost (mean Gauss points per element including refills)."""
    plan, out, _ = learned_fill(ctx, w, p_cover, 1e300, k_direct)
    tau = plan.tail_values()
    pts = np.prod(plan.rules(), axis=1).astype(np.float64)
    err = ctx.rel_error(out, ref, offsets=off).cpu().numpy()
    plan.close()
    del out
    bad = err > tol
    theta = safety * float(tau[bad].min()) if bad.any() else max(float(tau.max()) * 2.0, 1e-300)
    back = tau > theta
    cost = float((pts + back * KMAX ** 3).mean())
    return theta, dict(n=int(w.E), p_cover=p_cover, k_direct=k_direct, missed_without_check=int(bad.sum()),
                       fallback_rate=float(back.mean()), max_err_accepted=float(err[~back].max()),
                       mean_points=float(pts.mean()), cost_points=cost, theta=theta)


def calibrate(ctx, w, tol, covers=(0.9, 0.95, 0.99), directs=(16, 18, 20, 22, KMAX + 1)):
    """Pick (p_cover, k_direct, theta) with no miss on w and the least
    expected cost."""
    pf, ref, off = full_fill(ctx, w)
    pf.close()
    best = None
    rows = []
    for p in covers:
        for kd in directs:
            theta, info = calibrate_theta(ctx, w, tol, p, kd, ref, off)
            rows.append(info)
            if best is None or info["cost_points"] < best[3]["cost_points"]:
                best = (p, kd, theta, info)
    return best[0], best[1], best[2], rows


def evaluate(ctx, w, p_cover, theta, tol, k_direct=KMAX + 1, reps=3):
    """Learned fill against the full-rule fill: time, errors, rules."""
    import torch
    nodes, mat = _dev(w, torch)
    pf, ref, off = full_fill(ctx, w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        pf.execute(nodes, mat, ref)
    torch.cuda.synchronize()
    t_full = (time.perf_counter() - t0) / reps
    plan, out, st = learned_fill(ctx, w, p_cover, theta, k_direct)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.execute(nodes, mat, out, st)
    torch.cuda.synchronize()
    t_learned = (time.perf_counter() - t0) / reps
    err = ctx.rel_error(out, ref, offsets=off).cpu().numpy()
    stn = st.cpu().numpy()
    rules = plan.rules()
    return dict(E=int(w.E), full_s=t_full, learned_s=t_learned, speedup=t_full / t_learned,
                max_err=float(err.max()), frac_over_tol=float((err > tol).mean()),
                fallback=float(((stn & 4) != 0).mean()),
                mean_points=float(np.prod(rules, axis=1).mean()), mean_rule=rules.mean(0).tolist())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=200000, help="training elements")
    ap.add_argument("--val", type=int, default=16384)
    ap.add_argument("--test", type=int, default=50000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--p-cover", type=float, default=0.95)
    ap.add_argument("--out", default=DEFAULT_MODEL)
    ap.add_argument("--report", default=None)
    ap.add_argument("--model", default=None, help="calibrate and evaluate this trained network (no training)")
    args = ap.parse_args()
    import torch
    import paper_1703_09619_amd as p2s
    log = lambda m: print(m, flush=True)
    ctx = p2s.Context(0)
    ctx.mlp_init(seed=1703, max_batch=4096)
    rep = {}
    t0 = time.perf_counter()
    if args.model:
        ctx.mlp_load(args.model)
        out_path = args.model
    else:
        wtr = W.make("scalar_planewave", E=args.train, seed=W.BASE_SEED + 40)
        ratio = matrix_vs_moment_ratio(ctx, wtr)
        tol_m = 0.5 * args.tol / max(ratio, 1.0)
        log("matrix/moment error ratio %.3g -> moment tolerance %.3g" % (ratio, tol_m))
        errs = moment_errors(ctx, wtr, log=log)
        Y = labels_from_errors(errs, tol_m)
        hist_labels = np.bincount((KMIN + Y).reshape(-1), minlength=KMAX + 1)[KMIN:].tolist()
        nodes, mat = _dev(wtr, torch)
        X = ctx.features(wtr.material, nodes, mat)
        Yd = torch.from_numpy(Y).cuda()
        t1 = time.perf_counter()
        hist = train(ctx, X, Yd, epochs=args.epochs, lr=args.lr, log=log)
        t2 = time.perf_counter()
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        ctx.mlp_save(args.out)
        out_path = args.out
        rep.update(train_elements=args.train, epochs=args.epochs, lr=args.lr, tol_moment=tol_m,
                   matrix_moment_ratio=ratio, label_histogram_K6_to_24=hist_labels, loss=hist,
                   label_seconds=t1 - t0, train_seconds=t2 - t1)
    wval = W.make("scalar_planewave", E=args.val, seed=W.BASE_SEED + 41)
    p_cover, k_direct, theta, rows = calibrate(ctx, wval, args.tol)
    log("calibration: p_cover %.2f k_direct %d theta %.3g" % (p_cover, k_direct, theta))
    for r in rows:
        log("  %s" % r)
    wte = W.make("scalar_planewave", E=args.test)
    ev = evaluate(ctx, wte, p_cover, theta, args.tol, k_direct)
    log("evaluation %s" % ev)
    rep.update(tol=args.tol, p_cover=p_cover, k_direct=k_direct, theta=theta, calibration=rows, evaluation=ev)
    meta = os.path.splitext(out_path)[0] + ".json"
    with open(meta, "w") as f:
        json.dump(dict(p_cover=p_cover, k_direct=k_direct, theta=theta, tol=args.tol), f, indent=1)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
