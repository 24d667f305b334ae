"""GPU parity: the HIP product-to-sum fill against the CPU oracle (direct
quadrature of eq. (2)) on the same seeded inputs, through the C ABI.

Bar: per-element relative Frobenius error <= 1e-10 for the FP64 path.
Both sides use the same tensor Gauss rule, and eq. (3) is an exact
polynomial identity, so the two agree to rounding (the paper's claim that
the method leaves accuracy unchanged, Section V)."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_1703_09619_amd as p2s
    from paper_1703_09619_amd import workloads as W
    oracle.build(force=False)
    ctx = p2s.Context(0)
    return dict(torch=torch, oracle=oracle, p2s=p2s, W=W, ctx=ctx)


def gpu_fill(env, w, **kw):
    torch, p2s = env["torch"], env["p2s"]
    plan = env["ctx"].plan(w["problem"], w["material"], w["orders"], w["quad"], **kw)
    nodes = torch.from_numpy(np.ascontiguousarray(w["nodes"])).cuda()
    mat = torch.from_numpy(np.ascontiguousarray(w["mat"])).cuda()
    out, status = plan.execute(nodes, mat)
    torch.cuda.synchronize()
    return out.cpu().numpy(), plan.offsets, status.cpu().numpy(), plan


def rel_errors(a, b, off):
    errs = []
    for e in range(len(off) - 1):
        x, y = a[off[e]:off[e + 1]], b[off[e]:off[e + 1]]
        errs.append(np.linalg.norm(x - y) / np.linalg.norm(y))
    return np.array(errs)


def check_against_oracle(env, w, sK=1.0, sM=1.0, tol=TOL, method=0):
    print("case", w.get("name"), "E", w["E"], "orders", sorted(set(np.asarray(w["orders"]).tolist())),
          "quad0", np.asarray(w["quad"])[0].tolist(), "method", method, flush=True)
    out, off, st, _ = gpu_fill(env, w, stiff_scale=sK, mass_scale=sM, method=method)
    ref, roff, rst = env["oracle"].fill(w["problem"], w["material"], w["nodes"], w["mat"],
                                        w["orders"], w["quad"], sK, sM)
    assert np.array_equal(off, roff)
    assert np.array_equal(st, rst.astype(st.dtype))
    errs = rel_errors(out, ref, off)
    print("max rel Frobenius error %.3e" % errs.max(), flush=True)
    assert errs.max() <= tol
    return errs


def make_small(env, problem, N, E, Q, seed, material=None):
    W = env["W"]
    rng = np.random.default_rng(seed)
    nodes, _, _ = W.perturbed_nodes(rng, E, 0.12)
    if problem == W.SCALAR:
        material = W.MAT_SINCOSEXP if material is None else material
        if material == W.MAT_SINCOSEXP:
            mat = rng.uniform(math.pi, 4 * math.pi, size=(E, 1))
        else:
            mat = np.concatenate([W.unit_vectors(rng, E) * 6.0, rng.uniform(0, 6, (E, 1))], 1)
    else:
        material = W.MAT_ROTDIAG
        mat = np.zeros((E, 12))
        for e in range(E):
            mat[e, :9] = W.haar_rotation(rng).reshape(-1)
        mat[:, 9:] = W.unit_vectors(rng, E) * rng.uniform(0, 4 * math.pi, (E, 1))
    return W.Workload(name="small", problem=problem, material=material, E=E, nodes=nodes, mat=mat,
                      orders=np.full(E, N, np.int32), quad=np.tile(np.array(Q, np.int32), (E, 1)))


def test_scalar_n4_all_64_elements(env):
    """The 64-element scalar workload (N=4, 8^3 points), every element."""
    w = env["W"].make("scalar_n4")
    check_against_oracle(env, w)


def test_vector_n6_subset(env):
    """Vector curl-curl + mass, N=6 (540 dofs), 12^3 points: a seeded
    subset of the 4096-element workload."""
    W = env["W"]
    w = W.make("vector_n6", E=16)
    check_against_oracle(env, W.subset(w, np.arange(6)))


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7, 8])
def test_scalar_orders_anisotropic_rule(env, N):
    w = make_small(env, 0, N, 3, (N + 1, N + 2, N + 3), seed=100 + N)
    check_against_oracle(env, w)


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7, 8])
def test_vector_orders_anisotropic_rule(env, N):
    Q = (N + 2, N + 1, N + 3) if N < 7 else (5, 6, 7)
    w = make_small(env, 1, N, 2, Q, seed=200 + N)
    check_against_oracle(env, w)


@pytest.mark.parametrize("problem,N,Q,E", [(0, 8, (30, 30, 30), 1), (1, 6, (32, 17, 24), 2)])
def test_largest_rules(env, problem, N, Q, E):
    """Rules above 16 points (the matrix-core form of the moment stage) up
    to the largest the stage's LDS takes: 30^3 at order 8, 32 per axis at
    order 6."""
    w = make_small(env, problem, N, E, Q, seed=400 + N)
    check_against_oracle(env, w)


def test_rule_beyond_moment_lds_is_refused(env):
    """Order 8 with 32^3 points needs 182 KB of LDS in the moment stage:
    plan creation refuses it (no launch)."""
    with pytest.raises(env["p2s"].P2SError):
        env["ctx"].plan(0, 0, np.array([8], np.int32), np.array([[32, 32, 32]], np.int32))


def test_planewave_material_and_scales(env):
    w = make_small(env, 0, 5, 4, (9, 10, 11), seed=7, material=2)
    check_against_oracle(env, w, sK=0.0, sM=1.0)
    check_against_oracle(env, w, sK=1.0, sM=0.0)
    check_against_oracle(env, w, sK=1.0, sM=-2.5)


def test_vector_scales(env):
    w = make_small(env, 1, 4, 3, (6, 6, 6), seed=8)
    check_against_oracle(env, w, sK=1.0, sM=0.0)
    check_against_oracle(env, w, sK=0.0, sM=1.0)


def test_mixed_orders_batch(env):
    """Elements of orders 2..8 in one plan (Q = 2N per element), ragged."""
    W = env["W"]
    w = W.make("scalar_mixed", E=200)
    idx = []
    for N in range(2, 9):
        idx += list(np.nonzero(w["orders"] == N)[0][:2])
    sub = W.subset(w, np.array(sorted(idx)))
    check_against_oracle(env, sub)


def test_sampled_coupling_input(env):
    """Coupling fields given directly at the Gauss points (no geometry)."""
    W = env["W"]
    rng = np.random.default_rng(5)
    for problem, F in ((0, 7), (1, 12)):
        N, Q = 4, (5, 6, 7)
        E = 3
        a = rng.standard_normal((E, F, int(np.prod(Q))))
        w = W.Workload(name="sampled", problem=problem, material=W.ALPHA_SAMPLED, E=E,
                       nodes=np.zeros((E, 27, 3)), mat=a.reshape(E, -1),
                       orders=np.full(E, N, np.int32), quad=np.tile(np.array(Q, np.int32), (E, 1)))
        check_against_oracle(env, w)


def test_coupling_stage(env):
    """Stage (geometry + coupling factors) against the oracle's samples."""
    torch, oracle, W = env["torch"], env["oracle"], env["W"]
    for name, E in (("scalar_n4", 5), ("vector_n6", 3)):
        w = W.subset(W.make(name, E=64 if name == "scalar_n4" else 8), np.arange(E))
        plan = env["ctx"].plan(w.problem, w.material, w.orders, w.quad)
        a = plan.coupling(torch.from_numpy(w.nodes).cuda(), torch.from_numpy(w.mat).cuda()).cpu().numpy()
        for e in range(E):
            ref = oracle.coupling(w.problem, w.material, w.mat[e], w.nodes[e], *w.quad[e])
            assert np.abs(a[e] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_moment_stage(env):
    """Stage (a): moments against their plain definition in the oracle."""
    torch, oracle, W = env["torch"], env["oracle"], env["W"]
    for name, E in (("scalar_n4", 4), ("vector_n6", 2)):
        w = W.subset(W.make(name, E=64 if name == "scalar_n4" else 8), np.arange(E))
        plan = env["ctx"].plan(w.problem, w.material, w.orders, w.quad)
        m = plan.moments(torch.from_numpy(w.nodes).cuda(), torch.from_numpy(w.mat).cuda()).cpu().numpy()
        K = 2 * int(w.orders[0]) - 1
        for e in range(E):
            ref = oracle.moments(w.problem, w.material, w.mat[e], w.nodes[e], *w.quad[e], K)
            assert np.abs(m[e] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_inverted_element_status(env):
    W = env["W"]
    w = make_small(env, 0, 3, 3, (4, 4, 4), seed=3)
    w["nodes"][1, 13] = (2.0, 2.0, 2.0)
    out, off, st, _ = gpu_fill(env, w)
    assert st[1] & 1 and st[0] == 0 and st[2] == 0


def test_empty_batch(env):
    torch, p2s = env["torch"], env["p2s"]
    plan = env["ctx"].plan(0, 0, np.zeros(0, np.int32), np.zeros((0, 3), np.int32))
    out, st = plan.execute(torch.zeros(1, dtype=torch.float64, device="cuda"),
                           torch.zeros(1, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert out.numel() == 0 and st.numel() == 0


def test_argument_errors(env):
    p2s = env["p2s"]
    ctx = env["ctx"]
    with pytest.raises(p2s.P2SError, match="order"):
        ctx.plan(0, 0, [9], [[4, 4, 4]])
    with pytest.raises(p2s.P2SError, match="Gauss"):
        ctx.plan(0, 0, [4], [[33, 4, 4]])
    with pytest.raises(p2s.P2SError, match="isotropic"):
        ctx.plan(0, 1, [4], [[4, 4, 4]])
    with pytest.raises(p2s.P2SError, match="material"):
        ctx.plan(0, 7, [4], [[4, 4, 4]])
    with pytest.raises(p2s.P2SError, match="one order"):
        ctx.plan(0, 3, [4, 5], [[4, 4, 4], [4, 4, 4]])


def test_vector_n6_full_size_sampled(env):
    """The full 4096-element vector workload in the benchmark's launch
    configuration: sampled elements against the oracle, symmetry of every
    element matrix, and bitwise repeatability."""
    torch, W = env["torch"], env["W"]
    w = W.make("vector_n6")
    plan = env["ctx"].plan(w.problem, w.material, w.orders, w.quad)
    nodes = torch.from_numpy(w.nodes).cuda()
    mat = torch.from_numpy(w.mat).cuda()
    out, st = plan.execute(nodes, mat)
    out2, _ = plan.execute(nodes, mat)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    assert torch.equal(out, out2)
    nd = 540
    M = out.view(w.E, nd, nd)
    asym = (M - M.transpose(1, 2)).abs().amax(dim=(1, 2)) / M.abs().amax(dim=(1, 2))
    assert float(asym.max()) <= 1e-13
    pick = [0, 1234, 4095]
    sub = W.subset(w, pick)
    ref, roff, _ = env["oracle"].fill(sub.problem, sub.material, sub.nodes, sub.mat, sub.orders, sub.quad)
    for i, e in enumerate(pick):
        x = M[e].cpu().numpy().reshape(-1)
        y = ref[roff[i]:roff[i + 1]]
        err = np.linalg.norm(x - y) / np.linalg.norm(y)
        print("element", e, "rel err %.3e" % err, flush=True)
        assert err <= TOL


def test_persistent_schedule_matches_per_class(env):
    """Mixed orders: the persistent launch over the cost-sorted work list
    and the per-order-class launches give bit-identical matrices."""
    torch, W = env["torch"], env["W"]
    w = W.make("scalar_mixed", E=300)
    plan = env["ctx"].plan(w.problem, w.material, w.orders, w.quad)
    assert plan.schedule()[0] == 0
    nodes = torch.from_numpy(w.nodes).cuda()
    mat = torch.from_numpy(w.mat).cuda()
    plan.set_schedule(1, 1)
    a, sa = plan.execute(nodes, mat)
    plan.set_schedule(0)
    b, sb = plan.execute(nodes, mat)
    plan.set_schedule(1, 3)
    c, _ = plan.execute(nodes, mat)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c) and torch.equal(sa, sb)
    with pytest.raises(env["p2s"].P2SError):
        env["ctx"].plan(1, 1, [4], [[4, 4, 4]]).set_schedule(1, 1)


def test_autotune_and_cache(env, tmp_path):
    torch, W = env["torch"], env["W"]
    w = W.make("scalar_mixed", E=200)
    plan = env["ctx"].plan(w.problem, w.material, w.orders, w.quad)
    nodes = torch.from_numpy(w.nodes).cuda()
    mat = torch.from_numpy(w.mat).cuda()
    out = torch.empty(int(plan.offsets[-1]), dtype=torch.float64, device="cuda")
    st = torch.empty(w.E, dtype=torch.int32, device="cuda")
    cache = str(tmp_path / "tune.json")
    ms = plan.autotune(nodes, mat, out, st, cache)
    assert ms > 0
    choice = plan.schedule()
    import json
    entries = json.load(open(cache))
    assert len(entries) == 1
    plan2 = env["ctx"].plan(w.problem, w.material, w.orders, w.quad)
    ms2 = plan2.autotune(nodes, mat, out, st, cache)
    assert plan2.schedule() == choice and abs(ms2 - ms) <= 1e-12 * ms
    ref, roff, _ = env["oracle"].fill(w.problem, w.material, w.nodes[:3], w.mat[:3], w.orders[:3], w.quad[:3])
    plan2.execute(nodes, mat, out, st)
    torch.cuda.synchronize()
    g = out[:int(roff[-1])].cpu().numpy()
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name,E,mode", [("scalar_mixed", 150, 0), ("scalar_mixed", 150, 1), ("vector_n6", 40, 0)])
def test_graph_replay(env, name, E, mode):
    """Captured execution replayed several times, with eager work and
    synchronizations between replays; every replay equals the eager fill
    (mode 1: the persistent launch, whose work counter is reset inside the
    graph)."""
    torch, W = env["torch"], env["W"]
    w = W.make(name, E=E)
    plan = env["ctx"].plan(w.problem, w.material, w.orders, w.quad)
    plan.set_schedule(mode, 1)
    nodes = torch.from_numpy(w.nodes).cuda()
    mat = torch.from_numpy(w.mat).cuda()
    ref, rst = plan.execute(nodes, mat)
    torch.cuda.synchronize()
    out = torch.empty_like(ref)
    st = torch.empty_like(rst)
    s = torch.cuda.Stream()
    plan.capture(nodes, mat, out, st, s)
    for k in range(4):
        out.fill_(float("nan"))
        st.fill_(-1)
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        plan.replay(s)
        s.synchronize()
        assert torch.equal(out, ref), k
        assert torch.equal(st, rst), k
        float(junk)


@pytest.mark.parametrize("problem,N,Q", [(0, 4, (8, 8, 8)), (0, 5, (6, 7, 8)), (1, 3, (5, 5, 5)),
                                         (1, 4, (6, 5, 7)), (1, 6, (12, 12, 12))])
def test_direct_quadrature_method(env, problem, N, Q):
    """The GPU direct-quadrature baseline (eq. (2) without eq. (3))."""
    w = make_small(env, problem, N, 2, Q, seed=300 + N)
    check_against_oracle(env, w, method=1)


def test_fill_element_matrices_one_shot(env):
    """p2s_fill_element_matrices through the C ABI: all 64 elements of the
    scalar N=4 workload and a subset of the vector N=6 workload against the
    oracle; a repeated call of the same shape (cached plan) gives the same
    bits; nine shapes in turn (one eviction) stay correct."""
    torch, W, ctx = env["torch"], env["W"], env["ctx"]
    for w in (W.make("scalar_n4"), W.subset(W.make("vector_n6", E=16), np.arange(8))):
        nodes = torch.from_numpy(w.nodes).cuda()
        mat = torch.from_numpy(w.mat).cuda()
        out, st = ctx.fill_element_matrices(w.problem, w.material, nodes, mat, w.orders, w.quad)
        out2, st2 = ctx.fill_element_matrices(w.problem, w.material, nodes, mat, w.orders, w.quad)
        torch.cuda.synchronize()
        assert torch.equal(out, out2) and torch.equal(st, st2)
        ref, roff, rst = env["oracle"].fill(w.problem, w.material, w.nodes, w.mat, w.orders, w.quad)
        assert np.array_equal(st.cpu().numpy(), rst.astype(np.int32))
        errs = rel_errors(out.cpu().numpy(), ref, roff)
        print("one-shot", w.name, "max rel err %.3e" % errs.max(), flush=True)
        assert errs.max() <= TOL
    base = W.make("scalar_n4")
    ref, roff, _ = env["oracle"].fill(base.problem, base.material, base.nodes[:9], base.mat[:9],
                                      base.orders[:9], base.quad[:9])
    for E in range(1, 10):
        sub = W.subset(base, np.arange(E))
        out, _ = ctx.fill_element_matrices(sub.problem, sub.material, torch.from_numpy(sub.nodes).cuda(),
                                           torch.from_numpy(sub.mat).cuda(), sub.orders, sub.quad)
        torch.cuda.synchronize()
        errs = rel_errors(out.cpu().numpy(), ref[:int(roff[E])], roff[:E + 1])
        assert errs.max() <= TOL, E


def test_scalar_mixed_full_size_autotuned(env):
    """The 20000-element mixed-order workload (N ~ U{2..8}, Q = 2N) under
    the schedule the autotuner picks: one sampled element per order class
    against the oracle, symmetry of those blocks, status clean."""
    torch, W = env["torch"], env["W"]
    w = W.make("scalar_mixed")
    plan = env["ctx"].plan(w.problem, w.material, w.orders, w.quad)
    nodes = torch.from_numpy(w.nodes).cuda()
    mat = torch.from_numpy(w.mat).cuda()
    out = torch.empty(int(plan.offsets[-1]), dtype=torch.float64, device="cuda")
    st = torch.empty(w.E, dtype=torch.int32, device="cuda")
    plan.autotune(nodes, mat, out, st)
    print("schedule", plan.schedule(), flush=True)
    out.fill_(float("nan"))
    plan.execute(nodes, mat, out, st)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    assert not bool(torch.isnan(out).any())
    rng = np.random.default_rng(2024)
    pick = sorted(int(rng.choice(np.nonzero(w.orders == N)[0])) for N in range(2, 9))
    sub = W.subset(w, pick)
    ref, roff, _ = env["oracle"].fill(sub.problem, sub.material, sub.nodes, sub.mat, sub.orders, sub.quad)
    off = plan.offsets
    for i, e in enumerate(pick):
        x = out[int(off[e]):int(off[e + 1])].cpu().numpy()
        y = ref[roff[i]:roff[i + 1]]
        n = int(round(len(y) ** 0.5))
        err = np.linalg.norm(x - y) / np.linalg.norm(y)
        print("element", e, "N", int(w.orders[e]), "rel err %.3e" % err, flush=True)
        assert err <= TOL
        X = x.reshape(n, n)
        assert np.abs(X - X.T).max() <= 1e-13 * np.abs(X).max()


def test_vector_n8_full_size_sampled(env):
    """The 8192-element vector N=8 workload (1344 dofs, 16^3 points), FP64:
    first, middle and last element against the oracle, symmetry of every
    element matrix, and bitwise repeatability (per-element integer
    checksums of the bits, so that one output buffer suffices)."""
    torch, W = env["torch"], env["W"]
    w = W.make("vector_n8")
    plan = env["ctx"].plan(w.problem, w.material, w.orders, w.quad)
    nodes = torch.from_numpy(w.nodes).cuda()
    mat = torch.from_numpy(w.mat).cuda()
    nd = 1344
    out = torch.empty(w.E * nd * nd, dtype=torch.float64, device="cuda")
    st = torch.empty(w.E, dtype=torch.int32, device="cuda")
    plan.execute(nodes, mat, out, st)
    torch.cuda.synchronize()
    cks1 = out.view(torch.int64).view(w.E, -1).sum(1)
    plan.execute(nodes, mat, out, st)
    torch.cuda.synchronize()
    cks2 = out.view(torch.int64).view(w.E, -1).sum(1)
    assert torch.equal(cks1, cks2)
    assert int(st.abs().sum()) == 0
    M = out.view(w.E, nd, nd)
    worst = 0.0
    for c in range(0, w.E, 128):
        blk = M[c:c + 128]
        asym = (blk - blk.transpose(1, 2)).abs().amax(dim=(1, 2)) / blk.abs().amax(dim=(1, 2))
        worst = max(worst, float(asym.max()))
    print("max asymmetry %.3e" % worst, flush=True)
    assert worst <= 1e-13
    pick = [0, w.E // 2, w.E - 1]
    sub = W.subset(w, pick)
    ref, roff, _ = env["oracle"].fill(sub.problem, sub.material, sub.nodes, sub.mat, sub.orders, sub.quad)
    for i, e in enumerate(pick):
        x = M[e].cpu().numpy().reshape(-1)
        y = ref[roff[i]:roff[i + 1]]
        err = np.linalg.norm(x - y) / np.linalg.norm(y)
        print("element", e, "rel err %.3e" % err, flush=True)
        assert err <= TOL


def test_nonfinite_status(env):
    """A sampled coupling field holding a NaN or an infinity at one point
    makes that element's matrix non-finite: its status carries
    P2S_STATUS_NONFINITE, the other elements stay clean."""
    torch, W, p2s = env["torch"], env["W"], env["p2s"]
    rng = np.random.default_rng(17)
    for problem, F in ((0, 7), (1, 12)):
        N, Q, E = 4, (6, 5, 7), 4
        a = rng.standard_normal((E, F, int(np.prod(Q))))
        a[1, F - 1, 17] = float("nan")
        a[3, 0, 3] = float("inf")
        w = W.Workload(name="nonfinite", problem=problem, material=W.ALPHA_SAMPLED, E=E,
                       nodes=np.zeros((E, 27, 3)), mat=a.reshape(E, -1),
                       orders=np.full(E, N, np.int32), quad=np.tile(np.array(Q, np.int32), (E, 1)))
        out, off, st, _ = gpu_fill(env, w)
        assert st[0] == 0 and st[2] == 0
        assert st[1] & p2s.STATUS_NONFINITE and st[3] & p2s.STATUS_NONFINITE


@pytest.mark.parametrize("problem,N,E", [(0, 2, 3), (0, 3, 3), (0, 5, 2), (0, 7, 1), (0, 8, 1),
                                         (1, 2, 2), (1, 3, 2), (1, 4, 2), (1, 5, 1), (1, 7, 1), (1, 8, 1)])
def test_direct_sf_orders(env, problem, N, E):
    """Sum-factorized direct quadrature (rules of 2N points per axis)
    against the oracle, every order of both problems."""
    w = make_small(env, problem, N, E, (2 * N, 2 * N, 2 * N), seed=500 + 10 * problem + N)
    check_against_oracle(env, w, method=2)


def test_direct_sf_workloads(env):
    """Sum-factorized direct quadrature on the scalar N=4 workload (all 64
    elements, 8^3 points) and a subset of the vector N=6 workload (12^3
    points), against the oracle; and on mixed orders (Q = 2N) with the
    stiffness and mass weights changed."""
    W = env["W"]
    check_against_oracle(env, W.make("scalar_n4"), method=2)
    check_against_oracle(env, W.subset(W.make("vector_n6", E=16), np.arange(5)), method=2)
    w = W.make("scalar_mixed", E=200)
    idx = []
    for N in range(2, 9):
        idx += list(np.nonzero(w["orders"] == N)[0][:1])
    check_against_oracle(env, W.subset(w, np.array(sorted(idx))), sK=0.7, sM=-1.3, method=2)


def test_direct_sf_rule_restriction(env):
    p2s, ctx = env["p2s"], env["ctx"]
    with pytest.raises(p2s.P2SError, match="2N Gauss points"):
        ctx.plan(0, 0, [4], [[8, 8, 7]], method=p2s.METHOD_DIRECT_SF)
    with pytest.raises(p2s.P2SError, match="FP64"):
        ctx.plan(1, 1, [4], [[8, 8, 8]], method=p2s.METHOD_DIRECT_SF, precision=p2s.SPLIT_FP32)


@pytest.mark.parametrize("name,E", [("vector_n6", 40), ("scalar_mixed", 150), ("scalar_n4", 64)])
def test_packed_upper_output(env, name, E):
    """Packed symmetric output (upper triangle, row by row): every packed
    entry equals the dense fill's entry bit for bit (the same kernels write
    both; the packed form skips the mirrored half)."""
    torch, W, p2s = env["torch"], env["W"], env["p2s"]
    w = W.make(name, E=E)
    nodes, mat = torch.from_numpy(w.nodes).cuda(), torch.from_numpy(w.mat).cuda()
    dense_plan = env["ctx"].plan(w.problem, w.material, w.orders, w.quad)
    pk_plan = env["ctx"].plan(w.problem, w.material, w.orders, w.quad, output=p2s.OUTPUT_PACKED_UPPER)
    dense, sd = dense_plan.execute(nodes, mat)
    packed = torch.full((int(pk_plan.offsets[-1]),), float("nan"), dtype=torch.float64, device="cuda")
    sp = torch.empty_like(sd)
    pk_plan.execute(nodes, mat, packed, sp)
    torch.cuda.synchronize()
    assert torch.equal(sd, sp)
    d, p = dense.cpu().numpy(), packed.cpu().numpy()
    for e in range(w.E):
        n = p2s.num_dofs(w.problem, int(w.orders[e]))
        A = d[dense_plan.offsets[e]:dense_plan.offsets[e + 1]].reshape(n, n)
        iu = np.triu_indices(n)
        got = p[pk_plan.offsets[e]:pk_plan.offsets[e + 1]]
        assert got.size == n * (n + 1) // 2
        assert np.array_equal(got, A[iu]), e
    with pytest.raises(p2s.P2SError):
        pk_plan.set_schedule(1, 1)
    with pytest.raises(p2s.P2SError, match="packed"):
        env["ctx"].plan(w.problem, w.material, w.orders, w.quad, output=p2s.OUTPUT_PACKED_UPPER,
                        method=p2s.METHOD_DIRECT)
