"""Learned-theta kernels vs the FP64 oracles (features, network, Adam), through the C ABI.

* group features within 1e-4 of the oracle's (from its brute-force moments);
* per-group RMS error kernel against numpy;
* fp32 forward within 1e-5, bf16 forward within 0.01 of the FP64 network;
* gradient within 1e-4 (relative to its largest entry) of the FP64 gradient;
* Adam steps track the FP64 Adam; training lowers the loss;
* the learned path (features -> bf16 network -> per-group walk) equals a walk
  given the same theta array, and the fallback triggers on an impossible target;
* the one-pass inference (matrix-core network, 16 groups per wavefront) equals
  features + bf16 forward, snapped, on every group of a grid whose last
  wavefront holds 8 groups;
* a network's theta floor lifts exactly the groups below it, in the inference
  and in the fused learned walk, and a network trained for the paper's opening
  test and monopole far field runs the walk with those options.
"""
import numpy as np
import pytest

from amr_inputs import maclaurin_spheroid, random_amr
from amr_inputs.mlp_init import glorot_init
from oracle import OracleTree
from oracle import mlp as omlp
from oracle.features import group_features as oracle_features

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1509_07370_amd import binding as B  # noqa: E402
from paper_1509_07370_amd import learned_theta as LT  # noqa: E402
from paper_1509_07370_amd.solver import BarnesHut  # noqa: E402


@pytest.fixture(scope="module")
def amr():
    g = random_amr(21, nbase=2, max_level=3, p_refine=0.3, zero_fraction=0.1)
    bh = BarnesHut(g)
    rho = torch.tensor(g.rho, device="cuda")
    yield g, bh, rho
    bh.close()


def test_features_parity(amr):
    g, bh, rho = amr
    F = LT.group_features(bh, rho).cpu().numpy()
    ref = oracle_features(OracleTree(g), g)
    assert F.shape == ref.shape
    assert np.max(np.abs(F - ref)) <= 1e-4


def test_group_rms_error_kernel(amr):
    g, bh, rho = amr
    rng = np.random.default_rng(0)
    ref = torch.tensor(-rng.uniform(1, 2, g.rho.shape), device="cuda")
    phi = ref * torch.tensor(1 + rng.normal(scale=1e-3, size=g.rho.shape), device="cuda")
    rms = torch.empty(bh.info["n_groups"], dtype=torch.float32, device="cuda")
    B.bh_group_rms_error(bh.ctx, bh.grid, phi, ref, rms)
    r = ((phi - ref) / ref).cpu().numpy()
    # canonical group g = leaf*8 + Morton run of 64 cells
    want = np.empty(g.nleaf * 8)
    for sub in range(8):
        m = sub * 64 + np.arange(64)
        i = sum(((m >> (3 * p)) & 1) << p for p in range(3))
        j = sum(((m >> (3 * p + 1)) & 1) << p for p in range(3))
        k = sum(((m >> (3 * p + 2)) & 1) << p for p in range(3))
        want[np.arange(g.nleaf) * 8 + sub] = np.sqrt((r[:, k, j, i] ** 2).mean(1))
    assert np.allclose(rms.cpu().numpy(), want, rtol=1e-5, atol=0)


def _net_data(n=3000, seed=1):
    rng = np.random.default_rng(seed)
    X = (rng.normal(size=(n, 12)) * 2 + 0.5).astype(np.float32)
    y = rng.uniform(0.2, 1.0, n).astype(np.float32)
    mean = X.mean(0).astype(np.float32)
    scale = (1 / X.std(0)).astype(np.float32)
    return X, y, mean, scale


def test_forward_fp32_and_bf16_parity():
    ctx = B.bh_ctx_create(0)
    X, y, mean, scale = _net_data()
    p = (glorot_init(5) * 3).astype(np.float32)
    net = B.bh_mlp_create(ctx, p, mean, scale)
    fx = torch.tensor(X, device="cuda")
    out = torch.empty(len(X), dtype=torch.float32, device="cuda")
    ref, _ = omlp.forward(p.astype(np.float64), X.astype(np.float64), mean.astype(np.float64),
                          scale.astype(np.float64))
    B.bh_mlp_forward(ctx, net, fx, out, bf16=False)
    ref_shift = np.clip(ref - 0.1, 0.05, 1.0)
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-5
    B.bh_mlp_forward(ctx, net, fx, out, bf16=True)
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 0.01
    B.bh_mlp_forward(ctx, net, fx, out, bf16=False, shift=0.1)
    assert np.max(np.abs(out.cpu().numpy() - ref_shift)) <= 1e-5
    B.bh_mlp_destroy(net)
    B.bh_ctx_destroy(ctx)


def test_gradient_parity():
    ctx = B.bh_ctx_create(0)
    X, y, mean, scale = _net_data(2500, seed=3)
    fx, fy = torch.tensor(X, device="cuda"), torch.tensor(y, device="cuda")
    grad = torch.empty(B.MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    args64 = (X.astype(np.float64), y.astype(np.float64), mean.astype(np.float64), scale.astype(np.float64))
    for seed, gain in ((6, 2.0), (7, 0.5), (8, 4.0)):
        p = (glorot_init(seed) * gain).astype(np.float32)
        net = B.bh_mlp_create(ctx, p, mean, scale)
        B.bh_mlp_grad(ctx, net, fx, fy, grad, loss)
        g_ref = omlp.grad(p.astype(np.float64), *args64)
        L = omlp.loss(p.astype(np.float64), *args64)
        assert np.max(np.abs(grad.cpu().numpy() - g_ref)) <= 1e-4 * np.abs(g_ref).max()
        assert abs(float(loss[0]) - L) <= 1e-5 * L
        B.bh_mlp_destroy(net)
    B.bh_ctx_destroy(ctx)


def test_adam_parity():
    """Adam kernel on seeded gradients (inputs drawn by the test, not by the GPU)."""
    ctx = B.bh_ctx_create(0)
    _, _, mean, scale = _net_data(10)
    p = glorot_init(9).astype(np.float32)
    net = B.bh_mlp_create(ctx, p, mean, scale)
    rng = np.random.default_rng(11)
    pq = p.astype(np.float64)
    m = np.zeros_like(pq)
    v = np.zeros_like(pq)
    for step in range(1, 6):
        g = (rng.normal(size=B.MLP_PARAMS) * 10.0 ** rng.uniform(-3, 0, B.MLP_PARAMS)).astype(np.float32)
        B.bh_mlp_adam_step(ctx, net, torch.tensor(g, device="cuda"), 1e-3, 0.9, 0.999, 1e-8)
        pq, m, v = omlp.adam_step(pq, g.astype(np.float64), m, v, step, 1e-3)
        assert np.max(np.abs(B.bh_mlp_get_params(ctx, net) - pq)) <= 1e-6
    B.bh_mlp_destroy(net)
    B.bh_ctx_destroy(ctx)


def test_training_lowers_the_loss():
    ctx = B.bh_ctx_create(0)
    rng = np.random.default_rng(8)
    X = rng.normal(size=(8192, 12)).astype(np.float32)
    y = (0.6 + 0.3 * np.tanh(X[:, 1] - 0.5 * X[:, 4])).astype(np.float32)
    net = LT.ThetaNet.fresh(ctx, X, glorot_init(42).astype(np.float32))
    hist = net.train(torch.tensor(X, device="cuda"), torch.tensor(y, device="cuda"), epochs=40, batch=1024, lr=3e-3)
    assert hist[-1] < 0.1 * hist[0]
    net.close()
    B.bh_ctx_destroy(ctx)


def test_learned_path_equals_walk_with_same_thetas_and_fallback():
    g = maclaurin_spheroid(max_level=1)
    bh = BarnesHut(g)
    rho = torch.tensor(g.rho, device="cuda")
    ng = bh.info["n_groups"]
    feat = torch.empty((ng, 12), dtype=torch.float32, device="cuda")
    theta = torch.empty(ng, dtype=torch.float32, device="cuda")
    phi = torch.empty_like(rho)
    X = LT.group_features(bh, rho).cpu().numpy()
    net = LT.ThetaNet.fresh(bh.ctx, X, glorot_init(42).astype(np.float32))
    LT.solve_learned(bh, rho, net, phi, feat, theta)
    th = theta.cpu().numpy()
    # the one-pass inference equals features + bf16 forward, snapped up to the 0.05 grid of the labels
    two = torch.empty_like(theta)
    B.bh_group_features(bh.ctx, bh.grid, bh.m, feat)
    B.bh_mlp_forward(bh.ctx, net.h, feat, two, True, net.shift)
    cont = two.cpu().numpy().astype(np.float64)
    k = np.clip(np.ceil((cont - 1e-6 - 0.2) * 20.0), 0, 16)
    snapped = (0.2 + 0.05 * k).astype(np.float32)
    # features are the same up to rounding (fp64 kernel vs fp32 logs): a prediction within 5e-3 of a
    # grid boundary may snap to the neighbouring value
    near_edge = np.abs((cont - 0.2) * 20.0 - np.round((cont - 0.2) * 20.0)) < 0.1
    assert np.all((th == snapped) | near_edge)
    assert np.all(np.isin(np.round(th * 20).astype(int), np.arange(4, 21)))
    assert np.all(th >= 0.2) and np.all(th <= 1.0)
    ref = torch.empty_like(rho)
    bh.walk(0.5, theta, B.BH_FP32)
    bh.potential(ref, 1.0, B.BH_FP32)
    assert torch.equal(phi, ref)
    _, info = LT.solve_with_fallback(bh, rho, net, phi, feat, theta, target=1e-12)
    assert info["mode"] == "fallback"
    _, info = LT.solve_with_fallback(bh, rho, net, phi, feat, theta, target=1.0)
    assert info["mode"] == "learned"
    net.close()
    bh.close()


@pytest.mark.parametrize("seed,scale", [(7, 3.0), (11, 1.0)])
def test_theta_infer_equals_features_and_forward_on_a_ragged_grid(seed, scale):
    g = random_amr(23, nbase=2, max_level=3, p_refine=0.3, zero_fraction=0.1)
    bh = BarnesHut(g)
    rho = torch.tensor(g.rho, device="cuda")
    ng = bh.info["n_groups"]
    assert ng % 16 == 8  # the last wavefront of the inference kernel holds 8 groups
    X = LT.group_features(bh, rho).cpu().numpy()
    net = LT.ThetaNet.fresh(bh.ctx, X, (glorot_init(seed) * scale).astype(np.float32))
    for shift in (0.0, 0.1):
        th = torch.full((ng,), float("nan"), device="cuda")
        feat = torch.empty((ng, 12), dtype=torch.float32, device="cuda")
        cont = torch.empty(ng, dtype=torch.float32, device="cuda")
        bh.build_moments(rho)
        B.bh_theta_infer(bh.ctx, bh.grid, bh.m, net.h, th, shift)
        B.bh_group_features(bh.ctx, bh.grid, bh.m, feat)
        B.bh_mlp_forward(bh.ctx, net.h, feat, cont, True, shift)
        bh.check()
        t = th.cpu().numpy()
        c = cont.cpu().numpy().astype(np.float64)
        k = np.clip(np.ceil((c - 1e-6 - 0.2) * 20.0), 0, 16)
        snapped = (0.2 + 0.05 * k).astype(np.float32)
        # the two sides round their sums differently (matrix-core products vs fused multiply-adds, fp64-argument
        # features vs fp32 logs): a prediction within 5e-3 of a grid boundary may snap to the neighbour
        near_edge = np.abs((c - 0.2) * 20.0 - np.round((c - 0.2) * 20.0)) < 0.1
        assert np.all(np.isfinite(t))
        assert np.all((t == snapped) | near_edge)
        assert np.mean(t == snapped) > 0.95 and np.unique(t).size > 3
    net.close()
    bh.close()


@pytest.mark.parametrize("precision", [B.BH_FP32, B.BH_FP64])
def test_one_launch_learned_walk_equals_two_launches(precision):
    """bh_learned_walk_potential (inference, then the walk with those thetas):
    the same thetas as bh_theta_infer and the same potentials as
    bh_walk_potential given them, bit for bit."""
    g = random_amr(23, nbase=2, max_level=3, p_refine=0.3, zero_fraction=0.1)
    bh = BarnesHut(g)
    rho = torch.tensor(g.rho, device="cuda")
    ng = bh.info["n_groups"]
    X = LT.group_features(bh, rho).cpu().numpy()
    net = LT.ThetaNet.fresh(bh.ctx, X, (glorot_init(7) * 3).astype(np.float32))
    for shift in (0.0, 0.1):
        net.meta["theta_shift"] = shift
        th1, th2 = (torch.full((ng,), float("nan"), device="cuda") for _ in range(2))
        p1, p2 = torch.empty_like(rho), torch.empty_like(rho)
        c1, c2 = (torch.zeros((ng, 2), dtype=torch.int32, device="cuda") for _ in range(2))
        bh.build_moments(rho)
        B.bh_learned_walk_potential(bh.ctx, bh.grid, bh.m, net.h, net.shift, precision, 1.0, p1, th1, c1)
        B.bh_theta_infer(bh.ctx, bh.grid, bh.m, net.h, th2, net.shift)
        B.bh_walk_potential(bh.ctx, bh.grid, bh.m, 0.5, th2, precision, 1.0, p2, c2)
        bh.check()
        assert torch.equal(th1, th2)
        assert float(th1.min()) >= 0.05 and float(th1.max()) <= 1.0 and float(th1.std()) > 0
        assert torch.equal(p1, p2) and torch.equal(c1, c2)
    net.close()
    bh.close()


@pytest.mark.parametrize("which", ["glorot", "shipped_1e-4"])
def test_theta_infer_equals_the_oracle_features_and_bf16_network(which):
    """bh_theta_infer (features from node rows and the bf16 network on the matrix cores, snapped) against
    the oracle: its fp64 features from brute-force node moments, the bf16-rounded fp64 network, the same
    snap.  Every group of a MacLaurin grid and of a ragged random grid; the two sides round differently
    (fp32 logs and fp32 accumulation against fp64), so a prediction within 5e-3 of a grid boundary may
    take the neighbouring value."""
    import os
    for g in (maclaurin_spheroid(max_level=1), random_amr(23, nbase=2, max_level=3, p_refine=0.3,
                                                           zero_fraction=0.1)):
        bh = BarnesHut(g)
        rho = torch.tensor(g.rho, device="cuda")
        ng = bh.info["n_groups"]
        F = oracle_features(OracleTree(g), g)
        if which == "glorot":
            net = LT.ThetaNet.fresh(bh.ctx, F.astype(np.float32), (glorot_init(7) * 3).astype(np.float32))
        else:
            net = LT.ThetaNet.load(bh.ctx, os.path.join(LT.DATA_DIR, "theta_mlp_1e-4.npz"))
        p = net.params().astype(np.float64)
        for shift in (0.0, 0.1):
            th = torch.full((ng,), float("nan"), device="cuda")
            bh.build_moments(rho)
            B.bh_theta_infer(bh.ctx, bh.grid, bh.m, net.h, th, shift)
            bh.check()
            t = th.cpu().numpy().astype(np.float64)
            cont = omlp.forward_bf16(p, F, net.mean.astype(np.float64), net.scale.astype(np.float64)) - shift
            # the shipped network carries a floor (its smallest training label, on the grid)
            want = np.maximum(omlp.snap_up(cont), net.floor)
            near_edge = np.abs((cont - 0.2) * 20.0 - np.round((cont - 0.2) * 20.0)) < 0.1
            same = np.abs(t - want) < 1e-6
            print("[theta_infer vs oracle] %s %s shift %.1f: %d groups, %d differ (%d near a grid edge), "
                  "%d distinct thetas" % (which, g.name, shift, ng, int((~same).sum()), int(near_edge.sum()),
                                          np.unique(t).size))
            assert np.all(same | (near_edge & (np.abs(t - want) < 0.05 + 1e-6)))
            assert same.mean() > 0.97
            assert np.unique(t).size > 2
        net.close()
        bh.close()


def test_what_the_shipped_networks_gain():
    """What the trained network gains over the method without it, on a held-out MacLaurin core (e ~ 0.87,
    1.4M cells, fp32):
    * at the headline target 1e-3 the network saturates at the theta <= 1 cap: every group walks at theta 1 and
      the potential is the fixed-theta-1 walk's, bit for bit -- it gains nothing there (the quadrupole and the
      exact group vote already keep theta 1 at RMS ~3e-4);
    * at 1e-4 the learned step, judged by its 1% sampled check with the fixed 0.4 fallback, meets the target on
      the whole grid; its time against the best fixed theta of the grid (the largest meeting the target, from a
      full sweep) is measured and printed -- on these cores it is slower (0.6-0.8x, per-group theta spread costs
      more than it saves because the cost is steeply convex in theta)."""
    import os
    import time
    g = LT.evaluation_grids()[0]
    bh = BarnesHut(g)
    rho = torch.tensor(g.rho, device="cuda")
    ng = bh.info["n_groups"]
    direct = LT.direct_potential(bh, rho)
    phi, ref = torch.empty_like(rho), torch.empty_like(rho)
    theta = torch.empty(ng, dtype=torch.float32, device="cuda")
    feat = torch.empty((ng, 12), dtype=torch.float32, device="cuda")

    def rms(p):
        rel = ((p - direct) / direct).reshape(-1)
        return float(torch.sqrt((rel * rel).mean()))

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    net = LT.ThetaNet.load(bh.ctx, os.path.join(LT.DATA_DIR, "theta_mlp_1e-3.npz"))
    LT.solve_learned(bh, rho, net, phi, feat, theta)
    bh.build_moments(rho)
    B.bh_walk_potential(bh.ctx, bh.grid, bh.m, 1.0, None, B.BH_FP32, 1.0, ref, None)
    assert float(theta.min()) == 1.0 and torch.equal(phi, ref)
    assert rms(phi) <= 1e-3
    net.close()

    net = LT.ThetaNet.load(bh.ctx, os.path.join(LT.DATA_DIR, "theta_mlp_1e-4.npz"))
    out, info = LT.solve_with_fallback(bh, rho, net, phi, feat, theta, 1e-4)
    assert rms(out) <= 1e-4, info
    ms_learned = timed(lambda: LT.solve_learned(bh, rho, net, phi, feat, theta))
    best = None
    for th in LT.THETA_GRID[::-1]:
        bh.build_moments(rho)
        B.bh_walk_potential(bh.ctx, bh.grid, bh.m, float(th), None, B.BH_FP32, 1.0, ref, None)
        if rms(ref) <= 1e-4:
            best = float(th)
            break

    def fixed():
        bh.build_moments(rho)
        B.bh_walk_potential(bh.ctx, bh.grid, bh.m, best, None, B.BH_FP32, 1.0, ref, None)
    ms_fixed = timed(fixed)
    print("[learned gain] target 1e-4: learned %.3f ms (%s), best fixed theta %.2f %.3f ms: x%.3f" % (
        ms_learned, info["mode"], best, ms_fixed, ms_fixed / ms_learned))
    net.close()
    bh.close()


def test_theta_floor_and_walk_options():
    """bh_mlp_set_theta_floor: the inference returns max(theta, floor snapped up to the grid) for every group,
    the fused learned walk writes and walks with the same thetas, out-of-range floors are rejected; a network
    whose metadata names the group-cube opening test and the monopole far field drives bh_walk_potential_ex with
    them."""
    g = maclaurin_spheroid(max_level=1)
    bh = BarnesHut(g)
    rho = torch.tensor(g.rho, device="cuda")
    ng = bh.info["n_groups"]
    X = LT.group_features(bh, rho).cpu().numpy()
    net = LT.ThetaNet.fresh(bh.ctx, X, (glorot_init(7) * 3).astype(np.float32))
    free = torch.empty(ng, dtype=torch.float32, device="cuda")
    bh.build_moments(rho)
    B.bh_theta_infer(bh.ctx, bh.grid, bh.m, net.h, free, 0.1)
    t0 = free.cpu().numpy()
    assert t0.min() < 0.5 < t0.max(), "the test needs predictions on both sides of the floor"
    for floor, want_floor in ((0.5, 0.5), (0.52, 0.55), (0.2, 0.2), (1.0, 1.0)):
        B.bh_mlp_set_theta_floor(bh.ctx, net.h, floor)
        th = torch.empty_like(free)
        B.bh_theta_infer(bh.ctx, bh.grid, bh.m, net.h, th, 0.1)
        assert np.array_equal(th.cpu().numpy(), np.maximum(t0, np.float32(0.2 + 0.05 * round((want_floor - 0.2) * 20))))
    B.bh_mlp_set_theta_floor(bh.ctx, net.h, 0.5)
    phi, ref = torch.empty_like(rho), torch.empty_like(rho)
    used = torch.empty_like(free)
    B.bh_learned_walk_potential(bh.ctx, bh.grid, bh.m, net.h, 0.1, B.BH_FP32, 1.0, phi, used)
    assert float(used.min()) == 0.5 and np.array_equal(used.cpu().numpy(), np.maximum(t0, np.float32(0.5)))
    B.bh_walk_potential(bh.ctx, bh.grid, bh.m, 0.5, used, B.BH_FP32, 1.0, ref, None)
    assert torch.equal(phi, ref)
    for bad in (0.1, 1.5, float("nan")):
        with pytest.raises(B.BHError):
            B.bh_mlp_set_theta_floor(bh.ctx, net.h, bad)
    net.close()
    # the paper's walk options travel with the network
    paper = LT.ThetaNet.fresh(bh.ctx, X, glorot_init(7).astype(np.float32),
                              meta=dict(theta_floor=0.3, mac=B.BH_MAC_GROUP_BOX, order=0, theta_shift=0.05))
    assert paper.walk_options == (B.BH_MAC_GROUP_BOX, 0) and paper.floor == 0.3
    theta = torch.empty_like(free)
    LT.solve_learned(bh, rho, paper, phi, None, theta)
    assert float(theta.min()) >= 0.3
    bh.build_moments(rho)
    B.bh_walk_potential_ex(bh.ctx, bh.grid, bh.m, 0.5, theta, B.BH_FP32, 1.0, ref, None,
                           mac=B.BH_MAC_GROUP_BOX, order=0)
    assert torch.equal(phi, ref)
    B.bh_walk_potential(bh.ctx, bh.grid, bh.m, 0.5, theta, B.BH_FP32, 1.0, ref, None)
    assert not torch.equal(phi, ref)
    paper.close()
    bh.close()
