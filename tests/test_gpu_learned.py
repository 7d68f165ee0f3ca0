"""GPU tests of the learned post-smoother: network forward and gradients
against the CPU oracle on the same BF16-rounded inputs, features, the Adam
step's closed form, the training-pair invariant, the stagnation fallback,
and the C4 training and evaluation protocol with its contraction guard."""
import sys

import numpy as np
import pytest

import oracle
from paper_1902_00095_amd import learned, solver, synth
from paper_1902_00095_amd import tpsolve as tps

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _init():
    import torch
    assert torch.cuda.is_available()
    tps.init(0)
    yield


def bf16(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def np_(t):
    return t.detach().cpu().numpy()


def dev(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


def _case(seed=0, dims=(10, 9, 8)):
    g = synth.Grid(*dims, 1, 1, 1)
    rng = np.random.default_rng(seed)
    th = learned.init_params(seed)
    th[3456:3472] = rng.standard_normal(16).astype(np.float32) * 0.1
    th[3472:3904] *= 10
    th = bf16(th)
    f = bf16(rng.standard_normal((8, g.n)).astype(np.float32))
    return g, th, f


# one partial tile; several tiles with ragged ends in x, y and z; more tiles (768)
# than the gradient kernel has workgroups, so that workgroups visit several
DIMS = [(10, 9, 8), (37, 11, 9), (40, 64, 64)]


@pytest.mark.parametrize("dims", DIMS)
def test_forward_matches_oracle(dims):
    say("cnn forward", dims)
    g, th, f = _case(0, dims)
    net = tps.Net(th)
    out = net.forward(g, dev(f.reshape(-1))).cpu().numpy()
    ref, _ = oracle.cnn_forward(g, th.astype(np.float64), f.astype(np.float64))
    assert np.abs(out - ref).max() <= 1e-4 * np.abs(ref).max()


@pytest.mark.parametrize("dims", DIMS)
def test_gradient_matches_oracle(dims):
    say("cnn gradient", dims)
    import torch
    g, th, f = _case(1, dims)
    y = np.random.default_rng(5).standard_normal(g.n).astype(np.float32)
    net = tps.Net(th)
    grad = torch.zeros(tps.CNN_NPARAM, dtype=torch.float32, device="cuda")
    loss = net.loss_grad(g, dev(f.reshape(-1)), dev(y), grad)
    lo, go = oracle.cnn_backward(g, th.astype(np.float64), f.astype(np.float64), y.astype(np.float64))
    assert abs(loss - lo) <= 1e-4 * lo
    gg = grad.cpu().numpy()
    for a, b in ((0, 3456), (3456, 3472), (3472, 3904), (3904, 3905)):
        assert np.abs(gg[a:b] - go[a:b]).max() <= 1e-3 * np.abs(go[a:b]).max(), (a, b)


def test_adam_first_step_closed_form():
    """From zero moments the bias-corrected first step is -lr g / (|g| + eps)."""
    import torch
    g, th, f = _case(2)
    y = np.random.default_rng(6).standard_normal(g.n).astype(np.float32)
    net = tps.Net(th)
    grad = torch.zeros(tps.CNN_NPARAM, dtype=torch.float32, device="cuda")
    net.loss_grad(g, dev(f.reshape(-1)), dev(y), grad)
    net.adam_step(1e-3)
    new = net.params()
    gr = grad.cpu().numpy().astype(np.float64)
    expect = th - 1e-3 * gr / (np.abs(gr) + 1e-8)
    assert np.abs(new - expect).max() <= 2e-6


def test_features_match_oracle():
    say("features")
    p = synth.make_problem("W2", grid=synth.Grid(12, 10, 8, 1, 1, 1))
    d = solver.to_device(p)
    J, G = solver.assemble(p, d)
    a_S = learned.schur_hierarchy(J, coarse_max=64)   # keep the tiny grid multi-level
    net = tps.Net(learned.init_params())
    a_S.attach(net, p.grid)
    r = synth.random_rhs(4, p.grid.n) * 1e3
    f, s = a_S.features(dev(r))
    Jo = oracle.jacobian(p)
    fo, so = oracle.cnn_features(p.grid, Jo.rowptr, Jo.col, Jo.S, r)
    assert abs(s - so) <= 1e-6 * so
    np.testing.assert_allclose(f.cpu().numpy().reshape(8, -1), fo, rtol=2e-6, atol=1e-6)


@pytest.mark.parametrize("storage,dims", [(0, (24, 24, 24)), (1, (24, 24, 24)), (0, (19, 13, 11))])
def test_smoother_in_vcycle_is_state_plus_scaled_forward(storage, dims):
    """The learned post-smoother inside the V-cycle (one fused kernel staging
    the packed static channels and the unscaled residual plane) equals its
    definition assembled from separately tested pieces: the cycle's state
    before post-smoothing x_pre = y - e (from the pair of b = S y), the
    features of r = b - S x_pre with their scale s, the forward pass checked
    against the oracle, and x_post = x_pre + s out.  Grids with full and
    ragged 8 x 8 x 8 tiles; FP64 and FP32 hierarchies."""
    import scipy.sparse as sp
    import torch
    say("smoother in vcycle", storage, dims)
    p = synth.make_problem("W4", seed=1003, grid=synth.Grid(*dims, 1, 1, 1))
    d = solver.to_device(p)
    J, G = solver.assemble(p, d)
    a_S = learned.schur_hierarchy(J, storage=storage, coarse_max=64)
    net = tps.Net(learned.init_params(11) * 2)
    a_S.attach(net, p.grid)
    y = torch.as_tensor(synth.random_rhs(6, p.grid.n), device="cuda")
    r, e = a_S.presmoothed_pair(y)
    x_pre = y - e
    f, sc = a_S.features(r)
    out = net.forward(p.grid, f)
    expect = (x_pre + sc * out.double()).cpu().numpy()
    S = sp.csr_matrix((np_(J.S), np_(J.col), np_(J.rowptr)), shape=(p.grid.n, p.grid.n))
    b = torch.as_tensor(S @ np_(y), device="cuda")
    got = np_(a_S.vcycle(b))
    tol = 1e-6 if storage == 0 else 1e-4
    err = np.abs(got - expect).max() / np.abs(expect).max()
    say(f"  rel err {err:.2e}")
    assert err <= tol
    a_S.attach(None, None)
    net.close()
    a_S.close()


def test_pair_invariant():
    """r = S e exactly up to rounding (r = S y - S x, e = y - x)."""
    import torch
    say("pair")
    p = synth.make_problem("W4", seed=1000, grid=synth.Grid(16, 16, 16, 1, 1, 1))
    d = solver.to_device(p)
    J, G = solver.assemble(p, d)
    a_S = learned.schur_hierarchy(J, coarse_max=64)   # keep the tiny grid multi-level
    y = torch.randn(p.grid.n, dtype=torch.float64, device="cuda")
    r, e = a_S.presmoothed_pair(y)
    Jo = oracle.jacobian(p)
    Se = oracle.spmv(Jo.rowptr, Jo.col, J.S.cpu().numpy(), e.cpu().numpy())
    rn = r.cpu().numpy()
    assert np.abs(Se - rn).max() <= 1e-9 * np.abs(rn).max()
    assert np.linalg.norm(e.cpu().numpy()) < np.linalg.norm(y.cpu().numpy())


def test_untrained_and_adversarial_networks_fall_back():
    say("fallback")
    p = synth.make_problem("W4", seed=4001, grid=synth.Grid(24, 24, 24, 1, 1, 1))
    good = tps.Net(learned.init_params())
    res = learned.compare(good, p)
    say(f"  untrained: plain {res['plain']['iters']} learned {res['learned']['iters']} "
        f"fallback {res['learned']['fallback_iter']}")
    assert res["learned"]["converged"] and res["learned"]["rel_true"] <= 1e-8
    th = learned.init_params(7) * 1e4            # huge corrections: stagnation
    bad = tps.Net(th)
    res = learned.compare(bad, p)
    say(f"  adversarial: learned {res['learned']['iters']} fallback {res['learned']['fallback_iter']}")
    assert res["learned"]["converged"] and res["learned"]["rel_true"] <= 1e-8
    assert res["learned"]["fallback_iter"] >= 0
    with pytest.raises(tps.TpError):
        tps.Net(np.full(tps.CNN_NPARAM, np.nan, dtype=np.float32))


def test_learned_graph_replay_matches_eager():
    """With the learned post-smoother attached, the preconditioner replayed from
    its captured graph gives the same iterates, bit for bit, as eager launches;
    after a new network is attached the graph is captured again (the results
    follow the new network), and after detaching the plain graph is used."""
    import torch
    say("learned graph replay")
    p = synth.make_problem("W4", seed=4001, grid=synth.Grid(24, 24, 24, 1, 1, 1))
    d = solver.to_device(p)
    J, G = solver.assemble(p, d)
    cfg = solver.SolveConfig()
    a_pp, a_S, M = solver.setup(J, cfg)
    nets = [tps.Net(learned.init_params(3)), tps.Net(learned.init_params(5) * 3)]
    scratch = torch.ones(128, 128, device="cuda", dtype=torch.float64)
    seen = []
    for net in nets + [None]:
        a_S.attach(net, p.grid if net is not None else None)
        runs = []
        for graph in (False, True, True, False, True):
            scratch = scratch @ scratch.t() / 128.0     # unrelated device work between solves
            torch.cuda.synchronize()
            x, st = tps.fgmres_solve(J, M, -G, rtol=1e-8, history=True, graph=graph)
            torch.cuda.synchronize()
            runs.append((np_(x), st))
        x0, s0 = runs[0]
        say(f"  its {s0['iters']} fallback {s0['fallback_iter']} rel {s0['rel_true']:.2e}")
        assert s0["converged"] and s0["rel_true"] <= 1e-8
        for x, st in runs[1:]:
            assert st["iters"] == s0["iters"] and st["fallback_iter"] == s0["fallback_iter"]
            assert np.array_equal(st["history"], s0["history"])
            assert np.array_equal(x, x0)
        seen.append(s0["history"])
    # each attachment changes the iterates (a stale graph would repeat them)
    assert not np.array_equal(seen[0][:3], seen[1][:3])
    assert not np.array_equal(seen[1][:3], seen[2][:3])
    for net in nets:
        net.close()
    M.close(); a_pp.close(); a_S.close()


@pytest.mark.parametrize("ew", [0.0, 0.5])
def test_operator_loss_gradient_matches_oracle(ew):
    """Gradient of L = mean((D^{-1} S (out - t))^2) + ew mean((out - t)^2) on
    the GPU against central differences of the same loss built from the
    oracle's FP64 forward pass and the oracle Jacobian, at the BF16-rounded
    weights."""
    import scipy.sparse as sp
    say("operator loss gradient", ew)
    p = synth.make_problem("W4", seed=1001, grid=synth.Grid(10, 9, 8, 1, 1, 1))
    d = solver.to_device(p)
    J, G = solver.assemble(p, d)
    g, th, f = _case(4, (10, 9, 8))
    th = bf16(th)
    net = tps.Net(th)
    a_S = learned.schur_hierarchy(J, coarse_max=64)   # keep the tiny grid multi-level
    a_S.attach(net, p.grid)
    t = np.random.default_rng(8).standard_normal(g.n).astype(np.float32)
    loss = a_S.op_loss_grad(dev(f.reshape(-1)), dev(t), ew)
    gg = net.grad().astype(np.float64)
    Jo = oracle.jacobian(p)
    A = sp.csr_matrix((Jo.S, Jo.col, Jo.rowptr))
    Dinv = 1.0 / np.abs(A).sum(axis=1).A1
    th64 = th.astype(np.float64)
    f64 = f.astype(np.float64)

    def L(theta):
        out, _ = oracle.cnn_forward(g, theta, f64)
        e = out - t.astype(np.float64)
        v = Dinv * (A @ e)
        return float(np.mean(v * v) + ew * np.mean(e * e))

    assert abs(loss - L(th64)) <= 1e-4 * L(th64)
    scale = np.abs(gg).max()
    for k in list(range(0, 3456, 331)) + [3460, 3500, 3700, 3904]:
        h = 1e-3 * max(1.0, abs(th64[k]))
        tp_, tm = th64.copy(), th64.copy()
        tp_[k] += h
        tm[k] -= h
        fd = (L(tp_) - L(tm)) / (2 * h)
        assert abs(fd - gg[k]) <= 2e-3 * scale, (k, fd, gg[k])


def test_c4_training_and_guarded_evaluation():
    """The C4 protocol: train on pairs from plain solves of fields 1000-1199
    (24^3), then evaluate at 96^3 on held-out fields 4001 and 4002.

    Training must work and generalise: the loss falls at least fivefold, and
    on held-out pairs at 96^3 the network removes most of the residual it is
    given (operator-norm loss at most 0.2 of what no correction leaves).
    The measured outcome in FGMRES is negative -- the learned
    post-smoother needs more iterations than the Chebyshev post-smoother it
    replaces, at the same cost per iteration -- so what is asserted is the
    guard: with the contraction guard (the plain solve's mean contraction as
    reference) the learned form still reaches true rtol 1e-8, never takes
    more iterations than the unguarded learned form, and stays within 1.6x
    of plain's iterations; when it falls behind the guard has switched it
    off (fallback_iter set).  The iteration counts of every form are printed."""
    import torch
    say("C4 training")
    net, rec = learned.train_c4()
    say(f"  {rec['pairs']} pairs, loss {rec['loss_first']:.3e} -> {rec['loss_last_100_mean']:.3e}")
    assert rec["pairs"] == 600
    assert rec["loss_last_100_mean"] < 0.2 * rec["loss_first"]
    g96 = synth.Grid(96, 96, 96, 1.0, 1.0, 1.0)
    zero = tps.Net(np.zeros(learned.NPARAM, dtype=np.float32))
    held = learned.plain_solve_pairs(synth.make_problem("W4", seed=4001, grid=g96), net, arnoldi_steps=2)
    ln = learned.eval_loss(net, held)
    held[0].amg.attach(zero, g96)
    lz = learned.eval_loss(zero, held)
    held[0].amg.attach(None, None)
    held[0].amg.close()
    say(f"  held-out 96^3 pairs: loss {ln:.3e}, no correction {lz:.3e}")
    assert ln < 0.2 * lz
    rows = learned.evaluate_c4(net, seeds=(4001, 4002))
    for r in rows:
        say("  seed", r["seed"], {k: (v["iters"], v["fgmres_ms"], v["fallback_iter"]) for k, v in r.items()
                                  if k != "seed"})
        p, l, gd = r["plain"], r["learned"], r["learned_guarded"]
        for key in ("plain", "learned", "learned_guarded", "no_post"):
            assert r[key]["converged"] and r[key]["rel_true"] <= 1e-8, (key, r[key])
        assert gd["iters"] <= l["iters"]
        assert gd["iters"] <= 1.6 * p["iters"]
        if gd["iters"] > p["iters"]:
            assert gd["fallback_iter"] >= 4
    zero.close()
    net.close()
    torch.cuda.synchronize()
