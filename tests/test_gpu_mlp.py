"""GPU checks of the warm-start network against the FP64 reference (oracle.mlp).

BF16 rounding of intermediate activations is a quantisation: where the GPU's
FP32 value and the reference's value straddle a bfloat16 rounding boundary the
two round differently by one bf16 ulp (2^-8 relative).  Such flips are rare
(~1e-5 of the elements); the gates are therefore a tight median and a max-norm
bound at the bf16 level.
"""
import numpy as np
import pytest

from oracle import mlp as ref

pytestmark = pytest.mark.gpu


def make_net(nfl, seed=3):
    W = nfl.WarmStart(n_classes=3, seed=seed)
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.25, size=ref.NP).astype(np.float32)
    W.set_params(p)
    return W, p


def features(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(B, 16)).astype(np.float32)
    X[:, 8:] = 0.0
    return X


def test_forward_matches_reference(nfl):
    W, p = make_net(nfl)
    for B in (1, 17, 1000):
        X = features(B, B)
        got = W.forward(X).cpu().numpy().astype(np.float64)
        want, _ = ref.forward(p, X, emulate=True)
        err = np.abs(got - want)
        scale = max(1.0, np.abs(want).max())
        assert np.median(err) <= 1e-5 * scale, (B, np.median(err))
        assert err.max() <= 2e-2 * scale, (B, err.max())


def test_gradient_matches_reference(nfl):
    W, p = make_net(nfl, seed=5)
    X = features(777, 9)
    t = np.random.default_rng(2).normal(size=777).astype(np.float32)
    loss, g = W.gradient(X, t)
    Lr, gr = ref.loss_and_grad(p, X, t, emulate=True)
    assert abs(loss - Lr) <= 1e-3 * abs(Lr)
    blocks = {"W1": (0, 1024), "b1": (1024, 1088), "W2": (1088, 5184), "b2": (5184, 5248),
              "W3": (5248, 9344), "b3": (9344, 9408), "W4": (9408, 9472), "b4": (9472, 9473)}
    for name, (a, b) in blocks.items():
        d = np.abs(g[a:b] - gr[a:b])
        nrm = np.abs(gr[a:b]).max()
        assert d.max() <= 2e-2 * nrm, (name, d.max(), nrm)
        assert np.median(d) <= 2e-3 * nrm, (name, np.median(d), nrm)


def test_training_reduces_loss_and_save_load(nfl, tmp_path):
    import torch
    import synth
    v, lab = synth.moons_and_roll(20000, seed=11)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), 0.04, N=32, m=4)
    W = nfl.WarmStart(n_classes=3, seed=1)
    f = synth.ssl_rhs(lab, 1, frac=0.05, seed=4)
    r = P.cg_solve(torch.as_tensor(f, device="cuda"), tau=10.0, tol=1e-8, maxit=300)
    losses = [W.train_step(P, f, r["u"], 1, 4096, s, 3e-3) for s in range(150)]
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:10]), (losses[:3], losses[-3:])
    path = str(tmp_path / "net.bin")
    W.save(path)
    W2 = nfl.WarmStart(n_classes=3, seed=99)
    W2.load(path)
    np.testing.assert_array_equal(W.params(), W2.params())
    u1 = W.predict(P, f, 1).cpu().numpy()
    u2 = W2.predict(P, f, 1).cpu().numpy()
    np.testing.assert_array_equal(u1, u2)


def test_cg_with_learned_warm_start_reaches_same_solution(nfl):
    """CG always runs to tolerance: the warm start changes iterations, not the
    answer."""
    import torch
    import synth
    v, lab = synth.moons_and_roll(30000, seed=12)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), 0.04, N=32, m=4)
    W = nfl.WarmStart(n_classes=3, seed=2)
    fs = [synth.ssl_rhs(lab, c, frac=0.02, seed=20 + c) for c in range(3)]
    sols = [P.cg_solve(torch.as_tensor(f, device="cuda"), tau=10.0, tol=1e-8, maxit=300)["u"] for f in fs]
    for s in range(200):
        c = s % 3
        W.train_step(P, fs[c], sols[c], c, 8192, s, 3e-3)
    f = synth.ssl_rhs(lab, 0, frac=0.02, seed=77)
    fd = torch.as_tensor(f, device="cuda")
    plain = P.cg_solve(fd, tau=10.0, tol=1e-6, maxit=300)
    W.attach(P, 0)
    warm = P.cg_solve(fd, tau=10.0, tol=1e-6, maxit=300, warm=nfl.WARM_MLP)
    assert plain["converged"] and warm["converged"]
    assert warm["relres"] <= 2e-6
    u0 = plain["u"].cpu().numpy()
    u1 = warm["u"].cpu().numpy()
    assert np.abs(u0 - u1).max() <= 2e-5 * np.abs(u0).max()


def test_trained_network_reduces_cg_iterations(nfl):
    """The committed network (trained by paper_1808_04580_amd.train_warmstart on
    clouds 1..100) on a held-out cloud: fewer CG iterations to 1e-6 than u0 = 0,
    same solution."""
    import os
    import torch
    import synth
    path = os.path.join(os.path.dirname(nfl.__file__), "warmstart_moons_roll.bin")
    v, lab = synth.moons_and_roll(1_000_000, seed=100002)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), 0.04, N=64, m=6)
    W = nfl.WarmStart(n_classes=3)
    W.load(path)
    plain, warm = [], []
    for c in range(3):
        f = torch.as_tensor(synth.ssl_rhs(lab, c, frac=0.02, seed=300 + c), device="cuda")
        r0 = P.cg_solve(f, tau=10.0, tol=1e-6, maxit=300)
        W.attach(P, c)
        r1 = P.cg_solve(f, tau=10.0, tol=1e-6, maxit=300, warm=nfl.WARM_MLP)
        assert r0["converged"] and r1["converged"] and r1["relres"] <= 2e-6
        u0, u1 = r0["u"].cpu().numpy(), r1["u"].cpu().numpy()
        assert np.abs(u0 - u1).max() <= 2e-5 * np.abs(u0).max()
        plain.append(r0["iters"])
        warm.append(r1["iters"])
    print("CG iterations plain", plain, "learned", warm)
    assert np.mean(warm) < np.mean(plain), (plain, warm)
