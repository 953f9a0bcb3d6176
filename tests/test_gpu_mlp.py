"""Surrogate MLP kernels (include/mlp.h) against the FP64 oracle in its
bfloat16 mode (weights, layer inputs and back-propagated signals rounded to
bfloat16 where the matrix cores take them; products accumulated exactly).
Differences come from FP32 accumulation and erff, and from the rare element
whose FP32 value rounds to the other bfloat16 neighbour."""
import numpy as np
import pytest

from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sur():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2609_26332_amd import surrogate

    return surrogate


def case(seed, n):
    rng = np.random.default_rng(seed)
    theta = M.init_params(seed) + rng.normal(scale=0.02, size=M.n_params())
    X = rng.uniform(-1, 1, size=(n, 5))
    T = rng.normal(size=(n, 2))
    Mk = (rng.random((n, 2)) > 0.2).astype(float)
    return theta.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64), T, Mk


@pytest.mark.parametrize("n", [1, 67, 300])
def test_forward_matches_oracle(sur, n):
    theta, X, T, Mk = case(1, n)
    net = sur.Mlp(members=2, max_batch=512)
    net.set_params(1, theta)
    y = net.forward(1, X).cpu().numpy()
    yo, _ = M.forward(theta, X, bf16=True)
    err = np.abs(y - yo).max() / np.abs(yo).max()
    assert err < 2e-3, err


def test_gradient_matches_oracle(sur):
    theta, X, T, Mk = case(2, 200)
    net = sur.Mlp(members=1, max_batch=256)
    net.set_params(0, theta)
    loss, g = net.loss_grad(0, X, T, Mk)
    assert loss == pytest.approx(M.loss(theta, X, T, Mk, bf16=True), rel=2e-3)
    go = M.gradient(theta, X, T, Mk, bf16=True)
    for (a0, a1) in [(0, 1280), (1280, 1536), (1536, 67072), (67072, 67328), (67328, 132864), (132864, 133120),
                     (133120, 133632), (133632, 133634)]:
        d = np.abs(g[a0:a1] - go[a0:a1]).max() / np.abs(go[a0:a1]).max()
        assert d < 5e-3, (a0, a1, d)


def test_training_and_ensemble(sur):
    import torch

    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, size=(1024, 5)).astype(np.float32)
    T = np.stack([np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2], X[:, 3] ** 2 - X[:, 4]], 1).astype(np.float32)
    Mk = np.ones_like(T)
    net = sur.Mlp(members=3, max_batch=1024)
    xd, td, md = (torch.as_tensor(a).cuda() for a in (X, T, Mk))
    for k in range(3):
        net.set_params(k, sur.glorot_params(10 + k, net.n_params))
    l0 = net.loss_grad(0, X, T, Mk)[0]
    for k in range(3):
        for s in range(300):
            net.train_step(k, xd, td, md, 2e-3)
    l1 = net.loss_grad(0, X, T, Mk)[0]
    assert l1 < 0.05 * l0, (l0, l1)
    # the updated master weights agree with one FP64 Adam step of the oracle
    theta = net.get_params(1).astype(np.float64)
    _, g = net.loss_grad(1, X[:64], T[:64], Mk[:64])
    net2 = sur.Mlp(members=1, max_batch=64)
    net2.set_params(0, theta)
    net2.train_step(0, xd[:64].contiguous(), td[:64].contiguous(), md[:64].contiguous(), 1e-3)
    t1 = net2.get_params(0).astype(np.float64)
    to, _, _ = M.adam_step(theta, np.zeros_like(theta), np.zeros_like(theta), g.astype(np.float64), 1, 1e-3)
    assert np.abs(t1 - to).max() < 1e-6
    # ensemble statistics equal the members' outputs combined
    mean, sd = net.predict(X[:100])
    ys = np.stack([net.forward(k, X[:100]).cpu().numpy() for k in range(3)])
    assert np.allclose(mean.cpu().numpy(), ys.mean(0), atol=1e-6)
    assert np.allclose(sd.cpu().numpy(), ys.std(0), atol=1e-6)


def test_ensemble_step_equals_member_steps(sur):
    """mlp_train_step_ensemble (every member in the same launches, each on its
    own batch) leaves every member's parameters and loss equal, bit for bit,
    to one mlp_train_step per member on that member's batch; three steps, a
    ragged batch of 77 samples."""
    import torch

    rng = np.random.default_rng(11)
    members, n = 3, 77
    X = rng.uniform(-1, 1, size=(members, n, 5)).astype(np.float32)
    T = rng.normal(size=(members, n, 2)).astype(np.float32)
    Mk = (rng.random((members, n, 2)) > 0.3).astype(np.float32)
    a, b = sur.Mlp(members=members, max_batch=128), sur.Mlp(members=members, max_batch=128)
    for k in range(members):
        theta = sur.glorot_params(20 + k, a.n_params)
        a.set_params(k, theta)
        b.set_params(k, theta)
    xd, td, md = (torch.as_tensor(v).cuda() for v in (X, T, Mk))
    for step in range(3):
        la = a.train_step_ensemble(xd, td, md, 1e-3 * (step + 1), want_loss=True)
        lb = [b.train_step(k, xd[k].contiguous(), td[k].contiguous(), md[k].contiguous(), 1e-3 * (step + 1),
                           want_loss=True) for k in range(members)]
        assert la == lb, (step, la, lb)
    for k in range(members):
        assert np.array_equal(a.get_params(k), b.get_params(k)), k


def test_surrogate_gain_over_plain_sweep(sur, tmp_path):
    """What the trained ensemble gains over the plain batched solver on held-out
    cases of the sweep distribution (reduced here: 192 training and 96 held-out
    cases stopped at 3000 steps): every delivered angle is the solver's or an
    ensemble prediction whose spread is within 0.5 degree; the delivery is
    several times faster than solving all held-out cases."""
    from paper_2609_26332_amd import train_surrogate as ts

    files = []
    for seed, count in ((3000, 96), (3001, 96), (4000, 96)):
        files.append(ts.generate(seed, count, 3000, str(tmp_path / f"d{seed}.npz"), log=print))
    r = ts.evaluate(files[:2], files[2], threshold=0.5, epochs=150, members=5, log=print)
    assert r["gain"] > 2.0, r
    assert r["within_0p5_deg"] > 0.6, r
    assert r["mean_err_deg"] < 1.0, r


def test_calibrated_surrogate_on_committed_sweep(sur):
    """The calibrated rule on the committed solver runs of the sweep
    distribution: the ensemble trains on seeds 1000-1014 (7680 cases),
    calibrates its fallback threshold on seeds 1015-1016 and delivers the 512
    held-out cases of seed 2000 (the solver runs the declined ones).  At least
    99% of the delivered angles lie within 0.5 degree of the solver's (the
    committed labels), and the delivery is at least ten times faster than the
    plain sweep of the same cases (the time stored with them, measured on this
    GPU model)."""
    import os

    from paper_2609_26332_amd import sweep, train_surrogate as ts

    data = os.path.join(os.path.dirname(__file__), "..", "paper_2609_26332_amd", "data")
    f = lambda k: os.path.join(data, "sweep_seed%d.npz" % k)
    model, train_s, _, _ = ts.train([f(k) for k in range(1000, 1015)], log=None)
    cal = ts.calibrate(model, [f(1015), f(1016)], log=None)
    va, parts = ts.load([f(2000)])
    cases = sweep.batch_cases(2000, 512)
    delivered, pred, fb, pred_s, fb_s = ts.deliver(model, cases, cal["threshold_deg"], int(parts[0]["cap"]))
    acc = ts.accuracy(delivered, pred, fb, va)
    gain = float(parts[0]["seconds"]) / (pred_s + fb_s)
    print(dict(calibration=cal, gain=round(gain, 2), train_seconds=round(train_s, 1), **acc))
    assert acc["within_0p5_deg"] >= 0.99, acc
    assert gain >= 10.0, (gain, acc)
