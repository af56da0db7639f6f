"""Pins of the FP64 MLP reference (oracle/mlp.py), each against something other than itself:
  - forward against the same network built from torch.nn.Linear / ReLU layers (FP64, CPU);
  - backward against torch autograd, and against central finite differences;
  - the weighted BCE against torch's binary_cross_entropy_with_logits and its autograd;
  - Adam against torch.optim.Adam over 25 steps, and its first step against the closed form."""
import numpy as np

from oracle import mlp


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init(rng)
    X = rng.random((37, mlp.IN))
    w = rng.standard_normal(37)
    _, cache = mlp.forward(theta, X)
    g = mlp.backward(theta, cache, w)
    f = lambda t: float(w @ mlp.forward(t, X)[0])
    idx = rng.choice(mlp.NPARAMS, 300, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.NPARAMS)
        e[k] = h
        fd = (f(theta + e) - f(theta - e)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_bce_derivative_matches_finite_differences():
    rng = np.random.default_rng(1)
    s = rng.standard_normal(50) * 3
    y = (rng.random(50) < 0.3).astype(float)
    loss, ds = mlp.bce(s, y, 4.0)
    h = 1e-6
    for k in range(50):
        e = np.zeros(50)
        e[k] = h
        fd = (mlp.bce(s + e, y, 4.0)[0] - mlp.bce(s - e, y, 4.0)[0]) / (2 * h)
        assert abs(fd - ds[k]) < 1e-8
    # y = 1 with a large positive score and y = 0 with a large negative score cost ~0
    assert mlp.bce(np.array([40.0, -40.0]), np.array([1.0, 0.0]), 1.0)[0] < 1e-15


def test_adam_first_step_is_signed_lr():
    g = np.array([0.5, -2.0, 1e-3])
    t, m1, m2 = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(t, -0.01 * np.sign(g))


# ---- pins against an independent definition: torch (CPU, FP64) modules, autograd and Adam ----
import torch  # noqa: E402


def _torch_net(theta):
    """The same network built from torch.nn layers, its parameters copied from the flat vector
    (W1[64][8], b1, W2[64][64], b2, W3[64], b3; a weight row is one output unit, as in nn.Linear)."""
    p = mlp.unpack(np.asarray(theta, np.float64))
    net = torch.nn.Sequential(torch.nn.Linear(mlp.IN, mlp.HID), torch.nn.ReLU(),
                              torch.nn.Linear(mlp.HID, mlp.HID), torch.nn.ReLU(),
                              torch.nn.Linear(mlp.HID, 1)).double()
    with torch.no_grad():
        net[0].weight.copy_(torch.from_numpy(p["W1"]))
        net[0].bias.copy_(torch.from_numpy(p["b1"]))
        net[2].weight.copy_(torch.from_numpy(p["W2"]))
        net[2].bias.copy_(torch.from_numpy(p["b2"]))
        net[4].weight.copy_(torch.from_numpy(p["W3"]).reshape(1, mlp.HID))
        net[4].bias.copy_(torch.from_numpy(p["b3"]))
    return net


def _flat_grad(net):
    return np.concatenate([net[0].weight.grad.numpy().ravel(), net[0].bias.grad.numpy(),
                           net[2].weight.grad.numpy().ravel(), net[2].bias.grad.numpy(),
                           net[4].weight.grad.numpy().ravel(), net[4].bias.grad.numpy()])


def _random_theta(rng):
    # non-zero biases, so that a dropped or misplaced bias shows
    theta = mlp.init(rng)
    return theta + 0.1 * rng.standard_normal(mlp.NPARAMS)


def test_forward_matches_torch_modules():
    rng = np.random.default_rng(11)
    theta = _random_theta(rng)
    X = rng.standard_normal((301, mlp.IN))
    s, _ = mlp.forward(theta, X)
    ref = _torch_net(theta)(torch.from_numpy(X)).detach().numpy()[:, 0]
    assert np.allclose(s, ref, rtol=1e-12, atol=1e-12)
    # both ReLUs are active somewhere and inactive somewhere (the pin exercises them)
    _, (_, h1, h2) = mlp.forward(theta, X)
    assert 0 < (h1 > 0).mean() < 1 and 0 < (h2 > 0).mean() < 1


def test_backward_matches_torch_autograd():
    rng = np.random.default_rng(12)
    theta = _random_theta(rng)
    X = rng.standard_normal((173, mlp.IN))
    w = rng.standard_normal(173)
    _, cache = mlp.forward(theta, X)
    g = mlp.backward(theta, cache, w)
    net = _torch_net(theta)
    (net(torch.from_numpy(X))[:, 0] * torch.from_numpy(w)).sum().backward()
    assert np.allclose(g, _flat_grad(net), rtol=1e-11, atol=1e-11)


def test_bce_matches_torch_weighted_logit_loss():
    rng = np.random.default_rng(13)
    s = rng.standard_normal(257) * 4
    y = rng.random(257)                 # soft labels, as the row model trains on
    for pw in (1.0, 3.5):
        loss, ds = mlp.bce(s, y, pw)
        st = torch.from_numpy(s).requires_grad_(True)
        ref = torch.nn.functional.binary_cross_entropy_with_logits(
            st, torch.from_numpy(y), pos_weight=torch.tensor(pw, dtype=torch.float64))
        ref.backward()
        assert abs(loss - ref.item()) <= 1e-12 * max(1.0, abs(ref.item()))
        assert np.allclose(ds, st.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_adam_matches_torch_optimizer_over_many_steps():
    rng = np.random.default_rng(14)
    theta = rng.standard_normal(40)
    m1 = np.zeros(40)
    m2 = np.zeros(40)
    p = torch.from_numpy(theta.copy()).requires_grad_(True)
    opt = torch.optim.Adam([p], lr=2e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 26):
        grad = rng.standard_normal(40) * (1.0 + step % 3)
        theta, m1, m2 = mlp.adam(theta, grad, m1, m2, step, lr=2e-3, b1=0.9, b2=0.999, eps=1e-8)
        p.grad = torch.from_numpy(grad.copy())
        opt.step()
        assert np.allclose(theta, p.detach().numpy(), rtol=1e-12, atol=1e-14), step
