"""Pins of the MLP oracle: against PyTorch CPU (an independent library
implementation of BF16 rounding, GELU, linear layers, autograd and AdamW),
central finite differences, and the exact nearest-neighbour shells of a
lattice."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp as M
from paper_2405_05155_amd import inputs as I


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=4000), rng.normal(size=1000) * 1e-3, rng.normal(size=1000) * 1e3,
                        [0.0, -0.0, 1.0, -2.5]]).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x.astype(np.float64)), ref)


def test_gelu_matches_torch():
    z = np.linspace(-8, 8, 1001)
    ref = torch.nn.functional.gelu(torch.tensor(z), approximate="none").numpy()
    assert np.max(np.abs(M.gelu(z) - ref)) < 1e-15
    zt = torch.tensor(z, requires_grad=True)
    torch.nn.functional.gelu(zt, approximate="none").sum().backward()
    assert np.max(np.abs(M.gelu_grad(z) - zt.grad.numpy())) < 1e-14


def _torch_net(theta):
    p = M.unpack(theta)
    net = torch.nn.Sequential(torch.nn.Linear(100, 128), torch.nn.GELU(), torch.nn.Linear(128, 128),
                              torch.nn.GELU(), torch.nn.Linear(128, 3)).double()
    with torch.no_grad():
        for k, (w, b) in enumerate([("W1", "b1"), ("W2", "b2"), ("W3", "b3")]):
            net[2 * k].weight.copy_(torch.tensor(p[w]))
            net[2 * k].bias.copy_(torch.tensor(p[b]))
    return net


def test_exact_forward_and_gradient_match_torch_autograd():
    theta = M.init_params(0).astype(np.float64)
    rng = np.random.default_rng(1)
    X = rng.normal(size=(64, 100))
    T = rng.normal(size=(64, 3))
    Y, _ = M.forward(theta, X, exact=True)
    net = _torch_net(theta)
    Yt = net(torch.tensor(X))
    assert np.max(np.abs(Y - Yt.detach().numpy())) < 1e-12
    loss, g = M.loss_and_grad(theta, X, T, exact=True)
    lt = torch.mean((Yt - torch.tensor(T)) ** 2)
    lt.backward()
    gt = M.pack({"W1": net[0].weight.grad, "b1": net[0].bias.grad, "W2": net[2].weight.grad,
                 "b2": net[2].bias.grad, "W3": net[4].weight.grad, "b3": net[4].bias.grad})
    assert abs(loss - lt.item()) < 1e-12
    assert np.max(np.abs(g - gt)) < 1e-12 * np.max(np.abs(gt))


def test_gradient_central_differences():
    """P-M1: central differences of the FP64 loss agree with the analytic
    backward to 1e-7 relative (exact mode, no rounding points)."""
    theta = M.init_params(3).astype(np.float64)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(16, 100))
    T = rng.normal(size=(16, 3))
    _, g = M.loss_and_grad(theta, X, T, exact=True)
    idx = rng.choice(M.N_PARAMS, size=40, replace=False)
    for k in idx:
        e = np.zeros_like(theta)
        e[k] = 1e-6
        fd = (M.loss_and_grad(theta + e, X, T, exact=True)[0] - M.loss_and_grad(theta - e, X, T, exact=True)[0]) / 2e-6
        assert abs(fd - g[k]) <= 1e-7 * max(abs(g[k]), 1e-2 * np.max(np.abs(g)))


def test_rounded_gradient_is_close_to_exact():
    theta = M.init_params(5).astype(np.float64)
    rng = np.random.default_rng(6)
    X = rng.normal(size=(256, 100))
    T = rng.normal(size=(256, 3))
    _, ge = M.loss_and_grad(theta, X, T, exact=True)
    _, gr = M.loss_and_grad(theta, X, T, exact=False)
    assert np.linalg.norm(gr - ge) / np.linalg.norm(ge) < 2e-2


def test_zero_input_output():
    theta = M.init_params(7).astype(np.float64)
    p = M.unpack(theta)
    Y, _ = M.forward(theta, np.zeros((1, 100)), exact=True)
    ref = p["W3"] @ M.gelu(p["W2"] @ M.gelu(p["b1"]) + p["b2"]) + p["b3"]
    assert np.max(np.abs(Y[0] - ref)) < 1e-14


def test_adamw_matches_torch():
    theta = M.init_params(8).astype(np.float64)
    rng = np.random.default_rng(9)
    tt = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.AdamW([tt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    th = theta.copy()
    for step in range(1, 4):
        g = rng.normal(size=theta.shape)
        tt.grad = torch.tensor(g)
        opt.step()
        th, m, v = M.adamw(th, g, m, v, step)
    assert np.max(np.abs(th - tt.detach().numpy())) < 1e-14


def test_features_on_lattice_are_the_first_four_shells():
    """Interior lattice particle: the 32 nearest are the shells at 1, sqrt2,
    sqrt3 and 2 dx (6 + 12 + 8 + 6), all within 2h for h = 1.3 dx."""
    pos, dx = I.lattice(16, 3)
    h = 1.3 * dx
    i = (8 * 16 + 8) * 16 + 8
    f = M.features(pos, h, (0.5, 0.5, 0.5), 0.3, rows=[i])[0]
    off = f[:96].reshape(32, 3) * h / dx
    d2 = np.round((off ** 2).sum(1), 9)
    assert list(d2) == [1.0] * 6 + [2.0] * 12 + [3.0] * 8 + [4.0] * 6
    assert sorted(map(tuple, np.round(off[:6]).astype(int))) == sorted(
        [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)])
    e = pos[:, i] - 0.5
    assert abs(f[96] - (np.linalg.norm(e) - 0.3) / h) < 1e-12
    assert np.allclose(f[97:], e / np.linalg.norm(e))


def test_targets_of_a_rigid_rotation_and_a_shell_move():
    """Targets (r_to - r_from)/h, [n][3]: a rotation by 90 degrees about z
    sends (x, y, z) to (-y, x, z), so the target of particle i is
    (-y - x, x - y, 0)/h; a pure shift by one lattice spacing along y gives
    dx/h in the second column only."""
    pos, dx = I.lattice(6, 3)
    h = 1.3 * dx
    rot = np.stack([-pos[1], pos[0], pos[2]])
    t = M.targets(pos, rot, h)
    assert t.shape == (pos.shape[1], 3)
    for i in (0, 17, pos.shape[1] - 1):
        x, y, _ = (float(v) for v in pos[:, i])
        assert np.allclose(t[i], [(-y - x) / h, (x - y) / h, 0.0], rtol=0, atol=1e-12)
    shift = pos.astype(np.float64) + np.array([[0.0], [dx], [0.0]])
    t = M.targets(pos, shift, h)
    assert np.allclose(t[:, 1], 1.0 / 1.3) and np.all(t[:, [0, 2]] == 0.0)
