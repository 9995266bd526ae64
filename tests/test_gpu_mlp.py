"""GPU parity of the learned warm start (features, BF16-MFMA forward,
backward, AdamW, application) against the FP64 oracle with the same BF16
rounding points.  Tolerances (element errors relative to |x| plus the
tensor's RMS):
* features: bit-exact up to rare single-ulp BF16 rounding flips (>= 99.9%
  exact);
* forward outputs: normwise 1e-3; >= 99.5% of elements within 1e-4,
  >= 99.9% within 1e-3, all within 1e-2.  A hidden activation rounds to the
  other BF16 neighbour when its FP32 and FP64 pre-activations straddle a
  rounding boundary (about 3e-5 of the activations, so about one sample in
  a hundred carries a flip somewhere in its 256 activations); a flip moves
  the sample's output by up to ~1e-3 of its scale.  Measured on the GPU:
  99.69% within 1e-4, 99.91% within 3e-4, 99.99% within 1e-3, worst 1.3e-3;
* gradients: normwise 1e-3 and every element within 1e-3 (measured worst
  6e-4, on dW1 at batch 4,096); at the training batch of 65,536, where the
  flips average out over many samples, every element within 1e-4 (measured
  worst 6e-5).
A bar of 99.9% within 1e-4 for the forward pass is out of reach: the flip
rate above bounds it at about 99.7%."""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2405_05155_amd import inputs as I
from tests.gpu_helpers import normwise

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_05155_amd import sph
    sph.lib()
    return sph


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def bits_to_f64(b):
    u = np.asarray(b).astype(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def f64_to_bits(x):
    f = M.bf16(x).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16).astype(np.int16)


def close_elementwise(g, o, frac=0.999, rtol=1e-4):
    scale = np.sqrt(np.mean(o ** 2)) + 1e-30
    ok = np.abs(g - o) <= rtol * (np.abs(o) + scale)
    return ok.mean() >= frac, ok.mean()


def _sphere(S, dx=1.0 / 40, seed=2):
    w = I.sphere_fill(dx=dx, seed=seed)
    f = w.fields
    dom = S.Domain(dim=3, h=w.h, kappa=2.0, lo=w.lo, hi=w.hi, periodic=(0, 0, 0), kernel=S.LAGUERRE_GAUSS)
    prm = S.relax_params(f["center"], f["radius"])
    return w, dom, prm


def test_features_match_oracle(S):
    w, dom, prm = _sphere(S)
    ctx = S.Context(3)
    fg = bits_to_f64(host(ctx.mlp_features(dom, prm, dev(w.pos))))
    rows = np.arange(0, w.n, 7)
    fo = M.bf16(M.features(w.pos, w.h, w.fields["center"], w.fields["radius"], rows=rows))
    g = fg[rows, :100]
    exact = (g == fo)
    assert exact.mean() > 0.999, exact.mean()
    # where they differ it is one BF16 rounding step
    d = np.abs(g - fo)[~exact]
    assert np.all(d <= 2.0 ** -7 * np.maximum(np.abs(fo[~exact]), np.abs(g[~exact])) + 1e-30)
    assert np.all(fg[:, 100:] == 0.0)


def test_forward_matches_oracle(S):
    w, dom, prm = _sphere(S)
    ctx = S.Context(3)
    feat = ctx.mlp_features(dom, prm, dev(w.pos))
    theta = M.init_params(0)
    y = host(ctx.mlp_forward(dev(theta), feat))
    X = bits_to_f64(host(feat))[:, :100]
    yo, _ = M.forward(theta.astype(np.float64), X)
    assert normwise(y, yo) < 1e-3
    # a hidden activation rounds to the other BF16 neighbour when its FP32 and
    # FP64 pre-activations straddle a rounding boundary (~1e-6 relative
    # apart): about one sample in a few hundred carries such a flip
    ok, frac = close_elementwise(y, yo, frac=0.995)
    assert ok, frac
    ok, frac = close_elementwise(y, yo, frac=0.999, rtol=1e-3)
    assert ok, frac
    ok, frac = close_elementwise(y, yo, frac=1.0, rtol=1e-2)
    assert ok, frac


def test_targets_match_oracle(S):
    """Training targets (r_to - r_from)/h of two configurations, [n][3],
    within two FP32 ulps of the oracle's (the GPU multiplies by 1/h)."""
    w, dom, prm = _sphere(S)
    rng = np.random.default_rng(4)
    to = (w.pos + 0.05 * w.h * rng.standard_normal(w.pos.shape)).astype(np.float32)
    ctx = S.Context(3)
    t = host(ctx.mlp_targets(dev(w.pos), dev(to), w.h))
    ref = M.targets(w.pos, to, w.h)
    assert t.shape == ref.shape
    assert np.all(np.abs(t - ref) <= 2.5 * np.finfo(np.float32).eps * np.abs(ref) + 1e-12)


def test_gradient_matches_oracle(S):
    rng = np.random.default_rng(3)
    B = 4096
    X = rng.normal(size=(B, 100))
    Xp = np.zeros((B, 128), dtype=np.int16)
    Xp[:, :100] = f64_to_bits(X)
    T = rng.normal(size=(B, 3)).astype(np.float32)
    theta = M.init_params(1)
    ctx = S.Context(3)
    p = dev(theta)
    zero = torch.zeros_like(p)
    loss, grad = ctx.mlp_train_step(S.adamw_params(lr=0.0), 1, p, zero, zero.clone(), dev(Xp, torch.int16),
                                    dev(T), want_grad=True)
    lo, go = M.loss_and_grad(theta.astype(np.float64), M.bf16(X), T.astype(np.float64))
    assert abs(host(loss)[0] - lo) <= 1e-5 * lo
    gg = host(grad)
    k = 0
    for name, shp in M.SHAPES:
        sz = int(np.prod(shp))
        assert normwise(gg[k:k + sz], go[k:k + sz]) < 1e-3, name
        ok, frac = close_elementwise(gg[k:k + sz], go[k:k + sz], frac=1.0, rtol=1e-3)
        assert ok, (name, frac)
        k += sz
    assert np.array_equal(host(p), theta)  # lr = 0 leaves the masters untouched


def test_adamw_steps_track_oracle(S):
    rng = np.random.default_rng(5)
    B = 2048
    X = rng.normal(size=(B, 100))
    Xp = np.zeros((B, 128), dtype=np.int16)
    Xp[:, :100] = f64_to_bits(X)
    T = (0.1 * rng.normal(size=(B, 3))).astype(np.float32)
    theta0 = M.init_params(2)
    ctx = S.Context(3)
    p = dev(theta0)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    th, mo, vo = theta0.astype(np.float64), np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS)
    Xd, Xb = dev(Xp, torch.int16), M.bf16(X)
    losses = []
    for step in range(1, 6):
        loss, _ = ctx.mlp_train_step(S.adamw_params(), step, p, m, v, Xd, dev(T))
        lo, g = M.loss_and_grad(th, Xb, T.astype(np.float64))
        th, mo, vo = M.adamw(th, g, mo, vo, step)
        losses.append((float(host(loss)[0]), lo))
    upd_g = host(p).astype(np.float64) - theta0
    upd_o = th - theta0
    assert normwise(upd_g, upd_o) < 2e-2
    for lg, lo in losses:
        assert abs(lg - lo) <= 1e-3 * lo
    assert losses[-1][0] < losses[0][0]


def test_apply_moves_like_oracle(S):
    w, dom, prm = _sphere(S, dx=1.0 / 32, seed=4)
    ctx = S.Context(3)
    theta = (0.1 * M.init_params(3)).astype(np.float32)
    pos = dev(w.pos)
    ctx.mlp_apply(dom, prm, pos, dev(theta))
    X = M.bf16(M.features(w.pos, w.h, w.fields["center"], w.fields["radius"]))
    y, _ = M.forward(theta.astype(np.float64), X)
    new = w.pos.astype(np.float64) + w.h * y.T
    c = np.array(w.fields["center"])[:, None]
    e = new - c
    rr = np.sqrt((e ** 2).sum(0))
    phi = rr - w.fields["radius"]
    out = phi > 0
    new[:, out] -= phi[out] * e[:, out] / rr[out]
    d = host(pos) - new
    disp = w.h * np.abs(y).max()
    assert np.mean(np.abs(d) <= 1e-3 * disp + 2e-7) > 0.999


def _batch(rng, B):
    X = rng.normal(size=(B, 100))
    Xp = np.zeros((B, 128), dtype=np.int16)
    Xp[:, :100] = f64_to_bits(X)
    T = (0.1 * rng.normal(size=(B, 3))).astype(np.float32)
    return X, Xp, T


@pytest.mark.parametrize("B", [1, 17, 1000, 64 * 256 + 40, 65536])
def test_gradient_ragged_batches(S, B):
    """Batches that leave a partial 16-sample slab and a partial 64-sample
    block (and, from 16,424 on, more blocks than workgroups) against the
    oracle; 65,536 is the training batch of the bench."""
    rng = np.random.default_rng(B)
    X, Xp, T = _batch(rng, B)
    theta = M.init_params(4)
    ctx = S.Context(3)
    p = dev(theta)
    zero = torch.zeros_like(p)
    loss, grad = ctx.mlp_train_step(S.adamw_params(lr=0.0), 1, p, zero, zero.clone(), dev(Xp, torch.int16), dev(T),
                                    want_grad=True)
    lo, go = M.loss_and_grad(theta.astype(np.float64), M.bf16(X), T.astype(np.float64))
    assert abs(host(loss)[0] - lo) <= 1e-5 * lo
    gg = host(grad)
    k = 0
    for name, shp in M.SHAPES:
        sz = int(np.prod(shp))
        assert normwise(gg[k:k + sz], go[k:k + sz]) < 1e-3, (name, B)
        if B >= 1000:  # a flip in one of a few samples is not averaged out
            ok, frac = close_elementwise(gg[k:k + sz], go[k:k + sz], frac=1.0, rtol=1e-3 if B < 65536 else 1e-4)
            assert ok, (name, B, frac)
        k += sz


def test_gradient_deterministic(S):
    rng = np.random.default_rng(8)
    _, Xp, T = _batch(rng, 5000)
    theta = M.init_params(5)
    ctx = S.Context(3)
    out = []
    for _ in range(2):
        p = dev(theta)
        zero = torch.zeros_like(p)
        _, grad = ctx.mlp_train_step(S.adamw_params(lr=0.0), 1, p, zero, zero.clone(), dev(Xp, torch.int16), dev(T),
                                     want_grad=True)
        out.append(host(grad))
    assert np.array_equal(out[0], out[1])


def test_train_epoch_matches_steps(S):
    """The epoch call (batches gathered by row index in the kernel) against
    sph_mlp_train_step on the same batches gathered on the host: identical."""
    rng = np.random.default_rng(9)
    n, batch = 3 * 2048 + 100, 2048
    _, Xp, T = _batch(rng, n)
    X, Tt = dev(Xp, torch.int16), dev(T)
    theta = M.init_params(6)
    perm = torch.as_tensor(rng.permutation(n), dtype=torch.int64, device="cuda")
    adam = S.adamw_params()
    ctx = S.Context(3)
    p1, m1, v1 = dev(theta), torch.zeros(S.MLP_NPARAMS, device="cuda"), torch.zeros(S.MLP_NPARAMS, device="cuda")
    losses = ctx.mlp_train_epoch(adam, 1, p1, m1, v1, perm, X, Tt, batch)
    p2, m2, v2 = dev(theta), torch.zeros(S.MLP_NPARAMS, device="cuda"), torch.zeros(S.MLP_NPARAMS, device="cuda")
    ref = []
    for b in range(3):
        idx = perm[b * batch:(b + 1) * batch]
        loss, _ = ctx.mlp_train_step(adam, b + 1, p2, m2, v2, X.index_select(0, idx).contiguous(),
                                     Tt.index_select(0, idx).contiguous())
        ref.append(host(loss)[0])
    assert losses.numel() == 3
    assert np.array_equal(host(losses), np.array(ref, dtype=np.float32))
    assert np.array_equal(host(p1), host(p2)) and np.array_equal(host(m1), host(m2)) and np.array_equal(host(v1), host(v2))
    assert not np.array_equal(host(p1), theta)


def test_training_calls_reject_bad_arguments(S):
    """Checked on the host before anything is enqueued."""
    ctx = S.Context(3)
    p = dev(M.init_params(0))
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    X = torch.zeros((64, S.MLP_FEAT_STRIDE), dtype=torch.int16, device="cuda")
    T = torch.zeros((64, 3), device="cuda")
    rows = torch.arange(64, dtype=torch.int64, device="cuda")
    with pytest.raises(S.SphError):  # an update needs step >= 1
        ctx.mlp_train_step(S.adamw_params(), 0, p, m, v, X, T)
    with pytest.raises(S.SphError):  # an epoch always updates: lr > 0
        ctx.mlp_train_epoch(S.adamw_params(lr=0.0), 1, p, m, v, rows, X, T, 32)
    with pytest.raises(S.SphError):
        ctx.mlp_train_epoch(S.adamw_params(), 0, p, m, v, rows, X, T, 32)
    assert np.array_equal(host(p), M.init_params(0))  # nothing ran
    # an empty epoch (fewer rows than one batch) is a no-op
    losses = ctx.mlp_train_epoch(S.adamw_params(), 1, p, m, v, rows[:10], X, T, 32)
    assert losses.numel() == 0 and np.array_equal(host(p), M.init_params(0))
