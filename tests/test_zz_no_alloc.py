"""The allocation-free training step (sph_mlp_train_step_noalloc, for callers
that cannot allocate device memory) against sph_mlp_train_step through the
C ABI: two calls in a row, the second on a smaller batch, each an AdamW
update with loss and gradient; both entry points run the same kernels with
the same workgroup count, so every output must agree bit for bit (the
fixed workspace keeps the previous call's records, which the second call
must overwrite, not read)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_05155_amd import sph
    sph.lib()
    return sph


def _batch(rng, B):
    x = torch.zeros((B, 128), dtype=torch.float32)
    x[:, :100] = torch.as_tensor(rng.normal(size=(B, 100)), dtype=torch.float32)
    feat = x.to(torch.bfloat16).view(torch.int16).to("cuda")
    target = torch.as_tensor(0.1 * rng.normal(size=(B, 3)), dtype=torch.float32, device="cuda")
    return feat, target


def _init(seed, n):
    rng = np.random.default_rng(seed)
    return torch.as_tensor(rng.uniform(-0.1, 0.1, size=n), dtype=torch.float32, device="cuda")


def test_noalloc_train_step_matches_train_step(S):
    rng = np.random.default_rng(21)
    n = S.MLP_NPARAMS
    ctx = S.Context(3)
    adam = S.adamw_params()
    theta = _init(3, n)
    pa, ma, va = theta.clone(), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    pb, mb, vb = theta.clone(), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    loss_b = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad_b = torch.zeros(n, dtype=torch.float32, device="cuda")
    for step, B in ((1, 65536), (2, 1000)):
        feat, target = _batch(rng, B)
        loss_a, grad_a = ctx.mlp_train_step(adam, step, pa, ma, va, feat, target, want_loss=True, want_grad=True)
        ctx.mlp_train_step_noalloc(adam, step, pb, mb, vb, feat, target, loss=loss_b, grad=grad_b)
        torch.cuda.synchronize()
        assert torch.equal(loss_a, loss_b), (step, B)
        assert torch.equal(grad_a, grad_b), (step, B)
        assert torch.equal(pa, pb) and torch.equal(ma, mb) and torch.equal(va, vb), (step, B)
        assert not torch.equal(pb, theta)
    ctx.close()


def test_noalloc_train_step_rejects_bad_arguments(S):
    """Checked on the host before anything is enqueued."""
    n = S.MLP_NPARAMS
    ctx = S.Context(3)
    p = _init(4, n)
    m, v = torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    feat = torch.zeros((64, 128), dtype=torch.int16, device="cuda")
    target = torch.zeros((64, 3), device="cuda")
    before = p.clone()
    with pytest.raises(S.SphError):  # an update needs step >= 1
        ctx.mlp_train_step_noalloc(S.adamw_params(), 0, p, m, v, feat, target)
    torch.cuda.synchronize()
    assert torch.equal(p, before)
    ctx.close()
