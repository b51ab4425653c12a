"""Checkpoint and resume against uninterrupted runs through the C ABI:
GMRES in segments of whole restart cycles (the iterate saved after each) and
the warm-start network's training (its state saved after each epoch) give,
after an interruption and a resume from the file, the results of one
uninterrupted call bit for bit."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-case] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def test_checkpointed_gmres_resumes_bitwise(tmp_path):
    from paper_2507_23613_amd import inputs
    from paper_2507_23613_amd.problem import GpuProblem
    w = inputs.small(seed=21, shape=(33, 29), nf=3, order=4, hi=20.0, filter="adjusted")
    gp = GpuProblem(w, restart=16)
    v1, i1 = gp.gmres(restart=16, max_iter=600, tol=1e-8)
    n = i1["iterations"]
    assert i1["converged"] and n > 32, i1          # the oracle needs 157 iterations
    stop = (n - 1) // 32 * 16                       # whole cycles, before convergence
    path = tmp_path / "gmres.npz"
    # an interrupted solve: the budget runs out after `stop` iterations
    _, i2 = gp.gmres_checkpointed(path, every=16, restart=16, max_iter=stop, tol=1e-8)
    assert not i2["converged"] and i2["iterations"] == stop and path.exists()
    with np.load(path, allow_pickle=False) as d:
        assert int(d["iterations"]) == stop
    # resumed from the file, in longer segments
    v3, i3 = gp.gmres_checkpointed(path, every=32, restart=16, max_iter=600, tol=1e-8)
    assert i3["converged"] and i3["iterations"] == n, (i3["iterations"], n)
    assert torch.equal(v3, v1)
    # a finished checkpoint is returned as it is
    v4, i4 = gp.gmres_checkpointed(path, every=16, restart=16, max_iter=600, tol=1e-8)
    assert i4["converged"] and i4["iterations"] == n and torch.equal(v4, v1)
    with pytest.raises(ValueError):
        gp.gmres_checkpointed(tmp_path / "x.npz", every=24, restart=16)


def test_warm_start_training_resumes_bitwise(tmp_path):
    """Training interrupted after two epochs and resumed from its per-epoch
    checkpoint ends with the weights, Adam moments and losses of an
    uninterrupted three-epoch run (the kernels are deterministic)."""
    from paper_2507_23613_amd.warmstart import WarmStart
    nf, H, W, N = 2, 32, 32, 12
    g = torch.Generator(device="cpu").manual_seed(3)
    feats = torch.randn((N, H, W, 6 * nf), generator=g).float().cuda()
    targets = torch.randn((N, H, W, nf), generator=g).float().cuda()
    a = WarmStart(nf=nf, H=H, W=W, batch=4, seed=1)
    ha = a.train(feats, targets, epochs=3, lr=1e-3, seed=7)
    path = tmp_path / "net.npz"
    b = WarmStart(nf=nf, H=H, W=W, batch=4, seed=1)
    b.train(feats, targets, epochs=2, lr=1e-3, seed=7, checkpoint=path)
    c = WarmStart(nf=nf, H=H, W=W, batch=4, seed=1)
    hc = c.train(feats, targets, epochs=3, lr=1e-3, seed=7, checkpoint=path)
    assert hc == ha and c.step == a.step
    for name in ("params", "m", "v"):
        assert torch.equal(getattr(c, name), getattr(a, name)), name
    with pytest.raises(ValueError):
        WarmStart(nf=nf, H=H, W=W, batch=2, seed=1).train(feats, targets, epochs=3,
                                                          seed=7, checkpoint=path)
