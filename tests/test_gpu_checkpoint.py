"""Checkpointed GMRES (segments of whole restart cycles, the iterate saved
after each) against one uninterrupted call through the C ABI: the same
iterates, bit for bit, after an interruption and a resume from the file."""
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
