"""The no-allocation application entry point (mfwh_apply_static) against
mfwh_apply, through the C ABI: bitwise equal outputs on consecutive calls
whose sizes shrink (the static scratch keeps the previous call's contents),
in both precisions and with and without forcing; oversize problems are
refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2507_23613_amd import inputs  # noqa: E402


def _rand(gp, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    v = torch.randn((gp.nf,) + gp.shape, generator=g, dtype=torch.float64)
    return v.to("cuda")


def test_apply_static_equals_apply_on_shrinking_calls():
    from paper_2507_23613_amd import _lib as L
    from paper_2507_23613_amd.problem import GpuProblem
    cases = [  # each smaller than the one before
        (dict(seed=4, shape=(40, 45, 50), nf=4, order=4, varc=True), L.MFWH_FP64),
        (dict(seed=3, shape=(61, 67), nf=3, order=4, varc=True), L.MFWH_FP32_STENCIL),
        (dict(seed=5, shape=(21, 23), nf=2, order=2), L.MFWH_FP64),
    ]
    for k, (c, prec) in enumerate(cases):
        w = inputs.small(**c)
        gp = GpuProblem(w, precision=prec, restart=0)
        need = L.mfwh_workspace_bytes(gp.grid, gp.time, 0)
        assert need <= L.MFWH_STATIC_SCRATCH_BYTES
        print(f"[no-alloc] case {k}: {c['shape']} nf={c['nf']} precision={prec} "
              f"scratch {need} bytes", flush=True)
        v = _rand(gp, 10 + k)
        for forcing in (True, False):
            ref = gp.apply(v, forcing=forcing)
            out = torch.full_like(v, float("nan"))
            L.mfwh_apply_static(gp.grid, gp.time, gp.f if forcing else None, v, out, forcing)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (k, forcing,
                                           float((out - ref).abs().max() / ref.abs().max()))


def test_apply_static_refuses_oversize_problem():
    from paper_2507_23613_amd import _lib as L
    from paper_2507_23613_amd.problem import GpuProblem
    w = inputs.small(seed=5, shape=(700, 800), nf=8, order=4)
    gp = GpuProblem(w, restart=0)
    assert L.mfwh_workspace_bytes(gp.grid, gp.time, 0) > L.MFWH_STATIC_SCRATCH_BYTES
    v = torch.zeros((8,) + gp.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(L.MfwhError, match="EWORKSPACE"):
        L.mfwh_apply_static(gp.grid, gp.time, gp.f, v, torch.empty_like(v), 1)
