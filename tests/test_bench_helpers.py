"""Host-side checks of bench.py's helpers (no GPU): the relative Helmholtz
residual it reports for 3D solves (eq. errorAndResid) equals the one computed
with the oracle's Delta_h and vanishes at the oracle's sparse direct
solution; its convergence rates CR and ECR follow their definitions."""
import numpy as np
import pytest
import torch

import bench
from oracle import fd


def _case(n=9, nf=2, seed=0):
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    h = 1.0 / (n - 1)
    f = rng.standard_normal((nf,) + shape)
    c = 1.0 + 0.3 * rng.uniform(-1, 1, shape)
    for m in range(nf):
        fd.zero_boundary(f[m])
    return shape, h, f, c, np.array([3.1, 7.4][:nf])


def test_helmholtz_residual_matches_oracle_operator():
    shape, h, f, c, om = _case()
    rng = np.random.default_rng(1)
    v = rng.standard_normal((2,) + shape)
    for m in range(2):
        fd.zero_boundary(v[m])
    got = bench.helmholtz_residual_3d(torch.as_tensor(v), torch.as_tensor(f), torch.as_tensor(c),
                                      om, h)
    for m in range(2):
        r = f[m] - c ** 2 * fd.laplacian(v[m], (h, h, h), 2) - om[m] ** 2 * v[m]
        ref = np.abs(fd.interior(r)).max() / np.abs(f[m]).max()
        assert abs(got[m] - ref) <= 1e-12 * ref


def test_helmholtz_residual_vanishes_at_direct_solution():
    shape, h, f, c, om = _case()
    v = np.stack([fd.helmholtz_direct(f[m], om[m], (h, h, h), 2, c=c) for m in range(2)])
    got = bench.helmholtz_residual_3d(torch.as_tensor(v), torch.as_tensor(f), torch.as_tensor(c),
                                      om, h)
    assert max(got) < 1e-10


def test_convergence_rates_follow_the_definitions():
    """CR and ECR of Section 8: the paper's own example (CR = 0.5 at N_p = 1
    and CR = 0.25 at N_p = 2 both give ECR = 0.5), and CR of a geometric
    history r^(k) = q^(k-1) over N_it iterations, q^((N_it - 1) / N_it)."""
    import bench
    q, n = 0.8, 50
    hist = q ** np.arange(n)
    cr, ecr = bench.convergence_rates(hist, 1)
    assert cr == pytest.approx(q ** ((n - 1) / n), rel=1e-14) and ecr == cr
    for cr_p, np_ in ((0.5, 1), (0.25, 2)):
        h = np.array([1.0, cr_p ** 2])              # N_it = 2: CR = (r2 / r1)^(1/2)
        cr, ecr = bench.convergence_rates(h, np_)
        assert cr == pytest.approx(cr_p, rel=1e-14)
        assert ecr == pytest.approx(0.5, rel=1e-14)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with a message
    before touching a device (run as its own process, no GPU needed)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
