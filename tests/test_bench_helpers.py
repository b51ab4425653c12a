"""Host-side checks of bench.py's solution check (no GPU): the relative
Helmholtz residual it reports for 3D solves (eq. errorAndResid) equals the
one computed with the oracle's Delta_h, and vanishes at the oracle's sparse
direct solution."""
import numpy as np
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
