"""GPU check of the allocation-free matvec (dmrg_matvec_noalloc) against dmrg_matvec (needs an
MI355X).  Both run the same kernels on the same inputs, so the bar is bit equality.

Two calls in a row share the library's per-GPU scratch: the first, on the 2 x 16 ladder at
m = 1000, from an input with one NaN (the scratch is left holding non-finite values); the
second, on a smaller problem (the 2 x 16 ladder at m = 800 scaled down to m = 300), must still
equal dmrg_matvec and be finite: its intermediate's padding rows meet zero factors, so a scratch
that was not cleared would give NaN.  Then the first problem again with two vectors, and a
problem whose intermediate exceeds the scratch is refused before anything is launched.
"""
import sys

import numpy as np
import pytest

from paper_1103_5391_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1103_5391_amd import lib as L
    L.load()
    return torch, L


def _dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy()


def _both(torch, h, x, nvec=1):
    y_ref = torch.empty_like(x)
    y = torch.full_like(x, 7.0)
    h.matvec(x, y_ref, nvec)
    h.matvec_noalloc(x, y, nvec)
    torch.cuda.synchronize()
    return _host(y_ref), _host(y)


def test_noalloc_matvec_matches_matvec(env):
    torch, L = env
    say("noalloc: ladder16_m1000 with a NaN input")
    big = L.dmrg_create(I.make_workload("ladder16_m1000"))
    small = L.dmrg_create(I.make_workload("ladder16_m800", m=300))
    assert small.n < big.n
    try:
        rng = np.random.default_rng(I.SEED_BASE + 71)
        xb = I.random_psi(big.n, rng)
        xb_nan = xb.copy()
        xb_nan[big.n // 3] = np.nan
        y_ref, y = _both(torch, big, _dev(torch, xb_nan))
        assert np.array_equal(y, y_ref, equal_nan=True)
        assert np.isnan(y).any()

        say("noalloc: smaller problem after the NaN call")
        xs = I.random_psi(small.n, rng)
        y_ref, y = _both(torch, small, _dev(torch, xs))
        assert np.isfinite(y).all()
        assert np.array_equal(y, y_ref)

        say("noalloc: the larger problem again, two vectors")
        x2 = np.concatenate([xb, I.random_psi(big.n, rng)])
        y_ref, y = _both(torch, big, _dev(torch, x2), nvec=2)
        assert np.isfinite(y).all()
        assert np.array_equal(y, y_ref)
    finally:
        big.destroy()
        small.destroy()


def test_noalloc_refuses_an_intermediate_above_the_scratch(env):
    torch, L = env
    say("noalloc: ladder32_m2000 refused")
    h = L.dmrg_create(I.make_workload("ladder32_m2000"))
    try:
        x = _dev(torch, I.random_psi(h.n, np.random.default_rng(5)))
        y = torch.zeros_like(x)
        with pytest.raises(L.DmrgError) as e:
            h.matvec_noalloc(x, y)
        assert e.value.status == -1 and "scratch" in str(e.value)     # DMRG_EINVAL
        torch.cuda.synchronize()
        assert float(y.abs().max()) == 0.0        # nothing was launched
        # the handle stays usable
        h.matvec(x, y)
        torch.cuda.synchronize()
        assert np.isfinite(_host(y)).all()
    finally:
        h.destroy()
