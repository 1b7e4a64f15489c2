"""GPU checks of the persisted autotuner (needs an MI355X): the first call on a problem times the
kernel families and stores its choice under the problem's key; a later handle of the same key
applies the stored choice without timing and computes the same product bit for bit; a stored
choice is applied as stored (products against the oracle); an entry naming a family the problem
lacks is timed again and replaced; the batch's merged launches have their own entries."""
import sys

import numpy as np
import pytest

from oracle import matvec as M
from paper_1103_5391_amd import inputs as I

pytestmark = pytest.mark.gpu

MV_TOL = 1e-12


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1103_5391_amd import lib as L
    L.load()
    return torch, L


def _arch(torch):
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _problem(name):
    from tests.test_gpu_parity import problem
    return problem(name)


def _matvec(torch, h, x):
    xd = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    yd = torch.empty_like(xd)
    h.matvec(xd, yd)
    torch.cuda.synchronize()
    return yd


def _times(d, L):
    return [d[f] for f in L._TUNE_FIELDS]


def test_handle_cache_miss_then_hit(env, tmp_path):
    torch, L = env
    say("tune cache: miss then hit")
    path = tmp_path / "tune.json"
    pb = _problem("chain20_m150")
    h1 = L.dmrg_create(pb)
    r1 = h1.autotune(reps=2, cache=path)
    assert r1["cached"] is False and r1["variant"] == h1.get_gemm()
    key = L.tune_key(pb, L.DMRG_FP64, _arch(torch))
    e = L.tune_cache_lookup(path, key)
    assert e["variant"] == r1["variant"] and _times(e, L) == _times(r1, L)
    assert r1["stage1_register"] > 0 and r1["stage2_register"] > 0
    h2 = L.dmrg_create(pb)
    h2.set_gemm(L.DMRG_GEMM_STAGE1_LDS if r1["variant"] != L.DMRG_GEMM_STAGE1_LDS else 0)
    r2 = h2.autotune(reps=2, cache=path)
    assert r2["cached"] is True and r2["variant"] == r1["variant"] == h2.get_gemm()
    assert _times(r2, L) == _times(r1, L)
    x = I.random_psi(h1.n, np.random.default_rng(I.SEED_BASE + 401))
    assert torch.equal(_matvec(torch, h1, x), _matvec(torch, h2, x))
    # another arithmetic is another key: a miss that adds a second entry
    h2.set_precision(L.DMRG_FP32)
    r3 = h2.autotune(reps=2, cache=path)
    assert r3["cached"] is False
    assert L.tune_cache_lookup(path, L.tune_key(pb, L.DMRG_FP32, _arch(torch)))["variant"] == \
        h2.get_gemm()
    assert L.tune_cache_lookup(path, key)["variant"] == r1["variant"]
    h1.destroy()
    h2.destroy()


@pytest.mark.parametrize("variant", [0, 3, 6, 9, 12, 16, 32])
def test_stored_choice_is_applied(env, tmp_path, variant):
    torch, L = env
    say("tune cache: stored variant", variant)
    path = tmp_path / "tune.json"
    pb = _problem("ladder16_m800")
    key = L.tune_key(pb, L.DMRG_FP64, _arch(torch))
    ms = np.linspace(0.5, 0.95, 10)
    L.tune_cache_store(path, key, variant, ms)
    h = L.dmrg_create(pb)
    r = h.autotune(reps=1, cache=path)
    assert r["cached"] is True and r["variant"] == variant == h.get_gemm()
    assert _times(r, L) == list(ms)
    x = I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + 402))
    y = _matvec(torch, h, x).cpu().numpy()
    yref = M.matvec_sector(pb, x)
    err = float(np.linalg.norm(y - yref) / np.linalg.norm(yref))
    say("  rel err", err)
    assert err <= MV_TOL
    h.destroy()


def test_unrunnable_entry_is_timed_again(env, tmp_path):
    """The LDS-staged and K-split families run FP64 only: an FP32 entry naming them (a file
    edited by hand, say) is a miss, timed again and replaced."""
    torch, L = env
    say("tune cache: unrunnable entry")
    path = tmp_path / "tune.json"
    pb = _problem("chain20_m150")
    key = L.tune_key(pb, L.DMRG_FP32, _arch(torch))
    h = L.dmrg_create(pb)
    h.set_precision(L.DMRG_FP32)
    for bad in (L.DMRG_GEMM_X, L.DMRG_GEMM_K):
        L.tune_cache_store(path, key, bad)
        r = h.autotune(reps=1, cache=path)
        assert r["cached"] is False and r["variant"] not in (L.DMRG_GEMM_X, L.DMRG_GEMM_K)
        assert L.tune_cache_lookup(path, key)["variant"] == r["variant"] == h.get_gemm()
    h.destroy()


def test_unreadable_cache_leaves_handle_usable(env, tmp_path):
    torch, L = env
    say("tune cache: unreadable file")
    path = tmp_path / "tune.json"
    path.write_text("not json", encoding="utf-8")
    pb = _problem("chain12_m30")
    h = L.dmrg_create(pb)
    before = h.get_gemm()
    with pytest.raises(L.DmrgError) as e:
        h.autotune(reps=1, cache=path)
    assert e.value.status == L.STATUS_CODE["DMRG_EIO"] and "not JSON" in str(e.value)
    assert h.get_gemm() == before and path.read_text(encoding="utf-8") == "not json"
    # an unwritable cache: the tuned choice is applied, the error reported
    with pytest.raises(L.DmrgError) as e:
        h.autotune(reps=1, cache=tmp_path / "missing" / "tune.json")
    assert e.value.status == L.STATUS_CODE["DMRG_EIO"]
    x = I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + 403))
    y = _matvec(torch, h, x).cpu().numpy()
    yref = M.matvec_sector(pb, x)
    assert np.linalg.norm(y - yref) <= MV_TOL * np.linalg.norm(yref)
    h.destroy()


def test_batch_cache_miss_then_hit(env, tmp_path):
    torch, L = env
    say("tune cache: batch")
    path = tmp_path / "tune.json"
    pbs = I.batch_workloads(6, seed_offset=700, m_lo=100, m_hi=400)
    hs = [L.dmrg_create(pb) for pb in pbs]
    b1 = L.Batch(hs)
    r1 = b1.autotune(reps=2, cache=path)
    assert r1["cached"] is False
    b1.destroy()
    b2 = L.Batch(hs)
    r2 = b2.autotune(reps=2, cache=path)
    assert r2["cached"] is True and _times(r2, L) == _times(r1, L)
    # the batch key is not a single handle's key
    r3 = hs[0].autotune(reps=1, cache=path)
    assert r3["cached"] is False
    tau, kdim = 0.05, 10
    phis = [I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + 410 + i))
            for i, h in enumerate(hs)]
    pds = [torch.from_numpy(p).to("cuda") for p in phis]
    tds = [torch.full((8 * h.n,), float("nan"), dtype=torch.float64, device="cuda") for h in hs]
    b2.batch_tst_targets(pds, tau, kdim, tds)
    for h, p, t in zip(hs, pds, tds):
        # the handles run their own kernel families: equal up to rounding
        one = torch.empty_like(t)
        h.tst_targets(p, tau, kdim, one, info=False)
        torch.cuda.synchronize()
        err = float(torch.linalg.vector_norm(one - t) / torch.linalg.vector_norm(one))
        assert err <= 1e-11, err
    b2.destroy()
    for h in hs:
        h.destroy()
