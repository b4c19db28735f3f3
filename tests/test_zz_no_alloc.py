"""The allocation-free SpMV entry point (vbarms_spmv_noalloc) against vbarms_spmv.

Two calls in a row on different matrices, the second smaller, each compared bit for bit
with the allocating entry point; the library's device-memory counter shows that the
allocation-free calls reach no allocation; a matrix larger than the fixed array is refused.
"""
import numpy as np
import pytest

from paper_1508_02219_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vb():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_02219_amd import vbarms
    vbarms.lib()
    return vbarms


def _check_same(vb, s, tau, seed):
    import torch
    print(f"[case] noalloc spmv {s.name} n={s.n}", flush=True)
    sv = vb.Solver()
    sv.compress(*vb.csr_to_device(s), tau)
    x = torch.as_tensor(np.random.default_rng(seed).standard_normal(s.n), device="cuda")
    y_ref = sv.spmv(x)
    y = torch.full_like(x, float("nan"))
    torch.cuda.synchronize()
    before = vb.device_memory()["runtime_allocs"], vb.device_memory()["live"]
    sv.spmv_noalloc(x, y)
    torch.cuda.synchronize()
    after = vb.device_memory()["runtime_allocs"], vb.device_memory()["live"]
    assert after == before, "the allocation-free entry point allocated device memory"
    assert torch.equal(y, y_ref)
    sv.close()


def test_noalloc_spmv_matches_spmv_twice_second_smaller(vb):
    _check_same(vb, synth.grid_system(12, 10, 9, ell=5, stencil="14rand", perturb=0.1, seed=31), 0.8, 1)
    _check_same(vb, synth.upwind_system(5, 4, 3, seed=32), 1.0, 2)


def test_noalloc_spmv_refuses_oversized_matrix(vb):
    import torch
    n = vb.NOALLOC_MAX_N + 1
    rp = torch.arange(n + 1, dtype=torch.int64, device="cuda")
    ci = torch.arange(n, dtype=torch.int32, device="cuda")
    va = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    sv = vb.Solver()
    sv.compress(rp, ci, va, 1.0)
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(vb.VbarmsError) as e:
        sv.spmv_noalloc(x, y)
    assert e.value.code == vb.ERR_ARG
    assert torch.equal(sv.spmv(x), 2.0 * x)
    sv.close()
