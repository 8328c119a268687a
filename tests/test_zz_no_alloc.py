"""omp_solve_noalloc (the allocation-free entry point, for callers that cannot
allocate device memory) against omp_solve on the same inputs: two calls in a
row, the second on a smaller input, both bit-identical to omp_solve (same
kernels, same launch order); plus its size limit, refused on the host."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _host(r):
    return {k: v.cpu().numpy() for k, v in r._asdict().items() if v is not None}


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_matches_workspace_solve_twice(prec):
    torch = _torch()
    from paper_2407_06434_amd import omp, workloads
    dev = torch.device("cuda:0")
    cases = [workloads.custom(200, 520, 300, 24, seed=5, k_true=24),   # first call
             workloads.custom(100, 300, 77, 10, seed=6, k_true=10)]    # second call, smaller
    for w in cases:
        print(f"case noalloc {prec} M={w.A.shape[1]} N={w.A.shape[0]} B={w.B} S={w.S}", flush=True)
        A = torch.from_numpy(w.A).to(dev)
        Y = torch.from_numpy(w.Y).to(dev)
        need = omp.workspace_bytes(w.A.shape[1], w.A.shape[0], w.B, w.S, prec)
        assert 0 < need <= omp.load().omp_noalloc_max_bytes()
        ref = omp.solve(A, Y, w.S, precision=prec)
        got = omp.solve_noalloc(A, Y, w.S, precision=prec)
        torch.cuda.synchronize()
        r, g = _host(ref), _host(got)
        assert r.keys() == g.keys()
        for k in r:
            assert np.array_equal(r[k], g[k]), (k, w.B)


def test_noalloc_with_prepared_dictionary_and_per_signal_caps():
    torch = _torch()
    from paper_2407_06434_amd import omp, workloads
    dev = torch.device("cuda:0")
    w = workloads.custom(128, 512, 200, 20, seed=9, k_true=20)
    A = torch.from_numpy(w.A).to(dev)
    Y = torch.from_numpy(w.Y).to(dev)
    d = omp.Dictionary(A, "bf16")
    Sp = torch.from_numpy(np.random.default_rng(3).integers(0, 21, w.B).astype(np.int32)).to(dev)
    print("case noalloc prepared dictionary, per-signal S", flush=True)
    for _ in range(2):
        ref = omp.solve(A, Y, w.S, precision="bf16", dictionary=d, S_per_signal=Sp)
        got = omp.solve_noalloc(A, Y, w.S, precision="bf16", dictionary=d, S_per_signal=Sp)
        torch.cuda.synchronize()
        r, g = _host(ref), _host(got)
        for k in r:
            assert np.array_equal(r[k], g[k]), k


def test_noalloc_refuses_requests_beyond_its_scratch():
    torch = _torch()
    from paper_2407_06434_amd import omp
    dev = torch.device("cuda:0")
    M, N, B, S = 1024, 4096, 4096, 64
    assert omp.workspace_bytes(M, N, B, S) > omp.load().omp_noalloc_max_bytes()
    A = torch.zeros((N, M), device=dev)
    Y = torch.zeros((B, M), device=dev)
    with pytest.raises(omp.OmpError) as ei:
        omp.solve_noalloc(A, Y, S)
    assert ei.value.code == omp.OMP_ENOTSUPP
