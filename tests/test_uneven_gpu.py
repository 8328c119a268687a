"""Uneven batches through the slot scheduler (omp_solve_multi), on an MI355X.

Two dictionaries (128x512 and 512x2048) with per-signal S_i in 4..64 and
eps_i = 1e-2 ||y_i|| run in one call. Each signal's result must be
bit-identical to the plain batched solve (omp_solve with the same per-signal
arrays): a signal's arithmetic does not depend on its slot, on when it was
admitted or on its neighbours. A sample is also checked step by step against
the FP64 oracle. Slots fewer than signals force many retire/admit cycles.
"""
import numpy as np
import pytest

from tests import parity

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _to_np(r):
    out = dict(support=r.support.cpu().numpy(), coef=r.coef.cpu().numpy(), status=r.status.cpu().numpy(),
               rnorm=r.rnorm.cpu().numpy())
    if r.X is not None:
        out["X"] = r.X.cpu().numpy()
    return out


def _problems(ws, prec, dense=False, slots=0, lanes=0, cfg=0):
    torch = _torch()
    from paper_2407_06434_amd import omp
    dev = torch.device("cuda:0")
    probs = []
    for w in ws:
        A = torch.from_numpy(w.A).to(dev)
        d = omp.Dictionary(A, prec)
        Y = torch.from_numpy(w.Y).to(dev)
        Sp = torch.from_numpy(np.asarray(w.S_per_signal, np.int32)).to(dev)
        Ep = torch.from_numpy(np.asarray(w.eps_per_signal, np.float32)).to(dev)
        probs.append(omp.Problem(d, Y, w.S, 0.0, S_per_signal=Sp, eps_per_signal=Ep, dense=dense, slots=slots,
                                 residual_lanes=lanes, tile_config=cfg))
    return probs


def _plain(w, prec):
    torch = _torch()
    from paper_2407_06434_amd import omp
    dev = torch.device("cuda:0")
    A = torch.from_numpy(w.A).to(dev)
    Y = torch.from_numpy(w.Y).to(dev)
    r = omp.solve(A, Y, w.S, 0.0, precision=prec, dense=True,
                  S_per_signal=torch.from_numpy(np.asarray(w.S_per_signal, np.int32)).to(dev),
                  eps_per_signal=torch.from_numpy(np.asarray(w.eps_per_signal, np.float32)).to(dev))
    torch.cuda.synchronize()
    return _to_np(r)


def _same(a, b, keys=("support", "coef", "status", "rnorm")):
    for k in keys:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_uneven_pair_matches_plain_and_oracle(orc, prec):
    from paper_2407_06434_amd import omp, workloads
    ws = workloads.uneven_pair(B_each=700)
    print(f"case uneven_pair B_each=700 slots=256 {prec}", flush=True)
    probs = _problems(ws, prec, dense=True, slots=256)
    info = {}
    outs = omp.solve_multi(probs, precision=prec, info=info)
    print("multi info", info, flush=True)
    for w, o in zip(ws, outs):
        got = _to_np(o)
        ref = _plain(w, prec)
        _same(got, ref, keys=("support", "coef", "status", "rnorm", "X"))
        k = got["status"] >> 8
        assert np.all(k <= w.S_per_signal)
        idx = np.random.default_rng(1).choice(w.B, 40, replace=False)
        rep = parity.check(w, got, orc, idx=idx)
        print(w.name, rep)


def test_uneven_slot_counts_and_lanes_agree():
    """Different schedules (slots, residual lanes, tile configuration, chunk) give identical results."""
    from paper_2407_06434_amd import omp, workloads
    ws = workloads.uneven_pair(B_each=600)
    print("case uneven schedules", flush=True)
    base = [_to_np(o) for o in omp.solve_multi(_problems(ws, "bf16", slots=256), precision="bf16")]
    for slots, lanes, cfg, chunk in ((512, 0, 1, 8), (1024, 4, 4, 3), (256, 16, 3, 1)):
        outs = omp.solve_multi(_problems(ws, "bf16", slots=slots, lanes=lanes, cfg=cfg), precision="bf16",
                               iters_per_graph=chunk)
        for a, o in zip(base, outs):
            _same(a, _to_np(o))


def test_uneven_edge_cases(orc):
    """Non-finite and zero signals, S_i = 0, eps >= ||y||, fewer signals than slots, an empty problem."""
    torch = _torch()
    from paper_2407_06434_amd import omp, workloads
    ws = workloads.uneven_pair(B_each=300)
    w = ws[0]
    w.Y[3, 5] = np.inf
    w.Y[4] = 0.0
    w.S_per_signal[5] = 0
    w.eps_per_signal[6] = 1e9
    print("case uneven edge cases", flush=True)
    probs = _problems([w, ws[1]], "fp32", slots=256)
    empty = workloads.custom(64, 256, 1, 8, seed=9)
    pe = _problems([workloads.Workload("e", empty.A, empty.Y[:0], 8, 0.0,
                                       S_per_signal=np.zeros(0, np.int32),
                                       eps_per_signal=np.zeros(0, np.float32))], "fp32")
    outs = omp.solve_multi(probs + pe, precision="fp32")
    got = _to_np(outs[0])
    _same(got, _plain(w, "fp32"))
    st = got["status"]
    assert st[3] & omp.SIG_NONFINITE and st[3] >> 8 == 0
    assert st[4] >> 8 == 0 and st[4] & omp.SIG_EPS
    assert st[5] >> 8 == 0 and st[6] >> 8 == 0
    assert np.all(got["support"][5] == -1)
    rep = parity.check(w, got, orc, idx=np.arange(12))
    print(rep)
    torch.cuda.synchronize()


def test_tune_and_determinism():
    from paper_2407_06434_amd import omp, workloads
    ws = workloads.uneven_pair(B_each=2048)
    print("case tune", flush=True)
    probs = _problems(ws, "bf16")
    choice = omp.tune(probs, precision="bf16", sample=2048)
    print("tuned", choice, flush=True)
    for cfg, slots, lanes in choice:
        assert cfg in (1, 3, 4) and slots % 256 == 0 and 256 <= slots <= 2048 and lanes in (0, 1, 2, 4, 8, 16, 32, 64)
    a = [_to_np(o) for o in omp.solve_multi(probs, precision="bf16")]
    b = [_to_np(o) for o in omp.solve_multi(probs, precision="bf16")]
    for x, y, w in zip(a, b, ws):
        _same(x, y)
        _same(x, _plain(w, "bf16"))


def test_slots_with_large_support():
    """S = 150 through the slot scheduler (three solve wavefronts per block): identical
    to the plain batched solve with the same per-signal caps."""
    from paper_2407_06434_amd import workloads
    w = workloads.custom(256, 512, 300, 150, seed=29, k_true=100, snr_db=60.0)
    w.S_per_signal = np.random.default_rng(5).integers(100, 151, size=w.B).astype(np.int32)
    w.eps_per_signal = np.zeros(w.B, np.float32)
    print("case slots S=150", flush=True)
    from paper_2407_06434_amd import omp
    for prec in ("fp32", "bf16"):
        outs = omp.solve_multi(_problems([w], prec, dense=True, slots=256), precision=prec)
        _same(_to_np(outs[0]), _plain(w, prec), keys=("support", "coef", "status", "rnorm", "X"))
