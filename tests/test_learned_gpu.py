"""Learned support proposal on an MI355X: features, forward pass and gradients
against the FP64 oracle (same BF16 rounding points), the least-squares check
of a proposal against least squares in FP64, the fallback against plain OMP,
and a trained network's gain over plain OMP.

Tolerances. Both sides round the same stored intermediates to BF16, so they
differ only by FP32-versus-FP64 accumulation (relative ~K 2^-24 with K <= 1024
terms) and by the rare BF16 rounding of an intermediate that lands on the other
side of a rounding boundary (one BF16 unit, 2^-8 relative, on single
elements). A gradient entry sums B products, so one such flip moves it by at
most 2^-8 of its largest term: we allow 1e-2 of the largest gradient entry per
element and 2e-3 of the gradient's norm overall. Features carry the BF16
rounding of y and a (|error of a^T y| <= (2^-8 + 2^-16) ||a|| ||y|| by
Cauchy-Schwarz, i.e. 2^-8 after normalisation), FP32 accumulation
(M 2^-24) and the final BF16 rounding (2^-9 of |f| <= 1): 6e-3 of the unit-norm
correlation, i.e. 6e-3 sqrt(M) = 0.096 on the features' sqrt(M) scale.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _bf16_bits(x):
    """float64 array -> int16 tensor of BF16 bits (round to nearest even)."""
    import torch
    from oracle import learned_oracle as lo
    r = lo.bf16_round(x).astype(np.float32)
    return torch.from_numpy((r.view(np.uint32) >> 16).astype(np.uint16).view(np.int16))


def _bits_to_f64(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def _small_params(seed=11):
    from paper_2407_06434_amd import workloads
    return workloads.mlp_init_params(1024, 512, 1024, seed=seed)


def test_features_match_oracle():
    torch = _torch()
    from oracle import learned_oracle as lo
    from paper_2407_06434_amd import omp, workloads
    w = workloads.learned_256x1024(B=300, stream=7)
    w.Y[5] = 0.0
    w.Y[6, 3] = np.nan
    print("case features 256x1024 B=300", flush=True)
    dev = torch.device("cuda:0")
    A = torch.from_numpy(w.A).to(dev)
    d = omp.Dictionary(A, "bf16")
    net = omp.MLP(_small_params())
    F = _bits_to_f64(net.features(d, torch.from_numpy(w.Y).to(dev)))
    Y = w.Y.astype(np.float64)
    Y[6] = 0.0
    ref = lo.features(w.A, Y)
    err = np.abs(F - ref).max()
    print("max feature error", err)
    assert err <= 6e-3 * np.sqrt(256)
    assert np.all(F[5] == 0) and np.all(F[6] == 0)


def _oracle_inputs(B=300, seed=8):
    from oracle import learned_oracle as lo
    from paper_2407_06434_amd import workloads
    w = workloads.learned_256x1024(B=B, stream=seed)
    F = lo.bf16_round(lo.features(w.A, w.Y))
    return w, F


def test_forward_and_gradients_match_oracle():
    torch = _torch()
    from oracle import learned_oracle as lo
    from paper_2407_06434_amd import omp
    w, F = _oracle_inputs()
    p = _small_params()
    net = omp.MLP(p)
    dev = torch.device("cuda:0")
    Fb = _bf16_bits(F).to(dev)
    print("case forward/grad B=300 1024-512-512-1024", flush=True)
    Z = net.forward(Fb).cpu().numpy().astype(np.float64)
    pz = {k: v.astype(np.float64) for k, v in p.items()}
    Zr, _ = lo.forward(pz, F, lo.bf16_round)
    ez = np.abs(Z - Zr).max() / np.abs(Zr).max()
    print("forward max rel err", ez)
    assert ez < 1e-2
    sup = torch.from_numpy(w.true_support.astype(np.int32)).to(dev)
    loss, g = net.grad(Fb, sup)
    T = lo.multi_hot(w.true_support, 1024)
    lr, gr = lo.backward(pz, F, T, lo.bf16_round)
    print("loss gpu", float(loss.item()), "oracle", lr)
    assert abs(float(loss.item()) - lr) <= 1e-3 * abs(lr)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        gg = g[k].cpu().numpy().astype(np.float64)
        d = gg - gr[k]
        mx = np.abs(d).max() / np.abs(gr[k]).max()
        fr = np.linalg.norm(d) / np.linalg.norm(gr[k])
        print(k, "max", mx, "frob", fr)
        assert mx <= 1e-2 and fr <= 2e-3, k


def test_adam_steps_closed_form():
    """Adam's moments and bias correction: a step with learning rate 0 (moments only)
    followed by a step with lr on the same batch at the same weights sees the same
    gradient g twice, so the bias-corrected ratio m/sqrt(v) is exactly g/|g|: every
    weight moves by lr g/(|g| + 1e-8). Checked against the oracle's gradient where it is
    firm (|g| >= 1e-2 max |g|, far above the GPU-oracle gradient difference); elsewhere
    the displacement is bounded by lr. A wrong bias correction at t = 2 would move the
    firm weights by 1.9 lr or 0.1 lr."""
    torch = _torch()
    from oracle import learned_oracle as lo
    from paper_2407_06434_amd import omp
    w, F = _oracle_inputs(B=256, seed=9)
    p = _small_params(seed=12)
    net = omp.MLP(p)
    dev = torch.device("cuda:0")
    Fb = _bf16_bits(F).to(dev)
    sup = torch.from_numpy(w.true_support.astype(np.int32)).to(dev)
    print("case adam lr 0 then lr", flush=True)
    lr = 1e-3
    net.train_step(Fb, sup, 0.0)
    net.train_step(Fb, sup, lr)
    assert net.struct.step == 2
    pz = {k: v.astype(np.float64) for k, v in p.items()}
    _, g = lo.backward(pz, F, lo.multi_hot(w.true_support, 1024), lo.bf16_round)
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in net.export().items()}
    for k in pz:
        disp = got[k] - p[k].astype(np.float64)
        firm = np.abs(g[k]) >= 1e-2 * np.abs(g[k]).max()
        want = -lr * np.sign(g[k])
        err = np.abs(disp - want)[firm].max()
        print(k, "firm", int(firm.sum()), "of", firm.size, "max error / lr", err / lr)
        # FP32 weights of magnitude <= 0.08 carry 2^-24 * 0.08 of rounding per update
        assert err <= 1e-3 * lr, k
        assert np.abs(disp).max() <= lr * (1 + 1e-3), k


def test_ls_check_and_fallback_against_oracle_and_plain_omp(orc):
    """A network whose output layer is zero and whose output bias marks a fixed set P
    proposes P for every signal; signals built on P (plus noise) are accepted with the
    FP64 least-squares coefficients, the others fall back to plain OMP bit for bit."""
    torch = _torch()
    from oracle import learned_oracle as lo
    from paper_2407_06434_amd import omp, workloads
    w = workloads.learned_256x1024(B=512, stream=10)
    g = np.random.default_rng(13)
    Pset = np.sort(g.choice(1024, 32, replace=False))
    p = _small_params(seed=14)
    p["W3"][:] = 0.0
    p["b3"][:] = 0.0
    p["b3"][Pset] = 1.0 + np.arange(32)[::-1] * 0.01  # descending: proposal order = Pset order
    Y = w.Y.copy()
    xs = g.choice([-1, 1], size=(256, 32)) * (1 + np.abs(g.normal(size=(256, 32))))
    Y[:256] = (xs @ w.A[Pset].astype(np.float64) + 0.01 * g.normal(size=(256, 256))).astype(np.float32)
    eps = np.full(512, 0.5, np.float32)
    dev = torch.device("cuda:0")
    A = torch.from_numpy(w.A).to(dev)
    d = omp.Dictionary(A, "bf16")
    net = omp.MLP(p)
    Yt = torch.from_numpy(Y).to(dev)
    Et = torch.from_numpy(eps).to(dev)
    print("case ls_check fixed proposal B=512", flush=True)
    out, nacc = omp.learned_solve(d, net, Yt, 32, eps_per_signal=Et)
    torch.cuda.synchronize()
    st = out.status.cpu().numpy()
    acc = (st & omp.SIG_LEARNED) != 0
    P = np.tile(Pset, (512, 1))
    X, rn, ok = lo.ls_check(w.A, Y, P, eps)
    print("accepted", nacc, "oracle accepts", int(ok.sum()))
    assert nacc == int(acc.sum())
    assert np.array_equal(acc, ok)
    sup = out.support.cpu().numpy()
    coef = out.coef.cpu().numpy()
    assert np.all(sup[acc] == Pset)
    scale = np.maximum(np.abs(X[acc]), 1e-2 * np.abs(X[acc]).max(axis=1, keepdims=True))
    assert np.all(np.abs(coef[acc] - X[acc]) <= 1e-4 * scale)
    assert np.allclose(out.rnorm.cpu().numpy()[acc], rn[acc], rtol=1e-4, atol=1e-6)
    # rejects: identical to a plain BF16 OMP solve of the same signals
    rej = np.nonzero(~acc)[0]
    ref = omp.solve(A, Yt[torch.from_numpy(rej).to(dev)].contiguous(), 32, precision="bf16", dictionary=d,
                    eps_per_signal=Et[torch.from_numpy(rej).to(dev)].contiguous(), dense=False)
    torch.cuda.synchronize()
    assert np.array_equal(sup[rej], ref.support.cpu().numpy())
    assert np.array_equal(coef[rej], ref.coef.cpu().numpy())
    assert np.array_equal(st[rej], ref.status.cpu().numpy())
