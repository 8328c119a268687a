#!/usr/bin/env python3
"""Throughput benchmark of batched OMP on one MI355X.

One step = one complete omp_solve over the batch: every iteration of
Algorithm 1 for every signal (correlation product with the fused argmax, the
Cholesky append and both triangular solves, the residual and the stop test),
plus the set-up and output kernels. The dictionary is prepared once before the
timed region (the paper shares the Gram precomputation between batches) and its
time is reported separately. Inputs are resident in device memory before the
timed region starts. The timed steps replay the solve from the library's cached
hipGraph (its default). Per-kernel durations (the roofline figures) come from
the same number of steps launched one by one right after, with a HIP event pair
around each launch on the stream it runs on: events recorded by graph nodes
carry no timestamps. Both passes must give identical results.

Workload: A 1024 x 4096 Gaussian N(0, 1/M), a batch of 4096 signals, 64-sparse
x with values +-(1 + |N(0,1)|), noise at 30 dB SNR per signal, S = 64 and no
early stop (synthetic stand-in for the paper's unnamed application data).

The same line also carries the measurements beside the benchmark step: plain
FP32, the paper's ablations on these kernels (batching, Gram precomputation,
progressive Cholesky; inverse Cholesky against re-factorisation), the paper's
Algorithm v0 and the FP64 form, the Gram-domain form on the tall
face-recognition shape, uneven batches, the learned proposal and the oracle on
the host (CPU baseline, with every signal it solved checked against the GPU);
--no-* flags skip them. Other modes print their own JSON line instead: --sweep
(the paper's parameter sweep as a speed map), --sweep-tall and --sweep-wide (every
form on square and tall, or wide, dictionaries), --apps (the shapes of its
application table) and --only-gram-domain.

Prints ONE JSON line (rank 0, one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "signals/sec, M=1024 N=4096 S=64 batched OMP vs plain FP32, same supports"
PEAK = {"fp32_mfma": 157.3, "bf16_mfma": 2500.0, "hbm": 8000.0}  # TFLOP/s, TFLOP/s, GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def corr_flops_per_launch(M, N, B):
    """Algorithmic flops of one correlation launch: 2 M N per live signal."""
    return 2.0 * M * N * B


def corr_operand_bytes_per_launch(M, N, B, bf16, keys_per_signal):
    """Operand bytes of one correlation launch, each read or written once: the
    dictionary (N M elements), the residuals (B M), the selected-atom masks (N / 8 per
    signal) and the select keys written (4 bytes each in the BF16 form, 8 in FP32)."""
    e = 2.0 if bf16 else 4.0
    return e * N * M + e * B * M + B * N / 8.0 + B * keys_per_signal * (4.0 if bf16 else 8.0)


def solve_bytes_per_launch(M, S, B):
    """Algorithmic bytes of one solve launch, averaged over the S iterations. Per
    signal at support size K: the atom n* and y for beta (8 M), the packed factor
    read (2 K (K+1)), the Gram row G[n*, support] (4 K), u and the support read
    (8 K), one factor row and x appended or rewritten (~4 (K+1) + 4 (K+1))."""
    tot = 0.0
    for K in range(S):
        tot += 8.0 * M + 2.0 * K * (K + 1) + 12.0 * K + 8.0 * (K + 1)
    return B * tot / S


def residual_bytes_per_launch(M, N, S, B, bf16):
    """HBM-minimum bytes of one residual launch, averaged over the S iterations:
    per signal y read and r written (8 M, plus 2 M for the BF16 copy of r), x and
    the support read (8 K); the gathered atoms at most once per launch (4 M N).
    The per-signal gathers (4 M K) are served by L2 and are reported apart."""
    per = 0.0
    for K in range(1, S + 1):
        per += (10.0 if bf16 else 8.0) * M + 8.0 * K
    return B * per / S + 4.0 * M * N


def residual_gather_bytes_per_launch(M, S, B):
    return B * sum(4.0 * M * K for K in range(1, S + 1)) / S


def kernel_rooflines(w, precision, tim):
    """Per-kernel algorithmic rate against its roofline, from the library's own HIP
    events (recorded around every launch on the solve's stream)."""
    bf16 = precision == "bf16"
    out = {}

    def entry(name, phase, bound, work, unit_scale, peak, unit, extra=None):
        ms, n = tim[phase]
        avg = ms / max(n, 1)
        ach = work / (avg * 1e-3) / unit_scale
        e = dict(bound=bound, achieved=round(ach, 2), peak=peak, unit=unit, frac=round(ach / peak, 4),
                 avg_launch_ms=round(avg, 5), launches=n, total_ms=round(ms, 4),
                 algorithmic_per_launch=float(f"{work:.5e}"))
        if extra:
            e.update(extra)
        out[name] = e

    # keys per signal on the benchmark shape: 16 tiles of 256 atoms, 24 BF16 keys or 1 FP32 key each
    keys = (w.N // 256) * (24 if bf16 else 1)
    entry("k_corr_select", "corr", "mfma", corr_flops_per_launch(w.M, w.N, w.B), 1e12,
          PEAK["bf16_mfma"] if bf16 else PEAK["fp32_mfma"], "TFLOP/s",
          extra=dict(operand_bytes_per_launch=float(f"{corr_operand_bytes_per_launch(w.M, w.N, w.B, bf16, keys):.5e}")))
    entry("k_solve", "update", "hbm", solve_bytes_per_launch(w.M, w.S, w.B), 1e9, PEAK["hbm"], "GB/s")
    gb = residual_gather_bytes_per_launch(w.M, w.S, w.B)
    ms, n = tim["residual"]
    if n == 0:  # a dictionary that fits every XCD's L2: the solve formed the residual
        out["k_residual"] = dict(fused_into="k_solve", launches=0)
        return out
    entry("k_residual", "residual", "hbm", residual_bytes_per_launch(w.M, w.N, w.S, w.B, bf16), 1e9,
          PEAK["hbm"], "GB/s",
          extra=dict(l2_gather_bytes_per_launch=float(f"{gb:.5e}"),
                     l2_gather_GBps=round(gb / (ms / max(n, 1) * 1e-3) / 1e9, 1)))
    return out


def source_digest():
    """Digest of the kernel sources; a traffic figure measured on other sources is stale."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2407_06434_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".cpp", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, precision):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE passes, each scaled by a copy kernel of known size), or None when the
    summary is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"omp_{precision}_1024x4096_B4096_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    digest, val = None, None
    for ln in open(path):
        ln = ln.strip().strip("`")
        if ln.startswith("source digest:"):
            digest = ln.split(":", 1)[1].strip()
        if ln.startswith(f"traffic {kernel}:"):
            val = float(ln.split(":", 1)[1].split()[0])
    if digest != source_digest():
        return None
    return val


def run_gpu(w, precision, steps, warmup):
    import torch
    from paper_2407_06434_amd import omp

    dev = torch.device("cuda:0")
    A = torch.from_numpy(w.A).to(dev)
    Y = torch.from_numpy(w.Y).to(dev)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    d = omp.Dictionary(A, precision)
    e1.record()
    torch.cuda.synchronize()
    dict_ms = e0.elapsed_time(e1)
    ws = torch.empty(omp.workspace_bytes(w.M, w.N, w.B, w.S, precision, with_dict=True), dtype=torch.uint8,
                     device=dev)
    out = None
    for _ in range(warmup):
        out = omp.solve(A, Y, w.S, w.eps, precision=precision, dictionary=d, workspace=ws, out=out)
    torch.cuda.synchronize()
    # Headline pass: each step replays the solve from the library's cached hipGraph.
    t0 = time.perf_counter()
    for _ in range(steps):
        out = omp.solve(A, Y, w.S, w.eps, precision=precision, dictionary=d, workspace=ws, out=out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    res = dict(support=out.support.cpu().numpy(), coef=out.coef.cpu().numpy(),
               status=out.status.cpu().numpy(), rnorm=out.rnorm.cpu().numpy())
    # Kernel pass: the same steps launched one by one with a HIP event pair around every
    # launch, on the stream the kernels run on (events inside a graph carry no timestamps).
    timing = {}
    t0 = time.perf_counter()
    for _ in range(steps):
        out = omp.solve(A, Y, w.S, w.eps, precision=precision, dictionary=d, workspace=ws, out=out,
                        timing=timing)
    torch.cuda.synchronize()
    wall_direct = time.perf_counter() - t0
    same = bool(np.array_equal(res["support"], out.support.cpu().numpy()) and
                np.array_equal(res["coef"], out.coef.cpu().numpy()))
    return dict(wall=wall, wall_direct=wall_direct, timing=timing, dict_ms=dict_ms, res=res,
                graph_equals_direct=same)


def run_per_signal_loop(w, precision, n=32):
    """Ablation A1 of the paper (batching) on these kernels: the first n signals of the
    batch solved one call per signal (B = 1, kernels launched one by one, as a host loop
    over signals would), against the batched step's throughput. Results must equal the
    batched ones."""
    import torch
    from paper_2407_06434_amd import omp
    dev = torch.device("cuda:0")
    A = torch.from_numpy(w.A).to(dev)
    Y = torch.from_numpy(w.Y[:n].copy()).to(dev)
    d = omp.Dictionary(A, precision)
    outs = [omp.solve(A, Y[i:i + 1], w.S, w.eps, precision=precision, dictionary=d, graph=False) for i in range(2)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [omp.solve(A, Y[i:i + 1], w.S, w.eps, precision=precision, dictionary=d, graph=False) for i in range(n)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sup = np.concatenate([o.support.cpu().numpy() for o in outs])
    return dict(wall=wall, n=n, support=sup)


def run_ablation(w, precision, steps=3, **flags):
    """Ablations A2 and A3 of the paper on these kernels: the same step with one design
    choice undone (`gram_on_the_fly`: each pick's Gram row computed from the atoms
    instead of read from G; `refactor`: the Cholesky factor rebuilt at every step
    instead of extended by one row)."""
    import torch
    from paper_2407_06434_amd import omp
    dev = torch.device("cuda:0")
    A = torch.from_numpy(w.A).to(dev)
    Y = torch.from_numpy(w.Y).to(dev)
    d = omp.Dictionary(A, precision)
    out = omp.solve(A, Y, w.S, w.eps, precision=precision, dictionary=d, **flags)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = omp.solve(A, Y, w.S, w.eps, precision=precision, dictionary=d, out=out, **flags)
    torch.cuda.synchronize()
    return dict(wall=(time.perf_counter() - t0) / steps, support=out.support.cpu().numpy())


def run_uneven(precision, steps, warmup, B_each=10000):
    """Uneven batch: two dictionaries (128x512, 512x2048), 10,000 signals each, per-signal
    S_i in 4..64 and eps_i = 1e-2 ||y_i||, solved in one slot-scheduled call after the
    autotuner picked each problem's schedule; timed beside the keep-in-batch form
    (omp_solve per problem with the same per-signal arrays). Results must be identical."""
    import torch
    from paper_2407_06434_amd import omp, workloads
    dev = torch.device("cuda:0")
    ws = workloads.uneven_pair(B_each)
    probs, plain_args = [], []
    for w in ws:
        A = torch.from_numpy(w.A).to(dev)
        d = omp.Dictionary(A, precision)
        Y = torch.from_numpy(w.Y).to(dev)
        Sp = torch.from_numpy(w.S_per_signal).to(dev)
        Ep = torch.from_numpy(w.eps_per_signal).to(dev)
        probs.append(omp.Problem(d, Y, w.S, 0.0, S_per_signal=Sp, eps_per_signal=Ep))
        plain_args.append((A, Y, w.S, d, Sp, Ep))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    choice = omp.tune(probs, precision=precision, sample=4096)
    tune_s = time.perf_counter() - t0
    for _ in range(warmup):
        omp.solve_multi(probs, precision=precision)
    walls, gpu_ms, iters = [], [], 0
    for _ in range(steps):
        info = {}
        t0 = time.perf_counter()
        outs = omp.solve_multi(probs, precision=precision, info=info)
        walls.append(time.perf_counter() - t0)
        gpu_ms.append(info["elapsed_ms"])
        iters = info["iterations"]
    nsig = sum(w.B for w in ws)
    plain = [None] * len(ws)
    for _ in range(warmup):
        for i, (A, Y, S, d, Sp, Ep) in enumerate(plain_args):
            plain[i] = omp.solve(A, Y, S, 0.0, precision=precision, dictionary=d, S_per_signal=Sp,
                                 eps_per_signal=Ep, dense=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for i, (A, Y, S, d, Sp, Ep) in enumerate(plain_args):
            plain[i] = omp.solve(A, Y, S, 0.0, precision=precision, dictionary=d, S_per_signal=Sp,
                                 eps_per_signal=Ep, dense=False, out=plain[i])
    torch.cuda.synchronize()
    plain_wall = (time.perf_counter() - t0) / steps
    same = all(torch.equal(a.support, b.support) and torch.equal(a.coef, b.coef) and
               torch.equal(a.status, b.status) for a, b in zip(outs, plain))
    wall = float(np.median(walls))
    ks = [int(((o.status >> 8).sum()).item()) for o in outs]
    return {"workload": "uneven_128x512_512x2048_B20000", "value": round(nsig / wall, 1), "unit": "signals/s",
            "ms_per_call": round(1e3 * wall, 3), "gpu_ms_per_call": round(float(np.median(gpu_ms)), 3),
            "iterations": iters, "schedule": [dict(tile_config=c, slots=s, residual_lanes=l) for c, s, l in choice],
            "tune_s": round(tune_s, 2), "sum_k": ks,
            "keep_in_batch": {"value": round(nsig / plain_wall, 1), "ms_per_call": round(1e3 * plain_wall, 3)},
            "speedup_vs_keep_in_batch": round(plain_wall / wall, 3), "identical_to_keep_in_batch": bool(same)}


def run_learned(n_train, epochs, n_eval=65536, log=None):
    """Learned support proposal on 256x1024 (S=32, 20 dB, eps_i = sigma_i sqrt(M)):
    labels from our own BF16 OMP on n_train training signals, features, `epochs` of
    Adam, then the learned solve (proposal + least-squares check + OMP fallback) of the
    65,536 evaluation signals, timed beside plain BF16 and plain FP32 OMP on the same
    signals. Training and evaluation are on the GPU; the data is generated on the host."""
    import torch
    from paper_2407_06434_amd import learned, omp, workloads
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    tr = workloads.learned_256x1024(B=n_train, stream=1)
    ev = workloads.learned_256x1024(B=n_eval, stream=0)
    gen_s = time.perf_counter() - t0
    A = torch.from_numpy(tr.A).to(dev)
    d16 = omp.Dictionary(A, "bf16")
    d32 = omp.Dictionary(A, "fp32")
    Ytr = torch.from_numpy(tr.Y).to(dev)
    Etr = torch.from_numpy(tr.eps_per_signal).to(dev)
    Yev = torch.from_numpy(ev.Y).to(dev)
    Eev = torch.from_numpy(ev.eps_per_signal).to(dev)
    net = omp.MLP(workloads.mlp_init_params())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sup = learned.omp_labels(d16, Ytr, 32, Etr)
    F = learned.features(net, d16, Ytr)
    torch.cuda.synchronize()
    label_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    hist = learned.train(net, F, sup, epochs, batch=1024, lr=1e-3, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return r, float(np.median(ts))

    (out, nacc), t_l = timed(lambda: omp.learned_solve(d16, net, Yev, 32, eps_per_signal=Eev))
    ref, t_b = timed(lambda: omp.solve(A, Yev, 32, precision="bf16", dictionary=d16, eps_per_signal=Eev,
                                       dense=False))
    ref32, t_f = timed(lambda: omp.solve(A, Yev, 32, precision="fp32", dictionary=d32, eps_per_signal=Eev,
                                         dense=False))
    s_l = out.support.cpu().numpy()
    s_o = ref.support.cpu().numpy()

    def recall(network):
        """Mean number of plain OMP's atoms among the network's 32 best scores, and the
        number of signals whose 32 best scores are OMP's whole support."""
        Fe = learned.features(network, d16, Yev)
        top = network.forward(Fe).topk(32, dim=1).indices.cpu().numpy()
        hits = np.array([len(set(t.tolist()) & set(o[o >= 0].tolist())) for t, o in zip(top, s_o)])
        return round(float(hits.mean()), 3), int((hits == 32).sum())

    rec_trained = recall(net)
    rec_start = recall(omp.MLP(workloads.mlp_init_params()))
    acc = (out.status.cpu().numpy() & 128) != 0
    same = np.array([set(a[a >= 0]) == set(b[b >= 0]) for a, b in zip(s_l, s_o)])
    rn_ok = bool(np.all(out.rnorm.cpu().numpy()[acc] <= ev.eps_per_signal[acc]))
    rej_same = bool(np.array_equal(s_l[~acc], s_o[~acc]))
    return {"workload": "learned_256x1024_S32_eval65536", "value": round(n_eval / t_l, 1), "unit": "signals/s",
            "accepted": f"{int(nacc)}/{n_eval}", "accepted_same_support_as_omp": f"{int(same[acc].sum())}/{int(acc.sum())}",
            "recall_at_32_of_omp_support": {"trained": rec_trained[0], "untrained_start": rec_start[0],
                                            "signals_with_all_32_trained": rec_trained[1],
                                            "signals_with_all_32_untrained": rec_start[1]},
            "all_same_support_as_omp": f"{int(same.sum())}/{n_eval}", "accepted_residuals_within_eps": rn_ok,
            "rejects_identical_to_omp": rej_same,
            "plain_bf16_omp": round(n_eval / t_b, 1), "plain_fp32_omp": round(n_eval / t_f, 1),
            "speedup_vs_plain_bf16": round(t_b / t_l, 3), "speedup_vs_plain_fp32": round(t_f / t_l, 3),
            "train": {"signals": n_train, "epochs": epochs, "final_loss": round(hist[-1], 4), "train_s": round(train_s, 2),
                      "labels_and_features_s": round(label_s, 2), "host_generation_s": round(gen_s, 2)}}


def run_gram_domain(steps=3, warmup=1):
    """Tall dictionary (the face-recognition shape 8064 x 1207, S = 30, B = 1200): the
    Gram-domain form (P = A^T y once, correlations from P and G) against the
    residual-vector forms, FP32 and BF16, on the same prepared dictionaries. Signals/s
    over graph-replayed calls; supports compared with the FP32 residual-vector form."""
    import torch
    from paper_2407_06434_amd import omp, workloads
    dev = torch.device("cuda:0")
    w = workloads.face_8064x1207()
    A = torch.from_numpy(w.A).to(dev)
    Y = torch.from_numpy(w.Y).to(dev)
    res = {}
    for name, prec, gd in (("gram_domain_fp32", "fp32", True), ("residual_fp32", "fp32", False),
                           ("residual_bf16", "bf16", False)):
        d = omp.Dictionary(A, prec)
        out = None
        for _ in range(warmup):
            out = omp.solve(A, Y, w.S, precision=prec, dictionary=d, out=out, gram_domain=gd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = omp.solve(A, Y, w.S, precision=prec, dictionary=d, out=out, gram_domain=gd)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        res[name] = dict(value=round(w.B / dt, 1), ms_per_call=round(1e3 * dt, 3), support=out.support.cpu().numpy())
        del d
    # per-kernel figures of the Gram-domain form: one more call with the library's
    # HIP events around every launch (direct launches)
    d = omp.Dictionary(A, "fp32")
    tim = {}
    omp.solve(A, Y, w.S, precision="fp32", dictionary=d, gram_domain=True, timing=tim)
    del d
    Np = -(-w.N // 256) * 256
    kavg = (w.S - 1) / 2.0  # support size averaged over the S steps (every signal runs S steps here)
    ms, n = tim["corr"]
    sel_ms = ms / max(n, 1)
    hbm_min = w.B * (4 * Np + Np / 8 + 8)  # P row, mask, key
    g_rows = w.B * 4 * Np * kavg           # G rows of the support, served by the caches
    ums, un = tim["update"]
    ims, inn = tim["init"]
    kernels = {
        "k_gram_select": dict(bound="l2", avg_launch_ms=round(sel_ms, 5), launches=n,
                              hbm_min_bytes_per_launch=float(f"{hbm_min:.5e}"),
                              hbm_min_GBps=round(hbm_min / (sel_ms * 1e-3) / 1e9, 1),
                              g_row_bytes_per_launch=float(f"{g_rows:.5e}"),
                              g_row_GBps=round(g_rows / (sel_ms * 1e-3) / 1e9, 1)),
        "k_solve": dict(avg_launch_ms=round(ums / max(un, 1), 5), launches=un),
        "init_and_projection": dict(total_ms=round(ims, 4), launches=inn,
                                    projection_flop=float(f"{2.0 * (-(-w.B // 256) * 256) * Np * w.M:.5e}")),
    }
    ref = res["residual_fp32"]["support"]
    line = {"workload": f"{w.name}_B{w.B}_S{w.S}", "unit": "signals/s", "kernels": kernels}
    for name, r in res.items():
        same = sum(set(a.tolist()) == set(b.tolist()) for a, b in zip(r.pop("support"), ref))
        line[name] = dict(r, same_supports_as_residual_fp32=f"{same}/{w.B}")
    line["speedup_vs_residual_fp32"] = round(line["gram_domain_fp32"]["value"] / line["residual_fp32"]["value"], 2)
    line["speedup_vs_residual_bf16"] = round(line["gram_domain_fp32"]["value"] / line["residual_bf16"]["value"], 2)
    return line


def v0_bytes_per_launch(N, S, B, elem):
    """Algorithmic bytes of one v0 step launch, averaged over the S steps: per signal at
    support size k, the k columns of D read and the new one written ((k + 1) N), the Gram
    row G[n*, :] (N) and the correlations read and written (2 N), elem bytes each."""
    Np = -(-N // 256) * 256
    return B * elem * Np * sum(k + 4 for k in range(S)) / S


def run_v0_forms(w_main, steps=3, warmup=1):
    """Algorithm v0 of the paper (FP32, opts.v0) and the FP64 form (v0 in FP64) beside
    the residual-vector FP32 form and its re-factorising variant (ablation A3 of the
    paper: inverse Cholesky against re-factorisation), the Gram-domain form forced on
    these wide dictionaries (M < N: where it stops paying) and the FP16 form, on the
    benchmark workload and on the 256 x 1024 workload. Graph-replayed calls; supports compared with the FP32 form;
    one more direct call per form gives the v0 step kernel's launch time."""
    import torch
    from paper_2407_06434_amd import omp, workloads
    dev = torch.device("cuda:0")
    out_all = {}
    for w in (w_main, workloads.batched_256x1024()):
        A = torch.from_numpy(w.A).to(dev)
        Y = torch.from_numpy(w.Y).to(dev)
        res = {}
        for name, prec, flags in (("fp32", "fp32", {}), ("fp32_refactor", "fp32", {"refactor": True}),
                                  ("v0_fp32", "fp32", {"v0": True}), ("fp64", "fp64", {}),
                                  ("gram_domain_fp32", "fp32", {"gram_domain": True}), ("fp16", "fp16", {})):
            d = omp.Dictionary(A, prec)
            out = None
            for _ in range(warmup):
                out = omp.solve(A, Y, w.S, w.eps, precision=prec, dictionary=d, out=out, dense=False, **flags)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                out = omp.solve(A, Y, w.S, w.eps, precision=prec, dictionary=d, out=out, dense=False, **flags)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            r = dict(value=round(w.B / dt, 1), ms_per_call=round(1e3 * dt, 3), support=out.support.cpu().numpy())
            if name in ("v0_fp32", "fp64"):
                tim = {}
                omp.solve(A, Y, w.S, w.eps, precision=prec, dictionary=d, dense=False, timing=tim, **flags)
                ms, n = tim["update"]
                avg = ms / max(n, 1)
                byt = v0_bytes_per_launch(w.N, w.S, w.B, 8 if prec == "fp64" else 4)
                r["k_v0_step"] = dict(bound="hbm", avg_launch_ms=round(avg, 5), launches=n,
                                      algorithmic_per_launch=float(f"{byt:.5e}"),
                                      achieved_GBps=round(byt / (avg * 1e-3) / 1e9, 1),
                                      frac=round(byt / (avg * 1e-3) / 1e9 / PEAK["hbm"], 4))
                r["projection_and_first_pick_ms"] = round(tim["init"][0], 4)
            res[name] = r
            del d
            torch.cuda.empty_cache()
        ref = res["fp32"]["support"]
        line = {}
        for name, r in res.items():
            same = sum(set(a.tolist()) == set(b.tolist()) for a, b in zip(r.pop("support"), ref))
            line[name] = dict(r, same_supports_as_fp32=f"{same}/{w.B}")
        line["v0_speedup_vs_fp32"] = round(line["v0_fp32"]["value"] / line["fp32"]["value"], 3)
        line["fp64_speed_vs_fp32"] = round(line["fp64"]["value"] / line["fp32"]["value"], 3)
        line["fp64_speed_vs_v0_fp32"] = round(line["fp64"]["value"] / line["v0_fp32"]["value"], 3)
        line["gram_domain_speed_vs_fp32"] = round(line["gram_domain_fp32"]["value"] / line["fp32"]["value"], 3)
        line["ablation_inverse_cholesky"] = {
            "v0_fp32": line["v0_fp32"]["value"], "refactorised_each_step_fp32": line["fp32_refactor"]["value"],
            "speedup": round(line["v0_fp32"]["value"] / line["fp32_refactor"]["value"], 2)}
        out_all[f"{w.name}_{w.M}x{w.N}_S{w.S}_B{w.B}"] = line
    return out_all


# The paper's realistic-application shapes (Section 4.2) and its v0 GPU figures
# there (another GPU, precision unstated): context, not a ratio taken here.
APPS = (("image_patches_256x1024", 256, 1024, 32, 5000, 183904.0),
        ("face_8064x1207", 8064, 1207, 30, 1200, 25158.0),
        ("audio_512x2048", 512, 2048, 64, 5000, 28336.0))


def run_apps(steps=3, warmup=1):
    """Signals/s of every form on the shapes of the paper's application table, synthetic
    stand-ins for its data (image patches: the 256 x 1024 workload's first 5000 signals;
    face: face_8064x1207; audio: a 512 x 2048 N(0,1/M) dictionary with 64-sparse
    signals at 30 dB). Graph-replayed calls on prepared dictionaries."""
    import torch
    from paper_2407_06434_amd import omp, workloads
    dev = torch.device("cuda:0")
    out = []
    for name, M, N, S, B, paper in APPS:
        if name.startswith("image"):
            w = workloads.batched_256x1024(B=B)
        elif name.startswith("face"):
            w = workloads.face_8064x1207(B=B)
        else:
            w = workloads.custom(M, N, B, S, seed=2048, k_true=S)
        A = torch.from_numpy(w.A).to(dev)
        Y = torch.from_numpy(w.Y).to(dev)
        row = {"workload": name, "M": M, "N": N, "S": S, "B": B, "paper_v0_gpu": paper}
        forms = [("bf16", "bf16", False), ("fp32", "fp32", False)]
        if M >= N:
            forms.append(("gram_domain_fp32", "fp32", True))
        for fname, prec, gd in forms:
            d = omp.Dictionary(A, prec)
            r = None
            for _ in range(warmup):
                r = omp.solve(A, Y, S, precision=prec, dictionary=d, out=r, gram_domain=gd)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                r = omp.solve(A, Y, S, precision=prec, dictionary=d, out=r, gram_domain=gd)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            row[fname] = round(B / dt, 1)
            del d
        out.append(row)
        log(f"apps: {row}")
    return out


SWEEP_N = (64, 128, 256, 512, 1024, 2048, 4096, 8192)
SWEEP_B = (10, 50, 100, 500, 1000, 5000, 10000)
SWEEP_S = (8, 32, 64)


def run_sweep(precision, steps=3, warmup=1):
    """The paper's parameter sweep (Section 4, parameter sweep) as a speed map of these
    kernels: N in 64..8192, B in 10..10000, S in {8, 32, 64}, M = N/4, cells with S > M
    left out (OMP cannot pick more than M independent atoms). Each (N, S) draws one
    N(0, 1/M) dictionary and 10,000 S-sparse signals at 30 dB SNR; a cell of batch B
    solves the first B of them. Signals/s over `steps` calls replayed from the graph."""
    import torch
    from paper_2407_06434_amd import omp, workloads
    dev = torch.device("cuda:0")
    cells = []
    for N in SWEEP_N:
        M = N // 4
        for S in SWEEP_S:
            if S > M:
                continue
            w = workloads.custom(M, N, max(SWEEP_B), S, seed=N + S)
            A = torch.from_numpy(w.A).to(dev)
            Yall = torch.from_numpy(w.Y).to(dev)
            d = omp.Dictionary(A, precision)
            for B in SWEEP_B:
                Y = Yall[:B].contiguous()
                out = None
                for _ in range(warmup):
                    out = omp.solve(A, Y, S, precision=precision, dictionary=d, out=out)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    out = omp.solve(A, Y, S, precision=precision, dictionary=d, out=out)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / steps
                cells.append({"N": N, "M": M, "B": B, "S": S, "ms_per_call": round(1e3 * dt, 4),
                              "signals_per_s": round(B / dt, 1)})
                log(f"sweep N={N} M={M} B={B} S={S}: {1e3 * dt:.3f} ms, {B / dt:.0f} signals/s")
            del d, A, Yall
    return cells


TALL_M = (512, 2048, 8192)
TALL_N = (256, 1024, 2048)


def time_forms(cells, B=2000, S=32, steps=3, warmup=1, tag="sweep"):
    """Every form (BF16, FP32, Gram-domain FP32) on the (M, N) cells: B signals,
    S = 32, unit-norm N(0,1/M) atoms, S-sparse signals at 30 dB. Signals/s over
    graph-replayed calls on prepared dictionaries."""
    import torch
    from paper_2407_06434_amd import omp, workloads
    dev = torch.device("cuda:0")
    rows = []
    for M, N in cells:
        w = workloads.custom(M, N, B, S, seed=M + N, k_true=S, column_norm="unit")
        A = torch.from_numpy(w.A).to(dev)
        Y = torch.from_numpy(w.Y).to(dev)
        row = {"M": M, "N": N, "B": B, "S": S}
        for fname, prec, gd in (("bf16", "bf16", False), ("fp32", "fp32", False),
                                ("gram_domain_fp32", "fp32", True)):
            d = omp.Dictionary(A, prec)
            r = None
            for _ in range(warmup):
                r = omp.solve(A, Y, S, precision=prec, dictionary=d, out=r, gram_domain=gd)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                r = omp.solve(A, Y, S, precision=prec, dictionary=d, out=r, gram_domain=gd)
            torch.cuda.synchronize()
            row[fname] = round(B * steps / (time.perf_counter() - t0), 1)
            del d
        rows.append(row)
        log(f"{tag}: {row}")
    return rows


def run_sweep_tall(**kw):
    """Where the Gram-domain form pays: square and tall dictionaries (M >= N from the
    grid TALL_M x TALL_N)."""
    return time_forms([(M, N) for M in TALL_M for N in TALL_N if N <= M], tag="tall sweep", **kw)


WIDE_M = (256, 512, 1024)


def run_sweep_wide(**kw):
    """Where the Gram-domain form stops paying: wide dictionaries, N = 2M and N = 4M
    (M from WIDE_M; N = 4M at M = 1024 is the benchmark's shape)."""
    return time_forms([(M, f * M) for M in WIDE_M for f in (2, 4)], tag="wide sweep", **kw)


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, target_s):
    """The oracle, as it stands, on the first n signals of the same workload. Returns
    the baseline entry and the oracle's results on those n signals."""
    import oracle
    threads = oracle.default_threads()
    n0 = threads
    t0 = time.perf_counter()
    parts = [oracle.omp(w.A, w.Y[:n0], w.S, w.eps, threads=threads)]
    t1 = time.perf_counter() - t0
    n = n0
    if t1 < target_s:
        extra = int(max(0, (target_s - t1) / max(t1, 1e-6)) * n0)
        extra = min(extra, w.B - n0)
        if extra > 0:
            t0 = time.perf_counter()
            parts.append(oracle.omp(w.A, w.Y[n0:n0 + extra], w.S, w.eps, threads=threads))
            t1 += time.perf_counter() - t0
            n += extra
    res = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    return dict(value=n / t1, unit="signals/s", cores=threads, cpu_model=cpu_model(), kind="oracle",
                sample=f"first {n} of the {w.B} signals of the benchmark workload, FP64, "
                       f"{threads} host threads, {t1:.1f} s"), res


def oracle_parity(w, gpu_res, free, n):
    """The GPU's results on the n signals the oracle solved, checked pick by pick and
    coefficient by coefficient against it (tests/parity.py rules)."""
    import oracle
    from tests import parity
    idx = np.arange(n)
    rep = parity.check(w, gpu_res, oracle, idx=idx, free=free, raise_on_fail=False)
    return {k: rep[k] for k in ("checked", "passed", "exact_support", "near_tie_picks", "unresolved_fp32",
                                "n_fail", "worst_coef_rel", "worst_pick_ratio")}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16"])
    ap.add_argument("--no-compare", action="store_true",
                    help="skip timing the plain FP32 form beside the BF16 form")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-batch (slot scheduler) measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal measurement")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark step, run the paper's parameter sweep and print its speed map")
    ap.add_argument("--sweep-tall", action="store_true",
                    help="instead of the benchmark step, time every form on square and tall dictionaries")
    ap.add_argument("--sweep-wide", action="store_true",
                    help="instead of the benchmark step, time every form on wide dictionaries (N = 2M, 4M)")
    ap.add_argument("--apps", action="store_true",
                    help="instead of the benchmark step, time every form on the paper's application shapes")
    ap.add_argument("--only-gram-domain", action="store_true",
                    help="run only the Gram-domain measurement on the face-recognition shape and print it")
    ap.add_argument("--no-gram-domain", action="store_true",
                    help="skip the Gram-domain measurement on the tall face-recognition shape")
    ap.add_argument("--only-v0", action="store_true",
                    help="run only Algorithm v0 and the FP64 form (and their FP32 references) and print them")
    ap.add_argument("--no-v0", action="store_true",
                    help="skip Algorithm v0 (FP32) and the FP64 form on the benchmark and 256x1024 workloads")
    ap.add_argument("--no-ablations", action="store_true",
                    help="skip the ablation runs (per-signal loop, Gram rows from atoms, re-factorisation)")
    ap.add_argument("--learned-train", type=int, default=1 << 20, help="training signals for the learned proposal")
    ap.add_argument("--learned-epochs", type=int, default=8)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (scale reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the batch would shard by signals with no in-loop communication).", file=sys.stderr)
        sys.exit(2)

    if args.sweep_tall:
        print(json.dumps({"metric": "tall_sweep", "unit": "signals/s", "data": "synthetic", "steps": 3,
                          "rows": run_sweep_tall()}), flush=True)
        return
    if args.sweep_wide:
        print(json.dumps({"metric": "wide_sweep", "unit": "signals/s", "data": "synthetic", "steps": 3,
                          "rows": run_sweep_wide()}), flush=True)
        return
    if args.apps:
        print(json.dumps({"metric": "application_shapes", "unit": "signals/s", "data": "synthetic",
                          "steps": 3, "rows": run_apps()}), flush=True)
        return
    if args.only_v0:
        from paper_2407_06434_amd import workloads
        print(json.dumps(dict(metric="v0_and_fp64", data="synthetic",
                              **run_v0_forms(workloads.bf16_1024x4096()))), flush=True)
        return
    if args.only_gram_domain:
        print(json.dumps(dict(metric="gram_domain", data="synthetic", **run_gram_domain())), flush=True)
        return
    if args.sweep:
        cells = run_sweep(args.precision)
        print(json.dumps({"metric": "parameter_sweep", "unit": "signals/s", "dtype": args.precision,
                          "data": "synthetic", "steps": 3, "cells": cells}), flush=True)
        return

    from paper_2407_06434_amd import workloads

    t = time.perf_counter()
    w = workloads.bf16_1024x4096()
    log(f"workload {w.name} M={w.M} N={w.N} B={w.B} S={w.S} generated in {time.perf_counter() - t:.1f}s")

    if args.copy_mib > 0:
        import torch
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {src.numel() * 4} bytes read, {dst.numel() * 4} bytes written")
        del src, dst

    g = run_gpu(w, args.precision, args.steps, args.warmup)
    sps = w.B * args.steps / g["wall"]
    ms_step = 1e3 * g["wall"] / args.steps
    log(f"{args.precision}: {sps:.0f} signals/s, {ms_step:.2f} ms/step, phases {g['timing']}")

    tim = g["timing"]
    phase_ms = {k: v[0] / args.steps for k, v in tim.items()}
    kern = kernel_rooflines(w, args.precision, tim)
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    roof = dict(kernel=dom, **{k: v for k, v in kern[dom].items() if k != "total_ms"})
    roof["traffic"] = measured_traffic(dom, args.precision)
    if roof["traffic"] is not None:
        # bytes against bytes: an MFMA-bound kernel's counted traffic over its operand bytes
        base = roof.get("operand_bytes_per_launch", roof["algorithmic_per_launch"])
        roof["traffic_over_operand_bytes" if "operand_bytes_per_launch" in roof else
             "traffic_over_algorithmic"] = round(roof["traffic"] / base, 3)

    line = {
        "metric": METRIC, "value": round(sps, 1), "unit": "signals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else "bf16",
        "data": "synthetic (seeded Gaussian dictionary and sparse signals at 30 dB)",
        "config": {"workload": "omp_1024x4096_S64_B4096", "M": w.M, "N": w.N, "S": w.S, "B": w.B,
                   "precision": args.precision, "early_stop": False},
        "roofline": roof,
        "kernels": {k: {kk: vv for kk, vv in v.items() if kk not in ("per_launch",)} for k, v in kern.items()},
        "phase_ms_per_step": {k: round(v, 4) for k, v in phase_ms.items()},
        "direct_launches": {"value": round(w.B * args.steps / g["wall_direct"], 1),
                            "ms_per_step": round(1e3 * g["wall_direct"] / args.steps, 3),
                            "identical_to_graph": g["graph_equals_direct"]},
        "dict_prep_ms": round(g["dict_ms"], 3),
    }

    if not args.no_compare and args.precision != "fp32":
        fs = max(2, args.steps // 2)
        f = run_gpu(w, "fp32", fs, 1)
        fsps = w.B * fs / f["wall"]
        same = [set(a.tolist()) == set(b.tolist()) for a, b in zip(g["res"]["support"], f["res"]["support"])]
        fk = kernel_rooflines(w, "fp32", f["timing"])
        line["plain_fp32"] = {"value": round(fsps, 1), "unit": "signals/s", "steps": fs,
                              "avg_launch_ms": {k: v["avg_launch_ms"] for k, v in fk.items()},
                              "corr_frac_of_fp32_mfma": fk["k_corr_select"]["frac"]}
        line["speedup_vs_plain_fp32"] = round(sps / fsps, 3)
        line["same_supports_vs_fp32"] = f"{sum(same)}/{w.B}"
        log(f"fp32: {fsps:.0f} signals/s; same supports {sum(same)}/{w.B}")
    line["widened_signals"] = int(np.sum((g["res"]["status"] & 64) != 0))
    if not args.no_ablations:
        loop = run_per_signal_loop(w, args.precision)
        loop_sps = loop["n"] / loop["wall"]
        line["ablation_batching"] = {
            "per_signal_loop": {"value": round(loop_sps, 1), "unit": "signals/s", "signals": loop["n"]},
            "batched": {"value": round(sps, 1), "unit": "signals/s"},
            "speedup": round(sps / loop_sps, 1),
            "identical_supports": bool(np.array_equal(loop["support"], g["res"]["support"][: loop["n"]])),
        }
        log(f"ablation (batching): {line['ablation_batching']}")
        for key, flag, name, base in (("ablation_gram", "gram_on_the_fly", "gram_rows_from_atoms", "prepared_gram"),
                                      ("ablation_cholesky", "refactor", "refactorised_each_step",
                                       "progressive_update")):
            ab = run_ablation(w, args.precision, **{flag: True})
            same_ab = [set(a.tolist()) == set(b.tolist()) for a, b in zip(ab["support"], g["res"]["support"])]
            line[key] = {
                name: {"value": round(w.B / ab["wall"], 1), "unit": "signals/s",
                       "ms_per_step": round(1e3 * ab["wall"], 3)},
                base: {"value": round(sps, 1), "unit": "signals/s"},
                "speedup": round(sps / (w.B / ab["wall"]), 2),
                "same_supports": f"{sum(same_ab)}/{w.B}",
            }
            log(f"{key}: {line[key]}")

    if not args.no_v0:
        v0 = run_v0_forms(w)
        line["v0_and_fp64"] = v0
        log(f"v0 and fp64 forms: {v0}")
    if not args.no_gram_domain:
        gd = run_gram_domain()
        line["gram_domain"] = gd
        log(f"gram domain: {gd}")
    if not args.no_uneven:
        u = run_uneven(args.precision, max(3, args.steps // 2), 1)
        line["uneven"] = u
        log(f"uneven: {u}")
    if not args.no_learned:
        lr = run_learned(args.learned_train, args.learned_epochs, log=log)
        line["learned"] = lr
        log(f"learned: {lr}")

    if not args.no_cpu_baseline:
        cb, free = cpu_baseline(w, args.cpu_seconds)
        line["cpu_baseline"] = cb
        log(f"cpu baseline {cb}")
        n = free["support"].shape[0]
        t = time.perf_counter()
        line["oracle_parity"] = oracle_parity(w, g["res"], free, n)
        log(f"oracle parity on {n} signals ({time.perf_counter() - t:.1f} s): {line['oracle_parity']}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
