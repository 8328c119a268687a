"""The C-ABI library loads, exports every declared symbol, and rejects invalid
arguments on the host before touching a device (CPU only, no compute calls)."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "batched_omp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(omp_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2407_06434_amd import omp
    return omp.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), n
    from paper_2407_06434_amd import omp
    assert set(omp.EXPORTED) == set(names)


def test_opts_default_enables_graphs(lib):
    from paper_2407_06434_amd import omp
    o = omp.OmpOptsStruct()
    lib.omp_opts_default(ctypes.byref(o))
    assert o.use_graph == 1 and o.precision == 0 and o.workspace is None


def test_version_and_strings(lib):
    assert lib.omp_version().decode().count(".") == 2
    for code in (0, -1, -2, -3, -4):
        assert len(lib.omp_status_string(code)) > 0


def test_struct_layout_matches_header():
    from paper_2407_06434_amd import omp
    assert ctypes.sizeof(omp.OmpDictStruct) == 64
    assert ctypes.sizeof(omp.OmpOptsStruct) == 8 + 8 * 7 + 8 + 16 + 16 + 8


def _opts(ws=1 << 30, prec=0):
    from paper_2407_06434_amd import omp
    o = omp.OmpOptsStruct()
    omp.load().omp_opts_default(ctypes.byref(o))
    o.precision = prec
    o.workspace = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first or sizes are checked
    o.workspace_bytes = ws
    return o


def test_workspace_size_scales_and_rejects(lib):
    from paper_2407_06434_amd import omp
    o = _opts()
    s1 = lib.omp_workspace_size(1024, 4096, 4096, 64, ctypes.byref(o))
    s2 = lib.omp_workspace_size(1024, 4096, 8192, 64, ctypes.byref(o))
    assert 0 < s1 < s2
    assert lib.omp_workspace_size(0, 10, 1, 1, ctypes.byref(o)) == 0
    assert lib.omp_workspace_size(10, 10, 1, 0, ctypes.byref(o)) == 0
    assert lib.omp_workspace_size(10, 10, 1, omp.OMP_MAX_S + 1, ctypes.byref(o)) == 0
    ob = _opts(prec=1)
    assert lib.omp_workspace_size(1024, 4096, 4096, 64, ctypes.byref(ob)) > s1
    oh = _opts(prec=3)  # FP16: the BF16 layout plus one scale pair per signal
    assert lib.omp_workspace_size(1024, 4096, 4096, 64, ctypes.byref(oh)) > lib.omp_workspace_size(
        1024, 4096, 4096, 64, ctypes.byref(ob))
    assert lib.omp_dict_size(1024, 4096, 3) > lib.omp_dict_size(1024, 4096, 1)
    o64 = _opts(prec=2)  # FP64: D and the FP64 state per signal
    assert lib.omp_workspace_size(1024, 4096, 4096, 64, ctypes.byref(o64)) > 8 * 4096 * 64 * 4096
    assert lib.omp_dict_size(1024, 4096, 2) >= 8 * 4096 * 4096 + 4 * 4096 * 4096
    assert lib.omp_dict_size(1024, 4096, 0) >= 4096 * 4096 * 4
    assert lib.omp_dict_size(0, 4096, 0) == 0


FAKE = ctypes.c_void_p(1 << 20)  # an aligned non-null address; never dereferenced by validation


@pytest.mark.parametrize("case", [
    "M0", "N0", "Bneg", "S0", "S_gt_M", "S_gt_N", "nan_eps", "lda_lt_M", "ldy_lt_M", "nullA", "nullY",
    "nullsup", "noopts", "badprec", "misalignedA"])
def test_solve_rejects_invalid_arguments(lib, case):
    from paper_2407_06434_amd import omp
    args = dict(A=FAKE, M=64, N=256, lda=64, Y=FAKE, B=10, ldy=64, S=8, eps=0.0, X=FAKE, sup=FAKE)
    o = _opts()
    if case == "M0": args["M"] = 0
    if case == "N0": args["N"] = 0
    if case == "Bneg": args["B"] = -1
    if case == "S0": args["S"] = 0
    if case == "S_gt_M": args.update(M=8, lda=8, ldy=8, S=9)
    if case == "S_gt_N": args.update(N=7)
    if case == "nan_eps": args["eps"] = math.nan
    if case == "lda_lt_M": args["lda"] = 63
    if case == "ldy_lt_M": args["ldy"] = 63
    if case == "nullA": args["A"] = None
    if case == "nullY": args["Y"] = None
    if case == "nullsup": args["sup"] = None
    if case == "badprec": o.precision = 7
    if case == "misalignedA": args["A"] = ctypes.c_void_p((1 << 20) + 2)
    op = None if case == "noopts" else ctypes.byref(o)
    rc = lib.omp_solve(args["A"], args["M"], args["N"], args["lda"], args["Y"], args["B"], args["ldy"],
                       args["S"], args["eps"], args["X"], args["sup"], op, None)
    assert rc == omp.OMP_EINVAL, (case, rc)


def test_solve_rejects_small_or_missing_workspace(lib):
    from paper_2407_06434_amd import omp
    o = _opts(ws=1024)
    rc = lib.omp_solve(FAKE, 64, 256, 64, FAKE, 10, 64, 8, 0.0, FAKE, FAKE, ctypes.byref(o), None)
    assert rc == omp.OMP_EWORKSPACE
    o = _opts()
    o.workspace = None
    rc = lib.omp_solve(FAKE, 64, 256, 64, FAKE, 10, 64, 8, 0.0, FAKE, FAKE, ctypes.byref(o), None)
    assert rc == omp.OMP_EWORKSPACE
    o = _opts()
    o.workspace = ctypes.c_void_p((1 << 20) + 64)  # not 256-byte aligned
    rc = lib.omp_solve(FAKE, 64, 256, 64, FAKE, 10, 64, 8, 0.0, FAKE, FAKE, ctypes.byref(o), None)
    assert rc == omp.OMP_EWORKSPACE


def test_solve_rejects_bad_ablation_flag(lib):
    from paper_2407_06434_amd import omp
    o = _opts()
    o.gram_on_the_fly = 2
    rc = lib.omp_solve(FAKE, 64, 256, 64, FAKE, 10, 64, 8, 0.0, FAKE, FAKE, ctypes.byref(o), None)
    assert rc == omp.OMP_EINVAL
    o = _opts()
    o.refactor = -1
    rc = lib.omp_solve(FAKE, 64, 256, 64, FAKE, 10, 64, 8, 0.0, FAKE, FAKE, ctypes.byref(o), None)
    assert rc == omp.OMP_EINVAL
    o = _opts()
    o.gram_domain = 3
    rc = lib.omp_solve(FAKE, 64, 256, 64, FAKE, 10, 64, 8, 0.0, FAKE, FAKE, ctypes.byref(o), None)
    assert rc == omp.OMP_EINVAL


def test_gram_domain_form(lib):
    """The Gram-domain form is FP32 only, and its workspace holds P (B_pad x N_pad floats)."""
    from paper_2407_06434_amd import omp
    o = _opts()
    o.gram_domain = 1
    o.precision = omp.PREC["bf16"]
    rc = lib.omp_solve(FAKE, 64, 256, 64, FAKE, 10, 64, 8, 0.0, FAKE, FAKE, ctypes.byref(o), None)
    assert rc == omp.OMP_EINVAL
    a = omp.OmpOptsStruct()
    lib.omp_opts_default(ctypes.byref(a))
    g = omp.OmpOptsStruct()
    lib.omp_opts_default(ctypes.byref(g))
    g.gram_domain = 1
    s0 = lib.omp_workspace_size(2048, 1000, 300, 30, ctypes.byref(a))
    s1 = lib.omp_workspace_size(2048, 1000, 300, 30, ctypes.byref(g))
    assert s1 - s0 >= 512 * 1024 * 4
    # The face-recognition shape (8064 x 1207, B = 1200): 10 x 10 tiles of 128 leave CUs
    # idle, so P's product is split into 8 K chunks whose partials the workspace holds:
    # P plus 8 partials of B_pad x N_pad = 1280 x 1280 floats (and 8 keys per signal).
    f0 = lib.omp_workspace_size(8064, 1207, 1200, 30, ctypes.byref(a))
    f1 = lib.omp_workspace_size(8064, 1207, 1200, 30, ctypes.byref(g))
    assert 9 * 1280 * 1280 * 4 <= f1 - f0 < 9 * 1280 * 1280 * 4 + (1 << 20)
    # Automatic choice (2): the Gram-domain form for FP32 and 4M >= N, except a dictionary
    # under 1 MiB in a batch of more than 4096 signals.
    au = omp.OmpOptsStruct()
    lib.omp_opts_default(ctypes.byref(au))
    au.gram_domain = 2
    assert lib.omp_workspace_size(8064, 1207, 1200, 30, ctypes.byref(au)) == f1
    for (M, N, B), gd in {(1024, 4096, 4096): True, (1024, 8192, 4096): False, (256, 128, 5000): False,
                          (512, 512, 5000): True, (128, 512, 60): True}.items():
        want = g if gd else a
        assert lib.omp_workspace_size(M, N, B, 30, ctypes.byref(au)) == \
            lib.omp_workspace_size(M, N, B, 30, ctypes.byref(want)), (M, N, B)
    au.precision = omp.PREC["bf16"]
    ab = omp.OmpOptsStruct()
    lib.omp_opts_default(ctypes.byref(ab))
    ab.precision = omp.PREC["bf16"]
    assert lib.omp_workspace_size(8064, 1207, 1200, 30, ctypes.byref(au)) == \
        lib.omp_workspace_size(8064, 1207, 1200, 30, ctypes.byref(ab))
    # The 1024 x 4096 shape at B = 4096 has 1024 tiles: no split, P alone.
    b0 = lib.omp_workspace_size(1024, 4096, 4096, 64, ctypes.byref(a))
    b1 = lib.omp_workspace_size(1024, 4096, 4096, 64, ctypes.byref(g))
    assert 4096 * 4096 * 4 <= b1 - b0 < 4096 * 4096 * 4 + (1 << 20)


def test_solve_beyond_limits_is_not_supported(lib):
    from paper_2407_06434_amd import omp
    o = _opts()
    rc = lib.omp_solve(FAKE, 512, 1024, 512, FAKE, 10, 512, omp.OMP_MAX_S + 1, 0.0, FAKE, FAKE,
                       ctypes.byref(o), None)
    assert rc == omp.OMP_ENOTSUPP


def test_solve_whose_lds_does_not_fit_is_not_supported(lib):
    """The solve keeps the packed factor (and in the BF16 form one list entry per
    select key) in LDS: a problem whose single wavefront would need more than the
    160 KiB of a workgroup is refused before anything is launched; S = 256 with a
    4096-atom dictionary still fits (one wavefront per block)."""
    from paper_2407_06434_amd import omp
    o = _opts()
    o.precision = omp.PREC["bf16"]
    N = 1 << 20  # 98,304 BF16 keys per signal
    rc = lib.omp_solve(FAKE, 64, N, 64, FAKE, 10, 64, 64, 0.0, FAKE, FAKE, ctypes.byref(o), None)
    assert rc == omp.OMP_ENOTSUPP
    o = _opts(ws=1024)  # fits: the (too small) workspace is what is refused
    o.precision = omp.PREC["bf16"]
    rc = lib.omp_solve(FAKE, 512, 4096, 512, FAKE, 10, 512, 256, 0.0, FAKE, FAKE, ctypes.byref(o), None)
    assert rc == omp.OMP_EWORKSPACE


def test_solve_with_mismatched_dictionary_is_rejected(lib):
    from paper_2407_06434_amd import omp
    d = omp.OmpDictStruct()
    d.magic = 0x4F4D5044
    d.precision = 0
    d.M, d.N = 64, 255
    d.A = FAKE
    d.mem = FAKE
    o = _opts()
    o.dict = ctypes.pointer(d)
    rc = lib.omp_solve(FAKE, 64, 256, 64, FAKE, 10, 64, 8, 0.0, FAKE, FAKE, ctypes.byref(o), None)
    assert rc == omp.OMP_EINVAL
    d.N = 256
    d.magic = 0
    rc = lib.omp_solve(FAKE, 64, 256, 64, FAKE, 10, 64, 8, 0.0, FAKE, FAKE, ctypes.byref(o), None)
    assert rc == omp.OMP_EINVAL


def test_dict_init_rejects_invalid(lib):
    from paper_2407_06434_amd import omp
    d = omp.OmpDictStruct()
    assert lib.omp_dict_init(ctypes.byref(d), FAKE, 64, 256, 63, 0, FAKE, 1 << 30, None) == omp.OMP_EINVAL
    assert lib.omp_dict_init(ctypes.byref(d), FAKE, 64, 256, 64, 4, FAKE, 1 << 30, None) == omp.OMP_EINVAL
    assert lib.omp_dict_init(ctypes.byref(d), FAKE, 64, 256, 64, 0, FAKE, 16, None) == omp.OMP_EWORKSPACE
    assert lib.omp_dict_init(None, FAKE, 64, 256, 64, 0, FAKE, 1 << 30, None) == omp.OMP_EINVAL


def test_empty_batch_is_a_no_op(lib):
    from paper_2407_06434_amd import omp
    o = _opts()
    rc = lib.omp_solve(FAKE, 64, 256, 64, None, 0, 64, 8, 0.0, None, None, ctypes.byref(o), None)
    assert rc == omp.OMP_OK


def _fake_dict(M=128, N=512, prec=0):
    from paper_2407_06434_amd import omp
    d = omp.OmpDictStruct()
    d.magic = 0x4F4D5044
    d.precision = prec
    d.M, d.N = M, N
    d.A = FAKE
    d.mem = FAKE
    return d


def _problem(d, B=1000, S=32, slots=0):
    from paper_2407_06434_amd import omp
    p = omp.OmpProblemStruct()
    p.dict = ctypes.pointer(d)
    p.Y = FAKE.value
    p.B, p.ldy, p.S = B, d.M, S
    p.support_out = FAKE.value
    p.slots = slots
    return p


def _mopts(ws=1 << 40, prec=0):
    from paper_2407_06434_amd import omp
    o = omp.OmpMultiOptsStruct()
    o.precision = prec
    o.workspace = FAKE.value
    o.workspace_bytes = ws
    return o


def test_multi_struct_layout():
    from paper_2407_06434_amd import omp
    assert ctypes.sizeof(omp.OmpProblemStruct) == 8 * 4 + 8 + 8 * 7 + 16
    assert ctypes.sizeof(omp.OmpMultiOptsStruct) == 8 + 8 * 4


def test_multi_workspace_size(lib):
    d0, d1 = _fake_dict(128, 512), _fake_dict(512, 2048)
    o = _mopts()
    one = (type(_problem(d0)) * 1)(_problem(d0, slots=256))
    two = (type(_problem(d0)) * 2)(_problem(d0, slots=256), _problem(d1, slots=1024))
    big = (type(_problem(d0)) * 2)(_problem(d0, slots=512), _problem(d1, slots=1024))
    s1 = lib.omp_multi_workspace_size(one, 1, ctypes.byref(o))
    s2 = lib.omp_multi_workspace_size(two, 2, ctypes.byref(o))
    s3 = lib.omp_multi_workspace_size(big, 2, ctypes.byref(o))
    assert 0 < s1 < s2 < s3
    assert lib.omp_multi_workspace_size(two, 0, ctypes.byref(o)) == 0
    assert lib.omp_multi_workspace_size(two, 9, ctypes.byref(o)) == 0


@pytest.mark.parametrize("case", ["nprob0", "nprob9", "badprec", "dict_prec", "dict_magic", "S0", "S_gt_M",
                                  "nan_eps", "ldy", "nullY", "nullsup", "cfg", "lanes", "slots_neg", "chunk"])
def test_multi_rejects_invalid(lib, case):
    from paper_2407_06434_amd import omp
    d = _fake_dict()
    p = _problem(d)
    o = _mopts()
    n = 1
    if case == "nprob0": n = 0
    if case == "nprob9": n = 9
    if case == "badprec": o.precision = 5
    if case == "dict_prec": d.precision = 1
    if case == "dict_magic": d.magic = 1
    if case == "S0": p.S = 0
    if case == "S_gt_M": p.S = 129
    if case == "nan_eps": p.eps = math.nan
    if case == "ldy": p.ldy = 127
    if case == "nullY": p.Y = None
    if case == "nullsup": p.support_out = None
    if case == "cfg": p.tile_config = 5
    if case == "lanes": p.residual_lanes = 3
    if case == "slots_neg": p.slots = -256
    if case == "chunk": o.iters_per_graph = 65
    arr = (type(p) * 9)(*([p] * 9))
    assert lib.omp_solve_multi(arr, n, ctypes.byref(o), None) == omp.OMP_EINVAL, case
    assert lib.omp_tune(arr, n, ctypes.byref(o), 0, None) == omp.OMP_EINVAL, case


def test_multi_rejects_small_workspace(lib):
    from paper_2407_06434_amd import omp
    d = _fake_dict()
    arr = (type(_problem(d)) * 1)(_problem(d))
    o = _mopts(ws=4096)
    assert lib.omp_solve_multi(arr, 1, ctypes.byref(o), None) == omp.OMP_EWORKSPACE
    o = _mopts()
    o.workspace = (1 << 20) + 64
    assert lib.omp_solve_multi(arr, 1, ctypes.byref(o), None) == omp.OMP_EWORKSPACE
    p = _problem(d, S=300)
    arr = (type(p) * 1)(p)
    d.M, d.N = 512, 1024
    p.ldy = 512
    assert lib.omp_solve_multi(arr, 1, ctypes.byref(_mopts()), None) == omp.OMP_ENOTSUPP


def test_multi_all_empty_is_a_no_op(lib):
    from paper_2407_06434_amd import omp
    d = _fake_dict()
    p = _problem(d, B=0)
    p.Y = None
    p.support_out = None
    arr = (type(p) * 1)(p)
    assert lib.omp_solve_multi(arr, 1, ctypes.byref(_mopts()), None) == omp.OMP_OK


def test_mlp_struct_and_sizes(lib):
    from paper_2407_06434_amd import omp
    assert ctypes.sizeof(omp.OmpMlpStruct) == 4 * 4 + 8 * 3
    s = lib.omp_mlp_size(1024, 1024, 1024)
    assert s >= 3 * 1024 * 1024 * (4 * 3 + 2 * 2)
    assert lib.omp_mlp_size(1000, 1024, 1024) == 0
    assert lib.omp_mlp_size(1024, 0, 1024) == 0
    assert lib.omp_mlp_size(512, 256, 512) < s


def _fake_mlp(n=1024, h=512):
    from paper_2407_06434_amd import omp
    m = omp.OmpMlpStruct()
    m.magic = 0x4F4D4C50
    m.n_in, m.n_hidden, m.n_out = n, h, n
    m.mem = FAKE.value
    return m


def test_mlp_rejects_invalid(lib):
    from paper_2407_06434_amd import omp
    m = omp.OmpMlpStruct()
    ptrs = (ctypes.c_void_p * 6)(*([FAKE.value] * 6))
    assert lib.omp_mlp_init(ctypes.byref(m), 1024, 512, 1024, None, FAKE, 1 << 40, None) == omp.OMP_EINVAL
    assert lib.omp_mlp_init(ctypes.byref(m), 1000, 512, 1024, ptrs, FAKE, 1 << 40, None) == omp.OMP_EINVAL
    assert lib.omp_mlp_init(ctypes.byref(m), 1024, 512, 1024, ptrs, FAKE, 1024, None) == omp.OMP_EWORKSPACE
    bad = (ctypes.c_void_p * 6)(*([FAKE.value] * 5 + [None]))
    assert lib.omp_mlp_init(ctypes.byref(m), 1024, 512, 1024, bad, FAKE, 1 << 40, None) == omp.OMP_EINVAL
    fm = _fake_mlp()
    assert lib.omp_mlp_workspace_size(ctypes.byref(fm), 256, 100) > 0
    assert lib.omp_mlp_workspace_size(ctypes.byref(m), 256, 100) == 0  # not initialised
    # gradients need at least one signal and S within the output size
    assert lib.omp_mlp_grad(ctypes.byref(fm), FAKE, FAKE, None, 0, 32, None, None, FAKE, 1 << 40,
                            None) == omp.OMP_EINVAL
    assert lib.omp_mlp_train_step(ctypes.byref(fm), FAKE, FAKE, None, 10, 32, -1.0, None, FAKE, 1 << 40,
                                  None) == omp.OMP_EINVAL
    assert lib.omp_mlp_train_step(ctypes.byref(fm), FAKE, FAKE, None, 10, 1025, 1e-3, None, FAKE, 1 << 40,
                                  None) == omp.OMP_EINVAL
    assert lib.omp_mlp_forward(ctypes.byref(fm), FAKE, 10, FAKE, FAKE, 16, None) == omp.OMP_EWORKSPACE


def test_learned_solve_rejects_invalid(lib):
    from paper_2407_06434_amd import omp
    fm = _fake_mlp()
    d = _fake_dict(256, 1024, prec=1)
    o = _opts(prec=1)
    assert lib.omp_learned_workspace_size(ctypes.byref(d), ctypes.byref(fm), 100, 32, ctypes.byref(o)) > 0
    d0 = _fake_dict(256, 1024, prec=0)
    assert lib.omp_learned_workspace_size(ctypes.byref(d0), ctypes.byref(fm), 100, 32, ctypes.byref(o)) == 0
    d2 = _fake_dict(256, 2048, prec=1)
    assert lib.omp_learned_workspace_size(ctypes.byref(d2), ctypes.byref(fm), 100, 32, ctypes.byref(o)) == 0
    acc = ctypes.c_int64(0)
    args = [FAKE, 100, 256, 32, 0.0, None, FAKE, FAKE, FAKE, FAKE, ctypes.byref(acc), ctypes.byref(o), FAKE,
            1 << 40, None]
    a = list(args)
    a[3] = 65
    assert lib.omp_learned_solve(ctypes.byref(d), ctypes.byref(fm), *a) == omp.OMP_ENOTSUPP
    a = list(args)
    a[4] = math.nan
    assert lib.omp_learned_solve(ctypes.byref(d), ctypes.byref(fm), *a) == omp.OMP_EINVAL
    a = list(args)
    a[13] = 1024
    assert lib.omp_learned_solve(ctypes.byref(d), ctypes.byref(fm), *a) == omp.OMP_EWORKSPACE
    assert lib.omp_learned_solve(ctypes.byref(d0), ctypes.byref(fm), *args) == omp.OMP_EINVAL


def test_noalloc_limits_checked_on_the_host(lib):
    """omp_solve_noalloc refuses, before any device work, a request whose workspace
    exceeds its static scratch (OMP_ENOTSUPP) and a timed call (OMP_EINVAL)."""
    from paper_2407_06434_amd import omp
    cap = lib.omp_noalloc_max_bytes()
    assert cap == 64 << 20
    o = _opts(ws=0)
    o.workspace = None
    M, N, B, S = 1024, 4096, 4096, 64
    assert lib.omp_workspace_size(M, N, B, S, ctypes.byref(o)) > cap
    rc = lib.omp_solve_noalloc(FAKE, M, N, M, FAKE, B, M, S, 0.0, None, FAKE, ctypes.byref(o), None)
    assert rc == omp.OMP_ENOTSUPP
    ms = (ctypes.c_float * omp.NPHASE)()
    o.phase_ms = ms
    rc = lib.omp_solve_noalloc(FAKE, 64, 256, 64, FAKE, 10, 64, 8, 0.0, None, FAKE, ctypes.byref(o), None)
    assert rc == omp.OMP_EINVAL
    assert lib.omp_solve_noalloc(FAKE, 64, 256, 64, FAKE, 10, 64, 8, 0.0, None, FAKE, None, None) == omp.OMP_EINVAL
