"""The learned-proposal oracle against its pins, and planted mistakes against the pins (CPU only)."""
import importlib.util
import os

import pytest

from tests.learned_pins import PINS

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "learned_oracle.py")


def _load(path, name):
    spec = importlib.util.spec_from_file_location(name, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_learned_oracle_pin(pin):
    from oracle import learned_oracle
    pin(learned_oracle)


MUTATIONS = {
    "no_relu_mask_in_backward": ("dh2 = rnd((dz @ rnd(params[\"W3\"])) * (c[\"h2\"] > 0))",
                                 "dh2 = rnd((dz @ rnd(params[\"W3\"])))"),
    "weight_not_transposed_in_backward": ("dh1 = rnd((dh2 @ rnd(params[\"W2\"])) * (c[\"h1\"] > 0))",
                                          "dh1 = rnd((dh2 @ rnd(params[\"W2\"]).T) * (c[\"h1\"] > 0))"),
    "gradient_sign": ("dz = rnd((sigmoid(z) - T) / B)", "dz = rnd((T - sigmoid(z)) / B)"),
    "loss_not_averaged": ("return float(np.sum(softplus(z) - T * z) / z.shape[0])",
                          "return float(np.sum(softplus(z) - T * z))"),
    "bias_grad_wrong_axis": ("g[\"b2\"] = dh2.sum(axis=0)", "g[\"b2\"] = dh2.sum(axis=1)[: dh2.shape[1]]"),
    "no_bias_correction": ("mh = m / (1 - beta1 ** t)", "mh = m"),
    "adam_second_moment_unsquared": ("(1 - beta2) * gk * gk", "(1 - beta2) * np.abs(gk)"),
    "bf16_truncates": ("u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000", "u = u & 0xFFFF0000"),
    "features_no_atom_norm": ("return np.sqrt(A.shape[1]) * np.abs(C) * inv_a[None, :] * inv_y[:, None]",
                              "return np.sqrt(A.shape[1]) * np.abs(C) * inv_y[:, None]"),
    "features_signed": ("return np.sqrt(A.shape[1]) * np.abs(C) * inv_a[None, :] * inv_y[:, None]",
                        "return np.sqrt(A.shape[1]) * C * inv_a[None, :] * inv_y[:, None]"),
    "top_s_ties_high": ("key=lambda n: (-scores[b, n], n)", "key=lambda n: (-scores[b, n], -n)"),
    "ls_residual_wrong": ("rn[b] = np.linalg.norm(Y[b] - AP @ X[b])", "rn[b] = np.linalg.norm(Y[b])"),
    "first_layer_skips_bias": ("a1 = x0 @ rnd(params[\"W1\"]).T + params[\"b1\"]", "a1 = x0 @ rnd(params[\"W1\"]).T"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_learned_mutant_fails_a_pin(tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/present: {name}"
    path = tmp_path / "mutant.py"
    path.write_text(src.replace(old, new))
    mod = _load(str(path), "learned_mutant_" + name)
    failed = []
    for pin in PINS:
        try:
            pin(mod)
        except (AssertionError, ValueError, IndexError):
            failed.append(pin.__name__)
    assert failed, f"mutation {name} passed every pin"
