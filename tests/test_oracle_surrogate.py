"""Pins for the pre-screen oracle (CPU only): BF16 rounding on known values,
finite-difference gradients of the network and the loss (rounding off),
closed forms of the loss and of Adam's first step, and invariance of the
prediction under atom relabelling."""
import math

import numpy as np
import pytest

import synth
from oracle import surrogate as S


def test_bf16_rounding_known_values():
    one = 1.0
    ulp = 2.0 ** -7                    # bfloat16 spacing at 1
    assert S.bf16(one) == one
    assert S.bf16(one + ulp / 2) == one                 # tie -> even (1.0)
    assert S.bf16(one + 3 * ulp / 2) == one + 2 * ulp   # tie -> even (1 + 2 ulp)
    assert S.bf16(one + 0.6 * ulp) == one + ulp
    assert S.bf16(-one - 0.4 * ulp) == -one
    assert S.bf16(3.14159265) == 3.140625
    assert S.bf16(0.0) == 0.0


def graphs(seeds, n_range=(5, 30)):
    rng = np.random.default_rng(sum(seeds))
    out = []
    for s in seeds:
        lig = synth.ligand(s, int(rng.integers(*n_range)), int(rng.integers(0, 6)))
        out.append(S.features(lig))
    return out


def test_feature_layout():
    lig = synth.ligand(3, 12, 3)
    X, nbr = S.features(lig)
    assert X.shape == (12, 32)
    assert np.all(X[:, :16].sum(axis=1) == 1) and np.all(X[:, 18:23].sum(axis=1) == 1)
    assert np.all(X[:, 31] == 1)
    assert np.allclose(X[:, 16], lig.charges) and np.allclose(X[:, 17], np.abs(lig.charges))
    assert X[:, 23].sum() == lig.n_torsions          # each torsion counted at both ends, halved
    assert sum(len(n) for n in nbr) == 2 * (lig.n_atoms - 1)


def test_network_gradient_matches_finite_differences():
    theta = S.init_params(1) * 0.5
    rng = np.random.default_rng(2)
    theta += rng.normal(0, 0.01, size=theta.shape)   # nonzero biases
    G = graphs([11, 12, 13])
    dp = rng.normal(size=3)
    grad, p = S.backward(theta, G, dp, bf16_on=False)
    idx = rng.choice(S.N_PARAMS, size=60, replace=False)
    # make sure every tensor is probed
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in S.PARAM_SHAPES])
    idx = np.concatenate([idx, offs[:-1]])
    h = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (dp @ S.forward(tp, G, False) - dp @ S.forward(tm, G, False)) / (2 * h)
        assert fd == pytest.approx(grad[k], rel=1e-5, abs=1e-8), k


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    p = rng.normal(size=9)
    y = rng.normal(size=9)
    L, dp = S.loss_and_dp(p, y)
    for i in range(9):
        e = np.zeros(9)
        e[i] = 1e-6
        fd = (S.loss_and_dp(p + e, y)[0] - S.loss_and_dp(p - e, y)[0]) / 2e-6
        assert fd == pytest.approx(dp[i], rel=1e-6, abs=1e-9)


def test_loss_closed_forms():
    # two items, item 0 better: MSE + softplus((p0 - p1)/tau)
    p, y = np.array([0.3, -0.2]), np.array([-1.0, 1.0])
    L, _ = S.loss_and_dp(p, y)
    mse = ((0.3 + 1.0) ** 2 + (-0.2 - 1.0) ** 2) / 2
    assert L == pytest.approx(mse + math.log1p(math.exp((0.3 + 0.2) / S.TAU)), rel=1e-12)
    # ties in the labels give no ranking pairs
    L2, dp2 = S.loss_and_dp(np.array([1.0, 2.0]), np.array([0.5, 0.5]))
    assert L2 == pytest.approx(((0.5) ** 2 + 1.5 ** 2) / 2) and dp2 == pytest.approx([0.5, 1.5])


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th, m, v = S.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1)
    lr, eps = S.ADAM["lr"], S.ADAM["eps"]
    assert np.allclose(th, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)


def test_zero_weights_predict_the_output_bias():
    d = S.unflatten(np.zeros(S.N_PARAMS))
    d["c3"] = np.array([1.75])
    p = S.forward(S.flatten(d), graphs([5, 6]))
    assert np.all(p == 1.75)


def test_prediction_is_invariant_under_atom_relabelling():
    theta = S.init_params(3)
    lig = synth.ligand(21, 25, 5)
    rng = np.random.default_rng(0)
    lig2 = synth.permute(lig, rng.permutation(lig.n_atoms), rng.permutation(len(lig.bonds)), rng)
    p1 = S.forward(theta, [S.features(lig)], bf16_on=False)
    p2 = S.forward(theta, [S.features(lig2)], bf16_on=False)
    assert p1[0] == pytest.approx(p2[0], rel=1e-12)


def _emul_setup(n=12, seed=3):
    rng = np.random.default_rng(seed)
    ligs = [synth.ligand(700 + i, int(rng.integers(2, 60)), 3) for i in range(n)]
    G = [S.features(l) for l in ligs]
    theta = S.init_params(4) + rng.normal(0, 0.02, S.N_PARAMS)
    ys = rng.normal(0, 1, n)
    return G, theta, ys


def test_fp32_emulation_is_the_same_function():
    """Without BF16 rounding the float32 emulation and the FP64 oracle differ
    only by float32 accumulation (a dropped term, a wrong operand or a missed
    mask would show as a difference of order one)."""
    G, theta, ys = _emul_setup()
    po = S.forward(theta, G, bf16_on=False)
    Lo, dpo = S.loss_and_dp(po, ys)
    go, _ = S.backward(theta, G, dpo, bf16_on=False)
    for seed in (0, 1):
        p, L, g = S.emulate_fp32(theta, G, ys, seed=seed, bf16_on=False)
        assert np.linalg.norm(p - po) <= 1e-5 * np.linalg.norm(po)
        assert abs(L - Lo) <= 1e-5 * abs(Lo)
        assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)


def test_fp32_emulation_with_rounding_stays_near_the_oracle():
    """With BF16 rounding the emulation sits on other sides of a few rounding
    midpoints than the oracle: its results differ at the level of BF16 flips
    (well below a BF16 ulp of the predictions' scale normwise), and a seed
    fixes the order (reproducible)."""
    G, theta, ys = _emul_setup()
    po = S.forward(theta, G, bf16_on=True)
    Lo, dpo = S.loss_and_dp(po, ys)
    go, _ = S.backward(theta, G, dpo, bf16_on=True)
    p, L, g = S.emulate_fp32(theta, G, ys, seed=5)
    p2, L2, g2 = S.emulate_fp32(theta, G, ys, seed=5)
    assert np.array_equal(p, p2) and L == L2 and np.array_equal(g, g2)
    assert np.linalg.norm(p - po) <= 2 ** -8 * np.linalg.norm(po)
    assert np.linalg.norm(g - go) <= 2 ** -5 * np.linalg.norm(go)
