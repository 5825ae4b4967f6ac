"""Pins of the surrogate oracles: the network's FP64 backpropagation against
finite differences, the BF16 rounding against torch's conversion, Adam's first
step in closed form, the linear regime of the network, and the analytic
branch-wise model (paper Sec. 2.4, Eqs. (2) and (4)) in its special cases and
in the qualitative crisis behaviour the paper reports (Sec. 4.1)."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import analytic_oracle as A
from oracle import mlp_oracle as M


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(M.N_PARAM) * scale


def test_parameter_count():
    assert M.N_PARAM == 4609


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -0.0, 65504.0]]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(x), want)
    # ties go to even: 1 + 2^-8 is half-way between 1 and 1 + 2^-7
    assert M.bf16_round(np.float32(1.0 + 2.0 ** -8)) == 1.0
    assert M.bf16_round(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(2)
    p = _params(3)
    X = rng.standard_normal((16, 5))
    T = rng.standard_normal(16)
    _, g = M.loss_grad(p, X, T, weights_bf16=False)
    h = 1e-6
    idx = rng.choice(M.N_PARAM, 200, replace=False)
    fd = np.empty(len(idx))
    for k, i in enumerate(idx):
        e = np.zeros(M.N_PARAM)
        e[i] = h
        lp, _ = M.loss_grad(p + e, X, T, weights_bf16=False)
        lm, _ = M.loss_grad(p - e, X, T, weights_bf16=False)
        fd[k] = (lp - lm) / (2 * h)
    # ReLU kinks: skip the (rare) parameters whose finite difference straddles one
    ok = np.abs(fd - g[idx]) <= 1e-6 * (np.abs(g[idx]) + 1e-3)
    assert ok.mean() > 0.97
    assert np.median(np.abs(fd - g[idx]) / (np.abs(g[idx]) + 1e-12)) < 1e-7


def test_rounded_weights_gradient_is_straight_through():
    rng = np.random.default_rng(4)
    p = _params(5)
    X = rng.standard_normal((8, 5))
    T = rng.standard_normal(8)
    pr = M.unpack(p)
    for k in ("W1", "W2", "w3"):
        pr[k] = M.bf16_round(pr[k])
    a = M.loss_grad(p, X, T, weights_bf16=True)
    b = M.loss_grad(M.pack(pr), X, T, weights_bf16=False)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_linear_regime_is_a_matrix_product():
    """With every pre-activation positive the network is affine."""
    rng = np.random.default_rng(6)
    w = {"W1": rng.uniform(0.1, 0.5, (64, 5)), "b1": np.full(64, 1.0), "W2": rng.uniform(0.0, 0.1, (64, 64)),
         "b2": np.full(64, 0.5), "w3": rng.standard_normal(64), "b3": np.array([0.25])}
    X = rng.uniform(0.0, 1.0, (10, 5))
    y, _ = M.forward(M.pack(w), X, weights_bf16=False)
    direct = ((X @ w["W1"].T + w["b1"]) @ w["W2"].T + w["b2"]) @ w["w3"] + w["b3"][0]
    assert np.allclose(y, direct, rtol=1e-14, atol=1e-14)


def test_adam_first_step_moves_by_lr_times_sign():
    g = np.array([1e-3, -2.0, 5.0, -1e-6])
    p1, m, v = M.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-12)
    assert np.allclose(p1, -0.01 * np.sign(g), rtol=1e-5)


def test_cylinder_curve_values():
    # subcritical: White's correlation 1 + 10 Re^(-2/3)
    assert A.cylinder_cd(1000.0) == pytest.approx(1.1, rel=1e-6)
    assert A.cylinder_cd(8.0) == pytest.approx(3.5, rel=1e-6)
    # crisis: post-critical values well below the subcritical plateau
    assert A.cylinder_cd(2e6) < 0.5 < A.cylinder_cd(1e5)
    assert A.cylinder_cd(3e4, 0.08) < 0.5 < A.cylinder_cd(3e4, 0.0)


def test_single_normal_cylinder_reduces_to_its_drag_coefficient():
    """Eq. (4) with one branch normal to the flow and A_x = L D: C_D-est =
    C_d(Re_D); inclined by alpha it scales with sin^3(alpha); along the flow
    it vanishes."""
    L, D, H = 10.0, 1.0, 10.0
    for a_deg, fac in ((90.0, 1.0), (60.0, math.sin(math.radians(60.0)) ** 3), (0.0, 0.0)):
        a = math.radians(a_deg)
        b = np.array([[0.0, 0.0, 0.0, L * math.cos(a), 0.0, L * math.sin(a), D, 0, -1, 0]])
        c = A.tree_cd_est(b, [1e4, 1e6], H, L * D)
        want = A.cylinder_cd(np.array([1e4, 1e6]) * D / H) * fac
        assert np.allclose(c, want, rtol=1e-12, atol=1e-15)


def test_friction_estimate_of_a_hand_tree_with_a_constant_cf():
    """Eqs. (3), (5) with C_f = 0.3 at every Re_D on three branches: a vertical
    one (L D = 1, sin^3 = 1), one at 45 degrees to the flow (L = sqrt 2,
    D = 0.25, sin^3 = 2^(-3/2): L D sin^3 = 1/8) and one along the flow (no
    share); A_x = 2 gives 0.3 * 1.125 / 2."""
    b = np.array([_capsule((0, 0, 0), (0, 0, 2), 0.5), _capsule((0, 0, 2), (1, 0, 3), 0.25),
                  _capsule((0, 0, 2), (1.5, 0, 2), 0.2)])
    table = ([1.0, 2.0, 4.0], [0.3, 0.3, 0.3])
    got = A.tree_cf_est(b, [1e2, 1e5, 1e8], 3.0, 2.0, table)
    assert np.allclose(got, 0.16875, rtol=1e-13)


def test_friction_table_is_a_power_law_between_and_beyond_its_nodes():
    """A table sampled from C_f = 4 Re^(-1/2) reproduces that law everywhere,
    below and above its nodes too: one normal branch with A_x = L D and
    D / H = 1/10 gives C_F-est = 4 (Re_H / 10)^(-1/2): 4 at Re_H = 10,
    4 / sqrt(30) = 0.7302967433 at 300, 0.04 at 1e5.  A table with a kink
    (C_f = 1, 0.1, 0.1 at Re_D = 1, 10, 1000) takes the geometric mean
    sqrt(0.1) at Re_D = sqrt(10), stays at 0.1 above, and continues the first
    slope to 10 at Re_D = 0.1."""
    L, D, H = 10.0, 1.0, 10.0
    b = np.array([_capsule((0, 0, 0), (0, 0, L), D)])
    law = ([1.0, 2.0, 3.0], [4.0 / math.sqrt(10.0), 0.4, 4.0 / math.sqrt(1000.0)])
    got = A.tree_cf_est(b, [10.0, 300.0, 1e5], H, L * D, law)
    assert np.allclose(got, [4.0, 0.7302967433, 0.04], rtol=1e-9)
    kink = ([0.0, 1.0, 3.0], [1.0, 0.1, 0.1])
    got = A.cylinder_cf([math.sqrt(10.0), 100.0, 1e4, 0.1], *kink)
    assert np.allclose(got, [0.316227766, 0.1, 0.1, 10.0], rtol=1e-9)


def test_pressure_estimate_is_the_total_less_the_friction():
    """Eq. (6) on one normal branch at Re_D = 1000: C_D-est = 1.1 (the
    subcritical correlation), C_F-est = 4 / sqrt(1000) = 0.1264911064 from the
    power-law table, so C_P-est = 0.9735088936."""
    L, D, H = 10.0, 1.0, 10.0
    b = np.array([_capsule((0, 0, 0), (0, 0, L), D)])
    law = ([1.0, 2.0, 3.0], [4.0 / math.sqrt(10.0), 0.4, 4.0 / math.sqrt(1000.0)])
    got = A.tree_cp_est(b, [1e4], H, L * D, law)
    assert np.allclose(got, 0.9735088936, rtol=1e-7)


def test_crisis_of_the_paper_trees_starts_near_3e6_and_softens_with_n():
    """The paper finds the crisis near Re_H ~ 3e6 for every n and a less steep
    drop as the number of generations n grows (Sec. 4.1).  Onset here: the
    first Re_H where C_D-est falls 10 % below its value at Re_H = 1e5."""
    re = 10.0 ** np.linspace(4, 9, 201)
    slopes = []
    for n in (4, 6, 8):
        # the paper's n rewrites draw n generations (trunk and n - 1 child
        # levels), the reading that reproduces Table 3
        b = O.tree_generate(O.paper_tree_params(n - 1))
        c = A.tree_cd_est(b, re, O.tree_height(b), 1.0)
        ref = c[np.searchsorted(re, 1e5)]
        onset = re[np.argmax((re > 1e5) & (c < 0.9 * ref))]
        assert 1e6 < onset < 1e7
        s = np.diff(np.log(c)) / np.diff(np.log(re))
        slopes.append(-s.min())
    assert slopes[0] > slopes[1] > slopes[2]


def _capsule(p0, p1, d):
    """One branch record (rows of 10) from axis ends and diameter."""
    return [p0[0], p0[1], p0[2], p1[0], p1[1], p1[2], d, 0.0, -1.0, 0.0]


# Pixel counting misses at most the pixels the outline crosses: |error| below
# the perimeter times the pixel diagonal.
H_PIX = 1.0 / 1024


def _stadium(length, d):
    return length * d + math.pi * d * d / 4.0, 2.0 * length + math.pi * d


def test_projected_area_of_a_cross_flow_capsule_is_a_stadium():
    """A capsule whose axis lies in the (y, z) plane projects along x to the 2D
    stadium of area L D + pi D^2 / 4, at any orientation in that plane."""
    L, D = 0.5, 0.2
    want, per = _stadium(L, D)
    for ang in (0.0, 30.0, 90.0, 137.0):
        a = math.radians(ang)
        b = np.array([_capsule([0.3, 0.0, 0.0], [0.3, L * math.cos(a), L * math.sin(a)], D)])
        got = A.projected_area(b, H_PIX)
        assert abs(got - want) < per * H_PIX * math.sqrt(2.0)
        assert abs(got - want) < 2e-3 * want


def test_projected_area_of_a_streamwise_capsule_is_a_disc():
    """A capsule along the flow projects to the disc of its diameter; inclined
    by alpha to the flow, its projected axis shortens to L sin(alpha)."""
    L, D = 0.5, 0.2
    b = np.array([_capsule([0.0, 0.0, 0.0], [L, 0.0, 0.0], D)])
    disc = math.pi * D * D / 4.0
    assert abs(A.projected_area(b, H_PIX) - disc) < math.pi * D * H_PIX * math.sqrt(2.0)
    a = math.radians(40.0)
    b = np.array([_capsule([0.0, 0.0, 0.0], [L * math.cos(a), 0.0, L * math.sin(a)], D)])
    want, per = _stadium(L * math.sin(a), D)
    assert abs(A.projected_area(b, H_PIX) - want) < per * H_PIX * math.sqrt(2.0)


def test_projected_area_of_overlapping_capsules_is_their_union():
    """Two collinear capsules that overlap cover one longer stadium; two that
    cross at right angles through their midpoints cover both stadia less the
    D x D square they share (their round ends lie apart)."""
    L, D = 0.5, 0.1
    b = np.array([_capsule([0.0, 0.0, 0.0], [0.0, L, 0.0], D), _capsule([0.0, 0.3, 0.0], [0.0, 0.3 + L, 0.0], D)])
    want, per = _stadium(0.3 + L, D)
    assert abs(A.projected_area(b, H_PIX) - want) < per * H_PIX * math.sqrt(2.0)
    b = np.array([_capsule([0.0, -L / 2, 0.0], [0.0, L / 2, 0.0], D),
                  _capsule([0.0, 0.0, -L / 2], [0.0, 0.0, L / 2], D)])
    one, per = _stadium(L, D)
    want = 2.0 * one - D * D
    assert abs(A.projected_area(b, H_PIX) - want) < 2.0 * per * H_PIX * math.sqrt(2.0)


def _probe_network(kind):
    """Parameters whose output is known in closed form: 'const' gives y = 0.75
    for every input; 'lre' gives y = 0.5 + x0 / 4 with x0 the first (log10 Re_D)
    feature, which passes both ReLU layers unchanged while Re_D > 1."""
    w = {"W1": np.zeros((64, 5)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
         "w3": np.zeros(64), "b3": np.array([0.75])}
    if kind == "lre":
        w["W1"][0, 0] = 1.0
        w["W2"][0, 0] = 1.0
        w["w3"][0] = 0.25
        w["b3"][0] = 0.5
    return M.pack(w)


def _sweep_inputs():
    b = O.build_tree(O.seeded3_tree_params(2, 11), 1.0, [0.0, 0.0, 0.0])
    L, D, alpha, zmid = A.branch_geometry(b)
    fixed = np.column_stack([np.degrees(alpha), b[:, 7], zmid - b[0, 2]])
    return np.log10(D), L * D, fixed


def test_sweep_with_a_constant_network_is_its_value_times_the_summed_areas():
    """Inside the training range of Re_D the estimate is sum_b y_b L_b D_b / A_x
    (Eq. (4) with the network's coefficient): a constant y gives y sum L D / A."""
    lgd, w, fixed = _sweep_inputs()
    scale = (np.zeros(5), np.ones(5))
    area = 0.37
    re = np.array([2e3, 1e4])
    # every branch's Re_D = Re_H D / H inside [lo, hi] at both Re_H
    lo, hi = 10.0 ** (lgd.min() + math.log10(2e3) - 0.1), 10.0 ** (lgd.max() + 4.0 + 0.1)
    c = M.tree_cd_sweep(_probe_network("const"), scale, (0.0, 1.0), fixed, lgd, w, re, 0.0, lo, hi, area,
                        A.cylinder_cd)
    assert np.allclose(c, 0.75 * w.sum() / area, rtol=1e-12)
    # the output scale of the targets applies: y_mean + y_std * y
    c2 = M.tree_cd_sweep(_probe_network("const"), scale, (0.1, 2.0), fixed, lgd, w, re, 0.0, lo, hi, area,
                         A.cylinder_cd)
    assert np.allclose(c2, (0.1 + 2.0 * 0.75) * w.sum() / area, rtol=1e-12)


def test_sweep_outside_the_envelope_carries_the_cylinder_ratio():
    """A branch beyond the training range is evaluated at the clamped Re_D and
    scaled by C_d(Re_D) / C_d(Re_D,clamped): with y = 0.5 + log10(Re_D) / 4 the
    estimate is known per branch in closed form; it is continuous across both
    edges of the range and, far above it, follows the cylinder curve's crisis."""
    lgd, w, fixed = _sweep_inputs()
    scale = (np.zeros(5), np.ones(5))
    lo, hi = 30.0, 3000.0
    p = _probe_network("lre")
    for inten in (0.0, 0.08):
        re = 10.0 ** np.linspace(2.0, 8.0, 25)
        got = M.tree_cd_sweep(p, scale, (0.0, 1.0), fixed, lgd, w, re, inten, lo, hi, 1.0, A.cylinder_cd)
        for k, r in enumerate(re):
            lre = math.log10(r) + lgd
            lc = np.clip(lre, math.log10(lo), math.log10(hi))
            ratio = A.cylinder_cd(10.0 ** lre, inten) / A.cylinder_cd(10.0 ** lc, inten)
            # the inference form rounds the scaled features to BF16 before layer 1
            want = np.sum((0.5 + M.bf16_round(lc) / 4.0) * ratio * w)
            assert abs(got[k] - want) < 1e-12 * abs(want)
        # continuity across the edges: Re_H just below and above the point where
        # the trunk's Re_D meets each edge
        for edge in (lo, hi):
            r0 = edge / 10.0 ** lgd[0]
            a, b = M.tree_cd_sweep(p, scale, (0.0, 1.0), fixed, lgd, w, [r0 * (1 - 1e-9), r0 * (1 + 1e-9)], inten,
                                   lo, hi, 1.0, A.cylinder_cd)
            assert abs(a - b) < 1e-6 * abs(a)
