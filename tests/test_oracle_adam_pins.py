"""Pins of the oracle's Adam step (textbook bias-corrected Adam, Kingma & Ba
Alg. 1; the optimizer stage that visibility cropping relieves, Sec. 3.3):
closed forms of the first step and of a constant gradient, torch.optim.Adam
in float64, the visible-only variant and the zero-gradient fixed point."""
import numpy as np
import torch

import oracle

ROWS = dict(means=3, log_scales=3, quats=4, opacity_logits=1, sh=48)
LR = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 2.5e-3 / 20)


def planes(rng, n, scale=1.0):
    return {k: rng.normal(0.0, scale, (r, n)) for k, r in ROWS.items()}


def rate_rows(k):
    if k == "sh":
        r = np.full((48, 1), LR[5])
        r[:3] = LR[4]
        return r
    return np.full((ROWS[k], 1), LR[oracle.ADAM_GROUPS.index(k)])


def zeros_like(d):
    return {k: np.zeros_like(v) for k, v in d.items()}


def test_first_step_is_lr_times_normalised_gradient():
    rng = np.random.default_rng(1)
    p, g = planes(rng, 9), planes(rng, 9)
    eps = 1e-8
    P, M, V = oracle.adam_step(p, g, zeros_like(p), zeros_like(p), LR, 0.9, 0.999, eps, 1)
    for k in ROWS:
        want = p[k] - rate_rows(k) * g[k] / (np.abs(g[k]) + eps)
        assert np.allclose(P[k], want, rtol=1e-13, atol=1e-16)
        assert np.allclose(M[k], 0.1 * g[k], rtol=1e-14)
        assert np.allclose(V[k], 0.001 * g[k] ** 2, rtol=1e-13)


def test_constant_gradient_moves_by_lr_each_step():
    rng = np.random.default_rng(2)
    p, g = planes(rng, 5), planes(rng, 5)
    m, v = zeros_like(p), zeros_like(p)
    cur = p
    for t in range(1, 6):
        cur, m, v = oracle.adam_step(cur, g, m, v, LR, 0.9, 0.99, 1e-12, t)
        for k in ROWS:
            # bias correction makes m^ = g and v^ = g^2 exactly for a constant g
            assert np.allclose(cur[k], p[k] - t * rate_rows(k) * g[k] / (np.abs(g[k]) + 1e-12),
                               rtol=1e-11, atol=1e-14)


def test_matches_torch_adam_in_float64():
    rng = np.random.default_rng(3)
    n = 11
    p0 = planes(rng, n)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p0.items()}
    groups = [dict(params=[tp[k]], lr=LR[i]) for i, k in enumerate(("means", "log_scales", "quats",
                                                                  "opacity_logits"))]
    sh_dc = torch.tensor(p0["sh"][:3], dtype=torch.float64, requires_grad=True)
    sh_rest = torch.tensor(p0["sh"][3:], dtype=torch.float64, requires_grad=True)
    groups += [dict(params=[sh_dc], lr=LR[4]), dict(params=[sh_rest], lr=LR[5])]
    opt = torch.optim.Adam(groups, betas=(0.9, 0.999), eps=1e-15)
    cur, m, v = p0, zeros_like(p0), zeros_like(p0)
    for t in range(1, 8):
        g = planes(rng, n, scale=10.0 ** rng.uniform(-6, 1))
        for k in ("means", "log_scales", "quats", "opacity_logits"):
            tp[k].grad = torch.tensor(g[k])
        sh_dc.grad = torch.tensor(g["sh"][:3])
        sh_rest.grad = torch.tensor(g["sh"][3:])
        opt.step()
        cur, m, v = oracle.adam_step(cur, g, m, v, LR, 0.9, 0.999, 1e-15, t)
    for k in ("means", "log_scales", "quats", "opacity_logits"):
        assert np.allclose(cur[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-15)
    assert np.allclose(cur["sh"], np.concatenate([sh_dc.detach().numpy(), sh_rest.detach().numpy()]),
                       rtol=1e-12, atol=1e-15)


def test_visible_only_leaves_unseen_gaussians_untouched():
    rng = np.random.default_rng(4)
    n = 20
    p, g, m, v = planes(rng, n), planes(rng, n), planes(rng, n), planes(rng, n)
    v = {k: np.abs(x) for k, x in v.items()}
    vis = (rng.random(n) < 0.5).astype(np.uint32)
    Pd, Md, Vd = oracle.adam_step(p, g, m, v, LR, 0.9, 0.999, 1e-15, 3)
    Ps, Ms, Vs = oracle.adam_step(p, g, m, v, LR, 0.9, 0.999, 1e-15, 3, visible=vis)
    on = vis != 0
    for k in ROWS:
        assert np.array_equal(Ps[k][:, ~on], p[k][:, ~on])
        assert np.array_equal(Ms[k][:, ~on], m[k][:, ~on]) and np.array_equal(Vs[k][:, ~on], v[k][:, ~on])
        assert np.array_equal(Ps[k][:, on], Pd[k][:, on]) and np.array_equal(Ms[k][:, on], Md[k][:, on])


def test_zero_gradient_and_moments_is_a_fixed_point():
    rng = np.random.default_rng(5)
    p = planes(rng, 6)
    z = zeros_like(p)
    P, M, V = oracle.adam_step(p, z, z, z, LR, 0.9, 0.999, 1e-15, 1)
    for k in ROWS:
        assert np.array_equal(P[k], p[k]) and not M[k].any() and not V[k].any()
