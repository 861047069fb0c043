"""Pins for the oracle's optimisation step (Sec. 3.3 entropy loss; the 3D
Gaussian Splatting optimiser conventions the paper follows).

* Adam equals torch.optim.Adam over several steps, per group, with the opacity
  optimised as a logit whose gradient is the render's times o (1 - o);
* the first Adam step moves each parameter by lr g / (|g| + eps) (bias
  correction makes m_hat = g, v_hat = g^2);
* the position rate interpolates geometrically: lr(0) = lr0, lr(steps) = lr1
  (and beyond), lr(steps / 2) = sqrt(lr0 lr1);
* the entropy -o ln o is largest at o = 1/e, where it equals 1/e and its
  gradient vanishes; it is 0 at o = 1; its gradient matches central
  differences;
* opacity reset caps o and clears the opacity moments.
"""
import math

import numpy as np
import torch

from oracle import training as T

CFG = {"lr_means_init": 1.6e-4, "lr_means_final": 1.6e-6, "lr_means_steps": 30000,
       "lr_log_scales": 5e-3, "lr_rotors": 1e-3, "lr_opacity": 0.05, "lr_sh_dc": 2.5e-3,
       "lr_sh_rest": 2.5e-3 / 20, "beta1": 0.9, "beta2": 0.999, "eps": 1e-15}


def _problem(n=50, k=4, seed=0):
    rng = np.random.default_rng(seed)
    p = {"means": rng.normal(size=(4, n)), "log_scales": rng.normal(-3, .5, size=(4, n)),
         "rotors": rng.normal(size=(8, n)), "opacity": rng.uniform(.05, .95, size=n),
         "sh": rng.normal(size=(3 * k, n))}
    return p, T.logit(p["opacity"])


def test_adam_matches_torch_optim():
    p, lg = _problem()
    cfg = dict(CFG, lr_means_final=CFG["lr_means_init"])    # constant rates for torch
    rng = np.random.default_rng(1)
    leaves = {k: torch.tensor(p[k] if k != "opacity" else lg, requires_grad=True)
              for k in T.GROUPS}
    groups = [{"params": [leaves["means"]], "lr": cfg["lr_means_init"]},
              {"params": [leaves["log_scales"]], "lr": cfg["lr_log_scales"]},
              {"params": [leaves["rotors"]], "lr": cfg["lr_rotors"]},
              {"params": [leaves["opacity"]], "lr": cfg["lr_opacity"]}]
    sh_dc = torch.tensor(p["sh"][:3], requires_grad=True)
    sh_rest = torch.tensor(p["sh"][3:], requires_grad=True)
    groups += [{"params": [sh_dc], "lr": cfg["lr_sh_dc"]},
               {"params": [sh_rest], "lr": cfg["lr_sh_rest"]}]
    opt = torch.optim.Adam(groups, betas=(cfg["beta1"], cfg["beta2"]), eps=cfg["eps"])
    m = {k: np.zeros_like(p[k]) for k in T.GROUPS}
    v = {k: np.zeros_like(p[k]) for k in T.GROUPS}
    cur, cur_l = p, lg
    for step in range(6):
        g = {k: rng.normal(size=p[k].shape) * (10.0 ** rng.uniform(-3, 1)) for k in T.GROUPS}
        o = T.sigmoid(leaves["opacity"].detach().numpy())
        for k in ("means", "log_scales", "rotors"):
            leaves[k].grad = torch.tensor(g[k])
        leaves["opacity"].grad = torch.tensor(g["opacity"] * o * (1 - o))
        sh_dc.grad = torch.tensor(g["sh"][:3])
        sh_rest.grad = torch.tensor(g["sh"][3:])
        opt.step()
        cur, cur_l, m, v = T.adam_step(cur, cur_l, g, m, v, step, cfg)
        for k in ("means", "log_scales", "rotors"):
            assert np.abs(cur[k] - leaves[k].detach().numpy()).max() < 1e-12
        assert np.abs(cur_l - leaves["opacity"].detach().numpy()).max() < 1e-12
        assert np.abs(cur["opacity"] - T.sigmoid(cur_l)).max() < 1e-15
        sh = np.concatenate([sh_dc.detach().numpy(), sh_rest.detach().numpy()])
        assert np.abs(cur["sh"] - sh).max() < 1e-12


def test_first_step_is_signed_rate():
    p, lg = _problem(seed=2)
    g = {k: np.random.default_rng(3).normal(size=p[k].shape) for k in T.GROUPS}
    z = {k: np.zeros_like(p[k]) for k in T.GROUPS}
    cfg = dict(CFG, eps=1e-8)
    out, _, _, _ = T.adam_step(p, lg, g, z, z, 0, cfg)
    lr = CFG["lr_log_scales"]
    gs = g["log_scales"]
    assert np.abs((p["log_scales"] - out["log_scales"]) - lr * gs / (np.abs(gs) + 1e-8)).max() < 1e-15
    # SH: degree-0 rows at the DC rate, the rest at the other rate
    d = p["sh"] - out["sh"]
    gsh = g["sh"]
    assert np.abs(d[:3] - CFG["lr_sh_dc"] * gsh[:3] / (np.abs(gsh[:3]) + 1e-8)).max() < 1e-15
    assert np.abs(d[3:] - CFG["lr_sh_rest"] * gsh[3:] / (np.abs(gsh[3:]) + 1e-8)).max() < 1e-15


def test_position_rate_schedule():
    a, b, s = 1.6e-4, 1.6e-6, 30000
    assert T.position_lr(0, a, b, s) == a
    assert abs(T.position_lr(s, a, b, s) - b) < 1e-18
    assert abs(T.position_lr(3 * s, a, b, s) - b) < 1e-18
    assert abs(T.position_lr(s // 2, a, b, s) - math.sqrt(a * b)) < 1e-15


def test_entropy_loss():
    o = torch.full((7,), 1 / math.e, dtype=torch.float64, requires_grad=True)
    L = T.entropy_loss(o)
    assert abs(float(L.detach()) - 1 / math.e) < 1e-15
    L.backward()
    assert float(o.grad.abs().max()) < 1e-15
    assert float(T.entropy_loss(torch.ones(3, dtype=torch.float64))) == 0.0
    rng = np.random.default_rng(4)
    x = rng.uniform(0.01, 0.99, 20)
    t = torch.tensor(x, requires_grad=True)
    T.entropy_loss(t).backward()
    for i in range(0, 20, 3):
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (float(T.entropy_loss(torch.tensor(xp))) - float(T.entropy_loss(torch.tensor(xm)))) / (2 * h)
        assert abs(fd - float(t.grad[i])) < 1e-8


def test_opacity_reset():
    lg = T.logit(np.array([0.5, 0.005, 0.01, 0.9]))
    m = np.ones(4)
    lnew, o, m2, v2 = T.opacity_reset(lg, m, m, 0.01)
    assert np.allclose(o, [0.01, 0.005, 0.01, 0.01], rtol=1e-14, atol=0)
    assert np.allclose(T.sigmoid(lnew), o, rtol=1e-13, atol=0)
    assert not m2.any() and not v2.any()


DCFG = {"grad_threshold": 2e-4, "size_threshold": 0.05, "min_opacity": 0.005, "max_size": 0.0}


def _dstate(n, seed=5, k=4):
    rng = np.random.default_rng(seed)
    f = np.float32
    p = {"means": rng.uniform(-1, 1, (4, n)).astype(f),
         "log_scales": rng.normal(-3.5, 0.5, (4, n)).astype(f),
         "rotors": rng.normal(size=(8, n)).astype(f),
         "opacity": rng.uniform(0.01, 0.99, n).astype(f),
         "sh": rng.normal(size=(3 * k, n)).astype(f)}
    m = {key: rng.normal(size=p[key].shape) for key in T.GROUPS}
    v = {key: rng.uniform(size=p[key].shape) for key in T.GROUPS}
    return p, T.logit(p["opacity"].astype(np.float64)).astype(f), m, v


def test_densify_hand_case():
    p, lg, m, v = _dstate(4)
    p["log_scales"][:3, :] = np.log(0.02)           # small ...
    p["log_scales"][:3, 2] = np.log(0.2)            # ... except #2
    p["opacity"][3] = 0.001                         # #3 below the prune threshold
    accum = np.array([1e-4, 9e-4, 9e-4, 9e-4], dtype=np.float32)
    count = np.array([1, 3, 3, 3])
    z = np.random.default_rng(6).normal(size=(4, 8))
    out, ol, om, ov = T.densify(p, lg, m, v, accum, count, z, DCFG)
    # kept: 0, 1 (2 split, 3 pruned); clones: 1; children: 2, 2
    assert out["opacity"].shape == (5,)
    src = [0, 1, 1, 2, 2]
    for key in ("rotors", "opacity", "sh"):
        assert np.array_equal(out[key], p[key][..., src])
    assert np.array_equal(out["means"][:, :3], p["means"][:, [0, 1, 1]])
    assert np.array_equal(out["log_scales"][:, :3], p["log_scales"][:, [0, 1, 1]])
    shrink = np.float32(math.log(1.6))
    assert np.array_equal(out["log_scales"][:, 3:], np.repeat((p["log_scales"][:, 2:3] - shrink), 2, 1))
    assert np.array_equal(ol, lg[src])
    for key in T.GROUPS:
        assert np.array_equal(om[key][..., :2], m[key][..., :2])
        assert not om[key][..., 2:].any() and not ov[key][..., 2:].any()
    # children at mu + R diag(s) z with the parent's (unshrunk) scales
    from oracle import render as O
    R = O.rotor_to_matrix(O.rotor_normalize(torch.tensor(p["rotors"][:, 2:3].T.astype(np.float64)))).numpy()[0]
    s = np.exp(p["log_scales"][:, 2].astype(np.float64))
    for c in range(2):
        want = p["means"][:, 2].astype(np.float64) + R @ (s * z[:, 4 + c])
        assert np.abs(out["means"][:, 3 + c] - want).max() < 1e-6


def test_split_children_follow_the_4d_covariance():
    """Children of many copies of one Gaussian sample N(mu, Sigma_4)."""
    p, lg, m, v = _dstate(1, seed=7)
    p["log_scales"][:, 0] = np.log([0.3, 0.1, 0.2, 0.4])
    n = 3000
    P = {key: np.repeat(p[key], n, axis=-1) for key in T.GROUPS}
    M = {key: np.zeros_like(P[key], dtype=np.float64) for key in T.GROUPS}
    z = np.random.default_rng(8).normal(size=(4, 2 * n))
    out, _, _, _ = T.densify(P, np.repeat(lg, n), M, M, np.ones(n, np.float32), np.ones(n), z, DCFG)
    x = out["means"].astype(np.float64)
    assert x.shape == (4, 2 * n)
    from oracle import render as O
    r = O.rotor_normalize(torch.tensor(p["rotors"][:, :1].T.astype(np.float64)))
    S4 = O.covariance_4d(O.rotor_to_matrix(r), torch.tensor(p["log_scales"][:, :1].T.astype(np.float64)))[0].numpy()
    C = np.cov(x)
    assert np.abs(C - S4).max() < 0.08 * np.abs(S4).max()
    assert np.abs(x.mean(1) - p["means"][:, 0]).max() < 0.05


def test_prune_by_size():
    p, lg, m, v = _dstate(3, seed=9)
    p["log_scales"][:3] = np.log(0.01)
    p["log_scales"][1, 1] = np.log(0.5)
    out, _, _, _ = T.densify(p, lg, m, v, np.zeros(3, np.float32), np.zeros(3), np.zeros((4, 6)),
                             dict(DCFG, max_size=0.3))
    assert np.array_equal(out["opacity"], p["opacity"][[0, 2]])
