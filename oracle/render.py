"""FP64 CPU oracle for the 4D-rotor Gaussian splatting render path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke entry point and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library: it is a plain, slow, float64 PyTorch-CPU restatement of the
paper's equations, so that torch autograd yields the reference gradient.

Pipeline per render (view, time t), in the paper's order:
  1. rotor normalisation F_norm            (App. A "4D Rotor Normalization")
  2. rotor -> 4x4 rotation F_map           (App. A "4D Rotor to Rotation Matrix")
  3. Sigma_4 = R S S^T R^T                 (Sec. 3.2.1, covariance factorisation)
  4. temporal slice: lambda = 1/W, Sigma_3D = U - V V^T / W,
     mu(t) = mu_xyz + (t - mu_t) V / W, opacity decay exp(-lambda dt^2 / 2),
     visibility cull lambda dt^2 > tau      (Sec. 3.2.2, Eq. center-motion;
                                             App. A "Temporally-Slicing")
  5. view transform, near cull, EWA projection Sigma' = J W Sigma W^T J^T
                                            (Sec. 3.1, 3DGS preliminary)
  6. spherical-harmonic colour              (Sec. 3.1)
  7. depth-ordered alpha compositing        (Sec. 3.1, blending equation)
  (optional) speed field: each Gaussian's speed V/W at time t (Sec. 3.2.2,
     the motion speed of the slice) moved through the projection gives its
     2D flow d(mean2d)/dt, composited like a colour with zero background
     (the rendered optical flow of the paper's flow figure)

Readings where the paper is silent or inconsistent (all listed in the design
notes): the rotor storage order is the main-text one; epsilon uses the sign of
the first statement of the normalisation condition (the summary restatement in
App. A flips two signs and does not give a rotation); delta is evaluated in
its rationalised form -2 eps / (l^2 + sqrt(l^4 - 4 eps^2)); scales are passed
as logarithms; the 3DGS conventions (near plane, guard band, 0.3 dilation,
SH offset 0.5 with clamp at 0, alpha skip / clamp / stop rules, 3-sigma
per-pixel extent) are parameters.

Every pixel is composited over *all* surviving Gaussians in one global stable
depth order (ties by Gaussian index); there are no tiles.
"""
from __future__ import annotations

import math

import numpy as np
import torch

DT = torch.float64

# Rotor component order (Sec. 3.2.1): s, b01, b02, b12, b03, b13, b23, p.
ROTOR_NAMES = ("s", "b01", "b02", "b12", "b03", "b13", "b23", "p")


def _to64(a):
    if isinstance(a, torch.Tensor):
        return a.to(DT)
    return torch.as_tensor(np.asarray(a), dtype=DT)


# ---------------------------------------------------------------------------
# App. A: rotor normalisation F_norm


def rotor_epsilon(r: torch.Tensor) -> torch.Tensor:
    """First normalisation condition: the e0123 part of r r^dagger over 2,
    eps = p s - b01 b23 + b02 b13 - b03 b12 (App. A, definition of epsilon)."""
    s, b01, b02, b12, b03, b13, b23, p = r.unbind(-1)
    return p * s - b01 * b23 + b02 * b13 - b03 * b12


def rotor_epsilon_gradient(r: torch.Tensor) -> torch.Tensor:
    """Gradient of eps w.r.t. the 8 components, in storage order (App. A)."""
    s, b01, b02, b12, b03, b13, b23, p = r.unbind(-1)
    return torch.stack([p, -b23, b13, -b03, -b12, b02, -b01, s], dim=-1)


def rotor_normalize(r: torch.Tensor) -> torch.Tensor:
    """F_norm: one root-finding step along grad(eps) to reach eps = 0, then divide
    by the Euclidean norm (App. A).  r: [..., 8].

    delta solves eps(r + delta grad eps) = eps (1 + delta^2) + l^2 delta = 0 with
    the root that tends to 0; written in the rationalised form.  A rotor whose
    squared norm is below 1e-12 before or after the update maps to the identity,
    with zero gradient.  (The updated norm is |r + delta grad eps|^2 =
    (l^4 - 4 eps^2) / l^2, so a zero discriminant always takes that branch.)
    """
    eps = rotor_epsilon(r)
    l2 = (r * r).sum(-1)
    disc = torch.clamp(l2 * l2 - 4.0 * eps * eps, min=0.0)
    # sqrt(disc), with a finite derivative where disc = 0 (there the update
    # lands on 0, see below, and the identity is returned)
    pos = disc > 0
    root = torch.where(pos, torch.sqrt(torch.where(pos, disc, torch.ones_like(disc))),
                       torch.zeros_like(disc))
    denom = l2 + root
    safe = denom > 1e-300
    delta = torch.where(safe, -2.0 * eps / torch.where(safe, denom, torch.ones_like(denom)),
                        torch.zeros_like(denom))
    r1 = r + delta[..., None] * rotor_epsilon_gradient(r)
    n2 = (r1 * r1).sum(-1)
    ok = (l2 >= 1e-12) & (n2 >= 1e-12)
    out = r1 / torch.sqrt(torch.where(ok, n2, torch.ones_like(n2)))[..., None]
    ident = torch.zeros_like(r)
    ident[..., 0] = 1.0
    return torch.where(ok[..., None], out, ident)


# ---------------------------------------------------------------------------
# App. A: rotor -> rotation matrix F_map


def rotor_to_matrix(r: torch.Tensor) -> torch.Tensor:
    """F_map: the 16 quadratic forms of App. A giving R with u' = R u = r u r^dagger.
    r: [..., 8] normalised; returns [..., 4, 4] (row index first)."""
    s, b01, b02, b12, b03, b13, b23, p = r.unbind(-1)
    R00 = -b01**2 - b02**2 - b03**2 + b12**2 + b13**2 + b23**2 - p**2 + s**2
    R01 = 2 * (b01 * s - b02 * b12 - b03 * b13 + b23 * p)
    R02 = 2 * (b01 * b12 + b02 * s - b03 * b23 - b13 * p)
    R03 = 2 * (b01 * b13 + b02 * b23 + b03 * s + b12 * p)
    R10 = 2 * (-b01 * s - b02 * b12 - b03 * b13 - b23 * p)
    R11 = -b01**2 + b02**2 + b03**2 - b12**2 - b13**2 + b23**2 - p**2 + s**2
    R12 = 2 * (-b01 * b02 + b03 * p + b12 * s - b13 * b23)
    R13 = 2 * (-b01 * b03 - b02 * p + b12 * b23 + b13 * s)
    R20 = 2 * (b01 * b12 - b02 * s - b03 * b23 + b13 * p)
    R21 = 2 * (-b01 * b02 - b03 * p - b12 * s - b13 * b23)
    R22 = b01**2 - b02**2 + b03**2 - b12**2 + b13**2 - b23**2 - p**2 + s**2
    R23 = 2 * (b01 * p - b02 * b03 - b12 * b13 + b23 * s)
    R30 = 2 * (b01 * b13 + b02 * b23 - b03 * s - b12 * p)
    R31 = 2 * (-b01 * b03 + b02 * p + b12 * b23 - b13 * s)
    R32 = 2 * (-b01 * p - b02 * b03 - b12 * b13 - b23 * s)
    R33 = b01**2 + b02**2 - b03**2 + b12**2 - b13**2 - b23**2 - p**2 + s**2
    rows = [torch.stack(row, dim=-1) for row in (
        (R00, R01, R02, R03), (R10, R11, R12, R13), (R20, R21, R22, R23), (R30, R31, R32, R33))]
    return torch.stack(rows, dim=-2)


# ---------------------------------------------------------------------------
# Sec. 3.2.1 covariance factorisation and Sec. 3.2.2 temporal slicing


def covariance_4d(R: torch.Tensor, log_scales: torch.Tensor) -> torch.Tensor:
    """Sigma_4 = R S S^T R^T with S = diag(exp(log s)) (Sec. 3.2.1).
    R: [n,4,4], log_scales: [n,4]."""
    s = torch.exp(log_scales)
    RS = R * s[:, None, :]
    return RS @ RS.transpose(-1, -2)


def slice_at_time(mu4: torch.Tensor, cov4: torch.Tensor, t: float):
    """Temporal slice (Sec. 3.2.2; App. A, Schur-complement form).

    Blocks Sigma_4 = [[U, V], [V^T, W]]; lambda = 1/W; the 3D Gaussian at time t
    has mean mu_xyz + (t - mu_t) V / W, covariance U - V V^T / W and its density is
    scaled by exp(-lambda (t - mu_t)^2 / 2).
    Returns (mu3 [n,3], cov3 [n,3,3], lam_dt2 [n], decay [n]).
    """
    U = cov4[:, :3, :3]
    V = cov4[:, :3, 3]
    W = cov4[:, 3, 3]
    lam = 1.0 / W
    dt = t - mu4[:, 3]
    mu3 = mu4[:, :3] + (dt / W)[:, None] * V
    cov3 = U - V[:, :, None] * V[:, None, :] / W[:, None, None]
    lam_dt2 = lam * dt * dt
    decay = torch.exp(-0.5 * lam_dt2)
    return mu3, cov3, lam_dt2, decay


# ---------------------------------------------------------------------------
# Sec. 3.1: EWA projection (3DGS conventions)


def project_ewa(mu3: torch.Tensor, cov3: torch.Tensor, view: dict, st: dict):
    """Camera-space position, 2D mean, depth and 2D covariance of each 3D Gaussian.

    Sigma' = J Wv Sigma Wv^T J^T (Sec. 3.1), with Wv the world-to-camera rotation
    and J the Jacobian of the pinhole projection at the Gaussian's camera-space
    centre, whose x/z and y/z are clamped to guard_band * (half image) / focal
    before use; dilation * I is added to the 2D covariance.
    """
    w2c = _to64(view["world_to_cam"]).reshape(3, 4)
    Rw, tw = w2c[:, :3], w2c[:, 3]
    pc = mu3 @ Rw.T + tw
    px, py, pz = pc.unbind(-1)
    fx, fy = float(view["fx"]), float(view["fy"])
    cx, cy = float(view["cx"]), float(view["cy"])
    limx = st["guard_band"] * 0.5 * view["width"] / fx
    limy = st["guard_band"] * 0.5 * view["height"] / fy
    xr = torch.clamp(px / pz, -limx, limx) * pz
    yr = torch.clamp(py / pz, -limy, limy) * pz
    zero = torch.zeros_like(pz)
    J = torch.stack([
        torch.stack([fx / pz, zero, -fx * xr / (pz * pz)], dim=-1),
        torch.stack([zero, fy / pz, -fy * yr / (pz * pz)], dim=-1),
    ], dim=-2)                                        # [n,2,3]
    T = J @ Rw                                        # [n,2,3]
    cov2 = T @ cov3 @ T.transpose(-1, -2)
    cov2 = cov2 + st["dilation"] * torch.eye(2, dtype=DT)
    mean2 = torch.stack([fx * px / pz + cx, fy * py / pz + cy], dim=-1)
    return pc, mean2, pz, cov2


def speed_flow(cov4: torch.Tensor, pc: torch.Tensor, view: dict):
    """2D flow of each Gaussian: the time derivative of its projected mean.

    The sliced mean moves as mu(t) = mu_xyz + (t - mu_t) V / W, so its speed is
    s = V / W (Sec. 3.2.2); in camera space p' = Wv s, and the pinhole mean
    (fx x/z + cx, fy y/z + cy) moves at (fx (x' z - x z') / z^2,
    fy (y' z - y z') / z^2).  Returns [n, 2] in pixels per unit of t."""
    w2c = _to64(view["world_to_cam"]).reshape(3, 4)
    speed = cov4[:, :3, 3] / cov4[:, 3, 3][:, None]
    vc = speed @ w2c[:, :3].T
    px, py, pz = pc.unbind(-1)
    vx, vy, vz = vc.unbind(-1)
    fx, fy = float(view["fx"]), float(view["fy"])
    return torch.stack([fx * (vx * pz - px * vz) / (pz * pz),
                        fy * (vy * pz - py * vz) / (pz * pz)], dim=-1)


def conic_of(cov2: torch.Tensor):
    """Inverse of the symmetric 2x2 covariance, as (a, b, c) with
    q(d) = a dx^2 + 2 b dx dy + c dy^2."""
    a, b, c = cov2[:, 0, 0], cov2[:, 0, 1], cov2[:, 1, 1]
    det = a * c - b * b
    return torch.stack([c / det, -b / det, a / det], dim=-1), det


# ---------------------------------------------------------------------------
# Sec. 3.1: spherical-harmonic colour


def sh_basis(dirs: torch.Tensor, degree: int) -> torch.Tensor:
    """Real orthonormal spherical harmonics up to `degree` (<= 3) at unit
    directions dirs [n,3]; order l-major, m = -l..l; sign convention of the
    3DGS renderer lineage (Condon-Shortley phase folded in).  Returns [n, k]."""
    x, y, z = dirs.unbind(-1)
    pi = math.pi
    out = [torch.full_like(x, 0.5 / math.sqrt(pi))]
    if degree >= 1:
        c1 = math.sqrt(3.0 / (4.0 * pi))
        out += [-c1 * y, c1 * z, -c1 * x]
    if degree >= 2:
        a = math.sqrt(15.0 / (4.0 * pi))
        b = math.sqrt(5.0 / (16.0 * pi))
        c = math.sqrt(15.0 / (16.0 * pi))
        out += [a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y), -a * x * z,
                c * (x * x - y * y)]
    if degree >= 3:
        a = math.sqrt(35.0 / (32.0 * pi))
        b = math.sqrt(105.0 / (4.0 * pi))
        c = math.sqrt(21.0 / (32.0 * pi))
        d = math.sqrt(7.0 / (16.0 * pi))
        e = math.sqrt(105.0 / (16.0 * pi))
        out += [-a * y * (3 * x * x - y * y), b * x * y * z, -c * y * (4 * z * z - x * x - y * y),
                d * z * (2 * z * z - 3 * x * x - 3 * y * y), -c * x * (4 * z * z - x * x - y * y),
                e * z * (x * x - y * y), -a * x * (x * x - 3 * y * y)]
    return torch.stack(out, dim=-1)


def sh_colour(sh: torch.Tensor, degree: int, mu3: torch.Tensor, cam_centre: torch.Tensor):
    """rgb = max(0, sum_lm Y_lm(d) c_lm + 0.5), d = normalize(mu(t) - camera centre).
    sh: [n, k, 3]."""
    d = mu3 - cam_centre
    d = d / torch.sqrt((d * d).sum(-1, keepdim=True))
    Y = sh_basis(d, degree)                          # [n,k]
    raw = (Y[:, :, None] * sh).sum(1) + 0.5
    return torch.clamp(raw, min=0.0)


# ---------------------------------------------------------------------------
# Per-Gaussian preprocess


def settings_dict(st: dict | None) -> dict:
    base = {
        "near_plane": 0.2, "time_cull": 16.0, "extent_sigma": 3.0,
        "alpha_min": 1.0 / 255.0, "alpha_max": 0.99, "T_min": 1e-4,
        "dilation": 0.3, "guard_band": 1.3,
    }
    if st:
        base.update({k: v for k, v in st.items() if k in base})
    return base


def params_to_torch(g: dict, requires_grad: bool = False) -> dict:
    """SoA float32 numpy arrays -> float64 torch leaves (same layouts)."""
    out = {}
    for key in ("means", "log_scales", "rotors", "opacity", "sh"):
        t = _to64(g[key]).clone()
        if requires_grad:
            t.requires_grad_(True)
        out[key] = t
    out["sh_degree"] = int(g["sh_degree"])
    return out


def preprocess(P: dict, view: dict, st: dict) -> dict:
    """Everything that is per Gaussian for one render.

    P holds float64 tensors in the SoA layouts.  Returns per-Gaussian tensors
    (mean2, conic, depth, opacity_t, rgb, valid mask and decision margins)."""
    st = settings_dict(st)
    n = P["means"].shape[-1]
    deg = P["sh_degree"]
    k = (deg + 1) ** 2
    mu4 = P["means"].T                                # [n,4]
    r = rotor_normalize(P["rotors"].T)                # [n,8]
    R = rotor_to_matrix(r)
    cov4 = covariance_4d(R, P["log_scales"].T)
    mu3, cov3, lam_dt2, decay = slice_at_time(mu4, cov4, float(view["t"]))
    o_t = P["opacity"] * decay
    pc, mean2, depth, cov2 = project_ewa(mu3, cov3, view, st)
    conic, det = conic_of(cov2)
    flow = speed_flow(cov4, pc, view)
    w2c = _to64(view["world_to_cam"]).reshape(3, 4)
    cam_centre = -(w2c[:, :3].T @ w2c[:, 3])
    sh = P["sh"].reshape(k, 3, n).permute(2, 0, 1)    # [n,k,3]
    rgb = sh_colour(sh, deg, mu3, cam_centre)
    time_ok = lam_dt2 <= st["time_cull"]
    near_ok = depth > st["near_plane"]
    valid = time_ok & near_ok & (det > 0)
    return {
        "mean2": mean2, "conic": conic, "depth": depth, "opacity": o_t, "rgb": rgb, "flow": flow,
        "valid": valid.detach(), "lam_dt2": lam_dt2.detach(), "cov2": cov2,
        "mu3": mu3, "cov3": cov3, "R": R, "rotor_n": r,
    }


# ---------------------------------------------------------------------------
# Sec. 3.1: depth-ordered alpha compositing


# Margins inside which an FP32 evaluation may take the other side of a
# threshold than this FP64 one; a flipped decision only matters when the
# entry's weight a * T_before is above AMB_WEIGHT.
AMB_Q = 1e-4          # |q - extent^2|
AMB_ALPHA_REL = 5e-5  # |a - alpha_min| / alpha_min
AMB_T_REL = 1e-4      # |T (1 - a) - T_min| / T_min
AMB_DEPTH_REL = 2.0 ** -21   # a few float32 roundings of the depth
AMB_WEIGHT = 1e-5


def _depth_tie_flags(used, au, T_before, dep, rgb):
    """Rows in which two consecutive contributors have depths within
    AMB_DEPTH_REL of each other (their FP32 order may differ) and swapping them
    could move the pixel by more than AMB_WEIGHT: a swap of neighbours i, j
    changes the colour by T_i a_i a_j (c_j - c_i)."""
    c, G = used.shape
    if G < 2:
        return torch.zeros(c, dtype=torch.bool)
    ar = torch.arange(G)
    marks = torch.where(used, ar[None, :], torch.full_like(used, -1, dtype=torch.int64))
    last = torch.cummax(marks, dim=1).values                      # last used index <= j
    prev = torch.cat([torch.full((c, 1), -1, dtype=torch.int64), last[:, :-1]], dim=1)
    ok = used & (prev >= 0)
    pi = prev.clamp(min=0)
    close = (dep[None, :] - dep[pi]).abs() <= dep[None, :] * AMB_DEPTH_REL
    dc = (rgb[None, :, :] - rgb[pi]).abs().amax(-1)
    swap = au * au.gather(1, pi) * T_before.gather(1, pi) * dc
    return (ok & close & (swap > AMB_WEIGHT)).any(1)


def composite(pix: torch.Tensor, pre: dict, bg, st: dict, chunk: int = 64, flow: bool = False):
    """Front-to-back compositing of every pixel in `pix` ([P,2] pixel indices
    (x, y); the sample point is the pixel centre (x+.5, y+.5)) over all valid
    Gaussians, sorted stably by depth (ties by index).

    C = sum_i c_i a_i prod_{j<i} (1 - a_j) + T_final * bg (Sec. 3.1), where a
    Gaussian is skipped if q > extent^2 or a < alpha_min, with
    a = min(alpha_max, o_t exp(-q/2)), and the walk stops (without the current
    Gaussian) once T (1 - a) < T_min.  With flow, each Gaussian's 2D flow is
    composited with the same weights as two more channels (background 0).
    Returns (colour [P,3] or [P,5], aux) with aux = T_final, contributor count
    and an ambiguity flag per pixel.
    """
    st = settings_dict(st)
    q_max = st["extent_sigma"] ** 2
    amin, amax, tmin = st["alpha_min"], st["alpha_max"], st["T_min"]
    valid_idx = torch.nonzero(pre["valid"]).flatten()
    depth = pre["depth"].detach()[valid_idx]
    order = valid_idx[torch.sort(depth, stable=True).indices]   # valid_idx is ascending
    m2 = pre["mean2"][order]
    cn = pre["conic"][order]
    op = pre["opacity"][order]
    rgb = pre["rgb"][order]
    bg_t = _to64(list(bg))
    amb_feat = rgb.detach()
    if flow:
        fl = pre["flow"][order]
        rgb = torch.cat([rgb, fl], dim=1)
        bg_t = torch.cat([bg_t, torch.zeros(2, dtype=DT)])
        # depth-tie ambiguity judged on the flow relative to its largest value
        scale = float(fl.detach().abs().max()) if fl.numel() else 1.0
        amb_feat = torch.cat([amb_feat, fl.detach() / max(scale, 1e-30)], dim=1)
    nc = rgb.shape[1]
    dep = pre["depth"].detach()[order]
    G = order.numel()
    P = pix.shape[0]
    colours = []
    T_final = torch.ones(P, dtype=DT)
    n_contrib = torch.zeros(P, dtype=torch.int64)
    ambiguous = torch.zeros(P, dtype=torch.bool)
    centres = pix.to(DT) + 0.5
    ar = torch.arange(G)
    if G == 0:
        # nothing survives: every pixel is the background
        out = bg_t[None, :].expand(P, nc).clone()
        return out, {"T_final": T_final, "n_contrib": n_contrib, "ambiguous": ambiguous}
    for s0 in range(0, P, chunk):
        pts = centres[s0:s0 + chunk]
        c = pts.shape[0]
        with torch.no_grad():
            d = m2.detach()[None, :, :] - pts[:, None, :]          # [c,G,2]
            a_, b_, c_ = cn.detach().unbind(-1)
            q = a_ * d[..., 0] ** 2 + 2 * b_ * d[..., 0] * d[..., 1] + c_ * d[..., 1] ** 2
            a_raw = op.detach()[None, :] * torch.exp(-0.5 * q)
            alpha = torch.clamp(a_raw, max=amax)
            use = (q <= q_max) & (alpha >= amin)
            au = torch.where(use, alpha, torch.zeros_like(alpha))
            T_after = torch.cumprod(1.0 - au, dim=1)
            T_before = torch.cat([torch.ones(c, 1, dtype=DT), T_after[:, :-1]], dim=1)
            hit = use & (T_after < tmin)
            has = hit.any(1)
            stop = torch.where(has, hit.to(torch.int64).argmax(1), torch.full((c,), G))
            considered = ar[None, :] <= stop[:, None]
            used = use & (ar[None, :] < stop[:, None])
            # decision margins, weighted by what a flip could change
            weight = a_raw * T_before
            amb = ((q - q_max).abs() < AMB_Q) | (((a_raw - amin).abs() / amin) < AMB_ALPHA_REL)
            amb &= q <= q_max + 10 * AMB_Q
            amb |= use & (((T_after - tmin).abs() / tmin) < AMB_T_REL)
            amb &= considered & (weight > AMB_WEIGHT)
            amb_pix = amb.any(1)
        need_grad = torch.is_grad_enabled() and any(
            t.requires_grad for t in (m2, cn, op, rgb))
        if not need_grad:
            # same sums, evaluated densely (no autograd graph to keep)
            with torch.no_grad():
                w = torch.where(used, au * T_before, torch.zeros_like(au))
                tf = torch.where(has, T_before.gather(1, stop.clamp(max=G - 1)[:, None])[:, 0],
                                 T_after[:, -1] if G else torch.ones(c, dtype=DT))
                col = w @ rgb.detach() + tf[:, None] * bg_t[None, :]
                T_final[s0:s0 + c] = tf
                n_contrib[s0:s0 + c] = used.sum(1)
                amb_rows = amb_pix | _depth_tie_flags(used, au, T_before, dep, amb_feat)
                ambiguous[s0:s0 + c] = amb_rows
                colours.append(col)
            continue
        for row in range(c):
            p = s0 + row
            sel = torch.nonzero(used[row]).flatten()
            with torch.no_grad():
                flag = bool(amb_pix[row])
                if sel.numel() > 1:
                    flag |= bool(_depth_tie_flags(used[row:row + 1], au[row:row + 1],
                                                  T_before[row:row + 1], dep, amb_feat)[0])
                ambiguous[p] = flag
                n_contrib[p] = sel.numel()
            # the blending equation on the contributing Gaussians, differentiably
            dx = m2[sel, 0] - pts[row, 0]
            dy = m2[sel, 1] - pts[row, 1]
            qq = cn[sel, 0] * dx * dx + 2 * cn[sel, 1] * dx * dy + cn[sel, 2] * dy * dy
            aa = torch.clamp(op[sel] * torch.exp(-0.5 * qq), max=amax)
            Tex = torch.cumprod(torch.cat([torch.ones(1, dtype=DT), 1.0 - aa]), 0)
            w = aa * Tex[:-1]
            col = (rgb[sel] * w[:, None]).sum(0) + Tex[-1] * bg_t
            T_final[p] = Tex[-1].detach()
            colours.append(col[None])
    out = torch.cat(colours, 0) if colours else torch.zeros(0, nc, dtype=DT)
    aux = {"T_final": T_final, "n_contrib": n_contrib, "ambiguous": ambiguous}
    return out, aux


def gaussian_margin_flags(pre: dict, st: dict):
    """Per-Gaussian flags: the time-cull or near-plane decision is within FP32
    rounding of its threshold and the Gaussian is opaque enough to be blended
    somewhere if kept (o_t >= alpha_min)."""
    st = settings_dict(st)
    tau = st["time_cull"]
    f = (pre["lam_dt2"] - tau).abs() < 1e-5 * tau
    f |= (pre["depth"].detach() - st["near_plane"]).abs() < 1e-6
    o = pre["opacity"].detach()
    return f & (o >= st["alpha_min"] * (1 - 1e-5))


def render(g: dict, view: dict, st: dict | None = None, pixels=None,
           requires_grad: bool = False, P: dict | None = None, flow: bool = False):
    """Render one view.

    g: SoA parameter arrays (workloads layout).  pixels: None for the full
    frame, or a 1-D array of row-major pixel indices.  Returns a dict with
    'image' ([3,H,W] or [3,P]), with flow also 'flow' ([2,H,W] or [2,P]),
    'params' (the float64 leaves), 'pre' and aux.
    """
    st = settings_dict(st)
    if P is None:
        P = params_to_torch(g, requires_grad=requires_grad)
    pre = preprocess(P, view, st)
    H, W = int(view["height"]), int(view["width"])
    if pixels is None:
        ys, xs = torch.meshgrid(torch.arange(H), torch.arange(W), indexing="ij")
        pix = torch.stack([xs.flatten(), ys.flatten()], dim=-1)
    else:
        pidx = torch.as_tensor(np.asarray(pixels), dtype=torch.int64)
        pix = torch.stack([pidx % W, pidx // W], dim=-1)
    col, aux = composite(pix, pre, view["bg"], st, flow=flow)
    # Pixels a Gaussian with a marginal cull decision could be blended into.
    gflag = gaussian_margin_flags(pre, st)
    if bool(gflag.any()):
        with torch.no_grad():
            idx = torch.nonzero(gflag).flatten()
            d = pre["mean2"].detach()[idx][None] - (pix.to(DT) + 0.5)[:, None]
            cn = pre["conic"].detach()[idx]
            q = cn[:, 0] * d[..., 0] ** 2 + 2 * cn[:, 1] * d[..., 0] * d[..., 1] + cn[:, 2] * d[..., 1] ** 2
            o = pre["opacity"].detach()[idx]
            reach = torch.clamp(2.0 * torch.log(o / st["alpha_min"]), max=st["extent_sigma"] ** 2)
            aux["ambiguous"] |= (q <= reach[None, :] + 1e-3).any(1)
    image = col[:, :3].T.contiguous()
    out = {}
    if flow:
        out["flow"] = col[:, 3:].T.contiguous()
    if pixels is None:
        image = image.reshape(3, H, W)
        if flow:
            out["flow"] = out["flow"].reshape(2, H, W)
        for key in ("T_final", "n_contrib", "ambiguous"):
            aux[key] = aux[key].reshape(H, W)
    return {"image": image, "params": P, "pre": pre, **out, **aux}
