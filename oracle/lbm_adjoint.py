"""CPU oracle of the differentiated lattice path.

Test infrastructure: only the tests, the smoke check and the CPU baseline of
the benchmark use this module; the library never imports it.

A plain PyTorch (CPU, FP64) restatement of
  * one BGK collide-and-stream step with the Hermite force term and the
    half-step velocity shift (Section 3.1, Eq. (tau) for the relaxation time;
    the force term is the reading written down for the forward oracle),
  * the Hermite coefficients a(n) = sum_a f_a H(n)(xi_a) of the populations up
    to third order (the expansion of Eq. (discretefunctions)),
  * the DSMC2LB projection of sampled moments (Eq. (nordercoefficients) into
    Eq. (discretefunctions)),
written from those definitions without any blocking or fusion.  Gradients
come from reverse-mode automatic differentiation of these definitions, so they
are the exact derivatives (up to rounding) that a hand-written adjoint has to
reproduce.

Array layouts follow the library: populations [Q][ny*nx] (node = iy*nx + ix),
moment averages [11][ncells], Hermite coefficients [NH][nsel] with the row
order (1, x, y, xx, xy, yy, xxx, xxy, xyy, yyy).
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64
NH_OF_ORDER = {0: 1, 1: 3, 2: 6, 3: 10}


def _t(a):
    return torch.as_tensor(np.asarray(a), dtype=F64)


def _lat(lat):
    xi = _t(lat["xi"])
    return xi[:, 0], xi[:, 1], _t(lat["w"]), np.asarray(lat["e"], dtype=np.int64)


def _buffer_rows(lat, ny):
    """Rows held fixed when y_mode is 1: the max|e_y| rows at each y edge."""
    K = int(np.abs(np.asarray(lat["e"])[:, 1]).max())
    rows = torch.zeros(ny, dtype=torch.bool)
    rows[:K] = True
    rows[ny - K:] = True
    return rows


def collide(f, lat, tau, g):
    """BGK relaxation with the Hermite force term at every node.
    f: [Q, ny, nx]; tau, g: scalars (tensors allowed).  Per node:
    rho = sum f, u = (sum f xi + rho g e_x / 2) / rho, the Hermite equilibrium
    w rho [1 + xi.u + ((xi.u)^2 - u.u)/2 (+ xi.u((xi.u)^2 - 3 u.u)/6 on D2Q37)],
    force (1 - 1/(2 tau)) w rho [xi_x g + (xi_x g)(xi.u) - g u_x],
    post-collision f - (f - f_eq)/tau + force."""
    xx, xy, w, _ = _lat(lat)
    Q = len(w)
    xx, xy, w = xx[:, None, None], xy[:, None, None], w[:, None, None]
    rho = f.sum(0)
    jx = (f * xx).sum(0)
    jy = (f * xy).sum(0)
    ux = (jx + 0.5 * rho * g) / rho
    uy = jy / rho
    uu = ux * ux + uy * uy
    cu = xx * ux + xy * uy
    eq = 1.0 + cu + 0.5 * (cu * cu - uu)
    if Q != 9:
        eq = eq + cu * (cu * cu - 3.0 * uu) / 6.0
    feq = w * rho * eq
    cg = xx * g
    force = (1.0 - 0.5 / tau) * w * rho * (cg + cg * cu - g * ux)
    return f - (f - feq) / tau + force


def step(f, lat, nx, ny, tau, g, y_mode):
    """One collide-and-stream step on f [Q][ny*nx] (returns a new tensor).
    Streaming moves population a from node x to x + e_a, x periodic; y
    periodic (y_mode 0) or, with y_mode 1, the buffer rows keep their
    populations uncollided, send them on into the interior, and nothing
    streamed into a buffer row is kept."""
    _, _, _, e = _lat(lat)
    Q = len(e)
    f3 = f.reshape(Q, ny, nx)
    fe = collide(f3, lat, tau, g)
    if y_mode == 1:
        rows = _buffer_rows(lat, ny)[None, :, None]
        fe = torch.where(rows, f3, fe)
    out = torch.stack([torch.roll(fe[a], shifts=(int(e[a, 1]), int(e[a, 0])), dims=(0, 1)) for a in range(Q)])
    if y_mode == 1:
        out = torch.where(rows, f3, out)
    return out.reshape(Q, ny * nx)


def rollout(f0, lat, nx, ny, tau, g, y_mode, nsteps):
    f = f0
    for _ in range(nsteps):
        f = step(f, lat, nx, ny, tau, g, y_mode)
    return f


def hermite_rows(lat, order):
    """H(n)(xi_a) for n <= order: [NH][Q] in the row order of the module."""
    x, y, _, _ = _lat(lat)
    one = torch.ones_like(x)
    rows = [one]
    if order >= 1:
        rows += [x, y]
    if order >= 2:
        rows += [x * x - 1.0, x * y, y * y - 1.0]
    if order >= 3:
        rows += [x * x * x - 3.0 * x, x * x * y - y, x * y * y - x, y * y * y - 3.0 * y]
    return torch.stack(rows)


def hermite_coefficients(f, lat, order, nodes):
    """a(n) = sum_a f_a H(n)(xi_a) at the listed nodes: [NH][len(nodes)]."""
    H = hermite_rows(lat, order)
    return H @ f[:, torch.as_tensor(np.asarray(nodes), dtype=torch.long)]


def project(avg, ppc, lat, order, kT=1.0):
    """DSMC2LB projection of per-cell moment averages avg [11][ncells] (the
    means of N, sum vx, sum vy, sum vx^2, sum vx vy, sum vy^2, sum vx^3,
    sum vx^2 vy, sum vx vy^2, sum vy^3, sum vz^2): rho = <N>/ppc, absolute-
    frame Hermite coefficients from the normalised moments, then
    f_a = w_a sum_{n<=order} a(n):H(n)(xi_a)/n!.  Cells without particles get
    zero populations.  D2Q9 leaves out H_xxx and H_yyy (zero on its nodes)."""
    x, y, w, _ = _lat(lat)
    Q = len(w)
    m0 = avg[0]
    full = m0 > 0.0
    m0s = torch.where(full, m0, torch.ones_like(m0))
    s1 = float(np.sqrt(kT))
    s2, s3 = s1 * s1, s1 * s1 * s1
    rho = m0s / float(ppc)
    ex, ey = avg[1] / m0s / s1, avg[2] / m0s / s1
    exx, exy, eyy = avg[3] / m0s / s2, avg[4] / m0s / s2, avg[5] / m0s / s2
    exxx, exxy, exyy, eyyy = (avg[k] / m0s / s3 for k in (6, 7, 8, 9))
    X, Y = x[:, None], y[:, None]
    v = rho[None, :].expand(Q, -1)
    if order >= 1:
        v = v + (rho * ex)[None] * X + (rho * ey)[None] * Y
    if order >= 2:
        v = v + 0.5 * ((rho * (exx - 1.0))[None] * (X * X - 1.0) + 2.0 * (rho * exy)[None] * (X * Y)
                       + (rho * (eyy - 1.0))[None] * (Y * Y - 1.0))
    if order >= 3:
        t3 = 3.0 * (rho * (exxy - ey))[None] * (X * X * Y - Y) + 3.0 * (rho * (exyy - ex))[None] * (X * Y * Y - X)
        if Q != 9:
            t3 = t3 + (rho * (exxx - 3.0 * ex))[None] * (X * X * X - 3.0 * X) \
                + (rho * (eyyy - 3.0 * ey))[None] * (Y * Y * Y - 3.0 * Y)
        v = v + t3 / 6.0
    return torch.where(full[None, :], w[:, None] * v, torch.zeros_like(v))


def step_vjp(f, lam_next, lat, nx, ny, tau, g, y_mode):
    """(lam_n, dJ/dg, dJ/dtau) for one step: lam_n = (d f_{n+1} / d f_n)^T
    lam_next and the step's share of the parameter gradients."""
    f = _t(f).clone().requires_grad_(True)
    tau_t = torch.tensor(float(tau), dtype=F64, requires_grad=True)
    g_t = torch.tensor(float(g), dtype=F64, requires_grad=True)
    out = step(f, lat, nx, ny, tau_t, g_t, y_mode)
    lam, dg, dtau = torch.autograd.grad(out, (f, g_t, tau_t), grad_outputs=_t(lam_next), allow_unused=True)
    dg = 0.0 if dg is None else float(dg)
    dtau = 0.0 if dtau is None else float(dtau)
    return lam.numpy(), dg, dtau


def rollout_vjp(f0, lam_N, lat, nx, ny, tau, g, y_mode, nsteps):
    """(f_N, lam_0, dJ/dg, dJ/dtau) of nsteps steps for a terminal cotangent
    lam_N = dJ/df_N."""
    f = _t(f0).clone().requires_grad_(True)
    tau_t = torch.tensor(float(tau), dtype=F64, requires_grad=True)
    g_t = torch.tensor(float(g), dtype=F64, requires_grad=True)
    out = rollout(f, lat, nx, ny, tau_t, g_t, y_mode, nsteps)
    if nsteps == 0:
        return out.detach().numpy(), np.asarray(lam_N, dtype=np.float64).copy(), 0.0, 0.0
    lam, dg, dtau = torch.autograd.grad(out, (f, g_t, tau_t), grad_outputs=_t(lam_N), allow_unused=True)
    dg = 0.0 if dg is None else float(dg)
    dtau = 0.0 if dtau is None else float(dtau)
    return out.detach().numpy(), lam.numpy(), dg, dtau


def mismatch(f0, lat, nx, ny, tau, g, y_mode, nsteps, nodes, order, avg, cells, ppc, kT=1.0):
    """The coupling-node moment mismatch and its gradients.

    J = 1/2 sum_i sum_n (a(n)(f_N at nodes[i]) - a(n)(P(avg) at cells[i]))^2,
    with f_N the populations after nsteps steps from f0 and P the DSMC2LB
    projection (to the same order) of the DSMC moment averages.
    Returns dict(J, f0_bar, g_bar, tau_bar, avg_bar)."""
    f = _t(f0).clone().requires_grad_(True)
    tau_t = torch.tensor(float(tau), dtype=F64, requires_grad=True)
    g_t = torch.tensor(float(g), dtype=F64, requires_grad=True)
    m = _t(avg).clone().requires_grad_(True)
    fN = rollout(f, lat, nx, ny, tau_t, g_t, y_mode, nsteps)
    a_lb = hermite_coefficients(fN, lat, order, nodes)
    fD = project(m, ppc, lat, order, kT)
    a_d = hermite_coefficients(fD, lat, order, cells)
    J = 0.5 * ((a_lb - a_d) ** 2).sum()
    gf, gg, gt, gm = torch.autograd.grad(J, (f, g_t, tau_t, m), allow_unused=True)
    z = lambda t, like: torch.zeros_like(like) if t is None else t
    return {"J": float(J.detach()), "f0_bar": z(gf, f).numpy(), "g_bar": float(z(gg, g_t)), "tau_bar": float(z(gt, tau_t)),
            "avg_bar": z(gm, m).numpy()}
