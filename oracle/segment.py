"""FP64 oracle of the segmentation by convex relaxation (paper Sec. 3.2 and
Sec. 4).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module; the product library never does.

What it computes, in the paper's order and notation:

* the energy of Sec. 3.2 (eq:energy1): per label i the weighted boundary
  length (lambda/2) Per_g(Omega_i), the label cost nu delta_i (eq:mdl) and the
  data term f_i = -log P of the pixels given label i;
* the edge metric g(x) = exp(-|grad I(x)| / gamma) / (2 gamma) of Sec. 3.2,
  gamma the mean gradient magnitude over the image unless given;
* the relaxation of Sec. 4.1: indicator functions u_i (eq:thetas) relaxed to
  [0, 1] with sum_i u_i = 1 at every pixel, the boundary length as the
  weighted total variation sup over xi_i in K_g of -sum u_i div xi_i
  (eq:intbyparts), K_g = {|xi(x)| <= lambda g(x) / 2}, and for nu > 0 the
  label variables m_i >= u_i(x) with multipliers mu <= 0 (eq:sets);
* the primal-dual iteration of Sec. 4.2 (algo): projected ascent in xi and
  mu, projected descent in m and u, over-relaxation u_bar = 2 u^{t+1} - u^t
  and m_bar = 2 m^{t+1} - m^t, projections onto K_g, onto mu <= 0, onto
  [0, 1] and onto the simplex (Michelot's finite algorithm);
* the binary segmentation l(x) = argmax_i u_i(x) (Sec. 4.2) and the energies
  that bound its distance from the optimum: the relaxed primal energy, the
  energy of the binary segmentation and the dual energy (a lower bound of the
  relaxed optimum for any feasible xi, mu).

Readings of points the paper leaves open (each also stated in the design
notes):

* discretisation: forward differences with zero gradient across the last
  column and row (Neumann), and the divergence as minus their adjoint;
  |grad| is the Euclidean norm of the two differences (isotropic);
* |grad I| of the colour image: the Euclidean norm over the three channels
  and both differences;
* step sizes: the diagonal preconditioning (alpha = 1) of Pock and Chambolle
  cited for them, taken with the interior column sums: sigma_xi = 1/2,
  sigma_mu = 1/2, tau_u = 1/4 (1/5 with the label variables), tau_m = 1/N;
* start: u = 1/L, u_bar = u, xi = 0, mu = 0, m = m_bar = 1;
* nu = 0 (supervised, as the paper sets it): the label variables and their
  multipliers are left out (m = 1 and mu = 0 satisfy their optimality
  conditions for every u, so the relaxed problem is unchanged);
* argmax ties go to the lowest label index.
"""
from __future__ import annotations

import numpy as np


def grad(u: np.ndarray):
    """Forward differences of u (..., H, W): (d/dx, d/dy), zero across the last
    column and the last row."""
    dx = np.zeros_like(u)
    dy = np.zeros_like(u)
    dx[..., :, :-1] = u[..., :, 1:] - u[..., :, :-1]
    dy[..., :-1, :] = u[..., 1:, :] - u[..., :-1, :]
    return dx, dy


def div(px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """Divergence, minus the adjoint of grad: sum_x <grad u, p> = -sum_x u div p."""
    d = np.zeros_like(px)
    d[..., :, :-1] += px[..., :, :-1]
    d[..., :, 1:] -= px[..., :, :-1]
    d[..., :-1, :] += py[..., :-1, :]
    d[..., 1:, :] -= py[..., :-1, :]
    return d


def colour_gradient(rgb: np.ndarray) -> np.ndarray:
    """|grad I(x)|: Euclidean norm of the forward differences of the three
    colour planes (3, H, W) at every pixel."""
    I = np.asarray(rgb, np.float64)
    dx, dy = grad(I)
    return np.sqrt((dx * dx + dy * dy).sum(0))


def edge_weight(rgb: np.ndarray, gamma: float = 0.0):
    """g(x) = exp(-|grad I(x)| / gamma) / (2 gamma) (Sec. 3.2); gamma <= 0
    selects the mean of |grad I| over the image.  Returns (g, gamma)."""
    mag = colour_gradient(rgb)
    if not gamma > 0.0:
        gamma = float(mag.sum() / mag.size)
    return np.exp(-mag / gamma) / (2.0 * gamma), gamma


def project_simplex(v: np.ndarray) -> np.ndarray:
    """Euclidean projection of every row v[..., :] onto {u >= 0, sum u = 1}
    by Michelot's finite algorithm: project onto the hyperplane sum = 1 of the
    coordinates still in play, drop those that came out negative (set to 0),
    repeat until none does."""
    v = np.asarray(v, np.float64)
    flat = v.reshape(-1, v.shape[-1])
    out = np.empty_like(flat)
    for r in range(flat.shape[0]):
        y = flat[r]
        active = np.ones(y.size, dtype=bool)
        while True:
            theta = (y[active].sum() - 1.0) / active.sum()
            x = np.where(active, y - theta, 0.0)
            neg = active & (x < 0.0)
            if not neg.any():
                break
            active &= ~neg
        out[r] = x
    return out.reshape(v.shape)


def project_simplex_planes(v: np.ndarray) -> np.ndarray:
    """The same projection for label-major planes v (L, H, W): Michelot's
    algorithm run on every pixel at once (same steps, same order of sums)."""
    L = v.shape[0]
    active = np.ones(v.shape, dtype=bool)
    while True:
        cnt = active.sum(0)
        s = np.zeros(v.shape[1:])
        for i in range(L):  # sum in label order
            s = s + np.where(active[i], v[i], 0.0)
        theta = (s - 1.0) / cnt
        x = np.where(active, v - theta[None], 0.0)
        neg = active & (x < 0.0)
        if not neg.any():
            return x
        active &= ~neg


def project_ball(px: np.ndarray, py: np.ndarray, radius: np.ndarray):
    """Projection of each 2-vector (px, py) onto the disc |p| <= radius (K_g)."""
    n = np.sqrt(px * px + py * py)
    s = np.where(n > radius, radius / np.where(n > 0, n, 1.0), 1.0)
    return px * s, py * s


def primal_energy(u, f, g, lam, nu=0.0) -> float:
    """sum_i sum_x u_i f_i + (lambda/2) g |grad u_i| (+ nu max_x u_i)."""
    dx, dy = grad(u)
    e = float((u * f).sum() + (0.5 * lam * g[None] * np.sqrt(dx * dx + dy * dy)).sum())
    if nu > 0.0:
        e += nu * float(u.reshape(u.shape[0], -1).max(1).sum())
    return e


def dual_energy(px, py, mu, f, nu=0.0) -> float:
    """min over u in the simplex, m in [0,1] of the Lagrangian at (xi, mu):
    sum_x min_i (f_i - div xi_i - mu_i) + sum_i min(0, nu + sum_x mu_i)."""
    q = f - div(px, py)
    if mu is not None:
        q = q - mu
    e = float(q.min(0).sum())
    if mu is not None and nu > 0.0:
        e += float(np.minimum(0.0, nu + mu.reshape(mu.shape[0], -1).sum(1)).sum())
    return e


def labels_of(u) -> np.ndarray:
    """l(x) = argmax_i u_i(x), ties to the lowest label."""
    return np.argmax(u, axis=0).astype(np.int32)


def binary_energy(labels, f, g, lam, nu=0.0) -> float:
    """Energy of eq:energy1 of a segmentation given by its labels."""
    L = f.shape[0]
    u = (labels[None] == np.arange(L)[:, None, None]).astype(np.float64)
    e = primal_energy(u, f, g, lam, 0.0)
    if nu > 0.0:
        e += nu * float(len(np.unique(labels)))
    return e


def step_sizes(N: int, mdl: bool):
    """(sigma_xi, sigma_mu, tau_u, tau_m): diagonal preconditioning, alpha = 1."""
    return 0.5, 0.5, (0.2 if mdl else 0.25), 1.0 / N


def solve(f: np.ndarray, g: np.ndarray, lam: float, nu: float = 0.0, iterations: int = 100,
          trace: bool = False) -> dict:
    """The primal-dual iteration of Sec. 4.2 on the data term f (L, H, W) and
    the edge metric g (H, W).  Returns the final primal and dual variables,
    the labels and the three energies (and their values after every
    iteration when trace is set)."""
    f = np.asarray(f, np.float64)
    g = np.asarray(g, np.float64)
    L, H, W = f.shape
    N = H * W
    mdl = nu > 0.0
    s_xi, s_mu, t_u, t_m = step_sizes(N, mdl)
    radius = 0.5 * lam * g
    u = np.full(f.shape, 1.0 / L)
    ub = u.copy()
    px = np.zeros_like(u)
    py = np.zeros_like(u)
    mu = np.zeros_like(u) if mdl else None
    m = np.ones(L)
    mb = m.copy()
    hist = []
    for _ in range(iterations):
        # dual ascent in xi, projected onto K_g
        gx, gy = grad(ub)
        px, py = project_ball(px + s_xi * gx, py + s_xi * gy, radius[None])
        if mdl:
            # dual ascent in mu, projected onto mu <= 0
            mu = np.minimum(0.0, mu + s_mu * (mb[:, None, None] - ub))
            # primal descent in m, projected onto [0, 1]
            m_new = np.clip(m - t_m * (nu + mu.reshape(L, -1).sum(1)), 0.0, 1.0)
        # primal descent in u, projected onto the simplex
        step = -div(px, py) + f
        if mdl:
            step = step - mu
        u_new = project_simplex_planes(u - t_u * step)
        # over-relaxation
        ub = 2.0 * u_new - u
        u = u_new
        if mdl:
            mb = 2.0 * m_new - m
            m = m_new
        if trace:
            lab = labels_of(u)
            hist.append((primal_energy(u, f, g, lam, nu), binary_energy(lab, f, g, lam, nu),
                         dual_energy(px, py, mu, f, nu)))
    lab = labels_of(u)
    out = {"u": u, "ubar": ub, "px": px, "py": py, "mu": mu, "m": m, "labels": lab,
           "primal": primal_energy(u, f, g, lam, nu), "binary": binary_energy(lab, f, g, lam, nu),
           "dual": dual_energy(px, py, mu, f, nu)}
    if trace:
        out["trace"] = np.asarray(hist)
    return out


def data_term(loglik: np.ndarray, H: int, W: int) -> np.ndarray:
    """f_i = -l_i (Sec. 3.2) as label-major planes (L, H, W) from pixel-major
    log-likelihoods (N, L)."""
    ll = np.asarray(loglik, np.float64)
    return -ll.T.reshape(ll.shape[1], H, W)


def dice(labels: np.ndarray, truth: np.ndarray, L: int) -> np.ndarray:
    """Dice score 2 |A n B| / (|A| + |B|) of every label."""
    out = np.zeros(L)
    for i in range(L):
        a, b = labels == i, truth == i
        den = a.sum() + b.sum()
        out[i] = 2.0 * (a & b).sum() / den if den else 1.0
    return out
