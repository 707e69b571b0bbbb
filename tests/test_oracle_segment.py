"""Pins of the FP64 oracle of the convex relaxation (Sec. 3.2, Sec. 4) to what
the mathematics fixes: the adjoint identity of the discrete gradient and
divergence, an independent sort-based simplex projection and a generic
constrained minimiser, closed-form minimisers (no boundary term, constant
data terms), weak duality and the vanishing duality gap, brute force over
every labelling of tiny images, and the relaxation gap the paper reports
(the rounded solution within 1 % of the optimal energy)."""
import itertools

import numpy as np
import pytest

from oracle import segment as sg


def _proj_sort(y):
    """Projection onto the simplex by sorting (the textbook threshold form):
    the largest k with y_(k) > (sum_{j<=k} y_(j) - 1) / k sets theta."""
    z = np.sort(y)[::-1]
    cs = np.cumsum(z)
    k = np.nonzero(z - (cs - 1.0) / np.arange(1, y.size + 1) > 0)[0][-1] + 1
    theta = (cs[k - 1] - 1.0) / k
    return np.maximum(y - theta, 0.0)


def test_gradient_divergence_adjoint():
    rng = np.random.default_rng(1)
    for H, W in [(1, 1), (1, 7), (6, 1), (5, 8)]:
        u = rng.standard_normal((3, H, W))
        px, py = rng.standard_normal((2, 3, H, W))
        dx, dy = sg.grad(u)
        lhs = (dx * px + dy * py).sum()
        rhs = -(u * sg.div(px, py)).sum()
        assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs))
    # Neumann: nothing leaves through the last column and row
    dx, dy = sg.grad(rng.standard_normal((4, 6)))
    assert np.all(dx[:, -1] == 0) and np.all(dy[-1, :] == 0)


@pytest.mark.parametrize("L", [1, 2, 3, 7, 16])
def test_simplex_projection_matches_sort_form(L):
    rng = np.random.default_rng(L)
    Y = np.concatenate([rng.standard_normal((200, L)) * 3, rng.uniform(0, 1, (20, L)),
                        np.full((3, L), 0.25), rng.integers(-2, 3, (20, L)).astype(float)])
    got = sg.project_simplex(Y)
    ref = np.stack([_proj_sort(y) for y in Y])
    np.testing.assert_allclose(got, ref, atol=1e-13)
    assert np.all(got >= 0) and np.allclose(got.sum(1), 1.0, atol=1e-13)
    # points of the simplex are fixed points
    inside = sg.project_simplex(got)
    np.testing.assert_allclose(inside, got, atol=1e-13)
    # the per-pixel planes form runs the same algorithm
    planes = Y[:60].T.reshape(L, 6, 10)
    np.testing.assert_allclose(sg.project_simplex_planes(planes), got[:60].T.reshape(L, 6, 10), atol=1e-14)


def test_simplex_projection_is_the_nearest_point():
    from scipy.optimize import minimize
    rng = np.random.default_rng(3)
    for _ in range(5):
        y = rng.standard_normal(5) * 2
        x = sg.project_simplex(y[None])[0]
        r = minimize(lambda z: ((z - y) ** 2).sum(), np.full(5, 0.2), method="SLSQP",
                     bounds=[(0, None)] * 5, constraints=[{"type": "eq", "fun": lambda z: z.sum() - 1}],
                     options={"ftol": 1e-14, "maxiter": 500})
        np.testing.assert_allclose(x, r.x, atol=1e-6)


def test_edge_weight_closed_form():
    rgb = np.zeros((3, 4, 5))
    rgb[0, :, 3:] = 1.0   # a vertical step in red between columns 2 and 3
    rgb[2, 2:, :] = 0.5   # a horizontal step in blue between rows 1 and 2
    mag = sg.colour_gradient(rgb)
    assert mag[0, 2] == 1.0 and mag[1, 2] == np.sqrt(1.25) and mag[1, 0] == 0.5 and mag[0, 0] == 0.0
    g, gamma = sg.edge_weight(rgb)
    assert gamma == mag.mean()
    np.testing.assert_allclose(g, np.exp(-mag / gamma) / (2 * gamma), rtol=1e-15)
    g5, gm5 = sg.edge_weight(rgb, 5.0)
    assert gm5 == 5.0 and g5[0, 0] == 0.1


def test_no_boundary_term_gives_pointwise_minimum():
    """lambda = 0: the energy is sum_x sum_i u_i f_i, minimised at every pixel by
    the label of smallest f (distinct values)."""
    rng = np.random.default_rng(4)
    f = rng.standard_normal((4, 6, 7)) * 3
    g = np.ones((6, 7))
    r = sg.solve(f, g, lam=0.0, iterations=200)
    assert np.array_equal(r["labels"], np.argmin(f, axis=0))
    np.testing.assert_allclose(r["u"], (np.arange(4)[:, None, None] == np.argmin(f, 0)[None]).astype(float),
                               atol=1e-12)
    assert abs(r["primal"] - f.min(0).sum()) <= 1e-9


def test_constant_data_terms_give_one_label():
    f = np.zeros((3, 5, 6))
    f[0] += 2.0
    f[1] += 0.5
    f[2] += 1.0
    rng = np.random.default_rng(5)
    g = rng.uniform(0.1, 2.0, (5, 6))
    r = sg.solve(f, g, lam=1.0, iterations=400)
    assert np.all(r["labels"] == 1)
    assert abs(r["binary"] - 0.5 * 30) <= 1e-12


@pytest.mark.parametrize("nu", [0.0, 0.7])
def test_weak_duality_and_vanishing_gap(nu):
    """Every dual energy of the iteration is at most every primal energy
    (feasible duals), and the gap closes as the iteration converges."""
    rng = np.random.default_rng(6)
    f = rng.standard_normal((3, 8, 9)) * 2
    g, _ = sg.edge_weight(rng.uniform(0, 1, (3, 8, 9)))
    r = sg.solve(f, g, lam=1.5, nu=nu, iterations=3000, trace=True)
    tr = r["trace"]
    assert tr[:, 2].max() <= tr[:, 0].min() + 1e-9
    assert r["primal"] - r["dual"] <= 1e-3 * abs(r["primal"])
    # the rounded segmentation is feasible for the unrelaxed problem
    assert r["binary"] >= r["dual"] - 1e-9


def test_brute_force_tiny_images():
    """Every labelling of 3x3 images with 3 labels: the dual energy bounds the
    optimum from below, and the rounded solution attains the optimum on most
    draws (the relaxation is near-tight)."""
    rng = np.random.default_rng(7)
    hits = 0
    for _ in range(12):
        f = rng.standard_normal((3, 3, 3)) * 2
        g = rng.uniform(0.2, 1.5, (3, 3))
        lam = float(rng.uniform(0.5, 3.0))
        best = min(sg.binary_energy(np.array(lab, np.int32).reshape(3, 3), f, g, lam)
                   for lab in itertools.product(range(3), repeat=9))
        r = sg.solve(f, g, lam=lam, iterations=1500)
        assert r["dual"] <= best + 1e-9
        assert r["binary"] >= best - 1e-12
        hits += r["binary"] <= best + 1e-9
    assert hits >= 10, hits


def test_label_variables_leave_the_supervised_optimum_unchanged():
    """With a vanishing label cost the relaxed optimum with the label
    variables and multipliers equals the one without them (the reading for
    nu = 0)."""
    rng = np.random.default_rng(8)
    f = rng.standard_normal((3, 7, 8))
    g, _ = sg.edge_weight(rng.uniform(0, 1, (3, 7, 8)))
    a = sg.solve(f, g, lam=1.0, nu=0.0, iterations=3000)
    b = sg.solve(f, g, lam=1.0, nu=1e-12, iterations=3000)
    assert abs(a["primal"] - b["primal"]) <= 1e-4 * abs(a["primal"])


def test_label_cost_removes_labels():
    """A label that is slightly better on a small patch only: without a label
    cost it wins there; a label cost above that gain removes it."""
    f = np.zeros((2, 10, 10))
    f[1] += 1.0
    f[1, 4:6, 4:6] = -0.5  # label 1 gains 1.5 per pixel on 4 pixels (6 in all)
    g = np.full((10, 10), 0.05)
    r0 = sg.solve(f, g, lam=1.0, nu=0.0, iterations=2000)
    assert np.all(r0["labels"][4:6, 4:6] == 1)
    r1 = sg.solve(f, g, lam=1.0, nu=20.0, iterations=4000)
    assert np.all(r1["labels"] == 0)


def test_relaxation_gap_below_one_percent_on_the_tiny_workload():
    """The paper reports the rounded solution typically within 1 % of the
    optimal energy; the dual energy bounds the optimum from below."""
    import oracle
    from workloads import make_config
    w = make_config(0)
    masks, _, _ = oracle.full_masks(w)
    ll = oracle.label_loglik(w.rgb, masks, w.k, w.sample_pix, w.sample_label, w.L)
    f = sg.data_term(ll, w.H, w.W)
    g, _ = sg.edge_weight(w.rgb)
    r = sg.solve(f, g, lam=1.0, iterations=600)
    assert (r["binary"] - r["dual"]) <= 0.01 * abs(r["dual"]), (r["binary"], r["dual"])
    # the boundary term helps: the segmentation agrees better with the regions
    # than the pointwise most likely label
    d0 = sg.dice(np.argmax(ll, 1).reshape(w.H, w.W), w.region, w.L).mean()
    d1 = sg.dice(r["labels"], w.region, w.L).mean()
    assert d1 >= d0


def test_dice_closed_form():
    a = np.array([[0, 0, 1], [1, 1, 2]])
    b = np.array([[0, 1, 1], [1, 2, 2]])
    np.testing.assert_allclose(sg.dice(a, b, 3), [2 * 1 / 3, 2 * 2 / 6, 2 * 1 / 3])


def test_two_iterations_worked_by_hand():
    """Iterates of the scheme itself (over-relaxation and the K_g clip
    included), not only its fixed point: tests/golden/primal_dual_1x2.txt."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "primal_dual_1x2.txt")
    rows = np.loadtxt(path, comments="#")
    f = np.array([[[0.0, 2.0]], [[1.0, 0.0]]])
    g = np.ones((1, 2))
    for lam, *u2 in rows:
        r = sg.solve(f, g, lam=lam, iterations=2)
        assert np.array_equal(r["u"].reshape(2, 2), np.array(u2).reshape(2, 2)), (lam, r["u"])
