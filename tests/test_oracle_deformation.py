"""Pins of the deformation-graph oracle (Section V, eqs. (10)-(17)): the
analytic Jacobians against central differences, the identity as the exact
minimiser of consistent zero-motion constraints, exact recovery of a rigid
motion about gravity (every term vanishes), the gravity term resisting a
tilt, influence weights, and a monotone energy decrease."""
import numpy as np
import pytest

from oracle import deformation as D


def _grid_nodes(n_side=3, spacing=0.5):
    g = np.arange(n_side) * spacing
    return np.array([[x, y, z] for x in g for y in g for z in g[:2]], dtype=np.float64)


def _rot(axis, deg):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    t = np.radians(deg)
    return np.eye(3) + np.sin(t) * K + (1 - np.cos(t)) * K @ K


def _rigid_params(prob, R, t):
    """Node parameters of the rigid motion v -> R v + t: A_l = R, t_l = R g_l + t - g_l."""
    x = np.zeros(12 * len(prob["nodes"]))
    for l, g in enumerate(prob["nodes"]):
        x[12 * l:12 * l + 9] = R.ravel()
        x[12 * l + 9:12 * l + 12] = R @ g + t - g
    return x


def test_influence_weights():
    nodes = _grid_nodes()
    v = nodes[4] + np.array([0.01, 0.02, 0.0])
    idx, w = D.influence(nodes, v)
    assert len(idx) == D.K_NEAREST and abs(w.sum() - 1.0) < 1e-15 and np.all(w >= 0)
    assert idx[0] == 4 and w[0] == w.max()       # the nearest node weighs most
    # a point exactly on a node, with the (K+1)-th neighbour at the lattice spacing
    idx, w = D.influence(nodes, nodes[0])
    assert idx[0] == 0


def test_jacobians_match_central_differences():
    rng = np.random.default_rng(1)
    nodes = _grid_nodes()
    src = nodes[rng.integers(0, len(nodes), 6)] + rng.normal(size=(6, 3)) * 0.05
    prob = D.problem(nodes, con=[(s, s + rng.normal(size=3) * 0.05) for s in src],
                     pin=list(nodes[:3] + 0.1), rel=[(src[0], src[1])], global_=True)
    x = D.identity_params(len(nodes)) + rng.normal(size=12 * len(nodes)) * 0.05
    terms = D.residuals(x, prob)
    h = 1e-6
    for k in rng.integers(0, len(x), 25):
        xp, xm = x.copy(), x.copy()
        xp[k] += h
        xm[k] -= h
        for (w, r, J), (_, rp, _), (_, rm, _) in zip(terms, D.residuals(xp, prob), D.residuals(xm, prob)):
            assert np.allclose((rp - rm) / (2 * h), J[:, k], atol=1e-8)


def test_identity_is_the_minimiser_of_zero_motion():
    nodes = _grid_nodes()
    pts = nodes[::3] + 0.03
    prob = D.problem(nodes, con=[(p, p) for p in pts], pin=list(nodes[1::4] - 0.02))
    x = D.solve(prob, iters=3)
    assert np.abs(x - D.identity_params(len(nodes))).max() < 1e-12
    assert D.energy(x, prob) < 1e-24


def test_rigid_motion_about_gravity_is_recovered_exactly():
    nodes = _grid_nodes()
    rng = np.random.default_rng(3)
    R, t = _rot([0, 0, 1], 4.0), np.array([0.05, -0.03, 0.02])  # yaw: the gravity term allows it
    src = nodes + rng.normal(size=nodes.shape) * 0.1
    prob = D.problem(nodes, con=[(s, R @ s + t) for s in src])
    x_star = _rigid_params(prob, R, t)
    assert D.energy(x_star, prob) < 1e-20  # every term vanishes
    x = D.solve(prob, iters=6)
    assert np.abs(x - x_star).max() < 1e-9
    for s in src[:5]:
        assert np.abs(D.deform(x, prob, s) - (R @ s + t)).max() < 1e-9


def test_gravity_term_resists_a_tilt(monkeypatch):
    nodes = _grid_nodes()
    rng = np.random.default_rng(4)
    R, t = _rot([1, 0, 0], 3.0), np.zeros(3)  # a tilt: R g != g
    src = nodes + rng.normal(size=nodes.shape) * 0.1
    prob = D.problem(nodes, con=[(s, R @ s + t) for s in src])
    g = prob["g_W"]
    x = D.solve(prob, iters=6)
    A = x.reshape(-1, 12)[:, :9].reshape(-1, 3, 3)
    tilt = max(np.linalg.norm(a @ g - g) for a in A)
    assert tilt < np.linalg.norm(R @ g - g)  # less tilted than the constraints ask
    assert D.energy(x, prob) < D.energy(_rigid_params(prob, R, t), prob)
    # without the gravity term the tilt is taken in full
    monkeypatch.setattr(D, "W_IMU", 0.0)
    x0 = D.solve(prob, iters=6)
    assert np.abs(x0 - _rigid_params(prob, R, t)).max() < 1e-9


def test_energy_decreases_over_gauss_newton_steps():
    nodes = _grid_nodes()
    rng = np.random.default_rng(5)
    src = nodes[rng.integers(0, len(nodes), 10)] + rng.normal(size=(10, 3)) * 0.1
    prob = D.problem(nodes, con=[(s, s + np.array([0.1, 0.0, 0.05]) + rng.normal(size=3) * 0.02) for s in src],
                     pin=list(nodes[-4:]))
    x = D.identity_params(len(nodes))
    e = [D.energy(x, prob)]
    for _ in range(4):
        x = D.solve(prob, iters=1, x0=x)
        e.append(D.energy(x, prob))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(e, e[1:])) and e[-1] < e[0]


@pytest.mark.parametrize("n_side,seed", [(2, 7), (3, 8)])
def test_gauss_newton_reaches_the_least_squares_minimiser(n_side, seed):
    """The converged Gauss-Newton parameters equal scipy's trust-region least-squares minimiser of the same
    weighted residuals (started from the same identity parameters).  The constraints conflict (non-zero
    residual at the minimum), where Gauss-Newton converges linearly: 60 steps."""
    from scipy.optimize import least_squares
    rng = np.random.default_rng(seed)
    g = np.arange(n_side) * 0.5
    nodes = np.array([[x, y, z] for x in g for y in g for z in (0.0, 0.4, 0.8)], dtype=np.float64)
    src = nodes[rng.integers(0, len(nodes), 8)] + rng.normal(size=(8, 3)) * 0.1
    R = _rot(rng.normal(size=3), 4.0)
    prob = D.problem(nodes, con=[(s, R @ s + np.array([0.03, -0.02, 0.01]) + rng.normal(size=3) * 0.01)
                                 for s in src],
                     pin=list(nodes[:2] + 0.05), rel=[(src[0], src[1] + 0.01)], global_=True)

    def stacked(x):
        return np.concatenate([np.sqrt(w) * r for w, r, _ in D.residuals(x, prob)])

    def jac(x):
        return np.vstack([np.sqrt(w) * J for w, _, J in D.residuals(x, prob)])

    x0 = D.identity_params(len(nodes))
    x_gn = D.solve(prob, iters=60)
    ls = least_squares(stacked, x0, jac=jac, xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=500)
    assert abs(D.energy(x_gn, prob) - 2 * ls.cost) <= 1e-12 * max(D.energy(x_gn, prob), 1e-30)
    assert np.abs(x_gn - ls.x).max() < 1e-6


def test_deform_surfels_rigid_graph_rotates_normals():
    """A graph whose nodes all carry the same rigid motion (A_l = R,
    t_l = R g_l + t - g_l) moves every surfel rigidly: p' = R p + t and
    n' = R n, whatever each surfel's influence weights.  Rotations come from
    scipy's axis-angle conversion (an independent route); a transposed A, a
    dropped weight normalisation or an affine instead of linear normal map
    fails it."""
    from scipy.spatial.transform import Rotation
    nodes = _grid_nodes(n_side=4, spacing=0.4)
    prob = D.problem(nodes, con=[(nodes[0], nodes[0])])
    rng = np.random.default_rng(12)
    R = Rotation.from_rotvec(np.radians(25.0) * np.array([0.3, -0.8, 0.52]) / np.linalg.norm([0.3, -0.8, 0.52]))
    R = R.as_matrix()
    t = np.array([0.4, -0.25, 0.1])
    x = _rigid_params(prob, R, t)
    pos = (rng.uniform(-0.1, 1.3, size=(200, 3))).astype(np.float32)
    nrm = rng.normal(size=(200, 3))
    nrm = (nrm / np.linalg.norm(nrm, axis=1, keepdims=True)).astype(np.float32)
    P, Q = D.deform_surfels(x, prob, pos, nrm)
    want_p = pos.astype(np.float64) @ R.T + t
    want_n = nrm.astype(np.float64) @ R.T
    # one float32 rounding of a float64 value: within an ulp of the float32 result
    assert np.abs(P - want_p).max() < 4 * np.finfo(np.float32).eps * np.abs(want_p).max()
    assert np.abs(Q - want_n).max() < 4 * np.finfo(np.float32).eps
    assert np.abs(np.linalg.norm(Q.astype(np.float64), axis=1) - 1.0).max() < 4 * np.finfo(np.float32).eps


def test_deform_surfels_uniform_scale_keeps_normals():
    """A_l = s I (the same uniform scaling at every node) changes no normal
    direction: n' = n after renormalisation, while positions scale about
    the nodes."""
    nodes = _grid_nodes(n_side=3, spacing=0.5)
    prob = D.problem(nodes, con=[(nodes[0], nodes[0])])
    N = len(nodes)
    x = np.zeros(12 * N)
    for l in range(N):
        x[12 * l:12 * l + 9] = (1.7 * np.eye(3)).ravel()
    rng = np.random.default_rng(5)
    pos = rng.uniform(0.0, 1.0, size=(50, 3)).astype(np.float32)
    nrm = rng.normal(size=(50, 3))
    nrm = (nrm / np.linalg.norm(nrm, axis=1, keepdims=True)).astype(np.float32)
    _, Q = D.deform_surfels(x, prob, pos, nrm)
    assert np.abs(Q - nrm).max() < 4 * np.finfo(np.float32).eps
