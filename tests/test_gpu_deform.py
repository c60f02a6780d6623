"""GPU deformation-graph solver (dslam_deform_*) against the oracle's
Gauss-Newton (float64): node parameters and per-step costs agree to
rounding, a yaw-rigid motion is recovered exactly, and singular or invalid
problems are refused."""
import numpy as np
import pytest

import paper_2207_10940_amd as P
from oracle import deformation as D

pytestmark = pytest.mark.gpu


def _rot(axis, deg):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    t = np.radians(deg)
    return np.eye(3) + np.sin(t) * K + (1 - np.cos(t)) * K @ K


def _case(seed, n_nodes, n_con, n_pin, n_rel):
    rng = np.random.default_rng(seed)
    nodes = rng.uniform(-1.0, 1.0, size=(n_nodes, 3)) * np.array([2.0, 2.0, 1.0])
    R, t = _rot(rng.normal(size=3), 3.0), rng.normal(size=3) * 0.05
    src = nodes[rng.integers(0, n_nodes, n_con)] + rng.normal(size=(n_con, 3)) * 0.2
    con = [(s, R @ s + t + rng.normal(size=3) * 0.01) for s in src]
    pin = list(nodes[rng.integers(0, n_nodes, n_pin)] + rng.normal(size=(n_pin, 3)) * 0.2)
    rsrc = nodes[rng.integers(0, n_nodes, n_rel)] + rng.normal(size=(n_rel, 3)) * 0.2
    rel = [(s, s + rng.normal(size=3) * 0.01) for s in rsrc]
    return nodes, con, pin, rel


# 6, 7, 13 and 37 nodes give 12 N unknowns that are not a multiple of the
# 16-column panel: a short last panel, and a residual column that shares its
# tile with node columns.
@pytest.mark.parametrize("seed,n_nodes,n_con,n_pin,n_rel,glob", [(1, 16, 40, 20, 0, False), (2, 32, 96, 64, 24, True),
                                                                  (3, 64, 256, 128, 64, True), (5, 6, 12, 6, 4, True),
                                                                  (6, 7, 20, 8, 0, False), (7, 13, 40, 16, 8, True),
                                                                  (8, 37, 100, 40, 20, True)])
def test_solve_matches_oracle(seed, n_nodes, n_con, n_pin, n_rel, glob):
    print(f"deform {n_nodes} nodes {n_con}+{n_pin}+{n_rel} points global {glob}", flush=True)
    nodes, con, pin, rel = _case(seed, n_nodes, n_con, n_pin, n_rel)
    prob = D.problem(nodes, con=con, pin=pin, rel=rel, global_=glob)
    iters = 4
    ctx = P.Context(0)
    df = P.Deform(ctx, 64, 512)
    try:
        x, cost = df.solve(nodes, con=con, pin=pin, rel=rel, global_=glob, iters=iters)
    finally:
        df.close()
        ctx.close()
    xo = D.identity_params(n_nodes)
    for it in range(iters):
        eo = D.energy(xo, prob)
        assert abs(cost[it] - eo) <= 1e-9 * max(eo, 1e-12), (it, cost[it], eo)
        xo = D.solve(prob, iters=1, x0=xo)
    assert np.abs(x.ravel() - xo).max() < 1e-9


# 24 nodes, and the largest graphs (256 nodes: 3,072 unknowns, more
# right-hand-side rows than the triangular solves have threads; 255 nodes:
# the same with a short last panel), where the exact answer needs no oracle.
@pytest.mark.parametrize("n_nodes", [24, 255, 256])
def test_yaw_rigid_motion_recovered(n_nodes):
    print(f"deform yaw {n_nodes} nodes", flush=True)
    rng = np.random.default_rng(4)
    nodes = rng.uniform(-1.0, 1.0, size=(n_nodes, 3)) * (n_nodes / 24) ** (1 / 3)
    R, t = _rot([0, 0, 1], 5.0), np.array([0.1, -0.05, 0.02])
    src = nodes + rng.normal(size=nodes.shape) * 0.1
    ctx = P.Context(0)
    df = P.Deform(ctx, max(32, n_nodes), max(64, n_nodes))
    try:
        x, cost = df.solve(nodes, con=[(s, R @ s + t) for s in src], iters=6)
    finally:
        df.close()
        ctx.close()
    for l, g in enumerate(nodes):
        assert np.abs(x[l, :9] - R.ravel()).max() < 1e-9
        assert np.abs(x[l, 9:] - (R @ g + t - g)).max() < 1e-9
    assert cost[-1] < 1e-16 * cost[0]


def test_singular_and_invalid():
    rng = np.random.default_rng(6)
    nodes = rng.uniform(-1.0, 1.0, size=(12, 3))
    ctx = P.Context(0)
    df = P.Deform(ctx, 16, 16)
    try:
        with pytest.raises(P.DslamError) as ei:  # no point constraints: the global translation is free
            df.solve(nodes, iters=2)
        assert ei.value.code == P._abi.ERR_SINGULAR
        with pytest.raises(P.DslamError):  # more nodes than the solver holds
            df.solve(rng.normal(size=(20, 3)), pin=[nodes[0]], iters=1)
        bad = nodes.copy()
        bad[3, 1] = np.inf
        with pytest.raises(P.DslamError):
            df.solve(bad, pin=[nodes[0]], iters=1)
    finally:
        df.close()
        ctx.close()


def test_map_deformation_matches_oracle():
    """A fused map deformed by a solved graph: every surfel's position and normal within float32 rounding
    of the oracle's phi (float64, rounded once)."""
    import synth
    from oracle import mapping as M
    from oracle import pyramid as pyr
    from tests.gpu_common import cuda, session
    seq = synth.configs.sequence(seed=3003, n_frames=1, width=160, height=120)
    cam = seq["camera"]
    g = seq["gt"][0]
    T = np.eye(4)
    T[:3, :3] = synth.configs._rot_from_quat(g["q"])
    T[:3, 3] = g["r"]
    rng = np.random.default_rng(9)
    with session(160, 120, 2, [1, 1], mode="rgbd") as s:
        mp = P.Map(s.ctx, cam, 10**5)
        try:
            s.build_pyramid(P.PYR_CURRENT, cuda(seq["depth"][0].numpy()), cuda(seq["intensity"][0].numpy()))
            mp.fuse(s, T)
            before = mp.arrays()
            pos = np.stack([before["px"], before["py"], before["pz"]], 1)
            nodes = pos[rng.choice(len(pos), 24, replace=False)].astype(np.float64)
            R, t = _rot([0.3, 1, 0.2], 2.0), np.array([0.02, -0.01, 0.03])
            src = pos[rng.choice(len(pos), 60, replace=False)].astype(np.float64)
            prob = D.problem(nodes, con=[(p_, R @ p_ + t) for p_ in src[:40]], pin=list(src[40:]))
            x = D.solve(prob, iters=4)
            mp.deform(nodes, x.reshape(-1, 12))
            after = mp.arrays()
        finally:
            mp.close()
    nrm = np.stack([before["nx"], before["ny"], before["nz"]], 1)
    Pw, Qw = D.deform_surfels(x, prob, pos, nrm)
    got_p = np.stack([after["px"], after["py"], after["pz"]], 1)
    got_n = np.stack([after["nx"], after["ny"], after["nz"]], 1)
    assert np.abs(got_p - Pw).max() <= 4 * np.finfo(np.float32).eps * max(1.0, np.abs(Pw).max())
    assert np.abs(got_n - Qw).max() <= 4 * np.finfo(np.float32).eps
    assert np.abs(got_p - pos).max() > 1e-3  # it moved
    for k in ("inten", "radius", "conf"):
        assert np.array_equal(after[k], before[k])
