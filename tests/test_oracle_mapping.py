"""Pins of the surfel-map oracle (fusion and model-view prediction) against
closed forms and invariants: back-projected pixels land on their own pixel,
the nearest surfel (then the lowest index) wins a cell, a fronto-parallel
plane renders its own depth exactly, repeated and offset observations average
with the stated weights, and capacity and association limits hold."""
import numpy as np

from oracle import mapping as M
from oracle import pyramid as pyr

W, H = 48, 36
CAM = (40.0, 40.0, 24.0, 18.0)  # fx, fy, cx, cy (level 0)


def _frame(depth, inten=None):
    if inten is None:
        inten = (np.arange(W * H) % 251).reshape(H, W).astype(np.uint8)
    levels = pyr.build(depth.astype(np.float32), inten, *CAM, 2)
    I16 = (levels[0]["I"] * np.float32(64.0)).astype(np.uint16)
    return levels[0]["V"], M.fusion_normals(levels), I16


def _plane(Z):
    return np.full((H, W), Z, dtype=np.float32)


def _valid(V, N):
    return (V[..., 2] > 0) & np.any(N != 0, axis=-1)


def test_first_frame_creates_one_surfel_per_valid_pixel_in_pixel_order():
    depth = _plane(2.0)
    depth[5:9, 10:20] = 0.0  # a hole
    V, N, I16 = _frame(depth)
    T = np.eye(4)
    T[:3, 3] = [0.3, -0.2, 0.1]
    m, dropped = M.fuse(M.empty_map(), V, N, I16, T, CAM, W, H, capacity=10**6)
    ok = _valid(V, N).ravel()
    assert dropped == 0 and len(m["px"]) == ok.sum()
    P = V.reshape(-1, 3)[ok].astype(np.float64) + T[:3, 3]  # identity rotation
    assert np.abs(np.stack([m["px"], m["py"], m["pz"]], 1) - P).max() < 1e-6
    assert np.allclose(m["nz"], 1.0) and np.all(m["conf"] >= 0.5) and np.all(m["conf"] <= 1.0)


def test_index_map_marks_back_projected_pixels_nearest_then_lowest_index():
    fx, fy, cx, cy = CAM
    pts = []
    for (u, v, z) in [(3, 4, 2.0), (10, 7, 1.5), (10, 7, 1.2), (20, 20, 3.0), (20, 20, 3.0)]:
        pts.append(((u - cx) / fx * z, (v - cy) / fy * z, z))
    pts = np.array(pts, dtype=np.float32)
    m = M.empty_map()
    for k, f in enumerate(("px", "py", "pz")):
        m[f] = pts[:, k].copy()
    for f, val in (("nx", 0.0), ("ny", 0.0), ("nz", 1.0), ("inten", 10.0), ("radius", 0.01), ("conf", 1.0)):
        m[f] = np.full(len(pts), val, dtype=np.float32)
    _, _, D_cw, t_cw = M.transforms(np.eye(4))
    idx = M.index_map(m, D_cw, t_cw, CAM, W, H)
    s = lambda u, v: int(idx[v, u] & np.uint64(0xFFFFFFFF))
    assert s(3, 4) == 0
    assert s(10, 7) == 2          # the nearer of two on one ray
    assert s(20, 20) == 3         # equal depth: the lower index
    assert (idx != M.EMPTY).sum() == 3


def test_fusion_normals_are_the_level1_parents():
    depth = (2.0 + 0.01 * np.random.default_rng(2).random((H, W))).astype(np.float32)
    levels = pyr.build(depth, np.zeros((H, W), np.uint8), *CAM, 2)
    Nf = M.fusion_normals(levels)
    assert np.array_equal(Nf[7, 9], levels[1]["N"][3, 4]) and np.array_equal(Nf[6, 8], levels[1]["N"][3, 4])
    assert np.array_equal(M.fusion_normals(levels[:1]), levels[0]["N"])


def test_render_front_surface_prefers_the_central_surfel_within_the_band():
    """Two surfels cover a pixel: one 1 cm nearer but off-centre, one centred.  Within a 3 cm band the
    centred one wins; with a 5 mm band only the nearer one is in the front surface."""
    fx, fy, cx, cy = CAM
    m = M.empty_map()
    # surfel 0: centred on pixel (20, 15) at 2.00 m; surfel 1: centred one pixel left at 1.99 m
    pts = [((20 - cx) / fx * 2.0, (15 - cy) / fy * 2.0, 2.0), ((19 - cx) / fx * 1.99, (15 - cy) / fy * 1.99, 1.99)]
    for k, f in enumerate(("px", "py", "pz")):
        m[f] = np.array([p[k] for p in pts], dtype=np.float32)
    for f, vals in (("nx", (0, 0)), ("ny", (0, 0)), ("nz", (1, 1)), ("inten", (10, 200)), ("radius", (0.08, 0.08)),
                    ("conf", (1, 1))):
        m[f] = np.array(vals, dtype=np.float32)
    d, i = M.render(m, np.eye(4), CAM, W, H, band=0.03)
    assert i[15, 20] == 10 and d[15, 20] == np.float32(2.0)
    d, i = M.render(m, np.eye(4), CAM, W, H, band=0.005)
    assert i[15, 20] == 200 and d[15, 20] == np.float32(1.99)


def test_plane_renders_its_own_depth_and_intensity():
    V, N, I16 = _frame(_plane(2.0), np.full((H, W), 77, dtype=np.uint8))
    m, _ = M.fuse(M.empty_map(), V, N, I16, np.eye(4), CAM, W, H, capacity=10**6)
    depth, inten = M.render(m, np.eye(4), CAM, W, H)
    ok = _valid(V, N)
    assert np.all(depth[ok] == np.float32(2.0))
    assert np.all(inten[ok] == 77)
    _, _, nrm = M.render(m, np.eye(4), CAM, W, H, with_normals=True)
    assert np.all(nrm[ok] == np.array([0, 0, 1], dtype=np.float32))
    assert np.all(nrm[depth == 0] == 0)
    # every pixel of the plane shows its own surfel: the most central of the equally near ones
    V2, N2, I2 = _frame(_plane(2.0))
    m2, _ = M.fuse(M.empty_map(), V2, N2, I2, np.eye(4), CAM, W, H, capacity=10**6)
    _, inten2 = M.render(m2, np.eye(4), CAM, W, H)
    assert np.array_equal(inten2[ok], (I2[ok] // 64).astype(np.uint8))
    # camera moved 0.25 m towards the plane: depth 1.75 wherever covered, and the centre is covered
    T = np.eye(4)
    T[2, 3] = 0.25
    depth2, _ = M.render(m, T, CAM, W, H)
    cov = depth2 > 0
    assert cov[H // 2 - 5:H // 2 + 5, W // 2 - 5:W // 2 + 5].all()
    assert np.all(depth2[cov] == np.float32(1.75))


def test_repeated_and_offset_observations_average_with_their_weights():
    V, N, I16 = _frame(_plane(2.0))
    m1, _ = M.fuse(M.empty_map(), V, N, I16, np.eye(4), CAM, W, H, capacity=10**6)
    n1 = len(m1["px"])
    # the same frame again: every pixel finds its own surfel, nothing new, confidence doubles
    m2, _ = M.fuse(m1, V, N, I16, np.eye(4), CAM, W, H, capacity=10**6)
    assert len(m2["px"]) == n1
    assert np.array_equal(m2["conf"], m1["conf"] * np.float32(2.0))
    assert np.abs(m2["pz"] - m1["pz"]).max() <= 2e-7 * 2.0
    # a plane 1 cm further (inside the 5 cm gate) with the same weights: the surfels move half way
    V3, N3, I3 = _frame(_plane(2.01))
    m3, _ = M.fuse(m1, V3, N3, I3, np.eye(4), CAM, W, H, capacity=10**6)
    assert len(m3["px"]) == n1
    assert np.abs(m3["pz"] - 2.005).max() < 1e-6
    # 20 cm further (outside the gate): no association, every pixel is a new surfel
    V4, N4, I4 = _frame(_plane(2.2))
    m4, _ = M.fuse(m1, V4, N4, I4, np.eye(4), CAM, W, H, capacity=10**6)
    assert len(m4["px"]) == 2 * n1 and np.array_equal(m4["pz"][:n1], m1["pz"])


def test_cells_next_to_mapped_ones_add_no_surfels():
    """A plane mapped at 2.0 m and seen again from 1.9 m: the surfel centres spread out and leave empty
    cells between them, but each has a mapped neighbour at the plane's depth, so nothing is added."""
    V, N, I16 = _frame(_plane(2.0))
    m1, _ = M.fuse(M.empty_map(), V, N, I16, np.eye(4), CAM, W, H, capacity=10**6)
    T = np.eye(4)
    T[2, 3] = 0.1
    V2, N2, I2 = _frame(_plane(1.9))
    _, _, D_cw, t_cw = M.transforms(T)
    empty = M.index_map(m1, D_cw, t_cw, CAM, W, H) == M.EMPTY
    assert empty[2:-2, 2:-2].sum() > 20  # interior cells with no surfel centre
    m2, _ = M.fuse(m1, V2, N2, I2, T, CAM, W, H, capacity=10**6)
    assert len(m2["px"]) == len(m1["px"])


def test_weight_and_radius_closed_forms():
    V, N, I16 = _frame(_plane(3.0))
    m, _ = M.fuse(M.empty_map(), V, N, I16, np.eye(4), CAM, W, H, capacity=10**6)
    fx, _, cx, cy = CAM
    ok = _valid(V, N)
    jj, ii = np.nonzero(ok)
    g2 = ((ii - cx) ** 2 + (jj - cy) ** 2) / (cx ** 2 + cy ** 2)
    assert np.abs(m["conf"] - 1.0 / (1.0 + g2)).max() < 1e-6
    assert np.abs(m["radius"] - 3.0 * np.sqrt(2.0) / fx).max() < 1e-6  # |n_z| = 1


def test_capacity_keeps_the_first_pixels():
    V, N, I16 = _frame(_plane(2.0))
    ok = _valid(V, N).ravel()
    cap = 100
    m, dropped = M.fuse(M.empty_map(), V, N, I16, np.eye(4), CAM, W, H, capacity=cap)
    assert len(m["px"]) == cap and dropped == ok.sum() - cap
    P = V.reshape(-1, 3)[ok][:cap]
    assert np.array_equal(m["px"], P[:, 0]) and np.array_equal(m["pz"], P[:, 2])


def test_rotated_pose_round_trip():
    """A tilted plane fused at a rotated, translated pose and rendered at the same pose gives back its
    depth within float32 rounding of the two transforms."""
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    fx, fy, cx, cy = CAM
    # plane n.X = d in the camera frame, n = (0.2, -0.1, 1) / |.|, d = 2: depth along pixel rays
    n = np.array([0.2, -0.1, 1.0]) / np.linalg.norm([0.2, -0.1, 1.0])
    rx, ry = (ii - cx) / fx, (jj - cy) / fy
    depth = (2.0 / (n[0] * rx + n[1] * ry + n[2])).astype(np.float32)
    V, N, I16 = _frame(depth)
    a = np.array([0.1, -0.2, 0.15])
    th = np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]]) / th
    T = np.eye(4)
    T[:3, :3] = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K
    T[:3, 3] = [0.5, -0.3, 0.2]
    m, _ = M.fuse(M.empty_map(), V, N, I16, T, CAM, W, H, capacity=10**6)
    d2, _ = M.render(m, T, CAM, W, H)
    ok = _valid(V, N)
    assert (d2[ok] > 0).all()
    assert np.abs(d2[ok] - depth[ok]).max() < 1e-4
