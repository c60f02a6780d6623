"""Pins of the oracle's FP32 pyramid mirror (pyramid reading of Section IV-D)."""
import json
import os

import numpy as np
import torch

from oracle import pyramid as pyr
from synth.scene import Scene, render

GOLD = os.path.join(os.path.dirname(__file__), "golden", "pyramid_hand.json")


def test_hand_computed_2x2_means():
    g = json.load(open(GOLD))
    D, I = pyr.level0(np.array(g["depth"], np.float32), np.array(g["intensity"], np.uint8))
    D1, I1 = pyr.downsample(D, I)
    assert np.array_equal(D1, np.array(g["depth_level1"], np.float32))
    assert np.array_equal(I1, np.array(g["intensity_level1"], np.float32))
    c = g["camera"]
    assert list(pyr.intrinsics(c["fx"], c["fy"], c["cx"], c["cy"], 1)) == g["intrinsics_level1"]
    assert list(pyr.intrinsics(c["fx"], c["fy"], c["cx"], c["cy"], 2)) == g["intrinsics_level2"]


def test_invalid_depth_inputs_are_cleaned():
    d = np.array([[np.nan, -1.0], [np.inf, 2.0]], np.float32)
    D, _ = pyr.level0(d, np.zeros((2, 2), np.uint8))
    assert np.array_equal(D, np.array([[0, 0], [0, 2.0]], np.float32))


def test_vertices_lie_on_the_rendered_plane_and_normals_match():
    # a tilted plane n.x = -2 seen by a camera at the origin of I = C
    n = np.array([0.3, -0.4, -1.0])
    n /= np.linalg.norm(n)
    sc = Scene(planes=[(n, -2.0)], spheres=[], seed=1)
    z, _ = render(sc, np.eye(3), np.zeros(3), 64, 48, 52.0, 52.0, 32.0, 24.0)
    P = pyr.build(z.numpy(), np.zeros((48, 64), np.uint8), 52.0, 52.0, 32.0, 24.0, levels=1)[0]
    V = P["V"].astype(np.float64)
    assert np.abs(V @ n + 2.0).max() < 2e-6          # on the plane, to float32 rounding
    N = P["N"][:-1, :-1].astype(np.float64)
    # forward-difference cross product points away from the camera (+z-ish), i.e. along -n
    assert np.abs(N @ (-n) - 1.0).max() < 1e-5
    assert np.all(P["N"][-1, :] == 0) and np.all(P["N"][:, -1] == 0)


def test_fronto_parallel_plane_normal_is_plus_z():
    D = np.full((6, 8), 1.5, np.float32)
    P = pyr.build(D, np.zeros((6, 8), np.uint8), 10.0, 10.0, 4.0, 3.0, levels=1)[0]
    assert np.array_equal(P["N"][:-1, :-1, 2], np.ones((5, 7), np.float32))
    assert np.all(P["N"][:-1, :-1, :2] == 0)


def test_gradient_of_a_ramp_is_its_slope():
    jj, ii = np.mgrid[0:6, 0:8].astype(np.float32)
    I = 3 * ii + 5 * jj
    G = pyr.gradient_map(I)
    assert np.all(G[1:-1, 1:-1, 0] == 3) and np.all(G[1:-1, 1:-1, 1] == 5)
    assert np.all(G[0] == 0) and np.all(G[:, 0] == 0) and np.all(G[-1] == 0) and np.all(G[:, -1] == 0)


def test_normal_invalid_next_to_a_hole():
    D = np.full((6, 8), 2.0, np.float32)
    D[2, 3] = 0
    N = pyr.normal_map(pyr.vertex_map(D, 10.0, 10.0, 4.0, 3.0), D)
    for (j, i) in [(2, 3), (2, 2), (1, 3)]:  # the hole, its left and upper neighbours
        assert np.all(N[j, i] == 0)
    assert N[3, 3, 2] == 1.0
