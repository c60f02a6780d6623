"""Deformation graph with the gravity term (Section V, eqs. (10)-(17)) (TEST INFRASTRUCTURE).

Nodes l = 0..N-1 sit at positions g_l and carry a 3x3 matrix A_l (the
paper's node "rotation", kept orthonormal by E_rot only) and a translation
t_l.  Readings of what the paper leaves to its base system:

* influence of the nodes on a point v: its K = 4 nearest nodes (Euclidean
  distance, ties by index), with weights w_k = (1 - |v - g_k| / d_max)^2,
  d_max the distance of the (K+1)-th nearest node, normalised to sum to one
  (equal weights if they all vanish); the deformation is
  phi(v) = sum_k w_k (A_k (v - g_k) + g_k + t_k);
* the neighbours N(l) of a node in E_reg: its K nearest other nodes;
* E_rot = sum_l |A_l^T A_l - I|_F^2 as written (all nine entries);
* E_reg, E_con, E_pin, E_rel and E_imu as written in eqs. (11)-(15), with
  the vision-world gravity g_W given;
* E_loc = w_f E_rot + w_r E_reg + w_c (E_con + E_pin) + w_i E_imu, E_glo
  adds w_c E_rel; w_f = 1, w_r = 10, w_c = w_i = 100 (eqs. (16), (17));
* minimised by Gauss-Newton from A = I, t = 0 for a fixed number of steps,
  each step solving the normal equations by Cholesky.

Everything is float64; the Jacobians are the analytic derivatives of the
residuals below (pinned against central differences in the tests).
"""
from __future__ import annotations

import numpy as np

K_NEAREST = 4
W_ROT, W_REG, W_CON, W_IMU = 1.0, 10.0, 100.0, 100.0


def nearest(nodes, v, k, exclude=-1):
    """Indices of the k nearest nodes to v (ties by index), skipping `exclude`, and the distance of the
    next one (d_max)."""
    d = np.linalg.norm(nodes - v, axis=1)
    idx = np.arange(len(nodes))
    keep = idx != exclude
    d, idx = d[keep], idx[keep]
    order = np.lexsort((idx, d))
    return idx[order[:k]], d[order[:k]], d[order[k]]


def influence(nodes, v, k=K_NEAREST):
    """(node indices, weights) of point v."""
    idx, d, dmax = nearest(nodes, v, k)
    w = (1.0 - d / dmax) ** 2
    s = w.sum()
    w = w / s if s > 0 else np.full(k, 1.0 / k)
    return idx, w


def node_neighbours(nodes, k=K_NEAREST):
    return np.array([nearest(nodes, nodes[l], k, exclude=l)[0] for l in range(len(nodes))], dtype=np.int64)


def _phi_rows(nodes, idx, w, v, N):
    """phi(v) as J x + c: (3 x 12N) matrix J and offset c for x = [A_l (9, row-major), t_l (3)]_l."""
    J = np.zeros((3, 12 * N))
    c = np.zeros(3)
    for k, wk in zip(idx, w):
        dv = v - nodes[k]
        for r in range(3):
            J[r, 12 * k + 3 * r:12 * k + 3 * r + 3] += wk * dv
            J[r, 12 * k + 9 + r] += wk
        c += wk * nodes[k]
    return J, c


def residuals(x, prob):
    """List of (weight, residual vector, Jacobian rows) of every term at parameters x (12N)."""
    nodes, N = prob["nodes"], len(prob["nodes"])
    A = x.reshape(N, 12)[:, :9].reshape(N, 3, 3)
    out = []
    for l in range(N):  # E_rot
        r = (A[l].T @ A[l] - np.eye(3)).ravel()
        J = np.zeros((9, 12 * N))
        for i in range(3):
            for j in range(3):
                for a in range(3):
                    J[3 * i + j, 12 * l + 3 * a + j] += A[l][a, i]   # d/dA_aj of A_ai A_aj
                    J[3 * i + j, 12 * l + 3 * a + i] += A[l][a, j]   # d/dA_ai
        out.append((W_ROT, r, J))
    for l in range(N):  # E_reg
        for n in prob["neighbours"][l]:
            d = nodes[n] - nodes[l]
            r = A[l] @ d + nodes[l] + x[12 * l + 9:12 * l + 12] - (nodes[n] + x[12 * n + 9:12 * n + 12])
            J = np.zeros((3, 12 * N))
            for a in range(3):
                J[a, 12 * l + 3 * a:12 * l + 3 * a + 3] = d
                J[a, 12 * l + 9 + a] = 1.0
                J[a, 12 * n + 9 + a] -= 1.0
            out.append((W_REG, r, J))
    for (s, d), (si, sw) in zip(prob["con"], prob["con_inf"]):  # E_con
        Jp, c = _phi_rows(nodes, si, sw, s, N)
        out.append((W_CON, Jp @ x + c - d, Jp))
    for d, (di, dw) in zip(prob["pin"], prob["pin_inf"]):  # E_pin
        Jp, c = _phi_rows(nodes, di, dw, d, N)
        out.append((W_CON, Jp @ x + c - d, Jp))
    if prob.get("global", False):
        for (s, d), (si, sw), (di, dw) in zip(prob["rel"], prob["rel_src_inf"], prob["rel_dst_inf"]):  # E_rel
            Js, cs = _phi_rows(nodes, si, sw, s, N)
            Jd, cd = _phi_rows(nodes, di, dw, d, N)
            out.append((W_CON, (Js @ x + cs) - (Jd @ x + cd), Js - Jd))
    g = prob["g_W"]
    for l in range(N):  # E_imu
        r = A[l] @ g - g
        J = np.zeros((3, 12 * N))
        for a in range(3):
            J[a, 12 * l + 3 * a:12 * l + 3 * a + 3] = g
        out.append((W_IMU, r, J))
    return out


def energy(x, prob):
    return float(sum(w * r @ r for w, r, _ in residuals(x, prob)))


def problem(nodes, con=(), pin=(), rel=(), g_W=(0.0, 0.0, -9.81), global_=False):
    """A problem with its influences and node neighbours precomputed: con and rel are (source, destination)
    pairs, pin destination points (all 3-vectors)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    con = [(np.asarray(s, float), np.asarray(d, float)) for s, d in con]
    pin = [np.asarray(d, float) for d in pin]
    rel = [(np.asarray(s, float), np.asarray(d, float)) for s, d in rel]
    return {"nodes": nodes, "neighbours": node_neighbours(nodes), "con": con, "pin": pin, "rel": rel,
            "con_inf": [influence(nodes, s) for s, _ in con], "pin_inf": [influence(nodes, d) for d in pin],
            "rel_src_inf": [influence(nodes, s) for s, _ in rel], "rel_dst_inf": [influence(nodes, d) for _, d in rel],
            "g_W": np.asarray(g_W, dtype=np.float64), "global": bool(global_)}


def identity_params(N):
    x = np.zeros(12 * N)
    for l in range(N):
        x[12 * l:12 * l + 9] = np.eye(3).ravel()
    return x


def solve(prob, iters=5, x0=None):
    """Gauss-Newton from A = I, t = 0 (or x0): returns the parameters after `iters` steps."""
    N = len(prob["nodes"])
    x = identity_params(N) if x0 is None else np.array(x0, dtype=np.float64)
    for _ in range(iters):
        H = np.zeros((12 * N, 12 * N))
        b = np.zeros(12 * N)
        for w, r, J in residuals(x, prob):
            H += w * J.T @ J
            b -= w * J.T @ r
        L = np.linalg.cholesky(H)
        x = x + np.linalg.solve(L.T, np.linalg.solve(L, b))
    return x


def deform(x, prob, v):
    """phi(v) at parameters x."""
    idx, w = influence(prob["nodes"], np.asarray(v, float))
    J, c = _phi_rows(prob["nodes"], idx, w, np.asarray(v, float), len(prob["nodes"]))
    return J @ x + c


def deform_surfels(x, prob, pos, nrm):
    """Deformed surfel positions and normals (float32 arrays N x 3 in, float32 out): p' = phi(p) and
    n' = normalised sum_k w_k A_k n over p's influence, evaluated in float64 and rounded once."""
    nodes, N = prob["nodes"], len(prob["nodes"])
    A = x.reshape(N, 12)[:, :9].reshape(N, 3, 3)
    t = x.reshape(N, 12)[:, 9:]
    P = np.empty_like(pos)
    Q = np.empty_like(nrm)
    for i, (v, n) in enumerate(zip(pos.astype(np.float64), nrm.astype(np.float64))):
        idx, w = influence(nodes, v)
        P[i] = sum(wk * (A[k] @ (v - nodes[k]) + nodes[k] + t[k]) for k, wk in zip(idx, w))
        m = sum(wk * (A[k] @ n) for k, wk in zip(idx, w))
        ln = np.linalg.norm(m)
        Q[i] = m / ln if ln > 0 else n
    return P.astype(np.float32), Q.astype(np.float32)
