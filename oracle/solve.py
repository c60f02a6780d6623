"""Gauss-Newton step, prior and marginalisation (Section IV-D/E, eqs. (6)-(9)), float64.

Unknowns z = [dx0 (15), dx1 (15), dg (3)] (33): per-frame tangents
[dr, dalpha, dv, dbg, dba] for the previous and current states, and one
gravity-orientation tangent dg.  Reading taken here: the paper's per-state
q_IW (eq. (1)) is kept as a single orientation shared by both states, which is
its zero-process-noise limit; the prior therefore lives on (x0, q_IW), 18-d.

* Normal equations, eq. (7): H dz = b with H = sum J^T W J and
  b = -sum J^T W e over the photometric, ICP, IMU and prior terms.
* Prior, eq. (6) with the first-order correction of eq. (9): its residual is
  (x0, q_IW) [-] xbar - H*^-1 b*, with identity Jacobian, contributing H* to H
  and b* - H* ((x0, q_IW) [-] xbar) to b (eq. (9b) with Dx = xbar [-] x).
* After the update, the system is re-expressed at the new point
  (b' = b - H dz) and x0 is eliminated by the Schur complement, eq. (8):
  H* = H11 - H10 H00^-1 H01, b* = b'1 - H10 H00^-1 b'0.
"""
from __future__ import annotations

import numpy as np

from .lie import quat_boxminus, quat_boxplus, state_boxminus, state_boxplus

X0 = slice(0, 15)
X1 = slice(15, 30)
G = slice(30, 33)
KEEP = np.r_[15:33]
POSE0 = np.r_[0:6]
POSE1 = np.r_[15:21]


def prior_terms(x0, q_IW, prior):
    """Contribution (H, b) of the marginal prior to the 33-d system."""
    delta = np.concatenate([state_boxminus(x0, prior["xbar"]), quat_boxminus(q_IW, prior["qIW_bar"])])
    Hs = prior["H"]
    bs = prior["b"] - Hs @ delta
    H = np.zeros((33, 33))
    b = np.zeros(33)
    idx = np.r_[0:15, 30:33]
    H[np.ix_(idx, idx)] = Hs
    b[idx] = bs
    return H, b


def is_spd(H) -> bool:
    try:
        np.linalg.cholesky(H)
        return True
    except np.linalg.LinAlgError:
        return False


def gn_step(H, b):
    """Solve eq. (7) for the Gauss-Newton increment."""
    return np.linalg.solve(H, b)


def apply_update(x0, x1, q_IW, dz):
    """Box-plus of the increment onto both states and the gravity orientation (Section IV-D)."""
    return state_boxplus(x0, dz[X0]), state_boxplus(x1, dz[X1]), quat_boxplus(q_IW, dz[G])


def marginalise(H, b, dz, x1, q_IW):
    """Schur complement of x0 (eq. (8)) at the updated point; returns the new prior."""
    bp = b - H @ dz
    H00 = H[X0, X0]
    H0k = H[X0, KEEP]
    Hk0 = H[KEEP, X0]
    Hkk = H[np.ix_(KEEP, KEEP)]
    Hs = Hkk - Hk0 @ np.linalg.solve(H00, H0k)
    bs = bp[KEEP] - Hk0 @ np.linalg.solve(H00, bp[X0])
    Hs = 0.5 * (Hs + Hs.T)
    return {"H": Hs, "b": bs, "xbar": {k: np.array(v).copy() for k, v in x1.items()},
            "qIW_bar": np.array(q_IW).copy()}
