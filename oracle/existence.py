"""Existence and uniqueness of the minimiser for arbitrary symmetric costs
(TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``).

Section II (the paragraph after eq. (convexity)): the reduction holds for any
symmetric quadratic costs; in minimal affine coordinates of the feasible
trajectories, a minimiser exists exactly when the Hessian there is positive
semidefinite and the linear term is orthogonal to its null space, and it is
unique exactly when that Hessian is positive definite.  This module states
that definition plainly on the dense problem:

    feasible trajectories  w = w_p + W zeta,  W an orthonormal basis of null(J),
    reduced Hessian        H_r = W' H W,
    reduced linear term    g_r = W' (H w_p + h),

and classifies by the eigenvalues of H_r.
"""

from __future__ import annotations

from typing import Dict

import numpy as np

from .dense import dense_kkt, split_primal

EIG_TOL = 1e-9  # eigenvalues within EIG_TOL * max(1, |largest|) of zero count as zero


def classify(prob, tol: float = EIG_TOL, rcond: float = 1e-12) -> Dict:
    """{"kind": "infeasible" | "unbounded" | "not_unique" | "unique", the
    reduced eigenvalues, and for "unbounded" a feasible direction d along
    which the objective decreases without bound, for "not_unique" a feasible
    direction d along which it is constant, and for the existing cases one
    minimiser w}."""
    import scipy.linalg as sla
    H, h, J, b, layout = dense_kkt(prob)
    wp = -np.linalg.pinv(J, rcond=rcond) @ b
    if np.linalg.norm(J @ wp + b) > 1e-8 * max(1.0, np.linalg.norm(b)):
        return {"kind": "infeasible"}
    W = sla.null_space(J, rcond=rcond)
    Hr = W.T @ H @ W
    Hr = 0.5 * (Hr + Hr.T)
    gr = W.T @ (H @ wp + h)
    lam, V = np.linalg.eigh(Hr)
    scale = max(1.0, float(np.max(np.abs(lam), initial=0.0)))
    out = {"eigenvalues": lam, "layout": layout}
    if lam.size and lam[0] < -tol * scale:
        out.update(kind="unbounded", direction=W @ V[:, 0])
        return out
    zero = np.abs(lam) <= tol * scale
    if np.any(zero):
        Nz = V[:, zero]
        resid = Nz.T @ gr
        gscale = max(1.0, float(np.linalg.norm(gr)))
        if np.linalg.norm(resid) > tol * gscale:
            # a null direction with a nonzero slope: linear decrease without bound
            k = int(np.argmax(np.abs(resid)))
            d = W @ Nz[:, k]
            out.update(kind="unbounded", direction=-np.sign(resid[k]) * d)
            return out
        pos = ~zero
        zeta = -V[:, pos] @ ((V[:, pos].T @ gr) / lam[pos])
        out.update(kind="not_unique", direction=W @ Nz[:, 0], w=wp + W @ zeta)
        return out
    zeta = -np.linalg.solve(Hr, gr)
    out.update(kind="unique", w=wp + W @ zeta)
    return out


def objective_dense(prob, w) -> float:
    H, h, J, b, layout = dense_kkt(prob)
    return float(0.5 * w @ H @ w + h @ w)


def as_trajectory(prob, cls: Dict) -> Dict:
    """x, u blocks of the minimiser of an existing case."""
    return split_primal(prob, cls["w"], cls["layout"])
