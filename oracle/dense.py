"""The plain definition: the KKT system of eq. (problem), assembled densely and
solved by SVD least squares.  Tiny inputs only (a few thousand unknowns).

Variables w = (x_0, u_0, x_1, u_1, ..., u_{N-1}, x_N).  Constraints, in order,
with the Lagrangian f(w) + nu^T c(w) (the sign of Section VII, where the
multiplier of x_0 - s_0 = 0 is alpha and lambda_0 = -alpha):

    x_0 - s_0 = 0                                  (alpha)
    A_i x_i + B_i u_i + c_i - x_{i+1} = 0           (lambda_{i+1})
    E_i x_i + F_i u_i + g_i = 0                     (mu_i)      i = 0..N-1
    E_N x_N + g_N = 0                               (mu_N)

The KKT system [[H, J^T], [J, 0]] [w; nu] = -[h; b] is solved with
``numpy.linalg.lstsq``.  When the Hessian is positive definite on null(J) the
primal part is unique and the minimum-norm solution carries the
minimum-norm multipliers (the null space of the KKT matrix is {0} x null(J^T)).
"""

from __future__ import annotations

from typing import Dict, List

import numpy as np


def _offsets(prob):
    N = prob.N
    nx, nu, nc = prob.nx, prob.nu, prob.nc
    xo, uo = [], []
    o = 0
    for i in range(N):
        xo.append(o); o += nx[i]
        uo.append(o); o += nu[i]
    xo.append(o); o += nx[N]
    nw = o
    # multipliers: alpha, then per stage (lambda_{i+1}, mu_i), then mu_N
    ao = 0
    lo, mo = [None] * (N + 1), [None] * (N + 1)
    o = nx[0]
    for i in range(N):
        lo[i + 1] = o; o += nx[i + 1]
        mo[i] = o; o += nc[i]
    mo[N] = o; o += nc[N]
    nnu = o
    return xo, uo, nw, ao, lo, mo, nnu


def dense_kkt(prob):
    """Return (H, h, J, b, layout) with constraints c(w) = J w + b."""
    N = prob.N
    nx, nu, nc = prob.nx, prob.nu, prob.nc
    xo, uo, nw, ao, lo, mo, nnu = _offsets(prob)
    H = np.zeros((nw, nw)); h = np.zeros(nw)
    J = np.zeros((nnu, nw)); b = np.zeros(nnu)
    for i in range(N):
        xs = slice(xo[i], xo[i] + nx[i]); us = slice(uo[i], uo[i] + nu[i])
        H[xs, xs] += prob.Q[i]; H[xs, us] += prob.M[i]; H[us, xs] += prob.M[i].T; H[us, us] += prob.R[i]
        h[xs] += prob.q[i]; h[us] += prob.r[i]
    xs = slice(xo[N], xo[N] + nx[N])
    H[xs, xs] += prob.Q[N]; h[xs] += prob.q[N]
    # x_0 - s_0 = 0
    J[ao:ao + nx[0], xo[0]:xo[0] + nx[0]] = np.eye(nx[0]); b[ao:ao + nx[0]] = -prob.x0
    for i in range(N):
        rs = slice(lo[i + 1], lo[i + 1] + nx[i + 1])
        J[rs, xo[i]:xo[i] + nx[i]] = prob.A[i]
        J[rs, uo[i]:uo[i] + nu[i]] = prob.B[i]
        J[rs, xo[i + 1]:xo[i + 1] + nx[i + 1]] = -np.eye(nx[i + 1])
        b[rs] = prob.c[i]
        rs = slice(mo[i], mo[i] + nc[i])
        J[rs, xo[i]:xo[i] + nx[i]] = prob.E[i]
        J[rs, uo[i]:uo[i] + nu[i]] = prob.F[i]
        b[rs] = prob.g[i]
    rs = slice(mo[N], mo[N] + nc[N])
    J[rs, xo[N]:xo[N] + nx[N]] = prob.E[N]
    b[rs] = prob.g[N]
    return H, h, J, b, (xo, uo, ao, lo, mo)


def split_primal(prob, w, layout) -> Dict[str, List[np.ndarray]]:
    xo, uo = layout[0], layout[1]
    N = prob.N
    x = [w[xo[i]:xo[i] + prob.nx[i]].copy() for i in range(N + 1)]
    u = [w[uo[i]:uo[i] + prob.nu[i]].copy() for i in range(N)]
    return {"x": x, "u": u}


def split_dual(prob, nu, layout) -> Dict[str, List[np.ndarray]]:
    """lam[0] = lambda_0 = -alpha, lam[i] = lambda_i; mu[i] for i = 0..N."""
    _, _, ao, lo, mo = layout
    N = prob.N
    lam = [-nu[ao:ao + prob.nx[0]].copy()]
    lam += [nu[lo[i]:lo[i] + prob.nx[i]].copy() for i in range(1, N + 1)]
    mu = [nu[mo[i]:mo[i] + prob.nc[i]].copy() for i in range(N + 1)]
    return {"lam": lam, "mu": mu}


def solve_dense(prob, rcond: float = 1e-12) -> Dict[str, list]:
    """Primal part: least-squares solution of the dense KKT system.  Multipliers:
    the minimum-norm solution of J^T nu = -(H w + h) at that primal point (the
    full-KKT least-squares multipliers are avoided because truncating the tiny
    singular values of a rank-deficient KKT matrix perturbs them)."""
    H, h, J, b, layout = dense_kkt(prob)
    nw, nnu = H.shape[0], J.shape[0]
    K = np.block([[H, J.T], [J, np.zeros((nnu, nnu))]])
    rhs = -np.concatenate([h, b])
    sol = np.linalg.lstsq(K, rhs, rcond=rcond)[0]
    w = sol[:nw]
    nu = -np.linalg.pinv(J.T, rcond=rcond) @ (H @ w + h)
    out = split_primal(prob, w, layout)
    out.update(split_dual(prob, nu, layout))
    return out


def solve_nullspace(prob, rcond: float = 1e-12) -> Dict[str, list]:
    """Independent primal route (textbook null-space method): w = w_p + N z with
    w_p = -pinv(J) b and N an orthonormal basis of null(J); z minimises the
    reduced quadratic."""
    import scipy.linalg as sla
    H, h, J, b, layout = dense_kkt(prob)
    wp = -np.linalg.pinv(J, rcond=rcond) @ b
    Nb = sla.null_space(J, rcond=rcond)
    z = -np.linalg.solve(Nb.T @ H @ Nb, Nb.T @ (H @ wp + h))
    w = wp + Nb @ z
    nu = -np.linalg.pinv(J.T, rcond=rcond) @ (H @ w + h)
    out = split_primal(prob, w, layout)
    out.update(split_dual(prob, nu, layout))
    return out


def minnorm_multipliers_dense(prob, x, u) -> Dict[str, list]:
    """Minimum-norm nu with J^T nu = -grad f(w) at the given primal point."""
    H, h, J, b, layout = dense_kkt(prob)
    w = np.concatenate([np.concatenate([x[i], u[i]]) for i in range(prob.N)] + [x[prob.N]])
    grad = H @ w + h
    nu = -np.linalg.pinv(J.T, rcond=1e-12) @ grad
    return split_dual(prob, nu, layout)


def sparse_jacobian(prob):
    """J and H, h, b of dense_kkt as scipy.sparse matrices (any size)."""
    import scipy.sparse as sp
    N = prob.N
    nx, nu, nc = prob.nx, prob.nu, prob.nc
    xo, uo, nw, ao, lo, mo, nnu = _offsets(prob)
    rows, cols, vals = [], [], []

    def put(r0, c0, M):
        M = np.asarray(M)
        if M.size == 0:
            return
        rr, cc = np.nonzero(M)
        rows.append(rr + r0); cols.append(cc + c0); vals.append(M[rr, cc])

    put(ao, xo[0], np.eye(nx[0]))
    for i in range(N):
        put(lo[i + 1], xo[i], prob.A[i]); put(lo[i + 1], uo[i], prob.B[i])
        put(lo[i + 1], xo[i + 1], -np.eye(nx[i + 1]))
        put(mo[i], xo[i], prob.E[i]); put(mo[i], uo[i], prob.F[i])
    put(mo[N], xo[N], prob.E[N])
    r = np.concatenate(rows) if rows else np.zeros(0, int)
    c = np.concatenate(cols) if cols else np.zeros(0, int)
    v = np.concatenate(vals) if vals else np.zeros(0)
    J = sp.csr_matrix((v, (r, c)), shape=(nnu, nw))
    return J, (xo, uo, ao, lo, mo)


def minnorm_multipliers_lsqr(prob, x, u, tol: float = 1e-15, maxiter: int = 200000):
    """Minimum-norm least-squares solution of J^T nu = -grad f(w) at the given
    primal point, by LSQR on the sparse J^T (started at zero, LSQR returns the
    minimum-norm solution)."""
    from scipy.sparse.linalg import lsqr
    N = prob.N
    J, layout = sparse_jacobian(prob)
    grad = []
    for i in range(N):
        grad.append(prob.Q[i] @ x[i] + prob.M[i] @ u[i] + prob.q[i])
        grad.append(prob.M[i].T @ x[i] + prob.R[i] @ u[i] + prob.r[i])
    grad.append(prob.Q[N] @ x[N] + prob.q[N])
    g = np.concatenate(grad)
    res = lsqr(J.T.tocsr(), -g, atol=tol, btol=tol, conlim=1e14, iter_lim=maxiter)
    return split_dual(prob, res[0], layout), res


def jacobian_full_row_rank(prob, rtol: float = 1e-10) -> bool:
    """LICQ by definition: the stacked constraint Jacobian J of eq. (problem)
    (rows x_0 - s_0, dynamics, stage rows, terminal rows) has full row rank,
    judged by its singular values.  Tiny inputs only."""
    _, _, J, _, _ = dense_kkt(prob)
    if J.shape[0] == 0:
        return True
    s = np.linalg.svd(J, compute_uv=False)
    return int(np.sum(s > rtol * s[0])) == J.shape[0]
