"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check that
the pins catch every one of them: a dropped term, a wrong sign, a transposed
operand, a wrong index."""

from __future__ import annotations

import importlib
import os
import shutil
import sys

import numpy as np
import pytest

from oracle.dense import solve_nullspace
from oracle.gradients import fd_directional_corrected, random_direction
from tests._util import problem_family, rel_err, tiny_problem

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")

MUTATIONS = [
    ("relations.py", "[np.zeros((rbc.rows, n_a)), rbc.R]])", "[np.zeros((rbc.rows, n_a)), -rbc.R]])"),
    ("relations.py", "Gm = np.block([[A, -np.eye(n1)], [E, np.zeros((k, n1))]])",
     "Gm = np.block([[A, np.eye(n1)], [E, np.zeros((k, n1))]])"),
    ("relations.py", "return Vt[:r].copy(), beta[:r] / s[:r], consistent",
     "return Vt[:r].copy(), beta[:r] * s[:r], consistent"),
    ("relations.py", "Fm = np.vstack([rab.R, rbc.L])", "Fm = np.vstack([rab.R, rbc.L * 0.5])"),
    ("sequential.py", "res.cbar.append(S1 @ (A @ t + B @ y + c - t1))", "res.cbar.append(S1 @ (A @ t + B @ y + c))"),
    ("sequential.py", "res.t.append(-H.T @ h)", "res.t.append(H.T @ h)"),
    ("sequential.py", "res.kappa.append(float(0.5 * t @ Q @ t + q @ t + 0.5 * y @ R @ y + rz @ y))",
     "res.kappa.append(float(0.5 * t @ Q @ t + 0.5 * y @ R @ y + rz @ y))"),
    ("sequential.py", "res.qbar.append(qz + Mz @ y + Y.T @ (R @ y + rz))", "res.qbar.append(qz + Mz @ y + Y.T @ (R @ y))"),
    ("sequential.py", "Hux = res.Mbar[i].T + Bb.T @ Pn @ Ab", "Hux = Bb.T @ Pn @ Ab"),
    ("sequential.py", "p[i] = res.qbar[i] + Ab.T @ (Pn @ cb + pn) + Hux.T @ kg[i]",
     "p[i] = res.qbar[i] + Ab.T @ (Pn @ cb) + Hux.T @ kg[i]"),
    ("sequential.py", "Phi = np.vstack([E @ T, H1 @ A @ T])", "Phi = np.vstack([E @ T, H1 @ A.T @ T])"),
    ("sequential.py", "Qz = T.T @ Q @ T", "Qz = T.T @ Q.T @ T + 0.0 * T.T @ T"),  # control: semantically identical
    ("multipliers.py", "B.append(prob.E[i].T.copy()); c.append(gx[i].copy())",
     "B.append(-prob.E[i].T.copy()); c.append(gx[i].copy())"),
    ("multipliers.py", "E.append(prob.B[i].T.copy()); F.append(prob.F[i].T.copy()); g.append(gu[i].copy())",
     "E.append(prob.B[i].T.copy()); F.append(prob.F[i].T.copy()); g.append(-gu[i].copy())"),
    ("multipliers.py", "gx.append(prob.Q[N] @ x[N] + prob.q[N])", "gx.append(prob.Q[N] @ x[N])"),
    ("multipliers.py", "lam[N - j + 1] = sol.x[j]", "lam[N - j + 1] = sol.x[j] * (1.0 if j > 1 else -1.0)"),
    ("residual.py", "sx = gx - lam[i] + prob.A[i].T @ lam[i + 1] + prob.E[i].T @ mu[i]",
     "sx = gx + lam[i] + prob.A[i].T @ lam[i + 1] + prob.E[i].T @ mu[i]"),
    ("residual.py", "den = max(1.0, _inf(E[j]), _inf(F[j]), abs(float(g[j])))", "den = max(1.0, _inf(E[j]), _inf(F[j]))"),
    ("gradients.py", "G[\"A\"] = [np.outer(lam[i + 1], ax[i]) + np.outer(al[i + 1], x[i]) for i in range(N)]",
     "G[\"A\"] = [np.outer(ax[i], lam[i + 1]) + np.outer(al[i + 1], x[i]) for i in range(N)]"),
    ("gradients.py", "G[\"c\"] = [al[i + 1].copy() for i in range(N)]", "G[\"c\"] = [al[i].copy() for i in range(N)]"),
    ("gradients.py", "G[\"x0\"] = al[0].copy()", "G[\"x0\"] = -al[0].copy()"),
    ("dense.py", "b[ao:ao + nx[0]] = -prob.x0", "b[ao:ao + nx[0]] = prob.x0"),
]

# mutations that do not change any value: they must NOT be flagged.  The second
# drops S_{i+1} t_{i+1} from c-bar, which vanishes for S = T^T and the
# minimum-norm t (t lies in range(H^T), orthogonal to range(T)).
EQUIVALENT = {("sequential.py", "Qz = T.T @ Q @ T"),
              ("sequential.py", "res.cbar.append(S1 @ (A @ t + B @ y + c - t1))")}


def _load_mutant(tmp_path, fname, old, new):
    pkg = f"oracle_mut_{abs(hash((fname, old, new))) % 10**8}"
    dst = tmp_path / pkg
    shutil.copytree(ORACLE_DIR, dst, ignore=shutil.ignore_patterns("__pycache__"))
    src = (dst / fname).read_text()
    assert old in src, (fname, old)
    (dst / fname).write_text(src.replace(old, new, 1))
    sys.path.insert(0, str(tmp_path))
    try:
        return importlib.import_module(pkg)
    finally:
        sys.path.remove(str(tmp_path))


def _pins_hold(mod) -> bool:
    fam = dict(problem_family())
    try:
        for name in ("mixed-state-0", "redundant-1", "varying-dims", "with-M"):
            p = fam[name]
            # the battery pins the reversed-time route; the LSQR fallback has pins of its own
            s = mod.solve_with_multipliers(p, lsqr_fallback=False)
            if s["status"] != "ok":
                return False
            ref = solve_nullspace(p)
            for key, tol in (("x", 1e-9), ("u", 1e-9), ("lam", 1e-7), ("mu", 1e-7)):
                if rel_err(s[key], ref[key]) > tol:
                    return False
            sq = s["seq"]
            if abs(sq.objective - (sq.reduced_objective + sum(sq.kappa))) > 1e-8 * max(1, abs(sq.objective)):
                return False
            r = mod.kkt_residual(p, ref["x"], ref["u"], ref["lam"], ref["mu"])
            if r["total"] > 1e-8:
                return False
            d = mod.solve_dense(p)
            if rel_err(d["x"], ref["x"]) > 1e-9 or rel_err(d["lam"], ref["lam"]) > 1e-7:
                return False
        # Proposition 1: a balanced parenthesisation gives the same suffix sets
        rel_mod = importlib.import_module(mod.__name__ + ".relations")
        p = fam["state-heavy"]
        sq = mod.solve_sequential(p, keep_relations=True)

        def tree(lo, hi):
            if hi - lo == 1:
                return sq.relations[lo]
            mid = (lo + hi) // 2
            return rel_mod.compose(tree(lo, mid), tree(mid, hi))
        for i in range(p.N + 1):
            if not rel_mod.same_set(tree(i, p.N + 1), sq.suffix[i], tol=1e-9):
                return False
        # residual normalisation
        p = fam["random-g-mixed"].copy()
        ref = solve_nullspace(p)
        p.g[p.N] = p.g[p.N] + 5.0
        r = mod.kkt_residual(p, ref["x"], ref["u"], ref["lam"], ref["mu"])
        EN, gN, xN = p.E[p.N], p.g[p.N], ref["x"][p.N]
        expect = max(abs(EN[j] @ xN + gN[j]) / max(1.0, np.abs(EN[j]).max(), abs(gN[j]))
                     for j in range(EN.shape[0]))
        if abs(r["equality"] - expect) > 1e-9:
            return False
        # gradients
        from oracle.gradients import sumsq_loss_grad
        p = tiny_problem(600, N=6, n=4, m=3, kinds=[["mixed"]] * 6, terminal_rows=1, g_mode="random")
        sol = mod.solve_with_multipliers(p, lsqr_fallback=False)
        if sol["status"] != "ok":
            return False
        gx, gu = sumsq_loss_grad(sol["x"], sol["u"])
        grad = importlib.import_module(mod.__name__ + ".gradients")
        G = grad.adjoint_gradients(p, sol, gx, gu)
        rng = np.random.default_rng(2)
        for fields in (("A",), ("c",), ("x0",), ("Q", "q", "R", "r", "B", "E", "F", "g", "M")):
            d = random_direction(p, rng, fields)
            an = grad.directional(G, d)
            fd = fd_directional_corrected(p, solve_nullspace(p), d, 1e-6)
            if abs(fd - an) > 1e-6 * max(abs(fd), abs(an), 1e-3):
                return False
    except Exception:
        return False
    return True


def test_unmutated_oracle_passes_battery():
    import oracle
    assert _pins_hold(oracle)


@pytest.mark.parametrize("fname,old,new", MUTATIONS, ids=[f"{m[0]}:{i}" for i, m in enumerate(MUTATIONS)])
def test_mutation_is_caught(tmp_path, fname, old, new):
    mod = _load_mutant(tmp_path, fname, old, new)
    held = _pins_hold(mod)
    if (fname, old) in EQUIVALENT:
        assert held
    else:
        assert not held, f"planted mistake in {fname} not caught: {new}"
