"""Pins of the CPU oracle against things other than itself.

* exact rational arithmetic on a tiny integer problem (Fractions Gauss-Jordan);
* the textbook null-space method and the dense KKT definition;
* special cases with closed forms (minimum-energy control via the reachability
  matrix, cost-independence when no input is free, T = I without constraints);
* Theorem 1 by brute-force suffix feasibility;
* Lemma 2, Theorem 2, Propositions 1-3 as invariants;
* infeasibility outcomes of Algorithm 1;
* minimum-norm multipliers against pinv(J^T) and the KKT residual of Section IX.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

from oracle import solve_sequential, solve_dense, solve_with_multipliers
from oracle.dense import dense_kkt, solve_nullspace, minnorm_multipliers_dense
from oracle.relations import compose, same_set, base_relation, terminal_relation, Relation
from oracle.residual import kkt_residual
from oracle.sequential import objective
from workloads.generate import Problem
from tests._util import problem_family, rel_err, tiny_problem

FAMILY = problem_family()


# ---------------------------------------------------------------------------
# exact arithmetic
# ---------------------------------------------------------------------------

def _gauss_jordan_exact(K, rhs):
    n = len(K)
    M = [[Fraction(K[i][j]) for j in range(n)] + [Fraction(rhs[i])] for i in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        pv = M[col][col]
        M[col] = [v / pv for v in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [a - f * b for a, b in zip(M[r], M[col])]
    return [M[i][n] for i in range(n)]


def _integer_problem():
    """N=3, n=2, m=2 with integer data; one mixed row per stage, one terminal
    row; the KKT matrix is nonsingular (LICQ holds)."""
    I2 = np.eye(2)
    A = [np.array([[1., 1.], [0., 1.]]), np.array([[1., 0.], [1., 1.]]), np.array([[2., 1.], [0., 1.]])]
    B = [np.array([[1., 0.], [1., 1.]]), np.array([[0., 1.], [1., 0.]]), np.array([[1., 2.], [0., 1.]])]
    c = [np.array([1., 0.]), np.array([0., -1.]), np.array([1., 1.])]
    Q = [2 * I2, np.array([[2., 1.], [1., 2.]]), I2, np.array([[3., 1.], [1., 1.]])]
    R = [I2, 2 * I2, np.array([[2., 1.], [1., 1.]])]
    M = [np.zeros((2, 2))] * 3
    q = [np.array([1., -1.]), np.array([0., 2.]), np.array([-1., 0.]), np.array([1., 1.])]
    r = [np.array([0., 1.]), np.array([1., 0.]), np.array([-1., 1.])]
    E = [np.array([[1., 0.]]), np.array([[0., 1.]]), np.array([[1., 1.]]), np.array([[1., -1.]])]
    F = [np.array([[1., 1.]]), np.array([[1., -1.]]), np.array([[0., 1.]])]
    g = [np.array([1.]), np.array([-2.]), np.array([0.]), np.array([3.])]
    x0 = np.array([1., 2.])
    return Problem(Q, q, R, r, M, A, B, c, E, F, g, x0)


def test_exact_rational_kkt():
    p = _integer_problem()
    H, h, J, b, layout = dense_kkt(p)
    nw, nn = H.shape[0], J.shape[0]
    K = np.block([[H, J.T], [J, np.zeros((nn, nn))]])
    ex = _gauss_jordan_exact(K.astype(int).tolist(), (-np.concatenate([h, b])).astype(int).tolist())
    exf = np.array([float(v) for v in ex])
    d = solve_dense(p)
    s = solve_with_multipliers(p)
    assert s["status"] == "ok"
    from oracle.dense import split_dual, split_primal
    ep = split_primal(p, exf[:nw], layout)
    ed = split_dual(p, exf[nw:], layout)
    for key, ref in (("x", ep["x"]), ("u", ep["u"]), ("lam", ed["lam"]), ("mu", ed["mu"])):
        assert rel_err(d[key], ref) < 1e-12, key
        assert rel_err(s[key], ref) < 1e-11, key


# ---------------------------------------------------------------------------
# primal: sequential method vs dense definition vs null-space method
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,p", FAMILY, ids=[f[0] for f in FAMILY])
def test_sequential_matches_dense_and_nullspace(name, p):
    s = solve_with_multipliers(p)
    assert s["status"] == "ok", s["status"]
    d = solve_dense(p)
    ns = solve_nullspace(p)
    assert rel_err(d["x"], ns["x"]) < 1e-10
    assert rel_err(s["x"], ns["x"]) < 1e-10
    assert rel_err(s["u"], ns["u"]) < 1e-10
    # canonical multipliers: minimum-norm solution of J^T nu = -grad f at the optimum
    assert rel_err(s["lam"], ns["lam"]) < 1e-10
    assert rel_err(s["mu"], ns["mu"]) < 1e-10 if sum(p.nc) else True
    r = kkt_residual(p, s["x"], s["u"], s["lam"], s["mu"])
    assert r["total"] < 1e-10, r


def test_minimum_energy_control_closed_form():
    """Q = 0, R = I, no stage rows, terminal x_N = target: the minimiser is the
    minimum-norm input of the reachability equation."""
    rng = np.random.default_rng(7)
    N, n, m = 5, 3, 1
    A = [np.eye(n) + 0.1 * rng.standard_normal((n, n)) for _ in range(N)]
    B = [rng.standard_normal((n, m)) for _ in range(N)]
    c = [0.1 * rng.standard_normal(n) for _ in range(N)]
    x0 = rng.standard_normal(n)
    target = rng.standard_normal(n)
    Z = lambda a, b: np.zeros((a, b))  # noqa: E731
    p = Problem([Z(n, n)] * (N + 1), [np.zeros(n)] * (N + 1), [np.eye(m)] * N, [np.zeros(m)] * N,
                [Z(n, m)] * N, A, B, c, [Z(0, n)] * N + [np.eye(n)], [Z(0, m)] * N,
                [np.zeros(0)] * N + [-target], x0)
    s = solve_sequential(p)
    assert s.status == "ok"
    blocks, free, Phi = [], np.zeros(n), np.eye(n)
    for j in range(N - 1, -1, -1):
        blocks.append(Phi @ B[j]); free += Phi @ c[j]; Phi = Phi @ A[j]
    blocks.reverse(); free += Phi @ x0
    u_ref = np.linalg.pinv(np.hstack(blocks)) @ (target - free)
    assert rel_err(s.u, np.split(u_ref, N)) < 1e-11
    assert np.allclose(s.x[N], target, atol=1e-11)


def test_no_free_input_is_cost_independent():
    """m-bar_i = 0 everywhere: the feasible trajectory is unique, so costs do not matter."""
    p = dict(FAMILY)["no-free-input"]
    s1 = solve_sequential(p)
    p2 = p.copy()
    rng = np.random.default_rng(3)
    p2.q = [rng.standard_normal(v.shape) * 10 for v in p.q]
    p2.Q = [Qi + 5 * np.eye(Qi.shape[0]) for Qi in p.Q]
    s2 = solve_sequential(p2)
    assert all(Z.shape[1] == 0 for Z in s1.Z)
    assert rel_err(s2.x, s1.x) < 1e-12 and rel_err(s2.u, s1.u) < 1e-12


def test_unconstrained_has_identity_bases():
    p = dict(FAMILY)["no-rows"]
    s = solve_sequential(p)
    for T, t in zip(s.T, s.t):
        assert T.shape[0] == T.shape[1] and np.allclose(np.abs(T @ T.T), np.eye(T.shape[0]), atol=1e-14)
        assert np.allclose(t, 0)
    for Z in s.Z:
        assert Z.shape[0] == Z.shape[1]


# ---------------------------------------------------------------------------
# Theorem 1: X_i is exactly the set of states with a feasible suffix
# ---------------------------------------------------------------------------

def _suffix_residual(p, i, xi):
    """Least-squares residual of all constraints of stages i..N with x_i fixed."""
    N = p.N
    nx, nu = p.nx, p.nu
    # unknowns: u_i, x_{i+1}, u_{i+1}, ..., x_N
    offs, o = {}, 0
    for j in range(i, N):
        offs[("u", j)] = o; o += nu[j]
        offs[("x", j + 1)] = o; o += nx[j + 1]
    rows, rhs = [], []

    def put(row_blocks, const):
        row = np.zeros((const.size, o))
        for key, mat in row_blocks:
            row[:, offs[key]:offs[key] + mat.shape[1]] += mat
        rows.append(row); rhs.append(-const)

    for j in range(i, N):
        xj_const = p.A[j] @ xi + p.c[j] if j == i else p.c[j]
        blk = [(("u", j), p.B[j]), (("x", j + 1), -np.eye(nx[j + 1]))]
        if j > i:
            blk.append((("x", j), p.A[j]))
        put(blk, xj_const)
        econst = p.E[j] @ xi + p.g[j] if j == i else p.g[j]
        blk = [(("u", j), p.F[j])] + ([(("x", j), p.E[j])] if j > i else [])
        put(blk, econst)
    put([(("x", N), p.E[N])], p.g[N]) if N > i else None
    Mx = np.vstack(rows); bv = np.concatenate(rhs)
    sol = np.linalg.lstsq(Mx, bv, rcond=None)[0]
    return float(np.max(np.abs(Mx @ sol - bv))) if bv.size else 0.0


@pytest.mark.parametrize("name", ["mixed-state-0", "redundant-1", "varying-dims", "pinned-state"])
def test_theorem1_suffix_domains_brute_force(name):
    p = dict(FAMILY)[name]
    s = solve_sequential(p)
    rng = np.random.default_rng(11)
    for i in range(p.N):
        T, t, H = s.T[i], s.t[i], s.H[i]
        for _ in range(3):
            xin = T @ rng.standard_normal(T.shape[1]) + t
            assert _suffix_residual(p, i, xin) < 1e-9
            if H.shape[0]:
                xout = xin + H.T @ rng.standard_normal(H.shape[0])
                assert _suffix_residual(p, i, xout) > 1e-3


# ---------------------------------------------------------------------------
# invariants: Lemma 2, Theorem 2, Propositions 1 and 2
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,p", FAMILY, ids=[f[0] for f in FAMILY])
def test_lemma2_theorem2_prop2(name, p):
    s = solve_sequential(p)
    for i in range(p.N):
        G, Phi, gam, Y, Z, y = s.Gam[i], s.Phi[i], s.gam[i], s.Y[i], s.Z[i], s.y[i]
        sc = max(1.0, np.abs(G).max() if G.size else 0)
        assert np.abs(G @ Z).max(initial=0) < 1e-11 * sc
        assert np.abs(G @ Y + Phi).max(initial=0) < 1e-9 * sc
        assert np.abs(G @ y + gam).max(initial=0) < 1e-9 * max(sc, np.abs(gam).max(initial=1))
        Rb = s.Rbar[i]
        if Rb.size:
            assert np.linalg.eigvalsh(Rb).min() > 0
        Hred = np.block([[s.Qbar[i], s.Mbar[i]], [s.Mbar[i].T, Rb]])
        if Hred.size:
            assert np.linalg.eigvalsh(0.5 * (Hred + Hred.T)).min() > -1e-9 * max(1, np.abs(Hred).max())
    assert abs(s.objective - (s.reduced_objective + sum(s.kappa))) < 1e-9 * max(1, abs(s.objective))


def _tree_suffix(rels, lo, hi):
    """Balanced parenthesisation of rels[lo] o ... o rels[hi-1]."""
    if hi - lo == 1:
        return rels[lo]
    mid = (lo + hi) // 2
    return compose(_tree_suffix(rels, lo, mid), _tree_suffix(rels, mid, hi))


@pytest.mark.parametrize("name", ["mixed-state-1", "redundant-0", "varying-dims-2", "random-g-mixed", "state-heavy"])
def test_prop1_associativity_tree_vs_sequential(name):
    p = dict(FAMILY)[name]
    s = solve_sequential(p, keep_relations=True)
    for i in range(p.N + 1):
        tree = _tree_suffix(s.relations, i, p.N + 1)
        assert tree.consistent
        assert same_set(tree, s.suffix[i], tol=1e-9)


# ---------------------------------------------------------------------------
# infeasibility outcomes of Algorithm 1
# ---------------------------------------------------------------------------

def test_infeasible_suffix_detected():
    p = tiny_problem(400, N=4, n=3, m=1, kinds=[[], [], [], ["state", "state", "state"]], terminal_rows=3)
    p.g[p.N] = p.g[p.N] + 1.0  # x_N pinned by two inconsistent row sets
    assert solve_sequential(p).status == "infeasible_suffix"


def test_infeasible_initial_detected():
    p = tiny_problem(401, N=4, n=3, m=2, kinds=[["state"], [], [], []], terminal_rows=0)
    p.g[0] = p.g[0] + 1.0
    s = solve_sequential(p)
    assert s.status == "infeasible_initial"


def test_not_convex_detected():
    p = tiny_problem(402, N=3, n=2, m=2, kinds=[[]] * 3, terminal_rows=0)
    p.R[1] = -p.R[1]
    assert solve_sequential(p).status == "not_convex"


# ---------------------------------------------------------------------------
# multipliers
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["mixed-state-2", "redundant-2", "pinned-state", "with-M", "varying-dims"])
def test_minnorm_multipliers_against_pinv(name):
    p = dict(FAMILY)[name]
    s = solve_with_multipliers(p)
    md = minnorm_multipliers_dense(p, s["x"], s["u"])
    assert rel_err(s["lam"], md["lam"]) < 1e-9
    if sum(p.nc):
        assert rel_err(s["mu"], md["mu"]) < 1e-9


def test_unique_multipliers_under_licq():
    """With LICQ the KKT matrix is nonsingular and every route gives the same nu."""
    p = tiny_problem(500, N=6, n=3, m=2, kinds=[["mixed"]] * 6, terminal_rows=1, g_mode="random")
    H, h, J, b, _ = dense_kkt(p)
    nn = J.shape[0]
    K = np.block([[H, J.T], [J, np.zeros((nn, nn))]])
    assert np.linalg.matrix_rank(K) == K.shape[0]
    sol = np.linalg.solve(K, -np.concatenate([h, b]))
    from oracle.dense import split_dual
    ref = split_dual(p, sol[H.shape[0]:], dense_kkt(p)[4])
    s = solve_with_multipliers(p)
    assert rel_err(s["lam"], ref["lam"]) < 1e-10 and rel_err(s["mu"], ref["mu"]) < 1e-10


def test_residual_definition():
    """Section IX residual: a planted error shows up in the right component with
    the right normalisation."""
    p = _integer_problem()
    s = solve_with_multipliers(p)
    base = kkt_residual(p, s["x"], s["u"], s["lam"], s["mu"])
    assert base["total"] < 1e-11
    x = [v.copy() for v in s["x"]]
    x[1][0] += 1e-3
    r = kkt_residual(p, x, s["u"], s["lam"], s["mu"])
    # dynamics row of stage 0 moves by exactly 1e-3
    assert abs(r["dynamics"] - 1e-3) < 1e-12
    # equality row E_1 = [0, 1]: unaffected by x_1[0]; E_1 x_1 residual unchanged
    mu = [v.copy() for v in s["mu"]]
    mu[2][0] += 2e-3
    r2 = kkt_residual(p, s["x"], s["u"], s["lam"], mu)
    # stationarity of x_2 moves by E_2^T * 2e-3 = [2e-3, 2e-3]; of u_2 by F_2^T*2e-3 = [0, 2e-3]
    assert abs(r2["stationarity"] - 2e-3) < 1e-12
    g = [v.copy() for v in p.g]
    p2 = p.copy(); p2.g = g; p2.g[3] = p.g[3] + 8.0
    r3 = kkt_residual(p2, s["x"], s["u"], s["lam"], s["mu"])
    # terminal row [1, -1] with offset 3 + 8 = 11: residual 8 / max(1, 1, 11)
    assert abs(r3["equality"] - 8.0 / 11.0) < 1e-12


def test_objective_matches_definition():
    p = _integer_problem()
    s = solve_sequential(p)
    w_obj = objective(p, s.x, s.u)
    H, h, J, b, _ = dense_kkt(p)
    w = np.concatenate([np.concatenate([s.x[i], s.u[i]]) for i in range(p.N)] + [s.x[p.N]])
    assert abs(w_obj - (0.5 * w @ H @ w + h @ w)) < 1e-10


@pytest.mark.parametrize("name", ["redundant-1", "pinned-state", "with-M", "state-heavy"])
def test_lsqr_multipliers_match_pinv(name):
    """The LSQR fallback returns the minimum-norm least-squares multipliers."""
    from oracle.dense import minnorm_multipliers_lsqr
    p = dict(FAMILY)[name]
    s = solve_with_multipliers(p)
    ref = minnorm_multipliers_dense(p, s["x"], s["u"])
    d, _ = minnorm_multipliers_lsqr(p, s["x"], s["u"])
    assert rel_err(d["lam"], ref["lam"]) < 1e-10
    if sum(p.nc):
        assert rel_err(d["mu"], ref["mu"]) < 1e-10


def test_degenerate_batched_instance_uses_lsqr_route():
    """A heavily state-constrained instance of the batched workload whose
    reversed-time reduction loses accuracy: the oracle's multipliers still
    match the null-space method."""
    from workloads import config_c3
    p = config_c3(B=9)[8]
    s = solve_with_multipliers(p)
    assert s["status"] == "ok"
    ns = solve_nullspace(p)
    assert rel_err(s["lam"], ns["lam"]) < 1e-10 and rel_err(s["mu"], ns["mu"]) < 1e-10
    assert rel_err(s["x"], ns["x"]) < 1e-10


def _f_full_row_rank(p) -> bool:
    return all(p.F[i].shape[0] == 0 or np.linalg.matrix_rank(p.F[i]) == p.F[i].shape[0] for i in range(p.N))


def test_whole_space_domains_condition():
    """Section VI: with no terminal rows and every F_i of full row rank, every
    suffix relation of the oracle's scan is empty (X_i is the whole space);
    a state-only row, a terminal row, or more mixed rows than inputs at a
    stage leaves rows in some suffix.  This is the condition the domain
    shortcut tests per instance on the device."""
    from workloads import config_c4
    vac = config_c4(B=2, N=12) + [tiny_problem(1204, N=7, n=3, m=2, kinds=[[]] * 7, terminal_rows=0),
                                  tiny_problem(1206, N=6, n=4, m=3, kinds=[["mixed", "mixed"]] * 6,
                                               terminal_rows=0)]
    for p in vac:
        assert p.E[p.N].shape[0] == 0 and _f_full_row_rank(p)
        r = solve_sequential(p, keep_relations=True)
        assert r.status == "ok"
        assert all(S.L.shape[0] == 0 for S in r.suffix)
        # the base relations themselves are not empty: the dynamics live there
        assert all(R.L.shape[0] > 0 for R in r.relations[:p.N])
    nonvac = [tiny_problem(1201, N=6, n=4, m=3, kinds=[["mixed", "state"]] * 6, terminal_rows=0),
              tiny_problem(1202, N=6, n=4, m=3, kinds=[["mixed"]] * 6, terminal_rows=1),
              tiny_problem(1203, N=5, n=3, m=2, kinds=[["mixed"] * 3] + [["mixed"]] * 4, terminal_rows=0)]
    for p in nonvac:
        r = solve_sequential(p, keep_relations=True)
        assert r.status == "ok"
        assert any(S.L.shape[0] > 0 for S in r.suffix)


def test_indefinite_costs_with_convex_reduction():
    """Costs indefinite only along directions the constraints fix: the
    oracle's reduction (Algorithm 1) equals the dense KKT solve, and the
    reduced input and state Hessians it forms are positive definite."""
    from tests._util import indefinite_cost_problems
    p1, p2, _ = indefinite_cost_problems()
    for p in (p1, p2):
        assert min(np.linalg.eigvalsh(R).min() for R in p.R) < 0 or min(np.linalg.eigvalsh(Q).min() for Q in p.Q) < 0
        r = solve_sequential(p)
        assert r.status == "ok"
        d = solve_dense(p)
        for key in ("x", "u"):
            assert rel_err(getattr(r, key), d[key]) <= 1e-10, key
        assert all(np.linalg.eigvalsh(Rb).min() > 0 for Rb in r.Rbar if Rb.size)


# ---------------------------------------------------------------------------
# relation equality has negatives; LICQ from the rank decisions
# ---------------------------------------------------------------------------

def test_same_set_accepts_bases_of_one_set_and_rejects_others():
    """same_set is the Definition 1 equivalence: another row basis of the same
    set (rows mixed by an invertible matrix, offsets mixed alike) is equal;
    a shifted offset, a tilted row space, a dropped row and a unary versus
    binary split are not."""
    rng = np.random.default_rng(31)
    L = rng.standard_normal((2, 3))
    R = rng.standard_normal((2, 2))
    ell = rng.standard_normal(2)
    base = Relation(L, R, ell)
    T = np.array([[2.0, 1.0], [-1.0, 3.0]])
    assert same_set(base, Relation(T @ L, T @ R, T @ ell))
    assert same_set(base, Relation(L[::-1].copy(), R[::-1].copy(), ell[::-1].copy()))
    assert not same_set(base, Relation(L, R, ell + np.array([1e-3, 0.0])))
    tilt = R.copy()
    tilt[0, 1] += 1e-3
    assert not same_set(base, Relation(L, tilt, ell))
    assert not same_set(base, Relation(L[:1], R[:1], ell[:1]))
    assert not same_set(Relation(np.hstack([L, R]), np.zeros((2, 0)), ell), Relation(L, R, ell + 1.0))


def test_rows_independent_matches_dense_rank():
    """LICQ read off the sequential method's rank decisions (sum of
    eliminated input dims against the row count) equals the rank of the
    dense constraint Jacobian, on the structural family and on instances
    built to fail it: a redundant row, a state row at stage 0, a terminal
    row repeating a stage row's restriction."""
    from oracle import rows_independent
    from oracle.dense import jacobian_full_row_rank
    cases = [p for _, p in FAMILY]
    cases.append(tiny_problem(1601, N=5, n=3, m=2, kinds=[["mixed"]] * 5, terminal_rows=0, redundant=(2,)))
    cases.append(tiny_problem(1602, N=4, n=3, m=2, kinds=[["state"], [], ["mixed"], []], terminal_rows=0))
    cases.append(tiny_problem(1603, N=4, n=3, m=2, kinds=[[], ["state"], [], []], terminal_rows=1))
    pinned = tiny_problem(1604, N=3, n=2, m=1, kinds=[[], [], ["state", "state"]], terminal_rows=0)
    cases.append(pinned)
    seen = set()
    for p in cases:
        res = solve_sequential(p)
        assert res.status == "ok"
        a, b = rows_independent(p, res), jacobian_full_row_rank(p)
        assert a == b, (a, b)
        seen.add(a)
    assert seen == {True, False}


# ---------------------------------------------------------------------------
# existence and uniqueness for arbitrary symmetric costs (Section II)
# ---------------------------------------------------------------------------

def _flat_input_problem(seed, slope):
    """An instance whose input 1 of stage 2 acts on nothing (zero column of
    B and F) and costs nothing quadratically (R_2 zero in that row and
    column): a flat feasible direction, with linear cost `slope` along it."""
    from tests._util import tiny_problem
    p = tiny_problem(seed, N=4, n=3, m=2, kinds=[["mixed"]] * 4, terminal_rows=0)
    p.B[2][:, 1] = 0.0
    p.F[2][:, 1] = 0.0
    p.R[2][1, :] = 0.0
    p.R[2][:, 1] = 0.0
    p.r[2][1] = slope
    return p


def test_classify_against_the_definition():
    """The classifier reproduces what the definition fixes on instances built
    to be in each class, and each answer is witnessed on the objective
    itself: the unique minimiser is the dense KKT solution; along the
    unbounded direction the objective falls without bound; along the flat
    direction it is constant and the two points satisfy the optimality
    conditions; a convex instance is unique."""
    from oracle.dense import solve_dense
    from oracle.existence import as_trajectory, classify, objective_dense
    from tests._util import indefinite_cost_problems, tiny_problem
    p1, p2, p3 = indefinite_cost_problems()
    convex = tiny_problem(4001, N=6, n=3, m=2, terminal_rows=1)
    for p in (convex, p1, p2):
        c = classify(p)
        assert c["kind"] == "unique", c["kind"]
        d = solve_dense(p)
        t = as_trajectory(p, c)
        assert rel_err(t["x"], d["x"]) <= 1e-9 and rel_err(t["u"], d["u"]) <= 1e-9
    for p, want in ((p3, None), (_flat_input_problem(4002, 0.7), "unbounded")):
        c = classify(p)
        if want:
            assert c["kind"] == want
        if c["kind"] == "unbounded":
            from oracle.dense import dense_kkt
            H, h, J, b, _ = dense_kkt(p)
            w0 = -np.linalg.pinv(J) @ b
            dvec = c["direction"]
            assert np.linalg.norm(J @ dvec) <= 1e-9  # feasible direction
            f = [objective_dense(p, w0 + t * dvec) for t in (0.0, 1e3, 1e6)]
            assert f[2] < f[1] < f[0]
    c = classify(_flat_input_problem(4002, 0.0))
    assert c["kind"] == "not_unique"
    from oracle.dense import dense_kkt
    H, h, J, b, _ = dense_kkt(_flat_input_problem(4002, 0.0))
    w, dvec = c["w"], c["direction"]
    assert np.linalg.norm(J @ dvec) <= 1e-9 and np.linalg.norm(J @ w + b) <= 1e-9
    f0 = objective_dense(_flat_input_problem(4002, 0.0), w)
    f1 = objective_dense(_flat_input_problem(4002, 0.0), w + 5.0 * dvec)
    assert abs(f1 - f0) <= 1e-9 * max(1.0, abs(f0))
    # both points are stationary on the feasible set
    Wn = __import__("scipy.linalg", fromlist=["null_space"]).null_space(J)
    for pt in (w, w + 5.0 * dvec):
        assert np.linalg.norm(Wn.T @ (H @ pt + h)) <= 1e-9
