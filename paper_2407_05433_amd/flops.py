"""Algorithmic FP64 flop model of one solve, per kernel class.

Nominal dense counts (a multiply-add = 2 flops) at the actual sizes of every
unit of work: per stage for the stage-parallel kernels, per task for the scan
combines.  Reduced dimensions and relation row counts are read back from the
workspace after a solve.  Householder QR of a p x c matrix with r reflections
counts sum_{j<r} 4 (p - j)(c - j); row-pivoted Gram-Schmidt of p rows over kc
columns choosing r rows counts sum_{j<r} (4 j kc + 4 (p - j - 1)(kc + 1)).
A solve with multipliers runs the problem's engine and, by the multiplier
route of the plan, either the reversed-time stationarity problem's engine or
the theta LQR (local minimum-norm systems, value-function scan, gains and
forward scan over the normal coordinates of the domains) once in full;
refinement steps and the adjoint replay the logged factors on new vectors
(kernel class "replay", whose matrix-vector work is not counted here).
"""

from __future__ import annotations

from collections import defaultdict
from typing import Dict

import numpy as np


def _qr(p, c, r):
    """sum_{j<r} 4 (p - j)(c - j)"""
    r = float(r)
    return 4.0 * (r * p * c - (p + c) * r * (r - 1) / 2.0 + (r - 1) * r * (2 * r - 1) / 6.0)


def _gs(p, kc, r):
    """sum_{j<r} 4 j kc + 4 (p - j - 1)(kc + 1)  (r <= p)"""
    r = float(r)
    return 2.0 * kc * r * (r - 1) + 4.0 * (kc + 1) * (r * (p - 1) - r * (r - 1) / 2.0)


def engine_flops(plan, ws, dual: bool, weight=None) -> Dict[str, float]:
    """Flops per kernel class of one engine pass; instance b counted weight[b] times."""
    dims = plan.stage_dims(dual)
    nbar, mbar = plan.reduced_dims(ws, dual)
    rows = plan.scan_rows(ws, dual)
    inst, first, last = plan.slot_info(dual)
    horizons = [h + 1 for h in plan.horizons] if dual else list(plan.horizons)
    sbase = np.concatenate([[0], np.cumsum([h + 1 for h in horizons])[:-1]]).astype(np.int64)
    W = np.ones(len(horizons)) if weight is None else np.asarray(weight, dtype=np.float64)
    F = defaultdict(float)
    leaf_base = np.full(len(horizons), -1, dtype=np.int64)
    for q in range(len(inst) - 1, -1, -1):
        leaf_base[inst[q]] = q  # leaves are the first slots of each instance
    stage_inst = np.repeat(np.arange(len(horizons)), [h + 1 for h in horizons])

    # per-stage kernels
    for s, (n, np_, m, k) in enumerate(dims):
        nb = int(nbar[s])
        b = int(stage_inst[s])
        i = s - int(sbase[b])
        # domain parameterisation: QR of H^T (n x r), T formation, t
        r = n - nb
        w = W[b]
        F["domain"] += w * (_qr(n, r, r) + 4.0 * nb * (r * n - r * (r - 1) / 2.0) + 2.0 * n * r)
        if i == horizons[b]:
            F["eliminate"] += w * (2.0 * n * n * nb + 2.0 * nb * n * nb + 2.0 * n * n + 2.0 * n * nb)
            F["base_relation"] += w * _gs(k, n, rows[leaf_base[b] + i])
            continue
        nb1, mb = int(nbar[s + 1]), int(mbar[s])
        r1 = np_ - nb1
        q = k + r1
        rho = m - mb
        f = 0.0
        f += 2.0 * r1 * np_ * (m + n + 1)                    # H' [B A c]
        f += 2.0 * q * n * (nb + 1)                          # Phi, gamma
        f += _qr(m, q, rho) + sum(4.0 * (m - j) * m for j in range(rho))   # QR of Gamma^T, form Q
        f += rho * rho * (nb + 1) + 2.0 * m * (nb + 1) * rho  # R11^{-T}, Y, y
        f += 2.0 * np_ * nb * (n + m) + 2.0 * nb1 * np_ * nb  # A T + B Y, T'^T (.)
        f += 2.0 * np_ * m * mb + 2.0 * nb1 * np_ * mb        # B Z, T'^T B Z
        f += 2.0 * np_ * (n + m) + 2.0 * nb1 * np_            # c-bar
        f += 2.0 * n * n * nb + 2.0 * nb * n * nb             # Q T, T^T Q T
        f += 2.0 * m * m * (nb + mb) + 2.0 * nb * m * nb      # R Y, R Z, Mz Y
        f += 2.0 * nb * m * nb + 2.0 * nb * m * mb * 2 + 2.0 * mb * m * mb  # Y^T R Y, Mz Z, Y^T R Z, Z^T R Z
        f += 2.0 * n * n + 2.0 * m * m + 2.0 * nb * n + 2.0 * nb * m * 2 + 2.0 * mb * m  # vectors
        f += mb ** 3 / 3.0 + mb * mb * (nb1 + nb + 1)         # Cholesky of R-bar, L^{-1} [B^T M^T r]
        f += 2.0 * nb1 * nb * mb + 2.0 * nb1 * nb1 * mb + 2.0 * nb * nb * mb + 2.0 * (nb1 + nb) * mb
        F["eliminate"] += w * f
        # base relation: QR of [B; F] over the input columns, row basis of the rest
        p = np_ + k
        c = m + n + np_ + 1
        rho_u = min(m, p)
        F["base_relation"] += w * (_qr(p, c, rho_u) + _gs(p - rho_u, n + np_, rows[leaf_base[b] + i]))
        # gains
        g = 2.0 * nb1 * nb1 * (mb + nb) + 2.0 * mb * mb * nb1 + 2.0 * mb * nb * nb1 + mb ** 3 / 3.0
        g += 2.0 * mb * mb * (nb + 1) + 2.0 * nb1 * mb * nb + 2.0 * nb1 * (nb1 + mb)
        F["gains"] += w * g
        F["recover"] += w * 2.0 * (n * nb + m * (nb + mb) + mb * nb)

    # scan combines
    levels = plan.schedule(dual)
    def sdim(b, leaf):  # noqa: E301
        return dims[sbase[b] + leaf][0]

    def rdim(b, leaf):
        return int(nbar[sbase[b] + leaf])

    for lv in levels:
        for a, bb, o in lv:
            b = int(inst[a])
            w = W[b]
            L = horizons[b] + 1
            s0, mid, e0 = int(first[a]), int(last[a]), int(last[bb])
            # relation composition
            na, nb_, nc = sdim(b, s0), sdim(b, mid), (sdim(b, e0) if e0 < L else 0)
            p = int(rows[a] + rows[bb])
            rr = int(rows[o])
            rho = min(nb_, max(p - rr, 0))
            F["rel_compose"] += w * (_qr(p, na + nb_ + nc + 1, rho) + _gs(p - rho, na + nc, rr))
            # value-function combine
            ds, dm, de = rdim(b, s0), rdim(b, mid), (rdim(b, e0) if e0 < L else 0)
            f = 2.0 * dm ** 3 + 2.0 / 3.0 * dm ** 3 + 2.0 * dm * dm * (dm + 1) + 2.0 * dm * dm
            f += 2.0 * ds * dm * dm + 2.0 * ds * ds * dm + 2.0 * ds * dm
            if e0 < L:
                f += 2.0 * dm * dm * (ds + 1 + dm) + 2.0 * dm * dm + 2.0 * de * ds * dm + 2.0 * de * dm
                f += 2.0 * de * dm * dm + 2.0 * de * de * dm
            F["ric_combine"] += w * f
            # forward map composition: slot interval reflected (output z_{N-s}, input z_{N-e})
            N = horizons[b]
            do, dmid = rdim(b, N - s0), rdim(b, N - mid)
            din = rdim(b, N - e0) if e0 < L else 0
            F["fwd_combine"] += w * 2.0 * do * dmid * (din + 1)
    return dict(F)


def theta_flops(plan, ws) -> Dict[str, float]:
    """Flops of the theta LQR route: per stage the minimum-norm local system
    (QR of the q x R transposed system with rho reflections, Q formed, the
    triangular solve and Q1 X for r + 1 right-hand sides, Y'Y), the gains; per
    task the value-function and forward combines at dims r."""
    dims = plan.stage_dims(False)
    nb_p, _ = plan.reduced_dims(ws)
    r, f = plan.reduced_dims(ws, which=2)
    F = defaultdict(float)
    horizons = list(plan.horizons)
    stage_inst = np.repeat(np.arange(len(horizons)), [h + 1 for h in horizons])
    sbase = np.concatenate([[0], np.cumsum([h + 1 for h in horizons])[:-1]]).astype(np.int64)
    for s, (n, np_, m, k) in enumerate(dims):
        b = int(stage_inst[s])
        term = (s - int(sbase[b])) == horizons[b]
        ri = int(r[s])
        r1 = 0 if term else int(r[s + 1])
        q = k + r1
        R = n + (0 if term else m)
        rho = q - (0 if term else int(f[s]))
        nc = ri + 1
        t = 2.0 * r1 * np_ * (n + m) + _qr(q, R, rho) + sum(4.0 * (q - j) * q for j in range(rho))
        t += rho * rho * nc + 2.0 * q * rho * nc + 2.0 * ri * ri * q + 2.0 * ri * q
        t += 2.0 * n * (n + m) + 2.0 * int(nb_p[s]) * (n + 1)  # gradients, costate
        F["multipliers_theta"] += t
        if not term:
            mb, nb, nb1 = int(f[s]), ri, r1
            g = 2.0 * nb1 * nb1 * (mb + nb) + 2.0 * mb * mb * nb1 + 2.0 * mb * nb * nb1 + mb ** 3 / 3.0
            g += 2.0 * mb * mb * (nb + 1) + 2.0 * nb1 * mb * nb + 2.0 * nb1 * (nb1 + mb)
            F["gains"] += g
    inst, first, last = plan.slot_info(False)
    for lv in plan.schedule(False):
        for a, bb, o in lv:
            b = int(inst[a])
            L = horizons[b] + 1
            s0, mid, e0 = int(first[a]), int(last[a]), int(last[bb])
            ds, dm = int(r[sbase[b] + s0]), int(r[sbase[b] + mid])
            de = int(r[sbase[b] + e0]) if e0 < L else 0
            fl = 2.0 * dm ** 3 + 2.0 / 3.0 * dm ** 3 + 2.0 * dm * dm * (dm + 1) + 2.0 * dm * dm
            fl += 2.0 * ds * dm * dm + 2.0 * ds * ds * dm + 2.0 * ds * dm
            if e0 < L:
                fl += 2.0 * dm * dm * (ds + 1 + dm) + 2.0 * dm * dm + 2.0 * de * ds * dm + 2.0 * de * dm
                fl += 2.0 * de * dm * dm + 2.0 * de * de * dm
            F["ric_combine"] += fl
            N = horizons[b]
            do, dmid = int(r[sbase[b] + N - s0]), int(r[sbase[b] + N - mid])
            din = int(r[sbase[b] + N - e0]) if e0 < L else 0
            F["fwd_combine"] += 2.0 * do * dmid * (din + 1)
    return dict(F)


def solve_flops(plan, problems, ws, multipliers: bool = True, steps=None) -> Dict[str, float]:
    """Flops per kernel class of the full passes of one solve: the problem and,
    with multipliers, the route the plan takes (the reversed-time problem or
    the theta LQR), each once."""
    from .solver import get_tuning
    out = defaultdict(float)
    for k, v in engine_flops(plan, ws, False).items():
        out[k] += v
    if multipliers:
        theta = int(plan.options.multipliers) == 1 and get_tuning(plan).get("multiplier_route", 0) == 1
        extra = theta_flops(plan, ws) if theta else engine_flops(plan, ws, True)
        for k, v in extra.items():
            out[k] += v
    return dict(out)
