"""CPU model of the BF16 candidate arithmetic in the super-chunk frames and
of the error bound the kernel applies to it.

The candidate pass quantises a row point x and a column point y in a frame
centred at c and scaled by a power of two sigma:

  u_x = sigma (x - c) in FP32, row q = qh + ql with qh = bf16(u_x) and
  ql = bf16(u_x - qh) (two chained MFMAs); column p = bf16(u_y);
  t = ||q||^2 + ||p||^2 - 2 p.q, with the squared norms carried as three
  BF16 parts in the operands' norm slots and every product accumulated in
  FP32.

and keeps every column with t - E(t) <= U, where

  E(t) = k [eps + eta' (2 sqrt(t + eps) + eta')],
  eps = gamma (2 Q_i Q_j + P_i + P_j) + rho_i + rho_j,  eta' = eta_i + eta_j,
  gamma = 67 2^-23 (64 products in two chained MFMAs),
  Q_i = ||qh|| + ||ql||, eta_i = (2^-16 + 2^-22) ||u_x|| + beta sqrt(d),
  Q_j = ||p||,          eta_j = (2^-8 + 2^-22) ||u_y|| + beta sqrt(d).

This test emulates the arithmetic in numpy (round-to-nearest-even BF16,
FP32 sums in several orders) and checks |t - sigma^2 s| <= E(t) for every
pair, with s the exact squared distance of eq. (1); it also checks the
bound is not vacuous (the largest error reaches a fair fraction of it).
It models the kernel's formulas; the GPU tests check the kernel itself.
"""
import math

import numpy as np
import pytest

KFAC = 1.0 + 2.0 ** -20
BETA = 2.0 ** -125
UP = 1.0 + 2.0 ** -18


def bf16(a):
    """Round float32 values to BF16 (nearest, ties to even), as float32."""
    a = np.asarray(a, np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return (r.astype(np.uint32) << 16).view(np.float32)


def f32_fma_sum(terms, order):
    """FP32 accumulation of exact float64 terms in the given order (one
    rounding per addition, as an accumulator that adds exact products)."""
    acc = np.float32(0.0)
    for k in order:
        acc = np.float32(np.float64(acc) + terms[k])
    return acc


def norm_parts(n32):
    """Three BF16 parts of a float32 value; residual after them."""
    r = np.float32(n32)
    parts = []
    for _ in range(3):
        p = bf16(r)
        parts.append(float(p))
        r = np.float32(r - p)
    return parts, float(r)


def row_operand(u, d):
    qh = bf16(u)
    ql = bf16(np.float32(u - qh))
    q = np.float32(qh + ql)
    nrm = f32_fma_sum(np.asarray(q, np.float64) ** 2, range(d))
    parts, res = norm_parts(nrm)
    Q = (math.sqrt(float(np.sum(np.asarray(qh, np.float64) ** 2))) +
         math.sqrt(float(np.sum(np.asarray(ql, np.float64) ** 2)))) * UP
    P = sum(abs(x) for x in parts) * UP
    rho = (abs(res) + float(nrm) * 30.0 * 2.0 ** -24) * UP
    eta = ((2.0 ** -16 + 2.0 ** -22) * math.sqrt(float(np.sum(np.asarray(u, np.float64) ** 2))) * UP
           + BETA * math.sqrt(d)) * UP
    return qh, ql, parts, (Q, P, rho, eta)


def col_operand(u, d):
    p = bf16(u)
    nrm = f32_fma_sum(np.asarray(p, np.float64) ** 2, range(d))
    parts, res = norm_parts(nrm)
    Q = math.sqrt(float(np.sum(np.asarray(p, np.float64) ** 2))) * UP
    P = sum(abs(x) for x in parts) * UP
    rho = (abs(res) + float(nrm) * 27.0 * 2.0 ** -24) * UP
    eta = ((2.0 ** -8 + 2.0 ** -22) * math.sqrt(float(np.sum(np.asarray(u, np.float64) ** 2))) * UP
           + BETA * math.sqrt(d)) * UP
    return p, parts, (Q, P, rho, eta)


def candidate(qh, ql, rparts, p, cparts, order):
    """t from two chained 32-product accumulations (high half with the norm
    slots, then the low half), each summed in the given order."""
    d = len(p)
    hi = [float(-2.0 * np.float64(p[k]) * np.float64(qh[k])) for k in range(d)]
    hi += rparts + cparts                               # parts x 1 and 1 x parts
    lo = [float(-2.0 * np.float64(p[k]) * np.float64(ql[k])) for k in range(d)]
    t1 = f32_fma_sum(np.asarray(hi), order(len(hi)))
    acc = np.float32(t1)
    for k in order(len(lo)):
        acc = np.float32(np.float64(acc) + lo[k])
    return float(acc)


def bound(t, ri, cj):
    Qi, Pi, rhoi, etai = ri
    Qj, Pj, rhoj, etaj = cj
    gamma = 67.0 * 2.0 ** -23
    eps = gamma * (2.0 * Qi * Qj + Pi + Pj) + rhoi + rhoj
    eta = etai + etaj
    return KFAC * (eps + eta * (2.0 * math.sqrt(max(t, 0.0) + eps) + eta))


ORDERS = {
    "forward": lambda n: range(n),
    "backward": lambda n: range(n - 1, -1, -1),
    "shuffled": lambda n: np.random.default_rng(n).permutation(n),
}


@pytest.mark.parametrize("d", [4, 25, 26])
@pytest.mark.parametrize("order", list(ORDERS))
def test_split_bf16_bound_holds(d, order):
    rng = np.random.default_rng(1000 * d + len(order))
    worst = 0.0
    checked = 0
    for trial in range(6):
        # a column super-chunk (tight cluster) and rows near and far from it
        centre = rng.uniform(0.0, 1.0, d).astype(np.float32)
        spread = float(rng.choice([0.002, 0.02, 0.2]))
        cols = (centre + rng.normal(0.0, spread, (24, d))).astype(np.float32)
        rows = np.concatenate([
            (centre + rng.normal(0.0, spread, (12, d))),
            (centre + rng.normal(0.0, 3.0 * spread, (12, d))),
            rng.uniform(0.0, 1.0, (12, d)),
        ]).astype(np.float32)
        frame = cols.mean(axis=0).astype(np.float32)   # the super-chunk's ball centre
        span = float(np.max(np.abs(np.concatenate([rows, cols]) - 0.5)))
        sigma = np.float32(2.0 ** -math.frexp(span)[1])
        ur = ((rows - frame).astype(np.float32) * sigma).astype(np.float32)
        uc = ((cols - frame).astype(np.float32) * sigma).astype(np.float32)
        R = [row_operand(ur[i], d) for i in range(len(rows))]
        C = [col_operand(uc[j], d) for j in range(len(cols))]
        for i in range(len(rows)):
            qh, ql, rparts, ri = R[i]
            for j in range(len(cols)):
                p, cparts, cj = C[j]
                t = candidate(qh, ql, rparts, p, cparts, ORDERS[order])
                diff = rows[i].astype(np.float64) - cols[j].astype(np.float64)
                s = float(np.dot(diff, diff)) * float(sigma) ** 2
                E = bound(t, ri, cj)
                err = abs(t - s)
                assert err <= E, (trial, i, j, t, s, err, E)
                worst = max(worst, err / E)
                checked += 1
    assert checked == 6 * 36 * 24
    assert worst > 1e-3, worst          # the bound is not vacuous


def test_single_bf16_would_not_do():
    """The split matters: with a single BF16 row operand the error of a far
    row exceeds the split bound (so the low half is really needed)."""
    rng = np.random.default_rng(5)
    d = 25
    centre = rng.uniform(0.0, 1.0, d).astype(np.float32)
    col = (centre + rng.normal(0.0, 0.002, d)).astype(np.float32)
    row = rng.uniform(0.0, 1.0, d).astype(np.float32)
    sigma = np.float32(2.0)
    frame = col
    ur = ((row - frame) * sigma).astype(np.float32)
    uc = ((col - frame) * sigma).astype(np.float32)
    qh, ql, rparts, ri = row_operand(ur, d)
    p, cparts, cj = col_operand(uc, d)
    zero = np.zeros_like(ql)
    diff = row.astype(np.float64) - col.astype(np.float64)
    s = float(np.dot(diff, diff)) * 4.0
    t_split = candidate(qh, ql, rparts, p, cparts, ORDERS["forward"])
    # single BF16 row: the same high half, no low half, norm of qh alone
    nh = f32_fma_sum(np.asarray(qh, np.float64) ** 2, range(d))
    hparts, _ = norm_parts(nh)
    t_single = candidate(qh, zero, hparts, p, cparts, ORDERS["forward"])
    E = bound(t_split, ri, cj)
    assert abs(t_split - s) <= E
    assert abs(t_single - s) > E


def test_split_representation_error():
    """|qh + ql - u| <= 2^-16 |u| per value (plus BF16's subnormal floor),
    the per-feature fact behind the rows' eta; and qh + ql and u - qh are
    exact in FP32."""
    rng = np.random.default_rng(9)
    u = np.concatenate([
        rng.uniform(-2.0, 2.0, 200000),
        rng.standard_normal(100000) * 1e-3,
        np.ldexp(rng.uniform(1.0, 2.0, 100000), rng.integers(-140, 2, 100000)) * rng.choice([-1, 1], 100000),
    ]).astype(np.float32)
    qh = bf16(u)
    r = np.float32(u - qh)
    assert np.array_equal(r.astype(np.float64), u.astype(np.float64) - qh.astype(np.float64))
    ql = bf16(r)
    q = np.float32(qh + ql)
    assert np.array_equal(q.astype(np.float64), qh.astype(np.float64) + ql.astype(np.float64))
    err = np.abs(q.astype(np.float64) - u.astype(np.float64))
    assert np.all(err <= 2.0 ** -16 * np.abs(u.astype(np.float64)) + 2.0 ** -134)
    # and the single BF16 rounding is within 2^-8 (the columns' alpha)
    e1 = np.abs(qh.astype(np.float64) - u.astype(np.float64))
    assert np.all(e1 <= 2.0 ** -8 * np.abs(u.astype(np.float64)) + 2.0 ** -134)


# ---- rows in their tile's frame, columns in their super-chunk's frame ------
#
# The rows are split once in the frame of their tile's centre c_T
# (a = ah + al of sigma (x - c_T)); a column super-chunk's frame (centre
# c_S) enters through the offset delta = sigma (c_T - c_S) in FP32:
#   t = ||a + delta||^2 + ||p||^2 - 2 a.p - 2 delta.p,
# the row's norm slots carry R = ||a||^2 + 2 a.delta + ||delta||^2 and the
# column's C = ||p||^2 - 2 delta.p, each evaluated in FP32 and split into
# three BF16 parts.  Bound inputs: Q_i = ||ah|| + ||al||, Q_j = ||p||;
# P and rho of the rewritten slots from the FP32 error of R and C:
#   rho_R <= 30 u (||a||^2 + 2 Q_i ||delta|| + ||delta||^2) + |residual|,
#   rho_C <= rho_p + 30 u (||p||^2 + 2 Q_j ||delta||) + |residual|,
# and the represented row point moves by at most 2^-22 ||delta|| (the FP32
# rounding of delta), added to eta_i.

U32 = 2.0 ** -24


def f32_dot_fma(x, y):
    """sum_k x_k y_k with one FP32 rounding per step (fused multiply-add)."""
    acc = np.float32(0.0)
    for a, b in zip(np.asarray(x, np.float64), np.asarray(y, np.float64)):
        acc = np.float32(np.float64(acc) + a * b)
    return acc


def tile_rows(u, d):
    """Split rows of the tile frame: halves, ||a||^2 (FP32), Q, eta."""
    ah = bf16(u)
    al = bf16(np.float32(u - ah))
    a = np.float32(ah + al)
    nA = f32_dot_fma(a, a)
    Q = (math.sqrt(float(np.sum(np.asarray(ah, np.float64) ** 2))) +
         math.sqrt(float(np.sum(np.asarray(al, np.float64) ** 2)))) * UP
    eta = ((2.0 ** -16 + 2.0 ** -22) * math.sqrt(float(np.sum(np.asarray(u, np.float64) ** 2))) * UP
           + BETA * math.sqrt(d)) * UP
    return ah, al, a, nA, Q, eta


def frame_row(a, nA, Q, eta, delta, dn):
    """The row's norm slots in a column frame: parts of R, P, rho, eta."""
    dot = f32_dot_fma(a, delta)
    dd = f32_dot_fma(delta, delta)
    R = np.float32(np.float32(nA + np.float32(2.0 * dot)) + dd)
    parts, res = norm_parts(R)
    P = sum(abs(x) for x in parts) * UP
    rho = (abs(res) + 30.0 * U32 * (float(nA) + 2.0 * Q * dn + float(dd))) * UP
    return parts, (Q, P, rho, (eta + 2.0 ** -22 * dn) * UP)


def frame_col(p, nrm_parts, rho_p, Qp, delta, dn):
    """The column's norm slots in the row tile's frame: parts of C."""
    normP = np.float32(np.float32(nrm_parts[0] + nrm_parts[1]) + nrm_parts[2])
    dotP = f32_dot_fma(np.float32(-2.0) * p, delta)
    C = np.float32(normP + dotP)
    parts, res = norm_parts(C)
    P = sum(abs(x) for x in parts) * UP
    rho = (rho_p + abs(res) + 30.0 * U32 * (float(normP) + 2.0 * Qp * dn)) * UP
    return parts, P, rho


@pytest.mark.parametrize("d", [4, 25, 26])
@pytest.mark.parametrize("order", list(ORDERS))
def test_offset_frames_bound_holds(d, order):
    rng = np.random.default_rng(7000 + 10 * d + len(order))
    worst = 0.0
    for trial in range(5):
        spread = float(rng.choice([0.002, 0.02, 0.2]))
        c_row = rng.uniform(0.0, 1.0, d).astype(np.float32)
        c_col = (c_row + rng.normal(0.0, float(rng.choice([0.0, 0.05, 0.5])), d)).astype(np.float32)
        rows = (c_row + rng.normal(0.0, spread, (16, d))).astype(np.float32)
        cols = (c_col + rng.normal(0.0, spread, (24, d))).astype(np.float32)
        c_T = rows.mean(axis=0).astype(np.float32)
        c_S = cols.mean(axis=0).astype(np.float32)
        span = float(np.max(np.abs(np.concatenate([rows, cols]) - 0.5)))
        sigma = np.float32(2.0 ** -math.frexp(span)[1])
        ur = ((rows - c_T).astype(np.float32) * sigma).astype(np.float32)
        uc = ((cols - c_S).astype(np.float32) * sigma).astype(np.float32)
        delta = ((c_T - c_S).astype(np.float32) * sigma).astype(np.float32)
        dn = math.sqrt(float(np.sum(np.asarray(delta, np.float64) ** 2))) * UP
        C = [col_operand(uc[j], d) for j in range(len(cols))]
        # the chunk's maxima as the kernel keeps them, and the bounds it
        # derives from them for the rewritten column slots
        Qs = max(c[2][0] for c in C)
        rhos = max(c[2][2] for c in C)
        etas = max(c[2][3] for c in C)
        mag = Qs * Qs + rhos + 2.0 * Qs * dn
        Ps = mag * (1.0 + 2.0 ** -6)
        rhoS = (rhos + 32.0 * U32 * mag) * UP
        for i in range(len(rows)):
            ah, al, a, nA, Qi, etai = tile_rows(ur[i], d)
            rparts, ri = frame_row(a, nA, Qi, etai, delta, dn)
            for j in range(len(cols)):
                p, cparts0, (Qj, Pj0, rhoj0, etaj) = C[j]
                cparts, Pj, rhoj = frame_col(p, cparts0, rhoj0, Qj, delta, dn)
                assert Pj <= Ps and rhoj <= rhoS, (Pj, Ps, rhoj, rhoS)
                t = candidate(ah, al, rparts, p, cparts, ORDERS[order])
                diff = rows[i].astype(np.float64) - cols[j].astype(np.float64)
                s = float(np.dot(diff, diff)) * float(sigma) ** 2
                E = bound(t, ri, (Qs, Ps, rhoS, etas))
                err = abs(t - s)
                assert err <= E, (trial, i, j, t, s, err, E)
                worst = max(worst, err / E)
    assert worst > 1e-3, worst
