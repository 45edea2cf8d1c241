"""Slot-level simulator of a plan on cleartext vectors (test infrastructure only).

A "ciphertext" here is its slot vector (length M, float64).  Every homomorphic
operation of the plan is replaced by what it does to the slots (paper Sec. 2.1):
PMult -> slotwise product, Rot(v, k) -> v shifted left by k, scalar MAC ->
weighted sum.  The simulator checks the routing of a plan (the FP64 output
must equal the plaintext GCN to rounding) and counts its operations.
"""
from __future__ import annotations

from typing import List

import numpy as np

from . import radix2
from .planner import LayerPlan, Plan, reduce_shift


def rot(v: np.ndarray, k: int) -> np.ndarray:
    """Rot(v, k)_j = v_{j+k} (left rotation)."""
    return np.roll(v, -k)


def client_layout(plan: Plan, x: np.ndarray, lp: LayerPlan) -> List[List[np.ndarray]]:
    """Input slot vectors the client packs for the first layer.
    inter : copies[k][f][pi(v)] = x[src_k(v), f] (zero when v has no k-th term)
    spintra: copies[0][f][pi(v)] = x[v, f] (one column per ciphertext)."""
    M = plan.M
    n = plan.n_v
    if lp.kind == "inter" and lp.pack == "rep":
        return rep_client_layout(plan, x, lp)
    if lp.kind == "inter":
        out = []
        for k in range(lp.K):
            src = lp.copy_src[k]
            have = src >= 0
            vecs = []
            for f in range(lp.f_in):
                v = np.zeros(M)
                v[plan.pi[have]] = x[src[have], f]
                vecs.append(v)
            out.append(vecs)
        return out
    vecs = []
    for f in range(lp.f_in):
        v = np.zeros(M)
        v[plan.pi[np.arange(n)]] = x[:, f]
        vecs.append(v)
    return [vecs]


def inter_plaintexts(plan: Plan, lp: LayerPlan) -> List[np.ndarray]:
    """P_k[pi(v)] = A_hat[v, src_k(v)]."""
    out = []
    for k in range(lp.K):
        src = lp.copy_src[k]
        have = src >= 0
        p = np.zeros(plan.M)
        p[plan.pi[have]] = lp.copy_val[k][have]
        out.append(p)
    return out


def rep_slot(lp: LayerPlan, b: int, l: int) -> int:
    """First slot of the block of input column b (within the ciphertext) and output column l
    in the case-1 layout: (b pow2(F') + l) Bc."""
    Fp = 1
    while Fp < lp.f_out:
        Fp *= 2
    return (b * Fp + l) * lp.B


def rep_client_layout(plan: Plan, x: np.ndarray, lp: LayerPlan) -> List[List[np.ndarray]]:
    """Case-1 layout (Sec. 3.2, App. B): ciphertext j of copy k holds input columns
    j t + b (b < t) of the copy, column b repeated for every output column l < F':
    slot rep_slot(b, l) + pi(v) = x[src_k(v), j t + b]."""
    J = -(-lp.f_in // lp.t)
    out = []
    for k in range(lp.K):
        src = lp.copy_src[k]
        have = src >= 0
        vecs = []
        for j in range(J):
            v = np.zeros(plan.M)
            for b in range(lp.t):
                f = j * lp.t + b
                if f >= lp.f_in:
                    break
                for l in range(lp.f_out):
                    v[rep_slot(lp, b, l) + plan.pi[have]] = x[src[have], f]
            vecs.append(v)
        out.append(vecs)
    return out


def rep_plaintexts(plan: Plan, lp: LayerPlan, w: np.ndarray) -> List[np.ndarray]:
    """Operand k * J + j of the case-1 layout: slot rep_slot(b, l) + pi(v) =
    A_hat[v, src_k(v)] * W[j t + b, l] (the copy's adjacency value times the weight)."""
    J = -(-lp.f_in // lp.t)
    out = []
    for k in range(lp.K):
        src = lp.copy_src[k]
        have = src >= 0
        for j in range(J):
            p = np.zeros(plan.M)
            for b in range(lp.t):
                f = j * lp.t + b
                if f >= lp.f_in:
                    break
                for l in range(lp.f_out):
                    p[rep_slot(lp, b, l) + plan.pi[have]] = lp.copy_val[k][have] * w[f, l]
            out.append(p)
    return out


def diag_masks(plan: Plan, lp: LayerPlan, w: np.ndarray) -> dict:
    """Block-rotation combination of an input packed in blocks of B: cm_s[c B + pi(v)] =
    W[c + s, c] for output column c < F' and input column c + s < F, so that
    sum_s Rot_{sB}(H) (.) cm_s holds sum_l W[l, c] H_l in block c."""
    out = {}
    for s_ in lp.comb_shifts:
        v = np.zeros(plan.M)
        for c in range(lp.f_out):
            l = c + s_
            if 0 <= l < lp.f_in:
                v[c * lp.B + plan.pi] = w[l, c]
        out[s_] = v
    return out


def masks(plan: Plan, lp: LayerPlan, n_cols: int) -> dict:
    """mask_delta[c*B + pi(v)] = A_hat[v, u] for the demand (v, u) whose shift is
    delta, in every block c < n_cols of the packed ciphertext."""
    M, B = plan.M, lp.B
    wrap = B == M
    out = {d: np.zeros(M) for d in lp.shifts}
    for v, row in enumerate(plan.rows):
        for u, a in row:
            d = reduce_shift(int(plan.pi[u] - plan.pi[v]), M, wrap)
            for c in range(n_cols):
                out[d][c * B + plan.pi[v]] = a
    return out


def aggregate_packed(plan: Plan, lp: LayerPlan, y: np.ndarray, n_cols: int, counts: dict) -> np.ndarray:
    if lp.family == 3:
        return radix2.run_slots(lp.program, y, lp.B, n_cols, counts)
    mk = masks(plan, lp, n_cols)
    out = np.zeros(plan.M)
    if lp.family in (1, 4):
        for d in lp.shifts:
            out += rot(y, d) * mk[d]
            counts["pmult"] += 1
            counts["rot"] += d != 0
        return out
    G = lp.G
    giants = {}
    for d in lp.shifts:
        giants.setdefault(d // G, []).append(d)
    babies = {d % G for d in lp.shifts} - {0}
    counts["rot"] += len(babies)
    for g, ds in sorted(giants.items()):
        inner = np.zeros(plan.M)
        for d in ds:
            b = d % G
            inner += rot(y, b) * rot(mk[d], -g * G)
            counts["pmult"] += 1
        out += rot(inner, g * G)
        counts["rot"] += g != 0
    return out


def run(plan: Plan, x: np.ndarray, weights, counts: dict = None) -> List[np.ndarray]:
    """Run every layer on slot vectors; returns the final output as an n_v x F'
    matrix read from the output layout."""
    if counts is None:
        counts = dict(rot=0, pmult=0, smult=0, cmult=0)
    n = plan.n_v
    cur = None          # list of slot vectors, one column per vector (t = 1) or packed
    layout = None       # ("cols", None) or ("packed", t, B)
    for li, (lp, w) in enumerate(zip(plan.layers, weights)):
        if lp.kind == "inter" and lp.pack == "rep":
            copies = client_layout(plan, x, lp)
            pts = rep_plaintexts(plan, lp, w)
            J = len(copies[0])
            acc = sum(pts[k * J + j] * copies[k][j] for k in range(lp.K) for j in range(J))
            counts["pmult"] += lp.K * J
            for st in lp.fold_steps:
                acc = acc + rot(acc, st)
                counts["rot"] += 1
            cur = [acc]
            layout = ("packed", plan.M // lp.B, lp.B)
        elif lp.kind == "inter":
            copies = client_layout(plan, x, lp)
            pts = inter_plaintexts(plan, lp)
            z = [sum(pts[k] * copies[k][f] for k in range(lp.K)) for f in range(lp.f_in)]
            counts["pmult"] += lp.K * lp.f_in
            cur = [sum(w[f, l] * z[f] for f in range(lp.f_in)) for l in range(lp.f_out)]
            counts["smult"] += lp.f_in * lp.f_out
            layout = ("cols",)
        elif lp.comb == "diag":
            cm = diag_masks(plan, lp, w)
            y = sum(rot(cur[0], s_ * lp.B) * cm[s_] for s_ in lp.comb_shifts)
            counts["pmult"] += len(lp.comb_shifts)
            counts["rot"] += sum(1 for s_ in lp.comb_shifts if s_ != 0)
            cur = [aggregate_packed(plan, lp, y, lp.f_out, counts)]
            layout = ("packed", lp.t, lp.B)
        else:
            if li == 0:
                cur = client_layout(plan, x, lp)[0]
            cols = [sum(w[f, l] * cur[f] for f in range(lp.f_in)) for l in range(lp.f_out)]
            counts["smult"] += lp.f_in * lp.f_out
            packed = []
            for g in range(-(-lp.f_out // lp.t)):
                acc = np.zeros(plan.M)
                for l in range(g * lp.t, min(lp.f_out, (g + 1) * lp.t)):
                    c = l % lp.t
                    acc += rot(cols[l], -c * lp.B)
                    counts["rot"] += c != 0
                n_cols = min(lp.t, lp.f_out - g * lp.t)
                packed.append(aggregate_packed(plan, lp, acc, n_cols, counts))
            cur = packed
            layout = ("packed", lp.t, lp.B)
        if lp.activation:
            cur = [v * v for v in cur]
            counts["cmult"] += len(cur)
    return read_output(plan, cur, layout)


def read_output(plan: Plan, cts: List[np.ndarray], layout) -> np.ndarray:
    return read_output_layer(plan, plan.layers[-1], cts, layout)


def read_output_layer(plan: Plan, lp: LayerPlan, cts: List[np.ndarray], layout) -> np.ndarray:
    """Column l of the layer output: slot pi(v) of ciphertext l (one column per
    ciphertext) or slot (l mod t) B + pi(v) of packed ciphertext l div t."""
    n = plan.n_v
    out = np.zeros((n, lp.f_out))
    for l in range(lp.f_out):
        if layout[0] == "cols":
            out[:, l] = np.real(cts[l][plan.pi])
        else:
            t, B = layout[1], layout[2]
            out[:, l] = np.real(cts[l // t][(l % t) * B + plan.pi])
    return out
