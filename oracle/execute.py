"""A plan executed on oracle ciphertexts (test infrastructure only).

The words produced here are the bit-exact target for the GPU library.

Scale and level schedule (reading of Sec. 2.1's "each multiplication consumes
a level" with 50-bit primes and Delta = 2^40; the paper leaves it to its
library).  The scale is a double tracked through this exact sequence of IEEE
operations, starting from s = 2^log_scale at the top level L-1:
  Inter-CA layer at level l : P_k encoded at sP = q_l, weights at sW = q_{l-1};
                              s = (s * sP) * sW; s = s / q_l; s = s / q_{l-1}; l -= 2
  SpIntra-CA layer at level l, input not squared:
                              weights at sW = (q_l * Delta) / s;
                              s = s * sW; s = s / q_l; l -= 1
  SpIntra-CA layer at level l, input squared by the previous activation:
                              weights at sW = ((q_l * q_{l-1}) * Delta) / s;
                              s = s * sW; s = s / q_l; s = s / q_{l-1}; l -= 2
  then (SpIntra-CA)          masks at sM = q_l; s = s * sM; s = s / q_l; l -= 1
  (radix-2 routing, D steps)  the masks of a step at level l are encoded at
                              q_l and the step rescales by q_l, so every
                              result term keeps the scale s exactly; l -= D
  x^2 activation at level l : s = s * s (the rescale is deferred to the next
                              combination, or never for the model output, so
                              that no rounding happens below scale Delta)
Weights become integers c = round_half_even(w * sW); plaintexts are encoded
with round_half_even of the scaled inverse embedding.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List

import numpy as np

from . import ckks
from . import encoding as enc
from . import radix2
from . import simulate as sim
from .params import Params
from .planner import Plan


OUT_LEVEL = 1   # the model output keeps two primes (its scale reaches Delta^2 after x^2)


def levels_needed(plan: Plan) -> int:
    """Levels the layers consume: Inter-CA 2 (combination by integer weights) or 1 (case-1
    layout), SpIntra-CA 1 or 2 combination rescales (2 after a squared input) plus 1 mask
    level (the radix-2 program: its depth)."""
    need, pending = 0, False
    for lp in plan.layers:
        if lp.kind == "inter":
            need += 1 if lp.pack == "rep" else 2
        else:
            need += (2 if pending else 1) + (lp.program.depth if lp.family == 3 else 1)
        pending = lp.activation
    return need


def schedule(prm: Params, plan: Plan) -> List[dict]:
    s = float(2 ** prm.log_scale)
    delta = float(2 ** prm.log_scale)
    lv = prm.L - 1
    if plan.low_level:
        # the client's ciphertexts at the lowest level that leaves OUT_LEVEL for the output
        lv = min(lv, levels_needed(plan) + OUT_LEVEL)
    pending = False
    out = []
    for lp in plan.layers:
        st = dict(level_in=lv, scale_in=s)
        if lp.kind == "inter" and lp.pack == "rep":
            # case-1 layout: the plaintexts carry A_hat_k (x) W, one level
            if lv < 1:
                raise ValueError("not enough levels")
            st["sP"] = float(prm.q[lv])
            st["sW"] = 0.0
            s = s * st["sP"]
            s = s / float(prm.q[lv])
            lv -= 1
        elif lp.kind == "inter":
            if lv < 2:
                raise ValueError("not enough levels")
            st["sP"] = float(prm.q[lv])
            st["sW"] = float(prm.q[lv - 1])
            s = s * st["sP"]
            s = s * st["sW"]
            s = s / float(prm.q[lv])
            s = s / float(prm.q[lv - 1])
            lv -= 2
        else:
            st["n_rescale_comb"] = 2 if pending else 1
            if lv < st["n_rescale_comb"] + 1:
                raise ValueError("not enough levels")
            if pending:
                st["sW"] = ((float(prm.q[lv]) * float(prm.q[lv - 1])) * delta) / s
                s = s * st["sW"]
                s = s / float(prm.q[lv])
                s = s / float(prm.q[lv - 1])
                lv -= 2
            else:
                st["sW"] = (float(prm.q[lv]) * delta) / s
                s = s * st["sW"]
                s = s / float(prm.q[lv])
                lv -= 1
            st["level_agg"] = lv
            st["scale_agg"] = s
            st["sM"] = float(prm.q[lv])
            if lp.family == 3:
                depth = lp.program.depth
                if lv < depth:
                    raise ValueError("not enough levels for the radix-2 aggregation")
                lv -= depth
            else:
                s = s * st["sM"]
                s = s / float(prm.q[lv])
                lv -= 1
        st["level_pre_act"] = lv
        st["scale_pre_act"] = s
        pending = False
        if lp.activation:
            s = s * s
            pending = True
        st["squared_out"] = pending
        st["level_out"] = lv
        st["scale_out"] = s
        out.append(st)
    return out


def weight_ints(w: np.ndarray, sW: float) -> np.ndarray:
    return np.rint(np.asarray(w, dtype=np.float64) * np.float64(sW)).astype(np.int64)


def mask_vectors(plan: Plan, li: int) -> List[Dict[int, np.ndarray]]:
    """Per packed ciphertext g: slot vector per shift as the aggregation
    multiplies it (family 2 masks are pre-rotated by -g*G)."""
    lp = plan.layers[li]
    out = []
    for g in range(-(-lp.f_out // lp.t)):
        n_cols = min(lp.t, lp.f_out - g * lp.t)
        mk = sim.masks(plan, lp, n_cols)
        if lp.family == 2:
            mk = {d: sim.rot(v, -(d // lp.G) * lp.G) for d, v in mk.items()}
        out.append(mk)
    return out


def radix2_mask_vectors(plan: Plan, li: int):
    """Family 3: per packed ciphertext g, the program's masks in operand order
    as (depth, slot vector)."""
    lp = plan.layers[li]
    out = []
    for g in range(-(-lp.f_out // lp.t)):
        n_cols = min(lp.t, lp.f_out - g * lp.t)
        out.append([(dep, radix2.mask_vector(e, plan.M, lp.B, n_cols))
                    for dep, e in radix2.operand_list(lp.program)])
    return out


def encode_operands(prm: Params, plan: Plan, weights, sched=None) -> List[dict]:
    """Plaintext operands of every layer (the FP64 encoding step)."""
    sched = sched or schedule(prm, plan)
    ops = []
    for li, (lp, w, st) in enumerate(zip(plan.layers, weights, sched)):
        d = dict(W=weight_ints(w, st["sW"]))
        if lp.kind == "spintra" and lp.comb == "diag":
            # block-rotation combination masks at the weight scale, on the key basis for the
            # nonzero offsets (their products are taken before the one ModDown)
            cm = sim.diag_masks(plan, lp, w)
            lv = st["level_in"]
            d["CM"] = {s_: (enc.encode(prm, cm[s_], st["sW"], lv) if s_ == 0
                            else enc.encode_ext(prm, cm[s_], st["sW"], lv)) for s_ in lp.comb_shifts}
        if lp.kind == "inter" and lp.pack == "rep":
            lv = st["level_in"]
            d["P"] = [enc.encode(prm, p, st["sP"], lv) for p in sim.rep_plaintexts(plan, lp, w)]
        elif lp.kind == "inter":
            lv = st["level_in"]
            d["P"] = [enc.encode(prm, p, st["sP"], lv) for p in sim.inter_plaintexts(plan, lp)]
        elif lp.family == 4:
            lv = st["level_agg"]
            d["masks"] = [{dd: (enc.encode(prm, v, st["sM"], lv), enc.encode_ext(prm, v, st["sM"], lv))
                           for dd, v in mk.items()} for mk in mask_vectors(plan, li)]
        elif lp.family == 3:
            lv = st["level_agg"]
            d["masks"] = [[enc.encode(prm, v, float(prm.q[lv - dep]), lv - dep) for dep, v in per_g]
                          for per_g in radix2_mask_vectors(plan, li)]
        else:
            lv = st["level_agg"]
            d["masks"] = [{dd: enc.encode(prm, v, st["sM"], lv) for dd, v in mk.items()}
                          for mk in mask_vectors(plan, li)]
        ops.append(d)
    return ops


def client_encrypt(prm: Params, plan: Plan, x: np.ndarray, keys: ckks.Keys, seed: int) -> List[ckks.Ciphertext]:
    """The client's input ciphertexts, ct id = k * J + j (copy k, ciphertext j of the copy:
    column j, or columns j t .. j t + t - 1 in the case-1 layout)."""
    lp = plan.layers[0]
    copies = sim.client_layout(plan, x, lp)
    level = schedule(prm, plan)[0]["level_in"]
    cts = []
    for k, vecs in enumerate(copies):
        for f, v in enumerate(vecs):
            pt = enc.encode(prm, v, prm.scale, level)
            cts.append(ckks.encrypt(prm, seed, k * len(vecs) + f, keys.s, pt))
    return cts


def _zero(prm, level, scale):
    return ckks.zero_ct(prm, level, scale)


def run_layer(prm: Params, plan: Plan, li: int, keys: ckks.Keys, cts: List[ckks.Ciphertext],
              ops: dict, st: dict) -> List[ckks.Ciphertext]:
    lp = plan.layers[li]
    if lp.kind == "inter" and lp.pack == "rep":
        # Sec. 3.2 case 1: every input ciphertext times its A_hat_k (x) W plaintext, summed;
        # rescale; the t column blocks folded onto the first by ceil(log2 t) rotations
        lv = st["level_in"]
        acc = ckks.pt_mul_acc(prm, _zero(prm, lv, st["scale_in"] * st["sP"]), cts, ops["P"])
        acc = ckks.rescale(prm, acc)
        for step in lp.fold_steps:
            acc = ckks.add(prm, acc, ckks.rotate(prm, keys, acc, step))
        outs = [acc]
    elif lp.kind == "spintra" and lp.comb == "diag":
        # block-rotation combination of the packed input (one ModUp, the mask products on the
        # key basis, one ModDown), its rescales, then the aggregation on the packed blocks
        h = cts[0]
        steps = [s_ for s_ in lp.comb_shifts if s_ != 0]
        y = ckks.rotate_masked_sum(prm, keys, h, [s_ * lp.B for s_ in steps], [ops["CM"][s_] for s_ in steps])
        if 0 in lp.comb_shifts:
            y = ckks.pt_mul_acc(prm, y, [h], [ops["CM"][0]])
        y.scale = st["scale_in"] * st["sW"]
        for _ in range(st["n_rescale_comb"]):
            y = ckks.rescale(prm, y)
        outs = [aggregate(prm, plan, li, keys, y, ops["masks"][0], st)]
    elif lp.kind == "inter":
        lv = st["level_in"]
        F = lp.f_in
        Z = []
        for f in range(F):
            acc = _zero(prm, lv, st["scale_in"] * st["sP"])
            Z.append(ckks.pt_mul_acc(prm, acc, [cts[k * F + f] for k in range(lp.K)], ops["P"]))
        outs = []
        for l in range(lp.f_out):
            acc = _zero(prm, lv, st["scale_in"] * st["sP"] * st["sW"])
            h = ckks.scalar_mul_acc(prm, acc, Z, [int(ops["W"][f, l]) for f in range(F)])
            outs.append(ckks.rescale(prm, ckks.rescale(prm, h)))
    else:
        outs = [aggregate(prm, plan, li, keys, y, ops["masks"][g], st)
                for g, y in enumerate(combine_and_pack(prm, plan, li, keys, cts, ops, st))]
    if lp.activation:
        outs = [ckks.ct_mul_relin(prm, keys, c, c) for c in outs]
    return outs


def combine_and_pack(prm: Params, plan: Plan, li: int, keys: ckks.Keys, cts: List[ckks.Ciphertext],
                     ops: dict, st: dict) -> List[ckks.Ciphertext]:
    """SpIntra-CA layer with integer-weight combination: H_l = sum_f w_{f,l} X_f, its
    rescales, then columns g t .. g t + t - 1 packed into ciphertext g (column c moved
    to block c by a rotation of -c B).  One packed ciphertext per g."""
    lp = plan.layers[li]
    lv = st["level_in"]
    cols = []
    for l in range(lp.f_out):
        acc = _zero(prm, lv, st["scale_in"] * st["sW"])
        h = ckks.scalar_mul_acc(prm, acc, cts, [int(ops["W"][f, l]) for f in range(lp.f_in)])
        for _ in range(st["n_rescale_comb"]):
            h = ckks.rescale(prm, h)
        cols.append(h)
    packed = []
    for g in range(-(-lp.f_out // lp.t)):
        y = None
        for l in range(g * lp.t, min(lp.f_out, (g + 1) * lp.t)):
            c = l % lp.t
            term = cols[l] if c == 0 else ckks.rotate(prm, keys, cols[l], -c * lp.B)
            y = term if y is None else ckks.add(prm, y, term)
        packed.append(y)
    return packed


def aggregate_radix2(prm: Params, lp, keys, y: ckks.Ciphertext, masks: list, st: dict) -> ckks.Ciphertext:
    """The radix-2 program on one packed ciphertext (Sec. 3.3): every step's
    rotations hoisted on its register, Keep/Move masks summed into the next
    registers (rescaled once complete), Fin masks into the result term of
    the step's level; the result terms rescaled, dropped to the output level
    and summed."""
    prog = lp.program
    lv = y.level
    q = lambda dep: float(prm.q[lv - dep])
    it = iter(masks)
    regs = {0: y}
    pending = {}
    rots = {}

    def reg(r):
        if r in pending:
            regs[r] = ckks.rescale(prm, pending.pop(r))
        return regs[r]

    O = {0: ckks.pt_mul_acc(prm, _zero(prm, lv, y.scale * q(0)), [y], [next(it)])}
    for op in prog.ops:
        src = reg(op.src)
        need = [m for m in prog.amounts_of(op) if m != 0 and (op.src, m) not in rots]
        for m, c in zip(need, ckks.rotate_hoisted(prm, keys, src, need)):
            rots[(op.src, m)] = c
        rot = lambda m: src if m == 0 else rots[(op.src, m)]
        for t in sorted(op.keep):
            ms = sorted(op.keep[t])
            pts = [next(it) for _ in ms]
            acc = pending.get(t) or _zero(prm, src.level, src.scale * q(op.depth))
            pending[t] = ckks.pt_mul_acc(prm, acc, [rot(m) for m in ms], pts)
        fms = sorted(op.fin)
        if fms:
            pts = [next(it) for _ in fms]
            acc = O.get(op.depth) or _zero(prm, src.level, y.scale * q(op.depth))
            O[op.depth] = ckks.pt_mul_acc(prm, acc, [rot(m) for m in fms], pts)
    lo = lv - prog.depth
    out = None
    for dep in sorted(O):
        term = ckks.drop_to(ckks.rescale(prm, O[dep]), lo)
        out = term if out is None else ckks.add(prm, out, term)
    out.scale = y.scale
    return out


def aggregate(prm: Params, plan: Plan, li: int, keys, y: ckks.Ciphertext, masks, st: dict):
    lp = plan.layers[li]
    if lp.family == 3:
        return aggregate_radix2(prm, lp, keys, y, masks, st)
    acc = _zero(prm, y.level, y.scale * st["sM"])
    if lp.family == 4:
        # Sum_delta Rot_delta(Y) (.) mask_delta with the products on the key
        # basis and one ModDown; the identity shift is a plain mask product
        steps = [d for d in lp.shifts if d != 0]
        out = ckks.rotate_masked_sum(prm, keys, y, steps, [masks[d][1] for d in steps])
        if 0 in lp.shifts:
            out = ckks.pt_mul_acc(prm, out, [y], [masks[0][0]])
        out.scale = y.scale * st["sM"]
        return ckks.rescale(prm, out)
    if lp.family == 1:
        steps = [d for d in lp.shifts if d != 0]
        rots = dict(zip(steps, ckks.rotate_hoisted(prm, keys, y, steps)))
        rots[0] = y
        acc = ckks.pt_mul_acc(prm, acc, [rots[d] for d in lp.shifts], [masks[d] for d in lp.shifts])
    else:
        G = lp.G
        babies = sorted({d % G for d in lp.shifts} - {0})
        rb = dict(zip(babies, ckks.rotate_hoisted(prm, keys, y, babies)))
        rb[0] = y
        giants = {}
        for d in lp.shifts:
            giants.setdefault(d // G, []).append(d)
        # inner sums per giant step; the giant rotations are summed with one
        # ModDown (their key inner products added on the key basis first)
        rot_in, rot_k = [], []
        for g in sorted(giants):
            ds = giants[g]
            inner = ckks.pt_mul_acc(prm, _zero(prm, y.level, y.scale * st["sM"]),
                                    [rb[d % G] for d in ds], [masks[d] for d in ds])
            if (g * G) % prm.M == 0:
                acc = ckks.add(prm, acc, inner)
            else:
                rot_in.append(inner)
                rot_k.append(g * G)
        if rot_in:
            acc = ckks.add(prm, acc, ckks.rotate_sum(prm, keys, rot_in, rot_k))
    return ckks.rescale(prm, acc)


def run(prm: Params, plan: Plan, keys: ckks.Keys, cts: List[ckks.Ciphertext], ops: List[dict],
        sched=None, upto: int = None) -> List[List[ckks.Ciphertext]]:
    """Outputs of every layer (list per layer)."""
    sched = sched or schedule(prm, plan)
    outs = []
    cur = cts
    for li in range(len(plan.layers) if upto is None else upto):
        cur = run_layer(prm, plan, li, keys, cur, ops[li], sched[li])
        outs.append(cur)
    return outs


def decrypt_output(prm: Params, plan: Plan, keys: ckks.Keys, cts: List[ckks.Ciphertext], li: int = None) -> np.ndarray:
    li = len(plan.layers) - 1 if li is None else li
    lp = plan.layers[li]
    slots = [np.real(enc.decode(prm, ckks.decrypt(prm, keys.s, c))) for c in cts]
    if lp.kind == "inter" and lp.pack == "rep":
        return sim.read_output_layer(plan, lp, slots, ("packed", plan.M // lp.B, lp.B))
    if lp.kind == "inter":
        return sim.read_output_layer(plan, lp, slots, ("cols",))
    return sim.read_output_layer(plan, lp, slots, ("packed", lp.t, lp.B))
