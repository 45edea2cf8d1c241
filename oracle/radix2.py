"""The paper's own SpIntra-CA form: radix-2 routing with per-round masks
(Sec. 3.3), with the CPOO merges of Sec. 3.3.1 (test infrastructure only).

What is computed.  A packed ciphertext Y holds node u's value at slot pi(u)
(of every column block).  A demand (u -> v, A_hat[v, u]) must bring that value
to slot pi(v); its shift is delta = pi(u) - pi(v) (AOO-reduced on the wrapped
ring when t = 1).  The shift is decomposed into bits: in round r every demand
whose |delta| has bit r set moves by sign(delta) * 2^r, the others stay.  One
round of one working ciphertext C is

    C' = C (.) Keep + Rot(C, 2^r) (.) Move+ + Rot(C, -2^r) (.) Move-

(masks applied after the rotations, so the two rotations share one ModUp),
followed by a rescale: one level per round.  A demand that has reached its
target in round r is taken out of the working ciphertext and added to the
result with its coefficient:  O += Rot(C, +-2^r) (.) Fin (coefficients A_hat).
Demands with delta = 0 (the self loops) are Y (.) Fin0 at the top.  The
result terms of different rounds sit at different levels; each is rescaled
and dropped to the lowest one and the terms are summed.

Readings (each also listed in the design notes):
  * working ciphertexts ("lanes"): the demands are taken neighbour index by
    neighbour index (row v's non-self entries sorted by (|delta|, delta); the
    k-th of every row, rows in id order, before the (k+1)-th), each placed in
    the first lane (creation order) where it causes no slot conflict, else in
    a new lane -- the paper's "n neighbouring ciphertexts" with conflicts
    spilling into extra ciphertexts.  Every lane starts as Y itself (the
    masks of its first round remove what it does not carry).
  * slot conflict: after every round in which a demand is still travelling,
    each slot of a lane may hold values of one source node only (demands of
    one source at one slot carry the same value and share the slot);
  * rounds run r = 0, 1, ... up to the highest bit of any |delta|; a lane
    joins a round while it carries a demand whose highest bit is >= r, and
    skips it (no rotation, no mask, no level) when none of its demands moves
    in it: the step would be the identity on what the lane carries (at r = 0
    the lane still holds all of Y; the masks of its next step clear it).
  * CPOO (threshold theta on the ciphertext utilisation of Sec. 4.2.2): a
    lane is sparse when its live slots (distinct slots of the demands it
    carries on, per column block) are fewer than theta * B.
    (1) Postponing: a lane sparse at boundary r runs the rounds r .. r+w-1
        as one step: each demand moves by its window amount
        sign * (|delta| mod 2^(r+w) - |delta| mod 2^r); w is the largest
        whose distinct nonzero window amounts are no more than the rotations
        the w rounds would take one by one (ties -> the longer window, one
        level for w rounds).  The per-round assignment keeps the slots after
        the window conflict-free.
    (2) Merging: at boundary r the demands a sparse lane carries past round
        r are moved, slot by slot, into the first earlier lane that is not
        sparse, steps in round r, sits at the same level and causes no slot
        conflict for them
        in round r or later (the slot they reach after round r must be free
        there).  The move costs no level: the sparse lane's step writes
        those slots (after one round) into the other lane's next ciphertext.
        Merging comes first; then (1) applies to what the sparse lane keeps.
  * rotations of one ciphertext register by one amount are computed once
    (every lane's first round reads Y, so those rotations are shared).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np


def reduce_shift(delta: int, M: int, wrap: bool) -> int:
    """AOO (Sec. 3.3.1): with wrap, the representative of delta mod M in (-M/2, M/2]."""
    if not wrap:
        return delta
    r = delta % M
    return r - M if r > M // 2 else r


@dataclass
class Demand:
    u: int          # source node
    v: int          # target node
    s: int          # source slot pi(u) (inside a column block)
    e: int          # target slot pi(v)
    delta: int      # shift, e = s - delta (mod M)
    a: float        # A_hat[v, u]

    @property
    def mag(self) -> int:
        return abs(self.delta)

    @property
    def sign(self) -> int:
        return 1 if self.delta > 0 else -1

    @property
    def hb(self) -> int:
        """Round in which the demand arrives (its highest set bit)."""
        return self.mag.bit_length() - 1

    def partial(self, r: int) -> int:
        """Signed distance travelled after rounds 0 .. r."""
        return self.sign * (self.mag % (1 << (r + 1)))

    def pos(self, r: int, M: int) -> int:
        """Slot after round r (r = -1: the source slot)."""
        if r < 0:
            return self.s
        return (self.s - self.partial(r)) % M


@dataclass
class Step:
    """One step of one lane: rounds [r0, r1) on register `src` (level offset
    `depth` below the aggregation level).  keep[dst][m]: slots of register
    dst (depth + 1) fed from Rot(src, m); fin[m]: result slots with their
    coefficients fed from Rot(src, m)."""
    lane: int
    r0: int
    r1: int
    depth: int
    src: int
    keep: Dict[int, Dict[int, List[Tuple[int, float]]]]
    fin: Dict[int, List[Tuple[int, float]]]


@dataclass
class Program:
    self_fin: List[Tuple[int, float]]               # Y (.) Fin0: (slot, A_hat[v, v])
    ops: List[Step]                                 # execution order
    depth: int                                      # levels the aggregation consumes
    n_lanes: int                                    # lanes created by the assignment
    reg_depth: Dict[int, int] = field(default_factory=dict)
    n_moved: int = 0                                # demands moved by CPOO merging

    def amounts_of(self, op: Step) -> List[int]:
        ms = set(op.fin)
        for d in op.keep.values():
            ms |= set(d)
        return sorted(ms)

    def rotations(self) -> List[Tuple[int, int]]:
        """Distinct (register, amount != 0) rotations of the program."""
        out = []
        seen = set()
        for op in self.ops:
            for m in self.amounts_of(op):
                if m != 0 and (op.src, m) not in seen:
                    seen.add((op.src, m))
                    out.append((op.src, m))
        return out

    def amounts(self) -> List[int]:
        return sorted({m for _, m in self.rotations()})

    def n_steps(self) -> int:
        return len(self.ops)

    def out_depths(self) -> List[int]:
        """Depths at which result terms are accumulated (0: the self terms)."""
        return sorted({0} | {op.depth for op in self.ops if op.fin})

    def n_rescales(self) -> int:
        return len(self.reg_depth) - 1 + len(self.out_depths())


def demands(pi: np.ndarray, rows, M: int, wrap: bool):
    """Self terms and the travelling demands in assignment order."""
    self_fin = []
    per_row = []
    for v, row in enumerate(rows):
        lst = []
        for u, a in row:
            d = reduce_shift(int(pi[u] - pi[v]), M, wrap)
            if d == 0:
                self_fin.append((int(pi[v]), float(a)))
            else:
                lst.append(Demand(int(u), v, int(pi[u]), int(pi[v]), d, float(a)))
        lst.sort(key=lambda x: (x.mag, x.delta))
        per_row.append(lst)
    order = []
    k = 0
    while True:
        took = False
        for lst in per_row:
            if k < len(lst):
                order.append(lst[k])
                took = True
        if not took:
            break
        k += 1
    return self_fin, order


def assign_lanes(order: List[Demand], M: int):
    """First-fit of every demand into the lanes (creation order)."""
    lanes: List[List[Demand]] = []
    occ: List[Dict[Tuple[int, int], int]] = []
    for dm in order:
        traj = [(r, dm.pos(r, M)) for r in range(dm.hb)]     # slots while still travelling
        placed = False
        for k in range(len(lanes)):
            o = occ[k]
            if all(o.get(key, dm.u) == dm.u for key in traj):
                lanes[k].append(dm)
                for key in traj:
                    o[key] = dm.u
                placed = True
                break
        if not placed:
            lanes.append([dm])
            occ.append({key: dm.u for key in traj})
    return lanes, occ


def _live(lane: List[Demand], r: int) -> List[Demand]:
    return [d for d in lane if d.hb >= r]


def _live_slots(lane: List[Demand], r: int, M: int) -> set:
    """Slots of the demands still travelling after round r - 1."""
    return {d.pos(r - 1, M) for d in lane if d.hb >= r}


def _window_amount(d: Demand, r: int, w: int) -> int:
    return d.sign * ((d.mag % (1 << (r + w))) - (d.mag % (1 << r)))


def _window(lane: List[Demand], r: int) -> int:
    """CPOO (1): the longest window from r whose rotation count is no more
    than that of its rounds taken one by one."""
    live = _live(lane, r)
    r_end = max(d.hb for d in live) + 1
    best = 1
    single = 0
    for w in range(1, r_end - r + 1):
        rr = r + w - 1
        single += len({_window_amount(d, rr, 1) for d in live if d.hb >= rr} - {0})
        merged = len({_window_amount(d, r, w) for d in live} - {0})
        if merged <= single:
            best = w
    return best


def _occupancy(lane: List[Demand], M: int) -> Dict[Tuple[int, int], int]:
    occ = {}
    for d in lane:
        for r in range(d.hb):
            occ[(r, d.pos(r, M))] = d.u
    return occ


def build_program(pi: np.ndarray, rows, M: int, B: int, wrap: bool, theta: Optional[float] = None) -> Program:
    """The radix-2 aggregation program of one packed layout (Sec. 3.3; CPOO
    of Sec. 3.3.1 when theta is given).  Slots are block-local (< B); with
    t = 1 (B = M) positions wrap around the ring."""
    self_fin, order = demands(pi, rows, M, wrap)
    lane_dm, occ = assign_lanes(order, M)
    lanes = [dict(dm=list(d), occ=dict(o), reg=0, depth=0, bnd=0) for d, o in zip(lane_dm, occ)]
    R = max((d.hb + 1 for d in order), default=0)
    ops: List[Step] = []
    reg_depth = {0: 0}
    next_reg = 1
    out_depth = 1       # the self terms land one level down
    n_moved = 0
    for r in range(R):
        at = [k for k, ln in enumerate(lanes) if ln["bnd"] == r and _live(ln["dm"], r)]
        if not at:
            continue
        # the demands whose values sit in each lane's register now
        stepping = {k: _live(lanes[k]["dm"], r) for k in at}
        sparse = {k: theta is not None and len(_live_slots(lanes[k]["dm"], r, M)) < theta * B for k in at}
        home = {k: {id(d): k for d in stepping[k] if d.hb > r} for k in at}
        # CPOO (2): a sparse lane's demands that travel on after this round move
        # into an earlier, denser lane of the same level that takes one round
        for j in at:
            if not sparse[j]:
                continue
            slots = {}
            for d in stepping[j]:
                if d.hb > r:
                    slots.setdefault(d.pos(r, M), []).append(d)
            for i in at:
                if i >= j or not slots:
                    break
                if sparse[i] or lanes[i]["depth"] != lanes[j]["depth"]:
                    continue
                if not any((d.mag >> r) & 1 for d in stepping[i]):     # i skips this round
                    continue
                oi = lanes[i]["occ"]
                for q in sorted(slots):
                    ds = slots[q]
                    if (r, q) in oi:                  # one writer per slot of the next register
                        continue
                    u = ds[0].u
                    keys = {(x, d.pos(x, M)) for d in ds for x in range(r + 1, d.hb)}
                    if all(oi.get(key, u) == u for key in keys):
                        oi[(r, q)] = u
                        for key in keys:
                            oi[key] = u
                        for d in ds:
                            home[j][id(d)] = i
                            lanes[i]["dm"].append(d)
                        n_moved += len(ds)
                        del slots[q]
            moved = {i_ for i_, h in home[j].items() if h != j}
            if moved:
                lanes[j]["dm"] = [d for d in lanes[j]["dm"] if id(d) not in moved]
                lanes[j]["occ"] = _occupancy(lanes[j]["dm"], M)
        # CPOO (1): what a sparse lane still carries takes the longest useful window
        win = {}
        for k in at:
            own = [d for d in stepping[k] if d.hb == r or home[k][id(d)] == k]
            win[k] = _window(own, r) if sparse[k] and own else 1
        carry = {k: [d for d in stepping[k] if d.hb > r and (home[k][id(d)] != k or d.hb >= r + win[k])]
                 for k in at}
        idle = {k for k in at if all(h == k for h in home[k].values())
                and all(_window_amount(d, r, win[k]) == 0 for d in stepping[k])}
        # next registers, lanes in creation order
        receives = {home[k][id(d)] for k in at for d in carry[k]}
        dst = {}
        for k in at:
            if k in receives and k not in idle:
                dst[k] = next_reg
                reg_depth[next_reg] = lanes[k]["depth"] + 1
                next_reg += 1
        for k in at:
            if k in idle:
                continue
            ln = lanes[k]
            w = win[k]
            keep: Dict[int, Dict[int, List[Tuple[int, float]]]] = {}
            fin: Dict[int, List[Tuple[int, float]]] = {}
            seen = {}
            for d in stepping[k]:
                wd = w if d.hb == r or home[k][id(d)] == k else 1   # moved demands take one round
                m = _window_amount(d, r, wd)
                if d.hb < r + wd:
                    fin.setdefault(m, []).append((d.e, d.a))
                    continue
                tgt = dst[home[k][id(d)]]
                q = d.pos(r + wd - 1, M)
                if (tgt, q) in seen:
                    assert seen[(tgt, q)] == (d.u, m)
                    continue
                seen[(tgt, q)] = (d.u, m)
                keep.setdefault(tgt, {}).setdefault(m, []).append((q, 1.0))
            ops.append(Step(k, r, r + w, ln["depth"], ln["reg"],
                            {t: {m: sorted(e) for m, e in km.items()} for t, km in keep.items()},
                            {m: sorted(e) for m, e in fin.items()}))
            out_depth = max(out_depth, ln["depth"] + 1)
        for k in at:
            ln = lanes[k]
            ln["bnd"] = r + win[k]
            if k not in idle:
                ln["depth"] += 1
                ln["reg"] = dst.get(k, -1)
    return Program(self_fin=sorted(self_fin), ops=ops, depth=out_depth, n_lanes=len(lane_dm),
                   reg_depth=reg_depth, n_moved=n_moved)


# ----------------------------------------------------------------------------
# the program on cleartext slot vectors
# ----------------------------------------------------------------------------
def mask_vector(entries, M: int, B: int, n_cols: int) -> np.ndarray:
    """Block-local (slot, value) entries replicated over the first n_cols blocks."""
    v = np.zeros(M)
    for q, a in entries:
        for c in range(n_cols):
            v[c * B + q] = a
    return v


def operand_list(prog: Program):
    """The program's masks in their fixed order: Fin0 first, then per step its
    Keep/Move masks by (next register, amount) (amount 0 = Keep), then its
    Fin masks by amount.  Entries: (depth, entries)."""
    out = [(0, prog.self_fin)]
    for op in prog.ops:
        for t in sorted(op.keep):
            for m in sorted(op.keep[t]):
                out.append((op.depth, op.keep[t][m]))
        for m in sorted(op.fin):
            out.append((op.depth, op.fin[m]))
    return out


def run_slots(prog: Program, y: np.ndarray, B: int, n_cols: int, counts: Optional[dict] = None) -> np.ndarray:
    """The program on a slot vector y (Rot(v, k)_j = v_{j+k})."""
    M = len(y)
    regs = {0: y}
    rots = {}
    out = y * mask_vector(prog.self_fin, M, B, n_cols)
    if counts is not None:
        counts["pmult"] += 1

    def rot(reg, m):
        if m == 0:
            return regs[reg]
        if (reg, m) not in rots:
            rots[(reg, m)] = np.roll(regs[reg], -m)
            if counts is not None:
                counts["rot"] += 1
        return rots[(reg, m)]

    for op in prog.ops:
        for t in sorted(op.keep):
            for m in sorted(op.keep[t]):
                regs[t] = regs.get(t, 0) + rot(op.src, m) * mask_vector(op.keep[t][m], M, B, n_cols)
                if counts is not None:
                    counts["pmult"] += 1
        for m in sorted(op.fin):
            out = out + rot(op.src, m) * mask_vector(op.fin[m], M, B, n_cols)
            if counts is not None:
                counts["pmult"] += 1
    return out
