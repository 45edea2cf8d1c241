"""Plan construction for the encrypted GCN (test infrastructure only).

What a plan fixes, following the paper:
  * packing (Sec. 3.2, App. B): t feature columns per ciphertext, column-major:
    column c of a ciphertext sits in slots [c*B, (c+1)*B), B = M/t, node v at
    slot c*B + pi(v);
  * aggregation mode per layer (Sec. 3.3.2): the first layer is Inter-CA over
    client-provided neighbour copies; later layers use SpIntra-CA;
  * SpIntra-CA routing (Sec. 3.3): every nonzero A_vu is a demand moving u's
    value by the shift delta = pi(u) - pi(v) onto v's slot; demands that share a
    shift share one rotation and one mask (the diagonal form), or one baby and
    one giant rotation (the baby-step/giant-step form), or travel bit by bit
    through per-round masks (the paper's radix-2 form, oracle.radix2);
  * node order pi (Sec. 3.4, Alg. 1): sibling-BFS regions capped at TH nodes,
    interleaved region by region, then a greedy conflict-least placement;
  * AOO (Sec. 3.3.1): with one column per ciphertext (t = 1) a shift is taken
    mod M in (-M/2, M/2], the shorter way round the ring.

Readings of points the paper leaves open (each also listed in the design notes):
  * the region loop of Alg. 1 (stage 1) runs while the region has fewer than
    TH nodes and the sibling BFS is not exhausted; when
    the sibling BFS runs dry before TH, it restarts inside the same region
    from the highest-degree node not yet in any region.
  * degree(v) = number of u != v with A_vu != 0 or A_uv != 0; ties -> smaller id.
  * sibling of x: w != x with A_vx != 0 and A_vw != 0 for some v (diagonal
    included), enqueued in ascending id.
  * interleave: round-robin over regions; an exhausted region's turn takes a
    blank slot while blanks remain, else it is skipped.
  * greedy placement (Alg. 1, stage 3): nodes of a region in BFS order, the
    first at the region's first slot; every later node goes to the free slot
    of its region that adds the fewest shifts not yet in the plan's shift set
    (ties -> lowest slot).  For the diagonal form every distinct shift is one
    rotation, so "conflicts" are counted as new distinct shifts.
"""
from __future__ import annotations

import math
from collections import deque
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import radix2


# ----------------------------------------------------------------------------
# the paper's analytic cost formulas (Sec. 3.2, Sec. 3.3.2, App. B)
# ----------------------------------------------------------------------------
def ceil_div(a: int, b: int) -> int:
    return -(-a // b)


def clog2(x: int) -> int:
    return 0 if x <= 1 else int(math.ceil(math.log2(x)))


def j_objective(t: int, F: int, n: int) -> int:
    """Case M > N F': J(t; F, n) = 2 ceil(F n / t) + 20 ceil(log t)."""
    return 2 * ceil_div(F * n, t) + 20 * clog2(t)


def case2_pmults(t: int, F: int, n: int, n_nodes: int, F_out: int, M: int) -> int:
    """Case M <= N F': #PMult = #Add = ceil(F n / t) * ceil(N F' / ceil(M / t))."""
    return ceil_div(F * n, t) * ceil_div(n_nodes * F_out, ceil_div(M, t))


def paper_packing_t(F: int, n: int, n_nodes: int, F_out: int, M: int) -> int:
    """t from the paper's rule: t = 1 when M <= N F'; otherwise the argmin of J
    over powers of two with t N F' <= M (ties -> smaller t)."""
    if M <= n_nodes * F_out:
        return 1
    best, best_j = 1, j_objective(1, F, n)
    t = 2
    while t * n_nodes * F_out <= M:
        j = j_objective(t, F, n)
        if j < best_j:
            best, best_j = t, j
        t *= 2
    return best


def rep_block(t: int, f_out: int, n_nodes: int, M: int) -> Optional[int]:
    """Node block Bc of the case-1 layout (Sec. 3.2, App. B): a ciphertext holds t input
    columns, each repeated for the layer's F' output columns, every (input column, output
    column) pair a block of Bc = M / (t pow2(F')) slots holding the nodes; None when
    pow2(n_nodes) does not fit Bc (the paper's t N F' <= M with N and F' rounded up to
    powers of two)."""
    if t < 1 or f_out < 1:
        return None
    Bc = M // (t * next_pow2(f_out))
    return Bc if Bc >= next_pow2(n_nodes) else None


def rule_packing(F: int, n: int, n_nodes: int, F_out: int, M: int, later_widths=()) -> tuple:
    """The first layer's packing by the paper's rule (Sec. 3.2, App. B): case M <= N F' ->
    one column per ciphertext ("cols", 1); else the case-1 layout at the J argmin t
    (paper_packing_t), halved while the layout does not fit or a later layer's width
    exceeds its column capacity M / Bc."""
    if M <= n_nodes * F_out:
        return ("cols", 1)
    t = paper_packing_t(F, n, n_nodes, F_out, M)
    while t >= 1:
        Bc = rep_block(t, F_out, n_nodes, M)
        if Bc is not None and all(f <= M // Bc for f in later_widths):
            return ("rep", t)
        t //= 2
    return ("cols", 1)


def paper_agg_mode(F: int, n: int, t: int, n_nodes: int, c: float) -> str:
    """argmin{ Inter-CA: 2 ceil(F n / t), SpIntra-CA: 10 c n log^2 N } (Sec. 3.3.2)."""
    inter = 2 * ceil_div(F * n, t)
    spintra = 10.0 * c * n * math.log2(n_nodes) ** 2
    return "inter" if inter <= spintra else "spintra"


def spintra_worst_case_rots(n: int, n_nodes: int) -> int:
    """Worst case of Sec. 3.3.1: (n - 1) log^2 N rotations."""
    return (n - 1) * clog2(n_nodes) ** 2


# ----------------------------------------------------------------------------
# graph helpers
# ----------------------------------------------------------------------------
def support(rows) -> List[set]:
    """Undirected support of A_hat without the diagonal."""
    n = len(rows)
    s = [set() for _ in range(n)]
    for v, row in enumerate(rows):
        for u, _ in row:
            if u != v:
                s[v].add(u)
                s[u].add(v)
    return s


def siblings(rows) -> List[List[int]]:
    """sib[x] = sorted w != x sharing a row of A_hat (diagonal included) with x."""
    n = len(rows)
    sib = [set() for _ in range(n)]
    for row in rows:
        us = [u for u, _ in row]
        for a in us:
            sib[a].update(us)
    return [sorted(x - {i}) for i, x in enumerate(sib)]


def reduce_shift(delta: int, M: int, wrap: bool) -> int:
    """AOO: with wrap, the representative of delta mod M in (-M/2, M/2]."""
    if not wrap:
        return delta
    r = delta % M
    return r - M if r > M // 2 else r


# ----------------------------------------------------------------------------
# node order optimisation (Alg. 1)
# ----------------------------------------------------------------------------
def noo_regions(rows, TH: int) -> List[List[int]]:
    """Stage 1 of Alg. 1 (detection): sibling-BFS regions of at most TH nodes."""
    n = len(rows)
    deg = [len(x) for x in support(rows)]
    sib = siblings(rows)
    order = sorted(range(n), key=lambda v: (-deg[v], v))   # highest degree first
    remaining = [True] * n
    regions = []
    ptr = 0
    n_left = n
    while n_left > 0:
        region = []
        visited = set()
        while len(region) < TH and n_left > 0:
            while not remaining[order[ptr]]:
                ptr += 1
            start = order[ptr]
            queue = deque([start])
            visited.add(start)
            while queue and len(region) < TH:
                x = queue.popleft()
                region.append(x)
                remaining[x] = False
                n_left -= 1
                for w in sib[x]:
                    if remaining[w] and w not in visited:
                        visited.add(w)
                        queue.append(w)
        regions.append(region)
    return regions


def interleave_slots(sizes: Sequence[int], B: int) -> List[List[int]]:
    """Stage 2 of Alg. 1 (interleaved arrangement): slots of each region in the interleaved
    arrangement ABCABC... over [0, B)."""
    R = len(sizes)
    left = list(sizes)
    blanks = B - sum(sizes)
    if blanks < 0:
        raise ValueError("graph does not fit the block")
    slots = [[] for _ in range(R)]
    j = 0
    while any(x > 0 for x in left):
        for r in range(R):
            if left[r] > 0:
                slots[r].append(j)
                left[r] -= 1
                j += 1
            elif blanks > 0:
                blanks -= 1
                j += 1
    return slots


def demand_cells(s: int, delta: int, M: int) -> List[Tuple[int, int]]:
    """The (round, slot) cells a radix-2 demand occupies (Sec. 3.3): it starts at slot s
    and, in round r, moves by sign(delta) 2^r when bit r of |delta| is set; after each
    round r below its highest bit it still travels and sits at
    s - sign (|delta| mod 2^(r+1)) (mod M); in the round of its highest bit it arrives
    and leaves the working ciphertext."""
    mag, sg = abs(delta), (1 if delta > 0 else -1)
    return [(r, (s - sg * (mag % (1 << (r + 1)))) % M) for r in range(max(0, mag.bit_length() - 1))]


def noo_place(rows, regions, slots, M: int, wrap: bool, objective: str = "shifts") -> np.ndarray:
    """Stage 3 of Alg. 1 (conflict-least search): nodes in BFS order, each at the free
    slot of its region with the least cost (ties -> lowest slot).  objective "shifts"
    (the diagonal and baby-step/giant-step forms, which pay per distinct shift): the
    number of shifts the node's demands add to the plan.  objective "conflicts" (the
    radix-2 form, whose extra working ciphertexts come from slot conflicts, Sec. 3.3):
    the number of (round, slot) cells where the node's demands with already placed
    nodes meet a placed demand of another source node (demand_cells)."""
    if objective not in ("shifts", "conflicts"):
        raise ValueError(objective)
    n = len(rows)
    out_nb = [[u for u, _ in row if u != v] for v, row in enumerate(rows)]   # v needs u
    in_nb = [[] for _ in range(n)]                                           # v needs x: x's in
    for v in range(n):
        for u in out_nb[v]:
            in_nb[u].append(v)
    pi = np.full(n, -1, dtype=np.int64)
    shiftset = set()
    R = M.bit_length()
    occ = np.full((R, M), -1, dtype=np.int64)       # source node per (round, slot); -2: several

    def occupy(src, s_, delta):
        for r, c in demand_cells(s_, delta, M):
            cur = occ[r, c]
            occ[r, c] = src if cur == -1 else (cur if cur == src else -2)

    def add_shifts(x):
        for u in out_nb[x]:
            if pi[u] >= 0:
                d = reduce_shift(int(pi[u] - pi[x]), M, wrap)
                shiftset.add(d)
                if objective == "conflicts":
                    occupy(u, int(pi[u]), d)
        for v in in_nb[x]:
            if pi[v] >= 0:
                d = reduce_shift(int(pi[x] - pi[v]), M, wrap)
                shiftset.add(d)
                if objective == "conflicts":
                    occupy(x, int(pi[x]), d)

    def red(D):
        if wrap:
            D = D % M
            D = np.where(D > M // 2, D - M, D)
        return D

    def conflict_cost(x, pos):
        cost = np.zeros(len(pos), dtype=np.int64)

        def walk(src, s_, D):
            mag, sg = np.abs(D), np.where(D > 0, 1, -1)
            for r in range(R):
                live = (mag >> (r + 1)) > 0                  # still travelling after round r
                if not live.any():
                    break
                c = (s_ - sg * (mag % (1 << (r + 1)))) % M
                o = occ[r, c]
                cost[:] += live & (o != -1) & (o != src)

        for u in out_nb[x]:
            if pi[u] >= 0:                                   # demand u -> x
                walk(u, int(pi[u]), red(pi[u] - pos))
        for v in in_nb[x]:
            if pi[v] >= 0:                                   # demand x -> v
                walk(x, pos, red(pos - pi[v]))
        return cost

    for region, sl in zip(regions, slots):
        free = np.array(sl, dtype=np.int64)
        taken = np.zeros(len(free), dtype=bool)
        first = region[0]
        pi[first] = free[0]
        taken[0] = True
        add_shifts(first)
        for x in region[1:]:
            cand = np.nonzero(~taken)[0]
            pos = free[cand]
            if objective == "conflicts":
                has = any(pi[u] >= 0 for u in out_nb[x]) or any(pi[v] >= 0 for v in in_nb[x])
                k = int(np.argmin(conflict_cost(x, pos))) if has else 0
            else:
                rows_d = []
                for u in out_nb[x]:
                    if pi[u] >= 0:
                        rows_d.append(pi[u] - pos)
                for v in in_nb[x]:
                    if pi[v] >= 0:
                        rows_d.append(pos - pi[v])
                if rows_d:
                    D = red(np.stack(rows_d))
                    D = np.sort(D, axis=0)
                    known = np.isin(D, np.fromiter(shiftset, dtype=np.int64, count=len(shiftset)))
                    first_of_run = np.ones_like(known)
                    first_of_run[1:] = D[1:] != D[:-1]
                    cost = np.sum(~known & first_of_run, axis=0)
                    k = int(np.argmin(cost))          # lowest slot among minima
                else:
                    k = 0
            pi[x] = pos[k]
            taken[cand[k]] = True
            add_shifts(x)
    return pi


def noo(rows, B: int, M: int, TH: int, objective: str = "shifts") -> tuple:
    regions = noo_regions(rows, TH)
    slots = interleave_slots([len(r) for r in regions], B)
    pi = noo_place(rows, regions, slots, M, wrap=(B == M), objective=objective)
    return pi, regions


# ----------------------------------------------------------------------------
# plans
# ----------------------------------------------------------------------------
@dataclass
class LayerPlan:
    kind: str                 # "inter" | "spintra"
    f_in: int
    f_out: int
    activation: bool
    # inter
    K: int = 0
    copy_src: Optional[np.ndarray] = None     # (K, n_v) source node, -1 = none
    copy_val: Optional[np.ndarray] = None     # (K, n_v) A_hat value
    # spintra
    t: int = 1                # columns per packed ciphertext
    B: int = 0                # block = M / t
    shifts: List[int] = field(default_factory=list)      # sorted distinct shifts
    family: int = 1           # 1 = diagonal, 2 = baby-step/giant-step, 3 = radix-2 per-round masks,
                              # 4 = diagonal with the mask products before one ModDown (double hoisting)
    G: int = 1                # baby-step count of the family-2 split
    program: object = None    # family 3: the radix-2 program (oracle.radix2.Program)
    cpoo: Optional[float] = None   # family 3: CPOO sparsity threshold (None = off)
    # shifts per (ciphertext) of the pack step: -l*B for l = 1..t-1
    pack_steps: List[int] = field(default_factory=list)
    # inter: "cols" (one input column per ciphertext, the combination as integer-weight
    # sums) or "rep" (the case-1 layout of Sec. 3.2 / App. B: t input columns per
    # ciphertext repeated over the F' output columns, plaintexts A_hat_k (x) W-slice,
    # the t column blocks summed by ceil(log2 t) rotations; t, B = Bc, fold_steps)
    pack: str = "cols"
    fold_steps: List[int] = field(default_factory=list)
    # spintra: "scalar" (columns combined by integer weights, then packed by rotations)
    # or "diag" (input already packed in blocks of B: output block c = sum_l W[l, c] *
    # input block l, as sum over s of Rot_{sB}(input) (.) cm_s with cm_s block c =
    # W[c + s, c]; s in comb_shifts)
    comb: str = "scalar"
    comb_shifts: List[int] = field(default_factory=list)
    # Sec. 3.3.2's aggregation-mode formula for this layer (later layers): the chosen mode
    # and both costs (Inter-CA 2 ceil(F n / t), SpIntra-CA 10 c n log2(N)^2)
    paper_mode: Optional[str] = None
    paper_mode_costs: tuple = ()


@dataclass
class Plan:
    n_v: int
    M: int
    B_pi: int
    pi: np.ndarray
    rows: list
    layers: List[LayerPlan]
    regions: List[List[int]] = field(default_factory=list)
    # the client encrypts at the lowest level the layers need (the spare primes of the chain
    # are never used) instead of the top level
    low_level: bool = False

    @property
    def n_out_cts(self) -> int:
        last = self.layers[-1]
        if last.kind == "inter":
            return 1 if last.pack == "rep" else last.f_out
        return ceil_div(last.f_out, last.t)

    def rot_steps(self, M: int) -> List[int]:
        steps = set()
        for lp in self.layers:
            steps.update(s % M for s in lp.fold_steps)
            steps.update((s * lp.B) % M for s in lp.comb_shifts)
            if lp.kind != "spintra":
                continue
            steps.update(s % M for s in lp.pack_steps)
            for s in rotation_steps_of(lp):
                steps.add(s % M)
        steps.discard(0)
        return sorted(steps)


def next_pow2(x: int) -> int:
    p = 1
    while p < x:
        p *= 2
    return p


def bsgs_split(shifts: Sequence[int], B: int):
    """Baby-step count G (a power of two <= B) minimising distinct nonzero
    babies + giants for delta = g*G + b, b in [0, G); ties -> smaller G."""
    best = None
    G = 1
    while G <= max(B, 1):
        babies = {d % G for d in shifts} - {0}
        giants = {d // G for d in shifts} - {0}
        c = len(babies) + len(giants)
        if best is None or c < best[0]:
            best = (c, G)
        G *= 2
    return best[1], best[0]


def rotation_steps_of(lp: LayerPlan) -> List[int]:
    """Rotation steps the aggregation uses (nonzero)."""
    if lp.family == 3:
        return lp.program.amounts()
    if lp.family in (1, 4):
        return sorted(set(lp.shifts) - {0})
    babies = {d % lp.G for d in lp.shifts} - {0}
    giants = {(d // lp.G) * lp.G for d in lp.shifts} - {0}
    return sorted(babies | giants)


def _inter_copies(n_v: int, rows, K: int):
    """Copy k of node v: its k-th non-self term (copy 0 = the node itself)."""
    src = np.full((K, n_v), -1, dtype=np.int64)
    val = np.zeros((K, n_v))
    for v, row in enumerate(rows):
        k = 1
        for u, a in row:
            if u == v:
                src[0, v], val[0, v] = v, a
            else:
                src[k, v], val[k, v] = u, a
                k += 1
    return src, val


def _mode_costs(f_in: int, n: int, t: int, n_v: int, c: float):
    inter = 2 * ceil_div(f_in * n, t)
    spintra = 10.0 * c * n * math.log2(max(n_v, 2)) ** 2
    return ("inter" if inter <= spintra else "spintra"), (inter, spintra)


def _spintra_layer(n_v, rows, pi, M, B, f_in, f_out, activation, family, cpoo, aoo):
    """SpIntra-CA routing of one layer on blocks of B slots (shared by both layouts)."""
    wrap = B == M
    shifts = sorted({reduce_shift(int(pi[u] - pi[v]), M, wrap) for v, row in enumerate(rows) for u, _ in row})
    G, c2 = bsgs_split(shifts, B)
    c1 = len(set(shifts) - {0})
    fam = family if family is not None else (2 if c2 < c1 else 1)
    prog = radix2.build_program(pi, rows, M, B, wrap and aoo, cpoo) if fam == 3 else None
    return LayerPlan("spintra", f_in, f_out, activation, t=M // B, B=B, shifts=shifts, family=fam, G=G,
                     program=prog, cpoo=cpoo if fam == 3 else None)


def _build_rep_plan(n_v, rows, dims, activation, M, use_noo, TH, family, t1, cpoo, agg_c, K):
    """Inter-CA first layer in the case-1 layout at packing t1; every later layer is
    SpIntra-CA on the packed blocks of Bc slots with the block-rotation combination."""
    n_layers = len(dims) - 1
    Bc = rep_block(t1, dims[1], n_v, M)
    if TH is None:
        TH = 1024 if n_v < 10000 else 4096
    if use_noo:
        pi, regions = noo(rows, Bc, M, TH, "conflicts" if family == 3 else "shifts")
    else:
        if n_v > Bc:
            raise ValueError("graph does not fit the column block")
        pi, regions = np.arange(n_v, dtype=np.int64), [list(range(n_v))]
    src, val = _inter_copies(n_v, rows, K)
    S = next_pow2(dims[1]) * Bc
    lp0 = LayerPlan("inter", dims[0], dims[1], activation, K=K, copy_src=src, copy_val=val, pack="rep",
                    t=t1, B=Bc, fold_steps=[(1 << i) * S for i in range(clog2(t1))])
    layers = [lp0]
    for li in range(1, n_layers):
        f_in, f_out = dims[li], dims[li + 1]
        lp = _spintra_layer(n_v, rows, pi, M, Bc, f_in, f_out, activation, family, cpoo, True)
        lp.comb = "diag"
        lp.comb_shifts = list(range(-(f_out - 1), f_in))
        lp.paper_mode, lp.paper_mode_costs = _mode_costs(f_in, K - 1, lp.t, n_v, agg_c)
        layers.append(lp)
    return Plan(n_v=n_v, M=M, B_pi=Bc, pi=pi, rows=rows, layers=layers, regions=regions)


def build_plan(n_v: int, rows, dims: Sequence[int], activation: bool, M: int,
               use_noo: bool = True, TH: Optional[int] = None, family: Optional[int] = None,
               first_mode: str = "inter", t: Optional[int] = None, cpoo: Optional[float] = None,
               aoo: bool = True, first_pack="cols", agg_c: float = 1.0, low_level: bool = False) -> Plan:
    """The executable plan (_build_plan); low_level: the client encrypts at the lowest level
    the layers need instead of the top of the chain (execute.schedule)."""
    plan = _build_plan(n_v, rows, dims, activation, M, use_noo, TH, family, first_mode, t, cpoo, aoo, first_pack,
                       agg_c)
    plan.low_level = low_level
    return plan


def _build_plan(n_v: int, rows, dims: Sequence[int], activation: bool, M: int,
                use_noo: bool = True, TH: Optional[int] = None, family: Optional[int] = None,
                first_mode: str = "inter", t: Optional[int] = None, cpoo: Optional[float] = None,
                aoo: bool = True, first_pack="cols", agg_c: float = 1.0) -> Plan:
    """The executable plan: layer 1 by `first_mode` ("inter" per the paper's
    first-layer rule, or "spintra"), later layers SpIntra-CA; SpIntra layers
    combine first (F -> F' at one column per ciphertext), pack t = min(pow2(F'),
    M / pow2(n_v)) columns per ciphertext, then aggregate on the packed layout
    (t = 1 for every SpIntra layer when one of them feeds another layer).
    A given t (a power of two no larger than pow2(F') of every SpIntra layer
    and M / pow2(n_v)) replaces that rule for every SpIntra layer.
    family: None = the cheaper of 1 and 2 by rotation count; 3 = the paper's
    radix-2 routing (Sec. 3.3), with CPOO at threshold `cpoo` when given;
    aoo=False takes its shifts unreduced around the ring (the AOO ablation).
    first_pack (Inter-CA first layer): "cols" = one column per ciphertext; "rule" = the
    paper's packing rule (rule_packing: case 1 layout at the J argmin t, else "cols"); an
    int t = the case-1 layout at that t.  With the case-1 layout every later layer takes its
    input packed in blocks of Bc and combines it by block rotations ("diag").
    agg_c: the factor c of Sec. 3.3.2's aggregation-mode formula, recorded per later layer."""
    n_layers = len(dims) - 1
    if first_mode == "spintra" and n_layers > 1:
        raise ValueError("a SpIntra-CA layer leaves packed ciphertexts; only the last layer may be SpIntra-CA "
                         "when it is also the first")
    K_all = 1 + max(sum(1 for u, _ in row if u != v) for v, row in enumerate(rows))
    pack1, t1 = "cols", 1
    if first_mode == "inter" and first_pack != "cols":
        later = list(dims[2:])
        if first_pack == "rule":
            pack1, t1 = rule_packing(dims[0], K_all - 1, n_v, dims[1], M, later)
        else:
            t1 = int(first_pack)
            Bc = rep_block(t1, dims[1], n_v, M) if t1 >= 1 and not t1 & (t1 - 1) else None
            if Bc is None or any(f > M // Bc for f in later):
                raise ValueError("the case-1 layout does not fit at t = %d" % t1)
            pack1 = "rep"
    if pack1 == "rep":
        return _build_rep_plan(n_v, rows, dims, activation, M, use_noo, TH, family, t1, cpoo, agg_c, K_all)
    # packing of the SpIntra layers fixes the block the node order must fit; a
    # SpIntra layer that feeds another layer leaves one column per ciphertext
    # (the next combination reads columns), so then every SpIntra layer packs t = 1
    spin = [i for i in range(n_layers) if i > 0 or first_mode == "spintra"]
    spin_f = [dims[i + 1] for i in spin]
    t_pack = min([next_pow2(f) for f in spin_f] + [M // next_pow2(n_v)]) if spin_f else 1
    if any(i < n_layers - 1 for i in spin):
        t_pack = 1
    if t is not None and spin_f:
        if t < 1 or t & (t - 1) or t > t_pack:
            raise ValueError("packing t must be a power of two no larger than %d" % t_pack)
        t_pack = t
    B = M // t_pack
    if TH is None:
        TH = 1024 if n_v < 10000 else 4096
    if use_noo:
        pi, regions = noo(rows, B, M, TH, "conflicts" if family == 3 else "shifts")
    else:
        pi, regions = np.arange(n_v, dtype=np.int64), [list(range(n_v))]
    layers = []
    for li in range(n_layers):
        f_in, f_out = dims[li], dims[li + 1]
        kind = first_mode if li == 0 else "spintra"
        if kind == "inter":
            K = 1 + max(sum(1 for u, _ in row if u != v) for v, row in enumerate(rows))
            src = np.full((K, n_v), -1, dtype=np.int64)
            val = np.zeros((K, n_v))
            for v, row in enumerate(rows):
                k = 1
                for u, a in row:
                    if u == v:
                        src[0, v], val[0, v] = v, a
                    else:
                        src[k, v], val[k, v] = u, a
                        k += 1
            layers.append(LayerPlan("inter", f_in, f_out, activation, K=K, copy_src=src, copy_val=val))
        else:
            t_l = t_pack
            Bl = M // t_l
            wrap = Bl == M
            shifts = sorted({reduce_shift(int(pi[u] - pi[v]), M, wrap) for v, row in enumerate(rows)
                             for u, _ in row})
            G, c2 = bsgs_split(shifts, Bl)
            c1 = len(set(shifts) - {0})
            fam = family if family is not None else (2 if c2 < c1 else 1)
            prog = radix2.build_program(pi, rows, M, Bl, wrap and aoo, cpoo) if fam == 3 else None
            pack = [-(l % t_l) * Bl for l in range(f_out) if l % t_l != 0]
            lpl = LayerPlan("spintra", f_in, f_out, activation, t=t_l, B=Bl, shifts=shifts,
                            family=fam, G=G, pack_steps=sorted(set(pack)), program=prog,
                            cpoo=cpoo if fam == 3 else None)
            if li > 0:
                lpl.paper_mode, lpl.paper_mode_costs = _mode_costs(f_in, K_all - 1, 1, n_v, agg_c)
            layers.append(lpl)
    return Plan(n_v=n_v, M=M, B_pi=B, pi=pi, rows=rows, layers=layers, regions=regions)


# ----------------------------------------------------------------------------
# operation counts of a plan (HE operation counts, Table 1)
# ----------------------------------------------------------------------------
def op_counts(plan: Plan) -> dict:
    c = dict(rot=0, pmult=0, cmult=0, smult=0, add=0, rescale=0, keyswitch=0)
    n_cts = None
    for li, lp in enumerate(plan.layers):
        if lp.kind == "inter" and lp.pack == "rep":
            # Sec. 3.2 case 1: ceil(F K / t) PMult and Add (one per input ciphertext, each with its
            # A_hat_k (x) W plaintext, accumulated), ceil(log2 t) rotations folding the column blocks
            n_in = lp.K * ceil_div(lp.f_in, lp.t)
            c["pmult"] += n_in
            c["add"] += n_in
            c["rot"] += clog2(lp.t)
            c["rescale"] += 1
            n_cts = 1
        elif lp.kind == "inter":
            c["pmult"] += lp.K * lp.f_in
            c["add"] += lp.K * lp.f_in
            c["smult"] += lp.f_in * lp.f_out
            c["rescale"] += 2 * lp.f_out
            n_cts = lp.f_out
        else:
            n_packed = ceil_div(lp.f_out, lp.t)
            if lp.comb == "diag":
                # the block-rotation combination: one mask product per block offset, a rotation per
                # nonzero offset (one packed input, one packed output)
                c["pmult"] += len(lp.comb_shifts)
                c["add"] += len(lp.comb_shifts)
                c["rot"] += sum(1 for d in lp.comb_shifts if d != 0)
                c["rescale"] += 1
            else:
                c["smult"] += lp.f_in * lp.f_out
                c["rescale"] += lp.f_out
                c["rot"] += lp.f_out - n_packed
            steps = rotation_steps_of(lp)
            if lp.family == 3:
                c["rot"] += n_packed * len(lp.program.rotations())
                n_ops = len(radix2.operand_list(lp.program))
                c["pmult"] += n_packed * n_ops
                c["add"] += n_packed * n_ops
                c["rescale"] += n_packed * lp.program.n_rescales()
                n_cts = n_packed
                if lp.activation:
                    c["cmult"] += n_cts
                    c["rescale"] += n_cts
                continue
            if lp.family in (1, 4):
                c["rot"] += n_packed * len(steps)
            else:
                babies = {d % lp.G for d in lp.shifts} - {0}
                giants = {d // lp.G for d in lp.shifts} - {0}
                c["rot"] += n_packed * (len(babies) + len(giants))
            c["pmult"] += n_packed * len(lp.shifts)
            c["add"] += n_packed * len(lp.shifts)
            c["rescale"] += n_packed
            n_cts = n_packed
        if lp.activation:
            c["cmult"] += n_cts
            c["rescale"] += n_cts
    c["keyswitch"] = c["rot"] + c["cmult"]
    return c
