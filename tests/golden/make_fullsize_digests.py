"""Writes fullsize_layer2_digests.json: the oracle's output words of the second
(SpIntra-CA) layer of the citation-graph and clustered-graph shapes at their full
sizes (N = 2^16), as SHA-256 digests, for tests/test_gpu_fullsize.py.

Inputs: the layer's input ciphertexts are seeded uniform residues
(workload.uniform_ct_words) at the level and scale the plan schedules; keys come
from the oracle's key generation with a fixed seed (the GPU generates the same
words from the same seed); the layer's masks and weights are the oracle's
encodings.  Only oracle/ and workload/ are used.

Rotation keys at N = 2^16 take 60 MiB each, so they are generated when a
rotation asks for one and dropped afterwards; the packed ciphertexts of a layer
are aggregated in parallel processes.  A full run takes tens of minutes on a
few cores:  python tests/golden/make_fullsize_digests.py [names...]
"""
from __future__ import annotations

import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import ckks, gcn, planner, execute as ex, encoding as enc  # noqa: E402
from oracle.params import Params  # noqa: E402
from workload import make_workload, uniform_ct_words, CONFIGS  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_layer2_digests.json")
KEY_SEED = 21
LAYER = 1
NAMES = ("cora", "citeseer", "pubmed")


def case_options(name: str) -> dict:
    """Plan options of the full-size case: one NOO region over the whole graph, the
    baby-step/giant-step family, client ciphertexts at the lowest level they need."""
    n_v = CONFIGS[name]["graph"][1]
    return dict(TH=n_v, family=2, low_level=True)


def input_seed(name: str) -> int:
    return 1000 * CONFIGS[name]["id"] + 77


def digest(words: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(words, dtype=np.uint64).tobytes()).hexdigest()


class LazyRotationKeys:
    """Galois element -> rotation key, generated on each request (nothing kept)."""

    def __init__(self, prm, seed, s, steps):
        self.prm, self.seed, self.s = prm, seed, s
        self.g2k = {ckks.galois_element(k, prm): k for k in steps}

    def __contains__(self, g):
        return g in self.g2k

    def __getitem__(self, g):
        return ckks.gen_rotation_key(self.prm, self.seed, self.s, self.g2k[g])


class LazyMasks:
    """Shift -> the mask's encoding, computed on each request."""

    def __init__(self, prm, vecs, scale, level):
        self.prm, self.vecs, self.scale, self.level = prm, vecs, scale, level

    def __getitem__(self, d):
        return enc.encode(self.prm, self.vecs[d], self.scale, self.level)


def setup(name: str):
    """Everything both the oracle run and the GPU test derive from the case."""
    w = make_workload(name)
    prm = Params.from_dict(w.params)
    rows = gcn.normalized_rows(w.graph.n, w.neighbors, w.norm)
    o = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, prm.M, **case_options(name))
    sched = ex.schedule(prm, o)
    st = sched[LAYER]
    lp = o.layers[LAYER]
    qs = prm.q_level(st["level_in"])
    words = uniform_ct_words(input_seed(name), qs, prm.N, lp.f_in)
    return w, prm, o, sched, st, lp, words


_STATE = {}
_MASK_CACHE = {}


def encode_mask_chunk(args):
    """(name, g, lo, hi) -> (g, lo, the oracle's encodings of packed ciphertext g's masks
    for shifts lo..hi-1, as residue arrays).  The case is set up once per process."""
    name, g, lo, hi = args
    if name not in _MASK_CACHE:
        _MASK_CACHE.clear()
        w, prm, o, sched, st, lp, _ = setup(name)
        _MASK_CACHE[name] = (prm, st, lp, ex.mask_vectors(o, LAYER))
    prm, st, lp, vecs = _MASK_CACHE[name]
    return g, lo, [enc.encode(prm, vecs[g][d], st["sM"], st["level_agg"]).m for d in lp.shifts[lo:hi]]


def _aggregate_one(g):
    s = _STATE
    prm, o, st = s["prm"], s["o"], s["st"]
    keys = ckks.Keys(s=s["sk"], rot=LazyRotationKeys(prm, KEY_SEED, s["sk"], s["steps"]))
    masks = LazyMasks(prm, s["mask_vecs"][g], st["sM"], st["level_agg"])
    out = ex.aggregate(prm, o, LAYER, keys, s["packed"][g], masks, st)
    if o.layers[LAYER].activation:
        keys.relin = ckks.gen_relin_key(prm, KEY_SEED, s["sk"])
        out = ckks.ct_mul_relin(prm, keys, out, out)
    return g, np.stack([out.c0, out.c1]), out.level


def run_case(name: str, procs: int) -> dict:
    t0 = time.time()
    w, prm, o, sched, st, lp, words = setup(name)
    if lp.kind != "spintra" or lp.family != 2 or lp.comb != "scalar":
        raise SystemExit("%s: the full-size case expects a baby-step/giant-step layer after a scalar combination"
                         % name)
    steps = o.rot_steps(prm.M)
    sk = ckks.gen_secret(prm, KEY_SEED)
    keys = ckks.Keys(s=sk, rot=LazyRotationKeys(prm, KEY_SEED, sk, steps))
    W = ex.weight_ints(w.weights[LAYER], st["sW"])
    cts = [ckks.Ciphertext(words[i, 0], words[i, 1], st["level_in"], st["scale_in"]) for i in range(lp.f_in)]
    packed = ex.combine_and_pack(prm, o, LAYER, keys, cts, dict(W=W), st)
    print("[%s] combined and packed %d ciphertexts in %.0f s" % (name, len(packed), time.time() - t0), flush=True)
    _STATE.update(prm=prm, o=o, st=st, sk=sk, steps=steps, packed=packed, mask_vecs=ex.mask_vectors(o, LAYER))
    with mp.get_context("fork").Pool(min(procs, len(packed))) as pool:
        res = sorted(pool.map(_aggregate_one, range(len(packed))))
        pool.close()
        pool.join()
    _STATE.clear()
    print("[%s] layer done in %.0f s" % (name, time.time() - t0), flush=True)
    return dict(options=case_options(name), key_seed=KEY_SEED, input_seed=input_seed(name), layer=LAYER,
                level_in=st["level_in"], n_in=lp.f_in, level_out=res[0][2], n_out=len(res),
                n_shifts=len(lp.shifts), G=lp.G, t=lp.t,
                node_order_sha256=digest(np.asarray(o.pi, dtype=np.int64).astype(np.uint64)),
                sha256=[digest(x) for _, x, _ in res],
                head=[[int(v) for v in x[0, 0, :4]] for _, x, _ in res],
                oracle_seconds=round(time.time() - t0, 1))


def main():
    names = sys.argv[1:] or list(NAMES)
    procs = int(os.environ.get("DIGEST_PROCS", "4"))
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        data[name] = run_case(name, procs)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main()
