"""Python binding of libficgcn.so (the C ABI of include/ficgcn.h).

Argument marshalling only: every step runs in the HIP library.  Device
buffers are torch tensors (int64 storage holding uint64 words); host arrays
are numpy arrays.  Importing this module does not load the library; the
first call does, and raises FicgcnError if libficgcn.so is missing -- there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FICGCN_LIB", os.path.join(HERE, "libficgcn.so"))

_lib = None

c_u64p = ctypes.POINTER(ctypes.c_uint64)
c_vp = ctypes.c_void_p


class FicgcnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("ficgcn status %d: %s" % (status, msg))
        self.status = status


class CkksParams(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_q", ctypes.c_uint32), ("q_bits", ctypes.c_uint32),
                ("n_p", ctypes.c_uint32), ("p_bits", ctypes.c_uint32), ("log_scale", ctypes.c_uint32)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("first_mode", ctypes.c_int32), ("use_noo", ctypes.c_int32), ("family", ctypes.c_int32),
                ("TH", ctypes.c_int32), ("activation", ctypes.c_int32), ("t", ctypes.c_int32),
                ("aoo_off", ctypes.c_int32), ("cpoo", ctypes.c_double), ("first_pack", ctypes.c_int32),
                ("agg_c", ctypes.c_double), ("low_level", ctypes.c_int32), ("max_key_bytes", ctypes.c_double)]


class Operand(ctypes.Structure):
    """ckks_operand: a device buffer with its level and scale (the library checks them)."""
    _fields_ = [("data", c_vp), ("level", ctypes.c_uint32), ("n_poly", ctypes.c_uint32), ("scale", ctypes.c_double)]


class SearchStats(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_uint32), ("n_built", ctypes.c_uint32), ("best_cost", ctypes.c_double),
                ("build_seconds", ctypes.c_double)]


N_FEATURES = 24


class Request(ctypes.Structure):
    _fields_ = [("plan", c_vp), ("eval_keys", c_vp), ("inputs_host", c_vp), ("n_in", ctypes.c_size_t),
                ("output_host", c_vp), ("n_out", ctypes.c_size_t), ("operands_host", c_vp),
                ("seeded", ctypes.c_uint32), ("a_id0", ctypes.c_uint32), ("a_seed", ctypes.c_uint64),
                ("packed_bits", ctypes.c_uint32)]


class RequestResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double), ("footprint_bytes", ctypes.c_uint64)]


class ServerSummary(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint32), ("failed", ctypes.c_uint32), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double), ("throughput_per_s", ctypes.c_double),
                ("peak_bytes", ctypes.c_uint64), ("max_concurrent", ctypes.c_uint32),
                ("resident_bytes", ctypes.c_uint64), ("arena_allocs", ctypes.c_uint64),
                ("scratch_overruns", ctypes.c_uint64)]

# name -> (restype, argtypes); every status-returning call returns c_int
_SIGS = {
    "ficgcn_last_error": (ctypes.c_char_p, []),
    "ckks_context_create": (ctypes.c_int, [ctypes.POINTER(CkksParams), ctypes.POINTER(c_vp)]),
    "ckks_ctx_destroy": (None, [c_vp]),
    "ckks_ctx_set_stream": (ctypes.c_int, [c_vp, c_vp]),
    "ckks_ctx_moduli": (ctypes.c_int, [c_vp, c_vp]),
    "ckks_galois_element": (ctypes.c_int, [c_vp, ctypes.c_int64, c_u64p]),
    "ckks_sync": (ctypes.c_int, [c_vp]),
    "ckks_ntt_autotune": (ctypes.c_int, [c_vp, ctypes.c_uint32, c_vp]),
    "ckks_ntt_config": (ctypes.c_int, [c_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "ficgcn_profile_enable": (ctypes.c_int, [c_vp, ctypes.c_int]),
    "ficgcn_profile_read": (ctypes.c_int, [c_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_uint64)]),
    "ckks_keygen": (ctypes.c_int, [c_vp, ctypes.c_uint64, c_vp, ctypes.c_size_t, ctypes.c_int,
                                   ctypes.POINTER(c_vp), ctypes.POINTER(c_vp)]),
    "ckks_keys_tags": (ctypes.c_int, [c_vp, c_vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    "ckks_keys_export": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint64, c_vp]),
    "ckks_keys_import": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint64, c_vp]),
    "ckks_keys_create_empty": (ctypes.c_int, [c_vp, ctypes.POINTER(c_vp)]),
    "ckks_keys_destroy": (None, [c_vp]),
    "ckks_encode": (ctypes.c_int, [c_vp, c_vp, c_vp, ctypes.c_size_t, ctypes.c_double, ctypes.c_uint32, c_vp]),
    "ckks_encode_batch": (ctypes.c_int, [c_vp, c_vp, ctypes.c_size_t, ctypes.c_size_t, ctypes.c_double,
                                         ctypes.c_uint32, c_vp]),
    "ckks_pt_load": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint32, c_vp]),
    "ckks_encrypt": (ctypes.c_int, [c_vp, c_vp, c_vp, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, c_vp]),
    "ckks_encrypt_seeded": (ctypes.c_int, [c_vp, c_vp, c_vp, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.c_uint32, c_vp]),
    "ckks_expand_seeded": (ctypes.c_int, [c_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_uint32,
                                          c_vp]),
    "ckks_pack_residues": (ctypes.c_int, [c_vp, c_vp, ctypes.c_size_t, ctypes.c_uint32, c_vp]),
    "ckks_unpack_residues": (ctypes.c_int, [c_vp, c_vp, ctypes.c_size_t, ctypes.c_uint32, c_vp]),
    "ckks_decrypt": (ctypes.c_int, [c_vp, c_vp, c_vp, ctypes.c_uint32, ctypes.c_double, c_vp, c_vp,
                                    ctypes.c_size_t]),
    "ckks_ct_load": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint32, c_vp]),
    "ckks_poly_store": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint32, ctypes.c_uint32, c_vp]),
    "ckks_ntt": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int]),
    "ckks_rotate_hoisted": (ctypes.c_int, [c_vp, c_vp, c_vp, ctypes.c_uint32, c_vp, ctypes.c_size_t, c_vp]),
    "ckks_rotate_batch": (ctypes.c_int, [c_vp, c_vp, c_vp, ctypes.c_uint32, c_vp, ctypes.c_size_t, c_vp]),
    "ckks_pt_mul_acc": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint32, c_vp, c_vp, ctypes.c_size_t]),
    "ckks_scalar_mul_acc": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint32, c_vp, c_vp, ctypes.c_size_t]),
    "ckks_add": (ctypes.c_int, [c_vp, c_vp, c_vp, ctypes.c_uint32]),
    "ckks_rescale": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint32]),
    "ckks_mul_relin": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, ctypes.c_uint32, c_vp]),
    "ckks_mul_relin_noalloc": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, ctypes.c_uint32, c_vp]),
    "ckks_mul_relin_noalloc_limit": (ctypes.c_size_t, []),
    "ckks_encrypt_op": (ctypes.c_int, [c_vp, c_vp, ctypes.POINTER(Operand), ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(Operand)]),
    "ckks_decrypt_op": (ctypes.c_int, [c_vp, c_vp, ctypes.POINTER(Operand), c_vp, c_vp, ctypes.c_size_t]),
    "ckks_rotate_hoisted_op": (ctypes.c_int, [c_vp, c_vp, ctypes.POINTER(Operand), c_vp, ctypes.c_size_t, ctypes.POINTER(Operand)]),
    "ckks_pt_mul_acc_op": (ctypes.c_int, [c_vp, ctypes.POINTER(Operand), ctypes.POINTER(Operand), ctypes.POINTER(Operand), ctypes.c_size_t]),
    "ckks_scalar_mul_acc_op": (ctypes.c_int, [c_vp, ctypes.POINTER(Operand), ctypes.POINTER(Operand), c_vp, ctypes.c_double, ctypes.c_size_t]),
    "ckks_add_op": (ctypes.c_int, [c_vp, ctypes.POINTER(Operand), ctypes.POINTER(Operand)]),
    "ckks_rescale_op": (ctypes.c_int, [c_vp, ctypes.POINTER(Operand)]),
    "ckks_mul_relin_op": (ctypes.c_int, [c_vp, c_vp, ctypes.POINTER(Operand), ctypes.POINTER(Operand), ctypes.POINTER(Operand)]),
    "ficgcn_plan_create": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, ctypes.c_uint32, c_vp, ctypes.c_uint32, c_vp,
                                          ctypes.POINTER(PlanOpts), ctypes.POINTER(c_vp)]),
    "ficgcn_plan_destroy": (None, [c_vp]),
    "ficgcn_plan_node_order": (ctypes.c_int, [c_vp, c_vp]),
    "ficgcn_plan_copy_sources": (ctypes.c_int, [c_vp, ctypes.c_uint32, c_vp]),
    "ficgcn_plan_rot_steps": (ctypes.c_int, [c_vp, c_vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    "ficgcn_plan_info": (ctypes.c_int, [c_vp, c_vp, c_vp, ctypes.POINTER(ctypes.c_uint32)]),
    "ficgcn_plan_shifts": (ctypes.c_int, [c_vp, ctypes.c_uint32, c_vp, ctypes.c_size_t,
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "ficgcn_plan_weights_int": (ctypes.c_int, [c_vp, ctypes.c_uint32, c_vp]),
    "ficgcn_plan_operand_count": (ctypes.c_int, [c_vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_size_t)]),
    "ficgcn_plan_operand_slots": (ctypes.c_int, [c_vp, ctypes.c_uint32, ctypes.c_size_t, c_vp]),
    "ficgcn_plan_operand_level": (ctypes.c_int, [c_vp, ctypes.c_uint32, ctypes.c_size_t,
                                                 ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_double)]),
    "ficgcn_plan_radix2_stats": (ctypes.c_int, [c_vp, ctypes.c_uint32, c_vp]),
    "ficgcn_plan_encode": (ctypes.c_int, [c_vp, c_vp]),
    "ficgcn_plan_packed_input_words": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint32, c_vp]),
    "ficgcn_plan_pack_inputs": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint32, c_vp, ctypes.c_size_t, c_vp,
                                               ctypes.c_uint64]),
    "ficgcn_plan_load_operand": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint32, ctypes.c_size_t, c_vp]),
    "ficgcn_gcn_layer": (ctypes.c_int, [c_vp, c_vp, c_vp, ctypes.c_uint32, c_vp, ctypes.c_size_t, c_vp,
                                        ctypes.c_size_t, ctypes.c_int32]),
    "ficgcn_plan_fill_operands": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint64]),
    "ficgcn_plan_candidates": (ctypes.c_int, [ctypes.c_uint32, c_vp, ctypes.c_uint32, ctypes.c_uint32,
                                              ctypes.POINTER(PlanOpts), c_vp, ctypes.c_size_t,
                                              ctypes.POINTER(ctypes.c_size_t)]),
    "ficgcn_candidate_features": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint32, c_vp, ctypes.c_uint32,
                                                 ctypes.c_uint32, ctypes.POINTER(PlanOpts), c_vp]),
    "ficgcn_plan_cost": (ctypes.c_int, [c_vp, ctypes.POINTER(ctypes.c_double)]),
    "ficgcn_plan_search": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, ctypes.c_uint32, c_vp, ctypes.c_uint32, c_vp,
                                          ctypes.POINTER(PlanOpts), c_vp, ctypes.c_uint32,
                                          ctypes.POINTER(PlanOpts), ctypes.POINTER(SearchStats)]),
    "ficgcn_server_create": (ctypes.c_int, [ctypes.POINTER(CkksParams), ctypes.c_uint32, ctypes.c_uint64,
                                            ctypes.POINTER(c_vp)]),
    "ficgcn_server_destroy": (None, [c_vp]),
    "ficgcn_server_submit": (ctypes.c_int, [c_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "ficgcn_server_wait": (ctypes.c_int, [c_vp, ctypes.c_uint64, ctypes.POINTER(RequestResult)]),
    "ficgcn_server_stats": (ctypes.c_int, [c_vp, ctypes.POINTER(ServerSummary)]),
    "ficgcn_mlp_create": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint32, c_vp, ctypes.POINTER(c_vp)]),
    "ficgcn_mlp_destroy": (None, [c_vp]),
    "ficgcn_mlp_param_count": (ctypes.c_int, [c_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "ficgcn_mlp_get_params": (ctypes.c_int, [c_vp, c_vp]),
    "ficgcn_mlp_forward": (ctypes.c_int, [c_vp, c_vp, ctypes.c_uint32, c_vp]),
    "ficgcn_mlp_gradient": (ctypes.c_int, [c_vp, c_vp, c_vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_float), c_vp]),
    "ficgcn_mlp_train_step": (ctypes.c_int, [c_vp, c_vp, c_vp, ctypes.c_uint32, ctypes.c_float,
                                             ctypes.POINTER(ctypes.c_float)]),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FicgcnError(-6, "HIP library %s is not built (run __graft_entry__.build())" % LIB_PATH)
        # PyTorch's HIP runtime is loaded first, so the library binds to the
        # same runtime as the tensors it is handed (one runtime per process)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols() -> List[str]:
    return list(_SIGS)


def _check(st: int):
    if st != 0:
        raise FicgcnError(st, lib().ficgcn_last_error().decode())


def _ptr(x) -> int:
    """Address of a torch tensor, numpy array or raw integer."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        assert x.flags["C_CONTIGUOUS"]
        return x.ctypes.data
    raise TypeError(type(x))


def _ptr_array(xs) -> ctypes.Array:
    arr = (c_vp * max(1, len(xs)))()
    for i, x in enumerate(xs):
        arr[i] = _ptr(x)
    return arr


class Context:
    """A CKKS context on the current HIP device, bound to torch's current stream."""

    def __init__(self, log_n: int, n_q: int, q_bits: int, n_p: int, p_bits: int, log_scale: int = 40,
                 stream=None):
        self.params = CkksParams(log_n, n_q, q_bits, n_p, p_bits, log_scale)
        h = c_vp()
        _check(lib().ckks_context_create(ctypes.byref(self.params), ctypes.byref(h)))
        self.h = h
        self.log_n = log_n
        self.N = 1 << log_n
        self.M = self.N // 2
        self.L, self.alpha, self.log_scale = n_q, n_p, log_scale
        self.beta = -(-n_q // n_p)
        if stream is None:
            import torch
            # host-only use (planning) needs no device; device tables upload on first device call
            stream = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else 0
        self.ckks_ctx_set_stream(stream)

    @classmethod
    def from_dict(cls, d: dict) -> "Context":
        return cls(d["log_n"], d["n_q"], d["q_bits"], d["n_p"], d["p_bits"], d.get("log_scale", 40))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ckks_ctx_destroy(self.h)
            self.h = None

    # ---- context
    def ckks_ctx_set_stream(self, stream):
        _check(lib().ckks_ctx_set_stream(self.h, stream))

    def ckks_ctx_moduli(self) -> List[int]:
        out = np.zeros(self.L + self.alpha, dtype=np.uint64)
        _check(lib().ckks_ctx_moduli(self.h, _ptr(out)))
        return [int(x) for x in out]

    def ckks_galois_element(self, step: int) -> int:
        g = ctypes.c_uint64()
        _check(lib().ckks_galois_element(self.h, step, ctypes.byref(g)))
        return g.value

    def ckks_sync(self):
        _check(lib().ckks_sync(self.h))

    def ckks_ntt_autotune(self, n_limbs: int):
        """(column width, row width, column-pass log size) chosen for this context."""
        out = np.zeros(3, dtype=np.int32)
        _check(lib().ckks_ntt_autotune(self.h, n_limbs, _ptr(out)))
        return int(out[0]), int(out[1]), int(out[2])

    def ckks_ntt_config(self, split: int, cols_column: int, cols_row: int):
        _check(lib().ckks_ntt_config(self.h, split, cols_column, cols_row))

    def ficgcn_profile_enable(self, on: bool):
        _check(lib().ficgcn_profile_enable(self.h, int(on)))

    def ficgcn_profile_read(self, kernel: str):
        ms, n = ctypes.c_double(), ctypes.c_uint64()
        _check(lib().ficgcn_profile_read(self.h, kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    # ---- buffers
    def ct_buffer(self, level: int, count: Optional[int] = None):
        import torch
        shape = (2, level + 1, self.N) if count is None else (count, 2, level + 1, self.N)
        return torch.empty(shape, dtype=torch.int64, device="cuda")

    def pt_buffer(self, level: int, count: Optional[int] = None):
        import torch
        shape = (level + 1, self.N) if count is None else (count, level + 1, self.N)
        return torch.empty(shape, dtype=torch.int64, device="cuda")

    # ---- keys
    def ckks_keygen(self, seed: int, rot_steps: Sequence[int] = (), with_relin: bool = True):
        steps = np.ascontiguousarray(np.array(list(rot_steps), dtype=np.int64))
        cl, ev = c_vp(), c_vp()
        _check(lib().ckks_keygen(self.h, seed, _ptr(steps) if len(steps) else None, len(steps), int(with_relin),
                                 ctypes.byref(cl), ctypes.byref(ev)))
        return Keys(self, cl), Keys(self, ev)

    def ckks_keys_create_empty(self):
        k = c_vp()
        _check(lib().ckks_keys_create_empty(self.h, ctypes.byref(k)))
        return Keys(self, k)

    # ---- encode / encrypt / decrypt
    def ckks_encode(self, z, scale: float, level: int, out=None):
        out = self.pt_buffer(level) if out is None else out
        z = np.asarray(z)
        re = np.ascontiguousarray(np.real(z), dtype=np.float64)
        im = np.ascontiguousarray(np.imag(z), dtype=np.float64) if np.iscomplexobj(z) else None
        _check(lib().ckks_encode(self.h, _ptr(re), _ptr(im), len(re), scale, level, _ptr(out)))
        return out

    def ckks_encode_batch(self, rows: np.ndarray, scale: float, level: int, out=None):
        rows = np.ascontiguousarray(rows, dtype=np.float64)
        out = self.pt_buffer(level, rows.shape[0]) if out is None else out
        _check(lib().ckks_encode_batch(self.h, _ptr(rows), rows.shape[0], rows.shape[1], scale, level, _ptr(out)))
        return out

    def ckks_pt_load(self, coeffs: np.ndarray, level: int, out=None):
        out = self.pt_buffer(level) if out is None else out
        coeffs = np.ascontiguousarray(coeffs, dtype=np.uint64)
        _check(lib().ckks_pt_load(self.h, _ptr(coeffs), level, _ptr(out)))
        return out

    def ckks_encrypt(self, client_keys: "Keys", pt, level: int, seed: int, ct_id: int, out=None):
        out = self.ct_buffer(level) if out is None else out
        _check(lib().ckks_encrypt(self.h, client_keys.h, _ptr(pt), level, seed, ct_id, _ptr(out)))
        return out

    def ckks_encrypt_seeded(self, client_keys: "Keys", pt, level: int, e_seed: int, a_seed: int, ct_id: int,
                            out=None):
        out = self.ct_buffer(level) if out is None else out
        _check(lib().ckks_encrypt_seeded(self.h, client_keys.h, _ptr(pt), level, e_seed, a_seed, ct_id, _ptr(out)))
        return out

    def ckks_expand_seeded(self, a_seed: int, ct_id0: int, count: int, level: int, cts):
        """cts: device buffer [count][2][level+1][N]; rewrites every second polynomial."""
        _check(lib().ckks_expand_seeded(self.h, a_seed, ct_id0, count, level, _ptr(cts)))
        return cts

    def ckks_pack_residues(self, src, n_limbs: int, bits: int, out=None):
        """src: device words, n_limbs limbs of N residues -> n_limbs * N * bits / 64 packed words."""
        import torch
        if out is None:
            out = torch.empty(n_limbs * self.N * bits // 64, dtype=torch.int64, device="cuda")
        _check(lib().ckks_pack_residues(self.h, _ptr(src), n_limbs, bits, _ptr(out)))
        return out

    def ckks_unpack_residues(self, src, n_limbs: int, bits: int, out=None):
        import torch
        if out is None:
            out = torch.empty(n_limbs * self.N, dtype=torch.int64, device="cuda")
        _check(lib().ckks_unpack_residues(self.h, _ptr(src), n_limbs, bits, _ptr(out)))
        return out

    def ckks_decrypt(self, client_keys: "Keys", ct, level: int, scale: float, n_slots: int) -> np.ndarray:
        re = np.zeros(n_slots, dtype=np.float64)
        im = np.zeros(n_slots, dtype=np.float64)
        _check(lib().ckks_decrypt(self.h, client_keys.h, _ptr(ct), level, scale, _ptr(re), _ptr(im), n_slots))
        return re + 1j * im

    # ---- transfers
    def ckks_ct_load(self, coeffs: np.ndarray, level: int, out=None):
        out = self.ct_buffer(level) if out is None else out
        coeffs = np.ascontiguousarray(coeffs, dtype=np.uint64)
        _check(lib().ckks_ct_load(self.h, _ptr(coeffs), level, _ptr(out)))
        return out

    def ckks_poly_store(self, dev, level: int, n_polys: int) -> np.ndarray:
        out = np.zeros((n_polys, level + 1, self.N), dtype=np.uint64)
        _check(lib().ckks_poly_store(self.h, _ptr(dev), level, n_polys, _ptr(out)))
        return out

    def ckks_ntt(self, dev, n_limbs: int, first_mod: int, inverse: bool):
        _check(lib().ckks_ntt(self.h, _ptr(dev), n_limbs, first_mod, int(inverse)))

    # ---- evaluation
    def ckks_rotate_hoisted(self, eval_keys: "Keys", ct, level: int, steps: Sequence[int], outs=None):
        steps = np.ascontiguousarray(np.array(list(steps), dtype=np.int64))
        outs = [self.ct_buffer(level) for _ in steps] if outs is None else outs
        _check(lib().ckks_rotate_hoisted(self.h, eval_keys.h, _ptr(ct), level, _ptr(steps), len(steps),
                                         _ptr_array(outs)))
        return outs

    def ckks_rotate_batch(self, eval_keys: "Keys", cts, level: int, steps: Sequence[int], outs=None):
        steps = np.ascontiguousarray(np.array(list(steps), dtype=np.int64))
        if len(cts) != len(steps):
            raise ValueError("one step per ciphertext")
        outs = [self.ct_buffer(level) for _ in steps] if outs is None else outs
        _check(lib().ckks_rotate_batch(self.h, eval_keys.h, _ptr_array(cts), level, _ptr(steps), len(steps),
                                       _ptr_array(outs)))
        return outs

    def ckks_pt_mul_acc(self, acc, level: int, cts, pts):
        _check(lib().ckks_pt_mul_acc(self.h, _ptr(acc), level, _ptr_array(cts), _ptr_array(pts), len(cts)))

    def ckks_scalar_mul_acc(self, acc, level: int, cts, consts):
        c = np.ascontiguousarray(np.array(list(consts), dtype=np.int64))
        _check(lib().ckks_scalar_mul_acc(self.h, _ptr(acc), level, _ptr_array(cts), _ptr(c), len(cts)))

    def ckks_add(self, acc, x, level: int):
        _check(lib().ckks_add(self.h, _ptr(acc), _ptr(x), level))

    def ckks_rescale(self, ct, level: int):
        _check(lib().ckks_rescale(self.h, _ptr(ct), level))

    def ckks_mul_relin(self, eval_keys: "Keys", x, y, level: int, out=None):
        out = self.ct_buffer(level) if out is None else out
        _check(lib().ckks_mul_relin(self.h, eval_keys.h, _ptr(x), _ptr(y), level, _ptr(out)))
        return out

    def ckks_mul_relin_noalloc(self, eval_keys: "Keys", x, y, level: int, out):
        _check(lib().ckks_mul_relin_noalloc(self.h, eval_keys.h, _ptr(x), _ptr(y), level, _ptr(out)))
        return out

    # ---- the same operations on level/scale descriptors (Operand); the library
    # checks levels and scales and updates the outputs' descriptors
    @staticmethod
    def operand(buf, level: int, scale: float, n_poly: int = 2) -> Operand:
        return Operand(_ptr(buf), level, n_poly, scale)

    @staticmethod
    def _ops(xs) -> ctypes.Array:
        arr = (Operand * max(1, len(xs)))()
        for i, x in enumerate(xs):
            arr[i] = x
        return arr

    def ckks_encrypt_op(self, client_keys: "Keys", pt: Operand, seed: int, ct_id: int, ct: Operand):
        _check(lib().ckks_encrypt_op(self.h, client_keys.h, ctypes.byref(pt), seed, ct_id, ctypes.byref(ct)))

    def ckks_decrypt_op(self, client_keys: "Keys", ct: Operand, n_slots: int) -> np.ndarray:
        re = np.zeros(n_slots)
        im = np.zeros(n_slots)
        _check(lib().ckks_decrypt_op(self.h, client_keys.h, ctypes.byref(ct), _ptr(re), _ptr(im), n_slots))
        return re + 1j * im

    def ckks_rotate_hoisted_op(self, eval_keys: "Keys", ct: Operand, steps: Sequence[int], outs: List[Operand]):
        steps = np.ascontiguousarray(np.array(list(steps), dtype=np.int64))
        arr = self._ops(outs)
        _check(lib().ckks_rotate_hoisted_op(self.h, eval_keys.h, ctypes.byref(ct), _ptr(steps), len(steps), arr))
        for i in range(len(outs)):
            outs[i].level, outs[i].scale = arr[i].level, arr[i].scale

    def ckks_pt_mul_acc_op(self, acc: Operand, cts: List[Operand], pts: List[Operand]):
        _check(lib().ckks_pt_mul_acc_op(self.h, ctypes.byref(acc), self._ops(cts), self._ops(pts), len(cts)))

    def ckks_scalar_mul_acc_op(self, acc: Operand, cts: List[Operand], consts, const_scale: float):
        c = np.ascontiguousarray(np.array(list(consts), dtype=np.int64))
        _check(lib().ckks_scalar_mul_acc_op(self.h, ctypes.byref(acc), self._ops(cts), _ptr(c), const_scale, len(cts)))

    def ckks_add_op(self, acc: Operand, x: Operand):
        _check(lib().ckks_add_op(self.h, ctypes.byref(acc), ctypes.byref(x)))

    def ckks_rescale_op(self, ct: Operand):
        _check(lib().ckks_rescale_op(self.h, ctypes.byref(ct)))

    def ckks_mul_relin_op(self, eval_keys: "Keys", x: Operand, y: Operand, out: Operand):
        _check(lib().ckks_mul_relin_op(self.h, eval_keys.h, ctypes.byref(x), ctypes.byref(y), ctypes.byref(out)))


class Keys:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ckks_keys_destroy(self.h)
            self.h = None

    def ckks_keys_tags(self) -> List[int]:
        n = ctypes.c_size_t()
        _check(lib().ckks_keys_tags(self.h, None, 0, ctypes.byref(n)))
        out = np.zeros(max(1, n.value), dtype=np.uint64)
        _check(lib().ckks_keys_tags(self.h, _ptr(out), n.value, ctypes.byref(n)))
        return [int(x) for x in out[: n.value]]

    def ckks_keys_export(self, tag: int) -> np.ndarray:
        c = self.ctx
        out = np.zeros((c.beta, 2, c.L + c.alpha, c.N), dtype=np.uint64)
        _check(lib().ckks_keys_export(c.h, self.h, tag, _ptr(out)))
        return out

    def ckks_keys_import(self, tag: int, coeffs: np.ndarray):
        coeffs = np.ascontiguousarray(coeffs, dtype=np.uint64)
        _check(lib().ckks_keys_import(self.ctx.h, self.h, tag, _ptr(coeffs)))


class Plan:
    """ficgcn_plan: node order, per-layer routing and schedule, operands."""

    def __init__(self, ctx: Context, rowptr, col, val, n_v: int, dims: Sequence[int], weights,
                 first_mode: int = 0, use_noo: bool = True, family: int = 0, TH: int = 0, activation: bool = False,
                 t: int = 0, cpoo: float = 0.0, aoo: bool = True, first_pack: int = 0, agg_c: float = 0.0,
                 low_level: bool = False, opts: "PlanOpts" = None):
        self.ctx = ctx
        self._rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        self._col = np.ascontiguousarray(col, dtype=np.int32)
        self._val = np.ascontiguousarray(val, dtype=np.float64)
        self._dims = np.ascontiguousarray(dims, dtype=np.uint32)
        self._w = [np.ascontiguousarray(w, dtype=np.float64) for w in weights]
        wp = _ptr_array(self._w)
        if opts is None:
            opts = PlanOpts(first_mode=first_mode, use_noo=int(use_noo), family=family, TH=TH,
                            activation=int(activation), t=t, aoo_off=int(not aoo), cpoo=cpoo,
                            first_pack=first_pack, agg_c=agg_c, low_level=int(low_level))
        self.opts = opts
        h = c_vp()
        _check(lib().ficgcn_plan_create(ctx.h, _ptr(self._rowptr), _ptr(self._col), _ptr(self._val), n_v,
                                        _ptr(self._dims), len(self._w), wp, ctypes.byref(opts), ctypes.byref(h)))
        self.h = h
        self.n_v = n_v

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ficgcn_plan_destroy(self.h)
            self.h = None

    def ficgcn_plan_node_order(self) -> np.ndarray:
        out = np.zeros(self.n_v, dtype=np.int32)
        _check(lib().ficgcn_plan_node_order(self.h, _ptr(out)))
        return out

    def ficgcn_plan_copy_sources(self, layer: int) -> np.ndarray:
        K = self.ficgcn_plan_info()[layer]["K"]
        out = np.zeros((K, self.n_v), dtype=np.int32)
        _check(lib().ficgcn_plan_copy_sources(self.h, layer, _ptr(out)))
        return out

    def ficgcn_plan_rot_steps(self) -> List[int]:
        n = ctypes.c_size_t()
        _check(lib().ficgcn_plan_rot_steps(self.h, None, 0, ctypes.byref(n)))
        out = np.zeros(max(1, n.value), dtype=np.int64)
        _check(lib().ficgcn_plan_rot_steps(self.h, _ptr(out), n.value, ctypes.byref(n)))
        return [int(x) for x in out[: n.value]]

    def ficgcn_plan_fill_operands(self, seed: int):
        _check(lib().ficgcn_plan_fill_operands(self.ctx.h, self.h, seed))

    def ficgcn_plan_cost(self) -> float:
        c = ctypes.c_double()
        _check(lib().ficgcn_plan_cost(self.h, ctypes.byref(c)))
        return c.value

    def ficgcn_plan_info(self) -> List[dict]:
        n = ctypes.c_uint32()
        _check(lib().ficgcn_plan_info(self.h, None, None, ctypes.byref(n)))
        info = np.zeros(18 * n.value, dtype=np.int64)
        sc = np.zeros(5 * n.value, dtype=np.float64)
        _check(lib().ficgcn_plan_info(self.h, _ptr(info), _ptr(sc), ctypes.byref(n)))
        keys = ["kind", "f_in", "f_out", "K", "t", "B", "family", "G", "n_shifts", "level_in", "level_out",
                "n_in_cts", "n_out_cts", "pack", "comb", "n_fold", "n_comb_shifts", "paper_mode"]
        out = []
        for li in range(n.value):
            d = {k: int(info[18 * li + i]) for i, k in enumerate(keys)}
            d.update(scale_in=float(sc[5 * li]), scale_out=float(sc[5 * li + 1]), sW=float(sc[5 * li + 2]),
                     mode_cost_inter=float(sc[5 * li + 3]), mode_cost_spintra=float(sc[5 * li + 4]))
            out.append(d)
        return out

    def ficgcn_plan_shifts(self, layer: int) -> List[int]:
        n = ctypes.c_size_t()
        _check(lib().ficgcn_plan_shifts(self.h, layer, None, 0, ctypes.byref(n)))
        out = np.zeros(max(1, n.value), dtype=np.int64)
        _check(lib().ficgcn_plan_shifts(self.h, layer, _ptr(out), n.value, ctypes.byref(n)))
        return [int(x) for x in out[: n.value]]

    def ficgcn_plan_weights_int(self, layer: int) -> np.ndarray:
        info = self.ficgcn_plan_info()[layer]
        out = np.zeros((info["f_in"], info["f_out"]), dtype=np.int64)
        _check(lib().ficgcn_plan_weights_int(self.h, layer, _ptr(out)))
        return out

    def ficgcn_plan_operand_count(self, layer: int) -> int:
        n = ctypes.c_size_t()
        _check(lib().ficgcn_plan_operand_count(self.h, layer, ctypes.byref(n)))
        return n.value

    def ficgcn_plan_operand_slots(self, layer: int, i: int) -> np.ndarray:
        out = np.zeros(self.ctx.M, dtype=np.float64)
        _check(lib().ficgcn_plan_operand_slots(self.h, layer, i, _ptr(out)))
        return out

    def ficgcn_plan_operand_level(self, layer: int, i: int):
        lv = ctypes.c_uint32()
        sc = ctypes.c_double()
        _check(lib().ficgcn_plan_operand_level(self.h, layer, i, ctypes.byref(lv), ctypes.byref(sc)))
        return lv.value, sc.value

    def ficgcn_plan_radix2_stats(self, layer: int) -> dict:
        out = np.zeros(8, dtype=np.int64)
        _check(lib().ficgcn_plan_radix2_stats(self.h, layer, _ptr(out)))
        keys = ["lanes", "steps", "rotations", "amounts", "depth", "masks", "moved", "registers"]
        return {k: int(v) for k, v in zip(keys, out)}

    def ficgcn_plan_encode(self):
        _check(lib().ficgcn_plan_encode(self.ctx.h, self.h))

    def ficgcn_plan_load_operand(self, layer: int, i: int, coeffs: np.ndarray):
        coeffs = np.ascontiguousarray(coeffs, dtype=np.uint64)
        _check(lib().ficgcn_plan_load_operand(self.ctx.h, self.h, layer, i, _ptr(coeffs)))

    def ficgcn_gcn_layer(self, eval_keys: Keys, layer: int, in_cts, out_cts, mode: int = 1):
        """in_cts None: the layer reads the inputs ficgcn_plan_pack_inputs rearranged."""
        ins = None if in_cts is None else _ptr_array(in_cts)
        _check(lib().ficgcn_gcn_layer(self.ctx.h, eval_keys.h, self.h, layer, ins, 0 if in_cts is None else len(in_cts),
                                      _ptr_array(out_cts), len(out_cts), mode))

    def ficgcn_plan_packed_input_words(self, layer: int) -> int:
        n = ctypes.c_uint64()
        _check(lib().ficgcn_plan_packed_input_words(self.h, self.ctx.h, layer, ctypes.byref(n)))
        return int(n.value)

    def ficgcn_plan_pack_inputs(self, layer: int, in_cts, out=None):
        """Rearranges the layer's input ciphertexts into a device buffer (a new
        int64 tensor unless `out` is given) and registers it with the plan."""
        import torch
        words = self.ficgcn_plan_packed_input_words(layer)
        if out is None:
            out = torch.empty(words, dtype=torch.int64, device="cuda")
        _check(lib().ficgcn_plan_pack_inputs(self.ctx.h, self.h, layer, _ptr_array(in_cts), len(in_cts), _ptr(out),
                                             out.numel()))
        self._packed = out   # the plan reads it until replaced
        return out


# ------------------------------------------------------------------ plan search
def ficgcn_plan_candidates(n_v: int, dims: Sequence[int], log_n: int, base: PlanOpts) -> List[PlanOpts]:
    d = np.ascontiguousarray(dims, dtype=np.uint32)
    n = ctypes.c_size_t()
    _check(lib().ficgcn_plan_candidates(n_v, _ptr(d), len(d) - 1, log_n, ctypes.byref(base), None, 0,
                                        ctypes.byref(n)))
    arr = (PlanOpts * n.value)()
    _check(lib().ficgcn_plan_candidates(n_v, _ptr(d), len(d) - 1, log_n, ctypes.byref(base), arr, n.value,
                                        ctypes.byref(n)))
    return list(arr)


def ficgcn_candidate_features(rowptr, col, n_v: int, dims: Sequence[int], log_n: int, opts: PlanOpts) -> np.ndarray:
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    d = np.ascontiguousarray(dims, dtype=np.uint32)
    out = np.zeros(N_FEATURES, dtype=np.float32)
    _check(lib().ficgcn_candidate_features(_ptr(rp), _ptr(cl), n_v, _ptr(d), len(d) - 1, log_n,
                                           ctypes.byref(opts), _ptr(out)))
    return out


def ficgcn_plan_search(ctx: Context, rowptr, col, val, n_v: int, dims: Sequence[int], weights, base: PlanOpts,
                       model: "Mlp" = None, keep: int = 0):
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    vl = np.ascontiguousarray(val, dtype=np.float64)
    d = np.ascontiguousarray(dims, dtype=np.uint32)
    ws = [np.ascontiguousarray(w, dtype=np.float64) for w in weights]
    best = PlanOpts()
    stats = SearchStats()
    _check(lib().ficgcn_plan_search(ctx.h, _ptr(rp), _ptr(cl), _ptr(vl), n_v, _ptr(d), len(ws), _ptr_array(ws),
                                    ctypes.byref(base), model.h if model is not None else None, keep,
                                    ctypes.byref(best), ctypes.byref(stats)))
    return best, stats


class Mlp:
    """ficgcn_mlp: the learned cost model (fp32 network, trained on the GPU)."""

    def __init__(self, ctx: Context, widths: Sequence[int], params: np.ndarray):
        self.ctx = ctx
        w = np.ascontiguousarray(widths, dtype=np.uint32)
        p = np.ascontiguousarray(params, dtype=np.float32)
        h = c_vp()
        _check(lib().ficgcn_mlp_create(ctx.h, _ptr(w), len(w), _ptr(p), ctypes.byref(h)))
        self.h = h
        n = ctypes.c_size_t()
        _check(lib().ficgcn_mlp_param_count(self.h, ctypes.byref(n)))
        self.n_params = n.value
        self.widths = list(widths)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ficgcn_mlp_destroy(self.h)
            self.h = None

    def ficgcn_mlp_get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().ficgcn_mlp_get_params(self.h, _ptr(out)))
        return out

    def ficgcn_mlp_forward(self, x, y=None):
        y = self._buf(x.shape[0], self.widths[-1]) if y is None else y
        _check(lib().ficgcn_mlp_forward(self.h, _ptr(x), x.shape[0], _ptr(y)))
        return y

    def ficgcn_mlp_gradient(self, x, y):
        loss = ctypes.c_float()
        g = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().ficgcn_mlp_gradient(self.h, _ptr(x), _ptr(y), x.shape[0], ctypes.byref(loss), _ptr(g)))
        return float(loss.value), g

    def ficgcn_mlp_train_step(self, x, y, lr: float) -> float:
        loss = ctypes.c_float()
        _check(lib().ficgcn_mlp_train_step(self.h, _ptr(x), _ptr(y), x.shape[0], lr, ctypes.byref(loss)))
        return float(loss.value)

    @staticmethod
    def _buf(rows, cols):
        import torch
        return torch.empty((rows, cols), dtype=torch.float32, device="cuda")


class Server:
    """ficgcn_server: continuous batching of encrypted inferences on one GPU."""

    def __init__(self, params: dict, n_slots: int, hbm_budget_bytes: int):
        p = CkksParams(params["log_n"], params["n_q"], params["q_bits"], params["n_p"], params["p_bits"],
                       params.get("log_scale", 40))
        h = c_vp()
        _check(lib().ficgcn_server_create(ctypes.byref(p), n_slots, hbm_budget_bytes, ctypes.byref(h)))
        self.h = h
        self._held = {}

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ficgcn_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def ficgcn_server_submit(self, plan: "Plan", eval_keys: "Keys", inputs_host, n_in: int, output_host,
                             n_out: int, operands_host=None, a_seed=None, a_id0: int = 0,
                             packed_bits: int = 0) -> int:
        """operands_host: None (the slot encodes the plan's operands) or, per layer, a uint64 array
        of every operand's coefficient-form residues in operand order, concatenated.
        a_seed: None (inputs_host holds whole ciphertexts) or the public seed of seeded inputs
        (inputs_host holds their first polynomials; input i has id a_id0 + i); packed_bits: those
        first polynomials packed at that many bits per residue (ckks_pack_residues)."""
        ops = None
        if operands_host is not None:
            operands_host = [np.ascontiguousarray(a, dtype=np.uint64) for a in operands_host]
            ops = _ptr_array(operands_host)
        r = Request(plan.h, eval_keys.h, _ptr(inputs_host), n_in, _ptr(output_host), n_out,
                    ctypes.cast(ops, c_vp) if ops is not None else None,
                    0 if a_seed is None else 1, a_id0, 0 if a_seed is None else a_seed, packed_bits)
        rid = ctypes.c_uint64()
        _check(lib().ficgcn_server_submit(self.h, ctypes.byref(r), ctypes.byref(rid)))
        # alive until waited for
        self._held[rid.value] = (plan, eval_keys, inputs_host, output_host, operands_host, ops)
        return rid.value

    def ficgcn_server_wait(self, rid: int) -> dict:
        res = RequestResult()
        st = lib().ficgcn_server_wait(self.h, rid, ctypes.byref(res))
        self._held.pop(rid, None)
        out = {f: getattr(res, f) for f, _ in RequestResult._fields_}
        if st != 0:
            raise FicgcnError(st, lib().ficgcn_last_error().decode())
        return out

    def ficgcn_server_stats(self) -> dict:
        s = ServerSummary()
        _check(lib().ficgcn_server_stats(self.h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerSummary._fields_}
