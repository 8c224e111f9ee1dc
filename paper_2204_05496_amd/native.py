"""ctypes binding of liblrhe.so (include/lrhe.h): argument marshalling only.

Every step of the encrypted path runs in the library's HIP kernels; torch is
used for device buffers (ciphertexts, inputs, workspaces) and the current HIP
stream.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LRHE_LIB names another build of the same library (the sanitizer build of the
# CPU tests); there is no other implementation to fall back to
LIBPATH = os.environ.get("LRHE_LIB") or os.path.join(HERE, "liblrhe.so")

LRHE_OK, LRHE_EINVAL, LRHE_EPARAM, LRHE_ENOMEM, LRHE_EAGAIN, LRHE_EDEVICE, LRHE_ENOISE = 0, -1, -2, -3, -4, -5, -6
WIRE_CT, WIRE_GK, WIRE_PK, WIRE_SK = 1, 2, 3, 4
WS_ENCRYPT_ROWS, WS_ENCRYPT_COLS, WS_MATMUL_FAST, WS_MATMUL_STANDARD = 1, 2, 3, 4
CT_HOST = 1   # decryption flag: the ciphertexts are in host memory
# variants of the key-switch inner-product kernel behind the "mac_mode" tuning key;
# MAC_MODE_HALF (digit halves on two workgroups per item) is a small-tile choice only
MAC_MODES = 8
MAC_MODE_HALF = 4
MAC_MODE_XCD = 5   # target moduli spread by XCD (L = 7, even tiles)
MAC_MODE_SPLIT = 6   # special-prime items, then data-modulus items ending with part 3
MAC_MODE_SPLIT64 = 7   # as MAC_MODE_SPLIT, data-modulus items double-buffered with 64-bit inner products

vp = ctypes.c_void_p
u32, u64, i32, i64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_int64
sz = ctypes.c_size_t


class LrheParams(ctypes.Structure):
    _fields_ = [("n", u32), ("L", u32), ("q", ctypes.POINTER(u32)), ("P", u32), ("t", u32), ("allow_insecure", u32)]


class LrheRequest(ctypes.Structure):
    _fields_ = [("xct", ctypes.c_void_p), ("rows", u32), ("model", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("gk", ctypes.c_void_p)]


class LrheError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lrhe error {code}: {msg}")
        self.code = code


# name -> (restype, argtypes); mirrors include/lrhe.h
SIGNATURES = {
    "lrhe_last_error": (ctypes.c_char_p, []),
    "lrhe_ctx_create": (i32, [ctypes.POINTER(LrheParams), i32, ctypes.POINTER(vp)]),
    "lrhe_ctx_destroy": (None, [vp]),
    "lrhe_ctx_info": (i32, [vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u64)]),
    "lrhe_galois_element": (i32, [vp, u32, ctypes.POINTER(u32)]),
    "lrhe_keygen": (i32, [vp, u64, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp)]),
    "lrhe_sk_destroy": (None, [vp]),
    "lrhe_pk_destroy": (None, [vp]),
    "lrhe_gk_destroy": (None, [vp]),
    "lrhe_workspace_bytes": (i32, [vp, i32, u32, u32, u32, ctypes.POINTER(u64)]),
    "lrhe_encrypt_rows": (i32, [vp, vp, vp, u32, u32, u64, u64, vp, vp, sz, vp]),
    "lrhe_encrypt_cols": (i32, [vp, vp, vp, u32, u32, u64, u64, vp, vp, sz, vp]),
    "lrhe_model_create": (i32, [vp, vp, vp, u32, u32, vp, ctypes.POINTER(vp)]),
    "lrhe_model_destroy": (None, [vp]),
    "lrhe_matmul_fast": (i32, [vp, vp, vp, vp, u32, vp, vp, sz, vp]),
    "lrhe_fixed_point": (i32, [vp, u64, i32, vp]),
    "lrhe_crt_combine": (i32, [vp, vp, u64, u64, u64, vp]),
    "lrhe_matmul_fast_noalloc": (i32, [vp, vp, vp, vp, u32, vp, vp]),
    "lrhe_matmul_fast_pairs": (i32, [vp, vp, vp, vp, u32, u32, u32, i32, vp, vp, sz, vp]),
    "lrhe_matmul_standard": (i32, [vp, vp, vp, vp, vp, sz, vp]),
    "lrhe_decrypt_slots": (i32, [vp, vp, vp, u32, vp, vp, vp]),
    "lrhe_decrypt_slots_host": (i32, [vp, vp, vp, u32, vp, vp]),
    "lrhe_decrypt_scores": (i32, [vp, vp, vp, u32, u32, u32, vp, ctypes.POINTER(ctypes.c_double), vp]),
    "lrhe_decrypt_scores_standard": (i32, [vp, vp, vp, u32, u32, u32, vp, ctypes.POINTER(ctypes.c_double), vp]),
    "lrhe_decrypt_check": (i32, [vp, vp, vp, u32, vp, u32, vp, ctypes.POINTER(u64), vp]),
    "lrhe_fault_inject": (i64, [i64]),
    "lrhe_wire_bytes": (i32, [vp, i32, u64, ctypes.POINTER(u64)]),
    "lrhe_ct_serialize": (i32, [vp, vp, u32, u32, vp, u64, vp]),
    "lrhe_ct_deserialize": (i32, [vp, vp, u64, u32, vp, u32, ctypes.POINTER(u32), vp]),
    "lrhe_key_serialize": (i32, [vp, i32, vp, vp, u64]),
    "lrhe_gk_deserialize": (i32, [vp, vp, u64, ctypes.POINTER(vp)]),
    "lrhe_pk_deserialize": (i32, [vp, vp, u64, ctypes.POINTER(vp)]),
    "lrhe_sk_deserialize": (i32, [vp, vp, u64, ctypes.POINTER(vp)]),
    "lrhe_host_transform": (i32, [vp, u32, vp, i32]),
    "lrhe_to_coeff": (i32, [vp, vp, u64, vp, vp]),
    "lrhe_pk_export": (i32, [vp, vp, vp]),
    "lrhe_gk_export": (i32, [vp, vp, vp]),
    "lrhe_sk_export": (i32, [vp, vp, vp]),
    "lrhe_ntt": (i32, [vp, vp, u64, i32, vp]),
    "lrhe_batch_create": (i32, [vp, vp, u32, ctypes.POINTER(vp)]),
    "lrhe_batch_info": (i32, [vp, ctypes.POINTER(u64), ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32)]),
    "lrhe_batch_run": (i32, [vp, vp, vp, vp, sz, vp]),
    "lrhe_batch_capture": (i32, [vp, vp, vp, vp, sz, vp]),
    "lrhe_batch_destroy": (None, [vp]),
    "lrhe_server_create": (i32, [vp, vp, sz, ctypes.POINTER(vp)]),
    "lrhe_server_submit": (i32, [vp, vp, vp, u32, vp, vp, ctypes.POINTER(u64)]),
    "lrhe_server_submit_keys": (i32, [vp, vp, vp, vp, u32, vp, vp, ctypes.POINTER(u64)]),
    "lrhe_server_release": (i32, [vp, u64]),
    "lrhe_server_poll": (i32, [vp, u64, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]),
    "lrhe_server_drain": (i32, [vp]),
    "lrhe_server_stats": (i32, [vp, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u32), ctypes.POINTER(u32),
                                ctypes.POINTER(u32)]),
    "lrhe_server_destroy": (None, [vp]),
    "lrhe_tune_set": (i32, [vp, ctypes.c_char_p, i32]),
    "lrhe_tune_get": (i32, [vp, ctypes.c_char_p, ctypes.POINTER(i32)]),
    "lrhe_autotune_fast": (i32, [vp, vp, vp, vp, u32, vp, vp, sz, vp, i32]),
    "lrhe_tune_save": (i32, [vp, ctypes.c_char_p, ctypes.c_char_p]),
    "lrhe_tune_load": (i32, [vp, ctypes.c_char_p, ctypes.c_char_p]),
    "lrhe_prof_enable": (None, [i32]),
    "lrhe_prof_reset": (None, []),
    "lrhe_prof_get": (i32, [ctypes.c_char_p, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_double)]),
    "lrhe_prof_valu_rate": (i32, [i32, i32, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


def lib():
    """Load liblrhe.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} not built: run paper_2204_05496_amd/build.py (or __graft_entry__.build())")
        L = ctypes.CDLL(LIBPATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code: int):
    if code != LRHE_OK:
        raise LrheError(code, lib().lrhe_last_error().decode())


def ptr(x) -> int:
    """Address of a torch tensor or numpy array (no copies)."""
    if isinstance(x, np.ndarray):
        assert x.flags["C_CONTIGUOUS"]
        return x.ctypes.data
    assert x.is_contiguous()
    return x.data_ptr()
