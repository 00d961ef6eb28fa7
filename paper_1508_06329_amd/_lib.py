"""ctypes view of the C ABI declared in include/lexbfs.h.

Argument marshalling only: every step of the computation runs in the HIP
kernels of liblexbfs.so. Loading fails loudly when the library is missing;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "liblexbfs.so")
SOURCES = [os.path.join(PKG, "csrc", "lexbfs.hip")]
HEADERS = [os.path.join(ROOT, "include", "lexbfs.h"), os.path.join(PKG, "csrc", "lexbfs_device.h")]

LEXBFS_OK = 0
LEXBFS_EINVAL = -1
LEXBFS_ENOWS = -2
LEXBFS_EHIP = -3
LEXBFS_EGRAPH = -4
LEXBFS_ETOOBIG = -5
LEXBFS_MAX_N = 65536
LEXBFS_FLAG_FORCE_FALLBACK = 0x1
LEXBFS_FLAG_PER_STEP = 0x2
LEXBFS_FLAG_MCS = 0x4
LEXBFS_FLAG_VALIDATE = 0x8
LEXBFS_KERNEL_KINDS = 4
KERNEL_KIND_NAMES = ("lexbfs", "sweep", "certificate", "setup")

EXPORTED = ["lexbfs_workspace_bytes", "lexbfs_validate", "lexbfs_order", "chordal_test", "lexbfs_batch_workspace_bytes",
            "chordal_test_batch", "lexbfs_batch_plan_create", "lexbfs_batch_plan_launch",
            "lexbfs_batch_plan_destroy", "lexbfs_strerror", "lexbfs_last_error", "lexbfs_profile_enable",
            "lexbfs_profile_collect", "lexbfs_batch_max_n", "lexbfs_build_bitset", "lexbfs_plus_workspace_bytes",
            "lexbfs_plus_order", "unit_interval_workspace_bytes", "unit_interval_test",
            "unit_interval_batch_workspace_bytes", "unit_interval_test_batch", "lexbfs_abi_version",
            "chordal_test_noalloc_max_bytes", "chordal_test_noalloc"]


class lexbfs_graph_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("bits", ctypes.c_void_p),
                ("words_per_row", ctypes.c_int64)]


class lexbfs_result_t(ctypes.Structure):
    _fields_ = [("chordal", ctypes.c_int32), ("witness_v", ctypes.c_int32), ("witness_p", ctypes.c_int32),
                ("witness_z", ctypes.c_int32), ("cycle_len", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class lexbfs_outputs_t(ctypes.Structure):
    _fields_ = [("order", ctypes.c_void_p), ("rank", ctypes.c_void_p), ("parent", ctypes.c_void_p),
                ("cycle", ctypes.c_void_p)]


class lexbfs_interval_result_t(ctypes.Structure):
    _fields_ = [("unit_interval", ctypes.c_int32), ("witness", ctypes.c_int32 * 3), ("reserved", ctypes.c_int32 * 4)]


class lexbfs_tuning_t(ctypes.Structure):
    _fields_ = [("wave_max_n", ctypes.c_int32), ("block_threads", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


def hipcc_command(out: str = LIB_PATH):
    return ["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
            "-o", out] + SOURCES


def build() -> str:
    """Compile liblexbfs.so for gfx950 in-tree (cross-compiles without a GPU)."""
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(hipcc_command(tmp))
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    gp = ctypes.POINTER(lexbfs_graph_t)
    lib.lexbfs_workspace_bytes.restype = sz
    lib.lexbfs_workspace_bytes.argtypes = [ctypes.c_int32]
    lib.lexbfs_validate.restype = ctypes.c_int
    lib.lexbfs_validate.argtypes = [gp, vp, sz, vp]
    lib.lexbfs_order.restype = ctypes.c_int
    lib.lexbfs_order.argtypes = [gp, vp, vp, vp, vp, sz, vp]
    lib.chordal_test.restype = ctypes.c_int
    lib.chordal_test.argtypes = [gp, vp, ctypes.POINTER(lexbfs_outputs_t), vp, sz, ctypes.c_uint32, vp]
    lib.lexbfs_batch_workspace_bytes.restype = sz
    lib.lexbfs_batch_workspace_bytes.argtypes = [gp, ctypes.c_int32]
    lib.chordal_test_batch.restype = ctypes.c_int
    lib.chordal_test_batch.argtypes = [gp, ctypes.c_int32, ctypes.POINTER(lexbfs_outputs_t), vp,
                                       ctypes.POINTER(lexbfs_tuning_t), vp, sz, ctypes.c_uint32, vp]
    lib.lexbfs_batch_plan_create.restype = ctypes.c_int
    lib.lexbfs_batch_plan_create.argtypes = [gp, ctypes.c_int32, ctypes.POINTER(lexbfs_outputs_t), vp,
                                             ctypes.POINTER(lexbfs_tuning_t), vp, sz, ctypes.c_uint32, vp,
                                             ctypes.POINTER(ctypes.c_void_p)]
    lib.lexbfs_batch_plan_launch.restype = ctypes.c_int
    lib.lexbfs_batch_plan_launch.argtypes = [vp, vp]
    lib.lexbfs_batch_plan_destroy.restype = None
    lib.lexbfs_batch_plan_destroy.argtypes = [vp]
    lib.lexbfs_strerror.restype = ctypes.c_char_p
    lib.lexbfs_strerror.argtypes = [ctypes.c_int]
    lib.lexbfs_last_error.restype = ctypes.c_char_p
    lib.lexbfs_last_error.argtypes = []
    lib.lexbfs_profile_enable.restype = ctypes.c_int
    lib.lexbfs_profile_enable.argtypes = [ctypes.c_int]
    lib.lexbfs_profile_collect.restype = ctypes.c_int
    lib.lexbfs_profile_collect.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
    lib.lexbfs_build_bitset.restype = ctypes.c_int
    lib.lexbfs_build_bitset.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_int64, vp]
    lib.lexbfs_plus_workspace_bytes.restype = sz
    lib.lexbfs_plus_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64]
    lib.lexbfs_plus_order.restype = ctypes.c_int
    lib.lexbfs_plus_order.argtypes = [gp, vp, vp, vp, vp, vp, sz, vp]
    lib.unit_interval_workspace_bytes.restype = sz
    lib.unit_interval_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64]
    lib.unit_interval_test.restype = ctypes.c_int
    lib.unit_interval_test.argtypes = [gp, vp, vp, vp, sz, vp]
    lib.unit_interval_batch_workspace_bytes.restype = sz
    lib.unit_interval_batch_workspace_bytes.argtypes = [gp, ctypes.c_int32]
    lib.unit_interval_test_batch.restype = ctypes.c_int
    lib.unit_interval_test_batch.argtypes = [gp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_void_p), vp, sz, vp]
    lib.lexbfs_batch_max_n.restype = ctypes.c_int32
    lib.lexbfs_batch_max_n.argtypes = []
    lib.lexbfs_abi_version.restype = ctypes.c_int
    lib.lexbfs_abi_version.argtypes = []
    lib.chordal_test_noalloc_max_bytes.restype = sz
    lib.chordal_test_noalloc_max_bytes.argtypes = []
    lib.chordal_test_noalloc.restype = ctypes.c_int
    lib.chordal_test_noalloc.argtypes = [gp, vp, ctypes.POINTER(lexbfs_outputs_t), ctypes.c_uint32, vp]
    _lib = lib
    return lib


class LexbfsError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        lib = load()
        msg = lib.lexbfs_strerror(code).decode()
        detail = lib.lexbfs_last_error().decode()
        if detail:
            msg = f"{msg} [{detail}]"
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")
        self.code = code


def check(code: int, what: str = ""):
    if code != LEXBFS_OK:
        raise LexbfsError(code, what)
