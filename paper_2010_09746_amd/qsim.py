"""Python binding of the C boundary (include/qsim.h).

Argument marshalling only: every gate, permutation and read-out runs in the
HIP library ``libqsim.so``.  PyTorch provides device memory (a state's
amplitudes live in a torch tensor) and the HIP stream the work is enqueued on.

The ``qs_*`` functions mirror the C entry points one to one; ``State`` and
``Program`` are small owners of the corresponding handles.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

try:  # torch first: the library then binds to the HIP runtime torch loaded
    import torch
except ImportError:  # pragma: no cover - torch is part of the image
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("QSIM_LIB") or os.path.join(_HERE, "libqsim.so")

QS_C64, QS_C128 = 0, 1
QS_FORM_PLAIN, QS_FORM_PASS = 0, 1
QS_PERM_MOVE, QS_PERM_RELABEL = 0, 1
QS_GATE_U, QS_GATE_CX, QS_GATE_CZ, QS_GATE_CU = 0, 1, 2, 3
NOALLOC_MAX_OPS = 32768  # QS_NOALLOC_MAX_OPS

STATUS = {0: "QS_OK", -1: "QS_ERR_ARG", -2: "QS_ERR_OOM", -3: "QS_ERR_BUDGET", -4: "QS_ERR_HIP",
          -5: "QS_ERR_UNSUPPORTED", -6: "QS_ERR_STATE"}

# record layout of qs_gate (80 bytes)
GATE_DTYPE = np.dtype([("kind", np.int32), ("q0", np.int32), ("q1", np.int32), ("pad", np.int32),
                       ("u", np.float64, (8,))])

EXPORTS = [
    "qs_last_error", "qs_device_info", "qs_state_create", "qs_state_destroy", "qs_state_set_stream",
    "qs_state_info", "qs_state_set_basis", "qs_get_permutation", "qs_apply_gate", "qs_apply_gates",
    "qs_permute_qubits", "qs_compile", "qs_program_destroy", "qs_program_get_stats", "qs_program_op_counts",
    "qs_program_instructions", "qs_run_program", "qs_run_circuit", "qs_read_amplitudes", "qs_read_state",
    "qs_expect_z", "qs_norm", "qs_fidelity", "qs_synchronize", "qs_profile_enable", "qs_profile_read",
    "qs_batch_create", "qs_batch_run", "qs_batch_results", "qs_batch_read_state", "qs_batch_get_stats",
    "qs_batch_synchronize", "qs_batch_destroy", "qs_batch_plan",
    "qs_server_create", "qs_server_destroy", "qs_server_fits", "qs_server_admit", "qs_server_step_launch",
    "qs_server_step_wait", "qs_server_result", "qs_server_release", "qs_server_set_solo_tiles",
    "qs_run_program_noalloc", "qs_compile_costed", "qs_run_circuit_costed", "qs_run_circuit_expect_z",
]


class QsimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class qs_run_opts(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("k_tile", ctypes.c_int32), ("max_swaps", ctypes.c_int32),
                ("pinned", ctypes.c_int32), ("perm_exec", ctypes.c_int32), ("max_fuse", ctypes.c_int32),
                ("reg_bits", ctypes.c_int32), ("flags", ctypes.c_int32)]


class qs_pass_costs(ctypes.Structure):
    _fields_ = [("tile_pass", ctypes.c_double), ("in_pass", ctypes.c_double * 3), ("move", ctypes.c_double),
                ("plain", ctypes.c_double * 4)]


def make_pass_costs(tile_pass, in_pass, move, plain) -> qs_pass_costs:
    c = qs_pass_costs()
    c.tile_pass = tile_pass
    c.move = move
    for i in range(3):
        c.in_pass[i] = in_pass[i]
    for i in range(4):
        c.plain[i] = plain[i]
    return c


class qs_program_stats(ctypes.Structure):
    _fields_ = [("n_gates", ctypes.c_int64), ("n_apply", ctypes.c_int64), ("n_perm", ctypes.c_int64),
                ("n_global", ctypes.c_int64), ("n_swaps", ctypes.c_int64), ("n_tile_passes", ctypes.c_int64),
                ("n_move_passes", ctypes.c_int64), ("n_plain", ctypes.c_int64), ("n_remaps", ctypes.c_int64),
                ("compile_ms", ctypes.c_double)]


class qs_batch_opts(ctypes.Structure):
    _fields_ = [("k_tile", ctypes.c_int32), ("max_swaps", ctypes.c_int32), ("pinned", ctypes.c_int32),
                ("reg_bits", ctypes.c_int32), ("max_fuse", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("wait_ms", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class qs_batch_pass_info(ctypes.Structure):
    _fields_ = [("circuit", ctypes.c_int32), ("level", ctypes.c_int32), ("k_tile", ctypes.c_int32),
                ("last", ctypes.c_int32), ("tiles", ctypes.c_int64)]


class qs_batch_item_info(ctypes.Structure):
    _fields_ = [("pass_", ctypes.c_int32), ("dep", ctypes.c_int32), ("t0", ctypes.c_int64), ("t1", ctypes.c_int64),
                ("need", ctypes.c_int64)]


class qs_batch_stats(ctypes.Structure):
    _fields_ = [("n_gates", ctypes.c_int64), ("n_perm", ctypes.c_int64), ("n_passes", ctypes.c_int64),
                ("n_tiles", ctypes.c_int64), ("n_items", ctypes.c_int64), ("state_bytes", ctypes.c_double),
                ("compile_ms", ctypes.c_double)]


class qs_profile_entry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p
_ip = ctypes.POINTER(ctypes.c_int)


def load() -> ctypes.CDLL:
    """Load libqsim.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2010_09746_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.qs_last_error.restype = ctypes.c_char_p
    L.qs_device_info.argtypes = [_ip, _ip, ctypes.POINTER(ctypes.c_size_t), ctypes.c_char_p, ctypes.c_int]
    L.qs_state_create.argtypes = [ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]
    L.qs_state_destroy.argtypes = [_vp]
    L.qs_state_set_stream.argtypes = [_vp, _vp]
    L.qs_state_info.argtypes = [_vp, _ip, _ip, ctypes.POINTER(_vp)]
    L.qs_state_set_basis.argtypes = [_vp, ctypes.c_uint64]
    L.qs_get_permutation.argtypes = [_vp, _ip]
    L.qs_apply_gate.argtypes = [_vp, _vp]
    L.qs_apply_gates.argtypes = [_vp, _vp, ctypes.c_int64]
    L.qs_permute_qubits.argtypes = [_vp, _ip]
    L.qs_compile.argtypes = [_vp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _ip,
                             ctypes.POINTER(qs_run_opts), ctypes.POINTER(_vp)]
    L.qs_compile_costed.argtypes = [_vp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _ip,
                                    ctypes.POINTER(qs_run_opts), ctypes.POINTER(qs_pass_costs), ctypes.POINTER(_vp)]
    L.qs_program_destroy.argtypes = [_vp]
    L.qs_program_get_stats.argtypes = [_vp, ctypes.POINTER(qs_program_stats)]
    L.qs_program_op_counts.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    L.qs_program_instructions.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64,
                                          ctypes.POINTER(ctypes.c_int64)]
    L.qs_run_program.argtypes = [_vp, _vp]
    L.qs_run_program_noalloc.argtypes = [_vp, _vp]
    L.qs_run_circuit.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.POINTER(qs_run_opts)]
    L.qs_run_circuit_costed.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.POINTER(qs_run_opts),
                                        ctypes.POINTER(qs_pass_costs)]
    L.qs_run_circuit_expect_z.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.POINTER(qs_run_opts),
                                          ctypes.POINTER(qs_pass_costs), ctypes.POINTER(ctypes.c_double)]
    L.qs_read_amplitudes.argtypes = [_vp, _vp, ctypes.c_int64, _vp]
    L.qs_read_state.argtypes = [_vp, _vp]
    L.qs_expect_z.argtypes = [_vp, _vp]
    L.qs_norm.argtypes = [_vp, ctypes.POINTER(ctypes.c_double)]
    L.qs_fidelity.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.qs_synchronize.argtypes = [_vp]
    L.qs_batch_create.argtypes = [ctypes.c_int, _ip, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.c_int, ctypes.POINTER(qs_batch_opts), ctypes.POINTER(_vp)]
    L.qs_batch_run.argtypes = [_vp]
    L.qs_batch_results.argtypes = [_vp, _vp, _vp]
    L.qs_batch_read_state.argtypes = [_vp, ctypes.c_int, _vp]
    L.qs_batch_get_stats.argtypes = [_vp, ctypes.POINTER(qs_batch_stats)]
    L.qs_batch_synchronize.argtypes = [_vp]
    L.qs_batch_destroy.argtypes = [_vp]
    L.qs_batch_plan.argtypes = [ctypes.c_int, _ip, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
                                ctypes.c_int, ctypes.POINTER(qs_batch_opts), ctypes.POINTER(qs_batch_pass_info),
                                ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(qs_batch_item_info),
                                ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    L.qs_server_create.argtypes = [ctypes.c_int, ctypes.POINTER(qs_batch_opts), ctypes.c_size_t, ctypes.c_int,
                                   ctypes.c_int, ctypes.POINTER(_vp)]
    L.qs_server_destroy.argtypes = [_vp]
    L.qs_server_set_solo_tiles.argtypes = [_vp, ctypes.c_int64]
    L.qs_server_fits.argtypes = [_vp, ctypes.c_int, _ip]
    L.qs_server_admit.argtypes = [_vp, _vp, _vp, ctypes.c_size_t, _vp, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_int64)]
    L.qs_server_step_launch.argtypes = [_vp, _ip]
    L.qs_server_step_wait.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, _ip]
    L.qs_server_result.argtypes = [_vp, ctypes.c_int64, _vp, _vp, ctypes.POINTER(ctypes.c_double)]
    L.qs_server_release.argtypes = [_vp, ctypes.c_int64]
    L.qs_profile_enable.argtypes = [ctypes.c_int]
    L.qs_profile_read.argtypes = [ctypes.POINTER(qs_profile_entry), ctypes.c_int, _ip]
    for name in EXPORTS:
        if name != "qs_last_error":
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _chk(rc: int) -> None:
    if rc != 0:
        raise QsimError(rc, load().qs_last_error().decode())


def _dtype_code(dtype) -> int:
    if dtype in (QS_C64, "c64", "complex64"):
        return QS_C64
    if dtype in (QS_C128, "c128", "complex128"):
        return QS_C128
    raise ValueError(f"unknown dtype {dtype!r}")


def elem_bytes(dtype) -> int:
    return 8 if _dtype_code(dtype) == QS_C64 else 16


def as_gates(gates) -> np.ndarray:
    g = np.ascontiguousarray(gates)
    if g.dtype.itemsize != 80 or g.dtype.names is None or "u" not in g.dtype.names:
        raise TypeError("gates must be a structured array of 80-byte qs_gate records")
    return g


def _ints(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.intc))


QS_OPT_FULL_MATRICES = 1
QS_OPT_LANE_GATES = 2
QS_OPT_LANE_GATES_WIDE = 4
QS_OPT_LANE_EAGER = 8
QS_OPT_FROM_ZERO = 16
QS_OPT_X_FACTORS = 32


def make_opts(form="pass", k_tile=12, max_swaps=1, pinned=0, perm_exec="move", max_fuse=0,
              reg_bits=0, full_matrices=False, lane_gates=0, lane_eager=False, from_zero=False,
              x_factors=False) -> qs_run_opts:
    o = qs_run_opts()
    o.form = {"plain": QS_FORM_PLAIN, "pass": QS_FORM_PASS}.get(form, form)
    o.k_tile = k_tile
    o.max_swaps = max_swaps
    o.pinned = pinned
    o.perm_exec = {"move": QS_PERM_MOVE, "relabel": QS_PERM_RELABEL}.get(perm_exec, perm_exec)
    o.max_fuse = max_fuse
    o.reg_bits = reg_bits
    if lane_gates not in (0, 2, 4):
        raise ValueError("lane_gates: 0, 2 or 4 thread bits")
    o.flags = ((QS_OPT_FULL_MATRICES if full_matrices else 0)
               | {0: 0, 2: QS_OPT_LANE_GATES, 4: QS_OPT_LANE_GATES_WIDE}[lane_gates]
               | (QS_OPT_LANE_EAGER if lane_eager else 0)
               | (QS_OPT_FROM_ZERO if from_zero else 0)
               | (QS_OPT_X_FACTORS if x_factors else 0))
    return o


# ---------------------------------------------------------------------------
# one function per C entry point


def qs_last_error() -> str:
    return load().qs_last_error().decode()


def qs_device_info():
    cu, lds, hbm = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
    name = ctypes.create_string_buffer(256)
    _chk(load().qs_device_info(ctypes.byref(cu), ctypes.byref(lds), ctypes.byref(hbm), name, 256))
    return dict(cu_count=cu.value, lds_bytes_per_cu=lds.value, hbm_bytes=hbm.value, name=name.value.decode())


def qs_state_create(n: int, dtype, device_buf: int, buf_bytes: int, stream: int) -> int:
    h = _vp()
    _chk(load().qs_state_create(n, _dtype_code(dtype), device_buf, buf_bytes, stream, ctypes.byref(h)))
    return h.value


def qs_state_destroy(h: int) -> None:
    _chk(load().qs_state_destroy(h))


def qs_state_set_stream(h: int, stream: int) -> None:
    _chk(load().qs_state_set_stream(h, stream))


def qs_state_set_basis(h: int, x: int) -> None:
    _chk(load().qs_state_set_basis(h, x))


def qs_get_permutation(h: int, n: int) -> list:
    s = np.zeros(n, dtype=np.intc)
    _chk(load().qs_get_permutation(h, s.ctypes.data_as(_ip)))
    return [int(x) for x in s]


def qs_apply_gates(h: int, gates) -> None:
    g = as_gates(gates)
    _chk(load().qs_apply_gates(h, g.ctypes.data, len(g)))


def qs_apply_gate(h: int, gate) -> None:
    g = as_gates(np.asarray([gate], dtype=GATE_DTYPE) if not isinstance(gate, np.ndarray) else gate.reshape(1))
    _chk(load().qs_apply_gate(h, g.ctypes.data))


def qs_permute_qubits(h: int, sigma_new) -> None:
    _chk(load().qs_permute_qubits(h, _ints(sigma_new).ctypes.data_as(_ip)))


def qs_compile(gates, n: int, dtype, sigma0=None, opts: qs_run_opts | None = None) -> int:
    g = as_gates(gates)
    h = _vp()
    s0 = _ints(sigma0).ctypes.data_as(_ip) if sigma0 is not None else None
    _chk(load().qs_compile(g.ctypes.data, len(g), n, _dtype_code(dtype), s0,
                           ctypes.byref(opts) if opts is not None else None, ctypes.byref(h)))
    return h.value


def qs_compile_costed(gates, n: int, dtype, sigma0=None, opts: qs_run_opts | None = None,
                      costs: qs_pass_costs | None = None) -> int:
    g = as_gates(gates)
    h = _vp()
    s0 = _ints(sigma0).ctypes.data_as(_ip) if sigma0 is not None else None
    _chk(load().qs_compile_costed(g.ctypes.data, len(g), n, _dtype_code(dtype), s0,
                                  ctypes.byref(opts) if opts is not None else None,
                                  ctypes.byref(costs) if costs is not None else None, ctypes.byref(h)))
    return h.value


def qs_program_destroy(h: int) -> None:
    _chk(load().qs_program_destroy(h))


def qs_program_get_stats(h: int) -> dict:
    st = qs_program_stats()
    _chk(load().qs_program_get_stats(h, ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in qs_program_stats._fields_}


OPC_NAMES = ["tile_pass", "u", "u_ctrl", "x_reg", "x_lane", "neg", "diag", "remap", "dispatch", "plain_u",
             "plain_cu", "plain_cx", "plain_cz", "move", "move_fraction", "shear", "phase", "lswap", "lane",
             "remap_wave"]


def qs_program_op_counts(h: int) -> dict:
    """Work of a compiled program by class (see qs_program_op_counts in qsim.h)."""
    out = np.zeros(len(OPC_NAMES), dtype=np.float64)
    _chk(load().qs_program_op_counts(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(OPC_NAMES)))
    return dict(zip(OPC_NAMES, (float(v) for v in out)))


def qs_program_instructions(h: int, n: int):
    ln = ctypes.c_int64()
    _chk(load().qs_program_instructions(h, None, 0, ctypes.byref(ln)))
    buf = np.zeros(max(ln.value, 1), dtype=np.int32)
    _chk(load().qs_program_instructions(h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ln.value,
                                        ctypes.byref(ln)))
    out, k = [], 0
    while k < ln.value:
        op = int(buf[k])
        if op == 1:
            out.append(("perm", tuple(int(x) for x in buf[k + 1:k + 1 + n])))
            k += 1 + n
        else:
            out.append(("apply" if op == 0 else "global", int(buf[k + 1])))
            k += 2
    return out


def qs_run_program(h: int, prog: int) -> None:
    _chk(load().qs_run_program(h, prog))


def qs_run_program_noalloc(h: int, prog: int) -> None:
    _chk(load().qs_run_program_noalloc(h, prog))


def qs_run_circuit(h: int, gates, opts: qs_run_opts | None = None) -> None:
    g = as_gates(gates)
    _chk(load().qs_run_circuit(h, g.ctypes.data, len(g), ctypes.byref(opts) if opts is not None else None))


def qs_run_circuit_costed(h: int, gates, opts: qs_run_opts | None = None, costs: qs_pass_costs | None = None) -> None:
    g = as_gates(gates)
    _chk(load().qs_run_circuit_costed(h, g.ctypes.data, len(g), ctypes.byref(opts) if opts is not None else None,
                                      ctypes.byref(costs) if costs is not None else None))


def qs_run_circuit_expect_z(h: int, n: int, gates, opts: qs_run_opts | None = None,
                            costs: qs_pass_costs | None = None) -> np.ndarray:
    g = as_gates(gates)
    out = np.zeros(n, dtype=np.float64)
    _chk(load().qs_run_circuit_expect_z(h, g.ctypes.data, len(g), ctypes.byref(opts) if opts is not None else None,
                                        ctypes.byref(costs) if costs is not None else None,
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def qs_read_amplitudes(h: int, idx) -> np.ndarray:
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
    out = np.zeros(2 * len(idx), dtype=np.float64)
    _chk(load().qs_read_amplitudes(h, idx.ctypes.data, len(idx), out.ctypes.data))
    return out[0::2] + 1j * out[1::2]


def qs_read_state(h: int, n: int) -> np.ndarray:
    out = np.zeros(2 << n, dtype=np.float64)
    _chk(load().qs_read_state(h, out.ctypes.data))
    return out[0::2] + 1j * out[1::2]


def qs_expect_z(h: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    _chk(load().qs_expect_z(h, out.ctypes.data))
    return out


def qs_norm(h: int) -> float:
    v = ctypes.c_double()
    _chk(load().qs_norm(h, ctypes.byref(v)))
    return v.value


def qs_fidelity(a: int, b: int):
    loss, mx = ctypes.c_double(), ctypes.c_double()
    _chk(load().qs_fidelity(a, b, ctypes.byref(loss), ctypes.byref(mx)))
    return loss.value, mx.value


def qs_synchronize(h: int) -> None:
    _chk(load().qs_synchronize(h))


def qs_profile_enable(on: bool) -> None:
    _chk(load().qs_profile_enable(1 if on else 0))


def qs_profile_read() -> dict:
    """{kernel class: dict(launches, total_ms, avg_ms, bytes)} since the last read."""
    buf = (qs_profile_entry * 32)()
    n = ctypes.c_int()
    _chk(load().qs_profile_read(buf, 32, ctypes.byref(n)))
    out = {}
    for i in range(min(n.value, 32)):
        e = buf[i]
        out[e.name.decode()] = dict(launches=e.launches, total_ms=e.total_ms,
                                    avg_ms=e.total_ms / max(e.launches, 1), bytes=e.bytes)
    return out


def make_batch_opts(k_tile=12, max_swaps=8, pinned=3, reg_bits=0, max_fuse=0, wg_per_cu=4, chunk=4,
                    use_graph=1, wait_ms=0) -> qs_batch_opts:
    o = qs_batch_opts()
    o.k_tile, o.max_swaps, o.pinned, o.reg_bits = k_tile, max_swaps, pinned, reg_bits
    o.max_fuse, o.wg_per_cu, o.chunk, o.use_graph = max_fuse, wg_per_cu, chunk, use_graph
    o.wait_ms = wait_ms
    return o


def qs_batch_create(circuits, dtype, opts: qs_batch_opts) -> int:
    """circuits: sequence of (n, gates)."""
    arrs = [as_gates(g) for _, g in circuits]
    cnt = len(arrs)
    ns = np.ascontiguousarray([int(n) for n, _ in circuits], dtype=np.intc)
    ptrs = (ctypes.c_void_p * cnt)(*[a.ctypes.data for a in arrs])
    ngs = (ctypes.c_int64 * cnt)(*[len(a) for a in arrs])
    h = _vp()
    _chk(load().qs_batch_create(cnt, ns.ctypes.data_as(_ip), ptrs, ngs, _dtype_code(dtype), ctypes.byref(opts),
                                ctypes.byref(h)))
    return h.value


def qs_batch_plan(circuits, dtype, opts: qs_batch_opts):
    """Host-only plan of a batch: (passes, items) as lists of dicts, items in
    ticket order (see qs_batch_plan in qsim.h)."""
    arrs = [as_gates(g) for _, g in circuits]
    cnt = len(arrs)
    ns = np.ascontiguousarray([int(n) for n, _ in circuits], dtype=np.intc)
    ptrs = (ctypes.c_void_p * cnt)(*[a.ctypes.data for a in arrs])
    ngs = (ctypes.c_int64 * cnt)(*[len(a) for a in arrs])
    npass, nitem = ctypes.c_int64(), ctypes.c_int64()
    _chk(load().qs_batch_plan(cnt, ns.ctypes.data_as(_ip), ptrs, ngs, _dtype_code(dtype), ctypes.byref(opts),
                              None, 0, ctypes.byref(npass), None, 0, ctypes.byref(nitem)))
    P = (qs_batch_pass_info * max(1, npass.value))()
    I = (qs_batch_item_info * max(1, nitem.value))()
    _chk(load().qs_batch_plan(cnt, ns.ctypes.data_as(_ip), ptrs, ngs, _dtype_code(dtype), ctypes.byref(opts),
                              P, npass.value, ctypes.byref(npass), I, nitem.value, ctypes.byref(nitem)))
    passes = [dict(circuit=p.circuit, level=p.level, k_tile=p.k_tile, last=p.last, tiles=p.tiles)
              for p in P[:npass.value]]
    items = [dict(pass_=i.pass_, dep=i.dep, t0=i.t0, t1=i.t1, need=i.need) for i in I[:nitem.value]]
    return passes, items


def qs_batch_run(h: int) -> None:
    _chk(load().qs_batch_run(h))


def qs_batch_results(h: int, count: int):
    z = np.zeros(count, dtype=np.float64)
    nrm = np.zeros(count, dtype=np.float64)
    _chk(load().qs_batch_results(h, z.ctypes.data, nrm.ctypes.data))
    return z, nrm


def qs_batch_read_state(h: int, c: int, n: int) -> np.ndarray:
    out = np.zeros(2 << n, dtype=np.float64)
    _chk(load().qs_batch_read_state(h, c, out.ctypes.data))
    return out[0::2] + 1j * out[1::2]


def qs_batch_get_stats(h: int) -> dict:
    st = qs_batch_stats()
    _chk(load().qs_batch_get_stats(h, ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in qs_batch_stats._fields_}


def qs_batch_synchronize(h: int) -> None:
    _chk(load().qs_batch_synchronize(h))


def qs_batch_destroy(h: int) -> None:
    _chk(load().qs_batch_destroy(h))


def qs_server_create(dtype, opts: qs_batch_opts, hbm_budget: int, max_slots: int, max_samples: int) -> int:
    h = _vp()
    _chk(load().qs_server_create(_dtype_code(dtype), ctypes.byref(opts), int(hbm_budget), max_slots, max_samples,
                                 ctypes.byref(h)))
    return h.value


def qs_server_set_solo_tiles(h: int, min_tiles: int) -> None:
    """Passes with at least min_tiles tiles run as launches of their own (0: never)."""
    _chk(load().qs_server_set_solo_tiles(h, int(min_tiles)))


def qs_server_destroy(h: int) -> None:
    _chk(load().qs_server_destroy(h))


def qs_server_fits(h: int, n: int) -> bool:
    f = ctypes.c_int()
    _chk(load().qs_server_fits(h, n, ctypes.byref(f)))
    return bool(f.value)


def qs_server_admit(h: int, prog: int, buf_ptr: int, buf_bytes: int, samples) -> int:
    smp = np.ascontiguousarray(np.asarray(samples, dtype=np.uint64))
    rid = ctypes.c_int64()
    _chk(load().qs_server_admit(h, prog, buf_ptr, buf_bytes, smp.ctypes.data if len(smp) else None, len(smp),
                                ctypes.byref(rid)))
    return rid.value


def qs_server_step_launch(h: int) -> int:
    n = ctypes.c_int()
    _chk(load().qs_server_step_launch(h, ctypes.byref(n)))
    return n.value


def qs_server_step_wait(h: int, cap: int = 4096):
    ids = (ctypes.c_int64 * cap)()
    n = ctypes.c_int()
    _chk(load().qs_server_step_wait(h, ids, cap, ctypes.byref(n)))
    return [ids[i] for i in range(min(n.value, cap))]


def qs_server_result(h: int, rid: int, n: int, count: int):
    z = np.zeros(n, dtype=np.float64)
    amps = np.zeros(2 * max(count, 1), dtype=np.float64)
    nrm = ctypes.c_double()
    _chk(load().qs_server_result(h, rid, z.ctypes.data, amps.ctypes.data, ctypes.byref(nrm)))
    a = amps[0:2 * count:2] + 1j * amps[1:2 * count:2]
    return z, a, nrm.value


def qs_server_release(h: int, rid: int) -> None:
    _chk(load().qs_server_release(h, rid))


# ---------------------------------------------------------------------------
# owners


def _current_stream() -> int:
    return int(torch.cuda.current_stream().cuda_stream)


class State:
    """A state vector in a torch-owned device buffer."""

    def __init__(self, n: int, dtype="c128", device: str = "cuda", stream: int | None = None,
                 buffer=None):
        if torch is None or not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        self.n = n
        self.dtype = _dtype_code(dtype)
        nbytes = elem_bytes(dtype) << n
        if buffer is None:
            buffer = torch.empty(nbytes, dtype=torch.uint8, device=device)
        elif buffer.numel() * buffer.element_size() < nbytes:
            raise ValueError("buffer too small")
        self.buffer = buffer
        self.stream = _current_stream() if stream is None else stream
        self.h = qs_state_create(n, self.dtype, buffer.data_ptr(), nbytes, self.stream)

    def close(self):
        if getattr(self, "h", None):
            qs_state_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # preparation, gates, data movement
    def set_basis(self, x: int) -> "State":
        qs_state_set_basis(self.h, x)
        return self

    def apply_gates(self, gates) -> "State":
        qs_apply_gates(self.h, gates)
        return self

    def permute(self, sigma_new) -> "State":
        qs_permute_qubits(self.h, sigma_new)
        return self

    def run(self, gates, costs: qs_pass_costs | None = None, **opts) -> "State":
        if costs is None:
            qs_run_circuit(self.h, gates, make_opts(**opts))
        else:
            qs_run_circuit_costed(self.h, gates, make_opts(**opts), costs)
        return self

    def run_expect_z(self, gates, costs: qs_pass_costs | None = None, **opts) -> np.ndarray:
        """run() and then expect_z(), the read-out folded into the last tile pass."""
        return qs_run_circuit_expect_z(self.h, self.n, gates, make_opts(**opts), costs)

    def run_program(self, prog: "Program", noalloc: bool = False) -> "State":
        (qs_run_program_noalloc if noalloc else qs_run_program)(self.h, prog.h)
        return self

    # read-out
    @property
    def sigma(self):
        return qs_get_permutation(self.h, self.n)

    def amplitudes(self, idx) -> np.ndarray:
        return qs_read_amplitudes(self.h, idx)

    def to_numpy(self) -> np.ndarray:
        return qs_read_state(self.h, self.n)

    def expect_z(self) -> np.ndarray:
        return qs_expect_z(self.h, self.n)

    def norm(self) -> float:
        return qs_norm(self.h)

    def fidelity(self, other: "State"):
        return qs_fidelity(self.h, other.h)

    def synchronize(self) -> None:
        qs_synchronize(self.h)


class Program:
    """A compiled circuit (pass of Section 3 + lowering to launches)."""

    def __init__(self, gates, n: int, dtype="c128", sigma0=None, costs: qs_pass_costs | None = None, **opts):
        self.n = n
        if costs is None:
            self.h = qs_compile(gates, n, dtype, sigma0, make_opts(**opts))
        else:
            self.h = qs_compile_costed(gates, n, dtype, sigma0, make_opts(**opts), costs)

    def stats(self) -> dict:
        return qs_program_get_stats(self.h)

    def op_counts(self) -> dict:
        return qs_program_op_counts(self.h)

    def instructions(self):
        return qs_program_instructions(self.h, self.n)

    def close(self):
        if getattr(self, "h", None):
            qs_program_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many circuits (list of (n, gates)) run by one persistent launch."""

    def __init__(self, circuits, dtype="c64", **opts):
        self.ns = [int(n) for n, _ in circuits]
        self.count = len(self.ns)
        self.opts = dict(opts)
        self.h = qs_batch_create(circuits, dtype, make_batch_opts(**opts))

    def run(self) -> "Batch":
        qs_batch_run(self.h)
        return self

    def results(self):
        """(<Z_0>, norm) per circuit after the last run."""
        return qs_batch_results(self.h, self.count)

    def state(self, c: int) -> np.ndarray:
        return qs_batch_read_state(self.h, c, self.ns[c])

    def stats(self) -> dict:
        return qs_batch_get_stats(self.h)

    def synchronize(self) -> None:
        qs_batch_synchronize(self.h)

    def close(self):
        if getattr(self, "h", None):
            qs_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
