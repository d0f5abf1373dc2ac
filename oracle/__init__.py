"""CPU oracle: plain complex128 simulator, dense checker and reference pass.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  Nothing in the product package
imports this module, and this module imports nothing from the product package:
the two share only the seeded inputs of ``workloads``.

Contents (each follows the passage cited on it):
* ``run`` / ``apply_gate`` / ``norm`` / ``expect_z`` / ``gather``: gate-by-gate
  state-vector simulation (``sim.c``).
* ``permute`` / ``index_map``: the amplitude placement j(i, sigma) and the data
  movement of PermuteQubits (paper, Section 2).
* ``pass_ref``: the permutation-inserting pass (paper, Section 3, Algorithm 1)
  in ``pass_ref.c``.
* ``run_program``: executes a compiled instruction list on a physical vector
  while tracking the placement sigma.
* ``dense_unitary``: the circuit unitary as a product of numpy Kronecker
  products, for n <= 8 (an independent library check of ``run``).
* ``decompose_permutation``: the three-step split of a placement change
  (paper, Appendix A, Algorithm 2).
* ``model_time``: the step-function cost model of Section 4 (communicating
  operations cost a fixed multiple of local ones).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)

U, CX, CZ, CU = 0, 1, 2, 3
APPLY, PERM, GLOBAL = 0, 1, 2


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_apply_gate.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
        L.orc_apply_gate.restype = ctypes.c_int
        L.orc_run.argtypes = [_dp, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64]
        L.orc_run.restype = ctypes.c_int
        L.orc_set_basis.argtypes = [_dp, ctypes.c_int, ctypes.c_uint64]
        L.orc_norm.argtypes = [_dp, ctypes.c_int]
        L.orc_norm.restype = ctypes.c_double
        L.orc_expect_z.argtypes = [_dp, ctypes.c_int, _dp]
        L.orc_index_map.argtypes = [ctypes.c_uint64, ctypes.c_int, _ip]
        L.orc_index_map.restype = ctypes.c_uint64
        L.orc_permute.argtypes = [_dp, _dp, ctypes.c_int, _ip, _ip]
        L.orc_pass.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int64, _i64p]
        L.orc_pass.restype = ctypes.c_int64
        L.orc_dag_edges.argtypes = [ctypes.c_void_p, ctypes.c_int64, _i64p, ctypes.c_int64]
        L.orc_dag_edges.restype = ctypes.c_int64
        L.orc_gate_is_local.argtypes = [ctypes.c_void_p, _ip, ctypes.c_int]
        L.orc_gate_is_local.restype = ctypes.c_int
        L.orc_commute.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_commute.restype = ctypes.c_int
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        _lib = L
    return _lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _ints(seq) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(seq, dtype=np.intc))


def _gates(g: np.ndarray) -> np.ndarray:
    g = np.ascontiguousarray(g)
    assert g.dtype.itemsize == 80
    return g


# ----------------------------------------------------------------------------
# state vectors (complex128, logical order unless stated)

def zero_state(n: int, x: int = 0) -> np.ndarray:
    s = np.zeros(1 << n, dtype=np.complex128)
    s[x] = 1.0
    return s


def apply_gate(state: np.ndarray, n: int, kind: int, p0: int, p1: int, u8) -> None:
    """Apply one gate in place, its qubits read as bit positions p0, p1."""
    u = np.ascontiguousarray(np.asarray(u8, dtype=np.float64))
    rc = lib().orc_apply_gate(_d(state.view(np.float64)), n, kind, p0, p1, _d(u))
    assert rc == 0, "unknown gate kind"


def run(gates: np.ndarray, n: int, x: int = 0, state: np.ndarray | None = None) -> np.ndarray:
    """Plain gate-by-gate simulation from |x> (or from ``state``, copied)."""
    s = zero_state(n, x) if state is None else np.array(state, dtype=np.complex128, copy=True)
    g = _gates(gates)
    rc = lib().orc_run(_d(s.view(np.float64)), n, g.ctypes.data, len(g))
    assert rc == 0
    return s


def threads() -> int:
    """OpenMP threads used by the simulator loops."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Run the simulator loops with n threads."""
    lib().orc_set_threads(int(n))


def norm(state: np.ndarray, n: int) -> float:
    return lib().orc_norm(_d(np.ascontiguousarray(state).view(np.float64)), n)


def expect_z(state: np.ndarray, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    lib().orc_expect_z(_d(np.ascontiguousarray(state).view(np.float64)), n, _d(out))
    return out


def index_map(i: int, n: int, sigma) -> int:
    """j(i, sigma) = sum_q i_q 2^sigma(q) (paper, Section 2)."""
    return int(lib().orc_index_map(i, n, _ints(sigma).ctypes.data_as(_ip)))


def permute(vec: np.ndarray, n: int, sigma_from, sigma_to) -> np.ndarray:
    """New physical vector: dst[j(i, sigma_to)] = vec[j(i, sigma_from)]."""
    src = np.ascontiguousarray(vec, dtype=np.complex128)
    dst = np.empty_like(src)
    lib().orc_permute(_d(src.view(np.float64)), _d(dst.view(np.float64)), n,
                      _ints(sigma_from).ctypes.data_as(_ip), _ints(sigma_to).ctypes.data_as(_ip))
    return dst


def to_logical(vec: np.ndarray, n: int, sigma) -> np.ndarray:
    """Logical amplitudes a_i = vec[j(i, sigma)]."""
    return permute(vec, n, sigma, list(range(n)))


def gather(state: np.ndarray, idx) -> np.ndarray:
    return np.asarray(state)[np.asarray(idx, dtype=np.int64)]


# ----------------------------------------------------------------------------
# dense checker (numpy Kronecker products), n <= 8

def _mat(g) -> np.ndarray:
    u = np.asarray(g["u"], dtype=np.float64)
    return (u[0::2] + 1j * u[1::2]).reshape(2, 2)


def _embed_1q(m: np.ndarray, q: int, n: int) -> np.ndarray:
    # basis index bit q <-> qubit q; numpy kron puts the first factor on the
    # most significant bit, so qubit n-1 comes first.
    out = np.array([[1.0 + 0j]])
    for k in range(n - 1, -1, -1):
        out = np.kron(out, m if k == q else np.eye(2))
    return out


def _proj(q: int, n: int, bit: int) -> np.ndarray:
    p = np.zeros((2, 2), dtype=np.complex128)
    p[bit, bit] = 1.0
    return _embed_1q(p, q, n)


def gate_matrix(g, n: int) -> np.ndarray:
    kind, q0, q1 = int(g["kind"]), int(g["q0"]), int(g["q1"])
    if kind == U:
        return _embed_1q(_mat(g), q0, n)
    if kind in (CX, CU):
        m = np.array([[0, 1], [1, 0]], dtype=np.complex128) if kind == CX else _mat(g)
        return _proj(q0, n, 0) + _proj(q0, n, 1) @ _embed_1q(m, q1, n)
    if kind == CZ:
        z = np.diag([1.0, -1.0]).astype(np.complex128)
        return _proj(q0, n, 0) + _proj(q0, n, 1) @ _embed_1q(z, q1, n)
    raise ValueError(kind)


def dense_unitary(gates: np.ndarray, n: int) -> np.ndarray:
    assert n <= 8, "dense checker is for small n"
    m = np.eye(1 << n, dtype=np.complex128)
    for g in gates:
        m = gate_matrix(g, n) @ m
    return m


# ----------------------------------------------------------------------------
# reference pass (paper, Section 3, Algorithm 1)

def pass_ref(gates: np.ndarray, n: int, m: int, r: int = 1, pinned: int = 0):
    """Returns (instructions, stats).  instructions: list of
    ('apply', v) | ('perm', sigma tuple) | ('global', v).
    stats: dict(apply, perm, global, swaps)."""
    g = _gates(gates)
    cap = 4 * len(g) + 64
    while True:
        out = np.zeros(cap, dtype=np.int32)
        st = np.zeros(4, dtype=np.int64)
        w = lib().orc_pass(g.ctypes.data, len(g), n, m, r, pinned,
                           out.ctypes.data_as(_i32p), cap, st.ctypes.data_as(_i64p))
        if w == -2:
            cap *= 4
            continue
        if w < 0:
            raise ValueError("orc_pass rejected its arguments")
        break
    ins, k = [], 0
    while k < w:
        op = int(out[k])
        if op == PERM:
            ins.append(("perm", tuple(int(x) for x in out[k + 1:k + 1 + n])))
            k += 1 + n
        else:
            ins.append(("apply" if op == APPLY else "global", int(out[k + 1])))
            k += 2
    stats = dict(apply=int(st[0]), perm=int(st[1]), glob=int(st[2]), swaps=int(st[3]))
    return ins, stats


def dag_edges(gates: np.ndarray):
    g = _gates(gates)
    e = lib().orc_dag_edges(g.ctypes.data, len(g), None, 0)
    buf = np.zeros(2 * max(e, 1), dtype=np.int64)
    lib().orc_dag_edges(g.ctypes.data, len(g), buf.ctypes.data_as(_i64p), len(buf))
    return [(int(buf[2 * k]), int(buf[2 * k + 1])) for k in range(e)]


def gate_is_local(gate_rec, sigma, m: int) -> bool:
    one = np.ascontiguousarray(np.array([gate_rec]))
    return bool(lib().orc_gate_is_local(one.ctypes.data, _ints(sigma).ctypes.data_as(_ip), m))


def commute(a, b) -> bool:
    A = np.ascontiguousarray(np.array([a]))
    B = np.ascontiguousarray(np.array([b]))
    return bool(lib().orc_commute(A.ctypes.data, B.ctypes.data))


def run_program(gates: np.ndarray, n: int, instructions, x: int = 0, sigma0=None):
    """Execute a compiled instruction list on a physical vector: a gate on
    logical qubit q acts on bit sigma(q); PermuteQubits moves the data.
    Returns (physical vector, final sigma)."""
    sigma = list(range(n)) if sigma0 is None else list(sigma0)
    v = zero_state(n, index_map(x, n, sigma))
    for op, arg in instructions:
        if op == "perm":
            v = permute(v, n, sigma, arg)
            sigma = list(arg)
        else:
            gr = gates[arg]
            q1 = int(gr["q1"])
            apply_gate(v, n, int(gr["kind"]), sigma[int(gr["q0"])], sigma[q1] if q1 >= 0 else -1,
                       gr["u"])
    return v, sigma


# ----------------------------------------------------------------------------
# three-step placement change (paper, Appendix A, Algorithm 2)

def decompose_permutation(sigma, sigma_new, m: int):
    """Split sigma -> sigma_new into sigma -> s1 (local positions reordered among
    themselves) -> s2 (global positions reordered among themselves) ->
    sigma_new (local/global pairs exchanged).

    The printed initialisation sets both intermediates to the identity, which
    leaves entries unassigned for non-trivial sigma; they are read here as
    starting from sigma (for s1) and from s1 (for s2), so that untouched
    entries keep their current position."""
    n = len(sigma)
    inv = [0] * n
    for q, p in enumerate(sigma):
        inv[p] = q
    s1_inv = list(inv)
    for p in range(m):
        pp = sigma_new[inv[p]]
        while pp >= m:
            pp = sigma_new[inv[pp]]
        s1_inv[pp] = inv[p]
    s2_inv = list(s1_inv)
    for p in range(m, n):
        pp = sigma_new[s1_inv[p]]
        while pp < m:
            pp = sigma_new[s1_inv[pp]]
        s2_inv[pp] = s1_inv[p]
    s1 = [0] * n
    s2 = [0] * n
    for p in range(n):
        s1[s1_inv[p]] = p
        s2[s2_inv[p]] = p
    return s1, s2


# ----------------------------------------------------------------------------
# step-function cost model (paper, Section 4)

def communicating_fraction_original(gates: np.ndarray, n: int, m: int) -> float:
    ident = list(range(n))
    return sum(0 if gate_is_local(g, ident, m) else 1 for g in gates) / len(gates)


def model_time_original(gates: np.ndarray, n: int, m: int, overhead: float) -> float:
    ident = list(range(n))
    return float(sum(1.0 if gate_is_local(g, ident, m) else overhead for g in gates))


def model_time_compiled(stats, overhead: float) -> float:
    """Local ApplyGate costs 1; every PermuteQubits (one local/global exchange
    for r = 1) and every communicating gate costs ``overhead``."""
    return stats["apply"] + overhead * (stats["perm"] + stats["glob"])


def model_reduction_from_fractions(f_orig: float, f_opt: float, overhead: float) -> float:
    """1 - t_opt/t_orig with times per original operation written as
    (1 - f) + f * overhead (paper, Section 4)."""
    return 1.0 - ((1 - f_opt) + f_opt * overhead) / ((1 - f_orig) + f_orig * overhead)
