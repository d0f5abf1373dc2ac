"""Seeded circuit generators.

A circuit is a numpy structured array of ``GATE_DTYPE`` records (80 bytes
each, the layout the C boundary reads directly):

* ``kind``: 0 = U (one-qubit 2x2), 1 = CX, 2 = CZ, 3 = CU (controlled 2x2)
* ``q0``: target of U, control of CX/CU, first qubit of CZ
* ``q1``: target of CX/CU, second qubit of CZ, unused (-1) for U
* ``u``: the 2x2 matrix row-major as interleaved (re, im) doubles
  (u00, u01, u10, u11); CX/CZ carry X / diag(1,-1) for completeness.

Qubit q is bit q of the basis index (paper, Section 2, the index map
i = sum_q i_q 2^q).

Workloads
---------
* ``layered_circuit``: every layer applies a Haar-random U(2) to each qubit in
  ascending order, then a two-qubit gate on every pair of a random perfect
  matching (CX; CZ on layers l with l % 3 == 2 when requested).
* ``paper_random_circuit``: the random family of the paper's Section 4: each
  gate is a CNOT with probability p on two distinct uniform qubits, otherwise
  H or Y (uniformly) on a uniform qubit.
* ``qft_like_circuit``: the Appendix C family, QFT structure with CNOTs in
  place of the controlled rotations.
* ``qft_circuit``, ``ghz_circuit``: closed-form test circuits.
"""

from __future__ import annotations

import math

import numpy as np

KIND_U, KIND_CX, KIND_CZ, KIND_CU = 0, 1, 2, 3

GATE_DTYPE = np.dtype([
    ("kind", np.int32), ("q0", np.int32), ("q1", np.int32), ("pad", np.int32),
    ("u", np.float64, (8,)),
])

MASTER_SEED = 20100946

_S2 = 1.0 / math.sqrt(2.0)
H = np.array([[_S2, _S2], [_S2, -_S2]], dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def phase(theta: float) -> np.ndarray:
    """diag(1, e^{i theta})."""
    return np.array([[1, 0], [0, complex(math.cos(theta), math.sin(theta))]],
                    dtype=np.complex128)


def _pack(m: np.ndarray) -> np.ndarray:
    m = np.asarray(m, dtype=np.complex128).reshape(4)
    out = np.empty(8, dtype=np.float64)
    out[0::2] = m.real
    out[1::2] = m.imag
    return out


def make_gates(records) -> np.ndarray:
    """Build a gate array from (kind, q0, q1, matrix_or_None) tuples."""
    g = np.zeros(len(records), dtype=GATE_DTYPE)
    for i, (kind, q0, q1, m) in enumerate(records):
        g[i]["kind"] = kind
        g[i]["q0"] = q0
        g[i]["q1"] = q1
        if m is None:
            m = X if kind == KIND_CX else (Z if kind == KIND_CZ else np.eye(2))
        g[i]["u"] = _pack(m)
    return g


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def haar_u2(rng: np.random.Generator) -> np.ndarray:
    """Haar-random U(2) from the Euler-angle parametrisation of Zyczkowski and
    Kus: U = e^{i a} [[e^{i p} cos f, e^{i c} sin f], [-e^{-i c} sin f,
    e^{-i p} cos f]] with a, p, c uniform in [0, 2 pi) and f = asin(sqrt(x)),
    x uniform in [0, 1)."""
    a, p, c = rng.uniform(0.0, 2.0 * math.pi, size=3)
    f = math.asin(math.sqrt(rng.uniform(0.0, 1.0)))
    e = np.exp
    return e(1j * a) * np.array(
        [[e(1j * p) * math.cos(f), e(1j * c) * math.sin(f)],
         [-e(-1j * c) * math.sin(f), e(-1j * p) * math.cos(f)]],
        dtype=np.complex128)


def _haar_batch(rng: np.random.Generator, count: int) -> np.ndarray:
    """``count`` Haar-random U(2) matrices (same parametrisation as haar_u2),
    as a (count, 2, 2) complex array."""
    a, p, c = (rng.uniform(0.0, 2.0 * math.pi, size=count) for _ in range(3))
    f = np.arcsin(np.sqrt(rng.uniform(0.0, 1.0, size=count)))
    ph = np.exp(1j * a)
    m = np.empty((count, 2, 2), dtype=np.complex128)
    m[:, 0, 0] = ph * np.exp(1j * p) * np.cos(f)
    m[:, 0, 1] = ph * np.exp(1j * c) * np.sin(f)
    m[:, 1, 0] = -ph * np.exp(-1j * c) * np.sin(f)
    m[:, 1, 1] = ph * np.exp(-1j * p) * np.cos(f)
    return m


def layered_circuit(n: int, layers: int, seed: int, cz_every_third: bool = True) -> np.ndarray:
    """Haar-U(2) on every qubit, then a 2q gate on each pair of a random perfect
    matching (control = first of the pair; odd n leaves the last qubit idle).
    With ``cz_every_third`` the 2q gate is CZ on layers l with l % 3 == 2."""
    rng = _rng(seed, n, layers)
    per = n + n // 2
    g = np.zeros(layers * per, dtype=GATE_DTYPE)
    x_mat, z_mat = _pack(X), _pack(Z)
    for layer in range(layers):
        base = layer * per
        mats = _haar_batch(rng, n)
        blk = g[base:base + n]
        blk["kind"] = KIND_U
        blk["q0"] = np.arange(n)
        blk["q1"] = -1
        u = mats.reshape(n, 4)
        blk["u"][:, 0::2] = u.real
        blk["u"][:, 1::2] = u.imag
        g[base:base + n] = blk
        perm = rng.permutation(n)
        two = g[base + n:base + per]
        cz = cz_every_third and layer % 3 == 2
        two["kind"] = KIND_CZ if cz else KIND_CX
        two["q0"] = perm[0:2 * (n // 2):2]
        two["q1"] = perm[1:2 * (n // 2):2]
        two["u"] = z_mat if cz else x_mat
        g[base + n:base + per] = two
    return g


def paper_random_circuit(n: int, n_gates: int, p: float, seed: int) -> np.ndarray:
    """Random family of the paper's Section 4: CNOT with probability p (distinct
    uniform control and target), else H or Y with equal probability on a
    uniform qubit."""
    rng = _rng(seed, n, n_gates, int(round(p * 1e6)))
    recs = []
    for _ in range(n_gates):
        if rng.uniform() < p:
            c, t = rng.choice(n, size=2, replace=False)
            recs.append((KIND_CX, int(c), int(t), None))
        else:
            q = int(rng.integers(n))
            recs.append((KIND_U, q, -1, H if rng.uniform() < 0.5 else Y))
    return make_gates(recs)


def qft_like_circuit(n: int) -> np.ndarray:
    """Appendix C: the QFT layout where each controlled rotation is replaced by
    a CNOT. Qubit j gets H, then a CNOT from every higher qubit k > j."""
    recs = []
    for j in range(n):
        recs.append((KIND_U, j, -1, H))
        for k in range(j + 1, n):
            recs.append((KIND_CX, k, j, None))
    return make_gates(recs)


def qft_circuit(n: int) -> np.ndarray:
    """QFT without the final qubit reversal: for j = n-1 .. 0, H on j followed
    by controlled phases 2 pi / 2^(j-k+1) controlled by each k < j.
    On |x> it yields sum_y e^{2 pi i x y / 2^n} |rev(y)> / sqrt(2^n), where
    rev reverses the n bits of y."""
    recs = []
    for j in range(n - 1, -1, -1):
        recs.append((KIND_U, j, -1, H))
        for k in range(j - 1, -1, -1):
            recs.append((KIND_CU, k, j, phase(2.0 * math.pi / 2 ** (j - k + 1))))
    return make_gates(recs)


def ghz_circuit(n: int) -> np.ndarray:
    recs = [(KIND_U, 0, -1, H)]
    for q in range(1, n):
        recs.append((KIND_CX, q - 1, q, None))
    return make_gates(recs)


def mixed_circuit(n: int, n_gates: int, seed: int) -> np.ndarray:
    """Every supported gate kind on random qubits: Haar U, diagonal U, CX, CZ,
    controlled Haar U and controlled phase. Used to cover all code paths."""
    rng = _rng(seed, n, n_gates, 7)
    recs = []
    for _ in range(n_gates):
        r = rng.integers(6)
        if r == 0 or n == 1:
            recs.append((KIND_U, int(rng.integers(n)), -1, haar_u2(rng)))
            continue
        a, b = (int(v) for v in rng.choice(n, size=2, replace=False))
        if r == 1:
            recs.append((KIND_U, a, -1, np.diag(np.exp(1j * rng.uniform(0, 6.283, 2)))))
        elif r == 2:
            recs.append((KIND_CX, a, b, None))
        elif r == 3:
            recs.append((KIND_CZ, a, b, None))
        elif r == 4:
            recs.append((KIND_CU, a, b, haar_u2(rng)))
        else:
            recs.append((KIND_CU, a, b, phase(rng.uniform(0, 6.283))))
    return make_gates(recs)


def sample_indices(n: int, count: int, seed: int) -> np.ndarray:
    """``count`` distinct basis indices uniform in [0, 2^n), sorted."""
    count = min(count, 1 << n)
    rng = _rng(seed, n, count, 11)
    idx = rng.choice(1 << n, size=count, replace=False)
    return np.sort(idx.astype(np.uint64))


# Workload configurations (seeded, synthetic).
CONFIGS = {
    1: dict(n=16, layers=20, cz_every_third=False, dtype="c128", samples=0),
    2: dict(n=30, layers=40, cz_every_third=True, dtype="c128", samples=1024),
    3: dict(n=32, layers=50, cz_every_third=True, dtype="c64", samples=1024),
}


def config_circuit(cfg: int, n: int | None = None, layers: int | None = None) -> np.ndarray:
    c = CONFIGS[cfg]
    return layered_circuit(n or c["n"], layers or c["layers"], MASTER_SEED + cfg,
                           c["cz_every_third"])


def config_samples(cfg: int, n: int | None = None, count: int | None = None) -> np.ndarray:
    c = CONFIGS[cfg]
    return sample_indices(n or c["n"], count or c["samples"], MASTER_SEED + cfg)


def batch_workload(count: int = 256, n_lo: int = 10, n_hi: int = 24, d_lo: int = 10,
                   d_hi: int = 60, seed: int = MASTER_SEED + 4):
    """Independent layered circuits with qubit count and depth drawn uniformly
    (inclusive bounds). Returns a list of (n, depth, gates)."""
    rng = _rng(seed, count)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ds = rng.integers(d_lo, d_hi + 1, size=count)
    return [(int(ns[i]), int(ds[i]), layered_circuit(int(ns[i]), int(ds[i]), seed * 1000 + i))
            for i in range(count)]


def request_trace(count: int = 1000, rate: float = 200.0, n_lo: int = 12, n_hi: int = 30,
                  d_lo: int = 20, d_hi: int = 100, samples: int = 16,
                  seed: int = MASTER_SEED + 5):
    """Finite Poisson arrival trace. Each request: arrival time (s), n, depth,
    the circuit seed and its sampled basis indices. Circuits are generated
    lazily by the caller with ``layered_circuit(n, depth, circuit_seed)``."""
    rng = _rng(seed, count, int(rate * 1000))
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ds = rng.integers(d_lo, d_hi + 1, size=count)
    reqs = []
    for i in range(count):
        cseed = seed * 1000 + i
        reqs.append(dict(id=i, arrival=float(t[i]), n=int(ns[i]), depth=int(ds[i]),
                         seed=cseed, samples=sample_indices(int(ns[i]), samples, cseed)))
    return reqs
