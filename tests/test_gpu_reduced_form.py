"""The reduced one-qubit update (each uncontrolled gate M of a tile pass as
two in-place shears L(q) U(p) with a left factor kept pending on the qubit:
M00 diag(1, z), M00 moved into one scalar, or a I + b X when the qubit's next
operations are CNOT targets) against the whole-matrix form and the oracle, on
every path that has to settle a pending factor: controlled-gate targets
inside a pass, targets whose shears ended an earlier pass, gates run as
launches of their own (fusion without the pass, and the fallback of
Algorithm 1 when no exchange is allowed), gates whose larger first-row entry
is off the diagonal (an exchange first), singular and non-unitary matrices,
long programs whose scalar has to be taken by a whole gate, and the last gate
of each qubit; and the a I + b X form through CNOT and span{I, X} targets."""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import KIND_CU, KIND_CX, KIND_U, haar_u2, layered_circuit, make_gates, mixed_circuit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2010_09746_amd import qsim as Q  # noqa: E402

TOL = {"c128": 1e-12, "c64": 1e-5}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(g, n, dt, **opts):
    st = Q.State(n, dt)
    st.run(g, **opts)
    v = st.to_numpy()
    st.close()
    return v


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("k,r,pinned,perm_exec", [(10, 4, 3, "relabel"), (9, 1, 0, "move"), (12, 16, 3, "relabel")])
def test_reduced_equals_whole_matrices_and_oracle(dt, k, r, pinned, perm_exec):
    n = 15
    _say(f"reduced form {dt} k={k} r={r}")
    g = mixed_circuit(n, 500, seed=40 + k)
    opts = dict(form="pass", k_tile=k, max_swaps=r, pinned=pinned, perm_exec=perm_exec)
    P = Q.Program(g, n, dt, **opts)
    c = P.op_counts()
    P.close()
    Pf = Q.Program(g, n, dt, full_matrices=True, **opts)
    cf = Pf.op_counts()
    Pf.close()
    assert c["shear"] > 0 and cf["shear"] == 0 and cf["phase"] == 0
    ref = O.run(g, n)
    a = _run(g, n, dt, **opts)
    b = _run(g, n, dt, full_matrices=True, **opts)
    assert np.abs(a - ref).max() <= TOL[dt]
    assert np.abs(b - ref).max() <= TOL[dt]


def _layers(n, layers, seed, two_qubit):
    """Haar U(2) on every qubit, then two_qubit(rng, c, t, layer) on a random
    perfect matching, per layer."""
    rng = np.random.default_rng(seed)
    recs = []
    for layer in range(layers):
        for q in range(n):
            recs.append((KIND_U, q, -1, haar_u2(rng)))
        perm = rng.permutation(n)
        for i in range(0, n - 1, 2):
            recs.extend(two_qubit(rng, int(perm[i]), int(perm[i + 1]), layer))
    return recs


def test_pending_phase_settled_across_passes():
    """Small tiles and bundles of one exchange: controlled Haar gates' targets
    meet a pending diagonal left by shears of an earlier pass (applied on its
    own)."""
    n = 14
    _say("pending phases across passes")
    g = make_gates(_layers(n, 30, 77, lambda rng, c, t, layer: [(KIND_CU, c, t, haar_u2(rng))]))
    opts = dict(form="pass", k_tile=8, max_swaps=1, pinned=3, perm_exec="relabel")
    P = Q.Program(g, n, "c128", **opts)
    assert P.op_counts()["phase"] > 50
    P.close()
    assert np.abs(_run(g, n, "c128", **opts) - O.run(g, n)).max() <= 1e-12


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_pending_factor_commuting_with_cnot_targets(dt):
    """complex128: a qubit whose next operations are CNOT targets (or targets
    of controlled gates in span{I, X}) keeps a I + b X pending: it commutes
    with them, so no pending factor is applied on its own.  Exchange gates on
    the targets absorb it; such a gate commutes with the CNOT target before it
    and may be scheduled first, and the target then meets the exchange gate's
    own diagonal factor (applied on its own).  complex64 keeps diagonal
    factors only (their phases are applied before the targets).  Against the
    oracle and the whole-matrix form."""
    n = 14
    _say(f"a I + b X pending factors {dt}")
    X = np.array([[0, 1], [1, 0]], dtype=complex)

    def circuit(exchanges):
        def two(rng, c, t, layer):
            out = []
            if layer % 3 == 2:
                th = rng.uniform(0, 6.283)
                out.append((KIND_CU, c, t, np.array([[np.cos(th), 1j * np.sin(th)], [1j * np.sin(th), np.cos(th)]])))
            else:
                out.append((KIND_CX, c, t, None))
            if exchanges and layer % 5 == 4:
                out.append((KIND_U, t, -1, X))
            return out
        return make_gates(_layers(n, 24, 11, two))

    opts = dict(form="pass", k_tile=10, max_swaps=8, pinned=3, perm_exec="relabel")
    counts = {}
    for ex in (False, True):
        P = Q.Program(circuit(ex), n, dt, **opts)
        counts[ex] = P.op_counts()
        P.close()
    g = circuit(True)
    n_u = int(sum(1 for k in g["kind"] if k == KIND_U))
    n_x = int(sum(1 for i in range(len(g)) if g["kind"][i] == KIND_U and g["u"][i][0] == 0 and g["u"][i][1] == 0))
    if dt == "c128":
        assert counts[False]["phase"] == 0
        assert counts[True]["phase"] <= n_x and counts[True]["shear"] > 0.8 * (n_u - n_x)
    else:
        assert counts[False]["phase"] > n_x and counts[True]["shear"] > 0.8 * (n_u - n_x)
    ref = O.run(g, n)
    a = _run(g, n, dt, **opts)
    b = _run(g, n, dt, full_matrices=True, **opts)
    assert np.abs(a - ref).max() <= TOL[dt]
    assert np.abs(b - ref).max() <= TOL[dt]
    if dt == "c64":
        fid = abs(np.vdot(ref, a)) ** 2 / np.vdot(a, a).real
        assert 1 - fid <= 1e-6


def test_complex64_x_factors_on_request():
    """complex64 with QS_OPT_X_FACTORS keeps a I + b X factors: no phase
    operation before CNOT targets, within the complex64 bounds against the
    oracle (its rounding errors are larger than with diagonal factors)."""
    n = 16
    _say("complex64 with a I + b X factors")
    g = layered_circuit(n, 20, seed=13)
    opts = dict(form="pass", k_tile=11, max_swaps=8, pinned=4, perm_exec="relabel")
    P = Q.Program(g, n, "c64", **opts)
    diag_only = P.op_counts()
    P.close()
    P = Q.Program(g, n, "c64", x_factors=True, **opts)
    with_x = P.op_counts()
    P.close()
    assert diag_only["phase"] > 0 and with_x["phase"] < diag_only["phase"] / 4
    ref = O.run(g, n)
    got = _run(g, n, "c64", x_factors=True, **opts)
    assert np.abs(got - ref).max() <= TOL["c64"]
    fid = abs(np.vdot(ref, got)) ** 2 / np.vdot(got, got).real
    assert 1 - fid <= 1e-6


@pytest.mark.parametrize("r,pinned", [(0, 0), (2, 9)])
def test_launches_of_their_own_settle_phases(r, pinned):
    """r = 0 (fusion without the pass) and pinned = k (no exchange allowed, so
    Algorithm 1's fallback applies non-local gates as launches of their own):
    one-qubit launches absorb the pending diagonal, CNOT and controlled-gate
    launches get it applied first."""
    n, k = 13, 9
    _say(f"own launches r={r} pinned={pinned}")
    g = mixed_circuit(n, 300, seed=5 + r)
    opts = dict(form="pass", k_tile=k, max_swaps=r, pinned=pinned)
    P = Q.Program(g, n, "c128", **opts)
    st = P.stats()
    P.close()
    assert st["n_plain"] > 0
    assert np.abs(_run(g, n, "c128", **opts) - O.run(g, n)).max() <= 1e-12


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_singular_non_unitary_and_off_diagonal_pivots(dt):
    """Non-unitary matrices are factored like unitary ones while their pending
    factors stay in bounds, and applied whole otherwise; a singular matrix
    (a projector) cannot be factored; near-exchanges put the larger
    first-row entry off the diagonal (an exchange runs first).  The oracle's
    literal products are reproduced."""
    n = 12
    _say(f"non-unitary, singular and off-diagonal pivots {dt}")
    rng = np.random.default_rng(3)
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    recs = []
    for layer in range(8):
        for q in range(n):
            m = haar_u2(rng)
            sel = (q + layer) % 6
            if sel == 0:
                m = 0.9 * m  # not unitary
            elif sel == 1:
                m = X @ np.diag([1.0, np.exp(0.3j * q)]) + 1e-3 * haar_u2(rng)  # near an exchange
            elif sel == 2 and layer % 4 == 1:
                m = np.array([[1, 0], [0, 0]], dtype=complex)  # projector: singular
            elif sel == 3:
                m = np.array([[1.0, 0.2], [0.1, 7.0]], dtype=complex)  # far from unitary
            recs.append((KIND_U, q, -1, m))
        for q in range(layer % 2, n - 1, 2):
            recs.append((KIND_CU, q, q + 1, haar_u2(rng)))
        recs.append((KIND_CX, (layer * 5) % n, (layer * 5 + 3) % n, None))
    g = make_gates(recs)
    ref = O.run(g, n)
    scale = max(1.0, np.abs(ref).max())
    got = _run(g, n, dt, form="pass", k_tile=9, max_swaps=4)
    assert np.abs(got - ref).max() <= TOL[dt] * scale


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_long_program_scalar_stays_bounded(dt):
    """400 layers on 12 qubits: without the bound the product of the pivots
    would leave complex64's range; a gate applied whole takes the scalar
    whenever its magnitude would leave [2^-8, 2^8]."""
    n = 12
    _say(f"long program {dt}")
    g = layered_circuit(n, 400, seed=91)
    opts = dict(form="pass", k_tile=10, max_swaps=4, pinned=3, perm_exec="relabel")
    P = Q.Program(g, n, dt, **opts)
    c = P.op_counts()
    P.close()
    n_u = int(sum(1 for k in g["kind"] if k == KIND_U))
    assert c["shear"] > 0.9 * n_u and c["u"] > n
    ref = O.run(g, n)
    got = _run(g, n, dt, **opts)
    assert np.abs(got - ref).max() <= TOL[dt]
    if dt == "c64":
        fid = abs(np.vdot(ref, got)) ** 2 / np.vdot(got, got).real
        assert 1 - fid <= 1e-6
