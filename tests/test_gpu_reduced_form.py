"""The reduced one-qubit update (each uncontrolled gate as e^{i phi}
diag(1, e^{i theta}) W with the phases kept pending on the qubit) against the
whole-matrix form and the oracle, on every path that has to settle a pending
phase: CNOT and controlled-gate targets inside a pass, targets whose W ended
an earlier pass, gates run as launches of their own (fusion without the pass,
and the fallback of Algorithm 1 when no exchange is allowed), non-unitary
matrices (applied whole), and the last gate of each qubit (which carries the
accumulated scalar)."""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import KIND_CU, KIND_U, haar_u2, layered_circuit, make_gates, mixed_circuit

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
    assert c["w"] > 0 and cf["w"] == 0 and cf["phase"] == 0
    ref = O.run(g, n)
    a = _run(g, n, dt, **opts)
    b = _run(g, n, dt, full_matrices=True, **opts)
    assert np.abs(a - ref).max() <= TOL[dt]
    assert np.abs(b - ref).max() <= TOL[dt]


def test_pending_phase_settled_across_passes():
    """Small tiles and bundles of one exchange: many CNOT targets meet a
    pending phase left by a W of an earlier pass (applied as a phase of its
    own)."""
    n = 14
    _say("pending phases across passes")
    g = layered_circuit(n, 30, seed=77)
    opts = dict(form="pass", k_tile=8, max_swaps=1, pinned=3, perm_exec="relabel")
    P = Q.Program(g, n, "c128", **opts)
    assert P.op_counts()["phase"] > 0
    P.close()
    assert np.abs(_run(g, n, "c128", **opts) - O.run(g, n)).max() <= 1e-12


@pytest.mark.parametrize("r,pinned", [(0, 0), (2, 9)])
def test_launches_of_their_own_settle_phases(r, pinned):
    """r = 0 (fusion without the pass) and pinned = k (no exchange allowed, so
    Algorithm 1's fallback applies non-local gates as launches of their own):
    one-qubit launches absorb the pending phase, CNOT and controlled-gate
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


def test_non_unitary_matrices_applied_whole():
    """A matrix that is not unitary cannot be factored; it is applied whole
    (with the pending phase absorbed) and the oracle's literal product is
    reproduced."""
    n = 12
    _say("non-unitary matrices")
    rng = np.random.default_rng(3)
    recs = []
    for layer in range(6):
        for q in range(n):
            m = haar_u2(rng)
            if (q + layer) % 5 == 0:
                m = 0.9 * m  # not unitary
            recs.append((KIND_U, q, -1, m))
        for q in range(0, n - 1, 2):
            recs.append((KIND_CU, q, q + 1, haar_u2(rng)))
    g = make_gates(recs)
    assert np.abs(_run(g, n, "c128", form="pass", k_tile=9, max_swaps=4) - O.run(g, n)).max() <= 1e-12
