"""Uncontrolled one-qubit gates applied on the lowest thread bits of a tile
layout through lane exchanges (OP_LANE, DPP moves) instead of a register
re-layout: every thread bit 0..3, both placements of the choice (only when a
re-layout can be put off, or whenever ready), both precisions, against the
oracle and the default lowering."""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import layered_circuit, mixed_circuit

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
@pytest.mark.parametrize("lanes,eager,circuit", [(2, True, "layered"), (4, True, "layered"), (4, False, "layered"),
                                                 (4, True, "mixed")])
@pytest.mark.parametrize("full", [False, True])
def test_lane_gates_match_oracle(dt, lanes, eager, circuit, full):
    """On 15 qubits with 2^11-amplitude tiles the eager 4-bit case puts 9-16
    gates on each of thread bits 0..3 of the layered workload (counted on the
    host), the 2-bit case 8 and 16 on bits 0 and 1."""
    n = 15
    _say(f"lane gates {dt} bits={lanes} eager={eager} {circuit} full={full}")
    g = layered_circuit(n, 20, 31) if circuit == "layered" else mixed_circuit(n, 600, seed=125)
    opts = dict(form="pass", k_tile=11, max_swaps=4, pinned=3, perm_exec="relabel", lane_gates=lanes,
                lane_eager=eager, full_matrices=full)
    P = Q.Program(g, n, dt, **opts)
    c = P.op_counts()
    P.close()
    if eager:
        assert c["lane"] >= 10
    ref = O.run(g, n)
    got = _run(g, n, dt, **opts)
    assert np.abs(got - ref).max() <= TOL[dt]
