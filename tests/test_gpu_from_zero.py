"""Runs from |0...0> (QS_OPT_FROM_ZERO): the first tile pass generates the
basis state in registers instead of reading the state; a first launch that is
not a tile pass (a one-gate launch, a data-moving permutation) gets the state
set first; an empty circuit leaves |0...0>.  Each starts from a state holding
another circuit's result and is compared with the oracle."""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import KIND_CX, KIND_U, layered_circuit, make_gates, mixed_circuit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2010_09746_amd import qsim as Q  # noqa: E402

TOL = {"c128": 1e-12, "c64": 1e-5}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dirty(st, n):
    # leave another circuit's (nonzero everywhere) result in the state
    st.set_basis(0)
    st.run(layered_circuit(n, 2, 5), form="plain")


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("opts", [
    dict(form="pass", k_tile=10, max_swaps=8, pinned=3, perm_exec="relabel"),
    dict(form="pass", k_tile=9, max_swaps=1, pinned=0, perm_exec="move"),
    dict(form="plain"),
], ids=["pass-relabel", "pass-move", "plain"])
def test_run_from_zero_matches_oracle(dt, opts):
    n = 14
    _say(f"from zero {dt} {opts}")
    g = mixed_circuit(n, 400, seed=17)
    ref = O.run(g, n)
    st = Q.State(n, dt)
    _dirty(st, n)
    st.run(g, from_zero=True, **opts)
    got = st.to_numpy()
    st.close()
    assert np.abs(got - ref).max() <= TOL[dt]


@pytest.mark.parametrize("noalloc", [False, True])
def test_program_from_zero_first_launch_kinds(noalloc):
    """Compiled programs keep the flag: one whose first launch is a tile pass,
    one whose first gate runs as a launch of its own (pinned = k: no exchange
    allowed) and an empty one; each run twice on a dirty state."""
    n, dt = 13, "c128"
    _say(f"program from zero noalloc={noalloc}")
    H = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
    # every gate waits for the first, which is outside the tile: a one-gate launch comes first
    first_global = make_gates([(KIND_U, 12, -1, H), (KIND_CX, 12, 0, None), (KIND_CX, 12, 1, None),
                               (KIND_U, 0, -1, H), (KIND_U, 1, -1, H)])
    cases = [(mixed_circuit(n, 300, seed=4), dict(k_tile=10, max_swaps=4, pinned=3, perm_exec="relabel")),
             (first_global, dict(k_tile=9, max_swaps=2, pinned=9)),
             (make_gates([]), dict(k_tile=10, max_swaps=4))]
    for g, o in cases:
        P = Q.Program(g, n, dt, form="pass", from_zero=True, **o)
        if len(g) == 5:
            assert P.instructions()[0][0] == "global"
        st = Q.State(n, dt)
        ref = O.run(g, n) if len(g) else np.eye(1 << n, 1, dtype=complex)[:, 0]
        for _ in range(2):
            _dirty(st, n)
            st.run_program(P, noalloc=noalloc)
            assert np.abs(st.to_numpy() - ref).max() <= 1e-12
        st.close()
        P.close()
