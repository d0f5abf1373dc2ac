"""<Z_q> folded into the last launch (qs_run_circuit_expect_z): when the last
launch is a tile pass over whole 128-byte lines, each tile writes its
per-position probability sums and a small kernel folds them; otherwise the
read-out pass runs after the last launch.  Against the oracle and against
qs_run_circuit followed by qs_expect_z, for the launch kinds a circuit can end
with, both precisions, runs from |0...0> and the pass deciding by measured
costs."""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import KIND_CX, KIND_CZ, KIND_U, haar_u2, layered_circuit, make_gates, mixed_circuit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2010_09746_amd import qsim as Q  # noqa: E402

TOL = {"c128": 1e-12, "c64": 1e-5}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _separate(g, n, dt, opts, costs=None):
    st = Q.State(n, dt)
    st.run(g, costs=costs, **opts)
    z = st.expect_z()
    st.close()
    return z


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("name,opts", [
    ("pass-relabel", dict(form="pass", k_tile=10, max_swaps=8, pinned=3, perm_exec="relabel")),
    ("pass-move", dict(form="pass", k_tile=9, max_swaps=1, pinned=0, perm_exec="move")),
    ("pass-from-zero", dict(form="pass", k_tile=11, max_swaps=4, pinned=3, perm_exec="relabel", from_zero=True)),
    ("pass-unpinned", dict(form="pass", k_tile=8, max_swaps=2, pinned=0, perm_exec="relabel")),
    ("plain", dict(form="plain")),
])
def test_fused_expect_z_matches_oracle_and_separate_readout(dt, name, opts):
    n = 15
    _say(f"fused read-out {dt} {name}")
    g = mixed_circuit(n, 500, seed=21)
    ref = O.expect_z(O.run(g, n), n)
    st = Q.State(n, dt)
    Q.qs_profile_read()
    Q.qs_profile_enable(True)
    z = st.run_expect_z(g, **opts)
    Q.qs_profile_enable(False)
    prof = Q.qs_profile_read()
    st.close()
    folded = prof.get("zfold", {}).get("launches", 0)
    passes = prof.get("zsum", {}).get("launches", 0)
    assert folded + passes == 1
    if name in ("pass-relabel", "pass-from-zero"):
        assert folded == 1  # the last tile pass covers whole lines: no read-out pass
    if name == "plain":
        assert passes == 1
    sep = _separate(g, n, dt, opts)
    assert np.abs(z - ref).max() <= TOL[dt]
    assert np.abs(z - sep).max() <= (1e-13 if dt == "c128" else 1e-6)


def _profiled_expect_z(st, g, **opts):
    Q.qs_profile_read()
    Q.qs_profile_enable(True)
    z = st.run_expect_z(g, **opts)
    Q.qs_profile_enable(False)
    prof = Q.qs_profile_read()
    return z, prof.get("zfold", {}).get("launches", 0), prof.get("zsum", {}).get("launches", 0)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_fused_expect_z_through_trailing_cnots(dt):
    """CNOTs run on their own after the last tile pass (targets outside the
    tile): each makes its target bit the XOR of two bits, folded from the
    pass's per-tile sums (a tile control, or two bits outside the tile); two
    tile bits XORed into one target need the read-out pass."""
    n = 14
    _say(f"fused read-out through trailing CNOTs {dt}")
    rng = np.random.default_rng(7)
    head = [(KIND_U, q, -1, haar_u2(rng)) for q in range(9)]
    head += [(KIND_CX, 0, 9, None), (KIND_CX, 1, 10, None)]
    head += [(KIND_U, q, -1, haar_u2(rng)) for q in range(9)]
    opts = dict(form="pass", k_tile=9, max_swaps=2, pinned=9)
    for tail, folds in (([(KIND_CX, 3, 13, None), (KIND_CX, 10, 12, None), (KIND_CZ, 2, 11, None)], True),
                        ([(KIND_CX, 3, 13, None), (KIND_CX, 4, 13, None)], False)):
        g = make_gates(head + tail)
        P = Q.Program(g, n, dt, **opts)
        ins = P.instructions()
        P.close()
        assert ins[-1][0] == "global" and ins[-2][0] == "global"
        st = Q.State(n, dt)
        z, folded, passes = _profiled_expect_z(st, g, **opts)
        st.close()
        assert (folded, passes) == ((1, 0) if folds else (0, 1))
        assert np.abs(z - O.expect_z(O.run(g, n), n)).max() <= TOL[dt]


def test_fused_expect_z_last_launch_kinds():
    """A circuit ending in a gate outside the tile (a launch of its own), an
    empty circuit (|0...0> from the start), the 24-qubit layered workload at
    the headline's launch configuration with measured costs, and two runs in
    a row on one state (the second reuses the read-out buffer)."""
    n, dt = 14, "c128"
    _say("fused read-out: last launch kinds")
    H = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
    g = make_gates([(KIND_U, q, -1, H) for q in range(n)] + [(KIND_CX, 0, 13, None), (KIND_U, 13, -1, H)])
    opts = dict(form="pass", k_tile=9, max_swaps=2, pinned=9)
    P = Q.Program(g, n, dt, **opts)
    assert P.instructions()[-1][0] == "global"
    P.close()
    st = Q.State(n, dt)
    z = st.run_expect_z(g, **opts)
    assert np.abs(z - O.expect_z(O.run(g, n), n)).max() <= 1e-12
    st.set_basis(5)
    z = st.run_expect_z(make_gates([]), from_zero=True, form="pass", k_tile=10)
    assert np.abs(z - 1.0).max() <= 1e-15
    st.close()

    n = 24
    g = layered_circuit(n, 12, 31)
    ref = O.expect_z(O.run(g, n), n)
    costs = Q.make_pass_costs(7.7, [0.08, 0.1, 0.11], 0.0, [6.0, 5.0, 3.4, 5.1])
    opts = dict(form="pass", k_tile=12, max_swaps=16, pinned=3, perm_exec="relabel", from_zero=True)
    st = Q.State(n, dt)
    for _ in range(2):
        z = st.run_expect_z(g, costs=costs, **opts)
        assert np.abs(z - ref).max() <= 1e-12
    st.close()
