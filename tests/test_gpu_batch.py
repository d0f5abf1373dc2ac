"""Batching form: many uneven circuits in one persistent launch (HIP graph
replay).  Every circuit's read-out must equal its solo run and the oracle."""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import batch_workload, layered_circuit, mixed_circuit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2010_09746_amd import qsim as Q  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _small_batch(seed=1, count=12, n_lo=10, n_hi=16):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.integers(2, 12))
        out.append((n, layered_circuit(n, d, seed=seed * 100 + i)))
    return out


@pytest.mark.parametrize("dt,tol", [("c128", 1e-12), ("c64", 1e-5)])
@pytest.mark.parametrize("k,r,reg", [(10, 8, 0), (9, 4, 3), (8, 2, 2)])
def test_batch_matches_oracle(dt, tol, k, r, reg):
    _say(f"batch vs oracle {dt} k={k} r={r} reg={reg}")
    circ = _small_batch()
    b = Q.Batch(circ, dt, k_tile=k, max_swaps=r, reg_bits=reg, wg_per_cu=4, chunk=4)
    z, nrm = b.run().results()
    for c, (n, g) in enumerate(circ):
        ref = O.run(g, n)
        assert abs(z[c] - O.expect_z(ref, n)[0]) <= tol
        assert abs(nrm[c] - 1.0) <= tol
        if c < 4:
            assert np.abs(b.state(c) - ref).max() <= tol
    b.close()


def test_batch_all_gate_kinds_c128():
    _say("batch all gate kinds")
    circ = [(n, mixed_circuit(n, 120, seed=n)) for n in (10, 11, 12, 13, 14)]
    b = Q.Batch(circ, "c128", k_tile=10, max_swaps=3, wg_per_cu=2, chunk=2)
    b.run()
    b.results()
    for c, (n, g) in enumerate(circ):
        assert np.abs(b.state(c) - O.run(g, n)).max() <= 1e-12
    b.close()


def test_batch_equals_solo_runs():
    """The batch result of each circuit equals the same circuit run alone
    through the single-state path with the same options."""
    _say("batch vs solo")
    circ = _small_batch(seed=5, count=10, n_lo=10, n_hi=18)
    b = Q.Batch(circ, "c64", k_tile=10, max_swaps=8, pinned=3, wg_per_cu=8, chunk=8)
    z, nrm = b.run().results()
    for c, (n, g) in enumerate(circ):
        st = Q.State(n, "c64").run(g, form="pass", k_tile=10, max_swaps=8, pinned=3, perm_exec="relabel")
        if n <= 18:
            assert np.abs(b.state(c) - st.to_numpy()).max() <= 1e-6
        assert abs(z[c] - st.expect_z()[0]) <= 1e-12
        assert abs(nrm[c] - st.norm()) <= 1e-12
        st.close()
    b.close()


def test_graph_replays_are_identical():
    """Several replays of the captured graph, with unrelated eager device work
    and synchronizations between them, each give the eager result."""
    _say("graph replays")
    circ = _small_batch(seed=9, count=16, n_lo=10, n_hi=17)
    eager = Q.Batch(circ, "c64", k_tile=10, max_swaps=4, use_graph=0)
    z0, n0 = eager.run().results()
    eager.close()
    g = Q.Batch(circ, "c64", k_tile=10, max_swaps=4, use_graph=1)
    side = Q.State(12, "c128")
    for rep in range(4):
        z, nrm = g.run().results()
        assert np.array_equal(z, z0) and np.array_equal(nrm, n0), rep
        side.run(layered_circuit(12, 3, seed=rep), form="plain")
        side.synchronize()
    g.close()


@pytest.mark.parametrize("dt,tol", [("c64", 1e-5), ("c128", 1e-12)])
def test_large_passes_in_their_own_launches(dt, tol):
    """Passes of at least the solo threshold of tiles run as tile-pass
    launches of their own, in the captured graph and eagerly: the results are
    those of the level launches alone, replay after replay, and the oracle's."""
    _say(f"batch solo launches {dt}")
    circ = _small_batch(seed=11, count=14, n_lo=10, n_hi=17)
    assert any(n >= 15 for n, _ in circ) and any(n < 15 for n, _ in circ)
    base = Q.Batch(circ, dt, k_tile=10, max_swaps=4, wg_per_cu=4, chunk=4, use_graph=0, solo_tiles=0)
    z0, n0 = base.run().results()
    s0 = [base.state(c) for c in range(len(circ))]
    base.close()
    for graph in (0, 1):
        b = Q.Batch(circ, dt, k_tile=10, max_swaps=4, wg_per_cu=4, chunk=4, use_graph=graph)
        b.run().results()
        b.set_solo_tiles(32)  # circuits of 15 qubits and more: 32+ tiles of 2^10
        for rep in range(3):
            z, nrm = b.run().results()
            assert np.abs(z - z0).max() <= tol and np.abs(nrm - n0).max() <= tol, (graph, rep)
        for c, (n, g) in enumerate(circ):
            assert np.abs(b.state(c) - s0[c]).max() <= tol
            if c % 4 == 0:
                assert np.abs(b.state(c) - O.run(g, n)).max() <= tol
        b.set_solo_tiles(0)
        z, nrm = b.run().results()
        assert np.abs(z - z0).max() <= tol
        b.close()
    b = Q.Batch(circ[:2], dt, k_tile=10)
    with pytest.raises(Q.QsimError):
        b.set_solo_tiles(-1)
    b.close()


def test_batch_workload_shape_subset():
    """A slice of the 256-circuit workload (uneven sizes up to 20 qubits)."""
    _say("batch workload slice")
    wl = [(n, g) for n, d, g in batch_workload(count=256) if n <= 20][:40]
    b = Q.Batch(wl, "c64", k_tile=10, max_swaps=8, wg_per_cu=8, chunk=8)
    z, nrm = b.run().results()
    assert np.abs(nrm - 1).max() <= 1e-5
    for c in range(0, len(wl), 9):
        n, g = wl[c]
        assert abs(z[c] - O.expect_z(O.run(g, n), n)[0]) <= 1e-5
    b.close()


def test_batch_rejects_small_circuits():
    with pytest.raises(Q.QsimError):
        Q.Batch([(8, layered_circuit(8, 2, seed=1))], "c64", k_tile=10)
