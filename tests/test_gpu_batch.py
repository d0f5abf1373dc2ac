"""Batching form: many uneven circuits in one persistent launch (HIP graph
replay), each with its own tile size.  Every circuit's read-out must equal
its solo run and the oracle."""

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
    """Seeded layered circuits of n_lo..n_hi qubits and 2..11 layers."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.integers(2, 12))
        out.append((n, layered_circuit(n, d, seed=seed * 100 + i)))
    return out


@pytest.mark.parametrize("dt,tol", [("c128", 1e-12), ("c64", 1e-5)])
@pytest.mark.parametrize("k,r,chunk", [(12, 8, 4), (10, 4, 1), (9, 2, 3)])
def test_batch_matches_oracle(dt, tol, k, r, chunk):
    _say(f"batch vs oracle {dt} k={k} r={r} chunk={chunk}")
    circ = _small_batch(n_lo=9)
    b = Q.Batch(circ, dt, k_tile=k, max_swaps=r, wg_per_cu=4, chunk=chunk)
    z, nrm = b.run().results()
    for c, (n, g) in enumerate(circ):
        ref = O.run(g, n)
        assert abs(z[c] - O.expect_z(ref, n)[0]) <= tol
        assert abs(nrm[c] - 1.0) <= tol
        if c < 5:
            assert np.abs(b.state(c) - ref).max() <= tol
    b.close()


def test_batch_all_gate_kinds_c128():
    _say("batch all gate kinds")
    circ = [(n, mixed_circuit(n, 120, seed=n)) for n in (9, 10, 11, 12, 13, 14)]
    b = Q.Batch(circ, "c128", k_tile=10, max_swaps=3, wg_per_cu=2, chunk=2)
    b.run()
    b.results()
    for c, (n, g) in enumerate(circ):
        assert np.abs(b.state(c) - O.run(g, n)).max() <= 1e-12
    b.close()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_batch_equals_solo_runs(dt):
    """Each circuit's batch result equals the same program run alone through
    the single-state path (tile of min(n, k) qubits, 256 threads): the same
    operations in the same order."""
    _say(f"batch vs solo {dt}")
    K, r = 11, 8
    circ = _small_batch(seed=5, count=10, n_lo=9, n_hi=17)
    b = Q.Batch(circ, dt, k_tile=K, max_swaps=r, pinned=3, wg_per_cu=4, chunk=8)
    z, nrm = b.run().results()
    for c, (n, g) in enumerate(circ):
        k = min(n, K)
        st = Q.State(n, dt).run(g, form="pass", k_tile=k, max_swaps=r, pinned=3, perm_exec="relabel",
                                reg_bits=k - 8)
        assert np.abs(b.state(c) - st.to_numpy()).max() <= (1e-14 if dt == "c128" else 1e-6)
        assert abs(z[c] - st.expect_z()[0]) <= 1e-12
        assert abs(nrm[c] - st.norm()) <= 1e-12
        st.close()
    b.close()


def test_graph_replays_are_identical():
    """Several replays of the captured graph, with unrelated eager device work
    and synchronizations between them, each give the eager result."""
    _say("graph replays")
    circ = _small_batch(seed=9, count=16, n_lo=9, n_hi=17)
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


def test_whole_state_circuits():
    """Circuits of at most k_tile qubits run as one tile in one pass (the whole
    state in one workgroup), mixed with larger ones."""
    _say("batch whole-state circuits")
    circ = [(n, layered_circuit(n, 20, seed=40 + n)) for n in (9, 10, 11, 12, 12, 11, 16)]
    passes, _ = Q.qs_batch_plan(circ, "c64", Q.make_batch_opts(k_tile=12, max_swaps=8))
    assert sum(1 for p in passes if p["circuit"] < 6) == 6
    b = Q.Batch(circ, "c64", k_tile=12, max_swaps=8, chunk=1)
    z, nrm = b.run().results()
    for c, (n, g) in enumerate(circ):
        ref = O.run(g, n)
        assert np.abs(b.state(c) - ref).max() <= 1e-5
        assert abs(z[c] - O.expect_z(ref, n)[0]) <= 1e-5
    b.close()


def test_wait_that_gives_up_is_reported():
    """wait_ms = -1 makes every dependency wait give up at once: the launch
    still drains and the run reports QS_ERR_HIP; a second run reports it again,
    and a batch with the default bound afterwards is correct."""
    _say("batch wait give-up")
    circ = _small_batch(seed=3, count=6, n_lo=13, n_hi=15)
    b = Q.Batch(circ, "c64", k_tile=10, max_swaps=2, wait_ms=-1)
    for _ in range(2):
        with pytest.raises(Q.QsimError) as e:
            b.run().results()
        assert e.value.code == -4 and "waited" in str(e.value)
    b.close()
    b = Q.Batch(circ, "c64", k_tile=10, max_swaps=2)
    z, nrm = b.run().results()
    for c, (n, g) in enumerate(circ):
        assert abs(z[c] - O.expect_z(O.run(g, n), n)[0]) <= 1e-5
    b.close()


def test_batch_workload_shape_subset():
    """A slice of the 256-circuit workload (uneven sizes up to 20 qubits)."""
    _say("batch workload slice")
    wl = [(n, g) for n, d, g in batch_workload(count=256) if n <= 20][:40]
    b = Q.Batch(wl, "c64", k_tile=12, max_swaps=16, pinned=4, wg_per_cu=4, chunk=4)
    z, nrm = b.run().results()
    assert np.abs(nrm - 1).max() <= 1e-5
    for c in range(0, len(wl), 9):
        n, g = wl[c]
        assert abs(z[c] - O.expect_z(O.run(g, n), n)[0]) <= 1e-5
    b.close()


def test_batch_rejects_small_circuits():
    with pytest.raises(Q.QsimError):
        Q.Batch([(8, layered_circuit(8, 2, seed=1))], "c64", k_tile=10)
