"""Serving form: continuous batching of resident requests.  Each request's
results are the same alone and in the mix (complex64 tolerance), and match the
oracle; the memory budget bounds what is resident."""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import layered_circuit, request_trace, sample_indices

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2010_09746_amd import qsim as Q  # noqa: E402
from paper_2010_09746_amd.serving import Server, latency_summary  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _requests(count, n_lo, n_hi, d_lo, d_hi, seed, spacing=0.0):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.integers(d_lo, d_hi + 1))
        out.append(dict(id=i, arrival=i * spacing, n=n, gates=layered_circuit(n, d, seed=seed * 1000 + i),
                        samples=sample_indices(n, 16, seed * 1000 + i)))
    return out


def test_results_same_alone_and_in_the_mix():
    _say("serving: mix vs alone")
    reqs = _requests(24, 12, 17, 3, 10, seed=3)
    srv = Server("c64", k_tile=10, max_swaps=8, pinned=3, reg_bits=3, max_slots=64)
    res, rec = srv.serve(reqs, realtime=False)
    assert srv.last_stats["max_resident"] > 1  # work did overlap
    for r in reqs:
        n, g = r["n"], r["gates"]
        st = Q.State(n, "c64").run(g, form="pass", k_tile=10, max_swaps=8, pinned=3, perm_exec="relabel",
                                   reg_bits=3)
        alone_z, alone_a = st.expect_z(), st.amplitudes(r["samples"])
        mix = res[r["id"]]
        assert np.abs(mix["z"] - alone_z).max() <= 1e-6
        assert np.abs(mix["amps"] - alone_a).max() <= 1e-6
        ref = O.run(g, n)
        assert np.abs(mix["z"] - O.expect_z(ref, n)).max() <= 1e-5
        assert np.abs(mix["amps"] - ref[np.asarray(r["samples"], dtype=np.int64)]).max() <= 1e-5
        assert abs(mix["norm"] - 1) <= 1e-5
        st.close()
    srv.close()


def test_large_requests_in_their_own_launch():
    """Requests whose passes have at least the solo threshold of tiles run
    each pass as a tile-pass launch of their own inside the step; the results
    are those of the shared launch (complex64 tolerance) and of the oracle."""
    _say("serving: solo launches for large requests")
    reqs = _requests(12, 12, 17, 3, 8, seed=5)
    out = {}
    for solo in (0, 32):  # 0: all passes in the shared launch; 32: n >= 15 alone
        srv = Server("c64", k_tile=10, max_swaps=8, pinned=3, reg_bits=3, max_slots=64, solo_tiles=solo)
        res, _ = srv.serve(reqs, realtime=False)
        out[solo] = res
        srv.close()
    assert any(r["n"] >= 15 for r in reqs) and any(r["n"] < 15 for r in reqs)
    for r in reqs:
        a, b = out[0][r["id"]], out[32][r["id"]]
        assert np.abs(a["z"] - b["z"]).max() <= 1e-6
        assert np.abs(a["amps"] - b["amps"]).max() <= 1e-6
        ref = O.run(r["gates"], r["n"])
        assert np.abs(b["z"] - O.expect_z(ref, r["n"])).max() <= 1e-5
        assert np.abs(b["amps"] - ref[np.asarray(r["samples"], dtype=np.int64)]).max() <= 1e-5
    with pytest.raises(Q.QsimError):
        srv = Server("c64", k_tile=10, solo_tiles=-1)


def test_budget_bounds_resident_states():
    _say("serving: budget")
    reqs = _requests(10, 16, 16, 4, 6, seed=4)
    budget = 2 * (8 << 16)  # two 16-qubit complex64 states
    srv = Server("c64", k_tile=10, max_swaps=8, hbm_budget=budget, max_slots=8)
    res, rec = srv.serve(reqs, realtime=False)
    assert srv.last_stats["max_resident"] <= 2
    assert len(res) == len(reqs)
    # a state beyond the budget is refused with QS_ERR_BUDGET
    assert not Q.qs_server_fits(srv.h, 18)
    big = torch.empty(8 << 17, dtype=torch.uint8, device="cuda")
    p = srv.compile(layered_circuit(17, 2, seed=1), 17)
    with pytest.raises(Q.QsimError) as e:
        for _ in range(3):
            Q.qs_server_admit(srv.h, p.h, big.data_ptr(), big.numel(), [])
    assert e.value.code == -3
    srv.close()


def test_realtime_trace_latencies():
    _say("serving: realtime trace")
    trace = request_trace(count=40, rate=400.0, n_lo=12, n_hi=18, d_lo=5, d_hi=12)
    reqs = [dict(r, gates=layered_circuit(r["n"], r["depth"], r["seed"])) for r in trace]
    srv = Server("c64", k_tile=10, max_swaps=16, max_slots=32)
    res, rec = srv.serve(reqs, realtime=True)
    s = latency_summary(rec)
    assert s["requests"] == 40 and 0 < s["p50_s"] <= s["p99_s"]
    for r in reqs[::7]:
        ref = O.run(r["gates"], r["n"])
        assert np.abs(res[r["id"]]["z"] - O.expect_z(ref, r["n"])).max() <= 1e-5
    srv.close()


@pytest.mark.parametrize("dt,k", [("c128", 11), ("c64", 12)])
def test_default_register_shape_at_large_tiles(dt, k):
    """With reg_bits = 0 the server and the compiled programs take the same
    register shape (16 amplitudes per thread here); results match the oracle."""
    _say(f"serving: default shape {dt} k={k}")
    reqs = _requests(6, k, k + 3, 3, 8, seed=11)
    srv = Server(dt, k_tile=k, max_swaps=8, pinned=3, max_slots=16)
    res, _ = srv.serve(reqs, realtime=False)
    tol = 1e-12 if dt == "c128" else 1e-5
    for r in reqs:
        n, g = r["n"], r["gates"]
        ref = O.run(g, n)
        mix = res[r["id"]]
        assert np.abs(mix["z"] - O.expect_z(ref, n)).max() <= tol
        assert np.abs(mix["amps"] - ref[np.asarray(r["samples"], dtype=np.int64)]).max() <= tol
    srv.close()
