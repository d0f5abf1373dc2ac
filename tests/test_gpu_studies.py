"""Second workloads on the device: the QFT (closed form), the QFT-like
circuit of Appendix C and the paper's random family of Section 4, all through
the permutation pass, plus the measurement studies that bench.py reports."""

import math

import numpy as np
import pytest

import oracle as O
from workloads import paper_random_circuit, qft_circuit, qft_like_circuit, sample_indices

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2010_09746_amd import qsim as Q  # noqa: E402
from paper_2010_09746_amd import studies  # noqa: E402


def _rev(y, n):
    r = 0
    for b in range(n):
        r |= ((y >> b) & 1) << (n - 1 - b)
    return r


@pytest.mark.parametrize("n,k", [(14, 8), (18, 10), (20, 12)])
def test_qft_pass_matches_closed_form(n, k):
    x = (0x5DEECE66D * n) % (1 << n)
    st = Q.State(n, "c128")
    st.set_basis(x)
    st.run(qft_circuit(n), form="pass", k_tile=k, max_swaps=4, pinned=3, perm_exec="relabel")
    a = st.to_numpy()
    N = 1 << n
    y = np.arange(N)
    want = np.empty(N, dtype=np.complex128)
    rev = np.array([_rev(int(v), n) for v in y])
    want[rev] = np.exp(2j * math.pi * ((x * y) % N) / N) / math.sqrt(N)
    assert np.abs(a - want).max() < 1e-12
    st.close()


@pytest.mark.parametrize("dt,tol", [("c128", 1e-12), ("c64", 1e-5)])
def test_qft_like_pass_matches_oracle(dt, tol):
    n = 14
    g = qft_like_circuit(n)
    st = Q.State(n, dt)
    st.run(g, form="pass", k_tile=8, max_swaps=1, pinned=0, perm_exec="move")
    assert np.abs(st.to_numpy() - O.run(g, n)).max() < tol
    st.close()


@pytest.mark.parametrize("p", [0.0, 0.3, 1.0])
def test_random_family_pass_matches_oracle(p):
    n = 15
    g = paper_random_circuit(n, 30 * n, p, 20100946 + 8)
    ref = O.run(g, n)
    for opts in (dict(form="plain"), dict(form="pass", k_tile=9, max_swaps=8, pinned=3, perm_exec="relabel"),
                 dict(form="pass", k_tile=9, max_swaps=1, pinned=0, perm_exec="move")):
        st = Q.State(n, "c128")
        st.run(g, **opts)
        assert np.abs(st.to_numpy() - ref).max() < 1e-12, opts
        st.close()


def test_qft_study_small():
    r = studies.qft_study(n=18, k=10, r=4, samples=256, reps=1)
    assert r["qft"]["max_abs_error_vs_closed_form"] < 1e-12
    assert r["qft"]["n_global"] == 0 and r["qft_like"]["n_global"] == 0
    # Appendix C: at most 2 (n - k) permutations for the QFT-like circuit
    assert r["qft_like"]["n_perm"] <= 2 * (18 - 10)
    assert abs(r["qft_like"]["norm"] - 1.0) < 1e-12


def test_random_family_study_small():
    r = studies.random_family_study(n=16, ps=(0.0, 0.5), k=9, r=4)
    for row in r["rows"]:
        assert row["plain_ms"] > 0 and row["pass_ms"] > 0 and row["n_tile_passes"] >= 1
    # with p = 0 only single-qubit gates: exactly n - k permutations with r = 1
    # would be the paper's count; with r > 1 the pass needs at most that many
    assert r["rows"][0]["n_perm"] <= 16 - 9


def test_kernel_sweep_small():
    r = studies.kernel_sweep(n=20, reps=1)
    assert len(r["plain_u_per_target"]) == 20
    assert all(x["gbs"] > 0 for x in r["plain_u_per_target"])
    assert [m["pairs"] for m in r["permute"]] == list(range(1, 9))
    assert [x["gates"] for x in r["tile_pass_by_gates"]] == [1, 2, 4, 8, 12, 16, 24, 32, 48] * 2
    assert {x["k"] for x in r["tile_pass_by_gates"]} == {12, 13}
    assert all(x["gbs"] > 0 for x in r["tile_pass_by_gates"])
    assert r["zsum"]["launches"] == 1


def test_ablation_study_small():
    r = studies.ablation_study(n=16, layers=8, ks=(10, 14), k_ref=10, r=8)
    rows = {x["variant"]: x for x in r["rows"]}
    lane = {k for k in rows if "lane gates" in k}
    assert set(rows) - lane == {"fusion without pass", "Algorithm 1 (r=1), moved", "r=1, 3 pinned, relabelled",
                                "pass r=8 k=10", "pass r=8 k=14"}
    assert len(lane) == 3 and all(rows[k]["opts"]["k_tile"] == 10 for k in lane)
    assert max(rows[k]["lane_gates"] for k in lane) > 0
    nopass = rows["fusion without pass"]
    assert nopass["n_perm"] == 0 and nopass["n_global"] > 0 and nopass["n_plain"] == nopass["n_global"]
    alg1 = rows["Algorithm 1 (r=1), moved"]
    assert alg1["n_perm"] > 0 and alg1["n_global"] == 0
    assert rows["pass r=8 k=14"]["n_tile_passes"] >= 1
    assert all(x["ms"] > 0 for x in r["rows"])
