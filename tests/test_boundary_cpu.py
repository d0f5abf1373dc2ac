"""CPU checks of the C boundary: the library loads and exports every entry
point the header declares, and the host-only compiler (the permutation pass of
Section 3) matches the oracle pass instruction by instruction."""

import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2010_09746_amd import qsim as Q
from workloads import (config_circuit, layered_circuit, make_gates, mixed_circuit, paper_random_circuit,
                       qft_like_circuit, haar_u2, KIND_CU, KIND_CX, KIND_CZ, KIND_U, H)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "qsim.h")).read()
    return sorted(set(re.findall(r"\b(qs_[a-z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert _declared() == sorted(Q.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = Q.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_noalloc_limit_agrees_with_header():
    txt = open(os.path.join(ROOT, "include", "qsim.h")).read()
    m = re.search(r"#define QS_NOALLOC_MAX_OPS (\d+)", txt)
    assert m and int(m.group(1)) == Q.NOALLOC_MAX_OPS


def test_reduced_one_qubit_form_counts():
    """By default uncontrolled one-qubit gates of tile passes are lowered to
    two shears (all but each qubit's last and the few whose pending factors
    would leave their bounds); with full_matrices every one is a whole 2x2
    and no pending diagonal is applied on its own."""
    g = config_circuit(2, n=20, layers=10)
    a = Q.Program(g, 20, "c128", form="pass", k_tile=12, max_swaps=16, perm_exec="relabel", pinned=3).op_counts()
    b = Q.Program(g, 20, "c128", form="pass", k_tile=12, max_swaps=16, perm_exec="relabel", pinned=3,
                  full_matrices=True).op_counts()
    n_u = int(sum(1 for k in g["kind"] if k == KIND_U))
    assert b["u"] == n_u and b["shear"] == 0 and b["phase"] == 0
    # every one-qubit gate is either two shears or whole; the last one of each qubit is whole
    assert a["shear"] + a["u"] == n_u and a["u"] >= 20 and a["shear"] > 4 * a["u"]
    # a qubit whose next two-qubit gate makes it a CNOT target keeps a I + b X
    # pending (it commutes with the target), one that acts as a control or in a
    # CZ keeps diag(1, z): no pending factor is applied on its own
    assert a["phase"] == 0


def test_gate_record_layout():
    assert Q.GATE_DTYPE.itemsize == 80
    assert Q.GATE_DTYPE.fields["u"][1] == 16


def _same_as_oracle(g, n, m, r=1, pinned=0):
    ref, _ = O.pass_ref(g, n, m, r=r, pinned=pinned)
    P = Q.Program(g, n, "c128", k_tile=m, max_swaps=r, pinned=pinned)
    ins = P.instructions()
    st = P.stats()
    P.close()
    assert ins == ref
    return st


@pytest.mark.parametrize("n,m,p,seed", [(8, 6, 0.3, 1), (12, 9, 0.0, 2), (16, 13, 1.0, 3), (20, 16, 0.3, 4),
                                        (30, 24, 0.3, 5), (50, 40, 0.3, 6)])
def test_pass_matches_oracle_paper_family(n, m, p, seed):
    _same_as_oracle(paper_random_circuit(n, 30 * n, p, seed), n, m)


@pytest.mark.parametrize("n,m,seed", [(7, 3, 1), (9, 5, 2), (12, 7, 3)])
def test_pass_matches_oracle_all_gate_kinds(n, m, seed):
    _same_as_oracle(mixed_circuit(n, 150, seed), n, m)


@pytest.mark.parametrize("r,pinned", [(2, 0), (4, 3), (8, 3), (1, 3)])
def test_pass_extensions_match_oracle(r, pinned):
    _same_as_oracle(layered_circuit(16, 12, seed=9), 16, 10, r=r, pinned=pinned)


@pytest.mark.parametrize("m,r,pinned,seed", [(5, 1, 0, 1), (6, 4, 2, 2), (7, 8, 3, 3)])
def test_pass_matches_oracle_repeated_gates(m, r, pinned, seed):
    """Gates from a small alphabet (a Haar U(2), H, X, a diagonal, CX, CZ, a
    controlled Haar U(2)) repeat often, so identical gates (which commute)
    follow each other on a qubit: the dependency graph may leave out an edge
    only where another path implies it."""
    n = 10
    rng = np.random.default_rng(seed)
    u = [haar_u2(rng) for _ in range(2)]
    one = [u[0], H, np.array([[0, 1], [1, 0]], dtype=complex), np.diag([1.0, np.exp(0.7j)])]
    recs = []
    for _ in range(400):
        a = int(rng.integers(0, 7))
        q = int(rng.integers(0, 3 if a % 2 else n))  # crowd a few qubits
        t = int((q + 1 + rng.integers(0, n - 1)) % n)
        if a < 4:
            recs.append((KIND_U, q, -1, one[a]))
        elif a == 4:
            recs.append((KIND_CX, q, t, None))
        elif a == 5:
            recs.append((KIND_CZ, q, t, None))
        else:
            recs.append((KIND_CU, q, t, u[1]))
    _same_as_oracle(make_gates(recs), n, m, r=r, pinned=pinned)


def test_pass_matches_oracle_layered_config_shape():
    # the 30-qubit, 40-layer circuit shape at tile size 12
    st = _same_as_oracle(config_circuit(2), 30, 12)
    assert st["n_gates"] == 1800 and st["n_global"] == 0


def test_pass_matches_oracle_qft_like():
    for n in (10, 20, 30):
        _same_as_oracle(qft_like_circuit(n), n, n - n // 5)


def test_program_stats_consistent():
    g = config_circuit(2)
    P = Q.Program(g, 30, "c128", k_tile=12, max_swaps=4)
    s = P.stats()
    assert s["n_apply"] + s["n_global"] == 1800
    assert s["n_tile_passes"] >= s["n_perm"]
    assert s["n_move_passes"] == s["n_perm"]
    P2 = Q.Program(g, 30, "c128", k_tile=12, max_swaps=4, perm_exec="relabel")
    assert P2.instructions() == P.instructions()
    assert P2.stats()["n_move_passes"] == 0
    plain = Q.Program(g, 30, "c128", form="plain")
    assert plain.stats()["n_plain"] == 1800


def test_compile_rejects_bad_input():
    g = make_gates([(KIND_CX, 0, 0, None)])
    with pytest.raises(Q.QsimError) as e:
        Q.Program(g, 4, "c128")
    assert e.value.code == -1
    g = make_gates([(KIND_U, 5, -1, H)])
    with pytest.raises(Q.QsimError):
        Q.Program(g, 4, "c128")
    with pytest.raises(Q.QsimError):
        Q.Program(make_gates([(KIND_U, 0, -1, H)]), 4, "c128", sigma0=[0, 1, 1, 2])
    with pytest.raises(Q.QsimError):
        Q.Program(make_gates([(KIND_U, 0, -1, H)]), 4, "c128", max_swaps=-1)
    bad = make_gates([(KIND_U, 0, -1, H)])
    bad[0]["kind"] = 9
    with pytest.raises(Q.QsimError):
        Q.Program(bad, 4, "c128")


def test_fusion_without_pass():
    """r = 0: no PermuteQubits; a gate runs in a tile pass exactly when its
    non-diagonal targets are among the first k positions (diagonal gates are
    local anywhere), else on its own, and the program still computes the plain
    result."""
    n, k = 10, 6
    g = mixed_circuit(n, 120, seed=7)
    P = Q.Program(g, n, "c128", k_tile=k, max_swaps=0)
    ins = P.instructions()
    st = P.stats()
    P.close()
    assert {t for t, _ in ins} <= {"apply", "global"} and st["n_perm"] == 0
    ref, _ = O.pass_ref(g, n, k, r=1)
    local = {v for t, v in ref if t == "apply"}
    for t, v in ins:
        kind, q0, q1, u = int(g[v]["kind"]), int(g[v]["q0"]), int(g[v]["q1"]), g[v]["u"]
        diagonal = kind == 2 or (kind != 1 and not np.any(u[2:6]))   # CZ, or U/CU with u01 = u10 = 0
        targets = [] if diagonal else ([q0] if kind == KIND_U else [q1])
        assert (t == "apply") == all(q < k for q in targets), (t, v)
    assert sorted(v for _, v in ins) == list(range(len(g)))
    v, sig = O.run_program(g, n, ins)
    assert np.abs(O.to_logical(v, n, sig) - O.run(g, n)).max() < 1e-13
    assert len(local) > sum(t == "apply" for t, _ in ins)  # the pass makes more gates local


def test_compile_with_start_placement():
    n = 10
    g = mixed_circuit(n, 80, seed=5)
    sigma0 = list(np.random.default_rng(2).permutation(n))
    P = Q.Program(g, n, "c128", sigma0=sigma0, k_tile=7)
    ins = P.instructions()
    v, sig = O.run_program(g, n, ins, sigma0=sigma0)
    assert np.abs(O.to_logical(v, n, sig) - O.run(g, n)).max() < 1e-13


def test_empty_circuit_compiles():
    P = Q.Program(np.zeros(0, dtype=Q.GATE_DTYPE), 8, "c64")
    assert P.stats()["n_gates"] == 0 and P.instructions() == []


def test_op_counts_classify_tile_work():
    """Work counts by class on the host: one pass, its U gates, exchanges by
    where their control lives, and weights for conditional operations."""
    n, k = 16, 10
    g = make_gates([(KIND_U, q, -1, H) for q in range(3)] +
                   [(KIND_CX, 15, 0, None)] +    # control outside the tile: half the tiles, a relabel
                   [(KIND_CX, 1, 2, None)])      # in-tile control
    P = Q.Program(g, n, "c128", form="pass", k_tile=k, max_swaps=1, pinned=0, perm_exec="relabel")
    c = P.op_counts()
    P.close()
    assert c["tile_pass"] == 1 and c["u"] == 3 and c["remap"] >= 1
    assert c["x_reg"] + c["x_lane"] == 1
    assert c["dispatch"] == 1.0          # 0.5 skipped + 0.5 relabel
    assert c["plain_u"] == 0 and c["move"] == 0
    Pp = Q.Program(g, n, "c128", form="plain")
    cp = Pp.op_counts()
    Pp.close()
    assert cp["plain_u"] == 3 and cp["plain_cx"] == 2 and cp["tile_pass"] == 0


def test_lane_gate_options():
    """Lane gates (uncontrolled one-qubit gates on the lowest thread bits run
    through lane exchanges instead of waiting for a re-layout): off by
    default; each one-qubit gate of the 30-qubit workload is still one
    operation (a shear, a whole gate or a lane gate); running them whenever
    ready saves re-layouts, more with four thread bits than with two; gates
    with controls never take the lane form; unknown flag bits are rejected."""
    g = config_circuit(2)
    n_u = int(np.sum(g["kind"] == KIND_U))
    base = dict(form="pass", k_tile=12, max_swaps=16, pinned=3, perm_exec="relabel")
    res = {}
    for lanes, eager in ((0, False), (4, False), (2, True), (4, True)):
        P = Q.Program(g, 30, "c128", lane_gates=lanes, lane_eager=eager, **base)
        res[(lanes, eager)] = (P.op_counts(), P.stats())
        P.close()
    for c, st in res.values():
        assert c["shear"] + c["u"] + c["lane"] == n_u
        assert st["n_tile_passes"] == 43
    assert res[(0, False)][0]["lane"] == 0
    assert 0 < res[(2, True)][0]["lane"] < res[(4, True)][0]["lane"]
    assert res[(4, True)][1]["n_remaps"] < res[(2, True)][1]["n_remaps"] < res[(0, False)][1]["n_remaps"]
    two = mixed_circuit(14, 400, seed=3)
    two = two[two["kind"] != KIND_U]
    P = Q.Program(two, 14, "c128", form="pass", k_tile=10, max_swaps=4, lane_gates=4, lane_eager=True)
    assert P.op_counts()["lane"] == 0
    P.close()
    with pytest.raises(ValueError):
        Q.make_opts(lane_gates=3)
    o = Q.make_opts(**base)
    o.flags = 64
    with pytest.raises(Q.QsimError):
        Q.qs_compile(g[:10], 30, "c128", None, o)


def test_wavefront_local_relayouts():
    """Re-layouts that keep the tile bits on the wavefront bits of the thread
    id need no barrier.  On the 30-qubit workload (four wavefronts per
    workgroup) the choice of those bits by next use makes 81 of the 129
    re-layouts inside passes wavefront-local (the first layout of a pass never
    is); a workgroup of one wavefront has none to keep, and with lane gates
    (which name thread bits of the ascending map) none are made."""
    g = config_circuit(2)
    base = dict(form="pass", k_tile=12, max_swaps=16, pinned=3, perm_exec="relabel")
    P = Q.Program(g, 30, "c128", **base)
    c, st = P.op_counts(), P.stats()
    P.close()
    assert c["remap"] == 172 and c["remap_wave"] == 81
    assert c["remap_wave"] <= c["remap"] - st["n_tile_passes"]
    P = Q.Program(g, 30, "c128", lane_gates=2, **base)
    assert P.op_counts()["remap_wave"] == 0
    P.close()
    P = Q.Program(g[:200], 30, "c128", form="pass", k_tile=8, reg_bits=2, max_swaps=4)
    c = P.op_counts()
    P.close()
    assert c["remap"] > 0 and c["remap_wave"] == 0


def test_cost_model_prediction_is_linear_in_counts():
    from paper_2010_09746_amd.costmodel import TILE_CLASSES, CostModel
    cm = CostModel("c128", n_cal=20)
    cm.tile_costs[(10, 0)] = {c: 1.0 + i for i, c in enumerate(TILE_CLASSES)}
    cm.launch_costs = dict(plain_u=2.0, plain_cu=3.0, plain_cx=1.5, plain_cz=1.0, move=0.0, move_fraction=4.0)
    counts = {c: 0.0 for c in Q.OPC_NAMES}
    counts.update(tile_pass=2, u=10, remap=3, plain_cx=4, move_fraction=0.5)
    want = (2 * 1.0 + 10 * 2.0 + 3 * (1.0 + TILE_CLASSES.index("remap")) + 4 * 1.5 + 0.5 * 4.0) * 2 ** 4
    assert abs(cm.predict_counts(counts, 24, 10, 0) - want) < 1e-9


def test_relayouts_bounded_on_layered_workload():
    """Re-layouts of the 30-qubit layered workload (k = 12, 16 amplitudes per
    thread): at least one per pass and one per 4 distinct targets of a layer,
    at most one per gate; 172 with the look-ahead register choice."""
    g = config_circuit(2)
    P = Q.Program(g, 30, "c128", form="pass", k_tile=12, max_swaps=16, pinned=3, perm_exec="relabel", reg_bits=4)
    c = P.op_counts()
    st = P.stats()
    P.close()
    assert c["tile_pass"] == st["n_tile_passes"] == 43
    assert 40 * 3 <= c["remap"] <= 172      # 12 local targets per layer, 4 register bits
    assert c["remap"] == st["n_remaps"]


# ----------------------------------------------------------------------------
# The pass deciding by predicted time (qs_compile_costed; paper, Section 3,
# closing remark: a pass may use the simulator's benchmarks)

def _is_local(rec, sigma, m):
    k, q0, q1 = int(rec["kind"]), int(rec["q0"]), int(rec["q1"])
    u = rec["u"]
    diag = u[2] == 0 and u[3] == 0 and u[4] == 0 and u[5] == 0
    if k == KIND_U:
        return diag or sigma[q0] < m
    if k == 2:  # CZ
        return True
    if k == 3 and diag:  # controlled diagonal
        return True
    return sigma[q1] < m


def _cost_class(rec):
    k, u = int(rec["kind"]), rec["u"]
    diag = u[2] == 0 and u[3] == 0 and u[4] == 0 and u[5] == 0
    if k == 2 or (k in (0, 3) and diag):
        return 2
    return 0 if k == KIND_U else 1


def _closure_set(g, preds, done, sigma, m):
    mark = set()
    for v in range(len(g)):
        if v not in done and _is_local(g[v], sigma, m) and all(h in done or h in mark for h in preds[v]):
            mark.add(v)
    return mark


def _expected_decision(g, preds, done, sigma, m, r, pinned, costs):
    """Brute force of the decision: Algorithm 1's chain (first strict maximum
    over local qubits l, then global g, in ascending qubit order; each link
    strictly raises the count), every prefix priced as movement + tile pass +
    its gates per gate, against the first ready gate as a launch of its own."""
    n = len(sigma)
    prefixes, cur, base = [], list(sigma), 0
    for _ in range(r):
        best, arg = base, None
        for a in range(n):
            if not (pinned <= cur[a] < m):
                continue
            for b in range(n):
                if cur[b] >= m:
                    s2 = list(cur)
                    s2[a], s2[b] = cur[b], cur[a]
                    c = len(_closure_set(g, preds, done, s2, m))
                    if c > best:
                        best, arg = c, s2
        if arg is None:
            break
        cur, base = arg, best
        prefixes.append(cur)
    ready = [v for v in range(len(g)) if v not in done and preds[v] <= done]
    first = min(ready)
    if not prefixes:
        return ("global", first)
    rates = []
    for p in prefixes:
        s = _closure_set(g, preds, done, p, m)
        cls = [0, 0, 0]
        for v in s:
            cls[_cost_class(g[v])] += 1
        changed = sum(1 for q in range(n) if p[q] != sigma[q])
        t = costs["move"] * (1 - 2.0 ** -(changed // 2)) + costs["tile"] + sum(c * w for c, w in zip(cls, costs["in"]))
        rates.append(t / len(s))
    take = len(prefixes)
    for b in range(len(prefixes), 0, -1):
        if rates[b - 1] < rates[take - 1]:
            take = b
    if costs["plain"][int(g[first]["kind"])] < rates[take - 1]:
        return ("global", first)
    return ("perm", tuple(prefixes[take - 1]))


def _pc(c):
    return Q.make_pass_costs(c["tile"], c["in"], c["move"], c["plain"])


def test_costed_pass_is_algorithm1_when_communication_dominates():
    """No movement or in-pass cost and launches of their own costlier than a
    tile pass: the time per gate falls with every link of the chain and never
    favours the fallback, so the instructions are the oracle's Algorithm 1
    (with its r / pinned variants), word for word."""
    c = dict(tile=1.0, **{"in": (0.0, 0.0, 0.0)}, move=0.0, plain=(10.0,) * 4)
    for g, n, m, r, pinned in [(paper_random_circuit(20, 600, 0.3, 4), 20, 16, 1, 0),
                               (mixed_circuit(12, 150, 3), 12, 7, 1, 0),
                               (layered_circuit(16, 12, seed=9), 16, 10, 4, 3),
                               (config_circuit(2, n=20, layers=10), 20, 12, 16, 3)]:
        ref, _ = O.pass_ref(g, n, m, r=r, pinned=pinned)
        P = Q.Program(g, n, "c128", k_tile=m, max_swaps=r, pinned=pinned, costs=_pc(c))
        ins = P.instructions()
        P.close()
        assert ins == ref


@pytest.mark.parametrize("r,pinned,perm_exec,costs", [
    (1, 0, "move", dict(tile=1.0, **{"in": (0.01, 0.02, 0.005)}, move=2.0, plain=(1.0, 1.0, 0.7, 1.1))),
    (3, 0, "move", dict(tile=1.0, **{"in": (0.05, 0.08, 0.01)}, move=1.5, plain=(1.0, 1.0, 1.0, 1.0))),
    (4, 1, "relabel", dict(tile=1.0, **{"in": (0.3, 0.5, 0.05)}, move=0.0, plain=(0.9, 0.9, 0.6, 1.0))),
    (2, 0, "relabel", dict(tile=2.0, **{"in": (0.02, 0.4, 0.01)}, move=0.0, plain=(1.0, 1.0, 1.0, 1.0)))])
@pytest.mark.parametrize("seed", range(4))
def test_costed_pass_decisions_brute_force(r, pinned, perm_exec, costs, seed):
    """Tiny circuits: every PermuteQubits / fallback gate of the costed pass is
    the brute-force choice (see _expected_decision), every applied gate is
    local and ready, and the compiled program computes the circuit."""
    n, m = 6, 3 + seed % 2
    g = mixed_circuit(n, 40, seed=3000 + seed) if seed % 2 else paper_random_circuit(n, 40, 0.4, seed=3000 + seed)
    P = Q.Program(g, n, "c128", k_tile=m, max_swaps=r, pinned=pinned, perm_exec=perm_exec, costs=_pc(costs))
    ins = P.instructions()
    P.close()
    preds = {v: set() for v in range(len(g))}
    for h, v in O.dag_edges(g):
        preds[v].add(h)
    sigma, done = list(range(n)), set()
    for op, arg in ins:
        if op == "apply":
            assert arg not in done and preds[arg] <= done and _is_local(g[arg], sigma, m)
            done.add(arg)
            continue
        # a decision point: the sweep before it scheduled every local ready gate
        assert not _closure_set(g, preds, done, sigma, m)
        exp = _expected_decision(g, preds, done, sigma, m, r, pinned, costs)
        if op == "perm":
            assert exp == ("perm", tuple(arg))
            sigma = list(arg)
        else:
            assert exp == ("global", arg)
            done.add(arg)
    assert done == set(range(len(g)))
    v, sig = O.run_program(g, n, ins, x=7)
    assert np.abs(O.to_logical(v, n, sig) - O.run(g, n, x=7)).max() < 1e-13


def test_costed_pass_trades_permutations_for_launches_of_their_own():
    """With moved placements (the paper's PermuteQubits) priced at two passes,
    exchanges that make few gates local are replaced by gates run on their own
    (the layered workload's shape: fewer PermuteQubits than Algorithm 1); with
    relabelled placements a permutation costs nothing and the choices are
    Algorithm 1's with maximal chains."""
    n, m = 20, 12
    g = config_circuit(2, n=n, layers=20)
    c = dict(tile=1.0, **{"in": (0.02, 0.02, 0.005)}, move=2.0, plain=(1.0, 1.0, 1.0, 1.0))
    P = Q.Program(g, n, "c128", k_tile=m, max_swaps=1, perm_exec="move", costs=_pc(c))
    st = P.stats()
    P.close()
    ref = Q.Program(g, n, "c128", k_tile=m, max_swaps=1, perm_exec="move").stats()
    assert st["n_global"] > ref["n_global"] and st["n_perm"] < ref["n_perm"]
    c["move"] = 0.0
    P = Q.Program(g, n, "c128", k_tile=m, max_swaps=16, pinned=3, costs=_pc(c))
    ins = P.instructions()
    P.close()
    assert ins == Q.Program(g, n, "c128", k_tile=m, max_swaps=16, pinned=3).instructions()


def test_costed_compile_rejects_bad_costs():
    g = paper_random_circuit(8, 40, 0.3, seed=1)
    for bad in (dict(tile=-1.0, **{"in": (0, 0, 0)}, move=0.0, plain=(1,) * 4),
                dict(tile=1.0, **{"in": (0, float("nan"), 0)}, move=0.0, plain=(1,) * 4)):
        with pytest.raises(Q.QsimError):
            Q.Program(g, 8, "c128", k_tile=6, max_swaps=1, costs=_pc(bad))
