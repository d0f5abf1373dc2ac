"""CPU checks of the batching form's single-launch plan and of the protocol
its persistent launch follows (host model, no device).

The launch hands out work items by ticket in the plan's order; an item waits
until its circuit's previous pass has completed all its tiles; a workgroup
takes a ticket only while it runs.  Progress needs every item's dependency
to come earlier in the ticket order: then the lowest unfinished ticket is
always held by a running workgroup whose dependency is complete.  The model
below runs that protocol under adversarial scheduling (random interleavings,
few resident workgroups, random work lengths) and checks that it always
drains and never starts an item before its dependency is complete; a plan
whose order breaks the rule is shown to deadlock in the same model."""

import random

import numpy as np
import pytest

from paper_2010_09746_amd import qsim as Q
from workloads import batch_workload, layered_circuit, mixed_circuit


def _circuits(seed, count=14, n_lo=9, n_hi=15):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.integers(1, 10))
        g = layered_circuit(n, d, seed=seed * 100 + i) if i % 3 else mixed_circuit(n, 10 * d, seed=i)
        out.append((n, g))
    return out


def _check_plan(circ, passes, items, k_max):
    # pass table: each circuit's passes in order, tile size min(n, k_max)
    by_c = {}
    for pi, p in enumerate(passes):
        n = circ[p["circuit"]][0]
        assert p["k_tile"] == min(n, k_max)
        assert p["tiles"] == 1 << (n - p["k_tile"])
        by_c.setdefault(p["circuit"], []).append(pi)
    assert sorted(by_c) == list(range(len(circ)))
    for c, ps in by_c.items():
        assert [passes[pi]["level"] for pi in ps] == list(range(len(ps)))
        assert [passes[pi]["last"] for pi in ps] == [0] * (len(ps) - 1) + [1]
        if circ[c][0] <= k_max:  # the whole state is one tile
            assert all(passes[pi]["tiles"] == 1 for pi in ps)
    # items: every tile of every pass exactly once; dependency = previous pass
    cover = {pi: np.zeros(p["tiles"], dtype=int) for pi, p in enumerate(passes)}
    first = {}
    last = {}
    for t, it in enumerate(items):
        pi = it["pass_"]
        cover[pi][it["t0"]:it["t1"]] += 1
        first.setdefault(pi, t)
        last[pi] = t
        p = passes[pi]
        if p["level"] == 0:
            assert it["dep"] == -1 and it["need"] == 0
        else:
            dep = by_c[p["circuit"]][p["level"] - 1]
            assert it["dep"] == dep and it["need"] == passes[dep]["tiles"]
    for pi, cv in cover.items():
        assert (cv == 1).all(), pi
    # the order the progress argument needs: all of a dependency's items come
    # before the first item that waits for it
    for pi, p in enumerate(passes):
        if p["level"] > 0:
            dep = by_c[p["circuit"]][p["level"] - 1]
            assert last[dep] < first[pi]


def _model_run(passes, items, resident, grid, rng, max_steps=2_000_000):
    """Run the ticket protocol: `grid` workgroups of which at most `resident`
    run at a time (the others start when a running one exits).  Each step
    advances one running workgroup chosen at random.  Returns (drained,
    violations)."""
    done = [0] * len(passes)
    nxt = 0
    waiting = list(range(grid))
    running = []          # dicts: state, item, left
    for _ in range(min(resident, grid)):
        running.append(dict(wg=waiting.pop(0), state="take"))
    violations = 0
    for _ in range(max_steps):
        if not running:
            return True, violations
        w = running[rng.randrange(len(running))]
        if w["state"] == "take":
            t = nxt
            nxt += 1
            if t >= len(items):
                running.remove(w)
                if waiting:
                    running.append(dict(wg=waiting.pop(0), state="take"))
                continue
            w["item"], w["state"] = t, "wait"
        elif w["state"] == "wait":
            it = items[w["item"]]
            if it["dep"] < 0 or done[it["dep"]] >= it["need"]:
                if it["dep"] >= 0 and done[it["dep"]] != passes[it["dep"]]["tiles"]:
                    violations += 1
                w["state"], w["left"] = "work", rng.randrange(1, 6)
        else:
            w["left"] -= 1
            if w["left"] == 0:
                it = items[w["item"]]
                done[it["pass_"]] += it["t1"] - it["t0"]
                w["state"] = "take"
    return False, violations


@pytest.mark.parametrize("k_max,chunk,seed", [(12, 1, 1), (10, 2, 2), (9, 3, 3), (11, 4, 4)])
def test_plan_covers_work_in_dependency_order(k_max, chunk, seed):
    circ = _circuits(seed)
    passes, items = Q.qs_batch_plan(circ, "c64", Q.make_batch_opts(k_tile=k_max, max_swaps=4, chunk=chunk))
    _check_plan(circ, passes, items, k_max)


@pytest.mark.parametrize("resident,grid", [(1, 1), (2, 3), (3, 12), (5, 5), (8, 40)])
def test_protocol_drains_under_adversarial_scheduling(resident, grid):
    circ = _circuits(7, count=8, n_lo=9, n_hi=13)
    passes, items = Q.qs_batch_plan(circ, "c128", Q.make_batch_opts(k_tile=10, max_swaps=2, chunk=1))
    assert max(p["level"] for p in passes) >= 2
    rng = random.Random(resident * 1000 + grid)
    for _ in range(3):
        drained, bad = _model_run(passes, items, resident, grid, rng)
        assert drained and bad == 0


def test_model_detects_an_order_that_can_deadlock():
    """The same model with the items of each circuit's last pass moved to the
    front: one resident workgroup takes such an item first and waits for a
    pass whose items nobody can take any more."""
    circ = _circuits(9, count=4, n_lo=10, n_hi=12)
    passes, items = Q.qs_batch_plan(circ, "c64", Q.make_batch_opts(k_tile=10, max_swaps=2, chunk=1))
    bad = [it for it in items if it["dep"] >= 0 and passes[it["pass_"]]["last"]] + \
          [it for it in items if not (it["dep"] >= 0 and passes[it["pass_"]]["last"])]
    drained, _ = _model_run(passes, bad, 1, 1, random.Random(0), max_steps=200_000)
    assert not drained


def test_plan_of_the_256_circuit_workload():
    """The batching workload: circuits of at most 12 qubits are one tile (one
    pass); larger ones use 2^12-amplitude tiles."""
    wl = [(n, g) for n, d, g in batch_workload(count=256)][::8]
    passes, items = Q.qs_batch_plan(wl, "c64", Q.make_batch_opts(k_tile=12, max_swaps=16, pinned=4, chunk=4))
    _check_plan(wl, passes, items, 12)
    for c, (n, g) in enumerate(wl):
        ps = [p for p in passes if p["circuit"] == c]
        if n <= 12:
            assert len(ps) == 1


def test_plan_rejects_bad_options():
    circ = _circuits(1, count=2)
    for bad in (dict(k_tile=8), dict(k_tile=13), dict(chunk=-1), dict(wait_ms=-2)):
        with pytest.raises(Q.QsimError):
            Q.qs_batch_plan(circ, "c64", Q.make_batch_opts(**bad))
    with pytest.raises(Q.QsimError):
        Q.qs_batch_plan([(8, layered_circuit(8, 2, seed=1))], "c64", Q.make_batch_opts())
