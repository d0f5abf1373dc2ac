"""Benchmark-informed choice of the pass parameters.

The paper's pass decides with a step function: a gate on local qubits is
cheap, anything else costs a global exchange (Section 3 notes that a pass could
use the simulator's own benchmarks instead).  On one GPU every tile pass reads
and writes the whole state once, and what happens inside a pass has costs that
depend on the operation: a one-qubit butterfly, a controlled exchange on
register or thread bits, a sign flip, a register re-layout through LDS, or a
scalar-only relabel.  This module measures those costs on the device and picks
the tile size k, the exchange bundle r, the register shape and the permutation
executor that minimise the predicted time of a given circuit.

Model: for a compiled program with work counts c (``Program.op_counts``),

    t(program) = 2^(n - n_cal) * sum_class c[class] * cost[class]

where cost[tile_pass] is the fixed cost of a pass (load and store of every
tile), the other in-pass classes are per operation and tile weight, and the
one-gate and data-movement launches have their own per-launch costs.  The
costs are fitted by least squares from small calibration passes at n_cal
qubits, one per class, whose work counts come from the same compiler.

The same costs can also drive the pass's own choices (``pass_costs``, used by
``qsim.Program(costs=...)`` / ``qs_compile_costed``): at each PermuteQubits it
prices every prefix of Algorithm 1's chain of exchanges (data movement, tile
pass, gates) per gate against running the first ready gate as a launch of its
own, and ``choose`` can consider those programs beside the step-function ones.
"""

from __future__ import annotations

import itertools
import math
import time

import numpy as np
import torch

from . import qsim as Q

from workloads import KIND_CU, KIND_CX, KIND_CZ, KIND_U, haar_u2, make_gates, phase

TILE_CLASSES = ["tile_pass", "u", "shear", "u_ctrl", "x_reg", "x_lane", "neg", "diag", "remap", "dispatch"]
# compile options of calibration circuits that need them: "u" measures whole
# 2x2 updates, so its circuit keeps every matrix whole
CAL_OPTS = {"u": dict(full_matrices=True)}


def _pass_ms(st: Q.State, prog: Q.Program, reps: int = 3) -> float:
    """Median device time of one run of prog (sum of its timed launches)."""
    st.set_basis(0)
    st.run_program(prog)
    ts = []
    for _ in range(reps):
        st.set_basis(0)
        torch.cuda.synchronize()
        Q.qs_profile_read()
        Q.qs_profile_enable(True)
        st.run_program(prog)
        torch.cuda.synchronize()
        Q.qs_profile_enable(False)
        ts.append(sum(e["total_ms"] for name, e in Q.qs_profile_read().items() if name != "set_basis"))
    return float(np.median(ts))


def calibration_circuits(n: int, k: int, log_r: int, seed: int = 20100946 + 9) -> dict:
    """One single-pass circuit per in-pass class (all targets inside the tile)."""
    rng = np.random.default_rng(seed)
    R = max(1, log_r)
    N = 160
    st = next(s for s in (7, 5, 3, 11, 13) if math.gcd(s, k) == 1 and s % k)
    U = lambda q: (KIND_U, q, -1, haar_u2(rng))
    c = {
        "base": [U(0)],
        "u": [U(q % R) for q in range(N + 1)],
        # the same gates as shears (all but each qubit's last)
        "shear": [U(q % R) for q in range(N + 1)],
        "u_ctrl": [U(0)] + [(KIND_CU, (q + 1) % R, q % R, haar_u2(rng)) for q in range(N)] if R > 1 else None,
        "x_reg": [U(0)] + [(KIND_CX, (q + 1) % R, q % R, None) for q in range(N)] if R > 1 else None,
        "x_lane": [U(0)] + [(KIND_CX, R + 1, q % R, None) for q in range(N)],
        "neg": [U(0)] + [(KIND_CZ, q % (k - 1), q % (k - 1) + 1, None) for q in range(N)],
        "diag": [U(0)] + [(KIND_U, q % R, -1, phase(0.1 + 0.01 * q)) for q in range(N)],
        "dispatch": [U(0)] + [(KIND_CX, n - 1, q % R, None) for q in range(N)],
        # a dependency chain over all tile qubits: each gate's target is the
        # previous gate's, so most steps need a new register layout
        "remap": [g for i in range(N // 2) for g in (U((st * i) % k), (KIND_CX, (st * i) % k, (st * i + st) % k, None))],
    }
    return {name: make_gates(g) for name, g in c.items() if g is not None}


class CostModel:
    """Measured costs per (amplitude type, k, register bits) tile shape."""

    def __init__(self, dtype: str = "c128", n_cal: int = 27, perm_exec: str = "relabel", pinned: int = 3):
        self.dtype, self.n_cal, self.perm_exec, self.pinned = dtype, n_cal, perm_exec, pinned
        self.tile_costs = {}   # (k, reg_bits) -> {class: ms at n_cal}
        self.launch_costs = None
        self.fit_residual = {}

    # -- calibration ------------------------------------------------------------
    def calibrate_launches(self, st: Q.State) -> dict:
        n = self.n_cal
        H = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
        out = {}
        for name, cls, g in (("plain_u", "plain_u", [(KIND_U, t, -1, H) for t in (0, n // 2, n - 1)]),
                             ("plain_cu", "plain_cu", [(KIND_CU, 0, n - 1, H), (KIND_CU, n - 1, 0, H)]),
                             ("plain_cx", "plain_cx", [(KIND_CX, 0, n - 1, None), (KIND_CX, n - 1, 0, None)]),
                             ("plain_cz", "plain_cz", [(KIND_CZ, 0, n - 1, None), (KIND_CZ, 1, n - 2, None)])):
            gates = make_gates(g * 2)
            st.apply_gates(gates)
            torch.cuda.synchronize()
            Q.qs_profile_read()
            Q.qs_profile_enable(True)
            st.apply_gates(gates)
            torch.cuda.synchronize()
            Q.qs_profile_enable(False)
            out[name] = Q.qs_profile_read()[cls]["avg_ms"]
        # data movement: 4 exchanged position pairs (15/16 of the state moves)
        sig = list(range(n))
        for i in range(4):
            sig[i], sig[n - 1 - i] = sig[n - 1 - i], sig[i]
        st.permute(sig)
        st.permute(list(range(n)))
        torch.cuda.synchronize()
        Q.qs_profile_read()
        Q.qs_profile_enable(True)
        st.permute(sig)
        st.permute(list(range(n)))
        torch.cuda.synchronize()
        Q.qs_profile_enable(False)
        mv = Q.qs_profile_read()["move_involution"]
        out["move_fraction"] = mv["avg_ms"] / (1.0 - 2.0 ** -4)
        out["move"] = 0.0
        self.launch_costs = out
        return out

    def calibrate_tile(self, st: Q.State, k: int, reg_bits: int = 0) -> dict:
        n = self.n_cal
        rows, times = [], []
        for name, g in calibration_circuits(n, k, self._log_r(k, reg_bits)).items():
            prog = Q.Program(g, n, self.dtype, form="pass", k_tile=k, max_swaps=1, pinned=self.pinned,
                             perm_exec=self.perm_exec, reg_bits=reg_bits, **CAL_OPTS.get(name, {}))
            c = prog.op_counts()
            times.append(_pass_ms(st, prog))
            rows.append([c[x] for x in TILE_CLASSES])
            prog.close()
        A, t = np.array(rows), np.array(times)
        cost, *_ = np.linalg.lstsq(A, t, rcond=None)
        cost = np.maximum(cost, 0.0)
        self.fit_residual[(k, reg_bits)] = float(np.abs(A @ cost - t).max() / max(t.max(), 1e-9))
        self.tile_costs[(k, reg_bits)] = dict(zip(TILE_CLASSES, (float(v) for v in cost)))
        return self.tile_costs[(k, reg_bits)]

    def _log_r(self, k: int, reg_bits: int) -> int:
        # the library's tile shape of a pass: 16 amplitudes per thread by
        # default (8 for complex128 below 2^11-amplitude tiles), at most 1024
        # threads and at least one wavefront
        lr = reg_bits if reg_bits > 0 else ((4 if k >= 11 else 3) if self.dtype == "c128" else 4)
        lr = max(min(lr, 5), k - 10)
        return max(min(lr, k - 6), 1)

    def calibrate(self, shapes) -> None:
        st = Q.State(self.n_cal, self.dtype)
        if self.launch_costs is None:
            self.calibrate_launches(st)
        for k, rb in shapes:
            if (k, rb) not in self.tile_costs:
                self.calibrate_tile(st, k, rb)
        st.close()

    # -- prediction -----------------------------------------------------------
    def predict_counts(self, counts: dict, n: int, k: int, reg_bits: int) -> float:
        scale = 2.0 ** (n - self.n_cal)
        tc = self.tile_costs[(k, reg_bits)]
        ms = sum(counts[c] * tc[c] for c in TILE_CLASSES)
        # a pending phase applied on its own touches half the amplitudes of
        # a diagonal update (rare: the W that left it ended an earlier pass)
        ms += counts["phase"] * 0.5 * tc["diag"]
        lc = self.launch_costs
        ms += sum(counts[c] * lc[c] for c in ("plain_u", "plain_cu", "plain_cx", "plain_cz", "move",
                                               "move_fraction"))
        return ms * scale

    def pass_costs(self, n: int, k: int, reg_bits: int = 0, perm_exec: str = "relabel") -> dict:
        """The calibrated costs in the form the pass's own choices use
        (qs_pass_costs, ms at n qubits): a tile pass (its fixed cost plus the
        four re-layouts a pass of the layered workload makes), a gate inside
        it by class (non-diagonal one-qubit: a shear; two-qubit with a
        non-diagonal target: the mean of register- and lane-controlled
        exchanges; diagonal: a sign flip), moving the whole state (moved
        placements only) and each gate kind as a launch of its own."""
        self.calibrate([(k, reg_bits)])
        scale = 2.0 ** (n - self.n_cal)
        tc, lc = self.tile_costs[(k, reg_bits)], self.launch_costs
        return dict(tile=scale * (tc["tile_pass"] + 4 * tc["remap"]),
                    **{"in": (scale * tc["shear"], scale * 0.5 * (tc["x_reg"] + tc["x_lane"]), scale * tc["neg"])},
                    move=scale * lc["move_fraction"] if perm_exec == "move" else 0.0,
                    plain=tuple(scale * lc[c] for c in ("plain_u", "plain_cx", "plain_cz", "plain_cu")))

    @staticmethod
    def as_struct(c: dict):
        return Q.make_pass_costs(c["tile"], c["in"], c["move"], c["plain"])

    def predict(self, gates, n: int, costed: bool = False, **opts) -> tuple:
        costs = None
        if costed:
            costs = self.as_struct(self.pass_costs(n, opts.get("k_tile", 10), opts.get("reg_bits", 0),
                                                   opts.get("perm_exec", "relabel")))
        prog = Q.Program(gates, n, self.dtype, form="pass", costs=costs, **opts)
        counts = prog.op_counts()
        prog.close()
        return self.predict_counts(counts, n, opts.get("k_tile", 10), opts.get("reg_bits", 0)), counts

    def choose(self, gates, n: int, ks=(9, 10, 11, 12, 13), rs=(1, 4, 8, 16), reg_bits=(0,),
               perm_execs=("relabel",), costed=(False,)) -> tuple:
        """Predicted-best options for this circuit and the table of predictions
        (costed=(False, True) also considers the pass deciding by the
        measured costs; its entries carry costed=True)."""
        cands = []
        for k, r, rb, pe, cp in itertools.product(ks, rs, reg_bits, perm_execs, costed):
            if k > n or (16 if self.dtype == "c128" else 8) << k > 131072:
                continue
            c = dict(k_tile=k, max_swaps=r, reg_bits=rb, perm_exec=pe, pinned=self.pinned)
            if cp:
                c["costed"] = True
            cands.append(c)
        self.calibrate({(c["k_tile"], c["reg_bits"]) for c in cands})
        table = []
        for c in cands:
            ms, counts = self.predict(gates, n, **c)
            table.append(dict(opts=c, predicted_ms=ms, tile_passes=counts["tile_pass"], remaps=counts["remap"]))
        table.sort(key=lambda x: x["predicted_ms"])
        return table[0]["opts"], table


def measure_ms(gates, n: int, dtype: str, opts: dict, reps: int = 2, costs=None) -> float:
    """Device time of the pass form of a circuit with the given options (and,
    with costs, the pass deciding by them)."""
    st = Q.State(n, dtype)
    prog = Q.Program(gates, n, dtype, form="pass", costs=costs, **opts)
    ms = _pass_ms(st, prog, reps=reps)
    prog.close()
    st.close()
    return ms


def rank_correlation(a, b) -> float:
    ra = np.argsort(np.argsort(a)).astype(float)
    rb = np.argsort(np.argsort(b)).astype(float)
    ra -= ra.mean()
    rb -= rb.mean()
    return float((ra * rb).sum() / np.sqrt((ra * ra).sum() * (rb * rb).sum()))
