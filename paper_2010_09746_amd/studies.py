"""Measurement studies on the device, through the library only.

* ``kernel_sweep``: the single-purpose kernels one by one at their real size:
  a one-qubit gate on every target qubit (the GPU counterpart of the paper's
  Fig. 1, which times one gate per qubit index on a distributed state), CNOT
  and CZ for low / high qubit pairs, the position-exchange data movement for
  1..8 exchanged pairs (PermuteQubits, Section 2 and Appendix A), the
  fused tile pass against the number of gates it carries (HBM-bound with few
  gates, ALU-bound with many), and the read-out of every <Z_q>.
* ``qft_study``: the quantum Fourier transform and the QFT-like circuit of
  Appendix C through the permutation pass; the QFT output is checked against
  its closed form at sampled indices.
* ``random_family_study``: the paper's random family of Section 4 (CNOT with
  probability p, else H or Y), plain gate-by-gate against the pass form for a
  range of p: the measured counterpart of the paper's Fig. 2 estimate.
"""

from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import qsim as Q

from workloads import (H, KIND_CX, KIND_CZ, KIND_U, MASTER_SEED, haar_u2, make_gates, paper_random_circuit,
                       qft_circuit, qft_like_circuit, sample_indices)


def _profiled(fn):
    """Run fn with launch profiling on; return {class: {launches, avg_ms, gbs}}."""
    torch.cuda.synchronize()
    Q.qs_profile_read()
    Q.qs_profile_enable(True)
    fn()
    torch.cuda.synchronize()
    Q.qs_profile_enable(False)
    out = {}
    for name, e in Q.qs_profile_read().items():
        out[name] = dict(launches=e["launches"], avg_ms=e["avg_ms"],
                         gbs=e["bytes"] / max(e["total_ms"], 1e-9) / 1e6)
    return out


def kernel_sweep(n: int = 30, dtype: str = "c128", reps: int = 3) -> dict:
    st = Q.State(n, dtype)
    res = {"n": n, "dtype": dtype}
    # one-qubit gate on each target
    per_target = []
    for t in range(n):
        g = make_gates([(KIND_U, t, -1, H)] * reps)
        st.apply_gates(g)
        p = _profiled(lambda: st.apply_gates(g))["plain_u"]
        per_target.append(dict(target=t, avg_ms=p["avg_ms"], gbs=p["gbs"]))
    res["plain_u_per_target"] = per_target
    # two-qubit gates for low / mixed / high pairs
    pairs = [(0, 1), (1, 0), (2, n - 2), (n - 2, 2), (n - 2, n - 1), (n - 1, 0)]
    for kind, name, cls in ((KIND_CX, "cx", "plain_cx"), (KIND_CZ, "cz", "plain_cz")):
        rows = []
        for c, t in pairs:
            g = make_gates([(kind, c, t, None)] * reps)
            st.apply_gates(g)
            p = _profiled(lambda: st.apply_gates(g))[cls]
            rows.append(dict(control=c, target=t, avg_ms=p["avg_ms"], gbs=p["gbs"]))
        res["plain_" + name] = rows
    # position exchanges: P pairs (i, n-1-i), i < P, moved there and back
    moves = []
    ident = list(range(n))
    for npairs in range(1, 9):
        sig = list(range(n))
        for i in range(npairs):
            sig[i], sig[n - 1 - i] = sig[n - 1 - i], sig[i]
        st.permute(sig)
        st.permute(ident)

        def go():
            for _ in range(reps):
                st.permute(sig)
                st.permute(ident)
        p = _profiled(go)["move_involution"]
        moves.append(dict(pairs=npairs, moved_fraction=1.0 - 2.0 ** -npairs, avg_ms=p["avg_ms"], gbs=p["gbs"]))
    res["permute"] = moves
    # one fused tile pass carrying G Haar one-qubit gates on the tile's qubits,
    # at tile sizes 2^12 and 2^13
    rng = np.random.default_rng(MASTER_SEED + 17)
    fused = []
    for k in (min(12, n), min(13, n)):
        for ng in (1, 2, 4, 8, 12, 16, 24, 32, 48):
            g = make_gates([(KIND_U, i % k, -1, haar_u2(rng)) for i in range(ng)])
            prog = Q.Program(g, n, dtype, form="pass", k_tile=k, max_swaps=16, pinned=3, perm_exec="relabel")
            st.run_program(prog)
            p = _profiled(lambda: [st.run_program(prog) for _ in range(reps)])["tile_pass"]
            prog.close()
            fused.append(dict(k=k, gates=ng, avg_ms=p["avg_ms"], gbs=p["gbs"],
                              tflops=14.0 * ng * float(1 << n) / (p["avg_ms"] * 1e-3) / 1e12))
    res["tile_pass_by_gates"] = fused
    st.expect_z()
    p = _profiled(lambda: [st.expect_z() for _ in range(reps)])
    res["zsum"] = p.get("zsum")
    st.close()
    return res


def _rev(y: np.ndarray, n: int) -> np.ndarray:
    r = np.zeros_like(y)
    for b in range(n):
        r |= ((y >> np.uint64(b)) & np.uint64(1)) << np.uint64(n - 1 - b)
    return r


def qft_study(n: int = 30, dtype: str = "c128", k: int = 10, r: int = 8, pinned: int = 3, x: int = 0x2545F491,
              samples: int = 1024, reps: int = 2) -> dict:
    """QFT on |x> and the QFT-like circuit of Appendix C, pass form."""
    st = Q.State(n, dtype)
    out = {"n": n, "dtype": dtype, "k_tile": k, "max_swaps": r}
    x = x % (1 << n)
    idx = sample_indices(n, samples, 20100946 + 7)
    for name, gates in (("qft", qft_circuit(n)), ("qft_like", qft_like_circuit(n))):
        opts = dict(form="pass", k_tile=k, max_swaps=r, pinned=pinned, perm_exec="relabel")
        prog = Q.Program(gates, n, dtype, **opts)
        stats = prog.stats()
        ts = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st.set_basis(x if name == "qft" else 0)
            st.run_program(prog)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        sec = float(np.median(ts[1:]))
        row = dict(gates=len(gates), ms=sec * 1e3, amp_updates_per_s=len(gates) * float(1 << n) / sec,
                   n_perm=stats["n_perm"], n_global=stats["n_global"], n_tile_passes=stats["n_tile_passes"],
                   perm_bound_2_n_minus_k=2 * (n - k), norm=st.norm())
        if name == "qft":
            # closed form: amplitude at logical index rev(y) is e^{2 pi i x y / 2^n} / sqrt(2^n)
            y = _rev(idx, n)
            ph = 2.0 * math.pi * ((np.uint64(x) * y) % np.uint64(1 << n)).astype(np.float64) / float(1 << n)
            want = np.exp(1j * ph) / math.sqrt(float(1 << n))
            got = st.amplitudes(idx)
            row["max_abs_error_vs_closed_form"] = float(np.abs(got - want).max())
            row["checked_amplitudes"] = int(len(idx))
        prog.close()
        out[name] = row
    st.close()
    return out


def _comm_fraction(gates: np.ndarray, m: int) -> float:
    """Fraction of gates whose non-diagonal target is at a position >= m under
    the identity placement (gates that would communicate in the paper's
    setting without the pass)."""
    kinds, q0, q1 = gates["kind"], gates["q0"], gates["q1"]
    tgt = np.where(kinds == KIND_U, q0, q1)
    diag = (kinds == KIND_CZ)
    return float(np.mean((tgt >= m) & ~diag))


def random_family_study(n: int = 28, dtype: str = "c128", ps=(0.0, 0.1, 0.3, 0.5, 0.7, 1.0), k: int = 10,
                        r: int = 8, pinned: int = 3, seed: int = 20100946 + 8) -> dict:
    """Plain against pass form on the random family (30 n gates per circuit)."""
    st = Q.State(n, dtype)
    rows = []
    for p in ps:
        gates = paper_random_circuit(n, 30 * n, p, seed)
        res = {}
        for form in ("plain", "pass"):
            opts = dict(form=form) if form == "plain" else dict(form="pass", k_tile=k, max_swaps=r, pinned=pinned,
                                                                perm_exec="relabel")
            prog = Q.Program(gates, n, dtype, **opts)
            st.set_basis(0)
            st.run_program(prog)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st.set_basis(0)
            st.run_program(prog)
            torch.cuda.synchronize()
            res[form] = (time.perf_counter() - t0) * 1e3
            if form == "pass":
                s = prog.stats()
                res["n_perm"], res["n_tile_passes"] = s["n_perm"], s["n_tile_passes"]
            prog.close()
        rows.append(dict(p=p, gates=len(gates), plain_ms=res["plain"], pass_ms=res["pass"],
                         speedup=res["plain"] / res["pass"], n_perm=res["n_perm"], n_tile_passes=res["n_tile_passes"],
                         comm_fraction_without_pass=_comm_fraction(gates, k)))
    st.close()
    return {"n": n, "dtype": dtype, "k_tile": k, "max_swaps": r, "rows": rows}


def ablation_study(n: int = 30, dtype: str = "c128", layers: int = 40, reps: int = 1,
                   ks=(10, 11, 12, 13, 14), r: int = 16, k_ref: int = 12) -> dict:
    """The 30-qubit layered workload under the pass's variants: Algorithm 1 as
    printed (r = 1, no pinned qubits; each PermuteQubits moves the data, so
    tiles stay contiguous), r = 1 with 3 pinned positions and relabelled
    placements, the fused pass with bundled exchanges (r = 16) over tile sizes
    ks, fusion without the pass (r = 0: gates on the first k positions
    fused, every other gate one launch), and the pass at k_ref with one-qubit
    gates on the lowest thread bits run through lane exchanges instead of
    register re-layouts.  Device time of one run of the compiled program
    each."""
    from . import costmodel
    from workloads import config_circuit

    g = config_circuit(2, n=n, layers=layers)
    variants = [("fusion without pass", dict(k_tile=k_ref, max_swaps=0, pinned=0, perm_exec="relabel")),
                ("Algorithm 1 (r=1), moved", dict(k_tile=k_ref, max_swaps=1, pinned=0, perm_exec="move")),
                ("r=1, 3 pinned, relabelled", dict(k_tile=k_ref, max_swaps=1, pinned=3, perm_exec="relabel"))]
    variants += [(f"pass r={r} k={k}", dict(k_tile=k, max_swaps=r, pinned=3, perm_exec="relabel")) for k in ks]
    # gates on the lowest thread bits through lane exchanges instead of
    # register re-layouts (off by default)
    lane = dict(k_tile=k_ref, max_swaps=r, pinned=3, perm_exec="relabel")
    variants += [(f"pass r={r} k={k_ref}, lane gates on thread bits 0-3 when a re-layout is put off",
                  dict(lane, lane_gates=4)),
                 (f"pass r={r} k={k_ref}, lane gates on thread bits 0-1 whenever ready",
                  dict(lane, lane_gates=2, lane_eager=True)),
                 (f"pass r={r} k={k_ref}, lane gates on thread bits 0-3 whenever ready",
                  dict(lane, lane_gates=4, lane_eager=True))]
    rows = []
    for name, o in variants:
        prog = Q.Program(g, n, dtype, form="pass", **o)
        stt, cnt = prog.stats(), prog.op_counts()
        prog.close()
        ms = costmodel.measure_ms(g, n, dtype, o, reps=reps)
        rows.append(dict(variant=name, opts=o, ms=ms, amp_updates_per_s=len(g) * float(1 << n) / (ms * 1e-3),
                         n_perm=stt["n_perm"], n_global=stt["n_global"], n_tile_passes=stt["n_tile_passes"],
                         n_plain=stt["n_plain"], n_remaps=stt["n_remaps"], lane_gates=cnt["lane"]))
    return {"n": n, "dtype": dtype, "gates": int(len(g)), "rows": rows}
