"""Benchmark of the simulator's hot path on one MI355X.

Workload (synthetic, seeded): 30 qubits in complex128 (16 GiB state), 40
layers; each layer applies a Haar-random U(2) to every qubit, then CNOT on a
random perfect matching, with CZ instead of CNOT on every third layer (1800
gates).  One step = the whole path on that circuit: state preparation, the
compiler (DAG + permutation pass + lowering), every tile pass / data movement
on the device, and read-out of <Z_q> for all q plus 1024 sampled amplitudes.

Metric: amplitude-updates/s = gates x 2^n / step time (whole-job, inputs
resident in HBM).  The pass form is the reported value; the plain gate-by-gate
form is timed beside it.  The dominant kernel (the fused tile pass) is timed
with HIP events around each launch on its own stream and priced against HBM.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# MI355X vector FP64 (and FP32 without packed math): 256 CUs x 64 FMA lanes
# x 2 flops x 2.4 GHz
VALU_PEAK_TFLOPS = 78.6
FLOPS_PER_AMP_1Q = 14  # one 2x2 complex update per amplitude: 2 complex products + 1 complex sum


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--layers", type=int, default=40)
    ap.add_argument("--dtype", default="c128")
    # the measured cost model's choice for the 30-qubit workload (bench.py --form costmodel)
    ap.add_argument("--k", type=int, default=12)
    ap.add_argument("--r", type=int, default=16)
    ap.add_argument("--perm-exec", default="relabel")
    ap.add_argument("--pinned", type=int, default=3)
    ap.add_argument("--pinned-c64", type=int, default=4,
                    help="pinned positions for complex64 runs (precision and serving forms): 4 keeps the "
                         "lowest 16 amplitudes, one 128-byte line, in every tile")
    ap.add_argument("--reg-bits", type=int, default=0)
    ap.add_argument("--costed", type=int, default=1,
                    help="1: the pass decides each PermuteQubits by the measured cost model (calibrated once on "
                         "this device before the warm-up, at --cal-n qubits); 0: Algorithm 1's step function")
    ap.add_argument("--plain-steps", type=int, default=1, help="timed steps of the plain form (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample length (0 = skip)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads (0 = the OpenMP default)")
    ap.add_argument("--cal-n", type=int, default=27, help="costmodel: qubits of the calibration passes")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "tile_pass_traffic.json"))
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="after the timed steps, copy a buffer of this many GiB 3 times (a plain copy kernel of "
                         "known size, used to scale hardware byte counters)")
    ap.add_argument("--traffic-from", default=None, metavar="FETCH_DIR,WRITE_DIR",
                    help="write --traffic-json from two rocprofv3 --pmc runs of this script with --copy-calib "
                         "(FETCH_SIZE, then WRITE_SIZE; CSV output directories) and exit")
    ap.add_argument("--forms", default="precision,batch,serve",
                    help="forms timed after the headline and reported as sub-objects of its line (comma-separated "
                         "subset of precision, batch, serve; empty: none)")
    ap.add_argument("--form-steps", type=int, default=1, help="timed steps of each form after its warm-up")
    ap.add_argument("--retune", action="store_true", help="batch: ignore the autotuner's cache")
    ap.add_argument("--no-tune", action="store_true",
                    help="batch: skip the autotuner and use the options it chose on MI355X (k_tile 12, r 16, "
                         "4 pinned, 3 workgroups per CU, 8 tiles per item)")
    ap.add_argument("--accuracy-requests", type=int, default=64,
                    help="serve: requests re-run alone in complex128 to state the served accuracy")
    ap.add_argument("--cpu-one-core-seconds", type=float, default=4.0,
                    help="oracle sample length with one thread (0 = skip)")
    ap.add_argument("--requests", type=int, default=1000, help="serve: requests in the trace")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: Poisson arrival rate (1/s)")
    ap.add_argument("--rate-sweep", default="5,10,15",
                    help="serve: comma-separated lower arrival rates, each run with --sweep-requests requests after "
                         "the main trace (finds the load one GPU sustains)")
    ap.add_argument("--sweep-requests", type=int, default=60)
    ap.add_argument("--serve-k", type=int, default=12, help="serve: tile qubits of the server")
    ap.add_argument("--serve-wg", type=int, default=16, help="serve: workgroups per CU of each step's launch")
    ap.add_argument("--serve-solo-tiles", type=int, default=None,
                    help="serve: passes with at least this many tiles run as launches of their own (0: never; "
                         "default: the library's, 2^10)")
    ap.add_argument("--form", default="pass",
                    choices=["pass", "precision", "batch", "serve", "kernels", "qft", "random-family", "costmodel",
                             "ablation"],
                    help="pass: the 30-qubit complex128 workload (default line); precision: 32 qubits, complex64 "
                         "against complex128; batch / serve: the batching and serving forms; kernels: each "
                         "single-purpose kernel at 30 qubits; qft: QFT and QFT-like circuits; random-family: the "
                         "paper's random family, plain against pass form; costmodel: the measured cost model's "
                         "choice and ranking; ablation: r=1, r=0 (fusion without the pass) and tile sizes 10..14")
    return ap.parse_args()


def kernel_source_hash():
    """sha1 of the tile kernel sources (hardware counters are stored with it)."""
    import hashlib

    h = hashlib.sha1()
    for f in ("tile_kernel.cuh", "common.cuh", "tile_args.h"):
        with open(os.path.join(ROOT, "paper_2010_09746_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_from_counters(a):
    """HBM bytes per tile-pass launch from FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch, two rocprofv3 --pmc runs of this script with --copy-calib G),
    each scaled by what the same counter reads for the plain copies of G GiB
    (the largest copy dispatches of the run); written to --traffic-json with
    the hash of the kernel sources they describe."""
    import csv
    import glob

    dirs = a.traffic_from.split(",")
    out = {"kernel": None, "kernel_source_sha1": kernel_source_hash(), "calibration": {}, "counters_KiB": {}}
    scales = {}
    for ctr, d in zip(("FETCH_SIZE", "WRITE_SIZE"), dirs):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows += [r for r in csv.DictReader(open(f)) if r["Counter_Name"] == ctr]
        # the workload's own passes: the largest grid (the cost model's
        # calibration passes run on a smaller state first)
        tile_rows = [r for r in rows if "k_tile<double, 8, 4" in r["Kernel_Name"]]
        grid = max((int(r["Grid_Size"]) for r in tile_rows), default=0)
        tile = [float(r["Counter_Value"]) for r in tile_rows if int(r["Grid_Size"]) == grid]
        copy = sorted(float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"])[-3:]
        if not tile or len(copy) < 3:
            raise SystemExit(f"{d}: no tile-pass or copy dispatches for {ctr}")
        out["kernel"] = next(r["Kernel_Name"] for r in rows if "k_tile<double, 8, 4" in r["Kernel_Name"])
        copy_kib = sum(copy) / len(copy)
        scales[ctr] = (a.copy_calib << 30) / (copy_kib * 1024.0)
        out["calibration"][ctr] = {"copy_bytes_per_dispatch": a.copy_calib << 30, "copy_KiB": copy_kib,
                                   "scale": scales[ctr]}
        out["counters_KiB"][ctr] = sum(tile) / len(tile)
    per_launch = sum(out["counters_KiB"][c] * 1024.0 * scales[c] for c in scales)
    out["bytes_per_launch"] = {f"n{a.n}_{a.dtype}_k{a.k}_r{a.r}_{a.perm_exec}": per_launch}
    out["commands"] = [f"rocprofv3 --pmc {c} --output-format csv -d <dir> -o run -- python3 bench.py --steps 1 "
                       f"--warmup 0 --plain-steps 0 --cpu-seconds 0 --forms= --copy-calib {a.copy_calib}"
                       for c in ("FETCH_SIZE", "WRITE_SIZE")]
    with open(a.traffic_json, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


def cpu_model():
    """CPU model name of this host and the number of CPUs this process may use."""
    name = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return dict(model=name, cpus_available=avail, cpus_total=os.cpu_count())


def _oracle_rate(gates, n, seconds, threads):
    """Apply the gates one by one with the oracle until `seconds` have passed
    (or the circuit ends); returns (gates done, seconds, threads used)."""
    import oracle as O

    O.lib()
    if threads > 0:
        O.set_threads(threads)
    s = O.zero_state(n)
    done = 0
    t0 = time.perf_counter()
    while done < len(gates) and time.perf_counter() - t0 < seconds:
        g = gates[done]
        O.apply_gate(s, n, int(g["kind"]), int(g["q0"]), int(g["q1"]), g["u"])
        done += 1
    dt = time.perf_counter() - t0
    used = O.threads()
    del s
    return done, dt, used


def cpu_baseline(gates, n, seconds, threads=0, one_core_seconds=0.0):
    """The oracle (plain C, complex128, OpenMP) on this host: gates of the
    same circuit applied one by one until ``seconds`` have elapsed, with
    ``threads`` OpenMP threads (0: the OpenMP default), then the same with one
    thread, the 16-qubit plain workload in full and the 32-qubit precision
    workload's circuit at 28 qubits (a sample)."""
    import oracle as O
    from workloads import config_circuit

    default_threads = O.threads()
    done, dt, used = _oracle_rate(gates, n, seconds, threads)
    out = dict(value=done * float(1 << n) / dt, unit="amplitude-updates/s", cores=used, kind="oracle",
               sample=f"first {done} gates of the same {n}-qubit circuit, complex128, {dt:.1f} s, {used} threads",
               host=cpu_model())
    if one_core_seconds > 0:
        d1, t1, _ = _oracle_rate(gates, n, one_core_seconds, 1)
        out["one_core"] = dict(value=d1 * float(1 << n) / t1, sample=f"first {d1} gates, {t1:.1f} s, 1 thread")
    O.set_threads(threads if threads > 0 else default_threads)
    g1 = config_circuit(1)
    d, t, u = _oracle_rate(g1, 16, 60.0, threads)
    out["plain_16q"] = dict(value=d * float(1 << 16) / t, seconds=t, gates=d, threads=u,
                            workload="16 qubits, 20 layers, CNOT only, in full")
    g3 = config_circuit(3, n=28)
    d, t, u = _oracle_rate(g3, 28, max(1.0, seconds / 3), threads)
    out["precision_28q"] = dict(value=d * float(1 << 28) / t, seconds=t, gates=d, threads=u,
                                workload="the precision workload's layered circuit at 28 qubits, first gates")
    return out


def precision_form(a):
    """32 qubits, 50 layers: the pass form in complex64 and in complex128 on
    the same circuit; per-result error of complex64 against complex128 (FP64
    read-out on both).  Returns the form's sub-object."""
    import numpy as np
    import torch

    from paper_2010_09746_amd import qsim as Q
    from workloads import config_samples, layered_circuit, MASTER_SEED

    n = a.n if a.n != 30 else 32
    layers = a.layers if a.layers != 40 else 50
    gates = layered_circuit(n, layers, MASTER_SEED + 3, cz_every_third=True)
    samples = config_samples(3, n=n)
    upd = len(gates) * float(1 << n)
    out = {}
    states = {}
    steps = max(1, a.form_steps)
    for dt, k in (("c64", a.k), ("c128", a.k)):
        st = Q.State(n, dt)
        pin = a.pinned_c64 if (dt == "c64" and a.pinned_c64 is not None) else a.pinned
        opts = dict(form="pass", k_tile=k, max_swaps=a.r, perm_exec="relabel", pinned=pin)
        st.run(gates, **opts)  # warm-up
        torch.cuda.synchronize()
        ts = []
        for _ in range(steps):
            t0 = time.perf_counter()
            st.set_basis(0)
            st.run(gates, **opts)
            z = st.expect_z()
            amp = st.amplitudes(samples)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ms = float(np.median(ts))
        out[dt] = dict(ms_per_step=ms * 1e3, value=upd / ms, unit="amplitude-updates/s", k_tile=k, pinned=pin,
                       max_swaps=a.r, norm=st.norm())
        states[dt] = (st, z, amp)
        print(f"precision {dt}: {ms * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
    loss, mx = states["c64"][0].fidelity(states["c128"][0])
    err = dict(fidelity_loss=loss, max_abs_amp=mx,
               max_abs_expect_z=float(np.abs(states["c64"][1] - states["c128"][1]).max()),
               max_abs_sampled_amp=float(np.abs(states["c64"][2] - states["c128"][2]).max()),
               norm_c64_minus_1=states["c64"][0].norm() - 1.0, norm_c128_minus_1=states["c128"][0].norm() - 1.0)
    for st, _, _ in states.values():
        st.close()
    states.clear()
    torch.cuda.empty_cache()
    return {"workload": f"random circuit n={n}, {layers} layers ({len(gates)} gates), complex64 bulk with FP64 "
                        f"read-out against complex128 (the complex128 path is checked against the oracle at 28 "
                        f"qubits by the GPU tests)",
            "steps": steps, "c64": out["c64"], "c128": out["c128"], "c64_vs_c128": err,
            "tolerance": {"fidelity_loss": 1e-6, "max_abs_amp": 1e-5},
            "within_tolerance": bool(loss <= 1e-6 and mx <= 1e-5)}


def precision(a):
    r = precision_form(a)
    line = {
        "metric": "amplitude-updates/s", "value": r["c64"]["value"], "unit": "amplitude-updates/s", "n_gpus": 1,
        "steps": r["steps"], "warmup": 1, "ms_per_step": r["c64"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "precision form: " + r["workload"], "parallelism": "1 GPU"},
    }
    line.update({k: v for k, v in r.items() if k not in ("workload", "steps")})
    print(json.dumps(line), flush=True)


def batch_form(a):
    """256 seeded circuits, n uniform in [10, 24], depth uniform in [10, 60],
    complex64, with the autotuner's choice; tuning time reported apart from
    the replay time.  Accuracy against the oracle is covered by the GPU
    tests.  Returns the form's sub-object."""
    import numpy as np

    from paper_2010_09746_amd import autotune, qsim as Q
    from workloads import batch_workload

    wl = batch_workload(count=256)
    circuits = [(n, g) for n, d, g in wl]
    t0 = time.perf_counter()
    if a.no_tune:
        best, table = dict(k_tile=12, max_swaps=16, pinned=4, wg_per_cu=3, chunk=8, use_graph=1), []
    else:
        best, table = autotune.tune_batch(circuits, "c64", reps=2, refresh=a.retune,
                                          log=lambda m: print("tune " + m, file=sys.stderr, flush=True))
    tune_s = time.perf_counter() - t0
    t1 = time.perf_counter()
    b = Q.Batch(circuits, "c64", **best)
    build_s = time.perf_counter() - t1
    b.run()
    b.results()
    ts = []
    for _ in range(max(1, a.form_steps)):
        t2 = time.perf_counter()
        b.run()
        z, nrm = b.results()
        ts.append(time.perf_counter() - t2)
    sec = float(np.median(ts))
    st = b.stats()
    upd = sum(len(g) * float(1 << n) for n, g in circuits)
    b.close()
    print(f"batch: {sec * 1e3:.1f} ms per replay", file=sys.stderr, flush=True)
    return {"workload": "256 seeded layered circuits, n uniform in [10,24], depth uniform in [10,60], complex64; "
                        "output <Z_0> and norm per circuit",
            "value": upd / sec, "unit": "amplitude-updates/s", "ms_per_replay": sec * 1e3,
            "circuits_per_s": len(circuits) / sec, "replays": len(ts),
            "tuned": best, "tune_seconds": tune_s, "tune_candidates": len(table), "build_seconds": build_s,
            "batch_stats": st, "max_norm_error": float(np.abs(nrm - 1).max())}


def batch(a):
    r = batch_form(a)
    line = {
        "metric": "amplitude-updates/s", "value": r["value"], "unit": "amplitude-updates/s", "n_gpus": 1,
        "steps": r["replays"], "warmup": 1, "ms_per_step": r["ms_per_replay"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batching form: " + r["workload"], "parallelism": "1 GPU"},
    }
    line.update({k: v for k, v in r.items() if k not in ("workload", "value", "unit")})
    print(json.dumps(line), flush=True)


def serve_form(a):
    """Seeded Poisson trace (rate, count), n uniform in [12, 30], depth uniform
    in [20, 100], complex64 with FP64 reductions, 200 GB budget, states
    resident; each request returns <Z_q> for all q and 16 sampled amplitudes.
    The accuracy the latencies are quoted at is measured against complex128
    runs of the same circuits.  Returns the form's sub-object."""
    import numpy as np

    from paper_2010_09746_amd.serving import Server, latency_summary
    from workloads import layered_circuit, request_trace

    trace = request_trace(count=a.requests, rate=a.rate)
    reqs = [dict(r, gates=layered_circuit(r["n"], r["depth"], r["seed"])) for r in trace]
    srv = Server("c64", k_tile=a.serve_k, max_swaps=16,
                 pinned=a.pinned_c64 if a.pinned_c64 is not None else a.pinned, hbm_budget=200e9, max_slots=256,
                 wg_per_cu=a.serve_wg, solo_tiles=a.serve_solo_tiles)
    # warm-up: one small request outside the measured trace
    srv.serve([dict(id=-1, arrival=0.0, n=12, gates=layered_circuit(12, 4, 1), samples=[0])], realtime=False)
    res, rec = srv.serve(reqs, realtime=True, log=lambda m: print("serve " + m, file=sys.stderr, flush=True))
    st = latency_summary(rec)
    nerr = [abs(res[r["id"]]["norm"] - 1.0) for r in reqs]
    main_stats = dict(srv.last_stats)
    sweep = []
    for rate in [float(x) for x in a.rate_sweep.split(",") if x.strip()]:
        tr = request_trace(count=a.sweep_requests, rate=rate)
        rq = [dict(r, gates=layered_circuit(r["n"], r["depth"], r["seed"])) for r in tr]
        _, rc = srv.serve(rq, realtime=True)
        sweep.append(dict(rate=rate, **latency_summary(rc)))
    srv.close()
    accuracy = served_accuracy(reqs, res, a.serve_k, count=a.accuracy_requests)
    print(f"serve: p50 {st['p50_s']:.2f} s, p99 {st['p99_s']:.2f} s, {st['throughput_req_s']:.1f} requests/s",
          file=sys.stderr, flush=True)
    return {"workload": f"Poisson trace of {a.requests} requests at {a.rate}/s, n uniform in [12,30], depth "
                        f"uniform in [20,100], complex64 with FP64 reductions, 200 GB budget, <Z_q> all q + 16 "
                        f"sampled amplitudes per request; tile qubits {a.serve_k}",
            "p50_s": st["p50_s"], "p99_s": st["p99_s"], "throughput_req_s": st["throughput_req_s"],
            "latency": st, "server": main_stats, "max_norm_error": float(np.max(nerr)), "accuracy": accuracy,
            "rate_sweep": sweep}


def serve(a):
    r = serve_form(a)
    line = {
        "metric": "served p50/p99 latency", "value": r["p99_s"], "unit": "s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": r["latency"]["makespan_s"] * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving form: " + r["workload"], "parallelism": "1 GPU"},
    }
    line.update({k: v for k, v in r.items() if k != "workload"})
    print(json.dumps(line), flush=True)


def served_accuracy(reqs, res, k, count=64):
    """Error of the served complex64 results against complex128 runs of the
    same circuits (pass form, one at a time), on `count` requests spread over
    the trace: max |d<Z_q>| over all q and max |d amp| over the sampled
    amplitudes."""
    import numpy as np

    from paper_2010_09746_amd import qsim as Q

    pick = reqs[:: max(1, len(reqs) // count)][:count]
    dz = da = 0.0
    for r in pick:
        ref = Q.State(r["n"], "c128")
        ref.run(r["gates"], form="pass", k_tile=min(k, r["n"]), max_swaps=16, pinned=3, perm_exec="relabel")
        z = ref.expect_z()
        amps = ref.amplitudes(np.asarray(r["samples"], dtype=np.uint64))
        ref.close()
        got = res[r["id"]]
        dz = max(dz, float(np.abs(z - got["z"]).max()))
        da = max(da, float(np.abs(amps[: len(got["amps"])] - got["amps"]).max()))
    return {"reference": "complex128 pass form, same circuit, run alone", "requests_checked": len(pick),
            "qubits": [r["n"] for r in pick], "max_abs_expect_z": dz, "max_abs_amp": da}


def _study_line(metric, value, unit, ms, cfg, body, hib=True, dtype="f64"):
    line = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": 1, "warmup": 1,
            "ms_per_step": ms, "higher_is_better": hib, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": dict(cfg, parallelism="1 GPU")}
    line["result"] = body
    print(json.dumps(line), flush=True)


def kernels(a):
    """Each single-purpose kernel at 30 qubits, complex128."""
    from paper_2010_09746_amd import studies

    r = studies.kernel_sweep(n=a.n, dtype=a.dtype)
    u = [x["gbs"] for x in r["plain_u_per_target"]]
    _study_line("one-qubit gate bandwidth (median over targets)", float(sorted(u)[len(u) // 2]), "GB/s",
                sum(x["avg_ms"] for x in r["plain_u_per_target"]) / len(u),
                {"workload": f"single kernels at n={a.n} {a.dtype}: one-qubit gate on each target, CX/CZ on "
                             f"low/high pairs, position exchanges of 1..8 pairs, one fused tile pass (k=12, 13) "
                             f"carrying 1..48 gates, <Z_q> read-out"}, r)


def qft(a):
    """QFT (checked against its closed form) and the QFT-like circuit, 30 qubits."""
    from paper_2010_09746_amd import studies

    r = studies.qft_study(n=a.n, dtype=a.dtype, k=a.k, r=a.r, pinned=a.pinned)
    _study_line("amplitude-updates/s", r["qft"]["amp_updates_per_s"], "amplitude-updates/s", r["qft"]["ms"],
                {"workload": f"QFT on a basis state and the QFT-like circuit (CNOT for each controlled phase), "
                             f"n={a.n} {a.dtype}, pass form k={a.k} r={a.r}"}, r)


def random_family(a):
    """The paper's random family (Section 4): plain against pass form over p."""
    from paper_2010_09746_amd import studies

    n = a.n if a.n != 30 else 28
    r = studies.random_family_study(n=n, dtype=a.dtype, k=a.k, r=a.r, pinned=a.pinned)
    best = max(x["speedup"] for x in r["rows"])
    _study_line("pass-form speedup over plain (best p)", best, "x", sum(x["pass_ms"] for x in r["rows"]),
                {"workload": f"random family: 30n gates, CNOT with probability p else H or Y, n={n} {a.dtype}, "
                             f"pass form k={a.k} r={a.r} against one launch per gate"}, r)


def ablation(a):
    """The 30-qubit workload under Algorithm 1 as printed (r = 1), the bundled
    pass over tile sizes 10..14, fusion without the pass (r = 0) and gates on
    the lowest thread bits through lane exchanges."""
    from paper_2010_09746_amd import studies

    r = studies.ablation_study(n=a.n, dtype=a.dtype, layers=a.layers, r=a.r, k_ref=a.k)
    best = min(r["rows"], key=lambda x: x["ms"])
    ref = next(x for x in r["rows"] if x["variant"] == "fusion without pass")
    _study_line("pass speedup over fusion without the pass", ref["ms"] / best["ms"], "x", best["ms"],
                {"workload": f"layered circuit n={a.n} {a.dtype}, {r['gates']} gates: r=0 and r=1 at k={a.k}, "
                             f"r={a.r} at k=10..14, lane gates at k={a.k}; device time of one run each"}, r)


def costmodel_form(a):
    """Measured cost model: predict every candidate (k, r, register bits) for
    the 30-qubit workload, run a spread of them, and report how well the
    prediction ranks them and what the predicted choice costs.  Then the pass
    deciding by the same measured costs (each PermuteQubits' chain prefix
    against a gate run on its own) beside Algorithm 1's step function, on the
    30-qubit workload with relabelled placements and, with the paper's moved
    placements and single exchanges, on that workload and the paper's random
    family (p = 1, 28 qubits): predicted and measured device time."""
    import numpy as np

    from paper_2010_09746_amd import costmodel, qsim as Q
    from workloads import config_circuit, paper_random_circuit

    gates = config_circuit(2, n=a.n, layers=a.layers)
    cm = costmodel.CostModel(a.dtype, n_cal=a.cal_n)
    t0 = time.perf_counter()
    best, table = cm.choose(gates, a.n, ks=(9, 10, 11, 12, 13), rs=(1, 4, 8, 16), reg_bits=(3, 4))
    choose_s = time.perf_counter() - t0
    pick = table[:3] + table[3::max(1, (len(table) - 3) // 5)][:5]
    for row in pick:
        row["measured_ms"] = costmodel.measure_ms(gates, a.n, a.dtype, row["opts"], reps=1)
    pm = [r["predicted_ms"] for r in pick]
    mm = [r["measured_ms"] for r in pick]
    chosen = pick[0]["measured_ms"]
    in_pass = []
    n_rf = a.n - 2
    rf = {p: paper_random_circuit(n_rf, 30 * n_rf, p, 20100946 + 8) for p in (0.3, 1.0)}
    cases = [("layered", gates, a.n, dict(best))]
    for p, g in rf.items():
        # the best global options for this circuit (relabelled placements)
        b, _ = cm.choose(g, n_rf, ks=(11, 12, 13), rs=(8, 16), reg_bits=(4,))
        cases.append((f"random family p={p}", g, n_rf, dict(b)))
    cases += [("layered, moved placements, r=1", gates, a.n,
               dict(k_tile=a.k, max_swaps=1, pinned=0, perm_exec="move", reg_bits=0)),
              ("random family p=1, moved placements, r=1", rf[1.0], n_rf,
               dict(k_tile=a.k, max_swaps=1, pinned=0, perm_exec="move", reg_bits=0))]
    for name, g, n, opts in cases:
        row = {"workload": name, "n": n, "opts": opts}
        costs = cm.pass_costs(n, opts["k_tile"], opts["reg_bits"], opts["perm_exec"])
        for tag, c in (("step", None), ("costed", cm.as_struct(costs))):
            ms, counts = cm.predict(g, n, costed=c is not None, **opts)
            P = Q.Program(g, n, a.dtype, form="pass", costs=c, **opts)
            prog_stats = {k: P.stats()[k] for k in ("n_perm", "n_global", "n_tile_passes")}
            P.close()
            row[tag] = dict(predicted_ms=ms, measured_ms=costmodel.measure_ms(g, n, a.dtype, opts, reps=3, costs=c),
                            **prog_stats)
        row["pass_costs"] = costs
        in_pass.append(row)
        print(f"costed pass, {name}: step {row['step']['measured_ms']:.1f} ms, costed "
              f"{row['costed']['measured_ms']:.1f} ms", file=sys.stderr, flush=True)
    _study_line("cost-model regret (chosen / best measured)", chosen / min(mm), "x", chosen,
                {"workload": f"cost model on the layered circuit n={a.n} {a.dtype} ({len(gates)} gates): "
                             f"{len(table)} candidates predicted, {len(pick)} measured; the pass deciding by "
                             f"the measured costs against Algorithm 1's step function"},
                {"chosen": best, "choose_seconds": choose_s, "rank_correlation": costmodel.rank_correlation(pm, mm),
                 "measured": pick, "calibration": {f"k{k}_rb{rb}": v for (k, rb), v in cm.tile_costs.items()},
                 "launch_costs": cm.launch_costs, "in_pass_choices": in_pass,
                 "fit_residual": {f"k{k}_rb{rb}": v for (k, rb), v in cm.fit_residual.items()}},
                hib=False)


def main():
    a = parse()
    if a.traffic_from:
        return traffic_from_counters(a)
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if a.form == "precision":
        return precision(a)
    if a.form == "batch":
        return batch(a)
    if a.form == "kernels":
        return kernels(a)
    if a.form == "qft":
        return qft(a)
    if a.form == "random-family":
        return random_family(a)
    if a.form == "costmodel":
        return costmodel_form(a)
    if a.form == "ablation":
        return ablation(a)
    if a.form == "serve":
        return serve(a)

    import numpy as np
    import torch

    from paper_2010_09746_amd import qsim as Q
    from workloads import config_samples, layered_circuit, MASTER_SEED

    n, dt = a.n, a.dtype
    gates = layered_circuit(n, a.layers, MASTER_SEED + 2, cz_every_third=True)
    samples = config_samples(2, n=n)
    amp_updates = len(gates) * float(1 << n)
    dev = Q.qs_device_info()
    torch.cuda.init()
    st = Q.State(n, dt)
    stream = torch.cuda.current_stream()

    pass_opts = dict(form="pass", k_tile=a.k, max_swaps=a.r, perm_exec=a.perm_exec, pinned=a.pinned,
                     reg_bits=a.reg_bits)
    costs, cost_info = None, None
    if a.costed:
        from paper_2010_09746_amd import costmodel

        t0 = time.perf_counter()
        cm = costmodel.CostModel(dt, n_cal=a.cal_n, perm_exec=a.perm_exec, pinned=a.pinned)
        pc = cm.pass_costs(n, a.k, a.reg_bits, a.perm_exec)
        costs = cm.as_struct(pc)
        cost_info = dict(calibration_seconds=time.perf_counter() - t0, n_cal=a.cal_n, pass_costs_ms=pc)
        torch.cuda.empty_cache()

    def step(opts):
        st.set_basis(0)
        st.run(gates, costs=costs if opts.get("form") == "pass" else None, **opts)
        z = st.expect_z()
        amp = st.amplitudes(samples)
        return z, amp

    def timed(opts, warmup, steps):
        for _ in range(warmup):
            step(opts)
        torch.cuda.synchronize()
        Q.qs_profile_read()  # drop warm-up records
        Q.qs_profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            out = step(opts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        Q.qs_profile_enable(False)
        prof = Q.qs_profile_read()
        return el / steps, prof, out

    prog = Q.Program(gates, n, dt, costs=costs, **pass_opts)
    pstats = prog.stats()
    prog.close()

    ms_pass, prof_pass, (z_pass, amp_pass) = timed(pass_opts, a.warmup, a.steps)
    print(f"pass form: {ms_pass * 1e3:.1f} ms/step", file=sys.stderr, flush=True)

    plain = None
    if a.plain_steps > 0:
        ms_plain, prof_plain, (z_plain, amp_plain) = timed(dict(form="plain"), 0, a.plain_steps)
        agree = float(np.abs(amp_plain - amp_pass).max())
        plain = dict(value=amp_updates / ms_plain, ms_per_step=ms_plain * 1e3,
                     max_abs_diff_vs_pass=agree,
                     kernels={k: dict(launches=v["launches"], avg_ms=v["avg_ms"],
                                      achieved_gbs=v["bytes"] / (v["total_ms"] * 1e-3) / 1e9)
                              for k, v in prof_plain.items()})
        print(f"plain form: {ms_plain * 1e3:.1f} ms/step", file=sys.stderr, flush=True)

    if a.copy_calib > 0:
        src = torch.ones(a.copy_calib << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    tile = prof_pass.get("tile_pass")
    roofline = None
    if tile:
        per_launch = tile["bytes"] / tile["launches"]
        achieved = per_launch / (tile["avg_ms"] * 1e-3) / 1e9
        traffic = None
        if os.path.exists(a.traffic_json):
            try:
                tj = json.load(open(a.traffic_json))
                key = f"n{n}_{dt}_k{a.k}_r{a.r}_{a.perm_exec}"
                # counters only describe the kernel they were taken on
                if tj.get("kernel_source_sha1") == kernel_source_hash():
                    traffic = tj.get("bytes_per_launch", {}).get(key)
            except Exception:
                traffic = None
        # the tile pass is priced against both ceilings; the one whose floor is
        # higher (the binding one) is reported, the other is kept beside it
        n_1q = int(sum(1 for gk in gates["kind"] if gk == 0))
        flops_per_launch = n_1q * float(1 << n) * FLOPS_PER_AMP_1Q / max(1.0, tile["launches"] / a.steps)
        tflops = flops_per_launch / (tile["avg_ms"] * 1e-3) / 1e12
        hbm = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                   algorithmic_bytes_per_launch=per_launch)
        alu = dict(bound="alu", achieved=tflops, peak=VALU_PEAK_TFLOPS, unit="TFLOP/s",
                   frac=tflops / VALU_PEAK_TFLOPS, algorithmic_flops_per_launch=flops_per_launch)
        main, other = (alu, hbm) if alu["frac"] > hbm["frac"] else (hbm, alu)
        roofline = dict(main, traffic=traffic, kernel="k_tile", avg_ms=tile["avg_ms"],
                        launches_per_step=tile["launches"] / a.steps, other_ceiling=other)

    torch.cuda.synchronize()
    st.close()
    del st
    torch.cuda.empty_cache()
    cpu = None
    if a.cpu_seconds > 0:
        cpu = cpu_baseline(gates, n, a.cpu_seconds, a.cpu_threads, a.cpu_one_core_seconds)

    # the other forms of the metric, each timed after the headline
    forms = {}
    runners = {"precision": precision_form, "batch": batch_form, "serve": serve_form}
    for name in [x.strip() for x in a.forms.split(",") if x.strip()]:
        if name not in runners:
            forms[name] = {"error": "unknown form"}
            continue
        t0 = time.perf_counter()
        try:
            forms[name] = runners[name](a)
        except Exception as e:  # reported in the line; the headline stands
            forms[name] = {"error": f"{type(e).__name__}: {e}"}
        forms[name]["wall_seconds"] = time.perf_counter() - t0
        torch.cuda.empty_cache()

    value = amp_updates / ms_pass
    line = {
        "metric": "amplitude-updates/s",
        "value": value,
        "unit": "amplitude-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_pass * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if dt == "c128" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"random circuit, n={n} {dt}, {a.layers} layers of Haar U(2) on every qubit + CNOT on a "
                        f"random perfect matching (CZ every third layer), {len(gates)} gates; read-out <Z_q> all q "
                        f"+ {len(samples)} sampled amplitudes",
            "form": f"permutation pass k={a.k} r={a.r} pinned={a.pinned} perm_exec={a.perm_exec}"
                    + (" (PermuteQubits chosen by the measured cost model)" if a.costed else ""),
            "parallelism": "1 GPU",
        },
        "pass_stats": {k: pstats[k] for k in ("n_perm", "n_global", "n_swaps", "n_tile_passes", "n_move_passes",
                                              "n_remaps", "compile_ms")},
        "cost_model": cost_info,
        "kernels": {k: dict(launches=v["launches"], avg_ms=v["avg_ms"],
                            achieved_gbs=v["bytes"] / max(v["total_ms"], 1e-9) / 1e6)
                    for k, v in prof_pass.items()},
        "plain": plain,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "device": dev,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
