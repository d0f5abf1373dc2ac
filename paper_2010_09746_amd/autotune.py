"""Autotuner for the batching form.

Chooses the largest tile size k (each circuit uses min(n, k)), the
exchanges per permutation r (which sets the fusion depth: gates per tile
pass), the persistent launch shape (workgroups per CU, tiles per work item)
and the pinned positions, by timing graph replays of the actual batch on the
device.  Results are cached in JSON keyed by device name, amplitude type and a
signature of the workload (qubit-count histogram and gate count).
"""

from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import qsim as Q

DEFAULT_CACHE = os.environ.get("QSIM_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "qsim_autotune.json"))


def signature(circuits, dtype) -> str:
    ns = sorted(int(n) for n, _ in circuits)
    ng = sum(len(g) for _, g in circuits)
    h = hashlib.sha1(json.dumps([ns, ng, str(dtype)]).encode()).hexdigest()[:16]
    return h


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except Exception:
        return {}


def _save(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1)
        os.replace(tmp, path)
    except OSError:
        pass


def _time(circuits, dtype, opts, reps):
    b = Q.Batch(circuits, dtype, **opts)
    try:
        b.run()
        b.results()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            b.run()
            b.results()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), b.stats()
    finally:
        b.close()


def candidates(n_min: int, dtype):
    """Largest tile k (circuits of at most k qubits run as one tile) and the
    exchange bundle r, which sets the fusion depth (gates per pass)."""
    for k in (10, 11, 12):
        for r in (4, 8, 16):
            yield dict(k_tile=k, max_swaps=r)


def tune_batch(circuits, dtype="c64", cache_path=DEFAULT_CACHE, reps=2, refresh=False, log=None):
    """Returns (best options dict, table of (options, seconds)).  Stage 1
    searches the largest tile k and r with a default launch shape; stage 2
    the launch shape (workgroups per CU, tiles per work item); stage 3 the
    pinned positions."""
    dev = Q.qs_device_info()["name"]
    key = f"{dev}|{dtype}|queue|{signature(circuits, dtype)}"
    cache = _load(cache_path)
    if not refresh and key in cache:
        return cache[key]["best"], cache[key]["table"]
    n_min = min(int(n) for n, _ in circuits)
    table = []

    def trial(o):
        try:
            t, _ = _time(circuits, dtype, o, reps)
        except Q.QsimError as e:
            if log:
                log(f"skip {o}: {e}")
            return
        table.append((o, t))
        if log:
            log(f"{o} -> {t * 1e3:.2f} ms")

    base = dict(pinned=3 if Q.elem_bytes(dtype) == 16 else 4, wg_per_cu=4, chunk=4, use_graph=1)
    for c in candidates(n_min, dtype):
        trial(dict(base, **c))
    best = min(table, key=lambda x: x[1])[0]
    for wg in (3, 4, 5):
        for ch in (1, 2, 4, 8):
            o = dict(best, wg_per_cu=wg, chunk=ch)
            if o != best:
                trial(o)
    best = min(table, key=lambda x: x[1])[0]
    # a 128-byte line is 8 complex128 or 16 complex64 amplitudes
    for pin in (3, 4):
        o = dict(best, pinned=pin)
        if o != best:
            trial(o)
    best = min(table, key=lambda x: x[1])[0]
    cache[key] = dict(best=best, table=table)
    _save(cache_path, cache)
    return best, table
