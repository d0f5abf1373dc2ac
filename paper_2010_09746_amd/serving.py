"""Serving form: a request loop with continuous batching on one GPU.

Requests (circuits with their arrival times) are compiled on host threads as
they arrive, admitted in arrival order whenever the HBM budget and a slot
allow, and kept resident on the device.  Each step of the native server
(``qs_server_step_launch`` / ``_wait``) runs the next tile pass of every
resident request, so the work of requests that arrived at different times
overlaps on the device; two steps are kept in flight, so the host collects
and admits while the device works.  A request leaves after its last pass,
with <Z_q> for every qubit and its sampled amplitudes (FP64 accumulation)
copied back in the same step.

State buffers come from PyTorch's allocator; compiled tables live in the
server's own device arena.
"""

from __future__ import annotations

import collections
import concurrent.futures as cf
import time

import numpy as np
import torch

from . import qsim as Q


class Server:
    def __init__(self, dtype="c64", k_tile=10, max_swaps=16, pinned=3, reg_bits=0, chunk=8, wg_per_cu=16,
                 hbm_budget=200e9, max_slots=256, max_samples=16, compile_workers=8, solo_tiles=None):
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        self.dtype = dtype
        self.eb = Q.elem_bytes(dtype)
        self.k_tile, self.max_swaps, self.pinned, self.reg_bits = k_tile, max_swaps, pinned, reg_bits
        self.max_samples = max_samples
        opts = Q.make_batch_opts(k_tile=k_tile, max_swaps=max_swaps, pinned=pinned, reg_bits=reg_bits,
                                 chunk=chunk, wg_per_cu=wg_per_cu, use_graph=0)
        self.h = Q.qs_server_create(dtype, opts, int(hbm_budget), max_slots, max_samples)
        if solo_tiles is not None:  # else the library's default
            try:
                Q.qs_server_set_solo_tiles(self.h, solo_tiles)
            except Exception:
                Q.qs_server_destroy(self.h)
                self.h = None
                raise
        self.pool = cf.ThreadPoolExecutor(max_workers=compile_workers)

    def close(self):
        if getattr(self, "h", None):
            Q.qs_server_destroy(self.h)
            self.h = None
        self.pool.shutdown(wait=True)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def compile(self, gates, n) -> Q.Program:
        return Q.Program(gates, n, self.dtype, form="pass", k_tile=self.k_tile, max_swaps=self.max_swaps,
                         pinned=self.pinned, perm_exec="relabel", reg_bits=self.reg_bits)

    def serve(self, requests, realtime=True, log=None):
        """requests: dicts with id, arrival (s), n, gates, samples.  Returns
        (results {id: dict(z, amps, norm)}, records {id: dict(arrival, admit,
        done, n, gates)}).  Up to two steps are in flight: the next step is
        enqueued before the previous one is waited for, so the device has
        queued work while the host collects results and admits requests."""
        reqs = sorted(requests, key=lambda r: r["arrival"])
        total = len(reqs)
        waiting = collections.deque()      # arrived, not admitted: (req, future)
        running = {}                       # server id -> (req, buffer, program, samples)
        left = {}                          # server id -> passes not yet enqueued
        results, rec = {}, {}
        nxt = 0
        inflight = 0
        t0 = time.perf_counter()
        max_resident = 0
        steps = 0
        while len(results) < total:
            now = time.perf_counter() - t0
            while nxt < total and (not realtime or reqs[nxt]["arrival"] <= now):
                r = reqs[nxt]
                waiting.append((r, self.pool.submit(self.compile, r["gates"], r["n"])))
                rec[r["id"]] = dict(arrival=r["arrival"] if realtime else 0.0, n=r["n"], gates=len(r["gates"]))
                nxt += 1
            # admission in arrival order
            while waiting and waiting[0][1].done() and Q.qs_server_fits(self.h, waiting[0][0]["n"]):
                r, fut = waiting.popleft()
                prog = fut.result()
                nbytes = self.eb << r["n"]
                try:
                    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
                except torch.cuda.OutOfMemoryError:
                    torch.cuda.empty_cache()
                    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
                smp = np.asarray(r["samples"][: self.max_samples], dtype=np.uint64)
                try:
                    sid = Q.qs_server_admit(self.h, prog.h, buf.data_ptr(), nbytes, smp)
                except Q.QsimError as e:
                    # QS_ERR_BUDGET with requests resident: the server's table
                    # arena is full until one of them leaves
                    if e.code != -3 or not running:
                        raise
                    del buf
                    waiting.appendleft((r, fut))
                    break
                running[sid] = (r, buf, prog, len(smp))
                left[sid] = max(1, prog.stats()["n_tile_passes"])
                rec[r["id"]]["admit"] = time.perf_counter() - t0
            max_resident = max(max_resident, len(running))
            if inflight < 2 and any(v > 0 for v in left.values()):
                Q.qs_server_step_launch(self.h)
                for sid in left:
                    left[sid] = max(0, left[sid] - 1)
                inflight += 1
                steps += 1
                if inflight < 2:
                    continue  # enqueue the next step before waiting for this one
            if inflight:
                inflight -= 1
                for sid in Q.qs_server_step_wait(self.h):
                    r, buf, prog, cnt = running.pop(sid)
                    left.pop(sid, None)
                    z, amps, nrm = Q.qs_server_result(self.h, sid, r["n"], cnt)
                    Q.qs_server_release(self.h, sid)
                    del buf
                    prog.close()
                    results[r["id"]] = dict(z=z, amps=amps, norm=nrm)
                    rec[r["id"]]["done"] = time.perf_counter() - t0
                    if log and len(results) % 50 == 0:
                        log(f"{len(results)}/{total} done at {rec[r['id']]['done']:.2f} s, "
                            f"{len(running)} resident, {len(waiting)} waiting")
            elif nxt < total and realtime:
                time.sleep(min(0.001, max(0.0, reqs[nxt]["arrival"] - (time.perf_counter() - t0))))
            else:
                time.sleep(0.0002)
        self.last_stats = dict(steps=steps, max_resident=max_resident, makespan=time.perf_counter() - t0)
        return results, rec


def latency_summary(rec, results=None):
    lat = np.array([v["done"] - v["arrival"] for v in rec.values()])
    que = np.array([v["admit"] - v["arrival"] for v in rec.values()])
    svc = np.array([v["done"] - v["admit"] for v in rec.values()])
    span = max(v["done"] for v in rec.values()) - min(v["arrival"] for v in rec.values())
    upd = sum(v["gates"] * float(1 << v["n"]) for v in rec.values())
    return dict(requests=len(rec), p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_queue_s=float(que.mean()), p99_queue_s=float(np.percentile(que, 99)),
                mean_service_s=float(svc.mean()), p50_service_s=float(np.percentile(svc, 50)),
                throughput_req_s=len(rec) / span, amp_updates_per_s=upd / span, makespan_s=span)
