"""Serving loop over the C ABI: continuous batching of render requests of
mixed resolutions and scenes, resident fields, HBM-budget admission and
hipGraph replay per size bucket, with p50/p99 latency beside throughput.

* Fields are loaded once and stay resident (vrn_load_field); their device
  bytes count against the budget.
* A *slot* is a HIP stream with its own 4 KiB workspace and a device camera
  buffer; up to ``n_slots`` requests run concurrently, each on its own slot,
  so their kernels overlap on the device.
* Requests that arrive while others are on the GPU wait in a queue and are
  admitted as slots and memory free up (continuous batching): when a slot is
  free, pending single-camera requests of the same scene and resolution are
  merged into one launch of up to ``max_batch`` cameras.
* A *bucket* is (scene, W, H, n_cams, dtype).  Each slot keeps, per bucket,
  a small ring of output buffers, each with its own captured HIP graph of
  the render kernel (vrn_render_device_cams reads the cameras from the
  slot's device buffer, so a replay renders whatever cameras were copied in
  before it).  A finished request hands out views of its ring buffer, not a
  copy; the buffer stays with the request until ``Request.release()``.
  Every ring buffer, held or free, counts against the HBM budget; free
  buffers of idle buckets are evicted least-recently-used.
* A request may carry a timeout: one still queued at its deadline is never
  launched, and one that completes after it is failed and its buffer
  returned.  ``Request.cancel()`` removes a queued request, or discards the
  result of a running one when it completes.
* Latency is measured on the host clock from a request's arrival to the
  moment its completion event is observed.

Every render runs in the library's HIP kernels; this module only
schedules.
"""
from __future__ import annotations

import argparse
import collections
import ctypes
import json
import sys
import threading
import time

import numpy as np

from . import capi

CAM_BYTES = 72  # sizeof(vrn_camera)


class ServeError(RuntimeError):
    pass


class ServeTimeout(ServeError):
    pass


class ServeCancelled(ServeError):
    pass


class Request:
    __slots__ = ("rid", "scene", "cams", "W", "H", "t_arrival", "t_start", "t_done", "event", "error", "done",
                 "deadline", "keep", "cam_blob", "cancelled", "_out", "_off", "_server")

    def __init__(self, server, rid, scene, cams, W, H, t_arrival, deadline, keep, cam_blob):
        self._server = server
        self.rid, self.scene, self.cams, self.W, self.H = rid, scene, cams, W, H
        self.t_arrival = t_arrival
        self.deadline = deadline
        self.keep = keep
        self.cam_blob = cam_blob
        self.t_start = self.t_done = None
        self.event = None
        self.error = None
        self.cancelled = False
        self._out = None
        self._off = 0
        self.done = threading.Event()

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival

    @property
    def result(self):
        """(rgba [n_cams, H, W, 4], nsamples [n_cams, H, W]): views of the
        request's ring buffer, valid until release(); None if the request
        failed, was cancelled, or its buffer was released."""
        out = self._out
        if out is None or self.error is not None:
            return None
        k = len(self.cams)
        return out.rgba[self._off:self._off + k], out.ns[self._off:self._off + k]

    def release(self):
        """Return the request's output buffer to its ring."""
        self._server._release(self)

    def cancel(self) -> bool:
        """Cancel the request: a queued one is never launched; a running one
        has its result discarded when it completes.  False once done."""
        return self._server._cancel(self)


class _Out:
    """One ring buffer of a bucket: outputs plus the graph that renders into them."""
    __slots__ = ("rgba", "ns", "graph", "holders", "bytes", "last_use")

    def __init__(self, rgba, ns, graph, nbytes):
        self.rgba, self.ns, self.graph = rgba, ns, graph
        self.holders = 0
        self.bytes = nbytes
        self.last_use = time.perf_counter()


class _Slot:
    def __init__(self, torch, device, ws_bytes):
        self.stream = torch.cuda.Stream(device=device)
        self.ws = torch.zeros(ws_bytes, dtype=torch.uint8, device=device)
        self.cams = torch.zeros(capi.MAX_CAMS * CAM_BYTES, dtype=torch.uint8, device=device)
        self.cams_host = torch.zeros(capi.MAX_CAMS * CAM_BYTES, dtype=torch.uint8).pin_memory()
        self.cams_host_ptr = self.cams_host.data_ptr()
        self.rings: "collections.OrderedDict[tuple, list]" = collections.OrderedDict()
        self.busy = None          # list of requests in flight
        self.event = torch.cuda.Event()   # recorded after each launch; reused


class Server:
    def __init__(self, fields: dict, hbm_budget_bytes: int, n_slots: int = 4, compute: str = "f16",
                 use_graphs: bool = True, max_batch: int = 4, device: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.compute = compute
        self.use_graphs = use_graphs
        self.max_batch = max_batch
        self.budget = int(hbm_budget_bytes)
        self.ctx = capi.vrn_create(device, self.budget)
        self.fids = {}
        self._out_bytes = {}
        self.field_bytes = 0
        for name, f in fields.items():
            fid = capi.vrn_load_field(self.ctx, f)       # VRN_ERR_BUDGET if fields alone exceed it
            self.fids[name] = fid
            self.field_bytes += capi.vrn_field_bytes(self.ctx, fid)
        ws_bytes = capi.vrn_workspace_bytes(self.ctx)
        self.slots = [_Slot(torch, self.device, ws_bytes) for _ in range(n_slots)]
        for s in self.slots:
            capi.vrn_workspace_init(self.ctx, s.ws, stream=s.stream)
        self.fixed_bytes = self.field_bytes + n_slots * (ws_bytes + capi.MAX_CAMS * CAM_BYTES)
        if self.fixed_bytes > self.budget:
            raise ServeError("resident fields and slot workspaces exceed the HBM budget")
        self.pending = collections.deque()
        self._claimed = 0           # batches taken from `pending` and not yet launched or requeued
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        self.done_list = []
        self._rid = 0
        self._stop = threading.Event()
        self._thread = None
        torch.cuda.synchronize()

    # ---------------------------------------------------------------- API
    def out_bytes(self, n_cams, W, H):
        """Device bytes of one output buffer (RGBA + sample counts): the
        library's admission size of such a render less the workspace, which
        every slot already holds."""
        key = (n_cams, W, H)
        b = self._out_bytes.get(key)
        if b is None:
            fid = next(iter(self.fids.values()))
            b = (capi.vrn_render_bytes(self.ctx, fid, n_cams, W, H, self.compute)
                 - capi.vrn_workspace_bytes(self.ctx))
            self._out_bytes[key] = b
        return b

    def submit(self, scene, cams, W, H, t_arrival=None, timeout_s=None, keep=True) -> Request:
        """Queue a render request.  timeout_s bounds arrival -> completion;
        keep=False returns the output buffer to its ring as soon as the
        request completes (latency-only clients)."""
        if scene not in self.fids:
            raise ServeError(f"unknown scene {scene}")
        if len(cams) > capi.MAX_CAMS:
            raise ServeError("too many cameras in one request")
        arr = capi.make_cameras(cams, H)
        lib = capi.load_library()
        if lib.vrn_check_cameras(arr, len(cams), W, H) != capi.VRN_OK:
            raise ServeError("invalid cameras: " + lib.vrn_last_error().decode())
        if self.fixed_bytes + self.out_bytes(len(cams), W, H) > self.budget:
            raise ServeError("request can never fit the HBM budget")
        blob = bytes(arr)
        t = time.perf_counter() if t_arrival is None else t_arrival
        deadline = None if timeout_s is None else t + float(timeout_s)
        with self.cv:
            self._rid += 1
            r = Request(self, self._rid, scene, cams, W, H, t, deadline, keep, blob)
            self.pending.append(r)
            self.cv.notify()
        return r

    def warmup(self, shapes):
        """Allocate and capture, on every slot, one ring buffer per bucket of
        every scene for the given (W, H, n_cams) shapes, so that no capture
        (and its device synchronisation) happens while requests are being
        served.  Stops at the HBM budget."""
        for slot in self.slots:
            for scene in self.fids:
                for (W, H, n) in shapes:
                    key = (scene, W, H, n, self.compute)
                    if slot.rings.get(key):
                        continue
                    if self._used_bytes() + self.out_bytes(n, W, H) > self.budget:
                        return
                    self._new_out(slot, key, n, W, H)
        self.torch.cuda.synchronize()

    def start(self):
        self._stop.clear()
        self._thread = threading.Thread(target=self._loop, daemon=True)
        self._thread.start()

    def stop(self, drain=True):
        if drain:
            while True:
                with self.lock:
                    idle = (not self.pending and self._claimed == 0
                            and all(s.busy is None for s in self.slots))
                if idle:
                    break
                time.sleep(0.0005)
        self._stop.set()
        with self.cv:
            self.cv.notify()
        if self._thread:
            self._thread.join()

    def close(self):
        self.stop(drain=False)
        self.torch.cuda.synchronize()
        for s in self.slots:
            s.rings.clear()
        for fid in self.fids.values():
            capi.vrn_unload_field(self.ctx, fid)
        capi.vrn_destroy(self.ctx)

    def held_bytes(self):
        """Device bytes of ring buffers currently held by requests: in flight,
        or finished and not yet released."""
        with self.lock:
            return sum(o.bytes for s in self.slots for ring in s.rings.values() for o in ring if o.holders)

    # ------------------------------------------------------------ internals
    def _used_bytes(self):
        return self.fixed_bytes + sum(o.bytes for s in self.slots for ring in s.rings.values() for o in ring)

    def _new_out(self, slot, key, n_cams, W, H):
        torch = self.torch
        rgba = torch.zeros((n_cams, H, W, 4), dtype=torch.float32, device=self.device)
        ns = torch.zeros((n_cams, H, W), dtype=torch.int32, device=self.device)
        graph = None
        if self.use_graphs:
            # the graph uploads the slot's pinned cameras (a copy node, so a
            # replay takes whatever cameras were written there) and renders
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            nb = n_cams * CAM_BYTES
            with torch.cuda.graph(graph, stream=slot.stream, capture_error_mode="thread_local"):
                slot.cams[:nb].copy_(slot.cams_host[:nb], non_blocking=True)
                capi.vrn_render_device_cams(self.ctx, self.fids[key[0]], slot.cams, n_cams, W, H, rgba, ns,
                                            self.compute, workspace=slot.ws, stream=slot.stream)
        o = _Out(rgba, ns, graph, self.out_bytes(n_cams, W, H))
        with self.lock:
            slot.rings.setdefault(key, []).append(o)
            slot.rings.move_to_end(key)
        return o

    def _acquire_out(self, slot, key, n_cams, W, H):
        """A free ring buffer of the slot's bucket for key: an existing one,
        else a new one if the budget allows after evicting free buffers of
        idle buckets least-recently-used.  None if nothing can be freed."""
        with self.lock:
            for o in slot.rings.get(key, ()):
                if o.holders == 0:
                    o.last_use = time.perf_counter()
                    slot.rings.move_to_end(key)
                    return o
        need = self.out_bytes(n_cams, W, H)
        with self.lock:
            while self._used_bytes() + need > self.budget:
                victims = [(o.last_use, s, k, o) for s in self.slots if s.busy is None or s is slot
                           for k, ring_k in s.rings.items() for o in ring_k if o.holders == 0]
                if not victims:
                    return None
                _, s, k, o = min(victims, key=lambda v: v[0])
                s.rings[k].remove(o)
                if not s.rings[k]:
                    del s.rings[k]
                # drop the last references, so the buffer's memory is free
                # before the new one is allocated
                del victims, o
        return self._new_out(slot, key, n_cams, W, H)

    def _release(self, r):
        with self.cv:
            o, r._out = r._out, None
            if o is not None:
                o.holders -= 1
                self.cv.notify()

    def _cancel(self, r):
        with self.cv:
            if r.done.is_set():
                return False
            r.cancelled = True
            if r in self.pending:
                self.pending.remove(r)
                self._finish_failed(r, ServeCancelled("cancelled while queued"))
            self.cv.notify()
            return True

    def _finish_failed(self, r, err):
        # lock held by the caller
        r.error = err
        r.t_done = time.perf_counter()
        r.done.set()
        self.done_list.append(r)

    def _launch(self, slot, reqs):
        torch = self.torch
        r0 = reqs[0]
        n = sum(len(r.cams) for r in reqs)
        key = (r0.scene, r0.W, r0.H, n, self.compute)
        o = self._acquire_out(slot, key, n, r0.W, r0.H)
        if o is None:
            return False
        blob = r0.cam_blob if len(reqs) == 1 else b"".join(r.cam_blob for r in reqs)
        # the slot is idle, so the pinned buffer's previous upload has completed
        ctypes.memmove(slot.cams_host_ptr, blob, len(blob))
        with torch.cuda.stream(slot.stream):        # graphs replay on the current stream
            if o.graph is not None:
                o.graph.replay()
            else:
                slot.cams[:len(blob)].copy_(slot.cams_host[:len(blob)], non_blocking=True)
                capi.vrn_render_device_cams(self.ctx, self.fids[r0.scene], slot.cams, n, r0.W, r0.H, o.rgba,
                                            o.ns, self.compute, workspace=slot.ws, stream=slot.stream)
        ev = slot.event
        ev.record(slot.stream)
        now = time.perf_counter()
        off = 0
        with self.lock:
            for r in reqs:
                r._out, r._off = o, off
                o.holders += 1
                off += len(r.cams)
                r.t_start = now
        slot.busy = reqs
        slot.event = ev
        return True

    def _poll(self):
        for s in self.slots:
            if s.busy is not None and s.event.query():
                now = time.perf_counter()
                with self.lock:
                    for r in s.busy:
                        r.t_done = now
                        if r.cancelled:
                            r.error = ServeCancelled("cancelled while running")
                        elif r.deadline is not None and now > r.deadline:
                            r.error = ServeTimeout("completed after its deadline")
                        if r.error is not None or not r.keep:
                            o, r._out = r._out, None
                            if o is not None:
                                o.holders -= 1
                        r.done.set()
                    self.done_list.extend(s.busy)
                s.busy = None

    def _expire(self):
        """Fail queued requests whose deadline has passed (never launched)."""
        now = time.perf_counter()
        with self.lock:
            if not any(r.deadline is not None and now > r.deadline for r in self.pending):
                return
            keep = collections.deque()
            for r in self.pending:
                if r.deadline is not None and now > r.deadline:
                    self._finish_failed(r, ServeTimeout("deadline passed while queued"))
                else:
                    keep.append(r)
            self.pending = keep

    def _take_batch(self):
        """Oldest pending request plus same-scene, same-size single-camera
        requests behind it (up to max_batch cameras)."""
        with self.lock:
            if not self.pending:
                return None
            head = self.pending.popleft()
            batch = [head]
            # merged cameras must fit the budget beside the fixed allocations
            fit = (self.budget - self.fixed_bytes) // max(1, self.out_bytes(1, head.W, head.H))
            limit = min(self.max_batch, max(1, int(fit)))
            if len(head.cams) == 1 and limit > 1:
                keep = collections.deque()
                while self.pending:
                    r = self.pending.popleft()
                    if (len(batch) < limit and len(r.cams) == 1 and r.scene == head.scene
                            and r.W == head.W and r.H == head.H):
                        batch.append(r)
                    else:
                        keep.append(r)
                self.pending = keep
            self._claimed += 1
            return batch

    def _requeue(self, batch):
        with self.lock:
            for r in reversed(batch):
                self.pending.appendleft(r)

    def _loop(self):
        while not self._stop.is_set():
            self._poll()
            self._expire()
            free = [s for s in self.slots if s.busy is None]
            launched = False
            if free:
                batch = self._take_batch()
                if batch is not None:
                    try:
                        if self._launch(free[0], batch):
                            launched = True
                        elif len(free) == len(self.slots):
                            # nothing in flight will free memory: shrink to the head request;
                            # if even that cannot be admitted, it waits for held results to
                            # be released, and fails only when none are held
                            head, rest = batch[0], batch[1:]
                            self._requeue(rest)
                            if self._launch(free[0], [head]):
                                launched = True
                            elif self.held_bytes() > 0:
                                self._requeue([head])
                            else:
                                with self.lock:
                                    self._finish_failed(head, ServeError("request does not fit the HBM budget"))
                        else:
                            self._requeue(batch)
                    finally:
                        # the batch is now on a slot (busy), back in `pending` or
                        # failed: a draining stop() may look again
                        with self.lock:
                            self._claimed -= 1
            if launched:
                continue
            if any(s.busy is not None for s in self.slots):
                time.sleep(0)             # renders in flight: poll their events again at once
            else:
                # idle, or waiting for a held result to be released: a submit,
                # release, cancel or stop wakes the loop
                with self.cv:
                    if not self._stop.is_set():
                        self.cv.wait(0.001)


def summarize(reqs, wall_s):
    ok = [r for r in reqs if r.error is None and r.latency is not None]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    rays = sum(len(r.cams) * r.W * r.H for r in ok)
    return {"requests": len(reqs), "failed": len(reqs) - len(ok), "rays_per_s": rays / wall_s,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}


def request_stream(n, rate_hz, seed=5004):
    """The serving mix of sizes and scenes as (arrival time, scene, cameras,
    W, H), with cameras drawn before any timing starts."""
    from . import synth
    out = []
    for q in synth.serving_requests(n, rate_hz, seed):
        cams, W, H = synth.request_cameras(q["scene"], q["kind"], q["pose_seed"])
        out.append((q["t"], q["scene"], cams, W, H))
    return out


def drive(server, stream, keep=False):
    """Submit a request stream in real time (each request at its arrival
    time) and wait for all of them; returns (requests, wall seconds)."""
    server.start()
    t0 = time.perf_counter()
    reqs = []
    for (t, scene, cams, W, H) in stream:
        while True:
            # sleep through most of the gap (leaving the interpreter to the
            # scheduler thread) and spin for the last fraction of a millisecond
            left = t - (time.perf_counter() - t0)
            if left <= 0:
                break
            time.sleep(left - 3e-4 if left > 6e-4 else 0)
        reqs.append(server.submit(scene, cams, W, H, t_arrival=t0 + t, keep=keep))
    server.stop(drain=True)
    wall = time.perf_counter() - t0
    return reqs, wall


def mix_shapes(max_batch):
    """Every bucket shape the serving mix can produce: single-camera requests
    merge up to max_batch cameras; stereo requests carry two."""
    return ([(256, 256, k) for k in range(1, max_batch + 1)] +
            [(1024, 1024, k) for k in range(1, max_batch + 1)] + [(2048, 2048, 2)])


def run_serving(fields, rates_hz, n_requests=300, budget_bytes=24 << 30, slots=4, burst=True, log=None):
    """The serving benchmark: at each fixed offered rate, the same Poisson
    arrival trace is served (a) by the FP16 server (slots, batching, graphs),
    (b) by the baseline -- FP32, one request at a time through a one-slot
    FIFO, no graphs, no batching -- and (c) by that FIFO with the FP16 path,
    which separates the kernel's share of the difference from the server's.
    A saturating burst gives each mode's capacity.  Returns a dict of
    summaries."""
    out = {"rates_req_per_s": list(rates_hz), "requests_per_run": n_requests}
    traces = {rate: request_stream(n_requests, rate, seed=6000 + int(rate)) for rate in rates_hz}
    warm = request_stream(12, 1e6, seed=5999)
    flood = request_stream(n_requests, 1e6, seed=5004)

    def run(name, srv):
        drive(srv, warm)
        if burst:
            if log:
                log(f"serve: {name}, saturating burst")
            reqs, wall = drive(srv, flood)
            out[f"{name}_burst"] = dict(summarize(reqs, wall), req_per_s=len(reqs) / wall)
        for rate, tr in traces.items():
            if log:
                log(f"serve: {name} at {rate:g} req/s")
            reqs, wall = drive(srv, tr)
            out[f"{name}_at_{rate:g}"] = dict(summarize(reqs, wall), rate_req_per_s=rate)
        srv.close()

    run("baseline_f32_fifo", Server(fields, budget_bytes, n_slots=1, compute="f32", use_graphs=False, max_batch=1))
    run("fifo_f16", Server(fields, budget_bytes, n_slots=1, compute="f16", use_graphs=False, max_batch=1))
    srv = Server(fields, budget_bytes, n_slots=slots, compute="f16", use_graphs=True)
    srv.warmup(mix_shapes(srv.max_batch))
    run("server_f16", srv)
    return out


def main():
    ap = argparse.ArgumentParser(description="serving benchmark: mixed resolutions and scenes")
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--budget-gb", type=float, default=24.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--rates", default="250,500,1000,1500", help="offered loads, requests per second")
    args = ap.parse_args()
    from . import synth
    out = run_serving(synth.fields_serving(), [float(x) for x in args.rates.split(",")], args.requests,
                      int(args.budget_gb * (1 << 30)), args.slots,
                      log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
