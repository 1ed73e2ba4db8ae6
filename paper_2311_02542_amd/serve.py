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
  an output buffer and a captured HIP graph of the render kernel
  (vrn_render_device_cams reads the cameras from the slot's device buffer,
  so a replay renders whatever cameras were copied in before it).  Buffers
  are admitted against the HBM budget and evicted least-recently-used.
* Latency is measured on the host clock from a request's arrival to the
  moment its completion event is observed.

Every render runs in the library's HIP kernels; this module only
schedules.
"""
from __future__ import annotations

import argparse
import collections
import json
import math
import sys
import threading
import time

import numpy as np

from . import capi

CAM_BYTES = 72  # sizeof(vrn_camera)


class ServeError(RuntimeError):
    pass


class Request:
    __slots__ = ("rid", "scene", "cams", "W", "H", "t_arrival", "t_start", "t_done", "result", "event",
                 "error", "done")

    def __init__(self, rid, scene, cams, W, H, t_arrival):
        self.rid, self.scene, self.cams, self.W, self.H = rid, scene, cams, W, H
        self.t_arrival = t_arrival
        self.t_start = self.t_done = None
        self.result = None
        self.event = None
        self.error = None
        self.done = threading.Event()

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival


class _Bucket:
    def __init__(self, key, rgba, ns, graph):
        self.key, self.rgba, self.ns, self.graph = key, rgba, ns, graph
        self.bytes = rgba.numel() * 4 + ns.numel() * 4
        self.last_use = time.perf_counter()


class _Slot:
    def __init__(self, torch, device, ws_bytes):
        self.stream = torch.cuda.Stream(device=device)
        self.ws = torch.zeros(ws_bytes, dtype=torch.uint8, device=device)
        self.cams = torch.zeros(capi.MAX_CAMS * CAM_BYTES, dtype=torch.uint8, device=device)
        self.cams_host = torch.zeros(capi.MAX_CAMS * CAM_BYTES, dtype=torch.uint8).pin_memory()
        self.buckets: "collections.OrderedDict[tuple, _Bucket]" = collections.OrderedDict()
        self.busy = None          # list of requests in flight
        self.event = None


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
        self.done_list = []
        self._rid = 0
        self._stop = threading.Event()
        self._thread = None
        torch.cuda.synchronize()

    # ---------------------------------------------------------------- API
    def submit(self, scene, cams, W, H, t_arrival=None) -> Request:
        if scene not in self.fids:
            raise ServeError(f"unknown scene {scene}")
        if capi.vrn_check_cameras(cams, W, H) != capi.VRN_OK:
            raise ServeError("invalid cameras: " + capi.load_library().vrn_last_error().decode())
        need = len(cams) * W * H * 20
        if self.fixed_bytes + need > self.budget:
            raise ServeError("request can never fit the HBM budget")
        with self.lock:
            self._rid += 1
            r = Request(self._rid, scene, cams, W, H, time.perf_counter() if t_arrival is None else t_arrival)
            self.pending.append(r)
        return r

    def warmup(self, shapes):
        """Allocate and capture, on every slot, the buckets of every scene for
        the given (W, H, n_cams) shapes, so that no capture (and its device
        synchronisation) happens while requests are being served.  Stops at
        the HBM budget."""
        for slot in self.slots:
            for scene in self.fids:
                for (W, H, n) in shapes:
                    key = (scene, W, H, n, self.compute)
                    if self._used_bytes() + n * W * H * 20 > self.budget:
                        return
                    self._admit_bucket(slot, key, n, W, H)
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
        if self._thread:
            self._thread.join()

    def close(self):
        self.stop(drain=False)
        self.torch.cuda.synchronize()
        for s in self.slots:
            s.buckets.clear()
        for fid in self.fids.values():
            capi.vrn_unload_field(self.ctx, fid)
        capi.vrn_destroy(self.ctx)

    # ------------------------------------------------------------ internals
    def _used_bytes(self):
        return self.fixed_bytes + sum(b.bytes for s in self.slots for b in s.buckets.values())

    def _admit_bucket(self, slot, key, n_cams, W, H):
        """Return the slot's bucket for key, allocating (and capturing) it if
        the budget allows after evicting least-recently-used idle buffers."""
        torch = self.torch
        if key in slot.buckets:
            b = slot.buckets.pop(key)
            slot.buckets[key] = b
            b.last_use = time.perf_counter()
            return b
        need = n_cams * H * W * 20
        while self._used_bytes() + need > self.budget:
            victims = [(b.last_use, s, k) for s in self.slots if s.busy is None or s is slot
                       for k, b in s.buckets.items()]
            if not victims:
                return None
            _, s, k = min(victims, key=lambda v: v[0])
            del s.buckets[k]
        rgba = torch.zeros((n_cams, H, W, 4), dtype=torch.float32, device=self.device)
        ns = torch.zeros((n_cams, H, W), dtype=torch.int32, device=self.device)
        graph = None
        scene = key[0]
        if self.use_graphs:
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=slot.stream, capture_error_mode="thread_local"):
                capi.vrn_render_device_cams(self.ctx, self.fids[scene], slot.cams, n_cams, W, H, rgba, ns,
                                            self.compute, workspace=slot.ws, stream=slot.stream)
        b = _Bucket(key, rgba, ns, graph)
        slot.buckets[key] = b
        return b

    def _launch(self, slot, reqs):
        torch = self.torch
        r0 = reqs[0]
        cams = [c for r in reqs for c in r.cams]
        n = len(cams)
        key = (r0.scene, r0.W, r0.H, n, self.compute)
        b = self._admit_bucket(slot, key, n, r0.W, r0.H)
        if b is None:
            return False
        blob = bytes(capi.make_cameras(cams, r0.H))
        slot.cams_host[:len(blob)].copy_(torch.frombuffer(bytearray(blob), dtype=torch.uint8))
        with torch.cuda.stream(slot.stream):
            slot.cams[:len(blob)].copy_(slot.cams_host[:len(blob)], non_blocking=True)
            if b.graph is not None:
                b.graph.replay()
            else:
                capi.vrn_render_device_cams(self.ctx, self.fids[r0.scene], slot.cams, n, r0.W, r0.H, b.rgba,
                                            b.ns, self.compute, workspace=slot.ws, stream=slot.stream)
            off = 0
            for r in reqs:
                k = len(r.cams)
                r.result = (b.rgba[off:off + k].clone(), b.ns[off:off + k].clone())
                off += k
            ev = torch.cuda.Event()
            ev.record(slot.stream)
        now = time.perf_counter()
        for r in reqs:
            r.t_start = now
        slot.busy = reqs
        slot.event = ev
        return True

    def _poll(self):
        for s in self.slots:
            if s.busy is not None and s.event.query():
                now = time.perf_counter()
                for r in s.busy:
                    r.t_done = now
                    r.done.set()
                with self.lock:
                    self.done_list.extend(s.busy)
                s.busy = None

    def _take_batch(self):
        """Oldest pending request plus same-scene, same-size single-camera
        requests behind it (up to max_batch cameras)."""
        with self.lock:
            if not self.pending:
                return None
            head = self.pending.popleft()
            batch = [head]
            # merged cameras must fit the budget beside the fixed allocations
            fit = (self.budget - self.fixed_bytes) // max(1, head.W * head.H * 20)
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
            free = [s for s in self.slots if s.busy is None]
            launched = False
            if free:
                batch = self._take_batch()
                if batch is not None:
                    try:
                        if self._launch(free[0], batch):
                            launched = True
                        elif len(free) == len(self.slots):
                            # nothing in flight will free memory: shrink to the head
                            # request, and fail it if even that cannot be admitted
                            head, rest = batch[0], batch[1:]
                            self._requeue(rest)
                            if not self._launch(free[0], [head]):
                                head.error = ServeError("request does not fit the HBM budget")
                                head.done.set()
                                with self.lock:
                                    self.done_list.append(head)
                            else:
                                launched = True
                        else:
                            self._requeue(batch)
                    finally:
                        # the batch is now on a slot (busy), back in `pending` or
                        # failed: a draining stop() may look again
                        with self.lock:
                            self._claimed -= 1
            if not launched:
                time.sleep(0.00005)

    def run_serial(self, reqs_spec):
        """Baseline: one request at a time, no overlap, no graphs."""
        torch = self.torch
        lat = []
        slot = self.slots[0]
        for (scene, cams, W, H) in reqs_spec:
            t0 = time.perf_counter()
            rgba = torch.empty((len(cams), H, W, 4), dtype=torch.float32, device=self.device)
            capi.vrn_render(self.ctx, self.fids[scene], cams, W, H, rgba, None, self.compute,
                            workspace=slot.ws, stream=slot.stream)
            slot.stream.synchronize()
            lat.append(time.perf_counter() - t0)
        return lat


def summarize(reqs, wall_s):
    lat = np.array([r.latency for r in reqs if r.latency is not None])
    rays = sum(len(r.cams) * r.W * r.H for r in reqs)
    return {"requests": len(reqs), "rays_per_s": rays / wall_s, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3)}


def drive(server, n, rate_hz, seed=5004):
    """Submit a Poisson request stream (the serving mix of sizes and scenes) in real time and wait."""
    from . import synth
    spec = synth.serving_requests(n, rate_hz, seed)
    server.start()
    t0 = time.perf_counter()
    reqs = []
    for q in spec:
        while time.perf_counter() - t0 < q["t"]:
            time.sleep(0.00005)
        cams, W, H = synth.request_cameras(q["scene"], q["kind"], q["pose_seed"])
        reqs.append(server.submit(q["scene"], cams, W, H))
    server.stop(drain=True)
    wall = time.perf_counter() - t0
    return reqs, wall


def main():
    ap = argparse.ArgumentParser(description="serving benchmark: mixed resolutions and scenes")
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--budget-gb", type=float, default=8.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--loads", default="0.25,0.5,0.75,0.9")
    args = ap.parse_args()
    import torch
    from . import synth
    fields = synth.fields_serving()
    budget = int(args.budget_gb * (1 << 30))
    # serial FP32 baseline: one request at a time, no overlap, no graphs
    base = Server(fields, budget, n_slots=1, compute="f32", use_graphs=False)
    spec = synth.serving_requests(args.requests, 1.0)
    work = []
    for q in spec:
        cams, W, H = synth.request_cameras(q["scene"], q["kind"], q["pose_seed"])
        work.append((q["scene"], cams, W, H))
    print("serve: serial f32 baseline", file=sys.stderr, flush=True)
    base.run_serial(work[:10])
    t0 = time.perf_counter()
    lat = np.array(base.run_serial(work))
    wall = time.perf_counter() - t0
    rays = sum(len(w[1]) * w[2] * w[3] for w in work)
    capacity = len(work) / wall
    out = {"baseline_serial_f32": {"rays_per_s": rays / wall, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                                   "p99_ms": float(np.percentile(lat, 99) * 1e3), "req_per_s": capacity}}
    base.close()
    srv = Server(fields, budget, n_slots=args.slots, compute="f16", use_graphs=True)
    # graphs for every bucket the mix can produce (single-camera requests
    # merge up to max_batch cameras; stereo requests carry two)
    srv.warmup([(256, 256, k) for k in range(1, srv.max_batch + 1)] +
               [(1024, 1024, k) for k in range(1, srv.max_batch + 1)] + [(2048, 2048, 2)])
    # capacity of the serving path: a saturating burst
    print("serve: saturating burst", file=sys.stderr, flush=True)
    reqs, wall = drive(srv, args.requests, 1e6)
    cap = len(reqs) / wall
    out["burst"] = summarize(reqs, wall)
    out["burst"]["req_per_s"] = cap
    for load in [float(x) for x in args.loads.split(",")]:
        print(f"serve: load {load}", file=sys.stderr, flush=True)
        reqs, wall = drive(srv, args.requests, load * cap, seed=6000 + int(load * 100))
        out[f"load_{load:g}"] = summarize(reqs, wall)
        out[f"load_{load:g}"]["rate_hz"] = load * cap
    srv.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
