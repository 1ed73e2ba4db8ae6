"""Serving over the C ABI's serving engine (vrn_server_*): continuous
batching of render requests of mixed resolutions and scenes, resident
fields, admission against an HBM budget and one captured HIP graph per ring
buffer, with p50/p99 latency beside throughput.

The scheduler is native (csrc/server.cpp): one thread per engine polls
completion events, launches the oldest pending request -- merged with the
single-camera requests of the same scene and size behind it -- on a free
slot (a HIP stream with its own workspace), and hands out results that stay
in device memory until released.  This module marshals: it loads the
fields, gives the engine a device arena (a torch tensor) sized to what the
budget leaves after the fields and slot workspaces, submits requests and
turns finished ones into torch views of the arena.

* ``Request.result`` is (rgba [n_cams, H, W, 4], nsamples [n_cams, H, W]),
  views of the request's ring buffer in the arena, valid until
  ``Request.release()``.
* ``keep=False`` (latency-only clients) returns the buffer to its ring at
  completion; the request still reports its latency.
* ``timeout_s`` bounds arrival -> completion; ``Request.cancel()`` removes a
  queued request or discards a running one's result.
* Latency runs from the arrival time (the engine's monotonic clock,
  ``capi.vrn_server_clock``) to the moment the engine observed the
  completion event.

Every render runs in the library's HIP kernels; there is no Python
scheduling loop and no CPU fallback.
"""
from __future__ import annotations

import argparse
import atexit
import json
import sys
import time
import weakref

import numpy as np

from . import capi

CAM_BYTES = 72  # sizeof(vrn_camera)


class ServeError(RuntimeError):
    pass


class ServeTimeout(ServeError):
    pass


class ServeCancelled(ServeError):
    pass


_FAILURES = {capi.VRN_ERR_TIMEOUT: (ServeTimeout, "passed its deadline"),
             capi.VRN_ERR_CANCELLED: (ServeCancelled, "cancelled"),
             capi.VRN_ERR_BUDGET: (ServeError, "does not fit the HBM budget"),
             capi.VRN_ERR_NOT_FOUND: (ServeError, "its field was unloaded"),
             capi.VRN_ERR_DEVICE: (ServeError, "HIP error in serving")}


class _Done:
    """threading.Event-like view of a request's completion."""
    __slots__ = ("_r",)

    def __init__(self, r):
        self._r = r

    def is_set(self) -> bool:
        return self._r._fetch(0.0)

    def wait(self, timeout=None) -> bool:
        return self._r._fetch(1e6 if timeout is None else float(timeout))


class Request:
    __slots__ = ("rid", "scene", "cams", "W", "H", "keep", "done", "_server", "_status", "_t", "_ptrs",
                 "_views", "_released")

    def __init__(self, server, rid, scene, cams, W, H, keep):
        self._server = server
        self.rid, self.scene, self.cams, self.W, self.H, self.keep = rid, scene, cams, W, H, keep
        self.done = _Done(self)
        self._status = None            # vrn_status once finished
        self._t = None                 # (t_arrival, t_launch, t_done) once finished
        self._ptrs = None              # (d_rgba, d_nsamples) while held
        self._views = None
        self._released = False

    def _fetch(self, wait_s) -> bool:
        if self._status is not None:
            return True
        if self._released:
            return False
        fin, out = capi.vrn_server_wait(self._server.sv, self.rid, wait_s)
        if fin:
            self._t = (out.t_arrival, out.t_launch, out.t_done)
            self._ptrs = (out.d_rgba, out.d_nsamples) if out.d_rgba else None
            self._status = int(out.status)
        return fin

    @property
    def error(self):
        """None on success (or while running); else a ServeError."""
        if not self._fetch(0.0) or self._status == capi.VRN_OK:
            return None
        cls, what = _FAILURES.get(self._status, (ServeError, f"status {self._status}"))
        return cls(f"request {self.rid}: {what}")

    @property
    def t_arrival(self):
        return self._t[0] if self._fetch(0.0) else None

    @property
    def t_start(self):
        """Launch time on the engine's clock; None if never launched."""
        return self._t[1] if self._fetch(0.0) and self._t[1] > 0 else None

    @property
    def t_done(self):
        return self._t[2] if self._fetch(0.0) else None

    @property
    def latency(self):
        return self._t[2] - self._t[0] if self._fetch(0.0) else None

    @property
    def result(self):
        """(rgba [n_cams, H, W, 4] float32, nsamples [n_cams, H, W] int32):
        views of the request's ring buffer, valid until release(); None if
        it has not finished, failed, or was released or not kept."""
        if self._released or not self._fetch(0.0) or self._status != capi.VRN_OK or self._ptrs is None:
            return None
        if self._views is None:
            torch = self._server.torch
            arena, base = self._server.arena, self._server.arena_ptr
            n, px = len(self.cams), self.H * self.W
            a, b = self._ptrs[0] - base, self._ptrs[1] - base
            rgba = arena[a:a + n * px * 16].view(torch.float32).view(n, self.H, self.W, 4)
            ns = arena[b:b + n * px * 4].view(torch.int32).view(n, self.H, self.W)
            self._views = (rgba, ns)
        return self._views

    def release(self):
        """Forget the request and return its output buffer to its ring (the
        latency stays readable).  The request must have finished."""
        if self._released:
            return
        if not self._fetch(0.0):
            raise ServeError(f"request {self.rid} has not finished (cancel it first)")
        capi.vrn_server_release(self._server.sv, self.rid)
        self._released = True
        self._ptrs = self._views = None

    def cancel(self) -> bool:
        """Cancel: a queued request is never launched; a running one has its
        result discarded when it completes.  False once finished."""
        if self._released or self._status is not None:
            return False
        return capi.vrn_server_cancel(self._server.sv, self.rid)


# Engines still open at interpreter exit are destroyed while the HIP runtime
# is intact (their scheduler threads make HIP calls until stopped).
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_servers():
    for srv in list(_LIVE):
        try:
            srv.close()
        except Exception:
            pass


class Server:
    """Resident fields on one context plus a native serving engine.  The HBM
    budget covers the fields, the slot workspaces and the engine's arena, in
    which every output buffer -- held by a client or free -- lives."""

    def __init__(self, fields: dict, hbm_budget_bytes: int, n_slots: int = 4, compute: str = "f16",
                 use_graphs: bool = True, max_batch: int = 4, device: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.compute = compute
        self.use_graphs = use_graphs
        self.max_batch = max_batch
        self.n_slots = n_slots
        self.budget = int(hbm_budget_bytes)
        self.ctx = capi.vrn_create(device, self.budget)
        self.sv = None
        self.fids = {}
        self._out_bytes = {}
        self.field_bytes = 0
        for name, f in fields.items():
            fid = capi.vrn_load_field(self.ctx, f)       # VRN_ERR_BUDGET if fields alone exceed it
            self.fids[name] = fid
            self.field_bytes += capi.vrn_field_bytes(self.ctx, fid)
        ws_bytes = capi.vrn_workspace_bytes(self.ctx)
        self.fixed_bytes = self.field_bytes + n_slots * (ws_bytes + capi.MAX_CAMS * CAM_BYTES)
        arena_bytes = (self.budget - self.fixed_bytes) // 256 * 256
        if arena_bytes < 256:
            self._free_ctx()
            raise ServeError("resident fields and slot workspaces exceed the HBM budget")
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=self.device)
        self.arena_ptr = self.arena.data_ptr()
        try:
            self.sv = capi.vrn_server_create(self.ctx, arena_bytes, self.arena, n_slots, max_batch, use_graphs,
                                             compute)
        except capi.VrnError:
            self._free_ctx()
            raise
        _LIVE.add(self)

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

    def submit(self, scene, cams, W, H, t_arrival=None, timeout_s=None, keep=True, cam_array=None) -> Request:
        """Queue a render request.  t_arrival is on capi.vrn_server_clock()
        (default: now); cam_array: the cameras already marshalled by
        capi.make_cameras."""
        if scene not in self.fids:
            raise ServeError(f"unknown scene {scene}")
        if len(cams) > capi.MAX_CAMS:
            raise ServeError("too many cameras in one request")
        try:
            rid = capi.vrn_server_submit(self.sv, self.fids[scene], cams, W, H,
                                         t_arrival=0.0 if t_arrival is None else t_arrival,
                                         timeout_s=0.0 if timeout_s is None else timeout_s,
                                         flags=0 if keep else capi.VRN_SERVE_RELEASE_ON_DONE, cam_array=cam_array)
        except capi.VrnError as e:
            raise ServeError(str(e)) from e
        return Request(self, rid, scene, cams, W, H, keep)

    def warmup(self, shapes):
        """Allocate and capture, on every slot, one ring buffer per bucket of
        every scene for the given (W, H, n_cams) shapes, so that no capture
        happens while requests are being served.  Stops at the budget."""
        for scene, fid in self.fids.items():
            for (W, H, n) in shapes:
                try:
                    capi.vrn_server_prepare(self.sv, fid, n, W, H)
                except capi.VrnError as e:
                    if e.status == capi.VRN_ERR_BUDGET:
                        return
                    raise

    def start(self):
        capi.vrn_server_hold(self.sv, False)

    def stop(self, drain=True, max_wait_s=120.0):
        if drain:
            capi.vrn_server_drain(self.sv, max_wait_s)
        capi.vrn_server_hold(self.sv, True)

    def stats(self) -> dict:
        return capi.vrn_server_stats(self.sv)

    def held_bytes(self):
        """Device bytes of ring buffers held by requests: in flight, or
        finished and not yet released."""
        return self.stats()["held_bytes"]

    def _used_bytes(self):
        return self.fixed_bytes + self.stats()["used_bytes"]

    def _free_ctx(self):
        for fid in self.fids.values():
            capi.vrn_unload_field(self.ctx, fid)
        self.fids = {}
        capi.vrn_destroy(self.ctx)
        self.ctx = None

    def close(self):
        if self.sv is not None:
            capi.vrn_server_destroy(self.sv)   # waits for renders in flight
            self.sv = None
        if self.ctx is not None:
            self._free_ctx()
        self.arena = None
        _LIVE.discard(self)


def summarize(reqs, wall_s):
    """Throughput and latency percentiles of finished requests; wait_p50_ms
    is the median time from arrival to launch (queueing plus the host's
    share of a request)."""
    ok = [r for r in reqs if r.error is None and r.latency is not None]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    wait = np.array([r.t_start - r.t_arrival for r in ok]) if ok else np.zeros(1)
    rays = sum(len(r.cams) * r.W * r.H for r in ok)
    by_size = {}
    for key in sorted({(len(r.cams), r.W, r.H) for r in ok}):
        lk = np.array([r.latency for r in ok if (len(r.cams), r.W, r.H) == key])
        by_size[f"{key[0]}x{key[1]}x{key[2]}"] = {"requests": int(lk.size),
                                                 "p50_ms": float(np.percentile(lk, 50) * 1e3),
                                                 "p99_ms": float(np.percentile(lk, 99) * 1e3)}
    return {"requests": len(reqs), "failed": len(reqs) - len(ok), "rays_per_s": rays / wall_s,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "wait_p50_ms": float(np.percentile(wait, 50) * 1e3),
            "by_size": by_size}


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
    time, which is also its latency origin) and wait for all of them;
    returns (requests, wall seconds).  Requests not kept are released once
    their outcome has been read."""
    clock = capi.vrn_server_clock
    arrays = [capi.make_cameras(cams, H) for (_, _, cams, _, H) in stream]
    server.start()
    t0 = clock()
    reqs = []
    for (t, scene, cams, W, H), arr in zip(stream, arrays):
        while True:
            # sleep through most of the gap and spin for the last fraction of
            # a millisecond
            left = t - (clock() - t0)
            if left <= 0:
                break
            time.sleep(left - 3e-4 if left > 6e-4 else 0)
        reqs.append(server.submit(scene, cams, W, H, t_arrival=t0 + t, keep=keep, cam_array=arr))
    server.stop(drain=True)
    wall = clock() - t0
    for r in reqs:
        r.done.is_set()
        if not keep:
            r.release()
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
