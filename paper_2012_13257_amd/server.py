"""Python binding of the serving loop (interp_server_* in libgmminterp.so).

    srv = Server(budget_bytes=8 << 30, max_slots=128)
    t = srv.submit(pos, sigma, values, H, W)            # forward only
    t = srv.submit(pos, sigma, values, H, W, grad_out=G) # forward + backward
    ...
    res = srv.result(t)   # None while queued/running; dict when done
    pr = srv.prepare(pos, sigma, values, H, W)          # described ahead ...
    t = srv.submit_prepared(pr)                          # ... submitted when it arrives
    ts = srv.submit_many([srv.prepare(pos, sigma, values, H, W), ...])  # one call, many requests

Every request is one image (B = 1) with C <= 4 channels.  When torch's
current stream still has work queued, submit records an event on it after
the request's outputs are allocated, and the batch that runs the request
waits for it on the device, so inputs produced by earlier work on that
stream (and output memory the caching allocator hands back) are safe to use
without a host synchronisation; an idle stream needs no event.  The binding
keeps every tensor of a request, and the event, alive until its result has
been collected.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional

import torch

from . import _lib
from .interp import problem


class Server:
    def __init__(self, budget_bytes: int, max_slots: int = 128, max_queue: int = 1 << 20,
                 device: Optional[int] = None):
        L = _lib.lib()
        dev = torch.cuda.current_device() if device is None else int(device)
        cfg = _lib.ServerConfig(dev, int(max_slots), int(max_queue), 0, int(budget_bytes))
        h = ctypes.c_void_p()
        _lib.check("interp_server_create", L.interp_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._device = torch.device("cuda", dev)
        self._live: Dict[int, dict] = {}
        # Events that order each request after the caller's stream, created
        # here and reused: creating a HIP event per request occasionally
        # stalls for milliseconds (the runtime allocates events in batches).
        self._events = [self._new_event() for _ in range(256)]

    def _new_event(self) -> torch.cuda.Event:
        e = torch.cuda.Event()
        e.record(torch.cuda.current_stream(self._device))  # creates the HIP event now
        return e

    def prepare(self, pos, sigma, values, H: int, W: int, radius: float = 3.0, tile: int = 8,
                grad_out: Optional[torch.Tensor] = None, grads=("pos", "sigma", "values"),
                out: Optional[torch.Tensor] = None,
                grad_buffers: Optional[dict] = None) -> "Prepared":
        """A request described for submission (submit_many), its result tensors
        allocated.  out / grad_buffers ({"pos": t, "sigma": t, "values": t}) may
        supply preallocated result tensors."""
        prob = problem(pos, sigma, values, H, W, radius, tile)
        if out is None:
            out = torch.empty((1, prob.C, prob.H, prob.W), dtype=torch.float32, device=self._device)
        elif tuple(out.shape) != (1, prob.C, prob.H, prob.W) or not out.is_contiguous():
            raise ValueError("out must be a contiguous [1, C, H, W] tensor")
        gb = grad_buffers or {}
        keep = {"pos": pos, "sigma": sigma, "values": values, "out": out}
        req = _lib.Request()
        req.prob = prob
        req.pos, req.sigma, req.values, req.out = (pos.data_ptr(), sigma.data_ptr(),
                                                   values.data_ptr(), out.data_ptr())
        if grad_out is not None:
            if tuple(grad_out.shape) != (1, prob.C, prob.H, prob.W) or not grad_out.is_contiguous():
                raise ValueError("grad_out must be a contiguous [1, C, H, W] tensor")
            keep["grad_out"] = grad_out
            req.grad_out = grad_out.data_ptr()
            if "pos" in grads:
                keep["grad_pos"] = gb["pos"] if "pos" in gb else torch.empty_like(pos)
                req.grad_pos = keep["grad_pos"].data_ptr()
            if "sigma" in grads:
                keep["grad_sigma"] = gb["sigma"] if "sigma" in gb else torch.empty_like(sigma)
                req.grad_sigma = keep["grad_sigma"].data_ptr()
            if "values" in grads:
                keep["grad_values"] = gb["values"] if "values" in gb else torch.empty_like(values)
                req.grad_values = keep["grad_values"].data_ptr()
        return Prepared(req, keep)

    def _ready_event(self, after_stream: bool):
        """An event recorded on torch's current stream when it still has work
        queued, else None.  (An event recorded on an idle stream would be one
        more marker on a hardware queue that the runtime may share with a
        server stream, which would then order the request behind another
        batch.)"""
        stream = torch.cuda.current_stream(self._device)
        if not after_stream or stream.query():
            return None
        ready = self._events.pop() if self._events else self._new_event()
        ready.record(stream)
        return ready

    def submit(self, pos, sigma, values, H: int, W: int, radius: float = 3.0, tile: int = 8,
               grad_out: Optional[torch.Tensor] = None, grads=("pos", "sigma", "values"),
               out: Optional[torch.Tensor] = None, grad_buffers: Optional[dict] = None,
               after_stream: bool = True) -> int:
        """Queues one request (arguments as for prepare).  after_stream: order
        the request after the work queued so far on torch's current stream
        (False: the caller guarantees its inputs and buffers are ready)."""
        pr = self.prepare(pos, sigma, values, H, W, radius, tile, grad_out, grads, out, grad_buffers)
        return self.submit_prepared(pr, after_stream)

    def submit_prepared(self, pr: "Prepared", after_stream: bool = True) -> int:
        """Queues one request prepare() described (a client can describe its
        requests ahead and pay only this call when they arrive); as submit."""
        ready = self._ready_event(after_stream)
        pr.req.ready = ready.cuda_event if ready is not None else None
        ticket = ctypes.c_uint64()
        _lib.check("interp_submit", _lib.lib().interp_submit(self._h, ctypes.byref(pr.req),
                                                             ctypes.byref(ticket)))
        keep = pr.keep
        if ready is not None:
            keep = dict(keep, ready=ready)
        self._live[ticket.value] = keep
        return ticket.value

    def submit_many(self, prepared, after_stream: bool = True) -> List[int]:
        """Queues prepared requests (a list of prepare()'s results, or a Batch
        of them) in one call and returns their tickets in order.  One event on
        torch's current stream orders them all (see submit).  If the server
        cannot queue them all, the InterpError raised carries the tickets of
        those it queued (attribute tickets); the others were not queued."""
        batch = prepared if isinstance(prepared, Batch) else Batch(prepared)
        n = len(batch.items)
        ready = self._ready_event(after_stream)
        if ready is not None or batch.has_ready:
            # (a batch submitted again must not keep an earlier call's event)
            ev = ready.cuda_event if ready is not None else None
            for i in range(n):
                batch.array[i].ready = ev
            batch.has_ready = ready is not None
        tickets = (ctypes.c_uint64 * max(n, 1))()
        queued = ctypes.c_int32()
        rc = _lib.lib().interp_submit_many(self._h, batch.array, n, tickets, ctypes.byref(queued))
        out = []
        for i in range(queued.value):
            keep = dict(batch.items[i].keep)
            if ready is not None:
                keep["ready_shared"] = ready  # kept alive, not returned to the pool
            self._live[tickets[i]] = keep
            out.append(tickets[i])
        if rc != _lib.INTERP_OK:
            err = _lib.InterpError("interp_submit_many", rc, _lib.last_error())
            err.tickets = out
            raise err
        return out

    def poll(self, ticket: int) -> _lib.Status:
        st = _lib.Status()
        _lib.check("interp_poll", _lib.lib().interp_poll(self._h, ticket, ctypes.byref(st)))
        return st

    def result(self, ticket: int):
        """None while the request is queued or running; otherwise a dict with the
        status fields and the output tensors (out, grad_*) of the request."""
        st = self.poll(ticket)
        if st.state in (_lib.QUEUED, _lib.RUNNING):
            return None
        keep = self._live.pop(ticket)
        if "ready" in keep:
            self._events.append(keep["ready"])  # the server no longer waits on it
        res = {k: v for k, v in keep.items() if k == "out" or k.startswith("grad_")}
        res.pop("grad_out", None)
        res.update(state=st.state, err=st.err, t_submit_ns=st.t_submit_ns,
                   t_admit_ns=st.t_admit_ns, t_done_ns=st.t_done_ns)
        return res

    def drain(self, timeout_ms: int = -1) -> bool:
        rc = _lib.lib().interp_server_drain(self._h, int(timeout_ms))
        if rc == _lib.INTERP_EAGAIN:
            return False
        _lib.check("interp_server_drain", rc)
        return True

    def close(self) -> None:
        if self._h:
            _lib.check("interp_server_destroy", _lib.lib().interp_server_destroy(self._h))
            self._h = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Prepared:
    """One request described for the C ABI (interp_request) and the tensors it
    uses, which must stay alive until its result is collected."""
    __slots__ = ("req", "keep")

    def __init__(self, req, keep: dict):
        self.req = req
        self.keep = keep


class Batch:
    """Prepared requests laid out as the array interp_submit_many reads;
    building it once ahead keeps the copy out of the submitting call."""

    def __init__(self, prepared):
        self.items = list(prepared)
        self.array = (_lib.Request * max(len(self.items), 1))(*[p.req for p in self.items])
        self.has_ready = any(p.req.ready for p in self.items)
