"""GPU serving loop: every request's result equals the single-call result on
the same inputs (bitwise) whether it runs alone or inside a mix of requests
of other sizes and channel counts; results also match the oracle; budget and
argument errors are reported."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2012_13257_amd import synth
from gpu_helpers import check_grad, check_out_only, say

pytestmark = pytest.mark.gpu


def _requests(n, seed, sides=(16, 37, 64, 100, 128, 256)):
    trace = synth.config4_trace(n, None, seed=seed, sides=sides)
    out = []
    for r in trace:
        wl = r.workload()
        out.append((r, wl))
    return out


def _dev(wl):
    import torch
    return (torch.from_numpy(wl.pos).cuda(), torch.from_numpy(wl.sigma).cuda(),
            torch.from_numpy(wl.values).cuda(), torch.from_numpy(wl.grad_out()).cuda())


def _single(pos, sig, val, G, wl, bwd):
    from paper_2012_13257_amd import interp
    out, saved, _ = interp.forward(pos, sig, val, wl.H, wl.W, wl.radius)
    res = {"out": out}
    if bwd:
        gp, gs, gv = interp.backward(pos, sig, val, out, saved, G)
        res.update(grad_pos=gp, grad_sigma=gs, grad_values=gv)
    return res


def test_server_results_equal_single_call_alone_and_in_mix():
    import torch
    from paper_2012_13257_amd.server import Server
    reqs = _requests(48, 4321)
    dev = [_dev(wl) for _, wl in reqs]
    torch.cuda.synchronize()
    ref = [_single(p, s, v, G, wl, r.backward) for (r, wl), (p, s, v, G) in zip(reqs, dev)]
    torch.cuda.synchronize()
    with Server(budget_bytes=2 << 30, max_slots=16) as srv:
        # alone: one request at a time
        say("server alone")
        for k in (0, 5, 11):
            (r, wl), (p, s, v, G) = reqs[k], dev[k]
            t = srv.submit(p, s, v, wl.H, wl.W, wl.radius, grad_out=G if r.backward else None)
            assert srv.drain(60000)
            res = srv.result(t)
            assert res["state"] == 2, res
            for key, val in ref[k].items():
                assert torch.equal(res[key], val), (k, key)
        # in the mix: all at once (slots < requests, so admission interleaves)
        say("server mix")
        tickets = []
        for (r, wl), (p, s, v, G) in zip(reqs, dev):
            tickets.append(srv.submit(p, s, v, wl.H, wl.W, wl.radius,
                                      grad_out=G if r.backward else None))
        assert srv.drain(120000)
        nb = 0
        for k, t in enumerate(tickets):
            res = srv.result(t)
            assert res is not None and res["state"] == 2, (k, res)
            assert res["t_submit_ns"] <= res["t_admit_ns"] <= res["t_done_ns"]
            for key, val in ref[k].items():
                assert torch.equal(res[key], val), (k, key)
            nb += reqs[k][0].backward
        assert nb > 0


def test_server_submit_many_equals_single_call_and_checks_every_request():
    """interp_submit_many: one call queues a mix of requests in order; each
    result equals the single-call path bitwise.  A batch with one invalid
    request queues nothing; a batch that overflows the queue queues a
    prefix, whose results are still right."""
    import torch
    from paper_2012_13257_amd import _lib
    from paper_2012_13257_amd.server import Batch, Server
    reqs = _requests(40, 8765)
    dev = [_dev(wl) for _, wl in reqs]
    torch.cuda.synchronize()
    ref = [_single(p, s, v, G, wl, r.backward) for (r, wl), (p, s, v, G) in zip(reqs, dev)]
    torch.cuda.synchronize()
    with Server(budget_bytes=2 << 30, max_slots=16) as srv:
        say("server submit_many")
        prep = [srv.prepare(p, s, v, wl.H, wl.W, wl.radius, grad_out=G if r.backward else None)
                for (r, wl), (p, s, v, G) in zip(reqs, dev)]
        tickets = srv.submit_many(Batch(prep))
        assert len(tickets) == len(reqs) and tickets == sorted(tickets)
        assert srv.drain(120000)
        for k, t in enumerate(tickets):
            res = srv.result(t)
            assert res is not None and res["state"] == 2, (k, res)
            for key, val in ref[k].items():
                assert torch.equal(res[key], val), (k, key)
        # a prepared request submitted again on its own gives the same bits
        for k in (0, 7):
            t = srv.submit_prepared(prep[k])
            assert srv.drain(60000)
            res = srv.result(t)
            assert res["state"] == 2
            for key, val in ref[k].items():
                assert torch.equal(res[key], val), (k, key)
        # one invalid request (five channels) in the middle: nothing is queued
        p5 = torch.rand((1, 10, 2), device="cuda") * 16
        v5 = torch.rand((1, 10, 5), device="cuda")
        s5 = torch.full((1,), 1.0, device="cuda")
        bad = srv.prepare(p5, s5, v5, 16, 16)
        (r0, wl0), (p0, s0, v0, _) = reqs[0], dev[0]
        good = srv.prepare(p0, s0, v0, wl0.H, wl0.W, wl0.radius)
        with pytest.raises(_lib.InterpError) as ei:
            srv.submit_many([good, bad, good])
        assert ei.value.code == _lib.INTERP_EINVAL and ei.value.tickets == []
        assert "request 1" in str(ei.value)
    # a queue of three: the first three of five are queued and run
    with Server(budget_bytes=2 << 30, max_slots=2, max_queue=3) as srv:
        say("server submit_many, queue limit")
        prep = [srv.prepare(p, s, v, wl.H, wl.W, wl.radius) for (r, wl), (p, s, v, G) in
                zip(reqs[:5], dev[:5])]
        with pytest.raises(_lib.InterpError) as ei:
            srv.submit_many(prep)
        assert ei.value.code == _lib.INTERP_EAGAIN and len(ei.value.tickets) == 3
        assert srv.drain(60000)
        for k, t in enumerate(ei.value.tickets):
            res = srv.result(t)
            assert res["state"] == 2
            assert torch.equal(res["out"], ref[k]["out"]), k


def test_server_matches_oracle_on_small_requests():
    """Forward of every request and, for the requests that ask for it, every
    gradient, against the oracle (the server exports no Z: empty pixels are
    checked through the output, which must be exactly 0 there)."""
    from paper_2012_13257_amd.server import Server
    reqs = _requests(8, 99, sides=(24, 40))
    reqs[0][0].backward = reqs[3][0].backward = True
    reqs[1][0].backward = False
    with Server(budget_bytes=256 << 20, max_slots=8) as srv:
        dev = [_dev(wl) for _, wl in reqs]
        say("server vs oracle")
        ts = [srv.submit(p, s, v, wl.H, wl.W, wl.radius, grad_out=G if r.backward else None)
              for (r, wl), (p, s, v, G) in zip(reqs, dev)]
        assert srv.drain(60000)
        nb = 0
        for (r, wl), t in zip(reqs, ts):
            res = srv.result(t)
            assert res["state"] == 2, res
            if r.backward:
                G = wl.grad_out()
                ref = oracle.backward(wl.pos, wl.sigma, wl.values, G, wl.H, wl.W, wl.radius,
                                      workers=oracle.default_workers())
                fwd = ref["fwd"]
                check_grad(res["grad_pos"].cpu().numpy(), ref["grad_pos"], ref["scale_pos"],
                           f"server request {r.index} pos")
                check_grad(res["grad_values"].cpu().numpy(), ref["grad_values"],
                           ref["scale_values"], f"server request {r.index} values")
                check_grad(res["grad_sigma"].cpu().numpy(), ref["grad_sigma"], ref["scale_sigma"],
                           f"server request {r.index} sigma")
                nb += 1
            else:
                fwd = oracle.forward(wl.pos, wl.sigma, wl.values, wl.H, wl.W, wl.radius)
            og = res["out"].cpu().numpy().transpose(0, 2, 3, 1).reshape(-1, wl.C)
            r_ = {"out": fwd["out"].transpose(0, 2, 3, 1).reshape(-1, wl.C), "Z": fwd["Z"].ravel(),
                  "S": fwd["S"].transpose(0, 2, 3, 1).reshape(-1, wl.C)}
            check_out_only(og, r_, f"server request {r.index}")
        assert nb >= 2


def test_server_waits_for_the_callers_stream():
    """Inputs written by a kernel still running on torch's stream at submit
    time: the server's batch waits for the event submit records, so the
    result equals the single-call one on the final inputs."""
    import torch
    from paper_2012_13257_amd.server import Server
    (r, wl), = _requests(1, 123, sides=(128,))
    p, s, v, _ = _dev(wl)
    torch.cuda.synchronize()
    ref = _single(p, s, v, None, wl, False)
    torch.cuda.synchronize()
    with Server(budget_bytes=256 << 20, max_slots=4) as srv:
        say("server ordered after the caller's stream")
        v2 = torch.zeros_like(v)
        # a long chain of work on the current stream ends by writing the values
        junk = torch.randn(4096, 4096, device="cuda")
        for _ in range(8):
            junk = junk @ junk
            junk = junk / junk.norm()
        v2.copy_(v + 0.0 * junk[0, 0])
        t = srv.submit(p, s, v2, wl.H, wl.W, wl.radius)
        assert srv.drain(60000)
        res = srv.result(t)
        assert res["state"] == 2
        assert torch.equal(res["out"], ref["out"])
        # the same through submit_many, one batch submitted twice: behind a
        # busy stream (one shared event), then with the stream idle
        say("server submit_many ordered after the caller's stream")
        from paper_2012_13257_amd.server import Batch
        v3 = torch.zeros_like(v)
        batch = Batch([srv.prepare(p, s, v3, wl.H, wl.W, wl.radius) for _ in range(3)])
        for _ in range(8):
            junk = junk @ junk
            junk = junk / junk.norm()
        v3.copy_(v + 0.0 * junk[0, 0])
        ts = srv.submit_many(batch)
        assert srv.drain(60000)
        for t in ts:
            res = srv.result(t)
            assert res["state"] == 2 and torch.equal(res["out"], ref["out"])
        torch.cuda.synchronize()
        ts = srv.submit_many(batch)
        assert not batch.has_ready and all(batch.array[i].ready is None for i in range(3))
        assert srv.drain(60000)
        for t in ts:
            res = srv.result(t)
            assert res["state"] == 2 and torch.equal(res["out"], ref["out"])


def test_server_budget_and_argument_errors():
    import torch
    from paper_2012_13257_amd import _lib
    from paper_2012_13257_amd.server import Server
    wl = synth.random_workload(5, 1, 5000, 512, 512, C=3, sigma=1.0)
    p, s, v = (torch.from_numpy(wl.pos).cuda(), torch.from_numpy(wl.sigma).cuda(),
               torch.from_numpy(wl.values).cuda())
    with Server(budget_bytes=1 << 20, max_slots=4) as srv:
        with pytest.raises(_lib.InterpError) as e:
            srv.submit(p, s, v, wl.H, wl.W)           # needs more than 1 MiB of state
        assert e.value.code == _lib.INTERP_ENOMEM
    wl5 = synth.random_workload(6, 1, 100, 16, 16, C=5, sigma=1.0)
    with Server(budget_bytes=64 << 20, max_slots=4) as srv:
        p5, s5, v5 = (torch.from_numpy(wl5.pos).cuda(), torch.from_numpy(wl5.sigma).cuda(),
                      torch.from_numpy(wl5.values).cuda())
        with pytest.raises(_lib.InterpError) as e:
            srv.submit(p5, s5, v5, 16, 16)
        assert e.value.code == _lib.INTERP_EINVAL
        # float32 storage only on the serving path
        with pytest.raises(_lib.InterpError) as e:
            srv.submit(p5, s5, v5[:, :, :4].to(torch.bfloat16).contiguous(), 16, 16)
        assert e.value.code == _lib.INTERP_EINVAL
        # and the plain isotropic kernel only
        from paper_2012_13257_amd import interp
        v4 = v5[:, :, :4].contiguous()
        o4 = torch.empty((1, 4, 16, 16), device="cuda")
        for kern in (_lib.KERNEL_NORMALIZED, _lib.KERNEL_DIAGONAL):
            req = _lib.Request()
            req.prob = interp.problem(p5, s5, v4, 16, 16)
            req.prob.kernel = kern
            req.pos, req.sigma, req.values, req.out = (p5.data_ptr(), s5.data_ptr(),
                                                       v4.data_ptr(), o4.data_ptr())
            ticket = ctypes.c_uint64()
            rc = _lib.lib().interp_submit(srv._h, ctypes.byref(req), ctypes.byref(ticket))
            assert rc == _lib.INTERP_EINVAL, kern
        # the server still serves valid requests afterwards
        t = srv.submit(p5[:, :, :], s5, v5[:, :, :4].contiguous(), 16, 16)
        assert srv.drain(30000)
        assert srv.result(t)["state"] == 2


def test_server_many_requests_small_budget_completes():
    """More state than the budget holds at once: admission waits for memory."""
    import torch
    from paper_2012_13257_amd.server import Server
    reqs = _requests(40, 7, sides=(64, 128))
    dev = [_dev(wl) for _, wl in reqs]
    torch.cuda.synchronize()
    with Server(budget_bytes=24 << 20, max_slots=64) as srv:
        ts = [srv.submit(p, s, v, wl.H, wl.W, wl.radius, grad_out=G if r.backward else None)
              for (r, wl), (p, s, v, G) in zip(reqs, dev)]
        assert srv.drain(120000)
        for t in ts:
            assert srv.result(t)["state"] == 2


def test_server_three_pass_request_alone_and_in_mix():
    """A 2056 x 2056 request has 257 x 257 bins (17 key bits): its batch replays
    the graph with three radix passes; with and without the backward, alone and
    next to small requests, its bits equal the single-call path's."""
    import torch
    from paper_2012_13257_amd.server import Server
    big = synth.random_workload(4713, 1, 30000, 2056, 2056, C=3, sigma=1.1, blob_frac=0.5,
                                blob_std=(20.0, 80.0))
    small = _requests(6, 55, sides=(32, 64))
    pb, sb, vb, Gb = _dev(big)
    dev = [_dev(wl) for _, wl in small]
    torch.cuda.synchronize()
    ref_f = _single(pb, sb, vb, Gb, big, False)
    ref_b = _single(pb, sb, vb, Gb, big, True)
    ref_s = [_single(p, s, v, G, wl, r.backward) for (r, wl), (p, s, v, G) in zip(small, dev)]
    torch.cuda.synchronize()
    say("server three-pass request", big.H, big.W, big.N)
    with Server(budget_bytes=2 << 30, max_slots=16) as srv:
        for G, ref in ((None, ref_f), (Gb, ref_b)):
            t = srv.submit(pb, sb, vb, big.H, big.W, big.radius, grad_out=G)
            assert srv.drain(60000)
            res = srv.result(t)
            assert res["state"] == 2, res
            for key, val in ref.items():
                assert torch.equal(res[key], val), ("alone", key)
        tickets = [srv.submit(pb, sb, vb, big.H, big.W, big.radius, grad_out=Gb)]
        for (r, wl), (p, s, v, G) in zip(small, dev):
            tickets.append(srv.submit(p, s, v, wl.H, wl.W, wl.radius,
                                      grad_out=G if r.backward else None))
        assert srv.drain(60000)
        for k, (t, ref) in enumerate(zip(tickets, [ref_b] + ref_s)):
            res = srv.result(t)
            assert res["state"] == 2, (k, res)
            for key, val in ref.items():
                assert torch.equal(res[key], val), ("mix", k, key)
