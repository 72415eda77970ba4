"""Continuous-batching server: completion, alone == in-mix, budgeted admission."""
import numpy as np
import pytest
import torch

from helpers import TOL_F32, TOL_LOWP, dev, rel, to_np
from oracle import filters, nudft
from oracle.geometry import Geometry
from paper_2401_11101_amd import Plan
from paper_2401_11101_amd.serve import Request, Server, run_poisson

pytestmark = pytest.mark.gpu

CLASSES = [(32, 32, 40, 32, 32), (24, 48, 60, 24, 48), (40, 40, 30, 40, 40)]


def _data(shape, seed):
    nz, n, nt, h, w = shape
    g = torch.Generator(device="cpu").manual_seed(seed)
    return torch.randn((nt, h, w), generator=g).to(dev())


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_request_alone_equals_in_mix(storage):
    shape = CLASSES[0]
    tilt = np.deg2rad(27.0)
    data = _data(shape, 0)
    alone = Plan(*shape, tilt, storage_dtype=storage).fbp(data)
    torch.cuda.synchronize()
    srv = Server(max_slots=4, storage_dtype=storage)
    reqs = []
    for i in range(12):
        cls = CLASSES[i % 3]
        if i == 5:
            r = Request(i, *shape, tilt, data)
        else:
            r = Request(i, *cls, np.deg2rad(20 + i), _data(cls, 100 + i))
        reqs.append(r)
        srv.submit(r)
        srv.poll()
    srv.drain()
    assert len(srv.finished) == 12
    mixed = reqs[5].out
    torch.cuda.synchronize()
    diff = float((mixed - alone).abs().max())
    print(f"{storage}: max |in-mix - alone| = {diff:.3e}")
    assert diff <= 1e-6 * float(alone.abs().max())
    # every served volume against the exact FBP sums at its own shape and tilt
    tol = TOL_F32 if storage == "f32" else TOL_LOWP
    worst = 0.0
    for r in reqs:
        nz, n, nt, h, w = r.shape
        g = Geometry(nz=nz, n=n, n_theta=nt, h=h, w=w, phi=r.tilt)
        e = rel(to_np(r.out), nudft.fbp(to_np(r.data), g, filters.SHEPP_LOGAN))
        worst = max(worst, e)
        assert e < tol, (r.rid, e)
    print(f"{storage}: served volumes vs exact FBP, worst rel-L2 {worst:.2e}")
    srv.close()


def test_budget_limits_concurrency():
    shape = CLASSES[1]
    probe = Plan(*shape, 0.4, storage_dtype="f16")
    one = probe.tables.numel() + probe.work.numel()
    srv = Server(max_slots=4, hbm_budget=int(1.5 * one), storage_dtype="f16")
    for i in range(6):
        srv.submit(Request(i, *shape, 0.3 + 0.01 * i, _data(shape, i)))
        assert sum(s.busy is not None for s in srv.slots) <= 1
    srv.drain()
    assert len(srv.finished) == 6
    assert len(srv.slots) == 1
    srv.close()


def test_request_above_budget_is_refused_at_submission():
    # a request that cannot fit even alone (slot + output volume) raises
    # instead of waiting forever; the output volume counts against the budget
    shape = CLASSES[1]
    probe = Plan(*shape, 0.4, storage_dtype="f16")
    slot_bytes = probe.tables.numel() + probe.work.numel()
    out_bytes = shape[0] * shape[1] * shape[1] * 4
    srv = Server(max_slots=2, hbm_budget=slot_bytes + out_bytes - 1, storage_dtype="f16")
    with pytest.raises(ValueError):
        srv.submit(Request(0, *shape, 0.3, _data(shape, 0)))
    assert not srv.queue and not srv.slots
    srv.hbm_budget = slot_bytes + out_bytes
    r = Request(1, *shape, 0.3, _data(shape, 1))
    srv.submit(r)
    srv.drain()
    assert srv.finished == [r]
    srv.close()


def test_poisson_stream_reports_latency():
    classes = [(*c, _data(c, j)) for j, c in enumerate(CLASSES)]
    srv = Server(max_slots=3, storage_dtype="f16")
    st = run_poisson(srv, classes, rate=200.0, count=40, seed=0)
    print(st)
    assert st["requests"] == 40 and st["p99_ms"] >= st["p50_ms"] > 0
    srv.close()


def test_host_resident_requests_match_device_resident():
    # data in pinned host memory, volumes returned to pinned host memory:
    # the copies run on each request's slot stream, the results equal those
    # of device-resident requests bit for bit, and unpinned host data are
    # refused before anything is enqueued
    reqs_dev, reqs_host = [], []
    srv_d = Server(max_slots=3, storage_dtype="f16")
    srv_h = Server(max_slots=3, storage_dtype="f16", result_on_host=True)
    for i in range(9):
        cls = CLASSES[i % 3]
        tilt = np.deg2rad(22 + i)
        d = _data(cls, 200 + i)
        rd = Request(i, *cls, tilt, d)
        rh = Request(i, *cls, tilt, d.cpu().pin_memory())
        reqs_dev.append(rd)
        reqs_host.append(rh)
        srv_d.submit(rd)
        srv_h.submit(rh)
        srv_d.poll()
        srv_h.poll()
    srv_d.drain()
    srv_h.drain()
    torch.cuda.synchronize()
    for rd, rh in zip(reqs_dev, reqs_host):
        assert rh.out_host is not None and rh.out_host.device.type == "cpu" and rh.out_host.is_pinned()
        assert torch.equal(rh.out_host, rd.out.cpu()), rd.rid
        assert rh.done >= rh.arrival
    with pytest.raises(ValueError):
        srv_h.submit(Request(99, *CLASSES[0], 0.4, _data(CLASSES[0], 7).cpu()))
    assert not srv_h.queue
    srv_d.close()
    srv_h.close()
