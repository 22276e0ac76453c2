"""Serving loop: results are the same alone and in a concurrent mix; drift
steps with a recycled tree keep the accuracy; HBM admission limits
concurrency."""
import numpy as np
import pytest

import oracle
from paper_1405_2255_amd import workloads as W

pytestmark = pytest.mark.gpu


def _request(serve, kind, n, seed, eps, steps=1):
    import torch
    pos, vel = W.plummer(n, seed, with_velocities=True) if kind == "plummer" else (
        W.cluster(kind, n, seed)[0], np.zeros((n, 3)))
    m = np.full(n, 1.0 / n)
    dev = "cuda"
    return serve.Request(pos=torch.from_numpy(np.ascontiguousarray(pos)).to(dev),
                         mass=torch.from_numpy(m).to(dev), target_err=eps, steps=steps,
                         vel=torch.from_numpy(np.ascontiguousarray(vel)).to(dev), dt=1e-3)


def test_same_alone_and_in_the_mix():
    import torch
    from paper_1405_2255_amd import serve
    specs = [("plummer", 30000, 1, 1e-7, 3), ("dehnen1", 12000, 2, 1e-6, 1),
             ("uniform", 5000, 3, 1e-5, 2), ("plummer", 60000, 4, 1e-6, 2),
             ("dehnen0", 2000, 5, 1e-7, 1), ("plummer", 9000, 6, 1e-7, 4)]
    mix = serve.Server(slots=3)
    reqs = [mix.submit(_request(serve, *s)) for s in specs]
    out_mix = [r.result(120) for r in reqs]
    assert mix.max_running >= 2          # they did overlap
    mix.close()
    alone = serve.Server(slots=1)
    for s, (pm, am) in zip(specs, out_mix):
        print("request", s, flush=True)
        r = alone.submit(_request(serve, *s))
        pa, aa = r.result(120)
        assert torch.equal(pa, pm) and torch.equal(aa, am)
    alone.close()


def test_drift_steps_keep_accuracy():
    """10 drift steps with the tree recycled and the previous step's |a| as
    the scale: every step within the bound of a fresh evaluation."""
    import torch
    from paper_1405_2255_amd import serve
    srv = serve.Server(slots=1)
    req = _request(serve, "plummer", 20000, 11, 1e-7, steps=10)
    req.keep_all = True
    srv.submit(req).result(120)
    srv.close()
    pos0 = req.pos.cpu().numpy()
    vel = req.vel.cpu().numpy()
    m = req.mass.cpu().numpy()
    sinks = np.random.default_rng(0).choice(20000, 1500, replace=False)
    for step, (_, acc, st) in enumerate(req.history):
        pos = pos0 + step * 1e-3 * vel
        _, a0, _ = oracle.direct(pos, m, sinks=sinks)
        e = np.linalg.norm(acc.cpu().numpy()[sinks] - a0, axis=1) / np.linalg.norm(a0, axis=1)
        assert st["refitted"] == (1 if step > 0 else 0)
        assert np.sqrt(np.mean(e ** 2)) < 2e-7, step


def test_refit_without_motion_equals_fresh_build(gpu_lib):
    import torch
    pos, m = W.cluster("plummer", 15000, 3)
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(m).cuda()
    c = gpu_lib.Context()
    p1, a1 = c.forces(P, M, p=10, target_err=1e-7)
    p1, a1 = p1.clone(), a1.clone()
    p2, a2 = c.forces(P, M, p=10, target_err=1e-7, refit=True)
    torch.cuda.synchronize()
    assert c.stats()["refitted"] == 1
    assert torch.equal(p1, p2) and torch.equal(a1, a2)


def test_admission_budget_serialises():
    from paper_1405_2255_amd import fmm, serve
    need = fmm.footprint_bytes(20000, 11)
    srv = serve.Server(slots=4, budget_bytes=int(need * 1.5))
    reqs = [srv.submit(_request(serve, "plummer", 20000, 20 + i, 1e-7)) for i in range(4)]
    for r in reqs:
        r.result(120)
    assert srv.max_running == 1
    big = srv.submit(_request(serve, "plummer", 200000, 9, 1e-7))
    with pytest.raises(MemoryError):
        big.result(10)
    srv.close()
