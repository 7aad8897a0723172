"""GPU: the continuous-batching server.

Each request's result must be bitwise the same alone (a plain call) and in
the mix (submitted together with others, batched and run concurrently), and
match the CPU oracle; the server must respect its HBM budget and report its
limits with the documented status codes.
"""
import numpy as np
import pytest
import torch

from paper_2411_19702_amd import mi, synth
import oracle
from tests.gpu_util import say

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _requests(count, seed=5, m_range=(1000, 40_000), n_range=(128, 900)):
    reqs = synth.request_trace(seed=seed, count=count, qps=1e6, m_range=m_range, n_range=n_range)
    return [r.spec for r in reqs]


def test_results_identical_alone_and_in_the_mix():
    specs = _requests(24)
    say(f"[server] {len(specs)} requests, alone vs mix")
    Xs = [synth.generate(s, device=DEV) for s in specs]
    torch.cuda.synchronize()                          # the server runs on its own streams
    alone = []
    for X, s in zip(Xs, specs):
        o = torch.empty((s.n, s.n), device=DEV)
        mi.mi_all_pairs_ex(X, out=o)
        alone.append(o)
    torch.cuda.synchronize()
    outs = [torch.full((s.n, s.n), float("nan"), device=DEV) for s in specs]
    with mi.Server(hbm_budget_bytes=64 << 30, max_slots=4) as srv:
        tickets = [srv.submit(X, o) for X, o in zip(Xs, outs)]
        lat = [srv.wait(t, timeout_s=120) for t in tickets]
        st = srv.stats()
    assert all(v > 0 for v in lat)
    assert st["submitted"] == st["completed"] == len(specs)
    assert st["batches"] <= len(specs)
    for a, b in zip(alone, outs):
        assert torch.equal(a, b), "a request's result changed when it ran in the mix"
    order = np.argsort([s.m * s.n * s.n for s in specs])
    for d in order[:3]:
        _, o_mi = oracle.all_pairs(Xs[d].cpu().numpy())
        assert np.max(np.abs(outs[d].cpu().numpy().astype(np.float64) - o_mi)) <= 1e-5


def test_budget_is_respected_and_oversize_rejected():
    specs = _requests(10, seed=9, m_range=(20_000, 40_000), n_range=(300, 600))
    Xs = [synth.generate(s, device=DEV) for s in specs]
    torch.cuda.synchronize()                          # the server runs on its own streams
    outs = [torch.empty((s.n, s.n), device=DEV) for s in specs]
    need = [s.m * s.n + 4 * s.n * s.n for s in specs]
    budget = int(max(need) * 2.5) + (64 << 20)       # room for about two requests at once
    say(f"[server] budget {budget / 2**20:.0f} MiB")
    with mi.Server(hbm_budget_bytes=budget, max_slots=4) as srv:
        tickets = [srv.submit(X, o) for X, o in zip(Xs, outs)]
        for t in tickets:
            srv.wait(t, timeout_s=120)
        st = srv.stats()
        assert st["max_bytes_in_flight"] <= budget
        assert st["bytes_in_flight"] == 0
        big = torch.zeros((budget // 100 + 1, 128), dtype=torch.uint8, device=DEV)
        torch.cuda.synchronize()
        with pytest.raises(mi.MIError) as ei:
            srv.submit(big, torch.empty((128, 128), device=DEV))
        assert ei.value.status == 4                    # MI_ERR_BUDGET
    for X, o, s in list(zip(Xs, outs, specs))[:2]:
        ref = torch.empty_like(o)
        mi.mi_all_pairs_ex(X, out=ref)
        torch.cuda.synchronize()
        assert torch.equal(ref, o)


def test_poll_wait_and_unknown_ticket():
    spec = synth.spec_random(77, 50_000, 512, 0.01, 0.5)
    X = synth.generate(spec, device=DEV)
    out = torch.empty((512, 512), device=DEV)
    torch.cuda.synchronize()
    with mi.Server(hbm_budget_bytes=8 << 30, max_slots=1) as srv:
        t = srv.submit(X, out)
        lat = srv.wait(t, timeout_s=60)
        assert lat > 0
        with pytest.raises(mi.MIError) as ei:
            srv.poll(t)                                # already collected
        assert ei.value.status == 9
        t2 = srv.submit(X, out, n=256)
        while not srv.poll(t2):
            pass
        srv.wait(t2)
    ref = torch.empty((512, 512), device=DEV)
    mi.mi_all_pairs_ex(X, out=ref)
    torch.cuda.synchronize()
    got = out.view(-1)[: 256 * 256].view(256, 256)     # an n = 256 result is a dense 256 x 256 matrix
    assert torch.equal(ref[:256, :256], got)


def test_many_small_requests_are_batched():
    specs = _requests(64, seed=13, m_range=(1000, 3000), n_range=(128, 256))
    Xs = [synth.generate(s, device=DEV) for s in specs]
    torch.cuda.synchronize()                          # the server runs on its own streams
    outs = [torch.empty((s.n, s.n), device=DEV) for s in specs]
    with mi.Server(hbm_budget_bytes=16 << 30, max_slots=2) as srv:
        tickets = [srv.submit(X, o) for X, o in zip(Xs, outs)]
        for t in tickets:
            srv.wait(t, timeout_s=60)
        st = srv.stats()
    assert st["batches"] < len(specs), st
    for X, o in list(zip(Xs, outs))[::9]:
        ref = torch.empty_like(o)
        mi.mi_all_pairs_ex(X, out=ref)
        torch.cuda.synchronize()
        assert torch.equal(ref, o)
