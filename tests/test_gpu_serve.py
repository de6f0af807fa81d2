"""Continuous-batching service: each request's result is the same alone and in
the mix (bitwise: the batch runs the same march code on every grid and the
results do not depend on the tiling), requests that arrive while others run
are admitted as slots and memory free up, and the HBM pool never exceeds its
budget."""
import numpy as np
import pytest

from paper_2007_07760_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2007_07760_amd import _lib
    _lib.load()
    from paper_2007_07760_amd import serve as S
    return S


def _trace():
    return I.serve_trace(count=14, rate=2000.0, nmin=24, nmax=160, smin=20, smax=150,
                         seed=3)


def test_serve_mix_equals_alone(serve):
    trace = _trace()
    big = max(serve.state_bytes(r) for r in trace)
    budget = 3 * big + 4096          # at most ~3 large states at once: queueing
    print(f"case serve 14 requests, budget {budget} B", flush=True)
    srv = serve.Server(slots=5, budget_bytes=budget, graph_steps=8)
    res = srv.run(trace, keep_phi=[r["id"] for r in trace])
    assert [r.id for r in res] == [r["id"] for r in trace]
    assert srv.pool.used == 0 and srv.pool.peak <= srv.pool.nbytes
    assert 1 <= srv.slots_peak <= 5
    print(f"pool peak {srv.pool.peak} B, slots peak {srv.slots_peak}, rounds with a free "
          f"slot held back by the budget {srv.budget_blocked_rounds}", flush=True)
    for r, req in zip(res, trace):
        assert r.done >= r.admitted >= r.arrival - 1e-9
        ref = serve.run_alone(req)
        assert np.array_equal(r.phi, ref), req["id"]
    st = serve.summary(res)
    print(st, flush=True)
    assert st["p99_s"] >= st["p50_s"] > 0


def test_serve_fifo_baseline_equals_alone(serve):
    trace = _trace()[:4]
    print("case serve fifo", flush=True)
    res = serve.run_fifo(trace, keep_phi=[r["id"] for r in trace])
    for r, req in zip(res, trace):
        assert np.array_equal(r.phi, serve.run_alone(req)), req["id"]


def test_serve_rejects_oversized(serve):
    trace = _trace()[:2]
    srv = serve.Server(slots=2, budget_bytes=64 << 10)
    with pytest.raises(ValueError):
        srv.run(trace)


def test_serve_fails_only_the_blown_up_request(serve, monkeypatch):
    """A request whose solve is non-finite (here: a NaN planted in its phi0)
    fails alone with status ENUMERIC; every other request completes and equals
    its alone run."""
    from paper_2007_07760_amd import _lib as C
    trace = _trace()[:6]
    victim = trace[2]["id"]
    real = serve.request_phi0

    def poisoned(req, device):
        phi = real(req, device)
        if req["id"] == victim:
            phi[3, 4] = float("nan")
        return phi

    monkeypatch.setattr(serve, "request_phi0", poisoned)
    print("case serve blow-up", flush=True)
    srv = serve.Server(slots=3, budget_bytes=64 << 20, graph_steps=8)
    res = srv.run(trace, keep_phi=[r["id"] for r in trace])
    monkeypatch.setattr(serve, "request_phi0", real)
    assert srv.pool.used == 0
    for r, req in zip(res, trace):
        if req["id"] == victim:
            assert r.status == C.ENUMERIC and r.phi is None and r.steps < req["steps"]
        else:
            assert r.status == C.OK
            assert np.array_equal(r.phi, serve.run_alone(req)), req["id"]
    assert serve.summary(res)["failed"] == 1
