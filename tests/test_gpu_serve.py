"""Serving through the C ABI: continuous batching of solve requests with resident factors per matrix id.

Bars: every request's result is the same alone (one slot, each request
waited for before the next is submitted) and in the mix (four slots, all
requests queued at once, setups and solves overlapping): status and
iteration count equal and x bit-identical, since each request issues the
same deterministic kernels whatever else runs.  Served solves reach the
true relative residual rtol, and with FP64 factors they take the oracle's
iteration count +-1.  A tight budget evicts idle factors and still serves
every request; a request larger than the budget and one for an unknown id
are rejected with their codes.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

RTOL = 1e-8


def silu():
    import paper_2303_08881_amd as m

    return m


def opts(prec=None):
    m = silu()
    return dict(method=m.SCHUR, interior_fact=m.ILU0, interface_fact=m.MILU0, inner_iters=3,
                factor_prec=m.PREC_F32 if prec is None else prec)


@pytest.fixture(scope="module")
def stream():
    m = silu()
    reqs = synth.request_stream(16, seed=11, n_min=300, n_max=6000)
    mats, dev = {}, {}
    for r in reqs:
        if r.matrix_id not in mats:
            A, part, p = synth.build_matrix(r, part_rows=1500)
            mats[r.matrix_id] = (A, part, p)
            dev[r.matrix_id] = (m.DeviceCSR.from_host(A), torch.as_tensor(part).cuda(), p)
    bs = [torch.as_tensor(synth.uniform_rhs(mats[r.matrix_id][0].n, r.rhs_seed)).cuda() for r in reqs]
    torch.cuda.synchronize()
    print(f"[serve] {len(reqs)} requests, {len(mats)} matrices, n = "
          f"{sorted(a.n for a, _, _ in mats.values())}", flush=True)
    return reqs, mats, dev, bs


def serve(reqs, dev, bs, slots, serial, budget=4 << 30, prec=None):
    m = silu()
    S = m.Server(slots=slots, budget_bytes=budget, **opts(prec))
    xs = [torch.zeros_like(b) for b in bs]
    recs, tickets = [], []
    for q, r in enumerate(reqs):
        A, part, p = dev[r.matrix_id]
        t = S.submit(r.matrix_id, bs[q], xs[q], A=A if r.new else None, part=part, nparts=p, rtol=RTOL,
                     restart=50, maxit=500)
        if serial:
            recs.append(S.wait(t))
        else:
            tickets.append(t)
    if not serial:
        recs = [S.wait(t) for t in tickets]
    st = S.stats()
    S.close()
    return recs, [x.cpu().numpy() for x in xs], st


def test_alone_equals_in_the_mix(stream):
    reqs, mats, dev, bs = stream
    print("[serve] alone", flush=True)
    alone, xa, st_a = serve(reqs, dev, bs, slots=1, serial=True)
    print("[serve] mix", flush=True)
    mix, xm, st_m = serve(reqs, dev, bs, slots=4, serial=False)
    for q, r in enumerate(reqs):
        a, b = alone[q], mix[q]
        assert a["status"] == 0 and b["status"] == 0, (q, a, b)
        assert a["iterations"] == b["iterations"], (q, a["iterations"], b["iterations"])
        np.testing.assert_array_equal(xa[q], xm[q], err_msg=f"request {q}")
        A = mats[r.matrix_id][0]
        bh = bs[q].cpu().numpy()
        true = np.linalg.norm(oracle.residual(A, bh, xm[q])) / np.linalg.norm(bh)
        assert true <= RTOL, (q, true)
        assert a["cache_hit"] == (0 if r.new else 1) and b["cache_hit"] == a["cache_hit"]
    assert st_a["misses"] == st_m["misses"] == len(mats)
    assert st_a["hits"] == st_m["hits"] == len(reqs) - len(mats)
    # in the mix, requests overlapped in time (started before another one finished)
    spans = sorted((rec["start_us"], rec["done_us"]) for rec in mix)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    assert len({rec["slot"] for rec in mix}) > 1


def test_served_fp64_matches_oracle(stream):
    reqs, mats, dev, bs = stream
    m = silu()
    first = [r for r in reqs if r.new][:4]
    recs, xs, _ = serve(first, dev, [bs[r.index] for r in first], slots=2, serial=False, prec=m.PREC_F64)
    o = opts(m.PREC_F64)
    o.pop("factor_prec")
    for r, rec in zip(first, recs):
        A, part, p = mats[r.matrix_id]
        P = oracle.Precond(A, part, p, **o)
        ro = oracle.fgmres(A, P, bs[r.index].cpu().numpy(), rtol=RTOL, restart=50, maxit=500)
        assert rec["status"] == 0 and ro["converged"]
        assert abs(rec["iterations"] - ro["iterations"]) <= 1, (r, rec["iterations"], ro["iterations"])


def test_budget_evicts_and_rejects(stream):
    reqs, mats, dev, bs = stream
    m = silu()
    new = [r for r in reqs if r.new]
    # each matrix alone: its peak (the reservation while it runs) and its resident bytes afterwards
    peaks, resident = [], []
    for r in new:
        _, _, st = serve([r], dev, [bs[r.index]], slots=1, serial=True)
        peaks.append(st["peak_bytes"])
        resident.append(st["bytes"])
    assert min(resident) > 0
    # room for the largest request alone: serving all of them must evict idle factors on the way
    budget = max(peaks) + (1 << 20)
    assert sum(resident) > budget
    recs, xs, st = serve(new, dev, [bs[r.index] for r in new], slots=2, serial=False, budget=budget)
    assert all(rec["status"] == 0 for rec in recs), [rec["status"] for rec in recs]
    assert st["evictions"] >= 1 and st["peak_bytes"] <= budget and st["bytes"] <= budget, st
    big = new[int(np.argmax(peaks))]
    # a request larger than the whole budget, and one for an id never given a matrix
    S = m.Server(slots=1, budget_bytes=1 << 20, **opts())
    A, part, p = dev[big.matrix_id]
    x = torch.zeros_like(bs[big.index])
    t1 = S.submit(1000, bs[big.index], x, A=A, part=part, nparts=p)
    t2 = S.submit(1001, bs[big.index], x)
    r1, r2 = S.wait(t1), S.wait(t2)
    assert r1["status"] == m.SchurILUError(-4, "").code and "budget" in r1["error"]
    assert r2["status"] == -1 and "not resident" in r2["error"]
    with pytest.raises(m.SchurILUError):
        S.wait(t1)  # collected already
    S.close()
