"""Batched systems (ILU(0) + GMRES(m) each, one persistent launch) against the FP64 oracle, through the C ABI.

Bars: level of every row in L and U bit-exact; ILU(0) factor values bit-exact
(the same IKJ operations in the same order); per system the oracle's GMRES
iteration count +-1, the true relative residual <= rtol, and x close to the
oracle's.  Launch schedules (narrow-level merge, workgroups per CU) change no
arithmetic, so their results are compared bit for bit, and so are graph
replays with the direct launch.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def silu():
    import paper_2303_08881_amd as m

    return m


def small_batch():
    # ragged sizes (1x1 up to 40x40 grids, non-square counts of rows), all three stencil parameters varied
    sides = [1, 2, 3, 7, 16, 40, 33, 25, 9, 12, 31, 5]
    mats = []
    for k, s in enumerate(sides):
        eps = [1.0, 0.3, 0.01, 1e-3][k % 4]
        mats.append(synth.convdiff5(s, eps, 0.4 * k, 7.0 * k))
    mats.append(synth.aniso5(20, 0.01, Ny=13))
    mats.append(synth.rotated9(11))  # 4 entries per triangle
    return mats


@pytest.fixture(scope="module")
def batch_run():
    m = silu()
    mats = small_batch()
    A, sys_row = synth.block_diagonal(mats)
    b = np.concatenate([synth.uniform_rhs(M.n, 40 + k) for k, M in enumerate(mats)])
    print(f"[batch] small batch: {len(mats)} systems, n={A.n}", flush=True)
    Ad = m.DeviceCSR.from_host(A)
    B = m.batch_setup(Ad, sys_row, restart=20)
    bd = torch.as_tensor(b).cuda()
    x = torch.zeros_like(bd)
    B.solve(Ad.val, bd, x, rtol=1e-8, restart=20, maxit=2000)
    its, rel, st = B.results()
    return dict(m=m, mats=mats, A=A, sys_row=sys_row, b=b, Ad=Ad, B=B, bd=bd, x=x.cpu().numpy(), its=its, rel=rel,
                st=st)


def test_batch_levels_and_factors_bit_exact(batch_run):
    r = batch_run
    lev_L, lev_U, lu = r["B"].export("lev_L"), r["B"].export("lev_U"), r["B"].export("lu")
    A, sr = r["A"], r["sys_row"]
    for k, M in enumerate(r["mats"]):
        a, e = sr[k], sr[k + 1]
        F = oracle.factor(M, method=oracle.ILU0)
        Lo = M.row_ptr  # factor values on A's pattern: L | D | U of each row, in column order
        ref = np.empty(M.nnz)
        Lrp, Lci, Lv = F["L"]
        Urp, Uci, Uv = F["U"]
        for i in range(M.n):
            ref[Lo[i]:Lo[i + 1]] = np.concatenate([Lv[Lrp[i]:Lrp[i + 1]], [F["D"][i]], Uv[Urp[i]:Urp[i + 1]]])
        np.testing.assert_array_equal(lu[A.row_ptr[a]:A.row_ptr[e]], ref, err_msg=f"factor of system {k}")
        lower = oracle.levels(Lrp, Lci, True)
        upper = oracle.levels(Urp, Uci, False)
        np.testing.assert_array_equal(lev_L[a:e], lower, err_msg=f"L levels of system {k}")
        np.testing.assert_array_equal(lev_U[a:e], upper, err_msg=f"U levels of system {k}")


def test_batch_gmres_matches_oracle(batch_run):
    r = batch_run
    sr = r["sys_row"]
    assert np.all(r["st"] == 0), r["st"]
    for k, M in enumerate(r["mats"]):
        a, e = sr[k], sr[k + 1]
        P = oracle.Precond(M, None, 1, method=oracle.BJ, interior_fact=oracle.ILU0)
        ro = oracle.gmres(M, P, r["b"][a:e], rtol=1e-8, restart=20, maxit=2000)
        assert ro["converged"]
        assert abs(int(r["its"][k]) - ro["iterations"]) <= 1, (k, r["its"][k], ro["iterations"])
        xg = r["x"][a:e]
        true = np.linalg.norm(oracle.residual(M, r["b"][a:e], xg)) / np.linalg.norm(r["b"][a:e])
        assert true <= 1e-8 and abs(true - r["rel"][k]) <= 1e-12 * max(1.0, true), (k, true, r["rel"][k])
        np.testing.assert_allclose(xg, ro["x"], rtol=0, atol=1e-6 * np.abs(ro["x"]).max(), err_msg=f"system {k}")


def test_batch_schedules_and_graph_replay_are_bit_identical(batch_run):
    r = batch_run
    m, B, Ad, bd = r["m"], r["B"], r["Ad"], r["bd"]
    ref = r["x"]
    for merge, wpc in [(0, 1), (64, 1), (16, 2)]:
        B.schedule(merge, wpc)
        x = torch.zeros_like(bd)
        B.solve(Ad.val, bd, x, rtol=1e-8, restart=20, maxit=2000)
        np.testing.assert_array_equal(x.cpu().numpy(), ref, err_msg=f"schedule {merge} {wpc}")
        np.testing.assert_array_equal(B.results()[0], r["its"])
    # 512 threads per workgroup: dot products summed over 8 wavefronts instead of 4, so x agrees to rounding
    # (and the iteration counts within one); back to 256 threads for the graph replays below
    B.schedule(32, 1, 512)
    assert B.export("schedule")[4] == 512
    x = torch.zeros_like(bd)
    B.solve(Ad.val, bd, x, rtol=1e-8, restart=20, maxit=2000)
    its512, rel512, st512 = B.results()
    assert np.all(st512 == 0) and np.all(np.abs(its512 - r["its"]) <= 1)
    np.testing.assert_allclose(x.cpu().numpy(), ref, rtol=0, atol=1e-6 * np.abs(ref).max())
    B.schedule(32, 1, 256)
    side = torch.cuda.Stream()
    x = torch.zeros_like(bd)
    with torch.cuda.stream(side):
        B.capture(Ad.val, bd, x, rtol=1e-8, restart=20, maxit=2000)
    for rep in range(3):
        with torch.cuda.stream(side):
            x.zero_()
            B.replay()
        side.synchronize()
        np.testing.assert_array_equal(x.cpu().numpy(), ref, err_msg=f"replay {rep}")
        its, rel, st = B.results()
        np.testing.assert_array_equal(its, r["its"])
        y = m.spmv(Ad, torch.ones_like(bd))  # other eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()


def test_batch_tuner_picks_a_valid_schedule(batch_run):
    r = batch_run
    B, Ad, bd = r["B"], r["Ad"], r["bd"]
    x = torch.zeros_like(bd)
    merge, wpc, threads, ms = B.tune(Ad.val, bd, x, rtol=1e-8, restart=20, maxit=2000)
    assert merge in (0, 16, 32, 64) and wpc >= 1 and threads in (256, 512) and ms > 0
    sch = B.export("schedule")
    assert sch[1] == merge and sch[2] == wpc and sch[4] == threads
    assert float(x.abs().max()) == 0.0  # the initial guess is back
    # every candidate ran the whole solve: the last one's iteration counts are the batch's (to one)
    assert np.all(np.abs(B.results()[0] - r["its"]) <= 1)
    B.solve(Ad.val, bd, x, rtol=1e-8, restart=20, maxit=2000)
    if threads == 256:
        np.testing.assert_array_equal(x.cpu().numpy(), r["x"])
    else:
        np.testing.assert_allclose(x.cpu().numpy(), r["x"], rtol=0, atol=1e-6 * np.abs(r["x"]).max())
    B.schedule(32, 1, 256)


def test_batch_status_codes():
    m = silu()
    # system 0 converges, system 1 has a zero pivot, system 2 stops at maxit, system 3 has b = 0
    mats = [synth.convdiff5(6, 0.1, 0.3, 5.0), synth.CSR.from_dense(np.array([[0.0, 1.0], [1.0, 1.0]])),
            synth.aniso5(30, 1.0), synth.aniso5(3, 1.0)]
    A, sr = synth.block_diagonal(mats)
    b = np.concatenate([np.ones(mats[0].n), np.ones(2), synth.uniform_rhs(mats[2].n, 3), np.zeros(mats[3].n)])
    Ad = m.DeviceCSR.from_host(A)
    B = m.batch_setup(Ad, sr, restart=5)
    x = torch.full((A.n,), 2.0, dtype=torch.float64, device="cuda")
    print("[batch] status codes", flush=True)
    B.solve(Ad.val, torch.as_tensor(b).cuda(), x, rtol=1e-10, restart=5, maxit=12)
    its, rel, st = B.results()
    assert st[0] == 0 and st[1] == -3 and st[2] == m.NOT_CONVERGED and st[3] == 0
    assert its[2] == 12
    xs = x.cpu().numpy()
    assert np.all(xs[sr[3]:sr[4]] == 0.0)  # b = 0 gives x = 0 whatever the initial guess
    with pytest.raises(m.SchurILUError):
        B.solve(Ad.val, torch.as_tensor(b).cuda(), x, rtol=1e-10, restart=6, maxit=12)  # above the setup's restart


@pytest.mark.slow
def test_batch_full_512_systems():
    # the batched workload: 512 convection-diffusion systems, sides log-uniform in [32, 256]
    m = silu()
    mats, bs = synth.convdiff_batch(512, 4)
    A, sr = synth.block_diagonal(mats)
    b = np.concatenate(bs)
    print(f"[batch] 512 systems, n={A.n}, nnz={A.nnz}", flush=True)
    Ad = m.DeviceCSR.from_host(A)
    B = m.batch_setup(Ad, sr, restart=20)
    bd = torch.as_tensor(b).cuda()
    x = torch.zeros_like(bd)
    B.solve(Ad.val, bd, x, rtol=1e-8, restart=20, maxit=5000)
    its, rel, st = B.results()
    assert np.all(st == 0) and np.all(rel <= 1e-8), (st.min(), rel.max())
    xs = x.cpu().numpy()
    # sampled systems against the oracle: the largest, the smallest and a spread of others
    order = np.argsort([M.n for M in mats])
    for k in sorted(set([int(order[-1]), int(order[0])] + list(range(0, 512, 37)))):
        M = mats[k]
        P = oracle.Precond(M, None, 1, method=oracle.BJ, interior_fact=oracle.ILU0)
        ro = oracle.gmres(M, P, bs[k], rtol=1e-8, restart=20, maxit=5000)
        assert abs(int(its[k]) - ro["iterations"]) <= 1, (k, its[k], ro["iterations"])
        true = np.linalg.norm(oracle.residual(M, bs[k], xs[sr[k]:sr[k + 1]])) / np.linalg.norm(bs[k])
        assert true <= 1e-8
