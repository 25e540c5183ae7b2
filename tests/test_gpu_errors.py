"""Error paths, option paths and mode agreement of the HIP library, through the C ABI.

Every error case here is detected by a host check or by a device-side check
that ends its kernel normally (the CSR validation kernel bounds every access
by the stated nnz; the factorization reports an outgrown working row through
its status word): nothing faults or waits without a bound.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

ERR_CSR, ERR_OOM, ERR_BREAKDOWN, ERR_CAPACITY = -2, -4, -6, -7


def silu():
    import paper_2303_08881_amd as m

    return m


def _dev(n, rp, ci, v):
    m = silu()
    return m.DeviceCSR(n, torch.as_tensor(np.asarray(rp, np.int64)).cuda(),
                       torch.as_tensor(np.asarray(ci, np.int32)).cuda(), torch.as_tensor(np.asarray(v)).cuda())


@pytest.mark.parametrize("defect", ["missing_diag", "duplicate", "col_negative", "col_too_big",
                                    "row_ptr_decreasing", "row_ptr_end"])
def test_setup_rejects_bad_csr(defect):
    # 3x3 tridiagonal [[4,1,0],[1,4,1],[0,1,4]]: row_ptr [0,2,5,7], col [0,1,0,1,2,1,2]
    rp, ci, v = np.array([0, 2, 5, 7]), np.array([0, 1, 0, 1, 2, 1, 2]), np.array([4.0, 1, 1, 4, 1, 1, 4])
    if defect == "missing_diag":
        rp, ci, v = np.array([0, 2, 4, 6]), np.array([0, 1, 0, 2, 1, 2]), np.ones(6)
    elif defect == "duplicate":
        ci[3] = 0  # row 1 = {0, 0, 2}
    elif defect == "col_negative":
        ci[4] = -1
    elif defect == "col_too_big":
        ci[4] = 3
    elif defect == "row_ptr_decreasing":
        rp = np.array([0, 2, 1, 7])
    elif defect == "row_ptr_end":
        rp = np.array([0, 2, 5, 6])  # row_ptr[n] != nnz
    m = silu()
    print(f"[errors] bad csr {defect}", flush=True)
    with pytest.raises(m.SchurILUError) as e:
        m.setup(_dev(3, rp, ci, v))
    assert e.value.code == ERR_CSR, defect


def test_working_row_capacity_is_reported():
    # one row of 700 entries (an arrow matrix) outgrows the on-chip working row of the threshold
    # factorization; ILU(0), factored level by level in the rows' own output slots, has no such limit
    n = 700
    d = np.eye(n) * 4.0
    d[n - 1, :] = -1.0 / n
    d[:, n - 1] = -1.0 / n
    d[n - 1, n - 1] = 4.0
    A = synth.CSR.from_dense(d)
    m = silu()
    print("[errors] capacity", flush=True)
    with pytest.raises(m.SchurILUError) as e:
        m.setup(m.DeviceCSR.from_host(A), interior_fact=m.ILUT, droptol=0.0, lfil=-1)
    assert e.value.code == ERR_CAPACITY
    P = m.setup(m.DeviceCSR.from_host(A))
    r = synth.uniform_rhs(n, 5)
    zo = oracle.Precond(A, None, 1).apply(r)
    np.testing.assert_allclose(P.apply(torch.as_tensor(r).cuda()).cpu().numpy(), zo, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_non_finite_rhs_is_a_breakdown(bad):
    m = silu()
    A = synth.aniso5(12)
    Ad = m.DeviceCSR.from_host(A)
    P = m.setup(Ad)
    b = synth.uniform_rhs(A.n, 3)
    b[17] = bad
    print(f"[errors] rhs {bad}", flush=True)
    with pytest.raises(m.SchurILUError) as e:
        m.fgmres(Ad, P, torch.as_tensor(b).cuda(), rtol=1e-8, restart=30, maxit=100)
    assert e.value.code == ERR_BREAKDOWN


def test_iteration_limit_returns_not_converged():
    m = silu()
    A = synth.aniso5(32, 0.01)
    Ad = m.DeviceCSR.from_host(A)
    P = m.setup(Ad)
    b = synth.uniform_rhs(A.n, 4)
    print("[errors] not converged", flush=True)
    out = m.fgmres(Ad, P, torch.as_tensor(b).cuda(), rtol=1e-12, restart=10, maxit=7)
    assert out["rc"] == m.NOT_CONVERGED and not out["converged"] and out["iterations"] == 7
    x = out["x"].cpu().numpy()
    assert np.all(np.isfinite(x))
    true_rel = np.linalg.norm(oracle.residual(A, b, x)) / np.linalg.norm(b)
    assert abs(true_rel - out["relres"]) <= 1e-12 and true_rel > 1e-12
    Po = oracle.Precond(A, None, 1, method=oracle.BJ)
    ro = oracle.fgmres(A, Po, b, rtol=1e-12, restart=10, maxit=7)
    assert ro["rc"] == oracle.NOT_CONVERGED and ro["iterations"] == 7
    np.testing.assert_allclose(x, ro["x"], rtol=0, atol=1e-10 * np.abs(ro["x"]).max())


@pytest.mark.parametrize("mode", ["block", "levels"])
def test_inner_rtol_matches_oracle(mode):
    # the reduced-system GMRES stops once its estimate reaches inner_rtol ||rhs||
    m = silu()
    A = synth.aniso7(12, Nz=16)
    part = synth.slab_partition(12, 4, Nz=16)
    o = dict(method=oracle.SCHUR, interior_fact=oracle.ILU0, interface_fact=oracle.MILU0, inner_iters=10,
             inner_rtol=1e-3)
    mode_ = m.TRSV_BLOCK if mode == "block" else m.TRSV_LEVELS
    print(f"[errors] inner_rtol {mode}", flush=True)
    P = m.setup(m.DeviceCSR.from_host(A), part, 4, trsv_mode=mode_, **o)
    Po = oracle.Precond(A, part, 4, **o)
    Pk = oracle.Precond(A, part, 4, **dict(o, inner_rtol=0.0))
    r = synth.uniform_rhs(A.n, 21)
    zo, zk = Po.apply(r), Pk.apply(r)
    assert np.abs(zo - zk).max() > 1e-8 * np.abs(zk).max()  # the early exit changes the result
    zg = P.apply(torch.as_tensor(r).cuda()).cpu().numpy()
    np.testing.assert_allclose(zg, zo, rtol=1e-10, atol=1e-10 * np.abs(zo).max())


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_block_and_level_modes_build_one_preconditioner(prec):
    # With FP32 / FP16 factors both solve modes round the same factors (L_B,
    # U_B, L_S, U_S) and keep W and Z in FP64, so their applies agree with each
    # other to within the rounding of the lower-precision solves.
    m = silu()
    A = synth.aniso7(12, Nz=16)
    part = synth.slab_partition(12, 4, Nz=16)
    o = dict(method=oracle.SCHUR, interior_fact=oracle.ILUT, interface_fact=oracle.MILU0, inner_iters=5,
             droptol=1e-3, lfil=20)
    fp = m.PREC_F32 if prec == "f32" else m.PREC_F16
    print(f"[errors] block vs levels {prec}", flush=True)
    Ad = m.DeviceCSR.from_host(A)
    Pb = m.setup(Ad, part, 4, trsv_mode=m.TRSV_BLOCK, factor_prec=fp, **o)
    Pl = m.setup(Ad, part, 4, trsv_mode=m.TRSV_LEVELS, factor_prec=fp, **o)
    r = torch.as_tensor(synth.uniform_rhs(A.n, 23)).cuda()
    zb, zl = Pb.apply(r).cpu().numpy(), Pl.apply(r).cpu().numpy()
    zo = oracle.Precond(A, part, 4, **o).apply(r.cpu().numpy())
    tol = {"f32": 1e-5, "f16": 5e-3}[prec]
    scale = np.abs(zo).max()
    assert np.abs(zb - zo).max() <= tol * scale and np.abs(zl - zo).max() <= tol * scale
    # the two modes differ by the solves' rounding only (sum order, reciprocal of the diagonal)
    assert np.abs(zb - zl).max() <= {"f32": 1e-5, "f16": 1e-3}[prec] * scale


def test_workspace_allocation_failure_then_retry():
    # An FGMRES workspace that cannot be allocated returns ILU_ERR_OOM and leaves
    # nothing half-built behind: a second call with the same sizes tries to
    # allocate again (and fails the same way, without touching a buffer), and a
    # call with a workspace that fits then gives the result of a fresh handle.
    # A diagonal system of 20M rows: FGMRES(1000) needs 2001 n doubles = 320 GB,
    # more than the device holds; the basis V (160 GB) is allocated first.
    m = silu()
    n = 20_000_000
    d = 1.0 + (np.arange(n) % 7).astype(np.float64)
    A = synth.CSR(n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), d)
    Ad = m.DeviceCSR.from_host(A)
    P = m.setup(Ad)
    b = torch.as_tensor(synth.uniform_rhs(n, 5)).cuda()
    print(f"[errors] oom: n={n}, FGMRES(1000) workspace {(2001 * n * 8) >> 30} GiB", flush=True)
    for attempt in range(2):
        with pytest.raises(m.SchurILUError) as e:
            m.fgmres(Ad, P, b, rtol=1e-8, restart=1000, maxit=3)
        assert e.value.code == ERR_OOM, (attempt, e.value)
    m.memory_trim()
    out = m.fgmres(Ad, P, b, rtol=1e-8, restart=20, maxit=3)
    P2 = m.setup(Ad)
    ref = m.fgmres(Ad, P2, b, rtol=1e-8, restart=20, maxit=3)
    assert out["converged"] and out["iterations"] == ref["iterations"] == 1
    np.testing.assert_array_equal(out["x"].cpu().numpy(), ref["x"].cpu().numpy())
    P.close()
    P2.close()
    m.memory_trim()
