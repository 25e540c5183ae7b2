"""The mixed-precision workload at its full size: 2D rotated anisotropic 9-point diffusion on a 2048 x 2048 grid
(n = 4,194,304, nnz = 37,724,164, eps 1e-3, theta pi/6), one block, ILU(0), FGMRES(30) to rtol 1e-10.

The one block of 4.19M rows has 6,142 levels per factor, 683 rows each on average.  The default solve splits
it into 16 bands of 128 grid lines, one workgroup each, each band walking its own 2,300 levels and taking the
last line of the band before it through device memory (one workgroup of 1024 threads for the whole block, and
the level-scheduled solve over the whole GPU with a cross-CU wait per level, are checked too).  Bars: level of every row bit-exact, factors within 1e-12, the FP64 apply within
1e-12 of the oracle's in both solve modes; with FP32 / FP16 factor storage the apply error
against the FP64 oracle is printed and bounded, and FGMRES (FP64 Krylov, SpMV and convergence test) still
reaches the true relative residual 1e-10.  The oracle's full FGMRES at this size takes minutes, so iteration
counts are compared between the GPU precisions only.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

OPTS = dict(method=oracle.BJ, interior_fact=oracle.ILU0)
# measured apply errors of the stored-factor rounding, with margin (FP32: unit roundoff 2^-24 times the growth
# through 6,142 levels of a non-M-matrix; FP16 with row scaling: 2^-11 times that growth)
PREC_TOL = {"f32": 1e-3, "f16": 0.5}


@pytest.fixture(scope="module")
def rot9():
    import paper_2303_08881_amd as m

    A, b, part, p = synth.workload("rot9_2048")
    print(f"[rot9] n={A.n} nnz={A.nnz}", flush=True)
    P_o = oracle.Precond(A, None, 1, **OPTS)
    print("[rot9] oracle setup done", flush=True)
    Ad = m.DeviceCSR.from_host(A)
    P_g = m.setup(Ad, None, 1, **OPTS)
    torch.cuda.synchronize()
    print("[rot9] device setup done", flush=True)
    return m, A, b, P_o, Ad, P_g


def test_rot9_setup_matches(rot9):
    m, A, b, P_o, Ad, P_g = rot9
    assert A.n == 4194304 and A.nnz == 37724164
    for name in ("perm", "lev_LB", "lev_UB"):
        np.testing.assert_array_equal(P_g.export(name), P_o.export(name), err_msg=name)
    assert int(P_g.export("lev_LB").max()) + 1 == 6142
    for name in ("LB", "UB"):
        rg, cg, vg = P_g.csr(name)
        ro, co, vo = P_o.csr(name)
        np.testing.assert_array_equal(rg, ro, err_msg=f"{name} row_ptr")
        np.testing.assert_array_equal(cg, co, err_msg=f"{name} col")
        np.testing.assert_allclose(vg, vo, rtol=1e-12, atol=1e-12 * np.abs(vo).max(), err_msg=name)
    np.testing.assert_allclose(P_g.export("DB"), P_o.export("DB"), rtol=1e-12)
    sched = P_g.export("schedule")
    # block-local, the block split into 16 bands of 128 grid lines (levels of at most 128 rows per band)
    assert sched[0] == 1 and sched[4] == 1 and (sched[20], sched[21]) == (16, 16), sched
    assert sched[3] <= 384 and sched[7] <= 384, sched


def test_rot9_one_workgroup_identical(rot9):
    # the whole block on one workgroup of 1024 threads (the widest level has 1024 rows): the same arithmetic
    # for every row, so the same apply to the bit
    m, A, b, P_o, Ad, P_g = rot9
    P_1 = m.setup(Ad, None, 1, block_split=1, **OPTS)
    sched = P_1.export("schedule")
    assert sched[3] == 1024 and sched[7] == 1024 and (sched[20], sched[21]) == (1, 1), sched
    r = torch.as_tensor(synth.uniform_rhs(A.n, 17)).cuda()
    np.testing.assert_array_equal(P_1.apply(r).cpu().numpy(), P_g.apply(r).cpu().numpy())
    P_1.close()


def test_rot9_apply_fp64(rot9):
    m, A, b, P_o, Ad, P_g = rot9
    r = synth.uniform_rhs(A.n, 13)
    zo = P_o.apply(r)
    zg = P_g.apply(torch.as_tensor(r).cuda()).cpu().numpy()
    np.testing.assert_allclose(zg, zo, rtol=1e-12, atol=1e-12 * np.abs(zo).max())


def test_rot9_level_scheduled_apply(rot9):
    # every level spread over the whole GPU: the oracle's operations in its order, so the apply is bit-exact
    m, A, b, P_o, Ad, P_g = rot9
    P_l = m.setup(Ad, None, 1, trsv_mode=m.TRSV_LEVELS, **OPTS)
    sched = P_l.export("schedule")
    assert sched[0] == 0 and sched[4] == 0, sched
    r = synth.uniform_rhs(A.n, 13)
    zo = P_o.apply(r)
    zg = P_l.apply(torch.as_tensor(r).cuda()).cpu().numpy()
    np.testing.assert_array_equal(zg, zo)
    P_l.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_rot9_precisions(rot9, prec):
    m, A, b, P_o, Ad, P_64 = rot9
    fp = {"f64": m.PREC_F64, "f32": m.PREC_F32, "f16": m.PREC_F16}[prec]
    P_g = P_64 if prec == "f64" else m.setup(Ad, None, 1, factor_prec=fp, **OPTS)
    r = synth.uniform_rhs(A.n, 13)
    zo = P_o.apply(r)
    zg = P_g.apply(torch.as_tensor(r).cuda()).cpu().numpy()
    err = float(np.abs(zg - zo).max() / np.abs(zo).max())
    print(f"[rot9] {prec}: apply error vs FP64 oracle {err:.3e}", flush=True)
    if prec != "f64":
        assert 0.0 < err <= PREC_TOL[prec], err
    out = m.fgmres(Ad, P_g, torch.as_tensor(b).cuda(), rtol=1e-10, restart=30, maxit=3000)
    xg = out["x"].cpu().numpy()
    true = np.linalg.norm(oracle.residual(A, b, xg)) / np.linalg.norm(b)
    print(f"[rot9] {prec}: {out['iterations']} iterations, solve {out['solve_ms']:.1f} ms, relres {true:.2e}",
          flush=True)
    assert out["converged"] and true <= 1e-10, (out["iterations"], true)
