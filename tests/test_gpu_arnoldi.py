"""The Arnoldi orthogonalisation as one launch per step, against one launch per pass.

Both routes run the modified Gram-Schmidt of a step in the same order (pass i: h_i = <w, v_i>, then
w -= h_i v_i; Section 4.1's GMRES and the reduced-system GMRES of Section 3.2) and differ only in how the
partial sums of each dot product are grouped (per workgroup of each launch's grid).  Bars: applies of the
two routes (k inner GMRES steps on the reduced system) within 1e-12 relative of each other and within
1e-10 of the oracle; FGMRES of both within one iteration of the oracle, to a true relative residual
<= rtol; the one-launch route bit-identical over repeated runs; the outer loop takes one launch per
Arnoldi step on the one-launch route and one per pass on the other.  The operator has 76,800 rows:
the one-launch grid has 10 workgroups of 4,096 element pairs, the last one partly filled, and the
reduced system (9,600 rows) 2 workgroups; an odd length takes the per-pass route by itself.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

K_MGS = 6  # ilu_kernel_stats class of the outer orthogonalisation
OPTS = {
    "schur": dict(method=oracle.SCHUR, interior_fact=oracle.ILUT, interface_fact=oracle.MILU0, inner_iters=10,
                  droptol=1e-3, lfil=20),
    "rap": dict(method=oracle.RAP, interior_fact=oracle.MILU0, smooth_fact=oracle.ILU0, inner_iters=3),
}


def silu():
    import paper_2303_08881_amd as m

    return m


@pytest.fixture(scope="module")
def system():
    A = synth.aniso7(40, Nz=48)
    part = synth.slab_partition(40, 4, Nz=48)
    return A, part, synth.uniform_rhs(A.n, 21)


def _passes(steps, restart):
    return sum(j % restart + 1 for j in range(steps))


def _mgs_launches(m, fn):
    lib = m.lib()
    ms, cnt = C.c_double(), C.c_int64()
    lib.ilu_kernel_stats(K_MGS, None, None, None, 1)
    lib.ilu_kernel_timing(1 << K_MGS)
    try:
        out = fn()
        torch.cuda.synchronize()
    finally:
        lib.ilu_kernel_timing(0)
    lib.ilu_kernel_stats(K_MGS, C.byref(ms), C.byref(cnt), None, 1)
    return out, cnt.value


@pytest.mark.parametrize("method", ["schur", "rap"])
def test_one_launch_matches_per_pass_and_oracle(system, method):
    A, part, b = system
    m = silu()
    o = OPTS[method]
    print(f"[arnoldi] {method} n={A.n}", flush=True)
    P_o = oracle.Precond(A, part, 4, **o)
    Ad = m.DeviceCSR.from_host(A)
    P_one = m.setup(Ad, part, 4, **o)
    P_pass = m.setup(Ad, part, 4, arnoldi_mode=m.ARNOLDI_PER_PASS, **o)
    r = synth.uniform_rhs(A.n, 22)
    rd = torch.as_tensor(r).cuda()
    z_one = P_one.apply(rd).cpu().numpy()
    z_pass = P_pass.apply(rd).cpu().numpy()
    z_o = P_o.apply(r)
    np.testing.assert_allclose(z_one, z_pass, rtol=1e-12, atol=1e-12 * np.abs(z_pass).max())
    np.testing.assert_allclose(z_one, z_o, rtol=1e-10, atol=1e-10 * np.abs(z_o).max())
    # repeated applies of the one-launch route: the same bits
    assert np.array_equal(P_one.apply(rd).cpu().numpy().view(np.uint64), z_one.view(np.uint64))

    bd = torch.as_tensor(b).cuda()
    ro = oracle.fgmres(A, P_o, b, rtol=1e-8, restart=50, maxit=600)
    r_one, n_one = _mgs_launches(m, lambda: m.fgmres(Ad, P_one, bd, rtol=1e-8, restart=50, maxit=600))
    r_pass, n_pass = _mgs_launches(m, lambda: m.fgmres(Ad, P_pass, bd, rtol=1e-8, restart=50, maxit=600))
    assert ro["converged"] and r_one["converged"] and r_pass["converged"]
    for r_g in (r_one, r_pass):
        assert abs(r_g["iterations"] - ro["iterations"]) <= 1, (r_g["iterations"], ro["iterations"])
        xg = r_g["x"].cpu().numpy()
        assert np.linalg.norm(oracle.residual(A, b, xg)) / np.linalg.norm(b) <= 1e-8
        np.testing.assert_allclose(xg, ro["x"], rtol=0, atol=1e-5 * np.abs(ro["x"]).max())
    # one launch per Arnoldi step against one per pass (j + 1 passes at step j of a cycle); the solve may
    # have enqueued one step past the converged one (its results are read back one step late)
    assert n_one in (r_one["iterations"], r_one["iterations"] + 1), (n_one, r_one["iterations"])
    its = r_pass["iterations"]
    assert n_pass in (_passes(its, 50), _passes(its + 1, 50)), (n_pass, its)
    P_one.close()
    P_pass.close()


def test_odd_length_takes_the_per_pass_route():
    # 2D anisotropic operator on a 45 x 45 grid: n = 2025 is odd, so the one-launch kernel (element pairs)
    # cannot take the vectors and each pass runs as its own launch; results match the oracle as usual
    m = silu()
    A = synth.aniso5(45, 1e-2)
    b = synth.uniform_rhs(A.n, 23)
    Ad = m.DeviceCSR.from_host(A)
    P = m.setup(Ad)
    P_o = oracle.Precond(A, None, 1)
    ro = oracle.fgmres(A, P_o, b, rtol=1e-8, restart=30, maxit=600)
    rg, n = _mgs_launches(m, lambda: m.fgmres(Ad, P, torch.as_tensor(b).cuda(), rtol=1e-8, restart=30,
                                              maxit=600))
    assert rg["converged"] and abs(rg["iterations"] - ro["iterations"]) <= 1
    its = rg["iterations"]
    assert n in (_passes(its, 30), _passes(its + 1, 30)), (n, its)
    P.close()
