"""fgmres_solve_noalloc (the Krylov workspace in a fixed device array) against fgmres_solve, through the C ABI.

Bar: the same kernels on the same data, so x bit-identical and the same iteration count and residual, on two
calls in a row, the second on a smaller system (the array keeps the first call's contents); a workspace larger
than the array is refused with ILU_ERR_CAPACITY before any device work.
"""
import ctypes as C

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def silu():
    import paper_2303_08881_amd as m

    return m


def _noalloc(m, Ad, P, b, x, rtol, restart, maxit):
    lib = m.lib()
    fn = lib.fgmres_solve_noalloc
    vp, i32, d = C.c_void_p, C.c_int32, C.c_double
    fn.argtypes = [vp, vp, vp, vp, d, i32, i32, vp, vp, vp]
    res = m.binding._Res()
    rc = fn(Ad.ref, P._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), rtol, restart, maxit,
            C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(res), None)
    return rc, res


@pytest.mark.parametrize("case", ["schur_slabs", "bj_aniso2d"])
def test_noalloc_matches_fgmres_twice(case):
    m = silu()
    # first call on the larger system, second on a smaller one
    if case == "schur_slabs":
        systems = [(synth.aniso7(24, Nz=32), synth.slab_partition(24, 4, Nz=32), 4),
                   (synth.aniso7(12, Nz=16), synth.slab_partition(12, 4, Nz=16), 4)]
        opts = dict(method=m.SCHUR, interior_fact=m.ILUT, interface_fact=m.MILU0, droptol=1e-3, lfil=20,
                    inner_iters=5)
    else:
        systems = [(synth.aniso5(128, 0.01), None, 1), (synth.aniso5(40, 0.01), None, 1)]
        opts = dict(method=m.BJ, interior_fact=m.ILU0)
    for k, (A, part, p) in enumerate(systems):
        print(f"[noalloc] {case} call {k}: n={A.n}", flush=True)
        Ad = m.DeviceCSR.from_host(A)
        pd = torch.as_tensor(part).cuda() if part is not None else None
        P = m.setup(Ad, pd, p, **opts)
        b = torch.as_tensor(synth.uniform_rhs(A.n, 21 + k)).cuda()
        ref = m.fgmres(Ad, P, b, rtol=1e-8, restart=30, maxit=800)
        x = torch.zeros_like(b)
        rc, res = _noalloc(m, Ad, P, b, x, 1e-8, 30, 800)
        assert rc == 0, m.lib().ilu_last_error().decode()
        assert res.iterations == ref["iterations"] and res.converged == 1
        assert res.final_relres == ref["relres"]
        np.testing.assert_array_equal(x.cpu().numpy(), ref["x"].cpu().numpy())
        P.close()


def test_noalloc_refuses_workspace_beyond_the_array():
    m = silu()
    A = synth.aniso5(300, 0.01)  # n = 90,000: (2 * 50 + 2) n doubles > 64 MiB
    Ad = m.DeviceCSR.from_host(A)
    P = m.setup(Ad, None, 1)
    b = torch.ones(A.n, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    rc, _ = _noalloc(m, Ad, P, b, x, 1e-8, 50, 10)
    assert rc == -7 and "workspace" in m.lib().ilu_last_error().decode()
    assert float(x.abs().max()) == 0.0  # nothing ran
    rc, res = _noalloc(m, Ad, P, b, x, 1e-8, 40, 2000)  # 82 n doubles fit
    assert rc == 0 and res.converged == 1
    P.close()
