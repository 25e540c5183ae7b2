"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: permutations, interface flags, offsets, level sets and factor
sparsity patterns bit-exact; factor values, triangular solves, the RAP
product and the block-Jacobi apply within 1e-12 relative (FP64); the SCHUR
and RAP applies, whose inner GMRES divides by its own dot products (summed
in another order than the oracle's), within 1e-10; FGMRES within one
iteration of the oracle and a true relative residual <= rtol.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

ILUT_OPTS = dict(droptol=1e-3, lfil=20)


def silu():
    import paper_2303_08881_amd as m

    return m


def _case(name):
    if name == "aniso2d_64":
        A, b, part, p = synth.workload("aniso2d_64")
        return A, b, None, 1
    if name == "aniso3d_slabs":
        A = synth.aniso7(12, Nz=16)
        return A, synth.uniform_rhs(A.n, 2), synth.slab_partition(12, 4, Nz=16), 4
    if name == "random_blocks":
        A = synth.random_sparse(3001, 8, 31, band=40)
        return A, synth.uniform_rhs(A.n, 7), synth.block_partition(A.n, 3), 3
    if name == "rot9":
        A = synth.rotated9(40)
        return A, synth.uniform_rhs(A.n, 3), None, 1
    if name == "convdiff":
        A = synth.convdiff5(37, 0.05, 1.0, 30.0)
        return A, A.matvec(np.ones(A.n)), None, 1
    raise KeyError(name)


CONFIGS = [
    ("aniso2d_64", dict(method=oracle.BJ, interior_fact=oracle.ILU0)),
    ("rot9", dict(method=oracle.BJ, interior_fact=oracle.ILU0)),
    ("convdiff", dict(method=oracle.BJ, interior_fact=oracle.MILU0)),
    ("aniso3d_slabs", dict(method=oracle.BJ, interior_fact=oracle.ILU0)),
    ("aniso3d_slabs", dict(method=oracle.BJ, interior_fact=oracle.ILUT, **ILUT_OPTS)),
    ("aniso3d_slabs", dict(method=oracle.SCHUR, interior_fact=oracle.ILU0, interface_fact=oracle.ILU0,
                           inner_iters=3)),
    ("aniso3d_slabs", dict(method=oracle.SCHUR, interior_fact=oracle.ILUT, interface_fact=oracle.MILU0,
                           inner_iters=10, **ILUT_OPTS)),
    ("random_blocks", dict(method=oracle.BJ, interior_fact=oracle.ILUT, **ILUT_OPTS)),
    ("random_blocks", dict(method=oracle.SCHUR, interior_fact=oracle.ILUT, interface_fact=oracle.MILU0,
                           inner_iters=5, **ILUT_OPTS)),
    # (M)ILU(0) interiors with the rows of the local Schur complements (partial rows; with MILU(0) the dropped
    # fill of such a row goes to its diagonal), and rows of more than 12 entries in the random blocks
    ("aniso3d_slabs", dict(method=oracle.SCHUR, interior_fact=oracle.MILU0, interface_fact=oracle.MILU0,
                           inner_iters=3)),
    ("random_blocks", dict(method=oracle.SCHUR, interior_fact=oracle.ILU0, interface_fact=oracle.ILU0,
                           inner_iters=5)),
    # the multiplicative method: RAP-MILU (MILU(0) coarse factors, ILU(0) smoother) and RAP-ILU
    ("aniso3d_slabs", dict(method=oracle.RAP, interior_fact=oracle.MILU0, smooth_fact=oracle.ILU0, inner_iters=3)),
    ("random_blocks", dict(method=oracle.RAP, interior_fact=oracle.ILU0, smooth_fact=oracle.ILU0, inner_iters=5)),
]
RAP_IDX = [i for i, (_, o) in enumerate(CONFIGS) if o["method"] == oracle.RAP]


def _ids():
    out = []
    for name, o in CONFIGS:
        m = {oracle.BJ: "bj", oracle.SCHUR: "schur", oracle.RAP: "rap"}[o["method"]]
        f = {0: "ilu0", 1: "milu0", 2: "ilut"}[o["interior_fact"]]
        out.append(f"{name}-{m}-{f}")
    return out


@pytest.fixture(scope="module")
def built():
    cache = {}

    def get(idx, mode=None):
        key = (idx, mode)
        if key not in cache:
            name, o = CONFIGS[idx]
            A, b, part, p = _case(name)
            m = silu()
            mode_ = m.TRSV_BLOCK if mode == "block" else m.TRSV_LEVELS if mode == "levels" else m.TRSV_AUTO
            print(f"[parity] case {name} opts {o} trsv {mode} n={A.n}", flush=True)
            P_o = oracle.Precond(A, part, p, **o)
            Ad = m.DeviceCSR.from_host(A)
            P_g = m.setup(Ad, part, p, trsv_mode=mode_, **o)
            torch.cuda.synchronize()
            cache[key] = (A, b, part, p, o, P_o, Ad, P_g)
        return cache[key]

    return get


@pytest.mark.parametrize("idx", range(len(CONFIGS)), ids=_ids())
def test_setup_integer_outputs_bit_exact(built, idx):
    A, b, part, p, o, P_o, Ad, P_g = built(idx)
    for name in ("perm", "iperm", "iface", "offsets"):
        np.testing.assert_array_equal(P_g.export(name), P_o.export(name), err_msg=name)
    for name in ("lev_LB", "lev_UB", "lev_LS", "lev_US"):
        np.testing.assert_array_equal(P_g.export(name), P_o.export(name), err_msg=name)


@pytest.mark.parametrize("idx", range(len(CONFIGS)), ids=_ids())
def test_factors_match(built, idx):
    A, b, part, p, o, P_o, Ad, P_g = built(idx)
    for name in ("LB", "UB", "Z", "W", "LS", "US", "Coff"):
        rg, cg, vg = P_g.csr(name)
        ro, co, vo = P_o.csr(name)
        if len(ro) == 0:
            ro = np.zeros(1, np.int64)
        np.testing.assert_array_equal(rg, ro, err_msg=f"{name} row_ptr")
        np.testing.assert_array_equal(cg, co, err_msg=f"{name} col")
        scale = max(np.abs(vo).max(initial=0.0), 1e-300)
        np.testing.assert_allclose(vg, vo, rtol=1e-12, atol=1e-12 * scale, err_msg=f"{name} val")
    for name in ("DB", "DS"):
        np.testing.assert_allclose(P_g.export(name), P_o.export(name), rtol=1e-12, err_msg=name)


@pytest.mark.parametrize("mode", ["block", "levels"])
@pytest.mark.parametrize("idx", range(len(CONFIGS)), ids=_ids())
def test_apply_matches(built, idx, mode):
    A, b, part, p, o, P_o, Ad, P_g = built(idx, mode)
    r = synth.uniform_rhs(A.n, 100 + idx)
    zo = P_o.apply(r)
    zg = P_g.apply(torch.as_tensor(r).cuda()).cpu().numpy()
    # an inner GMRES (SCHUR, RAP) divides by its own dot products: 1e-10 there
    tol = 1e-12 if o["method"] == oracle.BJ else 1e-10
    np.testing.assert_allclose(zg, zo, rtol=tol, atol=tol * np.abs(zo).max())


@pytest.mark.parametrize("mode", ["block", "levels"])
@pytest.mark.parametrize("idx", RAP_IDX, ids=lambda i: _ids()[i])
def test_rap_matvec_matches(built, idx, mode):
    # R A P v with R, P unformed (Section 3.3, eq. (28)): two triangular solves and one product with A, each
    # summed in the oracle's order, so FP64 rounding differences only (block mode multiplies by 1/u_ii)
    A, b, part, p, o, P_o, Ad, P_g = built(idx, mode)
    nS = P_g.info()["nS"]
    assert nS > 0
    v = synth.uniform_rhs(nS, 300 + idx)
    out_o = P_o.rap_matvec(v)
    out_g = P_g.rap_matvec(torch.as_tensor(v).cuda()).cpu().numpy()
    np.testing.assert_allclose(out_g, out_o, rtol=1e-12, atol=1e-12 * np.abs(out_o).max())


@pytest.mark.parametrize("mode", ["block", "levels"])
@pytest.mark.parametrize("idx", range(len(CONFIGS)), ids=_ids())
def test_fgmres_matches(built, idx, mode):
    A, b, part, p, o, P_o, Ad, P_g = built(idx, mode)
    restart = 30 if A.n < 5000 else 50
    ro = oracle.fgmres(A, P_o, b, rtol=1e-8, restart=restart, maxit=600)
    rg = silu().fgmres(Ad, P_g, torch.as_tensor(b).cuda(), rtol=1e-8, restart=restart, maxit=600)
    assert ro["converged"] and rg["converged"]
    assert abs(rg["iterations"] - ro["iterations"]) <= 1, (rg["iterations"], ro["iterations"])
    xg = rg["x"].cpu().numpy()
    true_rel = np.linalg.norm(oracle.residual(A, b, xg)) / np.linalg.norm(b)
    assert true_rel <= 1e-8
    assert abs(true_rel - rg["relres"]) <= 1e-12
    np.testing.assert_allclose(xg, ro["x"], rtol=0, atol=1e-5 * np.abs(ro["x"]).max())


# Triangular factors stored in FP32, or in FP16 scaled per row, with the
# solves in FP32 and everything else in FP64.  The apply then differs from the
# FP64 oracle's by the rounding of the stored factors: unit roundoff 2^-24
# (FP32) or 2^-11 (FP16) per entry, times the growth through the solves, which
# stays below about 10 on these well-scaled factors (measured: at most 3.4e-7
# and 7.1e-4).  FGMRES, flexible in its preconditioner, still reaches the FP64
# tolerance, within two iterations of the oracle's count (measured: equal).
PREC_TOL = {"f32": 1e-5, "f16": 5e-3}


@pytest.mark.parametrize("prec", ["f32", "f16"])
@pytest.mark.parametrize("mode", ["block", "levels"])
@pytest.mark.parametrize("idx", [1, 6, 7], ids=lambda i: _ids()[i])
def test_low_precision_factors(built, idx, mode, prec):
    A, b, part, p, o, P_o, Ad, _ = built(idx)
    m = silu()
    fp = m.PREC_F32 if prec == "f32" else m.PREC_F16
    mode_ = m.TRSV_BLOCK if mode == "block" else m.TRSV_LEVELS
    print(f"[parity] low precision {prec} case {idx} trsv {mode}", flush=True)
    P_g = m.setup(Ad, part, p, trsv_mode=mode_, factor_prec=fp, **o)
    r = synth.uniform_rhs(A.n, 100 + idx)
    zo = P_o.apply(r)
    zg = P_g.apply(torch.as_tensor(r).cuda()).cpu().numpy()
    err = np.abs(zg - zo).max() / np.abs(zo).max()
    assert err <= PREC_TOL[prec], err
    assert err > 0.0  # the factors really are rounded
    restart = 30 if A.n < 5000 else 50
    ro = oracle.fgmres(A, P_o, b, rtol=1e-8, restart=restart, maxit=600)
    rg = m.fgmres(Ad, P_g, torch.as_tensor(b).cuda(), rtol=1e-8, restart=restart, maxit=600)
    assert rg["converged"] and rg["iterations"] <= ro["iterations"] + 2, (rg["iterations"], ro["iterations"])
    xg = rg["x"].cpu().numpy()
    assert np.linalg.norm(oracle.residual(A, b, xg)) / np.linalg.norm(b) <= 1e-8


def _far_coupled(n, far, width_rows):
    """Diagonally dominant matrix whose rows i >= far couple to row i - far (and back): with natural ordering the
    first `far` rows form one level, and the coupled rows depend on positions `far` back."""
    rows, cols, vals = [], [], []
    for i in range(n):
        ent = {i: 4.0}
        if i % width_rows and i - 1 >= 0:
            ent[i - 1] = -1.0
        if i % width_rows != width_rows - 1 and i + 1 < n:
            ent[i + 1] = -1.0
        if i >= far:
            ent[i - far] = -0.5
        if i + far < n:
            ent[i + far] = -0.5
        for c in sorted(ent):
            rows.append(i)
            cols.append(c)
            vals.append(ent[c])
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, np.array(rows) + 1, 1)
    return synth.CSR(n, np.cumsum(rp), np.array(cols, np.int32), np.array(vals))


# The block-local solve has a check-free variant (no slow row, every level
# within the workgroup) and a general one.  These matrices take the general
# one: a level of 2000 independent rows (wider than a 512-thread workgroup),
# and dependencies about 9600 positions back (older than the 8192-position
# window).
@pytest.mark.parametrize("kind", ["wide_level", "old_dependency"])
def test_block_solve_general_path(kind):
    m = silu()
    A = _far_coupled(4000, 2000, 1) if kind == "wide_level" else _far_coupled(12000, 9080, 100)
    print(f"[parity] block solve general path {kind} n={A.n}", flush=True)
    P_o = oracle.Precond(A, None, 1, method=oracle.BJ, interior_fact=oracle.ILU0)
    P_g = m.setup(m.DeviceCSR.from_host(A), None, 1, method=m.BJ, interior_fact=m.ILU0, trsv_mode=m.TRSV_BLOCK)
    r = synth.uniform_rhs(A.n, 11)
    zo = P_o.apply(r)
    zg = P_g.apply(torch.as_tensor(r).cuda()).cpu().numpy()
    np.testing.assert_allclose(zg, zo, rtol=1e-12, atol=1e-12 * np.abs(zo).max())


def test_spmv_bit_exact():
    A = synth.random_sparse(5003, 11, 41, band=60)
    x = synth.uniform_rhs(A.n, 9)
    m = silu()
    Ad = m.DeviceCSR.from_host(A)
    y = m.spmv(Ad, torch.as_tensor(x).cuda()).cpu().numpy()
    np.testing.assert_array_equal(y, oracle.spmv(A, x))


def test_errors_are_reported():
    m = silu()
    A = synth.aniso5(6)
    bad_val = A.val.copy()
    bad_col = A.col.copy()
    bad_col[1], bad_col[2] = bad_col[2], bad_col[1]
    Ad = m.DeviceCSR(A.n, torch.as_tensor(A.row_ptr).cuda(), torch.as_tensor(bad_col).cuda(),
                     torch.as_tensor(bad_val).cuda())
    with pytest.raises(m.SchurILUError) as e:
        m.setup(Ad)
    assert e.value.code == -2
    Z = synth.CSR.from_dense(np.array([[0.0, 1.0], [1.0, 1.0]]))
    with pytest.raises(m.SchurILUError) as e:
        m.setup(m.DeviceCSR.from_host(Z))
    assert e.value.code == -3
    P = m.setup(m.DeviceCSR.from_host(Z), pivot_mode=m.PIVOT_PERTURB, pivot_tol=1e-3)
    Po = oracle.Precond(Z, None, 1, pivot_mode=oracle.PIVOT_PERTURB, pivot_tol=1e-3)
    r = np.array([1.0, 2.0])
    np.testing.assert_allclose(P.apply(torch.as_tensor(r).cuda()).cpu().numpy(), Po.apply(r), rtol=1e-14)
    with pytest.raises(m.SchurILUError) as e:
        m.setup(m.DeviceCSR.from_host(synth.aniso5(6)), factor_prec=3)
    assert e.value.code == -1


def test_reduced_system_components(built):
    # 12 x 12 x 16 grid, 4 z-slabs: the interface rows of each inner slab are two planes that L_S + U_S never
    # couple, those of each end slab one plane, so the block-local L_S and U_S solves run on 6 workgroups
    # (connected components found on the device; the count is the connected_components of the pattern)
    idx = [i for i, (nm, o) in enumerate(CONFIGS) if nm == "aniso3d_slabs" and o["method"] == oracle.SCHUR][0]
    A, b, part, p, o, P_o, Ad, P_g = built(idx, "block")
    assert P_g.export("schedule")[19] == 6
    # block Jacobi splits each whole-block factor the same way: its interface part has the same 6 components
    idx_bj = [i for i, (nm, o) in enumerate(CONFIGS) if nm == "aniso3d_slabs" and o["method"] == oracle.BJ][0]
    assert built(idx_bj, "block")[7].export("schedule")[19] == 6
    # one subdomain: no interface rows, no reduced-system solve
    idx_one = [i for i, (nm, o) in enumerate(CONFIGS) if nm == "aniso2d_64"][0]
    assert built(idx_one, "block")[7].export("schedule")[19] == 0


def test_components_of_long_chains():
    # 512 x 64 grid, 4 bands of 16 lines (x fastest): the interface rows are the lines next to a neighbouring
    # band, 6 lines of 512 rows, each a chain in L_S + U_S (the union-find sees paths 512 long); the apply still
    # matches the oracle
    m = silu()
    A = synth.aniso5(512, 0.1, Ny=64)
    part = synth.block_partition(A.n, 4)
    o = dict(method=oracle.SCHUR, interior_fact=oracle.ILU0, interface_fact=oracle.ILU0, inner_iters=3)
    P_o = oracle.Precond(A, part, 4, **o)
    P_g = m.setup(m.DeviceCSR.from_host(A), part, 4, trsv_mode=m.TRSV_BLOCK, **o)
    assert P_g.info()["nS"] == 6 * 512
    assert P_g.export("schedule")[19] == 6
    r = synth.uniform_rhs(A.n, 9)
    zo = P_o.apply(r)
    zg = P_g.apply(torch.as_tensor(r).cuda()).cpu().numpy()
    np.testing.assert_allclose(zg, zo, rtol=1e-10, atol=1e-10 * np.abs(zo).max())


@pytest.mark.parametrize("kind", ["one_row", "all_interface", "empty_part"])
def test_edge_partitions(kind):
    m = silu()
    if kind == "one_row":
        A = synth.CSR.from_dense(np.array([[3.0]]))
        part, p = None, 1
    elif kind == "all_interface":
        A = synth.aniso5(5)
        part, p = np.arange(A.n, dtype=np.int32), A.n
    else:
        A = synth.aniso5(8)
        part, p = (synth.block_partition(A.n, 3) * 2).astype(np.int32), 6  # parts 1, 3, 5 empty
    for o in (dict(method=oracle.BJ), dict(method=oracle.SCHUR, interface_fact=oracle.MILU0, inner_iters=4)):
        Po = oracle.Precond(A, part, p, **o)
        Pg = m.setup(m.DeviceCSR.from_host(A), part, p, **o)
        np.testing.assert_array_equal(Pg.export("perm"), Po.export("perm"))
        np.testing.assert_array_equal(Pg.export("offsets"), Po.export("offsets"))
        r = synth.uniform_rhs(A.n, 4)
        zo = Po.apply(r)
        np.testing.assert_allclose(Pg.apply(torch.as_tensor(r).cuda()).cpu().numpy(), zo, rtol=1e-10, atol=1e-14)
        # the same degenerate shapes with factors stored in FP32 and FP16
        for fp, tol in ((m.PREC_F32, PREC_TOL["f32"]), (m.PREC_F16, PREC_TOL["f16"])):
            Pl = m.setup(m.DeviceCSR.from_host(A), part, p, factor_prec=fp, **o)
            zl = Pl.apply(torch.as_tensor(r).cuda()).cpu().numpy()
            assert np.abs(zl - zo).max() <= tol * np.abs(zo).max(), (fp, np.abs(zl - zo).max())


# ---- the 128^3 slab workload at full size, as the benchmark runs it ----
SLAB_OPTS = dict(method=oracle.SCHUR, interior_fact=oracle.ILUT, interface_fact=oracle.MILU0, droptol=1e-3, lfil=20,
                 inner_iters=10)


@pytest.fixture(scope="module")
def slab_full():
    A, b, part, p = synth.workload("aniso3d_128_slab16")
    print(f"[parity] full slab workload n={A.n} nnz={A.nnz}", flush=True)
    P_o = oracle.Precond(A, part, p, **SLAB_OPTS)
    m = silu()
    Ad = m.DeviceCSR.from_host(A)
    P_g = m.setup(Ad, torch.as_tensor(part).cuda(), p, **SLAB_OPTS)
    torch.cuda.synchronize()
    return A, b, part, p, P_o, Ad, P_g


@pytest.mark.slow
def test_full_slab_setup_matches(slab_full):
    """Every integer output bit-exact and every factor within 1e-12 at n = 2,097,152, 16 subdomains."""
    A, b, part, p, P_o, Ad, P_g = slab_full
    for name in ("perm", "iperm", "iface", "offsets", "lev_LB", "lev_UB", "lev_LS", "lev_US"):
        np.testing.assert_array_equal(P_g.export(name), P_o.export(name), err_msg=name)
    for name in ("LB", "UB", "Z", "W", "LS", "US", "Coff"):
        rg, cg, vg = P_g.csr(name)
        ro, co, vo = P_o.csr(name)
        np.testing.assert_array_equal(rg, ro, err_msg=f"{name} row_ptr")
        np.testing.assert_array_equal(cg, co, err_msg=f"{name} col")
        np.testing.assert_allclose(vg, vo, rtol=1e-12, atol=1e-12 * np.abs(vo).max(initial=1.0), err_msg=name)
    for name in ("DB", "DS"):
        np.testing.assert_allclose(P_g.export(name), P_o.export(name), rtol=1e-12, err_msg=name)
    sched = P_g.export("schedule")
    assert all(sched[4 * k] == 1 for k in range(4)), sched  # the benchmark's block-local solves
    # one workgroup per interface plane: 2 for each of the 14 inner slabs, 1 for each end slab
    assert sched[19] == 30, sched
    # the interior solves split over four workgroups per subdomain (98,304 interior rows each)
    assert (sched[20], sched[21]) == (4, 4), sched


@pytest.mark.slow
def test_full_slab_apply_and_fgmres(slab_full):
    A, b, part, p, P_o, Ad, P_g = slab_full
    r = synth.uniform_rhs(A.n, 11)
    zo = P_o.apply(r)
    zg = P_g.apply(torch.as_tensor(r).cuda()).cpu().numpy()
    np.testing.assert_allclose(zg, zo, rtol=1e-10, atol=1e-10 * np.abs(zo).max())
    ro = oracle.fgmres(A, P_o, b, rtol=1e-8, restart=50, maxit=600)
    rg = silu().fgmres(Ad, P_g, torch.as_tensor(b).cuda(), rtol=1e-8, restart=50, maxit=600)
    assert ro["converged"] and rg["converged"]
    assert abs(rg["iterations"] - ro["iterations"]) <= 1, (rg["iterations"], ro["iterations"])
    xg = rg["x"].cpu().numpy()
    assert np.linalg.norm(oracle.residual(A, b, xg)) / np.linalg.norm(b) <= 1e-8


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_full_slab_low_precision(slab_full, prec):
    """FP32 / FP16 factor storage at n = 2,097,152: apply within the bound of test_low_precision_factors, and FGMRES
    to the same tolerance within two iterations of the FP64 path (itself within one of the oracle)."""
    A, b, part, p, P_o, Ad, P_64 = slab_full
    m = silu()
    fp = m.PREC_F32 if prec == "f32" else m.PREC_F16
    print(f"[parity] full slab, factors in {prec}", flush=True)
    P_g = m.setup(Ad, torch.as_tensor(part).cuda(), p, factor_prec=fp, **SLAB_OPTS)
    r = synth.uniform_rhs(A.n, 11)
    zo = P_o.apply(r)
    zg = P_g.apply(torch.as_tensor(r).cuda()).cpu().numpy()
    err = np.abs(zg - zo).max() / np.abs(zo).max()
    assert 0.0 < err <= PREC_TOL[prec], err
    bd = torch.as_tensor(b).cuda()
    r64 = m.fgmres(Ad, P_64, bd, rtol=1e-8, restart=50, maxit=600)
    rg = m.fgmres(Ad, P_g, bd, rtol=1e-8, restart=50, maxit=600)
    assert rg["converged"] and rg["iterations"] <= r64["iterations"] + 2, (rg["iterations"], r64["iterations"])
    xg = rg["x"].cpu().numpy()
    assert np.linalg.norm(oracle.residual(A, b, xg)) / np.linalg.norm(b) <= 1e-8


def test_runs_are_deterministic():
    """Two setups of the same system give bitwise identical factors; two applies identical vectors."""
    m = silu()
    A = synth.aniso7(12, Nz=16)
    part = synth.slab_partition(12, 4, Nz=16)
    opts = dict(method=oracle.SCHUR, interior_fact=oracle.ILUT, interface_fact=oracle.MILU0, inner_iters=5,
                **ILUT_OPTS)
    Ad = m.DeviceCSR.from_host(A)
    P1 = m.setup(Ad, part, 4, **opts)
    P2 = m.setup(Ad, part, 4, **opts)
    for name in ("LB", "UB", "Z", "W", "LS", "US"):
        for a1, a2 in zip(P1.csr(name), P2.csr(name)):
            assert np.array_equal(a1, a2), name
    r = torch.as_tensor(synth.uniform_rhs(A.n, 3)).cuda()
    z1 = P1.apply(r).cpu().numpy()
    z2 = P1.apply(r).cpu().numpy()
    z3 = P2.apply(r).cpu().numpy()
    assert np.array_equal(z1.view(np.uint64), z2.view(np.uint64))
    assert np.array_equal(z1.view(np.uint64), z3.view(np.uint64))


def test_reused_device_blocks_give_identical_results():
    """Setups that run on device blocks released by an earlier setup (the library's block cache), and again
    after the cache was emptied, give bitwise identical preconditioners and FGMRES solutions."""
    m = silu()
    A = synth.aniso7(12, Nz=16)
    part = synth.slab_partition(12, 4, Nz=16)
    b = torch.as_tensor(synth.uniform_rhs(A.n, 4)).cuda()
    r = torch.as_tensor(synth.uniform_rhs(A.n, 6)).cuda()
    opts = dict(method=oracle.SCHUR, interior_fact=oracle.ILUT, interface_fact=oracle.MILU0, inner_iters=5,
                **ILUT_OPTS)
    Ad = m.DeviceCSR.from_host(A)
    runs = []
    for k in range(3):
        if k == 2:
            m.memory_trim()
        P = m.setup(Ad, part, 4, **opts)
        z = P.apply(r).cpu().numpy()
        out = m.fgmres(Ad, P, b, rtol=1e-8, restart=20, maxit=200)
        runs.append((z.view(np.uint64).copy(), out["x"].cpu().numpy().view(np.uint64).copy(), out["iterations"]))
        P.close()
    for z, x, its in runs[1:]:
        assert np.array_equal(z, runs[0][0])
        assert np.array_equal(x, runs[0][1])
        assert its == runs[0][2]
