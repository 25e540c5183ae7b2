"""The block-local L_B and U_B solves with each subdomain split over several workgroups, against the same
solves with one workgroup per subdomain and against the oracle.

A split solve does the arithmetic of every row exactly as the unsplit one (the same entries in the same lanes,
the same combination of the lanes' sums), so applies are bit-identical for any number of parts, and so are
whole FGMRES solves.  Each part takes the values it needs from earlier parts through device memory, and the
reader of each exchange slot resets it for the next solve, so every case applies several times in a row.
Where a split does not apply (too many imports for one level, a part too long) the setup keeps the solve
unsplit; the schedule export says which, and the results agree either way.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

ILUT = dict(droptol=1e-3, lfil=20)
SCHUR_ILUT = dict(method=oracle.SCHUR, interior_fact=oracle.ILUT, interface_fact=oracle.MILU0, inner_iters=10,
                  **ILUT)


def silu():
    import paper_2303_08881_amd as m

    return m


def _case(name):
    if name == "slabs":  # 12 x 12 x 16, 4 z-slabs
        A = synth.aniso7(12, Nz=16)
        return A, synth.slab_partition(12, 4, Nz=16), 4
    if name == "aniso2d":  # 64^2, one block
        A, b, part, p = synth.workload("aniso2d_64")
        return A, None, 1
    if name == "rot9":  # 40^2 rotated 9-point, one block
        return synth.rotated9(40), None, 1
    if name == "random":
        A = synth.random_sparse(3001, 8, 31, band=40)
        return A, synth.block_partition(A.n, 3), 3
    raise KeyError(name)


# (workload, options, parts per subdomain); with 3 or 4 parts a slab's part is less than two planes, and some
# rows are read by two later parts (one import each)
CASES = [
    ("slabs", SCHUR_ILUT, 2),
    ("slabs", SCHUR_ILUT, 3),
    ("slabs", SCHUR_ILUT, 4),
    ("slabs", dict(method=oracle.BJ, interior_fact=oracle.ILU0), 2),
    ("slabs", dict(method=oracle.RAP, interior_fact=oracle.MILU0, smooth_fact=oracle.ILU0, inner_iters=3), 2),
    ("aniso2d", dict(method=oracle.BJ, interior_fact=oracle.ILU0), 2),
    ("aniso2d", dict(method=oracle.BJ, interior_fact=oracle.ILU0), 8),
    ("rot9", dict(method=oracle.BJ, interior_fact=oracle.ILU0), 4),
    ("random", dict(method=oracle.BJ, interior_fact=oracle.ILUT, **ILUT), 2),
]
IWIN = 2048  # imports an LDS ring of a part holds


def _ids():
    return [f"{n}-{ {0: 'bj', 1: 'schur', 2: 'rap'}[o['method']] }-k{k}" for n, o, k in CASES]


def split_applies(rp, ci, lev, bs, nparts, k, backward):
    """Whether a k-way split of a block-local solve applies, from the oracle's factor and levels: the parts
    are k equal ranges of each block (counted from its end for a backward solve); every row that a part
    needs from another part lies in an earlier part (one import per row and importing part); no part spans
    more than 4096 levels; no level of a part needs more than 64 imports; and each import is still in the
    part's ring of the last IWIN imports (in the order of the level that first needs them) when a row of
    level l reads it, with the imports of level l + 1 already going in."""
    n = len(rp) - 1
    nlev = int(lev.max()) + 1
    blk = np.searchsorted(bs[:nparts + 1], np.arange(n), side="right") - 1
    b0, ln = bs[blk], bs[blk + 1] - bs[blk]
    kk = ((np.arange(n) - b0) * k) // ln
    prt = blk * k + (k - 1 - kk if backward else kk)
    for p_ in range(nparts * k):
        lv = lev[prt == p_]
        if lv.size and lv.max() - lv.min() + 1 > 4096:
            return False
    rows = np.repeat(np.arange(n), np.diff(rp))
    cols = ci.astype(np.int64)
    rows, cols = rows[cols < n], cols[cols < n]
    cross = prt[cols] != prt[rows]
    r, c = rows[cross], cols[cross]
    need = {}
    for cc, rr in zip(c.tolist(), r.tolist()):
        if prt[cc] >= prt[rr]:
            return False
        key = prt[rr] * nlev + lev[rr]
        imp = (cc, prt[rr])
        need[imp] = min(need.get(imp, key), key)
    order = sorted(need, key=lambda x: (need[x], x[0]))
    gi = {x: i for i, x in enumerate(order)}
    cnt = np.bincount([need[x] for x in order], minlength=nparts * k * nlev)
    if cnt.max(initial=0) > 64:
        return False
    ilp = np.concatenate([[0], np.cumsum(cnt)])
    return all(lev[rr] > 0 and gi[(cc, prt[rr])] >= ilp[prt[rr] * nlev + lev[rr] + (2 if lev[rr] + 1 < nlev else 1)]
               - IWIN for cc, rr in zip(c.tolist(), r.tolist()))


def _setup(m, A, part, p, opts, k, **kw):
    pd = None if part is None else torch.as_tensor(part).cuda()
    return m.setup(m.DeviceCSR.from_host(A), pd, p, trsv_mode=m.TRSV_BLOCK, block_split=k, **opts, **kw)


@pytest.mark.parametrize("case", range(len(CASES)), ids=_ids())
def test_split_apply_identical(case):
    name, opts, k = CASES[case]
    m = silu()
    A, part, p = _case(name)
    print(f"[split] {name} {opts['method']} k={k}", flush=True)
    Po = oracle.Precond(A, part, p, **opts)
    off = Po.export("offsets")
    want = [k if split_applies(*Po.csr(f)[:2], Po.export(lv), off, p, k, bw) else 1
            for f, lv, bw in (("LB", "lev_LB", False), ("UB", "lev_UB", True))]
    P1 = _setup(m, A, part, p, opts, 1)
    Pk = _setup(m, A, part, p, opts, k)
    s1, sk = P1.export("schedule"), Pk.export("schedule")
    assert (s1[20], s1[21]) == (1, 1), s1
    assert [sk[20], sk[21]] == want, (sk, want)
    r = torch.as_tensor(synth.uniform_rhs(A.n, 13)).cuda()
    z1 = P1.apply(r).cpu().numpy()
    for rep in range(3):
        np.testing.assert_array_equal(Pk.apply(r).cpu().numpy(), z1, err_msg=f"apply {rep}")
    zo = Po.apply(r.cpu().numpy())
    tol = 1e-12 if opts["method"] == oracle.BJ else 1e-10
    np.testing.assert_allclose(z1, zo, rtol=tol, atol=tol * np.abs(zo).max())


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_split_low_precision_identical(prec):
    m = silu()
    A, part, p = _case("slabs")
    fp = {"f32": m.PREC_F32, "f16": m.PREC_F16}[prec]
    P1 = _setup(m, A, part, p, SCHUR_ILUT, 1, factor_prec=fp)
    P2 = _setup(m, A, part, p, SCHUR_ILUT, 2, factor_prec=fp)
    assert P2.export("schedule")[20] == 2
    r = torch.as_tensor(synth.uniform_rhs(A.n, 14)).cuda()
    z1 = P1.apply(r).cpu().numpy()
    for _ in range(2):
        np.testing.assert_array_equal(P2.apply(r).cpu().numpy(), z1)


def test_split_fgmres_identical():
    m = silu()
    A, part, p = _case("slabs")
    b = torch.as_tensor(synth.uniform_rhs(A.n, 2)).cuda()
    out = []
    for k in (1, 2, 4):
        P = _setup(m, A, part, p, SCHUR_ILUT, k)
        Ad = m.DeviceCSR.from_host(A)
        out.append(m.fgmres(Ad, P, b, rtol=1e-10, restart=30, maxit=300))
    for o in out[1:]:
        assert o["iterations"] == out[0]["iterations"] and o["converged"]
        np.testing.assert_array_equal(o["x"].cpu().numpy(), out[0]["x"].cpu().numpy())


def test_split_auto():
    # 64 x 64 x 32, 2 z-slabs, the interior factored by ILUT: blocks of 61,440 rows take two workgroups each by
    # default (one per 24,576 rows; levels of at most 64 rows per part)
    m = silu()
    A = synth.aniso7(64, Nz=32)
    part = torch.as_tensor(synth.slab_partition(64, 2, Nz=32)).cuda()
    opts = dict(SCHUR_ILUT, inner_iters=5)
    Pa = m.setup(m.DeviceCSR.from_host(A), part, 2, **opts)
    P1 = m.setup(m.DeviceCSR.from_host(A), part, 2, block_split=1, **opts)
    sa = Pa.export("schedule")
    assert sa[0] == 1 and (sa[20], sa[21]) == (2, 2), sa
    r = torch.as_tensor(synth.uniform_rhs(A.n, 15)).cuda()
    np.testing.assert_array_equal(Pa.apply(r).cpu().numpy(), P1.apply(r).cpu().numpy())
    # ILU(0) of the same blocks has levels of up to 348 rows per part, too wide for the split solve's
    # workgroup: the default keeps one workgroup per subdomain
    o0 = dict(method=oracle.SCHUR, interior_fact=oracle.ILU0, interface_fact=oracle.MILU0, inner_iters=5)
    s0 = m.setup(m.DeviceCSR.from_host(A), part, 2, **o0).export("schedule")
    assert (s0[20], s0[21]) == (1, 1), s0


def _block_diag(B, copies):
    n = B.n
    rp = np.concatenate([[0]] + [B.row_ptr[1:] + c * B.nnz for c in range(copies)]).astype(np.int64)
    col = np.concatenate([B.col + c * n for c in range(copies)]).astype(np.int32)
    return synth.CSR(n * copies, rp, col, np.tile(B.val, copies))


@pytest.mark.parametrize("kind", ["more_parts_than_cus", "empty_parts"])
def test_split_extremes(kind):
    # more_parts_than_cus: 32 independent 128 x 16 grids, 16 parts each (one grid line per part): 512
    # workgroups, more than the device holds at once, so parts wait on parts that started before them while
    # others have not started yet.  empty_parts: a 10-row tridiagonal block in 16 parts, most of them empty.
    m = silu()
    if kind == "more_parts_than_cus":
        B = synth.aniso5(128, Ny=16)
        A = _block_diag(B, 32)
        part, p, k = (np.arange(A.n) // B.n).astype(np.int32), 32, 16
    else:
        A, part, p, k = synth.aniso5(10, Ny=1), None, 1, 16
    opts = dict(method=oracle.BJ, interior_fact=oracle.ILU0)
    Po = oracle.Precond(A, part, p, **opts)
    off = Po.export("offsets")
    want = [k if split_applies(*Po.csr(f)[:2], Po.export(lv), off, p, k, bw) else 1
            for f, lv, bw in (("LB", "lev_LB", False), ("UB", "lev_UB", True))]
    assert want == [k, k]
    print(f"[split] {kind}", flush=True)
    P1 = _setup(m, A, part, p, opts, 1)
    Pk = _setup(m, A, part, p, opts, k)
    sk = Pk.export("schedule")
    assert [sk[20], sk[21]] == want, sk
    r = torch.as_tensor(synth.uniform_rhs(A.n, 19)).cuda()
    z1 = P1.apply(r).cpu().numpy()
    for rep in range(3):
        np.testing.assert_array_equal(Pk.apply(r).cpu().numpy(), z1, err_msg=f"apply {rep}")
    zo = Po.apply(r.cpu().numpy())
    np.testing.assert_allclose(z1, zo, rtol=1e-12, atol=1e-12 * np.abs(zo).max())


def test_split_option_range():
    m = silu()
    A = synth.aniso5(8)
    with pytest.raises(m.SchurILUError) as e:
        m.setup(m.DeviceCSR.from_host(A), block_split=65)
    assert e.value.code == -1
    with pytest.raises(m.SchurILUError) as e:
        m.setup(m.DeviceCSR.from_host(A), block_split=-1)
    assert e.value.code == -1
