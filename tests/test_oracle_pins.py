"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these checks re-types the oracle's own loops: each compares it with a
closed form, a textbook factorization computed by a library routine (dense LU
without pivoting on column diagonally dominant matrices), a brute-force
definition on tiny inputs, or an invariant the paper states.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth
from synth import CSR

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def csr_dense(rp, ci, v, n, m=None):
    m = n if m is None else m
    d = np.zeros((n, m))
    rows = np.repeat(np.arange(n), np.diff(rp))
    d[rows, ci] = v
    return d


def lu_nopivot(A):
    """Dense LU by scipy; column diagonal dominance guarantees P = I."""
    P, L, U = sla.lu(A)
    assert np.array_equal(P, np.eye(A.shape[0])), "matrix must not need pivoting"
    return L, U


def col_dominant(n, seed, density=1.0):
    u = synth.uniform01(seed, n * n + n).reshape(-1)[: n * n].reshape(n, n) * 2 - 1
    mask = synth.uniform01(seed + 1, n * n).reshape(n, n) < density
    A = np.where(mask, u, 0.0)
    np.fill_diagonal(A, 0.0)
    np.fill_diagonal(A, np.abs(A).sum(axis=0) * 1.5 + 1.0)
    return A


# ---------------------------------------------------------------- P1, P2, P6
def test_p1_tridiagonal_ilu0_is_exact_lu():
    n = 40
    T = CSR.from_dense(2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1))
    F = oracle.factor(T, method=oracle.ILU0)
    i = np.arange(1, n + 1, dtype=float)
    np.testing.assert_allclose(F["D"], (i + 1) / i, rtol=1e-15)
    L = csr_dense(*F["L"], n)
    np.testing.assert_allclose(np.diag(L, -1), -(i[1:] - 1) / i[1:], rtol=1e-15)


@pytest.mark.parametrize("method", [oracle.ILU0, oracle.MILU0])
def test_p2_full_pattern_ilu0_equals_dense_lu(method):
    n = 24
    A = col_dominant(n, 11)
    F = oracle.factor(CSR.from_dense(A), method=method)
    Ld, Ud = lu_nopivot(A)
    L = csr_dense(*F["L"], n) + np.eye(n)
    U = csr_dense(*F["U"], n) + np.diag(F["D"])
    np.testing.assert_allclose(L, Ld, atol=1e-13)
    np.testing.assert_allclose(U, Ud, rtol=1e-12, atol=1e-12)


def test_p6_ilut_tau0_unlimited_equals_dense_lu():
    n = 20
    A = col_dominant(n, 21, density=0.25)
    F = oracle.factor(CSR.from_dense(A), method=oracle.ILUT, droptol=0.0, lfil=-1)
    Ld, Ud = lu_nopivot(A)
    L = csr_dense(*F["L"], n) + np.eye(n)
    U = csr_dense(*F["U"], n) + np.diag(F["D"])
    np.testing.assert_allclose(L, Ld, atol=1e-13)
    np.testing.assert_allclose(U, Ud, rtol=1e-12, atol=1e-12)


def test_p6_ilut_infinite_tau_keeps_diagonal():
    A = synth.aniso5(8)
    F = oracle.factor(A, method=oracle.ILUT, droptol=np.inf, lfil=-1)
    assert F["L"][1].size == 0 and F["U"][1].size == 0
    np.testing.assert_array_equal(F["D"], np.diag(A.dense()))


def test_ilut_lfil0_keeps_diagonal():
    A = synth.aniso5(8)
    F = oracle.factor(A, method=oracle.ILUT, droptol=0.0, lfil=0)
    assert F["L"][1].size == 0 and F["U"][1].size == 0
    np.testing.assert_array_equal(F["D"], np.diag(A.dense()))


def test_p6_partial_ilut_tau0_gives_exact_schur_blocks():
    n, nB = 14, 9
    A = col_dominant(n, 31, density=0.4)
    F = oracle.factor(CSR.from_dense(A), nfull=nB, method=oracle.ILUT, droptol=0.0, lfil=-1)
    B, Fm, E, Cm = A[:nB, :nB], A[:nB, nB:], A[nB:, :nB], A[nB:, nB:]
    LB, UB = lu_nopivot(B)
    Lf = csr_dense(*F["L"], n)
    Uf = csr_dense(*F["U"], nB, n)
    np.testing.assert_allclose(Lf[:nB, :nB] + np.eye(nB), LB, atol=1e-13)
    np.testing.assert_allclose(Uf[:, :nB] + np.diag(F["D"]), UB, atol=1e-12)
    W = Lf[nB:, :nB]
    np.testing.assert_allclose(W, E @ np.linalg.inv(UB), atol=1e-12)           # W = E U_B^-1
    np.testing.assert_allclose(Uf[:, nB:], np.linalg.solve(LB, Fm), atol=1e-12)  # Z = L_B^-1 F
    R = csr_dense(*F["R"], n - nB, n)[:, nB:]
    np.testing.assert_allclose(R, Cm - E @ np.linalg.solve(B, Fm), atol=1e-12)  # S = C - E B^-1 F


def test_ilut_hand_example():
    # A = [[4,0,1],[1,4,0],[0,1,4]], tau = 0.05: every row norm is sqrt(17), tau_i = 0.206.
    # row 1: w_0 = 1/4 = 0.25 >= tau_i -> kept, fill (1,2) = -0.25 * 1 = -0.25 kept, u_11 = 4.
    # row 2: w_1 = 1/4 kept, u_22 = 4 - 0.25 * (-0.25) = 4.0625.
    A = CSR.from_dense(np.array([[4.0, 0, 1], [1, 4, 0], [0, 1, 4]]))
    F = oracle.factor(A, method=oracle.ILUT, droptol=0.05, lfil=-1)
    np.testing.assert_array_equal(F["D"], [4.0, 4.0, 4.0625])
    np.testing.assert_array_equal(csr_dense(*F["L"], 3), [[0, 0, 0], [0.25, 0, 0], [0, 0.25, 0]])
    np.testing.assert_array_equal(csr_dense(*F["U"], 3), [[0, 0, 1], [0, 0, -0.25], [0, 0, 0]])
    # tau = 0.1: tau_i = 0.412 > 0.25, both multipliers are dropped before elimination.
    F = oracle.factor(A, method=oracle.ILUT, droptol=0.1, lfil=-1)
    np.testing.assert_array_equal(F["D"], [4.0, 4.0, 4.0])
    assert F["L"][1].size == 0
    # U keeps (0,2) = 1 since 1 >= tau_0 = 0.412
    np.testing.assert_array_equal(csr_dense(*F["U"], 3), [[0, 0, 1], [0, 0, 0], [0, 0, 0]])


def test_ilut_top_p_tie_breaks_on_column():
    A = CSR.from_dense(np.array([[4.0, 1.0, -1.0], [0, 4, 0], [0, 0, 4]]))
    F = oracle.factor(A, method=oracle.ILUT, droptol=0.0, lfil=1)
    assert list(F["U"][1]) == [1] and list(F["U"][2]) == [1.0]


# ---------------------------------------------------------------- P3, P4, P5
@pytest.mark.parametrize("gen", ["aniso5", "rot9", "random"])
def test_p3_ilu0_product_matches_a_on_pattern(gen):
    A = {"aniso5": lambda: synth.aniso5(12), "rot9": lambda: synth.rotated9(10),
         "random": lambda: synth.random_sparse(120, 6, 7)}[gen]()
    n = A.n
    for method in (oracle.ILU0, oracle.MILU0):
        F = oracle.factor(A, method=method)
        LU = (csr_dense(*F["L"], n) + np.eye(n)) @ (csr_dense(*F["U"], n) + np.diag(F["D"]))
        Ad = A.dense()
        pat = csr_dense(A.row_ptr, A.col, np.ones(A.nnz), n) != 0
        off = pat & ~np.eye(n, dtype=bool)
        np.testing.assert_allclose(LU[off], Ad[off], atol=1e-13)
        if method == oracle.ILU0:
            np.testing.assert_allclose(np.diag(LU), np.diag(Ad), atol=1e-13)
        else:  # P4: MILU keeps row sums, LU 1 = A 1
            np.testing.assert_allclose(LU.sum(axis=1), Ad.sum(axis=1), atol=1e-13 * np.abs(Ad).max())


def test_p5_closed_recurrences_on_the_5pt_grid():
    N, c = 64, 0.01
    A = synth.aniso5(N, c)
    d = 2 + 2 * c
    u_ilu = np.zeros(N * N)
    u_milu = np.zeros(N * N)
    for i in range(N * N):
        ix, iy = i % N, i // N
        u_ilu[i] = d - (1.0 / u_ilu[i - 1] if ix >= 1 else 0) - (c * c / u_ilu[i - N] if iy >= 1 else 0)
        u_milu[i] = (d - ((1 + (c if iy <= N - 2 else 0)) / u_milu[i - 1] if ix >= 1 else 0)
                     - ((c * c + (c if ix <= N - 2 else 0)) / u_milu[i - N] if iy >= 1 else 0))
    np.testing.assert_allclose(oracle.factor(A, method=oracle.ILU0)["D"], u_ilu, rtol=1e-14)
    np.testing.assert_allclose(oracle.factor(A, method=oracle.MILU0)["D"], u_milu, rtol=1e-14)
    # deep-interior fixed point of the ILU(0) recurrence: (1 + c) + sqrt(2 c)
    assert abs(u_ilu[(N // 2) * N + N // 2] - ((1 + c) + math.sqrt(2 * c))) < 1e-3


# ---------------------------------------------------------------- P7 levels
def brute_levels(A, lower):
    n = A.n
    lev = [None] * n
    deps = [[c for c in A.col[A.row_ptr[i]:A.row_ptr[i + 1]] if (c < i if lower else c > i)] for i in range(n)]

    def L(i):  # recursive definition, memoised
        if lev[i] is None:
            lev[i] = 0 if not deps[i] else 1 + max(L(j) for j in deps[i])
        return lev[i]

    order = range(n) if lower else range(n - 1, -1, -1)
    return np.array([L(i) for i in order])[:: 1 if lower else -1]


@pytest.mark.parametrize("lower", [True, False])
def test_p7_levels_match_definition(lower):
    A = synth.random_sparse(300, 5, 9)
    lv = oracle.levels(A.row_ptr, A.col, lower)
    np.testing.assert_array_equal(lv, brute_levels(A, lower))


def test_p7_level_count_closed_forms():
    A = synth.aniso5(64)
    assert oracle.levels(A.row_ptr, A.col, True).max() + 1 == 64 + 64 - 1
    A = synth.aniso7(6, Ny=5, Nz=4)
    assert oracle.levels(A.row_ptr, A.col, True).max() + 1 == 6 + 5 + 4 - 2
    A = synth.rotated9(40)
    assert oracle.levels(A.row_ptr, A.col, True).max() + 1 == 40 + 2 * 40 - 2
    assert oracle.levels(A.row_ptr, A.col, False).max() + 1 == 40 + 2 * 40 - 2


# ---------------------------------------------------------------- P8 partition
def test_p8_interface_counts_full_3d_slabs():
    A = synth.aniso7(128)
    part = synth.slab_partition(128, 16)
    iface = oracle.classify(A, part, 16)
    assert int(iface.sum()) == 491520
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    cross = part[rows] != part[A.col]
    assert int(cross.sum()) == 491520  # nnz(C_off)


def test_p8_permutation_invariants_random():
    A = synth.random_sparse(400, 6, 13, band=30)
    part = synth.block_partition(A.n, 5)
    iface = oracle.classify(A, part, 5)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    cross = part[rows] != part[A.col]
    expect = np.zeros(A.n, bool)
    expect[rows[cross]] = True
    expect[A.col[cross]] = True
    np.testing.assert_array_equal(iface.astype(bool), expect)
    perm, iperm, off = oracle.permutation(A.n, part, 5, iface)
    assert sorted(perm.tolist()) == list(range(A.n))
    np.testing.assert_array_equal(iperm[perm], np.arange(A.n))
    nB = off[5]
    assert nB == int((~expect).sum())
    # groups in order: interiors by part, then interfaces by part, ascending inside each group
    key = np.where(expect[perm], 5, 0) + part[perm]
    assert np.all(np.diff(key) >= 0)
    for s in range(10):
        g = perm[key == s]
        assert np.all(np.diff(g) > 0)


# ---------------------------------------------------------------- P9, P10, P11
def test_p9_exact_factors_give_exact_inverse_and_one_iteration():
    A = synth.aniso7(6)
    part = synth.slab_partition(6, 3)
    P = oracle.Precond(A, part, 3, method=oracle.SCHUR, interior_fact=oracle.ILUT, interface_fact=oracle.ILUT,
                       droptol=0.0, lfil=-1, inner_iters=200)
    r = synth.uniform_rhs(A.n, 5)
    z = P.apply(r)
    np.testing.assert_allclose(A.dense() @ z, r, atol=1e-10)
    out = oracle.fgmres(A, P, r, rtol=1e-8, restart=10, maxit=10)
    assert out["iterations"] == 1 and out["converged"]


def test_p10_one_subdomain_schur_is_block_jacobi():
    A = synth.aniso5(20)
    b = synth.uniform_rhs(A.n, 3)
    for f in (oracle.ILU0, oracle.MILU0, oracle.ILUT):
        Pb = oracle.Precond(A, None, 1, method=oracle.BJ, interior_fact=f, droptol=1e-3, lfil=5)
        Ps = oracle.Precond(A, None, 1, method=oracle.SCHUR, interior_fact=f, interface_fact=oracle.MILU0,
                            droptol=1e-3, lfil=5, inner_iters=3)
        np.testing.assert_array_equal(Pb.apply(b), Ps.apply(b))


def test_p11_two_routes_to_the_interface_factors_agree():
    A = synth.aniso7(8)
    part = synth.slab_partition(8, 4)
    Pb = oracle.Precond(A, part, 4, method=oracle.BJ, interior_fact=oracle.ILU0)
    Ps = oracle.Precond(A, part, 4, method=oracle.SCHUR, interior_fact=oracle.ILU0, interface_fact=oracle.ILU0)
    for name in ("LB", "UB", "Z", "W", "LS", "US"):
        for a, b in zip(Pb.csr(name), Ps.csr(name)):
            np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(Pb.export("DS"), Ps.export("DS"))
    Pb = oracle.Precond(A, part, 4, method=oracle.BJ, interior_fact=oracle.MILU0)
    Ps = oracle.Precond(A, part, 4, method=oracle.SCHUR, interior_fact=oracle.MILU0, interface_fact=oracle.MILU0)
    np.testing.assert_allclose(Pb.export("DS"), Ps.export("DS"), rtol=1e-14)


def test_bj_apply_is_block_lu_solve():
    A = synth.random_sparse(150, 6, 17, band=12)
    part = synth.block_partition(A.n, 3)
    P = oracle.Precond(A, part, 3, method=oracle.BJ, interior_fact=oracle.ILU0)
    perm = P.export("perm")
    n, nB = A.n, int(P.export("offsets")[3])
    L = np.eye(n)
    U = np.zeros((n, n))
    L[:nB, :nB] += csr_dense(*P.csr("LB"), nB)
    L[nB:, :nB] = csr_dense(*P.csr("W"), n - nB, nB)
    L[nB:, nB:] += csr_dense(*P.csr("LS"), n - nB)
    U[:nB, :nB] = csr_dense(*P.csr("UB"), nB) + np.diag(P.export("DB"))
    U[:nB, nB:] = csr_dense(*P.csr("Z"), nB, n)[:, nB:]
    U[nB:, nB:] = csr_dense(*P.csr("US"), n - nB) + np.diag(P.export("DS"))
    r = synth.uniform_rhs(n, 1)
    zp = np.linalg.solve(U, np.linalg.solve(L, r[perm]))
    z = np.empty(n)
    z[perm] = zp
    np.testing.assert_allclose(P.apply(r), z, rtol=1e-12, atol=1e-12)
    # (LU) agrees with the permuted intra-subdomain matrix on its pattern
    Ad = A.dense()[np.ix_(perm, perm)]
    pp = part[perm]
    intra = (pp[:, None] == pp[None, :]) & (Ad != 0)
    np.testing.assert_allclose((L @ U)[intra], Ad[intra], atol=1e-12)


# ---------------------------------------------------------------- P12 GMRES
@pytest.mark.parametrize("q", [2, 3, 5])
def test_p12_gmres_terminates_after_q_distinct_eigenvalues(q):
    # A = D (I + s C), C a q-cycle on each block; with one row per subdomain the
    # block-Jacobi preconditioner is D, so M^-1 A = I + s C has q distinct eigenvalues.
    nb = 7
    n = q * nb
    Cm = np.zeros((n, n))
    for b in range(nb):
        for k in range(q):
            Cm[b * q + k, b * q + (k + 1) % q] = 1.0
    D = np.diag(1.0 + np.arange(n) % 4)
    Ad = D @ (np.eye(n) + 0.5 * Cm)
    A = CSR.from_dense(Ad)
    P = oracle.Precond(A, np.arange(n, dtype=np.int32), n, method=oracle.BJ)
    out = oracle.fgmres(A, P, synth.uniform_rhs(n, 2), rtol=1e-10, restart=20, maxit=20)
    assert out["iterations"] == q


def test_p12_implicit_residual_tracks_true_residual_and_solution():
    A, b, part, _ = synth.workload("aniso2d_64")
    P = oracle.Precond(A, part, 1, method=oracle.BJ)
    out = oracle.fgmres(A, P, b, rtol=1e-8, restart=30, maxit=500, history=True)
    assert out["converged"]
    true_rel = np.linalg.norm(b - A.matvec(out["x"])) / np.linalg.norm(b)
    assert true_rel <= 1e-8
    assert abs(true_rel - out["relres"]) <= 1e-12
    assert abs(out["history"][-1] - true_rel) <= 1e-10
    np.testing.assert_allclose(out["x"], np.ones(A.n), atol=1e-5)


def test_spmv_and_residual_match_dense():
    A = synth.random_sparse(200, 8, 23)
    x = synth.uniform_rhs(A.n, 4)
    b = synth.uniform_rhs(A.n, 5)
    np.testing.assert_allclose(oracle.spmv(A, x), A.dense() @ x, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(oracle.residual(A, b, x), b - A.dense() @ x, rtol=1e-13, atol=1e-13)


def test_p13_soft_paper_sanity_2d_poisson():
    # BJ-ILU(0)+FGMRES(50), rtol 1e-8, one subdomain, 2D 256^2 5-pt Poisson (the paper
    # used RCM ordering and an unstated b; natural order here, so only +-25 %).
    ref = json.load(open(os.path.join(GOLDEN, "paper_values.json")))
    its = ref["weak_scaling_2d_256sq_np1_bj_ilu0_fgmres50_its"]["value"]
    A = synth.aniso5(256, 1.0)
    b = synth.uniform_rhs(A.n, 2)
    P = oracle.Precond(A, None, 1, method=oracle.BJ)
    out = oracle.fgmres(A, P, b, rtol=1e-8, restart=50, maxit=2000)
    assert out["converged"]
    assert 0.75 * its <= out["iterations"] <= 1.25 * its, out["iterations"]


def test_inner_gmres_is_krylov_least_squares():
    # The reduced system (I + D^-1 C_off) y = D^-1 g' (eq. (18)) solved by k GMRES steps
    # from zero: y minimises the residual over K_k(T, rhs).  Built densely from the
    # exported factors, independent of the oracle's Arnoldi loop.
    A = synth.aniso7(8)
    part = synth.slab_partition(8, 4)
    k = 3
    P = oracle.Precond(A, part, 4, method=oracle.SCHUR, interior_fact=oracle.ILU0,
                       interface_fact=oracle.MILU0, inner_iters=k)
    perm = P.export("perm")
    n, nB = A.n, int(P.export("offsets")[4])
    nS = n - nB
    r = synth.uniform_rhs(n, 8)
    z = P.apply(r)
    LB = csr_dense(*P.csr("LB"), nB) + np.eye(nB)
    UB = csr_dense(*P.csr("UB"), nB) + np.diag(P.export("DB"))
    Zm = csr_dense(*P.csr("Z"), nB, n)[:, nB:]
    W = csr_dense(*P.csr("W"), nS, nB)
    D = (csr_dense(*P.csr("LS"), nS) + np.eye(nS)) @ (csr_dense(*P.csr("US"), nS) + np.diag(P.export("DS")))
    Coff = csr_dense(*P.csr("Coff"), nS)
    assert np.count_nonzero(Coff) > 0
    fp = np.linalg.solve(LB, r[perm[:nB]])
    gp = r[perm[nB:]] - W @ fp
    T = np.eye(nS) + np.linalg.solve(D, Coff)
    rhs = np.linalg.solve(D, gp)
    K = np.stack([np.linalg.matrix_power(T, j) @ rhs for j in range(k)], axis=1)
    c = np.linalg.lstsq(T @ K, rhs, rcond=None)[0]
    y = K @ c
    np.testing.assert_allclose(z[perm[nB:]], y, rtol=1e-9, atol=1e-12)
    u = np.linalg.solve(UB, fp - Zm @ y)
    np.testing.assert_allclose(z[perm[:nB]], u, rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------- errors
def test_error_paths():
    A = synth.aniso5(4)
    bad = CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    bad.col[1], bad.col[2] = bad.col[2], bad.col[1]
    assert oracle.validate(bad) == oracle.ERR_CSR
    nodiag = CSR.from_dense(np.array([[0.0, 1.0], [1.0, 1.0]]))
    # from_dense always stores the diagonal; a stored zero pivot must be reported
    with pytest.raises(oracle.OracleError) as e:
        oracle.Precond(nodiag, None, 1, method=oracle.BJ)
    assert e.value.code == oracle.ERR_ZERO_PIVOT
    P = oracle.Precond(nodiag, None, 1, method=oracle.BJ, pivot_mode=oracle.PIVOT_PERTURB, pivot_tol=1e-3)
    assert np.all(np.isfinite(P.apply(np.ones(2))))
    with pytest.raises(oracle.OracleError):
        oracle.Precond(A, np.full(A.n, 3, np.int32), 2, method=oracle.BJ)


# ---------------------------------------------------------------- pivots (Section 4.1 reading R7)
@pytest.mark.parametrize("a00, a01, tol, u00", [
    (0.0, 1.0, 1e-3, 1e-3),      # zero pivot -> +tol * max_j |a_0j|
    (-1e-6, 1.0, 1e-3, -1e-3),   # small negative pivot keeps its sign
    (1.5e-3, 1.0, 1e-3, 1.5e-3),  # above the threshold: untouched
    (0.0, 4.0, 1e-3, 4e-3),      # threshold scales with the row's largest magnitude
])
def test_perturbed_pivot_hand_values(a00, a01, tol, u00):
    # [[a00, a01], [1, 1]]: u_00 as listed; then l_10 = 1 / u_00 and
    # u_11 = 1 - l_10 * a01 (row 1's largest magnitude is 1, so u_11 is never perturbed).
    A = CSR.from_dense(np.array([[a00, a01], [1.0, 1.0]]))
    F = oracle.factor(A, method=oracle.ILU0, pivot_mode=oracle.PIVOT_PERTURB, pivot_tol=tol)
    np.testing.assert_allclose(F["D"][0], u00, rtol=1e-15)
    np.testing.assert_allclose(F["L"][2], [1.0 / u00], rtol=1e-15)
    np.testing.assert_allclose(F["D"][1], 1.0 - a01 / u00, rtol=1e-12)


def test_perturbed_pivot_hand_example_values():
    # [[0, 1], [1, 1]] with tol 1e-3: u_00 = 1e-3, l_10 = 1000, u_11 = -999.
    A = CSR.from_dense(np.array([[0.0, 1.0], [1.0, 1.0]]))
    F = oracle.factor(A, method=oracle.ILU0, pivot_mode=oracle.PIVOT_PERTURB, pivot_tol=1e-3)
    np.testing.assert_allclose(F["D"], [1e-3, -999.0], rtol=1e-13)
    np.testing.assert_allclose(F["L"][2], [1000.0], rtol=1e-13)


# ---------------------------------------------------------------- partial ILUT rows (Section 3.2, eq. (17))
def _partial_example():
    # One interior row (nfull = 1) and five partially eliminated rows.
    #   row 0 = [4, 0, 2, 0, 0, 0]                        -> u_00 = 4, U row {2: 2}
    #   row 1 = [1, 8, 2, -1, 0.5, 2^-10]                 (||a_1||_2 = sqrt(70.25 + 2^-20))
    #   row 2 = [2^-9, 0, 8, 0, 0, 0]
    #   rows 3..5 = 8 on the diagonal.
    M = np.zeros((6, 6))
    M[0, 0], M[0, 2] = 4.0, 2.0
    M[1] = [1.0, 8.0, 2.0, -1.0, 0.5, 2.0 ** -10]
    M[2, 0], M[2, 2] = 2.0 ** -9, 8.0
    for r in (3, 4, 5):
        M[r, r] = 8.0
    return CSR.from_dense(M)


def test_partial_ilut_schur_part_hand_values():
    # droptol 2^-6: tau_1 = 2^-6 sqrt(70.25 + 2^-20) = 0.13096.
    # Row 1: w_0 = 1/4 = 0.25 >= tau_1 is kept and eliminated: w_2 = 2 - 0.25 * 2 = 1.5.
    # Its Schur part (columns >= 1, off the diagonal) then holds 1.5, -1, 0.5 and 2^-10;
    # 2^-10 < tau_1 is dropped.  With lfil = 2 the two largest (1.5, -1) are kept and the
    # diagonal 8 is kept on top of them, not counted.
    # Row 2: w_0 = 2^-9 / 4 = 2^-11 < tau_2 = 2^-6 * 8: the multiplier is dropped before
    # elimination, so neither W nor fill appears.
    A = _partial_example()
    F = oracle.factor(A, nfull=1, method=oracle.ILUT, droptol=2.0 ** -6, lfil=2)
    np.testing.assert_array_equal(F["R"][0], [0, 3, 4, 5, 6, 7])
    np.testing.assert_array_equal(F["R"][1], [1, 2, 3, 2, 3, 4, 5])
    np.testing.assert_array_equal(F["R"][2], [8.0, 1.5, -1.0, 8.0, 8.0, 8.0, 8.0])
    np.testing.assert_array_equal(F["L"][0], [0, 0, 1, 1, 1, 1, 1])
    np.testing.assert_array_equal(F["L"][2], [0.25])
    # no fill limit: 0.5 stays, 2^-10 is still below tau_1
    F = oracle.factor(A, nfull=1, method=oracle.ILUT, droptol=2.0 ** -6, lfil=-1)
    np.testing.assert_array_equal(F["R"][1], [1, 2, 3, 4, 2, 3, 4, 5])
    np.testing.assert_array_equal(F["R"][2], [8.0, 1.5, -1.0, 0.5, 8.0, 8.0, 8.0, 8.0])
    # lfil = 0: only the diagonal of each Schur row survives
    F = oracle.factor(A, nfull=1, method=oracle.ILUT, droptol=2.0 ** -6, lfil=0)
    np.testing.assert_array_equal(F["R"][1], [1, 2, 3, 4, 5])
    np.testing.assert_array_equal(F["L"][1].size, 0)


def test_partial_ilut_w_part_fill_limit():
    # [[4,0,0,1],[2,4,0,0],[0,0,4,1],[1,-3,2,8]], nfull = 3, lfil = 2, droptol 0.
    # Full rows: U row 0 = {3: 1}; row 1: l_10 = 2/4 = 0.5, fill u_13 = -0.5 * 1 = -0.5;
    # U row 2 = {3: 1}.  Partial row 3 eliminates columns 0, 1, 2 with every multiplier:
    # w_0 = 1/4, w_1 = -3/4, w_2 = 2/4, and its Schur entry is
    # 8 - 0.25 * 1 - (-0.75) * (-0.5) - 0.5 * 1 = 6.875.  The cap then keeps the two
    # largest multipliers (-0.75 at column 1, 0.5 at column 2) in W.
    M = np.array([[4.0, 0, 0, 1], [2, 4, 0, 0], [0, 0, 4, 1], [1, -3, 2, 8]])
    F = oracle.factor(CSR.from_dense(M), nfull=3, method=oracle.ILUT, droptol=0.0, lfil=2)
    L = csr_dense(*F["L"], 4)
    np.testing.assert_array_equal(L[3], [0.0, -0.75, 0.5, 0.0])
    np.testing.assert_array_equal(F["R"][2], [6.875])
    np.testing.assert_array_equal(L[1], [0.5, 0, 0, 0])
    np.testing.assert_array_equal(csr_dense(*F["U"], 3, 4)[1], [0, 0, 0, -0.5])


# ---------------------------------------------------------------- CSR validation (reading R10)
def _valid_3x3():
    return CSR.from_dense(np.array([[4.0, 1, 0], [1, 4, 1], [0, 1, 4]]))


@pytest.mark.parametrize("defect", ["missing_diag", "duplicate", "unsorted", "col_negative", "col_too_big",
                                    "row_ptr_start", "row_ptr_decreasing"])
def test_validate_rejects_each_defect(defect):
    A = _valid_3x3()
    assert oracle.validate(A) == 0
    rp, ci, v = A.row_ptr.copy(), A.col.copy(), A.val.copy()
    if defect == "missing_diag":   # row 1 = {0, 2}: no (1, 1)
        rp = np.array([0, 2, 4, 6]); ci = np.array([0, 1, 0, 2, 1, 2]); v = np.ones(6)
    elif defect == "duplicate":
        ci[2], ci[3] = 1, 1  # row 1 = {0, 1, 1, 2}: the diagonal twice
    elif defect == "unsorted":
        ci[2], ci[3] = ci[3], ci[2]
    elif defect == "col_negative":
        ci[4] = -1
    elif defect == "col_too_big":
        ci[4] = 3
    elif defect == "row_ptr_start":
        rp = rp.copy(); rp[0] = 1
    elif defect == "row_ptr_decreasing":
        rp = rp.copy(); rp[2] = rp[1] - 1
    assert oracle.validate(CSR(3, rp, ci.astype(np.int32), v)) == oracle.ERR_CSR, defect


# ---------------------------------------------------------------- inner GMRES early exit (reading R5)
def test_inner_rtol_stops_at_the_krylov_least_squares_step():
    # With inner_rtol the reduced-system GMRES stops at the first step j whose residual
    # min_{y in K_j} ||rhs - T y|| is <= inner_rtol ||rhs||.  The residuals r_j are computed
    # densely here; inner_rtol sits at the geometric mean of r_1 and r_2, so exactly two
    # steps are taken and the result is the 2-step least-squares solution, not the k-step one.
    A = synth.aniso7(8)
    part = synth.slab_partition(8, 4)
    k = 6
    base = dict(method=oracle.SCHUR, interior_fact=oracle.ILU0, interface_fact=oracle.MILU0, inner_iters=k)
    P = oracle.Precond(A, part, 4, **base)
    perm = P.export("perm")
    n, nB = A.n, int(P.export("offsets")[4])
    nS = n - nB
    r = synth.uniform_rhs(n, 8)
    LB = csr_dense(*P.csr("LB"), nB) + np.eye(nB)
    W = csr_dense(*P.csr("W"), nS, nB)
    D = (csr_dense(*P.csr("LS"), nS) + np.eye(nS)) @ (csr_dense(*P.csr("US"), nS) + np.diag(P.export("DS")))
    T = np.eye(nS) + np.linalg.solve(D, csr_dense(*P.csr("Coff"), nS))
    rhs = np.linalg.solve(D, r[perm[nB:]] - W @ np.linalg.solve(LB, r[perm[:nB]]))
    beta = np.linalg.norm(rhs)

    def ls(j):
        K = np.stack([np.linalg.matrix_power(T, i) @ rhs for i in range(j)], axis=1)
        c = np.linalg.lstsq(T @ K, rhs, rcond=None)[0]
        return K @ c, np.linalg.norm(rhs - T @ (K @ c))

    (y1, r1), (y2, r2), (yk, rk) = ls(1), ls(2), ls(k)
    assert r1 > r2 > rk and r1 / r2 < 1e3
    tol = math.sqrt(r1 * r2) / beta
    z = oracle.Precond(A, part, 4, inner_rtol=tol, **base).apply(r)
    np.testing.assert_allclose(z[perm[nB:]], y2, rtol=1e-9, atol=1e-12)
    assert np.linalg.norm(y2 - yk) > 1e-6 * np.linalg.norm(yk)


# ---------------------------------------------------------------- GMRES(m) of the batched systems
def _bj_factors(P, n):
    L = csr_dense(*P.csr("LB"), n) + np.eye(n)
    U = csr_dense(*P.csr("UB"), n) + np.diag(P.export("DB"))
    return L @ U


def _gmres_ls(A, M, b, x0, k):
    # x0 + M^-1 y, y minimising ||r0 - A M^-1 y|| over the Krylov space K_k(A M^-1, r0)
    T = A @ np.linalg.inv(M)
    r0 = b - A @ x0
    K = np.stack([np.linalg.matrix_power(T, j) @ r0 for j in range(k)], axis=1)
    c = np.linalg.lstsq(T @ K, r0, rcond=None)[0]
    return x0 + np.linalg.solve(M, K @ c)


def test_gmres_is_right_preconditioned_krylov_least_squares():
    # k < restart steps from x0 = 0, then a second cycle of 3 steps from that iterate:
    # each cycle's x is the least-squares solution over its own Krylov space.
    A = synth.convdiff5(9, 0.05, 0.7, 20.0)
    b = synth.uniform_rhs(A.n, 12)
    P = oracle.Precond(A, None, 1, method=oracle.BJ, interior_fact=oracle.ILU0)
    Ad, M = A.dense(), _bj_factors(P, A.n)
    k = 6
    out = oracle.gmres(A, P, b, rtol=0.0, restart=20, maxit=k)
    assert out["iterations"] == k and not out["converged"]
    x1 = _gmres_ls(Ad, M, b, np.zeros(A.n), k)
    np.testing.assert_allclose(out["x"], x1, rtol=1e-9, atol=1e-12 * np.abs(x1).max())
    out = oracle.gmres(A, P, b, rtol=0.0, restart=k, maxit=k + 3)
    x2 = _gmres_ls(Ad, M, b, x1, 3)
    np.testing.assert_allclose(out["x"], x2, rtol=1e-9, atol=1e-12 * np.abs(x2).max())
    # the flexible variant with a fixed preconditioner reaches the same iterates
    outf = oracle.fgmres(A, P, b, rtol=0.0, restart=k, maxit=k + 3)
    np.testing.assert_allclose(outf["x"], x2, rtol=1e-9, atol=1e-12 * np.abs(x2).max())


def test_gmres_exact_preconditioner_and_implicit_residual():
    # ILU(0) of a tridiagonal matrix is its exact LU, so M = A and one step solves
    # the system; on a general system the Givens estimate equals the true residual.
    T = CSR.from_dense(3 * np.eye(30) - np.eye(30, k=1) - 0.5 * np.eye(30, k=-1))
    b = synth.uniform_rhs(30, 13)
    P = oracle.Precond(T, None, 1, method=oracle.BJ, interior_fact=oracle.ILU0)
    out = oracle.gmres(T, P, b, rtol=1e-12, restart=20, maxit=50)
    assert out["converged"] and out["iterations"] == 1
    A = synth.convdiff5(12, 0.01, 2.0, 35.0)
    b = synth.uniform_rhs(A.n, 14)
    P = oracle.Precond(A, None, 1, method=oracle.BJ, interior_fact=oracle.ILU0)
    out = oracle.gmres(A, P, b, rtol=1e-10, restart=20, maxit=17, history=True)
    true = np.linalg.norm(b - A.dense() @ out["x"]) / np.linalg.norm(b)
    np.testing.assert_allclose(out["history"][-1], true, rtol=1e-6)


# ---------------------------------------------------------------- multiplicative RAP-ILU ("Two-level multiplicative solve", Section 3.3)
def _rap_pieces(P, A, nB):
    """Dense R, P (permuted numbering) and the permuted A, from the exported factors."""
    n = A.n
    nS = n - nB
    perm = P.export("perm")
    Ap = A.dense()[np.ix_(perm, perm)]
    LB = csr_dense(*P.csr("LB"), nB) + np.eye(nB)
    UB = csr_dense(*P.csr("UB"), nB) + np.diag(P.export("DB"))
    Zm = csr_dense(*P.csr("Z"), nB, n)[:, nB:]
    W = csr_dense(*P.csr("W"), nS, nB)
    R = np.hstack([-W @ np.linalg.inv(LB), np.eye(nS)])
    Pm = np.vstack([-np.linalg.solve(UB, Zm), np.eye(nS)])
    return Ap, R, Pm, LB, UB, W, Zm


@pytest.mark.parametrize("coarse", [oracle.ILU0, oracle.MILU0])
def test_rap_matvec_is_the_galerkin_product(coarse):
    # eq. (28): R A P with R = (-W L_B^-1, I) and P = (-U_B^-1 Z; I), unformed in the oracle
    A = synth.aniso7(8, Nz=12)
    part = synth.slab_partition(8, 3, Nz=12)
    P = oracle.Precond(A, part, 3, method=oracle.RAP, interior_fact=coarse, inner_iters=3)
    nB = int(P.export("offsets")[3])
    Ap, R, Pm, *_ = _rap_pieces(P, A, nB)
    nS = A.n - nB
    S2 = np.stack([P.rap_matvec(np.eye(nS)[:, j]) for j in range(nS)], axis=1)
    np.testing.assert_allclose(S2, R @ Ap @ Pm, atol=1e-12 * np.abs(S2).max())


def _cylinder_laplacian(nx, ny):
    """Graph Laplacian of an nx-by-ny grid closed in y (a cylinder): every row sums to zero."""
    n = nx * ny
    d = np.zeros((n, n))
    for y in range(ny):
        for x in range(nx):
            i = x + nx * y
            for j in ([i - 1] if x > 0 else []) + ([i + 1] if x < nx - 1 else []) + \
                     [x + nx * ((y + 1) % ny), x + nx * ((y - 1) % ny)]:
                d[i, j] = -1.0
    np.fill_diagonal(d, -d.sum(axis=1))
    return CSR.from_dense(d)


def test_rap_milu_keeps_constants():
    # With MILU(0) factors H 1 = 0, so P 1 = 1 when the interior rows have zero row sums, and
    # the constant vector passes the coarse operator as the local Schur factors pass it:
    # R A P 1 = L_S U_S 1 + C_off 1 (Section 3.3; C_off couples the subdomains' interfaces and
    # lies in no local factor).  Standard ILU(0) factors do not have this property.  The
    # cylinder puts interface rows at both ends of every slab, so no subdomain block is singular.
    A = _cylinder_laplacian(12, 12)
    part = (np.arange(A.n) // 48).astype(np.int32)  # three slabs of four grid lines
    out = {}
    for coarse in (oracle.MILU0, oracle.ILU0):
        P = oracle.Precond(A, part, 3, method=oracle.RAP, interior_fact=coarse, inner_iters=3)
        nB = int(P.export("offsets")[3])
        nS = A.n - nB
        one = np.ones(nS)
        LS = csr_dense(*P.csr("LS"), nS) + np.eye(nS)
        US = csr_dense(*P.csr("US"), nS) + np.diag(P.export("DS"))
        Coff = csr_dense(*P.csr("Coff"), nS)
        out[coarse] = np.abs(P.rap_matvec(one) - (LS @ (US @ one) + Coff @ one)).max()
        if coarse == oracle.MILU0:
            Ap, R, Pm, *_ = _rap_pieces(P, A, nB)
            np.testing.assert_allclose(Pm @ one, np.ones(A.n), atol=1e-13)  # P 1 = 1
    assert out[oracle.MILU0] <= 1e-13
    assert out[oracle.ILU0] > 1e-3


def test_rap_remark_difference_of_schur_complements():
    # Remark 1(3): with R = (-E B~^-1, I) and P = (-B~^-1 F; I), S_A2 = R A P and
    # S_A1 = C - E B~^-1 F differ by E B~^-1 B B~^-1 F - E B~^-1 F.  With dense E and F
    # blocks the (M)ILU(0) factors drop nothing in them (W U_B = E, L_B Z = F), so the
    # oracle's R and P are exactly these, while B~^-1 = (L_B U_B)^-1 != B^-1 (B drops fill).
    nb, ni = 6, 2  # interior and interface rows per subdomain
    n = 2 * (nb + ni)
    d = np.zeros((n, n))
    rng = synth.uniform01(77, 4 * n * n).reshape(4, n, n) - 0.5
    for k in range(2):
        o = k * (nb + ni)
        I = np.arange(o, o + nb)
        F = np.arange(o + nb, o + nb + ni)
        for i in range(nb - 1):
            d[I[i], I[i + 1]], d[I[i + 1], I[i]] = rng[0, I[i], I[i + 1]], rng[0, I[i + 1], I[i]]
        d[I[0], I[nb - 1]], d[I[nb - 1], I[0]] = 0.4, 0.3  # long-range coupling: ILU(0) drops fill in B
        d[np.ix_(F, I)] = rng[1][np.ix_(F, I)]
        d[np.ix_(I, F)] = rng[2][np.ix_(I, F)]
        d[np.ix_(F, F)] = rng[3][np.ix_(F, F)]
    o1, o2 = nb, (nb + ni) + nb  # cross-subdomain coupling of the interface rows
    d[o1, o2], d[o2, o1], d[o1 + 1, o2 + 1], d[o2 + 1, o1 + 1] = -0.2, -0.25, 0.15, -0.1
    np.fill_diagonal(d, 0.0)
    np.fill_diagonal(d, np.abs(d).sum(axis=1) + 1.0)
    A = CSR.from_dense(d)
    part = (np.arange(n) // (nb + ni)).astype(np.int32)
    P = oracle.Precond(A, part, 2, method=oracle.RAP, interior_fact=oracle.ILU0, inner_iters=3)
    nB = int(P.export("offsets")[2])
    assert nB == 2 * nb
    Ap, R, Pm, LB, UB, W, Zm = _rap_pieces(P, A, nB)
    B, Fm, E, Cm = Ap[:nB, :nB], Ap[:nB, nB:], Ap[nB:, :nB], Ap[nB:, nB:]
    Bt = np.linalg.inv(LB @ UB)
    np.testing.assert_allclose(W @ UB, E, atol=1e-13)
    np.testing.assert_allclose(LB @ Zm, Fm, atol=1e-13)
    S2 = np.stack([P.rap_matvec(np.eye(n - nB)[:, j]) for j in range(n - nB)], axis=1)
    S1 = Cm - E @ Bt @ Fm
    diff = E @ Bt @ B @ Bt @ Fm - E @ Bt @ Fm
    assert np.abs(diff).max() > 1e-4  # B~^-1 really is inexact
    np.testing.assert_allclose(S2 - S1, diff, atol=1e-12)


def test_rap_apply_closed_form():
    # Remark 1(2) with this smoother: z = S r + P (RAP)^-1 R (r - A S r), S the block-Jacobi
    # ILU(0) smoother; the reduced GMRES takes n_S steps, so it solves R A P v = R(...) exactly.
    A = synth.aniso7(6, Nz=8)
    part = synth.slab_partition(6, 2, Nz=8)
    Pb = oracle.Precond(A, part, 2, method=oracle.BJ, interior_fact=oracle.ILU0)
    probe = oracle.Precond(A, part, 2, method=oracle.RAP, interior_fact=oracle.MILU0, inner_iters=1)
    nB = int(probe.export("offsets")[2])
    nS = A.n - nB
    P = oracle.Precond(A, part, 2, method=oracle.RAP, interior_fact=oracle.MILU0, inner_iters=nS)
    Ap, R, Pm, *_ = _rap_pieces(P, A, nB)
    perm = P.export("perm")
    r = synth.uniform_rhs(A.n, 31)
    x = Pb.apply(r)
    res = r - A.dense() @ x
    v = np.linalg.solve(R @ Ap @ Pm, R @ res[perm])
    zref = x.copy()
    zref[perm] += Pm @ v
    np.testing.assert_allclose(P.apply(r), zref, rtol=1e-8, atol=1e-10 * np.abs(zref).max())


def test_rap_milu_converges_faster_than_block_jacobi():
    # the paper's Fig. 3: on 2D Poisson with many subdomains RAP-MILU(0) needs far fewer
    # iterations than BJ-ILU(0) (soft: only the ordering is checked)
    A = synth.aniso5(48, 1.0)
    part = (np.arange(A.n) // (48 * 6)).astype(np.int32)  # 8 horizontal slabs
    b = synth.uniform_rhs(A.n, 5)
    its = {}
    for name, o in (("bj", dict(method=oracle.BJ)), ("rap", dict(method=oracle.RAP, interior_fact=oracle.MILU0,
                                                                   inner_iters=3))):
        P = oracle.Precond(A, part, 8, **o)
        out = oracle.fgmres(A, P, b, rtol=1e-8, restart=50, maxit=2000)
        assert out["converged"]
        its[name] = out["iterations"]
    assert its["rap"] < its["bj"], its
