"""Pins for the oracle's solvers: Chambolle-Pock for eq. (priorsys) with TV and x >= 0,
nonnegative SIRT (eq. sirtit + eq. sirtbox), and the power-iteration step size."""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.optimize as sopt
import scipy.sparse as sp

import oracle


def _grad_matrix(rows, cols):
    """Forward differences (Neumann) as an explicit 2P x P matrix, built by loops -
    independent of the oracle's array code."""
    P = rows * cols
    D = np.zeros((2 * P, P))
    for r in range(rows):
        for c in range(cols):
            j = r * cols + c
            if r + 1 < rows:
                D[j, j] -= 1.0
                D[j, j + cols] += 1.0
            if c + 1 < cols:
                D[P + j, j] -= 1.0
                D[P + j, j + 1] += 1.0
    return D


def _admm_tv_nonneg(W, b, rows, cols, lam, rho=None, iters=100000, half=False, aniso=False):
    """Independent minimiser of c ||Wx - b||^2 + lam TV(x) s.t. x >= 0 (c = 1, or 1/2 with
    half), TV isotropic (sum_j ||(Dx)_j||_2) or anisotropic (||Dx||_1), by ADMM with the
    splittings u = Dx, v = x and dense Cholesky solves.  The u-step is the prox of the
    penalty: block shrinkage of each pixel's 2-vector (isotropic) or soft thresholding of
    each component (anisotropic)."""
    P = rows * cols
    D = _grad_matrix(rows, cols)
    cdat = 0.5 if half else 1.0
    if rho is None:
        rho = float(np.linalg.norm(W, 2) ** 2)
    A = 2 * cdat * W.T @ W + rho * D.T @ D + rho * np.eye(P)
    cf = sla.cho_factor(A)
    Wb2 = 2 * cdat * W.T @ b
    u = np.zeros(2 * P); a = np.zeros(2 * P)
    v = np.zeros(P); c = np.zeros(P)
    for _ in range(iters):
        x = sla.cho_solve(cf, Wb2 + rho * D.T @ (u - a) + rho * (v - c))
        Dx = D @ x
        q = Dx + a
        if aniso:
            u = np.sign(q) * np.maximum(0.0, np.abs(q) - lam / rho)
        else:
            nrm = np.sqrt(q[:P] ** 2 + q[P:] ** 2)
            scale = np.maximum(0.0, 1.0 - (lam / rho) / np.maximum(nrm, 1e-300))
            u = np.concatenate([q[:P] * scale, q[P:] * scale])
        v = np.maximum(0.0, x + c)
        a += Dx - u
        c += x - v
    return v.reshape(rows, cols)


def test_power_iteration_matches_eigvalsh():
    g = oracle.make_geometry(8, 6, 12)
    rect = (0, 0, 8, 8)
    WL = oracle.sparse_local(g, rect)
    D = _grad_matrix(8, 8)
    M = WL.toarray().T @ WL.toarray() + D.T @ D
    lam_max = np.linalg.eigvalsh(M)[-1]
    assert oracle.power_norm_sq(WL, (8, 8), iters=500) == pytest.approx(lam_max, rel=1e-9)
    s, t = oracle.cp_steps(WL, (8, 8), iters=500)
    assert s * t * lam_max < 1.0


@pytest.mark.parametrize("h", [1.0, 0.2, 1.0 / 64])
def test_cp_steps_bound_the_operator_norm(h):
    """sigma tau ||K||^2 < 1 for K = [h W_L; grad] whatever the data unit h, with
    ||K||^2 from eigvalsh of the explicit h^2 W^T W + D^T D, on a 64-grid part with the
    workload's 32 angles (the power iteration alone, started from all ones, misses most
    of the Laplacian's top eigenvalue when h is small); and the step is within 3 % of
    the largest admissible one when the data part dominates (h = 1)."""
    g = oracle.make_geometry(128, 32, 192)
    ext = (32, 32, 24, 24)
    WL = oracle.sparse_local(g, ext)
    D = _grad_matrix(24, 24)
    W = WL.toarray()
    norm2 = np.linalg.eigvalsh(h * h * W.T @ W + D.T @ D)[-1]
    s, t = oracle.cp_steps(WL, (24, 24), h=h)
    assert s * t * norm2 < 1.0
    assert np.linalg.eigvalsh(D.T @ D)[-1] < 8.0
    if h == 1.0:
        assert s * t * norm2 > 0.97


@pytest.mark.parametrize("n,na,nd,lam", [(8, 6, 12, 3.0), (12, 5, 17, 1.5)])
def test_cp_converges_to_independent_admm_minimiser(n, na, nd, lam):
    """CP's objective approaches the minimum found by an independent ADMM minimiser
    (ADMM itself agrees across penalty parameters to 1e-8), on tiny problems with TV
    and x >= 0 active.  CP's objective gap decays like O(1/k): under 3e-5 relative
    after 40000 iterations and at least 4x smaller than after 10000."""
    g = oracle.make_geometry(n, na, nd)
    rng = np.random.default_rng(n)
    truth = np.zeros((n, n))
    truth[2:n - 3, 3:n - 2] = 1.0
    truth[4:6, 4:7] = 0.0
    WL = oracle.sparse_local(g)
    b = WL @ truth.ravel() + 0.3 * rng.standard_normal(WL.shape[0])
    W = WL.toarray()
    rho = float(np.linalg.norm(W, 2) ** 2)
    f1 = oracle.cp_objective(WL, b, _admm_tv_nonneg(W, b, n, n, lam, rho=rho, iters=10000), lam)
    f2 = oracle.cp_objective(WL, b, _admm_tv_nonneg(W, b, n, n, lam, rho=rho / 10, iters=10000), lam)
    assert abs(f1 - f2) <= 1e-8 * f1
    s, t = oracle.cp_steps(WL, (n, n), iters=300)
    gaps = []
    x_cp = None

    def cb(it, x):
        nonlocal x_cp
        if it + 1 in (10000, 40000):
            gaps.append(oracle.cp_objective(WL, b, x, lam) - f1)
            x_cp = x
    oracle.cp_tv_nonneg(WL, b, (n, n), lam, s, t, 40000, callback=cb)
    assert x_cp.min() >= 0.0 and (x_cp == 0).sum() > 0          # nonnegativity active
    assert gaps[1] >= -1e-9 * f1                                  # ADMM found the minimum
    assert gaps[1] <= 3e-5 * f1, gaps
    assert gaps[1] * 4 <= gaps[0], gaps


def test_cp_unregularised_converges_to_exact_solution():
    """lambda = 0 and no prox: with consistent data and W_L of full column rank, CP
    converges to the unique solution (the phantom)."""
    g = oracle.make_geometry(32, 64, 48)
    rng = np.random.default_rng(5)
    truth = rng.random((8, 8))
    rect = (12, 12, 8, 8)
    WL = oracle.sparse_local(g, rect)
    b = WL @ truth.ravel()
    assert np.linalg.matrix_rank(WL.toarray()) == 64
    s, t = oracle.cp_steps(WL, (8, 8))
    x = oracle.cp_tv_nonneg(WL, b, (8, 8), 0.0, s, t, 5000, nonneg=False)
    assert np.abs(x - truth).max() < 1e-6


@pytest.mark.parametrize("half,aniso,lam,h", [(True, False, 1.5, 1.0), (False, True, 1.0, 1.0),
                                              (True, True, 0.5, 1.0), (False, False, 0.1875, 0.25)])
def test_cp_variants_converge_to_independent_admm_minimiser(half, aniso, lam, h):
    """The 1/2-data reading (prox of sigma F1* divides by 1 + sigma), the anisotropic
    reading of ||grad x||_1 (per-component clamp to [-lambda, lambda]) and a data length
    unit h != 1 (data term ||h W x - h b||^2) each converge to the minimiser of their own
    objective, found by ADMM with the matching data weight, operator and shrinkage
    (eq. priorsys with and without 1/2; Section 2.3, g = ||grad x||_1).  A swapped
    divisor, a wrong clamp bound or a dropped unit lands on another problem's minimiser:
    those minima differ by far more than the 3e-5 gap allowed here.  lambda is chosen
    per reading so that nonnegativity is active at the minimiser."""
    n, na, nd = 8, 6, 12
    g = oracle.make_geometry(n, na, nd)
    rng = np.random.default_rng(n)
    truth = np.zeros((n, n))
    truth[2:n - 3, 3:n - 2] = 1.0
    truth[4:6, 4:7] = 0.0
    WL = oracle.sparse_local(g)
    b = WL @ truth.ravel() + 0.3 * rng.standard_normal(WL.shape[0])
    W = WL.toarray()
    rho = float(np.linalg.norm(h * W, 2) ** 2)
    mins = {}
    for hh in (False, True):
        for aa in (False, True):
            for hu in {h, 1.0}:
                xa = _admm_tv_nonneg(hu * W, hu * b, n, n, lam, rho=rho, iters=10000, half=hh,
                                     aniso=aa)
                mins[hh, aa, hu] = xa
    xa = mins[half, aniso, h]
    f1 = oracle.cp_objective(WL, b, xa, lam, half=half, aniso=aniso, h=h)
    xa2 = _admm_tv_nonneg(h * W, h * b, n, n, lam, rho=rho / 10, iters=10000, half=half,
                          aniso=aniso)
    assert abs(oracle.cp_objective(WL, b, xa2, lam, half=half, aniso=aniso, h=h) - f1) <= 1e-8 * f1
    # the other readings' minimisers are clearly suboptimal for this objective
    for key, xo in mins.items():
        if key != (half, aniso, h):
            assert oracle.cp_objective(WL, b, xo, lam, half=half, aniso=aniso, h=h) - f1 > 1e-3 * f1
    s, t = oracle.cp_steps(WL, (n, n), iters=300, h=h)
    x = oracle.cp_tv_nonneg(WL, b, (n, n), lam, s, t, 40000, half=half, aniso=aniso, h=h)
    gap = oracle.cp_objective(WL, b, x, lam, half=half, aniso=aniso, h=h) - f1
    assert x.min() >= 0.0 and (x == 0).sum() > 0
    assert -1e-9 * f1 <= gap <= 3e-5 * f1, gap
    assert np.abs(x - xa).max() < 2e-2


def test_cp_dual_callback_sees_the_unprojected_dual():
    """dual_callback receives z + sigma grad xbar before the projection: on the first
    iteration (z = 0, xbar = 0) it is zero, on the second sigma grad(xbar_1); the
    projected dual never leaves the lambda-ball while the unprojected one does."""
    g = oracle.make_geometry(12, 8, 18)
    WL = oracle.sparse_local(g)
    truth = np.zeros((12, 12)); truth[3:9, 2:7] = 5.0
    b = WL @ truth.ravel()
    seen, xs = [], []
    oracle.cp_tv_nonneg(WL, b, (12, 12), 0.05, 0.05, 0.05, 30,
                        dual_callback=lambda it, z: seen.append(z.copy()),
                        callback=lambda it, x: xs.append(x.copy()))
    assert np.all(seen[0] == 0.0)
    xbar1 = 2 * xs[0]                        # x0 = 0, so xbar1 = 2 x1 - x0
    np.testing.assert_allclose(seen[1], 0.05 * oracle.grad(xbar1), rtol=0, atol=1e-15)
    assert max(np.hypot(z[0], z[1]).max() for z in seen) > 0.05


def test_cp_is_stable_under_data_perturbation():
    """A 1e-6 relative change of b moves the 100th iterate by <= 1e-5 relative:
    FP32-level input differences cannot be amplified past the 1e-3 parity bar."""
    g = oracle.make_geometry(64, 32, 96)
    rng = np.random.default_rng(6)
    truth = np.zeros((64, 64)); truth[10:50, 20:40] = 1.0
    WL = oracle.sparse_local(g)
    b = WL @ truth.ravel() + 0.5 * rng.standard_normal(WL.shape[0])
    s, t = oracle.cp_steps(WL, (64, 64))
    x1 = oracle.cp_tv_nonneg(WL, b, (64, 64), 5.0, s, t, 100)
    db = 1e-6 * np.linalg.norm(b) * rng.standard_normal(len(b)) / np.sqrt(len(b))
    x2 = oracle.cp_tv_nonneg(WL, b + db, (64, 64), 5.0, s, t, 100)
    assert np.linalg.norm(x2 - x1) <= 1e-5 * np.linalg.norm(x1)


def test_sirt_nonneg_reaches_nnls_solution():
    """Projected Landweber with alpha = 1/(N_theta N_d) converges to the
    nonnegative least-squares solution (compared with scipy's NNLS)."""
    g = oracle.make_geometry(6, 8, 10)
    rng = np.random.default_rng(7)
    WL = oracle.sparse_local(g)
    b = WL @ (rng.random(36) - 0.3) + 0.05 * rng.standard_normal(WL.shape[0])
    alpha = 1.0 / (8 * 10)
    x = oracle.sirt_nonneg(WL, b, (6, 6), alpha, 60000)
    ref, _ = sopt.nnls(WL.toarray(), b, maxiter=10000)
    assert np.abs(x.ravel() - ref).max() < 1e-8


def test_sirt_step_is_stable_for_workload_geometry():
    """alpha ||W_L||^2 < 2 for the 128-grid workload's local part (Landweber condition)."""
    import scipy.sparse.linalg as sla2
    g = oracle.make_geometry(128, 32, 192)
    WL = oracle.sparse_local(g, (32, 32, 64, 64))
    smax = sla2.svds(WL, k=1, return_singular_vectors=False)[0]
    assert smax ** 2 / (32 * 192) < 2.0
