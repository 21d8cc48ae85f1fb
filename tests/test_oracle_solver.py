"""Pins of the oracle's regulariser and solver pieces (paper Sec. 2.2).

D and D^T against Kronecker products and closed forms; the TV weights against
closed forms; the augmented system against the functional it encodes; LSQR
against SciPy's independent implementation and against its own invariants;
LSQR vs CGLS (mathematically equivalent, Sec. 2.2.2); the majorise-minimise
descent of IRN (Sec. 2.2.1); and the x_p fixed point.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def tiny(orc, nx=4, ny=3, nz=5, nu=6, nv=5, V=6):
    return orc.Geometry(nx=nx, ny=ny, nz=nz, vx=1.0, vy=1.0, vz=1.0, nu=nu, nv=nv, du=1.5,
                        dv=1.5, dso=30.0, dsd=50.0, n_views=V)


# ---------------------------------------------------------------- D, D^T

def _D1(n):
    """D_1 with rows (1, -1), padded with a zero last row to n x n."""
    m = sp.lil_matrix((n, n))
    for i in range(n - 1):
        m[i, i] = 1.0
        m[i, i + 1] = -1.0
    return m.tocsr()


def _dense_D(nx, ny, nz):
    # x is flattened with i fastest: index = (k*ny + j)*nx + i, so the x-difference
    # acts on the last Kronecker factor.
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    Dx = sp.kron(Iz, sp.kron(Iy, _D1(nx)))
    Dy = sp.kron(Iz, sp.kron(_D1(ny), Ix))
    Dz = sp.kron(_D1(nz), sp.kron(Iy, Ix))
    return sp.vstack([Dx, Dy, Dz]).tocsr()


def test_D_matches_kronecker(orc):
    nz, ny, nx = 5, 4, 6
    x = np.random.default_rng(1).normal(size=(nz, ny, nx))
    want = (_dense_D(nx, ny, nz) @ x.ravel()).reshape(3, nz, ny, nx)
    np.testing.assert_array_equal(orc.D(x), want)


def test_DT_matches_kronecker_transpose(orc):
    nz, ny, nx = 5, 4, 6
    y = np.random.default_rng(2).normal(size=(3, nz, ny, nx))
    want = (_dense_D(nx, ny, nz).T @ y.ravel()).reshape(nz, ny, nx)
    np.testing.assert_allclose(orc.DT(y), want, rtol=0, atol=1e-14)


def test_D_of_ramp(orc):
    nz, ny, nx = 4, 5, 6
    a, b, c = 0.3, -1.2, 2.5
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    g = orc.D(a * i + b * j + c * k + 0.7)
    assert np.allclose(g[0][:, :, :-1], -a) and np.all(g[0][:, :, -1] == 0)
    assert np.allclose(g[1][:, :-1, :], -b) and np.all(g[1][:, -1, :] == 0)
    assert np.allclose(g[2][:-1], -c) and np.all(g[2][-1] == 0)


def test_D_adjoint_identity(orc):
    rng = np.random.default_rng(3)
    x = rng.normal(size=(7, 6, 5))
    y = rng.normal(size=(3, 7, 6, 5))
    assert float(np.vdot(orc.D(x), y)) == pytest.approx(float(np.vdot(x, orc.DT(y))), rel=1e-14)


# ---------------------------------------------------------------- weights

def test_weights_closed_forms(orc):
    tau = 0.3
    x = np.full((4, 5, 6), 2.0)
    w1, w2 = orc.weights(x, x, tau)
    np.testing.assert_allclose(w1, 1.0 / tau, rtol=1e-15)   # zero gradient -> 1/tau
    np.testing.assert_allclose(w2, 1.0 / tau, rtol=1e-15)
    a, b, c = 0.5, -0.25, 1.5
    k, j, i = np.meshgrid(np.arange(4), np.arange(5), np.arange(6), indexing="ij")
    ramp = a * i + b * j + c * k
    w1, w2 = orc.weights(ramp, np.zeros_like(ramp), tau)
    want = 1.0 / math.sqrt(math.sqrt(a * a + b * b + c * c) + tau * tau)
    np.testing.assert_allclose(w1[:-1, :-1, :-1], want, rtol=1e-15)
    np.testing.assert_allclose(w2[:-1, :-1, :-1], want, rtol=1e-15)
    # at the far corner every difference is zero
    assert w1[-1, -1, -1] == pytest.approx(1.0 / tau, rel=1e-15)
    # W2 depends on x - x_p only
    w1b, w2b = orc.weights(ramp + 3.0, ramp, tau)
    np.testing.assert_allclose(w2b, 1.0 / tau, rtol=1e-15)


# ---------------------------------------------------------------- augmented system

def test_augmented_residual_is_the_piccs_functional(orc):
    g = tiny(orc)
    rng = np.random.default_rng(4)
    x = rng.uniform(size=g.vol_shape)
    xp = rng.uniform(size=g.vol_shape)
    xk = rng.uniform(size=g.vol_shape)
    b = rng.uniform(size=g.proj_shape)
    alpha, lam, tau = 0.7, 1.3, 0.2
    w1, w2 = orc.weights(xk, xp, tau)
    aug = orc.Augmented(g, alpha, lam, w1, w2)
    r = tuple(p - q for p, q in zip(aug.forward(x), aug.rhs(b, xp)))
    lhs = sum(float(np.vdot(p, p)) for p in r)
    Ax = orc.forward(g, x)
    rhs = (float(np.sum((Ax - b) ** 2)) + alpha ** 2 * float(np.sum((w1 * orc.D(x)) ** 2))
           + lam ** 2 * float(np.sum((w2 * orc.D(x - xp)) ** 2)))
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_augmented_adjoint(orc):
    g = tiny(orc)
    rng = np.random.default_rng(5)
    w1, w2 = rng.uniform(0.5, 2, size=(2,) + g.vol_shape)
    aug = orc.Augmented(g, 0.8, 1.7, w1, w2)
    x = rng.normal(size=g.vol_shape)
    u = (rng.normal(size=g.proj_shape), rng.normal(size=(3,) + g.vol_shape),
         rng.normal(size=(3,) + g.vol_shape))
    lhs = sum(float(np.vdot(p, q)) for p, q in zip(aug.forward(x), u))
    assert lhs == pytest.approx(float(np.vdot(x, aug.back(u))), rel=1e-12)


def _explicit(orc, g, alpha, lam, w1, w2, b, xp):
    """Sparse explicit A~ and stacked b~ built from the dense A and Kronecker D."""
    A = sp.csr_matrix(orc.dense_A(g))
    Dm = _dense_D(g.nx, g.ny, g.nz)
    W1 = sp.diags(np.tile(w1.ravel(), 3))
    W2 = sp.diags(np.tile(w2.ravel(), 3))
    At = sp.vstack([A, alpha * W1 @ Dm, lam * W2 @ Dm]).tocsr()
    bt = np.concatenate([b.ravel(), np.zeros(Dm.shape[0]), lam * (W2 @ Dm @ xp.ravel())])
    return At, bt


def _problem(orc, seed=6):
    g = tiny(orc)
    rng = np.random.default_rng(seed)
    xp = rng.uniform(size=g.vol_shape)
    x0 = xp + 0.1 * rng.normal(size=g.vol_shape)
    b = orc.forward(g, xp + 0.2 * rng.uniform(size=g.vol_shape))
    alpha, lam, tau = 0.6, 1.1, 0.3
    w1, w2 = orc.weights(x0, xp, tau)
    return g, xp, x0, b, alpha, lam, tau, w1, w2


def test_lsqr_matches_scipy(orc):
    g, xp, x0, b, alpha, lam, tau, w1, w2 = _problem(orc)
    aug = orc.Augmented(g, alpha, lam, w1, w2)
    At, bt = _explicit(orc, g, alpha, lam, w1, w2, b, xp)
    for k in (1, 3, 8):
        mine = orc.lsqr(aug.forward, aug.back, aug.rhs(b, xp), x0, k)
        ref = spla.lsqr(At, bt, atol=0.0, btol=0.0, conlim=0.0, iter_lim=k, x0=x0.ravel())
        assert ref[2] == k
        np.testing.assert_allclose(mine.x.ravel(), ref[0], rtol=1e-10, atol=1e-12)


def test_lsqr_phibar_is_residual_norm_and_monotone(orc):
    g, xp, x0, b, alpha, lam, tau, w1, w2 = _problem(orc)
    aug = orc.Augmented(g, alpha, lam, w1, w2)
    At, bt = _explicit(orc, g, alpha, lam, w1, w2, b, xp)
    res = orc.lsqr(aug.forward, aug.back, aug.rhs(b, xp), x0, 12)
    assert len(res.phibar) == 12
    for k in range(1, 13):
        xk = orc.lsqr(aug.forward, aug.back, aug.rhs(b, xp), x0, k).x
        true = float(np.linalg.norm(At @ xk.ravel() - bt))
        assert res.phibar[k - 1] == pytest.approx(true, rel=1e-10)
    assert all(res.phibar[i + 1] <= res.phibar[i] * (1 + 1e-12) for i in range(11))


def test_lsqr_with_reorth_reaches_least_squares_solution(orc):
    g, xp, x0, b, alpha, lam, tau, w1, w2 = _problem(orc)
    aug = orc.Augmented(g, alpha, lam, w1, w2)
    At, bt = _explicit(orc, g, alpha, lam, w1, w2, b, xp)
    M = g.nx * g.ny * g.nz
    res = orc.lsqr(aug.forward, aug.back, aug.rhs(b, xp), x0, M, reorth=True)
    ref = np.linalg.lstsq(At.toarray(), bt, rcond=None)[0]
    np.testing.assert_allclose(res.x.ravel(), ref, rtol=1e-8, atol=1e-8)


def test_lsqr_equals_cgls(orc):
    from paper_2509_08574_amd import synth
    g = orc.Geometry(nx=24, ny=24, nz=20, vx=1.0, vy=1.0, vz=1.0, nu=36, nv=30, du=1.5,
                     dv=1.5, dso=200.0, dsd=320.0, n_views=16)
    rng = np.random.default_rng(8)
    xp, _ = synth.ellipsoid_phantom(g.vol_shape, 5, (2.0, 8.0), 9)
    b = orc.forward(g, xp + 0.05 * rng.uniform(size=g.vol_shape))
    w1, w2 = orc.weights(xp, xp, 0.2)
    aug = orc.Augmented(g, 0.5, 1.0, w1, w2)
    bt = aug.rhs(b, xp)
    for k in (5, 15):
        xl = orc.lsqr(aug.forward, aug.back, bt, xp, k).x
        xc, _ = orc.cgls(aug.forward, aug.back, bt, xp, k)
        assert np.linalg.norm(xl - xc) <= 1e-9 * np.linalg.norm(xl)


# ---------------------------------------------------------------- IRN

def test_irn_objective_descends_with_exact_inner_solves(orc):
    g, xp, x0, b, alpha, lam, tau, _, _ = _problem(orc, seed=12)
    M = g.nx * g.ny * g.nz
    res = orc.irn_piccs(g, b, xp, x0, alpha, lam, tau, n_outer=5, n_inner=M, reorth=True,
                        keep_iterates=True)
    F = [orc.irn_objective(g, x0, b, xp, alpha, lam, tau)]
    F += [orc.irn_objective(g, xk, b, xp, alpha, lam, tau) for xk in res.outer]
    assert all(F[k + 1] <= F[k] * (1 + 1e-12) for k in range(len(F) - 1)), F
    assert F[-1] < F[0]


def test_irn_psi_is_integral_of_squared_weight(orc):
    tau = 0.35
    s = np.linspace(0.01, 4.0, 50)
    h = 1e-6
    dpsi = (orc.psi(s + h, tau) - orc.psi(s - h, tau)) / (2 * h)
    np.testing.assert_allclose(dpsi, 1.0 / (np.sqrt(s) + tau * tau), rtol=1e-7)
    assert orc.psi(np.array([0.0]), tau)[0] == 0.0


def test_prior_is_a_fixed_point(orc):
    g = tiny(orc)
    xp = np.random.default_rng(13).uniform(size=g.vol_shape)
    b = orc.forward(g, xp)
    res = orc.irn_piccs(g, b, xp, xp, 0.0, 1.5, 0.2, n_outer=2, n_inner=4)
    assert np.array_equal(res.x, xp)
    assert res.breakdown


def test_irn_reduces_to_plain_lsqr_without_regularisation(orc):
    g, xp, x0, b, _, _, tau, _, _ = _problem(orc, seed=14)
    res = orc.irn_piccs(g, b, xp, x0, 0.0, 0.0, tau, n_outer=1, n_inner=6)
    A = sp.csr_matrix(orc.dense_A(g))
    ref = spla.lsqr(A, b.ravel(), atol=0, btol=0, conlim=0, iter_lim=6, x0=x0.ravel())[0]
    np.testing.assert_allclose(res.x.ravel(), ref, rtol=1e-10, atol=1e-12)


def test_irn_converges_to_a_stationary_point_of_F(orc):
    """MM with exact inner solves converges to a point where grad F = 0.

    grad F(x) = 2 A^T(Ax - b) + 2 alpha^2 D^T(psi'(|Dx|^2) Dx)
                + 2 lambda^2 D^T(psi'(|D(x-x_p)|^2) D(x-x_p)),  psi'(s) = 1/(sqrt(s)+tau^2).
    """
    g, xp, x0, b, alpha, lam, tau, _, _ = _problem(orc, seed=15)
    M = g.nx * g.ny * g.nz

    def grad(x):
        g1 = orc.D(x)
        g2 = orc.D(x - xp)
        p1 = 1.0 / (np.sqrt((g1 ** 2).sum(0)) + tau * tau)
        p2 = 1.0 / (np.sqrt((g2 ** 2).sum(0)) + tau * tau)
        return 2 * (orc.back(g, orc.forward(g, x) - b, nthreads=1)
                    + alpha ** 2 * orc.DT(p1[None] * g1) + lam ** 2 * orc.DT(p2[None] * g2))

    res = orc.irn_piccs(g, b, xp, x0, alpha, lam, tau, n_outer=60, n_inner=M, reorth=True)
    assert np.linalg.norm(grad(res.x)) < 1e-6 * np.linalg.norm(grad(x0))


# ---------------------------------------------------------------- IRN-PIPLE (eq. seq_W_2)

def test_piple_augmented_residual_and_adjoint(orc):
    """||A~x - b~||^2 is the PIPLE quadratic of eq. seq_W_2, and A~^T is its adjoint."""
    g = tiny(orc)
    rng = np.random.default_rng(21)
    x, xp, xk = rng.uniform(size=(3,) + g.vol_shape)
    b = rng.uniform(size=g.proj_shape)
    alpha, lam, tau = 0.7, 1.3, 0.2
    w1 = orc.weight_of_gradient(orc.D(xk), tau)
    aug = orc.AugmentedPiple(g, alpha, lam, w1)
    r = tuple(p - q for p, q in zip(aug.forward(x), aug.rhs(b, xp)))
    lhs = sum(float(np.vdot(p, p)) for p in r)
    rhs = (float(np.sum((orc.forward(g, x) - b) ** 2))
           + alpha ** 2 * float(np.sum((w1 * orc.D(x)) ** 2))
           + lam ** 2 * float(np.sum((x - xp) ** 2)))
    assert lhs == pytest.approx(rhs, rel=1e-13)
    u = (rng.normal(size=g.proj_shape), rng.normal(size=(3,) + g.vol_shape),
         rng.normal(size=g.vol_shape))
    lhs = sum(float(np.vdot(p, q)) for p, q in zip(aug.forward(x), u))
    assert lhs == pytest.approx(float(np.vdot(x, aug.back(u))), rel=1e-12)


def test_piple_without_tv_is_tikhonov_towards_the_prior(orc):
    """alpha = 0: one outer step solved to convergence is the solution of the
    normal equations (A^T A + lambda^2 I) x = A^T b + lambda^2 x_p."""
    g, xp, x0, b, _, lam, tau, _, _ = _problem(orc, seed=22)
    M = g.nx * g.ny * g.nz
    A = orc.dense_A(g)
    x_ref = np.linalg.solve(A.T @ A + lam ** 2 * np.eye(M), A.T @ b.ravel() + lam ** 2 * xp.ravel())
    res = orc.irn_piple(g, b, xp, x0, 0.0, lam, tau, 1, 2 * M, reorth=True)
    np.testing.assert_allclose(res.x.ravel(), x_ref, rtol=1e-9, atol=1e-10)


def test_piple_with_lambda_zero_is_irn_tv(orc):
    g, xp, x0, b, alpha, _, tau, _, _ = _problem(orc, seed=23)
    a = orc.irn_piple(g, b, xp, x0, alpha, 0.0, tau, 2, 5)
    c = orc.irn_piccs(g, b, xp, x0, alpha, 0.0, tau, 2, 5)
    np.testing.assert_allclose(a.x, c.x, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(a.phibar, c.phibar, rtol=1e-12)


def test_piple_objective_descends_and_reaches_stationarity(orc):
    """Majorise-minimise: F decreases every outer step, and with exact inner
    solves the iterates reach grad F = 0, where
    grad F(x) = 2 A^T(Ax - b) + 2 alpha^2 D^T(psi'(|Dx|^2) Dx) + 2 lambda^2 (x - x_p)."""
    g, xp, x0, b, alpha, lam, tau, _, _ = _problem(orc, seed=24)
    M = g.nx * g.ny * g.nz
    res = orc.irn_piple(g, b, xp, x0, alpha, lam, tau, n_outer=8, n_inner=M, reorth=True,
                        keep_iterates=True)
    F = [orc.piple_objective(g, x0, b, xp, alpha, lam, tau)]
    F += [orc.piple_objective(g, x, b, xp, alpha, lam, tau) for x in res.outer]
    assert all(b_ <= a_ * (1 + 1e-12) for a_, b_ in zip(F, F[1:]))

    def grad(x):
        g1 = orc.D(x)
        p1 = 1.0 / (np.sqrt((g1 ** 2).sum(0)) + tau * tau)
        return 2 * (orc.back(g, orc.forward(g, x) - b, nthreads=1)
                    + alpha ** 2 * orc.DT(p1[None] * g1) + lam ** 2 * (x - xp))

    res = orc.irn_piple(g, b, xp, x0, alpha, lam, tau, n_outer=60, n_inner=M, reorth=True)
    assert np.linalg.norm(grad(res.x)) < 1e-6 * np.linalg.norm(grad(x0))
