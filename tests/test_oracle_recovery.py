"""Pins of the oracle's decoder: DCT basis, step constant, lambda and the
l1 recovery of eq. (1) read as a LASSO solved by FISTA.  FISTA is pinned to
the LASSO optimality conditions (closed form on the support), to brute-force
support enumeration on a tiny problem, to scikit-learn's coordinate-descent
Lasso, to ISTA/MFISTA monotonicity and to FISTA's O(1/k^2) rate bound."""
import itertools

import numpy as np
import pytest
from scipy.fft import dctn, idctn

from oracle import cs, philox


def _problem(m, b, seed=0):
    n = b * b
    q = philox.measurement_matrix_q(m, n, 0x1311141900010000 + seed, seed)
    s_phi = philox.phi_scale(m)
    return q, s_phi, cs.operator(q, s_phi, b)


def test_basis_matches_scipy_idct():
    rng = np.random.default_rng(0)
    for b in (4, 16, 32):
        s = rng.standard_normal((b, b))
        psi = cs.synthesis_basis(b)
        assert np.allclose((psi @ s.reshape(-1)).reshape(b, b), idctn(s, norm="ortho"), atol=1e-12)
        assert np.allclose(psi.T @ psi, np.eye(b * b), atol=1e-12)
        assert np.allclose(cs.synthesise(s.reshape(-1, 1), b)[:, 0].reshape(b, b),
                           idctn(s, norm="ortho"), atol=1e-12)


def test_operator_rows_are_dct_of_phi_rows():
    q, s_phi, a = _problem(8, 16)
    for i in range(8):
        row = dctn((s_phi * q[i]).reshape(16, 16).astype(np.float64), norm="ortho").reshape(-1)
        assert np.allclose(a[i], row, atol=1e-12)


@pytest.mark.parametrize("m,n", [(13, 256), (64, 256), (128, 256), (256, 1024), (410, 1024)])
def test_lipschitz_vs_eigvalsh(m, n):
    q = philox.measurement_matrix_q(m, n, 17, 3)
    s_phi = philox.phi_scale(m)
    L, rq, it = cs.lipschitz(q, s_phi)
    g = q.astype(np.float64) @ q.T.astype(np.float64)
    lmax = np.linalg.eigvalsh(g)[-1]
    assert abs(rq - lmax) <= 1e-9 * lmax
    assert L == pytest.approx(1.001 * s_phi**2 * lmax, rel=1e-9)
    # Marchenko-Pastur edge: ||Phi||^2 ~ (1 + sqrt(n/M))^2 for Var = 1/M
    mp = (1 + np.sqrt(n / m)) ** 2
    assert 0.85 * mp < s_phi**2 * lmax < 1.1 * mp


def _kkt_solution(a, y, lam, support, signs):
    a_s = a[:, support]
    s_s = np.linalg.solve(a_s.T @ a_s, a_s.T @ y - lam * signs)
    return s_s


def _sparse_dct_blocks(n, k, nb, seed):
    rng = np.random.default_rng(seed)
    s = np.zeros((n, nb))
    for j in range(nb):
        idx = rng.choice(n, size=k, replace=False)
        s[idx, j] = rng.choice([-1, 1], size=k) * rng.uniform(20, 60, size=k)
    return s


@pytest.mark.parametrize("m,k", [(64, 2), (64, 4), (128, 4)])
def test_fista_matches_kkt_closed_form(m, k):
    q, s_phi, a = _problem(m, 16, seed=m + k)
    s_true = _sparse_dct_blocks(256, k, 6, seed=k)
    y = a @ s_true
    lam = cs.lambdas(a, y)
    L, _, _ = cs.lipschitz(q, s_phi)
    s_hat = cs.fista(a, y, lam, L, 3000)
    for j in range(y.shape[1]):
        supp = np.flatnonzero(s_true[:, j])
        sg = np.sign(s_true[supp, j])
        s_s = _kkt_solution(a, y[:, j], lam[j], supp, sg)
        assert np.all(np.sign(s_s) == sg)
        resid = y[:, j] - a[:, supp] @ s_s
        off = np.setdiff1d(np.arange(256), supp)
        assert np.max(np.abs(a[:, off].T @ resid)) < lam[j]      # certificate
        full = np.zeros(256); full[supp] = s_s
        assert np.max(np.abs(s_hat[:, j] - full)) <= 1e-10 * np.max(np.abs(full))


def test_exact_recovery_support_and_debiased_values():
    q, s_phi, a = _problem(64, 16, seed=3)
    s_true = _sparse_dct_blocks(256, 4, 8, seed=9)
    y = a @ s_true
    lam = cs.lambdas(a, y)
    L, _, _ = cs.lipschitz(q, s_phi)
    s_hat = cs.fista(a, y, lam, L, 3000)
    for j in range(8):
        supp = np.flatnonzero(np.abs(s_hat[:, j]) > 1e-6)
        assert np.array_equal(supp, np.flatnonzero(s_true[:, j]))
        deb = np.linalg.lstsq(a[:, supp], y[:, j], rcond=None)[0]
        assert np.max(np.abs(deb - s_true[supp, j])) <= 1e-10 * np.max(np.abs(s_true[:, j]))


def test_brute_force_support_enumeration_tiny():
    m, b = 8, 4
    q, s_phi, a = _problem(m, b, seed=21)
    n = b * b
    s_true = np.zeros(n); s_true[[3, 10]] = [25.0, -18.0]
    y = a @ s_true + np.random.default_rng(4).normal(0, 0.05, m)
    lam = 0.1 * np.max(np.abs(a.T @ y))
    found = []
    for size in range(0, 5):
        for supp in itertools.combinations(range(n), size):
            supp = list(supp)
            a_s = a[:, supp]
            if size and np.linalg.matrix_rank(a_s) < size:
                continue
            for sg in itertools.product((-1.0, 1.0), repeat=size):
                sg = np.array(sg)
                s_s = _kkt_solution(a, y, lam, supp, sg) if size else np.zeros(0)
                if size and not np.all(np.sign(s_s) == sg):
                    continue
                resid = y - a_s @ s_s if size else y
                off = np.setdiff1d(np.arange(n), supp)
                if np.max(np.abs(a[:, off].T @ resid)) <= lam:
                    full = np.zeros(n); full[supp] = s_s
                    found.append(full)
    assert len(found) == 1
    L, _, _ = cs.lipschitz(q, s_phi)
    s_hat = cs.fista(a, y[:, None], np.array([lam]), L, 20000)[:, 0]
    assert np.max(np.abs(s_hat - found[0])) <= 1e-9 * max(1.0, np.abs(found[0]).max())


def test_objective_matches_sklearn_lasso():
    from sklearn.linear_model import Lasso
    q, s_phi, a = _problem(32, 8, seed=5)
    rng = np.random.default_rng(6)
    for trial in range(3):
        y = rng.normal(0, 3.0, size=32)
        lam = 0.05 * np.max(np.abs(a.T @ y))
        L, _, _ = cs.lipschitz(q, s_phi)
        s_hat = cs.fista(a, y[:, None], np.array([lam]), L, 20000)[:, 0]
        model = Lasso(alpha=lam / 32, fit_intercept=False, tol=1e-14, max_iter=200000)
        model.fit(a, y)
        f_ours = cs.objective(a, y[:, None], s_hat[:, None], np.array([lam]))[0]
        f_sk = cs.objective(a, y[:, None], model.coef_[:, None], np.array([lam]))[0]
        assert f_ours <= f_sk * (1 + 1e-9)
        assert abs(f_ours - f_sk) <= 1e-9 * f_sk


def test_objective_orthonormal_closed_form():
    """With an orthonormal operator (A = I) the LASSO minimiser is soft(y,
    lam), and the minimal objective is the Huber function of y:
    sum_i y_i^2 / 2 where |y_i| <= lam, else lam |y_i| - lam^2 / 2."""
    rng = np.random.default_rng(11)
    n, nb = 64, 5
    a = np.eye(n)
    y = rng.normal(0, 2.0, size=(n, nb))
    lam = rng.uniform(0.3, 2.5, size=nb)
    s = cs.soft(y, lam[None, :])
    ay = np.abs(y)
    huber = np.where(ay <= lam[None, :], 0.5 * y * y, lam[None, :] * ay - 0.5 * lam[None, :] ** 2)
    assert np.allclose(cs.objective(a, y, s, lam), huber.sum(axis=0), rtol=1e-13, atol=0)
    # FISTA with L = 1 reaches that minimiser in one step from zero
    assert np.allclose(cs.fista(a, y, lam, 1.0, 5), s, rtol=0, atol=1e-12)


def test_round_to_u8_ties_to_even_and_clips():
    """Synthesis rounding reading: round half to even, then clip to [0, 255]."""
    f = np.array([0.5, 1.5, 2.5, 3.49999, -0.5, -3.0, 254.5, 255.5, 300.0, 127.5])
    assert cs.round_to_u8(f).tolist() == [0, 2, 2, 3, 0, 0, 254, 255, 255, 128]


def test_ista_and_mfista_monotone_fista_rate_bound():
    q, s_phi, a = _problem(64, 16, seed=8)
    rng = np.random.default_rng(8)
    y = rng.normal(0, 50.0, size=(64, 10))
    lam = cs.lambdas(a, y)
    L, _, _ = cs.lipschitz(q, s_phi)
    for solver in (cs.ista, cs.mfista):
        _, hist = solver(a, y, lam, L, 300, history=True)
        h = np.array(hist)
        assert np.all(np.diff(h, axis=0) <= 1e-12 * np.abs(h[:-1]))
    s_star = cs.mfista(a, y, lam, L, 20000)
    f_star = cs.objective(a, y, s_star, lam)
    _, hist = cs.fista(a, y, lam, L, 300, history=True)
    for k, fk in enumerate(hist, start=1):
        bound = 2 * L * np.sum(s_star ** 2, axis=0) / (k + 1) ** 2
        assert np.all(fk - f_star <= bound * (1 + 1e-9) + 1e-9 * f_star)


def test_zero_measurements_give_zero_and_scaling_is_exact():
    q, s_phi, a = _problem(64, 16, seed=2)
    L, _, _ = cs.lipschitz(q, s_phi)
    y0 = np.zeros((64, 3))
    lam0 = cs.lambdas(a, y0)
    assert np.all(lam0 == 0) and np.all(cs.fista(a, y0, lam0, L, 50) == 0)
    y = np.random.default_rng(3).normal(0, 10, size=(64, 4))
    s1 = cs.fista(a, y, cs.lambdas(a, y), L, 100)
    s2 = cs.fista(a, 2 * y, cs.lambdas(a, 2 * y), L, 100)
    assert np.array_equal(s2, 2 * s1)       # soft(2u, 2t) = 2 soft(u, t), exact in binary FP


def test_lambda_pixel_domain_reading():
    q, s_phi, a = _problem(64, 16, seed=1)
    y = np.random.default_rng(5).normal(0, 10, size=(64, 3))
    phi = s_phi * q.astype(np.float64)
    lam_pix = cs.lambdas(a, y, pixel_domain=True, phi=phi)
    assert np.allclose(lam_pix, 0.01 * np.max(np.abs(phi.T @ y), axis=0))
    # orthonormal Psi preserves the 2-norm of A^T y, not its max
    assert np.allclose(np.linalg.norm(a.T @ y, axis=0), np.linalg.norm(phi.T @ y, axis=0))
