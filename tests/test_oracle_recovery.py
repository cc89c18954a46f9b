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


def _t_sequence(count):
    """t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2 (Beck and Teboulle)."""
    t = [1.0]
    for _ in range(count):
        t.append((1.0 + np.sqrt(1.0 + 4.0 * t[-1] ** 2)) / 2.0)
    return t


def _kkt_problem(m, k, seed):
    """A sparse-recovery LASSO whose minimiser is the KKT closed form on the
    true support (certified), as in test_fista_matches_kkt_closed_form."""
    q, s_phi, a = _problem(m, 16, seed=m + k + seed)
    s_true = _sparse_dct_blocks(256, k, 5, seed=k + 7 * seed)
    y = a @ s_true
    lam = cs.lambdas(a, y)
    L, _, _ = cs.lipschitz(q, s_phi)
    s_star = np.zeros_like(s_true)
    for j in range(y.shape[1]):
        supp = np.flatnonzero(s_true[:, j])
        sg = np.sign(s_true[supp, j])
        s_s = _kkt_solution(a, y[:, j], lam[j], supp, sg)
        assert np.all(np.sign(s_s) == sg)
        resid = y[:, j] - a[:, supp] @ s_s
        off = np.setdiff1d(np.arange(256), supp)
        assert np.max(np.abs(a[:, off].T @ resid)) < lam[j]
        s_star[supp, j] = s_s
    return a, y, lam, L, s_star


@pytest.mark.parametrize("m,k,seed", [(64, 2, 0), (64, 4, 2), (128, 4, 2)])
def test_mfista_and_ista_match_kkt_closed_form(m, k, seed):
    """At convergence MFISTA and ISTA reach the certified KKT minimiser."""
    a, y, lam, L, s_star = _kkt_problem(m, k, seed)
    tol = 1e-10 * np.max(np.abs(s_star))
    assert np.max(np.abs(cs.mfista(a, y, lam, L, 3000) - s_star)) <= tol
    assert np.max(np.abs(cs.ista(a, y, lam, L, 60000) - s_star)) <= tol


@pytest.mark.parametrize("m,k,seed", [(64, 2, 0), (64, 4, 2), (128, 4, 2)])
def test_mfista_estimate_sequence_is_nonincreasing(m, k, seed):
    """MFISTA's convergence proof (Beck and Teboulle, IEEE TIP 2009, the
    monotone variant of FISTA's Lemma 4.1): with x* a minimiser, F* = F(x*),
    u_k = t_k z_k - (t_k - 1) s_{k-1} - x*, the quantity
    E_k = (2 / L) t_k^2 (F(s_k) - F*) + ||u_k||^2 never increases, and
    F(s_k) - F* <= 2 L ||x*||^2 / (k + 1)^2 (s_0 = 0).  The test also checks
    that the monotone branch (z_k rejected) is taken, so that the momentum
    coefficients of both branches are exercised.

    The proof chains these inequalities through its auxiliary sequence
    w_k = s_{k-1} + t_k (z_k - s_{k-1}): the next extrapolation point is
    v_{k+1} = (1 - 1 / t_{k+1}) s_k + w_k / t_{k+1}, which the test checks
    on every iteration (this is what fixes the coefficient of z_k - s_k,
    which only matters on rejected steps).  While no step is rejected MFISTA
    is FISTA, iterate for iterate."""
    a, y, lam, L, s_star = _kkt_problem(m, k, seed)
    f_star = cs.objective(a, y, s_star, lam)
    T = 400
    _, hist, its = cs.mfista(a, y, lam, L, T, history=True, iterates=True)
    t = _t_sequence(T)
    for kk in range(1, T):
        _, z, s = its[kk - 1]
        s_before = its[kk - 2][2] if kk > 1 else np.zeros_like(s)
        w = s_before + t[kk - 1] * (z - s_before)
        v_next = (1.0 - 1.0 / t[kk]) * s + w / t[kk]
        assert np.allclose(its[kk][0], v_next, rtol=0, atol=1e-12 * np.max(np.abs(s_star)))
    first_rej = next((i for i, (_, z, s) in enumerate(its) if np.any(z != s)), T)
    assert first_rej > 2
    s_f = cs.fista(a, y, lam, L, first_rej)
    assert np.allclose(its[first_rej - 1][2], s_f, rtol=0, atol=1e-12 * np.max(np.abs(s_star)))
    prev_s = np.zeros_like(s_star)
    e_prev = None
    rejected = 0
    for kk, (_, z, s) in enumerate(its, start=1):
        gap = cs.objective(a, y, s, lam) - f_star
        assert np.all(gap <= 2 * L * np.sum(s_star ** 2, axis=0) / (kk + 1) ** 2
                      * (1 + 1e-9) + 1e-9 * f_star)
        u = t[kk - 1] * z - (t[kk - 1] - 1.0) * prev_s - s_star
        e = (2.0 / L) * t[kk - 1] ** 2 * gap + np.sum(u * u, axis=0)
        if e_prev is not None:
            assert np.all(e <= e_prev * (1 + 1e-9) + 1e-9), kk
        rejected += int(np.sum(np.any(z != s, axis=0)))
        e_prev, prev_s = e, s
    assert rejected > 0


def test_fista_estimate_sequence_is_nonincreasing():
    """FISTA's Lemma 4.1 (Beck and Teboulle 2009): E_k = (2 / L) t_k^2
    (F(s_k) - F*) + ||t_k s_k - (t_k - 1) s_{k-1} - x*||^2 never increases."""
    a, y, lam, L, s_star = _kkt_problem(64, 4, 2)
    f_star = cs.objective(a, y, s_star, lam)
    T = 300
    t = _t_sequence(T)
    e_prev = None
    prev_s = np.zeros_like(s_star)
    for kk in range(1, T + 1):
        s = cs.fista(a, y, lam, L, kk)
        u = t[kk - 1] * s - (t[kk - 1] - 1.0) * prev_s - s_star
        e = (2.0 / L) * t[kk - 1] ** 2 * (cs.objective(a, y, s, lam) - f_star) + np.sum(u * u, 0)
        if e_prev is not None:
            assert np.all(e <= e_prev * (1 + 1e-9) + 1e-9), kk
        e_prev, prev_s = e, s


def test_ista_closed_form_on_orthogonal_columns():
    """ISTA on an operator with orthogonal columns, A = U diag(sigma)
    (U orthonormal): the gradient step decouples per coefficient, and where
    sigma_i c_i > lam (c = U^T y) every iterate stays on the active branch,
    so s_k = s*_i (1 - (1 - sigma_i^2 / L)^k) with s*_i = (sigma_i c_i -
    lam) / sigma_i^2 (and the mirror image for sigma_i c_i < -lam; zero
    where |sigma_i c_i| <= lam).  This fixes the step 1 / L."""
    rng = np.random.default_rng(12)
    n = 24
    u, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sigma = rng.uniform(0.5, 2.0, size=n)
    a = u * sigma[None, :]
    c = rng.normal(0, 5.0, size=(n, 3))
    y = u @ c
    lam = np.array([0.4, 1.1, 2.0])
    L = 1.3 * np.max(sigma) ** 2
    sc = sigma[:, None] * c
    s_star = np.sign(sc) * np.maximum(np.abs(sc) - lam[None, :], 0) / sigma[:, None] ** 2
    for k in (1, 2, 7, 40):
        want = s_star * (1 - (1 - sigma[:, None] ** 2 / L) ** k)
        assert np.allclose(cs.ista(a, y, lam, L, k), want, rtol=1e-12, atol=1e-12)
