"""Pins of the oracle's total-variation recovery (the TVAL3-style solver of
Section 4): the difference operator and its adjoint, the norm bound behind
the step size, closed forms, and optimality of the recovered block by the
problem's KKT conditions (independent of the iteration that found it)."""
import numpy as np

import synthvid as sv
from oracle import codec, cs, philox, tv


def test_grad_adjoint_and_norm():
    rng = np.random.default_rng(0)
    for b in (4, 16, 32):
        x = rng.standard_normal((b * b, 3))
        ph, pv = rng.standard_normal((b * b, 3)), rng.standard_normal((b * b, 3))
        dh, dv = tv.grad(x, b)
        lhs = np.sum(dh * ph + dv * pv)
        rhs = np.sum(x * tv.grad_adj(ph, pv, b))
        assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs))
        # ||D||^2: D^T D is the 2-D Neumann Laplacian, the sum of two 1-D
        # ones with eigenvalues 2 - 2 cos(k pi / b); largest 4 + 4 cos(pi / b) < 8
        dtd = np.stack([tv.grad_adj(*tv.grad(e[:, None], b), b)[:, 0]
                        for e in np.eye(b * b)], axis=1)
        nrm = np.max(np.linalg.eigvalsh(dtd))
        assert abs(nrm - (4 + 4 * np.cos(np.pi / b))) < 1e-9 and nrm < 8


def test_tv_closed_forms():
    b = 8
    assert np.all(tv.tv_norm(np.full((b * b, 2), 3.7), b) == 0)
    # a vertical edge of height h across the block: TV = h * b (one jump per row)
    X = np.zeros((b, b))
    X[:, 5:] = 2.5
    assert abs(tv.tv_norm(X.reshape(-1, 1), b)[0] - 2.5 * b) < 1e-12
    # a single pixel bump: four unit differences, two per neighbour pair;
    # pixel (i, j) interior: ||(x_{i,j+1}-x, x_{i+1,j}-x)|| = sqrt2, plus the
    # left and upper neighbours' differences of 1 each
    X = np.zeros((b, b))
    X[3, 3] = 1.0
    assert abs(tv.tv_norm(X.reshape(-1, 1), b)[0] - (np.sqrt(2) + 2.0)) < 1e-12


def _kkt_residuals(phi, y, x, nh, nv, lam, b):
    g = phi.T @ (phi @ x - y) + tv.grad_adj(nh, nv, b)
    dh, dv = tv.grad(x, b)
    mag = np.sqrt(dh * dh + dv * dv)
    nmag = np.sqrt(nh * nh + nv * nv)
    active = mag > 1e-6
    align = np.max(np.abs(np.where(active, nh - lam * dh / np.where(active, mag, 1), 0))
                   + np.abs(np.where(active, nv - lam * dv / np.where(active, mag, 1), 0)))
    # the multiplier of the last column/row difference is unconstrained by D
    # (it never enters D^T); only the interior pairs matter
    return np.max(np.abs(g)), np.max(nmag) - lam, align


def test_recovered_block_satisfies_kkt():
    """On a small problem, the iterate after many steps is the minimiser of
    lam TV(x) + 1/2 ||Phi x - y||^2: stationarity Phi^T(Phi x - y) + D^T nu = 0,
    dual feasibility ||nu_i|| <= lam, and nu_i = lam D_i x / ||D_i x|| on the
    pixels where D_i x != 0."""
    b, m = 4, 10
    q = philox.measurement_matrix_q(m, b * b, 21, 3)
    s_phi = philox.phi_scale(m)
    phi = s_phi * q.astype(np.float64)
    L, _, _ = cs.lipschitz(q, s_phi)
    X = np.zeros((b, b))
    X[:, 2:] = 3.0
    X[1, 1] = -2.0
    y = phi @ X.reshape(-1, 1)
    lam = np.array([0.05 * np.max(np.abs(phi.T @ y))])
    x, nh, nv = tv.recover(phi, y, lam, L, b, 60000, return_dual=True)
    stat, feas, align = _kkt_residuals(phi, y, x, nh, nv, lam[0], b)
    assert stat < 1e-7
    assert feas < 1e-7
    assert align < 1e-5
    # and its objective is below that of nearby perturbations
    f0 = tv.objective(phi, y, x, lam, b)[0]
    rng = np.random.default_rng(2)
    for _ in range(50):
        xp = x + 1e-3 * rng.standard_normal(x.shape)
        assert tv.objective(phi, y, xp, lam, b)[0] >= f0 - 1e-12


def test_zero_measurements_give_zero_and_lambda_rule():
    b, m = 8, 16
    q = philox.measurement_matrix_q(m, b * b, 1, 1)
    phi = philox.phi_scale(m) * q.astype(np.float64)
    y = np.zeros((m, 2))
    lam = tv.lambdas(phi, y, 0.01)
    assert np.all(lam == 0)
    x = tv.recover(phi, y, lam, 1.0, b, 20)
    assert np.all(x == 0)


def test_tv_decode_beats_dct_lasso_on_surveillance_video():
    """The reason the paper uses TVAL3: on piecewise-smooth surveillance
    residuals TV recovery is more accurate than l1 in the DCT basis at the
    same measurements (a property of this input family, checked loosely)."""
    spec = sv.qcif_tiny().with_(gop=2)
    frames = spec.video()
    p = codec.Params.from_spec(spec)
    gs = codec.encode_gop(frames, p)
    d_l1 = codec.decode_gop(gs, p)
    d_tv = codec.decode_gop(gs, codec.Params.from_spec(spec, solver="tv"))
    assert codec.psnr(frames[1], d_tv.frames[1]) > codec.psnr(frames[1], d_l1.frames[1]) + 1.0


def test_step_of_the_iteration_closed_form():
    """With Phi = I (L = 1) and lambda = 0 (beta = 1) the shrinkage is the
    identity, the multipliers stay zero, and the iteration is gradient
    descent on 1/2 ||x - y||^2 with the step alpha = 1 / (L + 8 beta) = 1/9:
    x_k = y (1 - (8/9)^k) exactly (up to rounding), for blocks and frames."""
    rng = np.random.default_rng(3)
    for b in (8, (6, 10)):
        hh, ww = (b, b) if isinstance(b, int) else b
        n = hh * ww
        y = rng.normal(0, 5.0, size=(n, 3))
        for k in (1, 2, 7):
            x = tv.recover(np.eye(n), y, np.zeros(3), 1.0, b, k)
            assert np.allclose(x, y * (1.0 - (8.0 / 9.0) ** k), rtol=0, atol=1e-12)
