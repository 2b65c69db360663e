"""Pins of the oracle's solvers and hypergradient (CPU only).

  lower_solve:  closed-form Fourier solution (periodic, quadratic R),
                dense normal equations (zero boundary, quadratic R),
                dense-Hessian Newton limit plus the a-posteriori bound of
                Lemma 2 (TV), the alpha = 0 / delta-kernel special case, the
                stop certificate recomputed by torch autograd, backtracking.
  adjoint_solve: dense solve with the autograd Hessian, exact iteration
                counts, the not-positive-definite error path.
  hypergrad:    dense implicit-function route of Eq. (3.2) with autograd
                Jacobians, central finite differences of F(theta) with tight
                solves, and the bilinear identity tying it to scipy's
                convolution.
"""
import numpy as np
import pytest
import scipy.signal as ss
import torch

import oracle as O
import _ref_torch as R
from paper_2502_09758_amd import synth

rng = np.random.default_rng(11)


def small_instance(C=1, H=16, W=16, K=5, alpha=2e-3, seed=5):
    inst = synth.make("cfg1", H=H, W=W, C=C, K=K, seed=seed)
    p = O.Problem(C, H, W, K, alpha=alpha, eps_tv=1e-2, beta=0.5 * alpha)
    return inst, p


# ----------------------------------------------------------------------------- lower level
def test_lower_solve_periodic_quadratic_fourier_closed_form():
    C, H, W, K, alpha = 1, 16, 12, 5, 0.05
    p = O.Problem(C, H, W, K, alpha=alpha, periodic=True, reg=2)
    th = synth.gaussian_kernel(K, 1.0)
    y = rng.standard_normal((C, H, W))
    x, info, _ = O.lower_solve(p, th, y, np.zeros((C, H, W)), tol=1e-12, max_iter=20000)
    assert info["status"] == O.OK
    c0 = (K - 1) // 2
    kp = np.zeros((H, W))
    for u in range(K):
        for v in range(K):
            kp[(u - c0) % H, (v - c0) % W] = th[u, v]
    kh = np.fft.fft2(kp)
    dh2 = (2 - 2 * np.cos(2 * np.pi * np.arange(W) / W))[None, :]
    dv2 = (2 - 2 * np.cos(2 * np.pi * np.arange(H) / H))[:, None]
    xhat = np.real(np.fft.ifft2(np.conj(kh) * np.fft.fft2(y[0]) / (np.abs(kh) ** 2 + alpha * (dh2 + dv2))))
    assert np.linalg.norm(x[0] - xhat) <= 1e-9 * np.linalg.norm(xhat)


def _conv_matrix(th, H, W):
    N = H * W
    M = np.zeros((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1
        M[:, k] = ss.convolve2d(e.reshape(H, W), th, mode="same").ravel()
    return M


def _diff_matrices(H, W):
    N = H * W
    Dh = np.zeros((N, N))
    Dv = np.zeros((N, N))
    for i in range(H):
        for j in range(W):
            k = i * W + j
            if j < W - 1:
                Dh[k, k], Dh[k, k + 1] = -1, 1
            if i < H - 1:
                Dv[k, k], Dv[k, k + W] = -1, 1
    return Dh, Dv


def test_lower_solve_zero_boundary_quadratic_dense():
    H, W, K, alpha = 16, 16, 5, 0.02
    p = O.Problem(1, H, W, K, alpha=alpha, reg=2)
    th = synth.gaussian_kernel(K, 1.2)
    y = rng.standard_normal((1, H, W))
    A = _conv_matrix(th, H, W)
    Dh, Dv = _diff_matrices(H, W)
    xhat = np.linalg.solve(A.T @ A + alpha * (Dh.T @ Dh + Dv.T @ Dv), A.T @ y.ravel())
    x, info, _ = O.lower_solve(p, th, y, np.zeros_like(y), tol=1e-12, max_iter=50000)
    assert info["status"] == O.OK
    assert np.linalg.norm(x.ravel() - xhat) <= 1e-9 * np.linalg.norm(xhat)


@pytest.mark.parametrize("C,reg", [(1, 0), (3, 0), (3, 1)])
def test_lower_solve_tv_newton_limit_and_lemma2(C, reg):
    inst, p = small_instance(C=C)
    p.reg = reg
    th = inst.a
    x, info, _ = O.lower_solve(p, th, inst.y, inst.y, tol=1e-10, max_iter=100000)
    assert info["status"] == O.OK
    tt, ty = R.t(th), R.t(inst.y)
    xhat = R.newton_solve(tt, ty, R.t(inst.y), p.alpha, p.eps_tv, reg)
    # Lemma 2: ||x - xhat|| <= ||grad h(x)|| / mu with mu the smallest Hessian
    # eigenvalue along the segment (taken at both ends, min, with margin)
    g_here = R.grad_h(tt, ty, R.t(x), p.alpha, p.eps_tv, reg).norm().item()
    lam = min(torch.linalg.eigvalsh(R.hess_h(tt, ty, R.t(v), p.alpha, p.eps_tv, reg)).min().item()
              for v in (x, xhat.numpy()))
    err = np.linalg.norm(x - xhat.numpy())
    assert g_here <= 1e-10 * 1.0001
    assert err <= g_here / lam * 1.5 + 1e-13
    assert err <= 1e-6 * np.linalg.norm(xhat.numpy())


def test_lower_solve_stop_certificate_independent():
    inst, p = small_instance(C=3, H=20, W=17, K=7)
    x, info, _ = O.lower_solve(p, inst.a, inst.y, inst.y, tol=1e-4, max_iter=3000)
    assert info["status"] == O.OK and info["iters"] > 0
    gn = R.grad_h(R.t(inst.a), R.t(inst.y), R.t(x), p.alpha, p.eps_tv).norm().item()
    assert gn <= 1e-4 * (1 + 1e-9)
    assert abs(gn - info["res_norm"]) <= 1e-10
    assert abs(info["obj"] - float(R.h(R.t(inst.a), R.t(inst.y), R.t(x), p.alpha, p.eps_tv))) < 1e-11


def test_lower_solve_identity_kernel_alpha_zero_returns_data():
    C, H, W, K = 2, 9, 7, 3
    p = O.Problem(C, H, W, K, alpha=0.0)
    th = np.zeros((K, K))
    th[1, 1] = 1.0
    y = rng.standard_normal((C, H, W))
    x, info, _ = O.lower_solve(p, th, y, np.zeros_like(y), tol=1e-14, max_iter=100, L=1.0)
    np.testing.assert_allclose(x, y, atol=1e-14)


def test_lower_solve_backtracking_and_replay():
    inst, p = small_instance(C=1, H=24, W=24, K=7)
    x0 = inst.y.copy()
    x, info, trace = O.lower_solve(p, inst.a, inst.y, x0, tol=1e-6, max_iter=2000, L=1e-3)
    assert info["status"] == O.OK
    assert trace.sum() == info["backtracks"] > 0
    # L stays within a factor 2 of a global Lipschitz bound of grad h
    Lbound = np.abs(inst.a).sum() ** 2 + 8 * p.alpha / p.eps_tv
    assert 1e-3 * 2 ** info["backtracks"] == pytest.approx(info["L"])
    assert info["L"] <= 2 * Lbound
    # replaying the recorded decisions gives the same iterate, bit for bit
    xr, ir, tr = O.lower_solve(p, inst.a, inst.y, x0, tol=1e-6, max_iter=info["iters"], L=1e-3,
                               replay_bt=trace)
    np.testing.assert_array_equal(xr, x)
    np.testing.assert_array_equal(tr, trace)
    assert ir["L"] == info["L"]


def test_lower_solve_maxiter_status():
    inst, p = small_instance()
    x, info, _ = O.lower_solve(p, inst.a, inst.y, inst.y, tol=1e-14, max_iter=3)
    assert info["status"] == O.MAXITER and info["iters"] == 3


# ----------------------------------------------------------------------------- adjoint (CG)
@pytest.mark.parametrize("C", [1, 3])
def test_adjoint_solve_matches_dense(C):
    inst, p = small_instance(C=C)
    x, _, _ = O.lower_solve(p, inst.a, inst.y, inst.y, tol=1e-8, max_iter=50000)
    tt, ty, tx = R.t(inst.a), R.t(inst.y), R.t(x)
    Hm = R.hess_h(tt, ty, tx, p.alpha, p.eps_tv).numpy()
    b = rng.standard_normal(p.N)
    qhat = np.linalg.solve(Hm, b)
    q, info = O.adjoint_solve(p, inst.a, x, b.reshape(p.shape), tol=1e-11, max_iter=20 * p.N)
    assert info["status"] == O.OK
    assert np.linalg.norm(q.ravel() - qhat) <= 1e-7 * np.linalg.norm(qhat)
    assert info["true_res"] <= 1e-9
    # oracle Hessian-vector product equals the dense autograd Hessian
    d = rng.standard_normal(p.N)
    np.testing.assert_allclose(O.h_hvp(p, inst.a, x, d.reshape(p.shape)).ravel(), Hm @ d, rtol=1e-10, atol=1e-10)


def test_adjoint_solve_fixed_iterations_and_warm_start():
    inst, p = small_instance()
    b = rng.standard_normal(p.shape)
    q5, i5 = O.adjoint_solve(p, inst.a, inst.y, b, tol=0.0, max_iter=5)
    assert i5["status"] == O.MAXITER and i5["iters"] == 5
    # warm start from the solution: zero iterations
    qt, it = O.adjoint_solve(p, inst.a, inst.y, b, tol=1e-10, max_iter=5000)
    qw, iw = O.adjoint_solve(p, inst.a, inst.y, b, q0=qt, tol=1e-8, max_iter=10)
    assert iw["iters"] == 0 and np.array_equal(qw, qt)


def test_adjoint_solve_not_spd():
    H, W, K = 8, 8, 3
    p = O.Problem(1, H, W, K, alpha=-5.0, reg=2)
    th = np.zeros((K, K))
    th[1, 1] = 1.0
    b = np.indices((1, H, W)).sum(0) % 2 * 2.0 - 1.0      # checkerboard: <b, Hb> < 0
    q, info = O.adjoint_solve(p, th, np.zeros((1, H, W)), b, tol=1e-12, max_iter=50)
    assert info["status"] == O.NOT_SPD
    assert np.all(q == 0)


# ----------------------------------------------------------------------------- hypergradient
def _tight(p, th, y, x0):
    return R.newton_solve(R.t(th), R.t(y), R.t(x0), p.alpha, p.eps_tv, p.reg)


def _F(p, th, a, y, x0):
    xh = _tight(p, th, y, x0)
    return float(R.g(R.t(a), R.t(y), xh) + R.sobolev(R.t(th), R.t(a), p.beta)), xh


def test_hypergrad_dense_ift_route():
    inst, p = small_instance(C=1, H=14, W=14, K=5)
    th = inst.a + 0.01 * rng.standard_normal(inst.a.shape)
    tt, ty = R.t(th), R.t(inst.y)
    xh = _tight(p, th, inst.y, inst.y)
    Hm = R.hess_h(tt, ty, xh, p.alpha, p.eps_tv)
    ggrad, _, _ = O.upper_value_grad(p, inst.a, inst.y, xh.numpy())
    q = torch.linalg.solve(Hm, R.t(ggrad).reshape(-1))
    J = R.mixed_jac(tt, ty, xh, p.alpha, p.eps_tv)                 # N x K^2
    tr = tt.clone().requires_grad_(True)
    (gr,) = torch.autograd.grad(R.sobolev(tr, R.t(inst.a), p.beta), tr)
    zref = (-(J.T @ q)).reshape(p.K, p.K) + gr
    z, zn = O.hypergrad(p, th, inst.a, inst.y, xh.numpy(), q.reshape(p.shape).numpy())
    assert np.linalg.norm(z - zref.numpy()) <= 1e-10 * np.linalg.norm(zref.numpy())
    assert zn == pytest.approx(np.linalg.norm(z), rel=1e-14)


def test_hypergrad_central_differences_of_F():
    inst, p = small_instance(C=1, H=12, W=12, K=5, alpha=5e-3)
    th = inst.a.copy()
    xh = _tight(p, th, inst.y, inst.y).numpy()
    ggrad, _, _ = O.upper_value_grad(p, inst.a, inst.y, xh)
    q, _ = O.adjoint_solve(p, th, xh, ggrad, tol=1e-13, max_iter=20000)
    z, _ = O.hypergrad(p, th, inst.a, inst.y, xh, q)
    hstep = 1e-4
    for d in synth.directions(8, p.K):
        Fp, _ = _F(p, th + hstep * d, inst.a, inst.y, xh)
        Fm, _ = _F(p, th - hstep * d, inst.a, inst.y, xh)
        fd = (Fp - Fm) / (2 * hstep)
        dz = float(np.vdot(z, d))
        assert abs(fd - dz) <= 1e-5 * max(abs(dz), np.linalg.norm(z) * 1e-2)


def test_hypergrad_bilinear_identity():
    # sum_{uv} d(u,v) Z(u,v) = <rho, d*q> + <theta*q, d*x>   (scipy convolution)
    C, H, W, K = 2, 11, 13, 5
    p = O.Problem(C, H, W, K, alpha=1e-3)
    th, y, x, q, d = (rng.standard_normal(s) for s in [(K, K), (C, H, W), (C, H, W), (C, H, W), (K, K)])
    z, _ = O.hypergrad(p, th, None, y, x, q, with_r=False)
    cs = lambda k, u: np.stack([ss.convolve2d(u[c], k, mode="same") for c in range(C)])
    rho = cs(th, x) - y
    rhs = np.vdot(rho, cs(d, q)) + np.vdot(cs(th, q), cs(d, x))
    assert abs(-np.vdot(z, d) - rhs) <= 1e-11 * (1 + abs(rhs))


def test_upper_value_grad_matches_autograd():
    inst, p = small_instance(C=3, H=10, W=9, K=5)
    x = inst.y + 0.01
    grad, g, gn = O.upper_value_grad(p, inst.a, inst.y, x)
    xt = R.t(x).requires_grad_(True)
    v = R.g(R.t(inst.a), R.t(inst.y), xt)
    (gr,) = torch.autograd.grad(v, xt)
    assert g == pytest.approx(float(v), rel=1e-13)
    np.testing.assert_allclose(grad, gr.numpy(), rtol=1e-12, atol=1e-13)
    assert gn == pytest.approx(np.linalg.norm(gr.numpy()), rel=1e-13)
