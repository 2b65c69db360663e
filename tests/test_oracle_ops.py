"""Pins of the oracle's operators (CPU only).

Each check ties an oracle function to something other than itself: scipy's
direct convolution, the DFT diagonalisation of a circular convolution,
shifted-delta brute force, an independently written numpy Laplacian,
torch autograd of an independently written objective, closed-form TV
values, and central finite differences."""
import numpy as np
import pytest
import scipy.signal as ss
import torch

import oracle as O
import _ref_torch as R

rng = np.random.default_rng(7)


def rnd(*shape):
    return rng.standard_normal(shape)


@pytest.mark.parametrize("K", [1, 3, 5, 7])
@pytest.mark.parametrize("C,H,W", [(1, 9, 8), (2, 7, 11), (3, 5, 6)])
def test_conv_matches_scipy_same_convolution(K, C, H, W):
    if K > min(H, W):
        pytest.skip("kernel larger than image")
    p = O.Problem(C, H, W, K)
    th, x = rnd(K, K), rnd(C, H, W)
    ref = np.stack([ss.convolve2d(x[c], th, mode="same", boundary="fill") for c in range(C)])
    np.testing.assert_allclose(O.conv(p, th, x), ref, rtol=1e-13, atol=1e-13)
    r = rnd(C, H, W)
    refa = np.stack([ss.correlate2d(r[c], th, mode="same", boundary="fill") for c in range(C)])
    np.testing.assert_allclose(O.conv_adj(p, th, r), refa, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("periodic", [False, True])
def test_conv_adjoint_identity(periodic):
    p = O.Problem(2, 10, 13, 5, periodic=periodic)
    th, x, r = rnd(5, 5), rnd(2, 10, 13), rnd(2, 10, 13)
    lhs = np.vdot(O.conv(p, th, x), r)
    rhs = np.vdot(x, O.conv_adj(p, th, r))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1)


def test_conv_periodic_is_dft_diagonal():
    H, W, K = 12, 10, 5
    p = O.Problem(1, H, W, K, periodic=True)
    th, x = rnd(K, K), rnd(1, H, W)
    c0 = (K - 1) // 2
    kp = np.zeros((H, W))
    for u in range(K):
        for v in range(K):
            kp[(u - c0) % H, (v - c0) % W] = th[u, v]
    ref = np.real(np.fft.ifft2(np.fft.fft2(kp) * np.fft.fft2(x[0])))
    np.testing.assert_allclose(O.conv(p, th, x)[0], ref, atol=1e-12)


def test_conv_shifted_delta_orientation():
    # theta = delta at (u0, v0) must give out(i,j) = x(i + c0 - u0, j + c0 - v0)
    H, W, K = 9, 11, 5
    p = O.Problem(1, H, W, K)
    x = rnd(1, H, W)
    c0 = 2
    for (u0, v0) in [(0, 0), (0, 4), (3, 1), (2, 2)]:
        th = np.zeros((K, K))
        th[u0, v0] = 1.0
        out = O.conv(p, th, x)[0]
        for i in range(H):
            for j in range(W):
                ii, jj = i + c0 - u0, j + c0 - v0
                ref = x[0, ii, jj] if (0 <= ii < H and 0 <= jj < W) else 0.0
                assert out[i, j] == ref


def test_differences_and_laplacian():
    C, H, W = 2, 6, 7
    p = O.Problem(C, H, W, 1)
    x = rnd(C, H, W)
    dh, dv = O.diff(p, x)
    np.testing.assert_array_equal(dh, np.concatenate([np.diff(x, axis=2), np.zeros((C, H, 1))], axis=2))
    np.testing.assert_array_equal(dv, np.concatenate([np.diff(x, axis=1), np.zeros((C, 1, W))], axis=1))
    # adjoint identity
    ph, pv = rnd(C, H, W), rnd(C, H, W)
    lhs = np.vdot(dh, ph) + np.vdot(dv, pv)
    rhs = np.vdot(x, O.diff_adj(p, ph, pv))
    assert abs(lhs - rhs) < 1e-12
    # D^T D = - (5-point Neumann Laplacian), built independently
    lap = O.diff_adj(p, dh, dv)
    ref = np.zeros_like(x)
    for c in range(C):
        for i in range(H):
            for j in range(W):
                s = 0.0
                for (a, b) in [(i - 1, j), (i + 1, j), (i, j - 1), (i, j + 1)]:
                    if 0 <= a < H and 0 <= b < W:
                        s += x[c, i, j] - x[c, a, b]
                ref[c, i, j] = s
    np.testing.assert_allclose(lap, ref, atol=1e-12)


def test_tv_closed_form_step_edge():
    # vertical step edge 0 | 1: the gradient magnitude is 1 on exactly H pixels
    H, W, eps = 8, 10, 1e-2
    x = np.zeros((1, H, W))
    x[:, :, 5:] = 1.0
    for reg in (0, 1):
        p = O.Problem(1, H, W, 1, eps_tv=eps, reg=reg)
        assert abs(O.reg_value(p, x) - H * (np.sqrt(1 + eps ** 2) - eps)) < 1e-12
    # vectorial coupling: two channels with steps of 3 and 4 at the same place -> |s| = 5
    x2 = np.zeros((2, H, W))
    x2[0, :, 5:] = 3.0
    x2[1, :, 5:] = 4.0
    pv = O.Problem(2, H, W, 1, eps_tv=eps, reg=0)
    pc = O.Problem(2, H, W, 1, eps_tv=eps, reg=1)
    assert abs(O.reg_value(pv, x2) - H * (np.sqrt(25 + eps ** 2) - eps)) < 1e-11
    assert abs(O.reg_value(pc, x2) - H * (np.sqrt(9 + eps ** 2) + np.sqrt(16 + eps ** 2) - 2 * eps)) < 1e-11
    assert O.reg_value(pv, np.zeros((2, H, W))) == 0.0


@pytest.mark.parametrize("reg", [0, 1, 2])
@pytest.mark.parametrize("periodic", [False, True])
def test_reg_grad_hvp_match_autograd(reg, periodic):
    C, H, W, eps = 3, 7, 9, 1e-2
    p = O.Problem(C, H, W, 1, eps_tv=eps, reg=reg, periodic=periodic)
    x = rnd(C, H, W) * 0.1
    d = rnd(C, H, W)
    xt = R.t(x).requires_grad_(True)
    v = R.reg(xt, eps, reg, periodic)
    (gx,) = torch.autograd.grad(v, xt, create_graph=True)
    (hv,) = torch.autograd.grad(gx, xt, grad_outputs=R.t(d))
    assert abs(O.reg_value(p, x) - float(v)) < 1e-12 * (1 + abs(float(v)))
    np.testing.assert_allclose(O.reg_grad(p, x), gx.detach().numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(O.reg_hvp(p, x, d), hv.numpy(), rtol=1e-10, atol=1e-9)


def test_reg_central_differences():
    C, H, W, eps = 2, 6, 5, 1e-2
    p = O.Problem(C, H, W, 1, eps_tv=eps)
    x = rnd(C, H, W) * 0.05
    d = rnd(C, H, W)
    tau = 1e-5
    fd = (O.reg_value(p, x + tau * d) - O.reg_value(p, x - tau * d)) / (2 * tau)
    assert abs(fd - np.vdot(O.reg_grad(p, x), d)) < 1e-6 * max(1.0, abs(fd))
    fdg = (O.reg_grad(p, x + tau * d) - O.reg_grad(p, x - tau * d)) / (2 * tau)
    hv = O.reg_hvp(p, x, d)
    assert np.linalg.norm(fdg - hv) < 1e-5 * np.linalg.norm(hv)


def test_reg_hessian_symmetric_psd_constant_nullspace():
    C, H, W, eps = 2, 5, 6, 1e-2
    p = O.Problem(C, H, W, 1, eps_tv=eps)
    x = rnd(C, H, W) * 0.1
    N = C * H * W
    Hm = np.zeros((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1
        Hm[:, k] = O.reg_hvp(p, x, e.reshape(C, H, W)).ravel()
    assert np.abs(Hm - Hm.T).max() < 1e-9 * np.abs(Hm).max()
    assert np.linalg.eigvalsh(0.5 * (Hm + Hm.T)).min() > -1e-9
    for c in range(C):
        one = np.zeros((C, H, W))
        one[c] = 1.0
        assert np.abs(O.reg_hvp(p, x, one)).max() < 1e-12
        assert np.abs(O.reg_grad(p, x + one) - O.reg_grad(p, x)).max() < 1e-9


def test_reg_large_eps_limit_is_quadratic():
    # phi(s) -> s^2 / (2 eps) for s << eps; error bounded by sum s^4 / (8 eps^3)
    C, H, W, eps = 1, 6, 6, 10.0
    x = rnd(C, H, W) * 0.1
    pt = O.Problem(C, H, W, 1, eps_tv=eps, reg=0)
    pq = O.Problem(C, H, W, 1, reg=2)
    dh, dv = O.diff(pq, x)
    s4 = ((dh ** 2 + dv ** 2) ** 2).sum()
    assert abs(O.reg_value(pt, x) - O.reg_value(pq, x) / eps) <= s4 / (8 * eps ** 3) + 1e-15


@pytest.mark.parametrize("periodic", [False, True])
def test_h_grad_hvp_match_autograd(periodic):
    C, H, W, K = 2, 8, 9, 5
    p = O.Problem(C, H, W, K, alpha=3e-3, eps_tv=1e-2, periodic=periodic)
    th, y, x, d = rnd(K, K) * 0.2, rnd(C, H, W), rnd(C, H, W) * 0.3, rnd(C, H, W)
    ref_h = float(R.h(R.t(th), R.t(y), R.t(x), p.alpha, p.eps_tv, 0, periodic))
    assert abs(O.h_value(p, th, y, x) - ref_h) < 1e-12 * (1 + abs(ref_h))
    gref = R.grad_h(R.t(th), R.t(y), R.t(x), p.alpha, p.eps_tv, 0, periodic).numpy()
    np.testing.assert_allclose(O.h_grad(p, th, y, x), gref, rtol=1e-11, atol=1e-11)
    xt = R.t(x).requires_grad_(True)
    v = R.h(R.t(th), R.t(y), xt, p.alpha, p.eps_tv, 0, periodic)
    (gx,) = torch.autograd.grad(v, xt, create_graph=True)
    (hv,) = torch.autograd.grad(gx, xt, grad_outputs=R.t(d))
    np.testing.assert_allclose(O.h_hvp(p, th, x, d), hv.numpy(), rtol=1e-10, atol=1e-10)


def test_per_pixel_evaluations_match_whole_image():
    C, H, W, K = 2, 10, 12, 5
    p = O.Problem(C, H, W, K, alpha=2e-3)
    th, y, x, d = rnd(K, K), rnd(C, H, W), rnd(C, H, W), rnd(C, H, W)
    idx = np.arange(C * H * W)
    np.testing.assert_allclose(O.h_grad_at(p, th, y, x, idx), O.h_grad(p, th, y, x).ravel(), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(O.h_hvp_at(p, th, x, d, idx), O.h_hvp(p, th, x, d).ravel(), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(O.conv_at(p, th, x, idx), O.conv(p, th, x).ravel(), rtol=1e-13, atol=1e-13)


def test_sobolev_value_grad():
    K = 5
    p = O.Problem(1, 8, 8, K, beta=0.3)
    th, a = rnd(K, K), rnd(K, K)
    ref = float(R.sobolev(R.t(th), R.t(a), 0.3))
    assert abs(O.sobolev_value(p, th, a) - ref) < 1e-12 * (1 + ref)
    tt = R.t(th).requires_grad_(True)
    (gr,) = torch.autograd.grad(R.sobolev(tt, R.t(a), 0.3), tt)
    np.testing.assert_allclose(O.sobolev_grad(p, th, a), gr.numpy(), rtol=1e-12, atol=1e-12)
    # seminorm flag: w0 = 0 drops the L2 part
    p0 = O.Problem(1, 8, 8, K, beta=0.3, h1_w0=0.0)
    c = np.full((K, K), 2.0)
    assert O.sobolev_value(p0, a + c, a) == pytest.approx(0.0, abs=1e-12)
    assert O.sobolev_value(O.Problem(1, 8, 8, K, beta=0.0), th, a) == 0.0
