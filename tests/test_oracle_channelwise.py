"""Pins of the oracle with one blur kernel per colour channel (theta in
R^{C x K x K}, kc = C), CPU only.

  - the convolution and its adjoint against scipy, channel by channel with
    each channel's own kernel;
  - h's gradient and Hessian product, the upper level and the Sobolev term
    against torch autograd of independently written objectives (a grouped
    torch convolution);
  - the hypergradient of Eq. (3.2) against the dense implicit-function route
    with autograd Jacobians, and against the bilinear identity with scipy;
  - reductions to the shared-kernel case: equal per-channel kernels give the
    shared kernel's convolution, and the shared kernel's hypergradient is the
    sum over channels of the per-channel one;
  - decoupling: with channelwise TV the C-channel problem splits into C
    single-channel problems, so its tight lower-level solution and its
    hypergradient equal the single-channel ones channel by channel;
  - Lemma 1's sufficient decrease for MAID steps with per-channel kernels.
"""
import numpy as np
import pytest
import scipy.signal as ss
import torch

import oracle as O
import _ref_torch as R
from paper_2502_09758_amd import synth

rng = np.random.default_rng(23)


def rnd(*shape):
    return rng.standard_normal(shape)


@pytest.mark.parametrize("C,H,W,K", [(2, 9, 8, 3), (3, 7, 11, 5), (3, 6, 6, 1)])
def test_conv_per_channel_matches_scipy(C, H, W, K):
    p = O.Problem(C, H, W, K, kc=C)
    th, x, r = rnd(C, K, K), rnd(C, H, W), rnd(C, H, W)
    ref = np.stack([ss.convolve2d(x[c], th[c], mode="same") for c in range(C)])
    np.testing.assert_allclose(O.conv(p, th, x), ref, rtol=1e-13, atol=1e-13)
    refa = np.stack([ss.correlate2d(r[c], th[c], mode="same") for c in range(C)])
    np.testing.assert_allclose(O.conv_adj(p, th, r), refa, rtol=1e-13, atol=1e-13)


def test_kc_must_be_one_or_C():
    with pytest.raises(ValueError):
        O.Problem(3, 8, 8, 3, kc=2)


@pytest.mark.parametrize("reg", [0, 1])
def test_h_grad_hvp_match_autograd_per_channel(reg):
    C, H, W, K = 3, 8, 9, 5
    p = O.Problem(C, H, W, K, alpha=3e-3, eps_tv=1e-2, reg=reg, kc=C)
    th, y, x, d = rnd(C, K, K) * 0.2, rnd(C, H, W), rnd(C, H, W) * 0.3, rnd(C, H, W)
    ref_h = float(R.h(R.t(th), R.t(y), R.t(x), p.alpha, p.eps_tv, reg))
    assert abs(O.h_value(p, th, y, x) - ref_h) < 1e-12 * (1 + abs(ref_h))
    gref = R.grad_h(R.t(th), R.t(y), R.t(x), p.alpha, p.eps_tv, reg).numpy()
    np.testing.assert_allclose(O.h_grad(p, th, y, x), gref, rtol=1e-11, atol=1e-11)
    xt = R.t(x).requires_grad_(True)
    v = R.h(R.t(th), R.t(y), xt, p.alpha, p.eps_tv, reg)
    (gx,) = torch.autograd.grad(v, xt, create_graph=True)
    (hv,) = torch.autograd.grad(gx, xt, grad_outputs=R.t(d))
    np.testing.assert_allclose(O.h_hvp(p, th, x, d), hv.numpy(), rtol=1e-10, atol=1e-10)
    idx = np.arange(C * H * W)[::7]
    np.testing.assert_allclose(O.h_grad_at(p, th, y, x, idx), gref.ravel()[idx], rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(O.h_hvp_at(p, th, x, d, idx), hv.numpy().ravel()[idx], rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(O.conv_at(p, th, x, idx), R.conv(R.t(th), R.t(x)).numpy().ravel()[idx],
                               rtol=1e-13, atol=1e-13)


def test_upper_and_sobolev_match_autograd_per_channel():
    C, H, W, K = 3, 10, 9, 5
    p = O.Problem(C, H, W, K, beta=0.3, kc=C)
    a, th, y, x = rnd(C, K, K), rnd(C, K, K), rnd(C, H, W), rnd(C, H, W)
    grad, g, gn = O.upper_value_grad(p, a, y, x)
    xt = R.t(x).requires_grad_(True)
    v = R.g(R.t(a), R.t(y), xt)
    (gr,) = torch.autograd.grad(v, xt)
    assert g == pytest.approx(float(v.detach()), rel=1e-13)
    np.testing.assert_allclose(grad, gr.numpy(), rtol=1e-12, atol=1e-13)
    ref = float(R.sobolev(R.t(th), R.t(a), 0.3))
    assert abs(O.sobolev_value(p, th, a) - ref) < 1e-12 * (1 + ref)
    tt = R.t(th).requires_grad_(True)
    (gs,) = torch.autograd.grad(R.sobolev(tt, R.t(a), 0.3), tt)
    np.testing.assert_allclose(O.sobolev_grad(p, th, a), gs.numpy(), rtol=1e-12, atol=1e-12)
    # no coupling across kernel channels: the sum of the single-channel terms
    p1 = O.Problem(1, H, W, K, beta=0.3)
    assert O.sobolev_value(p, th, a) == pytest.approx(sum(O.sobolev_value(p1, th[c], a[c]) for c in range(C)),
                                                      rel=1e-14)


def test_hypergrad_per_channel_dense_ift_route():
    inst = synth.make_channelwise("cfg3", H=8, W=8, K=3, seed=4)
    C, K = inst.C, inst.K
    p = O.Problem(C, 8, 8, K, alpha=2e-3, eps_tv=1e-2, beta=1e-3, kc=C)
    th = inst.a + 0.01 * rnd(C, K, K)
    tt, ty = R.t(th), R.t(inst.y)
    xh = R.newton_solve(tt, ty, ty, p.alpha, p.eps_tv, 0)
    Hm = R.hess_h(tt, ty, xh, p.alpha, p.eps_tv)
    ggrad, _, _ = O.upper_value_grad(p, inst.a, inst.y, xh.numpy())
    q = torch.linalg.solve(Hm, R.t(ggrad).reshape(-1))
    J = R.mixed_jac(tt, ty, xh, p.alpha, p.eps_tv)                 # N x C K^2
    tr = tt.clone().requires_grad_(True)
    (gr,) = torch.autograd.grad(R.sobolev(tr, R.t(inst.a), p.beta), tr)
    zref = (-(J.T @ q)).reshape(C, K, K) + gr
    z, zn = O.hypergrad(p, th, inst.a, inst.y, xh.numpy(), q.reshape(p.shape).numpy())
    assert z.shape == (C, K, K)
    assert np.linalg.norm(z - zref.numpy()) <= 1e-10 * np.linalg.norm(zref.numpy())
    assert zn == pytest.approx(np.linalg.norm(z), rel=1e-14)


def test_hypergrad_per_channel_bilinear_identity():
    # sum_{c,uv} d_c(u,v) Z_c(u,v) = <rho, d*q> + <theta*q, d*x>, all per channel (scipy)
    C, H, W, K = 3, 11, 13, 5
    p = O.Problem(C, H, W, K, alpha=1e-3, kc=C)
    th, d = rnd(C, K, K), rnd(C, K, K)
    y, x, q = rnd(C, H, W), rnd(C, H, W), rnd(C, H, W)
    z, _ = O.hypergrad(p, th, None, y, x, q, with_r=False)
    cs = lambda k, u: np.stack([ss.convolve2d(u[c], k[c], mode="same") for c in range(C)])
    rho = cs(th, x) - y
    rhs = np.vdot(rho, cs(d, q)) + np.vdot(cs(th, q), cs(d, x))
    assert abs(-np.vdot(z, d) - rhs) <= 1e-11 * (1 + abs(rhs))


def test_equal_channel_kernels_reduce_to_shared():
    C, H, W, K = 3, 9, 10, 5
    p1 = O.Problem(C, H, W, K, alpha=2e-3, beta=1e-3)
    pc = O.Problem(C, H, W, K, alpha=2e-3, beta=1e-3, kc=C)
    th, a = rnd(K, K), rnd(K, K)
    thc, ac = np.stack([th] * C), np.stack([a] * C)
    y, x, q = rnd(C, H, W), rnd(C, H, W), rnd(C, H, W)
    np.testing.assert_array_equal(O.conv(pc, thc, x), O.conv(p1, th, x))
    np.testing.assert_array_equal(O.h_grad(pc, thc, y, x), O.h_grad(p1, th, y, x))
    z1, _ = O.hypergrad(p1, th, a, y, x, q, with_r=False)
    zc, _ = O.hypergrad(pc, thc, ac, y, x, q, with_r=False)
    np.testing.assert_allclose(zc.sum(0), z1, rtol=1e-12, atol=1e-12 * np.abs(z1).max())


def test_channelwise_tv_decouples_into_single_channel_problems():
    inst = synth.make_channelwise("cfg3", H=12, W=12, K=5, seed=9)
    C, K = inst.C, inst.K
    kw = dict(alpha=3e-3, eps_tv=1e-2, beta=1.5e-3)
    pc = O.Problem(C, 12, 12, K, reg=1, kc=C, **kw)
    p1 = O.Problem(1, 12, 12, K, **kw)
    th = inst.a + 0.02 * rnd(C, K, K)
    x, info, _ = O.lower_solve(pc, th, inst.y, inst.y, tol=1e-11, max_iter=20000)
    assert info["status"] == O.OK
    grad, _, _ = O.upper_value_grad(pc, inst.a, inst.y, x)
    q, ci = O.adjoint_solve(pc, th, x, grad, tol=1e-12, max_iter=20000)
    assert ci["status"] == O.OK
    z, _ = O.hypergrad(pc, th, inst.a, inst.y, x, q)
    for c in range(C):
        xc, ic, _ = O.lower_solve(p1, th[c], inst.y[c:c + 1], inst.y[c:c + 1], tol=1e-11, max_iter=20000)
        assert ic["status"] == O.OK
        assert np.abs(x[c] - xc[0]).max() <= 1e-8
        gc, _, _ = O.upper_value_grad(p1, inst.a[c], inst.y[c:c + 1], xc)
        qc, _ = O.adjoint_solve(p1, th[c], xc, gc, tol=1e-12, max_iter=20000)
        zc, _ = O.hypergrad(p1, th[c], inst.a[c], inst.y[c:c + 1], xc, qc)
        assert np.linalg.norm(z[c] - zc) <= 1e-6 * np.linalg.norm(zc)


def _F(p, th, a, y, x0):
    xh = R.newton_solve(R.t(th), R.t(y), R.t(x0), p.alpha, p.eps_tv, p.reg)
    return float(R.g(R.t(a), R.t(y), xh) + R.sobolev(R.t(th), R.t(a), p.beta))


def test_lemma1_sufficient_decrease_per_channel():
    """As the shared-kernel pin: mu certified as the smallest eigenvalue of
    the block-diagonal data Hessian (smallest over channels), every accepted
    step decreases the exact F by at least lambda * s * ||z||^2, and
    L_g defaults to (max_c ||a_c||_1)^2."""
    C, H, W = 2, 10, 10
    a1 = np.array([[0.0, 0.1, 0.0], [0.1, 0.6, 0.1], [0.0, 0.1, 0.0]])
    a = np.stack([a1, 0.9 * a1 + 0.1 * np.eye(3) / 3])
    inst = synth.make("cfg1", H=H, W=W, C=C, K=7, seed=3)
    true = a + 0.05 * np.array([[1, 0, -1], [0, 0, 0], [-1, 0, 1.0]])
    y = np.stack([ss.convolve2d(inst.x_true[c], true[c], mode="same") for c in range(C)])
    y = y + 0.01 * np.random.default_rng(3).standard_normal(y.shape)
    p = O.Problem(C, H, W, 3, alpha=2e-3, eps_tv=1e-2, beta=1e-3, kc=C)
    mus = []
    for c in range(C):
        A = np.stack([ss.convolve2d(e.reshape(H, W), a[c], mode="same").ravel() for e in np.eye(H * W)], 1)
        mus.append(np.linalg.eigvalsh(A.T @ A).min())
    mu = min(mus)
    assert mu > 1e-3
    lam = 0.05
    st = O.MaidState(a, y, np.zeros_like(y), eps=1e-4, delta=1e-4, step=0.3)
    F_prev = _F(p, st.theta, a, y, y)
    accepted = 0
    for k in range(4):
        s_before = st.step
        rc, info = O.maid_step(p, a, y, st, mu=mu, lambda_=lam, max_lower_iter=100000,
                               max_cg_iter=100000, eps_min=1e-6)
        if rc == O.ACCURACY_FLOOR:
            break
        assert rc == O.OK and info["accepted"] and info["psi"] <= 0.0
        accepted += 1
        s_used = s_before * 0.5 ** (info["trials"] - 1)
        F_new = _F(p, st.theta, a, y, st.x)
        assert F_new - F_prev <= -lam * s_used * info["znorm"] ** 2 * (1 - 1e-9)
        F_prev = F_new
    assert accepted >= 2
    assert st.theta.shape == (C, 3, 3) and not np.allclose(st.theta[0], st.theta[1])
