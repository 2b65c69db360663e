"""Pins of the oracle's Section 4.1 baselines (CPU only).

  gd_solve:   the fixed-step iteration against its closed form in Fourier
              space (periodic boundary, quadratic R: every frequency is a
              scalar linear recursion) and against the same iteration with
              torch autograd gradients (TV, zero boundary);
  lista_grad: against torch autograd through the unrolled iterations
              (independent reverse mode) and against central differences
              of the unrolled loss (a finite computation, so O(h^2) only);
  ift_step:   with many lower-level iterations and a tight CG, z equals the
              dense implicit-function route (torch Hessian and mixed
              Jacobian, LAPACK solve) at the step's point, and the step is
              theta - step z.
"""
import numpy as np
import pytest
import torch

import oracle as O
import _ref_torch as R
from paper_2502_09758_amd import synth

rng = np.random.default_rng(31)


def test_gd_solve_fourier_closed_form():
    C, H, W, K, alpha, lam, n = 1, 14, 10, 5, 0.04, 0.3, 25
    p = O.Problem(C, H, W, K, alpha=alpha, periodic=True, reg=2)
    th = synth.gaussian_kernel(K, 1.0)
    y = rng.standard_normal((C, H, W))
    x0 = rng.standard_normal((C, H, W))
    xn, xs = O.gd_solve(p, th, y, x0, lam, n)
    assert len(xs) == n and np.array_equal(xs[0], x0)
    c0 = (K - 1) // 2
    kp = np.zeros((H, W))
    for u in range(K):
        for v in range(K):
            kp[(u - c0) % H, (v - c0) % W] = th[u, v]
    kh = np.fft.fft2(kp)
    d2 = (2 - 2 * np.cos(2 * np.pi * np.arange(W) / W))[None, :] + (2 - 2 * np.cos(2 * np.pi * np.arange(H) / H))[:, None]
    a = np.abs(kh) ** 2 + alpha * d2                   # the Hessian's eigenvalues
    rho = 1 - lam * a                                  # per-frequency contraction
    b = lam * np.conj(kh) * np.fft.fft2(y[0])
    geo = np.where(np.abs(1 - rho) > 1e-14, (1 - rho ** n) / np.where(np.abs(1 - rho) > 1e-14, 1 - rho, 1), n)
    ref = np.real(np.fft.ifft2(rho ** n * np.fft.fft2(x0[0]) + b * geo))
    assert np.linalg.norm(xn[0] - ref) <= 1e-12 * np.linalg.norm(ref)


def test_gd_solve_matches_torch_gradient_iteration():
    inst = synth.make("cfg1", H=12, W=15, C=2, K=5, seed=8)
    p = O.Problem(2, 12, 15, 5, alpha=3e-3, eps_tv=2e-2)
    lam, n = 0.2, 12
    xn, _ = O.gd_solve(p, inst.a, inst.y, inst.y, lam, n)
    x = R.t(inst.y)
    for _ in range(n):
        x = x - lam * R.grad_h(R.t(inst.a), R.t(inst.y), x, p.alpha, p.eps_tv)
    assert np.linalg.norm(xn - x.numpy()) <= 1e-12 * np.linalg.norm(xn)


def _torch_lista(a, y, th, x0, n, lam, alpha, eps, beta):
    tt = R.t(th).requires_grad_(True)
    ty, x = R.t(y), R.t(x0)
    for _ in range(n):
        x = x - lam * R.grad_h_graph(tt, ty, x, alpha, eps)
    F = R.g(R.t(a), ty, x) + R.sobolev(tt, R.t(a), beta)
    (gr,) = torch.autograd.grad(F, tt)
    return gr.numpy(), float(F.detach()), x.detach().numpy()


@pytest.mark.parametrize("beta", [0.0, 2e-3])
def test_lista_grad_matches_torch_reverse_mode(beta):
    inst = synth.make("cfg1", H=10, W=13, C=1, K=3, seed=12)
    p = O.Problem(1, 10, 13, 3, alpha=4e-3, eps_tv=3e-2, beta=beta)
    th = inst.a + 0.02 * rng.standard_normal(inst.a.shape)
    lam, n = 0.25, 7
    g, F, xn = O.lista_grad(p, inst.a, inst.y, th, inst.y, n, lam)
    gt, Ft, xt = _torch_lista(inst.a, inst.y, th, inst.y, n, lam, p.alpha, p.eps_tv, beta)
    assert np.linalg.norm(xn - xt) <= 1e-12 * np.linalg.norm(xt)
    assert F == pytest.approx(Ft, rel=1e-12)
    assert np.linalg.norm(g - gt) <= 1e-10 * np.linalg.norm(gt)


def test_lista_grad_central_differences():
    inst = synth.make("cfg1", H=11, W=9, C=2, K=5, seed=14)
    p = O.Problem(2, 11, 9, 5, alpha=2e-3, eps_tv=2e-2, beta=1e-3)
    th = inst.a.copy()
    lam, n, hstep = 0.2, 6, 1e-5
    g, _, _ = O.lista_grad(p, inst.a, inst.y, th, inst.y, n, lam)

    def F(t):
        x, _ = O.gd_solve(p, t, inst.y, inst.y, lam, n)
        _, gv, _ = O.upper_value_grad(p, inst.a, inst.y, x)
        return gv + O.sobolev_value(p, t, inst.a)

    for d in synth.directions(4, p.K):
        fd = (F(th + hstep * d) - F(th - hstep * d)) / (2 * hstep)
        assert abs(fd - float(np.vdot(g, d))) <= 1e-7 * np.linalg.norm(g)


def test_ift_step_dense_route():
    inst = synth.make("cfg1", H=12, W=12, C=1, K=5, seed=16)
    p = O.Problem(1, 12, 12, 5, alpha=5e-3, eps_tv=2e-2, beta=1e-3)
    th = inst.a + 0.01 * rng.standard_normal(inst.a.shape)
    out = O.ift_step(p, inst.a, inst.y, th, inst.y, None, 4000, 0.4, 1e-13, 5000, 0.05)
    x = R.t(out["x"])
    gstep = R.grad_h(R.t(th), R.t(inst.y), x, p.alpha, p.eps_tv)
    assert float(gstep.norm()) <= 1e-9                    # the lower level is solved
    Hm = R.hess_h(R.t(th), R.t(inst.y), x, p.alpha, p.eps_tv)
    J = R.mixed_jac(R.t(th), R.t(inst.y), x, p.alpha, p.eps_tv)
    ggrad, g, _ = O.upper_value_grad(p, inst.a, inst.y, out["x"])
    q = torch.linalg.solve(Hm, R.t(ggrad).reshape(-1))
    tr = R.t(th).requires_grad_(True)
    (gr,) = torch.autograd.grad(R.sobolev(tr, R.t(inst.a), p.beta), tr)
    zref = ((-(J.T @ q)).reshape(p.K, p.K) + gr).numpy()
    assert np.linalg.norm(out["z"] - zref) <= 1e-8 * np.linalg.norm(zref)
    assert np.array_equal(out["theta"], th - 0.05 * out["z"])
    assert out["loss"] == pytest.approx(g + O.sobolev_value(p, th, inst.a), rel=1e-14)
