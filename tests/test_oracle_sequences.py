"""Pins of the oracle's iterate sequences (CPU only).

The limit pins in test_oracle_solvers.py check where the lower-level solve
and the CG solve end up; a solver with a wrong momentum or a wrong conjugacy
coefficient still gets there, only more slowly.  The GPU parity tests compare
the kernels with the oracle at fixed iteration counts, so the sequences
themselves are pinned here against references written independently from
the published methods:

  * FISTA with backtracking (Beck and Teboulle, 2009, smooth case): t_1 = 1,
    t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2, extrapolation
    y_{k+1} = x_k + ((t_k - 1) / t_{k+1}) (x_k - x_{k-1}), step
    x_k = y_k - grad f(y_k) / L_k with L_k the first eta^i L_{k-1} that passes
    f(x_k) <= f(y_k) - ||grad f(y_k)||^2 / (2 L_k).  Written in torch with
    autograd gradients and direct objective differences (the oracle evaluates
    the decrease through the increment): the oracle's extrapolated point after
    n iterations must equal y_{n+1} for every n, and its rejection counts must
    equal the reference's;
  * conjugate gradients (Hestenes and Stiefel, 1952) on the dense Hessian
    assembled by autograd: the oracle's iterate after n steps must equal the
    reference's for every n;
  * CG's finite termination: on a system whose matrix has m distinct
    eigenvalues (a periodic quadratic problem, diagonal in the Fourier basis,
    eigenvalues counted from the closed form), CG reaches the solution in at
    most m iterations; a wrong coefficient does not.
"""
import numpy as np
import pytest
import torch

import oracle as O
import _ref_torch as R
from paper_2502_09758_amd import synth


def _instance(C=1, H=12, W=10, K=5, alpha=4e-3, seed=21):
    inst = synth.make("cfg1", H=H, W=W, C=C, K=K, seed=seed)
    p = O.Problem(C, H, W, K, alpha=alpha, eps_tv=1e-2)
    return inst, p


def fista_reference(th, y, x0, alpha, eps, L0, n_iter, eta=2.0, reg=0):
    """Beck-Teboulle FISTA with backtracking, smooth case; returns the points
    y_1 .. y_{n_iter+1} at which the gradient is evaluated and the number of
    rejected trial steps per iteration."""
    th, y = R.t(th), R.t(y)
    f = lambda z: float(R.h(th, y, z, alpha, eps, reg))
    x_prev = R.t(x0).clone()
    x = x_prev.clone()
    yk = x.clone()                 # y_1 = x_0
    t = 1.0
    L = L0
    points, rejects = [yk.numpy().copy()], []
    for _ in range(n_iter):
        g = R.grad_h(th, y, yk, alpha, eps, reg)
        fy = f(yk)
        gn2 = float((g * g).sum())
        nrej = 0
        while True:
            xn = yk - g / L
            if f(xn) <= fy - gn2 / (2.0 * L):
                break
            L *= eta
            nrej += 1
        rejects.append(nrej)
        t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        x_prev, x = x, xn
        yk = x + ((t - 1.0) / t_next) * (x - x_prev)
        t = t_next
        points.append(yk.numpy().copy())
    return points, rejects, L


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.mark.parametrize("C,reg", [(1, 0), (2, 0), (2, 1), (1, 2)])
def test_fista_sequence_fixed_step(C, reg):
    """L above the global Lipschitz bound: no rejection, the iterates differ
    only through the momentum sequence."""
    inst, p = _instance(C=C)
    p.reg = reg
    Lbig = 2.0 * (np.abs(inst.a).sum() ** 2 + 8.0 * p.alpha / (p.eps_tv if reg != 2 else 1.0))
    n = 25
    pts, rej, _ = fista_reference(inst.a, inst.y, inst.y, p.alpha, p.eps_tv, Lbig, n, reg=reg)
    assert sum(rej) == 0
    for k in range(n + 1):
        v, info, trace = O.lower_solve(p, inst.a, inst.y, inst.y, tol=0.0, max_iter=k, L=Lbig)
        assert info["iters"] == k and info["backtracks"] == 0
        assert _rel(v, pts[k]) <= 1e-12, (k, _rel(v, pts[k]))
    # the momentum matters from the third point on: a plain gradient method
    # (y = x) would sit measurably away from it
    assert _rel(pts[3], pts[2]) > 1e-3


def test_fista_sequence_with_backtracking():
    """Starting far below the Lipschitz constant: the reference and the
    oracle reject the same trials and produce the same points."""
    inst, p = _instance(C=1, H=14, W=11, K=7, seed=22)
    L0 = 1e-2
    n = 30
    pts, rej, Lref = fista_reference(inst.a, inst.y, inst.y, p.alpha, p.eps_tv, L0, n)
    assert sum(rej) >= 3
    v, info, trace = O.lower_solve(p, inst.a, inst.y, inst.y, tol=0.0, max_iter=n, L=L0)
    assert list(trace) == rej
    assert info["L"] == pytest.approx(Lref, rel=1e-15)
    for k in (1, 2, 3, 5, 8, 13, 21, 30):
        vk, _, _ = O.lower_solve(p, inst.a, inst.y, inst.y, tol=0.0, max_iter=k, L=L0)
        assert _rel(vk, pts[k]) <= 1e-11, (k, _rel(vk, pts[k]))


def cg_reference(A, b, x0, n_iter):
    """Hestenes-Stiefel conjugate gradients on a dense SPD matrix; returns the
    iterates x_0 .. x_n."""
    x = x0.copy()
    r = b - A @ x
    d = r.copy()
    rr = r @ r
    out = [x.copy()]
    for _ in range(n_iter):
        Ad = A @ d
        step = rr / (d @ Ad)
        x = x + step * d
        r = r - step * Ad
        rr_new = r @ r
        d = r + (rr_new / rr) * d
        rr = rr_new
        out.append(x.copy())
    return out


@pytest.mark.parametrize("C", [1, 2])
def test_cg_sequence_matches_dense_reference(C):
    inst, p = _instance(C=C, H=8, W=7, K=3, alpha=5e-3, seed=23)
    xt, _, _ = O.lower_solve(p, inst.a, inst.y, inst.y, tol=1e-6, max_iter=5000)
    Hm = R.hess_h(R.t(inst.a), R.t(inst.y), R.t(xt), p.alpha, p.eps_tv).numpy()
    rng = np.random.default_rng(24)
    b = rng.standard_normal(p.N)
    q0 = 0.1 * rng.standard_normal(p.N)
    n = 20
    ref = cg_reference(Hm, b, q0, n)
    for k in range(n + 1):
        q, info = O.adjoint_solve(p, inst.a, xt, b.reshape(p.shape), q0=q0.reshape(p.shape), tol=0.0, max_iter=k)
        assert info["iters"] == k
        assert _rel(q, ref[k]) <= 1e-9, (k, _rel(q, ref[k]))


def test_cg_finite_termination_distinct_eigenvalues():
    """Periodic quadratic problem with the identity kernel: H = I + alpha D^T D
    is diagonal in the 2D Fourier basis with eigenvalues 1 + alpha (|d_h^(f)|^2
    + |d_v^(f)|^2), |d^(f)|^2 = 2 - 2 cos(2 pi f / n); with m distinct values
    (a spread of 400 here) CG is exact after m iterations and not before."""
    C, H, W, K, alpha = 1, 8, 6, 3, 50.0
    p = O.Problem(C, H, W, K, alpha=alpha, periodic=True, reg=2)
    th = np.zeros((K, K))
    th[1, 1] = 1.0
    lam = 1.0 + alpha * ((2 - 2 * np.cos(2 * np.pi * np.arange(W) / W))[None, :]
                         + (2 - 2 * np.cos(2 * np.pi * np.arange(H) / H))[:, None])
    m = len(np.unique(np.round(lam.ravel(), 9)))
    assert m == 17
    b = np.random.default_rng(25).standard_normal((C, H, W))
    qhat = np.real(np.fft.ifft2(np.fft.fft2(b[0]) / lam))[None]
    q, info = O.adjoint_solve(p, th, np.zeros((C, H, W)), b, tol=1e-12 * np.linalg.norm(b), max_iter=H * W)
    assert info["status"] == O.OK
    assert info["iters"] == m, (info["iters"], m)
    assert _rel(q, qhat) <= 1e-12
    # one step short of m the residual is still far from zero
    _, short = O.adjoint_solve(p, th, np.zeros((C, H, W)), b, tol=0.0, max_iter=m - 1)
    assert short["res_norm"] > 1e-5 * np.linalg.norm(b)
