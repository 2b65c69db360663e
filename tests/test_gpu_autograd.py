"""Autograd form (torch.autograd.Function over the C ABI): the forward is the
lower-level solve, the backward the CG adjoint plus the theta correlation.

Checks: torch.autograd.gradcheck in FP64 on a tiny image; the oracle's
implicit-function route (tight oracle solve, oracle CG, oracle correlation)
on a small image; the dense implicit-function route on 16x16 (Hessian and
mixed Jacobian assembled by torch autograd, solved by LAPACK); central
finite differences (step 1e-4, 8 random unit directions) of
L(theta) = <w, xhat(theta)> against the FP64 autograd gradient, at a reduced
size and at the full 512x512x3, 15x15 size; the FP32 form call by call
against the oracle (decision replay of the forward solve, CG at equal
iteration counts, the correlation and theta*q at the GPU's points); and the
FP32 form end to end against the FP64 form."""
import numpy as np
import pytest
import scipy.signal as ss
import torch

import _ref_torch as R
import oracle as O
from paper_2502_09758_amd import synth
from paper_2502_09758_amd.autograd import maid_solve
from paper_2502_09758_amd.maid import Maid

pytestmark = pytest.mark.gpu


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda").contiguous()


def well_conditioned(H=10, W=10, C=1, seed=1):
    a = np.array([[0.0, 0.1, 0.0], [0.1, 0.6, 0.1], [0.0, 0.1, 0.0]])
    inst = synth.make("cfg1", H=H, W=W, C=C, K=3, seed=seed)
    y = np.stack([ss.convolve2d(inst.x_true[c], a, mode="same") for c in range(C)])
    y = y + 0.01 * np.random.default_rng(seed).standard_normal(y.shape)
    return a, y


def test_gradcheck_fp64_tiny():
    print("[case] autograd gradcheck fp64 10x10", flush=True)
    a, y = well_conditioned()
    m = Maid(1, 10, 10, 3, torch.float64, alpha=0.02, eps_tv=0.05)
    th = dev(a, torch.float64).requires_grad_(True)
    yt = dev(y, torch.float64).requires_grad_(True)

    def f(theta, yy):
        return maid_solve(theta, yy, m, tol=1e-13, cg_tol=1e-14, max_iter=20000, max_cg=5000)

    assert torch.autograd.gradcheck(f, (th, yt), eps=1e-5, atol=1e-6, rtol=1e-4, nondet_tol=1e-10)


def test_backward_matches_oracle_ift_route():
    print("[case] autograd vs oracle IFT route", flush=True)
    C, H, W = 2, 14, 12
    a, y = well_conditioned(H, W, C, seed=2)
    alpha, eps = 0.01, 0.05
    m = Maid(C, H, W, 3, torch.float64, alpha=alpha, eps_tv=eps)
    th = dev(a, torch.float64).requires_grad_(True)
    yt = dev(y, torch.float64).requires_grad_(True)
    x = maid_solve(th, yt, m, tol=1e-12, cg_tol=1e-13, max_iter=20000, max_cg=5000)
    wv = np.random.default_rng(5).standard_normal((C, H, W))
    (x * dev(wv, torch.float64)).sum().backward()
    p = O.Problem(C, H, W, 3, alpha=alpha, eps_tv=eps)
    xo, _, _ = O.lower_solve(p, a, y, y, tol=1e-12, max_iter=50000)
    qo, _ = O.adjoint_solve(p, a, xo, wv, tol=1e-13, max_iter=20000)
    zo, _ = O.hypergrad(p, a, None, y, xo, qo, with_r=False)
    dyo = O.conv(p, a, qo)
    g = th.grad.cpu().numpy()
    assert np.linalg.norm(g - zo) <= 1e-7 * np.linalg.norm(zo)
    assert np.linalg.norm(yt.grad.cpu().numpy() - dyo) <= 1e-7 * np.linalg.norm(dyo)


@pytest.mark.parametrize("C", [1, 2])
def test_backward_matches_dense_hessian_route(C):
    """dL/dtheta = -J^T H^{-1} w and dL/dy = theta*(H^{-1} w) with H the dense
    lower-level Hessian and J the dense mixed Jacobian d(grad_x h)/dtheta at
    the GPU's solution, on 16x16 with a 5x5 kernel, to 1e-10."""
    print(f"[case] autograd vs dense Hessian route C={C} 16x16 K=5", flush=True)
    H = W = 16
    K = 5
    inst = synth.make("cfg1", H=H, W=W, C=C, K=K, seed=40 + C)
    alpha, eps = 5e-3, 2e-2
    m = Maid(C, H, W, K, torch.float64, alpha=alpha, eps_tv=eps)
    th = dev(inst.a, torch.float64).requires_grad_(True)
    yt = dev(inst.y, torch.float64).requires_grad_(True)
    x = maid_solve(th, yt, m, tol=1e-12, cg_tol=1e-14, max_iter=200000, max_cg=20000)
    wv = np.random.default_rng(9).standard_normal((C, H, W))
    (x * dev(wv, torch.float64)).sum().backward()
    xh = x.detach().cpu()
    ta, ty = R.t(inst.a), R.t(inst.y)
    Hm = R.hess_h(ta, ty, xh, alpha, eps)
    J = R.mixed_jac(ta, ty, xh, alpha, eps)                          # N x K^2
    q = torch.linalg.solve(Hm, R.t(wv).reshape(-1))
    gth = (-(J.T @ q)).reshape(K, K).numpy()
    gy = R.conv(ta, q.reshape(C, H, W)).numpy()
    eth = np.linalg.norm(th.grad.cpu().numpy() - gth) / np.linalg.norm(gth)
    ey = np.linalg.norm(yt.grad.cpu().numpy() - gy) / np.linalg.norm(gy)
    print(f"   dtheta {eth:.2e}  dy {ey:.2e}", flush=True)
    assert eth <= 1e-10 and ey <= 1e-10
    m.close()


def _setup(C, H, W, K, seed=303):
    inst = synth.make("cfg3", H=H, W=W, C=C, K=K, seed=seed)
    kw = dict(alpha=inst.alpha, eps_tv=inst.eps_tv)
    wv = np.random.default_rng(7).standard_normal((C, H, W))
    return inst, kw, wv


def _autograd(m, inst, wv, dt, tol, cg_tol):
    th = dev(inst.a, torch.float64).requires_grad_(True)
    x = maid_solve(th, dev(inst.y, dt), m, tol=tol, cg_tol=cg_tol, max_iter=100000, max_cg=100000)
    (x * dev(wv, dt)).sum().backward()
    return th.grad.double().cpu().numpy(), x.detach()


def _fd_check(C, H, W, K, ndir):
    """central differences (h = 1e-4) of L(theta) = <w, xhat(theta)>, tight FP64
    solves warm-started at xhat(theta), against the FP64 autograd gradient;
    the error is measured against ||g|| (random unit directions)."""
    inst, kw, wv = _setup(C, H, W, K)
    m64 = Maid(C, H, W, K, torch.float64, **kw)
    g, x = _autograd(m64, inst, wv, torch.float64, 1e-11, 1e-12)
    y64, w64 = dev(inst.y, torch.float64), dev(wv, torch.float64)

    def L(theta):
        xx = x.clone()
        info = m64.lower_solve(dev(theta, torch.float64), y64, xx, 1e-10, max_iter=100000)
        assert info.status == 0
        return float((xx * w64).sum())

    h = 1e-4
    errs = []
    for d in synth.directions(ndir, K):
        fd = (L(inst.a + h * d) - L(inst.a - h * d)) / (2 * h)
        errs.append(abs(fd - float(np.vdot(g, d))) / np.linalg.norm(g))
    print(f"[fd] {C}x{H}x{W} K={K}: max |fd - <g,d>| / ||g|| = {max(errs):.2e}", flush=True)
    # O(h^2) truncation of the central difference dominates (measured 1.2e-5)
    assert max(errs) <= 5e-5


def test_fd_fp64_autograd_reduced():
    print("[case] autograd FD 3x128x128 K=15, 8 directions", flush=True)
    _fd_check(3, 128, 128, 15, 8)


@pytest.mark.timeout(600)
def test_fd_fp64_autograd_full_size():
    print("[case] autograd FD 3x512x512 K=15, 8 directions", flush=True)
    _fd_check(3, 512, 512, 15, 8)


@pytest.mark.timeout(300)
def test_fp32_autograd_per_call_against_oracle():
    """Each call the FP32 autograd form makes, against the oracle at the
    GPU's own inputs: the forward solve by decision replay, the backward CG at
    its iteration count from the GPU's xhat, the theta correlation and
    theta*q from the GPU's q.  Bar: 1e-5 relative (the FP32 parity bar)."""
    print("[case] autograd FP32 per call vs oracle 3x128x128 K=15", flush=True)
    C, H, W, K = 3, 128, 128, 15
    inst, kw, wv = _setup(C, H, W, K)
    p = O.Problem(C, H, W, K, alpha=kw["alpha"], eps_tv=kw["eps_tv"])
    y32 = np.asarray(inst.y, np.float32).astype(np.float64)
    w32 = np.asarray(wv, np.float32).astype(np.float64)
    m = Maid(C, H, W, K, torch.float32, **kw)
    th = dev(inst.a, torch.float64).requires_grad_(True)
    yt = dev(y32, torch.float32).requires_grad_(True)
    rec = {}
    x = maid_solve(th, yt, m, tol=1e-3, cg_tol=1e-6, max_iter=5000, max_cg=5000, record=rec)
    (x * dev(w32, torch.float32)).sum().backward()
    li, ci = rec["lower"], rec["cg"]
    assert li.status == 0 and ci.status == 0 and li.iters > 3
    xg = x.detach().double().cpu().numpy()
    qg = rec["q"].double().cpu().numpy()
    xr, _, _ = O.lower_solve(p, inst.a, y32, y32, tol=0.0, max_iter=li.iters, L=0.0, replay_bt=li.trace)
    qr, _ = O.adjoint_solve(p, inst.a, xg, w32, tol=0.0, max_iter=ci.iters)
    zr, _ = O.hypergrad(p, inst.a, None, y32, xg, qg, with_r=False)
    dyr = O.conv(p, inst.a, qg)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    ex, eq = rel(xg, xr), rel(qg, qr)
    ez, ey = rel(th.grad.cpu().numpy(), zr), rel(yt.grad.double().cpu().numpy(), dyr)
    print(f"   forward {li.iters} it: x {ex:.2e}; CG {ci.iters} it: q {eq:.2e}; dtheta {ez:.2e}; dy {ey:.2e}",
          flush=True)
    assert max(ex, eq, ez, ey) <= 1e-5
    m.close()


def test_fp32_autograd_against_fp64():
    """The FP32-storage form at its accuracy floor against the FP64 form:
    the end-to-end gradient error is set by how accurately FP32 can solve the
    forward and adjoint systems at this conditioning (alpha = 2e-4), not by
    the kernels (per-call parity to 1e-5 is checked separately)."""
    print("[case] autograd FP32 vs FP64 3x128x128 K=15", flush=True)
    C, H, W, K = 3, 128, 128, 15
    inst, kw, wv = _setup(C, H, W, K)
    g64, _ = _autograd(Maid(C, H, W, K, torch.float64, **kw), inst, wv, torch.float64, 1e-11, 1e-12)
    errs = []
    for tol in (1e-3, 1e-4, 3e-5):
        g32, _ = _autograd(Maid(C, H, W, K, torch.float32, **kw), inst, wv, torch.float32, tol, 1e-6)
        errs.append(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))
    print(f"[fp32] rel err vs FP64 at lower tol 1e-3, 1e-4, 3e-5: {errs}", flush=True)
    assert errs[0] > errs[1] > errs[2]       # converges as the FP32 solve tightens
    assert errs[2] <= 2e-2
