"""Autograd form (torch.autograd.Function over the C ABI): the forward is the
lower-level solve, the backward the CG adjoint plus the theta correlation.

Checks: torch.autograd.gradcheck in FP64 on a tiny image; the oracle's
implicit-function route (tight oracle solve, oracle CG, oracle correlation)
on a small image; central finite differences (step 1e-4, random unit
directions) of L(theta) = <w, xhat(theta)> against the FP64 autograd
gradient, at a reduced size (8 directions) and at the full 512x512x3, 15x15
size (2 directions); and the FP32 form against the FP64 form."""
import numpy as np
import pytest
import scipy.signal as ss
import torch

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


def test_fd_fp64_autograd_full_size():
    print("[case] autograd FD 3x512x512 K=15, 2 directions", flush=True)
    _fd_check(3, 512, 512, 15, 2)


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
