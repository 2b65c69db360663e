"""Section 4.1's baselines (ADP-IFT, ADP-LISTA) through the C ABI, against
the oracle: the fixed-step lower-level iteration and its kept iterates, the
Hessian product, one ADP-IFT iteration (its CG replayed by the oracle at the
GPU's iteration count) and one ADP-LISTA iteration (the gradient through the
unrolled iterations).  FP64 to 1e-10, FP32 to the 1e-5 parity bar; shapes
cover the per-XCD team loops (small), the multi-kernel passes with ragged
tile tails, three channels, and the matrix-core correlations (K >= 13)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2502_09758_amd import _lib as L
from paper_2502_09758_amd import synth
from paper_2502_09758_amd.maid import Maid, MaidState

pytestmark = pytest.mark.gpu

DT = {"f32": torch.float32, "f64": torch.float64}
TOL = {"f32": 1e-5, "f64": 1e-10}
SHAPES = [(1, 40, 70, 5), (3, 130, 150, 9), (1, 90, 210, 15)]


def dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda").contiguous()


def host(t):
    return t.detach().double().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def stored(a, dt):
    return np.asarray(a, np.float32).astype(np.float64) if dt == "f32" else np.asarray(a, np.float64)


def setup(C, H, W, K, dt, seed=50, beta=1e-3):
    inst = synth.make("cfg1", H=H, W=W, C=C, K=K, seed=seed)
    p = O.Problem(C, H, W, K, alpha=inst.alpha, eps_tv=inst.eps_tv, beta=beta)
    m = Maid(C, H, W, K, DT[dt], alpha=p.alpha, eps_tv=p.eps_tv, beta=beta)
    m.set_one_pass(0)            # the kept iterates need the two-pass form
    return inst, p, m, stored(inst.y, dt)


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("C,H,W,K", SHAPES)
def test_gd_solve_and_kept_iterates(C, H, W, K, dt):
    print(f"[case] gd_solve {C}x{H}x{W} K={K} {dt}", flush=True)
    inst, p, m, y = setup(C, H, W, K, dt)
    lam, n = 0.4, 24
    th = dev(inst.a, torch.float64)
    x = dev(y, DT[dt])
    hist = torch.zeros((n, C, H, W), dtype=DT[dt], device="cuda")
    info = m.gd_solve(th, dev(y, DT[dt]), x, lam, n, hist=hist)
    assert info.status == L.MAXITER and info.iters == n and info.backtracks == 0
    xr, xs = O.gd_solve(p, inst.a, y, y, lam, n)
    ex = rel(host(x), xr)
    eh = max(rel(host(hist[k]), xs[k + 1] if k + 1 < n else xr) for k in range(n))
    print(f"   x_n {ex:.2e}  iterates {eh:.2e}", flush=True)
    assert ex <= TOL[dt] and eh <= TOL[dt]
    # a tolerance stops it early, at the first iterate that meets it
    gr = [np.linalg.norm(O.h_grad(p, inst.a, y, xk)) for xk in xs]
    tol = 0.5 * (gr[5] + gr[6])
    x2 = dev(y, DT[dt])
    i2 = m.gd_solve(th, dev(y, DT[dt]), x2, lam, n, tol=tol)
    assert i2.status == L.OK and i2.iters == 6, (i2, gr[4:8])


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("C,H,W,K", SHAPES)
def test_hessian_apply(C, H, W, K, dt):
    print(f"[case] hessian_apply {C}x{H}x{W} K={K} {dt}", flush=True)
    inst, p, m, y = setup(C, H, W, K, dt)
    rng = np.random.default_rng(3)
    w = stored(rng.standard_normal((C, H, W)), dt)
    out = m.hessian_apply(dev(inst.a, torch.float64), dev(y, DT[dt]), dev(w, DT[dt]))
    ref = O.h_hvp(p, inst.a, y, w)
    err = np.abs(host(out) - ref).max() / np.abs(ref).max()
    print(f"   {err:.2e}", flush=True)
    assert err <= (2e-6 if dt == "f32" else 1e-12)


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("C,H,W,K", SHAPES)
def test_ift_step(C, H, W, K, dt):
    print(f"[case] ift_step {C}x{H}x{W} K={K} {dt}", flush=True)
    inst, p, m, y = setup(C, H, W, K, dt)
    lam, n_lower, step = 0.4, 40, 0.05
    th0 = inst.a + 0.02 * np.random.default_rng(4).standard_normal(inst.a.shape)
    st = MaidState(dev(th0, torch.float64), dev(y, DT[dt]), torch.zeros((C, H, W), dtype=DT[dt], device="cuda"),
                   step=step)
    rc, info = m.ift_step(dev(inst.a, torch.float64), dev(y, DT[dt]), st, n_lower=n_lower, lambda_x=lam,
                          cg_tol=1e-6, max_cg=3000)
    assert rc == L.OK and info["lower_iters"] == n_lower and st.k == 1
    xg = host(st.x)
    xr, _ = O.gd_solve(p, th0, y, y, lam, n_lower)
    grad, g, _ = O.upper_value_grad(p, inst.a, y, xg)
    qr, _ = O.adjoint_solve(p, th0, xg, grad, tol=0.0, max_iter=info["cg_iters"])
    zr, _ = O.hypergrad(p, th0, inst.a, y, xg, host(st.q), with_r=True)
    zg = (th0 - host(st.theta)) / step
    ex, eq, ez = rel(xg, xr), rel(host(st.q), qr), rel(zg, zr)
    el = abs(info["ell_k"] - (g + O.sobolev_value(p, th0, inst.a))) / abs(g)
    print(f"   x {ex:.2e}  CG {info['cg_iters']} it: q {eq:.2e}  z {ez:.2e}  loss {el:.2e}", flush=True)
    assert max(ex, eq, ez, el) <= TOL[dt]


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("C,H,W,K", SHAPES)
def test_lista_step(C, H, W, K, dt):
    print(f"[case] lista_step {C}x{H}x{W} K={K} {dt}", flush=True)
    inst, p, m, y = setup(C, H, W, K, dt)
    lam, n, step = 0.4, 12, 0.05
    th0 = inst.a + 0.02 * np.random.default_rng(5).standard_normal(inst.a.shape)
    st = MaidState(dev(th0, torch.float64), dev(y, DT[dt]), torch.zeros((C, H, W), dtype=DT[dt], device="cuda"),
                   step=step)
    rc, info = m.lista_step(dev(inst.a, torch.float64), dev(y, DT[dt]), st, n_unroll=n, lambda_x=lam)
    assert rc == L.OK and info["lower_iters"] == n and info["cg_iters"] == n - 1 and st.k == 1
    gr, F, xr = O.lista_grad(p, inst.a, y, th0, y, n, lam)
    zg = (th0 - host(st.theta)) / step
    ex, ez = rel(host(st.x), xr), rel(zg, gr)
    el = abs(info["ell_k"] - F) / abs(F)
    en = abs(info["znorm"] - np.linalg.norm(gr)) / np.linalg.norm(gr)
    print(f"   x_n {ex:.2e}  dtheta {ez:.2e}  loss {el:.2e}  |dtheta| {en:.2e}", flush=True)
    assert max(ex, ez, el, en) <= TOL[dt]


@pytest.mark.skip(reason="the one-pass forms are opt-in and kept off the GPU: GPUs were lost while one-pass tests ran (no fault message in the process; cause not found) and a later benchmark run that included them faulted the GPU; kept off until a cause is shown")
def test_kept_iterates_need_the_two_pass_form():
    print("[case] ADP error paths", flush=True)
    inst = synth.make("cfg1", H=48, W=64, C=1, K=5, seed=9)
    m = Maid(1, 48, 64, 5, torch.float32, alpha=inst.alpha, eps_tv=inst.eps_tv)
    m.set_one_pass(1)
    assert m.one_pass_forms() == [1]
    th, y = dev(inst.a, torch.float64), dev(inst.y, torch.float32)
    hist = torch.zeros((4, 1, 48, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(L.MaidError, match="two-pass"):
        m.gd_solve(th, y, y.clone(), 0.3, 4, hist=hist)
    st = MaidState(th.clone(), y.clone(), torch.zeros_like(y), step=0.1)
    with pytest.raises(L.MaidError, match="two-pass"):
        m.lista_step(th, y, st, n_unroll=4)
    with pytest.raises(L.MaidError, match="step"):
        m.gd_solve(th, y, y.clone(), 0.0, 4)
    # without kept iterates the one-pass form runs the fixed-step iteration too
    x1 = y.clone()
    m.gd_solve(th, y, x1, 0.3, 10)
    m.set_one_pass(0)
    x0 = y.clone()
    m.gd_solve(th, y, x0, 0.3, 10)
    assert float((x1 - x0).norm() / x0.norm()) <= 1e-5
