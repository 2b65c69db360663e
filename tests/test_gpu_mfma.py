"""The matrix-core correlations (FP32 storage, K >= 13, 4 or 8 rows per
thread) against the FP64 oracle, and against the vector-ALU path.

Each FP32 operand is split into two FP16 parts and the product formed from
three FP16 products accumulated in FP32, so a correlation lands within a
few 1e-7 of the exact one relative to its largest output (the vector path's
FP32 sums are of the same order).  Solvers are compared by decision replay
at the FP32 bar of 1e-5 relative.  Instances here are above the team loops'
size rule, so the multi-kernel passes run."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2502_09758_amd import _lib as L
from paper_2502_09758_amd import synth
from paper_2502_09758_amd.maid import Maid, MaidBatch

pytestmark = pytest.mark.gpu


def dev(a, dt=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda").contiguous()


def host(t):
    return t.detach().double().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def problem(C, H, W, K, seed=1):
    inst = synth.make("cfg1", H=H, W=W, C=C, K=K, seed=seed)
    p = O.Problem(C, H, W, K, alpha=inst.alpha, eps_tv=inst.eps_tv, beta=inst.beta)
    return inst, p


CONV = [(1, 70, 150, 13, 4), (3, 70, 100, 15, 4), (3, 70, 100, 15, 8), (1, 90, 130, 21, 8), (2, 75, 140, 31, 4),
        (1, 90, 130, 31, 8)]


@pytest.mark.parametrize("C,H,W,K,R", CONV)
def test_operator_matches_oracle(C, H, W, K, R):
    """theta*x and its adjoint, matrix cores and vector ALUs, against the
    oracle: max error over the largest output magnitude."""
    print(f"[case] mfma operator C={C} H={H} W={W} K={K} R={R}", flush=True)
    inst, p = problem(C, H, W, K)
    rng = np.random.default_rng(11)
    th = inst.a + 0.2 * rng.standard_normal(inst.a.shape) * np.abs(inst.a).max()   # mixed signs
    x = f32(rng.standard_normal((C, H, W)))
    m = Maid(C, H, W, K, torch.float32, alpha=p.alpha, eps_tv=p.eps_tv)
    m.set_tile_rows(R)
    assert "mfma" in m.config(), m.config()
    ref = {0: O.conv(p, th, x), 1: O.conv_adj(p, th, x)}
    for mf in (True, False):
        m.set_mfma(mf)
        assert ("mfma" in m.config()) == mf
        for adj in (0, 1):
            out = torch.empty((C, H, W), dtype=torch.float32, device="cuda")
            m.apply_operator(dev(th, torch.float64), dev(x), out, adjoint=adj)
            err = np.abs(host(out) - ref[adj]).max() / np.abs(ref[adj]).max()
            print(f"   mfma={mf} adjoint={adj}: {err:.2e}", flush=True)
            assert err <= 2e-6, (mf, adj, err)
    m.close()


SOLVE = [(3, 70, 100, 15, 4), (1, 90, 130, 31, 8), (2, 60, 140, 21, 8)]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("C,H,W,K,R", SOLVE)
def test_solvers_match_oracle(C, H, W, K, R):
    """Lower-level solve (decision replay), CG at equal iteration counts and
    the hypergradient, on the matrix-core passes."""
    print(f"[case] mfma solvers C={C} H={H} W={W} K={K} R={R}", flush=True)
    inst, p = problem(C, H, W, K, seed=6)
    y = f32(inst.y)
    m = Maid(C, H, W, K, torch.float32, alpha=p.alpha, eps_tv=p.eps_tv, beta=p.beta)
    m.set_tile_rows(R)
    assert "mfma" in m.config(), m.config()
    th = dev(inst.a, torch.float64)
    x = dev(y)
    info = m.lower_solve(th, dev(y), x, 3e-3, max_iter=3000, trace=True)
    assert info.status == L.OK and info.iters > 3
    xr, _, _ = O.lower_solve(p, inst.a, y, y, tol=0.0, max_iter=info.iters, L=0.0, replay_bt=info.trace)
    ex = rel(host(x), xr)
    xt = host(x)
    b, _, _ = O.upper_value_grad(p, inst.a, y, xt)
    b = f32(b)
    q = torch.zeros((C, H, W), dtype=torch.float32, device="cuda")
    ci = m.adjoint_solve(th, x, dev(b), q, 1e-2 * np.linalg.norm(b), max_iter=2000)
    assert ci.status == L.OK
    qr, _ = O.adjoint_solve(p, inst.a, xt, b, tol=0.0, max_iter=ci.iters)
    eq = rel(host(q), qr)
    z, _ = m.hypergrad(th, th, dev(y), x, q)
    zr, _ = O.hypergrad(p, inst.a, inst.a, y, xt, host(q))
    ez = rel(host(z), zr)
    print(f"   lower {info.iters} it: x {ex:.2e}; CG {ci.iters} it: q {eq:.2e}; z {ez:.2e}", flush=True)
    assert ex <= 1e-5 and eq <= 1e-5 and ez <= 1e-5
    m.close()


def test_deterministic_and_batch_equals_solo():
    """The matrix-core passes give bitwise the same results run twice, and
    an instance alone or inside a ragged batch."""
    shapes = [(1, 70, 150, 13), (3, 60, 90, 15), (1, 50, 300, 13)]
    print("[case] mfma determinism and batch " + str(shapes), flush=True)
    insts = [problem(C, H, W, K, seed=20 + k)[0] for k, (C, H, W, K) in enumerate(shapes)]
    specs = [dict(C=i.C, H=i.H, W=i.W, K=i.K, alpha=i.alpha, eps_tv=i.eps_tv) for i in insts]
    ths = [dev(i.a, torch.float64) for i in insts]
    ys = [dev(f32(i.y)) for i in insts]
    mb = MaidBatch(specs, torch.float32)
    mb.set_tile_rows(4)
    assert "mfma" in mb.config()
    outs = []
    for _ in range(2):
        xs = [y.clone() for y in ys]
        mb.lower_solve(ths, ys, xs, [2e-3] * len(insts), max_iter=500)
        qs = [torch.zeros_like(y) for y in ys]
        mb.adjoint_solve(ths, xs, ys, qs, [1e-2] * len(insts), max_iter=500)
        outs.append((xs, qs))
    for a, b in zip(outs[0][0] + outs[0][1], outs[1][0] + outs[1][1]):
        assert torch.equal(a, b)
    for k, i in enumerate(insts):
        m = Maid(i.C, i.H, i.W, i.K, torch.float32, alpha=i.alpha, eps_tv=i.eps_tv)
        m.set_tile_rows(4)
        x = ys[k].clone()
        m.lower_solve(ths[k], ys[k], x, 2e-3, max_iter=500)
        q = torch.zeros_like(x)
        m.adjoint_solve(ths[k], x, ys[k], q, 1e-2, max_iter=500)
        assert torch.equal(x, outs[0][0][k]) and torch.equal(q, outs[0][1][k]), k
        m.close()
    mb.close()
