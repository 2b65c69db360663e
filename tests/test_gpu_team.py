"""Persistent team loops (one team of blocks per XCD, barriers through the
XCD's L2) against the multi-kernel passes, through the C ABI.

The team loops run the same pass bodies over the same tiles and sum the same
partials in the same order, so every result must be bitwise that of the
multi-kernel path: iterates, CG solutions, iteration and backtracking
counts, Lipschitz estimates, residual norms, backtracking traces and MAID
steps.  Team sizes from one block to more blocks than tiles (capped), ragged
tile tails, three channels, both storage types, and batches with more
instances than XCDs (a team then serves several instances in turn).  The
fallback (a team that cannot assemble) is forced from the host with a zero
barrier wait: the kernels leave at their first wait and the solve is
repeated on the multi-kernel passes."""
import os

import numpy as np
import pytest
import torch

from paper_2502_09758_amd import _lib as L
from paper_2502_09758_amd import synth
from paper_2502_09758_amd.maid import Maid, MaidBatch, MaidState

pytestmark = pytest.mark.gpu

SHAPES = [(1, 40, 70, 5), (3, 67, 33, 7), (1, 130, 96, 9), (1, 64, 64, 3), (3, 45, 90, 11)]


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda").contiguous()


def solo(inst, dt):
    return Maid(inst.C, inst.H, inst.W, inst.K, dt, alpha=inst.alpha, eps_tv=inst.eps_tv, beta=inst.beta)


def solve_pair(m, inst, dt, tol):
    th = dev(inst.a, torch.float64)
    y = dev(inst.y, dt)
    x = y.clone()
    info = m.lower_solve(th, y, x, tol, max_iter=400, trace=True)
    g = dev(np.sin(np.arange(y.numel()).reshape(y.shape) * 0.37), dt) * 0.05 + y * 0.1
    q = torch.zeros_like(y)
    ci = m.adjoint_solve(th, x, g, q, 1e-4 * float(g.norm()), max_iter=600)
    return x, q, info, ci


def same_info(a, b):
    return (a.status, a.iters, a.backtracks, a.L, a.res_norm) == (b.status, b.iters, b.backtracks, b.L, b.res_norm)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("shape", SHAPES)
def test_team_loops_bitwise_equal_multikernel(dt, shape):
    C, H, W, K = shape
    print(f"[case] team vs multi-kernel {shape} {dt}", flush=True)
    inst = synth.make("cfg1", H=H, W=W, C=C, K=K, seed=900 + K)
    tol = 1e-4 if dt == torch.float32 else 1e-6
    m = solo(inst, dt)
    m.set_team(0)
    assert "team=" not in m.config()
    ref = solve_pair(m, inst, dt, tol)
    for members in (1, 5, -1, 128):
        m.set_team(members)
        # -1 (the size rule) takes the team path only up to 64 tiles
        assert members == -1 or "team=" in m.config(), m.config()
        got = solve_pair(m, inst, dt, tol)
        assert torch.equal(ref[0], got[0]), f"members={members}: lower-level iterate differs"
        assert torch.equal(ref[1], got[1]), f"members={members}: CG solution differs"
        assert same_info(ref[2], got[2]), (members, ref[2], got[2])
        assert same_info(ref[3], got[3]), (members, ref[3], got[3])
        assert ref[2].trace == got[2].trace
    m.close()


@pytest.mark.parametrize("rows", [1, 2, 4])
def test_team_loops_every_tile_height(rows):
    print(f"[case] team vs multi-kernel, rows {rows}", flush=True)
    inst = synth.make("cfg1", H=72, W=150, C=1, K=9, seed=77)
    m = solo(inst, torch.float32)
    m.set_tile_rows(rows)
    m.set_team(0)
    ref = solve_pair(m, inst, torch.float32, 1e-4)
    m.set_team(-1)
    assert "team=" in m.config()
    got = solve_pair(m, inst, torch.float32, 1e-4)
    assert torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])
    assert same_info(ref[2], got[2]) and same_info(ref[3], got[3])
    m.close()


def tiny_batch(n):
    """n instances, several per K (ragged sizes within a group)."""
    out = []
    for i in range(n):
        K = (3, 5, 7)[i % 3]
        H, W = 20 + 3 * i, 80 - 2 * i
        inst = synth.make("cfg1", H=H, W=W, C=1 + 2 * (i % 2), K=K, seed=1200 + i)
        inst.alpha = 1e-3 * (1 + i % 4)
        out.append(inst)
    return out


def spec(inst):
    return dict(C=inst.C, H=inst.H, W=inst.W, K=inst.K, alpha=inst.alpha, eps_tv=inst.eps_tv, beta=inst.beta)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_team_batch_more_instances_than_xcds(dt):
    print(f"[case] team batch of 19, {dt}", flush=True)
    insts = tiny_batch(19)
    th = [dev(i.a, torch.float64) for i in insts]
    ys = [dev(i.y, dt) for i in insts]
    tols = [1e-4 if dt == torch.float32 else 1e-6] * len(insts)
    grads = [y * 0.1 + 0.01 for y in ys]
    res = []
    for members in (0, -1, 3):
        mb = MaidBatch([spec(i) for i in insts], dt)
        mb.set_team(members)
        assert ("team=" in mb.config()) == (members != 0), mb.config()
        xs = [y.clone() for y in ys]
        rc, infos = mb.lower_solve(th, ys, xs, tols, max_iter=400)
        assert rc in (L.OK, L.MAXITER)
        qs = [torch.zeros_like(y) for y in ys]
        rc2, cinfos = mb.adjoint_solve(th, xs, grads, qs, [1e-4 * float(g.norm()) for g in grads], max_iter=600)
        assert rc2 in (L.OK, L.MAXITER)
        res.append((xs, qs, infos, cinfos))
        mb.close()
    for k in range(1, len(res)):
        for i in range(len(insts)):
            assert torch.equal(res[0][0][i], res[k][0][i]), f"instance {i}: lower-level iterate differs"
            assert torch.equal(res[0][1][i], res[k][1][i]), f"instance {i}: CG solution differs"
            assert same_info(res[0][2][i], res[k][2][i])
            assert same_info(res[0][3][i], res[k][3][i])


def test_team_maid_steps_bitwise():
    """Algorithm 2 iterations (InexactGradient, psi trials, step control) on
    the team loops equal those on the multi-kernel passes."""
    print("[case] team MAID steps", flush=True)
    inst = synth.make("cfg1", H=64, W=96, C=1, K=7, seed=31)
    out = []
    for members in (0, -1):
        m = solo(inst, torch.float32)
        m.set_team(members)
        assert ("team=" in m.config()) == (members != 0)
        a = dev(inst.a, torch.float64)
        y = dev(inst.y, torch.float32)
        st = MaidState(a.clone(), y.clone(), torch.zeros_like(y), eps=1e-3, delta=1e-3, step=1e-3)
        infos = []
        for _ in range(4):
            rc, info = m.maid_step(a, y, st)
            assert rc >= 0
            infos.append(tuple(sorted(info.items())))
        out.append((st.theta.clone(), st.x.clone(), infos))
        m.close()
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]


def test_team_fallback_when_a_team_cannot_assemble():
    """Zero barrier wait: members leave at their first wait, the error word is
    raised, and the solve is repeated on the multi-kernel passes."""
    print("[case] team fallback", flush=True)
    inst = synth.make("cfg1", H=64, W=64, C=1, K=5, seed=8)
    m = solo(inst, torch.float32)
    m.set_team(0)
    ref = solve_pair(m, inst, torch.float32, 1e-4)
    m.close()
    os.environ["MAID_TEAM_WAIT"] = "0"
    try:
        m = solo(inst, torch.float32)
    finally:
        del os.environ["MAID_TEAM_WAIT"]
    m.set_team(16)
    assert "team=16" in m.config()
    got = solve_pair(m, inst, torch.float32, 1e-4)
    assert "team=" not in m.config(), "the context should have left the team path"
    assert torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])
    assert same_info(ref[2], got[2]) and same_info(ref[3], got[3])
    m.close()


def test_team_size_rule():
    print("[case] team size rule", flush=True)
    small = synth.make("cfg1", H=64, W=64, C=1, K=9, seed=2)
    m = solo(small, torch.float32)
    m.set_tile_rows(1)
    assert "team=16" in m.config(), m.config()
    m.close()
    big = synth.make("cfg1", H=256, W=256, C=1, K=9, seed=2)
    m = solo(big, torch.float32)
    assert "team=" not in m.config(), m.config()
    m.close()


@pytest.mark.skip(reason="the one-pass forms are opt-in and kept off the GPU: GPUs were lost while one-pass tests ran (no fault message in the process; cause not found) and a later benchmark run that included them faulted the GPU; kept off until a cause is shown")
@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_team_one_pass_cg_bitwise(dt):
    """The opt-in one-pass CG on team loops equals it on kernels."""
    print(f"[case] team one-pass CG {dt}", flush=True)
    inst = synth.make("cfg1", H=64, W=96, C=1, K=7, seed=44)
    tol = 1e-4 if dt == torch.float32 else 1e-6
    out = []
    for members in (0, -1):
        m = solo(inst, dt)
        m.set_one_pass_cg(True)
        m.set_team(members)
        assert "cg-one-pass" in m.config() and ("team=" in m.config()) == (members != 0), m.config()
        out.append(solve_pair(m, inst, dt, tol))
        m.close()
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    assert same_info(out[0][2], out[1][2]) and same_info(out[0][3], out[1][3])
