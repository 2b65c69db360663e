"""Batched (ragged) form through the C ABI: one context over instances of
different sizes, channel counts, kernel sizes and regularisation weights.

The property checked is that batching changes nothing: every instance's
lower-level solve, CG solve and MAID iterations are bitwise those of a
context created for that instance alone (same tile configuration), and a
failing instance leaves the others untouched.  The small batch is also
checked against the FP64 oracle directly; the 64-instance ragged batch at its
full sizes is checked on a sample of instances against solo runs."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2502_09758_amd import _lib as L
from paper_2502_09758_amd import synth
from paper_2502_09758_amd.maid import Maid, MaidBatch, MaidState

pytestmark = pytest.mark.gpu


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda").contiguous()


def small_batch():
    """Ragged instances covering C in {1,3}, K in {3..15}, ragged tile tails."""
    shapes = [(1, 40, 70, 5), (3, 67, 33, 7), (1, 130, 96, 9), (3, 21, 150, 3), (1, 96, 96, 15), (1, 64, 64, 9)]
    out = []
    for i, (C, H, W, K) in enumerate(shapes):
        inst = synth.make("cfg1", H=H, W=W, C=C, K=K, seed=700 + i)
        inst.alpha = [1e-3, 5e-4, 2e-3, 1e-3, 3e-4, 1e-3][i]
        out.append(inst)
    return out


def spec(inst):
    return dict(C=inst.C, H=inst.H, W=inst.W, K=inst.K, alpha=inst.alpha, eps_tv=inst.eps_tv, beta=inst.beta)


def solo(inst, dt):
    return Maid(inst.C, inst.H, inst.W, inst.K, dt, alpha=inst.alpha, eps_tv=inst.eps_tv, beta=inst.beta)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_batch_lower_and_adjoint_equal_solo_bitwise(dt):
    print(f"[case] batch lower+adjoint == solo, {dt}", flush=True)
    insts = small_batch()
    mb = MaidBatch([spec(i) for i in insts], dt)
    th = [dev(i.a, torch.float64) for i in insts]
    ys = [dev(i.y, dt) for i in insts]
    xs = [y.clone() for y in ys]
    tols = [1e-3 if dt == torch.float32 else 1e-5] * len(insts)
    rc, infos = mb.lower_solve(th, ys, xs, tols, max_iter=500)
    assert rc in (L.OK, L.MAXITER)
    grads = [torch.randn_like(y) for y in ys]
    qs = [torch.zeros_like(y) for y in ys]
    rc2, cinfos = mb.adjoint_solve(th, xs, grads, qs, [1e-4 * float(g.norm()) for g in grads], max_iter=2000)
    assert rc2 in (L.OK, L.MAXITER)
    for k, inst in enumerate(insts):
        m = solo(inst, dt)
        x = ys[k].clone()
        info = m.lower_solve(th[k], ys[k], x, tols[k], max_iter=500)
        assert (info.status, info.iters, info.backtracks) == (infos[k].status, infos[k].iters, infos[k].backtracks)
        assert info.L == infos[k].L and info.res_norm == infos[k].res_norm
        assert torch.equal(x, xs[k]), f"instance {k}: batched lower solve differs from solo"
        q = torch.zeros_like(x)
        ci = m.adjoint_solve(th[k], x, grads[k], q, 1e-4 * float(grads[k].norm()), max_iter=2000)
        assert (ci.status, ci.iters, ci.res_norm) == (cinfos[k].status, cinfos[k].iters, cinfos[k].res_norm)
        assert torch.equal(q, qs[k]), f"instance {k}: batched CG differs from solo"
        m.close()
    mb.close()


def test_batch_lower_matches_oracle():
    """Each instance of the ragged FP64 batch against the oracle replaying the
    GPU's backtracking decisions (trace from the equal solo run)."""
    print("[case] batch lower vs oracle, f64", flush=True)
    insts = small_batch()
    mb = MaidBatch([spec(i) for i in insts], torch.float64)
    th = [dev(i.a, torch.float64) for i in insts]
    ys = [dev(i.y, torch.float64) for i in insts]
    xs = [y.clone() for y in ys]
    rc, infos = mb.lower_solve(th, ys, xs, [1e-4] * len(insts), max_iter=3000)
    assert rc == L.OK
    for k, inst in enumerate(insts):
        m = solo(inst, torch.float64)
        x = ys[k].clone()
        info = m.lower_solve(th[k], ys[k], x, 1e-4, max_iter=3000, trace=True)
        assert torch.equal(x, xs[k])
        p = O.Problem.of(inst)
        xo, oi, _ = O.lower_solve(p, inst.a, inst.y, inst.y, tol=0.0, max_iter=info.iters, L=0.0, replay_bt=info.trace)
        err = np.abs(xs[k].cpu().numpy() - xo).max() / max(1e-30, np.abs(xo).max())
        print(f"[batch-oracle] instance {k} {inst.C}x{inst.H}x{inst.W} K={inst.K}: iters {info.iters} rel {err:.2e}",
              flush=True)
        assert err <= 1e-9
        m.close()
    mb.close()


def test_batch_maid_steps_equal_solo_bitwise():
    print("[case] batch maid_step x3 == solo, f32", flush=True)
    dt = torch.float32
    insts = small_batch()[:4]
    mb = MaidBatch([spec(i) for i in insts], dt)
    a = [dev(i.a, torch.float64) for i in insts]
    ys = [dev(i.y, dt) for i in insts]

    def fresh(k):
        return MaidState(a[k].clone(), ys[k].clone(), torch.zeros_like(ys[k]), eps=1e-3, delta=1e-3, step=1e-3)

    bst = [fresh(k) for k in range(len(insts))]
    hp = dict(eps_min=1e-6)
    binfo = []
    for _ in range(3):
        rc, infos = mb.maid_step(a, ys, bst, **hp)
        binfo.append(infos)
    for k, inst in enumerate(insts):
        m = solo(inst, dt)
        s = fresh(k)
        for it in range(3):
            rc, info = m.maid_step(a[k], ys[k], s, **hp)
            assert info == binfo[it][k], f"instance {k} step {it}: {info} vs {binfo[it][k]}"
        assert torch.equal(s.theta, bst[k].theta) and torch.equal(s.x, bst[k].x) and torch.equal(s.q, bst[k].q)
        assert (s.eps, s.delta, s.step, s.L, s.k) == (bst[k].eps, bst[k].delta, bst[k].step, bst[k].L, bst[k].k)
        m.close()
    mb.close()


def test_batch_multi_step_call_equals_single_steps():
    """maid_batch_steps(n = 4) in one call: bitwise the states of four
    maid_batch_step calls, the counts summed over the steps, the last step's
    values."""
    print("[case] maid_batch_steps(4) == 4 x maid_batch_step, f32", flush=True)
    dt = torch.float32
    insts = small_batch()[:4]
    a = [dev(i.a, torch.float64) for i in insts]
    ys = [dev(i.y, dt) for i in insts]

    def fresh():
        return [MaidState(a[k].clone(), ys[k].clone(), torch.zeros_like(ys[k]), eps=1e-3, delta=1e-3, step=1e-3)
                for k in range(len(insts))]

    hp = dict(eps_min=1e-12)
    mb = MaidBatch([spec(i) for i in insts], dt)
    one = fresh()
    steps = [mb.maid_step(a, ys, one, **hp)[1] for _ in range(4)]
    print("   statuses per step: " + str([[f["status"] for f in st] for st in steps]), flush=True)
    # no instance ends its run early here (else the single calls go on where the multi-step call stops)
    assert all(st[k]["status"] in (L.OK, L.MAXITER) for st in steps[:-1] for k in range(len(insts)))
    many = fresh()
    rc, tot = mb.maid_steps(a, ys, many, 4, **hp)
    assert rc in (L.OK, L.MAXITER), rc
    for k in range(len(insts)):
        assert torch.equal(one[k].theta, many[k].theta) and torch.equal(one[k].x, many[k].x)
        assert torch.equal(one[k].q, many[k].q)
        assert (one[k].eps, one[k].delta, one[k].step, one[k].L, one[k].k) == \
            (many[k].eps, many[k].delta, many[k].step, many[k].L, many[k].k)
        for f in ("accepted", "trials", "retries", "lower_iters", "cg_iters"):
            assert tot[k][f] == sum(st[k][f] for st in steps), (k, f)
        for f in ("psi", "ell_k", "ell_next", "znorm"):
            assert tot[k][f] == steps[-1][k][f], (k, f)
    mb.close()


def test_batch_failing_instance_isolated():
    """A NaN in one instance's data: that instance reports NONFINITE and keeps
    its x unwritten; every other instance equals its solo run."""
    print("[case] batch with one non-finite instance", flush=True)
    dt = torch.float32
    insts = small_batch()[:3]
    mb = MaidBatch([spec(i) for i in insts], dt)
    th = [dev(i.a, torch.float64) for i in insts]
    ys = [dev(i.y, dt) for i in insts]
    ys[1][0, 3, 4] = float("nan")
    xs = [torch.full_like(y, 0.25) for y in ys]
    rc, infos = mb.lower_solve(th, ys, xs, [1e-3] * 3, max_iter=300)
    assert rc == L.NONFINITE and infos[1].status == L.NONFINITE
    assert torch.all(xs[1] == 0.25)
    for k in (0, 2):
        m = solo(insts[k], dt)
        x = torch.full_like(ys[k], 0.25)
        info = m.lower_solve(th[k], ys[k], x, 1e-3, max_iter=300)
        assert info.status == infos[k].status and torch.equal(x, xs[k])
        m.close()
    mb.close()


def test_batch_tile_rows_override():
    print("[case] batch with forced tile rows 2 == solo with rows 2", flush=True)
    dt = torch.float32
    insts = small_batch()[:3]
    mb = MaidBatch([spec(i) for i in insts], dt)
    mb.set_tile_rows(2)
    th = [dev(i.a, torch.float64) for i in insts]
    ys = [dev(i.y, dt) for i in insts]
    xs = [y.clone() for y in ys]
    mb.lower_solve(th, ys, xs, [1e-3] * 3, max_iter=300)
    for k in range(3):
        m = solo(insts[k], dt)
        m.set_tile_rows(2)
        x = ys[k].clone()
        m.lower_solve(th[k], ys[k], x, 1e-3, max_iter=300)
        assert torch.equal(x, xs[k])
        m.close()
    mb.close()


def test_ragged_64_instance_batch_full_size():
    """The 64-instance ragged batch (H, W in 128..1024, C in {1,3}, K in 5..21)
    at full size: every lower solve converges; three sampled instances equal
    their solo runs bitwise."""
    print("[case] ragged 64-instance batch, full size, f32", flush=True)
    dt = torch.float32
    insts = synth.make_batch()
    mb = MaidBatch([spec(i) for i in insts], dt)
    th = [dev(i.a, torch.float64) for i in insts]
    ys = [dev(i.y, dt) for i in insts]
    xs = [y.clone() for y in ys]
    rc, infos = mb.lower_solve(th, ys, xs, [1e-2] * len(insts), max_iter=300)
    print(f"[ragged] rc {rc}, iters {[i.iters for i in infos]}", flush=True)
    assert all(i.status in (L.OK, L.MAXITER) for i in infos)
    assert all(torch.isfinite(x).all() for x in xs)
    for k in (0, 17, 63):
        m = solo(insts[k], dt)
        x = ys[k].clone()
        info = m.lower_solve(th[k], ys[k], x, 1e-2, max_iter=300)
        assert info.iters == infos[k].iters and torch.equal(x, xs[k]), f"instance {k}"
        m.close()
    mb.close()


def test_autotune_plain_and_batch():
    """The autotuner picks a valid tile height per K group, writes nothing the
    caller owns, and a solve afterwards equals a solo solve forced to the
    chosen tile height (bitwise)."""
    print("[case] autotune plain + batch", flush=True)
    dt = torch.float32
    insts = small_batch()[:4]
    th = [dev(i.a, torch.float64) for i in insts]
    ys = [dev(i.y, dt) for i in insts]
    ys_before = [y.clone() for y in ys]
    m = solo(insts[2], dt)
    r = m.autotune(th[2], ys[2], probe_iters=4)
    assert r in (1, 2, 4) and f"rows_per_thread={r}" in m.config()
    assert torch.equal(ys[2], ys_before[2])
    mb = MaidBatch([spec(i) for i in insts], dt)
    rows = mb.autotune(th, ys, probe_iters=4)
    assert len(rows) == len(insts) and all(v in (1, 2, 4) for v in rows)
    for k in range(len(insts)):
        assert torch.equal(ys[k], ys_before[k])
        for j in range(len(insts)):
            if insts[j].K == insts[k].K:
                assert rows[j] == rows[k]
    xs = [y.clone() for y in ys]
    mb.lower_solve(th, ys, xs, [1e-3] * len(insts), max_iter=300)
    for k in range(len(insts)):
        ms = solo(insts[k], dt)
        ms.set_tile_rows(rows[k])
        x = ys[k].clone()
        ms.lower_solve(th[k], ys[k], x, 1e-3, max_iter=300)
        assert torch.equal(x, xs[k]), f"instance {k}"
        ms.close()
    m.close()
    mb.close()


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_batch_upper_and_hypergrad_equal_solo_bitwise(dt):
    print(f"[case] batch upper_value_grad + hypergrad == solo, {dt}", flush=True)
    insts = small_batch()
    for i in insts:
        i.beta = i.alpha / 2
    mb = MaidBatch([spec(i) for i in insts], dt)
    th = [dev(i.a + 0.01 * synth.directions(1, i.K, seed=5)[0], torch.float64) for i in insts]
    a = [dev(i.a, torch.float64) for i in insts]
    ys = [dev(i.y, dt) for i in insts]
    gen = torch.Generator(device="cuda").manual_seed(3)
    xs = [y + 0.01 * torch.randn(y.shape, generator=gen, device="cuda", dtype=dt) for y in ys]
    qs = [torch.randn(y.shape, generator=gen, device="cuda", dtype=dt) for y in ys]
    grads = [torch.empty_like(y) for y in ys]
    g, gn = mb.upper_value_grad(a, ys, xs, grads)
    zs, zn = mb.hypergrad(th, a, ys, xs, qs, with_r=True)
    for k, inst in enumerate(insts):
        m = solo(inst, dt)
        gk = torch.empty_like(ys[k])
        gv, gnv = m.upper_value_grad(a[k], ys[k], xs[k], gk)
        assert (gv, gnv) == (g[k], gn[k]) and torch.equal(gk, grads[k])
        z, znv = m.hypergrad(th[k], a[k], ys[k], xs[k], qs[k], with_r=True)
        assert znv == zn[k] and torch.equal(z, zs[k]), f"instance {k}"
        m.close()
    mb.close()
