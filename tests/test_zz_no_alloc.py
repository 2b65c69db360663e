"""maid_upper_value_grad_noalloc (the entry point for callers that cannot
allocate) against maid_upper_value_grad on a context of the same
description: the same kernels and tile rows, so bitwise-equal gradients and
equal values.  Two calls in a row share the library's fixed workspace, the
second on a smaller instance; an instance beyond the workspace is refused
before any GPU work."""
import ctypes as ct

import numpy as np
import pytest
import torch

from paper_2502_09758_amd import _lib as L
from paper_2502_09758_amd import synth
from paper_2502_09758_amd.maid import Maid

pytestmark = pytest.mark.gpu


def desc(C, H, W, K, dt, inst):
    return L.maid_desc(H=H, W=W, C=C, K=K, dtype=L.MAID_F64 if dt == torch.float64 else L.MAID_F32, boundary=0,
                       reg=L.MAID_REG_TV, alpha=inst.alpha, eps_tv=inst.eps_tv, beta=inst.beta, h1_w0=1.0)


def noalloc(d, a, y, x, grad):
    g, gn = ct.c_double(), ct.c_double()
    why = ct.c_char_p()
    rc = L.lib().maid_upper_value_grad_noalloc(ct.byref(d), a.data_ptr(), y.data_ptr(), x.data_ptr(),
                                               grad.data_ptr() if grad is not None else None,
                                               ct.byref(g), ct.byref(gn), ct.byref(why), None)
    return rc, g.value, gn.value, (why.value or b"").decode()


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_noalloc_matches_context_two_calls(dt):
    shapes = [(3, 300, 260, 15), (1, 96, 130, 9)]          # the second call on a smaller instance
    for C, H, W, K in shapes:
        print(f"[case] noalloc upper {dt} C={C} H={H} W={W} K={K}", flush=True)
        inst = synth.make("cfg1", H=H, W=W, C=C, K=K, seed=70 + K)
        rng = np.random.default_rng(K)
        a = torch.tensor(inst.a, dtype=torch.float64, device="cuda")
        y = torch.tensor(inst.y, dtype=dt, device="cuda")
        x = torch.tensor(inst.y + 0.02 * rng.standard_normal(inst.y.shape), dtype=dt, device="cuda")
        m = Maid(C, H, W, K, dt, alpha=inst.alpha, eps_tv=inst.eps_tv, beta=inst.beta)
        ref = torch.empty_like(y)
        g0, gn0 = m.upper_value_grad(a, y, x, ref)
        m.close()
        d = desc(C, H, W, K, dt, inst)
        out = torch.full_like(y, float("nan"))
        rc, g, gn, why = noalloc(d, a, y, x, out)
        assert rc == L.OK, why
        assert torch.equal(out, ref)
        assert g == g0 and gn == gn0
        # without grad_out: the gradient stays in the workspace, the values are the same
        rc, g2, gn2, why = noalloc(d, a, y, x, None)
        assert rc == L.OK, why
        assert g2 == g0 and gn2 == gn0


def test_noalloc_refuses_oversized_instance():
    inst = synth.make("cfg1", H=64, W=64, C=1, K=7, seed=1)
    d = L.maid_desc(H=4096, W=4096, C=3, K=7, dtype=L.MAID_F32, boundary=0, reg=L.MAID_REG_TV, alpha=inst.alpha,
                    eps_tv=inst.eps_tv, beta=0.0, h1_w0=1.0)
    t = torch.zeros(4, dtype=torch.float32, device="cuda")
    a = torch.zeros(49, dtype=torch.float64, device="cuda")
    rc, _, _, why = noalloc(d, a, t, t, t)
    assert rc == L.EINVAL and "64 MiB" in why
