"""Independent float64 reference of the lower- and upper-level objectives,
written with plain PyTorch CPU ops (conv2d, diff, autograd) for pinning the
oracle.  Shares nothing with the oracle's C code: the convolution is torch's
cross-correlation with a flipped kernel, differences are tensor slices, and
derivatives come from autograd instead of hand-written formulas."""
import torch
import torch.nn.functional as F

torch.set_default_dtype(torch.float64)


def t(a):
    return torch.as_tensor(a, dtype=torch.float64)


def conv(th, x, periodic=False):
    """(th*x)(i,j) = sum th(u,v) x(i+c0-u, j+c0-v): correlation with the flipped kernel.
    th (K, K) blurs every channel; th (C, K, K) blurs channel c with th[c]
    (a grouped convolution)."""
    K = th.shape[-1]
    c0 = (K - 1) // 2
    if th.dim() == 3:
        w = th.flip(-2, -1)[:, None]
        xx = x[None]
        if periodic:
            return F.conv2d(F.pad(xx, (c0, c0, c0, c0), mode="circular"), w, groups=th.shape[0])[0]
        return F.conv2d(xx, w, padding=c0, groups=th.shape[0])[0]
    w = th.flip(0, 1)[None, None]
    xx = x[:, None]
    if periodic:
        xx = F.pad(xx, (c0, c0, c0, c0), mode="circular")
        return F.conv2d(xx, w)[:, 0]
    return F.conv2d(xx, w, padding=c0)[:, 0]


def diffs(x, periodic=False):
    if periodic:
        return torch.roll(x, -1, dims=2) - x, torch.roll(x, -1, dims=1) - x
    dh = torch.zeros_like(x)
    dv = torch.zeros_like(x)
    dh[:, :, :-1] = x[:, :, 1:] - x[:, :, :-1]
    dv[:, :-1, :] = x[:, 1:, :] - x[:, :-1, :]
    return dh, dv


def reg(x, eps, mode=0, periodic=False):
    dh, dv = diffs(x, periodic)
    if mode == 2:
        return 0.5 * (dh * dh + dv * dv).sum()
    if mode == 0:
        s2 = (dh * dh + dv * dv).sum(0)
    else:
        s2 = dh * dh + dv * dv
    return (torch.sqrt(s2 + eps * eps) - eps).sum()


def h(th, y, x, alpha, eps, mode=0, periodic=False):
    r = conv(th, x, periodic) - y
    return 0.5 * (r * r).sum() + alpha * reg(x, eps, mode, periodic)


def g(a, y, x):
    r = conv(a, x) - y
    return 0.5 * (r * r).sum()


def sobolev(th, a, beta, w0=1.0):
    e = th - a
    e = e if e.dim() == 3 else e[None]     # one KxK grid per kernel channel
    dh, dv = diffs(e)
    return beta * (w0 * (e * e).sum() + (dh * dh).sum() + (dv * dv).sum())


def grad_h(th, y, x, alpha, eps, mode=0, periodic=False):
    x = x.clone().requires_grad_(True)
    v = h(th, y, x, alpha, eps, mode, periodic)
    (gx,) = torch.autograd.grad(v, x)
    return gx.detach()


def hess_h(th, y, x, alpha, eps, mode=0, periodic=False):
    """Dense Hessian d^2 h / dx^2 as an N x N matrix (autograd)."""
    n = x.numel()
    shape = x.shape

    def f(flat):
        return h(th, y, flat.reshape(shape), alpha, eps, mode, periodic)

    return torch.autograd.functional.hessian(f, x.reshape(-1).clone()).reshape(n, n)


def mixed_jac(th, y, x, alpha, eps, mode=0):
    """J = d(grad_x h)/d theta as an N x (number of taps) matrix (autograd)."""
    shape = th.shape

    def f(thf):
        return grad_h_graph(thf.reshape(shape), y, x, alpha, eps, mode).reshape(-1)

    return torch.autograd.functional.jacobian(f, th.reshape(-1).clone())


def grad_h_graph(th, y, x, alpha, eps, mode=0):
    x = x.clone().requires_grad_(True)
    v = h(th, y, x, alpha, eps, mode)
    (gx,) = torch.autograd.grad(v, x, create_graph=True)
    return gx


def newton_solve(th, y, x0, alpha, eps, mode=0, periodic=False, tol=1e-13, maxit=100):
    """Damped Newton with the dense autograd Hessian: the tight lower-level
    solution used as the reference limit object."""
    x = x0.clone()
    for _ in range(maxit):
        gx = grad_h(th, y, x, alpha, eps, mode, periodic)
        if gx.norm() <= tol:
            break
        Hm = hess_h(th, y, x, alpha, eps, mode, periodic)
        step = torch.linalg.solve(Hm, gx.reshape(-1)).reshape(x.shape)
        f0 = h(th, y, x, alpha, eps, mode, periodic)
        s = 1.0
        while s > 1e-8:
            xn = x - s * step
            if h(th, y, xn, alpha, eps, mode, periodic) <= f0 + 1e-16 * abs(float(f0)):
                break
            s *= 0.5
        x = xn
    return x
