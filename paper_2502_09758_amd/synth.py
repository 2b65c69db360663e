"""Seeded synthetic workloads for semi-blind deblurring with MAID.

The paper's experiments (Section 4.2: 300x400x3 colour images, 5x5 motion and
Gaussian kernels, noise 0.02) use images that are not available, so every
input here is drawn from a fixed-seed generator with the structure of those
workloads: piecewise-constant colour images (flat regions plus sharp edges,
which is what smoothed TV is built for), an optional smooth texture, a known
blur kernel that is only approximately right (the semi-blind setting of
Section 4.2, where the assumed kernel b0 differs from the true blur), and
additive Gaussian noise.

This module only *makes data*.  It holds none of the method's arithmetic: the
blurred data is produced with ``scipy.signal.fftconvolve`` (zero boundary,
"same" output size, true convolution), a library routine that neither the
oracle nor the HIP path uses.  Both sides consume exactly the float64 arrays
made here (cast to float32 for the FP32 path).

Workload table (sizes, kernels, noise, regularisation weights):

========  =============  ======  ======================  ===================  ======  =======
name      H x W x C      K       true blur               assumed kernel a     noise   alpha
========  =============  ======  ======================  ===================  ======  =======
cfg1      64x64x1        7       Gaussian s=1.5          Gaussian s=1.0       0.01    1e-3
cfg2      256x256x1      9       Gaussian s=2.0          Gaussian s=4/3       0.02    5e-4
cfg3      512x512x3      15      aniso s=(3,1.5), 30deg  Gaussian s=1.5       0.01    2e-4
cfg4      64 instances   5..21   Gaussian s=K/6          Gaussian s=K/9       U[.005,.03]  logU[1e-4,1e-2]
cfg5      2048x2048x3    31      21px line at 45deg*G1   raw 21px line        0.01    1e-4
paper     300x400x3      5       diag motion * G0.5      diag motion          0.02    0.3
========  =============  ======  ======================  ===================  ======  =======

The TV smoothing parameter is 1e-2 everywhere and the upper-level Sobolev
weight is beta = alpha/2, the ratio of the paper's 2D weights (Section 4.2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.signal import fftconvolve

__all__ = [
    "Instance", "CONFIGS", "make", "make_batch", "gaussian_kernel",
    "anisotropic_kernel", "motion_kernel", "piecewise_constant",
    "value_noise", "blur_same", "directions",
]


# ----------------------------------------------------------------------------
# kernels (all normalised to unit sum, centred at (c0, c0), c0 = (K-1)/2)
# ----------------------------------------------------------------------------
def _offsets(K: int):
    c0 = (K - 1) // 2
    ii, jj = np.meshgrid(np.arange(K) - c0, np.arange(K) - c0, indexing="ij")
    return ii.astype(np.float64), jj.astype(np.float64)


def gaussian_kernel(K: int, sigma: float) -> np.ndarray:
    """Isotropic Gaussian exp(-(di^2+dj^2)/(2 sigma^2)) on a KxK grid."""
    di, dj = _offsets(K)
    k = np.exp(-(di * di + dj * dj) / (2.0 * sigma * sigma))
    return k / k.sum()


def anisotropic_kernel(K: int, sigma_x: float, sigma_y: float, angle_deg: float) -> np.ndarray:
    """Gaussian with std sigma_x along the direction at `angle_deg` counter-
    clockwise from the column axis (x to the right, y up) and sigma_y across."""
    di, dj = _offsets(K)
    x, y = dj, -di
    phi = math.radians(angle_deg)
    xr = x * math.cos(phi) + y * math.sin(phi)
    yr = -x * math.sin(phi) + y * math.cos(phi)
    k = np.exp(-(xr * xr) / (2 * sigma_x ** 2) - (yr * yr) / (2 * sigma_y ** 2))
    return k / k.sum()


def motion_kernel(K: int, length: float, angle_deg: float, smooth_sigma: float = 0.0,
                  n_samples: int = 1001) -> np.ndarray:
    """Centred line segment of `length` px at `angle_deg` (45 = "/"), sampled at
    `n_samples` points and splatted bilinearly into KxK, optionally convolved
    with a Gaussian of std `smooth_sigma`, then normalised."""
    c0 = (K - 1) / 2.0
    phi = math.radians(angle_deg)
    k = np.zeros((K, K))
    for t in np.linspace(-length / 2.0, length / 2.0, n_samples):
        r = c0 - t * math.sin(phi)
        c = c0 + t * math.cos(phi)
        r0, c0i = int(math.floor(r)), int(math.floor(c))
        fr, fc = r - r0, c - c0i
        for dr, wr in ((0, 1 - fr), (1, fr)):
            for dc, wc in ((0, 1 - fc), (1, fc)):
                rr, cc = r0 + dr, c0i + dc
                if 0 <= rr < K and 0 <= cc < K:
                    k[rr, cc] += wr * wc
    if smooth_sigma > 0:
        k = fftconvolve(k, gaussian_kernel(K, smooth_sigma), mode="same")
        k = np.maximum(k, 0.0)
    return k / k.sum()


def diagonal_motion_kernel(K: int) -> np.ndarray:
    """KxK kernel with equal weights on the anti-diagonal ("/" motion)."""
    k = np.fliplr(np.eye(K))
    return k / k.sum()


# ----------------------------------------------------------------------------
# images
# ----------------------------------------------------------------------------
def piecewise_constant(rng: np.random.Generator, H: int, W: int, C: int, n_shapes: int) -> np.ndarray:
    """Background 0; `n_shapes` rectangles or disks (probability 1/2 each),
    painted in order (later shapes overwrite earlier ones), one shared geometry
    for all channels and an independent U[0,1] intensity per channel."""
    img = np.zeros((C, H, W))
    m = min(H, W)
    for _ in range(n_shapes):
        if rng.random() < 0.5:
            r0 = int(rng.integers(0, H))
            c0 = int(rng.integers(0, W))
            hh = int(round(rng.uniform(H / 16.0, H / 4.0)))
            ww = int(round(rng.uniform(W / 16.0, W / 4.0)))
            val = rng.random(C)
            img[:, r0:r0 + hh, c0:c0 + ww] = val[:, None, None]
        else:
            cr = rng.uniform(0, H)
            cc = rng.uniform(0, W)
            rad = rng.uniform(m / 32.0, m / 8.0)
            val = rng.random(C)
            ra, rb = max(0, int(cr - rad) - 1), min(H, int(cr + rad) + 2)
            ca, cb = max(0, int(cc - rad) - 1), min(W, int(cc + rad) + 2)
            ii, jj = np.meshgrid(np.arange(ra, rb) + 0.5, np.arange(ca, cb) + 0.5, indexing="ij")
            mask = (ii - cr) ** 2 + (jj - cc) ** 2 <= rad * rad
            for ch in range(C):
                sub = img[ch, ra:rb, ca:cb]
                sub[mask] = val[ch]
    return img


def value_noise(rng: np.random.Generator, H: int, W: int, cells=(8, 16, 32, 64),
                amps=(1.0, 0.5, 0.25, 0.125), scale: float = 0.05) -> np.ndarray:
    """Sum of octaves of lattice value noise (values U[-1,1], smoothstep
    interpolation), normalised to max|.| = 1 and multiplied by `scale`."""
    out = np.zeros((H, W))
    for n, a in zip(cells, amps):
        lat = rng.uniform(-1.0, 1.0, size=(n + 1, n + 1))
        ys = np.arange(H) * (n / H)
        xs = np.arange(W) * (n / W)
        y0 = np.floor(ys).astype(int)
        x0 = np.floor(xs).astype(int)
        fy = ys - y0
        fx = xs - x0
        sy = fy * fy * (3 - 2 * fy)
        sx = fx * fx * (3 - 2 * fx)
        v00 = lat[y0][:, x0]
        v01 = lat[y0][:, x0 + 1]
        v10 = lat[y0 + 1][:, x0]
        v11 = lat[y0 + 1][:, x0 + 1]
        top = v00 + (v01 - v00) * sx[None, :]
        bot = v10 + (v11 - v10) * sx[None, :]
        out += a * (top + (bot - top) * sy[:, None])
    out /= np.abs(out).max()
    return scale * out


def blur_same(x: np.ndarray, k: np.ndarray) -> np.ndarray:
    """Data synthesis only: zero-boundary, same-size true convolution of every
    channel of x [C,H,W] with k [K,K] (scipy FFT convolution)."""
    return np.stack([fftconvolve(x[c], k, mode="same") for c in range(x.shape[0])])


def directions(n: int, K: int, seed: int = 909) -> np.ndarray:
    """`n` random unit directions in R^{KxK} for finite-difference checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.standard_normal((n, K, K))
    return d / np.linalg.norm(d.reshape(n, -1), axis=1)[:, None, None]


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
@dataclass
class Instance:
    """One semi-blind deblurring problem.  Arrays are float64, images planar
    [C][H][W], kernels [K][K] (one kernel for every channel) or [C][K][K]
    (one per channel, from make_channelwise)."""
    name: str
    x_true: np.ndarray
    y: np.ndarray
    k_true: np.ndarray
    a: np.ndarray            # assumed kernel = theta_0 = upper-level operator kernel
    alpha: float
    eps_tv: float
    beta: float
    sigma_n: float
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def C(self): return self.y.shape[0]

    @property
    def H(self): return self.y.shape[1]

    @property
    def W(self): return self.y.shape[2]

    @property
    def K(self): return self.a.shape[-1]

    @property
    def kc(self):
        """kernel channels: 1 for one shared [K][K] kernel, C for [C][K][K]"""
        return 1 if self.a.ndim == 2 else self.a.shape[0]


CONFIGS = {
    "cfg1": dict(H=64, W=64, C=1, K=7, shapes=12, seed=101, sigma_n=0.01, alpha=1e-3,
                 true=("gauss", 1.5), init=("gauss", 1.0), dtype="f64", maid_steps=10),
    "cfg2": dict(H=256, W=256, C=1, K=9, shapes=40, seed=202, sigma_n=0.02, alpha=5e-4,
                 true=("gauss", 2.0), init=("gauss", 4.0 / 3.0), dtype="f32", maid_steps=50),
    "cfg3": dict(H=512, W=512, C=3, K=15, shapes=40, seed=303, sigma_n=0.01, alpha=2e-4,
                 true=("aniso", 3.0, 1.5, 30.0), init=("gauss", 1.5), dtype="f32"),
    "cfg5": dict(H=2048, W=2048, C=3, K=31, shapes=400, seed=505, sigma_n=0.01, alpha=1e-4,
                 true=("motion", 21.0, 45.0, 1.0), init=("motion", 21.0, 45.0, 0.0),
                 texture=True, dtype="f32", maid_steps=5),
    "paper": dict(H=300, W=400, C=3, K=5, shapes=40, seed=606, sigma_n=0.02, alpha=0.3,
                  true=("diagmix", 0.5), init=("diag",), dtype="f32", maid_steps=20),
}
EPS_TV = 1e-2


def _kernel(spec, K):
    kind = spec[0]
    if kind == "gauss":
        return gaussian_kernel(K, spec[1])
    if kind == "aniso":
        return anisotropic_kernel(K, spec[1], spec[2], spec[3])
    if kind == "motion":
        return motion_kernel(K, spec[1], spec[2], spec[3])
    if kind == "diag":
        return diagonal_motion_kernel(K)
    if kind == "diagmix":   # semi-blind mixed blur: Gaussian applied after the motion blur
        k = fftconvolve(np.pad(diagonal_motion_kernel(K), K // 2), gaussian_kernel(K, spec[1]), mode="same")
        return k / k.sum()
    raise ValueError(kind)


def _generate(name, H, W, C, K, shapes, seed, sigma_n, alpha, true, init, texture=False,
              size_override=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = piecewise_constant(rng, H, W, C, shapes)
    if texture:
        x = x + value_noise(rng, H, W)[None, :, :]
    k_true = _kernel(true, K) if true[0] != "diagmix" else None
    if k_true is None:   # mixed blur is applied as two successive blurs
        y_clean = blur_same(blur_same(x, diagonal_motion_kernel(K)), gaussian_kernel(K, true[1]))
        k_true = _kernel(true, K)
    else:
        y_clean = blur_same(x, k_true)
    y = y_clean + sigma_n * rng.standard_normal(x.shape)
    a = _kernel(init, K)
    return Instance(name=name, x_true=x, y=y, k_true=k_true, a=a, alpha=alpha, eps_tv=EPS_TV,
                    beta=0.5 * alpha, sigma_n=sigma_n, seed=seed)


def make(name: str, H: int | None = None, W: int | None = None, C: int | None = None,
         K: int | None = None, seed: int | None = None) -> Instance:
    """Build a named workload; H, W, C, K, seed may be overridden to make
    smaller cases with the same recipe (used by the parity tests)."""
    if name == "cfg4":
        raise ValueError("cfg4 is a batch: use make_batch()")
    p = dict(CONFIGS[name])
    H0, W0 = p["H"], p["W"]
    H = H or H0
    W = W or W0
    C = C or p["C"]
    K = K or p["K"]
    shapes = p["shapes"]
    if (H, W) != (H0, W0):
        shapes = int(np.clip(round(shapes * math.sqrt(H * W / (H0 * W0))), 4, 400))
    kw = dict(texture=p.get("texture", False))
    inst = _generate(name, H, W, C, K, shapes, seed if seed is not None else p["seed"],
                     p["sigma_n"], p["alpha"], p["true"], p["init"], **kw)
    inst.meta = dict(dtype=p["dtype"], maid_steps=p.get("maid_steps"), shapes=shapes)
    return inst


def _scaled(spec, f):
    """The kernel recipe `spec` with its width scaled by f (Gaussian sigmas,
    motion length)."""
    kind = spec[0]
    if kind in ("gauss", "diagmix"):
        return (kind, spec[1] * f)
    if kind == "aniso":
        return (kind, spec[1] * f, spec[2] * f, spec[3])
    if kind == "motion":
        return (kind, spec[1] * f, spec[2], spec[3])
    return spec


def make_channelwise(name: str, H: int | None = None, W: int | None = None, C: int | None = None,
                     K: int | None = None, seed: int | None = None, spread: float = 0.2) -> Instance:
    """A workload of `make` with one blur kernel per colour channel, the way
    lateral chromatic aberration blurs the channels of a lens image
    differently: channel c's true kernel is the recipe's with its width
    scaled by 1 + spread * (c - (C-1)/2) / ((C-1)/2), and each channel's
    data is blurred by its own kernel.  The assumed kernel a is the recipe's
    assumed kernel in every channel (the semi-blind start knows nothing of
    the channels' differences).  k_true and a are [C][K][K]."""
    inst = make(name, H=H, W=W, C=C, K=K, seed=seed)
    p = CONFIGS[name]
    C, K = inst.C, inst.K
    half = max((C - 1) / 2.0, 1.0)
    ks = np.stack([_kernel(_scaled(p["true"], 1.0 + spread * (c - (C - 1) / 2.0) / half), K)
                   for c in range(C)])
    rng = np.random.Generator(np.random.PCG64(inst.seed + 7919))
    y = np.stack([fftconvolve(inst.x_true[c], ks[c], mode="same") for c in range(C)])
    y = y + inst.sigma_n * rng.standard_normal(y.shape)
    a = np.stack([inst.a] * C)
    out = Instance(name=name + "_channelwise", x_true=inst.x_true, y=y, k_true=ks, a=a, alpha=inst.alpha,
                   eps_tv=inst.eps_tv, beta=inst.beta, sigma_n=inst.sigma_n, seed=inst.seed)
    out.meta = dict(inst.meta, spread=spread)
    return out


CFG4_SIZES = (128, 256, 384, 512, 768, 1024)
CFG4_KS = (5, 9, 13, 17, 21)


def make_batch(n: int = 64, seed: int = 404, size_cap: int | None = None) -> list:
    """The ragged batch: per instance H and W drawn independently from
    {128..1024}, C in {1,3}, K in {5,...,21}, Gaussian blur sigma K/6 against
    an assumed sigma K/9, noise U[0.005,0.03], alpha log-uniform [1e-4,1e-2].
    `size_cap` clips H and W (for small test batches with the same draws)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(n):
        H = int(rng.choice(CFG4_SIZES))
        W = int(rng.choice(CFG4_SIZES))
        C = int(rng.choice((1, 3)))
        K = int(rng.choice(CFG4_KS))
        sigma_n = float(rng.uniform(0.005, 0.03))
        alpha = float(10 ** rng.uniform(-4, -2))
        if size_cap:
            H, W = min(H, size_cap), min(W, size_cap)
            K = min(K, (min(H, W) // 2) * 2 - 1)
        shapes = int(np.clip(round(40 * math.sqrt(H * W) / 256), 12, 400))
        inst = _generate(f"cfg4[{b}]", H, W, C, K, shapes, 4000 + b, sigma_n, alpha,
                         ("gauss", K / 6.0), ("gauss", K / 9.0))
        inst.meta = dict(dtype="f32", shapes=shapes, index=b)
        out.append(inst)
    return out


# ----------------------------------------------------------------------------
# Section 4.1's 1D deconvolution data
# ----------------------------------------------------------------------------
@dataclass
class Signal1D:
    name: str
    n: int
    A: np.ndarray        # n x n Gaussian blur matrix (the known operator; B_0 = A)
    x_true: np.ndarray
    y: np.ndarray
    alpha1: float
    alpha2: float
    meta: dict


def gaussian_matrix(n: int, sigma: float) -> np.ndarray:
    """The full n x n matrix of a 1D convolution with a Gaussian of standard
    deviation sigma (samples), truncated at 4 sigma, zero boundary, taps
    normalised to sum 1 in the interior."""
    r = int(np.ceil(4 * sigma))
    t = np.arange(-r, r + 1, dtype=np.float64)
    k = np.exp(-0.5 * (t / sigma) ** 2)
    k /= k.sum()
    A = np.zeros((n, n))
    for i in range(n):
        for o, w in zip(range(-r, r + 1), k):
            j = i + o
            if 0 <= j < n:
                A[i, j] = w
    return A


def make_1d(n: int = 512, seed: int = 7, sigma: float = 5.0, noise: float = 5e-3, alpha1: float = 1.2e-3,
            alpha2: float = 4e-3, pieces: int | None = None) -> Signal1D:
    """A piecewise-constant signal (jumps at random positions, levels
    U[-1, 1], a quarter of the pieces at zero), blurred by the Gaussian
    matrix of Section 4.1 (sigma 5) plus N(0, noise^2) noise; Section 4.1's
    elastic-net weights."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = pieces or max(4, n // 32)
    cuts = np.sort(rng.choice(np.arange(1, n), size=m - 1, replace=False))
    levels = rng.uniform(-1.0, 1.0, size=m)
    levels[rng.random(m) < 0.25] = 0.0
    x = np.zeros(n)
    for lv, a, b in zip(levels, np.concatenate([[0], cuts]), np.concatenate([cuts, [n]])):
        x[a:b] = lv
    A = gaussian_matrix(n, sigma)
    y = A @ x + noise * rng.standard_normal(n)
    return Signal1D("1d", n, A, x, y, alpha1, alpha2, dict(sigma=sigma, noise=noise, seed=seed, pieces=m))
