"""Seeded synthetic workloads for the PRISM analysis-by-synthesis pass.

This module only draws inputs: acquisitions (b-values in ms/um^2, unit gradient
directions), brain masks, ground-truth tissue, noisy measurements and the
initial parameters of a fit.  It holds none of the fitted model's arithmetic
(no synthesis, calibration, loss or gradient of the method): the ground-truth
signal is drawn from a *different* tissue model -- every fibre is a
cylindrically symmetric diffusion tensor with its own (d_par, d_perp) and the
isotropic balls use D = 3.0 / 0.8 / 0.1 -- which is the deliberate
model/data mismatch of the paper's synthetic experiments (Sec. 4, crossing-fibre
benchmark).  Both the FP64 oracle and the HIP path consume what this module
returns; neither imports the other.

Layout conventions shared by every consumer:
  * a *group* is one independent problem (one calibration group): a box
    (nx, ny, nz), a boolean mask, one acquisition, one K and one data mode;
  * voxels are the masked voxels of the box in C (raster) order, last axis
    fastest, i.e. ``np.argwhere(mask)`` order;
  * per-voxel parameters are parameter-major arrays ``[..., V]``:
      s0 [V], logits [K+3, V] (csf, gm, wm_1..wm_K, res), v [K, 3, V],
      fin [V] and, with learned diffusivities, dpar [V], dperp [V];
  * calibration parameters: bias [n_bias], alpha [N], beta [N], sigma_log ();
  * measurements y are ``[N, V]`` float32.

Seeds: the i-th generator below (0 patch8_crossings, 1 patch16_hcp,
2 brain_volume, 3 batched_patches, 4 tube_phantom) uses ``SeedSequence(1000 + i)``
spawned into independent streams (acquisition, tissue, directions, noise,
calibration, init).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

B_UNIT = 1e-3  # s/mm^2 -> ms/um^2 (b * D is then O(1))

# ground-truth generator constants (not the fitted model's constants)
TRUTH_D_CSF = 3.0
TRUTH_D_GM = 0.8
TRUTH_D_RES = 0.1

PRIOR_NAMES = ("spatial", "rep", "sparse", "cal")


@dataclasses.dataclass
class Acquisition:
    bval: np.ndarray  # [N] float64, ms/um^2
    bvec: np.ndarray  # [N, 3] float64, unit rows (b=0 rows carry (1,0,0))
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.bval.shape[0])


@dataclasses.dataclass
class Group:
    shape: tuple
    mask: np.ndarray  # bool [nx, ny, nz]
    acq: Acquisition
    K: int
    mode: str  # "mse" | "nll"
    bias: str = "none"  # "none" | "poly2" | "trilinear8"
    learn_diffusivity: bool = False
    neighbourhood: int = 6  # 0 (spatial prior off), 6 or 26
    priors: tuple = PRIOR_NAMES
    y: Optional[np.ndarray] = None  # float32 [N, V]
    theta: Optional[dict] = None  # initial raw parameters (float32 arrays)
    truth: Optional[dict] = None
    sigma_true: float = 0.0

    @property
    def n_vox(self) -> int:
        return int(self.mask.sum())

    @property
    def coords(self) -> np.ndarray:
        return np.argwhere(self.mask).astype(np.int32)

    @property
    def n_bias(self) -> int:
        return {"none": 0, "poly2": 10, "trilinear8": 512}[self.bias]


@dataclasses.dataclass
class Workload:
    name: str
    groups: list
    iterations: int
    lr: float = 1e-2
    description: str = ""

    @property
    def n_vox(self) -> int:
        return sum(g.n_vox for g in self.groups)


def streams(index: int, seed: Optional[int] = None, n: int = 6):
    ss = np.random.SeedSequence(1000 + index if seed is None else seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


# ----------------------------------------------------------------------------
# acquisitions
# ----------------------------------------------------------------------------

def uniform_sphere(n: int, rng) -> np.ndarray:
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def electrostatic_hemisphere(n: int, rng, steps: int = 2000) -> np.ndarray:
    """Antipodally symmetric electrostatic repulsion: minimise
    sum_{i<j} 1/|u_i-u_j| + 1/|u_i+u_j| by projected gradient steps."""
    u = uniform_sphere(n, rng)
    step = 0.01
    for _ in range(steps):
        dm = u[:, None, :] - u[None, :, :]
        dp = u[:, None, :] + u[None, :, :]
        rm = np.linalg.norm(dm, axis=2) + np.eye(n)
        rp = np.linalg.norm(dp, axis=2)
        # gradient of the energy w.r.t. u_i (force is its negative)
        gm = -(dm / rm[:, :, None] ** 3)
        np.einsum("iij->ij", gm)[:] = 0.0
        gp = -(dp / rp[:, :, None] ** 3)
        grad = gm.sum(1) + gp.sum(1)
        # project on the tangent plane and take a normalised step
        grad -= (grad * u).sum(1, keepdims=True) * u
        gn = np.abs(grad).max() + 1e-30
        u = u - step * grad / gn
        u /= np.linalg.norm(u, axis=1, keepdims=True)
    u[u[:, 2] < 0] *= -1.0  # fold onto the upper hemisphere
    return u


def make_acquisition(kind: str, rng) -> Acquisition:
    """kind: 'single33' (1 b0 + 32 @ b=1000), 'two96' (6 b0 + 45 @ 1000 + 45 @ 2000),
    'three288' (18 b0 + 90 @ 1000/2000/3000), 'three193' (1 b0 + 64 @ 1000/2000/3000),
    'hardi160' (10 b0 + 150 @ b=2000, the shape of a single-shell HARDI scan)."""
    if kind == "single33":
        shells = [(0.0, 1), (1000.0, 32)]
        dirs = [np.array([[1.0, 0.0, 0.0]]), electrostatic_hemisphere(32, rng)]
    else:
        shells = {
            "two96": [(0.0, 6), (1000.0, 45), (2000.0, 45)],
            "three288": [(0.0, 18), (1000.0, 90), (2000.0, 90), (3000.0, 90)],
            "three193": [(0.0, 1), (1000.0, 64), (2000.0, 64), (3000.0, 64)],
            "hardi160": [(0.0, 10), (2000.0, 150)],
        }[kind]
        dirs = []
        for b, cnt in shells:
            if b == 0.0:
                dirs.append(np.tile([[1.0, 0.0, 0.0]], (cnt, 1)))
            else:
                dirs.append(uniform_sphere(cnt, rng))
    bval = np.concatenate([np.full(c, b * B_UNIT) for b, c in shells])
    bvec = np.concatenate(dirs, axis=0)
    return Acquisition(bval=bval.astype(np.float64), bvec=bvec.astype(np.float64), name=kind)


# ----------------------------------------------------------------------------
# ground truth tissue and measurements
# ----------------------------------------------------------------------------

def _rotate_towards(a: np.ndarray, angle_deg: np.ndarray, rng) -> np.ndarray:
    """Unit vectors at `angle_deg` from the unit rows of `a`, random azimuth."""
    r = uniform_sphere(a.shape[0], rng)
    perp = r - (r * a).sum(1, keepdims=True) * a
    perp /= np.linalg.norm(perp, axis=1, keepdims=True) + 1e-30
    t = np.deg2rad(angle_deg)[:, None]
    return np.cos(t) * a + np.sin(t) * perp


def _axial_angle(a, b):
    return np.rad2deg(np.arccos(np.clip(np.abs((a * b).sum(-1)), 0.0, 1.0)))


def random_crossings(V: int, rng, max_fib: int = 3, min_angle: float = 20.0,
                     max_angle: float = 90.0, n_fib: Optional[np.ndarray] = None):
    """Per voxel: 1..max_fib fibres, fibres 2.. at U(min,max) degrees from fibre 1
    (re-drawn until every pair is at least `min_angle` apart)."""
    if n_fib is None:
        n_fib = rng.integers(1, max_fib + 1, size=V)
    dirs = np.zeros((max_fib, V, 3))
    dirs[0] = uniform_sphere(V, rng)
    for k in range(1, max_fib):
        ang = rng.uniform(min_angle, max_angle, size=V)
        cand = _rotate_towards(dirs[0], ang, rng)
        for _ in range(100):
            bad = np.zeros(V, dtype=bool)
            for j in range(1, k):
                bad |= _axial_angle(cand, dirs[j]) < min_angle
            if not bad.any():
                break
            ang_b = rng.uniform(min_angle, max_angle, size=int(bad.sum()))
            cand[bad] = _rotate_towards(dirs[0][bad], ang_b, rng)
        dirs[k] = cand
    return n_fib, dirs


def tissue_truth(V: int, rng, max_fib: int = 3, n_fib=None, dirs=None, frac=None):
    if dirs is None:
        n_fib, dirs = random_crossings(V, rng, max_fib=max_fib, n_fib=n_fib)
    dpar = rng.uniform(1.5, 2.2, size=(max_fib, V))
    dperp = rng.uniform(0.3, 0.7, size=(max_fib, V))
    if frac is None:
        # Dirichlet(1) over (csf, gm, res, fibre_1..fibre_nfib)
        frac = np.zeros((3 + max_fib, V))
        for nf in range(1, max_fib + 1):
            sel = n_fib == nf
            if sel.any():
                w = rng.dirichlet(np.ones(3 + nf), size=int(sel.sum())).T
                frac[: 3 + nf, sel] = w
    return dict(n_fib=np.asarray(n_fib), dirs=dirs, dpar=dpar, dperp=dperp, frac=frac,
                s0=np.ones(V))


def truth_signal(acq: Acquisition, truth: dict, dtype=np.float64, chunk: int = 65536):
    """Noise-free ground-truth signal [N, V] from the generator's tissue model:
    balls exp(-b D) with D = 3.0 / 0.8 / 0.1 and, per fibre, a cylindrically
    symmetric tensor exp(-b g^T (d_perp I + (d_par - d_perp) u u^T) g)."""
    frac, dirs = truth["frac"], truth["dirs"]
    V = frac.shape[1]
    nf = dirs.shape[0]
    b = acq.bval.astype(dtype)[:, None]
    G = acq.bvec.astype(dtype)
    out = np.empty((acq.n, V), dtype=dtype)
    for lo in range(0, V, chunk):
        hi = min(V, lo + chunk)
        acc = (frac[0, lo:hi].astype(dtype) * np.exp(-b * TRUTH_D_CSF)
               + frac[1, lo:hi].astype(dtype) * np.exp(-b * TRUTH_D_GM)
               + frac[2, lo:hi].astype(dtype) * np.exp(-b * TRUTH_D_RES))
        for k in range(nf):
            u = dirs[k, lo:hi].astype(dtype)
            q = (G @ u.T) ** 2  # (g.u)^2
            dp = truth["dpar"][k, lo:hi].astype(dtype)
            dq = truth["dperp"][k, lo:hi].astype(dtype)
            adc = dq + (dp - dq) * q
            acc += frac[3 + k, lo:hi].astype(dtype) * np.exp(-b * adc)
        out[:, lo:hi] = acc * truth["s0"][lo:hi].astype(dtype)
    return out


def rician(signal: np.ndarray, sigma, rng, dtype=np.float32, chunk: int = 1 << 22):
    """|signal + sigma (n1 + i n2)|, Gaussian n1, n2; `sigma` scalar or [V]."""
    flat = signal.reshape(-1)
    out = np.empty(flat.shape, dtype=dtype)
    sig = np.asarray(sigma, dtype=dtype)
    per_vox = sig.ndim > 0
    V = signal.shape[-1]
    for lo in range(0, flat.size, chunk):
        hi = min(flat.size, lo + chunk)
        s = flat[lo:hi].astype(dtype)
        sg = sig[np.arange(lo, hi) % V] if per_vox else sig
        n1 = rng.standard_normal(hi - lo, dtype=dtype)
        n2 = rng.standard_normal(hi - lo, dtype=dtype)
        out[lo:hi] = np.hypot(s + sg * n1, sg * n2)
    return out.reshape(signal.shape)


# ----------------------------------------------------------------------------
# nuisance truth: a smooth quadratic log-bias and per-measurement gains
# ----------------------------------------------------------------------------

def box_unit_coords(shape, coords):
    """Coordinates mapped to [-1, 1] across the box (0 along an axis of size 1)."""
    out = np.zeros(coords.shape, dtype=np.float64)
    for a in range(3):
        n = shape[a]
        if n > 1:
            out[:, a] = (2.0 * coords[:, a] - (n - 1)) / (n - 1)
    return out


def quadratic_log_bias_truth(shape, rng, max_dev: float = 0.15):
    """A random quadratic form q(x) = c + b.x + x^T A x over the unit box,
    rescaled so that max |exp(q) - 1| <= max_dev.  Returned as the ten
    coefficients of (1, x, y, z, x^2, y^2, z^2, xy, xz, yz)."""
    c = rng.normal(0.0, 1.0)
    bl = rng.normal(0.0, 1.0, size=3)
    A = rng.normal(0.0, 0.5, size=(3, 3))
    A = 0.5 * (A + A.T)
    coef = np.array([c, bl[0], bl[1], bl[2], A[0, 0], A[1, 1], A[2, 2],
                     2 * A[0, 1], 2 * A[0, 2], 2 * A[1, 2]])
    grid = np.stack(np.meshgrid(*[np.linspace(-1, 1, max(n, 2)) for n in shape],
                                indexing="ij"), -1).reshape(-1, 3)
    q = (coef[0] + grid @ bl + np.einsum("vi,ij,vj->v", grid, A, grid))
    # largest scale s with max |exp(s q) - 1| <= max_dev
    lo, hi = 0.0, 10.0
    for _ in range(80):
        s = 0.5 * (lo + hi)
        if np.abs(np.exp(s * q) - 1.0).max() <= max_dev:
            lo = s
        else:
            hi = s
    return coef * lo


def eval_quadratic_log_bias(coef, shape, coords):
    x = box_unit_coords(shape, coords)
    A = np.array([[coef[4], coef[7] / 2, coef[8] / 2],
                  [coef[7] / 2, coef[5], coef[9] / 2],
                  [coef[8] / 2, coef[9] / 2, coef[6]]])
    return coef[0] + x @ coef[1:4] + np.einsum("vi,ij,vj->v", x, A, x)


# ----------------------------------------------------------------------------
# initial parameters
# ----------------------------------------------------------------------------

def init_theta(V: int, K: int, N: int, n_bias: int, rng, sigma_init: float = 0.0,
               learn_diffusivity: bool = False, dtype=np.float32) -> dict:
    """Random unit directions, zero logits, S0 = 1, f_intra = 0.5, calibration at
    identity and sigma_log = log(sigma_init) (NLL mode)."""
    v = rng.standard_normal((K, 3, V))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    th = dict(
        s0=np.full(V, math.log(math.e - 1.0)),
        logits=np.zeros((K + 3, V)),
        v=v,
        fin=np.zeros(V),
        bias=np.zeros(n_bias),
        alpha=np.zeros(N),
        beta=np.zeros(N),
        sigma_log=np.array(math.log(sigma_init) if sigma_init > 0 else 0.0),
    )
    if learn_diffusivity:
        th["dpar"] = np.full(V, math.log(math.expm1(1.7)))
        th["dperp"] = np.full(V, math.log(math.expm1(0.4)))
    return {k: np.asarray(a, dtype=dtype) for k, a in th.items()}


def perturb_theta(theta: dict, rng, scale: float = 0.5) -> dict:
    """A generic (non-initial) parameter point for gradient checks: every raw
    parameter moved by N(0, scale) so that no symmetry of the init survives."""
    out = {}
    for k, a in theta.items():
        a = np.asarray(a, dtype=np.float64)
        if k == "sigma_log":
            out[k] = a + rng.normal(0.0, 0.1)
        elif k in ("alpha", "beta"):
            out[k] = a + rng.normal(0.0, 0.05, size=a.shape)
        elif k == "bias":
            out[k] = a + rng.normal(0.0, 0.05, size=a.shape)
        else:
            out[k] = a + rng.normal(0.0, scale, size=a.shape)
    return {k: np.asarray(v, dtype=theta[k].dtype) for k, v in out.items()}


# ----------------------------------------------------------------------------
# smooth random fields (for the whole-brain-shaped volume and the phantom)
# ----------------------------------------------------------------------------

def smooth_field(shape, rng, sigma_vox: float, dtype=np.float32):
    """Unit-variance Gaussian-smoothed white noise."""
    from scipy.ndimage import gaussian_filter
    f = gaussian_filter(rng.standard_normal(shape).astype(dtype), sigma_vox, mode="wrap")
    f -= f.mean()
    f /= f.std() + 1e-12
    return f


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def _single_patch(index, edge, acq_kind, K, mode, snr, bias, sigma_init_factor,
                  iterations, calib_truth, seed=None, name=""):
    r_acq, r_tis, r_dir, r_noise, r_cal, r_init = streams(index, seed)
    acq = make_acquisition(acq_kind, r_acq)
    shape = (edge, edge, edge)
    mask = np.ones(shape, dtype=bool)
    V = int(mask.sum())
    n_fib, dirs = random_crossings(V, r_dir, max_fib=3)
    truth = tissue_truth(V, r_tis, max_fib=3, n_fib=n_fib, dirs=dirs)
    S = truth_signal(acq, truth)
    coords = np.argwhere(mask)
    if calib_truth:
        coef = quadratic_log_bias_truth(shape, r_cal)
        logB = eval_quadratic_log_bias(coef, shape, coords)
        gain = r_cal.normal(1.0, 0.03, size=acq.n)
        off = r_cal.normal(0.0, 0.01, size=acq.n)
        S = gain[:, None] * np.exp(logB)[None, :] * S + off[:, None]
        truth.update(bias_coef=coef, alpha=np.log(gain), beta=off)
    sigma = 1.0 / snr
    y = rician(S, sigma, r_noise)
    n_bias = {"none": 0, "poly2": 10, "trilinear8": 512}[bias]
    theta = init_theta(V, K, acq.n, n_bias, r_init,
                       sigma_init=sigma_init_factor * sigma if mode == "nll" else 0.0)
    g = Group(shape=shape, mask=mask, acq=acq, K=K, mode=mode, bias=bias, y=y,
              theta=theta, truth=truth, sigma_true=sigma)
    return Workload(name=name, groups=[g], iterations=iterations)


def patch8_crossings(seed=None, priors=("rep",)) -> Workload:
    """8^3 patch, K=3, 33 single-shell measurements, MSE, SNR 30, 100 Adam steps."""
    w = _single_patch(0, 8, "single33", 3, "mse", 30.0, "none", 0.0, 100, False, seed,
                      name="patch8_n33_k3_mse")
    w.groups[0].priors = tuple(priors)
    w.description = "one 8^3 patch, N=33 (1 b0 + 32 @ b=1000), K=3, MSE, SNR 30"
    return w


def patch16_hcp(seed=None) -> Workload:
    """16^3 patch, K=3, 288 three-shell measurements, Rician NLL with learned
    sigma (initialised at twice the truth), quadratic bias + gains, 500 iterations."""
    w = _single_patch(1, 16, "three288", 3, "nll", 30.0, "poly2", 2.0, 500, True, seed,
                      name="patch16_n288_k3_nll_cal")
    w.description = ("one 16^3 patch, N=288 (18 b0 + 90 @ b=1000/2000/3000), K=3, Rician NLL, "
                     "learned sigma, quadratic log-bias + per-measurement gain/offset, SNR 30")
    return w


def ellipsoid_mask(shape, centre, scale):
    axes = [np.arange(n, dtype=np.float32) for n in shape]
    semi = [scale * n / 2.0 for n in shape]
    r2 = np.zeros(shape, dtype=np.float32)
    for a in range(3):
        sh = [1, 1, 1]
        sh[a] = shape[a]
        r2 = r2 + (((axes[a] - centre[a]) / semi[a]) ** 2).reshape(sh)
    return r2


def whole_brain_mask(shape, rng, target: int = 741_000, tol: float = 0.005):
    centre = np.array([(n - 1) / 2.0 for n in shape]) + rng.uniform(-2, 2, size=3)
    lo, hi = 0.3, 1.0
    for _ in range(60):
        s = 0.5 * (lo + hi)
        cnt = int((ellipsoid_mask(shape, centre, s) <= 1.0).sum())
        if abs(cnt - target) <= tol * target:
            break
        if cnt < target:
            lo = s
        else:
            hi = s
    r2 = ellipsoid_mask(shape, centre, s)
    return r2 <= 1.0, np.sqrt(r2)


def _smooth_directions(shape, mask, rng, sigma_vox=6.0):
    comps = np.stack([smooth_field(shape, rng, sigma_vox)[mask] for _ in range(3)], -1)
    comps /= np.linalg.norm(comps, axis=1, keepdims=True) + 1e-12
    return comps.astype(np.float64)


def _separate(dirs, min_angle=20.0):
    """Move later fibres away from earlier ones until every pair is >= min_angle."""
    cmin = math.cos(math.radians(min_angle))
    for k in range(1, dirs.shape[0]):
        for _ in range(4):
            for j in range(k):
                dot = (dirs[k] * dirs[j]).sum(1)
                bad = np.abs(dot) > cmin
                if not bad.any():
                    continue
                s = np.sign(dot[bad])[:, None]
                a = dirs[j][bad] * s
                perp = dirs[k][bad] - (dirs[k][bad] * a).sum(1, keepdims=True) * a
                nrm = np.linalg.norm(perp, axis=1, keepdims=True)
                fallback = np.cross(a, np.array([0.0, 0.0, 1.0]))
                fb_n = np.linalg.norm(fallback, axis=1, keepdims=True)
                fallback = np.where(fb_n > 1e-6, fallback, np.cross(a, np.array([1.0, 0.0, 0.0])))
                perp = np.where(nrm > 1e-6, perp, fallback)
                perp /= np.linalg.norm(perp, axis=1, keepdims=True)
                t = math.radians(min_angle + 1.0)
                dirs[k][bad] = math.cos(t) * a + math.sin(t) * perp
    return dirs


def brain_volume(seed=None, shape=(145, 174, 145), target=741_000, with_y=True, acq_kind="three288") -> Workload:
    """Whole-brain-shaped volume: ellipsoid mask of ~741k voxels, smooth tissue
    maps (CSF shell, GM rim, WM core with 1-3 fibres following smooth direction
    fields), N=288 three-shell, K=3, MSE, calibration on at identity, SNR 30.
    `shape`, `target` and `acq_kind` give smaller or differently sampled
    volumes of the same construction."""
    r_acq, r_tis, r_dir, r_noise, r_cal, r_init = streams(2, seed)
    acq = make_acquisition(acq_kind, r_acq)
    mask, rho_full = whole_brain_mask(shape, r_tis, target=target)
    V = int(mask.sum())
    rho = rho_full[mask] + 0.03 * smooth_field(shape, r_tis, 4.0)[mask]
    sig = lambda x: 1.0 / (1.0 + np.exp(-x))  # noqa: E731  (smooth region weights)
    w_csf = sig((rho - 0.9) / 0.015)
    w_gm = sig((rho - 0.75) / 0.015) * (1.0 - w_csf)
    w_wm = 1.0 - w_csf - w_gm
    h1 = smooth_field(shape, r_tis, 5.0)[mask]
    h2 = smooth_field(shape, r_tis, 5.0)[mask]
    n_fib = 1 + (h1 > 0.0).astype(int) + ((h1 > 0.0) & (h2 > 0.3)).astype(int)
    dirs = np.stack([_smooth_directions(shape, mask, r_dir) for _ in range(3)], 0)
    dirs = _separate(dirs)
    frac = np.zeros((6, V))
    frac[0] = 0.85 * w_csf + 0.05 * w_gm + 0.03 * w_wm
    frac[1] = 0.08 * w_csf + 0.75 * w_gm + 0.10 * w_wm
    frac[2] = 0.02 * w_csf + 0.10 * w_gm + 0.12 * w_wm
    wm_tot = 0.05 * w_csf + 0.10 * w_gm + 0.75 * w_wm
    share = r_tis.dirichlet(np.ones(3), size=V).T * 0.5 + 0.5 / 3.0
    for k in range(3):
        share[k] = np.where(n_fib > k, share[k], 0.0)
    share /= share.sum(0, keepdims=True)
    frac[3:6] = wm_tot[None] * share
    truth = tissue_truth(V, r_tis, max_fib=3, n_fib=n_fib, dirs=dirs, frac=frac)
    truth["mask_rho"] = rho
    sigma = 1.0 / 30.0
    y = None
    if with_y:
        S = truth_signal(acq, truth, dtype=np.float32)
        y = rician(S, sigma, r_noise)
        del S
    theta = init_theta(V, 3, acq.n, 10, r_init)
    g = Group(shape=tuple(shape), mask=mask, acq=acq, K=3, mode="mse", bias="poly2", y=y,
              theta=theta, truth=truth, sigma_true=sigma)
    return Workload(name="brain145x174x145_n288_k3_mse", groups=[g], iterations=1000,
                    description=("145x174x145 grid, ellipsoid mask ~741k voxels, N=288, K=3, MSE, "
                                 "calibration (quadratic log-bias, gains, offsets) at identity, SNR 30"))


def batched_patches(seed=None, n_patches=4096, edge_range=(4, 24), with_y=True) -> Workload:
    """Many independent patches of uneven size: edge round(exp U(ln4, ln24)),
    acquisition in {33, 96, 288}, K in 1..5, MSE or NLL (p = 1/2), SNR U(10, 50)."""
    r_acq, r_tis, r_dir, r_noise, r_cal, r_init = streams(3, seed)
    acqs = {k: make_acquisition(k, r_acq) for k in ("single33", "two96", "three288")}
    kinds = list(acqs)
    groups = []
    for p in range(n_patches):
        edge = int(round(math.exp(r_tis.uniform(math.log(edge_range[0]), math.log(edge_range[1])))))
        kind = kinds[int(r_tis.integers(0, 3))]
        K = int(r_tis.integers(1, 6))
        mode = "mse" if r_tis.random() < 0.5 else "nll"
        snr = float(r_tis.uniform(10.0, 50.0))
        shape = (edge, edge, edge)
        mask = np.ones(shape, dtype=bool)
        V = int(mask.sum())
        truth = tissue_truth(V, r_tis, max_fib=3)
        sigma = 1.0 / snr
        y = rician(truth_signal(acqs[kind], truth, dtype=np.float32), sigma, r_noise) if with_y else None
        theta = init_theta(V, K, acqs[kind].n, 0, r_init,
                           sigma_init=2.0 * sigma if mode == "nll" else 0.0)
        groups.append(Group(shape=shape, mask=mask, acq=acqs[kind], K=K, mode=mode, bias="none",
                            y=y, theta=theta, truth=None, sigma_true=sigma, neighbourhood=6))
    return Workload(name=f"batched{n_patches}_mixed", groups=groups, iterations=100,
                    description=(f"{n_patches} independent patches, edge log-uniform "
                                 f"{edge_range[0]}-{edge_range[1]}, N in {{33,96,288}}, K in 1..5, "
                                 "MSE or NLL, SNR U(10,50)"))


def tube_phantom(seed=None, edge=40, n_tubes=8) -> Workload:
    """40^3 volume with 8 straight tubular bundles (radius U(3,6)) crossing at
    20-90 degrees, N=96 two-shell, K=4, Rician NLL with learned sigma and
    learned diffusivities, SNR 20."""
    r_acq, r_tis, r_dir, r_noise, r_cal, r_init = streams(4, seed)
    acq = make_acquisition("two96", r_acq)
    shape = (edge, edge, edge)
    mask = np.ones(shape, dtype=bool)
    coords = np.argwhere(mask).astype(np.float64)
    V = coords.shape[0]
    axes = [uniform_sphere(1, r_dir)[0]]
    while len(axes) < n_tubes:
        c = uniform_sphere(1, r_dir)[0]
        ang = [_axial_angle(c, a) for a in axes]
        if min(ang) >= 20.0:
            axes.append(c)
    members = np.zeros((n_tubes, V), dtype=bool)
    for t in range(n_tubes):
        p0 = r_tis.uniform(0.3 * edge, 0.7 * edge, size=3)
        rad = r_tis.uniform(3.0, 6.0)
        d = coords - p0
        dist = np.linalg.norm(d - (d @ axes[t])[:, None] * axes[t][None, :], axis=1)
        members[t] = dist <= rad
    max_fib = 4
    dirs = np.tile(uniform_sphere(1, r_dir)[0], (max_fib, V, 1))
    n_fib = np.zeros(V, dtype=int)
    for v in np.nonzero(members.any(0))[0]:
        ts = np.nonzero(members[:, v])[0][:max_fib]
        for i, t in enumerate(ts):
            dirs[i, v] = axes[t]
        n_fib[v] = len(ts)
    frac = np.zeros((3 + max_fib, V))
    bg = n_fib == 0
    frac[0, bg] = 0.3
    frac[1, bg] = 0.6
    frac[2, bg] = 0.1
    fb = ~bg
    frac[0, fb] = 0.05
    frac[1, fb] = 0.1
    frac[2, fb] = 0.1
    for v in np.nonzero(fb)[0]:
        frac[3:3 + n_fib[v], v] = 0.75 / n_fib[v]
    truth = tissue_truth(V, r_tis, max_fib=max_fib, n_fib=n_fib, dirs=dirs, frac=frac)
    truth["members"] = members
    sigma = 1.0 / 20.0
    y = rician(truth_signal(acq, truth), sigma, r_noise)
    theta = init_theta(V, 4, acq.n, 10, r_init, sigma_init=2.0 * sigma, learn_diffusivity=True)
    g = Group(shape=shape, mask=mask, acq=acq, K=4, mode="nll", bias="poly2",
              learn_diffusivity=True, y=y, theta=theta, truth=truth, sigma_true=sigma)
    return Workload(name="phantom40_n96_k4_nll", groups=[g], iterations=300,
                    description="40^3 bundle phantom, 8 tubes, N=96, K=4, NLL, learned sigma and diffusivities, SNR 20")


def crossing_subpatch(w: Workload, edge: int = 4):
    """The edge^3 sub-box of the phantom whose voxels hold the most fibres."""
    g = w.groups[0]
    nf = g.truth["n_fib"].reshape(g.shape)
    best, best_c = -1, (0, 0, 0)
    for i in range(0, g.shape[0] - edge + 1, 2):
        for j in range(0, g.shape[1] - edge + 1, 2):
            for k in range(0, g.shape[2] - edge + 1, 2):
                s = int((nf[i:i + edge, j:j + edge, k:k + edge] >= 2).sum())
                if s > best:
                    best, best_c = s, (i, j, k)
    return best_c


def sub_box(g: Group, corner, edge) -> Group:
    """The group restricted to a sub-box (its own box coordinates)."""
    i, j, k = corner
    sub = np.zeros(g.shape, dtype=bool)
    sub[i:i + edge, j:j + edge, k:k + edge] = True
    keep = sub[g.mask]
    mask = g.mask[i:i + edge, j:j + edge, k:k + edge].copy()
    th = {}
    for key, a in g.theta.items():
        if key in ("bias", "alpha", "beta", "sigma_log"):
            th[key] = a.copy()
        else:
            th[key] = a[..., keep].copy()
    return dataclasses.replace(g, shape=(edge, edge, edge), mask=mask, y=g.y[:, keep].copy(),
                               theta=th, truth=None)


CROSSING_ANGLES = tuple(range(15, 95, 5))   # 16 crossing angles, degrees


def crossing_benchmark(snr: float = 30.0, seed=None, per_angle: int = 200, n_single: int = 200,
                       mode: str = "mse", gain_sigma: float = 0.0, angles=CROSSING_ANGLES,
                       K: int = 2) -> Workload:
    """Crossing-fibre voxels on the shape of the paper's synthetic benchmark
    (Sec. 3 dataset i, Table 1): `per_angle` voxels at each crossing angle
    (15-90 degrees in 5-degree steps) and `n_single` single-fibre voxels;
    N = 193 (1 b0 + 64 directions at each of b = 1000, 2000, 3000); K = 2;
    Rician noise at `snr`.  Two crossing fibres share the WM fraction equally;
    d_par ~ U(1.5, 2.2), d_perp ~ U(0.3, 0.7); WM carries U(0.7, 0.9) of the
    signal, the rest is split by Dirichlet(1) between the three balls.  With
    `gain_sigma` > 0 every diffusion-weighted measurement is multiplied by a
    gain drawn from N(1, gain_sigma) (the artifact sweep of Sec. 4; b0 stays
    the normaliser).  Voxels fill a (rows, per_angle, 1) box, one row per
    angle and a last row of single fibres, and are fitted independently (no
    neighbourhood).  The paper's DIPY-generated set is not available; this
    generator reproduces its shape only."""
    r_acq, r_tis, r_dir, r_noise, r_cal, r_init = streams(5, seed)
    acq = make_acquisition("three193", r_acq)
    if n_single > per_angle:
        raise ValueError("n_single must not exceed per_angle (one box row each)")
    rows = len(angles) + (1 if n_single else 0)
    mask = np.zeros((rows, per_angle, 1), dtype=bool)
    mask[: len(angles)] = True
    if n_single:
        mask[len(angles), :n_single] = True
    V = int(mask.sum())
    row = np.argwhere(mask)[:, 0]
    crossing = row < len(angles)
    angle = np.where(crossing, np.asarray(angles, dtype=np.float64)[np.minimum(row, len(angles) - 1)], 0.0)
    dirs = np.zeros((2, V, 3))
    dirs[0] = uniform_sphere(V, r_dir)
    dirs[1] = _rotate_towards(dirs[0], angle, r_dir)
    n_fib = np.where(crossing, 2, 1)
    wm = r_tis.uniform(0.7, 0.9, size=V)
    frac = np.zeros((5, V))
    frac[:3] = r_tis.dirichlet(np.ones(3), size=V).T * (1.0 - wm)[None]
    frac[3] = np.where(crossing, 0.5 * wm, wm)
    frac[4] = np.where(crossing, 0.5 * wm, 0.0)
    truth = tissue_truth(V, r_tis, max_fib=2, n_fib=n_fib, dirs=dirs, frac=frac)
    truth["angle"] = angle
    S = truth_signal(acq, truth)
    if gain_sigma > 0:
        gain = np.where(acq.bval > 0, r_cal.normal(1.0, gain_sigma, size=acq.n), 1.0)
        S = gain[:, None] * S
        truth["gain"] = gain
    sigma = 1.0 / snr
    y = rician(S, sigma, r_noise)
    theta = init_theta(V, K, acq.n, 0, r_init, sigma_init=2.0 * sigma if mode == "nll" else 0.0)
    g = Group(shape=mask.shape, mask=mask, acq=acq, K=K, mode=mode, bias="none", neighbourhood=0,
              priors=("rep", "sparse", "cal"), y=y, theta=theta, truth=truth, sigma_true=sigma)
    name = f"crossing{len(angles)}x{per_angle}+{n_single}_n193_k{K}_{mode}_snr{snr:g}"
    if gain_sigma > 0:
        name += f"_gain{gain_sigma:g}"
    return Workload(name=name, groups=[g], iterations=300, description=name)


WORKLOADS = {"patch8_crossings": patch8_crossings, "patch16_hcp": patch16_hcp,
             "brain_volume": brain_volume, "batched_patches": batched_patches,
             "tube_phantom": tube_phantom}


def make_workload(name: str, seed=None, **kw) -> Workload:
    return WORKLOADS[name](seed=seed, **kw)
