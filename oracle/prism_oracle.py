"""FP64 CPU oracle for PRISM's per-iteration analysis-by-synthesis pass.

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import or call this module; the product path never does.
It shares no code, table or constant with the HIP implementation.

What it computes (PRISM, arxiv 2604.00250), all in float64 with plain NumPy:

  * per-voxel transforms (Sec. 2.2 "per-voxel parameters", Sec. 2.5
    "constraints"): S0 = softplus, fractions = softmax over
    (csf, gm, wm_1..wm_K, res), directions = v / |v|, f_intra = sigmoid;
  * tissue signal, Eq. 3, with the isotropic balls of Eq. 4 and the
    stick-and-zeppelin fibre of Eq. 5;
  * calibration chain, Eq. 6: yhat = exp(alpha_n) B(x) S_n(x) + beta_n with
    B = exp(linear log-bias basis) (Sec. 2.3, item 1);
  * data terms: MSE, Eq. 8, and Rician NLL, Eq. 9, with sigma = exp(sigma_log);
  * priors (Sec. 2.4): local Huber-Laplacian on the fractions (Eq. 7),
    direction repulsion, L1 sparsity of minor fibre fractions, the three
    stabilisation terms (orphan-WM suppression, directional continuity,
    fibre ordering), L2 calibration penalties and total variation of the
    bias field;
  * the exact gradient of the total objective (Sec. 2.5) with respect to
    every raw parameter, derived by hand (chain rule of Eq. 3-9);
  * Adam (Kingma & Ba, Algorithm 1, with PyTorch's conventions) and Rprop
    (Riedmiller & Braun 1993, PyTorch's variant);
  * the whole-volume slab layout and the weighted stitching of per-slab
    maps (Sec. 2.5), with the readings stated at each function.

Readings where the paper is silent (each is listed with its reason in the
design notes): f_intra is per voxel and shared by the K fibres; the MSE is
normalised by |M| only (as printed); the NLL is a plain sum without the
-log y constant (as printed); repulsion and sparsity are averaged over |M|
like Eq. 7; the sparsity indicator 1[f_k < tau] is held constant in the
derivative; the derivative of |u| at 0 is 0; the calibration L2 weights are
0.01 each; sigma_log is not regularised; N(x) is the set of in-mask
neighbours inside the problem and a voxel without neighbours contributes 0.
The stabilisation terms have printed weights but no printed form; they are
read as: orphan-WM = sum_x max(0, 1 - S0/s_o) sum_k f_wm,k with s_o = 0.1;
continuity = sum_x 1/|N(x)| sum_{x' in N(x)} sum_k (1 - (d_k(x).d_k(x'))^2);
ordering = sum_x sum_k max(0, f_wm,k+1 - f_wm,k); all three averaged over
|M|.  Bias TV = (lam_tv/|M|) sum over in-mask face-neighbour pairs
(x, x + e_a) of |B(x + e_a) - B(x)|, lam_tv = 0.01.

The Bessel functions of Eq. 9 use scipy.special.i0e / i1e (exponentially
scaled I0, I1) so that log I0(z) = |z| + log i0e(|z|) cannot overflow.

Parity pins for every part live in the CPU test-suite (closed forms,
invariants, finite differences, brute force, quadrature of the Bessel
integrals); nothing here is "parity unpinned".
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
from scipy.special import i0e, i1e

LN2 = np.log(2.0)


@dataclasses.dataclass(frozen=True)
class Constants:
    # Eq. 4 (isotropic diffusivities, um^2/ms) and the text after Eq. 5
    d_csf: float = 3.0
    d_gm: float = 0.9
    d_res: float = 0.2
    d_par: float = 1.7
    d_perp: float = 0.4
    # Sec. 2.4, Eq. 7 and the text after it; Sec. 2.5 implementation details
    lam_sp: float = 0.01
    huber_delta: float = 0.05
    lam_rep: float = 0.01
    lam_sparse: float = 0.02
    tau_sparse: float = 0.15
    # Sec. 2.4 calibration regularisers: weights not printed, read as 0.01
    lam_alpha: float = 0.01
    lam_beta: float = 0.01
    lam_bias: float = 0.01
    # Sec. 2.4 stabilisation terms: weights printed, forms and the S0 level read
    lam_orphan: float = 0.01
    s0_orphan: float = 0.1
    lam_cont: float = 0.005
    lam_order: float = 0.01
    # Sec. 2.4 total variation of the upsampled bias field: weight read as 0.01
    lam_tv: float = 0.01


@dataclasses.dataclass
class Problem:
    """One independent problem: masked voxels of a box with one acquisition."""
    coords: np.ndarray           # int [V, 3] voxel coordinates inside the box
    shape: tuple                 # (nx, ny, nz) of the box (bias-basis coordinates)
    bval: np.ndarray             # [N] b-values, ms/um^2
    bvec: np.ndarray             # [N, 3] unit gradient directions
    K: int
    mode: str = "mse"            # "mse" | "nll"
    bias: str = "none"           # "none" | "poly2" | "trilinear8"
    learn_diffusivity: bool = False
    neighbourhood: int = 6       # 0, 6 or 26
    priors: tuple = ("spatial", "rep", "sparse", "cal")
    norm_count: Optional[int] = None   # |M|; defaults to the voxel count

    @property
    def V(self):
        return int(self.coords.shape[0])

    @property
    def N(self):
        return int(self.bval.shape[0])

    @property
    def M(self):
        # an empty group has only empty sums; any finite |M| leaves them at zero
        return float(max(self.V, 1) if self.norm_count is None else self.norm_count)

    @property
    def C(self):
        return self.K + 3


MICRO_KEYS = ("s0", "logits", "v", "fin", "dpar", "dperp")
CAL_KEYS = ("bias", "alpha", "beta", "sigma_log")


# ----------------------------------------------------------------------------
# elementary transforms (Sec. 2.2 per-voxel parameters; Sec. 2.5 constraints)
# ----------------------------------------------------------------------------

def softplus(x):
    x = np.asarray(x, dtype=np.float64)
    return np.logaddexp(0.0, x)


def sigmoid(x):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def softmax(logits, axis=0):
    z = np.asarray(logits, dtype=np.float64)
    z = z - z.max(axis=axis, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=axis, keepdims=True)


def transforms(prob: Problem, th: dict, c: Constants = Constants()):
    S0 = softplus(th["s0"])
    f = softmax(th["logits"], axis=0)                  # [C, V]
    v = np.asarray(th["v"], dtype=np.float64)          # [K, 3, V]
    vn = np.linalg.norm(v, axis=1)                     # [K, V]
    d = v / vn[:, None, :]
    fin = sigmoid(th["fin"])
    V = prob.V
    if prob.learn_diffusivity:
        dpar = softplus(th["dpar"])
        dperp = softplus(th["dperp"])
    else:
        dpar = np.full(V, c.d_par)
        dperp = np.full(V, c.d_perp)
    return dict(S0=S0, f=f, d=d, vn=vn, fin=fin, dpar=dpar, dperp=dperp)


# ----------------------------------------------------------------------------
# bias basis (Sec. 2.3 item 1; a linear log-bias basis)
# ----------------------------------------------------------------------------

def unit_box_coords(prob: Problem):
    """xi_a = (2 i_a - (n_a - 1)) / (n_a - 1) in [-1, 1]; 0 on an axis of size 1."""
    xi = np.zeros((prob.V, 3))
    for a in range(3):
        n = prob.shape[a]
        if n > 1:
            xi[:, a] = (2.0 * prob.coords[:, a] - (n - 1)) / (n - 1)
    return xi


def bias_basis(prob: Problem) -> np.ndarray:
    """Phi [n_bias, V] with log B(x) = sum_j c_j Phi_j(x)."""
    if prob.bias == "none":
        return np.zeros((0, prob.V))
    if prob.bias == "poly2":
        x, y, z = unit_box_coords(prob).T
        return np.stack([np.ones_like(x), x, y, z, x * x, y * y, z * z, x * y, x * z, y * z])
    if prob.bias == "trilinear8":
        # trilinear upsampling of an 8^3 control grid, corners aligned with the
        # first and last voxel of each axis (control point i sits at i (n-1)/7)
        phi = np.zeros((8, 8, 8, prob.V))
        idx = []
        for a in range(3):
            n = prob.shape[a]
            p = prob.coords[:, a] * (7.0 / (n - 1)) if n > 1 else np.zeros(prob.V)
            i0 = np.minimum(np.floor(p).astype(int), 6)
            idx.append((i0, p - i0))
        vox = np.arange(prob.V)
        for cx in (0, 1):
            wx = idx[0][1] if cx else 1.0 - idx[0][1]
            for cy in (0, 1):
                wy = idx[1][1] if cy else 1.0 - idx[1][1]
                for cz in (0, 1):
                    wz = idx[2][1] if cz else 1.0 - idx[2][1]
                    np.add.at(phi, (idx[0][0] + cx, idx[1][0] + cy, idx[2][0] + cz, vox), wx * wy * wz)
        return phi.reshape(512, prob.V)
    raise ValueError(prob.bias)


# ----------------------------------------------------------------------------
# forward model
# ----------------------------------------------------------------------------

def fibre_terms(b, G, d_k, dpar, dperp, fin):
    """Eq. 5 for one fibre: returns E, cos(theta), exp(-b Dpar c^2), exp(-b Dperp sin^2)."""
    cth = G @ d_k                                   # [N, V]  cos(theta) = g_n . d_k
    c2 = cth * cth
    e1 = np.exp(-b * dpar[None, :] * c2)            # stick
    e2 = np.exp(-b * dperp[None, :] * (1.0 - c2))   # extra radial decay of the zeppelin
    E = fin[None, :] * e1 + (1.0 - fin[None, :]) * e1 * e2
    return E, cth, e1, e2


def forward_constrained(bval, bvec, S0, f, d, fin, dpar, dperp, logB, alpha, beta,
                        c: Constants = Constants()):
    """Eq. 3-6 from constrained parameters: f [C, V] (csf, gm, wm_1..K, res),
    d [K, 3, V] unit, fin [V], dpar/dperp [V], logB [V], alpha/beta [N]."""
    b = np.asarray(bval, dtype=np.float64)[:, None]
    G = np.asarray(bvec, dtype=np.float64)
    K = d.shape[0]
    S = (f[0][None] * np.exp(-b * c.d_csf)          # Eq. 4
         + f[1][None] * np.exp(-b * c.d_gm)
         + f[K + 2][None] * np.exp(-b * c.d_res))
    for k in range(K):
        E, _, _, _ = fibre_terms(b, G, d[k], dpar, dperp, fin)
        S = S + f[2 + k][None] * E
    S = S0[None] * S                                 # Eq. 3
    return np.exp(alpha)[:, None] * np.exp(logB)[None, :] * S + np.asarray(beta)[:, None]  # Eq. 6


def synthesize(prob: Problem, th: dict, c: Constants = Constants()):
    tr = transforms(prob, th, c)
    Phi = bias_basis(prob)
    logB = Phi.T @ np.asarray(th["bias"], dtype=np.float64) if Phi.shape[0] else np.zeros(prob.V)
    return forward_constrained(prob.bval, prob.bvec, tr["S0"], tr["f"], tr["d"], tr["fin"],
                               tr["dpar"], tr["dperp"], logB,
                               np.asarray(th["alpha"], dtype=np.float64),
                               np.asarray(th["beta"], dtype=np.float64), c)


# ----------------------------------------------------------------------------
# Bessel functions for Eq. 9
# ----------------------------------------------------------------------------

def log_i0(z):
    """log I0(z) = |z| + log(exp(-|z|) I0(z)), finite for every real z."""
    z = np.abs(np.asarray(z, dtype=np.float64))
    return z + np.log(i0e(z))


def bessel_ratio(z):
    """R(z) = I1(z) / I0(z) (odd in z)."""
    z = np.asarray(z, dtype=np.float64)
    return i1e(z) / i0e(z)


# ----------------------------------------------------------------------------
# data terms (Eq. 8, Eq. 9)
# ----------------------------------------------------------------------------

def data_term(prob: Problem, yhat, y, sigma_log):
    y = np.asarray(y, dtype=np.float64)
    if prob.mode == "mse":
        return float(((yhat - y) ** 2).sum() / prob.M)
    s2 = np.exp(2.0 * float(sigma_log))
    z = y * yhat / s2
    terms = np.log(s2) + (y * y + yhat * yhat) / (2.0 * s2) - log_i0(z)
    return float(terms.sum())


def data_term_grad(prob: Problem, yhat, y, sigma_log):
    """dL_data / dyhat [N, V] and dL_data / dsigma_log."""
    y = np.asarray(y, dtype=np.float64)
    if prob.mode == "mse":
        return 2.0 * (yhat - y) / prob.M, 0.0
    s2 = np.exp(2.0 * float(sigma_log))
    z = y * yhat / s2
    R = bessel_ratio(z)
    gy = yhat / s2 - (y / s2) * R
    # d/dsigma_log of log s2 + (y^2+yhat^2)/(2 s2) - log I0(y yhat / s2)
    gs = (2.0 - (y * y + yhat * yhat) / s2 + 2.0 * z * R).sum()
    return gy, float(gs)


# ----------------------------------------------------------------------------
# priors (Sec. 2.4)
# ----------------------------------------------------------------------------

def neighbour_table(prob: Problem):
    """nb [V, n_off] indices of in-mask neighbours inside the box, -1 if absent."""
    if prob.neighbourhood == 0:
        return np.zeros((prob.V, 0), dtype=np.int64)
    if prob.neighbourhood == 6:
        offs = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    elif prob.neighbourhood == 26:
        offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
                if (a, b, c) != (0, 0, 0)]
    else:
        raise ValueError(prob.neighbourhood)
    grid = -np.ones(prob.shape, dtype=np.int64)
    cx, cy, cz = prob.coords.T
    grid[cx, cy, cz] = np.arange(prob.V)
    nb = -np.ones((prob.V, len(offs)), dtype=np.int64)
    for j, (a, b, c) in enumerate(offs):
        x, y, z = cx + a, cy + b, cz + c
        ok = (x >= 0) & (x < prob.shape[0]) & (y >= 0) & (y < prob.shape[1]) & (z >= 0) & (z < prob.shape[2])
        nb[ok, j] = grid[x[ok], y[ok], z[ok]]
    return nb


def huber(r, delta):
    a = np.abs(r)
    return np.where(a <= delta, 0.5 * r * r, delta * (a - 0.5 * delta))


def huber_grad(r, delta):
    return np.where(np.abs(r) <= delta, r, delta * np.sign(r))


def spatial_prior(prob: Problem, f, c: Constants, with_grad=True):
    """Eq. 7: (lam_sp/|M|) sum_x rho(f(x) - mean_{N(x)} f), rho per component."""
    nb = neighbour_table(prob)
    V = prob.V
    valid = nb >= 0
    cnt = valid.sum(1)                              # |N(x)|
    has = cnt > 0
    acc = np.zeros_like(f)
    for j in range(nb.shape[1]):
        sel = valid[:, j]
        acc[:, sel] += f[:, nb[sel, j]]
    mean = np.where(has[None], acc / np.maximum(cnt, 1)[None], 0.0)
    r = np.where(has[None], f - mean, 0.0)
    scale = c.lam_sp / prob.M
    loss = scale * float(huber(r, c.huber_delta).sum())
    if not with_grad:
        return loss, None
    q = np.where(has[None], huber_grad(r, c.huber_delta), 0.0)   # rho'(r(x))
    g = q.copy()
    w = q / np.maximum(cnt, 1)[None]
    for j in range(nb.shape[1]):
        sel = valid[:, j]
        # f(x') with x' in N(x) enters r(x) with weight -1/|N(x)|
        np.add.at(g, (slice(None), nb[sel, j]), -w[:, sel])
    return loss, scale * g


def repulsion_prior(prob: Problem, f, d, c: Constants):
    """lam_rep/|M| sum_x sum_{i<j} f_i f_j |d_i . d_j| over the WM fibres."""
    K = prob.K
    fw = f[2:2 + K]
    scale = c.lam_rep / prob.M
    loss = 0.0
    gf = np.zeros_like(fw)
    gd = np.zeros_like(d)
    for i in range(K):
        for j in range(i + 1, K):
            dot = (d[i] * d[j]).sum(0)
            loss += float((fw[i] * fw[j] * np.abs(dot)).sum())
            s = np.sign(dot)
            gf[i] += fw[j] * np.abs(dot)
            gf[j] += fw[i] * np.abs(dot)
            gd[i] += (fw[i] * fw[j] * s)[None] * d[j]
            gd[j] += (fw[i] * fw[j] * s)[None] * d[i]
    return scale * loss, scale * gf, scale * gd


def sparsity_prior(prob: Problem, f, c: Constants):
    """lam_sparse/|M| sum_x sum_k f_k 1[f_k < tau] over the WM fibres."""
    K = prob.K
    fw = f[2:2 + K]
    ind = (fw < c.tau_sparse).astype(np.float64)
    scale = c.lam_sparse / prob.M
    return scale * float((fw * ind).sum()), scale * ind


def calibration_prior(th: dict, c: Constants):
    a = np.asarray(th["alpha"], dtype=np.float64)
    b = np.asarray(th["beta"], dtype=np.float64)
    w = np.asarray(th["bias"], dtype=np.float64)
    loss = c.lam_alpha * (a * a).sum() + c.lam_beta * (b * b).sum() + c.lam_bias * (w * w).sum()
    return float(loss), 2 * c.lam_alpha * a, 2 * c.lam_beta * b, 2 * c.lam_bias * w


def orphan_prior(prob: Problem, S0, f, c: Constants):
    """Orphan-WM suppression (Sec. 2.4): WM fractions are penalised where S0 is
    near zero, read as (lam/|M|) sum_x h(S0(x)) sum_k f_wm,k(x) with the hinge
    h(s) = max(0, 1 - s/s_o).  Returns the loss and dR/dS0, dR/df_wm."""
    K = prob.K
    fw_sum = f[2:2 + K].sum(0)
    h = np.maximum(0.0, 1.0 - S0 / c.s0_orphan)
    scale = c.lam_orphan / prob.M
    loss = scale * float((h * fw_sum).sum())
    g_S0 = np.where(S0 < c.s0_orphan, -(scale / c.s0_orphan) * fw_sum, 0.0)
    g_f = scale * np.repeat(h[None], K, axis=0)
    return loss, g_S0, g_f


def continuity_prior(prob: Problem, d, c: Constants):
    """Directional continuity (Sec. 2.4): fibre k of a voxel is pulled toward
    fibre k of its neighbours, read as
    (lam/|M|) sum_x 1/|N(x)| sum_{x' in N(x)} sum_k (1 - (d_k(x).d_k(x'))^2),
    sign-free like the fibre model.  N(x) is the Eq. 7 neighbourhood.
    Returns the loss and dR/dd (unit directions)."""
    K = prob.K
    scale = c.lam_cont / prob.M
    gd = np.zeros_like(d)
    nb = neighbour_table(prob)
    if nb.shape[1] == 0:
        return 0.0, gd
    valid = nb >= 0
    cnt = valid.sum(1)
    a = np.where(cnt > 0, 1.0 / np.maximum(cnt, 1), 0.0)       # 1/|N(x)|
    loss = 0.0
    for j in range(nb.shape[1]):
        x = np.nonzero(valid[:, j])[0]
        u = nb[x, j]
        for k in range(K):
            dot = (d[k][:, x] * d[k][:, u]).sum(0)
            loss += float((a[x] * (1.0 - dot * dot)).sum())
            # the pair (x, u) appears in the sums of x and of u (N is symmetric)
            gd[k][:, x] += (-2.0 * (a[x] + a[u]) * dot)[None] * d[k][:, u]
    return scale * loss, scale * gd


def ordering_prior(prob: Problem, f, c: Constants):
    """Fibre ordering (Sec. 2.4): fibre slots are kept in descending order of
    fraction, read as (lam/|M|) sum_x sum_k max(0, f_wm,k+1 - f_wm,k).
    Returns the loss and dR/df_wm."""
    K = prob.K
    fw = f[2:2 + K]
    scale = c.lam_order / prob.M
    g = np.zeros_like(fw)
    loss = 0.0
    for k in range(K - 1):
        gap = fw[k + 1] - fw[k]
        on = gap > 0
        loss += float(gap[on].sum())
        g[k + 1] += on
        g[k] -= on
    return scale * loss, scale * g


def face_neighbours(prob: Problem):
    """nb [V, 6] in-mask face neighbours (-x, +x, -y, +y, -z, +z), -1 if absent."""
    grid = -np.ones(prob.shape, dtype=np.int64)
    cx, cy, cz = prob.coords.T
    grid[cx, cy, cz] = np.arange(prob.V)
    nb = -np.ones((prob.V, 6), dtype=np.int64)
    for a in range(3):
        for s, col in ((-1, 2 * a), (1, 2 * a + 1)):
            p = [cx.copy(), cy.copy(), cz.copy()]
            p[a] = p[a] + s
            ok = (p[a] >= 0) & (p[a] < prob.shape[a])
            nb[ok, col] = grid[p[0][ok], p[1][ok], p[2][ok]]
    return nb


def tv_prior(prob: Problem, logB, c: Constants):
    """Total variation of the bias field (Sec. 2.4 calibration regularisers),
    read as (lam_tv/|M|) sum over in-mask pairs (x, x + e_a) of
    |B(x + e_a) - B(x)|, B = exp(log-bias).  Returns the loss and dR/dlogB."""
    B = np.exp(logB)
    nb = face_neighbours(prob)
    scale = c.lam_tv / prob.M
    g = np.zeros(prob.V)
    loss = 0.0
    for a in range(3):
        x = np.nonzero(nb[:, 2 * a + 1] >= 0)[0]
        u = nb[x, 2 * a + 1]
        diff = B[u] - B[x]
        loss += float(np.abs(diff).sum())
        s = np.sign(diff)
        np.add.at(g, u, s * B[u])          # d|B(u) - B(x)| / dlogB(u)
        np.add.at(g, x, -s * B[x])         # d|B(u) - B(x)| / dlogB(x)
    return scale * loss, scale * g


# ----------------------------------------------------------------------------
# objective and its gradient (Sec. 2.5: L_data + sum_i lam_i R_i + R_cal)
# ----------------------------------------------------------------------------

TERMS = ("data", "spatial", "rep", "sparse", "orphan", "continuity", "ordering", "cal", "tv", "total")


def objective(prob: Problem, th: dict, y, c: Constants = Constants()):
    tr = transforms(prob, th, c)
    yhat = synthesize(prob, th, c)
    out = dict.fromkeys(TERMS, 0.0)
    out["data"] = data_term(prob, yhat, y, th.get("sigma_log", 0.0))
    if "spatial" in prob.priors and prob.neighbourhood:
        out["spatial"] = spatial_prior(prob, tr["f"], c, with_grad=False)[0]
    if "rep" in prob.priors:
        out["rep"] = repulsion_prior(prob, tr["f"], tr["d"], c)[0]
    if "sparse" in prob.priors:
        out["sparse"] = sparsity_prior(prob, tr["f"], c)[0]
    if "orphan" in prob.priors:
        out["orphan"] = orphan_prior(prob, tr["S0"], tr["f"], c)[0]
    if "continuity" in prob.priors:
        out["continuity"] = continuity_prior(prob, tr["d"], c)[0]
    if "ordering" in prob.priors:
        out["ordering"] = ordering_prior(prob, tr["f"], c)[0]
    if "cal" in prob.priors:
        out["cal"] = calibration_prior(th, c)[0]
    if "tv" in prob.priors and prob.bias != "none":
        Phi = bias_basis(prob)
        out["tv"] = tv_prior(prob, Phi.T @ np.asarray(th["bias"], dtype=np.float64), c)[0]
    out["total"] = sum(out[k] for k in TERMS[:-1])
    return out


def loss_grad(prob: Problem, th: dict, y, c: Constants = Constants()):
    """Loss terms and the exact gradient w.r.t. every raw parameter in `th`."""
    K, N, V = prob.K, prob.N, prob.V
    tr = transforms(prob, th, c)
    S0, f, d, vn, fin = tr["S0"], tr["f"], tr["d"], tr["vn"], tr["fin"]
    dpar, dperp = tr["dpar"], tr["dperp"]
    b = np.asarray(prob.bval, dtype=np.float64)[:, None]
    G = np.asarray(prob.bvec, dtype=np.float64)
    alpha = np.asarray(th["alpha"], dtype=np.float64)
    beta = np.asarray(th["beta"], dtype=np.float64)
    Phi = bias_basis(prob)
    logB = Phi.T @ np.asarray(th["bias"], dtype=np.float64) if Phi.shape[0] else np.zeros(V)
    sigma_log = float(th.get("sigma_log", 0.0))

    # forward (Eq. 3-6), keeping what the adjoint needs
    E_iso = [np.exp(-b * c.d_csf), np.exp(-b * c.d_gm), np.exp(-b * c.d_res)]   # [N, 1]
    fib = [fibre_terms(b, G, d[k], dpar, dperp, fin) for k in range(K)]
    mix = f[0][None] * E_iso[0] + f[1][None] * E_iso[1] + f[K + 2][None] * E_iso[2]
    for k in range(K):
        mix = mix + f[2 + k][None] * fib[k][0]
    S = S0[None] * mix
    AB = np.exp(alpha)[:, None] * np.exp(logB)[None, :]
    q = AB * S                          # yhat - beta
    yhat = q + beta[:, None]

    out = dict.fromkeys(TERMS, 0.0)
    out["data"] = data_term(prob, yhat, y, sigma_log)
    gy, g_sigma = data_term_grad(prob, yhat, y, sigma_log)

    grad = {}
    # calibration (Eq. 6)
    g_beta = gy.sum(1)
    g_alpha = (gy * q).sum(1)
    g_logB = (gy * q).sum(0)
    if "tv" in prob.priors and prob.bias != "none":
        l, gtv = tv_prior(prob, logB, c)
        out["tv"] = l
        g_logB = g_logB + gtv
    g_bias = Phi @ g_logB if Phi.shape[0] else np.zeros(0)
    gS = gy * AB                        # dL/dS [N, V]
    # tissue signal (Eq. 3)
    g_S0 = (gS * mix).sum(0)
    gSm = gS * S0[None]                 # dL/d(mix)
    g_f = np.zeros_like(f)
    g_f[0] = (gSm * E_iso[0]).sum(0)
    g_f[1] = (gSm * E_iso[1]).sum(0)
    g_f[K + 2] = (gSm * E_iso[2]).sum(0)
    g_d = np.zeros_like(d)
    g_fin = np.zeros(V)
    g_dpar = np.zeros(V)
    g_dperp = np.zeros(V)
    for k in range(K):
        E, cth, e1, e2 = fib[k]
        g_f[2 + k] = (gSm * E).sum(0)
        gE = gSm * f[2 + k][None]       # dL/dE_k
        # Eq. 5: E = fin e1 + (1-fin) e1 e2
        g_fin += (gE * (e1 - e1 * e2)).sum(0)
        dE_dc = (-2.0 * b * dpar[None] * cth * E
                 + 2.0 * b * dperp[None] * cth * (1.0 - fin[None]) * e1 * e2)
        gc = gE * dE_dc                 # dL/dcos(theta) [N, V]
        g_d[k] = G.T @ gc               # [3, V]
        if prob.learn_diffusivity:
            c2 = cth * cth
            g_dpar += (gE * (-b * c2) * E).sum(0)
            g_dperp += (gE * (-b * (1.0 - c2)) * (1.0 - fin[None]) * e1 * e2).sum(0)

    # priors
    if "spatial" in prob.priors and prob.neighbourhood:
        l, gsp = spatial_prior(prob, f, c)
        out["spatial"] = l
        g_f = g_f + gsp
    if "rep" in prob.priors:
        l, gfr, gdr = repulsion_prior(prob, f, d, c)
        out["rep"] = l
        g_f[2:2 + K] += gfr
        g_d = g_d + gdr
    if "sparse" in prob.priors:
        l, gfs = sparsity_prior(prob, f, c)
        out["sparse"] = l
        g_f[2:2 + K] += gfs
    if "orphan" in prob.priors:
        l, gso, gfo = orphan_prior(prob, S0, f, c)
        out["orphan"] = l
        g_S0 = g_S0 + gso
        g_f[2:2 + K] += gfo
    if "continuity" in prob.priors:
        l, gdc = continuity_prior(prob, d, c)
        out["continuity"] = l
        g_d = g_d + gdc
    if "ordering" in prob.priors:
        l, gfo = ordering_prior(prob, f, c)
        out["ordering"] = l
        g_f[2:2 + K] += gfo
    if "cal" in prob.priors:
        l, ga, gb, gw = calibration_prior(th, c)
        out["cal"] = l
        g_alpha = g_alpha + ga
        g_beta = g_beta + gb
        g_bias = g_bias + gw
    out["total"] = sum(out[k] for k in TERMS[:-1])

    # chain rule to the raw parameters (Sec. 2.5 constraints)
    grad["s0"] = sigmoid(th["s0"]) * g_S0                               # softplus'
    grad["logits"] = f * (g_f - (f * g_f).sum(0, keepdims=True))        # softmax'
    gv = np.zeros_like(g_d)
    for k in range(K):
        proj = (g_d[k] * d[k]).sum(0)
        gv[k] = (g_d[k] - proj[None] * d[k]) / vn[k][None]              # (I - d d^T)/|v|
    grad["v"] = gv
    grad["fin"] = fin * (1.0 - fin) * g_fin                             # sigmoid'
    if prob.learn_diffusivity:
        grad["dpar"] = sigmoid(th["dpar"]) * g_dpar
        grad["dperp"] = sigmoid(th["dperp"]) * g_dperp
    grad["bias"] = g_bias
    grad["alpha"] = g_alpha
    grad["beta"] = g_beta
    grad["sigma_log"] = np.array(g_sigma if prob.mode == "nll" else 0.0)
    return out, grad, yhat


# ----------------------------------------------------------------------------
# whole-volume slabs and their stitching (Sec. 2.5)
# ----------------------------------------------------------------------------

def slab_ranges(nz: int, thickness: int = 30, overlap: int = 5):
    """(first slice, slices) of each slab along z.  Slabs start every
    thickness - overlap slices until one reaches the end of the volume; the
    last one stops at the volume's edge and may be thinner (reading: the paper
    gives only the thickness and the overlap).  Needs thickness >= 2 overlap,
    so that no slice lies in more than two slabs."""
    if not (0 <= 2 * overlap <= thickness):
        raise ValueError("need 0 <= 2 overlap <= thickness")
    out = []
    z = 0
    while True:
        out.append((z, min(thickness, nz - z)))
        if z + thickness >= nz:
            return out
        z += thickness - overlap


def slab_weights(z0, thickness):
    """Blend weight of each slab at each of its slices (reading of the paper's
    weighted averaging): a linear ramp across each overlap with a neighbouring
    slab, (s + 1)/(o + 1) at the s-th slice counted from the slab's edge for an
    overlap of o slices, and 1 elsewhere.  The two ramps over an overlap sum to
    one at every slice."""
    G = len(z0)
    out = []
    for g in range(G):
        a, b = z0[g], z0[g] + thickness[g]
        o_lo = max(0, z0[g - 1] + thickness[g - 1] - a) if g > 0 else 0
        o_hi = max(0, b - z0[g + 1]) if g + 1 < G else 0
        z = np.arange(a, b, dtype=np.float64)
        w = np.ones(b - a)
        if o_lo:
            w = np.minimum(w, (z - a + 1.0) / (o_lo + 1.0))
        if o_hi:
            w = np.minimum(w, (b - z) / (o_hi + 1.0))
        out.append(w)
    return out


def constrained_maps(prob: Problem, th: dict, c: Constants = Constants()):
    """Per-voxel constrained quantities [P][V] in the row order of theta_micro:
    S0, fractions, unit directions, f_intra (and D_par, D_perp)."""
    tr = transforms(prob, th, c)
    rows = [tr["S0"][None], tr["f"], tr["d"].reshape(3 * prob.K, prob.V), tr["fin"][None]]
    if prob.learn_diffusivity:
        rows += [tr["dpar"][None], tr["dperp"][None]]
    return np.concatenate(rows, axis=0)


def stitch_slabs(full_shape, z0, slabs, thetas, c: Constants = Constants()):
    """Stitch per-slab fits into whole-volume maps (Sec. 2.5).

    slabs[g] is the Problem of slab g (box nx x ny x nz_g, its own voxel
    list), placed at slices z0[g].. of a volume of shape `full_shape`.
    Returns (coords [V_out, 3] of the union of the slabs' voxels in raster
    order, maps [P][V_out]).  A voxel seen by one slab takes its values.  In
    an overlap the two slabs are blended with the `slab_weights`; the fibres
    of the lighter slab (the upper one on a tie) are first matched to the
    heavier slab's slots, taking for each slot in turn the unmatched fibre
    with the largest |cos| (the lowest index on ties; decided in float32, the
    precision of the fitted directions), and flipped to the same sign.  The
    blended directions are renormalised; the output keeps the heavier slab's
    slot order."""
    nx, ny, nz = full_shape
    K = slabs[0].K
    w = slab_weights(list(z0), [p.shape[2] for p in slabs])
    maps = [constrained_maps(p, th, c) for p, th in zip(slabs, thetas)]
    src = {}
    for g, p in enumerate(slabs):
        for v, (i, j, k) in enumerate(p.coords):
            r = (int(i) * ny + int(j)) * nz + int(z0[g]) + int(k)
            src.setdefault(r, []).append((g, v, w[g][int(k)]))
    keys = sorted(src)
    C = K + 3
    P = maps[0].shape[0]
    out = np.zeros((P, len(keys)))
    coords = np.zeros((len(keys), 3), dtype=np.int64)
    for o, r in enumerate(keys):
        coords[o] = (r // (ny * nz), (r // nz) % ny, r % nz)
        s = src[r]
        if len(s) == 1:
            g, v, _ = s[0]
            out[:, o] = maps[g][:, v]
            continue
        (ga, va, wa), (gb, vb, wb) = s
        tot = wa + wb
        wa, wb = wa / tot, wb / tot
        if wa >= wb:
            (gr, vr, wr), (go, vo, wo) = (ga, va, wa), (gb, vb, wb)
        else:
            (gr, vr, wr), (go, vo, wo) = (gb, vb, wb), (ga, va, wa)
        mr, mo = maps[gr][:, vr], maps[go][:, vo]
        res = wr * mr + wo * mo                       # S0, csf, gm, res, f_intra, D
        dr = mr[1 + C:1 + C + 3 * K].reshape(K, 3)
        do = mo[1 + C:1 + C + 3 * K].reshape(K, 3)
        used = []
        dots = dr.astype(np.float32) @ do.astype(np.float32).T      # float32 [K, K]
        for k in range(K):
            best, bj = -1.0, -1
            for j in range(K):
                if j not in used and abs(float(dots[k, j])) > best:
                    best, bj = abs(float(dots[k, j])), j
            used.append(bj)
            sg = -1.0 if float(dots[k, bj]) < 0 else 1.0
            res[3 + k] = wr * mr[3 + k] + wo * mo[3 + bj]
            d = wr * dr[k] + wo * sg * do[bj]
            res[1 + C + 3 * k:1 + C + 3 * k + 3] = d / np.linalg.norm(d)
        out[:, o] = res
    return coords, out


# ----------------------------------------------------------------------------
# optimisers
# ----------------------------------------------------------------------------

def adam_step(p, g, m, v, t, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, Algorithm 1) at step t >= 1, PyTorch form:
    p -= lr / (1 - beta1^t) * m / (sqrt(v) / sqrt(1 - beta2^t) + eps)."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    bc1 = 1.0 - beta1 ** t
    bc2 = 1.0 - beta2 ** t
    p = p - (lr / bc1) * m / (np.sqrt(v) / np.sqrt(bc2) + eps)
    return p, m, v


def rprop_step(p, g, prev_g, step, etas=(0.5, 1.2), step_sizes=(1e-6, 50.0)):
    """One Rprop step (Riedmiller & Braun 1993) in PyTorch's variant: the step
    size grows by eta+ when the gradient keeps its sign, shrinks by eta- when it
    flips (and that coordinate does not move and forgets its gradient), and the
    parameter moves by -sign(g) * step."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64).copy()
    prod = g * np.asarray(prev_g, dtype=np.float64)
    fac = np.where(prod > 0, etas[1], np.where(prod < 0, etas[0], 1.0))
    step = np.clip(np.asarray(step, dtype=np.float64) * fac, step_sizes[0], step_sizes[1])
    g = np.where(prod < 0, 0.0, g)
    p = p - np.sign(g) * step
    return p, g, step
