"""Generate bessel_fit.h: coefficient tables for the Rician NLL (Eq. 9).

The kernels need, for z >= 0,
    log I0e(z) = log I0(z) - z          (the cancellation-free NLL term)
    1 - R(z),  R = I1 / I0              (the NLL adjoint)
    q(z) = 2 z (1 - R(z))               (the d/dsigma_log term)

Small arguments, z < 3.75, are evaluated in float64 (on CDNA3/4 a float64
FMA issues at the rate of a float32 one) from two even functions of t = z^2,
fitted here as Chebyshev series in x = 2 t / 3.75^2 - 1 and stored as
polynomials in x (evaluated by Estrin's scheme in float64; the coefficients
stay below 0.3 in magnitude, so the conversion is well conditioned):
    G(t)   = log I0(z) / t      ->  log I0e(z) = t G(t) - z
    rho(t) = R(z) / z           ->  1 - R(z)   = 1 - z rho(t)
each result rounded to float32 once.

Large arguments use two functions of u = 3.75 / z in (0, 1],
    l(u) = log(sqrt(2 pi z) I0e(z))     (-> 0 as z -> inf, like u/30)
    d(u) = 2 z (1 - R(z)) - 1           (-> 0 as z -> inf, like u/15)
as rational functions u P(x) / Q(x) of x = 2u - 1 (Q(x) = 1 + q1 x + ...,
fitted by Sanathanan-Koerner iterations of linear least squares with relative
weights; Horner in float32, one reciprocal), so that
log I0e(z) = (l - log(2 pi)/2) - log(z)/2, q = 1 + d and
1 - R = (1 + d) / (2z) = d r + r with r = 1/(2z): l and d are small
corrections to leading terms that are exact or a single rounding, so the
rational's own rounding hardly shows, and nothing cancels.  d's rational
covers z <= 2000 (fitted over the whole range its denominator comes near
zero); above, d = w/4 + w^2/4 + 25 w^3/64 with w = 1/z, the large-argument
expansion of 2z(1 - I1/I0), whose next term is below 1e-11 relative there.

`evaluate_f32` below is the kernels' algorithm step by step in float32 and
float64 arithmetic on the host (hardware reciprocal and log2 modelled as
correctly rounded float32), used by the tests to bound the error against
SciPy's float64 i0e / i1e.  Run from the repository root to regenerate:
    python paper_2604_00250_amd/csrc/gen_bessel_fit.py
"""
import os

import numpy as np
from scipy.special import i0e, i1e

Z_SPLIT = 3.75
DEG_G = 12
DEG_RHO = 14
DEG_L = (5, 5)     # numerator, denominator degrees of l
DEG_D = (6, 6)     # ... of d, fitted for z <= Z_ASYM
Z_ASYM = 2000.0
HALF_LOG_2PI = 0.5 * np.log(2.0 * np.pi)
HALF_LN2 = 0.5 * np.log(2.0)


# ----------------------------------------------------------------------------
# target functions (float64, SciPy)
# ----------------------------------------------------------------------------

def small_targets(t):
    """G(t) = log I0(z)/t and rho(t) = R(z)/z at z = sqrt(t) (limits 1/4, 1/2 at t = 0)."""
    t = np.asarray(t, dtype=np.float64)
    z = np.sqrt(t)
    e0, e1 = i0e(z), i1e(z)
    with np.errstate(invalid="ignore", divide="ignore"):
        G = np.where(t > 1e-12, (np.log(e0) + z) / t, 0.25 - t / 64.0)
        rho = np.where(t > 1e-12, e1 / (e0 * z), 0.5 - t / 16.0)
    return G, rho


def large_targets(u):
    z = Z_SPLIT / np.asarray(u, dtype=np.float64)
    e0 = i0e(z)
    l = np.log(np.sqrt(2 * np.pi * z) * e0)
    d = 2 * z * (e0 - i1e(z)) / e0 - 1.0
    return l, d


def fit(deg, fn, relative, n=None):
    """Least squares on Chebyshev nodes of (-1, 1); fn takes x."""
    k = np.arange(n or 8 * deg)
    x = -np.cos(np.pi * (k + 0.5) / len(k))
    y = fn(x)
    w = 1.0 / np.abs(y) if relative else np.ones_like(y)
    V = np.polynomial.chebyshev.chebvander(x, deg)
    coef, *_ = np.linalg.lstsq(V * w[:, None], y * w, rcond=None)
    return coef


def rational_fit(fn, m, n, u_lo=Z_SPLIT / 1e5, iters=40, npts=6000):
    """fn(u) ~ u P(x)/Q(x), x = 2u - 1 over u in [u_lo, 1]; P, Q monomial in x
    (lowest degree first), Q[0] = 1.  Sanathanan-Koerner: repeated linear least
    squares of u P - fn Q, reweighted by 1/|Q| and by the target's size."""
    k = np.arange(npts)
    x = -np.cos(np.pi * (k + 0.5) / npts)
    x = x[(x + 1.0) * 0.5 >= u_lo]
    u = (x + 1.0) * 0.5
    y = fn(u) / u
    w = np.ones_like(u)
    for _ in range(iters):
        A = np.concatenate([np.vander(x, m + 1, increasing=True),
                            -y[:, None] * np.vander(x, n + 1, increasing=True)[:, 1:]], 1)
        s = w / np.abs(y)
        sol, *_ = np.linalg.lstsq(A * s[:, None], y * s, rcond=None)
        p, q = sol[:m + 1], np.concatenate([[1.0], sol[m + 1:]])
        w = 1.0 / np.abs(np.polyval(q[::-1], x))
    # no pole in the interval: the denominator keeps its sign and stays away from zero
    xs = np.linspace(-1.0, 1.0, 100_001)
    Q = np.polyval(q[::-1], xs)
    assert Q.min() > 0.05, f"denominator of the rational fit comes near zero ({Q.min():.3g})"
    return p, q


def fits():
    tmax = Z_SPLIT ** 2
    # small branch: Chebyshev fits converted to polynomials in x
    cG = np.polynomial.chebyshev.cheb2poly(
        fit(DEG_G, lambda x: small_targets((x + 1) * 0.5 * tmax)[0], relative=True))
    cR = np.polynomial.chebyshev.cheb2poly(
        fit(DEG_RHO, lambda x: small_targets((x + 1) * 0.5 * tmax)[1], relative=True))
    lP, lQ = rational_fit(lambda u: large_targets(u)[0], *DEG_L)
    dP, dQ = rational_fit(lambda u: large_targets(u)[1], *DEG_D, u_lo=Z_SPLIT / Z_ASYM)
    return cG, cR, (lP, lQ), (dP, dQ)


# ----------------------------------------------------------------------------
# host emulation of the kernels' evaluation
# ----------------------------------------------------------------------------

f32 = np.float32


def _fma32(a, b, c):
    # the product of two float32 values is exact in float64; one rounding to float32
    return f32(np.float64(a) * np.float64(b) + np.float64(c))


def _horner32(p, x):
    p = np.asarray(p, dtype=f32)
    acc = np.full_like(x, p[-1])
    for a in p[-2::-1]:
        acc = _fma32(acc, x, a)
    return acc


def _rcp32(x):
    return f32(1.0 / np.asarray(x, np.float64))                  # v_rcp_f32


def _rational32(pq, x, u):
    P, Q = pq
    return f32(f32(u * _horner32(P, x)) * _rcp32(_horner32(Q, x)))


def _horner64(p, x):
    acc = np.full_like(x, p[-1])
    for a in p[-2::-1]:
        acc = acc * x + a
    return acc


def _estrin64(p, x):
    """Estrin's scheme in float64, in the kernels' order: pairs with x, then
    pairs of pairs with x^2, x^4, x^8."""
    p = [np.float64(a) for a in p]
    x2 = x * x
    x4 = x2 * x2
    x8 = x4 * x4
    lvl = [p[2 * i + 1] * x + p[2 * i] if 2 * i + 1 < len(p) else np.full_like(x, p[2 * i])
           for i in range((len(p) + 1) // 2)]
    for xp in (x2, x4, x8):
        if len(lvl) == 1:
            break
        lvl = [lvl[2 * i + 1] * xp + lvl[2 * i] if 2 * i + 1 < len(lvl) else lvl[2 * i]
               for i in range((len(lvl) + 1) // 2)]
    return lvl[0]


def _estrin32(p, x, x2, x4, x8):
    """Estrin's scheme in float32 (each step one FMA rounding), the kernels' order."""
    lvl = [_fma32(p[2 * i + 1], x, p[2 * i]) if 2 * i + 1 < len(p) else np.full_like(x, p[2 * i])
           for i in range((len(p) + 1) // 2)]
    for xp in (x2, x4, x8):
        if len(lvl) == 1:
            break
        lvl = [_fma32(lvl[2 * i + 1], xp, lvl[2 * i]) if 2 * i + 1 < len(lvl) else lvl[2 * i]
               for i in range((len(lvl) + 1) // 2)]
    return lvl[0]


def _small_poly(c, x):
    """sum_i c_i x^i for |x| <= 1 as the kernels take it: the four lowest terms in
    float64, the rest (weight x^4, coefficients below 0.015) as a float32
    polynomial with float32 coefficients, added in float64."""
    c = np.asarray(c, np.float64)
    x2 = x * x
    low = (c[3] * x + c[2]) * x2 + (c[1] * x + c[0])
    xf = x.astype(f32)
    xf2 = f32(xf * xf)
    xf4 = f32(xf2 * xf2)
    xf8 = f32(xf4 * xf4)
    hi = _estrin32(c[4:].astype(f32), xf, xf2, xf4, xf8)
    return (x2 * x2) * hi.astype(np.float64) + low


def _clenshaw64(c, x):
    x2 = x + x
    b1 = np.zeros_like(x)
    b2 = np.zeros_like(x)
    for a in c[:0:-1]:
        b1, b2 = x2 * b1 + (a - b2), b1
    return x * b1 + (c[0] - b2)


def evaluate_f32(z, coefs=None):
    """(log I0e(z), 1 - R(z), q(z)) for float32 z >= 0, as the kernels compute them."""
    cG, cR, cL, cD = fits() if coefs is None else coefs
    z = np.asarray(z, dtype=f32)
    li = np.zeros_like(z)
    omr = np.zeros_like(z)
    q = np.zeros_like(z)
    s = z < f32(Z_SPLIT)
    # small arguments: float64
    zd = z[s].astype(np.float64)
    t = zd * zd
    x = t * (2.0 / Z_SPLIT ** 2) - 1.0
    G = _small_poly(cG, x)
    rho = _small_poly(cR, x)
    w = 1.0 - zd * rho
    omr[s] = w.astype(f32)
    q[s] = (2.0 * zd * w).astype(f32)
    li[s] = (t * G - zd).astype(f32)
    # large arguments: float32
    zl = z[~s]
    iz0 = _rcp32(zl)
    iz = _fma32(_fma32(-zl, iz0, f32(1.0)), iz0, iz0)              # one Newton step
    x = _fma32(f32(2.0 * Z_SPLIT), iz, f32(-1.0))
    u = f32(f32(Z_SPLIT) * iz)
    l = _rational32(cL, x, u)
    d_asym = f32(iz * _fma32(iz, _fma32(iz, f32(25.0 / 64.0), f32(0.25)), f32(0.25)))
    d = np.where(zl > f32(Z_ASYM), d_asym, _rational32(cD, x, u))
    r = f32(f32(0.5) * iz)
    omr[~s] = _fma32(d, r, r)
    q[~s] = f32(f32(1.0) + d)
    lg = f32(np.log2(zl.astype(np.float64)))                      # v_log_f32
    li[~s] = _fma32(f32(-HALF_LN2), lg, f32(l - f32(HALF_LOG_2PI)))
    return li, omr, q


def reference(z):
    """float64 values at the float32 arguments."""
    z = np.asarray(z, dtype=np.float64)
    e0, e1 = i0e(z), i1e(z)
    omr = (e0 - e1) / e0
    return np.log(e0), omr, 2.0 * z * omr


def relative_errors(z, values):
    li, omr, q = (np.asarray(v, dtype=np.float64) for v in values)
    rl, ro, rq = reference(z)
    with np.errstate(invalid="ignore", divide="ignore"):
        e_li = np.where(rl != 0.0, np.abs(li - rl) / np.abs(rl), np.abs(li))
        e_omr = np.abs(omr - ro) / ro
        e_q = np.where(rq != 0.0, np.abs(q - rq) / np.abs(rq), np.abs(q))
    return e_li, e_omr, e_q


def test_grid():
    """float32 arguments over [0, 1e5]: zero, a log-spaced sweep, a dense linear
    sweep over the branch region and both sides of the split."""
    bits = np.array([Z_SPLIT], dtype=f32).view(np.uint32)[0]
    near = (np.int64(bits) + np.arange(-64, 64)).astype(np.uint32).view(f32)   # consecutive float32
    z = np.concatenate([np.array([0.0], f32), np.geomspace(1e-7, 1e5, 400_000).astype(f32),
                        np.linspace(0.0, 40.0, 400_000).astype(f32), near])
    z = np.unique(z)
    return z[(z >= 0) & (z <= f32(1e5))]


def main(out=None):
    cG, cR, cL, cD = fits()
    tmax = Z_SPLIT ** 2
    x = np.linspace(-1.0, 1.0, 200_001)
    G, rho = small_targets((x + 1) * 0.5 * tmax)
    eG = np.abs(_horner64(cG, x) / G - 1).max()
    eR = np.abs(_horner64(cR, x) / rho - 1).max()
    xl = np.linspace(2.0 * Z_SPLIT / 1e5 - 1.0, 1.0, 200_001)      # z in [3.75, 1e5]
    ul = (xl + 1) * 0.5
    l, d = large_targets(ul)
    rat = lambda pq: ul * np.polyval(pq[0][::-1], xl) / np.polyval(pq[1][::-1], xl)  # noqa: E731
    eL = np.abs(rat(cL) - l).max()
    zz = Z_SPLIT / ul
    d_asym = 1 / (4 * zz) + 1 / (4 * zz ** 2) + 25 / (64 * zz ** 3)
    eD = np.abs(np.where(zz > Z_ASYM, d_asym, rat(cD)) - d).max()
    z = test_grid()
    e_li, e_omr, e_q = relative_errors(z, evaluate_f32(z, (cG, cR, cL, cD)))
    print(f"fits: G rel {eG:.2e}, rho rel {eR:.2e}, l abs {eL:.2e}, d abs {eD:.2e}")
    print(f"float32 algorithm over {z.size} arguments in [0, 1e5]: max relative error "
          f"log I0e {e_li.max():.3e} (z={z[e_li.argmax()]:.6g}), 1-R {e_omr.max():.3e} "
          f"(z={z[e_omr.argmax()]:.6g}), q {e_q.max():.3e} (z={z[e_q.argmax()]:.6g})")
    out = out or os.path.join(os.path.dirname(os.path.abspath(__file__)), "bessel_fit.h")
    f32s = lambda cs: ", ".join(f"{float(f32(c))!r}f" for c in cs)  # noqa: E731
    f64s = lambda cs: ", ".join(f"{float(c)!r}" for c in cs)  # noqa: E731
    with open(out, "w") as f:
        f.write("// Generated by gen_bessel_fit.py -- do not edit.\n")
        f.write("// Eq. 9 special functions.  z < 3.75 (float64 with a float32 tail): polynomials in\n")
        f.write("// x = 2t/3.75^2 - 1, t = z^2,\n")
        f.write("// lowest degree first, of G = log I0(z)/t (kSmallG) and rho = I1(z)/(z I0(z)) (kSmallRho).\n")
        f.write("// z >= 3.75 (float32): rational functions u P(x)/Q(x), x = 2u - 1, u = 3.75/z, of\n")
        f.write("// l = log(sqrt(2 pi z) I0e(z)) (kLargeLP / kLargeLQ) and d = 2z(1 - I1/I0) - 1\n")
        f.write("// (kLargeDP / kLargeDQ); polynomials lowest degree first, Q[0] = 1.\n")
        f.write(f"// fit errors: G {eG:.1e} rel, rho {eR:.1e} rel, l {eL:.1e} abs, d {eD:.1e} abs;\n")
        f.write(f"// float32 algorithm on the host: log I0e {e_li.max():.2e}, 1-R {e_omr.max():.2e}, "
                f"q {e_q.max():.2e} max relative error over [0, 1e5]\n")
        f.write("#pragma once\n")
        f.write(f"#define PRISM_SMALL_G_N {len(cG)}\n#define PRISM_SMALL_RHO_N {len(cR)}\n")
        f.write(f"#define PRISM_LARGE_LP_N {len(cL[0])}\n#define PRISM_LARGE_LQ_N {len(cL[1])}\n")
        f.write(f"#define PRISM_LARGE_DP_N {len(cD[0])}\n#define PRISM_LARGE_DQ_N {len(cD[1])}\n")
        f.write(f"static constexpr float kBesselSplit = {Z_SPLIT!r}f;\n")
        f.write("// in constant memory: the float64 branch reads its four lowest coefficients where it\n")
        f.write("// runs (as literals, the compiler would hold them in scalar registers across the\n")
        f.write("// measurement loop); the higher ones, times x^4, are float32 literals (kSmallGHi,\n")
        f.write("// kSmallRhoHi)\n")
        f.write(f"static __constant__ double kSmallG[PRISM_SMALL_G_N] = {{{f64s(cG)}}};\n")
        f.write(f"static __constant__ double kSmallRho[PRISM_SMALL_RHO_N] = {{{f64s(cR)}}};\n")
        f.write(f"static constexpr float kSmallGHi[PRISM_SMALL_G_N - 4] = {{{f32s(cG[4:])}}};\n")
        f.write(f"static constexpr float kSmallRhoHi[PRISM_SMALL_RHO_N - 4] = {{{f32s(cR[4:])}}};\n")
        f.write(f"static constexpr float kLargeLP[PRISM_LARGE_LP_N] = {{{f32s(cL[0])}}};\n")
        f.write(f"static constexpr float kLargeLQ[PRISM_LARGE_LQ_N] = {{{f32s(cL[1])}}};\n")
        f.write(f"static constexpr float kLargeDP[PRISM_LARGE_DP_N] = {{{f32s(cD[0])}}};\n")
        f.write(f"static constexpr float kLargeDQ[PRISM_LARGE_DQ_N] = {{{f32s(cD[1])}}};\n")
        f.write(f"static constexpr float kAsymZ = {Z_ASYM!r}f;   // d from its expansion above this z\n")
        f.write(f"static constexpr float kHalfLog2Pi = {float(f32(HALF_LOG_2PI))!r}f;\n")
        f.write(f"static constexpr float kHalfLn2 = {float(f32(HALF_LN2))!r}f;\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
