"""The Rician NLL's special functions (Eq. 9) as the kernels evaluate them.

The generator's host emulation runs the kernels' algorithm step by step in
float32 / float64 (the hardware reciprocal and log2 modelled as correctly
rounded) over float32 arguments in [0, 1e5]; its results must lie within
2e-7 relative of SciPy's float64 i0e / i1e for log I0e(z), 1 - I1(z)/I0(z)
and 2z (1 - I1/I0).  The committed coefficient table must be the one the
generator writes, and the emulation must agree with independent limits:
the small-argument series and the large-argument expansion."""
import importlib.util
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2604_00250_amd", "csrc")
BOUND = 2e-7


def _gen():
    spec = importlib.util.spec_from_file_location("gen_bessel_fit", os.path.join(CSRC, "gen_bessel_fit.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def gen():
    return _gen()


@pytest.fixture(scope="module")
def emulated(gen):
    z = gen.test_grid()
    return z, gen.evaluate_f32(z)


def test_float32_algorithm_meets_the_bound_on_0_to_1e5(gen, emulated):
    z, vals = emulated
    assert z[0] == 0.0 and z[-1] == np.float32(1e5) and z.size > 500_000
    e_li, e_omr, e_q = gen.relative_errors(z, vals)
    print(f"max relative error: log I0e {e_li.max():.3e}, 1-R {e_omr.max():.3e}, q {e_q.max():.3e}")
    assert e_li.max() <= BOUND
    assert e_omr.max() <= BOUND
    assert e_q.max() <= BOUND


def test_both_branches_are_exercised_and_continuous_at_the_split(gen, emulated):
    z, (li, omr, q) = emulated
    split = np.float32(gen.Z_SPLIT)
    below, above = z[z < split].max(), z[z >= split].min()
    assert below == np.nextafter(split, np.float32(0)) and above == split
    i, j = np.searchsorted(z, below), np.searchsorted(z, above)
    # neighbouring float32 arguments on either side of the split: the jump is a few ulp
    assert abs(li[j] - li[i]) <= 4 * np.spacing(abs(li[i]))
    assert abs(omr[j] - omr[i]) <= 4 * np.spacing(omr[i])


def test_limits_independent_of_scipy(gen):
    """z -> 0: log I0e(z) = -z + z^2/4 - z^4/64 + ..., 1 - R = 1 - z/2 + z^3/16 - ...;
    z -> inf: log I0e(z) = -log(2 pi z)/2 + 1/(8z) + 9/(128 z^2) + ...,
    2z(1 - R) = 1 + 1/(4z) + 3/(16 z^2) + ..."""
    zs = np.array([1e-6, 1e-4, 1e-3], dtype=np.float32)
    li, omr, _ = gen.evaluate_f32(zs)
    z = zs.astype(np.float64)
    assert np.allclose(li, -z + z ** 2 / 4 - z ** 4 / 64, rtol=2e-7, atol=0)
    assert np.allclose(omr, 1 - z / 2 + z ** 3 / 16, rtol=2e-7, atol=0)
    zl = np.array([2e4, 5e4, 1e5], dtype=np.float32)
    li, omr, q = gen.evaluate_f32(zl)
    z = zl.astype(np.float64)
    assert np.allclose(li, -0.5 * np.log(2 * np.pi * z) + 1 / (8 * z) + 9 / (128 * z ** 2), rtol=2e-7, atol=0)
    assert np.allclose(q, 1 + 1 / (4 * z) + 3 / (16 * z ** 2), rtol=2e-7, atol=0)


def _arrays(text):
    import re
    out = {}
    for m in re.finditer(r"(k\w+)\[[^\]]+\] = \{([^}]*)\}", text):
        out[m.group(1)] = np.array([float(v.strip().rstrip("f")) for v in m.group(2).split(",")])
    return out


def test_committed_table_is_the_generators(gen, tmp_path):
    """The kernels' coefficient tables are what the generator fits (up to the
    last bits a different LAPACK build may change)."""
    out = tmp_path / "bessel_fit.h"
    gen.main(out=str(out))
    new = _arrays(out.read_text())
    old = _arrays(open(os.path.join(CSRC, "bessel_fit.h")).read())
    assert set(new) == set(old) and len(old) == 8
    for k in old:
        assert np.allclose(new[k], old[k], rtol=1e-6, atol=1e-12), k
