"""Eq. 9 on the GPU: the device's special functions against SciPy over
float32 arguments in [0, 1e5] (the 2e-7 relative bound), and parity of the
Rician NLL pass with the oracle where z = |y| |yhat| / sigma^2 reaches 1e4
(high SNR) and where every z is below the branch split (low SNR)."""
import importlib.util
import math
import os

import numpy as np
import pytest

import oracle as O

from gpu_helpers import assert_parity, masked_group, merged_grad, run_gpu, run_oracle, say, theta32, oracle_problem

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _gen():
    spec = importlib.util.spec_from_file_location(
        "gen_bessel_fit", os.path.join(HERE, "..", "paper_2604_00250_amd", "csrc", "gen_bessel_fit.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_device_special_functions_meet_the_bound():
    import torch
    from paper_2604_00250_amd import _lib as L
    gen = _gen()
    z = gen.test_grid()
    dev = torch.from_numpy(z).cuda()
    out = [torch.empty_like(dev) for _ in range(3)]
    L.check(L.lib().prism_rician_terms(dev.data_ptr(), out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
                                       z.size, None))
    torch.cuda.synchronize()
    vals = [o.cpu().numpy() for o in out]
    errs = gen.relative_errors(z, vals)
    emu = gen.evaluate_f32(z)
    ulps = [float(np.max(np.abs(a.astype(np.float64) - b) / np.spacing(np.abs(b).astype(np.float32)).astype(np.float64)))
            for a, b in zip(vals, emu)]
    say(f"[bessel] {z.size} arguments: max relative error log I0e {errs[0].max():.3e} (z={z[errs[0].argmax()]:.6g}), "
        f"1-R {errs[1].max():.3e} (z={z[errs[1].argmax()]:.6g}), q {errs[2].max():.3e}; "
        f"device vs host emulation within {ulps} ulp")
    for e in errs:
        assert e.max() <= 2e-7


def _z_range(g, th):
    prob = oracle_problem(g)
    yhat = O.synthesize(prob, theta32(th))
    s2 = math.exp(2.0 * float(th["sigma_log"]))
    z = np.abs(np.asarray(g.y, np.float64)) * np.abs(yhat) / s2
    return z


@pytest.mark.parametrize("K,acq", [(3, "three288"), (2, "two96")])
def test_nll_parity_at_high_snr(K, acq):
    g = masked_group((7, 6, 5), K=K, mode="nll", seed=91 + K, acq_kind=acq, snr=100.0)
    th = dict(g.theta)
    th["sigma_log"] = np.float32(math.log(0.01))
    z = _z_range(g, th)
    say(f"[nll high snr] K={K} N={g.acq.n} z in [{z.min():.3g}, {z.max():.3g}], "
        f"{(z >= 3.75).mean() * 100:.0f}% above the split")
    assert z.max() > 1e3
    r = run_gpu([g], [th])
    out, grad, _ = run_oracle(g, th)
    assert r["status"] == 0
    assert_parity(f"nll-high-snr K={K}", r["loss"][0], merged_grad(r["gmicro"][0], r["gcal"][0]), out, grad)


def test_nll_parity_with_every_z_below_the_split():
    g = masked_group((6, 6, 6), K=3, mode="nll", seed=97, acq_kind="three288", snr=3.0)
    th = dict(g.theta)
    th["sigma_log"] = np.float32(0.0)
    z = _z_range(g, th)
    # sigma such that the largest argument sits at 3.0
    th["sigma_log"] = np.float32(0.5 * math.log(z.max() / 3.0))
    z = _z_range(g, th)
    say(f"[nll low z] z in [{z.min():.3g}, {z.max():.3g}]")
    assert z.max() < 3.75
    r = run_gpu([g], [th])
    out, grad, _ = run_oracle(g, th)
    assert r["status"] == 0
    assert_parity("nll-low-z", r["loss"][0], merged_grad(r["gmicro"][0], r["gcal"][0]), out, grad)
