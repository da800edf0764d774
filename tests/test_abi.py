"""CPU tests of the C ABI: the library loads, exports every declared entry
point, and rejects bad arguments with the documented codes before touching
the GPU."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

from paper_2604_00250_amd import _lib as L
from paper_2604_00250_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "prism.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int32_t|void|const char\*)\s+(prism_\w+)\s*\(", src, flags=re.M)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
        assert n in L.SIGNATURES, f"binding misses {n}"
    assert lib.prism_abi_version() == 4


def test_model_defaults_are_the_papers_constants():
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_constants.json")))
    m = L.model_defaults()
    for k in ("d_csf", "d_gm", "d_res", "d_par", "d_perp", "huber_delta", "lam_sp", "lam_rep",
              "lam_sparse", "tau_sparse", "lam_orphan"):
        assert getattr(m, k) == pytest.approx(gold[k]["value"], rel=1e-7), k
    assert m.lam_cont == pytest.approx(gold["lam_continuity"]["value"], rel=1e-7)
    assert m.lam_order == pytest.approx(gold["lam_ordering"]["value"], rel=1e-7)


def test_model_defaults_equal_the_oracles_constants():
    """Every constant the library defaults to (printed or a reading) is the
    value the oracle uses."""
    import oracle as O
    m = L.model_defaults()
    c = O.Constants()
    for name, _ in L.Model._fields_:
        assert getattr(m, name) == pytest.approx(getattr(c, name), rel=1e-7), name


def test_loss_layout_matches_the_oracle_terms():
    import oracle as O
    assert L.LOSS_TERMS == O.TERMS
    assert L.LOSS_TERMS[L.LOSS_TOTAL] == "total"
    hdr = open(os.path.join(ROOT, "include", "prism.h")).read()
    assert f"#define PRISM_LOSS_TERMS {len(L.LOSS_TERMS)}" in hdr
    assert f"#define PRISM_LOSS_TOTAL {L.LOSS_TOTAL}" in hdr


def _acq(n=5, bad_norm=False, neg_b=False):
    bval = np.linspace(0, 2, n).astype(np.float32)
    bvec = I.uniform_sphere(n, np.random.default_rng(0)).astype(np.float32)
    if bad_norm:
        bvec[2] *= 1.1
    if neg_b:
        bval[1] = -1.0
    return bval, bvec


def _create(edit_group=None, edit_acq=None, n_groups=1, model=None):
    bval, bvec = _acq(**(edit_acq or {}))
    acq = L.Acq(bval.shape[0], bval.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                bvec.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    acqs = (L.Acq * 1)(acq)
    descs = (L.GroupDesc * max(n_groups, 1))()
    for i in range(max(n_groups, 1)):
        descs[i] = L.GroupDesc(4, 3, 2, 2, L.MSE, 0, 0, 6, 0, 15, None)
        if edit_group:
            for k, v in edit_group.items():
                setattr(descs[i], k, v)
    m = model if model is not None else L.model_defaults()
    h = ctypes.c_void_p()
    rc = L.lib().prism_problem_create(ctypes.byref(h), descs, n_groups, acqs, 1, ctypes.byref(m))
    if rc == 0:
        L.lib().prism_problem_destroy(h)
    return rc, L.lib().prism_last_error().decode()


@pytest.mark.parametrize("edit,needle", [
    ({"K": 0}, "K must be"), ({"K": 7}, "K must be"), ({"mode": 2}, "data mode"),
    ({"bias": 3}, "bias"), ({"acq": 1}, "acquisition index"), ({"neighbourhood": 4}, "neighbourhood"),
    ({"nx": 0}, "box"), ({"nz": 1024}, "box"), ({"learn_diffusivity": 2}, "learn_diffusivity"),
    ({"priors": 256}, "prior bits"),
])
def test_create_rejects_bad_group(edit, needle):
    rc, msg = _create(edit_group=edit)
    assert rc == L.PRISM_E_INVALID
    assert needle in msg


def test_create_rejects_bad_acquisition_and_counts():
    rc, msg = _create(edit_acq={"bad_norm": True})
    assert rc == L.PRISM_E_INVALID and "unit vector" in msg
    rc, msg = _create(edit_acq={"neg_b": True})
    assert rc == L.PRISM_E_INVALID and "negative" in msg
    rc, msg = _create(n_groups=0)
    assert rc == L.PRISM_E_INVALID and "at least one group" in msg
    m = L.model_defaults()
    m.lam_sp = float("nan")
    rc, msg = _create(model=m)
    assert rc == L.PRISM_E_INVALID and "finite" in msg
    m = L.model_defaults()
    m.s0_orphan = 0.0
    rc, msg = _create(model=m)
    assert rc == L.PRISM_E_INVALID and "s0_orphan" in msg
    m = L.model_defaults()
    m.d_par = 0.0
    rc, msg = _create(model=m)
    assert rc == L.PRISM_E_INVALID and "d_par" in msg
    lib = L.lib()
    assert lib.prism_problem_create(None, None, 0, None, 0, None) == L.PRISM_E_INVALID
    n = np.zeros(1025, dtype=np.float32)
    g = np.zeros((1025, 3), dtype=np.float32)
    acq = L.Acq(1025, n.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    descs = (L.GroupDesc * 1)(L.GroupDesc(2, 2, 2, 1, 0, 0, 0, 0, 0, 0, None))
    h = ctypes.c_void_p()
    m = L.model_defaults()
    assert lib.prism_problem_create(ctypes.byref(h), descs, 1, (L.Acq * 1)(acq), 1, ctypes.byref(m)) == L.PRISM_E_INVALID
    assert "n_meas" in lib.prism_last_error().decode()


def test_valid_create_without_gpu_reports_alloc_not_crash():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: creation succeeds there")
    rc, msg = _create()
    assert rc == L.PRISM_E_ALLOC


def test_null_handles_and_optimiser_arguments():
    lib = L.lib()
    assert lib.prism_problem_destroy(None) == L.PRISM_E_INVALID
    assert lib.prism_loss_grad(None, None, None, None, None, None, None, None, 0, None, None) == L.PRISM_E_INVALID
    assert lib.prism_synthesize(None, None, None, None, None) == L.PRISM_E_INVALID
    assert lib.prism_loss_grad_noalloc(None, None, None, None, None, None, None, None, None) == L.PRISM_E_INVALID
    n = ctypes.c_size_t()
    assert lib.prism_workspace_bytes(None, ctypes.byref(n)) == L.PRISM_E_INVALID
    assert lib.prism_adam_step(None, None, None, None, -1, 1e-2, 0.9, 0.999, 1e-8, None, None) == L.PRISM_E_INVALID
    assert lib.prism_adam_step(None, None, None, None, 10, 1e-2, 0.9, 0.999, 1e-8, None, None) == L.PRISM_E_INVALID
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the hyper-parameter check fails first
    assert lib.prism_adam_step(fake, fake, fake, fake, 10, 1e-2, 1.5, 0.999, 1e-8, fake, None) == L.PRISM_E_INVALID
    assert lib.prism_rprop_step(fake, fake, fake, fake, 10, 1.5, 1.2, 1e-6, 50.0, None) == L.PRISM_E_INVALID
    assert lib.prism_rprop_step(fake, fake, fake, fake, 10, 0.5, 0.9, 1e-6, 50.0, None) == L.PRISM_E_INVALID
    assert lib.prism_profile_enable(None, 1, 4) == L.PRISM_E_INVALID
    assert lib.prism_iteration_adam(None, None, None, None, None, None, None, None, None, 1e-2, 0.9, 0.999, 1e-8,
                                    1, None, None, 0, None, None, None, 0, None, None) == L.PRISM_E_INVALID
    assert lib.prism_stitch_plan(None, 4, 4, 4, None, None) == L.PRISM_E_INVALID
    assert lib.prism_stitch_maps(None, None, None, None) == L.PRISM_E_INVALID
    assert "NULL" in lib.prism_last_error().decode() or "handle" in lib.prism_last_error().decode()


def test_product_path_has_no_cpu_fallback(tmp_path, monkeypatch):
    """The binding raises when the HIP library is missing instead of computing anything."""
    import importlib
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(ImportError):
        L.lib()
    importlib.reload(L)
