"""Host-side checks of the C-ABI library (no GPU needed, no compute calls)."""
import ctypes
import os
import re

import pytest

from paper_2608_05787_amd import binding, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "lbm_ehd.h")).read()
    return sorted(set(re.findall(r"\b(lbm_ehd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = declared_symbols()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(binding.EXPORTS)


def _bytes(cfg, n=1, precision="fp32"):
    lib = binding.load()
    arr = (binding.Params * n)(*[binding.make_params(cfg, precision) for _ in range(n)])
    nb = ctypes.c_size_t(0)
    rc = lib.lbm_ehd_workspace_bytes(arr, n, ctypes.byref(nb))
    return rc, nb.value, lib.lbm_ehd_last_error(None).decode()


def test_workspace_size_scales_with_nodes_and_precision():
    p, _ = inputs.parity_case(64, 32)
    rc, b32, _ = _bytes(p)
    assert rc == 0
    rc, b64, _ = _bytes(p, precision="fp64")
    assert rc == 0 and 1.9 < b64 / b32 < 2.1
    # 45 populations x 2 buffers + 9 potential x 2 + 25 planes, 4 bytes each
    assert b32 >= 64 * 32 * 4 * (90 + 18 + 25)
    rc, b3, _ = _bytes(p, n=3)
    assert rc == 0 and b3 > 2.9 * b32


@pytest.mark.parametrize("key,val,msg", [
    ("gamma23", 1.0, "lambda"), ("tau_f", 0.5, "tau"), ("tau_l", 0.4, "tau"),
    ("nx", 1, "nx"), ("width", 0.0, "width"), ("sub_max", 0, "sub_min"),
    ("eps_ref_phase", 3, "eps_ref_phase"), ("bc_y", 2, "bc_y"),
])
def test_invalid_parameters_are_rejected(key, val, msg):
    p, _ = inputs.parity_case(16, 16)
    p[key] = val
    rc, _, err = _bytes(p)
    assert rc == -1 and msg in err


def test_negative_density_rejected_and_messages():
    p, _ = inputs.parity_case(16, 16)
    p["rho"] = (1.0, -1.0, 1.0)
    rc, _, err = _bytes(p)
    assert rc == -1 and "densit" in err
    lib = binding.load()
    assert lib.lbm_ehd_strerror(-7) == b"not supported by this build"
    assert lib.lbm_ehd_strerror(0) == b"ok"


def test_batch_settings_must_match():
    lib = binding.load()
    p, _ = inputs.parity_case(16, 16)
    q = dict(p, sub_max=3)
    arr = (binding.Params * 2)(binding.make_params(p), binding.make_params(q))
    nb = ctypes.c_size_t(0)
    assert lib.lbm_ehd_workspace_bytes(arr, 2, ctypes.byref(nb)) == -1


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(binding.LbmEhdError):
        binding.load()
