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
    assert lib.lbm_ehd_strerror(-7) == b"not supported by this library"
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


def test_two_drop_workload_geometry():
    """The two-drop inputs (Sec. 4.5): phases sum to one, two shells and two
    cores mirror-symmetric about the box centre along the field, the shells
    the stated gap apart, and the regime's ratios in this code's numbering."""
    import numpy as np
    from scipy import ndimage
    from paper_2608_05787_amd import inputs
    p, init = inputs.two_compound_drops(nx=96, ny=160, r_shell=20.0, r_core=12.0, gap=8.0, regime="coalescence")
    phi = init["phi0"]
    np.testing.assert_allclose(phi.sum(0), 1.0, atol=1e-14)
    assert phi.min() >= 0.0
    np.testing.assert_allclose(phi, phi[:, ::-1, :], atol=1e-12)
    assert ndimage.label(phi[0] < 0.5)[1] == 2 and ndimage.label(phi[2] > 0.5)[1] == 2
    col = phi[0][:, 47]
    inside = np.nonzero(col < 0.5)[0]
    gap = np.nonzero(np.diff(inside) > 1)[0]
    assert len(gap) == 1 and inside[gap[0] + 1] - inside[gap[0]] - 1 == 8
    assert p["eps"][1] / p["eps"][0] == 8.0 and p["sigma"][1] / p["sigma"][0] == 6.0
    q, _ = inputs.two_compound_drops(regime="separation")
    assert abs(q["eps"][1] / q["eps"][0] - 0.2) < 1e-12 and abs(q["sigma"][1] / q["sigma"][0] - 1.04) < 1e-12
    assert p["bc_y"] == 1 and p["wall_phi"][1] > 0


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of lbm_ehd_params and lbm_ehd_init have the C
    header's size and field offsets (compiled with the host compiler)."""
    import ctypes
    import subprocess
    from paper_2608_05787_amd import binding
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    fields = [f[0] for f in binding.Params._fields_ if not f[0].startswith("reserved")]
    src = tmp_path / "probe.c"
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "lbm_ehd.h"', "int main(void) {",
             '  printf("params %zu\\n", sizeof(lbm_ehd_params));',
             '  printf("init %zu\\n", sizeof(lbm_ehd_init));']
    lines += ['  printf("%s %%zu\\n", offsetof(lbm_ehd_params, %s));' % (f, f) for f in fields]
    lines += ['  printf("ions0 %zu\\n", offsetof(lbm_ehd_init, ions0));', "  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(root, "include"), "-o", str(exe), str(src)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    assert int(got["params"]) == ctypes.sizeof(binding.Params)
    assert int(got["init"]) == ctypes.sizeof(binding.Init)
    for f in fields:
        assert int(got[f]) == getattr(binding.Params, f).offset, f
    assert int(got["ions0"]) == binding.Init.ions0.offset
