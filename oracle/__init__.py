"""FP64 CPU oracle of the three-phase EHD lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: the slow, plain reference the GPU path is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import it.  It shares no code with the HIP library and
never reads anything the HIP path produced.

The arithmetic lives in ``lbm_ehd_oracle.c`` (plain C, double precision); this
module only compiles it with gcc and marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_ehd_oracle.c")
_LIB = os.path.join(_HERE, "_lbm_ehd_oracle.so")

FIELDS = ["phi1", "phi2", "phi3", "rho", "ux", "uy", "p", "psi", "Ex", "Ey",
          "q", "mu1", "mu2", "mu3", "eps", "R", "uz", "Ez", "n_plus", "n_minus"]
FAMILIES = {"f": (0, 3), "g": (1, 1), "l": (2, 1), "h": (3, 1)}  # id, planes per lattice direction


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=c99", "-Wall", "-shared",
                               "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("wall_q_mode", ctypes.c_int32), ("eps_ref_phase", ctypes.c_int32),
        ("phase_mode", ctypes.c_int32), ("sub_min", ctypes.c_int32),
        ("sub_max", ctypes.c_int32), ("init_sub_max", ctypes.c_int32),
        ("pad0", ctypes.c_int32),
        ("sub_tol", ctypes.c_double), ("init_tol", ctypes.c_double),
        ("wall_u", ctypes.c_double * 2), ("wall_phi", ctypes.c_double * 2),
        ("wall_q", ctypes.c_double * 2), ("E_ext", ctypes.c_double * 2),
        ("gamma12", ctypes.c_double), ("gamma13", ctypes.c_double),
        ("gamma23", ctypes.c_double), ("width", ctypes.c_double),
        ("rho", ctypes.c_double * 3), ("visc", ctypes.c_double * 3),
        ("eps", ctypes.c_double * 3), ("sigma", ctypes.c_double * 3),
        ("tau_f", ctypes.c_double), ("tau_l", ctypes.c_double),
        ("nz", ctypes.c_int32), ("lattice", ctypes.c_int32), ("E_ext_z", ctypes.c_double),
        ("charge_model", ctypes.c_int32), ("sum_relax", ctypes.c_int32),
        ("ion_tau", ctypes.c_double), ("ion_beta", ctypes.c_double), ("ion_charge", ctypes.c_double),
    ]


_libs = {}


def compile_variant(src_text: str, out_path: str) -> str:
    """Compile a variant of the oracle source (used only by the tests that
    check a pin rejects a planted mistake) into out_path."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=c99", "-w", "-shared", "-fPIC",
                           "-o", out_path, src, "-lm"])
    return out_path


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def _load(path=None):
    key = path or _LIB
    if key not in _libs:
        lib = ctypes.CDLL(path or build())
        dp = ctypes.POINTER(ctypes.c_double)
        lib.or_create.restype = ctypes.c_void_p
        lib.or_create.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp, dp]
        lib.or_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        lib.or_free.argtypes = [ctypes.c_void_p]
        lib.or_field.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
        lib.or_pops.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
        lib.or_scalars.argtypes = [ctypes.c_void_p, dp]
        lib.or_stencil.argtypes = [ctypes.POINTER(_Params), dp, dp, dp]
        lib.or_sizeof_params.restype = ctypes.c_int
        assert lib.or_sizeof_params() == ctypes.sizeof(_Params)
        _libs[key] = lib
    return _libs[key]


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _params(cfg: dict) -> _Params:
    p = _Params()
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    p.bc_y = int(cfg.get("bc_y", 0))
    p.wall_q_mode = int(cfg.get("wall_q_mode", 0))
    p.eps_ref_phase = int(cfg.get("eps_ref_phase", 0))
    p.phase_mode = int(cfg.get("phase_mode", 0))
    p.sub_min = int(cfg.get("sub_min", 1))
    p.sub_max = int(cfg.get("sub_max", 1))
    p.init_sub_max = int(cfg.get("init_sub_max", 0))
    p.sub_tol = float(cfg.get("sub_tol", 0.0))
    p.init_tol = float(cfg.get("init_tol", 0.0))
    for k in ("wall_u", "wall_phi", "wall_q", "E_ext"):
        v = cfg.get(k, (0.0, 0.0))
        getattr(p, k)[0], getattr(p, k)[1] = float(v[0]), float(v[1])
    p.gamma12, p.gamma13, p.gamma23 = (float(cfg[k]) for k in ("gamma12", "gamma13", "gamma23"))
    p.width = float(cfg["width"])
    for k in ("rho", "visc", "eps", "sigma"):
        arr = getattr(p, k)
        for i in range(3):
            arr[i] = float(cfg[k][i])
    p.tau_f, p.tau_l = float(cfg["tau_f"]), float(cfg["tau_l"])
    p.nz = int(cfg.get("nz", 1))
    p.lattice = int(cfg.get("lattice", 0))
    p.E_ext_z = float(cfg.get("E_ext_z", 0.0))
    p.charge_model = int(cfg.get("charge_model", 0))
    p.sum_relax = int(cfg.get("sum_relax", 0))
    p.ion_tau = float(cfg.get("ion_tau", 0.8))
    p.ion_beta = float(cfg.get("ion_beta", 0.0))
    p.ion_charge = float(cfg.get("ion_charge", 0.0))
    return p


def _geometry(cfg: dict):
    """(plane shape, spatial dimension, velocities): D2Q9 planes are
    [ny, nx]; D3Q15 boxes [nz, ny, nx]."""
    nx, ny = int(cfg["nx"]), int(cfg["ny"])
    if int(cfg.get("lattice", 0)) == 1:
        return (int(cfg.get("nz", 1)), ny, nx), 3, 15
    return (ny, nx), 2, 9


class Oracle:
    """One simulation instance of the FP64 oracle.

    ``cfg`` is a plain dict of physical/lattice parameters (see
    ``paper_2608_05787_amd.inputs``); ``init`` holds the initial fields as
    float64 arrays on the lattice's grid G ([ny, nx] for D2Q9, [nz, ny, nx]
    for D3Q15): ``phi0`` [3, *G], optional ``u0`` [D, *G], ``q0`` and
    ``psi0`` G; under the Nernst-Planck charge model ``ions0`` [2, *G]
    (n_+, n_-).
    """

    def __init__(self, cfg: dict, init: dict, lib_path=None):
        lib = self._lib = _load(lib_path)
        self.nx, self.ny = int(cfg["nx"]), int(cfg["ny"])
        self._p = _params(cfg)
        shp, self.dim, self.q = _geometry(cfg)
        self.shape = shp

        def arr(name, lead):
            v = init.get(name)
            if v is None:
                return None
            v = np.ascontiguousarray(v, dtype=np.float64)
            assert v.shape == ((lead,) + shp if lead else shp), (name, v.shape)
            return v

        self.nl = 2 if int(cfg.get("charge_model", 0)) == 1 else 1
        self._keep = [arr("phi0", 3), arr("u0", self.dim), arr("q0", 0), arr("psi0", 0), arr("ions0", 2)]
        h = lib.or_create(ctypes.byref(self._p), *[_ptr(a) for a in self._keep])
        if not h:
            raise ValueError("oracle rejected the parameters")
        self._h = ctypes.c_void_p(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and getattr(self, "_lib", None) is not None:
            self._lib.or_free(h)
            self._h = None

    def step(self, n: int = 1):
        self._lib.or_step(self._h, int(n))

    def field(self, name: str) -> np.ndarray:
        out = np.empty(self.shape, np.float64)
        rc = self._lib.or_field(self._h, FIELDS.index(name), _ptr(out))
        assert rc == 0
        return out

    def fields(self, names=None) -> dict:
        return {k: self.field(k) for k in (names or FIELDS[:16])}

    def pops(self, fam: str) -> np.ndarray:
        idx, mult = FAMILIES[fam]
        if fam == "l":
            mult = self.nl
        out = np.empty((mult * self.q,) + self.shape, np.float64)
        assert self._lib.or_pops(self._h, idx, _ptr(out)) == 0
        return out

    def scalars(self) -> dict:
        out = np.zeros(9, np.float64)
        self._lib.or_scalars(self._h, _ptr(out))
        return {"steps": int(out[0]), "k_used": int(out[1]), "residual": out[2],
                "lambda": tuple(out[3:6]), "m0": out[6], "alpha": out[7], "tau_h": out[8]}


def stencil(cfg: dict, chi: np.ndarray):
    """Eq. (33) gradient components and Laplacian of a plain field (unit
    checks): (gx, gy, lap) on D2Q9, (gx, gy, gz, lap) on D3Q15."""
    p = _params(cfg)
    _, dim, _ = _geometry(cfg)
    chi = np.ascontiguousarray(chi, np.float64)
    g = np.empty((dim,) + chi.shape, np.float64)
    lap = np.empty_like(chi)
    _load().or_stencil(ctypes.byref(p), _ptr(chi), _ptr(g), _ptr(lap))
    return tuple(g) + (lap,)
