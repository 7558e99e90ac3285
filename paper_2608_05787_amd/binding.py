"""ctypes binding of the C ABI in include/lbm_ehd.h (argument marshalling only).

Every step of the method runs in the HIP library ``liblbm_ehd.so``; PyTorch
only provides the device workspace, the output buffers and the stream.
Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm_ehd.so")

FIELDS = ["phi1", "phi2", "phi3", "rho", "ux", "uy", "p", "psi", "Ex", "Ey",
          "q", "mu1", "mu2", "mu3", "eps", "R", "uz", "Ez",  # uz, Ez: D3Q15 only
          "n_plus", "n_minus"]  # Nernst-Planck charge model only
PRECISION = {"fp32": 0, "fp16s": 1, "fp64": 2, "tangent": 3}
FAMILY = {"f": (0, 3), "g": (1, 1), "l": (2, 1), "h": (3, 1)}  # id, planes per lattice velocity
DIAG_KEYS = ["mass1", "mass2", "mass3", "charge", "max_sum_dev", "residual", "k_sub",
             "nonfinite", "D_outer", "D_inner", "D_outer_moment", "D_inner_moment",
             "r_par_outer", "r_perp_outer", "r_par_inner", "r_perp_inner"]
EDIVERGED, ENOCONV = -4, -5


class LbmEhdError(RuntimeError):
    pass


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("wall_q_mode", ctypes.c_int32), ("eps_ref_phase", ctypes.c_int32),
        ("phase_mode", ctypes.c_int32), ("sub_min", ctypes.c_int32), ("sub_max", ctypes.c_int32),
        ("init_sub_max", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("lattice", ctypes.c_int32),
        ("sub_tol", ctypes.c_double), ("init_tol", ctypes.c_double),
        ("wall_u", ctypes.c_double * 2), ("wall_phi", ctypes.c_double * 2),
        ("wall_q", ctypes.c_double * 2), ("E_ext", ctypes.c_double * 2),
        ("gamma12", ctypes.c_double), ("gamma13", ctypes.c_double),
        ("gamma23", ctypes.c_double), ("width", ctypes.c_double),
        ("rho", ctypes.c_double * 3), ("visc", ctypes.c_double * 3),
        ("eps", ctypes.c_double * 3), ("sigma", ctypes.c_double * 3),
        ("tau_f", ctypes.c_double), ("tau_l", ctypes.c_double),
        ("dtheta", ctypes.c_double * 5),
        ("E_ext_z", ctypes.c_double),
        ("charge_model", ctypes.c_int32), ("sum_relax", ctypes.c_int32),
        ("ion_tau", ctypes.c_double), ("ion_beta", ctypes.c_double), ("ion_charge", ctypes.c_double),
    ]


_dp = ctypes.POINTER(ctypes.c_double)


class Init(ctypes.Structure):
    _fields_ = [("phi0", _dp), ("u0", _dp), ("q0", _dp), ("psi0", _dp), ("ions0", _dp)]


EXPORTS = ["lbm_ehd_adjoint_workspace_bytes", "lbm_ehd_workspace_bytes", "lbm_ehd_create", "lbm_ehd_step", "lbm_ehd_fields",
           "lbm_ehd_populations", "lbm_ehd_diagnostics", "lbm_ehd_diagnostics_static", "lbm_ehd_status",
           "lbm_ehd_scalars",
           "lbm_ehd_checkpoint_bytes", "lbm_ehd_checkpoint", "lbm_ehd_restore",
           "lbm_ehd_adjoint", "lbm_ehd_record", "lbm_ehd_tangent_workspace_bytes", "lbm_ehd_tangent_gradient",
           "lbm_ehd_profile_begin", "lbm_ehd_profile_end", "lbm_ehd_graph", "lbm_ehd_step_persistent",
           "lbm_ehd_set_persistent_polls", "lbm_ehd_set_persistent_timing", "lbm_ehd_persistent_stage_times",
           "lbm_ehd_set_tuning", "lbm_ehd_get_tuning", "lbm_ehd_tune",
           "lbm_ehd_destroy", "lbm_ehd_strerror", "lbm_ehd_last_error"]
TUNE_LINEAR_ORDER, TUNE_SINGLE_POTENTIAL, TUNE_COLLIDE_PER_FAMILY, TUNE_TALL_TILES = 1, 2, 4, 8
KERNELS = ["moments", "pre", "poisson", "mu", "collide", "diag", "poisson2", "poisson2_pre"]

_lib = None


def load():
    """Load liblbm_ehd.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LbmEhdError("HIP library %s is not built; run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.lbm_ehd_workspace_bytes.argtypes = [ctypes.POINTER(Params), ctypes.c_int32, ctypes.POINTER(sz)]
    lib.lbm_ehd_create.argtypes = [ctypes.POINTER(Params), ctypes.c_int32, ctypes.POINTER(Init), vp, vp,
                                   ctypes.POINTER(vp)]
    lib.lbm_ehd_step.argtypes = [vp, ctypes.c_int64]
    lib.lbm_ehd_fields.argtypes = [vp, ctypes.c_int32, ctypes.c_uint32, vp, ctypes.c_int32]
    lib.lbm_ehd_populations.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int32]
    lib.lbm_ehd_diagnostics.argtypes = [vp, ctypes.c_int32, _dp]
    lib.lbm_ehd_status.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.lbm_ehd_diagnostics_static.argtypes = [vp, ctypes.c_int32, _dp]
    lib.lbm_ehd_scalars.argtypes = [vp, _dp]
    lib.lbm_ehd_checkpoint_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    lib.lbm_ehd_checkpoint.argtypes = [vp, vp]
    lib.lbm_ehd_restore.argtypes = [vp, vp]
    lib.lbm_ehd_adjoint.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, vp, ctypes.c_uint32, vp, sz, _dp]
    lib.lbm_ehd_adjoint_workspace_bytes.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(sz)]
    lib.lbm_ehd_record.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, vp, sz]
    lib.lbm_ehd_tangent_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    lib.lbm_ehd_tangent_gradient.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_uint32, vp, sz, _dp]
    lib.lbm_ehd_profile_begin.argtypes = [vp]
    lib.lbm_ehd_profile_end.argtypes = [vp, _dp, ctypes.POINTER(ctypes.c_int64)]
    lib.lbm_ehd_graph.argtypes = [vp, ctypes.c_int32]
    lib.lbm_ehd_step_persistent.argtypes = [vp, ctypes.c_int64]
    lib.lbm_ehd_set_persistent_polls.argtypes = [vp, ctypes.c_int32]
    lib.lbm_ehd_persistent_stage_times.argtypes = [vp, _dp]
    lib.lbm_ehd_set_persistent_timing.argtypes = [vp, ctypes.c_int32]
    lib.lbm_ehd_set_tuning.argtypes = [vp, ctypes.c_int32]
    lib.lbm_ehd_get_tuning.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.lbm_ehd_tune.argtypes = [vp, ctypes.c_int32, vp, _dp, ctypes.POINTER(ctypes.c_int32)]
    lib.lbm_ehd_destroy.argtypes = [vp]
    lib.lbm_ehd_destroy.restype = None
    lib.lbm_ehd_strerror.argtypes = [ctypes.c_int]
    lib.lbm_ehd_strerror.restype = ctypes.c_char_p
    lib.lbm_ehd_last_error.argtypes = [vp]
    lib.lbm_ehd_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def make_params(cfg: dict, precision: str = "fp32") -> Params:
    p = Params()
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    p.bc_y = int(cfg.get("bc_y", 0))
    p.wall_q_mode = int(cfg.get("wall_q_mode", 0))
    p.eps_ref_phase = int(cfg.get("eps_ref_phase", 0))
    p.phase_mode = int(cfg.get("phase_mode", 0))
    p.sub_min = int(cfg.get("sub_min", 1))
    p.sub_max = int(cfg.get("sub_max", 1))
    p.init_sub_max = int(cfg.get("init_sub_max", 0))
    p.precision = PRECISION[precision]
    p.sub_tol = float(cfg.get("sub_tol", 0.0))
    p.init_tol = float(cfg.get("init_tol", 0.0))
    for k in ("wall_u", "wall_phi", "wall_q", "E_ext"):
        v = cfg.get(k, (0.0, 0.0))
        getattr(p, k)[0], getattr(p, k)[1] = float(v[0]), float(v[1])
    p.gamma12, p.gamma13, p.gamma23 = (float(cfg[k]) for k in ("gamma12", "gamma13", "gamma23"))
    p.width = float(cfg["width"])
    for k in ("rho", "visc", "eps", "sigma"):
        for i in range(3):
            getattr(p, k)[i] = float(cfg[k][i])
    p.tau_f, p.tau_l = float(cfg["tau_f"]), float(cfg["tau_l"])
    for i, v in enumerate(cfg.get("dtheta", (0.0,) * 5)):
        p.dtheta[i] = float(v)
    p.nz = int(cfg.get("nz", 1))
    p.lattice = int(cfg.get("lattice", 0))
    p.E_ext_z = float(cfg.get("E_ext_z", 0.0))
    p.charge_model = int(cfg.get("charge_model", 0))
    p.sum_relax = int(cfg.get("sum_relax", 0))
    p.ion_tau = float(cfg.get("ion_tau", 0.8))
    p.ion_beta = float(cfg.get("ion_beta", 0.0))
    p.ion_charge = float(cfg.get("ion_charge", 0.0))
    return p


def grid_shape(cfg: dict):
    """Shape of a field: [ny, nx] on D2Q9, [nz, ny, nx] on D3Q15."""
    if int(cfg.get("lattice", 0)) == 1:
        return (int(cfg.get("nz", 1)), int(cfg["ny"]), int(cfg["nx"]))
    return (int(cfg["ny"]), int(cfg["nx"]))


class Sim:
    """A handle over one or more instances (a batch when several are given).

    cfgs: parameter dict or list of dicts; inits: dict or list of dicts of
    float64 host arrays on the lattice's grid G ([ny, nx] for D2Q9,
    [nz, ny, nx] for D3Q15): phi0 [3, *G], optional u0 [D, *G], q0, psi0 G;
    under the Nernst-Planck charge model ions0 [2, *G] (n_+, n_-).
    """

    def __init__(self, cfgs, inits, precision: str = "fp32", device="cuda", stream=None):
        import torch
        lib = load()
        if isinstance(cfgs, dict):
            cfgs, inits = [cfgs], [inits]
        self.n_inst = len(cfgs)
        self.shapes = [grid_shape(c) for c in cfgs]
        self.q = 15 if int(cfgs[0].get("lattice", 0)) == 1 else 9
        self.ions = int(cfgs[0].get("charge_model", 0)) == 1
        self.precision = precision
        self.device = torch.device(device)
        n = self.n_inst
        self._params = (Params * n)(*[make_params(c, precision) for c in cfgs])
        nbytes = ctypes.c_size_t()
        rc = lib.lbm_ehd_workspace_bytes(self._params, n, ctypes.byref(nbytes))
        self._check(rc, None)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self._keep = []
        init_arr = (Init * n)()
        for i, ini in enumerate(inits):
            for k in ("phi0", "u0", "q0", "psi0", "ions0"):
                v = ini.get(k)
                if v is not None:
                    v = np.ascontiguousarray(v, dtype=np.float64)
                    self._keep.append(v)
                    setattr(init_arr[i], k, v.ctypes.data_as(_dp))
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = lib.lbm_ehd_create(self._params, n, init_arr, ctypes.c_void_p(self.workspace.data_ptr()),
                                    ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        self._check(rc, None)
        self._h = h
        self._keep = []

    # -- helpers
    def _handoff(self, out):
        """Outputs are written on the handle's stream: make the caller's
        current stream wait for it and keep the allocation alive there."""
        import torch
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            out.record_stream(self.stream)
            cur.wait_stream(self.stream)
        return out

    def _check(self, rc, h):
        if rc != 0:
            lib = load()
            msg = lib.lbm_ehd_last_error(h if h is not None else None)
            raise LbmEhdError("%s: %s" % (lib.lbm_ehd_strerror(rc).decode(), (msg or b"").decode()))

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.lbm_ehd_destroy(h)
            self._h = None

    __del__ = close

    # -- API
    def step(self, n: int = 1):
        self._check(load().lbm_ehd_step(self._h, int(n)), self._h)

    def step_persistent(self, n: int = 1):
        """n steps in grid-resident launches (lbm_ehd_step_persistent);
        synchronises."""
        self._check(load().lbm_ehd_step_persistent(self._h, int(n)), self._h)

    def set_persistent_polls(self, polls: int):
        self._check(load().lbm_ehd_set_persistent_polls(self._h, int(polls)), self._h)

    def set_persistent_timing(self, on: bool):
        self._check(load().lbm_ehd_set_persistent_timing(self._h, 1 if on else 0), self._h)

    def persistent_stage_times(self) -> dict:
        """Microseconds per step of each stage of the last timed
        step_persistent call (barrier included)."""
        us = (ctypes.c_double * 4)()
        self._check(load().lbm_ehd_persistent_stage_times(self._h, us), self._h)
        return dict(zip(("moments", "potential", "mu", "collide"), list(us)))

    def fields(self, names=None, inst: int = 0, dtype=None, tangent: bool = False):
        """Fields of the last step as [ny, nx] tensors; tangent=True gives the
        derivative parts of a tangent-mode handle (float64)."""
        import torch
        names = list(names or (FIELDS if self.q == 15 else FIELDS[:16]))
        mask = 0
        for k in names:
            mask |= 1 << FIELDS.index(k)
        order = [k for k in FIELDS if mask & (1 << FIELDS.index(k))]
        dtype = torch.float64 if tangent else (dtype or torch.float64)
        out = torch.empty((len(order),) + self.shapes[inst], dtype=dtype, device=self.device)
        dt = 2 if tangent else (1 if dtype == torch.float64 else 0)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(load().lbm_ehd_fields(self._h, inst, mask, ctypes.c_void_p(out.data_ptr()), dt), self._h)
        self._handoff(out)
        return {k: out[i] for i, k in enumerate(order)}

    def populations(self, fam: str, inst: int = 0, dtype=None):
        import torch
        idx, mult = FAMILY[fam]
        if fam == "l" and self.ions:
            mult = 2
        dtype = dtype or torch.float64
        out = torch.empty((mult * self.q,) + self.shapes[inst], dtype=dtype, device=self.device)
        dt = 1 if dtype == torch.float64 else 0
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(load().lbm_ehd_populations(self._h, inst, idx, ctypes.c_void_p(out.data_ptr()), dt), self._h)
        return self._handoff(out)

    def diagnostics(self, inst: int = 0, static: bool = False) -> dict:
        """The 16 outputs of lbm_ehd_diagnostics by name, plus "status": its
        return code (0, EDIVERGED or the warning ENOCONV; other codes
        raise).  static=True calls lbm_ehd_diagnostics_static (the partial
        sums in the library's static device buffer)."""
        out = (ctypes.c_double * 16)()
        fn = load().lbm_ehd_diagnostics_static if static else load().lbm_ehd_diagnostics
        rc = fn(self._h, inst, out)
        d = dict(zip(DIAG_KEYS, list(out)))
        if rc not in (0, EDIVERGED, ENOCONV):
            self._check(rc, self._h)
        d["status"] = rc
        return d

    def status(self):
        """(return code, flags) of lbm_ehd_status: the latched conditions of
        every instance (bit 1 non-finite, bit 2 potential cap reached)."""
        flags = ctypes.c_int32()
        rc = load().lbm_ehd_status(self._h, ctypes.byref(flags))
        if rc not in (0, EDIVERGED, ENOCONV):
            self._check(rc, self._h)
        return rc, int(flags.value)

    def scalars(self) -> dict:
        out = (ctypes.c_double * 3)()
        self._check(load().lbm_ehd_scalars(self._h, out), self._h)
        return {"steps": int(out[0]), "k_total": int(out[1]), "n_inst": int(out[2])}

    def _seed_planes(self, seed: dict):
        import torch
        mask = 0
        for k in seed:
            mask |= 1 << FIELDS.index(k)
        order = [k for k in FIELDS if mask & (1 << FIELDS.index(k))]
        planes = torch.stack([seed[k].to(self.device, torch.float64) for k in order]).contiguous()
        return mask, planes

    def _adjoint_work(self, n_steps: int, ckpt_every: int):
        import torch
        nb = ctypes.c_size_t()
        self._check(load().lbm_ehd_adjoint_workspace_bytes(self._h, int(n_steps), int(ckpt_every), ctypes.byref(nb)),
                    self._h)
        work = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        base = (work.data_ptr() + 255) // 256 * 256
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        work.record_stream(self.stream)
        return work, base, int(nb.value)

    def record(self, n_steps: int, ckpt_every: int = 250):
        """Step n_steps from the creation state (the same states as step())
        while checkpointing every ckpt_every steps for adjoint()."""
        work, base, nb = self._adjoint_work(n_steps, ckpt_every)
        self._check(load().lbm_ehd_record(self._h, int(n_steps), int(ckpt_every), ctypes.c_void_p(base), nb),
                    self._h)
        self._rec = (work, base, nb, int(n_steps), int(ckpt_every))

    def adjoint(self, n_steps: int, seed: dict, ckpt_every: int = 250):
        """dJ/dtheta by the reverse (adjoint) sweep, for J = sum over the seed's
        fields (phi1..phi3) of seed * field after n_steps from this handle's
        creation state; theta = (eps2/eps1, eps3/eps1, sigma2/sigma1,
        sigma3/sigma1, E0).  seed: {field name: [ny, nx] tensor}.  Uses the
        checkpoints of record() when it ran with the same n_steps and
        ckpt_every, else records its own run first."""
        mask, planes = self._seed_planes(seed)
        rec = getattr(self, "_rec", None)
        if rec is not None and rec[3] == int(n_steps) and rec[4] == int(ckpt_every):
            work, base, nb = rec[0], rec[1], rec[2]
        else:
            work, base, nb = self._adjoint_work(n_steps, ckpt_every)
        grad = (ctypes.c_double * 5)()
        self._check(load().lbm_ehd_adjoint(self._h, int(n_steps), int(ckpt_every), ctypes.c_void_p(planes.data_ptr()),
                                           mask, ctypes.c_void_p(base), nb, grad), self._h)
        return list(grad)

    def tangent_gradient(self, n_steps: int, seed: dict):
        """The same gradient as adjoint() by forward mode: five FP64 tangent
        runs inside the library; any fields may be seeded."""
        import torch
        lib = load()
        mask, planes = self._seed_planes(seed)
        nb = ctypes.c_size_t()
        self._check(lib.lbm_ehd_tangent_workspace_bytes(self._h, ctypes.byref(nb)), self._h)
        work = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        base = (work.data_ptr() + 255) // 256 * 256
        grad = (ctypes.c_double * 5)()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(lib.lbm_ehd_tangent_gradient(self._h, int(n_steps), ctypes.c_void_p(planes.data_ptr()), mask,
                                                 ctypes.c_void_p(base), int(nb.value), grad), self._h)
        return list(grad)

    def graph(self, steps_per_graph: int):
        """Capture a block of steps into a HIP graph replayed by step()."""
        self._check(load().lbm_ehd_graph(self._h, int(steps_per_graph)), self._h)

    # -- launch configuration (results are bitwise the same in every one)
    def set_tuning(self, config: int):
        self._check(load().lbm_ehd_set_tuning(self._h, int(config)), self._h)

    def get_tuning(self) -> int:
        c = ctypes.c_int32()
        self._check(load().lbm_ehd_get_tuning(self._h, ctypes.byref(c)), self._h)
        return int(c.value)

    def tuning_key(self) -> str:
        """What the timing of a configuration depends on: lattice, precision,
        sub-iteration settings, charge model and the instance sizes."""
        import json
        p = self._params
        return json.dumps({"lattice": int(p[0].lattice), "precision": self.precision,
                           "sub": [int(p[0].sub_min), int(p[0].sub_max), float(p[0].sub_tol)],
                           "charge_model": int(p[0].charge_model),
                           "sizes": [list(s) for s in self.shapes]}, sort_keys=True)

    def autotune(self, steps: int = 20, cache: str = None) -> dict:
        """Pick the fastest launch configuration for this handle.  With a
        cache file (JSON), a configuration stored under this handle's
        tuning_key() is applied without timing; otherwise lbm_ehd_tune times
        the configurations on the handle's own state (which it restores) and
        the choice is stored.  Returns {"config", "ms_per_step", "cached"}."""
        import json
        import torch
        key = self.tuning_key()
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                self.set_tuning(int(table[key]["config"]))
                return dict(table[key], cached=True)
        nb = ctypes.c_size_t()
        self._check(load().lbm_ehd_checkpoint_bytes(self._h, ctypes.byref(nb)), self._h)
        scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        ms = (ctypes.c_double * 16)()
        best = ctypes.c_int32()
        self._check(load().lbm_ehd_tune(self._h, int(steps), ctypes.c_void_p(scratch.data_ptr()), ms,
                                        ctypes.byref(best)), self._h)
        entry = {"config": int(best.value), "ms_per_step": [float(v) for v in ms]}
        if cache:
            table[key] = entry
            tmp = cache + ".tmp%d" % os.getpid()
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return dict(entry, cached=False)

    def profile_begin(self):
        self._check(load().lbm_ehd_profile_begin(self._h), self._h)

    def profile_end(self) -> dict:
        ms = (ctypes.c_double * 16)()
        cnt = (ctypes.c_int64 * 8)()
        self._check(load().lbm_ehd_profile_end(self._h, ms, cnt), self._h)
        return {k: (ms[i], int(cnt[i])) for i, k in enumerate(KERNELS)}

    def checkpoint(self):
        import torch
        nb = ctypes.c_size_t()
        self._check(load().lbm_ehd_checkpoint_bytes(self._h, ctypes.byref(nb)), self._h)
        buf = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(load().lbm_ehd_checkpoint(self._h, ctypes.c_void_p(buf.data_ptr())), self._h)
        return self._handoff(buf)

    def restore(self, buf):
        import torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(load().lbm_ehd_restore(self._h, ctypes.c_void_p(buf.data_ptr())), self._h)
