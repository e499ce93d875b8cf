"""ctypes wrapper of the plain FP64 CPU oracle (``vlb_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU
baseline leg of ``bench.py`` may import this module.  It imports nothing from
the product package; inputs come as plain dicts (``workloads`` builds them).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vlb_oracle.c")
LIB = os.path.join(HERE, "liboracle_vlb.so")
# The same source built with fused multiply-adds: a second FP64
# implementation that differs from the first only in rounding.  The gap
# between the two measures how closely FP64 can reproduce a result at all.
LIB_FMA = os.path.join(HERE, "liboracle_vlb_fma.so")
# The three-dimensional oracle (vlb3_oracle.c; it uses the disk-cell area of
# vlb_oracle.c for the sections of a sphere).
SRC3 = os.path.join(HERE, "vlb3_oracle.c")
LIB3 = os.path.join(HERE, "liboracle_vlb3.so")

FACE_FLOW = {"periodic": 0, "wall": 1}
FACE_THERMAL = {"adiabatic": 0, "dirichlet": 1}


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no contraction of multiply-adds),
    and its rounding twin with contraction into fused multiply-adds."""
    for out, flags in ((LIB, ["-ffp-contract=off"]),
                       (LIB_FMA, ["-mfma", "-ffp-contract=fast"])):
        cmd = ["gcc", "-std=c11", "-O2", *flags, "-fopenmp", "-fPIC",
               "-shared", "-Wall", "-o", out + ".tmp", SRC, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-o", LIB3 + ".tmp", SRC3, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB3 + ".tmp", LIB3)
    return LIB


def host_has_fma() -> bool:
    try:
        with open("/proc/cpuinfo") as fh:
            return " fma " in fh.read().replace("\n", " ")
    except OSError:
        return False


class _Domain(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("face_flow", ctypes.c_int32 * 4),
        ("u_wall", (ctypes.c_double * 2) * 4),
        ("face_thermal", ctypes.c_int32 * 4),
        ("T_wall", ctypes.c_double * 4),
        ("tau_f", ctypes.c_double), ("rho_f", ctypes.c_double),
        ("cv_f", ctypes.c_double), ("lambda_f", ctypes.c_double),
        ("R_lambda", ctypes.c_double), ("R_cv", ctypes.c_double),
        ("body_force", ctypes.c_double * 2), ("gravity", ctypes.c_double * 2),
        ("beta", ctypes.c_double), ("T_ref", ctypes.c_double),
        ("sigma_rule", ctypes.c_int32),
        ("fluid_gravity", ctypes.c_int32),
        ("coll_range", ctypes.c_double), ("coll_stiff_pp", ctypes.c_double),
        ("coll_stiff_pw", ctypes.c_double),
        ("init_rho", ctypes.c_double), ("init_u", ctypes.c_double * 2),
        ("init_T", ctypes.c_double),
        ("kmax", ctypes.c_int32),
    ]


class _Particle(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("x", "y", "theta", "ux", "uy", "omega", "radius", "rho_s",
                 "T_init", "radius_minor")] + [("fixed", ctypes.c_int32),
                                               ("hold_T", ctypes.c_int32)]


class _PState(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("x", "y", "theta", "ux", "uy", "omega", "Fx", "Fy", "Tz",
                 "T_mean", "T_min", "E_solid", "fs_sum", "F_abs")]


class _Hooks(ctypes.Structure):
    _fields_ = [("beta1", ctypes.c_double), ("dfs_backward", ctypes.c_int32),
                ("thermal_only", ctypes.c_int32),
                ("u_pres", ctypes.c_double * 2),
                ("fs_from_array", ctypes.c_int32)]


_libs: dict = {}


def lib(variant: str = "plain"):
    if variant not in _libs:
        path = LIB if variant == "plain" else LIB_FMA
        if not os.path.exists(path):
            build()
        L = ctypes.CDLL(path)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        dptr = ctypes.POINTER(ctypes.c_double)
        iptr = ctypes.POINTER(ctypes.c_int32)
        L.or_create.argtypes = [ctypes.POINTER(_Domain), i32,
                                ctypes.POINTER(_Particle), ctypes.POINTER(vp)]
        L.or_create.restype = ctypes.c_int
        L.or_destroy.argtypes = [vp]
        L.or_destroy.restype = None
        L.or_default_hooks.argtypes = [ctypes.POINTER(_Hooks)]
        L.or_set_hooks.argtypes = [vp, ctypes.POINTER(_Hooks)]
        L.or_init.argtypes = [vp]
        L.or_step.argtypes = [vp, i64]
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_step_count.argtypes = [vp]
        L.or_step_count.restype = i64
        for name in ("or_f", "or_g", "or_d", "or_fs", "or_rho", "or_ux",
                     "or_uy", "or_T", "or_eps", "or_qc", "or_fs_next"):
            fn = getattr(L, name)
            fn.argtypes = [vp]
            fn.restype = dptr
        for name in ("or_own_count", "or_own_ids", "or_own_full"):
            fn = getattr(L, name)
            fn.argtypes = [vp]
            fn.restype = iptr
        L.or_read_particles.argtypes = [vp, i32, ctypes.POINTER(_PState)]
        L.or_overlap_count.argtypes = [vp]
        L.or_disk_cell_area.argtypes = [ctypes.c_double] * 5
        L.or_disk_cell_area.restype = ctypes.c_double
        L.or_ellipse_cell_area.argtypes = [ctypes.c_double] * 7
        L.or_ellipse_cell_area.restype = ctypes.c_double
        L.or_cell_in_band.argtypes = [ctypes.c_double] * 3 + [i32, i32]
        L.or_cell_inside.argtypes = [ctypes.c_double] * 3 + [i32, i32]
        L.or_collision_force.argtypes = [vp, i32, dptr, dptr]
        _libs[variant] = L
    return _libs[variant]


def set_threads(n: int) -> int:
    return lib().or_set_threads(int(n))


def _domain_struct(d: dict) -> _Domain:
    s = _Domain()
    s.nx, s.ny = int(d["nx"]), int(d["ny"])
    for k in range(4):
        s.face_flow[k] = FACE_FLOW[d["face_flow"][k]]
        s.u_wall[k][0], s.u_wall[k][1] = d["u_wall"][k]
        s.face_thermal[k] = FACE_THERMAL[d["face_thermal"][k]]
        s.T_wall[k] = d["T_wall"][k]
    for name in ("tau_f", "rho_f", "cv_f", "lambda_f", "R_lambda", "R_cv",
                 "beta", "T_ref", "coll_range", "coll_stiff_pp",
                 "coll_stiff_pw", "init_rho", "init_T"):
        setattr(s, name, float(d[name]))
    s.body_force[0], s.body_force[1] = d["body_force"]
    s.gravity[0], s.gravity[1] = d["gravity"]
    s.init_u[0], s.init_u[1] = d["init_u"]
    s.sigma_rule = int(d["sigma_rule"])
    s.fluid_gravity = int(d.get("fluid_gravity", 0))
    s.kmax = int(d["kmax"])
    return s


def _particles_struct(ps):
    arr = (_Particle * max(1, len(ps)))()
    for k, p in enumerate(ps):
        for name in ("x", "y", "theta", "ux", "uy", "omega", "radius", "rho_s",
                     "T_init"):
            setattr(arr[k], name, float(p[name]))
        arr[k].radius_minor = float(p.get("radius_minor", 0.0))
        arr[k].fixed = int(p["fixed"])
        arr[k].hold_T = int(p.get("hold_T", 0))
    return arr


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"oracle {where} failed with status {code}")
        self.code = code


class Oracle:
    """One oracle domain.  Field accessors return numpy copies shaped
    (ny, nx) or (9, ny, nx)."""

    def __init__(self, domain: dict, particles=(), hooks: dict | None = None,
                 variant: str = "plain"):
        self._variant = variant
        L = lib(variant)
        self.domain = dict(domain)
        self.nx, self.ny = int(domain["nx"]), int(domain["ny"])
        self.np_ = len(particles)
        self._dom = _domain_struct(domain)
        self._parts = _particles_struct(list(particles))
        h = ctypes.c_void_p()
        rc = L.or_create(ctypes.byref(self._dom), self.np_, self._parts,
                         ctypes.byref(h))
        if rc != 0:
            raise OracleError(rc, "create")
        self._h = h
        if hooks:
            hk = _Hooks()
            L.or_default_hooks(ctypes.byref(hk))
            for k, v in hooks.items():
                if k == "u_pres":
                    hk.u_pres[0], hk.u_pres[1] = v
                else:
                    setattr(hk, k, v)
            rc = L.or_set_hooks(h, ctypes.byref(hk))
            if rc != 0:
                raise OracleError(rc, "set_hooks")

    def close(self):
        if getattr(self, "_h", None):
            lib(self._variant).or_destroy(self._h)
            self._h = None

    __del__ = close

    def init(self):
        rc = lib(self._variant).or_init(self._h)
        if rc != 0:
            raise OracleError(rc, "init")
        return self

    def step(self, n: int = 1):
        rc = lib(self._variant).or_step(self._h, int(n))
        if rc != 0:
            raise OracleError(rc, "step")
        return self

    @property
    def step_count(self) -> int:
        return int(lib(self._variant).or_step_count(self._h))

    def _view(self, name, shape, dtype=np.float64):
        ptr = getattr(lib(self._variant), name)(self._h)
        n = int(np.prod(shape))
        ct = ctypes.c_double if dtype == np.float64 else ctypes.c_int32
        buf = ctypes.cast(ptr, ctypes.POINTER(ct * n)).contents
        return np.frombuffer(buf, dtype=dtype).reshape(shape)

    def field(self, name: str) -> np.ndarray:
        """'f', 'g' -> (9, ny, nx); 'd', 'fs', 'rho', 'ux', 'uy', 'T', 'eps',
        'qc' -> (ny, nx).  Returns a copy."""
        if name in ("f", "g"):
            return self._view("or_" + name, (9, self.ny, self.nx)).copy()
        return self._view("or_" + name, (self.ny, self.nx)).copy()

    def raw(self, name: str) -> np.ndarray:
        """Writable view (for the caller-driven hooks: 'fs_next', 'T')."""
        return self._view("or_" + name, (self.ny, self.nx))

    def ownership(self):
        K = int(self.domain["kmax"])
        cnt = self._view("or_own_count", (self.ny, self.nx), np.int32).copy()
        ids = self._view("or_own_ids", (self.ny, self.nx, K), np.int32).copy()
        full = self._view("or_own_full", (self.ny, self.nx, K), np.int32).copy()
        return cnt, ids, full

    def particles(self) -> np.ndarray:
        """Structured array with the fields of or_particle_state."""
        n = self.np_
        arr = (_PState * max(1, n))()
        rc = lib(self._variant).or_read_particles(self._h, n, arr)
        if rc != 0:
            raise OracleError(rc, "read_particles")
        names = [f[0] for f in _PState._fields_]
        out = np.zeros(n, dtype=[(k, np.float64) for k in names])
        for i in range(n):
            for k in names:
                out[i][k] = getattr(arr[i], k)
        return out

    def overlap_count(self) -> int:
        return int(lib(self._variant).or_overlap_count(self._h))

    def collision_force(self, i: int):
        fx, fy = ctypes.c_double(), ctypes.c_double()
        lib(self._variant).or_collision_force(self._h, int(i), ctypes.byref(fx),
                                 ctypes.byref(fy))
        return fx.value, fy.value


def disk_cell_area(cx, cy, R, x0, y0) -> float:
    return lib().or_disk_cell_area(float(cx), float(cy), float(R), float(x0),
                                   float(y0))


def ellipse_cell_area(cx, cy, a, b, th, x0, y0) -> float:
    return lib().or_ellipse_cell_area(float(cx), float(cy), float(a), float(b),
                                      float(th), float(x0), float(y0))


def cell_in_band(X, Y, R, i, j) -> bool:
    return bool(lib().or_cell_in_band(float(X), float(Y), float(R), int(i),
                                      int(j)))


def cell_inside(X, Y, R, i, j) -> bool:
    return bool(lib().or_cell_inside(float(X), float(Y), float(R), int(i),
                                     int(j)))
