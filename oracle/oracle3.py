"""ctypes wrapper of the three-dimensional FP64 CPU oracle
(``vlb3_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU
baseline leg of ``bench.py`` may import this module.  It imports nothing from
the product package; inputs come as plain dicts (``workloads3`` builds them).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import oracle as _o2

FACE_FLOW = {"periodic": 0, "wall": 1}
FACE_THERMAL = {"adiabatic": 0, "dirichlet": 1}


class _Domain(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("face_flow", ctypes.c_int32 * 6),
        ("u_wall", (ctypes.c_double * 3) * 6),
        ("face_thermal", ctypes.c_int32 * 6),
        ("T_wall", ctypes.c_double * 6),
        ("tau_f", ctypes.c_double), ("rho_f", ctypes.c_double),
        ("cv_f", ctypes.c_double), ("lambda_f", ctypes.c_double),
        ("R_lambda", ctypes.c_double), ("R_cv", ctypes.c_double),
        ("body_force", ctypes.c_double * 3), ("gravity", ctypes.c_double * 3),
        ("beta", ctypes.c_double), ("T_ref", ctypes.c_double),
        ("sigma_rule", ctypes.c_int32),
        ("coll_range", ctypes.c_double), ("coll_stiff_pp", ctypes.c_double),
        ("coll_stiff_pw", ctypes.c_double),
        ("init_rho", ctypes.c_double), ("init_u", ctypes.c_double * 3),
        ("init_T", ctypes.c_double),
        ("kmax", ctypes.c_int32),
    ]


PARTICLE_FIELDS = ("x", "y", "z", "ux", "uy", "uz", "ox", "oy", "oz",
                   "radius", "rho_s", "T_init")


class _Particle(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in PARTICLE_FIELDS] + \
        [("fixed", ctypes.c_int32)]


STATE_FIELDS = ("x", "y", "z", "ux", "uy", "uz", "ox", "oy", "oz", "Fx", "Fy",
                "Fz", "Tx", "Ty", "Tz", "T_mean", "T_min", "E_solid", "fs_sum",
                "F_abs")


class _PState(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in STATE_FIELDS]


class _Hooks(ctypes.Structure):
    _fields_ = [("thermal_only", ctypes.c_int32),
                ("u_pres", ctypes.c_double * 3),
                ("fs_from_array", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_o2.LIB3):
            _o2.build()
        L = ctypes.CDLL(_o2.LIB3)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        dptr = ctypes.POINTER(ctypes.c_double)
        iptr = ctypes.POINTER(ctypes.c_int32)
        L.o3_create.argtypes = [ctypes.POINTER(_Domain), i32,
                                ctypes.POINTER(_Particle), ctypes.POINTER(vp)]
        L.o3_destroy.argtypes = [vp]
        L.o3_destroy.restype = None
        L.o3_set_hooks.argtypes = [vp, ctypes.POINTER(_Hooks)]
        L.o3_init.argtypes = [vp]
        L.o3_step.argtypes = [vp, i64]
        for name in ("o3_f", "o3_g", "o3_d", "o3_fs", "o3_rho", "o3_ux",
                     "o3_uy", "o3_uz", "o3_T", "o3_fs_next"):
            fn = getattr(L, name)
            fn.argtypes = [vp]
            fn.restype = dptr
        for name in ("o3_own_count", "o3_own_ids"):
            fn = getattr(L, name)
            fn.argtypes = [vp]
            fn.restype = iptr
        L.o3_read_particles.argtypes = [vp, i32, ctypes.POINTER(_PState)]
        L.o3_sphere_cell_volume.argtypes = [ctypes.c_double] * 7
        L.o3_sphere_cell_volume.restype = ctypes.c_double
        L.o3_cell_in_band.argtypes = [ctypes.c_double] * 4 + [i32] * 3
        L.o3_cell_inside.argtypes = [ctypes.c_double] * 4 + [i32] * 3
        _lib = L
    return _lib


def _domain_struct(d: dict) -> _Domain:
    s = _Domain()
    s.nx, s.ny, s.nz = int(d["nx"]), int(d["ny"]), int(d["nz"])
    for k in range(6):
        s.face_flow[k] = FACE_FLOW[d["face_flow"][k]]
        for a in range(3):
            s.u_wall[k][a] = d["u_wall"][k][a]
        s.face_thermal[k] = FACE_THERMAL[d["face_thermal"][k]]
        s.T_wall[k] = d["T_wall"][k]
    for name in ("tau_f", "rho_f", "cv_f", "lambda_f", "R_lambda", "R_cv",
                 "beta", "T_ref", "coll_range", "coll_stiff_pp",
                 "coll_stiff_pw", "init_rho", "init_T"):
        setattr(s, name, float(d[name]))
    for a in range(3):
        s.body_force[a] = d["body_force"][a]
        s.gravity[a] = d["gravity"][a]
        s.init_u[a] = d["init_u"][a]
    s.sigma_rule = int(d["sigma_rule"])
    s.kmax = int(d["kmax"])
    return s


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"3-D oracle {where} failed with status {code}")
        self.code = code


class Oracle3:
    """One three-dimensional oracle domain.  Fields are numpy copies shaped
    (nz, ny, nx), populations (19 or 7, nz, ny, nx)."""

    def __init__(self, domain: dict, particles=(), hooks: dict | None = None):
        L = lib()
        self.domain = dict(domain)
        self.shape = (int(domain["nz"]), int(domain["ny"]), int(domain["nx"]))
        self.np_ = len(particles)
        self._dom = _domain_struct(domain)
        arr = (_Particle * max(1, self.np_))()
        for k, p in enumerate(particles):
            for n in PARTICLE_FIELDS:
                setattr(arr[k], n, float(p[n]))
            arr[k].fixed = int(p.get("fixed", 0))
        self._parts = arr
        h = ctypes.c_void_p()
        rc = L.o3_create(ctypes.byref(self._dom), self.np_, arr, ctypes.byref(h))
        if rc != 0:
            raise OracleError(rc, "create")
        self._h = h
        if hooks:
            hk = _Hooks()
            for k, v in hooks.items():
                if k == "u_pres":
                    for a in range(3):
                        hk.u_pres[a] = v[a]
                else:
                    setattr(hk, k, v)
            L.o3_set_hooks(h, ctypes.byref(hk))

    def close(self):
        if getattr(self, "_h", None):
            lib().o3_destroy(self._h)
            self._h = None

    __del__ = close

    def init(self):
        rc = lib().o3_init(self._h)
        if rc != 0:
            raise OracleError(rc, "init")
        return self

    def step(self, n: int = 1):
        rc = lib().o3_step(self._h, int(n))
        if rc != 0:
            raise OracleError(rc, "step")
        return self

    def _view(self, name, shape, dtype=np.float64):
        ptr = getattr(lib(), name)(self._h)
        n = int(np.prod(shape))
        ct = ctypes.c_double if dtype == np.float64 else ctypes.c_int32
        buf = ctypes.cast(ptr, ctypes.POINTER(ct * n)).contents
        return np.frombuffer(buf, dtype=dtype).reshape(shape)

    def field(self, name: str) -> np.ndarray:
        """'f' (19, nz, ny, nx), 'g' (7, ...); 'd', 'fs', 'rho', 'ux',
        'uy', 'uz', 'T' (nz, ny, nx).  A copy."""
        if name == "f":
            return self._view("o3_f", (19,) + self.shape).copy()
        if name == "g":
            return self._view("o3_g", (7,) + self.shape).copy()
        return self._view("o3_" + name, self.shape).copy()

    def raw(self, name: str) -> np.ndarray:
        """Writable view ('fs_next', 'T') for the caller-driven hooks."""
        return self._view("o3_" + name, self.shape)

    def ownership(self):
        K = int(self.domain["kmax"])
        cnt = self._view("o3_own_count", self.shape, np.int32).copy()
        ids = self._view("o3_own_ids", self.shape + (K,), np.int32).copy()
        return cnt, ids

    def particles(self) -> np.ndarray:
        n = self.np_
        arr = (_PState * max(1, n))()
        rc = lib().o3_read_particles(self._h, n, arr)
        if rc != 0:
            raise OracleError(rc, "read_particles")
        out = np.zeros(n, dtype=[(k, np.float64) for k in STATE_FIELDS])
        for i in range(n):
            for k in STATE_FIELDS:
                out[i][k] = getattr(arr[i], k)
        return out


def sphere_cell_volume(cx, cy, cz, R, x0, y0, z0) -> float:
    return lib().o3_sphere_cell_volume(*(float(v) for v in
                                         (cx, cy, cz, R, x0, y0, z0)))


def cell_in_band(X, Y, Z, R, i, j, k) -> bool:
    return bool(lib().o3_cell_in_band(float(X), float(Y), float(Z), float(R),
                                      int(i), int(j), int(k)))


def cell_inside(X, Y, Z, R, i, j, k) -> bool:
    return bool(lib().o3_cell_inside(float(X), float(Y), float(Z), float(R),
                                     int(i), int(j), int(k)))
