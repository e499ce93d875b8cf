"""Python binding of the C ABI in include/vlb.h (argument marshalling only).

Every step of the lattice update runs in the HIP kernels of libvlb.so; this
module only converts Python values to the C structs and back.  It raises
``VlbLibraryMissing`` when the library has not been built -- there is no
fallback path.

Functions keep the C names (``vlb_create``, ``vlb_step``, ...).  ``Domain``
is a small convenience wrapper over one context.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvlb.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "vlb.h")
HEADER3 = os.path.join(os.path.dirname(HERE), "include", "vlb3.h")

VLB_OK, VLB_EINVAL, VLB_ENOMEM, VLB_EHIP = 0, -1, -2, -3
VLB_EUNSTABLE, VLB_EOVERLAP, VLB_ESTATE = -4, -5, -6
STATUS_NAMES = {0: "VLB_OK", -1: "VLB_EINVAL", -2: "VLB_ENOMEM",
                -3: "VLB_EHIP", -4: "VLB_EUNSTABLE", -5: "VLB_EOVERLAP",
                -6: "VLB_ESTATE"}
PRECISIONS = {"fp64": 0, "fp32": 1, "fp16s": 2, "bf16s": 3}
FIELDS = {"rho": 0, "ux": 1, "uy": 2, "T": 3, "fs": 4, "dfs": 5, "f": 6,
          "g": 7}
FACE_FLOW = {"periodic": 0, "wall": 1}
FACE_THERMAL = {"adiabatic": 0, "dirichlet": 1}


class VlbLibraryMissing(RuntimeError):
    pass


class VlbLibraryStale(RuntimeError):
    """The built library does not match the sources beside it."""


class VlbError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class vlb_domain_desc(ctypes.Structure):
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
        ("kmax", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("shift_rho0", ctypes.c_double), ("shift_T0", ctypes.c_double),
    ]


class vlb_particle_desc(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("x", "y", "theta", "ux", "uy", "omega", "radius", "rho_s",
                 "T_init", "radius_minor")] + [("fixed", ctypes.c_int32),
                                               ("hold_T", ctypes.c_int32)]


class vlb3_domain_desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("face_flow", ctypes.c_int32 * 6),
        ("u_wall", (ctypes.c_double * 3) * 6),
        ("face_thermal", ctypes.c_int32 * 6),
        ("T_wall", ctypes.c_double * 6),
        ("tau_f", ctypes.c_double),
        ("rho_f", ctypes.c_double), ("cv_f", ctypes.c_double),
        ("lambda_f", ctypes.c_double),
        ("R_lambda", ctypes.c_double), ("R_cv", ctypes.c_double),
        ("body_force", ctypes.c_double * 3), ("gravity", ctypes.c_double * 3),
        ("beta", ctypes.c_double), ("T_ref", ctypes.c_double),
        ("sigma_rule", ctypes.c_int32),
        ("coll_range", ctypes.c_double), ("coll_stiff_pp", ctypes.c_double),
        ("coll_stiff_pw", ctypes.c_double),
        ("init_rho", ctypes.c_double), ("init_u", ctypes.c_double * 3),
        ("init_T", ctypes.c_double),
        ("kmax", ctypes.c_int32), ("precision", ctypes.c_int32),
    ]


class vlb3_sphere_desc(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("x", "y", "z", "ux", "uy", "uz", "ox", "oy", "oz", "radius",
                 "rho_s", "T_init")] + [("fixed", ctypes.c_int32)]


class vlb3_sphere_state(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("x", "y", "z", "ux", "uy", "uz", "ox", "oy", "oz", "Fx", "Fy",
                 "Fz", "Tx", "Ty", "Tz", "T_mean", "T_min", "E_solid",
                 "fs_sum")]


FIELDS3 = {"rho": 0, "ux": 1, "uy": 2, "uz": 3, "T": 4, "fs": 5, "dfs": 6}


class vlb_batch_tuning(ctypes.Structure):
    _fields_ = [("grid_blocks", ctypes.c_int32), ("order", ctypes.c_int32),
                ("use_graph", ctypes.c_int32),
                ("pair_min_tiles", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("us_per_step", ctypes.c_double)]


class vlb_particle_state(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("x", "y", "theta", "ux", "uy", "omega", "Fx", "Fy", "Tz",
                 "T_mean", "T_min", "E_solid", "fs_sum")]


_lib = None


def lib():
    """Load libvlb.so (built by paper_2410_23802_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise VlbLibraryMissing(
            f"{LIB_PATH} is not built; run paper_2410_23802_amd.build.build()")
    # PyTorch carries its own HIP runtime (soname libamdhip64.so.7), and the
    # binding hands torch's device pointers and streams across the ABI, so
    # the library must run on that same runtime: with torch loaded first,
    # the library's HIP and HSA dependencies resolve to torch's copies.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    # the binary must come from the sources beside it
    from . import build as _build
    L.vlb_build_hash.restype = ctypes.c_char_p
    L.vlb_build_hash.argtypes = []
    built, want = L.vlb_build_hash().decode(), _build.source_hash()
    if built != want:
        raise VlbLibraryStale(
            f"{LIB_PATH} was built from other sources (hash {built}, sources "
            f"{want}); run paper_2410_23802_amd.build.build()")
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "vlb_create": ([ctypes.POINTER(vlb_domain_desc), vp,
                        ctypes.POINTER(vp)], ctypes.c_int),
        "vlb_set_particles": ([vp, i32, ctypes.POINTER(vlb_particle_desc)],
                              ctypes.c_int),
        "vlb_init": ([vp], ctypes.c_int),
        "vlb_step": ([vp, i64], ctypes.c_int),
        "vlb_read_field": ([vp, i32, vp, i32], ctypes.c_int),
        "vlb_read_particles": ([vp, i32, ctypes.POINTER(vlb_particle_state)],
                               ctypes.c_int),
        "vlb_read_ownership": ([vp, vp, vp, vp], ctypes.c_int),
        "vlb_read_ownership_noalloc": ([vp, vp, vp, vp], ctypes.c_int),
        "vlb_save": ([vp, vp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "vlb_load": ([vp, vp, ctypes.c_size_t], ctypes.c_int),
        "vlb_step_count": ([vp], i64),
        "vlb_timing_enable": ([vp, i32], ctypes.c_int),
        "vlb_timing_read": ([vp, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(i64)], ctypes.c_int),
        "vlb_stream_probe": ([vp, i32, ctypes.POINTER(ctypes.c_double)],
                             ctypes.c_int),
        "vlb_device_bytes": ([vp], ctypes.c_size_t),
        "vlb_last_error": ([vp], ctypes.c_char_p),
        "vlb_build_hash": ([], ctypes.c_char_p),
        "vlb_destroy": ([vp], None),
        "vlb_batch_create": ([i32, ctypes.POINTER(vlb_domain_desc),
                              ctypes.POINTER(i32),
                              ctypes.POINTER(vlb_particle_desc),
                              ctypes.POINTER(vp)], ctypes.c_int),
        "vlb_batch_init": ([vp], ctypes.c_int),
        "vlb_batch_step": ([vp, i64], ctypes.c_int),
        "vlb_batch_autotune": ([vp, i32, ctypes.POINTER(vlb_batch_tuning)],
                               ctypes.c_int),
        "vlb_batch_set_tuning": ([vp, ctypes.POINTER(vlb_batch_tuning)],
                                 ctypes.c_int),
        "vlb_batch_get_tuning": ([vp, ctypes.POINTER(vlb_batch_tuning)],
                                 ctypes.c_int),
        "vlb_batch_read_field": ([vp, i32, i32, vp, i32], ctypes.c_int),
        "vlb_batch_read_particles": ([vp, i32, i32,
                                      ctypes.POINTER(vlb_particle_state)],
                                     ctypes.c_int),
        "vlb_batch_size": ([vp], i32),
        "vlb_batch_cells": ([vp], i64),
        "vlb_batch_step_count": ([vp], i64),
        "vlb_batch_device_bytes": ([vp], ctypes.c_size_t),
        "vlb_batch_last_error": ([vp], ctypes.c_char_p),
        "vlb_batch_destroy": ([vp], None),
        "vlb3_create": ([ctypes.POINTER(vlb3_domain_desc), i32,
                         ctypes.POINTER(vlb3_sphere_desc), vp,
                         ctypes.POINTER(vp)], ctypes.c_int),
        "vlb3_init": ([vp], ctypes.c_int),
        "vlb3_step": ([vp, i64], ctypes.c_int),
        "vlb3_read_field": ([vp, i32, vp, i32], ctypes.c_int),
        "vlb3_read_populations": ([vp, i32, vp], ctypes.c_int),
        "vlb3_read_spheres": ([vp, i32, ctypes.POINTER(vlb3_sphere_state)],
                              ctypes.c_int),
        "vlb3_save": ([vp, vp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "vlb3_load": ([vp, vp, ctypes.c_size_t], ctypes.c_int),
        "vlb3_timing_enable": ([vp, i32], ctypes.c_int),
        "vlb3_timing_read": ([vp, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(i64)], ctypes.c_int),
        "vlb3_step_count": ([vp], i64),
        "vlb3_device_bytes": ([vp], ctypes.c_size_t),
        "vlb3_last_error": ([vp], ctypes.c_char_p),
        "vlb3_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def header_functions() -> list[str]:
    """Names of the functions include/vlb.h and include/vlb3.h declare."""
    names = set()
    for path in (HEADER, HEADER3):
        with open(path) as fh:
            txt = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        names |= set(re.findall(r"\b(vlb3?_\w+)\s*\(", txt))
    return sorted(names)


def make_domain_desc(d: dict, precision="fp64", shift_rho0=None,
                     shift_T0=None) -> vlb_domain_desc:
    s = vlb_domain_desc()
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
    s.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    s.shift_rho0 = float(d["init_rho"] if shift_rho0 is None else shift_rho0)
    s.shift_T0 = float(0.5 if shift_T0 is None else shift_T0)
    return s


def make_particles(ps) -> ctypes.Array:
    arr = (vlb_particle_desc * max(1, len(ps)))()
    for k, p in enumerate(ps):
        for name in ("x", "y", "theta", "ux", "uy", "omega", "radius", "rho_s",
                     "T_init"):
            setattr(arr[k], name, float(p[name]))
        arr[k].radius_minor = float(p.get("radius_minor", 0.0))
        arr[k].fixed = int(p["fixed"])
        arr[k].hold_T = int(p.get("hold_T", 0))
    return arr


def _check(status: int, where: str, handle=None):
    if status != VLB_OK:
        msg = lib().vlb_last_error(handle)
        raise VlbError(status, where, msg.decode() if msg else "")


def _stream_handle(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except Exception:
            pass
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


# ---- C-named wrappers -------------------------------------------------------


def vlb_create(desc: vlb_domain_desc, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().vlb_create(ctypes.byref(desc), _stream_handle(stream),
                            ctypes.byref(h)), "vlb_create")
    return h


def vlb_set_particles(h, particles) -> None:
    arr = make_particles(particles)
    _check(lib().vlb_set_particles(h, len(particles), arr),
           "vlb_set_particles", h)


def vlb_init(h) -> None:
    _check(lib().vlb_init(h), "vlb_init", h)


def vlb_step(h, nsteps: int) -> None:
    _check(lib().vlb_step(h, int(nsteps)), "vlb_step", h)


def vlb_read_field(h, field, dst_ptr: int, dst_is_device: bool) -> None:
    fid = FIELDS[field] if isinstance(field, str) else int(field)
    _check(lib().vlb_read_field(h, fid, ctypes.c_void_p(dst_ptr),
                                int(bool(dst_is_device))), "vlb_read_field", h)


def vlb_read_particles(h, n: int) -> np.ndarray:
    arr = (vlb_particle_state * max(1, n))()
    _check(lib().vlb_read_particles(h, n, arr), "vlb_read_particles", h)
    names = [f[0] for f in vlb_particle_state._fields_]
    out = np.zeros(n, dtype=[(k, np.float64) for k in names])
    for i in range(n):
        out[i] = tuple(getattr(arr[i], k) for k in names)
    return out


def vlb_read_ownership(h, nx, ny, kmax):
    cnt = np.zeros((ny, nx), np.int32)
    ids = np.zeros((ny, nx, kmax), np.int32)
    full = np.zeros((ny, nx, kmax), np.int32)
    _check(lib().vlb_read_ownership(h, cnt.ctypes.data, ids.ctypes.data,
                                    full.ctypes.data), "vlb_read_ownership", h)
    return cnt, ids, full


def vlb_read_ownership_noalloc(h, nx, ny, kmax):
    """vlb_read_ownership through the entry point that allocates no device
    memory (the library's static staging array)."""
    cnt = np.zeros((ny, nx), np.int32)
    ids = np.zeros((ny, nx, kmax), np.int32)
    full = np.zeros((ny, nx, kmax), np.int32)
    _check(lib().vlb_read_ownership_noalloc(
        h, cnt.ctypes.data, ids.ctypes.data, full.ctypes.data),
        "vlb_read_ownership_noalloc", h)
    return cnt, ids, full


def vlb_save(h) -> bytes:
    n = ctypes.c_size_t(0)
    _check(lib().vlb_save(h, None, ctypes.byref(n)), "vlb_save", h)
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().vlb_save(h, buf, ctypes.byref(n)), "vlb_save", h)
    return buf.raw[: n.value]


def vlb_load(h, data: bytes) -> None:
    buf = ctypes.create_string_buffer(data, len(data))
    _check(lib().vlb_load(h, buf, len(data)), "vlb_load", h)


def vlb_step_count(h) -> int:
    return int(lib().vlb_step_count(h))


def vlb_timing_enable(h, on: bool) -> None:
    _check(lib().vlb_timing_enable(h, int(bool(on))), "vlb_timing_enable", h)


def vlb_timing_read(h):
    """(summed ms, launches) of the timed lattice-step launches since the
    last read."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().vlb_timing_read(h, ctypes.byref(ms), ctypes.byref(n)),
           "vlb_timing_read", h)
    return ms.value, n.value


def vlb_stream_probe(h, reps: int) -> float:
    """Average microseconds of one launch of the step's memory pattern
    without its arithmetic (state unchanged)."""
    us = ctypes.c_double()
    _check(lib().vlb_stream_probe(h, int(reps), ctypes.byref(us)),
           "vlb_stream_probe", h)
    return us.value


def vlb_device_bytes(h) -> int:
    return int(lib().vlb_device_bytes(h))


def vlb_last_error(h=None) -> str:
    m = lib().vlb_last_error(h)
    return m.decode() if m else ""


def vlb_destroy(h) -> None:
    lib().vlb_destroy(h)


# ---- convenience wrapper ----------------------------------------------------


class Domain:
    """One simulation context.  `domain` and `particles` are the plain dicts
    of the `workloads` module."""

    def __init__(self, domain: dict, particles=(), precision="fp64",
                 stream=None, shift_rho0=None, shift_T0=None):
        self.domain = dict(domain)
        self.nx, self.ny = int(domain["nx"]), int(domain["ny"])
        self.kmax = int(domain["kmax"])
        self.np_ = len(particles)
        self.precision = precision
        self._desc = make_domain_desc(domain, precision, shift_rho0, shift_T0)
        # kept on the object: at interpreter exit the module globals may
        # already be gone when close() runs from __del__
        self._destroy = lib().vlb_destroy
        self.h = vlb_create(self._desc, stream)
        try:
            vlb_set_particles(self.h, list(particles))
        except Exception:
            self.close()
            raise

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self._destroy(self.h)
            self.h = None

    __del__ = close

    def init(self):
        vlb_init(self.h)
        return self

    def step(self, n: int = 1):
        vlb_step(self.h, n)
        return self

    @property
    def step_count(self) -> int:
        return vlb_step_count(self.h)

    def field(self, name: str) -> np.ndarray:
        """Host copy, (ny, nx) or (9, ny, nx) for 'f' and 'g'."""
        shape = (9, self.ny, self.nx) if name in ("f", "g") else (self.ny, self.nx)
        out = np.empty(shape, np.float64)
        vlb_read_field(self.h, name, out.ctypes.data, False)
        return out

    def field_device(self, name: str, out):
        """Copy into a CUDA/HIP torch tensor of float64 on this device."""
        vlb_read_field(self.h, name, out.data_ptr(), True)
        return out

    def particles(self) -> np.ndarray:
        return vlb_read_particles(self.h, self.np_)

    def ownership(self):
        return vlb_read_ownership(self.h, self.nx, self.ny, self.kmax)

    def save(self) -> bytes:
        return vlb_save(self.h)

    def load(self, data: bytes):
        vlb_load(self.h, data)
        return self

    def timing(self, on: bool = True):
        vlb_timing_enable(self.h, on)

    def timing_read(self):
        return vlb_timing_read(self.h)

    def stream_probe(self, reps: int = 50) -> float:
        return vlb_stream_probe(self.h, reps)


# ---- batches ------------------------------------------------------------------


def _bcheck(status: int, where: str, h=None) -> None:
    if status != VLB_OK:
        m = lib().vlb_batch_last_error(h)
        raise VlbError(status, where, m.decode() if m else "")


def _state_array(arr, n) -> np.ndarray:
    names = [f[0] for f in vlb_particle_state._fields_]
    out = np.zeros(n, dtype=[(k, np.float64) for k in names])
    for i in range(n):
        for k in names:
            out[i][k] = getattr(arr[i], k)
    return out


class Batch:
    """Independent domains advanced together: `cases` is a list of
    (domain dict, particle list) pairs of the `workloads` module."""

    def __init__(self, cases, precision="fp32", shift_T0=None):
        n = len(cases)
        self.cases = [(dict(d), list(ps)) for d, ps in cases]
        descs = (vlb_domain_desc * n)()
        counts = (ctypes.c_int32 * n)()
        allp = []
        for i, (d, ps) in enumerate(self.cases):
            descs[i] = make_domain_desc(d, precision, None, shift_T0)
            counts[i] = len(ps)
            allp.extend(ps)
        parts = make_particles(allp)
        self._destroy = lib().vlb_batch_destroy   # see Domain.__init__
        h = ctypes.c_void_p()
        _bcheck(lib().vlb_batch_create(n, descs, counts, parts,
                                       ctypes.byref(h)), "vlb_batch_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self._destroy(self.h)
            self.h = None

    __del__ = close

    def __len__(self):
        return int(lib().vlb_batch_size(self.h))

    @property
    def cells(self) -> int:
        return int(lib().vlb_batch_cells(self.h))

    def init(self):
        _bcheck(lib().vlb_batch_init(self.h), "vlb_batch_init", self.h)
        return self

    def step(self, n: int = 1):
        _bcheck(lib().vlb_batch_step(self.h, int(n)), "vlb_batch_step", self.h)
        return self

    def autotune(self, steps: int = 5) -> dict:
        t = vlb_batch_tuning()
        _bcheck(lib().vlb_batch_autotune(self.h, int(steps), ctypes.byref(t)),
                "vlb_batch_autotune", self.h)
        return {k: getattr(t, k) for k, _ in vlb_batch_tuning._fields_}

    def tuning(self) -> dict:
        t = vlb_batch_tuning()
        _bcheck(lib().vlb_batch_get_tuning(self.h, ctypes.byref(t)),
                "vlb_batch_get_tuning", self.h)
        return {k: getattr(t, k) for k, _ in vlb_batch_tuning._fields_}

    def set_tuning(self, grid_blocks: int, order: int, use_graph: bool = True,
                   pair_min_tiles: int = -1, waves: int = 0):
        t = vlb_batch_tuning(int(grid_blocks), int(order), int(bool(use_graph)),
                             int(pair_min_tiles), int(waves), 0.0)
        _bcheck(lib().vlb_batch_set_tuning(self.h, ctypes.byref(t)),
                "vlb_batch_set_tuning", self.h)
        return self

    def field(self, i: int, name: str) -> np.ndarray:
        d = self.cases[i][0]
        shape = ((9, d["ny"], d["nx"]) if name in ("f", "g")
                 else (d["ny"], d["nx"]))
        out = np.empty(shape, np.float64)
        _bcheck(lib().vlb_batch_read_field(self.h, int(i), FIELDS[name],
                                           out.ctypes.data, 0),
                "vlb_batch_read_field", self.h)
        return out

    def particles(self, i: int) -> np.ndarray:
        n = len(self.cases[i][1])
        arr = (vlb_particle_state * max(1, n))()
        _bcheck(lib().vlb_batch_read_particles(self.h, int(i), n, arr),
                "vlb_batch_read_particles", self.h)
        return _state_array(arr, n)


# ---------------------------------------------------------------------------
# Three dimensions (include/vlb3.h)

def make_domain3_desc(d: dict, precision="fp64") -> vlb3_domain_desc:
    s = vlb3_domain_desc()
    s.nx, s.ny, s.nz = int(d["nx"]), int(d["ny"]), int(d["nz"])
    for k in range(6):
        s.face_flow[k] = FACE_FLOW[d["face_flow"][k]]
        s.face_thermal[k] = FACE_THERMAL[d["face_thermal"][k]]
        s.T_wall[k] = float(d["T_wall"][k])
        for a in range(3):
            s.u_wall[k][a] = float(d["u_wall"][k][a])
    for name in ("tau_f", "rho_f", "cv_f", "lambda_f", "R_lambda", "R_cv",
                 "beta", "T_ref", "coll_range", "coll_stiff_pp",
                 "coll_stiff_pw", "init_rho", "init_T"):
        setattr(s, name, float(d[name]))
    for a in range(3):
        s.body_force[a] = float(d["body_force"][a])
        s.gravity[a] = float(d["gravity"][a])
        s.init_u[a] = float(d["init_u"][a])
    s.sigma_rule = int(d["sigma_rule"])
    s.kmax = int(d["kmax"])
    s.precision = (PRECISIONS[precision] if isinstance(precision, str)
                   else int(precision))
    return s


def make_spheres(ps) -> ctypes.Array:
    arr = (vlb3_sphere_desc * max(1, len(ps)))()
    for k, p in enumerate(ps):
        for n in ("x", "y", "z", "ux", "uy", "uz", "ox", "oy", "oz", "radius",
                  "rho_s", "T_init"):
            setattr(arr[k], n, float(p[n]))
        arr[k].fixed = int(p.get("fixed", 0))
    return arr


def _check3(status: int, where: str, handle=None):
    if status != VLB_OK:
        msg = lib().vlb3_last_error(handle)
        raise VlbError(status, where, msg.decode() if msg else "")


class Domain3:
    """One three-dimensional domain on the GPU, through the vlb3_* C ABI:
    populations stored in FP64 or FP32 ("fp64", "fp32"), the arithmetic in
    FP64.  Fields are numpy arrays shaped (nz, ny, nx)."""

    def __init__(self, d: dict, spheres=(), stream=None, precision="fp64"):
        self.d = dict(d)
        self.spheres = list(spheres)
        self.shape = (int(d["nz"]), int(d["ny"]), int(d["nx"]))
        self.precision = precision
        desc = make_domain3_desc(d, precision)
        arr = make_spheres(self.spheres)
        self._destroy = lib().vlb3_destroy    # see Domain.__init__
        h = ctypes.c_void_p()
        _check3(lib().vlb3_create(ctypes.byref(desc), len(self.spheres), arr,
                                  _stream_handle(stream), ctypes.byref(h)),
                "vlb3_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self._destroy(self.h)
            self.h = None

    __del__ = close

    def init(self):
        _check3(lib().vlb3_init(self.h), "vlb3_init", self.h)
        return self

    def step(self, n: int = 1):
        _check3(lib().vlb3_step(self.h, int(n)), "vlb3_step", self.h)
        return self

    def field(self, name: str) -> np.ndarray:
        out = np.empty(self.shape, np.float64)
        _check3(lib().vlb3_read_field(self.h, FIELDS3[name], out.ctypes.data,
                                      0), "vlb3_read_field", self.h)
        return out

    def populations(self, which: str) -> np.ndarray:
        q = 19 if which == "f" else 7
        out = np.empty((q,) + self.shape, np.float64)
        _check3(lib().vlb3_read_populations(self.h, 0 if which == "f" else 1,
                                            out.ctypes.data),
                "vlb3_read_populations", self.h)
        return out

    def particles(self) -> np.ndarray:
        n = len(self.spheres)
        arr = (vlb3_sphere_state * max(1, n))()
        _check3(lib().vlb3_read_spheres(self.h, n, arr), "vlb3_read_spheres",
                self.h)
        names = [f[0] for f in vlb3_sphere_state._fields_]
        out = np.zeros(n, dtype=[(k, np.float64) for k in names])
        for i in range(n):
            for k in names:
                out[i][k] = getattr(arr[i], k)
        return out

    def save(self) -> bytes:
        n = ctypes.c_size_t(0)
        _check3(lib().vlb3_save(self.h, None, ctypes.byref(n)), "vlb3_save",
                self.h)
        buf = ctypes.create_string_buffer(n.value)
        _check3(lib().vlb3_save(self.h, buf, ctypes.byref(n)), "vlb3_save",
                self.h)
        return buf.raw[:n.value]

    def load(self, data: bytes):
        buf = ctypes.create_string_buffer(bytes(data), len(data))
        _check3(lib().vlb3_load(self.h, buf, len(data)), "vlb3_load", self.h)
        return self

    def timing(self, on: bool):
        _check3(lib().vlb3_timing_enable(self.h, int(bool(on))),
                "vlb3_timing_enable", self.h)
        return self

    def timing_read(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check3(lib().vlb3_timing_read(self.h, ctypes.byref(ms),
                                       ctypes.byref(n)), "vlb3_timing_read",
                self.h)
        return ms.value, n.value

    @property
    def device_bytes(self) -> int:
        return int(lib().vlb3_device_bytes(self.h))
