"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the tests, the benchmark, the GPU library's Python
binding callers and the CPU oracle's callers.  It holds none of the lattice
Boltzmann arithmetic: it only builds plain-dict descriptors of a domain and
its particles, derives the descriptor's physical parameters from the
dimensionless groups the paper uses (Sec. 3.3, eq. nodim.paras: density
ratio, Re, Pr, Gr) and places particles by seeded random sequential
addition.

Units are lattice units (dx = dt = 1).  Cell (i, j) covers [i, i+1] x
[j, j+1], so a particle centre at (nx/2, ny/2) sits on the domain centre.

Descriptor keys (both sides read the same dict):
  nx, ny; face_flow[4] ('periodic' | 'wall'), u_wall[4] (2-vectors),
  face_thermal[4] ('adiabatic' | 'dirichlet'), T_wall[4]  -- faces are
  ordered x-, x+, y-, y+;
  tau_f, rho_f, cv_f, lambda_f, R_lambda, R_cv, body_force, gravity, beta,
  T_ref, sigma_rule (0: Lambda_g = 1/4 rule, 1: sigma_e = 1),
  fluid_gravity (1: situation II of Sec. 3.2), coll_range,
  coll_stiff_pp, coll_stiff_pw, init_rho, init_u, init_T, kmax.
Particle keys: x, y, theta, ux, uy, omega, radius, rho_s, T_init, fixed,
hold_T (temperature held at T_init).
"""
from __future__ import annotations

import math

import numpy as np

XLO, XHI, YLO, YHI = 0, 1, 2, 3


def viscosity(tau_f: float) -> float:
    """Kinematic viscosity of the flow lattice, nu = c_s^2 (tau_f - 1/2)
    (Sec. 2.1), used here only to turn Pr and Gr into descriptor values."""
    return (tau_f - 0.5) / 3.0


def domain(nx: int, ny: int, **kw) -> dict:
    """A descriptor with defaults: periodic box, tau_f = 0.8, unit fluid
    properties, no forces, no collisions, fluid at rest at T = 1."""
    d = dict(
        nx=int(nx), ny=int(ny),
        face_flow=["periodic"] * 4,
        u_wall=[(0.0, 0.0)] * 4,
        face_thermal=["adiabatic"] * 4,
        T_wall=[0.0] * 4,
        tau_f=0.8, rho_f=1.0, cv_f=1.0, lambda_f=0.1,
        R_lambda=1.0, R_cv=1.0,
        body_force=(0.0, 0.0), gravity=(0.0, 0.0), beta=0.0, T_ref=1.0,
        sigma_rule=0, fluid_gravity=0,
        coll_range=0.0, coll_stiff_pp=0.0, coll_stiff_pw=0.0,
        init_rho=1.0, init_u=(0.0, 0.0), init_T=1.0,
        kmax=4,
    )
    for k, v in kw.items():
        if k not in d:
            raise KeyError(f"unknown descriptor key {k!r}")
        d[k] = v
    d["face_flow"] = list(d["face_flow"])
    d["u_wall"] = [tuple(map(float, u)) for u in d["u_wall"]]
    d["face_thermal"] = list(d["face_thermal"])
    d["T_wall"] = [float(t) for t in d["T_wall"]]
    return d


def walls(d: dict, which=(XLO, XHI, YLO, YHI), thermal="adiabatic",
          T_wall=None) -> dict:
    """Turn the listed faces into no-slip walls with the given thermal
    condition."""
    d = dict(d)
    ff, ft, tw = list(d["face_flow"]), list(d["face_thermal"]), list(d["T_wall"])
    for k in which:
        ff[k] = "wall"
        ft[k] = thermal
        if T_wall is not None:
            tw[k] = float(T_wall if np.isscalar(T_wall) else T_wall[k])
    d["face_flow"], d["face_thermal"], d["T_wall"] = ff, ft, tw
    return d


def particle(x, y, radius, rho_s=1.0, T_init=0.0, ux=0.0, uy=0.0, omega=0.0,
             theta=0.0, fixed=False, hold_T=False, radius_minor=0.0) -> dict:
    """A disk of the given radius, or (radius_minor in (0, radius)) an
    ellipse of semi-axes radius and radius_minor whose major axis makes the
    angle theta with the x axis."""
    return dict(x=float(x), y=float(y), theta=float(theta), ux=float(ux),
                uy=float(uy), omega=float(omega), radius=float(radius),
                rho_s=float(rho_s), T_init=float(T_init), fixed=int(bool(fixed)),
                hold_T=int(bool(hold_T)), radius_minor=float(radius_minor))


def collision_params(rho_r: float, radius: float, g: float, zeta=2.0,
                     eps_p=0.01) -> dict:
    """Repulsion constants of the short-range collision model (range zeta;
    force scale c = (rho_s - rho_f) pi R^2 |g| divided by eps_p between
    particles and by eps_w = eps_p / 2 against walls)."""
    c = (rho_r - 1.0) * math.pi * radius * radius * abs(g)
    return dict(coll_range=float(zeta), coll_stiff_pp=c / eps_p,
                coll_stiff_pw=c / (0.5 * eps_p))


def beta_from_grashof(Gr, g, dT, D, nu):
    """Gr = |g| beta dT D^3 / nu^2 (eq. nodim.paras) solved for beta."""
    return Gr * nu * nu / (abs(g) * dT * D ** 3)


def u_ref(rho_r, g, D):
    """U_ref = sqrt((rho_r - 1) |g| pi D / 2) (Sec. 3.3)."""
    return math.sqrt((rho_r - 1.0) * abs(g) * math.pi * D / 2.0)


# --------------------------------------------------------------------------
# The workloads


def c1_tiny() -> tuple[dict, list]:
    """128 x 64 channel, periodic in x, no-slip adiabatic walls in y; one
    fixed disk of diameter 16 at the centre at T = 0 in fluid at T = 1;
    tau_f = 0.8, Pr = 0.7, R_lambda = 10, R_cv = 2, body force 1e-6 along x.
    1000 steps."""
    tau_f, Pr = 0.8, 0.7
    nu = viscosity(tau_f)
    d = domain(128, 64, tau_f=tau_f, lambda_f=nu / Pr, R_lambda=10.0,
               R_cv=2.0, body_force=(1e-6, 0.0), init_T=1.0)
    d = walls(d, (YLO, YHI), thermal="adiabatic")
    return d, [particle(64.0, 32.0, 8.0, rho_s=1.0, T_init=0.0, fixed=True)]


def c2_channel(nx=200, ny=4000) -> tuple[dict, list]:
    """One cold disk (D = 20, density ratio 1.5, T = 0) sedimenting from the
    top centre of a 200 x 4000 channel, walls on all sides held at T = 1,
    fluid at T = 1; tau_f = 0.53, Pr = 0.7, R_lambda = 10, R_cv = 2,
    |g| = 1e-5, Gr = 1000 (beta = 1.25), T_ref = 1."""
    tau_f, Pr, D, rho_r, g, Gr = 0.53, 0.7, 20.0, 1.5, 1e-5, 1000.0
    nu = viscosity(tau_f)
    d = domain(nx, ny, tau_f=tau_f, lambda_f=nu / Pr, R_lambda=10.0, R_cv=2.0,
               gravity=(0.0, -g), beta=beta_from_grashof(Gr, g, 1.0, D, nu),
               T_ref=1.0, init_T=1.0, **collision_params(rho_r, D / 2, g))
    d = walls(d, thermal="dirichlet", T_wall=1.0)
    p = particle(nx / 2.0, ny - 3.0 * D, D / 2, rho_s=rho_r, T_init=0.0)
    return d, [p]


def e5_held_channel(Gr, length_D=180, start_D=5, D=20.0) -> tuple[dict, list]:
    """The paper's sedimentation of one cold particle of fixed temperature
    (Sec. 3.3): a channel of width L = 4 D with walls held at T_h = 1, a disk
    of diameter D = 20 cells starting D / 2 left of the centre line (x =
    1.5 D) and held at T_c = 0, density ratio 1.00232, Re = 40.5, Pr = 0.7,
    the given Gr, tau_f = 0.53, R_lambda = R_cv = 1, T_ref = T_h.  The paper
    gives no channel length: length_D diameters here, the disk starting
    start_D diameters below the top.  U_ref = Re nu / D sets |g| and Gr
    sets beta, as for e6_cht_channel."""
    tau_f, Pr, rho_r, Re = 0.53, 0.7, 1.00232, 40.5
    nu = viscosity(tau_f)
    U = Re * nu / D
    g = U * U / ((rho_r - 1.0) * math.pi * D / 2.0)
    nx, ny = int(round(4 * D)), int(round(length_D * D))
    d = domain(nx, ny, tau_f=tau_f, lambda_f=nu / Pr, R_lambda=1.0,
               R_cv=1.0, gravity=(0.0, -g),
               beta=beta_from_grashof(Gr, g, 1.0, D, nu), T_ref=1.0,
               init_T=1.0, **collision_params(rho_r, D / 2, g))
    d = walls(d, thermal="dirichlet", T_wall=1.0)
    p = particle(1.5 * D, ny - start_D * D, D / 2, rho_s=rho_r, T_init=0.0,
                 hold_T=True)
    return d, [p]


def e4_ellipse_channel(tau_f=0.6, fluid_gravity=0, length_L=30, start_L=3,
                       theta=math.pi / 4) -> tuple[dict, list]:
    """The isothermal sedimentation of an ellipse (Sec. 3.2): semi-axes
    a = 0.05 cm and b = 0.025 cm in a channel of width L = 0.4 cm resolved
    by 104 cells (dx = 1/260 cm), so a = 13 and b = 6.5 cells;
    rho_s / rho_f = 1.1, nu = 0.01 cm^2/s, |g| = 980 cm/s^2.  tau_f fixes
    dt through nu = (tau_f - 1/2) dx^2 / (3 dt), and |g| = 980 dt^2 / dx in
    lattice units.  The channel is 30 L long with no-slip walls at both
    ends (the paper's top is a no-flow wall and its bottom an outflow that
    the particle does not reach); the ellipse starts on the centre line
    3 L below the top with its major axis at theta = pi/4.  Isothermal: no
    buoyancy.  fluid_gravity = 1 is situation II (the fluid carries its
    weight, from a hydrostatic start)."""
    L, a, b = 104, 13.0, 6.5
    dx = 0.4 / L
    dt = (tau_f - 0.5) / 3.0 * dx * dx / 0.01
    g = 980.0 * dt * dt / dx
    ny = int(length_L * L)
    d = domain(L, ny, tau_f=tau_f, lambda_f=0.1, gravity=(0.0, -g),
               fluid_gravity=fluid_gravity, init_T=1.0, T_ref=1.0,
               **collision_params(1.1, a, g))
    d = walls(d, thermal="adiabatic")
    p = particle(L / 2.0, ny - start_L * L, a, radius_minor=b, theta=theta,
                 rho_s=1.1, T_init=1.0)
    return d, [p]


def e6_cht_channel(R_lambda=1.0, R_cv=1.0, length_D=60, start_D=10,
                   D=20.0) -> tuple[dict, list]:
    """The paper's sedimentation of one cold particle with conjugate heat
    transfer (Sec. 3.3 and the section after it): a channel of width 4 D
    with walls held at T_h = 1, a disk of diameter D = 20 cells starting on
    the centre line at T_c = 0 in fluid at T_h, density ratio 1.00232,
    Re = 10.5, Pr = 0.7, Gr = 1000, tau_f = 0.53, T_ref = T_h.  The paper
    gives no channel length: length_D diameters here, the disk starting
    start_D diameters below the top.  U_ref = Re nu / D sets |g| through
    U_ref = sqrt((rho_r - 1) |g| pi D / 2) and Gr sets beta."""
    tau_f, Pr, rho_r, Re, Gr = 0.53, 0.7, 1.00232, 10.5, 1000.0
    nu = viscosity(tau_f)
    U = Re * nu / D
    g = U * U / ((rho_r - 1.0) * math.pi * D / 2.0)
    nx, ny = int(round(4 * D)), int(round(length_D * D))
    d = domain(nx, ny, tau_f=tau_f, lambda_f=nu / Pr, R_lambda=R_lambda,
               R_cv=R_cv, gravity=(0.0, -g),
               beta=beta_from_grashof(Gr, g, 1.0, D, nu), T_ref=1.0,
               init_T=1.0, **collision_params(rho_r, D / 2, g))
    d = walls(d, thermal="dirichlet", T_wall=1.0)
    p = particle(nx / 2.0, ny - start_D * D, D / 2, rho_s=rho_r, T_init=0.0)
    return d, [p]


def e7_cht_cavity(L=1700, D=24.0, rows=32, cols=64, gap=2.0, left=19.0,
                  top=18.0) -> tuple[dict, list]:
    """The paper's sedimentation of 2048 cold particles with conjugate heat
    transfer in a square cavity (its last application section): L = 1700
    cells, adiabatic no-slip walls, disks of diameter D = 24 in 32 rows and
    64 columns with gaps of 2 cells, 19 cells from the left wall and 18 from
    the top; particles at T_c = 0 in fluid at T_h = 1 = T_ref; density ratio
    1.5, Re = 40.5, Pr = 0.71, Gr = 100, R_lambda = 1, R_cv = 2,
    tau_f = 0.55 and sigma_e = sigma_eps = 1 (the choice made there for
    stability)."""
    tau_f, Pr, rho_r, Re, Gr = 0.55, 0.71, 1.5, 40.5, 100.0
    nu = viscosity(tau_f)
    U = Re * nu / D
    g = U * U / ((rho_r - 1.0) * math.pi * D / 2.0)
    d = domain(L, L, tau_f=tau_f, lambda_f=nu / Pr, R_lambda=1.0, R_cv=2.0,
               gravity=(0.0, -g), beta=beta_from_grashof(Gr, g, 1.0, D, nu),
               T_ref=1.0, init_T=1.0, sigma_rule=1,
               **collision_params(rho_r, D / 2, g))
    d = walls(d, thermal="adiabatic")
    ps = []
    for i in range(rows):
        y = L - top - D / 2 - i * (D + gap)
        for j in range(cols):
            x = left + D / 2 + j * (D + gap)
            ps.append(particle(x, y, D / 2, rho_s=rho_r, T_init=0.0))
    return d, ps


def rsa_disks(n, radius, box, gap, seed, max_tries=5_000_000):
    """Random sequential addition of n equal disks in box = (x0, y0, x1, y1)
    keeping a surface gap >= gap between disks and from the box edges."""
    rng = np.random.default_rng(seed)
    x0, y0, x1, y1 = box
    lo_x, hi_x = x0 + radius + gap, x1 - radius - gap
    lo_y, hi_y = y0 + radius + gap, y1 - radius - gap
    min_d2 = (2 * radius + gap) ** 2
    cell = 2 * radius + gap
    grid: dict = {}
    pts = []
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not finish")
        px = rng.uniform(lo_x, hi_x)
        py = rng.uniform(lo_y, hi_y)
        gx, gy = int(px // cell), int(py // cell)
        ok = True
        for ix in (gx - 1, gx, gx + 1):
            for iy in (gy - 1, gy, gy + 1):
                for k in grid.get((ix, iy), ()):
                    qx, qy = pts[k]
                    if (qx - px) ** 2 + (qy - py) ** 2 < min_d2:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            grid.setdefault((gx, gy), []).append(len(pts))
            pts.append((px, py))
    return np.asarray(pts)


def c3_dense(n=2048, L=1536, D=16.0, seed=1) -> tuple[dict, list]:
    """2048 cold disks (D = 16, density ratio 1.5, T = 0) placed by seeded
    random sequential addition in the upper half of a 1536^2 cavity (surface
    gaps >= 2 cells), fluid at T = 1; bottom wall at T = 1, top at T = 0,
    adiabatic sides; tau_f = 0.55, Pr = 0.71, R_lambda = 10, R_cv = 2,
    |g| = 1e-5, Gr = 100, sigma_e = 1 (the dense-case choice of Sec. 3.5)."""
    tau_f, Pr, rho_r, g, Gr = 0.55, 0.71, 1.5, 1e-5, 100.0
    nu = viscosity(tau_f)
    d = domain(L, L, tau_f=tau_f, lambda_f=nu / Pr, R_lambda=10.0, R_cv=2.0,
               gravity=(0.0, -g), beta=beta_from_grashof(Gr, g, 1.0, D, nu),
               T_ref=1.0, init_T=1.0, sigma_rule=1,
               **collision_params(rho_r, D / 2, g))
    d = walls(d, (XLO, XHI), thermal="adiabatic")
    d = walls(d, (YLO, YHI), thermal="dirichlet", T_wall=[0, 0, 1.0, 0.0])
    pts = rsa_disks(n, D / 2, (0.0, L / 2.0, float(L), float(L)), 2.0, seed)
    ps = [particle(x, y, D / 2, rho_s=rho_r, T_init=0.0) for x, y in pts]
    return d, ps


def c5_batch(ncases=256, seed=2) -> list[tuple[dict, list]]:
    """Independent single-particle sedimentation cases of uneven size:
    W ~ U{64..256}, H ~ U{256..2048}, D ~ U(8, 24), density ratio
    U(1.1, 2.0), R_lambda log-uniform(0.1, 100), R_cv U(0.5, 4); walls as in
    the channel case; tau_f = 0.53, Pr = 0.7, |g| = 1e-5, Gr = 1000."""
    rng = np.random.default_rng(seed)
    tau_f, Pr, g, Gr = 0.53, 0.7, 1e-5, 1000.0
    nu = viscosity(tau_f)
    cases = []
    for _ in range(ncases):
        W = int(rng.integers(64, 257))
        H = int(rng.integers(256, 2049))
        D = float(rng.uniform(8.0, 24.0))
        rho_r = float(rng.uniform(1.1, 2.0))
        R_lam = float(10 ** rng.uniform(-1.0, 2.0))
        R_cv = float(rng.uniform(0.5, 4.0))
        d = domain(W, H, tau_f=tau_f, lambda_f=nu / Pr, R_lambda=R_lam,
                   R_cv=R_cv, gravity=(0.0, -g),
                   beta=beta_from_grashof(Gr, g, 1.0, D, nu), T_ref=1.0,
                   init_T=1.0, **collision_params(rho_r, D / 2, g))
        d = walls(d, thermal="dirichlet", T_wall=1.0)
        y0 = min(H - 3.0 * D, H - D / 2 - 4.0)
        cases.append((d, [particle(W / 2.0, y0, D / 2, rho_s=rho_r,
                                   T_init=0.0)]))
    return cases


WORKLOADS = {
    "c1_tiny": c1_tiny,
    "c2_channel": c2_channel,
    "c3_dense": c3_dense,
}


# --------------------------------------------------------------------------
# Three dimensions (D3Q19 flow, D3Q7 energy, spheres)

ZLO, ZHI = 4, 5


def domain3(nx: int, ny: int, nz: int, **kw) -> dict:
    """A three-dimensional descriptor with defaults: periodic box,
    tau_f = 0.8, unit fluid properties, no forces, fluid at rest at
    T = 1."""
    d = dict(
        nx=int(nx), ny=int(ny), nz=int(nz),
        face_flow=["periodic"] * 6,
        u_wall=[(0.0, 0.0, 0.0)] * 6,
        face_thermal=["adiabatic"] * 6,
        T_wall=[0.0] * 6,
        tau_f=0.8, rho_f=1.0, cv_f=1.0, lambda_f=0.1,
        R_lambda=1.0, R_cv=1.0,
        body_force=(0.0, 0.0, 0.0), gravity=(0.0, 0.0, 0.0), beta=0.0,
        T_ref=1.0, sigma_rule=0,
        coll_range=0.0, coll_stiff_pp=0.0, coll_stiff_pw=0.0,
        init_rho=1.0, init_u=(0.0, 0.0, 0.0), init_T=1.0,
        kmax=4,
    )
    for k, v in kw.items():
        if k not in d:
            raise KeyError(f"unknown descriptor key {k!r}")
        d[k] = v
    d["face_flow"] = list(d["face_flow"])
    d["u_wall"] = [tuple(map(float, u)) for u in d["u_wall"]]
    d["face_thermal"] = list(d["face_thermal"])
    d["T_wall"] = [float(t) for t in d["T_wall"]]
    return d


def walls3(d: dict, which=(XLO, XHI, YLO, YHI, ZLO, ZHI),
           thermal="adiabatic", T_wall=None) -> dict:
    """Turn the listed faces of a three-dimensional descriptor into no-slip
    walls with the given thermal condition."""
    d = dict(d)
    ff, ft, tw = list(d["face_flow"]), list(d["face_thermal"]), list(d["T_wall"])
    for k in which:
        ff[k] = "wall"
        ft[k] = thermal
        if T_wall is not None:
            tw[k] = float(T_wall if np.isscalar(T_wall) else T_wall[k])
    d["face_flow"], d["face_thermal"], d["T_wall"] = ff, ft, tw
    return d


def sphere(x, y, z, radius, rho_s=1.0, T_init=0.0, u=(0.0, 0.0, 0.0),
           omega=(0.0, 0.0, 0.0), fixed=False) -> dict:
    return dict(x=float(x), y=float(y), z=float(z), ux=float(u[0]),
                uy=float(u[1]), uz=float(u[2]), ox=float(omega[0]),
                oy=float(omega[1]), oz=float(omega[2]), radius=float(radius),
                rho_s=float(rho_s), T_init=float(T_init),
                fixed=int(bool(fixed)))


def c6_sphere_channel3(nx=80, ny=80, nz=320, D=16.0) -> tuple[dict, list]:
    """The channel's sedimentation in three dimensions: one cold sphere
    (D = 16, density ratio 1.5, T = 0) settling along z from near the top
    of an 80 x 80 x 320 box (5 D wide, 20 D long), walls on all faces held
    at T = 1, fluid at T = 1; tau_f = 0.53, Pr = 0.7, R_lambda = 10,
    R_cv = 2, |g| = 1e-5, Gr = 1000, the repulsion of the channel case."""
    tau_f, Pr, rho_r, g, Gr = 0.53, 0.7, 1.5, 1e-5, 1000.0
    nu = viscosity(tau_f)
    cp = collision_params(rho_r, D / 2, g)
    d = domain3(nx, ny, nz, tau_f=tau_f, lambda_f=nu / Pr, R_lambda=10.0,
                R_cv=2.0, gravity=(0.0, 0.0, -g),
                beta=beta_from_grashof(Gr, g, 1.0, D, nu), T_ref=1.0,
                init_T=1.0, **cp)
    d = walls3(d, thermal="dirichlet", T_wall=1.0)
    s = sphere(nx / 2.0, ny / 2.0, nz - 2.0 * D, D / 2, rho_s=rho_r,
               T_init=0.0)
    return d, [s]


def c7_spheres_box3(n=64, L=96, D=12.0, seed=3) -> tuple[dict, list]:
    """64 cold spheres (D = 12, density ratio 1.5, T = 0) placed by seeded
    random sequential addition in the upper half of a 96^3 box with
    adiabatic walls, fluid at T = 1; tau_f = 0.55, Pr = 0.71,
    R_lambda = 10, R_cv = 2, |g| = 1e-5, Gr = 100 (the dense cavity's
    parameters in three dimensions)."""
    tau_f, Pr, rho_r, g, Gr = 0.55, 0.71, 1.5, 1e-5, 100.0
    nu = viscosity(tau_f)
    d = domain3(L, L, L, tau_f=tau_f, lambda_f=nu / Pr, R_lambda=10.0,
                R_cv=2.0, gravity=(0.0, 0.0, -g),
                beta=beta_from_grashof(Gr, g, 1.0, D, nu), T_ref=1.0,
                init_T=1.0, sigma_rule=1, **collision_params(rho_r, D / 2, g))
    d = walls3(d, thermal="adiabatic")
    rng = np.random.default_rng(seed)
    R, gap, pts = D / 2, 2.0, []
    lo = np.array([R + gap, R + gap, L / 2 + R + gap])
    hi = np.array([L - R - gap, L - R - gap, L - R - gap])
    while len(pts) < n:
        p = rng.uniform(lo, hi)
        if all(np.linalg.norm(p - q) >= D + gap for q in pts):
            pts.append(p)
    return d, [sphere(*p, R, rho_s=rho_r, T_init=0.0) for p in pts]
