"""GPU parity of the three-dimensional path (D3Q19 flow, D3Q7 energy,
spheres; through the vlb3_* C ABI) against the FP64 oracle: every
population and field element by element, and the sphere states, forces,
torques and thermal outputs, on ragged domains (not multiples of the
256-cell tile) with periodic faces and with walls.

Bars (FP64): populations and fields within 1e-12 of their scale (the
field's largest magnitude, velocity components the largest speed but at
least 1e-3, f_s and [df_s/dt] 1);
sphere positions and velocities within 1e-12 relative; forces and torques
within 1e-12 of the populations that enter them (the oracle's F_abs); f_s
within 1e-13 (the two volume rules differ by about 1e-15 per cell).
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "ux", "uy", "uz", "T", "fs", "dfs")
# The smallest speed scale.  A momentum sum of 19 populations of order 1/3
# carries an absolute rounding floor of a few 1e-16, and the two sides
# compute the collision in different but equal forms (the GPU relaxes the
# moments of f - f^eq and adds the change, the oracle transforms f, f^eq
# and the force term separately and back): a velocity component that is
# zero but for rounding differs by about 2e-16, which is 1e-12 of 2e-4.
U_FLOOR = 1e-3


@pytest.fixture(scope="module")
def vlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_23802_amd import vlb as v
    v.lib()
    return v


def say(msg):
    print(msg, flush=True)


def compare(o, g, steps, tol=1e-12, fs_tol=1e-13):
    """Largest error of every population set and field over its scale."""
    errs = {}
    for name in ("f", "g"):
        a, b = g.populations(name), o.field(name)
        errs[name] = float(np.abs(a - b).max() / np.abs(b).max())
    speed = max(float(np.sqrt(o.field("ux") ** 2 + o.field("uy") ** 2 +
                              o.field("uz") ** 2).max()), U_FLOOR)
    for name in FIELDS:
        a, b = g.field(name), o.field(name if name != "dfs" else "d")
        # velocity components on the speed's scale; f_s is a fraction and
        # [df_s/dt] its rate, both on the scale 1
        scale = (speed if name in ("ux", "uy", "uz") else
                 1.0 if name in ("fs", "dfs") else
                 max(float(np.abs(b).max()), 1e-300))
        errs[name] = float(np.abs(a - b).max() / scale)
    say(f"  after {steps} steps: " + ", ".join(f"{k} {v:.1e}" for k, v in
                                                 errs.items()))
    for k, v in errs.items():
        assert v < (fs_tol if k == "fs" else tol), (steps, k, v)
    return errs


def compare_spheres(o, g, tol=1e-12):
    """Positions over the diameter, velocities over the largest sphere
    speed (at least U_FLOOR), spins over that speed over the radius, forces
    and torques over the populations that enter their sums (F_abs, times
    the radius for torques), the thermal outputs over their size (at
    least 1)."""
    po, pg = o.particles(), g.particles()
    Umax = max(float(np.sqrt(po["ux"] ** 2 + po["uy"] ** 2 +
                             po["uz"] ** 2).max()), U_FLOOR)
    for k in range(len(po)):
        R = g.spheres[k]["radius"]
        scales = {"x": 2 * R, "y": 2 * R, "z": 2 * R, "ux": Umax, "uy": Umax,
                  "uz": Umax, "ox": Umax / R, "oy": Umax / R, "oz": Umax / R,
                  "Fx": po["F_abs"][k], "Fy": po["F_abs"][k],
                  "Fz": po["F_abs"][k], "Tx": po["F_abs"][k] * R,
                  "Ty": po["F_abs"][k] * R, "Tz": po["F_abs"][k] * R}
        for key in ("T_mean", "T_min", "E_solid", "fs_sum"):
            scales[key] = max(1.0, abs(po[key][k]))
        for key, sc in scales.items():
            err = abs(pg[key][k] - po[key][k])
            assert err < tol * sc, (k, key, err, sc)


def box_case():
    """Periodic 21 x 19 x 17 box (6783 cells, a ragged last tile), two
    moving, spinning spheres of different density, temperature and radius,
    gravity with buoyancy, a body force and repulsion."""
    d = W.domain3(21, 19, 17, tau_f=0.7, lambda_f=0.05, R_lambda=3.0,
                  R_cv=2.0, init_T=0.6, gravity=(0.0, 0.0, -2e-5), beta=0.3,
                  T_ref=0.5, body_force=(1e-6, 0.0, 0.0), coll_range=1.5,
                  coll_stiff_pp=1e-4)
    ps = [W.sphere(6.3, 7.1, 8.2, 3.4, rho_s=1.5, T_init=0.1,
                   u=(0.01, 0.004, -0.006), omega=(0.002, -0.003, 0.004)),
          W.sphere(14.2, 11.7, 7.4, 2.6, rho_s=0.8, T_init=0.9,
                   u=(-0.008, 0.005, 0.007), omega=(-0.004, 0.001, 0.002))]
    return d, ps


def wall_case():
    """Walls on all six faces (a moving lid at z, Dirichlet and adiabatic
    faces), a sphere close to a wall (repulsion), one across the periodic
    seam is not possible here, so the second sits near a corner."""
    d = W.domain3(23, 18, 26, tau_f=0.62, lambda_f=0.04, R_lambda=0.3,
                  R_cv=0.7, gravity=(0.0, 0.0, -3e-5), beta=0.2, T_ref=0.3,
                  init_T=0.3, sigma_rule=1, coll_range=1.5,
                  coll_stiff_pp=1e-4, coll_stiff_pw=2e-4)
    d = W.walls3(d, thermal="dirichlet", T_wall=[0.2, 0.7, 0.4, 0.9, 1.0,
                                                  0.0])
    d["face_thermal"][0] = "adiabatic"
    d["u_wall"][W.ZHI] = (0.02, -0.01, 0.0)
    ps = [W.sphere(11.6, 9.2, 4.1, 3.3, rho_s=1.8, T_init=0.0,
                   u=(0.004, 0.0, -0.003)),
          W.sphere(5.2, 4.9, 20.3, 3.9, rho_s=0.7, T_init=1.0,
                   u=(-0.003, 0.002, 0.004), omega=(0.001, 0.002, -0.003))]
    return d, ps


def seam_case():
    """A sphere straddling the periodic seams in x and z (its cells are
    reached through the nearest copies)."""
    d = W.domain3(20, 17, 22, tau_f=0.8, lambda_f=0.06, R_lambda=2.0,
                  R_cv=1.5, init_T=0.4)
    ps = [W.sphere(0.7, 8.4, 21.2, 4.2, rho_s=1.3, T_init=1.0,
                   u=(-0.006, 0.003, 0.008), omega=(0.003, 0.0, -0.002))]
    return d, ps


@pytest.mark.parametrize("make", [box_case, wall_case, seam_case],
                         ids=["box", "walls", "seam"])
def test_gpu3_matches_oracle_fp64(vlb, oracle3_mod, make):
    d, ps = make()
    say(f"3-D {make.__name__}: {d['nx']} x {d['ny']} x {d['nz']}, "
        f"{len(ps)} spheres")
    o = oracle3_mod.Oracle3(d, ps).init()
    g = vlb.Domain3(d, ps).init()
    compare(o, g, 0)
    done = 0
    for n in (1, 1, 3, 5):
        o.step(n)
        g.step(n)
        done += n
        compare(o, g, done)
        compare_spheres(o, g)
    g.close()


def test_gpu3_large_sphere_volumes(vlb, oracle3_mod):
    """The solid fraction of spheres of radius 12 and 0.7 at init: the GPU's
    adaptive Gauss-Legendre over z against the oracle's tanh-sinh rule."""
    d = W.domain3(40, 33, 30)
    ps = [W.sphere(19.37, 16.21, 14.83, 12.0),
          W.sphere(36.5, 30.2, 27.9, 0.7)]
    o = oracle3_mod.Oracle3(d, ps).init()
    g = vlb.Domain3(d, ps).init()
    err = float(np.abs(g.field("fs") - o.field("fs")).max())
    say(f"fs at R = 12 and 0.7: {err:.1e}")
    assert err < 1e-13
    p = g.particles()
    assert abs(p["fs_sum"][0] - 4 / 3 * math.pi * 12 ** 3) < 1e-9
    g.close()


def test_gpu3_no_spheres_channel(vlb, oracle3_mod):
    """Force-driven flow between plates with a Dirichlet temperature
    difference and buoyancy, no spheres."""
    d = W.walls3(W.domain3(5, 7, 20, tau_f=0.9, body_force=(2e-6, 0.0, 0.0),
                           gravity=(0.0, 0.0, -1e-4), beta=0.5, T_ref=0.5),
                 (W.ZLO, W.ZHI), thermal="dirichlet",
                 T_wall=[0, 0, 0, 0, 1.0, 0.0])
    o = oracle3_mod.Oracle3(d, []).init()
    g = vlb.Domain3(d, []).init()
    for n in (1, 50):
        o.step(n)
        g.step(n)
        compare(o, g, n)
    g.close()


@pytest.mark.parametrize("name", ["c6_sphere_channel3", "c7_spheres_box3"])
def test_gpu3_full_size_matches_oracle(vlb, oracle3_mod, name):
    """The benchmarked workloads at full size (80 x 80 x 320 with one
    sphere; 96^3 with 64 spheres), element by element over three steps."""
    d, ps = getattr(W, name)()
    say(f"3-D {name}: {d['nx']} x {d['ny']} x {d['nz']}, {len(ps)} spheres")
    o = oracle3_mod.Oracle3(d, ps).init()
    g = vlb.Domain3(d, ps).init()
    done = 0
    for n in (1, 2):
        o.step(n)
        g.step(n)
        done += n
        compare(o, g, done)
        compare_spheres(o, g)
    g.close()


def test_gpu3_many_subintervals(vlb, oracle3_mod):
    """A sphere whose centre lies within 1e-7 of two lattice planes: its
    cells' section areas change form at clustered heights, so the
    quadrature grades towards them and some cells take up to 89
    sub-intervals (more than one pass of the exact-volume kernel's lists).
    The solid fraction after the step (the step's own geometry pass) and
    at init against the oracle; the sphere stays put, a second one moves."""
    d = W.domain3(21, 21, 22, tau_f=0.7, init_T=0.5)
    ps = [W.sphere(10.0000001, 10.0000001, 10.67475352631797,
                   8.705915644655517, rho_s=1.2, T_init=0.2, fixed=True),
          W.sphere(2.4, 18.3, 3.1, 1.6, u=(0.004, -0.002, 0.003))]
    o = oracle3_mod.Oracle3(d, ps).init()
    g = vlb.Domain3(d, ps).init()
    err0 = float(np.abs(g.field("fs") - o.field("fs")).max())
    for n in (1, 1):
        o.step(n)
        g.step(n)
    err = float(np.abs(g.field("fs") - o.field("fs")).max())
    say(f"clustered singular heights: fs at init {err0:.1e}, after 2 steps "
        f"{err:.1e}")
    assert err0 < 1e-13 and err < 1e-13
    compare(o, g, 2)
    g.close()


def test_gpu3_bit_for_bit_repeatable(vlb):
    """The 64-sphere box twice from the same start: populations, fields and
    sphere states agree bit for bit (every reduction, the exact-volume sums
    included, runs in a fixed order whatever the order in which the cells
    were listed)."""
    d, ps = W.c7_spheres_box3()
    out = []
    for _ in range(2):
        g = vlb.Domain3(d, ps).init()
        g.step(4)
        out.append(([g.populations(n) for n in ("f", "g")] +
                    [g.field(n) for n in FIELDS],
                    g.particles()))
        g.close()
    (a, pa), (b, pb) = out
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    for key in pa.dtype.names:
        assert np.array_equal(pa[key], pb[key]), key


FP32_BAR = 1e-6


@pytest.mark.parametrize("make", [box_case, wall_case], ids=["box", "walls"])
def test_gpu3_fp32_storage_against_oracle(vlb, oracle3_mod, make):
    """The FP32 storage form (populations and carrier in FP32, the
    populations as deviations from the equilibria of the state at rest,
    FP64 arithmetic) against the FP64 oracle over ten steps.  Each stored
    value is rounded to 24 bits once a step: the populations' deviations
    (up to about 0.1 in g) by a few 1e-9, the carrier h = 2 f_s + d, of
    order one, by about 6e-8 (the d recursion keeps every such rounding).
    Measured after ten steps: f up to 8e-10, g 1.3e-7, velocities 2.2e-8,
    T 5e-8, [df_s/dt] 4.4e-7 of their scales, f_s 1.8e-10 (the spheres
    move under slightly different forces); all held to 1e-6, sphere states
    too.  The
    GPU's FP64 form is held to 1e-12 by the cases above."""
    d, ps = make()
    o = oracle3_mod.Oracle3(d, ps).init()
    g = vlb.Domain3(d, ps, precision="fp32").init()
    done = 0
    for n in (1, 9):
        o.step(n)
        g.step(n)
        done += n
        compare(o, g, done, tol=FP32_BAR, fs_tol=FP32_BAR)
        compare_spheres(o, g, tol=FP32_BAR)
    g.close()


def test_gpu3_fp32_storage_rest_state(vlb):
    """A walled box at rest at the reference density and temperature, no
    spheres: the FP32 deviations are zero (to the rounding of the
    reference itself), so the FP32 form keeps the FP64 form's state."""
    d = W.walls3(W.domain3(17, 13, 11, init_T=0.7))
    out = {}
    for prec in ("fp64", "fp32"):
        g = vlb.Domain3(d, [], precision=prec).init()
        g.step(5)
        out[prec] = [g.field(n) for n in FIELDS]
        g.close()
    for a, b in zip(out["fp64"], out["fp32"]):
        assert np.abs(a - b).max() <= 1e-15 * max(1.0, np.abs(a).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gpu3_checkpoint_continues_bit_for_bit(vlb, prec):
    """Save after three steps of the walled two-sphere case, step four more;
    load the checkpoint into a fresh context and step the same four: every
    population, field and sphere state agrees bit for bit, and so does the
    step count.  A checkpoint of another shape is refused."""
    d, ps = wall_case()
    a = vlb.Domain3(d, ps, precision=prec).init()
    a.step(3)
    ck = a.save()
    a.step(4)
    b = vlb.Domain3(d, ps, precision=prec).init()
    b.load(ck)
    b.step(4)
    for n in ("f", "g"):
        assert np.array_equal(a.populations(n), b.populations(n)), n
    for n in FIELDS:
        assert np.array_equal(a.field(n), b.field(n)), n
    pa, pb = a.particles(), b.particles()
    for key in pa.dtype.names:
        assert np.array_equal(pa[key], pb[key]), key
    assert (vlb.lib().vlb3_step_count(a.h) == vlb.lib().vlb3_step_count(b.h)
            == 7)
    c = vlb.Domain3(W.domain3(9, 9, 9), [], precision=prec).init()
    with pytest.raises(Exception):
        c.load(ck)
    for dom in (a, b, c):
        dom.close()
