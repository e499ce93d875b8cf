"""Pins of the oracle's rotational coupling and of the per-particle thermal
outputs, against what the mathematics fixes:

- the first steps of a spinning, translating disk in closed form: the
  streamed state of the equilibrium start is a periodic shift of textbook
  D2Q9 equilibria, so the momentum-exchange force and torque of step 1
  follow from f_s (rho* u_s - j*) with u_s = U + Omega z x (x - X) (eq. us,
  Sec. 2.3), and the next velocities from eq. particle with I = M R^2 / 2
  and the inside-fluid terms of eq. inside.fluid;
- the angular-momentum budget of a periodic box: streaming moves every
  population along its own velocity (e x e = 0), the collision keeps each
  cell's momentum, and the volumetric step hands the fluid minus each
  particle's torque and the moment of its force about any fixed point;
- T_mean, T_min and E_solid (the particle temperature outputs; the paper
  reports the minimal temperature inside the particle, Sec. 3.4) in closed
  form at the equilibrium start and for a uniform temperature.
"""
import math

import numpy as np
import pytest

import workloads as W

E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1),
              (-1, -1), (1, -1)], dtype=float)
WGT = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def textbook_feq(rho, ux, uy):
    """Second-order D2Q9 equilibria on whole fields, shape (9, ny, nx)."""
    eu = E[:, 0, None, None] * ux + E[:, 1, None, None] * uy
    u2 = ux * ux + uy * uy
    return WGT[:, None, None] * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * u2)


def stream_periodic(f):
    """Pull streaming on a periodic grid: f*_i(x) = f_i(x - e_i)."""
    return np.stack([np.roll(f[q], (int(E[q, 1]), int(E[q, 0])), axis=(0, 1))
                     for q in range(9)])


def nodes(nx, ny):
    return np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)


def exchange(fs, fst, X, Y, U, V, Om):
    """Force and torque on a disk (centre X, Y, velocity U, V, angular
    velocity Om) from the streamed populations fst and its cover fs:
    minus the sums of f_s (rho* u_s - j*) and of its moment about the
    centre."""
    ny, nx = fs.shape
    xn, yn = nodes(nx, ny)
    rx, ry = xn - X, yn - Y
    usx, usy = U - Om * ry, V + Om * rx
    rho = fst.sum(axis=0)
    jx = (E[:, 0, None, None] * fst).sum(axis=0)
    jy = (E[:, 1, None, None] * fst).sum(axis=0)
    dpx, dpy = fs * (rho * usx - jx), fs * (rho * usy - jy)
    return -dpx.sum(), -dpy.sum(), -(rx * dpy - ry * dpx).sum(), \
        (np.abs(dpx) + np.abs(dpy)).sum()


@pytest.mark.parametrize("Rb", [0.0, 3.9])
def test_spinning_disk_first_steps_closed_form(oracle_mod, Rb):
    """A disk (or an ellipse of semi-axes R and Rb, Sec. 3.2) released
    spinning and translating in fluid at rest (no gravity, no fluid force).
    Step 1: the forces of the start are zero and U^{-1} = U^0, so U^1 = U^0,
    Omega^1 = Omega^0, X^1 = X^0 + U^0, theta^1 = theta^0 + Omega^0; the
    momentum exchange of step 1 is that of the streamed equilibrium start.
    Step 2: U^2 = U^1 + F^1 / M, Omega^2 = Omega^1 + T^1 / I with
    V = pi R Rb, I = M R^2 / 2 for a disk and M (R^2 + Rb^2) / 4 for an
    ellipse (the inside-fluid terms vanish, U^1 = U^0).  Step 3: the
    inside-fluid terms of eq. inside.fluid enter with M_in = rho_f V and
    I_in = (rho_f / rho_s) I."""
    O = oracle_mod
    nx, ny, R, rho_s = 48, 44, 7.3, 1.6
    X0, Y0, U0, V0, Om0, th0 = 23.7, 21.2, 0.012, -0.007, 0.004, 0.7
    d = W.domain(nx, ny, tau_f=0.7, R_cv=2.0, R_lambda=3.0)
    ps = [W.particle(X0, Y0, R, rho_s=rho_s, ux=U0, uy=V0, omega=Om0,
                     theta=th0, radius_minor=Rb)]
    Rb = Rb or R
    o = O.Oracle(d, ps).init()
    fs0 = o.field("fs")
    xn, yn = nodes(nx, ny)
    # the equilibrium start: fluid at rest, the disk's cells carry u_s
    ux0 = fs0 * (U0 - Om0 * (yn - Y0))
    uy0 = fs0 * (V0 + Om0 * (xn - X0))
    f0 = textbook_feq(1.0, ux0, uy0)
    assert np.abs(o.field("f") - f0).max() < 1e-15

    o.step(1)
    p1 = o.particles()[0]
    X1, Y1 = X0 + U0, Y0 + V0
    assert p1["ux"] == U0 and p1["uy"] == V0 and p1["omega"] == Om0
    assert abs(p1["x"] - X1) < 1e-14 and abs(p1["y"] - Y1) < 1e-14
    assert p1["theta"] == th0 + Om0
    assert abs(p1["fs_sum"] - math.pi * R * Rb) < 1e-11
    Fx, Fy, Tz, Fabs = exchange(o.field("fs"), stream_periodic(f0), X1, Y1,
                                U0, V0, Om0)
    assert abs(Tz) > 1e-4 * Fabs * R      # the rotation is felt
    assert abs(p1["Fx"] - Fx) < 1e-14 * Fabs
    assert abs(p1["Fy"] - Fy) < 1e-14 * Fabs
    assert abs(p1["Tz"] - Tz) < 1e-14 * Fabs * R
    # the fluid opposes the spin
    assert Tz * Om0 < 0

    M = rho_s * math.pi * R * Rb
    I = 0.25 * M * (R * R + Rb * Rb)
    o.step(1)
    p2 = o.particles()[0]
    assert abs(p2["omega"] - (Om0 + Tz / I)) < 1e-17
    assert abs(p2["ux"] - (U0 + Fx / M)) < 1e-17
    assert abs(p2["uy"] - (V0 + Fy / M)) < 1e-17

    o.step(1)
    p3 = o.particles()[0]
    Min = 1.0 * math.pi * R * Rb
    Iin = I / rho_s
    Om3 = p2["omega"] + (p2["Tz"] + Iin * (p2["omega"] - Om0)) / I
    U3 = p2["ux"] + (p2["Fx"] + Min * (p2["ux"] - U0)) / M
    assert abs(p3["omega"] - Om3) < 1e-17
    assert abs(p3["ux"] - U3) < 1e-17


def test_angular_momentum_budget_periodic(oracle_mod):
    """Two free disks, spinning and moving, in a periodic box with no force
    on the fluid.  About any fixed point X0:
    L^{n+1} - L_streamed^n = -sum_p [T_p + (X_p - X0) x F_p],
    with L = sum_x (x - X0) x j (j = rho u, the force being zero) and
    L_streamed the same sum over the populations of step n shifted by
    their velocities (which carries the periodic wrap exactly)."""
    O = oracle_mod
    nx, ny = 50, 46
    d = W.domain(nx, ny, tau_f=0.66, R_cv=2.5, R_lambda=4.0)
    ps = [W.particle(16.4, 15.1, 6.2, rho_s=1.3, ux=0.015, uy=0.006,
                     omega=0.005),
          W.particle(34.2, 30.7, 5.1, rho_s=0.9, ux=-0.01, uy=0.012,
                     omega=-0.004)]
    o = O.Oracle(d, ps).init()
    o.step(2)
    xn, yn = nodes(nx, ny)
    X0, Y0 = 21.3, 19.8
    worst, scale = 0.0, 0.0
    for _ in range(25):
        fst = stream_periodic(o.field("f"))
        jx = (E[:, 0, None, None] * fst).sum(axis=0)
        jy = (E[:, 1, None, None] * fst).sum(axis=0)
        Ls = ((xn - X0) * jy - (yn - Y0) * jx).sum()
        o.step(1)
        rho = o.field("rho")
        jx1, jy1 = rho * o.field("ux"), rho * o.field("uy")
        L1 = ((xn - X0) * jy1 - (yn - Y0) * jx1).sum()
        p = o.particles()
        handed = -sum(p["Tz"][k] + (p["x"][k] - X0) * p["Fy"][k]
                      - (p["y"][k] - Y0) * p["Fx"][k] for k in range(2))
        worst = max(worst, abs((L1 - Ls) - handed))
        scale = max(scale, float(np.abs((xn - X0) * jy1).sum()))
        assert abs(handed) > 1e-6
    assert worst < 1e-15 * scale, (worst, scale)


def test_thermal_outputs_at_equilibrium_start(oracle_mod):
    """At n = 0 each cell holds the energy-weighted mixture
    T = [(1 - f_s) c_vf T_f + f_s c_vs T_p] / [(1 - f_s) c_vf + f_s c_vs];
    then T_mean = sum f_s T / sum f_s, E_solid = sum f_s c_vs T, and T_min
    over the cells wholly inside is T_p itself; sum f_s = pi R^2."""
    O = oracle_mod
    R, Rcv = 6.6, 3.0
    cvs = Rcv * 1.0
    # a cold disk in warm fluid, and a warm disk in cold fluid (its partly
    # covered cells are colder than its inside)
    for Tp, Tf in ((0.15, 0.9), (0.9, 0.15)):
        d = W.domain(40, 38, R_cv=Rcv, R_lambda=5.0, init_T=Tf)
        ps = [W.particle(19.4, 18.9, R, T_init=Tp)]
        o = O.Oracle(d, ps).init()
        fs = o.field("fs")
        T = ((1 - fs) * Tf + fs * cvs * Tp) / ((1 - fs) + fs * cvs)
        p = o.particles()[0]
        assert abs(p["fs_sum"] - math.pi * R * R) < 1e-12
        assert abs(p["T_mean"] - (fs * T).sum() / fs.sum()) < 1e-14
        assert abs(p["E_solid"] - (fs * cvs * T).sum()) < 1e-12
        assert p["T_min"] == Tp
    # a uniform temperature: T_mean = T_min = T0, E_solid = c_vs T0 pi R^2,
    # also after the disk has moved (the isothermal invariant of Appendix A)
    T0 = 0.55
    d = W.domain(40, 38, R_cv=Rcv, R_lambda=5.0, init_T=T0)
    ps = [W.particle(19.4, 18.9, R, T_init=T0, ux=0.02, uy=-0.01,
                     omega=0.003)]
    o = O.Oracle(d, ps).init().step(60)
    p = o.particles()[0]
    assert abs(p["T_mean"] - T0) < 1e-14
    assert abs(p["T_min"] - T0) < 1e-14
    assert abs(p["E_solid"] - cvs * T0 * math.pi * R * R) < 1e-11
