"""Pins of the oracle's lattice update against what the paper and the
mathematics fix: equilibria, conservation laws, the isothermal invariant of
Appendix A, Galilean co-motion, closed-form channel flows and the first steps
of a released particle.
"""
import math

import numpy as np
import pytest

import workloads as W

E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1),
              (-1, -1), (1, -1)], dtype=float)
WGT = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def textbook_feq(rho, u):
    """Second-order D2Q9 equilibrium (Qian, d'Humieres & Lallemand 1992)."""
    eu = E @ np.asarray(u)
    return WGT * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * float(np.dot(u, u)))


def mixed_box(nx=48, ny=40, **kw):
    d = W.domain(nx, ny, tau_f=0.7, lambda_f=0.05, R_lambda=7.0, R_cv=3.0,
                 **kw)
    ps = [W.particle(15.3, 14.2, 5.5, rho_s=1.7, T_init=0.2, ux=0.02,
                     uy=0.01, omega=0.003),
          W.particle(33.1, 27.7, 4.2, rho_s=0.8, T_init=0.9, ux=-0.03,
                     omega=-0.002)]
    return d, ps


# --------------------------------------------------------------------------
# P1: equilibria


def test_flow_equilibrium_is_textbook_d2q9(oracle_mod):
    """M^{-1} m^eq (m^eq of Sec. 2.1) equals the textbook D2Q9 equilibrium:
    the initial populations of a uniform state."""
    O = oracle_mod
    u = (0.037, -0.021)
    d = W.domain(8, 8, init_u=u, init_rho=1.013)
    f = O.Oracle(d, []).init().field("f")
    ref = textbook_feq(1.013, u)
    assert np.abs(f[:, 3, 5] - ref).max() < 1e-15


def test_energy_equilibrium_closed_form(oracle_mod):
    """M^{-1} n^eq with alpha1 = -2, alpha2 = 1 gives g_i = w_i c_ref T for
    i >= 1 and g_0 = eps - 5/9 c_ref T (worked out by hand from the printed
    M and n^eq)."""
    O = oracle_mod
    T, Rcv = 0.37, 2.5
    d = W.domain(8, 8, init_T=T, R_cv=Rcv)
    g = O.Oracle(d, []).init().field("g")[:, 2, 2]
    cref = 2 * 1.0 * Rcv / (1.0 + Rcv)
    assert np.abs(g[1:] - WGT[1:] * cref * T).max() < 1e-16
    assert abs(g[0] - (T - 5 / 9 * cref * T)) < 1e-15


def test_no_particle_rest_state_is_fixed_point(oracle_mod):
    """Degeneration (f_s = 0): a uniform rest state with uniform T stays
    exactly put."""
    O = oracle_mod
    d = W.walls(W.domain(20, 12, init_T=0.4), (2, 3), thermal="dirichlet",
                T_wall=0.4)
    o = O.Oracle(d, []).init()
    f0, g0 = o.field("f"), o.field("g")
    o.step(25)
    assert np.abs(o.field("f") - f0).max() < 1e-15
    assert np.abs(o.field("g") - g0).max() < 1e-15


# --------------------------------------------------------------------------
# P2 / P3 / P6: conservation


def test_mass_conserved_with_moving_particles(oracle_mod):
    """eq. fi keeps rho = sum f*_i in every cell, streaming and bounce-back
    move mass without loss, so total mass is constant."""
    O = oracle_mod
    d, ps = mixed_box()
    d = W.walls(d, (2, 3))
    o = O.Oracle(d, ps).init()
    m0 = o.field("rho").sum()
    o.step(120)
    assert abs(o.field("rho").sum() - m0) < 1e-13 * m0 * 120


def test_energy_budget_identity(oracle_mod):
    """With adiabatic or periodic boundaries the energy collision adds q_c to
    the zeroth moment and eps = sum g + q_c/2 (eq. e), hence
    sum eps^{n+1} - sum eps^n = (sum q^n + sum q^{n+1}) / 2 exactly."""
    O = oracle_mod
    d, ps = mixed_box(init_u=(0.01, 0.0))
    d = W.walls(d, (2, 3), thermal="adiabatic")
    o = O.Oracle(d, ps).init()
    worst = 0.0
    for _ in range(60):
        e0, q0 = o.field("eps").sum(), o.field("qc").sum()
        o.step(1)
        e1, q1 = o.field("eps").sum(), o.field("qc").sum()
        worst = max(worst, abs((e1 - e0) - 0.5 * (q0 + q1)))
    assert worst < 1e-11


def test_adiabatic_equilibrium_temperature(oracle_mod):
    """Fixed cold particles (T = 0) in hot fluid (T = 1) in an adiabatic box
    with R_cv = 2 relax to T_eq = sum eps_0 / sum c_v = (1 - phi)/(1 + phi),
    the energy-balance relation behind the printed T_eq of Sec. 3.5."""
    O = oracle_mod
    d = W.walls(W.domain(28, 28, R_cv=2.0, R_lambda=1.0, lambda_f=0.15,
                         init_T=1.0), thermal="adiabatic")
    ps = [W.particle(14.2, 13.7, 6.3, T_init=0.0, fixed=True)]
    o = O.Oracle(d, ps).init()
    phi = o.field("fs").sum() / (28 * 28)
    e0 = o.field("eps").sum()
    o.step(14000)
    # nothing moves, so q_c = 0 and sum eps is conserved up to round-off
    assert abs(o.field("eps").sum() - e0) < 1e-15 * e0 * 14000
    T = o.field("T")
    assert np.abs(T - (1 - phi) / (1 + phi)).max() < 1e-9


def test_momentum_budget_periodic(oracle_mod):
    """Periodic box with a uniform external force F_ext on the fluid share:
    collision adds F to j, streaming conserves it, and the volumetric step
    changes it by -sum_p F_MES,p, so
    sum j^{n+1} - sum j^n = sum F^n - sum_p F_MES,p^{n+1} with
    j = rho u - F/2 (eq. rho.rhou)."""
    O = oracle_mod
    Fext = np.array([2e-5, -1e-5])
    d, ps = mixed_box(body_force=tuple(Fext))
    o = O.Oracle(d, ps).init()
    o.step(3)

    def jsum_and_F():
        fs = o.field("fs")
        Fx = (1 - fs) * Fext[0]
        Fy = (1 - fs) * Fext[1]
        rho = o.field("rho")
        jx = rho * o.field("ux") - 0.5 * Fx
        jy = rho * o.field("uy") - 0.5 * Fy
        return np.array([jx.sum(), jy.sum()]), np.array([Fx.sum(), Fy.sum()])

    worst = 0.0
    for _ in range(20):
        j0, F0 = jsum_and_F()
        o.step(1)
        j1, _ = jsum_and_F()
        p = o.particles()
        Fmes = np.array([p["Fx"].sum(), p["Fy"].sum()])
        worst = max(worst, np.abs((j1 - j0) - (F0 - Fmes)).max())
    assert worst < 1e-13


# --------------------------------------------------------------------------
# P4: the isothermal invariant of Appendix A


def test_isothermal_invariant_2d_moving_particles(oracle_mod):
    """Appendix A: with beta1 = -4 and the [df_s/dt] recursion (eq. dfs_dt,
    eq. con.dfs) a uniform T0 stays exact at the moving interfaces for any
    c_vs != c_vf; here in 2-D with flow and two moving disks."""
    O = oracle_mod
    d, ps = mixed_box(init_T=0.7, init_u=(0.03, -0.01))
    for p in ps:
        p["T_init"] = 0.7
    o = O.Oracle(d, ps).init()
    o.step(150)
    assert np.abs(o.field("T") - 0.7).max() < 2e-14


@pytest.mark.parametrize("hook,name", [({"beta1": -2.0}, "beta1 = -2"),
                                       ({"dfs_backward": 1}, "backward dfs")])
def test_isothermal_invariant_negative_controls(oracle_mod, hook, name):
    """The two violations Appendix A warns about each produce a visible
    interface error (the mistake is planted in the oracle only)."""
    O = oracle_mod
    d, ps = mixed_box(init_T=0.7, init_u=(0.03, -0.01))
    for p in ps:
        p["T_init"] = 0.7
    o = O.Oracle(d, ps, hooks=hook).init()
    o.step(150)
    assert np.abs(o.field("T") - 0.7).max() > 1e-4, name


def test_isothermal_invariant_1d_moving_interface(oracle_mod):
    """The 1-D system of Appendix A: solid left of X_i(t) = U t, fluid to the
    right, the whole moving at U; T stays T0."""
    O = oracle_mod
    nx, U, T0 = 120, 0.037, 0.55
    d = W.domain(nx, 1, lambda_f=0.08, R_lambda=6.0, R_cv=4.0)
    o = O.Oracle(d, [], hooks={"thermal_only": 1, "fs_from_array": 1,
                               "u_pres": (U, 0.0)})
    x = np.arange(nx, dtype=float)
    X0 = 40.0
    o.raw("fs_next")[0, :] = np.clip(X0 - x, 0.0, 1.0)
    o.raw("T")[0, :] = T0
    o.init()
    for n in range(1, 700):
        o.raw("fs_next")[0, :] = np.clip(X0 + U * n - x, 0.0, 1.0)
        o.step(1)
    assert np.abs(o.field("T") - T0).max() < 1e-14


# --------------------------------------------------------------------------
# P5: Galilean co-motion


def test_galilean_comoving_particle(oracle_mod):
    """Uniform flow U carrying a neutrally buoyant disk at U in a periodic
    box is an exact fixed point: the momentum exchange vanishes and the
    particle moves X = X0 + U n."""
    O = oracle_mod
    U = (0.031, -0.017)
    d = W.domain(40, 44, init_u=U, R_cv=2.0, R_lambda=3.0)
    ps = [W.particle(17.3, 21.9, 6.1, rho_s=1.0, ux=U[0], uy=U[1],
                     T_init=1.0)]
    o = O.Oracle(d, ps).init()
    n = 200
    o.step(n)
    p = o.particles()[0]
    assert abs(p["ux"] - U[0]) < 1e-15 and abs(p["uy"] - U[1]) < 1e-15
    assert abs(p["Fx"]) < 1e-13 and abs(p["Fy"]) < 1e-13
    assert abs(p["x"] - (17.3 + n * U[0])) < 1e-11
    assert abs(p["y"] - (21.9 + n * U[1])) < 1e-11
    assert np.abs(o.field("ux") - U[0]).max() < 1e-13


# --------------------------------------------------------------------------
# particle dynamics, closed forms of the first steps (Sec. 2.3)


def test_released_particle_first_two_steps(oracle_mod):
    """A disk released from rest in fluid at rest, no fluid force: with
    F_MES^0 = 0 the first forward-Euler step gives U^1 = (1 - rho_f/rho_s) g;
    at step 1 the numerical fluid inside has taken momentum V U^1 so
    F_MES^1 = -V U^1, the inside-fluid term F_in = -M_in U^1 cancels it and
    U^2 = 2 U^1.  Positions lag velocities by one step (X^1 = X^0)."""
    O = oracle_mod
    g = (0.0, -2e-4)
    rho_s = 1.8
    d = W.domain(48, 48, gravity=g)
    ps = [W.particle(24.3, 23.8, 7.0, rho_s=rho_s)]
    o = O.Oracle(d, ps).init()
    o.step(1)
    p1 = o.particles()[0]
    U1 = (1 - 1 / rho_s) * g[1]
    assert abs(p1["uy"] - U1) < 1e-18 and p1["ux"] == 0.0
    assert p1["y"] == 23.8
    V = math.pi * 49.0
    assert abs(p1["Fy"] - (-V * U1)) < 1e-15
    o.step(1)
    p2 = o.particles()[0]
    assert abs(p2["uy"] - 2 * U1) < 1e-17
    assert abs(p2["y"] - (23.8 + U1)) < 1e-15


def test_fixed_particle_keeps_velocity(oracle_mod):
    O = oracle_mod
    d = W.domain(40, 40, gravity=(0.0, -1e-4), body_force=(1e-5, 0.0))
    ps = [W.particle(20.0, 20.0, 6.0, rho_s=3.0, ux=0.01, fixed=True)]
    o = O.Oracle(d, ps).init()
    o.step(30)
    p = o.particles()[0]
    assert p["ux"] == 0.01 and p["uy"] == 0.0 and p["omega"] == 0.0
    assert abs(p["x"] - 20.3) < 1e-13


# --------------------------------------------------------------------------
# P7: channel flows


def test_poiseuille_exact_parabola_with_bounce_back_slip(oracle_mod):
    """Force-driven channel between halfway bounce-back walls.  The steady
    discrete solution is an exact parabola of curvature -F/nu; with the
    paper's Lambda = (1/s_p - 1/2)(1/s_q - 1/2) = 1/12 the bounce-back wall
    carries the known two-relaxation-time slip, so
    u(y) = F/(2 nu) [y (H - y) + (16 Lambda - 3)/12] with y the node
    coordinate (Ginzburg & d'Humieres, Phys. Rev. E 68, 066614, 2003)."""
    O = oracle_mod
    tau, F, H = 0.8, 1e-6, 24
    nu = (tau - 0.5) / 3
    d = W.walls(W.domain(3, H, tau_f=tau, body_force=(F, 0.0)), (2, 3))
    o = O.Oracle(d, []).init()
    o.step(40000)
    u = o.field("ux")[:, 1]
    y = np.arange(H) + 0.5
    Lam = 1.0 / 12.0
    ref = F / (2 * nu) * (y * (H - y) + (16 * Lam - 3) / 12)
    assert np.abs(u - ref).max() < 1e-10 * ref.max()
    assert np.abs(o.field("uy")).max() < 1e-14


def test_couette_exact_linear_profile(oracle_mod):
    """Moving upper wall, still lower wall: the steady profile is linear
    between the halfway walls, u(y) = U_w y / H, exactly in the low-Mach
    limit; the departure is a compressibility effect of order U_w^3."""
    O = oracle_mod
    H = 20
    y = np.arange(H) + 0.5

    def run(Uw):
        d = W.walls(W.domain(3, H, tau_f=0.9), (2, 3))
        d["u_wall"] = [(0, 0), (0, 0), (0.0, 0.0), (Uw, 0.0)]
        o = O.Oracle(d, []).init()
        o.step(20000)
        return np.abs(o.field("ux")[:, 0] - Uw * y / H).max()

    assert run(1e-4) < 1e-13
    e1, e2 = run(0.02), run(0.01)
    assert 7.0 < e1 / e2 < 9.0


# --------------------------------------------------------------------------
# Collision model (reading of the cited model): invariants that hold for any
# short-range central repulsion with the descriptor's meaning of its
# constants -- the law's shape and constants themselves are a reading the
# paper does not fix (parity unpinned).


def _pair(O, X1, Y1, R1, X2, Y2, R2, nx=200, ny=200, periodic=True, kpp=3e-3,
          kpw=5e-3, zeta=2.0):
    d = W.domain(nx, ny, coll_range=zeta, coll_stiff_pp=kpp,
                 coll_stiff_pw=kpw)
    if not periodic:
        d = W.walls(d)
    ps = [W.particle(X1, Y1, R1), W.particle(X2, Y2, R2)]
    o = O.Oracle(d, ps)
    return o.collision_force(0), o.collision_force(1)


def test_collision_equal_and_opposite_along_centre_line(oracle_mod):
    """F_ij = -F_ji, directed from j to i, also across a periodic face
    (minimum image)."""
    O = oracle_mod
    for (X1, Y1, X2, Y2) in ((100.0, 100.0, 112.5, 104.0),
                             (3.0, 50.0, 190.0, 53.0),       # wraps in x
                             (70.0, 198.5, 66.0, 9.0)):      # wraps in y
        (f1x, f1y), (f2x, f2y) = _pair(O, X1, Y1, 7.0, X2, Y2, 6.0)
        assert math.hypot(f1x, f1y) > 0
        assert f1x == -f2x and f1y == -f2y
        dx = X1 - X2
        dy = Y1 - Y2
        dx -= 200.0 * round(dx / 200.0)
        dy -= 200.0 * round(dy / 200.0)
        # parallel to the centre line, pointing away from the other disk
        assert abs(f1x * dy - f1y * dx) < 1e-15 * math.hypot(f1x, f1y) * 20
        assert f1x * dx + f1y * dy > 0


def test_collision_contact_value_and_range(oracle_mod):
    """At contact (gap 0) the force equals the stiffness constant; at and
    beyond the range zeta it is zero; inside it the force decreases
    monotonically with the gap and vanishes continuously at the range."""
    O = oracle_mod
    R1, R2, zeta, k = 7.0, 6.0, 2.0, 3e-3
    (fx, fy), _ = _pair(O, 100.0, 100.0, R1, 100.0 + R1 + R2, 100.0, R2,
                        kpp=k, zeta=zeta)
    assert abs(math.hypot(fx, fy) - k) < 1e-15 and fx < 0
    for gap in (zeta, zeta + 0.5, 10.0):
        (fx, fy), _ = _pair(O, 100.0, 100.0, R1, 100.0 + R1 + R2 + gap,
                            100.0, R2, kpp=k, zeta=zeta)
        assert fx == 0.0 and fy == 0.0
    mags = []
    for gap in np.linspace(0.0, zeta * (1 - 1e-9), 9):
        (fx, fy), _ = _pair(O, 100.0, 100.0, R1, 100.0 + R1 + R2 + gap,
                            100.0, R2, kpp=k, zeta=zeta)
        mags.append(math.hypot(fx, fy))
    assert all(a > b for a, b in zip(mags, mags[1:]))
    assert mags[-1] < 1e-15 * k


def test_collision_wall_is_mirror_pair(oracle_mod):
    """Against a wall a particle feels what it would feel from its mirror
    image (same radius, stiffness k_pw) across the wall."""
    O = oracle_mod
    R, kpw, delta = 6.0, 5e-3, 6.5          # centre 6.5 from the y- wall
    d = W.walls(W.domain(200, 200, coll_range=2.0, coll_stiff_pp=1e-3,
                         coll_stiff_pw=kpw))
    o = O.Oracle(d, [W.particle(100.0, delta, R)])
    wx, wy = o.collision_force(0)
    (px, py), _ = _pair(O, 100.0, 100.0, R, 100.0, 100.0 - 2 * delta, R,
                        kpp=kpw)
    assert wy > 0 and wx == 0.0
    assert abs(wy - py) <= 1e-15 * abs(py) and px == 0.0
