"""Pins of the oracle's fluid-gravity option (situation II of Sec. 3.2: the
fluid carries rho_f g, the particle rho_s V g, and the start is
hydrostatic).

  * Hydrostatic rest: a column with walls at the ends keeps the linear
    density rho_0 + 3 rho_f g (y - y_m) that grad p = rho_f g gives with p =
    rho / 3 (to the size of the acoustic wave the first step's force term
    launches, ~F / (2 rho) in velocity), and stays near rest; a uniform
    start under the same force sloshes 30 times harder.  An exponential
    profile, a wrong factor or sign would be off by 1.8e-3 or more here.
  * Situations I and II agree: a disk settling in a box moves the same way
    whether the buoyancy is put into the particle's force ((rho_s - rho_f)
    V g) or comes from the fluid's pressure gradient through the momentum
    exchange (the paper's check, Sec. 3.2; there with tau_f = 0.515 to keep
    the density variation small).
"""
import numpy as np

import workloads as W


def column(fluid_gravity, body_force=(0.0, 0.0), ny=400):
    return W.walls(W.domain(16, ny, tau_f=0.6, gravity=(0.0, -1e-4),
                            body_force=body_force,
                            fluid_gravity=fluid_gravity),
                   which=(W.YLO, W.YHI))


def test_hydrostatic_column_stays_at_rest(oracle_mod):
    o = oracle_mod.Oracle(column(1), []).init()
    y = np.arange(400) + 0.5
    lin = 1.0 + 3.0 * (-1e-4) * (y - 200.0)
    assert np.abs(o.field("rho") - lin[:, None]).max() < 1e-14
    o.step(1500)
    assert np.abs(o.field("rho") - lin[:, None]).max() < 5e-4
    u2 = np.hypot(o.field("ux"), o.field("uy")).max()
    assert u2 < 2e-4
    # the same force from a uniform start
    b = oracle_mod.Oracle(column(0, body_force=(0.0, -1e-4)), []).init()
    b.step(1500)
    assert np.hypot(b.field("ux"), b.field("uy")).max() > 30 * u2


def test_situations_one_and_two_agree(oracle_mod):
    res = {}
    for fg in (0, 1):
        d = W.walls(W.domain(80, 240, tau_f=0.515, gravity=(0.0, -2e-5),
                             fluid_gravity=fg, coll_range=2.0,
                             coll_stiff_pp=1e-3, coll_stiff_pw=2e-3),
                    thermal="adiabatic")
        o = oracle_mod.Oracle(d, [W.particle(37.3, 180.0, 8.0,
                                             rho_s=1.5)]).init()
        o.step(3000)
        res[fg] = o.particles()
    a, b = res[0], res[1]
    fall = 180.0 - float(a["y"][0])
    assert fall > 8.0                       # it did settle (0.6 D)
    assert abs(float(a["y"][0]) - float(b["y"][0])) / 16.0 < 0.01
    assert abs(float(a["uy"][0]) - float(b["uy"][0])) < 0.02 * abs(float(a["uy"][0]))
