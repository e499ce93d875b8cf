"""Pins of the oracle's held particle temperature (stage 5b): a particle of
fixed temperature (the cold particle of Sec. 3.3).  The paper does not give
the rule that holds the temperature; the oracle reads it as the volumetric
step of the energy distribution, g = (1 - sum_h f_s,p) g* + sum_h f_s,p
g^eq(c_v T_p, T_p) with c_v the cell's heat capacity.  What that reading
fixes, checked here:

  * a cell wholly inside a held disk at rest reads T = T_p after every step
    (its energy is the solid's equilibrium at T_p), whatever the fluid
    around it does;
  * a held disk at rest in fluid at its own temperature leaves the uniform
    state unchanged, also with a heat-capacity and conductivity jump (a
    wrong equilibrium or weighting in the step would disturb it);
  * with the flow at rest the energy update is affine in the temperatures,
    so swapping the held and wall temperatures (0 and 1) gives fields that
    add up to 1 everywhere (the uniform state of the sum).
"""
import numpy as np

import workloads as W


def held_box(T_p, T_fluid, R_cv, R_lambda, T_walls=None, hold=True):
    d = W.domain(48, 40, tau_f=0.8, lambda_f=0.08, R_lambda=R_lambda,
                 R_cv=R_cv, init_T=T_fluid)
    if T_walls is not None:
        d = W.walls(d, thermal="dirichlet", T_wall=T_walls)
    ps = [W.particle(23.3, 19.6, 7.5, T_init=T_p, fixed=True, hold_T=hold)]
    return d, ps


def test_held_disk_interior_stays_at_held_temperature(oracle_mod):
    d, ps = held_box(0.0, 1.0, R_cv=2.0, R_lambda=10.0, T_walls=1.0)
    o = oracle_mod.Oracle(d, ps).init()
    free = oracle_mod.Oracle(d, [dict(ps[0], hold_T=0)]).init()
    for _ in range(4):
        o.step(25)
        free.step(25)
        full = o.field("fs") == 1.0
        assert full.sum() > 100
        assert np.abs(o.field("T")[full]).max() < 1e-13
    # without the hold the solid warms up
    assert free.field("T")[full].max() > 0.05


def test_held_disk_in_fluid_at_its_temperature_is_steady(oracle_mod):
    d, ps = held_box(0.7, 0.7, R_cv=2.0, R_lambda=10.0)
    o = oracle_mod.Oracle(d, ps).init()
    o.step(80)
    assert np.abs(o.field("T") - 0.7).max() < 1e-13


def test_held_temperatures_superpose(oracle_mod):
    da, pa = held_box(0.0, 1.0, R_cv=1.0, R_lambda=10.0, T_walls=1.0)
    db, pb = held_box(1.0, 0.0, R_cv=1.0, R_lambda=10.0, T_walls=0.0)
    a = oracle_mod.Oracle(da, pa).init()
    b = oracle_mod.Oracle(db, pb).init()
    a.step(120)
    b.step(120)
    Ta, Tb = a.field("T"), b.field("T")
    assert np.abs(Ta + Tb - 1.0).max() < 1e-12
    # the fields are far from uniform (the held disk matters)
    assert Ta.min() < 0.2 and Ta.max() > 0.9


def test_fixed_temperature_channel_recipe():
    """The Sec. 3.3 channel as the workload builds it: Re = 40.5 with
    tau_f = 0.53 and D = 20 gives U_ref = 0.02025, |g| from U_ref =
    sqrt((rho_r - 1) |g| pi D / 2), beta from Gr; the disk starts D/2 left of
    the centre line and is held at T_c = 0."""
    import math
    d, ps = W.e5_held_channel(1000.0)
    nu = 0.01
    U = 40.5 * nu / 20.0
    g = U * U / (0.00232 * math.pi * 10.0)
    assert abs(W.u_ref(1.00232, d["gravity"][1], 20.0) - 0.02025) < 1e-15
    assert abs(-d["gravity"][1] - g) < 1e-15 and d["gravity"][0] == 0.0
    assert abs(d["beta"] - 1000.0 * nu * nu / (g * 20.0 ** 3)) < 1e-15
    assert d["nx"] == 80 and d["R_lambda"] == 1.0 and d["R_cv"] == 1.0
    assert abs(d["lambda_f"] - nu / 0.7) < 1e-15
    assert ps[0]["x"] == 30.0 and ps[0]["hold_T"] == 1 and ps[0]["T_init"] == 0.0
