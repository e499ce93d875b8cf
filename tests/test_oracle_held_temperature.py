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
