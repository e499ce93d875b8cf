"""The C oracle against a second, independent transcription of the time
step in numpy (tests/numpy_step.py), on 8 x 8 grids with two particles,
step by step over four steps: every population, the macroscopic fields,
[df_s/dt] and the particle states and outputs agree to rounding (1e-13
relative to each quantity's scale, the momentum-exchange sums 1e-14
relative to the populations that enter them; the exact areas, from a
different method, to 1e-14).

The transcription shares no code with the oracle; it builds the
transformation matrix from its defining polynomials, takes the textbook
D2Q9 equilibrium and Guo's velocity-space force term to moment space
through that matrix, integrates the areas by adaptive quadrature, solves
the coupled T and u as the root of the energy relation and streams whole
arrays.  Two pins on the paper's printed formulas come with it: the printed
matrix, equilibrium moments and force moments equal what the definitions
give."""
import math

import numpy as np
import pytest

import numpy_step as NS
import workloads as W


def test_printed_matrix_and_moments_follow_from_their_definitions():
    printed = np.array([
        [1, 1, 1, 1, 1, 1, 1, 1, 1],
        [-4, -1, -1, -1, -1, 2, 2, 2, 2],
        [4, -2, -2, -2, -2, 1, 1, 1, 1],
        [0, 1, 0, -1, 0, 1, -1, -1, 1],
        [0, -2, 0, 2, 0, 1, -1, -1, 1],
        [0, 0, 1, 0, -1, 1, 1, -1, -1],
        [0, 0, -2, 0, 2, 1, 1, -1, -1],
        [0, 1, -1, 1, -1, 0, 0, 0, 0],
        [0, 0, 0, 0, 0, 1, -1, 1, -1]], dtype=float)
    assert np.array_equal(NS.MT, printed)
    rng = np.random.default_rng(0)
    for _ in range(20):
        rho, ux, uy, Fx, Fy = rng.uniform(0.5, 1.5), *rng.uniform(-0.2, 0.2, 4)
        u2 = ux * ux + uy * uy
        meq = [rho, -2 * rho + 3 * rho * u2, rho - 3 * rho * u2, rho * ux,
               -rho * ux, rho * uy, -rho * uy, rho * (ux * ux - uy * uy),
               rho * ux * uy]
        assert np.allclose(NS.to_moments(NS.feq(rho, ux, uy)), meq,
                           rtol=0, atol=1e-15)
        Fu = Fx * ux + Fy * uy
        Fm = [0, 6 * Fu, -6 * Fu, Fx, -Fx, Fy, -Fy, 2 * (Fx * ux - Fy * uy),
              Fx * uy + Fy * ux]
        assert np.allclose(NS.to_moments(NS.guo(Fx, Fy, ux, uy)), Fm,
                           rtol=0, atol=1e-15)


def case_periodic():
    """A periodic box: a disk and an ellipse, moving and spinning, warm
    and cold, with gravity, buoyancy, a body force and repulsion."""
    d = W.domain(8, 8, tau_f=0.71, lambda_f=0.07, R_lambda=4.0, R_cv=2.5,
                 body_force=(3e-6, -1e-6), gravity=(0.0, -2e-5), beta=0.4,
                 T_ref=0.5, init_T=0.8, init_u=(0.004, -0.002),
                 coll_range=1.0, coll_stiff_pp=2e-4, coll_stiff_pw=3e-4)
    ps = [W.particle(2.3, 2.8, 1.7, rho_s=1.6, T_init=0.1, ux=0.01,
                     uy=-0.006, omega=0.004),
          W.particle(5.6, 5.4, 1.9, rho_s=1.3, T_init=0.9, ux=-0.008,
                     uy=0.003, omega=-0.006, theta=0.6, radius_minor=1.2)]
    return d, ps


def case_walls():
    """Walls on all four faces: a moving top lid, Dirichlet and adiabatic
    thermal faces, the fluid carrying its own weight, the dense-case
    relaxation rule, and a disk whose temperature is held."""
    d = W.domain(8, 8, tau_f=0.6, lambda_f=0.04, R_lambda=0.3, R_cv=0.7,
                 gravity=(1e-5, -3e-5), beta=0.2, T_ref=0.3, init_T=0.3,
                 sigma_rule=1, fluid_gravity=1, coll_range=1.5,
                 coll_stiff_pp=1e-4, coll_stiff_pw=2e-4)
    d = W.walls(d, thermal="dirichlet", T_wall=[0.2, 0.7, 0.4, 0.9])
    d["face_thermal"][0] = "adiabatic"
    d["u_wall"][3] = (0.02, 0.0)
    ps = [W.particle(2.6, 5.2, 1.6, rho_s=1.8, T_init=0.0, ux=0.005,
                     uy=0.004, omega=0.003, hold_T=True),
          W.particle(5.5, 2.2, 1.5, rho_s=0.7, T_init=1.0, ux=-0.004,
                     uy=0.006, omega=-0.002)]
    return d, ps


def scale(a):
    return max(1e-300, float(np.abs(a).max()))


@pytest.mark.parametrize("make", [case_periodic, case_walls],
                         ids=["periodic", "walls"])
def test_four_steps_agree(oracle_mod, make):
    d, ps = make()
    o = oracle_mod.Oracle(d, ps).init()
    t = NS.Step(d, ps).init()
    assert np.abs(o.field("fs") - t.fs).max() < 1e-14
    for name, a in (("f", t.f), ("g", t.g), ("T", t.T)):
        b = o.field(name)
        assert np.abs(b - a).max() < 1e-14 * scale(b), name
    for n in range(1, 5):
        o.step(1)
        t.step()
        assert np.abs(o.field("fs") - t.fs).max() < 1e-14, n
        assert np.abs(o.field("d") - t.dfs).max() < 1e-13, n
        for name, a in (("f", t.f), ("g", t.g), ("rho", t.rho),
                        ("ux", t.ux), ("uy", t.uy), ("T", t.T)):
            b = o.field(name)
            err = np.abs(b - a).max()
            assert err < 1e-13 * scale(b), (n, name, err, scale(b))
        po = o.particles()
        outs = t.particle_outputs()
        for k, p in enumerate(t.P):
            for key, mine in (("x", p["x"]), ("y", p["y"]),
                              ("theta", p["theta"]), ("ux", p["ux"]),
                              ("uy", p["uy"]), ("omega", p["omega"])):
                assert abs(po[key][k] - mine) < 1e-15 * max(1, abs(mine)), \
                    (n, k, key)
            # the sums cancel: their scale is that of the populations in
            # their terms
            for key, mine, lever in (("Fx", p["Fx"], 1), ("Fy", p["Fy"], 1),
                                     ("Tz", p["Tz"], p["radius"])):
                assert abs(po[key][k] - mine) < 1e-14 * p["Fabs"] * lever, \
                    (n, k, key, abs(po[key][k] - mine), p["Fabs"])
            for key, mine in outs[k].items():
                assert abs(po[key][k] - mine) < 1e-13 * max(1, abs(mine)), \
                    (n, k, key)
        # the step moved something: forces and torques are not zero
        assert all(abs(p["Fx"]) + abs(p["Fy"]) > 1e-8 for p in t.P)
