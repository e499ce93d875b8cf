"""GPU parity of the fluid-gravity option (situation II of Sec. 3.2) against
the oracle: the hydrostatic column, a settling disk (scan form) and 80
disks in a walled box (list form), FP64.  Tolerances as in
test_gpu_parity."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import (check, field_errors, particle_errors, run_pair,
                             say, twin_errors)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_23802_amd import vlb as v
    v.lib()  # fails loudly if the HIP library is missing
    return v


KEYS = ("x", "y", "ux", "uy", "omega", "Fx", "Fy", "Tz")


def test_hydrostatic_column_fp64(vlb, oracle_mod):
    d = W.walls(W.domain(16, 400, tau_f=0.6, gravity=(0.0, -1e-4),
                         fluid_gravity=1), which=(W.YLO, W.YHI))
    say("case: hydrostatic column fp64 500 steps")
    g, o = run_pair(vlb, oracle_mod, d, [], 0)
    assert np.abs(g.field("rho") - o.field("rho")).max() < 1e-14
    g.step(500)
    o.step(500)
    g._parts = []
    e = field_errors(g, o, ("rho", "ux", "uy", "T"))
    check(e, 500, twin=twin_errors(oracle_mod, d, [], 500, o,
                                   names=("rho", "ux", "uy", "T")))


def test_settling_disk_fluid_gravity_fp64(vlb, oracle_mod):
    d = W.walls(W.domain(80, 240, tau_f=0.515, gravity=(0.0, -2e-5),
                         fluid_gravity=1, coll_range=2.0, coll_stiff_pp=1e-3,
                         coll_stiff_pw=2e-3, beta=0.3, init_T=1.0),
                thermal="dirichlet", T_wall=1.0)
    ps = [W.particle(37.3, 180.0, 8.0, rho_s=1.5, T_init=0.0)]
    say("case: settling disk, fluid gravity, fp64 600 steps")
    g, o = run_pair(vlb, oracle_mod, d, ps, 600)
    e = field_errors(g, o)
    e.update(particle_errors(g, o, KEYS))
    check(e, 600, twin=twin_errors(oracle_mod, d, ps, 600, o, pkeys=KEYS))


def test_fluid_gravity_list_form_fp64(vlb, oracle_mod):
    rng = np.random.default_rng(31)
    d = W.walls(W.domain(160, 128, tau_f=0.6, lambda_f=0.05, R_lambda=4.0,
                         R_cv=1.5, gravity=(0.0, -4e-5), beta=0.2,
                         fluid_gravity=1, init_T=1.0, coll_range=2.0,
                         coll_stiff_pp=2e-3, coll_stiff_pw=4e-3),
                thermal="adiabatic")
    pts = W.rsa_disks(80, 5.0, (0.0, 0.0, 160.0, 128.0), 1.0, seed=7)
    ps = [W.particle(x, y, rng.uniform(3.0, 5.0), rho_s=rng.uniform(1.2, 2.0),
                     T_init=0.2, ux=rng.uniform(-0.01, 0.01),
                     uy=rng.uniform(-0.01, 0.01)) for x, y in pts]
    say("case: 80 particles, fluid gravity, list form fp64 120 steps")
    g, o = run_pair(vlb, oracle_mod, d, ps, 120)
    e = field_errors(g, o)
    e.update(particle_errors(g, o, KEYS))
    check(e, 120, twin=twin_errors(oracle_mod, d, ps, 120, o, pkeys=KEYS))
