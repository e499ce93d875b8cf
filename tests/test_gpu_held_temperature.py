"""GPU parity of particles whose temperature is held (the cold particle of
fixed temperature of Sec. 3.3), against the oracle's stage 5b: the scan
form (a held disk at rest and a held disk moving beside a free one, FP64,
and the held disk at rest at FP32) and the list form (80 moving disks, half
of them held).  Tolerances as in test_gpu_parity."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import (FP32_BAR, check, field_errors, particle_errors,
                             run_pair, say, twin_errors)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_23802_amd import vlb as v
    v.lib()  # fails loudly if the HIP library is missing
    return v


def held_channel():
    """128 x 64 channel, walls at T = 1 in y, periodic in x with a body
    force; a held disk at rest (T = 0) and conductivity / heat-capacity
    jumps that a wrong rule would show."""
    d = W.walls(W.domain(128, 64, tau_f=0.8, lambda_f=0.06, R_lambda=10.0,
                         R_cv=2.0, body_force=(1e-6, 0.0), init_T=1.0),
                which=(W.YLO, W.YHI), thermal="dirichlet", T_wall=1.0)
    return d, [W.particle(64.0, 32.0, 8.0, T_init=0.0, fixed=True,
                          hold_T=True)]


def test_held_disk_at_rest_fp64(vlb, oracle_mod):
    d, ps = held_channel()
    say("case: held disk at rest fp64 600 steps")
    g, o = run_pair(vlb, oracle_mod, d, ps, 600)
    e = field_errors(g, o)
    keys = ("Fx", "Fy", "Tz")
    e.update(particle_errors(g, o, keys))
    check(e, 600, twin=twin_errors(oracle_mod, d, ps, 600, o, pkeys=keys))
    full = o.field("fs") == 1.0
    assert np.abs(g.field("T")[full]).max() < 1e-13


def test_held_disk_at_rest_fp32(vlb, oracle_mod):
    d, ps = held_channel()
    say("case: held disk at rest fp32 600 steps")
    g, o = run_pair(vlb, oracle_mod, d, ps, 600, "fp32")
    e = field_errors(g, o)
    say(f"  fp32 errors after 600 steps: {e}")
    bad = {k: v for k, v in e.items() if v >= FP32_BAR.get(k, 1e-5)}
    assert not bad, (bad, e)


def test_held_and_free_moving_disks_fp64(vlb, oracle_mod):
    """A held cold disk and a free warm one, both moving, in a periodic box
    with gravity and buoyancy."""
    d = W.domain(96, 80, tau_f=0.7, lambda_f=0.05, R_lambda=7.0, R_cv=3.0,
                 body_force=(2e-6, 0.0), gravity=(0.0, -3e-5), beta=0.4,
                 init_T=0.8, init_u=(0.02, -0.01))
    ps = [W.particle(30.3, 34.2, 7.5, rho_s=1.7, T_init=0.1, ux=0.02,
                     uy=0.01, omega=0.003, hold_T=True),
          W.particle(66.1, 47.7, 5.2, rho_s=0.8, T_init=0.9, ux=-0.03,
                     omega=-0.002)]
    say("case: held and free moving disks fp64 300 steps")
    g, o = run_pair(vlb, oracle_mod, d, ps, 300)
    e = field_errors(g, o)
    keys = ("x", "y", "ux", "uy", "omega", "Fx", "Fy", "Tz")
    e.update(particle_errors(g, o, keys))
    check(e, 300, twin=twin_errors(oracle_mod, d, ps, 300, o, pkeys=keys))


def test_held_particles_list_form_fp64(vlb, oracle_mod):
    """80 moving disks with collisions in a walled box, every other one
    held at T = 0.2: the list form."""
    rng = np.random.default_rng(21)
    d = W.walls(W.domain(160, 128, tau_f=0.65, lambda_f=0.05, R_lambda=4.0,
                         R_cv=1.5, gravity=(0.0, -4e-5), beta=0.2,
                         init_T=1.0, coll_range=2.0, coll_stiff_pp=2e-3,
                         coll_stiff_pw=4e-3), thermal="adiabatic")
    pts = W.rsa_disks(80, 5.0, (0.0, 0.0, 160.0, 128.0), 1.0, seed=5)
    ps = [W.particle(x, y, rng.uniform(3.0, 5.0), rho_s=rng.uniform(1.2, 2.0),
                     T_init=0.2, ux=rng.uniform(-0.01, 0.01),
                     uy=rng.uniform(-0.01, 0.01), hold_T=(k % 2 == 0))
          for k, (x, y) in enumerate(pts)]
    say("case: 80 particles, 40 held, list form fp64 120 steps")
    g, o = run_pair(vlb, oracle_mod, d, ps, 120)
    e = field_errors(g, o)
    keys = ("x", "y", "ux", "uy", "omega", "Fx", "Fy", "Tz")
    e.update(particle_errors(g, o, keys))
    check(e, 120, twin=twin_errors(oracle_mod, d, ps, 120, o, pkeys=keys))


@pytest.mark.parametrize("list_form", [False, True])
def test_save_load_continues_bitwise_held_and_fluid_gravity(vlb, list_form):
    """A checkpoint taken with held particles and the fluid-gravity option
    restores both (the flag word is rebuilt from the descriptors on load)
    and the run continues bit for bit; scan and list form."""
    d = W.walls(W.domain(96, 160, tau_f=0.6, lambda_f=0.05, R_lambda=3.0,
                         R_cv=1.5, gravity=(0.0, -2e-5), beta=0.3,
                         fluid_gravity=1, init_T=1.0, coll_range=2.0,
                         coll_stiff_pp=1e-3, coll_stiff_pw=2e-3),
                thermal="dirichlet", T_wall=1.0)
    n = 70 if list_form else 2
    pts = W.rsa_disks(n, 4.0, (0.0, 0.0, 96.0, 160.0), 1.5, seed=9)
    ps = [W.particle(x, y, 4.0, rho_s=1.4, T_init=0.1 * (k % 3),
                     hold_T=(k % 2 == 0)) for k, (x, y) in enumerate(pts)]
    say(f"case: save/load held + fluid gravity, {n} particles")
    a = vlb.Domain(d, ps).init().step(23)
    blob = a.save()
    a.step(17)
    b = vlb.Domain(d, ps)
    b.load(blob)
    b.step(17)
    for k in ("f", "g", "T", "dfs"):
        assert np.array_equal(a.field(k), b.field(k)), k
    pa, pb = a.particles(), b.particles()
    assert all(np.array_equal(pa[k], pb[k]) for k in pa.dtype.names)
    a.close()
    b.close()
