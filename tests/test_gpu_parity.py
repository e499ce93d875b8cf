"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Floating point: FP64 storage must match to 1e-12 relative per field
(max |gpu - oracle| / max |oracle|); FP32 to 1e-5.  Integer work (cell
ownership, particle lists) must match bit for bit.
"""
import math
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "ux", "uy", "T", "fs", "dfs")


@pytest.fixture(scope="module")
def vlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_23802_amd import vlb as v
    v.lib()  # fails loudly if the HIP library is missing
    return v


def say(msg):
    print(msg, flush=True)


def rel(a, b, floor=1e-300):
    scale = max(float(np.abs(b).max()), floor)
    return float(np.abs(a - b).max()) / scale


def field_errors(g, o, names=FIELDS):
    out = {}
    for n in names:
        b = o.field("d" if n == "dfs" else n)
        a = g.field(n)
        # a field that is zero in the oracle is compared in absolute terms
        out[n] = rel(a, b, floor=1.0 if np.abs(b).max() == 0 else 1e-300)
    return out


def particle_errors(g, o, keys=("x", "y", "ux", "uy", "omega", "Fx", "Fy",
                                "Tz")):
    pa, pb = g.particles(), o.particles()
    out = {}
    for k in keys:
        scale = max(float(np.abs(pb[k]).max()), 1e-300)
        out[k] = float(np.abs(pa[k] - pb[k]).max()) / scale
    return out


def run_pair(vlb, oracle_mod, d, ps, nsteps, precision="fp64"):
    g = vlb.Domain(d, ps, precision).init()
    o = oracle_mod.Oracle(d, ps).init()
    if nsteps:
        g.step(nsteps)
        o.step(nsteps)
    return g, o


# --------------------------------------------------------------------------


def test_init_state_matches(vlb, oracle_mod):
    d, ps = W.c1_tiny()
    say("case: init c1_tiny fp64")
    g, o = run_pair(vlb, oracle_mod, d, ps, 0)
    e = field_errors(g, o, ("rho", "ux", "uy", "T", "fs"))
    assert max(e.values()) < 1e-13, e
    assert rel(g.field("f"), o.field("f")) < 1e-14
    assert rel(g.field("g"), o.field("g")) < 1e-14


def test_one_step_c1(vlb, oracle_mod):
    d, ps = W.c1_tiny()
    say("case: one step c1_tiny fp64")
    g, o = run_pair(vlb, oracle_mod, d, ps, 1)
    e = field_errors(g, o)
    e.update(particle_errors(g, o, ("Fx", "Fy", "Tz")))
    assert max(e.values()) < 1e-12, e
    assert rel(g.field("f"), o.field("f")) < 1e-12
    assert rel(g.field("g"), o.field("g")) < 1e-12


def test_c1_tiny_1000_steps_fp64(vlb, oracle_mod):
    """The tiny workload: 128 x 64 channel, one fixed cold disk, 1000 steps."""
    d, ps = W.c1_tiny()
    say("case: c1_tiny fp64 1000 steps")
    g, o = run_pair(vlb, oracle_mod, d, ps, 1000)
    e = field_errors(g, o)
    e.update(particle_errors(g, o, ("Fx", "Fy", "Tz")))
    pa, pb = g.particles()[0], o.particles()[0]
    for k in ("T_mean", "T_min", "E_solid", "fs_sum"):
        e[k] = abs(pa[k] - pb[k]) / max(abs(pb[k]), 1e-300)
    assert max(e.values()) < 1e-12, e


def test_moving_particles_periodic_fp64(vlb, oracle_mod):
    """Two free disks with different densities in a periodic box with a body
    force and buoyancy; the disks cross cell boundaries every few steps."""
    d = W.domain(96, 80, tau_f=0.7, lambda_f=0.05, R_lambda=7.0, R_cv=3.0,
                 body_force=(2e-6, 0.0), gravity=(0.0, -3e-5), beta=0.4,
                 init_T=0.8, init_u=(0.02, -0.01))
    ps = [W.particle(30.3, 34.2, 7.5, rho_s=1.7, T_init=0.2, ux=0.02,
                     uy=0.01, omega=0.003),
          W.particle(66.1, 47.7, 5.2, rho_s=0.8, T_init=0.9, ux=-0.03,
                     omega=-0.002)]
    say("case: periodic two moving disks fp64 300 steps")
    g, o = run_pair(vlb, oracle_mod, d, ps, 300)
    e = field_errors(g, o)
    e.update(particle_errors(g, o))
    assert max(e.values()) < 1e-12, e


def test_walls_dirichlet_channel_fp64(vlb, oracle_mod):
    """Scaled-down channel: walls on all sides at T = 1, one cold heavy disk
    released near the top, gravity and buoyancy, collisions with walls."""
    d, ps = W.c2_channel(nx=64, ny=240)
    ps[0]["y"] = 200.0
    say("case: small dirichlet channel fp64 400 steps")
    g, o = run_pair(vlb, oracle_mod, d, ps, 400)
    e = field_errors(g, o)
    e.update(particle_errors(g, o))
    assert max(e.values()) < 1e-12, e


def test_moving_wall_and_corners_fp64(vlb, oracle_mod):
    """Lid-driven cavity with a warm bottom wall: moving-wall bounce-back and
    corners of two walls."""
    d = W.walls(W.domain(40, 36, tau_f=0.6, init_T=0.5), thermal="adiabatic")
    d["u_wall"] = [(0, 0), (0, 0), (0.0, 0.0), (0.05, 0.0)]
    d["face_thermal"] = ["adiabatic", "adiabatic", "dirichlet", "dirichlet"]
    d["T_wall"] = [0.0, 0.0, 1.0, 0.0]
    say("case: lid-driven cavity fp64 500 steps")
    g, o = run_pair(vlb, oracle_mod, d, [], 500)
    e = field_errors(g, o, ("rho", "ux", "uy", "T"))
    assert max(e.values()) < 1e-12, e


# --------------------------------------------------------------------------
# integer work: ownership, bit for bit


def adversarial_particles():
    ps = [
        W.particle(20.0, 20.0, 6.0),            # centre on a grid corner
        W.particle(45.5, 20.5, 5.5),            # centre on a node, R half-int
        W.particle(70.0, 20.37, 4.0),           # centre on a vertical grid line
        W.particle(20.25, 50.0, 6.75),          # on a horizontal grid line
        W.particle(48.5, 50.5, 2.5),            # touches faces exactly
        W.particle(1.3, 70.6, 3.9),             # wraps across x
        W.particle(80.7, 2.2, 4.4),             # wraps across y
        W.particle(0.0, 0.0, 3.0),              # wraps across both
        W.particle(70.1, 49.9, 1e-3 + 0.5),     # tiny disk
    ]
    return ps


def test_ownership_bit_exact_adversarial(vlb, oracle_mod):
    d = W.domain(96, 88, kmax=4)
    ps = adversarial_particles()
    say("case: ownership adversarial")
    g = vlb.Domain(d, ps, "fp64").init()
    o = oracle_mod.Oracle(d, ps).init()
    gc, gi, gf = g.ownership()
    oc, oi, of = o.ownership()
    assert np.array_equal(gc, oc)
    assert np.array_equal(gi, oi)
    assert np.array_equal(gf, of)


def test_ownership_bit_exact_random(vlb, oracle_mod):
    rng = np.random.default_rng(7)
    d = W.domain(160, 128, kmax=4)
    pts = W.rsa_disks(60, 6.0, (0.0, 0.0, 160.0, 128.0), 0.5, seed=3)
    ps = [W.particle(x, y, rng.uniform(3.0, 6.0)) for x, y in pts]
    say("case: ownership random 60 disks")
    g = vlb.Domain(d, ps, "fp64").init()
    o = oracle_mod.Oracle(d, ps).init()
    for _ in range(3):
        gc, gi, gf = g.ownership()
        oc, oi, of = o.ownership()
        assert np.array_equal(gc, oc) and np.array_equal(gi, oi)
        assert np.array_equal(gf, of)
        g.step(7)
        o.step(7)


# --------------------------------------------------------------------------
# full sizes, in the configuration the benchmark runs


def test_channel_full_size_fp64(vlb, oracle_mod):
    """200 x 4000 channel, one cold disk: a few steps, every cell compared."""
    d, ps = W.c2_channel()
    say("case: c2_channel full size fp64 6 steps")
    g, o = run_pair(vlb, oracle_mod, d, ps, 6)
    e = field_errors(g, o)
    e.update(particle_errors(g, o))
    assert max(e.values()) < 1e-12, e


def test_isothermal_invariant_full_size(vlb):
    """Appendix A at full size on the GPU: uniform T0 with a moving disk of
    different heat capacity stays exactly uniform."""
    d, ps = W.c2_channel()
    d["init_T"] = 0.6
    d["T_wall"] = [0.6] * 4
    ps[0]["T_init"] = 0.6
    ps[0]["uy"] = -0.02
    say("case: isothermal invariant c2 full size 300 steps")
    g = vlb.Domain(d, ps, "fp64").init().step(300)
    assert np.abs(g.field("T") - 0.6).max() < 1e-13


def test_dense_full_size_fp64(vlb, oracle_mod):
    """1536^2 cavity with 2048 disks: ownership bit for bit, fields and
    forces after two steps."""
    d, ps = W.c3_dense()
    say("case: c3_dense full size fp64")
    g = vlb.Domain(d, ps, "fp64").init()
    o = oracle_mod.Oracle(d, ps).init()
    gc, gi, gf = g.ownership()
    oc, oi, of = o.ownership()
    assert np.array_equal(gc, oc) and np.array_equal(gi, oi)
    assert np.array_equal(gf, of)
    g.step(2)
    o.step(2)
    e = field_errors(g, o)
    e.update(particle_errors(g, o))
    assert max(e.values()) < 1e-12, e


# --------------------------------------------------------------------------
# storage forms


def test_fp32_c1(vlb, oracle_mod):
    d, ps = W.c1_tiny()
    say("case: c1_tiny fp32 1000 steps")
    g, o = run_pair(vlb, oracle_mod, d, ps, 1000, "fp32")
    e = field_errors(g, o, ("rho", "T", "fs"))
    # velocities are O(1e-4): compare on the scale of the velocity field
    assert max(e.values()) < 1e-5, e
    ue = rel(g.field("ux"), o.field("ux"))
    assert ue < 1e-3, ue


@pytest.mark.parametrize("prec,tol_T", [("fp16s", 5e-3), ("bf16s", 5e-2)])
def test_shifted_16bit_c1(vlb, oracle_mod, prec, tol_T):
    d, ps = W.c1_tiny()
    say(f"case: c1_tiny {prec} 1000 steps")
    g, o = run_pair(vlb, oracle_mod, d, ps, 1000, prec)
    eT = rel(g.field("T"), o.field("T"))
    erho = rel(g.field("rho"), o.field("rho"))
    say(f"  {prec}: rel err T {eT:.2e} rho {erho:.2e}")
    assert eT < tol_T and erho < tol_T


# --------------------------------------------------------------------------
# host logic on the GPU path


def test_bitwise_reproducible(vlb):
    d = W.domain(64, 64, tau_f=0.7, gravity=(0, -5e-5), beta=0.3,
                 coll_range=2.0, coll_stiff_pp=1e-3, coll_stiff_pw=2e-3)
    d = W.walls(d)
    ps = [W.particle(20.5 + 8 * k, 40.0 + 3 * (k % 2), 3.5, rho_s=1.6)
          for k in range(4)]
    say("case: reproducibility")
    a = vlb.Domain(d, ps).init().step(150)
    b = vlb.Domain(d, ps).init().step(150)
    for n in ("f", "g", "T", "ux"):
        assert np.array_equal(a.field(n), b.field(n))
    pa, pb = a.particles(), b.particles()
    assert all(np.array_equal(pa[k], pb[k]) for k in pa.dtype.names)


def test_save_load_continues_bitwise(vlb):
    d, ps = W.c2_channel(nx=48, ny=160)
    ps[0]["y"] = 120.0
    say("case: save/load")
    a = vlb.Domain(d, ps).init().step(37)
    blob = a.save()
    a.step(25)
    b = vlb.Domain(d, ps)
    b.load(blob)
    assert b.step_count == 37
    b.step(25)
    for n in ("f", "g", "T", "dfs"):
        assert np.array_equal(a.field(n), b.field(n))
    pa, pb = a.particles(), b.particles()
    assert all(np.array_equal(pa[k], pb[k]) for k in pa.dtype.names)


def test_unstable_flag(vlb):
    d = W.domain(32, 32, tau_f=0.5001, body_force=(0.5, 0.3))
    say("case: unstable flag")
    g = vlb.Domain(d, []).init()
    with pytest.raises(vlb.VlbError) as ei:
        g.step(400)
    assert ei.value.status == vlb.VLB_EUNSTABLE


def test_overlap_flag(vlb):
    d = W.domain(40, 40, kmax=1)
    ps = [W.particle(15.0, 20.0, 4.0), W.particle(22.5, 20.0, 4.0)]
    say("case: overlap flag")
    g = vlb.Domain(d, ps)
    with pytest.raises(vlb.VlbError) as ei:
        g.init()
    assert ei.value.status == vlb.VLB_EOVERLAP


def test_step_before_init_is_state_error(vlb):
    g = vlb.Domain(W.domain(16, 16), [])
    with pytest.raises(vlb.VlbError) as ei:
        g.step(1)
    assert ei.value.status == vlb.VLB_ESTATE
