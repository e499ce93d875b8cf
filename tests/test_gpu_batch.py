"""GPU parity of the batch path: many uneven domains advanced by one launch
per step (through the vlb_batch_* C ABI) against the FP64 oracle, against
the single-domain path, and across launch shapes, task orders and graph
replay."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import check, field_errors, particle_errors, twin_errors

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


def ragged_cases():
    """Six small domains of uneven, ragged sizes (not multiples of the
    256-cell tile), different walls and properties; one has no particle,
    one has two, one holds its particle's temperature in a fluid that
    carries its own weight."""
    cases = []
    d = W.walls(W.domain(40, 97, tau_f=0.62, lambda_f=0.05, R_lambda=5.0,
                         R_cv=1.5, gravity=(0.0, -2e-5), beta=0.3,
                         coll_range=2.0, coll_stiff_pp=1e-3,
                         coll_stiff_pw=2e-3),
                thermal="dirichlet", T_wall=1.0)
    cases.append((d, [W.particle(20.3, 70.1, 6.5, rho_s=1.6, T_init=0.0,
                                 uy=-0.002)]))
    d = W.walls(W.domain(64, 128, tau_f=0.8, lambda_f=0.1, R_lambda=0.2,
                         R_cv=3.0, body_force=(2e-6, 0.0)), (2, 3))
    cases.append((d, [W.particle(31.7, 60.2, 9.0, rho_s=1.2, T_init=0.4,
                                 ux=0.01, omega=0.001)]))
    d = W.domain(33, 70, tau_f=0.7, lambda_f=0.08, R_lambda=3.0, R_cv=0.7,
                 init_u=(0.01, -0.005))
    cases.append((d, []))
    d = W.walls(W.domain(100, 61, tau_f=0.55, lambda_f=0.03, R_lambda=10.0,
                         R_cv=2.0, gravity=(0.0, -1e-5), beta=0.5,
                         coll_range=2.0, coll_stiff_pp=1e-3,
                         coll_stiff_pw=2e-3),
                thermal="adiabatic")
    cases.append((d, [W.particle(30.2, 30.5, 7.0, rho_s=1.5, T_init=0.0),
                      W.particle(70.9, 33.3, 5.5, rho_s=1.8, T_init=0.2,
                                 ux=-0.004)]))
    d = W.walls(W.domain(72, 203, tau_f=0.53, lambda_f=0.01, R_lambda=30.0,
                         R_cv=0.6, gravity=(0.0, -1e-5), beta=1.0),
                thermal="dirichlet", T_wall=[1.0, 1.0, 1.0, 0.0])
    cases.append((d, [W.particle(36.0, 150.4, 10.5, rho_s=1.3, T_init=0.0)]))
    d = W.walls(W.domain(56, 150, tau_f=0.6, lambda_f=0.04, R_lambda=2.0,
                         R_cv=1.5, gravity=(0.0, -2e-5), beta=0.4,
                         fluid_gravity=1, coll_range=2.0, coll_stiff_pp=1e-3,
                         coll_stiff_pw=2e-3),
                thermal="dirichlet", T_wall=1.0)
    cases.append((d, [W.particle(27.4, 100.2, 7.5, rho_s=1.4, T_init=0.0,
                                 hold_T=True)]))
    return cases


class _Got:
    """Batch read-outs of one domain behind the accessors the parity
    helpers use."""

    def __init__(self, fields, particles, ps):
        self._f, self._p, self._parts = fields, particles, ps

    def field(self, n):
        return self._f[n]

    def particles(self):
        return self._p


PKEYS = ("x", "y", "ux", "uy", "omega", "Fx", "Fy", "Tz")


def check_case(oracle_mod, o, got_fields, got_particles, d, ps, nsteps,
               precision):
    """FP64: the single-domain bar (1e-12, or 4x the spread of the oracle's
    FMA twin).  FP32: per-field errors on the same scales, reported and
    held to the FP32 bars."""
    g = _Got(got_fields, got_particles, ps)
    e = field_errors(g, o)
    if ps:
        e.update(particle_errors(g, o, PKEYS))
    if precision == "fp64":
        check(e, nsteps, twin=twin_errors(oracle_mod, d, ps, nsteps, o,
                                          pkeys=PKEYS if ps else None))
    else:
        bad = {k: v for k, v in e.items() if v >= FP32_BAR.get(k, 1e-5)}
        assert not bad, (bad, e)
    return e


# FP32 bar: 1e-5 of each quantity's scale (the same scales as at FP64)
FP32_BAR = {}


def batch_state(b, i, ps):
    return ({n: b.field(i, n) for n in FIELDS},
            b.particles(i) if ps else None)


def test_batch_matches_oracle_and_single_path_fp64(vlb, oracle_mod):
    cases = ragged_cases()
    n = 15
    b = vlb.Batch(cases, "fp64").init()
    say(f"batch of {len(b)} ragged domains, {b.cells} cells, {n} steps")
    b.step(n)
    for i, (d, ps) in enumerate(cases):
        say(f"domain {i}: {d['nx']} x {d['ny']}, {len(ps)} particles")
        f, p = batch_state(b, i, ps)
        o = oracle_mod.Oracle(d, ps).init().step(n)
        e = check_case(oracle_mod, o, f, p, d, ps, n, "fp64")
        say(f"  vs oracle: {e}")
        # the single-domain path: same task code, same results bit for bit
        s = vlb.Domain(d, ps, "fp64").init().step(n)
        for k in FIELDS:
            assert np.array_equal(s.field(k), f[k]), (i, k)
        if ps:
            ps_single = s.particles()
            for k in ("x", "y", "ux", "uy", "omega", "Fx", "Fy", "Tz"):
                assert np.array_equal(ps_single[k], p[k]), (i, k)
        s.close()
    b.close()


def run_tunings(vlb, cases, prec, tunings, n):
    """Fields and particles of every domain after n steps under each
    tuning (grid, order, graph, pair_min_tiles, waves)."""
    out = []
    for t in tunings:
        say(f"{prec} tuning grid={t[0]} order={t[1]} graph={t[2]} "
            f"pair_min_tiles={t[3]} waves={t[4]}")
        b = vlb.Batch(cases, prec).init()
        b.set_tuning(*t)
        got = b.tuning()
        assert (got["pair_min_tiles"], got["waves"]) == (t[3], t[4])
        b.step(n)
        out.append([batch_state(b, i, ps) for i, (d, ps) in enumerate(cases)])
        b.close()
    return out


def assert_same(runs, tunings):
    ref = runs[0]
    for got, t in zip(runs[1:], tunings[1:]):
        for i, ((f, p), (rf, rp)) in enumerate(zip(got, ref)):
            for k in FIELDS:
                assert np.array_equal(f[k], rf[k]), (t, i, k)
            if p is not None:
                for k in ("x", "y", "ux", "uy", "omega"):
                    assert np.array_equal(p[k], rp[k]), (t, i, k)


def test_batch_results_independent_of_tuning(vlb):
    """Launch shape, task order, per-domain tiling (one or two tiles per
    block), occupancy and graph replay change nothing: every tile is the
    same update_cell computation and partial sums are reduced in slot
    order.  The tile counts are 10, 16, 24, 32, 33 (odd: its last pair
    has one tile) and 58; pair_min_tiles 32 pairs the larger three."""
    cases = ragged_cases()
    n = 9     # first step single, then graph pairs, then the last single
    tunings = ((0, 0, False, -1, 0), (1024, 1, True, -1, 4),
               (16, 0, True, -1, 5), (8, 1, False, 0, 4),
               (1024, 1, True, 0, 5), (2048, 0, True, 32, 5),
               (0, 1, True, 33, 4))
    assert_same(run_tunings(vlb, cases, "fp32", tunings, n), tunings)


@pytest.mark.parametrize("prec", ["fp64", "bf16s"])
def test_batch_tilings_agree_in_other_forms(vlb, prec):
    """Paired and single tiles give the same bits in FP64 (whose paired
    kernel spills) and in a 16-bit form."""
    cases = ragged_cases()
    tunings = ((1024, 1, True, -1, 0), (1024, 1, True, 0, 4),
               (0, 0, True, 32, 0))
    assert_same(run_tunings(vlb, cases, prec, tunings, 7), tunings)


def test_batch_tuning_rejects_bad_values(vlb):
    cases = ragged_cases()[:2]
    b = vlb.Batch(cases, "fp64").init()
    for t in ((12, 0, True, -1, 0), (0, 2, True, -1, 0), (0, 0, True, -2, 0),
              (0, 0, True, -1, 3), (0, 0, True, -1, 5)):   # FP64: 4 waves
        with pytest.raises(vlb.VlbError):
            b.set_tuning(*t)
    b.close()


def test_batch_graph_replays_with_eager_work_between(vlb):
    """Graph replays separated by reads (eager work and synchronisations)
    give what one long run gives."""
    cases = ragged_cases()
    a = vlb.Batch(cases, "fp32").init()
    a.set_tuning(1024, 1, True)
    a.step(31)
    b = vlb.Batch(cases, "fp32").init()
    b.set_tuning(1024, 1, True)
    for k in (5, 8, 1, 6, 11):
        b.step(k)
        b.field(k % len(cases), "T")
        b.particles(0)
    for i, (d, ps) in enumerate(cases):
        for n in FIELDS:
            assert np.array_equal(a.field(i, n), b.field(i, n)), (i, n)
    a.close()
    b.close()


def test_c5_batch_autotuned_sample_matches_oracle(vlb, oracle_mod):
    """The 256 uneven single-particle domains in FP32 (autotuned, graph
    replay); eight seeded domains checked against the FP64 oracle at the
    FP32 bar."""
    cases = W.c5_batch()
    b = vlb.Batch(cases, "fp32")
    say(f"C5: {len(b)} domains, {b.cells} cells")
    b.init()
    t = b.autotune(3)
    say(f"autotune: {t}")
    assert t["grid_blocks"] % 8 == 0 and t["order"] in (0, 1)
    assert t["waves"] in (4, 5) and t["pair_min_tiles"] >= -1
    n = 10
    b.step(n)
    rng = np.random.default_rng(7)
    for i in sorted(rng.choice(len(cases), size=8, replace=False)):
        d, ps = cases[i]
        say(f"domain {i}: {d['nx']} x {d['ny']}, D = {2 * ps[0]['radius']:.1f}")
        f, p = batch_state(b, int(i), ps)
        o = oracle_mod.Oracle(d, ps).init().step(n)
        e = check_case(oracle_mod, o, f, p, d, ps, n, "fp32")
        say(f"  vs oracle: {e}")
    b.close()


def test_c5_sample_long_horizon_fp64(vlb, oracle_mod):
    """Four seeded C5 domains batched in FP64 over 1000 steps against the
    FP64 oracle at the single-domain bar (1e-12 of each scale, or 4x the
    spread of the oracle's FMA twin): the batch keeps parity over a run a
    hundred times longer than the ten steps above."""
    cases = W.c5_batch()
    rng = np.random.default_rng(11)
    pick = sorted(int(i) for i in rng.choice(len(cases), size=4,
                                              replace=False))
    sub = [cases[i] for i in pick]
    b = vlb.Batch(sub, "fp64")
    say(f"C5 sample {pick}: {b.cells} cells, FP64, 1000 steps")
    b.init()
    n = 1000
    b.step(n)
    for k, (d, ps) in enumerate(sub):
        f, p = batch_state(b, k, ps)
        o = oracle_mod.Oracle(d, ps).init().step(n)
        e = check_case(oracle_mod, o, f, p, d, ps, n, "fp64")
        say(f"  domain {pick[k]} ({d['nx']} x {d['ny']}): "
            f"worst {max(e.values()):.1e}")
    b.close()
