"""Replays of the paper's conjugate-heat sedimentation runs on the GPU in
FP64, against what the paper prints.

One cold particle with conjugate heat transfer (the section after Sec. 3.3; channel of width 4 D, D = 20
cells, density ratio 1.00232, Re = 10.5, Pr = 0.7, Gr = 1000):

  * R_lambda = 1: the minimal temperature inside the particle at
    t* = U_ref t / D = 2.625 for R_cv = 1, 2, 4 and 8;
  * R_cv = 8: the duration of the accelerating stage (t* of the maximum of
    U*_y = U_c,y / U_ref) and that maximum, for R_lambda = 1 and 1000 (and
    the trend through 10 and 100).

The GPU path is held to the oracle elsewhere; these runs check what the
method and the readings chosen where the paper is silent (the weighting of
the fluid force in solid cells, the simultaneous velocity-temperature
solve, the wall rules, the unprinted channel length) give for the paper's
own physical setup.  The paper's numbers come from its own code, sampling
and channel length, so they are held within margins, not to rounding: the
minimal temperature within 0.02 (measured: 0.0007 at R_cv = 1 growing to
0.015 at R_cv = 8, our particle slightly colder), the maximum of U*_y
within 3 % (measured +1.5 % and +1.9 %) and its time within 5 % (measured
-3.2 % and -0.9 %).  The channel length does not matter at t* = 2.625:
40 D, 60 D and 80 D give the same minimal temperature to four digits.

2048 cold particles in a 1700^2 adiabatic cavity (the paper's last
application): the whole run to t* = 420.81 (359,091 steps, 1.04e12 cell
updates, about 90 s).  The paper reports a left-right symmetric process up
to t* = 42.08 that is asymmetric at t* = 63.12, particles packing at the
bottom from t* ~ 126 on, and a space-average temperature of 0.5199 at the
end against the energy-balance value T_eq = 0.5145.  Here the asymmetry
(largest mirror-pair mismatch of the particle centres) is 4e-4 D at
t* = 42.08 and 13-19 D at 63.12; the lowest centre reaches the wall
(0.53 D) by t* = 72.  The space-average temperature at t* = 420.81 is
held within 0.01 of the energy-balance T_eq, the paper's own gap being
0.0054 (0.5199 against 0.5145).  The average of T equals T_eq only once
the field is uniform (T still spans 0.44 to 0.56 at the end), and the
energy sum_x c_v(x) T(x) is not an exact invariant once the disks move
(the oracle drifts by 2e-5 in 2000 steps of 12 moving disks); both are
reported.  The runs here end 0.0005 to 0.0017 from T_eq: the run is
chaotic, and a change of rounding (such as the order of a sum) gives
another realisation of the same statistics.

One cold particle of fixed temperature (Sec. 3.3; the temperature held by
the reading described with the held-temperature tests): channel of width
4 D, D = 20, start D / 2 left of the centre line, density ratio 1.00232,
Re = 40.5, Pr = 0.7, R_lambda = R_cv = 1, t* = 150 (148 k steps, the disk
falls about 85 D of a 180 D channel).  The paper's five regimes by Gr:
steady on the centre line (100), periodic about it (564), settling near one
wall (1000, 2000: x* = 2.91 and 2.74, other methods 2.76-2.91 and
2.62-2.74), steady on the centre line again (2500), and periodic about it
with a large amplitude (4500: 1.27).  Here: 100, 564, 1000, 2000 and 2500
give the first four regimes (x* = 2.84 and 2.85 near the wall), but at
4500 the oscillation dies out (half-range 0.016), a failing replay kept as
a strict expected failure; the large-amplitude regime sets in between Gr =
4500 and 5000 instead (half-range 1.30 at 5000 and 1.32 at 5500; at 4500 a
run to t* = 400 stays on the centre line).  Other readings of
the unstated rules were run on the GPU (Gr = 1000 / 2000 / 4500 / 6000):
every touched cell held fully gives x* = 2.78 / 2.80 and half-range 0.015 /
1.37; the cells whose node lies inside held fully, 2.78 / 2.87 and 0.024 /
0.99; the buoyancy applied inside the disk too (no (1 - f_s) weight), a
large amplitude at 4500 (0.93) but x* = 1.98 / 2.05, no wall regime.  The
reading kept (share-weighted hold, weighted force) is the closest on the
printed wall positions.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W


def say(msg):
    print(msg, flush=True)

pytestmark = pytest.mark.gpu

D = 20.0
TMIN_PRINTED = {1.0: 0.841, 2.0: 0.656, 4.0: 0.399, 8.0: 0.162}
ACCEL_PRINTED = {1.0: (2.032, 0.818), 1000.0: (1.614, 0.928)}


@pytest.fixture(scope="module")
def vlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_23802_amd import vlb as v
    v.lib()  # fails loudly if the HIP library is missing
    return v


def u_ref(d):
    return W.u_ref(1.00232, d["gravity"][1], D)


def dump(name, rec):
    out = os.environ.get("VLB_REPLAY_OUT")
    if out:
        os.makedirs(out, exist_ok=True)
        with open(os.path.join(out, f"replay_{name}.json"), "w") as fh:
            json.dump(rec, fh, indent=1)


def min_temperature_at(vlb, R_lambda, R_cv, t_star, length_D=60):
    d, ps = W.e6_cht_channel(R_lambda, R_cv, length_D=length_D)
    steps = int(round(t_star * D / u_ref(d)))
    dom = vlb.Domain(d, ps, "fp64").init()
    dom.step(steps)
    p = dom.particles()
    dom.close()
    return float(p["T_min"][0]), steps


def velocity_history(vlb, R_lambda, R_cv, t_end, every=10):
    d, ps = W.e6_cht_channel(R_lambda, R_cv)
    U = u_ref(d)
    steps = int(round(t_end * D / U))
    dom = vlb.Domain(d, ps, "fp64").init()
    t, u = [], []
    done = 0
    while done < steps:
        dom.step(every)
        done += every
        p = dom.particles()
        t.append(U * done / D)
        u.append(-float(p["uy"][0]) / U)
    dom.close()
    return np.array(t), np.array(u)


def test_min_particle_temperature_vs_printed(vlb):
    got = {}
    for R_cv, printed in TMIN_PRINTED.items():
        T, steps = min_temperature_at(vlb, 1.0, R_cv, 2.625)
        got[R_cv] = T
        print(f"R_cv = {R_cv:g}: min T at t* = 2.625 ({steps} steps) "
              f"{T:.4f}, printed {printed}", flush=True)
    # the channel length the paper leaves open: 40 D and 80 D at R_cv = 2
    sens = {L: min_temperature_at(vlb, 1.0, 2.0, 2.625, length_D=L)[0]
            for L in (40, 80)}
    print(f"R_cv = 2, channel 40 D / 60 D / 80 D: {sens[40]:.4f} / "
          f"{got[2.0]:.4f} / {sens[80]:.4f}", flush=True)
    assert all(abs(v - got[2.0]) <= 1e-3 for v in sens.values()), sens
    dump("min_temperature", {"t_star": 2.625, "R_lambda": 1.0,
                             "got": got, "printed": TMIN_PRINTED,
                             "length_sensitivity_R_cv_2": sens})
    vals = [got[k] for k in sorted(got)]
    assert all(a > b for a, b in zip(vals, vals[1:])), got
    for R_cv, printed in TMIN_PRINTED.items():
        assert abs(got[R_cv] - printed) <= 0.02, (R_cv, got[R_cv], printed)


def test_accelerating_stage_vs_printed(vlb):
    rows = {}
    for R_lambda in (1.0, 10.0, 100.0, 1000.0):
        t, u = velocity_history(vlb, R_lambda, 8.0, 4.0)
        k = int(np.argmax(u))
        rows[R_lambda] = (float(t[k]), float(u[k]))
        pr = ACCEL_PRINTED.get(R_lambda)
        print(f"R_lambda = {R_lambda:g}, R_cv = 8: max U* {u[k]:.4f} at "
              f"t* {t[k]:.3f}" + (f", printed {pr[1]} at {pr[0]}" if pr else ""),
              flush=True)
    dump("accelerating_stage", {"R_cv": 8.0, "got": rows,
                                "printed": ACCEL_PRINTED})
    lam = sorted(rows)
    dur = [rows[k][0] for k in lam]
    umax = [rows[k][1] for k in lam]
    # the printed trends: shorter accelerating stage, higher maximum
    assert all(a >= b for a, b in zip(dur, dur[1:])), rows
    assert all(a <= b for a, b in zip(umax, umax[1:])), rows
    for R_lambda, (t_p, u_p) in ACCEL_PRINTED.items():
        t_g, u_g = rows[R_lambda]
        assert abs(u_g - u_p) <= 0.03 * u_p, (R_lambda, u_g, u_p)
        assert abs(t_g - t_p) <= 0.05 * t_p, (R_lambda, t_g, t_p)


def test_dense_cavity_replay(vlb):
    d, ps = W.e7_cht_cavity()
    Dc, L = 24.0, d["nx"]
    U = W.u_ref(1.5, d["gravity"][1], Dc)
    phi = len(ps) * np.pi * (Dc / 2) ** 2 / (L * L)
    T_eq = (1 - phi) / ((1 - phi) + 2.0 * phi)   # R_cv = 2, T_c = 0, T_h = 1
    checkpoints = (42.08, 63.12, 126.24, 420.81)
    # mirror partner of each disk: same row, column 63 - j
    mirror = np.array([(k // 64) * 64 + 63 - (k % 64) for k in range(len(ps))])
    cvf, cvs = d["cv_f"], d["cv_f"] * d["R_cv"]

    def energy(dom):
        fs = dom.field("fs")
        return float(np.sum((cvf * (1.0 - fs) + cvs * fs) * dom.field("T")))

    dom = vlb.Domain(d, ps, "fp64").init()
    E0 = energy(dom)
    done, rec = 0, {}
    for ts in checkpoints:
        n = int(round(ts * Dc / U)) - done
        dom.step(n)
        done += n
        p = dom.particles()
        T = dom.field("T")
        asym = max(np.abs(p["x"] + p["x"][mirror] - L).max(),
                   np.abs(p["y"] - p["y"][mirror]).max()) / Dc
        rec[ts] = {"steps": done, "asym_D": float(asym),
                   "y_min_D": float(p["y"].min() / Dc),
                   "T_mean": float(T.mean()), "T_min": float(T.min()),
                   "T_max": float(T.max()), "energy_rel": energy(dom) / E0 - 1.0}
        print(f"t* = {ts}: {rec[ts]}", flush=True)
    dom.close()
    dump("dense_cavity", {"T_eq": T_eq, "printed_T_mean": 0.5199,
                          "checkpoints": rec})
    assert rec[42.08]["asym_D"] < 1e-2, rec[42.08]
    assert rec[63.12]["asym_D"] > 1e-2, rec[63.12]
    assert rec[126.24]["y_min_D"] < 0.6, rec[126.24]
    assert abs(rec[420.81]["T_mean"] - T_eq) < 0.01, (rec[420.81], T_eq)


E5_GATES = {
    # Gr: (regime, printed x* or amplitude, gate); Gr = 4500 has its own
    # test below (a failing replay under this library's readings)
    100.0: ("centre", None, None),
    564.0: ("centre_periodic", None, None),
    1000.0: ("wall", 2.91, 0.12),
    2000.0: ("wall", 2.74, 0.15),
    2500.0: ("centre", None, None),
}


def held_run(vlb, Gr, t_end=150.0, every=100):
    d, ps = W.e5_held_channel(Gr)
    U = W.u_ref(1.00232, d["gravity"][1], D)
    steps = int(round(t_end * D / U))
    dom = vlb.Domain(d, ps, "fp64").init()
    t, x = [], []
    done = 0
    while done < steps:
        dom.step(every)
        done += every
        p = dom.particles()
        t.append(U * done / D)
        x.append(float(p["x"][0]) / D)
    dom.close()
    t, x = np.array(t), np.array(x)
    late = x[t > 0.6 * t_end]
    return {"steps": steps, "x_late_mean": float(late.mean()),
            "amplitude": float(0.5 * (late.max() - late.min()))}


def test_fixed_temperature_regimes(vlb):
    rows = {}
    for Gr, (regime, printed, gate) in E5_GATES.items():
        r = held_run(vlb, Gr)
        rows[Gr] = r
        print(f"Gr = {Gr:g}: late x* mean {r['x_late_mean']:.3f}, amplitude "
              f"{r['amplitude']:.3f} ({regime}"
              + (f", printed {printed}" if printed else "") + ")", flush=True)
    dump("fixed_temperature", {"t_end_star": 150.0, "rows": rows,
                               "printed": {1000: 2.91, 2000: 2.74,
                                           4500: 1.27}})
    for Gr, (regime, printed, gate) in E5_GATES.items():
        r = rows[Gr]
        off = abs(r["x_late_mean"] - 2.0)
        if regime == "centre":
            assert off < 0.05 and r["amplitude"] < 0.05, (Gr, r)
        elif regime == "centre_periodic":
            assert off < 0.05 and 0.005 < r["amplitude"] < 0.2, (Gr, r)
        elif regime == "wall":
            assert r["amplitude"] < 0.1, (Gr, r)
            assert abs(off - (printed - 2.0)) < gate, (Gr, r, printed)


@pytest.mark.xfail(strict=True, reason=(
    "Table 4's large-amplitude regime at Gr = 4500 (amplitude 1.27) is not "
    "reproduced: the oscillation dies out (half-range 0.016) and appears at "
    "Gr = 6000 instead.  Holding every touched cell fully, or the cells "
    "whose node lies inside, changes neither; applying the buoyancy inside "
    "the disk too brings it back at 4500 (0.93) but loses the wall regimes "
    "of Gr = 1000 and 2000.  The paper does not give its hold rule."))
def test_fixed_temperature_large_amplitude_at_printed_gr(vlb):
    """Sec. 3.3, Table 4: at Gr = 4500 the particle oscillates about the
    centre line with the amplitude 1.27 (x* = x / D)."""
    r = held_run(vlb, 4500.0)
    print(f"Gr = 4500: late x* mean {r['x_late_mean']:.3f}, amplitude "
          f"{r['amplitude']:.3f} (printed 1.27)", flush=True)
    assert abs(r["amplitude"] - 1.27) < 0.3, r


# --------------------------------------------------------------------------
# Sec. 3.2: the isothermal sedimentation of an elliptical particle


def ellipse_track(vlb, tau_f, situation, steps, every=1000):
    d, ps = W.e4_ellipse_channel(tau_f, situation)
    dom = vlb.Domain(d, ps, "fp64").init()
    L, y0 = float(d["nx"]), ps[0]["y"]
    tr = []
    for _ in range(steps // every):
        dom.step(every)
        p = dom.particles()[0]
        tr.append(((y0 - p["y"]) / L, p["x"] / L, p["theta"] / math.pi))
    dom.close()
    return np.array(tr)


def test_ellipse_sedimentation_settles_broadside_on_the_centre_line(vlb):
    """The ellipse of Sec. 3.2 (semi-axes 13 and 6.5 cells in a channel of
    104, density ratio 1.1, tau_f = 0.6, starting on the centre line at
    theta = pi/4).  The paper describes the path: at first it swings
    towards the left wall while it turns, then it settles along the
    centre line with its orientation tending to zero.  Measured: the
    centre comes to x/L = 0.369 after falling 0.63 L, theta passes zero
    and overshoots to -0.10 pi, and after 18.6 L of fall x/L = 0.499 with
    |theta| < 0.005 pi.  Gates: the swing reaches x/L < 0.42 within the
    first 2 L of fall, and over the last 3 L the centre stays within
    0.01 L of the centre line and |theta| below 0.02 pi.  (The FEM path the
    paper compares with is not available.)"""
    tr = ellipse_track(vlb, 0.6, 0, 120_000)
    fall, x, th = tr[:, 0], tr[:, 1], tr[:, 2]
    early = fall < 2.0
    say(f"ellipse tau_f = 0.6: fell {fall[-1]:.2f} L; swing to x/L = "
        f"{x[early].min():.3f}; theta/pi from {th[0]:.3f} to {th[-1]:.4f} "
        f"(min {th.min():.3f}); end x/L = {x[-1]:.4f}")
    assert fall[-1] > 15.0
    assert x[early].min() < 0.42
    late = fall > fall[-1] - 3.0
    assert np.abs(x[late] - 0.5).max() < 0.01
    assert np.abs(th[late]).max() < 0.02


def test_ellipse_situations_one_and_two_agree(vlb):
    """Sec. 3.2 repeats the run with the fluid carrying its own weight
    (situation II, from a hydrostatic start) against the fluid free of body
    force (situation I), both at tau_f = 0.515, and finds no
    distinguishable difference in the trajectory or the orientation.  Here
    the two paths, as x/L and theta/pi against the fall, differ by at most
    0.02 L and 0.02 pi over the first 4 L of fall (measured 0.0015 L and
    0.003 pi)."""
    a = ellipse_track(vlb, 0.515, 0, 200_000)
    b = ellipse_track(vlb, 0.515, 1, 200_000)
    span = min(a[-1, 0], b[-1, 0], 4.0)
    s = np.linspace(0.05, span, 200)
    dx = np.abs(np.interp(s, a[:, 0], a[:, 1]) - np.interp(s, b[:, 0], b[:, 1]))
    dth = np.abs(np.interp(s, a[:, 0], a[:, 2]) - np.interp(s, b[:, 0], b[:, 2]))
    say(f"ellipse situations I / II over {span:.2f} L of fall: max "
        f"|dx| = {dx.max():.4f} L, max |dtheta| = {dth.max():.4f} pi; swings "
        f"to x/L = {a[:, 1].min():.3f} / {b[:, 1].min():.3f}")
    assert span > 3.5
    assert dx.max() < 0.02 and dth.max() < 0.02
