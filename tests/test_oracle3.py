"""Pins of the three-dimensional oracle (D3Q19 flow, D3Q7 energy, spheres;
the paper's extension to three dimensions, Sec. 2) against what the
mathematics fixes:

- the exact sphere-cell volume: closed forms (a sphere inside one cell, a
  sphere centred on a lattice point, a spherical cap), the ball's volume
  over the grid, an independent integration in the other order (the
  z-chord over x and y by scipy), symmetries, and the band and inside
  readings;
- the flow: mass conservation with moving spheres, the momentum budget
  (the fluid's momentum changes by minus the momentum-exchange forces),
  the exact Poiseuille parabola with the two-relaxation-time bounce-back
  slip, the linear Couette profile;
- the energy: the uniform-temperature invariant with moving spheres of a
  different heat capacity, energy conservation between adiabatic walls,
  the exact piecewise-linear conduction across a layered slab with
  unequal conductivity and heat capacity;
- the particle coupling: the first steps of a spinning, translating sphere
  in closed form (momentum exchange of the streamed equilibrium start,
  V = 4 pi R^3/3, I = 2 M R^2/5, the inside-fluid terms).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W

# D3Q19 in the oracle's order, for the closed forms below
C19 = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                (0, 0, 1), (0, 0, -1), (1, 1, 0), (-1, -1, 0), (1, -1, 0),
                (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
                (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)], dtype=float)
W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def feq19(rho, u):
    """Textbook D3Q19 equilibria on fields: u (3, ...) -> (19, ...)."""
    eu = np.tensordot(C19, u, axes=1)
    u2 = (u * u).sum(axis=0)
    w = W19.reshape((19,) + (1,) * u2.ndim)
    return w * rho * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * u2)


def stream_periodic(f):
    return np.stack([np.roll(f[q], (int(C19[q, 2]), int(C19[q, 1]),
                                    int(C19[q, 0])), axis=(0, 1, 2))
                     for q in range(19)])


def boundary_cells(X, Y, Z, R, rng, n):
    out = []
    while len(out) < n:
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        p = np.array([X, Y, Z]) + R * v
        out.append(tuple(int(math.floor(c)) for c in p))
    return out


# ---- geometry -------------------------------------------------------------

def test_volume_closed_forms(oracle3_mod):
    O = oracle3_mod
    # a small sphere wholly inside one cell
    assert abs(O.sphere_cell_volume(3.5, 2.4, 7.6, 0.3, 3, 2, 7)
               - 4 / 3 * math.pi * 0.027) < 1e-15
    # centred on a lattice point: each of the eight cells holds an eighth
    for i in (-1, 0):
        for j in (-1, 0):
            for k in (-1, 0):
                v = O.sphere_cell_volume(5.0, 6.0, 7.0, 0.8, 5 + i, 6 + j,
                                         7 + k)
                assert abs(v - math.pi * 0.512 / 6) < 1e-15
    # a cap: the plane z = 1 cuts the sphere 0.1 above its centre
    R, h = 0.4, 0.5
    cap = math.pi * h * h * (3 * R - h) / 3   # the part above z = 1
    below = O.sphere_cell_volume(0.5, 0.5, 0.9, R, 0, 0, 0)
    above = O.sphere_cell_volume(0.5, 0.5, 0.9, R, 0, 0, 1)
    assert abs(above - math.pi * 0.3 ** 2 * (3 * R - 0.3) / 3) < 1e-15
    assert abs(below + above - 4 / 3 * math.pi * R ** 3) < 1e-15
    del cap


@pytest.mark.parametrize("seed", range(4))
def test_volumes_add_up_to_the_ball(oracle3_mod, seed):
    O = oracle3_mod
    rng = np.random.default_rng(seed)
    R = rng.uniform(1.0, 5.0)
    X, Y, Z = rng.uniform(10, 11, 3)
    r = range(int(X - R) - 2, int(X + R) + 3)
    tot = sum(O.sphere_cell_volume(X, Y, Z, R, i, j, k)
              for i in r for j in range(int(Y - R) - 2, int(Y + R) + 3)
              for k in range(int(Z - R) - 2, int(Z + R) + 3))
    assert abs(tot - 4 / 3 * math.pi * R ** 3) < 2e-13 * R ** 3, tot


def other_order_volume(X, Y, Z, R, i, j, k):
    """The ball's z-chord inside [k, k+1], integrated over y and then x by
    adaptive quadrature split where the chord's regime changes (the
    circle of the ball's section at the planes z = k, k + 1 and at its
    equator, and the lines y = j, j + 1)."""
    cz = [0.0, k - Z, k + 1.0 - Z]

    def chord(y, x):
        h2 = R * R - (x - X) ** 2 - (y - Y) ** 2
        if h2 <= 0:
            return 0.0
        h = math.sqrt(h2)
        return max(0.0, min(Z + h, k + 1.0) - max(Z - h, float(k)))

    def inner(x):
        pts = []
        for c in cz:
            r2 = R * R - c * c - (x - X) ** 2
            if r2 > 0:
                pts += [Y - math.sqrt(r2), Y + math.sqrt(r2)]
        pts = sorted(p for p in pts if j < p < j + 1)
        return integrate.quad(chord, j, j + 1, args=(x,), points=pts or None,
                              epsabs=1e-15, epsrel=1e-14, limit=200)[0]

    pts = []
    for c in cz:
        for e in (0.0, j - Y, j + 1.0 - Y):
            r2 = R * R - c * c - e * e
            if r2 > 0:
                pts += [X - math.sqrt(r2), X + math.sqrt(r2)]
    pts = sorted(p for p in pts if i < p < i + 1)
    return integrate.quad(inner, i, i + 1, points=pts or None, epsabs=1e-15,
                          epsrel=1e-14, limit=200)[0]


def test_volume_against_the_other_integration_order(oracle3_mod):
    """The oracle integrates cross-sectional areas over z; here the
    z-chord of the ball is integrated over y and x."""
    O = oracle3_mod
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(6):
        R = rng.uniform(1.2, 6.0)
        X, Y, Z = rng.uniform(20, 21, 3)
        for i, j, k in boundary_cells(X, Y, Z, R, rng, 2):
            ref = other_order_volume(X, Y, Z, R, i, j, k)
            worst = max(worst, abs(ref - O.sphere_cell_volume(X, Y, Z, R, i,
                                                              j, k)))
    assert worst < 1e-12, worst


def test_volume_symmetries_and_readings(oracle3_mod):
    O = oracle3_mod
    rng = np.random.default_rng(5)
    w = 0.0
    for _ in range(30):
        R = rng.uniform(0.7, 6.0)
        X, Y, Z = rng.uniform(30, 31, 3)
        for i, j, k in boundary_cells(X, Y, Z, R, rng, 3):
            v = O.sphere_cell_volume(X, Y, Z, R, i, j, k)
            # permuting the axes, mirroring x about the centre
            w = max(w, abs(v - O.sphere_cell_volume(Y, Z, X, R, j, k, i)))
            w = max(w, abs(v - O.sphere_cell_volume(-X, Y, Z, R, -i - 1, j,
                                                    k)))
            assert O.cell_in_band(X, Y, Z, R, i, j, k) or v == 0.0
            if O.cell_inside(X, Y, Z, R, i, j, k):
                assert abs(v - 1.0) < 1e-14
    assert w < 1e-14, w


# ---- flow -----------------------------------------------------------------

def moving_box():
    d = W.domain3(20, 18, 16, tau_f=0.7, lambda_f=0.05, R_lambda=3.0,
                  R_cv=2.0, init_T=0.6)
    ps = [W.sphere(6.3, 7.1, 8.2, 3.4, rho_s=1.5, T_init=0.1,
                   u=(0.01, 0.004, -0.006), omega=(0.002, -0.003, 0.004)),
          W.sphere(14.2, 11.7, 7.4, 2.6, rho_s=0.8, T_init=0.9,
                   u=(-0.008, 0.005, 0.007), omega=(-0.004, 0.001, 0.002))]
    return d, ps


def test_mass_and_momentum_budget_periodic(oracle3_mod):
    """Mass is conserved exactly; with no body force the fluid's momentum
    changes by minus the sum of the momentum-exchange forces."""
    O = oracle3_mod
    d, ps = moving_box()
    o = O.Oracle3(d, ps).init()
    C = C19.T[:, :, None, None, None]
    m0 = o.field("f").sum()
    worst_m = worst_p = 0.0
    for _ in range(12):
        P0 = (C * o.field("f")).sum(axis=(1, 2, 3, 4))
        o.step(1)
        f = o.field("f")
        P1 = (C * f).sum(axis=(1, 2, 3, 4))
        p = o.particles()
        F = np.array([p["Fx"].sum(), p["Fy"].sum(), p["Fz"].sum()])
        scale = p["F_abs"].sum()
        worst_p = max(worst_p, np.abs(P1 - P0 + F).max() / scale)
        worst_m = max(worst_m, abs(f.sum() - m0) / m0)
        assert np.abs(F).max() > 1e-6
    assert worst_m < 1e-14, worst_m
    assert worst_p < 1e-14, worst_p


def test_poiseuille_between_plates(oracle3_mod):
    """Force-driven flow between halfway bounce-back walls at z: the exact
    parabola with the two-relaxation-time slip of Lambda = 1/12,
    u(z) = F/(2 nu) [z (H - z) + (16 Lambda - 3)/12]."""
    O = oracle3_mod
    tau, F, H = 0.8, 1e-6, 16
    nu = (tau - 0.5) / 3
    d = W.walls3(W.domain3(2, 2, H, tau_f=tau, body_force=(F, 0.0, 0.0)),
                 (W.ZLO, W.ZHI))
    o = O.Oracle3(d, []).init()
    o.step(15000)
    u = o.field("ux")[:, 0, 0]
    z = np.arange(H) + 0.5
    ref = F / (2 * nu) * (z * (H - z) + (16 / 12 - 3) / 12)
    assert np.abs(u - ref).max() < 1e-10 * ref.max()
    # rounding only (the density drifts by about one ulp per step)
    assert np.abs(o.field("uz")).max() < 1e-13
    assert np.abs(o.field("uy")).max() < 1e-13


def test_couette_between_plates(oracle3_mod):
    O = oracle3_mod
    H, Uw = 12, 1e-4
    d = W.walls3(W.domain3(2, 2, H, tau_f=0.9), (W.ZLO, W.ZHI))
    d["u_wall"][W.ZHI] = (0.0, Uw, 0.0)
    o = O.Oracle3(d, []).init()
    o.step(8000)
    z = np.arange(H) + 0.5
    assert np.abs(o.field("uy")[:, 0, 0] - Uw * z / H).max() < 1e-13


# ---- energy ---------------------------------------------------------------

def test_uniform_temperature_stays_uniform(oracle3_mod):
    """Moving, spinning spheres of another heat capacity in fluid at the
    same temperature: T stays uniform (the invariant the paper's choice of
    the source weight secures, Appendix A, carried to three dimensions)."""
    O = oracle3_mod
    d, ps = moving_box()
    d["init_T"] = 0.45
    for p in ps:
        p["T_init"] = 0.45
    o = O.Oracle3(d, ps).init().step(30)
    assert np.abs(o.field("T") - 0.45).max() < 1e-13
    p = o.particles()
    assert np.abs(p["T_mean"] - 0.45).max() < 1e-13


def test_energy_conserved_between_adiabatic_walls(oracle3_mod):
    """A fixed cold sphere in warm fluid in a closed adiabatic box: the
    total internal energy sum c_v T is conserved every step."""
    O = oracle3_mod
    d = W.walls3(W.domain3(12, 12, 12, lambda_f=0.08, R_lambda=5.0,
                           R_cv=2.0, init_T=1.0), thermal="adiabatic")
    ps = [W.sphere(6.2, 5.8, 6.1, 3.1, T_init=0.0, fixed=True)]
    o = O.Oracle3(d, ps).init()
    cvs = 2.0

    def energy():
        fs = o.field("fs")
        return (((1 - fs) + fs * cvs) * o.field("T")).sum()
    e0 = energy()
    for _ in range(40):
        o.step(1)
        assert abs(energy() - e0) < 1e-12 * e0
    assert abs(o.field("T") - o.field("T").mean()).max() > 1e-3  # still mixing


@pytest.mark.parametrize("Rl,Rcv,rule", [(10.0, 2.0, 0), (0.25, 3.0, 0),
                                         (4.0, 0.5, 1)])
def test_layered_slab_conduction(oracle3_mod, Rl, Rcv, rule):
    """Solid layers k < 10, fluid above, Dirichlet T = 1 / 0 on the z
    faces, no flow: the steady state is piecewise linear with continuous T
    and flux (the conjugate condition), exactly."""
    O = oracle3_mod
    nz, ks, lam = 26, 10, 0.1
    d = W.domain3(2, 2, nz, lambda_f=lam, R_lambda=Rl, R_cv=Rcv,
                  sigma_rule=rule)
    d = W.walls3(d, (W.ZLO, W.ZHI), thermal="dirichlet",
                 T_wall=[0, 0, 0, 0, 1.0, 0.0])
    o = O.Oracle3(d, [], hooks={"thermal_only": 1, "fs_from_array": 1,
                                "u_pres": (0.0, 0.0, 0.0)})
    z = np.arange(nz)
    o.raw("fs_next")[...] = (z < ks).astype(float)[:, None, None]
    o.raw("T")[...] = 0.5
    o.init()
    o.step(60000)
    ls = lam * Rl
    Ti = (ls / ks) / (ls / ks + lam / (nz - ks))
    zc = z + 0.5
    Ta = np.where(zc < ks, 1 + (Ti - 1) * zc / ks, Ti * (nz - zc) / (nz - ks))
    assert np.abs(o.field("T")[:, 1, 0] - Ta).max() < 1e-10


# ---- particle coupling ----------------------------------------------------

def test_spinning_sphere_first_steps_closed_form(oracle3_mod):
    """A sphere released spinning and translating in fluid at rest.  Step 1:
    its forces are zero and U^1 = U^0, Omega^1 = Omega^0, X^1 = X^0 + U^0;
    the momentum exchange is that of the streamed equilibrium start,
    F = -sum f_s (rho u_s - j*), T = -sum (x - X) x f_s (rho u_s - j*) with
    u_s = U + Omega x (x - X).  Step 2: U^2 = U^1 + F^1/M,
    Omega^2 = Omega^1 + T^1/I with M = rho_s 4 pi R^3/3, I = 2 M R^2/5."""
    O = oracle3_mod
    n, R, rs = (22, 20, 18), 4.3, 1.7
    X0 = np.array([10.7, 9.2, 8.9])
    U0 = np.array([0.011, -0.006, 0.004])
    Om0 = np.array([0.003, -0.002, 0.005])
    d = W.domain3(*n, tau_f=0.75, R_cv=2.0, R_lambda=3.0)
    ps = [W.sphere(*X0, R, rho_s=rs, u=U0, omega=Om0)]
    o = O.Oracle3(d, ps).init()
    fs0 = o.field("fs")
    zz, yy, xx = np.meshgrid(*(np.arange(m) + 0.5 for m in n[::-1]),
                             indexing="ij")
    r = np.stack([xx - X0[0], yy - X0[1], zz - X0[2]])
    us = U0[:, None, None, None] + np.cross(Om0, r, axis=0)
    f0 = feq19(1.0, fs0 * us)
    assert np.abs(o.field("f") - f0).max() < 1e-15

    o.step(1)
    p = o.particles()[0]
    X1 = X0 + U0
    assert abs(p["x"] - X1[0]) < 1e-14 and abs(p["z"] - X1[2]) < 1e-14
    assert (p["ux"], p["uy"], p["uz"]) == tuple(U0)
    assert (p["ox"], p["oy"], p["oz"]) == tuple(Om0)
    assert abs(p["fs_sum"] - 4 / 3 * math.pi * R ** 3) < 1e-11
    fst = stream_periodic(f0)
    rho = fst.sum(axis=0)
    j = np.tensordot(C19.T, fst, axes=1)
    r1 = np.stack([xx - X1[0], yy - X1[1], zz - X1[2]])
    us1 = U0[:, None, None, None] + np.cross(Om0, r1, axis=0)
    fs1 = o.field("fs")
    dP = fs1 * (rho * us1 - j)
    F = -dP.sum(axis=(1, 2, 3))
    T = -np.cross(r1, dP, axis=0).sum(axis=(1, 2, 3))
    scale = p["F_abs"]
    for k, key in enumerate(("Fx", "Fy", "Fz")):
        assert abs(p[key] - F[k]) < 1e-14 * scale, key
    for k, key in enumerate(("Tx", "Ty", "Tz")):
        assert abs(p[key] - T[k]) < 1e-14 * scale * R, key
    assert np.abs(T).max() > 1e-3 * np.abs(F).max() * R   # the spin is felt
    assert np.dot(T, Om0) < 0                              # and opposed

    M = rs * 4 / 3 * math.pi * R ** 3
    I = 0.4 * M * R * R
    o.step(1)
    p2 = o.particles()[0]
    for k, (uk, ok) in enumerate((("ux", "ox"), ("uy", "oy"), ("uz", "oz"))):
        assert abs(p2[uk] - (U0[k] + p[("Fx", "Fy", "Fz")[k]] / M)) < 1e-17
        assert abs(p2[ok] - (Om0[k] + p[("Tx", "Ty", "Tz")[k]] / I)) < 1e-17
    # step 3: the inside-fluid terms enter (M_in = rho_f V, I_in = I/rho_s)
    o.step(1)
    p3 = o.particles()[0]
    Min, Iin = M / rs, I / rs
    U3 = p2["ux"] + (p2["Fx"] + Min * (p2["ux"] - U0[0])) / M
    O3z = p2["oz"] + (p2["Tz"] + Iin * (p2["oz"] - Om0[2])) / I
    assert abs(p3["ux"] - U3) < 1e-17
    assert abs(p3["oz"] - O3z) < 1e-17


@pytest.mark.parametrize("U", [0.0, 0.02])
def test_advected_sine_decays_and_travels(oracle3_mod, U):
    """A temperature sine along x in a periodic box, the velocity prescribed
    (thermal-only, no solid): it decays at the rate kappa k^2 with
    kappa = lambda/(rho_f c_v) (eq. lambda) and travels with the flow (the
    convection term as a source, Sec. 2.2); both to the lattice's
    O(k^2) accuracy on a 64-cell wavelength."""
    O = oracle3_mod
    L, lam, cv, t = 64, 0.05, 1.0, 400
    d = W.domain3(L, 2, 2, lambda_f=lam, cv_f=cv, R_cv=1.0, R_lambda=1.0)
    o = O.Oracle3(d, [], hooks={"thermal_only": 1, "fs_from_array": 1,
                                "u_pres": (U, 0.0, 0.0)})
    x = np.arange(L) + 0.5
    k = 2 * math.pi / L
    o.raw("fs_next")[...] = 0.0
    o.raw("T")[...] = (1 + 0.1 * np.sin(k * x))[None, None, :]
    o.init()
    o.step(t)
    T = o.field("T")[0, 0] - 1
    c = np.exp(-1j * k * x)
    amp = 2 * abs((T * c).mean())
    phase = -np.angle((T * c).mean() * 1j)       # k * shift
    kappa = lam / cv
    assert abs(amp / 0.1 - math.exp(-kappa * k * k * t)) < 2e-3
    assert abs(phase / k - U * t) < 0.02 * max(U * t, 1.0)


def test_two_dimensional_energy_collision_is_the_two_rate_form():
    """The reading behind the D3Q7 energy collision: with the paper's
    parameters (alpha_1 = -2, alpha_2 = 1, beta_1 = -4, beta_2 = 4,
    sigma_q = sigma_j, sigma_epsilon = sigma_e) the D2Q9 MRT energy
    collision of eq. lbe.e.col equals relaxing the even part of g - g^eq at
    sigma_e and the odd part at sigma_j, with g^eq_i = w_i c_ref T (i > 0),
    g^eq_0 = epsilon - (1 - w_0) c_ref T, plus (1 - sigma_e/2) q_c on the
    rest population, whatever sigma_0."""
    import numpy_step as NS
    rng = np.random.default_rng(3)
    opp = NS.OPP
    for _ in range(20):
        g = rng.uniform(0.0, 0.3, 9)
        qc, cref = rng.uniform(-0.01, 0.01), rng.uniform(0.5, 2.0)
        sj, se, s0 = rng.uniform(0.6, 1.9, 3)
        T = rng.uniform(0.2, 1.0)
        eps = g.sum() + 0.5 * qc                     # eq. e
        n = NS.MT @ g
        neq = NS.energy_eq_moments(np.array(eps), np.array(T), cref)
        Rd = np.array([s0, se, se, sj, sj, sj, sj, se, se])
        src = np.array([qc, -4 * qc, 4 * qc, 0, 0, 0, 0, 0, 0])
        mrt = NS.MTI @ (n - Rd * (n - neq) + (1 - Rd / 2) * src)
        geq = NS.WGT * cref * T
        geq[0] = eps - (1 - NS.WGT[0]) * cref * T
        ev, od = 0.5 * (g + g[opp]), 0.5 * (g - g[opp])
        trt = g - se * (ev - 0.5 * (geq + geq[opp])) - sj * od
        trt[0] += (1 - se / 2) * qc
        assert np.abs(mrt - trt).max() < 4e-15 * np.abs(mrt).max()
