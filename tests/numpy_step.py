"""A second, independent transcription of the method's time step in numpy
(test infrastructure: it checks the C oracle, nothing else uses it).

It is written from the paper's definitions in a form of its own, so that a
slip in the C oracle's arithmetic shows as a disagreement:

- the D2Q9 transformation matrix is built from its defining polynomials of
  the velocities (1, -4 + 3|e|^2, 4 - 21|e|^2/2 + 9|e|^4/2, e_x,
  (-5 + 3|e|^2) e_x, e_y, (-5 + 3|e|^2) e_y, e_x^2 - e_y^2, e_x e_y;
  Sec. 2.1) rather than taken as printed, and inverted numerically;
- the flow equilibrium is the textbook second-order D2Q9 distribution and
  its moments are obtained by multiplying with that matrix; the discrete
  force term is Guo's velocity-space term, taken to moment space the same
  way (eq. lbe.rho.col);
- the solid fraction of a cell is the area of the particle inside it by
  adaptive quadrature of the chord length over x (scipy), between the
  points where the boundary crosses the cell's edges (Sec. 2, Fig. 1);
- the coupled temperature and velocity of a cell (Sec. 2.2 with u from
  eq. rho.rhou) are found as the root of the energy relation, which is
  linear in T, from its residual at two temperatures;
- streaming is done on whole arrays (np.roll and masks for the walls).

The readings where the paper leaves a choice open are the ones the C oracle
states (walls on the cell faces with halfway bounce-back, the held-particle
temperature rule, the repulsion law, overlap scaling, nearest periodic
images, forward Euler on the position), taken here from their statements,
not from its code.
"""
from __future__ import annotations

import math
import warnings

import numpy as np
from scipy import integrate

E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1),
              (-1, -1), (1, -1)], dtype=float)
EX, EY = E[:, 0], E[:, 1]
WGT = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])
# free parameters of the energy LB fixed in Sec. 2.2 (beta_1 = -4)
ALPHA1, ALPHA2, BETA1, BETA2 = -2.0, 1.0, -4.0, 4.0


def transform_matrix() -> np.ndarray:
    e2 = EX * EX + EY * EY
    return np.array([np.ones(9), -4 + 3 * e2, 4 - 10.5 * e2 + 4.5 * e2 * e2,
                     EX, (-5 + 3 * e2) * EX, EY, (-5 + 3 * e2) * EY,
                     EX * EX - EY * EY, EX * EY])


MT = transform_matrix()
MTI = np.linalg.inv(MT)


def feq(rho, ux, uy):
    """Textbook D2Q9 equilibria; arrays broadcast, result (9, ...)."""
    rho, ux, uy = np.broadcast_arrays(np.asarray(rho, float),
                                      np.asarray(ux, float),
                                      np.asarray(uy, float))
    eu = np.multiply.outer(EX, ux) + np.multiply.outer(EY, uy)
    u2 = ux * ux + uy * uy
    w = WGT.reshape((9,) + (1,) * rho.ndim)
    return w * rho * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * u2)


def guo(Fx, Fy, ux, uy):
    """Guo's forcing term in velocity space (without the relaxation
    factor), (9, ...)."""
    eF = np.multiply.outer(EX, Fx) + np.multiply.outer(EY, Fy)
    eu = np.multiply.outer(EX, ux) + np.multiply.outer(EY, uy)
    uF = ux * Fx + uy * Fy
    w = WGT.reshape((9,) + (1,) * np.ndim(Fx))
    return w * (3 * eF + 9 * eu * eF - 3 * uF)


def to_moments(f):
    return np.tensordot(MT, f, axes=1)


def to_velocities(m):
    return np.tensordot(MTI, m, axes=1)


def energy_eq_moments(eps, T, cref):
    z = np.zeros_like(eps)
    return np.array([eps, -4 * eps + (4 + ALPHA1) * cref * T,
                     4 * eps - (4 - ALPHA2) * cref * T, z, z, z, z, z, z])


# ---- geometry --------------------------------------------------------

def quad_form(a, b, th):
    """Coefficients (A, B, C) of the particle's inside test
    A dx^2 + 2 B dx dy + C dy^2 <= 1 (a disk when a == b)."""
    c, s = math.cos(th), math.sin(th)
    A = c * c / (a * a) + s * s / (b * b)
    B = c * s * (1 / (a * a) - 1 / (b * b))
    C = s * s / (a * a) + c * c / (b * b)
    return A, B, C


def cell_area(X, Y, a, b, th, i, j):
    """Area of the particle inside the cell [i, i+1] x [j, j+1]."""
    A, B, C = quad_form(a, b, th)
    W = math.sqrt(C / (A * C - B * B))          # extreme |dx| of the boundary

    def chord(x):
        dx = x - X
        disc = B * B * dx * dx - C * (A * dx * dx - 1)
        if disc <= 0:
            return 0.0
        r = math.sqrt(disc)
        lo, hi = Y + (-B * dx - r) / C, Y + (-B * dx + r) / C
        return max(0.0, min(hi, j + 1.0) - max(lo, float(j)))

    x0, x1 = max(float(i), X - W), min(i + 1.0, X + W)
    if not x0 < x1:
        return 0.0
    pts = []
    for yl in (float(j), j + 1.0):
        dy = yl - Y
        disc = B * B * dy * dy - A * (C * dy * dy - 1)
        if disc > 0:
            r = math.sqrt(disc)
            pts += [X + (-B * dy - r) / A, X + (-B * dy + r) / A]
    pts = sorted(p for p in pts if x0 < p < x1)
    edges = [x0] + pts + [x1]
    tot = 0.0
    for u, v in zip(edges[:-1], edges[1:]):
        with warnings.catch_warnings():
            # a tolerance below rounding: quad reports reaching its floor
            warnings.simplefilter("ignore", integrate.IntegrationWarning)
            val, _ = integrate.quad(chord, u, v, epsabs=1e-17, epsrel=1e-15,
                                    limit=200)
        tot += val
    return min(1.0, max(0.0, tot))


def nearest_image(Xp, node, L, periodic):
    if periodic and node - Xp > L / 2:
        return Xp + L
    if periodic and Xp - node > L / 2:
        return Xp - L
    return Xp


class Step:
    """The whole state of one domain and its time step."""

    def __init__(self, d: dict, ps: list):
        self.d = d
        self.nx, self.ny = d["nx"], d["ny"]
        self.perx = d["face_flow"][0] == "periodic"
        self.pery = d["face_flow"][2] == "periodic"
        self.cvf = d["cv_f"]
        self.cvs = d["R_cv"] * d["cv_f"]
        self.lamf = d["lambda_f"]
        self.lams = d["R_lambda"] * d["lambda_f"]
        # c_v,ref: the harmonic mean of the two specific heats (Sec. 2.2)
        self.cref = 2 * self.cvf * self.cvs / (self.cvf + self.cvs)
        self.P = [dict(p) for p in ps]
        for p in self.P:
            p["Rb"] = p["radius_minor"] if 0 < p["radius_minor"] < p["radius"] \
                else p["radius"]

    def geometry(self):
        """Per cell: the list [(p, share, full, usx, usy)] and f_s."""
        nx, ny = self.nx, self.ny
        lists = [[[] for _ in range(nx)] for _ in range(ny)]
        for k, p in enumerate(self.P):
            R, Rb = p["radius"], p["Rb"]
            for j in range(ny):
                for i in range(nx):
                    X = nearest_image(p["x"], i + 0.5, nx, self.perx)
                    Y = nearest_image(p["y"], j + 0.5, ny, self.pery)
                    # the closed cell meets the open disk of radius R
                    ddx = max(0.0, i - X, X - (i + 1))
                    ddy = max(0.0, j - Y, Y - (j + 1))
                    if not ddx * ddx + ddy * ddy < R * R:
                        continue
                    # wholly inside the inscribed disk: farthest corner
                    fx = max(X - i, i + 1 - X)
                    fy = max(Y - j, j + 1 - Y)
                    full = fx * fx + fy * fy <= Rb * Rb
                    share = 1.0 if full else cell_area(X, Y, R, Rb,
                                                       p["theta"], i, j)
                    rx, ry = i + 0.5 - X, j + 0.5 - Y
                    lists[j][i].append([k, share, full,
                                        p["ux"] - p["omega"] * ry,
                                        p["uy"] + p["omega"] * rx])
        fs = np.zeros((ny, nx))
        for j in range(ny):
            for i in range(nx):
                S = sum(e[1] for e in lists[j][i])
                if S > 1.0:
                    for e in lists[j][i]:
                        e[1] /= S
                    S = 1.0
                fs[j, i] = S
        return lists, fs

    def init(self):
        d = self.d
        self.lists, self.fs = self.geometry()
        ny, nx = self.ny, self.nx
        rho0 = np.full((ny, nx), d["init_rho"])
        if d["fluid_gravity"]:
            xs = np.arange(nx) + 0.5 - nx / 2
            ys = np.arange(ny) + 0.5 - ny / 2
            gx, gy = d["gravity"]
            rho0 = d["init_rho"] + 3 * d["rho_f"] * (gx * xs[None, :]
                                                     + gy * ys[:, None])
        ux = (1 - self.fs) * d["init_u"][0]
        uy = (1 - self.fs) * d["init_u"][1]
        eps = (1 - self.fs) * self.cvf * d["init_T"]
        for j in range(ny):
            for i in range(nx):
                for k, w, full, sx, sy in self.lists[j][i]:
                    ux[j, i] += w * sx
                    uy[j, i] += w * sy
                    eps[j, i] += w * self.cvs * self.P[k]["T_init"]
        cv = (1 - self.fs) * self.cvf + self.fs * self.cvs
        T = eps / cv
        self.f = feq(rho0, ux, uy)
        self.g = to_velocities(energy_eq_moments(eps, T, self.cref))
        self.dfs = np.zeros((ny, nx))
        for p in self.P:
            p["uxp"], p["uyp"], p["omp"] = p["ux"], p["uy"], p["omega"]
            p["Fx"] = p["Fy"] = p["Tz"] = 0.0
        self.rho, self.ux, self.uy, self.T = rho0, ux, uy, T
        return self

    # ---- stage: particles ------------------------------------------------
    def repulsion(self, k):
        d = self.d
        zeta = d["coll_range"]
        if not zeta > 0:
            return 0.0, 0.0
        p = self.P[k]
        fx = fy = 0.0
        for m, q in enumerate(self.P):
            if m == k:
                continue
            rx = p["x"] - nearest_image(q["x"], p["x"], self.nx, self.perx)
            ry = p["y"] - nearest_image(q["y"], p["y"], self.ny, self.pery)
            dist = math.hypot(rx, ry)
            reach = p["radius"] + q["radius"] + zeta
            if 0 < dist < reach:
                mag = d["coll_stiff_pp"] * ((reach - dist) / zeta) ** 2
                fx += mag * rx / dist
                fy += mag * ry / dist
        gaps = ((0, p["x"], (1, 0)), (1, self.nx - p["x"], (-1, 0)),
                (2, p["y"], (0, 1)), (3, self.ny - p["y"], (0, -1)))
        for face, gap, n in gaps:
            if d["face_flow"][face] != "wall":
                continue
            reach = 2 * p["radius"] + zeta
            if 2 * gap < reach:
                mag = d["coll_stiff_pw"] * ((reach - 2 * gap) / zeta) ** 2
                fx += mag * n[0]
                fy += mag * n[1]
        return fx, fy

    def move_particles(self):
        d = self.d
        rep = [self.repulsion(k) for k in range(len(self.P))]
        for p, (rfx, rfy) in zip(self.P, rep):
            R, Rb, rs = p["radius"], p["Rb"], p["rho_s"]
            V = math.pi * R * Rb
            M = rs * V
            I = M * R * R / 2 if Rb == R else M * (R * R + Rb * Rb) / 4
            Min, Iin = d["rho_f"] * V, d["rho_f"] / rs * I
            U, Om = (p["ux"], p["uy"]), p["omega"]
            nU, nOm = U, Om
            if not p["fixed"]:
                # the numerical fluid inside: backward differences
                Fin = (-Min * (U[0] - p["uxp"]), -Min * (U[1] - p["uyp"]))
                Tin = -Iin * (Om - p["omp"])
                buoy = (rs if d["fluid_gravity"] else rs - d["rho_f"]) * V
                F = [p["Fx"] - Fin[0] + buoy * d["gravity"][0] + rfx,
                     p["Fy"] - Fin[1] + buoy * d["gravity"][1] + rfy]
                nU = (U[0] + F[0] / M, U[1] + F[1] / M)
                nOm = Om + (p["Tz"] - Tin) / I
            x, y = p["x"] + U[0], p["y"] + U[1]
            if self.perx:
                x = x - self.nx if x >= self.nx else x + self.nx if x < 0 else x
            if self.pery:
                y = y - self.ny if y >= self.ny else y + self.ny if y < 0 else y
            p["theta"] += Om
            p["uxp"], p["uyp"], p["omp"] = U[0], U[1], Om
            p["ux"], p["uy"], p["omega"] = nU[0], nU[1], nOm
            p["x"], p["y"] = x, y

    # ---- stage: streaming ------------------------------------------------
    def stream(self, a, thermal):
        """Pull streaming of a (9, ny, nx) array with the wall rules."""
        d = self.d
        out = np.stack([np.roll(a[q], (int(EY[q]), int(EX[q])), axis=(0, 1))
                        for q in range(9)])
        jj, ii = np.meshgrid(np.arange(self.ny), np.arange(self.nx),
                             indexing="ij")
        for q in range(9):
            si, sj = ii - EX[q], jj - EY[q]
            hit = np.full((self.ny, self.nx), -1)
            # an x wall, then a y wall (which decides at a corner)
            if not self.perx:
                hit[si < 0] = 0
                hit[si >= self.nx] = 1
            if not self.pery:
                hit[sj < 0] = 2
                hit[sj >= self.ny] = 3
            for face in range(4):
                m = hit == face
                if not m.any():
                    continue
                if not thermal:
                    uw = d["u_wall"][face]
                    out[q][m] = a[OPP[q]][m] + 6 * WGT[q] * d["init_rho"] * (
                        EX[q] * uw[0] + EY[q] * uw[1])
                elif d["face_thermal"][face] == "dirichlet":
                    out[q][m] = -a[OPP[q]][m] + 2 * WGT[q] * self.cref * \
                        d["T_wall"][face]
                else:
                    out[q][m] = a[OPP[q]][m]
        return out

    # ---- one step --------------------------------------------------------
    def step(self):
        d = self.d
        ny, nx = self.ny, self.nx
        if self.P:
            self.move_particles()
        lists, fs_new = self.geometry()
        self.dfs = 2 * (fs_new - self.fs) - self.dfs
        self.fs, self.lists = fs_new, lists
        fst = self.stream(self.f, False)
        g = self.stream(self.g, True)
        fs = self.fs
        # volumetric no-slip step (eq. fi) and each particle's share of the
        # momentum change
        rho = fst.sum(axis=0)
        f = (1 - fs) * fst
        dP = {}
        for j in range(ny):
            for i in range(nx):
                for k, w, full, sx, sy in lists[j][i]:
                    fe = feq(rho[j, i], sx, sy)
                    f[:, j, i] += w * fe
                    dP[(k, j, i)] = (w * np.dot(fe - fst[:, j, i], EX),
                                     w * np.dot(fe - fst[:, j, i], EY),
                                     w * np.abs(fe + fst[:, j, i]).sum())
        # held particle temperatures
        cv = (1 - fs) * self.cvf + fs * self.cvs
        for j in range(ny):
            for i in range(nx):
                held = [(k, w) for k, w, *_ in lists[j][i]
                        if self.P[k]["hold_T"]]
                if not held:
                    continue
                phi = sum(w for k, w in held)
                add = sum(w * to_velocities(energy_eq_moments(
                    np.array(cv[j, i] * self.P[k]["T_init"]),
                    np.array(self.P[k]["T_init"]), self.cref))
                    for k, w in held)
                g[:, j, i] = (1 - phi) * g[:, j, i] + add
        # properties: lambda/rho_f = (4 + alpha1)/6 c_ref (1/sigma_j - 1/2)
        lam = (1 - fs) * self.lamf + fs * self.lams
        tau_g = 0.5 + 6 * lam / (d["rho_f"] * (4 + ALPHA1) * self.cref)
        sj = 1 / tau_g
        se = np.ones_like(sj) if d["sigma_rule"] else \
            1 / (0.5 + 0.25 / (tau_g - 0.5))
        # temperature gradient from the energy flux
        G = g.sum(axis=0)
        gTx = -6 / (4 + ALPHA1) * np.tensordot(EX, g, 1) / (self.cref * tau_g)
        gTy = -6 / (4 + ALPHA1) * np.tensordot(EY, g, 1) / (self.cref * tau_g)
        jx, jy = np.tensordot(EX, f, 1), np.tensordot(EY, f, 1)
        wf = 1 - fs
        gwt = d["rho_f"] if d["fluid_gravity"] else 0.0
        gx, gy = d["gravity"]

        def force(T):
            buoy = -d["rho_f"] * d["beta"] * (T - d["T_ref"])
            return (wf * (d["body_force"][0] + gwt * gx + buoy * gx),
                    wf * (d["body_force"][1] + gwt * gy + buoy * gy))

        def residual(T):
            Fx, Fy = force(T)
            ux, uy = (jx + Fx / 2) / rho, (jy + Fy / 2) / rho
            dcv = self.cvs - self.cvf
            return cv * T - G + 0.5 * cv * (ux * gTx + uy * gTy) \
                - 0.5 * dcv * T * self.dfs
        r0, r1 = residual(np.zeros_like(G)), residual(np.ones_like(G))
        T = -r0 / (r1 - r0)
        Fx, Fy = force(T)
        ux, uy = (jx + Fx / 2) / rho, (jy + Fy / 2) / rho
        eps = cv * T
        qc = -cv * (ux * gTx + uy * gTy) + (self.cvs - self.cvf) * T * self.dfs
        # flow collision
        tf = d["tau_f"]
        sq = 1 / (0.5 + (1 / 12) / (tf - 0.5))
        S = np.array([1, 1.25, 1.25, 1, sq, 1, sq, 1 / tf, 1 / tf])
        m = to_moments(f)
        meq = to_moments(feq(rho, ux, uy))
        Fm = to_moments(guo(Fx, Fy, ux, uy))
        S3 = S[:, None, None]
        self.f = to_velocities(m - S3 * (m - meq) + (1 - S3 / 2) * Fm)
        # energy collision
        one = np.ones_like(sj)
        Rd = np.array([one, se, se, sj, sj, sj, sj, se, se])
        n = to_moments(g)
        neq = energy_eq_moments(eps, T, self.cref)
        z = np.zeros_like(qc)
        src = np.array([qc, BETA1 * qc, BETA2 * qc, z, z, z, z, z, z])
        self.g = to_velocities(n - Rd * (n - neq) + (1 - Rd / 2) * src)
        self.rho, self.ux, self.uy, self.T = rho, ux, uy, T
        # momentum exchange: F = -sum f_s,p (rho u_s - j*), torque about
        # the centre
        for k, p in enumerate(self.P):
            p["Fx"] = p["Fy"] = p["Tz"] = p["Fabs"] = 0.0
        for (k, j, i), (px, py, mag) in sorted(dP.items(),
                                          key=lambda e: (e[0][1], e[0][2],
                                                         e[0][0])):
            p = self.P[k]
            X = nearest_image(p["x"], i + 0.5, nx, self.perx)
            Y = nearest_image(p["y"], j + 0.5, ny, self.pery)
            p["Fx"] -= px
            p["Fy"] -= py
            p["Tz"] -= (i + 0.5 - X) * py - (j + 0.5 - Y) * px
            # the scale of the sums: their terms before they cancel
            p["Fabs"] += mag
        return self

    def particle_outputs(self):
        """T_mean, T_min (over the cells wholly inside, else over all it
        reaches), E_solid and sum f_s,p of every particle."""
        out = []
        for k in range(len(self.P)):
            cells = [(self.T[j, i], w, full)
                     for j in range(self.ny) for i in range(self.nx)
                     for kk, w, full, *_ in self.lists[j][i] if kk == k]
            ws = sum(w for _, w, _ in cells)
            inner = [t for t, _, full in cells if full]
            out.append(dict(
                T_mean=sum(t * w for t, w, _ in cells) / ws if ws else 0.0,
                T_min=min(inner) if inner else min(t for t, _, _ in cells),
                E_solid=sum(w * self.cvs * t for t, w, _ in cells),
                fs_sum=ws))
        return out
