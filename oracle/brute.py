"""Brute-force scalar reference for tiny grids (TEST INFRASTRUCTURE ONLY).

A second, deliberately different implementation of the FV semi-implicit +
Heun step (sec. 2.2, eq:semi and eq:semi-heun) and of the ST step (sec. 2.1,
eq:ST), used to pin the C oracle in ``oracle.c``.  It is written face by face
with Python floats, and the QUICK face value (sec. 2.2.3) is obtained by
fitting the upwind parabola a + b x + c x^2 through the three nodes with a
3x3 linear solve and evaluating it at the face, rather than from the
closed-form gamma coefficients.  The lattice tables are derived here from the
velocity set instead of being copied.  Only meant for grids of a few cells.
"""
import math

import numpy as np

VELOCITIES = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]


def _weight(c):
    # D2Q9 weights by speed class: rest 4/9, axis 1/9, diagonal 1/36
    s = c[0] * c[0] + c[1] * c[1]
    return {0: 4.0 / 9.0, 1: 1.0 / 9.0, 2: 1.0 / 36.0}[s]


WEIGHTS = [_weight(c) for c in VELOCITIES]
OPPOSITE = [VELOCITIES.index((-c[0], -c[1])) for c in VELOCITIES]
CS2 = 1.0 / 3.0


def _parabola_at(xs, vs, x):
    """Value at x of the parabola through the points (xs[k], vs[k])."""
    A = np.array([[1.0, xx, xx * xx] for xx in xs])
    coef = np.linalg.solve(A, np.array(vs, dtype=float))
    return float(coef[0] + coef[1] * x + coef[2] * x * x)


def _centres_with_ghosts(faces, periodic):
    """Node positions for indices -2..n+1 as a dict."""
    n = len(faces) - 1
    L = faces[-1] - faces[0]
    cen = {k: 0.5 * (faces[k] + faces[k + 1]) for k in range(n)}
    for k in (-2, -1, n, n + 1):
        if periodic:
            m = k % n
            cen[k] = cen[m] + (k - m) // n * L
        elif k < 0:
            cen[k] = 2 * faces[0] - cen[-k - 1]
        else:
            cen[k] = 2 * faces[n] - cen[2 * n - 1 - k]
    return cen


class _Case:
    def __init__(self, p, xf, yf):
        self.p = p
        self.nx, self.ny = p["nx"], p["ny"]
        self.xf, self.yf = list(map(float, xf)), list(map(float, yf))
        self.cx = _centres_with_ghosts(self.xf, not p["wall_x"])
        self.cy = _centres_with_ghosts(self.yf, not p["wall_y"])

    # ---- local model ----
    def macro(self, f, g, j, i, half):
        p = self.p
        rho = sum(f[a][j][i] for a in range(9))
        jx = sum(VELOCITIES[a][0] * f[a][j][i] for a in range(9))
        jy = sum(VELOCITIES[a][1] * f[a][j][i] for a in range(9))
        T = sum(g[a][j][i] for a in range(9)) if p["thermal"] else 0.0
        ax = p["ax"]
        ay = p["ay"] + (p["beta_g"] * (T - p["T0"]) if p["thermal"] else 0.0)
        return rho, jx / rho + half * ax, jy / rho + half * ay, T, ax, ay

    @staticmethod
    def feq(a, rho, ux, uy):
        cx, cy = VELOCITIES[a]
        cu = cx * ux + cy * uy
        return WEIGHTS[a] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy))

    @staticmethod
    def guo(a, rho, ux, uy, ax, ay):
        cx, cy = VELOCITIES[a]
        cu = cx * ux + cy * uy
        return WEIGHTS[a] * rho * (3 * ((cx - ux) * ax + (cy - uy) * ay) + 9 * cu * (cx * ax + cy * ay))

    def stage(self, f, g):
        p = self.p
        dt = p["dt"]
        tt, ttg = p["tau"] + dt / 2, p["tau_g"] + dt / 2
        ny, nx = self.ny, self.nx
        phf = [[[0.0] * nx for _ in range(ny)] for _ in range(9)]
        cf = [[[0.0] * nx for _ in range(ny)] for _ in range(9)]
        phg = [[[0.0] * nx for _ in range(ny)] for _ in range(9)]
        cg = [[[0.0] * nx for _ in range(ny)] for _ in range(9)]
        for j in range(ny):
            for i in range(nx):
                rho, ux, uy, T, ax, ay = self.macro(f, g, j, i, dt / 2)
                for a in range(9):
                    fe = self.feq(a, rho, ux, uy)
                    F = self.guo(a, rho, ux, uy, ax, ay)
                    fv = f[a][j][i]
                    phf[a][j][i] = fv + dt / (2 * tt) * (fe - fv) + dt / 2 * F
                    cf[a][j][i] = dt / tt * (fe - fv) + dt * (1 - dt / (2 * tt)) * F
                    if p["thermal"]:
                        gv = g[a][j][i]
                        ge = T / rho * fe
                        phg[a][j][i] = gv + dt / (2 * ttg) * (ge - gv)
                        cg[a][j][i] = dt / ttg * (ge - gv)
        return phf, cf, phg, cg

    # ---- advection ----
    def node(self, phi, thermal, a, axis, k, other):
        """phi of population a at node k along axis (ghosts included)."""
        p = self.p
        n = self.nx if axis == 0 else self.ny
        wall = p["wall_x"] if axis == 0 else p["wall_y"]
        if 0 <= k < n or not wall:
            k = k % n
            return phi[a][other][k] if axis == 0 else phi[a][k][other]
        mirror = -k - 1 if k < 0 else 2 * n - 1 - k
        if wall == 2:
            # fixed density on the boundary face: rescale the mirror cell's
            # population by (extrapolated ghost density) / (mirror density)
            at = (lambda q: phi[q][other][mirror]) if axis == 0 else (lambda q: phi[q][mirror][other])
            rho_m = sum(at(q) for q in range(9))
            rho_face = p["rho_lo"] if k < 0 else p["rho_hi"]
            rho_ghost = rho_m + 2.0 * (rho_face - rho_m)
            return at(a) * (rho_ghost / rho_m)
        b = OPPOSITE[a]
        v = phi[b][other][mirror] if axis == 0 else phi[b][mirror][other]
        if thermal and axis == 1:
            Tw = p["T_bottom"] if k < 0 else p["T_top"]
            v = 2 * WEIGHTS[a] * Tw - v
        return v

    def face(self, phi, thermal, a, axis, k, other):
        """Upwind-parabola value on the face between nodes k and k+1."""
        faces = self.xf if axis == 0 else self.yf
        cen = self.cx if axis == 0 else self.cy
        c = VELOCITIES[a][axis]
        # the face between nodes k and k+1 sits at faces[k+1] (k = -1: faces[0])
        xface = faces[k + 1]
        ks = (k - 1, k, k + 1) if c > 0 else (k, k + 1, k + 2)
        xs = [cen[q] for q in ks]
        vs = [self.node(phi, thermal, a, axis, q, other) for q in ks]
        return _parabola_at(xs, vs, xface)

    def divergence(self, phi, thermal):
        ny, nx = self.ny, self.nx
        D = [[[0.0] * nx for _ in range(ny)] for _ in range(9)]
        for a in range(9):
            cx, cy = VELOCITIES[a]
            for j in range(ny):
                for i in range(nx):
                    d = 0.0
                    if cx:
                        d += cx * (self.face(phi, thermal, a, 0, i, j) - self.face(phi, thermal, a, 0, i - 1, j)) / (
                            self.xf[i + 1] - self.xf[i])
                    if cy:
                        d += cy * (self.face(phi, thermal, a, 1, j, i) - self.face(phi, thermal, a, 1, j - 1, i)) / (
                            self.yf[j + 1] - self.yf[j])
                    D[a][j][i] = d
        return D


def fv_heun(p, xf, yf, f, g, nsteps):
    """Advance numpy arrays f, g ([9][ny][nx]) by nsteps of eq:semi-heun."""
    case = _Case(p, xf, yf)
    dt = p["dt"]
    f = f.tolist()
    g = g.tolist() if p["thermal"] else [[[0.0] * p["nx"] for _ in range(p["ny"])] for _ in range(9)]
    rng = [(a, j, i) for a in range(9) for j in range(p["ny"]) for i in range(p["nx"])]
    for _ in range(nsteps):
        phf, cf, phg, cg = case.stage(f, g)
        Df = case.divergence(phf, False)
        Dg = case.divergence(phg, True) if p["thermal"] else None
        fs = [[[f[a][j][i] - dt * Df[a][j][i] + cf[a][j][i] for i in range(p["nx"])] for j in range(p["ny"])]
              for a in range(9)]
        gs = g
        if p["thermal"]:
            gs = [[[g[a][j][i] - dt * Dg[a][j][i] + cg[a][j][i] for i in range(p["nx"])] for j in range(p["ny"])]
                  for a in range(9)]
        phs, _, phgs, _ = case.stage(fs, gs)
        Dfs = case.divergence(phs, False)
        Dgs = case.divergence(phgs, True) if p["thermal"] else None
        for a, j, i in rng:
            f[a][j][i] = f[a][j][i] - dt / 2 * (Df[a][j][i] + Dfs[a][j][i]) + cf[a][j][i]
            if p["thermal"]:
                g[a][j][i] = g[a][j][i] - dt / 2 * (Dg[a][j][i] + Dgs[a][j][i]) + cg[a][j][i]
    return np.array(f), (np.array(g) if p["thermal"] else None)


def st(p, f, g, nsteps):
    """Advance by nsteps of eq:ST (dt = dx = 1), half-way bounce-back walls,
    anti-bounce-back for g on the isothermal y walls."""
    nx, ny = p["nx"], p["ny"]
    tt, ttg = p["tau"] + 0.5, p["tau_g"] + 0.5
    f = f.tolist()
    g = g.tolist() if p["thermal"] else None
    case = _Case(p, list(range(nx + 1)), list(range(ny + 1)))
    for _ in range(nsteps):
        nf = [[[math.nan] * nx for _ in range(ny)] for _ in range(9)]
        ng = [[[math.nan] * nx for _ in range(ny)] for _ in range(9)]
        for j in range(ny):
            for i in range(nx):
                rho, ux, uy, T, ax, ay = case.macro(f, g, j, i, 0.5)
                for a in range(9):
                    cx, cy = VELOCITIES[a]
                    fe = case.feq(a, rho, ux, uy)
                    F = case.guo(a, rho, ux, uy, ax, ay)
                    fpost = f[a][j][i] + (fe - f[a][j][i]) / tt + (1 - 1 / (2 * tt)) * F
                    ti, tj = i + cx, j + cy
                    out_y = not (0 <= tj < ny)
                    out_x = not (0 <= ti < nx)
                    blocked = (out_y and p["wall_y"]) or (out_x and p["wall_x"])
                    if p["thermal"]:
                        gpost = g[a][j][i] + (T / rho * fe - g[a][j][i]) / ttg
                    if blocked:
                        b = OPPOSITE[a]
                        nf[b][j][i] = fpost
                        if p["thermal"]:
                            if out_y and p["wall_y"]:
                                Tw = p["T_bottom"] if tj < 0 else p["T_top"]
                                gpost = 2 * WEIGHTS[a] * Tw - gpost
                            ng[b][j][i] = gpost
                    else:
                        nf[a][tj % ny][ti % nx] = fpost
                        if p["thermal"]:
                            ng[a][tj % ny][ti % nx] = gpost
        f = nf
        g = ng if p["thermal"] else None
    return np.array(f), (np.array(g) if p["thermal"] else None)


# ---------------------------------------------------------------- 3D -------
# D3Q19, derived from the velocity set: all (cx, cy, cz) in {-1, 0, 1}^3 with
# at most two non-zero components, in an order of our own.

VEL3 = [c for c in ((x, y, z) for x in (-1, 0, 1) for y in (-1, 0, 1) for z in (-1, 0, 1))
        if abs(c[0]) + abs(c[1]) + abs(c[2]) <= 2]


def _w3(c):
    s = abs(c[0]) + abs(c[1]) + abs(c[2])
    return {0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0}[s]


W3 = [_w3(c) for c in VEL3]
OPP3 = [VEL3.index((-c[0], -c[1], -c[2])) for c in VEL3]


def fv_heun_3d(p, faces, f, g, nsteps, order):
    """eq:semi-heun in 3D on a tiny grid.  f, g: [19][nz][ny][nx] in the
    caller's population order `order` (a list of velocity tuples); the
    result is returned in that order."""
    nx, ny, nz = p["n"]
    dt = p["dt"]
    idx = [VEL3.index(tuple(c)) for c in order]     # caller a -> our a
    F = np.zeros((19, nz, ny, nx))
    G = np.zeros((19, nz, ny, nx))
    for a, b in enumerate(idx):
        F[b] = f[a]
        if p["thermal"]:
            G[b] = g[a]
    cen = [_centres_with_ghosts(list(map(float, faces[d])), not p["wall"][d]) for d in range(3)]

    def macro(F, G, k, j, i):
        rho = float(F[:, k, j, i].sum())
        T = float(G[:, k, j, i].sum()) if p["thermal"] else 0.0
        acc = list(p["a"])
        if p["thermal"]:
            acc[2] += p["beta_g"] * (T - p["T0"])
        u = [sum(VEL3[a][d] * F[a, k, j, i] for a in range(19)) / rho + dt / 2 * acc[d] for d in range(3)]
        return rho, u, T, acc

    def stage(F, G):
        tt, ttg = p["tau"] + dt / 2, p["tau_g"] + dt / 2
        ph, Cf, phg, Cg = (np.zeros_like(F) for _ in range(4))
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    rho, u, T, acc = macro(F, G, k, j, i)
                    uu = sum(x * x for x in u)
                    for a, c in enumerate(VEL3):
                        cu = sum(c[d] * u[d] for d in range(3))
                        fe = W3[a] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
                        Fa = W3[a] * rho * sum((3 * (c[d] - u[d]) + 9 * cu * c[d]) * acc[d] for d in range(3))
                        fv = F[a, k, j, i]
                        ph[a, k, j, i] = fv + dt / (2 * tt) * (fe - fv) + dt / 2 * Fa
                        Cf[a, k, j, i] = dt / tt * (fe - fv) + dt * (1 - dt / (2 * tt)) * Fa
                        if p["thermal"]:
                            gv, ge = G[a, k, j, i], T / rho * fe
                            phg[a, k, j, i] = gv + dt / (2 * ttg) * (ge - gv)
                            Cg[a, k, j, i] = dt / ttg * (ge - gv)
        return ph, Cf, phg, Cg

    def node(phi, thermal, a, axis, q, pos):
        n = p["n"][axis]
        pos = list(pos)
        b, sgn, add = a, 1.0, 0.0
        if 0 <= q < n or not p["wall"][axis]:
            pos[axis] = q % n
        else:
            pos[axis] = -q - 1 if q < 0 else 2 * n - 1 - q
            b = OPP3[a]
            if thermal and axis == 2:
                sgn, add = -1.0, 2 * W3[a] * (p["T_bottom"] if q < 0 else p["T_top"])
        return sgn * phi[b, pos[2], pos[1], pos[0]] + add

    def div(phi, thermal):
        D = np.zeros_like(phi)
        for a, c in enumerate(VEL3):
            for k in range(nz):
                for j in range(ny):
                    for i in range(nx):
                        pos = (i, j, k)
                        d = 0.0
                        for axis in range(3):
                            if c[axis] == 0:
                                continue
                            vals = []
                            for q in (pos[axis] - 1, pos[axis]):    # faces q | q+1
                                ks = (q - 1, q, q + 1) if c[axis] > 0 else (q, q + 1, q + 2)
                                xs = [cen[axis][m] for m in ks]
                                vs = [node(phi, thermal, a, axis, m, pos) for m in ks]
                                vals.append(_parabola_at(xs, vs, float(faces[axis][q + 1])))
                            d += c[axis] * (vals[1] - vals[0]) / (faces[axis][pos[axis] + 1] - faces[axis][pos[axis]])
                        D[a, k, j, i] = d
        return D

    for _ in range(nsteps):
        ph, Cf, phg, Cg = stage(F, G)
        Df, Dg = div(ph, False), (div(phg, True) if p["thermal"] else None)
        Fs = F - dt * Df + Cf
        Gs = G - dt * Dg + Cg if p["thermal"] else G
        phs, _, phgs, _ = stage(Fs, Gs)
        F = F - dt / 2 * (Df + div(phs, False)) + Cf
        if p["thermal"]:
            G = G - dt / 2 * (Dg + div(phgs, True)) + Cg
    fo, go = np.zeros_like(F), np.zeros_like(G)
    for a, b in enumerate(idx):
        fo[a] = F[b]
        go[a] = G[b]
    return fo, (go if p["thermal"] else None)
