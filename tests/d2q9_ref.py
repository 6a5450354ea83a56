"""Independent numpy helpers for pinning the oracle.

Nothing here is imported from the oracle: the lattice constants are restated
from the D2Q9 model named in Sec. 2, and the single-relaxation-time (BGK) model
with Guo forcing is a textbook scheme coded from scratch, vectorised over the
whole lattice with np.roll streaming.  It is the special case k0 = k1 = k2 of
Eq. (2), so the oracle must reproduce it.
"""
import numpy as np

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.int64)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.int64)
W = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])
CS2 = 1.0 / 3.0


def moments(p):
    """Raw moments of populations p[9, ...]: (M0, M1x, M1y, M2xx, M2xy, M2yy)."""
    p = np.asarray(p)
    sh = (9,) + (1,) * (p.ndim - 1)
    cx = CX.reshape(sh)
    cy = CY.reshape(sh)
    return ((p).sum(0), (cx * p).sum(0), (cy * p).sum(0),
            (cx * cx * p).sum(0), (cx * cy * p).sum(0), (cy * cy * p).sum(0))


def hermite_high(p):
    """Third- and fourth-order Hermite moments that D2Q9 carries:
    a_xxy, a_xyy, a_xxyy with H_xxy = cy (cx^2 - cs^2) etc."""
    p = np.asarray(p)
    sh = (9,) + (1,) * (p.ndim - 1)
    cx = CX.reshape(sh).astype(float)
    cy = CY.reshape(sh).astype(float)
    hxxy = cy * (cx * cx - CS2)
    hxyy = cx * (cy * cy - CS2)
    hxxyy = (cx * cx - CS2) * (cy * cy - CS2)
    return (hxxy * p).sum(0), (hxyy * p).sum(0), (hxxyy * p).sum(0)


class SRTLattice:
    """BGK (single rate omega_f for f, omega_g for g) with Guo forcing, on the
    same cavity: half-way bounce-back walls, anti-bounce-back at the heated
    bottom cells, liquid-fraction-scaled velocity and Boussinesq force."""

    def __init__(self, nx, ny, *, omega_f, omega_g, Cp, Th, Tm, rho0, latent, gbeta,
                 heater_cells, periodic_x=False, periodic_y=False):
        self.nx, self.ny = nx, ny
        self.of, self.og = omega_f, omega_g
        self.Cp, self.Th, self.Tm, self.rho0, self.L, self.gb = Cp, Th, Tm, rho0, latent, gbeta
        self.px, self.py = periodic_x, periodic_y
        self.heater = np.zeros(nx, dtype=bool)
        self.heater[list(heater_cells)] = True

    def macros(self, f, g):
        H = g.sum(0)
        Hs = self.Cp * self.Tm
        Hl = Hs + self.L
        fl = np.where(H <= Hs, 0.0, np.where(H >= Hl, 1.0, (H - Hs) / max(self.L, 1e-300)))
        T = np.where(H <= Hs, H / self.Cp, np.where(H >= Hl, self.Tm + (H - Hl) / self.Cp, self.Tm))
        rho = f.sum(0)
        jx = (CX[:, None, None] * f).sum(0)
        jy = (CY[:, None, None] * f).sum(0)
        Fy = self.rho0 * self.gb * (T - self.Tm)
        ux = fl * jx / self.rho0
        uy = fl * (jy + 0.5 * Fy) / self.rho0
        return H, T, fl, rho, ux, uy, Fy

    def collide(self, f, g):
        H, T, fl, rho, ux, uy, Fy = self.macros(f, g)
        cu = CX[:, None, None] * ux + CY[:, None, None] * uy
        uu = ux * ux + uy * uy
        w = W[:, None, None]
        feq = w * (rho + self.rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu))
        # Guo et al. forcing, F = (0, Fy)
        cF = CY[:, None, None] * Fy
        uF = uy * Fy
        guo = (1.0 - 0.5 * self.of) * w * (3.0 * cF + 9.0 * cu * cF - 3.0 * uF)
        fs = f - self.of * (f - feq) + guo
        geq = w * self.Cp * T * (1.0 + 3.0 * cu)
        geq[0] = H - self.Cp * T + W[0] * self.Cp * T
        gs = g - self.og * (g - geq)
        return fs, gs

    def stream(self, fs, gs):
        nx, ny = self.nx, self.ny
        f = np.empty_like(fs)
        g = np.empty_like(gs)
        yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        for i in range(9):
            f[i] = np.roll(np.roll(fs[i], CX[i], axis=1), CY[i], axis=0)
            g[i] = np.roll(np.roll(gs[i], CX[i], axis=1), CY[i], axis=0)
            sx = xx - CX[i]
            sy = yy - CY[i]
            out = np.zeros((ny, nx), dtype=bool)
            if not self.px:
                out |= (sx < 0) | (sx >= nx)
            below = np.zeros((ny, nx), dtype=bool)
            if not self.py:
                out |= (sy < 0) | (sy >= ny)
                below = sy < 0
            o = OPP[i]
            f[i] = np.where(out, fs[o], f[i])
            anti = below & self.heater[None, :]
            g[i] = np.where(out, np.where(anti, -gs[o] + 2.0 * W[i] * self.Cp * self.Th, gs[o]), g[i])
        return f, g

    def step(self, f, g, n=1):
        for _ in range(n):
            fs, gs = self.collide(f, g)
            f, g = self.stream(fs, gs)
        return f, g
