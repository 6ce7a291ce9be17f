"""TEST INFRASTRUCTURE ONLY -- complex-step derivatives of the lattice Boltzmann forward map.

A second FP64 implementation of the pseudopotential step, in complex128 numpy arithmetic:
the Smooth loop of Sec. III.D on a C-S or Peng-Robinson base (with the raised vapor branch
and the liquid shift of Sec. III.E), Eq. InteractionPotential, Eq. ShanChenForce with ghost
wall rows, Eq. Momentum, the MRT collision (Eq. OperatorMRT, Eq. MatrixMRT,
Eq. RelaxationMatrix, Eq. EquilibriumDistribution) with the Li source (Eq. LiFS), streaming
(Eq. LBE) and halfway bounce-back at walls.

Giving one real input an imaginary part i*h makes Im L / h equal dL/d(input) up to O(h^2)
with no subtractive cancellation (the complex-step derivative of Squire and Trapp, 1998), so
with h = 1e-30 the result is the exact derivative of the discrete map to rounding.  Every
branch (the EOS region, the wall rows) is chosen on the real part, as the real map does.

The real part of this map is the C oracle's map; a CPU test checks the two against each
other, and the derivative against central differences of the C oracle.  The two share no
code: this module takes only the built thermodynamic constants (Maxwell densities, the
saturation pressure, the branch slopes) from the C oracle's EOS record.  Constant relaxation
times only (Eq. RelaxationTime is not differentiated).
"""
from __future__ import annotations

import numpy as np

# D2Q9 (Eq. VelocitySet), weights (Sec. II.A)
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
WT = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])
# Eq. MatrixMRT: rows are the moments (rho, e, eps, jx, qx, jy, qy, pxx, pxy)
M = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
], dtype=np.float64)
# the rows are orthogonal, so M^-1 = M^T diag(1 / |row|^2)
MINV = M.T / (M * M).sum(axis=1)[None, :]


class Eos:
    """The shaped EOS with complex knots.  `built` is a built C oracle EOS record (Smooth or
    Modified Smooth); rho_max, p_max, rho_min, p_min default to its knots."""

    def __init__(self, built, rho_max=None, p_max=None, rho_min=None, p_min=None):
        b = built
        self.base, self.a, self.b, self.R, self.T, self.Tc = b.base, b.a, b.b, b.R, b.T, b.Tc
        self.omega, self.scale, self.k_vap, self.dP_liq = b.omega, b.scale, b.k_vap, b.dP_liq
        self.rho_v, self.rho_l, self.p_sat_new = b.rho_v, b.rho_l, b.p_sat_new
        self.slope_v, self.slope_l = b.slope_v, b.slope_l
        self.rho_max = complex(b.rho_max if rho_max is None else rho_max)
        self.p_max = complex(b.p_max if p_max is None else p_max)
        self.rho_min = complex(b.rho_min if rho_min is None else rho_min)
        self.p_min = complex(b.p_min if p_min is None else p_min)
        # ellipse 1 through (rho_v, p_sat) with the vapor branch's slope there and zero
        # slope at its top (rho_max, p_max); ellipse 3 mirrors it at (rho_min, p_min), rho_l
        self.a1sq, self.b1 = self._ellipse(self.rho_max - self.rho_v, self.p_max - self.p_sat_new, self.slope_v)
        self.a3sq, self.b3 = self._ellipse(self.rho_l - self.rho_min, self.p_sat_new - self.p_min, self.slope_l)

    @staticmethod
    def _ellipse(D, dp, slope):
        # semi-axes (a, b) of (rho - centre)^2 / a^2 + (p - p0)^2 / b^2 = 1 fixed by a rise dp
        # over a run D with the given end slope: k = dp D / slope - D^2, a^2 = -k^2 / (2k + D^2)
        k = dp * D / slope - D * D
        a2 = -k * k / (2 * k + D * D)
        return a2, dp / (1 - np.sqrt(1 - D * D / a2))

    def base_p(self, rho):
        if self.base == 0:  # Eq. CS
            eta = self.b * rho / 4
            return self.scale * (rho * self.R * self.T * (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3
                                 - self.a * rho * rho)
        # Eq. PR with the Soave alpha(T)
        kap = 0.37464 + 1.54226 * self.omega - 0.26992 * self.omega ** 2
        al = (1 + kap * (1 - np.sqrt(self.T / self.Tc))) ** 2
        b = self.b
        return self.scale * (rho * self.R * self.T / (1 - b * rho)
                             - self.a * al * rho * rho / (1 + 2 * b * rho - b * b * rho * rho))

    def p(self, rho):
        rho = np.asarray(rho, dtype=np.complex128)
        r = rho.real
        d1 = rho - self.rho_max
        d3 = rho - self.rho_min
        t = (rho - self.rho_max) / (self.rho_min - self.rho_max)
        with np.errstate(all="ignore"):
            br = [self.k_vap * self.base_p(rho),
                  self.base_p(rho) + self.dP_liq,
                  self.p_max - self.b1 + self.b1 * np.sqrt(1 - d1 * d1 / self.a1sq),
                  2 * (self.p_max - self.p_min) * t ** 3 + 3 * (self.p_min - self.p_max) * t ** 2 + self.p_max,
                  self.p_min + self.b3 - self.b3 * np.sqrt(1 - d3 * d3 / self.a3sq)]
        conds = [r <= self.rho_v, r >= self.rho_l, r <= self.rho_max.real, r < self.rho_min.real,
                 np.ones_like(r, dtype=bool)]
        return np.select(conds, br)


def psi(eos: Eos, rho, G):
    """Eq. InteractionPotential with c = 1; raises if psi^2 < 0 (the real map's failure)."""
    arg = 2 * (eos.p(rho) - rho / 3) / G
    if np.any(~(np.asarray(arg).real >= 0)):
        raise FloatingPointError("psi^2 < 0")
    return np.sqrt(arg)


def feq(rho, ux, uy):
    """Eq. EquilibriumDistribution, second order in u."""
    cu = CX[:, None, None] * ux + CY[:, None, None] * uy
    uu = ux * ux + uy * uy
    return WT[:, None, None] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)


class Lattice:
    """f_i on a [9][ny][nx] complex grid, periodic in x; periodic in y or walls at both ends."""

    def __init__(self, eos: Eos, nx, ny, G, sigma, tau, walls=False, rho_wall_lo=0.0, rho_wall_hi=0.0):
        self.eos, self.nx, self.ny = eos, nx, ny
        self.G, self.sigma = complex(G), complex(sigma)
        self.lam = 1.0 / np.asarray(tau, dtype=np.float64)
        self.tau = np.asarray(tau, dtype=np.float64)
        self.walls = walls
        if walls:
            self.psi_lo = psi(eos, np.complex128(rho_wall_lo), self.G)
            self.psi_hi = psi(eos, np.complex128(rho_wall_hi), self.G)
        self.f = None

    def init_eq(self, rho0):
        rho0 = np.asarray(rho0, dtype=np.complex128)
        self.f = feq(rho0, np.zeros_like(rho0), np.zeros_like(rho0))

    def _force_tilde(self, ps):
        """Eq. ShanChenForce divided by psi(x): -G sum_i w(|c_i|^2) psi(x + c_i) c_i."""
        ny = self.ny
        if self.walls:
            pad = np.empty((ny + 2, self.nx), dtype=np.complex128)
            pad[0], pad[ny + 1], pad[1:ny + 1] = self.psi_lo, self.psi_hi, ps
        sx = np.zeros_like(ps)
        sy = np.zeros_like(ps)
        for i in range(1, 9):
            w = 1 / 3 if CX[i] * CX[i] + CY[i] * CY[i] == 1 else 1 / 12
            if self.walls:
                nb = np.roll(pad[1 + CY[i]:1 + CY[i] + ny], -CX[i], axis=1)
            else:
                nb = np.roll(np.roll(ps, -CY[i], axis=0), -CX[i], axis=1)
            sx = sx + w * CX[i] * nb
            sy = sy + w * CY[i] * nb
        return -self.G * sx, -self.G * sy

    def fields(self):
        """rho, psi, F~ and u = (j + F/2)/rho (Eq. Momentum) of the current populations."""
        f = self.f
        rho = f.sum(axis=0)
        ps = psi(self.eos, rho, self.G)
        ftx, fty = self._force_tilde(ps)
        fx, fy = ps * ftx, ps * fty
        jx = (CX[:, None, None] * f).sum(axis=0)
        jy = (CY[:, None, None] * f).sum(axis=0)
        return rho, (jx + fx / 2) / rho, (jy + fy / 2) / rho, ps, ftx, fty, fx, fy

    def step(self):
        f = self.f
        rho, ux, uy, ps, ftx, fty, fx, fy = self.fields()
        m = np.tensordot(M, f - feq(rho, ux, uy), axes=1)
        # Eq. LiFS in moment space; |F|^2 / psi^2 is |F~|^2
        ftt = ftx * ftx + fty * fty
        uF = ux * fx + uy * fy
        t = self.tau
        S = np.stack([np.zeros_like(rho),
                      6 * uF + 12 * self.sigma * ftt / (t[1] - 0.5),
                      -6 * uF - 12 * self.sigma * ftt / (t[2] - 0.5),
                      fx, -fx, fy, -fy,
                      2 * (ux * fx - uy * fy),
                      ux * fy + uy * fx])
        lam = self.lam[:, None, None]
        post = f + np.tensordot(MINV, -lam * m + (1 - lam / 2) * S, axes=1)
        # streaming (Eq. LBE) with halfway bounce-back of what would leave through a wall
        out = np.empty_like(post)
        ny = self.ny
        for i in range(9):
            moved = np.roll(np.roll(post[i], CY[i], axis=0), CX[i], axis=1)
            if not self.walls or CY[i] == 0:
                out[i] = moved
            elif CY[i] > 0:
                out[i, 1:] = moved[1:]
            else:
                out[i, :ny - 1] = moved[:ny - 1]
        if self.walls:
            for i in range(9):
                if CY[i] > 0:
                    out[OPP[i], ny - 1] = post[i, ny - 1]
                elif CY[i] < 0:
                    out[OPP[i], 0] = post[i, 0]
        self.f = out

    def run(self, steps):
        for _ in range(steps):
            self.step()


def loss(built, nx, ny, rho0, w, steps, G=-1.0, sigma=0.0, tau=None, knots=None, walls=False,
         rho_wall_lo=0.0, rho_wall_hi=0.0):
    """L = sum w rho(T), or with w = (w_rho, w_ux, w_uy) sum w_rho rho + w_ux u_x + w_uy u_y at T.
    Any of G, sigma, knots, rho0 may be complex; the result is complex."""
    eos = Eos(built, *(knots if knots is not None else ()))
    L = Lattice(eos, nx, ny, G, sigma, tau, walls, rho_wall_lo, rho_wall_hi)
    L.init_eq(rho0)
    L.run(steps)
    rho, ux, uy = L.fields()[:3]
    if isinstance(w, tuple):
        return (w[0] * rho).sum() + (w[1] * ux).sum() + (w[2] * uy).sum()
    return (w * rho).sum()


H = 1e-30


def gradients(built, nx, ny, rho0, w, steps, G, sigma, tau, nodes=(), **walls):
    """dL/d(rho_max, p_max, rho_min, p_min, G, sigma) and dL/drho0 at the given (y, x) nodes,
    each from one complex-step evaluation."""
    k = [built.rho_max, built.p_max, built.rho_min, built.p_min]
    g = []
    for j in range(4):
        kk = [complex(v) for v in k]
        kk[j] += 1j * H * abs(k[j])
        g.append(loss(built, nx, ny, rho0, w, steps, G, sigma, tau, kk, **walls).imag / (H * abs(k[j])))
    g.append(loss(built, nx, ny, rho0, w, steps, G + 1j * H, sigma, tau, None, **walls).imag / H)
    g.append(loss(built, nx, ny, rho0, w, steps, G, sigma + 1j * H * abs(sigma), tau, None, **walls).imag
             / (H * abs(sigma)))
    d0 = []
    for (y, x) in nodes:
        r = np.asarray(rho0, dtype=np.complex128).copy()
        r[y, x] += 1j * H * abs(rho0[y, x])
        d0.append(loss(built, nx, ny, r, w, steps, G, sigma, tau, None, **walls).imag / (H * abs(rho0[y, x])))
    return np.array(g), np.array(d0)
