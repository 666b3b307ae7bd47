"""Flux functions, maximum wave speeds and admissible sets for the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

States are arrays u[c, ...] with the conserved component first.
  * advection  u_t + div(v u) = 0         [KHV §5.1.1 / §5.3.1]
  * KPP        f(u) = (sin u, cos u)       [KHV §5.3.2]
  * Euler      u = (rho, rho v, rho E), p = (gamma-1)(rho E - |rho v|^2/(2 rho))
                                           [KHV §5.2]
  * nonconvex  1D, f(u) = u (1 - u) / 4 for u <= 1/2, u (u - 1) / 2 + 3/16
               otherwise                   [KHV §5.1.2, eq. (1dkpp-flux)]
"""
import numpy as np


class Advection:
    def __init__(self, d, velocity):
        self.d = d
        self.m = 1
        self.v = np.asarray(velocity[:d], dtype=np.float64)

    def flux(self, u):
        """f_k(u) for k = 0..d-1 -> array (d, m, ...)."""
        return np.stack([self.v[k] * u for k in range(self.d)])

    def node_speed(self, u):
        """Local bound of the maximum speed used in the WENO viscosity
        nu_e = lambda_e h_e / (2p) [KHV eq. (6)]: |v|."""
        return np.full(u.shape[1:], np.sqrt(np.sum(self.v ** 2)))

    def riemann_speed(self, uL, uR, axis):
        """Maximum speed of the 1D Riemann problem along +e_axis
        [KHV eq. (18)]: |v . n|."""
        return np.full(uL.shape[1:], abs(self.v[axis]))

    def riemann_speed_n(self, uL, uR, n):
        """Along a unit normal n (the subcell bound of [KHV eq. (37)])."""
        return np.full(uL.shape[1:], abs(float(np.dot(self.v, n))))


class KPP:
    def __init__(self, d):
        assert d == 2
        self.d = d
        self.m = 1

    def flux(self, u):
        return np.stack([np.sin(u), np.cos(u)])

    def node_speed(self, u):
        # sup |f'(u)| = |(cos u, -sin u)| = 1
        return np.ones(u.shape[1:])

    def riemann_speed(self, uL, uR, axis):
        # |f'(u) . n| <= 1 for every state between u_L and u_R
        return np.ones(uL.shape[1:])

    def riemann_speed_n(self, uL, uR, n):
        return np.ones(uL.shape[1:])


class Euler:
    """Compressible Euler equations of an ideal gas [KHV §5.2]."""

    def __init__(self, d, gamma=1.4):
        self.d = d
        self.m = d + 2
        self.g = float(gamma)

    def pressure(self, u):
        rho = u[0]
        mom2 = np.sum(u[1:1 + self.d] ** 2, axis=0)
        return (self.g - 1.0) * (u[-1] - 0.5 * mom2 / rho)

    def sound_speed(self, u):
        """c = sqrt(max(0, gamma p / rho)) (guard of [KHV §5.2.2])."""
        return np.sqrt(np.maximum(0.0, self.g * self.pressure(u) / u[0]))

    def flux(self, u):
        rho = u[0]
        p = self.pressure(u)
        out = []
        for k in range(self.d):
            vk = u[1 + k] / rho
            comp = [u[1 + k]]
            for j in range(self.d):
                comp.append(u[1 + j] * vk + (p if j == k else 0.0))
            comp.append(vk * (u[-1] + p))
            out.append(np.stack(comp))
        return np.stack(out)

    def node_speed(self, u):
        v = np.sqrt(np.sum((u[1:1 + self.d] / u[0]) ** 2, axis=0))
        return v + self.sound_speed(u)

    def riemann_speed(self, uL, uR, axis):
        """Guaranteed upper bound of the maximum wave speed of the 1D Riemann
        problem (u_L, u_R) along +e_axis: the two-rarefaction estimate of the
        star pressure, which bounds p* from above for 1 < gamma <= 5/3
        (Guermond & Popov, J. Comput. Phys. 321, 2016)."""
        g = self.g
        rhoL, rhoR = uL[0], uR[0]
        vL, vR = uL[1 + axis] / rhoL, uR[1 + axis] / rhoR
        pL, pR = self.pressure(uL), self.pressure(uR)
        cL = np.sqrt(np.maximum(0.0, g * pL / rhoL))
        cR = np.sqrt(np.maximum(0.0, g * pR / rhoR))
        e = (g - 1.0) / (2.0 * g)
        num = np.maximum(cL + cR - 0.5 * (g - 1.0) * (vR - vL), 0.0)
        den = cL * pL ** (-e) + cR * pR ** (-e)
        pstar = (num / den) ** (1.0 / e)
        kappa = (g + 1.0) / (2.0 * g)
        lam1 = vL - cL * np.sqrt(1.0 + kappa * np.maximum(0.0, (pstar - pL) / pL))
        lam3 = vR + cR * np.sqrt(1.0 + kappa * np.maximum(0.0, (pstar - pR) / pR))
        return np.maximum(np.maximum(-lam1, 0.0), np.maximum(lam3, 0.0))

    def riemann_speed_n(self, uL, uR, n):
        """The same bound along a unit normal n (rotational invariance: the
        1D problem sees the normal velocity v . n)."""
        g = self.g
        rhoL, rhoR = uL[0], uR[0]
        vL = sum(n[k] * uL[1 + k] for k in range(self.d)) / rhoL
        vR = sum(n[k] * uR[1 + k] for k in range(self.d)) / rhoR
        pL, pR = self.pressure(uL), self.pressure(uR)
        cL = np.sqrt(np.maximum(0.0, g * pL / rhoL))
        cR = np.sqrt(np.maximum(0.0, g * pR / rhoR))
        e = (g - 1.0) / (2.0 * g)
        num = np.maximum(cL + cR - 0.5 * (g - 1.0) * (vR - vL), 0.0)
        den = cL * pL ** (-e) + cR * pR ** (-e)
        pstar = (num / den) ** (1.0 / e)
        kappa = (g + 1.0) / (2.0 * g)
        lam1 = vL - cL * np.sqrt(1.0 + kappa * np.maximum(0.0, (pstar - pL) / pL))
        lam3 = vR + cR * np.sqrt(1.0 + kappa * np.maximum(0.0, (pstar - pR) / pR))
        return np.maximum(np.maximum(-lam1, 0.0), np.maximum(lam3, 0.0))


class NonConvex:
    """The C^1 nonconvex flux of [KHV eq. (1dkpp-flux)] on a line: concave
    below u = 1/2, convex above, f'(u) = 1/4 - u/2 and u - 1/2 on the two
    branches."""

    def __init__(self, d):
        assert d == 1
        self.d = d
        self.m = 1

    def flux(self, u):
        return np.stack([np.where(u <= 0.5, 0.25 * u * (1.0 - u), 0.5 * u * (u - 1.0) + 3.0 / 16.0)])

    def dflux(self, u):
        return np.where(u <= 0.5, 0.25 - 0.5 * u, u - 0.5)

    def node_speed(self, u):
        return np.abs(self.dflux(u[0]))

    def riemann_speed(self, uL, uR, axis):
        """Largest |f'| over the states between u_L and u_R: |f'| is
        piecewise linear with its only minimum (0) at u = 1/2, so the
        largest value is at an end point."""
        return np.maximum(np.abs(self.dflux(uL[0])), np.abs(self.dflux(uR[0])))

    def riemann_speed_n(self, uL, uR, n):
        return self.riemann_speed(uL, uR, 0)


def make(kind, d, velocity=(1.0, 0.0, 0.0), gamma=1.4):
    if kind == "advection":
        return Advection(d, velocity)
    if kind == "kpp":
        return KPP(d)
    if kind == "euler":
        return Euler(d, gamma)
    if kind == "nonconvex":
        return NonConvex(d)
    raise ValueError(kind)
