"""Chandrasekhar's H-function for isotropic scattering with single-scatter
albedo omega (Radiative Transfer, 1950, ch. V): the solution of
    1 / H(mu) = 1 - (omega / 2) mu int_0^1 H(mu') / (mu + mu') dmu',
found by iteration on Gauss-Legendre nodes of [0, 1].  A semi-infinite,
isotropically scattering medium lit at normal incidence reflects the share
    A = 1 - H(1) sqrt(1 - omega)
of the incident flux (the plane albedo), and the share
    D(mu_c) = (omega / 2) H(1) int_{mu_c}^1 H(mu) mu / (mu + 1) dmu
leaves within the cone mu >= mu_c about the normal (the reflected intensity
is (omega/4) F mu0 H(mu) H(mu0) / (mu + mu0)).  Test reference only: it
shares nothing with the oracle or the library."""
import numpy as np


class HFunction:
    def __init__(self, omega: float, n: int = 96, tol: float = 1e-14, max_iter: int = 20000):
        x, w = np.polynomial.legendre.leggauss(n)
        self.mu = 0.5 * (x + 1.0)
        self.w = 0.5 * w
        self.omega = float(omega)
        h = np.ones(n)
        for _ in range(max_iter):
            s = (h * self.w)[None, :] / (self.mu[:, None] + self.mu[None, :])
            h_new = 1.0 / (1.0 - 0.5 * self.omega * self.mu * s.sum(axis=1))
            if np.max(np.abs(h_new - h)) < tol:
                h = h_new
                break
            h = h_new
        self.h = h

    def __call__(self, mu):
        mu = np.atleast_1d(np.asarray(mu, np.float64))
        s = (self.h * self.w)[None, :] / (mu[:, None] + self.mu[None, :])
        return 1.0 / (1.0 - 0.5 * self.omega * mu * s.sum(axis=1))

    def moment0(self) -> float:
        return float(np.sum(self.w * self.h))

    def plane_albedo(self, mu0: float = 1.0) -> float:
        return float(1.0 - self(mu0)[0] * np.sqrt(1.0 - self.omega))

    def cone_share(self, mu_c: float, mu0: float = 1.0, n: int = 64) -> float:
        x, w = np.polynomial.legendre.leggauss(n)
        mu = mu_c + 0.5 * (x + 1.0) * (1.0 - mu_c)
        ww = 0.5 * w * (1.0 - mu_c)
        return float(0.5 * self.omega * self(mu0)[0] * np.sum(ww * self(mu) * mu / (mu + mu0)))
