"""Closed-form results used to pin the oracle (test infrastructure only).

None of these is the method itself; they are textbook limits that the
dynamics must reproduce, chosen so that a wrong neighbour map, a dropped
term or a sign error in the oracle shows up.
"""

from __future__ import annotations

import math

from scipy.special import ellipk


def square_lattice_tc(J: float = 1.0) -> float:
    """Critical temperature of the square-lattice Ising model, 2J / ln(1 + sqrt 2)."""
    return 2.0 * J / math.log(1.0 + math.sqrt(2.0))


def square_lattice_magnetisation(T: float) -> float:
    """Spontaneous magnetisation per site (Onsager; Yang 1952): (1 - sinh(2/T)^-4)^(1/8) below Tc."""
    if T >= square_lattice_tc():
        return 0.0
    return (1.0 - math.sinh(2.0 / T) ** -4) ** 0.125


def square_lattice_energy(T: float) -> float:
    """Internal energy per site of the square-lattice Ising model at H = 0 (Onsager 1944).

    u = -coth(2K) [1 + (2/pi)(2 tanh^2(2K) - 1) K(kappa)],  kappa = 2 sinh(2K) / cosh^2(2K),
    K = 1/T, with K(kappa) the complete elliptic integral of the first kind (modulus kappa).
    """
    K = 1.0 / T
    kappa = 2.0 * math.sinh(2 * K) / math.cosh(2 * K) ** 2
    return -(1.0 / math.tanh(2 * K)) * (1.0 + (2.0 / math.pi) * (2.0 * math.tanh(2 * K) ** 2 - 1.0)
                                         * float(ellipk(kappa * kappa)))


def single_spin_magnetisation(H: float, T: float) -> float:
    """Mean spin of an isolated Ising spin in field H: tanh(H/T)."""
    return math.tanh(H / T)


def critical_concentration(z: float) -> float:
    """Eq. (2): p_c = 2 / z for mean coordination z."""
    return 2.0 / z


def two_free_spins_with_anisotropy(H: float, h_an: float, T: float):
    """Two spins without a bond in field H with the anisotropy term -h_an |M| of Eq. (7).

    The four states have E(++) = -2H - 2 h_an, E(--) = 2H - 2 h_an and E(+-) = E(-+) = 0, so
    <M> = 2 sinh(2H/T) / (cosh(2H/T) + exp(-2 h_an/T)) and
    <|M|> = 2 cosh(2H/T) / (cosh(2H/T) + exp(-2 h_an/T)).  Returns (<M>, <|M|>).
    """
    c, s, e = math.cosh(2.0 * H / T), math.sinh(2.0 * H / T), math.exp(-2.0 * h_an / T)
    return 2.0 * s / (c + e), 2.0 * c / (c + e)
