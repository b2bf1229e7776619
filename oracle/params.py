"""Grid and material parameters of the oracle (test infrastructure only).

Notation follows Section II-A of the paper: M = Ms*m, gamma (negative for
electrons, used as printed), gamma_L = gamma/(1+alpha^2), mu0, exchange
constant A, interfacial DMI constant D, uniaxial anisotropy Ku along eK and a
uniform bias field Hbias (A/m).  mu0 is not printed in the paper; the SI value
4*pi*1e-7 is used.
"""
from dataclasses import dataclass, field
import math

TERM_DEMAG = 1
TERM_EXCH = 2
TERM_DMI = 4
TERM_ANIS = 8
TERM_ZEEMAN = 16
TERM_ALL = 31


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float

    @property
    def shape(self):
        """Array shape of one field component: (nz, ny, nx), x fastest."""
        return (self.nz, self.ny, self.nx)

    @property
    def ncell(self):
        return self.nx * self.ny * self.nz

    @property
    def volume(self):
        return self.dx * self.dy * self.dz


@dataclass
class Params:
    Ms: float
    A: float = 0.0
    D: float = 0.0
    Ku: float = 0.0
    eK: tuple = (0.0, 0.0, 1.0)
    Hbias: tuple = (0.0, 0.0, 0.0)
    alpha: float = 0.0
    gamma: float = -1.759e11
    mu0: float = 4.0e-7 * math.pi
    terms: int = TERM_ALL
    # 0: never renormalise, 1: only m_{n+1}, 2: every stage input and m_{n+1}
    renorm: int = 2
    # optional geometry / space-dependent magnetisation: s(r) = Ms(r)/Ms per
    # cell, shape (nz, ny, nx), s >= 0, s = 0 outside the magnet
    ms_profile: object = None
    extra: dict = field(default_factory=dict)

    def has(self, flag):
        return bool(self.terms & flag)
