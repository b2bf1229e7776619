"""Standard Problem 3 set-up shared by the CPU and GPU Table I tests."""
import json
import math
import os

import numpy as np

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_sp3.json")))
MU0 = 4e-7 * math.pi


def setup():
    mat = GOLDEN["material"]
    Ms, A = mat["Ms"], mat["A"]
    Km = 0.5 * MU0 * Ms * Ms
    lex = math.sqrt(A / Km)
    N = GOLDEN["N"]
    h = GOLDEN["L_over_lex"] * lex / N
    return dict(N=N, h=h, Ms=Ms, A=A, Km=Km, Ku=mat["Ku_over_Km"] * Km, alpha=mat["alpha"])


def initial(kind, N):
    m = np.zeros((3, N, N, N))
    if kind == "flower":
        m[:] = 1.0 / math.sqrt(3.0)
    else:
        m[0, :, :, : N // 2] = 1.0
        m[0, :, :, N // 2:] = -1.0
    return m


def exch_density_central(m, h, A, Km):
    """A |grad m|^2 with cell-centred central differences, Neumann ghosts, in K_m."""
    g = np.pad(m, ((0, 0), (1, 1), (1, 1), (1, 1)), mode="edge")
    c = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    dx = (g[:, 1:-1, 1:-1, 2:] - g[:, 1:-1, 1:-1, :-2]) / (2 * h)
    dy = (g[:, 1:-1, 2:, 1:-1] - g[:, 1:-1, :-2, 1:-1]) / (2 * h)
    dz = (g[:, 2:, 1:-1, 1:-1] - g[:, :-2, 1:-1, 1:-1]) / (2 * h)
    del c
    return A * float(np.mean(np.sum(dx * dx + dy * dy + dz * dz, axis=0))) / Km
