"""Golden pin from the paper's Table I (Standard Problem 3, N = 10): the
oracle relaxes the flower state and reproduces the printed energy densities
and m_z to the paper's last digit (within 1.5e-3 K_m)."""
import numpy as np

from oracle import llg, newell
from oracle.params import Grid, Params, TERM_ANIS, TERM_DEMAG, TERM_EXCH
from tests.sp3_common import GOLDEN, exch_density_central, initial, setup


def test_flower_state_matches_table1():
    s = setup()
    N, h = s["N"], s["h"]
    g = Grid(N, N, N, h, h, h)
    p = Params(Ms=s["Ms"], A=s["A"], Ku=s["Ku"], eK=(0.0, 0.0, 1.0), alpha=s["alpha"],
               terms=TERM_DEMAG | TERM_EXCH | TERM_ANIS)
    spec = newell.spectrum(g)
    m = initial("flower", N)
    for _ in range(1500):          # 0.75 ns; the flower state is converged to 1e-4 by then
        m = llg.rk4_step(g, p, m, 5e-13, spec)
    e = llg.energy_parts(g, p, m, spec)
    V = g.volume * g.ncell * s["Km"]
    ref = GOLDEN["flower"]
    assert abs(e["demag"] / V - ref["e_demag"]) < 1.5e-3
    assert abs(e["anis"] / V - ref["e_anis"]) < 1.5e-3
    assert abs(exch_density_central(m, h, s["A"], s["Km"]) - ref["e_exch"]) < 1.5e-3
    assert abs(float(m[2].mean()) - ref["m_z"]) < 1.5e-3
