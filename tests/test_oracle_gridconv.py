"""Pins of the grid-convergence study (Appendix B) on the oracle: with the
range and the density of the grid each grown by sqrt(2) per doubling of the
points, a propagated smooth state converges exponentially (the error falls
by orders of magnitude per doubling, faster at every step), the initial
error -- a sampled Gaussian, no propagation -- converges likewise, and the
integration error is a share of the total, below it or comparable to it
(the paper finds about one half)."""
import math

import numpy as np

from gridconv_oracle import study
from paper_1903_04946_amd import synth


def test_propagated_state_converges_exponentially(orc):
    # 1D two-surface harmonic model with a Gaussian coupling: range and
    # density x sqrt(2) per doubling, 32 ... 256 points (256 the reference)
    models = []
    for n in (32, 64, 128, 256):
        L = 6.0 * math.sqrt(n / 32)
        m = synth.random_small([n], 2, seed=4, lo=-L, hi=L, coupling=0.3)
        models.append(m)
    rows = study(orc, models, orc.VTV, orc.SUZUKI, 6, 0.1, 20)
    tot = [r["total_error"] for r in rows]
    ini = [r["initial_error"] for r in rows]
    print(rows)
    # measured: 7.9e-4, 1.2e-5, 8.6e-9 (ratios 0.78, 0.64, 0.63)
    assert tot[0] > 1e-4 and tot[-1] < 1e-7          # orders of magnitude
    assert tot[1] / tot[0] < 0.05 and tot[2] / tot[1] < tot[1] / tot[0]  # faster and faster
    assert ini[0] > ini[1] > ini[2]
    for r in rows:
        assert 0.3 < r["ratio"] <= 1.0
