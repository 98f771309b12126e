"""The coupled bead dynamics is chaotic at the translocation parameters, which
bounds the horizon of any pointwise comparison.

Two oracle runs of the 128x64x64 translocation box whose only difference is a
1e-12 shift of one bead separate by many orders of magnitude within 100 LB steps:
an implementation that sums forces in another order (the GPU library, even in
FP64) can only match the oracle pointwise over a shorter horizon; past it,
results are compared through their statistics.
"""
import numpy as np

from tests.common import oracle_sim
from workloads import configs as WC
from workloads import generate as G


def test_perturbation_grows_exponentially():
    w = WC.c2_translocation()
    rep = w.replicas[0]
    beads = G.replica_beads(rep, w.md)
    a = oracle_sim(rep, w.md, beads=beads)
    b = oracle_sim(rep, w.md, beads=beads + np.array([1e-12, 0.0, 0.0]))
    sep = {}
    for s in range(1, 101):
        a.step(1)
        b.step(1)
        if s in (30, 100):
            sep[s] = float(np.max(np.abs(a.r - b.r)))
    assert sep[30] < 1e-10          # still at the size of the nudge
    assert sep[100] > 1e6 * sep[30]  # amplified by orders of magnitude
