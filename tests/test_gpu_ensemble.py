"""Distributional parity of translocation times, GPU ensemble against the oracle's ensemble.

Beyond a few tens of LB steps the coupled bead dynamics is chaotic (a 1e-12 perturbation
reaches the size of the signal within ~100 steps), so no two implementations with different
summation orders follow the same trajectory to completion.  What both must share is the
distribution of the completion step t_done (the first step at which every bead lies past the
wall's mid-plane, Sec. III).  The oracle's sample (FP64, stored in tests/golden by a script
that calls only the oracle) and the GPU's sample come from disjoint seed ranges, so they are
independent; the test asks for a two-sample Kolmogorov-Smirnov p-value above 0.01 and means
within three combined standard errors, for every storage format.  The same holds for the
per-event observables of the translocation analysis (Sec. III), taken from the record the bead
kernel writes every step: the means over the event of S_H, S_E and K, and the ratio R_T at
completion over R_U after the first step (KS p above 0.001 and means within four standard
errors, looser because four more quantities are tested per sample).
"""
from __future__ import annotations

import os

import numpy as np
import pytest

from tests.common import gpu_sim, log
from workloads import configs as WC
from workloads import generate as G

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GOLDEN = os.path.join(HERE, "transloc_pore48_n32.txt")
GOLDEN_NO_HYDRO = os.path.join(HERE, "transloc_pore48_n32_nohydro.txt")
GOLDEN_RIGID = os.path.join(HERE, "transloc_pore48_n32_rigid.txt")
N_GPU = 512
CHECK_EVERY = 250


# columns of the stored sample: seed t_done flags S_H S_E K R_T_end_over_R_U_start retracted
OBS_COLS = {"S_H": 3, "S_E": 4, "K": 5, "R_ratio": 6}


def oracle_rows(path=GOLDEN) -> np.ndarray:
    rows = np.loadtxt(path, comments="#", ndmin=2)
    assert np.all(rows[:, 2] == 0), "the oracle ensemble holds an event with error flags"
    return rows


def oracle_times(path=GOLDEN) -> np.ndarray:
    return oracle_rows(path)[:, 1].astype(np.int64)


@pytest.mark.parametrize("path", [GOLDEN, GOLDEN_NO_HYDRO, GOLDEN_RIGID], ids=["coupled", "nohydro", "rigid"])
def test_oracle_ensemble_file(path):
    """The stored sample is complete, uncensored and drawn from the oracle seed range."""
    rows = np.loadtxt(path, comments="#", ndmin=2)
    assert len(rows) >= 64 and rows.shape[1] == 8
    assert np.array_equal(rows[:, 0].astype(np.int64), WC.ENSEMBLE_SEED_ORACLE + np.arange(len(rows)))
    t = rows[:, 1]
    assert np.all(t > 0) and np.all(t < WC.ENSEMBLE_STEP_CAP)
    assert np.all(np.isfinite(rows[:, 3:7]))
    assert np.all(rows[:, 5] > 0) and np.all(rows[:, 6] > 0)


def test_solvent_speeds_translocation():
    """The oracle's own samples: with the lattice solvent the chain crosses faster than
    alone in a fluid at rest (Sec. III finds hydrodynamics speeds translocation)."""
    a, b = oracle_times(GOLDEN), oracle_times(GOLDEN_NO_HYDRO)
    se = np.sqrt(a.var(ddof=1) / len(a) + b.var(ddof=1) / len(b))
    assert b.mean() - a.mean() > 3 * se


@pytest.mark.gpu
@pytest.mark.parametrize("storage,hydro,model", [(WC.STORE_F64, True, "harmonic"), (WC.STORE_F32, True, "harmonic"),
                                                 (WC.STORE_F16, True, "harmonic"), (WC.STORE_BF16, True, "harmonic"),
                                                 (WC.STORE_F32, False, "harmonic"), (WC.STORE_F32, True, "paper")],
                         ids=["f64", "f32", "f16dev", "bf16dev", "nohydro", "rigid"])
def test_translocation_time_distribution(storage, hydro, model):
    from scipy import stats

    golden = GOLDEN_RIGID if model == "paper" else (GOLDEN if hydro else GOLDEN_NO_HYDRO)
    t_ora = oracle_times(golden)
    md = WC.paper_polymer() if model == "paper" else WC.MDParams()
    w = WC.ensemble48_n32(N_GPU, WC.ENSEMBLE_SEED_GPU, storage, md=md)
    log(f"ensemble {w.name} storage {WC.STORE_NAMES[storage]}{'' if hydro else ' without solvent'}: "
        f"{N_GPU} replicas, cap {WC.ENSEMBLE_STEP_CAP} steps")
    beads = np.concatenate(G.workload_beads(w))
    sim = gpu_sim(w.replicas, w.md, storage, beads=beads, obs_every=1, obs_capacity=WC.ENSEMBLE_STEP_CAP)
    try:
        steps = 0
        t_gpu = np.full(N_GPU, -1)
        while steps < WC.ENSEMBLE_STEP_CAP:
            n = min(CHECK_EVERY, WC.ENSEMBLE_STEP_CAP - steps)
            sim.step(n, hydro=hydro)
            steps += n
            t_gpu = np.array([sim.transloc(r)["t_done"] for r in range(N_GPU)])
            log(f"  step {steps}: {int(np.sum(t_gpu >= 0))} of {N_GPU} events complete")
            if np.all(t_gpu >= 0):
                break
        err, _ = sim.status()
        assert err == 0, f"error word {err:#x}"
        records = [sim.observables(r)[0] for r in range(N_GPU)]
    finally:
        sim.close()
    assert np.all(t_gpu > 0), f"{int(np.sum(t_gpu < 0))} GPU events censored at the step cap"
    ks = stats.ks_2samp(t_gpu, t_ora)
    m_g, m_o = t_gpu.mean(), t_ora.mean()
    se = np.sqrt(t_gpu.var(ddof=1) / len(t_gpu) + t_ora.var(ddof=1) / len(t_ora))
    log(f"  t_done mean gpu {m_g:.1f} (sd {t_gpu.std(ddof=1):.1f}) oracle {m_o:.1f} "
        f"(sd {t_ora.std(ddof=1):.1f}); KS D {ks.statistic:.4f} p {ks.pvalue:.4f}; "
        f"mean difference {abs(m_g - m_o) / se:.2f} standard errors")
    assert ks.pvalue > 0.01
    assert abs(m_g - m_o) < 3.0 * se

    # per-event observables of the Sec. III analysis
    from paper_0710_1272_amd import ensemble as E
    ora = oracle_rows(golden)
    gpu = {k: [] for k in OBS_COLS}
    for rows, t in zip(records, t_gpu):
        ev = E.event_rows(rows, int(t))
        assert len(ev) == t and ev[-1, E.STEP] == t
        gpu["S_H"].append(ev[:, E.S_H].mean())
        gpu["S_E"].append(ev[:, E.S_E].mean())
        gpu["K"].append(ev[:, E.K].mean())
        gpu["R_ratio"].append(np.sqrt(ev[-1, E.R_T2] / ev[0, E.R_U2]))
    for key, col in OBS_COLS.items():
        a, b = np.array(gpu[key]), ora[:, col]
        if not hydro and key == "S_H":
            assert np.all(a == 0.0) and np.all(b == 0.0)  # no solvent: no fluid work
            continue
        ks = stats.ks_2samp(a, b)
        se = np.sqrt(a.var(ddof=1) / len(a) + b.var(ddof=1) / len(b))
        log(f"  {key}: gpu {a.mean():.4e} oracle {b.mean():.4e}; KS p {ks.pvalue:.4f}; "
            f"{abs(a.mean() - b.mean()) / se:.2f} standard errors")
        assert ks.pvalue > 0.001, key
        assert abs(a.mean() - b.mean()) < 4.0 * se, key
