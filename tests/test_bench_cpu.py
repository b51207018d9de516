"""CPU checks of the benchmark's measurement helpers: the all-cores CPU
reference update equals the oracle's mini-batch update, and the roofline
entry's pipeline fraction follows its definition."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402
from oracle import ptycho  # noqa: E402
from paper_2608_01746_amd import synth  # noqa: E402

from _cases import tiny_scan  # noqa: E402


def test_all_cores_update_equals_oracle():
    O, P, pos, I = tiny_scan(120, 32, 32, 4, 20, 3, seed=9)
    rng = np.random.default_rng(1)
    O0 = O * (0.8 + 0.1 * rng.standard_normal(O.shape))
    P0 = P * np.exp(0.3j)
    A = ptycho.amplitudes(I)
    idx = np.array([5, 1, 12, 7, 3])
    prm = ptycho.PtychoParams("rpie", 0.2, 0.3, 5, True)
    Or, Pr, er = ptycho.batch_update(O0, P0, A, pos, idx, prm, True)
    Ob, Pb, eb = bench.batch_update_all_cores(O0, P0, A, pos, idx, 0.2, 0.3, True, 2)
    assert np.linalg.norm(Ob - Or) <= 1e-12 * np.linalg.norm(Or)
    assert np.linalg.norm(Pb - Pr) <= 1e-12 * np.linalg.norm(Pr)
    assert abs(eb - er) <= 1e-12 * er


def test_pipeline_fraction_definition():
    w = synth.lab_workload()
    r = bench.roofline("cols_modulus", 100, 1.0, w.J / 13, w.Nd, w.batch, counters=False,
                       updates_per_step=w.J * 200, ms_per_step=150.0)
    expect = bench.algo_bytes_per_update(256, 32) * 80000 / 0.150 / 8e12
    assert abs(r["pipeline_frac"] - expect) < 1e-4
    assert r["traffic_ratio"] is None
