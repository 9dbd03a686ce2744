"""Input generators: symmetries, determinism, selected-set sizes."""
import math

import numpy as np

import synth


def test_integral_symmetry_and_determinism():
    h, g = synth.integrals(7, 3)
    assert np.array_equal(h, h.T)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.array_equal(g, g.transpose(perm))
    h2, g2 = synth.integrals(7, 3)
    assert np.array_equal(h, h2) and np.array_equal(g, g2)
    assert not np.array_equal(h, synth.integrals(7, 4)[0])


def test_theta_shape_and_order():
    th = synth.nqs_theta(16, 16, 0)
    assert th.size == 288 == synth.n_params(16, 16)
    assert synth.n_params(24, 64) == 1624 and synth.n_params(40, 256) == 10536


def test_cisd_candidate_count_and_selection():
    keys, rank, _ = synth._pairs_up_to_rank(20, 10, 10, 4)
    assert keys.size == 7_516_876
    sel = synth.cisd_like_selected_set(10, 5, 5, 2000, seed=0)
    assert sel.size == 2000 and np.all(np.diff(sel.astype(np.int64)) > 0)
    assert np.array_equal(sel, synth.cisd_like_selected_set(10, 5, 5, 2000, seed=0))
    aufbau = synth.key_of(0b11111, 0b11111)
    assert aufbau in set(sel.tolist())


def test_capped_set():
    full = synth.capped_set(8, 4, 4, 1 << 18)
    assert full.size == math.comb(8, 4) ** 2
    cap = synth.capped_set(16, 8, 8, 1 << 18)
    assert cap.size == 1 << 18 and np.all(np.diff(cap.astype(np.int64)) > 0)


def test_batch_workloads():
    ws = synth.batch_workloads(64)
    assert len(ws) == 64
    assert all(8 <= w.n <= 16 and 16 <= w.H <= 128 and w.V == 2 * w.n for w in ws)
    assert all(w.size() <= 1 << 18 for w in ws)
