"""Double-majority matching of track candidates to generated particles (host logic of
paper_2501_05520_amd.evaluate_trained), on hand-built labellings."""
import numpy as np

from paper_2501_05520_amd.evaluate_trained import match_candidates


def test_perfect_candidates():
    pid = np.array([1, 1, 1, 2, 2, 2, 0])
    labels = np.array([0, 0, 0, 3, 3, 3, 6])
    assert match_candidates(labels, pid) == (2, 2, 2, 0)


def test_merged_particles_are_fake():
    # one component holding two whole particles: neither owns more than half of it
    pid = np.array([1, 1, 1, 2, 2, 2])
    labels = np.zeros(6, int)
    assert match_candidates(labels, pid) == (0, 2, 1, 1)


def test_majority_with_a_stray_hit():
    # particle 1 has 5 hits, 4 of them in a candidate that also holds one hit of particle 2
    pid = np.array([1, 1, 1, 1, 1, 2, 2, 2])
    labels = np.array([0, 0, 0, 0, 4, 0, 6, 7])
    found, n_true, n_cand, fake = match_candidates(labels, pid)
    assert (found, n_true, n_cand, fake) == (1, 2, 1, 0)


def test_short_candidates_and_noise_are_ignored():
    pid = np.array([1, 1, 0, 0, 0])
    labels = np.array([0, 0, 2, 2, 2])      # the particle has 2 hits; the noise cluster is fake
    assert match_candidates(labels, pid) == (0, 0, 1, 1)


def test_half_is_not_a_majority():
    # a 4-hit candidate with 2 hits of particle 1 and 2 of particle 2
    pid = np.array([1, 1, 2, 2, 1, 2])
    labels = np.array([0, 0, 0, 0, 4, 5])
    assert match_candidates(labels, pid) == (0, 2, 1, 1)
