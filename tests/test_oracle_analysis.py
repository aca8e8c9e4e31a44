"""Pins of the oracle's interstitial analysis: the Wigner-Seitz assignment of a perfect
lattice is the identity on its sites, the inserted dumbbell is found on the site it
replaced, every site of a jittered lattice holds one atom, and residence times of a hand
made history."""
import numpy as np

from oracle import analysis as OA
from paper_2212_10508_amd import workloads as W


def test_perfect_lattice_sites_are_themselves():
    x, box = W.bcc_sia(3, interstitial=False)
    site, occ = OA.ws_sites(x, 3, W.A_W)
    assert np.all(occ == 1)
    # a site's own position is nearest to itself; shifted by whole boxes it still is
    x2 = x + box[:, None] * np.array([[2], [-1], [3]])
    assert np.array_equal(OA.ws_sites(x2, 3, W.A_W)[0], site)


def test_dumbbell_occupies_the_replaced_site():
    x, box = W.bcc_sia(4, jitter=0.05, seed=3)
    site, occ = OA.ws_sites(x, 4, W.A_W)
    assert occ.sum() == x.shape[1] == 129
    assert np.count_nonzero(occ == 2) == 1 and np.count_nonzero(occ == 0) == 0
    assert int(np.argmax(occ)) == 0  # the dumbbell replaces site 0 (corner of cell 0)


def test_residence_times_of_a_history():
    assert OA.residence_times([5, 5, 5, 7, 7, 5, 9, 9, 9, 9]) == [3, 2, 1, 4]
    assert OA.residence_times([]) == []
    assert OA.residence_times([1]) == [1]
