"""Host logic of the droplet labels: equivalent diameters, passage detection
and the generation period, on synthetic inputs with known answers."""
import math

import numpy as np

from paper_2512_12934_amd import cases, labels


def test_diameter_of_disc_and_ball():
    # a digitised disc of radius 20 has ~pi 400 nodes: D within a node of 40
    n = 101
    y, x = np.mgrid[0:n, 0:n]
    area = int(((x - 50) ** 2 + (y - 50) ** 2 < 400).sum())
    assert abs(labels.diameter(area, 2) - 40.0) < 0.2
    assert math.isclose(labels.diameter(4.0 / 3.0 * math.pi * 1000.0, 3), 20.0, rel_tol=1e-12)


def test_passages_and_period():
    every = 100
    s = np.zeros(200, int)
    starts = [10, 30, 52, 71, 93, 112, 130]
    for t in starts:
        s[t:t + 6] = 5            # a droplet crossing the probe for 6 samples
    ev = labels.passages(s)
    assert list(ev) == starts
    # first two discarded; intervals 19, 22, 19, 18 samples, median 19
    assert labels.period(s, every) == 19 * every
    # one passage counted twice (a front that recedes and returns) splits an
    # interval into 3 + 16: the median moves to a neighbouring interval
    # (18 samples), where the mean would drop to 15.6
    s2 = s.copy()
    s2[95] = 0
    assert list(labels.passages(s2)) == [10, 30, 52, 71, 93, 96, 112, 130]
    assert labels.period(s2, every) == 18 * every
    # fewer than three passages after the first two: censored
    assert labels.period(s[:80], every) is None


def test_tjunction_regions_inside_main_channel():
    c = cases.tjunction(W=20, length=160, x_side=30, side_width=20, side_len=20)
    region, probe = labels.tjunction_regions(c)
    (lo, hi), (plo, phi) = region, probe
    W = c.meta["W"]
    assert lo[0] >= 30 + 20 and hi[0] <= c.n[0] - 1
    assert (lo[1], hi[1]) == (1, W + 1) and (plo[1], phi[1]) == (1, W + 1)
    assert lo[0] <= plo[0] < hi[0] and phi[0] == plo[0] + 1
    # every node of the region is fluid
    sol = c.solid.reshape(c.n[1], c.n[0])
    assert not sol[lo[1]:hi[1], lo[0]:hi[0]].any()


def test_threshold_between_bulk_densities():
    c = cases.tjunction(W=20, length=90, x_side=30, side_width=14, side_len=18)
    assert math.isclose(labels.threshold(c), 0.5 * (cases.COEX_G09[0] + cases.COEX_G09[1]))
