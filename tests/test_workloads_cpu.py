"""CPU tests of the benchmark workloads at their full sizes: the host builds the poset and
message layout only (no device), and the counts must match the configurations the bench line
names: the 512-lattice TFIM plaquette sweep and the interval hierarchy Y_8 on the 4096-site chain."""
from collections import Counter

import numpy as np

import lrh_workloads as W
from paper_2609_40336_amd import lrh


def test_plaquette_sweep_sizes():
    d = W.workload_c4()
    sites = np.bincount(d.site_instance, minlength=d.n_instances)
    L = np.rint(np.sqrt(sites)).astype(int)
    assert d.n_instances == 512
    assert np.array_equal(L * L, sites) and L.min() >= 8 and L.max() <= 64
    S = int(sites.sum())
    P = lrh.Problem(d, -1)
    # per periodic L x L lattice: L^2 plaquettes (16 x 16), 2 L^2 bonds (4 x 4), L^2 sites
    assert Counter(len(c) for c in P.clusters) == {4: S, 2: 2 * S, 1: S}
    # messages: 4 L^2 plaquette -> bond (10 real components) and 4 L^2 bond -> site (3)
    assert P.n_msgs == 8 * S
    assert [(b["D"], b["M"], b["comps"]) for b in P.buckets] == [(2, 4 * S, 3), (4, 4 * S, 10)]
    assert P.Lambda == 20.0


def test_interval_chain_y8_sizes():
    P = lrh.Problem(W.workload_c3(8), -1)
    n = 4096
    # level m = 1..8: n - m + 1 intervals of m sites (2^m-dimensional, complex)
    assert Counter(len(c) for c in P.clusters) == {m: n - m + 1 for m in range(1, 9)}
    assert len(P.clusters) == 32740
    # every interval of m >= 2 sites sends a message to each of its two sub-intervals
    assert P.n_msgs == sum(2 * (n - m + 1) for m in range(2, 9))
