"""Pins of the oracle's probe generator (Sec. 3.1: Rademacher probes, redrawn
at every EM iteration of Algorithm 1) against the published SplitMix64 stream."""
import os

import numpy as np

import oracle as O


def _published(golden_dir):
    vals = []
    with open(os.path.join(golden_dir, "splitmix64_seed0.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                vals.append(int(line, 16))
    return vals


def test_splitmix64_matches_published_stream(golden_dir):
    pub = _published(golden_dir)
    got = O.splitmix64_stream(0, np.arange(1, len(pub) + 1, dtype=np.uint64))
    assert [int(v) for v in got] == pub


def test_probe_bits_follow_stream_words(golden_dir):
    # entry (j, k=0) of EM iteration t=0 takes bit j of stream word 1 (seed 0)
    pub = _published(golden_dir)
    P = O.rademacher_probes(0, 0, 1, 128)
    for j in range(128):
        word = pub[j // 64]
        bit = (word >> (j % 64)) & 1
        assert P[j, 0] == (1.0 - 2.0 * bit)


def test_probe_counter_layout():
    # word index (t << 48) | (k << 32) | (j >> 6), 1-based counter
    seed, t, k, j = 987654321, 7, 3, 64 * 5 + 17
    P = O.rademacher_probes(seed, t, k + 1, j + 1)
    word = int(O.splitmix64_stream(seed, np.array([(t << 48) + (k << 32) + 5 + 1], dtype=np.uint64))[0])
    assert P[j, k] == 1.0 - 2.0 * ((word >> 17) & 1)


def test_probe_golden_file(golden_dir):
    path = os.path.join(golden_dir, "probes_seed12345_t3_K5_D300.txt")
    ref = np.loadtxt(path)
    P = O.rademacher_probes(12345, 3, 5, 300)
    assert np.array_equal(P, ref)


def test_probe_statistics():
    # zero mean, unit second moment, no correlation between columns or draws
    D, K = 1 << 14, 8
    P1 = O.rademacher_probes(1, 1, K, D)
    P2 = O.rademacher_probes(1, 2, K, D)
    assert set(np.unique(P1)) == {-1.0, 1.0}
    assert abs(P1.mean()) < 4.0 / np.sqrt(D * K)
    C = (P1.T @ P1) / D
    off = C - np.eye(K)
    assert np.max(np.abs(off)) < 5.0 / np.sqrt(D)
    assert np.max(np.abs(P1.T @ P2 / D)) < 5.0 / np.sqrt(D)
    # different seeds differ
    assert not np.array_equal(P1, O.rademacher_probes(2, 1, K, D))
